// se1p_plan.h -- host-side plan state shared by the single-system entry
// points (se1p_host.cpp) and the batched ones (se1p_batch.cpp).  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "se1p.h"
#include "se1p_internal.h"

using se1p::BinGeo;
using se1p::FftDesc;
using se1p::Geo;
using se1p::SlabDesc;

// Per-call device scratch of a plan: every buffer an evaluation writes
// besides its outputs.  se1p_eval uses the plan's own scratch, allocated
// with the plan for n_max particles; se1p_eval_noalloc lays the same
// buffers out in the library's static scratch array for the call's N.
struct PlanScratch {
    se1p::BinBufs bins{};
    int *lex_i[5] = {}, *blk_i[5] = {};   // cx, cy, cz, perm, start
    void *lex_f[7] = {}, *blk_f[7] = {};  // x, y, z, q, tx, ty, tz
    void *wz = nullptr, *wxp = nullptr, *wyq = nullptr;
    void* Hpart = nullptr;
    void *Hper = nullptr, *Htp = nullptr;   // SE3P: folded grid, transform output
    void *Gk = nullptr, *Htk = nullptr;     // ik-differentiation: slab copies, field grids
    void* Fz = nullptr;
    void* G = nullptr;
    void* Ht = nullptr;
    void *phiF = nullptr, *EF = nullptr, *phiR = nullptr, *ER = nullptr;
    double* partials = nullptr;
    int nblk_comb = 0;
    int* flag = nullptr;
    double* qsum = nullptr;
    int rs_parts = 1;       // real-space parts per 16-target chunk
};

// Geometry, tables and (for single-system plans) the device workspace.
struct se1p_plan {
    se1p_params prm;
    int prec = 0;           // SE1P_FP64 / SE1P_FP32
    size_t es = 8;          // element size
    long long n_max = 0;
    int device = 0;
    hipStream_t stream = nullptr;

    Geo g{};                // gridding / gather geometry (extended grid)
    Geo gf{};               // transform geometry: g itself for SE1P; the
                            // periodic M1 x M2 x M3 grid for SE3P
    bool periodic3 = false; // triply periodic (SE3P) plan
    BinGeo bg{};
    double cg = 0.0;        // (2 xi^2 / (pi eta))^{3/2}
    double R = 0.0;
    int M1 = 0, M2 = 0;
    int n0[2] = {0, 0}, nl[2] = {0, 0};
    int nslab = 0;
    int CZ = 0, KP = 0;
    bool in_batch = false;  // planned as a member of a batch: the batch, not
                            // the system alone, fills the chip
    std::vector<SlabDesc> slabs;
    FftDesc dz{};
    long long tw_elems = 0;
    long long slab_elems = 0;
    std::map<int, int> twoff;   // FFT length -> twiddle offset (complex elements)

    // device memory: one allocation, carved into the tables below and the
    // plan's own scratch (laid out for n_max particles)
    void* base = nullptr;
    size_t ws_bytes = 0;
    long long pstride = 0;      // elements between the KP partial grids
    void* S0 = nullptr;         // FP64 k3 = 0 scaling table (in T)
    void* tw = nullptr;         // FFT twiddles
    SlabDesc* d_slabs = nullptr;
    PlanScratch w{};

    // stage timing: events[call][boundary], boundaries 0..SE1P_NSTAGE
    int timing = 0;
    unsigned tstages = (1u << SE1P_NSTAGE) - 1u;   // stages whose events are recorded
    int tcalls = 0;
    std::vector<hipEvent_t> tev;
    std::vector<unsigned char> tmask;   // stages run per call
};

namespace se1p {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Parameter checks shared by plans and batches.
int plan_check_params(const se1p_params& p);
// Grid geometry, padded FFT sizes, slab descriptors, tiling and twiddle
// offsets of one system (no device memory).
int plan_geometry(se1p_plan& pl, const se1p_params& p, long long n_max);
// Lays out the per-call scratch of an evaluation of n particles at base
// (the plan's own workspace, or another buffer) and returns its size in
// bytes; base = 0 only sizes it.  The ik-differentiation buffers are laid
// out only when ik is set.
size_t layout_scratch(const se1p_plan& pl, long long n, PlanScratch& w, uintptr_t base,
                      bool ik = true);
// Makes the plan's device current.
int set_device(const se1p_plan* pl);
// Host-side argument checks shared by the evaluation entry points.
int eval_args(const se1p_plan* pl, long long N, const void* x, const void* q,
              unsigned flags);
// The evaluation proper (input checks, then the pipeline) on the plan's
// current scratch.
int eval_body(se1p_plan* pl, long long N, const void* x, const void* q,
              void* phi, void* efield, double* energy, unsigned flags);
// Host tables of a planned system: twiddles exp(-2 pi i k/n) for every length
// in pl.twoff (interleaved re/im, laid out by pl.twoff) and the FP64
// scaling table of slab n3 = 0, n0[0] x n0[1].
void plan_tables(const se1p_plan& pl, std::vector<double>& tw, std::vector<double>& s0);
}  // namespace se1p
