// se1p_internal.h -- shared between the host planner and the HIP kernels of
// the SE1P library.  Not part of the public C ABI (include/se1p.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace se1p {

constexpr int kMaxRad = 16;      // radix passes per FFT length
constexpr int kSpreadTile = 8;   // spread tile: 8 x 8 (x, y) pencils, one per lane
// Waves per spread tile, splitting its particles: worth it when a particle
// brings enough work (P z-points per lane) to pay for the per-plane LDS sum.
constexpr int spread_waves(int P) { return P >= 20 ? 8 : (P >= 16 ? 4 : 1); }
constexpr int kZfftCols = 32;    // columns per block in the z transforms
// Gather units of two blocks walk their z layers 64 per lane group: blocks
// of up to 64 kMaxLayerGroups - 1 z cells can be paired.
constexpr int kMaxLayerGroups = 2;
constexpr int kMaxP = 32;

// One 1D FFT length: radices in pass order and the offset of its twiddle
// table exp(-2 pi i k / n), k = 0..n-1, inside the plan's twiddle array.
struct FftDesc {
    int n;
    int nrad;
    int twoff;
    int rad[kMaxRad];
};

// Per-slab (n3 = 0 .. M3/2) description of the adaptive transform: padded
// sizes (eq. upsamplings), FFT descriptors and the slab's offset (complex
// elements) into the padded-slab workspace.
struct SlabDesc {
    int n1, n2;        // padded FFT lengths along x and y
    int n3;            // mode index
    int pad_;
    long long off;     // complex elements
    double pref;       // 4 pi h^3 cg^2 / (M3 n1 n2)
    FftDesc d1, d2;
};

// Geometry passed by value to kernels.
struct Geo {
    double h, inv_h, L3, alpha, eta, xi;
    int M1, M2, M3, P;
    int Mt1, Mt2;
    long long ncol;    // Mt1 * Mt2
};

// Binning: particle cells in two orders.
//   lex order   (cz, cx, cy)  -- spreading and the real-space sum
//   block order blocks of BZ x BX x BY cells, lexicographic inside  -- gather
struct BinGeo {
    int BX, BY, BZ;
    int CH;               // gather waves per gather unit (one chunk each)
    int pair;             // 1: a gather unit is two y-adjacent blocks, the
                          // even one and the next (nby even), 32 lanes
                          // each; 0: one block, 64 lanes
    int ldy;              // gather LDS row pitch: >= (1 + pair) BY + P - 1
                          // and == BY (mod nb), nb = 128 / word size; with
                          // BX * BY <= nb the window origins of distinct
                          // cells of one block then fall in distinct LDS
                          // banks
    int nbx, nby, nbz;
    int cpb;              // cells per block
    long long ncell_lex;  // M3 * M1 * M2
    long long ncell_blk;  // nbz * nbx * nby * cpb
};

template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using cplx = typename cplx_t<T>::type;

// ---- launchers (implemented in se1p_kernels.hip) ---------------------------
template <typename T>
struct DevParticles {        // sorted copies of the particles in one order
    T* x; T* y; T* z; T* q;  // z wrapped into [0, L3)
    T* tx; T* ty; T* tz;     // offsets inside the cell in units of h:
                             // x / h - cx, computed in FP64, so that the
                             // Gaussian weights do not lose the digits of
                             // x - grid point to the size of x
    int* cx; int* cy; int* cz;
    int* perm;               // sorted position -> input index
    int* start;              // cell starts, size ncell + 1
};

// Counting sort scratch.  Cell counts of both orders are scanned into the
// cell starts by hand-written reduce-then-scan kernels: one pass sums each
// tile of kScanTile counts, the next scans every tile with the sum of the
// tiles before it as offset (integer sums, so the starts do not depend on
// the order in which anything ran).
constexpr int kScanItems = 16;                 // counts per thread
constexpr int kScanTile = 256 * kScanItems;    // counts per workgroup
inline int scan_tiles(long long n) { return (int)((n + kScanTile - 1) / kScanTile); }

struct BinBufs {
    int* key_lex; int* key_blk;   // N: cell of each particle in both orders
    int* slot;                    // N: arrival slot in its lex cell
    int* tmp;                     // N: lex order by arrival (before ranking)
    int* cnt_lex; int* cnt_blk;   // ncl + 1, ncb + 1 cell counts
    int* tsum;                    // ntl + ntb particles per scan tile
    long long ncl, ncb;           // cells in the lex and block orders
    int ntl, ntb;                 // scan tiles over ncl + 1 and ncb + 1 entries
};
// Sizes of the per-cell parts of BinBufs for ncl lex and ncb block cells.
inline void bin_sizes(BinBufs& b, long long ncl, long long ncb) {
    b.ncl = ncl;
    b.ncb = ncb;
    b.ntl = scan_tiles(ncl + 1);
    b.ntb = scan_tiles(ncb + 1);
}

template <typename T>
int launch_bin(const T* x_in, const T* q_in, long long N, const Geo& g,
               const BinGeo& bg, const BinBufs& b, DevParticles<T>& lex,
               DevParticles<T>& blk, hipStream_t s);

template <typename T>
int launch_spread(const DevParticles<T>& lex, long long N, const Geo& g,
                  int CZ, int KP, T* wz, T* wxp, T* wyq, T* Hpart,
                  long long pstride, hipStream_t s);

template <typename T>
int launch_reduce_partials(const T* Hpart, int KP, long long pstride,
                           long long n, T scale, T* out, hipStream_t s);

template <typename T>
int launch_kspace(const T* Hin, int KP, long long pstride, T in_scale,
                  const Geo& g, int nslab, const SlabDesc* d_slabs,
                  const SlabDesc* h_slabs, const FftDesc& dz,
                  const cplx<T>* tw, const T* S0, cplx<T>* Fz, cplx<T>* G,
                  T out_scale, T* Ht, hipStream_t s);

template <typename T>
int launch_gather(const T* Ht, const DevParticles<T>& blk, long long N,
                  const Geo& g, const BinGeo& bg, T scale, T* phi_out,
                  T* E_out, hipStream_t s);

// nparts: the candidate rows of each 16-target chunk are split in nparts
// parts run as separate waves; part k writes slice k of phi_out / E_out.
// periodic3: sources from the images in x and y as well (SE3P).
template <typename T>
int launch_realspace(const DevParticles<T>& lex, const DevParticles<T>& blk,
                     long long N, const Geo& g, const BinGeo& bg, double xi,
                     double rc, int nparts, bool periodic3, T* phi_out, T* E_out,
                     hipStream_t s);

// The k-space solve with the field by ik-differentiation: potential grid Ht
// and the three field-component grids Htk + d gstride (d = 0, 1, 2); Gk is
// workspace for three copies of the slab data (slab_elems each).
template <typename T>
int launch_kspace_ik(const T* Hin, int KP, long long pstride, const Geo& g,
                     int nslab, const SlabDesc* d_slabs, const SlabDesc* h_slabs,
                     const FftDesc& dz, const cplx<T>* tw, const T* S0,
                     cplx<T>* Fz, cplx<T>* G, cplx<T>* Gk, long long slab_elems,
                     T* Ht, T* Htk, long long gstride, hipStream_t s);

// Potential-only gather of one grid into out[perm * ostride].
template <typename T>
int launch_gather_phi(const T* Ht, const DevParticles<T>& blk, const Geo& g,
                      const BinGeo& bg, T scale, T* out, int ostride, hipStream_t s);

// SE3P: sum the KP partial extended grids (geometry g) onto the periodic
// grid (geometry gf, Mt = M), and copy the periodic grid back out over the
// extended grid for the gather.
template <typename T>
int launch_fold(const T* Hpart, int KP, long long pstride, const Geo& g,
                const Geo& gf, T* Hper, hipStream_t s);
template <typename T>
int launch_unfold(const T* Htp, const Geo& g, const Geo& gf, T* Ht, hipStream_t s);

// Totals; the real-space input is the sum of its nparts slices.
template <typename T>
int launch_combine(long long N, const T* q_in, const T* phiF, const T* EF,
                   const T* phiR, const T* ER, int nparts, double self_c,
                   unsigned flags, T* phi, T* E, double* partials, int nblk,
                   double* energy, hipStream_t s);

template <typename T>
int launch_check(const T* x, const T* q, long long N, double L1, double L2,
                 int* flag, double* qsum, hipStream_t s);

int launch_fill_int(int* p, long long n, int v, hipStream_t s);

// ---- batches: many independent systems per launch --------------------------
// Particles of all systems are packed system after system; the cell arrays
// of all systems are packed the same way, so one scan over the packed counts
// yields global cell starts whose values index the packed particle arrays.
// Grid-shaped stages run as work queues over (system, tile) items.
template <typename T>
struct SysDesc {
    Geo g;
    BinGeo bg;
    FftDesc dz;
    const SlabDesc* slabs;      // device, offsets relative to G
    T* Hpart;                   // KP partial grids, pstride apart
    cplx<T>* Fz;
    cplx<T>* G;
    T* Ht;
    const T* S0;
    long long pstride;
    long long p0, n;            // packed particle range
    long long cl0, cb0;         // first lex / block cell in the packed cell arrays
    long long e0;               // first energy partial of this system
    int CZ, KP, R, nslab;
    int ncomb;                  // energy partial blocks (256 particles each)
    int rs;                     // real-space sum enabled (rc > 0)
    double xi, rc, self_c;
};

// One queue item: system and up to three tile coordinates.
struct Item {
    int sys, a, b, c;
};

// Stages with work queues, in launch order.
enum BatchQueue {
    kQSpread = 0, kQZfft, kQRowFwd, kQCols, kQRowInv, kQZifft, kQGather,
    kQReal, kQComb, kQEnergy, kNumQueues
};

constexpr int kQCtrStride = 32;   // ints between the queue counters (128 bytes)

struct BatchLaunch {           // one queue stage
    const Item* items;          // device
    const int* qb;              // device: bounds of the 8 per-XCD item ranges
    int nitems;
    int grid;                   // persistent blocks
    size_t lds;                 // dynamic LDS bytes
};

template <typename T>
struct BatchArgs {
    const SysDesc<T>* sys;      // device
    int nsys;
    int P;
    long long ntot;
    const int* sys_of;          // packed particle -> system
    long long ncl, ncb;         // total lex / block cells
    BinBufs bins;               // counting sort over the packed cells
    DevParticles<T> lex, blk;   // packed, start = global cell starts
    T* wz; T* wxp; T* wyq;
    const cplx<T>* tw;
    T* phiF; T* EF; T* phiR; T* ER;
    double* partials;
    int* qctr;                  // 8 counters per queue, kQCtrStride apart
    BatchLaunch q[kNumQueues];
};

template <typename T>
int launch_batch(const BatchArgs<T>& a, const T* x, const T* q, T* phi, T* E,
                 double* energy, unsigned flags, hipStream_t s);

// Blocks of one queue kernel that fit on the device at once.
template <typename T>
int batch_occupancy(int queue, int P, size_t lds, int* blocks_per_cu);

}  // namespace se1p
