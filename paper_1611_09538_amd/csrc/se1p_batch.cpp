// se1p_batch.cpp -- many independent SE1P systems per launch: batch planning
// (packed particles and cells, per-system grids and tables, work-queue items
// ordered largest first), HIP graph capture of the whole evaluation, and the
// cost-model autotuner with its on-device calibration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "se1p_plan.h"

using namespace se1p;

struct se1p_batch {
    int nsys = 0;
    int prec = 0;
    int P = 0;
    size_t es = 8;
    int device = 0;
    hipStream_t stream = nullptr;   // caller's stream (graph launches, eager runs)
    hipStream_t cap = nullptr;      // own stream, used only for capture
    std::vector<se1p_plan> sys;     // geometry of every system (no workspace)
    std::vector<long long> cnt, p0;
    long long ntot = 0, ncl = 0, ncb = 0;
    void* base = nullptr;
    size_t ws_bytes = 0;
    BatchArgs<double> a64{};
    BatchArgs<float> a32{};
    int nitems[kNumQueues] = {};
    int grid[kNumQueues] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[5] = {};
    unsigned key_flags = 0;
    int captures = 0;
};

namespace {

double log2d(double v) { return std::log2(std::max(v, 2.0)); }

// Work of every 1D transform of a planned system, in points x log2(length):
// z transforms (two real columns per complex transform, forward and
// inverse), zero-padded row transforms over Mt1 rows of every slab and the
// fused column passes (forward and inverse) over every padded column.
double fft_work(const se1p_plan& pl) {
    const Geo& g = pl.g;
    double w = (double)g.ncol * g.M3 * log2d(g.M3);
    for (const SlabDesc& sd : pl.slabs) {
        w += 2.0 * g.Mt1 * sd.n2 * log2d(sd.n2);
        w += 2.0 * sd.n2 * sd.n1 * log2d(sd.n1);
    }
    return w;
}

// Expected pairs within rc: N times the particles in a ball of radius rc
// at the mean density (the z-period makes the ball's images count too).
double pair_count(const se1p_params& p, long long N) {
    if (!(p.rc > 0.0)) return 0.0;
    const double V = p.box[0] * p.box[1] * p.box[2];
    return (double)N * (double)N / V * 4.0 / 3.0 * kPi * p.rc * p.rc * p.rc;
}

double predicted_ns(const se1p_cost_model& m, const se1p_plan& pl,
                    long long N) {
    const double P3 = (double)pl.g.P * pl.g.P * pl.g.P;
    return m.pair_ns * pair_count(pl.prm, N) + m.grid_ns * (double)N * P3 +
           m.fft_ns * fft_work(pl) + m.particle_ns * (double)N + m.system_ns;
}

// Built-in coefficients, measured on MI355X with the single-system path
// (stage times of the N = 1e5 unit-box FP64 system, P = 24; FP32 from the
// N = 1e6 2 x 2 x 1 system, P = 12).
se1p_cost_model default_model(int precision) {
    se1p_cost_model m{};
    if (precision == SE1P_FP64) {
        m.pair_ns = 0.024;
        m.grid_ns = 0.0011;
        m.fft_ns = 0.0066;
        m.particle_ns = 0.7;
    } else {
        m.pair_ns = 0.012;
        m.grid_ns = 0.0008;
        m.fft_ns = 0.004;
        m.particle_ns = 0.5;
    }
    m.system_ns = 3000.0;
    return m;
}

bool fft_friendly(int n) {
    int r = n;
    while (r % 2 == 0) r /= 2;
    while (r % 3 == 0) r /= 3;
    while (r % 5 == 0) r /= 5;
    return r == 1;
}

struct Req {
    void** ptr;
    size_t bytes;
};

template <typename T> BatchArgs<T>& args_of(se1p_batch& b);
template <> BatchArgs<double>& args_of<double>(se1p_batch& b) { return b.a64; }
template <> BatchArgs<float>& args_of<float>(se1p_batch& b) { return b.a32; }

template <typename T>
int build_batch(se1p_batch& b) {
    const int ns = b.nsys;
    const size_t es = sizeof(T), cs = 2 * sizeof(T);
    const int P = b.P;
    const int PW = P;                    // x / y weight row (no padding)
    BatchArgs<T>& a = args_of<T>(b);
    a = BatchArgs<T>{};

    // packed particles and cells
    b.p0.resize(ns);
    b.ntot = 0;
    b.ncl = 0;
    b.ncb = 0;
    std::vector<long long> cl0(ns), cb0(ns), e0(ns);
    long long ne = 0;
    for (int s = 0; s < ns; ++s) {
        b.p0[s] = b.ntot;
        b.ntot += b.cnt[s];
        cl0[s] = b.ncl;
        cb0[s] = b.ncb;
        b.ncl += b.sys[s].bg.ncell_lex;
        b.ncb += b.sys[s].bg.ncell_blk;
        e0[s] = ne;
        ne += (b.cnt[s] + 255) / 256;
    }
    if (b.ntot >= (1LL << 31) || b.ncl + 1 >= (1LL << 31) || b.ncb + 1 >= (1LL << 31))
        return SE1P_ERR_UNSUPPORTED;

    // global twiddle table over every length any system uses
    std::map<int, int> gtw;
    long long twn = 0;
    for (auto& pl : b.sys)
        for (auto& kv : pl.twoff)
            if (!gtw.count(kv.first)) { gtw[kv.first] = (int)twn; twn += kv.first; }

    // ---- work items, each with its estimated cost ----
    std::vector<std::pair<double, Item>> it[kNumQueues];
    size_t lds[kNumQueues] = {};
    for (int s = 0; s < ns; ++s) {
        const se1p_plan& pl = b.sys[s];
        const Geo& g = pl.g;
        const BinGeo& bg = pl.bg;
        const double rho = (double)b.cnt[s] / ((double)pl.M1 * pl.M2 * g.M3);
        const int tx = (g.Mt1 + kSpreadTile - 1) / kSpreadTile;
        const int ty = (g.Mt2 + kSpreadTile - 1) / kSpreadTile;
        const double csp = rho * (kSpreadTile + P - 1.0) * (kSpreadTile + P - 1.0) *
                           pl.CZ * P + pl.CZ * P;
        for (int jc = 0; jc < g.M3 / pl.CZ; ++jc)
            for (int i = 0; i < tx; ++i)
                for (int j = 0; j < ty; ++j)
                    it[kQSpread].push_back({csp, Item{s, i, j, jc}});
        const int ncb = (int)((g.ncol + kZfftCols - 1) / kZfftCols);
        const double cz = (double)kZfftCols * g.M3 * log2d(g.M3);
        for (int c = 0; c < ncb; ++c) {
            it[kQZfft].push_back({cz, Item{s, c, 0, 0}});
            it[kQZifft].push_back({cz, Item{s, c, 0, 0}});
        }
        lds[kQZfft] = std::max(lds[kQZfft], 2 * (kZfftCols / 2) * (size_t)(g.M3 + 1) * cs);
        lds[kQZifft] = lds[kQZfft];
        for (int sl = 0; sl < pl.nslab; ++sl) {
            const SlabDesc& sd = pl.slabs[sl];
            // rows / columns per item: about 1024 points per 256-thread
            // item, at least 4 and at most 32 transforms
            const int nrw = std::min(32, std::max(4, 1024 / sd.n2));
            const int ncl = std::min(32, std::max(4, 1024 / (sd.n1 + 1)));
            const double cr = (double)nrw * sd.n2 * log2d(sd.n2);
            for (int r = 0; r < (g.Mt1 + nrw - 1) / nrw; ++r) {
                it[kQRowFwd].push_back({cr, Item{s, r, sl, nrw}});
                it[kQRowInv].push_back({cr, Item{s, r, sl, nrw}});
            }
            const double cc = 2.0 * ncl * sd.n1 * log2d(sd.n1);
            for (int c = 0; c < (sd.n2 + ncl - 1) / ncl; ++c)
                it[kQCols].push_back({cc, Item{s, c, sl, ncl}});
            lds[kQRowFwd] = std::max(lds[kQRowFwd], 2 * (size_t)nrw * sd.n2 * cs);
            lds[kQCols] = std::max(lds[kQCols], 2 * (size_t)ncl * (sd.n1 + 1) * cs);
        }
        lds[kQRowInv] = lds[kQRowFwd];
        // gather units: blocks, or pairs of y-adjacent blocks
        const long long nunit = (long long)bg.nbx * bg.nby * bg.nbz / (1 + bg.pair);
        // a chunk spans about 64 / (rho * BX * BY) z cells of its block (a
        // pair's chunk about 32 / ...: plus one (FP64, cut at layers) or
        // plus the drift of its two runs (FP32))
        const double layer = std::max(rho * bg.BX * bg.BY, 1e-12);
        const double pspan = es == 8 ? 32.0 / layer + 1.0
                                     : 32.0 / layer + 0.9 * std::sqrt(rho * bg.cpb) / layer;
        const double span = std::min((double)bg.BZ, bg.pair ? pspan : 64.0 / layer);
        const double cg = (span + P - 1.0) * P * P;
        for (long long k = 0; k < nunit * bg.CH; ++k)
            it[kQGather].push_back({cg, Item{s, (int)k, 0, 0}});
        const int Ux = bg.BX + P - 1;
        lds[kQGather] = std::max(lds[kQGather], 2 * (size_t)Ux * bg.ldy * es);
        if (pl.prm.rc > 0.0) {
            // chunks of 16 consecutive targets of the system
            const double nb = rho / (g.h * g.h * g.h) * 4.0 / 3.0 * kPi *
                              std::pow(pl.prm.rc + g.h, 3.0);
            for (long long k = 0; k < (b.cnt[s] + 15) / 16; ++k)
                it[kQReal].push_back({16.0 * nb, Item{s, (int)k, 0, 0}});
        }
        for (long long k = 0; k < (b.cnt[s] + 255) / 256; ++k)
            it[kQComb].push_back({1.0, Item{s, (int)k, 0, 0}});
    }
    // Each stage's list (generated in spatial order) is split into 8
    // consecutive ranges of equal estimated cost, one per XCD, each sorted
    // most expensive first.
    std::vector<int> qb(9 * kNumQueues, 0);
    for (int k = 0; k < kNumQueues; ++k) {
        if (it[k].size() >= (size_t)(1 << 30)) return SE1P_ERR_UNSUPPORTED;
        b.nitems[k] = (int)it[k].size();
        double tot = 0.0;
        for (auto& e : it[k]) tot += e.first;
        int r = 1;
        double acc = 0.0;
        for (size_t i = 0; i < it[k].size() && r < 8; ++i) {
            while (r < 8 && acc >= tot * r / 8.0) qb[9 * k + r++] = (int)i;
            acc += it[k][i].first;
        }
        while (r < 8) qb[9 * k + r++] = b.nitems[k];
        qb[9 * k + 8] = b.nitems[k];
        for (int q = 0; q < 8; ++q)
            std::stable_sort(it[k].begin() + qb[9 * k + q], it[k].begin() + qb[9 * k + q + 1],
                             [](const std::pair<double, Item>& u,
                                const std::pair<double, Item>& v) { return u.first > v.first; });
    }
    for (int k = 0; k < kNumQueues; ++k)
        if (lds[k] > 160 * 1024) return SE1P_ERR_UNSUPPORTED;

    // persistent grid sizes from the occupancy of each queue kernel
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b.device) != hipSuccess)
        return SE1P_ERR_HIP;
    for (int k = 0; k < kNumQueues; ++k) {
        if (k == kQEnergy) continue;
        int bpc = 0;
        if (batch_occupancy<T>(k, P, lds[k], &bpc)) return SE1P_ERR_HIP;
        const long long cap = (long long)std::max(bpc, 1) * std::max(ncu, 1);
        // a multiple of 8 blocks: every XCD works on its own range
        b.grid[k] = (int)std::max<long long>(8, cap - cap % 8);
    }

    // ---- workspace ----
    const long long N = std::max<long long>(b.ntot, 1);
    std::vector<Req> req;
    auto add = [&](void** ptr, size_t bytes) { req.push_back({ptr, (bytes + 255) & ~size_t(255)}); };
    BinBufs& bb = a.bins;
    bin_sizes(bb, b.ncl, b.ncb);
    add((void**)&bb.key_lex, N * 4);
    add((void**)&bb.key_blk, N * 4);
    add((void**)&bb.slot, N * 4);
    add((void**)&bb.tmp, N * 4);
    add((void**)&bb.cnt_lex, (bb.ncl + 1) * 4);
    add((void**)&bb.cnt_blk, (bb.ncb + 1) * 4);
    add((void**)&bb.tsum, ((size_t)bb.ntl + bb.ntb) * 4);
    DevParticles<T>* dp[2] = {&a.lex, &a.blk};
    for (DevParticles<T>* d : dp) {
        add((void**)&d->x, N * es);
        add((void**)&d->y, N * es);
        add((void**)&d->z, N * es);
        add((void**)&d->q, N * es);
        add((void**)&d->tx, N * es);
        add((void**)&d->ty, N * es);
        add((void**)&d->tz, N * es);
        add((void**)&d->cx, N * 4);
        add((void**)&d->cy, N * 4);
        add((void**)&d->cz, N * 4);
        add((void**)&d->perm, N * 4);
    }
    add((void**)&a.lex.start, (b.ncl + 1) * 4);
    add((void**)&a.blk.start, (b.ncb + 1) * 4);
    add((void**)&a.wz, (size_t)N * P * es);
    add((void**)&a.wxp, (size_t)N * PW * es);
    add((void**)&a.wyq, (size_t)N * PW * es);
    add((void**)&a.phiF, N * es);
    add((void**)&a.EF, 3 * N * es);
    add((void**)&a.phiR, N * es);
    add((void**)&a.ER, 3 * N * es);
    int* sys_of = nullptr;
    add((void**)&sys_of, N * 4);
    add((void**)&a.partials, (size_t)std::max<long long>(ne, 1) * 8);
    add((void**)&a.qctr, 8 * kQCtrStride * kNumQueues * sizeof(int));
    int* dqb = nullptr;
    add((void**)&dqb, qb.size() * sizeof(int));
    cplx<T>* tw = nullptr;
    add((void**)&tw, (size_t)std::max<long long>(twn, 1) * cs);
    SysDesc<T>* dsys = nullptr;
    add((void**)&dsys, ns * sizeof(SysDesc<T>));
    Item* ditems[kNumQueues] = {};
    for (int k = 0; k < kNumQueues; ++k)
        add((void**)&ditems[k], std::max<size_t>(it[k].size(), 1) * sizeof(Item));
    std::vector<SysDesc<T>> hs(ns);
    std::vector<SlabDesc*> dslabs(ns, nullptr);
    std::vector<T*> dS0(ns, nullptr);
    for (int s = 0; s < ns; ++s) {
        const se1p_plan& pl = b.sys[s];
        SysDesc<T>& d = hs[s];
        const long long pstride = (long long)pl.g.M3 * pl.g.ncol;
        add((void**)&d.Hpart, (size_t)pl.KP * pstride * es);
        add((void**)&d.Fz, (size_t)pl.nslab * pl.g.ncol * cs);
        add((void**)&d.G, (size_t)pl.slab_elems * cs);
        add((void**)&d.Ht, (size_t)(pstride + 64) * es);
        add((void**)&dS0[s], (size_t)pl.n0[0] * pl.n0[1] * es);
        add((void**)&dslabs[s], pl.slabs.size() * sizeof(SlabDesc));
    }
    size_t total = 0;
    for (auto& r : req) total += r.bytes;
    b.ws_bytes = total;
    if (hipMalloc(&b.base, total) != hipSuccess) {
        b.base = nullptr;
        (void)hipGetLastError();
        return SE1P_ERR_NOMEM;
    }
    char* cur = (char*)b.base;
    for (auto& r : req) { *r.ptr = cur; cur += r.bytes; }

    // ---- tables and descriptors ----
    hipError_t e = hipSuccess;
    std::vector<T> twh(2 * std::max<long long>(twn, 1), (T)0);
    for (auto& kv : gtw) {
        const int n = kv.first, o = kv.second;
        for (int k = 0; k < n; ++k) {
            const double ang = -2.0 * kPi * (double)k / (double)n;
            twh[2 * (o + k)] = (T)std::cos(ang);
            twh[2 * (o + k) + 1] = (T)std::sin(ang);
        }
    }
    e = hipMemcpy(tw, twh.data(), twh.size() * es, hipMemcpyHostToDevice);
    std::vector<int> so(N, 0);
    for (int s = 0; s < ns; ++s)
        std::fill(so.begin() + b.p0[s], so.begin() + b.p0[s] + b.cnt[s], s);
    if (e == hipSuccess) e = hipMemcpy(sys_of, so.data(), N * 4, hipMemcpyHostToDevice);
    for (int s = 0; s < ns && e == hipSuccess; ++s) {
        se1p_plan& pl = b.sys[s];
        std::vector<double> twl, s0;
        plan_tables(pl, twl, s0);
        std::vector<T> s0t(s0.begin(), s0.end());
        e = hipMemcpy(dS0[s], s0t.data(), s0t.size() * es, hipMemcpyHostToDevice);
        std::vector<SlabDesc> sl = pl.slabs;
        for (SlabDesc& d : sl) {
            d.d1.twoff = gtw[d.n1];
            d.d2.twoff = gtw[d.n2];
        }
        if (e == hipSuccess)
            e = hipMemcpy(dslabs[s], sl.data(), sl.size() * sizeof(SlabDesc), hipMemcpyHostToDevice);
        SysDesc<T>& d = hs[s];
        d.g = pl.g;
        d.bg = pl.bg;
        d.dz = pl.dz;
        d.dz.twoff = gtw[pl.dz.n];
        d.slabs = dslabs[s];
        d.S0 = dS0[s];
        d.pstride = (long long)pl.g.M3 * pl.g.ncol;
        d.p0 = b.p0[s];
        d.n = b.cnt[s];
        d.cl0 = cl0[s];
        d.cb0 = cb0[s];
        d.e0 = e0[s];
        d.CZ = pl.CZ;
        d.KP = pl.KP;
        d.R = pl.prm.rc > 0.0 ? (int)std::ceil(pl.prm.rc / pl.g.h) : 0;
        d.nslab = pl.nslab;
        d.ncomb = (int)((b.cnt[s] + 255) / 256);
        d.rs = pl.prm.rc > 0.0 ? 1 : 0;
        d.xi = pl.prm.xi;
        d.rc = pl.prm.rc;
        d.self_c = 2.0 * pl.prm.xi / std::sqrt(kPi);
    }
    if (e == hipSuccess) e = hipMemcpy(dsys, hs.data(), ns * sizeof(SysDesc<T>), hipMemcpyHostToDevice);
    for (int k = 0; k < kNumQueues && e == hipSuccess; ++k) {
        std::vector<Item> v(it[k].size());
        for (size_t i = 0; i < v.size(); ++i) v[i] = it[k][i].second;
        if (!v.empty())
            e = hipMemcpy(ditems[k], v.data(), v.size() * sizeof(Item), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = hipMemcpy(dqb, qb.data(), qb.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return SE1P_ERR_HIP;

    a.sys = dsys;
    a.nsys = ns;
    a.P = P;
    a.ntot = b.ntot;
    a.sys_of = sys_of;
    a.ncl = b.ncl;
    a.ncb = b.ncb;
    a.tw = tw;
    for (int k = 0; k < kNumQueues; ++k) {
        a.q[k].items = ditems[k];
        a.q[k].qb = dqb + 9 * k;
        a.q[k].nitems = b.nitems[k];
        a.q[k].grid = b.grid[k];
        a.q[k].lds = lds[k];
    }
    return SE1P_OK;
}

int run_batch(se1p_batch& b, hipStream_t s, const void* x, const void* q,
              void* phi, void* E, double* energy, unsigned flags) {
    const unsigned comp = flags & (SE1P_ALL | SE1P_FORCE);
    if (b.prec == SE1P_FP64)
        return launch_batch<double>(b.a64, (const double*)x, (const double*)q,
                                    (double*)phi, (double*)E, energy, comp, s);
    return launch_batch<float>(b.a32, (const float*)x, (const float*)q,
                               (float*)phi, (float*)E, energy, comp, s);
}

void drop_graph(se1p_batch& b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
}

// Deterministic probe system for the calibration (splitmix64 stream).
struct SplitMix {
    unsigned long long s;
    unsigned long long next() {
        unsigned long long z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

}  // namespace

extern "C" {

int se1p_autotune(double tol, int nsys, const double* boxes,
                  const long long* counts, const double* Q, int precision,
                  int P, const se1p_cost_model* model, se1p_params* out) {
    if (nsys < 1 || !boxes || !counts || !out || !(tol > 0.0) || !(tol < 1.0))
        return SE1P_ERR_ARG;
    if (precision != SE1P_FP64 && precision != SE1P_FP32) return SE1P_ERR_ARG;
    if (P < 4 || P > kMaxP || (P & 1)) return SE1P_ERR_ARG;
    const se1p_cost_model m = model ? *model : default_model(precision);
    for (int s = 0; s < nsys; ++s) {
        if (counts[s] < 1) return SE1P_ERR_ARG;
        const double* box = boxes + 3 * s;
        const double Qs = Q ? Q[s] : (double)counts[s];
        double best = 1e300;
        se1p_params bp{};
        bool found = false;
        int worse = 0;
        for (int M3 = std::max(P + (P & 1), 8); M3 <= 1024; M3 += 2) {
            if (!fft_friendly(M3)) continue;
            se1p_params p{};
            if (se1p_suggest_params(tol, box, counts[s], Qs, 0.0, M3, P, -1,
                                    precision, &p) != SE1P_OK)
                continue;
            se1p_plan pl;
            if (plan_geometry(pl, p, counts[s]) != SE1P_OK) continue;
            const double c = predicted_ns(m, pl, counts[s]);
            if (c < best) {
                best = c;
                bp = p;
                found = true;
                worse = 0;
            } else if (found && ++worse >= 6) {
                break;   // past the minimum: the grid terms only grow
            }
        }
        if (!found) return SE1P_ERR_UNSUPPORTED;
        out[s] = bp;
    }
    return SE1P_OK;
}

int se1p_calibrate(double tol, int precision, int P, void* stream,
                   se1p_cost_model* out) {
    if (!out || !(tol > 0.0) || !(tol < 1.0)) return SE1P_ERR_ARG;
    if (precision != SE1P_FP64 && precision != SE1P_FP32) return SE1P_ERR_ARG;
    const long long N = 20000;
    const double box[3] = {1.0, 1.0, 1.0};
    se1p_params p{};
    const double one = (double)N;
    int rc = se1p_autotune(tol, 1, box, &N, &one, precision, P, nullptr, &p);
    if (rc) return rc;
    // probe: uniform positions, +-1 charges in equal numbers
    std::vector<double> xd(3 * N), qd(N);
    SplitMix g{12345};
    for (long long i = 0; i < N; ++i) {
        for (int d = 0; d < 3; ++d) xd[3 * i + d] = std::min(g.uniform() * box[d], std::nextafter(box[d], 0.0));
        qd[i] = (i & 1) ? 1.0 : -1.0;
    }
    const size_t es = precision == SE1P_FP64 ? 8 : 4;
    std::vector<float> xf(xd.begin(), xd.end()), qf(qd.begin(), qd.end());
    const void* hx = es == 8 ? (const void*)xd.data() : (const void*)xf.data();
    const void* hq = es == 8 ? (const void*)qd.data() : (const void*)qf.data();
    void *dx = nullptr, *dq = nullptr, *dphi = nullptr, *dE = nullptr;
    se1p_plan* pl = nullptr;
    auto cleanup = [&]() {
        if (pl) se1p_plan_destroy(pl);
        if (dx) (void)hipFree(dx);
        if (dq) (void)hipFree(dq);
        if (dphi) (void)hipFree(dphi);
        if (dE) (void)hipFree(dE);
    };
    if (hipMalloc(&dx, 3 * N * es) != hipSuccess || hipMalloc(&dq, N * es) != hipSuccess ||
        hipMalloc(&dphi, N * es) != hipSuccess || hipMalloc(&dE, 3 * N * es) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return SE1P_ERR_NOMEM;
    }
    if (hipMemcpy(dx, hx, 3 * N * es, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dq, hq, N * es, hipMemcpyHostToDevice) != hipSuccess) {
        cleanup();
        return SE1P_ERR_HIP;
    }
    if ((rc = se1p_plan_create(&p, N, stream, &pl))) { pl = nullptr; cleanup(); return rc; }
    rc = se1p_eval(pl, N, dx, dq, dphi, dE, nullptr, SE1P_ALL);   // warm-up
    if (!rc) rc = se1p_timing_enable(pl, 1);
    for (int k = 0; k < 5 && !rc; ++k) rc = se1p_eval(pl, N, dx, dq, dphi, dE, nullptr, SE1P_ALL);
    double ms[SE1P_NSTAGE] = {};
    int nc = 0;
    if (!rc) rc = se1p_timing_read(pl, ms, &nc);
    if (rc || nc < 1) { cleanup(); return rc ? rc : SE1P_ERR_HIP; }
    const double ns = 1e6 / nc;   // ms summed over nc calls -> ns per call
    se1p_cost_model m = default_model(precision);
    const double P3 = (double)P * P * P;
    const double pairs = pair_count(pl->prm, N);
    if (pairs > 0.0) m.pair_ns = ms[4] * ns / pairs;
    m.grid_ns = (ms[1] + ms[3]) * ns / ((double)N * P3);
    m.fft_ns = ms[2] * ns / fft_work(*pl);
    m.particle_ns = (ms[0] + ms[5]) * ns / (double)N;
    cleanup();
    *out = m;
    return SE1P_OK;
}

int se1p_batch_create(int nsys, const se1p_params* params,
                      const long long* counts, void* stream,
                      se1p_batch** out) {
    if (!out) return SE1P_ERR_ARG;
    *out = nullptr;
    if (nsys < 1 || !params || !counts) return SE1P_ERR_ARG;
    for (int s = 0; s < nsys; ++s) {
        if (counts[s] < 1 || counts[s] > (1LL << 30)) return SE1P_ERR_ARG;
        int rc = plan_check_params(params[s]);
        if (rc) return rc;
        if (params[s].precision != params[0].precision || params[s].P != params[0].P)
            return SE1P_ERR_PARAM;
    }
    se1p_batch* b = new (std::nothrow) se1p_batch();
    if (!b) return SE1P_ERR_NOMEM;
    b->nsys = nsys;
    b->prec = params[0].precision;
    b->P = params[0].P;
    b->es = b->prec == SE1P_FP64 ? 8 : 4;
    b->stream = (hipStream_t)stream;
    b->cnt.assign(counts, counts + nsys);
    b->sys.resize(nsys);
    int rc = SE1P_OK;
    if (hipGetDevice(&b->device) != hipSuccess) rc = SE1P_ERR_HIP;
    for (int s = 0; s < nsys && !rc; ++s) {
        b->sys[s].in_batch = true;
        rc = plan_geometry(b->sys[s], params[s], counts[s]);
    }
    if (!rc) rc = b->prec == SE1P_FP64 ? build_batch<double>(*b) : build_batch<float>(*b);
    if (!rc && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        b->cap = nullptr;
        rc = SE1P_ERR_HIP;
    }
    if (rc) {
        if (b->base) (void)hipFree(b->base);
        if (b->cap) (void)hipStreamDestroy(b->cap);
        delete b;
        return rc;
    }
    *out = b;
    return SE1P_OK;
}

int se1p_batch_destroy(se1p_batch* b) {
    if (!b) return SE1P_ERR_ARG;
    int rc = SE1P_OK;
    if (hipSetDevice(b->device) != hipSuccess) rc = SE1P_ERR_HIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) rc = SE1P_ERR_HIP;
    drop_graph(*b);
    if (b->cap && hipStreamDestroy(b->cap) != hipSuccess) rc = SE1P_ERR_HIP;
    if (b->base && hipFree(b->base) != hipSuccess) rc = SE1P_ERR_HIP;
    delete b;
    return rc;
}

int se1p_batch_eval(se1p_batch* b, const void* x, const void* q, void* phi,
                    void* efield, double* energy, unsigned flags) {
    if (!b || !x || !q) return SE1P_ERR_ARG;
    if (flags & ~(SE1P_ALL | SE1P_BATCH_EAGER | SE1P_FORCE)) return SE1P_ERR_ARG;
    if ((flags & SE1P_ALL) == 0) return SE1P_ERR_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return SE1P_ERR_HIP;
    if (flags & SE1P_BATCH_EAGER) return run_batch(*b, b->stream, x, q, phi, efield, energy, flags);
    const void* key[5] = {x, q, phi, efield, energy};
    const bool same = b->exec && b->key_flags == flags &&
                      std::equal(key, key + 5, b->key);
    if (!same) {
        drop_graph(*b);
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return SE1P_ERR_HIP;
        int rc = run_batch(*b, b->cap, x, q, phi, efield, energy, flags);
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->cap, &gr);
        if (rc || ec != hipSuccess || !gr) {
            if (gr) (void)hipGraphDestroy(gr);
            (void)hipGetLastError();
            return rc ? rc : SE1P_ERR_HIP;
        }
        b->graph = gr;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            b->exec = nullptr;
            drop_graph(*b);
            return SE1P_ERR_HIP;
        }
        std::copy(key, key + 5, b->key);
        b->key_flags = flags;
        ++b->captures;
    }
    return hipGraphLaunch(b->exec, b->stream) == hipSuccess ? SE1P_OK : SE1P_ERR_HIP;
}

int se1p_batch_get_info(const se1p_batch* b, se1p_batch_info* info) {
    if (!b || !info) return SE1P_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->nsys = b->nsys;
    info->precision = b->prec;
    info->P = b->P;
    info->n_total = b->ntot;
    info->workspace_bytes = b->ws_bytes;
    for (int k = 0; k < kNumQueues && k < 10; ++k) {
        info->items[k] = b->nitems[k];
        info->grid[k] = b->grid[k];
    }
    info->graph_captures = b->captures;
    return SE1P_OK;
}

int se1p_batch_system_info(const se1p_batch* b, int s, se1p_params* params,
                           se1p_plan_info* info) {
    if (!b || s < 0 || s >= b->nsys) return SE1P_ERR_ARG;
    if (params) *params = b->sys[s].prm;
    if (info) return se1p_plan_get_info(&b->sys[s], info);
    return SE1P_OK;
}

}  // extern "C"
