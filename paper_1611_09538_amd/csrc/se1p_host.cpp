// se1p_host.cpp -- host side of the SE1P library: parameter selection,
// planning (grid geometry, padded FFT sizes, FP64 k3 = 0 scaling table, FFT
// tables), workspace, argument checks and the C ABI of include/se1p.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "se1p_plan.h"

using namespace se1p;

namespace {

constexpr double kShapeC = 0.95;  // c in eq. comp_eta

// smallest integer >= n whose only prime factors are 2, 3, 5
int nice_size(int n) {
    if (n < 1) n = 1;
    for (int m = n;; ++m) {
        int r = m;
        while (r % 2 == 0) r /= 2;
        while (r % 3 == 0) r /= 3;
        while (r % 5 == 0) r /= 5;
        if (r == 1) return m;
    }
}

bool factorize(int n, FftDesc& d) {
    d.n = n;
    d.nrad = 0;
    int r = n;
    auto push = [&](int f) {
        if (d.nrad >= kMaxRad) return false;
        d.rad[d.nrad++] = f;
        return true;
    };
    while (r % 4 == 0) { if (!push(4)) return false; r /= 4; }
    while (r % 2 == 0) { if (!push(2)) return false; r /= 2; }
    while (r % 3 == 0) { if (!push(3)) return false; r /= 3; }
    while (r % 5 == 0) { if (!push(5)) return false; r /= 5; }
    return r == 1;
}

// Fourier transform of the truncated 2D Green's function
// (eqs. g_zeromod, g_zeromod0), FP64.
double G_R(double kappa, double R) {
    const double x = R * kappa;
    if (kappa == 0.0) return R * R / 4.0 * (1.0 - 2.0 * std::log(R));
    if (x < 1e-3) {
        // series: (1 - J0(x))/k^2 = R^2/4 (1 - x^2/16 + x^4/576),
        //         J1(x)/k        = R/2 (1 - x^2/8 + x^4/192)
        const double x2 = x * x;
        const double a = R * R / 4.0 * (1.0 - x2 / 16.0 + x2 * x2 / 576.0);
        const double b = R * std::log(R) * R / 2.0 * (1.0 - x2 / 8.0 + x2 * x2 / 192.0);
        return a - b;
    }
    return (1.0 - ::j0(x)) / (kappa * kappa) - R * std::log(R) * ::j1(x) / kappa;
}

double lambert_w(double x) {  // principal branch, x >= 0
    if (x <= 0.0) return 0.0;
    double w = x < 1.0 ? x : std::log(x) - std::log(std::log(x) + 1.0);
    if (w < 0.0) w = 0.0;
    for (int i = 0; i < 100; ++i) {
        const double ew = std::exp(w);
        const double f = w * ew - x;
        const double wn = w - f / (ew * (w + 1.0) - (w + 2.0) * f / (2.0 * w + 2.0));
        if (std::fabs(wn - w) < 1e-15 * (1.0 + std::fabs(wn))) return wn;
        w = wn;
    }
    return w;
}

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace


namespace {
constexpr int kTimingMaxCalls = 4096;

// boundary b opens stage b and closes stage b - 1: its event is recorded
// only when one of the two is selected
void tmark(se1p_plan& pl, int boundary) {
    if (!pl.timing || pl.tcalls >= kTimingMaxCalls) return;
    const unsigned near = (pl.tstages << 1 | pl.tstages) >> boundary;
    if (!(near & 1u)) return;
    const size_t k = (size_t)pl.tcalls * (SE1P_NSTAGE + 1) + boundary;
    if (k < pl.tev.size()) (void)hipEventRecord(pl.tev[k], pl.stream);
}
}  // namespace

namespace {

int check_params(const se1p_params& p) {
    for (int d = 0; d < 3; ++d)
        if (!(p.box[d] > 0.0) || !std::isfinite(p.box[d])) return SE1P_ERR_PARAM;
    if (!(p.xi > 0.0) || !std::isfinite(p.xi)) return SE1P_ERR_PARAM;
    if (p.M3 < 4 || (p.M3 & 1)) return SE1P_ERR_PARAM;
    if (p.P < 4 || p.P > kMaxP || (p.P & 1) || p.P > p.M3) return SE1P_ERR_PARAM;
    if (p.n_l < 0) return SE1P_ERR_PARAM;
    if (!(p.s_l >= 1.0) || !(p.s_l <= 16.0)) return SE1P_ERR_PARAM;
    if (!(p.s0 >= 0.0) || !(p.s0 <= 16.0)) return SE1P_ERR_PARAM;
    if (!(p.rc >= 0.0) || !std::isfinite(p.rc)) return SE1P_ERR_PARAM;
    if (p.precision != SE1P_FP64 && p.precision != SE1P_FP32) return SE1P_ERR_PARAM;
    if (p.pad_free < 0 || p.pad_free > 1024) return SE1P_ERR_PARAM;
    const double h = p.box[2] / p.M3;
    for (int d = 0; d < 2; ++d) {
        const double m = std::ceil(p.box[d] / h - 1e-9);
        if (m > 4096) return SE1P_ERR_PARAM;
    }
    return SE1P_OK;
}

// Gather block shape: lanes are particles and every lane sweeps the union of
// the supports of its chunk (64 consecutive particles of a block), so a
// chunk should be full while its z extent stays small.  Expected cost per
// particle: E[chunks] * union / m, with Poisson counts of mean m = rho *
// cells, penalised when the launch would not fill the chip.
double poisson_chunks(double m, int size = 64) {
    // E[ceil(k / size)] for k ~ Poisson(m); for large m, m / size + 1/2
    if (m > 400.0) return m / size + 0.5;
    double pk = std::exp(-m), acc = 0.0;
    const int kmax = (int)(m + 12.0 * std::sqrt(m + 1.0) + 80.0);
    for (int k = 0; k <= kmax; ++k) {
        if (k > 0) pk *= m / k;
        acc += pk * ((k + size - 1) / size);
    }
    return acc;
}

// fill: apply the penalty for launches too small to fill the chip (a system
// on its own); mt1, mt2 > 0: only blocks whose footprint fits an extended
// grid of that size (nb * B + P <= Mt).
void choose_blocks(se1p_plan& pl, bool fill, int mt1, int mt2) {
    // Each chunk stages BZ + P - 1 grid planes of (BX + P - 1) x (BY + P - 1)
    // values in LDS and every lane reads its own P x P window of each plane
    // its z support covers.  The LDS serves 128 bytes per cycle from 32
    // four-byte banks: 32 lanes per cycle for 4-byte words, 16 for 8-byte
    // words.  With nb = 128 / word size, blocks keep BX * BY <= nb and the
    // LDS pitch == BY (mod nb); the window origins of distinct (x, y) cells
    // then fall in distinct banks, and lanes of one cell read the same
    // address, so the window reads are free of bank conflicts.  Blocks may
    // be tall in z (up to whole columns): particles are sorted by z inside a
    // block, so a chunk of 64 spans about 64 / (rho * BX * BY) z cells and
    // sweeps that many planes plus P - 1.  Cost per particle: planes swept
    // per chunk times chunks over the particles per block, with Poisson
    // counts of mean m = rho * cells, penalised when the launch has fewer
    // waves than the chip has SIMDs.  A gather unit may also take two
    // y-adjacent blocks at once, 32 particles of each per chunk in lanes
    // 0-31 and 32-63: a 16- or 32-lane LDS cycle then still reads windows
    // of one block's cells only, and a chunk spans about half the z cells
    // (plus the drift between the two blocks' runs), over a footprint
    // BY cells wider.
    const double ncells = (double)pl.M1 * pl.M2 * pl.g.M3;
    const double rho = (double)std::max<long long>(pl.n_max, 1) / ncells;
    const int P = pl.g.P;
    double best = 1e300;
    const int bymin = std::max(2, 16 / (int)pl.es);   // whole 16-byte chunks
    const int nbank = 128 / (int)pl.es;
    int bx = 1, by = bymin, bz = 1, ch = 1, pair = 0;
    const int bys[4] = {2, 4, 8, 16};
    std::vector<int> bzs;
    for (int z = 1; z < pl.g.M3; z *= 2)
        if (pl.g.M3 % z == 0) bzs.push_back(z);
    bzs.push_back(pl.g.M3);
    // Cost of a block shape, with pr = 1 for units of two y-adjacent blocks
    // (nby even).  FP64 cuts a pair's chunks at z-layer boundaries where
    // neither block has more than 32 particles (on average a layer's worth
    // short of 32); FP32 takes runs of 32 from each block, which drift
    // apart in z like a random walk.
    const bool layer_cut = pl.es == 8;
    auto shape_cost = [&](int BX, int BY, int BZ, int pr, int& chs) {
        const double m = rho * BX * BY * BZ;
        const int nby = (pl.M2 + BY - 1) / BY;
        const double nblocks = (double)((pl.M1 + BX - 1) / BX) * nby * (pl.g.M3 / BZ);
        const double layer = std::max(rho * BX * BY, 1e-12);   // particles per z cell
        double per = 64.0, chunks = std::max(poisson_chunks(m, 64), 1e-9), span = per / layer;
        if (pr && layer_cut) {
            per = std::max(32.0 - 0.75 * std::min(layer, 32.0), 8.0);
            chunks = m / per + 0.5;
            span = per / layer + 1.0;
        } else if (pr) {
            per = 32.0;
            chunks = poisson_chunks(m, 32) + 0.3;
            span = per / layer + 0.9 * std::sqrt(m) / layer;
        }
        span = std::min((double)BZ, span);
        const double planes = span + P - 1.0;
        const double foot = (BX + P - 1.0) * ((1 + pr) * BY + P - 1.0);
        const double work = chunks * (planes * P * P * 2.0 + planes * foot / 16.0);
        double cost = (work + 200.0) / std::max((1 + pr) * m, 1e-6);
        const double waves = nblocks / (1 + pr) * chunks;
        if (fill && waves < 1024.0) cost *= 1024.0 / std::max(waves, 1.0);
        // waves per unit: enough for the chunks of a block 3 sigma above the
        // mean; FP32 pairs half as many again (shorter waves, 4% faster
        // at N = 1e6; FP64 pairs 2% slower with them)
        chs = std::max(1, (int)std::ceil((pr && !layer_cut ? 1.5 : 1.0) *
                                         (m + 3.0 * std::sqrt(m) + 1.0) / per));
        return cost;
    };
    // The shape is chosen for single blocks (it also shapes the chunks of
    // real-space targets, which follow the block order); the pairing is
    // then taken for that shape if it costs less.
    for (size_t iz = 0; iz < bzs.size(); ++iz) {
        const int BZ = bzs[iz];
        for (int iy = 0; iy < 4; ++iy) {
            const int BY = bys[iy];
            // planes are staged in 16-byte chunks: with ldy == BY (mod nb)
            // the pitch holds whole chunks only if BY does
            if ((BY * (int)pl.es) % 16) continue;
            for (int BX = 1; BX * BY <= nbank; ++BX) {
                if (mt1 > 0 && ((pl.M1 + BX - 1) / BX) * BX + P > mt1) continue;
                if (mt2 > 0 && ((pl.M2 + BY - 1) / BY) * BY + P > mt2) continue;
                int chs;
                const double cost = shape_cost(BX, BY, BZ, 0, chs);
                if (cost < best) {
                    best = cost; bx = BX; by = BY; bz = BZ; ch = chs;
                }
            }
        }
    }
    // (a pair's chunk walk holds the layer counts of 64 kMaxLayerGroups - 1
    // z cells at most)
    if (((pl.M2 + by - 1) / by) % 2 == 0 && (!layer_cut || bz < 64 * kMaxLayerGroups)) {
        int chs;
        if (shape_cost(bx, by, bz, 1, chs) < best) {
            pair = 1;
            ch = chs;
        }
    }
    BinGeo& b = pl.bg;
    b.BX = bx; b.BY = by; b.BZ = bz; b.CH = ch; b.pair = pair;
    const int Uy = (1 + pair) * by + P - 1;
    b.ldy = Uy + (((by - Uy) % nbank) + nbank) % nbank;   // >= Uy, == BY (mod nb)
    b.nbx = (pl.M1 + bx - 1) / bx;
    b.nby = (pl.M2 + by - 1) / by;
    b.nbz = pl.g.M3 / bz;
    b.cpb = bx * by * bz;
    b.ncell_lex = (long long)pl.g.M3 * pl.M1 * pl.M2;
    b.ncell_blk = (long long)b.nbx * b.nby * b.nbz * b.cpb;
}

// Spread chunking: CZ z-cells per wave, KP partial grids with KP | M3/CZ and
// KP*CZ >= CZ + P - 1.  Prefer enough waves to fill the chip, then fewer
// partial grids, then the smaller CZ.  Every divisor of M3 up to 10 is a
// candidate.  With powers of two only, an M3 such as 50 or 90 left CZ = 2
// and KP = 25 or 9: partial grids that gridding writes and the z transform
// reads back in full (the 64-system batch: 2.70 against 2.34 ms).  Chunks of
// 16 cells were slower, with their waves too long and too few (FP64, P 16:
// 0.47 against 0.40 ms at M3 = 64).
void choose_spread(se1p_plan& pl) {
    const int M3 = pl.g.M3, P = pl.g.P;
    const long long tiles = (long long)((pl.g.Mt1 + 7) / 8) * ((pl.g.Mt2 + 7) / 8);
    int bestCZ = 1, bestKP = M3;
    double bestScore = -1e300;
    for (int CZ = 1; CZ <= 10; ++CZ) {
        if (M3 % CZ) continue;
        const int ncz = M3 / CZ;
        const int need = (CZ + P - 1 + CZ - 1) / CZ;
        int KP = -1;
        for (int k = need; k <= ncz; ++k)
            if (ncz % k == 0) { KP = k; break; }
        if (KP < 0) continue;
        const double waves = (double)tiles * ncz * spread_waves(P);
        const double fill = pl.in_batch ? 1.0 : std::min(1.0, waves / 2048.0);
        const double score = fill * 4.0 - 0.05 * KP;
        if (score > bestScore) { bestScore = score; bestCZ = CZ; bestKP = KP; }
    }
    pl.CZ = bestCZ;
    pl.KP = bestKP;
}

template <typename T>
DevParticles<T> particles(const se1p_plan& pl, bool lex) {
    DevParticles<T> d;
    void* const* f = lex ? pl.w.lex_f : pl.w.blk_f;
    int* const* i = lex ? pl.w.lex_i : pl.w.blk_i;
    d.x = (T*)f[0]; d.y = (T*)f[1]; d.z = (T*)f[2]; d.q = (T*)f[3];
    d.tx = (T*)f[4]; d.ty = (T*)f[5]; d.tz = (T*)f[6];
    d.cx = i[0]; d.cy = i[1]; d.cz = i[2]; d.perm = i[3]; d.start = i[4];
    return d;
}

}  // namespace

int se1p::plan_check_params(const se1p_params& p) { return check_params(p); }

int se1p::plan_geometry(se1p_plan& pl, const se1p_params& p, long long n_max) {
    pl.prm = p;
    pl.prec = p.precision;
    pl.es = (p.precision == SE1P_FP64) ? 8 : 4;
    pl.n_max = n_max;
    Geo& g = pl.g;
    g.M3 = p.M3;
    g.P = p.P;
    g.L3 = p.box[2];
    g.h = p.box[2] / p.M3;
    g.inv_h = 1.0 / g.h;
    g.xi = p.xi;
    g.eta = p.P * p.xi * p.xi * g.h * g.h / (kShapeC * kShapeC * kPi);
    g.alpha = 2.0 * p.xi * p.xi / g.eta;
    pl.cg = std::pow(2.0 * p.xi * p.xi / (kPi * g.eta), 1.5);
    pl.M1 = (int)std::ceil(p.box[0] / g.h - 1e-9);
    pl.M2 = (int)std::ceil(p.box[1] / g.h - 1e-9);
    if (pl.M1 < 1) pl.M1 = 1;
    if (pl.M2 < 1) pl.M2 = 1;
    g.M1 = pl.M1;
    g.M2 = pl.M2;
    choose_blocks(pl, true, 0, 0);
    // Extended grid: M + P plus room for whole gather blocks, FFT-friendly.
    g.Mt1 = nice_size(std::max(pl.bg.nbx * pl.bg.BX + p.P, pl.M1 + p.P + p.pad_free));
    g.Mt2 = nice_size(std::max(pl.bg.nby * pl.bg.BY + p.P, pl.M2 + p.P + p.pad_free));
    // A batch member keeps the grid (so the discretisation) of the system
    // planned alone, and picks its gather blocks without the chip-fill
    // penalty among those that fit that grid.
    if (pl.in_batch) choose_blocks(pl, false, g.Mt1, g.Mt2);
    // the gather stages planes of Ux x ldy values in 16-byte chunks that
    // must not straddle LDS rows
    if ((pl.bg.ldy * pl.es) % 16 != 0) return SE1P_ERR_UNSUPPORTED;
    g.ncol = (long long)g.Mt1 * g.Mt2;
    choose_spread(pl);

    // Transform geometry.  SE3P transforms the periodic grid itself: the
    // gridded values are folded onto M1 x M2 x M3 and every slab is a plain
    // M1 x M2 transform, with Ghat = 1/k^2 for all k != 0.
    pl.gf = g;
    if (pl.periodic3) {
        pl.gf.Mt1 = pl.M1;
        pl.gf.Mt2 = pl.M2;
        pl.gf.ncol = (long long)pl.M1 * pl.M2;
    }
    const Geo& gf = pl.gf;

    // k3 = 0 slab: R spans the support region; the padded period must hold
    // the support plus R (section 3.2; s0 >= 1 + sqrt 2 for a square).
    const double e1 = (pl.M1 + p.P) * g.h, e2 = (pl.M2 + p.P) * g.h;
    pl.R = std::hypot(e1, e2);
    const int rcell = (int)std::ceil(pl.R / g.h - 1e-9);
    pl.n0[0] = nice_size(std::max({(int)std::ceil(p.s0 * (pl.M1 + p.P) - 1e-9),
                                   pl.M1 + p.P + rcell, g.Mt1}));
    pl.n0[1] = nice_size(std::max({(int)std::ceil(p.s0 * (pl.M2 + p.P) - 1e-9),
                                   pl.M2 + p.P + rcell, g.Mt2}));
    pl.nl[0] = nice_size(std::max((int)std::ceil(p.s_l * (pl.M1 + p.P) - 1e-9), g.Mt1));
    pl.nl[1] = nice_size(std::max((int)std::ceil(p.s_l * (pl.M2 + p.P) - 1e-9), g.Mt2));
    if (pl.periodic3) {
        pl.R = 0.0;
        pl.n0[0] = pl.nl[0] = pl.M1;
        pl.n0[1] = pl.nl[1] = pl.M2;
    }
    if (std::max({pl.n0[0], pl.n0[1], pl.nl[0], pl.nl[1]}) > 4096)
        return SE1P_ERR_UNSUPPORTED;

    // slabs n3 = 0 .. M3/2 (eq. upsamplings)
    pl.nslab = p.M3 / 2 + 1;
    pl.slabs.resize(pl.nslab);
    std::map<int, int>& twoff = pl.twoff;   // length -> offset
    twoff.clear();
    long long twn = 0;
    auto tw_of = [&](int n) {
        auto it = twoff.find(n);
        if (it != twoff.end()) return it->second;
        twoff[n] = (int)twn;
        twn += n;
        return (int)(twn - n);
    };
    if (!factorize(p.M3, pl.dz)) return SE1P_ERR_UNSUPPORTED;
    pl.dz.twoff = tw_of(p.M3);
    long long off = 0;
    for (int s = 0; s < pl.nslab; ++s) {
        SlabDesc& sd = pl.slabs[s];
        sd.n3 = s;
        if (s == 0) { sd.n1 = pl.n0[0]; sd.n2 = pl.n0[1]; }
        else if (s <= p.n_l) { sd.n1 = pl.nl[0]; sd.n2 = pl.nl[1]; }
        else { sd.n1 = gf.Mt1; sd.n2 = gf.Mt2; }
        sd.pad_ = 0;
        sd.off = off;
        off += (long long)gf.Mt1 * sd.n2;
        sd.pref = 4.0 * kPi * g.h * g.h * g.h * pl.cg * pl.cg /
                  ((double)p.M3 * sd.n1 * sd.n2);
        if (!factorize(sd.n1, sd.d1) || !factorize(sd.n2, sd.d2))
            return SE1P_ERR_UNSUPPORTED;
        sd.d1.twoff = tw_of(sd.n1);
        sd.d2.twoff = tw_of(sd.n2);
    }
    pl.slab_elems = off;
    pl.tw_elems = twn;

    // LDS limits of the transform kernels
    const size_t cs = 2 * pl.es;
    int n1max = 0, n2max = 0;
    for (auto& sd : pl.slabs) { n1max = std::max(n1max, sd.n1); n2max = std::max(n2max, sd.n2); }
    const size_t lds_z = 2 * (kZfftCols / 2) * (size_t)(p.M3 + 1) * cs;
    const size_t lds_r = 2 * 4 * (size_t)n2max * cs;
    const size_t lds_c = 2 * 4 * (size_t)(n1max + 1) * cs;
    if (std::max({lds_z, lds_r, lds_c}) > 160 * 1024) return SE1P_ERR_UNSUPPORTED;
    return SE1P_OK;
}

void se1p::plan_tables(const se1p_plan& pl, std::vector<double>& twd,
                       std::vector<double>& s0) {
    const Geo& g = pl.g;
    twd.assign(2 * pl.tw_elems, 0.0);
    for (auto& kv : pl.twoff) {
        const int n = kv.first, o = kv.second;
        for (int k = 0; k < n; ++k) {
            const double ang = -2.0 * kPi * (double)k / (double)n;
            twd[2 * (o + k)] = std::cos(ang);
            twd[2 * (o + k) + 1] = std::sin(ang);
        }
    }
    const int a0 = pl.n0[0], b0 = pl.n0[1];
    s0.assign(a0 * (size_t)b0, 0.0);
    const SlabDesc& z0 = pl.slabs[0];
    for (int kx = 0; kx < a0; ++kx) {
        const int fx = (kx <= a0 / 2) ? kx : kx - a0;
        const double k1 = 2.0 * kPi * fx / (a0 * g.h);
        for (int ky = 0; ky < b0; ++ky) {
            const int fy = (ky <= b0 / 2) ? ky : ky - b0;
            const double k2 = 2.0 * kPi * fy / (b0 * g.h);
            const double kap2 = k1 * k1 + k2 * k2;
            // SE1P: truncated Green's function of the k3 = 0 mode; SE3P:
            // the k3 = 0 plane of 1/k^2
            const double gk = pl.periodic3 ? (kap2 > 0.0 ? 1.0 / kap2 : 0.0)
                                           : G_R(std::sqrt(kap2), pl.R);
            double v = z0.pref * std::exp(-(1.0 - g.eta) * kap2 / (4.0 * pl.prm.xi * pl.prm.xi)) * gk;
            if (kx == 0 && ky == 0) v = 0.0;   // (kappa, k3) = (0, 0)
            s0[(size_t)kx * b0 + ky] = v;
        }
    }
}

namespace {

// Sequential carving of device memory: each buffer starts on a 256-byte
// boundary after the previous one.  Pure address arithmetic (no host or
// device allocation), so the same layout can be placed in any buffer.
struct Carver {
    uintptr_t base, off = 0;
    explicit Carver(uintptr_t b) : base(b) {}
    template <typename P> void take(P** ptr, size_t bytes) {
        *ptr = (P*)(base + off);
        off += (bytes + 255) & ~size_t(255);
    }
    size_t used() const { return off; }
};

}  // namespace

// Lays out the per-call scratch of an evaluation of N particles at base
// (the plan's own workspace, or the static scratch array) and returns its
// size in bytes.  Sizes depend on the plan's geometry and on N only.
size_t se1p::layout_scratch(const se1p_plan& pl, long long n, PlanScratch& w,
                            uintptr_t base, bool ik) {
    const se1p_params& p = pl.prm;
    const size_t cs = 2 * pl.es;
    const long long N = std::max<long long>(n, 1);
    Carver c(base);
    BinBufs& bb = w.bins;
    bin_sizes(bb, pl.bg.ncell_lex, pl.bg.ncell_blk);
    c.take(&bb.key_lex, N * 4);
    c.take(&bb.key_blk, N * 4);
    c.take(&bb.slot, N * 4);
    c.take(&bb.tmp, N * 4);
    c.take(&bb.cnt_lex, (bb.ncl + 1) * 4);
    c.take(&bb.cnt_blk, (bb.ncb + 1) * 4);
    c.take(&bb.tsum, ((size_t)bb.ntl + bb.ntb) * 4);
    for (int k = 0; k < 4; ++k) { c.take(&w.lex_i[k], N * 4); c.take(&w.blk_i[k], N * 4); }
    c.take(&w.lex_i[4], (pl.bg.ncell_lex + 1) * 4);
    c.take(&w.blk_i[4], (pl.bg.ncell_blk + 1) * 4);
    for (int k = 0; k < 7; ++k) { c.take(&w.lex_f[k], N * pl.es); c.take(&w.blk_f[k], N * pl.es); }
    const int PW = p.P;                  // x / y weight row (no padding)
    c.take(&w.wz, (size_t)N * p.P * pl.es);
    c.take(&w.wxp, (size_t)N * PW * pl.es);
    c.take(&w.wyq, (size_t)N * PW * pl.es);
    c.take(&w.Hpart, (size_t)pl.KP * pl.pstride * pl.es);
    c.take(&w.Fz, (size_t)pl.nslab * pl.gf.ncol * cs);
    if (pl.periodic3) {
        c.take(&w.Hper, (size_t)p.M3 * pl.gf.ncol * pl.es);
        c.take(&w.Htp, (size_t)p.M3 * pl.gf.ncol * pl.es);
    } else {
        w.Hper = w.Htp = nullptr;
    }
    c.take(&w.G, (size_t)pl.slab_elems * cs);
    c.take(&w.Ht, (size_t)(pl.pstride + 64) * pl.es);   // staging reads past the last row
    if (!pl.periodic3 && ik) {
        c.take(&w.Gk, 3 * (size_t)pl.slab_elems * cs);
        c.take(&w.Htk, 3 * (size_t)(pl.pstride + 64) * pl.es);
    } else {
        w.Gk = w.Htk = nullptr;
    }
    c.take(&w.phiF, N * pl.es);
    c.take(&w.EF, 3 * N * pl.es);
    // Real-space work units: 16-target chunks, each split into rs_parts
    // parts so that the launch has several units per resident wave slot
    // (1024 SIMDs x 4 waves) and the last round is short.
    const long long nchunks = (N + 15) / 16;
    w.rs_parts = (int)std::min<long long>(8, std::max<long long>(1, (32768 + nchunks - 1) / nchunks));
    c.take(&w.phiR, (size_t)w.rs_parts * N * pl.es);
    c.take(&w.ER, 3 * (size_t)w.rs_parts * N * pl.es);
    w.nblk_comb = (int)((N + 255) / 256);
    c.take(&w.partials, (size_t)w.nblk_comb * 8);
    c.take(&w.flag, 256);
    c.take(&w.qsum, 256);
    return c.used();
}

namespace {

int build_plan(se1p_plan& pl, const se1p_params& p, long long n_max) {
    int rc0 = plan_geometry(pl, p, n_max);
    if (rc0) return rc0;
    const Geo& g = pl.g;
    const size_t cs = 2 * pl.es;

    // ---- workspace: tables, then the plan's own scratch for n_max ----
    pl.pstride = (long long)p.M3 * g.ncol;
    Carver tables(0);
    tables.take(&pl.S0, (size_t)pl.n0[0] * pl.n0[1] * pl.es);
    tables.take(&pl.tw, (size_t)pl.tw_elems * cs);
    tables.take((void**)&pl.d_slabs, pl.slabs.size() * sizeof(SlabDesc));
    const size_t tb = tables.used();
    const size_t total = tb + layout_scratch(pl, n_max, pl.w, 0);
    pl.ws_bytes = total;
    if (hipMalloc(&pl.base, total) != hipSuccess) {
        pl.base = nullptr;
        (void)hipGetLastError();
        return SE1P_ERR_NOMEM;
    }
    const uintptr_t b0 = (uintptr_t)pl.base;
    pl.S0 = (void*)(b0 + (uintptr_t)pl.S0);
    pl.tw = (void*)(b0 + (uintptr_t)pl.tw);
    pl.d_slabs = (SlabDesc*)(b0 + (uintptr_t)pl.d_slabs);
    layout_scratch(pl, n_max, pl.w, b0 + tb);

    // ---- tables: twiddles, slab descriptors, FP64 scaling of slab 0 ----
    std::vector<double> twd, s0;
    plan_tables(pl, twd, s0);
    hipError_t e = hipSuccess;
    if (pl.prec == SE1P_FP64) {
        e = hipMemcpy(pl.tw, twd.data(), twd.size() * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl.S0, s0.data(), s0.size() * 8, hipMemcpyHostToDevice);
    } else {
        std::vector<float> twf(twd.begin(), twd.end()), s0f(s0.begin(), s0.end());
        e = hipMemcpy(pl.tw, twf.data(), twf.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl.S0, s0f.data(), s0f.size() * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = hipMemcpy(pl.d_slabs, pl.slabs.data(), pl.slabs.size() * sizeof(SlabDesc),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return SE1P_ERR_HIP;
    return SE1P_OK;
}

template <typename T>
int run_bin(se1p_plan& pl, long long N, const void* x, const void* q) {
    DevParticles<T> lex = particles<T>(pl, true), blk = particles<T>(pl, false);
    return launch_bin<T>((const T*)x, (const T*)q, N, pl.g, pl.bg, pl.w.bins, lex, blk,
                         pl.stream);
}

template <typename T>
int run_spread(se1p_plan& pl, long long N) {
    DevParticles<T> lex = particles<T>(pl, true);
    return launch_spread<T>(lex, N, pl.g, pl.CZ, pl.KP, (T*)pl.w.wz, (T*)pl.w.wxp,
                            (T*)pl.w.wyq, (T*)pl.w.Hpart, pl.pstride, pl.stream);
}

template <typename T>
int run_kspace(se1p_plan& pl, const T* Hin, int KP, T in_scale, T out_scale,
               T* Ht) {
    return launch_kspace<T>(Hin, KP, pl.periodic3 ? (long long)pl.g.M3 * pl.gf.ncol : pl.pstride,
                            in_scale, pl.gf, pl.nslab,
                            pl.d_slabs, pl.slabs.data(), pl.dz,
                            (const cplx<T>*)pl.tw, (const T*)pl.S0,
                            (cplx<T>*)pl.w.Fz, (cplx<T>*)pl.w.G, out_scale, Ht,
                            pl.stream);
}

template <typename T>
int run_eval(se1p_plan& pl, long long N, const void* x, const void* q,
             void* phi, void* efield, double* energy, unsigned flags) {
    int rc;
    unsigned char mask = 0;
    tmark(pl, 0);
    if ((rc = run_bin<T>(pl, N, x, q))) return rc;
    mask |= 1;
    tmark(pl, 1);
    unsigned comp = flags & SE1P_ALL;
    if (comp & SE1P_KSPACE) {
        if ((rc = run_spread<T>(pl, N))) return rc;
        tmark(pl, 2);
        if (pl.periodic3) {
            // fold the gridded values onto the periodic grid, transform,
            // and spread the result back over the gather's extended grid
            if ((rc = launch_fold<T>((const T*)pl.w.Hpart, pl.KP, pl.pstride, pl.g, pl.gf,
                                     (T*)pl.w.Hper, pl.stream))) return rc;
            if ((rc = run_kspace<T>(pl, (const T*)pl.w.Hper, 1, (T)1, (T)1, (T*)pl.w.Htp))) return rc;
            if ((rc = launch_unfold<T>((const T*)pl.w.Htp, pl.g, pl.gf, (T*)pl.w.Ht, pl.stream)))
                return rc;
        } else if (flags & SE1P_FIELD_IK) {
            if ((rc = launch_kspace_ik<T>((const T*)pl.w.Hpart, pl.KP, pl.pstride, pl.g,
                                          pl.nslab, pl.d_slabs, pl.slabs.data(), pl.dz,
                                          (const cplx<T>*)pl.tw, (const T*)pl.S0,
                                          (cplx<T>*)pl.w.Fz, (cplx<T>*)pl.w.G,
                                          (cplx<T>*)pl.w.Gk, pl.slab_elems, (T*)pl.w.Ht,
                                          (T*)pl.w.Htk, pl.pstride + 64, pl.stream)))
                return rc;
        } else {
            if ((rc = run_kspace<T>(pl, (const T*)pl.w.Hpart, pl.KP, (T)1, (T)1, (T*)pl.w.Ht))) return rc;
        }
        tmark(pl, 3);
        DevParticles<T> blk = particles<T>(pl, false);
        if (flags & SE1P_FIELD_IK) {
            // the potential and each field component from its own grid
            if ((rc = launch_gather_phi<T>((const T*)pl.w.Ht, blk, pl.g, pl.bg, (T)1,
                                           (T*)pl.w.phiF, 1, pl.stream)))
                return rc;
            for (int d = 0; d < 3; ++d)
                if ((rc = launch_gather_phi<T>((const T*)pl.w.Htk + d * (pl.pstride + 64), blk,
                                               pl.g, pl.bg, (T)1, (T*)pl.w.EF + d, 3,
                                               pl.stream)))
                    return rc;
        } else if ((rc = launch_gather<T>((const T*)pl.w.Ht, blk, N, pl.g, pl.bg, (T)1,
                                          (T*)pl.w.phiF, (T*)pl.w.EF, pl.stream))) {
            return rc;
        }
        mask |= 2 | 4 | 8;
    } else {
        tmark(pl, 2);
        tmark(pl, 3);
    }
    tmark(pl, 4);
    if ((comp & SE1P_REAL) && pl.prm.rc > 0.0) {
        DevParticles<T> lex = particles<T>(pl, true);
        DevParticles<T> blk = particles<T>(pl, false);
        if ((rc = launch_realspace<T>(lex, blk, N, pl.g, pl.bg, pl.prm.xi, pl.prm.rc,
                                      pl.w.rs_parts, pl.periodic3, (T*)pl.w.phiR, (T*)pl.w.ER,
                                      pl.stream)))
            return rc;
        mask |= 16;
    } else {
        comp &= ~SE1P_REAL;
    }
    tmark(pl, 5);
    const double self_c = 2.0 * pl.prm.xi / std::sqrt(kPi);
    const int nb = (int)((N + 255) / 256);
    rc = launch_combine<T>(N, (const T*)q, (const T*)pl.w.phiF, (const T*)pl.w.EF,
                           (const T*)pl.w.phiR, (const T*)pl.w.ER, pl.w.rs_parts, self_c,
                           comp | (flags & SE1P_FORCE),
                           (T*)phi, (T*)efield, pl.w.partials, nb, energy,
                           pl.stream);
    if (rc) return rc;
    mask |= 32;
    tmark(pl, 6);
    if (pl.timing && pl.tcalls < kTimingMaxCalls) {
        pl.tmask[pl.tcalls] = mask;
        ++pl.tcalls;
    }
    return SE1P_OK;
}

// Relative neutrality bar |sum q| <= tol sum |q| of SE1P_CHECK_INPUT.  FP64
// charges: 1e-10.  FP32 charges: 32 FP32 epsilons (3.8e-6), since charges
// that are neutral in exact arithmetic leave up to eps/2 sum |q| from the
// rounding to FP32 alone, plus about eps log2(N) sum |q| when the shift to
// zero sum was itself computed in FP32 with a tree reduction.
double neutral_tol(int prec) {
    return prec == SE1P_FP32 ? 32.0 * 1.1920928955078125e-7 : 1e-10;
}

template <typename T>
int run_check(se1p_plan& pl, long long N, const void* x, const void* q,
              bool neutral) {
    // cleared by a kernel: the flag and the two sums are 1 + 4 ints
    if (launch_fill_int(pl.w.flag, 1, 0, pl.stream)) return SE1P_ERR_HIP;
    if (launch_fill_int((int*)pl.w.qsum, 4, 0, pl.stream)) return SE1P_ERR_HIP;
    int rc = launch_check<T>((const T*)x, (const T*)q, N, pl.prm.box[0],
                             pl.prm.box[1], pl.w.flag, pl.w.qsum, pl.stream);
    if (rc) return rc;
    int hflag = 0;
    double hq[2] = {0, 0};
    if (hipMemcpyAsync(&hflag, pl.w.flag, 4, hipMemcpyDeviceToHost, pl.stream) != hipSuccess)
        return SE1P_ERR_HIP;
    if (hipMemcpyAsync(hq, pl.w.qsum, 16, hipMemcpyDeviceToHost, pl.stream) != hipSuccess)
        return SE1P_ERR_HIP;
    if (hipStreamSynchronize(pl.stream) != hipSuccess) return SE1P_ERR_HIP;
    if (hflag) return SE1P_ERR_OUT_OF_BOX;
    if (neutral && std::fabs(hq[0]) > neutral_tol(pl.prec) * hq[1]) return SE1P_ERR_NONNEUTRAL;
    return SE1P_OK;
}

}  // namespace

namespace se1p {

int set_device(const se1p_plan* pl) {
    return hipSetDevice(pl->device) == hipSuccess ? SE1P_OK : SE1P_ERR_HIP;
}

// Host-side argument checks of se1p_eval and se1p_eval_noalloc.
int eval_args(const se1p_plan* pl, long long N, const void* x, const void* q,
              unsigned flags) {
    if (!pl || !x || !q) return SE1P_ERR_ARG;
    if (flags & ~(SE1P_ALL | SE1P_CHECK_INPUT | SE1P_NO_NEUTRAL | SE1P_FIELD_IK | SE1P_FORCE))
        return SE1P_ERR_ARG;
    if ((flags & SE1P_FIELD_IK) && pl->periodic3) return SE1P_ERR_UNSUPPORTED;
    if ((flags & SE1P_ALL) == 0) return SE1P_ERR_ARG;
    if (N < 1 || N > (1LL << 30)) return SE1P_ERR_ARG;
    if ((flags & SE1P_REAL) && !(pl->prm.rc > 0.0)) return SE1P_ERR_PARAM;
    return SE1P_OK;
}

int eval_body(se1p_plan* pl, long long N, const void* x, const void* q,
              void* phi, void* efield, double* energy, unsigned flags) {
    if (flags & SE1P_CHECK_INPUT) {
        const bool neutral = !(flags & SE1P_NO_NEUTRAL);
        int rc = (pl->prec == SE1P_FP64) ? run_check<double>(*pl, N, x, q, neutral)
                                         : run_check<float>(*pl, N, x, q, neutral);
        if (rc) return rc;
    }
    if (pl->prec == SE1P_FP64)
        return run_eval<double>(*pl, N, x, q, phi, efield, energy, flags);
    return run_eval<float>(*pl, N, x, q, phi, efield, energy, flags);
}

}  // namespace se1p

extern "C" {

const char* se1p_error_string(int code) {
    switch (code) {
        case SE1P_OK: return "success";
        case SE1P_ERR_ARG: return "invalid argument";
        case SE1P_ERR_PARAM: return "inconsistent method parameters";
        case SE1P_ERR_NONNEUTRAL: return "charges are not neutral";
        case SE1P_ERR_OUT_OF_BOX: return "position outside the box in a free direction";
        case SE1P_ERR_HIP: return "HIP runtime error";
        case SE1P_ERR_NOMEM: return "device allocation failed";
        case SE1P_ERR_TOO_MANY: return "more particles than the plan allows";
        case SE1P_ERR_UNSUPPORTED: return "unsupported parameter combination";
        case SE1P_ERR_SCRATCH:
            return "the call needs more scratch than se1p_eval_noalloc's static buffer holds";
        default: return "unknown error";
    }
}

const char* se1p_version(void) { return "se1p-mi355x 0.1.0 (gfx950)"; }

int se1p_suggest_params(double tol, const double box[3], long long N, double Q,
                        double xi_in, int M3_in, int P_in, int n_l_in,
                        int precision, se1p_params* out) {
    if (!box || !out || !(tol > 0.0) || !(tol < 1.0) || N < 1 || !(Q > 0.0))
        return SE1P_ERR_ARG;
    if (precision != SE1P_FP64 && precision != SE1P_FP32) return SE1P_ERR_ARG;
    for (int d = 0; d < 3; ++d)
        if (!(box[d] > 0.0)) return SE1P_ERR_ARG;
    const double L = box[2];
    const double V = box[0] * box[1] * box[2];
    se1p_params p{};
    p.box[0] = box[0]; p.box[1] = box[1]; p.box[2] = box[2];
    p.precision = precision;
    // Fourier truncation estimate (eq. trunc_error_estimate_fourier)
    auto errF = [&](double xi, double kinf) {
        return xi / (kPi * kPi) * std::pow(kinf, -1.5) * std::sqrt(Q) *
               std::exp(-std::pow(kPi * kinf / (xi * L), 2));
    };
    if (M3_in > 0) {
        p.M3 = M3_in + (M3_in & 1);
        const double kinf = p.M3 / 2.0;
        if (xi_in > 0.0) {
            p.xi = xi_in;
        } else {
            double lo = 1e-3 / L, hi = 1e3 / L;
            for (int it = 0; it < 200; ++it) {
                const double mid = std::sqrt(lo * hi);
                if (errF(mid, kinf) < tol) lo = mid; else hi = mid;
            }
            p.xi = lo;
        }
    } else {
        if (!(xi_in > 0.0)) return SE1P_ERR_ARG;
        p.xi = xi_in;
        // eq. kinf
        const double D = 4.0 / (3.0 * L * L) * std::pow(Q / kPi, 2.0 / 3.0);
        const double kinf = std::sqrt(3.0) * L * p.xi / (2.0 * kPi) *
                            std::sqrt(lambert_w(D / std::pow(p.xi * tol * tol, 2.0 / 3.0)));
        // 2 k_inf, rounded up to an even size the transforms take (prime
        // factors 2, 3 and 5 only)
        int m = std::max(8, 2 * (int)std::ceil(kinf));
        while (nice_size(m) != m || (m & 1)) ++m;
        p.M3 = m;
    }
    // eq. rc with V for L^3
    const double C = Q / (2.0 * V * p.xi * tol * tol);
    p.rc = 1.0 / (2.0 * p.xi) * std::sqrt(3.0 * lambert_w(4.0 / 3.0 * std::pow(C, 2.0 / 3.0)));
    // eq. approximation_error_oneterm with A = sqrt(Q xi L) / L
    if (P_in > 0) {
        p.P = P_in;
    } else {
        const double A = std::sqrt(Q * p.xi * L) / L;
        int P = (int)std::ceil(2.0 * std::log(std::max(A / tol, 1.0)) / (kShapeC * kShapeC * kPi));
        P += P & 1;
        p.P = std::min(std::max(P, 4), kMaxP);
    }
    if (p.P > p.M3) p.P = p.M3 - (p.M3 & 1);
    // eq. choose_sl generalised to any box: the first k3 mode's kernel
    // decays like exp(-2 pi d / L3) with the distance d to the nearest
    // periodic image of the support in the padded period, d = (s_l - 1) Lt,
    // so exp(-2 pi (s_l - 1) Lt / L3) < tol
    const double h = L / p.M3;
    const double Lt = std::min(std::ceil(box[0] / h - 1e-9), std::ceil(box[1] / h - 1e-9)) * h + p.P * h;
    p.s_l = 1.0 + std::log(1.0 / tol) * L / (2.0 * kPi * Lt);
    // eq. choose_nl: M ~ 10 n_l
    p.n_l = (n_l_in >= 0) ? n_l_in : std::max(1, (int)std::lround(p.M3 / 10.0));
    p.s0 = 1.0 + std::sqrt(2.0);
    *out = p;
    return check_params(p);
}

namespace {
int plan_create(const se1p_params* params, long long n_max, void* stream,
                bool periodic3, se1p_plan** out) {
    if (!params || !out || n_max < 1 || n_max > (1LL << 30)) return SE1P_ERR_ARG;
    *out = nullptr;
    int rc = check_params(*params);
    if (rc) return rc;
    if (periodic3) {
        // the grid must tile each period exactly: L1 and L2 multiples of h
        const double h = params->box[2] / params->M3;
        for (int d = 0; d < 2; ++d) {
            const double m = params->box[d] / h;
            if (std::fabs(m - std::round(m)) > 1e-9 * m || std::round(m) < 2.0)
                return SE1P_ERR_PARAM;
        }
    }
    se1p_plan* pl = new (std::nothrow) se1p_plan();
    if (!pl) return SE1P_ERR_NOMEM;
    if (hipGetDevice(&pl->device) != hipSuccess) { delete pl; return SE1P_ERR_HIP; }
    pl->stream = (hipStream_t)stream;
    pl->periodic3 = periodic3;
    rc = build_plan(*pl, *params, n_max);
    if (rc) {
        if (pl->base) (void)hipFree(pl->base);
        delete pl;
        return rc;
    }
    *out = pl;
    return SE1P_OK;
}
}  // namespace

int se1p_plan_create(const se1p_params* params, long long n_max, void* stream,
                     se1p_plan** out) {
    return plan_create(params, n_max, stream, false, out);
}

int se3p_plan_create(const se1p_params* params, long long n_max, void* stream,
                     se1p_plan** out) {
    return plan_create(params, n_max, stream, true, out);
}

int se1p_timing_enable(se1p_plan* pl, int enable) {
    if (!pl) return SE1P_ERR_ARG;
    if (set_device(pl)) return SE1P_ERR_HIP;
    if (enable && pl->tev.empty()) {
        pl->tev.resize((size_t)kTimingMaxCalls * (SE1P_NSTAGE + 1));
        for (auto& e : pl->tev) {
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                e = nullptr;
                return SE1P_ERR_HIP;
            }
        }
        pl->tmask.assign(kTimingMaxCalls, 0);
    }
    pl->timing = enable ? 1 : 0;
    pl->tcalls = 0;
    return SE1P_OK;
}

int se1p_timing_select(se1p_plan* pl, unsigned stages) {
    if (!pl) return SE1P_ERR_ARG;
    if (stages == 0u || (stages >> SE1P_NSTAGE) != 0u) return SE1P_ERR_ARG;
    pl->tstages = stages;
    pl->tcalls = 0;
    return SE1P_OK;
}

int se1p_timing_read(se1p_plan* pl, double* ms_sum, int* ncalls) {
    if (!pl || !ms_sum) return SE1P_ERR_ARG;
    for (int s = 0; s < SE1P_NSTAGE; ++s) ms_sum[s] = 0.0;
    if (ncalls) *ncalls = pl->tcalls;
    if (pl->tcalls == 0) return SE1P_OK;
    if (set_device(pl)) return SE1P_ERR_HIP;
    if (hipStreamSynchronize(pl->stream) != hipSuccess) return SE1P_ERR_HIP;
    // stage s runs between boundaries: 0:[0,1] 1:[1,2] 2:[2,3] 3:[3,4]
    // 4:[4,5] 5:[5,6]
    for (int c = 0; c < pl->tcalls; ++c) {
        const hipEvent_t* e = &pl->tev[(size_t)c * (SE1P_NSTAGE + 1)];
        for (int s = 0; s < SE1P_NSTAGE; ++s) {
            if (!((pl->tstages >> s) & 1u)) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e[s], e[s + 1]) != hipSuccess) return SE1P_ERR_HIP;
            ms_sum[s] += ms;
        }
    }
    return SE1P_OK;
}

int se1p_plan_destroy(se1p_plan* plan) {
    if (!plan) return SE1P_ERR_ARG;
    int rc = SE1P_OK;
    if (set_device(plan)) rc = SE1P_ERR_HIP;
    if (hipStreamSynchronize(plan->stream) != hipSuccess) rc = SE1P_ERR_HIP;
    for (auto& e : plan->tev)
        if (e) (void)hipEventDestroy(e);
    if (plan->base && hipFree(plan->base) != hipSuccess) rc = SE1P_ERR_HIP;
    delete plan;
    return rc;
}

int se1p_plan_get_info(const se1p_plan* pl, se1p_plan_info* info) {
    if (!pl || !info) return SE1P_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->h = pl->g.h;
    info->eta = pl->g.eta;
    info->R = pl->R;
    info->M[0] = pl->M1;
    info->M[1] = pl->M2;
    info->Mt[0] = pl->g.Mt1;
    info->Mt[1] = pl->g.Mt2;
    info->M3 = pl->g.M3;
    info->P = pl->g.P;
    info->n0[0] = pl->n0[0];
    info->n0[1] = pl->n0[1];
    info->nl[0] = pl->nl[0];
    info->nl[1] = pl->nl[1];
    info->n_l = pl->prm.n_l;
    info->nslab = pl->nslab;
    info->precision = pl->prec;
    info->n_max = pl->n_max;
    info->workspace_bytes = pl->ws_bytes;
    info->gather_block[0] = pl->bg.BX;
    info->gather_block[1] = pl->bg.BY;
    info->gather_block[2] = pl->bg.BZ;
    info->gather_chunks = pl->bg.CH;
    info->spread_cz = pl->CZ;
    info->spread_kp = pl->KP;
    info->bin_cells[0] = pl->bg.ncell_lex;
    info->bin_cells[1] = pl->bg.ncell_blk;
    info->gather_pair = pl->bg.pair;
    return SE1P_OK;
}

int se1p_set_stream(se1p_plan* plan, void* stream) {
    if (!plan) return SE1P_ERR_ARG;
    plan->stream = (hipStream_t)stream;
    return SE1P_OK;
}

int se1p_eval(se1p_plan* pl, long long N, const void* x, const void* q,
              void* phi, void* efield, double* energy, unsigned flags) {
    int rc = eval_args(pl, N, x, q, flags);
    if (rc) return rc;
    if (N > pl->n_max) return SE1P_ERR_TOO_MANY;
    if (set_device(pl)) return SE1P_ERR_HIP;
    return eval_body(pl, N, x, q, phi, efield, energy, flags);
}

int se1p_spread(se1p_plan* pl, long long N, const void* x, const void* q,
                void* grid) {
    if (!pl || !x || !q || !grid) return SE1P_ERR_ARG;
    if (pl->periodic3) return SE1P_ERR_UNSUPPORTED;
    if (N < 1) return SE1P_ERR_ARG;
    if (N > pl->n_max) return SE1P_ERR_TOO_MANY;
    if (set_device(pl)) return SE1P_ERR_HIP;
    int rc;
    const long long n = pl->pstride;
    if (pl->prec == SE1P_FP64) {
        if ((rc = run_bin<double>(*pl, N, x, q))) return rc;
        if ((rc = run_spread<double>(*pl, N))) return rc;
        return launch_reduce_partials<double>((const double*)pl->w.Hpart, pl->KP, n, n,
                                              pl->cg, (double*)grid, pl->stream);
    }
    if ((rc = run_bin<float>(*pl, N, x, q))) return rc;
    if ((rc = run_spread<float>(*pl, N))) return rc;
    return launch_reduce_partials<float>((const float*)pl->w.Hpart, pl->KP, n, n,
                                         (float)pl->cg, (float*)grid, pl->stream);
}

int se1p_bin(se1p_plan* pl, long long N, const void* x, const void* q,
             int* lex_perm, int* lex_start, int* blk_perm, int* blk_start) {
    if (!pl || !x || !q) return SE1P_ERR_ARG;
    if (N < 1) return SE1P_ERR_ARG;
    if (N > pl->n_max) return SE1P_ERR_TOO_MANY;
    if (set_device(pl)) return SE1P_ERR_HIP;
    const int rc = pl->prec == SE1P_FP64 ? run_bin<double>(*pl, N, x, q)
                                         : run_bin<float>(*pl, N, x, q);
    if (rc) return rc;
    const size_t np = (size_t)N * 4;
    const struct { int* dst; const int* src; size_t bytes; } cp[4] = {
        {lex_perm, pl->w.lex_i[3], np},
        {lex_start, pl->w.lex_i[4], (size_t)(pl->bg.ncell_lex + 1) * 4},
        {blk_perm, pl->w.blk_i[3], np},
        {blk_start, pl->w.blk_i[4], (size_t)(pl->bg.ncell_blk + 1) * 4}};
    for (const auto& c : cp)
        if (c.dst && hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice,
                                    pl->stream) != hipSuccess)
            return SE1P_ERR_HIP;
    return SE1P_OK;
}

int se1p_kspace_solve(se1p_plan* pl, const void* grid_in, void* grid_out) {
    if (!pl || !grid_in || !grid_out) return SE1P_ERR_ARG;
    if (pl->periodic3) return SE1P_ERR_UNSUPPORTED;
    if (set_device(pl)) return SE1P_ERR_HIP;
    const double h3 = pl->g.h * pl->g.h * pl->g.h;
    const double in_s = 1.0 / pl->cg;
    const double out_s = 1.0 / (4.0 * kPi * h3 * pl->cg);
    if (pl->prec == SE1P_FP64)
        return run_kspace<double>(*pl, (const double*)grid_in, 1, in_s, out_s,
                                  (double*)grid_out);
    return run_kspace<float>(*pl, (const float*)grid_in, 1, (float)in_s,
                             (float)out_s, (float*)grid_out);
}

int se1p_gather(se1p_plan* pl, long long N, const void* x, const void* grid,
                void* phi, void* efield) {
    if (!pl || !x || !grid) return SE1P_ERR_ARG;
    if (pl->periodic3) return SE1P_ERR_UNSUPPORTED;
    if (N < 1) return SE1P_ERR_ARG;
    if (N > pl->n_max) return SE1P_ERR_TOO_MANY;
    if (set_device(pl)) return SE1P_ERR_HIP;
    const double h3 = pl->g.h * pl->g.h * pl->g.h;
    const double sc = 4.0 * kPi * h3 * pl->cg;
    int rc;
    // The gather reads grid rows in halves and may touch one element past
    // the last row; it runs on the plan's padded copy of the caller's grid.
    if (hipMemcpyAsync(pl->w.Ht, grid, (size_t)pl->pstride * pl->es,
                       hipMemcpyDeviceToDevice, pl->stream) != hipSuccess)
        return SE1P_ERR_HIP;
    // binning sorts charges along with positions; the gather does not use
    // them, so the plan's scratch phiF stands in for q.
    if (pl->prec == SE1P_FP64) {
        if ((rc = run_bin<double>(*pl, N, x, pl->w.phiF))) return rc;
        DevParticles<double> blk = particles<double>(*pl, false);
        return launch_gather<double>((const double*)pl->w.Ht, blk, N, pl->g, pl->bg, sc,
                                     (double*)phi, (double*)efield, pl->stream);
    }
    if ((rc = run_bin<float>(*pl, N, x, pl->w.phiF))) return rc;
    DevParticles<float> blk = particles<float>(*pl, false);
    return launch_gather<float>((const float*)pl->w.Ht, blk, N, pl->g, pl->bg, (float)sc,
                                (float*)phi, (float*)efield, pl->stream);
}

}  // extern "C"
