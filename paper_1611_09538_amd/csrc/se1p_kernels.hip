// se1p_kernels.hip -- HIP kernels of the SE1P k-space pipeline for gfx950.
//
// Pipeline (Algorithm 1 of the paper):
//   bin        counting sort of the particles by cell in two orders (cell
//              counts, a reduce-then-scan, placement by rank of the input
//              index inside a cell)
//   spread     step 2, eq. spread_1p: owner-computes gridding, a workgroup
//              of 1 to 8 waves per 8 x 8 (x, y) pencil tile sweeping a chunk
//              of z cells with the z-support in registers; the waves share
//              each z cell's particle list; per-particle z weights arrive as
//              wave-uniform (scalar) loads, x/y weights are per lane
//   kspace     steps 3-5: z FFT (real, two columns per complex transform),
//              per-slab zero-padded row FFTs, fused column FFT -> scaling
//              (eq. scale_1p with G of eq. G_kappa_k) -> inverse column FFT,
//              inverse row FFTs, inverse z FFT; Stockham FFTs in LDS
//   gather     step 6 (eq. se1p_complete_discretized) and its analytic
//              gradient (eq. force_se1p): one lane per particle, chunks of
//              one block or of two y-adjacent blocks, the grid planes a
//              chunk's supports touch staged in LDS
//   realspace  eq. ewald1p_real / eq. force_real over the cell list
//   combine    totals, self term (eq. ewald1p_self), energy 1/2 sum q phi
//
// Grid layout: real grids are [z][x][y] (y fastest); z-spectra [n3][x][y].
// The Gaussian normalisation and all transform normalisations are folded
// into the scaling factors, so spread and gather use exp(-alpha d^2).
#include <hip/hip_runtime.h>

#include "erfcx_poly.h"
#include "se1p.h"
#include "se1p_internal.h"

namespace se1p {

namespace {

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------
__device__ __forceinline__ int imod(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}

template <typename T> __device__ __forceinline__ T dexp(T v);
template <> __device__ __forceinline__ double dexp<double>(double v) { return exp(v); }
template <> __device__ __forceinline__ float dexp<float>(float v) { return __expf(v); }

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    cplx<T> r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // a * conj(b)
    cplx<T> r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
    cplx<T> r; r.x = a.x + b.x; r.y = a.y + b.y; return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
    cplx<T> r; r.x = a.x - b.x; r.y = a.y - b.y; return r;
}
// multiply by i*s (s = +1 or -1)
template <typename T>
__device__ __forceinline__ cplx<T> cmuli(cplx<T> a, T s) {
    cplx<T> r; r.x = -s * a.y; r.y = s * a.x; return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) {
    cplx<T> r; r.x = a.x * s; r.y = a.y * s; return r;
}

// Division by a divisor d >= 1 fixed for a loop: m = floor((2^32 - 1) / d)
// + 1 makes q = umulhi(a, m) exact for a d < 2^32 (the error a (m d - 2^32)
// / (d 2^32) stays below 1/d); d = 1 takes q = a.  The FFT index maps divide
// by pass lengths known only at run time, and the compiler's generic
// division costs about 15 instructions each.
struct UDiv {
    unsigned m;
    int d;
    __device__ __forceinline__ explicit UDiv(int dd)
        : m(dd > 1 ? 0xFFFFFFFFu / (unsigned)dd + 1u : 0u), d(dd) {}
    __device__ __forceinline__ int operator()(int a) const {
        return d > 1 ? (int)__umulhi((unsigned)a, m) : a;
    }
};

// Block-cooperative copy of count elements: load(i) reads element i from
// global memory, store(i, v) puts it into LDS.  Each thread issues kLoadBatch
// loads before it stores any of them, so their latencies overlap (a loop of
// one load and one store per element waits for every load in turn).
constexpr int kLoadBatch = 8;
template <typename V, typename L, typename S>
__device__ __forceinline__ void batched_copy(int count, L load, S store) {
    for (int i0 = threadIdx.x; i0 < count; i0 += kLoadBatch * blockDim.x) {
        V v[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < count) v[u] = load(i);
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < count) store(i, v[u]);
        }
    }
}

// ------------------------------------------------------------------------
// Stockham FFT in LDS, block-cooperative, mixed radix 2/3/4/5.
// 'batch' transforms of length n start at a + b*stride; b is scratch of the
// same shape.  Returns the buffer holding the result.  sgn = -1 forward
// (exp(-2 pi i jk/n)), +1 inverse (unnormalised).
// ------------------------------------------------------------------------
template <typename T>
__device__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, int batch, int stride,
                            const FftDesc& d, const cplx<T>* __restrict__ tw,
                            int sgn) {
    const int n = d.n;
    const T s = (T)sgn;
    int Ns = 1;
    for (int p = 0; p < d.nrad; ++p) {
        const int R = d.rad[p];
        const int nR = n / R;
        const int tstep = n / (Ns * R);
        const int total = batch * nR;
        const UDiv divR(nR), divN(Ns);
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int bi = divR(t);
            const int j = t - bi * nR;
            const cplx<T>* src = a + (long)bi * stride;
            cplx<T>* dst = b + (long)bi * stride;
            const int jq = divN(j);
            const int k = j - jq * Ns;
            const int base = jq * Ns * R + k;
            const int tb = k * tstep;
            if (R == 4) {
                cplx<T> v0 = src[j], v1 = src[j + nR], v2 = src[j + 2 * nR], v3 = src[j + 3 * nR];
                if (k) {
                    cplx<T> w1 = tw[tb], w2 = tw[2 * tb], w3 = tw[3 * tb];
                    if (sgn < 0) { v1 = cmul<T>(v1, w1); v2 = cmul<T>(v2, w2); v3 = cmul<T>(v3, w3); }
                    else { v1 = cmulc<T>(v1, w1); v2 = cmulc<T>(v2, w2); v3 = cmulc<T>(v3, w3); }
                }
                cplx<T> a0 = cadd<T>(v0, v2), a1 = csub<T>(v0, v2);
                cplx<T> b0 = cadd<T>(v1, v3), b1 = cmuli<T>(csub<T>(v1, v3), s);
                dst[base] = cadd<T>(a0, b0);
                dst[base + Ns] = cadd<T>(a1, b1);
                dst[base + 2 * Ns] = csub<T>(a0, b0);
                dst[base + 3 * Ns] = csub<T>(a1, b1);
            } else if (R == 2) {
                cplx<T> v0 = src[j], v1 = src[j + nR];
                if (k) {
                    cplx<T> w1 = tw[tb];
                    v1 = (sgn < 0) ? cmul<T>(v1, w1) : cmulc<T>(v1, w1);
                }
                dst[base] = cadd<T>(v0, v1);
                dst[base + Ns] = csub<T>(v0, v1);
            } else if (R == 3) {
                cplx<T> v0 = src[j], v1 = src[j + nR], v2 = src[j + 2 * nR];
                if (k) {
                    cplx<T> w1 = tw[tb], w2 = tw[2 * tb];
                    if (sgn < 0) { v1 = cmul<T>(v1, w1); v2 = cmul<T>(v2, w2); }
                    else { v1 = cmulc<T>(v1, w1); v2 = cmulc<T>(v2, w2); }
                }
                const T c1 = (T)-0.5;
                const T s1 = (T)0.86602540378443864676372317075294;
                cplx<T> t = cadd<T>(v1, v2), u = csub<T>(v1, v2);
                cplx<T> m;
                m.x = v0.x + c1 * t.x;
                m.y = v0.y + c1 * t.y;
                cplx<T> r = cmuli<T>(cscale<T>(u, s1), s);
                dst[base] = cadd<T>(v0, t);
                dst[base + Ns] = cadd<T>(m, r);
                dst[base + 2 * Ns] = csub<T>(m, r);
            } else {  // R == 5
                cplx<T> v0 = src[j], v1 = src[j + nR], v2 = src[j + 2 * nR],
                        v3 = src[j + 3 * nR], v4 = src[j + 4 * nR];
                if (k) {
                    cplx<T> w1 = tw[tb], w2 = tw[2 * tb], w3 = tw[3 * tb], w4 = tw[4 * tb];
                    if (sgn < 0) {
                        v1 = cmul<T>(v1, w1); v2 = cmul<T>(v2, w2);
                        v3 = cmul<T>(v3, w3); v4 = cmul<T>(v4, w4);
                    } else {
                        v1 = cmulc<T>(v1, w1); v2 = cmulc<T>(v2, w2);
                        v3 = cmulc<T>(v3, w3); v4 = cmulc<T>(v4, w4);
                    }
                }
                const T c1 = (T)0.30901699437494742410229341718282;
                const T c2 = (T)-0.80901699437494742410229341718282;
                const T s1 = (T)0.95105651629515357211643933337938;
                const T s2 = (T)0.58778525229247312916870595463907;
                cplx<T> t1 = cadd<T>(v1, v4), t2 = cadd<T>(v2, v3);
                cplx<T> u1 = csub<T>(v1, v4), u2 = csub<T>(v2, v3);
                cplx<T> m1, m2, r1, r2;
                m1.x = v0.x + c1 * t1.x + c2 * t2.x;
                m1.y = v0.y + c1 * t1.y + c2 * t2.y;
                m2.x = v0.x + c2 * t1.x + c1 * t2.x;
                m2.y = v0.y + c2 * t1.y + c1 * t2.y;
                cplx<T> q1, q2;
                q1.x = s1 * u1.x + s2 * u2.x;
                q1.y = s1 * u1.y + s2 * u2.y;
                q2.x = s2 * u1.x - s1 * u2.x;
                q2.y = s2 * u1.y - s1 * u2.y;
                r1 = cmuli<T>(q1, s);
                r2 = cmuli<T>(q2, s);
                cplx<T> y0;
                y0.x = v0.x + t1.x + t2.x;
                y0.y = v0.y + t1.y + t2.y;
                dst[base] = y0;
                dst[base + Ns] = cadd<T>(m1, r1);
                dst[base + 4 * Ns] = csub<T>(m1, r1);
                dst[base + 2 * Ns] = cadd<T>(m2, r2);
                dst[base + 3 * Ns] = csub<T>(m2, r2);
            }
        }
        __syncthreads();
        cplx<T>* tmp = a; a = b; b = tmp;
        Ns *= R;
    }
    return a;
}

// FP32 Gaussian weight exp(-alpha (u h)^2) of an offset u in units of h,
// with alpha h^2 carried as two FP32 parts (c_hi + c_lo): a single rounded
// constant would bias every weight of a launch the same way (by up to
// alpha (u h)^2 2^-24 relative), which shows in the self-interaction
// part of phi^F and from there in the energy.
__device__ __forceinline__ float gauss_u(float u, float c_hi, float c_lo) {
    const float u2 = u * u;
    return __expf(fmaf(-c_hi, u2, -c_lo * u2));
}
struct GaussC {
    float hi, lo;
};
__host__ __device__ __forceinline__ GaussC gauss_consts(const Geo& g) {
    const double c = g.alpha * g.h * g.h;
    const float hi = (float)c;
    return {hi, (float)(c - (double)hi)};
}

// ------------------------------------------------------------------------
// binning
// ------------------------------------------------------------------------
__global__ void fill_int_kernel(int* __restrict__ p, long long n, int v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__device__ __forceinline__ void cell_of(T x, T y, T z, const Geo& g, T& zw,
                                        int& cx, int& cy, int& cz) {
    const T L3 = (T)g.L3;
    const T h = (T)g.h;
    zw = z - L3 * floor(z / L3);
    if (!(zw < L3)) zw = (T)0;       // also maps NaN to 0
    if (zw < (T)0) zw = (T)0;
    cx = (int)floor(x / h);
    cy = (int)floor(y / h);
    cz = (int)floor(zw / h);
    cx = min(max(cx, 0), g.M1 - 1);
    cy = min(max(cy, 0), g.M2 - 1);
    cz = min(max(cz, 0), g.M3 - 1);
}

// Blocks of cells are numbered along a serpentine path (x reversed on odd
// z planes, y reversed on odd rows), so consecutive blocks are always face
// neighbours; inside a block the cells run z-major, with z reversed in odd
// blocks, so that the last cells of a block and the first of the next one
// share a z layer.  A run of consecutive particles of the block order thus
// stays spatially compact across block boundaries, also for blocks that
// are whole z columns.
__device__ __forceinline__ int block_index(int bz, int bx, int by, const BinGeo& bg) {
    const int bxs = (bz & 1) ? bg.nbx - 1 - bx : bx;
    const int row = bz * bg.nbx + bxs;
    const int bys = (row & 1) ? bg.nby - 1 - by : by;
    return row * bg.nby + bys;
}
__device__ __forceinline__ void block_coords(int b, const BinGeo& bg, int& bz,
                                             int& bx, int& by) {
    const int bys = b % bg.nby;
    const int row = b / bg.nby;
    const int bxs = row % bg.nbx;
    bz = row / bg.nbx;
    by = (row & 1) ? bg.nby - 1 - bys : bys;
    bx = (bz & 1) ? bg.nbx - 1 - bxs : bxs;
}

// XCD-aware work order.  The dispatcher deals workgroups round-robin to the
// 8 XCDs, each with its own L2; this bijection of [0, n) gives XCD r the
// contiguous range of the logical order, so work units that are neighbours
// in that order (and re-read the same data) share one L2.
__device__ __forceinline__ unsigned xcd_order(unsigned L, unsigned n) {
    const unsigned C = (n + 7) / 8, d = 8 * C - n, r = L % 8, k = L / 8;
    return r * C - (r > 8 - d ? r - (8 - d) : 0) + k;
}

// Lex and block cell keys of one particle.
template <typename T>
__device__ __forceinline__ void cell_keys(const T* __restrict__ xin, long long i,
                                          const Geo& g, const BinGeo& bg,
                                          int& kl, int& kb) {
    T zw;
    int cx, cy, cz;
    cell_of<T>(xin[3 * i], xin[3 * i + 1], xin[3 * i + 2], g, zw, cx, cy, cz);
    kl = (cz * g.M1 + cx) * g.M2 + cy;
    const int bz = cz / bg.BZ, iz = cz - bz * bg.BZ;
    const int bx = cx / bg.BX, ix = cx - bx * bg.BX;
    const int by = cy / bg.BY, iy = cy - by * bg.BY;
    const int b = block_index(bz, bx, by, bg);
    const int izs = (b & 1) ? bg.BZ - 1 - iz : iz;
    kb = b * bg.cpb + (izs * bg.BX + ix) * bg.BY + iy;
}

// Records the cell keys of particle i and takes its arrival slot in its lex
// cell; with blk_count it is also counted in its block-order cell (the
// batch, whose block-order counts are not derived from the lex counts).
__device__ __forceinline__ void count_keys(long long i, int kl, int kb,
                                           const BinBufs& b, bool blk_count) {
    b.key_lex[i] = kl;
    b.key_blk[i] = kb;
    b.slot[i] = atomicAdd(&b.cnt_lex[kl], 1);
    if (blk_count) atomicAdd(&b.cnt_blk[kb], 1);
}

template <typename T>
__global__ void bin_keys_kernel(const T* __restrict__ xin, long long N, Geo g,
                                BinGeo bg, BinBufs b) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int kl, kb;
    cell_keys<T>(xin, i, g, bg, kl, kb);
    count_keys(i, kl, kb, b, false);
}

// Zeroes the lex cell counts and, with both, the block-order ones.
__global__ void bin_clear_kernel(BinBufs b, bool both) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n1 = b.ncl + 1, n2 = both ? b.ncb + 1 : 0;
    if (k < n1) b.cnt_lex[k] = 0;
    else if (k < n1 + n2) b.cnt_blk[k - n1] = 0;
}

__device__ __forceinline__ int wave_sum_int(int v) {
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}
__device__ __forceinline__ int wave_incl_scan_int(int v) {
    const int lane = threadIdx.x & 63;
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan of n counts into starts (start[k] = sum of cnt[0..k)).
// With lexcnt set, the counts are those of the block-order cells, taken
// from the lex counts of the same cells by the first pass (which writes
// them to cnt for the second).
struct ScanJob {
    int* cnt;
    int* start;
    long long n;
    const int* tsum;   // particles per tile of kScanTile counts
    int ntiles;
    const int* lexcnt;
    BinGeo bg;
    int M1, M2;
};

// Lex counts of the block-order cells [k, k + kScanItems) (cells past the
// grid, in blocks that overhang it, and the end entry count zero).  The
// cell indices are decoded once and then stepped: y fastest, then x, then
// the block's z layer (counted backwards in odd blocks), then the block.
__device__ __forceinline__ void blk_counts_from_lex(const ScanJob& j, long long k,
                                                    int (&v)[kScanItems]) {
    const BinGeo& bg = j.bg;
    const long long ncb = j.n - 1;
    const int bxy = bg.BX * bg.BY;
    int b = (int)(k / bg.cpb);
    const int rem = (int)(k - (long long)b * bg.cpb);
    int izs = rem / bxy;
    int ix = (rem - izs * bxy) / bg.BY;
    int iy = rem - izs * bxy - ix * bg.BY;
    int bz = 0, bx = 0, by = 0;
    if (k < ncb) block_coords(b, bg, bz, bx, by);
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        int c = 0;
        if (k + t < ncb) {
            const int iz = (b & 1) ? bg.BZ - 1 - izs : izs;
            const int cz = bz * bg.BZ + iz, cx = bx * bg.BX + ix, cy = by * bg.BY + iy;
            if (cx < j.M1 && cy < j.M2)
                c = j.lexcnt[((long long)cz * j.M1 + cx) * j.M2 + cy];
            if (++iy == bg.BY) {
                iy = 0;
                if (++ix == bg.BX) {
                    ix = 0;
                    if (++izs == bg.BZ) {
                        izs = 0;
                        ++b;
                        if (k + t + 1 < ncb) block_coords(b, bg, bz, bx, by);
                    }
                }
            }
        }
        v[t] = c;
    }
}

// Loads the kScanItems counts of thread tid of tile t (zeros past n).
__device__ __forceinline__ bool scan_load(const ScanJob& j, int t, int tid,
                                          int (&v)[kScanItems]) {
    const long long base = (long long)t * kScanTile + (long long)tid * kScanItems;
    const bool full = base + kScanItems <= j.n;
    if (full) {
        const int4* p = reinterpret_cast<const int4*>(j.cnt + base);
#pragma unroll
        for (int k = 0; k < kScanItems / 4; ++k) {
            const int4 c = p[k];
            v[4 * k] = c.x; v[4 * k + 1] = c.y; v[4 * k + 2] = c.z; v[4 * k + 3] = c.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = base + k < j.n ? j.cnt[base + k] : 0;
    }
    return full;
}

// Particles per scan tile of both orders (one workgroup per tile), the
// first pass of the reduce-then-scan.
__global__ __launch_bounds__(256) void bin_tile_sum_kernel(ScanJob a, ScanJob b,
                                                           int* __restrict__ tsum) {
    __shared__ int red[4];
    int t = blockIdx.x;
    const bool second = t >= a.ntiles;
    const ScanJob j = second ? b : a;
    if (second) t -= a.ntiles;
    int v[kScanItems];
    if (j.lexcnt) {
        const long long base = (long long)t * kScanTile + (long long)threadIdx.x * kScanItems;
        if (base < j.n) {
            blk_counts_from_lex(j, base, v);
#pragma unroll
            for (int k = 0; k < kScanItems; ++k)
                if (base + k < j.n) j.cnt[base + k] = v[k];
        } else {
#pragma unroll
            for (int k = 0; k < kScanItems; ++k) v[k] = 0;
        }
    } else {
        scan_load(j, t, threadIdx.x, v);
    }
    int tot = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tot += v[k];
    tot = wave_sum_int(tot);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) tsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Both orders' scans in one launch, the second pass of the reduce-then-scan:
// workgroups [0, a.ntiles) scan job a, the rest job b.  A workgroup adds the
// tile sums before its own tile for its offset (a few thousand integers
// from L2 at most), then scans its kScanTile counts: kScanItems consecutive
// counts per thread, a wave scan of the thread totals and the four wave
// totals through LDS.
__global__ __launch_bounds__(256) void bin_scan_kernel(ScanJob a, ScanJob b) {
    __shared__ int red[4];
    int t = blockIdx.x;
    const bool second = t >= a.ntiles;
    const ScanJob j = second ? b : a;
    if (second) t -= a.ntiles;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

    int pre = 0;
    for (int k = tid; k < t; k += 256) pre += j.tsum[k];
    pre = wave_sum_int(pre);
    if (lane == 0) red[w] = pre;
    __syncthreads();
    pre = red[0] + red[1] + red[2] + red[3];
    __syncthreads();

    const long long base = (long long)t * kScanTile + (long long)tid * kScanItems;
    int v[kScanItems];
    const bool full = scan_load(j, t, tid, v);
    int tot = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int c = v[k];
        v[k] = tot;
        tot += c;
    }
    const int incl = wave_incl_scan_int(tot);
    if (lane == 63) red[w] = incl;
    __syncthreads();
    int off = pre + incl - tot;
    for (int k = 0; k < w; ++k) off += red[k];
    if (full) {
        int4* p = reinterpret_cast<int4*>(j.start + base);
#pragma unroll
        for (int k = 0; k < kScanItems / 4; ++k)
            p[k] = make_int4(off + v[4 * k], off + v[4 * k + 1], off + v[4 * k + 2],
                             off + v[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < j.n) j.start[base + k] = off + v[k];
    }
}

// Lex order by arrival: particle i at its cell start plus its slot (only
// in cells of two or more particles: alone in its cell a particle's rank
// is 0 without it).
__global__ void bin_scatter_kernel(long long N, BinBufs b,
                                   const int* __restrict__ start) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int kl = b.key_lex[i];
    const int s = start[kl];
    if (start[kl + 1] - s > 1) b.tmp[s + b.slot[i]] = (int)i;
}

// Final positions: inside its cell a particle takes the rank of its input
// index among the cell's particles, so both orders (and every floating-point
// sum downstream) are independent of the order in which the atomics were
// served.  A cell of the block order holds the same particles as its lex
// cell, so the rank is the same in both.
__global__ void bin_rank_kernel(long long N, BinBufs b,
                                const int* __restrict__ lex_start,
                                const int* __restrict__ blk_start,
                                int* __restrict__ lex_perm,
                                int* __restrict__ blk_perm) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int kl = b.key_lex[i];
    const int s = lex_start[kl], e = lex_start[kl + 1];
    int r = 0;
    if (e - s > 1)
        for (int k = s; k < e; ++k) r += b.tmp[k] < (int)i;
    lex_perm[s + r] = (int)i;
    blk_perm[blk_start[b.key_blk[i]] + r] = (int)i;
}

template <typename T>
__device__ __forceinline__ void bin_gather_one(const T* __restrict__ xin,
                                               const T* __restrict__ qin,
                                               long long p, const Geo& g,
                                               const DevParticles<T>& o) {
    const int i = o.perm[p];
    const T x = xin[3 * (long long)i], y = xin[3 * (long long)i + 1];
    T zw;
    int cx, cy, cz;
    cell_of<T>(x, y, xin[3 * (long long)i + 2], g, zw, cx, cy, cz);
    o.x[p] = x;
    o.y[p] = y;
    o.z[p] = zw;
    o.q[p] = qin[i];
    o.tx[p] = (T)((double)x * g.inv_h - (double)cx);
    o.ty[p] = (T)((double)y * g.inv_h - (double)cy);
    o.tz[p] = (T)((double)zw * g.inv_h - (double)cz);
    o.cx[p] = cx;
    o.cy[p] = cy;
    o.cz[p] = cz;
}

// Sorted copies of the particles in both orders.
template <typename T>
__global__ void bin_gather_kernel(const T* __restrict__ xin,
                                  const T* __restrict__ qin, long long N,
                                  Geo g, DevParticles<T> lex, DevParticles<T> blk) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    bin_gather_one<T>(xin, qin, p, g, lex);
    bin_gather_one<T>(xin, qin, p, g, blk);
}

// ------------------------------------------------------------------------
// spreading (step 2)
// ------------------------------------------------------------------------
// Per particle (lex order): z weights wz[P] (wave-uniform in the spread
// kernel), x weights wxp[P] and q * y weights wyq[P]; the gridding loop
// clamps a lane's index into the row and zeroes the weight outside the
// support (rows padded with zeros instead, 7 on each side, were slower in
// FP64 as well as FP32: more weight bytes through the caches).
//
// FP64: one weight per thread, each from its own exponential, so that the
// stores are coalesced: elements [0, N P) are wxp, [N P, 2 N P) wyq and
// [2 N P, 3 N P) wz.  (One row per thread with the Gaussian recurrence was
// slower here: 3N threads of long dependent chains.)
template <typename T, int P>
constexpr long long spread_weight_count(long long N) {
    return 3 * N * P;
}

template <typename T, int P>
__device__ __forceinline__ void spread_weight_elem(const DevParticles<T>& lx,
                                                   long long N, long long i,
                                                   const Geo& g,
                                                   T* __restrict__ wz,
                                                   T* __restrict__ wxp,
                                                   T* __restrict__ wyq) {
    static_assert(sizeof(T) == 8, "FP32 weights are written one row per thread");
    const T h = (T)g.h, a = (T)g.alpha;
    const long long nxy = N * P;
    if (i < 2 * nxy) {
        const bool isy = i >= nxy;
        const long long j = isy ? i - nxy : i;
        const long long p = j / P;
        // distance to grid point cx + 1 + u - P/2 (array index) in units of h
        const int u = (int)(j - p * P);
        const T t = isy ? lx.ty[p] : lx.tx[p];
        const T d = (t - (T)(1 + u - P / 2)) * h;
        T w = dexp<T>(-a * d * d);
        if (isy) w = lx.q[p] * w;
        (isy ? wyq : wxp)[j] = w;
    } else {
        const long long j = i - 2 * nxy;
        const long long p = j / P;
        const int d = (int)(j - p * P);
        const T dz = (lx.tz[p] - (T)(1 + d - P / 2)) * h;
        wz[j] = dexp<T>(-a * dz * dz);
    }
}

// FP32: one row per thread, threads [0, N) the x rows, [N, 2N) the y rows,
// [2N, 3N) the z rows (a wave's branch is uniform), every weight from its
// own offset in units of h, the row stored in 8-byte pieces.
template <int P>
__device__ __forceinline__ void spread_weight_row(const DevParticles<float>& lx,
                                                  long long p, int axis,
                                                  const Geo& g,
                                                  float* __restrict__ wz,
                                                  float* __restrict__ wxp,
                                                  float* __restrict__ wyq) {
    // offset in the cell in units of h; window point u is grid index
    // c + 1 + u - P/2 (c the particle's cell)
    const float t = axis == 0 ? lx.tx[p] : (axis == 1 ? lx.ty[p] : lx.tz[p]);
    const GaussC gc = gauss_consts(g);
    const float qp = axis == 1 ? lx.q[p] : 1.0f;
    float w[P];
#pragma unroll
    for (int u = 0; u < P; ++u) w[u] = gauss_u(t - (float)(1 + u - P / 2), gc.hi, gc.lo);
    if (axis == 1) {
#pragma unroll
        for (int u = 0; u < P; ++u) w[u] *= qp;
    }
    float2* dst = reinterpret_cast<float2*>((axis == 0 ? wxp : axis == 1 ? wyq : wz) + p * P);
#pragma unroll
    for (int u = 0; u < P; u += 2) dst[u / 2] = make_float2(w[u], w[u + 1]);
}

// Threads of the weight kernel for N particles.
template <typename T, int P>
constexpr long long spread_weight_threads(long long N) {
    return sizeof(T) == 8 ? spread_weight_count<T, P>(N) : 3 * N;
}

template <typename T, int P>
__device__ __forceinline__ void spread_weight_thread(const DevParticles<T>& lx,
                                                     long long N, long long i,
                                                     const Geo& g, T* __restrict__ wz,
                                                     T* __restrict__ wxp,
                                                     T* __restrict__ wyq) {
    if constexpr (sizeof(T) == 8) {
        spread_weight_elem<T, P>(lx, N, i, g, wz, wxp, wyq);
    } else {
        const int axis = (int)(i / N);
        spread_weight_row<P>(lx, i - axis * N, axis, g, wz, wxp, wyq);
    }
}

// Particle of weight-kernel thread i.
template <typename T, int P>
__device__ __forceinline__ long long spread_weight_particle(long long N, long long i) {
    if constexpr (sizeof(T) == 8) {
        return (i % (N * P)) / P;
    } else {
        return i % N;
    }
}

template <typename T, int P>
__global__ void spread_weights_kernel(DevParticles<T> lx, long long N, Geo g,
                                      T* __restrict__ wz, T* __restrict__ wxp,
                                      T* __restrict__ wyq) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= spread_weight_threads<T, P>(N)) return;
    spread_weight_thread<T, P>(lx, N, i, g, wz, wxp, wyq);
}

// A workgroup of spread_waves(P) waves owns the (x, y) pencils [X0, X0+8) x
// [Y0, Y0+8) (one lane per pencil) and the z cells [cz0, cz0+CZ); the waves
// split the particles of each cell row between them.  acc[d] holds grid
// point z = cz - P/2 + 1 + d while cell cz is processed; after cell cz the
// point z = cz - P/2 + 1 is final for this chunk: the waves' values are
// summed in LDS in a fixed order and written out.  Chunk jc writes KP*CZ
// consecutive z planes (mod M3) of partial grid jc % KP; with M3/CZ a
// multiple of KP, the chunks of one partial grid tile the period exactly, so
// every partial grid is fully written and the partial grids only need
// summing.
template <typename T, int P>
__device__ __forceinline__ void spread_body(
    const T* __restrict__ wz, const T* __restrict__ wxp,
    const T* __restrict__ wyq, const int* __restrict__ pcy,
    const int* __restrict__ cstart, T* __restrict__ Hpart,
    long long pstride, const Geo& g, int CZ, int KP, int tbx, int tby,
    int jc) {
    constexpr int W = spread_waves(P);
    __shared__ T red[W > 1 ? W : 1][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int X0 = tbx * kSpreadTile;
    const int Y0 = tby * kSpreadTile;
    const int lx = X0 + (lane >> 3);
    const int ly = Y0 + (lane & 7);
    const int cz0 = jc * CZ;
    const int cxlo = max(0, X0 - P), cxhi = min(g.M1 - 1, X0 + kSpreadTile - 2);
    const int cylo = max(0, Y0 - P), cyhi = min(g.M2 - 1, Y0 + kSpreadTile - 2);
    const bool writer = (lx < g.Mt1) && (ly < g.Mt2);
    T* __restrict__ out = Hpart + (long long)(jc % KP) * pstride +
                          (long long)lx * g.Mt2 + ly;
    const int zstart = cz0 - P / 2 + 1;

    T acc[P];
#pragma unroll
    for (int d = 0; d < P; ++d) acc[d] = (T)0;

    // sum one finished plane over the waves and write it
    auto finish = [&](T v, int zplane) {
        if constexpr (W == 1) {
            if (writer) out[(long long)imod(zplane, g.M3) * g.ncol] = v;
        } else {
            red[wv][lane] = v;
            __syncthreads();
            if (wv == 0 && writer) {
                T sum = red[0][lane];
#pragma unroll
                for (int w = 1; w < W; ++w) sum += red[w][lane];
                out[(long long)imod(zplane, g.M3) * g.ncol] = sum;
            }
            __syncthreads();
        }
    };

    // Bounds of the tile's cell rows (one x cell, the y cells in range) for
    // a z cell, one row per lane (at most kSpreadTile + P - 1 <= 64 rows),
    // loaded for the next z cell while the current one is processed.
    const int nr = (cxlo <= cxhi && cylo <= cyhi) ? cxhi - cxlo + 1 : 0;
    auto load_rows = [&](int cz, int& rs, int& re) {
        rs = re = 0;
        if (lane < nr) {
            const long long cb = ((long long)cz * g.M1 + cxlo + lane) * g.M2;
            rs = cstart[cb + cylo];
            re = cstart[cb + cyhi + 1];
        }
    };
    int rsA, reA;
    load_rows(cz0, rsA, reA);

    // Per z cell the rows' particles form one list (row k, then row k + 1,
    // in lex order), dealt round robin to the waves.  Lane i of a wave
    // looks up the wave's i-th particle of the list once: its index, x cell
    // and y cell stay in registers and are read back with readlane, so the
    // loop over the particles has no load whose address waits on another
    // load (only the weight loads of the particle itself).
    __shared__ int lst_incl[W][64], lst_off[W][64];
    for (int ci = 0; ci < CZ; ++ci) {
        int rsB = 0, reB = 0;
        if (ci + 1 < CZ) load_rows(cz0 + ci + 1, rsB, reB);
        {
            const int len = lane < nr ? reA - rsA : 0;
            int incl = len;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int v = __shfl_up(incl, d, 64);
                if (lane >= d) incl += v;
            }
            const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
            lst_incl[wv][lane] = incl;        // particles of rows 0..lane
            lst_off[wv][lane] = rsA - (incl - len);   // index = off + list position
            // the wave's own LDS rows: written and read by this wave only
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (int base = wv; base < total; base += 64 * W) {
                // lane i: list position base + W i, its row by binary search
                const int gi = base + W * lane;
                int k = 0;                    // rows 0..k-1 end at or before gi
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1)
                    if (k + step <= 63 && lst_incl[wv][k + step - 1] <= gi) k += step;
                const bool valid = gi < total;
                const int pi = valid ? lst_off[wv][k] + gi : 0;
                const int cxi = cxlo + k;
                const int cyi = valid ? pcy[pi] : 0;
                const int n = min(64, (total - base + W - 1) / W);
                auto coef = [&](int pp, int cxp, int cyp) -> T {
                    const int ux = lx - (cxp + 1);
                    const int uy = ly - (cyp + 1);
                    const T wx = wxp[(long long)pp * P + min(max(ux, 0), P - 1)];
                    const T wy = wyq[(long long)pp * P + min(max(uy, 0), P - 1)];
                    return ((unsigned)ux < (unsigned)P && (unsigned)uy < (unsigned)P)
                               ? wx * wy : (T)0;
                };
                // FP32: two particles per iteration (their loads in flight
                // together); FP64: one, since two particles' z weights (2 P
                // doubles in scalar registers) spill
                int i = 0;
                for (; sizeof(T) == 4 && i + 1 < n; i += 2) {
                    const int pA = __builtin_amdgcn_readlane(pi, i);
                    const int pB = __builtin_amdgcn_readlane(pi, i + 1);
                    const T cA = coef(pA, __builtin_amdgcn_readlane(cxi, i),
                                      __builtin_amdgcn_readlane(cyi, i));
                    const T cB = coef(pB, __builtin_amdgcn_readlane(cxi, i + 1),
                                      __builtin_amdgcn_readlane(cyi, i + 1));
                    const T* __restrict__ zA = wz + (long long)pA * P;
                    const T* __restrict__ zB = wz + (long long)pB * P;
#pragma unroll
                    for (int d = 0; d < P; ++d) acc[d] = fma(cA, zA[d], acc[d]);
#pragma unroll
                    for (int d = 0; d < P; ++d) acc[d] = fma(cB, zB[d], acc[d]);
                }
                for (; i < n; ++i) {
                    const int pA = __builtin_amdgcn_readlane(pi, i);
                    const T cA = coef(pA, __builtin_amdgcn_readlane(cxi, i),
                                      __builtin_amdgcn_readlane(cyi, i));
                    const T* __restrict__ zA = wz + (long long)pA * P;
#pragma unroll
                    for (int d = 0; d < P; ++d) acc[d] = fma(cA, zA[d], acc[d]);
                }
            }
        }
        rsA = rsB;
        reA = reB;
        // plane zstart + ci is final
        finish(acc[0], zstart + ci);
#pragma unroll
        for (int d = 0; d < P - 1; ++d) acc[d] = acc[d + 1];
        acc[P - 1] = (T)0;
    }
    // remaining planes of this chunk's KP*CZ-plane window
    const int base = zstart + CZ;
#pragma unroll
    for (int d = 0; d < P - 1; ++d) finish(acc[d], base + d);
    const int tail = KP * CZ - CZ;
    if (wv == 0 && writer) {
        for (int d = P - 1; d < tail; ++d)
            out[(long long)imod(base + d, g.M3) * g.ncol] = (T)0;
    }
}

template <typename T, int P>
__global__ __launch_bounds__(64 * spread_waves(P)) void spread_kernel(
    const T* __restrict__ wz, const T* __restrict__ wxp,
    const T* __restrict__ wyq, const int* __restrict__ pcy,
    const int* __restrict__ cstart, T* __restrict__ Hpart,
    long long pstride, Geo g, int CZ, int KP) {
    // (z chunk, y tile, x tile) in XCD order: the tiles that re-read a
    // particle's weights share one L2
    const unsigned ntile = gridDim.x * gridDim.y * gridDim.z;
    const unsigned lg = xcd_order(
        blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), ntile);
    spread_body<T, P>(wz, wxp, wyq, pcy, cstart, Hpart, pstride, g, CZ, KP,
                      (int)(lg % gridDim.x), (int)((lg / gridDim.x) % gridDim.y),
                      (int)(lg / (gridDim.x * gridDim.y)));
}

template <typename T>
__global__ void reduce_partials_kernel(const T* __restrict__ Hp, int KP,
                                       long long pstride, long long n, T scale,
                                       T* __restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T v = 0;
    for (int k = 0; k < KP; ++k) v += Hp[k * pstride + i];
    out[i] = v * scale;
}

// ------------------------------------------------------------------------
// k-space: z transforms
// ------------------------------------------------------------------------
// Forward real FFT along z of CB columns per block; columns 2t and 2t+1
// share one complex transform.  Sums the KP partial grids on load.
template <typename T, int CB = kZfftCols>
__device__ __forceinline__ void zfft_body(
    const T* __restrict__ H, int KP, long long pstride, T in_scale,
    cplx<T>* __restrict__ Fz, const Geo& g, const FftDesc& d,
    const cplx<T>* __restrict__ tw, int cbk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
    const int M3 = g.M3;
    const int stride = M3 + 1;
    cplx<T>* B = A + (CB / 2) * stride;
    const long long ncol = g.ncol;
    const long long c0 = (long long)cbk * CB;
    // kLoadBatch elements per thread at a time, their loads of one partial
    // grid issued together; the partial grids are added in order k = 0, 1,
    // ... as for a single element
    for (int i0 = threadIdx.x; i0 < CB * M3; i0 += kLoadBatch * blockDim.x) {
        T v[kLoadBatch];
        long long off[kLoadBatch];
        bool ok[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = i0 + u * blockDim.x;
            const int z = idx / CB, c = idx - z * CB;
            const long long col = c0 + c;
            ok[u] = idx < CB * M3 && col < ncol;
            off[u] = (long long)z * ncol + col;
            v[u] = 0;
        }
        for (int k = 0; k < KP; ++k) {
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u)
                if (ok[u]) v[u] += H[off[u] + k * pstride];
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = i0 + u * blockDim.x;
            if (idx < CB * M3) {
                const int z = idx / CB, c = idx - z * CB;
                T* at = reinterpret_cast<T*>(&A[(c >> 1) * stride + z]);
                at[c & 1] = v[u] * in_scale;
            }
        }
    }
    __syncthreads();
    cplx<T>* X = fft_lds<T>(A, B, CB / 2, stride, d, tw + d.twoff, -1);
    const int nh = M3 / 2 + 1;
    for (int idx = threadIdx.x; idx < nh * CB; idx += blockDim.x) {
        const int n3 = idx / CB, c = idx - n3 * CB;
        const long long col = c0 + c;
        if (col >= ncol) continue;
        const cplx<T> Xk = X[(c >> 1) * stride + n3];
        const cplx<T> Xm = X[(c >> 1) * stride + (n3 == 0 ? 0 : M3 - n3)];
        cplx<T> r;
        if ((c & 1) == 0) {
            r.x = (T)0.5 * (Xk.x + Xm.x);
            r.y = (T)0.5 * (Xk.y - Xm.y);
        } else {
            r.x = (T)0.5 * (Xk.y + Xm.y);
            r.y = (T)-0.5 * (Xk.x - Xm.x);
        }
        Fz[(long long)n3 * ncol + col] = r;
    }
}

template <typename T, int CB>
__global__ __launch_bounds__(256) void zfft_kernel(
    const T* __restrict__ H, int KP, long long pstride, T in_scale,
    cplx<T>* __restrict__ Fz, Geo g, FftDesc d,
    const cplx<T>* __restrict__ tw) {
    zfft_body<T, CB>(H, KP, pstride, in_scale, Fz, g, d, tw, blockIdx.x);
}

// Inverse real FFT along z; writes Ht[z][col] * out_scale.
template <typename T, int CB = kZfftCols>
__device__ __forceinline__ void zifft_body(
    const cplx<T>* __restrict__ Fz, T out_scale, T* __restrict__ Ht,
    const Geo& g, const FftDesc& d, const cplx<T>* __restrict__ tw, int cbk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
    const int M3 = g.M3;
    const int stride = M3 + 1;
    cplx<T>* B = A + (CB / 2) * stride;
    const long long ncol = g.ncol;
    const long long c0 = (long long)cbk * CB;
    const int half = M3 / 2;
    struct Two { cplx<T> a, b; };
    batched_copy<Two>(
        M3 * (CB / 2),
        [&](int idx) {
            const int k = idx / (CB / 2), t = idx - k * (CB / 2);
            const long long ca = c0 + 2 * t, cbb = ca + 1;
            const int src = (k <= half) ? k : M3 - k;
            Two f;
            f.a.x = f.a.y = f.b.x = f.b.y = (T)0;
            if (ca < ncol) f.a = Fz[(long long)src * ncol + ca];
            if (cbb < ncol) f.b = Fz[(long long)src * ncol + cbb];
            return f;
        },
        [&](int idx, Two f) {
            const int k = idx / (CB / 2), t = idx - k * (CB / 2);
            cplx<T> fa = f.a, fb = f.b;
            if (k == 0 || k == half) { fa.y = (T)0; fb.y = (T)0; }
            if (k > half) { fa.y = -fa.y; fb.y = -fb.y; }
            cplx<T> z;
            z.x = fa.x - fb.y;
            z.y = fa.y + fb.x;
            A[t * stride + k] = z;
        });
    __syncthreads();
    cplx<T>* X = fft_lds<T>(A, B, CB / 2, stride, d, tw + d.twoff, +1);
    for (int idx = threadIdx.x; idx < M3 * CB; idx += blockDim.x) {
        const int z = idx / CB, c = idx - z * CB;
        const long long col = c0 + c;
        if (col >= ncol) continue;
        const cplx<T> v = X[(c >> 1) * stride + z];
        Ht[(long long)z * ncol + col] = ((c & 1) ? v.y : v.x) * out_scale;
    }
}

template <typename T, int CB>
__global__ __launch_bounds__(256) void zifft_kernel(
    const cplx<T>* __restrict__ Fz, T out_scale, T* __restrict__ Ht, Geo g,
    FftDesc d, const cplx<T>* __restrict__ tw) {
    zifft_body<T, CB>(Fz, out_scale, Ht, g, d, tw, blockIdx.x);
}

// ------------------------------------------------------------------------
// k-space: slab transforms (eq. upsamplings: per-slab padded sizes)
// ------------------------------------------------------------------------
constexpr int kRowsPerBlock = 4;

// Zero-padded forward FFT along y of the Mt1 rows of slab blockIdx.y.
template <typename T>
__device__ __forceinline__ void rowfwd_body(
    const cplx<T>* __restrict__ Fz, cplx<T>* __restrict__ G,
    const SlabDesc* __restrict__ slabs, const Geo& g,
    const cplx<T>* __restrict__ tw, int rb, int slab, int nrb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SlabDesc& sd = slabs[slab];   // by reference: no private copy
    const int n2 = sd.n2;
    const UDiv divn2(n2);
    const int x0 = rb * nrb;
    if (x0 >= g.Mt1) return;
    const int nr = min(nrb, g.Mt1 - x0);
    cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* B = A + nrb * n2;
    const cplx<T>* src = Fz + (long long)slab * g.ncol;
    batched_copy<cplx<T>>(
        nr * n2,
        [&](int idx) {
            const int r = divn2(idx), j = idx - r * n2;
            cplx<T> v;
            v.x = v.y = (T)0;
            if (j < g.Mt2) v = src[(long long)(x0 + r) * g.Mt2 + j];
            return v;
        },
        [&](int idx, cplx<T> v) { A[idx] = v; });
    __syncthreads();
    cplx<T>* X = fft_lds<T>(A, B, nr, n2, sd.d2, tw + sd.d2.twoff, -1);
    cplx<T>* dst = G + sd.off;
    for (int idx = threadIdx.x; idx < nr * n2; idx += blockDim.x) {
        const int r = divn2(idx), j = idx - r * n2;
        dst[(long long)(x0 + r) * n2 + j] = X[r * n2 + j];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void rowfwd_kernel(
    const cplx<T>* __restrict__ Fz, cplx<T>* __restrict__ G,
    const SlabDesc* __restrict__ slabs, Geo g,
    const cplx<T>* __restrict__ tw) {
    rowfwd_body<T>(Fz, G, slabs, g, tw, blockIdx.x, blockIdx.y, kRowsPerBlock);
}

// Scaling factor (eq. scale_1p with G of eq. G_kappa_k), all constants and
// transform normalisations included.  Slab 0 uses the FP64 host table S0.
// Per-slab constants of the scaling: wave numbers k1 = c1 f1, k2 = c2 f2
// (f the signed frequency index), k3^2, and the Gaussian factor's
// coefficient (1 - eta) / (4 xi^2), so that no element divides by them.
struct SlabK {
    double c1, c2, k3s, ce;
    __device__ __forceinline__ SlabK(const SlabDesc& sd, const Geo& g) {
        const double twopi = 6.283185307179586476925286766559;
        c1 = twopi / (sd.n1 * g.h);
        c2 = twopi / (sd.n2 * g.h);
        const double k3 = twopi * sd.n3 / g.L3;
        k3s = k3 * k3;
        ce = (1.0 - g.eta) / (4.0 * g.xi * g.xi);
    }
};

template <typename T>
__device__ __forceinline__ T slab_scale(const SlabDesc& sd, const SlabK& kc, int kx,
                                        int ky, const T* __restrict__ S0) {
    if (sd.n3 == 0) return S0[(long long)kx * sd.n2 + ky];
    const int fx = (kx <= sd.n1 / 2) ? kx : kx - sd.n1;
    const int fy = (ky <= sd.n2 / 2) ? ky : ky - sd.n2;
    const double k1 = kc.c1 * fx;
    const double k2 = kc.c2 * fy;
    const double k2s = k1 * k1 + k2 * k2 + kc.k3s;
    if constexpr (sizeof(T) == 8) {
        return (T)(sd.pref * exp(-kc.ce * k2s) / k2s);
    } else {
        const float e = (float)(-kc.ce * k2s);
        return (float)sd.pref * __expf(e) / (float)k2s;
    }
}

constexpr int kColsPerBlock = 4;

// Wavenumber component d (0: x, 1: y, 2: z) of the mode (kx, ky, n3) of a
// slab, for ik-differentiation; zero at an even length's Nyquist index,
// whose sine mode the grid cannot carry.
__device__ __forceinline__ double slab_k(const SlabDesc& sd, int kx, int ky,
                                         const Geo& g, int d) {
    const double twopi = 6.283185307179586476925286766559;
    if (d == 0) {
        if (2 * kx == sd.n1) return 0.0;
        const int f = (kx <= sd.n1 / 2) ? kx : kx - sd.n1;
        return twopi * f / (sd.n1 * g.h);
    }
    if (d == 1) {
        if (2 * ky == sd.n2) return 0.0;
        const int f = (ky <= sd.n2 / 2) ? ky : ky - sd.n2;
        return twopi * f / (sd.n2 * g.h);
    }
    if (2 * sd.n3 == g.M3) return 0.0;
    return twopi * sd.n3 / g.L3;
}

// Fused column pass: zero-padded FFT along x, scaling, inverse FFT along x,
// restriction to the first Mt1 rows, for ncb columns ky.  dir >= 0 also
// multiplies the scaled spectrum by -i k_dir (the field component dir of
// the potential, E = -grad phi, by ik-differentiation).
template <typename T>
__device__ __forceinline__ void cols_body(
    cplx<T>* __restrict__ G, const SlabDesc* __restrict__ slabs, const Geo& g,
    const cplx<T>* __restrict__ tw, const T* __restrict__ S0, int cb,
    int slab, int ncb, int dir = -1) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SlabDesc& sd = slabs[slab];   // by reference: no private copy
    const int n1 = sd.n1, n2 = sd.n2;
    const int k0 = cb * ncb;
    if (k0 >= n2) return;
    const int nc = min(ncb, n2 - k0);
    const int stride = n1 + 1;
    const UDiv divc(ncb);
    cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* B = A + ncb * stride;
    cplx<T>* base = G + sd.off;
    batched_copy<cplx<T>>(
        n1 * ncb,
        [&](int idx) {
            const int x = divc(idx), c = idx - x * ncb;
            cplx<T> v;
            v.x = v.y = (T)0;
            if (x < g.Mt1 && c < nc) v = base[(long long)x * n2 + k0 + c];
            return v;
        },
        [&](int idx, cplx<T> v) {
            const int x = divc(idx), c = idx - x * ncb;
            A[c * stride + x] = v;
        });
    __syncthreads();
    cplx<T>* X = fft_lds<T>(A, B, ncb, stride, sd.d1,
                            tw + sd.d1.twoff, -1);
    cplx<T>* Y = (X == A) ? B : A;
    const SlabK kc(sd, g);
    const UDiv div1(n1);
    for (int idx = threadIdx.x; idx < n1 * ncb; idx += blockDim.x) {
        const int c = div1(idx), kx = idx - c * n1;
        const T s = (c < nc) ? slab_scale<T>(sd, kc, kx, k0 + c, S0) : (T)0;
        cplx<T> v = cscale<T>(X[c * stride + kx], s);
        if (dir >= 0) {
            // (-i k)(a + i b) = k b - i k a
            const T k = (T)slab_k(sd, kx, k0 + c, g, dir);
            const T a = v.x;
            v.x = k * v.y;
            v.y = -k * a;
        }
        X[c * stride + kx] = v;
    }
    __syncthreads();
    cplx<T>* Z = fft_lds<T>(X, Y, ncb, stride, sd.d1,
                            tw + sd.d1.twoff, +1);
    for (int idx = threadIdx.x; idx < g.Mt1 * ncb; idx += blockDim.x) {
        const int x = divc(idx), c = idx - x * ncb;
        if (c < nc) base[(long long)x * n2 + k0 + c] = Z[c * stride + x];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void cols_kernel(
    cplx<T>* __restrict__ G, const SlabDesc* __restrict__ slabs, Geo g,
    const cplx<T>* __restrict__ tw, const T* __restrict__ S0, int dir,
    unsigned ncblk, int nslab) {
    // The column blocks that share a 128-byte line of every row (GL of
    // them) run on one XCD, and these groups are dealt round robin to the
    // XCDs (the dispatcher deals blocks to XCD index % 8), so heavy slabs
    // still spread over the chip.  The grid is padded to a multiple of
    // 8 GL blocks; blocks mapped past the end return.
    constexpr int GL = 128 / (kColsPerBlock * 2 * (int)sizeof(T));
    const unsigned L = blockIdx.x + gridDim.x * blockIdx.y;
    const unsigned r = L % 8, m = L / 8;
    const unsigned idx = ((m / GL) * 8 + r) * GL + m % GL;
    if (idx >= ncblk * (unsigned)nslab) return;
    cols_body<T>(G, slabs, g, tw, S0, (int)(idx % ncblk), (int)(idx / ncblk),
                 kColsPerBlock, dir);
}

// Inverse FFT along y, restriction to the first Mt2 columns.
template <typename T>
__device__ __forceinline__ void rowinv_body(
    const cplx<T>* __restrict__ G, cplx<T>* __restrict__ Fz,
    const SlabDesc* __restrict__ slabs, const Geo& g,
    const cplx<T>* __restrict__ tw, int rb, int slab, int nrb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SlabDesc& sd = slabs[slab];   // by reference: no private copy
    const int n2 = sd.n2;
    const UDiv divn2(n2);
    const int x0 = rb * nrb;
    if (x0 >= g.Mt1) return;
    const int nr = min(nrb, g.Mt1 - x0);
    cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* B = A + nrb * n2;
    const cplx<T>* src = G + sd.off;
    batched_copy<cplx<T>>(
        nr * n2,
        [&](int idx) {
            const int r = divn2(idx), j = idx - r * n2;
            return src[(long long)(x0 + r) * n2 + j];
        },
        [&](int idx, cplx<T> v) { A[idx] = v; });
    __syncthreads();
    cplx<T>* X = fft_lds<T>(A, B, nr, n2, sd.d2, tw + sd.d2.twoff, +1);
    cplx<T>* dst = Fz + (long long)slab * g.ncol;
    const UDiv divm(g.Mt2);
    for (int idx = threadIdx.x; idx < nr * g.Mt2; idx += blockDim.x) {
        const int r = divm(idx), j = idx - r * g.Mt2;
        dst[(long long)(x0 + r) * g.Mt2 + j] = X[r * n2 + j];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void rowinv_kernel(
    const cplx<T>* __restrict__ G, cplx<T>* __restrict__ Fz,
    const SlabDesc* __restrict__ slabs, Geo g,
    const cplx<T>* __restrict__ tw) {
    rowinv_body<T>(G, Fz, slabs, g, tw, blockIdx.x, blockIdx.y, kRowsPerBlock);
}

// ------------------------------------------------------------------------
// gather (step 6) and its gradient
// ------------------------------------------------------------------------
// Lanes are particles: work unit bid / CH takes chunks of one block of
// BX x BY x BZ cells (64 consecutive particles per chunk), or of two
// y-adjacent blocks (32 of each per chunk); chunk slot bid % CH, further
// chunks strided by CH.  The grid planes the chunk's supports touch are
// staged one at a time in LDS (global_load_lds of the unit's footprint, the
// next plane in flight while the current one is read); each lane then reads
// its own P x P window of the plane from LDS.  FP64: the y weights of the
// window live in registers and x weights follow the Gaussian-gridding
// recurrence w(u+1) = w(u) r(u), r(u+1) = r(u) exp(-2 alpha h^2); FP32
// evaluates every x and y weight once from its offset; z weights are one
// exp per plane.

template <typename T, int P, bool FIELD = true>
__device__ __forceinline__ void gather_body(
    const T* __restrict__ Ht, const T* __restrict__ ptx,
    const T* __restrict__ pty, const T* __restrict__ ptz,
    const int* __restrict__ pcx, const int* __restrict__ pcy,
    const int* __restrict__ pcz, const int* __restrict__ perm,
    const int* __restrict__ cstart, const Geo& g, const BinGeo& bg, int CH,
    T scale, T* __restrict__ phi_out, T* __restrict__ E_out, int bid,
    int phi_stride = 1) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    constexpr int HP = P / 2;         // rows are read from LDS in two halves
    const int unit = bid / CH;
    const int slot = bid - unit * CH;
    // A unit is one block, or (pair) the even block 2 unit and the next one,
    // its y neighbour in the same row of blocks (nby is even).  The odd
    // block holds its cells with z reversed.
    const int b = bg.pair ? 2 * unit : unit;
    int bzk, bxk, byk;
    block_coords(b, bg, bzk, bxk, byk);
    int ylo = byk;
    if (bg.pair) {
        int bz2, bx2, by2;
        block_coords(b + 1, bg, bz2, bx2, by2);
        ylo = min(byk, by2);
    }
    const int sA = cstart[(long long)b * bg.cpb];
    const int eA = cstart[(long long)(b + 1) * bg.cpb];
    const int eB = bg.pair ? cstart[(long long)(b + 2) * bg.cpb] : eA;
    const int nA = eA - sA, nB = eB - eA;
    const int X0u = bxk * bg.BX + 1;  // array index of the footprint start
    const int Y0u = ylo * bg.BY + 1;
    const int Ux = bg.BX + P - 1;
    const int ldy = bg.ldy;           // LDS row pitch (see BinGeo)
    const int zl0 = bzk * bg.BZ - P / 2 + 1;  // z index of the union start
    const T h = (T)g.h, a = (T)g.alpha;
    const T C2 = (T)exp(-2.0 * g.alpha * g.h * g.h);
    const int lane = threadIdx.x;
    const int plane_stride = Ux * ldy;
    const int n16 = plane_stride * (int)sizeof(T) / 16;
    // 16-byte chunk c of a staged plane starts at row c per16 / ldy, column
    // c per16 % ldy of the footprint; lane's first chunk and the step of 64
    // chunks, so the staging loop carries row and column without dividing
    constexpr int per16 = 16 / (int)sizeof(T);
    const int rr0 = lane * per16 / ldy, cc0 = lane * per16 - rr0 * ldy;
    const int rstep = 64 * per16 / ldy, cstep = 64 * per16 - rstep * ldy;

    // Chunks.  One block: chunk k is its particles [64 k, 64 k + 64).  A
    // pair: the even block's particles go to lanes 0-31 and the odd one's
    // (stored with z reversed) to lanes 32-63, so that a 16- or 32-lane LDS
    // cycle reads windows of one block's cells only.
    //  - FP64: chunk k covers the z layers [z0, z1) of both blocks, z1 the
    //    last layer boundary at which neither block has more than 32
    //    particles in the chunk (a layer holding more is cut into runs of
    //    32); every wave of a unit walks the chunk sequence (a few ballots
    //    per chunk) up to its next chunk, chunks dealt round robin to the
    //    unit's CH waves.  Runs of 32 from each block drift apart in z like
    //    a random walk; cutting at shared layer boundaries was 20% faster
    //    for the FP64 gather at N = 1e5.
    //  - FP32: chunk k is the k-th run of 32 particles of each block from
    //    the bottom (the layer walk was 23% slower at FP32 N = 1e6, whose
    //    chunks are a third of the FP64 work).
    constexpr bool kLayerCut = sizeof(T) == 8;
    const int nchunk_single = (nA + 63) / 64;
    const int safe = nA > 0 ? sA : eA;   // a particle of the unit
    int knext = slot;                    // one block: the wave's next chunk
    // pair walk (uniform): the even block's particles below qA and the odd
    // block's from qB on (storage positions) are taken, layers below z0
    // complete; kw counts the chunks cut so far
    int z0 = 0, qA = sA, qB = eB, kw = 0;
    for (;;) {
        int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
        if (bg.pair && !kLayerCut) {
            const int kr = knext;
            if (kr >= max((nA + 31) / 32, (nB + 31) / 32)) break;
            a0 = sA + 32 * kr;
            a1 = min(a0 + 32, eA);
            b1 = eB - 32 * kr;
            b0 = max(b1 - 32, eA);
            knext += CH;
        } else if (bg.pair) {
            // layer boundaries as storage positions, z = 64 g + lane: the
            // even block's layer z starts at cA, the odd block's layers
            // below z occupy [cB, eB)
            int cAv[kMaxLayerGroups], cBv[kMaxLayerGroups];
            const int ng = bg.BZ / 64 + 1;
            const int cpl = bg.BX * bg.BY;
#pragma unroll
            for (int gq = 0; gq < kMaxLayerGroups; ++gq) {
                const int z = min(64 * gq + lane, bg.BZ);
                cAv[gq] = gq < ng ? cstart[(long long)b * bg.cpb + (long long)z * cpl] : 0;
                cBv[gq] = gq < ng ? cstart[(long long)(b + 1) * bg.cpb + (long long)(bg.BZ - z) * cpl] : 0;
            }
            auto at = [&](const int (&v)[kMaxLayerGroups], int z) {
                const int gq = z >> 6;
                int x = v[0];
#pragma unroll
                for (int t = 1; t < kMaxLayerGroups; ++t) x = gq == t ? v[t] : x;
                return __builtin_amdgcn_readlane(x, z & 63);
            };
            bool found = false;
            while (qA < eA || qB > eA) {
                int z1 = z0;
#pragma unroll
                for (int gq = 0; gq < kMaxLayerGroups; ++gq) {
                    const int z = 64 * gq + lane;
                    const bool ok = gq < ng && z > z0 && z <= bg.BZ && cAv[gq] - qA <= 32 &&
                                    qB - cBv[gq] <= 32;
                    z1 += __popcll(__ballot(ok));
                }
                int na, nb;                  // new qA, qB
                if (z1 > z0) {
                    na = at(cAv, z1);
                    nb = at(cBv, z1);
                    z0 = z1;
                } else {                     // layer z0 holds over 32 of a block
                    const int ea = at(cAv, z0 + 1), eb = at(cBv, z0 + 1);
                    na = min(qA + 32, ea);
                    nb = max(qB - 32, eb);
                    if (na == ea && nb == eb) ++z0;
                }
                const bool mine = kw % CH == slot;
                ++kw;
                if (mine) {
                    a0 = qA; a1 = na; b0 = nb; b1 = qB;
                    found = true;
                }
                qA = na;
                qB = nb;
                if (mine) break;
            }
            if (!found) break;
        } else if (knext >= nchunk_single) {
            break;
        }
        int p;
        bool act;
        if (bg.pair) {
            const int l = lane & 31;
            act = lane < 32 ? a0 + l < a1 : b0 + l < b1;
            p = lane < 32 ? a0 + l : b0 + l;
        } else {
            act = 64 * knext + lane < nA;
            p = sA + 64 * knext + lane;
            knext += CH;
        }
        const int pp = act ? p : safe;
        const T tx = ptx[pp], ty = pty[pp], tz = ptz[pp];
        const int ox = pcx[pp] - bxk * bg.BX;
        const int oy = pcy[pp] - ylo * bg.BY;
        const int oz = pcz[pp] - bzk * bg.BZ;
        int ozmin = act ? oz : 1 << 20, ozmax = act ? oz : -(1 << 20);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            ozmin = min(ozmin, __shfl_xor(ozmin, m));
            ozmax = max(ozmax, __shfl_xor(ozmax, m));
        }
        ozmin = __builtin_amdgcn_readfirstlane(ozmin);
        ozmax = __builtin_amdgcn_readfirstlane(ozmax);
        const int nplanes = ozmax - ozmin + P;

        // distances from the particle to the first point of its window
        // (array index cx + 1 - P/2), from the offset inside its cell
        const T dx0 = (tx - (T)(1 - P / 2)) * h;
        const T dy0 = (ty - (T)(1 - P / 2)) * h;
        // Gaussian-gridding recurrence seeds (FP64): value and ratio at the
        // window start
        T wx0 = 0, rx0 = 0, wyA = 0, ryA = 0;
        if constexpr (sizeof(T) == 8) {
            wx0 = dexp<T>(-a * dx0 * dx0);
            rx0 = dexp<T>(a * h * ((T)2 * dx0 - h));
            wyA = dexp<T>(-a * dy0 * dy0);
            ryA = dexp<T>(a * h * ((T)2 * dy0 - h));
        }
        T phi = 0, ex = 0, ey = 0, ez = 0;
        // FP32: every weight of the particle once, from offsets in units of
        // h (x and y in registers, z one per plane), and the sums taken per
        // row, then per plane, then over the planes, so that no level adds
        // the window's small edge terms to a much larger running sum (a flat
        // FP32 sum of the P^3 terms drops them and comes out low by a few
        // 1e-7, the same way for every particle)
        [[maybe_unused]] T wxa[sizeof(T) == 4 ? P : 1], txa[sizeof(T) == 4 ? P : 1];
        [[maybe_unused]] T wya[sizeof(T) == 4 ? P : 1], tya[sizeof(T) == 4 ? P : 1];
        [[maybe_unused]] GaussC gc{};
        if constexpr (sizeof(T) == 4) {
            gc = gauss_consts(g);
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const T ux = tx - (T)(1 + u - P / 2);
                const T uy = ty - (T)(1 + u - P / 2);
                wxa[u] = gauss_u(ux, gc.hi, gc.lo);
                txa[u] = ux * wxa[u];
                wya[u] = gauss_u(uy, gc.hi, gc.lo);
                tya[u] = uy * wya[u];
            }
        }

        // FP64: the y weights of the whole window, once per particle (the
        // Gaussian recurrence from the window's first point)
        [[maybe_unused]] T wyw[sizeof(T) == 8 ? P : 1], tyw[sizeof(T) == 8 ? P : 1];
        if constexpr (sizeof(T) == 8) {
            T w = wyA, rr = ryA;
#pragma unroll
            for (int u = 0; u < P; ++u) {
                wyw[u] = w;
                tyw[u] = (dy0 - (T)u * h) * w;
                w *= rr;
                rr *= C2;
            }
        }

        // Planes stream straight from global memory into LDS (16-byte
        // global_load_lds chunks, 64 per instruction), one plane ahead of
        // the plane being read.
        auto stage = [&](int ip, T* buf) {
            const T* src = Ht + (long long)imod(zl0 + ozmin + ip, g.M3) * g.ncol +
                           (long long)X0u * g.Mt2 + Y0u;
            int rr = rr0, cc = cc0;
            for (int k = 0; k * 64 < n16; ++k) {
                if (k * 64 + lane < n16) {
                    __builtin_amdgcn_global_load_lds(
                        (const void*)(src + (rr * g.Mt2 + cc)),
                        (__attribute__((address_space(3))) void*)(buf + k * 64 * per16),
                        16, 0, 0);
                }
                rr += rstep;
                cc += cstep;
                if (cc >= ldy) {
                    cc -= ldy;
                    ++rr;
                }
            }
        };
        stage(0, lds);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int ip = 0; ip < nplanes; ++ip) {
            T* cur = lds + (ip & 1) * plane_stride;
            T* nxt = lds + ((ip + 1) & 1) * plane_stride;
            if (ip + 1 < nplanes) stage(ip + 1, nxt);
            const int uz = ozmin + ip;
            const int dzi = uz - oz;
            const bool zin = act && dzi >= 0 && dzi < P;
            if constexpr (sizeof(T) == 4) {
                if (zin) {
                    const T vz = tz - (T)(dzi + 1 - P / 2);
                    const T wzv = gauss_u(vz, gc.hi, gc.lo);
                    const T* base = cur + ox * ldy + oy;
                    T sp = 0, spx = 0, spy = 0;
#pragma unroll
                    for (int dx = 0; dx < P; ++dx) {
                        const T* row = base + dx * ldy;
                        T sy = 0, sty = 0;
#pragma unroll
                        for (int u = 0; u < P; ++u) {
                            const T hv = row[u];
                            sy = fma(wya[u], hv, sy);
                            if constexpr (FIELD) sty = fma(tya[u], hv, sty);
                        }
                        sp = fma(wxa[dx], sy, sp);
                        if constexpr (FIELD) {
                            spx = fma(txa[dx], sy, spx);
                            spy = fma(wxa[dx], sty, spy);
                        }
                    }
                    phi = fma(wzv, sp, phi);
                    if constexpr (FIELD) {
                        ex = fma(wzv, spx, ex);
                        ey = fma(wzv, spy, ey);
                        ez = fma(vz * wzv, sp, ez);
                    }
                }
            }
            const T dz = (tz - (T)(dzi + 1 - P / 2)) * h;
            const T wzv = (zin && sizeof(T) == 8) ? dexp<T>(-a * dz * dz) : (T)0;
            const T tzw = dz * wzv;
            // lanes are sorted by z, so at the first and last planes whole
            // groups of lanes are idle and issue no LDS reads
            if (sizeof(T) == 8 && zin) {
                // whole rows (2 P FMAs each), summed over the plane with
                // the x weights, then scaled by the z weight once
                const T* base = cur + ox * ldy + oy;
                T wrec = wx0, rrec = rx0;
                T sp = 0, spx = 0, spy = 0;
                for (int dx = 0; dx < P; ++dx) {
                    const T wx = wrec;
                    wrec *= rrec;
                    rrec *= C2;
                    const T* row = base + dx * ldy;
                    T sy = 0, sty = 0;
#pragma unroll
                    for (int u0 = 0; u0 < P; u0 += HP) {
                        T hv[HP];
#pragma unroll
                        for (int u = 0; u < HP; ++u) hv[u] = row[u0 + u];
#pragma unroll
                        for (int u = 0; u < HP; ++u) {
                            sy = fma(wyw[u0 + u], hv[u], sy);
                            if constexpr (FIELD) sty = fma(tyw[u0 + u], hv[u], sty);
                        }
                    }
                    sp = fma(wx, sy, sp);
                    if constexpr (FIELD) {
                        spx = fma((dx0 - (T)dx * h) * wx, sy, spx);
                        spy = fma(wx, sty, spy);
                    }
                }
                phi = fma(wzv, sp, phi);
                if constexpr (FIELD) {
                    ex = fma(wzv, spx, ex);
                    ey = fma(wzv, spy, ey);
                    ez = fma(tzw, sp, ez);
                }
            }

            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        if (act) {
            const long long o = perm[p];
            if (phi_out) phi_out[o * phi_stride] = scale * phi;
            if (FIELD && E_out) {
                // FP32 sums offsets in units of h: the factor takes h
                const T f = sizeof(T) == 4 ? scale * (T)(2.0 * g.alpha * g.h) : scale * (T)2 * a;
                E_out[3 * o] = f * ex;
                E_out[3 * o + 1] = f * ey;
                E_out[3 * o + 2] = f * ez;
            }
        }
        __syncthreads();
    }
}

template <typename T, int P>
__global__ __launch_bounds__(64) void gather_kernel(
    const T* __restrict__ Ht, const T* __restrict__ ptx,
    const T* __restrict__ pty, const T* __restrict__ ptz,
    const int* __restrict__ pcx, const int* __restrict__ pcy,
    const int* __restrict__ pcz, const int* __restrict__ perm,
    const int* __restrict__ cstart, Geo g, BinGeo bg, int CH, T scale,
    T* __restrict__ phi_out, T* __restrict__ E_out) {
    // blocks in XCD order: neighbouring columns, whose footprints overlap,
    // stage their planes through one L2
    gather_body<T, P>(Ht, ptx, pty, ptz, pcx, pcy, pcz, perm, cstart, g, bg, CH,
                      scale, phi_out, E_out, (int)xcd_order(blockIdx.x, gridDim.x));
}

// ------------------------------------------------------------------------
// real-space sum over the cell list (eq. ewald1p_real, eq. force_real)
// ------------------------------------------------------------------------
// One wave takes a chunk of 16 consecutive targets of the block order
// (spatially compact: blocks of cells, cells in order inside a block); four
// lanes share a target and split its candidates.  Candidate sources are the
// cells within the cut-off of the chunk's cell box, walked as runs of the
// lex order (fixed z cell and x cell, a range of y cells clipped to the
// cut-off sphere around the box; z wraps with the image shift folded into
// the staged position).  Candidates are staged in LDS in batches of 64, the
// next batch's loads in flight while the current one is processed.  A first
// pass sets, per lane, one bit per candidate of its quarter within the
// cut-off (the target's own entry included: the second pass drops it); a
// second pass lets every lane pop its own bits, so the erfc and exp run for
// in-range pairs only, with most lanes busy (bits left over carry to the
// next batch's pass).  The four partial sums of a target are
// added with lane shuffles.
// erfc(xi r) / r and the radial field factor q (erfc(xi r)/r +
// 2 xi/sqrt(pi) exp(-xi^2 r^2)) / r^2 of one pair.  FP64 shares the
// exponential: erfc(x) = exp(-x^2) erfcx(x) with erfcx from the fitted
// polynomial of erfcx_poly.h (relative error 6e-12); FP32 does the same
// with a degree-8 float fit (2e-7).
// FP64 FMA in its three-operand form.  In polynomial loops the compiler
// otherwise picks the two-address form and copies the loop-invariant
// coefficient into the accumulator first, one extra move per step.
__device__ __forceinline__ double fma3(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// exp(y) for -708 < y <= 0: y = k ln2 + r with |r| <= ln2/2 (Cody-Waite
// reduction, with ln2 split into the two parts published with Sun's fdlibm
// exp, whose high part carries few enough bits that k ln2_hi is exact),
// exp(r) by a degree-8 Chebyshev fit on [-ln2/2, ln2/2] (3e-12 relative,
// below the erfcx fit's error; the Taylor series needs degree 9 for that),
// scaled by 2^k.
__device__ __forceinline__ double exp_neg(double y) {
    const double k = rint(y * 1.4426950408889634074);
    double r = fma3(k, -6.93147180369123816490e-01, y);
    r = fma3(k, -1.90821492927058770002e-10, r);
    double p = kExpC[kExpDeg];
#pragma unroll
    for (int j = kExpDeg - 1; j >= 0; --j) p = fma3(p, r, kExpC[j]);
    return ldexp(p, (int)k);
}

// Index of the lowest set bit of m, -1 for m = 0 (v_ffbl_b32 returns all
// ones for a zero input).
__device__ __forceinline__ int lowest_bit(unsigned m) {
    int b;
    asm("v_ffbl_b32 %0, %1" : "=v"(b) : "v"(m));
    return b;
}

// Smallest r^2 the pair terms are evaluated at: at the floor the field
// factor (about r^-3) stays finite in T, and a lane that adds nothing (charge
// 0) may sit there.  A pair closer than that is no physical input.
template <typename T> __device__ __forceinline__ constexpr T rs_r2_floor();
template <> __device__ __forceinline__ constexpr double rs_r2_floor<double>() { return 1e-150; }
template <> __device__ __forceinline__ constexpr float rs_r2_floor<float>() { return 1e-24f; }

template <typename T>
__device__ __forceinline__ void pair_terms(T r2, T xi, T xi2, T c_erf, T qn,
                                           T& ec, T& f);
template <>
__device__ __forceinline__ void pair_terms<double>(double r2, double xi,
                                                   double xi2, double c_erf,
                                                   double qn, double& ec,
                                                   double& f) {
    // hardware reciprocal square root and one Newton step (r2 is positive
    // and normal: distinct particles of a box of size ~1)
    double rinv = __builtin_amdgcn_rsq(r2);
    {
        const double hr = r2 * rinv;
        const double en = fma(-hr, rinv, 1.0);          // 1 - r2 y^2
        rinv = fma(0.5 * rinv, en, rinv);
    }
    const double r = r2 * rinv;
    const double x = fmin(xi * r, kErfcxXmax);
    const double e = exp_neg(-xi2 * r2);
    // hardware reciprocal (about 23 bits) and one Newton step: 1 / den to
    // about 2^-46, far below the fit's error (den is in [1, 1 + 8 A])
    const double den = 1.0 + kErfcxA * x;
    double t = __builtin_amdgcn_rcp(den);
    t = t * (2.0 - den * t);
    const double cu = 2.0 / (1.0 - kErfcxTmin);
    const double u = fma3(t, cu, -1.0 - kErfcxTmin * cu);
    double pv = kErfcxC[kErfcxDeg];
#pragma unroll
    for (int k = kErfcxDeg - 1; k >= 0; --k) pv = fma3(pv, u, kErfcxC[k]);
    ec = e * (t * pv) * rinv;
    f = qn * (ec + c_erf * e) * (rinv * rinv);
}
template <>
__device__ __forceinline__ void pair_terms<float>(float r2, float xi,
                                                  float xi2, float c_erf,
                                                  float qn, float& ec,
                                                  float& f) {
    // hardware reciprocal square root: r2 is positive and normal, so the
    // library's scaling for denormal inputs is not needed
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rinv;
    const float x = fminf(xi * r, (float)kErfcxXmax);
    const float e = __expf(-xi2 * r2);
    const float t = __builtin_amdgcn_rcpf(1.0f + (float)kErfcxA * x);
    const float cu = (float)(2.0 / (1.0 - kErfcxTmin));
    const float u = fmaf(t, cu, (float)(-1.0 - kErfcxTmin * 2.0 / (1.0 - kErfcxTmin)));
    float pv = kErfcxCF[kErfcxDegF];
#pragma unroll
    for (int k = kErfcxDegF - 1; k >= 0; --k) pv = fmaf(pv, u, kErfcxCF[k]);
    ec = e * (t * pv) * rinv;
    f = qn * (ec + c_erf * e) * (rinv * rinv);
}

// PXY: x and y periodic too (SE3P); sources are taken from every image
// within the cut-off.
template <typename T, bool PXY = false>
__device__ __forceinline__ void realspace_body(
    const DevParticles<T>& blk, const DevParticles<T>& lx, const Geo& g,
    T xi, T rc, int R, T* __restrict__ phi_out, T* __restrict__ E_out,
    int pbeg, int pend, int chunk, int part, int nparts) {
    __shared__ T cx_[128], cy_[128], cz_[128], cq_[128];
    __shared__ int rows_s[64], rows_e[64], rows_h[64];
    const int lane = threadIdx.x;
    const int tq = lane >> 2;         // target of this lane within the chunk
    const int kq = lane & 3;          // quarter of each candidate batch
    const T rc2 = rc * rc;
    const T c_erf = (T)1.1283791670955125738961589031215 * xi;  // 2 xi / sqrt(pi)
    const T xi2 = xi * xi;
    const T L3 = (T)g.L3;
    const T L1 = (T)(g.M1 * g.h), L2 = (T)(g.M2 * g.h);
    (void)L1; (void)L2;
    const double rcell2 = (double)rc * (double)rc / (g.h * g.h);

    // one chunk of 16 consecutive targets of the block order; four lanes
    // share a target and split its candidates
    {
        const int p = pbeg + 16 * chunk + tq;
        const bool act = p < pend;
        const int pp = act ? p : pend - 1;
        const T xt = blk.x[pp], yt = blk.y[pp], zt = blk.z[pp];
        // cell box of the chunk's targets
        int mnx = act ? blk.cx[pp] : 1 << 20, mxx = act ? blk.cx[pp] : -(1 << 20);
        int mny = act ? blk.cy[pp] : 1 << 20, mxy = act ? blk.cy[pp] : -(1 << 20);
        int mnz = act ? blk.cz[pp] : 1 << 20, mxz = act ? blk.cz[pp] : -(1 << 20);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            mnx = min(mnx, __shfl_xor(mnx, m)); mxx = max(mxx, __shfl_xor(mxx, m));
            mny = min(mny, __shfl_xor(mny, m)); mxy = max(mxy, __shfl_xor(mxy, m));
            mnz = min(mnz, __shfl_xor(mnz, m)); mxz = max(mxz, __shfl_xor(mxz, m));
        }
        const int bx0 = __builtin_amdgcn_readfirstlane(mnx), bx1 = __builtin_amdgcn_readfirstlane(mxx);
        const int by0 = __builtin_amdgcn_readfirstlane(mny), by1 = __builtin_amdgcn_readfirstlane(mxy);
        const int bz0 = __builtin_amdgcn_readfirstlane(mnz), bz1 = __builtin_amdgcn_readfirstlane(mxz);
        T phi = 0, ex = 0, ey = 0, ez = 0;

        // In-range bits of a lane: bits 0..15 for the older of the two
        // staged batches (LDS slot old_slot), bits 16..31 for the newer one.
        // Each pop pass runs until every lane's older bits are consumed;
        // lanes that finish early take bits of the newer batch meanwhile,
        // and what is left of those carries to the next pass.  Lanes whose
        // lists are long in one batch thus catch up in the next instead of
        // holding the whole wave (about 7% off the FP64 sum).
        unsigned int mask = 0u;
        auto pop = [&](int old_slot, bool drain) {
            // bit b < 16: candidate kq + 4 b of the older slot; b >= 16:
            // candidate kq + 4 (b - 16) of the newer one
            // every pass pops one bit per lane, lowest (oldest) first, so
            // the pass count is the largest count of the bits to consume
            const unsigned jbase = (unsigned)(kq + 64 * old_slot) * sizeof(T);
            int np = __popc(drain ? mask : (mask & 0xFFFFu));
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) np = max(np, __shfl_xor(np, m));
            np = __builtin_amdgcn_readfirstlane(np);
            for (int it = 0; it < np; ++it) {
                const bool has = mask != 0u;
                // lowest set bit; a lane out of bits (b = -1) reads some
                // staged candidate and adds nothing: its charge is taken
                // as 0
                const int b = lowest_bit(mask);
                // byte offset of entry (kq + 4 b + 64 old_slot) mod 128
                const unsigned jb = ((unsigned)b * (4u * sizeof(T)) + jbase) &
                                    (128u * sizeof(T) - 1u);
                mask &= mask - 1u;
                auto at = [&](const T* a) {
                    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(a) + jb);
                };
                const T dx = xt - at(cx_), dy = yt - at(cy_), dz = zt - at(cz_);
                const T r2v = dx * dx + dy * dy + dz * dz;
                const T qv = at(cq_);
                // the mask pass tests the cut-off only, so the target's own
                // entry (r2 = 0) has a bit too; it adds nothing either.  The
                // floor keeps those lanes' reciprocals finite.
                const bool use = has & (r2v > (T)0);
                const T r2 = fmax(r2v, rs_r2_floor<T>());
                const T qn = use ? qv : (T)0;
                T ec, f;
                pair_terms<T>(r2, xi, xi2, c_erf, qn, ec, f);
                phi = fma(qn, ec, phi);
                ex = fma(f, dx, ex);
                ey = fma(f, dy, ey);
                ez = fma(f, dz, ez);
            }

        };
        auto process = [&](int n, int slot) {
            // pass 1: one bit per in-range candidate j = kq + 4 i
            unsigned int nmask = 0u;
            auto test = [&](int i, bool full) {
                const int j = kq + 4 * i;
                const int jj = 64 * slot + j;
                const T dx = xt - cx_[jj], dy = yt - cy_[jj], dz = zt - cz_[jj];
                const T r2 = dx * dx + dy * dy + dz * dz;
                // bitwise, not short-circuit: straight-line compares instead
                // of a branch per candidate (all j < 64 are in the slot)
                const bool in = (full | (j < n)) & (r2 <= rc2);
                // candidates are tested from the last down, each bit shifted
                // in from below (one add with carry per candidate)
                nmask = nmask + nmask + (unsigned int)in;
            };
            if (n == 64) {             // a full batch: straight-line code
#pragma unroll
                for (int i = 15; i >= 0; --i) test(i, true);
            } else {
                for (int i = (n + 3) / 4 - 1; i >= 0; --i) test(i, false);
            }
            if (!act) nmask = 0u;
            mask |= nmask << 16;
            // pass 2: pop until the older batch is done (its slot is written
            // again by the next batch); the rest carries
            pop(slot ^ 1, false);
            mask >>= 16;
        };

        // Candidate rows: fixed z cell and x cell, the y cells of the row
        // clipped to the cut-off sphere around the chunk's cell box.  Rows
        // are set up 64 at a time by the lanes (bounds from the lex cell
        // starts, image shift in periods) with an exclusive scan of their
        // lengths in LDS; each batch's lanes then find their candidate by a
        // binary search of that scan, so a wave never walks rows one by one.
        // (PXY: x cells unclipped, wrapped with an image shift, and the y
        // range split into one row per period it touches, NYP at most)
        const int xlo = PXY ? bx0 - R : max(0, bx0 - R);
        const int xhi = PXY ? bx1 + R : min(g.M1 - 1, bx1 + R);
        const int nxr = xhi - xlo + 1;
        const int NYP = PXY ? (by1 - by0 + 2 * R) / g.M2 + 2 : 1;
        // this part's rows: r = part + nparts i for i in [0, nrows), so that
        // every part draws rows from the whole extent of the cut-off sphere
        // (contiguous row ranges gave the middle parts most of the work,
        // and with 4 or 8 parts the same part index always fell on the
        // same XCD)
        const int nrows_all = (bz1 - bz0 + 1 + 2 * R) * nxr * NYP;
        const int nrows = (nrows_all - part + nparts - 1) / nparts;
        // The part's rows are visited with a stride coprime to their count
        // (the first of 7, 11, 13, ... that does not divide it), so that a
        // batch of consecutive candidates mixes rows from across the sphere
        // and the targets' in-range counts per batch are more even (pop
        // passes fill 86% of the lane slots instead of 82% at FP64 N = 1e5,
        // in a CPU model of the wave).
        int rstride = 7;
        {
            constexpr int kPrimes[6] = {7, 11, 13, 17, 19, 23};
#pragma unroll
            for (int k = 5; k >= 0; --k)
                if (nrows % kPrimes[k] != 0) rstride = kPrimes[k];
        }
        int gbase = 0;                 // uniform: first row index of the current group
        int gtotal = 0, gdone = 0;     // uniform: candidates of the group, taken
        auto load_rows = [&](int base) {
            const int ri = base + lane;
            const int r = part + nparts * (int)(((long long)ri * rstride) % max(nrows, 1));
            int rs = 0, re = 0, rsh = 0;
            if (ri < nrows) {

                const int rz = PXY ? r / NYP : r;
                const int czu = bz0 - R + rz / nxr;
                const int cxu = xlo + rz % nxr;
                const int gz = max(0, max(bz0 - czu, czu - bz1) - 1);
                const int gx = max(0, max(bx0 - cxu, cxu - bx1) - 1);
                const double rem = rcell2 - (double)gz * gz - (double)gx * gx;
                if (rem >= 0.0) {
                    const int gy = (int)sqrt(rem) + 1;
                    const int czw = imod(czu, g.M3);
                    if constexpr (PXY) {
                        const int cxn = imod(cxu, g.M1);
                        const int ylu = by0 - gy, yhu = by1 + gy;
                        const int k = (ylu - imod(ylu, g.M2)) / g.M2 + r % NYP;   // period
                        const int ya = max(ylu, k * g.M2) - k * g.M2;
                        const int yb = min(yhu, k * g.M2 + g.M2 - 1) - k * g.M2;
                        if (ya <= yb) {
                            const long long cb = ((long long)czw * g.M1 + cxn) * g.M2;
                            rs = lx.start[cb + ya];
                            re = lx.start[cb + yb + 1];
                            // image shifts in periods, 10 bits each
                            rsh = (((cxu - cxn) / g.M1 + 512) << 20) | ((k + 512) << 10) |
                                  ((czu - czw) / g.M3 + 512);
                        }
                    } else {
                        const int cxn = cxu;
                        const int ylo = max(0, by0 - gy), yhi = min(g.M2 - 1, by1 + gy);
                        const long long cb = ((long long)czw * g.M1 + cxn) * g.M2;
                        rs = lx.start[cb + ylo];
                        re = lx.start[cb + yhi + 1];
                        rsh = (czu - czw) / g.M3;
                    }
                }
            }
            const int len = re - rs;
            int incl = len;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int v = __shfl_up(incl, d);
                if (lane >= d) incl += v;
            }
            __syncthreads();           // earlier rows no longer read
            rows_s[lane] = rs;
            rows_e[lane] = incl - len; // exclusive prefix of the lengths
            rows_h[lane] = rsh;
            __syncthreads();
            gtotal = __builtin_amdgcn_readfirstlane(__shfl(incl, 63));
            gdone = 0;
        };
        if (gbase < nrows) load_rows(gbase);
        // The next batch of up to 64 candidates: lane l takes candidate
        // cand (-1: none) of image shift csh periods.  Returns the count.
        // A batch never spans two row groups.
        auto next_batch = [&](int& cand, int& csh) {
            cand = -1;
            csh = 0;
            while (gdone >= gtotal) {
                gbase += 64;
                if (gbase >= nrows) return 0;
                load_rows(gbase);
            }
            const int n = min(64, gtotal - gdone);
            if (lane < n) {
                const int o = gdone + lane;
                int k = 0;             // last row whose prefix is <= o
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1)
                    if (rows_e[k + step] <= o) k += step;
                cand = rows_s[k] + (o - rows_e[k]);
                csh = rows_h[k];
            }
            gdone += n;
            return n;
        };
        // Software pipeline: the loads of the next batch are in flight
        // while the current batch is processed from LDS.
        int cand, csh;
        int nA = next_batch(cand, csh);
        // source position of candidate c in the image of packed shift sh
        auto src = [&](int c, int sh, T& px, T& py, T& pz) {
            if constexpr (PXY) {
                px = lx.x[c] + (T)((sh >> 20) - 512) * L1;
                py = lx.y[c] + (T)(((sh >> 10) & 1023) - 512) * L2;
                pz = lx.z[c] + (T)((sh & 1023) - 512) * L3;
            } else {
                px = lx.x[c];
                py = lx.y[c];
                pz = lx.z[c] + (T)sh * L3;
            }
        };
        T ax = 0, ay = 0, az = 0, aq = 0;
        if (cand >= 0) {
            src(cand, csh, ax, ay, az);
            aq = lx.q[cand];
        }
        int slot = 0;
        int nbatch = 0;                // uniform
        while (nA > 0) {
            ++nbatch;
            __syncthreads();           // the batch before the previous one is done
            cx_[64 * slot + lane] = ax;
            cy_[64 * slot + lane] = ay;
            cz_[64 * slot + lane] = az;
            cq_[64 * slot + lane] = aq;
            __syncthreads();
            const int nB = next_batch(cand, csh);
            T bx_ = 0, by_ = 0, bz_ = 0, bq_ = 0;
            if (cand >= 0) {
                src(cand, csh, bx_, by_, bz_);
                bq_ = lx.q[cand];
            }
            process(nA, slot);
            slot ^= 1;
            ax = bx_;
            ay = by_;
            az = bz_;
            aq = bq_;
            nA = nB;
        }
        // Lanes out of bits read an entry of the newer slot (and multiply it
        // by a charge of 0).  After a single batch that slot was never
        // staged: it gets finite values first.
        if (nbatch == 1) {
            cx_[64 + lane] = (T)0;
            cy_[64 + lane] = (T)0;
            cz_[64 + lane] = (T)0;
            cq_[64 + lane] = (T)0;
            __syncthreads();
        }
        // the last batch's carried bits (slot ^ 1 is the last one written)
        pop(slot ^ 1, true);
        // sum the four lanes of each target
#pragma unroll
        for (int m = 1; m <= 2; m <<= 1) {
            phi += __shfl_xor(phi, m);
            ex += __shfl_xor(ex, m);
            ey += __shfl_xor(ey, m);
            ez += __shfl_xor(ez, m);
        }
        if (act && kq == 0) {
            const long long o = blk.perm[p];
            phi_out[o] = phi;
            E_out[3 * o] = ex;
            E_out[3 * o + 1] = ey;
            E_out[3 * o + 2] = ez;
        }
    }
}

// Block b: chunk b / nparts, part b % nparts of its candidate rows; part k
// writes slice k of phi_out / E_out (N values / N x 3 each).
template <typename T, bool PXY>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void realspace_kernel(
    DevParticles<T> blk, DevParticles<T> lx, Geo g, int N, T xi, T rc, int R,
    int nparts, T* __restrict__ phi_out, T* __restrict__ E_out) {
    // With one part per chunk (large N) the blocks run in XCD order, so that
    // neighbouring chunks, which share most candidates, run on one L2 (3%
    // at FP32 N = 1e6).  With several parts it was slower, and is not used.
    const int bx = nparts == 1 ? (int)xcd_order(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int chunk = bx / nparts, part = bx - chunk * nparts;
    realspace_body<T, PXY>(blk, lx, g, xi, rc, R, phi_out + (long long)part * N,
                           E_out + 3LL * part * N, 0, N, chunk, part, nparts);
}

// ------------------------------------------------------------------------
// potential-only gather (ik-differentiation gathers each field component
// from its own grid with the potential's weights)
// ------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__(64) void gather_phi_kernel(
    const T* __restrict__ Ht, const T* __restrict__ ptx,
    const T* __restrict__ pty, const T* __restrict__ ptz,
    const int* __restrict__ pcx, const int* __restrict__ pcy,
    const int* __restrict__ pcz, const int* __restrict__ perm,
    const int* __restrict__ cstart, Geo g, BinGeo bg, int CH, T scale,
    T* __restrict__ out, int ostride) {
    gather_body<T, P, false>(Ht, ptx, pty, ptz, pcx, pcy, pcz, perm, cstart, g, bg, CH,
                             scale, out, nullptr, (int)xcd_order(blockIdx.x, gridDim.x),
                             ostride);
}

// ------------------------------------------------------------------------
// totals and energy
// ------------------------------------------------------------------------
constexpr int kCombineThreads = 256;

// Totals of the particles [p0 + 256 blk, ...) below p0 + N, and their
// energy partial sum into *partial.
template <typename T>
__device__ __forceinline__ void combine_body(
    long long p0, long long N, const T* __restrict__ q,
    const T* __restrict__ phiF, const T* __restrict__ EF,
    const T* __restrict__ phiR, const T* __restrict__ ER, int nparts,
    long long pstr, double self_c, unsigned flags, T* __restrict__ phi,
    T* __restrict__ E, double* __restrict__ partial, int blk) {
    __shared__ double red[kCombineThreads];
    const long long li = (long long)blk * kCombineThreads + threadIdx.x;
    const long long i = p0 + li;
    double u = 0.0;
    if (li < N) {
        const T qi = q[i];
        T ph = 0;
        if (flags & 1u) ph += phiF[i];
        if (flags & 2u) {       // real-space partial sums, in part order
            T r = phiR[i];
            for (int k = 1; k < nparts; ++k) r += phiR[k * pstr + i];
            ph += r;
        }
        if (flags & 4u) ph += (T)(-self_c) * qi;
        if (phi) phi[i] = ph;
        if (E) {
            for (int d = 0; d < 3; ++d) {
                T v = 0;
                if (flags & 1u) v += EF[3 * i + d];
                if (flags & 2u) {
                    T r = ER[3 * i + d];
                    for (int k = 1; k < nparts; ++k) r += ER[3 * (k * pstr + i) + d];
                    v += r;
                }
                E[3 * i + d] = (flags & SE1P_FORCE) ? qi * v : v;
            }
        }
        u = (double)qi * (double)ph;
    }
    red[threadIdx.x] = u;
    __syncthreads();
    for (int w = kCombineThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *partial = red[0];
}

template <typename T>
__global__ __launch_bounds__(kCombineThreads) void combine_kernel(
    long long N, const T* __restrict__ q, const T* __restrict__ phiF,
    const T* __restrict__ EF, const T* __restrict__ phiR,
    const T* __restrict__ ER, int nparts, double self_c, unsigned flags,
    T* __restrict__ phi, T* __restrict__ E, double* __restrict__ partials) {
    combine_body<T>(0, N, q, phiF, EF, phiR, ER, nparts, N, self_c, flags, phi,
                    E, partials + blockIdx.x, blockIdx.x);
}

__device__ __forceinline__ void energy_body(const double* __restrict__ partials,
                                            int n, double* __restrict__ energy) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *energy = 0.5 * red[0];
}

__global__ __launch_bounds__(256) void energy_final_kernel(
    const double* __restrict__ partials, int n, double* __restrict__ energy) {
    energy_body(partials, n, energy);
}

// ------------------------------------------------------------------------
// optional input validation (device side)
// ------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void check_kernel(
    const T* __restrict__ x, const T* __restrict__ q, long long N, double L1,
    double L2, int* __restrict__ flag, double* __restrict__ qsum) {
    __shared__ double r1[256], r2[256];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (i < N) {
        const double xx = x[3 * i], yy = x[3 * i + 1], zz = x[3 * i + 2];
        const bool ok = (xx >= 0.0) && (xx < L1) && (yy >= 0.0) && (yy < L2) &&
                        (zz == zz) && (zz - zz == 0.0);
        if (!ok) atomicOr(flag, 1);
        a = q[i];
        b = fabs((double)q[i]);
    }
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&qsum[0], r1[0]);
        atomicAdd(&qsum[1], r2[0]);
    }
}

// ------------------------------------------------------------------------
// batches: every system of a batch in one launch per stage
// ------------------------------------------------------------------------
// Particle-wise stages run over the packed particles and look their system
// up; grid-shaped stages are persistent: a fixed set of blocks pulls
// (system, tile) items from a global counter until the queue is empty, so
// uneven systems balance across the chip without one launch per system.
// A stage's items are split into 8 ranges, one per XCD, each holding a
// spatially contiguous part of the list (neighbouring tiles, which read the
// same particles and grid rows, then share one L2) with about an eighth of
// the estimated cost, most expensive items first inside the range.  The
// dispatcher deals blocks round-robin to the XCDs, so block b pulls from
// range b % 8, through that range's own counter (kQCtrStride ints apart, a
// cache line each).  qb holds the 9 bounds of the stage's ranges.
__device__ __forceinline__ int next_item(int* __restrict__ ctr,
                                         const int* __restrict__ qb) {
    __shared__ int s_item;
    __syncthreads();                 // the previous item is done with LDS
    if (threadIdx.x == 0) {
        const int r = (int)(blockIdx.x & 7u);
        const int i = qb[r] + atomicAdd(&ctr[r * kQCtrStride], 1);
        s_item = i < qb[r + 1] ? i : -1;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(s_item);
}

template <typename T>
__global__ void bbin_keys_kernel(const T* __restrict__ xin, long long N,
                                 const int* __restrict__ sys_of,
                                 const SysDesc<T>* __restrict__ sys,
                                 BinBufs b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SysDesc<T>& sd = sys[sys_of[i]];
    int kl, kb;
    cell_keys<T>(xin, i, sd.g, sd.bg, kl, kb);
    count_keys(i, kl + (int)sd.cl0, kb + (int)sd.cb0, b, true);
}

// Sorted position p belongs to the same system as its input index.
template <typename T>
__global__ void bbin_gather_kernel(const T* __restrict__ xin,
                                   const T* __restrict__ qin, long long N,
                                   const int* __restrict__ sys_of,
                                   const SysDesc<T>* __restrict__ sys,
                                   DevParticles<T> lex, DevParticles<T> blk) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const Geo& g = sys[sys_of[p]].g;
    bin_gather_one<T>(xin, qin, p, g, lex);
    bin_gather_one<T>(xin, qin, p, g, blk);
}

template <typename T, int P>
__global__ void bspread_weights_kernel(DevParticles<T> lx, long long N,
                                       const int* __restrict__ sys_of,
                                       const SysDesc<T>* __restrict__ sys,
                                       T* __restrict__ wz, T* __restrict__ wxp,
                                       T* __restrict__ wyq) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= spread_weight_threads<T, P>(N)) return;
    const long long p = spread_weight_particle<T, P>(N, i);
    spread_weight_thread<T, P>(lx, N, i, sys[sys_of[p]].g, wz, wxp, wyq);
}

template <typename T, int P>
__global__ __launch_bounds__(64 * spread_waves(P)) void bspread_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, const T* __restrict__ wz,
    const T* __restrict__ wxp, const T* __restrict__ wyq,
    const int* __restrict__ pcy, const int* __restrict__ cstart) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        spread_body<T, P>(wz, wxp, wyq, pcy, cstart + sd.cl0, sd.Hpart,
                          sd.pstride, g, sd.CZ, sd.KP, w.a, w.b, w.c);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void bzfft_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, const cplx<T>* __restrict__ tw) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        zfft_body<T>(sd.Hpart, sd.KP, sd.pstride, (T)1, sd.Fz, g, sd.dz, tw, w.a);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void browfwd_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, const cplx<T>* __restrict__ tw) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        rowfwd_body<T>(sd.Fz, sd.G, sd.slabs, g, tw, w.a, w.b, w.c);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void bcols_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, const cplx<T>* __restrict__ tw) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        cols_body<T>(sd.G, sd.slabs, g, tw, sd.S0, w.a, w.b, w.c);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void browinv_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, const cplx<T>* __restrict__ tw) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        rowinv_body<T>(sd.G, sd.Fz, sd.slabs, g, tw, w.a, w.b, w.c);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void bzifft_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, const cplx<T>* __restrict__ tw) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        zifft_body<T>(sd.Fz, (T)1, sd.Ht, g, sd.dz, tw, w.a);
    }
}

template <typename T, int P>
__global__ __launch_bounds__(64) void bgather_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, DevParticles<T> blk,
    T* __restrict__ phi_out, T* __restrict__ E_out) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        const BinGeo bg = sd.bg;
        gather_body<T, P>(sd.Ht, blk.tx, blk.ty, blk.tz, blk.cx, blk.cy, blk.cz,
                          blk.perm, blk.start + sd.cb0, g, bg, bg.CH, (T)1,
                          phi_out, E_out, w.a);
    }
}

template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void brealspace_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, DevParticles<T> blk,
    DevParticles<T> lx, T* __restrict__ phi_out, T* __restrict__ E_out) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const Geo g = sd.g;
        DevParticles<T> l = lx;
        l.start = lx.start + sd.cl0;
        realspace_body<T>(blk, l, g, (T)sd.xi, (T)sd.rc, sd.R, phi_out, E_out,
                          (int)sd.p0, (int)(sd.p0 + sd.n), w.a, 0, 1);
    }
}

// item (s, blk): particles [p0 + 256 blk, ...) of system s
template <typename T>
__global__ __launch_bounds__(kCombineThreads) void bcombine_kernel(
    const SysDesc<T>* __restrict__ sys, const Item* __restrict__ items,
    const int* __restrict__ qb, int* __restrict__ ctr, const T* __restrict__ q,
    const T* __restrict__ phiF, const T* __restrict__ EF,
    const T* __restrict__ phiR, const T* __restrict__ ER, unsigned flags,
    T* __restrict__ phi, T* __restrict__ E, double* __restrict__ partials) {
    for (;;) {
        const int it = next_item(ctr, qb);
        if (it < 0) return;
        const Item w = items[it];
        const SysDesc<T>& sd = sys[w.sys];
        const unsigned f = sd.rs ? flags : (flags & ~2u);
        combine_body<T>(sd.p0, sd.n, q, phiF, EF, phiR, ER, 1, 0, sd.self_c, f,
                        phi, E, partials + sd.e0 + w.a, w.a);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void benergy_kernel(
    const SysDesc<T>* __restrict__ sys, int nsys,
    const double* __restrict__ partials, double* __restrict__ energy) {
    for (int s = blockIdx.x; s < nsys; s += gridDim.x) {
        const SysDesc<T>& sd = sys[s];
        energy_body(partials + sd.e0, sd.ncomb, energy + s);
        __syncthreads();
    }
}

inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// Grid of the column pass: ncblk x nslab blocks padded to a multiple of
// 8 GL (cols_kernel maps dispatch index to block).
template <typename T>
dim3 cols_grid(unsigned ncblk, int nslab) {
    const unsigned gl = 128u / (kColsPerBlock * 2u * (unsigned)sizeof(T));
    const unsigned n = ncblk * (unsigned)nslab, q = 8u * gl;
    return dim3((n + q - 1) / q * q);
}

}  // namespace

// ==========================================================================
// launchers
// ==========================================================================
#define SE1P_CHECK_LAUNCH()                                  \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return -5;      \
    } while (0)

int launch_fill_int(int* p, long long n, int v, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fill_int_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, p,
                       n, v);
    SE1P_CHECK_LAUNCH();
    return 0;
}

// Clears the counts, then (after the key kernel has counted) scans both
// orders, places the particles by arrival and then by rank.
// both: clear the block-order counts too (the batch counts them by atomics;
// one system derives them from the lex counts).
static int bin_clear(const BinBufs& b, bool both, hipStream_t s) {
    const long long n = b.ncl + 1 + (both ? b.ncb + 1 : 0);
    hipLaunchKernelGGL(bin_clear_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, b, both);
    SE1P_CHECK_LAUNCH();
    return 0;
}

// bg, M1, M2 null / unused: block-order counts already in cnt_blk (batch);
// else taken from the lex counts of the one system's grid.
static int bin_sort(long long N, const BinBufs& b, int* lex_start, int* blk_start,
                    int* lex_perm, int* blk_perm, hipStream_t s,
                    const BinGeo* bg = nullptr, int M1 = 0, int M2 = 0) {
    const ScanJob ja{b.cnt_lex, lex_start, b.ncl + 1, b.tsum, b.ntl, nullptr, BinGeo{}, 0, 0};
    const ScanJob jb{b.cnt_blk, blk_start, b.ncb + 1, b.tsum + b.ntl, b.ntb,
                     bg ? b.cnt_lex : nullptr, bg ? *bg : BinGeo{}, M1, M2};
    hipLaunchKernelGGL(bin_tile_sum_kernel, dim3(b.ntl + b.ntb), dim3(256), 0, s, ja, jb,
                       b.tsum);
    hipLaunchKernelGGL(bin_scan_kernel, dim3(b.ntl + b.ntb), dim3(256), 0, s, ja, jb);
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(nblk(N, 256)), dim3(256), 0, s, N, b,
                       (const int*)lex_start);
    hipLaunchKernelGGL(bin_rank_kernel, dim3(nblk(N, 256)), dim3(256), 0, s, N, b,
                       (const int*)lex_start, (const int*)blk_start, lex_perm, blk_perm);
    SE1P_CHECK_LAUNCH();
    return 0;
}

template <typename T>
int launch_bin(const T* x_in, const T* q_in, long long N, const Geo& g,
               const BinGeo& bg, const BinBufs& b, DevParticles<T>& lex,
               DevParticles<T>& blk, hipStream_t s) {
    // counting sort into the lex and block orders (the block order numbers
    // the same cells, so both share each particle's rank in its cell)
    int rc;
    if ((rc = bin_clear(b, false, s))) return rc;
    hipLaunchKernelGGL(bin_keys_kernel<T>, dim3(nblk(N, 256)), dim3(256), 0, s,
                       x_in, N, g, bg, b);
    SE1P_CHECK_LAUNCH();
    if ((rc = bin_sort(N, b, lex.start, blk.start, lex.perm, blk.perm, s, &bg, g.M1, g.M2)))
        return rc;
    hipLaunchKernelGGL(bin_gather_kernel<T>, dim3(nblk(N, 256)), dim3(256), 0,
                       s, x_in, q_in, N, g, lex, blk);
    SE1P_CHECK_LAUNCH();
    return 0;
}

template <typename T, int P>
static int spread_p(const DevParticles<T>& lex, long long N, const Geo& g,
                    int CZ, int KP, T* wz, T* wxp, T* wyq, T* Hpart,
                    long long pstride, hipStream_t s) {
    hipLaunchKernelGGL((spread_weights_kernel<T, P>),
                       dim3(nblk(spread_weight_threads<T, P>(N), 256)), dim3(256), 0, s,
                       lex, N, g, wz, wxp, wyq);
    SE1P_CHECK_LAUNCH();
    dim3 grid((g.Mt1 + kSpreadTile - 1) / kSpreadTile,
              (g.Mt2 + kSpreadTile - 1) / kSpreadTile, g.M3 / CZ);
    hipLaunchKernelGGL((spread_kernel<T, P>), grid, dim3(64 * spread_waves(P)), 0, s, wz, wxp,
                       wyq, lex.cy, lex.start, Hpart, pstride, g, CZ, KP);
    SE1P_CHECK_LAUNCH();
    return 0;
}

#define SE1P_P_CASES(F) \
    F(4) F(6) F(8) F(10) F(12) F(14) F(16) F(18) F(20) F(22) F(24) F(26) F(28) F(30) F(32)

template <typename T>
int launch_spread(const DevParticles<T>& lex, long long N, const Geo& g,
                  int CZ, int KP, T* wz, T* wxp, T* wyq, T* Hpart,
                  long long pstride, hipStream_t s) {
    switch (g.P) {
#define SE1P_SPREAD_CASE(PP) \
    case PP: return spread_p<T, PP>(lex, N, g, CZ, KP, wz, wxp, wyq, Hpart, pstride, s);
        SE1P_P_CASES(SE1P_SPREAD_CASE)
#undef SE1P_SPREAD_CASE
        default: return -8;
    }
}

template <typename T>
int launch_reduce_partials(const T* Hpart, int KP, long long pstride,
                           long long n, T scale, T* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials_kernel<T>, dim3(nblk(n, 256)), dim3(256),
                       0, s, Hpart, KP, pstride, n, scale, out);
    SE1P_CHECK_LAUNCH();
    return 0;
}

// Columns per block of one system's z transforms: 16 on grids of fewer
// than 32768 columns (blocks of 32 would leave most CUs with one block:
// 0.065 against 0.070 ms for the transform stage at FP64 N = 1e5, 9216
// columns), 32 on larger ones (0.247 against 0.258 ms at FP32 N = 1e6).
inline int zfft_cols(long long ncol) { return ncol < 32768 ? 16 : 32; }

template <typename T>
void launch_zfft(const T* Hin, int KP, long long pstride, T in_scale, cplx<T>* Fz,
                 const Geo& g, const FftDesc& dz, const cplx<T>* tw, hipStream_t s) {
    const int CB = zfft_cols(g.ncol);
    const unsigned ncb = (unsigned)((g.ncol + CB - 1) / CB);
    const size_t zsm = 2 * (CB / 2) * (size_t)(g.M3 + 1) * sizeof(cplx<T>);
    if (CB == 16)
        hipLaunchKernelGGL((zfft_kernel<T, 16>), dim3(ncb), dim3(256), zsm, s, Hin, KP,
                           pstride, in_scale, Fz, g, dz, tw);
    else
        hipLaunchKernelGGL((zfft_kernel<T, 32>), dim3(ncb), dim3(256), zsm, s, Hin, KP,
                           pstride, in_scale, Fz, g, dz, tw);
}

template <typename T>
void launch_zifft(const cplx<T>* Fz, T out_scale, T* Ht, const Geo& g,
                  const FftDesc& dz, const cplx<T>* tw, hipStream_t s) {
    const int CB = zfft_cols(g.ncol);
    const unsigned ncb = (unsigned)((g.ncol + CB - 1) / CB);
    const size_t zsm = 2 * (CB / 2) * (size_t)(g.M3 + 1) * sizeof(cplx<T>);
    if (CB == 16)
        hipLaunchKernelGGL((zifft_kernel<T, 16>), dim3(ncb), dim3(256), zsm, s, Fz,
                           out_scale, Ht, g, dz, tw);
    else
        hipLaunchKernelGGL((zifft_kernel<T, 32>), dim3(ncb), dim3(256), zsm, s, Fz,
                           out_scale, Ht, g, dz, tw);
}

template <typename T>
int launch_kspace(const T* Hin, int KP, long long pstride, T in_scale,
                  const Geo& g, int nslab, const SlabDesc* d_slabs,
                  const SlabDesc* h_slabs, const FftDesc& dz,
                  const cplx<T>* tw, const T* S0, cplx<T>* Fz, cplx<T>* G,
                  T out_scale, T* Ht, hipStream_t s) {
    const size_t cs = sizeof(cplx<T>);
    launch_zfft<T>(Hin, KP, pstride, in_scale, Fz, g, dz, tw, s);
    SE1P_CHECK_LAUNCH();
    int n1max = 0, n2max = 0;
    for (int i = 0; i < nslab; ++i) {
        n1max = n1max > h_slabs[i].n1 ? n1max : h_slabs[i].n1;
        n2max = n2max > h_slabs[i].n2 ? n2max : h_slabs[i].n2;
    }
    const size_t rsm = 2 * (size_t)kRowsPerBlock * n2max * cs;
    dim3 rgrid((g.Mt1 + kRowsPerBlock - 1) / kRowsPerBlock, nslab);
    hipLaunchKernelGGL(rowfwd_kernel<T>, rgrid, dim3(256), rsm, s, Fz, G,
                       d_slabs, g, tw);
    SE1P_CHECK_LAUNCH();
    const size_t csm = 2 * (size_t)kColsPerBlock * (n1max + 1) * cs;
    const unsigned ncblk = (unsigned)((n2max + kColsPerBlock - 1) / kColsPerBlock);
    const dim3 cgrid = cols_grid<T>(ncblk, nslab);
    hipLaunchKernelGGL(cols_kernel<T>, cgrid, dim3(256), csm, s, G, d_slabs, g,
                       tw, S0, -1, ncblk, nslab);
    SE1P_CHECK_LAUNCH();
    hipLaunchKernelGGL(rowinv_kernel<T>, rgrid, dim3(256), rsm, s, G, Fz,
                       d_slabs, g, tw);
    SE1P_CHECK_LAUNCH();
    launch_zifft<T>(Fz, out_scale, Ht, g, dz, tw, s);
    SE1P_CHECK_LAUNCH();
    return 0;
}

// The k-space solve with the field by ik-differentiation: the forward
// transforms once, then per output (the potential and the three field
// components) the column pass with its multiplier on a copy of the
// row-transformed slabs, the inverse row and z transforms.  Gk holds three
// copies of G (slab_elems each); Htk three output grids of gstride values.
template <typename T>
int launch_kspace_ik(const T* Hin, int KP, long long pstride, const Geo& g,
                     int nslab, const SlabDesc* d_slabs, const SlabDesc* h_slabs,
                     const FftDesc& dz, const cplx<T>* tw, const T* S0,
                     cplx<T>* Fz, cplx<T>* G, cplx<T>* Gk, long long slab_elems,
                     T* Ht, T* Htk, long long gstride, hipStream_t s) {
    const size_t cs = sizeof(cplx<T>);
    launch_zfft<T>(Hin, KP, pstride, (T)1, Fz, g, dz, tw, s);
    SE1P_CHECK_LAUNCH();
    int n1max = 0, n2max = 0;
    for (int i = 0; i < nslab; ++i) {
        n1max = n1max > h_slabs[i].n1 ? n1max : h_slabs[i].n1;
        n2max = n2max > h_slabs[i].n2 ? n2max : h_slabs[i].n2;
    }
    const size_t rsm = 2 * (size_t)kRowsPerBlock * n2max * cs;
    dim3 rgrid((g.Mt1 + kRowsPerBlock - 1) / kRowsPerBlock, nslab);
    hipLaunchKernelGGL(rowfwd_kernel<T>, rgrid, dim3(256), rsm, s, Fz, G,
                       d_slabs, g, tw);
    SE1P_CHECK_LAUNCH();
    for (int d = 0; d < 3; ++d)
        if (hipMemcpyAsync(Gk + d * slab_elems, G, (size_t)slab_elems * cs,
                           hipMemcpyDeviceToDevice, s) != hipSuccess)
            return -5;
    const size_t csm = 2 * (size_t)kColsPerBlock * (n1max + 1) * cs;
    const unsigned ncblk = (unsigned)((n2max + kColsPerBlock - 1) / kColsPerBlock);
    const dim3 cgrid = cols_grid<T>(ncblk, nslab);
    for (int d = -1; d < 3; ++d) {
        cplx<T>* Gd = d < 0 ? G : Gk + d * slab_elems;
        T* Hd = d < 0 ? Ht : Htk + d * gstride;
        hipLaunchKernelGGL(cols_kernel<T>, cgrid, dim3(256), csm, s, Gd, d_slabs, g,
                           tw, S0, d, ncblk, nslab);
        SE1P_CHECK_LAUNCH();
        hipLaunchKernelGGL(rowinv_kernel<T>, rgrid, dim3(256), rsm, s, Gd, Fz,
                           d_slabs, g, tw);
        SE1P_CHECK_LAUNCH();
        launch_zifft<T>(Fz, (T)1, Hd, g, dz, tw, s);
        SE1P_CHECK_LAUNCH();
    }
    return 0;
}

template <typename T, int P>
static int gather_phi_p(const T* Ht, const DevParticles<T>& blk, const Geo& g,
                        const BinGeo& bg, T scale, T* out, int ostride, hipStream_t s) {
    const unsigned nb = (unsigned)(bg.nbx * bg.nby * bg.nbz / (1 + bg.pair)) * bg.CH;
    const size_t lds = 2 * (size_t)(bg.BX + P - 1) * bg.ldy * sizeof(T);
    hipLaunchKernelGGL((gather_phi_kernel<T, P>), dim3(nb), dim3(64), lds, s, Ht,
                       blk.tx, blk.ty, blk.tz, blk.cx, blk.cy, blk.cz, blk.perm,
                       blk.start, g, bg, bg.CH, scale, out, ostride);
    SE1P_CHECK_LAUNCH();
    return 0;
}

template <typename T>
int launch_gather_phi(const T* Ht, const DevParticles<T>& blk, const Geo& g,
                      const BinGeo& bg, T scale, T* out, int ostride, hipStream_t s) {
    switch (g.P) {
#define SE1P_GPHI_CASE(PP) \
    case PP: return gather_phi_p<T, PP>(Ht, blk, g, bg, scale, out, ostride, s);
        SE1P_P_CASES(SE1P_GPHI_CASE)
#undef SE1P_GPHI_CASE
        default: return -8;
    }
}

template <typename T, int P>
static int gather_p(const T* Ht, const DevParticles<T>& blk, const Geo& g,
                    const BinGeo& bg, T scale, T* phi_out, T* E_out,
                    hipStream_t s) {
    const unsigned nb = (unsigned)(bg.nbx * bg.nby * bg.nbz / (1 + bg.pair)) * bg.CH;
    const int Ux = bg.BX + P - 1;
    const size_t lds = 2 * (size_t)Ux * bg.ldy * sizeof(T);
    hipLaunchKernelGGL((gather_kernel<T, P>), dim3(nb), dim3(64), lds, s, Ht,
                       blk.tx, blk.ty, blk.tz, blk.cx, blk.cy, blk.cz, blk.perm,
                       blk.start, g, bg, bg.CH, scale, phi_out, E_out);
    SE1P_CHECK_LAUNCH();
    return 0;
}

template <typename T>
int launch_gather(const T* Ht, const DevParticles<T>& blk, long long N,
                  const Geo& g, const BinGeo& bg, T scale, T* phi_out,
                  T* E_out, hipStream_t s) {
    (void)N;
    switch (g.P) {
#define SE1P_GATHER_CASE(PP) \
    case PP: return gather_p<T, PP>(Ht, blk, g, bg, scale, phi_out, E_out, s);
        SE1P_P_CASES(SE1P_GATHER_CASE)
#undef SE1P_GATHER_CASE
        default: return -8;
    }
}

template <typename T>
int launch_realspace(const DevParticles<T>& lex, const DevParticles<T>& blk,
                     long long N, const Geo& g, const BinGeo& bg, double xi,
                     double rc, int nparts, bool periodic3, T* phi_out, T* E_out,
                     hipStream_t s) {
    (void)bg;
    const int R = (int)ceil(rc / g.h);
    const unsigned nb = (unsigned)((N + 15) / 16) * nparts;   // chunks of 16 targets
    if (periodic3) {
        // image shifts are packed in 10 bits per direction
        if (R + 2 > 200 * std::min(std::min(g.M1, g.M2), g.M3)) return -8;
        hipLaunchKernelGGL((realspace_kernel<T, true>), dim3(nb), dim3(64), 0, s, blk, lex,
                           g, (int)N, (T)xi, (T)rc, R, nparts, phi_out, E_out);
    } else {
        hipLaunchKernelGGL((realspace_kernel<T, false>), dim3(nb), dim3(64), 0, s, blk, lex,
                           g, (int)N, (T)xi, (T)rc, R, nparts, phi_out, E_out);
    }
    SE1P_CHECK_LAUNCH();
    return 0;
}

// ------------------------------------------------------------------------
// SE3P: periodic grid <-> extended grid
// ------------------------------------------------------------------------
// Array index a of the extended grid (Mt1 x Mt2, gridding and gather) holds
// grid point a - P/2 of the period; the periodic grid gf (M1 x M2) sums
// every extended point of its class mod (M1, M2) over the KP partial grids.
template <typename T>
__global__ void fold_kernel(const T* __restrict__ Hp, int KP, long long pstride,
                            Geo g, Geo gf, T* __restrict__ Hper) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)g.M3 * gf.ncol) return;
    const int y = (int)(i % gf.Mt2);
    const long long r = i / gf.Mt2;
    const int x = (int)(r % gf.Mt1);
    const int z = (int)(r / gf.Mt1);
    const int a0 = imod(x + g.P / 2, gf.Mt1), b0 = imod(y + g.P / 2, gf.Mt2);
    T v = 0;
    for (int k = 0; k < KP; ++k)
        for (int a = a0; a < g.Mt1; a += gf.Mt1)
            for (int b = b0; b < g.Mt2; b += gf.Mt2)
                v += Hp[k * pstride + (long long)z * g.ncol + (long long)a * g.Mt2 + b];
    Hper[i] = v;
}

template <typename T>
__global__ void unfold_kernel(const T* __restrict__ Htp, Geo g, Geo gf,
                              T* __restrict__ Ht) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)g.M3 * g.ncol) return;
    const int b = (int)(i % g.Mt2);
    const long long r = i / g.Mt2;
    const int a = (int)(r % g.Mt1);
    const int z = (int)(r / g.Mt1);
    Ht[i] = Htp[(long long)z * gf.ncol + (long long)imod(a - g.P / 2, gf.Mt1) * gf.Mt2 +
                imod(b - g.P / 2, gf.Mt2)];
}

template <typename T>
int launch_fold(const T* Hpart, int KP, long long pstride, const Geo& g,
                const Geo& gf, T* Hper, hipStream_t s) {
    const long long n = (long long)g.M3 * gf.ncol;
    hipLaunchKernelGGL(fold_kernel<T>, dim3(nblk(n, 256)), dim3(256), 0, s, Hpart, KP,
                       pstride, g, gf, Hper);
    SE1P_CHECK_LAUNCH();
    return 0;
}

template <typename T>
int launch_unfold(const T* Htp, const Geo& g, const Geo& gf, T* Ht, hipStream_t s) {
    const long long n = (long long)g.M3 * g.ncol;
    hipLaunchKernelGGL(unfold_kernel<T>, dim3(nblk(n, 256)), dim3(256), 0, s, Htp, g, gf, Ht);
    SE1P_CHECK_LAUNCH();
    return 0;
}

template <typename T>
int launch_combine(long long N, const T* q_in, const T* phiF, const T* EF,
                   const T* phiR, const T* ER, int nparts, double self_c,
                   unsigned flags, T* phi, T* E, double* partials, int nblkc,
                   double* energy, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel<T>, dim3(nblkc), dim3(kCombineThreads),
                       0, s, N, q_in, phiF, EF, phiR, ER, nparts, self_c, flags,
                       phi, E, partials);
    SE1P_CHECK_LAUNCH();
    if (energy) {
        hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(256), 0, s,
                           partials, nblkc, energy);
        SE1P_CHECK_LAUNCH();
    }
    return 0;
}

template <typename T>
int launch_check(const T* x, const T* q, long long N, double L1, double L2,
                 int* flag, double* qsum, hipStream_t s) {
    hipLaunchKernelGGL(check_kernel<T>, dim3(nblk(N, 256)), dim3(256), 0, s, x,
                       q, N, L1, L2, flag, qsum);
    SE1P_CHECK_LAUNCH();
    return 0;
}

// ---- batches --------------------------------------------------------------
template <typename T, int P>
static int batch_p(const BatchArgs<T>& a, const T* x, const T* q, T* phi,
                   T* E, double* energy, unsigned flags, hipStream_t s) {
    const long long N = a.ntot;
    int rc;
    // counts and queue counters are cleared by kernels (no memset nodes if
    // the sequence is captured in a graph)
    if ((rc = bin_clear(a.bins, true, s))) return rc;
    if ((rc = launch_fill_int(a.qctr, 8 * kQCtrStride * kNumQueues, 0, s))) return rc;
    hipLaunchKernelGGL(bbin_keys_kernel<T>, dim3(nblk(N, 256)), dim3(256), 0, s,
                       x, N, a.sys_of, a.sys, a.bins);
    SE1P_CHECK_LAUNCH();
    if ((rc = bin_sort(N, a.bins, a.lex.start, a.blk.start, a.lex.perm, a.blk.perm, s)))
        return rc;
    hipLaunchKernelGGL(bbin_gather_kernel<T>, dim3(nblk(N, 256)), dim3(256), 0,
                       s, x, q, N, a.sys_of, a.sys, a.lex, a.blk);
    SE1P_CHECK_LAUNCH();
    const BatchLaunch* L = a.q;
    if (flags & 1u) {
        hipLaunchKernelGGL((bspread_weights_kernel<T, P>),
                           dim3(nblk(spread_weight_threads<T, P>(N), 256)), dim3(256), 0, s,
                           a.lex, N, a.sys_of, a.sys, a.wz, a.wxp, a.wyq);
        hipLaunchKernelGGL((bspread_kernel<T, P>), dim3(L[kQSpread].grid),
                           dim3(64 * spread_waves(P)), L[kQSpread].lds, s, a.sys, L[kQSpread].items,
                           L[kQSpread].qb, a.qctr + 8 * kQCtrStride * kQSpread, a.wz, a.wxp,
                           a.wyq, a.lex.cy, a.lex.start);
        SE1P_CHECK_LAUNCH();
        hipLaunchKernelGGL(bzfft_kernel<T>, dim3(L[kQZfft].grid), dim3(256),
                           L[kQZfft].lds, s, a.sys, L[kQZfft].items,
                           L[kQZfft].qb, a.qctr + 8 * kQCtrStride * kQZfft, a.tw);
        hipLaunchKernelGGL(browfwd_kernel<T>, dim3(L[kQRowFwd].grid), dim3(256),
                           L[kQRowFwd].lds, s, a.sys, L[kQRowFwd].items,
                           L[kQRowFwd].qb, a.qctr + 8 * kQCtrStride * kQRowFwd, a.tw);
        hipLaunchKernelGGL(bcols_kernel<T>, dim3(L[kQCols].grid), dim3(256),
                           L[kQCols].lds, s, a.sys, L[kQCols].items,
                           L[kQCols].qb, a.qctr + 8 * kQCtrStride * kQCols, a.tw);
        hipLaunchKernelGGL(browinv_kernel<T>, dim3(L[kQRowInv].grid), dim3(256),
                           L[kQRowInv].lds, s, a.sys, L[kQRowInv].items,
                           L[kQRowInv].qb, a.qctr + 8 * kQCtrStride * kQRowInv, a.tw);
        hipLaunchKernelGGL(bzifft_kernel<T>, dim3(L[kQZifft].grid), dim3(256),
                           L[kQZifft].lds, s, a.sys, L[kQZifft].items,
                           L[kQZifft].qb, a.qctr + 8 * kQCtrStride * kQZifft, a.tw);
        SE1P_CHECK_LAUNCH();
        hipLaunchKernelGGL((bgather_kernel<T, P>), dim3(L[kQGather].grid),
                           dim3(64), L[kQGather].lds, s, a.sys, L[kQGather].items,
                           L[kQGather].qb, a.qctr + 8 * kQCtrStride * kQGather, a.blk, a.phiF,
                           a.EF);
        SE1P_CHECK_LAUNCH();
    }
    if ((flags & 2u) && L[kQReal].nitems > 0) {
        hipLaunchKernelGGL(brealspace_kernel<T>, dim3(L[kQReal].grid), dim3(64),
                           0, s, a.sys, L[kQReal].items, L[kQReal].qb, a.qctr + 8 * kQCtrStride * kQReal, a.blk, a.lex, a.phiR, a.ER);
        SE1P_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(bcombine_kernel<T>, dim3(L[kQComb].grid),
                       dim3(kCombineThreads), 0, s, a.sys, L[kQComb].items,
                       L[kQComb].qb, a.qctr + 8 * kQCtrStride * kQComb, q, a.phiF, a.EF,
                       a.phiR, a.ER, flags & (7u | SE1P_FORCE), phi, E, a.partials);
    SE1P_CHECK_LAUNCH();
    if (energy) {
        hipLaunchKernelGGL(benergy_kernel<T>, dim3(a.nsys), dim3(256), 0, s,
                           a.sys, a.nsys, a.partials, energy);
        SE1P_CHECK_LAUNCH();
    }
    return 0;
}

template <typename T>
int launch_batch(const BatchArgs<T>& a, const T* x, const T* q, T* phi, T* E,
                 double* energy, unsigned flags, hipStream_t s) {
    switch (a.P) {
#define SE1P_BATCH_CASE(PP) \
    case PP: return batch_p<T, PP>(a, x, q, phi, E, energy, flags, s);
        SE1P_P_CASES(SE1P_BATCH_CASE)
#undef SE1P_BATCH_CASE
        default: return -8;
    }
}

template <typename T, int P>
static int occ_p(int queue, size_t lds, int* bpc) {
    const void* f = nullptr;
    int bs = 256;
    switch (queue) {
        case kQSpread: f = (const void*)bspread_kernel<T, P>; bs = 64 * spread_waves(P); break;
        case kQZfft: f = (const void*)bzfft_kernel<T>; break;
        case kQRowFwd: f = (const void*)browfwd_kernel<T>; break;
        case kQCols: f = (const void*)bcols_kernel<T>; break;
        case kQRowInv: f = (const void*)browinv_kernel<T>; break;
        case kQZifft: f = (const void*)bzifft_kernel<T>; break;
        case kQGather: f = (const void*)bgather_kernel<T, P>; bs = 64; break;
        case kQReal: f = (const void*)brealspace_kernel<T>; bs = 64; break;
        case kQComb: f = (const void*)bcombine_kernel<T>; bs = kCombineThreads; break;
        default: return -1;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, f, bs, lds) != hipSuccess)
        return -5;
    return 0;
}

template <typename T>
int batch_occupancy(int queue, int P, size_t lds, int* blocks_per_cu) {
    switch (P) {
#define SE1P_OCC_CASE(PP) \
    case PP: return occ_p<T, PP>(queue, lds, blocks_per_cu);
        SE1P_P_CASES(SE1P_OCC_CASE)
#undef SE1P_OCC_CASE
        default: return -8;
    }
}

// explicit instantiations
#define SE1P_INST(T)                                                           \
    template int launch_bin<T>(const T*, const T*, long long, const Geo&,       \
                               const BinGeo&, const BinBufs&,                   \
                               DevParticles<T>&, DevParticles<T>&, hipStream_t); \
    template int launch_spread<T>(const DevParticles<T>&, long long,           \
                                  const Geo&, int, int, T*, T*, T*, T*,         \
                                  long long, hipStream_t);                      \
    template int launch_reduce_partials<T>(const T*, int, long long,           \
                                           long long, T, T*, hipStream_t);      \
    template int launch_kspace<T>(const T*, int, long long, T, const Geo&, int, \
                                  const SlabDesc*, const SlabDesc*,             \
                                  const FftDesc&, const cplx<T>*, const T*,     \
                                  cplx<T>*, cplx<T>*, T, T*, hipStream_t);      \
    template int launch_gather<T>(const T*, const DevParticles<T>&, long long, \
                                  const Geo&, const BinGeo&, T, T*, T*,         \
                                  hipStream_t);                                 \
    template int launch_realspace<T>(const DevParticles<T>&,                   \
                                     const DevParticles<T>&, long long,         \
                                     const Geo&, const BinGeo&, double, double, \
                                     int, bool, T*, T*, hipStream_t);           \
    template int launch_kspace_ik<T>(const T*, int, long long, const Geo&, int, \
                                     const SlabDesc*, const SlabDesc*,          \
                                     const FftDesc&, const cplx<T>*, const T*,  \
                                     cplx<T>*, cplx<T>*, cplx<T>*, long long,   \
                                     T*, T*, long long, hipStream_t);           \
    template int launch_gather_phi<T>(const T*, const DevParticles<T>&,         \
                                      const Geo&, const BinGeo&, T, T*, int,    \
                                      hipStream_t);                             \
    template int launch_fold<T>(const T*, int, long long, const Geo&,          \
                                const Geo&, T*, hipStream_t);                   \
    template int launch_unfold<T>(const T*, const Geo&, const Geo&, T*,        \
                                  hipStream_t);                                 \
    template int launch_combine<T>(long long, const T*, const T*, const T*,    \
                                   const T*, const T*, int, double, unsigned,   \
                                   T*, T*, double*, int, double*, hipStream_t); \
    template int launch_check<T>(const T*, const T*, long long, double, double, \
                                 int*, double*, hipStream_t);                   \
    template int launch_batch<T>(const BatchArgs<T>&, const T*, const T*, T*,  \
                                 T*, double*, unsigned, hipStream_t);           \
    template int batch_occupancy<T>(int, int, size_t, int*);

SE1P_INST(double)
SE1P_INST(float)

}  // namespace se1p
