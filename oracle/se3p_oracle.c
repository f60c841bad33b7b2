/*
 * se3p_oracle.c -- plain FP64 CPU oracle for the triply periodic Ewald sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * The paper compares SE1P with the triply periodic Spectral Ewald method
 * (SE3P, its reference Lindbo & Tornberg 2011) in the example on efficiency
 * compared to the triply periodic case.  The sum both SE3P and this oracle
 * evaluate is the classical Ewald decomposition of the potential of N point
 * charges in a box L1 x L2 x L3 periodic in all three directions (tin-foil
 * boundary, neutral system):
 *
 *   phi_m = phi^R_m + phi^F_m + phi^self_m
 *
 *   phi^R     sum over images p and sources n ((n, p) != (m, 0)) of
 *             q_n erfc(xi r) / r, r = |x_m - x_n + p L| <= rc
 *             (the same real-space kernel as eq. ewald1p_real)
 *   phi^F     (4 pi / V) sum_{k != 0} exp(-k^2 / 4 xi^2) / k^2
 *             sum_n q_n cos(k . (x_m - x_n)),  k = 2 pi (n1/L1, n2/L2, n3/L3)
 *   phi^self  -2 xi q_m / sqrt(pi)   (eq. ewald1p_self)
 *
 * and E_m = -grad_{x_m} phi_m:
 *
 *   E^R       sum q_n (erfc(xi r)/r + 2 xi/sqrt(pi) exp(-xi^2 r^2)) r_vec / r^2
 *   E^F       (4 pi / V) sum_{k != 0} k exp(-k^2/4xi^2) / k^2
 *             sum_n q_n sin(k . (x_m - x_n))
 *
 * The k sum is taken over the half space (n1 > 0, or n1 = 0 and n2 > 0, or
 * n1 = n2 = 0 and n3 > 0) with a factor 2, through the structure factor
 * S(k) = sum_n q_n exp(-i k . x_n): cos(k . (x_m - x_n)) summed over n is
 * Re(exp(i k . x_m) S(k)).  Modes with k^2 / 4 xi^2 > 46 are dropped
 * (exp(-46) < 1.1e-20).  Sums use Neumaier compensation; OpenMP runs over k
 * for the structure factors and over targets for the potentials, each sum in
 * a fixed order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define PI3_D 3.14159265358979323846264338327950288419716939937510
#define A3_MAX 46.0

typedef struct { double s, c; } ksum3;
static inline void kadd3(ksum3* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double kval3(const ksum3* a) { return a->s + a->c; }

/* per-target output record: phi^R, phi^F, phi^self, E^R[3], E^F[3] */
enum { T_PHI_R = 0, T_PHI_F = 1, T_PHI_SELF = 2, T_ER = 3, T_EF = 6, T_NREC = 9 };

int se3p_oracle_ewald(long N, const double* x, const double* q,
                      const double* box, double xi, double rc,
                      long ntarget, const long* targets, double* out) {
    if (N <= 0 || !x || !q || !box || !out || xi <= 0.0) return -1;
    const double L[3] = {box[0], box[1], box[2]};
    if (!(L[0] > 0.0 && L[1] > 0.0 && L[2] > 0.0)) return -1;
    const double V = L[0] * L[1] * L[2];
    const double xi2 = xi * xi;
    const double c_erf = 2.0 * xi / sqrt(PI3_D);

    /* half-space k modes with k^2 / 4 xi^2 <= A3_MAX */
    const double kmax = 2.0 * xi * sqrt(A3_MAX);
    int nmax[3];
    for (int d = 0; d < 3; ++d) nmax[d] = (int)floor(kmax * L[d] / (2.0 * PI3_D));
    long nk = 0;
    for (int a = 0; a <= nmax[0]; ++a)
        for (int b = -nmax[1]; b <= nmax[1]; ++b)
            for (int c = -nmax[2]; c <= nmax[2]; ++c) {
                if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                const double k1 = 2.0 * PI3_D * a / L[0], k2 = 2.0 * PI3_D * b / L[1],
                             k3 = 2.0 * PI3_D * c / L[2];
                if ((k1 * k1 + k2 * k2 + k3 * k3) / (4.0 * xi2) <= A3_MAX) ++nk;
            }
    double* kv = (double*)malloc(sizeof(double) * 4 * (size_t)(nk > 0 ? nk : 1));
    double* sre = (double*)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
    double* sim = (double*)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
    if (!kv || !sre || !sim) { free(kv); free(sre); free(sim); return -3; }
    long ik = 0;
    for (int a = 0; a <= nmax[0]; ++a)
        for (int b = -nmax[1]; b <= nmax[1]; ++b)
            for (int c = -nmax[2]; c <= nmax[2]; ++c) {
                if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                const double k1 = 2.0 * PI3_D * a / L[0], k2 = 2.0 * PI3_D * b / L[1],
                             k3 = 2.0 * PI3_D * c / L[2];
                const double k2s = k1 * k1 + k2 * k2 + k3 * k3;
                if (k2s / (4.0 * xi2) > A3_MAX) continue;
                kv[4 * ik] = k1; kv[4 * ik + 1] = k2; kv[4 * ik + 2] = k3;
                /* factor 2 for the mode -k */
                kv[4 * ik + 3] = 2.0 * (4.0 * PI3_D / V) * exp(-k2s / (4.0 * xi2)) / k2s;
                ++ik;
            }

    /* structure factors S(k) = sum_n q_n exp(-i k . x_n) */
    long j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < nk; ++j) {
        ksum3 re = {0, 0}, im = {0, 0};
        for (long n = 0; n < N; ++n) {
            const double ph = kv[4 * j] * x[3 * n] + kv[4 * j + 1] * x[3 * n + 1] +
                              kv[4 * j + 2] * x[3 * n + 2];
            kadd3(&re, q[n] * cos(ph));
            kadd3(&im, -q[n] * sin(ph));
        }
        sre[j] = kval3(&re);
        sim[j] = kval3(&im);
    }

    /* real-space images: |p_d| <= ceil(rc / L_d) + 1 */
    int pim[3];
    for (int d = 0; d < 3; ++d) pim[d] = (int)ceil(rc / L[d]) + 1;

    long i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < ntarget; ++i) {
        const long m = targets ? targets[i] : i;
        const double xm = x[3 * m], ym = x[3 * m + 1], zm = x[3 * m + 2];
        ksum3 pr = {0, 0}, pf = {0, 0};
        ksum3 er[3] = {{0, 0}, {0, 0}, {0, 0}}, ef[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (long n = 0; n < N; ++n) {
            for (int a = -pim[0]; a <= pim[0]; ++a)
                for (int b = -pim[1]; b <= pim[1]; ++b)
                    for (int c = -pim[2]; c <= pim[2]; ++c) {
                        if (n == m && a == 0 && b == 0 && c == 0) continue;
                        const double dx = xm - x[3 * n] + a * L[0];
                        const double dy = ym - x[3 * n + 1] + b * L[1];
                        const double dz = zm - x[3 * n + 2] + c * L[2];
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 > rc * rc) continue;
                        const double r = sqrt(r2);
                        const double ec = erfc(xi * r);
                        kadd3(&pr, q[n] * ec / r);
                        const double f = q[n] * (ec / r + c_erf * exp(-xi2 * r2)) / r2;
                        kadd3(&er[0], f * dx);
                        kadd3(&er[1], f * dy);
                        kadd3(&er[2], f * dz);
                    }
        }
        for (long t = 0; t < nk; ++t) {
            const double ph = kv[4 * t] * xm + kv[4 * t + 1] * ym + kv[4 * t + 2] * zm;
            const double cs = cos(ph), sn = sin(ph);
            /* Re(e^{i ph} S) and Im(e^{i ph} S) */
            const double re = cs * sre[t] - sn * sim[t];
            const double im = sn * sre[t] + cs * sim[t];
            kadd3(&pf, kv[4 * t + 3] * re);
            /* E = -grad_m: d/dx_m Re(e^{i k.x_m} S) = -k Im(...) */
            for (int d = 0; d < 3; ++d) kadd3(&ef[d], kv[4 * t + 3] * kv[4 * t + d] * im);
        }
        double* o = out + (size_t)i * T_NREC;
        o[T_PHI_R] = kval3(&pr);
        o[T_PHI_F] = kval3(&pf);
        o[T_PHI_SELF] = -c_erf * q[m];
        for (int d = 0; d < 3; ++d) {
            o[T_ER + d] = kval3(&er[d]);
            o[T_EF + d] = kval3(&ef[d]);
        }
    }
    free(kv);
    free(sre);
    free(sim);
    return 0;
}
