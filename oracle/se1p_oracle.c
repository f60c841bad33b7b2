/*
 * se1p_oracle.c -- plain FP64 CPU oracle for the singly periodic Ewald sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * What it computes (Saffar Shamshirgar & Tornberg, "The Spectral Ewald
 * method for singly periodic domains", section 2.1): for a neutral system of
 * N point charges in a box periodic along z only, the potential at a target
 * particle m is split as
 *
 *   phi_m = phi^R_m + phi^{F,k3!=0}_m + phi^{F,k3=0}_m + phi^self_m
 *
 *   phi^R      real-space sum of q_n erfc(xi r)/r over z-images, r <= rc
 *              (eq. ewald1p_real)
 *   phi^{Fk}   (1/L3) sum_{k3!=0} sum_n q_n exp(i k3 z_mn) K0(k3^2/4xi^2,
 *              xi^2 rho_mn^2) with the incomplete Bessel function K0(a,b)
 *              (eq. ewald1p_fourier_complete); evaluated here as
 *              (2/L3) sum_{j>=1} cos(k_j z_mn) K0(...) using k3 <-> -k3.
 *   phi^{F0}   -(1/L3) sum_{n!=m} q_n {gamma + log(u) + E1(u)},
 *              u = xi^2 rho_mn^2 (eq. ewald1p_zero)
 *   phi^self   -2 xi q_m / sqrt(pi)  (eq. ewald1p_self)
 *
 * and the field E_m = -grad_{x_m} phi_m (the force is F_m = q_m E_m):
 *
 *   E^R        sum' q_n (erfc(xi r)/r + 2 xi/sqrt(pi) exp(-xi^2 r^2)) r_vec/r^2
 *              (eq. force_real with the factor q_m removed)
 *   E^{Fk}_z   (2/L3) sum_j sum_n q_n k_j sin(k_j z_mn) K0(a_j, b_mn)
 *   E^{Fk}_r   (4 xi^2/L3) sum_j sum_n q_n cos(k_j z_mn) (r_m - r_n) K0m1(a_j, b_mn)
 *              where K0m1(a,b) = int_1^inf t^-2 exp(-a t - b/t) dt = -dK0/db
 *              (derivative of eq. ewald1p_fourier_complete)
 *   E^{F0}     (2/L3) sum_{n!=m} q_n (r_m - r_n)/rho^2 (1 - exp(-xi^2 rho^2))
 *              (derivative of eq. ewald1p_zero; eq. force_zero carries an extra
 *              factor 1/2 from the paper's energy convention, see the energy
 *              reading in the design notes: U = 1/2 sum q phi, F = q E).
 *
 * Special functions follow appendix A: E1 by its power series for x < 1 and
 * by its continued fraction for x >= 1; gamma + log x + E1(x) by the
 * alternating series for small x (its limit at 0 is 0); K0(a,b) by composite
 * Gauss-Legendre quadrature (here of the integral after the substitution
 * t = exp(u), which is smooth and decays double-exponentially).
 *
 * All sums use Neumaier compensated summation.  OpenMP parallelises over the
 * targets only; each target's sums run in source order, so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EULER_GAMMA 0.57721566490153286060651209008240243104215933593992
#define PI_D 3.14159265358979323846264338327950288419716939937510

/* ------------------------------------------------------------------------ */
/* Neumaier compensated accumulator                                          */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;
static inline void kadd(ksum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double kval(const ksum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Exponential integral E1 (appendix A, eqs. expint_n_fraction and           */
/* expint_1_series_rep)                                                       */
/* ------------------------------------------------------------------------ */
double se1p_oracle_E1(double x) {
    if (!(x > 0.0)) return INFINITY;
    if (x < 1.0) {
        /* E1(x) = -gamma - log x - sum_{m>=1} (-x)^m / (m m!) */
        double term = 1.0, sum = 0.0;
        for (int m = 1; m < 60; ++m) {
            term *= -x / m;              /* (-x)^m / m! */
            double t = term / m;
            sum += t;
            if (fabs(t) < 1e-18 * fabs(sum)) break;
        }
        return -EULER_GAMMA - log(x) - sum;
    }
    /* continued fraction, modified Lentz:
       E1(x) = e^-x / (x+1 - 1^2/(x+3 - 2^2/(x+5 - ...))) */
    const double tiny = 1e-300;
    double b = x + 1.0;
    double c = 1.0 / tiny;
    double d = 1.0 / b;
    double h = d;
    for (int i = 1; i < 10000; ++i) {
        double an = -(double)i * (double)i;
        b += 2.0;
        d = 1.0 / (an * d + b);
        c = b + an / c;
        double del = c * d;
        h *= del;
        if (fabs(del - 1.0) < 1e-17) break;
    }
    return h * exp(-x);
}

/* Ein(x) = gamma + log x + E1(x) = sum_{m>=1} (-1)^{m+1} x^m / (m m!),
   Ein(0) = 0 (eq. limit). */
double se1p_oracle_Ein(double x) {
    if (x <= 0.0) return 0.0;
    if (x < 2.0) {
        double term = 1.0, sum = 0.0;
        for (int m = 1; m < 80; ++m) {
            term *= x / m;               /* x^m / m! */
            double t = (m & 1 ? term : -term) / m;
            sum += t;
            if (fabs(t) < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return EULER_GAMMA + log(x) + se1p_oracle_E1(x);
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1,1] (Newton iteration on P_n)                  */
/* ------------------------------------------------------------------------ */
#define GL_N 16
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;

static void gl_init(void) {
    const int n = GL_N;
    for (int i = 0; i < n; ++i) {
        double z = cos(PI_D * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
    gl_ready = 1;
}

void se1p_oracle_init(void) { if (!gl_ready) gl_init(); }

/* ------------------------------------------------------------------------ */
/* Incomplete Bessel function K0(a,b) = int_1^inf t^-1 exp(-a t - b/t) dt    */
/* (definition after eq. ewald1p_self) and K0m1(a,b) with t^-2.              */
/* With t = e^u:  K0   = int_0^inf exp(-a e^u - b e^-u) du                   */
/*                K0m1 = int_0^inf exp(-a e^u - b e^-u - u) du               */
/* ------------------------------------------------------------------------ */
static double k0_quad(double a, double b, int extra_u) {
    if (!gl_ready) gl_init();
    /* minimum of g(u) = a e^u + b e^-u over u >= 0 */
    double us = 0.0;
    if (b > a) us = 0.5 * log(b / a);
    double gs = a * exp(us) + b * exp(-us);
    /* beyond U the integrand is below exp(-(gs + 60)) */
    double U = log((gs + 60.0) / a);
    if (U < us + 1.0) U = us + 1.0;
    /* panel width resolves the peak (curvature ~ g'') and the tail */
    double curv = a * exp(us) + b * exp(-us);
    double width = 0.5;
    if (curv > 1.0) {
        double sw = 1.5 / sqrt(curv);
        if (sw < width) width = sw;
    }
    int np = (int)ceil(U / width);
    if (np < 4) np = 4;
    if (np > 200000) np = 200000;
    double hw = U / np;
    ksum acc = {0.0, 0.0};
    for (int p = 0; p < np; ++p) {
        double mid = (p + 0.5) * hw;
        double half = 0.5 * hw;
        for (int i = 0; i < GL_N; ++i) {
            double u = mid + half * gl_x[i];
            double g = a * exp(u) + b * exp(-u) + (extra_u ? u : 0.0);
            kadd(&acc, half * gl_w[i] * exp(-g));
        }
    }
    return kval(&acc);
}

double se1p_oracle_K0inc(double a, double b) { return k0_quad(a, b, 0); }
double se1p_oracle_K0inc_m1(double a, double b) { return k0_quad(a, b, 1); }

/* ------------------------------------------------------------------------ */
/* Ewald1P components at a set of targets                                   */
/* ------------------------------------------------------------------------ */
enum {
    OR_REAL = 1u, OR_FK = 2u, OR_F0 = 4u, OR_SELF = 8u, OR_FIELD = 16u
};
/* per-target output record (13 doubles) */
enum {
    O_PHI_R = 0, O_PHI_FK = 1, O_PHI_F0 = 2, O_PHI_SELF = 3,
    O_ER = 4, O_EFK = 7, O_EF0 = 10, O_NREC = 13
};

/* Largest a = (k/2xi)^2 kept in the k3 != 0 sum: K0(a,b) <= E1(a) and
   E1(46) < 3e-22, far below FP64 resolution of any potential here. */
#define OR_A_MAX 46.0

int se1p_oracle_ewald(long N, const double* x, const double* q,
                      const double* box, double xi, double rc,
                      long ntarget, const long* targets, unsigned parts,
                      double* out) {
    if (N <= 0 || !x || !q || !box || !out || xi <= 0.0) return -1;
    if (!gl_ready) gl_init();
    const double L3 = box[2];
    const double xi2 = xi * xi;
    const double c_erf = 2.0 * xi / sqrt(PI_D);
    /* z-images needed by the real-space cut-off */
    const int jimg = (int)ceil(rc / L3) + 1;
    /* k3 != 0 modes: k_j = 2 pi j / L3, a_j = k_j^2 / (4 xi^2) */
    int jmax = 0;
    while (1) {
        double k = 2.0 * PI_D * (jmax + 1) / L3;
        if (k * k / (4.0 * xi2) > OR_A_MAX) break;
        ++jmax;
        if (jmax > 100000) return -2;
    }
    const int field = (parts & OR_FIELD) != 0;

    long i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < ntarget; ++i) {
        long m = targets ? targets[i] : i;
        const double xm = x[3 * m], ym = x[3 * m + 1], zm = x[3 * m + 2];
        ksum pr = {0, 0}, pk = {0, 0}, p0 = {0, 0};
        ksum er[3] = {{0, 0}, {0, 0}, {0, 0}};
        ksum ek[3] = {{0, 0}, {0, 0}, {0, 0}};
        ksum e0[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (long n = 0; n < N; ++n) {
            const double qn = q[n];
            const double dx = xm - x[3 * n], dy = ym - x[3 * n + 1];
            const double dz = zm - x[3 * n + 2];
            const double rho2 = dx * dx + dy * dy;
            if (parts & OR_REAL) {
                for (int j = -jimg; j <= jimg; ++j) {
                    if (n == m && j == 0) continue;
                    double zz = dz + j * L3;
                    double r2 = rho2 + zz * zz;
                    if (r2 > rc * rc) continue;
                    double r = sqrt(r2);
                    double ec = erfc(xi * r);
                    kadd(&pr, qn * ec / r);
                    if (field) {
                        double f = qn * (ec / r + c_erf * exp(-xi2 * r2)) / r2;
                        kadd(&er[0], f * dx);
                        kadd(&er[1], f * dy);
                        kadd(&er[2], f * zz);
                    }
                }
            }
            if (parts & OR_FK) {
                const double b = xi2 * rho2;
                for (int j = 1; j <= jmax; ++j) {
                    double k = 2.0 * PI_D * j / L3;
                    double a = k * k / (4.0 * xi2);
                    double K = se1p_oracle_K0inc(a, b);
                    double cs = cos(k * dz);
                    kadd(&pk, (2.0 / L3) * qn * cs * K);
                    if (field && n != m) {
                        double sn = sin(k * dz);
                        double Km = se1p_oracle_K0inc_m1(a, b);
                        double fr = (4.0 * xi2 / L3) * qn * cs * Km;
                        kadd(&ek[0], fr * dx);
                        kadd(&ek[1], fr * dy);
                        kadd(&ek[2], (2.0 / L3) * qn * k * sn * K);
                    }
                }
            }
            if ((parts & OR_F0) && n != m) {
                const double u = xi2 * rho2;
                kadd(&p0, -(1.0 / L3) * qn * se1p_oracle_Ein(u));
                if (field) {
                    /* (1 - e^-u)/rho^2 = xi^2 (1 - e^-u)/u, limit xi^2 */
                    double g = (u > 0.0) ? -expm1(-u) / u : 1.0;
                    double f = (2.0 * xi2 / L3) * qn * g;
                    kadd(&e0[0], f * dx);
                    kadd(&e0[1], f * dy);
                }
            }
        }
        double* o = out + (size_t)i * O_NREC;
        o[O_PHI_R] = kval(&pr);
        o[O_PHI_FK] = kval(&pk);
        o[O_PHI_F0] = kval(&p0);
        o[O_PHI_SELF] = (parts & OR_SELF) ? -c_erf * q[m] : 0.0;
        for (int d = 0; d < 3; ++d) {
            o[O_ER + d] = kval(&er[d]);
            o[O_EFK + d] = kval(&ek[d]);
            o[O_EF0 + d] = kval(&e0[d]);
        }
    }
    return 0;
}

/* Number of k3 != 0 modes the oracle keeps for a given xi and period. */
int se1p_oracle_kmodes(double xi, double L3) {
    int jmax = 0;
    while (1) {
        double k = 2.0 * PI_D * (jmax + 1) / L3;
        if (k * k / (4.0 * xi * xi) > OR_A_MAX) break;
        ++jmax;
        if (jmax > 100000) return -1;
    }
    return jmax;
}

int se1p_oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Brute-force image sum (eq. coulomb with the set P1) for tiny neutral      */
/* systems: symmetric partial sums over |j| <= J of                          */
/* sum'_n q_n / |x_m - x_n + j L3 e_z|.  Used only to pin the Ewald form.    */
/* ------------------------------------------------------------------------ */
int se1p_oracle_image_sum(long N, const double* x, const double* q,
                          double L3, long J, double* phi) {
    if (N <= 0 || J < 0) return -1;
    for (long m = 0; m < N; ++m) {
        ksum s = {0, 0};
        for (long j = -J; j <= J; ++j) {
            for (long n = 0; n < N; ++n) {
                if (n == m && j == 0) continue;
                double dx = x[3 * m] - x[3 * n];
                double dy = x[3 * m + 1] - x[3 * n + 1];
                double dz = x[3 * m + 2] - x[3 * n + 2] + j * L3;
                kadd(&s, q[n] / sqrt(dx * dx + dy * dy + dz * dz));
            }
        }
        phi[m] = kval(&s);
    }
    return 0;
}
