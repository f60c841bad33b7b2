/*
 * se1p.h -- C ABI of the MI355X (gfx950) Spectral Ewald library for singly
 * periodic Coulomb systems (SE1P; Saffar Shamshirgar & Tornberg,
 * "The Spectral Ewald method for singly periodic domains").
 *
 * Problem (section 1, eq. coulomb with the lattice P_1 of section 2.1):
 * N point charges q_n at x_n in a box [0,L1) x [0,L2) x [0,L3), periodic along
 * z (index 2) with period L3 and free along x and y, with sum_n q_n = 0.  For
 * every particle the library returns the potential
 *
 *     phi_m = phi^R_m + phi^F_m + phi^self_m           (eq. full_potential)
 *
 * and the field E_m = -grad_{x_m} phi_m, so that the force is F_m = q_m E_m
 * and the energy U = 1/2 sum_m q_m phi_m (section 3.5 read with the usual 1/2;
 * the paper's printed energy omits it while its force formula keeps it).
 *
 *   phi^F   Fourier-space part by the SE1P method (Algorithm 1): Gaussian
 *           gridding, the adaptive FFT of Algorithm 2 (k3 = 0 slab on an
 *           s0-upsampled grid with the truncated Green's function of
 *           eq. G_kappa_k, slabs 0 < |k3| <= 2 pi n_l / L3 upsampled by s_l,
 *           the rest not upsampled), scaling (eq. scale_1p), the inverse of
 *           Algorithm 3, and gathering (eq. se1p_complete_discretized) with
 *           its analytic gradient for E (eq. force_se1p).
 *   phi^R   real-space erfc sum over z-images within the cut-off rc
 *           (eq. ewald1p_real; field eq. force_real).
 *   phi^self  -2 xi q_m / sqrt(pi) (eq. ewald1p_self).
 *
 * Conventions for every entry point:
 *   - Return value: 0 on success, a negative SE1P_ERR_* code otherwise;
 *     se1p_error_string() turns it into text.  Argument checks run on the host
 *     before anything is enqueued; nothing is enqueued when a check fails.
 *   - Device pointers are HIP device memory on the plan's device.  The caller
 *     owns every particle and output buffer; the plan owns its workspace.
 *     No entry point allocates memory except se1p_plan_create (and
 *     se1p_batch_create); se1p_plan_destroy frees it.
 *   - Work is enqueued on the plan's stream (hipStream_t passed as void*,
 *     NULL = the default stream) without synchronising, except where a
 *     function says otherwise.
 *   - Floating-point buffers are double for SE1P_FP64 plans and float for
 *     SE1P_FP32 plans; the energy is always double.
 *   - Positions are row-major N x 3 (x, y, z).  x and y must lie in [0, L1)
 *     and [0, L2); z may be any finite value and is wrapped into [0, L3).
 */
#ifndef SE1P_H
#define SE1P_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define SE1P_OK               0
#define SE1P_ERR_ARG         -1  /* NULL pointer, bad size, unknown flag */
#define SE1P_ERR_PARAM       -2  /* inconsistent method parameters */
#define SE1P_ERR_NONNEUTRAL  -3  /* |sum q| > tol sum |q|, tol = 1e-10 (FP64) or
                                    3.8e-6 (FP32) (section 2.1 needs neutrality) */
#define SE1P_ERR_OUT_OF_BOX  -4  /* x or y outside [0,L1) x [0,L2), or non-finite */
#define SE1P_ERR_HIP         -5  /* a HIP runtime call failed */
#define SE1P_ERR_NOMEM       -6  /* device allocation failed */
#define SE1P_ERR_TOO_MANY    -7  /* N larger than the plan's n_max */
#define SE1P_ERR_UNSUPPORTED -8  /* valid request outside what this library supports */
#define SE1P_ERR_SCRATCH     -9  /* the call needs more scratch than the static
                                    buffer of se1p_eval_noalloc holds */

/* ---- precision ---------------------------------------------------------- */
#define SE1P_FP64 0
#define SE1P_FP32 1

/* ---- components for se1p_eval (bit mask) -------------------------------- */
#define SE1P_KSPACE        1u  /* phi^F, E^F (Algorithm 1) */
#define SE1P_REAL          2u  /* phi^R, E^R (eq. ewald1p_real, eq. force_real) */
#define SE1P_SELF          4u  /* phi^self (eq. ewald1p_self) */
#define SE1P_ALL           7u
#define SE1P_CHECK_INPUT  16u  /* validate positions and neutrality on the device;
                                  synchronises the plan's stream */
#define SE1P_NO_NEUTRAL   32u  /* evaluate the SE1P operator for any charge
                                  vector (used for adjoint products); the
                                  result is the discrete operator applied to
                                  q, not a physical Ewald sum */
#define SE1P_FIELD_IK    128u  /* E^F by ik-differentiation, the route of
                                  eq. force_fourier the paper sets aside for
                                  the analytic gradient (eq. force_se1p):
                                  -i k times the scaled spectrum, three more
                                  inverse transforms and potential-only
                                  gathers; SE1P plans only */
#define SE1P_FORCE       256u  /* efield receives the force q_m E_m on every
                                  particle (the field of eq. force_se1p and
                                  eq. force_real times the particle's charge)
                                  instead of E_m; the totals kernel forms
                                  the product */

/*
 * Method parameters (Algorithm 1 input, section 4.3 recipe).
 *   box      L1, L2, L3; z (index 2) is periodic.
 *   xi       Ewald splitting parameter (> 0).
 *   M3       grid points along z (even, >= P); h = L3 / M3.  The free
 *            directions use the same h over ceil(L_d / h) cells, extended by
 *            P points for the Gaussian support (L~ = L + P h, section 3.1).
 *   P        points in the support of the truncated Gaussians per direction
 *            (even, 4..32).  eta = P xi^2 h^2 / (c^2 pi), c = 0.95
 *            (eq. comp_eta).
 *   n_l      local pad size: modes 0 < |n3| <= n_l are upsampled by s_l
 *            (eq. I, eq. upsamplings).
 *   s_l      upsampling factor of the local pad set (>= 1).
 *   s0       upsampling factor of the k3 = 0 slab.  The padded period must
 *            be at least the support extent plus R = |(L~1, L~2)|
 *            (section 3.2, R = sqrt(2) L~ for a square cross-section), i.e.
 *            s0 >= 1 + sqrt(2) for a square cross-section; smaller values are
 *            raised to that minimum.
 *   rc       real-space cut-off (> 0 when SE1P_REAL is requested).
 *   pad_free extra grid points appended in each free direction beyond
 *            M + P (>= 0).  The paper's extension is pad_free = 0; a few
 *            extra zero points push the periodic images of the slabs that
 *            are not upsampled further away at almost no cost.
 *   precision SE1P_FP64 or SE1P_FP32.
 * Padded FFT lengths are rounded up to products of 2, 3 and 5.
 */
typedef struct se1p_params {
    double box[3];
    double xi;
    int    M3;
    int    P;
    int    n_l;
    double s_l;
    double s0;
    double rc;
    int    pad_free;
    int    precision;
} se1p_params;

/* Derived quantities of a plan (read-only). */
typedef struct se1p_plan_info {
    double h;            /* grid spacing L3 / M3 */
    double eta;          /* Gaussian width parameter, eq. comp_eta */
    double R;            /* truncation radius of the k3 = 0 Green's function */
    int    M[2];         /* cells across the charge box in x, y */
    int    Mt[2];        /* extended grid in x, y (>= M + P, FFT-friendly) */
    int    M3;
    int    P;
    int    n0[2];        /* padded 2D FFT size of the k3 = 0 slab */
    int    nl[2];        /* padded 2D FFT size of the slabs 0 < |n3| <= n_l */
    int    n_l;
    int    nslab;        /* slabs transformed: n3 = 0 .. M3/2 (Hermitian half) */
    int    precision;
    long long n_max;
    size_t workspace_bytes;
    int    gather_block[3];  /* cells per gather block (x, y, z) */
    int    gather_chunks;    /* waves (one chunk each) per gather unit */
    int    spread_cz;        /* z cells per gridding chunk */
    int    spread_kp;        /* partial grids written by gridding */
    long long bin_cells[2];  /* cells of the lex and block orders of binning */
    int    gather_pair;      /* 1: a gather unit is two y-adjacent blocks (32
                                particles of each per chunk), 0: one block
                                (64 particles per chunk) */
} se1p_plan_info;

typedef struct se1p_plan se1p_plan;

/*
 * se1p_suggest_params -- host only.  Parameter selection of section 4.3:
 * given a target RMS error tol, the box, N and Q = sum q^2, pick
 *   - M3 = 2 k_inf from the Fourier truncation estimate (eq. kinf),
 *     rounded up to an even size with prime factors 2, 3 and 5 only, when
 *     M3_in <= 0, else use M3_in and pick the largest xi that meets the same
 *     estimate (xi_in <= 0), or the given xi_in;
 *   - rc from the real-space estimate (eq. rc);
 *   - P from eq. approximation_error_oneterm when P_in <= 0 (rounded up to
 *     even), else P_in;
 *   - s_l from eq. choose_sl generalised to any box: the padded period
 *     leaves (s_l - 1) L~ between the support and its nearest image, and
 *     exp(-2 pi (s_l - 1) L~ / L3) < tol, with L~ the smaller extended side;
 *     n_l from eq. choose_nl (M3 ~ 10 n_l)
 *     when n_l_in < 0, else n_l_in;
 *   - s0 = 1 + sqrt(2) (minimum of section 3.4).
 * precision: SE1P_FP64 or SE1P_FP32.  Writes *out; returns an error code.
 */
int se1p_suggest_params(double tol, const double box[3], long long N,
                        double Q, double xi_in, int M3_in, int P_in,
                        int n_l_in, int precision, se1p_params* out);

/*
 * se1p_plan_create -- validates *params, derives the grid geometry, builds
 * the k3 = 0 scaling table (eq. G_kappa_k, FP64 on the host), the FFT
 * tables, and allocates the device workspace for up to n_max particles on
 * the current HIP device.  stream: hipStream_t (NULL = default stream).
 * On success *out owns everything; free it with se1p_plan_destroy.
 * The transforms take sizes with prime factors 2, 3 and 5 only: an M3 with
 * another factor returns SE1P_ERR_UNSUPPORTED (the padded x and y sizes are
 * rounded up to such sizes), as does an upsampled transform longer than
 * 4096 or a grid whose transforms or gather planes would not fit one
 * workgroup's LDS.
 */
int se1p_plan_create(const se1p_params* params, long long n_max,
                     void* stream, se1p_plan** out);

/*
 * se3p_plan_create -- the triply periodic counterpart (SE3P) the paper
 * compares SE1P with in its example on efficiency against the triply
 * periodic case: the same gridding, gather and real-space kernels, with the
 * box periodic in x and y as well.  The gridded values are folded onto the
 * periodic M1 x M2 x M3 grid, transformed without zero padding or
 * upsampling, scaled by exp(-(1 - eta) k^2 / 4 xi^2) / k^2 for every k != 0
 * (the k3 = 0 plane too, k = 0 dropped: tin-foil boundary), and the
 * real-space sum takes sources from every periodic image within rc.
 * Parameters as for se1p_plan_create; n_l, s_l and s0 are ignored; box[0]
 * and box[1] must be multiples of h = box[2] / M3 (else SE1P_ERR_PARAM).
 * The plan works with se1p_eval, se1p_plan_get_info, timing and
 * se1p_plan_destroy; the stage calls se1p_spread, se1p_kspace_solve and
 * se1p_gather return SE1P_ERR_UNSUPPORTED for it.
 */
int se3p_plan_create(const se1p_params* params, long long n_max,
                     void* stream, se1p_plan** out);

/* Releases the plan and its device workspace (synchronises its stream). */
int se1p_plan_destroy(se1p_plan* plan);

/* Copies the derived geometry of the plan into *info. */
int se1p_plan_get_info(const se1p_plan* plan, se1p_plan_info* info);

/* Changes the stream later calls enqueue on. */
int se1p_set_stream(se1p_plan* plan, void* stream);

/*
 * se1p_eval -- one evaluation.
 *   N          number of particles (1 .. n_max).
 *   x          device, N x 3 positions (row-major), FP64/FP32 per plan.
 *   q          device, N charges.  Must sum to zero (within 1e-10 sum |q|
 *              for FP64 plans, 32 FP32 epsilons = 3.8e-6 sum |q| for FP32
 *              plans, the rounding of FP32 charges that are neutral in exact
 *              arithmetic) unless SE1P_NO_NEUTRAL; only checked with
 *              SE1P_CHECK_INPUT.
 *   phi        device, N potentials out, or NULL.
 *   efield     device, N x 3 fields out (E = -grad phi), or NULL.
 *   energy     device, one double out: U = 1/2 sum q phi over the requested
 *              components, or NULL.
 *   flags      SE1P_KSPACE | SE1P_REAL | SE1P_SELF, optionally with
 *              SE1P_CHECK_INPUT, SE1P_NO_NEUTRAL and SE1P_FIELD_IK
 *              (SE1P_ERR_UNSUPPORTED on an SE3P plan).
 * Components left out contribute zero.  Without SE1P_CHECK_INPUT,
 * out-of-box x/y are clamped to the box edge cells (memory-safe, result
 * unspecified).
 */
int se1p_eval(se1p_plan* plan, long long N, const void* x, const void* q,
              void* phi, void* efield, double* energy, unsigned flags);

/*
 * se1p_eval_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the evaluation of se1p_eval, same arguments, flags and
 * results, with every per-call scratch buffer (binning arrays, weights,
 * partial grids, spectra, per-particle partial results, energy partials)
 * placed in one static device array of SE1P_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends, instead of
 * the plan's own scratch.  It allocates nothing and leaves the plan's own
 * scratch untouched; the plan supplies geometry and tables only, so N is
 * not limited by the plan's n_max (which sized the plan's scratch and
 * tuned its tiles) but by the static array: SE1P_ERR_SCRATCH when the
 * call's scratch (a function of the grid and N; the ik buffers count only
 * with SE1P_FIELD_IK) exceeds it, checked on the host before anything is
 * enqueued.  The N = 1e5 FP64 system with P = 24 and a 64 x 96 x 96 grid
 * needs about 190 MB.
 * All calls on one GPU share its array and leave their contents in it;
 * every buffer a call reads is written or cleared earlier in the same call.
 * Calls that overlap on one GPU (other host threads, other streams) race
 * on the array and must be serialised by the caller.  The array's address
 * on a device is looked up on the first call on that device.
 */
#define SE1P_NOALLOC_SCRATCH_BYTES (256ull << 20)
int se1p_eval_noalloc(se1p_plan* plan, long long N, const void* x, const void* q,
                      void* phi, void* efield, double* energy, unsigned flags);

/*
 * Stages of the k-space path, for testing and for callers that bring their
 * own real-space part.  All enqueue on the plan's stream.
 *
 * se1p_spread -- step 2 of Algorithm 1 (eq. spread_1p): H on the grid.
 *   grid: device, M3 x Mt1 x Mt2 values (z slowest, y fastest); grid point
 *   (l, i, j) sits at (x, y, z) = ((i - P/2) h, (j - P/2) h, l h).
 *   Values include the Gaussian normalisation (2 xi^2 / (pi eta))^{3/2}.
 */
int se1p_spread(se1p_plan* plan, long long N, const void* x, const void* q,
                void* grid);

/*
 * se1p_bin -- the binning stage alone: the counting sort of the particles by
 * grid cell that the cell lists of the real-space sum (section 2.2, sums
 * over neighbouring cells within rc) and the gridding and gathering tiles
 * run on.  A particle's cell is (floor(x/h), floor(y/h), floor(z'/h)) with
 * z' = z wrapped into [0, L3), each index clamped to the grid.
 *   lex order    cells numbered (cz, cx, cy), cy fastest;
 *   block order  cells grouped in blocks of gather_block[0..2] cells (x, y,
 *                z; se1p_plan_get_info), blocks numbered along a
 *                serpentine path (z slowest, then x reversed on odd z
 *                layers, then y reversed on odd rows), cells z-major inside
 *                a block (z reversed in odd blocks, then x, then y).
 * Inside a cell particles keep increasing input index, so both orders are
 * fully determined by x.  Writes (device, each may be NULL):
 *   lex_perm, blk_perm    N ints: sorted position -> input index;
 *   lex_start, blk_start  bin_cells[0] + 1 and bin_cells[1] + 1 ints: first
 *                         sorted position of each cell, then N.
 * q is read as se1p_eval reads it (its sorted copies are made as well).
 */
int se1p_bin(se1p_plan* plan, long long N, const void* x, const void* q,
             int* lex_perm, int* lex_start, int* blk_perm, int* blk_start);

/*
 * se1p_kspace_solve -- steps 3-5 of Algorithm 1 on a grid from se1p_spread:
 * AFT (Algorithm 2), scaling (eq. scale_1p, with the (kappa, k3) = (0, 0)
 * coefficient set to zero), AIFT (Algorithm 3).  grid_in and grid_out have
 * the layout above (they may alias).  The output is normalised so that
 * phi^F_m = 4 pi h^3 sum_grid Htilde g(x_m - x_grid), with g the normalised
 * truncated Gaussian of eq. spread_1p.
 */
int se1p_kspace_solve(se1p_plan* plan, const void* grid_in, void* grid_out);

/*
 * se1p_gather -- step 6 of Algorithm 1 and its analytic gradient: phi^F and
 * E^F at the particles from a grid produced by se1p_kspace_solve.
 * phi, efield as in se1p_eval (either may be NULL).
 */
int se1p_gather(se1p_plan* plan, long long N, const void* x,
                const void* grid, void* phi, void* efield);

/*
 * Stage timing with HIP events recorded on the plan's stream around each
 * stage of se1p_eval, for profiling.  Stages, in order:
 *   0 binning, 1 spreading, 2 AFT + scaling + AIFT, 3 gathering,
 *   4 real-space sum, 5 totals and energy.
 * se1p_timing_enable(plan, 1) starts recording (and clears earlier
 * records); 0 stops.  se1p_timing_read synchronises the plan's stream and
 * writes the summed milliseconds of each stage over the recorded calls
 * (ms_sum has SE1P_NSTAGE entries) and the number of calls; stages a call
 * skipped contribute zero.  Up to 4096 calls are kept.
 *
 * Each recorded event sits between two kernels of the stream and costs time
 * of its own.  se1p_timing_select(plan, stages) limits the recording to the
 * stages whose bits are set in `stages` (bit s for stage s; the default is
 * every stage), so that a timed run can price one stage with two events per
 * call; unselected stages read zero.  It clears earlier records and returns
 * SE1P_ERR_ARG for 0 or bits at or above SE1P_NSTAGE.
 */
#define SE1P_NSTAGE 6
int se1p_timing_enable(se1p_plan* plan, int enable);
int se1p_timing_select(se1p_plan* plan, unsigned stages);
int se1p_timing_read(se1p_plan* plan, double* ms_sum, int* ncalls);

/* ---- batches: many independent systems in one set of launches ----------
 *
 * A batch evaluates nsys independent neutral systems, each with its own box,
 * particle count and method parameters (all systems share the precision and
 * the support P), with one launch per stage for all of them: particle-wise
 * stages run over the packed particles, grid-shaped stages (gridding, the
 * transforms of Algorithms 2-3 with scaling, gathering, real space, totals)
 * are persistent kernels pulling (system, tile) work items, largest first,
 * from a queue.  Particles of system s occupy rows [p_s, p_s + counts[s]) of
 * the packed arrays, p_s = sum of the earlier counts.
 */
typedef struct se1p_batch se1p_batch;

/* Per-stage cost coefficients of the autotuner (nanoseconds per unit). */
typedef struct se1p_cost_model {
    double pair_ns;      /* real space, per particle pair within rc */
    double grid_ns;      /* gridding + gathering, per particle support point (P^3) */
    double fft_ns;       /* transforms, per point x log2(length) of every 1D FFT */
    double particle_ns;  /* binning, weights and totals, per particle */
    double system_ns;    /* fixed cost per system (tables, queue items) */
} se1p_cost_model;

/*
 * se1p_calibrate -- measures the cost model on the current device: builds a
 * probe plan (20000 neutral +-1 charges in a unit box at tol, with the given
 * precision and P), times its stages over a few evaluations with HIP events
 * and fits one coefficient per stage.  Synchronises; allocates and frees
 * the probe's workspace.
 */
int se1p_calibrate(double tol, int precision, int P, void* stream,
                   se1p_cost_model* out);

/*
 * se1p_autotune -- host only.  For every system s (box boxes[3s..3s+2],
 * counts[s] particles, Q[s] = sum q^2 or NULL for counts[s], i.e. unit
 * charges) picks the parameters meeting the RMS error tol (section 4.3
 * recipe as in se1p_suggest_params) with the smallest predicted cost: M3
 * runs over FFT-friendly even sizes >= P; each fixes xi by the Fourier
 * estimate, rc by the real-space estimate and the slab upsampling; the cost
 * adds the model's terms for the expected real-space pairs, the N P^3
 * gridding work and the transform work of the planned grid.  model NULL
 * uses built-in MI355X coefficients.  Tile shapes (gather blocks, gridding
 * chunks) are then chosen per system by the planner's own cost models.
 * Writes out[0..nsys-1].
 */
int se1p_autotune(double tol, int nsys, const double* boxes,
                  const long long* counts, const double* Q, int precision,
                  int P, const se1p_cost_model* model, se1p_params* out);

/*
 * se1p_batch_create -- plans every system (params[s], counts[s] >= 1
 * particles) and allocates one workspace for the batch on the current
 * device.  All params must share precision and P.  stream as for plans.
 */
int se1p_batch_create(int nsys, const se1p_params* params,
                      const long long* counts, void* stream,
                      se1p_batch** out);
int se1p_batch_destroy(se1p_batch* batch);

/*
 * se1p_batch_eval -- evaluates every system.
 *   x, q, phi, efield  packed device arrays as in se1p_eval over all
 *                      particles (phi / efield may be NULL).
 *   energy             device, nsys doubles (U of each system), or NULL.
 *   flags              SE1P_KSPACE | SE1P_REAL | SE1P_SELF, optionally
 *                      SE1P_BATCH_EAGER.
 * Unless SE1P_BATCH_EAGER, the whole sequence is captured once into a HIP
 * graph (on the batch's own capture stream) and replayed with one
 * hipGraphLaunch on the batch's stream; the graph is captured again when
 * the buffer addresses or flags differ from the previous call.  Inputs are
 * not validated on the device.
 */
#define SE1P_BATCH_EAGER 64u
int se1p_batch_eval(se1p_batch* batch, const void* x, const void* q,
                    void* phi, void* efield, double* energy, unsigned flags);

typedef struct se1p_batch_info {
    int       nsys;
    int       precision;
    int       P;
    long long n_total;          /* packed particles */
    size_t    workspace_bytes;
    int       items[10];        /* queue items per stage: spread, z FFT, row
                                   FFT, column pass, inverse rows, inverse z,
                                   gather, real space, totals, (unused) */
    int       grid[10];         /* persistent blocks launched per stage */
    int       graph_captures;   /* graphs captured so far */
} se1p_batch_info;
int se1p_batch_get_info(const se1p_batch* batch, se1p_batch_info* info);

/* Parameters and derived geometry of system s of a batch. */
int se1p_batch_system_info(const se1p_batch* batch, int s, se1p_params* params,
                           se1p_plan_info* info);

/* Human-readable text for an error code (static storage). */
const char* se1p_error_string(int code);

/* Library version string (static storage). */
const char* se1p_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SE1P_H */
