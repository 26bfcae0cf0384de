/*
 * mor.h - C ABI of the MI355X reduced-frequency Lippmann-Schwinger solver.
 *
 * Method: Gierden, Waimann, Svendsen, Reese, "A geometrically adapted reduced
 * set of frequencies for a FFT-based microstructure simulation" (arXiv
 * 2103.10203).  Section references below are to that paper.
 *
 * General conventions
 *  - Every call returns a mor_status.  No exception or signal crosses the ABI.
 *    On a status other than MOR_OK, mor_last_error() returns a thread-local,
 *    NUL-terminated message that stays valid until the next call on the same
 *    thread.
 *  - Grids are C-ordered: n[0] is the slowest axis.  Array axis a is the
 *    physical direction x_{a+1}; strain component "11" is the normal strain
 *    along axis 0.
 *  - Tensor components are tensor (not engineering) components, ordered
 *      2D (plane strain): strain [11, 22, 12], stress [11, 22, 12, 33]
 *      3D:                strain and stress [11, 22, 33, 23, 13, 12].
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the current device (e.g. torch CUDA tensors' data_ptr()).
 *  - Units are the caller's (the tests use GPa).
 *  - The caller owns every buffer it passes; the library owns plans.
 *  - All work is issued on the stream given in the options (NULL = the null
 *    stream).  Calls that return host results synchronise that stream.
 *  - The solve calls keep a workspace per (device, stream): device buffers
 *    and a pinned host staging buffer (at most 64 MiB) for their small
 *    transfers, grown on demand and held until the process ends
 *    (mor_solve_noalloc uses none of it).
 */
#ifndef MOR_H
#define MOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MOR_OK = 0,
  MOR_E_INVALID_ARG = 1,   /* argument outside its documented domain          */
  MOR_E_OUT_OF_MEMORY = 2, /* a device allocation failed                      */
  MOR_E_DEVICE = 3,        /* a HIP runtime call or kernel launch failed      */
  MOR_E_NOT_CONVERGED = 4, /* max_iter reached; outputs hold the last iterate */
  MOR_E_NONFINITE = 5,     /* a NaN/Inf appeared in the iteration             */
  MOR_E_UNSUPPORTED = 6    /* valid input the library does not handle         */
} mor_status;

/* Opaque plan: the adapted sampling pattern of one microstructure and the
 * device tables derived from it.  Immutable after creation, so one plan may
 * serve concurrent solves on different streams. */
typedef struct mor_plan* mor_plan_t;

typedef struct {
  int32_t ndim;   /* 2 or 3 */
  int32_t pad_;
  int64_t n[3];   /* points per axis; 2D uses n[0], n[1] */
} mor_grid;

enum { MOR_GAMMA_ROTATED = 0,     /* rotated first-order finite differences (Sec. 3, default) */
       MOR_GAMMA_CONTINUOUS = 1 };/* classic continuous wave vector                            */

/* Kind of sampling pattern:
 *   MOR_PATTERN_ADAPTED  the geometrically adapted pattern (Sec. 4.2): the M
 *                        frequencies of highest |FFT(g)| (default)
 *   MOR_PATTERN_RADIAL   the fixed radial pattern it is compared with (Sec. 4.1,
 *                        fig. FixedSampling), 2D only: `radial_lines` straight
 *                        lines through xi = 0 at angles l pi / L (l = 0..L-1)
 *                        from the axis-1 direction towards axis 0.  A line with
 *                        angle in [0, pi/4] or [3 pi/4, pi) (4l <= L or 4l >= 3L)
 *                        takes s1 = -(n1/2-1)..n1/2-1 and s0 = round(s1 tan angle);
 *                        the others take s0 = -(n0/2-1)..n0/2-1 and
 *                        s1 = round(s0 tan(pi/2 - angle)); round = nearest,
 *                        halves away from zero; points with |s_a| > n_a/2 - 1 are
 *                        dropped.  The pattern does not depend on g and its size
 *                        follows from L (the M argument is ignored, but must
 *                        still lie in [1, N]); its rank order is the adapted
 *                        ranking with equal keys (|s|^2, then lexicographic). */
enum { MOR_PATTERN_ADAPTED = 0, MOR_PATTERN_RADIAL = 1 };

typedef struct {
  int32_t gamma_kind;   /* MOR_GAMMA_* */
  int32_t pattern_kind; /* MOR_PATTERN_* */
  void* stream;         /* hipStream_t for the plan kernels, NULL = null stream */
  int32_t radial_lines; /* MOR_PATTERN_RADIAL: number of lines, 1 <= L <= 4096 */
  int32_t pad_;
} mor_plan_opts;

typedef struct {
  int64_t N;               /* grid points                                       */
  int64_t M;               /* requested number of frequencies                   */
  int64_t M_actual;        /* selected after conjugate-pair closure (M or M+1)  */
  int64_t n_coeff;         /* stored coefficients per strain component (the
                              half-spectrum part of the pattern)                */
  int64_t n_columns;       /* distinct frequency columns of the transform       */
  int64_t n_last;          /* distinct last-axis frequencies (3D), = n_columns in 2D */
  int64_t inclusion_count; /* voxels with g = 1                                 */
  int32_t ncomp;           /* strain components: 3 (2D) or 6 (3D)               */
  int32_t nstress;         /* stress components: 4 (2D) or 6 (3D)               */
  int32_t pattern_kind;    /* MOR_PATTERN_*                                     */
  int32_t radial_lines;    /* lines of a radial pattern, else 0                 */
} mor_plan_info;

/*
 * mor_plan_create - geometrically adapted sampling pattern (Sec. 4.2).
 *
 * Computes the FP64 power spectrum P(m) = |FFT(g)(m)|^2 of the phase
 * indicator g (1 = inclusion, 0 = matrix), ranks the frequencies by
 * amplitude and keeps the first M (whole conjugate pairs; xi = 0 always),
 * then builds the transform and Green-operator tables of the reduced scheme
 * (Sec. 4, steps b-d).  Ranking: key(m) = float32_rn(P(m)/P(0)), or 0 where
 * P(m) <= 2^-80 P(0), descending; ties by |s(m)|^2 ascending (s = signed
 * centred frequency, N/2 counted +N/2), then by the lexicographic rank of the
 * pair's representative (the member with the smaller rank over
 * u_a = s_a + (n_a-1)/2, axis 0 most significant).
 *
 *   grid      host; ndim 2 or 3; every n even, n = 2^a 3^b, 4 <= n <= 1024
 *             (other sizes: MOR_E_UNSUPPORTED).
 *   phase_map host uint8 [N], values 0 or 1 (else MOR_E_INVALID_ARG).
 *   M         1 <= M <= N.
 *   opts      NULL for defaults.
 *   out       receives the plan; release with mor_plan_destroy.
 */
mor_status mor_plan_create(const mor_grid* grid, const uint8_t* phase_map, int64_t M,
                           const mor_plan_opts* opts, mor_plan_t* out);

/*
 * mor_plan_create_batch - mor_plan_create for `count` microstructures on one
 * grid (Sec. 4.2, one pattern per microstructure, as for the integration
 * points of an FE-FFT computation, Sec. 1).  Each step of the construction
 * runs as one launch over the whole batch, so the cost per plan is device
 * work rather than launch and synchronisation latency.  The plans are the
 * ones mor_plan_create returns for each map and M, bit for bit.
 *
 *   grid        as for mor_plan_create, shared by every map.
 *   count       >= 0; 0 creates nothing and returns MOR_OK.
 *   phase_maps  host [count] pointers, each to a host uint8 [N] map (C
 *               order, values 0 or 1); the maps need not be adjacent.
 *   M           host int64 [count], each in [1, N].
 *   opts        NULL for defaults (gamma_kind and stream apply to all).
 *   out         host [count]; receives the plans.  On any error every
 *               entry is NULL: plans already built are destroyed.
 * Every map and M is checked before any device work.  Device scratch is
 * drawn in chunks of microstructures of at most 512 MiB (environment
 * variable MOR_PLAN_SCRATCH_BYTES overrides the size), held in the library's
 * block pool for reuse; each chunk's maps are staged in pinned host memory
 * allocated and released by the call.
 */
mor_status mor_plan_create_batch(const mor_grid* grid, int64_t count, const uint8_t* const* phase_maps,
                                 const int64_t* M, const mor_plan_opts* opts, mor_plan_t* out);

mor_status mor_plan_get_info(mor_plan_t plan, mor_plan_info* info);

/*
 * mor_plan_pattern - copy the pattern to host memory.
 *   sorted_idx host int64 [cap] or NULL: linear FFT indices, ascending.
 *   rank_idx   host int64 [cap] or NULL: the same set in selection order
 *              (each pair's representative, then its partner).
 *   cap must be >= M_actual when either array is given.
 */
mor_status mor_plan_pattern(mor_plan_t plan, int64_t* sorted_idx, int64_t* rank_idx,
                            int64_t cap, int64_t* M_actual);

/*
 * mor_plan_coeff_index - linear FFT index of every stored coefficient, in
 * the library's coefficient order (host int64 [n_coeff]).  Lets a caller
 * read or seed the coefficient arrays of mor_solve.
 */
mor_status mor_plan_coeff_index(mor_plan_t plan, int64_t* lin_idx, int64_t cap);

mor_status mor_plan_destroy(mor_plan_t plan);

/* Phase material (Sec. 2): isotropic Lame constants; J2 plasticity with
 * initial yield stress sigma_y0 and linear isotropic hardening modulus H when
 * plastic != 0.  phase[0] is the matrix (g = 0), phase[1] the inclusion. */
typedef struct {
  double lambda, mu, sigma_y0, H;
  int32_t plastic;
  int32_t pad_;
} mor_phase;

/* Arithmetic of the iteration (the residual and the grid mean of sigma are
 * FP64 sums in every mode):
 *   MOR_PREC_FP32    FP32 transforms and fields (default; specialised kernels)
 *   MOR_PREC_BF16X3  split-bf16 partial DFT on MFMA, FP32 accumulate
 *   MOR_PREC_FP64    FP64 transforms, Green operator and Hooke law (generic
 *                    kernels; Hooke phases, FFT transform and grid schedule
 *                    only, else MOR_E_UNSUPPORTED).  For tolerances below what
 *                    FP32 reaches (the paper's examples stop at 1e-8); field
 *                    and coefficient outputs are rounded to FP32. */
enum { MOR_PREC_FP32 = 0, MOR_PREC_BF16X3 = 1, MOR_PREC_FP64 = 2 };
enum { MOR_TRANSFORM_AUTO = 0, MOR_TRANSFORM_FFT = 1, MOR_TRANSFORM_DFT = 2 };
/* Work schedule of the iteration kernels (same results):
 *   MOR_SCHED_GRID        one workgroup per (RVE, tile); converged RVEs' workgroups exit at once
 *   MOR_SCHED_PERSISTENT  a grid sized to the device's residency walks a device-built queue of
 *                         the still-iterating RVEs' tiles (specialised row/column kernels; other
 *                         kernels keep the grid schedule) */
enum { MOR_SCHED_GRID = 0, MOR_SCHED_PERSISTENT = 1 };

typedef struct {
  int32_t max_iter;     /* 0 -> 10000                                            */
  int32_t precision;    /* MOR_PREC_*                                            */
  int32_t transform;    /* MOR_TRANSFORM_*                                       */
  int32_t check_every;  /* iterations between device->host convergence polls;
                           0 -> library default                                  */
  const float* warm_start; /* device complex64 [B][ncomp][n_coeff] strain
                              coefficients in plan coefficient order (the
                              zero frequency entry is ignored and set to
                              N * macro strain), or NULL for the cold start
                              eps0 = macro strain                                */
  void* stream;         /* hipStream_t, NULL = null stream                       */
  int32_t use_graph;    /* replay the iteration chunk from a captured hipGraph   */
  int32_t schedule;     /* MOR_SCHED_*: how workgroups map to (RVE, tile) work   */
} mor_solve_opts;

typedef struct {
  double* eff_stress;   /* host [B][nstress] or NULL: grid mean of sigma(eps_final), FP64 sum */
  float* strain;        /* device [B][ncomp][N] or NULL                                      */
  float* stress;        /* device [B][nstress][N] or NULL                                    */
  int32_t* iterations;  /* host [B] or NULL: Green-operator applications                     */
  double* residual;     /* host [B] or NULL: last residual                                   */
  float* coeffs;        /* device complex64 [B][ncomp][n_coeff] or NULL: final strain
                           coefficients (unnormalised DFT of eps_final)                      */
} mor_outputs;

/*
 * mor_solve - reduced basic fixed-point scheme (Sec. 4, steps a-d) for B
 * RVEs of one microstructure with different macro strains.
 *
 * Per iteration: a) tau = sigma(eps) - C0:eps at every grid point (C0 = mean
 * of the two phases' Lame constants, Sec. 3); b) tau^ on the pattern;
 * c) eps^ = -Gamma0^ : tau^ (eps^(0) = N eps_bar); d) eps on the grid.
 * Stops per RVE at the first residual
 *     r = sqrt(mean_x ||eps^{i+1}-eps^i||_F^2) / ||eps_bar||_F < tol
 * (denominator 1 if eps_bar = 0); r is evaluated in FP64 from the
 * coefficients (Parseval).  Then sigma(eps_final) and its FP64 grid mean.
 *
 *   macro_strain host double [B][ncomp], B >= 1 (an empty batch is
 *                rejected with MOR_E_INVALID_ARG before any device work).
 *   phase        host [2].
 *   tol > 0.
 * Returns MOR_E_NOT_CONVERGED (outputs = last iterate) if an RVE hits
 * max_iter, MOR_E_NONFINITE if an RVE's residual became NaN/Inf.
 */
mor_status mor_solve(mor_plan_t plan, const double* macro_strain, int64_t B,
                     const mor_phase phase[2], double tol, const mor_solve_opts* opts,
                     mor_outputs* out);

/*
 * mor_solve_noalloc - mor_solve without any device or pinned-memory
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Arguments, results and kernels are those of mor_solve.  Every workspace
 * buffer of the solve (coefficients, transform lines, residual and stress
 * partials, per-RVE states, the J2 state of Hooke/J2 solves) is carved from
 * one library-owned device array of MOR_NOALLOC_SCRATCH_BYTES per GPU,
 * which the GPU holds from the library's load until the process ends.
 *   - A solve that needs more than the array returns MOR_E_INVALID_ARG
 *     before any kernel runs (call again with fewer RVEs).
 *   - opts->use_graph must be 0 (MOR_E_UNSUPPORTED otherwise); per-kernel
 *     profiling events are not recorded.
 *   - Every call on one GPU shares that GPU's array and overwrites it:
 *     calls that overlap on one GPU (other streams or threads) race and give
 *     undefined results.  Serialise them.
 *   - Host results (eff_stress, iterations, residual) synchronise the stream
 *     as in mor_solve.
 */
#define MOR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mor_status mor_solve_noalloc(mor_plan_t plan, const double* macro_strain, int64_t B,
                             const mor_phase phase[2], double tol, const mor_solve_opts* opts,
                             mor_outputs* out);

/*
 * mor_solve_multi - as mor_solve for B RVEs that may use different plans
 * (different microstructures and grid sizes) in one call.  RVE b uses
 * plans[plan_of_rve[b]] (host arrays).  Field outputs are packed: RVE b's
 * strain starts at element offset ncomp * (sum of N of RVEs before b), and
 * likewise stress with nstress; eff_stress rows have 6 entries per RVE
 * (2D RVEs use the first 4).  Coefficient outputs/warm starts are packed the
 * same way with n_coeff.
 */
mor_status mor_solve_multi(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of_rve,
                           const double* macro_strain_packed, int64_t B, const mor_phase phase[2],
                           double tol, const mor_solve_opts* opts, mor_outputs* out);

/*
 * mor_solve_path - elasto-plastic load path (Secs. 2 and 5.2): `steps`
 * macro strains applied in order, one RVE.  Step n starts from the converged
 * strain of step n-1 plus the macro increment; the J2 state committed at the
 * end of step n-1 is held fixed during step n's iterations and replaced by
 * the state of step n's final constitutive evaluation.
 *
 *   macro_strain host double [steps][ncomp].
 *   state        device float [nstate][N], caller-owned, in/out; nstate = 5
 *                in 2D (eps_p 11, 22, 12, 33, accumulated plastic strain)
 *                and 7 in 3D (eps_p 11, 22, 33, 23, 13, 12, accumulated).
 *                Zero it for a virgin material.
 *   out          eff_stress host [steps][nstress], iterations/residual host
 *                [steps]; field and coefficient outputs hold the last step.
 */
mor_status mor_solve_path(mor_plan_t plan, const double* macro_strain, int32_t steps,
                          const mor_phase phase[2], double tol, const mor_solve_opts* opts,
                          float* state, mor_outputs* out);

/*
 * mor_solve_path_multi - load paths of B RVEs in one call (Secs. 2 and 5.2),
 * e.g. the integration points of an FE-FFT computation, each with its own
 * macro strain history and committed J2 state; RVE b uses
 * plans[plan_of_rve[b]] (host arrays; the plans may differ in grid).  Every
 * iteration runs one set of launches over all RVEs still iterating, so the
 * device is filled even when one RVE alone would not fill it.  Step rules as
 * in mor_solve_path, per RVE.  Per-step results stay on the device until the
 * call ends (no host synchronisation between steps beyond the convergence
 * polls).
 *
 *   macro_strain host double [B][steps][ncomp].
 *   state        device float, RVE b's [nstate][N_b] block at element offset
 *                nstate * (sum of N of RVEs before b); in/out; zero for a
 *                virgin material.
 *   out          eff_stress host [B][steps][6] (2D uses the first 4),
 *                iterations/residual host [B][steps]; strain/stress/coeffs
 *                packed as in mor_solve_multi, for the last step.
 */
mor_status mor_solve_path_multi(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of_rve,
                                const double* macro_strain, int64_t B, int32_t steps, const mor_phase phase[2],
                                double tol, const mor_solve_opts* opts, float* state, mor_outputs* out);

/*
 * mor_compat - compatibility step (Sec. 4.1 post-processing; applied alone to
 * the adapted-pattern results in Sec. 5.1): the Lippmann-Schwinger equation
 * solved once on the full set of frequencies from the fields of a reduced
 * solution.  One pass of steps a)-d) with every frequency kept, from eps_red:
 *   tau = sigma(eps_red) - C0 : eps_red,  eps^(xi) = -Gamma0^(xi) : tau^(xi)
 *   (xi != 0), eps^(0) = N eps_bar,  eps_comp = iFFT(eps^),
 * then sigma(eps_comp) and its FP64 grid mean.  Runs on the solver's kernels
 * with plan_full's tables (the reduced coefficients are placed at their
 * frequencies of the full set as the starting field).
 *
 *   plan       the plan the reduced solution was computed on.
 *   plan_full  a plan of the same grid and microstructure holding every
 *              frequency (mor_plan_create with M = N); MOR_E_INVALID_ARG if
 *              its grid, inclusion count or size do not fit.
 *   coeffs     device complex64 [B][ncomp][n_coeff of plan]: the reduced
 *              strain coefficients (mor_solve's coeffs output).
 *   macro_strain host double [B][ncomp]; phase as for the solve.
 *   state      J2 phases: device float [B][nstate][N], the committed state
 *              the reduced solution was computed with (read only; NULL =
 *              virgin material).  Ignored for Hooke phases.
 *   opts       precision/transform/stream as for mor_solve (max_iter,
 *              warm_start and use_graph are set by the call).
 *   out        as mor_solve on plan_full: eff_stress = grid mean of
 *              sigma(eps_comp); strain/stress = eps_comp, sigma(eps_comp);
 *              iterations = 1; residual = RMS ||eps_comp - eps_red||_F /
 *              ||eps_bar||_F; coeffs in plan_full's layout.
 */
mor_status mor_compat(mor_plan_t plan, mor_plan_t plan_full, const float* coeffs, const double* macro_strain,
                      int64_t B, const mor_phase phase[2], const float* state, const mor_solve_opts* opts,
                      mor_outputs* out);

/*
 * mor_stress_error - the error measures of Sec. 5 of a reduced solution
 * against a reference solution (the full set of frequencies):
 *   E_bar[b] = ||sigma_bar - sigma_bar_ref|| / ||sigma_bar_ref||
 *   E[b]     = mean over the kept grid points x of
 *              ||sigma(x) - sigma_ref(x)|| / ||sigma_ref(x)||
 * Norms are Frobenius norms of the full symmetric tensor (shear components
 * counted twice; sigma_33 included in 2D).  The pointwise quotient needs
 * ||sigma_ref(x)|| > 0: points with ||sigma_ref(x)|| <= skip_rel * max_x
 * ||sigma_ref|| are left out of the mean (E = 0 if none is kept).  FP64
 * arithmetic; fixed summation order.
 *
 *   sigma, sigma_ref  device float [B][nstress][N] (mor_solve's stress output
 *                     layout), needed when E != NULL.
 *   eff, eff_ref      host double [B][nstress], needed when E_bar != NULL.
 *   ndim              2 (nstress 4) or 3 (nstress 6).
 *   E_bar, E          host double [B] or NULL (that measure is skipped).
 * Synchronises `stream` when E is requested.  Device scratch (a few KB per
 * RVE) is kept per device and grown on demand.
 */
mor_status mor_stress_error(const float* sigma, const float* sigma_ref, const double* eff, const double* eff_ref,
                            int64_t B, int64_t N, int32_t ndim, double skip_rel, void* stream, double* E_bar,
                            double* E);

/* ----------------------------------------------------------------------
 * Learned warm start (an addition to the paper's method).  A 3-layer
 * perceptron x -> relu(x W1 + b1) -> relu(. W2 + b2) -> . W3 + b3 maps
 * features of a microstructure's adapted pattern to the per-unit-macro-strain
 * strain response at the pattern's first `nslots` conjugate pairs ("slots",
 * rank order, xi = 0 excluded).  The network learns the correction to the
 * first-order (Born) term  -Gamma^0(n) : ((C_I - C_M) : e_k) g^(xi)  with the
 * solver's reference medium C0 (mean Lame constants) -- the coefficients that
 * the cold start's first iteration produces -- so a zero network output
 * reproduces one cold iteration.  Its prediction only seeds the fixed-point
 * iteration, which still runs to tolerance (2D plans only).
 *
 * Layouts (row-major, FP32):
 *   features X [B][4*nslots + 1]: Re g^/count, Im g^/count of every slot's
 *     pair representative, then its signed frequency (k0/n0, k1/n1), then the
 *     inclusion volume fraction; zeros beyond the plan's slot count.
 *   targets / prediction Y [B][nslots][3 strain comps][3 unit macro strains]
 *     [re, im]: eps^(rep)[c] / N for the unit macro strain e_k, minus its
 *     Born term.
 *   phase[2]: the solve's phases (phase[0] matrix, phase[1] inclusion); they
 *     fix the Born term.  MOR_E_INVALID_ARG if the mean medium has mu0 <= 0.
 *   parameters: W1 [in][hid], b1 [hid], W2 [hid][hid], b2 [hid], W3 [hid][out], b3 [out].
 * ---------------------------------------------------------------------- */
typedef struct mor_mlp* mor_mlp_t;
enum { MOR_MLP_FP32 = 0, MOR_MLP_BF16 = 1 };

/* He-uniform weights from `seed`, zero biases, zero Adam moments. */
mor_status mor_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed, mor_mlp_t* out);
mor_status mor_mlp_destroy(mor_mlp_t net);
mor_status mor_mlp_num_params(mor_mlp_t net, int64_t* count);
/* Copy parameters (which = 0), last gradients (1), Adam first (2) or second
 * (3) moments to/from host memory, `count` = mor_mlp_num_params. */
mor_status mor_mlp_get_params(mor_mlp_t net, float* host, int64_t count, int32_t which);
mor_status mor_mlp_set_params(mor_mlp_t net, const float* host, int64_t count, int32_t which);
/* Y [B][out] = network(X [B][in]); device pointers; precision MOR_MLP_FP32 or
 * MOR_MLP_BF16 (weights and activations rounded to bfloat16, FP32 accumulate). */
mor_status mor_mlp_forward(mor_mlp_t net, const float* X, int64_t B, float* Y, int32_t precision, void* stream);
/* FP32 forward + analytic backward of loss = sum (Y - T)^2 / (B * out);
 * gradients are kept in the network; *loss (host, may be NULL) receives the
 * loss (synchronises the stream when non-NULL). */
mor_status mor_mlp_grad(mor_mlp_t net, const float* X, const float* T, int64_t B, double* loss, void* stream);
/* One Adam step with the stored gradients (bias-corrected, step counter kept). */
mor_status mor_mlp_adam(mor_mlp_t net, float lr, float beta1, float beta2, float eps, void* stream);
/* Network inputs for B RVEs (RVE b uses plans[plan_of[b]], host arrays). */
mor_status mor_warm_features(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of, int64_t B,
                             int32_t nslots, float* X, void* stream);
/* Training targets from converged coefficients of the three unit macro
 * strains per RVE: coeffs device complex64, packed per RVE as
 * [3 unit strains][3 comps][n_coeff] (the layout of mor_solve_multi's
 * coefficient output for RVEs ordered (b, k)). */
mor_status mor_warm_targets(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of, int64_t B,
                            int32_t nslots, const mor_phase phase[2], const float* coeffs, float* T, void* stream);
/* Warm-start coefficients eps^ = N sum_k (Born[..][k] + Y[..][k]) macro_strain[k]
 * (host double [B][3]) in the solver's packed coefficient layout (device complex64
 * [B][3][n_coeff]); the Born term covers every coefficient of the pattern,
 * the network's correction only slots below nslots; xi = 0 is zero.  The solver
 * projects a warm start onto compatible strains before iterating. */
mor_status mor_warm_apply(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of, int64_t B, int32_t nslots,
                          const mor_phase phase[2], const float* Y, const double* macro_strain, float* warm,
                          void* stream);

/* ----------------------------------------------------------------------
 * Kernel variants and autotuning (launch shape and FFT factorisation of the
 * row and column kernels; not part of the paper's method).  Variants of one
 * size give the same results up to FP32 rounding; a solve uses the variants
 * selected for its sizes when it starts.  Unselected sizes use variant 0,
 * except the row kernel with J2 phases on 512-point last axes (variant 4)
 * and 384-point last axes (variant 2), whose radix-4 register passes leave
 * room for the plastic state; mor_tune_get reports a selection, or 0 when
 * there is none.  The selection is per process, shared by all threads
 * and devices.
 *   kernel  MOR_KERNEL_ROW (last axis) or MOR_KERNEL_COL (axis 0)
 *   ndim    2 or 3; length = the grid's last-axis length n[ndim-1] (row) or
 *           its axis-0 length n[0] (column)
 * MOR_E_INVALID_ARG when that size has no specialised row kernel or the
 * variant is out of range.
 * ---------------------------------------------------------------------- */
enum { MOR_KERNEL_ROW = 0, MOR_KERNEL_COL = 1 };
mor_status mor_tune_variants(int32_t kernel, int32_t ndim, int32_t length, int32_t* count);
mor_status mor_tune_get(int32_t kernel, int32_t ndim, int32_t length, int32_t* variant);
mor_status mor_tune_set(int32_t kernel, int32_t ndim, int32_t length, int32_t variant);
/* Sub-batches of the batched solves: the RVEs of one grid are cut into the
 * fewest runs of about equal size whose transform lines fit `bytes`, but
 * into no runs of fewer than `min_rves` RVEs, and the iteration loop runs
 * each run's chunk of iterations before the next, so the lines stay in the
 * last-level cache between the row and column passes.  Results do not
 * depend on the cut (every RVE iterates on its own).  Defaults: 192 MiB
 * (MOR_SUBBATCH_MIB in the environment, in MiB, sets the start value) and
 * 128 RVEs; bytes = 0 keeps each grid's RVEs together; -1 keeps a value.
 * *prev_bytes, *prev_min (may be NULL) receive the values before the call.
 * Process-wide. */
mor_status mor_tune_subbatch(int64_t bytes, int64_t min_rves, int64_t* prev_bytes, int64_t* prev_min);
/* Autotuner: for every row and column length present among `plans`, runs the batched
 * solve (mor_solve_multi arguments) once untimed and `reps` times timed with
 * each variant, keeps the fastest (minimum wall time) and leaves it selected.
 * The solves' outputs are discarded. */
mor_status mor_autotune(const mor_plan_t* plans, int64_t nplans, const int64_t* plan_of_rve,
                        const double* macro_strain, int64_t B, const mor_phase phase[2], double tol,
                        int32_t reps, void* stream);

/* Per-kernel timing over solves while enabled: HIP events bracket every launch
 * of the named kernel on the solve stream; `items` counts the work units the
 * launches processed (converged RVEs exit early and are not counted) and
 * `bytes` the algorithmic HBM bytes of those units. */
mor_status mor_profile_enable(int32_t on);
mor_status mor_profile_reset(void);
mor_status mor_profile_query(const char* kernel, double* total_ms, int64_t* launches,
                             int64_t* items, double* bytes);

const char* mor_last_error(void);
const char* mor_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MOR_H */
