/*
 * se.h -- C ABI of the MI355X Spectral Ewald library (libse_mi355x.so).
 *
 * Evaluates the periodic Stokes potentials of Bagge & Tornberg, "Fast Ewald
 * summation for Stokes flow with arbitrary periodicity":
 *
 *   u^{DP}(x) = sum_n sum_{p in P_DP} G(x - x_n + p) . f(x_n)     eq. (periodic-potential)
 *
 * for the stokeslet, rotlet and stresslet kernels (Sec. 2, eq. stokes-kernels;
 * no 1/(8 pi) factor) with the first D in {0,1,2,3} axes periodic
 * (eq. periodic-images).  At targets that coincide with the sources the
 * starred sum (eq. periodic-potential-star) is returned: the term n = m,
 * p = 0 is omitted.  Conventions of the returned field:
 *   D = 3: Ewald zero-mode convention, i.e. zero mean flow for the stokeslet
 *          and rotlet, plus the non-periodic stresslet term (eq. k0-stresslet-3p);
 *   D = 2, 1: zero modes of the modified kernels (Sec. 3.1), with the D = 1
 *          stokeslet reported at the gauge l_B = 1, l_H = e^{-1}
 *          (eq. 1p-stokeslet-extra-contribution);
 *   D = 0: the free-space sum, decaying at infinity (eq. 0p-stokeslet-extra-contribution
 *          removed).
 * The evaluation is the Ewald decomposition (eq. Dp-ewald-decomp / -self):
 * real-space part on a cell list (Sec. 4.1.2), Fourier-space part by the
 * Spectral Ewald method (Algorithm 1), self and zero-mode terms.
 *
 * All arrays are owned by the caller.  Pointers marked (device) must be HIP
 * device (or managed) memory on the plan's device; they must stay valid until
 * the work queued on the given stream has completed.  The plan owns its
 * workspace (allocated once by se_plan_create) and never frees caller memory.
 * A plan is not thread safe; distinct plans are independent.  No exception or
 * abort crosses this ABI: every call returns an se_status.
 *
 * Layouts are row-major: positions [n][3] (x, y, z), strengths
 * [n_rhs][n][3], outputs [n_rhs][n_tgt][3], all IEEE FP64.
 */
#ifndef SE_MI355X_H
#define SE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t se_status;

#define SE_OK 0
#define SE_ERR_ARG (-1)             /* invalid argument (null pointer, bad size, bad enum) */
#define SE_ERR_UNSUPPORTED (-2)     /* valid request outside what this library implements */
#define SE_ERR_OUT_OF_BOX (-3)      /* a position lies outside [0, L_i) (device-detected) */
#define SE_ERR_NONFINITE (-4)       /* a position or strength is NaN/Inf (device-detected) */
#define SE_ERR_COINCIDENT (-5)      /* two distinct points coincide (device-detected) */
#define SE_ERR_TOL_UNREACHABLE (-6) /* tolerance below what the requested precision reaches */
#define SE_ERR_NOMEM (-7)           /* device allocation failed */
#define SE_ERR_HIP (-8)             /* a HIP runtime call failed */
#define SE_ERR_STATE (-9)           /* call out of order (e.g. execute before geometry) */
#define SE_ERR_SCRATCH (-10)        /* input larger than an allocation-free entry point's fixed scratch */

#define SE_STOKESLET 0
#define SE_ROTLET 1
#define SE_STRESSLET 2
/* Harmonic (Laplace) kernel H(r) = 1/|r| of Sec. 2, through the same
 * pipeline with the classical Ewald screening of Sec. 2.1, eq.
 * (ewald-screening), and the harmonic modified kernels of Sec. 3.1 (the ones
 * the rotlet is built from).  Applied
 * per component: the strengths f[n][3] are three independent scalar charge
 * sets and u[m][3] their three potentials, u_c(x_m) = sum_n q_{n,c} / |r|
 * summed over the periodic images.  Gauges: D = 3 drops the k = 0 mode (a
 * neutralising background); D = 2 uses -2 pi |z| for the zero mode
 * (no constant); D = 1 uses -2 log(rho) (l_H = 1); D = 0 is the free-space
 * sum.  For neutral charge sets (sum_n q_{n,c} = 0) the gauge drops out. */
#define SE_HARMONIC 3

#define SE_TOL_REL 0 /* rms-relative tolerance, mapped through the Fourier-part rms estimate U */
#define SE_TOL_ABS 1 /* absolute rms tolerance tau_rms (Sec. 4) */

#define SE_PREC_AUTO 0 /* FP32 grid path when tol >= 1e-6 (relative), else FP64 */
#define SE_PREC_FP64 1
#define SE_PREC_FP32 2

#define SE_SELECT_ANALYTIC 0 /* the paper's estimate-based procedure, Sec. 4.6 */
#define SE_SELECT_LEARNED 1  /* learned selector (se_selector_*) with analytic fallback */
#define SE_SELECT_MANUAL 2   /* caller supplies se_params */

/* Error-pollution adjustment of the estimated (h, P), eq. (error-pollution-fix)
 * and the alternative the same section reports as equally accurate. */
#define SE_POLLUTION_PAPER 0 /* (h/1.1, P+2) for D = 0, (h/1.05, P+4) for D = 1, 2, 3 */
#define SE_POLLUTION_FINE 1  /* (h/1.1, P+2) for every D: finer grid, narrower window */

/* Window function of gridding and gathering.
 * PKB: the polynomial Kaiser-Bessel window, eqs. (KB-window), (PKB-parameters),
 *   beta = 2.5 P, scaled by the exact Fourier transform of the KB window.
 * TG: the truncated Gaussian of Sec. 5.3 (window comparison), eq. (TG-window),
 *   w(r) = exp(-alpha (r/a)^2) on |r| <= a = h P / 2 with alpha = 0.91 (pi/2) P,
 *   evaluated exactly in gridding and gathering and scaled by the Fourier
 *   transform of the untruncated Gaussian, as the paper does. */
#define SE_WINDOW_PKB 0
#define SE_WINDOW_TG 1

/* Problem statement (Algorithm 1 inputs plus the error tolerance). */
typedef struct se_problem {
    int32_t struct_size;      /* sizeof(se_problem) */
    int32_t periodicity;      /* D in {0,1,2,3}: the first D axes are periodic */
    int32_t kernel;           /* SE_STOKESLET, SE_ROTLET, SE_STRESSLET or SE_HARMONIC */
    int32_t tol_kind;         /* SE_TOL_REL or SE_TOL_ABS */
    double box[3];            /* primary cell [0,L1) x [0,L2) x [0,L3), all > 0 */
    double tol;               /* rms tolerance (> 0) */
    double source_q;          /* Q = sum_n |f_n|^2 (eq. vector-source-quantity) or
                                 sum_n sum_lm f_lm^2 (eq. tensor-source-quantity);
                                 <= 0 means 3 per source (unit-variance components) */
    double xi;                /* Ewald splitting parameter; <= 0: derived from n_rc */
    double n_rc;              /* expected sources within r_c (Sec. 5.2); <= 0: the
                                 paper's uniform-system value for (kernel, D) */
    double safety;            /* tau_abs is divided by this factor; <= 0 means 1 */
    int32_t precision;        /* SE_PREC_* */
    int32_t selector;         /* SE_SELECT_* */
    int64_t n_src;            /* number of sources N >= 1 */
    int64_t n_tgt;            /* number of targets (ignored when targets_are_sources) */
    int32_t targets_are_sources; /* 1: evaluate at the sources, starred sum */
    int32_t n_rhs;            /* strength sets sharing one geometry (>= 1) */
    int32_t device;           /* HIP device ordinal */
    int32_t pollution;        /* SE_POLLUTION_PAPER or SE_POLLUTION_FINE */
    int32_t window;           /* SE_WINDOW_PKB (default 0) or SE_WINDOW_TG; the learned
                                 selector covers PKB only: TG problems take the analytic
                                 procedure, with P from 10 U e^{-alpha(P)} = tau_abs */
} se_problem;

/* Resolved method parameters (Sec. 3 and 4). */
typedef struct se_params {
    int32_t struct_size; /* sizeof(se_params) */
    int32_t P;           /* window support in grid points (even) */
    int32_t nu_deg;      /* PKB polynomial degree, eq. (PKB-parameters) */
    int32_t f_M;         /* grid-size granularity */
    int32_t M[3];        /* grid subintervals: M_i (periodic axis) or M'_i (free axis) */
    int32_t n_fft[3];    /* FFT length per axis for the bulk of the modes
                            (M_i periodic, M'_i free for D = 1, 2, 2 M'_i for D = 0) */
    int32_t n0_fft[3];   /* free axes, k^P = 0 class: length s0 M'_i (D = 1, 2) */
    int32_t nstar_fft[3];/* free axes, K_* class: length s_* M'_i (D = 1, 2) */
    int32_t kstar[2];    /* upsampling threshold kbar_* per periodic axis (x, y; D = 1, 2),
                            all 0: K_* empty */
    double xi;           /* splitting parameter */
    double rc;           /* real-space cut-off radius */
    double beta;         /* Kaiser-Bessel shape, eq. (PKB-parameters) */
    double h[3];         /* grid spacing per axis */
    double L_ext[3];     /* extended box side L'_i (= L_i on periodic axes) */
    double dL[3];        /* box padding delta L_i (0 on periodic axes) */
    double R;            /* truncation radius of the modified kernels, eq. (truncation-radius) */
    double s0;           /* k^P = 0 upsampling factor, eq. (upsampling-factor-s0) */
    double s_star;       /* K_* upsampling factor, eq. (upsampling-factor-sstar) */
    double tau_abs;      /* absolute tolerance used by the estimates */
    double U;            /* Fourier-part rms estimate U(L,Q,xi), eqs. (pot-mag-est-*) */
    double est_real;     /* real-space truncation estimate at rc */
    double est_fourier;  /* Fourier truncation estimate at pi/h */
    double est_window;   /* window estimate: 10 U e^{-2.5 P} (PKB), 10 U e^{-alpha} (TG) */
    int32_t window;      /* SE_WINDOW_* (always the problem's; ignored in manual parameters) */
    int32_t pad0;
    double alpha;        /* TG shape 0.91 (pi/2) P (0 for PKB); manual: <= 0 means that value */
} se_params;

typedef struct se_plan se_plan;

/* Library version (major*10000 + minor*100 + patch). */
int32_t se_version(void);

/* Human-readable text for a status code (static storage). */
const char* se_status_string(se_status s);

/* Parameter selection only (Sec. 4.6), no device work: fills *out exactly as
 * se_plan_create would.  Errors: SE_ERR_ARG, SE_ERR_TOL_UNREACHABLE. */
se_status se_params_select(const se_problem* prob, se_params* out);

/* Select parameters (Sec. 4.6, or `manual` when selector = SE_SELECT_MANUAL,
 * where `manual` must then be non-null: xi, rc, an even P <= 32 and, for
 * D = 3, the grid M[0..2]; for D = 2, 1 the periodic grid sizes M[0..D-1],
 * and for D = 0 the target spacing h[0], from which the free-direction
 * parameters (extended grid, truncation radius, upsampling; Sec. 4.6 steps
 * 6-7) are completed as the procedure completes its own; beta, nu_deg and
 * alpha <= 0 take the procedure's values) and allocate all device workspace on
 * prob->device.  On success *out owns the plan.  Errors: SE_ERR_ARG,
 * SE_ERR_UNSUPPORTED, SE_ERR_TOL_UNREACHABLE, SE_ERR_NOMEM, SE_ERR_HIP. */
se_status se_plan_create(const se_problem* prob, const se_params* manual, se_plan** out);

/* Release the plan and its workspace (null is a no-op).  Synchronises the
 * plan's last stream first. */
void se_plan_destroy(se_plan* plan);

/* Copy the resolved parameters. */
se_status se_plan_get_params(const se_plan* plan, se_params* out);

/* Device bytes owned by the plan. */
size_t se_plan_workspace_bytes(const se_plan* plan);

/* Text of the last error detected on the host for this plan ("" if none). */
const char* se_plan_last_message(const se_plan* plan);

/* Bind the geometry: sources src_xyz [n_src][3] (device), unit normals
 * nrm_xyz [n_src][3] (device; required for the stresslet, ignored otherwise),
 * targets tgt_xyz [n_tgt][3] (device; ignored when targets_are_sources).
 * Builds the cell list (binning, stable counting sort by cell) on `stream`
 * (a hipStream_t, null = default stream).  Asynchronous: invalid coordinates
 * are reported by se_sync_status (SE_ERR_OUT_OF_BOX / SE_ERR_NONFINITE) and
 * are replaced by 0 so that later launches stay in bounds. */
se_status se_set_geometry(se_plan* plan, const double* src_xyz, const double* nrm_xyz,
                          const double* tgt_xyz, void* stream);

/* Evaluate u = u^R + u^F + zero-mode, self and gauge terms for every strength
 * set: strengths [n_rhs][n_src][3] (device; f for S and Omega, q for T),
 * u_out [n_rhs][n_tgt][3] (device, overwritten).  Asynchronous on `stream`,
 * performs no allocation and no synchronisation.  SE_ERR_STATE if no geometry
 * was bound. */
se_status se_execute(se_plan* plan, const double* strengths, double* u_out, void* stream);

/* As se_execute but returns the real-space part in u_real and all other terms
 * (Fourier-space part, zero-mode, self and gauge terms) in u_fourier; their
 * sum is the se_execute result. */
se_status se_execute_split(se_plan* plan, const double* strengths, double* u_real,
                           double* u_fourier, void* stream);

/* Wait for the plan's queued work and return the first device-detected error
 * (SE_ERR_OUT_OF_BOX, SE_ERR_NONFINITE, SE_ERR_COINCIDENT) or SE_OK; the
 * device flag is cleared afterwards. */
se_status se_sync_status(se_plan* plan);

/* Phase timing with HIP events recorded on the execution stream around each
 * phase.  Phases: 0 geometry (se_set_geometry), 1 strengths staging,
 * 2 gridding, 3 forward x/y FFT passes, 4 z FFT + scaling + inverse z,
 * 5 inverse y/x FFT passes, 6 gathering, 7 real-space sum, 8 epilogue.
 * se_plan_set_timing(plan, 1) clears the accumulators and starts recording;
 * while it is on, every se_set_geometry / se_execute waits for its own events
 * before returning (a host synchronisation per call).  se_plan_phase_times
 * copies up to n accumulated milliseconds and launch counts. */
#define SE_NUM_PHASES 9
se_status se_plan_set_timing(se_plan* plan, int32_t on);
se_status se_plan_phase_times(const se_plan* plan, double* ms, int32_t* counts, int32_t n);

/* Debug/test access to the cell list built by se_set_geometry (device
 * pointers owned by the plan, valid until the next se_set_geometry or
 * se_plan_destroy).  which = 0: sources, 1: targets.  perm[n] = original
 * index of the n-th point in cell order; cell_start[nbins+1] = first sorted
 * index of each cell; nbins_xyz[3] = cells per axis, cell_width[3] = grid
 * cells per bin per axis. */
se_status se_debug_cell_list(const se_plan* plan, int32_t which, const int32_t** perm,
                             const int32_t** cell_start, int32_t* nbins_xyz,
                             int32_t* cell_width);

/* ---- Batches of independent systems (uneven sizes, any periodicity).
 *
 * A batch owns one plan per system (same rules as se_plan_create, selector
 * ANALYTIC or LEARNED).  se_batch_execute evaluates every system on one
 * stream.  With two or more members it runs phase by phase: one merged
 * launch per phase covers the work items of all members (tiles of gridding
 * and gathering, line bundles of the FFT passes, blocks of the real-space
 * sum), and only member-specific steps are launched per member.  The first
 * call with a given set of pointers runs the launches eagerly, then records
 * them into a HIP graph (relaxed stream capture, no memset nodes), and later
 * calls with the same pointers replay that graph as one launch.  A null
 * stream always runs eagerly.  The graph
 * is dropped by se_batch_tune, new launch shapes and pointer changes; it stays
 * valid across se_batch_set_geometry, which rewrites the plans' own buffers.
 * Arrays of pointers are host arrays of n_sys device pointers, laid out as
 * for the single-system calls.  Errors: as the single-system calls; a
 * failing system stops the call and reports its status. */
typedef struct se_batch se_batch;
se_status se_batch_create(const se_problem* probs, int32_t n_sys, se_batch** out);
se_status se_batch_destroy(se_batch* batch);
/* Member plan i (owned by the batch): parameters, timing, debug access. */
se_status se_batch_plan(se_batch* batch, int32_t i, se_plan** plan);
se_status se_batch_set_geometry(se_batch* batch, const double* const* src_xyz, const double* const* nrm_xyz,
                                const double* const* tgt_xyz, void* stream);
se_status se_batch_execute(se_batch* batch, const double* const* strengths, double* const* u_out, void* stream);
/* Autotuner: for every member plan, times the candidate launch shapes of the
 * real-space blocking (target bins per block: automatic, 1..4), then the FFT
 * column bundles (automatic, 2, 4, 8, 16), then the gridding and gathering
 * work item (automatic, 4, 8, 16, 64 batches of candidates) on the bound
 * geometry with the given strengths (synchronous, HIP events), one knob after
 * the other, and keeps the fastest of each.  The results are the same for
 * every candidate up to rounding. */
se_status se_batch_tune(se_batch* batch, const double* const* strengths, double* const* u_out, void* stream);

/* Opt-in wrapping of periodic coordinates: with on = 1, se_set_geometry
 * reduces the coordinates along the periodic axes modulo L_i into [0, L_i)
 * (the primary cell, in which eq. k0-stresslet-3p is stated) before binning;
 * with 0 (the default) a point outside the box raises SE_ERR_OUT_OF_BOX at
 * the next se_sync_status.  Free-axis coordinates must lie in [0, L_i) either
 * way.  Takes effect at the next se_set_geometry.  Errors: SE_ERR_ARG. */
se_status se_plan_set_wrap(se_plan* plan, int32_t on);

/* Launch-shape knobs of one plan (0 = automatic): real-space target bins per
 * block axis (1..4), the cap on FFT column bundles (1..16, power of 2) and
 * the work item of gridding and gathering, in batches of 64 candidate points
 * per grid tile (1..SE_TILE_ITEMS_MAX; a tile with more candidates is split
 * into further items that add their sums atomically).  Results are the same
 * for every shape up to rounding.  Errors: SE_ERR_ARG for a value out of
 * range; takes effect at the next evaluation. */
#define SE_TILE_ITEMS_MAX 16384
se_status se_plan_set_shape(se_plan* plan, int32_t real_tb, int32_t fft_cols, int32_t tile_items);
se_status se_plan_get_shape(const se_plan* plan, int32_t* real_tb, int32_t* fft_cols, int32_t* tile_items);

/* ---- Learned parameter selector.
 *
 * A fully connected FP32 network: SE_MLP_IN inputs, two tanh layers of
 * SE_MLP_HID units, SE_MLP_OUT linear outputs.  Features of a problem (raw,
 * before the normalisation stored with the weights): log10 N, ln(L_max/L_min),
 * one-hot periodicity D = 0..3, one-hot kernel (stokeslet, rotlet, stresslet),
 * log10 of the rms-relative tolerance.  Outputs: ln(xi Lc), ln(Lc/h), P and
 * ln(xi rc), with Lc = (L1 L2 L3)^(1/3) and h the grid spacing.  The
 * proposed xi is kept; the steps of Sec. 4.6 (fine pollution rule) at that
 * xi, over safety factors 1 .. 50, give a family of parameter sets, and the
 * member nearest to the proposed (rc, h, P) is used.  It is
 * rejected if the real-space, Fourier or window estimate, or their rms
 * combination, exceeds the tolerance; then, and when no weights are
 * loaded, selection falls back to SE_SELECT_ANALYTIC (se_plan_last_message
 * says which was used).  Weights are process-wide: the latest of
 * se_selector_train / se_selector_load, else the file named by the environment
 * variable SE_SELECTOR_WEIGHTS, else se_selector_weights.bin beside this
 * library.  Parameter vector (SE_MLP_NPARAM floats, row-major, output index
 * first): W1[64][10], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]. */
#define SE_MLP_IN 10
#define SE_MLP_HID 64
#define SE_MLP_OUT 4
#define SE_MLP_NPARAM 5124
#define SE_MLP_NORM (2 * SE_MLP_IN + 2 * SE_MLP_OUT) /* x mean, x std, y mean, y std */

typedef struct se_train_cfg {
    int32_t struct_size; /* sizeof(se_train_cfg) */
    int32_t epochs;      /* passes over the records (>= 1) */
    int32_t batch;       /* minibatch size (>= 1) */
    int32_t device;      /* HIP device ordinal */
    float lr, beta1, beta2, eps; /* Adam; lr > 0, 0 <= beta < 1, eps > 0 */
    uint64_t seed;       /* initial weights (Glorot-uniform) and sample order */
} se_train_cfg;

/* Feature row of a problem (host; x has SE_MLP_IN entries). */
se_status se_selector_features(const se_problem* prob, float* x);
/* Trains the process-wide network on n host records X[n][SE_MLP_IN] (raw
 * features) and Y[n][SE_MLP_OUT] (raw outputs): normalisation to zero mean and
 * unit variance from the records, then epochs of shuffled minibatches through
 * the device kernels.  loss_history (host, may be null) receives the mean
 * normalised loss of each epoch.  Synchronous. */
se_status se_selector_train(const se_train_cfg* cfg, const float* X, const float* Y, int64_t n, float* loss_history);
/* Versioned binary file (magic, sizes, normalisation, weights, checksum);
 * a corrupt or mismatched file is rejected with SE_ERR_ARG and changes nothing. */
se_status se_selector_save(const char* path);
se_status se_selector_load(const char* path);
/* 1 when weights are present (loading the default file if needed), else 0. */
int32_t se_selector_ready(void);
/* Copies out the weights (SE_MLP_NPARAM floats) and normalisation (SE_MLP_NORM). */
se_status se_selector_get(float* theta, float* norm);
/* Raw outputs for n raw feature rows (device pointers, stream-ordered). */
se_status se_selector_predict(const float* X, float* Y, int64_t n, void* stream);

/* Training building blocks on device buffers of normalised data, for checks:
 * loss = sum_i |mlp(theta, x_i) - y_i|^2 / (n SE_MLP_OUT) and grad = d loss / d
 * theta (n >= 1; grad SE_MLP_NPARAM floats, loss one float); forward gives
 * mlp(theta, x_i); adam applies one Adam step with bias corrections at step
 * t >= 1 to n parameters.  forward and adam are stream-ordered and allocate
 * nothing; loss_grad allocates a temporary buffer of per-block partial sums
 * and synchronises the stream before returning (training itself uses a
 * buffer kept for the whole run). */
se_status se_mlp_loss_grad(const float* theta, const float* X, const float* Y, int64_t n, float* grad, float* loss,
                           void* stream);
se_status se_mlp_forward(const float* theta, const float* X, int64_t n, float* Y, void* stream);
se_status se_mlp_adam(float* theta, float* m, float* v, const float* grad, int64_t n, int32_t t, float lr, float beta1,
                      float beta2, float eps, void* stream);

/* Allocation-free loss and gradient, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * se_mlp_loss_grad (bit for bit), but it allocates nothing and does not
 * synchronise: the per-block partial sums go to a fixed device array of the
 * library, SE_MLP_NOALLOC_MAX_N / 32 blocks of SE_MLP_NPARAM + 1 floats
 * (10.5 MB), which each GPU the library runs on holds until the process
 * ends.  Its address is looked up once per device, on the first call with
 * that device current; the stream must belong to the current device.  Every
 * call on a GPU uses that GPU's one array, and each call overwrites all the
 * entries it reads, so nothing carries over between calls; but calls that
 * overlap on one GPU (two streams, two threads) race on it and must be
 * ordered by the caller.  Stream-ordered: grad and loss are ready when the
 * stream reaches the end of the call.  Errors: SE_ERR_ARG (null pointer,
 * n < 1), SE_ERR_SCRATCH (n > SE_MLP_NOALLOC_MAX_N), SE_ERR_HIP. */
#define SE_MLP_NOALLOC_MAX_N 16384
se_status se_mlp_loss_grad_noalloc(const float* theta, const float* X, const float* Y, int64_t n, float* grad,
                                   float* loss, void* stream);

/* Direct Ewald reference on the GPU (no grid, no window), for checking the
 * fast method on large systems on every target.
 *   periodicity 2, 1: the decomposition of Sec. 2.3 with the same real
 *     space (images along the periodic axes, rc = min periodic side / 2),
 *     the modes k^P != 0 of eqs. (2p-fourier-space) / (1p-fourier-space) by
 *     the trapezoidal rule in the free wavenumbers (a lattice sum over the
 *     cell whose free sides are extended by 7 times the longest periodic
 *     side), the modes k^P = 0 in the closed forms of Appendices A.2 and B.2
 *     (the D = 1 stokeslet in the gauge l_B = 1, the harmonic with l_H = 1),
 *     and the self term; sources and targets must lie in the box;
 *   periodicity 3: the classical Ewald sum of Sec. 2.2, eqs.
 *     (3p-ewald-decomp-self), (real-space-potential-3p),
 *     (fourier-space-potential-3p), (k0-stresslet-3p), (self-term): the
 *     real-space part over all pairs at the minimum image with
 *     rc = min(L)/2 and the exact kernels (erfc, exp), the Fourier part as
 *     the explicit lattice sum over 0 < |k| <= 13 xi; the harmonic adds its
 *     neutralising background -pi Q_c/(V xi^2);
 *   periodicity 0: the free-space sum over all pairs.
 * Both truncations sit near e^{-42}.  xi <= 0 picks 13 / (least periodic side); a caller xi
 * below that is rejected (SE_ERR_ARG: the real-space tail would exceed the
 * cut-off).  Cost O(N_t N_s) pairs plus O((N_s + N_t) N_k) phases.
 * kernel: SE_STOKESLET, SE_ROTLET, SE_STRESSLET or SE_HARMONIC; strengths
 * [n_src][3] (f, q, or three charge sets), normals_xyz [n_src][3] for the
 * stresslet (else null); tgt_xyz null: targets are the sources (n_tgt
 * ignored, the pair m = n omitted).  All point arrays are caller-owned
 * device FP64 row-major; u_out [n_tgt][3] device.  Allocates and frees
 * temporary device memory and synchronises the stream before returning.
 * Errors: SE_ERR_ARG, SE_ERR_COINCIDENT (a distinct pair at r = 0, skipped
 * in the result), SE_ERR_NOMEM, SE_ERR_HIP. */
se_status se_ewald_reference(int32_t kernel, int32_t periodicity, const double box[3], double xi, int64_t n_src,
                             const double* src_xyz, const double* strengths, const double* normals_xyz,
                             int64_t n_tgt, const double* tgt_xyz, double* u_out, int32_t device, void* stream);

/* Boundary-integral driver: restarted GMRES over the plan's periodic
 * stresslet sum, the use the method is built for (Sec. 6), on the nodes x_n
 * of closed surfaces with quadrature weights w_n and unit outward normals
 * nu_n (the plan's sources and normals).  The double layer is regularised
 * with the stresslet identity (Sec. 2.4, eq. stresslet-identity), whose
 * value on the surface is 4 pi q0:
 *   (D q)_m = sum_{n != m} w_n T^{DP}(x_m - x_n) (q_n - q_m) nu_n + 4 pi q_m,
 * and the solver returns q with alpha q + D q = g for each of the plan's
 * n_rhs right-hand sides, in lock step (one evaluation covers all sets).
 * With outward normals the double layer of a constant density is 8 pi q0
 * inside and 0 outside, so alpha = +4 pi and -4 pi give its interior and
 * exterior limits.
 * plan: SE_STRESSLET, targets are sources, geometry bound.  weights [n]
 * device; g [n_rhs][n][3] device; q [n_rhs][n][3] device, the initial guess
 * on entry and the solution on return.  GMRES(restart) with classical
 * Gram-Schmidt applied twice; a cycle ends when every system's residual
 * estimate is <= tol |g| or after max_iter operator applications in total;
 * each cycle starts from the true residual.  iters (host, may be null)
 * receives the applications used, resid (host, n_rhs, may be null) the last
 * relative residuals (true residuals once converged).  Allocates and frees
 * its Krylov basis ((restart + 4) n_rhs 3 n doubles) and synchronises the
 * stream.  Errors: SE_ERR_ARG, SE_ERR_STATE (no geometry), SE_ERR_NOMEM,
 * SE_ERR_HIP and those of se_execute. */
se_status se_bie_solve(se_plan* plan, double alpha, const double* weights, const double* g, double* q,
                       int32_t restart, int32_t max_iter, double tol, int32_t* iters, double* resid, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SE_MI355X_H */
