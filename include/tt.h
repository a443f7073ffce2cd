/*
 * tt.h -- C ABI of the MI355X Toeplitz spatio-angular MMSE tomographic
 * reconstructor (Ono, Correia, Conan, Blanco, Neichel, Fusco, JOSA A 2018,
 * "Fast Iterative Tomographic Wave-front Estimation with Recursive Toeplitz
 * Reconstructor Structure for Large Scale Systems").
 *
 * The library solves the first step of the spatio-angular reconstructor
 * (§2.C, first two-step equation, with the aperture masks of §2.F)
 *
 *     W_s (Sigma_ss + Sigma_eta) W_s^T zeta = s
 *
 * by conjugate gradients (§2.G) whose matrix-vector products use the
 * two-level recursive block Toeplitz (2RBT) structure of Sigma_ss (§2.D) and
 * the circulant-embedding product of §2.E (shuffle, 2-D FFT, per-frequency
 * products summed over blocks, inverse FFT, reshuffle), and then the second
 * step phi = W_phi Sigma_{phi_beta s} zeta through the per-layer grids and
 * bilinear interpolation of the LGS phase-slope product (§2.D "Phase-Slope
 * Covariance Matrix", §2.E LGS equation).  Covariances follow the Hudgin-like
 * model with the von Karman structure function (App. A.2).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Subaperture (i, j) is row i (y) and column j (x); masks are row-major
 *   n*n bytes, index i*n + j.  Phase points are the (n+1)^2 subaperture
 *   corners, index i*(n+1) + j.
 * - Slope vectors hold only valid subapertures (W_s): channel c = 2*g + p
 *   (g = guide star, p = 0 x / 1 y), element c*n_vs + v where v enumerates
 *   the valid subapertures in row-major order.  Slopes are phase differences
 *   across one subaperture in radians at the wavelength of r0 (500 nm).
 * - Reconstructed phase phi holds only valid phase points (W_phi: corners of
 *   valid subapertures) in row-major order, in radians.
 * - Pointers named d_* are device pointers on the context's device and are
 *   owned by the caller; they must stay valid until the work enqueued on the
 *   context's stream has finished.  Every other pointer is a host pointer that
 *   is read during the call only (the library copies what it keeps).
 * - Work is enqueued on the context's stream; calls return without waiting
 *   unless documented otherwise.  A context is not thread-safe; use one
 *   context per stream.
 * - Errors: every call returns a tt_status; no exception crosses the ABI.
 *   Outputs are valid only when the status is TT_OK (or TT_NOT_CONVERGED for
 *   the solution of a solve).  tt_last_error() describes the last failure of
 *   the calling thread.
 */
#ifndef TT_H
#define TT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TT_OK = 0,
    TT_INVALID_ARG = 1,     /* bad size, pointer or parameter; nothing was enqueued */
    TT_HIP_ERROR = 2,       /* a HIP runtime call failed */
    TT_OUT_OF_MEMORY = 3,   /* device allocation failed */
    TT_NOT_CONVERGED = 4,   /* iteration cap reached; zeta holds the last iterate */
    TT_BREAKDOWN = 5,       /* p^T A p <= 0 or a non-finite scalar in CG */
    TT_NOT_READY = 6        /* tt_set_system (or a target) is missing */
} tt_status;

typedef enum {
    TT_PREC_F32 = 0,        /* FP32 spectra and vectors, FP64 dot products, FP64
                               residual refinement (true residual b - A x with the
                               FP64 operator each time the FP32 residual has
                               dropped by refine_drop); certifies tol in FP64 */
    TT_PREC_F64 = 1,        /* FP64 throughout */
    TT_PREC_F16 = 2,        /* reduced precision where the outer method stays exact:
                               with TT_SOLVER_BATCHED and TT_PRECOND_CIRCULANT the
                               preconditioner's spectra are stored in FP16 (each
                               frequency scaled by a power of two; half the bytes)
                               while the product stays FP32 and the FP64 true
                               residual certifies tol.  With TT_SOLVER_PERSISTENT
                               the column DFT stages of the product itself run on
                               the matrix cores with FP16 operands (data scaled per
                               column block) and FP32 accumulation: an inexact
                               operator, which at the conditioning of these systems
                               does not reach 1e-6 (TT_NOT_CONVERGED, with the FP64
                               residual of the returned iterate). */
    TT_PREC_BF16 = 3        /* as TT_PREC_F16 with BF16 (unscaled) */
} tt_precision;

typedef enum {
    TT_SOLVER_PERSISTENT = 0, /* one persistent launch per solve segment, grid
                                 barriers between phases, on-device convergence */
    TT_SOLVER_KERNELS = 1,    /* one launch per phase, host polls convergence */
    TT_SOLVER_BATCHED = 2     /* for tt_solve_batch: CG on every system of the call in
                                 lockstep, each iteration's products by one batched
                                 product (as tt_matvec_batch, whose size limits apply)
                                 and the vector updates by kernels over all systems;
                                 FP32 with the FP64 residual replacement per system,
                                 TT_METHOD_CG, no mode removal; TT_PRECOND_CIRCULANT
                                 applies the block-circulant preconditioner batched in
                                 the same way (spectra built once per context).
                                 tt_solve_frame with it solves a batch of one. */
} tt_solver_kind;

typedef enum {
    TT_METHOD_CG = 0,         /* conjugate gradients (§2.G) */
    TT_METHOD_MINRES = 1      /* minimum residual (Paige-Saunders Lanczos + Givens QR), the
                                 paper's solver for its Toeplitz system (§2.G); stops on the
                                 QR residual estimate, certified like CG by the FP64 true
                                 residual.  TT_SOLVER_PERSISTENT with TT_PREC_F32 or
                                 TT_PREC_F64, no preconditioner, and a block's grid rows
                                 must fit its threads (as TT_PRECOND_CIRCULANT). */
} tt_method;

typedef enum {
    TT_PRECOND_NONE = 0,      /* plain CG (§2.G) */
    TT_PRECOND_CIRCULANT = 1, /* CG preconditioned by the block-circulant inverse: the
                                 restriction to the valid subapertures of
                                 F^-1 (M_+(f) + sigma^2 I)^-1 F, with M(f) the per-frequency
                                 matrix of the embedded slope spectra of the product (§2.E),
                                 M_+ its positive part and sigma^2 the mean noise variance.
                                 Symmetric positive definite; built once per system (FP64,
                                 on the host) at the first solve that asks for it.  The
                                 paper leaves preconditioning open (§2.G).
                                 TT_SOLVER_PERSISTENT with TT_PREC_F32 or TT_PREC_F64 (and a
                                 block's grid rows must fit its threads:
                                 n * ceil(2 n_gs n / compute units) <= 512), or
                                 TT_SOLVER_BATCHED (FP32). */
    TT_PRECOND_LEARNED = 2    /* flexible CG preconditioned by the learned network attached
                                 with tt_set_learned: P = K^T K (see tt_learned_create),
                                 beta in the Polak-Ribiere form r'.(u' - u) / r.u, u = P r,
                                 restarted from P r at every FP64 residual replacement.
                                 Plain CG is the fallback: a system whose r.P r is not
                                 positive or finite, or whose recursive residual has not
                                 reached a new minimum for 256 iterations, restarts from
                                 its FP64 true residual as plain CG (tt_solve_info.fallback).
                                 The FP64 true residual certifies the tolerance either way.
                                 TT_SOLVER_BATCHED, TT_PREC_F32, no mode removal. */
} tt_preconditioner;

typedef enum {
    TT_MODEL_HUDGIN = 0,     /* App. A.2 Hudgin-like two-point slopes */
    TT_MODEL_FRIED = 1       /* App. A.3 Fried four-corner slopes */
} tt_gradient_model;

/* Sensor geometry (§2, §2.D, §2.F).  The library copies every array. */
typedef struct {
    int n;                        /* subapertures across one sensor, 1..512 */
    int n_gs;                     /* guide stars (one sensor each), 1..16 */
    int pad_L;                    /* FFT side of the slope-slope products, >= 2n-1,
                                     <= 1024 */
    int gradient_model;           /* tt_gradient_model */
    double D;                     /* pupil diameter [m]; subaperture d = D/n */
    double h_lgs;                 /* LGS altitude [m]; <= 0 or +inf: natural guide stars */
    const double* gs_xy;          /* 2*n_gs: direction (x, y) of each guide star [rad] */
    const unsigned char* valid;   /* n*n, row-major, nonzero = valid subaperture (W_s), or
                                     NULL: the rule of tt_pupil_mask with `obstruction` */
    double obstruction;           /* central obstruction (diameter ratio, [0, 1)); read only
                                     when valid is NULL */
} tt_geometry;

/* Layered von Karman atmosphere (§2, App. A.2).  Layer k contributes
 * w[k] * D(r) with D the von Karman structure function of r0, L0. */
typedef struct {
    int n_layer;                  /* 1..256 */
    const double* h;              /* n_layer altitudes [m], 0 <= h < h_lgs */
    const double* w;              /* n_layer fractional C_n^2 weights (not renormalised) */
    double r0;                    /* Fried parameter [m] at the phase wavelength */
    double L0;                    /* outer scale [m] */
} tt_atmosphere;

/* Reconstruction direction and the per-layer grids of the LGS phase-slope
 * product (§2.D, §2.E): every layer uses a common n' x n' grid of spacing
 * s_k d, s_k = 1 - h_k/h_lgs, centred on the direction. */
typedef struct {
    double beta_x, beta_y;        /* target direction [rad] (target at infinity) */
    int n_prime;                  /* 0: ceil(n / min_k s_k) + 1 */
    int pad_L;                    /* FFT side, >= n' + n - 1; 0: n' + n - 1 rounded up to even */
} tt_target;

typedef struct {
    double tol;                   /* stop at ||s - A zeta||_2 <= tol ||s||_2 */
    int max_iter;                 /* cap on CG iterations (all segments together) */
    int precision;                /* tt_precision */
    int solver;                   /* tt_solver_kind */
    double refine_drop;           /* TT_PREC_F32: FP64 residual replacement when the
                                     recursive residual fell by this factor since the
                                     last one (0 -> 1e-3) */
    int preconditioner;           /* tt_preconditioner (0: none) */
    int method;                   /* tt_method (0: CG) */
    int graph;                    /* TT_SOLVER_BATCHED: nonzero replays each chunk of 16
                                     lockstep iterations from a captured HIP graph while the
                                     set of iterating systems is unchanged (same kernels and
                                     results as launching them one by one, 0) */
} tt_solve_opts;

typedef struct {
    int iterations;               /* CG iterations done */
    int refinements;              /* FP64 residual replacements done */
    int status;                   /* tt_status of the solve */
    double rel_residual;          /* last FP64 ||s - A zeta|| / ||s|| (true residual) */
    double recursive_residual;    /* last recursive ||r|| / ||s|| of the inner CG */
    double kernel_ms;             /* device time of the persistent solver launches, measured
                                     with events on the context stream (0 for TT_SOLVER_KERNELS) */
    int kernel_launches;          /* persistent solver launches (1 + replacements) */
    int fallback;                 /* TT_PRECOND_LEARNED: iteration at which the solve fell back
                                     to plain CG, or -1 */
} tt_solve_info;

/* Sizes of a configured system. */
typedef struct {
    int n, n_gs, pad_L, n_vs, n_slopes;
    int n_vphi;                   /* valid phase points (0 without a target) */
    int n_prime, proj_pad_L;      /* projection grid and FFT side (0 without a target) */
    int n_layer;
    size_t spectra_bytes_f32;     /* packed slope-slope spectra, FP32 copy */
    size_t spectra_bytes_f64;     /* packed slope-slope spectra, FP64 copy */
    size_t proj_spectra_bytes;    /* phase-slope spectra of the projection (FP32) */
} tt_system_info;

typedef struct tt_ctx tt_ctx;
typedef struct tt_kernels tt_kernels;
typedef struct tt_learned tt_learned;

/* Training of a learned preconditioner (tt_learned_train). */
typedef struct {
    int n_pairs;                  /* (residual, exact solution) pairs drawn, e.g. 20000 */
    int steps;                    /* optimiser steps */
    int batch;                    /* pairs per step */
    double lr;                    /* Adam step size; cosine decay to lr / 100 over the steps */
} tt_train_opts;

typedef struct {
    double objective_first;       /* training objective J at the first step */
    double objective_last;        /* mean J over the last tenth of the steps */
    double ms;                    /* device time of pair generation and training */
} tt_train_info;

/* Create a context on HIP device `device`, enqueuing on `stream` (a hipStream_t,
 * NULL = the null stream).  Owns its device memory until tt_destroy. */
tt_status tt_create(tt_ctx** out, int device, void* stream);
tt_status tt_destroy(tt_ctx* ctx);

/* A view of a configured context: it shares the base's system (spectra, index
 * maps, noise, twiddles, and the block-circulant preconditioner spectra if
 * already built) and owns its stream (`stream`, a hipStream_t, NULL = the null
 * stream), solver vectors and transform buffers.  Several frames of one system
 * solved together (tt_solve_batch over the base and its views with
 * TT_SOLVER_BATCHED: multiple right-hand sides, e.g. the columns of an offline
 * reconstructor) then stream one copy of the spectra.  A view has no target
 * (its solves take d_phi = NULL) and cannot set a system, noise blocks or mode
 * removal; the base can do none of these, and tt_destroy refuses it, while it
 * has live views.  Views of views are refused. */
tt_status tt_create_view(tt_ctx** out, tt_ctx* base, void* stream);

/* Valid-subaperture rule of the aperture masks (§2.F): subaperture (i, j) of
 * the n x n grid laid over [-D/2, D/2]^2 is valid when at least half of its
 * area lies inside the annular pupil of outer diameter D and inner diameter
 * obstruction * D (exact areas).  out: n*n bytes, row-major (1 valid, 0 not),
 * written on success; n_valid (may be NULL) receives the count.  Host only: no
 * device or context is needed.  TT_INVALID_ARG for n outside [1, 512], D <= 0,
 * obstruction outside [0, 1) or out == NULL. */
tt_status tt_pupil_mask(int n, double D, double obstruction, unsigned char* out, int* n_valid);

/* Covariance generation, FP64 on the device (App. A.2 Hudgin slope-slope
 * equations with the §2.D cone scaling).  For every
 * unordered guide-star pair g <= h and component xx, xy (= yx), yy it evaluates
 * the (2n-1)^2 unique elements of the 2RBT block Theta^{gh}_{pq} (§2.D):
 *   t(u, v) = sum_k w_k Hud_pq( s_k (u d, v d) + h_k (alpha_h - alpha_g); s_k d ),
 * u = column lag, v = row lag of the second slope relative to the first.
 * The result is owned by the library until tt_kernels_destroy. Synchronous. */
tt_status tt_generate_kernels(tt_ctx* ctx, const tt_geometry* geom,
                              const tt_atmosphere* atm, tt_kernels** out);
tt_status tt_kernels_destroy(tt_kernels* k);
/* Copy the tables to host memory: `count` doubles laid out as
 * [pair][component][v + n-1][u + n-1], pairs (g, h), g <= h, in row-major
 * order of g then h, components xx, xy, yy.  count must equal
 * n_gs (n_gs + 1) / 2 * 3 * (2n-1)^2.  Synchronous. */
tt_status tt_kernels_copy(const tt_kernels* k, double* host_out, size_t count);

/* Build the system (spectra and set-up): FP64 2-D real DFT of every embedded
 * table (K[(-u) mod L, (-v) mod L] = t(u, v)), packed per frequency as the
 * 2 n_gs x 2 n_gs Hermitian matrix of §2.E's per-frequency products (FP64 and
 * FP32 copies), the W_s index maps, the noise variance Sigma_eta = diag
 * (noise_var[i] if noise_var != NULL, else noise_scalar; §2.C, §2.F), and, if
 * target != NULL, the projection operators of §2.D/§2.E for that direction.
 * Replaces any previous system of the context.  Synchronous. */
tt_status tt_set_system(tt_ctx* ctx, const tt_kernels* k, const double* noise_var,
                        double noise_scalar, const tt_target* target);
tt_status tt_get_system_info(const tt_ctx* ctx, tt_system_info* out);

/* Elongated LGS spots (§2.F): make Sigma_eta 2x2 block diagonal by giving the
 * covariance of the x and y slope noise of every valid subaperture of every
 * sensor.  cov_xy: host array of n_gs * n_vs doubles, index g * n_vs + v
 * (v: valid subaperture in row-major order), copied; NULL removes the blocks.
 * Every block [[var_x, cov], [cov, var_y]] (variances from tt_set_system) must
 * be positive definite, else TT_INVALID_ARG and nothing changes.  Applies to
 * every later product and solve of the context until the next tt_set_system
 * (which removes the blocks).  The block-circulant preconditioner keeps using
 * the mean variance.  Persistent solvers need a block's grid rows to fit its
 * threads (as TT_PRECOND_CIRCULANT); TT_PRECOND_CIRCULANT with the blocks needs
 * TT_PREC_F32.  Synchronous. */
tt_status tt_set_noise_xy(tt_ctx* ctx, const double* cov_xy);

/* Low-order mode removal (§2.F "Mode removal"): with on != 0 the products and
 * solves use M_s W_s in place of W_s, M_s = block diagonal of the per-sensor
 * projectors I - Z Z^+ removing tip, tilt and focus (Hudgin slopes of the
 * phase modes x, y, x^2 + y^2 on the valid subapertures), i.e. the system
 * (M_s W_s)(Sigma_ss + Sigma_eta)(M_s W_s)^T zeta = M_s s with zeta in the
 * range of M_s (rel_residual is relative to ||M_s s||), and the projection
 * applies M_phi (the same modes at the valid phase points) to
 * W_phi Sigma_phi_s M_s zeta.  tt_matvec / tt_matvec_f64 then apply
 * M_s A M_s.  Solves need TT_SOLVER_KERNELS.  Cleared by tt_set_system;
 * on = 0 removes it.  Synchronous. */
tt_status tt_set_mode_removal(tt_ctx* ctx, int on);

/* y = W_s (Sigma_ss + Sigma_eta) W_s^T x, once, by the fused 2RBT product of
 * §2.E.  d_x, d_y: n_slopes elements; they must not overlap. */
tt_status tt_matvec(tt_ctx* ctx, const float* d_x, float* d_y);
tt_status tt_matvec_f64(tt_ctx* ctx, const double* d_x, double* d_y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the product of
 * tt_matvec, same kernels and bitwise the same result, with its transform work
 * buffers taken from a fixed device array of the library instead of the
 * context.  The call allocates and frees nothing.  The array holds 8 MiB per
 * device (kept until the process ends); a system needs
 * 2 (pad_L / 2 + 1) 2 n_gs n complex floats (each half rounded up to 256
 * bytes), plus n_slopes floats with mode removal: larger systems get
 * TT_INVALID_ARG with the sizes in tt_last_error (use tt_matvec).  The array's
 * address is looked up when a context is created on the device; TT_HIP_ERROR
 * if that failed.  Every call on one device shares the array: calls that
 * overlap in time on one device (several streams or threads) race and must be
 * ordered by the caller.  Asynchronous on the context's stream. */
tt_status tt_matvec_noalloc(tt_ctx* ctx, const float* d_x, float* d_y);

/* The same FP32 product for count independent systems in one call (the §2.E
 * product of each system, batched over systems): y_i = A_i x_i,
 * d_x[i], d_y[i] on systems[i] (n_slopes of that system each, device memory,
 * not overlapping).  The systems may differ in every size; each context appears
 * at most once, all are on one device, and none has mode removal on
 * (TT_INVALID_ARG otherwise; an unset context gives TT_NOT_READY).  Sizes are
 * limited by the column phase: with S = 2 if every pad_L is even, else 1,
 * (pad_L / S) * n_gs <= 2048 and the LDS of one column item, 4 (pad_L / S)
 * (3 n_gs^2 + 1) + 16 n_gs (pad_L / S) (twice that when pad_L / S is not a
 * power of two) + 8 max(pad_L) bytes, at most 160 KiB.
 * All work is enqueued on the stream of systems[0] (three launches: row
 * transforms, column transforms with the per-frequency products, inverse row
 * transforms), in the per-system work buffers of each context: order the call
 * after other work on those contexts.  Asynchronous unless phase_ms != NULL:
 * then the call waits and phase_ms[0..2] receive the durations (ms, HIP events)
 * of the three launches. */
tt_status tt_matvec_batch(tt_ctx* const* systems, int count, const float* const* d_x,
                          float* const* d_y, float* phase_ms);

/* tt_matvec_batch with the spectra read in `precision` storage: TT_PREC_F32
 * (the same as tt_matvec_batch), TT_PREC_F16 (each frequency's values scaled by
 * the power of two that brings its largest magnitude to [2^14, 2^15), rounded
 * to FP16, restored exactly) or TT_PREC_BF16 (rounded, unscaled); products and
 * transforms in FP32.  The FP16 / BF16 copies are made once per system from the
 * FP32 spectra at the first call that needs them (device memory: half the FP32
 * spectra).  Relative error of the product: the spectra rounding, at most 2^-11
 * (FP16) or 2^-8 (BF16) of each frequency's largest value.  split: the
 * frequency split of the column kernel (1, 2 or 4, see tt_tune_batch; the batch
 * must admit it), or 0 for the tuned or default one. */
tt_status tt_matvec_batch_prec(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y,
                               int precision, int split, float* phase_ms);

/* Autotuner of the batched column kernel.  The column items of the batched
 * product (op 0) and of the batched block-circulant preconditioner (op 1) each
 * own one of S classes of frequencies f1 = S k + h of a column; S trades LDS
 * per item (items resident per compute unit) against the inverse shares
 * written.  This times one call for each S in {1, 2, 4} that every system of
 * the batch admits (S divides L, L / 4 >= n / 2 for S = 4, LDS limits), on
 * seeded vectors with spectra stored in `precision` (TT_PREC_F32 / F16 / BF16),
 * 2 warm-up and 5 timed calls each, and keeps the fastest S for later
 * tt_matvec_batch(_prec) calls and batched solves with exactly these systems
 * in this order (stored in systems[0]).  best_split (may be NULL) receives it;
 * ms_per_split (3 floats, may be NULL) the mean call time in ms for S = 1, 2, 4
 * (-1: not admitted).  Synchronous; allocates two vectors per system for the
 * duration of the call. */
tt_status tt_tune_batch(tt_ctx* const* systems, int count, int op, int precision, int* best_split,
                        float* ms_per_split);

/* Solve W_s (Sigma_ss + Sigma_eta) W_s^T zeta = s by CG (§2.G) and,
 * if d_phi != NULL, project phi = W_phi Sigma_{phi_beta s} zeta (§2.E).
 * d_s: n_slopes floats; d_x0: n_slopes doubles (warm start) or NULL (zeta0 = 0);
 * d_zeta: n_slopes doubles (out); d_phi: n_vphi floats (out) or NULL.
 * opts NULL = tol 1e-6, max_iter 20000, TT_PREC_F32, persistent.
 * Waits for completion; info (may be NULL) receives the iteration counts and
 * the final FP64 true residual.  Returns TT_OK, TT_NOT_CONVERGED or TT_BREAKDOWN
 * (zeta = last iterate) or an argument / runtime error. */
tt_status tt_solve_frame(tt_ctx* ctx, const float* d_s, const double* d_x0,
                         double* d_zeta, float* d_phi, const tt_solve_opts* opts,
                         tt_solve_info* info);

/* A batch of frames, each on its own configured context (systems may differ
 * in size and geometry; contexts must not repeat).  For i < count, frame i is
 * tt_solve_frame(systems[i], d_s[i], d_x0 ? d_x0[i] : NULL, d_zeta[i],
 * d_phi ? d_phi[i] : NULL, opts, infos ? &infos[i] : NULL), in order, one
 * after another (each solve occupies the whole device) -- except with
 * opts->solver == TT_SOLVER_BATCHED, where all frames iterate together and
 * every context must be on one device (the work runs on the stream of
 * systems[0] and on each context's own stream, the call waits for both).
 * Returns TT_OK when
 * every frame did, else the first non-OK status in the order TT_BREAKDOWN,
 * TT_NOT_CONVERGED (all frames are still attempted and infos filled), or the
 * first argument / runtime error (later frames are then not attempted). */
tt_status tt_solve_batch(tt_ctx* const* systems, int count, const float* const* d_s,
                         const double* const* d_x0, double* const* d_zeta, float* const* d_phi,
                         const tt_solve_opts* opts, tt_solve_info* infos);

/* phi = W_phi sum_k I'_k S2 F^-1 { sum_q Xi'~_{q,k} . F[S1 zeta_q] }
 * (§2.E LGS phase-slope equation with a common n').  d_zeta: n_slopes doubles
 * (rounded to FP32 for the products), d_phi: n_vphi floats.  Requires a target. */
tt_status tt_project(tt_ctx* ctx, const double* d_zeta, float* d_phi);

/* Learned preconditioner.  The paper leaves preconditioning of its Toeplitz
 * system open (§2.G; the conclusion names it the remaining challenge); this is
 * a factorised approximate inverse P = K^T K learned from the method's own
 * (residual, exact solution) pairs.  K is a four-layer linear convolutional
 * network over the 2 n_gs slope maps of the n x n grid (W_s^T r, zeros at
 * invalid subapertures, §2.F): 3 x 3 kernels, channels 2 n_gs -> hidden ->
 * hidden -> hidden -> 2 n_gs, zero padding, no bias, output restricted to the
 * valid subapertures.  Weights are masked so that K is lower triangular in the
 * order (pixel in row-major order, then channel): no tap on the next row or on
 * the next pixel of the row; the centre tap from input channel i to output o
 * only when deg(o) >= deg(i) (channel c of the slope maps has degree c, hidden
 * channel h degree h mod 2 n_gs).  Then log|det K| = n_vs sum_c log|d_c|, d the
 * diagonal of the product of the four centre taps, and training minimises
 * Kaporin's condition number of P A through
 *   J = N log(t / N) - 2 n_vs sum_c log|d_c|,   t = mean_b (K r_b).(K e_b),
 * N = n_slopes, over pairs r_b = A e_b with e_b ~ N(0, I) (E[t] = tr(K A K^T)).
 * Weights are FP32 masters (Adam); the network computes with them rounded to
 * bfloat16, FP32 accumulation on the matrix cores.
 *
 * Weight layout (count from tt_learned_weight_count): the four layers in
 * order, each [out][in][ky][kx] (ky: row offset - 1, kx: column offset - 1 of
 * the input read by output (y, x)), row-major. */
tt_status tt_learned_create(tt_learned** out, int device, int n_gs, int hidden, unsigned long long seed);
tt_status tt_learned_destroy(tt_learned* net);
tt_status tt_learned_weight_count(const tt_learned* net, size_t* count);
/* FP32 master weights (masked entries are zero); set_weights masks what it is
 * given and resets the optimiser state.  Synchronous. */
tt_status tt_learned_get_weights(const tt_learned* net, float* host, size_t count);
tt_status tt_learned_set_weights(tt_learned* net, const float* host, size_t count);
/* d_z = K^T K d_r on the geometry of ctx (n_slopes floats each), on ctx's stream. */
tt_status tt_learned_apply(tt_learned* net, tt_ctx* ctx, const float* d_r, float* d_z);
/* One optimiser step on caller pairs: d_R, d_E device arrays of batch rows of
 * n_slopes floats (r_b = A e_b).  objective, trace (may be NULL) receive J and t
 * at the weights used.  Synchronous.  TT_BREAKDOWN (step skipped) if t <= 0 or
 * a diagonal entry of K is zero. */
tt_status tt_learned_train_step(tt_learned* net, tt_ctx* ctx, const float* d_R, const float* d_E, int batch,
                                double lr, double* objective, double* trace);
/* Training on opts->n_pairs pairs drawn by the library (e ~ N(0, I) from a
 * Philox4x32-10 stream under the network's seed, r = A_j e by the FP32 product
 * of systems[j], j = pair mod count; the systems must share the grid and the
 * valid subapertures, and may differ in atmosphere and noise), then opts->steps
 * Adam steps on batches drawn by a counter-based hash.  Synchronous; the pairs
 * (2 n_pairs n_slopes floats of device memory) are freed on return. */
tt_status tt_learned_train(tt_learned* net, tt_ctx* const* systems, int count, const tt_train_opts* opts,
                           tt_train_info* info);
/* Attach (net != NULL) or detach the network used by TT_PRECOND_LEARNED solves
 * of ctx.  The network is not owned by the context and must outlive its use. */
tt_status tt_set_learned(tt_ctx* ctx, tt_learned* net);

const char* tt_status_string(tt_status s);
/* Message of the last failing call on the calling thread ("" if none). */
const char* tt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TT_H */
