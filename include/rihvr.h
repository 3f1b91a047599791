/*
 * rihvr.h - C ABI of the MI355X regularized inverse holographic volume
 * reconstruction library (Mallery & Hong, "Regularized Inverse Holographic
 * Volume Reconstruction for 3D Particle Tracking").
 *
 * The library solves, for one hologram b of ny x nx pixels, the problem of the
 * paper's Eq. (2) with the fused-lasso regulariser of Eq. (5) and a
 * non-negativity constraint:
 *
 *     min_x  1/2 ||A x - b||^2 + l1 * sum(x) + tv * TV3D(x),   x >= 0,
 *
 * where x is a real volume of nz planes and A is the linearised hologram
 * formation model (section "Methodology"): angular-spectrum propagation of
 * every plane j to the sensor and a sum over planes,
 *
 *     A x = Re( sum_j IFFT2( FFT2(x_j) . H_j ) ),
 *     H_j(f) = exp(i 2 pi z_j sqrt(1/lambda^2 - fx^2 - fy^2)),  z_j = z0 + j dz,
 *
 * with an unscaled forward and 1/(nx ny)-scaled inverse DFT on the fftfreq
 * grid.  TV3D is the isotropic total variation of Eq. (4) taken over forward
 * differences along x, y and z (last difference on each axis zero).
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers to C-contiguous arrays whose element
 *     type is the plan's dtype (float32 for RI_F32, float64 for RI_F64):
 *     volumes are [nz][ny][nx], holograms [ny][nx] (x fastest).
 *   - The caller owns every buffer.  The library allocates device memory only
 *     in ri_plan_create (phase and twiddle tables, a small state block) and
 *     frees it in ri_plan_destroy; the hot path never allocates.  Scratch space
 *     comes from the caller through (ws, ws_bytes); query ri_workspace_size.
 *   - Calls are asynchronous and ordered on `stream` (a hipStream_t, NULL for
 *     the default stream), except where stated.  A plan, and the workspace
 *     handed to it, may be used by one stream at a time.
 *   - Every call validates its arguments before launching anything and returns
 *     a status; on failure nothing has been launched and ri_last_error() holds
 *     a thread-local message.  HIP runtime failures map to RI_ERR_HIP.
 *   - Supported sizes: nx and ny of the form 2^a or 3 * 2^a, 16 <= nx <= 2048,
 *     16 <= ny <= 2048; nz >= 1.
 */
#ifndef RIHVR_H
#define RIHVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RI_OK = 0,
  RI_ERR_INVALID_ARG = 1,        /* null pointer, bad value, aliasing not allowed */
  RI_ERR_UNSUPPORTED_SIZE = 2,   /* nx / ny outside the supported set */
  RI_ERR_OUT_OF_MEMORY = 3,      /* plan tables could not be allocated */
  RI_ERR_WORKSPACE_TOO_SMALL = 4,
  RI_ERR_HIP = 5,                /* HIP runtime error; see ri_last_error */
  RI_ERR_NONFINITE = 6,          /* the objective became NaN / Inf during a solve */
  RI_ERR_NOT_CONVERGED = 7       /* the objective diverged (grew past 10x F(x0)) */
} ri_status;

/* Element type of a plan's arrays (every volume, hologram and spectrum argument).
 * RI_F32: the fast path (FP32 data, FP64 phase reduction and accumulations).
 * RI_F64: every array is double and every step computes in double, for telling
 * defects from FP32 rounding (it agrees with the FP64 reference to ~1e-12):
 * the same model from the same FP64 tables, but with plain complex transforms
 * of whole planes (every plane's spectrum held in the workspace), the
 * gradient-projection prox one step per two passes over memory, and the FISTA
 * scalars, objective and stop tests on the host (ri_solve synchronises once
 * per outer iteration when a gap stop or the restart needs the objective, and
 * evaluates the objective of the returned iterate for the report; no graph,
 * no row skipping, report.phase_ms stays 0).  RI_F64 plans take neither
 * RI_TV_FGP nor RI_TV_DUAL_BF16; ri_forward_noalloc, ri_solve_batched,
 * ri_plan_autotune, row stores and RI_SOLVE_DUAL_WARM reject them
 * (RI_ERR_INVALID_ARG). */
typedef enum { RI_F32 = 0, RI_F64 = 1 } ri_dtype;

/* Geometry flags */
#define RI_NO_CARRIER 0x1u  /* drop the exp(i 2 pi z / lambda) carrier from H_j */
#define RI_TV2D       0x2u  /* regularise with the per-plane 2D TV of Eq. (4) (the paper's
                               own regulariser: no differences across planes, GP step
                               1/(8 tau), a dual of two components) instead of TV3D */
#define RI_TV_FGP     0x4u  /* inner solver: the accelerated dual iteration (FGP of Beck and
                               Teboulle) instead of plain gradient projection; one dual
                               step per pass over memory, two duals per set in the workspace */
#define RI_TV_DUAL_BF16 0x8u /* keep the TV dual in bfloat16 between passes over memory (the
                               arithmetic stays FP32; the dual's bytes halve) */
#define RI_COMPLEX    0x10u /* complex-valued object (absorption and phase; section
                               "Methodology": the volume is stored as complex values and
                               Eq. (8) shrinks the modulus).  Every volume argument (x, v,
                               x_out, x_inout, A^T y) is then [2][nz][ny][nx] FP32: the real
                               parts of the nz planes, then their imaginary parts.  A x =
                               Re(sum_j IFFT2(FFT2(x_j) H_j)) and its adjoint under the real
                               inner product; ||x||_1 = sum |x_i|; TV(x) = sum over voxels of
                               sqrt(sum_d |D_d x|^2) (the modulus of complex differences, 3D
                               or with RI_TV2D per plane); prox = (1 - t l1/|u|)_+ u of the
                               complex TV prox u, computed by gradient projection on a
                               complex dual (one complex value per direction, projected
                               jointly), one step per two passes over memory.  ||A||^2 = nz.
                               nonneg must be 0.  Not combinable with RI_TV_FGP or
                               RI_TV_DUAL_BF16; ri_solve rejects RI_SOLVE_DUAL_WARM and row
                               stores, ri_solve_batched and ri_plan_autotune reject the plan
                               (RI_ERR_INVALID_ARG). */

typedef struct {
  int32_t nx, ny, nz;       /* hologram width, height; number of planes */
  double pixel_um;          /* lateral pixel pitch, micrometres */
  double wavelength_um;     /* illumination wavelength, micrometres */
  double z0_um, dz_um;      /* plane j at z0 + j*dz from the sensor */
  uint32_t flags;           /* RI_NO_CARRIER | RI_TV2D | RI_TV_FGP | RI_TV_DUAL_BF16 | RI_COMPLEX */
} ri_geometry;

/* Fused-lasso proximal operator settings (Eq. 5, Eq. 6). */
typedef struct {
  double l1;                /* l1 weight */
  double tv;                /* total-variation weight */
  int32_t inner_iters;      /* gradient-projection steps on the TV dual, >= 0 */
  int32_t nonneg;           /* 1: x >= 0 (soft threshold max(u - t l1, 0)); 0: signed */
} ri_prox_params;

/* Solve settings */
#define RI_INIT_ZERO  0     /* start from x0 = 0 */
#define RI_INIT_GIVEN 1     /* start from the contents of x_inout */

#define RI_SOLVE_DENSE    0x1u  /* do not skip empty rows / planes in A */
#define RI_SOLVE_NO_GRAPH 0x2u  /* launch kernels one by one instead of replaying a HIP graph */
#define RI_SOLVE_RESTART  0x4u  /* function-value restart of the momentum: s = 1, beta = 0 after an
                                   iterate whose objective rose (a FISTA variant; reference runs) */
#define RI_SOLVE_TIMING   0x8u  /* time each phase with HIP events (report.phase_ms) */
#define RI_SOLVE_DUAL_WARM 0x10u /* every prox starts its TV dual from the dual the previous
                                    outer iteration ended with (zero for the first) instead of
                                    from zero: an inexact inner solve that improves across
                                    outer iterations */
#define RI_SOLVE_GROUPED  0x20u /* ri_solve_batched (params[0].flags): launch each TV pass with
                                   one block per tile of every frame instead of the default
                                   persistent kernels (one block per compute unit taking the
                                   frames' tiles from a device work queue); the same results bit
                                   for bit.  No effect on ri_solve */

typedef struct {
  double l1, tv;            /* regularisation weights */
  int32_t max_iters;        /* outer FISTA iterations (upper bound) */
  int32_t inner_iters;      /* TV dual steps per outer iteration */
  double gap_tol;           /* stop once (F(x_k) - f_ref) / |f_ref| <= gap_tol ... */
  double f_ref;             /* ... when f_ref > 0; otherwise run max_iters */
  int32_t init;             /* RI_INIT_ZERO | RI_INIT_GIVEN */
  int32_t check_every;      /* host reads the device stop flag every this many iterations (>= 1) */
  uint32_t flags;           /* RI_SOLVE_* */
  int32_t nonneg;           /* 1: x >= 0 (the problem above); 0: signed soft threshold */
  double x0_scale;          /* RI_INIT_GIVEN: start from x0_scale * x_inout (scaled in place);
                               0 is read as 1; must be finite and >= 0 */
} ri_solve_params;

#define RI_NUM_PHASES 6     /* forward, hologram, adjoint, prox, objective, other */

typedef struct {
  int32_t iters;            /* outer iterations performed (prox applications) */
  int32_t converged;        /* 1 if the gap criterion was met */
  double objective;         /* F of the returned iterate (FP64 accumulation) */
  double objective_min;     /* smallest F over the evaluated iterates */
  double gap;               /* (objective - f_ref) / f_ref, or NaN if f_ref <= 0 */
  double lipschitz;         /* ||A||^2 used for the step t = 1/||A||^2 */
  double empty_plane_frac;  /* of the returned iterate */
  double empty_row_frac;    /* of the returned iterate */
  double phase_ms[RI_NUM_PHASES]; /* with RI_SOLVE_TIMING: device time per phase */
  int32_t phase_launches[RI_NUM_PHASES];
  int32_t store_rows_peak;  /* row stores: most occupied rows of any iterate (also
                               when a pool ran out); 0 with dense iterates */
} ri_solve_report;

typedef struct ri_plan ri_plan;

/* Workspace queries */
typedef enum { RI_OP_FORWARD = 0, RI_OP_ADJOINT = 1, RI_OP_PROX = 2, RI_OP_SOLVE = 3, RI_OP_AUTOTUNE = 4 } ri_op;

/*
 * Launch shape of a plan (no effect on what is computed; FP32 rounding of the
 * forward's plane sums depends on col_blocks).  Defaults: 3, 1536, 512.
 *   tv_levels   dual steps fused into one pass of the TV prox (2, 3 or 4): a
 *               pass streams the volume once, so fewer passes read less, but
 *               each pass recomputes a wider halo and uses more registers.
 *   tv_blocks   blocks per TV pass the z-range is cut for (64 .. 65536;
 *               chunks keep at least 16 planes).
 *   col_blocks  blocks of the per-plane column transforms of A and A^T the
 *               z-range is cut for (16 .. 8192).  More chunks mean more
 *               partial spectra: ri_workspace_size grows with it.
 */
typedef struct {
  int32_t tv_levels;
  int32_t tv_blocks;
  int32_t col_blocks;
} ri_tuning;

/*
 * Create a plan for one geometry and element type on the current HIP device
 * (the angular-spectrum model of section "Methodology"; the step of Eq. 7
 * is 1/||A||^2): FP64 phase table
 * theta(f) = sqrt(1/lambda^2 - f^2) - 1/lambda, per-plane carrier phases
 * frac(z_j / lambda), FFT twiddles, and the Lipschitz constant
 * ||A||^2 = max_f sum_j cos^2(2 pi z_j sqrt(1/lambda^2 - f^2)) (the spectrum of
 * A A^T; the FISTA step is 1/||A||^2).  Synchronous.  *out receives the plan.
 */
ri_status ri_plan_create(const ri_geometry* geometry, ri_dtype dtype, ri_plan** out);
ri_status ri_plan_destroy(ri_plan* plan);
/* ||A||^2 of the plan (host value). */
ri_status ri_plan_lipschitz(const ri_plan* plan, double* out);
/* Bytes of scratch space that suffice for every entry point taking this plan
 * (forward, adjoint, prox, solve and autotune) with its current tuning. */
ri_status ri_workspace_size(const ri_plan* plan, size_t* bytes);
/* The smaller amount that the one entry point `op` needs. */
ri_status ri_workspace_size_op(const ri_plan* plan, ri_op op, size_t* bytes);

/*
 * Tuning of a plan.  ri_plan_set_tuning validates every field (RI_ERR_INVALID_ARG
 * otherwise, plan unchanged) and drops the plan's cached solve graph; the
 * workspace sizes of RI_OP_FORWARD, RI_OP_ADJOINT and RI_OP_SOLVE may change.
 */
ri_status ri_plan_get_tuning(const ri_plan* plan, ri_tuning* out);
ri_status ri_plan_set_tuning(ri_plan* plan, const ri_tuning* tuning);

/*
 * Storage of the solver's iterates (section "Methodology", the paragraph on
 * storing the sparse particle volume; the paper keeps x_k as coordinate lists
 * per plane).  row_fraction = 0 (the default): x_k, x_{k-1} and x_{k+1} are
 * dense volumes (two in the workspace, one in x_inout).  row_fraction in
 * (0, 1]: the iterates live in two row stores (x_k in one; x_{k-1} in the
 * other until the gradient step has read it, then x_{k+1}), each a pool of
 * max(1, ceil(row_fraction * ny * nz - 1e-6)) rows of nx FP32 values plus a table of
 * ny * nz int32 slots (-1: the row is all zero), and x_inout holds the dense
 * gradient-step output during the solve.  The workspace of RI_OP_SOLVE (and of
 * ri_workspace_size_batched) then holds 2 * row_fraction volumes of iterates
 * instead of 2.  A row takes a pool row exactly when it holds a non-zero value,
 * so a fraction at least that of the occupied rows of every iterate (and of a
 * given x_0) always fits; the report's store_rows_peak gives that count.  Results are bit-identical to the dense storage.  An
 * iterate with more occupied rows than a pool holds stops the solve with status
 * RI_ERR_WORKSPACE_TOO_SMALL (returned by ri_solve when a report is requested;
 * x_inout then holds no valid result).  Not available with RI_TV_DUAL_BF16
 * plans (RI_ERR_INVALID_ARG from ri_solve).  ri_forward, ri_adjoint, ri_prox
 * and ri_plan_autotune are unaffected.  Drops the plan's cached solve graph.
 * RI_ERR_INVALID_ARG for a fraction outside [0, 1] or NaN.
 */
ri_status ri_plan_set_storage(ri_plan* plan, double row_fraction);

/*
 * The paper regularises each plane with its own 2D TV and computes the prox
 * one plane at a time, so that its dual needs the memory of one plane (section
 * "Methodology", the paragraph after Eq. 8).  For RI_TV2D plans, planes > 0
 * makes the prox (ri_prox_fused_lasso and inside ri_solve) run on groups of
 * `planes` planes in turn, each group taking all its dual steps before the
 * next starts, with the dual sets of the workspace holding `planes` planes
 * instead of nz (the dual shrinks from 4 volumes to 4 planes/nz of one).
 * Results are bit-identical to planes = 0 (the planes do not interact); the
 * solver's objective sums the same terms in another grouping (within FP64
 * rounding).  RI_ERR_INVALID_ARG for planes < 0, for planes > 0 on a plan
 * without RI_TV2D, with RI_TV_FGP, RI_COMPLEX or RI_F64; ri_solve rejects
 * RI_SOLVE_DUAL_WARM and row stores with a plane-group dual, ri_solve_batched
 * such plans.  Drops the plan's cached solve graph; changes the workspace
 * sizes of RI_OP_PROX, RI_OP_SOLVE and RI_OP_AUTOTUNE.
 */
ri_status ri_plan_set_dual_planes(ri_plan* plan, int32_t planes);
ri_status ri_plan_get_dual_planes(const ri_plan* plan, int32_t* planes);
ri_status ri_plan_get_storage(const ri_plan* plan, double* row_fraction);

typedef struct {
  ri_tuning best;           /* the tuning now set on the plan */
  int32_t from_cache;       /* 1: taken from the cache file, nothing was timed */
  int32_t cache_written;    /* 1: the cache file was updated; -1: writing it failed */
  int32_t candidates;       /* launch shapes timed */
  double default_ms;        /* forward + adjoint + prox of one iteration, default tuning */
  double best_ms;           /* the same with the chosen tuning */
  double tune_ms;           /* wall time of the call */
} ri_autotune_report;

/*
 * Choose the plan's tuning by timing its kernels on the device: the column
 * transforms of A and A^T for each distinct col_blocks chunking, and one TV
 * prox of `inner_iters` dual steps for each distinct (tv_levels, tv_blocks)
 * grid, on zero-filled data in the workspace (ri_workspace_size(RI_OP_AUTOTUNE)
 * bytes, contents overwritten), then set the fastest.  The choice is keyed by
 * device name, compute-unit count, nx, ny, nz and inner_iters; with a non-NULL
 * `cache_path` (a text file of one JSON object per line) a matching entry is
 * used without timing, and a new choice is added to the file (rewritten
 * through a temporary file and a rename).  Synchronises `stream`.  `report`
 * is nullable.
 */
ri_status ri_plan_autotune(ri_plan* plan, int32_t inner_iters, const char* cache_path, void* ws,
                           size_t ws_bytes, void* stream, ri_autotune_report* report);

/*
 * b_out = A x, the linearised hologram formation of section "Methodology"
 * (the operator inside the data term of Eq. 2): every plane propagated to the
 * sensor by the angular spectrum and summed.  x: volume [nz][ny][nx]; b_out:
 * hologram [ny][nx].  Exact in every voxel (no sparsity skipping on this
 * entry point).  x and b_out must not overlap.
 */
ri_status ri_forward(ri_plan* plan, const void* x, void* b_out,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * b_out = A x as ri_forward computes it (same kernels, same result), for
 * callers that cannot allocate device memory or hand over a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The scratch space lives in a fixed device array of
 * ri_forward_noalloc_max_scratch() bytes (64 MiB) that each device the library
 * runs on holds until the process ends; the call allocates nothing.  Sizes
 * whose forward needs more scratch than that (ri_workspace_size_op with
 * RI_OP_FORWARD, e.g. above about 512 x 512 x 64 planes) return
 * RI_ERR_UNSUPPORTED_SIZE.  All calls on one device share the array: calls
 * that overlap in time on one device (two streams, two threads) race.
 */
ri_status ri_forward_noalloc(ri_plan* plan, const void* x, void* b_out, void* stream);
size_t ri_forward_noalloc_max_scratch(void);

/*
 * x_out = A^T y, the back-propagation (A^T y)_j = Re(IFFT2(FFT2(y) . conj(H_j))):
 * the adjoint of the model of section "Methodology", which the gradient
 * A^T (A x - b) of the data term of Eq. 2 needs in the shrinkage step of
 * Eq. 7.  y: hologram [ny][nx]; x_out: volume [nz][ny][nx].  Must not overlap.
 */
ri_status ri_adjoint(ri_plan* plan, const void* y, void* x_out,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * x_out = prox of step*(l1 ||.||_1 + tv TV3D(.)) [restricted to x >= 0] at v,
 * the proximal operator of Eq. (6) for the fused lasso of Eq. (5): the TV prox
 * at weight tau = step*tv by `inner_iters` gradient-projection steps on its
 * dual (Beck & Teboulle; step 1/(12 tau), dual started at zero), followed by
 * the soft threshold at step*l1.  v and x_out are volumes [nz][ny][nx]; they
 * may be the same buffer (in place).
 */
ri_status ri_prox_fused_lasso(ri_plan* plan, const ri_prox_params* params, double step,
                              const void* v, void* x_out,
                              void* ws, size_t ws_bytes, void* stream);

/*
 * FISTA solve (section "Methodology": Eq. 2 with the fused lasso of Eq. 5,
 * shrinkage step Eq. 7 with the prox of Eq. 6 / Eq. 8, then the accelerated
 * update from the previous estimate) of the problem above with constant step
 * 1/||A||^2:
 *   x_k = prox(y_k - t A^T (A y_k - b)),  s_{k+1} = (1 + sqrt(1 + 4 s_k^2)) / 2,
 *   y_{k+1} = x_k + ((s_k - 1)/s_{k+1}) (x_k - x_{k-1}),
 * from x_0 = 0 or the given x_inout.  b: hologram [ny][nx]; x_inout: volume
 * [nz][ny][nx], overwritten with the returned iterate.  With f_ref > 0 the solve
 * stops at the first iterate whose objective gap is <= gap_tol (checked on the
 * device after every iteration; the host polls every check_every iterations).
 * If `report` is non-NULL the call synchronises the stream once at the end and
 * fills it; otherwise it returns after enqueueing (the host still polls the stop
 * flag when f_ref > 0).
 */
ri_status ri_solve(ri_plan* plan, const ri_solve_params* params, const void* b, void* x_inout,
                   void* ws, size_t ws_bytes, void* stream, ri_solve_report* report);

/*
 * Batched solve of n independent holograms that may differ in size and plane
 * count (one plan per frame): each frame is the FISTA solve of ri_solve
 * (section "Methodology", Eq. 2, 5, 7), as for the time series of holograms
 * the paper reconstructs for particle tracking (section "Synthetic Turbulent
 * Flow").  RI_F32 plans only.  Frames advance in lock-step, one outer
 * iteration for all frames at a time, each with its own step, momentum,
 * objective and stop flag; a frame that has met its criterion does no further
 * work.  Each kernel of an iteration is launched once per transform size (or
 * once for all frames); the TV passes, most of the time of an iteration, run
 * as persistent kernels of one block per compute unit that take the frames'
 * tiles from a device work queue (RI_SOLVE_GROUPED: one block per tile
 * instead).  One iteration of all frames is replayed as a HIP graph (unless
 * params[0].flags has RI_SOLVE_NO_GRAPH).  The workspace must
 * hold ri_workspace_size_batched() bytes.  params[i], b[i], x_inout[i] and
 * reports[i] (nullable array; filled after one synchronisation) belong to
 * frame i.  The x_inout volumes must not overlap each other, any b or ws.
 * Each frame runs with its own plan's tuning (TV passes are grouped by
 * tv_levels), so its result equals that of ri_solve with the same plan.
 */
ri_status ri_workspace_size_batched(int32_t n, ri_plan* const* plans, const ri_solve_params* params,
                                    size_t* bytes);
ri_status ri_solve_batched(int32_t n, ri_plan* const* plans, const ri_solve_params* params,
                           const void* const* b, void* const* x_inout,
                           void* ws, size_t ws_bytes, void* stream, ri_solve_report* reports);

/*
 * Learned warm start: a 3D U-Net proposes x_0 for ri_solve (RI_INIT_GIVEN).
 * The paper has no learned component; the network only changes where FISTA
 * starts, and the solve's objective still decides the result.
 *
 * Architecture: `levels` resolution levels with base * 2^l channels; per
 * level two 3x3x3 convolutions + ReLU, 2x2x2 max pooling down, 2x2x2 stride-2
 * transposed convolutions up, skip concatenation [up, skip], a 1x1x1 head and
 * a final ReLU (x_0 >= 0).  Activations and packed weights are BF16, matrix
 * products accumulate in FP32 on the matrix cores; the parameters and the Adam
 * moments are FP32 device arrays of ri_unet_param_count() floats, ordered
 * layer by layer (encoder levels 0..L-1: conv a, conv b; decoder levels
 * L-2..0: up, conv a, conv b; head), each layer weights then bias; conv
 * weights [kz][ky][kx][cin][cout], up weights [dz][dy][dx][cin][cout], head [cin].
 * Volumes are FP32 [d][h][w] device arrays; d, h, w must be multiples of
 * 2^(levels-1).  The network input is scale * in (the back-propagated
 * hologram A^T b, scaled by 1/||A||^2).  Workspaces come from the caller.
 */
typedef struct {
  int32_t levels;   /* 1..6 */
  int32_t base;     /* channels of level 0: 8, 16, 32, 64 or 128; base * 2^(levels-1) <= 128 */
} ri_unet_config;

ri_status ri_unet_param_count(const ri_unet_config* cfg, size_t* count);
/* He-normal weights from a seeded generator, biases 0.01; the head's weights
 * start at zero.  Synchronous. */
ri_status ri_unet_init_params(const ri_unet_config* cfg, uint64_t seed, float* params, void* stream);
ri_status ri_unet_workspace_size(const ri_unet_config* cfg, int32_t d, int32_t h, int32_t w, int32_t training,
                                 size_t* bytes);
/* out = network(scale * in). */
ri_status ri_unet_forward(const ri_unet_config* cfg, const float* params, const float* in, float scale, float* out,
                          int32_t d, int32_t h, int32_t w, void* ws, size_t ws_bytes, void* stream);
/*
 * One training step on one volume: forward, weighted mean-squared-error loss
 * (1/n) sum_v w_v (z_v - target_v)^2 on the head's pre-activation z (the
 * final ReLU applies at inference only, so voxels below zero still learn),
 * with w_v = pos_weight where target_v > 0 and 1 elsewhere (sparse targets;
 * pos_weight = 1 is the plain MSE; must be finite and > 0), written to
 * *loss_out (a device float) if non-NULL; backward into `grads`; then, if
 * lr > 0, an Adam update (beta 0.9 / 0.999, eps 1e-8, bias correction with
 * `step` >= 1) of params, adam_m, adam_v.
 */
ri_status ri_unet_train_step(const ri_unet_config* cfg, float* params, float* grads, float* adam_m, float* adam_v,
                             int32_t step, float lr, const float* in, float scale, const float* target,
                             float pos_weight, int32_t d, int32_t h, int32_t w, float* loss_out, void* ws,
                             size_t ws_bytes, void* stream);

/*
 * Particle tracking back end (section "Methodology", segmentation paragraph;
 * section "Synthetic Turbulent Flow": weighted centroids of connected
 * components, tracking by the method of Crocker & Grier with a maximum
 * displacement per frame and a minimum track duration).  All arrays are
 * device arrays; counts that the previous step produces stay on the device
 * (int32 pointers), so a whole frame's detection, linking and track update
 * run without a host synchronisation.
 */
typedef struct {
  double rel_threshold;     /* foreground: x > rel_threshold * max(x); the paper uses 1/256 (2/256) */
  int32_t min_voxels;       /* keep objects of at least this many voxels; the paper uses 5 */
} ri_detect_params;

/* One detected object: intensity-weighted centroid (voxel units, z y x),
 * intensity sum, voxel count and its smallest linear voxel index (the order
 * of the object table). */
typedef struct { double z, y, x, weight, voxels, first; } ri_object;

/* Workspace of ri_detect: a 32-bit label per voxel plus per-component sums for
 * up to max_components connected components (before the minimum-volume
 * filter).  Volumes up to 2^31 voxels. */
ri_status ri_detect_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t max_components, size_t* bytes);
/*
 * Segment the volume x [nz][ny][nx] (float32, device): foreground voxels
 * x > rel_threshold * max(x) (compared in FP64), 26-connected components,
 * objects of at least min_voxels voxels with their weighted centroids,
 * written to objects[0 .. counts[0]) in order of their smallest linear voxel
 * index.  counts (device int32[2]) receives the number of kept objects and
 * the number of components; objects beyond max_objects and components beyond
 * max_components are not written (the counts still tell).  Asynchronous.
 */
ri_status ri_detect(const ri_detect_params* params, const float* x, int32_t nx, int32_t ny, int32_t nz,
                    ri_object* objects, int32_t max_objects, int32_t* counts, int32_t max_components,
                    void* ws, size_t ws_bytes, void* stream);

ri_status ri_link_workspace_size(int32_t max_prev, int32_t max_cur, size_t* bytes);
/*
 * Crocker-Grier linking of the objects of two successive frames: *n_prev
 * objects in prev, *n_cur in cur (device counts, e.g. counts[0] of
 * ri_detect).  Distances are physical: the coordinate differences are scaled
 * by spacing[3] (z, y, x; host array).  Within each subnetwork of candidate
 * links (distance <= max_disp) the links minimise sum(d^2) + max_disp^2 *
 * (unlinked objects of prev), each object linked at most once; among equal
 * minima the first in a fixed enumeration order wins (sources ascending,
 * candidates by increasing distance then index, "unlinked" last).
 * link[i] (device int32[max_prev]) = index in cur or -1.  *status (device
 * int32): 0, or bit 0 set if a subnetwork had more than 8 sources (its links
 * are left at -1), bit 1 set if a source had more than 8 candidates (the
 * nearest 8 were used).
 */
ri_status ri_link(const ri_object* prev, const int32_t* n_prev, int32_t max_prev, const ri_object* cur,
                  const int32_t* n_cur, int32_t max_cur, const double spacing[3], double max_disp,
                  int32_t* link, int32_t* status, void* ws, size_t ws_bytes, void* stream);
/*
 * Track ids of the current frame: an object linked from the previous frame
 * takes its source's id (ids_prev), the others open new ids *next_id,
 * *next_id + 1, ... in ascending object order; track_len[id] grows by one for
 * every id present (ids >= max_tracks are not counted).  For the first frame
 * pass *n_prev = 0 (link and ids_prev may then be NULL).  track_len and
 * *next_id start at zero (device memory the caller clears).
 */
ri_status ri_track_update(const int32_t* link, const int32_t* n_prev, const int32_t* ids_prev,
                          const int32_t* n_cur, int32_t max_cur, int32_t* ids_cur, int32_t* next_id,
                          int32_t* track_len, int32_t max_tracks, void* stream);
/* kept[t] = 1 for tracks of at least min_len frames (t < *n_tracks); *n_kept their number. */
ri_status ri_track_filter(const int32_t* track_len, const int32_t* n_tracks, int32_t max_tracks, int32_t min_len,
                          uint8_t* kept, int32_t* n_kept, void* stream);

const char* ri_status_string(ri_status status);
const char* ri_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RIHVR_H */
