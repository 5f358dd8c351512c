/*
 * lrstv.h -- C ABI of the MI355X (gfx950) LRSTV ADMM library.
 *
 * The library runs the per-iteration ADMM sweep of the LRSTV / TDLRSTV
 * hyperspectral denoiser (Zeng et al., "Low-rank Meets Sparseness",
 * Sec. III-C, Algorithm 1) at full Tucker rank, for a batch of cubes of
 * possibly different sizes.  Model: the observed cube Y (the paper's O) is
 * split as Y = X + S + N with X the denoised cube (the paper's L), S sparse
 * noise and N = Y - X - S the remaining Gaussian part, by minimising
 *     2 tau ||D_w X||_1 + alpha sum_n TNN(w_n D_n X) + lambda ||S||_1
 * subject to Y = X + S (the factor 2 on tau is the weight for which the
 * paper's printed F-step threshold tau/mu is the exact block minimiser), or
 * with the isotropic term 2 tau sum_v ||(D_w X)_v||_2 (lrstv_params.tv).
 *
 * Conventions shared by every call
 *   - Return value: 0 = success, > 0 = warning with valid outputs,
 *     < 0 = error (outputs undefined).  lrstv_last_error() gives a message.
 *   - Every float* / double* argument documented as "device" is a pointer
 *     to GPU memory of the current HIP device; "host" pointers are CPU memory.
 *   - A cube is FP32, band-major [b][h][w] with w fastest (a contiguous
 *     torch tensor of shape (b, h, w)).  A batch of cubes is packed back to
 *     back in one buffer: cube c starts at element sum_{c' < c} b h w.
 *   - All GPU work is enqueued asynchronously on the caller's stream
 *     (a hipStream_t passed as void*); only calls documented as
 *     synchronising wait for it.
 *   - The library never allocates device memory in the solver calls: the
 *     caller provides a workspace of at least lrstv_workspace_size() bytes
 *     that outlives the handle.  A handle is not thread-safe; separate
 *     handles are independent.
 *   - Nothing throws across the ABI.
 */
#ifndef LRSTV_H
#define LRSTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LRSTV_OK                   0
#define LRSTV_WARN_NOT_CONVERGED   1   /* eps not reached within max_iter     */
#define LRSTV_ERR_INVALID_ARG     -1   /* bad size, weight, pointer or flag   */
#define LRSTV_ERR_WORKSPACE       -2   /* workspace too small                 */
#define LRSTV_ERR_UNSUPPORTED     -3   /* size beyond what the kernels handle */
#define LRSTV_ERR_HIP             -4   /* a HIP runtime call failed           */
#define LRSTV_ERR_NONFINITE       -5   /* NaN/Inf met in the input or state   */

/* ---- gradient-sparsity term (Sec. III-A) ---------------------------------- */
#define LRSTV_TV_ANISO    0   /* 2 tau ||D_w X||_1: soft-threshold per element     */
#define LRSTV_TV_ISO      1   /* 2 tau sum_v ||(D_w X)_v||_2 over the three
                                 directions of each voxel: group soft-threshold  */

/* ---- precision of the slice Gram / back-projection products ------------ */
#define LRSTV_FP32        0   /* plain FP32 products                           */
#define LRSTV_SPLIT_BF16  1   /* 3-term split-BF16 MFMA products, FP32 accum   */

/* Residuals recorded per iteration and per cube (FP64), in this order:
 *   0 ||Y - X - S||_inf, 1 ||X - Z||_inf   (Algorithm 1 stopping test)
 *   2 ||Y - X - S||_F,   3 ||X - Z||_F,   4 ||D_w Z - F||_F,  5 ||E - F||_F
 *   6 mu ||Z_new - Z_old||_F (dual residual)                                 */
#define LRSTV_NRES 7

/* Largest slice side (min(h, w)) the t-SVT kernels accept, and the largest
 * side of any FFT axis. */
#define LRSTV_MAX_SIDE 512

typedef struct lrstv_problem {
  int32_t n_cubes;         /* >= 1                                          */
  const int32_t* h;        /* host [n_cubes], each >= 1                     */
  const int32_t* w;        /* host [n_cubes], each >= 1                     */
  const int32_t* b;        /* host [n_cubes], each >= 1 (bands)             */
} lrstv_problem;

typedef struct lrstv_params {
  double tau;      /* gradient-sparsity weight  (>= 0)                       */
  double alpha;    /* gradient low-rank weight  (>= 0), t-SVT threshold alpha/mu */
  double lambda;   /* sparse-noise weight       (>= 0); the paper's rule is
                      lambda = C / sqrt(h w)                                 */
  double w[3];     /* difference weights w_1 (height), w_2 (width),
                      w_3 (bands), each >= 0                                 */
  double mu0;      /* initial penalty (> 0)                                  */
  double rho;      /* penalty growth (>= 1): mu <- min(rho mu, mu_max)       */
  double mu_max;   /* penalty cap (>= mu0)                                   */
  int32_t precision;  /* LRSTV_FP32 or LRSTV_SPLIT_BF16                      */
  int32_t tv;         /* LRSTV_TV_ANISO (the paper's TDLRSTV) or LRSTV_TV_ISO  */
  double beta;        /* >= 0; > 0 adds the explicit Gaussian term beta ||N||_F^2
                         with Y = X + S + N (N updated after S by its block
                         minimiser); 0: no N variable, N = Y - X - S          */
  double tucker[3];   /* Tucker ranks of X as fractions of the cube's sides,
                         modes 1 (height), 2 (width), 3 (bands): r_n =
                         floor(f_n d_n + 1/2) clipped to [1, d_n]; f_n <= 0 or
                         >= 1 keeps mode n at full rank.  Any truncated mode
                         turns the L-update into the HOOI Tucker approximation
                         (Sec. III-C, eq. X_solution); the paper's choice is
                         r1 = 0.8 h, r2 = 0.8 w, r3 tuned                       */
  int32_t hooi_sweeps;  /* HOOI sweeps after its truncated-HOSVD start (>= 0) */
} lrstv_params;

typedef struct lrstv_state_view {
  /* Device pointers into the workspace, each a packed batch of cubes, or
   * for the gradient-shaped variables three packed batches back to back
   * ([3][batch]: component n of cube c starts at n * total + offset(c),
   * with total = sum_c b h w).  Valid until lrstv_destroy.               */
  float* X;     /* L of the last iteration (the denoised estimate)        */
  float* Y;     /* the observed cube O (read-only for the solver)         */
  float* Z;
  float* S;
  float* G1;
  float* G2;
  float* F;     /* [3][batch] */
  float* E;     /* [3][batch] */
  float* G3;    /* [3][batch] */
  float* G4;    /* [3][batch] */
  float* N;     /* explicit noise term (beta > 0); may be NULL in views
                   passed to set_state / save_state: then left untouched  */
  double* mu;   /* device scalar: the penalty the next iteration uses     */
  int64_t total;   /* sum over cubes of b h w                             */
} lrstv_state_view;

typedef struct lrstv_report {
  int32_t iters;                 /* iterations run                        */
  double residuals[LRSTV_NRES];  /* last iteration, max over cubes        */
  double mu;                     /* penalty after the last iteration      */
} lrstv_report;

typedef struct lrstv_handle_s* lrstv_handle;

/* Bytes of device workspace a solver handle needs for this batch.
 * Errors: INVALID_ARG (null pointers, sizes < 1, bad params),
 * UNSUPPORTED (a side above LRSTV_MAX_SIDE). */
int lrstv_workspace_size(const lrstv_problem* prob, const lrstv_params* par, size_t* bytes);

/* Create a solver for the batch in `prob`.  `workspace` (device, >= the
 * queried size, 256-byte aligned) is owned by the caller and must outlive
 * the handle; `stream` (hipStream_t) is where all work is enqueued.
 * The host-side handle is allocated by the library and freed by
 * lrstv_destroy.  Errors: INVALID_ARG, WORKSPACE, UNSUPPORTED, HIP. */
int lrstv_create(lrstv_handle* out, const lrstv_problem* prob, const lrstv_params* par,
                 void* workspace, size_t ws_bytes, void* stream);

/* Algorithm 1 initialisation: O <- Y (device, packed batch, borrowed for the
 * call), Z <- Y, S = F = E = Gamma_i = 0, mu <- mu0.
 * Errors: INVALID_ARG, HIP. */
int lrstv_reset(lrstv_handle hd, const float* Y);

/* Run n_iter ADMM iterations (Sec. III-C steps 1-7).  If `residuals` is not
 * NULL it is a device array of n_iter * n_cubes * LRSTV_NRES doubles that
 * receives [iter][cube][LRSTV_NRES].  Asynchronous; no host sync.
 * A non-finite residual latches a device flag (until lrstv_reset); after the
 * iterations the flag is copied to host memory asynchronously, and any later
 * lrstv_iterate / lrstv_read_output whose copy has already landed returns
 * ERR_NONFINITE without running (lrstv_check waits for it).
 * Errors: INVALID_ARG, NONFINITE, HIP. */
int lrstv_iterate(lrstv_handle hd, int32_t n_iter, double* residuals);

/* Synchronise with the last lrstv_iterate's copy of the non-finite flag and
 * return ERR_NONFINITE if an iteration since the last reset met a NaN/Inf
 * residual (an input with NaN/Inf does), else OK. */
int lrstv_check(lrstv_handle hd);

/* Replay iterations from a hipGraph of one iteration captured on the
 * handle's stream (enable = 1; captured on first use) or launch them one by
 * one (0, the default).  Results are bit-identical either way.  Stage
 * timing (lrstv_profile) forces eager launches while it is on. */
int lrstv_set_graph(lrstv_handle hd, int32_t enable);

/* Copy X = L of the last iteration and S into caller buffers (device,
 * packed batch).  Either may be NULL.  Asynchronous.  Returns ERR_NONFINITE
 * (copying nothing) when the non-finite latch is already known to be set. */
int lrstv_read_output(lrstv_handle hd, float* X, float* S);

/* reset + iterate until max{||Y-X-S||_inf, ||X-Z||_inf} <= eps (Algorithm 1's
 * convergence check) + copy X and S out (device, may be NULL).  eps <= 0
 * runs exactly max_iter iterations.  With eps > 0 the test is made on the
 * device after every iteration, per cube: a cube that meets it halts (every
 * later kernel of the iteration returns at once for it, so its state stays
 * that of its stopping iteration), and iterations are replayed in chunks
 * whose halt flags the host reads one chunk behind, so there is no host
 * synchronisation per iteration.  X and S of every cube are those of the
 * first iteration at which it met the test.  Afterwards the test is off
 * again (later lrstv_iterate calls continue from the stopped state).
 * Synchronises the stream.  `rep` (host, may be NULL): the largest
 * per-cube iteration count, the residuals of each cube's last iteration
 * (max over cubes), mu after the last iteration run.  Returns
 * WARN_NOT_CONVERGED if eps > 0 was not met by every cube, ERR_NONFINITE
 * (copying nothing) if a residual is NaN/Inf. */
int lrstv_solve(lrstv_handle hd, const float* Y, float* X, float* S, int32_t max_iter,
                double eps, lrstv_report* rep);

/* Iterations each cube ran since the last reset (per-cube counts of the
 * last lrstv_solve), host array iters[n], n >= n_cubes.  Synchronises the
 * stream.  Returns n_cubes or an error. */
int lrstv_cube_iterations(lrstv_handle hd, int32_t* iters, int32_t n);

/* Device pointers to the state (checkpoint / resume / adjoint). */
int lrstv_get_state(lrstv_handle hd, lrstv_state_view* view);

/* Copy a state (device pointers with the layout of lrstv_state_view; the
 * X, Y and mu members may be NULL to leave them) into the handle.
 * Asynchronous on the handle's stream. */
int lrstv_set_state(lrstv_handle hd, const lrstv_state_view* src);

/* Copy the handle's state into dst (every member but X, Y and mu required;
 * those three are copied when non-NULL).  For per-iteration checkpoints
 * of the adjoint.  Asynchronous on the handle's stream. */
int lrstv_save_state(lrstv_handle hd, const lrstv_state_view* dst);

void lrstv_destroy(lrstv_handle hd);

/* ---- adjoint of the iteration ------------------------------------------ */

/* Bytes of the extra device workspace lrstv_iterate_vjp needs for this
 * handle's batch (direction slices and their SVT-derivative products, and
 * cube-sized cotangent scratch). */
int lrstv_vjp_workspace_size(lrstv_handle hd, size_t* bytes);

/* Vector-Jacobian product of one iteration of Algorithm 1 (Sec. III-C),
 * the map (state before, O, tau, alpha, lambda) -> (state after, X = L of
 * this iteration), taken in reverse with the chain rule:
 *   soft-threshold R_d(u): mask 1[|u| > d], d-cotangent -sign(u) 1[|u| > d]
 *     (masks and signs read from the iteration's outputs S', F');
 *   t-SVT: symmetric Jacobian (prox of a convex function), so the input
 *     cotangent is the derivative along the output cotangent, computed per
 *     Fourier slice from the Gram eigendecomposition by the Daleckii-Krein
 *     rule; threshold cotangent -sum_{s > t} Re<D v, M v>/s per slice;
 *   Z-update: the solve operator mu (I + D_w^* D_w) is symmetric, so its
 *     VJP is the same FFT solve; D_w's VJP is D_w^*.
 * before: state the iteration started from (G4 and mu required: mu is the
 *   device scalar the iteration used); its Y is not read.
 * after: state the iteration produced (S and F required).
 * grad_after: cotangents of the state after (every member but X, Y, mu),
 *   or NULL for zero.  grad_X: cotangent of X = L of this iteration, or
 *   NULL for zero.
 * grad_before (written): cotangents of the state before.  Must not alias
 *   grad_after or the states.
 * grad_weights (device, [n_cubes][3] doubles, accumulated): cotangents of
 *   (tau, alpha, lambda) per cube.  grad_Y (device floats, packed batch,
 *   accumulated): cotangent of O.
 * flags: LRSTV_VJP_INITIAL when `before` is the initial state of a reset
 *   (Z = O), so that the cotangent of Z also flows into grad_Y; else 0.
 * ws: device workspace of lrstv_vjp_workspace_size bytes, 256-byte aligned.
 * The solver's slice scratch is reused; the solver state is not touched.
 * FP32 arithmetic with FP64 parameter sums.  Asynchronous on the handle's
 * stream.  Errors: INVALID_ARG, WORKSPACE, HIP. */
#define LRSTV_VJP_INITIAL 1
int lrstv_iterate_vjp(lrstv_handle hd, const lrstv_state_view* before, const lrstv_state_view* after,
                      const lrstv_state_view* grad_after, const float* grad_X,
                      lrstv_state_view* grad_before, double* grad_weights, float* grad_Y,
                      int32_t flags, void* ws, size_t ws_bytes);

/* ---- standalone primitives --------------------------------------------- */

/* Workspace bytes for lrstv_svt on `batch` tensors of shape (b, h, w). */
int lrstv_svt_workspace_size(int32_t h, int32_t w, int32_t b, int32_t batch, int32_t precision,
                             size_t* bytes);

/* t-SVT (Sec. III-C, E-update; t-SVD of Theorem 4.2): for each of `batch`
 * real tensors A (device, packed [batch][b][h][w]) compute
 *   E = IDFT_b( SVT_thresh( DFT_b(A)_k ) for every Fourier slice k ),
 * i.e. the prox of thresh * TNN.  Only the floor(b/2)+1 non-redundant
 * slices are decomposed; the others follow by conjugate symmetry.
 * E (device) may not alias A.  Errors: INVALID_ARG, WORKSPACE, UNSUPPORTED,
 * HIP. */
int lrstv_svt(const float* A, float* E, int32_t h, int32_t w, int32_t b, int32_t batch,
              float thresh, int32_t precision, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for lrstv_svt_vjp on `batch` tensors of shape (b, h, w). */
int lrstv_svt_vjp_workspace_size(int32_t h, int32_t w, int32_t b, int32_t batch, size_t* bytes);

/* Vector-Jacobian product of the t-SVT (the derivative of lrstv_svt): for
 * each of `batch` tensors, gA = J(A)^T G = J(A) G (the Jacobian of a prox
 * map is symmetric) and, when grad_thresh (device, [batch] doubles,
 * overwritten) is non-NULL, d<E, G>/d thresh.  A, G, gA device, packed
 * [batch][b][h][w]; gA may not alias A or G.  FP32 products with a full
 * FP64 eigendecomposition of each slice Gram.  Synchronises the stream
 * before returning.  Errors: INVALID_ARG, WORKSPACE, UNSUPPORTED, HIP. */
int lrstv_svt_vjp(const float* A, const float* G, float* gA, int32_t h, int32_t w, int32_t b,
                  int32_t batch, float thresh, double* grad_thresh, void* ws, size_t ws_bytes,
                  void* stream);

/* Workspace bytes for lrstv_zsolve on one (b, h, w) cube. */
int lrstv_zsolve_workspace_size(int32_t h, int32_t w, int32_t b, size_t* bytes);

/* Z-update (Sec. III-C): solve mu (I + sum_n w_n^2 D_n^T D_n) Z = T for a
 * periodic (b, h, w) cube (device T, Z; they may alias).  Errors as above. */
int lrstv_zsolve(const float* T, float* Z, int32_t h, int32_t w, int32_t b, double mu,
                 const double wts[3], void* ws, size_t ws_bytes, void* stream);

/* Size of the built-in scratch of lrstv_zsolve_noalloc (64 MiB per device). */
#define LRSTV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* lrstv_zsolve for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, with the half spectrum b h (w/2+1) complex (8 bytes each)
 * held in a scratch array built into the library instead of a caller
 * workspace.  No device memory is allocated or freed by the call.  T, Z
 * (device, may alias), sizes, mu and wts as for lrstv_zsolve.  The scratch
 * is one array per device, shared by every call on that device, and keeps
 * the last call's contents: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.  The
 * first call on a device looks up the array's address there.
 * Errors: INVALID_ARG, UNSUPPORTED (a side above LRSTV_MAX_SIDE),
 * WORKSPACE (b h (w/2+1) * 8 > LRSTV_NOALLOC_SCRATCH_BYTES), HIP. */
int lrstv_zsolve_noalloc(const float* T, float* Z, int32_t h, int32_t w, int32_t b, double mu,
                         const double wts[3], void* stream);

/* ---- autotuner ---------------------------------------------------------- */

/* Launch shapes chosen per handle.  The slice tridiagonalisation (the
 * dominant kernel) has compiled shapes, each named by a code 100 k + w:
 * k = 0 keeps the packed Gram's rows in registers and LDS and reduces them
 * on the vector units (w = 8, 12, 16 waves per slice); k = 1 keeps the
 * whole Gram in 32 x 32 register tiles and applies the rank-2 update on the
 * matrix cores (w = 12, 8; slices up to 256).  Which is fastest depends on
 * the slice sizes of the batch. */
#define LRSTV_MAX_TRI_SHAPES 8
typedef struct lrstv_tuning {
  int32_t tridiag_shape;                        /* chosen shape code        */
  int32_t n_shapes;                             /* entries below            */
  int32_t shapes_tried[LRSTV_MAX_TRI_SHAPES];   /* codes                    */
  double  tridiag_ms[LRSTV_MAX_TRI_SHAPES];     /* mean ms per launch over the
                                                   handle's slices, -1 if the
                                                   shape cannot hold them on
                                                   chip                     */
} lrstv_tuning;

/* Time every tridiagonalisation shape on this handle's slice sizes (slices
 * filled with hashed values, so the timing does not depend on the state;
 * `reps` timed launches each after one warm-up) and keep the fastest.  The
 * solver state is not touched (the slice scratch is overwritten); a
 * captured iteration graph is dropped and recaptured on the next iterate.
 * Synchronises the stream.  out may be NULL.  Errors: INVALID_ARG, HIP. */
int lrstv_autotune(lrstv_handle hd, int32_t reps, lrstv_tuning* out);

/* Apply a stored choice (only tridiag_shape is read).  INVALID_ARG for a
 * shape that does not exist. */
int lrstv_set_tuning(lrstv_handle hd, const lrstv_tuning* t);

/* The handle's current choice (timings -1). */
int lrstv_get_tuning(lrstv_handle hd, lrstv_tuning* t);

/* ---- diagnostics ------------------------------------------------------- */

/* Stages of one iteration, in launch order (lrstv_stage_name gives the
 * names): L/T_z, rfft along w, FFT along h (both directions), tridiagonal
 * band solve, inverse rfft, difference/shrink/multipliers, band DFT, slice
 * Gram, tridiagonalisation, tridiagonal eigenvalues, tridiagonal
 * eigenvectors, back-transform,
 * back-projection B, shrink factors, back-projection Ehat, inverse band DFT
 * + Gamma4, residual reduction + mu step, and the HOOI Tucker approximation
 * of the L-update (with truncated Tucker ranks only). */
#define LRSTV_NSTAGES 18

/* Start (enable = 1, discarding what was recorded) or stop (0) recording a
 * pair of hipEvents around every stage launched by lrstv_iterate / solve,
 * on the handle's stream.  Adds a few microseconds of host work per stage. */
int lrstv_profile(lrstv_handle hd, int32_t enable);

/* Synchronise the stream and return, per stage, the summed GPU
 * milliseconds (ms[LRSTV_NSTAGES]) and launch counts (counts, may be NULL)
 * recorded since lrstv_profile(hd, 1); clears the record.  n >= LRSTV_NSTAGES. */
int lrstv_stage_times(lrstv_handle hd, double* ms, int32_t* counts, int32_t n);
const char* lrstv_stage_name(int32_t stage);

/* Number of singular values kept (those not below the threshold, up to the
 * Gram's FP32 resolution) in each Fourier slice by the last iteration, host
 * array ranks[n] in slice order (cube, gradient tensor, frequency).
 * Synchronises the stream.  Returns the number of slices, or an error. */
int lrstv_slice_ranks(lrstv_handle hd, int32_t* ranks, int32_t n);

const char* lrstv_status_string(int status);
const char* lrstv_last_error(void);   /* thread-local, "" if none */
int lrstv_version(void);              /* 100 * major + minor */

#ifdef __cplusplus
}
#endif
#endif /* LRSTV_H */
