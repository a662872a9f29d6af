/*
 * gs.h -- C ABI of the MI355X generalized-sampling library (libgs.so).
 *
 * Generalized sampling (Jacobsen, Nielsen, Rasmussen, "Generalized Sampling
 * in Julia", arXiv 1607.04091): given M Fourier samples y_m of a function on
 * [-1/2, 1/2]^d at frequencies xi_m, find the coefficients x of its
 * approximation in V_J^int (boundary-corrected Daubechies scaling functions
 * with p vanishing moments, N = 2^J functions per dimension, Sec. 3.3) as the
 * weighted least-squares solution of T x = y (Sec. 2 eq. least_squares,
 * Sec. 4.1 eq. weighted_least_squares).  T is the M x N^d change-of-basis
 * matrix of Sec. 4 (1D block form [L I R], eq. CoB_block_1D) and Sec. 5 /
 * App. C (2D tensor product, eq. 2Dwavelet_border_division).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Frequencies xi are unnormalized (the paper's xi_m); 2D points are stored
 *   interleaved (xi_x, xi_y) per point.
 * - Column n (0-based) of the 1D basis is: n < p  -> left boundary function
 *   phi^L_n shifted to -1/2; p <= n < N-p -> interior phi_{J, n-N/2};
 *   n >= N-p -> right boundary function phi^R_{N-1-n} shifted to +1/2
 *   (Sec. 3.3 ordering: phi^L_0 .. phi^L_{p-1}, interior, phi^R_{p-1} .. phi^R_0).
 *   For Haar (p = 1) every column is interior.
 * - 2D coefficients are ROW-MAJOR X[i][j], i the x index (fast index j = y).
 *   This differs from the column-major vec() of App. C.
 * - Complex vectors are interleaved (re, im): complex128 for FP64 data,
 *   complex64 for FP32 data.
 * - Device pointers are HIP device pointers on the current device; the
 *   caller owns them.  `stream` is a hipStream_t (NULL = default stream).
 *   Every apply is stream-ordered and does not synchronize the host.
 * - Return value 0 = success, negative = error (see GS_ERR_*).  Argument
 *   validation happens before any device work, so invalid input never
 *   launches a kernel.  No C++ exception crosses this interface.
 */
#ifndef GS_H
#define GS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_VERSION 100

/* status codes */
#define GS_OK               0
#define GS_NOT_CONVERGED    1   /* gs_solve hit max_iter; x holds the last iterate */
#define GS_ERR_INVALID_ARG (-1) /* NULL pointer, bad dim/J/M/flags/options      */
#define GS_ERR_UNSUPPORTED (-2) /* p outside 1..8, 2^J < 2p, grid too large      */
#define GS_ERR_BAD_NODES   (-3) /* non-finite frequency, negative/non-finite weight */
#define GS_ERR_NOMEM       (-4) /* device or host allocation failed              */
#define GS_ERR_HIP         (-5) /* HIP runtime error (text via gs_strerror)       */
#define GS_ERR_BREAKDOWN   (-6) /* CGLS breakdown: ||A p||^2 <= 0 or non-finite  */
#define GS_ERR_PRECISION   (-7) /* requested precision not held by this plan     */
#define GS_ERR_TOO_LARGE   (-8) /* gs_apply_TH_noalloc: workspace above its limit */

/* plan precision */
#define GS_F64        0  /* applies in FP64, complex128 vectors                       */
#define GS_F32        1  /* applies in FP32, complex64 vectors                        */
#define GS_F32_MIXED  2  /* FP32 applies plus FP64 data for refinement (both held)    */

/* apply flags */
#define GS_WEIGHTED  1   /* apply W^{1/2} T (resp. T^H W^{1/2}) instead of T (T^H)      */
#define GS_SORTED    2   /* sample vectors are in the plan's internal point order       */
#define GS_WEIGHT_FULL 8 /* with GS_WEIGHTED: W T (T^H W) instead of W^{1/2} T (T^H W^{1/2});
                            T^H W y is A^H b, the warm-start network's input            */
#define GS_APPLY_F64 4   /* on a GS_F32_MIXED plan: run the FP64 apply (complex128 IO)  */

typedef struct gs_plan gs_plan_t;

/*
 * gs_plan -- build the matrix-free representation of T (the paper's
 * Freq2Wave, Sec. 6.2; its "init").  The per-point tables (wrapped nodes,
 * the cell sort, D, L and R of App. A / A.1) are computed on the device; only
 * the filters (taps, boundary recursion matrices) are constructed on the host.
 *   out        receives the handle (freed with gs_destroy).
 *   dim        1 or 2.
 *   J          scale, N = 2^J coefficients per dimension; 2^J >= 2p and
 *              1 <= J <= 20 (1D) or 11 (2D).  Plans holding FP32 data
 *              (GS_F32, GS_F32_MIXED) need J <= 14: FP32 positions are 32-bit
 *              fixed point with J + 1 bits of grid cell, and the window needs
 *              17 bits of in-cell offset for FP32 accuracy (else
 *              GS_ERR_UNSUPPORTED; GS_F64 plans cover the whole range).
 *   p          vanishing moments: 1 = Haar, 2..8 = Daubechies dbp with CDV
 *              boundary functions (App. A.1).
 *   M          number of samples, >= 1.
 *   xi         HOST array of M*dim doubles (interleaved for dim 2), finite.
 *   mu         HOST array of M non-negative finite weights (Voronoi measures,
 *              App. B), or NULL for unit weights.
 *   precision  GS_F64, GS_F32 or GS_F32_MIXED.
 *   stream     stream for the uploads.
 * Uniform nodes (Sec. 3.2): when every frequency lies on a grid eps Z with
 * eps = 2^-a, a <= 3 (e.g. xi_k = k/2), every wrapped node is a node of an
 * oversampled grid of side max(2N, 2^a N); the interior block is then computed
 * exactly -- a zero-padded FFT read at the nodes, the paper's phase-shifted,
 * zero-interleaved DFT -- with no window error and no deapodization
 * (gs_plan_info.exact_nodes reports it).  Other node sets use the windowed NFFT.
 * Host inputs are copied; the caller may free them on return.  The plan owns
 * all of its device memory (point data, transform grids, solver vectors).
 * A plan is not thread-safe: calls on one plan share its workspace and must
 * be ordered on one stream.
 */
int gs_plan(gs_plan_t** out, int dim, int J, int p, int64_t M, const double* xi,
            const double* mu, int precision, void* stream);

/*
 * gs_apply_T -- y = T x (or W^{1/2} T x with GS_WEIGHTED).
 * Sec. 4: T x = L x_L + D NFFT(x_I) + R x_R; Sec. 5 / App. C: nine blocks,
 * interior by a 2D NFFT, sides by 1D NFFTs, corners dense.
 *   x  device, N^dim complex (row-major X[i][j] in 2D).
 *   y  device, M complex; in the caller's point order unless GS_SORTED.
 * Element type: complex128 for GS_F64 plans and GS_APPLY_F64, else complex64.
 */
int gs_apply_T(const gs_plan_t* plan, const void* x, void* y, int flags, void* stream);

/*
 * gs_apply_TH -- x = T^H u (or T^H W^{1/2} u with GS_WEIGHTED); App. C
 * adjoint, same layouts and element types as gs_apply_T.  Deterministic:
 * repeated calls give bitwise-identical results (no atomics).
 */
int gs_apply_TH(const gs_plan_t* plan, const void* u, void* x, int flags, void* stream);

/*
 * gs_apply_TH_noalloc -- gs_apply_TH (same operation, arguments, flags,
 * layouts, element types and results, bit for bit) for callers that cannot
 * allocate device memory or call allocating routines: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It calls no
 * hipMalloc, hipFree or allocating library routine.  Its transform workspace
 * (the oversampled grid, the 2D side grids, the tile partial sums and the
 * input in sorted order) is carved from one static device array of
 * GS_NOALLOC_SCRATCH_BYTES (64 MiB) per device, which each device holds until
 * the process ends; the plan's own workspace is not touched.  The workspace
 * grows with the grid (n_g^dim complex), the tiles (about 2,900 complex per
 * 32 x 32-cell tile in 2D) and the points (M complex): about 39 MB for the
 * 1,048,576-point J = 9 problem in FP32 (78 MB in FP64, which is refused).
 * A plan whose workspace exceeds the array returns GS_ERR_TOO_LARGE before
 * any device work.  The array is shared by every call on a device and keeps
 * the last call's contents: calls that overlap on one device (on different
 * streams, or from several host threads) race and must be serialized by the
 * caller.  The first call on a device looks up the array's device address.
 */
#define GS_NOALLOC_SCRATCH_BYTES (64ll << 20)
int gs_apply_TH_noalloc(const gs_plan_t* plan, const void* u, void* x, int flags, void* stream);

/* CGLS options / results (Sec. 2: conjugate gradients on the LS problem). */
typedef struct gs_solve_opts {
    double rel_tol;        /* stop when ||A^H(b - A x)|| <= rel_tol ||A^H b||, A = W^{1/2}T */
    int    max_iter;       /* >= 1                                                        */
    int    warm_start;     /* 0: x0 = 0; 1: x holds x0 on entry; 2: guarded -- x0 is
                              kept only if ||A^H(b - A x0)|| < ||A^H b||, else x0 = 0     */
    int    refine_fp64;    /* GS_F32_MIXED plans: FP64 residual refinement at the end    */
    int    max_restarts;   /* refinement restarts allowed (mixed form), >= 0             */
    int    check_every;    /* iterations between host reads of the stop flag (>= 1)      */
    double* history;       /* optional HOST buffer for the residual history, or NULL     */
    int    history_len;    /* its length                                                 */
} gs_solve_opts;

typedef struct gs_solve_info {
    int    iterations;          /* CGLS iterations run (all restarts)                  */
    int    restarts;            /* refinement restarts taken                            */
    int    status;              /* GS_OK, GS_NOT_CONVERGED or GS_ERR_BREAKDOWN          */
    double rel_residual;        /* final relative normal residual (recurred)           */
    double rel_residual_fp64;   /* recomputed with FP64 applies (mixed form), else -1  */
    int    warm_start_used;     /* 1 if the iteration started from the caller's x0     */
    int    batch_class;         /* gs_solve_batch: the geometry class whose kernels ran
                                   this problem batched, or -1 (plain launches)          */
    int    batch_streams;       /* gs_solve_batch: streams the classes were spread over  */
} gs_solve_info;

/*
 * gs_solve -- weighted LS solution argmin ||W^{1/2}(T x - y)|| by CGLS
 * (Sec. 2, Sec. 4.1).  y: device, M complex128 in caller order; x: device,
 * N^dim complex128 (read as x0 when opts->warm_start).  All CGLS vectors and
 * reductions are FP64 and device-resident; applies run in the plan's
 * precision.  Returns GS_OK, GS_NOT_CONVERGED (x = last iterate) or an error.
 * Synchronizes `stream` every opts->check_every iterations.
 * Mixed form (GS_F32_MIXED with refine_fp64): the FP32-apply recurrence stops
 * when its normal residual rises 100x above its smallest value (it has passed
 * the FP32 accuracy floor) or breaks down; the FP64 residual is then
 * recomputed and the recurrence restarted from x (at most max_restarts
 * times).  Status follows the FP64 residual: GS_OK at or below rel_tol, else
 * GS_NOT_CONVERGED; GS_ERR_BREAKDOWN only if it is not finite.
 */
int gs_solve(const gs_plan_t* plan, const void* y, void* x, const gs_solve_opts* opts,
             gs_solve_info* info, void* stream);

/*
 * gs_plan_batch -- the plans of many problems in one call (the batched
 * form's set-up; each plan is the paper's Freq2Wave set-up of Sec. 6.2, as
 * gs_plan builds it): out[i] = gs_plan(descs[i]...) for i = 0..count-1,
 * every plan built on `stream`.
 *   out    HOST array of count handles (written).
 *   count  >= 1.
 *   descs  HOST array of count descriptors; each carries gs_plan's arguments
 *          with the same meaning and limits (host inputs are copied).
 * NULL out or descs, or count < 1: GS_ERR_INVALID_ARG.  All or nothing: on
 * the first failure the plans already built are destroyed, every out[i] is
 * NULL, and that failure's status is returned.  The plans are ordinary
 * plans: gs_solve_batch takes them, and so does every other call; free each
 * with gs_destroy.
 */
typedef struct gs_plan_desc {
    int dim;
    int J;
    int p;
    int precision;
    int64_t M;
    const double* xi;   /* HOST, M*dim doubles */
    const double* mu;   /* HOST, M weights, or NULL */
} gs_plan_desc;

int gs_plan_batch(gs_plan_t** out, int count, const gs_plan_desc* descs, void* stream);

/*
 * gs_solve_batch -- many independent weighted LS problems (Sec. 2, Sec. 4.1),
 * each with its own plan (sizes, point sets and precisions may differ), solved
 * together.  plans[i], y[i], x[i] follow gs_solve's layouts; plans and x
 * buffers must be pairwise distinct (each problem owns its plan's work
 * vectors).  One options struct serves every problem; opts->history must be
 * NULL.  infos: HOST array of `count` results.
 *
 * Problems whose plans share one geometry (2D, grids of at least 32 x 32
 * cells, same apply precision, N and p) form a class: every kernel of the
 * class's CGLS iteration runs as ONE launch for all of its active problems,
 * each problem reading its own arguments; the iterations of a class are
 * captured as HIP graphs and replayed round after round on one of up to
 * n_streams internal streams (classes placed heaviest first).  Other plans
 * run their own captured iterations.  Every opts->check_every rounds one host
 * synchronization reads all stop flags; finished problems leave their class
 * (its launches are compacted when a quarter of them have finished).
 * n_streams = 0 picks the stream count (1, 2, 4, 8, capped at the class
 * count) from short timed trial rounds; otherwise 1..64 are accepted and at
 * most 8 internal streams are used (more only take turns on the hardware
 * queues).  Per problem the
 * kernels and their arithmetic are those of gs_solve, so every result equals
 * gs_solve's bit for bit.  The internal streams wait for `stream` on entry;
 * the call returns after all work is done.  Returns GS_OK when every problem
 * converged, GS_NOT_CONVERGED when some did not (see infos[i].status), or the
 * worst error; every problem is finished and reported either way.
 */
int gs_solve_batch(const gs_plan_t* const* plans, int count, const void* const* y, void* const* x,
                   const gs_solve_opts* opts, gs_solve_info* infos, int n_streams, void* stream);

/*
 * gs_weval -- evaluate a representation in V_J^int on a dyadic grid (the
 * paper's weval, Sec. 6.2; the image-space output of Figs. 1-2):
 *   1D: out[j] = sum_n coef[n] s_n(x_j), x_j = -1/2 + j 2^-R, j = 0..2^R;
 *   2D: out[a (2^R+1) + b] = sum_{i,j} coef[i N + j] s_i(x_a) s_j(x_b).
 * s_n is basis function n of Sec. 3.3 in space (the column order of gs_plan:
 * left boundary functions, interior translates, right boundary functions),
 * evaluated by the cascade algorithm: phi at the integers from the
 * refinement equation, then doubling the resolution to R - J; the boundary
 * functions are their defining combinations of restricted translates
 * (App. A.1).  coef and out: device complex128 (N^dim and (2^R+1)^dim).
 * R >= J, R - J <= 20, R <= 26 (1D) or 13 (2D).  Allocates temporary device
 * memory and returns after the result is complete (synchronizes `stream`).
 */
int gs_weval(int dim, int J, int p, int R, const void* coef, void* out, void* stream);

/* Releases every resource of the plan (NULL is ignored). */
void gs_destroy(gs_plan_t* plan);

/* Plan geometry, for callers that size buffers. */
typedef struct gs_plan_info {
    int     dim, J, p, N, precision;
    int64_t M;
    int     grid_n;          /* oversampled NFFT grid size per dimension (2N) */
    int     window_w32;      /* KB window taps per dimension, FP32 path (0 if absent) */
    int     window_w64;      /* KB window taps per dimension, FP64 path (0 if absent) */
    int64_t device_bytes;    /* device memory held by the plan */
    int     exact_nodes;     /* 1: every frequency lies on a grid 2^-a Z (a <= 3) and the
                                transform is exact (Sec. 3.2 uniform nodes), see gs_plan */
} gs_plan_info;
int gs_get_plan_info(const gs_plan_t* plan, gs_plan_info* info);

/* Copies the plan's point permutation (internal order -> caller index) to a
 * HOST buffer of M int32. */
int gs_get_permutation(const gs_plan_t* plan, int32_t* perm_host);

/* Copies the plan's per-point basis table of one dimension (0 = x, 1 = y) to
 * a HOST buffer, in the plan's internal point order (see gs_get_permutation):
 * (2nb+1) x M complex, channel-major, channels [L_0..L_{nb-1}, D,
 * R_0..R_{nb-1}] as in gs_eval_basis_1d (nb = 0 for Haar, else p); complex128
 * with f64 != 0, else complex64.  GS_ERR_PRECISION if the plan does not hold
 * that precision.  (The tables are built on the device by gs_plan.) */
int gs_get_channels(const gs_plan_t* plan, int dimension, int f64, void* host_out);

const char* gs_strerror(int code);
int gs_version(void);

/* ------------------------------------------------------------------------
 * Per-kernel timing (measurement support).  gs_profile_enable(1) clears the
 * record and makes every subsequent library kernel launch record a pair of
 * HIP events on its launch stream; gs_profile_enable(0) stops recording (and
 * clears).  gs_profile_read synchronizes on the recorded events and returns,
 * per kernel that ran, its name (names[32*i], NUL-terminated), launch count
 * and total elapsed milliseconds; *n_kernels receives the number of entries
 * (<= max_kernels).  Process-wide; not for concurrent use from several threads.
 * ------------------------------------------------------------------------ */
int gs_profile_enable(int enable);
int gs_profile_read(int max_kernels, char* names, int64_t* counts, double* total_ms, int* n_kernels);

/* ------------------------------------------------------------------------
 * Host-only basis queries (no device work; usable without a GPU).
 * ------------------------------------------------------------------------ */

/* Daubechies taps h_k, k = -p+1..p (App. A, m0(0) = 1), into h[2p]. */
int gs_filter_taps(int p, double* h);

/*
 * Boundary recursion data of App. A.1 for p >= 2: U (p x p, row-major),
 * V (p x (2p-1), row-major, columns m = p..3p-2) and v1(0) (p), for the left
 * edge and for the right edge.  Any output pointer may be NULL.
 */
int gs_boundary_filters(int p, double* U_left, double* V_left, double* v0_left,
                        double* U_right, double* V_right, double* v0_right);

/*
 * 1D basis values at host points, FP64: out[m*(2nb+1) + c] (complex128,
 * interleaved) with nb = 0 for Haar else p and channel c:
 *   c <  nb      : column c        (left boundary)    2^{-J/2} e^{+i pi xi} phiL_c(2^-J xi)
 *   c == nb      : the interior scale D = 2^{-J/2} phi-hat(2^-J xi)
 *   c >  nb      : column N-1-(c-nb-1) (right boundary) 2^{-J/2} e^{-i pi xi} phiR_{c-nb-1}(2^-J xi)
 * (Sec. 4 entries of T; an interior column n is D * exp(-2 pi i (n-N/2) 2^-J xi).)
 */
int gs_eval_basis_1d(int J, int p, int64_t M, const double* xi, double* out);

/* ------------------------------------------------------------------------
 * Learned warm start (not from the paper, which starts CGLS from zero).
 * A residual CNN maps the adjoint image A^H b = T^H W y of a 2D problem to an
 * estimate of the LS solution, used as gs_solve's x0 (opts.warm_start).
 *
 * Network: u = s * input (fixed scale s); conv3x3 2->32 + ReLU,
 * 4 x (conv3x3 32->32 + ReLU), conv3x3 32->2; output = u + last conv.  Convolutions are cross-correlations with zero
 * padding, no biases; weights w[ky][kx][ci][co].  Images are (batch, H, W)
 * complex arrays (channels re, im), H x W = N x N coefficients, row-major as
 * gs_solve's x.  Activations and hidden-layer gradients are stored in
 * bfloat16, products use bf16 copies of FP32 master weights, sums are FP32;
 * the 32->32 layers run on MFMA.  Loss: sum ||out - t||^2 / sum ||t||^2 over
 * the batch.  Optimizer: Adam.  Deterministic (no atomics).
 *
 * Parameters, as one FP32 host array of gs_cnn_param_count() = 38016 values:
 * layers 1..6 in order, each w[ky][kx][ci][co] row-major.
 * One handle serves one stream at a time.
 * ------------------------------------------------------------------------ */
typedef struct gs_cnn gs_cnn_t;

#define GS_CNN_IN_F64   1   /* forward input is complex128 (else complex64)               */
#define GS_CNN_OUT_F64  2   /* forward output is complex128 (else complex64)              */
#define GS_CNN_TRAIN    4   /* keep what gs_cnn_backward needs; out may then be NULL      */
#define GS_CNN_TGT_F64  8   /* backward target is complex128 (else complex64)             */

int gs_cnn_param_count(void);

/* Fixed (untrained) input scale s > 0: the network sees s * input and its
 * output is s * input + last conv.  It brings A^H b to the size of x.
 * Default 1. */
int gs_cnn_set_input_scale(gs_cnn_t* cnn, float scale);
int gs_cnn_get_input_scale(const gs_cnn_t* cnn, float* scale);

/* Allocates a network for images of height x width and batches up to
 * max_batch (device memory ~ 7 x 64 B per pixel of the largest batch).
 * Weights start at zero: set them with gs_cnn_set_weights. */
int gs_cnn_create(gs_cnn_t** out, int height, int width, int max_batch);
void gs_cnn_destroy(gs_cnn_t* cnn);

/* Host FP32 parameter arrays (38016 values).  set_weights also clears the
 * Adam moments and step count; it rejects non-finite values. */
int gs_cnn_set_weights(gs_cnn_t* cnn, const float* host_params);
int gs_cnn_get_weights(const gs_cnn_t* cnn, float* host_params);
int gs_cnn_get_grads(const gs_cnn_t* cnn, float* host_params);   /* of the last backward */
/* Adam state (checkpoint / resume): first and second moments, step count. */
int gs_cnn_get_state(const gs_cnn_t* cnn, float* m, float* v, int* step);
int gs_cnn_set_state(gs_cnn_t* cnn, const float* m, const float* v, int step);

/* in: device, batch x H x W complex; out: device, same shape (may be NULL
 * with GS_CNN_TRAIN).  Asynchronous on `stream`. */
int gs_cnn_forward(gs_cnn_t* cnn, const void* in, void* out, int batch, int flags, void* stream);

/* Loss and parameter gradients for the preceding GS_CNN_TRAIN forward of the
 * same batch (else GS_ERR_INVALID_ARG).  target: device, batch x H x W complex.
 * If loss != NULL, synchronizes `stream` and stores the loss there. */
int gs_cnn_backward(gs_cnn_t* cnn, const void* target, int batch, int flags, double* loss, void* stream);

/* One Adam step on the gradients of the last backward (bias-corrected,
 * step count kept by the handle). */
int gs_cnn_step(gs_cnn_t* cnn, float lr, float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
