/*
 * lskum.h -- C ABI of the MI355X (gfx950) implicit LSKUM solver.
 *
 * The library computes, on one GPU, the implicit least squares kinetic
 * upwind method (LSKUM) for the 2D Euler equations on a point cloud with the
 * modified LU-SGS scheme of Verma, Mamidi and Nemili (2024):
 *   - the second-order LSKUM residual R: least-squares derivatives of the
 *     kinetic split fluxes Gx+-, Gy+- over each point's split stencils, built
 *     from q-variables with defect-corrected q-derivatives
 *     (Section 2, eq. 11 and eq. 13-16);
 *   - the LU-SGS forward/backward sweeps (Section 3, eq. 25-27) with the
 *     scalar diagonal of eq. (34)-(35), in point-colour order
 *     (Section 4, Algorithms 4, 6 and 7); the split-flux Jacobian-vector
 *     products are exact tangents (the paper's "+AD" solvers) or the flux
 *     differences of eq. (28) (the paper's baseline).
 *
 * Conventions
 *   - Every function returns int: 0 (LSKUM_OK) or a negative LSKUM_ERR_*
 *     code; lskum_last_error() gives a message for the calling thread.
 *   - Point fields are passed as structure-of-arrays [4][n] of double:
 *     field v of point p at index v*n + p.  U = (rho, rho u1, rho u2, rho E)
 *     with E the total specific energy.
 *   - Point types: 0 wall, 1 interior, 2 outer (held at free stream, or
 *     with the kinetic far field of lskum_params.farfield).
 *   - Wall frame: unit tangent (tx, ty); the normal n = (-ty, tx) must point
 *     into the fluid.  Outer points use their frame only with the kinetic far
 *     field, and then n = (-ty, tx) must point out of the domain.  Interior
 *     points ignore the frame.
 *   - Wall points, in storage order, must trace one closed body contour
 *     (used only by lskum_forces).
 *   - Connectivity is CSR (nbr_off[n+1], nbr_idx[nnz]) and must be symmetric
 *     without self edges.
 *   - Colours are 0-based; points of one colour share no edge.
 *   - Flow condition: rho_inf = 1, p_inf = 1/gamma, velocity
 *     M (cos aoa, sin aoa).
 *   - "on_device" pointers are HIP device pointers (e.g. a torch tensor's
 *     data_ptr()); otherwise host pointers.  The caller owns every pointer it
 *     passes; create calls copy what they need.
 *   - All GPU work of a state is ordered on the HIP stream given at
 *     lskum_state_create (NULL = the default stream).  Calls that return
 *     host data synchronise that stream.
 */
#ifndef LSKUM_H
#define LSKUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LSKUM_OK = 0,
    LSKUM_ERR_ARG = -1,              /* invalid argument or size */
    LSKUM_ERR_CONNECTIVITY = -2,     /* asymmetric CSR, self edge, bad index */
    LSKUM_ERR_DEGENERATE = -3,       /* full stencil without a 2x2 LS solve */
    LSKUM_ERR_COLOURING = -4,        /* given colours put an edge in a colour */
    LSKUM_ERR_NONPHYSICAL = -5,      /* rho <= 0, p <= 0 or q~ with beta <= 0 */
    LSKUM_ERR_NOT_CONVERGED = -6,    /* max_iters reached (report is filled) */
    LSKUM_ERR_HIP = -7,              /* HIP runtime error */
    LSKUM_ERR_OOM = -8               /* device allocation failed */
};

enum { LSKUM_JVP_EXACT = 0, LSKUM_JVP_FLUXDIFF = 1 };
enum { LSKUM_FP64 = 0, LSKUM_MIXED = 1 };
enum { LSKUM_ANANDH = 0, LSKUM_MANISH = 1 };
enum { LSKUM_IMPLICIT = 0, LSKUM_EXPLICIT = 1 };
enum { LSKUM_ORDER_COLOUR = 0, LSKUM_ORDER_WALL_FIRST = 1 };
enum { LSKUM_FARFIELD_DIRICHLET = 0, LSKUM_FARFIELD_KINETIC = 1 };

typedef struct lskum_cloud lskum_cloud; /* device geometry, CSR, colours */
typedef struct lskum_state lskum_state; /* device flow state and work arrays */
typedef struct lskum_batch lskum_batch; /* many flow conditions iterated together */

typedef struct {
    double gamma;       /* ratio of specific heats (1.4) */
    double cfl;         /* CFL number of the local time step
                           dt0 = cfl * min_i |r_i - r_0| / (|u_0| + a_0) */
    int32_t inner_iters;/* inner iterations of the q-derivative defect
                           correction (eq. 16) after the first-order pass */
    int32_t jvp_mode;   /* LSKUM_JVP_EXACT or LSKUM_JVP_FLUXDIFF */
    int32_t precision;  /* LSKUM_FP64, or LSKUM_MIXED: fp32 sweeps and
                           Jacobian products, fp64 residual and update */
    int32_t check_every;/* lskum_solve reads the residual every k steps */
    double tol_rel;     /* lskum_solve stops when res <= tol_rel * res_fs */
    int32_t max_iters;  /* lskum_solve iteration cap */
    int32_t sweep_lanes;    /* lanes per point in the sweep kernels: 1, 2, 4, 8,
                               16; 0 = library choice */
    int32_t residual_lanes; /* lanes per point in the residual kernel: 1, 2, 4,
                               8; 0 = library choice */
    int32_t limiter;        /* 0: none (the paper's scheme); 1: Venkatakrishnan
                               limiter on the q~ reconstruction (an addition
                               for flows with shocks) */
    double limiter_k;       /* limiter constant K: eps^2 = (K h)^3, h the
                               nearest-neighbour distance */
    int32_t variant;        /* LSKUM_ANANDH: scalar diagonal of Anandhanarayanan
                               et al. (eq. 34-35); LSKUM_MANISH: Manish et al.
                               (eq. 29-33, 36-38): diagonal with rho(A)/2 and
                               the term S on the forward right-hand side R - S,
                               S from the previous iteration's increment (zero
                               after state creation or a new U) */
    int32_t scheme;         /* LSKUM_IMPLICIT: the LU-SGS iteration above;
                               LSKUM_EXPLICIT: the paper's explicit solver,
                               U <- U - dt R with the same local time step
                               (the CFL number must suit an explicit scheme,
                               e.g. 0.4); no sweeps, no increment kept */
    int32_t order;          /* LSKUM_ORDER_COLOUR: each sweep visits the colours
                               in turn (Algorithm 6); LSKUM_ORDER_WALL_FIRST:
                               wall, interior and outer points in turn, colours
                               ascending (forward) / descending (backward)
                               within each (Algorithm 5); a point still sums
                               over its lower-/upper-colour neighbours, reading
                               what the increment array holds (zero at the
                               start of the forward sweep) */
    int32_t farfield;       /* LSKUM_FARFIELD_DIRICHLET: outer points stay at
                               the free stream (the paper names no outer
                               boundary treatment).  LSKUM_FARFIELD_KINETIC (a
                               reading of our own): an outer point with
                               outward normal n takes the splits t+, t- and
                               n+ (inner side) of its own stencil in its frame,
                               and the molecules entering from outside from a
                               free-stream ghost one nearest-neighbour distance
                               h outside, R += (G_n-(U_inf) - G_n-(U_0)) / h,
                               with (1/h) max(a - u_n, 0) in the diagonal
                               (eq. 34-35; Anandhanarayanan variant); outer
                               points are then swept and updated like the
                               others and stay out of the residual norm */
    int32_t qgrad_lanes;    /* q-derivative kernels: 0 = library choice (each
                               64-point tile -- 16 points by 4 rows when the
                               points are stored row by row, else 64
                               consecutive points -- stages its points'
                               neighbours in LDS, four lanes per point, when
                               every tile's neighbour list fits; direct
                               gathers otherwise);
                               1, 2, 4, 8 = direct gathers with that many
                               lanes per point (the same sums; the forms can
                               differ in the last bits). */
} lskum_params;

typedef struct {
    int32_t iters;      /* iterations run */
    int32_t status;     /* LSKUM_OK or the error that stopped the solve */
    double res_fs;      /* residual norm of the free-stream state */
    double res_first;   /* residual norm at the first iteration of the solve */
    double res_final;   /* residual norm at the last iteration */
    double seconds;     /* wall time of the iteration loop */
    double cl, cd;      /* force coefficients of the final state */
} lskum_report;

/* Fills p with the defaults: gamma 1.4, cfl 100, inner_iters 1, exact JVP,
 * fp64, check_every 10, tol_rel 1e-8, max_iters 20000, lanes 0 (library
 * choice), no limiter (limiter_k 5), Anandhanarayanan variant, implicit
 * scheme, colour order, Dirichlet far field. */
void lskum_default_params(lskum_params* p);

/* Creates a cloud on the current HIP device from host arrays of n points.
 * colour == NULL runs the greedy colouring of Algorithm 4 on the host
 * (point 0 first, then neighbours in storage/CSR order each take the smallest
 * colour absent from their own neighbours); otherwise the given colours are
 * validated.  tx/ty may be NULL when the cloud has no wall points.
 * Errors: ARG, CONNECTIVITY, DEGENERATE (a point whose full-stencil
 * least-squares matrix is singular), COLOURING, HIP, OOM. */
int lskum_cloud_create(int64_t n, const double* x, const double* y, const int8_t* type,
                       const double* tx, const double* ty, const int32_t* nbr_off,
                       const int32_t* nbr_idx, const int32_t* colour, lskum_cloud** out);

/* Point count, edge count, colour count and the number of degenerate split
 * stencils (fewer than two members or a singular 2x2 system; such a half
 * stencil contributes nothing). */
int lskum_cloud_info(const lskum_cloud* c, int64_t* n, int64_t* nnz, int32_t* n_colours,
                     int64_t* n_degenerate);

/* Copies the 0-based colours (n int32) to host memory. */
int lskum_cloud_colours(const lskum_cloud* c, int32_t* colour_out);

void lskum_cloud_destroy(lskum_cloud* c);

/* Creates a state on the cloud's device, initialised to the free stream
 * (wall points keep only the tangential velocity), and evaluates res_fs, the
 * residual norm of that free-stream state.  hip_stream is a hipStream_t or
 * NULL.  The cloud must outlive the state. */
int lskum_state_create(const lskum_cloud* c, double mach, double aoa_deg,
                       const lskum_params* prm, void* hip_stream, lskum_state** out);

void lskum_state_destroy(lskum_state* s);

/* Replaces the parameters of a state (the free-stream residual is kept). */
int lskum_state_set_params(lskum_state* s, const lskum_params* prm);

/* Sets / gets the conserved state U ([4][n] doubles). set_U does not
 * re-project wall velocities. */
int lskum_state_set_U(lskum_state* s, const double* U, int on_device);
int lskum_state_get_U(lskum_state* s, double* U, int on_device);

/* Increment dU ([4][n]) of the last lskum_lusgs_step. */
int lskum_state_get_dU(lskum_state* s, double* dU, int on_device);

/* Residual of the current state (Algorithm 1 steps q_variables,
 * q_derivatives, flux_residual).  R ([4][n], may be NULL) receives it;
 * *res (may be NULL) the norm sqrt(sum_{non-outer} R_rho^2) / n_non_outer.
 * Errors: NONPHYSICAL when a q~ has beta <= 0. */
int lskum_residual(lskum_state* s, double* R, int on_device, double* res);

/* Allocation-free residual, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the residual of lskum_residual for the flow condition
 * (mach, aoa_deg) and the parameters' gamma, cfl, inner_iters, limiter,
 * limiter_k and farfield, on the given cloud, with no state object.
 *   U    device, [4][n] doubles (SoA), read;
 *   R    device, [4][n] doubles, written (may be NULL);
 *   res  device, 2 doubles written: [0] the norm of lskum_residual, [1] 1.0 if
 *        a non-physical state (rho <= 0, p <= 0, or a q~ with beta <= 0) was
 *        met, else 0.0.
 * Every work array lies in a fixed device array of the library (64 MiB per
 * GPU, held until the process ends), so clouds are limited to
 * lskum_residual_noalloc_max_points() points; calls on one GPU share it, and
 * calls that overlap on one GPU (other streams or threads) race.  All work is
 * enqueued on hip_stream (NULL = the default stream) and nothing is
 * synchronised; the call allocates nothing, copies nothing between host and
 * device, and issues no memset (graph capture is allowed).  The first call on
 * a device looks up the array's device address (HIP symbol lookup).
 * Errors: ARG (NULL pointer, invalid parameters or flow condition, too many
 * points, the cloud on another device than the current one), HIP. */
int lskum_residual_noalloc(const lskum_cloud* c, double mach, double aoa_deg,
                           const lskum_params* p, const double* U, double* R, double* res,
                           void* hip_stream);
int64_t lskum_residual_noalloc_max_points(void);

/* q-derivatives of the current state after the first-order pass and
 * inner_iters inner iterations (eq. 16): qx, qy ([4][n]). */
int lskum_q_derivatives(lskum_state* s, double* qx, double* qy, int on_device);

/* One iteration of the state's scheme.  Implicit: residual, local time step
 * and diagonal, forward and backward colour sweeps (eq. 27), U += dU.
 * Explicit: residual, U -= dt R.  *res (may be NULL) receives
 * the norm of the residual of the state the step started from; passing NULL
 * keeps the step free of host synchronisation.
 * Errors: NONPHYSICAL (the state then holds the non-physical result). */
int lskum_lusgs_step(lskum_state* s, double* res);

/* One lskum_lusgs_step launched eagerly with HIP events between its
 * phases on the state's stream; ms[6] receives the GPU milliseconds of
 * (0) q-derivatives, (1) residual kernel, (2) residual norm, (3) forward
 * sweep, (4) backward sweep, (5) state update (0 for the sweeps of the
 * explicit scheme).  Synchronises the stream. */
int lskum_step_timed(lskum_state* s, double* ms);

/* Iterates lusgs steps until res <= tol_rel * res_fs or max_iters; the
 * iteration is captured once in a HIP graph (check_every iterations) and
 * replayed; convergence is tested on the device, so the state stops at the
 * first iteration whose residual meets the tolerance.  rep may be NULL.
 * Returns NOT_CONVERGED when max_iters is reached (report filled). */
int lskum_solve(lskum_state* s, lskum_report* rep);

/* Lift and drag coefficients of the current state from the wall pressure:
 * trapezoidal pressure on each edge of the wall polygon, unit chord,
 * dynamic pressure M^2/2. */
int lskum_forces(lskum_state* s, double* cl, double* cd);

/* ---- Batches: many flow conditions (Mach, AoA) on one or more clouds,
 * iterated together.  The batch holds one copy of its cloud per condition;
 * every kernel of an iteration (each colour phase of both sweeps included)
 * is one launch over all conditions, colour c of every cloud in phase c.
 * Conditions that reach their tolerance (tol_rel times their own free-stream
 * residual) or fail (non-finite residual) retire on the device and skip
 * further work.  The clouds must outlive the batch creation only. */

/* Creates a batch of n_cond conditions; condition k uses
 * clouds[cond_cloud[k]] and (mach[k], aoa_deg[k]).  All conditions start at
 * their free stream.  Errors: ARG, HIP, OOM. */
int lskum_batch_create(int32_t n_clouds, const lskum_cloud* const* clouds, int32_t n_cond,
                       const int32_t* cond_cloud, const double* mach, const double* aoa_deg,
                       const lskum_params* prm, void* hip_stream, lskum_batch** out);

/* Total points and edges over all conditions, and colour phases. */
int lskum_batch_info(const lskum_batch* b, int64_t* n_points, int64_t* nnz, int32_t* n_colours);

int lskum_batch_set_params(lskum_batch* b, const lskum_params* prm);

/* Sets the CFL number of each condition (cfl: n_cond finite values > 0, host
 * memory, copied): the local time step of eq. (25) uses its condition's
 * value, so conditions with strong shocks can run a smaller CFL than the rest
 * of the batch (a choice of the caller; the paper uses one CFL).  Until this
 * is called, and again after lskum_batch_set_params changes params.cfl,
 * every condition uses params.cfl.  Errors: LSKUM_ERR_ARG for NULL or a
 * non-positive value. */
int lskum_batch_set_cfl(lskum_batch* b, const double* cfl);

/* Copies the current CFL number of each condition (n_cond doubles, host). */
int lskum_batch_get_cfl(const lskum_batch* b, double* cfl);

/* Residual-driven CFL control (an addition: the paper runs one CFL number;
 * strong-shock conditions of a batch can stall in a limit cycle at a CFL
 * number that suits the rest).  During lskum_batch_solve the host reads every
 * condition's residual norm after each replay of check_every iterations; at
 * the end of each window of `window` iterations, a condition still iterating
 * whose lowest residual over the window is not below its lowest residual over
 * the previous window has its CFL number multiplied by `factor`, but not
 * below cfl_min; the new numbers act from the next iteration on.  The
 * window's memory persists across lskum_batch_solve calls and is cleared by
 * this call.  window = 0 (the default) switches the control off.
 * Errors: ARG unless window >= 0 and, for window > 0, 0 < factor < 1 and
 * cfl_min > 0. */
int lskum_batch_set_cfl_control(lskum_batch* b, int32_t window, double factor, double cfl_min);

/* Solves all conditions (graph-replayed iterations, device-side retirement)
 * until all retire or max_iters.  reps (n_cond entries, may be NULL): per
 * condition iterations, status (OK, NOT_CONVERGED or NONPHYSICAL), residual
 * norms, the wall time at which it retired, CL and CD.  *seconds_total (may be
 * NULL): wall time of the whole solve.  Returns the first non-OK status. */
int lskum_batch_solve(lskum_batch* b, lskum_report* reps, double* seconds_total);

/* One iteration of all conditions with per-phase GPU times (as
 * lskum_step_timed). */
int lskum_batch_step_timed(lskum_batch* b, double* ms);

/* Gets / sets the state ([4][n_k] doubles) of condition k. */
int lskum_batch_get_U(lskum_batch* b, int32_t cond, double* U, int on_device);
int lskum_batch_set_U(lskum_batch* b, int32_t cond, const double* U, int on_device);

/* Autotuner: times `iters` iterations with 1, 2, 4, 8 (and, for the sweeps,
 * 16) lanes per point and keeps the fastest lane count for the sweep and for
 * the residual kernels, and times the q-derivative passes in their LDS-tiled
 * form and with direct gathers at 1, 2, 4, 8 lanes and keeps the fastest
 * (written to *sweep_lanes, *residual_lanes, *qgrad_lanes as lskum_params
 * values; any of the three may be NULL).  The batch's state is restored
 * afterwards. */
int lskum_batch_autotune(lskum_batch* b, int32_t iters, int32_t* sweep_lanes,
                         int32_t* residual_lanes, int32_t* qgrad_lanes);

void lskum_batch_destroy(lskum_batch* b);

/* ---- Learned warm start (an addition; the paper starts every solve from
 * the free stream).  A per-point perceptron 5 -> 128 -> 128 -> 128 -> 4 with
 * GELU (erf form) hidden layers maps the features of a point to its
 * deviation from the free stream, (rho - 1, u - u_inf, v - v_inf,
 * gamma p - 1).  Features: f0 = (x - 1/2) / (1 + r), f1 = y / (1 + r) with
 * r = |(x - 1/2, y)|; f2 = 2 d / (d + 0.1) - 1 with d the distance to the
 * nearest wall point of the point's own cloud; f3 = (M - 0.6) / 0.25;
 * f4 = (aoa_deg - 2) / 6.
 * Numerics: bfloat16 copies (round to nearest even) of the weights, the
 * features and each hidden activation; fp32 accumulation (the two
 * 128 x 128 layers and their backward products on the matrix cores); the
 * backward pass rounds the pre-activation gradients of layers 3 and 2 to
 * bfloat16; fp32 master weights and Adam moments.
 * Parameters: one flat fp32 vector of LSKUM_MLP_PARAMS entries laid out as
 * W1[128][5], b1[128], W2[128][128], b2, W3[128][128], b3, W4[4][128], b4[4]
 * (W[out][in]).  Loss: mean over rows and outputs of (y - t)^2.
 * Feature rows X are [m][5] fp32 and target/prediction rows [m][4] fp32,
 * row-major, always device pointers.  Work runs on the stream given at
 * lskum_mlp_create (NULL = a private stream); calls that take a state or
 * batch synchronise both streams. */
#define LSKUM_MLP_PARAMS 34308
#define LSKUM_MLP_FEATURES 5
#define LSKUM_MLP_OUTPUTS 4
typedef struct lskum_mlp lskum_mlp;

/* Creates a network on the current device with Glorot-uniform weights drawn
 * from splitmix64(seed) (zero biases) and a workspace of max_rows rows
 * (the largest m of lskum_mlp_gradient / train_step, and the minibatch
 * limit of lskum_mlp_train).  Errors: ARG (max_rows < 1 or > 2^24), HIP, OOM. */
int lskum_mlp_create(uint64_t seed, int64_t max_rows, void* hip_stream, lskum_mlp** out);
void lskum_mlp_destroy(lskum_mlp* net);

/* Copies the fp32 parameters out / in (LSKUM_MLP_PARAMS floats).  Setting
 * the parameters also clears the Adam moments and step count. */
int lskum_mlp_get_params(lskum_mlp* net, float* theta, int on_device);
int lskum_mlp_set_params(lskum_mlp* net, const float* theta, int on_device);

/* Predictions Y[m][4] for features X[m][5] (any m >= 0; processed in chunks
 * of max_rows). */
int lskum_mlp_forward(lskum_mlp* net, int64_t m, const float* X, float* Y);

/* Loss (host double, may be NULL) and its gradient with respect to the
 * parameters (device, LSKUM_MLP_PARAMS floats, may be NULL) over m rows
 * (1 <= m <= max_rows), without changing the parameters. */
int lskum_mlp_gradient(lskum_mlp* net, int64_t m, const float* X, const float* T, float* grad,
                       double* loss);

/* One full-batch Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate
 * lr) on m rows (1 <= m <= max_rows); *loss (may be NULL) is the loss before
 * the step. */
int lskum_mlp_train_step(lskum_mlp* net, int64_t m, const float* X, const float* T, float lr,
                         double* loss);

/* Minibatch Adam training on a device data set of n rows: `steps` steps of
 * `batch` rows (batch <= max_rows); row r of step t is data-set row
 * floor(h n / 2^64), h = splitmix64(seed + t batch + r).  The learning rate
 * decays from lr to lr_final on a half cosine.  loss_hist (host, `steps`
 * doubles, may be NULL): minibatch loss of each step; *seconds (may be NULL):
 * GPU wall time. */
int lskum_mlp_train(lskum_mlp* net, int64_t n, const float* X, const float* T, int32_t steps,
                    int32_t batch, float lr, float lr_final, uint64_t seed, double* loss_hist,
                    double* seconds);

/* Features X[n][5] of every point of a state / batch (points in storage
 * order, conditions one after the other) and, with T != NULL, training
 * targets T[n][4] from the current state U. */
int lskum_state_features(lskum_state* s, float* X, float* T);
int lskum_batch_features(lskum_batch* b, float* X, float* T);

/* Warm start: sets U of every point to the network's prediction (outer
 * points at the free stream, wall points with tangential velocity only),
 * then checks each condition's residual norm: a condition whose
 * prediction is non-finite or non-physical (rho < 0.05 or gamma p < 0.05),
 * or whose residual is not below its free-stream residual, goes back to the
 * free stream.  fallback / res_warm (host, 1 entry for a state, n_cond for a
 * batch; may be NULL): 1 where the free stream was kept, and the residual
 * norm of the predicted state.  The tolerance of later solves stays
 * tol_rel times the free-stream residual. */
int lskum_mlp_warm_start(lskum_mlp* net, lskum_state* s, int32_t* fallback, double* res_warm);
int lskum_mlp_warm_start_batch(lskum_mlp* net, lskum_batch* b, int32_t* fallback,
                               double* res_warm);

/* Message of the last error on the calling thread ("" if none). */
const char* lskum_last_error(void);

/* Identifier of the sources the library was compiled from (16 hex digits of
 * a SHA-256 over the sources and headers; "unknown" when not set at build
 * time), so that callers can refuse a binary that does not match the sources
 * they were written against. */
const char* lskum_build_hash(void);

#ifdef __cplusplus
}
#endif

#endif /* LSKUM_H */
