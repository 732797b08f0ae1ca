/*
 * matamg: material-aware smoothed-aggregation AMG and AMG-preconditioned CG
 * for the material-weighted Laplacian -div(sigma(x) grad u) = f on MI355X
 * (gfx950).
 *
 * Method: Firmbach, Phillips, Glusa, Popp, Siefert, Mayr, "Smoothed
 * aggregation algebraic multigrid for problems with heterogeneous and
 * anisotropic materials".  Section numbers below refer to that paper.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - extern "C", no exceptions cross the boundary; every call returns an
 *   amg_status and leaves a thread-local message for amg_last_error().
 * - Pointers are borrowed for the duration of the call; the library copies
 *   what it keeps.  `kind` says whether array arguments are host memory
 *   (AMG_PTR_HOST) or device memory of the current HIP device
 *   (AMG_PTR_DEVICE).  Host arrays are copied to the device inside the call.
 * - `hip_stream` is a hipStream_t (NULL = the default stream).  All device
 *   work of the call is ordered on it; calls that return sizes or statuses
 *   synchronise it before returning.
 * - Matrices are CSR with int32 row pointers (n+1) and int32 column indices
 *   sorted ascending and unique within each row, FP64 values.  A must be
 *   square and symmetric in pattern and value.
 * - A hierarchy is owned by the library until amg_free().  Distinct
 *   hierarchies may be used concurrently on distinct streams; one hierarchy
 *   is not re-entrant.
 */
#ifndef MATAMG_AMG_H
#define MATAMG_AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMG_OK = 0,
    AMG_ERR_INVALID_ARG = 1,        /* malformed CSR, bad sizes or options */
    AMG_ERR_OUT_OF_MEMORY = 2,      /* device or host allocation failed */
    AMG_ERR_HIP = 3,                /* a HIP runtime call failed */
    AMG_ERR_NOT_SPD = 4,            /* sigma not SPD, or coarse Cholesky failed */
    AMG_ERR_COARSENING_STAGNATED = 5, /* level cap reached above max_coarse, or no reduction */
    AMG_ERR_NOT_CONVERGED = 6,      /* max_iter reached above tol */
    AMG_ERR_BREAKDOWN = 7,          /* CG breakdown: p^T A p <= 0 or non-finite */
    AMG_ERR_BUDGET = 8              /* serving: request larger than the HBM budget */
} amg_status;

typedef enum { AMG_PTR_HOST = 0, AMG_PTR_DEVICE = 1 } amg_ptr_kind;

/* strength-of-connection measure (section 2.1 and section 3) */
typedef enum {
    AMG_SOC_MATERIAL = 0, /* material distance Laplacian (the paper's measure) */
    AMG_SOC_DISTANCE = 1, /* Euclidean distance Laplacian */
    AMG_SOC_SA = 2        /* classical |A_ij| / sqrt(|A_ii A_jj|) */
} amg_soc;

/* dropping criterion C (section 2.1): pointwise |S_ij| >= theta, or cut-drop
 * (each row's strengths in decreasing order are cut after the first pair
 * with theta * s_k >= s_{k+1}; kept where both rows keep the entry) */
typedef enum { AMG_DROP_POINTWISE = 0, AMG_DROP_CUT = 1 } amg_drop;
typedef enum { AMG_PREC_FP64 = 0, AMG_PREC_FP32_HIER = 1 } amg_precision;
/* smoother (solver settings of the numerical section; Chebyshev is the
 * paper's):
 *   CHEBYSHEV      Jacobi-preconditioned Chebyshev of degree cheb_degree on
 *                  [beta/cheb_ratio, beta], beta = cheb_boost * lambda, with
 *                  lambda the level's power-method estimate of rho(D^{-1}A)
 *   JACOBI         jacobi_sweeps sweeps of x <- x + w D^{-1}(b - A x) with
 *                  the fixed weight w = jacobi_omega.  The V-cycle is
 *                  symmetric positive definite only if w rho(D^{-1}A) < 2 on
 *                  every level; 3D Q1 operators (stretched, layered or
 *                  rotated) reach rho(D^{-1}A) of 3-4.5, where w = 2/3 breaks
 *                  this and CG may stall or fail
 *   JACOBI_SCALED  the same sweeps with w_l = jacobi_omega * 2 / beta_l per
 *                  level (beta_l as for Chebyshev): w_l = jacobi_omega where
 *                  beta_l = 2 (the five-point Laplacian, for which 2/3 is the
 *                  classical weight), and w_l beta_l = 2 jacobi_omega < 2
 *                  keeps the V-cycle positive definite for jacobi_omega < 1 */
typedef enum { AMG_SMOOTH_CHEBYSHEV = 0, AMG_SMOOTH_JACOBI = 1, AMG_SMOOTH_JACOBI_SCALED = 2 } amg_smoother;

/* Setup and solve options.  Defaults (amg_options_default) follow the
 * numerical section: pointwise dropping, 2nd-order Chebyshev smoothing,
 * direct coarse solve, coarsening to <= 5000 unknowns, at most 10 levels. */
typedef struct {
    int32_t dim;            /* spatial dimension of coords / tensors: 1, 2 or 3 */
    double theta;           /* drop tolerance (0.08) */
    int32_t soc;            /* amg_soc */
    int32_t drop;           /* amg_drop */
    int32_t smoother;       /* amg_smoother */
    int32_t max_coarse;     /* stop coarsening at <= this many unknowns (5000) */
    int32_t max_levels;     /* level cap, <= 16 (10) */
    int32_t cheb_degree;    /* Chebyshev polynomial degree (2) */
    double cheb_ratio;      /* eigen-interval [lambda/ratio, lambda] (30) */
    double cheb_boost;      /* lambda = boost * power-method estimate (1.1) */
    int32_t power_iters;    /* power-method steps for omega and Chebyshev (10) */
    double omega_sym;       /* prolongator damping numerator (4/3) */
    double jacobi_omega;    /* damped-Jacobi weight, > 0 (2/3) */
    int32_t jacobi_sweeps;  /* damped-Jacobi sweeps per smoothing (2) */
    int32_t precision;      /* amg_precision */
    uint64_t seed;          /* aggregation priorities and power-method starts */
} amg_options;

typedef struct amg_hierarchy amg_hierarchy;

typedef struct {
    int32_t iterations;     /* preconditioned CG steps taken */
    double rel_res_true;    /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit */
    double t_solve_s;       /* device-synchronised wall time of the solve */
    int32_t status;         /* amg_status of the solve */
} amg_solve_info;

typedef struct {
    int32_t levels;
    int64_t n[16], nnz[16], nnz_p[16]; /* rows, nnz(A), nnz(P) per level */
    int32_t mis_rounds[16];
    double omega[16], lam_pf[16], lam_cheb[16];
    double op_complexity;              /* sum nnz(A_l) / nnz(A_1) */
    double vcycle_alg_bytes;           /* algorithmic HBM bytes of one V-cycle */
    double t_setup_s;
    int64_t device_bytes;              /* device memory held by the hierarchy */
    int64_t device_peak_bytes;         /* most device memory held at once during setup and solves */
    double t_update_s;                 /* duration of the last amg_update_values (0: none yet) */
} amg_hierarchy_stats;

/* Fill *o with the defaults listed above (dim = 3). */
amg_status amg_options_default(amg_options* o);

/*
 * Build the multigrid hierarchy for A (sections 2 and 3):
 *   level 1: Dirichlet rows (every stored off-diagonal exactly zero) are
 *   isolated; nodal tensors are the Clement patch means of elem_sigma;
 *   every level: material distance Laplacian strength, pointwise dropping,
 *   distance-2 MIS aggregation, tentative and filtered-Jacobi-smoothed
 *   prolongator (1-norm diagonal), Galerkin product P^T A P, aggregate-mean
 *   coordinates and tensors; coarsest level: dense FP64 Cholesky.
 *
 * n          rows of A (> 0)
 * rowptr,col,val  A in CSR (see conventions)
 * nelem, nodes_per_elem, elem_nodes  element -> node connectivity,
 *            int32 [nelem][nodes_per_elem], node ids in [0, n)
 * elem_sigma FP64 [nelem][dim][dim] symmetric positive definite tensors
 * coords     FP64 [n][dim] nodal coordinates
 * opt        options (NULL = defaults with dim 3)
 * out        receives the new hierarchy
 * Errors: INVALID_ARG (bad sizes, unsorted/out-of-range columns, bad options,
 * a NaN or infinity in val, coords or elem_sigma), NOT_SPD (a nodal tensor is
 * not SPD, or the coarse Cholesky fails), COARSENING_STAGNATED,
 * OUT_OF_MEMORY, HIP.  On error *out is NULL.
 */
amg_status amg_setup(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                     int64_t nelem, int32_t nodes_per_elem, const int32_t* elem_nodes,
                     const double* elem_sigma, const double* coords, const amg_options* opt,
                     amg_ptr_kind kind, void* hip_stream, amg_hierarchy** out);

/*
 * Solve A x = b by CG preconditioned with one V-cycle (Algorithm "Vcycle",
 * zero initial guess on every level) per step.  Stops when the recurrence
 * residual satisfies ||r||/||b|| <= tol and the recomputed FP64 residual
 * confirms it (otherwise the true residual replaces the recurrence one and
 * the iteration continues).  b and x are FP64 [n]; x holds the initial guess
 * on entry and the solution on exit.  The outer CG, its dot products and
 * residual recomputation are FP64 in both precisions.
 * Errors: NOT_CONVERGED, BREAKDOWN (x holds the last iterate), INVALID_ARG
 * (null vectors, tol <= 0, max_iter < 0, a NaN or infinity in b or in the
 * initial guess, or a 2-norm of b that overflows; x is left as it was).
 */
amg_status amg_pcg_solve(amg_hierarchy* h, const double* b, double* x, double tol, int32_t max_iter,
                         amg_ptr_kind kind, void* hip_stream, amg_solve_info* info);

/*
 * amg_pcg_solve without any allocation, for callers that cannot allocate
 * device memory during a solve (tight serving loops, harnesses that forbid
 * it, work ordered among captured graphs).  The same preconditioned CG with
 * the same kernels and stopping rule, launched directly on hip_stream (no
 * captured graphs, no solve stream of the library): results are bitwise
 * those of amg_pcg_solve with device pointers.
 *
 * b, x   FP64 [n] device pointers of the current device; x holds the initial
 *        guess on entry and is iterated in place (on NOT_CONVERGED or
 *        BREAKDOWN it holds the last iterate)
 * Workspace: the CG vectors, scalars and reduction partials live in one
 * fixed 256 MiB device array of the library per device (allocated when the
 * library is loaded, held until the process ends): the finest level may
 * have at most about 8.3 million unknowns (4 n doubles plus the partials of
 * its row blocks); a larger hierarchy gets INVALID_ARG with the bytes
 * needed.  The array keeps the last call's contents.  Every call on one
 * device shares it, so calls that overlap on one device (any hierarchies,
 * any streams, any threads) race and must be serialised by the caller.
 * The call returns after synchronising hip_stream.
 * Errors: INVALID_ARG (null vectors, tol <= 0, max_iter < 0, workspace too
 * small, a NaN or infinity in b or in the initial guess), NOT_CONVERGED,
 * BREAKDOWN, HIP.
 */
amg_status amg_pcg_solve_noalloc(amg_hierarchy* h, const double* b, double* x, double tol, int32_t max_iter,
                                 void* hip_stream, amg_solve_info* info);

/*
 * New values of A on the setup's sparsity pattern, for instance after a
 * change of material.  The paper weighs the material measure's higher setup
 * cost against solves that reuse one hierarchy (numerical results, thermally
 * activated batteries); this keeps the costly, value-independent part of the
 * setup.  The drop masks, aggregates,
 * number of levels, coordinates and nodal tensors of amg_setup are kept; the
 * diagonals, filtered matrices, damping factors, prolongators, restrictions,
 * Galerkin products, smoother bounds, coarse inverse and FP32 copies are
 * recomputed from val exactly as amg_setup computes them.  For a material
 * that leaves the strength measure unchanged the result is the hierarchy
 * amg_setup would build; otherwise it is a valid preconditioner built on the
 * old coarsening (its quality may differ from a fresh setup's).
 *
 * val   FP64 [nnz] values on the rowptr/col pattern given to amg_setup
 * kind  whether val is a host or a device pointer; the call returns after
 *       the update is complete on hip_stream
 * Errors: INVALID_ARG (null arguments, bad kind, a NaN or infinity in val,
 * or the rows whose off-diagonals are all exactly zero -- the Dirichlet
 * rows -- differ from the setup's; the hierarchy is left unchanged), NOT_SPD
 * (the new coarsest operator is not positive definite; the hierarchy must
 * then be freed), HIP.
 * Not to be called while a solve on the same hierarchy is running.
 */
amg_status amg_update_values(amg_hierarchy* h, const double* val, amg_ptr_kind kind, void* hip_stream);

/* z = M^{-1} r: one V-cycle.  r, z FP64 [n] device pointers. */
amg_status amg_vcycle(amg_hierarchy* h, const double* r, double* z, void* hip_stream);

/* y = A_level x (FP64), device pointers; for kernel tests and benchmarks. */
amg_status amg_level_spmv(amg_hierarchy* h, int32_t level, const double* x, double* y, void* hip_stream);

amg_status amg_hierarchy_info(const amg_hierarchy* h, amg_hierarchy_stats* s);

/* Copy level data to host memory (for parity checks):
 * agg  int32 [n_level] aggregate id per node (-1: Dirichlet), levels < last
 * mask uint8 [nnz_level] kept flag per stored entry of A_level, levels < last
 * csr  which = 0: A_level, 1: P_level, 2: R_level; rowptr [rows+1], col, val
 * aux  which = 0: coordinates [n][dim], 1: nodal tensors [n][dim(dim+1)/2]
 *      (upper triangle row-wise), 2: Dirichlet flags as doubles (level 0),
 *      3: strength values S per stored entry. */
amg_status amg_get_aggregates(const amg_hierarchy* h, int32_t level, int32_t* agg);
amg_status amg_get_soc_mask(const amg_hierarchy* h, int32_t level, uint8_t* mask);
amg_status amg_get_level_csr(const amg_hierarchy* h, int32_t level, int32_t which, int32_t* rowptr,
                             int32_t* col, double* val);
amg_status amg_get_level_aux(const amg_hierarchy* h, int32_t level, int32_t which, double* out);

/* Roofline timing of the dominant kernel (benchmarks): runs `reps`
 * back-to-back launches of the level's fused smoother step (the Chebyshev
 * SpMV with its vector epilogue) on the hierarchy's own work vectors between
 * two HIP events recorded on `hip_stream`, and returns the average launch
 * duration in ms and the algorithmic bytes one launch moves: matrix values,
 * column indices and row pointers once, the gathered iterate once, b, D^{-1}
 * and the direction read, the direction and the new iterate written.
 * Overwrites the level's work vectors.  Errors: INVALID_ARG (no smoother on
 * that level, reps < 1). */
amg_status amg_time_smoother(amg_hierarchy* h, int32_t level, int32_t reps, void* hip_stream, double* avg_ms,
                             double* bytes_per_launch);

/* Frees a hierarchy (null: no-op).  Waits for every stream of the device,
 * then keeps the hierarchy's device buffers in the library (up to 32 GiB per
 * process) for later setups of the same sizes, which skip the runtime's
 * allocation cost; the memory stays reserved to the process.  The hierarchy
 * must not be in use on any stream. */
void amg_free(amg_hierarchy* h);

/* Hands the device buffers kept by amg_free on the current device back to the
 * device's memory pool (for callers that need the memory elsewhere).  Waits
 * for every stream of the device.  bytes (optional, host): the number of
 * bytes handed back.  Errors: HIP. */
amg_status amg_trim_cache(int64_t* bytes);

/* ------------------------------------------------------------------------
 * Serving: a solve server that keeps many hierarchies on the device and
 * advances all their solves together (continuous batching).
 *
 * Requests carry the same problem arrays as amg_setup (host memory, copied
 * inside amg_server_submit, so the caller may free them on return), a
 * right-hand side b, an optional initial guess x0 (NULL = zero), the
 * tolerance and an iteration cap.  Each request is solved exactly as
 * amg_setup + amg_pcg_solve would solve it with the server's options: same
 * hierarchy, same kernels per row block, same CG control (section 4's
 * preconditioned CG with one V-cycle per step), so its result does not
 * depend on which other requests share the device with it.
 *
 * Admission: requests wait in arrival order; the head is admitted once its
 * estimated device-memory peak fits in what the budget has left and fewer
 * than max_active requests are admitted.  A request whose estimate exceeds
 * the whole budget is refused at submission (AMG_ERR_BUDGET).  After setup
 * the reservation shrinks to the bytes the hierarchy keeps resident.
 *
 * Work: setup_workers threads (own HIP streams) build hierarchies of
 * admitted requests while an engine thread runs one preconditioned CG step
 * of every solving request per round as shared launches, one per V-cycle
 * step and level and per CG update, on its own stream; new requests join at
 * the next round and finished ones leave.  All device memory comes from the
 * current device's stream-ordered pool.
 *
 * Thread safety: submit, poll, result and stats may be called from any
 * thread.  amg_server_destroy drops unfinished requests.
 * ------------------------------------------------------------------------ */
typedef struct amg_server amg_server;

typedef struct {
    int64_t submitted, completed, failed, rejected;
    int64_t budget_bytes;         /* the admission budget */
    int64_t reserved_bytes;       /* reserved now by admitted requests */
    int64_t peak_reserved_bytes;  /* most reserved at once */
    int32_t active;               /* admitted, unfinished requests */
    int64_t waiting;              /* submitted, not yet admitted */
    int64_t steps;                /* batched CG rounds run */
    int64_t launches;             /* kernel launches issued by those rounds */
    double mean_batch;            /* mean number of requests per round */
    int64_t max_batch;            /* most requests in one round */
    int64_t estimate_exceeded;    /* requests whose setup peak exceeded the estimate */
} amg_server_stats;

typedef struct {
    double t_arrival, t_admit, t_setup_done, t_done; /* seconds since amg_server_create */
    int64_t est_bytes;            /* reservation at admission (estimated setup peak) */
    int64_t setup_peak_bytes;     /* measured setup peak */
    int64_t resident_bytes;       /* kept while solving */
    int32_t levels;
    int32_t max_batch;            /* most requests that shared a round with it */
    int64_t n, nnz;
} amg_request_stats;

/* opt: NULL = defaults; budget_bytes > 0; max_active in [1, 1024];
 * setup_workers in [1, 8].  Uses the current HIP device. */
amg_status amg_server_create(const amg_options* opt, int64_t budget_bytes, int32_t max_active, int32_t setup_workers,
                             amg_server** out);
/* Arrays as in amg_setup (host memory); b, x0 FP64 [n].  On success
 * *request_id identifies the request.  Errors: INVALID_ARG (also for a NaN
 * or infinity in b or x0; one in the problem arrays is reported as the
 * request's INVALID_ARG status when its setup runs), BUDGET. */
amg_status amg_server_submit(amg_server* s, int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                             int64_t nelem, int32_t nodes_per_elem, const int32_t* elem_nodes,
                             const double* elem_sigma, const double* coords, const double* b, const double* x0,
                             double tol, int32_t max_iter, uint64_t* request_id);
/* Up to cap ids of finished requests, each reported once; waits up to
 * timeout_s seconds (0: return at once) while none is ready. */
amg_status amg_server_poll(amg_server* s, double timeout_s, uint64_t* ids, int32_t cap, int32_t* ndone);
/* Hands over a finished request and forgets it: x (host, n doubles, may be
 * NULL) receives the solution, info its solve record (info->status: the
 * request's outcome, e.g. NOT_CONVERGED or a setup error, whose message
 * amg_last_error then returns), rs (may be NULL) its timeline and memory.
 * Returns INVALID_ARG for an unknown, unfinished or already taken id. */
amg_status amg_server_result(amg_server* s, uint64_t id, double* x, amg_solve_info* info, amg_request_stats* rs);
amg_status amg_server_info(amg_server* s, amg_server_stats* out);
/* Dynamic batching delay: when no request is being solved and the first
 * ones become ready while others are still in setup, the engine waits up to
 * `seconds` (in [0, 10]; 0 = start at once, the default) for those setups so
 * that they join the first round; it starts as soon as none is left in
 * setup.  Trades the first requests' latency for larger rounds.  Errors:
 * INVALID_ARG. */
amg_status amg_server_set_batch_wait(amg_server* s, double seconds);
void amg_server_destroy(amg_server* s);
const char* amg_status_string(amg_status s);
const char* amg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MATAMG_AMG_H */
