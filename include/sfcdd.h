/*
 * sfcdd.h - C ABI of the space-filling-curve two-level overlapping Schwarz
 * solver (Griebel, Schweitzer, Troska: "A dimension-oblivious domain
 * decomposition method based on space-filling curves") for MI355X (gfx950).
 *
 * The library solves A x = b (Sec. 3.1, eq. LES) for the assembled
 * (2d+1)-point finite-difference matrix of -sum_j a_j d^2u/dx_j^2 = f on
 * [0,1]^d with homogeneous Dirichlet data, on the anisotropic grid of level
 * vector l (N = prod_j (2^{l_j} - 1) unknowns, eq. dof), preconditioned by
 * the two-level Schwarz operator built from P contiguous, cyclically
 * overlapping pieces of the Z-order curve (Sec. 3.3, Alg. 1-3).
 *
 * Conventions shared by every entry point
 *  - Memory.  The library allocates no device memory.  The caller queries
 *    sfcdd_workspace_size, allocates one device buffer of that size (any
 *    allocator; 256-byte alignment) and passes it to sfcdd_setup; the buffer
 *    must stay alive and untouched until sfcdd_destroy.  (sfcdd_setup_noalloc
 *    instead takes the library's static per-device workspace.)  Vectors passed to the
 *    compute calls are caller-owned device buffers of N doubles.  The context
 *    owns only host memory.
 *  - Streams.  All device work is enqueued on the HIP stream given to
 *    sfcdd_setup (NULL = the default stream), except that sfcdd_setup runs
 *    the coarse setup on an internal stream of the device (created on first
 *    use, shared by all contexts of the device, default priority) and joins
 *    it before returning.  sfcdd_apply_precond and sfcdd_matvec are
 *    asynchronous; sfcdd_setup and sfcdd_solve return after their work is
 *    complete (they synchronise the stream).
 *  - Vector order.  Vectors are in natural order (first coordinate fastest,
 *    point k -> sum_j (k_j - 1) prod_{i<j} n_i) unless params.layout = 1, in
 *    which case they are in curve order (entry p = point sfc_index[p]).
 *  - Errors.  Every call returns an sfcdd_status; nothing aborts and no
 *    exception crosses the ABI.  A message for the last failure is available
 *    from sfcdd_last_error(ctx) (or sfcdd_last_error(NULL) for failures before
 *    a context exists).  A failed call leaves output buffers unspecified.
 *  - Threads.  A context may be used from one host thread at a time.
 */
#ifndef SFCDD_H
#define SFCDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfcdd_ctx sfcdd_ctx;

typedef enum {
  SFCDD_OK = 0,
  SFCDD_EINVAL = -1,     /* invalid argument (null pointer, out-of-range size) */
  SFCDD_ENOMEM = -2,     /* workspace too small / host allocation failed       */
  SFCDD_EDEVICE = -3,    /* a HIP runtime call failed                          */
  SFCDD_ENOTCONV = -4,   /* solve reached max_iter before rtol                 */
  SFCDD_EOVERFLOW = -5,  /* N >= 2^31, or d * max_j l_j > 64 key bits          */
  SFCDD_ENOTSPD = -6,    /* a local or coarse matrix was not positive definite */
  SFCDD_ESTAGNATED = -7  /* the true residual stopped decreasing above rtol: the
                            FP64 rounding floor of the grid lies above rtol      */
} sfcdd_status;

/* Weights of the one-level sum (eqs. w1levprec, Di, omegai): none, the scalar
 * omega_i per subdomain, or D_i = diag(1 / multiplicity) per point (a
 * non-symmetric preconditioner unless every multiplicity agrees: use
 * SFCDD_FCG). */
enum { SFCDD_WEIGHT_NONE = 0, SFCDD_WEIGHT_OMEGA = 1, SFCDD_WEIGHT_D = 2 };
/* Two-level forms: additive C1^{-1} + F (eq. addSW), balanced
 * G^T C1^{-1} G + F (eq. balSW) and deflated G^T C1^{-1} + F (Sec. 3.1),
 * F = R_0^T A_0^{-1} R_0, G = I - A F. */
enum { SFCDD_ADDITIVE = 0, SFCDD_BALANCED = 1, SFCDD_DEFLATED = 2 };
enum { SFCDD_FP64 = 0, SFCDD_FP32 = 1 };
enum { SFCDD_LOCAL_CHOLESKY = 0, SFCDD_LOCAL_INVERSE = 1 };
enum { SFCDD_PCG = 0, SFCDD_FCG = 1, SFCDD_RICHARDSON = 2 };
/* Space-filling curve of the point order (Sec. 3.2, Alg. 1): Z-order
 * (Morton), or Hilbert (Skilling's construction), both at the resolution of
 * the finest direction on the scaled coordinates k_j 2^(max l - l_j). */
enum { SFCDD_CURVE_ZORDER = 0, SFCDD_CURVE_HILBERT = 1 };
/* Precision of the coarse operator (see sfcdd_params.coarse_precision). */
enum { SFCDD_COARSE_AUTO = 0, SFCDD_COARSE_FP64 = 1 };
/* Solver of the coarse problem (see sfcdd_params.coarse_solver). */
enum { SFCDD_COARSE_DENSE = 0, SFCDD_COARSE_ITERATIVE = 1 };
/* Elimination order of the subdomain matrices (see sfcdd_params.local_order). */
enum { SFCDD_ORDER_DIAGONAL = 0, SFCDD_ORDER_CURVE = 1, SFCDD_ORDER_DENSE = 2 };
/* Dissection of the dense coarse matrix (see sfcdd_params.coarse_split). */
enum { SFCDD_SPLIT_AUTO = 0, SFCDD_SPLIT_OFF = 1 };
/* Flags OR-ed into the method of sfcdd_solve: start from x0 exactly as given
 * and apply the full balanced operator every iteration; stop on the recursive
 * residual alone (see sfcdd_solve). */
enum { SFCDD_SOLVE_PLAIN_START = 256, SFCDD_SOLVE_RECURSIVE = 512, SFCDD_SOLVE_ENERGY = 1024 };

typedef struct {
  int32_t d;                 /* dimension, 1 <= d <= 16                                */
  const int32_t* level;      /* host, length d: level l_j >= 1 (n_j = 2^l_j - 1), or   */
  const int32_t* npts;       /* host, length d: explicit n_j >= 1 (h_j = 1/(n_j+1));    */
                             /*   exactly one of level / npts is non-NULL              */
  const double* coeff;       /* host, length d: a_j > 0, NULL = all 1                  */
  int32_t P;                 /* number of subdomains, 1 <= P <= N                      */
  int64_t gamma_num;         /* overlap gamma = gamma_num / gamma_den >= 0 (eq. enlarge) */
  int64_t gamma_den;         /*   gamma_den >= 1                                       */
  int32_t q;                 /* coarse unknowns per subdomain (eq. restr), 1..floor(N/P);
                                0 = 2^(floor(log2(N/P)) - 4), capped at qP <= 16384    */
  int32_t weighting;         /* SFCDD_WEIGHT_NONE, _OMEGA (eq. omegai) or _D (eq. Di)    */
  int32_t variant;           /* SFCDD_ADDITIVE, SFCDD_BALANCED or SFCDD_DEFLATED         */
  int32_t factor_dtype;      /* SFCDD_FP64 or SFCDD_FP32 subdomain factors and solves
                                (see coarse_precision for the coarse operator)         */
  int32_t local_solver;      /* SFCDD_LOCAL_CHOLESKY: forward/backward substitution
                                with the Cholesky factor; SFCDD_LOCAL_INVERSE: the
                                explicit inverse formed from it, applied as a
                                symmetric matrix-vector product                        */
  int32_t layout;            /* 0 natural order, 1 curve order                          */
  int32_t curve;             /* SFCDD_CURVE_ZORDER or SFCDD_CURVE_HILBERT (Sec. 3.2)    */
  int32_t coarse_precision;  /* SFCDD_COARSE_AUTO: beside FP32 subdomain factors the
                                coarse inverse X_0 is FP32 and the coarse Cholesky
                                factor too when the coarse matrices are well
                                conditioned (sfcdd_info.coarse_fp32); FP64 otherwise.
                                SFCDD_COARSE_FP64: factor, inverse and coarse solves
                                in FP64 whatever the subdomain factors               */
  int32_t coarse_solver;     /* SFCDD_COARSE_DENSE: A_0 factored and inverted densely;
                                q = 0 takes the four-levels-coarser rule capped at
                                qP <= 16384.  SFCDD_COARSE_ITERATIVE (single grids
                                only): A_0 kept sparse and solved by an inner FP64 CG
                                at every application (see sfcdd_setup); q = 0 takes
                                the rule uncapped; qP <= 2^22                          */
  double coarse_tol;         /* SFCDD_COARSE_ITERATIVE: relative residual of the inner
                                CG, 0 = 1e-6 (the outer flexible CG absorbs the rest:
                                on the 8.26 M-unknown grid 1e-4 .. 1e-10 all take the
                                same outer iteration count)                            */
  int32_t local_order;       /* elimination order of the subdomain matrices for the
                                direct solves (Sec. 3.1; A_i^{-1} does not depend on it).
                                SFCDD_ORDER_DIAGONAL: the points of each subdomain
                                sorted by a coordinate diagonal sum_j s_j x_j (signs
                                chosen per subdomain for the narrowest level), ties
                                in curve order; SFCDD_ORDER_CURVE: curve order.  Both
                                store and stream only the tile envelope of the factor
                                (Cholesky creates no entries left of the first
                                nonzero of a row).  SFCDD_ORDER_DENSE: curve order,
                                the whole packed triangle.  The explicit-inverse
                                local solver always uses the last.                    */
  int32_t coarse_split;      /* elimination order of the dense coarse matrix (any
                                symmetric order gives the same A_0^{-1}).
                                SFCDD_SPLIT_AUTO: for a single grid with FP32 coarse
                                factor and inverse, one level of nested dissection
                                when it pays: the coarse blocks of the two halves of
                                the curve, each in the centroid-diagonal order, then
                                the separator (the first half's blocks with a
                                neighbour in the second).  The halves factor as two
                                concurrent chains of column steps, and X_0 = L_0^{-1}
                                has no tiles coupling them, so the coarse solves
                                read fewer tiles (sfcdd_info.coarse_split).  It is
                                used when both halves have at least two 64-row tiles
                                and the separator at most an eighth of the tile rows,
                                and the halves' envelopes are at most 24 tiles wide;
                                otherwise, and with SFCDD_SPLIT_OFF, the
                                centroid-diagonal order alone                         */
} sfcdd_params;

typedef struct {
  int32_t iterations;        /* outer iterations taken                                 */
  int32_t restarts;          /* residual replacements (iterative refinement steps)     */
  double rel_residual;       /* ||b - A x||_2 / ||b||_2, recomputed at exit            */
  double xi;                 /* Richardson damping used (0 for CG)                     */
  double lambda_min;         /* Lanczos estimates of the extreme eigenvalues of        */
  double lambda_max;         /*   C^{-1} A (Richardson with xi <= 0 only)              */
  int32_t coarse_steps;      /* iterative coarse solve: most inner CG steps one coarse
                                solve of this call took (0 with the dense solver)     */
  int32_t coarse_unconverged; /* iterative coarse solve: coarse solves of this call
                                whose inner CG stopped at its step budget (each is
                                followed by a larger budget)                           */
} sfcdd_solve_info;

typedef struct {
  int64_t N;                 /* unknowns                                               */
  int32_t P, q, N0;          /* subdomains, coarse points per subdomain, coarse size   */
  int32_t max_Ni, min_Ni;    /* largest / smallest overlapping subdomain               */
  int32_t tile;              /* tile edge of the packed factor layout                  */
  int64_t sum_Ni;            /* sum_i N_i                                              */
  int64_t factor_bytes;      /* bytes of the subdomain factor tiles stored (the tile
                                envelopes; the workspace reserves the packed triangles) */
  int64_t factor_algo_bytes; /* bytes of factor entries one substitution sweep reads:
                                the off-diagonal envelope tiles and the lower triangles
                                of the diagonal tiles, padding rows excluded
                                (sum_i N_i (N_i + 1) / 2 entries with
                                SFCDD_ORDER_DENSE) times sizeof(factor element)       */
  int64_t coarse_bytes;      /* bytes of the coarse operator tiles                     */
  double setup_ms[6];        /* sfc rank, neighbours, assembly, subdomain factorisation,
                                coarse setup (runs concurrently with the factorisation),
                                total                                                  */
  int32_t ngrids;            /* grids in the context (1 unless set up as a batch)      */
  int32_t trsv_waves;        /* waves per workgroup of the substitution kernel          */
  int32_t coarse_fp32;       /* 1: the coarse Cholesky factor is FP32 (FP32 subdomain
                                factors, automatic coarse precision and every coarse
                                matrix well conditioned by the bound
                                kappa(A) * max block / min block <= 4096); 0: FP64    */
  int32_t coarse_inv_fp32;   /* 1: the coarse inverse X_0 = L_0^{-1} and the coarse
                                solves' matrix reads are FP32 (FP32 subdomain factors,
                                automatic coarse precision); 0: FP64                  */
  int32_t coarse_iterative;  /* 1: SFCDD_COARSE_ITERATIVE: then N0d below is the size of
                                the inner CG's dense second level (the factor and
                                inverse above belong to it), ell_width the entries
                                per row kept for A_0, coarse_steps the inner CG's
                                current step budget                                    */
  int32_t N0d, ell_width, coarse_steps;
  int32_t factor_rows;       /* launch shape of the batched factorisation: row tiles  */
  int32_t factor_pair;       /*   per panel step, and 1 for two columns per step      */
  int32_t spmv_points;       /* launch shape of the SpMV: points per thread,          */
  int32_t spmv_window;       /*   and points of x staged in LDS per workgroup (256 u) */
  int32_t local_order;       /* elimination order of the subdomain matrices in use      */
  double factor_flops;       /* floating-point operations of the subdomain
                                factorisation: 2 TS^3 per tile product and 2 TS^3 / 3
                                per diagonal tile (its Cholesky factor and inverse)     */
  int32_t coarse_split[3];   /* dissected coarse matrix: 64-row tiles of its first
                                half, second half and separator (zeros when not
                                dissected)                                             */
} sfcdd_info;

/* Workspace bytes that sfcdd_setup needs for these parameters (Alg. 1
 * inputs d, l, P, gamma, q).  Validates the parameters: EINVAL for sizes out
 * of range, EOVERFLOW when N >= 2^31 or d * max_j l_j > 64. */
sfcdd_status sfcdd_workspace_size(const sfcdd_params* params, size_t* bytes);

/* Workspace bytes for a batch of ngrids independent grids (params[ngrids]);
 * see sfcdd_setup_batch. */
sfcdd_status sfcdd_workspace_size_batch(int32_t ngrids, const sfcdd_params* params, size_t* bytes);

/* Setup phase (Alg. 1): curve order of the grid points, disjoint pieces
 * (eq. sloc), overlapping subdomains (eq. enlarge, cyclic), weights
 * (eq. omegai), coarse blocks and A_0 = R_0 A R_0^T (eqs. restr, csm), and a
 * Cholesky factorisation of every A_i = R_i A R_i^T and of A_0 (factor once,
 * Sec. 3.1).  With coarse_solver = SFCDD_COARSE_ITERATIVE, A_0 is kept as a
 * sparse matrix (one row per coarse block: the blocks its points couple to)
 * and every coarse solve runs an FP64 CG on it to relative residual
 * coarse_tol, preconditioned by the explicit inverses of its 64 x 64 diagonal
 * blocks (64 consecutive coarse unknowns) plus a dense correction on the
 * Galerkin aggregation of A_0 over those blocks; the setup sizes the inner
 * step budget with one trial solve.  This lifts the dense coarse size limit
 * (the paper's four-levels-coarser rule, Sec. 4.1, on many subdomains; the
 * paper leaves the coarse problem's scalable solution open).  The inner solve
 * makes the preconditioner vary slightly between applications, so sfcdd_solve
 * uses the flexible CG update for SFCDD_PCG as well.  workspace_dev: device
 * buffer of at least the queried size; hip_stream: hipStream_t or NULL.  On
 * success *out receives a new context.  ENOTSPD if a factorisation breaks
 * down; EINVAL if a coarse row of the iterative solver couples to more blocks
 * than its table holds. */
sfcdd_status sfcdd_setup(const sfcdd_params* params, void* workspace_dev, size_t bytes,
                         void* hip_stream, sfcdd_ctx** out);

/* Setup of a batch of ngrids (1..65535) independent subproblems, e.g. all
 * subgrids of one layer of the combination technique (Sec. 2, eq. combi; the
 * subproblems are independent and solved in parallel), in one context: every
 * setup phase and every operator of the solve runs as one launch over all
 * grids.  params[ngrids] may differ in d, levels, coefficients, P, gamma and q;
 * weighting, variant, factor_dtype, local_solver and layout must agree.
 * Vectors of a batch context concatenate the grids in order: grid k owns the
 * entries [sum_{k'<k} N_k', sum_{k'<=k} N_k').  sfcdd_solve then solves all
 * grids, each to its own relative residual ||b_k - A_k x_k|| / ||b_k|| <= rtol
 * (converged grids stop iterating); info reports the largest iteration count
 * and residual, sfcdd_get_batch_stats the per-grid ones.  sfcdd_grad_coeff is
 * not available for batches (EINVAL). */
sfcdd_status sfcdd_setup_batch(int32_t ngrids, const sfcdd_params* params, void* workspace_dev,
                               size_t bytes, void* hip_stream, sfcdd_ctx** out);

/* Bytes of the device workspace behind sfcdd_setup_noalloc: one static array
 * per device, resident from the first allocation-free setup on the device
 * until the process ends. */
#define SFCDD_NOALLOC_WORKSPACE_BYTES ((size_t)256 << 20)

/* Allocation-free variant of sfcdd_setup, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same setup of one grid, with the workspace taken from the
 * library's static per-device array of SFCDD_NOALLOC_WORKSPACE_BYTES instead of
 * a caller buffer.  It calls no hipMalloc, hipHostMalloc, hipFree or other
 * device or pinned-host allocator; the context's host tables live on the C++
 * heap, and its scalar read-backs go to pageable host memory (each waits for
 * the stream, so a solve does not overlap its host checks with the next
 * preconditioner application).  Parameters, stream and errors as sfcdd_setup;
 * ENOMEM (message gives the size) when sfcdd_workspace_size exceeds
 * SFCDD_NOALLOC_WORKSPACE_BYTES.  The array is shared by every allocation-free
 * context of the device: a new sfcdd_setup_noalloc on the device overwrites it,
 * after which every call on an earlier allocation-free context of that device
 * fails with EINVAL (destroy it as usual).  Allocation-free setups and their
 * contexts' calls that overlap in time on one device race on the array; keep
 * them on one thread or ordered.  Everything else (apply, solve, destroy) is
 * used as with sfcdd_setup. */
sfcdd_status sfcdd_setup_noalloc(const sfcdd_params* params, void* hip_stream, sfcdd_ctx** out);

/* h = C^{-1} g (Alg. 2; balanced form eq. balSW when variant = BALANCED).
 * g_dev, h_dev: device, N doubles each, may not alias.  Asynchronous. */
sfcdd_status sfcdd_apply_precond(sfcdd_ctx* ctx, const double* g_dev, double* h_dev);

/* y = A x with the (2d+1)-point FD matrix.  Device, N doubles each, no alias. */
sfcdd_status sfcdd_matvec(sfcdd_ctx* ctx, const double* x_dev, double* y_dev);

/* Solve A x = b (Alg. 3 / preconditioned CG, Sec. 3.3).  b_dev: device, N
 * doubles.  x_dev: device, N doubles, initial guess on entry (zero it for
 * x0 = 0), solution on exit; may not alias b_dev.  Stops when the relative
 * residual ||b - A x||_2 / ||b||_2 <= rtol (checked on the recursive residual
 * and confirmed on the true residual, restarting from the current x when they
 * disagree), or after max_iter iterations (ENOTCONV).  A grid whose true
 * residual has not halved since its previous restart has reached the rounding
 * floor of FP64 for its matrix (about eps ||A|| ||x|| / ||b||, which exceeds
 * 1e-8 on strongly anisotropic grids with 2^14 points along one direction):
 * it stops there, and the call returns ESTAGNATED with x the last iterate.
 * With SFCDD_SOLVE_RECURSIVE OR-ed into method, the stopping test is the
 * recursive residual of the iteration alone, as in the paper's algorithms
 * (Sec. 4: ||r_k|| / ||r_0|| with r_0 = b for x0 = 0); info.rel_residual is then
 * the recursive one.
 * With SFCDD_SOLVE_ENERGY OR-ed into method (only for b = 0, EINVAL otherwise:
 * the protocol of the paper's Sec. 4.1 experiments, a homogeneous problem
 * from a random start), the error is the iterate itself and a grid stops when
 * its energy norm sqrt(x_k^T A x_k) <= rtol, evaluated as -(x_k . r_k) with
 * the iteration's residual; the test is on the iteration alone (as with
 * SFCDD_SOLVE_RECURSIVE) and info.rel_residual is that energy norm.
 * method: SFCDD_PCG, SFCDD_FCG (flexible CG, beta = z'(r_new - r_old)/z'r_old,
 * for the FP32-factor preconditioner) or SFCDD_RICHARDSON (x += xi C^{-1} r;
 * xi <= 0 estimates xi = 2/(lmin + lmax) from 30 Lanczos steps on the residual
 * of the start).
 * Balanced and deflated variants: unless SFCDD_SOLVE_PLAIN_START is OR-ed into
 * method, the start is first corrected to x0 + F (b - A x0), F = R_0^T A_0^{-1}
 * R_0.  Its residual, and every later one, satisfies R_0 r = 0, where the
 * balanced operator reduces to (I - F A) C1^{-1}: one coarse solve per
 * iteration instead of two, same iterates as the full operator from that start
 * (on such residuals the two variants coincide).
 * info: host, may be NULL. */
sfcdd_status sfcdd_solve(sfcdd_ctx* ctx, const double* b_dev, double* x_dev, double rtol,
                         int32_t max_iter, int32_t method, double xi, sfcdd_solve_info* info);

/* Coefficient part of the adjoint gradient of J(u) with A(a) u = f:
 * grad_a[j] = -lambda^T (dA/da_j) u = -(1/h_j^2) sum_k lambda_k (2 u_k - u_{k-e_j}
 * - u_{k+e_j}) (Sec. 4 model problem with alpha = diag(a_j)).  lambda_dev, u_dev:
 * device, N doubles; grad_a_host: host, d doubles.  Synchronous. */
sfcdd_status sfcdd_grad_coeff(sfcdd_ctx* ctx, const double* lambda_dev, const double* u_dev,
                              double* grad_a_host);

/* Copies the partition of grid `grid` (0 for a single-grid context) to host
 * arrays (each may be NULL), in the grid's own numbering: sfc_index[N]
 * (natural index of curve position p), ta[P] (first curve position of
 * Omega_i), Ni[P] (its size; Omega_i = {(ta_i + s) mod N : s < N_i}), omega[P]
 * (eq. omegai weight actually applied), q_out (coarse points per subdomain). */
sfcdd_status sfcdd_get_partition(sfcdd_ctx* ctx, int32_t grid, int32_t* sfc_index_host,
                                 int64_t* ta_host, int64_t* Ni_host, double* omega_host,
                                 int32_t* q_out);

/* Per-grid outer iteration counts and final relative residuals of the last
 * sfcdd_solve (host arrays of ngrids entries, each may be NULL). */
sfcdd_status sfcdd_get_batch_stats(sfcdd_ctx* ctx, int32_t* iterations, double* rel_residual);

/* The substitution-kernel part of sfcdd_tune (SFCDD_TUNE_TRSV): times the
 * substitution sweeps with 4, 8 and 16 waves per workgroup, each with and
 * without the non-temporal hint on the factor loads, on the context's own
 * factors, keeps the fastest, and returns its time per application in
 * *best_ms (may be NULL).  Repeats and the per-shape record as in sfcdd_tune.
 * With the explicit-inverse local solver there is nothing to tune and only
 * the time is measured.  Synchronous. */
sfcdd_status sfcdd_autotune(sfcdd_ctx* ctx, int32_t repeats, double* best_ms);

/* Launch shapes chosen by sfcdd_tune and their times (ms) against the default
 * shapes on the context's own data. */
typedef struct {
  int32_t trsv_waves;        /* waves per workgroup of the substitution kernel (4, 8, 16) */
  int32_t spmv_points;       /* SpMV points per thread (1, 2, 4)                          */
  int32_t spmv_window;       /* SpMV LDS window per workgroup: 256 spmv_points            */
  int32_t factor_rows;       /* row tiles per step of the batched factorisation (1..4;
                                1: the light kernel for matrices of a few tile rows)     */
  int32_t factor_pair;       /* 1: two columns per step                                   */
  int32_t tuned;             /* SFCDD_TUNE_* bits that were timed now (the rest came
                                from the per-shape record of earlier tunings, or were
                                not asked for)                                           */
  double trsv_ms, trsv_default_ms;    /* one application of the subdomain solves        */
  double spmv_ms, spmv_default_ms;    /* one SpMV y = A x                               */
  double setup_ms, setup_default_ms;  /* one whole setup (Alg. 1 and the factorisations) */
  int32_t trsv_stream;       /* non-temporal hint on the substitution kernel's factor
                                loads: 1 on, 0 off, -1 the default (off)                 */
} sfcdd_tuning;
enum { SFCDD_TUNE_TRSV = 1, SFCDD_TUNE_SPMV = 2, SFCDD_TUNE_SETUP = 4, SFCDD_TUNE_ALL = 7 };

/* Autotuner of the launch shapes (the `what` bits): the substitution kernel's
 * waves per workgroup (4, 8, 16) with and without the non-temporal hint; the
 * SpMV's points per thread (1, 2, 4; the LDS window is 256 of them); and the
 * batched factorisation's shape: the light kernel for small matrices, or row
 * tiles per panel step (2, 3, 4; 2, 3 with FP64 factors) with one or two
 * columns per step, each
 * candidate timed with events on the context's stream (repeats runs each,
 * 0 = 3; the factorisation shapes by repeating the whole setup of this
 * context, which is left set up with the winner).  The fastest shapes are used
 * by this context from then on and recorded for the process per launch shape
 * (device, precision, grid sizes, subdomain sizes): every later setup of the
 * same shape starts from them, and a later sfcdd_tune call on such a context
 * returns the recorded choice and times without timing again.  A negative
 * repeats times again (|repeats| runs) regardless.  report: host, may be
 * NULL.  Synchronous. */
sfcdd_status sfcdd_tune(sfcdd_ctx* ctx, int32_t repeats, int32_t what, sfcdd_tuning* report);

/* The same partition computed on the host alone, before any setup (no GPU
 * needed): ta[P], Ni[P], omega[P] and q_out as in sfcdd_get_partition, each
 * may be NULL.  Validation and error codes as sfcdd_workspace_size. */
sfcdd_status sfcdd_partition_host(const sfcdd_params* params, int64_t* ta_host, int64_t* Ni_host,
                                  double* omega_host, int32_t* q_out);

/* Kernel classes timed by the profiling counters: the subdomain solves, the
 * weighted sum, the SpMV y = A x (with or without the x . y partials), the
 * coarse solve, and the SpMV y = b - A x (which also reads b). */
enum { SFCDD_K_LOCAL_SOLVE = 0, SFCDD_K_SCATTER = 1, SFCDD_K_SPMV = 2, SFCDD_K_COARSE = 3,
       SFCDD_K_SPMV_B = 4, SFCDD_K_COUNT = 5 };

/* Turns per-kernel timing on (1) or off (0) and clears the counters.  When on,
 * every launch of a timed kernel class is bracketed by HIP events on the
 * context's stream; the elapsed times are accumulated whenever the library
 * synchronises (end of sfcdd_solve) or on sfcdd_get_kernel_time.  Adds a few
 * microseconds per launch. */
sfcdd_status sfcdd_set_profiling(sfcdd_ctx* ctx, int32_t on);

/* Accumulated device time (ms) and launch count of kernel class `kind`
 * (SFCDD_K_*) since profiling was enabled.  Synchronises the stream. */
sfcdd_status sfcdd_get_kernel_time(sfcdd_ctx* ctx, int32_t kind, double* total_ms,
                                   int64_t* launches);

/* Combination technique (Sec. 2, eq. combi): out[m] = sum_g weights[g] u_g(x_m)
 * over the grids of the context (a batch set up with sfcdd_setup_batch, all
 * of one dimension d <= 10), where u_g is the piecewise multilinear function
 * of grid g's values (zero on the boundary of [0,1]^d).  weights_dev: device,
 * ngrids doubles (e.g. (-1)^i binom(d-1, i) for the grids of layer i);
 * u_dev: device, the concatenated grid vectors in the context's layout (as
 * sfcdd_solve returns them); x_dev: device, M points of d coordinates,
 * row-major (points outside [0,1]^d are extrapolated from the boundary cell);
 * out_dev: device, M doubles.  The summation order over the grids is fixed, so
 * the result is reproducible.  Asynchronous on the context stream. */
sfcdd_status sfcdd_ct_combine(sfcdd_ctx* ctx, const double* weights_dev, const double* u_dev,
                              const double* x_dev, int64_t M, double* out_dev);

/* Grids of the combination technique of level L in d dimensions (Sec. 2,
 * eq. combi): the anisotropic full grids of the layers |l|_1 = L + d - 1 - i,
 * l_j >= 1, i = 0 .. d-1, in layer order and lexicographically within a layer
 * (first entry slowest), each with its combination weight (-1)^i binom(d-1, i)
 * and its subdomain count P = phat 2^(d-1-i) (eq. Pchoice) capped at the
 * grid's point count.  Host only, no GPU needed.  *ngrids receives the number
 * of grids; when any of levels (ngrids * d int32, row-major), layer (int32),
 * weight (double) or P (int32) is non-NULL, all non-NULL arrays are filled,
 * which needs capacity >= *ngrids (ENOMEM otherwise, *ngrids still set).
 * EINVAL for d outside 1..16, L outside 1..60 or phat < 1. */
sfcdd_status sfcdd_ct_layout(int32_t d, int32_t L, int32_t phat, int32_t capacity, int32_t* ngrids,
                             int32_t* levels, int32_t* layer, double* weight, int32_t* P);

/* Streaming-read rate of the device, for roofline context: reads the device
 * buffer buf_dev (bytes, a multiple of 16, 16-byte aligned; its contents are
 * not changed) with a 16-byte-per-lane grid-stride kernel (non-temporal
 * loads, as the substitution kernel streams its factors) `repeats` times on
 * hip_stream (NULL = default stream) and returns the shortest time in
 * *best_ms.  Needs no context.  Synchronous. */
sfcdd_status sfcdd_read_probe(const void* buf_dev, size_t bytes, void* hip_stream, int32_t repeats,
                              double* best_ms);

/* Sizes and setup timings of a context. */
sfcdd_status sfcdd_get_info(sfcdd_ctx* ctx, sfcdd_info* info);

/* Releases the context's host memory.  The workspace may be freed afterwards. */
sfcdd_status sfcdd_destroy(sfcdd_ctx* ctx);

/* Message describing the last failure on ctx (or of a call without a context
 * when ctx is NULL).  Valid until the next call on the same context. */
const char* sfcdd_last_error(const sfcdd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SFCDD_H */
