/*
 * pcloth.h -- C ABI of the MI355X implicit cloth step (P-Cloth, Li et al.,
 * arXiv 2008.00409).
 *
 * One backward-Euler step (paper Sec. 2.5, Eq. 1-3) assembles and solves
 *     A dv = b,   A = M - h*df/dv - h^2*df/dx = M + h*(h+beta)*K,
 *                 b = h*[ f(x + h*v) - beta*K*v ]          (rhs_mode 0, Eq. 3)
 *                 b = h*[ f(x) - (h+beta)*K*v ]            (rhs_mode 1, linearised)
 * then v += dv, x += h*v.  K = -df/dx is the positive semi-definite solver
 * Jacobian of the per-triangle membrane (St. Venant-Kirchhoff, stress clamped
 * to its PSD part in the geometric term) and per-hinge dihedral bending
 * (Gauss-Newton) energies; f holds those forces plus gravity.  Pinned vertices
 * are Dirichlet: A_ij = A_ji = 0 (j != i), A_ii = m_i I, b_i = 0.
 *
 * The matrix is rebuilt every step from the element list (Sec. 3.2.2: the
 * block pattern is derived from the elements, duplicates removed, values
 * summed per block), and solved by Jacobi-preconditioned CG (Sec. 3.1).
 *
 * Conventions (all entry points):
 *  - Vectors (x, v, b, dv) are DEVICE arrays of nv*3 doubles, vertex-major
 *    ((nv, 3) row-major), owned by the caller.  Mesh arrays in pc_mesh are HOST
 *    arrays, copied by pc_create.
 *  - All GPU work is enqueued on `stream` (a hipStream_t; NULL = default
 *    stream).  Only calls that fill host outputs (pc_solve_info, status of
 *    device-side checks) synchronise that stream.
 *  - Errors are return codes; pc_last_error() gives a message.  No exception
 *    crosses the ABI.  Calls on one context must not overlap; distinct
 *    contexts are independent.
 */
#ifndef PCLOTH_H
#define PCLOTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pc_ctx pc_ctx;

typedef enum {
    PC_OK = 0,
    PC_ERR_ARG = 1,            /* bad argument (null pointer, size, option) */
    PC_ERR_MESH = 2,           /* bad index, degenerate rest triangle, edge in >2 triangles,
                                  inconsistently oriented neighbours */
    PC_ERR_HIP = 3,            /* a HIP runtime call failed */
    PC_ERR_OOM = 4,            /* device allocation failed */
    PC_ERR_NONFINITE = 5,      /* NaN/Inf in the right-hand side or the residual */
    PC_ERR_NOT_CONVERGED = 6,  /* maxit reached; dv holds the last iterate */
    PC_ERR_CAPACITY = 7        /* a vertex exceeds the per-row limits (512 incident
                                  element corners, 64 distinct block columns), or at
                                  pc_create is the lower end of more than 64 edges */
} pc_status;

/* Storage type of the matrix blocks.  The assembly evaluates every element
 * and sums every block in FP64 and then rounds to this type.  The state,
 * b, the dots of the CG recurrences and the refinement residual b - A dv
 * (through the FP64 copy of the blocks) stay FP64 for every type.  With FP32
 * or FP64 blocks the CG product accumulates in FP64.  With BF16 or FP16
 * blocks the CG product's row sums are FP32, and (PC_OPT_INNER_FP32, the
 * default) each refinement sweep keeps its correction, residual and product
 * in FP32; the sweep's start residual and the final convergence test are
 * FP64.  FP16 blocks (IEEE binary16, 11 significant bits against BF16's 8)
 * are stored multiplied by a power of two S chosen at each assembly so that
 * the largest stored magnitude lies in [2^13, 2^14); the product divides S
 * out of its row sums, and cloth_export_blocks returns the unscaled values. */
typedef enum { PC_F64 = 0, PC_F32 = 1, PC_BF16 = 2, PC_F16 = 3 } pc_dtype;

/* Device memory allocator of a context (pc_set_allocator): alloc returns
 * `bytes` of device memory on the current device, 256-byte aligned as
 * hipMalloc's blocks are (NULL on failure; a misaligned block is returned to
 * free and the call fails with PC_ERR_ARG), free releases a block that alloc
 * returned.  `user` is passed through. */
typedef void *(*pc_alloc_fn)(size_t bytes, void *user);
typedef void (*pc_free_fn)(void *ptr, void *user);

typedef struct {
    double h;            /* time step (s) */
    double mu, lambda;   /* membrane Lame constants (N/m) */
    double k_bend;       /* bending stiffness (N m) */
    double beta;         /* stiffness-proportional damping (s); 0 reproduces Eq. 3 */
    double gravity[3];   /* m/s^2 */
    int32_t rhs_mode;    /* 0: Eq. 3 as printed, lookahead force f(x + h v);
                            1: the same force linearised with the matrix's own Jacobian
                            (Eq. 2 applied to the right-hand side): h [f(x) - (h+beta) K v].
                            With the PSD solver Jacobian only mode 1 is stable on cloth with
                            compressed regions (mode 0 integrates the negative stiffness
                            explicitly and grows exponentially); mode 1 is the recommended
                            setting. */
    int32_t reserved;
} pc_params;

typedef struct {
    int32_t nv, nt;
    const int32_t *tris;   /* host, nt*3, counter-clockwise w.r.t. the rest normal */
    const double *rest;    /* host, nv*3 rest positions */
    const double *mass;    /* host, nv, kg, > 0 */
    const uint8_t *pinned; /* host, nv, 1 = Dirichlet vertex (may be NULL: none) */
} pc_mesh;

/* View of the assembled matrix, valid until the next cloth_assemble on the
 * same context.  rowptr/colidx are the block-CSR pattern (columns ascending,
 * diagonal included, pinned rows/columns kept as explicit zero blocks), device
 * int32.  Values live in the context in a solver layout; cloth_export_blocks
 * copies them out in block-CSR order. */
typedef struct {
    const int32_t *rowptr;   /* device, nrows+1 */
    const int32_t *colidx;   /* device, nnzb */
    pc_dtype dtype;
    int32_t nrows, nnzb;
} pc_bsr3;

typedef struct {
    double tol;            /* stop when ||b - A dv||_2 <= tol * ||b||_2, A with FP64 blocks */
    double inner_rho;      /* each refinement sweep's CG stops once its residual has fallen by
                              this factor (or reached tol); 0: default (BF16 and FP16
                              blocks 1e-2, FP16 keeping the direction 0.5,
                              FP32/FP64 blocks: run each sweep to tol) */
    int32_t maxit;         /* total CG iterations over all sweeps; default 20000 when <= 0 */
    int32_t warm;          /* 0: zero start, 1: caller's dv as start, 2: learned start predicted
                              from the caller's dv taken as the previous step's increment
                              (needs pc_ws_set_params; see pc_ws_predict for the safeguard) */
    int32_t check_every;   /* iterations between host convergence checks (0: auto) */
    int32_t max_sweeps;    /* refinement sweeps; 0: default (BF16 and FP16 40, FP16
                              keeping the direction 400, otherwise 4) */
    int32_t precond;       /* 0: Jacobi, P = diag(A) (the paper's preconditioner, Sec. 2.5);
                              1: block Jacobi, P = the 3x3 diagonal blocks A_ii, inverted in
                              FP64 at assembly and applied in FP32 x FP64 */
    int32_t method;        /* 0: the textbook PCG recurrences (two reductions per iteration);
                              1: the single-reduction form of Chronopoulos and Gear (1989):
                              gamma = r.u and delta = u.Au from one product per iteration,
                              the direction and its product by recurrences (project solver
                              variant; same iterates in exact arithmetic) */
} pc_solve_opts;

typedef struct {
    int32_t iters;             /* CG iterations performed */
    int32_t sweeps;            /* outer refinement sweeps (1 without refinement) */
    double rel_res_recursive;  /* ||r_k|| / ||b|| from the CG recurrence */
    double rel_res_true;       /* ||b - A dv|| / ||b|| recomputed at exit with the FP64 blocks */
    double bnorm;              /* ||b||_2 */
    int32_t fallback;          /* 1 if the inner CG switched to the FP64 blocks after a
                                  breakdown on the low-precision copy, or after a sweep on
                                  it that did not halve the FP64 residual it started from */
    int32_t warm_used;         /* start actually used: 0 zero, 1 given / previous increment,
                                  2 learned (previous increment plus a nonzero step along the
                                  network's correction) */
} pc_solve_info;

/* Create a context for one cloth (or several, pc_set_instances): the
 * problem statement of Sec. 2.5 (Eq. 1-3) fixes its inputs, i.e. the
 * triangle mesh with its rest shape (the reference configuration of the
 * elastic forces), the lumped masses M, the Dirichlet vertices and the
 * material constants and time step of Eq. 3 (params).  pc_create copies the
 * mesh to the device, derives the rest shape data (per-triangle inverse rest
 * frame and area, per-hinge coefficient and rest angle) and the hinge list
 * (one per interior edge; the bending elements, Sec. 5) on the GPU.
 * Ownership: *out is owned by the caller and released by pc_destroy; the
 * host mesh arrays are only read during the call.  Device memory comes from
 * the allocator installed with pc_set_allocator(NULL, ...), else hipMalloc.
 * Errors: PC_ERR_ARG (sizes, null), PC_ERR_MESH (index out of range,
 * degenerate rest triangle, non-manifold or misoriented mesh), PC_ERR_OOM,
 * PC_ERR_HIP.  Synchronises the default stream. */
pc_status pc_create(const pc_mesh *mesh, const pc_params *params, pc_ctx **out);
/* Release a context and every device buffer it owns (each returned to the
 * allocator it came from), after draining the device.  The caller's x, v,
 * b and dv buffers are not touched.  PC_ERR_ARG for NULL. */
pc_status pc_destroy(pc_ctx *ctx);
/* Replace the time step and material constants of Eq. 3 for the following
 * assemblies (same checks as pc_create). */
pc_status pc_set_params(pc_ctx *ctx, const pc_params *params);
/* Device memory of the library.  With ctx != NULL, the context's following
 * device allocations (workspaces, the assembled matrix, buffers that grow
 * with contact sets or schedules, the warm-start network's state) call
 * alloc, and each block goes back to the free routine of the allocator that
 * allocated it, so allocators may be switched at any time.  With ctx ==
 * NULL the pair becomes the default of contexts created afterwards,
 * including pc_create's own buffers.  alloc = free = NULL restores
 * hipMalloc / hipFree; giving only one is PC_ERR_ARG.  Before a block goes
 * back to a caller's free routine the library synchronises the device,
 * since such an allocator (a caching allocator such as PyTorch's) may hand
 * the block out again at once; this happens only when a buffer grows and at
 * pc_destroy.  Pinned host staging (a few bytes per instance) stays with
 * hipHostMalloc.  The routines are called from the thread that calls the
 * library. */
pc_status pc_set_allocator(pc_ctx *ctx, pc_alloc_fn alloc, pc_free_fn free, void *user);
const char *pc_last_error(const pc_ctx *ctx);   /* NULL ctx: last pc_create error */

/* Topology sizes: [nv, nt, nhinges, nnzb capacity]. */
pc_status pc_sizes(const pc_ctx *ctx, int64_t out[4]);
/* Copy the hinge list (nh*4 int32 a,b,c,d: edge a-b, wings c,d) and per-hinge
 * (coefficient, rest angle) pairs to host memory (either pointer may be NULL). */
pc_status pc_get_hinges(pc_ctx *ctx, int32_t *hinges_host, double *coef_host);

/* Assemble A and b at state (x, v) (paper Sec. 3.2.2 and Eq. 3): rebuild the
 * block pattern from the element list, sum the element blocks of each block
 * (deterministic order: triangles then hinges, by index), eliminate pinned
 * vertices, and form b and the Jacobi diagonal.  Block values are stored as
 * `dtype`; diag_out (optional, device nv*3 doubles) receives diag(A).
 * x, v: device nv*3 doubles.  b: device nv*3 doubles (output).
 * A_out (optional, host struct) receives the pattern view.
 * Asynchronous; capacity overflows detected on the device are reported by the
 * next synchronising call (cloth_pcg_solve, cloth_step, pc_check). */
pc_status cloth_assemble(pc_ctx *ctx, const double *x, const double *v, pc_dtype dtype,
                         pc_bsr3 *A_out, double *b, double *diag_out, void *stream);

/* Solve A dv = b by Jacobi-preconditioned CG on the most recently assembled
 * matrix (Sec. 2.5: the linear system of Eq. 3, solved by PCG; Sec. 3.1).
 * The off-diagonal blocks are applied in difference form,
 *   (A y)_i = m_i y_i + D_i y_i + sum_{j != i} A_ij (y_j - y_i),
 * with D_i = A_ii - m_i I + sum_{j != i} A_ij kept separately, so that rounding
 * of the stored blocks does not disturb the mass term.  CG runs on the
 * solver copy of the blocks (the assembled dtype); each sweep starts from the
 * residual b - A dv computed with the FP64 copy, and sweeps repeat (iterative
 * refinement) until that FP64 residual meets tol.  Dots accumulate in
 * FP64.  The product accumulates in FP64 for FP32 and FP64 blocks and in
 * FP32 for BF16 and FP16 blocks (whose values carry 8 and 11 significant
 * bits).  Vectors are FP64 except the search direction (FP32) and, with BF16
 * or FP16 blocks and PC_OPT_INNER_FP32, the sweep's correction, residual and
 * product (FP32; x stays FP64).  A low-precision sweep runs at most half of
 * maxit iterations if it is the first and three times the instance's longest
 * earlier sweep (at least 256) otherwise; a sweep that does not halve the
 * FP64 residual it started from moves the instance to the FP64 blocks.  The sweep's start residual and the final test use FP64
 * vectors and the FP64 blocks, so the returned dv meets tol through an FP64
 * matrix whatever the storage.
 * dv: device nv*3 doubles, the start when opts->warm = 1, the solution on
 * return (also when PC_ERR_NOT_CONVERGED).  info: host, optional.
 * Synchronises the stream. */
pc_status cloth_pcg_solve(pc_ctx *ctx, const double *b, double *dv, const pc_solve_opts *opts,
                          pc_solve_info *info, void *stream);

/* nsteps backward-Euler steps of Eq. 3 (Sec. 2.5): assemble A and b at
 * (x, v) (Sec. 3.2), solve A dv = b (Sec. 3.1), then v += dv (dv is the
 * velocity increment of Eq. 3) and x += h v (pinned vertices keep x, and
 * v = 0).  x, v: device nv*3 doubles, updated in place.
 * A step whose solve fails (not converged, non-finite) is not committed:
 * x and v keep the values they had before that step, bit for bit, and the
 * call returns that status (infos[k] of the failed step is still filled).
 * infos: host array of nsteps, optional.
 * The previous step's dv is used as the start when opts->warm = 1. */
pc_status cloth_step(pc_ctx *ctx, double *x, double *v, int32_t nsteps, pc_dtype dtype,
                     const pc_solve_opts *opts, pc_solve_info *infos, void *stream);

/* y = A x with the assembled matrix (difference form; FP64 accumulation,
 * FP32 row sums of a BF16 or FP16 copy),
 * using the FP64 blocks (solver_blocks = 0) or the solver copy in the
 * assembled dtype (solver_blocks = 1).  x, y: device nv*3 doubles. */
pc_status cloth_spmv(pc_ctx *ctx, const double *x, double *y, int32_t solver_blocks, void *stream);

/* Copy the assembled blocks out in block-CSR order as FP64 (device nnzb*9,
 * row-major 3x3), with the true diagonal blocks A_ii = m_i I + D_i -
 * sum_{j != i} A_ij, and optionally the remainders D_i (device nv*9); from
 * the FP64 copy (solver_blocks = 0) or the solver copy (solver_blocks = 1). */
pc_status cloth_export_blocks(pc_ctx *ctx, double *vals_out, double *D_out, int32_t solver_blocks,
                              void *stream);

/* Proximity (contact) forces inside the implicit solve (paper Sec. 3.2:
 * the assembly elements include contact forces; Sec. 4: proximity forces
 * are integrated in the implicit step).  Each of the ncontacts pairs that a
 * proximity query reported is a repulsion element on 4 vertices: verts
 * (device nc x 4 int32), weights c (device nc x 4 doubles, summing to zero:
 * (1, -w_a, -w_b, -w_c) for a vertex-face pair with the closest point's
 * barycentric weights, (1 - s, s, -(1 - t), -t) for an edge-edge pair) and a
 * unit normal n (device nc x 3 doubles).  With the gap g = n . sum_k c_k x_k
 * the element's energy is stiffness/2 (thickness - g)^2 while g < thickness:
 * forces stiffness (thickness - g) c_k n and stiffness blocks
 * stiffness c_k c_l n n^T (the exact Hessian, PSD).  The arrays are copied;
 * the set applies to every following assembly until replaced, and
 * ncontacts = 0 removes it.  The block pattern changes with the set.
 * Synchronises the stream; PC_ERR_ARG for an index out of range, repeated
 * vertices in a pair, weights not summing to zero, a normal that is not
 * unit length, or a pair joining two instances (pc_set_instances); the set
 * is then empty. */
pc_status cloth_set_contacts(pc_ctx *ctx, int32_t ncontacts, const int32_t *verts, const double *weights,
                             const double *normals, double thickness, double stiffness, void *stream);

/* ---- The paper's own matrix filling and layout (Sec. 3.2.2), for comparison ----
 * cloth_assemble_bell assembles the same system as cloth_assemble (A = M +
 * h (h + beta) K with pinned rows and columns eliminated, and b) in the five
 * steps of the paper's GPU filling: per-row index-table sizes (every element
 * corner adds one slot per vertex of its element, plus one diagonal slot per
 * row), index filling with integer atomics, per-row sort and de-duplication
 * (compacting), a BELL value table as wide as the longest compacted row,
 * and value filling with one thread per element adding its 3x3 blocks with
 * floating-point atomics.  Values: dtype PC_F32 or PC_F64 (else PC_ERR_ARG).
 * Layout: slot k of row i at k*nv + i; columns ascending within a row, the
 * padding repeats the row's own index with zero blocks; plane q (row-major
 * 3x3 entry q) of slot k of row i at (q*width + k)*nv + i.  The atomics add
 * in an order that varies between runs, so the last bits of A and b do.
 * x, v: device nv*3 doubles; b: device nv*3 doubles (output); width_out
 * (host, optional): the table width.  Synchronises the stream (the table
 * sizes are read back to allocate, as in the paper).  The table lives in
 * the context, independent of cloth_assemble's matrix. */
pc_status cloth_assemble_bell(pc_ctx *ctx, const double *x, const double *v, pc_dtype dtype, double *b,
                              int32_t *width_out, void *stream);
/* y = A x over the BELL table, one thread per row: x (device nv*3 doubles)
 * is rounded to FP32, as the solver's search direction is; FP64 accumulation
 * into y (device nv*3 doubles).  PC_ERR_ARG before cloth_assemble_bell. */
pc_status cloth_spmv_bell(pc_ctx *ctx, const double *x, double *y, void *stream);
/* Copy the BELL table out: width_out (host, optional), cols_out (device
 * nv*width int32, optional), vals_out (device 9*nv*width doubles, optional),
 * in the layout above.  Enqueued on the stream. */
pc_status cloth_export_bell(pc_ctx *ctx, int32_t *width_out, int32_t *cols_out, double *vals_out, void *stream);

/* Preconditioners of the last assembly: inv_diag_out (device nv*3 floats)
 * receives 1 / diag(A); inv_blocks_out (device nv*6 floats) the inverses of
 * the 3x3 diagonal blocks A_ii as (xx, xy, xz, yy, yz, zz).  Either may be
 * NULL.  Enqueued on the stream. */
pc_status cloth_export_precond(pc_ctx *ctx, float *inv_diag_out, float *inv_blocks_out, void *stream);

/* Block-CSR pattern of the last assembly.  Synchronises the stream, writes
 * nnzb to *nnzb_out (host, optional) and copies rowptr (device nrows+1 int32)
 * and colidx (device nnzb int32) into the caller's buffers when they are not
 * NULL. */
pc_status cloth_export_pattern(pc_ctx *ctx, int32_t *rowptr_out, int32_t *colidx_out, int64_t *nnzb_out,
                               void *stream);

/* Kernel timing with HIP events on the launch stream: with every > 0, one in
 * `every` launches of each timed kernel is bracketed by an event pair (0 turns
 * sampling off; any call resets the statistics).  Inside a CG solve only one
 * chunk of iterations in 8 is sampled, so that the events add little to the
 * solve's time (with graph replay that chunk runs as plain launches).
 * pc_profile_read synchronises
 * the device and writes, for each kind k in 0..7 (0 SpMV in CG, 1 CG vector
 * update, 2 CG direction update, 3 row assembly, 4 row pattern, 5 whole
 * assembly, 6 element evaluation), out[5k..5k+4] = {samples, mean ms, min ms, max ms, median ms}
 * (host, 40 doubles; the median is over the first 65536 samples). */
pc_status pc_profile(pc_ctx *ctx, int32_t every);
pc_status pc_profile_read(pc_ctx *ctx, double *out);

/* ---- Learned warm start (project addition to the paper's method) ----
 * A per-vertex MLP (27 features -> 64 -> 64 -> 64 -> 3, ReLU) predicts a
 * correction u = s_v y to the previous step's increment on free vertices
 * (s_v = mean rest edge length / h).  As the CG start of Eq. 3 (warm = 2) it
 * is dv_prev + g u with the step g = u.(b - A dv_prev) / u.A u that minimises
 * the A-norm error along u (g = 0 when u.A u <= 0), so the start is never
 * worse in the A-norm than dv_prev itself.  One step g is taken for all
 * instances of the context (pc_set_instances), so with several instances
 * the guarantee holds for the sum of their A-norm errors, not for each
 * instance.  Features of vertex i (N(i): block
 * columns of row i other than i): v/s_v, (b/m)/s_v, dv_prev/s_v, mean_N dv_prev/s_v,
 * (b/diag A)/s_v, (mean_N b/m - b_i/m_i)/s_v, (mean_N v - v_i)/s_v,
 * (mean_N x - x_i)/l, pinned, log10(mean diag A_i / m_i), |N(i)|/12.
 * It runs on BF16 matrix cores with FP32 accumulation and is trained with
 * the energy loss L = (dv0.A dv0 / 2 - b.dv0) / (b.D^-1 b), whose gradient is
 * the residual of the start.  Parameters cross the ABI as PC_WS_PARAMS host
 * floats: per layer the weights [in][out] row-major, then the biases.
 * All calls use the most recent cloth_assemble of the context. */
#define PC_WS_PARAMS 10307
pc_status pc_ws_set_params(pc_ctx *ctx, const float *params_host, int32_t n);
pc_status pc_ws_get_params(pc_ctx *ctx, float *params_host, int32_t n);
/* Features as BF16 bits (device nv*32 uint16, features 27..31 zero). */
pc_status pc_ws_features(pc_ctx *ctx, const double *x, const double *v, const double *b, const double *dv_prev,
                         uint16_t *feat_out, void *stream);
/* Unscaled prediction dv0 = dv_prev + s_v y (device nv*3 doubles). */
pc_status pc_ws_predict(pc_ctx *ctx, const double *x, const double *v, const double *b, const double *dv_prev,
                        double *dv0_out, void *stream);
/* pc_ws_predict without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same result, bit for bit, from the
 * same two kernels, with the network's input rows kept in a scratch array of
 * the library (64 MiB in each GPU's memory, held from the library's first use
 * on that GPU until the process ends) instead of the context's buffer.  The
 * call allocates nothing and does not synchronise; the context must hold
 * the network's parameters (pc_ws_set_params) and an assembly.
 * Limit: nv rounded up to a multiple of 16 at most 1,048,576 vertices, else
 * PC_ERR_CAPACITY (pc_ws_predict has no such limit).  All contexts on one
 * GPU share the scratch, so calls that overlap on one GPU (other threads,
 * other streams without ordering between them) race and must be serialised
 * by the caller.  PC_ERR_ARG for null pointers, missing parameters or
 * assembly. */
pc_status pc_ws_predict_noalloc(pc_ctx *ctx, const double *x, const double *v, const double *b,
                                const double *dv_prev, double *dv0_out, void *stream);
/* The learned CG start used by warm = 2: dv_prev + g u (device nv*3
 * doubles), step g to step_host (optional).  Synchronises the stream. */
pc_status pc_ws_start(pc_ctx *ctx, const double *x, const double *v, const double *b, const double *dv_prev,
                      double *dv0_out, double *step_host, void *stream);
/* Loss and its gradient with respect to the parameters (host floats, same
 * layout as the parameters); no update.  Synchronises the stream. */
pc_status pc_ws_gradient(pc_ctx *ctx, const double *x, const double *v, const double *b, const double *dv_prev,
                         float *grad_host, double *loss_host, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, FP32 master weights) on
 * the loss of the assembled system.  loss_host (optional) synchronises. */
pc_status pc_ws_train_step(pc_ctx *ctx, const double *x, const double *v, const double *b, const double *dv_prev,
                           double lr, double *loss_host, void *stream);
/* Matrix-core lane-layout self test: D = A*B for two known 16x16 BF16 pairs
 * (A[i][k] = 16i+k, B = I; then A = I, B[k][j] = 16k+j) with the 16x16x16
 * instruction, then the 16x16x32 instruction on the concatenated tile pairs
 * (A0, A1) with A0[i][k] = 16i+k, A1[i][k] = 256-16i-k, and (B0, B1) = (I, 0),
 * then (0, I); out_host receives the four 16x16 FP32 results, row-major
 * (1024 floats: A, B, A0, A1 when the layout is the one the kernels use). */
pc_status pc_mfma_probe(pc_ctx *ctx, float *out_host);

/* Context options.  The schedule options (graph chunk, slices and rows per
 * block, LDS window, narrow columns) do not change results bit for bit,
 * except that the rows per vector block regroup the partial sums of the CG
 * dots; PC_OPT_INNER_FP32 changes them at the inner solves' rounding level.
 * PC_OPT_GRAPH_CHUNK: when > 0, CG iterations are captured once into a HIP
 *   graph of that many iterations (rounded up to even) and replayed on the
 *   caller's stream; the per-instance convergence flags make iterations
 *   after convergence exit at once.  0 (default): plain launches.  While
 *   pc_profile sampling is on, the sampled chunk (one in 8) runs as plain
 *   launches, which the events time.
 * PC_OPT_SPMV_SLICES_PER_BLOCK: 64-row slices per SpMV work item / block
 *   (1, 2, 4, 8 (default) or 16).
 * PC_OPT_VECTOR_ROWS_PER_BLOCK: rows per work item of the CG vector kernels
 *   (multiple of 64 in [64, 4096], default 2048; 1024 threads per block).
 *   Every block of the update kernel sums its instance's SpMV partials and
 *   every block of the direction kernel its instance's update partials, so
 *   fewer, larger work items cost less per iteration on large instances.
 * PC_OPT_LDS_WINDOW: 1 (default): each SpMV work item whose block columns
 *   span at most 4096 rows first copies that window of the search direction
 *   to LDS and gathers from there; 0: all gathers from global memory.
 * PC_OPT_NARROW_COLUMNS: 1 (default): when every block column lies within
 *   +-32767 rows of its 64-row slice (true for meshes numbered in grid
 *   order), the CG SpMV reads 16-bit column offsets instead of 32-bit
 *   columns; 0: always 32-bit.  Results do not change.
 * PC_OPT_SPMV_NARROW_ACTIVE (read only, pc_get_option): 1 when the CG SpMV
 *   of the last solve read 16-bit column offsets, else 0.
 * PC_OPT_INNER_FP32: 1 (default): with BF16 or FP16 blocks and the textbook
 *   recurrences, each refinement sweep solves for a correction e (x += e at
 *   the sweep's end) with the correction, residual and product vectors in
 *   FP32 (dots still accumulate in FP64; the sweep's start residual and the
 *   convergence test use FP64 x and the FP64 blocks); 0: FP64 vectors.
 *   Results change at the inner solves' rounding level only.
 * PC_OPT_KEEP_DIRECTION: 0 (default): every refinement sweep restarts CG
 *   from P^-1 r (default inner reduction 1e-2); 1 (experimental): with FP16
 *   blocks and the textbook recurrences, a sweep that follows a sweep
 *   without breakdown keeps the search direction: its residual is replaced
 *   by the FP64 one and the next direction is P^-1 r + beta p with beta =
 *   r.P^-1 r over the r.P^-1 r the old direction was built from (residual
 *   replacement), with a default inner reduction of 0.5.  It saves
 *   iterations on small sheets and costs them on large ones at some steps.
 *   BF16 blocks always restart. */
typedef enum { PC_OPT_GRAPH_CHUNK = 0, PC_OPT_SPMV_SLICES_PER_BLOCK = 1, PC_OPT_VECTOR_ROWS_PER_BLOCK = 2,
               PC_OPT_LDS_WINDOW = 3, PC_OPT_NARROW_COLUMNS = 4, PC_OPT_SPMV_NARROW_ACTIVE = 5,
               PC_OPT_INNER_FP32 = 6, PC_OPT_KEEP_DIRECTION = 7 } pc_option;
pc_status pc_set_option(pc_ctx *ctx, int32_t option, int64_t value);
pc_status pc_get_option(pc_ctx *ctx, int32_t option, int64_t *value);

/* Autotuner: on the assembled system and right-hand side b (device nv*3),
 * time `iters` CG iterations for every candidate schedule (slices per SpMV
 * block 2/4/8/16 x rows per vector block 1024/2048/4096 and, for k = 1, 2, the
 * smallest multiple of 64 giving at most k vector work items per compute unit
 * x graph chunk 0/32) with HIP events on the stream, and keep the fastest.  precond: the
 * preconditioner the iterations use (as pc_solve_opts.precond).  chosen
 * (host, optional) receives {slices per block, rows per block, graph chunk};
 * ms_per_iter (host, optional) the best time per iteration.  Overwrites the
 * solver's work vectors (not dv, not b).  Synchronises the stream. */
pc_status pc_autotune(pc_ctx *ctx, const double *b, int32_t iters, int32_t precond, int64_t *chosen,
                      double *ms_per_iter, void *stream);

/* ---- Many independent cloths in one context (project addition) ----
 * The mesh given to pc_create is the concatenation of ninst cloths occupying
 * the vertex ranges [vertex_begin[i], vertex_begin[i+1]) (host, ninst+1
 * entries, vertex_begin[0] = 0, vertex_begin[ninst] = nv); no triangle may
 * join two ranges (PC_ERR_MESH).  Each instance then gets its own CG scalars,
 * convergence test and refinement sweeps, while every kernel launch covers all
 * instances (instances that have converged skip their work).  Call before
 * cloth_assemble.  After a solve, pc_get_instance_info copies the per-instance
 * results (host array of ninst); the pc_solve_info of cloth_pcg_solve /
 * cloth_step then holds the largest iteration count and residuals. */
pc_status pc_set_instances(pc_ctx *ctx, const int32_t *vertex_begin, int32_t ninst);
pc_status pc_get_instance_info(pc_ctx *ctx, pc_solve_info *infos, int32_t n);

/* Synchronise the stream and report device-side errors of earlier calls. */
pc_status pc_check(pc_ctx *ctx, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PCLOTH_H */
