/*
 * fem.h -- C ABI of libfem.so: element-based P1 finite-element operators and
 * solvers for -Laplace(u) + nu u = f on MI355X (gfx950).
 *
 * Method (Marcinkowski & Valdman, "MATLAB Implementation of Element-based
 * Solvers"): the local stiffness and mass matrices K_e, M_e of every element
 * are built at once and kept as element arrays (Section 1, eq. (2)-(3));
 * the residual r = b - A x with A = sum_e C_e^T (K_e + nu M_e) C_e is formed
 * element by element without ever assembling a sparse matrix (Section 2,
 * eq. (4), Algorithm 1), and iterative solvers are driven by it.
 *
 * Conventions shared by every entry point
 *  - Device memory: every d_* pointer is caller-owned device memory on the
 *    current HIP device.  The library never frees it.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  All
 *    calls only enqueue work on it and return before it runs, except
 *    fem_plan_create and the solvers, which synchronise `stream` before
 *    returning.
 *  - Layouts (structure of arrays, n_b = dim + 1, or 6 / 10 for quadratic triangles / tetrahedra):
 *      coordinates      double [dim][n_nodes]
 *      connectivity     int32  [n_b][n_elems], 0-based node ids
 *      element matrices [n_b*n_b][n_elems]: entry (i,j) of element e at
 *                       (i*n_b + j)*n_elems + e, element order as given to
 *                       fem_plan_create.
 *      dtype FEM_F64    double entries
 *      dtype FEM_F32    float entries
 *      dtype FEM_F32X2  float [2][n_b*n_b][n_elems]: first block hi = fl32(a),
 *                       second block lo = fl32(a - hi); hi + lo represents the
 *                       FP64 value to about 2^-48 relative.
 *      nodal vectors    double [n_nodes] unless the name says f32.
 *  - Errors: every function returns a fem_status; nothing is launched when
 *    argument validation fails.  fem_last_error() returns a thread-local
 *    message for the last failure.  No C++ exception crosses this boundary.
 *  - Determinism: no floating-point atomics are used; each node's sum is
 *    taken in a fixed order, so repeated calls give bitwise identical results.
 */
#ifndef FEM_H
#define FEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FEM_OK = 0,
    FEM_EINVAL = -1,      /* bad size, pointer, index, element or parameter */
    FEM_EHIP = -2,        /* a HIP runtime call failed */
    FEM_ENOCONV = -3,     /* iteration limit reached; last iterate kept */
    FEM_ESINGULAR = -4,   /* nu = 0 without Dirichlet nodes (Section 1) */
    FEM_EBREAKDOWN = -5,  /* p^T A p <= 0 or a non-finite scalar in CG */
    FEM_ENOMEM = -6       /* device or host allocation failed */
} fem_status;

/* FEM_MFREE: matrix-free.  No element array is read: K_e and M_e are rebuilt
 * in FP64 from the plan's coordinates inside every element pass (the formulas
 * of Section 1, eq. (2)).  Accepted by fem_element_residual, fem_jacobi_diag,
 * fem_assemble_rhs and fem_pcg_solve, whose d_K_e / d_M_e are then ignored
 * (NULL allowed); the pass's LDS also holds the chunk's node coordinates, so
 * large chunks may exceed the workgroup limit (FEM_EINVAL: build the plan
 * with smaller chunk_elems). */
typedef enum { FEM_F64 = 0, FEM_F32 = 1, FEM_F32X2 = 2, FEM_MFREE = 3 } fem_dtype;

typedef enum { FEM_PRECOND_NONE = 0, FEM_PRECOND_JACOBI = 1 } fem_precond;

typedef struct fem_plan fem_plan; /* opaque */

typedef struct {
    int dim, n_b;
    int64_t n_nodes, n_elems;
    int64_t n_dirichlet;
    int chunk_elems;          /* elements per chunk (one workgroup pass) */
    int64_t n_chunks;
    int64_t n_local;          /* sum over chunks of distinct nodes touched */
    int64_t n_shared;         /* nodes touched by more than one chunk */
    int64_t n_partials;       /* (chunk, shared node) pairs */
    int64_t index_bytes;      /* device bytes of the plan's index arrays */
} fem_plan_stats;

/* Build the device plan of a simplicial mesh (Section 1: the element -> node
 * tables that replace the Boolean C_e / R_e of eq. (3) and Algorithm 1).
 *  dim            2 (triangles, n_b = 3) or 3 (tetrahedra, n_b = 4)
 *  d_coords       double [dim][n_nodes]   (read; not kept)
 *  d_conn         int32  [n_b][n_elems]   (read; not kept)
 *  d_dirichlet    int32  [n_dirichlet] node ids of the Dirichlet part nd
 *                 (duplicates allowed; may be NULL when n_dirichlet = 0)
 *  chunk_elems    elements per chunk, 0 = default (1024 for triangles, 1536
 *                 for tetrahedra); one of 64, 128, 256, 512, 1024, 1536 and,
 *                 for triangles only, 2048
 * The plan partitions the element list into chunks of consecutive elements;
 * element orders with spatial locality (e.g. a Morton order of the cells)
 * give compact chunks and the fewest shared nodes.  Errors: FEM_EINVAL for a
 * node id out of range, repeated nodes in an element, a Dirichlet id out of
 * range or a degenerate (zero-volume) element; FEM_ENOMEM; FEM_EHIP. */
int fem_plan_create(int dim, int64_t n_nodes, int64_t n_elems, const double *d_coords,
                    const int32_t *d_conn, const int32_t *d_dirichlet, int64_t n_dirichlet,
                    int chunk_elems, void *stream, fem_plan **out);

/* The same for quadratic (P2) elements, the higher-order elements of the
 * paper's outlook, with straight edges.  dim 2: triangles, connectivity int32
 * [6][n_elems] listing each triangle's vertices, then the midpoints of its
 * edges (0,1), (1,2), (2,0); chunk_elems 64 ... 1024 (default 1024).  dim 3:
 * tetrahedra, connectivity int32 [10][n_elems] listing the vertices, then the
 * midpoints of the edges (0,1), (0,2), (0,3), (1,2), (1,3), (2,3);
 * chunk_elems 64 ... 512 (default 512).  Element matrices are [n_b^2][n_elems]
 * in the same layouts; fem_build_local_matrices integrates the quadratic
 * Lagrange functions exactly.  The residual, diagonal, right-hand side and
 * fem_pcg_solve (stored FEM_F64 / FEM_F32X2 / FEM_F32 matrices, FP64 vectors)
 * accept such a plan; the matrix-free operator, the iterations, flexible CG,
 * multigrid and the batched solver return FEM_EINVAL.  FEM_EINVAL for dim
 * other than 2 or 3. */
int fem_plan_create_p2(int dim, int64_t n_nodes, int64_t n_elems, const double *d_coords, const int32_t *d_conn,
                       const int32_t *d_dirichlet, int64_t n_dirichlet, int chunk_elems, void *stream,
                       fem_plan **out);

/* Host-only dry run of fem_plan_create on host arrays (coords double
 * [dim][n_nodes], conn int32 [n_b][n_elems], dirichlet int32 [n_dirichlet]):
 * the same validation and chunking, no device memory and no HIP call.  Fills
 * *out (index_bytes counts the arrays that fem_plan_create would upload).
 * Useful to validate a mesh or size a plan on a machine without a GPU. */
int fem_plan_check_host(int dim, int64_t n_nodes, int64_t n_elems, const double *coords,
                        const int32_t *conn, const int32_t *dirichlet, int64_t n_dirichlet,
                        int chunk_elems, fem_plan_stats *out);

/* The same dry run for quadratic elements (conn int32 [6][n_elems] in 2D,
 * [10][n_elems] in 3D, as fem_plan_create_p2).  FEM_EINVAL for dim other than
 * 2 or 3. */
int fem_plan_check_host_p2(int dim, int64_t n_nodes, int64_t n_elems, const double *coords,
                           const int32_t *conn, const int32_t *dirichlet, int64_t n_dirichlet,
                           int chunk_elems, fem_plan_stats *out);

/* Free the plan and all device memory it owns.  NULL is accepted. */
int fem_plan_destroy(fem_plan *plan);

/* Sizes of the plan (host struct, caller-owned). */
int fem_plan_get_stats(const fem_plan *plan, fem_plan_stats *out);

/* Local matrices of every element (Section 1, eq. (2) restricted to one
 * element, computed for all elements at once as in Section 1):
 *   vol  = |det B| / dim!,  B = [p_1 - p_0, ..., p_dim - p_0]
 *   K_e  = vol * G G^T,  G = D_ref B^{-1},  D_ref = [-1 ... -1 ; I]
 *   M_e  = vol / ((dim+1)(dim+2)) * (1 + delta_ij)
 * computed in FP64 and stored in `dtype`.  d_K_e / d_M_e / d_vol (double
 * [n_elems]) may each be NULL to skip that output. */
int fem_build_local_matrices(const fem_plan *plan, int dtype, void *d_K_e, void *d_M_e,
                             double *d_vol, void *stream);

/* A_e = K_e + nu M_e (definition under Algorithm 1), evaluated in FP64 from
 * inputs of dtype_in and stored as dtype_out.  d_M_e may be NULL (A_e = K_e).
 * Output must not alias the inputs. */
int fem_combine_local(const fem_plan *plan, int dtype_in, const void *d_K_e, const void *d_M_e,
                      double nu, int dtype_out, void *d_A_e, void *stream);

/* Residual r = b - sum_e C_e^T (K_e + nu M_e) C_e x  (eq. (4), Algorithm 1),
 * computed in FP64 from local matrices of `dtype` (FEM_F32X2 uses hi + lo).
 * d_M_e may be NULL (then A_e = K_e and nu is ignored); d_b may be NULL
 * (b = 0, i.e. r = -A x).  With mask_dirichlet != 0 the rows of the Dirichlet
 * nodes are set to 0 (r(nd) = 0 in the Section 2 listings).  d_r must not
 * alias d_x or d_b. */
int fem_element_residual(const fem_plan *plan, int dtype, const void *d_K_e, const void *d_M_e,
                         double nu, const double *d_b, const double *d_x, double *d_r,
                         int mask_dirichlet, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * residual as fem_element_residual, same arguments, validation and results
 * bit for bit, with the shared-node partials of the element pass in a
 * file-scope device array of the library (2^22 FP64 values, 32 MiB, held on
 * every GPU the library runs on until the process ends) instead of the plan's
 * workspace.  FEM_EINVAL if the plan has more than 2^22 shared-node partials
 * (fem_plan_stats.n_partials).  Calls nothing that allocates.  Every call on
 * one GPU uses that GPU's one array: calls that overlap on a GPU (two streams,
 * two host threads) race and must be serialised by the caller.  No slot needs
 * to start at zero: each one read is written earlier in the same call. */
int fem_element_residual_noalloc(const fem_plan *plan, int dtype, const void *d_K_e, const void *d_M_e, double nu,
                                 const double *d_b, const double *d_x, double *d_r, int mask_dirichlet,
                                 void *stream);

/* The same residual entirely in FP32: combined local matrices d_A_e (float,
 * [n_b*n_b][n_elems]), float vectors and float accumulation.  This is the
 * inner operator of the mixed-precision solver.  d_b may be NULL. */
int fem_element_residual_f32(const fem_plan *plan, const float *d_A_e, const float *d_b,
                             const float *d_x, float *d_r, int mask_dirichlet, void *stream);

/* Diagonal of the assembled operator, d_i = sum_{e contains i} (A_e)_{ii},
 * A_e = K_e + nu M_e (Jacobi preconditioner).  Rows of Dirichlet nodes are
 * not masked. */
int fem_jacobi_diag(const fem_plan *plan, int dtype, const void *d_K_e, const void *d_M_e,
                    double nu, double *d_diag, void *stream);

/* Right-hand side b = sum_e C_e^T M_e f_e (eq. (2) with f replaced by its
 * nodal interpolant d_f, eq. (3) assembly), FP64. */
int fem_assemble_rhs(const fem_plan *plan, int dtype, const void *d_M_e, const double *d_f,
                     double *d_b, void *stream);

typedef struct {
    int dtype;          /* storage of d_K_e / d_M_e.  FEM_F64: FP64 solve.
                           FEM_F32X2 or FEM_F32: mixed precision -- the CG
                           iterations read FP32 local matrices, while dot
                           products, alpha/beta and every refresh of the
                           residual b - A x are FP64 (iterative refinement,
                           the refresh using the full input precision).
                           FEM_MFREE: FP64 solve with the matrix-free
                           operator (d_K_e, d_M_e ignored; vectors = 0). */
    double nu;          /* >= 0 */
    double rtol;        /* stop at ||b - A x||_2 <= rtol ||b - A x0||_2 */
    int max_iter;       /* cap on CG iterations (inner ones summed) */
    int precond;        /* fem_precond */
    double inner_rtol;  /* mixed precision: the FP64 residual is refreshed
                           whenever the iterated residual norm has fallen by
                           this factor since the last refresh */
    int max_outer;      /* mixed precision: cap on refreshes */
    int check_every;    /* host reads the convergence flag every k iterations */
    int profile;        /* record HIP events around every `profile`-th matvec */
    int vectors;        /* mixed precision: 0 = FP64 iteration vectors,
                           1 = FP32 iteration vectors */
    int block;          /* workgroup size of the element pass: 256, 512,
                           1024, or 0 for the default */
} fem_solve_opts;

typedef struct {
    int status;          /* fem_status of the solve */
    int iters;           /* CG iterations performed (all inner ones) */
    int outer;           /* refinement steps (mixed precision), else 0 */
    int replacements;    /* FP64 residual replacements after the recursive
                            residual met rtol but the true one did not */
    double relres;       /* true FP64 ||b - A x||_2 / ||b - A x0||_2 (masked) */
    double r0;           /* ||b - A x0||_2 (masked) */
    double seconds;      /* host wall time of the call */
    double matvec_ms;    /* profile: summed time of the timed matvecs */
    int matvec_samples;  /* profile: number of timed matvecs */
    int matvec_calls;    /* matvecs issued (inner + outer residuals) */
} fem_solve_info;

void fem_solve_opts_default(fem_solve_opts *o);

/* Preconditioned conjugate gradients for (K + nu M) u = b with the Dirichlet
 * rows masked (Section 1 problem, residual of eq. (4) with r(nd) = 0).
 * d_K_e, d_M_e are the local matrices in opts->dtype layout (d_M_e may be NULL
 * when nu = 0).  d_x holds x0 on entry, including the Dirichlet values on nd,
 * and the last iterate on exit.  Returns FEM_OK, FEM_ENOCONV (iteration cap;
 * d_x holds the last iterate and info is filled), FEM_EBREAKDOWN,
 * FEM_ESINGULAR (nu == 0 and no Dirichlet node), FEM_EINVAL.  The plan keeps
 * per-dtype workspace that is allocated on the first solve; the iterations
 * themselves allocate nothing.  Synchronises `stream` before returning. */
int fem_pcg_solve(const fem_plan *plan, const fem_solve_opts *opts, const void *d_K_e,
                  const void *d_M_e, const double *d_b, double *d_x, fem_solve_info *info,
                  void *stream);

/* ------------------------------------------------------------------------ */
/* Batches of independent problems solved in one persistent launch.           */
/* ------------------------------------------------------------------------ */
typedef struct fem_batch fem_batch; /* opaque */

/* Plan for n_problems independent meshes given back to back:
 *  node_off, elem_off, dir_off  host int64 [n_problems + 1] prefix offsets
 *  d_coords     double [dim][node_off[P]] (union of all problems, SoA)
 *  d_conn       int32  [n_b][elem_off[P]], node ids LOCAL to each problem
 *  d_dirichlet  int32  [dir_off[P]], node ids local to each problem
 * Every problem is validated and chunked as by fem_plan_create (no chunk
 * holds elements of two problems).  The union of the problems is itself a
 * mesh: the union-level calls below act on all problems at once. */
int fem_batch_create(int dim, int n_problems, const int64_t *node_off, const int64_t *elem_off,
                     const int64_t *dir_off, const double *d_coords, const int32_t *d_conn,
                     const int32_t *d_dirichlet, int chunk_elems, void *stream, fem_batch **out);
int fem_batch_destroy(fem_batch *batch);
int fem_batch_get_stats(const fem_batch *batch, fem_plan_stats *out);

/* Union-level operations, same layouts and semantics as the single-plan calls
 * (element arrays over elem_off[P] elements, vectors over node_off[P] nodes). */
int fem_batch_build_local_matrices(const fem_batch *batch, int dtype, void *d_K_e, void *d_M_e,
                                   void *stream);
int fem_batch_assemble_rhs(const fem_batch *batch, int dtype, const void *d_M_e, const double *d_f,
                           double *d_b, void *stream);

typedef struct {
    int dtype;               /* storage of K_e / M_e (FEM_F64, FEM_F32, FEM_F32X2) */
    double rtol;             /* per problem: ||b - A x|| <= rtol ||b - A x0|| */
    int max_iter;            /* per-problem cap on CG iterations */
    double refresh;          /* FP64 residual refresh when r.r fell by refresh^2 */
    int max_refresh;         /* per-problem cap on refreshes */
    int block;               /* workgroup size 256/512/1024, 0 = default */
    int grid;                /* persistent workgroups, 0 = fill the GPU */
    double watchdog_seconds; /* abort if the work queue stays empty this long */
    int use_graph;           /* 1: capture the solve in a HIP graph and replay it */
    int group;               /* chunks per work item, 0 = per-problem schedule */
    int items_per_phase;     /* per-problem schedule: target work items per
                                phase (a problem of n chunks takes
                                ceil(n / items_per_phase) chunks per item;
                                default 4) */
    int inline_segments;     /* a problem with at most this many shared-node
                                segments (1024 nodes each) has its fix-up and
                                scalar step run by the workgroup finishing its
                                last chunk item, one queue trip per iteration
                                (default 64; 0: always separate items) */
    int adaptive;            /* 1 (default; ignored when group > 0): once fewer
                                problems are left than the workgroups can keep
                                busy, a problem's phases are cut into more work
                                items (down to one chunk each) and its fix-up
                                runs as separate items.  Results are identical
                                either way (partials are per chunk/segment). */
} fem_batch_opts;

typedef struct {
    int status;              /* fem_status of this problem */
    int iters, refreshes;
    double relres;           /* true FP64 relative residual */
    double r0;
} fem_batch_result;

void fem_batch_opts_default(fem_batch_opts *o);

/* Solves every problem p: (K + nu[p] M) u = b with its Dirichlet rows masked,
 * x holding x0 (Dirichlet values) on entry and the solutions on exit; all
 * problems in one persistent kernel launch (work queue of (problem, chunk)
 * items, per-problem phase counters), optionally replayed from a captured
 * HIP graph.  h_nu: host double [P]; results: host [P]; *seconds: wall time.
 * Returns FEM_OK when every problem converged, else the first failing
 * problem's status (FEM_EHIP if the watchdog aborted the launch). */
int fem_batch_solve(fem_batch *batch, const fem_batch_opts *opts, const void *d_K_e, const void *d_M_e,
                    const double *h_nu, const double *d_b, double *d_x, fem_batch_result *results,
                    double *seconds, void *stream);

/* ------------------------------------------------------------------------ */
/* The paper's iterations on the element residual (Section 2)                 */
/* ------------------------------------------------------------------------ */
typedef enum {
    FEM_RICHARDSON = 0,         /* x += omega r, omega = 2 / (lam1 + lam2) (eq. (richardson)) */
    FEM_CHEBYSHEV2 = 1,         /* x += r / alpha_{k mod N}, roots of the scaled Chebyshev
                                   polynomial of degree N in the listing's order
                                   (eq. (Czebyshev2lev)) */
    FEM_CHEBYSHEV3 = 2,         /* three-level recurrence with C_{k+1} = 2 sigma C_k - C_{k-1}
                                   (eqs. (recrCk), (Czebyshev3lev)); first step r0 / d */
    FEM_CHEBYSHEV3_LISTING = 3  /* the alpha/beta form of the 3-level listing (its first
                                   beta is (c alpha / 2)^2) */
} fem_iteration;

typedef struct {
    int method;      /* fem_iteration */
    int dtype;       /* storage of K_e / M_e */
    double nu;
    double lam1, lam2; /* spectral bounds 0 < lam1 < lam2 of the masked operator */
    int cycle;       /* N of the 2-level method */
    int iters;       /* number of iterations (no stopping test, as in Section 3) */
} fem_iter_opts;

typedef struct {
    int status;
    int iters;
    double relres;   /* ||b - A x|| / ||b - A x0|| (masked, FP64) after the last step */
    double r0;
    double seconds;
} fem_iter_info;

void fem_iter_opts_default(fem_iter_opts *o);

/* Runs opts->iters steps of the chosen iteration on (K + nu M) u = b with the
 * Dirichlet rows masked (x holds the Dirichlet values, which stay fixed).
 * Each step is one element residual (eq. (4), Algorithm 1, through the FP64
 * packed difference form of A_e) and one vector update; the step sizes are
 * formed on the host in FP64 from (lam1, lam2, N, k).  Allocates a workspace
 * for the call; synchronises `stream`. */
int fem_iterate(const fem_plan *plan, const fem_iter_opts *opts, const void *d_K_e, const void *d_M_e,
                const double *d_b, double *d_x, fem_iter_info *info, void *stream);

/* ------------------------------------------------------------------------ */
/* Learned preconditioner: a U-Net on the structured nodal grid, used as     */
/* z = N(r) in flexible CG.  Section 3 notes that the iteration counts grow  */
/* with the condition number on finer meshes, so the solvers need a          */
/* preconditioner, and the Outlooks name preconditioners as the next step;   */
/* this one is trained on (residual, error) pairs from the Jacobi-PCG solver. */
/* ------------------------------------------------------------------------ */
typedef struct fem_unet fem_unet; /* opaque */

/* Create a U-Net for images of H x W pixels (multiples of 8) and batches of
 * up to max_batch images; channels = base width c (16 or 32).
 *  Architecture, level l at (H >> l) x (W >> l), NHWC BF16 activations:
 *    encoder  two 3x3 conv + ReLU per level (8->c, c->c | c->2c, 2c->2c |
 *             2c->4c, 4c->4c | 4c->8c, 8c->8c), 2x2 average pooling between
 *    decoder  2x2 stride-2 transposed conv (8c->4c, 4c->2c, 2c->c), concat
 *             with the encoder output of that level (up-sampled first), two
 *             3x3 conv + ReLU (2k->k, k->k)
 *    output   1x1 conv c->1 in FP32
 *  Input channels: 2 (the rest of the first layer's 8 are zero padding).
 *  Parameters: one FP32 vector, layer by layer, weights then bias:
 *    3x3 conv   W[ky*3+kx][ci][co] (input pixel (y+ky-1, x+kx-1), zero
 *               outside the image), bias[co]
 *    transposed W[ci][a*2+b][co]: output pixel (2y+a, 2x+b) gets
 *               sum_ci in(y,x,ci) W[ci][a*2+b][co] + bias[co]
 *    output     w[c], bias
 *  Arithmetic: BF16 operands on MFMA with FP32 accumulation; FP32 master
 *  weights, Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * Initial weights are He-normal from `seed` (biases 0).  Allocates its own
 * device memory; synchronises `stream`. */
int fem_unet_create(int H, int W, int max_batch, int channels, uint64_t seed, void *stream, fem_unet **out);
int fem_unet_destroy(fem_unet *net);
int fem_unet_param_count(const fem_unet *net, int64_t *count);
/* FP32 parameter vector in the layout above (device memory, count floats).
 * set_params also clears the Adam state. */
int fem_unet_get_params(const fem_unet *net, float *d_params, void *stream);
int fem_unet_set_params(fem_unet *net, const float *d_params, void *stream);
/* d_in float [batch][H][W][2] (NHWC), d_out float [batch][H][W]. */
int fem_unet_forward(fem_unet *net, int batch, const float *d_in, float *d_out, void *stream);
/* Training loss (fem_unet_set_loss; FEM_UNET_LOSS_L2 at creation), with
 * y_b = N(in_b) and t_b the target image of sample b:
 *  FEM_UNET_LOSS_L2      L = (1/batch) sum_b ||y_b - t_b||^2 / ||t_b||^2.
 *  FEM_UNET_LOSS_ENERGY  L = (1/batch) sum_b [1 - (y_b.A t_b)^2 / ((y_b.A y_b)(t_b.A t_b))]
 *      = the mean over b of min_s ||s y_b - t_b||_A^2 / ||t_b||_A^2: what is
 *      left of the error's energy after the energy-optimal step along y_b,
 *      the step flexible CG and the two-level cycle take.  A is the P1
 *      operator -Delta + nu I of Section 2 (eq. (4)) on the interior nodes of
 *      the unit square cut into H x H squares, each split by its diagonal from
 *      the lower-left to the upper-right corner, with u = 0 on the boundary:
 *      pixel (y, x) is node (x + 1, y + 1) as in fem_unet_precondition; the
 *      last row and column hold no node and enter neither y_b nor t_b.  On
 *      this grid A is the 5-point Laplacian plus nu h^2 (1/2 at the node, 1/12
 *      at its four axis and two diagonal neighbours), h = 1 / H.  nu_b =
 *      nu_scale * in_b(0, 0, channel 1).  A sample with y.Ay <= 0 or t.At <= 0
 *      counts 1 with zero gradient.  Needs H == W.
 * fem_unet_set_loss: kind FEM_UNET_LOSS_L2 or FEM_UNET_LOSS_ENERGY, nu_scale
 * finite >= 0 (ignored for L2); FEM_EINVAL otherwise. */
enum { FEM_UNET_LOSS_L2 = 0, FEM_UNET_LOSS_ENERGY = 1 };
int fem_unet_set_loss(fem_unet *net, int kind, double nu_scale);
/* Output smoothing (0 passes at creation): the 1x1 layer's output is followed
 * by `passes` (0..8) passes of the 3x3 binomial filter (1 2 1; 2 4 2; 1 2 1)/16
 * in FP32 over the pixels x < W-1, y < H-1 (the grid layout's nodes; the last
 * row and column are read and written as 0), in forward, loss, training and
 * fem_unet_precondition alike.  It damps the pixel-wise rounding noise of the
 * BF16 layers, which otherwise dominates the energy norm of a smooth output
 * (the noise's A-norm is ~4x its L2 norm, a smooth mode's ~2 pi^2 / H^2 x).
 * FEM_EINVAL outside [0, 8]. */
int fem_unet_set_output_smoothing(fem_unet *net, int passes);
/* Loss L (d_loss: one device double) and its gradient with respect to every
 * parameter (d_grad: device float [count], may be NULL).  d_target float
 * [batch][H][W]. */
int fem_unet_loss_grad(fem_unet *net, int batch, const float *d_in, const float *d_target, double *d_loss,
                       float *d_grad, void *stream);
/* One Adam step on L with learning rate lr (d_loss may be NULL). */
int fem_unet_train_step(fem_unet *net, int batch, const float *d_in, const float *d_target, float lr,
                        double *d_loss, void *stream);
/* z = N(r) on the structured grid of (grid_n + 1)^2 nodes numbered
 * i + j (grid_n + 1) (grid_n = H = W): the interior residual (1 <= i, j <=
 * grid_n - 1), divided by its RMS, is pixel (i-1, j-1) of channel 0, with the
 * last row and column zero; channel 1 is the constant cval.  The output is
 * written to the interior nodes; boundary nodes and nodes with d_mask != 0
 * (uint8 [n_nodes], may be NULL) get 0.  Allocates nothing. */
int fem_unet_precondition(fem_unet *net, int grid_n, const double *d_r, double cval, const uint8_t *d_mask,
                          double *d_z, void *stream);
/* One training pair of the learned preconditioner on the same grid (the
 * network's image size; grid_n = H = W): d_in (float [grid_n][grid_n][2]) gets
 * the network input of residual d_r exactly as fem_unet_precondition forms it,
 * d_target (float [grid_n][grid_n]) the error e = d_u - d_x on the interior
 * nodes divided by its RMS there (pixel (i-1, j-1) <- node (i, j); last row
 * and column 0; a zero e gives a zero image).  d_r, d_u, d_x: FP64
 * [(grid_n + 1)^2], caller-owned.  Uses the network's scratch, so calls on one
 * network must not overlap.  Allocates nothing. */
int fem_unet_make_pair(fem_unet *net, int grid_n, const double *d_r, const double *d_u, const double *d_x,
                       double cval, float *d_in, float *d_target, void *stream);

typedef struct {
    int dtype;          /* storage of K_e / M_e */
    double nu;
    double rtol;        /* stop when the FP64 ||b - A x|| <= rtol ||b - A x0|| */
    int max_iter;       /* FCG iterations, plus as many Jacobi-PCG ones after a handover */
    int grid_n;         /* structured grid of (grid_n + 1)^2 nodes (see fem_unet_precondition) */
    double cval;        /* constant second input channel of the network */
    int stall_iters;    /* hand over to Jacobi-PCG when ||r|| has not halved in this many
                           iterations (default 200) */
    int max_replace;    /* true-residual restarts allowed */
    int smooth;         /* 0: z = N(r); k > 0: two-level cycle with the network as
                           coarse correction: k damped-Jacobi steps
                           z += omega D^-1 (r - A z) from z = 0, then
                           z += s N(r - A z) with s = (n.rz)/(n.A n), then k
                           more Jacobi steps (default 4) */
    double omega;       /* Jacobi damping of the cycle, (0, 2) (default 2/3) */
    int graph;          /* 1: one whole iteration (cycle, network and FCG update) is
                           captured once per solve into a HIP graph and replayed
                           (default); 0: its kernels are launched one by one */
    int check_every;    /* iterations between two reads of the device state by the host,
                           [1, 4096] (default 16); the scalars never leave the device */
    int cycle_dtype;    /* FEM_F64: the cycle's element passes read the FP64 packed
                           operator (default); FEM_F32: its FP32 heads */
} fem_fcg_opts;

typedef struct {
    int status;
    int iters;          /* FCG iterations */
    int pcg_iters;      /* Jacobi-PCG iterations after a handover */
    int precond_calls;  /* network applications */
    int fell_back;      /* FCG iteration at which Jacobi-PCG took over, -1 if never */
    int fallback_reason;/* 0 none, 1 non-finite or zero network output,
                           2 p.q <= 0, 3 stall */
    int replacements;
    double relres;      /* true FP64 ||b - A x|| / ||b - A x0|| */
    double r0;
    double seconds;
} fem_fcg_info;

void fem_fcg_opts_default(fem_fcg_opts *o);

/* Flexible CG (FCG(1), Notay, SIAM J. Sci. Comput. 22 (2000), with one
 * previous direction) for (K + nu M) u = b with the Dirichlet rows masked --
 * the problem statement of Section 1, the operator applied through the
 * element residual of Section 2 (eq. (4), Algorithm 1) -- preconditioned by
 * the network (net != NULL; the mesh must be the structured 2D grid described
 * at fem_unet_precondition), alone or inside the two-level cycle of
 * opts->smooth, or by Jacobi (net == NULL; linear triangles or tetrahedra).
 * With a network, a non-finite or zero output, p.q <= 0, or stall_iters
 * iterations without halving ||r|| end the FCG phase: x is reset to x0 and
 * the Jacobi-PCG solver (fem_pcg_solve with opts->dtype) solves from there, so
 * that the fallback never needs more Jacobi-PCG iterations than a cold start
 * (from an iterate the network cycle has shaped it can need more).  The true FP64 residual decides convergence.  x: x0 on
 * entry (Dirichlet values included), the solution on exit; after
 * FEM_ENOCONV the last iterate.  Allocates a workspace for the call;
 * synchronises `stream`. */
int fem_fcg_solve(const fem_plan *plan, const fem_fcg_opts *opts, fem_unet *net, const void *d_K_e,
                  const void *d_M_e, const double *d_b, double *d_x, fem_fcg_info *info, void *stream);

/* z = B(r) once, B the preconditioner fem_fcg_solve uses with the same
 * opts and net: the two-level cycle (net, opts->smooth > 0), N(r)
 * (net, smooth == 0) or D^-1 r (net == NULL); D^-1 is 0 on Dirichlet nodes.
 * r: [n_nodes] FP64 (a masked residual: 0 on Dirichlet nodes), z: [n_nodes]
 * FP64, caller-owned, must not alias r.  Validation as fem_fcg_solve.
 * Allocates a workspace for the call; synchronises `stream`. */
int fem_fcg_precondition(const fem_plan *plan, const fem_fcg_opts *opts, fem_unet *net, const void *d_K_e,
                         const void *d_M_e, const double *d_r, double *d_z, void *stream);

/* ---- Geometric multigrid on nested square and cube meshes -----------------
 * The P1 operator's condition number grows like h^-2 (the reason the Section 3
 * iterations need spectral bounds, and the preconditioning the paper calls for
 * on fine meshes).  For the structured 2D meshes -- n x n squares cut along the
 * (0,0)-(1,1) diagonal, node (i, j) numbered j (n + 1) + i -- the mesh of n/2
 * squares is nested in that of n squares (red refinement); so is the 3D Kuhn
 * mesh of (n/2)^3 cubes in that of n^3 cubes (6 tetrahedra per cube around its
 * (0,0,0)-(1,1,1) diagonal, node (i, j, k) numbered (k (n+1) + j)(n+1) + i,
 * every vertex joined to its 14 neighbours +-e, e in {0,1}^3 \ {0}).  A V-cycle
 * over the hierarchy preconditions flexible CG:
 *   prolongation  exact P1 interpolation (fine (2I,2J) <- coarse (I,J); an odd
 *                 fine node <- the average of the two coarse ends of its edge,
 *                 the diagonal edge included);
 *   restriction   its transpose;
 *   smoothing     `smooth` damped-Jacobi steps before and after (omega), or
 *                 as many Chebyshev steps (fem_smoother);
 *   coarsest      exact solve through a dense inverse formed at setup.
 * Every operator application is the element residual (eq. (4), Algorithm 1)
 * through the FP64 packed difference form of the level's own K_e, M_e. */
typedef struct fem_mg fem_mg;

/* Smoothers of the V-cycle.  FEM_SMOOTH_CHEBYSHEV: `smooth` steps of the
 * three-level Chebyshev iteration (Section 2, eq. (9) with the scaling factors
 * of eq. (8)) for D^-1 A z = D^-1 r on [cheb_lower g, g], g the level's
 * Gershgorin bound of D^-1 A from the element matrices
 * (max over free i of D_ii^-1 sum_e sum_j |(A_e)_ij|, fem_mg_level_bound);
 * the same polynomial before and after the correction keeps the V-cycle
 * symmetric. */
typedef enum { FEM_SMOOTH_JACOBI = 0, FEM_SMOOTH_CHEBYSHEV = 1 } fem_smoother;

typedef struct {
    double rtol;      /* stop at ||b - A x|| <= rtol ||b - A x0|| (true FP64 residual) */
    int max_iter;     /* FCG iterations */
    int smooth;       /* smoothing steps before and after the coarse correction, in [1, 64] */
    double omega;     /* Jacobi damping, in (0, 2); default 2/3 (FEM_SMOOTH_JACOBI only) */
    int max_replace;  /* restarts from the true residual when the recursive one met rtol */
    int cycle_dtype;  /* FEM_F64 (default): the V-cycle's operator products in FP64; FEM_F32:
                         they read the FP32 heads of the packed operator (half the bytes;
                         FCG's own products and the true residual stay FP64) */
    int smoother;       /* fem_smoother; default FEM_SMOOTH_JACOBI */
    double cheb_lower;  /* FEM_SMOOTH_CHEBYSHEV: lower end of the interval as a fraction of g,
                           in (0, 1); default 0.3 */
} fem_mg_opts;

void fem_mg_opts_default(fem_mg_opts *o);

/* levels >= 2 plans, finest first: plans[l] a plan of the grid_n[l] x grid_n[l]
 * square mesh (or of the grid_n[l]^3 cube mesh; all levels of one dimension)
 * with grid_n[l] = 2 grid_n[l+1], its own Dirichlet set; d_K_e[l], d_M_e[l]
 * its local matrices in `dtype` layout (d_M_e may be NULL when nu == 0).  The
 * coarsest mesh may have at most 1089 nodes (33 x 33, 10^3).  The plans must
 * outlive the hierarchy; the matrices are read during the call only (packed
 * copies are kept).  FEM_EINVAL for a hierarchy that is not nested as
 * described, FEM_ESINGULAR for a non-positive diagonal or a singular coarsest
 * operator.  Synchronises `stream`. */
int fem_mg_create(int levels, const fem_plan *const *plans, const int *grid_n, int dtype,
                  const void *const *d_K_e, const void *const *d_M_e, double nu, void *stream, fem_mg **out);
int fem_mg_destroy(fem_mg *mg);

/* FCG(1) preconditioned by one V-cycle per iteration on the finest level's
 * problem (K + nu M) u = b, Dirichlet rows masked; x: x0 on entry (Dirichlet
 * values included), the solution on exit; info as fem_fcg_solve (pcg_iters,
 * fell_back unused).  Synchronises `stream`. */
int fem_mg_solve(fem_mg *mg, const fem_mg_opts *opts, const double *d_b, double *d_x, fem_fcg_info *info,
                 void *stream);

/* z = B r: one V-cycle on the finest level, as the solver applies it, with
 * the smoothing fields of opts (smooth, omega, smoother, cheb_lower,
 * cycle_dtype; the others are ignored).  r (n_nodes of the finest level, mesh
 * order) is read on free nodes only; z is written on every node, 0 on
 * Dirichlet nodes.  r and z must not alias.  Uses the hierarchy's own level
 * vectors, so calls on one hierarchy must not overlap (launches on one stream
 * are fine).  FEM_EINVAL for options out of range.  Asynchronous on `stream`. */
int fem_mg_vcycle(fem_mg *mg, const fem_mg_opts *opts, const double *d_r, double *d_z, void *stream);

/* *g = the Gershgorin bound of D^-1 A on `level` (0 = finest) that places the
 * Chebyshev smoother's interval, computed at fem_mg_create (1 on a level
 * without free nodes).  g is a host pointer. */
int fem_mg_level_bound(const fem_mg *mg, int level, double *g);

/* out = P^T A_level P zc for a vector zc of level level+1 (the Galerkin
 * product; on nested meshes without jitter it equals A_{level+1} zc on free
 * nodes).  For checking the transfer operators. */
int fem_mg_galerkin_apply(fem_mg *mg, int level, const double *d_zc, double *d_out, void *stream);

/* Thread-local message describing the last failure ("" if none). */
const char *fem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FEM_H */
