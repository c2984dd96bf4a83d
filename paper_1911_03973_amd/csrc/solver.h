// solver.h -- solver workspace and device state record (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fem.h"
#include "plan.h"

namespace fem {

// The device index of a plan created by fem_plan_create (api.hip).
DevPlan plan_device(const fem_plan *p);

enum IterMode { MODE_CONTINUE = 0, MODE_FRESH = 1, MODE_FIRST = 2 };

// Every solver stops once its FP64 true residual is at most
// kCertify * rtol * ||r_0||.  The margin covers what separates this residual
// from an independent FP64 evaluation of b - A x: the hi + lo pair carries
// A_e to about 2^-48 relative instead of FP64's 2^-53, and the sums run in
// another order.  Measured at 2048^2 squares the two evaluations agree to
// about 1e-4 relative, a hundredth of the margin.
constexpr double kCertify = 0.99;

// Scalars of the CG recurrence.  Each field has exactly one writer kernel
// (the single-block finalize / refresh kernels); the element kernels only read
// it, after a kernel boundary on the same stream.
struct IterState {
    int flag;       // 0 running, 1 trigger (target or reliable update), 2 breakdown
    int mode;       // IterMode of the next element pass
    int pending;    // 1: alpha * (p, q) not yet applied to (x, r)
    int n_updates;  // CG iterations completed (alpha known)
    double alpha;   // step of the last completed iteration
    double beta;    // p = z + beta p for the next element pass
    double rz;      // r.z of the residual behind the current p (summed directly)
    double rr;      // r.r of the same residual
    double rz_next, rr_next;
    double rr64;    // r.r of the FP64 residual at the last refresh
    double pq;      // last p.q
    double thr2;    // (kCertify rtol ||r_0||)^2: a recursive r.r at or below it triggers a refresh
    double rel2;    // delta^2 r.r at the last refresh: the reliable-update trigger (0: none)
};

struct Grids {
    size_t lds = 0;
    int gm = 1, gf = 0, gu = 1;
};

// Per-plan, per-precision workspace (one device arena).
struct SolverWork {
    int kind = -1;
    void *arena = nullptr;
    size_t bytes = 0;
    void *Apk = nullptr;          // packed difference form: FP64 [np][ne] or FP32 pair [2][np][ne]
    double *d64 = nullptr;        // diagonal of the operator
    void *dinv = nullptr;         // D^{-1} (0 on Dirichlet nodes), vector type
    void *r = nullptr, *p = nullptr, *q = nullptr, *xc = nullptr;  // iteration vectors
    double *r64 = nullptr;        // FP64 residual of a refresh
    double *part64 = nullptr;     // shared-node partials of FP64 passes
    void *partv = nullptr;        // shared-node partials of iteration passes
    double *dots = nullptr;       // [8][npart] per-block dot partials
    void *xl = nullptr;           // FP64 iterate in the solver-local node order
    int32_t *perm = nullptr;      // local index -> mesh node id
    double *upd = nullptr;        // [3][gu] init partials
    IterState *st = nullptr;
    int *bad = nullptr;
    // check_every iterations of the element pass, fix-up and finalize captured
    // into a HIP graph (kernel arguments are all workspace pointers and plan
    // sizes, so one capture serves every later solve with the same kernels)
    hipStream_t cap = nullptr;
    hipGraphExec_t graph = nullptr;
    const void *graph_key = nullptr;
    int graph_m = 0;
};

Grids solver_grids(const DevPlan &P, size_t elem_lds);

// Per-problem record of the batched solver (written by that problem's FIN
// item, read by its element items after a release/acquire hand-over).
struct BatchProblem {
    int flag;       // 1 once the problem is finished
    int status;     // fem_status of the problem
    int round;      // 0 iteration round, 1 refresh round
    int mode;       // IterMode of the next iteration round
    int pending;    // alpha * p not yet applied to x
    int iters, refreshes, first, broken;
    int grp;        // chunks per CHUNK item of the current phase
    double alpha, beta, rz;
    double r0, thr2, rel2, rr_true;
};

// Everything one persistent batched launch needs (device pointers).
constexpr int kBatchSeg = 1024;  // shared nodes per fix-up segment of the batched solver

struct BatchLaunch {
    DevPlan P;  // union of all problems
    const void *A;
    double *x, *r, *p, *q;  // solver-local order (DevPlan::comp_off); shared nodes are the tail
    const double *dinv, *b;
    double *part;
    const int32_t *pchunk0, *pshared0, *pseg0;
    const int32_t *pgroup;  // [P] chunks per work item
    int inline_segs;        // fix-up segments run inline by the last chunk item
    int adaptive;           // regroup a problem's items by the number of problems left
    const int32_t *pitem0;  // [P+1] prefix of the work items of a chunk round
    int64_t n_seed;         // work items of one chunk round of all problems
    int nprob;
    BatchProblem *prob;
    int *cnt;
    double *cdots, *sdots;
    unsigned long long *qitems, *qtags, *qhead, *qtail;
    unsigned long long qcap;
    int *ndone, *abort_flag;
    double rtol, delta;
    int max_iter, max_refresh;
    double watchdog_seconds;
    int block, grid;
};

int batch_pack(const DevPlan &P, int kin, const void *K, const void *M, const double *d_nu, const int64_t *d_elem0,
               int nprob, float *A, hipStream_t s);
int batch_launch(const BatchLaunch &L, hipStream_t s);

int solve_pcg(const DevPlan &P, SolverWork &w, int dtype, int vec64, int block, const void *K, const void *M,
              double nu, const double *b, double *x, double rtol, int max_iter, int jacobi, double delta,
              int max_outer, int check_every, int profile, fem_solve_info *info, hipStream_t s);

// Number of values of the packed symmetric difference form of one element:
// n_b row sums followed by the n_b (n_b - 1) / 2 upper off-diagonal entries.
__host__ __device__ constexpr int packed_count(int nb) { return nb + nb * (nb - 1) / 2; }

// Flexible CG (fcg.hip).  With a network, a non-finite or zero network
// output, p.q <= 0, or stall_iters iterations without halving ||r|| end the
// FCG phase with kFcgHandover (x reset to x0, res.rnorm its true residual
// norm) so that the caller continues with Jacobi-PCG; without a network the
// preconditioner is Jacobi throughout.
struct FcgResult {
    int status, iters, precond_calls, fell_back, fallback_reason, replacements;
    double relres, r0, rnorm;
};
constexpr int kFcgHandover = 1;

// The paper's iterations (iterate.hip); numbering as fem_iteration in fem.h.
enum IterMethod { ITER_RICHARDSON = 0, ITER_CHEB2 = 1, ITER_CHEB3 = 2, ITER_CHEB3_LISTING = 3 };
struct IterResult {
    int iters;
    double r0, relres;
};
int run_iteration(const DevPlan &P, int dtype, const void *K, const void *M, double nu, const double *b, double *x,
                  int method, double lam1, double lam2, int cycle, int iters, IterResult &res, hipStream_t s);
int solve_fcg(const DevPlan &P, int dtype, const void *K, const void *M, double nu, const double *b, double *x,
              double rtol, int max_iter, fem_unet *net, int grid_n, double cval, int smooth, double omega,
              int stall_iters, int max_replace, int graph, int check_every, int cycle_heads, FcgResult &res,
              hipStream_t s);
// z = B(r) once: the preconditioner of solve_fcg with the same arguments.
int fcg_precondition(const DevPlan &P, int dtype, const void *K, const void *M, double nu, fem_unet *net, int grid_n,
                     double cval, int smooth, double omega, int cycle_heads, const double *r, double *z,
                     hipStream_t s);

}  // namespace fem
