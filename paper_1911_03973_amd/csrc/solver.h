// solver.h -- solver workspace and device state record (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fem.h"
#include "plan.h"

namespace fem {

// Written only by thread 0 of block 0 of the kernel that owns each field,
// read by later kernels on the same stream.
struct SolveState {
    int flag;          // 0 running, 1 trigger (converged / reliable update), 2 breakdown
    int n_updates;     // CG updates executed
    double rz_cur;     // r.z of the current iteration (written by main)
    double rz_prev;    // r.z of the previous iteration (written by update)
    double beta, alpha;
    double rr_trigger;
    double rz_init, rr_init, rr64_init;  // totals of a fresh residual
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
    void *A = nullptr;             // combined local matrices: FP64 or FP32 hi/lo pair
    double *d64 = nullptr, *dinv64 = nullptr, *r64 = nullptr, *p64 = nullptr, *q64 = nullptr;
    float *dinv32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *xc32 = nullptr;
    double *part64 = nullptr;
    float *part32 = nullptr;
    double *upd = nullptr, *mv = nullptr;
    SolveState *st = nullptr;
    int *bad = nullptr;
};

Grids solver_grids(const DevPlan &P, size_t elem_lds);

int solve_pcg(const DevPlan &P, SolverWork &w, int dtype, const void *K, const void *M, double nu,
              const double *b, double *x, double rtol, int max_iter, int jacobi, double delta, int max_outer,
              int check_every, int profile, fem_solve_info *info, hipStream_t s);

}  // namespace fem
