// fcg.hip -- flexible conjugate gradients (FCG(1)) on the element residual,
// with a U-Net or Jacobi preconditioner.
//
// The operator is the residual of Section 2 (eq. (4), Algorithm 1) through the
// packed difference form in FP64.  FCG(1) keeps one previous direction and
// orthogonalises the new preconditioned residual against it explicitly,
//   p_k = z_k - (z_k . q_{k-1}) / (p_{k-1} . q_{k-1}) p_{k-1},  q_k = A p_k,
//   alpha_k = (p_k . r_k) / (p_k . q_k),
// which stays a descent method when the preconditioner z = B(r) is nonlinear
// or changes between iterations (Notay, SIAM J. Sci. Comput. 22 (2000)).
// The true residual judges convergence: when the recursive residual meets the
// tolerance, r = b - A x is recomputed in FP64 and the iteration restarts
// from it if the tolerance is not met.
//
// With a network and smooth > 0 the preconditioner is a two-level cycle in
// which the network plays the coarse correction: `smooth` damped-Jacobi steps
// z += omega D^-1 (r - A z) from z = 0, the network correction
// z += s N(r - A z) with the energy-optimal s = (n . rz) / (n . A n), and
// `smooth` more Jacobi steps.  The Jacobi steps are fused into one element
// pass each (the residual r - A z is never stored), except the first of each
// half: from z = 0 it is omega D^-1 r, and after the coarse correction the
// residual is r_z - s A n from the products the correction formed already.
//
// The scalars live on the device: single-workgroup kernels add the per-block
// dot partials in a fixed order and write the FCG scalars and a stop flag
// into a state record, which every later kernel of the iteration reads after
// a kernel boundary.  A whole iteration -- the cycle with the network's
// launches and the FCG update -- is captured once into a HIP graph and
// replayed; the host reads the state record every `check_every` iterations
// only.  Once a kernel has raised the flag, the FCG kernels of the iterations
// still queued return at once (the cycle's own launches run on scratch
// vectors and change nothing the solve keeps).
//
// With a network, x0 is kept: a hand-over to Jacobi-PCG restarts from it.
// Measured at 1024^2, Jacobi-PCG from an iterate the network cycle had
// shaped (even one that had halved ||r|| several times) needed 1.4-1.9x the
// iterations of a cold start, so the fallback costs at most the FCG steps
// already taken plus a cold Jacobi-PCG solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "chunk.h"
#include "common.h"
#include "kernels.h"
#include "solver.h"
#include "unet.h"
#include "vec.h"

namespace fem {

namespace {

enum FcgFlag { FCG_RUN = 0, FCG_TARGET = 1, FCG_HANDOVER = 2, FCG_BREAKDOWN = 3, FCG_LIMIT = 4, FCG_DONE = 5 };

// Scalars of one solve.  Each field has one writer kernel per iteration
// (a single-workgroup finalize); the vector kernels only read it.
struct FcgState {
    int flag;      // FcgFlag
    int reason;    // hand-over: 1 network output unusable, 2 p.q <= 0, 3 stall; breakdown: where
    int iters;     // completed steps (x updated)
    int restart;   // the next direction is p = z
    int best_it;   // step of the last halving of ||r||
    int pcalls;    // cycles whose output entered a step
    int stall;     // steps without halving that end the network phase
    int max_iter;
    int use_net;
    double target;   // kCertify rtol ||r_0||
    double coef;     // (z . q_prev) / (p_prev . q_prev)
    double pq_prev;
    double alpha;
    double rn;       // recursive ||r|| after the last step
    double best;     // ||r|| at best_it
    double rtrue;    // last true residual norm
};

// Fixed-order totals of NV dot partials (part[b * NV + j]) in one workgroup;
// thread 0 receives them.
template <int NV>
__device__ __forceinline__ void sum_partials(const double *__restrict__ part, int blocks, double (&v)[NV],
                                             double *red) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = 0.0;
    for (int b = threadIdx.x; b < blocks; b += kBlock)
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] += part[(int64_t)b * NV + j];
    block_sum_n<kBlock, NV>(v, red);
}

// (z.r, z.z, z.q_prev) -> checks and the orthogonalisation coefficient
__global__ __launch_bounds__(kBlock) void k_fcg_coef(const double *__restrict__ part, int blocks, FcgState *st) {
    __shared__ double red[3 * kBlock / kWave];
    if (st->flag != FCG_RUN) return;
    double v[3];
    sum_partials<3>(part, blocks, v, red);
    if (threadIdx.x != 0) return;
    const double zr = v[0], zz = v[1], zq = v[2];
    const bool restart = st->restart != 0;
    if (st->use_net) {
        st->pcalls += 1;
        // a non-finite or zero output cannot give a direction (z.q_prev
        // enters only after a first step)
        if (!(isfinite(zz) && isfinite(zr) && (restart || isfinite(zq)) && zz > 0.0)) {
            st->flag = FCG_HANDOVER;
            st->reason = 1;
            return;
        }
    } else if (!(isfinite(zr) && zr > 0.0)) {
        st->flag = FCG_BREAKDOWN;
        st->reason = 1;
        return;
    }
    st->coef = restart ? 0.0 : zq / st->pq_prev;
}

// p = z (restart) or p = z - coef p
__global__ __launch_bounds__(kBlock) void k_fcg_dir(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                                                    const FcgState *st) {
    if (st->flag != FCG_RUN) return;
    const bool restart = st->restart != 0;
    const double c = st->coef;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = restart ? z[i] : z[i] - c * p[i];
}

// (p.q, p.r) -> alpha
__global__ __launch_bounds__(kBlock) void k_fcg_alpha(const double *__restrict__ part, int blocks, FcgState *st) {
    __shared__ double red[2 * kBlock / kWave];
    if (st->flag != FCG_RUN) return;
    double v[2];
    sum_partials<2>(part, blocks, v, red);
    if (threadIdx.x != 0) return;
    const double pq = v[0], pr = v[1];
    if (!(isfinite(pq) && pq > 0.0 && isfinite(pr))) {
        st->flag = st->use_net ? FCG_HANDOVER : FCG_BREAKDOWN;
        st->reason = 2;
        return;
    }
    st->alpha = pr / pq;
    st->pq_prev = pq;
    st->restart = 0;
}

// x += alpha p, r -= alpha q; per-block partial of r.r
__global__ __launch_bounds__(kBlock) void k_fcg_step(int64_t n, const double *__restrict__ p,
                                                     const double *__restrict__ q, double *__restrict__ x,
                                                     double *__restrict__ r, double *__restrict__ part,
                                                     const FcgState *st) {
    __shared__ double red[kBlock / kWave];
    if (st->flag != FCG_RUN) return;
    const double alpha = st->alpha;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s += ri * ri;
    }
    s = block_sum<kBlock>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ||r|| after the step: convergence, best iterate, stall and the step limit
__global__ __launch_bounds__(kBlock) void k_fcg_check(const double *__restrict__ part, int blocks, FcgState *st) {
    __shared__ double red[kBlock / kWave];
    if (st->flag != FCG_RUN) return;
    double v[1];
    sum_partials<1>(part, blocks, v, red);
    if (threadIdx.x != 0) return;
    const double rn = sqrt(v[0]);
    const int it = st->iters + 1;
    st->iters = it;
    st->rn = rn;
    if (!isfinite(rn)) {
        st->flag = FCG_BREAKDOWN;
        st->reason = 3;
        return;
    }
    if (rn <= 0.5 * st->best) {
        st->best = rn;
        st->best_it = it;
    }
    if (rn <= st->target) {
        st->flag = FCG_TARGET;
    } else if (st->use_net && it - st->best_it >= st->stall) {
        st->flag = FCG_HANDOVER;
        st->reason = 3;
    } else if (it >= st->max_iter) {
        st->flag = FCG_LIMIT;
    }
}

// True residual norm into the state; on a miss the iteration restarts from it
__global__ __launch_bounds__(kBlock) void k_fcg_true(const double *__restrict__ part, int blocks, FcgState *st,
                                                     int judge) {
    __shared__ double red[kBlock / kWave];
    double v[1];
    sum_partials<1>(part, blocks, v, red);
    if (threadIdx.x != 0) return;
    const double rt = sqrt(v[0]);
    st->rtrue = rt;
    if (!judge) return;
    st->rn = rt;
    if (rt <= st->target) {
        st->flag = FCG_DONE;
    } else {
        st->flag = FCG_RUN;
        st->restart = 1;
    }
}

__global__ void k_jacobi(int64_t n, const double *__restrict__ dinv, const double *__restrict__ r,
                         double *__restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        z[i] = dinv[i] * r[i];
}

// s = (n . rz) / (n . A n), 0 when the network output is zero or the ratio is not finite
__global__ __launch_bounds__(kBlock) void k_coarse_scale(const double *__restrict__ part, int blocks,
                                                         double *__restrict__ sc) {
    __shared__ double red[2 * kBlock / kWave];
    double v[2];
    sum_partials<2>(part, blocks, v, red);
    if (threadIdx.x != 0) return;
    const double s = v[0] / v[1];
    sc[0] = (v[1] > 0.0 && isfinite(s)) ? s : 0.0;
}

// The coarse correction z_c = z + s nz followed by the first post-smoothing
// step zn = z_c + omega D^-1 (r - A z_c) without an element pass: the
// residual of z_c is r - A z - s A nz = rz - s An, both already formed
// (0 on Dirichlet nodes, where D^-1 is 0 as well).
__global__ void k_coarse_step(int64_t n, const double *__restrict__ sc, const double *__restrict__ nz,
                              const double *__restrict__ rz, const double *__restrict__ An,
                              const double *__restrict__ dinv, double omega, const double *__restrict__ z,
                              double *__restrict__ zn) {
    const double c = sc[0];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        zn[i] = (z[i] + c * nz[i]) + omega * dinv[i] * (rz[i] - c * An[i]);
}

// out = (b ? b : 0) + sign * A x, 0 on Dirichlet nodes
struct OpLin {
    static constexpr bool kLocal = false;
    const double *x, *b;
    double *out;
    const uint8_t *mask;
    double sign;
    __device__ __forceinline__ bool begin() const { return true; }
    __device__ __forceinline__ double gather(int g, int) const { return x[g]; }
    struct Pre {
        double bv;
        bool zero;
    };
    __device__ __forceinline__ Pre fixup_load(int, int g) const { return {b ? b[g] : 0.0, mask[g] != 0}; }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &pr, double acc) const {
        out[g] = pr.zero ? 0.0 : pr.bv + sign * acc;
    }
    __device__ __forceinline__ void finish(int g, double acc) const { fixup_store(0, g, fixup_load(0, g), acc); }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

// One damped-Jacobi step zn = z + omega D^-1 (r - A z) in one element pass
// (D^-1 is 0 on Dirichlet nodes, so z keeps its zeros there).  zn must not
// alias z: other workgroups still gather z.
struct OpJacobiStep {
    static constexpr bool kLocal = false;
    const double *z, *r, *dinv;
    double *zn;
    double omega;
    __device__ __forceinline__ bool begin() const { return true; }
    __device__ __forceinline__ double gather(int g, int) const { return z[g]; }
    struct Pre {
        double rv, zv, dv;
    };
    __device__ __forceinline__ Pre fixup_load(int, int g) const { return {r[g], z[g], dinv[g]}; }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &pr, double acc) const {
        zn[g] = pr.zv + omega * pr.dv * (pr.rv - acc);
    }
    __device__ __forceinline__ void finish(int g, double acc) const { fixup_store(0, g, fixup_load(0, g), acc); }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

// One element pass (+ fix-up) of op over the packed operator: FP64 values, or
// the FP32 heads of the hi/lo pair (heads).
template <int NB, class Op>
int pass_nb(const DevPlan &P, const void *A, bool heads, const Op &op, double *scratch, hipStream_t s) {
    const size_t lds = chunk_lds_bytes<NB, double>(P.E);
    if (lds > device_lds_limit())
        return set_error(FEM_EINVAL, "the chunk's LDS exceeds the workgroup limit; use smaller chunk_elems");
    const ChunkGrid cg = chunk_grid(P.n_chunks, lds);
    int rc = dispatch_ept(P.E, [&](auto ept) -> int {
        constexpr int EPT = decltype(ept)::value;
        if (heads) {
            LdPk<NB, MAT_F32> ld{A, P.n_elems};
            k_chunk_main<NB, EPT, kBlock, double, decltype(ld), Op, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, scratch, cg.xcd);
        } else {
            LdPk<NB, MAT_F64> ld{A, P.n_elems};
            k_chunk_main<NB, EPT, kBlock, double, decltype(ld), Op, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, scratch, cg.xcd);
        }
        return 0;
    });
    if (rc) return rc;
    FEM_HIP_CHECK(hipGetLastError());
    if (P.n_shared > 0) {
        k_chunk_fixup<kFixBlock, double, Op><<<fixup_grid(P.n_shared), kFixBlock, 0, s>>>(P, op, scratch, 0);
        FEM_HIP_CHECK(hipGetLastError());
    }
    return 0;
}

template <class Op>
int pass(const DevPlan &P, const void *A, bool heads, const Op &op, double *scratch, hipStream_t s) {
    if (P.nb == 4) return pass_nb<4>(P, A, heads, op, scratch, s);
    return pass_nb<3>(P, A, heads, op, scratch, s);
}

// Workspace of one solve (one device arena).
struct FcgWork {
    void *arena = nullptr;
    double *A = nullptr;   // packed operator, FP64
    void *A32 = nullptr;   // packed operator as FP32 hi/lo pair (cycle on FP32 heads)
    double *d = nullptr, *dinv = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *t = nullptr, *rz = nullptr, *nz = nullptr, *An = nullptr;  // two-level cycle
    double *xb = nullptr;  // x0, for a hand-over
    double *scratch = nullptr, *part = nullptr, *sc = nullptr;
    const double **ptrs = nullptr;  // device pointer tables of k_dots
    FcgState *st = nullptr;
    int *bad = nullptr;
    ~FcgWork() {
        if (arena) (void)hipFree(arena);
    }
};

struct CycleOpts {
    fem_unet *net;
    int grid_n;
    double cval;
    int smooth;
    double omega;
    bool heads;
};

// Allocates the workspace and forms the packed operator and D^-1.
int setup(const DevPlan &P, int dtype, const void *K, const void *M, double nu, bool heads, FcgWork &w,
          hipStream_t s) {
    const int64_t n = P.n_nodes;
    const int64_t npk = (int64_t)packed_count(P.nb) * P.n_elems;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return o;
    };
    const size_t oA = take(npk * 8), oA32 = take(heads ? npk * 8 : 0), od = take(n * 8), odi = take(n * 8),
                 or_ = take(n * 8), oz = take(n * 8), op = take(n * 8), oq = take(n * 8), ot = take(n * 8),
                 orz = take(n * 8), onz = take(n * 8), oAn = take(n * 8), oxb = take(n * 8),
                 osc = take(std::max<int64_t>(P.n_partials, 1) * 8), opart = take((size_t)kDotBlocks * 4 * 8),
                 osc2 = take(8), optr = take(16 * sizeof(void *)), ost = take(sizeof(FcgState)),
                 obad = take(sizeof(int));
    if (hipMalloc(&w.arena, off) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FEM_ENOMEM, "device allocation of the FCG workspace failed");
    }
    char *base = static_cast<char *>(w.arena);
    auto at = [&](size_t o) { return reinterpret_cast<double *>(base + o); };
    w.A = at(oA);
    w.A32 = heads ? static_cast<void *>(base + oA32) : nullptr;
    w.d = at(od);
    w.dinv = at(odi);
    w.r = at(or_);
    w.z = at(oz);
    w.p = at(op);
    w.q = at(oq);
    w.t = at(ot);
    w.rz = at(orz);
    w.nz = at(onz);
    w.An = at(oAn);
    w.xb = at(oxb);
    w.scratch = at(osc);
    w.part = at(opart);
    w.sc = at(osc2);
    w.ptrs = reinterpret_cast<const double **>(base + optr);
    w.st = reinterpret_cast<FcgState *>(base + ost);
    w.bad = reinterpret_cast<int *>(base + obad);

    // pointer tables: [0..2] (z, z, z) x [3..5] (r, z, q); [6..7] (p, p) x [8..9] (q, r);
    // [10..11] (nz, nz) x [12..13] (rz, An); [3] x [3]: r.r
    const double *tab[16] = {w.z, w.z, w.z, w.r, w.z, w.q, w.p, w.p, w.q, w.r, w.nz, w.nz, w.rz, w.An};
    FEM_HIP_CHECK(hipMemcpyAsync(w.ptrs, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    FEM_HIP_CHECK(hipMemsetAsync(w.bad, 0, sizeof(int), s));
    // q and p hold the previous direction's products; the first iteration's
    // z.q_prev must read defined values (the memory is recycled)
    FEM_HIP_CHECK(hipMemsetAsync(w.q, 0, n * 8, s));
    FEM_HIP_CHECK(hipMemsetAsync(w.p, 0, n * 8, s));
    if (int rc = launch_pack(P, dtype, K, M, nu, MAT_F64, w.A, s)) return rc;
    if (heads)
        if (int rc = launch_pack(P, dtype, K, M, nu, MAT_F32X2, w.A32, s)) return rc;
    if (int rc = launch_diag_pk64(P, MAT_F64, w.A, w.d, w.scratch, s)) return rc;
    k_dinv_fcg<<<grid_for(n), kBlock, 0, s>>>(n, w.d, P.mask, w.dinv, w.bad);
    FEM_HIP_CHECK(hipGetLastError());
    int bad = 0;
    FEM_HIP_CHECK(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    if (bad) return set_error(FEM_EBREAKDOWN, "the operator has a non-positive diagonal entry");
    return 0;
}

// z = B(r): the two-level cycle (net, smooth > 0), N(r) (net, smooth == 0) or
// D^-1 r.  Uses w.t, w.rz, w.nz, w.An, w.part, w.sc; z must not be w.t.
int precondition(const DevPlan &P, const FcgWork &w, const CycleOpts &c, const double *r, double *z, hipStream_t s) {
    const int64_t n = P.n_nodes;
    const int gv = grid_for(n);
    if (!c.net) {
        k_jacobi<<<gv, kBlock, 0, s>>>(n, w.dinv, r, z);
        FEM_HIP_CHECK(hipGetLastError());
        return 0;
    }
    if (c.smooth == 0) return unet_grid_precondition(c.net, c.grid_n, r, c.cval, P.mask, z, s);
    const void *A = c.heads ? w.A32 : static_cast<const void *>(w.A);
    // 2 smooth - 1 fused steps alternate between t and z, starting in t so
    // that the last one ends in z
    double *cur = w.t, *oth = z;
    k_smooth<<<gv, kBlock, 0, s>>>(n, c.omega, w.dinv, r, cur, 1);
    FEM_HIP_CHECK(hipGetLastError());
    for (int k = 1; k < c.smooth; ++k) {
        if (int rc = pass(P, A, c.heads, OpJacobiStep{cur, r, w.dinv, oth, c.omega}, w.scratch, s)) return rc;
        std::swap(cur, oth);
    }
    // coarse correction by the network on rz = r - A z
    if (int rc = pass(P, A, c.heads, OpLin{cur, r, w.rz, P.mask, -1.0}, w.scratch, s)) return rc;
    if (int rc = unet_grid_precondition(c.net, c.grid_n, w.rz, c.cval, P.mask, w.nz, s)) return rc;
    if (int rc = pass(P, A, c.heads, OpLin{w.nz, nullptr, w.An, P.mask, 1.0}, w.scratch, s)) return rc;
    k_dots<2><<<gv, kBlock, 0, s>>>(n, w.ptrs + 10, w.ptrs + 12, w.part);
    k_coarse_scale<<<1, kBlock, 0, s>>>(w.part, gv, w.sc);
    k_coarse_step<<<gv, kBlock, 0, s>>>(n, w.sc, w.nz, w.rz, w.An, w.dinv, c.omega, cur, oth);
    FEM_HIP_CHECK(hipGetLastError());
    std::swap(cur, oth);
    for (int k = 1; k < c.smooth; ++k) {
        if (int rc = pass(P, A, c.heads, OpJacobiStep{cur, r, w.dinv, oth, c.omega}, w.scratch, s)) return rc;
        std::swap(cur, oth);
    }
    if (cur != z) return set_error(FEM_EINVAL, "internal error: the cycle ended outside z");
    return 0;
}

// r = b - A x (masked) and its norm into the state (st->rtrue; judge: the
// convergence decision too)
int true_residual(const DevPlan &P, const FcgWork &w, const double *b, const double *x, int judge, hipStream_t s) {
    const int64_t n = P.n_nodes;
    const int gv = grid_for(n);
    if (int rc = launch_apply_pk64(P, MAT_F64, w.A, x, b, w.r, -1.0, 1, w.scratch, s)) return rc;
    k_dots<1><<<gv, kBlock, 0, s>>>(n, w.ptrs + 3, w.ptrs + 3, w.part);
    k_fcg_true<<<1, kBlock, 0, s>>>(w.part, gv, w.st, judge);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

// One FCG iteration (enqueued on s; captured into the solve's graph).
int iteration(const DevPlan &P, const FcgWork &w, const CycleOpts &c, double *x, hipStream_t s) {
    const int64_t n = P.n_nodes;
    const int gv = grid_for(n);
    if (int rc = precondition(P, w, c, w.r, w.z, s)) return rc;
    k_dots<3><<<gv, kBlock, 0, s>>>(n, w.ptrs, w.ptrs + 3, w.part);  // z.r, z.z, z.q_prev
    k_fcg_coef<<<1, kBlock, 0, s>>>(w.part, gv, w.st);
    k_fcg_dir<<<gv, kBlock, 0, s>>>(n, w.z, w.p, w.st);
    FEM_HIP_CHECK(hipGetLastError());
    if (int rc = launch_apply_pk64(P, MAT_F64, w.A, w.p, nullptr, w.q, 1.0, 1, w.scratch, s)) return rc;
    k_dots<2><<<gv, kBlock, 0, s>>>(n, w.ptrs + 6, w.ptrs + 8, w.part);  // p.q, p.r
    k_fcg_alpha<<<1, kBlock, 0, s>>>(w.part, gv, w.st);
    k_fcg_step<<<gv, kBlock, 0, s>>>(n, w.p, w.q, x, w.r, w.part, w.st);
    k_fcg_check<<<1, kBlock, 0, s>>>(w.part, gv, w.st);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

// The iteration captured into a HIP graph on an internal stream of default
// priority; replayed on the solve's stream.
struct IterGraph {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    ~IterGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
    int build(const DevPlan &P, const FcgWork &w, const CycleOpts &c, double *x) {
        FEM_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t g;
        FEM_HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        const int rc = iteration(P, w, c, x, cap);
        const hipError_t e = hipStreamEndCapture(cap, &g);
        if (rc) {
            if (e == hipSuccess) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return set_error(FEM_EHIP, "capture of the FCG iteration failed");
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            exec = nullptr;
            return set_error(FEM_EHIP, "instantiation of the FCG iteration graph failed");
        }
        return 0;
    }
};

int read_state(const FcgWork &w, FcgState &h, hipStream_t s) {
    FEM_HIP_CHECK(hipMemcpyAsync(&h, w.st, sizeof(FcgState), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    return 0;
}

}  // namespace

int fcg_precondition(const DevPlan &P, int dtype, const void *K, const void *M, double nu, fem_unet *net, int grid_n,
                     double cval, int smooth, double omega, int cycle_heads, const double *r, double *z,
                     hipStream_t s) {
    FcgWork w;
    const CycleOpts c{net, grid_n, cval, smooth, omega, net != nullptr && cycle_heads != 0};
    if (int rc = setup(P, dtype, K, M, nu, c.heads, w, s)) return rc;
    if (int rc = precondition(P, w, c, r, z, s)) return rc;
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    return 0;
}

int solve_fcg(const DevPlan &P, int dtype, const void *K, const void *M, double nu, const double *b, double *x,
              double rtol, int max_iter, fem_unet *net, int grid_n, double cval, int smooth, double omega,
              int stall_iters, int max_replace, int graph, int check_every, int cycle_heads, FcgResult &res,
              hipStream_t s) {
    std::memset(&res, 0, sizeof(res));
    res.fell_back = -1;
    const int64_t n = P.n_nodes;
    FcgWork w;
    const CycleOpts c{net, grid_n, cval, smooth, omega, net != nullptr && cycle_heads != 0};
    if (int rc = setup(P, dtype, K, M, nu, c.heads, w, s)) return rc;

    FcgState h{};
    if (int rc = true_residual(P, w, b, x, 0, s)) return rc;
    if (int rc = read_state(w, h, s)) return rc;
    const double r0 = h.rtrue;
    res.r0 = r0;
    res.rnorm = r0;
    if (!std::isfinite(r0)) return set_error(FEM_EBREAKDOWN, "non-finite initial residual");
    if (r0 == 0.0) {
        res.relres = 0.0;
        res.status = FEM_OK;
        return FEM_OK;
    }
    h = FcgState{};
    h.flag = FCG_RUN;
    h.restart = 1;
    h.stall = stall_iters;
    h.max_iter = max_iter;
    h.use_net = net != nullptr;
    h.target = kCertify * rtol * r0;
    h.pq_prev = 1.0;
    h.rn = r0;
    h.best = r0;
    h.rtrue = r0;
    FEM_HIP_CHECK(hipMemcpyAsync(w.st, &h, sizeof(h), hipMemcpyHostToDevice, s));
    if (net) FEM_HIP_CHECK(hipMemcpyAsync(w.xb, x, n * 8, hipMemcpyDeviceToDevice, s));

    IterGraph ig;
    if (graph)
        if (int rc = ig.build(P, w, c, x)) return rc;
    auto finish = [&](int status) {
        res.iters = h.iters;
        res.precond_calls = h.pcalls;
        res.relres = h.rtrue / r0;
        res.rnorm = h.rtrue;
        res.status = status;
        return status;
    };
    // Batches of up to check_every iterations between state reads.  Once the
    // device has raised its flag the queued iterations' FCG kernels return at
    // once but their cycles still run, so near the target the batch is cut to
    // the iterations that the last batch's rate of decrease of ||r|| predicts
    // (at least 2).  The iterates do not depend on the batch sizes: the device
    // stops itself.
    int launched = 0, est = check_every, m_prev = 0, it_prev = 0;
    double rn_prev = r0;
    while (true) {
        const int m = std::max(1, std::min(std::min(check_every, est), max_iter - launched));
        for (int j = 0; j < m; ++j) {
            if (graph) {
                FEM_HIP_CHECK(hipGraphLaunch(ig.exec, s));
            } else if (int rc = iteration(P, w, c, x, s)) {
                return rc;
            }
        }
        launched += m;
        m_prev = m;
        if (int rc = read_state(w, h, s)) return rc;
        est = check_every;
        const int done = h.iters - it_prev;
        if (h.flag == FCG_RUN && done == m_prev && h.rn > h.target && h.rn < rn_prev && rn_prev > 0.0) {
            const double rate = std::pow(h.rn / rn_prev, 1.0 / done);
            const double k = std::log(h.target / h.rn) / std::log(rate);
            if (std::isfinite(k)) est = std::max(2, (int)std::min<double>(check_every, std::ceil(k)));
        }
        rn_prev = h.rn;
        it_prev = h.iters;
        if (h.flag == FCG_RUN) {
            if (launched < max_iter) continue;
            h.flag = FCG_LIMIT;
        }
        if (h.flag == FCG_BREAKDOWN) {
            return set_error(FEM_EBREAKDOWN, h.reason == 1   ? "r.z <= 0 in FCG"
                                             : h.reason == 2 ? "p.q <= 0 in FCG"
                                                             : "non-finite residual in FCG");
        }
        if (h.flag == FCG_TARGET) {
            if (int rc = true_residual(P, w, b, x, 1, s)) return rc;
            if (int rc = read_state(w, h, s)) return rc;
            if (h.flag == FCG_DONE) return finish(FEM_OK);
            if (res.replacements >= max_replace || h.iters >= max_iter) break;
            res.replacements += 1;
            launched = h.iters;
            continue;  // the state already says: run, restart from the true residual
        }
        if (h.flag == FCG_HANDOVER) {
            // restart from x0 (see the head of this file)
            FEM_HIP_CHECK(hipMemcpyAsync(x, w.xb, n * 8, hipMemcpyDeviceToDevice, s));
            if (int rc = true_residual(P, w, b, x, 0, s)) return rc;
            if (int rc = read_state(w, h, s)) return rc;
            res.fallback_reason = h.reason;
            res.fell_back = h.iters;
            finish(FEM_OK);
            return kFcgHandover;
        }
        break;  // FCG_LIMIT
    }
    if (int rc = true_residual(P, w, b, x, 0, s)) return rc;
    if (int rc = read_state(w, h, s)) return rc;
    const int status = h.rtrue <= h.target ? FEM_OK : FEM_ENOCONV;
    if (status == FEM_ENOCONV) set_error(FEM_ENOCONV, "FCG reached the iteration limit");
    return finish(status);
}

}  // namespace fem
