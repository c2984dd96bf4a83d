// fcg.hip -- flexible conjugate gradients (FCG(1)) on the element residual,
// with a U-Net or Jacobi preconditioner.
//
// The operator is the residual of Section 2 (eq. (4), Algorithm 1) through the
// packed difference form in FP64.  FCG(1) keeps one previous direction and
// orthogonalises the new preconditioned residual against it explicitly,
//   p_k = z_k - (z_k . q_{k-1}) / (p_{k-1} . q_{k-1}) p_{k-1},  q_k = A p_k,
// which stays a descent method when the preconditioner z = N(r) is nonlinear
// or changes between iterations (Notay, SIAM J. Sci. Comput. 22 (2000)).
// The true residual judges convergence: when the recursive residual meets the
// tolerance, r = b - A x is recomputed in FP64 and the iteration restarts
// from it if the tolerance is not met.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "solver.h"
#include "unet.h"

namespace fem {

namespace {

constexpr int kDotBlocks = 512;

// partial[b][j] = sum over this block's rows of a_j[i] * b_j[i], j < NV
template <int NV>
__global__ __launch_bounds__(kBlock) void k_dots(int64_t n, const double *const *__restrict__ av,
                                                 const double *const *__restrict__ bv, double *__restrict__ part) {
    __shared__ double red[NV * kBlock / kWave];
    double v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = 0.0;
    const double *a[NV], *b[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        a[j] = av[j];
        b[j] = bv[j];
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] += a[j][i] * b[j][i];
    block_sum_n<kBlock, NV>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) part[(int64_t)blockIdx.x * NV + j] = v[j];
}

// out[j] = sum_b part[b][j] in block order (one thread per j)
__global__ void k_dots_fin(const double *__restrict__ part, int blocks, int nv, double *__restrict__ out) {
    const int j = threadIdx.x;
    if (j >= nv) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += part[(int64_t)b * nv + j];
    out[j] = s;
}

__global__ void k_jacobi(int64_t n, const double *__restrict__ dinv, const double *__restrict__ r,
                         double *__restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        z[i] = dinv[i] * r[i];
}

__global__ void k_dinv_fcg(int64_t n, const double *__restrict__ d, const uint8_t *__restrict__ mask,
                           double *__restrict__ dinv, int *__restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double v = 0.0;
        if (!mask[i]) {
            if (!(d[i] > 0.0)) *bad = 1;
            v = 1.0 / d[i];
        }
        dinv[i] = v;
    }
}

// p = z - beta p
__global__ void k_dir(int64_t n, const double *__restrict__ z, double beta, double *__restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = z[i] - beta * p[i];
}

// x += alpha p, r -= alpha q; partial r.r per block
__global__ __launch_bounds__(kBlock) void k_step(int64_t n, double alpha, const double *__restrict__ p,
                                                 const double *__restrict__ q, double *__restrict__ x,
                                                 double *__restrict__ r, double *__restrict__ part) {
    __shared__ double red[kBlock / kWave];
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

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kDotBlocks)); }

struct FcgWork {
    void *arena = nullptr;
    double *A = nullptr, *d = nullptr, *dinv = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *scratch = nullptr, *part = nullptr, *sums = nullptr;
    const double **ptrs = nullptr;  // device pointer tables of k_dots
    int *bad = nullptr;
    ~FcgWork() {
        if (arena) (void)hipFree(arena);
    }
};

}  // namespace

int solve_fcg(const DevPlan &P, int dtype, const void *K, const void *M, double nu, const double *b, double *x,
              double rtol, int max_iter, fem_unet *net, int grid_n, double cval, int stall_iters, int max_replace,
              FcgResult &res, hipStream_t s) {
    std::memset(&res, 0, sizeof(res));
    res.fell_back = -1;
    const int64_t n = P.n_nodes;
    const int64_t npk = (int64_t)packed_count(P.nb) * P.n_elems;
    FcgWork w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return o;
    };
    const size_t oA = take(npk * 8), od = take(n * 8), odi = take(n * 8), or_ = take(n * 8), oz = take(n * 8),
                 op = take(n * 8), oq = take(n * 8), osc = take(std::max<int64_t>(P.n_partials, 1) * 8),
                 opart = take((size_t)kDotBlocks * 4 * 8), osum = take(8 * 8), optr = take(16 * sizeof(void *)),
                 obad = take(sizeof(int));
    if (hipMalloc(&w.arena, off) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FEM_ENOMEM, "device allocation of the FCG workspace failed");
    }
    char *base = static_cast<char *>(w.arena);
    w.A = reinterpret_cast<double *>(base + oA);
    w.d = reinterpret_cast<double *>(base + od);
    w.dinv = reinterpret_cast<double *>(base + odi);
    w.r = reinterpret_cast<double *>(base + or_);
    w.z = reinterpret_cast<double *>(base + oz);
    w.p = reinterpret_cast<double *>(base + op);
    w.q = reinterpret_cast<double *>(base + oq);
    w.scratch = reinterpret_cast<double *>(base + osc);
    w.part = reinterpret_cast<double *>(base + opart);
    w.sums = reinterpret_cast<double *>(base + osum);
    w.ptrs = reinterpret_cast<const double **>(base + optr);
    w.bad = reinterpret_cast<int *>(base + obad);

    // pointer tables: [0..2] (z, z, z) x (r, z, q); [3..4] (p, p) x (q, r)
    const double *tab[16] = {w.z, w.z, w.z, w.r, w.z, w.q, w.p, w.p, w.q, w.r};
    FEM_HIP_CHECK(hipMemcpyAsync(w.ptrs, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    FEM_HIP_CHECK(hipMemsetAsync(w.bad, 0, sizeof(int), s));
    if (int rc = launch_pack(P, dtype, K, M, nu, MAT_F64, w.A, s)) return rc;
    if (int rc = launch_diag_pk64(P, MAT_F64, w.A, w.d, w.scratch, s)) return rc;
    const int gv = grid_for(n);
    k_dinv_fcg<<<gv, kBlock, 0, s>>>(n, w.d, P.mask, w.dinv, w.bad);
    FEM_HIP_CHECK(hipGetLastError());

    double h[8];
    auto fetch = [&](int cnt) -> int {
        FEM_HIP_CHECK(hipMemcpyAsync(h, w.sums, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        return 0;
    };
    // r = b - A x (masked) and ||r||
    auto true_residual = [&](double &rn) -> int {
        if (int rc = launch_apply_pk64(P, MAT_F64, w.A, x, b, w.r, -1.0, 1, w.scratch, s)) return rc;
        k_dots<1><<<gv, kBlock, 0, s>>>(n, w.ptrs + 3, w.ptrs + 3, w.part);
        k_dots_fin<<<1, 64, 0, s>>>(w.part, gv, 1, w.sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(1)) return rc;
        rn = std::sqrt(h[0]);
        return 0;
    };
    int bad = 0;
    FEM_HIP_CHECK(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    double rn = 0.0;
    if (int rc = true_residual(rn)) return rc;
    if (bad) return set_error(FEM_EBREAKDOWN, "the operator has a non-positive diagonal entry");
    res.r0 = rn;
    res.rnorm = rn;
    if (!std::isfinite(rn)) return set_error(FEM_EBREAKDOWN, "non-finite initial residual");
    if (rn == 0.0) {
        res.relres = 0.0;
        res.status = FEM_OK;
        return FEM_OK;
    }
    const double target = rtol * rn;
    bool use_net = net != nullptr;
    bool restart = true;
    double pq_prev = 1.0, best = rn;
    int best_it = 0;
    for (int it = 0; it < max_iter; ++it) {
        // z = N(r) or D^-1 r; then (z.r, z.z, z.q_prev)
        bool net_ok = use_net;
        if (use_net) {
            if (int rc = unet_grid_precondition(net, grid_n, w.r, cval, P.mask, w.z, s)) return rc;
            res.precond_calls += 1;
        } else {
            k_jacobi<<<gv, kBlock, 0, s>>>(n, w.dinv, w.r, w.z);
        }
        k_dots<3><<<gv, kBlock, 0, s>>>(n, w.ptrs, w.ptrs + 3, w.part);
        k_dots_fin<<<1, 64, 0, s>>>(w.part, gv, 3, w.sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(3)) return rc;
        double zr = h[0], zz = h[1], zq = h[2];
        // a network output that is non-finite or zero cannot give a direction
        if (use_net && !(std::isfinite(zz) && std::isfinite(zr) && std::isfinite(zq) && zz > 0.0)) {
            res.fallback_reason = 1;
            net_ok = false;
        }
        if (use_net && !net_ok) {
            res.fell_back = it;
            res.iters = it;
            res.rnorm = rn;
            return kFcgHandover;
        }
        if (!use_net && !(std::isfinite(zr) && zr > 0.0)) return set_error(FEM_EBREAKDOWN, "r.z <= 0 in FCG");
        if (restart) {
            FEM_HIP_CHECK(hipMemcpyAsync(w.p, w.z, n * 8, hipMemcpyDeviceToDevice, s));
        } else {
            k_dir<<<gv, kBlock, 0, s>>>(n, w.z, zq / pq_prev, w.p);
        }
        restart = false;
        if (int rc = launch_apply_pk64(P, MAT_F64, w.A, w.p, nullptr, w.q, 1.0, 1, w.scratch, s)) return rc;
        k_dots<2><<<gv, kBlock, 0, s>>>(n, w.ptrs + 6, w.ptrs + 8, w.part);
        k_dots_fin<<<1, 64, 0, s>>>(w.part, gv, 2, w.sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(2)) return rc;
        const double pq = h[0], pr = h[1];
        if (!(std::isfinite(pq) && pq > 0.0 && std::isfinite(pr))) {
            if (use_net) {
                res.fallback_reason = 2;
                res.fell_back = it;
                res.iters = it;
                res.rnorm = rn;
                return kFcgHandover;
            }
            return set_error(FEM_EBREAKDOWN, "p.q <= 0 in FCG");
        }
        const double alpha = pr / pq;
        pq_prev = pq;
        k_step<<<gv, kBlock, 0, s>>>(n, alpha, w.p, w.q, x, w.r, w.part);
        k_dots_fin<<<1, 64, 0, s>>>(w.part, gv, 1, w.sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(1)) return rc;
        rn = std::sqrt(h[0]);
        res.iters = it + 1;
        res.rnorm = rn;
        if (!std::isfinite(rn)) return set_error(FEM_EBREAKDOWN, "non-finite residual in FCG");
        if (rn <= target) {
            double rt = 0.0;
            if (int rc = true_residual(rt)) return rc;
            rn = rt;
            res.rnorm = rt;
            if (rt <= target) {
                res.relres = rt / res.r0;
                res.status = FEM_OK;
                return FEM_OK;
            }
            if (res.replacements >= max_replace) break;
            res.replacements += 1;
            restart = true;
        }
        if (rn <= 0.5 * best) {
            best = rn;
            best_it = it + 1;
        } else if (use_net && it + 1 - best_it >= stall_iters) {
            res.fallback_reason = 3;
            res.fell_back = it + 1;
            return kFcgHandover;
        }
    }
    double rt = 0.0;
    if (int rc = true_residual(rt)) return rc;
    res.rnorm = rt;
    res.relres = rt / res.r0;
    res.status = rt <= target ? FEM_OK : FEM_ENOCONV;
    if (res.status == FEM_ENOCONV) set_error(FEM_ENOCONV, "FCG reached the iteration limit");
    return res.status;
}

}  // namespace fem
