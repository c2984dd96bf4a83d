// iterate.hip -- the paper's own iterations driven by the element residual.
//
// Section 2 builds every solver on the residual r = b - A x of eq. (4)
// (Algorithm 1) and eigenvalue bounds lam1 <= lambda(A) <= lam2:
//   Richardson           x <- x + omega r, omega = 2 / (lam1 + lam2)
//   2-level Chebyshev    x <- x + r / alpha_{k mod N}, alpha_j the roots of the
//                        shifted and scaled Chebyshev polynomial of degree N,
//                        alpha_j = d + c cos(pi (j + 1/2) / N),
//                        d = (lam1 + lam2) / 2, c = (lam2 - lam1) / 2
//                        (eq. (Czebyshev2lev), in the order of the listing)
//   3-level Chebyshev    x^1 = x^0 + r_0 / d, then
//                        x^{k+1} = x^k + C_{k-1}/C_{k+1} (x^k - x^{k-1})
//                                  + (2 / c) C_k / C_{k+1} r_k
//                        with C_{k+1} = 2 sigma C_k - C_{k-1}, C_0 = 1,
//                        C_1 = sigma = d / c (eqs. (recrCk), (Czebyshev3lev))
//   3-level, listing     p = r (first) or r + beta p, x <- x + alpha p with
//                        alpha = 1/d first, then beta = (c alpha / 2)^2,
//                        alpha = 1 / (d - beta / alpha) (the alpha/beta form
//                        of the Section 2 listing)
// The scalars depend only on (lam1, lam2, N, k) and are formed on the host in
// FP64; each iteration is one element residual pass plus one vector update.
// The ratio C_{k+1}/C_k is carried instead of C_k, which overflows after a
// few thousand steps when lam1 << lam2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "kernels.h"
#include "solver.h"
#include "vec.h"

namespace fem {

namespace {

// x += w r
__global__ void k_axpy(int64_t n, double w, const double *__restrict__ r, double *__restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        x[i] += w * r[i];
}

// three-term step: x_new = x + a (x - x_prev) + w r; x_prev = x; x = x_new
__global__ void k_three_term(int64_t n, double a, double w, const double *__restrict__ r, double *__restrict__ x,
                             double *__restrict__ xp) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double xi = x[i];
        x[i] = xi + a * (xi - xp[i]) + w * r[i];
        xp[i] = xi;
    }
}

// p = r + beta p (beta ignored when first), x += alpha p
__global__ void k_dir_step(int64_t n, double beta, double alpha, int first, const double *__restrict__ r,
                           double *__restrict__ p, double *__restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double pi = first ? r[i] : r[i] + beta * p[i];
        p[i] = pi;
        x[i] += alpha * pi;
    }
}

struct IterWork {
    void *arena = nullptr;
    ~IterWork() {
        if (arena) (void)hipFree(arena);
    }
};

}  // namespace

int run_iteration(const DevPlan &P, int dtype, const void *K, const void *M, double nu, const double *b, double *x,
                  int method, double lam1, double lam2, int cycle, int iters, IterResult &res, hipStream_t s) {
    std::memset(&res, 0, sizeof(res));
    const int64_t n = P.n_nodes;
    const int64_t npk = (int64_t)packed_count(P.nb) * P.n_elems;
    IterWork w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return o;
    };
    const size_t oA = take(npk * 8), or_ = take(n * 8), ov = take(n * 8),
                 osc = take(std::max<int64_t>(P.n_partials, 1) * 8), opart = take((size_t)kDotBlocks * 8),
                 osum = take(64), optr = take(2 * sizeof(void *));
    if (hipMalloc(&w.arena, off) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FEM_ENOMEM, "device allocation of the iteration workspace failed");
    }
    char *base = static_cast<char *>(w.arena);
    double *A = reinterpret_cast<double *>(base + oA), *r = reinterpret_cast<double *>(base + or_),
           *v = reinterpret_cast<double *>(base + ov), *scratch = reinterpret_cast<double *>(base + osc),
           *part = reinterpret_cast<double *>(base + opart), *sums = reinterpret_cast<double *>(base + osum);
    const double **ptrs = reinterpret_cast<const double **>(base + optr);
    const double *tab[2] = {r, r};
    FEM_HIP_CHECK(hipMemcpyAsync(ptrs, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    if (int rc = launch_pack(P, dtype, K, M, nu, MAT_F64, A, s)) return rc;
    const int gv = grid_for(n);
    auto residual = [&]() { return launch_apply_pk64(P, MAT_F64, A, x, b, r, -1.0, 1, scratch, s); };
    auto norm = [&](double &out) -> int {
        k_dots<1><<<gv, kBlock, 0, s>>>(n, ptrs, ptrs + 1, part);
        k_dots_fin<<<1, 64, 0, s>>>(part, gv, 1, sums);
        FEM_HIP_CHECK(hipGetLastError());
        double h = 0.0;
        FEM_HIP_CHECK(hipMemcpyAsync(&h, sums, sizeof(double), hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        out = std::sqrt(h);
        return 0;
    };
    if (int rc = residual()) return rc;
    if (int rc = norm(res.r0)) return rc;

    const double d = 0.5 * (lam1 + lam2), c = 0.5 * (lam2 - lam1);
    const double pi = 3.14159265358979323846;
    if (method == ITER_RICHARDSON || method == ITER_CHEB2) {
        for (int k = 0; k < iters; ++k) {
            if (k > 0)
                if (int rc = residual()) return rc;
            const double wk =
                method == ITER_RICHARDSON ? 1.0 / d : 1.0 / (d + c * std::cos(pi * ((k % cycle) + 0.5) / cycle));
            k_axpy<<<gv, kBlock, 0, s>>>(n, wk, r, x);
        }
    } else if (method == ITER_CHEB3) {
        const double sigma = d / c;
        double t_prev = 0.0, t = sigma;  // t = C_{k+1} / C_k at step k (C_1 / C_0 = sigma)
        for (int k = 0; k < iters; ++k) {
            if (k > 0)
                if (int rc = residual()) return rc;
            if (k == 0) {
                // x_prev = x0, x1 = x0 + r0 / d
                FEM_HIP_CHECK(hipMemcpyAsync(v, x, n * 8, hipMemcpyDeviceToDevice, s));
                k_axpy<<<gv, kBlock, 0, s>>>(n, 1.0 / d, r, x);
                continue;
            }
            t_prev = t;
            t = 2.0 * sigma - 1.0 / t_prev;  // C_{k+1}/C_k from C_k/C_{k-1}
            // C_{k-1}/C_{k+1} = 1 / (t_prev t), C_k/C_{k+1} = 1 / t
            k_three_term<<<gv, kBlock, 0, s>>>(n, 1.0 / (t_prev * t), 2.0 / (c * t), r, x, v);
        }
    } else {
        double alpha = 1.0 / d;
        for (int k = 0; k < iters; ++k) {
            double beta = 0.0;
            if (k > 0) {
                beta = 0.25 * (c * alpha) * (c * alpha);
                alpha = 1.0 / (d - beta / alpha);
            }
            k_dir_step<<<gv, kBlock, 0, s>>>(n, beta, alpha, k == 0, r, v, x);
            if (int rc = residual()) return rc;
        }
    }
    FEM_HIP_CHECK(hipGetLastError());
    if (method != ITER_CHEB3_LISTING || iters == 0)
        if (int rc = residual()) return rc;
    double rn = 0.0;
    if (int rc = norm(rn)) return rc;
    res.iters = iters;
    res.relres = res.r0 > 0.0 ? rn / res.r0 : 0.0;
    return 0;
}

}  // namespace fem
