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
// FP64.  Each iteration is one element pass (OpStep): it forms the residual
// of the current iterate node by node and applies the method's update to
// that node at once, writing the new iterate to another buffer, so the
// residual is never stored (the buffers rotate between steps).  The ratio
// C_{k+1}/C_k is carried instead of C_k, which overflows after a few
// thousand steps when lam1 << lam2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "chunk.h"
#include "common.h"
#include "kernels.h"
#include "solver.h"
#include "vec.h"

namespace fem {

namespace {

// One step of an iteration inside the element pass: r = b - A x on the node
// (0 on Dirichlet nodes, as the masked residual), then
//   STEP_AXPY   x_new = x + w r                      (Richardson, 2-level)
//   STEP_THREE  x_new = x + a (x - x_prev) + w r     (3-level Chebyshev)
//   STEP_DIR    p = r (first) or r + beta p, x_new = x + alpha p   (listing)
// x is only read (the gather of every chunk needs it); x_new goes to its own
// buffer.  The expressions are those of the stand-alone update kernels.
enum StepKind { STEP_AXPY = 0, STEP_THREE = 1, STEP_DIR = 2 };
struct OpStep {
    static constexpr bool kLocal = false;
    const double *x, *b, *xp;
    double *xn, *p;
    const uint8_t *mask;
    int kind, first;
    double w, a, beta;
    __device__ __forceinline__ bool begin() const { return true; }
    __device__ __forceinline__ double gather(int g, int) const { return x[g]; }
    struct Pre {
        double bv, xv, xpv, pv;
        bool zero;
    };
    __device__ __forceinline__ Pre fixup_load(int, int g) const {
        Pre pr;
        pr.bv = b[g];
        pr.xv = x[g];
        pr.xpv = kind == STEP_THREE ? xp[g] : 0.0;
        pr.pv = (kind == STEP_DIR && !first) ? p[g] : 0.0;
        pr.zero = mask[g] != 0;
        return pr;
    }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &pr, double acc) const {
        double r = pr.bv + (-1.0) * acc;
        if (pr.zero) r = 0.0;
        if (kind == STEP_AXPY) {
            xn[g] = pr.xv + w * r;
        } else if (kind == STEP_THREE) {
            xn[g] = pr.xv + a * (pr.xv - pr.xpv) + w * r;
        } else {
            const double pi = first ? r : r + beta * pr.pv;
            p[g] = pi;
            xn[g] = pr.xv + a * pi;
        }
    }
    __device__ __forceinline__ void finish(int g, double acc) const { fixup_store(0, g, fixup_load(0, g), acc); }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

// The fused step over the FP64 packed operator A (chunk pass + fix-up).
int launch_step(const DevPlan &P, const double *A, const OpStep &op, double *scratch, hipStream_t s) {
    const size_t lds = chunk_lds_bytes<3, double>(P.E) / 3 * P.nb;
    const ChunkGrid cg = chunk_grid(P.n_chunks, lds);
    int rc = dispatch_ept(P.E, [&](auto ept) -> int {
        constexpr int EPT = decltype(ept)::value;
        if (P.nb == 3) {
            LdPk<3, MAT_F64> ld{A, P.n_elems};
            k_chunk_main<3, EPT, kBlock, double, decltype(ld), OpStep, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, scratch, cg.xcd);
        } else {
            LdPk<4, MAT_F64> ld{A, P.n_elems};
            k_chunk_main<4, EPT, kBlock, double, decltype(ld), OpStep, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, scratch, cg.xcd);
        }
        return 0;
    });
    if (rc) return rc;
    FEM_HIP_CHECK(hipGetLastError());
    if (P.n_shared > 0) {
        k_chunk_fixup<kFixBlock, double, OpStep><<<fixup_grid(P.n_shared), kFixBlock, 0, s>>>(P, op, scratch, 0);
        FEM_HIP_CHECK(hipGetLastError());
    }
    return 0;
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
    const size_t oA = take(npk * 8), or_ = take(n * 8), ov = take(n * 8), ou = take(n * 8),
                 osc = take(std::max<int64_t>(P.n_partials, 1) * 8), opart = take((size_t)kDotBlocks * 8),
                 osum = take(64), optr = take(2 * sizeof(void *));
    if (hipMalloc(&w.arena, off) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FEM_ENOMEM, "device allocation of the iteration workspace failed");
    }
    char *base = static_cast<char *>(w.arena);
    double *A = reinterpret_cast<double *>(base + oA), *r = reinterpret_cast<double *>(base + or_),
           *v = reinterpret_cast<double *>(base + ov), *u = reinterpret_cast<double *>(base + ou),
           *scratch = reinterpret_cast<double *>(base + osc),
           *part = reinterpret_cast<double *>(base + opart), *sums = reinterpret_cast<double *>(base + osum);
    const double **ptrs = reinterpret_cast<const double **>(base + optr);
    const double *tab[2] = {r, r};
    FEM_HIP_CHECK(hipMemcpyAsync(ptrs, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    if (int rc = launch_pack(P, dtype, K, M, nu, MAT_F64, A, s)) return rc;
    const int gv = grid_for(n);
    auto residual = [&]() { return launch_apply_pk64(P, MAT_F64, A, x, b, r, -1.0, 1, scratch, s); };
    auto norm = [&](double &out) -> int {
        k_dots<1><<<gv, kBlock, 0, s>>>(n, ptrs, ptrs + 1, part);
        k_dots_fin<<<1, kBlock, 0, s>>>(part, gv, 1, sums);
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
    // iterate buffers: the caller's x and two workspace vectors rotate
    double *xc = x, *xo = v, *xt = u;  // current, next, third (previous iterate of the 3-level method)
    OpStep op{nullptr, b, nullptr, nullptr, nullptr, P.mask, STEP_AXPY, 0, 0.0, 0.0, 0.0};
    auto step = [&](int kind, const double *xprev, double w_, double a_, double beta_, int first) -> int {
        op.x = xc;
        op.xp = xprev;
        op.xn = xo;
        op.p = u;
        op.kind = kind;
        op.first = first;
        op.w = w_;
        op.a = a_;
        op.beta = beta_;
        return launch_step(P, A, op, scratch, s);
    };
    if (method == ITER_RICHARDSON || method == ITER_CHEB2) {
        for (int k = 0; k < iters; ++k) {
            const double wk =
                method == ITER_RICHARDSON ? 1.0 / d : 1.0 / (d + c * std::cos(pi * ((k % cycle) + 0.5) / cycle));
            if (int rc = step(STEP_AXPY, nullptr, wk, 0.0, 0.0, 0)) return rc;
            std::swap(xc, xo);
        }
    } else if (method == ITER_CHEB3) {
        const double sigma = d / c;
        double t_prev = 0.0, t = sigma;  // t = C_{k+1} / C_k at step k (C_1 / C_0 = sigma)
        const double *xprev = nullptr;
        for (int k = 0; k < iters; ++k) {
            if (k == 0) {
                // x1 = x0 + r0 / d; x0 stays in its buffer as the previous iterate
                if (int rc = step(STEP_AXPY, nullptr, 1.0 / d, 0.0, 0.0, 0)) return rc;
                xprev = xc;
                xc = xo;
                xo = xt;
                continue;
            }
            t_prev = t;
            t = 2.0 * sigma - 1.0 / t_prev;  // C_{k+1}/C_k from C_k/C_{k-1}
            // C_{k-1}/C_{k+1} = 1 / (t_prev t), C_k/C_{k+1} = 1 / t
            if (int rc = step(STEP_THREE, xprev, 2.0 / (c * t), 1.0 / (t_prev * t), 0.0, 0)) return rc;
            double *old_prev = const_cast<double *>(xprev);
            xprev = xc;
            xc = xo;
            xo = old_prev;
        }
    } else {
        // direction form: p in u, the iterate alternates between x and v
        xo = v;
        double alpha = 1.0 / d;
        for (int k = 0; k < iters; ++k) {
            double beta = 0.0;
            if (k > 0) {
                beta = 0.25 * (c * alpha) * (c * alpha);
                alpha = 1.0 / (d - beta / alpha);
            }
            if (int rc = step(STEP_DIR, nullptr, 0.0, alpha, beta, k == 0)) return rc;
            std::swap(xc, xo);
        }
    }
    if (xc != x) FEM_HIP_CHECK(hipMemcpyAsync(x, xc, n * 8, hipMemcpyDeviceToDevice, s));
    FEM_HIP_CHECK(hipGetLastError());
    if (int rc = residual()) return rc;
    double rn = 0.0;
    if (int rc = norm(rn)) return rc;
    res.iters = iters;
    res.relres = res.r0 > 0.0 ? rn / res.r0 : 0.0;
    return 0;
}

}  // namespace fem
