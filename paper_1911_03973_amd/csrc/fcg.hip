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
//
// With a network and smooth > 0 the preconditioner is a two-level cycle in
// which the network plays the coarse correction: `smooth` damped-Jacobi steps
// z += omega D^-1 (r - A z) from z = 0, the network correction
// z += s N(r - A z) with the energy-optimal s = (n . rz) / (n . A n), and
// `smooth` more Jacobi steps.  The network is trained on smooth solver
// residuals; the smoothing steps remove the rough components it has not seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "solver.h"
#include "unet.h"
#include "vec.h"

namespace fem {

namespace {

__global__ void k_jacobi(int64_t n, const double *__restrict__ dinv, const double *__restrict__ r,
                         double *__restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        z[i] = dinv[i] * r[i];
}

// s = (n . rz) / (n . A n), 0 when the network output is zero or the ratio is not finite
__global__ void k_coarse_scale(const double *__restrict__ part, int blocks, double *__restrict__ sc) {
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < blocks; ++k) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    const double v = a / b;
    sc[0] = (b > 0.0 && isfinite(v)) ? v : 0.0;
}

// z += s nz, rz -= s An
__global__ void k_coarse_update(int64_t n, const double *__restrict__ sc, const double *__restrict__ nz,
                                const double *__restrict__ An, double *__restrict__ z, double *__restrict__ rz) {
    const double c = sc[0];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        z[i] += c * nz[i];
        rz[i] -= c * An[i];
    }
}


// The preconditioner's launches captured once per solve into a HIP graph (on
// an internal stream of default priority) and replayed on the solver's
// stream; the inputs and outputs are the solve's fixed workspace vectors.
struct PrecondGraph {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    const double *r = nullptr;
    double *z = nullptr;
    ~PrecondGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
    int run(fem_unet *net, int grid_n, const double *rr, double cval, const uint8_t *mask, double *zz, hipStream_t s) {
        if (!exec || rr != r || zz != z) {
            if (exec) {
                FEM_HIP_CHECK(hipGraphExecDestroy(exec));
                exec = nullptr;
            }
            if (!cap) FEM_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t g;
            FEM_HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            const int rc = unet_grid_precondition(net, grid_n, rr, cval, mask, zz, cap);
            const hipError_t e = hipStreamEndCapture(cap, &g);
            if (rc) return rc;
            if (e != hipSuccess) return set_error(FEM_EHIP, "capture of the preconditioner failed");
            const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) {
                exec = nullptr;
                return set_error(FEM_EHIP, "instantiation of the preconditioner graph failed");
            }
            r = rr;
            z = zz;
        }
        FEM_HIP_CHECK(hipGraphLaunch(exec, s));
        return 0;
    }
};

struct FcgWork {
    void *arena = nullptr;
    double *A = nullptr, *d = nullptr, *dinv = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *rz = nullptr, *nz = nullptr, *An = nullptr;  // two-level preconditioner vectors
    double *scratch = nullptr, *part = nullptr, *sums = nullptr, *sc = nullptr;
    const double **ptrs = nullptr;  // device pointer tables of k_dots
    int *bad = nullptr;
    ~FcgWork() {
        if (arena) (void)hipFree(arena);
    }
};

}  // namespace

int solve_fcg(const DevPlan &P, int dtype, const void *K, const void *M, double nu, const double *b, double *x,
              double rtol, int max_iter, fem_unet *net, int grid_n, double cval, int smooth, double omega,
              int stall_iters, int max_replace, int graph, FcgResult &res, hipStream_t s) {
    std::memset(&res, 0, sizeof(res));
    PrecondGraph pg;
    auto precondition = [&](const double *rr, double *zz) -> int {
        if (graph) return pg.run(net, grid_n, rr, cval, P.mask, zz, s);
        return unet_grid_precondition(net, grid_n, rr, cval, P.mask, zz, s);
    };
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
                 obad = take(sizeof(int)), orz = take(n * 8), onz = take(n * 8), oAn = take(n * 8), osc2 = take(8);
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
    w.rz = reinterpret_cast<double *>(base + orz);
    w.nz = reinterpret_cast<double *>(base + onz);
    w.An = reinterpret_cast<double *>(base + oAn);
    w.sc = reinterpret_cast<double *>(base + osc2);

    // pointer tables: [0..2] (z, z, z) x (r, z, q); [3..4] (p, p) x (q, r)
    // [10..11] (nz, nz) x (rz, An)
    const double *tab[16] = {w.z, w.z, w.z, w.r, w.z, w.q, w.p, w.p, w.q, w.r, w.nz, w.nz, w.rz, w.An};
    FEM_HIP_CHECK(hipMemcpyAsync(w.ptrs, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    FEM_HIP_CHECK(hipMemsetAsync(w.bad, 0, sizeof(int), s));
    // q and p hold the previous direction's products; the first iteration's
    // z.q_prev must read defined values (the memory is recycled)
    FEM_HIP_CHECK(hipMemsetAsync(w.q, 0, n * 8, s));
    FEM_HIP_CHECK(hipMemsetAsync(w.p, 0, n * 8, s));
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
        k_dots_fin<<<1, kBlock, 0, s>>>(w.part, gv, 1, w.sums);
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
        if (use_net && smooth == 0) {
            if (int rc = precondition(w.r, w.z)) return rc;
            res.precond_calls += 1;
        } else if (use_net) {
            // pre-smoothing: z = omega D^-1 r, then (smooth - 1) steps on rz = r - A z
            k_smooth<<<gv, kBlock, 0, s>>>(n, omega, w.dinv, w.r, w.z, 1);
            for (int k = 1; k < smooth; ++k) {
                if (int rc = launch_apply_pk64(P, MAT_F64, w.A, w.z, w.r, w.rz, -1.0, 1, w.scratch, s)) return rc;
                k_smooth<<<gv, kBlock, 0, s>>>(n, omega, w.dinv, w.rz, w.z, 0);
            }
            if (int rc = launch_apply_pk64(P, MAT_F64, w.A, w.z, w.r, w.rz, -1.0, 1, w.scratch, s)) return rc;
            // coarse correction by the network
            if (int rc = precondition(w.rz, w.nz)) return rc;
            res.precond_calls += 1;
            if (int rc = launch_apply_pk64(P, MAT_F64, w.A, w.nz, nullptr, w.An, 1.0, 1, w.scratch, s)) return rc;
            k_dots<2><<<gv, kBlock, 0, s>>>(n, w.ptrs + 10, w.ptrs + 12, w.part);
            k_coarse_scale<<<1, 64, 0, s>>>(w.part, gv, w.sc);
            k_coarse_update<<<gv, kBlock, 0, s>>>(n, w.sc, w.nz, w.An, w.z, w.rz);
            // post-smoothing
            for (int k = 0; k < smooth; ++k) {
                if (k > 0) {
                    if (int rc = launch_apply_pk64(P, MAT_F64, w.A, w.z, w.r, w.rz, -1.0, 1, w.scratch, s))
                        return rc;
                }
                k_smooth<<<gv, kBlock, 0, s>>>(n, omega, w.dinv, w.rz, w.z, 0);
            }
            FEM_HIP_CHECK(hipGetLastError());
        } else {
            k_jacobi<<<gv, kBlock, 0, s>>>(n, w.dinv, w.r, w.z);
        }
        k_dots<3><<<gv, kBlock, 0, s>>>(n, w.ptrs, w.ptrs + 3, w.part);
        k_dots_fin<<<1, kBlock, 0, s>>>(w.part, gv, 3, w.sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(3)) return rc;
        double zr = h[0], zz = h[1], zq = h[2];
        // a network output that is non-finite or zero cannot give a direction
        // (z.q_prev enters only after a first step)
        if (use_net && !(std::isfinite(zz) && std::isfinite(zr) && (restart || std::isfinite(zq)) && zz > 0.0)) {
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
        k_dots_fin<<<1, kBlock, 0, s>>>(w.part, gv, 2, w.sums);
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
        k_dots_fin<<<1, kBlock, 0, s>>>(w.part, gv, 1, w.sums);
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
