// pcg.hip -- Jacobi-preconditioned conjugate gradients driven by the element
// operator, in FP64 and in FP32 with FP64 reliable updates.
//
// One CG iteration is three kernels:
//   main    reduces the previous update's partials (r.z, r.r) in a fixed order,
//           decides convergence / reliable-update on the device, forms
//           beta and p = z + beta p inside the restriction phase of the
//           element operator, q = A p (masked), and per-block p.q partials;
//   fixup   the same for the nodes shared between chunks;
//   update  reduces p.q, alpha = r.z / p.q, x += alpha p, r -= alpha q, and
//           per-block partials of r.z and r.r (z = D^{-1} r is never stored).
// Every reduction has one fixed order (wave64 xor butterfly, then the block's
// four waves, then the blocks in index order), so a solve is bitwise
// reproducible.  The host only enqueues; it reads a small state record every
// `check_every` iterations.  Once the device has raised its flag the remaining
// enqueued kernels return at once.
//
// Mixed precision (FP32 inner, FP64 outer): r, p, q, the correction of x and
// D^{-1} are FP32 and the operator is the FP32 head of the hi/lo pair of the
// combined local matrices; dot products are accumulated in FP64 and alpha /
// beta are FP64.  Whenever the FP32 residual has fallen by a factor `delta`
// since the last refresh (or below the target), the correction is folded into
// the FP64 x, the true residual b - A x is recomputed in FP64 from hi + lo,
// and CG continues from it with the same search direction -- iterative
// refinement in the "reliable update" form of Sleijpen & van der Vorst.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "chunk.h"
#include "kernels.h"
#include "solver.h"

namespace fem {

namespace {

// ---------------------------------------------------------------- ops ----
template <class T>
struct OpPcg {
    const T *r;
    const T *dinv;
    T *p;
    T *q;
    const uint8_t *mask;
    SolveState *st;
    const double *upd;  // [2][n_upd] r.z then r.r partials
    int n_upd;
    double *mv;         // p.q partials: [gm] main blocks then [gf] fixup blocks
    int gm;
    int first;
    double thr2;        // trigger when r.r <= thr2
    double rel2;        // or when r.r < rel2 (reliable update), 0 = off
    T beta;

    __device__ bool begin(double *red) {
        if (st->flag) return false;
        const double rz = reduce_partials(upd, n_upd, red);
        const double rr = reduce_partials(upd + n_upd, n_upd, red);
        if (!(rr > thr2) || (rel2 > 0.0 && rr < rel2) || !isfinite(rz) || !isfinite(rr)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->flag = (isfinite(rz) && isfinite(rr)) ? 1 : 2;
                st->rr_trigger = rr;
            }
            return false;
        }
        const double b = first ? 0.0 : rz / st->rz_prev;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->rz_cur = rz;
            st->beta = b;
        }
        beta = (T)b;
        return true;
    }
    __device__ bool begin_fixup(double *) {
        if (st->flag) return false;
        beta = first ? (T)0 : (T)st->beta;
        return true;
    }
    __device__ __forceinline__ T pnew(int g) const {
        const T z = dinv[g] * r[g];
        return first ? z : z + beta * p[g];
    }
    __device__ __forceinline__ T gather(int g, bool complete) {
        const T v = pnew(g);
        if (complete) p[g] = v;
        return v;
    }
    __device__ __forceinline__ void gather_shared(int g) { p[g] = pnew(g); }
    __device__ __forceinline__ double finish(int g, T acc) const {
        const T qv = mask[g] ? (T)0 : acc;
        q[g] = qv;
        return (double)p[g] * (double)qv;
    }
    __device__ void end(double d, double *red) const {
        const double t = block_sum(d, red);
        if (threadIdx.x == 0) mv[blockIdx.x] = t;
    }
    __device__ void end_fixup(double d, double *red) const {
        const double t = block_sum(d, red);
        if (threadIdx.x == 0) mv[gm + blockIdx.x] = t;
    }
};

// ------------------------------------------------------------- kernels ----
template <class T>
__global__ __launch_bounds__(kBlock) void k_update(int64_t n, T *__restrict__ x, T *__restrict__ r,
                                                   const T *__restrict__ p, const T *__restrict__ q,
                                                   const T *__restrict__ dinv, SolveState *st,
                                                   const double *__restrict__ mv, int n_mv,
                                                   double *__restrict__ upd) {
    __shared__ double red[kBlock / kWave];
    if (st->flag) return;
    const double pq = reduce_partials(mv, n_mv, red);
    const double rz = st->rz_cur;
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->flag = 2;
        return;
    }
    const double ad = rz / pq;
    const T a = (T)ad;
    double srz = 0.0, srr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        x[i] += a * p[i];
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        const double rd = (double)ri;
        srz += rd * (double)(dinv[i] * ri);
        srr += rd * rd;
    }
    srz = block_sum(srz, red);
    srr = block_sum(srr, red);
    if (threadIdx.x == 0) {
        upd[blockIdx.x] = srz;
        upd[gridDim.x + blockIdx.x] = srr;
        if (blockIdx.x == 0) {
            st->rz_prev = rz;
            st->alpha = ad;
            st->n_updates += 1;
        }
    }
}

// Partials of r.z and r.r for a fresh residual (start / refresh).  For the
// mixed-precision path r64 is given: r32 = fl32(r64) is written and the
// r.r partials of r64 go to upd[2 n_upd ...].
template <class T>
__global__ __launch_bounds__(kBlock) void k_init_dots(int64_t n, T *__restrict__ r, const T *__restrict__ dinv,
                                                      const double *__restrict__ r64, double *__restrict__ upd) {
    __shared__ double red[kBlock / kWave];
    double srz = 0.0, srr = 0.0, s64 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        T ri;
        if (r64) {
            const double v = r64[i];
            s64 += v * v;
            ri = (T)v;
            r[i] = ri;
        } else {
            ri = r[i];
        }
        const double rd = (double)ri;
        srz += rd * (double)(dinv[i] * ri);
        srr += rd * rd;
    }
    srz = block_sum(srz, red);
    srr = block_sum(srr, red);
    s64 = block_sum(s64, red);
    if (threadIdx.x == 0) {
        upd[blockIdx.x] = srz;
        upd[gridDim.x + blockIdx.x] = srr;
        upd[2 * gridDim.x + blockIdx.x] = s64;
    }
}

// One block: totals of the init partials into the state record.
__global__ __launch_bounds__(kBlock) void k_reduce_state(SolveState *st, const double *__restrict__ upd, int n_upd) {
    __shared__ double red[kBlock / kWave];
    const double rz = reduce_partials(upd, n_upd, red);
    const double rr = reduce_partials(upd + n_upd, n_upd, red);
    const double r64 = reduce_partials(upd + 2 * n_upd, n_upd, red);
    if (threadIdx.x == 0) {
        st->rz_init = rz;
        st->rr_init = rr;
        st->rr64_init = r64;
        st->flag = 0;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_dinv(int64_t n, const double *__restrict__ d,
                                                 const uint8_t *__restrict__ mask, T *__restrict__ dinv,
                                                 int jacobi, int *__restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        T v;
        if (mask[i]) v = (T)0;
        else {
            if (!(d[i] > 0.0)) *bad = 1;  // benign race: any writer stores 1
            v = jacobi ? (T)(1.0 / d[i]) : (T)1;
        }
        dinv[i] = v;
    }
}

// x64 += xc, xc = 0
__global__ __launch_bounds__(kBlock) void k_fold(int64_t n, double *__restrict__ x, float *__restrict__ xc) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        x[i] += (double)xc[i];
        xc[i] = 0.0f;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T *__restrict__ v, T val) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) v[i] = val;
}

__global__ void k_clear_state(SolveState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        SolveState z{};
        *st = z;
    }
}

__global__ void k_clear_flag(SolveState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->flag = 0;
}

}  // namespace

Grids solver_grids(const DevPlan &P, size_t elem_lds) {
    Grids g;
    g.lds = elem_lds;
    const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / (elem_lds + 1024))));
    g.gm = (int)std::max<int64_t>(1, std::min<int64_t>(P.n_chunks, (int64_t)per_cu * device_cu_count()));
    g.gf = P.n_shared > 0 ? (int)std::min<int64_t>((P.n_shared + kBlock - 1) / kBlock, 1024) : 0;
    g.gu = (int)std::max<int64_t>(1, std::min<int64_t>((P.n_nodes + 4 * kBlock - 1) / (4 * kBlock), 1024));
    return g;
}

// ------------------------------------------------------------ the driver ----
namespace {

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double s() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

int read_state(SolveState *d_st, SolveState &h, hipStream_t s) {
    FEM_HIP_CHECK(hipMemcpyAsync(&h, d_st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    return 0;
}

struct EventPool {
    std::vector<hipEvent_t> a, b;
    int used = 0;
    double ms = 0.0;
    int samples = 0;
    int ensure(int n) {
        while ((int)a.size() < n) {
            hipEvent_t e0, e1;
            FEM_HIP_CHECK(hipEventCreate(&e0));
            FEM_HIP_CHECK(hipEventCreate(&e1));
            a.push_back(e0);
            b.push_back(e1);
        }
        return 0;
    }
    // stream already synchronised
    void harvest() {
        for (int i = 0; i < used; ++i) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, a[i], b[i]) == hipSuccess) {
                ms += t;
                samples++;
            }
        }
        used = 0;
    }
    ~EventPool() {
        for (auto e : a) (void)hipEventDestroy(e);
        for (auto e : b) (void)hipEventDestroy(e);
    }
};

}  // namespace

template <int NB, class T, class Ld>
static int cg_loop(const DevPlan &P, const Ld &ld, SolverWork &w, T *x, T *r, T *p, T *q, const T *dinv,
                   T *scratch, const double *b64, double *x64, const void *A64, int kind64, double rtol, double r0,
                   double delta, int max_iter, int max_outer, int check_every, int profile, fem_solve_info *info,
                   hipStream_t s, const Grids &gr) {
    // x, r, p, q: iteration vectors (T).  For T = float, x is the FP32
    // correction and x64 / b64 / A64 drive the FP64 refresh.
    const bool mixed = !std::is_same<T, double>::value;
    SolveState h{};
    EventPool ev;
    if (profile > 0) {
        int rc = ev.ensure(check_every);
        if (rc) return rc;
    }
    const double thr2 = (rtol * r0) * (rtol * r0);
    double rmax2 = r0 * r0;
    int launched = 0, first = 1, replacements = 0, outer = 0, status = FEM_OK;
    int64_t calls = 0;
    while (true) {
        const int m = std::min(check_every, max_iter - launched);
        for (int j = 0; j < m; ++j) {
            OpPcg<T> op{r, dinv, p, q, P.mask, w.st, w.upd, gr.gu, w.mv, gr.gm, first, thr2,
                        mixed ? delta * delta * rmax2 : 0.0, (T)0};
            const bool timed = profile > 0 && ((launched + j) % profile == 0) && ev.used < (int)ev.a.size();
            if (timed) FEM_HIP_CHECK(hipEventRecord(ev.a[ev.used], s));
            k_chunk_main<NB, T, Ld, OpPcg<T>, false><<<gr.gm, kBlock, gr.lds, s>>>(P, ld, op, scratch);
            if (P.n_shared > 0) k_chunk_fixup<T, OpPcg<T>><<<gr.gf, kBlock, 0, s>>>(P, op, scratch);
            if (timed) {
                FEM_HIP_CHECK(hipEventRecord(ev.b[ev.used], s));
                ev.used++;
            }
            k_update<T><<<gr.gu, kBlock, 0, s>>>(P.n_nodes, x, r, p, q, dinv, w.st, w.mv, gr.gm + gr.gf, w.upd);
            FEM_HIP_CHECK(hipGetLastError());
            first = 0;
            ++calls;
        }
        launched += m;
        int rc = read_state(w.st, h, s);
        if (rc) return rc;
        if (profile > 0) ev.harvest();
        if (h.flag == 2) {
            status = FEM_EBREAKDOWN;
            break;
        }
        if (h.flag == 1) {
            // refresh: true residual in FP64
            if (mixed) {
                k_fold<<<gr.gu, kBlock, 0, s>>>(P.n_nodes, x64, reinterpret_cast<float *>(x));
                FEM_HIP_CHECK(hipGetLastError());
            }
            double *rt = mixed ? w.r64 : reinterpret_cast<double *>(r);
            rc = launch_apply64(P, kind64, A64, nullptr, 0.0, mixed ? x64 : reinterpret_cast<double *>(x), b64, rt,
                                -1.0, 1, w.part64, s);
            if (rc) return rc;
            ++calls;
            k_init_dots<T><<<gr.gu, kBlock, 0, s>>>(P.n_nodes, r, dinv, mixed ? w.r64 : nullptr, w.upd);
            k_reduce_state<<<1, kBlock, 0, s>>>(w.st, w.upd, gr.gu);
            FEM_HIP_CHECK(hipGetLastError());
            rc = read_state(w.st, h, s);
            if (rc) return rc;
            const double rtrue = std::sqrt(mixed ? h.rr64_init : h.rr_init);
            ++outer;
            if (rtrue <= rtol * r0) break;
            if (!mixed && ++replacements > 3) {
                status = FEM_ENOCONV;
                break;
            }
            if (mixed && outer >= max_outer) {
                status = FEM_ENOCONV;
                break;
            }
            rmax2 = h.rr_init;  // FP32 (or FP64) r.r of the refreshed residual
        }
        if (launched >= max_iter) {
            status = FEM_ENOCONV;
            break;
        }
    }
    info->iters = h.n_updates;
    info->outer = mixed ? outer : 0;
    info->replacements = mixed ? 0 : replacements;
    info->matvec_calls = (int)calls;
    info->matvec_ms = ev.ms;
    info->matvec_samples = ev.samples;
    return status;
}

int solve_pcg(const DevPlan &P, SolverWork &w, int dtype, const void *K, const void *M, double nu,
              const double *b, double *x, double rtol, int max_iter, int jacobi, double delta, int max_outer,
              int check_every, int profile, fem_solve_info *info, hipStream_t s) {
    const bool mixed = dtype != MAT_F64;
    const int64_t n = P.n_nodes;
    const int gv = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
    // combined operator: FP64 (dtype F64) or hi/lo pair (mixed)
    const int kout = mixed ? MAT_F32X2 : MAT_F64;
    int rc = launch_combine(P, dtype, K, (nu != 0.0) ? M : nullptr, nu, kout, w.A, s);
    if (rc) return rc;
    // Jacobi diagonal of the combined operator (FP64), then D^{-1} (0 on nd)
    rc = launch_diag64(P, kout, w.A, nullptr, 0.0, w.d64, w.part64, s);
    if (rc) return rc;
    FEM_HIP_CHECK(hipMemsetAsync(w.bad, 0, sizeof(int), s));
    k_clear_state<<<1, 1, 0, s>>>(w.st);
    // x0 residual in FP64 from the full operator
    rc = launch_apply64(P, kout, w.A, nullptr, 0.0, x, b, w.r64, -1.0, 1, w.part64, s);
    if (rc) return rc;
    if (!mixed) {
        double *dinv = w.dinv64;
        k_dinv<double><<<gv, kBlock, 0, s>>>(n, w.d64, P.mask, dinv, jacobi, w.bad);
        FEM_HIP_CHECK(hipGetLastError());
        const Grids gr = solver_grids(P, chunk_lds_bytes<3, double>(P.E) / 3 * P.nb);
        k_init_dots<double><<<gr.gu, kBlock, 0, s>>>(n, w.r64, dinv, nullptr, w.upd);
        k_reduce_state<<<1, kBlock, 0, s>>>(w.st, w.upd, gr.gu);
        FEM_HIP_CHECK(hipGetLastError());
        SolveState h{};
        rc = read_state(w.st, h, s);
        if (rc) return rc;
        int bad = 0;
        FEM_HIP_CHECK(hipMemcpy(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost));
        if (bad) return set_error(FEM_ESINGULAR, "a free node has a non-positive diagonal entry");
        const double r0 = std::sqrt(h.rr_init);
        info->r0 = r0;
        if (r0 == 0.0) {
            info->relres = 0.0;
            return FEM_OK;
        }
        int st;
        if (P.nb == 3) {
            LdKM<3, MAT_F64, double> ld{w.A, nullptr, 0.0, P.n_elems};
            st = cg_loop<3, double>(P, ld, w, x, w.r64, w.p64, w.q64, dinv, w.part64, b, x, w.A, MAT_F64, rtol, r0,
                                    0.0, max_iter, 0, check_every, profile, info, s, gr);
        } else {
            LdKM<4, MAT_F64, double> ld{w.A, nullptr, 0.0, P.n_elems};
            st = cg_loop<4, double>(P, ld, w, x, w.r64, w.p64, w.q64, dinv, w.part64, b, x, w.A, MAT_F64, rtol, r0,
                                    0.0, max_iter, 0, check_every, profile, info, s, gr);
        }
        if (st < 0 && st != FEM_ENOCONV && st != FEM_EBREAKDOWN) return st;
        // final true residual (x is the FP64 solution)
        rc = launch_apply64(P, MAT_F64, w.A, nullptr, 0.0, x, b, w.q64, -1.0, 1, w.part64, s);
        if (rc) return rc;
        k_init_dots<double><<<gr.gu, kBlock, 0, s>>>(n, w.q64, dinv, nullptr, w.upd);
        k_reduce_state<<<1, kBlock, 0, s>>>(w.st, w.upd, gr.gu);
        rc = read_state(w.st, h, s);
        if (rc) return rc;
        info->relres = std::sqrt(h.rr_init) / r0;
        return st;
    }
    // ---- mixed precision ----
    float *dinv = w.dinv32;
    k_dinv<float><<<gv, kBlock, 0, s>>>(n, w.d64, P.mask, dinv, jacobi, w.bad);
    k_fill<float><<<gv, kBlock, 0, s>>>(n, w.xc32, 0.0f);
    FEM_HIP_CHECK(hipGetLastError());
    const Grids gr = solver_grids(P, chunk_lds_bytes<3, float>(P.E) / 3 * P.nb);
    k_init_dots<float><<<gr.gu, kBlock, 0, s>>>(n, w.r32, dinv, w.r64, w.upd);
    k_reduce_state<<<1, kBlock, 0, s>>>(w.st, w.upd, gr.gu);
    FEM_HIP_CHECK(hipGetLastError());
    SolveState h{};
    rc = read_state(w.st, h, s);
    if (rc) return rc;
    int bad = 0;
    FEM_HIP_CHECK(hipMemcpy(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost));
    if (bad) return set_error(FEM_ESINGULAR, "a free node has a non-positive diagonal entry");
    const double r0 = std::sqrt(h.rr64_init);
    info->r0 = r0;
    if (r0 == 0.0) {
        info->relres = 0.0;
        return FEM_OK;
    }
    const float *Ahi = reinterpret_cast<const float *>(w.A);
    int st;
    if (P.nb == 3) {
        LdF32<3> ld{Ahi, P.n_elems};
        st = cg_loop<3, float>(P, ld, w, w.xc32, w.r32, w.p32, w.q32, dinv, w.part32, b, x, w.A, MAT_F32X2, rtol, r0,
                               delta, max_iter, max_outer, check_every, profile, info, s, gr);
    } else {
        LdF32<4> ld{Ahi, P.n_elems};
        st = cg_loop<4, float>(P, ld, w, w.xc32, w.r32, w.p32, w.q32, dinv, w.part32, b, x, w.A, MAT_F32X2, rtol, r0,
                               delta, max_iter, max_outer, check_every, profile, info, s, gr);
    }
    if (st < 0 && st != FEM_ENOCONV && st != FEM_EBREAKDOWN) return st;
    // fold any pending correction and measure the true FP64 residual
    k_fold<<<gr.gu, kBlock, 0, s>>>(n, x, w.xc32);
    rc = launch_apply64(P, MAT_F32X2, w.A, nullptr, 0.0, x, b, w.r64, -1.0, 1, w.part64, s);
    if (rc) return rc;
    k_init_dots<float><<<gr.gu, kBlock, 0, s>>>(n, w.r32, dinv, w.r64, w.upd);
    k_reduce_state<<<1, kBlock, 0, s>>>(w.st, w.upd, gr.gu);
    rc = read_state(w.st, h, s);
    if (rc) return rc;
    info->relres = std::sqrt(h.rr64_init) / r0;
    return st;
}

}  // namespace fem
