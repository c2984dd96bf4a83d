// pcg.hip -- Jacobi-preconditioned conjugate gradients driven by the element
// operator, in FP64 and with FP32-stored local matrices inside FP64
// iterative refinement.
//
// One iteration is a single pass over the elements plus two small kernels:
//   element pass  (k_chunk_main with OpIter, then k_chunk_fixup for the nodes
//                  shared between chunks) completes the previous iteration's
//                  update r -= alpha q, x += alpha p while gathering,
//                  forms p = D^{-1} r + beta p in the restriction phase,
//                  computes q = A p, and accumulates seven per-block dot
//                  products: p.q, q.Dr, q.Dq, q.r, q.q and, directly, r.Dr
//                  and r.r of the residual just formed;
//   finalize      one workgroup adds the partials in a fixed order and
//                  advances the scalars: alpha = r.z / p.q and, without a
//                  second reduction, the next r'.z' = r.z - 2 alpha q.Dr +
//                  alpha^2 q.Dq and r'.r' = r.r - 2 alpha q.r + alpha^2 q.q
//                  (the single-reduction form of Chronopoulos & Gear), beta,
//                  and the convergence / refresh decision.  The recurrence
//                  always starts from the directly summed r.z and r.r of the
//                  current residual, so its rounding error cannot accumulate
//                  over iterations (it would, relative to the shrinking r.z,
//                  after a few decades of convergence).
// The element kernels read the scalars that the previous finalize wrote, so
// each value has one writer and a kernel boundary between writer and reader.
// The host only enqueues; it reads the state record every `check_every`
// iterations.  Once the device has raised its flag, the kernels still queued
// return at once.
//
// The iteration vectors live in a solver-local node order: the complete
// nodes of chunk 0, 1, ... (each chunk's block contiguous, in the order of
// its node list), then the shared nodes in shared-node order (DevPlan::
// comp_off).  The element pass then reads and writes each chunk's nodes as
// one contiguous run instead of scattered row segments of the mesh
// numbering, and the shared nodes form the compact tail that the fix-up
// streams.  The caller's x and the FP64 residual refreshes stay in mesh order;
// x is gathered into the local order at the start and scattered back at
// every refresh and at the end.
//
// The operator is stored in the packed symmetric difference form (chunk.h,
// LdPk): FP64 values for the FP64 solver, or FP32 hi/lo pairs for the mixed
// solver, whose iterations read only the FP32 heads.  Every refresh (reliable
// update of Sleijpen & van der Vorst: when r.r has fallen by delta^2 since the
// last refresh, or below the target) applies the pending step, recomputes the
// true residual b - A x in FP64 from hi + lo, and continues CG from it with
// the same search direction.  Iteration vectors are FP64 by default; FP32
// vectors (with an FP32 correction of x folded into the FP64 x at each
// refresh) are the low-traffic variant.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "chunk.h"
#include "kernels.h"
#include "solver.h"

namespace fem {

namespace {

constexpr int kDots = 7;

// r_new = r - alpha q, x_new = x + alpha p, p_new = D^{-1} r_new + beta p
// rounded to the vector type VT.  Written with explicit fma so that the
// element pass and the fix-up produce identical bits for a shared node.
template <class VT>
struct Step {
    __device__ __forceinline__ static VT r_next(VT r, VT q, double alpha) {
        return (VT)__builtin_fma(-alpha, (double)q, (double)r);
    }
    __device__ __forceinline__ static VT x_next(VT x, VT p, double alpha) {
        return (VT)__builtin_fma(alpha, (double)p, (double)x);
    }
    __device__ __forceinline__ static VT p_next(VT d, VT rn, VT p, double beta) {
        return (VT)__builtin_fma(beta, (double)p, (double)d * (double)rn);
    }
};

// The element pass of one CG iteration on solver-local vectors: complete
// nodes by their local index, shared nodes through the tail pointers
// (sx = x + n_complete, ...) by their shared-node number.  A Dirichlet node is
// recognised by D^{-1} = 0.
template <class VT>
struct OpIter {
    static constexpr bool kLocal = true;
    VT *x, *r, *p, *q;
    const VT *dinv;
    VT *sx, *sr, *sp, *sq;
    const VT *sd;
    const IterState *st;
    double *dots;  // [kDots][npart]
    int npart;
    int n_main;  // dot slots [0, n_main) of the element pass, folded in by the fix-up
    // per-thread
    int mode;
    double alpha, beta;
    double d[kDots];

    __device__ __forceinline__ bool begin() {
        if (st->flag) return false;
        mode = st->mode;
        alpha = st->alpha;
        beta = st->beta;
#pragma unroll
        for (int j = 0; j < kDots; ++j) d[j] = 0.0;
        return true;
    }
    // new r, x, p from the old values; wr: r and x changed
    __device__ __forceinline__ void advance(VT r0, VT q0, VT x0, VT p0, VT dv, VT &rn, VT &xn, VT &pn,
                                            bool &wr) const {
        if (mode == MODE_CONTINUE) {
            rn = Step<VT>::r_next(r0, q0, alpha);
            xn = Step<VT>::x_next(x0, p0, alpha);
            pn = Step<VT>::p_next(dv, rn, p0, beta);
            wr = true;
        } else {
            rn = r0;
            xn = x0;
            pn = (mode == MODE_FIRST) ? (VT)((double)dv * (double)rn) : Step<VT>::p_next(dv, rn, p0, beta);
            wr = false;
        }
    }
    __device__ __forceinline__ void direct_dots(VT rn, VT dv) {
        const double rd = (double)rn;
        d[5] += rd * (double)dv * rd;
        d[6] += rd * rd;
    }
    __device__ __forceinline__ void pq_dots(VT pn, VT rn, VT dv, VT qv) {
        const double qd = (double)qv, pd = (double)pn, rd = (double)rn, dd = (double)dv;
        d[0] += pd * qd;
        d[1] += qd * dd * rd;
        d[2] += qd * dd * qd;
        d[3] += qd * rd;
        d[4] += qd * qd;
    }
    __device__ __forceinline__ VT gather(int g, int sidx) {
        VT rn, xn, pn;
        bool wr;
        if (sidx < 0) {
            const VT dv = dinv[g];
            const bool cont = mode == MODE_CONTINUE;
            advance(r[g], cont ? q[g] : (VT)0, cont ? x[g] : (VT)0, mode == MODE_FIRST ? (VT)0 : p[g], dv, rn, xn,
                    pn, wr);
            if (wr) {
                r[g] = rn;
                x[g] = xn;
            }
            p[g] = pn;
            direct_dots(rn, dv);
        } else {
            advance(sr[sidx], sq[sidx], sx[sidx], sp[sidx], sd[sidx], rn, xn, pn, wr);
        }
        return pn;
    }
    __device__ __forceinline__ void finish(int g, VT acc) {
        const VT dv = dinv[g];
        const VT qv = (dv == (VT)0) ? (VT)0 : acc;
        q[g] = qv;
        pq_dots(p[g], r[g], dv, qv);
    }
    struct Pre {
        VT dv, r0, q0, x0, p0;
    };
    // fix-up workgroup b of nb starts from the element pass's dot slots
    // [b per, (b + 1) per): the finalize then adds the fix-up's slots only
    __device__ __forceinline__ void fixup_begin(int b, int nb) {
        const int per = (n_main + nb - 1) / nb;
        const int e = min(n_main, (b + 1) * per);
        for (int i = b * per + (int)threadIdx.x; i < e; i += (int)blockDim.x)
#pragma unroll
            for (int j = 0; j < kDots; ++j) d[j] += dots[(int64_t)j * npart + i];
    }
    __device__ __forceinline__ Pre fixup_load(int s, int) const { return {sd[s], sr[s], sq[s], sx[s], sp[s]}; }
    __device__ __forceinline__ void fixup_store(int s, int, const Pre &pr, VT acc) {
        const VT dv = pr.dv;
        VT rn, xn, pn;
        bool wr;
        advance(pr.r0, pr.q0, pr.x0, pr.p0, dv, rn, xn, pn, wr);
        if (wr) {
            sr[s] = rn;
            sx[s] = xn;
        }
        sp[s] = pn;
        direct_dots(rn, dv);
        const VT qv = (dv == (VT)0) ? (VT)0 : acc;
        sq[s] = qv;
        pq_dots(pn, rn, dv, qv);
    }
    template <int BS>
    __device__ void end(double *red, int slot) {
        block_sum_n<BS, kDots>(d, red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < kDots; ++j) dots[(int64_t)j * npart + slot] = d[j];
    }
};

// perm[local] = mesh node id: complete nodes chunk by chunk, then shared nodes
__global__ __launch_bounds__(kBlock) void k_perm_complete(const DevPlan P, int32_t *__restrict__ perm) {
    for (int64_t c = blockIdx.x; c < P.n_chunks; c += gridDim.x) {
        const int nb0 = P.chunk_node_off[c], ncomp = P.chunk_info[2 * c], off = P.comp_off[c];
        for (int k = threadIdx.x; k < ncomp; k += kBlock) perm[off + k] = P.loc_nodes[nb0 + k];
    }
}
__global__ __launch_bounds__(kBlock) void k_perm_shared(const DevPlan P, int32_t *__restrict__ perm) {
    const int64_t nc = P.comp_off[P.n_chunks];
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < P.n_shared; s += (int64_t)gridDim.x * kBlock)
        perm[nc + s] = P.fix_nodes[s];
}

// dst[i] = src[perm[i]] (mesh order -> local order)
template <class VT>
__global__ __launch_bounds__(kBlock) void k_gather_perm(int64_t n, const int32_t *__restrict__ perm,
                                                        const double *__restrict__ src, VT *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        dst[i] = (VT)src[perm[i]];
}

// Local x back to the caller's x64: copy (FP64 vectors) or add and clear the
// FP32 correction (FP32 vectors).
template <class VT>
__global__ __launch_bounds__(kBlock) void k_scatter_x(int64_t n, const int32_t *__restrict__ perm,
                                                      VT *__restrict__ xl, double *__restrict__ x64, int fold) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int g = perm[i];
        if (fold) {
            x64[g] += (double)xl[i];
            xl[i] = (VT)0;
        } else {
            x64[g] = (double)xl[i];
        }
    }
}

// One workgroup: totals of the dot partials in slots [first, npart), then the
// scalar recurrence.
__global__ __launch_bounds__(kBlock) void k_finalize(IterState *st, const double *__restrict__ dots, int npart,
                                                     int first) {
    __shared__ double red[kDots * (kBlock / kWave)];
    if (st->flag) return;
    // every thread sums a fixed, strided subset of each partial list, four
    // partials in flight per list, then one block reduction of all seven
    double t[kDots];
#pragma unroll
    for (int j = 0; j < kDots; ++j) t[j] = 0.0;
    int k = first + threadIdx.x;
    for (; k + 3 * kBlock < npart; k += 4 * kBlock) {
#pragma unroll
        for (int j = 0; j < kDots; ++j) {
            const double *dj = dots + (int64_t)j * npart;
            t[j] += ((dj[k] + dj[k + kBlock]) + (dj[k + 2 * kBlock] + dj[k + 3 * kBlock]));
        }
    }
    for (; k < npart; k += kBlock)
#pragma unroll
        for (int j = 0; j < kDots; ++j) t[j] += dots[(int64_t)j * npart + k];
    block_sum_n<kBlock, kDots>(t, red);
    if (threadIdx.x != 0) return;
    const double pq = t[0], qDr = t[1], qDq = t[2], qr = t[3], qq = t[4];
    const double rz = t[5], rr = t[6];  // r.Dr and r.r of the residual behind p
    st->rz = rz;
    st->rr = rr;
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
        st->flag = 2;
        st->pending = 0;
        return;
    }
    const double alpha = rz / pq;
    const double rzn = rz - alpha * (2.0 * qDr - alpha * qDq);
    const double rrn = rr - alpha * (2.0 * qr - alpha * qq);
    st->alpha = alpha;
    st->pq = pq;
    st->pending = 1;
    st->n_updates += 1;
    st->rz_next = rzn;
    st->rr_next = rrn;
    const double thr2 = st->thr2, rel2 = st->rel2;
    if (!(rrn > thr2) || (rel2 > 0.0 && rrn < rel2) || !(rzn > 0.0) || !isfinite(rrn)) {
        st->flag = 1;  // the host refreshes; rz stays that of the residual behind p
        return;
    }
    st->beta = rzn / rz;
    st->mode = MODE_CONTINUE;
}

// Applies the pending step to every node (after a trigger or at the end).
template <class VT>
__global__ __launch_bounds__(kBlock) void k_pending(int64_t n, VT *__restrict__ x, VT *__restrict__ r,
                                                    const VT *__restrict__ p, const VT *__restrict__ q,
                                                    const IterState *st) {
    if (!st->pending || st->flag == 2) return;
    const double alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        r[i] = Step<VT>::r_next(r[i], q[i], alpha);
        x[i] = Step<VT>::x_next(x[i], p[i], alpha);
    }
}

// r (VT, local order) = r64 (mesh order), per-block partials of r.D r, r.r
// (VT values) and r64.r64.
template <class VT>
__global__ __launch_bounds__(kBlock) void k_init_dots(int64_t n, VT *__restrict__ r, const VT *__restrict__ dinv,
                                                      const double *__restrict__ r64, const int32_t *__restrict__ perm,
                                                      double *__restrict__ upd) {
    __shared__ double red[kBlock / kWave];
    double srz = 0.0, srr = 0.0, s64 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double v = r64[perm[i]];
        s64 += v * v;
        const VT ri = (VT)v;
        r[i] = ri;
        const double rd = (double)ri;
        srz += rd * (double)dinv[i] * rd;
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

// One workgroup: a fresh residual's totals into the state; the next element
// pass starts a new p (first) or continues the old one with
// beta = r'.z' / r.z (fresh).  The refresh triggers follow: the target
// (tscale ||r_0||)^2 at the first refresh, delta^2 r.r at every one.
__global__ __launch_bounds__(kBlock) void k_refresh_state(IterState *st, const double *__restrict__ upd, int n_upd,
                                                          int first, double tscale, double dd) {
    __shared__ double red[kBlock / kWave];
    const double rz = reduce_partials(upd, n_upd, red);
    const double rr = reduce_partials(upd + n_upd, n_upd, red);
    const double r64 = reduce_partials(upd + 2 * n_upd, n_upd, red);
    if (threadIdx.x == 0) {
        if (first) {
            st->n_updates = 0;
            st->beta = 0.0;
            st->mode = MODE_FIRST;
        } else {
            st->beta = (st->rz > 0.0) ? rz / st->rz : 0.0;
            st->mode = MODE_FRESH;
        }
        st->rz = rz;
        st->rr = rr;
        st->rr64 = r64;
        if (first) st->thr2 = (tscale * sqrt(r64)) * (tscale * sqrt(r64));
        st->rel2 = dd * rr;
        st->flag = 0;
        st->pending = 0;
        st->alpha = 0.0;
    }
}

// D^{-1} in local order (0 on Dirichlet nodes)
template <class VT>
__global__ __launch_bounds__(kBlock) void k_dinv(int64_t n, const double *__restrict__ d,
                                                 const uint8_t *__restrict__ mask, const int32_t *__restrict__ perm,
                                                 VT *__restrict__ dinv, int jacobi, int *__restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int g = perm[i];
        VT v;
        if (mask[g]) v = (VT)0;
        else {
            if (!(d[g] > 0.0)) *bad = 1;  // every writer stores the same value
            v = jacobi ? (VT)(1.0 / d[g]) : (VT)1;
        }
        dinv[i] = v;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T *__restrict__ v, T val) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) v[i] = val;
}

__global__ void k_zero_int(int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

int read_state(IterState *d_st, IterState &h, hipStream_t s) {
    FEM_HIP_CHECK(hipMemcpyAsync(&h, d_st, sizeof(IterState), hipMemcpyDeviceToHost, s));
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
    void harvest() {  // stream already synchronised
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

// The solve for one (NB, EPT, matrix head kind, vector type).
// MK == MAT_MF: matrix-free passes over the coordinates, which w.Apk holds
// in the solver-local order (nu enters the rebuilt A_e).
template <int NB, int EPT, int BS, int MK, class VT>
int cg_run(const DevPlan &P, SolverWork &w, int pk_kind, double nu, const double *b, double *x64, double rtol,
           int max_iter, double delta, int max_outer, int check_every, int profile, fem_solve_info *info,
           hipStream_t s) {
    const bool fold = std::is_same<VT, float>::value;  // FP32 vectors: x is an FP32 correction
    const int64_t n = P.n_nodes;
    const int64_t nc = n - P.n_shared;  // complete nodes; the shared ones are the tail
    VT *xv = fold ? reinterpret_cast<VT *>(w.xc) : reinterpret_cast<VT *>(w.xl);
    VT *r = reinterpret_cast<VT *>(w.r), *p = reinterpret_cast<VT *>(w.p), *q = reinterpret_cast<VT *>(w.q);
    const VT *dinv = reinterpret_cast<const VT *>(w.dinv);
    VT *partv = reinterpret_cast<VT *>(w.partv);
    using LdT = typename std::conditional<MK == MAT_MF, LdMf<NB>, LdPk<NB, MK == MAT_MF ? MAT_F64 : MK>>::type;
    const size_t lds = chunk_lds_for<NB, VT, LdT>(P);
    if (lds > device_lds_limit())
        return set_error(FEM_EINVAL, "the chunk's LDS exceeds the workgroup limit; use smaller chunk_elems");
    const ChunkGrid cg = chunk_grid(P.n_chunks, lds, BS);
    const int gf = P.n_shared > 0 ? fixup_grid(P.n_shared, kFixDotsCap) : 0;
    const int npart = cg.grid + gf;
    const int gu = (int)std::max<int64_t>(1, std::min<int64_t>((n + 4 * kBlock - 1) / (4 * kBlock), 1024));
    const int gv = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
    auto make_ld = [&]() -> LdT {
        if constexpr (MK == MAT_MF)
            return LdT{static_cast<const double *>(w.Apk), n, 1.0, nu};
        else
            return LdT{w.Apk, P.n_elems};
    };
    const LdT ld = make_ld();
    VT *sx = xv + nc, *sr = r + nc, *sp = p + nc, *sq = q + nc;
    const VT *sd = dinv + nc;
    // with a fix-up, its workgroups fold the element pass's dot partials in
    // and the finalize reads the fix-up's slots [cg.grid, npart) only
    const int fin_first = gf ? cg.grid : 0;
    OpIter<VT> op{xv, r, p, q, dinv, sx, sr, sp, sq, sd, w.st, w.dots, npart, fin_first, 0, 0.0, 0.0,
                  {0, 0, 0, 0, 0, 0, 0}};
    auto scatter_x = [&]() { k_scatter_x<VT><<<gv, kBlock, 0, s>>>(n, w.perm, xv, x64, fold ? 1 : 0); };
    const double dd = delta > 0.0 ? delta * delta : 0.0;  // reliable-update factor (0: refresh only at the target)

    // refresh: finish the pending step, x back to mesh order, true FP64
    // residual of x64 into r64 -> local r, totals into the state
    auto refresh = [&](int first) -> int {
        if (!first) k_pending<VT><<<gv, kBlock, 0, s>>>(n, xv, r, p, q, w.st);
        scatter_x();
        int rc = MK == MAT_MF ? launch_apply_mf(P, 1.0, nu, x64, b, w.r64, -1.0, 1, w.part64, s)
                              : launch_apply_pk64(P, pk_kind, w.Apk, x64, b, w.r64, -1.0, 1, w.part64, s);
        if (rc) return rc;
        k_init_dots<VT><<<gu, kBlock, 0, s>>>(n, r, dinv, w.r64, w.perm, w.upd);
        k_refresh_state<<<1, kBlock, 0, s>>>(w.st, w.upd, gu, first, kCertify * rtol, dd);
        FEM_HIP_CHECK(hipGetLastError());
        return 0;
    };

    if (!fold) k_gather_perm<VT><<<gv, kBlock, 0, s>>>(n, w.perm, x64, xv);
    IterState h{};
    int rc = refresh(1);
    if (rc) return rc;
    rc = read_state(w.st, h, s);
    if (rc) return rc;
    const double r0 = std::sqrt(h.rr64);
    info->r0 = r0;
    if (r0 == 0.0) {
        info->relres = 0.0;
        return FEM_OK;
    }
    const double target = kCertify * rtol * r0;
    EventPool ev;
    if (profile > 0 && (rc = ev.ensure(check_every))) return rc;
    int launched = 0, refreshes = 0, status = FEM_OK;
    int64_t calls = 0;
    // one iteration: element pass, fix-up, finalize
    auto iteration = [&](hipStream_t st) {
        k_chunk_main<NB, EPT, BS, VT, LdT, OpIter<VT>, false><<<cg.grid, BS, lds, st>>>(P, ld, op, partv, cg.xcd);
        if (gf) k_chunk_fixup<kFixBlock, VT, OpIter<VT>><<<gf, kFixBlock, 0, st>>>(P, op, partv, cg.grid);
        k_finalize<<<1, kBlock, 0, st>>>(w.st, w.dots, npart, fin_first);
    };
    // without per-pass timing, check_every iterations replay as one HIP graph,
    // captured once per workspace and kernel instance
    const void *key = reinterpret_cast<const void *>(&k_chunk_main<NB, EPT, BS, VT, LdT, OpIter<VT>, false>);
    if (profile == 0 && check_every > 1 && (w.graph_key != key || w.graph_m != check_every)) {
        if (w.graph) {
            FEM_HIP_CHECK(hipGraphExecDestroy(w.graph));
            w.graph = nullptr;
            w.graph_key = nullptr;
        }
        if (!w.cap) FEM_HIP_CHECK(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking));
        hipGraph_t g;
        FEM_HIP_CHECK(hipStreamBeginCapture(w.cap, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < check_every; ++j) iteration(w.cap);
        const hipError_t e = hipStreamEndCapture(w.cap, &g);
        if (e != hipSuccess) return set_error(FEM_EHIP, "capture of the CG iterations failed");
        const hipError_t ei = hipGraphInstantiate(&w.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            w.graph = nullptr;
            return set_error(FEM_EHIP, "instantiation of the CG iteration graph failed");
        }
        w.graph_key = key;
        w.graph_m = check_every;
    }
    const bool use_graph = profile == 0 && check_every > 1 && w.graph_key == key;
    while (true) {
        const int m = std::min(check_every, max_iter - launched);
        if (use_graph && m == check_every) {
            FEM_HIP_CHECK(hipGraphLaunch(w.graph, s));
            calls += m;
        } else for (int j = 0; j < m; ++j) {
            const bool timed = profile > 0 && ((launched + j) % profile == 0) && ev.used < (int)ev.a.size();
            if (timed) FEM_HIP_CHECK(hipEventRecord(ev.a[ev.used], s));
            k_chunk_main<NB, EPT, BS, VT, LdT, OpIter<VT>, false>
                <<<cg.grid, BS, lds, s>>>(P, ld, op, partv, cg.xcd);
            if (gf) k_chunk_fixup<kFixBlock, VT, OpIter<VT>><<<gf, kFixBlock, 0, s>>>(P, op, partv, cg.grid);
            if (timed) {
                FEM_HIP_CHECK(hipEventRecord(ev.b[ev.used], s));
                ev.used++;
            }
            k_finalize<<<1, kBlock, 0, s>>>(w.st, w.dots, npart, fin_first);
            FEM_HIP_CHECK(hipGetLastError());
            ++calls;
        }
        launched += m;
        if ((rc = read_state(w.st, h, s))) return rc;
        if (profile > 0) ev.harvest();
        if (h.flag == 2) {
            status = FEM_EBREAKDOWN;
            scatter_x();
            break;
        }
        if (h.flag == 1) {
            if ((rc = refresh(0))) return rc;
            ++calls;
            if ((rc = read_state(w.st, h, s))) return rc;
            ++refreshes;
            if (std::sqrt(h.rr64) <= target) break;
            if (refreshes >= max_outer) {
                status = FEM_ENOCONV;
                break;
            }
        }
        if (launched >= max_iter) {
            status = FEM_ENOCONV;
            if ((rc = refresh(0))) return rc;
            if ((rc = read_state(w.st, h, s))) return rc;
            break;
        }
    }
    info->iters = h.n_updates;
    info->outer = refreshes;
    info->replacements = refreshes;
    info->matvec_calls = (int)calls;
    info->matvec_ms = ev.ms;
    info->matvec_samples = ev.samples;
    info->relres = std::sqrt(h.rr64) / r0;
    return status;
}

}  // namespace

int solve_pcg(const DevPlan &P, SolverWork &w, int dtype, int vec64, int block, const void *K, const void *M,
              double nu, const double *b, double *x, double rtol, int max_iter, int jacobi, double delta,
              int max_outer, int check_every, int profile, fem_solve_info *info, hipStream_t s) {
    const bool mf = dtype == MAT_MF;
    const bool mixed = dtype != MAT_F64 && !mf;
    const int64_t n = P.n_nodes;
    const int gv = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
    const int pk_kind = mixed ? MAT_F32X2 : MAT_F64;
    const void *Mu = (nu != 0.0) ? M : nullptr;
    int rc = 0;
    if (mf) {
        rc = launch_diag_mf(P, nu, w.d64, w.part64, s);
    } else {
        rc = launch_pack(P, dtype, K, Mu, nu, pk_kind, w.Apk, s);
        if (!rc) rc = launch_diag64(P, dtype, K, Mu, nu, w.d64, w.part64, s);
    }
    if (rc) return rc;
    k_zero_int<<<1, 1, 0, s>>>(w.bad);
    if (P.n_chunks > 0)
        k_perm_complete<<<(int)std::min<int64_t>(P.n_chunks, 4096), kBlock, 0, s>>>(P, w.perm);
    if (P.n_shared > 0)
        k_perm_shared<<<(int)std::max<int64_t>(1, std::min<int64_t>((P.n_shared + kBlock - 1) / kBlock, 4096)),
                        kBlock, 0, s>>>(P, w.perm);
    if (mf)  // coordinates into the solver-local order
        for (int d = 0; d < P.dim; ++d)
            k_gather_perm<double><<<gv, kBlock, 0, s>>>(n, w.perm, P.coords + (int64_t)d * n,
                                                        static_cast<double *>(w.Apk) + (int64_t)d * n);
    const bool v32 = mixed && !vec64;
    if (v32) {
        k_dinv<float><<<gv, kBlock, 0, s>>>(n, w.d64, P.mask, w.perm, reinterpret_cast<float *>(w.dinv), jacobi,
                                            w.bad);
        k_fill<float><<<gv, kBlock, 0, s>>>(n, reinterpret_cast<float *>(w.xc), 0.0f);
    } else {
        k_dinv<double><<<gv, kBlock, 0, s>>>(n, w.d64, P.mask, w.perm, reinterpret_cast<double *>(w.dinv), jacobi,
                                             w.bad);
    }
    FEM_HIP_CHECK(hipGetLastError());
    int bad = 0;
    FEM_HIP_CHECK(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    if (bad) return set_error(FEM_ESINGULAR, "a free node has a non-positive diagonal entry");
    // delta = 0 disables refreshes before the target (FP64 solver)
    const double dl = mixed ? delta : 0.0;
    const int outer_cap = mixed ? max_outer : 4;
    return dispatch_tile(P.E, block, [&](auto bs, auto ept) -> int {
        constexpr int BS = decltype(bs)::value;
        constexpr int EPT = decltype(ept)::value;
        if (P.nb == 3) {
            if (mf) return cg_run<3, EPT, BS, MAT_MF, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                             check_every, profile, info, s);
            if (!mixed) return cg_run<3, EPT, BS, MAT_F64, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                                  check_every, profile, info, s);
            if (v32) return cg_run<3, EPT, BS, MAT_F32, float>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                              check_every, profile, info, s);
            return cg_run<3, EPT, BS, MAT_F32, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                       check_every, profile, info, s);
        }
        if (P.nb == 6) {  // quadratic triangles: stored matrices, FP64 iteration vectors
            if constexpr (EPT * BS <= 1024) {
                if (mf || v32) return set_error(FEM_EINVAL, "quadratic elements need stored matrices and FP64 vectors");
                if (!mixed) return cg_run<6, EPT, BS, MAT_F64, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl,
                                                                      outer_cap, check_every, profile, info, s);
                return cg_run<6, EPT, BS, MAT_F32, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                           check_every, profile, info, s);
            }
            return set_error(FEM_EINVAL, "chunk size too large for quadratic triangles");
        }
        if (P.nb == 10) {  // quadratic tetrahedra: as quadratic triangles
            if constexpr (EPT * BS <= 512) {
                if (mf || v32) return set_error(FEM_EINVAL, "quadratic elements need stored matrices and FP64 vectors");
                if (!mixed) return cg_run<10, EPT, BS, MAT_F64, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl,
                                                                       outer_cap, check_every, profile, info, s);
                return cg_run<10, EPT, BS, MAT_F32, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                            check_every, profile, info, s);
            }
            return set_error(FEM_EINVAL, "chunk size too large for quadratic tetrahedra");
        }
        if constexpr (EPT * BS <= 1536 || (EPT <= 2 && BS == 1024)) {
            if (mf) return cg_run<4, EPT, BS, MAT_MF, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                             check_every, profile, info, s);
            if (!mixed) return cg_run<4, EPT, BS, MAT_F64, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                                  check_every, profile, info, s);
            if (v32) return cg_run<4, EPT, BS, MAT_F32, float>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                              check_every, profile, info, s);
            return cg_run<4, EPT, BS, MAT_F32, double>(P, w, pk_kind, nu, b, x, rtol, max_iter, dl, outer_cap,
                                                       check_every, profile, info, s);
        }
        return set_error(FEM_EINVAL, "chunk size too large for tetrahedra");
    });
}

}  // namespace fem
