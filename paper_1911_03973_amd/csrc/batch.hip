// batch.hip -- many independent problems solved by one persistent kernel.
//
// Every problem keeps its own Jacobi-PCG (FP32 operator heads, FP64 vectors,
// FP64 reliable refreshes; the scheme of pcg.hip).  All problems share one
// launch: its workgroups take work items from a device queue,
//   CHUNK(p, j)  the element pass of chunk j of problem p,
//   FIX(p, j)    the shared-node fix-up of segment j of problem p,
//   FIN(p)       the scalar step of problem p,
// and each problem alternates between iteration rounds (element pass with
// the CG updates) and refresh rounds (pending step + FP64 residual b - A x).
// Per problem, an integer counter counts the finished items of the current
// phase; the workgroup that finishes the last one enqueues the next phase.
// The workgroup finishing a problem's last CHUNK item also runs its fix-up
// (when it has at most inline_segs segments) and its scalar step, and the one
// finishing the last FIX item runs the scalar step, so one iteration of a
// problem costs one or two trips through the queue instead of three.  With
// `adaptive`, once fewer problems are left than the grid can keep busy, a
// problem's next phase is cut into more CHUNK items (down to one chunk each,
// aiming at one item per workgroup over the live problems) and its fix-up
// goes to FIX items instead of running inline; partials are per chunk and
// per segment, so the grouping never changes a result.
// Nothing ever waits for another workgroup: a workgroup only waits for the
// queue to hold an item, so the launch needs no co-residency, and it ends
// when every problem is finished.  A wall-clock watchdog bounds every wait,
// so a logic error ends the launch with an abort flag instead of a hang.
//
// Memory ordering: producers release (agent-scope fence) before they count or
// publish an item; the counter's last arriver and every consumer acquire
// after reading it.  All floating-point sums keep a fixed order (per-chunk and
// per-segment partials summed in index order by FIN), so the result does not
// depend on which workgroup ran which item.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "chunk.h"
#include "kernels.h"
#include "solver.h"

namespace fem {

namespace {

constexpr int kSeg = kBatchSeg;  // shared nodes per fix-up item
constexpr int kBDots = 7;
enum ItemType : unsigned long long { IT_CHUNK = 1, IT_FIX = 2, IT_FIN = 3 };

__device__ __forceinline__ unsigned long long make_item(unsigned long long t, int p, int j) {
    return (t << 56) | ((unsigned long long)(unsigned)p << 28) | (unsigned long long)(unsigned)j;
}

struct BatchArgs {
    DevPlan P;
    const void *A;  // packed pair [2][NP][n_elems]: heads for iterations, hi + lo for refreshes
    double *x, *r, *p, *q;
    const double *dinv, *b;
    double *sx, *sr, *sp, *sq, *sd;  // shared-node tails of the local vectors [n_shared]
    const double *sb;
    double *part;                    // shared-node partials [n_partials]
    const int32_t *pchunk0, *pshared0, *pseg0;  // [P+1]
    const int32_t *pgroup;                      // [P] chunks per CHUNK item
    int nprob;
    BatchProblem *prob;
    int *cnt;        // [P] finished items of the current phase
    double *cdots;   // [n_chunks][kBDots]
    double *sdots;   // [n_segments][kBDots]
    unsigned long long *qitems, *qtags, *qhead, *qtail;
    unsigned long long qmask;
    int *ndone, *abort_flag;
    double rtol, delta;
    int max_iter, max_refresh;
    int inline_segs;       // the last CHUNK item runs up to this many fix-up segments itself
    int adaptive;          // regroup items by the number of live problems
    long long spin_ticks;  // watchdog, in 100 MHz ticks
};

__device__ __forceinline__ long long now_ticks() { return (long long)__builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ unsigned long long ld_acq(unsigned long long *a) {
    return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_acq_i(int *a) {
    return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Whole workgroup: append items (type, p, 0..n-1) to the queue.  The items
// are written by all threads; after a barrier one thread releases them and
// publishes their tags.
template <int BS>
__device__ void enqueue(const BatchArgs &a, unsigned long long type, int p, int n, unsigned long long *s_base) {
    if (threadIdx.x == 0) *s_base = atomicAdd(a.qtail, (unsigned long long)n);
    __syncthreads();
    const unsigned long long base = *s_base;
    for (int i = threadIdx.x; i < n; i += BS)
        __hip_atomic_store(&a.qitems[(base + i) & a.qmask], make_item(type, p, i), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        for (int i = 0; i < n; ++i)
            __hip_atomic_store(&a.qtags[(base + i) & a.qmask], base + i + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Whole workgroup, after an item of problem p's current phase is done:
// returns true in every thread of the workgroup that finished the phase.
template <int BS>
__device__ bool phase_done(const BatchArgs &a, int p, int n_items, int *s_last) {
    __syncthreads();  // every store of the workgroup has completed
    if (threadIdx.x == 0) {
        __threadfence();  // release them at agent scope
        const int old = atomicAdd(&a.cnt[p], 1);
        int last = old == n_items - 1;
        if (last) {
            __threadfence();  // acquire the other workgroups' stores
            __hip_atomic_store(&a.cnt[p], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *s_last = last;
    }
    __syncthreads();
    return *s_last != 0;
}

// ---- element-pass policies ------------------------------------------------
struct BOpIter {  // iteration round (see OpIter in pcg.hip), solver-local vectors
    static constexpr bool kLocal = true;
    double *x, *r, *p, *q;
    const double *dinv;
    double *sx, *sr, *sp, *sq;
    const double *sd;
    int mode;
    double alpha, beta;
    double d[kBDots];
    __device__ __forceinline__ void advance(double r0, double q0, double x0, double p0, double dv, double &rn,
                                            double &xn, double &pn, bool &wr) const {
        if (mode == MODE_CONTINUE) {
            rn = __builtin_fma(-alpha, q0, r0);
            xn = __builtin_fma(alpha, p0, x0);
            pn = __builtin_fma(beta, p0, dv * rn);
            wr = true;
        } else {
            rn = r0;
            xn = x0;
            pn = (mode == MODE_FIRST) ? dv * rn : __builtin_fma(beta, p0, dv * rn);
            wr = false;
        }
    }
    __device__ __forceinline__ void direct(double rn, double dv) {
        d[5] += rn * dv * rn;
        d[6] += rn * rn;
    }
    __device__ __forceinline__ void pqd(double pn, double rn, double dv, double qv) {
        d[0] += pn * qv;
        d[1] += qv * dv * rn;
        d[2] += qv * dv * qv;
        d[3] += qv * rn;
        d[4] += qv * qv;
    }
    __device__ __forceinline__ double gather(int g, int sidx) {
        double rn, xn, pn;
        bool wr;
        if (sidx < 0) {
            const double dv = dinv[g];
            const bool cont = mode == MODE_CONTINUE;
            advance(r[g], cont ? q[g] : 0.0, cont ? x[g] : 0.0, mode == MODE_FIRST ? 0.0 : p[g], dv, rn, xn, pn, wr);
            if (wr) {
                r[g] = rn;
                x[g] = xn;
            }
            p[g] = pn;
            direct(rn, dv);
        } else {
            advance(sr[sidx], sq[sidx], sx[sidx], mode == MODE_FIRST ? 0.0 : sp[sidx], sd[sidx], rn, xn, pn, wr);
        }
        return pn;
    }
    __device__ __forceinline__ void finish(int g, double acc) {
        const double dv = dinv[g];
        const double qv = dv == 0.0 ? 0.0 : acc;
        q[g] = qv;
        pqd(p[g], r[g], dv, qv);
    }
    __device__ __forceinline__ void fixup_node(int s, int, double acc) {
        const double dv = sd[s];
        double rn, xn, pn;
        bool wr;
        advance(sr[s], sq[s], sx[s], mode == MODE_FIRST ? 0.0 : sp[s], dv, rn, xn, pn, wr);
        if (wr) {
            sr[s] = rn;
            sx[s] = xn;
        }
        sp[s] = pn;
        direct(rn, dv);
        const double qv = dv == 0.0 ? 0.0 : acc;
        sq[s] = qv;
        pqd(pn, rn, dv, qv);
    }
};

struct BOpRefresh {  // refresh round: pending step on x, then r = b - A x (solver-local vectors)
    static constexpr bool kLocal = true;
    double *x, *r;
    const double *p, *dinv, *b;
    double *sx, *sr;
    const double *sp, *sd, *sb;
    double alpha;  // 0 when nothing is pending
    double d[kBDots];
    __device__ __forceinline__ double gather(int g, int sidx) {
        if (sidx < 0) {
            const double xn = alpha != 0.0 ? __builtin_fma(alpha, p[g], x[g]) : x[g];
            if (alpha != 0.0) x[g] = xn;
            return xn;
        }
        return alpha != 0.0 ? __builtin_fma(alpha, sp[sidx], sx[sidx]) : sx[sidx];
    }
    __device__ __forceinline__ void finish(int g, double acc) {
        const double dv = dinv[g];
        const double rv = dv == 0.0 ? 0.0 : b[g] - acc;
        r[g] = rv;
        d[5] += rv * dv * rv;
        d[6] += rv * rv;
    }
    __device__ __forceinline__ void fixup_node(int s, int, double acc) {
        const double dv = sd[s];
        if (alpha != 0.0) sx[s] = __builtin_fma(alpha, sp[s], sx[s]);
        const double rv = dv == 0.0 ? 0.0 : sb[s] - acc;
        sr[s] = rv;
        d[5] += rv * dv * rv;
        d[6] += rv * rv;
    }
};

template <int BS>
__device__ void store_dots(double (&d)[kBDots], double *red, double *dst) {
    block_sum_n<BS, kBDots>(d, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < kBDots; ++j) dst[j] = d[j];
}

// The element pass of chunks c_first .. c_first + n - 1 of one problem (the
// phases of chunk_pass), each chunk's dot partials to cdots[c].  The union
// plan of the batch has ragged chunks, so a chunk's element range is a load
// that its matrix fetch depends on; it is requested one chunk ahead, and only
// the first chunk of the item waits for it.
template <int NB, int EPT, int BS, class Ld, class Op>
__device__ __forceinline__ void batch_chunks(const DevPlan &P, const Ld &ld, Op &op, double *__restrict__ partial,
                                             int64_t c_first, int n, double *buf, uint16_t *sl, double *red,
                                             double *cdots) {
    static_assert(Op::kLocal, "the batched ops address vectors in the solver-local node order");
    int64_t e0n = 0;
    int nen = 0;
    if (n > 0) chunk_range(P, c_first, e0n, nen);
    for (int i = 0; i < n; ++i) {
        const int64_t c = c_first + i;
        const int64_t e0 = e0n;
        const int ne = nen;
        typename Ld::Regs R[EPT];
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int le = t * BS + threadIdx.x;
            if (le < ne) ld.fetch(e0 + le, R[t]);
        }
        if (i + 1 < n) chunk_range(P, c + 1, e0n, nen);
        __syncthreads();  // every thread is done with buf / sl of the previous chunk
        const int nb0 = P.chunk_node_off[c];
        const int nl = P.chunk_node_off[c + 1] - nb0;
        const int ncomp = P.chunk_info[2 * c];
        const int pbase = P.chunk_info[2 * c + 1];
        const int coff = P.comp_off[c];
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(P.slots + c * (int64_t)NB * P.E);
            uint4 *dst = reinterpret_cast<uint4 *>(sl);
            const int nv = (ne * NB + 7) >> 3;
            for (int k = threadIdx.x; k < nv; k += BS) dst[k] = src[k];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nl; k += BS) {
            const int g = k < ncomp ? coff + k : -1;
            const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
            const int s1 = P.loc_end[nb0 + k];
            const double v = op.gather(g, k < ncomp ? -1 : P.part_owner[pbase + (k - ncomp)]);
            for (int s = s0; s < s1; ++s) buf[sl[s]] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int le = t * BS + threadIdx.x;
            if (le < ne) {
                double xe[NB], y[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) xe[j] = buf[le * NB + j];
                Ld::apply(R[t], xe, y);
#pragma unroll
                for (int j = 0; j < NB; ++j) buf[le * NB + j] = y[j];
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nl; k += BS) {
            const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
            const int s1 = P.loc_end[nb0 + k];
            double acc = 0.0;
            for (int s = s0; s < s1; ++s) acc += buf[sl[s]];
            if (k < ncomp) op.finish(coff + k, acc);
            else partial[pbase + (k - ncomp)] = acc;
        }
        store_dots<BS>(op.d, red, cdots + c * kBDots);
#pragma unroll
        for (int t = 0; t < kBDots; ++t) op.d[t] = 0.0;
    }
}

// ---- the persistent kernel -------------------------------------------------
template <int NB, int EPT, int BS>
__global__ __launch_bounds__(BS) void k_batch(const BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *buf = reinterpret_cast<double *>(smem);
    uint16_t *sl = reinterpret_cast<uint16_t *>(smem + (size_t)NB * a.P.E * sizeof(double));
    __shared__ RedBuf<BS> red;
    __shared__ unsigned long long s_item, s_base;
    __shared__ int s_exit, s_last, s_few;
    __shared__ double s_sc[8];
    const DevPlan &P = a.P;
    while (true) {
        if (threadIdx.x == 0) {
            const unsigned long long idx = atomicAdd(a.qhead, 1ull);
            const long long t0 = now_ticks();
            int ex = 0;
            unsigned long long item = 0;
            // second bound, independent of the clock: about 2^28 sleeps of
            // ~60 ns each
            for (unsigned spins = 0;; ++spins) {
                if (__hip_atomic_load(&a.qtags[idx & a.qmask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                    idx + 1) {
                    __threadfence();  // acquire the item and everything released before it
                    item = __hip_atomic_load(&a.qitems[idx & a.qmask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if ((spins & 63) == 63 && (ld_acq_i(a.ndone) >= a.nprob || ld_acq_i(a.abort_flag))) {
                    ex = 1;
                    break;
                }
                if (now_ticks() - t0 > a.spin_ticks || spins > (1u << 28)) {
                    __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    ex = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            s_item = item;
            s_exit = ex;
        }
        __syncthreads();
        if (s_exit) break;
        const unsigned long long item = s_item;
        const int type = (int)(item >> 56);
        const int p = (int)((item >> 28) & 0xFFFFFFFull);
        const int j = (int)(item & 0xFFFFFFFull);
        BatchProblem *pr = a.prob + p;
        const int c0 = a.pchunk0[p], nch = a.pchunk0[p + 1] - c0;
        const int grp = pr->grp;  // chunks per CHUNK item of this phase
        const int nci = (nch + grp - 1) / grp;
        const int sh0 = a.pshared0[p], nsh = a.pshared0[p + 1] - sh0;
        const int sg0 = a.pseg0[p], nseg = a.pseg0[p + 1] - sg0;
        const int round = pr->round;
        // fix-up of shared-node segment jj of p; its dot partials into sdots
        auto fix_loop = [&](auto &op, int jj) {
            const int s1 = min(nsh, (jj + 1) * kSeg);
            for (int sl_ = jj * kSeg + threadIdx.x; sl_ < s1; sl_ += BS) {
                const int sg = sh0 + sl_;
                double acc = 0.0;
                for (int k = P.fix_off[sg]; k < P.fix_off[sg + 1]; ++k) acc += a.part[P.fix_parts[k]];
                op.fixup_node(sg, P.fix_nodes[sg], acc);
            }
        };
        auto fix_segment = [&](int jj) {
            double d[kBDots];
            if (round == 0) {
                BOpIter op{a.x, a.r, a.p, a.q, a.dinv, a.sx, a.sr, a.sp, a.sq, a.sd, pr->mode, pr->alpha, pr->beta,
                           {0, 0, 0, 0, 0, 0, 0}};
                fix_loop(op, jj);
#pragma unroll
                for (int t = 0; t < kBDots; ++t) d[t] = op.d[t];
            } else {
                BOpRefresh op{a.x, a.r, a.p, a.dinv, a.b, a.sx, a.sr, a.sp, a.sd, a.sb,
                              pr->pending ? pr->alpha : 0.0, {0, 0, 0, 0, 0, 0, 0}};
                fix_loop(op, jj);
#pragma unroll
                for (int t = 0; t < kBDots; ++t) d[t] = op.d[t];
            }
            store_dots<BS>(d, red.v, a.sdots + (int64_t)(sg0 + jj) * kBDots);
        };
        // the scalar step of p (every partial of the phase is visible to this
        // workgroup), then the next phase or the end of p
        auto finish_phase = [&]() {
            __syncthreads();  // sdots written by this workgroup
            double t[kBDots];
#pragma unroll
            for (int k = 0; k < kBDots; ++k) t[k] = 0.0;
            for (int c = threadIdx.x; c < nch; c += BS)
#pragma unroll
                for (int k = 0; k < kBDots; ++k) t[k] += a.cdots[(int64_t)(c0 + c) * kBDots + k];
            for (int sgi = threadIdx.x; sgi < nseg; sgi += BS)
#pragma unroll
                for (int k = 0; k < kBDots; ++k) t[k] += a.sdots[(int64_t)(sg0 + sgi) * kBDots + k];
            block_sum_n<BS, kBDots>(t, red.v);
            if (threadIdx.x == 0) {
                int next = 0;  // 0 done, 1 iterate, 2 refresh
                const double rz = t[5], rr = t[6];
                if (round == 1) {
                    pr->refreshes += pr->first ? 0 : 1;
                    if (pr->first) {
                        pr->r0 = sqrt(rr);
                        pr->thr2 = (kCertify * a.rtol * pr->r0) * (kCertify * a.rtol * pr->r0);
                    }
                    pr->rr_true = rr;
                    if (pr->broken) {
                        pr->status = FEM_EBREAKDOWN;
                    } else if (!(pr->r0 > 0.0) || rr <= pr->thr2) {
                        pr->status = 0;
                    } else if (pr->iters >= a.max_iter || pr->refreshes > a.max_refresh || !isfinite(rr)) {
                        pr->status = FEM_ENOCONV;
                    } else {
                        pr->beta = pr->first ? 0.0 : rz / pr->rz;
                        pr->mode = pr->first ? MODE_FIRST : MODE_FRESH;
                        pr->rel2 = a.delta * a.delta * rr;
                        pr->first = 0;
                        pr->pending = 0;
                        pr->round = 0;
                        next = 1;
                    }
                } else {
                    const double pq = t[0], qDr = t[1], qDq = t[2], qr = t[3], qq = t[4];
                    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
                        pr->broken = 1;
                        pr->pending = 0;
                        pr->round = 1;
                        next = 2;  // one refresh round writes back a consistent x, then stops
                    } else {
                        const double alpha = rz / pq;
                        const double rzn = rz - alpha * (2.0 * qDr - alpha * qDq);
                        const double rrn = rr - alpha * (2.0 * qr - alpha * qq);
                        pr->alpha = alpha;
                        pr->rz = rz;
                        pr->pending = 1;
                        pr->iters += 1;
                        if (!(rrn > pr->thr2) || rrn < pr->rel2 || !(rzn > 0.0) || pr->iters >= a.max_iter) {
                            pr->round = 1;
                            next = 2;
                        } else {
                            pr->beta = rzn / rz;
                            pr->mode = MODE_CONTINUE;
                            next = 1;
                        }
                    }
                }
                int items = (nch + pr->grp - 1) / pr->grp;
                if (next != 0 && a.adaptive) {
                    // aim at one item per workgroup over the problems still live
                    // (longer items cost fewer queue trips; two or four per
                    // workgroup were measured slower)
                    const int live = max(1, a.nprob - __hip_atomic_load(a.ndone, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT));
                    const int want = (int)((gridDim.x + live - 1) / live);
                    const int base = (nch + a.pgroup[p] - 1) / a.pgroup[p];
                    items = min(nch, max(base, want));
                    pr->grp = (nch + items - 1) / items;
                    items = (nch + pr->grp - 1) / pr->grp;
                }
                s_sc[0] = (double)next;
                s_sc[1] = (double)items;
            }
            __syncthreads();
            const int next = (int)s_sc[0];
            if (next == 0) {
                if (threadIdx.x == 0) {
                    pr->flag = 1;
                    __threadfence();
                    atomicAdd(a.ndone, 1);
                }
            } else {
                enqueue<BS>(a, IT_CHUNK, p, (int)s_sc[1], &s_base);
            }
        };
        if (type == IT_CHUNK) {
            if (round == 0) {
                BOpIter op{a.x, a.r, a.p, a.q, a.dinv, a.sx, a.sr, a.sp, a.sq, a.sd, pr->mode, pr->alpha, pr->beta,
                           {0, 0, 0, 0, 0, 0, 0}};
                LdPk<NB, MAT_F32> ld{a.A, P.n_elems};
                const int cj0 = j * grp, cj1 = min(nch, (j + 1) * grp);
                batch_chunks<NB, EPT, BS>(P, ld, op, a.part, c0 + cj0, cj1 - cj0, buf, sl, red.v, a.cdots);
            } else {
                BOpRefresh op{a.x, a.r, a.p, a.dinv, a.b, a.sx, a.sr, a.sp, a.sd, a.sb,
                              pr->pending ? pr->alpha : 0.0, {0, 0, 0, 0, 0, 0, 0}};
                LdPk<NB, MAT_F32X2> ld{a.A, P.n_elems};
                const int cj0 = j * grp, cj1 = min(nch, (j + 1) * grp);
                batch_chunks<NB, EPT, BS>(P, ld, op, a.part, c0 + cj0, cj1 - cj0, buf, sl, red.v, a.cdots);
            }
            if (phase_done<BS>(a, p, nci, &s_last)) {
                // the last CHUNK item of the phase: a few fix-up segments and the
                // scalar step run here, so the phase costs one queue trip --
                // unless few problems are left (fewer than one per eight
                // workgroups; one per two to one per 64 measured), when
                // parallel FIX items are faster
                if (threadIdx.x == 0)
                    s_few = a.adaptive && nseg > 1 &&
                            8 * (a.nprob - __hip_atomic_load(a.ndone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) <
                                (int)gridDim.x;
                __syncthreads();
                if (nseg > a.inline_segs || s_few) {
                    enqueue<BS>(a, IT_FIX, p, nseg, &s_base);
                } else {
                    for (int jj = 0; jj < nseg; ++jj) fix_segment(jj);
                    finish_phase();
                }
            }
        } else if (type == IT_FIX) {
            fix_segment(j);
            if (phase_done<BS>(a, p, nseg, &s_last)) finish_phase();
        } else {
            finish_phase();
        }
        __syncthreads();
    }
}

// ---- setup kernels -----------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_batch_init(BatchArgs a, int64_t n_items) {
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = tid; i <= a.qmask; i += stride) a.qtags[i] = 0;
    for (int p = (int)tid; p < a.nprob; p += (int)stride) {
        BatchProblem z{};
        z.round = 1;
        z.first = 1;
        z.status = FEM_ENOCONV;
        z.grp = a.pgroup[p];
        a.prob[p] = z;
        a.cnt[p] = 0;
    }
    if (tid == 0) {
        *a.qhead = 0;
        *a.qtail = (unsigned long long)n_items;
        *a.ndone = 0;
        *a.abort_flag = 0;
    }
}

// Initial items: the first (refresh) round of every problem, in problem
// order; item k of the seed is group j of problem p with pitem0[p] + j = k.
__global__ __launch_bounds__(kBlock) void k_batch_seed(BatchArgs a, const int32_t *__restrict__ pitem0,
                                                       int64_t n_items) {
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n_items; c += (int64_t)gridDim.x * kBlock) {
        int lo = 0, hi = a.nprob;
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (pitem0[mid] <= c) lo = mid;
            else hi = mid;
        }
        a.qitems[c & a.qmask] = make_item(IT_CHUNK, lo, (int)(c - pitem0[lo]));
        a.qtags[c & a.qmask] = (unsigned long long)c + 1;
    }
}

// A problem with no element at all finishes at once (no item would start it).
__global__ void k_batch_empty(BatchArgs a) {
    for (int p = threadIdx.x; p < a.nprob; p += blockDim.x)
        if (a.pchunk0[p + 1] == a.pchunk0[p]) {
            a.prob[p].flag = 1;
            a.prob[p].status = 0;
            atomicAdd(a.ndone, 1);
        }
}

// Packed pair of A_e = K_e + nu_p M_e with the problem's own nu.
template <int NB, int KIN>
__global__ __launch_bounds__(kBlock) void k_pack_batch(const void *__restrict__ K, const void *__restrict__ M,
                                                       const double *__restrict__ nu, const int64_t *__restrict__ elem0,
                                                       int nprob, int64_t n_elems, float *__restrict__ A) {
    constexpr int NP = NB + NB * (NB - 1) / 2;
    const int64_t blk_in = (int64_t)NB * NB * n_elems;
    const int64_t blk_out = (int64_t)NP * n_elems;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n_elems; e += (int64_t)gridDim.x * kBlock) {
        int lo = 0, hi = nprob;
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (elem0[mid] <= e) lo = mid;
            else hi = mid;
        }
        const double v = nu[lo];
        double a[NB][NB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
                const int64_t idx = (int64_t)(i * NB + jj) * n_elems + e;
                a[i][jj] = load_entry<KIN>(K, idx, blk_in) + v * load_entry<KIN>(M, idx, blk_in);
            }
        auto put = [&](int k, double val) {
            const float hi32 = (float)val;
            A[(int64_t)k * n_elems + e] = hi32;
            A[blk_out + (int64_t)k * n_elems + e] = (float)(val - (double)hi32);
        };
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            double rho = a[i][i];
#pragma unroll
            for (int jj = 0; jj < NB; ++jj)
                if (jj != i) rho += 0.5 * (a[i][jj] + a[jj][i]);
            put(i, rho);
        }
        int k = NB;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int jj = i + 1; jj < NB; ++jj) put(k++, 0.5 * (a[i][jj] + a[jj][i]));
    }
}

}  // namespace

int batch_pack(const DevPlan &P, int kin, const void *K, const void *M, const double *d_nu, const int64_t *d_elem0,
               int nprob, float *A, hipStream_t s) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((P.n_elems + kBlock - 1) / kBlock, 65536));
#define FEM_PB(NB, KI) k_pack_batch<NB, KI><<<g, kBlock, 0, s>>>(K, M, d_nu, d_elem0, nprob, P.n_elems, A)
    if (P.nb == 3) {
        if (kin == MAT_F64) FEM_PB(3, MAT_F64);
        else if (kin == MAT_F32) FEM_PB(3, MAT_F32);
        else FEM_PB(3, MAT_F32X2);
    } else {
        if (kin == MAT_F64) FEM_PB(4, MAT_F64);
        else if (kin == MAT_F32) FEM_PB(4, MAT_F32);
        else FEM_PB(4, MAT_F32X2);
    }
#undef FEM_PB
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int batch_launch(const BatchLaunch &L, hipStream_t s) {
    BatchArgs a{};
    a.P = L.P;
    a.A = L.A;
    a.x = L.x;
    a.r = L.r;
    a.p = L.p;
    a.q = L.q;
    a.dinv = L.dinv;
    a.b = L.b;
    const int64_t nc = L.P.n_nodes - L.P.n_shared;  // complete nodes; the shared ones are the tail
    a.sx = L.x + nc;
    a.sr = L.r + nc;
    a.sp = L.p + nc;
    a.sq = L.q + nc;
    a.sd = const_cast<double *>(L.dinv) + nc;
    a.sb = L.b + nc;
    a.part = L.part;
    a.pchunk0 = L.pchunk0;
    a.pshared0 = L.pshared0;
    a.pseg0 = L.pseg0;
    a.pgroup = L.pgroup;
    a.inline_segs = L.inline_segs;
    a.adaptive = L.adaptive;
    a.nprob = L.nprob;
    a.prob = L.prob;
    a.cnt = L.cnt;
    a.cdots = L.cdots;
    a.sdots = L.sdots;
    a.qitems = L.qitems;
    a.qtags = L.qtags;
    a.qhead = L.qhead;
    a.qtail = L.qtail;
    a.qmask = L.qcap - 1;
    a.ndone = L.ndone;
    a.abort_flag = L.abort_flag;
    a.rtol = L.rtol;
    a.delta = L.delta;
    a.max_iter = L.max_iter;
    a.max_refresh = L.max_refresh;
    a.spin_ticks = (long long)(L.watchdog_seconds * 1e8);
    const int gi = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)(L.qcap / kBlock), 4096));
    k_batch_init<<<gi, kBlock, 0, s>>>(a, L.n_seed);
    k_batch_seed<<<gi, kBlock, 0, s>>>(a, L.pitem0, L.n_seed);
    k_batch_empty<<<1, kBlock, 0, s>>>(a);
    FEM_HIP_CHECK(hipGetLastError());
    const size_t lds = chunk_lds_bytes<3, double>(L.P.E) / 3 * L.P.nb;
    const int per_cu = std::max(1, std::min(2048 / L.block, (int)(160 * 1024 / (lds + 2048))));
    const int grid = L.grid > 0 ? L.grid : per_cu * device_cu_count();
    int rc = dispatch_tile(L.P.E, L.block, [&](auto bs, auto ept) -> int {
        constexpr int BS = decltype(bs)::value;
        constexpr int EPT = decltype(ept)::value;
        if (L.P.nb == 3) {
            k_batch<3, EPT, BS><<<grid, BS, lds, s>>>(a);
        } else {
            if constexpr (EPT * BS <= 1536 || (EPT <= 2 && BS == 1024)) k_batch<4, EPT, BS><<<grid, BS, lds, s>>>(a);
            else return set_error(FEM_EINVAL, "chunk size too large for tetrahedra");
        }
        return 0;
    });
    if (rc) return rc;
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace fem
