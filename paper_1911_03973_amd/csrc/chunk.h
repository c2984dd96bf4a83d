// chunk.h -- the element-by-element operator application (Algorithm 1) as a
// chunked, atomic-free gather on gfx950.
//
// Algorithm 1 restricts x to every element (x_e = R_e x), applies the local
// matrix and assembles r = sum_e C_e^T r_e.  Here one workgroup takes a chunk
// of E consecutive elements at a time (grid-stride over chunks):
//
//   fetch   the E elements' matrix values are requested first, straight into
//           registers (EPT = E/256 elements per thread), so their HBM latency
//           overlaps the rest of the pass
//   stage   the chunk's slot list (uint16, grouped by local node) -> LDS
//   phase A node-driven: every local node loads its input value once and
//           writes it into all its slots                == restriction R_e x
//   phase B element-driven: y = A_e x_e from registers; y overwrites the
//           element's slots                              == local product
//   phase C node-driven: every local node sums its slots in ascending slot
//           order (fixed); nodes of this chunk only are finished in place,
//           shared nodes leave a partial                 == assembly C_e^T
//   fix-up  one thread per shared node adds its partials in ascending chunk
//           order.  Ops may keep the values of shared nodes in compact
//           arrays indexed by the shared-node number (phase A passes it).
//
// Every sum has one fixed order: results are bitwise reproducible and no
// floating-point atomics are used.  Chunks are dealt to workgroups so that
// each of the 8 XCDs (workgroup i runs on XCD i mod 8) walks a contiguous
// range of chunks: neighbouring chunks share halo nodes, which then hit the
// same L2.  What is loaded in phase A and stored in phase C is an `Op`
// policy; the element matrix is an `Ld` policy.
#pragma once

#include <type_traits>

#include "common.h"

namespace fem {

// ---------------------------------------------------------------------------
// Element matrix policies.  fetch() issues the loads of element e into a
// register record; apply() computes y = A_e x_e; diag() returns (A_e)_ii.
// ---------------------------------------------------------------------------

// Full n_b x n_b storage, A_e = K_e + nu M_e combined at fetch time.
template <int NB, int KIND, class T>
struct LdKM {
    const void *K;
    const void *M;  // nullable
    double nu;
    int64_t ne;
    struct Regs {
        T a[NB * NB];
    };
    __device__ __forceinline__ void fetch(int64_t e, Regs &R) const {
        const int64_t blk = (int64_t)NB * NB * ne;
#pragma unroll
        for (int ij = 0; ij < NB * NB; ++ij) {
            double v = load_entry<KIND>(K, (int64_t)ij * ne + e, blk);
            if (M) v += nu * load_entry<KIND>(M, (int64_t)ij * ne + e, blk);
            R.a[ij] = (T)v;
        }
    }
    __device__ __forceinline__ static void apply(const Regs &R, const T (&x)[NB], T (&y)[NB]) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            T s = R.a[i * NB] * x[0];
#pragma unroll
            for (int j = 1; j < NB; ++j) s += R.a[i * NB + j] * x[j];
            y[i] = s;
        }
    }
    __device__ __forceinline__ static void diag(const Regs &R, T (&y)[NB]) {
#pragma unroll
        for (int i = 0; i < NB; ++i) y[i] = R.a[i * NB + i];
    }
};

// FP32 combined full storage, FP32 arithmetic.
template <int NB>
struct LdF32 {
    const float *A;
    int64_t ne;
    struct Regs {
        float a[NB * NB];
    };
    __device__ __forceinline__ void fetch(int64_t e, Regs &R) const {
#pragma unroll
        for (int ij = 0; ij < NB * NB; ++ij) R.a[ij] = __builtin_nontemporal_load(A + (int64_t)ij * ne + e);
    }
    __device__ __forceinline__ static void apply(const Regs &R, const float (&x)[NB], float (&y)[NB]) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            float s = R.a[i * NB] * x[0];
#pragma unroll
            for (int j = 1; j < NB; ++j) s += R.a[i * NB + j] * x[j];
            y[i] = s;
        }
    }
    __device__ __forceinline__ static void diag(const Regs &R, float (&y)[NB]) {
#pragma unroll
        for (int i = 0; i < NB; ++i) y[i] = R.a[i * NB + i];
    }
};

// Packed symmetric difference form of A_e (see solver.h, packed_count):
// values 0..NB-1 are the row sums rho_i = sum_j (A_e)_ij, then the upper
// off-diagonal entries a_ij (i < j) row by row, and
//   (A_e x)_i = rho_i x_i + sum_{j != i} a_ij (x_j - x_i),
// evaluated in FP64.  For a matrix with zero row sums (a stiffness matrix)
// the rounding error then scales with the differences x_j - x_i rather than
// with x itself, which keeps an FP32-stored operator accurate on smooth
// vectors.  KIND: MAT_F64 (double values), MAT_F32 (float; the head of a
// hi/lo pair) or MAT_F32X2 (hi + lo).
template <int NB, int KIND>
struct LdPk {
    static constexpr int NP = NB + NB * (NB - 1) / 2;
    using V = typename std::conditional<KIND == MAT_F32, float, double>::type;
    const void *A;
    int64_t ne;
    struct Regs {
        V v[NP];
    };
    __device__ __forceinline__ void fetch(int64_t e, Regs &R) const {
        const int64_t blk = (int64_t)NP * ne;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if constexpr (KIND == MAT_F32)
                R.v[k] = __builtin_nontemporal_load(static_cast<const float *>(A) + (int64_t)k * ne + e);
            else
                R.v[k] = load_entry<KIND>(A, (int64_t)k * ne + e, blk);
        }
    }
    template <class T>
    __device__ __forceinline__ static void apply(const Regs &R, const T (&xt)[NB], T (&yt)[NB]) {
        double x[NB], y[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            x[i] = (double)xt[i];
            y[i] = (double)R.v[i] * x[i];
        }
        int k = NB;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) {
                const double t = (double)R.v[k++] * (x[j] - x[i]);
                y[i] += t;
                y[j] -= t;
            }
#pragma unroll
        for (int i = 0; i < NB; ++i) yt[i] = (T)y[i];
    }
    template <class T>
    __device__ __forceinline__ static void diag(const Regs &R, T (&yt)[NB]) {
        double y[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) y[i] = (double)R.v[i];
        int k = NB;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) {
                y[i] -= (double)R.v[k];
                y[j] -= (double)R.v[k];
                ++k;
            }
#pragma unroll
        for (int i = 0; i < NB; ++i) yt[i] = (T)y[i];
    }
};

template <int NB, class T>
__host__ __device__ constexpr size_t chunk_lds_bytes(int E) {
    return (size_t)NB * E * sizeof(T) + (size_t)NB * E * sizeof(uint16_t);
}

// Matrix-free operator: the vectorized assembly of Section 1 (eq. (2) per
// element) moved into the element pass.  The packed difference form of
// A_e = kk K_e + nu M_e is rebuilt in registers from the element's vertex
// coordinates on every pass, so no element array is read; the arithmetic is
// FP64.  With the edge vectors e_k = p_k - p_0 and det = det[e_1 .. e_d], the
// scaled barycentric gradients c_k = det grad(lambda_k) are the rows of the
// adjugate (2D: c_1 = (e2y, -e2x), c_2 = (-e1y, e1x); 3D: c_1 = e2 x e3,
// c_2 = e3 x e1, c_3 = e1 x e2) and c_0 = -(c_1 + ... + c_d).  Then
// K_ij = (c_i . c_j) / (d! |det|) (vol = |det| / d!), the row sums of K_e are
// 0, M_e has vol / ((d+1)(d+2)) off the diagonal and row sums vol / (d+1).
// Vertex coordinates reach the pass through LDS: phase A stores each local
// node's coordinates once (a per-chunk table of max_local entries) and the
// node's index into a 4-entry record per element; phase B reads the record
// with one 8-byte load and the vertices through it.  Measured alternatives, all slower or no faster:
// the coordinates written into every slot beside x (1.2x slower in 2D, 2x in
// 3D: phase A's scattered LDS writes tripled), and a precomputed slot -> node
// index read from HBM into registers or staged into LDS.
template <int NB>
struct LdMf {
    static constexpr bool kCoords = true;
    static constexpr int DIM = NB - 1;
    using Base = LdPk<NB, MAT_F64>;
    using Regs = typename Base::Regs;
    const double *xyz;  // [DIM][n] coordinates, indexed like the op's nodes
    int64_t n;
    double kk, nu;
    __device__ __forceinline__ void fetch(int64_t, Regs &) const {}
    __device__ __forceinline__ double coord(int64_t i, int d) const { return xyz[(int64_t)d * n + i]; }
    __device__ __forceinline__ void build(const double (&p)[NB][DIM], Regs &R) const {
        double c[NB][DIM];
        double det;
        if constexpr (DIM == 2) {
            const double e1x = p[1][0] - p[0][0], e1y = p[1][1] - p[0][1];
            const double e2x = p[2][0] - p[0][0], e2y = p[2][1] - p[0][1];
            det = e1x * e2y - e1y * e2x;
            c[1][0] = e2y;
            c[1][1] = -e2x;
            c[2][0] = -e1y;
            c[2][1] = e1x;
        } else {
            double e[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) e[k][d] = p[k + 1][d] - p[0][d];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double *a = e[(k + 1) % 3], *b = e[(k + 2) % 3];
                c[k + 1][0] = a[1] * b[2] - a[2] * b[1];
                c[k + 1][1] = a[2] * b[0] - a[0] * b[2];
                c[k + 1][2] = a[0] * b[1] - a[1] * b[0];
            }
            det = e[0][0] * c[1][0] + e[0][1] * c[1][1] + e[0][2] * c[1][2];
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double t = 0.0;
#pragma unroll
            for (int k = 1; k < NB; ++k) t += c[k][d];
            c[0][d] = -t;
        }
        const double fact = DIM == 2 ? 2.0 : 6.0;
        const double ad = fabs(det);
        const double vol = ad / fact;
        const double ks = kk / (fact * ad);
        const double moff = nu * vol / (double)((DIM + 1) * (DIM + 2));
        const double mrow = nu * vol / (double)(DIM + 1);
#pragma unroll
        for (int i = 0; i < NB; ++i) R.v[i] = mrow;
        int k = NB;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) {
                double g = 0.0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) g += c[i][d] * c[j][d];
                R.v[k++] = ks * g + moff;
            }
    }
    template <class T>
    __device__ __forceinline__ static void apply(const Regs &R, const T (&xt)[NB], T (&yt)[NB]) {
        Base::apply(R, xt, yt);
    }
    template <class T>
    __device__ __forceinline__ static void diag(const Regs &R, T (&yt)[NB]) {
        Base::diag(R, yt);
    }
};

// Loaders without kCoords read their element arrays from HBM.
template <class L, class = void>
struct HasCoords : std::false_type {};
template <class L>
struct HasCoords<L, std::void_t<decltype(L::kCoords)>> : std::integral_constant<bool, L::kCoords> {};

// LDS of one chunk pass: slot buffer and slot list, plus (matrix-free) the
// slot -> local node index and the coordinates of up to max_local nodes.
template <int NB, class T, class Ld>
size_t chunk_lds_for(const DevPlan &P) {
    size_t b = chunk_lds_bytes<NB, T>(P.E);
    if constexpr (HasCoords<Ld>::value)
        b += (size_t)4 * P.E * sizeof(uint16_t) + (size_t)(NB - 1) * sizeof(double) * (size_t)P.max_local;
    return b;
}

// Chunk visited by workgroup b at its it-th step, or -1 when done.  With
// xcd != 0 (grid a multiple of 8) XCD b%8 walks chunks [x*cpx, (x+1)*cpx).
__device__ __forceinline__ int64_t chunk_of(int64_t b, int64_t it, int64_t n_chunks, int64_t grid, int xcd) {
    if (!xcd) {
        const int64_t c = b + it * grid;
        return c < n_chunks ? c : -1;
    }
    const int64_t cpx = (n_chunks + 7) / 8;
    const int64_t bpx = grid / 8;
    const int64_t j = (b >> 3) + it * bpx;
    if (j >= cpx) return -1;
    const int64_t c = (b & 7) * cpx + j;
    return c < n_chunks ? c : -1;
}

// Stage the chunk's slot list (16-byte aligned, padded to n_b*E) into LDS.
__device__ __forceinline__ void stage_slots(const uint16_t *__restrict__ src_u16, uint16_t *sl, int ns) {
    const uint4 *src = reinterpret_cast<const uint4 *>(src_u16);
    uint4 *dst = reinterpret_cast<uint4 *>(sl);
    const int nv = (ns + 7) >> 3;
    for (int k = threadIdx.x; k < nv; k += kBlock) dst[k] = src[k];
}

// Shared scratch of the chunk kernels for block reductions (up to 8 sums).
template <int BS>
struct RedBuf {
    double v[8 * (BS / kWave)];
};

// Elements [e0, e0 + ne) of chunk c.
__device__ __forceinline__ void chunk_range(const DevPlan &P, int64_t c, int64_t &e0, int &ne) {
    if (P.chunk_elem0) {
        e0 = P.chunk_elem0[c];
        ne = (int)(P.chunk_elem0[c + 1] - e0);
    } else {
        e0 = c * (int64_t)P.E;
        ne = (int)((P.n_elems - e0) < P.E ? (P.n_elems - e0) : P.E);
    }
}

// One pass of the workgroup over chunk c (fetch, stage, phases A-C).  buf /
// sl are the dynamic LDS areas.  The element-matrix loads are issued first;
// the barrier after them waits until no thread still reads buf / sl for the
// previous chunk, so the load latency overlaps that wait.
template <int NB, int EPT, int BS, class T, class Ld, class Op, bool DIAG>
__device__ __forceinline__ void chunk_pass(const DevPlan &P, const Ld &ld, Op &op, T *__restrict__ partial,
                                           int64_t c, T *buf, uint16_t *sl) {
    int64_t e0;
    int ne;
    chunk_range(P, c, e0, ne);
    typename Ld::Regs R[EPT];
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int le = t * BS + threadIdx.x;
        if (le < ne) ld.fetch(e0 + le, R[t]);
    }
    __syncthreads();
    const int nb0 = P.chunk_node_off[c];
    const int nl = P.chunk_node_off[c + 1] - nb0;
    const int ncomp = P.chunk_info[2 * c];
    const int pbase = P.chunk_info[2 * c + 1];
    const int coff = Op::kLocal ? P.comp_off[c] : 0;
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.slots + c * (int64_t)NB * P.E);
        uint4 *dst = reinterpret_cast<uint4 *>(sl);
        const int nv = (ne * NB + 7) >> 3;
        for (int k = threadIdx.x; k < nv; k += BS) dst[k] = src[k];
    }
    __syncthreads();
    if constexpr (!DIAG) {
        for (int k = threadIdx.x; k < nl; k += BS) {
            const int g = Op::kLocal ? (k < ncomp ? coff + k : -1) : P.loc_nodes[nb0 + k];
            const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
            const int s1 = P.loc_end[nb0 + k];
            const T v = op.gather(g, k < ncomp ? -1 : P.part_owner[pbase + (k - ncomp)]);
            for (int s = s0; s < s1; ++s) buf[sl[s]] = v;
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int le = t * BS + threadIdx.x;
        if (le < ne) {
            T y[NB];
            if constexpr (DIAG) {
                Ld::diag(R[t], y);
            } else {
                T xe[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) xe[j] = buf[le * NB + j];
                Ld::apply(R[t], xe, y);
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) buf[le * NB + i] = y[i];
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nl; k += BS) {
        const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
        const int s1 = P.loc_end[nb0 + k];
        T acc = (T)0;
        for (int s = s0; s < s1; ++s) acc += buf[sl[s]];
        if (k < ncomp) op.finish(Op::kLocal ? coff + k : P.loc_nodes[nb0 + k], acc);
        else partial[pbase + (k - ncomp)] = acc;
    }
}

// One workgroup of BS threads walks chunks of E = P.E elements; each thread
// owns EPT = ceil(E / BS) element slots.  DIAG = true: phase A is skipped
// and phase B yields y_i = A_ii.  The chunk body is chunk_pass written out:
// handing the kernel-argument Op to that helper by reference costs the CG
// pass 25 more VGPRs (81 -> 106, occupancy 5 -> 4 waves per SIMD).
template <int NB, int EPT, int BS, class T, class Ld, class Op, bool DIAG>
__global__ __launch_bounds__(BS) void k_chunk_main(const DevPlan P, const Ld ld, Op op, T *__restrict__ partial,
                                                   int xcd) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *buf = reinterpret_cast<T *>(smem);
    uint16_t *sl = reinterpret_cast<uint16_t *>(smem + (size_t)NB * P.E * sizeof(T));
    constexpr bool kMf = HasCoords<Ld>::value;
    // matrix-free only: element le's local nodes at lnode[4 le + j] (one 8-byte
    // LDS read per element), then the coordinates of the chunk's local nodes,
    // [local node][dim]
    static_assert(!kMf || NB <= 4, "the matrix-free record holds four vertices");
    uint16_t *lnode = sl + (size_t)NB * P.E;
    double *crd = reinterpret_cast<double *>(lnode + (size_t)4 * P.E);
    __shared__ RedBuf<BS> red;
    if (!op.begin()) return;
    for (int64_t it = 0;; ++it) {
        const int64_t c = chunk_of(blockIdx.x, it, P.n_chunks, gridDim.x, xcd);
        if (c < 0) break;
        int64_t e0;
        int ne;
        chunk_range(P, c, e0, ne);
        typename Ld::Regs R[EPT];
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int le = t * BS + threadIdx.x;
            if (le < ne) ld.fetch(e0 + le, R[t]);
        }
        const int nb0 = P.chunk_node_off[c];
        const int nl = P.chunk_node_off[c + 1] - nb0;
        const int ncomp = P.chunk_info[2 * c];
        const int pbase = P.chunk_info[2 * c + 1];
        const int coff = Op::kLocal ? P.comp_off[c] : 0;
        __syncthreads();  // the previous chunk's phase C is done with buf / sl
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(P.slots + c * (int64_t)NB * P.E);
            uint4 *dst = reinterpret_cast<uint4 *>(sl);
            const int nv = (ne * NB + 7) >> 3;
            for (int k = threadIdx.x; k < nv; k += BS) dst[k] = src[k];
        }
        __syncthreads();
        if constexpr (kMf) {
            for (int k = threadIdx.x; k < nl; k += BS) {
                const int g = Op::kLocal ? (k < ncomp ? coff + k : -1) : P.loc_nodes[nb0 + k];
                const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
                const int s1 = P.loc_end[nb0 + k];
                const int own = k < ncomp ? -1 : P.part_owner[pbase + (k - ncomp)];
                if constexpr (!DIAG) {
                    const T v = op.gather(g, own);
                    for (int s = s0; s < s1; ++s) buf[sl[s]] = v;
                }
                // the coordinates in the op's node order: shared nodes of a
                // solver-local op follow the complete ones by shared index
                const int64_t ci = (Op::kLocal && own >= 0) ? (P.n_nodes - P.n_shared) + own : (int64_t)g;
#pragma unroll
                for (int d = 0; d < NB - 1; ++d) crd[k * (NB - 1) + d] = ld.coord(ci, d);
                for (int s = s0; s < s1; ++s) {
                    const int q = sl[s];  // slot = le * NB + j
                    lnode[(q / NB) * 4 + q % NB] = (uint16_t)k;
                }
            }
            __syncthreads();
        } else if constexpr (!DIAG) {
            for (int k = threadIdx.x; k < nl; k += BS) {
                // Op::kLocal: complete nodes by solver-local index, shared ones by their shared index only
                const int g = Op::kLocal ? (k < ncomp ? coff + k : -1) : P.loc_nodes[nb0 + k];
                const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
                const int s1 = P.loc_end[nb0 + k];
                const T v = op.gather(g, k < ncomp ? -1 : P.part_owner[pbase + (k - ncomp)]);
                for (int s = s0; s < s1; ++s) buf[sl[s]] = v;
            }
            __syncthreads();
        }
        if constexpr (kMf) {
            // all of the thread's elements first: these LDS reads do not wait
            // behind the slot-buffer writes of the loop below
#pragma unroll
            for (int t = 0; t < EPT; ++t) {
                const int le = t * BS + threadIdx.x;
                if (le < ne) {
                    const uint2 ln4 = *reinterpret_cast<const uint2 *>(lnode + 4 * le);
                    const int kn[4] = {(int)(ln4.x & 0xFFFFu), (int)(ln4.x >> 16), (int)(ln4.y & 0xFFFFu),
                                       (int)(ln4.y >> 16)};
                    double pv[NB][NB - 1];
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int d = 0; d < NB - 1; ++d) pv[j][d] = crd[kn[j] * (NB - 1) + d];
                    ld.build(pv, R[t]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int le = t * BS + threadIdx.x;
            if (le < ne) {
                T y[NB];
                if constexpr (DIAG) {
                    Ld::diag(R[t], y);
                } else {
                    T xe[NB];
#pragma unroll
                    for (int j = 0; j < NB; ++j) xe[j] = buf[le * NB + j];
                    Ld::apply(R[t], xe, y);
                }
#pragma unroll
                for (int i = 0; i < NB; ++i) buf[le * NB + i] = y[i];
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nl; k += BS) {
            const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
            const int s1 = P.loc_end[nb0 + k];
            T acc = (T)0;
            for (int s = s0; s < s1; ++s) acc += buf[sl[s]];
            if (k < ncomp) op.finish(Op::kLocal ? coff + k : P.loc_nodes[nb0 + k], acc);
            else partial[pbase + (k - ncomp)] = acc;
        }
    }
    op.template end<BS>(red.v, blockIdx.x);
}

// Chunk pass of ops that gather and finish by mesh node id (Op::kLocal
// false; DIAG false): each thread keeps the node id, slot run and input
// value of its first KN local nodes in registers, loaded right after the
// element-matrix fetch and before the workgroup barrier, and requests the
// op's finishing operands (fixup_load) before the barrier ahead of phase C,
// so neither phase waits on a chain of dependent global loads.  Nodes beyond
// KN * BS take the plain path.
template <int NB, int EPT, int BS, int KN, class T, class Ld, class Op>
__global__ __launch_bounds__(BS) void k_chunk_affine(const DevPlan P, const Ld ld, Op op, T *__restrict__ partial,
                                                     int xcd) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *buf = reinterpret_cast<T *>(smem);
    uint16_t *sl = reinterpret_cast<uint16_t *>(smem + (size_t)NB * P.E * sizeof(T));
    for (int64_t it = 0;; ++it) {
        const int64_t c = chunk_of(blockIdx.x, it, P.n_chunks, gridDim.x, xcd);
        if (c < 0) break;
        int64_t e0;
        int ne;
        chunk_range(P, c, e0, ne);
        typename Ld::Regs R[EPT];
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int le = t * BS + threadIdx.x;
            if (le < ne) ld.fetch(e0 + le, R[t]);
        }
        const int nb0 = P.chunk_node_off[c];
        const int nl = P.chunk_node_off[c + 1] - nb0;
        const int ncomp = P.chunk_info[2 * c];
        const int pbase = P.chunk_info[2 * c + 1];
        int gk[KN];
        unsigned run[KN];  // slot run [low 16 bits, high 16 bits)
#pragma unroll
        for (int j = 0; j < KN; ++j) {
            const int k = threadIdx.x + j * BS;
            gk[j] = 0;
            run[j] = 0;
            if (k < nl) {
                gk[j] = P.loc_nodes[nb0 + k];
                run[j] = (k ? (unsigned)P.loc_end[nb0 + k - 1] : 0u) | ((unsigned)P.loc_end[nb0 + k] << 16);
            }
        }
        T xk[KN];
#pragma unroll
        for (int j = 0; j < KN; ++j) {
            const int k = threadIdx.x + j * BS;
            if (k < nl) xk[j] = op.gather(gk[j], -1);
        }
        __syncthreads();  // the previous chunk's phase C is done with buf / sl
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(P.slots + c * (int64_t)NB * P.E);
            uint4 *dst = reinterpret_cast<uint4 *>(sl);
            const int nv = (ne * NB + 7) >> 3;
            for (int k = threadIdx.x; k < nv; k += BS) dst[k] = src[k];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KN; ++j) {
            const int k = threadIdx.x + j * BS;
            if (k < nl)
                for (int s = (int)(run[j] & 0xFFFFu); s < (int)(run[j] >> 16); ++s) buf[sl[s]] = xk[j];
        }
        for (int k = threadIdx.x + KN * BS; k < nl; k += BS) {
            const int s0 = P.loc_end[nb0 + k - 1], s1 = P.loc_end[nb0 + k];
            const T v = op.gather(P.loc_nodes[nb0 + k], -1);
            for (int s = s0; s < s1; ++s) buf[sl[s]] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int le = t * BS + threadIdx.x;
            if (le < ne) {
                T xe[NB], y[NB];
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) xe[jj] = buf[le * NB + jj];
                Ld::apply(R[t], xe, y);
#pragma unroll
                for (int i = 0; i < NB; ++i) buf[le * NB + i] = y[i];
            }
        }
        typename Op::Pre pk[KN];  // requested before the barrier: its latency overlaps the wait
#pragma unroll
        for (int j = 0; j < KN; ++j) {
            const int k = threadIdx.x + j * BS;
            if (k < ncomp) pk[j] = op.fixup_load(-1, gk[j]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KN; ++j) {
            const int k = threadIdx.x + j * BS;
            if (k < nl) {
                T acc = (T)0;
                for (int s = (int)(run[j] & 0xFFFFu); s < (int)(run[j] >> 16); ++s) acc += buf[sl[s]];
                if (k < ncomp) op.fixup_store(-1, gk[j], pk[j], acc);
                else partial[pbase + (k - ncomp)] = acc;
            }
        }
        for (int k = threadIdx.x + KN * BS; k < nl; k += BS) {
            const int s0 = P.loc_end[nb0 + k - 1], s1 = P.loc_end[nb0 + k];
            T acc = (T)0;
            for (int s = s0; s < s1; ++s) acc += buf[sl[s]];
            if (k < ncomp) op.finish(P.loc_nodes[nb0 + k], acc);
            else partial[pbase + (k - ncomp)] = acc;
        }
    }
}

// Partials of shared node s added in ascending chunk order; the slots come
// from one 16-byte record (DevPlan::fix_rec), longer lists continue in
// fix_parts.
template <class T>
__device__ __forceinline__ T fix_sum(const DevPlan &P, const T *__restrict__ partial, int64_t s) {
    T acc = (T)0;
    if (P.fix_rec) {
        const int4 rc = reinterpret_cast<const int4 *>(P.fix_rec)[s];
        if (rc.x >= 0) acc += partial[rc.x];
        if (rc.y >= 0) acc += partial[rc.y];
        if (rc.z >= 0) acc += partial[rc.z];
        if (rc.w >= 0) {
            acc += partial[rc.w];
        } else if (rc.w < -1) {
            const int k1 = P.fix_off[s + 1];
            for (int k = -2 - rc.w; k < k1; ++k) acc += partial[P.fix_parts[k]];
        }
    } else {
        const int k0 = P.fix_off[s], k1 = P.fix_off[s + 1];
        for (int k = k0; k < k1; ++k) acc += partial[P.fix_parts[k]];
    }
    return acc;
}

// Ops whose fix-up workgroups start with extra work (OpIter: a share of the
// element pass's dot partials) define fixup_begin(block, n_blocks).
template <class Op, class = void>
struct HasFixupBegin : std::false_type {};
template <class Op>
struct HasFixupBegin<Op, std::void_t<decltype(&Op::fixup_begin)>> : std::true_type {};

// Shared nodes: each thread finishes two nodes, BS apart, with the op's own
// loads (fixup_load) and the partial loads of both issued before either node
// is stored, so a node costs two dependent memory round trips and every
// thread has both nodes' loads in flight.  Dot-product partials of this
// kernel go to slot_base + block.
template <int BS, class T, class Op>
__global__ __launch_bounds__(BS) void k_chunk_fixup(const DevPlan P, Op op, const T *__restrict__ partial,
                                                    int slot_base) {
    __shared__ RedBuf<BS> red;
    if (!op.begin()) return;
    if constexpr (HasFixupBegin<Op>::value) op.fixup_begin(blockIdx.x, gridDim.x);
    const int64_t step = (int64_t)gridDim.x * 2 * BS;
    for (int64_t sa = (int64_t)blockIdx.x * 2 * BS + threadIdx.x; sa < P.n_shared; sa += step) {
        const int64_t sb = sa + BS;
        const bool hb = sb < P.n_shared;
        const int ga = Op::kLocal ? -1 : P.fix_nodes[sa];
        const int gb = (Op::kLocal || !hb) ? -1 : P.fix_nodes[sb];
        const typename Op::Pre pa = op.fixup_load((int)sa, ga);
        typename Op::Pre pb{};
        if (hb) pb = op.fixup_load((int)sb, gb);
        const T aa = fix_sum(P, partial, sa);
        const T ab = hb ? fix_sum(P, partial, sb) : (T)0;
        op.fixup_store((int)sa, ga, pa, aa);
        if (hb) op.fixup_store((int)sb, gb, pb, ab);
    }
    op.template end<BS>(red.v, slot_base + blockIdx.x);
}

// Grid of the chunk kernels: enough workgroups to fill every CU at the
// occupancy the LDS footprint allows (at most 2048 threads per CU), a
// multiple of 8 when possible (XCD-aware chunk order), never more than
// there are chunks.
struct ChunkGrid {
    int grid;
    int xcd;
};

ChunkGrid chunk_grid(int64_t n_chunks, size_t lds, int bs = kBlock);

// Fix-up launches: kFixBlock threads, two shared nodes each, grid-stride
// beyond `cap` workgroups.  Passes that leave one dot-product partial per
// workgroup cap the grid at kFixDotsCap, so that the single-workgroup
// finalize has few partials to add.
constexpr int kFixBlock = 256;
constexpr int kFixDotsCap = 1024;
inline int fixup_grid(int64_t n_shared, int cap = 16384) {
    int64_t g = (n_shared + 2 * kFixBlock - 1) / (2 * kFixBlock);
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// Calls f(std::integral_constant<int, EPT>) for the plan's chunk size and a
// block of 256 threads.
template <class F>
int dispatch_ept(int E, F &&f) {
    switch (E) {
        case 64:
        case 128:
        case 256: return f(std::integral_constant<int, 1>());
        case 512: return f(std::integral_constant<int, 2>());
        case 1024: return f(std::integral_constant<int, 4>());
        case 1536: return f(std::integral_constant<int, 6>());
        case 2048: return f(std::integral_constant<int, 8>());
        default: return set_error(-1, "unsupported chunk size");
    }
}

// Calls f(integral_constant<NB>) for the element sizes the library runs:
// linear triangles (3), linear tetrahedra (4), quadratic triangles (6) and
// quadratic tetrahedra (10).
template <class F>
int dispatch_nb(int nb, F &&f) {
    switch (nb) {
        case 3: return f(std::integral_constant<int, 3>());
        case 4: return f(std::integral_constant<int, 4>());
        case 6: return f(std::integral_constant<int, 6>());
        case 10: return f(std::integral_constant<int, 10>());
        default: return set_error(-1, "unsupported element size");
    }
}

// Calls f(integral_constant<BS>, integral_constant<EPT>) for a chunk size E
// and a workgroup size BS in {256, 512, 1024} (EPT = ceil(E / BS)).
template <class F>
int dispatch_tile(int E, int BS, F &&f) {
    using std::integral_constant;
    if (BS == 256) return dispatch_ept(E, [&](auto ept) { return f(integral_constant<int, 256>(), ept); });
    if (BS == 512) {
        switch (E) {
            case 64: case 128: case 256: case 512: return f(integral_constant<int, 512>(), integral_constant<int, 1>());
            case 1024: return f(integral_constant<int, 512>(), integral_constant<int, 2>());
            case 1536: return f(integral_constant<int, 512>(), integral_constant<int, 3>());
            case 2048: return f(integral_constant<int, 512>(), integral_constant<int, 4>());
            default: break;
        }
    }
    if (BS == 1024) {
        switch (E) {
            case 64: case 128: case 256: case 512: case 1024:
                return f(integral_constant<int, 1024>(), integral_constant<int, 1>());
            case 1536: case 2048: return f(integral_constant<int, 1024>(), integral_constant<int, 2>());
            default: break;
        }
    }
    return set_error(-1, "unsupported chunk size / workgroup size");
}

}  // namespace fem
