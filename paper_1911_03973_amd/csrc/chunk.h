// chunk.h -- the element-by-element operator application (Algorithm 1) as a
// chunked, atomic-free gather on gfx950.
//
// Algorithm 1 restricts x to every element (x_e = R_e x), applies the local
// matrix and assembles r = sum_e C_e^T r_e.  Here one workgroup takes a chunk
// of consecutive elements at a time (grid-stride over chunks):
//
//   stage   the chunk's slot list (uint16, grouped by local node) -> LDS
//   phase A node-driven: every local node loads its input value once (a
//           coalesced-ish gather of the chunk's node footprint) and writes it
//           into all its slots                         == restriction R_e x
//   phase B element-driven, one thread per element: the n_b^2 entries of A_e
//           stream in coalesced from the SoA arrays, y = A_e x_e, and y
//           overwrites the element's slots              == local product
//   phase C node-driven: every local node sums its slots in ascending slot
//           order (fixed), complete nodes are finished in place, shared
//           nodes leave a partial                       == assembly C_e^T
//   fix-up  one thread per shared node adds its partials in ascending chunk
//           order.
//
// Every sum therefore has one fixed order: the result is bitwise
// reproducible and no floating-point atomics are used.  The operation-specific
// parts (what is loaded in phase A, what is stored in phase C) are `Op`
// policies; the element-matrix access is a `Ld` policy.
#pragma once

#include "common.h"

namespace fem {

// Matrix access: A(i,j) of element e as type T.
template <int NB, int KIND, class T>
struct LdKM {
    const void *K;
    const void *M;  // nullable
    double nu;
    int64_t ne;
    __device__ __forceinline__ void load(int64_t e, T (&a)[NB * NB]) const {
        const int64_t blk = (int64_t)NB * NB * ne;
#pragma unroll
        for (int ij = 0; ij < NB * NB; ++ij) {
            double v = load_entry<KIND>(K, (int64_t)ij * ne + e, blk);
            if (M) v += nu * load_entry<KIND>(M, (int64_t)ij * ne + e, blk);
            a[ij] = (T)v;
        }
    }
};

// FP32 combined matrix, loaded as float.
template <int NB>
struct LdF32 {
    const float *A;
    int64_t ne;
    __device__ __forceinline__ void load(int64_t e, float (&a)[NB * NB]) const {
#pragma unroll
        for (int ij = 0; ij < NB * NB; ++ij) a[ij] = __builtin_nontemporal_load(A + (int64_t)ij * ne + e);
    }
};

struct ChunkShape {
    int E;           // elements per chunk
    size_t lds;      // dynamic LDS bytes
};

template <int NB, class T>
__host__ __device__ constexpr size_t chunk_lds_bytes(int E) {
    return (size_t)NB * E * sizeof(T) + (size_t)NB * E * sizeof(uint16_t);
}

// DIAG = true: phase A is skipped and phase B yields y_i = A_ii.
template <int NB, class T, class Ld, class Op, bool DIAG>
__global__ __launch_bounds__(kBlock) void k_chunk_main(const DevPlan P, const Ld ld, Op op,
                                                       T *__restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int E = P.E;
    T *buf = reinterpret_cast<T *>(smem);
    uint16_t *sl = reinterpret_cast<uint16_t *>(smem + (size_t)NB * E * sizeof(T));
    __shared__ double red[kBlock / kWave];
    if (!op.begin(red)) return;
    double dacc = 0.0;
    for (int64_t c = blockIdx.x; c < P.n_chunks; c += gridDim.x) {
        const int64_t e0 = c * (int64_t)E;
        const int ne = (int)((P.n_elems - e0) < E ? (P.n_elems - e0) : E);
        const int ns = ne * NB;
        const int nb0 = P.chunk_node_off[c];
        const int nl = P.chunk_node_off[c + 1] - nb0;
        const int ncomp = P.chunk_info[2 * c];
        const int pbase = P.chunk_info[2 * c + 1];
        __syncthreads();  // the previous chunk's phase C is done with buf / sl
        {
            // slot list -> LDS, 16-byte vectors (n_b*E*2 bytes is a multiple of 16)
            const uint4 *src = reinterpret_cast<const uint4 *>(P.slots + c * (int64_t)NB * E);
            uint4 *dst = reinterpret_cast<uint4 *>(sl);
            const int nv = (ns + 7) >> 3;
            for (int k = threadIdx.x; k < nv; k += kBlock) dst[k] = src[k];
        }
        __syncthreads();
        if constexpr (!DIAG) {
            for (int k = threadIdx.x; k < nl; k += kBlock) {
                const int g = P.loc_nodes[nb0 + k];
                const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
                const int s1 = P.loc_end[nb0 + k];
                const T v = op.gather(g, k < ncomp);
                for (int s = s0; s < s1; ++s) buf[sl[s]] = v;
            }
            __syncthreads();
        }
        for (int le = threadIdx.x; le < ne; le += kBlock) {
            T a[NB * NB];
            ld.load(e0 + le, a);
            T y[NB];
            if constexpr (DIAG) {
#pragma unroll
                for (int i = 0; i < NB; ++i) y[i] = a[i * NB + i];
            } else {
                T xe[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) xe[j] = buf[le * NB + j];
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    T s = a[i * NB] * xe[0];
#pragma unroll
                    for (int j = 1; j < NB; ++j) s += a[i * NB + j] * xe[j];
                    y[i] = s;
                }
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) buf[le * NB + i] = y[i];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nl; k += kBlock) {
            const int s0 = k ? P.loc_end[nb0 + k - 1] : 0;
            const int s1 = P.loc_end[nb0 + k];
            T acc = (T)0;
            for (int s = s0; s < s1; ++s) acc += buf[sl[s]];
            if (k < ncomp) dacc += op.finish(P.loc_nodes[nb0 + k], acc);
            else partial[pbase + (k - ncomp)] = acc;
        }
    }
    op.end(dacc, red);
}

template <class T, class Op>
__global__ __launch_bounds__(kBlock) void k_chunk_fixup(const DevPlan P, Op op, const T *__restrict__ partial) {
    __shared__ double red[kBlock / kWave];
    if (!op.begin_fixup(red)) return;
    double dacc = 0.0;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < P.n_shared; s += (int64_t)gridDim.x * kBlock) {
        const int g = P.fix_nodes[s];
        const int k0 = P.fix_off[s], k1 = P.fix_off[s + 1];
        T acc = (T)0;
        for (int k = k0; k < k1; ++k) acc += partial[P.fix_parts[k]];
        op.gather_shared(g);
        dacc += op.finish(g, acc);
    }
    op.end_fixup(dacc, red);
}

}  // namespace fem
