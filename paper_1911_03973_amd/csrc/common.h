// common.h -- shared device helpers of libfem (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "plan.h"

namespace fem {

constexpr int kBlock = 256;  // 4 wave64 per workgroup
constexpr int kWave = 64;

// MAT_MF: no stored element matrices, K_e and M_e rebuilt from the
// coordinates inside every element pass (matrix-free).
enum MatKind { MAT_F64 = 0, MAT_F32 = 1, MAT_F32X2 = 2, MAT_MF = 3 };

// Element-matrix entry (i*nb+j) of element e, promoted to double.
// `blk` is the size of one [nb*nb][n_elems] block (for the lo half of a pair).
template <int KIND>
__device__ __forceinline__ double load_entry(const void *base, int64_t idx, int64_t blk) {
    if constexpr (KIND == MAT_F64) {
        return __builtin_nontemporal_load(static_cast<const double *>(base) + idx);
    } else if constexpr (KIND == MAT_F32) {
        return (double)__builtin_nontemporal_load(static_cast<const float *>(base) + idx);
    } else {
        const float *p = static_cast<const float *>(base);
        return (double)__builtin_nontemporal_load(p + idx) + (double)__builtin_nontemporal_load(p + idx + blk);
    }
}

// Deterministic wave64 sum: fixed xor butterfly, every lane ends with the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Deterministic block sum of one value per thread (blockDim == BS).
// Every thread receives the same total.  `red` must hold BS/64 doubles.
template <int BS = kBlock>
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < BS / kWave; ++k) t += red[k];
    return t;
}

// N block sums at once (one LDS exchange).  `red` must hold N*BS/64 doubles.
template <int BS, int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double *red) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int j = 0; j < N; ++j) red[j * (BS / kWave) + w] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < BS / kWave; ++k) t += red[j * (BS / kWave) + k];
        v[j] = t;
    }
}

// Sum n partials (fixed assignment and order; identical result in every block).
template <int BS = kBlock>
__device__ __forceinline__ double reduce_partials(const double *part, int n, double *red) {
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += BS) v += part[k];
    return block_sum<BS>(v, red);
}

std::string &last_error();
int set_error(int code, const std::string &msg);

}  // namespace fem

#define FEM_HIP_CHECK(expr)                                                                  \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return ::fem::set_error(-2, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
    } while (0)
