// vec.h -- deterministic nodal-vector reductions shared by the host-driven
// solvers (fcg.hip, iterate.hip).  Each translation unit gets its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.h"

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

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kDotBlocks)); }

}  // namespace
}  // namespace fem
