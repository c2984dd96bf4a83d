// vec.h -- deterministic nodal-vector reductions and updates shared by the
// host-driven solvers (fcg.hip, iterate.hip, mg.hip).  Each translation unit
// gets its own copy.
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

// out[j] = sum_b part[b][j], one workgroup of kBlock threads: thread t adds
// blocks t, t + kBlock, ... in order, then a fixed-order block sum (a serial
// sum over 512 partials took 45 us per call)
__global__ __launch_bounds__(kBlock) void k_dots_fin(const double *__restrict__ part, int blocks, int nv,
                                                     double *__restrict__ out) {
    __shared__ double red[kBlock / kWave];
    for (int j = 0; j < nv; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < blocks; b += kBlock) v += part[(int64_t)b * nv + j];
        v = block_sum<kBlock>(v, red);
        if (threadIdx.x == 0) out[j] = v;
    }
}

// D^-1, 0 on Dirichlet nodes; *bad = 1 if a free node has d <= 0
__global__ void k_dinv_fcg(int64_t n, const double *__restrict__ d, const uint8_t *__restrict__ mask,
                           double *__restrict__ dinv, int *__restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double v = 0.0;
        if (!mask[i]) {
            if (!(d[i] > 0.0)) *bad = 1;
            v = 1.0 / d[i];
        }
        dinv[i] = v;
    }
}

// p = z - beta p
__global__ void k_dir(int64_t n, const double *__restrict__ z, double beta, double *__restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = z[i] - beta * p[i];
}

// x += alpha p, r -= alpha q; partial r.r per block
__global__ __launch_bounds__(kBlock) void k_step(int64_t n, double alpha, const double *__restrict__ p,
                                                 const double *__restrict__ q, double *__restrict__ x,
                                                 double *__restrict__ r, double *__restrict__ part) {
    __shared__ double red[kBlock / kWave];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s += ri * ri;
    }
    s = block_sum<kBlock>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// z = omega D^-1 r (first smoothing step from z = 0), or z += omega D^-1 rz
__global__ void k_smooth(int64_t n, double omega, const double *__restrict__ dinv, const double *__restrict__ rz,
                         double *__restrict__ z, int first) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double v = omega * dinv[i] * rz[i];
        z[i] = first ? v : z[i] + v;
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kDotBlocks)); }

}  // namespace
}  // namespace fem
