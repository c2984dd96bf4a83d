// local.hip -- all local P1 matrices at once (Section 1, eq. (2) per element).
//
// One thread per element.  The element's vertices are gathered through the
// SoA connectivity, B = [p_1 - p_0, ..., p_d - p_0] is inverted by its
// adjugate, the barycentric gradients are the rows of G = D_ref B^{-1},
// K_e = vol G G^T and M_e = vol/((d+1)(d+2)) (1 + delta_ij), vol = |det B|/d!.
// The FP64 results are written in the requested storage with coalesced SoA
// stores (entry (i,j) of consecutive elements is contiguous).  The kernel is
// bound by the stores: 2 n_b^2 values per element against n_b gathered
// vertices.
#include "common.h"
#include "kernels.h"

namespace fem {

namespace {

template <int KIND>
__device__ __forceinline__ void store_entry(void *base, int64_t idx, int64_t blk, double v) {
    if constexpr (KIND == MAT_F64) {
        static_cast<double *>(base)[idx] = v;
    } else if constexpr (KIND == MAT_F32) {
        static_cast<float *>(base)[idx] = (float)v;
    } else {
        float hi = (float)v;
        float lo = (float)(v - (double)hi);
        static_cast<float *>(base)[idx] = hi;
        static_cast<float *>(base)[idx + blk] = lo;
    }
}

template <int DIM, int KIND>
__global__ __launch_bounds__(kBlock) void k_local_matrices(const double *__restrict__ coords,
                                                           const int32_t *__restrict__ conn,
                                                           int64_t n_nodes, int64_t n_elems,
                                                           void *__restrict__ K, void *__restrict__ M,
                                                           double *__restrict__ vol) {
    constexpr int NB = DIM + 1;
    const int64_t blk = (int64_t)NB * NB * n_elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        double p[NB][DIM];
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const int32_t v = conn[(int64_t)a * n_elems + e];
#pragma unroll
            for (int r = 0; r < DIM; ++r) p[a][r] = coords[(int64_t)r * n_nodes + v];
        }
        double B[DIM][DIM];
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) B[r][c] = p[c + 1][r] - p[0][r];
        double Bi[DIM][DIM];
        double det;
        if constexpr (DIM == 2) {
            det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
            Bi[0][0] = B[1][1] / det;
            Bi[0][1] = -B[0][1] / det;
            Bi[1][0] = -B[1][0] / det;
            Bi[1][1] = B[0][0] / det;
        } else {
            const double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
            const double c01 = -(B[1][0] * B[2][2] - B[1][2] * B[2][0]);
            const double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
            const double c10 = -(B[0][1] * B[2][2] - B[0][2] * B[2][1]);
            const double c11 = B[0][0] * B[2][2] - B[0][2] * B[2][0];
            const double c12 = -(B[0][0] * B[2][1] - B[0][1] * B[2][0]);
            const double c20 = B[0][1] * B[1][2] - B[0][2] * B[1][1];
            const double c21 = -(B[0][0] * B[1][2] - B[0][2] * B[1][0]);
            const double c22 = B[0][0] * B[1][1] - B[0][1] * B[1][0];
            det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
            Bi[0][0] = c00 / det; Bi[0][1] = c10 / det; Bi[0][2] = c20 / det;
            Bi[1][0] = c01 / det; Bi[1][1] = c11 / det; Bi[1][2] = c21 / det;
            Bi[2][0] = c02 / det; Bi[2][1] = c12 / det; Bi[2][2] = c22 / det;
        }
        const double ve = fabs(det) / (DIM == 2 ? 2.0 : 6.0);
        // G (NB x DIM): row 0 = -(column sums of Bi), row k+1 = row k of Bi.
        double G[NB][DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s += Bi[k][c];
            G[0][c] = -s;
#pragma unroll
            for (int k = 0; k < DIM; ++k) G[k + 1][c] = Bi[k][c];
        }
        if (K) {
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    double g = 0.0;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) g += G[i][c] * G[j][c];
                    store_entry<KIND>(K, (int64_t)(i * NB + j) * n_elems + e, blk, ve * g);
                }
        }
        if (M) {
            const double m = ve / (double)((DIM + 1) * (DIM + 2));
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    store_entry<KIND>(M, (int64_t)(i * NB + j) * n_elems + e, blk, i == j ? 2.0 * m : m);
        }
        if (vol) vol[e] = ve;
    }
}

template <int NB, int KIN, int KOUT>
__global__ __launch_bounds__(kBlock) void k_combine(const void *__restrict__ K, const void *__restrict__ M,
                                                    double nu, int64_t n_elems, void *__restrict__ A) {
    const int64_t blk = (int64_t)NB * NB * n_elems;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < blk;
         idx += (int64_t)gridDim.x * blockDim.x) {
        double a = load_entry<KIN>(K, idx, blk);
        if (M) a += nu * load_entry<KIN>(M, idx, blk);
        store_entry<KOUT>(A, idx, blk, a);
    }
}

// Packed symmetric difference form of A_e = K_e + nu M_e: row sums, then the
// symmetrised upper off-diagonal entries a_ij = (A_ij + A_ji) / 2.
template <int NB, int KIN, int KOUT>
__global__ __launch_bounds__(kBlock) void k_pack(const void *__restrict__ K, const void *__restrict__ M, double nu,
                                                 int64_t n_elems, void *__restrict__ A) {
    constexpr int NP = NB + NB * (NB - 1) / 2;
    const int64_t blk_in = (int64_t)NB * NB * n_elems;
    const int64_t blk_out = (int64_t)NP * n_elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        double a[NB][NB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int64_t idx = (int64_t)(i * NB + j) * n_elems + e;
                double v = load_entry<KIN>(K, idx, blk_in);
                if (M) v += nu * load_entry<KIN>(M, idx, blk_in);
                a[i][j] = v;
            }
        double off[NB][NB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) {
                off[i][j] = 0.5 * (a[i][j] + a[j][i]);
                off[j][i] = off[i][j];
            }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            double rho = a[i][i];
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j != i) rho += off[i][j];
            store_entry<KOUT>(A, (int64_t)i * n_elems + e, blk_out, rho);
        }
        int k = NB;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) store_entry<KOUT>(A, (int64_t)(k++) * n_elems + e, blk_out, off[i][j]);
    }
}

int grid_for(int64_t n, int64_t cap) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int launch_local_matrices(const DevPlan &P, int kind, void *K, void *M, double *vol, hipStream_t s) {
    const int g = grid_for(P.n_elems, 65536);
#define FEM_LM(D, KND) \
    k_local_matrices<D, KND><<<g, kBlock, 0, s>>>(P.coords, P.conn, P.n_nodes, P.n_elems, K, M, vol)
    if (P.dim == 2) {
        if (kind == MAT_F64) FEM_LM(2, MAT_F64);
        else if (kind == MAT_F32) FEM_LM(2, MAT_F32);
        else FEM_LM(2, MAT_F32X2);
    } else {
        if (kind == MAT_F64) FEM_LM(3, MAT_F64);
        else if (kind == MAT_F32) FEM_LM(3, MAT_F32);
        else FEM_LM(3, MAT_F32X2);
    }
#undef FEM_LM
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_combine(const DevPlan &P, int kin, const void *K, const void *M, double nu, int kout, void *A,
                   hipStream_t s) {
    const int g = grid_for((int64_t)P.nb * P.nb * P.n_elems, 65536);
#define FEM_CB(NB, KI, KO) k_combine<NB, KI, KO><<<g, kBlock, 0, s>>>(K, M, nu, P.n_elems, A)
#define FEM_CB_OUT(NB, KI)                         \
    do {                                           \
        if (kout == MAT_F64) FEM_CB(NB, KI, MAT_F64); \
        else if (kout == MAT_F32) FEM_CB(NB, KI, MAT_F32); \
        else FEM_CB(NB, KI, MAT_F32X2);            \
    } while (0)
#define FEM_CB_IN(NB)                              \
    do {                                           \
        if (kin == MAT_F64) FEM_CB_OUT(NB, MAT_F64); \
        else if (kin == MAT_F32) FEM_CB_OUT(NB, MAT_F32); \
        else FEM_CB_OUT(NB, MAT_F32X2);            \
    } while (0)
    if (P.nb == 3) FEM_CB_IN(3);
    else FEM_CB_IN(4);
#undef FEM_CB_IN
#undef FEM_CB_OUT
#undef FEM_CB
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int launch_pack(const DevPlan &P, int kin, const void *K, const void *M, double nu, int kout, void *A,
                hipStream_t s) {
    const int g = grid_for(P.n_elems, 65536);
#define FEM_PK(NB, KI, KO) k_pack<NB, KI, KO><<<g, kBlock, 0, s>>>(K, M, nu, P.n_elems, A)
#define FEM_PK_OUT(NB, KI)                                  \
    do {                                                    \
        if (kout == MAT_F64) FEM_PK(NB, KI, MAT_F64);       \
        else FEM_PK(NB, KI, MAT_F32X2);                     \
    } while (0)
#define FEM_PK_IN(NB)                                       \
    do {                                                    \
        if (kin == MAT_F64) FEM_PK_OUT(NB, MAT_F64);        \
        else if (kin == MAT_F32) FEM_PK_OUT(NB, MAT_F32);   \
        else FEM_PK_OUT(NB, MAT_F32X2);                     \
    } while (0)
    if (P.nb == 3) FEM_PK_IN(3);
    else FEM_PK_IN(4);
#undef FEM_PK_IN
#undef FEM_PK_OUT
#undef FEM_PK
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace fem
