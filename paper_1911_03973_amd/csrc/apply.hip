// apply.hip -- element residual, operator application, right-hand side and
// Jacobi diagonal through the chunked gather of chunk.h.
//
//   residual  r = b - sum_e C_e^T (K_e + nu M_e) C_e x     (eq. (4), Algorithm 1)
//   rhs       b = sum_e C_e^T M_e f_e                      (eq. (2)-(3))
//   diagonal  d = sum_e C_e^T diag(K_e + nu M_e)
#include <algorithm>

#include "chunk.h"
#include "kernels.h"

namespace fem {

namespace {

// out = (b ? b : 0) + sign * acc, zeroed on Dirichlet nodes if use_mask.
template <class T>
struct OpAffine {
    const T *x;
    const T *b;
    T *out;
    const uint8_t *mask;
    T sign;
    int use_mask;
    __device__ __forceinline__ bool begin(double *) { return true; }
    __device__ __forceinline__ bool begin_fixup(double *) { return true; }
    __device__ __forceinline__ T gather(int g, bool) const { return x[g]; }
    __device__ __forceinline__ void gather_shared(int) {}
    __device__ __forceinline__ double finish(int g, T acc) const {
        T v = (b ? b[g] : (T)0) + sign * acc;
        if (use_mask && mask[g]) v = (T)0;
        out[g] = v;
        return 0.0;
    }
    __device__ __forceinline__ void end(double, double *) const {}
    __device__ __forceinline__ void end_fixup(double, double *) const {}
};

int g_cu = 0;

template <int NB, class T, class Ld, class Op, bool DIAG>
int run_chunked(const DevPlan &P, const Ld &ld, const Op &op, T *scratch, hipStream_t s) {
    const size_t lds = chunk_lds_bytes<NB, T>(P.E);
    const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / (lds + 1024))));
    const int64_t cap = (int64_t)per_cu * device_cu_count();
    const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(P.n_chunks, cap));
    k_chunk_main<NB, T, Ld, Op, DIAG><<<gm, kBlock, lds, s>>>(P, ld, op, scratch);
    FEM_HIP_CHECK(hipGetLastError());
    if (P.n_shared > 0) {
        const int gf = (int)std::min<int64_t>((P.n_shared + kBlock - 1) / kBlock, 2048);
        k_chunk_fixup<T, Op><<<gf, kBlock, 0, s>>>(P, op, scratch);
        FEM_HIP_CHECK(hipGetLastError());
    }
    return 0;
}

template <int NB, int KIND>
int apply64_nb(const DevPlan &P, const void *K, const void *M, double nu, const double *x, const double *b,
               double *out, double sign, int use_mask, double *scratch, hipStream_t s) {
    LdKM<NB, KIND, double> ld{K, M, nu, P.n_elems};
    OpAffine<double> op{x, b, out, P.mask, sign, use_mask};
    return run_chunked<NB, double, decltype(ld), decltype(op), false>(P, ld, op, scratch, s);
}

template <int NB, int KIND>
int diag64_nb(const DevPlan &P, const void *K, const void *M, double nu, double *d, double *scratch,
              hipStream_t s) {
    LdKM<NB, KIND, double> ld{K, M, nu, P.n_elems};
    OpAffine<double> op{nullptr, nullptr, d, P.mask, 1.0, 0};
    return run_chunked<NB, double, decltype(ld), decltype(op), true>(P, ld, op, scratch, s);
}

}  // namespace

int device_cu_count() {
    if (g_cu <= 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            g_cu = prop.multiProcessorCount;
        if (g_cu <= 0) g_cu = 256;
    }
    return g_cu;
}

int max_chunk_elems(int nb) {
    // FP64 slot buffer + uint16 slot list within kMaxChunkLds, multiple of 64
    int e = kMaxChunkLds / (nb * (8 + 2));
    return (e / 64) * 64;
}

int default_chunk_elems(int nb) { return nb == 3 ? 2048 : 1536; }

int launch_apply64(const DevPlan &P, int kind, const void *K, const void *M, double nu, const double *x,
                   const double *b, double *out, double sign, int use_mask, double *scratch, hipStream_t s) {
#define FEM_A64(NB, KND) return apply64_nb<NB, KND>(P, K, M, nu, x, b, out, sign, use_mask, scratch, s)
    if (P.nb == 3) {
        if (kind == MAT_F64) FEM_A64(3, MAT_F64);
        if (kind == MAT_F32) FEM_A64(3, MAT_F32);
        FEM_A64(3, MAT_F32X2);
    }
    if (kind == MAT_F64) FEM_A64(4, MAT_F64);
    if (kind == MAT_F32) FEM_A64(4, MAT_F32);
    FEM_A64(4, MAT_F32X2);
#undef FEM_A64
}

int launch_apply32(const DevPlan &P, const float *A, const float *x, const float *b, float *out, float sign,
                   int use_mask, float *scratch, hipStream_t s) {
    OpAffine<float> op{x, b, out, P.mask, sign, use_mask};
    if (P.nb == 3) {
        LdF32<3> ld{A, P.n_elems};
        return run_chunked<3, float, decltype(ld), decltype(op), false>(P, ld, op, scratch, s);
    }
    LdF32<4> ld{A, P.n_elems};
    return run_chunked<4, float, decltype(ld), decltype(op), false>(P, ld, op, scratch, s);
}

int launch_diag64(const DevPlan &P, int kind, const void *K, const void *M, double nu, double *d,
                  double *scratch, hipStream_t s) {
#define FEM_D64(NB, KND) return diag64_nb<NB, KND>(P, K, M, nu, d, scratch, s)
    if (P.nb == 3) {
        if (kind == MAT_F64) FEM_D64(3, MAT_F64);
        if (kind == MAT_F32) FEM_D64(3, MAT_F32);
        FEM_D64(3, MAT_F32X2);
    }
    if (kind == MAT_F64) FEM_D64(4, MAT_F64);
    if (kind == MAT_F32) FEM_D64(4, MAT_F32);
    FEM_D64(4, MAT_F32X2);
#undef FEM_D64
}

}  // namespace fem
