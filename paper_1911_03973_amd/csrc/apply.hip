// apply.hip -- element residual, operator application, right-hand side and
// Jacobi diagonal through the chunked gather of chunk.h.
//
//   residual  r = b - sum_e C_e^T (K_e + nu M_e) C_e x     (eq. (4), Algorithm 1)
//   rhs       b = sum_e C_e^T M_e f_e                      (eq. (2)-(3))
//   diagonal  d = sum_e C_e^T diag(K_e + nu M_e)
#include <algorithm>
#include <string>
#include <type_traits>

#include "chunk.h"
#include "kernels.h"

namespace fem {

namespace {

// out = (b ? b : 0) + sign * acc, zeroed on Dirichlet nodes if use_mask.
template <class T>
struct OpAffine {
    static constexpr bool kLocal = false;
    const T *x;
    const T *b;
    T *out;
    const uint8_t *mask;
    T sign;
    int use_mask;
    __device__ __forceinline__ bool begin() { return true; }
    __device__ __forceinline__ T gather(int g, int) const { return x[g]; }
    struct Pre {
        T bv;
        bool zero;
    };
    __device__ __forceinline__ Pre fixup_load(int, int g) const {
        return {b ? b[g] : (T)0, use_mask && mask[g]};
    }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &pr, T acc) const {
        const T v = pr.bv + sign * acc;
        out[g] = pr.zero ? (T)0 : v;
    }
    __device__ __forceinline__ void finish(int g, T acc) const {
        T v = (b ? b[g] : (T)0) + sign * acc;
        if (use_mask && mask[g]) v = (T)0;
        out[g] = v;
    }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

int g_cu = 0;

// local nodes per thread held in registers by k_chunk_affine (a 1024-triangle
// chunk of a structured mesh has about 560).  Used for the FP32 pass only:
// with FP64 element matrices in registers the extra registers cost more
// occupancy than the shorter load chains gain.
constexpr int kAffineNodes = 3;

// Element pass plus fix-up.  FP32 passes use k_chunk_affine with the
// solver's workgroup size for the chunk size (default_block); FP64 passes,
// whose element matrices take most of the registers, use k_chunk_main with
// 256 threads (more elements in flight per thread: measured faster than
// 512 threads for 1536-tetrahedron chunks).
template <int NB, class T, class Ld, class Op, bool DIAG>
int run_chunked(const DevPlan &P, const Ld &ld, const Op &op, T *scratch, hipStream_t s) {
    const size_t lds = chunk_lds_for<NB, T, Ld>(P);
    if (lds > device_lds_limit())
        return set_error(-1, "the chunk's LDS (" + std::to_string(lds) + " bytes) exceeds the workgroup limit; "
                             "build the plan with smaller chunk_elems");
    constexpr bool kAffine = !DIAG && std::is_same<T, float>::value;
    const int block = kAffine ? default_block(NB, P.E) : kBlock;
    const ChunkGrid cg = chunk_grid(P.n_chunks, lds, block);
    int rc = dispatch_tile(P.E, block, [&](auto bs, auto ept) {
        constexpr int BS = decltype(bs)::value, EPT = decltype(ept)::value;
        if constexpr (kAffine)
            k_chunk_affine<NB, EPT, BS, kAffineNodes, T, Ld, Op><<<cg.grid, BS, lds, s>>>(P, ld, op, scratch, cg.xcd);
        else if constexpr (BS == kBlock)
            k_chunk_main<NB, EPT, BS, T, Ld, Op, DIAG><<<cg.grid, BS, lds, s>>>(P, ld, op, scratch, cg.xcd);
        else
            return set_error(-1, "internal error: unexpected workgroup size");
        return 0;
    });
    if (rc) return rc;
    FEM_HIP_CHECK(hipGetLastError());
    if (P.n_shared > 0) {
        k_chunk_fixup<kFixBlock, T, Op><<<fixup_grid(P.n_shared), kFixBlock, 0, s>>>(P, op, scratch, 0);
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

template <int NB, int KIND>
int apply_pk64_nb(const DevPlan &P, const void *A, const double *x, const double *b, double *out, double sign,
                  int use_mask, double *scratch, hipStream_t s) {
    LdPk<NB, KIND> ld{A, P.n_elems};
    OpAffine<double> op{x, b, out, P.mask, sign, use_mask};
    return run_chunked<NB, double, decltype(ld), decltype(op), false>(P, ld, op, scratch, s);
}

template <int NB>
int apply_mf_nb(const DevPlan &P, double kk, double nu, const double *x, const double *b, double *out,
                double sign, int use_mask, double *scratch, hipStream_t s) {
    LdMf<NB> ld{P.coords, P.n_nodes, kk, nu};
    OpAffine<double> op{x, b, out, P.mask, sign, use_mask};
    return run_chunked<NB, double, decltype(ld), decltype(op), false>(P, ld, op, scratch, s);
}

template <int NB>
int diag_mf_nb(const DevPlan &P, double nu, double *d, double *scratch, hipStream_t s) {
    LdMf<NB> ld{P.coords, P.n_nodes, 1.0, nu};
    OpAffine<double> op{nullptr, nullptr, d, P.mask, 1.0, 0};
    return run_chunked<NB, double, decltype(ld), decltype(op), true>(P, ld, op, scratch, s);
}

int g_lds = 0;

}  // namespace

size_t device_lds_limit() {
    if (g_lds <= 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            g_lds = v;
        if (g_lds <= 0) g_lds = kMaxChunkLds;
    }
    return (size_t)g_lds;
}

int launch_apply_mf(const DevPlan &P, double kk, double nu, const double *x, const double *b, double *out,
                    double sign, int use_mask, double *scratch, hipStream_t s) {
    if (P.nb == 3) return apply_mf_nb<3>(P, kk, nu, x, b, out, sign, use_mask, scratch, s);
    if (P.nb == 4) return apply_mf_nb<4>(P, kk, nu, x, b, out, sign, use_mask, scratch, s);
    return set_error(-1, "the matrix-free operator covers linear (P1) elements only");
}

int launch_diag_mf(const DevPlan &P, double nu, double *d, double *scratch, hipStream_t s) {
    if (P.nb == 3) return diag_mf_nb<3>(P, nu, d, scratch, s);
    if (P.nb == 4) return diag_mf_nb<4>(P, nu, d, scratch, s);
    return set_error(-1, "the matrix-free operator covers linear (P1) elements only");
}

ChunkGrid chunk_grid(int64_t n_chunks, size_t lds, int bs) {
    const int per_cu = std::max(1, std::min(2048 / bs, (int)(160 * 1024 / (lds + 512))));
    const int64_t cap = (int64_t)per_cu * device_cu_count();
    ChunkGrid g;
    if (n_chunks >= 8) {
        int64_t gr = std::min<int64_t>(cap, n_chunks);
        gr = std::max<int64_t>(8, gr / 8 * 8);
        g.grid = (int)gr;
        g.xcd = 1;
    } else {
        g.grid = (int)std::max<int64_t>(1, n_chunks);
        g.xcd = 0;
    }
    return g;
}

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


// Quadratic triangles: two elements per thread (their 21 packed values per
// element leave room for no more; measured at 1024-element chunks: 512
// threads 117 us per pass, 256 threads 144 us, 1024 threads 124 us).
int default_block(int nb, int E) {
    if (nb == 6) return E >= 1024 ? 512 : 256;
    if (nb == 10) return E >= 512 ? 512 : 256;  // one quadratic tetrahedron (55 packed values) per thread
    return E > 1024 ? 512 : 256;
}

int launch_apply64(const DevPlan &P, int kind, const void *K, const void *M, double nu, const double *x,
                   const double *b, double *out, double sign, int use_mask, double *scratch, hipStream_t s) {
    return dispatch_nb(P.nb, [&](auto nbc) -> int {
        constexpr int NB = decltype(nbc)::value;
        if (kind == MAT_F64) return apply64_nb<NB, MAT_F64>(P, K, M, nu, x, b, out, sign, use_mask, scratch, s);
        if (kind == MAT_F32) return apply64_nb<NB, MAT_F32>(P, K, M, nu, x, b, out, sign, use_mask, scratch, s);
        return apply64_nb<NB, MAT_F32X2>(P, K, M, nu, x, b, out, sign, use_mask, scratch, s);
    });
}

int launch_apply_pk64(const DevPlan &P, int kind, const void *A, const double *x, const double *b, double *out,
                      double sign, int use_mask, double *scratch, hipStream_t s) {
    return dispatch_nb(P.nb, [&](auto nbc) -> int {
        constexpr int NB = decltype(nbc)::value;
        if (kind == MAT_F64) return apply_pk64_nb<NB, MAT_F64>(P, A, x, b, out, sign, use_mask, scratch, s);
        return apply_pk64_nb<NB, MAT_F32X2>(P, A, x, b, out, sign, use_mask, scratch, s);
    });
}

int launch_diag_pk64(const DevPlan &P, int kind, const void *A, double *d, double *scratch, hipStream_t s) {
    OpAffine<double> op{nullptr, nullptr, d, P.mask, 1.0, 0};
    return dispatch_nb(P.nb, [&](auto nbc) -> int {
        constexpr int NB = decltype(nbc)::value;
        if (kind == MAT_F64) {
            LdPk<NB, MAT_F64> ld{A, P.n_elems};
            return run_chunked<NB, double, decltype(ld), decltype(op), true>(P, ld, op, scratch, s);
        }
        LdPk<NB, MAT_F32X2> ld{A, P.n_elems};
        return run_chunked<NB, double, decltype(ld), decltype(op), true>(P, ld, op, scratch, s);
    });
}

int launch_apply32(const DevPlan &P, const float *A, const float *x, const float *b, float *out, float sign,
                   int use_mask, float *scratch, hipStream_t s) {
    OpAffine<float> op{x, b, out, P.mask, sign, use_mask};
    return dispatch_nb(P.nb, [&](auto nbc) -> int {
        constexpr int NB = decltype(nbc)::value;
        LdF32<NB> ld{A, P.n_elems};
        return run_chunked<NB, float, decltype(ld), decltype(op), false>(P, ld, op, scratch, s);
    });
}

int launch_diag64(const DevPlan &P, int kind, const void *K, const void *M, double nu, double *d,
                  double *scratch, hipStream_t s) {
    return dispatch_nb(P.nb, [&](auto nbc) -> int {
        constexpr int NB = decltype(nbc)::value;
        if (kind == MAT_F64) return diag64_nb<NB, MAT_F64>(P, K, M, nu, d, scratch, s);
        if (kind == MAT_F32) return diag64_nb<NB, MAT_F32>(P, K, M, nu, d, scratch, s);
        return diag64_nb<NB, MAT_F32X2>(P, K, M, nu, d, scratch, s);
    });
}

}  // namespace fem
