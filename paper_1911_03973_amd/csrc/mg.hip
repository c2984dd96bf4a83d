// mg.hip -- geometric multigrid preconditioner on nested diagonal-cut square
// grids and Kuhn cube grids.
//
// The condition number of the P1 operator grows like h^-2, which is why the
// experiment of Section 3 needs its spectral bounds and why the paper points
// to better preconditioning for fine meshes.  On the structured meshes of the
// workloads (n x n squares cut along the (0,0)-(1,1) diagonal, node (i, j)
// numbered j (n + 1) + i) the mesh of n/2 squares is nested in the mesh of n
// squares: its triangles split into four (red refinement).  The P1 space of
// the coarse mesh is then a subspace of the fine one, and the prolongation is
// exact P1 interpolation:
//   fine (2I, 2J)         <- coarse (I, J)
//   fine (2I+1, 2J)       <- average of coarse (I, J), (I+1, J)
//   fine (2I, 2J+1)       <- average of coarse (I, J), (I, J+1)
//   fine (2I+1, 2J+1)     <- average of coarse (I, J), (I+1, J+1)  (diagonal edge)
// The Kuhn split of the cube lattice (6 tetrahedra around each cube's
// (0,0,0)-(1,1,1) diagonal) refines the same way: a fine node with parity
// pattern e != 0 is the midpoint of the coarse edge from (i, j, k) >> 1 along
// e, and the restriction gathers the 14 lattice neighbours +-e.
// The restriction is its transpose: a coarse node collects its fine node with
// weight 1 and the six fine edge neighbours of that node, (+-1, 0), (0, +-1),
// (1, 1) and (-1, -1), with weight 1/2.  With these, P^T A_h P equals the
// operator assembled on the coarse mesh (Galerkin), which the tests check.
//
// One V-cycle from level l with residual r: `smooth` damped-Jacobi steps
// z += omega D^-1 (r - A z) from z = 0, restriction of r - A z, the cycle on
// the next level, z += P z_coarse, `smooth` more Jacobi steps; on the
// coarsest level z = A^-1 r with a dense inverse formed once at setup.
// The Chebyshev smoother replaces the Jacobi steps by `smooth` steps of the
// three-level Chebyshev iteration of Section 2 (eq. (9), scaling factors of
// eq. (8)) on the Jacobi-scaled level system D^-1 A z = D^-1 r over
// [lower g, g], g = max over free nodes of D_ii^-1 sum_e sum_j |(A_e)_ij|
// (Gershgorin's bound of D^-1 A from the element matrices, one element pass
// at setup).  A step keeps the increment d = z^{k+1} - z^k:
//   d <- rho_k / (2 sigma - rho_k) d + 4 / (lam2 - lam1) / (2 sigma - rho_k) D^-1 (r - A z),
//   z <- z + d,
// rho_1 = 1 / sigma, rho_{k+1} = 1 / (2 sigma - rho_k), sigma = (lam1 + lam2) / (lam2 - lam1);
// the first step of either side is d = 2 / (lam1 + lam2) D^-1 (r - A z).  Every
// operator application is the element residual through the FP64 packed form;
// Dirichlet rows stay zero in every correction.  The cycle preconditions
// flexible CG (FCG(1), as in fcg.hip), judged by the true residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "chunk.h"
#include "common.h"
#include "fem.h"
#include "kernels.h"
#include "solver.h"
#include "vec.h"

namespace fem {

namespace {

// rc = P^T rf on the coarse grid of nc squares per side, 0 on coarse Dirichlet nodes
__global__ void k_restrict(int nc, const double *__restrict__ rf, const uint8_t *__restrict__ mask_c,
                           double *__restrict__ rc) {
    const int mc = nc + 1, mf = 2 * nc + 1;
    const int64_t total = (int64_t)mc * mc;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        const int I = (int)(id % mc), J = (int)(id / mc);
        double v = 0.0;
        if (!mask_c[id]) {
            const int i = 2 * I, j = 2 * J;
            auto f = [&](int a, int b) -> double {
                return (a >= 0 && a < mf && b >= 0 && b < mf) ? rf[(int64_t)b * mf + a] : 0.0;
            };
            v = f(i, j) + 0.5 * (((f(i - 1, j) + f(i + 1, j)) + (f(i, j - 1) + f(i, j + 1))) +
                                 (f(i + 1, j + 1) + f(i - 1, j - 1)));
        }
        rc[id] = v;
    }
}

// zf += P zc, 0 on fine Dirichlet nodes (nc coarse squares per side)
__global__ void k_prolong_add(int nc, const double *__restrict__ zc, const uint8_t *__restrict__ mask_f,
                              double *__restrict__ zf) {
    const int mc = nc + 1, mf = 2 * nc + 1;
    const int64_t total = (int64_t)mf * mf;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        if (mask_f[id]) continue;
        const int i = (int)(id % mf), j = (int)(id / mf);
        const int I = i >> 1, J = j >> 1;
        const double c00 = zc[(int64_t)J * mc + I];
        double v;
        if (!(i & 1) && !(j & 1)) v = c00;
        else if ((i & 1) && !(j & 1)) v = 0.5 * (c00 + zc[(int64_t)J * mc + I + 1]);
        else if (!(i & 1)) v = 0.5 * (c00 + zc[(int64_t)(J + 1) * mc + I]);
        else v = 0.5 * (c00 + zc[(int64_t)(J + 1) * mc + I + 1]);
        zf[id] += v;
    }
}

// Kuhn cube meshes (node (i, j, k) numbered (k m + j) m + i): every lattice
// vertex is joined to its 14 neighbours +-e, e in {0,1}^3 \ {0}, so a fine
// node with an odd index is the midpoint of the coarse edge from
// (i, j, k) >> 1 along its parity pattern.
// rc = P^T rf: fine (2I, 2J, 2K) with weight 1, the 14 neighbours with 1/2
__global__ void k_restrict3(int nc, const double *__restrict__ rf, const uint8_t *__restrict__ mask_c,
                            double *__restrict__ rc) {
    const int mc = nc + 1, mf = 2 * nc + 1;
    const int64_t total = (int64_t)mc * mc * mc;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        const int I = (int)(id % mc), J = (int)((id / mc) % mc), K = (int)(id / ((int64_t)mc * mc));
        double v = 0.0;
        if (!mask_c[id]) {
            const int i = 2 * I, j = 2 * J, k = 2 * K;
            auto f = [&](int a, int b, int c) -> double {
                return (a >= 0 && a < mf && b >= 0 && b < mf && c >= 0 && c < mf)
                           ? rf[((int64_t)c * mf + b) * mf + a]
                           : 0.0;
            };
            double h = 0.0;
#pragma unroll
            for (int e = 1; e < 8; ++e) {
                const int a = e & 1, b = (e >> 1) & 1, c = e >> 2;
                h += f(i + a, j + b, k + c) + f(i - a, j - b, k - c);
            }
            v = f(i, j, k) + 0.5 * h;
        }
        rc[id] = v;
    }
}

// zf += P zc, 0 on fine Dirichlet nodes (nc coarse cubes per side)
__global__ void k_prolong_add3(int nc, const double *__restrict__ zc, const uint8_t *__restrict__ mask_f,
                               double *__restrict__ zf) {
    const int mc = nc + 1, mf = 2 * nc + 1;
    const int64_t total = (int64_t)mf * mf * mf;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        if (mask_f[id]) continue;
        const int i = (int)(id % mf), j = (int)((id / mf) % mf), k = (int)(id / ((int64_t)mf * mf));
        const int a = i & 1, b = j & 1, c = k & 1;
        const int64_t lo = ((int64_t)(k >> 1) * mc + (j >> 1)) * mc + (i >> 1);
        double v = zc[lo];
        if (a | b | c) v = 0.5 * (v + zc[lo + ((int64_t)c * mc + b) * mc + a]);
        zf[id] += v;
    }
}

// z = Ainv r (dense, row-major n x n): one wave per row, the lanes stride
// the row (coalesced) and a butterfly adds their sums in a fixed order
__global__ __launch_bounds__(kBlock) void k_dense_mv(int n, const double *__restrict__ Ainv,
                                                     const double *__restrict__ r, double *__restrict__ z) {
    const int lane = threadIdx.x % kWave;
    const int row = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (row >= n) return;  // uniform across the wave
    const double *a = Ainv + (int64_t)row * n;
    double s = 0.0;
    for (int j = lane; j < n; j += kWave) s += a[j] * r[j];
    for (int off = kWave / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (lane == 0) z[row] = s;
}

// One damped-Jacobi step fused into the element pass: zn = z + omega D^-1
// (r - A z), 0 on Dirichlet nodes, without storing r - A z.  zn must not
// alias z (other workgroups still gather z).
struct OpSmooth {
    static constexpr bool kLocal = false;
    const double *z, *r, *dinv;
    double *zn;
    const uint8_t *mask;
    double omega;
    __device__ __forceinline__ bool begin() const { return true; }
    __device__ __forceinline__ double gather(int g, int) const { return z[g]; }
    struct Pre {
        double rv, zv, dv;
        bool zero;
    };
    __device__ __forceinline__ Pre fixup_load(int, int g) const { return {r[g], z[g], dinv[g], mask[g] != 0}; }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &pr, double acc) const {
        double t = pr.rv + (-1.0) * acc;
        if (pr.zero) t = 0.0;
        zn[g] = pr.zv + omega * pr.dv * t;
    }
    __device__ __forceinline__ void finish(int g, double acc) const { fixup_store(0, g, fixup_load(0, g), acc); }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

// One Chebyshev step: t = r - A z (0 on Dirichlet nodes), d <- c1 d +
// c2 D^-1 t, zn = z + d.  c1 == 0 restarts the recurrence and does not read d
// (whose old contents may be anything).
struct OpCheb {
    static constexpr bool kLocal = false;
    const double *z, *r, *dinv;
    double *zn, *d;
    const uint8_t *mask;
    double c1, c2;
    __device__ __forceinline__ bool begin() const { return true; }
    __device__ __forceinline__ double gather(int g, int) const { return z[g]; }
    struct Pre {
        double rv, zv, dv, cv;
        bool zero;
    };
    __device__ __forceinline__ Pre fixup_load(int, int g) const {
        return {r[g], z[g], dinv[g], c1 != 0.0 ? d[g] : 0.0, mask[g] != 0};
    }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &pr, double acc) const {
        double t = pr.rv + (-1.0) * acc;
        if (pr.zero) t = 0.0;
        const double dn = c1 * pr.cv + c2 * pr.dv * t;
        d[g] = dn;
        zn[g] = pr.zv + dn;
    }
    __device__ __forceinline__ void finish(int g, double acc) const { fixup_store(0, g, fixup_load(0, g), acc); }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

// |A_e| x: the element matrix with every entry in absolute value, read from
// the FP64 packed difference form (A_ij = v_ij off the diagonal, A_ii = the
// row sum v_i minus the row's off-diagonal entries).
template <int NB>
struct LdAbs {
    using Base = LdPk<NB, MAT_F64>;
    using Regs = typename Base::Regs;
    Base base;
    __device__ __forceinline__ void fetch(int64_t e, Regs &R) const { base.fetch(e, R); }
    template <class T>
    __device__ __forceinline__ static void apply(const Regs &R, const T (&xt)[NB], T (&yt)[NB]) {
        double dg[NB], y[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) dg[i] = R.v[i];
        int k = NB;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) {
                dg[i] -= R.v[k];
                dg[j] -= R.v[k];
                ++k;
            }
#pragma unroll
        for (int i = 0; i < NB; ++i) y[i] = fabs(dg[i]) * (double)xt[i];
        k = NB;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) {
                const double a = fabs(R.v[k++]);
                y[i] += a * (double)xt[j];
                y[j] += a * (double)xt[i];
            }
#pragma unroll
        for (int i = 0; i < NB; ++i) yt[i] = (T)y[i];
    }
};

// out = sum_e C_e^T |A_e| 1 (the element absolute row sums at the nodes)
struct OpAbsRow {
    static constexpr bool kLocal = false;
    double *out;
    __device__ __forceinline__ bool begin() const { return true; }
    __device__ __forceinline__ double gather(int, int) const { return 1.0; }
    struct Pre {};
    __device__ __forceinline__ Pre fixup_load(int, int) const { return {}; }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &, double acc) const { out[g] = acc; }
    __device__ __forceinline__ void finish(int g, double acc) const { out[g] = acc; }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

// part[block] = max over the block's free nodes of dinv[i] * absrow[i]
__global__ __launch_bounds__(kBlock) void k_gersh(int64_t n, const double *__restrict__ absrow,
                                                  const double *__restrict__ dinv, const uint8_t *__restrict__ mask,
                                                  double *__restrict__ part) {
    __shared__ double red[kBlock];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        if (!mask[i]) m = fmax(m, dinv[i] * absrow[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// z = d = w D^-1 r: the first Chebyshev step from z = 0 (no product needed)
__global__ __launch_bounds__(kBlock) void k_cheb_first(int64_t n, double w, const double *__restrict__ dinv,
                                                       const double *__restrict__ r, double *__restrict__ z,
                                                       double *__restrict__ d) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double v = w * dinv[i] * r[i];
        z[i] = v;
        d[i] = v;
    }
}

// t = r - A z, 0 on Dirichlet nodes (the residual restricted to the next level)
struct OpResid {
    static constexpr bool kLocal = false;
    const double *z, *r;
    double *t;
    const uint8_t *mask;
    __device__ __forceinline__ bool begin() const { return true; }
    __device__ __forceinline__ double gather(int g, int) const { return z[g]; }
    struct Pre {
        double rv;
        bool zero;
    };
    __device__ __forceinline__ Pre fixup_load(int, int g) const { return {r[g], mask[g] != 0}; }
    __device__ __forceinline__ void fixup_store(int, int g, const Pre &pr, double acc) const {
        const double v = pr.rv + (-1.0) * acc;
        t[g] = pr.zero ? 0.0 : v;
    }
    __device__ __forceinline__ void finish(int g, double acc) const { fixup_store(0, g, fixup_load(0, g), acc); }
    template <int BS>
    __device__ __forceinline__ void end(double *, int) const {}
};

// e = unit vector j (length n)
__global__ void k_unit(int64_t n, int64_t j, double *__restrict__ e) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        e[i] = i == j ? 1.0 : 0.0;
}

// Gauss-Jordan inversion with partial pivoting of a row-major n x n matrix
bool invert(int n, std::vector<double> &a, std::vector<double> &inv) {
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
        const double pv = a[(size_t)piv * n + c];
        if (!(std::fabs(pv) > 0.0) || !std::isfinite(pv)) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)piv * n + k], a[(size_t)c * n + k]);
                std::swap(inv[(size_t)piv * n + k], inv[(size_t)c * n + k]);
            }
        const double s = 1.0 / pv;
        for (int k = 0; k < n; ++k) {
            a[(size_t)c * n + k] *= s;
            inv[(size_t)c * n + k] *= s;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    return true;
}

}  // namespace

struct MgLevel {
    DevPlan P{};
    int n = 0;    // squares (cubes) per side
    int dim = 2;
    double *A = nullptr, *dinv = nullptr, *r = nullptr, *z = nullptr, *t = nullptr, *scratch = nullptr;
    double *c = nullptr;  // the Chebyshev smoother's increment
    void *A32 = nullptr;  // the packed operator as FP32 hi/lo pair; the cycle may read its heads
    double gersh = 1.0;   // Gershgorin bound of D^-1 A (element absolute row sums)
};

// What one V-cycle does on every level above the coarsest.
struct Cycle {
    int smooth;
    double omega;  // damped Jacobi
    bool f32;      // products read the FP32 heads
    int smoother;  // FEM_SMOOTH_JACOBI or FEM_SMOOTH_CHEBYSHEV
    double lower;  // Chebyshev interval [lower g, g]
};

}  // namespace fem

struct fem_mg {
    std::vector<fem::MgLevel> lv;
    void *arena = nullptr;
    double *Ainv = nullptr;  // coarsest level, dense inverse (Dirichlet rows / columns: identity)
    int nc = 0;              // coarsest node count
    // FCG vectors on the finest level
    double *p = nullptr, *q = nullptr, *part = nullptr, *sums = nullptr;
    const double **ptrs = nullptr;
    int *bad = nullptr;
    ~fem_mg() {
        if (arena) (void)hipFree(arena);
    }
};

namespace fem {

// apply P^T A P on level l+1 vectors: used by tests through the C ABI
int mg_galerkin_apply(fem_mg *mg, int l, const double *zc, double *out, hipStream_t s);

namespace {

int64_t level_nodes(const MgLevel &L) {
    const int64_t m = L.n + 1;
    return L.dim == 3 ? m * m * m : m * m;
}

// rc = P^T rf and zf += P zc between level F and the next coarser level C
int restrict_to(const MgLevel &C, const double *rf, double *rc, hipStream_t s) {
    const int g = grid_for(level_nodes(C));
    if (C.dim == 3) k_restrict3<<<g, kBlock, 0, s>>>(C.n, rf, C.P.mask, rc);
    else k_restrict<<<g, kBlock, 0, s>>>(C.n, rf, C.P.mask, rc);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}
int prolong_add(const MgLevel &F, const MgLevel &C, const double *zc, double *zf, hipStream_t s) {
    const int g = grid_for(level_nodes(F));
    if (C.dim == 3) k_prolong_add3<<<g, kBlock, 0, s>>>(C.n, zc, F.P.mask, zf);
    else k_prolong_add<<<g, kBlock, 0, s>>>(C.n, zc, F.P.mask, zf);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

template <int NB, class Op>
int level_pass_nb(const MgLevel &L, const Op &op, bool f32, hipStream_t s) {
    const DevPlan &P = L.P;
    const size_t lds = chunk_lds_bytes<NB, double>(P.E);
    const ChunkGrid cg = chunk_grid(P.n_chunks, lds);
    int rc = dispatch_ept(P.E, [&](auto ept) -> int {
        constexpr int EPT = decltype(ept)::value;
        if (f32) {
            LdPk<NB, MAT_F32> ld{L.A32, P.n_elems};
            k_chunk_main<NB, EPT, kBlock, double, decltype(ld), Op, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, L.scratch, cg.xcd);
        } else {
            LdPk<NB, MAT_F64> ld{L.A, P.n_elems};
            k_chunk_main<NB, EPT, kBlock, double, decltype(ld), Op, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, L.scratch, cg.xcd);
        }
        return 0;
    });
    if (rc) return rc;
    FEM_HIP_CHECK(hipGetLastError());
    if (P.n_shared > 0) {
        k_chunk_fixup<kFixBlock, double, Op><<<fixup_grid(P.n_shared), kFixBlock, 0, s>>>(P, op, L.scratch, 0);
        FEM_HIP_CHECK(hipGetLastError());
    }
    return 0;
}

// One element pass (+ fix-up) of op over level L's packed operator: FP64
// values, or the FP32 heads of the hi/lo pair (f32); triangles or tetrahedra.
template <class Op>
int level_pass(const MgLevel &L, const Op &op, bool f32, hipStream_t s) {
    if (L.P.nb == 4) return level_pass_nb<4>(L, op, f32, s);
    return level_pass_nb<3>(L, op, f32, s);
}

// zn = z + omega D^-1 (r - A z) on level L
int smooth_step(const MgLevel &L, const double *r, const double *z, double *zn, double omega, bool f32,
                hipStream_t s) {
    return level_pass(L, OpSmooth{z, r, L.dinv, zn, L.P.mask, omega}, f32, s);
}

// `steps` Chebyshev steps on level L that continue from cur (first: cur is
// z = 0 and the first step needs no product); cur / oth swap after every
// fused pass.
int cheb_steps(const MgLevel &L, const Cycle &c, const double *r, double *&cur, double *&oth, bool from_zero,
               hipStream_t s) {
    const double lam2 = L.gersh, lam1 = c.lower * lam2;
    const double sigma = (lam1 + lam2) / (lam2 - lam1), w0 = 2.0 / (lam1 + lam2), w = 4.0 / (lam2 - lam1);
    if (from_zero) {
        const int64_t n = level_nodes(L);
        k_cheb_first<<<grid_for(n), kBlock, 0, s>>>(n, w0, L.dinv, r, cur, L.c);
        FEM_HIP_CHECK(hipGetLastError());
    } else {
        if (int rc = level_pass(L, OpCheb{cur, r, L.dinv, oth, L.c, L.P.mask, 0.0, w0}, c.f32, s)) return rc;
        std::swap(cur, oth);
    }
    double rho = 1.0 / sigma;
    for (int k = 1; k < c.smooth; ++k) {
        const double ck = 1.0 / (2.0 * sigma - rho);  // C_k / C_{k+1}
        if (int rc = level_pass(L, OpCheb{cur, r, L.dinv, oth, L.c, L.P.mask, rho * ck, w * ck}, c.f32, s))
            return rc;
        std::swap(cur, oth);
        rho = ck;
    }
    return 0;
}

// The smoothing steps alternate between z and the level's t, starting in t
// so that the 2 smooth - 1 fused steps end in z; the restricted residual
// r - A z goes to whichever of the two does not hold the iterate.
int vcycle(fem_mg *mg, size_t l, const double *r, double *z, const Cycle &c, hipStream_t s) {
    MgLevel &L = mg->lv[l];
    const int64_t n = level_nodes(L);
    const int gv = grid_for(n);
    if (l + 1 == mg->lv.size()) {
        k_dense_mv<<<(mg->nc + kBlock / kWave - 1) / (kBlock / kWave), kBlock, 0, s>>>(mg->nc, mg->Ainv, r, z);
        FEM_HIP_CHECK(hipGetLastError());
        return 0;
    }
    const bool cheb = c.smoother == FEM_SMOOTH_CHEBYSHEV;
    double *cur = L.t, *oth = z;
    if (cheb) {
        if (int rc = cheb_steps(L, c, r, cur, oth, true, s)) return rc;
    } else {
        k_smooth<<<gv, kBlock, 0, s>>>(n, c.omega, L.dinv, r, cur, 1);
        for (int k = 1; k < c.smooth; ++k) {
            if (int rc = smooth_step(L, r, cur, oth, c.omega, c.f32, s)) return rc;
            std::swap(cur, oth);
        }
    }
    if (int rc = level_pass(L, OpResid{cur, r, oth, L.P.mask}, c.f32, s)) return rc;
    MgLevel &C = mg->lv[l + 1];
    if (int rc = restrict_to(C, oth, C.r, s)) return rc;
    if (int rc = vcycle(mg, l + 1, C.r, C.z, c, s)) return rc;
    if (int rc = prolong_add(L, C, C.z, cur, s)) return rc;
    if (cheb) {
        if (int rc = cheb_steps(L, c, r, cur, oth, false, s)) return rc;
    } else {
        for (int k = 0; k < c.smooth; ++k) {
            if (int rc = smooth_step(L, r, cur, oth, c.omega, c.f32, s)) return rc;
            std::swap(cur, oth);
        }
    }
    if (cur != z) return set_error(FEM_EINVAL, "internal error: smoothing ended outside z");
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

// Options -> the cycle; FEM_EINVAL for parameters outside their ranges.
int cycle_from(const fem_mg_opts *o, Cycle &c) {
    if (o->smooth < 1 || o->smooth > 64) return set_error(FEM_EINVAL, "smooth must be in [1, 64]");
    if (o->cycle_dtype != FEM_F64 && o->cycle_dtype != FEM_F32)
        return set_error(FEM_EINVAL, "cycle_dtype: FEM_F64 or FEM_F32");
    if (o->smoother == FEM_SMOOTH_JACOBI) {
        if (!(o->omega > 0.0 && o->omega < 2.0)) return set_error(FEM_EINVAL, "omega must be in (0, 2)");
    } else if (o->smoother == FEM_SMOOTH_CHEBYSHEV) {
        if (!(o->cheb_lower > 0.0 && o->cheb_lower < 1.0)) return set_error(FEM_EINVAL, "cheb_lower must be in (0, 1)");
    } else {
        return set_error(FEM_EINVAL, "smoother: FEM_SMOOTH_JACOBI or FEM_SMOOTH_CHEBYSHEV");
    }
    c = Cycle{o->smooth, o->omega, o->cycle_dtype == FEM_F32, o->smoother, o->cheb_lower};
    return 0;
}

// g of level L: one element pass of |A_e| over the all-ones vector into the
// level's t, then the maximum of D^-1 times it over free nodes (a level
// without free nodes keeps g = 1: its smoothing is zero either way).
int level_gersh(MgLevel &L, double *part, hipStream_t s) {
    const int64_t n = level_nodes(L);
    const DevPlan &P = L.P;
    const size_t lds = P.nb == 4 ? chunk_lds_bytes<4, double>(P.E) : chunk_lds_bytes<3, double>(P.E);
    const ChunkGrid cg = chunk_grid(P.n_chunks, lds);
    const OpAbsRow op{L.t};
    int rc = dispatch_ept(P.E, [&](auto ept) -> int {
        constexpr int EPT = decltype(ept)::value;
        if (P.nb == 4) {
            LdAbs<4> ld{{L.A, P.n_elems}};
            k_chunk_main<4, EPT, kBlock, double, LdAbs<4>, OpAbsRow, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, L.scratch, cg.xcd);
        } else {
            LdAbs<3> ld{{L.A, P.n_elems}};
            k_chunk_main<3, EPT, kBlock, double, LdAbs<3>, OpAbsRow, false>
                <<<cg.grid, kBlock, lds, s>>>(P, ld, op, L.scratch, cg.xcd);
        }
        return 0;
    });
    if (rc) return rc;
    FEM_HIP_CHECK(hipGetLastError());
    if (P.n_shared > 0) {
        k_chunk_fixup<kFixBlock, double, OpAbsRow><<<fixup_grid(P.n_shared), kFixBlock, 0, s>>>(P, op, L.scratch, 0);
        FEM_HIP_CHECK(hipGetLastError());
    }
    const int g = grid_for(n);
    k_gersh<<<g, kBlock, 0, s>>>(n, L.t, L.dinv, L.P.mask, part);
    FEM_HIP_CHECK(hipGetLastError());
    std::vector<double> h(g);
    FEM_HIP_CHECK(hipMemcpyAsync(h.data(), part, g * sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    const double m = *std::max_element(h.begin(), h.end());
    L.gersh = m > 0.0 ? m : 1.0;
    return 0;
}

}  // namespace

int mg_galerkin_apply(fem_mg *mg, int l, const double *zc, double *out, hipStream_t s) {
    MgLevel &F = mg->lv[l], &C = mg->lv[l + 1];
    const int64_t nf = level_nodes(F);
    const int gv = grid_for(nf);
    k_unit<<<gv, kBlock, 0, s>>>(nf, -1, F.z);  // zero
    if (int rc = prolong_add(F, C, zc, F.z, s)) return rc;
    if (int rc = launch_apply_pk64(F.P, MAT_F64, F.A, F.z, nullptr, F.t, 1.0, 1, F.scratch, s)) return rc;
    return restrict_to(C, F.t, out, s);
}

}  // namespace fem

namespace {
fem_plan_stats plan_stats(const fem_plan *p) {
    fem_plan_stats st{};
    (void)fem_plan_get_stats(p, &st);
    return st;
}
}  // namespace

extern "C" {

void fem_mg_opts_default(fem_mg_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-8;
    o->max_iter = 500;
    o->smooth = 2;
    o->omega = 2.0 / 3.0;
    o->max_replace = 4;
    o->cycle_dtype = FEM_F64;
    o->smoother = FEM_SMOOTH_JACOBI;
    o->cheb_lower = 0.3;
}

int fem_mg_create(int levels, const fem_plan *const *plans, const int *grid_n, int dtype, const void *const *K,
                  const void *const *M, double nu, void *stream, fem_mg **out) {
    using fem::set_error;
    fem::last_error().clear();
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (levels < 2 || levels > 16 || !plans || !grid_n || !K) return set_error(FEM_EINVAL, "bad level list");
    if (dtype != FEM_F64 && dtype != FEM_F32 && dtype != FEM_F32X2) return set_error(FEM_EINVAL, "unknown dtype");
    if (!std::isfinite(nu) || nu < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    int dim0 = 0;
    for (int l = 0; l < levels; ++l) {
        if (!plans[l] || !K[l] || (nu != 0.0 && (!M || !M[l]))) return set_error(FEM_EINVAL, "NULL plan or matrix");
        const fem_plan_stats st = plan_stats(plans[l]);
        const int64_t g = grid_n[l], m = g + 1;
        const bool sq = st.dim == 2 && st.n_b == 3 && st.n_nodes == m * m && st.n_elems == 2 * g * g;
        const bool cu = st.dim == 3 && st.n_b == 4 && st.n_nodes == m * m * m && st.n_elems == 6 * g * g * g;
        if (g < 1 || !(sq || cu))
            return set_error(FEM_EINVAL, "level " + std::to_string(l) +
                                             " is not an n x n diagonal-cut square mesh or an n^3 Kuhn cube mesh");
        if (l > 0 && st.dim != dim0) return set_error(FEM_EINVAL, "all levels must have the same dimension");
        if (l == 0) dim0 = st.dim;
        if (l > 0 && grid_n[l - 1] != 2 * grid_n[l])
            return set_error(FEM_EINVAL, "each level must halve the squares (cubes) per side");
    }
    const int mcs = grid_n[levels - 1] + 1;
    const int nc = dim0 == 3 ? mcs * mcs * mcs : mcs * mcs;
    if (nc > 1089) return set_error(FEM_EINVAL, "the coarsest level may have at most 1089 nodes (33^2, 10^3)");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    fem_mg *mg = new (std::nothrow) fem_mg();
    if (!mg) return set_error(FEM_ENOMEM, "host allocation failed");
    mg->lv.resize(levels);
    mg->nc = nc;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return o;
    };
    std::vector<size_t> oA(levels), oA32(levels), od(levels), odi(levels), or_(levels), oz(levels), ot(levels),
        oc(levels), osc(levels);
    for (int l = 0; l < levels; ++l) {
        mg->lv[l].P = fem::plan_device(plans[l]);
        mg->lv[l].n = grid_n[l];
        mg->lv[l].dim = dim0;
        const fem::DevPlan &P = mg->lv[l].P;
        const int64_t n = P.n_nodes;
        oA[l] = take((size_t)fem::packed_count(P.nb) * P.n_elems * 8);
        oA32[l] = take((size_t)fem::packed_count(P.nb) * P.n_elems * 8);  // float [2][np][ne]
        od[l] = take(n * 8);
        odi[l] = take(n * 8);
        or_[l] = take(n * 8);
        oz[l] = take(n * 8);
        ot[l] = take(n * 8);
        oc[l] = take(n * 8);
        osc[l] = take(std::max<int64_t>(P.n_partials, 1) * 8);
    }
    const int64_t n0 = mg->lv[0].P.n_nodes;
    const size_t oinv = take((size_t)nc * nc * 8), ocol = take((size_t)nc * nc * 8), op = take(n0 * 8),
                 oq = take(n0 * 8), opart = take((size_t)fem::kDotBlocks * 4 * 8), osum = take(8 * 8),
                 optr = take(16 * sizeof(void *)), obad = take(sizeof(int));
    if (hipMalloc(&mg->arena, off) != hipSuccess) {
        (void)hipGetLastError();
        delete mg;
        return set_error(FEM_ENOMEM, "device allocation of the multigrid workspace failed");
    }
    char *b = static_cast<char *>(mg->arena);
    for (int l = 0; l < levels; ++l) {
        fem::MgLevel &L = mg->lv[l];
        L.A = reinterpret_cast<double *>(b + oA[l]);
        L.A32 = b + oA32[l];
        L.dinv = reinterpret_cast<double *>(b + odi[l]);
        L.r = reinterpret_cast<double *>(b + or_[l]);
        L.z = reinterpret_cast<double *>(b + oz[l]);
        L.t = reinterpret_cast<double *>(b + ot[l]);
        L.c = reinterpret_cast<double *>(b + oc[l]);
        L.scratch = reinterpret_cast<double *>(b + osc[l]);
    }
    mg->Ainv = reinterpret_cast<double *>(b + oinv);
    double *cols = reinterpret_cast<double *>(b + ocol);
    mg->p = reinterpret_cast<double *>(b + op);
    mg->q = reinterpret_cast<double *>(b + oq);
    mg->part = reinterpret_cast<double *>(b + opart);
    mg->sums = reinterpret_cast<double *>(b + osum);
    mg->ptrs = reinterpret_cast<const double **>(b + optr);
    mg->bad = reinterpret_cast<int *>(b + obad);
    auto fail = [&](int rc) {
        delete mg;
        return rc;
    };
    int rc = 0;
    if (hipMemsetAsync(mg->bad, 0, sizeof(int), s) != hipSuccess) rc = set_error(FEM_EHIP, "memset failed");
    for (int l = 0; l < levels && !rc; ++l) {
        fem::MgLevel &L = mg->lv[l];
        const void *Ml = nu != 0.0 ? M[l] : nullptr;
        rc = fem::launch_pack(L.P, dtype, K[l], Ml, nu, fem::MAT_F64, L.A, s);
        if (!rc) rc = fem::launch_pack(L.P, dtype, K[l], Ml, nu, fem::MAT_F32X2, L.A32, s);
        if (!rc) rc = fem::launch_diag_pk64(L.P, fem::MAT_F64, L.A, reinterpret_cast<double *>(b + od[l]), L.scratch, s);
        if (!rc) {
            fem::k_dinv_fcg<<<fem::grid_for(L.P.n_nodes), fem::kBlock, 0, s>>>(
                L.P.n_nodes, reinterpret_cast<double *>(b + od[l]), L.P.mask, L.dinv, mg->bad);
            if (hipGetLastError() != hipSuccess) rc = set_error(FEM_EHIP, "kernel launch failed");
        }
    }
    if (rc) return fail(rc);
    int bad = 0;
    if (hipMemcpyAsync(&bad, mg->bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(FEM_EHIP, "setup of the multigrid levels failed"));
    }
    if (bad) return fail(set_error(FEM_ESINGULAR, "a free node has a non-positive diagonal entry"));
    for (int l = 0; l < levels && !rc; ++l) rc = fem::level_gersh(mg->lv[l], mg->part, s);
    if (rc) return fail(rc);
    // coarsest level: columns of the masked operator, Dirichlet rows / columns identity
    fem::MgLevel &C = mg->lv[levels - 1];
    for (int j = 0; j < nc && !rc; ++j) {
        fem::k_unit<<<fem::grid_for(nc), fem::kBlock, 0, s>>>(nc, j, C.z);
        rc = fem::launch_apply_pk64(C.P, fem::MAT_F64, C.A, C.z, nullptr, cols + (size_t)j * nc, 1.0, 1, C.scratch, s);
    }
    if (rc) return fail(rc);
    std::vector<double> colh((size_t)nc * nc);
    std::vector<uint8_t> mk(nc);
    if (hipMemcpyAsync(colh.data(), cols, colh.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(mk.data(), C.P.mask, nc, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(FEM_EHIP, "download of the coarse operator failed"));
    }
    std::vector<double> a((size_t)nc * nc), inv;
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) {
            double v = colh[(size_t)j * nc + i];  // column j, row i
            if (mk[i] || mk[j]) v = (i == j) ? 1.0 : 0.0;
            a[(size_t)i * nc + j] = v;
        }
    if (!fem::invert(nc, a, inv)) return fail(set_error(FEM_ESINGULAR, "the coarsest operator is singular"));
    if (hipMemcpyAsync(mg->Ainv, inv.data(), inv.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(FEM_EHIP, "upload of the coarse inverse failed"));
    }
    *out = mg;
    return FEM_OK;
}

int fem_mg_destroy(fem_mg *mg) {
    delete mg;
    return FEM_OK;
}

int fem_mg_galerkin_apply(fem_mg *mg, int level, const double *d_zc, double *d_out, void *stream) {
    using fem::set_error;
    if (!mg || !d_zc || !d_out) return set_error(FEM_EINVAL, "NULL argument");
    if (level < 0 || level + 1 >= (int)mg->lv.size()) return set_error(FEM_EINVAL, "bad level");
    return fem::mg_galerkin_apply(mg, level, d_zc, d_out, reinterpret_cast<hipStream_t>(stream));
}

int fem_mg_vcycle(fem_mg *mg, const fem_mg_opts *opts, const double *d_r, double *d_z, void *stream) {
    using fem::set_error;
    fem::last_error().clear();
    if (!mg || !opts || !d_r || !d_z) return set_error(FEM_EINVAL, "NULL argument");
    if (d_r == d_z) return set_error(FEM_EINVAL, "r and z must not alias");
    fem::Cycle c{};
    if (int rc = fem::cycle_from(opts, c)) return rc;
    return fem::vcycle(mg, 0, d_r, d_z, c, reinterpret_cast<hipStream_t>(stream));
}

int fem_mg_level_bound(const fem_mg *mg, int level, double *g) {
    using fem::set_error;
    fem::last_error().clear();
    if (!mg || !g) return set_error(FEM_EINVAL, "NULL argument");
    if (level < 0 || level >= (int)mg->lv.size()) return set_error(FEM_EINVAL, "bad level");
    *g = mg->lv[level].gersh;
    return FEM_OK;
}

int fem_mg_solve(fem_mg *mg, const fem_mg_opts *o, const double *d_b, double *d_x, fem_fcg_info *info, void *stream) {
    using namespace fem;
    auto t0 = std::chrono::steady_clock::now();
    last_error().clear();
    if (!mg || !o || !info || !d_b || !d_x) return set_error(FEM_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->fell_back = -1;
    if (!(o->rtol > 0.0 && o->rtol < 1.0) || o->max_iter < 1 || o->max_replace < 0)
        return set_error(FEM_EINVAL, "bad multigrid options");
    Cycle cyc{};
    if (int rc = cycle_from(o, cyc)) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    MgLevel &F = mg->lv[0];
    const DevPlan &P = F.P;
    const int64_t n = P.n_nodes;
    const int gv = grid_for(n);
    double *r = F.r, *z = F.z, *p = mg->p, *q = mg->q;
    // the finest level's r / z are the FCG residual and preconditioned residual;
    // the V-cycle from level 0 reads r and writes z, using level-0 t as scratch.
    // Dot tables: [0..2] x [3..5] = (z.r, z.p, z.q); [6..7] x [8..9] = (p.q, p.r); [3] x [3] = r.r
    const double *tab[16] = {z, z, z, r, p, q, p, p, q, r};
    FEM_HIP_CHECK(hipMemcpyAsync(mg->ptrs, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    // the first iteration's z.p and z.q read the previous direction: defined zeros
    FEM_HIP_CHECK(hipMemsetAsync(p, 0, n * 8, s));
    FEM_HIP_CHECK(hipMemsetAsync(q, 0, n * 8, s));
    double h[8];
    auto fetch = [&](int cnt) -> int {
        FEM_HIP_CHECK(hipMemcpyAsync(h, mg->sums, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        return 0;
    };
    auto true_residual = [&](double &rn) -> int {
        if (int rc = launch_apply_pk64(P, MAT_F64, F.A, d_x, d_b, r, -1.0, 1, F.scratch, s)) return rc;
        k_dots<1><<<gv, kBlock, 0, s>>>(n, mg->ptrs + 3, mg->ptrs + 3, mg->part);
        k_dots_fin<<<1, kBlock, 0, s>>>(mg->part, gv, 1, mg->sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(1)) return rc;
        rn = std::sqrt(h[0]);
        return 0;
    };
    int status = FEM_OK;
    double rn = 0.0;
    auto finish = [&](int st) {
        info->status = st;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return st;
    };
    if (int rc = true_residual(rn)) return finish(rc);
    info->r0 = rn;
    if (!std::isfinite(rn)) return finish(set_error(FEM_EBREAKDOWN, "non-finite initial residual"));
    if (rn == 0.0) return finish(FEM_OK);
    const double target = fem::kCertify * o->rtol * rn;
    bool restart = true;
    double pq_prev = 1.0;
    for (int it = 0; it < o->max_iter; ++it) {
        if (int rc = vcycle(mg, 0, r, z, cyc, s)) return finish(rc);
        info->precond_calls += 1;
        k_dots<3><<<gv, kBlock, 0, s>>>(n, mg->ptrs, mg->ptrs + 3, mg->part);  // z.r, z.p, z.q
        k_dots_fin<<<1, kBlock, 0, s>>>(mg->part, gv, 3, mg->sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(3)) return finish(rc);
        const double zr = h[0], zq = h[2];
        if (!(std::isfinite(zr) && zr > 0.0)) return finish(set_error(FEM_EBREAKDOWN, "r.z <= 0 in MG-FCG"));
        if (restart) {
            FEM_HIP_CHECK(hipMemcpyAsync(p, z, n * 8, hipMemcpyDeviceToDevice, s));
        } else {
            k_dir<<<gv, kBlock, 0, s>>>(n, z, zq / pq_prev, p);
        }
        restart = false;
        if (int rc = launch_apply_pk64(P, MAT_F64, F.A, p, nullptr, q, 1.0, 1, F.scratch, s)) return finish(rc);
        k_dots<2><<<gv, kBlock, 0, s>>>(n, mg->ptrs + 6, mg->ptrs + 8, mg->part);
        k_dots_fin<<<1, kBlock, 0, s>>>(mg->part, gv, 2, mg->sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(2)) return finish(rc);
        const double pq = h[0], pr = h[1];
        if (!(std::isfinite(pq) && pq > 0.0 && std::isfinite(pr)))
            return finish(set_error(FEM_EBREAKDOWN, "p.q <= 0 in MG-FCG"));
        const double alpha = pr / pq;
        pq_prev = pq;
        k_step<<<gv, kBlock, 0, s>>>(n, alpha, p, q, d_x, r, mg->part);
        k_dots_fin<<<1, kBlock, 0, s>>>(mg->part, gv, 1, mg->sums);
        FEM_HIP_CHECK(hipGetLastError());
        if (int rc = fetch(1)) return finish(rc);
        rn = std::sqrt(h[0]);
        info->iters = it + 1;
        if (!std::isfinite(rn)) return finish(set_error(FEM_EBREAKDOWN, "non-finite residual in MG-FCG"));
        if (rn <= target) {
            double rt = 0.0;
            if (int rc = true_residual(rt)) return finish(rc);
            rn = rt;
            if (rt <= target) {
                info->relres = rt / info->r0;
                return finish(FEM_OK);
            }
            if (info->replacements >= o->max_replace) break;
            info->replacements += 1;
            restart = true;
        }
    }
    double rt = 0.0;
    if (int rc = true_residual(rt)) return finish(rc);
    info->relres = rt / info->r0;
    status = rt <= target ? FEM_OK : FEM_ENOCONV;
    if (status == FEM_ENOCONV) set_error(FEM_ENOCONV, "MG-FCG reached the iteration limit");
    return finish(status);
}

}  // extern "C"
