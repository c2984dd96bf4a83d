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

// Quadratic (P2) triangles.  With barycentric coordinates lambda_0..2 the six
// Lagrange functions are phi_k = lambda_k (2 lambda_k - 1) (vertices) and
// phi_{3+e} = 4 lambda_u lambda_v for the edges e = (0,1), (1,2), (2,0).  Their
// gradients are sum_a c_ka grad(lambda_a) with factors c_ka linear in lambda,
// so K_ij = area * sum_ab (grad lambda_a . grad lambda_b) S[i][a][j][b] with
// S[i][a][j][b] = (1/area) int c_ia c_jb, and M_ij = area * Mref[i][j] with
// Mref[i][j] = (1/area) int phi_i phi_j.  Both tables are integrals of
// barycentric monomials, (1/area) int lambda^alpha = 2 alpha! / (|alpha| + 2)!,
// evaluated at compile time.
struct P2Tables {
    double S[6][3][6][3];
    double M[6][6];
};

constexpr double p2_fact(int n) { return n <= 1 ? 1.0 : n * p2_fact(n - 1); }

// (1/area) int over the triangle of lambda_0^a0 lambda_1^a1 lambda_2^a2
constexpr double p2_mono(int a0, int a1, int a2) {
    return 2.0 * p2_fact(a0) * p2_fact(a1) * p2_fact(a2) / p2_fact(a0 + a1 + a2 + 2);
}

constexpr P2Tables p2_tables() {
    P2Tables t{};
    // c_ka = sum_p A[k][a][p] lambda_p + B[k][a]
    double A[6][3][3] = {};
    double B[6][3] = {};
    const int eu[3] = {0, 1, 2}, ev[3] = {1, 2, 0};
    for (int k = 0; k < 3; ++k) {
        A[k][k][k] = 4.0;
        B[k][k] = -1.0;
    }
    for (int e = 0; e < 3; ++e) {
        A[3 + e][eu[e]][ev[e]] = 4.0;
        A[3 + e][ev[e]][eu[e]] = 4.0;
    }
    for (int i = 0; i < 6; ++i)
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 6; ++j)
                for (int b = 0; b < 3; ++b) {
                    double v = B[i][a] * B[j][b];
                    for (int p = 0; p < 3; ++p) {
                        int ep[3] = {0, 0, 0};
                        ep[p] = 1;
                        v += (A[i][a][p] * B[j][b] + B[i][a] * A[j][b][p]) * p2_mono(ep[0], ep[1], ep[2]);
                        for (int q = 0; q < 3; ++q) {
                            int eq[3] = {ep[0], ep[1], ep[2]};
                            eq[q] += 1;
                            v += A[i][a][p] * A[j][b][q] * p2_mono(eq[0], eq[1], eq[2]);
                        }
                    }
                    t.S[i][a][j][b] = v;
                }
    // phi_k as a quadratic form in lambda: phi_k = sum_pq C[k][p][q] lambda_p lambda_q
    // (lambda_k (2 lambda_k - 1) = lambda_k^2 - sum_{m != k} lambda_k lambda_m, since sum lambda = 1)
    double C[6][3][3] = {};
    for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) {
            if (m == k) C[k][k][k] = 1.0;
            else {
                C[k][k][m] = -0.5;
                C[k][m][k] = -0.5;
            }
        }
    for (int e = 0; e < 3; ++e) {
        C[3 + e][eu[e]][ev[e]] = 2.0;
        C[3 + e][ev[e]][eu[e]] = 2.0;
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double v = 0.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    for (int r = 0; r < 3; ++r)
                        for (int u = 0; u < 3; ++u) {
                            const double c = C[i][p][q] * C[j][r][u];
                            if (c == 0.0) continue;
                            int ex[3] = {0, 0, 0};
                            ex[p] += 1;
                            ex[q] += 1;
                            ex[r] += 1;
                            ex[u] += 1;
                            v += c * p2_mono(ex[0], ex[1], ex[2]);
                        }
            t.M[i][j] = v;
        }
    return t;
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_local_matrices_p2(const double *__restrict__ coords,
                                                              const int32_t *__restrict__ conn,
                                                              int64_t n_nodes, int64_t n_elems,
                                                              void *__restrict__ K, void *__restrict__ M,
                                                              double *__restrict__ vol) {
    constexpr int NB = 6;
    constexpr P2Tables T = p2_tables();
    const int64_t blk = (int64_t)NB * NB * n_elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        double p[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int32_t v = conn[(int64_t)a * n_elems + e];
            p[a][0] = coords[v];
            p[a][1] = coords[n_nodes + v];
        }
        const double b00 = p[1][0] - p[0][0], b01 = p[2][0] - p[0][0];
        const double b10 = p[1][1] - p[0][1], b11 = p[2][1] - p[0][1];
        const double det = b00 * b11 - b01 * b10;
        // grad lambda_1, grad lambda_2 are the rows of B^{-1}; grad lambda_0 = -(their sum)
        double G[3][2];
        G[1][0] = b11 / det;
        G[1][1] = -b01 / det;
        G[2][0] = -b10 / det;
        G[2][1] = b00 / det;
        G[0][0] = -(G[1][0] + G[2][0]);
        G[0][1] = -(G[1][1] + G[2][1]);
        const double area = 0.5 * fabs(det);
        if (K) {
            double g[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) g[a][b] = G[a][0] * G[b][0] + G[a][1] * G[b][1];
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    double v = 0.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b)
                            if (T.S[i][a][j][b] != 0.0) v += T.S[i][a][j][b] * g[a][b];
                    store_entry<KIND>(K, (int64_t)(i * NB + j) * n_elems + e, blk, area * v);
                }
        }
        if (M) {
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    store_entry<KIND>(M, (int64_t)(i * NB + j) * n_elems + e, blk, area * T.M[i][j]);
        }
        if (vol) vol[e] = area;
    }
}

// Quadratic (P2) tetrahedra: the ten functions phi_k = lambda_k (2 lambda_k - 1)
// (vertices k = 0..3) and phi_{4+e} = 4 lambda_u lambda_v for the edges
// e = (0,1), (0,2), (0,3), (1,2), (1,3), (2,3).  As for triangles, the
// gradients are sum_a c_ka grad(lambda_a) with c_ka linear in lambda, and
// the tables hold (1/vol) int c_ia c_jb and (1/vol) int phi_i phi_j, from
// (1/vol) int lambda^alpha = 6 alpha! / (|alpha| + 3)!.
struct P2TetTables {
    double S[10][4][10][4];
    double M[10][10];
};

// n! for n <= 8 (the largest argument is |alpha| + 3 = 7)
struct FactTable {
    double v[9];
};
constexpr FactTable fact_table() {
    FactTable t{};
    t.v[0] = 1.0;
    for (int n = 1; n < 9; ++n) t.v[n] = n * t.v[n - 1];
    return t;
}

// (1/vol) int over the tetrahedron of lambda_0^a0 .. lambda_3^a3
constexpr double p2t_mono(const int (&a)[4]) {
    constexpr FactTable F = fact_table();
    return 6.0 * F.v[a[0]] * F.v[a[1]] * F.v[a[2]] * F.v[a[3]] / F.v[a[0] + a[1] + a[2] + a[3] + 3];
}

constexpr P2TetTables p2_tet_tables() {
    P2TetTables t{};
    const int eu[6] = {0, 0, 0, 1, 1, 2}, ev[6] = {1, 2, 3, 2, 3, 3};
    // c_ka = sum_p A[k][a][p] lambda_p + B[k][a]
    double A[10][4][4] = {};
    double B[10][4] = {};
    for (int k = 0; k < 4; ++k) {
        A[k][k][k] = 4.0;
        B[k][k] = -1.0;
    }
    for (int e = 0; e < 6; ++e) {
        A[4 + e][eu[e]][ev[e]] = 4.0;
        A[4 + e][ev[e]][eu[e]] = 4.0;
    }
    for (int i = 0; i < 10; ++i)
        for (int a = 0; a < 4; ++a)
            for (int j = 0; j < 10; ++j)
                for (int b = 0; b < 4; ++b) {
                    double v = B[i][a] * B[j][b];  // (1/vol) int 1 = 1
                    for (int p = 0; p < 4; ++p) {
                        int ep[4] = {0, 0, 0, 0};
                        ep[p] = 1;
                        v += (A[i][a][p] * B[j][b] + B[i][a] * A[j][b][p]) * p2t_mono(ep);
                        for (int q = 0; q < 4; ++q) {
                            int eq[4] = {ep[0], ep[1], ep[2], ep[3]};
                            eq[q] += 1;
                            v += A[i][a][p] * A[j][b][q] * p2t_mono(eq);
                        }
                    }
                    t.S[i][a][j][b] = v;
                }
    // phi_k as a quadratic form in lambda (sum lambda = 1 turns the linear term into products)
    double C[10][4][4] = {};
    for (int k = 0; k < 4; ++k)
        for (int m = 0; m < 4; ++m) {
            if (m == k) C[k][k][k] = 1.0;
            else {
                C[k][k][m] = -0.5;
                C[k][m][k] = -0.5;
            }
        }
    for (int e = 0; e < 6; ++e) {
        C[4 + e][eu[e]][ev[e]] = 2.0;
        C[4 + e][ev[e]][eu[e]] = 2.0;
    }
    for (int i = 0; i < 10; ++i)
        for (int j = 0; j < 10; ++j) {
            double v = 0.0;
            for (int p = 0; p < 4; ++p)
                for (int q = 0; q < 4; ++q)
                    for (int r = 0; r < 4; ++r)
                        for (int u = 0; u < 4; ++u) {
                            const double c = C[i][p][q] * C[j][r][u];
                            if (c == 0.0) continue;
                            int ex[4] = {0, 0, 0, 0};
                            ex[p] += 1;
                            ex[q] += 1;
                            ex[r] += 1;
                            ex[u] += 1;
                            v += c * p2t_mono(ex);
                        }
            t.M[i][j] = v;
        }
    return t;
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_local_matrices_p2_tet(const double *__restrict__ coords,
                                                                  const int32_t *__restrict__ conn,
                                                                  int64_t n_nodes, int64_t n_elems,
                                                                  void *__restrict__ K, void *__restrict__ M,
                                                                  double *__restrict__ vol) {
    constexpr int NB = 10;
    constexpr P2TetTables T = p2_tet_tables();
    const int64_t blk = (int64_t)NB * NB * n_elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        double p[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int32_t v = conn[(int64_t)a * n_elems + e];
#pragma unroll
            for (int d = 0; d < 3; ++d) p[a][d] = coords[(int64_t)d * n_nodes + v];
        }
        double b[3][3];  // b[r][c]: component r of edge vector c
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) b[r][c] = p[c + 1][r] - p[0][r];
        const double c00 = b[1][1] * b[2][2] - b[1][2] * b[2][1];
        const double c01 = b[1][2] * b[2][0] - b[1][0] * b[2][2];
        const double c02 = b[1][0] * b[2][1] - b[1][1] * b[2][0];
        const double det = b[0][0] * c00 + b[0][1] * c01 + b[0][2] * c02;
        // rows of B^{-1} are grad lambda_1..3 (adjugate / det); grad lambda_0 = -(their sum)
        double G[4][3];
        G[1][0] = c00 / det;
        G[2][0] = c01 / det;
        G[3][0] = c02 / det;
        G[1][1] = (b[0][2] * b[2][1] - b[0][1] * b[2][2]) / det;
        G[2][1] = (b[0][0] * b[2][2] - b[0][2] * b[2][0]) / det;
        G[3][1] = (b[0][1] * b[2][0] - b[0][0] * b[2][1]) / det;
        G[1][2] = (b[0][1] * b[1][2] - b[0][2] * b[1][1]) / det;
        G[2][2] = (b[0][2] * b[1][0] - b[0][0] * b[1][2]) / det;
        G[3][2] = (b[0][0] * b[1][1] - b[0][1] * b[1][0]) / det;
#pragma unroll
        for (int d = 0; d < 3; ++d) G[0][d] = -(G[1][d] + G[2][d] + G[3][d]);
        const double ve = fabs(det) / 6.0;
        if (K) {
            double g[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) g[a][c] = G[a][0] * G[c][0] + G[a][1] * G[c][1] + G[a][2] * G[c][2];
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    double v = 0.0;
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (T.S[i][a][j][c] != 0.0) v += T.S[i][a][j][c] * g[a][c];
                    store_entry<KIND>(K, (int64_t)(i * NB + j) * n_elems + e, blk, ve * v);
                }
        }
        if (M) {
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    store_entry<KIND>(M, (int64_t)(i * NB + j) * n_elems + e, blk, ve * T.M[i][j]);
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
#define FEM_LM2(KND) \
    k_local_matrices_p2<KND><<<g, kBlock, 0, s>>>(P.coords, P.conn, P.n_nodes, P.n_elems, K, M, vol)
#define FEM_LM3(KND) \
    k_local_matrices_p2_tet<KND><<<g, kBlock, 0, s>>>(P.coords, P.conn, P.n_nodes, P.n_elems, K, M, vol)
    if (P.nb == 10) {
        if (kind == MAT_F64) FEM_LM3(MAT_F64);
        else if (kind == MAT_F32) FEM_LM3(MAT_F32);
        else FEM_LM3(MAT_F32X2);
    } else if (P.nb == 6) {
        if (kind == MAT_F64) FEM_LM2(MAT_F64);
        else if (kind == MAT_F32) FEM_LM2(MAT_F32);
        else FEM_LM2(MAT_F32X2);
    } else if (P.dim == 2) {
        if (kind == MAT_F64) FEM_LM(2, MAT_F64);
        else if (kind == MAT_F32) FEM_LM(2, MAT_F32);
        else FEM_LM(2, MAT_F32X2);
    } else {
        if (kind == MAT_F64) FEM_LM(3, MAT_F64);
        else if (kind == MAT_F32) FEM_LM(3, MAT_F32);
        else FEM_LM(3, MAT_F32X2);
    }
#undef FEM_LM
#undef FEM_LM2
#undef FEM_LM3
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
    else if (P.nb == 4) FEM_CB_IN(4);
    else if (P.nb == 6) FEM_CB_IN(6);
    else FEM_CB_IN(10);
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
    else if (P.nb == 4) FEM_PK_IN(4);
    else if (P.nb == 6) FEM_PK_IN(6);
    else FEM_PK_IN(10);
#undef FEM_PK_IN
#undef FEM_PK_OUT
#undef FEM_PK
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace fem
