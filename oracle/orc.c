/*
 * orc.c -- plain FP64 CPU oracle for the element-based solvers of
 * Marcinkowski & Valdman, "MATLAB Implementation of Element-based Solvers".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the GPU
 * library.  Everything is double precision, one thread, straightforward loops
 * in ascending element / node order, with no blocking or reordering.
 *
 * Conventions (the paper's array view, Section 1 / Fig. 2):
 *   coords  [n_nodes][dim]      node-major coordinates
 *   elems   [n_elems][nb]       0-based node ids of each element, nb = dim+1
 *   K, M    [n_elems][nb][nb]   one dense local matrix per element
 *   mask    [n_nodes]           1 on Dirichlet nodes (the set nd), else 0
 * Return values: 0 on success, a negative code on invalid input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOCONV (-3)
#define ORC_EBREAKDOWN (-5)

/* ------------------------------------------------------------------------ */
/* Local P1 matrices: eq. (2) of Section 1 restricted to one element.        */
/*                                                                          */
/* For the simplex with vertices p_0..p_d let B = [p_1-p_0, ..., p_d-p_0].   */
/* The barycentric coordinates are affine; their gradients are the rows of   */
/* G = D_ref * B^{-1} with D_ref = [-1 ... -1 ; I_d] (rows = reference       */
/* gradients).  With vol = |det B| / d!:                                     */
/*   K_e(i,j) = int_e grad(phi_i).grad(phi_j) = vol * (G G^T)(i,j)           */
/*   M_e(i,j) = int_e phi_i phi_j = vol/((d+1)(d+2)) * (1 + delta_ij)        */
/* (the second by the classical integral of products of barycentric coords). */
/* ------------------------------------------------------------------------ */
static int inverse_small(int d, const double *B, double *Binv, double *det_out)
{
    double det;
    if (d == 2) {
        det = B[0] * B[3] - B[1] * B[2];
        if (det == 0.0) return ORC_EINVAL;
        Binv[0] = B[3] / det;
        Binv[1] = -B[1] / det;
        Binv[2] = -B[2] / det;
        Binv[3] = B[0] / det;
    } else if (d == 3) {
        /* cofactor expansion, B row-major: B[r*3+c] */
        double c00 = B[4] * B[8] - B[5] * B[7];
        double c01 = -(B[3] * B[8] - B[5] * B[6]);
        double c02 = B[3] * B[7] - B[4] * B[6];
        double c10 = -(B[1] * B[8] - B[2] * B[7]);
        double c11 = B[0] * B[8] - B[2] * B[6];
        double c12 = -(B[0] * B[7] - B[1] * B[6]);
        double c20 = B[1] * B[5] - B[2] * B[4];
        double c21 = -(B[0] * B[5] - B[2] * B[3]);
        double c22 = B[0] * B[4] - B[1] * B[3];
        det = B[0] * c00 + B[1] * c01 + B[2] * c02;
        if (det == 0.0) return ORC_EINVAL;
        /* inverse = adjugate / det, adjugate = cofactor^T */
        Binv[0] = c00 / det; Binv[1] = c10 / det; Binv[2] = c20 / det;
        Binv[3] = c01 / det; Binv[4] = c11 / det; Binv[5] = c21 / det;
        Binv[6] = c02 / det; Binv[7] = c12 / det; Binv[8] = c22 / det;
    } else {
        return ORC_EINVAL;
    }
    *det_out = det;
    return ORC_OK;
}

int orc_local_matrices(int dim, int64_t n_nodes, int64_t n_elems, const double *coords,
                       const int32_t *elems, double *K, double *M, double *vol)
{
    if (dim != 2 && dim != 3) return ORC_EINVAL;
    const int nb = dim + 1;
    const double fact = (dim == 2) ? 2.0 : 6.0;           /* d! */
    const double mscale = 1.0 / (double)((dim + 1) * (dim + 2));
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *v = elems + e * nb;
        for (int a = 0; a < nb; ++a)
            if (v[a] < 0 || v[a] >= n_nodes) return ORC_EINVAL;
        /* B: column c is p_{c+1} - p_0, stored row-major B[r*dim + c] */
        double B[9], Binv[9], det;
        for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c)
                B[r * dim + c] = coords[(int64_t)v[c + 1] * dim + r] - coords[(int64_t)v[0] * dim + r];
        if (inverse_small(dim, B, Binv, &det) != ORC_OK) return ORC_EINVAL;
        const double ve = fabs(det) / fact;
        /* G (nb x dim): row 0 = -(sum of the rows of Binv), row k = row k-1 of Binv */
        double G[4][3];
        for (int c = 0; c < dim; ++c) {
            double s = 0.0;
            for (int k = 0; k < dim; ++k) s += Binv[k * dim + c];
            G[0][c] = -s;
            for (int k = 0; k < dim; ++k) G[k + 1][c] = Binv[k * dim + c];
        }
        double *Ke = K + e * nb * nb;
        double *Me = M ? M + e * nb * nb : NULL;
        for (int i = 0; i < nb; ++i) {
            for (int j = 0; j < nb; ++j) {
                double g = 0.0;
                for (int c = 0; c < dim; ++c) g += G[i][c] * G[j][c];
                Ke[i * nb + j] = ve * g;
                if (Me) Me[i * nb + j] = ve * mscale * (i == j ? 2.0 : 1.0);
            }
        }
        if (vol) vol[e] = ve;
    }
    return ORC_OK;
}

/* A_e := K_e + nu M_e (Section 2, definition under Algorithm 1). */
static inline double Aentry(const double *K, const double *M, double nu, int64_t e, int nb, int i, int j)
{
    double a = K[e * nb * nb + i * nb + j];
    if (M && nu != 0.0) a += nu * M[e * nb * nb + i * nb + j];
    return a;
}

static int check_elems(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems)
{
    for (int64_t k = 0; k < n_elems * nb; ++k)
        if (elems[k] < 0 || elems[k] >= n_nodes) return ORC_EINVAL;
    return ORC_OK;
}

/* Right-hand side b_j = int f phi_j (eq. (2)) with f taken as its nodal
 * interpolant, i.e. b_e = M_e f_e and b = sum_e C_e^T b_e (eq. (3)). */
int orc_rhs(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems, const double *M,
            const double *f, double *b)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    for (int64_t i = 0; i < n_nodes; ++i) b[i] = 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *v = elems + e * nb;
        for (int i = 0; i < nb; ++i) {
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += M[e * nb * nb + i * nb + j] * f[v[j]];
            b[v[i]] += s;
        }
    }
    return ORC_OK;
}

/* Local right-hand sides b_e = M_e f_e, stored [n_elems][nb]. */
int orc_rhs_local(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems, const double *M,
                  const double *f, double *be)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *v = elems + e * nb;
        for (int i = 0; i < nb; ++i) {
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += M[e * nb * nb + i * nb + j] * f[v[j]];
            be[e * nb + i] = s;
        }
    }
    return ORC_OK;
}

/* Algorithm 1 as printed: for every element restrict x (x_e = R_e x), form
 * the local residual r_e = b_e - A_e x_e, then assemble r = sum_e C_e^T r_e.
 * b_e are local right-hand sides [n_elems][nb]; NULL means b_e = 0. */
int orc_residual_alg1(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems,
                      const double *K, const double *M, double nu, const double *be,
                      const double *x, double *r)
{
    if (nb > 16 || check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    for (int64_t i = 0; i < n_nodes; ++i) r[i] = 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *v = elems + e * nb;
        double xe[16], re[16];
        for (int j = 0; j < nb; ++j) xe[j] = x[v[j]];                /* restriction */
        for (int i = 0; i < nb; ++i) {                                /* local residual */
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += Aentry(K, M, nu, e, nb, i, j) * xe[j];
            re[i] = (be ? be[e * nb + i] : 0.0) - s;
        }
        for (int i = 0; i < nb; ++i) r[v[i]] += re[i];               /* assembly */
    }
    return ORC_OK;
}

/* Residual r = b - A x, eq. (4), with A applied element by element
 * (A = sum_e C_e^T A_e C_e, eq. (3)) and b already assembled; NULL b means 0.
 * Rows on Dirichlet nodes are zeroed when mask is given (r(nd)=0 in the
 * Section 2 listings). */
int orc_residual(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems, const double *K,
                 const double *M, double nu, const double *b, const double *x,
                 const uint8_t *mask, double *r)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    for (int64_t i = 0; i < n_nodes; ++i) r[i] = b ? b[i] : 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *v = elems + e * nb;
        for (int i = 0; i < nb; ++i) {
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += Aentry(K, M, nu, e, nb, i, j) * x[v[j]];
            r[v[i]] -= s;
        }
    }
    if (mask)
        for (int64_t i = 0; i < n_nodes; ++i)
            if (mask[i]) r[i] = 0.0;
    return ORC_OK;
}

/* Componentwise rounding scale of the residual: s = |b| + sum_e C_e^T |A_e| |x_e|.
 * Used by the tests to state error bounds; not part of the method. */
int orc_residual_scale(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems,
                       const double *K, const double *M, double nu, const double *b,
                       const double *x, double *s)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    for (int64_t i = 0; i < n_nodes; ++i) s[i] = b ? fabs(b[i]) : 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *v = elems + e * nb;
        for (int i = 0; i < nb; ++i) {
            double t = 0.0;
            for (int j = 0; j < nb; ++j) t += fabs(Aentry(K, M, nu, e, nb, i, j)) * fabs(x[v[j]]);
            s[v[i]] += t;
        }
    }
    return ORC_OK;
}

/* Diagonal of the assembled operator: d_i = sum over elements containing
 * node i of (A_e)_{ii}.  (Jacobi preconditioner; not in the paper.) */
int orc_jacobi_diag(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems,
                    const double *K, const double *M, double nu, double *d)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    for (int64_t i = 0; i < n_nodes; ++i) d[i] = 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t *v = elems + e * nb;
        for (int i = 0; i < nb; ++i) d[v[i]] += Aentry(K, M, nu, e, nb, i, i);
    }
    return ORC_OK;
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Masked operator application q = A p, q(nd) = 0. */
static void apply_masked(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems,
                         const double *K, const double *M, double nu, const uint8_t *mask,
                         const double *p, double *q)
{
    orc_residual(nb, n_nodes, n_elems, elems, K, M, nu, NULL, p, mask, q);
    for (int64_t i = 0; i < n_nodes; ++i) q[i] = -q[i];
}

/* Jacobi-preconditioned conjugate gradients (Hestenes-Stiefel form, M^-1 =
 * diag(A)^-1) on the system of eq. (1) with the Dirichlet rows masked as in
 * the Section 2 listings.  x holds x0 on entry (Dirichlet values on nd) and
 * the last iterate on exit.  Stops when ||r_k||_2 <= rtol ||r_0||_2; the
 * recursive residual is then replaced by the true one b - A x, and the
 * iteration continues from it if the true residual still misses rtol
 * (at most 3 replacements).
 * out[0] = iterations, out[1] = true relative residual, out[2] = ||r_0||_2,
 * out[3] = replacements.  alpha_hist / beta_hist (nullable, length max_iter)
 * receive the CG coefficients. */
int orc_pcg(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems, const double *K,
            const double *M, double nu, const double *b, const uint8_t *mask, int use_jacobi,
            double rtol, int max_iter, double *x, double *out, double *alpha_hist,
            double *beta_hist)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    int64_t n = n_nodes;
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    double *dinv = malloc(n * sizeof(double));
    int status = ORC_OK;
    orc_jacobi_diag(nb, n, n_elems, elems, K, M, nu, dinv);
    for (int64_t i = 0; i < n; ++i) {
        if (mask && mask[i]) dinv[i] = 0.0;
        else dinv[i] = use_jacobi ? 1.0 / dinv[i] : 1.0;
    }
    orc_residual(nb, n, n_elems, elems, K, M, nu, b, x, mask, r);
    const double r0 = sqrt(dot(n, r, r));
    int it = 0, repl = 0;
    double relres = 0.0;
    if (r0 == 0.0) goto done;
    for (int64_t i = 0; i < n; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
    double rz = dot(n, r, z);
    while (1) {
        if (it >= max_iter) { status = ORC_ENOCONV; break; }
        apply_masked(nb, n, n_elems, elems, K, M, nu, mask, p, q);
        double pq = dot(n, p, q);
        if (!(pq > 0.0)) { status = ORC_EBREAKDOWN; break; }
        double alpha = rz / pq;
        if (alpha_hist) alpha_hist[it] = alpha;
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        ++it;
        double rn = sqrt(dot(n, r, r));
        if (rn <= rtol * r0) {
            /* certify with the true residual */
            orc_residual(nb, n, n_elems, elems, K, M, nu, b, x, mask, q);
            double tn = sqrt(dot(n, q, q));
            if (tn <= rtol * r0 || repl >= 3) break;
            ++repl;
            memcpy(r, q, n * sizeof(double));
        }
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
        if (beta_hist) beta_hist[it - 1] = beta;
        rz = rz_new;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    orc_residual(nb, n, n_elems, elems, K, M, nu, b, x, mask, q);
    relres = sqrt(dot(n, q, q)) / r0;
done:
    if (out) { out[0] = it; out[1] = relres; out[2] = r0; out[3] = repl; }
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* The paper's own iterations (Section 2.1, 2.2).  Each step computes the    */
/* residual r = b - A x with r(nd) = 0 and updates x.                        */
/* ------------------------------------------------------------------------ */

/* Richardson, eq. (5): x^{k+1} = x^k + omega r^k with omega = 2/(lam1+lam2)
 * (the value giving the stated contraction factor). */
int orc_richardson(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems,
                   const double *K, const double *M, double nu, const double *b,
                   const uint8_t *mask, double lam1, double lam2, int iters, double *x)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    double *r = malloc(n_nodes * sizeof(double));
    const double omega = 2.0 / (lam1 + lam2);
    for (int k = 0; k < iters; ++k) {
        orc_residual(nb, n_nodes, n_elems, elems, K, M, nu, b, x, mask, r);
        for (int64_t i = 0; i < n_nodes; ++i) x[i] += omega * r[i];
    }
    free(r);
    return ORC_OK;
}

/* Two-level cyclic Chebyshev, eq. (6): x^{k+1} = x^k + r^k / alpha_{k mod N},
 * alpha_k = (lam1+lam2)/2 + (lam2-lam1)/2 cos(pi (k+1/2)/N), k = 0..N-1
 * (the roots of the scaled Chebyshev polynomial P_N, in the order of the
 * Section 2.2 listing). */
int orc_cheb2(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems, const double *K,
              const double *M, double nu, const double *b, const uint8_t *mask, double lam1,
              double lam2, int N, int iters, double *x)
{
    if (check_elems(nb, n_nodes, n_elems, elems) || N < 1) return ORC_EINVAL;
    const double pi = 3.14159265358979323846;
    double *r = malloc(n_nodes * sizeof(double));
    const double d = 0.5 * (lam2 + lam1), c = 0.5 * (lam2 - lam1);
    for (int k = 0; k < iters; ++k) {
        orc_residual(nb, n_nodes, n_elems, elems, K, M, nu, b, x, mask, r);
        const double alpha = d + c * cos(pi * (0.5 + (double)(k % N)) / (double)N);
        for (int64_t i = 0; i < n_nodes; ++i) x[i] += r[i] / alpha;
    }
    free(r);
    return ORC_OK;
}

/* Three-level Chebyshev, eq. (9) with the scaling factors of eq. (8):
 *   sigma = (lam1+lam2)/(lam2-lam1), C_0 = 1, C_1 = sigma,
 *   C_{k+1} = 2 sigma C_k - C_{k-1},
 *   x^1 = x^0 + 2/(lam1+lam2) r_0,
 *   x^{k+1} = x^k + C_{k-1}/C_{k+1} (x^k - x^{k-1}) + 4/(lam2-lam1) C_k/C_{k+1} r_k, k >= 1.
 * The ratios C_{k-1}/C_{k+1} and C_k/C_{k+1} are carried as the ratio
 * rho_k = C_{k-1}/C_k (rho_1 = 1/sigma, rho_{k+1} = 1/(2 sigma - rho_k)), which
 * is the same recurrence divided through by C_k and does not overflow. */
int orc_cheb3(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems, const double *K,
              const double *M, double nu, const double *b, const uint8_t *mask, double lam1,
              double lam2, int iters, double *x)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    double *r = malloc(n_nodes * sizeof(double)), *xprev = malloc(n_nodes * sizeof(double));
    const double sigma = (lam1 + lam2) / (lam2 - lam1);
    double rho = 1.0 / sigma; /* C_0 / C_1 */
    for (int k = 0; k < iters; ++k) {
        orc_residual(nb, n_nodes, n_elems, elems, K, M, nu, b, x, mask, r);
        if (k == 0) {
            const double w = 2.0 / (lam1 + lam2);
            for (int64_t i = 0; i < n_nodes; ++i) { xprev[i] = x[i]; x[i] += w * r[i]; }
        } else {
            /* C_k/C_{k+1} = 1/(2 sigma - rho_k);  C_{k-1}/C_{k+1} = rho_k * C_k/C_{k+1} */
            const double ck_ck1 = 1.0 / (2.0 * sigma - rho);
            const double ckm1_ck1 = rho * ck_ck1;
            const double w = 4.0 / (lam2 - lam1) * ck_ck1;
            for (int64_t i = 0; i < n_nodes; ++i) {
                const double xn = x[i] + ckm1_ck1 * (x[i] - xprev[i]) + w * r[i];
                xprev[i] = x[i];
                x[i] = xn;
            }
            rho = ck_ck1;
        }
    }
    free(r); free(xprev);
    return ORC_OK;
}

/* The three-level Chebyshev method as the Section 2.2 program runs it.
 *
 * The program advances a search direction with a coefficient beta and a step
 * alpha, and starts its beta recurrence from (c / (2 d))^2 with d = (lam1+lam2)/2,
 * c = (lam2-lam1)/2.  Eliminating the direction gives a three-term recurrence
 * for the iterates of exactly the form of eq. (9), with the scaling factors
 * C_k of eq. (8) -- the Chebyshev polynomials of the first kind T_k at
 * sigma = d / c -- replaced by those of the second kind, U_k(sigma)
 * (U_0 = 1, U_1 = 2 sigma, U_{k+1} = 2 sigma U_k - U_{k-1}): the program's
 * first beta is rho_0^2 with rho_0 = U_0 / U_1, and every later step keeps the
 * three-term relation.  Its error after k steps is therefore
 *   e_k = U_k((d - A) / c) / U_k(d / c) e_0,
 * where eq. (9) gives T_k((d - A) / c) / T_k(d / c) e_0.  The equations are
 * taken as the method (orc_cheb3); this is the program's variant.
 *
 * Here it is written as that three-term recurrence:
 *   x^1     = x^0 + (2/c) (U_0 / U_1) r_0  = x^0 + r_0 / d,
 *   x^{k+1} = x^k + (U_{k-1} / U_{k+1}) (x^k - x^{k-1}) + (2/c) (U_k / U_{k+1}) r_k,
 * with the ratio u_k = U_k / U_{k+1} (u_0 = 1 / (2 sigma),
 * u_k = 1 / (2 sigma - u_{k-1})) so that nothing overflows; U_{k-1} / U_{k+1}
 * = u_{k-1} u_k. */
int orc_cheb3_listing(int nb, int64_t n_nodes, int64_t n_elems, const int32_t *elems,
                      const double *K, const double *M, double nu, const double *b,
                      const uint8_t *mask, double lam1, double lam2, int iters, double *x)
{
    if (check_elems(nb, n_nodes, n_elems, elems)) return ORC_EINVAL;
    double *r = malloc(n_nodes * sizeof(double)), *xprev = malloc(n_nodes * sizeof(double));
    const double c = 0.5 * (lam2 - lam1);
    const double sigma = (lam1 + lam2) / (lam2 - lam1);
    double u_prev = 0.0;               /* u_{k-1} */
    double u = 1.0 / (2.0 * sigma);    /* u_k, starting at u_0 = U_0 / U_1 */
    for (int k = 0; k < iters; ++k) {
        orc_residual(nb, n_nodes, n_elems, elems, K, M, nu, b, x, mask, r);
        const double w_r = (2.0 / c) * u;      /* (2/c) U_k / U_{k+1} */
        const double w_x = u_prev * u;         /* U_{k-1} / U_{k+1}, 0 at k = 0 */
        for (int64_t i = 0; i < n_nodes; ++i) {
            const double xn = x[i] + (k > 0 ? w_x * (x[i] - xprev[i]) : 0.0) + w_r * r[i];
            xprev[i] = x[i];
            x[i] = xn;
        }
        u_prev = u;
        u = 1.0 / (2.0 * sigma - u);
    }
    free(r); free(xprev);
    return ORC_OK;
}
