"""FP64 reference of the geometric multigrid V-cycle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU library.

Why multigrid: the spectral bounds of the paper's iterations (Section 2) and
the growth of the iteration count with the mesh size in its experiment
(Section 3) come from the h^-2 conditioning of the P1 operator; the paper
names better preconditioning as the remedy for fine meshes.  This module holds
the textbook two-grid / V-cycle construction on the nested diagonal-cut
square meshes and Kuhn cube meshes of the workloads, written from its
definitions:

  prolongation   P maps a coarse P1 function to the same function on the fine
                 mesh: each fine node's row holds the coarse hat functions
                 evaluated at that node.  The evaluation is geometric, in the
                 lattice coordinates of the coarse mesh (node (I, J) at the
                 point (I, J); square [I, I+1] x [J, J+1] cut along its
                 (0,0)-(1,1) diagonal), by barycentric coordinates of the
                 coarse triangle that holds the fine point (in 3D: of the
                 coarse Kuhn tetrahedron, `prolongation3`);
  restriction    P^T;
  smoother       damped Jacobi z <- z + omega D^-1 (r - A z), starting from
                 z = 0, `smooth` steps before and after the coarse correction;
                 or the paper's three-level Chebyshev iteration (Section 2,
                 eq. (9) with the scaling factors of eq. (8)) applied to the
                 Jacobi-scaled level system D^-1 A z = D^-1 r on the interval
                 [lower * g, g], where g is the Gershgorin bound of D^-1 A
                 built from the element matrices (`Level.gersh`);
  coarsest       exact solve of the free-node system (dense LU of numpy).

Dirichlet nodes carry zero corrections on every level: residuals there are
ignored and corrections stay zero, so every level works with the free-node
block of its operator.  Operator applications go through the oracle's element
residual (Algorithm 1, eq. (4)) with the level's own K_e, M_e.

Pins (tests/test_oracle_mg.py): g is 2 on the uniform square mesh and bounds
the largest eigenvalue of the free-node pencil (A, D) from above; m Chebyshev
smoothing steps multiply the error along each eigenvector of that pencil by
the scaled Chebyshev polynomial T_m((theta - lambda) / delta) / T_m(theta /
delta) (numpy's Chebyshev series, not the recurrence); P reproduces linear functions exactly; the
Galerkin identity P^T A_h P = A_2h of nested P1 spaces on dense matrices
assembled here by the definition; the V-cycle operator is symmetric; a
one-level cycle solves the coarse system; the V-cycle contracts the error by
a mesh-independent factor well below one.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse

from . import jacobi_diag, local_matrices, mask_from_nodes, residual


def prolongation3(n_coarse: int):
    """P ((2n+1)^3 x (n+1)^3, scipy CSR) for a Kuhn cube mesh of n^3 cubes,
    node (i, j, k) of a mesh with m nodes per side numbered (k m + j) m + i.
    In lattice units a point with local cube coordinates sorted as
    x_(1) >= x_(2) >= x_(3) lies in the Kuhn tetrahedron that walks from the
    cube's corner along the axes in that order; its barycentric coordinates
    are 1 - x_(1), x_(1) - x_(2), x_(2) - x_(3) and x_(3)."""
    nc = n_coarse
    mc, mf = nc + 1, 2 * nc + 1
    rows, cols, vals = [], [], []
    step = (1, mc, mc * mc)
    for k in range(mf):
        for j in range(mf):
            for i in range(mf):
                x = (i / 2.0, j / 2.0, k / 2.0)
                c0 = [min(int(np.floor(v)), nc - 1) for v in x]
                loc = [x[a] - c0[a] for a in range(3)]
                order = sorted(range(3), key=lambda a: -loc[a])
                srt = [loc[a] for a in order]
                node = (c0[2] * mc + c0[1]) * mc + c0[0]
                lam = [(node, 1.0 - srt[0])]
                for q in range(3):
                    node += step[order[q]]
                    lam.append((node, srt[q] - (srt[q + 1] if q < 2 else 0.0)))
                row = (k * mf + j) * mf + i
                for nd, w in lam:
                    if w != 0.0:
                        rows.append(row)
                        cols.append(nd)
                        vals.append(w)
    return scipy.sparse.coo_matrix((vals, (rows, cols)), shape=(mf ** 3, mc ** 3)).tocsr()


def prolongation(n_coarse: int):
    """P ((2n+1)^2 x (n+1)^2, scipy CSR) for a coarse mesh of n x n squares,
    node (i, j) of a mesh with m nodes per side numbered j m + i."""
    nc = n_coarse
    mc, mf = nc + 1, 2 * nc + 1
    rows, cols, vals = [], [], []
    for j in range(mf):
        for i in range(mf):
            x, y = i / 2.0, j / 2.0  # the fine node in coarse lattice units
            I = min(int(np.floor(x)), nc - 1)
            J = min(int(np.floor(y)), nc - 1)
            s, t = x - I, y - J
            a = J * mc + I
            b = a + 1
            c = a + mc + 1
            d = a + mc
            row = j * mf + i
            if s >= t:  # triangle [a, b, c]
                lam = ((a, 1.0 - s), (b, s - t), (c, t))
            else:  # triangle [a, c, d]
                lam = ((a, 1.0 - t), (c, s), (d, t - s))
            for node, w in lam:
                if w != 0.0:
                    rows.append(row)
                    cols.append(node)
                    vals.append(w)
    return scipy.sparse.coo_matrix((vals, (rows, cols)), shape=(mf * mf, mc * mc)).tocsr()


def assemble_dense(n_nodes, elems, K, M, nu) -> np.ndarray:
    """A = sum_e C_e^T (K_e + nu M_e) C_e as a dense matrix (eq. (3))."""
    A = np.zeros((n_nodes, n_nodes))
    el = np.asarray(elems, dtype=np.int64)
    Ae = np.asarray(K, dtype=np.float64) + nu * np.asarray(M, dtype=np.float64)
    for e in range(el.shape[0]):
        idx = el[e]
        A[np.ix_(idx, idx)] += Ae[e]
    return A


class Level:
    """One mesh of the hierarchy: its element arrays, Dirichlet mask, Jacobi
    diagonal and (for the coarsest) the dense free-node block."""

    def __init__(self, mesh, dirichlet, nu):
        self.n = int(mesh.n)
        self.dim = int(mesh.dim)
        self.n_nodes = int(mesh.n_nodes)
        self.elems = np.ascontiguousarray(mesh.elems, dtype=np.int32)
        self.K, self.M, _ = local_matrices(mesh.coords, mesh.elems)
        self.nu = float(nu)
        self.mask = mask_from_nodes(self.n_nodes, dirichlet)
        d = jacobi_diag(self.n_nodes, self.elems, self.K, self.M, self.nu)
        self.free = self.mask == 0
        self.dinv = np.where(self.free, 1.0 / np.where(self.free, d, 1.0), 0.0)

    @functools.cached_property
    def gersh(self):
        """g = max over free nodes i of D_ii^-1 sum_e sum_j |(A_e)_ij| (the
        element matrices' absolute row sums gathered to the nodes, every
        column counted).  Since sum_e |(A_e)_ij| >= |a_ij|, Gershgorin's
        theorem for D^-1 A bounds its eigenvalues by g."""
        Ae = np.asarray(self.K, dtype=np.float64) + self.nu * np.asarray(self.M, dtype=np.float64)
        absrow = np.zeros(self.n_nodes)
        np.add.at(absrow, self.elems.astype(np.int64).ravel(), np.abs(Ae).sum(axis=2).ravel())
        return float((self.dinv * absrow)[self.free].max()) if self.free.any() else 0.0

    def residual(self, r, z):
        """r - A z on free nodes, 0 on Dirichlet nodes."""
        return residual(self.n_nodes, self.elems, self.K, self.M, self.nu, r, z, self.mask)

    def dense_free(self):
        A = assemble_dense(self.n_nodes, self.elems, self.K, self.M, self.nu)
        f = np.flatnonzero(self.free)
        return A[np.ix_(f, f)], f


def hierarchy(meshes, dirichlets, nu):
    """Levels (finest first) and the prolongations P_l from level l+1 to l."""
    levels = [Level(m, d, nu) for m, d in zip(meshes, dirichlets)]
    for a, b in zip(levels[:-1], levels[1:]):
        if a.n != 2 * b.n:
            raise ValueError("each level must halve the squares per side")
    Ps = [(prolongation3(lv.n) if lv.dim == 3 else prolongation(lv.n)) for lv in levels[1:]]
    return levels, Ps


def chebyshev_smooth(L, r, z, steps, lower, lam_hi=None):
    """`steps` iterations of the paper's three-level Chebyshev method (eq. (9),
    scaling factors of eq. (8)) for D^-1 A z = D^-1 r on [lam1, lam2] =
    [lower g, g], from z (None: z = 0, whose first step needs no product):
      z^1 = z^0 + 2 / (lam1 + lam2) D^-1 r_0,
      z^{k+1} = z^k + C_{k-1} / C_{k+1} (z^k - z^{k-1}) + 4 / (lam2 - lam1) C_k / C_{k+1} D^-1 r_k,
    r_k = r - A z^k, C_0 = 1, C_1 = sigma = (lam1 + lam2) / (lam2 - lam1),
    C_{k+1} = 2 sigma C_k - C_{k-1}; the ratio rho_k = C_{k-1} / C_k follows
    rho_1 = 1 / sigma, rho_{k+1} = 1 / (2 sigma - rho_k)."""
    lam2 = L.gersh if lam_hi is None else lam_hi
    lam1 = lower * lam2
    sigma = (lam1 + lam2) / (lam2 - lam1)
    res = r if z is None else L.residual(r, z)
    z_old = np.zeros(L.n_nodes) if z is None else z
    z = z_old + (2.0 / (lam1 + lam2)) * L.dinv * res
    rho = 1.0 / sigma
    for _ in range(steps - 1):
        ck = 1.0 / (2.0 * sigma - rho)  # C_k / C_{k+1}
        z_new = z + (rho * ck) * (z - z_old) + (4.0 / (lam2 - lam1) * ck) * L.dinv * L.residual(r, z)
        z_old, z = z, z_new
        rho = ck
    return z


def vcycle(levels, Ps, r, smooth, omega, l=0, smoother="jacobi", lower=0.3):
    """z = B r: one V-cycle from level l (the coarsest level solves exactly).
    smoother "jacobi": `smooth` damped-Jacobi steps (factor omega) before and
    after the coarse correction; "chebyshev": `smooth` Chebyshev steps on
    [lower g, g] instead (omega unused)."""
    L = levels[l]
    r = np.where(L.free, np.asarray(r, dtype=np.float64), 0.0)
    if l == len(levels) - 1:
        A, f = L.dense_free()
        z = np.zeros(L.n_nodes)
        if f.size:
            z[f] = np.linalg.solve(A, r[f])
        return z
    if smoother == "chebyshev":
        z = chebyshev_smooth(L, r, None, smooth, lower)
    elif smoother == "jacobi":
        z = omega * L.dinv * r
        for _ in range(smooth - 1):
            z = z + omega * L.dinv * L.residual(r, z)
    else:
        raise ValueError("smoother: 'jacobi' or 'chebyshev'")
    rc = Ps[l].T @ L.residual(r, z)
    zc = vcycle(levels, Ps, rc, smooth, omega, l + 1, smoother, lower)
    z = z + np.where(L.free, Ps[l] @ zc, 0.0)
    if smoother == "chebyshev":
        z = chebyshev_smooth(L, r, z, smooth, lower)
    else:
        for _ in range(smooth):
            z = z + omega * L.dinv * L.residual(r, z)
    return z
