"""Quadratic (P2) tetrahedra on the GPU against the P2 oracle (oracle/p2.py).

As for P2 triangles: the GPU integrates barycentric monomials in closed form,
the oracle uses a collapsed Gauss rule on the tetrahedron, and FP64 entries
must agree to 1e-12.  The residual, diagonal and right-hand side go through
the chunked pass with 10 slots per element (chunks of at most 512 elements)
and must match the oracle's nb-generic routines to 1e-12 of the residual
scale; the solver is judged by its first iterates, its iteration count and
the exact reproduction of a quadratic solution.
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.p2 as op2
from paper_1911_03973_amd import inputs

from problems import cuda, from_soa, max_rel, pair_value, to_soa

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_1911_03973_amd.fem")


def _shuffled(mesh, seed):
    order = np.random.default_rng(seed).permutation(mesh.n_elems)
    return inputs.Mesh(coords=mesh.coords, elems=np.ascontiguousarray(mesh.elems[order]), n=mesh.n)


class TetProblem:
    def __init__(self, mesh, nu, dirichlet="all", seed=0):
        self.mesh = mesh
        self.nu = float(nu)
        self.nd = inputs.boundary_nodes(mesh, dirichlet)
        self.mask = oracle.mask_from_nodes(mesh.n_nodes, self.nd)
        self.K, self.M, self.vol = op2.local_matrices_p2_tet(mesh.coords, mesh.elems)
        self.f = inputs.random_sine(mesh.coords, seed)
        self.b = oracle.rhs(mesh.n_nodes, mesh.elems, self.M, self.f)

    @property
    def n(self):
        return self.mesh.n_nodes


MESHES = [
    ("p2t_1_single_cube", inputs.cube_mesh_p2(1, order="rowmajor"), 0),
    ("p2t_3_jitter_E64", inputs.cube_mesh_p2(3, jitter=0.2, seed=3), 64),
    ("p2t_5_jitter_E256", inputs.cube_mesh_p2(5, jitter=0.2, seed=4), 256),
    ("p2t_10_default", inputs.cube_mesh_p2(10, jitter=0.15, seed=5), 0),   # 12 chunks, ragged tail of 368
    ("p2t_7_rowmajor_E512", inputs.cube_mesh_p2(7, order="rowmajor", jitter=0.1, seed=6), 512),
    ("p2t_4_shuffled_E128", _shuffled(inputs.cube_mesh_p2(4, jitter=0.2, seed=7), 8), 128),
]


@pytest.fixture(params=MESHES, ids=[m[0] for m in MESHES])
def case(request):
    name, mesh, E = request.param
    print(f"[case] {name} n_nodes={mesh.n_nodes} n_elems={mesh.n_elems} E={E}", flush=True)
    prob = TetProblem(mesh, nu=0.75, seed=11)
    plan = fem.Plan.from_mesh(mesh, prob.nd, chunk_elems=E)
    assert plan.nb == 10 and plan.stats()["n_b"] == 10
    return prob, plan


def test_p2_tet_local_matrices(case):
    prob, plan = case
    K = plan.empty_matrix(fem.F64)
    M = plan.empty_matrix(fem.F64)
    vol = torch.empty(plan.n_elems, dtype=torch.float64, device="cuda")
    fem.build_local_matrices(plan, fem.F64, K, M, vol)
    Kp = plan.empty_matrix(fem.F32X2)
    Mp = plan.empty_matrix(fem.F32X2)
    fem.build_local_matrices(plan, fem.F32X2, Kp, Mp, None)
    torch.cuda.synchronize()
    assert max_rel(from_soa(K.cpu().numpy(), 10), prob.K) <= 1e-12
    assert max_rel(from_soa(M.cpu().numpy(), 10), prob.M) <= 1e-12
    assert max_rel(vol.cpu().numpy(), prob.vol) <= 1e-12
    assert max_rel(from_soa(pair_value(Kp), 10), prob.K) <= 1e-12
    assert max_rel(from_soa(pair_value(Mp), 10), prob.M) <= 1e-12


def test_p2_tet_residual_diagonal_rhs(case):
    prob, plan = case
    K = cuda(to_soa(prob.K))
    M = cuda(to_soa(prob.M))
    x = np.random.default_rng(1).standard_normal(prob.n)
    r = plan.empty_vector()
    for mask in (True, False):
        fem.element_residual(plan, fem.F64, K, M, prob.nu, cuda(prob.b), cuda(x), r, mask=mask)
        torch.cuda.synchronize()
        ro = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x, prob.mask if mask else None)
        s = oracle.residual_scale(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x)
        assert max_rel(r.cpu().numpy(), ro, scale=s.max()) <= 1e-12, mask
    d = plan.empty_vector()
    fem.jacobi_diag(plan, fem.F64, K, M, prob.nu, d)
    b = plan.empty_vector()
    fem.assemble_rhs(plan, fem.F64, M, cuda(prob.f), b)
    torch.cuda.synchronize()
    do = oracle.jacobi_diag(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu)
    assert max_rel(d.cpu().numpy(), do) <= 1e-12
    assert max_rel(b.cpu().numpy(), prob.b) <= 1e-12


def test_p2_tet_residual_f32_error_bound(case):
    """The FP32 residual within c * gamma_k * (|b| + sum |A_e||x_e|), k = n_b +
    deg + 2, c = 2 (inputs rounded to FP32 once), as for P1."""
    prob, plan = case
    A = prob.K + prob.nu * prob.M
    A32 = cuda(to_soa(A).astype(np.float32))
    x = np.random.default_rng(3).standard_normal(prob.n)
    r = plan.empty_vector(torch.float32)
    fem.element_residual_f32(plan, A32, cuda(prob.b.astype(np.float32)), cuda(x.astype(np.float32)), r, mask=True)
    torch.cuda.synchronize()
    ro = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x, prob.mask)
    s = oracle.residual_scale(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x)
    deg = np.bincount(prob.mesh.elems.ravel(), minlength=prob.n).max()
    k = 10 + deg + 2
    u = 2.0 ** -24
    gamma = k * u / (1 - k * u)
    assert np.all(np.abs(r.double().cpu().numpy() - ro) <= 2 * gamma * s + 1e-30)


def test_p2_tet_first_iterates_match_oracle():
    mesh = inputs.cube_mesh_p2(4, jitter=0.2, seed=9)
    prob = TetProblem(mesh, nu=2.5, seed=3)
    plan = fem.Plan.from_mesh(mesh, prob.nd, chunk_elems=128)
    K, M = cuda(to_soa(prob.K)), cuda(to_soa(prob.M))
    u = 1.0 + mesh.coords[:, 0]
    x0 = np.zeros(prob.n)
    x0[prob.nd] = u[prob.nd]
    for k in (1, 2, 5, 10):
        x = cuda(x0)
        info = fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F64, nu=prob.nu, max_iter=k, check_every=4), K, M,
                             cuda(prob.b), x)
        xo, io = oracle.pcg(prob.n, mesh.elems, prob.K, prob.M, prob.nu, prob.b, prob.mask, x0.copy(), max_iter=k,
                            raise_on_noconv=False)
        assert info["iters"] == io["iters"] == k
        assert max_rel(x.cpu().numpy(), xo) <= 1e-10, k


@pytest.mark.parametrize("dtype", ["f64", "f32x2"])
def test_p2_tet_solve_meets_target_and_reproduces_a_quadratic(dtype):
    """GPU-built matrices, GPU right-hand side of f = -Lap u + nu u for a
    quadratic u, Dirichlet data u on the boundary: the P2 solution is u."""
    dt = fem.F64 if dtype == "f64" else fem.F32X2
    mesh = inputs.cube_mesh_p2(12, jitter=0.2, seed=12)
    nu = 3.0
    nd = inputs.boundary_nodes(mesh, "all")
    plan = fem.Plan.from_mesh(mesh, nd)
    K, M = plan.empty_matrix(dt), plan.empty_matrix(dt)
    fem.build_local_matrices(plan, dt, K, M, None)
    xq, yq, zq = mesh.coords[:, 0], mesh.coords[:, 1], mesh.coords[:, 2]
    u = 1.0 + xq - 2.0 * yq + 0.5 * zq + 3.0 * xq * xq - xq * yq + 2.0 * yq * yq + yq * zq - zq * zq
    f = -(2 * 3.0 + 2 * 2.0 - 2 * 1.0) + nu * u
    b = plan.empty_vector()
    fem.assemble_rhs(plan, dt, M, cuda(f), b)
    x0 = np.zeros(mesh.n_nodes)
    x0[nd] = u[nd]
    x = cuda(x0)
    info = fem.pcg_solve(plan, fem.solve_opts(dtype=dt, nu=nu, rtol=1e-12), K, M, b, x)
    assert info["status"] == fem.FEM_OK
    assert np.abs(x.cpu().numpy() - u).max() <= 1e-9 * np.abs(u).max()
    Ko, Mo, _ = op2.local_matrices_p2_tet(mesh.coords, mesh.elems)
    bo = oracle.rhs(mesh.n_nodes, mesh.elems, Mo, f)
    mask = oracle.mask_from_nodes(mesh.n_nodes, nd)
    _, io = oracle.pcg(mesh.n_nodes, mesh.elems, Ko, Mo, nu, bo, mask, x0.copy(), rtol=1e-12)
    if dt == fem.F64:
        assert abs(info["iters"] - io["iters"]) <= max(2, 0.02 * io["iters"]), (info["iters"], io["iters"])


def test_p2_tet_rejects_unsupported_paths():
    mesh = inputs.cube_mesh_p2(3)
    nd = inputs.boundary_nodes(mesh)
    plan = fem.Plan.from_mesh(mesh, nd)
    assert plan.stats()["chunk_elems"] == 512
    b = plan.empty_vector()
    b.zero_()
    x = plan.empty_vector()
    K, M = plan.empty_matrix(fem.F32X2), plan.empty_matrix(fem.F32X2)
    fem.build_local_matrices(plan, fem.F32X2, K, M, None)
    with pytest.raises(fem.FemError):
        fem.pcg_solve(plan, fem.solve_opts(dtype=fem.MFREE), None, None, b, x)
    with pytest.raises(fem.FemError):
        fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F32X2, vectors=1), K, M, b, x)
    with pytest.raises(fem.FemError):
        fem.element_residual(plan, fem.MFREE, None, None, 1.0, None, b, x)
    with pytest.raises(fem.FemError):
        fem.Plan.from_mesh(mesh, nd, chunk_elems=1024)


def test_p2_tet_isolated_node_empty_mesh_and_bad_dim():
    m = inputs.cube_mesh_p2(2, jitter=0.1, seed=2)
    mesh = inputs.Mesh(np.vstack([m.coords, [[3.0, 3.0, 3.0]]]), m.elems, m.n)
    K, M, _ = op2.local_matrices_p2_tet(mesh.coords, mesh.elems)
    plan = fem.Plan.from_mesh(mesh, None, chunk_elems=64)
    x = np.random.default_rng(0).standard_normal(mesh.n_nodes)
    b = np.random.default_rng(1).standard_normal(mesh.n_nodes)
    r = plan.empty_vector()
    fem.element_residual(plan, fem.F64, cuda(to_soa(K)), cuda(to_soa(M)), 1.0, cuda(b), cuda(x), r, mask=False)
    torch.cuda.synchronize()
    ro = oracle.residual(mesh.n_nodes, mesh.elems, K, M, 1.0, b, x)
    assert max_rel(r.cpu().numpy(), ro) <= 1e-12
    assert r[-1].item() == b[-1]  # the isolated node keeps b
    empty = fem.Plan(3, cuda(m.coords.T), torch.zeros((10, 0), dtype=torch.int32, device="cuda"))
    r = empty.empty_vector()
    fem.element_residual(empty, fem.F64, None, None, 0.0, cuda(b[: m.n_nodes]), cuda(x[: m.n_nodes]), r, mask=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.cpu().numpy(), b[: m.n_nodes])
    # a 10-node connectivity on 2D coordinates is neither P1 nor P2
    with pytest.raises(ValueError):
        fem.Plan(2, cuda(m.coords[:, :2].T), cuda(m.elems.T.astype(np.int32)))
    h = fem.ctypes.c_void_p()
    rc = fem.library().fem_plan_create_p2(4, m.n_nodes, m.n_elems, None, None, None, 0, 0, None, fem.ctypes.byref(h))
    assert rc == fem.FEM_EINVAL and not h.value
