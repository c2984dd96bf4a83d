"""fem_element_residual_noalloc (the allocation-free residual, partials in the
library's static device array) against fem_element_residual on the same
inputs: bit for bit, on two calls in a row -- the second on a smaller mesh --
for FP64, FP32 hi/lo and matrix-free operators, and the rejection of a plan
with more shared-node partials than the array holds."""
import numpy as np
import pytest
import torch

from paper_1911_03973_amd import inputs

from problems import cuda

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_1911_03973_amd.fem")


def _case(mesh, dirichlet, dtype, nu, seed):
    nd = inputs.boundary_nodes(mesh, dirichlet)
    # matrix-free tetrahedra: 512-element chunks keep the coordinate table within the LDS limit
    plan = fem.Plan.from_mesh(mesh, nd, chunk_elems=512 if mesh.dim == 3 else 0)
    K = M = None
    if dtype != fem.MFREE:
        K = plan.empty_matrix(dtype)
        M = plan.empty_matrix(dtype)
        fem.build_local_matrices(plan, dtype, K, M, None)
    rng = np.random.default_rng(seed)
    x = cuda(rng.standard_normal(mesh.n_nodes))
    b = cuda(rng.standard_normal(mesh.n_nodes))
    return plan, K, M, x, b


@pytest.mark.parametrize("dtype", [fem.F64, fem.F32X2, fem.MFREE])
def test_noalloc_residual_equals_residual_twice_second_smaller(dtype):
    cases = [(inputs.square_mesh(256, jitter=0.2, seed=1), "x2=0", 1.5, 1),
             (inputs.square_mesh(48, jitter=0.2, seed=2), "all", 7.0, 2)]
    if dtype != fem.F32X2:
        cases.insert(1, (inputs.cube_mesh(24, jitter=0.1, seed=3), "all", 3.0, 3))
    for mesh, d, nu, seed in cases:
        plan, K, M, x, b = _case(mesh, d, dtype, nu, seed)
        print(f"noalloc case dtype {dtype} nodes {mesh.n_nodes} partials {plan.stats()['n_partials']}", flush=True)
        r_ref = torch.empty_like(x)
        r_na = torch.full_like(x, float("nan"))
        fem.element_residual(plan, dtype, K, M, nu, b, x, r_ref, mask=True)
        fem.element_residual_noalloc(plan, dtype, K, M, nu, b, x, r_na, mask=True)
        torch.cuda.synchronize()
        assert torch.equal(r_na, r_ref)
        # b absent, no mask
        fem.element_residual(plan, dtype, K, M, nu, None, x, r_ref, mask=False)
        fem.element_residual_noalloc(plan, dtype, K, M, nu, None, x, r_na, mask=False)
        torch.cuda.synchronize()
        assert torch.equal(r_na, r_ref)


def test_noalloc_rejects_plan_beyond_scratch():
    mesh = inputs.cube_mesh(112)
    nd = inputs.boundary_nodes(mesh, "all")
    st = fem.plan_check_host(mesh, nd, chunk_elems=64)
    assert st["n_partials"] > (1 << 22)
    plan = fem.Plan.from_mesh(mesh, nd, chunk_elems=64)
    x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
    r = torch.empty_like(x)
    with pytest.raises(fem.FemError, match="allocation-free"):
        fem.element_residual_noalloc(plan, fem.MFREE, None, None, 1.0, None, x, r)
