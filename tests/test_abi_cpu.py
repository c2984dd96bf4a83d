"""CPU-side checks of the C ABI: the library loads, exports what include/fem.h
declares, and its host-side plan logic validates meshes and sizes chunks."""
import os
import re

import numpy as np
import pytest

from paper_1911_03973_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

fem = pytest.importorskip("paper_1911_03973_amd.fem", reason="libfem.so not built")


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    decl = declared_symbols()
    assert len(decl) >= 12
    lib = fem.library()
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(fem.EXPORTED) == decl


def test_oracle_and_library_share_nothing():
    """The oracle never imports the product package and vice versa."""
    pkg = os.path.join(ROOT, "paper_1911_03973_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "orc_" not in src, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            src = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1911_03973_amd" not in src and "fem_" not in src, f


def test_host_plan_stats_square():
    m = inputs.square_mesh(64)
    st = fem.plan_check_host(m, inputs.boundary_nodes(m), chunk_elems=2048)
    assert st["n_nodes"] == 65 * 65 and st["n_elems"] == 8192
    assert st["n_chunks"] == 4 and st["n_dirichlet"] == 256
    # Morton chunks of 1024 squares are 32x32 blocks: 33^2 local nodes each,
    # the shared nodes are the two interior grid lines (65 + 65 - 1)
    assert st["n_local"] == 4 * 33 * 33
    assert st["n_shared"] == 129
    # partials: 128 line nodes on two chunks + the centre on four
    assert st["n_partials"] == 128 * 2 + 4


def test_host_plan_counts_are_consistent():
    for mesh in (inputs.square_mesh(37, jitter=0.2, seed=1), inputs.cube_mesh(9, jitter=0.1, seed=2)):
        for E in (64, 512, 1024):
            st = fem.plan_check_host(mesh, inputs.boundary_nodes(mesh), chunk_elems=E)
            assert st["n_chunks"] == -(-mesh.n_elems // E)
            # every node is counted once per chunk that touches it
            touched = np.zeros(mesh.n_nodes, np.int64)
            for c in range(st["n_chunks"]):
                touched[np.unique(mesh.elems[c * E:(c + 1) * E])] += 1
            assert st["n_local"] == touched.sum()
            assert st["n_shared"] == (touched != 1).sum()
            assert st["n_partials"] == touched[touched > 1].sum()


def test_host_plan_rejects_bad_meshes():
    m = inputs.square_mesh(4)
    bad = inputs.Mesh(m.coords, m.elems.copy(), m.n)
    bad.elems[5, 2] = m.n_nodes
    with pytest.raises(fem.FemError, match="outside"):
        fem.plan_check_host(bad)
    rep = inputs.Mesh(m.coords, m.elems.copy(), m.n)
    rep.elems[3, 1] = rep.elems[3, 0]
    with pytest.raises(fem.FemError, match="repeats"):
        fem.plan_check_host(rep)
    flat = inputs.Mesh(m.coords.copy(), m.elems, m.n)
    flat.coords[6] = flat.coords[0]
    with pytest.raises(fem.FemError, match="volume"):
        fem.plan_check_host(flat)
    with pytest.raises(fem.FemError, match="Dirichlet"):
        fem.plan_check_host(m, np.array([m.n_nodes + 3]))
    with pytest.raises(fem.FemError, match="chunk_elems"):
        fem.plan_check_host(m, chunk_elems=100)
    with pytest.raises(fem.FemError, match="chunk_elems"):
        fem.plan_check_host(m, chunk_elems=1 << 16)
    nan = inputs.Mesh(m.coords.copy(), m.elems, m.n)
    nan.coords[7, 0] = np.nan
    with pytest.raises(fem.FemError, match="non-finite"):
        fem.plan_check_host(nan)


def test_host_plan_isolated_nodes_and_empty_mesh():
    m = inputs.square_mesh(3)
    coords = np.vstack([m.coords, [[2.0, 2.0]]])  # one node outside every element
    st = fem.plan_check_host(inputs.Mesh(coords, m.elems, m.n))
    assert st["n_shared"] >= 1
    empty = inputs.Mesh(m.coords, np.zeros((0, 3), np.int32), m.n)
    st = fem.plan_check_host(empty)
    assert st["n_chunks"] == 0 and st["n_shared"] == m.n_nodes


def test_solve_opts_defaults():
    o = fem.solve_opts()
    assert o.rtol == 1e-8 and o.precond == fem.PRECOND_JACOBI and o.check_every >= 1


def test_square_hierarchy_is_nested():
    """Every coarse node sits on the fine node (2^l I, 2^l J) and every level is
    the generator's own mesh of n / 2^l squares (same triangles)."""
    import numpy as np

    from paper_1911_03973_amd import inputs

    fine = inputs.square_mesh(32, jitter=0.2, seed=4)
    levels = inputs.square_hierarchy(fine, coarsest=4)
    assert [m.n for m in levels] == [32, 16, 8, 4]
    for l, m in enumerate(levels):
        ref = inputs.square_mesh(m.n)
        np.testing.assert_array_equal(m.elems, ref.elems)
        k = 1 << l
        for J in range(m.n + 1):
            for I in range(m.n + 1):
                assert np.array_equal(m.coords[J * (m.n + 1) + I], fine.coords[(k * J) * 33 + k * I])


def test_cube_hierarchy_is_nested():
    """Every coarse node sits on the fine node (2^l I, 2^l J, 2^l K) and every
    level is the generator's own Kuhn mesh of n / 2^l cubes."""
    import numpy as np

    from paper_1911_03973_amd import inputs

    fine = inputs.cube_mesh(20, jitter=0.1, seed=5)
    levels = inputs.cube_hierarchy(fine, coarsest=5)
    assert [m.n for m in levels] == [20, 10, 5]
    for l, m in enumerate(levels):
        np.testing.assert_array_equal(m.elems, inputs.cube_mesh(m.n).elems)
        k, mf, mc = 1 << l, 21, m.n + 1
        K, rem = np.divmod(np.arange(mc ** 3), mc * mc)
        J, I = np.divmod(rem, mc)
        np.testing.assert_array_equal(m.coords, fine.coords[((k * K) * mf + k * J) * mf + k * I])


def test_p2_mesh_lattice_and_midpoints():
    """P2 nodes are the (2n+1)^2 lattice; each element lists its vertices,
    then the midpoints of edges (0,1), (1,2), (2,0), at the middle of the
    (jittered, straight) edges."""
    import numpy as np

    from paper_1911_03973_amd import inputs

    m = inputs.square_mesh_p2(6, jitter=0.2, seed=3)
    assert m.n_nodes == 13 * 13 and m.n_elems == 72 and m.nb == 6
    c = m.coords
    e = m.elems
    for a, b, mid in ((0, 1, 3), (1, 2, 4), (2, 0, 5)):
        np.testing.assert_allclose(c[e[:, mid]], 0.5 * (c[e[:, a]] + c[e[:, b]]), rtol=0, atol=1e-15)
    assert len(np.unique(e)) == m.n_nodes


def test_p2_tet_mesh_lattice_and_midpoints():
    """P2 tetrahedron nodes are the (2n+1)^3 lattice; each element lists its
    vertices, then the midpoints of edges (0,1), (0,2), (0,3), (1,2), (1,3),
    (2,3), at the middle of the (jittered, straight) edges; the vertices are
    those of the linear Kuhn mesh."""
    import numpy as np

    from paper_1911_03973_amd import inputs

    m = inputs.cube_mesh_p2(3, jitter=0.2, seed=3)
    lin = inputs.cube_mesh(3, jitter=0.2, seed=3)
    assert m.n_nodes == 7 ** 3 and m.n_elems == 6 * 27 and m.nb == 10 and m.n == 6
    c, e = m.coords, m.elems
    edges = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
    for k, (a, b) in enumerate(edges):
        np.testing.assert_allclose(c[e[:, 4 + k]], 0.5 * (c[e[:, a]] + c[e[:, b]]), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(c[e[:, :4]], lin.coords[lin.elems])
    assert len(np.unique(e)) == m.n_nodes


def test_host_plan_for_quadratic_meshes():
    """The host dry run of quadratic meshes: 6 or 10 nodes per element, the
    same chunk bookkeeping as for linear elements, chunk limits of 1024 (P2
    triangles) and 512 (P2 tetrahedra), and the usual mesh checks."""
    for mesh, cap in ((inputs.square_mesh_p2(9, jitter=0.2, seed=1), 1024),
                      (inputs.cube_mesh_p2(3, jitter=0.1, seed=2), 512)):
        nb = mesh.elems.shape[1]
        for E in (64, 128):
            st = fem.plan_check_host(mesh, inputs.boundary_nodes(mesh), chunk_elems=E)
            assert st["n_b"] == nb and st["n_chunks"] == -(-mesh.n_elems // E)
            touched = np.zeros(mesh.n_nodes, np.int64)
            for c in range(st["n_chunks"]):
                touched[np.unique(mesh.elems[c * E:(c + 1) * E])] += 1
            assert st["n_local"] == touched.sum()
            assert st["n_shared"] == (touched != 1).sum()
        assert fem.plan_check_host(mesh)["chunk_elems"] == cap
        with pytest.raises(fem.FemError, match="chunk_elems"):
            fem.plan_check_host(mesh, chunk_elems=2 * cap)
        rep = inputs.Mesh(mesh.coords, mesh.elems.copy(), mesh.n)
        rep.elems[1, nb - 1] = rep.elems[1, 0]
        with pytest.raises(fem.FemError, match="repeats"):
            fem.plan_check_host(rep)
