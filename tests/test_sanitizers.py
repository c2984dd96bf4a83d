"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The planner (plan.cpp, plan_check.cpp) is built on its own with g++ and
-fsanitize=address,undefined and driven through fem_plan_check_host /
fem_plan_check_host_p2 on 2D, 3D and quadratic meshes (shuffled and ragged
element lists, every chunk size, isolated nodes, empty meshes) and on the
inputs it must reject.  The C oracle is built the same way and the oracle's
pin tests run against it.  Each run is a child Python process with the ASan
runtime preloaded; a sanitizer report or a non-zero exit fails the test.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


ASAN = _runtime()
pytestmark = pytest.mark.skipif(ASAN is None, reason="no libasan for the host compiler")


def _env(**extra):
    env = dict(os.environ)
    env.update({"LD_PRELOAD": ASAN, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "PYTHONPATH": ROOT})
    env.update(extra)
    return env


def _check(p):
    out = p.stdout + p.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]


PLANNER_SCRIPT = textwrap.dedent("""
    import ctypes, sys
    import numpy as np
    from paper_1911_03973_amd import inputs

    class Stats(ctypes.Structure):
        _fields_ = [("dim", ctypes.c_int), ("n_b", ctypes.c_int), ("n_nodes", ctypes.c_int64),
                    ("n_elems", ctypes.c_int64), ("n_dirichlet", ctypes.c_int64), ("chunk_elems", ctypes.c_int),
                    ("n_chunks", ctypes.c_int64), ("n_local", ctypes.c_int64), ("n_shared", ctypes.c_int64),
                    ("n_partials", ctypes.c_int64), ("index_bytes", ctypes.c_int64)]

    L = ctypes.CDLL(sys.argv[1])
    ctypes.CDLL(None)["__asan_init"]  # the sanitizer runtime is in this process

    def check(coords, elems, dim, nd, chunk):
        c = np.ascontiguousarray(np.asarray(coords, dtype=np.float64).T)
        e = np.ascontiguousarray(np.asarray(elems, dtype=np.int32).T)
        d = np.ascontiguousarray(nd, dtype=np.int32)
        st = Stats()
        fn = L.fem_plan_check_host_p2 if e.shape[0] > dim + 1 else L.fem_plan_check_host
        return fn(dim, ctypes.c_int64(c.shape[1]), ctypes.c_int64(e.shape[1]), c.ctypes.data_as(ctypes.c_void_p),
                  e.ctypes.data_as(ctypes.c_void_p) if e.size else None,
                  d.ctypes.data_as(ctypes.c_void_p) if d.size else None, ctypes.c_int64(d.size), chunk,
                  ctypes.byref(st)), st

    rng = np.random.default_rng(0)
    meshes = [(inputs.square_mesh(20, jitter=0.2, seed=1), [64, 128, 256, 512, 1024, 2048]),
              (inputs.square_mesh(17, order="rowmajor"), [64, 256, 1024]),
              (inputs.cube_mesh(6, jitter=0.1, seed=2), [64, 128, 512, 1536]),
              (inputs.square_mesh_p2(8, jitter=0.1, seed=3), [64, 256, 1024]),
              (inputs.cube_mesh_p2(3), [64, 128, 512])]
    n_ok = 0
    for m, chunks in meshes:
        nd = inputs.boundary_nodes(m, "all")
        for chunk in chunks:
            for shuffle in (False, True):
                el = m.elems[rng.permutation(len(m.elems))] if shuffle else m.elems
                rc, st = check(m.coords, el, m.dim, nd, chunk)
                assert rc == 0 and st.n_elems == len(el), (rc, chunk)
                n_ok += 1
        # ragged tail, duplicate Dirichlet ids, an isolated node, an empty element list
        rc, _ = check(m.coords, m.elems[: len(m.elems) - 7], m.dim, np.concatenate([nd, nd[:5]]), 64)
        assert rc == 0
        coords = np.vstack([m.coords, m.coords[-1:] + 5.0])
        rc, st = check(coords, m.elems, m.dim, nd, 0)
        assert rc == 0
        rc, _ = check(m.coords, m.elems[:0], m.dim, nd, 0)
        assert rc == 0
        # rejected: node index out of range, negative index, non-finite coordinate,
        # Dirichlet id out of range, unsupported chunk size
        bad = m.elems.copy(); bad[3, 1] = len(m.coords)
        assert check(m.coords, bad, m.dim, nd, 0)[0] != 0
        bad = m.elems.copy(); bad[0, 0] = -1
        assert check(m.coords, bad, m.dim, nd, 0)[0] != 0
        c2 = m.coords.copy(); c2[4, 0] = np.nan
        assert check(c2, m.elems, m.dim, nd, 0)[0] != 0
        assert check(m.coords, m.elems, m.dim, np.array([len(m.coords)]), 0)[0] != 0
        assert check(m.coords, m.elems, m.dim, nd, 100)[0] != 0
    # a degenerate (zero-volume) triangle
    m = inputs.square_mesh(4)
    bad = m.elems.copy(); bad[2] = [0, 1, 2]
    assert check(m.coords, bad, 2, inputs.boundary_nodes(m, "all"), 0)[0] != 0
    print("planner cases ok", n_ok)
""")


def test_host_planner_under_asan_and_ubsan(tmp_path):
    from paper_1911_03973_amd import build as hipbuild

    lib = hipbuild.build_host_sanitized()
    script = tmp_path / "planner.py"
    script.write_text(PLANNER_SCRIPT)
    p = subprocess.run([sys.executable, str(script), lib], capture_output=True, text=True, env=_env(), timeout=300,
                       cwd=ROOT)
    _check(p)
    assert "planner cases ok" in p.stdout


def test_oracle_pins_under_asan_and_ubsan():
    from oracle import build as obuild

    lib = obuild.build_oracle(sanitized=True)
    probe = ("import ctypes, oracle; L = oracle.lib(); assert L._name.endswith('liborc_san.so'), L._name; "
             "ctypes.CDLL(None)['__asan_init']; print('sanitized oracle loaded')")
    p = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, env=_env(ORACLE_LIB=lib),
                       timeout=120, cwd=ROOT)
    _check(p)
    assert "sanitized oracle loaded" in p.stdout
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_oracle_pins.py", "tests/test_oracle_fcg.py", "tests/test_oracle_mg.py",
                        "tests/test_oracle_p2.py"],
                       capture_output=True, text=True, env=_env(ORACLE_LIB=lib), timeout=600, cwd=ROOT)
    _check(p)
    assert " passed" in p.stdout
