"""The oracle's C code under gcc's AddressSanitizer and UndefinedBehaviorSanitizer:
built with both into a temporary library and driven, in a child process with
the ASan runtime preloaded, through every entry point on small meshes.  Any
sanitizer report (or a wrong result on the way) fails the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_DRIVER = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import meshgen
    import oracle
    oracle._LIB_PATH = {lib!r}
    oracle.set_threads(2)
    ref = {{2: np.array([[0., 0.], [1., 0.], [0., 1.]]),
            3: np.array([[0., 0., 0.], [1., 0., 0.], [0., 1., 0.], [0., 0., 1.]])}}
    for dim in (2, 3):
        for form in ("laplace_p1", "laplace_p2", "elastic_p1", "elastic_p2"):
            A = oracle.element(form, ref[dim], 1.0, 0.5)
            assert np.allclose(A, A.T), form
        x, w = oracle.gm_rule(dim, 2)
        assert abs(w.sum() - (0.5 if dim == 2 else 1.0 / 6.0)) < 1e-14
    m2 = meshgen.square_mesh(4, 0.2, 11, np.float64)
    m3 = meshgen.cube_mesh(2, 2, 2, 0.15, 12)
    mu, lam = meshgen.lame(m3.n_elements, 13)
    for form, m, a, b in (("laplace_p1", m2, None, None), ("laplace_p1", m3, None, None),
                          ("elastic_p1", m3, mu, lam)):
        A = oracle.integrate(form, m.coords, m.conn, a, b)
        dA = np.random.default_rng(14).standard_normal(A.shape)
        oracle.gradient(form, m.coords, m.conn, dA, a, b)
        K = oracle.assemble(form, m.coords, m.conn, a, b)
        assert K.shape[0] == K.shape[1]
    oracle.integrate_coefficient("laplace_p1", m3.coords, m3.conn,
                                 np.linspace(1.0, 2.0, m3.n_vertices))
    W = np.zeros((1, 4, 4))
    W[0, 1:, 1:] = np.eye(3)
    Ag = oracle.integrate_general(1, 1, W, m3.coords, m3.conn)
    assert np.allclose(Ag, oracle.integrate("laplace_p1", m3.coords, m3.conn), atol=1e-12)
    wi = meshgen.iso3d(2)
    oracle.integrate_iso(wi.mesh.coords, wi.mesh.conn, "projected")
    oracle.integrate_iso(wi.mesh.coords, wi.mesh.conn, "exact")
    print("oracle sanitized run OK")
""")


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's ASan runtime is not installed")
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "oracle.c"),
                    "-o", lib, "-lm"], check=True, cwd=str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", _DRIVER.format(root=ROOT, lib=lib)], env=env,
                       capture_output=True, text=True, timeout=900)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "oracle sanitized run OK" in r.stdout, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
