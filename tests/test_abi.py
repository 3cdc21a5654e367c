"""The C-ABI boundary on the CPU: exports, host-only entry points, argument
validation.  Nothing here launches a kernel."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

import meshgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

fei = pytest.importorskip("paper_1103_0066_amd")
from paper_1103_0066_amd import _lib  # noqa: E402


def _declared_entry_points():
    text = open(os.path.join(ROOT, "include", "fei.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fei_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_entry_points()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_version_and_status_strings():
    lib = _lib.load()
    assert lib.fei_abi_version() == _lib.ABI_VERSION == 2
    for s in (0, -1, -2, -3, -4):
        assert lib.fei_status_str(s)
    assert lib.fei_status_str(-99) == b"unknown status"


@pytest.mark.parametrize("form,dim,n", [("laplace_p1", 2, 3), ("laplace_p1", 3, 4),
                                        ("elastic_p1", 2, 6), ("elastic_p1", 3, 12),
                                        ("laplace_p2", 2, 6), ("laplace_p2", 3, 10)])
def test_local_size(form, dim, n):
    assert fei.local_size(form, dim) == n


def test_local_size_rejects_bad_args():
    with pytest.raises(fei.FeiError):
        fei.local_size("laplace_p1", 4)


def _physical(rng, dim):
    while True:
        x = rng.uniform(-1, 1, size=(dim + 1, dim))
        J = (x[1:] - x[0]).T
        if abs(np.linalg.det(J)) > 0.05:
            return x, J


@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3),
                                      ("laplace_p2", 2), ("laplace_p2", 3)])
def test_block_reference_tensor_reproduces_oracle(form, dim):
    """A_ij = K^{ij}_{mu nu} G^{mu nu}, G = J^-1 J^-T |J| (eqs. 6-8), against the oracle."""
    K = fei.reference_tensor(form, dim, "block")
    rng = np.random.default_rng(1)
    for _ in range(10):
        x, J = _physical(rng, dim)
        B = np.linalg.inv(J)
        G = B @ B.T * abs(np.linalg.det(J))
        A = np.einsum("ijmn,mn->ij", K.astype(np.float64), G)
        Ao = oracle.element(form, x)
        np.testing.assert_allclose(A, Ao, rtol=0, atol=2e-7 * np.abs(Ao).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_block_reference_tensor_elasticity(dim):
    """Vector element: A_(a,c),(b,d) = K^{ab}_{mu nu} T^{(mu c),(nu d)} with the Lame
    geometric tensor T; checks K (and the reading of eq. 15) against the oracle."""
    K = fei.reference_tensor("elastic_p1", dim, "block").astype(np.float64)
    rng = np.random.default_rng(2)
    for _ in range(10):
        x, J = _physical(rng, dim)
        B = np.linalg.inv(J)
        s = abs(np.linalg.det(J))
        mu, lam = 0.8, 1.7
        M = B @ B.T
        T = np.zeros((dim, dim, dim, dim))  # T[mu][c][nu][d]
        for m, c, n, d in itertools.product(range(dim), repeat=4):
            T[m, c, n, d] = s * (mu * ((c == d) * M[m, n] + B[m, d] * B[n, c])
                                 + lam * B[m, c] * B[n, d])
        A = np.einsum("abmn,mcnd->acbd", K, T).reshape(dim * (dim + 1), dim * (dim + 1))
        Ao = oracle.element("elastic_p1", x, mu, lam)
        np.testing.assert_allclose(A, Ao, rtol=0, atol=2e-7 * np.abs(Ao).max())


@pytest.mark.parametrize("form,dim", [("laplace_p1", 3), ("elastic_p1", 3), ("laplace_p2", 3),
                                      ("elastic_p1", 2)])
def test_folded_reference_tensor(form, dim):
    """Folded K is integer-valued (exact in FP16/BF16) and Gf . Kf equals the block form."""
    Kf = fei.reference_tensor(form, dim, "folded").astype(np.float64)
    assert np.all(Kf == np.round(Kf)) and np.abs(Kf).max() <= 256
    Kb = fei.reference_tensor(form, dim, "block").astype(np.float64)
    scale = fei.reference_scale(form, dim)
    n = fei.local_size(form, dim)
    gd = dim * dim if form == "elastic_p1" else dim
    rng = np.random.default_rng(3)
    S = rng.normal(size=(gd, gd)); S = S + S.T            # any symmetric geometric tensor
    gf = np.array([S[p, q] for p in range(gd) for q in range(p, gd)])
    A_fold = (gf @ Kf).reshape(n, n) * scale
    if form == "elastic_p1":
        T = S.reshape(dim, dim, dim, dim)                 # (mu c),(nu d)
        A_blk = np.einsum("abmn,mcnd->acbd", Kb, T).reshape(n, n)
    else:
        A_blk = np.einsum("ijmn,mn->ij", Kb, S)
    # the block tensor is returned in FP32 (entries like 1/6 round), the folded one is exact
    np.testing.assert_allclose(A_fold, A_blk, rtol=0, atol=1e-6 * np.abs(A_blk).max())


# ---------------------------------------------------------------------------
# argument validation (host side, returns before any device call)
# ---------------------------------------------------------------------------

FAKE = 0x10000  # never dereferenced: every call below fails validation first


def _fake_mesh(dim=3, E=10, nv=20, dtype=_lib.F32):
    m = _lib.FeiMesh()
    m.dim, m.coord_dtype, m.n_vertices, m.n_elements = dim, dtype, nv, E
    m.x = m.y = FAKE
    m.z = FAKE if dim == 3 else None
    m.conn = FAKE
    return m


def _opts(**kw):
    o = _lib.FeiOptions()
    _lib.load().fei_options_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _call(m, form=1, mu=None, lam=None, A=FAKE, opt=None):
    lib = _lib.load()
    return lib.fei_integrate(ctypes.byref(m) if m is not None else None, form, mu, lam, A,
                             ctypes.byref(opt) if opt is not None else None, None)


def test_options_default():
    o = _opts()
    assert o.precision == 0 and math.isclose(o.tau, 100.0) and not o.counters


@pytest.mark.parametrize("case", ["null_mesh", "bad_dim", "bad_dtype", "neg_E", "huge_E", "bad_form",
                                  "mu_for_laplace", "missing_mu", "bad_precision", "nan_tau",
                                  "reserved", "null_A", "misaligned_A", "null_conn",
                                  "misaligned_conn", "null_z", "zero_nv"])
def test_integrate_rejects(case):
    m = _fake_mesh()
    kw = {}
    if case == "null_mesh":
        m = None
    elif case == "bad_dim":
        m.dim = 4
    elif case == "bad_dtype":
        m.coord_dtype = 7
    elif case == "neg_E":
        m.n_elements = -1
    elif case == "huge_E":          # one launch covers at most 2^32 threads
        m.n_elements = 2 ** 32
    elif case == "bad_form":
        kw["form"] = 9
    elif case == "mu_for_laplace":
        kw["mu"] = FAKE
    elif case == "missing_mu":
        kw["form"] = 2
    elif case == "bad_precision":
        kw["opt"] = _opts(precision=5)
    elif case == "nan_tau":
        kw["opt"] = _opts(tau=float("nan"))
    elif case == "reserved":
        o = _opts(); o.reserved[1] = 3; kw["opt"] = o
    elif case == "null_A":
        kw["A"] = None
    elif case == "misaligned_A":
        kw["A"] = FAKE + 4
    elif case == "null_conn":
        m.conn = None
    elif case == "misaligned_conn":
        m.conn = FAKE + 4
    elif case == "null_z":
        m.z = None
    elif case == "zero_nv":
        m.n_vertices = 0
    rc = _call(m, **kw)
    assert rc == _lib.FEI_EINVAL, (case, rc)
    assert _lib.load().fei_last_error()


def test_empty_mesh_is_a_noop():
    m = _fake_mesh(E=0)
    assert _call(m, A=None) == 0
    lib = _lib.load()
    rc = lib.fei_integrate_adjoint(ctypes.byref(m), 1, None, None, None, None, None, None,
                                   None, None, None, None)
    assert rc == 0


def test_split_precision_adjoint_rejections():
    """Split-precision adjoints need FP32 coordinates, whole-matrix staging and
    n*n a multiple of 4: every other variant is refused before any launch."""
    lib = _lib.load()
    for prec in (1, 2, 3):
        cases = [(_fake_mesh(dtype=_lib.F64), 1, _opts(precision=prec)),     # FP64 coordinates
                 (_fake_mesh(dim=2), 1, _opts(precision=prec)),              # 3 x 3 matrices
                 (_fake_mesh(), 2, _opts(precision=prec, store_rows=2)),     # row chunks
                 (_fake_mesh(), 3, _opts(precision=prec, store_rows=-1))]    # direct reads
        for m, form, o in cases:
            coef = FAKE if form == 2 else None
            rc = lib.fei_integrate_adjoint(ctypes.byref(m), form, coef, coef, FAKE, FAKE, FAKE,
                                           FAKE if m.dim == 3 else None, None, None,
                                           ctypes.byref(o), None)
            assert rc == _lib.FEI_EUNSUPPORTED, (prec, form, m.dim, m.coord_dtype)


def test_adjoint_rejects_coefficient_grads_for_laplace():
    lib = _lib.load()
    m = _fake_mesh()
    rc = lib.fei_integrate_adjoint(ctypes.byref(m), 1, None, None, FAKE, FAKE, FAKE, FAKE,
                                   FAKE, None, None, None)
    assert rc == _lib.FEI_EINVAL


def test_reference_tensor_rejects():
    lib = _lib.load()
    n = ctypes.c_int64()
    assert lib.fei_reference_tensor(1, 3, 7, None, ctypes.byref(n), None) == _lib.FEI_EINVAL
    assert lib.fei_reference_tensor(1, 3, 0, None, None, None) == _lib.FEI_EINVAL
    assert lib.fei_reference_tensor(5, 3, 0, None, ctypes.byref(n), None) == _lib.FEI_EINVAL


def test_python_binding_refuses_cpu_tensors():
    import torch
    m = meshgen.cube_mesh(1, 1, 1, 0.0)
    coords = torch.from_numpy(m.soa())
    conn = torch.from_numpy(m.conn)
    with pytest.raises(ValueError):
        fei.integrate(coords, conn, "laplace_p1")


@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3), ("laplace_p2", 2),
                                      ("laplace_p2", 3)])
def test_coefficient_reference_tensor_reproduces_oracle(form, dim):
    """A_ij = sum_k w_k K^{ijk}_{mu nu} G^{mu nu} (Sec. 3.1, eq. 23) with the
    library's arity-3 K, against the oracle's quadrature with w interpolated."""
    K = fei.reference_tensor_coefficient(form, dim).astype(np.float64)
    rng = np.random.default_rng(3)
    for _ in range(10):
        x, J = _physical(rng, dim)
        B = np.linalg.inv(J)
        G = B @ B.T * abs(np.linalg.det(J))
        w = np.exp(rng.normal(size=dim + 1))
        A = np.einsum("ijkmn,k,mn->ij", K, w, G)
        Ao = oracle.integrate_coefficient(form, x, np.arange(dim + 1)[None], w)[0]
        np.testing.assert_allclose(A, Ao, rtol=0, atol=2e-7 * np.abs(Ao).max())


def test_coefficient_entry_point_rejects_without_device_work():
    """Argument checks of fei_integrate_coefficient run before any launch."""
    lib = _lib.load()
    m = _lib.FeiMesh()
    m.dim, m.coord_dtype, m.n_vertices, m.n_elements = 3, _lib.F32, 4, 0
    o = _lib.FeiOptions()
    lib.fei_options_default(ctypes.byref(o))
    # elasticity takes no scalar coefficient; E = 0 with a Laplacian is a no-op
    assert lib.fei_integrate_coefficient(ctypes.byref(m), 2, None, None, ctypes.byref(o),
                                         None) == _lib.FEI_EUNSUPPORTED
    assert lib.fei_integrate_coefficient(ctypes.byref(m), 1, None, None, ctypes.byref(o),
                                         None) == _lib.FEI_OK
    assert lib.fei_integrate_coefficient(ctypes.byref(m), 9, None, None, ctypes.byref(o),
                                         None) == _lib.FEI_EINVAL


def _det_workspace(dim, E, nv):
    up = lambda b: (b + 255) // 256 * 256
    return up(4 * (nv + 1)) + up(4 * nv) + up(4 * (dim + 1) * E) + up(4 * dim * dim * E)


def test_noalloc_adjoint_rejects_oversized_meshes_without_device_work():
    """The allocation-free deterministic adjoint refuses a mesh whose workspace
    exceeds its fixed array (checked on the host before any HIP call), and the
    deterministic path's other limits, with FEI_EINVAL / FEI_EUNSUPPORTED."""
    lib = _lib.load()
    cap = _lib.NOALLOC_SCRATCH_BYTES
    # 3D, 300,000 vertices: the smallest element count (in steps of 1,000) over the cap
    nv = 300000
    E = next(e for e in range(1_900_000, 2_100_000, 1000) if _det_workspace(3, e, nv) > cap)
    assert _det_workspace(3, 1572864, 290353) <= cap       # the 3D elasticity workload fits
    m = _fake_mesh(E=E, nv=nv)
    rc = lib.fei_integrate_adjoint_det_noalloc(ctypes.byref(m), 1, None, None, FAKE, FAKE, FAKE,
                                               FAKE, None, None, None, None)
    assert rc == _lib.FEI_EINVAL
    assert b"workspace" in lib.fei_last_error()
    m = _fake_mesh(dtype=_lib.F64)                       # FP32 coordinates only
    rc = lib.fei_integrate_adjoint_det_noalloc(ctypes.byref(m), 1, None, None, FAKE, FAKE, FAKE,
                                               FAKE, None, None, None, None)
    assert rc == _lib.FEI_EUNSUPPORTED
    o = _opts(store_rows=2)                              # its own dA staging
    rc = lib.fei_integrate_adjoint_det_noalloc(ctypes.byref(_fake_mesh()), 1, None, None, FAKE,
                                               FAKE, FAKE, FAKE, None, None, ctypes.byref(o), None)
    assert rc == _lib.FEI_EUNSUPPORTED
    m = _fake_mesh(E=0)                                  # E = 0: a no-op
    assert lib.fei_integrate_adjoint_det_noalloc(ctypes.byref(m), 1, None, None, None, None, None,
                                                 None, None, None, None, None) == 0


def test_iso_entry_point_rejects_without_device_work():
    lib = _lib.load()
    o = _opts()
    m = _fake_mesh(E=0)
    assert lib.fei_integrate_iso(ctypes.byref(m), None, ctypes.byref(o), None) == 0
    m = _fake_mesh(dtype=_lib.F64)
    assert lib.fei_integrate_iso(ctypes.byref(m), FAKE, ctypes.byref(o), None) == _lib.FEI_EUNSUPPORTED
    m = _fake_mesh()
    assert lib.fei_integrate_iso(ctypes.byref(m), None, ctypes.byref(o), None) == _lib.FEI_EINVAL
    assert lib.fei_integrate_iso(ctypes.byref(m), FAKE + 4, ctypes.byref(o), None) == _lib.FEI_EINVAL
    o2 = _opts(precision=1)
    assert lib.fei_integrate_iso(ctypes.byref(m), FAKE, ctypes.byref(o2), None) == _lib.FEI_EUNSUPPORTED


def test_tune_table_round_trip_and_lookup(tmp_path):
    """The tune table (host-only): a JSON-lines file loads, answers lookups by
    size bucket, saves back, and malformed lines are reported."""
    lib = _lib.load()
    lib.fei_tune_clear()
    src = tmp_path / "tune.jsonl"
    src.write_text('{"form": 2, "dim": 3, "precision": 0, "coord": 0, "ebucket": 20, '
                   '"block_elements": 512, "store_rows": 0, "ms": 0.2}\n'
                   '{"form": 1, "dim": 3, "precision": 1, "coord": 0, "ebucket": 20, '
                   '"block_elements": 256, "store_rows": -1, "ms": 0.05}\n')
    assert lib.fei_tune_load(str(src).encode()) == 0
    r = _lib.FeiTuneResult()
    assert lib.fei_tune_lookup(2, 3, 0, 0, 1572864, ctypes.byref(r)) == 1     # 2^20 <= E < 2^21
    assert (r.block_elements, r.store_rows) == (512, 0)
    assert lib.fei_tune_lookup(2, 3, 0, 0, 3 * 2 ** 20, ctypes.byref(r)) == 0  # other bucket
    assert lib.fei_tune_lookup(1, 3, 1, 0, 2 ** 20, ctypes.byref(r)) == 1 and r.store_rows == -1
    dst = tmp_path / "out.jsonl"
    assert lib.fei_tune_save(str(dst).encode()) == 0
    lines = dst.read_text().splitlines()
    assert len(lines) == 2 and all('"block_elements"' in l for l in lines)
    lib.fei_tune_clear()
    assert lib.fei_tune_lookup(2, 3, 0, 0, 1572864, ctypes.byref(r)) == 0
    assert lib.fei_tune_load(str(dst).encode()) == 0
    assert lib.fei_tune_lookup(2, 3, 0, 0, 1572864, ctypes.byref(r)) == 1
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"form": 2, "dim": 3}\n')
    assert lib.fei_tune_load(str(bad).encode()) == _lib.FEI_EINVAL
    assert lib.fei_tune_load(str(tmp_path / "missing").encode()) == _lib.FEI_EINVAL
    lib.fei_tune_clear()


def test_tune_file_from_environment(tmp_path):
    """FEI_TUNE_FILE is read on first use of the table (a fresh process)."""
    import subprocess
    import sys
    src = tmp_path / "env.jsonl"
    src.write_text('{"form": 3, "dim": 3, "precision": 0, "coord": 0, "ebucket": 10, '
                   '"block_elements": 128, "store_rows": 0, "ms": 0.01}\n')
    code = ("import ctypes, sys; sys.path.insert(0, %r)\n"
            "from paper_1103_0066_amd import _lib\n"
            "lib = _lib.load(); r = _lib.FeiTuneResult()\n"
            "print(lib.fei_tune_lookup(3, 3, 0, 0, 1500, ctypes.byref(r)), r.block_elements)\n" % ROOT)
    env = dict(os.environ, FEI_TUNE_FILE=str(src))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=120)
    assert out.stdout.split() == ["1", "128"], out.stderr


def test_block_elements_is_validated():
    m = _fake_mesh()
    assert _call(m, opt=_opts(block_elements=96)) == _lib.FEI_EINVAL
