"""Split-precision MFMA adjoint: the fold of dA with K (the contraction of
eq. 1 in reverse) on the matrix cores with dA split into 16-bit terms, against
the oracle's gradients, with the FP32 reverse geometry and the FP64 path for
flagged elements.  Tolerances are those of the split forward (the split error
sits in the data operand of the same contraction: G forward, dA here)."""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import TOL, mesh_to_device, vec_to_device, vertex_scale

pytestmark = pytest.mark.gpu

fei = pytest.importorskip("paper_1103_0066_amd")

PRECS = ["fp16x2", "bf16x2", "bf16x3"]


def _case(name):
    if name == "lap3d":
        return meshgen.flatten_elements(meshgen.cube_mesh(5, 5, 4, 0.15, 142), 6, 143), "laplace_p1", None, None
    if name == "elast3d":
        m = meshgen.flatten_elements(meshgen.cube_mesh(6, 5, 5, 0.15, 143), 9, 144)
        mu, lam = meshgen.lame(m.n_elements, 145)
        return m, "elastic_p1", mu, lam
    if name == "elast2d":
        m = meshgen.square_mesh(17, 0.2, 146, np.float32)
        mu, lam = meshgen.lame(m.n_elements, 147)
        return m, "elastic_p1", mu, lam
    if name == "p2_3d":
        return meshgen.flatten_elements(meshgen.cube_mesh(4, 4, 4, 0.15, 148), 5, 149), "laplace_p2", None, None
    if name == "p2_2d":
        return meshgen.square_mesh(13, 0.2, 150, np.float32), "laplace_p2", None, None
    raise KeyError(name)


def _coeff_scale(coords, conn, dA):
    E = conn.shape[0]
    one, zero = np.ones(E), np.zeros(E)
    d = np.abs(np.asarray(dA, np.float64).reshape(E, -1))
    Am = np.abs(oracle.integrate("elastic_p1", coords, conn, one, zero).reshape(E, -1))
    Al = np.abs(oracle.integrate("elastic_p1", coords, conn, zero, one).reshape(E, -1))
    return (d * Am).sum(axis=1), (d * Al).sum(axis=1)


def _errors(m, form, mu, lam, dA, g, dmu, dlam):
    gv, gm, gl, _ = oracle.gradient(form, m.coords, m.conn, dA, mu, lam)
    go = oracle.vertex_gradient(gv, m.conn, m.n_vertices)
    scale = vertex_scale(gv, m.conn, m.n_vertices)
    used = scale > 0
    verr = float((np.abs(g - go).max(axis=1)[used] / scale[used]).max())
    cerr = 0.0
    if dmu is not None:
        sm, sl = _coeff_scale(m.coords, m.conn, dA)
        cerr = float(np.maximum(np.abs(dmu - gm) / sm, np.abs(dlam - gl) / sl).max())
    return verr, cerr


def _run(m, form, mu, lam, dA, prec, **kw):
    coords, conn = mesh_to_device(m)
    extra = {}
    if form == "elastic_p1":
        extra = {k: torch.full((m.n_elements,), float("nan"), device="cuda") for k in ("dmu", "dlam")}
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, vec_to_device(dA), vec_to_device(mu),
                                          vec_to_device(lam), precision=prec, **extra, **kw)
    torch.cuda.synchronize()
    return (dc.cpu().numpy().T.astype(np.float64), None if dmu is None else dmu.cpu().numpy(),
            None if dlam is None else dlam.cpu().numpy())


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["lap3d", "elast3d", "elast2d", "p2_3d", "p2_2d"])
def test_mfma_adjoint_matches_oracle(case, prec):
    m, form, mu, lam = _case(case)
    n = fei.local_size(form, m.dim)
    dA = meshgen.upstream(m.n_elements, n, 151)
    print(f"[mfma adjoint] {case} {prec} E={m.n_elements}", flush=True)
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    g, dmu, dlam = _run(m, form, mu, lam, dA, prec, counters=cnt)
    verr, cerr = _errors(m, form, mu, lam, dA, g, dmu, dlam)
    print(f"  vertex err {verr:.3e}  coeff err {cerr:.3e}", flush=True)
    assert verr <= TOL[prec] and cerr <= TOL[prec]
    assert cnt.cpu().tolist()[0] == (0 if m.flattened is None else len(m.flattened))
    # whole-matrix staging asked for explicitly: the same kernel, the same bits
    g2, _, _ = _run(m, form, mu, lam, dA, prec, store_rows=n)
    assert np.abs(g2 - g).max() <= 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("form", ["elastic_p1", "laplace_p2", "laplace_p1"])
def test_mfma_adjoint_with_many_flagged_elements(form, prec):
    """A third of the elements flattened: each wave folds its first two flagged
    elements in FP64 while their chunk is staged and rereads the dA of the
    rest; all of them against the oracle."""
    m = meshgen.cube_mesh(6, 5, 4, 0.15, 171)
    m = meshgen.flatten_elements(m, m.n_elements // 3, 172)
    mu = lam = None
    if form == "elastic_p1":
        mu, lam = meshgen.lame(m.n_elements, 173)
    dA = meshgen.upstream(m.n_elements, fei.local_size(form, 3), 174)
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    g, dmu, dlam = _run(m, form, mu, lam, dA, prec, counters=cnt)
    verr, cerr = _errors(m, form, mu, lam, dA, g, dmu, dlam)
    print(f"[mfma flagged] {form} {prec}: vertex {verr:.3e} coeff {cerr:.3e}", flush=True)
    assert verr <= TOL[prec] and cerr <= TOL[prec]
    assert cnt.cpu().tolist() == [len(m.flattened), 0]


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x3"])
def test_mfma_adjoint_every_tile_count(prec):
    """1 to 11 tiles of the persistent grid, ragged tails: every element and
    vertex contribution counted once."""
    m = meshgen.flatten_elements(meshgen.cube_mesh(8, 8, 8, 0.15, 161), 20, 162)
    mu, lam = meshgen.lame(m.n_elements, 163)
    for E in (1, 15, 17, 63, 255, 257, 3 * 256 + 5, 8 * 256 + 1, 2600):
        sub = meshgen.Mesh(m.coords, np.ascontiguousarray(m.conn[:E]))
        dA = meshgen.upstream(E, 12, 164 + E)
        g, dmu, dlam = _run(sub, "elastic_p1", mu[:E], lam[:E], dA, prec)
        gv, _, _, _ = oracle.gradient("elastic_p1", m.coords, sub.conn, dA, mu[:E], lam[:E])
        scale = vertex_scale(gv, sub.conn, m.n_vertices)
        assert np.all(g[scale == 0] == 0), E
        verr, cerr = _errors(sub, "elastic_p1", mu[:E], lam[:E], dA, g, dmu, dlam)
        assert verr <= TOL[prec] and cerr <= TOL[prec], (E, verr, cerr)


@pytest.mark.parametrize("prec", PRECS)
def test_mfma_deterministic_adjoint_repeats(prec):
    """The deterministic form (J-bar per element, vertex gather) with the MFMA
    fold: against the oracle, and the same bits on every call."""
    m, form, mu, lam = _case("elast3d")
    dA = meshgen.upstream(m.n_elements, 12, 181)
    g1, dmu, dlam = _run(m, form, mu, lam, dA, prec, deterministic=True)
    g2, _, _ = _run(m, form, mu, lam, dA, prec, deterministic=True)
    assert np.array_equal(g1, g2)
    verr, cerr = _errors(m, form, mu, lam, dA, g1, dmu, dlam)
    assert verr <= TOL[prec] and cerr <= TOL[prec]


def test_mfma_adjoint_scale_extremes():
    """FP16x2 scales each element by a power of two: matrices of 1e-30 and 1e30
    (far outside FP16's range) fold as accurately as unit ones, and Inf in dA
    stays in its element's gradients."""
    m, form, mu, lam = _case("elast3d")
    dA = meshgen.upstream(m.n_elements, 12, 191)
    s = np.ones(m.n_elements, np.float32)
    s[::3] = 1e-30
    s[1::3] = 1e30
    dA_s = dA * s[:, None, None]
    g, dmu, dlam = _run(m, form, mu, lam, dA_s, "fp16x2")
    gv, gm, gl, _ = oracle.gradient(form, m.coords, m.conn, dA_s.astype(np.float64), mu, lam)
    # per-element coefficient gradients, each against its own element's scale
    sm, sl = _coeff_scale(m.coords, m.conn, dA_s)
    assert float(np.maximum(np.abs(dmu - gm) / sm, np.abs(dlam - gl) / sl).max()) <= TOL["fp16x2"]
    bad = dA.copy()
    bad[5, 3, 7] = np.inf
    _, dmu_b, _ = _run(m, form, mu, lam, bad, "fp16x2")
    assert not np.isfinite(dmu_b[5])
    assert np.isfinite(np.delete(dmu_b, 5)).all()


def test_mfma_adjoint_rejections():
    m2 = meshgen.square_mesh(5, 0.2, 201, np.float32)
    coords, conn = mesh_to_device(m2)
    dA = vec_to_device(meshgen.upstream(m2.n_elements, 3, 202))
    with pytest.raises(fei.FeiError) as ex:      # 3 x 3 matrices: no whole-matrix staging
        fei.integrate_adjoint(coords, conn, "laplace_p1", dA, precision="fp16x2")
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED
    m, form, mu, lam = _case("elast3d")
    coords, conn = mesh_to_device(m)
    dA = vec_to_device(meshgen.upstream(m.n_elements, 12, 203))
    with pytest.raises(fei.FeiError) as ex:      # row-chunk staging
        fei.integrate_adjoint(coords, conn, form, dA, vec_to_device(mu), vec_to_device(lam),
                              precision="bf16x2", store_rows=2)
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED
    with pytest.raises(fei.FeiError) as ex:      # FP64 coordinates
        fei.integrate_adjoint(coords.double(), conn, form, dA, vec_to_device(mu),
                              vec_to_device(lam), precision="bf16x3")
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x2"])
def test_full_mfma_adjoint_sampled(prec):
    """The full 1.57M-tet elasticity adjoint in split precision (bench.py's
    launch): sampled coefficient and vertex gradients against the oracle."""
    w = meshgen.elast3d_adjoint(64)
    m = w.mesh
    print(f"[full mfma adjoint] {prec}", flush=True)
    coords, conn = mesh_to_device(m)
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, w.form, vec_to_device(w.dA),
                                          vec_to_device(w.mu), vec_to_device(w.lam),
                                          precision=prec)
    rng = np.random.Generator(np.random.PCG64(19))
    idx = np.union1d(rng.choice(m.n_elements, 3000, replace=False), m.flattened[:500])
    _, gm, gl, _ = oracle.gradient(w.form, m.coords, m.conn[idx], w.dA[idx], w.mu[idx], w.lam[idx])
    sm, sl = _coeff_scale(m.coords, m.conn[idx], w.dA[idx])
    dmu_s, dlam_s = dmu.cpu().numpy()[idx], dlam.cpu().numpy()[idx]
    cerr = float(np.maximum(np.abs(dmu_s - gm) / sm, np.abs(dlam_s - gl) / sl).max())
    verts = rng.choice(m.n_vertices, 300, replace=False)
    inc = np.nonzero(np.isin(m.conn, verts).any(axis=1))[0]
    gv, _, _, _ = oracle.gradient(w.form, m.coords, m.conn[inc], w.dA[inc], w.mu[inc], w.lam[inc])
    go = oracle.vertex_gradient(gv, m.conn[inc], m.n_vertices)[verts]
    sc = vertex_scale(gv, m.conn[inc], m.n_vertices)[verts]
    gg = dc.cpu().numpy().T[verts]
    ok = sc > 0
    verr = float((np.abs(gg - go).max(axis=1)[ok] / sc[ok]).max())
    print(f"  sampled vertex err {verr:.3e}, coeff err {cerr:.3e}", flush=True)
    assert verr <= TOL[prec] and cerr <= TOL[prec]


def test_autograd_backward_on_the_matrix_cores():
    """element_matrices(..., adjoint_precision=...) runs the split-precision
    adjoint as its backward: the same gradients as the direct call."""
    m, form, mu, lam = _case("elast3d")
    coords, conn = mesh_to_device(m)
    c = coords.clone().requires_grad_(True)
    mu_d = vec_to_device(mu).requires_grad_(True)
    lam_d = vec_to_device(lam).requires_grad_(True)
    dA = vec_to_device(meshgen.upstream(m.n_elements, 12, 211))
    A = fei.element_matrices(c, conn, form, mu_d, lam_d, adjoint_precision="fp16x2")
    (A * dA).sum().backward()
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, dA, vec_to_device(mu),
                                          vec_to_device(lam), precision="fp16x2")
    tol = 1e-6
    torch.testing.assert_close(c.grad, dc, rtol=0, atol=tol * float(dc.abs().max()))
    torch.testing.assert_close(mu_d.grad, dmu, rtol=0, atol=tol * float(dmu.abs().max()))
    torch.testing.assert_close(lam_d.grad, dlam, rtol=0, atol=tol * float(dlam.abs().max()))
