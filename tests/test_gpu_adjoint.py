"""Adjoint parity: HIP adjoint against the oracle's complex-step gradients,
central differences, invariants at full size, and the autograd wiring."""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import (TOL_COEFF, TOL_FD_FLAT, TOL_VERTEX, mesh_to_device, vec_to_device,
                      vertex_scale)

pytestmark = pytest.mark.gpu

fei = pytest.importorskip("paper_1103_0066_amd")


def _case(name):
    if name == "lap2d_f64":
        return meshgen.square_mesh(17, 0.2, 41, np.float64), "laplace_p1", None, None
    if name == "lap3d":
        return meshgen.cube_mesh(5, 5, 4, 0.15, 42), "laplace_p1", None, None
    if name == "elast3d":
        m = meshgen.flatten_elements(meshgen.cube_mesh(6, 5, 5, 0.15, 43), 9, 44)
        mu, lam = meshgen.lame(m.n_elements, 45)
        return m, "elastic_p1", mu, lam
    if name == "elast2d":
        m = meshgen.square_mesh(17, 0.2, 46, np.float32)
        mu, lam = meshgen.lame(m.n_elements, 47)
        return m, "elastic_p1", mu, lam
    if name == "p2_3d":
        return meshgen.cube_mesh(4, 4, 4, 0.15, 48), "laplace_p2", None, None
    raise KeyError(name)


def _nan_coeff_buffers(mesh, form):
    if form != "elastic_p1":
        return {}
    return {k: torch.full((mesh.n_elements,), float("nan"), device="cuda") for k in ("dmu", "dlam")}


def _gpu_adjoint(mesh, form, mu, lam, dA):
    coords, conn = mesh_to_device(mesh)
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, vec_to_device(dA),
                                          vec_to_device(mu), vec_to_device(lam),
                                          **_nan_coeff_buffers(mesh, form))
    torch.cuda.synchronize()
    g = dc.cpu().numpy().T.astype(np.float64)      # [N_v, dim]
    return (g, None if dmu is None else dmu.cpu().numpy(),
            None if dlam is None else dlam.cpu().numpy())


def _check_against_oracle(mesh, form, mu, lam, dA, conn_sel=None):
    g, dmu, dlam = _gpu_adjoint(mesh, form, mu, lam, dA)
    gv, gm, gl, Le = oracle.gradient(form, mesh.coords, mesh.conn, dA, mu, lam)
    go = oracle.vertex_gradient(gv, mesh.conn, mesh.n_vertices)
    scale = vertex_scale(gv, mesh.conn, mesh.n_vertices)
    used = scale > 0
    verr = np.abs(g - go).max(axis=1)[used] / scale[used]
    print(f"  vertex err max {verr.max():.3e}")
    assert verr.max() <= TOL_VERTEX
    if gm is not None:
        merr = _coeff_errors(mesh.coords, mesh.conn, dA, dmu, dlam, gm, gl)
        print(f"  coeff err max {merr.max():.3e}")
        assert merr.max() <= TOL_COEFF
    return g, go


def _coeff_errors(coords, conn, dA, dmu, dlam, gm, gl):
    """A is linear in (mu, lambda), so dL/dmu_e = <dA_e, A_e(mu=1, lambda=0)>; each
    coefficient gradient is judged against sum |dA_e| |A_e(1, 0)| (resp. (0, 1)),
    the scale of the sum it is made of."""
    E = conn.shape[0]
    one, zero = np.ones(E), np.zeros(E)
    dA = np.asarray(dA, np.float64).reshape(E, -1)
    Am = oracle.integrate("elastic_p1", coords, conn, one, zero).reshape(E, -1)
    Al = oracle.integrate("elastic_p1", coords, conn, zero, one).reshape(E, -1)
    sm = (np.abs(dA) * np.abs(Am)).sum(axis=1)
    sl = (np.abs(dA) * np.abs(Al)).sum(axis=1)
    return np.maximum(np.abs(dmu - gm) / sm, np.abs(dlam - gl) / sl)


@pytest.mark.parametrize("case", ["lap2d_f64", "lap3d", "elast3d", "elast2d", "p2_3d"])
def test_adjoint_matches_oracle(case):
    mesh, form, mu, lam = _case(case)
    n = fei.local_size(form, mesh.dim)
    dA = meshgen.upstream(mesh.n_elements, n, 49)
    print(f"[adjoint] {case} E={mesh.n_elements}", flush=True)
    _check_against_oracle(mesh, form, mu, lam, dA)


@pytest.mark.parametrize("case,rows", [("elast3d", r) for r in (-1, 2, 3, 4, 12)] +
                         [("lap3d", r) for r in (-1, 2, 4)] + [("p2_3d", r) for r in (-1, 2, 10)] +
                         [("elast2d", r) for r in (-1, 2, 6)])
def test_adjoint_staging_modes(case, rows):
    mesh, form, mu, lam = _case(case)
    n = fei.local_size(form, mesh.dim)
    dA = meshgen.upstream(mesh.n_elements, n, 52)
    coords, conn = mesh_to_device(mesh)
    outs = []
    for r in (rows, 0):
        dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, vec_to_device(dA),
                                              vec_to_device(mu), vec_to_device(lam),
                                              store_rows=r, **_nan_coeff_buffers(mesh, form))
        outs.append((dc.cpu().numpy().T.astype(np.float64),
                     None if dmu is None else dmu.cpu().numpy(),
                     None if dlam is None else dlam.cpu().numpy()))
    gv, gm, gl, _ = oracle.gradient(form, mesh.coords, mesh.conn, dA, mu, lam)
    go = oracle.vertex_gradient(gv, mesh.conn, mesh.n_vertices)
    scale = vertex_scale(gv, mesh.conn, mesh.n_vertices)
    used = scale > 0
    for g, dmu, dlam in outs:
        assert (np.abs(g - go).max(axis=1)[used] / scale[used]).max() <= TOL_VERTEX
        # per-element outputs: each mode against the oracle (the modes are
        # separate kernel instantiations, whose multiply-add fusion may differ)
        if dmu is not None:
            assert _coeff_errors(mesh.coords, mesh.conn, dA, dmu, dlam, gm, gl).max() <= TOL_COEFF


def test_adjoint_staging_beyond_register_budget_is_rejected():
    # two 6-row chunks of a 12x12 dA (72 floats each) do not fit a lane's registers
    mesh, form, mu, lam = _case("elast3d")
    coords, conn = mesh_to_device(mesh)
    dA = meshgen.upstream(mesh.n_elements, 12, 53)
    with pytest.raises(fei.FeiError) as ex:
        fei.integrate_adjoint(coords, conn, form, vec_to_device(dA), vec_to_device(mu),
                              vec_to_device(lam), store_rows=6)
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED


@pytest.mark.parametrize("form,rows", [("elastic_p1", 12), ("laplace_p2", 0), ("laplace_p1", 0)])
def test_adjoint_whole_staging_with_many_flagged_elements(form, rows):
    """Whole-matrix staging folds the first two flagged elements of a wave in
    FP64 while their chunk is staged and rereads the dA of further ones: a
    mesh with a third of its elements flattened (many per wave) against the
    oracle, and the FP64-path counter."""
    m = meshgen.cube_mesh(6, 5, 4, 0.15, 71)
    m = meshgen.flatten_elements(m, m.n_elements // 3, 72)
    mu = lam = None
    if form == "elastic_p1":
        mu, lam = meshgen.lame(m.n_elements, 73)
    n = fei.local_size(form, 3)
    dA = meshgen.upstream(m.n_elements, n, 74)
    coords, conn = mesh_to_device(m)
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, vec_to_device(dA), vec_to_device(mu),
                                          vec_to_device(lam), store_rows=rows, counters=cnt,
                                          **_nan_coeff_buffers(m, form))
    g = dc.cpu().numpy().T.astype(np.float64)
    gv, gm, gl, _ = oracle.gradient(form, m.coords, m.conn, dA, mu, lam)
    go = oracle.vertex_gradient(gv, m.conn, m.n_vertices)
    scale = vertex_scale(gv, m.conn, m.n_vertices)
    used = scale > 0
    assert (np.abs(g - go).max(axis=1)[used] / scale[used]).max() <= TOL_VERTEX
    if dmu is not None:
        assert _coeff_errors(m.coords, m.conn, dA, dmu.cpu().numpy(), dlam.cpu().numpy(),
                             gm, gl).max() <= TOL_COEFF
    assert cnt.cpu().tolist() == [len(m.flattened), 0]


@pytest.mark.parametrize("rows", [0, -1, 2, 12])
def test_adjoint_every_tile_count_is_covered(rows):
    """1 to 11 workgroup tiles (the persistent adjoint splits tiles over the XCDs
    that have workgroups): every element and vertex contribution counted once."""
    m = meshgen.flatten_elements(meshgen.cube_mesh(8, 8, 8, 0.15, 61), 20, 62)
    mu, lam = meshgen.lame(m.n_elements, 63)
    for E in (1, 63, 255, 256, 257, 3 * 256 + 5, 7 * 256, 8 * 256 + 1, 9 * 256 + 100, 2600):
        sub = meshgen.Mesh(m.coords, np.ascontiguousarray(m.conn[:E]))
        dA = meshgen.upstream(E, 12, 64 + E)
        coords, conn = mesh_to_device(sub)
        dc, dmu, dlam = fei.integrate_adjoint(coords, conn, "elastic_p1", vec_to_device(dA),
                                              vec_to_device(mu[:E]), vec_to_device(lam[:E]),
                                              store_rows=rows, **_nan_coeff_buffers(sub, "elastic_p1"))
        g = dc.cpu().numpy().T.astype(np.float64)
        gv, gm, gl, _ = oracle.gradient("elastic_p1", m.coords, sub.conn, dA, mu[:E], lam[:E])
        go = oracle.vertex_gradient(gv, sub.conn, m.n_vertices)
        scale = vertex_scale(gv, sub.conn, m.n_vertices)
        used = scale > 0
        assert np.all(g[~used] == 0), E                      # untouched vertices stay zero
        assert (np.abs(g - go).max(axis=1)[used] / scale[used]).max() <= TOL_VERTEX, E
        assert _coeff_errors(m.coords, sub.conn, dA, dmu.cpu().numpy(), dlam.cpu().numpy(),
                             gm, gl).max() <= TOL_COEFF, E


@pytest.mark.parametrize("flat", [False, True])
def test_adjoint_fd_submesh(flat):
    """The 48-tet sub-mesh: GPU vs the oracle gradient and FP64 central differences."""
    w = meshgen.fd_submesh(flat)
    m = w.mesh
    g, go = _check_against_oracle(m, w.form, w.mu, w.lam, w.dA)
    X = m.coords.astype(np.float64)
    h = 1e-9 if flat else 1e-6 / 64

    def L(Xp):
        return float(np.sum(oracle.integrate(w.form, Xp, m.conn, w.mu, w.lam) * w.dA))
    fd = np.zeros_like(X)
    for v in range(m.n_vertices):
        for a in range(3):
            Xp = X.copy(); Xp[v, a] += h
            Xm = X.copy(); Xm[v, a] -= h
            fd[v, a] = (L(Xp) - L(Xm)) / (2 * h)
    np.testing.assert_allclose(go, fd, rtol=0, atol=1e-7 * np.abs(fd).max())
    err = np.abs(g - fd).max() / np.abs(fd).max()
    print(f"  GPU vs FD: {err:.3e}")
    assert err <= (TOL_FD_FLAT if flat else TOL_VERTEX)


def test_adjoint_accumulates_into_given_buffer():
    mesh, form, mu, lam = _case("lap3d")
    coords, conn = mesh_to_device(mesh)
    dA = vec_to_device(meshgen.upstream(mesh.n_elements, 4, 50))
    d1, _, _ = fei.integrate_adjoint(coords, conn, form, dA)
    base = torch.full_like(d1, 0.5)
    d2, _, _ = fei.integrate_adjoint(coords, conn, form, dA, dcoords=base.clone())
    torch.testing.assert_close(d2 - 0.5, d1, rtol=0, atol=1e-5 * float(d1.abs().max()))


def test_autograd_function_matches_adjoint():
    mesh, form, mu, lam = _case("elast3d")
    coords, conn = mesh_to_device(mesh)
    c = coords.clone().requires_grad_(True)
    m_ = vec_to_device(mu).requires_grad_(True)
    l_ = vec_to_device(lam).requires_grad_(True)
    A = fei.element_matrices(c, conn, form, m_, l_)
    dA = vec_to_device(meshgen.upstream(mesh.n_elements, 12, 51))
    (A * dA).sum().backward()
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, dA, vec_to_device(mu),
                                          vec_to_device(lam))
    torch.testing.assert_close(c.grad, dc, rtol=0, atol=TOL_VERTEX * float(dc.abs().max()))
    torch.testing.assert_close(m_.grad, dmu, rtol=0, atol=1e-5 * float(dmu.abs().max()))
    torch.testing.assert_close(l_.grad, dlam, rtol=0, atol=1e-5 * float(dlam.abs().max()))


def test_full_adjoint_sampled_and_invariants():
    """The full elasticity adjoint workload (bench.py's launch): sampled
    coefficient gradients and vertex gradients against the oracle, and the
    translation / Euler / Lame-linearity invariants over the whole mesh."""
    w = meshgen.elast3d_adjoint(64)
    m = w.mesh
    print(f"[full adjoint] {w.name}", flush=True)
    coords, conn = mesh_to_device(m)
    mu, lam = vec_to_device(w.mu), vec_to_device(w.lam)
    dA = vec_to_device(w.dA)
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, w.form, dA, mu, lam,
                                          **_nan_coeff_buffers(m, w.form))
    assert not bool(torch.isnan(dmu).any() or torch.isnan(dlam).any())
    A = fei.integrate(coords, conn, w.form, mu, lam)
    L = float((A.double() * dA.double()).sum())
    # invariants
    g = dc.double()
    X = coords.double()
    absg = g.abs().sum()
    assert float(g.sum(dim=1).abs().max()) <= 1e-4 * float(absg)
    euler = float((X * g).sum())
    assert abs(euler - L) <= 1e-4 * (float((X * g).abs().sum()) + abs(L))
    lin = float((mu.double() * dmu.double() + lam.double() * dlam.double()).sum())
    assert abs(lin - L) <= 1e-5 * float((mu.double() * dmu.double()).abs().sum()
                                       + (lam.double() * dlam.double()).abs().sum())
    # sampled coefficient gradients
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.union1d(rng.choice(m.n_elements, 3000, replace=False), m.flattened[:500])
    gv, gm, gl, _ = oracle.gradient(w.form, m.coords, m.conn[idx], w.dA[idx], w.mu[idx],
                                    w.lam[idx])
    dmu_s, dlam_s = dmu.cpu().numpy()[idx], dlam.cpu().numpy()[idx]
    merr = _coeff_errors(m.coords, m.conn[idx], w.dA[idx], dmu_s, dlam_s, gm, gl)
    assert merr.max() <= TOL_COEFF
    # sampled vertex gradients: every element incident to the sampled vertices
    verts = rng.choice(m.n_vertices, 300, replace=False)
    inc = np.nonzero(np.isin(m.conn, verts).any(axis=1))[0]
    gv, _, _, _ = oracle.gradient(w.form, m.coords, m.conn[inc], w.dA[inc], w.mu[inc], w.lam[inc])
    go = oracle.vertex_gradient(gv, m.conn[inc], m.n_vertices)[verts]
    sc = vertex_scale(gv, m.conn[inc], m.n_vertices)[verts]
    gg = dc.cpu().numpy().T[verts]
    ok = sc > 0
    verr = (np.abs(gg - go).max(axis=1)[ok] / sc[ok]).max()
    print(f"  sampled vertex err {verr:.3e}, coeff err {merr.max():.3e}")
    assert verr <= TOL_VERTEX


# ---------------------------------------------------------------------------
# degenerate elements and non-finite coordinates
# ---------------------------------------------------------------------------

def _vertices_of(conn, elems):
    return np.unique(conn[elems].ravel())


@pytest.mark.parametrize("form,dim", [("laplace_p1", 3), ("elastic_p1", 3), ("laplace_p1", 2),
                                      ("elastic_p1", 2)])
def test_adjoint_degenerate_elements_counted_and_isolated(form, dim):
    """det J == 0 (also with adj J == 0): counted as singular, non-finite only in
    that element's dmu, dlam and at its own vertices."""
    from test_gpu_forward import _degenerate_mesh
    mesh, bad = _degenerate_mesh(dim)
    n = fei.local_size(form, dim)
    mu = lam = None
    if form == "elastic_p1":
        mu, lam = meshgen.lame(mesh.n_elements, 91)
    dA = meshgen.upstream(mesh.n_elements, n, 92)
    coords, conn = mesh_to_device(mesh)
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, vec_to_device(dA), vec_to_device(mu),
                                          vec_to_device(lam), counters=cnt,
                                          **_nan_coeff_buffers(mesh, form))
    assert cnt.cpu().tolist() == [len(bad), len(bad)]
    g = dc.cpu().numpy().T
    good = np.setdiff1d(np.arange(mesh.n_elements), bad)
    hit = _vertices_of(mesh.conn, bad)
    clean = np.setdiff1d(np.arange(mesh.n_vertices), hit)
    assert np.all(np.isfinite(g[clean]))
    gv, gm, gl, _ = oracle.gradient(form, mesh.coords, mesh.conn[good], dA[good],
                                    None if mu is None else mu[good],
                                    None if lam is None else lam[good])
    go = oracle.vertex_gradient(gv, mesh.conn[good], mesh.n_vertices)
    sc = vertex_scale(gv, mesh.conn[good], mesh.n_vertices)
    ok = np.intersect1d(clean, np.nonzero(sc > 0)[0])
    assert (np.abs(g[ok] - go[ok]).max(axis=1) / sc[ok]).max() <= TOL_VERTEX
    for e in bad:
        assert not np.all(np.isfinite(g[mesh.conn[e]]))
    if dmu is not None:
        dmu_h, dlam_h = dmu.cpu().numpy(), dlam.cpu().numpy()
        assert not np.isfinite(dmu_h[bad]).any() or not np.isfinite(dlam_h[bad]).any()
        assert _coeff_errors(mesh.coords, mesh.conn[good], dA[good], dmu_h[good], dlam_h[good],
                             gm, gl).max() <= TOL_COEFF


@pytest.mark.parametrize("plan", [False, True])
@pytest.mark.parametrize("case", ["lap3d", "elast3d"])
def test_adjoint_nonfinite_coordinate_stays_local(case, plan):
    """A NaN coordinate reaches only the gradients of the elements that use the
    vertex and of their vertices, through the atomic scatter (single call) and
    through the vertex gather (one-mesh plan)."""
    mesh, form, mu, lam = _case(case)
    X = mesh.coords.copy()
    v = int(mesh.conn[len(mesh.conn) // 2, 1])
    X[v, 2] = np.nan
    n = fei.local_size(form, mesh.dim)
    dA = meshgen.upstream(mesh.n_elements, n, 93)
    bad_mesh = meshgen.Mesh(X, mesh.conn)
    coords, conn = mesh_to_device(bad_mesh)
    dcoords = torch.zeros((mesh.dim, mesh.n_vertices), dtype=torch.float32, device="cuda")
    bufs = _nan_coeff_buffers(mesh, form)
    if plan:
        it = {"form": form, "coords": coords, "conn": conn, "dA": vec_to_device(dA),
              "dcoords": dcoords}
        if mu is not None:
            it.update(mu=vec_to_device(mu), lam=vec_to_device(lam), **bufs)
        b = fei.Batch([it])
        b.set_config({"mode": 3, "variant": 0, "gather": 1}, adjoint=True)
        b.run_adjoint()
        torch.cuda.synchronize()
        dmu, dlam = it.get("dmu"), it.get("dlam")
        b.close()
    else:
        _, dmu, dlam = fei.integrate_adjoint(coords, conn, form, vec_to_device(dA),
                                             vec_to_device(mu), vec_to_device(lam),
                                             dcoords=dcoords, **bufs)
    g = dcoords.cpu().numpy().T
    touched = np.nonzero(np.isin(mesh.conn, [v]).any(axis=1))[0]
    good = np.setdiff1d(np.arange(mesh.n_elements), touched)
    hit = _vertices_of(mesh.conn, touched)
    clean = np.setdiff1d(np.arange(mesh.n_vertices), hit)
    assert np.isnan(g[hit]).any(axis=1).all()
    assert np.all(np.isfinite(g[clean]))
    gv, gm, gl, _ = oracle.gradient(form, mesh.coords, mesh.conn[good], dA[good],
                                    None if mu is None else mu[good],
                                    None if lam is None else lam[good])
    go = oracle.vertex_gradient(gv, mesh.conn[good], mesh.n_vertices)
    sc = vertex_scale(gv, mesh.conn[good], mesh.n_vertices)
    ok = np.intersect1d(clean, np.nonzero(sc > 0)[0])
    assert (np.abs(g[ok] - go[ok]).max(axis=1) / sc[ok]).max() <= TOL_VERTEX
    if dmu is not None:
        dmu_h, dlam_h = dmu.cpu().numpy(), dlam.cpu().numpy()
        assert np.isnan(dmu_h[touched]).all() and np.isnan(dlam_h[touched]).all()
        assert _coeff_errors(mesh.coords, mesh.conn[good], dA[good], dmu_h[good], dlam_h[good],
                             gm, gl).max() <= TOL_COEFF


# ---------------------------------------------------------------------------
# full-size adjoints as bench.py launches them, sampled
# ---------------------------------------------------------------------------

def _sampled_vertex_check(mesh, form, g, dA, mu, lam, nverts, seed):
    """Vertex gradients g [N_v, dim] at sampled vertices against the oracle over
    every element incident to them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    verts = np.union1d(rng.choice(mesh.n_vertices, nverts, replace=False),
                       [0, mesh.n_vertices - 1])
    inc = np.nonzero(np.isin(mesh.conn, verts).any(axis=1))[0]
    gv, _, _, _ = oracle.gradient(form, mesh.coords, mesh.conn[inc], dA[inc],
                                  None if mu is None else mu[inc],
                                  None if lam is None else lam[inc])
    go = oracle.vertex_gradient(gv, mesh.conn[inc], mesh.n_vertices)[verts]
    sc = vertex_scale(gv, mesh.conn[inc], mesh.n_vertices)[verts]
    ok = sc > 0
    err = (np.abs(g[verts] - go).max(axis=1)[ok] / sc[ok]).max()
    print(f"  sampled {len(verts)} vertices ({len(inc)} elements): max err {err:.3e}")
    assert err <= TOL_VERTEX
    assert np.all(g[verts][~ok] == 0)


@pytest.mark.parametrize("plan", [False, True])
def test_full_laplace3d_adjoint_sampled(plan):
    """3D P1 Laplacian adjoint on the full 64^3 cube: the single call (atomic
    scatter) and the one-mesh plan in vertex-gather form (bench.py's legs)."""
    w = meshgen.lap3d(64)
    m = w.mesh
    print(f"[full laplace adjoint] plan={plan}", flush=True)
    coords, conn = mesh_to_device(m)
    dA_h = meshgen.upstream(m.n_elements, 4, 1104)
    dA = vec_to_device(dA_h)
    dc = torch.zeros((3, m.n_vertices), dtype=torch.float32, device="cuda")
    if plan:
        b = fei.Batch([{"form": "laplace_p1", "coords": coords, "conn": conn, "dA": dA,
                        "dcoords": dc}])
        b.set_config({"mode": 3, "variant": 1, "gather": 1}, adjoint=True)
        b.run_adjoint()
        torch.cuda.synchronize()
        # the plan's incidence is the CSR of conn: ptr = cumsum of vertex degrees
        ptr, inc = b.incidence(0)
        deg = np.bincount(m.conn.ravel(), minlength=m.n_vertices)
        assert np.array_equal(ptr.cpu().numpy(), np.concatenate([[0], np.cumsum(deg)]))
        ih = inc.cpu().numpy()
        assert np.array_equal(np.sort(ih), np.arange(m.conn.size))
        owner = m.conn.ravel()[ih]
        assert np.array_equal(owner, np.repeat(np.arange(m.n_vertices), deg))
        assert np.all(np.diff(ih)[np.diff(owner) == 0] > 0)       # sorted per vertex
        b.close()
    else:
        fei.integrate_adjoint(coords, conn, "laplace_p1", dA, dcoords=dc)
    g = dc.cpu().numpy().T.astype(np.float64)
    assert np.all(np.isfinite(g))
    # invariants over the whole mesh: translation and rotation (Laplacian)
    X = m.coords.astype(np.float64)
    absg = np.abs(g).sum()
    assert np.abs(g.sum(axis=0)).max() <= 1e-5 * absg
    assert np.abs(np.cross(X, g).sum(axis=0)).max() <= 1e-5 * np.abs(X).max() * absg
    _sampled_vertex_check(m, "laplace_p1", g, dA_h, None, None, 400, 10)


def test_full_elasticity_adjoint_plan_gather_sampled():
    """The elasticity adjoint through a one-mesh plan in vertex-gather form (the
    bench's plan leg), sampled vertices and coefficient gradients."""
    w = meshgen.elast3d_adjoint(64)
    m = w.mesh
    coords, conn = mesh_to_device(m)
    mu, lam, dA = vec_to_device(w.mu), vec_to_device(w.lam), vec_to_device(w.dA)
    dc = torch.zeros((3, m.n_vertices), dtype=torch.float32, device="cuda")
    dmu = torch.full((m.n_elements,), float("nan"), device="cuda")
    dlam = torch.full((m.n_elements,), float("nan"), device="cuda")
    b = fei.Batch([{"form": w.form, "coords": coords, "conn": conn, "mu": mu, "lam": lam,
                    "dA": dA, "dcoords": dc, "dmu": dmu, "dlam": dlam}])
    b.set_config({"mode": 3, "variant": 1, "gather": 1}, adjoint=True)
    b.run_adjoint()
    torch.cuda.synchronize()
    b.close()
    g = dc.cpu().numpy().T.astype(np.float64)
    assert np.all(np.isfinite(g))
    assert not bool(torch.isnan(dmu).any() or torch.isnan(dlam).any())
    # flattened tets' vertices are sampled too (each has a private vertex)
    _sampled_vertex_check(m, w.form, g, w.dA, w.mu, w.lam, 400, 11)
    priv = np.unique(m.conn[m.flattened[:200], 3])
    inc = np.nonzero(np.isin(m.conn, priv).any(axis=1))[0]
    gv, _, _, _ = oracle.gradient(w.form, m.coords, m.conn[inc], w.dA[inc], w.mu[inc], w.lam[inc])
    go = oracle.vertex_gradient(gv, m.conn[inc], m.n_vertices)[priv]
    sc = vertex_scale(gv, m.conn[inc], m.n_vertices)[priv]
    assert (np.abs(g[priv] - go).max(axis=1) / sc).max() <= TOL_VERTEX
    rng = np.random.Generator(np.random.PCG64(12))
    idx = np.union1d(rng.choice(m.n_elements, 3000, replace=False), m.flattened[:500])
    _, gm, gl, _ = oracle.gradient(w.form, m.coords, m.conn[idx], w.dA[idx], w.mu[idx],
                                   w.lam[idx])
    merr = _coeff_errors(m.coords, m.conn[idx], w.dA[idx], dmu.cpu().numpy()[idx],
                         dlam.cpu().numpy()[idx], gm, gl)
    assert merr.max() <= TOL_COEFF


# ---------------------------------------------------------------------------
# deterministic single-call adjoint (incidence + J-bar + vertex gather)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["lap3d", "elast3d", "elast2d", "p2_3d"])
def test_deterministic_adjoint_matches_oracle_and_repeats(case):
    mesh, form, mu, lam = _case(case)
    n = fei.local_size(form, mesh.dim)
    dA = meshgen.upstream(mesh.n_elements, n, 94)
    coords, conn = mesh_to_device(mesh)
    runs = []
    for _ in range(3):
        dc, dmu, dlam = fei.integrate_adjoint(coords, conn, form, vec_to_device(dA),
                                              vec_to_device(mu), vec_to_device(lam),
                                              deterministic=True,
                                              **_nan_coeff_buffers(mesh, form))
        torch.cuda.synchronize()
        runs.append((dc.cpu().numpy(), None if dmu is None else dmu.cpu().numpy(),
                     None if dlam is None else dlam.cpu().numpy()))
    for r in runs[1:]:
        assert np.array_equal(r[0].view(np.uint32), runs[0][0].view(np.uint32))
        if r[1] is not None:
            assert np.array_equal(r[1], runs[0][1]) and np.array_equal(r[2], runs[0][2])
    g = runs[0][0].T.astype(np.float64)
    gv, gm, gl, _ = oracle.gradient(form, mesh.coords, mesh.conn, dA, mu, lam)
    go = oracle.vertex_gradient(gv, mesh.conn, mesh.n_vertices)
    sc = vertex_scale(gv, mesh.conn, mesh.n_vertices)
    used = sc > 0
    assert np.all(g[~used] == 0)
    assert (np.abs(g - go).max(axis=1)[used] / sc[used]).max() <= TOL_VERTEX
    if gm is not None:
        assert _coeff_errors(mesh.coords, mesh.conn, dA, runs[0][1], runs[0][2], gm,
                             gl).max() <= TOL_COEFF


@pytest.mark.parametrize("nfan", [63, 64, 65, 200])
def test_deterministic_adjoint_high_degree_vertex(nfan):
    """Incidence lists up to 64 entries are ranked by a wave, longer ones
    heap-sorted: a vertex of degree 63 to 200 against the oracle, repeated."""
    m = meshgen.fan_mesh(nfan, 97 + nfan)
    dA = meshgen.upstream(m.n_elements, 3, 98)
    coords, conn = mesh_to_device(m)
    runs = [fei.integrate_adjoint(coords, conn, "laplace_p1", vec_to_device(dA),
                                  deterministic=True)[0].cpu().numpy() for _ in range(2)]
    assert np.array_equal(runs[0].view(np.uint32), runs[1].view(np.uint32))
    gv, _, _, _ = oracle.gradient("laplace_p1", m.coords, m.conn, dA)
    go = oracle.vertex_gradient(gv, m.conn, m.n_vertices)
    sc = vertex_scale(gv, m.conn, m.n_vertices)
    g = runs[0].T.astype(np.float64)
    assert (np.abs(g - go).max(axis=1) / sc).max() <= TOL_VERTEX


def test_deterministic_adjoint_accumulates_and_rejects():
    mesh, form, mu, lam = _case("lap3d")
    coords, conn = mesh_to_device(mesh)
    dA = vec_to_device(meshgen.upstream(mesh.n_elements, 4, 95))
    d1, _, _ = fei.integrate_adjoint(coords, conn, form, dA, deterministic=True)
    base = torch.full_like(d1, 0.25)
    d2, _, _ = fei.integrate_adjoint(coords, conn, form, dA, dcoords=base, deterministic=True)
    # one FP32 rounding of 0.25 + d1 per entry
    torch.testing.assert_close(d2 - 0.25, d1, rtol=0, atol=1e-7 + 1e-6 * float(d1.abs().max()))
    with pytest.raises(fei.FeiError) as ex:      # FP64 coordinates: no gather kernel
        fei.integrate_adjoint(coords.double(), conn, form, dA, deterministic=True)
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED
    with pytest.raises(fei.FeiError):
        fei.integrate_adjoint(coords, conn, form, dA, deterministic=True, store_rows=2)
    e0, _, _ = fei.integrate_adjoint(coords, conn[:0], form, dA[:0], deterministic=True)
    assert float(e0.abs().max()) == 0.0


def test_autograd_is_deterministic_when_asked():
    mesh, form, mu, lam = _case("elast3d")
    coords, conn = mesh_to_device(mesh)
    dA = vec_to_device(meshgen.upstream(mesh.n_elements, 12, 96))
    grads = []
    torch.use_deterministic_algorithms(True)
    try:
        for _ in range(2):
            c = coords.clone().requires_grad_(True)
            A = fei.element_matrices(c, conn, form, vec_to_device(mu), vec_to_device(lam))
            (A * dA).sum().backward()
            grads.append(c.grad.cpu().numpy())
    finally:
        torch.use_deterministic_algorithms(False)
    assert np.array_equal(grads[0].view(np.uint32), grads[1].view(np.uint32))
    ref, _, _ = fei.integrate_adjoint(coords, conn, form, dA, vec_to_device(mu),
                                      vec_to_device(lam), deterministic=True)
    assert np.array_equal(grads[0].view(np.uint32), ref.cpu().numpy().view(np.uint32))
