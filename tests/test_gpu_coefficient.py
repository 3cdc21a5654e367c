"""The Laplacian with a P1 coefficient (Sec. 3.1, eqs. 20-23): the HIP path
against the oracle's quadrature with w interpolated at the points."""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import TOL, element_errors, mesh_to_device

pytestmark = pytest.mark.gpu

fei = pytest.importorskip("paper_1103_0066_amd")


def _case(name):
    if name == "p1_2d_f64":
        return meshgen.square_mesh(23, 0.2, 111, np.float64), "laplace_p1"
    if name == "p1_3d":
        return meshgen.flatten_elements(meshgen.cube_mesh(6, 5, 5, 0.15, 112), 9, 113), "laplace_p1"
    if name == "p2_2d":
        return meshgen.square_mesh(19, 0.2, 114, np.float32), "laplace_p2"
    if name == "p2_3d":
        return meshgen.flatten_elements(meshgen.cube_mesh(5, 5, 5, 0.15, 115), 7, 116), "laplace_p2"
    raise KeyError(name)


def _run(mesh, form, w, **kw):
    coords, conn = mesh_to_device(mesh)
    n = fei.local_size(form, mesh.dim)
    out = torch.full((mesh.n_elements, n, n), float("nan"), device=coords.device)
    fei.integrate_coefficient(coords, conn, form, torch.from_numpy(w).cuda(), out=out, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("rows", [0, -1, 2])
@pytest.mark.parametrize("case", ["p1_2d_f64", "p1_3d", "p2_2d", "p2_3d"])
def test_coefficient_forward_matches_oracle(case, rows):
    mesh, form = _case(case)
    if rows == 2 and fei.local_size(form, mesh.dim) == 3:
        pytest.skip("3 x 3 matrices are staged whole or stored directly")
    w = meshgen.lame(mesh.n_vertices, 117)[0]          # lognormal, one value per vertex
    print(f"[coefficient] {case} rows={rows} E={mesh.n_elements}", flush=True)
    A = _run(mesh, form, w, store_rows=rows)
    Ao = oracle.integrate_coefficient(form, mesh.coords, mesh.conn, w)
    err = element_errors(A, Ao)
    print(f"  max err {err.max():.3e}")
    assert np.all(np.isfinite(A))
    assert err.max() <= TOL["fp32"]


def test_coefficient_ragged_tiles_and_counters():
    mesh, form = _case("p2_3d")
    w = meshgen.lame(mesh.n_vertices, 118)[1]
    for E in (1, 63, 255, 257, 3 * 256 + 7):
        sub = meshgen.Mesh(mesh.coords, np.ascontiguousarray(mesh.conn[:E]))
        A = _run(sub, form, w)
        Ao = oracle.integrate_coefficient(form, mesh.coords, sub.conn, w)
        assert element_errors(A, Ao).max() <= TOL["fp32"], E
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    _run(mesh, form, w, counters=cnt)
    assert cnt.cpu().tolist() == [len(mesh.flattened), 0]


def test_coefficient_one_equals_constant_form():
    """w = 1 gives the constant-coefficient matrices (the same integral)."""
    mesh, form = _case("p2_3d")
    A1 = _run(mesh, form, np.ones(mesh.n_vertices, np.float32))
    coords, conn = mesh_to_device(mesh)
    A = fei.integrate(coords, conn, form).cpu().numpy()
    assert element_errors(A1, A.astype(np.float64)).max() <= 2 * TOL["fp32"]


def test_coefficient_rejections():
    mesh, form = _case("p1_3d")
    coords, conn = mesh_to_device(mesh)
    w = torch.ones(mesh.n_vertices, device="cuda")
    with pytest.raises(fei.FeiError) as ex:
        fei.integrate_coefficient(coords, conn, "elastic_p1", w)
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED
    with pytest.raises(fei.FeiError):
        fei.integrate_coefficient(coords, conn, form, w, store_rows=3)


def test_full_coefficient_p2_sampled():
    """3D P2 Laplacian with a lognormal P1 coefficient on the full 64^3 cube
    (bench.py's coefficient leg), sampled."""
    wl = meshgen.lap3d(64)
    m = wl.mesh
    w = meshgen.lame(m.n_vertices, 119)[0]
    coords, conn = mesh_to_device(m)
    A = torch.full((m.n_elements, 10, 10), float("nan"), device="cuda")
    fei.integrate_coefficient(coords, conn, "laplace_p2", torch.from_numpy(w).cuda(), out=A)
    assert not bool(torch.isnan(A).any())
    rng = np.random.Generator(np.random.PCG64(120))
    idx = np.union1d(rng.choice(m.n_elements, 20000, replace=False), [0, m.n_elements - 1])
    As = A[torch.from_numpy(idx).cuda()].cpu().numpy()
    Ao = oracle.integrate_coefficient("laplace_p2", m.coords, m.conn[idx], w)
    err = element_errors(As, Ao)
    print(f"  sampled {len(idx)}: max err {err.max():.3e}")
    assert err.max() <= TOL["fp32"]
    rowsum = A.sum(dim=2).abs().amax(dim=1) / A.abs().amax(dim=(1, 2))
    assert float(rowsum.max()) <= 20 * TOL["fp32"]
