"""The isoparametric P2 Laplacian on curved elements (fei_integrate_iso)
against the oracle's quadrature of the paper's projected scheme, element by
element at the FP32 bound: 2D and 3D, ragged sizes, near-degenerate elements
(FP64 path and its counter), straight edges against the affine P2 kernel, and
the full-size curved cube sampled."""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import TOL, element_errors

pytestmark = pytest.mark.gpu

fei = pytest.importorskip("paper_1103_0066_amd")


def _dev(m):
    return (torch.from_numpy(m.soa()).cuda(),
            torch.from_numpy(np.ascontiguousarray(m.conn)).cuda())


def _curved(dim, amp, seed, flat=0):
    base = (meshgen.square_mesh(11, 0.2, seed, np.float32) if dim == 2
            else meshgen.cube_mesh(6, 5, 5, 0.15, seed))
    if flat:
        base = meshgen.flatten_elements(base, flat, seed + 1)
    return meshgen.p2_mesh(base, amp), base


@pytest.mark.parametrize("dim", [2, 3])
def test_iso_matches_oracle(dim):
    m, _ = _curved(dim, 0.05, 500 + dim)
    print(f"[iso] dim={dim} E={m.n_elements} nodes={m.n_vertices}", flush=True)
    coords, conn = _dev(m)
    A = fei.integrate_iso(coords, conn).cpu().numpy()
    Ao = oracle.integrate_iso(m.coords, m.conn)
    err = element_errors(A, Ao)
    print(f"  max element error {err.max():.2e}")
    assert err.max() <= TOL["fp32"]


def test_iso_ragged_sizes_flagged_elements_and_counters():
    # barely curved edges: a curvature comparable to the flattened tets'
    # thickness (1e-3 of their edges) would invert them
    m, base = _curved(3, 1e-4, 510, flat=25)
    coords, conn = _dev(m)
    Ao = oracle.integrate_iso(m.coords, m.conn)
    for E in (0, 1, 63, 65, 257, 300, m.n_elements):
        cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
        out = torch.full((E, 10, 10), float("nan"), device="cuda")
        A = fei.integrate_iso(coords, conn[:E].contiguous(), counters=cnt, out=out).cpu().numpy()
        if E == 0:
            continue
        assert element_errors(A, Ao[:E]).max() <= TOL["fp32"], E
        assert cnt.cpu().tolist() == [int(np.sum(base.flattened < E)), 0], E


@pytest.mark.parametrize("dim", [2, 3])
def test_iso_straight_edges_equal_the_affine_p2_kernel(dim):
    m, base = _curved(dim, 0.0, 520 + dim)
    coords, conn = _dev(m)
    A = fei.integrate_iso(coords, conn).cpu().numpy().astype(np.float64)
    bc, bk = _dev(base)
    Ap = fei.integrate(bc, bk, "laplace_p2").cpu().numpy()
    assert element_errors(A, Ap).max() <= TOL["fp32"]


def test_iso_full_curved_cube_sampled():
    """bench.py's isoparametric workload: the curved 64^3 cube, sampled."""
    w = meshgen.iso3d(64)
    m = w.mesh
    print(f"[iso full] {w.name}", flush=True)
    coords, conn = _dev(m)
    A = fei.integrate_iso(coords, conn)
    rng = np.random.Generator(np.random.PCG64(530))
    idx = np.union1d(rng.choice(m.n_elements, 20000, replace=False), [0, m.n_elements - 1])
    As = A[torch.from_numpy(idx).cuda()].cpu().numpy()
    Ao = oracle.integrate_iso(m.coords, m.conn[idx])
    err = element_errors(As, Ao)
    print(f"  sampled max element error {err.max():.2e}")
    assert err.max() <= TOL["fp32"]
