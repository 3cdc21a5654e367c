"""Fused global assembly: the HIP path against the oracle's COO -> CSR sum of
its FP64 element matrices -- the same sparsity pattern exactly, every value
within the FP32 bound relative to the sum of magnitudes it is made of."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import meshgen
import oracle
from gpu_util import mesh_to_device, vec_to_device

pytestmark = pytest.mark.gpu

fei = pytest.importorskip("paper_1103_0066_amd")

TOL_ASM = 1e-5


def _case(name):
    if name == "lap2d":
        return meshgen.square_mesh(21, 0.2, 101, np.float32), "laplace_p1", None, None
    if name == "lap3d":
        return meshgen.cube_mesh(7, 6, 5, 0.15, 102), "laplace_p1", None, None
    if name == "elast2d":
        m = meshgen.square_mesh(19, 0.2, 103, np.float32)
        mu, lam = meshgen.lame(m.n_elements, 104)
        return m, "elastic_p1", mu, lam
    if name == "elast3d":
        m = meshgen.flatten_elements(meshgen.cube_mesh(7, 6, 6, 0.15, 105), 15, 106)
        mu, lam = meshgen.lame(m.n_elements, 107)
        return m, "elastic_p1", mu, lam
    raise KeyError(name)


def _to_csr(asm, rowptr, colidx, values):
    nc = asm.block
    B = sp.bsr_matrix((values.reshape(-1, nc, nc), colidx, rowptr),
                      shape=(nc * asm.n_rows, nc * asm.n_rows))
    K = B.tocsr()
    K.sort_indices()
    return K


def _scale(form, coords, conn, mu, lam, nrows_scalar):
    """Per stored entry: the sum, over the elements whose matrices add into it, of
    that element matrix's norm max_ij |A_e,ij| -- the normwise FP32 bound of each
    element matrix summed over the entry's terms (never zero for a stored entry;
    an entry's own terms may cancel, or vanish exactly on a right-angled element)."""
    A = oracle.integrate(form, coords, conn, mu, lam)
    E = len(conn)
    nrm = np.abs(A).reshape(E, -1).max(axis=1)
    nc = coords.shape[1] if form == "elastic_p1" else 1
    conn = conn.astype(np.int64)
    dofs = (nc * conn[:, :, None] + np.arange(nc)).reshape(E, -1)
    n = dofs.shape[1]
    r = np.broadcast_to(dofs[:, :, None], (E, n, n)).ravel()
    c = np.broadcast_to(dofs[:, None, :], (E, n, n)).ravel()
    v = np.broadcast_to(nrm[:, None, None], (E, n, n)).ravel()
    S = sp.coo_matrix((v, (r, c)), shape=(nrows_scalar,) * 2).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return S


def _gpu_assemble(mesh, form, mu, lam, **kw):
    coords, conn = mesh_to_device(mesh)
    asm = fei.Assembly(coords, conn, form)
    vals = asm.assemble(vec_to_device(mu), vec_to_device(lam), **kw)
    rowptr, colidx = asm.pattern()
    torch.cuda.synchronize()
    return asm, rowptr.cpu().numpy(), colidx.cpu().numpy(), vals.cpu().numpy()


@pytest.mark.parametrize("case", ["lap2d", "lap3d", "elast2d", "elast3d"])
def test_assembly_matches_oracle(case):
    mesh, form, mu, lam = _case(case)
    print(f"[assembly] {case} E={mesh.n_elements} Nv={mesh.n_vertices}", flush=True)
    asm, rowptr, colidx, vals = _gpu_assemble(mesh, form, mu, lam)
    K = _to_csr(asm, rowptr, colidx, vals)
    Ko = oracle.assemble(form, mesh.coords, mesh.conn, mu, lam)
    assert np.array_equal(K.indptr, Ko.indptr) and np.array_equal(K.indices, Ko.indices)
    S = _scale(form, mesh.coords, mesh.conn, mu, lam, Ko.shape[0])
    assert np.array_equal(S.indices, Ko.indices)
    err = np.abs(K.data - Ko.data) / S.data
    print(f"  max err {err.max():.3e}")
    assert np.all(np.isfinite(K.data))
    assert err.max() <= TOL_ASM
    asm.close()


def test_assembly_repeats_and_takes_new_coordinates():
    mesh, form, mu, lam = _case("elast3d")
    coords, conn = mesh_to_device(mesh)
    asm = fei.Assembly(coords, conn, form)
    mu_d, lam_d = vec_to_device(mu), vec_to_device(lam)
    v1 = asm.assemble(mu_d, lam_d).cpu().numpy()
    v2 = asm.assemble(mu_d, lam_d).cpu().numpy()
    assert np.array_equal(v1.view(np.uint32), v2.view(np.uint32))
    # a moved mesh, same connectivity
    rng = np.random.Generator(np.random.PCG64(108))
    X2 = (mesh.coords.astype(np.float64) * 1.3 + rng.uniform(-0.01, 0.01, mesh.coords.shape))
    X2 = X2.astype(np.float32)
    c2 = torch.from_numpy(np.ascontiguousarray(X2.T)).cuda()
    v3 = asm.assemble(mu_d, lam_d, coords=c2).cpu().numpy()
    rowptr, colidx = asm.pattern()
    K = _to_csr(asm, rowptr.cpu().numpy(), colidx.cpu().numpy(), v3)
    Ko = oracle.assemble(form, X2, mesh.conn, mu, lam)
    S = _scale(form, X2, mesh.conn, mu, lam, Ko.shape[0])
    assert (np.abs(K.data - Ko.data) / S.data).max() <= TOL_ASM
    asm.close()


def test_assembly_counts_fp64_elements_once():
    mesh, form, mu, lam = _case("elast3d")
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    _gpu_assemble(mesh, form, mu, lam, counters=cnt)
    assert cnt.cpu().tolist() == [len(mesh.flattened), 0]
    cnt.zero_()
    _gpu_assemble(mesh, form, mu, lam, counters=cnt, tau=0.0)
    assert cnt.cpu().tolist() == [mesh.n_elements, 0]


@pytest.mark.parametrize("nfan", [60, 200])
def test_assembly_high_degree_vertex(nfan):
    """A row of nfan + 1 blocks whose nfan incidences the four row owners share
    unevenly, against the oracle, repeated bit for bit; a vertex with more
    neighbours than a wave's accumulator holds is refused at plan creation."""
    m = meshgen.fan_mesh(nfan, 111 + nfan)
    asm, rowptr, colidx, vals = _gpu_assemble(m, "laplace_p1", None, None)
    assert rowptr[1] - rowptr[0] == nfan + 1
    K = _to_csr(asm, rowptr, colidx, vals)
    Ko = oracle.assemble("laplace_p1", m.coords, m.conn)
    assert np.array_equal(K.indptr, Ko.indptr) and np.array_equal(K.indices, Ko.indices)
    S = _scale("laplace_p1", m.coords, m.conn, None, None, Ko.shape[0])
    assert (np.abs(K.data - Ko.data) / S.data).max() <= TOL_ASM
    _, _, _, vals2 = _gpu_assemble(m, "laplace_p1", None, None)
    assert np.array_equal(vals.view(np.uint32), vals2.view(np.uint32))


@pytest.mark.parametrize("case", ["lap2d", "elast3d", "fan", "kuhn"])
def test_assembly_schedule_is_conflict_free(case):
    """The plan's schedule, which the kernel's unserialized adds rely on: each
    row lists every incidence of its vertex exactly once, in steps of four
    (-1 padding) whose elements share no vertex but the row's; on the Kuhn
    cube the search reaches ceil(n / 4) steps for nearly every interior row."""
    if case == "fan":
        m, form = meshgen.fan_mesh(200, 113), "laplace_p1"
    elif case == "kuhn":
        m, form = meshgen.elast3d(12).mesh, "elastic_p1"
    else:
        m, form = _case(case)[:2]
    coords, conn = mesh_to_device(m)
    asm = fei.Assembly(coords, conn, form)
    ptr, inc = (t.cpu().numpy() for t in asm.schedule())
    nv = m.conn.shape[1]
    want = [[] for _ in range(m.n_vertices)]
    for e, row in enumerate(m.conn):
        for a, v in enumerate(row):
            want[v].append(e * nv + a)
    assert ptr[0] == 0 and np.all(np.diff(ptr) % 4 == 0) and ptr[-1] == len(inc)
    tight = rows24 = 0
    for v in range(m.n_vertices):
        ent = inc[ptr[v]:ptr[v + 1]]
        assert sorted(ent[ent >= 0].tolist()) == sorted(want[v])
        for st in ent.reshape(-1, 4):
            seen = set()
            for x in st[st >= 0]:
                e, a = divmod(int(x), nv)
                assert m.conn[e, a] == v
                others = set(m.conn[e].tolist()) - {v}
                assert not (others & seen)
                seen |= others
        if len(want[v]) == 24:
            rows24 += 1
            tight += len(ent) == 24
    if case == "kuhn":
        assert rows24 > 0 and tight >= 0.99 * rows24


def test_assembly_refuses_a_row_beyond_the_accumulator():
    m = meshgen.fan_mesh(300, 112)
    coords, conn = mesh_to_device(m)
    with pytest.raises(fei.FeiError) as ex:
        fei.Assembly(coords, conn, "laplace_p1")
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED


def test_assembly_unused_vertices_and_rejections():
    """A vertex no element uses has an empty row; P2 forms and bad connectivity
    are refused at plan creation."""
    mesh, form, mu, lam = _case("lap3d")
    X = np.vstack([mesh.coords, np.array([[5.0, 5.0, 5.0]], np.float32)])
    m2 = meshgen.Mesh(X, mesh.conn)
    asm, rowptr, colidx, vals = _gpu_assemble(m2, form, None, None)
    assert rowptr[-1] == rowptr[-2]
    K = _to_csr(asm, rowptr, colidx, vals)
    Ko = oracle.assemble(form, X, mesh.conn)
    assert np.array_equal(K.indptr, Ko.indptr)
    coords, conn = mesh_to_device(mesh)
    with pytest.raises(fei.FeiError) as ex:
        fei.Assembly(coords, conn, "laplace_p2")
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED
    bad = conn.clone()
    bad[5, 2] = mesh.n_vertices + 3
    with pytest.raises(fei.FeiError) as ex:
        fei.Assembly(coords, bad, form)
    assert ex.value.status == fei._lib.FEI_EINVAL


def test_full_elasticity_assembly_sampled():
    """The 1.57M-tet elasticity workload (bench.py's assembly leg): sampled block
    rows against the oracle, and the six rigid motions in the kernel of the
    whole assembled matrix."""
    w = meshgen.elast3d(64)
    m = w.mesh
    print(f"[full assembly] {w.name}", flush=True)
    asm, rowptr, colidx, vals = _gpu_assemble(m, w.form, w.mu, w.lam)
    assert np.all(np.isfinite(vals))
    K = _to_csr(asm, rowptr, colidx, vals)
    rng = np.random.Generator(np.random.PCG64(109))
    verts = np.union1d(rng.choice(m.n_vertices, 300, replace=False),
                       np.unique(m.conn[m.flattened[:50]].ravel()))
    inc = np.nonzero(np.isin(m.conn, verts).any(axis=1))[0]
    Ko = oracle.assemble(w.form, m.coords, m.conn[inc], w.mu[inc], w.lam[inc])
    S = _scale(w.form, m.coords, m.conn[inc], w.mu[inc], w.lam[inc], Ko.shape[0])
    rows = (3 * verts[:, None] + np.arange(3)).ravel()
    Kr, Kor, Sr = K[rows], Ko[rows], S[rows]
    Kr.sort_indices(); Kor.sort_indices(); Sr.sort_indices()
    assert np.array_equal(Kr.indptr, Kor.indptr) and np.array_equal(Kr.indices, Kor.indices)
    err = np.abs(Kr.data - Kor.data) / Sr.data
    print(f"  sampled rows {len(rows)}: max err {err.max():.3e}")
    assert err.max() <= TOL_ASM
    X = m.coords.astype(np.float64)
    R = np.zeros((3 * m.n_vertices, 6))
    for c in range(3):
        R[c::3, c] = 1.0
    for k, axis in enumerate(range(3)):
        wv = np.zeros(3); wv[axis] = 1
        R[:, 3 + k] = np.cross(wv, X).ravel()
    absK = abs(K)
    res = np.abs(K @ R) / (absK @ np.abs(R))
    print(f"  rigid-mode residual {np.nanmax(res):.3e}")
    assert np.nanmax(res) <= 1e-5
    asm.close()
