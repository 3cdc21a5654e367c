"""Seeded synthetic inputs for element integration.

This module builds meshes, Lame coefficients and upstream gradients.  It holds
none of the integration arithmetic (no Jacobians, geometric tensors, reference
tensors or quadrature): both the FP64 oracle and the GPU path consume what it
produces, and neither imports the other.

Workload recipes (the paper integrates P1 Laplacian and elasticity operators on
synthetic simplicial meshes, Sec. 5; sizes below are this project's choice):

* ``square_mesh``  -- n x n unit square, every cell cut along its (i,j)->(i+1,j+1)
  diagonal into two counter-clockwise triangles, interior vertices jittered.
* ``cube_mesh``    -- nx x ny x nz box of cubes, each cube Kuhn-split into six
  positively oriented tetrahedra, interior vertices jittered.
* ``flatten_elements`` -- replaces the fourth vertex of chosen tets by a private
  vertex placed at 1e-3 of the base face's longest edge above that face
  (aspect ratio ~1e3), which exercises the FP64 Jacobian path.
* ``lame``         -- per-element mu, lambda = exp(0.5 Z), Z ~ N(0, 1).
* ``upstream``     -- dL/dA_e ~ N(0, 1), not symmetric.
* ``workload``     -- the named workloads (2D/3D P1 Laplacian, 3D P1 elasticity,
  its adjoint, the heterogeneous batch) at full or reduced size.

All random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Optional

import numpy as np

SEED_BASE = 1103

# Kuhn permutations of (x, y, z) in lexicographic order, with their parity.
_PERMS = list(itertools.permutations(range(3)))


def _perm_is_odd(p) -> bool:
    inv = sum(1 for i in range(3) for j in range(i + 1, 3) if p[i] > p[j])
    return inv % 2 == 1


@dataclasses.dataclass
class Mesh:
    """A simplicial mesh.

    coords: float array [N_v, dim] (row per vertex).
    conn:   int32 array [E, dim+1]; vertex 0 of each element is the origin of
            its local frame.
    """

    coords: np.ndarray
    conn: np.ndarray
    flattened: Optional[np.ndarray] = None  # indices of near-degenerate elements

    @property
    def dim(self) -> int:
        return self.coords.shape[1]

    @property
    def n_vertices(self) -> int:
        return self.coords.shape[0]

    @property
    def n_elements(self) -> int:
        return self.conn.shape[0]

    def soa(self) -> np.ndarray:
        """Coordinates as a contiguous [dim, N_v] array (x row, y row, z row)."""
        return np.ascontiguousarray(self.coords.T)


def _interior_mask(idx, n):
    return (idx > 0) & (idx < n)


def _assert_positive(coords: np.ndarray, conn: np.ndarray):
    """Input validity: every simplex is positively oriented (signed volume of its
    edge vectors from vertex 0, in FP64 of the stored coordinates, is > 0)."""
    X = coords.astype(np.float64)
    e = [X[conn[:, k]] - X[conn[:, 0]] for k in range(1, conn.shape[1])]
    if len(e) == 2:
        vol = e[0][:, 0] * e[1][:, 1] - e[0][:, 1] * e[1][:, 0]
    else:
        vol = np.einsum("ij,ij->i", e[0], np.cross(e[1], e[2]))
    if vol.size and not (vol > 0).all():
        raise AssertionError(f"{int((vol <= 0).sum())} simplices are not positively oriented")


def square_mesh(n: int, jitter: float = 0.2, seed: Optional[int] = None,
                dtype=np.float64) -> Mesh:
    """Unit square, n x n cells of size h = 1/n, 2 n^2 triangles.

    Vertex (i, j) has index i + (n+1) j.  Cell (i, j) (x fastest) yields
    [v00, v10, v11] then [v00, v11, v01], both counter-clockwise.  Interior
    vertices move by independent U(-jitter*h, jitter*h) per coordinate.
    """
    h = 1.0 / n
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    i = i.ravel(); j = j.ravel()
    coords = np.stack([i * h, j * h], axis=1).astype(np.float64)
    if seed is not None and jitter > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        d = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        inner = _interior_mask(i, n) & _interior_mask(j, n)
        coords[inner] += d[inner]
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel(); cj = cj.ravel()
    v = lambda a, b: (ci + a) + (n + 1) * (cj + b)
    t0 = np.stack([v(0, 0), v(1, 0), v(1, 1)], axis=1)
    t1 = np.stack([v(0, 0), v(1, 1), v(0, 1)], axis=1)
    conn = np.stack([t0, t1], axis=1).reshape(-1, 3).astype(np.int32)
    coords = coords.astype(dtype)
    _assert_positive(coords, conn)
    return Mesh(coords, conn)


def cube_mesh(nx: int, ny: int, nz: int, jitter: float = 0.15,
              seed: Optional[int] = None, dtype=np.float32,
              h: Optional[float] = None) -> Mesh:
    """Box of nx*ny*nz cubes of side h (default 1/nx), 6 Kuhn tets per cube.

    Vertex (i, j, k) has index i + (nx+1)(j + (ny+1) k).  Cells are ordered x
    fastest; cell c holds tets 6c..6c+5, one per permutation p of the axes in
    lexicographic order, with vertices v000, v000+e_p0, v000+e_p0+e_p1, v111.
    For odd p the last two vertices are swapped so that every tet is positively
    oriented.  Interior vertices move by independent U(-jitter*h, jitter*h)
    per coordinate (drawn in FP64, then rounded to ``dtype``).
    """
    if h is None:
        h = 1.0 / nx
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1),
                             np.arange(nz + 1), indexing="ij")
    # x fastest: order by (k, j, i)
    ii = ii.transpose(2, 1, 0).ravel(); jj = jj.transpose(2, 1, 0).ravel()
    kk = kk.transpose(2, 1, 0).ravel()
    coords = np.stack([ii * h, jj * h, kk * h], axis=1).astype(np.float64)
    if seed is not None and jitter > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        d = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        inner = (_interior_mask(ii, nx) & _interior_mask(jj, ny)
                 & _interior_mask(kk, nz))
        coords[inner] += d[inner]
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel(); cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()

    def vid(off):
        return ((ci + off[0]) + (nx + 1) * ((cj + off[1]) + (ny + 1) * (ck + off[2])))

    tets = []
    for p in _PERMS:
        o0 = np.zeros(3, int)
        o1 = o0.copy(); o1[p[0]] = 1
        o2 = o1.copy(); o2[p[1]] = 1
        o3 = np.ones(3, int)
        vs = [vid(o0), vid(o1), vid(o2), vid(o3)]
        if _perm_is_odd(p):
            vs = [vs[0], vs[1], vs[3], vs[2]]
        tets.append(np.stack(vs, axis=1))
    conn = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    coords = coords.astype(dtype)
    _assert_positive(coords, conn)
    return Mesh(coords, conn)


def fan_mesh(nfan: int, seed: int) -> Mesh:
    """A 2D fan: vertex 0 shared by nfan triangles around it (degree nfan, nfan
    neighbours), beside a small jittered square mesh of ordinary degrees; the
    elements in a random order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = np.sort(rng.uniform(0, 2 * np.pi, nfan))
    ring = np.stack([np.cos(ang), np.sin(ang)], axis=1) * rng.uniform(0.8, 1.2, (nfan, 1))
    sq = square_mesh(9, 0.2, seed + 1, np.float32)
    coords = np.concatenate([[[0.0, 0.0]], ring, sq.coords + 3.0]).astype(np.float32)
    k = np.arange(nfan)
    fan = np.stack([np.zeros(nfan, np.int64), 1 + k, 1 + (k + 1) % nfan], 1)
    conn = np.concatenate([fan, sq.conn + 1 + nfan]).astype(np.int32)
    conn = np.ascontiguousarray(conn[rng.permutation(len(conn))])
    _assert_positive(coords, conn)
    return Mesh(coords, conn)


def flatten_elements(mesh: Mesh, count: int, seed: int, ratio: float = 1e-3) -> Mesh:
    """Make ``count`` tets (chosen without replacement) near-degenerate.

    For each chosen tet (v0, v1, v2, v3) a private vertex is appended at
    P(v3) + ratio * l_max * n, where P(v3) is the orthogonal projection of v3 on
    the plane of (v0, v1, v2), n the unit normal of that plane on v3's side and
    l_max the longest edge of the face; conn[e][3] is rewritten to it.  The
    construction runs in FP64 and the new vertices are rounded to the mesh
    dtype.  Orientation is preserved because the new vertex stays on v3's side.
    """
    assert mesh.dim == 3
    rng = np.random.Generator(np.random.PCG64(seed))
    E = mesh.n_elements
    sel = np.sort(rng.choice(E, size=count, replace=False)) if count > 0 else np.zeros(0, np.int64)
    X = mesh.coords.astype(np.float64)
    c = mesh.conn[sel]
    p0, p1, p2, p3 = (X[c[:, k]] for k in range(4))
    nrm = np.cross(p1 - p0, p2 - p0)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    side = np.sign(np.einsum("ij,ij->i", p3 - p0, nrm))
    nrm *= side[:, None]
    proj = p3 - np.einsum("ij,ij->i", p3 - p0, nrm)[:, None] * nrm
    lmax = np.maximum.reduce([np.linalg.norm(p1 - p0, axis=1),
                              np.linalg.norm(p2 - p0, axis=1),
                              np.linalg.norm(p2 - p1, axis=1)])
    newv = proj + (ratio * lmax)[:, None] * nrm
    coords = np.concatenate([mesh.coords, newv.astype(mesh.coords.dtype)], axis=0)
    conn = mesh.conn.copy()
    conn[sel, 3] = (mesh.n_vertices + np.arange(count)).astype(np.int32)
    _assert_positive(coords, conn)
    return Mesh(coords, conn, flattened=sel)


def lame(E: int, seed: int, sigma: float = 0.5):
    """Per-element Lame coefficients mu = exp(sigma Z1), lambda = exp(sigma Z2), FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal(size=(2, E))
    return (np.exp(sigma * z[0]).astype(np.float32),
            np.exp(sigma * z[1]).astype(np.float32))


def upstream(E: int, n: int, seed: int) -> np.ndarray:
    """dL/dA_e, iid N(0, 1) FP32, shape [E, n, n] (not symmetric)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=(E, n, n), dtype=np.float32)


def p2_mesh(mesh: Mesh, amp: float = 0.0, wavelength: float = 1.0) -> Mesh:
    """Quadratic (P2) geometry on a simplicial mesh: every edge gets one node,
    shared by the elements around it, at its midpoint moved by the smooth field
    amp * l * f(x), f = (sin(2 pi y/L) sin(2 pi z/L), sin(2 pi z/L) sin(2 pi x/L),
    sin(2 pi x/L) sin(2 pi y/L)) in 3D and (sin(2 pi y/L), sin(2 pi x/L)) in 2D,
    l the edge's length (amp = 0: straight edges, the affine element).
    The returned conn is [E, nb]: the element's vertices, then its edge nodes in
    the P2 order (0,1), (0,2), .., (d-1,d); coordinates are FP64 before
    rounding to the mesh dtype.  Asserts det J > 0 at the vertices, the
    barycenter and the edge midpoints of every element."""
    dim = mesh.dim
    nv = dim + 1
    pairs = [(a, b) for a in range(nv) for b in range(a + 1, nv)]
    c = mesh.conn.astype(np.int64)
    E = c.shape[0]
    ev = np.stack([np.sort(np.stack([c[:, a], c[:, b]], axis=1), axis=1) for a, b in pairs], axis=1)
    key = ev[..., 0] * mesh.n_vertices + ev[..., 1]
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    X = mesh.coords.astype(np.float64)
    a, b = uniq // mesh.n_vertices, uniq % mesh.n_vertices
    mid = 0.5 * (X[a] + X[b])
    h = np.linalg.norm(X[a] - X[b], axis=1)[:, None]
    w = 2.0 * np.pi / wavelength
    if dim == 3:
        f = np.stack([np.sin(w * mid[:, 1]) * np.sin(w * mid[:, 2]),
                      np.sin(w * mid[:, 2]) * np.sin(w * mid[:, 0]),
                      np.sin(w * mid[:, 0]) * np.sin(w * mid[:, 1])], axis=1)
    else:
        f = np.stack([np.sin(w * mid[:, 1]), np.sin(w * mid[:, 0])], axis=1)
    nodes = mid + amp * h * f
    coords = np.concatenate([X, nodes]).astype(mesh.coords.dtype)
    conn = np.concatenate([c, mesh.n_vertices + inv.reshape(E, len(pairs))], axis=1).astype(np.int32)
    _assert_positive_p2(coords, conn)
    return Mesh(coords, conn)


def _assert_positive_p2(coords: np.ndarray, conn: np.ndarray):
    """det J(xi) > 0 for the quadratic map at the vertices, the barycenter and
    the edge midpoints of every element (FP64)."""
    dim = coords.shape[1]
    nv = dim + 1
    X = coords.astype(np.float64)[conn]                     # [E, nb, dim]
    gl = np.vstack([-np.ones(dim), np.eye(dim)])            # reference grad lambda_a
    pairs = [(a, b) for a in range(nv) for b in range(a + 1, nv)]
    pts = [np.eye(nv)[k] for k in range(nv)] + [np.full(nv, 1.0 / nv)]
    pts += [0.5 * (np.eye(nv)[a] + np.eye(nv)[b]) for a, b in pairs]
    for bc in pts:
        g = [(4 * bc[k] - 1) * gl[k] for k in range(nv)]
        g += [4 * (bc[a] * gl[b] + bc[b] * gl[a]) for a, b in pairs]
        J = np.einsum("enx,nm->exm", X, np.array(g))
        det = np.linalg.det(J)
        if det.size and not (det > 0).all():
            raise AssertionError(f"{int((det <= 0).sum())} curved elements are inverted")


def iso3d(n: int = 64, amp: float = 0.05) -> "Workload":
    """Isoparametric P2 Laplacian: the lap3d mesh (jittered Kuhn cube, 6 n^3
    tets) with quadratic geometry, edge nodes moved by up to amp times the
    edge length (curved edges)."""
    m = p2_mesh(_cube(n), amp)
    return Workload(f"3D isoparametric P2 Laplacian, {n}^3 Kuhn cube, {m.n_elements} curved tets, "
                    f"{m.n_vertices} nodes, FP32", "laplace_iso_p2", m)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

FORMS = ("laplace_p1", "elastic_p1", "laplace_p2")


@dataclasses.dataclass
class Workload:
    name: str
    form: str
    mesh: Mesh
    mu: Optional[np.ndarray] = None
    lam: Optional[np.ndarray] = None
    dA: Optional[np.ndarray] = None

    @property
    def n_local(self) -> int:
        d = self.mesh.dim
        if self.form == "laplace_p1":
            return d + 1
        if self.form == "elastic_p1":
            return d * (d + 1)
        if self.form == "laplace_p2":
            return (d + 1) * (d + 2) // 2
        raise ValueError(self.form)


def lap2d(n: int = 64) -> Workload:
    """2D P1 Laplacian: n x n square, 2 n^2 triangles, 0.2h jitter, FP64 coords."""
    return Workload(f"2D P1 Laplacian, {n}x{n} square, {2*n*n} triangles, FP64 coords",
                    "laplace_p1", square_mesh(n, 0.2, SEED_BASE + 1, np.float64))


def _cube(n: int) -> Mesh:
    return cube_mesh(n, n, n, 0.15, SEED_BASE + 2, np.float32)


def lap3d(n: int = 64) -> Workload:
    """3D P1 Laplacian: n^3 Kuhn cube, 6 n^3 tets, 0.15h jitter, FP32 coords."""
    return Workload(f"3D P1 Laplacian, {n}^3 Kuhn cube, {6*n**3} tets, FP32",
                    "laplace_p1", _cube(n))


def elast3d(n: int = 64, degenerate_frac: float = 0.01) -> Workload:
    """3D P1 elasticity: the lap3d mesh, 1% flattened tets, lognormal mu, lambda."""
    m = _cube(n)
    count = int(math.floor(m.n_elements * degenerate_frac))
    m = flatten_elements(m, count, SEED_BASE + 3)
    mu, lam = lame(m.n_elements, SEED_BASE + 30)
    return Workload(f"3D P1 elasticity, {n}^3 Kuhn cube, {m.n_elements} tets, "
                    f"{count} flattened, FP32", "elastic_p1", m, mu, lam)


def elast3d_adjoint(n: int = 64) -> Workload:
    """Adjoint workload: elast3d plus dL/dA_e ~ N(0, 1)."""
    w = elast3d(n)
    w.dA = upstream(w.mesh.n_elements, 12, SEED_BASE + 4)
    w.name = "adjoint of " + w.name
    return w


def fd_submesh(with_flattened: bool = False) -> Workload:
    """48 tets: the 8 cells [31,33)^3 of the 64^3 elasticity mesh.

    Vertices are renumbered compactly (27 vertices).  With ``with_flattened``
    one tet's fourth vertex is replaced by a flattened private vertex (28
    vertices), for the FP64 adjoint branch.
    """
    n = 64
    base = _cube(n)
    cells = [(i, j, k) for k in range(31, 33) for j in range(31, 33) for i in range(31, 33)]
    idx = np.array([6 * (i + n * (j + n * k)) + t for (i, j, k) in cells for t in range(6)])
    conn = base.conn[idx]
    verts, inv = np.unique(conn.ravel(), return_inverse=True)
    m = Mesh(base.coords[verts].copy(), inv.reshape(conn.shape).astype(np.int32))
    if with_flattened:
        m = flatten_elements(m, 1, SEED_BASE + 5)
    mu, lam = lame(m.n_elements, SEED_BASE + 31)
    dA = upstream(m.n_elements, 12, SEED_BASE + 41)
    return Workload("FD sub-mesh, 48 tets" + (" (one flattened)" if with_flattened else ""),
                    "elastic_p1", m, mu, lam, dA)


def batch_items(count: int = 64, lo: float = 1e3, hi: float = 5e5,
                seed: int = SEED_BASE + 5):
    """Heterogeneous batch: ``count`` meshes, E_i = floor(exp(U(ln lo, ln hi))).

    Forms are assigned round-robin over (2D P1 Laplacian, 3D P1 Laplacian,
    3D P1 elasticity, 3D P2 Laplacian), then shuffled.  Each mesh is the
    smallest structured box (2D: n x n squares; 3D: n x n x m cubes with
    n = round(cbrt(E/6))) holding at least E_i elements, truncated to its
    first E_i elements.  Elasticity items get lognormal mu, lambda.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Es = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    kinds = [("laplace_p1", 2), ("laplace_p1", 3), ("elastic_p1", 3), ("laplace_p2", 3)]
    assign = [kinds[i % 4] for i in range(count)]
    order = rng.permutation(count)
    assign = [assign[i] for i in order]
    items = []
    for i, (E, (form, dim)) in enumerate(zip(Es, assign)):
        s = int(SEED_BASE + 1000 + i)
        if dim == 2:
            n = max(1, math.ceil(math.sqrt(E / 2)))
            m = square_mesh(n, 0.2, s, np.float32)
        else:
            n = max(1, int(round((E / 6) ** (1 / 3))))
            nz = max(1, math.ceil(E / (6 * n * n)))
            m = cube_mesh(n, n, nz, 0.15, s, np.float32, h=1.0 / n)
        m = Mesh(m.coords, np.ascontiguousarray(m.conn[:E]))
        w = Workload(f"batch item {i}: {form} {dim}D E={E}", form, m)
        if form == "elastic_p1":
            w.mu, w.lam = lame(E, s + 500)
        items.append(w)
    return items
