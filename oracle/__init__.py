"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this package.  It wraps ``liboracle.so`` (plain C, built from
``oracle.c`` with gcc) through ctypes and shares nothing with the GPU library.

Forms are named by strings: ``"laplace_p1"``, ``"elastic_p1"``,
``"laplace_p2"`` (and ``"elastic_p2"``, which the oracle also supports).
Coordinates are [N_v, dim] arrays (any float dtype, promoted to double).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_KIND = {"laplace": 0, "elastic": 1}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP over elements)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    # -std=c11 keeps floating-point contraction off (no FMA fusion), so the
    # results do not depend on the instruction set; x86-64-v3 (AVX2, FMA) runs
    # on every host this library is copied to, where -march=native might not.
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_version.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    lib.oracle_gm_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    lib.oracle_gm_rule.restype = ctypes.c_int
    lib.oracle_element.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   dp, dp]
    lib.oracle_element.restype = ctypes.c_int
    lib.oracle_integrate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int64, dp, dp, dp, ctypes.c_int64,
                                     ip, dp, dp, ctypes.c_int, dp]
    lib.oracle_integrate.restype = ctypes.c_int
    lib.oracle_gradient.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int64, dp, dp, dp, ctypes.c_int64,
                                    ip, dp, dp, dp, ctypes.c_int, dp, dp, dp, dp]
    lib.oracle_gradient.restype = ctypes.c_int
    lib.oracle_integrate_w.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp, dp,
                                       ctypes.c_int64, ip, dp, ctypes.c_int, dp]
    lib.oracle_integrate_w.restype = ctypes.c_int
    lib.oracle_integrate_general.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int64, dp, dp, dp, ctypes.c_int64, ip,
                                             ctypes.c_int, dp, dp, ctypes.c_int, dp]
    lib.oracle_integrate_general.restype = ctypes.c_int
    lib.oracle_integrate_iso.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, dp, ctypes.c_int64,
                                         ip, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_integrate_iso.restype = ctypes.c_int
    _lib = lib
    return lib


def set_threads(n: int) -> int:
    """Number of OpenMP threads for the loops over elements (timing only)."""
    return int(_load().oracle_set_threads(int(n)))


def _parse(form: str):
    kind, deg = form.split("_p")
    return _KIND[kind], int(deg)


def local_size(form: str, dim: int) -> int:
    kind, deg = _parse(form)
    nv = dim + 1
    nb = nv if deg == 1 else nv * (nv + 1) // 2
    return dim * nb if kind == 1 else nb


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def gm_rule(dim: int, s: int):
    """Grundmann-Moeller points (barycentric, [nq, dim+1]) and weights (sum 1/dim!)."""
    lib = _load()
    pts = np.zeros((128, 4)); w = np.zeros(128)
    nq = lib.oracle_gm_rule(dim, s, _ptr(pts), _ptr(w))
    if nq < 0:
        raise ValueError("rule too large")
    return pts[:nq, :dim + 1].copy(), w[:nq].copy()


def element(form: str, xv, mu: float = 0.0, lam: float = 0.0, qs: int = 1):
    """Element matrix of one simplex with vertices xv [dim+1, dim]."""
    lib = _load()
    kind, deg = _parse(form)
    xv = np.ascontiguousarray(xv, dtype=np.float64)
    dim = xv.shape[1]
    n = local_size(form, dim)
    A = np.zeros((n, n))
    det = ctypes.c_double()
    rc = lib.oracle_element(kind, deg, dim, _ptr(xv), float(mu), float(lam), qs,
                            _ptr(A), ctypes.byref(det))
    if rc:
        raise ValueError("oracle_element failed")
    return A


def _coords_soa(coords):
    c = np.asarray(coords, dtype=np.float64)
    dim = c.shape[1]
    x = np.ascontiguousarray(c[:, 0]); y = np.ascontiguousarray(c[:, 1])
    z = np.ascontiguousarray(c[:, 2]) if dim == 3 else None
    return dim, x, y, z


def integrate(form: str, coords, conn, mu=None, lam=None, qs: int = 1) -> np.ndarray:
    """Element matrices [E, n, n] (float64) of every element of a mesh."""
    lib = _load()
    kind, deg = _parse(form)
    dim, x, y, z = _coords_soa(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E = conn.shape[0]
    n = local_size(form, dim)
    m = np.ascontiguousarray(mu, dtype=np.float64) if mu is not None else None
    l = np.ascontiguousarray(lam, dtype=np.float64) if lam is not None else None
    A = np.empty((E, n, n))
    rc = lib.oracle_integrate(kind, deg, dim, x.shape[0], _ptr(x), _ptr(y), _ptr(z),
                              E, _ptr(conn, ctypes.c_int32), _ptr(m), _ptr(l), qs,
                              _ptr(A))
    if rc:
        raise ValueError(f"oracle_integrate failed ({rc})")
    return A


def integrate_coefficient(form: str, coords, conn, w, qs: int = 1) -> np.ndarray:
    """Element matrices [E, n, n] (float64) of the Laplacian with a P1
    coefficient w given per vertex ([N_v]): A_ij = int w grad phi_i . grad phi_j
    (Sec. 3.1, eqs. 20-21), form "laplace_p1" or "laplace_p2"."""
    lib = _load()
    kind, deg = _parse(form)
    if kind != 0:
        raise ValueError("integrate_coefficient: Laplacian forms only")
    dim, x, y, z = _coords_soa(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E = conn.shape[0]
    n = local_size(form, dim)
    wv = np.ascontiguousarray(w, dtype=np.float64)
    if wv.shape != (x.shape[0],):
        raise ValueError("w must hold one value per vertex")
    A = np.empty((E, n, n))
    rc = lib.oracle_integrate_w(deg, dim, x.shape[0], _ptr(x), _ptr(y), _ptr(z), E,
                                _ptr(conn, ctypes.c_int32), _ptr(wv), qs, _ptr(A))
    if rc:
        raise ValueError(f"oracle_integrate_w failed ({rc})")
    return A


def integrate_general(degree: int, ncomp: int, W, coords, conn, coefs=(), qs: int = 2):
    """Element matrices [E, n, n] of a general bilinear form of Lagrange
    elements: A_{(i,c),(j,d)} = int sum_{a,b} C[(a,c),(b,d)] D_a phi_i D_b phi_j,
    D_0 the value, D_{1+alpha} = d/dx_alpha, C = W[0] + sum_k coefs[k][e] W[k+1].
    W: [n_coef + 1, m, m] with m = (dim + 1) * ncomp, index a * ncomp + c.
    The default rule (qs = 2, degree 5) is exact for P2 mass terms (degree 4)."""
    lib = _load()
    dim, x, y, z = _coords_soa(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E = conn.shape[0]
    nb = dim + 1 if degree == 1 else (dim + 1) * (dim + 2) // 2
    n = ncomp * nb
    W = np.ascontiguousarray(W, dtype=np.float64)
    m = (dim + 1) * ncomp
    if W.ndim != 3 or W.shape[1:] != (m, m):
        raise ValueError(f"W must be [n_coef + 1, {m}, {m}]")
    n_coef = W.shape[0] - 1
    cf = np.ascontiguousarray(np.reshape(coefs, (n_coef, E)) if n_coef else np.zeros(1),
                              dtype=np.float64)
    A = np.empty((E, n, n))
    rc = lib.oracle_integrate_general(degree, dim, ncomp, x.shape[0], _ptr(x), _ptr(y), _ptr(z),
                                      E, _ptr(conn, ctypes.c_int32), n_coef, _ptr(W), _ptr(cf),
                                      qs, _ptr(A))
    if rc:
        raise ValueError(f"oracle_integrate_general failed ({rc})")
    return A


def integrate_iso(coords, conn, mode: str = "projected", qs: int = 2) -> np.ndarray:
    """Element matrices [E, nb, nb] (float64) of the isoparametric P2 Laplacian on
    elements with quadratic geometry (Sec. 3.1, eqs. 16-19); conn [E, nb] lists
    each element's nodes, vertices then edge nodes (the P2 order).
    mode "projected": the paper's scheme -- J^-1 interpolated linearly from its
    values at the vertices, |J| the constant |det J| at the barycenter;
    mode "exact": the isoparametric integral with J(xi) at every point."""
    lib = _load()
    dim, x, y, z = _coords_soa(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E, nb = conn.shape
    if nb != (dim + 1) * (dim + 2) // 2:
        raise ValueError("conn must list the P2 nodes of each element")
    A = np.empty((E, nb, nb))
    rc = lib.oracle_integrate_iso(dim, x.shape[0], _ptr(x), _ptr(y), _ptr(z), E,
                                  _ptr(conn, ctypes.c_int32), {"projected": 0, "exact": 1}[mode],
                                  qs, _ptr(A))
    if rc:
        raise ValueError(f"oracle_integrate_iso failed ({rc})")
    return A


def gradient(form: str, coords, conn, dA, mu=None, lam=None, qs: int = 1):
    """Complex-step gradient of L = sum_e <dA_e, A_e>.

    Returns (gvert [E, dim+1, dim], gmu [E] or None, glam [E] or None, L_e [E]).
    """
    lib = _load()
    kind, deg = _parse(form)
    dim, x, y, z = _coords_soa(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E = conn.shape[0]
    n = local_size(form, dim)
    dA = np.ascontiguousarray(dA, dtype=np.float64).reshape(E, n, n)
    m = np.ascontiguousarray(mu, dtype=np.float64) if mu is not None else None
    l = np.ascontiguousarray(lam, dtype=np.float64) if lam is not None else None
    gv = np.zeros((E, dim + 1, dim))
    gm = np.zeros(E) if kind == 1 else None
    gl = np.zeros(E) if kind == 1 else None
    Lv = np.zeros(E)
    rc = lib.oracle_gradient(kind, deg, dim, x.shape[0], _ptr(x), _ptr(y), _ptr(z),
                             E, _ptr(conn, ctypes.c_int32), _ptr(m), _ptr(l),
                             _ptr(dA), qs, _ptr(gv), _ptr(gm), _ptr(gl), _ptr(Lv))
    if rc:
        raise ValueError(f"oracle_gradient failed ({rc})")
    return gv, gm, gl, Lv


def assemble(form: str, coords, conn, mu=None, lam=None, qs: int = 1):
    """Global matrix K = sum_e P_e^T A_e P_e of a P1 form (the global portion of
    the computation that element integration feeds, Sec. 1), as a
    scipy.sparse CSR matrix over scalar DOFs with sorted column indices.

    DOFs: vertex v for the Laplacian; dim * v + c for elasticity (node-major,
    the element's DOF I = dim * a + c maps to dim * conn[e][a] + c).  Every
    (row, column) pair that shares an element is stored, even where the sum is
    zero.  The element matrices come from integrate(); COO entries with equal
    (row, column) are summed by scipy's COO -> CSR conversion."""
    import scipy.sparse as sp
    kind, deg = _parse(form)
    if deg != 1:
        raise ValueError("assemble: P1 forms only")
    conn = np.ascontiguousarray(conn, dtype=np.int64)
    dim = np.asarray(coords).shape[1]
    A = integrate(form, coords, conn, mu, lam, qs)
    nc = dim if kind == 1 else 1
    nv = np.asarray(coords).shape[0]
    dofs = (nc * conn[:, :, None] + np.arange(nc)[None, None, :]).reshape(conn.shape[0], -1)
    n = dofs.shape[1]
    rows = np.broadcast_to(dofs[:, :, None], (conn.shape[0], n, n)).ravel()
    cols = np.broadcast_to(dofs[:, None, :], (conn.shape[0], n, n)).ravel()
    K = sp.coo_matrix((A.ravel(), (rows, cols)), shape=(nc * nv, nc * nv)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K


def vertex_gradient(gvert: np.ndarray, conn, n_vertices: int) -> np.ndarray:
    """Sum per-element vertex gradients into [N_v, dim] (dL/dx_v = sum_e dL_e/dx_v)."""
    conn = np.asarray(conn)
    dim = gvert.shape[2]
    g = np.zeros((n_vertices, dim))
    np.add.at(g, conn.ravel(), gvert.reshape(-1, dim))
    return g
