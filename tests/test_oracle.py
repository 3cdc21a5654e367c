"""Pins for the FP64 oracle: closed forms, brute force and invariants.

None of these re-types the oracle's own formula: each check comes from a
different route (cotangent formulas, exact rational integration, textbook
reference-element matrices, physical invariances), so that a dropped term, a
wrong sign or index or a transposed operand in the oracle fails at least one.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import meshgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

REF = {2: np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
       3: np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])}


def _load_golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def _random_simplex(rng, dim, scale=1.0):
    while True:
        x = rng.uniform(-1, 1, size=(dim + 1, dim)) * scale
        if abs(np.linalg.det((x[1:] - x[0]).T)) > 0.05 * scale ** dim:
            return x


# --------------------------------------------------------------------------
# Quadrature
# --------------------------------------------------------------------------

def _compositions(total, parts):
    if parts == 1:
        yield (total,)
        return
    for i in range(total + 1):
        for rest in _compositions(total - i, parts - 1):
            yield (i,) + rest


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("s", [0, 1, 2, 3])
def test_gm_rule_integrates_barycentric_monomials(dim, s):
    """int_ref lambda^alpha = alpha! d! / (|alpha| + d)! * (1/d!), |alpha| <= 2s+1."""
    pts, w = oracle.gm_rule(dim, s)
    assert np.isclose(w.sum(), 1.0 / math.factorial(dim), rtol=0, atol=1e-15)
    for deg in range(2 * s + 2):
        for alpha in _compositions(deg, dim + 1):
            exact = (math.prod(math.factorial(a) for a in alpha) * math.factorial(dim)
                     / math.factorial(deg + dim)) / math.factorial(dim)
            q = float(np.sum(w * np.prod(pts ** np.array(alpha), axis=1)))
            assert abs(q - exact) < 1e-15, (alpha, q, exact)


# --------------------------------------------------------------------------
# Closed forms on the reference simplex
# --------------------------------------------------------------------------

def test_reference_triangle_laplace():
    A = oracle.element("laplace_p1", REF[2])
    np.testing.assert_allclose(A, _load_golden("ref_triangle_laplace_p1.txt"), atol=1e-15)


def test_reference_tet_laplace():
    A = oracle.element("laplace_p1", REF[3])
    np.testing.assert_allclose(6 * A, _load_golden("ref_tet_laplace_p1.txt"), atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_reference_elasticity_closed_form(dim):
    """On the unit simplex, with g the constant barycentric gradients (J = I):
    A_(a,c),(b,d) = vol [mu (delta_cd g_a.g_b + g_ad g_bc) + lam g_ac g_bd]."""
    g = np.vstack([-np.ones(dim), np.eye(dim)])
    vol = 1.0 / math.factorial(dim)
    mu, lam = 0.7, 1.9
    n = dim * (dim + 1)
    Aref = np.zeros((n, n))
    for a, c, b, d in itertools.product(range(dim + 1), range(dim), range(dim + 1), range(dim)):
        Aref[dim * a + c, dim * b + d] = vol * (
            mu * ((c == d) * g[a] @ g[b] + g[a, d] * g[b, c]) + lam * g[a, c] * g[b, d])
    A = oracle.element("elastic_p1", REF[dim], mu, lam)
    np.testing.assert_allclose(A, Aref, atol=1e-14)
    # the lambda part is rank one: vol * b b^T with b_(a,c) = g_ac
    Al = oracle.element("elastic_p1", REF[dim], 0.0, 1.0)
    b = g.reshape(-1)
    np.testing.assert_allclose(Al, vol * np.outer(b, b), atol=1e-15)


def _p2_exact_reference(dim):
    """P2 Laplacian on the unit simplex in exact rational arithmetic."""
    K = _p2_exact_tensor(dim)
    return sum(K[:, :, k, k] for k in range(dim))


def _p2_exact_tensor(dim, weight=None):
    """K[i, j, mu, nu] = int_ref dphi_i/dxi_mu dphi_j/dxi_nu for the P2 basis on
    the unit simplex, in exact rational arithmetic (returned as floats); with
    ``weight`` = m the integrand carries the extra factor lambda_m.

    grad phi_i = sum_a c_ia(lambda) grad lambda_a with c linear in lambda;
    int_ref lambda^alpha = alpha! / (|alpha| + d)!  (volume 1/d! included).
    """
    nv = dim + 1
    glam = [[Fraction(-1)] * dim] + [[Fraction(int(i == j)) for j in range(dim)] for i in range(dim)]
    # c[i][a] is a linear polynomial: dict {monomial exponent tuple: coeff}
    def mono(*idx):
        e = [0] * nv
        for k in idx:
            e[k] += 1
        return tuple(e)
    c = []
    for a in range(nv):          # vertex functions: grad = (4 lambda_a - 1) grad lambda_a
        row = [dict() for _ in range(nv)]
        row[a] = {mono(a): Fraction(4), mono(): Fraction(-1)}
        c.append(row)
    for a in range(nv):          # edge functions: 4 (lambda_a grad lambda_b + lambda_b grad lambda_a)
        for b in range(a + 1, nv):
            row = [dict() for _ in range(nv)]
            row[b] = {mono(a): Fraction(4)}
            row[a] = {mono(b): Fraction(4)}
            c.append(row)

    def integ(p, q):
        tot = Fraction(0)
        for ea, ca in p.items():
            for eb, cb in q.items():
                alpha = [x + y for x, y in zip(ea, eb)]
                if weight is not None:
                    alpha[weight] += 1
                tot += ca * cb * Fraction(math.prod(math.factorial(x) for x in alpha),
                                          math.factorial(sum(alpha) + dim))
        return tot

    n = len(c)
    K = np.zeros((n, n, dim, dim))
    for i in range(n):
        for j in range(n):
            for mu in range(dim):
                for nu in range(dim):
                    s = Fraction(0)
                    for a in range(nv):
                        for b in range(nv):
                            g = glam[a][mu] * glam[b][nu]
                            if g != 0 and c[i][a] and c[j][b]:
                                s += g * integ(c[i][a], c[j][b])
                    K[i, j, mu, nu] = float(s)
    return K


@pytest.mark.parametrize("dim", [2, 3])
def test_reference_p2_laplace_exact_rational(dim):
    A = oracle.element("laplace_p2", REF[dim])
    np.testing.assert_allclose(A, _p2_exact_reference(dim), atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_reference_p2_elasticity_exact_rational(dim):
    """P2 elasticity on the unit simplex: int mu (delta_cd grad phi_i . grad phi_j
    + d_d phi_i d_c phi_j) + lambda d_c phi_i d_d phi_j, node-major DOFs
    I = dim * i + c, from the exact-rational P2 tensor (isotropic Lame form of
    Sec. 3, eqs. 9-12, with the quadratic basis)."""
    K = _p2_exact_tensor(dim)
    nb = K.shape[0]
    mu, lam = 1.7, 0.6
    ref = np.zeros((dim * nb, dim * nb))
    for i in range(nb):
        for j in range(nb):
            for c in range(dim):
                for d in range(dim):
                    v = mu * K[i, j, d, c] + lam * K[i, j, c, d]
                    if c == d:
                        v += mu * np.trace(K[i, j])
                    ref[dim * i + c, dim * j + d] = v
    A = oracle.element("elastic_p2", REF[dim], mu, lam)
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def _p2_nodes(x):
    """P2 node positions: the vertices, then the edge midpoints in DOF order."""
    nv = x.shape[0]
    mids = [(x[a] + x[b]) / 2 for a in range(nv) for b in range(a + 1, nv)]
    return np.vstack([x] + mids)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_elasticity_rigid_modes_and_rank(dim):
    """P2 elasticity on random simplices: symmetric, PSD, rigid motions sampled at
    the P2 nodes span the null space exactly (rank n - 3 in 2D, n - 6 in 3D)."""
    rng = np.random.default_rng(17)
    for _ in range(15):
        x = _random_simplex(rng, dim)
        mu, lam = np.exp(rng.normal(size=2) * 0.5)
        A = oracle.element("elastic_p2", x, mu, lam)
        scale = np.abs(A).max()
        np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-13 * scale)
        R = _rigid_modes(_p2_nodes(x), dim)
        np.testing.assert_allclose(A @ R, 0, atol=1e-12 * scale)
        ev = np.linalg.eigvalsh(A)
        assert ev.min() > -1e-12 * scale
        nrig = 3 if dim == 2 else 6
        assert np.sum(ev > 1e-9 * scale) == A.shape[0] - nrig


# --------------------------------------------------------------------------
# Cotangent formulas: every element of jittered meshes
# --------------------------------------------------------------------------

def test_cotangent_formula_2d_every_element():
    """A_ij = -1/2 cot(theta_k), theta_k the angle at the third vertex."""
    m = meshgen.square_mesh(8, 0.2, 7)
    A = oracle.integrate("laplace_p1", m.coords, m.conn)
    X = m.coords
    for e in range(m.n_elements):
        v = X[m.conn[e]]
        ref = np.zeros((3, 3))
        for i, j in itertools.combinations(range(3), 2):
            k = 3 - i - j
            a, b = v[i] - v[k], v[j] - v[k]
            cot = (a @ b) / abs(a[0] * b[1] - a[1] * b[0])
            ref[i, j] = ref[j, i] = -0.5 * cot
        ref[np.diag_indices(3)] = -ref.sum(axis=1)
        np.testing.assert_allclose(A[e], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_cotangent_formula_3d_every_element():
    """A_ij = -1/6 l_kl cot(theta_kl), kl the opposite edge, theta its dihedral angle."""
    m = meshgen.cube_mesh(3, 3, 3, 0.15, 9, np.float64)
    A = oracle.integrate("laplace_p1", m.coords, m.conn)
    X = m.coords
    for e in range(m.n_elements):
        v = X[m.conn[e]]
        ref = np.zeros((4, 4))
        for i, j in itertools.combinations(range(4), 2):
            k, l = [t for t in range(4) if t not in (i, j)]
            ed = v[l] - v[k]
            L = np.linalg.norm(ed)
            t = ed / L
            u = (v[i] - v[k]) - ((v[i] - v[k]) @ t) * t
            w = (v[j] - v[k]) - ((v[j] - v[k]) @ t) * t
            cot = (u @ w) / np.linalg.norm(np.cross(u, w))
            ref[i, j] = ref[j, i] = -L * cot / 6.0
        ref[np.diag_indices(4)] = -ref.sum(axis=1)
        np.testing.assert_allclose(A[e], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# --------------------------------------------------------------------------
# The paper's elasticity form (eq. 24, UFL listing): mu = 1/2, lambda = 0
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_elasticity_is_symmetric_gradient_form(dim):
    """mu = 1/2, lambda = 0 gives int eps(v):eps(u), eps(u) = (grad u + grad u^T)/2.

    The strains of the vector basis Phi_(a,c) = phi_a e_c come from physical
    gradients solved from the edge matrix, not from the oracle's route."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = _random_simplex(rng, dim)
        E = (x[1:] - x[0]).T                      # columns are edges
        vol = abs(np.linalg.det(E)) / math.factorial(dim)
        g_ref = np.vstack([-np.ones(dim), np.eye(dim)])
        grads = g_ref @ np.linalg.inv(E)          # row a: grad phi_a
        eps = []
        for a in range(dim + 1):
            for c in range(dim):
                Du = np.zeros((dim, dim))
                Du[c, :] = grads[a]               # d(phi_a e_c)_c / dx
                eps.append(0.5 * (Du + Du.T))
        n = len(eps)
        ref = np.array([[vol * np.sum(eps[i] * eps[j]) for j in range(n)] for i in range(n)])
        A = oracle.element("elastic_p1", x, 0.5, 0.0)
        np.testing.assert_allclose(A, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        # and the lambda part is vol * div div
        div = np.array([grads[a, c] for a in range(dim + 1) for c in range(dim)])
        Al = oracle.element("elastic_p1", x, 0.0, 1.0)
        np.testing.assert_allclose(Al, vol * np.outer(div, div), rtol=0,
                                   atol=1e-12 * np.abs(Al).max())


# --------------------------------------------------------------------------
# Symmetry, definiteness, kernels
# --------------------------------------------------------------------------

def _rigid_modes(x, dim):
    """Translations and infinitesimal rotations evaluated at the nodes x, node-major."""
    modes = []
    for c in range(dim):
        t = np.zeros((x.shape[0], dim)); t[:, c] = 1
        modes.append(t.ravel())
    if dim == 2:
        modes.append(np.stack([-x[:, 1], x[:, 0]], axis=1).ravel())
    else:
        for axis in range(3):
            w = np.zeros(3); w[axis] = 1
            modes.append(np.cross(w, x).ravel())
    return np.array(modes).T


@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3), ("elastic_p1", 2),
                                      ("elastic_p1", 3), ("laplace_p2", 2), ("laplace_p2", 3)])
def test_symmetry_psd_and_kernel(form, dim):
    rng = np.random.default_rng(11)
    for _ in range(25):
        x = _random_simplex(rng, dim)
        mu, lam = np.exp(rng.normal(size=2) * 0.5)
        A = oracle.element(form, x, mu, lam)
        scale = np.abs(A).max()
        np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-13 * scale)
        ev = np.linalg.eigvalsh(A)
        assert ev.min() > -1e-12 * scale
        if form.startswith("laplace"):
            np.testing.assert_allclose(A.sum(axis=1), 0, atol=1e-12 * scale)
            assert np.sum(ev > 1e-9 * scale) == A.shape[0] - 1
        else:
            R = _rigid_modes(x, dim)
            np.testing.assert_allclose(A @ R, 0, atol=1e-12 * scale)
            nrig = 3 if dim == 2 else 6
            assert np.sum(ev > 1e-9 * scale) == A.shape[0] - nrig


# --------------------------------------------------------------------------
# Affine invariance
# --------------------------------------------------------------------------

def _rotation(rng, dim):
    q, r = np.linalg.qr(rng.normal(size=(dim, dim)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3), ("elastic_p1", 2),
                                      ("elastic_p1", 3), ("laplace_p2", 3)])
def test_affine_invariance(form, dim):
    rng = np.random.default_rng(5)
    for _ in range(10):
        x = _random_simplex(rng, dim)
        mu, lam = 1.3, 0.4
        A = oracle.element(form, x, mu, lam)
        tol = 1e-12 * np.abs(A).max()
        # translation
        np.testing.assert_allclose(oracle.element(form, x + rng.normal(size=dim), mu, lam), A, atol=tol)
        # rotation
        Q = _rotation(rng, dim)
        Ar = oracle.element(form, x @ Q.T, mu, lam)
        if form.startswith("laplace"):
            np.testing.assert_allclose(Ar, A, atol=tol)
        else:
            Rb = np.kron(np.eye(dim + 1), Q)
            np.testing.assert_allclose(Ar, Rb @ A @ Rb.T, atol=tol)
        # scaling: A -> alpha^(d-2) A
        alpha = 1.7
        np.testing.assert_allclose(oracle.element(form, alpha * x, mu, lam),
                                   alpha ** (dim - 2) * A, atol=tol * max(1, alpha ** (dim - 2)))
        # vertex permutation (P1 forms): rows/columns permute with the nodes
        if form.endswith("p1"):
            p = rng.permutation(dim + 1)
            Ap = oracle.element(form, x[p], mu, lam)
            nc = dim if form.startswith("elastic") else 1
            idx = np.array([nc * p[a] + c for a in range(dim + 1) for c in range(nc)])
            np.testing.assert_allclose(Ap, A[np.ix_(idx, idx)], atol=tol)


# --------------------------------------------------------------------------
# Brute force: a much higher quadrature degree changes nothing
# --------------------------------------------------------------------------

@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3), ("elastic_p1", 3),
                                      ("laplace_p2", 2), ("laplace_p2", 3), ("elastic_p2", 3)])
def test_quadrature_degree_7_equals_degree_3(form, dim):
    m = meshgen.cube_mesh(2, 2, 2, 0.15, 4, np.float64) if dim == 3 else meshgen.square_mesh(4, 0.2, 4)
    mu, lam = meshgen.lame(m.n_elements, 8)
    if form.startswith("elastic"):
        A3 = oracle.integrate(form, m.coords, m.conn, mu, lam, qs=1)
        A7 = oracle.integrate(form, m.coords, m.conn, mu, lam, qs=3)
    else:
        A3 = oracle.integrate(form, m.coords, m.conn, qs=1)
        A7 = oracle.integrate(form, m.coords, m.conn, qs=3)
    np.testing.assert_allclose(A7, A3, rtol=0, atol=1e-13 * np.abs(A3).max())


# --------------------------------------------------------------------------
# Global energy (patch) tests
# --------------------------------------------------------------------------

def _assemble(A, conn, nc, nv):
    n = A.shape[1]
    K = np.zeros((nv * nc, nv * nc))
    for e in range(conn.shape[0]):
        dofs = np.array([nc * v + c for v in conn[e] for c in range(nc)])
        K[np.ix_(dofs, dofs)] += A[e]
    return K


def test_patch_laplace_linear_field():
    """u = g.x linear: u^T K u = |g|^2 |Omega|, for a jittered unit cube."""
    m = meshgen.cube_mesh(3, 3, 3, 0.15, 21, np.float64)
    A = oracle.integrate("laplace_p1", m.coords, m.conn)
    K = _assemble(A, m.conn, 1, m.n_vertices)
    g = np.array([0.3, -1.2, 0.8])
    u = m.coords @ g
    assert np.isclose(u @ K @ u, g @ g * 1.0, rtol=1e-12)


def test_patch_elasticity_linear_field():
    """u = M x: u^T K u = sum_e vol_e (2 mu_e eps:eps + lam_e tr(eps)^2), eps = sym M."""
    m = meshgen.cube_mesh(2, 2, 2, 0.15, 22, np.float64)
    mu, lam = meshgen.lame(m.n_elements, 23)
    A = oracle.integrate("elastic_p1", m.coords, m.conn, mu, lam)
    K = _assemble(A, m.conn, 3, m.n_vertices)
    M = np.array([[0.1, 0.4, -0.2], [0.3, -0.5, 0.7], [0.05, 0.2, 0.9]])
    u = (m.coords @ M.T).ravel()
    eps = 0.5 * (M + M.T)
    X = m.coords
    vols = np.array([abs(np.linalg.det((X[c[1:]] - X[c[0]]).T)) / 6 for c in m.conn])
    ref = np.sum(vols * (2 * mu * np.sum(eps * eps) + lam * np.trace(eps) ** 2))
    assert np.isclose(u @ K @ u, ref, rtol=1e-12)


# --------------------------------------------------------------------------
# Laplacian with a P1 coefficient (Sec. 3.1, eqs. 20-23)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3), ("laplace_p2", 2),
                                      ("laplace_p2", 3)])
def test_coefficient_one_is_the_laplacian(form, dim):
    m = (meshgen.square_mesh(5, 0.2, 41, np.float64) if dim == 2
         else meshgen.cube_mesh(2, 2, 2, 0.15, 42, np.float64))
    A1 = oracle.integrate_coefficient(form, m.coords, m.conn, np.ones(m.n_vertices))
    A = oracle.integrate(form, m.coords, m.conn)
    np.testing.assert_allclose(A1, A, rtol=0, atol=1e-14 * np.abs(A).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_coefficient_p1_is_mean_times_laplacian(dim):
    """P1: grad phi constant, so int w grad phi_i . grad phi_j = mean_e(w) A_ij."""
    m = (meshgen.square_mesh(6, 0.2, 43, np.float64) if dim == 2
         else meshgen.cube_mesh(2, 3, 2, 0.15, 44, np.float64))
    rng = np.random.default_rng(45)
    w = np.exp(rng.normal(size=m.n_vertices))
    Aw = oracle.integrate_coefficient("laplace_p1", m.coords, m.conn, w)
    A = oracle.integrate("laplace_p1", m.coords, m.conn)
    ref = A * w[m.conn].mean(axis=1)[:, None, None]
    np.testing.assert_allclose(Aw, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_coefficient_p2_reference_exact_rational(dim):
    """P2 on the unit simplex with w = lambda_m (w = 1 at vertex m, 0 at the
    others): the exact-rational K^{ij m} traced over mu = nu."""
    for mvert in range(dim + 1):
        K = _p2_exact_tensor(dim, weight=mvert)
        ref = sum(K[:, :, k, k] for k in range(dim))
        w = np.zeros(dim + 1)
        w[mvert] = 1.0
        A = oracle.integrate_coefficient("laplace_p2", REF[dim], np.arange(dim + 1)[None], w)[0]
        np.testing.assert_allclose(A, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("form", ["laplace_p1", "laplace_p2"])
def test_coefficient_linear_kernel_patch_and_degree(form):
    """Linear in w; constants in the kernel; linear u: u^T K u = |g|^2 int w; a
    degree-7 rule agrees with the default degree-3 rule."""
    m = meshgen.cube_mesh(2, 2, 2, 0.15, 46, np.float64)
    rng = np.random.default_rng(47)
    w1, w2 = np.exp(rng.normal(size=(2, m.n_vertices)))
    A1 = oracle.integrate_coefficient(form, m.coords, m.conn, w1)
    A2 = oracle.integrate_coefficient(form, m.coords, m.conn, w2)
    A12 = oracle.integrate_coefficient(form, m.coords, m.conn, w1 + w2)
    np.testing.assert_allclose(A12, A1 + A2, rtol=0, atol=1e-14 * np.abs(A12).max())
    assert np.abs(A1.sum(axis=2)).max() <= 1e-13 * np.abs(A1).max()
    A7 = oracle.integrate_coefficient(form, m.coords, m.conn, w1, qs=3)
    np.testing.assert_allclose(A7, A1, rtol=0, atol=1e-13 * np.abs(A1).max())
    if form == "laplace_p1":
        K = _assemble(A1, m.conn, 1, m.n_vertices)
        g = np.array([0.4, -0.9, 0.3])
        u = m.coords @ g
        X = m.coords
        vols = np.array([abs(np.linalg.det((X[c[1:]] - X[c[0]]).T)) / 6 for c in m.conn])
        ref = g @ g * np.sum(vols * w1[m.conn].mean(axis=1))
        assert np.isclose(u @ K @ u, ref, rtol=1e-12)


# --------------------------------------------------------------------------
# General bilinear forms (the plain definition a form language describes)
# --------------------------------------------------------------------------

def _W_laplace(dim):
    W = np.zeros((1, dim + 1, dim + 1))
    for a in range(dim):
        W[0, 1 + a, 1 + a] = 1.0
    return W


def _W_elasticity(dim):
    """[const, mu, lambda] tables of 2 mu eps(u):eps(v) + lambda div u div v,
    index (direction a, component c) -> a * dim + c, direction 0 = value."""
    m = (dim + 1) * dim
    W = np.zeros((3, m, m))
    for al in range(dim):
        for c in range(dim):
            for be in range(dim):
                for d in range(dim):
                    i, j = (1 + al) * dim + c, (1 + be) * dim + d
                    W[1, i, j] = (c == d) * (al == be) + (al == d) * (be == c)
                    W[2, i, j] = (al == c) * (be == d)
    return W


@pytest.mark.parametrize("degree,dim", [(1, 2), (1, 3), (2, 2), (2, 3)])
def test_general_form_reproduces_laplacian_and_elasticity(degree, dim):
    m = (meshgen.square_mesh(4, 0.2, 51, np.float64) if dim == 2
         else meshgen.cube_mesh(2, 2, 1, 0.15, 52, np.float64))
    A = oracle.integrate_general(degree, 1, _W_laplace(dim), m.coords, m.conn)
    Ao = oracle.integrate(f"laplace_p{degree}", m.coords, m.conn)
    np.testing.assert_allclose(A, Ao, rtol=0, atol=1e-13 * np.abs(Ao).max())
    mu, lam = meshgen.lame(m.n_elements, 53)
    A = oracle.integrate_general(degree, dim, _W_elasticity(dim), m.coords, m.conn,
                                 np.stack([mu, lam]))
    Ao = oracle.integrate(f"elastic_p{degree}", m.coords, m.conn, mu, lam)   # Voigt B^T D B
    np.testing.assert_allclose(A, Ao, rtol=0, atol=1e-13 * np.abs(Ao).max())


@pytest.mark.parametrize("degree,dim", [(1, 2), (1, 3), (2, 2), (2, 3)])
def test_general_form_mass_matrix_exact_rational(degree, dim):
    """int_ref phi_i phi_j on the unit simplex, from exact barycentric integrals."""
    W = np.zeros((1, dim + 1, dim + 1))
    W[0, 0, 0] = 1.0
    A = oracle.integrate_general(degree, 1, W, REF[dim], np.arange(dim + 1)[None])[0]
    nv = dim + 1
    # basis as barycentric polynomials {exponent tuple: coefficient}
    def mono(*idx):
        e = [0] * nv
        for k in idx:
            e[k] += 1
        return tuple(e)
    basis = [{mono(a, a): Fraction(2), mono(a): Fraction(-1)} if degree == 2 else {mono(a): Fraction(1)}
             for a in range(nv)]
    if degree == 2:
        basis += [{mono(a, b): Fraction(4)} for a in range(nv) for b in range(a + 1, nv)]
    def integ(p, q):
        tot = Fraction(0)
        for ea, ca in p.items():
            for eb, cb in q.items():
                al = [x + y for x, y in zip(ea, eb)]
                tot += ca * cb * Fraction(math.prod(math.factorial(x) for x in al),
                                          math.factorial(sum(al) + dim))
        return tot
    ref = np.array([[float(integ(p, q)) for q in basis] for p in basis])
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_general_form_value_derivative_p1_closed_form(dim):
    """int (b . grad u) v + (b . grad v) u for P1: grad lambda constant and
    int lambda_i = vol / (d + 1), so A_ij = vol/(d+1) (b.g_j + b.g_i)."""
    rng = np.random.default_rng(54)
    b = rng.normal(size=dim)
    W = np.zeros((1, dim + 1, dim + 1))
    W[0, 0, 1:] = b
    W[0, 1:, 0] = b
    for _ in range(5):
        x = _random_simplex(rng, dim)
        A = oracle.integrate_general(1, 1, W, x, np.arange(dim + 1)[None])[0]
        V = np.hstack([np.ones((dim + 1, 1)), x])
        G = np.linalg.inv(V)[1:].T                       # grad lambda_a, [a][alpha]
        vol = abs(np.linalg.det(V)) / math.factorial(dim)
        bg = G @ b
        ref = vol / (dim + 1) * (bg[None, :] + bg[:, None])
        np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# --------------------------------------------------------------------------
# Global assembly (sparse), pinned by dense loops, energy and kernel
# --------------------------------------------------------------------------

@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3), ("elastic_p1", 2),
                                      ("elastic_p1", 3)])
def test_assemble_equals_dense_loops(form, dim):
    """The sparse COO -> CSR sum equals element-by-element dense accumulation
    (a different route: index arithmetic written out per element)."""
    m = (meshgen.square_mesh(4, 0.2, 31, np.float64) if dim == 2
         else meshgen.cube_mesh(2, 2, 1, 0.15, 32, np.float64))
    mu = lam = None
    if form == "elastic_p1":
        mu, lam = meshgen.lame(m.n_elements, 33)
    K = oracle.assemble(form, m.coords, m.conn, mu, lam)
    A = oracle.integrate(form, m.coords, m.conn, mu, lam)
    nc = dim if form == "elastic_p1" else 1
    D = _assemble(A, m.conn, nc, m.n_vertices)
    np.testing.assert_allclose(K.toarray(), D, rtol=0, atol=1e-15 * np.abs(D).max())
    # the pattern: exactly the DOF pairs that share an element
    P = np.zeros((nc * m.n_vertices,) * 2, bool)
    for c in m.conn:
        d = np.array([nc * v + k for v in c for k in range(nc)])
        P[np.ix_(d, d)] = True
    S = np.zeros_like(P)
    S[np.repeat(np.arange(K.shape[0]), np.diff(K.indptr)), K.indices] = True
    assert np.array_equal(S, P)
    assert np.all(np.diff(K.indices)[np.diff(np.repeat(np.arange(K.shape[0]),
                                                       np.diff(K.indptr))) == 0] > 0)


def test_assembled_laplace_energy_rowsums_symmetry():
    """u = g.x linear: u^T K u = |g|^2 |Omega| (unit cube); constants in the kernel."""
    m = meshgen.cube_mesh(3, 3, 3, 0.15, 34, np.float64)
    K = oracle.assemble("laplace_p1", m.coords, m.conn)
    g = np.array([-0.7, 0.2, 1.1])
    u = m.coords @ g
    assert np.isclose(u @ (K @ u), g @ g, rtol=1e-12)
    assert np.abs(K @ np.ones(K.shape[0])).max() <= 1e-14 * abs(K).max()
    assert abs(K - K.T).max() <= 1e-16 * abs(K).max()


def test_assembled_elasticity_energy_and_rigid_modes():
    """u = M x: u^T K u = sum_e vol_e (2 mu eps:eps + lam tr(eps)^2); the six rigid
    motions of the whole body are in the kernel of K."""
    m = meshgen.cube_mesh(3, 2, 2, 0.15, 35, np.float64)
    mu, lam = meshgen.lame(m.n_elements, 36)
    K = oracle.assemble("elastic_p1", m.coords, m.conn, mu, lam)
    M = np.array([[0.2, -0.4, 0.1], [0.6, 0.3, -0.7], [0.15, 0.25, -0.9]])
    u = (m.coords @ M.T).ravel()
    eps = 0.5 * (M + M.T)
    X = m.coords
    vols = np.array([abs(np.linalg.det((X[c[1:]] - X[c[0]]).T)) / 6 for c in m.conn])
    ref = np.sum(vols * (2 * mu * np.sum(eps * eps) + lam * np.trace(eps) ** 2))
    assert np.isclose(u @ (K @ u), ref, rtol=1e-12)
    R = _rigid_modes(m.coords, 3)
    assert np.abs(K @ R).max() <= 1e-13 * abs(K).max()


# --------------------------------------------------------------------------
# Oracle gradient: finite differences and invariants
# --------------------------------------------------------------------------

def _loss(form, coords, conn, dA, mu, lam):
    if form.startswith("elastic"):
        A = oracle.integrate(form, coords, conn, mu, lam)
    else:
        A = oracle.integrate(form, coords, conn)
    return float(np.sum(A * dA))


@pytest.mark.parametrize("flat", [False, True])
def test_gradient_matches_central_fd(flat):
    """Complex-step gradient vs FP64 central differences on the 48-tet sub-mesh."""
    w = meshgen.fd_submesh(flat)
    m = w.mesh
    X = m.coords.astype(np.float64)
    mu = w.mu.astype(np.float64); lam = w.lam.astype(np.float64)
    dA = w.dA.astype(np.float64)
    gv, gmu, glam, Le = oracle.gradient("elastic_p1", X, m.conn, dA, mu, lam)
    gx = oracle.vertex_gradient(gv, m.conn, m.n_vertices)
    # step: ~1e-6 h for regular tets; the flattened tet's altitude is ~1e-3 of
    # its edges, so its truncation error needs a smaller step (FD floor ~3e-8)
    h = 1e-9 if flat else 1e-6 / 64
    fd = np.zeros_like(X)
    for v in range(m.n_vertices):
        for a in range(3):
            Xp = X.copy(); Xp[v, a] += h
            Xm = X.copy(); Xm[v, a] -= h
            fd[v, a] = (_loss("elastic_p1", Xp, m.conn, dA, mu, lam)
                        - _loss("elastic_p1", Xm, m.conn, dA, mu, lam)) / (2 * h)
    np.testing.assert_allclose(gx, fd, rtol=0, atol=1e-7 * np.abs(fd).max())
    hm = 1e-6
    for e in range(0, m.n_elements, 7):
        mp = mu.copy(); mp[e] += hm
        mm = mu.copy(); mm[e] -= hm
        fdm = (_loss("elastic_p1", X, m.conn, dA, mp, lam)
               - _loss("elastic_p1", X, m.conn, dA, mm, lam)) / (2 * hm)
        assert abs(fdm - gmu[e]) < 1e-7 * max(1, abs(fdm))
        lp = lam.copy(); lp[e] += hm
        lm = lam.copy(); lm[e] -= hm
        fdl = (_loss("elastic_p1", X, m.conn, dA, mu, lp)
               - _loss("elastic_p1", X, m.conn, dA, mu, lm)) / (2 * hm)
        assert abs(fdl - glam[e]) < 1e-7 * max(1, abs(fdl))


@pytest.mark.parametrize("form,dim", [("laplace_p1", 2), ("laplace_p1", 3), ("elastic_p1", 3),
                                      ("laplace_p2", 3)])
def test_gradient_invariants(form, dim):
    """Translation: sum_v xbar_v = 0.  Euler (A is homogeneous of degree d-2 in x):
    sum_v x_v . xbar_v = (d-2) L.  Linearity in mu, lambda: sum (mu mubar + lam lambar) = L.
    Laplacian rotation invariance: sum_v x_v x xbar_v = 0."""
    m = meshgen.cube_mesh(2, 2, 2, 0.15, 31, np.float64) if dim == 3 else meshgen.square_mesh(3, 0.2, 31)
    n = oracle.local_size(form, dim)
    dA = meshgen.upstream(m.n_elements, n, 32).astype(np.float64)
    mu, lam = meshgen.lame(m.n_elements, 33)
    mu = mu.astype(np.float64); lam = lam.astype(np.float64)
    el = form.startswith("elastic")
    gv, gmu, glam, Le = oracle.gradient(form, m.coords, m.conn, dA,
                                        mu if el else None, lam if el else None)
    L = Le.sum()
    for e in range(m.n_elements):          # per element
        xe = m.coords[m.conn[e]]
        scale = np.abs(gv[e]).max() * np.abs(xe).max() + abs(Le[e])
        np.testing.assert_allclose(gv[e].sum(axis=0), 0, atol=1e-12 * np.abs(gv[e]).max())
        assert abs(np.sum(xe * gv[e]) - (dim - 2) * Le[e]) < 1e-12 * scale
        if el:
            assert abs(mu[e] * gmu[e] + lam[e] * glam[e] - Le[e]) < 1e-12 * (abs(Le[e]) + 1e-300 + scale)
    gx = oracle.vertex_gradient(gv, m.conn, m.n_vertices)
    scale = np.abs(gx).max()
    np.testing.assert_allclose(gx.sum(axis=0), 0, atol=1e-12 * scale * m.n_vertices)
    assert abs(np.sum(m.coords * gx) - (dim - 2) * L) < 1e-11 * (scale * m.n_vertices + abs(L))
    if el:
        assert abs(np.sum(mu * gmu + lam * glam) - L) < 1e-11 * abs(L)
    elif dim == 3:
        np.testing.assert_allclose(np.cross(m.coords, gx).sum(axis=0), 0,
                                   atol=1e-11 * scale * m.n_vertices)
    else:
        tq = m.coords[:, 0] * gx[:, 1] - m.coords[:, 1] * gx[:, 0]
        assert abs(tq.sum()) < 1e-11 * scale * m.n_vertices


def test_oracle_rejects_bad_connectivity():
    m = meshgen.square_mesh(2, 0.0)
    conn = m.conn.copy(); conn[0, 0] = m.n_vertices
    with pytest.raises(ValueError):
        oracle.integrate("laplace_p1", m.coords, conn)
