"""The form front end on the CPU: the form language's lowering to operator
tables, the library's exact reference tensor Khat (against exact rational
integration written here and against the block tensor of eq. 7), the
contraction A = G : Khat with the recipe G = |J| That^T C That evaluated in
numpy against the oracle's direct quadrature, and the entry points' argument
checks.  Nothing here launches a kernel."""
import ctypes
import math
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle

fei = pytest.importorskip("paper_1103_0066_amd")
from paper_1103_0066_amd import _lib  # noqa: E402
from paper_1103_0066_amd import forms as F  # noqa: E402


def _random_simplex(rng, dim):
    while True:
        x = rng.uniform(-1, 1, size=(dim + 1, dim))
        if abs(np.linalg.det((x[1:] - x[0]).T)) > 0.05:
            return x


# ---- the language ------------------------------------------------------------

def _W_elasticity_by_hand(dim):
    """(lam, mu) tables of 2 mu eps:eps + lam div div, written out entry by entry."""
    m = (dim + 1) * dim
    Wl, Wm = np.zeros((m, m)), np.zeros((m, m))
    for al, c, be, d in product(range(dim), repeat=4):
        i, j = (1 + al) * dim + c, (1 + be) * dim + d
        Wm[i, j] = (c == d) * (al == be) + (al == d) * (be == c)
        Wl[i, j] = (al == c) * (be == d)
    return Wl, Wm


@pytest.mark.parametrize("dim", [2, 3])
def test_lowering_of_laplacian_mass_and_elasticity(dim):
    el = F.Element(dim, 1)
    u, v = F.TrialFunction(el), F.TestFunction(el)
    W, names = F.lower(F.inner(F.grad(u), F.grad(v)) + 3.0 * u * v)
    ref = np.diag([3.0] + [1.0] * dim)[None]
    assert names == [] and np.array_equal(W, ref)
    ev = F.Element(dim, 2, vector=True)
    u, v = F.TrialFunction(ev), F.TestFunction(ev)
    mu, lam = F.Coefficient("mu"), F.Coefficient("lam")
    W, names = F.lower(2 * mu * F.inner(F.eps(u), F.eps(v)) + lam * F.div(u) * F.div(v))
    Wl, Wm = _W_elasticity_by_hand(dim)
    assert names == ["lam", "mu"]
    assert np.array_equal(W[0], np.zeros_like(Wl))
    np.testing.assert_array_equal(W[1], Wl)
    np.testing.assert_array_equal(W[2], Wm)


def test_lowering_orientation_and_rejections():
    """Rows belong to the test function whichever side it is written on; a
    product of two test (or trial) operands, or two coefficients, is refused."""
    el = F.Element(3, 1)
    u, v = F.TrialFunction(el), F.TestFunction(el)
    b = F.Coefficient("b")
    W, names = F.lower(b * (u * v))
    assert names == ["b"] and W[1][0, 0] == 1.0 and np.count_nonzero(W) == 1
    # advection-like term (du/dx_0) v: row = value of v, column = d/dx_0 of u
    W, _ = F.lower(F.grad(u)[0] * v)
    assert W[0][0, 1] == 1.0 and W[0][1, 0] == 0.0 and np.count_nonzero(W) == 1
    W2, _ = F.lower(v * F.grad(u)[0])
    assert np.array_equal(W, W2)
    with pytest.raises(ValueError):
        u * u
    with pytest.raises(ValueError):
        (b * u) * (F.Coefficient("c") * v)
    with pytest.raises(ValueError):
        F.grad(F.grad(u)[0])


# ---- the reference tensor ------------------------------------------------------

def _basis_fractions(dim, degree):
    """Scalar Lagrange basis as barycentric polynomials {exponents: Fraction}."""
    nv = dim + 1

    def mono(*idx):
        e = [0] * nv
        for k in idx:
            e[k] += 1
        return tuple(e)
    if degree == 1:
        return [{mono(a): Fraction(1)} for a in range(nv)]
    B = [{mono(a, a): Fraction(2), mono(a): Fraction(-1)} for a in range(nv)]
    B += [{mono(a, b): Fraction(4)} for a in range(nv) for b in range(a + 1, nv)]
    return B


def _dxi(p, mu):
    out = {}
    for e, c in p.items():
        for k, sgn in ((mu + 1, 1), (0, -1)):
            if e[k]:
                f = list(e)
                f[k] -= 1
                out[tuple(f)] = out.get(tuple(f), 0) + sgn * e[k] * c
    return out


def _integ(p, q, dim):
    tot = Fraction(0)
    for ea, ca in p.items():
        for eb, cb in q.items():
            al = [x + y for x, y in zip(ea, eb)]
            tot += ca * cb * Fraction(math.prod(math.factorial(x) for x in al),
                                      math.factorial(sum(al) + dim))
    return tot


@pytest.mark.parametrize("dim,degree", [(2, 1), (3, 1), (2, 2), (3, 2)])
def test_reference_tensor_is_exact(dim, degree):
    K = F.reference_tensor(dim, degree)
    B = _basis_fractions(dim, degree)
    D = [[b] + [_dxi(b, mu) for mu in range(dim)] for b in B]
    nb = len(B)
    assert K.shape == (nb, nb, dim + 1, dim + 1)
    for i, j, p, q in product(range(nb), range(nb), range(dim + 1), range(dim + 1)):
        assert K[i, j, p, q] == float(_integ(D[i][p], D[j][q], dim)), (i, j, p, q)


@pytest.mark.parametrize("dim,degree", [(2, 1), (3, 1), (2, 2), (3, 2)])
def test_reference_tensor_derivative_block_is_eq7(dim, degree):
    """The derivative-derivative block equals the library's block tensor of eq. 7
    (built from exact integer formulas), and the value-value block sums to the
    reference volume (partition of unity)."""
    K = F.reference_tensor(dim, degree)
    Kb = fei.reference_tensor(f"laplace_p{degree}", dim, "block").astype(np.float64)
    np.testing.assert_allclose(K[:, :, 1:, 1:], Kb, rtol=0, atol=1e-7)
    assert abs(K[:, :, 0, 0].sum() - 1.0 / math.factorial(dim)) < 1e-15


def _contract_on_host(K, W, coefs, x, ncomp):
    """A = sum_pq G_{(p,c),(q,d)} Khat_ij^{pq}, G = |J| That^T C That (the kernel's
    recipe, evaluated here in numpy for one element with vertices x)."""
    dim = x.shape[1]
    nd, nb = dim + 1, K.shape[0]
    J = (x[1:] - x[0]).T
    B = np.linalg.inv(J)
    s = abs(np.linalg.det(J))
    C = W[0] + sum(c * Wk for c, Wk in zip(coefs, W[1:]))
    T = np.zeros((nd, nd))
    T[0, 0] = 1.0
    T[1:, 1:] = B.T                          # That[1+alpha][1+mu] = B[mu][alpha]
    Tt = np.kron(T, np.eye(ncomp))           # index a * ncomp + c
    G = s * Tt.T @ C @ Tt
    n = ncomp * nb
    A = np.zeros((n, n))
    for i, c, j, d in product(range(nb), range(ncomp), range(nb), range(ncomp)):
        A[ncomp * i + c, ncomp * j + d] = sum(
            G[p * ncomp + c, q * ncomp + d] * K[i, j, p, q] for p in range(nd) for q in range(nd))
    return A


@pytest.mark.parametrize("dim,degree,vector", [(2, 1, False), (3, 2, False), (2, 2, True),
                                               (3, 1, True), (3, 2, True)])
def test_khat_and_recipe_reproduce_the_oracle(dim, degree, vector):
    """The library's Khat contracted with the recipe's G reaches the oracle's
    direct quadrature (for affine elements the method is exact)."""
    rng = np.random.default_rng(7 + dim + degree)
    el = F.Element(dim, degree, vector)
    u, v = F.TrialFunction(el), F.TestFunction(el)
    k1, k2 = F.Coefficient("k1"), F.Coefficient("k2")
    if vector:
        a = (2 * k1 * F.inner(F.eps(u), F.eps(v)) + k2 * F.div(u) * F.div(v) + 0.5 * F.dot(u, v)
             + F.grad(u)[0, 1] * v[dim - 1])           # a non-symmetric coupling
    else:
        a = k1 * F.inner(F.grad(u), F.grad(v)) + k2 * u * v + 0.7 * (F.grad(u)[0] * v)
    W, names = F.lower(a)
    K = F.reference_tensor(dim, degree)
    for _ in range(4):
        x = _random_simplex(rng, dim)
        cf = rng.uniform(0.5, 2.0, size=len(names))
        A = _contract_on_host(K, W, cf, x, el.ncomp)
        Ao = oracle.integrate_general(degree, el.ncomp, W, x, np.arange(dim + 1)[None],
                                      cf[:, None])[0]
        np.testing.assert_allclose(A, Ao, rtol=0, atol=1e-12 * np.abs(Ao).max())


# ---- the C ABI -------------------------------------------------------------------

@pytest.mark.parametrize("args", [(4, 1, 1, 0), (3, 3, 1, 0), (3, 1, 2, 0), (3, 1, 1, 5),
                                  (3, 1, 1, -1)])
def test_form_create_rejects_before_any_device_work(args):
    lib = _lib.load()
    dim, degree, ncomp, n_coef = args
    W = np.zeros((max(n_coef, 0) + 1, 16, 16))
    h = ctypes.c_void_p()
    assert lib.fei_form_create(dim, degree, ncomp, n_coef, W.ctypes.data,
                               ctypes.byref(h)) == _lib.FEI_EINVAL
    W = np.full((1, 4, 4), np.nan)
    assert lib.fei_form_create(3, 1, 1, 0, W.ctypes.data, ctypes.byref(h)) == _lib.FEI_EINVAL
    assert lib.fei_form_create(3, 1, 1, 0, None, ctypes.byref(h)) == _lib.FEI_EINVAL
    n = ctypes.c_int64()
    assert lib.fei_form_reference_tensor(4, 1, None, ctypes.byref(n)) == _lib.FEI_EINVAL
    assert lib.fei_form_reference_tensor(3, 1, None, None) == _lib.FEI_EINVAL


def test_form_compile_rejects_a_null_form():
    lib = _lib.load()
    assert lib.fei_form_compile(None) == _lib.FEI_EINVAL
    assert lib.fei_form_is_compiled(None) == 0
