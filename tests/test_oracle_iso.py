"""Pins of the oracle's isoparametric P2 Laplacian (Sec. 3.1, eqs. 16-19) on
elements with quadratic geometry: the affine special case, symmetry and the
constants in the kernel, invariance under rigid motions and the scaling law,
exactness of the quadrature for the projected integrand, convergence of the
paper's projected scheme to the isoparametric integral as the curvature goes
to zero, and an independent route to the projected scheme through the
arity-4 reference tensor K^{ijkl}_{mu nu} of eq. 18, integrated exactly."""
import math
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import meshgen
import oracle


def _curved(dim, amp, seed=5):
    base = (meshgen.square_mesh(3, 0.2, seed, np.float64) if dim == 2
            else meshgen.cube_mesh(2, 2, 2, 0.15, seed, np.float64))
    return meshgen.p2_mesh(base, amp)


@pytest.mark.parametrize("dim", [2, 3])
def test_straight_geometry_is_the_affine_p2_laplacian(dim):
    base = (meshgen.square_mesh(4, 0.2, 81, np.float64) if dim == 2
            else meshgen.cube_mesh(2, 2, 2, 0.15, 82, np.float64))
    m = meshgen.p2_mesh(base, 0.0)
    Ap = oracle.integrate("laplace_p2", base.coords, base.conn)
    for mode in ("projected", "exact"):
        A = oracle.integrate_iso(m.coords, m.conn, mode)
        np.testing.assert_allclose(A, Ap, rtol=0, atol=1e-13 * np.abs(Ap).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_symmetry_and_constants_in_the_kernel(dim):
    m = _curved(dim, 0.05)
    for mode in ("projected", "exact"):
        A = oracle.integrate_iso(m.coords, m.conn, mode)
        np.testing.assert_allclose(A, A.transpose(0, 2, 1), rtol=0, atol=1e-15 * np.abs(A).max())
        assert np.abs(A.sum(axis=2)).max() <= 1e-14 * np.abs(A).max()
        assert (np.einsum("eii->ei", A) > 0).all()


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_motions_and_scaling(dim):
    """A(Qx + t) = A(x) and A(alpha x) = alpha^(d-2) A(x) for the projected
    scheme on curved elements (J -> Q J, J^-1 -> J^-1 Q^T, |J| unchanged)."""
    m = _curved(dim, 0.05)
    A = oracle.integrate_iso(m.coords, m.conn)
    rng = np.random.default_rng(83)
    Q, _ = np.linalg.qr(rng.normal(size=(dim, dim)))
    X = m.coords @ Q.T + rng.normal(size=dim)
    np.testing.assert_allclose(oracle.integrate_iso(X, m.conn), A, rtol=0,
                               atol=1e-13 * np.abs(A).max())
    np.testing.assert_allclose(oracle.integrate_iso(2.5 * m.coords, m.conn), 2.5 ** (dim - 2) * A,
                               rtol=0, atol=1e-13 * np.abs(A).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_projected_integrand_is_integrated_exactly(dim):
    """The projected integrand is a polynomial of degree 4: rules of degree 5
    and 7 agree to rounding."""
    m = _curved(dim, 0.05)
    A5 = oracle.integrate_iso(m.coords, m.conn, qs=2)
    A7 = oracle.integrate_iso(m.coords, m.conn, qs=3)
    np.testing.assert_allclose(A5, A7, rtol=0, atol=1e-14 * np.abs(A7).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_projected_scheme_converges_to_the_isoparametric_integral(dim):
    """Halving the curvature at least halves (to within 20 %) the distance
    between the paper's projected scheme and the isoparametric integral (J
    at every point, a rule of degree 9), which vanishes for straight edges."""
    errs = []
    for amp in (0.04, 0.02, 0.01):
        m = _curved(dim, amp)
        A0 = oracle.integrate_iso(m.coords, m.conn)
        A1 = oracle.integrate_iso(m.coords, m.conn, "exact", qs=4)
        errs.append(np.abs(A0 - A1).max() / np.abs(A1).max())
    assert errs[0] < 0.1
    assert errs[1] <= 0.6 * errs[0] and errs[2] <= 0.6 * errs[1], errs


# ---- the arity-4 reference tensor of eq. 18, exactly ---------------------------

def _p2_grad_polys(dim):
    """dphi_i/dxi_mu of the P2 basis as barycentric polynomials {exponents: Fraction}."""
    nv = dim + 1

    def mono(*idx):
        e = [0] * nv
        for k in idx:
            e[k] += 1
        return tuple(e)
    B = [{mono(a, a): Fraction(2), mono(a): Fraction(-1)} for a in range(nv)]
    B += [{mono(a, b): Fraction(4)} for a in range(nv) for b in range(a + 1, nv)]

    def dxi(p, mu):
        out = {}
        for e, c in p.items():
            for k, sgn in ((mu + 1, 1), (0, -1)):
                if e[k]:
                    f = list(e)
                    f[k] -= 1
                    out[tuple(f)] = out.get(tuple(f), 0) + sgn * e[k] * c
        return out
    return [[dxi(b, mu) for mu in range(dim)] for b in B], mono


def _times_lambda(p, k, nv):
    out = {}
    for e, c in p.items():
        f = list(e)
        f[k] += 1
        out[tuple(f)] = out.get(tuple(f), 0) + c
    return out


def _integ(p, q, dim):
    tot = Fraction(0)
    for ea, ca in p.items():
        for eb, cb in q.items():
            al = [x + y for x, y in zip(ea, eb)]
            tot += ca * cb * Fraction(math.prod(math.factorial(x) for x in al),
                                      math.factorial(sum(al) + dim))
    return tot


def _k4(dim):
    """K^{ijkl}_{mu nu} = int_ref lambda_k dphi_i/dxi_mu lambda_l dphi_j/dxi_nu (eq. 18,
    with the inverse Jacobian projected on the P1 basis lambda_k)."""
    D, _ = _p2_grad_polys(dim)
    nb, nv = len(D), dim + 1
    P = {(i, mu, k): _times_lambda(D[i][mu], k, nv)
         for i in range(nb) for mu in range(dim) for k in range(nv)}
    K = np.zeros((nb, nb, nv, nv, dim, dim))
    for (i, mu, k), p in P.items():
        for (j, nu, l), q in P.items():
            if (j, nu, l) < (i, mu, k):
                continue
            K[i, j, k, l, mu, nu] = K[j, i, l, k, nu, mu] = float(_integ(p, q, dim))
    return K


@pytest.mark.parametrize("dim", [2, 3])
def test_projected_scheme_equals_the_contraction_of_eq_19(dim):
    """A_ij = G^{mu nu}_{kl} K^{ijkl}_{mu nu} with G^{mu nu}_{kl} = J^-1_{mu alpha,k}
    J^-1_{nu alpha,l} |J| (eqs. 18-19): the exact tensor contracted here in
    numpy equals the oracle's quadrature of the projected integrand."""
    K = _k4(dim)
    m = _curved(dim, 0.05)
    A = oracle.integrate_iso(m.coords, m.conn)
    nv = dim + 1
    pairs = [(a, b) for a in range(nv) for b in range(a + 1, nv)]
    gl = np.vstack([-np.ones(dim), np.eye(dim)])

    def jac(xn, bc):
        g = [(4 * bc[k] - 1) * gl[k] for k in range(nv)]
        g += [4 * (bc[a] * gl[b] + bc[b] * gl[a]) for a, b in pairs]
        return xn.T @ np.array(g)                       # J[alpha][mu]
    for e in range(m.n_elements):
        xn = m.coords[m.conn[e]].astype(np.float64)
        Bk = [np.linalg.inv(jac(xn, np.eye(nv)[k])) for k in range(nv)]    # [mu][alpha]
        s = abs(np.linalg.det(jac(xn, np.full(nv, 1.0 / nv))))
        G = np.einsum("kma,lna->klmn", np.array(Bk), np.array(Bk)) * s
        Ae = np.einsum("ijklmn,klmn->ij", K, G)
        np.testing.assert_allclose(Ae, A[e], rtol=0, atol=1e-13 * np.abs(A[e]).max())
