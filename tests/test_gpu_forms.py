"""Forms from the form front end on the GPU (fei_form_integrate) against the
oracle's direct quadrature of the same tables (oracle.integrate_general),
element by element at the FP32 bound: scalar and vector P1/P2 forms in 2D and
3D, symmetric and not, with per-element coefficients, near-degenerate
elements, ragged sizes; and the elasticity form against the library's
specialized elasticity kernel."""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import TOL, element_errors, mesh_to_device, vec_to_device

pytestmark = pytest.mark.gpu

fei = pytest.importorskip("paper_1103_0066_amd")
from paper_1103_0066_amd import forms as F  # noqa: E402


def _mesh(dim, seed, flat=0):
    m = (meshgen.square_mesh(9, 0.2, seed, np.float32) if dim == 2
         else meshgen.cube_mesh(5, 4, 4, 0.15, seed))
    return meshgen.flatten_elements(m, flat, seed + 1) if flat else m


def _forms(dim, degree):
    """(name, bilinear form) pairs of one element family."""
    out = []
    el = F.Element(dim, degree)
    u, v = F.TrialFunction(el), F.TestFunction(el)
    k = F.Coefficient("k")
    out.append(("laplace", F.inner(F.grad(u), F.grad(v))))
    out.append(("mass", u * v))
    out.append(("diffusion_reaction_advection",
                k * F.inner(F.grad(u), F.grad(v)) + 0.3 * u * v + 0.5 * (F.grad(u)[0] * v)))
    ev = F.Element(dim, degree, vector=True)
    u, v = F.TrialFunction(ev), F.TestFunction(ev)
    mu, lam = F.Coefficient("mu"), F.Coefficient("lam")
    out.append(("elasticity", 2 * mu * F.inner(F.eps(u), F.eps(v)) + lam * F.div(u) * F.div(v)))
    out.append(("vector_mass_coupled", lam * F.dot(u, v) + F.grad(u)[0, 1] * v[dim - 1]))
    return out


CASES = [(dim, degree, name) for dim in (2, 3) for degree in (1, 2)
         for name, _ in _forms(2, 1)]


@pytest.mark.parametrize("dim,degree,name", CASES)
def test_form_matches_oracle(dim, degree, name):
    a = dict(_forms(dim, degree))[name]
    form = F.compile_form(a)
    m = _mesh(dim, 300 + 10 * dim + degree, flat=4 if dim == 3 else 0)
    rng = np.random.Generator(np.random.PCG64(17))
    cf = {nm: np.exp(0.5 * rng.standard_normal(m.n_elements)).astype(np.float32)
          for nm in form.names}
    print(f"[form] {name} dim={dim} P{degree} E={m.n_elements} sym={form.symmetric}", flush=True)
    coords, conn = mesh_to_device(m)
    A = form.integrate(coords, conn, {k: vec_to_device(v) for k, v in cf.items()}).cpu().numpy()
    W, names = F.lower(a)
    Ao = oracle.integrate_general(degree, a.el.ncomp, W, m.coords, m.conn,
                                  np.stack([cf[nm] for nm in names]) if names else ())
    err = element_errors(A, Ao)
    print(f"  max element error {err.max():.2e}")
    assert err.max() <= TOL["fp32"]


def test_form_ragged_sizes_and_counters():
    """E = 0, 1 and ragged tails of a vector P2 form (staged in row chunks);
    the FP64-path counter counts every flattened element."""
    a = dict(_forms(3, 2))["elasticity"]
    form = F.compile_form(a)
    m = _mesh(3, 331, flat=20)
    mu, lam = meshgen.lame(m.n_elements, 332)
    for E in (0, 1, 63, 65, 257, m.n_elements):
        sub = meshgen.Mesh(m.coords, np.ascontiguousarray(m.conn[:E]))
        coords, conn = mesh_to_device(sub)
        out = torch.full((E, form.n, form.n), float("nan"), device="cuda")
        cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
        A = form.integrate(coords, conn, {"lam": vec_to_device(lam[:E]), "mu": vec_to_device(mu[:E])},
                           out=out, counters=cnt).cpu().numpy()
        if E == 0:
            continue
        W, names = F.lower(a)
        Ao = oracle.integrate_general(2, 3, W, m.coords, sub.conn, np.stack([lam[:E], mu[:E]]))
        assert element_errors(A, Ao).max() <= TOL["fp32"], E
        assert cnt.cpu().tolist() == [int(np.sum(m.flattened < E)), 0], E


def test_form_elasticity_equals_specialized_kernel():
    """The 3D P1 elasticity form from the front end against fei_integrate's
    elasticity kernel on the flattened cube (two routes to the same matrices)."""
    a = dict(_forms(3, 1))["elasticity"]
    form = F.compile_form(a)
    m = meshgen.flatten_elements(meshgen.cube_mesh(12, 10, 9, 0.15, 341), 60, 342)
    mu, lam = meshgen.lame(m.n_elements, 343)
    coords, conn = mesh_to_device(m)
    mu_d, lam_d = vec_to_device(mu), vec_to_device(lam)
    A1 = form.integrate(coords, conn, {"mu": mu_d, "lam": lam_d}).cpu().numpy()
    A2 = fei.integrate(coords, conn, "elastic_p1", mu_d, lam_d).cpu().numpy().astype(np.float64)
    assert element_errors(A1, A2).max() <= 2e-6


def test_form_rejects_bad_calls():
    a = dict(_forms(3, 1))["elasticity"]
    form = F.compile_form(a)
    m = _mesh(3, 351)
    coords, conn = mesh_to_device(m)
    with pytest.raises(ValueError):
        form.integrate(coords, conn, {"mu": vec_to_device(np.ones(m.n_elements, np.float32))})
    m2 = _mesh(2, 352)
    c2, k2 = mesh_to_device(m2)
    ones = vec_to_device(np.ones(m2.n_elements, np.float32))
    with pytest.raises(ValueError):
        form.integrate(c2, k2, {"mu": ones, "lam": ones})


# ---------------------------------------------------------------------------
# forms with a kernel of their own (fei_form_compile)
# ---------------------------------------------------------------------------

COMPILED = [(3, 1, "elasticity"), (2, 2, "diffusion_reaction_advection"),
            (3, 1, "vector_mass_coupled"), (3, 2, "laplace")]


@pytest.mark.parametrize("dim,degree,name", COMPILED)
def test_compiled_form_matches_generic_and_oracle(dim, degree, name, tmp_path, monkeypatch):
    """The generated kernel (W and Khat as constants, zero terms dropped) gives
    the generic kernel's results up to the sign of zero, and the oracle's at
    the FP32 bound; ragged sizes included."""
    monkeypatch.setenv("FEI_JIT_DIR", str(tmp_path))
    a = dict(_forms(dim, degree))[name]
    generic = F.compile_form(a)
    compiled = F.compile_form(a).compile()
    assert compiled.compiled and not generic.compiled
    m = _mesh(dim, 350 + 10 * dim + degree, flat=4 if dim == 3 else 0)
    rng = np.random.Generator(np.random.PCG64(19))
    cf = {nm: np.exp(0.5 * rng.standard_normal(m.n_elements)).astype(np.float32)
          for nm in generic.names}
    print(f"[compiled form] {name} dim={dim} P{degree} E={m.n_elements}", flush=True)
    W, names = F.lower(a)
    Ao = oracle.integrate_general(degree, a.el.ncomp, W, m.coords, m.conn,
                                  np.stack([cf[nm] for nm in names]) if names else ())
    for E in sorted({min(x, m.n_elements) for x in (1, 63, 257, m.n_elements)}):
        sub = meshgen.Mesh(m.coords, np.ascontiguousarray(m.conn[:E]))
        coords, conn = mesh_to_device(sub)
        c = {k: vec_to_device(v[:E]) for k, v in cf.items()}
        out = torch.full((E, compiled.n, compiled.n), float("nan"), device="cuda")
        Ac = compiled.integrate(coords, conn, c, out=out).cpu().numpy()
        Ag = generic.integrate(coords, conn, c).cpu().numpy()
        assert np.array_equal(np.abs(Ac), np.abs(Ag)), (E, float(np.abs(Ac - Ag).max()))
        assert element_errors(Ac, Ao[:E]).max() <= TOL["fp32"]


def test_compiled_form_is_cached(tmp_path, monkeypatch):
    """A form compiled once is loaded from the cache by the next form object
    with the same tables (one code object on disk)."""
    import time
    monkeypatch.setenv("FEI_JIT_DIR", str(tmp_path))
    a = dict(_forms(2, 1))["laplace"]
    F.compile_form(a).compile()
    objs = sorted(p.name for p in tmp_path.iterdir())
    assert len(objs) == 1 and objs[0].endswith(".co"), objs
    t0 = time.perf_counter()
    f2 = F.compile_form(a).compile()
    assert f2.compiled and time.perf_counter() - t0 < 2.0
    assert sorted(p.name for p in tmp_path.iterdir()) == objs
