"""A small form language for bilinear forms of Lagrange elements (the role a
form language plays in Sec. 3.2), compiled by the library (fei_form_create)
into the reference tensor Khat over values and reference derivatives and the
recipe of the geometric tensor G, then integrated on the device by
fei_form_integrate.

A form is written with a test function v and a trial function u of one
element and a few operators; every term is linear in v and in u:

    from paper_1103_0066_amd import forms as F
    el = F.Element(dim=3, degree=1, vector=True)
    u, v = F.TrialFunction(el), F.TestFunction(el)
    mu, lam = F.Coefficient("mu"), F.Coefficient("lam")
    a = 2 * mu * F.inner(F.eps(u), F.eps(v)) + lam * F.div(u) * F.div(v)
    form = F.compile_form(a)                  # Khat + recipe, on the device
    A = form.integrate(coords, conn, {"mu": mu_e, "lam": lam_e})

Operators: the function itself (value), grad, div, eps (= sym grad), sym,
tr, inner, dot, transpose (.T), components ([i]), + - and scalar factors;
per-element constant
coefficients (Coefficient) multiply whole terms (at most one per term).

Lowering: every term becomes sum_{a,b} C[(a,c),(b,d)] D_a v_c D_b u_d with
D_0 the value and D_{1+alpha} = d/dx_alpha; the tables W_k (one per
coefficient, W_0 for the constant part) are what fei_form_create takes.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional

import numpy as np
import torch

from . import _lib

__all__ = ["Element", "TestFunction", "TrialFunction", "Coefficient", "grad", "div", "eps",
           "sym", "tr", "inner", "dot", "compile_form", "Form", "Bilinear"]


class Element:
    """Lagrange element of degree 1 or 2 on a simplex of dimension 2 or 3,
    scalar or vector (dim components)."""

    def __init__(self, dim: int, degree: int = 1, vector: bool = False):
        if dim not in (2, 3) or degree not in (1, 2):
            raise ValueError("dim must be 2 or 3 and degree 1 or 2")
        self.dim, self.degree, self.vector = dim, degree, vector
        self.ncomp = dim if vector else 1

    @property
    def m(self) -> int:
        return (self.dim + 1) * self.ncomp

    def __eq__(self, o):
        return (isinstance(o, Element) and (self.dim, self.degree, self.ncomp) ==
                (o.dim, o.degree, o.ncomp))

    def __hash__(self):
        return hash((self.dim, self.degree, self.ncomp))


class Coefficient:
    """A per-element constant coefficient (one value per element at run time),
    with a numeric factor."""

    def __init__(self, name: str, factor: float = 1.0):
        self.name, self.factor = name, float(factor)

    def __mul__(self, o):
        if isinstance(o, (int, float)):
            return Coefficient(self.name, self.factor * o)
        if isinstance(o, Bilinear):
            return (self.factor * o)._with_coefficient(self.name)
        if isinstance(o, Operand):
            return _Scaled(self.factor * o, self.name)
        return NotImplemented

    __rmul__ = __mul__


class Operand:
    """A tensor (shape () , (d,) or (d, d)) whose entries are linear in one
    argument ('v' test or 'u' trial): entry -> {m index a * ncomp + c: weight}."""

    def __init__(self, arg: str, el: Element, data: np.ndarray, coef: Optional[str] = None):
        self.arg, self.el, self.data, self.coef = arg, el, data, coef

    @property
    def shape(self):
        return self.data.shape

    def _map(self, f) -> "Operand":
        out = np.empty(self.shape, dtype=object)
        for idx in np.ndindex(self.shape):
            out[idx] = f(self.data[idx])
        return Operand(self.arg, self.el, out, self.coef)

    def __add__(self, o):
        if not isinstance(o, Operand) or o.arg != self.arg or o.shape != self.shape:
            raise ValueError("only operands of the same argument and shape add")
        if o.coef != self.coef:
            raise ValueError("attach coefficients after adding operands")
        out = np.empty(self.shape, dtype=object)
        for idx in np.ndindex(self.shape):
            out[idx] = _lin_add(self.data[idx], o.data[idx], 1.0)
        return Operand(self.arg, self.el, out, self.coef)

    def __sub__(self, o):
        return self + (-1.0) * o

    def __neg__(self):
        return (-1.0) * self

    def __mul__(self, o):
        if isinstance(o, (int, float)):
            return self._map(lambda l: {k: float(o) * w for k, w in l.items()})
        if isinstance(o, Operand):
            return _product(self, o)
        return NotImplemented

    __rmul__ = __mul__

    def __getitem__(self, idx):
        sub = self.data[idx]
        return Operand(self.arg, self.el, sub if isinstance(sub, np.ndarray) else _scalar(sub),
                       self.coef)

    @property
    def T(self):
        if len(self.shape) != 2:
            raise ValueError("transpose of a matrix operand only")
        return Operand(self.arg, self.el, self.data.T.copy(), self.coef)


def _lin_add(a: dict, b: dict, s: float) -> dict:
    out = dict(a)
    for k, w in b.items():
        out[k] = out.get(k, 0.0) + s * w
    return out


class _Scaled(Operand):
    def __init__(self, o: Operand, name: str):
        if o.coef is not None:
            raise ValueError("at most one coefficient per term")
        super().__init__(o.arg, o.el, o.data, name)


def _argument(el: Element, arg: str) -> Operand:
    nc = el.ncomp
    if not el.vector:
        d = np.empty((), dtype=object)
        d[()] = {0: 1.0}
    else:
        d = np.empty((nc,), dtype=object)
        for c in range(nc):
            d[c] = {c: 1.0}                   # a = 0 (value), component c
    return Operand(arg, el, d)


def TestFunction(el: Element) -> Operand:
    return _argument(el, "v")


def TrialFunction(el: Element) -> Operand:
    return _argument(el, "u")


def grad(f: Operand) -> Operand:
    """grad of a value operand: scalar -> [d] (d/dx_alpha), vector -> [c][alpha]."""
    el, nc, dim = f.el, f.el.ncomp, f.el.dim
    for l in f.data.flat:
        if any(k // nc != 0 for k in l):
            raise ValueError("grad applies to the function itself (values), not to derivatives")
    out = np.empty(f.shape + (dim,), dtype=object)
    for idx in np.ndindex(f.shape):
        for al in range(dim):
            # value index c -> derivative index (1 + alpha) * nc + c
            out[idx + (al,)] = {(1 + al) * nc + (k % nc): w for k, w in f.data[idx].items()}
    return Operand(f.arg, el, out, f.coef)


def tr(A: Operand) -> Operand:
    if len(A.shape) != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("trace of a square matrix operand only")
    acc = {}
    for i in range(A.shape[0]):
        acc = _lin_add(acc, A.data[i, i], 1.0)
    d = np.empty((), dtype=object)
    d[()] = acc
    return Operand(A.arg, A.el, d, A.coef)


def div(f: Operand) -> Operand:
    if len(f.shape) != 1:
        raise ValueError("div of a vector operand only")
    return tr(grad(f))


def sym(A: Operand) -> Operand:
    return 0.5 * (A + A.T)


def eps(f: Operand) -> Operand:
    """Symmetric gradient (strain) of a vector operand."""
    return sym(grad(f))


class Bilinear:
    """sum over coefficient names (None: constant) of W[name]: m x m tables,
    rows the test operand (a * ncomp + c), columns the trial operand."""

    def __init__(self, el: Element, tables: Dict[Optional[str], np.ndarray]):
        self.el, self.tables = el, tables

    def __add__(self, o):
        if o == 0:
            return self
        if not isinstance(o, Bilinear) or o.el != self.el:
            raise ValueError("forms of one element add")
        t = {k: v.copy() for k, v in self.tables.items()}
        for k, v in o.tables.items():
            t[k] = t.get(k, 0.0) + v
        return Bilinear(self.el, t)

    __radd__ = __add__

    def __sub__(self, o):
        return self + (-1.0) * o

    def __neg__(self):
        return (-1.0) * self

    def __mul__(self, o):
        if isinstance(o, (int, float)):
            return Bilinear(self.el, {k: float(o) * v for k, v in self.tables.items()})
        if isinstance(o, Coefficient):
            return self._with_coefficient(o.name)
        return NotImplemented

    __rmul__ = __mul__

    def _with_coefficient(self, name: str) -> "Bilinear":
        if any(k is not None for k in self.tables):
            raise ValueError("at most one coefficient per term")
        return Bilinear(self.el, {name: self.tables.get(None, 0.0)})


def _product(x: Operand, y: Operand) -> Bilinear:
    if {x.arg, y.arg} != {"u", "v"}:
        raise ValueError("a term multiplies one test and one trial operand")
    if x.el != y.el:
        raise ValueError("test and trial functions of one element")
    if x.shape != () or y.shape != ():
        raise ValueError("multiply scalars; use inner or dot for tensors")
    v, u = (x, y) if x.arg == "v" else (y, x)
    if v.coef is not None and u.coef is not None:
        raise ValueError("at most one coefficient per term")
    name = v.coef if v.coef is not None else u.coef
    W = np.zeros((x.el.m, x.el.m))
    for a, wa in v.data[()].items():
        for b, wb in u.data[()].items():
            W[a, b] += wa * wb
    return Bilinear(x.el, {name: W})


def _scalar(l: dict) -> np.ndarray:
    d = np.empty((), dtype=object)
    d[()] = l
    return d


def inner(x: Operand, y: Operand) -> Bilinear:
    if x.shape != y.shape:
        raise ValueError("inner of operands of one shape")
    total = 0
    for idx in np.ndindex(x.shape):
        xi = Operand(x.arg, x.el, _scalar(x.data[idx]), x.coef)
        yi = Operand(y.arg, y.el, _scalar(y.data[idx]), y.coef)
        total = total + _product(xi, yi)
    return total


def dot(x: Operand, y: Operand) -> Bilinear:
    if len(x.shape) != 1 or len(y.shape) != 1:
        raise ValueError("dot of vector operands; use inner for matrices")
    return inner(x, y)


class Form:
    """A compiled form on the device (fei_form_create): Khat and the recipe."""

    def __init__(self, el: Element, W: np.ndarray, names):
        self.el, self.W, self.names = el, W, list(names)
        lib = _lib.load()
        h = ctypes.c_void_p()
        Wc = np.ascontiguousarray(W, dtype=np.float64)
        _lib.check(lib.fei_form_create(el.dim, el.degree, el.ncomp, len(self.names), Wc.ctypes.data,
                                       ctypes.byref(h)))
        self._h = h
        n, s, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(lib.fei_form_info(h, ctypes.byref(n), ctypes.byref(s), ctypes.byref(k)))
        self.n, self.symmetric = n.value, bool(s.value)

    def integrate(self, coords: torch.Tensor, conn: torch.Tensor,
                  coefficients: Optional[Dict[str, torch.Tensor]] = None, *, tau: float = 100.0,
                  counters: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Element matrices [E, n, n] float32 (fei_form_integrate)."""
        from . import _mesh, _options, _require, _stream
        m = _mesh(coords, conn)
        if m.dim != self.el.dim:
            raise ValueError(f"mesh of dimension {m.dim} for a form of dimension {self.el.dim}")
        dev = coords.device
        E = m.n_elements
        coefficients = coefficients or {}
        missing = [nm for nm in self.names if nm not in coefficients]
        if missing:
            raise ValueError(f"coefficients {missing} not given")
        coef = None
        if self.names:
            for nm in self.names:
                _require(coefficients[nm], nm, torch.float32, dev, (E,))
            coef = torch.stack([coefficients[nm] for nm in self.names]).contiguous()
        if out is None:
            out = torch.empty((E, self.n, self.n), dtype=torch.float32, device=dev)
        else:
            _require(out, "out", torch.float32, dev, (E, self.n, self.n))
        o = _options("fp32", tau, counters)
        _lib.check(_lib.load().fei_form_integrate(
            self._h, ctypes.byref(m), None if coef is None else coef.data_ptr(), out.data_ptr(),
            ctypes.byref(o), _stream(dev)))
        return out

    def compile(self) -> "Form":
        """Generates and compiles a kernel for this form (fei_form_compile: W and
        Khat as constants; cached on disk), used by later integrate() calls."""
        _lib.check(_lib.load().fei_form_compile(self._h))
        return self

    @property
    def compiled(self) -> bool:
        return bool(_lib.load().fei_form_is_compiled(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fei_form_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lower(a: Bilinear):
    """The tables W [n_coef + 1, m, m] (W[0] constant) and the coefficient names."""
    names = sorted(k for k in a.tables if k is not None)
    m = a.el.m
    W = np.zeros((len(names) + 1, m, m))
    if None in a.tables:
        W[0] = a.tables[None]
    for k, nm in enumerate(names):
        W[k + 1] = a.tables[nm]
    return W, names


def compile_form(a: Bilinear) -> Form:
    W, names = lower(a)
    return Form(a.el, W, names)


def reference_tensor(dim: int, degree: int) -> np.ndarray:
    """Khat [nb, nb, dim + 1, dim + 1] (host-only, exact rationals rounded once)."""
    lib = _lib.load()
    n = ctypes.c_int64()
    _lib.check(lib.fei_form_reference_tensor(dim, degree, None, ctypes.byref(n)))
    K = np.zeros(n.value)
    _lib.check(lib.fei_form_reference_tensor(dim, degree, K.ctypes.data, ctypes.byref(n)))
    nb = int(round((n.value / (dim + 1) ** 2) ** 0.5))
    return K.reshape(nb, nb, dim + 1, dim + 1)
