"""Orthonormal modal bases on the unit tetrahedron and unit triangle (test
infrastructure: CPU oracle).

Sec. III-A (Discrete Formulation) takes the element basis from the tetrahedral
expansion of Karniadakis & Sherwin, with B(O) = O(O+1)(O+2)/6 functions
(B(4)=20, B(5)=35) and a diagonal mass matrix; faces use F(O) = O(O+1)/2
triangular functions (F(5)=15).  Here each basis function is built *exactly*
as a polynomial in monomial coefficients by running the scaled Jacobi
recurrences with polynomial arithmetic, and is normalised with the exact
monomial integrals over the simplex.  Values and derivatives then follow from
the monomial representation.

Reading of the paper (it does not fix these): unit reference tetrahedron
(0,0,0),(1,0,0),(0,1,0),(0,0,1); functions orthonormal on it (so the physical
mass matrix is |det J| * I, diagonal as the paper requires); ordering by total
degree n ascending, then i descending, then j descending (k = n-i-j).

Pins (tests/test_oracle_basis.py): mass matrix = identity; counts B(O), F(O);
scaled Jacobi against scipy.special.eval_jacobi; the constant mode equals
sqrt(6); derivative exactness against finite differences; the integration by
parts identity on the reference tetrahedron.
"""
from __future__ import annotations

import math
import numpy as np


def n_basis(order: int) -> int:
    return order * (order + 1) * (order + 2) // 6


def n_face_basis(order: int) -> int:
    return order * (order + 1) // 2


def tet_index_list(order: int):
    out = []
    for n in range(order):
        for i in range(n, -1, -1):
            for j in range(n - i, -1, -1):
                out.append((i, j, n - i - j))
    return out


def tri_index_list(order: int):
    out = []
    for n in range(order):
        for i in range(n, -1, -1):
            out.append((i, n - i))
    return out


# ------------------------------------------------------------ dense polynomials
# A polynomial in d variables of degree < D per variable is an array of shape
# (D,)*d holding monomial coefficients: P[a,b,c] multiplies u^a v^b w^c.

def _pmul(p, q):
    D = p.shape[0]
    out = np.zeros_like(p)
    for idx in zip(*np.nonzero(p)):
        c = p[idx]
        sl_dst = tuple(slice(i, D) for i in idx)
        sl_src = tuple(slice(0, D - i) for i in idx)
        out[sl_dst] += c * q[sl_src]
        # terms pushed past degree D-1 are dropped; callers only form products
        # whose true degree stays below D (checked by _check_trunc)
    return out


def _check_trunc(p, q, prod):
    # total-degree bookkeeping: deg(p)+deg(q) must fit in the array
    def deg(x):
        nz = np.nonzero(x)
        return max((sum(t) for t in zip(*nz)), default=0)
    assert deg(p) + deg(q) < p.shape[0], "polynomial product overflowed its degree"
    return prod


def pmul(p, q):
    return _check_trunc(p, q, _pmul(p, q))


def _const(D, d, c=1.0):
    p = np.zeros((D,) * d)
    p[(0,) * d] = c
    return p


def _var(D, d, axis):
    p = np.zeros((D,) * d)
    idx = [0] * d
    idx[axis] = 1
    p[tuple(idx)] = 1.0
    return p


def scaled_jacobi(nmax: int, alpha: float, x, y):
    """[Q_0..Q_nmax] with Q_n(x, y) = y^n P_n^{(alpha,0)}(x / y) as polynomials
    (x, y are polynomials themselves).  Three-term Jacobi recurrence with beta=0,
    multiplied through by y^n."""
    D, d = x.shape[0], x.ndim
    Q = [_const(D, d)]
    if nmax >= 1:
        Q.append(((alpha + 2.0) * x + alpha * y) / 2.0)
    a, b = alpha, 0.0
    for n in range(2, nmax + 1):
        c1 = 2.0 * n * (n + a + b) * (2 * n + a + b - 2)
        c2 = (2 * n + a + b - 1) * (2 * n + a + b) * (2 * n + a + b - 2)
        c3 = (2 * n + a + b - 1) * (a * a - b * b)
        c4 = 2.0 * (n + a - 1) * (n + b - 1) * (2 * n + a + b)
        Q.append((pmul(c2 * x + c3 * y, Q[n - 1]) - c4 * pmul(pmul(y, y), Q[n - 2])) / c1)
    return Q


def _simplex_monomial_integrals(D, d):
    """I[a,b,(c)] = integral of the monomial over the unit simplex in d dims:
    a! b! c! / (a+b+c+d)!"""
    I = np.zeros((D,) * d)
    for idx in np.ndindex(*I.shape):
        I[idx] = math.prod(math.factorial(i) for i in idx) / math.factorial(sum(idx) + d)
    return I


def integrate(p):
    return float(np.sum(p * _simplex_monomial_integrals(p.shape[0], p.ndim)))


def inner(p, q):
    """Exact integral of p*q over the unit simplex (the product may exceed the
    arrays' degree, so it is summed monomial pair by monomial pair)."""
    d = p.ndim
    tot = 0.0
    for ia in zip(*np.nonzero(p)):
        for ib in zip(*np.nonzero(q)):
            e = [a + b for a, b in zip(ia, ib)]
            tot += p[ia] * q[ib] * math.prod(math.factorial(x) for x in e) / math.factorial(sum(e) + d)
    return tot


def tet_basis_polys(order: int):
    """List of B(order) polynomials (arrays (O,O,O)) of the orthonormal
    tetrahedral basis on the unit tetrahedron, in the documented order."""
    D, d = max(order, 2), 3
    u, v, w = (_var(D, d, a) for a in range(3))
    one = _const(D, d)
    y1 = one - v - w
    x1 = 2.0 * u - y1
    y2 = one - w
    x2 = 2.0 * v - y2
    z3 = 2.0 * w - one
    polys = []
    for (i, j, k) in tet_index_list(order):
        qi = scaled_jacobi(i, 0.0, x1, y1)[i]
        qj = scaled_jacobi(j, 2.0 * i + 1.0, x2, y2)[j]
        pk = scaled_jacobi(k, 2.0 * i + 2.0 * j + 2.0, z3, one)[k]
        p = pmul(pmul(qi, qj), pk)
        p /= math.sqrt(inner(p, p))
        polys.append(p[:order, :order, :order].copy())
    return polys


def tri_basis_polys(order: int):
    """List of F(order) polynomials (arrays (O,O)) of the orthonormal triangle
    basis on the unit triangle (0,0),(1,0),(0,1)."""
    D, d = max(order, 2), 2
    a, b = _var(D, d, 0), _var(D, d, 1)
    one = _const(D, d)
    y1 = one - b
    x1 = 2.0 * a - y1
    z2 = 2.0 * b - one
    polys = []
    for (i, j) in tri_index_list(order):
        qi = scaled_jacobi(i, 0.0, x1, y1)[i]
        pj = scaled_jacobi(j, 2.0 * i + 1.0, z2, one)[j]
        p = pmul(qi, pj)
        p /= math.sqrt(inner(p, p))
        polys.append(p[:order, :order].copy())
    return polys


# ------------------------------------------------------------ evaluation

def _monomials(pts, D):
    """pts [N,d] -> M [N, D^d] monomial values in C order of the coefficient array."""
    pts = np.asarray(pts, dtype=np.float64)
    N, d = pts.shape
    pw = pts[:, :, None] ** np.arange(D)[None, None, :]  # [N,d,D]
    M = pw[:, 0, :]
    for ax in range(1, d):
        M = (M[:, :, None] * pw[:, ax, None, :]).reshape(N, -1)
    return M


def _deriv(p, axis):
    D = p.shape[0]
    out = np.zeros_like(p)
    sl_dst = [slice(None)] * p.ndim
    sl_src = [slice(None)] * p.ndim
    sl_dst[axis] = slice(0, D - 1)
    sl_src[axis] = slice(1, D)
    shape = [1] * p.ndim
    shape[axis] = D - 1
    out[tuple(sl_dst)] = p[tuple(sl_src)] * np.arange(1, D).reshape(shape)
    return out


class Basis:
    """Values and reference gradients of the tetrahedral basis at points."""

    def __init__(self, order: int):
        self.order = order
        self.nb = n_basis(order)
        self.polys = tet_basis_polys(order)
        self.C = np.stack([p.ravel() for p in self.polys], axis=1)  # [D^3, B]
        self.dC = [np.stack([_deriv(p, a).ravel() for p in self.polys], axis=1) for a in range(3)]

    def eval(self, pts):
        return _monomials(pts, self.order) @ self.C  # [N,B]

    def grad(self, pts):
        M = _monomials(pts, self.order)
        return np.stack([M @ dc for dc in self.dC], axis=0)  # [3,N,B]


class FaceBasis:
    def __init__(self, order: int):
        self.order = order
        self.nf = n_face_basis(order)
        self.polys = tri_basis_polys(order)
        self.C = np.stack([p.ravel() for p in self.polys], axis=1)

    def eval(self, pts):
        return _monomials(pts, self.order) @ self.C
