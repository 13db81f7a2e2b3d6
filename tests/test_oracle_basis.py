"""Pins of the oracle's basis and quadrature against closed forms, library
routines and exact identities (no GPU)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import eval_jacobi

from oracle import poly, quad
from oracle.mesh import REF_VERTS, FACE_LOCAL

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_counts_match_paper():
    g = GOLD["basis_counts"]
    for o, b in g["B"].items():
        assert poly.n_basis(int(o)) == b == len(poly.tet_index_list(int(o)))
    for o, f in g["F"].items():
        assert poly.n_face_basis(int(o)) == f == len(poly.tri_index_list(int(o)))
    d = GOLD["derivative_values"]
    assert d["order"] * 9 * poly.n_basis(d["order"]) == d["values"]


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_quadrature_exact_on_monomials(n):
    pts, w = quad.tet_rule(n)
    for a in range(2 * n - 2):
        for b in range(2 * n - 2 - a):
            for c in range(2 * n - 2 - a - b):
                if a + b + c > 2 * n - 3:
                    continue
                exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
                assert abs(got - exact) <= 1e-14 * max(1.0, exact) + 1e-16
    tp, tw = quad.tri_rule(n)
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(tw * tp[:, 0] ** a * tp[:, 1] ** b) - exact) <= 1e-14


@pytest.mark.parametrize("alpha", [0.0, 1.0, 3.0, 6.0])
def test_scaled_jacobi_matches_scipy(alpha):
    D = 7
    x = np.zeros((D,))
    x[1] = 1.0          # the polynomial "t"
    one = np.zeros((D,))
    one[0] = 1.0
    Q = poly.scaled_jacobi(6, alpha, x, one)
    ts = np.linspace(-1, 1, 9)
    for n in range(7):
        got = np.polynomial.polynomial.polyval(ts, Q[n])
        np.testing.assert_allclose(got, eval_jacobi(n, alpha, 0.0, ts), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_tet_basis_orthonormal(order):
    B = poly.Basis(order)
    pts, w = quad.tet_rule(order + 2)
    Phi = B.eval(pts)
    M = Phi.T @ (w[:, None] * Phi)
    np.testing.assert_allclose(M, np.eye(B.nb), atol=1e-13)
    # constant mode: 1/sqrt(volume) = sqrt(6)
    np.testing.assert_allclose(Phi[:, 0], math.sqrt(6.0), rtol=1e-14)


@pytest.mark.parametrize("order", [1, 3, 5])
def test_tri_basis_orthonormal(order):
    F = poly.FaceBasis(order)
    pts, w = quad.tri_rule(order + 2)
    Phi = F.eval(pts)
    np.testing.assert_allclose(Phi.T @ (w[:, None] * Phi), np.eye(F.nf), atol=1e-13)


def test_basis_degrees_hierarchical():
    # the first B(p) functions span all polynomials of degree < p: a random
    # polynomial of degree p-1 is reproduced exactly by projection onto them
    rng = np.random.default_rng(0)
    order = 5
    B = poly.Basis(order)
    pts, w = quad.tet_rule(order + 2)
    for p in range(1, order + 1):
        coef = rng.normal(size=(p, p, p))
        f = lambda x: sum(coef[a, b, c] * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c
                          for a in range(p) for b in range(p) for c in range(p) if a + b + c < p)
        nb = poly.n_basis(p)
        Phi = B.eval(pts)[:, :nb]
        proj = Phi.T @ (w * f(pts))
        test = rng.uniform(0, 0.3, size=(20, 3))
        np.testing.assert_allclose(B.eval(test)[:, :nb] @ proj, f(test), rtol=1e-10, atol=1e-10)


def test_gradients_match_finite_differences():
    B = poly.Basis(4)
    x = np.array([[0.1, 0.2, 0.3], [0.25, 0.05, 0.4]])
    g = B.grad(x)
    h = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (B.eval(x + e) - B.eval(x - e)) / (2 * h)
        np.testing.assert_allclose(g[c], fd, atol=1e-6)


@pytest.mark.parametrize("order", [2, 5])
def test_integration_by_parts_identity(order):
    # int d_c(phi_a) phi_b + int phi_a d_c(phi_b) = sum_faces n_c int_face phi_a phi_b
    B = poly.Basis(order)
    pts, w = quad.tet_rule(order + 2)
    Phi, dPhi = B.eval(pts), B.grad(pts)
    fpts, fw = quad.tri_rule(order + 2)
    bary = np.stack([1 - fpts.sum(1), fpts[:, 0], fpts[:, 1]], axis=1)
    for c in range(3):
        S = dPhi[c].T @ (w[:, None] * Phi)
        rhs = np.zeros_like(S)
        for i in range(4):
            V = REF_VERTS[FACE_LOCAL[i]]
            cr = np.cross(V[1] - V[0], V[2] - V[0])
            area2 = np.linalg.norm(cr)             # 2 * face area
            n = cr / area2
            if np.dot(n, REF_VERTS[i] - V[0]) > 0:
                n = -n
            P = B.eval(bary @ V)
            rhs += n[c] * area2 * (P.T @ (fw[:, None] * P))
        np.testing.assert_allclose(S + S.T, rhs, atol=1e-12)
