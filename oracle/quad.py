"""Quadrature rules on the unit tetrahedron and triangle (test infrastructure:
CPU oracle).

Collapsed (Duffy) tensor Gauss-Legendre rules, built from numpy's Gauss-Legendre
nodes.  An n-point rule per direction integrates every polynomial of total
degree <= 2n-3 exactly on the tetrahedron (the collapse adds at most two
degrees in the last direction) and <= 2n-2 on the triangle.

Pins (tests/test_oracle_basis.py): volumes 1/6 and 1/2; exact monomial
integrals a!b!c!/(a+b+c+3)! up to the advertised degree.
"""
from __future__ import annotations

import numpy as np


def gauss01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0


def tet_rule(n: int):
    """Points [N,3] (unit-tet coordinates xi1, xi2, xi3) and weights summing to 1/6."""
    x, w = gauss01(n)
    a, b, c = np.meshgrid(x, x, x, indexing="ij")
    wa, wb, wc = np.meshgrid(w, w, w, indexing="ij")
    xi3 = c
    xi2 = b * (1.0 - c)
    xi1 = a * (1.0 - b) * (1.0 - c)
    wt = wa * wb * wc * (1.0 - b) * (1.0 - c) ** 2
    return np.stack([xi1.ravel(), xi2.ravel(), xi3.ravel()], axis=1), wt.ravel()


def tri_rule(n: int):
    """Points [N,2] on the unit triangle and weights summing to 1/2."""
    x, w = gauss01(n)
    a, b = np.meshgrid(x, x, indexing="ij")
    wa, wb = np.meshgrid(w, w, indexing="ij")
    return np.stack([(a * (1.0 - b)).ravel(), b.ravel()], axis=1), (wa * wb * (1.0 - b)).ravel()
