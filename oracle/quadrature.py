"""Quadrature rules for the oracle (FP64).

The paper states only that its code contains the quadrature (implementation
paragraph of its numerical-tests section).  The oracle integrates with
Gauss-Legendre on segments and the collapsed (Duffy) Gauss-Jacobi conical
product on triangles; nodes and weights come from scipy's Jacobi root finder,
a library primitive.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi, roots_legendre


def segment_rule(k: int):
    """k-point Gauss-Legendre on [0, 1]: exact for degree 2k-1."""
    x, w = roots_legendre(k)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(k: int):
    """Collapsed Gauss-Jacobi rule on {xi, eta >= 0, xi + eta <= 1}.

    xi = (1+a)(1-b)/4, eta = (1+b)/2 maps [-1,1]^2 onto the triangle with
    Jacobian (1-b)/8; Gauss-Legendre in a, Gauss-Jacobi with weight (1-b) in b.
    Exact for total degree 2k-1.  Returns (xi, eta, w), each of length k*k.
    """
    a, wa = roots_legendre(k)
    b, wb = roots_jacobi(k, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    xi = (1.0 + A) * (1.0 - B) / 4.0
    eta = (1.0 + B) / 2.0
    w = WA * WB / 8.0
    return xi.ravel(), eta.ravel(), w.ravel()


def map_to_triangle(corners, xi, eta, w):
    """Push a reference rule onto the physical triangle with the given corners."""
    c0, c1, c2 = (np.asarray(c, float) for c in corners)
    e1 = c1 - c0
    e2 = c2 - c0
    det = abs(e1[0] * e2[1] - e1[1] * e2[0])
    x = c0[0] + xi * e1[0] + eta * e2[0]
    y = c0[1] + xi * e1[1] + eta * e2[1]
    return x, y, w * det
