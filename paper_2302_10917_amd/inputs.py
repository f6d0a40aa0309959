"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module holds only input data: macro meshes (vertex coordinates and
connectivity), refinement levels, coefficient fields, random trace vectors and
the closed-form manufactured solutions whose samples are fed to the solver.
It contains none of the discretisation's arithmetic (no basis, quadrature,
assembly or solve), so that it can serve both the GPU path and the independent
CPU oracle without coupling them.

Mesh convention (structured unit square, the paper's N = d! n^d macro count of
its complexity section with d = 2): vertex (i, j) sits at (i/n, j/n) with index
j*(n+1)+i; square (i, j) is cut along the diagonal (i,j)-(i+1,j+1) into a lower
triangle [(i,j), (i+1,j), (i+1,j+1)] and an upper triangle [(i,j), (i+1,j+1),
(i,j+1)], both counter-clockwise.  Square (i, j) contributes triangles
2*(j*n+i) (lower) and 2*(j*n+i)+1 (upper).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable

import numpy as np


# --------------------------------------------------------------------------
# macro meshes
# --------------------------------------------------------------------------
def structured_mesh(n: int, jitter: float = 0.0, seed: int | None = None):
    """Unit square split into n x n squares, each cut into two triangles.

    jitter > 0 moves every interior vertex by U(-jitter/n, jitter/n) in each
    coordinate (seeded); jitter <= 0.15 keeps all triangles counter-clockwise.
    Returns (xy float64 [(n+1)^2, 2], tri int32 [2 n^2, 3]).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    xy = np.stack([ii.ravel() / n, jj.ravel() / n], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        interior = ((ii.ravel() > 0) & (ii.ravel() < n) &
                    (jj.ravel() > 0) & (jj.ravel() < n))
        d = rng.uniform(-jitter / n, jitter / n, size=(xy.shape[0], 2))
        xy[interior] += d[interior]
    tri = np.empty((2 * n * n, 3), dtype=np.int32)
    for j in range(n):
        for i in range(n):
            v00 = j * (n + 1) + i
            v10 = v00 + 1
            v01 = v00 + (n + 1)
            v11 = v01 + 1
            s = j * n + i
            tri[2 * s] = (v00, v10, v11)
            tri[2 * s + 1] = (v00, v11, v01)
    return xy, tri


def two_macro_mesh():
    """Two triangles sharing one edge (the layout of the paper's worked example
    in its matrix-free methodology section)."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return xy, tri


def random_levels(n_macro: int, choices=(1, 2, 3, 4), seed: int = 3):
    """Per-macro refinement level r drawn uniformly from `choices` (seeded)."""
    rng = np.random.default_rng(seed)
    return rng.choice(np.asarray(choices, dtype=np.int32), size=n_macro).astype(np.int32)


def lognormal_kappa(n_macro: int, sigma: float = 0.5, seed: int = 5):
    """kappa_K = exp(sigma * xi_K), xi ~ N(0, 1) (seeded)."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal(n_macro))


def coefficient_instances(n_inst: int, seed: int = 33):
    """Coefficient instances: kappa log-uniform in [1e-3, 1], beta with a
    uniform random direction and magnitude uniform in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    kappa = 10.0 ** rng.uniform(-3.0, 0.0, size=n_inst)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n_inst)
    s = rng.uniform(0.5, 2.0, size=n_inst)
    beta = np.stack([s * np.cos(theta), s * np.sin(theta)], axis=1)
    return kappa, beta


def random_vector(n: int, seed: int = 1):
    """Standard normal vector (seeded), e.g. a trace vector for apply tests."""
    return np.random.default_rng(seed).standard_normal(n)


# --------------------------------------------------------------------------
# manufactured solutions: u, q = -grad u, f = div(beta u) - kappa lap u
# (beta constant, so f = beta . grad u - kappa lap u)
# --------------------------------------------------------------------------
@dataclass
class Manufactured:
    u: Callable
    q: Callable          # returns (qx, qy)
    f: Callable
    name: str


def sin_sin(kappa: float, beta):
    """u = sin(pi x) sin(pi y): homogeneous Dirichlet data on the unit square."""
    bx, by = float(beta[0]), float(beta[1])
    pi = math.pi

    def u(x, y):
        return np.sin(pi * x) * np.sin(pi * y)

    def q(x, y):
        return (-pi * np.cos(pi * x) * np.sin(pi * y),
                -pi * np.sin(pi * x) * np.cos(pi * y))

    def f(x, y):
        return (2 * pi * pi * kappa * np.sin(pi * x) * np.sin(pi * y)
                + pi * (bx * np.cos(pi * x) * np.sin(pi * y)
                        + by * np.sin(pi * x) * np.cos(pi * y)))

    return Manufactured(u, q, f, "sin_sin")


def exp_sin(kappa: float, beta):
    """u = exp(x) sin(2 pi y)."""
    bx, by = float(beta[0]), float(beta[1])
    tp = 2 * math.pi

    def u(x, y):
        return np.exp(x) * np.sin(tp * y)

    def q(x, y):
        return (-np.exp(x) * np.sin(tp * y), -tp * np.exp(x) * np.cos(tp * y))

    def f(x, y):
        return np.exp(x) * ((kappa * (tp * tp - 1.0) + bx) * np.sin(tp * y)
                            + tp * by * np.cos(tp * y))

    return Manufactured(u, q, f, "exp_sin")


def tanh_layer(kappa: float, beta):
    """u = (1 + tanh((y - 2x + 0.4)/kappa)) / 2, the 2D internal-layer
    benchmark of the paper's accuracy section; f includes beta . grad u."""
    bx, by = float(beta[0]), float(beta[1])

    def s(x, y):
        return (y - 2 * x + 0.4) / kappa

    def u(x, y):
        return 0.5 * (1.0 + np.tanh(s(x, y)))

    def q(x, y):
        sech2 = 1.0 / np.cosh(s(x, y)) ** 2
        return (sech2 / kappa, -0.5 * sech2 / kappa)

    def f(x, y):
        t = np.tanh(s(x, y))
        sech2 = 1.0 / np.cosh(s(x, y)) ** 2
        # lap u = (5 / kappa^2) * (-sech^2 tanh); grad u = sech^2/(2 kappa) * (-2, 1)
        lap = -5.0 * sech2 * t / kappa ** 2
        adv = (by - 2 * bx) * sech2 / (2 * kappa)
        return -kappa * lap + adv

    return Manufactured(u, q, f, "tanh_layer")


def polynomial(p: int, kappa: float, beta, seed: int = 0):
    """A random polynomial u of total degree p (seeded coefficients)."""
    rng = np.random.default_rng(seed)
    exps = [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]
    c = rng.standard_normal(len(exps))
    bx, by = float(beta[0]), float(beta[1])

    def _pw(x, e):
        return x ** e if e > 0 else np.ones_like(x)

    def u(x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        return sum(ci * _pw(x, a) * _pw(y, b) for ci, (a, b) in zip(c, exps))

    def ux(x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        return sum(ci * a * _pw(x, a - 1) * _pw(y, b)
                   for ci, (a, b) in zip(c, exps) if a > 0) + 0 * x

    def uy(x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        return sum(ci * b * _pw(x, a) * _pw(y, b - 1)
                   for ci, (a, b) in zip(c, exps) if b > 0) + 0 * x

    def lap(x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        t = 0 * x
        for ci, (a, b) in zip(c, exps):
            if a > 1:
                t = t + ci * a * (a - 1) * _pw(x, a - 2) * _pw(y, b)
            if b > 1:
                t = t + ci * b * (b - 1) * _pw(x, a) * _pw(y, b - 2)
        return t

    def q(x, y):
        return (-ux(x, y), -uy(x, y))

    def f(x, y):
        return bx * ux(x, y) + by * uy(x, y) - kappa * lap(x, y)

    return Manufactured(u, q, f, f"poly{p}")
