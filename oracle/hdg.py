"""Plain FP64 oracle of the macro-element HDG discretisation (2D, triangles).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (paper section 2.1, eqs. C21/C22): div(a u + kappa q) = f, q = -grad u
in Omega, u = g_D on the boundary (Dirichlet only), a constant.

Discretisation (section 3.1, eq. weak_form; spaces of section 3.2):
  A(U,V) = (q,v)_K - (u, div v)_K - (a u + kappa q, grad w)_K
           + <kappa q.n + tau u, w>_dK
  B(v^,V) = <v^, v.n>_dK + <(a.n - tau) v^, w>_dK
  C(U,mu) = sum_K <kappa q.n + tau u, mu>_F ,  D(v^,mu) = sum_K <(a.n-tau) v^, mu>_F
  l(V)   = (f, w)_K - <g, v.n>_{Gamma_D} - <(a.n - tau) g, w>_{Gamma_D}
The last term of l is the Dirichlet part of B, carried to the right-hand side
(the trace is split as v^ + g^ in section 3.1); the printed l omits it.

Spaces (section 3.2): W(K), V(K) are continuous piecewise P_p on the uniform
subdivision of macro K into m^2 = 4^r triangles; M(F) is continuous piecewise
P_p on the face subdivided into 2^{r_F} segments, r_F = max of the adjacent
levels, so the trace represents the finer side exactly (local refinement
paragraph of section 4).  Dirichlet traces are the L2 projection onto M(F)
(section 2.3).

Conventions shared (as a written specification, not as code) with the GPU
library:
  * macro lattice node (i, j), i + j <= P = m p, sits at
    X0 + (i/P)(X1 - X0) + (j/P)(X2 - X0), index j(P+1) - j(j-1)/2 + i;
  * local unknowns U_K = [q_x(Q), q_y(Q), u(Q)], Q = (P+1)(P+2)/2;
  * faces are the unique macro edges sorted by (low vertex id, high vertex
    id); trace node t of face F (n_F = 2^{r_F} p + 1 nodes) sits at
    A + t/(n_F - 1) (B - A), A the lower-id vertex;
  * the global trace vector lists the interior faces in that order;
    Dirichlet data lists the boundary faces in that order;
  * f enters as nodal values at the macro lattice nodes (its interpolant
    in W(K)); g_D enters as samples at k_b = p + 2 Gauss-Legendre points on
    each of the 2^{r_F} segments of every boundary face (faces in sorted
    order, segments and points in increasing t), from which the L2
    projection onto M(F) is formed by that quadrature.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .quadrature import map_to_triangle, segment_rule, triangle_rule


# ---------------------------------------------------------------------------
# O2: faces, orientation, trace levels, numbering
# ---------------------------------------------------------------------------
class Topology:
    def __init__(self, xy, tri, r, p):
        self.xy = np.asarray(xy, dtype=np.float64)
        self.tri = np.asarray(tri, dtype=np.int64)
        n_macro = self.tri.shape[0]
        self.n_macro = n_macro
        self.r = np.broadcast_to(np.asarray(r, dtype=np.int64), (n_macro,)).copy()
        self.p = int(p)
        for K in range(n_macro):
            X = self.xy[self.tri[K]]
            e1, e2 = X[1] - X[0], X[2] - X[0]
            if e1[0] * e2[1] - e1[1] * e2[0] <= 0.0:
                raise ValueError(f"macro {K} is not counter-clockwise")
        incid: dict[tuple[int, int], list[tuple[int, int]]] = {}
        for K in range(n_macro):
            for k in range(3):
                a, b = int(self.tri[K, k]), int(self.tri[K, (k + 1) % 3])
                incid.setdefault((min(a, b), max(a, b)), []).append((K, k))
        keys = sorted(incid)
        self.n_faces = len(keys)
        self.face_verts = np.array(keys, dtype=np.int64)
        self.face_incid = [incid[key] for key in keys]
        if any(len(v) > 2 for v in self.face_incid):
            raise ValueError("non-manifold macro mesh")
        self.interior = np.array([len(v) == 2 for v in self.face_incid])
        self.face_level = np.array([max(self.r[K] for K, _ in v) for v in self.face_incid])
        self.face_nodes = 2 ** self.face_level * self.p + 1
        self.macro_face = np.zeros((n_macro, 3), dtype=np.int64)
        self.macro_orient = np.zeros((n_macro, 3), dtype=np.int64)
        for f, v in enumerate(self.face_incid):
            for K, k in v:
                self.macro_face[K, k] = f
                self.macro_orient[K, k] = 1 if self.tri[K, k] < self.tri[K, (k + 1) % 3] else -1
        # global numbering: interior faces then (separately) boundary faces
        self.trace_off = -np.ones(self.n_faces, dtype=np.int64)
        self.bnd_off = -np.ones(self.n_faces, dtype=np.int64)
        o = 0
        ob = 0
        for f in range(self.n_faces):
            if self.interior[f]:
                self.trace_off[f] = o
                o += self.face_nodes[f]
            else:
                self.bnd_off[f] = ob
                ob += 2 ** int(self.face_level[f]) * (self.p + 2)
        self.n_trace = o
        self.n_bnd = ob      # number of Dirichlet sampling points
        self.m = 2 ** self.r
        self.P = self.m * self.p
        self.Q = (self.P + 1) * (self.P + 2) // 2
        self.N_e = 3 * self.Q
        self.local_off = np.concatenate([[0], np.cumsum(self.N_e)])
        self.node_off = np.concatenate([[0], np.cumsum(self.Q)])

    # -- geometry ---------------------------------------------------------
    def lattice(self, K):
        """(i, j) lattice coordinates of macro K's nodes in index order."""
        P = int(self.P[K])
        return [(i, j) for j in range(P + 1) for i in range(P + 1 - j)]

    def node_xy(self, K):
        """Physical coordinates of macro K's lattice nodes."""
        P = int(self.P[K])
        X = self.xy[self.tri[K]]
        ij = np.array(self.lattice(K), dtype=np.float64)
        return X[0] + np.outer(ij[:, 0] / P, X[1] - X[0]) + np.outer(ij[:, 1] / P, X[2] - X[0])

    def trace_xy(self, f):
        """Physical coordinates of face f's trace nodes (canonical order)."""
        A, B = self.xy[self.face_verts[f, 0]], self.xy[self.face_verts[f, 1]]
        t = np.linspace(0.0, 1.0, int(self.face_nodes[f]))
        return A + np.outer(t, B - A)

    def all_node_xy(self):
        return np.concatenate([self.node_xy(K) for K in range(self.n_macro)])

    def boundary_trace_xy(self):
        fs = [f for f in range(self.n_faces) if not self.interior[f]]
        if not fs:
            return np.zeros((0, 2))
        return np.concatenate([self.trace_xy(f) for f in fs])

    def boundary_qp(self, f):
        """Parameters t and weights (for the full face length) of face f's
        Dirichlet sampling points: k_b = p + 2 Gauss-Legendre points on each
        of its 2^{r_F} segments."""
        kb = self.p + 2
        ts, ws = segment_rule(kb)
        npc = 2 ** int(self.face_level[f])
        L = float(np.linalg.norm(self.xy[self.face_verts[f, 1]] - self.xy[self.face_verts[f, 0]]))
        t = np.concatenate([(c + ts) / npc for c in range(npc)])
        w = np.concatenate([ws * L / npc for c in range(npc)])
        return t, w

    def boundary_qp_xy(self):
        """Physical coordinates of all Dirichlet sampling points."""
        out = []
        for f in range(self.n_faces):
            if not self.interior[f]:
                A, B = self.xy[self.face_verts[f, 0]], self.xy[self.face_verts[f, 1]]
                t, _ = self.boundary_qp(f)
                out.append(A + np.outer(t, B - A))
        return np.concatenate(out) if out else np.zeros((0, 2))


def lattice_index(P):
    idx = -np.ones((P + 1, P + 1), dtype=np.int64)
    n = 0
    for j in range(P + 1):
        for i in range(P + 1 - j):
            idx[i, j] = n
            n += 1
    return idx


def sub_triangles(m, p):
    """Uniform subdivision of the macro lattice into m^2 P_p sub-triangles.

    Returns a list of (corner lattice coords [3, 2], node lattice coords
    [(p+1)(p+2)/2, 2]).  Up triangles (a, b), a + b <= m-1, have corners
    (ap, bp), ((a+1)p, bp), (ap, (b+1)p); down triangles, a + b <= m-2,
    have corners ((a+1)p, (b+1)p), (ap, (b+1)p), ((a+1)p, bp).
    """
    out = []
    loc = [(s, t) for t in range(p + 1) for s in range(p + 1 - t)]
    for b in range(m):
        for a in range(m - b):
            corners = np.array([(a * p, b * p), ((a + 1) * p, b * p), (a * p, (b + 1) * p)])
            nodes = np.array([(a * p + s, b * p + t) for s, t in loc])
            out.append((corners, nodes))
    for b in range(m - 1):
        for a in range(m - 1 - b):
            corners = np.array([((a + 1) * p, (b + 1) * p), (a * p, (b + 1) * p),
                                ((a + 1) * p, b * p)])
            nodes = np.array([((a + 1) * p - s, (b + 1) * p - t) for s, t in loc])
            out.append((corners, nodes))
    return out


# ---------------------------------------------------------------------------
# Lagrange bases by nodal interpolation (the defining property psi_k(y_l) = d_kl)
# ---------------------------------------------------------------------------
def _monomials(p):
    return [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]


def lagrange_2d(nodes_xy, p, x, y):
    """Values and gradients at (x, y) of the P_p Lagrange basis on the given
    physical nodes.  Returns phi, dphi_dx, dphi_dy, each [n_pts, n_nodes]."""
    c = nodes_xy.mean(axis=0)
    h = np.max(np.linalg.norm(nodes_xy - c, axis=1))
    ex = _monomials(p)
    X = (nodes_xy[:, 0] - c[0]) / h
    Y = (nodes_xy[:, 1] - c[1]) / h
    V = np.stack([X ** a * Y ** b for a, b in ex], axis=1)
    Cinv = np.linalg.inv(V)
    xs = (np.asarray(x) - c[0]) / h
    ys = (np.asarray(y) - c[1]) / h
    mono = np.stack([xs ** a * ys ** b for a, b in ex], axis=1)
    mdx = np.stack([a * xs ** max(a - 1, 0) * ys ** b / h if a > 0 else 0 * xs
                    for a, b in ex], axis=1)
    mdy = np.stack([b * xs ** a * ys ** max(b - 1, 0) / h if b > 0 else 0 * xs
                    for a, b in ex], axis=1)
    return mono @ Cinv, mdx @ Cinv, mdy @ Cinv


def lagrange_2d_lap(nodes_xy, p, x, y):
    """Laplacian at (x, y) of the P_p Lagrange basis on the given physical
    nodes (the same monomial representation as lagrange_2d): [n_pts, n_nodes]."""
    c = nodes_xy.mean(axis=0)
    h = np.max(np.linalg.norm(nodes_xy - c, axis=1))
    ex = _monomials(p)
    X = (nodes_xy[:, 0] - c[0]) / h
    Y = (nodes_xy[:, 1] - c[1]) / h
    V = np.stack([X ** a * Y ** b for a, b in ex], axis=1)
    Cinv = np.linalg.inv(V)
    xs = (np.asarray(x) - c[0]) / h
    ys = (np.asarray(y) - c[1]) / h
    lap = np.stack([(a * (a - 1) * xs ** max(a - 2, 0) * ys ** b if a > 1 else 0 * xs)
                    / h ** 2
                    + (b * (b - 1) * xs ** a * ys ** max(b - 2, 0) if b > 1 else 0 * xs) / h ** 2
                    for a, b in ex], axis=1)
    return lap @ Cinv


def supg_tau(h, a_norm, kappa):
    """SUPG parameter of section 3.4 with the element Peclet number
    Pe = |a| h / (2 kappa): tau = h / (2 |a|) (coth Pe - 1/Pe), the classical
    optimal value for 1D advection-diffusion (the printed '+ 1/Pe' read as
    '- 1/Pe'); zero without advection.  For small Pe the difference
    coth Pe - 1/Pe is taken from its series Pe/3 - Pe^3/45 + 2 Pe^5/945."""
    if a_norm == 0.0:
        return 0.0
    pe = a_norm * h / (2.0 * kappa)
    if pe < 1e-2:
        xi = pe / 3.0 - pe ** 3 / 45.0 + 2.0 * pe ** 5 / 945.0
    else:
        xi = 1.0 / np.tanh(pe) - 1.0 / pe
    return h / (2.0 * a_norm) * xi


def lagrange_1d(nodes_t, t):
    """Values at t of the 1D Lagrange basis on nodes_t: [n_pts, n_nodes]."""
    nodes_t = np.asarray(nodes_t, float)
    t = np.asarray(t, float)
    out = np.ones((t.size, nodes_t.size))
    for k in range(nodes_t.size):
        for l in range(nodes_t.size):
            if l != k:
                out[:, k] *= (t - nodes_t[l]) / (nodes_t[k] - nodes_t[l])
    return out


# ---------------------------------------------------------------------------
# O5/O6: local blocks of one macro element
# ---------------------------------------------------------------------------
class MacroBlocks:
    """Blocks of macro K: A (N_e x N_e), per local edge k the coupling
    G_k[i, l] = <mu_l, phi_i>_F (Q x n_F), B_k (N_e x n_F), C_k (n_F x N_e),
    the macro mass matrix M (Q x Q) and the boundary mass Mb = <phi_j, phi_i>_dK."""


def _locate(sub, lat_pts):
    """Index of the sub-triangle that contains the lattice point (largest
    smallest barycentric coordinate)."""
    best, best_v = -1, -np.inf
    for s, (corners, _) in enumerate(sub):
        c = corners.astype(float)
        T = np.array([c[1] - c[0], c[2] - c[0]]).T
        lam = np.linalg.solve(T, lat_pts - c[0])
        v = min(lam[0], lam[1], 1.0 - lam[0] - lam[1])
        if v > best_v:
            best, best_v = s, v
    return best


def macro_blocks(topo: Topology, K: int, kappa: float, beta, tau: float, nq: int | None = None,
                 supg: bool = False):
    p = topo.p
    m = int(topo.m[K])
    P = int(topo.P[K])
    Q = int(topo.Q[K])
    nq = nq or (p + 3)
    X = topo.xy[topo.tri[K]]
    e1, e2 = X[1] - X[0], X[2] - X[0]
    idx = lattice_index(P)
    sub = sub_triangles(m, p)

    # The blocks are integrals of the local basis over the macro and its edges,
    # unchanged by a translation; they are formed in coordinates relative to the
    # macro's first vertex X0, so that the rounding of quadrature points is
    # relative to the macro's size rather than to its distance from the origin.
    def lat2xy(ij):
        ij = np.asarray(ij, float)
        return np.outer(ij[..., 0] / P, e1) + np.outer(ij[..., 1] / P, e2)

    xi, eta, wref = triangle_rule(nq)
    M = np.zeros((Q, Q))
    Ex = np.zeros((Q, Q))
    Ey = np.zeros((Q, Q))
    bx, by = float(beta[0]), float(beta[1])
    # SUPG (section 3.4): tau_e (a.grad w, a.grad u - kappa lap u)_e summed over
    # the sub-triangles e of K; all of them are congruent, h is their diameter
    Ks = np.zeros((Q, Q))
    tau_s = 0.0
    if supg:
        Xc = lat2xy(sub[0][0])
        h = max(np.linalg.norm(Xc[1] - Xc[0]), np.linalg.norm(Xc[2] - Xc[1]),
                np.linalg.norm(Xc[0] - Xc[2]))
        tau_s = supg_tau(h, float(np.hypot(bx, by)), float(kappa))
    for corners, nodes in sub:
        ids = idx[nodes[:, 0], nodes[:, 1]]
        cxy = lat2xy(corners)
        xq, yq, wq = map_to_triangle(cxy, xi, eta, wref)
        phi, dx, dy = lagrange_2d(lat2xy(nodes), p, xq, yq)
        W = wq[:, None]
        # row = test function index, column = trial function index
        M[np.ix_(ids, ids)] += phi.T @ (W * phi)
        Ex[np.ix_(ids, ids)] += dx.T @ (W * phi)     # (phi_j, d_x phi_i)
        Ey[np.ix_(ids, ids)] += dy.T @ (W * phi)
        if tau_s != 0.0:
            adv = bx * dx + by * dy                   # a.grad of each basis function
            lap = lagrange_2d_lap(lat2xy(nodes), p, xq, yq)
            Ks[np.ix_(ids, ids)] += tau_s * (adv.T @ (W * (adv - kappa * lap)))

    # boundary terms on the face partitions (level r_F >= r_K)
    ts, ws = segment_rule(nq)
    Mb = np.zeros((Q, Q))
    Mbx = np.zeros((Q, Q))
    Mby = np.zeros((Q, Q))
    G, normals, lengths = [], [], []
    for k in range(3):
        f = int(topo.macro_face[K, k])
        nF = int(topo.face_nodes[f])
        rF = int(topo.face_level[f])
        A = topo.xy[topo.face_verts[f, 0]] - X[0]
        B = topo.xy[topo.face_verts[f, 1]] - X[0]
        L = float(np.linalg.norm(B - A))
        tvec = X[(k + 1) % 3] - X[k]
        n = np.array([tvec[1], -tvec[0]]) / np.linalg.norm(tvec)
        normals.append(n)
        lengths.append(L)
        Gk = np.zeros((Q, nF))
        t_nodes = np.linspace(0.0, 1.0, nF)
        npc = 2 ** rF
        # inverse of the macro's affine map, to locate points in lattice coords
        Tm = np.array([e1, e2]).T
        for c in range(npc):
            t = (c + ts) / npc
            w = ws * L / npc
            pts = A + np.outer(t, B - A)
            mid = A + ((c + 0.5) / npc) * (B - A)
            lat_mid = np.linalg.solve(Tm, mid) * P
            s = _locate(sub, lat_mid)
            corners, nodes = sub[s]
            ids = idx[nodes[:, 0], nodes[:, 1]]
            phi, _, _ = lagrange_2d(lat2xy(nodes), p, pts[:, 0], pts[:, 1])
            lr = np.arange(c * p, c * p + p + 1)
            mu = lagrange_1d(t_nodes[lr], t)
            Wb = w[:, None]
            mm = phi.T @ (Wb * phi)
            Mb[np.ix_(ids, ids)] += mm
            Mbx[np.ix_(ids, ids)] += n[0] * mm
            Mby[np.ix_(ids, ids)] += n[1] * mm
            Gk[np.ix_(ids, lr)] += phi.T @ (Wb * mu)
        G.append(Gk)

    Hx = -Ex + Mbx
    Hy = -Ey + Mby
    Kuu = -(bx * Ex + by * Ey) + tau * Mb + Ks
    Z = np.zeros((Q, Q))
    Amat = np.block([[M, Z, -Ex], [Z, M, -Ey], [kappa * Hx, kappa * Hy, Kuu]])
    Bk, Ck = [], []
    for k in range(3):
        n = normals[k]
        an = bx * n[0] + by * n[1]
        Bk.append(np.vstack([n[0] * G[k], n[1] * G[k], (an - tau) * G[k]]))
        Ck.append(np.hstack([kappa * n[0] * G[k].T, kappa * n[1] * G[k].T, tau * G[k].T]))
    out = MacroBlocks()
    out.A, out.B, out.C, out.G = Amat, Bk, Ck, G
    out.M, out.Mb, out.Ex, out.Ey = M, Mb, Ex, Ey
    out.normals, out.lengths = normals, lengths
    # SUPG: the stabilisation block and the matrix of the source term
    # tau (a.grad w, f_h)_K = tau (a_x E^x + a_y E^y) f_K (E^d_ij = (phi_j, d_d phi_i))
    out.Ksupg, out.tau_supg = Ks, tau_s
    out.Fsupg = tau_s * (bx * Ex + by * Ey)
    return out


def face_mass(topo: Topology, f: int, nq: int | None = None):
    """<mu_l, mu_l'>_F on the face partition."""
    nq = nq or (topo.p + 3)
    nF = int(topo.face_nodes[f])
    npc = 2 ** int(topo.face_level[f])
    L = float(np.linalg.norm(topo.xy[topo.face_verts[f, 1]] - topo.xy[topo.face_verts[f, 0]]))
    ts, ws = segment_rule(nq)
    t_nodes = np.linspace(0.0, 1.0, nF)
    MF = np.zeros((nF, nF))
    p = topo.p
    for c in range(npc):
        t = (c + ts) / npc
        w = ws * L / npc
        lr = np.arange(c * p, c * p + p + 1)
        mu = lagrange_1d(t_nodes[lr], t)
        MF[np.ix_(lr, lr)] += mu.T @ (w[:, None] * mu)
    return MF


# ---------------------------------------------------------------------------
# the whole discrete problem
# ---------------------------------------------------------------------------
class Oracle:
    """Condensed direct solution of the macro-element HDG system.

    kappa: scalar or per-macro array; beta: constant advection (a in the
    paper); tau: LDG-H stabilisation, the same on every macro side.
    """

    def __init__(self, xy, tri, r, p, kappa, beta, tau=1.0, nq=None, cache=True, supg=False):
        self.topo = Topology(xy, tri, r, p)
        self.supg = bool(supg)
        self.kappa = np.broadcast_to(np.asarray(kappa, float), (self.topo.n_macro,)).copy()
        self.beta = np.asarray(beta, float).reshape(2)
        self.tau = float(tau)
        self.nq = nq
        self._cache = {} if cache else None

    # -- blocks -----------------------------------------------------------
    def blocks(self, K):
        if self._cache is not None and K in self._cache:
            return self._cache[K]
        b = macro_blocks(self.topo, K, self.kappa[K], self.beta, self.tau, self.nq,
                         supg=self.supg)
        if self._cache is not None:
            self._cache[K] = b
        return b

    def lu(self, K):
        """Partial-pivoting LU of A_K, computed once and reused (the in-place
        factorisation remark of section 3.3.2)."""
        b = self.blocks(K)
        if getattr(b, "lu", None) is None:
            b.lu = sla.lu_factor(b.A)
        return b.lu

    def D_face(self, f):
        """D_F = sum over the macros of F of <(a.n_K - tau) mu_j, mu_l>_F."""
        topo = self.topo
        MF = face_mass(topo, f, self.nq)
        D = np.zeros_like(MF)
        for K, k in topo.face_incid[f]:
            X = topo.xy[topo.tri[K]]
            tvec = X[(k + 1) % 3] - X[k]
            n = np.array([tvec[1], -tvec[0]]) / np.linalg.norm(tvec)
            D += (self.beta @ n - self.tau) * MF
        return D

    # -- data ---------------------------------------------------------------
    def dirichlet_trace(self, g_bnd):
        """L2 projection P (section 2.3) of the Dirichlet data onto M(F), per
        boundary face: M_F lam_F = (g, mu)_F, the right side by the sampling
        quadrature (g_bnd holds g at the points of Topology.boundary_qp)."""
        topo = self.topo
        lamD = {}
        for f in range(topo.n_faces):
            if topo.interior[f]:
                continue
            t, w = topo.boundary_qp(f)
            o = topo.bnd_off[f]
            g = np.asarray(g_bnd[o:o + t.size], float)
            nF = int(topo.face_nodes[f])
            p = topo.p
            npc = 2 ** int(topo.face_level[f])
            t_nodes = np.linspace(0.0, 1.0, nF)
            rhs = np.zeros(nF)
            kb = p + 2
            for c in range(npc):
                sl = slice(c * kb, (c + 1) * kb)
                lr = np.arange(c * p, c * p + p + 1)
                mu = lagrange_1d(t_nodes[lr], t[sl])
                rhs[lr] += mu.T @ (w[sl] * g[sl])
            MF = face_mass(topo, f, self.nq)
            lamD[f] = np.linalg.solve(MF, rhs)
        return lamD

    def local_rhs(self, K, f_nodal, lamD):
        """R_K: (f_h, w)_K (plus the SUPG source term tau (a.grad w, f_h)_K when
        stabilised) on the w rows minus the Dirichlet columns of B_K."""
        topo = self.topo
        b = self.blocks(K)
        Q = int(topo.Q[K])
        fo = topo.node_off[K]
        fK = np.asarray(f_nodal[fo:fo + Q], float)
        R = np.zeros(3 * Q)
        R[2 * Q:] = b.M @ fK + b.Fsupg @ fK
        for k in range(3):
            f = int(topo.macro_face[K, k])
            if not topo.interior[f]:
                R -= b.B[k] @ lamD[f]
        return R

    def _interior_cols(self, K):
        """For macro K: list of (local edge k, global trace offset, n_F)."""
        topo = self.topo
        out = []
        for k in range(3):
            f = int(topo.macro_face[K, k])
            if topo.interior[f]:
                out.append((k, int(topo.trace_off[f]), int(topo.face_nodes[f])))
        return out

    # -- O7: condensation ----------------------------------------------------
    def condensed(self, f_nodal, g_bnd):
        """S = D - sum_K C_K A_K^-1 B_K and f^ = -sum_K C_K A_K^-1 R_K on the
        interior trace unknowns (eq. global_problem; R_u^ = 0)."""
        topo = self.topo
        lamD = self.dirichlet_trace(g_bnd)
        n = topo.n_trace
        rows, cols, vals = [], [], []
        fhat = np.zeros(n)
        for f in range(topo.n_faces):
            if topo.interior[f]:
                o, nF = int(topo.trace_off[f]), int(topo.face_nodes[f])
                D = self.D_face(f)
                ii, jj = np.meshgrid(np.arange(o, o + nF), np.arange(o, o + nF), indexing="ij")
                rows.append(ii.ravel())
                cols.append(jj.ravel())
                vals.append(D.ravel())
        for K in range(topo.n_macro):
            b = self.blocks(K)
            lu = self.lu(K)
            icols = self._interior_cols(K)
            if not icols:
                continue
            Bi = np.hstack([b.B[k] for k, _, _ in icols])
            Ci = np.vstack([b.C[k] for k, _, _ in icols])
            gidx = np.concatenate([np.arange(o, o + nF) for _, o, nF in icols])
            Se = -Ci @ sla.lu_solve(lu, Bi)
            ii, jj = np.meshgrid(gidx, gidx, indexing="ij")
            rows.append(ii.ravel())
            cols.append(jj.ravel())
            vals.append(Se.ravel())
            R = self.local_rhs(K, f_nodal, lamD)
            np.add.at(fhat, gidx, -Ci @ sla.lu_solve(lu, R))
        if not vals:            # a mesh without interior faces has no trace unknowns
            return sp.csc_matrix((n, n)), fhat, lamD
        S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n)).tocsc()
        return S, fhat, lamD

    # -- O8/O9 ----------------------------------------------------------------
    def solve(self, f_nodal, g_bnd):
        """Direct solve of the global problem, then local recovery.
        Returns (lam [n_trace], U list per macro, lamD dict)."""
        S, fhat, lamD = self.condensed(f_nodal, g_bnd)
        if S.shape[0] == 0:
            lam = np.zeros(0)
        elif S.shape[0] <= 2000:
            lam = np.linalg.solve(S.toarray(), fhat)
        else:
            lam = spla.splu(S).solve(fhat)
        U = self.recover(lam, f_nodal, lamD)
        return lam, U, lamD

    def recover(self, lam, f_nodal, lamD):
        """Local problem A_K U_K = R_K - B_K lam_K (eq. local_problem)."""
        topo = self.topo
        U = []
        for K in range(topo.n_macro):
            b = self.blocks(K)
            rhs = self.local_rhs(K, f_nodal, lamD)
            for k, o, nF in self._interior_cols(K):
                rhs = rhs - b.B[k] @ lam[o:o + nF]
            U.append(sla.lu_solve(self.lu(K), rhs))
        return U

    # -- O12: the trace operator, steps 1-4 of the matrix-free algorithm ------
    def macro_contribution(self, K, lam, transpose=False):
        """Steps 1-3 on macro K: x = B_K lam_K, y = A_K^-1 x, v^ = C_K y.
        With transpose, the same product for the transposed operator:
        x = C_K^T lam_K, y = A_K^-T x, v^ = B_K^T y.
        Returns {face: v^ restricted to that interior face}."""
        b = self.blocks(K)
        icols = self._interior_cols(K)
        if not icols:
            return {}
        if transpose:
            x = sum(b.C[k].T @ lam[o:o + nF] for k, o, nF in icols)
            y = sla.lu_solve(self.lu(K), x, trans=1)
            return {int(self.topo.macro_face[K, k]): b.B[k].T @ y for k, _, _ in icols}
        x = sum(b.B[k] @ lam[o:o + nF] for k, o, nF in icols)
        y = sla.lu_solve(self.lu(K), x)
        return {int(self.topo.macro_face[K, k]): b.C[k] @ y for k, _, _ in icols}

    def apply(self, lam, precondition=False, faces=None, transpose=False):
        """S lam (or D^-1 S lam: step 4 with the D^-1 preconditioner,
        w_F = lam_F - D_F^-1 (v^_F1 + v^_F2)).  With transpose, S^T lam (or
        D^-1 S^T lam): S^T = D^T - sum_K B_K^T A_K^-T C_K^T and D_F is
        symmetric.  If `faces` is given, only those interior faces are
        computed (others left zero)."""
        topo = self.topo
        lam = np.asarray(lam, float)
        out = np.zeros(topo.n_trace)
        fs = range(topo.n_faces) if faces is None else faces
        macros = sorted({K for f in fs if topo.interior[f] for K, _ in topo.face_incid[f]})
        contrib = {K: self.macro_contribution(K, lam, transpose) for K in macros}
        for f in fs:
            if not topo.interior[f]:
                continue
            o, nF = int(topo.trace_off[f]), int(topo.face_nodes[f])
            v = sum(contrib[K][f] for K, _ in topo.face_incid[f])
            D = self.D_face(f)
            if precondition:
                # D_F is negative definite (-D_F = (tau+ + tau-) M_F): Cholesky of -D_F
                c = sla.cho_factor(-D)
                out[o:o + nF] = lam[o:o + nF] + sla.cho_solve(c, v)
            else:
                out[o:o + nF] = D @ lam[o:o + nF] - v
        return out

    def precondition(self, v):
        """D^-1 v on the interior trace vector."""
        topo = self.topo
        out = np.zeros_like(v)
        for f in range(topo.n_faces):
            if topo.interior[f]:
                o, nF = int(topo.trace_off[f]), int(topo.face_nodes[f])
                c = sla.cho_factor(-self.D_face(f))
                out[o:o + nF] = -sla.cho_solve(c, v[o:o + nF])
        return out

    def local_solve(self, K, x, transpose=False):
        """A_K^-1 x (or A_K^-T x) with partial-pivoting LU."""
        return sla.lu_solve(self.lu(K), x, trans=1 if transpose else 0)

    # -- boundary-condensed blocks (steps 1-3 restricted to the macro boundary) -
    def boundary_rows(self, K):
        """Rows of U_K = [q_x, q_y, u] that sit on the boundary of macro K, in
        the compact boundary order: field-major, then position b = kP + s, the
        lattice node at step s = 0 .. P-1 of local edge k walked from vertex k
        towards vertex k+1 (lattice (s, 0), (P-s, s), (0, P-s) for k = 0, 1, 2);
        3P nodes, each corner once."""
        P, Q = int(self.topo.P[K]), int(self.topo.Q[K])
        idx = lattice_index(P)
        walk = [lambda s: (s, 0), lambda s: (P - s, s), lambda s: (0, P - s)]
        nodes = np.array([idx[walk[k](s)] for k in range(3) for s in range(P)], dtype=np.int64)
        return np.concatenate([f * Q + nodes for f in range(3)])

    def boundary_block(self, K):
        """W_K = (A_K^-1)_bb: the block of A_K^-1 on the boundary rows and
        columns of boundary_rows(K).  B_K (boundary integrals against the
        macro basis) vanishes off those rows and C_K off those columns, so
        steps 1-3 of section 3.3.2 equal C_b W_K B_b.  Formed here as the
        boundary rows of A_K^-1 e_c for every boundary unit vector e_c."""
        rows = self.boundary_rows(K)
        N = self.blocks(K).A.shape[0]
        E = np.zeros((N, rows.size))
        E[rows, np.arange(rows.size)] = 1.0
        return self.local_solve(K, E)[rows, :]

    # -- O11: brute force on the unhybridised system ---------------------------
    def brute_force(self, f_nodal, g_bnd):
        """Dense solve of [A B; C D][U; lam] = [R; 0] over all macros."""
        topo = self.topo
        lamD = self.dirichlet_trace(g_bnd)
        nU = int(topo.local_off[-1])
        n = nU + topo.n_trace
        Kmat = np.zeros((n, n))
        F = np.zeros(n)
        for K in range(topo.n_macro):
            b = self.blocks(K)
            lo, hi = topo.local_off[K], topo.local_off[K + 1]
            Kmat[lo:hi, lo:hi] = b.A
            F[lo:hi] = self.local_rhs(K, f_nodal, lamD)
            for k, o, nF in self._interior_cols(K):
                Kmat[lo:hi, nU + o:nU + o + nF] += b.B[k]
                Kmat[nU + o:nU + o + nF, lo:hi] += b.C[k]
        for f in range(topo.n_faces):
            if topo.interior[f]:
                o, nF = int(topo.trace_off[f]), int(topo.face_nodes[f])
                Kmat[nU + o:nU + o + nF, nU + o:nU + o + nF] += self.D_face(f)
        X = np.linalg.solve(Kmat, F)
        U = [X[topo.local_off[K]:topo.local_off[K + 1]] for K in range(topo.n_macro)]
        return X[nU:], U, lamD

    # -- O10: diagnostics --------------------------------------------------------
    def l2_errors(self, U, exact, nq=None):
        """L2 errors of u and q against a manufactured solution."""
        topo = self.topo
        p = topo.p
        nq = nq or (p + 6)
        xi, eta, wref = triangle_rule(nq)
        eu = eq = 0.0
        for K in range(topo.n_macro):
            m, P, Q = int(topo.m[K]), int(topo.P[K]), int(topo.Q[K])
            X = topo.xy[topo.tri[K]]
            e1, e2 = X[1] - X[0], X[2] - X[0]
            idx = lattice_index(P)
            qx, qy, u = U[K][:Q], U[K][Q:2 * Q], U[K][2 * Q:]

            def lat2xy(ij):
                ij = np.asarray(ij, float)
                return X[0] + np.outer(ij[..., 0] / P, e1) + np.outer(ij[..., 1] / P, e2)

            for corners, nodes in sub_triangles(m, p):
                ids = idx[nodes[:, 0], nodes[:, 1]]
                xq, yq, wq = map_to_triangle(lat2xy(corners), xi, eta, wref)
                phi, _, _ = lagrange_2d(lat2xy(nodes), p, xq, yq)
                ue = exact.u(xq, yq)
                qe = exact.q(xq, yq)
                eu += np.sum(wq * (phi @ u[ids] - ue) ** 2)
                eq += np.sum(wq * ((phi @ qx[ids] - qe[0]) ** 2 + (phi @ qy[ids] - qe[1]) ** 2))
        return float(np.sqrt(eu)), float(np.sqrt(eq))

    def flux_balance(self, U, lam, lamD, f_nodal, macros=None):
        """Per macro: <flux^.n, 1>_dK - (f_h, 1)_K with the LDG-H flux
        flux^.n = a.n u^ + kappa q.n + tau (u - u^) (section 3.1); zero for
        the discrete solution because w = 1 lies in W(K).  macros: the macros
        to evaluate (default all; the others are left zero)."""
        topo = self.topo
        res = np.zeros(topo.n_macro)
        for K in (range(topo.n_macro) if macros is None else macros):
            b = self.blocks(K)
            Q = int(topo.Q[K])
            qx, qy, u = U[K][:Q], U[K][Q:2 * Q], U[K][2 * Q:]
            ones = np.ones(Q)
            fo = topo.node_off[K]
            tot = -(ones @ (b.M @ f_nodal[fo:fo + Q]))
            for k in range(3):
                f = int(topo.macro_face[K, k])
                lh = lam[topo.trace_off[f]:topo.trace_off[f] + topo.face_nodes[f]] \
                    if topo.interior[f] else lamD[f]
                n = b.normals[k]
                an = self.beta @ n
                G = b.G[k]                 # <mu_l, phi_i>_F
                # <a.n u^ + kappa q.n + tau (u - u^), 1>_F
                tot += (an - self.tau) * (ones @ (G @ lh))
                wsum = G.sum(axis=1)      # <1, phi_i>_F summed over mu (partition of unity)
                tot += self.kappa[K] * (n[0] * wsum @ qx + n[1] * wsum @ qy) + self.tau * wsum @ u
            res[K] = tot
        return res

    def transmission_residual(self, U, lam):
        """Per interior trace dof: (C U + D lam)_F = weak normal-flux jump
        tested with each mu (eq. transmission with g_N = 0)."""
        topo = self.topo
        out = np.zeros(topo.n_trace)
        for f in range(topo.n_faces):
            if not topo.interior[f]:
                continue
            o, nF = int(topo.trace_off[f]), int(topo.face_nodes[f])
            v = self.D_face(f) @ lam[o:o + nF]
            for K, k in topo.face_incid[f]:
                v = v + self.blocks(K).C[k] @ U[K]
            out[o:o + nF] = v
        return out

    # -- sampling of data at the oracle's own node positions -----------------
    def sample(self, exact):
        """f at every macro lattice node, g_D at every Dirichlet sampling point."""
        topo = self.topo
        nx = topo.all_node_xy()
        bx = topo.boundary_qp_xy()
        return exact.f(nx[:, 0], nx[:, 1]), exact.u(bx[:, 0], bx[:, 1]) if len(bx) else np.zeros(0)
