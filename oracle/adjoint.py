"""Oracle adjoint of the macro-element HDG solution (FP64, small meshes).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Objective J(X) = sum_K (u_K - u_obs,K)^T M_K (u_K - u_obs,K): the squared L2
distance of the discrete u to a given field in the same space.  With the full
system K(theta) X = F(theta), X = (U, lam_interior) (paper eq. D before
condensation), the gradient is

    dJ/dtheta = Psi^T (dF/dtheta - dK/dtheta X),   K^T Psi = dJ/dX.

The forms of section 3.2 are affine in kappa_K (A_K through kappa H, C_K
through kappa q.n) and in the advection a (A_K through -(a u, grad w), B_K and
the Dirichlet columns through (a.n - tau)), so each dK/dtheta is computed
exactly as the difference of two assemblies (parameter 1 minus parameter 0).
f is held fixed.  The adjoint system is solved directly (sparse LU).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .hdg import Oracle, macro_blocks


def full_system(orc: Oracle, f_nodal, g_bnd):
    """Sparse K and F of the unhybridised system over (U, lam_interior)."""
    topo = orc.topo
    lamD = orc.dirichlet_trace(g_bnd)
    nU = int(topo.local_off[-1])
    n = nU + topo.n_trace
    rows, cols, vals = [], [], []
    F = np.zeros(n)

    def put(r0, c0, Mat):
        ii, jj = np.nonzero(Mat)
        rows.append(ii + r0)
        cols.append(jj + c0)
        vals.append(Mat[ii, jj])

    for K in range(topo.n_macro):
        b = orc.blocks(K)
        lo = int(topo.local_off[K])
        put(lo, lo, b.A)
        F[lo:lo + b.A.shape[0]] = orc.local_rhs(K, f_nodal, lamD)
        for k, o, nF in orc._interior_cols(K):
            put(lo, nU + o, b.B[k])
            put(nU + o, lo, b.C[k])
    for fc in range(topo.n_faces):
        if topo.interior[fc]:
            o = int(topo.trace_off[fc])
            put(nU + o, nU + o, orc.D_face(fc))
    Kmat = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsc()
    return Kmat, F, lamD


def objective(orc: Oracle, U, u_obs):
    """J = sum_K (u_K - u_obs,K)^T M_K (u_K - u_obs,K); u_obs per macro (nodal u)."""
    topo = orc.topo
    J = 0.0
    for K in range(topo.n_macro):
        Q = int(topo.Q[K])
        d = U[K][2 * Q:] - u_obs[K]
        J += d @ orc.blocks(K).M @ d
    return J


def gradient(orc: Oracle, f_nodal, g_bnd, u_obs):
    """(J, dJ/dkappa [n_macro], dJ/da [2], Psi_U list, Psi_lam) by the adjoint.
    Unstabilised forms only: with SUPG the forms are not affine in kappa and a."""
    if orc.supg:
        raise ValueError("the adjoint gradient covers the forms without SUPG")
    topo = orc.topo
    Kmat, F, lamD = full_system(orc, f_nodal, g_bnd)
    X = spla.splu(Kmat).solve(F)
    nU = int(topo.local_off[-1])
    U = [X[topo.local_off[K]:topo.local_off[K + 1]] for K in range(topo.n_macro)]
    lam = X[nU:]
    g = np.zeros_like(X)
    for K in range(topo.n_macro):
        Q = int(topo.Q[K])
        lo = int(topo.local_off[K])
        d = U[K][2 * Q:] - u_obs[K]
        g[lo + 2 * Q:lo + 3 * Q] = 2.0 * orc.blocks(K).M @ d
    Psi = spla.splu(Kmat.T.tocsc()).solve(g)
    PsiU = [Psi[topo.local_off[K]:topo.local_off[K + 1]] for K in range(topo.n_macro)]
    Psil = Psi[nU:]

    def lam_of(K, k):
        f = int(topo.macro_face[K, k])
        if topo.interior[f]:
            o = int(topo.trace_off[f])
            return lam[o:o + topo.face_nodes[f]]
        return lamD[f]

    # kappa_K: dK/dkappa_K = K(kappa_K = 1) - K(kappa_K = 0), local to macro K
    dkap = np.zeros(topo.n_macro)
    for K in range(topo.n_macro):
        b1 = macro_blocks(topo, K, 1.0, orc.beta, orc.tau, orc.nq)
        b0 = macro_blocks(topo, K, 0.0, orc.beta, orc.tau, orc.nq)
        v = PsiU[K] @ ((b1.A - b0.A) @ U[K])
        for k, o, nF in orc._interior_cols(K):
            v += Psil[o:o + nF] @ ((b1.C[k] - b0.C[k]) @ U[K])
        dkap[K] = -v
    # advection a_d: A_K and B_K (interior and Dirichlet columns) are affine in a
    dbeta = np.zeros(2)
    for d in range(2):
        e = np.zeros(2)
        e[d] = 1.0
        tot = 0.0
        for K in range(topo.n_macro):
            kap = orc.kappa[K]
            b1 = macro_blocks(topo, K, kap, e, orc.tau, orc.nq)
            b0 = macro_blocks(topo, K, kap, np.zeros(2), orc.tau, orc.nq)
            dA = b1.A - b0.A
            v = -(PsiU[K] @ (dA @ U[K]))
            for k in range(3):
                dB = b1.B[k] - b0.B[k]
                f = int(topo.macro_face[K, k])
                if topo.interior[f]:
                    v -= PsiU[K] @ (dB @ lam_of(K, k))      # -Psi^T dK X (trace columns)
                else:
                    v -= PsiU[K] @ (dB @ lamD[f])           # Psi^T dF (R = ... - B_D lam_D)
            tot += v
        # D_F is independent of a on interior faces (the two normals cancel)
        for fc in range(topo.n_faces):
            if topo.interior[fc]:
                o, nF = int(topo.trace_off[fc]), int(topo.face_nodes[fc])
                saved = orc.beta.copy()
                orc.beta = e
                D1 = orc.D_face(fc)
                orc.beta = np.zeros(2)
                D0 = orc.D_face(fc)
                orc.beta = saved
                tot -= Psil[o:o + nF] @ ((D1 - D0) @ lam[o:o + nF])
        dbeta[d] = tot
    J = objective(orc, U, u_obs)
    return J, dkap, dbeta, PsiU, Psil, U, lam
