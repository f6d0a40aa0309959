"""Oracle quantities over a whole mesh, computed in worker processes.

Test infrastructure for the full-size GPU checks: a solve's residual bound
there is relative to the norm of the preconditioned right side D^-1 f^ over
every interior face (f^_F = -sum over the macros of F of C_K A_K^-1 R_K,
eq. global_problem), which needs every macro's local solve.  The workers
start fresh interpreters (spawn), import only numpy, scipy and the oracle,
and run single-threaded BLAS.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from oracle import hdg

_STATE: dict = {}


def _init(args):
    from threadpoolctl import threadpool_limits
    _STATE["limits"] = threadpool_limits(1)
    xy, tri, r, p, kappa, beta, tau, f_nodal, lamD = args
    _STATE["orc"] = hdg.Oracle(xy, tri, r, p, kappa, beta, tau)
    _STATE["f"] = f_nodal
    _STATE["lamD"] = lamD


def _macro_part(chunk):
    """-C_K A_K^-1 R_K restricted to each interior face of the macros in chunk."""
    orc = _STATE["orc"]
    out = []
    for K in chunk:
        icols = orc._interior_cols(K)
        if icols:
            b = orc.blocks(K)
            y = orc.local_solve(K, orc.local_rhs(K, _STATE["f"], _STATE["lamD"]))
            for k, _, _ in icols:
                out.append((int(orc.topo.macro_face[K, k]), -(b.C[k] @ y)))
        orc._cache.clear()
    return out


def _face_part(items):
    """Squared norms of D_F^-1 f^_F."""
    orc = _STATE["orc"]
    return sum(float(w @ w) for w in (np.linalg.solve(orc.D_face(f), v) for f, v in items))


def preconditioned_rhs_norm(xy, tri, r, p, kappa, beta, tau, f_nodal, lamD, workers=None):
    """||D^-1 f^|| over all interior trace unknowns (FP64 oracle)."""
    args = (np.asarray(xy), np.asarray(tri), r, p, kappa, beta, tau, np.asarray(f_nodal), lamD)
    n = len(tri)
    workers = workers if workers is not None else min(16, os.cpu_count() or 1)
    if workers <= 1:
        _init(args)
        acc = {}
        for f, v in _macro_part(range(n)):
            acc[f] = acc.get(f, 0.0) + v
        return float(np.sqrt(_face_part(list(acc.items()))))
    nchunk = 4 * workers
    chunks = [list(range(i, n, nchunk)) for i in range(nchunk)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_init, initargs=(args,)) as pool:
        acc = {}
        for part in pool.map(_macro_part, chunks):
            for f, v in part:
                acc[f] = acc.get(f, 0.0) + v
        items = list(acc.items())
        total = sum(pool.map(_face_part, [items[i::nchunk] for i in range(nchunk)]))
    return float(np.sqrt(total))


def _init_full(args):
    from threadpoolctl import threadpool_limits
    _STATE["limits"] = threadpool_limits(1)
    xy, tri, r, p, kappa, beta, tau, f_nodal, lamD = args
    _STATE["orc"] = hdg.Oracle(xy, tri, r, p, kappa, beta, tau)
    _STATE["f"] = f_nodal
    _STATE["lamD"] = lamD


def _macro_condensed(chunk):
    """Per macro of chunk: the interior trace indices, S_K = -C_K A_K^-1 B_K on
    them and f^_K = -C_K A_K^-1 R_K (eq. global_problem), as Oracle.condensed
    forms them."""
    import scipy.linalg as sla
    orc = _STATE["orc"]
    out = []
    for K in chunk:
        icols = orc._interior_cols(K)
        if icols:
            b = orc.blocks(K)
            lu = orc.lu(K)
            Bi = np.hstack([b.B[k] for k, _, _ in icols])
            Ci = np.vstack([b.C[k] for k, _, _ in icols])
            gidx = np.concatenate([np.arange(o, o + nF) for _, o, nF in icols])
            R = orc.local_rhs(K, _STATE["f"], _STATE["lamD"])
            out.append((gidx, -Ci @ sla.lu_solve(lu, Bi), -Ci @ sla.lu_solve(lu, R)))
        orc._cache.clear()
    return out


def direct_solve(xy, tri, r, p, kappa, beta, tau, f_nodal, g_bnd, workers=None):
    """lam = S^-1 f^ by a sparse direct solve (SuperLU) of the assembled
    condensed system, the same definition as Oracle.solve, with the per-macro
    condensation in worker processes.  Returns (lam, ||D^-1 f^||)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    orc = hdg.Oracle(np.asarray(xy), np.asarray(tri), r, p, kappa, beta, tau)
    topo = orc.topo
    lamD = orc.dirichlet_trace(np.asarray(g_bnd))
    args = (np.asarray(xy), np.asarray(tri), r, p, kappa, beta, tau, np.asarray(f_nodal), lamD)
    n = int(topo.n_trace)
    workers = workers if workers is not None else min(16, os.cpu_count() or 1)
    nchunk = 4 * workers
    chunks = [list(range(i, len(tri), nchunk)) for i in range(nchunk)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_init_full, initargs=(args,)) as pool:
        parts = pool.map(_macro_condensed, chunks)
    rows, cols, vals = [], [], []
    fhat = np.zeros(n)
    Dinv_blocks = []
    for f in range(topo.n_faces):
        if topo.interior[f]:
            o, nF = int(topo.trace_off[f]), int(topo.face_nodes[f])
            D = orc.D_face(f)
            ii, jj = np.meshgrid(np.arange(o, o + nF), np.arange(o, o + nF), indexing="ij")
            rows.append(ii.ravel())
            cols.append(jj.ravel())
            vals.append(D.ravel())
            Dinv_blocks.append((o, nF, D))
    for part in parts:
        for gidx, Se, fe in part:
            ii, jj = np.meshgrid(gidx, gidx, indexing="ij")
            rows.append(ii.ravel())
            cols.append(jj.ravel())
            vals.append(Se.ravel())
            np.add.at(fhat, gidx, fe)
    del parts
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsc()
    del rows, cols, vals
    lam = spla.splu(S).solve(fhat)
    pf2 = sum(float(np.linalg.solve(D, fhat[o:o + nF]) @ np.linalg.solve(D, fhat[o:o + nF]))
              for o, nF, D in Dinv_blocks)
    return lam, float(np.sqrt(pf2))
