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
