"""Blockwise comparison of GPU results with the oracle.

A relative norm over a whole vector lets a block with small values be wrong
without failing.  Every comparison here is made per block instead:

* a face's trace values, for a trace vector;
* one field (q_x, q_y or u) of one macro, for a local vector;
* one entry, for a gradient.

A block B passes when

    ||a_B - b_B|| <= tol * (||b_B|| + FLOOR * max_B' ||b_B'||).

FLOOR = 1e-2 covers blocks whose own values vanish, such as a face on a zero
line of the solution.  There the difference is rounding spread over the
whole vector, not a fault of that block.  Any difference above
tol * FLOOR = 1e-12 of the largest block still fails, wherever it sits.

The three fields of one macro are coupled through A_K: the rounding of a
local solve is bounded in the norm of the macro's whole vector, not field by
field.  So `fields` and `macros` measure each field against the largest
field of its macro (floor 1), which still fails a field that is wrong by
more than 1e-10 of the macro's scale.

Each function returns the worst ratio ||a_B - b_B|| / (||b_B|| +
FLOOR * max ||b_B'||), so a test asserts ``ratio <= tol``.
"""
from __future__ import annotations

import numpy as np

FLOOR = 1e-2


def worst(pairs, floor: float = FLOOR) -> float:
    """Worst blockwise ratio over (a_B, b_B) pairs."""
    pairs = [(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)) for a, b in pairs]
    if not pairs:
        return 0.0
    for a, b in pairs:
        assert a.shape == b.shape, (a.shape, b.shape)
    nb = np.array([np.linalg.norm(b) for _, b in pairs])
    err = np.array([np.linalg.norm(a - b) for a, b in pairs])
    if not np.all(np.isfinite(err)):
        return float("inf")
    den = nb + floor * nb.max()
    if den.max() == 0.0:
        return 0.0 if err.max() == 0.0 else float("inf")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0.0, err / np.where(den > 0.0, den, 1.0), np.where(err > 0, np.inf, 0.0))
    return float(r.max())


def split(v, sizes):
    """Consecutive blocks of v with the given sizes."""
    v = np.asarray(v)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    assert off[-1] == len(v), (off[-1], len(v))
    return [v[off[i]:off[i + 1]] for i in range(len(sizes))]


def face_sizes(topo):
    """Trace values per interior face, in the trace vector's order."""
    f = np.flatnonzero(np.asarray(topo.interior))
    o = np.asarray(topo.trace_off)[f]
    n = np.asarray(topo.face_nodes)[f]
    order = np.argsort(o)
    return [int(x) for x in n[order]]


def faces(a, b, topo, floor: float = FLOOR) -> float:
    """Per interior face; a and b hold one or more trace vectors back to back
    (coefficient instances or right-hand sides), each compared face by face
    with the scale taken per vector."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    n = int(topo.n_trace)
    assert a.shape == b.shape and n > 0 and len(b) % n == 0, (a.shape, b.shape, n)
    sz = face_sizes(topo)
    return max(worst(list(zip(split(a[i:i + n], sz), split(b[i:i + n], sz))), floor)
               for i in range(0, len(b), n))


MACRO_FLOOR = 1.0


def fields(a, b, floor: float = MACRO_FLOOR) -> float:
    """One macro's local vector (q_x, q_y, u; three equal fields)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert a.shape == b.shape and len(b) % 3 == 0
    q = len(b) // 3
    return worst([(a[c * q:(c + 1) * q], b[c * q:(c + 1) * q]) for c in range(3)], floor)


def macros(a, b, topo, floor: float = MACRO_FLOOR) -> float:
    """Per macro and field over whole local vectors (one or more back to back);
    each field against the largest field of its macro."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nl = int(topo.local_off[-1])
    assert a.shape == b.shape and len(b) % nl == 0, (a.shape, b.shape, nl)
    off = np.asarray(topo.local_off)
    out = 0.0
    for i in range(0, len(b), nl):
        for K in range(int(topo.n_macro)):
            lo, hi = i + int(off[K]), i + int(off[K + 1])
            out = max(out, fields(a[lo:hi], b[lo:hi], floor))
    return out


def entries(a, b, floor: float = FLOOR) -> float:
    """Per entry (gradients, per-macro scalars)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return worst(list(zip(a[:, None], b[:, None])), floor)


def blocks(a, b, sizes, floor: float = FLOOR) -> float:
    """Consecutive blocks of the given sizes (e.g. sampled faces gathered)."""
    return worst(list(zip(split(a, sizes), split(b, sizes))), floor)
