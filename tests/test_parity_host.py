"""The blockwise comparisons of tests/parity.py fail the mistakes they are
for: a wrong block whose values are small, and a wrong field of one macro."""
import numpy as np

from oracle import hdg
from paper_2302_10917_amd import inputs

import parity as P


def _topo():
    xy, tri = inputs.structured_mesh(2)
    return hdg.Topology(xy, tri, 1, 2)


def test_small_face_wrong_fails_while_the_whole_vector_norm_passes():
    topo = _topo()
    b = inputs.random_vector(topo.n_trace, seed=1)
    sz = P.face_sizes(topo)
    b[:sz[0]] *= 1e-6                       # a face with small values
    a = b.copy()
    a[:sz[0]] *= 1.5                        # ... computed 50% wrong
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-6   # normwise: invisible
    assert P.faces(a, b, topo) > 1e-5
    assert P.faces(b * (1 + 1e-14), b, topo) <= 1e-13


def test_instances_are_compared_one_by_one():
    topo = _topo()
    b = np.concatenate([inputs.random_vector(topo.n_trace, seed=s) for s in (1, 2)])
    b[topo.n_trace:] *= 1e-8                # the second instance is small throughout
    a = b.copy()
    a[topo.n_trace:] *= 1.01
    assert P.faces(a, b, topo) > 1e-3


def test_wrong_field_of_one_macro_fails():
    topo = _topo()
    nl = int(topo.local_off[-1])
    b = inputs.random_vector(nl, seed=3)
    a = b.copy()
    q = int(topo.Q[1])
    lo = int(topo.local_off[1])
    a[lo + q:lo + 2 * q] += 1e-8 * np.abs(b[lo:lo + 3 * q]).max()   # q_y of macro 1
    assert P.macros(a, b, topo) > 1e-10
    assert P.fields(a[lo:lo + 3 * q], b[lo:lo + 3 * q]) > 1e-10
    assert P.macros(b, b, topo) == 0.0


def test_entries_and_blocks():
    b = np.array([1.0, -2.0, 1e-9, 3.0])
    a = b.copy()
    a[2] = 2e-9
    assert P.entries(a, b) > 1e-9
    assert P.blocks(a, b, [2, 1, 1]) > 1e-9
    assert P.blocks(a, b, [2, 2]) < 1e-9     # the block norm hides it: blocks are the unit
    assert P.entries(b, b) == 0.0
