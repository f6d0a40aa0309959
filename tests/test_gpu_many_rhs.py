"""GPU parity of the trace operator applied to many vectors at once.

mhdg_apply_trace_operator_many carries several vectors through each macro's
local solve; per vector it is the same operator as the single apply (steps
1-4 of section 3.3.2).  Every output vector must equal the oracle's S lambda
(D^-1 S lambda) to the FP64 bound (relative 1e-10) and the single-vector GPU
apply to 1e-12, for vector counts that leave ragged groups in every size
class (8, 4, 2 and 1 vectors per wavefront, and from 12 vectors on macros of
up to 1024 unknowns 16 vectors per workgroup, whose sweeps run on MFMA), on
uniform and mixed-level meshes and with coefficient instances.  Error paths
are checked through the C-ABI.
"""

import numpy as np
import pytest

from oracle import hdg
from paper_2302_10917_amd import inputs

import parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_10917_amd import mhdg  # noqa: E402

DEV = "cuda"


def gpu(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# (mesh n, levels, p): local sizes 24..180 (8 vectors per wavefront), 273 (8),
# 975 (4), 1683 (2) and the uneven levels 1..4 with 84, 273, 975 and 3675
# (8, 8, 4, 1); 11 vectors leave a partial last group in every class, and 19
# a partial second group of the 16-vector workgroups (N_K <= 1024).
CASES = {"mixed_p2": (3, "mixed", 2), "uniform_r2_p3": (3, 2, 3), "r3_p3": (2, 3, 3),
         "r3_p4": (2, 3, 4), "mixed_r1to4_p3": (2, "mixed4", 3)}


def _case(name):
    n, lev, p = CASES[name]
    xy, tri = inputs.structured_mesh(n, jitter=0.1, seed=7)
    if lev == "mixed":
        r = inputs.random_levels(len(tri), (0, 1, 2), seed=3)
    elif lev == "mixed4":
        r = inputs.random_levels(len(tri), (1, 2, 3, 4), seed=3)
    else:
        r = lev
    kap = 0.2 * inputs.lognormal_kappa(len(tri), 0.3, seed=9)
    return xy, tri, r, p, kap, (1.0, -0.4)


@pytest.mark.parametrize("name", list(CASES))
def test_many_matches_oracle_and_single(name):
    xy, tri, r, p, kap, beta = _case(name)
    print(f"\n[apply many {name}]", flush=True)
    orc = hdg.Oracle(xy, tri, r, p, kap, beta, 1.0)
    m = mhdg.MacroMesh(xy, tri, r, p)
    m.factor_local(gpu(kap), beta, 1.0)
    n = orc.topo.n_trace
    for n_rhs in (11, 19):   # 8+3, 4+4+3, 2*5+1, 11*1; 16+3 (MFMA sweeps), 8+8+3, ...
        _many_against_single_and_oracle(orc, m, n, n_rhs)


def _many_against_single_and_oracle(orc, m, n, n_rhs):
    lam_h = np.stack([inputs.random_vector(n, seed=20 + v) for v in range(n_rhs)])
    lam = gpu(lam_h)
    out = torch.full((n_rhs, n), np.nan, dtype=torch.float64, device=DEV)
    one = torch.empty(n, dtype=torch.float64, device=DEV)
    for flags, prec in ((0, False), (mhdg.MHDG_PRECONDITION, True)):
        m.apply_trace_operator_many(lam, out, flags)
        outh = host(out)
        for v in range(n_rhs):
            m.apply_trace_operator(lam[v], one, flags)
            assert P.faces(outh[v], host(one), orc.topo) <= 1e-12, (flags, v)
        for v in (0, 5, n_rhs - 1):
            err = P.faces(outh[v], orc.apply(lam_h[v], precondition=prec), orc.topo)
            print(f"  flags={flags} vector {v}: {err:.2e} against the oracle", flush=True)
            assert err <= 1e-10, (flags, v)


@pytest.mark.parametrize("n_rhs", [1, 3, 16, 40])
def test_many_vector_counts(n_rhs):
    """One vector, fewer than a group, one full group and three groups (the
    last one partial) of the 16-vector workgroups, against single applies."""
    xy, tri, r, p, kap, beta = _case("mixed_p2")
    m = mhdg.MacroMesh(xy, tri, r, p)
    m.factor_local(gpu(kap), beta, 1.0)
    n = m.sizes.n_trace
    lam = gpu(np.stack([inputs.random_vector(n, seed=40 + v) for v in range(n_rhs)]))
    out = torch.empty((n_rhs, n), dtype=torch.float64, device=DEV)
    one = torch.empty(n, dtype=torch.float64, device=DEV)
    m.apply_trace_operator_many(lam, out, mhdg.MHDG_PRECONDITION)
    outh = host(out)
    topo = hdg.Topology(xy, tri, r, p)
    for v in range(n_rhs):
        m.apply_trace_operator(lam[v], one, mhdg.MHDG_PRECONDITION)
        assert P.faces(outh[v], host(one), topo) <= 1e-12, v


@pytest.mark.parametrize("name,precision", [("r3_p3", mhdg.MHDG_FP64),
                                            ("mixed_r1to4_p3", mhdg.MHDG_FP64),
                                            ("mixed_r1to4_p3", mhdg.MHDG_QELIM),
                                            ("mixed_p2", mhdg.MHDG_QELIM)])
def test_folded_many_matches_single_and_oracle(name, precision):
    """MHDG_FOLDED: T_K read once per group of 8 vectors; 11 vectors (a full
    and a partial group) against single folded applies (1e-12) and the
    oracle (1e-10)."""
    xy, tri, r, p, kap, beta = _case(name)
    orc = hdg.Oracle(xy, tri, r, p, kap, beta, 1.0)
    m = mhdg.MacroMesh(xy, tri, r, p)
    m.factor_local(gpu(kap), beta, 1.0, precision=precision)
    m.fold_operator()
    n = orc.topo.n_trace
    lam_h = np.stack([inputs.random_vector(n, seed=90 + v) for v in range(11)])
    lam = gpu(lam_h)
    out = torch.empty((11, n), dtype=torch.float64, device=DEV)
    one = torch.empty(n, dtype=torch.float64, device=DEV)
    for flags, prec in ((mhdg.MHDG_FOLDED, False),
                        (mhdg.MHDG_FOLDED | mhdg.MHDG_PRECONDITION, True)):
        m.apply_trace_operator_many(lam, out, flags)
        outh = host(out)
        for v in range(11):
            m.apply_trace_operator(lam[v], one, flags)
            assert P.faces(outh[v], host(one), orc.topo) <= 1e-12, (flags, v)
        for v in (0, 10):
            assert P.faces(outh[v], orc.apply(lam_h[v], precondition=prec), orc.topo) <= 1e-10, (flags, v)


def test_many_with_instances():
    """Coefficient instances: each vector spans every instance's trace."""
    xy, tri, r, p, _, _ = _case("mixed_p2")
    n_inst = 3
    m = mhdg.MacroMesh(xy, tri, r, p)
    n_one = m.sizes.n_trace
    m.set_instances(n_inst)
    kap = np.concatenate([0.1 * (i + 1) * inputs.lognormal_kappa(len(tri), 0.3, seed=9 + i)
                          for i in range(n_inst)])
    beta = np.array([[1.0, -0.4], [0.3, 0.8], [-0.6, 0.2]])
    m.factor_local(gpu(kap), beta, 1.0)
    n = m.sizes.n_trace
    assert n == n_inst * n_one
    lam_h = np.stack([inputs.random_vector(n, seed=60 + v) for v in range(5)])
    out = torch.empty((5, n), dtype=torch.float64, device=DEV)
    one = torch.empty(n, dtype=torch.float64, device=DEV)
    m.apply_trace_operator_many(gpu(lam_h), out, mhdg.MHDG_PRECONDITION)
    outh = host(out)
    topo = hdg.Topology(xy, tri, r, p)
    for v in range(5):
        m.apply_trace_operator(gpu(lam_h[v]), one, mhdg.MHDG_PRECONDITION)
        # n_inst instances back to back: P.faces compares each one face by face
        assert P.faces(outh[v], host(one), topo) <= 1e-12, v
    # instance 1 of vector 2 against the oracle of that instance
    i, v = 1, 2
    orc = hdg.Oracle(xy, tri, r, p, kap[i * len(tri):(i + 1) * len(tri)], tuple(beta[i]), 1.0)
    seg = slice(i * n_one, (i + 1) * n_one)
    assert P.faces(outh[v][seg], orc.apply(lam_h[v][seg], precondition=True), orc.topo) <= 1e-10


def test_many_errors():
    """Argument and state errors come back as status codes; n_rhs = 0 is a
    no-op that leaves out untouched."""
    xy, tri, r, p, kap, beta = _case("mixed_p2")
    m = mhdg.MacroMesh(xy, tri, r, p)
    lib, h = m._lib, m.h
    n = m.sizes.n_trace
    lam = gpu(np.stack([inputs.random_vector(n, seed=1), inputs.random_vector(n, seed=2)]))
    out = torch.zeros((2, n), dtype=torch.float64, device=DEV)
    ws = torch.empty(int(lib.mhdg_apply_many_ws_bytes(h, 2)), dtype=torch.uint8, device=DEV)
    assert ws.numel() > 0 and lib.mhdg_apply_many_ws_bytes(h, 4) == 2 * ws.numel()
    assert lib.mhdg_apply_many_ws_bytes(h, -1) == 0
    s = torch.cuda.current_stream().cuda_stream

    def call(n_rhs, a, b, flags, w, nbytes):
        return lib.mhdg_apply_trace_operator_many(h, n_rhs, a, b, flags, w, nbytes, s)

    P = lambda t: t.data_ptr()  # noqa: E731
    assert call(2, P(lam), P(out), 0, P(ws), ws.numel()) == 7          # before factor_local
    m.factor_local(gpu(kap), beta, 1.0)
    assert call(-1, P(lam), P(out), 0, P(ws), ws.numel()) == 1
    assert call(2, P(lam), P(out), mhdg.MHDG_TRANSPOSE, P(ws), ws.numel()) == 1
    assert call(2, P(lam), P(out), mhdg.MHDG_GRAPH, P(ws), ws.numel()) == 1
    assert call(2, P(lam), P(out), mhdg.MHDG_FOLDED, P(ws), ws.numel()) == 7  # not folded
    assert call(2, None, P(out), 0, P(ws), ws.numel()) == 1
    assert call(2, P(lam), P(lam[1:]), 0, P(ws), ws.numel()) == 1      # overlapping ranges
    assert call(2, P(lam), P(out), 0, P(ws), ws.numel() - 8) == 5      # workspace too small
    assert call(2, P(lam), P(out), 0, None, 0) == 5
    assert call(0, P(lam), P(out), 0, None, 0) == 0
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    assert call(2, P(lam), P(out), mhdg.MHDG_PRECONDITION, P(ws), ws.numel()) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all()) and float(out.abs().max()) > 0.0
    m.factor_local(gpu(kap), beta, 1.0, precision=mhdg.MHDG_FP32)
    assert call(2, P(lam), P(out), 0, P(ws), ws.numel()) == 7
    m.factor_local(gpu(kap), beta, 1.0, precision=mhdg.MHDG_QELIM)
    assert call(2, P(lam), P(out), 0, P(ws), ws.numel()) == 7
    assert b"FP64" in lib.mhdg_last_error(h)
