"""GPU parity of coefficient-instance batching.

One handle carries several instances (kappa, a) of a mesh with uneven
levels; every vector is instance-major.  Checks: the batched operator and
local solves against the oracle of each instance (relative 1e-10, the FP64
bound); the batched solve against the oracle's direct solve per instance
(rtol 1e-13 -> relative 1e-10); the batched solve against single-instance
solves of the same data (the per-instance Krylov recurrences use the same
arithmetic, so the results agree to rounding, here required to 1e-13); a
zero-data instance inside a batch (masked from the first iteration, its
trace exactly zero); and the rejected combinations.
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


N_INST = 3


def _problem(n=3, p=2, levels=(0, 1, 2), n_inst=N_INST):
    xy, tri = inputs.structured_mesh(n, jitter=0.1, seed=7)
    r = inputs.random_levels(len(tri), levels, seed=3)
    kap_i, beta = inputs.coefficient_instances(n_inst, seed=33)
    field = inputs.lognormal_kappa(len(tri), 0.3, seed=9)
    kappa = np.stack([k * field for k in kap_i])          # [n_inst][n_macro]
    return xy, tri, r, p, kappa, beta, kap_i


@pytest.fixture(scope="module")
def batch():
    xy, tri, r, p, kappa, beta, kap_i = _problem()
    print(f"\n[batched n_inst={N_INST} n_macro={len(tri)}]", flush=True)
    m = mhdg.MacroMesh(xy, tri, r, p)
    one = m.sizes
    m.set_instances(N_INST)
    m.factor_local(gpu(kappa.ravel()), beta, 1.0)
    orcs = [hdg.Oracle(xy, tri, r, p, kappa[i], beta[i], 1.0) for i in range(N_INST)]
    return m, one, orcs, (xy, tri, r, p, kappa, beta, kap_i)


def test_sizes_are_totals(batch):
    m, one, _, _ = batch
    s = m.sizes
    assert s.n_instances == N_INST
    for f in ("n_macro", "n_trace", "n_local", "n_nodes", "n_bnd_points", "n_faces"):
        assert getattr(s, f) == N_INST * getattr(one, f), f


def test_batched_apply_and_local_solve_match_oracle(batch):
    m, one, orcs, _ = batch
    nt, nl = one.n_trace, one.n_local
    lam = inputs.random_vector(N_INST * nt, seed=1)
    out = torch.empty(N_INST * nt, dtype=torch.float64, device=DEV)
    for flags, prec in ((0, False), (mhdg.MHDG_PRECONDITION, True)):
        m.apply_trace_operator(gpu(lam), out, flags)
        o = host(out)
        for i, orc in enumerate(orcs):
            sl = slice(i * nt, (i + 1) * nt)
            assert P.faces(o[sl], orc.apply(lam[sl], precondition=prec), orc.topo) <= 1e-10, (i, flags)
    x = inputs.random_vector(N_INST * nl, seed=11)
    y = torch.empty(len(x), dtype=torch.float64, device=DEV)
    m.local_solve(gpu(x), y)
    yh = host(y)
    for i, orc in enumerate(orcs):
        topo = orc.topo
        for e in (0, topo.n_macro // 2, topo.n_macro - 1):
            lo, hi = i * nl + topo.local_off[e], i * nl + topo.local_off[e + 1]
            assert P.fields(yh[lo:hi], orc.local_solve(e, x[lo:hi])) <= 1e-10, (i, e)


def _data(m, beta, kap_i, n_inst):
    node, bnd = m.sample_points()
    s = m.sizes
    nn, nb = s.n_nodes // n_inst, s.n_bnd_points // n_inst
    f = np.empty(s.n_nodes)
    g = np.empty(s.n_bnd_points)
    for i in range(n_inst):
        ex = inputs.exp_sin(float(kap_i[i]), beta[i])
        f[i * nn:(i + 1) * nn] = ex.f(node[i * nn:(i + 1) * nn, 0], node[i * nn:(i + 1) * nn, 1])
        g[i * nb:(i + 1) * nb] = ex.u(bnd[i * nb:(i + 1) * nb, 0], bnd[i * nb:(i + 1) * nb, 1])
    return f, g


def test_batched_solve_matches_oracle_per_instance(batch):
    m, one, orcs, (xy, tri, r, p, kappa, beta, kap_i) = batch
    f, g = _data(m, beta, kap_i, N_INST)
    lam = torch.zeros(m.sizes.n_trace, dtype=torch.float64, device=DEV)
    m.solve(gpu(f), gpu(g), lam, rtol=1e-13, restart=300, max_iter=5000)
    infos = m.last_solve_infos
    assert len(infos) == N_INST
    qu = torch.empty(m.sizes.n_local, dtype=torch.float64, device=DEV)
    res = torch.empty(m.sizes.n_trace, dtype=torch.float64, device=DEV)
    m.recover_local(lam, qu, res)
    lh, uh, rh = host(lam), host(qu), host(res)
    nt, nl = one.n_trace, one.n_local
    for i, orc in enumerate(orcs):
        assert infos[i]["status"] == 0 and infos[i]["rel_res_prec"] <= 1e-13
        ex = inputs.exp_sin(float(kap_i[i]), beta[i])
        fo, go = orc.sample(ex)
        lam_o, U_o, _ = orc.solve(fo, go)
        assert P.faces(lh[i * nt:(i + 1) * nt], lam_o, orc.topo) <= 1e-10, i
        assert P.macros(uh[i * nl:(i + 1) * nl], np.concatenate(U_o), orc.topo) <= 1e-10, i
        _, fhat, _ = orc.condensed(fo, go)
        assert np.linalg.norm(rh[i * nt:(i + 1) * nt]) <= 1e-10 * np.linalg.norm(fhat)


def test_batched_solve_equals_single_instance_solves(batch):
    """Lockstep GMRES with masking reproduces each instance's own solve:
    the same iteration count and the same iterate to rounding."""
    m, one, _, (xy, tri, r, p, kappa, beta, kap_i) = batch
    f, g = _data(m, beta, kap_i, N_INST)
    lam = torch.zeros(m.sizes.n_trace, dtype=torch.float64, device=DEV)
    m.solve(gpu(f), gpu(g), lam, rtol=1e-10, restart=25, max_iter=5000)
    infos = m.last_solve_infos
    lh = host(lam)
    nt, nn, nb = one.n_trace, one.n_nodes, one.n_bnd_points
    its = []
    topo = hdg.Topology(xy, tri, r, p)
    for i in range(N_INST):
        s1 = mhdg.MacroMesh(xy, tri, r, p)
        s1.factor_local(gpu(kappa[i]), beta[i], 1.0)
        l1 = torch.zeros(nt, dtype=torch.float64, device=DEV)
        s1.solve(gpu(f[i * nn:(i + 1) * nn]), gpu(g[i * nb:(i + 1) * nb]), l1, rtol=1e-10,
                 restart=25, max_iter=5000)
        its.append(s1.last_solve_info["iterations"])
        assert infos[i]["iterations"] == its[-1], (i, infos[i]["iterations"], its[-1])
        assert P.faces(lh[i * nt:(i + 1) * nt], host(l1), topo) <= 1e-13, i
    # the instances need different iteration counts, so masking was exercised
    assert len(set(its)) > 1, its


def test_zero_instance_in_batch_stays_zero(batch):
    m, one, orcs, (xy, tri, r, p, kappa, beta, kap_i) = batch
    f, g = _data(m, beta, kap_i, N_INST)
    nn, nb, nt = one.n_nodes, one.n_bnd_points, one.n_trace
    f[nn:2 * nn] = 0.0
    g[nb:2 * nb] = 0.0
    lam = torch.full((m.sizes.n_trace,), 7.0, dtype=torch.float64, device=DEV)
    m.solve(gpu(f), gpu(g), lam, rtol=1e-12, restart=300, max_iter=5000)
    lh = host(lam)
    assert np.all(lh[nt:2 * nt] == 0.0)
    assert m.last_solve_infos[1]["iterations"] == 0
    ex = inputs.exp_sin(float(kap_i[2]), beta[2])
    fo, go = orcs[2].sample(ex)
    lam_o, _, _ = orcs[2].solve(fo, go)
    assert P.faces(lh[2 * nt:3 * nt], lam_o, orcs[2].topo) <= 1e-9


def test_rejected_combinations():
    xy, tri, r, p, kappa, beta, kap_i = _problem(n=2, levels=(1,), n_inst=2)
    m = mhdg.MacroMesh(xy, tri, r, p)
    m.set_instances(2)
    m.factor_local(gpu(kappa.ravel()), beta, 1.0, precision=mhdg.MHDG_FP32)
    f, g = _data(m, beta, kap_i, 2)
    lam = torch.zeros(m.sizes.n_trace, dtype=torch.float64, device=DEV)
    with pytest.raises(mhdg.MhdgError) as e:
        m.solve(gpu(f), gpu(g), lam)
    assert e.value.status == 7
    m.factor_local(gpu(kappa.ravel()), beta, 1.0)
    m.solve(gpu(f), gpu(g), lam, rtol=1e-10, restart=100)
    qu = torch.empty(m.sizes.n_local, dtype=torch.float64, device=DEV)
    m.recover_local(lam, qu)
    n_l, n_t = m.sizes.n_local, m.sizes.n_trace
    z = torch.zeros(n_l, dtype=torch.float64, device=DEV)
    with pytest.raises(mhdg.MhdgError) as e:
        m.adjoint(lam, qu, z, torch.empty(n_t, dtype=torch.float64, device=DEV),
                  torch.empty(n_l, dtype=torch.float64, device=DEV),
                  torch.empty(m.sizes.n_macro, dtype=torch.float64, device=DEV),
                  torch.empty(2, dtype=torch.float64, device=DEV))
    assert e.value.status == 7
