"""GPU checks of the hipGraph-captured apply.

The captured apply (every size class and instance, then the face combine)
must give the eager launches' result bit for bit on every replay, with the
program's own eager work, other applies and synchronisations between the
replays and with the input vector rewritten in place; a GMRES solve that
replays the graph every iteration must give the same iterates as one that
launches eagerly.
"""
import numpy as np
import pytest

from paper_2302_10917_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_10917_amd import mhdg  # noqa: E402

DEV = "cuda"


def gpu(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device=DEV)


def _mesh(n_inst):
    xy, tri = inputs.structured_mesh(3, jitter=0.1, seed=7)
    r = inputs.random_levels(len(tri), (0, 1, 2), seed=3)
    kap_i, beta = inputs.coefficient_instances(n_inst, seed=33)
    field = inputs.lognormal_kappa(len(tri), 0.3, seed=9)
    kappa = np.concatenate([k * field for k in kap_i])
    m = mhdg.MacroMesh(xy, tri, r, 2)
    if n_inst > 1:
        m.set_instances(n_inst)
    m.factor_local(gpu(kappa), beta if n_inst > 1 else beta[0], 1.0)
    return m, kap_i, beta


@pytest.mark.parametrize("n_inst", [1, 2])
@pytest.mark.parametrize("flags", [0, 1, 3])
def test_graph_replays_match_eager_launches(n_inst, flags):
    m, _, _ = _mesh(n_inst)
    n = m.sizes.n_trace
    lam = gpu(inputs.random_vector(n, seed=1))
    out_g = torch.empty(n, dtype=torch.float64, device=DEV)
    out_e = torch.empty(n, dtype=torch.float64, device=DEV)
    other = gpu(inputs.random_vector(n, seed=2))
    other_out = torch.empty(n, dtype=torch.float64, device=DEV)
    for rep in range(5):
        m.apply_trace_operator(lam, out_g, flags | mhdg.MHDG_GRAPH)
        # eager work between replays: another apply into other buffers, a sync
        m.apply_trace_operator(other, other_out, flags)
        torch.cuda.synchronize()
        m.apply_trace_operator(lam, out_e, flags)
        torch.cuda.synchronize()
        assert torch.equal(out_g, out_e), rep
        # rewrite the captured input in place: the next replay must see it
        lam.mul_(-0.5).add_(other)


def test_solve_with_graph_equals_eager_solve():
    m, kap_i, beta = _mesh(2)
    node, bnd = m.sample_points()
    s = m.sizes
    nn, nb = s.n_nodes // 2, s.n_bnd_points // 2
    f = np.empty(s.n_nodes)
    g = np.empty(s.n_bnd_points)
    for i in range(2):
        ex = inputs.exp_sin(float(kap_i[i]), beta[i])
        f[i * nn:(i + 1) * nn] = ex.f(node[i * nn:(i + 1) * nn, 0], node[i * nn:(i + 1) * nn, 1])
        g[i * nb:(i + 1) * nb] = ex.u(bnd[i * nb:(i + 1) * nb, 0], bnd[i * nb:(i + 1) * nb, 1])
    res = []
    for graph in (True, False, True):
        lam = torch.zeros(s.n_trace, dtype=torch.float64, device=DEV)
        m.solve(gpu(f), gpu(g), lam, rtol=1e-11, restart=20, max_iter=5000, graph=graph)
        res.append((lam.clone(), [x["iterations"] for x in m.last_solve_infos]))
    for lam, its in res[1:]:
        assert its == res[0][1]
        assert torch.equal(lam, res[0][0])
