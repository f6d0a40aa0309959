"""GPU parity of the transposed operator and the hand-written adjoint.

Transposed applies and A^-T solves against the oracle (relative 1e-10, per
face and per macro field).  dJ/dkappa and dJ/dbeta against the oracle
adjoint, which solves the unhybridised system and its transpose directly, at
the FP64 bar: relative 1e-10 per entry.  Both GPU solves (forward and
transposed) run to a preconditioned residual of 1e-14 there.  On this 8-macro
mesh D^-1 S (40 unknowns) has a condition number of 69, so each solve's
forward error stays below 1e-12, and the gradient, bilinear in the two solutions,
inherits about twice that.  Against central finite differences of the GPU
forward solve the bound is 1e-5 relative: the truncation error of a step of
1e-5 and the solve tolerance set it.  The torch.autograd path runs end to
end.
"""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import hdg
from paper_2302_10917_amd import inputs

import parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_10917_amd import autograd as ad  # noqa: E402
from paper_2302_10917_amd import mhdg  # noqa: E402

DEV = "cuda"


def gpu(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _problem(n=2, r=1, p=2, jitter=0.1):
    xy, tri = inputs.structured_mesh(n, jitter=jitter, seed=3)
    kappa = inputs.lognormal_kappa(len(tri), 0.5, seed=5)
    beta = np.array([1.0, 1.0])
    return xy, tri, r, p, kappa, beta


@pytest.mark.parametrize("spec", [(2, 1, 2), (3, 2, 3), (2, 3, 3)])
def test_transposed_apply_and_local_solve(spec):
    n, r, p = spec
    xy, tri, r, p, kappa, beta = _problem(n, r, p)
    orc = hdg.Oracle(xy, tri, r, p, kappa, beta, 1.0)
    m = mhdg.MacroMesh(xy, tri, r, p)
    m.factor_local(gpu(kappa), beta, 1.0)
    ex = inputs.exp_sin(1.0, beta)
    fo, go = orc.sample(ex)
    S, _, _ = orc.condensed(fo, go)
    lam = inputs.random_vector(orc.topo.n_trace, seed=4)
    out = torch.empty(orc.topo.n_trace, dtype=torch.float64, device=DEV)
    m.apply_trace_operator(gpu(lam), out, mhdg.MHDG_TRANSPOSE)
    assert P.faces(host(out), S.T @ lam, orc.topo) <= 1e-10
    m.apply_trace_operator(gpu(lam), out, mhdg.MHDG_TRANSPOSE | mhdg.MHDG_PRECONDITION)
    assert P.faces(host(out), orc.precondition(S.T @ lam), orc.topo) <= 1e-10
    x = inputs.random_vector(int(orc.topo.local_off[-1]), seed=6)
    y = torch.empty(len(x), dtype=torch.float64, device=DEV)
    m.local_solve(gpu(x), y, mhdg.MHDG_TRANSPOSE)
    yh = host(y)
    for K in range(orc.topo.n_macro):
        lo, hi = orc.topo.local_off[K], orc.topo.local_off[K + 1]
        assert P.fields(yh[lo:hi], orc.local_solve(K, x[lo:hi], transpose=True)) <= 1e-10


def _u_obs(xy, tri, r, p, kappa, beta, ex, m):
    """u_obs: the GPU solution for kappa exp(0.1 eta) (FE field, local layout)."""
    eta = np.random.default_rng(55).standard_normal(len(tri))
    node, bnd = m.sample_points()
    f = gpu(ex.f(node[:, 0], node[:, 1]))
    g = gpu(ex.u(bnd[:, 0], bnd[:, 1]))
    with torch.no_grad():
        qu_obs = ad.solve(gpu(kappa * np.exp(0.1 * eta)), torch.tensor(beta), m, f, g)
    return qu_obs.clone(), f, g


def test_adjoint_matches_oracle_adjoint():
    xy, tri, r, p, kappa, beta = _problem(2, 1, 2)
    ex = inputs.exp_sin(1.0, (1.0, 1.0))
    m = mhdg.MacroMesh(xy, tri, r, p)
    qu_obs, f, g = _u_obs(xy, tri, r, p, kappa, beta, ex, m)
    k = gpu(kappa).requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    qu = ad.solve(k, b, m, f, g, rtol=1e-14)
    J = ad.l2_misfit(m, qu, qu_obs)
    J.backward()
    # oracle adjoint with the same u_obs field
    orc = hdg.Oracle(xy, tri, r, p, kappa, beta, 1.0)
    Q = int(orc.topo.Q[0])
    uo = host(qu_obs).reshape(len(tri), 3, Q)[:, 2, :]
    fo, go = orc.sample(ex)
    Jo, dko, dbo, _, _, _, _ = oadj.gradient(orc, fo, go, [uo[K] for K in range(len(tri))])
    ek, eb = P.entries(host(k.grad), dko), P.entries(b.grad.numpy(), dbo)
    print(f"  J {abs(J.item() - Jo) / abs(Jo):.2e}  dJ/dkappa {ek:.2e}  dJ/dbeta {eb:.2e}",
          flush=True)
    assert abs(J.item() - Jo) <= 1e-10 * abs(Jo)
    assert ek <= 1e-10
    assert eb <= 1e-10


def test_adjoint_matches_central_differences_on_gpu():
    """Differentiation workload shape (r = 2, p = 2, log-normal kappa, a = (1, 1),
    f fixed, g_D = 0) on a 4x4-square mesh."""
    xy, tri, r, p, kappa, beta = _problem(4, 2, 2, jitter=0.0)
    ex = inputs.sin_sin(1.0, (1.0, 1.0))
    m = mhdg.MacroMesh(xy, tri, r, p)
    qu_obs, f, g = _u_obs(xy, tri, r, p, kappa, beta, ex, m)
    k = gpu(kappa).requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    J = ad.l2_misfit(m, ad.solve(k, b, m, f, g, 1e-13), qu_obs)
    J.backward()
    dk, db = host(k.grad), b.grad.numpy()

    def Jof(kap, bet):
        with torch.no_grad():
            qu = ad.solve(gpu(kap), torch.tensor(bet), m, f, g, 1e-13)
            return ad.l2_misfit(m, qu, qu_obs).item()

    h = 1e-5
    for K in (0, 7, 19, len(tri) - 1):
        kp, km = kappa.copy(), kappa.copy()
        kp[K] *= 1 + h
        km[K] *= 1 - h
        fd = (Jof(kp, beta) - Jof(km, beta)) / (2 * h * kappa[K])
        assert abs(fd - dk[K]) <= 1e-5 * abs(fd) + 1e-9 * abs(J.item()), (K, fd, dk[K])
    for d in range(2):
        bp, bm = beta.copy(), beta.copy()
        bp[d] += h
        bm[d] -= h
        fd = (Jof(kappa, bp) - Jof(kappa, bm)) / (2 * h)
        assert abs(fd - db[d]) <= 1e-5 * abs(fd) + 1e-9 * abs(J.item()), (d, fd, db[d])


def test_adjoint_gradient_on_a_large_mesh():
    """The gradient on a mesh of the differentiation workload's kind at 2048
    macros (32 x 32 squares, r = 2, p = 2, log-normal kappa with sigma 0.5,
    a = (1, 1), u = sin(pi x) sin(pi y), g_D = 0), J = ||u_h||^2_{L2} (u_obs =
    0, so J and its derivatives are of order one), folded applies in both
    solves.  The adjoint's dJ/dkappa and dJ/da against central differences of
    the GPU forward solve along directions that move every macro at once:
    kappa -> (1 + t) kappa (so sum_K kappa_K dJ/dkappa_K) and a_0 -> a_0 + t
    (one macro's derivative is 1/2048 of J's scale).  Solves to a
    preconditioned residual of 1e-12, t = 1e-3: truncation (t^2) and solve
    error below 1e-6 relative; the bound is 1e-5.  (At the full 32,768-macro
    size the folded solve stalls above 1e-11, so differences of full-size
    solves cannot resolve the gradient to this bound; the operators the
    gradient runs on are checked there in test_gpu_fullsize.py.)"""
    xy, tri = inputs.structured_mesh(32)
    r, p = 2, 2
    kappa = inputs.lognormal_kappa(len(tri), 0.5, seed=5)
    beta = np.array([1.0, 1.0])
    ex = inputs.sin_sin(1.0, (1.0, 1.0))
    m = mhdg.MacroMesh(xy, tri, r, p)
    s = m.sizes
    node, bnd = m.sample_points()
    f = gpu(ex.f(node[:, 0], node[:, 1]))
    g = gpu(ex.u(bnd[:, 0], bnd[:, 1]))
    kw = dict(rtol=1e-12, restart=1000, max_iter=30000, folded=True)
    qu_obs = torch.zeros(s.n_local, dtype=torch.float64, device=DEV)

    def forward(kap, bet, lam):
        m.factor_local(gpu(kap), (float(bet[0]), float(bet[1])), 1.0)
        m.fold_operator()
        info = m.solve(f, g, lam, **kw)
        print(f"  forward solve: {info.iterations} it, status {info.status}", flush=True)
        assert info.status == 0, info.status
        qu = torch.empty(s.n_local, dtype=torch.float64, device=DEV)
        m.recover_local(lam, qu)
        return qu, info.iterations

    lam0 = torch.zeros(s.n_trace, dtype=torch.float64, device=DEV)
    qu0, it0 = forward(kappa, beta, lam0)
    qt = qu0.clone().requires_grad_(True)
    J = ad.l2_misfit(m, qt, qu_obs)
    J.backward()
    dk = torch.empty(s.n_macro, dtype=torch.float64, device=DEV)
    db = torch.empty(2, dtype=torch.float64, device=DEV)
    psi_lam = torch.empty(s.n_trace, dtype=torch.float64, device=DEV)
    psi_U = torch.empty(s.n_local, dtype=torch.float64, device=DEV)
    info = m.adjoint(lam0, qu0, qt.grad.contiguous(), psi_lam, psi_U, dk, db, rtol=1e-12,
                     restart=1000, max_iter=30000, folded=True)
    print(f"  adjoint solve: {info.iterations} it, status {info.status}", flush=True)
    assert info.status == 0
    grad_scale = float((host(dk) * kappa).sum())
    grad_b0 = float(host(db)[0])
    t = 1e-3

    def Jat(kap, bet):
        lam = lam0.clone()
        qu, it = forward(kap, bet, lam)
        with torch.no_grad():
            return ad.l2_misfit(m, qu, qu_obs).item(), it

    (jp, ip), (jm, im) = Jat((1 + t) * kappa, beta), Jat((1 - t) * kappa, beta)
    fd_scale = (jp - jm) / (2 * t)
    (jp, ip2), (jm, im2) = Jat(kappa, beta + [t, 0.0]), Jat(kappa, beta - [t, 0.0])
    fd_b0 = (jp - jm) / (2 * t)
    es, eb = abs(grad_scale - fd_scale) / abs(fd_scale), abs(grad_b0 - fd_b0) / abs(fd_b0)
    print(f"  J {J.item():.6e} ({it0} it; perturbed {ip} {im} {ip2} {im2} it); "
          f"sum kappa dJ/dkappa {grad_scale:.10e} fd {fd_scale:.10e} ({es:.1e}); "
          f"dJ/da0 {grad_b0:.10e} fd {fd_b0:.10e} ({eb:.1e})", flush=True)
    assert es <= 1e-5 and eb <= 1e-5
