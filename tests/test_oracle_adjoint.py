"""Pin of the oracle adjoint: central finite differences of the oracle's own
forward solve (a different computation: no adjoint system, no derivative
matrices)."""
import numpy as np

from oracle import adjoint, hdg
from paper_2302_10917_amd import inputs


def _setup(seed=5):
    xy, tri = inputs.structured_mesh(2, jitter=0.1, seed=3)
    kappa = inputs.lognormal_kappa(len(tri), 0.5, seed=seed)
    beta = np.array([1.0, 1.0])
    ex = inputs.sin_sin(1.0, (1.0, 1.0))          # f fixed: kappa = 1, a = (1, 1)
    return xy, tri, kappa, beta, ex


def _J(xy, tri, kappa, beta, ex, u_obs, r=1, p=2):
    o = hdg.Oracle(xy, tri, r, p, kappa, beta, 1.0)
    f, g = o.sample(ex)
    K, F, _ = adjoint.full_system(o, f, g)
    import scipy.sparse.linalg as spla
    X = spla.splu(K).solve(F)
    U = [X[o.topo.local_off[e]:o.topo.local_off[e + 1]] for e in range(o.topo.n_macro)]
    return adjoint.objective(o, U, u_obs)


def test_adjoint_gradient_matches_central_differences():
    xy, tri, kappa, beta, ex = _setup()
    # u_obs: the solution for a perturbed kappa
    eta = np.random.default_rng(55).standard_normal(len(tri))
    o_obs = hdg.Oracle(xy, tri, 1, 2, kappa * np.exp(0.1 * eta), beta, 1.0)
    fo, go = o_obs.sample(ex)
    _, Uo, _ = o_obs.solve(fo, go)
    u_obs = [Uo[K][2 * int(o_obs.topo.Q[K]):] for K in range(len(tri))]
    # a non-trivial Dirichlet trace exercises the data term of dJ/da
    ex2 = inputs.exp_sin(1.0, (1.0, 1.0))
    o = hdg.Oracle(xy, tri, 1, 2, kappa, beta, 1.0)
    f, g = o.sample(ex2)
    J, dk, db, _, _, _, _ = adjoint.gradient(o, f, g, u_obs)
    h = 1e-6
    for K in (0, 3, 7):
        kp, km = kappa.copy(), kappa.copy()
        kp[K] *= 1 + h
        km[K] *= 1 - h
        fd = (_J(xy, tri, kp, beta, ex2, u_obs) - _J(xy, tri, km, beta, ex2, u_obs)) / (2 * h * kappa[K])
        assert abs(fd - dk[K]) <= 1e-6 * max(abs(fd), 1e-3 * abs(J)), (K, fd, dk[K])
    for d in range(2):
        bp, bm = beta.copy(), beta.copy()
        bp[d] += h
        bm[d] -= h
        fd = (_J(xy, tri, kappa, bp, ex2, u_obs) - _J(xy, tri, kappa, bm, ex2, u_obs)) / (2 * h)
        assert abs(fd - db[d]) <= 1e-6 * max(abs(fd), 1e-3 * abs(J)), (d, fd, db[d])
