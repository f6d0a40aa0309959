"""GPU parity of the reduced-precision form: FP32 local factors on MFMA with
FP64 iterative refinement of the whole hybridised system.

The FP32-factor operator itself is only an approximation (checked loosely);
the refined solve must reach the FP64 oracle's solution to the FP64 bar
(relative 1e-10 for lambda and U after local refinement) when run to a tight
refinement tolerance.
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


CASES = {
    "r2_p3_kappa1e-3": (3, 0.0, 2, 3, 1e-3, (1.0, 0.5)),
    "r3_p3_kappa1e-2": (2, 0.0, 3, 3, 1e-2, (1.0, 0.5)),
    "mixed_p2_jitter": (3, 0.1, "mixed", 2, 0.1, (-0.5, 1.0)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[fp32 case {request.param}]", flush=True)
    n, jit, lev, p, kappa, beta = CASES[request.param]
    xy, tri = inputs.structured_mesh(n, jitter=jit, seed=7)
    r = inputs.random_levels(len(tri), (0, 1, 2), seed=3) if lev == "mixed" else lev
    orc = hdg.Oracle(xy, tri, r, p, kappa, beta, 1.0)
    m = mhdg.MacroMesh(xy, tri, r, p)
    m.factor_local(gpu(np.full(len(tri), kappa)), beta, 1.0, precision=mhdg.MHDG_FP32)
    return orc, m, kappa, beta


def test_fp32_factor_operator_is_close(case):
    orc, m, _, _ = case
    lam = inputs.random_vector(orc.topo.n_trace, seed=1)
    out = torch.empty(orc.topo.n_trace, dtype=torch.float64, device=DEV)
    m.apply_trace_operator(gpu(lam), out, mhdg.MHDG_PRECONDITION)
    err = P.faces(host(out), orc.apply(lam, precondition=True), orc.topo)
    assert err < 1e-3, err        # FP32 factors: an approximation only


def test_fp32_refined_solve_matches_fp64_oracle(case):
    orc, m, kappa, beta = case
    topo = orc.topo
    node, bnd = m.sample_points()
    ex = inputs.exp_sin(kappa, beta)
    fo, go = orc.sample(ex)
    lam_o, U_o, _ = orc.solve(fo, go)
    lam = torch.zeros(topo.n_trace, dtype=torch.float64, device=DEV)
    info = m.solve(gpu(ex.f(node[:, 0], node[:, 1])), gpu(ex.u(bnd[:, 0], bnd[:, 1])), lam,
                   rtol=1e-13, restart=300, max_iter=20000, inner_rtol=1e-4)
    print(f"  outer={info.outer_iterations} inner={info.iterations} rel={info.rel_res_prec:.2e}")
    assert info.status == 0 and info.outer_iterations >= 2
    assert P.faces(host(lam), lam_o, topo) <= 1e-10
    qu = torch.empty(int(topo.local_off[-1]), dtype=torch.float64, device=DEV)
    res = torch.empty(topo.n_trace, dtype=torch.float64, device=DEV)
    m.recover_local(lam, qu, res)
    U = np.concatenate(U_o)
    assert P.macros(host(qu), U, topo) <= 1e-10
    S, fhat, _ = orc.condensed(fo, go)
    assert np.linalg.norm(host(res)) <= 1e-10 * np.linalg.norm(fhat)


def test_fp32_solve_reaches_1e10_like_the_plain_form(case):
    """At the benchmark tolerance (1e-10) the refined solution's error against
    the FP64 oracle is of the same order as the plain FP64 solve's."""
    orc, m, kappa, beta = case
    node, bnd = m.sample_points()
    ex = inputs.exp_sin(kappa, beta)
    fo, go = orc.sample(ex)
    lam_o, _, _ = orc.solve(fo, go)
    lam = torch.zeros(orc.topo.n_trace, dtype=torch.float64, device=DEV)
    m.solve(gpu(ex.f(node[:, 0], node[:, 1])), gpu(ex.u(bnd[:, 0], bnd[:, 1])), lam,
            rtol=1e-10, restart=300, max_iter=20000)
    assert P.faces(host(lam), lam_o, orc.topo) <= 1e-7


# ---------------------------------------------------------------- BF16 factors
# FP32 LU rounded to BF16 (8-bit mantissa) for storage.  The contraction of
# the refinement measured with the oracle's own blocks for these shapes is
# about 1e-2 per step (spectral radius of I - S~^-1 S with BF16-rounded LU
# factors), so the operator is a rough approximation and the refined solve
# needs about two refinement steps per two digits.

@pytest.fixture(scope="module", params=["r2_p3_kappa1e-3", "r3_p3_kappa1e-2"])
def bf16_case(request):
    print(f"\n[bf16 case {request.param}]", flush=True)
    n, jit, lev, p, kappa, beta = CASES[request.param]
    xy, tri = inputs.structured_mesh(n, jitter=jit, seed=7)
    orc = hdg.Oracle(xy, tri, lev, p, kappa, beta, 1.0)
    m = mhdg.MacroMesh(xy, tri, lev, p)
    m.factor_local(gpu(np.full(len(tri), kappa)), beta, 1.0, precision=mhdg.MHDG_BF16)
    return orc, m, kappa, beta


def test_bf16_factor_operator_is_close(bf16_case):
    orc, m, _, _ = bf16_case
    lam = inputs.random_vector(orc.topo.n_trace, seed=1)
    out = torch.empty(orc.topo.n_trace, dtype=torch.float64, device=DEV)
    m.apply_trace_operator(gpu(lam), out, mhdg.MHDG_PRECONDITION)
    err = P.faces(host(out), orc.apply(lam, precondition=True), orc.topo)
    assert 1e-5 < err < 5e-2, err   # BF16 factors: visibly inexact, within the analysis


def test_bf16_refined_solve_matches_fp64_oracle(bf16_case):
    orc, m, kappa, beta = bf16_case
    topo = orc.topo
    node, bnd = m.sample_points()
    ex = inputs.exp_sin(kappa, beta)
    fo, go = orc.sample(ex)
    lam_o, U_o, _ = orc.solve(fo, go)
    lam = torch.zeros(topo.n_trace, dtype=torch.float64, device=DEV)
    info = m.solve(gpu(ex.f(node[:, 0], node[:, 1])), gpu(ex.u(bnd[:, 0], bnd[:, 1])), lam,
                   rtol=1e-12, restart=300, max_iter=20000, inner_rtol=1e-2, max_outer=60)
    print(f"  outer={info.outer_iterations} inner={info.iterations} rel={info.rel_res_prec:.2e}")
    assert info.status == 0 and info.outer_iterations >= 4
    assert P.faces(host(lam), lam_o, topo) <= 1e-9
    qu = torch.empty(int(topo.local_off[-1]), dtype=torch.float64, device=DEV)
    m.recover_local(lam, qu)
    assert P.macros(host(qu), np.concatenate(U_o), topo) <= 1e-9


def test_bf16_limits():
    xy, tri = inputs.structured_mesh(1)
    m = mhdg.MacroMesh(xy, tri, 4, 3)     # N_K = 3675 > 1024
    with pytest.raises(mhdg.MhdgError):
        m.factor_local(gpu(np.full(len(tri), 0.3)), (1.0, 0.5), 1.0, precision=mhdg.MHDG_BF16)


def test_bf16_at_scale_matches_fp64_operator():
    """The 8192-macro mesh: 7.8e9 factor entries, more than one dispatch's
    2^32 work-items, are all converted (the BF16 apply is finite and within
    the BF16 bound of the FP64 apply)."""
    xy, tri = inputs.structured_mesh(64)
    kap = gpu(np.full(len(tri), 1e-2))
    lam = gpu(inputs.random_vector(304000, seed=1))
    out = []
    for prec in (mhdg.MHDG_FP64, mhdg.MHDG_BF16):
        m = mhdg.MacroMesh(xy, tri, 3, 3)
        m.factor_local(kap, (1.0, 0.5), 1.0, precision=prec)
        o = torch.empty(m.sizes.n_trace, dtype=torch.float64, device=DEV)
        m.apply_trace_operator(lam, o, mhdg.MHDG_PRECONDITION)
        out.append(host(o))
        del m
        torch.cuda.empty_cache()
    assert np.all(np.isfinite(out[1]))
    # every face within 5% of the largest face norm (a bound of the BF16 storage, not parity)
    assert P.faces(out[1], out[0], hdg.Topology(xy, tri, 3, 3), floor=1.0) < 5e-2
