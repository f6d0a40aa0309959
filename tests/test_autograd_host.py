"""Host logic of the torch.autograd wrapper (no GPU): backward reuses the
handle's factors when nothing has changed them since the forward, and runs
the forward again when another solve has.  A stand-in handle with the
binding's call signatures counts the calls; it computes nothing of the
method."""
import types

import pytest

torch = pytest.importorskip("torch")

from paper_2302_10917_amd import autograd  # noqa: E402


class CountingMesh:
    def __init__(self):
        self.sizes = types.SimpleNamespace(n_trace=4, n_local=6, n_macro=2)
        self.state_gen = 0
        self.calls = {"factor_local": 0, "solve": 0, "recover_local": 0, "adjoint": 0,
                      "fold_operator": 0}

    def factor_local(self, kappa, beta, tau):
        self.state_gen += 1
        self.calls["factor_local"] += 1

    def fold_operator(self):
        self.state_gen += 1
        self.calls["fold_operator"] += 1

    def solve(self, f, g, lam, **kw):
        self.state_gen += 1
        self.calls["solve"] += 1

    def recover_local(self, lam, qu):
        self.calls["recover_local"] += 1
        qu.zero_()

    def adjoint(self, lam, qu, dJ, psi_lam, psi_U, dk, db, **kw):
        self.calls["adjoint"] += 1
        dk.fill_(1.0)
        db.fill_(2.0)


def _run(mesh, kappa, beta, folded=False):
    return autograd.solve(kappa, beta, mesh, None, None, rtol=1e-10, restart=10, folded=folded)


@pytest.mark.parametrize("folded", [False, True])
def test_backward_after_single_forward_does_not_refactor(folded):
    mesh = CountingMesh()
    kappa = torch.ones(2, dtype=torch.float64, requires_grad=True)
    beta = torch.tensor([1.0, 1.0], dtype=torch.float64, requires_grad=True)
    qu = _run(mesh, kappa, beta, folded)
    qu.sum().backward()
    assert mesh.calls["factor_local"] == 1 and mesh.calls["solve"] == 1
    assert mesh.calls["adjoint"] == 1
    assert mesh.last_backward_reforwarded is False
    assert torch.equal(kappa.grad, torch.ones(2, dtype=torch.float64))
    assert torch.equal(beta.grad, torch.full((2,), 2.0, dtype=torch.float64))


def test_backward_after_another_solve_restores_the_factors():
    mesh = CountingMesh()
    k1 = torch.ones(2, dtype=torch.float64, requires_grad=True)
    k2 = torch.full((2,), 3.0, dtype=torch.float64, requires_grad=True)
    beta = torch.tensor([1.0, 1.0], dtype=torch.float64)
    qu1 = _run(mesh, k1, beta)
    qu2 = _run(mesh, k2, beta)
    qu1.sum().backward()          # the handle now holds k2's factors
    assert mesh.last_backward_reforwarded is True
    assert mesh.calls["factor_local"] == 3
    qu2.sum().backward()          # and now k1's again
    assert mesh.last_backward_reforwarded is True
    assert mesh.calls["factor_local"] == 4
