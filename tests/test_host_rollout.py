"""Host logic of the autograd rollout (no GPU): a rollout whose tape was
replaced by a later rollout on the same Sim refuses its backward pass instead
of returning the later rollout's gradients."""
import numpy as np
import pytest

from paper_2311_16080_amd import lbm


class _FakeSim:
    """Stands in for lbm.Sim: records the tape identity the way the library
    does (one more per tape_begin) and returns fixed moments and gradients."""
    storage = "f64"
    tau = 0.6

    def __init__(self, torch):
        self.torch = torch
        self.tid = 0
        self.backward_calls = 0

    def set_params(self, tau=None, faces=None):
        pass

    def set_solid_fraction(self, s):
        pass

    def set_force(self, *args):
        pass

    def init_equilibrium(self, rho=None, u=None):
        pass

    def tape_begin(self, K, n):
        self.tid += 1

    def step(self, n):
        pass

    def tape_end(self):
        pass

    def tape_id(self):
        return self.tid

    def moments(self, dtype=None):
        return self.torch.ones(4, dtype=dtype), self.torch.zeros(2, 4, dtype=dtype)

    def backward(self, g_rho, g_u, want_s=False):
        self.backward_calls += 1
        return None, np.array([2.5]), np.zeros((1, 6, 3))


def test_rollout_refuses_a_replaced_tape():
    torch = pytest.importorskip("torch")
    sim = _FakeSim(torch)
    tau1 = torch.tensor(0.6, dtype=torch.float64, requires_grad=True)
    tau2 = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    _, u1 = lbm.rollout(sim, 4, 2, tau=tau1)
    _, u2 = lbm.rollout(sim, 4, 2, tau=tau2)
    with pytest.raises(lbm.LbmError) as err:
        u1.sum().backward()
    assert err.value.code == lbm.LBM_ESTATE
    assert sim.backward_calls == 0
    # the rollout that owns the current tape differentiates normally
    u2.sum().backward()
    assert sim.backward_calls == 1
    assert float(tau2.grad) == 2.5
    assert tau1.grad is None
