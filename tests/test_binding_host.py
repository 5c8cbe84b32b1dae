"""Host-side checks of the Python binding (no GPU): argument validation
before any device address reaches the library, and the guard that ties an
autograd backward to its own forward."""
import os

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_00705_amd", "libimexds.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def test_device_pointers_must_have_the_expected_length():
    from paper_2211_00705_amd import imexds
    x = torch.zeros(5, dtype=torch.float64)
    with pytest.raises(ValueError, match="expected 6 elements"):
        imexds._dev_ptr(x, 6)
    with pytest.raises(ValueError, match="float64"):
        imexds._dev_ptr(torch.zeros(6, dtype=torch.float32), 6)
    with pytest.raises(ValueError, match="contiguous"):
        imexds._dev_ptr(torch.zeros(12, dtype=torch.float64)[::2], 6)
    # right length, but host memory: still refused
    with pytest.raises(ValueError, match="GPU"):
        imexds._dev_ptr(torch.zeros(6, dtype=torch.float64), 6)


def test_creation_arguments_must_have_the_expected_length():
    from paper_2211_00705_amd import creation
    with pytest.raises(ValueError, match="expected 4 elements"):
        creation._dev(torch.zeros(3, dtype=torch.float64), torch.float64, 4)
    with pytest.raises(ValueError, match="GPU"):
        creation._dev(torch.zeros(4, dtype=torch.int32), torch.int32, 4)


class _FakeSolver:
    """Stands in for an IMEXDS context: records nothing, returns zeros on the
    host, counts generations like the real holder."""

    def __init__(self, n):
        self.n_slots = n
        self.generation = 0
        self.adjoint_calls = 0

    def set_tau(self, tau):
        self.generation += 1

    def set_state(self, rho, mom):
        self.generation += 1

    def forward_ckpt(self, n, c):
        self.generation += 1

    def state(self):
        return torch.zeros(self.n_slots, dtype=torch.float64), torch.zeros(self.n_slots,
                                                                              dtype=torch.float64)

    def interfaces(self):
        return np.zeros(1, np.int32), np.zeros(1), np.zeros(1)

    def adjoint(self, g_rho, g_mom, g_hl):
        self.adjoint_calls += 1
        z = torch.zeros(self.n_slots, dtype=torch.float64)
        return z, z.clone(), torch.zeros(1, dtype=torch.float64), torch.zeros(1,
                                                                              dtype=torch.float64)


def test_backward_refuses_a_solver_that_ran_again():
    from paper_2211_00705_amd.autograd import evolve
    s = _FakeSolver(4)
    r0 = torch.ones(4, dtype=torch.float64, requires_grad=True)
    m0 = torch.zeros(4, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor([1e-9], dtype=torch.float64, requires_grad=True)
    a, am, ah = evolve(s, r0, m0, tau, 3)
    b, bm, bh = evolve(s, r0, m0, tau, 3)
    with pytest.raises(RuntimeError, match="run again"):
        (a.sum() + am.sum() + ah.sum()).backward()
    assert s.adjoint_calls == 0
    (b.sum() + bm.sum() + bh.sum()).backward()
    assert s.adjoint_calls == 1
