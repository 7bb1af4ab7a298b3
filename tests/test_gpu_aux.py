"""GPU parity of the energy (Eq. 1) and optimality-gap (Eq. 2) kernels and
of the instance checks."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_17267_amd as sg
from gpu_util import instance, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L", [4, 6, 12, 32, 64])
def test_energy_kernel_matches_oracle(L):
    log("energy parity", L)
    inst, Jo, go, egs = instance(L, 31 + L, 0)
    rng = np.random.default_rng(L)
    n = 5 if L < 64 else 2
    s = rng.choice(np.array([-1, 1], np.int8), size=(n, L ** 3))
    s[0] = go
    e = sg.energy(inst, torch.from_numpy(s).cuda()).cpu().numpy()
    for r in range(n):
        assert e[r] == oracle.energy(Jo, s[r], (L, L, L))
    assert e[0] == egs


def test_epsilon_kernel_bit_exact():
    rng = np.random.default_rng(3)
    E = rng.integers(-300000, 300000, size=5000).astype(np.int32)
    for egs in (-360, -123457, -3000001, 777):
        eps = sg.epsilon(torch.from_numpy(E).cuda(), egs).cpu().numpy()
        ref = np.array([oracle.epsilon(int(e), egs) for e in E])
        np.testing.assert_array_equal(eps, ref)


def test_check_instance_flags_bad_couplings():
    L = 8
    inst, Jo, go, egs = instance(L, 8, 0)
    assert sg.check_instance(inst) == 0
    J = Jo.copy()
    J[0, 5] = 5              # out of range and breaks the pair copy
    bad = sg.Instance(L, J, egs, 0)
    assert sg.check_instance(bad) > 0
    J = Jo.copy()
    J[3, 17] = -J[3, 17] if J[3, 17] != 0 else 1   # only the pair copy broken
    bad = sg.Instance(L, J, egs, 0)
    assert sg.check_instance(bad) > 0
