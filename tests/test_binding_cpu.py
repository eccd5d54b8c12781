"""The Python binding rejects arguments the library cannot check itself (host tensors,
wrong dtypes) before any call into it (CPU)."""
import pytest
import torch

import workloads as wl


def test_host_tensors_and_wrong_dtypes_are_rejected():
    import paper_2511_15629_amd as dp
    inst = wl.random_small(1, 3, 2, 11, 2, 2)
    lam = torch.from_numpy(inst.lam)
    P = torch.from_numpy(inst.P)
    with pytest.raises(TypeError):
        dp.solve(lam, P, inst.storage)                      # host memory
    with pytest.raises(TypeError):
        dp.solve_independent(lam, P[:, 0, :], 11, 0.1, 0.9, 1.0)
    with pytest.raises(TypeError):
        dp.adjoint(lam, P, inst.storage, torch.zeros(2, 11))
