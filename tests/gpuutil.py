"""Helpers shared by the GPU tests: device staging and the library handle."""

import numpy as np
import pytest

# float64 tolerances of a single operator application (rel-L2 against the oracle)
TOL = {0: 1e-13, 1: 1e-5, 2: 5e-3}


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch


def to_dev(a: np.ndarray):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def from_dev(t) -> np.ndarray:
    return t.cpu().numpy()


def lattice(dims, U, kappa, csw, t_bc=-1):
    from paper_2303_05883_amd import lqcd
    lat = lqcd.Lattice(dims, t_bc)
    lat.set_gauge(to_dev(U))
    lat.set_clover(kappa, csw)
    return lat
