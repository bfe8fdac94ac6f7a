"""Batched solves: several lattices of different sizes with several right-hand
sides each, in one persistent launch per operator step. Every right-hand side
must reach a true FP64 residual <= 1e-10 measured by the CPU oracle.
"""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dirac
from paper_2303_05883_amd import lqcd
from tests.gpuutil import from_dev, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def point_sources(dims, n):
    return np.stack([fg.point_source(dims, k // 3, k % 3) for k in range(n)])


@pytest.mark.parametrize("prec", [lqcd.F32, lqcd.F16, lqcd.F64])
@pytest.mark.parametrize("csw", [1.0, 0.0])
def test_batch_matches_oracle(prec, csw):
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    specs = [((8, 8, 8, 8), 12, 11), ((4, 6, 8, 10), 5, 12), ((4, 4, 4, 4), 3, 13)]
    lats, ops, bs, xs = [], [], [], []
    for dims, n, seed in specs:
        U = fg.gauge_field(dims, seed, "smooth", 0.3)
        lat = lqcd.Lattice(dims, -1, stream=stream)
        lat.set_gauge(to_dev(U))
        lat.set_clover(0.136, csw)
        b = point_sources(dims, n) if n == 12 else np.stack([fg.gaussian_spinor(dims, seed + 100 + k) for k in range(n)])
        lats.append(lat)
        ops.append(dirac.Operator(U, 0.136, csw, -1))
        bs.append(to_dev(b))
        xs.append(to_dev(np.zeros_like(b)))
    stats = lqcd.solve_batch(lats, bs, xs, inner_prec=prec)
    assert len(stats) == 20
    k = 0
    for op, b, x in zip(ops, bs, xs):
        bh, xh = from_dev(b), from_dev(x)
        for r in range(bh.shape[0]):
            res = dirac.rel_l2(op.D(xh[r]), bh[r])
            assert res <= 1e-10 and stats[k].true_rel_resid <= 1e-10, (r, res, stats[k])
            k += 1


def test_batch_host_pointers_and_zero_rhs():
    specs = [((4, 4, 4, 8), 4, 21), ((4, 4, 4, 4), 2, 22)]
    lats, ops, bs, xs = [], [], [], []
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    for dims, n, seed in specs:
        U = fg.gauge_field(dims, seed, "smooth", 0.3)
        lat = lqcd.Lattice(dims, -1, stream=stream)
        lat.set_gauge(U)
        lat.set_clover(0.13, 1.0)
        b = np.stack([fg.gaussian_spinor(dims, seed + k) for k in range(n)])
        b[-1] = 0.0
        lats.append(lat)
        ops.append(dirac.Operator(U, 0.13, 1.0, -1))
        bs.append(b)
        xs.append(np.ones_like(b))
    stats = lqcd.solve_batch(lats, bs, xs, inner_prec=lqcd.F32)
    for op, b, x in zip(ops, bs, xs):
        for r in range(b.shape[0] - 1):
            assert dirac.rel_l2(op.D(x[r]), b[r]) <= 1e-10
        assert not np.any(x[-1])
    assert stats[3].true_rel_resid == 0.0


def test_batch_rejects_mixed_streams():
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 1, "smooth", 0.3)
    a, b = lqcd.Lattice(dims, -1), lqcd.Lattice(dims, -1)
    for lat in (a, b):
        lat.set_gauge(to_dev(U))
        lat.set_clover(0.12, 0.0)
    v = to_dev(np.zeros((1, 4, 4, 4, 4, 4, 3), complex))
    with pytest.raises(lqcd.LqcdError) as e:
        lqcd.solve_batch([a, b], [v, v], [v.clone(), v.clone()])
    assert e.value.status == lqcd.EINVAL
