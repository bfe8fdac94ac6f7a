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


@pytest.mark.parametrize("prec", [lqcd.F32, lqcd.F16])
def test_batch_is_deterministic(prec):
    """Fixed-order per-RHS reductions: two batched solves give the same x bit
    for bit."""
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    specs = [((4, 6, 8, 10), 3, 31), ((4, 4, 4, 4), 2, 32)]
    lats, bs = [], []
    for dims, n, seed in specs:
        U = fg.gauge_field(dims, seed, "smooth", 0.3)
        lat = lqcd.Lattice(dims, -1, stream=stream)
        lat.set_gauge(to_dev(U))
        lat.set_clover(0.136, 1.0)
        lats.append(lat)
        bs.append(to_dev(np.stack([fg.gaussian_spinor(dims, seed + 100 + k) for k in range(n)])))
    runs = []
    for _ in range(2):
        xs = [to_dev(np.zeros(tuple(b.shape), dtype=np.complex128)) for b in bs]
        st = lqcd.solve_batch(lats, bs, xs, inner_prec=prec)
        runs.append(([from_dev(x) for x in xs], [s.inner_iters for s in st]))
    assert runs[0][1] == runs[1][1]
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [lqcd.F32, lqcd.F16])
def test_batch_graph_replays_match_eager(prec):
    """The batched solve's captured iteration chunks, replayed with the host
    checks between them, give the eager launches' x bit for bit."""
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    specs = [((4, 6, 8, 10), 3, 33), ((4, 4, 4, 4), 2, 34)]
    lats, bs = [], []
    for dims, n, seed in specs:
        U = fg.gauge_field(dims, seed, "smooth", 0.3)
        lat = lqcd.Lattice(dims, -1, stream=stream)
        lat.set_gauge(to_dev(U))
        lat.set_clover(0.136, 1.0)
        lats.append(lat)
        bs.append(to_dev(np.stack([fg.gaussian_spinor(dims, seed + 100 + k) for k in range(n)])))
    runs = []
    for graph in (False, True, True):
        xs = [to_dev(np.zeros(tuple(b.shape), dtype=np.complex128)) for b in bs]
        st = lqcd.solve_batch(lats, bs, xs, inner_prec=prec, use_graph=graph, check_every=4)
        runs.append(([from_dev(x) for x in xs], [s.inner_iters for s in st]))
    for xs_g, it_g in runs[1:]:
        assert it_g == runs[0][1]
        for a, b in zip(runs[0][0], xs_g):
            assert np.array_equal(a, b)


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


def batch_system(torch, specs, kappa, csw, stream=None):
    stream = stream or torch.cuda.Stream()
    lats, ops, bs = [], [], []
    for dims, n, seed in specs:
        U = fg.gauge_field(dims, seed, "smooth", 0.3)
        lat = lqcd.Lattice(dims, -1, stream=stream)
        lat.set_gauge(to_dev(U))
        lat.set_clover(kappa, csw)
        lats.append(lat)
        ops.append(dirac.Operator(U, kappa, csw, -1))
        bs.append(np.stack([fg.gaussian_spinor(dims, seed + 100 + k) for k in range(n)]))
    return lats, ops, bs


# (rhs per lane, waves per workgroup, workgroups per XCD, walk, non-temporal)
SHAPES = {lqcd.F64: [(1, 8, 16, 0, 0), (2, 3, 64, 2, 1), (2, 1, 128, 1, 0)],
          lqcd.F32: [(1, 8, 64, 1, 0), (2, 2, 16, 0, 1), (3, 4, 128, 3, 1), (4, 3, 256, 0, 0), (4, 1, 8, 2, 0)],
          lqcd.F16: [(1, 8, 64, 0, 1), (2, 6, 128, 2, 0), (3, 2, 32, 1, 1), (4, 3, 256, 0, 0), (4, 1, 64, 3, 1)]}


@pytest.mark.parametrize("prec", [lqcd.F64, lqcd.F32, lqcd.F16])
@pytest.mark.parametrize("csw", [1.0, 0.0])
def test_batched_schur_matches_oracle(prec, csw):
    """The batched Schur operator, element by element against the oracle's
    S = D_ee - D_eo D_oo^-1 D_oe for every right-hand side, for every launch
    shape (right-hand sides per lane, waves per workgroup fewer or more than
    the groups of a lattice, workgroups per XCD); lattices of uneven sizes and
    right-hand side counts, ragged last site block (4x6x8x10)."""
    from tests.gpuutil import TOL
    torch = torch_cuda()
    specs = [((8, 8, 8, 8), 12, 31), ((4, 6, 8, 10), 5, 32), ((4, 4, 4, 4), 3, 33)]
    lats, ops, bs = batch_system(torch, specs, 0.136, csw)
    ins = [to_dev(b) for b in bs]
    want = []
    for op, b in zip(ops, bs):
        w = []
        for r in range(b.shape[0]):
            w.append(op.schur(dirac.mask(b[r], 0)))
        want.append(np.stack(w))
    for shape in SHAPES[prec]:
        outs = [to_dev(np.full_like(b, np.nan)) for b in bs]
        got_shape, us = lqcd.batch_autotune(lats, [b.shape[0] for b in bs], prec, shape)
        assert got_shape == shape and us > 0
        lqcd.batch_apply_schur(lats, ins, outs, prec)
        for w, o in zip(want, outs):
            oh = from_dev(o)
            for r in range(w.shape[0]):
                err = dirac.rel_l2(oh[r], w[r])
                assert err <= TOL[prec], (shape, r, err)


def test_batch_autotune_picks_a_valid_shape_and_solves():
    torch = torch_cuda()
    specs = [((8, 8, 8, 8), 12, 41), ((4, 4, 4, 8), 7, 42)]
    lats, ops, bs = batch_system(torch, specs, 0.136, 1.0)
    shape, us = lqcd.batch_autotune(lats, [12, 7], lqcd.F32)
    assert 1 <= shape[0] <= 4 and 1 <= shape[1] <= 8 and shape[2] >= 1 and 0 <= shape[3] <= 3 and us > 0
    ds = [to_dev(b) for b in bs]
    xs = [to_dev(np.zeros_like(b)) for b in bs]
    stats = lqcd.solve_batch(lats, ds, xs, inner_prec=lqcd.F32)
    k = 0
    for op, b, x in zip(ops, bs, xs):
        xh = from_dev(x)
        for r in range(b.shape[0]):
            assert dirac.rel_l2(op.D(xh[r]), b[r]) <= 1e-10, (r, stats[k])
            k += 1
    with pytest.raises(lqcd.LqcdError) as e:
        lqcd.batch_autotune(lats, [12, 7], lqcd.F64, (3, 2, 64, 0, 0))  # 3 RHS per lane is not built in FP64
    assert e.value.status == lqcd.EINVAL


def test_batch_rejects_bad_arguments():
    """A lattice with no right-hand side, an initial guess, the unpreconditioned
    operator and a batch that names one context twice are argument errors."""
    import ctypes as C
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    lats, _, bs = batch_system(torch, [((4, 4, 4, 4), 2, 51), ((4, 4, 4, 8), 1, 52)], 0.12, 1.0, stream)
    lib = lqcd.load()
    ds = [to_dev(b) for b in bs]
    xs = [to_dev(np.zeros_like(b)) for b in bs]

    def call(lat_list, nrhs, **kw):
        n = len(lat_list)
        ctxs = (C.c_void_p * n)(*[lat.handle.value for lat in lat_list])
        nr = (C.c_int * n)(*nrhs)
        prm = lqcd.default_params()
        prm.inner_prec, prm.on_device = lqcd.F32, 1
        for k, v in kw.items():
            setattr(prm, k, v)
        st = (lqcd.SolveStats * max(1, sum(nrhs)))()
        pb = (C.c_void_p * n)(*[b.data_ptr() for b in ds[:n]])
        px = (C.c_void_p * n)(*[x.data_ptr() for x in xs[:n]])
        torch.cuda.synchronize()
        return lib.lqcd_solve_batch(ctxs, nr, pb, px, n, C.byref(prm), st)

    assert call(lats, [2, 0]) == lqcd.EINVAL
    assert call(lats, [2, 1], even_odd=0) == lqcd.EINVAL
    assert call(lats, [2, 1], x0=ds[0].data_ptr()) == lqcd.EINVAL
    assert call([lats[0], lats[0]], [2, 2]) == lqcd.EINVAL
    # the valid call still works afterwards
    assert call(lats, [2, 1]) == lqcd.OK
    for lat in lats:
        lat.close()
