"""Parity at the sizes and in the launch configurations that bench.py times
for the batched workload (12 point sources on each of 32^3x64, 24^3x48 and
16^3x32 clover lattices, one launch per operator step) and the large lattice
(64^3x128 clover): outputs at sampled sites against the oracle evaluated site
by site (oracle.sampled), solutions by the oracle's residual at sampled sites.
"""

import numpy as np
import pytest

import bench
import fieldgen as fg
from oracle import dirac, sampled
from paper_2303_05883_amd import lqcd
from tests.gpuutil import TOL, from_dev, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

KAPPA_C4, CSW = 0.1370, 1.0


def device_lookup(x):
    """psi_at(sites) for oracle.sampled from a device field [Lt, Lz, Ly, Lx, 4, 3]."""
    torch = torch_cuda()

    def look(s):
        s = np.asarray(s)
        idx = [torch.as_tensor(s[:, k], device=x.device) for k in (3, 2, 1, 0)]
        return x[idx[0], idx[1], idx[2], idx[3]].cpu().numpy()
    return look


def dirac_at_dev(U, x, kappa, csw, sites):
    look = device_lookup(x)
    return sampled.site_mul(sampled.clover_at(U, kappa, csw, sites), look(sites)) \
        - kappa * sampled.hop_at(U, look, -1, sites)


def _source_slice(args):
    dims, seed, t = args
    return fg.gaussian_spinor(dims, seed, t_slices=[t])


def gaussians(dims, seeds):
    """fieldgen's Gaussian spinors, generated time slice by time slice in worker processes."""
    import concurrent.futures as cf
    import os
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    jobs = [(dims, sd, t) for sd in seeds for t in range(dims[3])]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(_source_slice, jobs, chunksize=4))
    lt = dims[3]
    return [np.concatenate(parts[k * lt:(k + 1) * lt]) for k in range(len(seeds))]


def sample_sites(dims, n, seed, parity=None):
    """Random sites plus the origin, its eight neighbours and the far corner."""
    s = sampled.random_sites(dims, n, seed, parity)
    extra = [np.zeros(4, dtype=s.dtype), np.array(dims) - 1]
    for mu in range(4):
        for d in (1, -1):
            e = np.zeros(4, dtype=s.dtype)
            e[mu] = d % dims[mu]
            extra.append(e)
    extra = np.array(extra)
    if parity is not None:
        extra = extra[extra.sum(axis=1) % 2 == parity]
    return np.concatenate([s, extra])


@pytest.fixture(scope="module")
def c4():
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    lats, Us = [], []
    for dims, seed in bench.BATCH:
        U, _ = bench.generate(dims, seed, 0.3, source=False)
        lat = lqcd.Lattice(dims, -1, stream=stream)
        lat.set_gauge(to_dev(U))
        lat.set_clover(KAPPA_C4, CSW)
        for p in (lqcd.F64, lqcd.F32, lqcd.F16):
            lat.autotune(p)
        lats.append(lat)
        Us.append(U)
    yield lats, Us
    for lat in lats:
        lat.close()


@pytest.mark.parametrize("prec", [lqcd.F32, lqcd.F16])
def test_c4_batched_schur_sampled(c4, prec):
    """The batched Schur operator on 12 Gaussian right-hand sides per lattice,
    in the tuned launch shape, at sampled even sites of every right-hand side."""
    torch = torch_cuda()
    lats, Us = c4
    shape, _ = lqcd.batch_autotune(lats, [12, 12, 12], prec)
    ins, outs = [], []
    for (dims, seed), lat in zip(bench.BATCH, lats):
        b = torch.empty((12,) + tuple(dims[::-1]) + (4, 3), dtype=torch.complex128, device="cuda")
        for r, g in enumerate(gaussians(dims, [5000 + 16 * seed + r for r in range(12)])):
            b[r] = to_dev(g)
        ins.append(b)
        outs.append(torch.zeros_like(b))
    lqcd.batch_apply_schur(lats, ins, outs, prec)
    for (dims, seed), U, b, o in zip(bench.BATCH, Us, ins, outs):
        se = sample_sites(dims, 12, seed + 7, parity=0)
        for r in range(12):
            want = sampled.schur_at(U, None, KAPPA_C4, CSW, -1, se, x_at=_even_lookup(b[r]))
            got = device_lookup(o[r])(se)
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            assert err <= TOL[prec], (dims, r, shape, err)


def _even_lookup(x):
    look = device_lookup(x)

    def even(s):
        v = look(s)
        v[np.asarray(s).sum(axis=1) % 2 == 1] = 0
        return v
    return even


@pytest.mark.parametrize("prec", [lqcd.F32, lqcd.F16])
def test_c4_batched_solve_residual_sampled(c4, prec):
    """The 36 point-source solves of one batched call (FP64 outer loop): each
    returned x has |b - D x| <= 1e-10 at every sampled site (the global bound
    |b - D x| <= 1e-10 |b| = 1e-10 holds site by site), the origin and its
    neighbours included."""
    torch = torch_cuda()
    lats, Us = c4
    bs, xs = [], []
    for dims, _ in bench.BATCH:
        src = np.stack([fg.point_source(dims, k // 3, k % 3) for k in range(12)])
        bs.append(to_dev(src))
        xs.append(torch.zeros_like(bs[-1]))
    stats = lqcd.solve_batch(lats, bs, xs, inner_prec=prec)
    assert max(s.true_rel_resid for s in stats) <= 1e-10
    for (dims, seed), U, b, x in zip(bench.BATCH, Us, bs, xs):
        sa = sample_sites(dims, 16, seed + 11)
        for r in range(12):
            res = dirac_at_dev(U, x[r], KAPPA_C4, CSW, sa) - device_lookup(b[r])(sa)
            assert np.abs(res).max() <= 1.1e-10, (dims, r, np.abs(res).max())


C5_DIMS = (64, 64, 64, 128)


@pytest.fixture(scope="module")
def c5():
    torch = torch_cuda()
    w = bench.WORKLOADS["large"]
    assert tuple(w["dims"]) == C5_DIMS
    U, b = bench.generate(C5_DIMS, w["seed"], w["eps"], scale=w["scale"])
    lat = lqcd.Lattice(C5_DIMS, -1)
    Ud = to_dev(U)
    lat.set_gauge(Ud)
    del Ud
    torch.cuda.empty_cache()
    lat.set_clover(w["kappa"], w["csw"])
    for p in (lqcd.F64, lqcd.F32, lqcd.F16):
        lat.autotune(p)
    yield U, b, lat, w
    lat.close()


def c5_sites(parity, n, seed):
    s = sample_sites(C5_DIMS, n, seed, parity)
    # time-boundary and far-corner sites of the right parity
    edges = []
    for t in (0, C5_DIMS[3] - 1):
        for x in (0, C5_DIMS[0] - 1):
            c = np.array([x, C5_DIMS[1] - 1, 0, t])
            if c.sum() % 2 != parity:
                c[2] = 1
            edges.append(c)
    return np.concatenate([s, np.array(edges)])


def test_c5_operators_sampled(c5):
    """64^3 x 128 (the large workload): the full FP64 D at sampled sites of
    both parities and the FP64 Schur operator at sampled even sites within
    1e-13 of the oracle; the hop in FP32 and FP16 within their tolerances."""
    torch = torch_cuda()
    U, b, lat, w = c5
    kappa, csw = w["kappa"], w["csw"]
    bd = to_dev(b)
    out = torch.empty_like(bd)
    lat.apply("D", lqcd.F64, bd, out)
    sa = np.concatenate([c5_sites(0, 24, 21), c5_sites(1, 24, 22)])
    got = device_lookup(out)(sa)
    ref = sampled.dirac_at(U, b, kappa, csw, -1, sa)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13
    lat.apply("DPREC_SCHUR", lqcd.F64, bd, out)
    se = c5_sites(0, 24, 23)
    got = device_lookup(out)(se)
    ref = sampled.schur_at(U, dirac.mask(b, 0), kappa, csw, -1, se)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13
    ref = sampled.hop_at(U, sampled.full_lookup(dirac.mask(b, 1)), -1, se)
    for prec in (lqcd.F32, lqcd.F16):
        lat.apply("HOP_EO", prec, bd, out)
        got = device_lookup(out)(se)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= TOL[prec], prec


def test_c5_mixed_f16_solve_residual_sampled(c5):
    """The FP16-inner solve of the large workload: the library's FP64
    residual is at most 1e-10 and the oracle's residual at sampled sites
    agrees (rms per site well below the 1e-8 a wrong solution would exceed)."""
    torch = torch_cuda()
    U, b, lat, w = c5
    bd = to_dev(b)
    x = torch.zeros_like(bd)
    st = lat.solve(bd, x, inner_prec=lqcd.F16)
    assert st.true_rel_resid <= 1e-10 and st.outer_iters >= 2
    sa = np.concatenate([c5_sites(0, 32, 24), c5_sites(1, 32, 25)])
    r = dirac_at_dev(U, x, w["kappa"], w["csw"], sa) - sampled.gather(b, sa)
    assert np.sqrt(np.mean(np.abs(r) ** 2) * 12) <= 1e-8
