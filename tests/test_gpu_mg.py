"""GPU parity of the two-level multigrid against the oracle (oracle/mg.py),
through the C ABI: restriction, prolongation and the coarse operator from
the same start vectors (with and without SAP-smoothing setup rounds), the
two-level preconditioner, the multigrid-preconditioned solve, and the error
paths.

Tolerances: the GPU builds and applies everything in FP32. One restriction,
prolongation or coarse-operator application from unsmoothed vectors carries
the FP32 rounding of a few hundred-term sums (rel-L2 1e-5). With setup
rounds the basis has gone through FP32 SAP applications (rel-L2 ~1e-6 each)
and the orthonormalisation, and the preconditioner adds a coarse solve run
to 1e-6 and an FP32 SAP pass, so those comparisons use 1e-4 and 1e-3.
Solves reach the FP64 true residual 1e-10."""

import numpy as np
import pytest

import fieldgen as fg
from gpuutil import from_dev, lattice, to_dev
from oracle import dirac, mg, sap

pytestmark = pytest.mark.gpu

DIMS = (8, 4, 4, 8)
ADIMS = (2, 2, 2, 2)
SBLK = (4, 2, 2, 4)
KAPPA, CSW = 0.13, 1.0


def build(n, iters, seed=51, ncy=2, nmr=3, csw=CSW):
    U = fg.gauge_field(DIMS, seed, "smooth", 0.3)
    op = dirac.Operator(U, KAPPA, csw)
    start = np.stack([fg.gaussian_spinor(DIMS, seed + 1 + k) for k in range(n)])
    lat = lattice(DIMS, U, KAPPA, csw)
    kw = dict(agg=ADIMS, nvec=n, setup_iters=iters, sap_block=SBLK, ncycles=ncy, nmr=nmr)
    P = mg.setup(op.D, mg.Aggregates(DIMS, ADIMS), list(start), sap.Blocks(DIMS, SBLK), iters, ncy, nmr)
    return U, op, lat, start, kw, P


def coarse_vec(n, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=n) + 1j * rng.normal(size=n)) / np.sqrt(2)


@pytest.mark.parametrize("n,iters,tol", [(4, 0, 1e-5), (3, 2, 1e-4)])
def test_restrict_prolong_coarse_apply_match_oracle(n, iters, tol):
    U, op, lat, start, kw, P = build(n, iters)
    lat.mg_setup(to_dev(start), **kw)
    nc = lat.mg_coarse_size()
    assert nc == P.ncoarse == 4 * 2 * 2 * 4 * 2 * n
    r = fg.gaussian_spinor(DIMS, 60)
    rc = to_dev(np.zeros(nc, dtype=np.complex128))
    lat.mg_restrict(to_dev(r), rc)
    assert dirac.rel_l2(from_dev(rc), P.restrict(r)) <= tol
    e = coarse_vec(nc, 61)
    x = to_dev(np.zeros_like(r))
    lat.mg_prolong(to_dev(e), x)
    assert dirac.rel_l2(from_dev(x), P.prolong(e)) <= tol
    # the coarse operator against the oracle's P^dag D P (columns by definition)
    Dc = mg.coarse_operator(op.D, P)
    y = to_dev(np.zeros(nc, dtype=np.complex128))
    lat.mg_coarse_apply(to_dev(e), y)
    assert dirac.rel_l2(from_dev(y), Dc @ e) <= tol
    # host pointers give the same
    yh = lat.mg_coarse_apply(e, np.zeros(nc, dtype=np.complex128))
    assert dirac.rel_l2(yh, Dc @ e) <= tol


def test_full_size_aggregates_match_oracle():
    """4^4 aggregates (256 sites: four-wave workgroups in the Gram-Schmidt and
    the restriction, as in the benchmarked configuration)."""
    dims, adims, sblk, n = (8, 8, 8, 8), (4, 4, 4, 4), (4, 4, 2, 2), 3
    U = fg.gauge_field(dims, 71, "smooth", 0.3)
    op = dirac.Operator(U, KAPPA, CSW)
    start = np.stack([fg.gaussian_spinor(dims, 72 + k) for k in range(n)])
    lat = lattice(dims, U, KAPPA, CSW)
    lat.mg_setup(to_dev(start), agg=adims, nvec=n, setup_iters=1, sap_block=sblk, ncycles=1, nmr=2)
    P = mg.setup(op.D, mg.Aggregates(dims, adims), list(start), sap.Blocks(dims, sblk), 1, 1, 2)
    nc = lat.mg_coarse_size()
    assert nc == P.ncoarse == 16 * 2 * n
    r = fg.gaussian_spinor(dims, 73)
    rc = to_dev(np.zeros(nc, dtype=np.complex128))
    lat.mg_restrict(to_dev(r), rc)
    assert dirac.rel_l2(from_dev(rc), P.restrict(r)) <= 1e-4
    e = coarse_vec(nc, 74)
    x = to_dev(np.zeros_like(r))
    lat.mg_prolong(to_dev(e), x)
    assert dirac.rel_l2(from_dev(x), P.prolong(e)) <= 1e-4
    y = to_dev(np.zeros(nc, dtype=np.complex128))
    lat.mg_coarse_apply(to_dev(e), y)
    assert dirac.rel_l2(from_dev(y), mg.coarse_operator(op.D, P) @ e) <= 1e-4


def test_two_level_preconditioner_matches_oracle():
    U, op, lat, start, kw, P = build(4, 1)
    lat.mg_setup(to_dev(start), coarse_tol=1e-6, coarse_max_iter=2000, **kw)
    Dc = mg.coarse_operator(op.D, P)
    pre = mg.TwoLevel(op.D, P, Dc, sap.Blocks(DIMS, SBLK), kw["ncycles"], kw["nmr"], coarse_tol=1e-12,
                      coarse_max_iter=5000)
    r = fg.gaussian_spinor(DIMS, 62)
    x = to_dev(np.zeros_like(r))
    lat.mg_apply(to_dev(r), x)
    assert dirac.rel_l2(from_dev(x), pre(r)) <= 1e-3


@pytest.mark.parametrize("iters,csw", [(0, CSW), (2, CSW), (2, 0.0)])
def test_solve_mg_matches_oracle(iters, csw):
    U, op, lat, start, kw, P = build(4, iters, csw=csw)
    lat.mg_setup(to_dev(start), **kw)
    b = fg.gaussian_spinor(DIMS, 63)
    x = to_dev(np.zeros_like(b))
    st = lat.solve_mg(to_dev(b), x, tol=1e-10)
    xh = from_dev(x)
    r = np.linalg.norm(b - op.D(xh)) / np.linalg.norm(b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    xo, info = sap.fbicgstab(op.D, lambda v: sap.sap(op.D, sap.Blocks(DIMS, SBLK), v, 2, 3), b, tol=1e-12)
    assert info.converged
    assert dirac.rel_l2(xh, xo) <= 1e-8


def test_solve_mg_is_deterministic():
    """Two multigrid-preconditioned solves after one setup give the same x bit
    for bit."""
    U, op, lat, start, kw, P = build(4, 2)
    lat.mg_setup(to_dev(start), **kw)
    b = to_dev(fg.gaussian_spinor(DIMS, 65))
    xs = []
    for _ in range(2):
        x = to_dev(np.zeros(tuple(b.shape), dtype=np.complex128))
        lat.solve_mg(b, x, tol=1e-10)
        xs.append(from_dev(x))
    assert np.array_equal(xs[0], xs[1])


def test_mg_errors_and_state():
    from paper_2303_05883_amd import lqcd
    U, op, lat, start, kw, P = build(2, 0)
    r = fg.gaussian_spinor(DIMS, 64)
    assert lat.mg_coarse_size() == 0
    with pytest.raises(lqcd.LqcdError) as e:
        lat.mg_apply(r, np.zeros_like(r))
    assert e.value.status == lqcd.ESTATE
    bad = [dict(kw, agg=(2, 2, 2, 8)),            # one aggregate in t
           dict(kw, agg=(8, 4, 4, 8)),            # too many sites, one aggregate per direction
           dict(kw, nvec=0), dict(kw, nvec=25), dict(kw, setup_iters=-1),
           dict(kw, coarse_tol=0.0), dict(kw, coarse_max_iter=0), dict(kw, sap_block=(3, 2, 2, 4))]
    for k in bad:
        with pytest.raises(lqcd.LqcdError) as e:
            lat.mg_setup(start, **k)  # parameters are checked before the start vectors are read
        assert e.value.status == lqcd.EINVAL, k
    lat.mg_setup(start, **kw)
    assert lat.mg_coarse_size() > 0
    lat.set_clover(KAPPA, CSW)  # drops the setup
    assert lat.mg_coarse_size() == 0
    with pytest.raises(lqcd.LqcdError) as e:
        lat.solve_mg(r, np.zeros_like(r))
    assert e.value.status == lqcd.ESTATE


def test_mg_properties_at_benchmark_size():
    """On the benchmarked 32^3x64 clover system with 4^4 aggregates: P^dag P = 1
    and the coarse operator is Gamma5-hermitian (<x, G D_c y> = <G D_c x, y>,
    G = +1 on the c_+ and -1 on the c_- coarse entries), to FP32 rounding."""
    import torch
    dims, n = (32, 32, 32, 64), 4
    U = fg.gauge_field(dims, 75, "smooth", 0.3)
    lat = lattice(dims, U, 0.137, 1.0)
    lx, ly, lz, lt = dims
    gen = torch.Generator(device="cuda")
    gen.manual_seed(76)
    shape = (n, lt, lz, ly, lx, 4, 3)
    start = torch.complex(torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64),
                          torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64))
    lat.mg_setup(start, agg=(4, 4, 4, 4), nvec=n, setup_iters=1, sap_block=(16, 4, 2, 2), ncycles=1, nmr=2)
    del start
    nc = lat.mg_coarse_size()
    assert nc == 8 * 8 * 8 * 16 * 2 * n
    e = to_dev(coarse_vec(nc, 77))
    fine = torch.empty((lt, lz, ly, lx, 4, 3), dtype=torch.complex128, device="cuda")
    lat.mg_prolong(e, fine)
    back = torch.empty_like(e)
    lat.mg_restrict(fine, back)
    assert (torch.linalg.vector_norm(back - e) / torch.linalg.vector_norm(e)).item() <= 1e-5
    g = torch.tensor([1.0] * n + [-1.0] * n, dtype=torch.float64, device="cuda").repeat(nc // (2 * n))
    x, y = to_dev(coarse_vec(nc, 78)), to_dev(coarse_vec(nc, 79))
    dx, dy = torch.empty_like(x), torch.empty_like(y)
    lat.mg_coarse_apply(x, dx)
    lat.mg_coarse_apply(y, dy)
    lhs = torch.vdot(x, g * dy).item()
    rhs = torch.vdot(g * dx, y).item()
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs), (lhs, rhs)
