"""GPU parity of the staggered operator and its even-odd CG against the oracle
(oracle/staggered.py), through the C ABI. Tolerances as for the Wilson
operator: rel-L2 1e-13 in FP64, 1e-5 in FP32 (one application); solves to a
true FP64 residual of 1e-10."""

import numpy as np
import pytest

import fieldgen as fg
from gpuutil import from_dev, lattice, to_dev
from oracle import dirac, staggered
from paper_2303_05883_amd import lqcd

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-5}
DIMS = [(4, 4, 4, 4), (2, 2, 2, 4), (4, 6, 8, 10), (8, 8, 8, 16)]


def colour_field(dims, seed):
    rng = np.random.default_rng(seed)
    lx, ly, lz, lt = dims
    return (rng.normal(size=(lt, lz, ly, lx, 3)) + 1j * rng.normal(size=(lt, lz, ly, lx, 3))) / np.sqrt(2)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("t_bc", [-1, 1])
def test_stag_apply_matches_oracle(dims, prec, t_bc):
    U = fg.gauge_field(dims, 81, "haar")
    psi = colour_field(dims, 82)
    op = staggered.Staggered(U, 0.07, t_bc)
    lat = lattice(dims, U, 0.12, 0.0, t_bc)
    out = to_dev(np.zeros_like(psi))
    lat.stag_apply("D", prec, 0.07, to_dev(psi), out)
    assert dirac.rel_l2(from_dev(out), op.D(psi)) <= TOL[prec]
    lat.stag_apply("SCHUR", prec, 0.07, to_dev(psi), out)
    assert dirac.rel_l2(from_dev(out), op.schur(psi)) <= TOL[prec]


def test_stag_host_pointers_and_errors():
    from paper_2303_05883_amd import lqcd
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 83, "haar")
    psi = colour_field(dims, 84)
    lat = lattice(dims, U, 0.12, 0.0)
    out = lat.stag_apply("D", 0, 0.3, psi, np.zeros_like(psi))
    assert dirac.rel_l2(out, staggered.Staggered(U, 0.3).D(psi)) <= 1e-13
    for call in (lambda: lat.stag_apply("D", 2, 0.3, psi, np.zeros_like(psi)),
                 lambda: lat.stag_apply(7, 0, 0.3, psi, np.zeros_like(psi)),
                 lambda: lat.stag_apply("D", 0, float("nan"), psi, np.zeros_like(psi)),
                 lambda: lat.stag_solve(0.0, psi, np.zeros_like(psi))):
        with pytest.raises(lqcd.LqcdError) as e:
            call()
        assert e.value.status == lqcd.EINVAL


@pytest.mark.parametrize("dims,mass", [((4, 4, 4, 4), 0.1), ((8, 8, 8, 16), 0.05)])
def test_stag_solve_matches_oracle(dims, mass):
    U = fg.gauge_field(dims, 85, "smooth", 0.3)
    b = colour_field(dims, 86)
    op = staggered.Staggered(U, mass)
    lat = lattice(dims, U, 0.12, 0.0)
    x = to_dev(np.zeros_like(b))
    st = lat.stag_solve(mass, to_dev(b), x, tol=1e-10)
    xh = from_dev(x)
    r = np.linalg.norm(b - op.D(xh)) / np.linalg.norm(b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    xo, info = staggered.solve(op, b, tol=1e-11)
    assert info.converged
    assert dirac.rel_l2(xh, xo) <= 1e-8


@pytest.mark.parametrize("dims,mass", [((4, 4, 4, 4), 0.1), ((8, 8, 8, 16), 0.05)])
@pytest.mark.parametrize("inner_tol", [0.0, 1e-3])
def test_stag_solve_mixed_matches_oracle(dims, mass, inner_tol):
    """FP32 inner CG under FP64 defect correction reaches the FP64 tolerance:
    the oracle's residual of the GPU's x and the oracle's solution agree as
    for the FP64 solve; an FP16 inner precision is rejected."""
    U = fg.gauge_field(dims, 88, "smooth", 0.3)
    b = colour_field(dims, 89)
    op = staggered.Staggered(U, mass)
    lat = lattice(dims, U, 0.12, 0.0)
    x = to_dev(np.zeros_like(b))
    st = lat.stag_solve(mass, to_dev(b), x, tol=1e-10, inner_prec=lqcd.F32, inner_tol=inner_tol)
    xh = from_dev(x)
    r = np.linalg.norm(b - op.D(xh)) / np.linalg.norm(b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    assert st.outer_iters >= 2, st  # FP32 alone cannot reach 1e-10: at least one correction pass
    xo, info = staggered.solve(op, b, tol=1e-11)
    assert info.converged
    assert dirac.rel_l2(xh, xo) <= 1e-8
    st = lat.stag_solve(mass, to_dev(b), x, inner_prec=lqcd.F16, raise_on_fail=False)
    assert st.status == lqcd.EINVAL


@pytest.mark.parametrize("inner_prec", [0, 1])
def test_stag_solve_is_deterministic(inner_prec):
    """Fixed-order reductions: two solves of the same system give the same x
    bit for bit (FP64 and FP32-inner)."""
    dims = (4, 6, 8, 10)
    U = fg.gauge_field(dims, 98, "smooth", 0.3)
    b = to_dev(colour_field(dims, 99))
    lat = lattice(dims, U, 0.12, 0.0)
    xs, its = [], []
    for _ in range(2):
        x = to_dev(np.zeros(b.shape, dtype=np.complex128))
        st = lat.stag_solve(0.05, b, x, inner_prec=inner_prec)
        xs.append(from_dev(x))
        its.append(st.inner_iters)
    assert np.array_equal(xs[0], xs[1]) and its[0] == its[1]


@pytest.mark.parametrize("inner_prec", [0, 1])
def test_stag_zero_source(inner_prec):
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 87, "haar")
    lat = lattice(dims, U, 0.12, 0.0)
    b = np.zeros((4, 4, 4, 4, 3), dtype=np.complex128)
    x = to_dev(np.ones_like(b))
    st = lat.stag_solve(0.1, to_dev(b), x, inner_prec=inner_prec)
    assert st.true_rel_resid == 0.0 and st.inner_iters == 0 and np.all(from_dev(x) == 0)


def test_stag_mixed_solve_at_benchmark_size():
    """The FP32-inner staggered CG at the benchmarked 32^3x64 size: the
    oracle's D applied to the GPU's x at random and edge sites reproduces b
    there (sampled residual against the sampled b)."""
    from oracle import sampled
    dims, mass = (32, 32, 32, 64), 0.05
    U = fg.gauge_field(dims, 93, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    b = colour_field(dims, 96)
    x = to_dev(np.zeros_like(b))
    st = lat.stag_solve(mass, to_dev(b), x, inner_prec=lqcd.F32)
    assert st.true_rel_resid <= 1e-10 and st.outer_iters >= 2, st
    xh = from_dev(x)
    edges = np.array([[xx, yy, zz, tt] for xx in (0, 31) for yy in (0, 31) for zz in (0, 31) for tt in (0, 63)])
    sites = np.concatenate([sampled.random_sites(dims, 64, 97), edges])
    dx = sampled.stag_dirac_at(U, xh, mass, -1, sites)
    bs = sampled.gather(b, sites)
    assert np.linalg.norm(bs - dx) / np.linalg.norm(bs) <= 1e-9


def test_stag_native_hop_matches_oracle():
    import torch
    dims = (4, 6, 8, 10)
    U = fg.gauge_field(dims, 88, "haar")
    psi = colour_field(dims, 89)
    op = staggered.Staggered(U, 0.0)
    lat = lattice(dims, U, 0.12, 0.0)
    for prec in (0, 1):
        nb = lat.stag_field_bytes(prec)
        src = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty(nb, dtype=torch.uint8, device="cuda")
        for out_parity in (0, 1):
            lat.stag_import(prec, 1 - out_parity, to_dev(psi), src)
            lat.stag_hop_native_repeat(prec, out_parity, [src], [dst], 1)
            got = to_dev(np.zeros_like(psi))
            lat.stag_export(prec, out_parity, dst, got)
            torch.cuda.synchronize()
            want = op.hop_pq(out_parity, 1 - out_parity, psi)
            assert dirac.rel_l2(from_dev(got), want) <= TOL[prec]


def test_stag_antihermitian_at_benchmark_size():
    """H = D - m is anti-Hermitian: <a, H b> = -<H a, b>, checked on the
    benchmarked 32^3x64 lattice (a property that holds at any size), FP64."""
    import torch
    dims, mass = (32, 32, 32, 64), 0.05
    U = fg.gauge_field(dims, 90, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    a, b = (to_dev(colour_field(dims, s)) for s in (91, 92))
    ha, hb = torch.empty_like(a), torch.empty_like(b)
    lat.stag_apply("D", 0, mass, a, ha)
    lat.stag_apply("D", 0, mass, b, hb)
    ha -= mass * a
    hb -= mass * b
    lhs = torch.vdot(a.flatten(), hb.flatten()).item()
    rhs = -torch.vdot(ha.flatten(), b.flatten()).item()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs), (lhs, rhs)


def test_stag_sampled_at_benchmark_size():
    """D = m + H at the benchmarked 32^3x64 size against the oracle evaluated
    site by site (oracle.sampled) at random sites and at sites on both ends of
    every direction (the antiperiodic t boundary), FP64 to 1e-13 and FP32 to
    1e-5."""
    from oracle import sampled
    dims, mass = (32, 32, 32, 64), 0.05
    U = fg.gauge_field(dims, 93, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    chi = colour_field(dims, 94)
    a = to_dev(chi)
    out = to_dev(np.zeros_like(chi))
    edges = np.array([[x, y, z, t] for x in (0, 31) for y in (0, 31) for z in (0, 31) for t in (0, 63)])
    sites = np.concatenate([sampled.random_sites(dims, 64, 95), edges])
    want = sampled.stag_dirac_at(U, chi, mass, -1, sites)
    for prec in (0, 1):
        lat.stag_apply("D", prec, mass, a, out)
        got = sampled.gather(from_dev(out), sites)
        assert dirac.rel_l2(got, want) <= TOL[prec], prec
