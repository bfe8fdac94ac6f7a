"""GPU solvers, checked against the oracle: the returned x must satisfy
||b - D x|| / ||b|| <= 1e-10 with the oracle's FP64 operator, for the plain
FP64 BiCGStab and for the FP32 and FP16 inner solvers inside the FP64 outer
loop. Solutions are also compared with LAPACK's dense solve on a tiny lattice.
"""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dense, dirac
from paper_2303_05883_amd import lqcd
from tests.gpuutil import from_dev, lattice, to_dev

pytestmark = pytest.mark.gpu


def true_residual(op, x, b):
    return dirac.rel_l2(op.D(x), b) if np.any(b) else float(np.linalg.norm(op.D(x)))


@pytest.mark.parametrize("prec", [lqcd.F64, lqcd.F32, lqcd.F16])
@pytest.mark.parametrize("graph", [True, False])
def test_wilson_haar_8(prec, graph):
    # 8^4, Haar links, kappa = 0.12, antiperiodic in time (the small FP64 workload)
    dims = (8, 8, 8, 8)
    U = fg.gauge_field(dims, 1001, "haar")
    b = fg.gaussian_spinor(dims, 1001)
    lat = lattice(dims, U, 0.12, 0.0)
    x = to_dev(np.zeros_like(b))
    st = lat.solve(to_dev(b), x, inner_prec=prec, use_graph=graph)
    r = true_residual(dirac.Operator(U, 0.12, 0.0), from_dev(x), b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)


@pytest.mark.parametrize("prec", [lqcd.F64, lqcd.F32, lqcd.F16])
def test_graph_replays_match_eager(prec):
    """The captured iteration chunk, replayed many times per solve with the
    solver's own host checks and FP64 outer work between the replays, gives the
    eager launches' x bit for bit, solve after solve."""
    dims = (8, 8, 8, 8)
    U = fg.gauge_field(dims, 1004, "smooth", 0.3)
    b = to_dev(fg.gaussian_spinor(dims, 1004))
    lat = lattice(dims, U, 0.137, 1.0)
    res = {}
    for graph in (False, True, True):
        x = to_dev(np.zeros(tuple(b.shape), dtype=np.complex128))
        st = lat.solve(b, x, inner_prec=prec, use_graph=graph, check_every=4)
        res.setdefault(graph, []).append((from_dev(x), st.inner_iters))
    eager_x, eager_it = res[False][0]
    for gx, git in res[True]:
        assert git == eager_it and np.array_equal(gx, eager_x)


@pytest.mark.parametrize("prec", [lqcd.F64, lqcd.F32, lqcd.F16])
@pytest.mark.parametrize("split", [1, 4, 0])
@pytest.mark.parametrize("reliable", [True, False])
def test_clover_smooth(prec, split, reliable):
    dims = (8, 8, 8, 8)
    U = fg.gauge_field(dims, 1003, "smooth", 0.3)
    b = fg.gaussian_spinor(dims, 1003)
    lat = lattice(dims, U, 0.137, 1.0)
    # split 0: the plane march, whole 4 x 8 plane per block, 2 z planes per block
    shape = {1: (256, 1, 1, 1), 4: (128, 4, 1, 1), 0: (32, 0, 2, 1)}[split]
    for p in (lqcd.F64, lqcd.F32, lqcd.F16):
        lat.set_hop_shape(p, *shape)
    x = to_dev(np.zeros_like(b))
    st = lat.solve(to_dev(b), x, inner_prec=prec, reliable_update=reliable)
    r = true_residual(dirac.Operator(U, 0.137, 1.0), from_dev(x), b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    if prec != lqcd.F64:
        assert st.outer_iters >= 2


def test_matches_dense_solve():
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 5, "smooth", 0.3)
    b = fg.gaussian_spinor(dims, 6)
    lat = lattice(dims, U, 0.13, 1.0)
    x = np.zeros_like(b)
    lat.solve(b, x, tol=1e-12)
    xd = np.linalg.solve(dense.dense_dirac(U, 0.13, 1.0), dense.to_vector(b)).reshape(b.shape)
    assert dirac.rel_l2(x, xd) <= 1e-9


@pytest.mark.parametrize("inner_prec", [0, 1, 2])
def test_solve_is_deterministic(inner_prec):
    """Fixed-order reductions: repeated solves of one system give the same x
    bit for bit, in FP64 and with FP32 or FP16 inner solves."""
    dims = (4, 6, 8, 10)
    U = fg.gauge_field(dims, 11, "smooth", 0.3)
    b = fg.gaussian_spinor(dims, 12)
    lat = lattice(dims, U, 0.135, 1.0)
    x1, x2 = np.zeros_like(b), np.zeros_like(b)
    s1 = lat.solve(b, x1, inner_prec=inner_prec)
    s2 = lat.solve(b, x2, inner_prec=inner_prec)
    assert np.array_equal(x1, x2) and s1.inner_iters == s2.inner_iters


def test_point_source_and_zero_source():
    dims = (4, 4, 4, 8)
    U = fg.gauge_field(dims, 21, "smooth", 0.3)
    lat = lattice(dims, U, 0.137, 1.0)
    op = dirac.Operator(U, 0.137, 1.0)
    for prec in (lqcd.F64, lqcd.F32, lqcd.F16):
        b = fg.point_source(dims, 1, 2)
        x = np.zeros_like(b)
        st = lat.solve(b, x, inner_prec=prec)
        assert true_residual(op, x, b) <= 1e-10, (prec, st)
    z = np.zeros_like(b)
    x = np.ones_like(b)
    st = lat.solve(z, x)
    assert not np.any(x) and st.true_rel_resid == 0.0


def test_initial_guess_is_used():
    dims = (4, 4, 4, 8)
    U = fg.gauge_field(dims, 31, "smooth", 0.3)
    b = fg.gaussian_spinor(dims, 32)
    lat = lattice(dims, U, 0.13, 1.0)
    x = np.zeros_like(b)
    st1 = lat.solve(b, x)
    x2 = np.zeros_like(b)
    st2 = lat.solve(b, x2, x0=x)
    assert st2.inner_iters < st1.inner_iters
    assert st2.true_rel_resid <= 1e-10


def test_iteration_cap_reports_noconv():
    dims = (4, 4, 4, 8)
    U = fg.gauge_field(dims, 41, "smooth", 0.3)
    b = fg.gaussian_spinor(dims, 42)
    lat = lattice(dims, U, 0.137, 1.0)
    x = np.zeros_like(b)
    st = lat.solve(b, x, max_iter=3, raise_on_fail=False)
    assert st.status == lqcd.ENOCONV and st.inner_iters <= 3 + 8 and st.true_rel_resid > 1e-10


def test_unpreconditioned_c1():
    """BiCGStab on the full operator (no even-odd preconditioning) for the 8^4
    Haar Wilson system at kappa 0.12: the oracle's FP64 residual of the
    returned x is at most 1e-10, and so is the library's own."""
    dims = (8, 8, 8, 8)
    U = fg.gauge_field(dims, 1001, "haar")
    b = fg.gaussian_spinor(dims, 1001)
    lat = lattice(dims, U, 0.12, 0.0)
    x = to_dev(np.zeros_like(b))
    st = lat.solve(to_dev(b), x, even_odd=False)
    r = true_residual(dirac.Operator(U, 0.12, 0.0), from_dev(x), b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    assert st.inner_iters > 0 and st.outer_iters >= 1


def test_unpreconditioned_matches_dense_solve():
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 5, "smooth", 0.3)
    b = fg.gaussian_spinor(dims, 6)
    lat = lattice(dims, U, 0.13, 1.0)
    x = np.zeros_like(b)
    lat.solve(b, x, tol=1e-12, even_odd=False)
    xd = np.linalg.solve(dense.dense_dirac(U, 0.13, 1.0), dense.to_vector(b)).reshape(b.shape)
    assert dirac.rel_l2(x, xd) <= 1e-9
    # an initial guess is used: starting from the solution needs no iteration
    x2 = np.zeros_like(b)
    st = lat.solve(b, x2, tol=1e-10, even_odd=False, x0=x)
    assert st.inner_iters == 0 and st.true_rel_resid <= 1e-10


def test_unpreconditioned_rejects_mixed_precision():
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 5, "smooth", 0.3)
    lat = lattice(dims, U, 0.13, 1.0)
    b = fg.gaussian_spinor(dims, 6)
    with pytest.raises(lqcd.LqcdError) as e:
        lat.solve(b, np.zeros_like(b), inner_prec=lqcd.F32, even_odd=False)
    assert e.value.status == lqcd.EINVAL
