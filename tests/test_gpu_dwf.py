"""GPU parity of the Moebius domain-wall operator (Shamir included), its
adjoint and the normal-equation CG against the oracle (oracle/dwf.py),
through the C ABI. Tolerances:
rel-L2 1e-13 (FP64) and 1e-5 (FP32) per application; solves to a true FP64
residual of 1e-10 (also with FP32 inner CG)."""

import numpy as np
import pytest

import fieldgen as fg
from gpuutil import from_dev, lattice, to_dev
from oracle import dirac, dwf
from paper_2303_05883_amd import lqcd

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-5}


def field5(dims, Ls, seed):
    rng = np.random.default_rng(seed)
    lx, ly, lz, lt = dims
    shape = (Ls, lt, lz, ly, lx, 4, 3)
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)) / np.sqrt(2)


# walks: (4, 4, 16, 4) XCD z-slabs of two planes; (8, 8, 8, 8), (4, 8, 4, 4),
# (4, 16, 2, 4) XCD y-ranges (as the benchmarked 64x32x16x8 in FP32);
# (16, 4, 2, 4) XCD x-ranges of one column in FP64 (as 64x32x16x8 in FP64) and
# linear in FP32; the rest linear
@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 4), ((2, 2, 2, 4), 5), ((4, 6, 8, 10), 3), ((8, 8, 8, 8), 8),
                                     ((4, 4, 4, 4), 1), ((4, 4, 16, 4), 8), ((4, 8, 4, 4), 3), ((4, 16, 2, 4), 5),
                                     ((16, 4, 2, 4), 6)])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("t_bc", [-1, 1])
@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5), (1.3, 0.0)])
def test_dwf_apply_matches_oracle(dims, Ls, prec, t_bc, b5, c5):
    U = fg.gauge_field(dims, 111, "haar")
    psi = field5(dims, Ls, 112)
    op = dwf.DomainWall(U, 1.8, 0.03, Ls, t_bc, b5, c5)
    lat = lattice(dims, U, 0.12, 0.0, t_bc)
    out = to_dev(np.zeros_like(psi))
    lat.dwf_apply(Ls, 1.8, 0.03, prec, to_dev(psi), out, b5=b5, c5=c5)
    assert dirac.rel_l2(from_dev(out), op.D(psi)) <= TOL[prec]
    lat.dwf_apply(Ls, 1.8, 0.03, prec, to_dev(psi), out, dag=True, b5=b5, c5=c5)
    assert dirac.rel_l2(from_dev(out), op.Ddag(psi)) <= TOL[prec]


def test_dwf_host_pointers_and_errors():
    from paper_2303_05883_amd import lqcd
    dims, Ls = (4, 4, 4, 4), 3
    U = fg.gauge_field(dims, 113, "haar")
    psi = field5(dims, Ls, 114)
    lat = lattice(dims, U, 0.12, 0.0)
    out = lat.dwf_apply(Ls, 1.5, 0.1, 0, psi, np.zeros_like(psi))
    assert dirac.rel_l2(out, dwf.DomainWall(U, 1.5, 0.1, Ls).D(psi)) <= 1e-13
    for call in (lambda: lat.dwf_apply(0, 1.5, 0.1, 0, psi, np.zeros_like(psi)),
                 lambda: lat.dwf_apply(Ls, float("inf"), 0.1, 0, psi, np.zeros_like(psi)),
                 lambda: lat.dwf_apply(Ls, 1.5, 0.1, 0, psi, np.zeros_like(psi), c5=float("nan")),
                 lambda: lat.dwf_apply(257, 1.5, 0.1, 0, psi, np.zeros_like(psi)),
                 lambda: lat.dwf_apply(Ls, 1.5, 0.1, 2, psi, np.zeros_like(psi))):
        with pytest.raises(lqcd.LqcdError) as e:
            call()
        assert e.value.status == lqcd.EINVAL


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_dwf_solve_matches_oracle(b5, c5):
    dims, Ls = (4, 4, 4, 8), 6
    U = fg.gauge_field(dims, 115, "smooth", 0.3)
    b = field5(dims, Ls, 116)
    op = dwf.DomainWall(U, 1.8, 0.1, Ls, -1, b5, c5)
    lat = lattice(dims, U, 0.12, 0.0)
    x = to_dev(np.zeros_like(b))
    st = lat.dwf_solve(Ls, 1.8, 0.1, to_dev(b), x, tol=1e-10, b5=b5, c5=c5)
    xh = from_dev(x)
    r = np.linalg.norm(b - op.D(xh)) / np.linalg.norm(b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    xo, info = dwf.solve(op, b, tol=1e-12)
    assert info.converged
    assert dirac.rel_l2(xh, xo) <= 1e-8


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_dwf_native_apply_matches_oracle(prec, b5, c5):
    """The bench's path: import, D and D^dag on native fields (left
    uninitialised before the import, padding included), export."""
    import torch
    dims, Ls = (4, 6, 8, 10), 5
    U = fg.gauge_field(dims, 117, "haar")
    psi = field5(dims, Ls, 118)
    op = dwf.DomainWall(U, 1.8, 0.04, Ls, -1, b5, c5)
    lat = lattice(dims, U, 0.12, 0.0)
    nb = lat.dwf_field_bytes(prec, Ls)
    src, dst, tmp = (torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(3))
    lat.dwf_import(prec, Ls, to_dev(psi), src)
    for dag, want in ((False, op.D(psi)), (True, op.Ddag(psi))):
        lat.dwf_apply_native_repeat(Ls, 1.8, 0.04, prec, [src], [dst], 1, dag=dag, b5=b5, c5=c5, tmp=tmp)
        got = to_dev(np.zeros_like(psi))
        lat.dwf_export(prec, Ls, dst, got)
        torch.cuda.synchronize()
        assert dirac.rel_l2(from_dev(got), want) <= TOL[prec]


@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 4), ((4, 6, 8, 10), 3), ((4, 4, 16, 4), 8), ((2, 2, 2, 4), 1)])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_dwf_schur_matches_oracle(dims, Ls, prec, b5, c5):
    U = fg.gauge_field(dims, 119, "haar")
    op = dwf.DomainWall(U, 1.8, 0.05, Ls, -1, b5, c5)
    eo = dwf.EvenOdd(op)
    psi = field5(dims, Ls, 120)
    lat = lattice(dims, U, 0.12, 0.0)
    for dag, want in ((False, eo.schur(psi)), (True, eo.schur_dag(psi))):
        out = to_dev(np.ones_like(psi))
        lat.dwf_apply_schur(Ls, 1.8, 0.05, prec, to_dev(psi), out, dag=dag, b5=b5, c5=c5)
        assert dirac.rel_l2(from_dev(out), want) <= TOL[prec]


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_dwf_solve_eo_matches_oracle(b5, c5):
    dims, Ls = (4, 4, 4, 8), 6
    U = fg.gauge_field(dims, 121, "smooth", 0.3)
    b = field5(dims, Ls, 122)
    op = dwf.DomainWall(U, 1.8, 0.1, Ls, -1, b5, c5)
    lat = lattice(dims, U, 0.12, 0.0)
    x = to_dev(np.zeros_like(b))
    st = lat.dwf_solve_eo(Ls, 1.8, 0.1, to_dev(b), x, tol=1e-10, b5=b5, c5=c5)
    xh = from_dev(x)
    r = np.linalg.norm(b - op.D(xh)) / np.linalg.norm(b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    xo, info = dwf.EvenOdd(op).solve(b, tol=1e-12)
    assert info.converged
    assert dirac.rel_l2(xh, xo) <= 1e-8
    # the even-odd system needs fewer iterations than the full normal equations
    st_full = lat.dwf_solve(Ls, 1.8, 0.1, to_dev(b), to_dev(np.zeros_like(b)), tol=1e-10, b5=b5, c5=c5)
    assert st.inner_iters < st_full.inner_iters, (st, st_full)


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
@pytest.mark.parametrize("inner_tol", [0.0, 1e-3])
def test_dwf_solve_eo_mixed_matches_oracle(b5, c5, inner_tol):
    """FP32 inner CG under FP64 defect correction reaches the FP64 tolerance:
    the oracle's residual of the GPU's x and the oracle's solution agree as
    for the FP64 solve."""
    dims, Ls = (4, 4, 4, 8), 6
    U = fg.gauge_field(dims, 125, "smooth", 0.3)
    b = field5(dims, Ls, 126)
    op = dwf.DomainWall(U, 1.8, 0.1, Ls, -1, b5, c5)
    lat = lattice(dims, U, 0.12, 0.0)
    x = to_dev(np.zeros_like(b))
    st = lat.dwf_solve_eo(Ls, 1.8, 0.1, to_dev(b), x, tol=1e-10, b5=b5, c5=c5, inner_prec=lqcd.F32,
                          inner_tol=inner_tol)
    xh = from_dev(x)
    r = np.linalg.norm(b - op.D(xh)) / np.linalg.norm(b)
    assert st.true_rel_resid <= 1e-10 and r <= 1e-10, (st, r)
    assert st.outer_iters >= 2, st  # FP32 alone cannot reach 1e-10: at least one correction pass
    xo, info = dwf.EvenOdd(op).solve(b, tol=1e-12)
    assert info.converged
    assert dirac.rel_l2(xh, xo) <= 1e-8


@pytest.mark.parametrize("form", ["full", "eo_f64", "eo_f32"])
def test_dwf_solve_zero_source(form):
    """b = 0 gives x = 0 with no iteration, whatever x held."""
    dims, Ls = (4, 4, 4, 4), 4
    U = fg.gauge_field(dims, 129, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    b = np.zeros((Ls, 4, 4, 4, 4, 4, 3), dtype=np.complex128)
    x = to_dev(np.ones_like(b))
    if form == "full":
        st = lat.dwf_solve(Ls, 1.8, 0.1, to_dev(b), x)
    else:
        st = lat.dwf_solve_eo(Ls, 1.8, 0.1, to_dev(b), x, inner_prec=lqcd.F64 if form == "eo_f64" else lqcd.F32)
    assert st.true_rel_resid == 0.0 and st.inner_iters == 0 and np.all(from_dev(x) == 0), st


@pytest.mark.parametrize("inner_prec", [0, 1])
def test_dwf_solve_eo_is_deterministic(inner_prec):
    """Fixed-order reductions: two even-odd solves of the same system give the
    same x bit for bit (FP64 and FP32-inner)."""
    dims, Ls = (4, 4, 8, 8), 6
    U = fg.gauge_field(dims, 132, "smooth", 0.3)
    b = to_dev(field5(dims, Ls, 133))
    lat = lattice(dims, U, 0.12, 0.0)
    xs, its = [], []
    for _ in range(2):
        x = to_dev(np.zeros(b.shape, dtype=np.complex128))
        st = lat.dwf_solve_eo(Ls, 1.8, 0.1, b, x, b5=1.5, c5=0.5, inner_prec=inner_prec)
        xs.append(from_dev(x))
        its.append(st.inner_iters)
    assert np.array_equal(xs[0], xs[1]) and its[0] == its[1]


@pytest.mark.parametrize("Ls", [256, 255])
def test_dwf_largest_ls_matches_oracle(Ls):
    """The largest fifth dimension a workgroup holds (one 4-d site of 256
    lanes) and an odd one just below (255 lanes of 256 live): D and D^dag
    against the oracle in FP64 and FP32."""
    dims = (2, 2, 2, 4)
    U = fg.gauge_field(dims, 134, "haar")
    psi = field5(dims, Ls, 135)
    op = dwf.DomainWall(U, 1.8, 0.05, Ls, -1, 1.5, 0.5)
    lat = lattice(dims, U, 0.12, 0.0)
    for prec in (0, 1):
        for dag in (False, True):
            out = to_dev(np.zeros_like(psi))
            lat.dwf_apply(Ls, 1.8, 0.05, prec, to_dev(psi), out, dag=dag, b5=1.5, c5=0.5)
            want = op.Ddag(psi) if dag else op.D(psi)
            assert dirac.rel_l2(from_dev(out), want) <= TOL[prec], (prec, dag)


def test_dwf_solve_eo_rejects_fp16_inner():
    dims, Ls = (4, 4, 4, 4), 4
    U = fg.gauge_field(dims, 127, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    b = to_dev(field5(dims, Ls, 128))
    st = lat.dwf_solve_eo(Ls, 1.8, 0.1, b, to_dev(np.zeros(b.shape, dtype=np.complex128)), inner_prec=lqcd.F16,
                          raise_on_fail=False)
    assert st.status == lqcd.EINVAL


def test_dwf_adjoint_at_benchmark_size():
    """<a, D b> = <D^dag a, b> and the same for S_ee at the benchmarked size
    (64x32x16x8, Ls 8, Moebius), where the oracle would be slow: a property
    that holds at any size, FP64."""
    import torch
    dims, Ls, M5, mf, b5, c5 = (64, 32, 16, 8), 8, 1.8, 0.05, 1.5, 0.5
    U = fg.gauge_field(dims, 123, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    lx, ly, lz, lt = dims
    gen = torch.Generator(device="cuda")
    gen.manual_seed(124)
    shape = (Ls, lt, lz, ly, lx, 4, 3)

    def rnd():
        return torch.complex(torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64),
                             torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64))

    a, b = rnd(), rnd()
    out = torch.empty_like(a)
    for apply in (lat.dwf_apply, lat.dwf_apply_schur):
        apply(Ls, M5, mf, 0, b, out, b5=b5, c5=c5)
        lhs = torch.vdot(a.flatten(), out.flatten()).item()
        apply(Ls, M5, mf, 0, a, out, dag=True, b5=b5, c5=c5)
        rhs = torch.vdot(out.flatten(), b.flatten()).item()
        # (S_ee: both outputs vanish on the odd sites, so only the even sites of a and b enter)
        assert abs(lhs - rhs) <= 1e-11 * abs(lhs), (apply, lhs, rhs)


def test_dwf_sampled_at_benchmark_size():
    """D, D^dag, S_ee and S_ee^dag at the benchmarked size (64x32x16x8, Ls 8,
    Moebius b5 1.5, c5 0.5) against the oracle evaluated site by site
    (oracle.sampled) at random sites and at sites on the edges of every
    direction (the antiperiodic t boundary and the XCD z-slab boundaries),
    FP64 to 1e-13 and FP32 to 1e-5."""
    from oracle import sampled
    dims, Ls, M5, mf, b5, c5 = (64, 32, 16, 8), 8, 1.8, 0.05, 1.5, 0.5
    U = fg.gauge_field(dims, 125, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    psi = field5(dims, Ls, 126)
    x = to_dev(psi)
    out = to_dev(np.zeros_like(psi))

    def sites(parity, seed):
        s = sampled.random_sites(dims, 40, seed, parity)
        edges = []
        for t in (0, dims[3] - 1):
            for z in (0, 1, 2, dims[2] - 1):
                for xx in (0, dims[0] - 1):
                    c = np.array([xx, dims[1] - 1, z, t])
                    if c.sum() % 2 != parity:
                        c[1] = 0
                    edges.append(c)
        return np.concatenate([s, np.array(edges)])

    sa = np.concatenate([sites(0, 127), sites(1, 128)])
    se = sites(0, 129)
    xe = dwf.parity5(dwf.DomainWall(U, M5, mf, Ls, -1, b5, c5), psi, 0)
    for dag in (False, True):
        want = sampled.dwf_at(U, psi, M5, mf, b5, c5, -1, sa, dag)
        want_s = sampled.dwf_schur_at(U, xe, M5, mf, b5, c5, -1, se, dag)
        for prec in (0, 1):
            lat.dwf_apply(Ls, M5, mf, prec, x, out, dag=dag, b5=b5, c5=c5)
            got = sampled.gather5(from_dev(out), sa)
            assert dirac.rel_l2(got, want) <= TOL[prec], ("D", dag, prec)
            lat.dwf_apply_schur(Ls, M5, mf, prec, x, out, dag=dag, b5=b5, c5=c5)
            got = sampled.gather5(from_dev(out), se)
            assert dirac.rel_l2(got, want_s) <= TOL[prec], ("S_ee", dag, prec)


def test_dwf_mixed_solve_at_benchmark_size():
    """The even-odd solve with FP32 inner CG at the benchmarked size
    (64x32x16x8, Ls 8, Moebius): the oracle's D applied to the GPU's x at
    random and edge sites reproduces b there (sampled residual against the
    sampled b), independently of the library's own residual."""
    from oracle import sampled
    dims, Ls, M5, mf, b5, c5 = (64, 32, 16, 8), 8, 1.8, 0.05, 1.5, 0.5
    U = fg.gauge_field(dims, 125, "smooth", 0.3)
    lat = lattice(dims, U, 0.12, 0.0)
    b = field5(dims, Ls, 130)
    x = to_dev(np.zeros_like(b))
    st = lat.dwf_solve_eo(Ls, M5, mf, to_dev(b), x, b5=b5, c5=c5, inner_prec=lqcd.F32)
    assert st.true_rel_resid <= 1e-10 and st.outer_iters >= 2, st
    xh = from_dev(x)
    del x
    edges = np.array([[xx, yy, zz, tt] for xx in (0, 63) for yy in (0, 31) for zz in (0, 15) for tt in (0, 7)])
    sites = np.concatenate([sampled.random_sites(dims, 48, 131), edges])
    dx = sampled.dwf_at(U, xh, M5, mf, b5, c5, -1, sites)
    bs = sampled.gather5(b, sites)
    assert np.linalg.norm(bs - dx) / np.linalg.norm(bs) <= 1e-9


def test_dwf_walks_agree(monkeypatch):
    """The four XCD walks (linear, z-slabs, y-ranges, x-ranges) only reorder
    the sites: D, D^dag and S_ee agree bit for bit on a lattice all four fit,
    and match the oracle."""
    dims, Ls, b5, c5 = (16, 8, 8, 4), 4, 1.5, 0.5
    U = fg.gauge_field(dims, 131, "haar")
    op = dwf.DomainWall(U, 1.8, 0.05, Ls, -1, b5, c5)
    psi = field5(dims, Ls, 132)
    lat = lattice(dims, U, 0.12, 0.0)
    results = {}
    for walk in ("0", "1", "2", "3"):
        monkeypatch.setenv("LQCD_DWF_WALK", walk)
        outs = []
        for prec in (0, 1):
            for dag in (False, True):
                out = to_dev(np.zeros_like(psi))
                lat.dwf_apply(Ls, 1.8, 0.05, prec, to_dev(psi), out, dag=dag, b5=b5, c5=c5)
                outs.append(from_dev(out))
            out = to_dev(np.zeros_like(psi))
            lat.dwf_apply_schur(Ls, 1.8, 0.05, prec, to_dev(psi), out, b5=b5, c5=c5)
            outs.append(from_dev(out))
        results[walk] = outs
    for walk in ("1", "2", "3"):
        for a, b in zip(results["0"], results[walk]):
            assert np.array_equal(a, b), walk
    assert dirac.rel_l2(results["2"][0], op.D(psi)) <= TOL[0]
    assert dirac.rel_l2(results["2"][1], op.Ddag(psi)) <= TOL[0]
