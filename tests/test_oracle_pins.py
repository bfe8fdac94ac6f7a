"""Pins of the CPU oracle against facts fixed independently of it.

Each test checks the oracle against one of: the gamma-matrix algebra, a
brute-force dense matrix built entry by entry, the free-field closed form in
momentum space, gamma5-hermiticity, gauge covariance under random SU(3)
transformations, the closed-form clover term of a constant abelian flux, the
even-odd identities of Eq. (1), and LAPACK's dense solve.
"""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dense, dirac, freefield, sampled, solvers

TINY = [(2, 2, 2, 2), (2, 2, 2, 4), (4, 4, 4, 4)]


def field(dims, seed, kind="haar", eps=0.3):
    return fg.gauge_field(dims, seed, kind, eps)


def test_gamma_algebra():
    g = dirac.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu))
    # gamma5 = gamma_x gamma_y gamma_z gamma_t anticommutes with every gamma
    for mu in range(4):
        assert np.allclose(dirac.GAMMA5 @ g[mu], -g[mu] @ dirac.GAMMA5)
    assert np.allclose(dirac.GAMMA5 @ dirac.GAMMA5, np.eye(4))
    # each (1 -+ gamma_mu) is twice a rank-2 projector
    for mu in range(4):
        for s in (+1, -1):
            p = (np.eye(4) - s * g[mu]) / 2
            assert np.allclose(p @ p, p) and np.linalg.matrix_rank(p) == 2
    # the gamma matrices written entry by entry in the dense builder agree
    assert np.allclose(dense.G, g)


def test_generated_links_are_su3():
    for kind in ("haar", "smooth"):
        u = field((4, 4, 4, 4), 5, kind).reshape(-1, 3, 3)
        assert np.abs(u @ u.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-14
        assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
        # row 2 = conj(row 0 x row 1), the identity the two-row storage relies on
        assert np.abs(np.conj(np.cross(u[:, 0], u[:, 1])) - u[:, 2]).max() < 1e-14


def _plaquette(U):
    """Average Re tr / 3 of the 1x1 loops U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag."""
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            umu, unu = U[..., mu, :, :], U[..., nu, :, :]
            loop = (umu @ np.roll(unu, -1, axis=3 - mu)
                    @ np.conj(np.swapaxes(np.roll(umu, -1, axis=3 - nu), -1, -2))
                    @ np.conj(np.swapaxes(unu, -1, -2)))
            tot += np.trace(loop, axis1=-2, axis2=-1).real.mean() / 3
    return tot / 6


@pytest.mark.parametrize("eps,scale", [(0.3, 1.0), (0.25, 2 ** 0.5)])
def test_smooth_link_normalisation(eps, scale):
    """U = exp(i eps H) with H traceless Hermitian and E tr H^2 = 8 scale^2:
    H is recovered from the eigenphases of each link (theta = eps lambda), so
    the check does not repeat the generator's construction. The 5-sigma window
    excludes a dropped trace subtraction (E tr H^2 = 9 scale^2)."""
    u = fg.gauge_field((8, 8, 8, 8), 1003, "smooth", eps, scale).reshape(-1, 3, 3)
    theta = np.angle(np.linalg.eigvals(u))
    assert np.abs(theta).max() < 3.0  # no phase wrapped past pi
    lam = theta / eps
    assert np.abs(lam.sum(axis=-1)).max() <= 1e-12  # traceless
    tr = (lam ** 2).sum(axis=-1)
    sigma = tr.std() / np.sqrt(tr.size)
    assert 5 * sigma < 0.5 * scale ** 2
    assert abs(tr.mean() - 8 * scale ** 2) <= 5 * sigma


def test_smooth_link_plaquettes():
    """Links drawn independently with a conjugation-invariant law have
    E[U] = c 1, so the average plaquette is c^4 with c = E[Re tr U] / 3; and
    the recorded plaquettes of the two smooth ensembles (0.611 at eps 0.3,
    0.713 at eps 0.25)."""
    for eps, want in ((0.3, 0.611), (0.25, 0.713)):
        U = fg.gauge_field((8, 8, 8, 8), 1003, "smooth", eps)
        c = np.trace(U, axis1=-2, axis2=-1).real.mean() / 3
        p = _plaquette(U)
        assert abs(p - c ** 4) <= 3e-3
        assert abs(p - want) <= 3e-3


def test_generator_slicewise_equals_whole():
    dims = (4, 4, 2, 6)
    whole = fg.gauge_field(dims, 9, "smooth", 0.3)
    part = fg.gauge_field(dims, 9, "smooth", 0.3, t_slices=[2, 5])
    assert np.array_equal(whole[[2, 5]], part)


@pytest.mark.parametrize("dims", TINY)
@pytest.mark.parametrize("csw", [0.0, 1.3])
@pytest.mark.parametrize("t_bc", [-1, 1])
def test_dense_brute_force(dims, csw, t_bc):
    U = field(dims, 11)
    psi = fg.gaussian_spinor(dims, 12)
    op = dirac.Operator(U, 0.11, csw, t_bc)
    m = dense.dense_dirac(U, 0.11, csw, t_bc)
    ref = (m @ dense.to_vector(psi)).reshape(psi.shape)
    assert dirac.rel_l2(op.D(psi), ref) < 1e-14


@pytest.mark.parametrize("t_bc", [-1, 1])
def test_free_field_plane_waves(t_bc):
    dims = (4, 6, 8, 10)
    U = field(dims, 0, "unit")
    op = dirac.Operator(U, 0.13, 0.0, t_bc)
    rng = np.random.default_rng(3)
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 2, 0, 1), (1, 1, 3, 4), (3, 5, 7, 9)]:
        p = freefield.momentum(dims, n, t_bc)
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = freefield.plane_wave(dims, p, u)
        expect = freefield.plane_wave(dims, p, freefield.symbol(p, 0.13) @ u)
        assert dirac.rel_l2(op.D(psi), expect) < 1e-13


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 6)
    U = field(dims, 21, "smooth", 0.5)
    op = dirac.Operator(U, 0.125, 1.7, -1)
    phi = fg.gaussian_spinor(dims, 22)
    psi = fg.gaussian_spinor(dims, 23)
    lhs = np.vdot(phi, op.D(psi))
    rhs = np.vdot(dirac.gamma5(op.D(dirac.gamma5(phi))), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    # the adjoint written out term by term equals gamma5 D gamma5
    assert dirac.rel_l2(op.Ddag(phi), dirac.gamma5(op.D(dirac.gamma5(phi)))) < 1e-14
    # and is the adjoint: <phi, D psi> = <D^dag phi, psi>
    assert abs(np.vdot(op.Ddag(phi), psi) - lhs) / abs(lhs) < 1e-13


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_gauge_covariance(csw):
    dims = (4, 4, 6, 4)
    U = field(dims, 31, "smooth", 0.4)
    G = fg.random_su3_field(dims, 32)
    psi = fg.gaussian_spinor(dims, 33)
    op = dirac.Operator(U, 0.12, csw, -1)
    opg = dirac.Operator(dirac.gauge_transform(U, G), 0.12, csw, -1)
    lhs = opg.D(dirac.transform_spinor(psi, G))
    rhs = dirac.transform_spinor(op.D(psi), G)
    assert dirac.rel_l2(lhs, rhs) < 1e-13


def abelian_flux(dims, n):
    """Constant flux through every xy plaquette: each plaquette equals
    diag(e^{i phi}, e^{-i phi}, 1) with phi = 2 pi n / (Lx Ly)."""
    lx, ly, lz, lt = dims
    phi = 2 * np.pi * n / (lx * ly)
    U = fg.gauge_field(dims, 0, "unit").copy()
    for x in range(lx):
        U[:, :, :, x, 1] = np.diag([np.exp(1j * phi * x), np.exp(-1j * phi * x), 1])
    for y in range(ly):
        U[:, :, y, lx - 1, 0] = np.diag([np.exp(-1j * phi * lx * y), np.exp(1j * phi * lx * y), 1])
    return U, phi


def test_clover_abelian_flux_closed_form():
    dims = (4, 6, 2, 4)
    U, phi = abelian_flux(dims, 1)
    kappa, csw = 0.13, 1.1
    a = dirac.clover_matrix(U, kappa, csw)
    # sigma_xy = [gamma_x, gamma_y]/(2i) = diag(1, -1, 1, -1) in this basis
    sig_xy = np.diag([1.0, -1.0, 1.0, -1.0])
    f_xy = np.diag([np.sin(phi), -np.sin(phi), 0.0])
    expect = np.eye(12) + kappa * csw * np.kron(sig_xy, f_xy)
    assert np.abs(a - expect).max() < 1e-14
    assert np.abs(dirac.average_plaquette(U) - (16 + 2 * np.cos(phi)) / 18) < 1e-14


def test_clover_special_cases():
    dims = (4, 4, 4, 4)
    U = field(dims, 41, "smooth", 0.3)
    psi = fg.gaussian_spinor(dims, 42)
    # c_SW = 0 is exactly Wilson
    assert np.array_equal(dirac.Operator(U, 0.12, 0.0).D(psi), dirac.wilson(U, psi, 0.12, -1))
    # kappa = 0 is the identity
    assert np.array_equal(dirac.Operator(U, 0.0, 1.0).D(psi), psi)
    # unit links give A = 1
    a = dirac.clover_matrix(field(dims, 0, "unit"), 0.12, 1.0)
    assert np.abs(a - np.eye(12)).max() < 1e-15


def test_clover_hermitian_covariant_chiral():
    dims = (4, 4, 4, 4)
    U = field(dims, 51, "smooth", 0.6)
    G = fg.random_su3_field(dims, 52)
    a = dirac.clover_matrix(U, 0.13, 1.0)
    assert np.abs(a - dirac.dagger(a)).max() < 1e-15
    ag = dirac.clover_matrix(dirac.gauge_transform(U, G), 0.13, 1.0)
    g12 = np.einsum("st,...ab->...satb", np.eye(4), G).reshape(G.shape[:4] + (12, 12))
    assert np.abs(ag - g12 @ a @ dirac.dagger(g12)).max() < 1e-13
    # A commutes with gamma5: in the basis chi_+- = (psi_01 -+ psi_23)/sqrt2 it is
    # two 6x6 blocks, and gamma5 is diag(1, 1, -1, -1) there
    r = np.kron(np.array([[1, 0, -1, 0], [0, 1, 0, -1], [1, 0, 1, 0], [0, 1, 0, 1]]) / np.sqrt(2), np.eye(3))
    assert np.allclose(r @ np.kron(dirac.GAMMA5, np.eye(3)) @ r.T, np.diag([1.0] * 6 + [-1.0] * 6))
    b = r @ a @ r.T
    assert np.abs(b[..., :6, 6:]).max() < 1e-15 and np.abs(b[..., 6:, :6]).max() < 1e-15


def test_even_odd_blocks_sum_to_D():
    dims = (4, 4, 4, 6)
    U = field(dims, 61, "smooth", 0.3)
    op = dirac.Operator(U, 0.13, 1.0, -1)
    psi = fg.gaussian_spinor(dims, 62)
    total = op.Dee(psi) + op.Deo(psi) + op.Doe(psi) + op.Doo(psi)
    assert dirac.rel_l2(total, op.D(psi)) < 1e-15
    # the diagonal blocks are site-local: D_ee = P_e A P_e
    assert dirac.rel_l2(op.Dee(psi), dirac.mask(dirac.site_apply(op.A, psi), 0)) < 1e-15
    # the paper form D^(eo) = D_ee^-1 S
    xe = dirac.mask(psi, 0)
    assert dirac.rel_l2(op.dprec(xe), op.site_inverse(0, op.schur(xe))) < 1e-13
    # Wilson: S = 1 - kappa^2 H_eo H_oe
    w = dirac.Operator(U, 0.13, 0.0, -1)
    heh = dirac.mask(w.hop(dirac.mask(w.hop(xe), 1)), 0)
    assert dirac.rel_l2(w.schur(xe), xe - 0.13 ** 2 * heh) < 1e-14


def test_schur_solve_matches_dense_solve():
    dims = (4, 4, 4, 4)
    U = field(dims, 71, "smooth", 0.3)
    op = dirac.Operator(U, 0.13, 1.0, -1)
    b = fg.gaussian_spinor(dims, 72)
    x_dense = np.linalg.solve(dense.dense_dirac(U, 0.13, 1.0, -1), dense.to_vector(b)).reshape(b.shape)
    be = op.eo_source(b)
    xe, info = solvers.bicgstab(op.schur, be, tol=1e-12)
    assert info.converged
    x = op.eo_reconstruct(xe, b)
    assert dirac.rel_l2(x, x_dense) < 1e-10
    assert dirac.rel_l2(op.D(x), b) < 1e-11
    # the paper form reaches the same even solution
    xe2, info2 = solvers.bicgstab(op.dprec, op.site_inverse(0, be), tol=1e-12)
    assert info2.converged and dirac.rel_l2(xe2, xe) < 1e-9


def test_bicgstab_unpreconditioned_matches_lapack():
    dims = (4, 4, 4, 4)
    U = field(dims, 81, "haar")
    op = dirac.Operator(U, 0.12, 0.0, -1)
    b = fg.gaussian_spinor(dims, 82)
    x, info = solvers.bicgstab(op.D, b, tol=1e-10)
    assert info.converged and info.residual <= 1e-10
    x_dense = np.linalg.solve(dense.dense_dirac(U, 0.12), dense.to_vector(b)).reshape(b.shape)
    # ||x - x*|| <= ||D^-1|| ||r|| <= 25 * 1e-10 * ||b|| for kappa = 0.12
    assert np.linalg.norm(x - x_dense) <= 25 * 1e-10 * np.linalg.norm(b) * 1.01


def test_free_field_solve_closed_form():
    dims = (4, 4, 4, 8)
    U = field(dims, 0, "unit")
    op = dirac.Operator(U, 0.124, 0.0, -1)
    p = freefield.momentum(dims, (1, 0, 2, 3))
    u = np.arange(12).reshape(4, 3) + 1j
    b = freefield.plane_wave(dims, p, u)
    x, info = solvers.bicgstab(op.D, b, tol=1e-12)
    expect = freefield.plane_wave(dims, p, freefield.symbol_inverse(p, 0.124) @ u)
    assert info.converged and dirac.rel_l2(x, expect) < 1e-9


def test_defect_correction_reaches_tolerance():
    dims = (4, 4, 4, 4)
    U = field(dims, 91, "smooth", 0.3)
    op = dirac.Operator(U, 0.135, 1.0, -1)
    b = fg.gaussian_spinor(dims, 92)
    be = op.eo_source(b)

    def loose(r):
        return solvers.bicgstab(op.schur, r, tol=1e-3)[0]

    xe, info = solvers.defect_correction(op.schur, be, loose, tol=1e-10)
    assert info.converged and info.iterations >= 2
    assert dirac.rel_l2(op.schur(xe), be) <= 1e-10


def test_sampled_matches_whole_field():
    dims = (4, 6, 4, 8)
    U = field(dims, 101, "smooth", 0.4)
    psi = fg.gaussian_spinor(dims, 102)
    op = dirac.Operator(U, 0.13, 1.2, -1)
    sites = sampled.random_sites(dims, 40, 7)
    whole = op.D(psi)
    got = sampled.dirac_at(U, psi, 0.13, 1.2, -1, sites)
    assert np.abs(got - sampled.gather(whole, sites)).max() < 1e-13
    xe = dirac.mask(psi, 0)
    se = sampled.random_sites(dims, 40, 8, parity=0)
    got = sampled.schur_at(U, xe, 0.13, 1.2, -1, se)
    assert np.abs(got - sampled.gather(op.schur(xe), se)).max() < 1e-12


@pytest.mark.parametrize("b5,c5,t_bc", [(1.5, 0.5, -1), (1.0, 0.0, 1)])
def test_sampled_domain_wall_matches_whole_field(b5, c5, t_bc):
    """The site-sampled domain-wall D, D^dag, S_ee and S_ee^dag (H^dag as
    gamma5 H gamma5, M5op^-1 from its (s, spin) matrix) against the whole-field
    forms of oracle.dwf (H^dag term by term, M5op^-1 from unit vectors) on a
    small lattice; a wrong projector, wall sign or coefficient on either side
    fails."""
    from oracle import dwf
    dims, Ls, M5, mf = (4, 6, 4, 8), 5, 1.8, 0.07
    U = field(dims, 111, "smooth", 0.4)
    rng = np.random.default_rng(112)
    shape = (Ls, dims[3], dims[2], dims[1], dims[0], 4, 3)
    psi = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    op = dwf.DomainWall(U, M5, mf, Ls, t_bc, b5, c5)
    sites = sampled.random_sites(dims, 30, 9)
    for dag, whole in ((False, op.D(psi)), (True, op.Ddag(psi))):
        got = sampled.dwf_at(U, psi, M5, mf, b5, c5, t_bc, sites, dag)
        assert np.abs(got - sampled.gather5(whole, sites)).max() < 1e-12, dag
    eo = dwf.EvenOdd(op)
    xe = dwf.parity5(op, psi, 0)
    se = sampled.random_sites(dims, 30, 10, parity=0)
    for dag, whole in ((False, eo.schur(xe)), (True, eo.schur_dag(xe))):
        got = sampled.dwf_schur_at(U, xe, M5, mf, b5, c5, t_bc, se, dag)
        assert np.abs(got - sampled.gather5(whole, se)).max() < 1e-11, dag


def test_pins_catch_planted_mistakes(monkeypatch):
    """A plausible mistake planted in the oracle (on the CPU) fails a pin."""
    dims = (4, 4, 4, 4)
    U = field(dims, 0, "unit")
    p = freefield.momentum(dims, (1, 2, 0, 1))
    u = np.ones((4, 3), dtype=complex)
    psi = freefield.plane_wave(dims, p, u)
    expect = freefield.plane_wave(dims, p, freefield.symbol(p, 0.12) @ u)
    assert dirac.rel_l2(dirac.Operator(U, 0.12).D(psi), expect) < 1e-13
    # wrong hopping sign (1 + gamma forward)
    g = dirac.GAMMA.copy()
    monkeypatch.setattr(dirac, "GAMMA", -g)
    assert dirac.rel_l2(dirac.Operator(U, 0.12).D(psi), expect) > 1e-3
    monkeypatch.setattr(dirac, "GAMMA", g)
    # periodic instead of antiperiodic time
    monkeypatch.setattr(dirac, "boundary_factor", lambda d, mu, s, bc: np.ones((d[3], d[2], d[1], d[0])))
    assert dirac.rel_l2(dirac.Operator(U, 0.12).D(psi), expect) > 1e-3


def test_sampled_staggered_and_sap_match_whole_field():
    """The site-sampled staggered operator and the block-by-block SAP cycle
    against the whole-field oracle (oracle.staggered, oracle.sap) on small
    lattices."""
    from oracle import sap, staggered
    dims = (4, 6, 4, 8)
    U = field(dims, 121, "smooth", 0.4)
    rng = np.random.default_rng(122)
    chi = rng.normal(size=(dims[3], dims[2], dims[1], dims[0], 3)) + 1j * rng.normal(
        size=(dims[3], dims[2], dims[1], dims[0], 3))
    op = staggered.Staggered(U, 0.07, -1)
    sites = sampled.random_sites(dims, 40, 11)
    got = sampled.stag_dirac_at(U, chi, 0.07, -1, sites)
    assert np.abs(got - sampled.gather(op.D(chi), sites)).max() < 1e-13
    dims = (8, 4, 4, 8)
    U = field(dims, 123, "smooth", 0.4)
    eta = fg.gaussian_spinor(dims, 124)
    bdims = (4, 2, 2, 2)
    d = dirac.Operator(U, 0.13, 1.1, -1)
    whole = sap.sap(d.D, sap.Blocks(dims, bdims), eta, 1, 3)
    for origin in ((0, 0, 0, 0), (4, 0, 0, 0), (0, 2, 2, 6), (4, 2, 0, 4)):
        s, v = sampled.sap_one_cycle_at(U, 0.13, 1.1, -1, eta, bdims, origin, 3)
        assert np.abs(v - sampled.gather(whole, s)).max() < 1e-12 * np.abs(v).max(), origin
