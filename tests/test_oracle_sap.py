"""Pins of the SAP preconditioner and flexible BiCGStab oracle (oracle/sap.py)
against facts fixed independently of it: the brute-force dense matrix
restricted to the block sites, LAPACK solves of the block systems and of the
full system (Schwarz iteration with exact block solves converges to D^-1),
homogeneity and gauge covariance of the preconditioner, and BiCGStab itself
(flexible BiCGStab with the identity as preconditioner is BiCGStab)."""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dense, dirac, sap, solvers

DIMS = (4, 4, 4, 4)
BDIMS = (2, 2, 2, 2)


def setup(kappa, csw, seed=31, kind="smooth"):
    U = fg.gauge_field(DIMS, seed, kind, 0.3)
    op = dirac.Operator(U, kappa, csw)
    return U, op


def colour_index(blocks, colour):
    """Dense-vector indices (12 * site + 3 * spin + colour) of one colour's sites."""
    lx, ly, lz, lt = DIMS
    idx = []
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    if blocks.colour[t, z, y, x] == colour:
                        s = dense.site_index(DIMS, x, y, z, t)
                        idx.extend(range(12 * s, 12 * s + 12))
    return np.array(idx)


def test_blocks_colouring():
    b = sap.Blocks(DIMS, BDIMS)
    assert b.count == 16 and b.nblocks == (2, 2, 2, 2)
    # neighbouring blocks differ in colour; every block holds 16 sites
    assert np.bincount(b.block_id.ravel()).tolist() == [16] * 16
    for axis in range(4):
        assert np.all(b.colour != np.roll(b.colour, 2, axis=axis))
    with pytest.raises(ValueError):
        sap.Blocks((4, 4, 4, 6), (2, 2, 2, 2))  # three blocks in t


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_block_operator_is_dense_restriction(csw):
    U, op = setup(0.13, csw)
    blocks = sap.Blocks(DIMS, BDIMS)
    M = dense.dense_dirac(U, 0.13, csw)
    psi = fg.gaussian_spinor(DIMS, 7)
    v = dense.to_vector(psi)
    for colour in (0, 1):
        idx = colour_index(blocks, colour)
        want = np.zeros_like(v)
        want[idx] = M[np.ix_(idx, idx)] @ v[idx]
        got = dense.to_vector(sap.block_apply(op.D, blocks, colour, psi))
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_mr_converges_to_block_solve():
    U, op = setup(0.10, 1.0)
    blocks = sap.Blocks(DIMS, BDIMS)
    M = dense.dense_dirac(U, 0.10, 1.0)
    rho = fg.gaussian_spinor(DIMS, 8)
    for colour in (0, 1):
        idx = colour_index(blocks, colour)
        want = np.zeros(M.shape[0], dtype=np.complex128)
        want[idx] = np.linalg.solve(M[np.ix_(idx, idx)], dense.to_vector(rho)[idx])
        got = dense.to_vector(sap.mr_blocks(op.D, blocks, colour, rho, 200))
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


def test_sap_with_exact_blocks_converges_to_solution():
    U, op = setup(0.10, 1.0)
    blocks = sap.Blocks(DIMS, BDIMS)
    M = dense.dense_dirac(U, 0.10, 1.0)
    eta = fg.gaussian_spinor(DIMS, 9)
    want = np.linalg.solve(M, dense.to_vector(eta))
    got = dense.to_vector(sap.sap(op.D, blocks, eta, ncy=40, n_mr=60))
    assert np.linalg.norm(got - want) <= 1e-8 * np.linalg.norm(want)
    # a planted mistake: the block right-hand side taken from eta alone
    # instead of the current residual eta - D psi does not converge
    psi = np.zeros_like(eta)
    for _ in range(40):
        for colour in (0, 1):
            rho = np.where(blocks.mask(colour), eta, 0)
            psi = psi + sap.mr_blocks(op.D, blocks, colour, rho, 60)
    assert np.linalg.norm(dense.to_vector(psi) - want) > 1e-3 * np.linalg.norm(want)


def test_sap_homogeneous_and_gauge_covariant():
    U, op = setup(0.13, 1.0, kind="haar")
    blocks = sap.Blocks(DIMS, BDIMS)
    eta = fg.gaussian_spinor(DIMS, 10)
    m = sap.sap(op.D, blocks, eta, ncy=2, n_mr=4)
    c = 0.7 - 1.9j
    assert np.abs(sap.sap(op.D, blocks, c * eta, 2, 4) - c * m).max() <= 1e-12 * np.abs(c * m).max()
    G = fg.random_su3_field(DIMS, 11)
    opg = dirac.Operator(dirac.gauge_transform(U, G), 0.13, 1.0)
    mg = sap.sap(opg.D, blocks, dirac.transform_spinor(eta, G), ncy=2, n_mr=4)
    want = dirac.transform_spinor(m, G)
    assert np.abs(mg - want).max() <= 1e-12 * np.abs(want).max()


def test_fbicgstab_with_identity_is_bicgstab():
    U, op = setup(0.13, 1.0)
    b = fg.gaussian_spinor(DIMS, 12)
    x1, i1 = solvers.bicgstab(op.D, b, tol=1e-10)
    x2, i2 = sap.fbicgstab(op.D, lambda v: v, b, tol=1e-10)
    assert i1.iterations == i2.iterations and i1.converged and i2.converged
    assert np.abs(x1 - x2).max() <= 1e-10 * np.abs(x1).max()


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_fbicgstab_sap_matches_lapack(csw):
    kappa = 0.135
    U, op = setup(kappa, csw)
    blocks = sap.Blocks(DIMS, BDIMS)
    b = fg.gaussian_spinor(DIMS, 13)
    x, info = sap.fbicgstab(op.D, lambda v: sap.sap(op.D, blocks, v, 2, 4), b, tol=1e-10)
    assert info.converged and info.residual <= 1e-10
    want = np.linalg.solve(dense.dense_dirac(U, kappa, csw), dense.to_vector(b))
    assert np.linalg.norm(dense.to_vector(x) - want) <= 1e-8 * np.linalg.norm(want)
    _, plain = solvers.bicgstab(op.D, b, tol=1e-10)
    assert info.iterations < plain.iterations


def dense_block_mr(M, blocks, colour, rho_vec, n_mr):
    """n_mr minimal-residual steps on each block of one colour separately, with
    the block matrix M[B, B] cut out of the brute-force dense matrix and one
    coefficient per block, written without the oracle's block machinery."""
    delta = np.zeros_like(rho_vec)
    lx, ly, lz, lt = DIMS
    for blk in range(blocks.count):
        idx = []
        for t in range(lt):
            for z in range(lz):
                for y in range(ly):
                    for x in range(lx):
                        if blocks.block_id[t, z, y, x] == blk and blocks.colour[t, z, y, x] == colour:
                            s = dense.site_index(DIMS, x, y, z, t)
                            idx.extend(range(12 * s, 12 * s + 12))
        if not idx:
            continue
        idx = np.array(idx)
        MB = M[np.ix_(idx, idx)]
        r = rho_vec[idx].copy()
        d = np.zeros_like(r)
        for _ in range(n_mr):
            q = MB @ r
            a = np.vdot(q, r) / np.vdot(q, q).real
            d += a * r
            r -= a * q
        delta[idx] = d
    return delta


@pytest.mark.parametrize("n_mr", [1, 2, 5])
def test_mr_steps_equal_blockwise_dense_mr(n_mr):
    """A few MR steps (far from converged) equal the same steps taken block by
    block on the dense block matrices, each block with its own coefficient
    (Sec. 3: the SAP smoother solves every block approximately on its own)."""
    U, op = setup(0.13, 1.0)
    blocks = sap.Blocks(DIMS, BDIMS)
    M = dense.dense_dirac(U, 0.13, 1.0)
    rho = fg.gaussian_spinor(DIMS, 14)
    for colour in (0, 1):
        rho_c = np.where(blocks.mask(colour), rho, 0)
        want = dense_block_mr(M, blocks, colour, dense.to_vector(rho_c), n_mr)
        got = dense.to_vector(sap.mr_blocks(op.D, blocks, colour, rho_c, n_mr))
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_mr_one_coefficient_per_colour_is_caught():
    """A planted mistake, one MR coefficient for all blocks of a colour instead
    of one per block, fails the blockwise dense MR pin."""
    U, op = setup(0.13, 1.0)
    blocks = sap.Blocks(DIMS, BDIMS)
    M = dense.dense_dirac(U, 0.13, 1.0)
    rho = fg.gaussian_spinor(DIMS, 14)
    colour = 0
    m = blocks.mask(colour)
    r = np.where(m, rho, 0)
    delta = np.zeros_like(rho)
    for _ in range(2):
        q = sap.block_apply(op.D, blocks, colour, r)
        a = np.vdot(q, r) / np.vdot(q, q).real
        delta = delta + np.where(m, a * r, 0)
        r = r - np.where(m, a * q, 0)
    want = dense_block_mr(M, blocks, colour, dense.to_vector(np.where(m, rho, 0)), 2)
    assert np.abs(dense.to_vector(delta) - want).max() > 1e-3 * np.abs(want).max()


def blockwise_dense_eo(M, blocks, colour, rho_vec, n_mr):
    """The even-odd block solve written on the dense matrices, block by block:
    with MB = M[B, B] split by site parity, S = MB_ee - MB_eo MB_oo^-1 MB_oe,
    n_mr MR steps on S delta_e = rho_e - MB_eo MB_oo^-1 rho_o (one coefficient
    per block), delta_o = MB_oo^-1 (rho_o - MB_oe delta_e)."""
    delta = np.zeros_like(rho_vec)
    lx, ly, lz, lt = DIMS
    for blk in range(blocks.count):
        ev, od = [], []
        for t in range(lt):
            for z in range(lz):
                for y in range(ly):
                    for x in range(lx):
                        if blocks.block_id[t, z, y, x] == blk and blocks.colour[t, z, y, x] == colour:
                            s = dense.site_index(DIMS, x, y, z, t)
                            (ev if (x + y + z + t) % 2 == 0 else od).extend(range(12 * s, 12 * s + 12))
        if not ev:
            continue
        ev, od = np.array(ev), np.array(od)
        Mee, Meo = M[np.ix_(ev, ev)], M[np.ix_(ev, od)]
        Moe, Moo = M[np.ix_(od, ev)], M[np.ix_(od, od)]
        Mooi = np.linalg.inv(Moo)
        S = Mee - Meo @ Mooi @ Moe
        r = rho_vec[ev] - Meo @ Mooi @ rho_vec[od]
        d = np.zeros_like(r)
        for _ in range(n_mr):
            q = S @ r
            a = np.vdot(q, r) / np.vdot(q, q).real
            d += a * r
            r -= a * q
        delta[ev] = d
        delta[od] = Mooi @ (rho_vec[od] - Moe @ d)
    return delta


@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("n_mr", [1, 2, 4])
def test_mr_eo_steps_equal_blockwise_dense_schur(csw, n_mr):
    """The even-odd block solve (a few MR steps on each block's Schur
    complement, the odd sites exact) equals the same steps written on the
    dense block matrix split by site parity."""
    U, op = setup(0.13, csw)
    blocks = sap.Blocks(DIMS, BDIMS)
    M = dense.dense_dirac(U, 0.13, csw)
    rho = fg.gaussian_spinor(DIMS, 15)
    for colour in (0, 1):
        rho_c = np.where(blocks.mask(colour), rho, 0)
        want = blockwise_dense_eo(M, blocks, colour, dense.to_vector(rho_c), n_mr)
        got = dense.to_vector(sap.mr_blocks_eo(op, blocks, colour, rho_c, n_mr))
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_mr_eo_converges_to_block_solve_and_a_planted_sign_fails():
    U, op = setup(0.10, 1.0)
    blocks = sap.Blocks(DIMS, BDIMS)
    M = dense.dense_dirac(U, 0.10, 1.0)
    rho = fg.gaussian_spinor(DIMS, 16)
    for colour in (0, 1):
        idx = colour_index(blocks, colour)
        want = np.zeros(M.shape[0], dtype=np.complex128)
        want[idx] = np.linalg.solve(M[np.ix_(idx, idx)], dense.to_vector(rho)[idx])
        got = dense.to_vector(sap.mr_blocks_eo(op, blocks, colour, rho, 60))
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
    # planted: the odd-site correction of the even right-hand side with the
    # wrong sign converges to something else
    colour = 0
    idx = colour_index(blocks, colour)
    want = np.linalg.solve(M[np.ix_(idx, idx)], dense.to_vector(rho)[idx])
    bad = dirac.Operator(U, 0.10, 1.0)
    bad.kappa = -0.10  # flips kappa in the rhs correction and the odd solve, not in A
    got = dense.to_vector(sap.mr_blocks_eo(bad, blocks, colour, rho, 60))[idx]
    assert np.linalg.norm(got - want) > 1e-3 * np.linalg.norm(want)


def test_sap_eo_homogeneous_covariant_and_fbicgstab_matches_lapack():
    kappa = 0.135
    U, op = setup(kappa, 1.0, kind="haar")
    blocks = sap.Blocks(DIMS, BDIMS)
    eta = fg.gaussian_spinor(DIMS, 17)
    m = sap.sap_eo(op, blocks, eta, 2, 2)
    c = -1.3 + 0.4j
    assert np.abs(sap.sap_eo(op, blocks, c * eta, 2, 2) - c * m).max() <= 1e-12 * np.abs(c * m).max()
    G = fg.random_su3_field(DIMS, 18)
    opg = dirac.Operator(dirac.gauge_transform(U, G), kappa, 1.0)
    mg = sap.sap_eo(opg, blocks, dirac.transform_spinor(eta, G), 2, 2)
    want = dirac.transform_spinor(m, G)
    assert np.abs(mg - want).max() <= 1e-12 * np.abs(want).max()
    U, op = setup(kappa, 1.0)
    b = fg.gaussian_spinor(DIMS, 19)
    x, info = sap.fbicgstab(op.D, lambda v: sap.sap_eo(op, blocks, v, 2, 2), b, tol=1e-10)
    assert info.converged
    want = np.linalg.solve(dense.dense_dirac(U, kappa, 1.0), dense.to_vector(b))
    assert np.linalg.norm(dense.to_vector(x) - want) <= 1e-8 * np.linalg.norm(want)
