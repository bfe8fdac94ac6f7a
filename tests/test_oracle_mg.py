"""Pins of the two-level multigrid oracle (oracle/mg.py) against facts fixed
independently of it: the chiral change of basis against gamma5's action,
orthonormality and chirality of the prolongation's columns, the span of the
test vectors, the nearest-neighbour stencil and Gamma5-hermiticity that the
coarse operator inherits from D, exactness of the coarse-grid correction on
the coarse space, and the multigrid-preconditioned solve against LAPACK (a
planted mistake, aggregation without the chiral split, breaks the coarse
operator's Gamma5-hermiticity)."""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dense, dirac, mg, sap

DIMS = (4, 4, 4, 4)
ADIMS = (2, 2, 2, 2)


def system(n=3, kappa=0.125, csw=1.0, seed=41):
    U = fg.gauge_field(DIMS, seed, "smooth", 0.3)
    op = dirac.Operator(U, kappa, csw)
    agg = mg.Aggregates(DIMS, ADIMS)
    vecs = [fg.gaussian_spinor(DIMS, seed + 1 + k) for k in range(n)]
    return U, op, agg, vecs


def test_chiral_basis():
    psi = fg.gaussian_spinor(DIMS, 3)
    c = mg.to_chiral(psi)
    # unitary, invertible, and gamma5 = diag(+1, -1) in the chiral basis
    assert np.isclose(np.vdot(c, c), np.vdot(psi, psi))
    assert np.abs(mg.from_chiral(c) - psi).max() <= 1e-14
    g5c = mg.to_chiral(dirac.spin_mul(dirac.GAMMA5, psi))
    assert np.abs(g5c[..., 0, :, :] - c[..., 0, :, :]).max() <= 1e-14
    assert np.abs(g5c[..., 1, :, :] + c[..., 1, :, :]).max() <= 1e-14


def test_prolongation_orthonormal_chiral_and_spans_vectors():
    _, _, agg, vecs = system()
    P = mg.Prolongation(agg, vecs)
    nc = P.ncoarse
    assert nc == 16 * 2 * 3
    cols = [P.prolong(np.eye(nc)[j]) for j in range(nc)]
    G = np.array([[np.vdot(a, b) for b in cols] for a in cols])
    assert np.abs(G - np.eye(nc)).max() <= 1e-12
    for j, v in enumerate(cols):
        chi = (j // P.n) % 2
        sign = 1.0 if chi == 0 else -1.0
        assert np.abs(dirac.spin_mul(dirac.GAMMA5, v) - sign * v).max() <= 1e-13
    # every test vector lies in the coarse space: P P^dag v = v
    for v in vecs:
        assert np.abs(P.prolong(P.restrict(v)) - v).max() <= 1e-12


def neighbours(agg, a):
    nbx, nby, nbz, nbt = agg.blocks.nblocks
    x, r = a % nbx, a // nbx
    y, r = r % nby, r // nby
    z, t = r % nbz, r // nbz
    out = {a}
    for d, (c, n) in enumerate(zip((x, y, z, t), (nbx, nby, nbz, nbt))):
        for s in (-1, 1):
            cc = [x, y, z, t]
            cc[d] = (c + s) % n
            out.add(cc[0] + nbx * (cc[1] + nby * (cc[2] + nbz * cc[3])))
    return out


def gamma5_coarse(P):
    return np.tile(np.repeat([1.0, -1.0], P.n), P.agg.count)


def test_coarse_operator_stencil_and_gamma5_hermiticity():
    U, op, agg, vecs = system()
    P = mg.Prolongation(agg, vecs)
    Dc = mg.coarse_operator(op.D, P)
    n2 = 2 * P.n
    for a in range(agg.count):
        nb = neighbours(agg, a)
        for b in range(agg.count):
            blk = Dc[a * n2:(a + 1) * n2, b * n2:(b + 1) * n2]
            if b not in nb:
                assert np.abs(blk).max() == 0.0
    G = gamma5_coarse(P)
    GD = G[:, None] * Dc
    assert np.abs(GD - GD.conj().T).max() <= 1e-12
    # D_c against the dense fine matrix: P^dag M P with P assembled column-wise
    M = dense.dense_dirac(U, 0.125, 1.0)
    Pm = np.stack([dense.to_vector(P.prolong(e)) for e in np.eye(P.ncoarse)], axis=1)
    assert np.abs(Pm.conj().T @ M @ Pm - Dc).max() <= 1e-12


def test_without_chiral_split_gamma5_hermiticity_fails():
    """Planted mistake: aggregating whole spinors (no chiral split) gives a
    coarse operator that is not Gamma5-hermitian in the coarse basis."""

    class Whole(mg.Prolongation):
        def __init__(self, agg, vectors):
            super().__init__(agg, vectors)
            n = self.n
            for a in range(agg.count):
                idx = tuple(agg.sites[a].T)
                A = np.stack([vectors[k][idx].reshape(-1) for k in range(n)], axis=1)
                Q, _ = np.linalg.qr(A)
                self.basis[a] = [Q, Q]

        def restrict(self, r):
            out = np.zeros(self.ncoarse, dtype=np.complex128)
            for a in range(self.agg.count):
                idx = tuple(self.agg.sites[a].T)
                o = a * 2 * self.n
                out[o:o + self.n] = self.basis[a][0].conj().T @ r[idx].reshape(-1)
            return out

        def prolong(self, e):
            lx, ly, lz, lt = self.agg.dims
            out = np.zeros((lt, lz, ly, lx, 4, 3), dtype=np.complex128)
            for a in range(self.agg.count):
                idx = tuple(self.agg.sites[a].T)
                o = a * 2 * self.n
                out[idx] = (self.basis[a][0] @ e[o:o + self.n]).reshape(-1, 4, 3)
            return out

    _, op, agg, vecs = system()
    P = Whole(agg, vecs)
    Dc = mg.coarse_operator(op.D, P)
    G = gamma5_coarse(P)
    GD = G[:, None] * Dc
    assert np.abs(GD - GD.conj().T).max() > 1e-2


def test_coarse_correction_exact_on_coarse_space():
    _, op, agg, vecs = system()
    P = mg.Prolongation(agg, vecs)
    Dc = mg.coarse_operator(op.D, P)
    y = np.random.default_rng(5).normal(size=P.ncoarse) + 0j
    b = op.D(P.prolong(y))
    x = P.prolong(np.linalg.solve(Dc, P.restrict(b)))
    assert np.abs(x - P.prolong(y)).max() <= 1e-10


@pytest.mark.parametrize("n_iter", [0, 2])
def test_multigrid_solve_matches_lapack(n_iter):
    U, op, agg, vecs = system(n=4, kappa=0.13)
    blocks = sap.Blocks(DIMS, (2, 2, 2, 2))
    P = mg.setup(op.D, agg, vecs, blocks, n_iter, 2, 3)
    # after the setup the basis is still orthonormal
    nc = P.ncoarse
    cols = [P.prolong(np.eye(nc)[j]) for j in range(0, nc, 7)]
    G = np.array([[np.vdot(a, b) for b in cols] for a in cols])
    assert np.abs(G - np.eye(len(cols))).max() <= 1e-12
    Dc = mg.coarse_operator(op.D, P)
    pre = mg.TwoLevel(op.D, P, Dc, blocks, 2, 3, coarse_tol=0.05)
    b = fg.gaussian_spinor(DIMS, 77)
    x, info = mg.solve(op.D, b, pre, tol=1e-11)
    assert info.converged
    want = np.linalg.solve(dense.dense_dirac(U, 0.13, 1.0), dense.to_vector(b))
    assert np.linalg.norm(dense.to_vector(x) - want) <= 1e-9 * np.linalg.norm(want)


def _null_space_system():
    """Unit links, periodic in t, kappa = 1/8, no clover term: every constant
    spinor is an exact zero mode of D (the free operator at zero momentum is
    1 - 8 kappa)."""
    U = fg.gauge_field(DIMS, 0, "unit")
    op = dirac.Operator(U, 0.125, 0.0, t_bc=+1)
    c = np.random.default_rng(8).normal(size=(4, 3, 2)) @ np.array([1.0, 1j])
    v0 = np.broadcast_to(c, DIMS[::-1] + (4, 3)).copy()
    assert np.abs(op.D(v0)).max() <= 1e-14 * np.abs(v0).max()
    agg = mg.Aggregates(DIMS, ADIMS)
    start = [v0] + [fg.gaussian_spinor(DIMS, 50 + k) for k in range(2)]
    return op, agg, start, v0


@pytest.mark.parametrize("n_iter", [1, 3])
def test_setup_keeps_exact_zero_mode(n_iter):
    """The setup smooths the homogeneous equation D v = 0 (Sec. 3: SAP smoothing
    of the test vectors), which leaves an exact zero mode of D where it is, so
    the coarse space still holds it after every round: P P^dag v0 = v0."""
    op, agg, start, v0 = _null_space_system()
    blocks = sap.Blocks(DIMS, (2, 2, 2, 2))
    P = mg.setup(op.D, agg, start, blocks, n_iter, 2, 3)
    assert np.abs(P.prolong(P.restrict(v0)) - v0).max() <= 1e-12 * np.abs(v0).max()


def test_setup_reading_v_from_sap_of_v_is_caught():
    """A planted mistake, the setup round v <- M_SAP v instead of
    v <- v - M_SAP D v, moves the zero mode out of the coarse space."""
    op, agg, start, v0 = _null_space_system()
    blocks = sap.Blocks(DIMS, (2, 2, 2, 2))
    v = [np.asarray(s) for s in start]
    for _ in range(3):
        v = [sap.sap(op.D, blocks, vk, 2, 3) for vk in v]
        v = mg.Prolongation(agg, v).vectors()
    P = mg.Prolongation(agg, v)
    assert np.abs(P.prolong(P.restrict(v0)) - v0).max() > 1e-3 * np.abs(v0).max()
