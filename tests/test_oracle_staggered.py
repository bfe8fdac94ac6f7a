"""Pins of the staggered-operator oracle (oracle/staggered.py) against facts
fixed independently of it: a brute-force dense matrix built entry by entry,
anti-hermiticity of the hopping term, the free-field identity
H^2 = 1/4 sum_mu (T_2mu + T_-2mu - 2) (which holds only with the correct
staggered phases), gauge covariance, and LAPACK solves of the full and the
even-odd systems."""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dirac, staggered


def dense_staggered(U, mass, t_bc):
    """3V x 3V matrix of D = m + H, written site by site with explicit
    coordinates (index 3 * site + colour, site = x + Lx (y + Ly (z + Lz t)))."""
    lt, lz, ly, lx = U.shape[:4]
    dims = (lx, ly, lz, lt)
    n = 3 * lx * ly * lz * lt
    M = mass * np.eye(n, dtype=np.complex128)

    def idx(c):
        x, y, z, t = c
        return x + lx * (y + ly * (z + lz * t))

    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = (x, y, z, t)
                    eta = (1, (-1) ** x, (-1) ** (x + y), (-1) ** (x + y + z))
                    i = idx(c)
                    for mu in range(4):
                        f = list(c)
                        f[mu] = (c[mu] + 1) % dims[mu]
                        b = list(c)
                        b[mu] = (c[mu] - 1) % dims[mu]
                        sf = t_bc if (mu == 3 and c[3] == dims[3] - 1) else 1
                        sb = t_bc if (mu == 3 and c[3] == 0) else 1
                        j = idx(f)
                        M[3 * i:3 * i + 3, 3 * j:3 * j + 3] += 0.5 * eta[mu] * sf * U[t, z, y, x, mu]
                        bx, by, bz, bt = b
                        k = idx(b)
                        M[3 * i:3 * i + 3, 3 * k:3 * k + 3] -= 0.5 * eta[mu] * sb * np.conj(U[bt, bz, by, bx, mu]).T
    return M


def vec(psi):
    return psi.reshape(-1)


def colour_field(dims, seed):
    rng = np.random.default_rng(seed)
    lx, ly, lz, lt = dims
    return (rng.normal(size=(lt, lz, ly, lx, 3)) + 1j * rng.normal(size=(lt, lz, ly, lx, 3))) / np.sqrt(2)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 4), (4, 4, 4, 4)])
@pytest.mark.parametrize("t_bc", [-1, 1])
def test_dense_brute_force(dims, t_bc):
    U = fg.gauge_field(dims, 61, "haar")
    op = staggered.Staggered(U, 0.2, t_bc)
    psi = colour_field(dims, 62)
    M = dense_staggered(U, 0.2, t_bc)
    assert np.abs(vec(op.D(psi)) - M @ vec(psi)).max() <= 1e-13


def test_hop_anti_hermitian():
    dims = (4, 4, 4, 6)
    U = fg.gauge_field(dims, 63, "haar")
    op = staggered.Staggered(U, 0.0)
    a, b = colour_field(dims, 64), colour_field(dims, 65)
    assert abs(np.vdot(a, op.hop(b)) + np.vdot(op.hop(a), b)) <= 1e-12 * np.abs(a).sum()


def test_free_field_square():
    dims = (4, 6, 4, 8)
    lt, lz, ly, lx = dims[3], dims[2], dims[1], dims[0]
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (lt, lz, ly, lx, 4, 3, 3)).copy()
    psi = colour_field(dims, 66)
    h2 = staggered.hop(U, staggered.hop(U, psi, +1), +1)
    want = np.zeros_like(psi)
    for mu in range(4):
        want += 0.25 * (dirac.shift(psi, mu, 2) + dirac.shift(psi, mu, -2) - 2 * psi)
    assert np.abs(h2 - want).max() <= 1e-13
    # a planted mistake, eta_y = (-1)^y instead of (-1)^x, breaks it
    orig = staggered.phases

    def wrong(d):
        e = orig(d)
        lx_, ly_, lz_, lt_ = d
        y = np.arange(ly_)[None, None, :, None]
        e[..., 1] = np.broadcast_to((-1.0) ** y, e[..., 1].shape)
        return e

    staggered.phases = wrong
    try:
        bad = staggered.hop(U, staggered.hop(U, psi, +1), +1)
    finally:
        staggered.phases = orig
    assert np.abs(bad - want).max() > 1e-3


def test_gauge_covariance():
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 67, "haar")
    G = fg.random_su3_field(dims, 68)
    psi = colour_field(dims, 69)
    op = staggered.Staggered(U, 0.3)
    opg = staggered.Staggered(dirac.gauge_transform(U, G), 0.3)
    gpsi = np.einsum("...ab,...b->...a", G, psi)
    want = np.einsum("...ab,...b->...a", G, op.D(psi))
    assert np.abs(opg.D(gpsi) - want).max() <= 1e-12


def test_even_odd_solve_matches_lapack():
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 70, "smooth", 0.3)
    b = colour_field(dims, 71)
    op = staggered.Staggered(U, 0.1)
    # the normal operator is Hermitian positive definite
    u, v = colour_field(dims, 72) * (op.par == 0), colour_field(dims, 73) * (op.par == 0)
    assert abs(np.vdot(u, op.schur(v)) - np.conj(np.vdot(v, op.schur(u)))) <= 1e-12 * np.abs(u).sum()
    assert np.vdot(v, op.schur(v)).real > 0
    x, info = staggered.solve(op, b, tol=1e-11)
    assert info.converged
    want = np.linalg.solve(dense_staggered(U, 0.1, -1), vec(b))
    assert np.linalg.norm(vec(x) - want) <= 1e-8 * np.linalg.norm(want)
    assert np.linalg.norm(vec(b - op.D(x))) <= 1e-10 * np.linalg.norm(vec(b))
