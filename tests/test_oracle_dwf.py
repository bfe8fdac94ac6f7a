"""Pins of the domain-wall oracle (oracle/dwf.py) against facts fixed
independently of it: a dense 5-d matrix assembled from the brute-force dense
4-d hopping matrix (oracle/dense.py) and explicit chiral projectors written
from gamma5's entries, Gamma5-hermiticity (D^dag = gamma5 R D R gamma5 with
R the reflection s -> Ls-1-s), the Ls = 1 reduction to a Wilson operator,
gauge covariance, the adjoint, and the CG solve of the normal equations
against LAPACK."""

import numpy as np
import pytest

import fieldgen as fg
from oracle import dense, dirac, dwf


def field5(dims, Ls, seed):
    rng = np.random.default_rng(seed)
    lx, ly, lz, lt = dims
    shape = (Ls, lt, lz, ly, lx, 4, 3)
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)) / np.sqrt(2)


def gamma5_written():
    """gamma5 = gamma_x gamma_y gamma_z gamma_t of the Dirac-Pauli basis,
    entry by entry: minus the identity on the off-diagonal 2x2 blocks."""
    g = np.zeros((4, 4))
    g[0, 2] = g[1, 3] = g[2, 0] = g[3, 1] = -1.0
    return g


def dense_dwf(U, M5, mf, Ls, t_bc):
    H = dense.dense_hop(U, t_bc)
    n4 = H.shape[0]
    V = n4 // 12
    g5 = gamma5_written()
    pp = np.kron(np.eye(V), np.kron((np.eye(4) + g5) / 2, np.eye(3)))
    pm = np.kron(np.eye(V), np.kron((np.eye(4) - g5) / 2, np.eye(3)))
    D = np.zeros((Ls * n4, Ls * n4), dtype=np.complex128)
    blk = (5.0 - M5) * np.eye(n4) - 0.5 * H
    for s in range(Ls):
        rs = slice(s * n4, (s + 1) * n4)
        D[rs, rs] += blk
        up = (s + 1) % Ls
        dn = (s - 1) % Ls
        D[rs, up * n4:(up + 1) * n4] -= (1.0 if s + 1 < Ls else -mf) * pm
        D[rs, dn * n4:(dn + 1) * n4] -= (1.0 if s > 0 else -mf) * pp
    return D


def vec5(psi):
    return np.concatenate([dense.to_vector(psi[s]) for s in range(psi.shape[0])])


def test_gamma5_entries():
    assert np.allclose(dirac.GAMMA5, gamma5_written())


@pytest.mark.parametrize("dims,Ls", [((2, 2, 2, 2), 4), ((2, 2, 2, 4), 3), ((4, 2, 2, 2), 1)])
@pytest.mark.parametrize("t_bc", [-1, 1])
def test_dense_brute_force(dims, Ls, t_bc):
    U = fg.gauge_field(dims, 91, "haar")
    op = dwf.DomainWall(U, 1.8, 0.07, Ls, t_bc)
    psi = field5(dims, Ls, 92)
    D = dense_dwf(U, 1.8, 0.07, Ls, t_bc)
    assert np.abs(vec5(op.D(psi)) - D @ vec5(psi)).max() <= 1e-13


def test_gamma5_hermiticity():
    dims, Ls = (4, 4, 2, 4), 5
    U = fg.gauge_field(dims, 93, "haar")
    op = dwf.DomainWall(U, 1.6, 0.1, Ls)
    a, b = field5(dims, Ls, 94), field5(dims, Ls, 95)

    def gamma5_R(v):
        return np.stack([dirac.spin_mul(dirac.GAMMA5, v[Ls - 1 - s]) for s in range(Ls)])

    # <a, D b> = <gamma5 R D R gamma5 a, b> for D^dag = gamma5 R D R gamma5
    lhs = np.vdot(a, op.D(b))
    rhs = np.vdot(gamma5_R(op.D(gamma5_R(a))), b)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_ls1_is_wilson():
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 96, "haar")
    M5, mf = 1.4, 0.2
    op = dwf.DomainWall(U, M5, mf, 1)
    psi = field5(dims, 1, 97)
    m = 5.0 - M5 + mf
    want = m * dirac.wilson(U, psi[0], 1.0 / (2 * m), -1)
    assert np.abs(op.D(psi)[0] - want).max() <= 1e-12


def test_gauge_covariance():
    dims, Ls = (4, 4, 4, 4), 4
    U = fg.gauge_field(dims, 98, "haar")
    G = fg.random_su3_field(dims, 99)
    psi = field5(dims, Ls, 100)
    op = dwf.DomainWall(U, 1.8, 0.05, Ls)
    opg = dwf.DomainWall(dirac.gauge_transform(U, G), 1.8, 0.05, Ls)
    gpsi = np.stack([dirac.transform_spinor(psi[s], G) for s in range(Ls)])
    want = np.stack([dirac.transform_spinor(v, G) for v in op.D(psi)])
    assert np.abs(opg.D(gpsi) - want).max() <= 1e-12


def test_adjoint_and_normal_solve_match_lapack():
    dims, Ls = (2, 2, 2, 4), 4
    U = fg.gauge_field(dims, 101, "smooth", 0.3)
    op = dwf.DomainWall(U, 1.8, 0.1, Ls)
    a, b = field5(dims, Ls, 102), field5(dims, Ls, 103)
    assert abs(np.vdot(a, op.D(b)) - np.vdot(op.Ddag(a), b)) <= 1e-12 * np.abs(a).sum()
    x, info = dwf.solve(op, b, tol=1e-12)
    assert info.converged
    want = np.linalg.solve(dense_dwf(U, 1.8, 0.1, Ls, -1), vec5(b))
    assert np.linalg.norm(vec5(x) - want) <= 1e-8 * np.linalg.norm(want)
    assert np.linalg.norm(vec5(b - op.D(x))) <= 1e-10 * np.linalg.norm(vec5(b))
