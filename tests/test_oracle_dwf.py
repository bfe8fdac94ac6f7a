"""Pins of the domain-wall oracle (oracle/dwf.py) against facts fixed
independently of it: a dense 5-d matrix assembled from the brute-force dense
4-d hopping matrix (oracle/dense.py) and explicit chiral projectors written
from gamma5's entries; the textbook effective 4-d operator of a finite-Ls
domain-wall operator, (1 + m_f)/2 + (1 - m_f)/2 gamma5 tanh(Ls artanh H_M)
with the Moebius kernel H_M = gamma5 (b5 + c5) D_W (2 + (b5 - c5) D_W)^-1
(exact at every Ls, computed here with dense inverses and matrix powers);
Gamma5-hermiticity of the Shamir case (D^dag = gamma5 R D R gamma5 with R the
reflection s -> Ls-1-s); the Ls = 1 reduction to a Wilson operator; gauge
covariance; the adjoint; and the CG solve of the normal equations against
LAPACK."""

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


def dense_parts(U, M5, t_bc):
    """Dense 4-d D_W = (4 - M5) - H/2, gamma5 and the chiral projectors over
    the lattice, from the brute-force hopping matrix and gamma5's entries."""
    H = dense.dense_hop(U, t_bc)
    n4 = H.shape[0]
    V = n4 // 12
    g5 = gamma5_written()
    G5 = np.kron(np.eye(V), np.kron(g5, np.eye(3)))
    pp = np.kron(np.eye(V), np.kron((np.eye(4) + g5) / 2, np.eye(3)))
    pm = np.kron(np.eye(V), np.kron((np.eye(4) - g5) / 2, np.eye(3)))
    return (4.0 - M5) * np.eye(n4) - 0.5 * H, G5, pp, pm


def dense_dwf(U, M5, mf, Ls, t_bc, b5=1.0, c5=0.0):
    """Block by block: diagonal blocks b5 D_W + 1, the s+1 block
    (c5 D_W - 1) P_- and the s-1 block (c5 D_W - 1) P_+, the wall blocks
    times -m_f."""
    DW, _, pp, pm = dense_parts(U, M5, t_bc)
    n4 = DW.shape[0]
    D = np.zeros((Ls * n4, Ls * n4), dtype=np.complex128)
    off = c5 * DW - np.eye(n4)
    for s in range(Ls):
        rs = slice(s * n4, (s + 1) * n4)
        D[rs, rs] += b5 * DW + np.eye(n4)
        up = (s + 1) % Ls
        dn = (s - 1) % Ls
        D[rs, up * n4:(up + 1) * n4] += (1.0 if s + 1 < Ls else -mf) * off @ pm
        D[rs, dn * n4:(dn + 1) * n4] += (1.0 if s > 0 else -mf) * off @ pp
    return D


def vec5(psi):
    return np.concatenate([dense.to_vector(psi[s]) for s in range(psi.shape[0])])


def test_gamma5_entries():
    assert np.allclose(dirac.GAMMA5, gamma5_written())


@pytest.mark.parametrize("dims,Ls", [((2, 2, 2, 2), 4), ((2, 2, 2, 4), 3), ((4, 2, 2, 2), 1)])
@pytest.mark.parametrize("t_bc", [-1, 1])
@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_dense_brute_force(dims, Ls, t_bc, b5, c5):
    U = fg.gauge_field(dims, 91, "haar")
    op = dwf.DomainWall(U, 1.8, 0.07, Ls, t_bc, b5, c5)
    psi = field5(dims, Ls, 92)
    D = dense_dwf(U, 1.8, 0.07, Ls, t_bc, b5, c5)
    assert np.abs(vec5(op.D(psi)) - D @ vec5(psi)).max() <= 1e-13
    assert np.abs(vec5(op.Ddag(psi)) - D.conj().T @ vec5(psi)).max() <= 1e-13


def dense_of(apply, dims, Ls):
    """The matrix of a linear map on 5-d fields, column by column."""
    n = Ls * int(np.prod(dims)) * 12
    lx, ly, lz, lt = dims
    cols = []
    for k in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[k] = 1.0
        cols.append(vec5(apply(e.reshape(Ls, lt, lz, ly, lx, 4, 3))))
    return np.array(cols).T


def effective_4d(D, D1, n4, Ls, pp, pm):
    """[P^-1 D(1)^-1 D(m_f) P] restricted to the s = 0 block, with
    P = P_- delta_{s,s'} + P_+ delta_{s+1,s'} (s + 1 mod Ls)."""
    P = np.zeros((Ls * n4, Ls * n4), dtype=np.complex128)
    for s in range(Ls):
        P[s * n4:(s + 1) * n4, s * n4:(s + 1) * n4] += pm
        sp = (s + 1) % Ls
        P[s * n4:(s + 1) * n4, sp * n4:(sp + 1) * n4] += pp
    return (np.linalg.solve(P, np.linalg.solve(D1, D @ P)))[:n4, :n4]


def polar_approx(DW, G5, mf, Ls, b5, c5):
    n4 = DW.shape[0]
    I = np.eye(n4)
    Hm = G5 @ ((b5 + c5) * DW) @ np.linalg.inv(2 * I + (b5 - c5) * DW)
    A = np.linalg.matrix_power(I + Hm, Ls)
    B = np.linalg.matrix_power(I - Hm, Ls)
    return (1 + mf) / 2 * I + (1 - mf) / 2 * G5 @ (A - B) @ np.linalg.inv(A + B)


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5), (2.0, 1.0)])
def test_effective_operator_is_polar_approximation(b5, c5):
    dims, Ls, M5, mf = (2, 2, 2, 2), 5, 1.8, 0.07
    U = fg.gauge_field(dims, 104, "haar")
    DW, G5, pp, pm = dense_parts(U, M5, -1)
    n4 = DW.shape[0]
    D = dense_of(dwf.DomainWall(U, M5, mf, Ls, -1, b5, c5).D, dims, Ls)
    D1 = dense_of(dwf.DomainWall(U, M5, 1.0, Ls, -1, b5, c5).D, dims, Ls)
    got = effective_4d(D, D1, n4, Ls, pp, pm)
    assert np.abs(got - polar_approx(DW, G5, mf, Ls, b5, c5)).max() <= 1e-11


def test_effective_operator_catches_wrong_order():
    """A planted mistake in the oracle (c5 S applied after D_W instead of
    before) fails the effective-operator pin."""

    class Swapped(dwf.DomainWall):
        def D(self, psi):
            return self.b5 * self.DW(psi) + self.c5 * self.S(self.DW(psi)) + psi - self.S(psi)

    dims, Ls, M5, mf, b5, c5 = (2, 2, 2, 2), 5, 1.8, 0.07, 1.5, 0.5
    U = fg.gauge_field(dims, 104, "haar")
    DW, G5, pp, pm = dense_parts(U, M5, -1)
    D = dense_of(Swapped(U, M5, mf, Ls, -1, b5, c5).D, dims, Ls)
    D1 = dense_of(Swapped(U, M5, 1.0, Ls, -1, b5, c5).D, dims, Ls)
    got = effective_4d(D, D1, DW.shape[0], Ls, pp, pm)
    assert np.abs(got - polar_approx(DW, G5, mf, Ls, b5, c5)).max() > 1e-3


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


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.7, 0.6)])
def test_ls1_is_wilson(b5, c5):
    """At Ls = 1, S = -m_f, so D = (b5 - c5 m_f) D_W + 1 + m_f: a Wilson
    operator A (1 - kappa H) with A = (b5 - c5 m_f)(4 - M5) + 1 + m_f and
    kappa = (b5 - c5 m_f) / (2 A)."""
    dims = (4, 4, 4, 4)
    U = fg.gauge_field(dims, 96, "haar")
    M5, mf = 1.4, 0.2
    op = dwf.DomainWall(U, M5, mf, 1, -1, b5, c5)
    psi = field5(dims, 1, 97)
    B = b5 - c5 * mf
    A = B * (4.0 - M5) + 1.0 + mf
    want = A * dirac.wilson(U, psi[0], B / (2 * A), -1)
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


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_adjoint_and_normal_solve_match_lapack(b5, c5):
    dims, Ls = (2, 2, 2, 4), 4
    U = fg.gauge_field(dims, 101, "smooth", 0.3)
    op = dwf.DomainWall(U, 1.8, 0.1, Ls, -1, b5, c5)
    a, b = field5(dims, Ls, 102), field5(dims, Ls, 103)
    assert abs(np.vdot(a, op.D(b)) - np.vdot(op.Ddag(a), b)) <= 1e-12 * np.abs(a).sum()
    x, info = dwf.solve(op, b, tol=1e-12)
    assert info.converged
    want = np.linalg.solve(dense_dwf(U, 1.8, 0.1, Ls, -1, b5, c5), vec5(b))
    assert np.linalg.norm(vec5(x) - want) <= 1e-8 * np.linalg.norm(want)
    assert np.linalg.norm(vec5(b - op.D(x))) <= 1e-10 * np.linalg.norm(vec5(b))


def parity_index(dims, Ls, parity):
    """vec5 indices of the components on 4-d sites of one parity."""
    par = dirac.parity_field(dims)  # [t, z, y, x]
    per_site = np.repeat((par == parity).reshape(-1), 12)
    n4 = per_site.size
    return np.concatenate([s * n4 + np.nonzero(per_site)[0] for s in range(Ls)])


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_even_odd_schur_is_dense_schur_complement(b5, c5):
    dims, Ls = (2, 2, 2, 4), 4
    U = fg.gauge_field(dims, 105, "haar")
    op = dwf.DomainWall(U, 1.8, 0.07, Ls, -1, b5, c5)
    eo = dwf.EvenOdd(op)
    D = dense_dwf(U, 1.8, 0.07, Ls, -1, b5, c5)
    e, o = parity_index(dims, Ls, 0), parity_index(dims, Ls, 1)
    S = D[np.ix_(e, e)] - D[np.ix_(e, o)] @ np.linalg.solve(D[np.ix_(o, o)], D[np.ix_(o, e)])
    psi = dwf.parity5(op, field5(dims, Ls, 106), 0)
    got = vec5(eo.schur(psi))
    assert np.abs(got[e] - S @ vec5(psi)[e]).max() <= 1e-12
    assert np.abs(got[o]).max() == 0.0
    got = vec5(eo.schur_dag(psi))
    assert np.abs(got[e] - S.conj().T @ vec5(psi)[e]).max() <= 1e-12


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
def test_even_odd_solve_matches_lapack(b5, c5):
    dims, Ls = (2, 2, 2, 4), 4
    U = fg.gauge_field(dims, 107, "smooth", 0.3)
    op = dwf.DomainWall(U, 1.8, 0.1, Ls, -1, b5, c5)
    b = field5(dims, Ls, 108)
    x, info = dwf.EvenOdd(op).solve(b, tol=1e-12)
    assert info.converged
    want = np.linalg.solve(dense_dwf(U, 1.8, 0.1, Ls, -1, b5, c5), vec5(b))
    assert np.linalg.norm(vec5(x) - want) <= 1e-9 * np.linalg.norm(want)
