"""Domain-wall fermion operator (Moebius form, Shamir as its special case)
on the Wilson kernel.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain float64 NumPy.

The paper lists the Moebius domain-wall operator among Bridge++'s fermion
kinds (Sec. 2; it benchmarks its multiplication and a CG solve, Sec. 3) and
prints no matrix elements; the definition here is the textbook Moebius one, on
the conventions of ``oracle.dirac`` (the same hopping term H and Dirac-Pauli
gammas), with a fifth coordinate ``s = 0 .. Ls-1`` (fields indexed
``[s, t, z, y, x, spin, colour]``):

    D = D_W (b5 + c5 S) + (1 - S),    D_W = (4 - M5) - 1/2 H  (per slice),

    (S psi)_s = P_- psi_{s+1} + P_+ psi_{s-1},   P_+- = (1 +- gamma5) / 2,
    psi_{Ls} -> -m_f psi_0,  psi_{-1} -> -m_f psi_{Ls-1},

i.e. D_W is the 4-d Wilson operator with mass -M5 on every slice, applied to
(b5 + c5 S) psi. b5 = 1, c5 = 0 gives the Shamir operator
(5 - M5) psi_s - 1/2 H psi_s - (S psi)_s. D is not positive definite (its
Wilson kernel has mass -M5), so the solver is CG on the normal equations.

The paper implements the even-odd forms of every operator (Sec. 2, Eq. (1));
``EvenOdd`` is the even-odd Schur complement of D over the 4-d parity of the
sites, with its adjoint and solve.
"""

from __future__ import annotations

import numpy as np

from . import dirac, solvers

P_PLUS = (dirac.ONE4 + dirac.GAMMA5) / 2
P_MINUS = (dirac.ONE4 - dirac.GAMMA5) / 2


class DomainWall:
    def __init__(self, U: np.ndarray, M5: float, mf: float, Ls: int, t_bc: int = -1, b5: float = 1.0,
                 c5: float = 0.0):
        if Ls < 1:
            raise ValueError("Ls must be >= 1")
        self.U = U
        self.M5 = float(M5)
        self.mf = float(mf)
        self.Ls = int(Ls)
        self.t_bc = int(t_bc)
        self.b5 = float(b5)
        self.c5 = float(c5)
        self._hd = dirac.Operator(U, 0.0, 0.0, self.t_bc)

    def _neighbours(self, psi, s):
        """psi_{s+1} and psi_{s-1} with the walls' -m_f."""
        Ls = self.Ls
        up = psi[s + 1] if s + 1 < Ls else -self.mf * psi[0]
        dn = psi[s - 1] if s > 0 else -self.mf * psi[Ls - 1]
        return up, dn

    def S(self, psi):
        out = np.empty_like(psi)
        for s in range(self.Ls):
            up, dn = self._neighbours(psi, s)
            out[s] = dirac.spin_mul(P_MINUS, up) + dirac.spin_mul(P_PLUS, dn)
        return out

    def Sdag(self, psi):
        """The adjoint of S: the projectors exchanged (P_+- are Hermitian and
        m_f is real)."""
        out = np.empty_like(psi)
        for s in range(self.Ls):
            up, dn = self._neighbours(psi, s)
            out[s] = dirac.spin_mul(P_PLUS, up) + dirac.spin_mul(P_MINUS, dn)
        return out

    def DW(self, psi):
        return np.stack([(4.0 - self.M5) * v - 0.5 * dirac.hop(self.U, v, self.t_bc) for v in psi])

    def DWdag(self, psi):
        """D_W^dagger, with H^dagger taken term by term (Operator.hop_dag)."""
        return np.stack([(4.0 - self.M5) * v - 0.5 * self._hd.hop_dag(v) for v in psi])

    def D(self, psi: np.ndarray) -> np.ndarray:
        return self.DW(self.b5 * psi + self.c5 * self.S(psi)) + psi - self.S(psi)

    def Ddag(self, psi: np.ndarray) -> np.ndarray:
        """D^dagger = (b5 + c5 S^dag) D_W^dagger + (1 - S^dag)."""
        u = self.DWdag(psi)
        return self.b5 * u + self.c5 * self.Sdag(u) + psi - self.Sdag(psi)

    def normal(self, psi: np.ndarray) -> np.ndarray:
        return self.Ddag(self.D(psi))


def solve(op: DomainWall, b: np.ndarray, tol: float = 1e-10):
    """D x = b through the normal equations D^dag D x = D^dag b and CG."""
    return solvers.cg(op.normal, op.Ddag(b), tol=tol)


# ---------------------------------------------------------------- even-odd form
# With the 4-d parity of the sites (s does not enter it), D splits into the
# site-local part M5op = (4 - M5)(b5 + c5 S) + 1 - S, which acts on s and spin
# only, and the hopping part Dhop = -1/2 H (b5 + c5 S), which couples the two
# parities. The even-odd Schur complement on the even sites is
#   S_ee = M5op - Dhop_eo M5op^-1 Dhop_oe,
# D x = b is S_ee x_e = b_e - Dhop_eo M5op^-1 b_o, x_o = M5op^-1 (b_o - Dhop_oe x_e).

def parity5(op: DomainWall, psi: np.ndarray, parity: int) -> np.ndarray:
    par = dirac.parity_field(dirac.dims_of(op.U))[None, ..., None, None]
    return np.where(par == parity, psi, 0)


def m5op(op: DomainWall, psi):
    return (4.0 - op.M5) * (op.b5 * psi + op.c5 * op.S(psi)) + psi - op.S(psi)


def m5op_dag(op: DomainWall, psi):
    return (4.0 - op.M5) * (op.b5 * psi + op.c5 * op.Sdag(psi)) + psi - op.Sdag(psi)


def dhop(op: DomainWall, psi):
    return np.stack([-0.5 * dirac.hop(op.U, v, op.t_bc) for v in op.b5 * psi + op.c5 * op.S(psi)])


def dhop_dag(op: DomainWall, psi):
    h = np.stack([-0.5 * op._hd.hop_dag(v) for v in psi])
    return op.b5 * h + op.c5 * op.Sdag(h)


def local_matrix(op: DomainWall, fn) -> np.ndarray:
    """The (Ls 4) x (Ls 4) matrix over (s, spin) of a site-local map fn (the
    same at every site and colour), from its action on unit vectors."""
    Ls = op.Ls
    cols = []
    for s in range(Ls):
        for a in range(4):
            e = np.zeros((Ls, 1, 1, 1, 1, 4, 3), dtype=np.complex128)
            e[s, 0, 0, 0, 0, a, 0] = 1.0
            cols.append(fn(e)[:, 0, 0, 0, 0, :, 0].reshape(-1))
    return np.array(cols).T


def apply_local(K: np.ndarray, psi: np.ndarray) -> np.ndarray:
    Ls = psi.shape[0]
    Kr = K.reshape(Ls, 4, Ls, 4)
    return np.einsum("sarb,rtzyxbc->stzyxac", Kr, psi)


class EvenOdd:
    def __init__(self, op: DomainWall):
        self.op = op
        # M5op does not involve the links: its matrix is built on one site
        self.Kinv = np.linalg.inv(local_matrix(op, lambda e: m5op(op, e)))

    def m5inv(self, psi):
        return apply_local(self.Kinv, psi)

    def m5inv_dag(self, psi):
        return apply_local(self.Kinv.conj().T, psi)

    def schur(self, xe):
        op = self.op
        xe = parity5(op, xe, 0)
        t = parity5(op, dhop(op, xe), 1)
        t = parity5(op, dhop(op, self.m5inv(t)), 0)
        return m5op(op, xe) - t

    def schur_dag(self, xe):
        op = self.op
        xe = parity5(op, xe, 0)
        t = parity5(op, dhop_dag(op, xe), 1)
        t = parity5(op, dhop_dag(op, self.m5inv_dag(t)), 0)
        return m5op_dag(op, xe) - t

    def solve(self, b, tol: float = 1e-10):
        """D x = b through the even-odd Schur complement and CG on its normal
        equations, then the odd sites."""
        op = self.op
        be, bo = parity5(op, b, 0), parity5(op, b, 1)
        bp = be - parity5(op, dhop(op, self.m5inv(bo)), 0)
        xe, info = solvers.cg(lambda v: self.schur_dag(self.schur(v)), self.schur_dag(bp), tol=0.1 * tol)
        xo = self.m5inv(bo - parity5(op, dhop(op, xe), 1))
        return parity5(op, xe, 0) + parity5(op, xo, 1), info
