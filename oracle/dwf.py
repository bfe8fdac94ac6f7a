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
