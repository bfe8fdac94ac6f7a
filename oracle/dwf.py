"""Domain-wall fermion operator (Shamir form) on the Wilson kernel.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain float64 NumPy.

The paper lists the domain-wall operator among Bridge++'s fermion kinds
(Sec. 2; it benchmarks its multiplication, Sec. 3) and prints no matrix
elements; the definition here is the textbook Shamir one, on the conventions
of ``oracle.dirac`` (the same hopping term H and Dirac-Pauli gammas), with a
fifth coordinate ``s = 0 .. Ls-1`` (fields indexed ``[s, t, z, y, x, spin,
colour]``):

    (D psi)_s = (5 - M5) psi_s - 1/2 H psi_s - P_- psi_{s+1} - P_+ psi_{s-1},

    P_+- = (1 +- gamma5) / 2,  psi_{Ls} -> -m_f psi_0,  psi_{-1} -> -m_f psi_{Ls-1},

i.e. the 4-d Wilson operator with mass -M5 on every slice plus the hops in s
with chiral projectors, closed by the quark mass m_f at the walls. D is not
positive definite (its Wilson kernel has mass -M5), so the solver is CG on
the normal equations.
"""

from __future__ import annotations

import numpy as np

from . import dirac, solvers

P_PLUS = (dirac.ONE4 + dirac.GAMMA5) / 2
P_MINUS = (dirac.ONE4 - dirac.GAMMA5) / 2


class DomainWall:
    def __init__(self, U: np.ndarray, M5: float, mf: float, Ls: int, t_bc: int = -1):
        if Ls < 1:
            raise ValueError("Ls must be >= 1")
        self.U = U
        self.M5 = float(M5)
        self.mf = float(mf)
        self.Ls = int(Ls)
        self.t_bc = int(t_bc)

    def D(self, psi: np.ndarray) -> np.ndarray:
        Ls = self.Ls
        out = np.empty_like(psi)
        for s in range(Ls):
            w = (5.0 - self.M5) * psi[s] - 0.5 * dirac.hop(self.U, psi[s], self.t_bc)
            up = psi[s + 1] if s + 1 < Ls else -self.mf * psi[0]
            dn = psi[s - 1] if s > 0 else -self.mf * psi[Ls - 1]
            out[s] = w - dirac.spin_mul(P_MINUS, up) - dirac.spin_mul(P_PLUS, dn)
        return out

    def Ddag(self, psi: np.ndarray) -> np.ndarray:
        """D^dagger written out: the adjoint of each term, with H^dagger taken
        term by term (oracle.dirac.Operator.hop_dag) and the s-hops' projectors
        exchanged (P_+- are Hermitian)."""
        Ls = self.Ls
        hd = dirac.Operator(self.U, 0.0, 0.0, self.t_bc)
        out = np.empty_like(psi)
        for s in range(Ls):
            w = (5.0 - self.M5) * psi[s] - 0.5 * hd.hop_dag(psi[s])
            up = psi[s + 1] if s + 1 < Ls else -self.mf * psi[0]
            dn = psi[s - 1] if s > 0 else -self.mf * psi[Ls - 1]
            out[s] = w - dirac.spin_mul(P_PLUS, up) - dirac.spin_mul(P_MINUS, dn)
        return out

    def normal(self, psi: np.ndarray) -> np.ndarray:
        return self.Ddag(self.D(psi))


def solve(op: DomainWall, b: np.ndarray, tol: float = 1e-10):
    """D x = b through the normal equations D^dag D x = D^dag b and CG."""
    return solvers.cg(op.normal, op.Ddag(b), tol=tol)
