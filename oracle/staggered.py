"""Staggered fermion operator, its even-odd form and CG.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain float64 NumPy.

The paper lists the staggered operator among Bridge++'s fermion kinds
(Sec. 2) and prints no matrix elements; the definitions here are the
textbook (Kogut-Susskind) ones, with the conventions of ``oracle.dirac``
(fields indexed ``[t, z, y, x, ...]``, direction ``mu = 0..3 = x, y, z, t``,
parity ``(x + y + z + t) mod 2``, fermion boundary factor ``t_bc`` on hops
that cross the t boundary):

* one colour vector (3 complex) per site;
* staggered phases ``eta_x = 1``, ``eta_y = (-1)^x``, ``eta_z = (-1)^(x+y)``,
  ``eta_t = (-1)^(x+y+z)``;
* ``D = m + H`` with the hopping term

      (H psi)(x) = 1/2 sum_mu eta_mu(x) [ U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu) ]

  (each cross-boundary t hop times ``t_bc``); ``H`` is anti-Hermitian;
* even-odd: ``H`` couples opposite parities, so on the even sites
  ``(m^2 - H_eo H_oe) x_e = m b_e - H_eo b_o`` with ``m^2 - H_eo H_oe =
  m^2 + H_eo H_eo^dag`` Hermitian positive definite, solved by CG, and
  ``x_o = (b_o - H_oe x_e) / m``.
"""

from __future__ import annotations

import numpy as np

from . import dirac, solvers


def phases(dims) -> np.ndarray:
    """eta[t, z, y, x, mu] = +-1."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    eta = np.empty((lt, lz, ly, lx, 4))
    eta[..., 0] = 1.0
    eta[..., 1] = (-1.0) ** x
    eta[..., 2] = (-1.0) ** (x + y)
    eta[..., 3] = (-1.0) ** (x + y + z)
    return eta


def hop(U: np.ndarray, psi: np.ndarray, t_bc: int) -> np.ndarray:
    """H psi for a colour-vector field psi[t, z, y, x, c]."""
    dims = dirac.dims_of(U)
    eta = phases(dims)
    out = np.zeros_like(psi)
    for mu in range(4):
        u = U[..., mu, :, :]
        fwd = np.einsum("...ab,...b->...a", u, dirac.shift(psi, mu, +1))
        fwd *= dirac.boundary_factor(dims, mu, +1, t_bc)[..., None]
        ub = dirac.shift(u, mu, -1)
        bwd = np.einsum("...ba,...b->...a", np.conj(ub), dirac.shift(psi, mu, -1))
        bwd *= dirac.boundary_factor(dims, mu, -1, t_bc)[..., None]
        out += 0.5 * eta[..., mu, None] * (fwd - bwd)
    return out


class Staggered:
    def __init__(self, U: np.ndarray, mass: float, t_bc: int = -1):
        self.U = U
        self.mass = float(mass)
        self.t_bc = int(t_bc)
        self.dims = dirac.dims_of(U)
        self.par = dirac.parity_field(self.dims)[..., None]

    def hop(self, psi):
        return hop(self.U, psi, self.t_bc)

    def D(self, psi):
        return self.mass * psi + self.hop(psi)

    def mask(self, psi, parity):
        return np.where(self.par == parity, psi, 0)

    def hop_pq(self, p, q, psi):
        """P_p H P_q psi."""
        return self.mask(self.hop(self.mask(psi, q)), p)

    def schur(self, xe):
        """(m^2 - H_eo H_oe) on even sites."""
        return self.mass ** 2 * self.mask(xe, 0) - self.hop_pq(0, 1, self.hop_pq(1, 0, xe))

    def eo_source(self, b):
        return self.mass * self.mask(b, 0) - self.hop_pq(0, 1, b)

    def eo_reconstruct(self, xe, b):
        return self.mask(xe, 0) + (self.mask(b, 1) - self.hop_pq(1, 0, xe)) / self.mass


def solve(op: Staggered, b: np.ndarray, tol: float = 1e-10):
    """D x = b through the even-odd normal system and CG."""
    be = op.eo_source(b)
    xe, info = solvers.cg(op.schur, be, tol=tol * 0.1)
    return op.eo_reconstruct(xe, b), info
