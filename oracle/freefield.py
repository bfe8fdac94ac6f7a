"""Closed forms of the Wilson operator on unit links (the free field).

TEST INFRASTRUCTURE ONLY. For U = 1 a plane wave psi(x) = exp(i p.x) u is an
eigenvector of every hop, so

  D psi = Dt(p) psi,  Dt(p) = 1 - 2 kappa sum_mu cos p_mu + 2 i kappa sum_mu gamma_mu sin p_mu,

with p_j = 2 pi n_j / L_j in space and p_t = (2 n_t + 1) pi / L_t in time for
antiperiodic boundary conditions (2 pi n_t / L_t for periodic). Because the
gamma matrices anticommute, (sum gamma_mu s_mu)^2 = sum s_mu^2 and

  Dt(p)^-1 = [(1 - 2 kappa sum cos p) - 2 i kappa sum gamma_mu sin p_mu]
             / [(1 - 2 kappa sum cos p)^2 + 4 kappa^2 sum sin^2 p_mu].
"""

from __future__ import annotations

import numpy as np

from .dense import G


def momentum(dims, n, t_bc: int = -1):
    lx, ly, lz, lt = dims
    nx, ny, nz, nt = n
    pt = (2 * nt + (1 if t_bc == -1 else 0)) * np.pi / lt
    return np.array([2 * np.pi * nx / lx, 2 * np.pi * ny / ly, 2 * np.pi * nz / lz, pt])


def plane_wave(dims, p, u: np.ndarray) -> np.ndarray:
    """psi[t, z, y, x, s, a] = exp(i p.x) u[s, a]."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return phase[..., None, None] * u[None, None, None, None]


def symbol(p, kappa: float) -> np.ndarray:
    """Dt(p), a 4x4 spin matrix (colour is untouched)."""
    m = (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        m = m + 2j * kappa * np.sin(p[mu]) * G[mu]
    return m


def symbol_inverse(p, kappa: float) -> np.ndarray:
    a = 1 - 2 * kappa * np.sum(np.cos(p))
    den = a * a + 4 * kappa * kappa * np.sum(np.sin(p) ** 2)
    m = a * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        m = m - 2j * kappa * np.sin(p[mu]) * G[mu]
    return m / den
