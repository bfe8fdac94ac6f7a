"""The oracle's operators evaluated at a list of sites only.

TEST INFRASTRUCTURE ONLY. Used to check outputs on lattices too large for the
whole-field oracle (32^3 x 64 and up): each requested output site is computed
from the definitions in ``oracle.dirac`` by gathering exactly the links and
spinor values it depends on. Site lists are integer arrays of shape (N, 4)
holding (x, y, z, t).

Pinned against the whole-field oracle on small lattices (tests/
test_oracle_sampled.py).
"""

from __future__ import annotations

import numpy as np

from .dirac import GAMMA, ONE4, sigma


def _dims(U):
    lt, lz, ly, lx = U.shape[:4]
    return np.array([lx, ly, lz, lt])


def step(dims, sites, mu, s):
    out = np.array(sites, copy=True)
    out[:, mu] = (out[:, mu] + s) % dims[mu]
    return out


def gather(field, sites):
    return field[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def hop_at(U, psi_at, t_bc: int, sites):
    """(H psi)(x) at each listed x; ``psi_at(sites)`` returns psi there, (N, 4, 3)."""
    dims = _dims(U)
    sites = np.asarray(sites)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for mu in range(4):
        f = step(dims, sites, mu, +1)
        eta = np.ones(len(sites))
        if mu == 3:
            eta[sites[:, 3] == dims[3] - 1] = t_bc
        u = gather(U, sites)[:, mu]
        v = psi_at(f) @ np.swapaxes(u, -1, -2)
        out += eta[:, None, None] * ((ONE4 - GAMMA[mu]) @ v)
        b = step(dims, sites, mu, -1)
        eta = np.ones(len(sites))
        if mu == 3:
            eta[sites[:, 3] == 0] = t_bc
        ub = gather(U, b)[:, mu]
        v = psi_at(b) @ np.conj(ub)
        out += eta[:, None, None] * ((ONE4 + GAMMA[mu]) @ v)
    return out


def clover_at(U, kappa: float, csw: float, sites):
    """A(x) at each listed x, (N, 12, 12)."""
    dims = _dims(U)
    sites = np.asarray(sites)
    n = len(sites)
    a = np.broadcast_to(np.eye(12, dtype=np.complex128), (n, 12, 12)).copy()
    if csw == 0.0:
        return a
    for mu in range(4):
        for nu in range(mu + 1, 4):
            def link(d, da, db):
                s = sites
                if da:
                    s = step(dims, s, mu, da)
                if db:
                    s = step(dims, s, nu, db)
                return gather(U, s)[:, d]
            q = link(mu, 0, 0) @ link(nu, 1, 0) @ _dag(link(mu, 0, 1)) @ _dag(link(nu, 0, 0))
            q += link(nu, 0, 0) @ _dag(link(mu, -1, 1)) @ _dag(link(nu, -1, 0)) @ link(mu, -1, 0)
            q += _dag(link(mu, -1, 0)) @ _dag(link(nu, -1, -1)) @ link(mu, -1, -1) @ link(nu, 0, -1)
            q += _dag(link(nu, 0, -1)) @ link(mu, 0, -1) @ link(nu, 1, -1) @ _dag(link(mu, 0, 0))
            f = (q - _dag(q)) / 8j
            a += kappa * csw * np.einsum("st,nab->nsatb", sigma(mu, nu), f).reshape(n, 12, 12)
    return a


def site_mul(a, v):
    return (a @ v.reshape(len(v), 12, 1)).reshape(len(v), 4, 3)


def full_lookup(psi):
    return lambda s: gather(psi, s)


def dirac_at(U, psi, kappa, csw, t_bc, sites):
    """(D psi)(x) = A(x) psi(x) - kappa (H psi)(x)."""
    sites = np.asarray(sites)
    return site_mul(clover_at(U, kappa, csw, sites), gather(psi, sites)) \
        - kappa * hop_at(U, full_lookup(psi), t_bc, sites)


def _linear(dims, s):
    return s[:, 0] + dims[0] * (s[:, 1] + dims[1] * (s[:, 2] + dims[2] * s[:, 3]))


def schur_at(U, x_even, kappa, csw, t_bc, sites, x_at=None):
    """(S x)(x) = A(x) x(x) - kappa^2 (H A_oo^-1 H x)(x) at even sites x, for a
    field x supported on even sites: S = D_ee - D_eo D_oo^-1 D_oe. x is the
    whole field x_even, or (x_at given) a function returning x at listed sites."""
    if x_at is None:
        x_at = full_lookup(x_even)
    dims = _dims(U)
    sites = np.asarray(sites)
    nbr = np.concatenate([step(dims, sites, mu, s) for mu in range(4) for s in (+1, -1)])
    lin = _linear(dims, nbr)
    uniq, first = np.unique(lin, return_index=True)
    odd_sites = nbr[first]
    y = hop_at(U, x_at, t_bc, odd_sites)
    y = site_mul(np.linalg.inv(clover_at(U, kappa, csw, odd_sites)), y)

    def y_at(s):
        return y[np.searchsorted(uniq, _linear(dims, s))]

    return site_mul(clover_at(U, kappa, csw, sites), x_at(sites)) \
        - kappa * kappa * hop_at(U, y_at, t_bc, sites)


def random_sites(dims, n: int, seed: int, parity=None):
    """n distinct-ish random sites (x, y, z, t), optionally of one parity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.stack([rng.integers(0, d, n) for d in dims], axis=1)
    if parity is not None:
        bad = (s.sum(axis=1) % 2) != parity
        s[bad, 0] = (s[bad, 0] + 1) % dims[0]
    return s
