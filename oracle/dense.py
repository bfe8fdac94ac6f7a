"""Brute-force dense matrix of the Wilson/clover operator on tiny lattices.

TEST INFRASTRUCTURE ONLY. This is an independent construction used to pin
the whole-field oracle: it walks every site and every direction with explicit
coordinate arithmetic and writes each 12x12 block D(x, y) of the 12V x 12V
matrix (row/column index ``12 * site + 3 * spin + colour``, site index
``x + Lx (y + Ly (z + Lz t))``). It shares no helper with ``oracle.dirac``
beyond the gamma matrices, which are written out again here.

Definition (Sec. 2 of the paper names the operator; the entries are the
textbook ones): D = A - kappa H with

  H(x, x+mu) += eta (1 - gamma_mu) (x) U_mu(x),
  H(x, x-mu) += eta (1 + gamma_mu) (x) U_mu(x-mu)^dag,

the blocks of both terms added when x+mu and x-mu coincide (extent 2).
"""

from __future__ import annotations

import numpy as np


def _gammas():
    i = 1j
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    # gamma_x, gamma_y, gamma_z in the Dirac-Pauli basis, written entry by entry
    g[0][0, 3] = -i; g[0][1, 2] = -i; g[0][2, 1] = i; g[0][3, 0] = i
    g[1][0, 3] = -1; g[1][1, 2] = 1; g[1][2, 1] = 1; g[1][3, 0] = -1
    g[2][0, 2] = -i; g[2][1, 3] = i; g[2][2, 0] = i; g[2][3, 1] = -i
    g[3][0, 0] = 1; g[3][1, 1] = 1; g[3][2, 2] = -1; g[3][3, 3] = -1
    return g


G = _gammas()


def site_index(dims, x, y, z, t):
    lx, ly, lz, lt = dims
    return x + lx * (y + ly * (z + lz * t))


def coords(dims):
    lx, ly, lz, lt = dims
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    yield x, y, z, t


def _link(U, c, mu):
    x, y, z, t = c
    return U[t, z, y, x, mu]


def _step(dims, c, mu, s):
    c = list(c)
    c[mu] = (c[mu] + s) % dims[mu]
    return tuple(c)


def dense_hop(U, t_bc: int) -> np.ndarray:
    lt, lz, ly, lx = U.shape[:4]
    dims = (lx, ly, lz, lt)
    n = 12 * lx * ly * lz * lt
    h = np.zeros((n, n), dtype=np.complex128)
    one = np.eye(4)
    for c in coords(dims):
        i = site_index(dims, *c)
        for mu in range(4):
            f = _step(dims, c, mu, +1)
            eta = t_bc if (mu == 3 and c[3] == dims[3] - 1) else 1
            blk = eta * np.kron(one - G[mu], _link(U, c, mu))
            j = site_index(dims, *f)
            h[12 * i:12 * i + 12, 12 * j:12 * j + 12] += blk
            b = _step(dims, c, mu, -1)
            eta = t_bc if (mu == 3 and c[3] == 0) else 1
            blk = eta * np.kron(one + G[mu], np.conj(_link(U, b, mu)).T)
            j = site_index(dims, *b)
            h[12 * i:12 * i + 12, 12 * j:12 * j + 12] += blk
    return h


def _leaf_sum(U, dims, c, mu, nu):
    """Clover leaves at c, each walked link by link around its plaquette."""

    def walk(path):
        # path: list of (direction, +1 | -1) steps starting at c
        m = np.eye(3, dtype=np.complex128)
        pos = c
        for d, s in path:
            if s > 0:
                m = m @ _link(U, pos, d)
                pos = _step(dims, pos, d, +1)
            else:
                pos = _step(dims, pos, d, -1)
                m = m @ np.conj(_link(U, pos, d)).T
        assert pos == c
        return m

    return (walk([(mu, 1), (nu, 1), (mu, -1), (nu, -1)])
            + walk([(nu, 1), (mu, -1), (nu, -1), (mu, 1)])
            + walk([(mu, -1), (nu, -1), (mu, 1), (nu, 1)])
            + walk([(nu, -1), (mu, 1), (nu, 1), (mu, -1)]))


def dense_clover(U, kappa: float, csw: float) -> np.ndarray:
    lt, lz, ly, lx = U.shape[:4]
    dims = (lx, ly, lz, lt)
    n = 12 * lx * ly * lz * lt
    a = np.eye(n, dtype=np.complex128)
    if csw == 0.0:
        return a
    for c in coords(dims):
        i = site_index(dims, *c)
        blk = np.zeros((12, 12), dtype=np.complex128)
        for mu in range(4):
            for nu in range(mu + 1, 4):
                q = _leaf_sum(U, dims, c, mu, nu)
                f = (q - np.conj(q).T) / 8j
                sig = (G[mu] @ G[nu] - G[nu] @ G[mu]) / 2j
                blk += np.kron(sig, f)
        a[12 * i:12 * i + 12, 12 * i:12 * i + 12] += kappa * csw * blk
    return a


def dense_dirac(U, kappa: float, csw: float = 0.0, t_bc: int = -1) -> np.ndarray:
    return dense_clover(U, kappa, csw) - kappa * dense_hop(U, t_bc)


def to_vector(psi: np.ndarray) -> np.ndarray:
    """[t, z, y, x, spin, colour] -> the dense index order (identical C order)."""
    return psi.reshape(-1)
