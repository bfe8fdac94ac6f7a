"""Two-level aggregation multigrid preconditioner (the DD-alpha-AMG kind).

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain float64 NumPy.

The paper's headline solver (Sec. 3) is a two-level multigrid in the style of
DD-alpha-AMG: test vectors that approximate the low modes of D span, block by
block, the coarse space; the coarse operator is D restricted to it; the
preconditioner combines a coarse-grid correction, solved by BiCGStab, with SAP
smoothing, inside a flexible BiCGStab in double precision. The paper names
the pieces and prints no steps; the definitions here are the textbook ones:

* aggregates: blocks of extent ``adims`` (every lattice extent an even number,
  at least 2, of aggregates; every aggregate extent at least 2);
* chirality: in the Dirac-Pauli basis gamma5 mixes the upper (spins 0, 1) and
  lower (spins 2, 3) pairs, so a spinor is taken to the chiral basis
  ``c_+ = (u - l)/sqrt2``, ``c_- = (u + l)/sqrt2`` (a unitary change of basis;
  ``P_+- psi`` has only ``c_+-`` non-zero);
* test vectors ``v_1 .. v_n`` on the whole lattice; the prolongation P has one
  column per (aggregate a, chirality chi, k): the chiral part chi of ``v_k`` on
  the sites of a, the n columns of each (a, chi) orthonormalised in the order
  k = 1 .. n (the Q of a QR factorisation with a positive real diagonal in R);
  coarse index ``(a * 2 + chi) * n + k`` with chi = 0 for c_+, 1 for c_-;
* the coarse operator is ``D_c = P^dag D P``;
* setup: from given start vectors, ``n_iter`` times: one SAP-smoothing step
  of the homogeneous equation ``D v = 0``, ``v_k <- v_k - M_SAP D v_k``, for
  every k (it damps the modes SAP resolves and keeps the near-null space),
  then the aggregate-wise orthonormalisation (the test vectors become the
  orthonormalised basis);
* the two-level preconditioner: ``x = P D_c^-1 P^dag r`` with the coarse
  system solved by BiCGStab to a relative residual ``coarse_tol``, then one SAP
  post-smoothing ``x <- x + M_SAP (r - D x)``.
"""

from __future__ import annotations

import numpy as np

from . import sap, solvers

SQ2 = np.sqrt(2.0)


def to_chiral(psi: np.ndarray) -> np.ndarray:
    """[..., 4, 3] -> [..., 2 (chi), 2 (spin pair), 3]: (c_+, c_-)."""
    u, l = psi[..., 0:2, :], psi[..., 2:4, :]
    return np.stack([(u - l) / SQ2, (u + l) / SQ2], axis=-3)


def from_chiral(c: np.ndarray) -> np.ndarray:
    cp, cm = c[..., 0, :, :], c[..., 1, :, :]
    return np.concatenate([(cp + cm) / SQ2, (cm - cp) / SQ2], axis=-2)


class Aggregates:
    def __init__(self, dims, adims):
        self.dims = tuple(int(d) for d in dims)
        self.adims = tuple(int(b) for b in adims)
        for d, b in zip(self.dims, self.adims):
            if b < 2 or d % b != 0 or (d // b) % 2 != 0:
                raise ValueError("aggregate extents must be >= 2 and leave an even number of aggregates")
        self.blocks = sap.Blocks(self.dims, self.adims)
        self.count = self.blocks.count
        self.id = self.blocks.block_id  # [t, z, y, x]
        self.sites = [np.argwhere(self.id == a) for a in range(self.count)]  # (t, z, y, x) rows


class Prolongation:
    """P from test vectors v[k] (fields [t, z, y, x, 4, 3])."""

    def __init__(self, agg: Aggregates, vectors):
        self.agg = agg
        self.n = len(vectors)
        n = self.n
        ch = np.stack([to_chiral(v) for v in vectors])  # [k, t, z, y, x, chi, 2, 3]
        # basis[a][chi]: (sites * 6, n) orthonormal columns
        self.basis = []
        for a in range(agg.count):
            idx = tuple(agg.sites[a].T)
            per = []
            for chi in range(2):
                A = np.stack([ch[k][idx][:, chi].reshape(-1) for k in range(n)], axis=1)
                Q, R = np.linalg.qr(A)
                ph = np.diag(R) / np.abs(np.diag(R))
                per.append(Q * ph[None, :])  # R diagonal made positive real
            self.basis.append(per)

    @property
    def ncoarse(self) -> int:
        return self.agg.count * 2 * self.n

    def restrict(self, r: np.ndarray) -> np.ndarray:
        c = to_chiral(r)
        out = np.zeros(self.ncoarse, dtype=np.complex128)
        for a in range(self.agg.count):
            idx = tuple(self.agg.sites[a].T)
            for chi in range(2):
                vec = c[idx][:, chi].reshape(-1)
                o = (a * 2 + chi) * self.n
                out[o:o + self.n] = self.basis[a][chi].conj().T @ vec
        return out

    def prolong(self, e: np.ndarray) -> np.ndarray:
        lx, ly, lz, lt = self.agg.dims
        c = np.zeros((lt, lz, ly, lx, 2, 2, 3), dtype=np.complex128)
        for a in range(self.agg.count):
            idx = tuple(self.agg.sites[a].T)
            for chi in range(2):
                o = (a * 2 + chi) * self.n
                c[idx + (chi,)] = (self.basis[a][chi] @ e[o:o + self.n]).reshape(-1, 2, 3)
        return from_chiral(c)

    def vectors(self):
        """The orthonormalised test vectors: column k of every (a, chi)."""
        out = []
        for k in range(self.n):
            e = np.zeros(self.ncoarse, dtype=np.complex128)
            e[k::self.n] = 1.0
            out.append(self.prolong(e))
        return out


def coarse_operator(D, P: Prolongation) -> np.ndarray:
    """D_c = P^dag D P, column by column."""
    nc = P.ncoarse
    Dc = np.zeros((nc, nc), dtype=np.complex128)
    for j in range(nc):
        e = np.zeros(nc, dtype=np.complex128)
        e[j] = 1.0
        Dc[:, j] = P.restrict(D(P.prolong(e)))
    return Dc


def setup(D, agg: Aggregates, start, sap_blocks: sap.Blocks, n_iter: int, ncy: int, nmr: int) -> Prolongation:
    """Test vectors by n_iter rounds of SAP smoothing of D v = 0 and
    aggregate-wise orthonormalisation of the given start vectors."""
    v = [np.asarray(s, dtype=np.complex128) for s in start]
    P = Prolongation(agg, v)
    for _ in range(n_iter):
        v = [vk - sap.sap(D, sap_blocks, D(vk), ncy, nmr) for vk in v]
        P = Prolongation(agg, v)
        v = P.vectors()
    return P


class TwoLevel:
    """The preconditioner r -> x: coarse correction, then SAP post-smoothing."""

    def __init__(self, D, P: Prolongation, Dc: np.ndarray, sap_blocks: sap.Blocks, ncy: int, nmr: int,
                 coarse_tol: float = 0.05, coarse_max_iter: int = 200):
        self.D, self.P, self.Dc = D, P, Dc
        self.sap_blocks, self.ncy, self.nmr = sap_blocks, ncy, nmr
        self.coarse_tol, self.coarse_max_iter = coarse_tol, coarse_max_iter

    def coarse_solve(self, rc: np.ndarray) -> np.ndarray:
        e, _ = solvers.bicgstab(lambda v: self.Dc @ v, rc, tol=self.coarse_tol, max_iter=self.coarse_max_iter)
        return e

    def __call__(self, r: np.ndarray) -> np.ndarray:
        x = self.P.prolong(self.coarse_solve(self.P.restrict(r)))
        return x + sap.sap(self.D, self.sap_blocks, r - self.D(x), self.ncy, self.nmr)


def solve(D, b, pre: TwoLevel, tol: float = 1e-10, max_iter: int = 500):
    """D x = b by flexible BiCGStab with the two-level preconditioner."""
    return sap.fbicgstab(D, pre, b, tol=tol, max_iter=max_iter)
