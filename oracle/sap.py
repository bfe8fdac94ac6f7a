"""Schwarz alternating procedure (SAP) preconditioner and flexible BiCGStab.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain float64 NumPy.

The paper's multigrid solver (Sec. 3) smooths with the Schwarz alternating
procedure: the lattice is cut into rectangular blocks, the blocks are coloured
like a checkerboard, and the Dirac equation restricted to each block (with
the hops that leave the block removed) is solved approximately by a fixed
number of iterations (Jacobi in QWS, a minimal-residual method in Bridge++),
the two colours one after the other; the outer solver is a flexible
BiCGStab. The paper prints none of these steps; the definitions here are the
textbook ones:

* blocks of extent ``bdims`` starting at multiples of ``bdims``; the colour of
  a block is the parity of the sum of its block coordinates; every lattice
  extent must hold an even number (at least 2) of blocks, so that two blocks
  of one colour never share a face and the blocks of one colour decouple;
* the block operator of a set of blocks ``P`` is ``P D P`` (Dirichlet: no hop
  enters or leaves a block), ``P`` the projector on the sites of the set;
* the block solve is the minimal-residual iteration ``q = D_B r``,
  ``alpha_B = <q, r> / <q, q>``, ``delta += alpha_B r``, ``r -= alpha_B q``, run
  ``n_mr`` times from ``delta = 0``, ``r = rho``, with one ``alpha`` per block;
* one SAP cycle updates the blocks of colour 0 and then those of colour 1;
  the update of colour ``c`` solves the block equations with right-hand side
  the current residual ``P_c (eta - D psi)`` and adds the block solutions to
  ``psi``; the preconditioner ``M eta`` runs ``ncy`` cycles from ``psi = 0``;
* even-odd block solves (``sap_eo``): the block equation ``D_B delta = rho``
  splits by site parity like the whole-lattice operator (Eq. (1)),
  ``D_B = [[A_ee, -kappa H_eo], [-kappa H_oe, A_oo]]`` with ``H`` the hops
  inside the block; the minimal-residual steps run on the block's Schur
  complement ``S_B = A_ee - kappa^2 H_eo A_oo^-1 H_oe`` with right-hand side
  ``rho_e + kappa H_eo A_oo^-1 rho_o`` (one ``alpha`` per block), and the odd
  sites follow as ``delta_o = A_oo^-1 (rho_o + kappa H_oe delta_e)``: the
  block LU solve of ``D_B`` with the even block solved approximately;
* flexible BiCGStab: BiCGStab for ``D x = b`` with right preconditioning by a
  possibly varying ``M`` (the preconditioned vectors ``M p`` and ``M s`` are
  used directly in the solution update, so no fixed ``M`` is assumed).
"""

from __future__ import annotations

from typing import Callable, Optional

import numpy as np

from . import dirac, solvers


class Blocks:
    """Block decomposition of a lattice ``dims = (Lx, Ly, Lz, Lt)``."""

    def __init__(self, dims, bdims):
        self.dims = tuple(int(d) for d in dims)
        self.bdims = tuple(int(b) for b in bdims)
        nb = []
        for d, b in zip(self.dims, self.bdims):
            if b < 1 or d % b != 0 or (d // b) % 2 != 0:
                raise ValueError("every extent must hold an even number of blocks")
            nb.append(d // b)
        self.nblocks = tuple(nb)
        lx, ly, lz, lt = self.dims
        t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
        bx, by, bz, bt = x // self.bdims[0], y // self.bdims[1], z // self.bdims[2], t // self.bdims[3]
        nbx, nby, nbz, _ = self.nblocks
        # block id of every site, array indexed [t, z, y, x]
        self.block_id = bx + nbx * (by + nby * (bz + nbz * bt))
        self.colour = (bx + by + bz + bt) % 2
        self.count = int(np.prod(self.nblocks))

    def mask(self, colour: int) -> np.ndarray:
        return (self.colour == colour)[..., None, None]


def block_apply(D: Callable[[np.ndarray], np.ndarray], blocks: Blocks, colour: int, psi: np.ndarray) -> np.ndarray:
    """P_c D P_c psi: the Dirichlet block operator on every block of one colour."""
    m = blocks.mask(colour)
    return np.where(m, D(np.where(m, psi, 0)), 0)


def _per_block_sum(blocks: Blocks, values: np.ndarray) -> np.ndarray:
    """Sum of a per-site complex quantity over each block."""
    ids = blocks.block_id.ravel()
    re = np.bincount(ids, weights=values.real.ravel(), minlength=blocks.count)
    im = np.bincount(ids, weights=values.imag.ravel(), minlength=blocks.count)
    return re + 1j * im


def mr_blocks(D, blocks: Blocks, colour: int, rho: np.ndarray, n_mr: int) -> np.ndarray:
    """n_mr minimal-residual steps on every block of one colour, from delta = 0."""
    m = blocks.mask(colour)
    r = np.where(m, rho, 0)
    delta = np.zeros_like(rho)
    for _ in range(n_mr):
        q = block_apply(D, blocks, colour, r)
        qr = _per_block_sum(blocks, np.sum(np.conj(q) * r, axis=(-2, -1)))
        qq = _per_block_sum(blocks, np.sum(np.abs(q) ** 2, axis=(-2, -1))).real
        alpha = np.where(qq > 0, qr / np.where(qq > 0, qq, 1), 0)
        a = alpha[blocks.block_id][..., None, None]
        delta = delta + np.where(m, a * r, 0)
        r = r - np.where(m, a * q, 0)
    return delta


def sap(D, blocks: Blocks, eta: np.ndarray, ncy: int, n_mr: int) -> np.ndarray:
    """The SAP preconditioner M eta: ncy cycles over the two colours from psi = 0."""
    psi = np.zeros_like(eta)
    for _ in range(ncy):
        for colour in (0, 1):
            rho = np.where(blocks.mask(colour), eta - D(psi), 0)
            psi = psi + mr_blocks(D, blocks, colour, rho, n_mr)
    return psi


def block_hop(op, blocks: Blocks, colour: int, psi: np.ndarray) -> np.ndarray:
    """H_B psi: the hopping term with only the hops inside the blocks of one
    colour (op a dirac.Operator, D = A - kappa H)."""
    m = blocks.mask(colour)
    return np.where(m, op.hop(np.where(m, psi, 0)), 0)


def mr_blocks_eo(op, blocks: Blocks, colour: int, rho: np.ndarray, n_mr: int) -> np.ndarray:
    """The block equations of one colour solved through each block's even-odd
    Schur complement (n_mr minimal-residual steps on it, from zero), then the
    odd sites exactly."""
    m = blocks.mask(colour)
    par = dirac.parity_field(blocks.dims)[..., None, None]
    ev, od = m & (par == 0), m & (par == 1)
    k = op.kappa

    def A(v, where):
        return np.where(where, dirac.site_apply(op.A, v), 0)

    def Ainv(v, where):
        return np.where(where, dirac.site_apply(op.Ainv, v), 0)

    def H(v, where):
        return np.where(where, block_hop(op, blocks, colour, v), 0)

    rho_e, rho_o = np.where(ev, rho, 0), np.where(od, rho, 0)
    r = rho_e + k * H(Ainv(rho_o, od), ev)
    de = np.zeros_like(rho)
    for _ in range(n_mr):
        q = A(r, ev) - k * k * H(Ainv(H(r, od), od), ev)
        qr = _per_block_sum(blocks, np.sum(np.conj(q) * r, axis=(-2, -1)))
        qq = _per_block_sum(blocks, np.sum(np.abs(q) ** 2, axis=(-2, -1))).real
        alpha = np.where(qq > 0, qr / np.where(qq > 0, qq, 1), 0)
        a = alpha[blocks.block_id][..., None, None]
        de = de + np.where(ev, a * r, 0)
        r = r - np.where(ev, a * q, 0)
    do = Ainv(rho_o + k * H(de, od), od)
    return de + do


def sap_eo(op, blocks: Blocks, eta: np.ndarray, ncy: int, n_mr: int) -> np.ndarray:
    """The SAP preconditioner with even-odd block solves: ncy cycles over the
    two colours from psi = 0."""
    psi = np.zeros_like(eta)
    for _ in range(ncy):
        for colour in (0, 1):
            rho = np.where(blocks.mask(colour), eta - op.D(psi), 0)
            psi = psi + mr_blocks_eo(op, blocks, colour, rho, n_mr)
    return psi


def fbicgstab(apply: Callable[[np.ndarray], np.ndarray], precond: Callable[[np.ndarray], np.ndarray],
              b: np.ndarray, tol: float = 1e-10, max_iter: int = 1000,
              x0: Optional[np.ndarray] = None, max_restarts: int = 10):
    """Flexible BiCGStab for A x = b with right preconditioner M (precond),
    stopping on the true residual ||b - A x|| <= tol ||b||; restarts from the
    current x when the iterated residual passes or on a breakdown."""
    info = solvers.SolveInfo()
    bnorm = solvers.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128, copy=True)
    if bnorm == 0.0:
        info.converged, info.residual = True, 0.0
        return np.zeros_like(b), info
    target = tol * bnorm
    while True:
        r = b - apply(x)
        rnorm = solvers.norm(r)
        info.residual = rnorm / bnorm
        if rnorm <= target:
            info.converged = True
            return x, info
        if info.iterations >= max_iter or info.restarts > max_restarts:
            return x, info
        r_hat = r.copy()
        rho_old = alpha = omega = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        while info.iterations < max_iter:
            rho = solvers.dot(r_hat, r)
            if rho == 0:
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            p_hat = precond(p)
            v = apply(p_hat)
            rv = solvers.dot(r_hat, v)
            if rv == 0:
                break
            alpha = rho / rv
            s = r - alpha * v
            s_hat = precond(s)
            t = apply(s_hat)
            tt = solvers.dot(t, t).real
            omega = solvers.dot(t, s) / tt if tt != 0 else 0.0
            x = x + alpha * p_hat + omega * s_hat
            r = s - omega * t
            rho_old = rho
            info.iterations += 1
            rn = solvers.norm(r)
            info.history.append(rn / bnorm)
            if rn <= target or omega == 0:
                break
        info.restarts += 1
