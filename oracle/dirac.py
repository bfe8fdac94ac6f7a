"""Whole-field oracle: Wilson and clover Dirac operators and their even-odd blocks.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain float64 NumPy.

The paper (Sec. 2) names the Wilson/clover operator and its even-odd
decomposition, Eq. (1), without printing matrix elements. The definitions
below are the textbook ones with the conventions this project fixes:

* sites ``(x, y, z, t)``; arrays are indexed ``[t, z, y, x, ...]``;
  direction ``mu = 0, 1, 2, 3`` is ``x, y, z, t``;
* parity of a site is ``(x + y + z + t) mod 2``; even = 0;
* neighbours wrap periodically; a hop in ``t`` that crosses the boundary
  carries the fermion boundary factor ``eta = t_bc`` (``-1`` = antiperiodic);
* Dirac-Pauli gamma matrices: ``gamma_j = [[0, -i sigma_j], [i sigma_j, 0]]``
  for ``j = x, y, z`` and ``gamma_t = diag(1, 1, -1, -1)``;
* hopping term (forward hop with ``1 - gamma``)::

      (H psi)(x) = sum_mu  eta (1 - gamma_mu) U_mu(x)          psi(x + mu)
                         + eta (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)

* Wilson operator ``D = 1 - kappa H``; clover operator ``D = A - kappa H``
  with the site matrix ``A`` of :func:`clover_matrix`;
* parity blocks ``D_pq = P_p D P_q`` (Eq. (1)), the Schur complement
  ``S = D_ee - D_eo D_oo^-1 D_oe`` and the paper's form
  ``D^(eo) = 1 - D_ee^-1 D_eo D_oo^-1 D_oe = D_ee^-1 S``.
"""

from __future__ import annotations

import numpy as np

# direction mu -> array axis of a field indexed [t, z, y, x, ...]
MU_AXIS = (3, 2, 1, 0)
T_DIR = 3


def dims_of(field: np.ndarray):
    lt, lz, ly, lx = field.shape[:4]
    return (lx, ly, lz, lt)


def _pauli():
    s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    return s1, s2, s3


def gamma_matrices() -> np.ndarray:
    """Dirac-Pauli Euclidean gamma matrices, index 0..3 = x, y, z, t."""
    z = np.zeros((2, 2), dtype=np.complex128)
    gs = [np.block([[z, -1j * s], [1j * s, z]]) for s in _pauli()]
    gs.append(np.diag([1, 1, -1, -1]).astype(np.complex128))
    return np.array(gs)


GAMMA = gamma_matrices()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)


def sigma(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = [gamma_mu, gamma_nu] / (2i), a Hermitian 4x4 matrix."""
    return (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu]) / 2j


def parity_field(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return (x + y + z + t) % 2


def mask(field: np.ndarray, parity: int) -> np.ndarray:
    """P_parity applied to a spinor field (sites of the other parity set to zero)."""
    p = parity_field(dims_of(field)) == parity
    return field * p[..., None, None]


def shift(field: np.ndarray, mu: int, step: int) -> np.ndarray:
    """The field seen from x: returns f(x + step * mu) at x, periodic wrap."""
    return np.roll(field, -step, axis=MU_AXIS[mu])


def boundary_factor(dims, mu: int, step: int, t_bc: int) -> np.ndarray:
    """eta(x) for the hop from x to x + step*mu: t_bc where a t hop wraps, else 1."""
    lx, ly, lz, lt = dims
    eta = np.ones((lt, lz, ly, lx))
    if mu == T_DIR and t_bc != 1:
        if step > 0:
            eta[lt - 1] = t_bc
        else:
            eta[0] = t_bc
    return eta


def dagger(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def colour_mul(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(u psi)[..., s, a] = sum_b u[..., a, b] psi[..., s, b]."""
    return psi @ np.swapaxes(u, -1, -2)


def spin_mul(g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(g psi)[..., s, a] = sum_r g[s, r] psi[..., r, a]."""
    return g @ psi


def hop(U: np.ndarray, psi: np.ndarray, t_bc: int) -> np.ndarray:
    """The hopping term H psi written out direction by direction."""
    dims = dims_of(psi)
    out = np.zeros_like(psi)
    for mu in range(4):
        u = U[..., mu, :, :]
        fwd = shift(psi, mu, +1) * boundary_factor(dims, mu, +1, t_bc)[..., None, None]
        out += spin_mul(ONE4 - GAMMA[mu], colour_mul(u, fwd))
        u_back = shift(u, mu, -1)
        bwd = shift(psi, mu, -1) * boundary_factor(dims, mu, -1, t_bc)[..., None, None]
        out += spin_mul(ONE4 + GAMMA[mu], colour_mul(dagger(u_back), bwd))
    return out


def wilson(U: np.ndarray, psi: np.ndarray, kappa: float, t_bc: int) -> np.ndarray:
    """Wilson operator D psi = psi - kappa H psi."""
    return psi - kappa * hop(U, psi, t_bc)


def clover_leaves(U: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x): sum of the four plaquettes in the (mu, nu) plane that start
    and end at x, each run in the mu-then-nu sense, so Q_{nu mu} = Q_{mu nu}^dag."""

    def link(d, a, b):
        # U_d(x + a*mu + b*nu) seen from x
        f = U[..., d, :, :]
        if a:
            f = shift(f, mu, a)
        if b:
            f = shift(f, nu, b)
        return f

    um, un = mu, nu
    q = link(um, 0, 0) @ link(un, 1, 0) @ dagger(link(um, 0, 1)) @ dagger(link(un, 0, 0))
    q += link(un, 0, 0) @ dagger(link(um, -1, 1)) @ dagger(link(un, -1, 0)) @ link(um, -1, 0)
    q += dagger(link(um, -1, 0)) @ dagger(link(un, -1, -1)) @ link(um, -1, -1) @ link(un, 0, -1)
    q += dagger(link(un, 0, -1)) @ link(um, 0, -1) @ link(un, 1, -1) @ dagger(link(um, 0, 0))
    return q


def field_strength(U: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag) / (8i): Hermitian, zero for unit links."""
    q = clover_leaves(U, mu, nu)
    return (q - dagger(q)) / 8j


def clover_matrix(U: np.ndarray, kappa: float, csw: float) -> np.ndarray:
    """Site matrix A(x) = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x).

    12x12 per site, row/column index ``3*spin + colour``. This is the
    Sheikholeslami-Wohlert term in the hopping-parameter normalisation, with
    Hermitian sigma and F and no trace subtraction. Its overall sign and trace
    convention are a reading (the paper prints neither); no invariant fixes
    them, so they are parity unpinned. The fermion boundary factor does not
    enter: A is built from the plain periodic links.
    """
    dims = dims_of(U)
    lx, ly, lz, lt = dims
    a = np.zeros((lt, lz, ly, lx, 12, 12), dtype=np.complex128)
    a[...] = np.eye(12)
    if csw == 0.0:
        return a
    for mu in range(4):
        for nu in range(mu + 1, 4):
            f = field_strength(U, mu, nu)
            k = np.einsum("st,...ab->...satb", sigma(mu, nu), f).reshape(lt, lz, ly, lx, 12, 12)
            a += kappa * csw * k
    return a


def site_apply(a: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(A psi)(x) = A(x) psi(x) with A a 12x12 matrix per site."""
    shape = psi.shape
    flat = psi.reshape(shape[:4] + (12, 1))
    return (a @ flat).reshape(shape)


class Operator:
    """The clover (or, with c_SW = 0, Wilson) operator on one gauge field.

    ``D = A - kappa H``; ``A`` and its per-site inverse are built once.
    """

    def __init__(self, U: np.ndarray, kappa: float, csw: float = 0.0, t_bc: int = -1):
        self.U = U
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.t_bc = int(t_bc)
        self.dims = dims_of(U)
        self.A = clover_matrix(U, self.kappa, self.csw)
        self._Ainv = None

    @property
    def Ainv(self) -> np.ndarray:
        if self._Ainv is None:
            self._Ainv = np.linalg.inv(self.A)
        return self._Ainv

    # full operator --------------------------------------------------------
    def hop(self, psi):
        return hop(self.U, psi, self.t_bc)

    def D(self, psi):
        return site_apply(self.A, psi) - self.kappa * self.hop(psi)

    def Ddag(self, psi):
        """D^dagger through gamma5-hermiticity is NOT used here: written out
        from the definition, D^dag = A - kappa H^dag."""
        return site_apply(dagger(self.A), psi) - self.kappa * self.hop_dag(psi)

    def hop_dag(self, psi):
        """H^dagger psi: the adjoint of each hop, taken term by term."""
        dims = self.dims
        out = np.zeros_like(psi)
        for mu in range(4):
            u = self.U[..., mu, :, :]
            # adjoint of  eta (1-g) U(x) psi(x+mu)  contributes at x+mu from x
            a = spin_mul(ONE4 - GAMMA[mu], colour_mul(dagger(shift(u, mu, -1)),
                                                      shift(psi, mu, -1)))
            out += a * boundary_factor(dims, mu, -1, self.t_bc)[..., None, None]
            # adjoint of  eta (1+g) U(x-mu)^dag psi(x-mu)  contributes at x-mu from x
            b = spin_mul(ONE4 + GAMMA[mu], colour_mul(u, shift(psi, mu, +1)))
            out += b * boundary_factor(dims, mu, +1, self.t_bc)[..., None, None]
        return out

    # parity blocks D_pq = P_p D P_q (Eq. (1)) ---------------------------------
    def block(self, p: int, q: int, psi):
        return mask(self.D(mask(psi, q)), p)

    def Dee(self, psi):
        return self.block(0, 0, psi)

    def Doo(self, psi):
        return self.block(1, 1, psi)

    def Deo(self, psi):
        return self.block(0, 1, psi)

    def Doe(self, psi):
        return self.block(1, 0, psi)

    def site_inverse(self, p: int, psi):
        """D_pp^-1 psi on parity p (zero elsewhere): the per-site inverse of A."""
        return mask(site_apply(self.Ainv, mask(psi, p)), p)

    def schur(self, x):
        """S x = D_ee x - D_eo D_oo^-1 D_oe x, for x supported on even sites."""
        return self.Dee(x) - self.Deo(self.site_inverse(1, self.Doe(x)))

    def dprec(self, x):
        """Eq. (1): D^(eo) x = x - D_ee^-1 D_eo D_oo^-1 D_oe x on even sites."""
        xe = mask(x, 0)
        return xe - self.site_inverse(0, self.Deo(self.site_inverse(1, self.Doe(xe))))

    def eo_source(self, b):
        """Even-site right-hand side of the Schur system: b_e - D_eo D_oo^-1 b_o."""
        return mask(b, 0) - self.Deo(self.site_inverse(1, b))

    def eo_reconstruct(self, xe, b):
        """Odd-site solution x_o = D_oo^-1 (b_o - D_oe x_e); returns x_e + x_o."""
        xe = mask(xe, 0)
        return xe + self.site_inverse(1, mask(b, 1) - self.Doe(xe))


def gamma5(psi: np.ndarray) -> np.ndarray:
    return spin_mul(GAMMA5, psi)


def gauge_transform(U: np.ndarray, G: np.ndarray) -> np.ndarray:
    """U_mu(x) -> G(x) U_mu(x) G(x + mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ dagger(shift(G, mu, +1))
    return out


def transform_spinor(psi: np.ndarray, G: np.ndarray) -> np.ndarray:
    return colour_mul(G, psi)


def norm2(v: np.ndarray) -> float:
    return float(np.vdot(v, v).real)


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b|| / ||b||."""
    nb = np.sqrt(norm2(b))
    return float(np.sqrt(norm2(a - b)) / (nb if nb > 0 else 1.0))


def average_plaquette(U: np.ndarray) -> float:
    """(1/3) Re tr of the plaquette averaged over sites and the six planes."""
    acc = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            p = U[..., mu, :, :] @ shift(U[..., nu, :, :], mu, 1) @ dagger(shift(U[..., mu, :, :], nu, 1)) \
                @ dagger(U[..., nu, :, :])
            acc += np.trace(p, axis1=-2, axis2=-1).real.mean() / 3.0
    return acc / 6.0
