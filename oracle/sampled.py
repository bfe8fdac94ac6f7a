"""The oracle's operators evaluated at a list of sites only.

TEST INFRASTRUCTURE ONLY. Used to check outputs on lattices too large for the
whole-field oracle (32^3 x 64 and up): each requested output site is computed
from the definitions in ``oracle.dirac`` by gathering exactly the links and
spinor values it depends on. Site lists are integer arrays of shape (N, 4)
holding (x, y, z, t).

Pinned against the whole-field oracle on small lattices
(tests/test_oracle_pins.py).
"""

from __future__ import annotations

import numpy as np

from .dirac import GAMMA, GAMMA5, ONE4, sigma


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


# ---------------------------------------------------------------- domain wall
# Five-dimensional fields are indexed [s, t, z, y, x, spin, colour] as in
# oracle.dwf; the forms below return every s at the listed 4-d sites,
# (Ls, N, 4, 3). The operator is the Moebius one of oracle.dwf:
#   D = D_W (b5 + c5 S) + 1 - S,  D^dag = (b5 + c5 S^dag) D_W^dag + 1 - S^dag,
#   D_W = (4 - M5) - H/2 on every slice,
# with H^dag = gamma5 H gamma5 here (oracle.dwf takes H^dag term by term, so
# the two agree only if both are right).

P_PLUS = (ONE4 + GAMMA5) / 2
P_MINUS = (ONE4 - GAMMA5) / 2


def gather5(field, sites):
    return field[:, sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]


def s_hop(v, mf: float, dag: bool = False):
    """S v (or S^dag v) of values v at the same sites, (Ls, N, 4, 3):
    (S v)_s = P_- v_{s+1} + P_+ v_{s-1}, v_{Ls} = -m_f v_0, v_{-1} = -m_f v_{Ls-1};
    the adjoint exchanges the projectors."""
    Ls = v.shape[0]
    pu, pd = (P_PLUS, P_MINUS) if dag else (P_MINUS, P_PLUS)
    out = np.empty_like(v)
    for s in range(Ls):
        up = v[s + 1] if s + 1 < Ls else -mf * v[0]
        dn = v[s - 1] if s > 0 else -mf * v[Ls - 1]
        out[s] = pu @ up + pd @ dn
    return out


def _hop5(U, v_at, t_bc, sites, Ls, gamma5_sandwich=False):
    """H applied slice by slice at the sites; v_at(sites) gives (Ls, N, 4, 3).
    With gamma5_sandwich the result is gamma5 H gamma5 = H^dag."""
    out = np.empty((Ls, len(sites), 4, 3), dtype=np.complex128)
    for s in range(Ls):
        if gamma5_sandwich:
            out[s] = GAMMA5 @ hop_at(U, lambda x, s=s: GAMMA5 @ v_at(x)[s], t_bc, sites)
        else:
            out[s] = hop_at(U, lambda x, s=s: v_at(x)[s], t_bc, sites)
    return out


def dwf_at(U, psi, M5, mf, b5, c5, t_bc, sites, dag: bool = False):
    """(D psi) or (D^dag psi) at the listed 4-d sites, every s."""
    sites = np.asarray(sites)
    Ls = psi.shape[0]
    own = gather5(psi, sites)
    if not dag:
        def phi_at(x):
            v = gather5(psi, x)
            return b5 * v + c5 * s_hop(v, mf)
        dw = (4.0 - M5) * phi_at(sites) - 0.5 * _hop5(U, phi_at, t_bc, sites, Ls)
        return dw + own - s_hop(own, mf)
    u = (4.0 - M5) * own - 0.5 * _hop5(U, lambda x: gather5(psi, x), t_bc, sites, Ls, gamma5_sandwich=True)
    return b5 * u + c5 * s_hop(u, mf, True) + own - s_hop(own, mf, True)


def m5op_matrix(Ls, M5, mf, b5, c5):
    """The site-local part M5op = (4 - M5)(b5 + c5 S) + 1 - S as an
    (Ls 4) x (Ls 4) matrix over (s, spin), row and column index s 4 + spin."""
    cols = []
    for s in range(Ls):
        for a in range(4):
            e = np.zeros((Ls, 1, 4, 1), dtype=np.complex128)
            e[s, 0, a, 0] = 1.0
            col = (4.0 - M5) * (b5 * e + c5 * s_hop(e, mf)) + e - s_hop(e, mf)
            cols.append(col[:, 0, :, 0].reshape(-1))
    return np.array(cols).T


def local_apply(K, v):
    """(K v) at every site and colour for K over (s, spin), v (Ls, N, 4, 3)."""
    Ls, n = v.shape[:2]
    w = v.transpose(1, 3, 0, 2).reshape(n, 3, Ls * 4) @ K.T
    return w.reshape(n, 3, Ls, 4).transpose(2, 0, 3, 1)


def dwf_schur_at(U, x_even, M5, mf, b5, c5, t_bc, sites, dag: bool = False):
    """(S_ee x) or (S_ee^dag x) at listed even sites, every s, for x supported
    on the even sites: S_ee = M5op - Dhop M5op^-1 Dhop with the hopping part
    Dhop = -1/2 H (b5 + c5 S), and S_ee^dag = M5op^dag - Dhop^dag M5op^-dag Dhop^dag,
    Dhop^dag = -1/2 (b5 + c5 S^dag) H^dag."""
    sites = np.asarray(sites)
    Ls = x_even.shape[0]
    dims = _dims(U)
    K = m5op_matrix(Ls, M5, mf, b5, c5)
    if dag:
        K = np.conj(K.T)
    Kinv = np.linalg.inv(K)

    def dhop(v_at, at):
        if not dag:
            return -0.5 * _hop5(U, lambda x: b5 * v_at(x) + c5 * s_hop(v_at(x), mf), t_bc, at, Ls)
        h = -0.5 * _hop5(U, v_at, t_bc, at, Ls, gamma5_sandwich=True)
        return b5 * h + c5 * s_hop(h, mf, True)

    nbr = np.concatenate([step(dims, sites, mu, s) for mu in range(4) for s in (+1, -1)])
    lin = _linear(dims, nbr)
    uniq, first = np.unique(lin, return_index=True)
    odd_sites = nbr[first]
    z = local_apply(Kinv, dhop(lambda x: gather5(x_even, x), odd_sites))

    def z_at(x):
        return z[:, np.searchsorted(uniq, _linear(dims, x))]

    return local_apply(K, gather5(x_even, sites)) - dhop(z_at, sites)


# ---------------------------------------------------------------- staggered
def stag_phase(sites, mu):
    """The staggered phase eta_mu at each listed site (oracle.staggered)."""
    x, y, z = sites[:, 0], sites[:, 1], sites[:, 2]
    return [np.ones(len(sites)), (-1.0) ** x, (-1.0) ** (x + y), (-1.0) ** (x + y + z)][mu]


def stag_dirac_at(U, psi, mass, t_bc, sites):
    """(m + H) psi at the listed sites for a colour-vector field psi[t, z, y, x, c]:
    (H psi)(x) = 1/2 sum_mu eta_mu(x) [U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu)]."""
    dims = _dims(U)
    sites = np.asarray(sites)
    out = mass * gather(psi, sites)
    for mu in range(4):
        f = step(dims, sites, mu, +1)
        b = step(dims, sites, mu, -1)
        ef = np.ones(len(sites))
        eb = np.ones(len(sites))
        if mu == 3:
            ef[sites[:, 3] == dims[3] - 1] = t_bc
            eb[sites[:, 3] == 0] = t_bc
        fwd = (gather(U, sites)[:, mu] @ gather(psi, f)[..., None])[..., 0]
        bwd = (_dag(gather(U, b)[:, mu]) @ gather(psi, b)[..., None])[..., 0]
        out = out + 0.5 * stag_phase(sites, mu)[:, None] * (ef[:, None] * fwd - eb[:, None] * bwd)
    return out


# ---------------------------------------------------------------- SAP, one cycle at listed blocks
def _block_sites(origin, bdims):
    bx, by, bz, bt = bdims
    t, z, y, x = np.meshgrid(np.arange(bt), np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1) + np.asarray(origin)


def _block_mr(U, kappa, csw, t_bc, sites, rho, n_mr):
    """n_mr minimal-residual steps on one block, D_B = A - kappa H with the hops
    that leave the block removed, from delta = 0 (oracle.sap.mr_blocks on one
    block); rho and the result are (N, 4, 3) at the block's sites."""
    dims = _dims(U)
    lin = _linear(dims, sites)
    order = np.argsort(lin)
    slin = lin[order]
    A = clover_at(U, kappa, csw, sites)

    def DB(v):
        def v_at(x):
            lx = _linear(dims, x)
            pos = np.clip(np.searchsorted(slin, lx), 0, len(slin) - 1)
            inside = slin[pos] == lx
            out = np.zeros((len(x), 4, 3), dtype=np.complex128)
            out[inside] = v[order[pos[inside]]]
            return out
        return site_mul(A, v) - kappa * hop_at(U, v_at, t_bc, sites)

    r = rho.copy()
    delta = np.zeros_like(rho)
    for _ in range(n_mr):
        q = DB(r)
        qq = np.sum(np.abs(q) ** 2)
        a = np.sum(np.conj(q) * r) / qq if qq > 0 else 0.0
        delta = delta + a * r
        r = r - a * q
    return delta


def sap_one_cycle_at(U, kappa, csw, t_bc, eta, bdims, block_origin, n_mr):
    """M eta of one SAP cycle (colour 0 blocks from eta, then colour 1 blocks
    from eta - D psi), at the sites of the block starting at block_origin:
    a colour-0 block depends only on its own sites; a colour-1 block also on
    the colour-0 updates of the blocks across its faces, computed here
    (oracle.sap.sap with ncy = 1, evaluated block by block)."""
    dims = _dims(U)
    origin = np.asarray(block_origin)
    colour = int(np.sum(origin // np.asarray(bdims)) % 2)
    sites = _block_sites(origin, bdims)
    if colour == 0:
        return sites, _block_mr(U, kappa, csw, t_bc, sites, gather(eta, sites), n_mr)
    # psi after the colour-0 half cycle, on the neighbouring colour-0 blocks
    psi0 = {}
    for mu in range(4):
        for sg in (+1, -1):
            o = origin.copy()
            o[mu] = (o[mu] + sg * bdims[mu]) % dims[mu]
            key = tuple(o)
            if key not in psi0:
                s0 = _block_sites(o, bdims)
                psi0[key] = (s0, _block_mr(U, kappa, csw, t_bc, s0, gather(eta, s0), n_mr))
    all_s = np.concatenate([v[0] for v in psi0.values()])
    all_v = np.concatenate([v[1] for v in psi0.values()])
    alin = _linear(dims, all_s)
    order = np.argsort(alin)
    slin = alin[order]

    def psi_at(x):
        lx = _linear(dims, x)
        pos = np.clip(np.searchsorted(slin, lx), 0, len(slin) - 1)
        out = np.zeros((len(x), 4, 3), dtype=np.complex128)
        hit = slin[pos] == lx
        out[hit] = all_v[order[pos[hit]]]
        return out

    # rho = eta - D psi at the block (psi is zero on the block itself)
    rho = gather(eta, sites) + kappa * hop_at(U, psi_at, t_bc, sites)
    return sites, _block_mr(U, kappa, csw, t_bc, sites, rho, n_mr)
