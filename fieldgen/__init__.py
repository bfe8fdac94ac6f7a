"""Seeded synthetic inputs for the Wilson/clover operator and its solver.

This module is the only code shared by the CPU oracle and the GPU path. It
generates input fields and nothing else: it holds none of the operator's or
the solver's arithmetic.

Layouts (NumPy C order, complex128):

* gauge field ``U[t, z, y, x, mu, a, b]`` with ``mu = 0, 1, 2, 3 = x, y, z, t``;
  every link is an SU(3) matrix (unitary, determinant 1);
* spinor field ``psi[t, z, y, x, spin, colour]`` with 4 spins and 3 colours.

Randomness. Every field is drawn time slice by time slice, and slice ``t`` of
field ``field_id`` under ``seed`` uses its own PCG64 stream seeded with
``SeedSequence([seed, field_id, t])``. A field is therefore the same whether it
is generated whole or slice by slice, and any slice can be regenerated alone.

Link generators (the operator is defined for any SU(3) field; the paper fixes
no ensemble, so these are synthetic stand-ins for a gauge configuration):

* ``haar``: a complex Ginibre matrix (real and imaginary parts of each entry
  standard normal) whose rows 0 and 1 are Gram-Schmidt orthonormalised; row 2
  is then the complex conjugate of the cross product of rows 0 and 1, which
  makes the matrix special unitary.
* ``smooth``: ``U = exp(i * eps * H)`` with ``H`` a random traceless Hermitian
  matrix, ``H = scale * ((G + G^dagger)/2 - tr(...)/3)`` for a Ginibre ``G``,
  so that ``E[tr H^2] = 8 * scale^2``. The exponential is taken through the
  Hermitian eigendecomposition and the result is re-projected onto SU(3) as in
  ``haar``, so that the two-row form of every link is exact to rounding.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "GAUGE_ID", "SOURCE_ID", "slice_rng", "project_su3", "haar_links",
    "smooth_links", "gauge_field", "gaussian_spinor", "point_source",
    "random_su3_field", "site_count",
]

GAUGE_ID = 0
SOURCE_ID = 1
TRANSFORM_ID = 2


def site_count(dims) -> int:
    lx, ly, lz, lt = dims
    return int(lx) * int(ly) * int(lz) * int(lt)


def slice_rng(seed: int, field_id: int, t: int) -> np.random.Generator:
    """The PCG64 stream of time slice ``t`` of field ``field_id``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(field_id), int(t)])))


def _ginibre(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def project_su3(m: np.ndarray) -> np.ndarray:
    """Gram-Schmidt rows 0 and 1 of each 3x3 matrix; row 2 = conj(row0 x row1)."""
    m = np.asarray(m, dtype=np.complex128)
    r0 = m[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = m[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def haar_links(rng: np.random.Generator, n: int) -> np.ndarray:
    return project_su3(_ginibre(rng, n))


def smooth_links(rng: np.random.Generator, n: int, eps: float, scale: float = 1.0) -> np.ndarray:
    g = _ginibre(rng, n)
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[:, None, None] * np.eye(3)
    h = scale * h
    lam, vec = np.linalg.eigh(h)
    u = np.einsum("nab,nb,ncb->nac", vec, np.exp(1j * eps * lam), np.conj(vec))
    return project_su3(u)


def gauge_field(dims, seed: int, kind: str = "haar", eps: float = 0.3, scale: float = 1.0,
                t_slices=None) -> np.ndarray:
    """Gauge field ``U[t, z, y, x, mu, a, b]`` (or only the listed time slices)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    ts = range(lt) if t_slices is None else list(t_slices)
    per = lz * ly * lx * 4
    out = np.empty((len(ts), lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    for i, t in enumerate(ts):
        rng = slice_rng(seed, GAUGE_ID, t)
        if kind == "haar":
            u = haar_links(rng, per)
        elif kind == "smooth":
            u = smooth_links(rng, per, eps, scale)
        elif kind == "unit":
            u = np.broadcast_to(np.eye(3, dtype=np.complex128), (per, 3, 3))
        else:
            raise ValueError(f"unknown link generator {kind!r}")
        out[i] = u.reshape(lz, ly, lx, 4, 3, 3)
    return out


def gaussian_spinor(dims, seed: int, field_id: int = SOURCE_ID, t_slices=None) -> np.ndarray:
    """Complex Gaussian spinor, E|z|^2 = 1 per component (re, im ~ N(0, 1/2))."""
    lx, ly, lz, lt = (int(d) for d in dims)
    ts = range(lt) if t_slices is None else list(t_slices)
    out = np.empty((len(ts), lz, ly, lx, 4, 3), dtype=np.complex128)
    for i, t in enumerate(ts):
        g = slice_rng(seed, field_id, t).standard_normal((lz, ly, lx, 4, 3, 2)) * np.sqrt(0.5)
        out[i] = g[..., 0] + 1j * g[..., 1]
    return out


def point_source(dims, spin: int, colour: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """Unit source at one site (x, y, z, t) in one spin and colour; zero elsewhere."""
    lx, ly, lz, lt = (int(d) for d in dims)
    out = np.zeros((lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    x, y, z, t = site
    out[t, z, y, x, spin, colour] = 1.0
    return out


def random_su3_field(dims, seed: int) -> np.ndarray:
    """One Haar SU(3) matrix per site, ``G[t, z, y, x, a, b]`` (gauge transformations)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    out = np.empty((lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    for t in range(lt):
        out[t] = haar_links(slice_rng(seed, TRANSFORM_ID, t), lz * ly * lx).reshape(lz, ly, lx, 3, 3)
    return out
