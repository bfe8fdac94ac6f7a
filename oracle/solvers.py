"""Oracle solvers: BiCGStab, CG and the FP64 defect-correction outer loop.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain float64 NumPy.

The paper (Sec. 3, the clover solver benchmark and the mixed-precision
comparison) names BiCGStab and a mixed-precision BiCGStab without giving
their steps. BiCGStab here is van der Vorst's 1992 algorithm as published;
the mixed-precision method is represented by its outer loop, defect
correction, with an inner solver passed in (the oracle runs it in FP64).

Inner products are ``<a, b> = sum conj(a) b`` over every component.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


def dot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a, b))


def norm(a: np.ndarray) -> float:
    return float(np.sqrt(np.vdot(a, a).real))


@dataclass
class SolveInfo:
    converged: bool = False
    iterations: int = 0
    restarts: int = 0
    residual: float = float("inf")          # true relative residual at exit
    history: list = field(default_factory=list)


def bicgstab(apply: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float = 1e-10,
             max_iter: int = 10000, x0: Optional[np.ndarray] = None,
             max_restarts: int = 10) -> tuple[np.ndarray, SolveInfo]:
    """Solve A x = b by BiCGStab until ||b - A x|| <= tol ||b|| (true residual).

    The iterated residual is the stopping test of the inner iteration; when it
    passes, the true residual is recomputed and, if it has not reached the
    tolerance, the iteration restarts from the current x with r = r_hat =
    b - A x. A breakdown (rho or <r_hat, v> exactly zero) restarts the same way.
    """
    info = SolveInfo()
    bnorm = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128, copy=True)
    if bnorm == 0.0:
        info.converged, info.residual = True, 0.0
        return np.zeros_like(b), info
    target = tol * bnorm
    while True:
        r = b - apply(x)
        rnorm = norm(r)
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
            rho = dot(r_hat, r)
            if rho == 0:
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = apply(p)
            rv = dot(r_hat, v)
            if rv == 0:
                break
            alpha = rho / rv
            s = r - alpha * v
            t = apply(s)
            tt = dot(t, t).real
            omega = dot(t, s) / tt if tt != 0 else 0.0
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho_old = rho
            info.iterations += 1
            rn = norm(r)
            info.history.append(rn / bnorm)
            if rn <= target or omega == 0:
                break
        info.restarts += 1


def defect_correction(apply: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
                      inner: Callable[[np.ndarray], np.ndarray], tol: float = 1e-10,
                      max_outer: int = 50) -> tuple[np.ndarray, SolveInfo]:
    """Outer loop of a mixed-precision solve, in FP64.

    x = 0, r = b; while ||r|| > tol ||b||: e = inner(r / ||r||) (an approximate
    solve of A e = r / ||r||), x += ||r|| e, r = b - A x.
    """
    info = SolveInfo()
    bnorm = norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        info.converged, info.residual = True, 0.0
        return x, info
    r = b.copy()
    rnorm = bnorm
    while rnorm > tol * bnorm and info.iterations < max_outer:
        e = inner(r / rnorm)
        x = x + rnorm * e
        r = b - apply(x)
        rnorm = norm(r)
        info.iterations += 1
        info.history.append(rnorm / bnorm)
    info.residual = rnorm / bnorm
    info.converged = rnorm <= tol * bnorm
    return x, info


def cg(apply: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float = 1e-10, max_iter: int = 10000):
    """Conjugate gradients for a Hermitian positive-definite operator, stopping
    on the recomputed true residual ||b - A x|| <= tol ||b|| (restarting from
    x whenever the iterated residual passes but the true one does not)."""
    info = SolveInfo()
    bnorm = norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        info.converged, info.residual = True, 0.0
        return x, info
    target = tol * bnorm
    while True:
        r = b - apply(x)
        rr = np.vdot(r, r).real
        info.residual = np.sqrt(rr) / bnorm
        if np.sqrt(rr) <= target:
            info.converged = True
            return x, info
        if info.iterations >= max_iter or info.restarts > 10:
            return x, info
        p = r.copy()
        while info.iterations < max_iter:
            q = apply(p)
            alpha = rr / np.vdot(p, q).real
            x = x + alpha * p
            r = r - alpha * q
            rr_new = np.vdot(r, r).real
            info.iterations += 1
            info.history.append(np.sqrt(rr_new) / bnorm)
            if np.sqrt(rr_new) <= target:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        info.restarts += 1
