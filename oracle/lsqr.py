"""LSQR and CGLS oracles, FP64 (test infrastructure only).

LSQR follows Paige & Saunders, "LSQR: An algorithm for sparse linear
equations and sparse least squares", ACM TOMS 8(1), 1982: Golub-Kahan
bidiagonalisation with the QR update written in their notation (alpha, beta,
rho, rhobar, c, s, theta, phi, phibar).  Damping 0, x0 = 0 and a fixed number
of iterations (no stopping test), as the solves here run fixed counts.

CGLS is the solver the paper runs for the Marchenko equations (10 iterations,
Applications section); LSQR and CGLS produce the same iterates in exact
arithmetic, which the tests use as a pin.

Operators are given as callables on lists of real arrays (the Marchenko
unknown is a pair of blocks); inner products sum over every element of every
block.
"""
from __future__ import annotations

import math

import numpy as np


def _dot(a, b) -> float:
    return float(sum(np.vdot(p.ravel(), q.ravel()).real for p, q in zip(a, b)))


def _nrm(a) -> float:
    return math.sqrt(_dot(a, a))


def _lin(alpha, a, beta, b):
    return [alpha * p + beta * q for p, q in zip(a, b)]


def lsqr(A, AH, b, niter: int):
    """Returns (x, history) with history[i] = phibar after i iterations (residual norm estimate).

    A maps model blocks -> data blocks, AH maps data -> model; b is a list of arrays.
    """
    b = [np.asarray(p, dtype=np.float64) for p in b]
    beta = _nrm(b)
    u = [p / beta for p in b] if beta > 0 else [np.zeros_like(p) for p in b]
    v = AH(u)
    alpha = _nrm(v)
    v = [p / alpha for p in v] if alpha > 0 else v
    w = [p.copy() for p in v]
    x = [np.zeros_like(p) for p in v]
    phibar, rhobar = beta, alpha
    hist = [phibar]
    for _ in range(niter):
        Av = A(v)
        u = _lin(1.0, Av, -alpha, u)
        beta = _nrm(u)
        if beta > 0:
            u = [p / beta for p in u]
        ATu = AH(u)
        v = _lin(1.0, ATu, -beta, v)
        alpha = _nrm(v)
        if alpha > 0:
            v = [p / alpha for p in v]
        rho = math.hypot(rhobar, beta)
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = _lin(1.0, x, phi / rho, w)
        w = _lin(1.0, v, -theta / rho, w)
        hist.append(phibar)
    return x, np.asarray(hist)


def cgls(A, AH, b, niter: int):
    """Conjugate gradients on the normal equations (Hestenes-Stiefel form), x0 = 0."""
    b = [np.asarray(p, dtype=np.float64) for p in b]
    r = [p.copy() for p in b]
    s = AH(r)
    p = [q.copy() for q in s]
    x = [np.zeros_like(q) for q in s]
    gamma = _dot(s, s)
    hist = [_nrm(r)]
    for _ in range(niter):
        q = A(p)
        delta = _dot(q, q)
        if delta == 0:
            break
        a = gamma / delta
        x = _lin(1.0, x, a, p)
        r = _lin(1.0, r, -a, q)
        s = AH(r)
        gnew = _dot(s, s)
        p = _lin(1.0, s, gnew / gamma, p)
        gamma = gnew
        hist.append(_nrm(r))
    return x, np.asarray(hist)
