"""Periodic r^-6 lattice sums for the oracle (TEST INFRASTRUCTURE ONLY).

The coarsest MLS grid needs its kernel summed over every periodic image
(Sec. II.C, eq:last-grid-periodic-transformed; the paper only says the sum is
absolutely convergent and can be precalculated).  The image sum converges like
R^-3, so the oracle evaluates it with a Gaussian-screened (Ewald) split of
r^-6, derived here from the Gamma-function integral

    r^-6 = 1/2 int_0^inf t^2 exp(-r^2 t) dt,

cut at t = beta^2.  The part above the cut is short ranged,

    r^-6 exp(-x) (1 + x + x^2/2),   x = beta^2 r^2,

and the part below is smooth with Fourier transform

    fhat(k) = (pi^1.5 beta^3 / 3) [(1 - 2 b^2) exp(-b^2) + 2 sqrt(pi) b^3 erfc(b)],
    b = |k| / (2 beta),

whose value at r = 0 is beta^6 / 6.  Poisson summation turns the smooth part
into (1/V) sum_k fhat(k) cos(k.v).

``direct_r6_sum`` is the slow cross-check: plain image summation inside a
sphere plus the continuum tail 4 pi / (3 V R^3).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

__all__ = ["lattice_r6_sum", "direct_r6_sum", "ewald_screened_real", "ewald_fhat"]


def ewald_screened_real(r, beta):
    """Short-range part r^-6 exp(-x)(1 + x + x^2/2), x = beta^2 r^2."""
    x = (beta * r) ** 2
    return np.exp(-x) * (1.0 + x + 0.5 * x * x) / r ** 6


def ewald_fhat(k, beta):
    """Fourier transform of the smooth part at wavenumber |k|."""
    b = np.asarray(k, dtype=np.float64) / (2.0 * beta)
    return (math.pi ** 1.5 * beta ** 3 / 3.0) * (
        (1.0 - 2.0 * b * b) * np.exp(-b * b) + 2.0 * math.sqrt(math.pi) * b ** 3 * erfc(b))


def lattice_r6_sum(v, box, beta=None, tol=1e-17):
    """Z(v) = sum over n in Z^3 with v + n o L != 0 of |v + n o L|^-6.

    ``v``: (M,3) displacement vectors; ``box``: (3,) orthorhombic lengths.
    ``beta``: screening parameter (default: balanced for the box).
    """
    v = np.atleast_2d(np.asarray(v, dtype=np.float64))
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    if beta is None:
        beta = 3.0 / float(np.min(box))
    # real space: exp(-beta^2 r^2) below tol well before rc
    rc = math.sqrt(-math.log(tol)) / beta + float(np.max(box))
    nr = np.ceil(rc / box).astype(int)
    real = np.zeros(len(v))
    for nx in range(-nr[0], nr[0] + 1):
        for ny in range(-nr[1], nr[1] + 1):
            for nz in range(-nr[2], nr[2] + 1):
                rv = v + np.array([nx, ny, nz]) * box
                r = np.sqrt(np.sum(rv * rv, axis=1))
                ok = r > 0.0
                real[ok] += ewald_screened_real(r[ok], beta)
    # reciprocal space: fhat decays like exp(-b^2)
    kc = 2.0 * beta * math.sqrt(-math.log(tol))
    nk = np.ceil(kc * box / (2.0 * math.pi)).astype(int)
    mx, my, mz = (np.arange(-m, m + 1) for m in nk)
    MX, MY, MZ = np.meshgrid(mx, my, mz, indexing="ij")
    kvec = 2.0 * math.pi * np.stack([MX.ravel(), MY.ravel(), MZ.ravel()], axis=1) / box
    kn = np.sqrt(np.sum(kvec * kvec, axis=1))
    fh = ewald_fhat(kn, beta)
    recip = (np.cos(v @ kvec.T) @ fh) / V
    # remove the r = 0 term of the smooth part where v sits on the lattice
    frac = v / box
    on_lattice = np.all(np.abs(frac - np.round(frac)) == 0.0, axis=1)
    self_term = np.where(on_lattice, beta ** 6 / 6.0, 0.0)
    return real + recip - self_term


def direct_r6_sum(v, box, R):
    """Image sum over |v + n o L| <= R plus the continuum tail beyond R."""
    v = np.atleast_2d(np.asarray(v, dtype=np.float64))
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    nr = np.ceil(R / box).astype(int) + 1
    gx, gy, gz = (np.arange(-m, m + 1) for m in nr)
    NX, NY, NZ = np.meshgrid(gx, gy, gz, indexing="ij")
    shifts = np.stack([NX.ravel(), NY.ravel(), NZ.ravel()], axis=1) * box
    out = np.zeros(len(v))
    for i, vi in enumerate(v):
        rv = vi[None, :] + shifts
        r = np.sqrt(np.sum(rv * rv, axis=1))
        ok = (r > 0.0) & (r <= R)
        out[i] = np.sum(r[ok] ** -6.0)
    return out + 4.0 * math.pi / (3.0 * V * R ** 3)
