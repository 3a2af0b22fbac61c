"""Exact periodic r^-6 dispersion energy and forces (TEST INFRASTRUCTURE ONLY).

The quantity MLS approximates (Sec. II.A.1, eq:pot-vec-mat-vec with
G_ij = r_ij^-6 and G_ii = 0, summed over periodic images):

    E* = -1/2 sum_i sum_{(j,n) != (i,0)} xi_i xi_j |x_i - x_j - n o L|^-6,
    xi_i = sqrt(C6_i),   F*_i = -dE*/dx_i.

Two independent evaluations are provided: ``exact_ewald`` (Gaussian-screened
split, exponentially convergent; see ``lattice``) and ``exact_direct`` (plain
image summation inside a sphere plus a continuum tail; tiny systems only).
"""
from __future__ import annotations

import math

import numpy as np

from .lattice import ewald_fhat

__all__ = ["ewald_field", "exact_ewald", "exact_ewald_lb", "exact_direct"]


def ewald_field(pos, w, box, beta=None, tol=1e-16, chunk=2048, targets=None):
    """Potential u_i = sum'_{(j,n)} w_j |x_i - x_j - n o L|^-6 of source
    weights w at every atom (or at the atoms ``targets`` only), and
    g_i = sum' w_j (dphi/dr / r)(x_i - x_j - n o L), so that an atom of weight
    v_i feels the force v_i g_i.  Ewald split."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    tidx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    n = len(tidx)
    V = float(np.prod(box))
    if beta is None:
        beta = 3.0 / float(np.min(box))
    # ---- real space
    rc = math.sqrt(-math.log(tol)) / beta
    nr = np.ceil(rc / box).astype(int) + 1
    u = np.zeros(n)
    g = np.zeros((n, 3))
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        ti = tidx[i0:i1]
        for nx in range(-nr[0], nr[0] + 1):
            for ny in range(-nr[1], nr[1] + 1):
                for nz in range(-nr[2], nr[2] + 1):
                    s = np.array([nx, ny, nz]) * box
                    d = pos[ti, None, :] - pos[None, :, :] - s      # (ci, N, 3)
                    r2 = np.sum(d * d, axis=2)
                    if nx == 0 and ny == 0 and nz == 0:
                        r2[np.arange(i1 - i0), ti] = np.inf
                    m = r2 < rc * rc
                    if not m.any():
                        continue
                    r2m = np.where(m, r2, 1.0)
                    x = beta * beta * r2m
                    ex = np.exp(-x)
                    phi = np.where(m, ex * (1.0 + x + 0.5 * x * x) / r2m ** 3, 0.0)
                    r = np.sqrt(r2m)
                    dphi = np.where(m, -6.0 * ex * (1.0 + x + 0.5 * x * x) / r ** 7
                                    - beta ** 6 * ex / r, 0.0)
                    u[i0:i1] += phi @ w
                    coef = dphi / r * w[None, :]
                    g[i0:i1] += np.einsum("ij,ijk->ik", coef, d)
    # ---- reciprocal space
    kc = 2.0 * beta * math.sqrt(-math.log(tol))
    nk = np.ceil(kc * box / (2.0 * math.pi)).astype(int)
    mx, my, mz = (np.arange(-m, m + 1) for m in nk)
    MX, MY, MZ = np.meshgrid(mx, my, mz, indexing="ij")
    kvec = 2.0 * math.pi * np.stack([MX.ravel(), MY.ravel(), MZ.ravel()], axis=1) / box
    kn = np.sqrt(np.sum(kvec * kvec, axis=1))
    fh = ewald_fhat(kn, beta)
    keep = fh > tol * fh.max()
    kvec, fh = kvec[keep], fh[keep]
    for k0 in range(0, len(kvec), 512):
        kv = kvec[k0:k0 + 512]
        f = fh[k0:k0 + 512]
        ph = pos @ kv.T                                # (N, K)
        c, s = np.cos(ph), np.sin(ph)
        Sc = w @ c                                     # Re S(k)
        Ss = w @ s                                     # Im S(k)
        c, s = c[tidx], s[tidx]
        # u_i gets (1/V) sum_k fhat Re(e^{-ik x_i} S(k))
        u += (c * Sc + s * Ss) @ f / V
        # g_i = -(1/V) sum_k fhat k sum_j w_j sin(k.(x_i - x_j))
        sinterm = s * Sc - c * Ss                       # sum_j w_j sin(k.(x_i-x_j))
        g -= ((sinterm * f) @ kv) / V
    # remove the r = 0 term of the smooth part
    u -= beta ** 6 / 6.0 * w[tidx]
    return u, g


def exact_ewald(pos, c6, box, beta=None, tol=1e-16, chunk=2048):
    """E*, F*, and the per-atom potential u*_i = sum' xi_j r^-6 by Ewald."""
    xi = np.sqrt(np.asarray(c6, dtype=np.float64))
    u, g = ewald_field(pos, xi, box, beta, tol, chunk)
    E = -0.5 * float(np.dot(xi, u))
    return E, xi[:, None] * g, u


def exact_ewald_lb(pos, eps, sigma, box, beta=None, tol=1e-16):
    """E* and F* under Lorentz-Berthelot mixing (Sec. II.D): pair coefficient
    C_ij = 2 sqrt(eps_i eps_j) ((sigma_i + sigma_j) / 2)^6, written as the
    bilinear sum over the seven charge vectors
    xi_{i,k} = sigma_i^k sqrt(binom(6, k) 2 eps_i) / 8 paired k with 6 - k."""
    eps = np.asarray(eps, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    xi = [sigma ** k * np.sqrt(math.comb(6, k) * 2.0 * eps) / 8.0 for k in range(7)]
    fields = [ewald_field(pos, xi[m], box, beta, tol) for m in range(7)]
    E = 0.0
    F = np.zeros((len(eps), 3))
    for k in range(7):
        u, g = fields[6 - k]
        E += -0.5 * float(np.dot(xi[k], u))
        F += xi[k][:, None] * g
    return E, F


def exact_direct(pos, c6, box, R):
    """E* and F* by direct image summation to radius R (+ energy tail)."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    xi = np.sqrt(np.asarray(c6, dtype=np.float64))
    n = len(pos)
    V = float(np.prod(box))
    nr = np.ceil(R / box).astype(int) + 1
    u = np.zeros(n)
    F = np.zeros((n, 3))
    for nx in range(-nr[0], nr[0] + 1):
        for ny in range(-nr[1], nr[1] + 1):
            for nz in range(-nr[2], nr[2] + 1):
                s = np.array([nx, ny, nz]) * box
                d = pos[:, None, :] - pos[None, :, :] - s
                r2 = np.sum(d * d, axis=2)
                if nx == 0 and ny == 0 and nz == 0:
                    np.fill_diagonal(r2, np.inf)
                m = r2 <= R * R
                r2m = np.where(m, r2, 1.0)
                phi = np.where(m, r2m ** -3, 0.0)
                u += phi @ xi
                coef = np.where(m, -6.0 * r2m ** -4, 0.0) * xi[None, :]
                F += xi[:, None] * np.einsum("ij,ijk->ik", coef, d)
    u += 4.0 * math.pi / (3.0 * V * R ** 3) * np.sum(xi)
    E = -0.5 * float(np.dot(xi, u))
    return E, F, u
