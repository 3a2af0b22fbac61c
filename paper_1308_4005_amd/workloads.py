"""Seeded synthetic particle configurations shaped like the paper's LJ workloads.

The paper's test systems (Sec. III.A) are Lennard-Jones liquids: a slab whose
liquid fills a quarter of an elongated periodic box, cubes of the same side at
two densities, their scaled-up versions, and an equimolar two-species mixture.
The actual minimised configurations are not published, so this module builds
stand-ins with the same shapes, sizes and density structure by random
sequential addition (RSA): uniform proposals inside a target region, accepted
in proposal order when the periodic minimum-image distance to every accepted
atom is at least ``dmin``.

This module holds no part of the summation method: it only places atoms and
assigns C6 factors.  Both the GPU library's tests and the CPU oracle's tests
take their inputs from here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "rsa_fill", "cube", "slab", "mixture_slab", "batch_boxes",
    "named", "NAMED",
]


@dataclasses.dataclass
class Workload:
    """One periodic system: positions (N,3) float64, C6 (N,) float64, box (3,)."""
    name: str
    pos: np.ndarray
    c6: np.ndarray
    box: np.ndarray
    params: dict            # suggested MLS parameters: a, h, order, levels

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


class _Occupancy:
    """Cell hash whose cells are small enough to hold at most one accepted atom.

    The hash carries a periodic ghost layer ``reach`` cells wide, so the cells
    around any proposal are one gather at fixed flat offsets.
    """

    def __init__(self, box, dmin, capacity):
        self.box = np.asarray(box, dtype=np.float64)
        self.dmin = float(dmin)
        s = 0.999 * dmin / math.sqrt(3.0)
        self.g = np.maximum(1, np.ceil(self.box / s).astype(np.int64))
        self.cs = self.box / self.g
        self.reach = np.ceil(dmin / self.cs).astype(np.int64)
        self.gp = self.g + 2 * self.reach
        self.occ = np.full(int(np.prod(self.gp)), -1, dtype=np.int64)
        self.pos = np.empty((capacity, 3), dtype=np.float64)
        self.count = 0
        rx, ry, rz = (np.arange(-r, r + 1) for r in self.reach)
        ox, oy, oz = np.meshgrid(rx, ry, rz, indexing="ij")
        offs = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=1)
        gap = np.maximum(np.abs(offs) - 1, 0) * self.cs
        offs = offs[np.einsum("ij,ij->i", gap, gap) < dmin * dmin]
        self.offs_flat = (offs[:, 2] * self.gp[1] + offs[:, 1]) * self.gp[0] + offs[:, 0]
        sh = np.array([-1, 0, 1])
        sx, sy, sz = np.meshgrid(sh, sh, sh, indexing="ij")
        self.images = np.stack([sx.ravel(), sy.ravel(), sz.ravel()], axis=1)

    def cell3(self, p):
        c = np.floor(p / self.cs).astype(np.int64)
        return np.minimum(np.maximum(c, 0), self.g - 1)

    def pflat(self, c3):
        """Flat index into the padded hash of unpadded cell coordinates."""
        gp, r = self.gp, self.reach
        return ((c3[..., 2] + r[2]) * gp[1] + (c3[..., 1] + r[1])) * gp[0] + (c3[..., 0] + r[0])

    def conflicts_with_accepted(self, p):
        """Boolean per proposal: closer than dmin to an already accepted atom."""
        base = self.pflat(self.cell3(p))
        idx = self.occ[base[:, None] + self.offs_flat[None, :]]
        has = idx >= 0
        bad = np.zeros(p.shape[0], dtype=bool)
        if has.any():
            b, k = np.nonzero(has)
            d = p[b] - self.pos[idx[b, k]]
            d -= self.box * np.round(d / self.box)
            close = np.einsum("ij,ij->i", d, d) < self.dmin * self.dmin
            bad[b[close]] = True
        return bad

    def insert(self, p):
        c3 = self.cell3(p)
        n0 = self.count
        self.pos[n0:n0 + len(p)] = p
        ids = np.arange(n0, n0 + len(p))
        for im in self.images:
            q = c3 + im * self.g
            ok = np.all((q >= -self.reach) & (q < self.g + self.reach), axis=1)
            if ok.any():
                self.occ[self.pflat(q[ok])] = ids[ok]
        self.count += len(p)


def _resolve_within_batch(p, dmin, box):
    """Accept, in order, the proposals of one batch that clear each other."""
    m = len(p)
    if m <= 1:
        return np.ones(m, dtype=bool)
    # bucket the batch on a coarse hash to find close pairs
    cs = np.maximum(box / np.maximum(1, np.floor(box / dmin)), dmin)
    g = np.maximum(1, np.floor(box / cs).astype(np.int64))
    c3 = np.minimum(np.floor(p / (box / g)).astype(np.int64), g - 1)
    key = (c3[:, 2] * g[1] + c3[:, 1]) * g[0] + c3[:, 0]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    starts = np.searchsorted(ks, np.arange(int(np.prod(g)) + 1))
    earlier = [[] for _ in range(m)]
    found = False
    for ox in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for oz in (-1, 0, 1):
                nb = np.mod(c3 + np.array([ox, oy, oz]), g)
                nk = (nb[:, 2] * g[1] + nb[:, 1]) * g[0] + nb[:, 0]
                lo, hi = starts[nk], starts[nk + 1]
                cnt = hi - lo
                if cnt.max(initial=0) == 0:
                    continue
                src = np.repeat(np.arange(m), cnt)
                rel = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
                dst = order[np.repeat(lo, cnt) + rel]
                keep = dst < src
                src, dst = src[keep], dst[keep]
                d = p[src] - p[dst]
                d -= box * np.round(d / box)
                close = np.einsum("ij,ij->i", d, d) < dmin * dmin
                for s, t in zip(src[close], dst[close]):
                    earlier[s].append(t)
                    found = True
    ok = np.ones(m, dtype=bool)
    if found:
        for s in range(m):
            if earlier[s] and any(ok[t] for t in earlier[s]):
                ok[s] = False
    return ok


def rsa_fill(rng, occ: _Occupancy, n, sampler, batch=None):
    """Add ``n`` atoms by RSA with proposals drawn by ``sampler(rng, k)``."""
    target = occ.count + n
    while occ.count < target:
        need = target - occ.count
        k = batch or int(min(max(4 * need, 256), 65536))
        p = sampler(rng, k)
        p = np.mod(p, occ.box)
        p[p >= occ.box] = 0.0
        keep = ~occ.conflicts_with_accepted(p)
        p = p[keep]
        ok = _resolve_within_batch(p, occ.dmin, occ.box)
        p = p[ok][:need]
        occ.insert(p)
    return occ


def _uniform_box(lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)

    def sample(rng, k):
        return lo + (hi - lo) * rng.random((k, 3))
    return sample


def cube(n, density=0.8, seed=0, dmin=0.8, c6=4.0, params=None, name="cube"):
    """Homogeneous periodic cube of ``n`` atoms at ``density``."""
    L = (n / density) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    rng = np.random.Generator(np.random.PCG64(seed))
    occ = _Occupancy(box, dmin, n)
    rsa_fill(rng, occ, n, _uniform_box([0, 0, 0], box))
    pos = occ.pos[:occ.count].copy()
    return Workload(name, pos, np.full(n, float(c6)), box, dict(params or {}))


def cube_box(n, L, seed=0, dmin=0.8, c6=4.0, params=None, name="cube"):
    """Homogeneous periodic cube of side ``L`` holding ``n`` atoms."""
    return fill_box(n, (L, L, L), seed, dmin, c6, params, name)


def fill_box(n, box, seed=0, dmin=0.8, c6=4.0, params=None, name="box"):
    """Homogeneous periodic orthorhombic ``box`` holding ``n`` atoms."""
    box = np.array(box, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    occ = _Occupancy(box, dmin, n)
    rsa_fill(rng, occ, n, _uniform_box([0, 0, 0], box))
    pos = occ.pos[:occ.count].copy()
    return Workload(name, pos, np.full(n, float(c6)), box, dict(params or {}))


def slab(n, box, zlo, zhi, rho_liquid=0.8, rho_vapour=0.02, seed=0, dmin=0.8,
         c6=4.0, params=None, name="slab"):
    """Liquid layer in z in [zlo, zhi)*Lz at ``rho_liquid``; vapour elsewhere.

    The liquid is placed first, then the vapour.  Counts follow from the
    densities and the region volumes; the vapour count absorbs rounding so the
    total is exactly ``n``.  With ``rho_vapour = 0`` the liquid takes all ``n``.
    """
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    f = zhi - zlo
    if rho_vapour > 0:
        n_liq = int(round(rho_liquid * f * V))
        n_liq = min(n_liq, n)
    else:
        n_liq = n
    n_vap = n - n_liq
    rng = np.random.Generator(np.random.PCG64(seed))
    occ = _Occupancy(box, dmin, n)
    rsa_fill(rng, occ, n_liq,
             _uniform_box([0, 0, zlo * box[2]], [box[0], box[1], zhi * box[2]]))
    if n_vap:
        gap = (1.0 - f) * box[2]

        def vap(rng, k):
            p = rng.random((k, 3)) * np.array([box[0], box[1], gap])
            hi = p[:, 2] >= zlo * box[2]
            p[hi, 2] += f * box[2]
            return p
        rsa_fill(rng, occ, n_vap, vap)
    pos = occ.pos[:occ.count].copy()
    return Workload(name, pos, np.full(n, float(c6)), box, dict(params or {}))


def mixture_slab(n=100_000, box=(50.0, 50.0, 100.0), zlo=0.25, zhi=0.75,
                 c6_pair=(4.0, 9.0), seed=5, dmin=0.8, params=None,
                 name="mixture"):
    """Equimolar binary mixture in a liquid layer, empty elsewhere."""
    w = slab(n, box, zlo, zhi, rho_liquid=0.8, rho_vapour=0.0, seed=seed,
             dmin=dmin, params=params, name=name)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    species = np.zeros(n, dtype=np.int64)
    species[n // 2:] = 1
    species = rng.permutation(species)
    w.c6 = np.where(species == 0, c6_pair[0], c6_pair[1]).astype(np.float64)
    return w


def batch_boxes(nbox=256, seed=4, n_lo=500, n_hi=20000, dmin=0.8, c6=4.0,
                params=None):
    """Independent periodic boxes of uneven size, aspect ratio and density.

    Per box, in this order: N ~ floor(exp(U(ln n_lo, ln n_hi))),
    aspect alpha ~ U(1, 4), density rho ~ U(0.02, 0.85); box (L, L, alpha L)
    with L = (N / (rho alpha))^(1/3).  Positions of box b use seed 4000 + b.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(nbox):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        alpha = rng.uniform(1.0, 4.0)
        rho = rng.uniform(0.02, 0.85)
        L = (n / (rho * alpha)) ** (1.0 / 3.0)
        box = np.array([L, L, alpha * L])
        r2 = np.random.Generator(np.random.PCG64(4000 + b))
        occ = _Occupancy(box, dmin, n)
        rsa_fill(r2, occ, n, _uniform_box([0, 0, 0], box))
        out.append(Workload(f"batch{b}", occ.pos[:occ.count].copy(),
                            np.full(n, float(c6)), box, dict(params or {})))
    return out


def _c1():
    return cube_box(1000, 10.77, seed=1, params=dict(a=3.0, h=1.0, order=4, levels=2),
                    name="cube1k")


def _c2():
    # N and the two densities are kept; the box keeps the 1:1:4 shape.
    V = 32000 / (0.4 * 0.8 + 0.6 * 0.02)
    Lxy = (V / 4.0) ** (1.0 / 3.0)
    return slab(32000, (Lxy, Lxy, 4 * Lxy), 0.3, 0.7, seed=2,
                params=dict(a=3.0, h=1.0, order=4, levels=4), name="slab32k")


def _c3():
    return cube(1_000_000, 0.8, seed=3, params=dict(a=3.0, h=1.0, order=4, levels=5),
                name="cube1M")


def _c5():
    return mixture_slab(params=dict(a=3.0, h=1.0, order=4, levels=0))


NAMED = {"cube1k": _c1, "slab32k": _c2, "cube1M": _c3, "mixture100k": _c5}
NAMED_PARAMS = {"cube1k": dict(a=3.0, h=1.0, order=4, levels=2),
                "slab32k": dict(a=3.0, h=1.0, order=4, levels=4),
                "cube1M": dict(a=3.0, h=1.0, order=4, levels=5),
                "mixture100k": dict(a=3.0, h=1.0, order=4, levels=0)}


def named_batch(name: str = "batch256"):
    """The batched workload (256 boxes of ``batch_boxes`` with seed 4) as a
    list of Workloads, cached like ``named``."""
    import os
    if name != "batch256":
        raise KeyError(name)
    cache = os.environ.get("MLS_WORKLOAD_CACHE")
    path = os.path.join(cache, f"{name}.npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        off, boxes = z["off"], z["boxes"]
        return [Workload(f"batch{b}", z["pos"][off[b]:off[b + 1]], z["c6"][off[b]:off[b + 1]], boxes[b], {})
                for b in range(len(boxes))]
    ws = batch_boxes(256, seed=4)
    if path:
        os.makedirs(cache, exist_ok=True)
        off = np.concatenate([[0], np.cumsum([w.n for w in ws])])
        np.savez(path, pos=np.concatenate([w.pos for w in ws]), c6=np.concatenate([w.c6 for w in ws]),
                 boxes=np.stack([w.box for w in ws]), off=off)
    return ws


_MEMO = {}


def named(name: str) -> Workload:
    """Build one of the named workloads (see ``NAMED``).

    Generated arrays are kept for the life of the process (each call returns
    its own copies).  If the environment variable MLS_WORKLOAD_CACHE names a
    directory, they are also stored there and reused by later processes.
    """
    import os
    if name in _MEMO:
        wname, pos, c6, box, params = _MEMO[name]
        return Workload(wname, pos.copy(), c6.copy(), box.copy(), dict(params))
    w = _named_uncached(name)
    _MEMO[name] = (w.name, w.pos.copy(), w.c6.copy(), np.array(w.box, dtype=np.float64), dict(w.params))
    return w


def _named_uncached(name: str) -> Workload:
    import os
    cache = os.environ.get("MLS_WORKLOAD_CACHE")
    if cache:
        path = os.path.join(cache, f"{name}.npz")
        if os.path.exists(path):
            z = np.load(path, allow_pickle=False)
            return Workload(name, z["pos"], z["c6"], z["box"], NAMED_PARAMS.get(name, {}))
    w = NAMED[name]()
    if cache:
        os.makedirs(cache, exist_ok=True)
        np.savez(os.path.join(cache, f"{name}.npz"), pos=w.pos, c6=w.c6, box=w.box)
    return w
