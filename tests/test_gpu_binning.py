"""Linked-cell binning (Sec. III.D) through both sorts of the library: the
bucketed sort of single plans (buckets of 512..2048 consecutive cells; a
bucket of more than 4096 atoms takes the global-memory path) and the counting
sort with device-wide atomics (MLS_BIN_BUCKETS=0, and every batched plan).
The permutation and the cell starts must equal the oracle's stable counting
sort bit for bit."""
import os

import numpy as np
import pytest

from oracle import mls as M
from paper_1308_4005_amd import workloads as W

from gpu_common import gpu_eval, say, stages

pytestmark = pytest.mark.gpu

A, H, P = 3.0, 1.0, 4


def _uniform(n, box, seed, lo=None, hi=None):
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=float)
    lo = np.zeros(3) if lo is None else np.asarray(lo, dtype=float)
    hi = box if hi is None else np.asarray(hi, dtype=float)
    pos = lo + rng.random((n, 3)) * (hi - lo)
    # unwrapped copies: the binning wraps them itself
    pos += rng.integers(-1, 2, size=pos.shape) * box
    return W.Workload("uniform", pos, rng.uniform(1.0, 9.0, n), box, {})


CASES = [
    # 7^3 half-width cells, one bucket of 5000 atoms: the global-memory path
    ("one_bucket_overflow", lambda: _uniform(5000, (12.0, 12.0, 12.0), 1)),
    # a corner cluster: 8 cells hold every atom of the bucket
    ("corner_cluster", lambda: _uniform(4500, (12.0, 12.0, 12.0), 2, hi=(2.9, 2.9, 2.9))),
    # 11^3 cells: two full buckets and a ragged one of 307 cells
    ("ragged_last_bucket", lambda: _uniform(3000, (16.5, 16.5, 16.5), 3)),
    # 19^3 cells in 14 buckets, ten blocks of atoms per bucket histogram
    ("cube20k", lambda: W.cube(20000, 0.8, seed=4)),
    # exactly one block of atoms, a single atom in the last block
    ("block_edge", lambda: _uniform(2049, (15.0, 15.0, 15.0), 5)),
]


def _check(w, plan):
    st = stages(plan, w.n)
    half = 0.5 * A
    width = half if np.all(M.cells_per_dim(w.box, half) >= 5) else A
    nc, cid, start, perm = M.bin_cells(M.wrap(w.pos, w.box), w.box, width)
    assert tuple(plan.info["cells"]) == tuple(int(x) for x in nc)
    np.testing.assert_array_equal(st["cell_start"], start)
    np.testing.assert_array_equal(st["perm"], perm)
    return int(np.max(np.diff(start)))


@pytest.mark.parametrize("k", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bucketed_sort_is_the_stable_counting_sort(k, precision):
    name, make = CASES[k]
    w = make()
    say(f"[binning] {name} {precision}: n={w.n} box={w.box.tolist()}")
    plan, _ = gpu_eval(w.pos, w.c6, w.box, A, H, P, 2, precision=precision)
    mx = _check(w, plan)
    say(f"[binning] {name}: largest cell {mx}")
    plan.close()


@pytest.mark.parametrize("k", [0, 3], ids=[CASES[0][0], CASES[3][0]])
def test_counting_sort_with_atomics_agrees(k, monkeypatch):
    name, make = CASES[k]
    w = make()
    monkeypatch.setenv("MLS_BIN_BUCKETS", "0")
    assert os.environ["MLS_BIN_BUCKETS"] == "0"
    plan, out0 = gpu_eval(w.pos, w.c6, w.box, A, H, P, 2)
    _check(w, plan)
    plan.close()
    monkeypatch.delenv("MLS_BIN_BUCKETS")
    plan, out1 = gpu_eval(w.pos, w.c6, w.box, A, H, P, 2)
    _check(w, plan)
    plan.close()
    # the same permutation, so the same sums (up to the order of the FP64
    # atomics of the anterpolation)
    assert out0["energy"] == pytest.approx(out1["energy"], rel=1e-12)
    np.testing.assert_allclose(out0["F"], out1["F"], rtol=0, atol=1e-12 * np.max(np.abs(out1["F"])))
