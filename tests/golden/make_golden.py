"""Write oracle reference values for full-size workloads (sampled outputs).

Calls only the oracle (``oracle.mls``) on the seeded inputs of
``paper_1308_4005_amd.workloads`` and stores the energy and the forces,
potentials and dE/dC6 of a seeded sample of atoms, so GPU tests and the
benchmark can check full-size runs without re-running the slow oracle.

    python tests/golden/make_golden.py cube1M_a3_h1_p4_l5 [...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import mls as M  # noqa: E402
from paper_1308_4005_amd import workloads as W  # noqa: E402

SPECS = {
    # name: (workload, a, h, order, levels)
    "slab32k_a3_h1_p4_l4": ("slab32k", 3.0, 1.0, 4, 4),
    "mixture100k_a3_h1_p4_l0": ("mixture100k", 3.0, 1.0, 4, 0),
}


def _tag(x):
    return f"{x:g}".replace(".", "p")


# the precision-at-scale sweep: 10^6 atoms, a in {2.5, 3, 4}, h in {0.8, 1,
# 1.25}, p in {4, 6}, five levels
for _a in (2.5, 3.0, 4.0):
    for _h in (0.8, 1.0, 1.25):
        for _p in (4, 6):
            SPECS[f"cube1M_a{_tag(_a)}_h{_tag(_h)}_p{_p}_l5"] = ("cube1M", _a, _h, _p, 5)
NSAMPLE = 512


def make(name):
    wname, a, h, order, levels = SPECS[name]
    w = W.named(wname)
    t0 = time.time()
    r = M.mls(w.pos, w.c6, w.box, a, h, order, levels)
    dt = time.time() - t0
    rng = np.random.Generator(np.random.PCG64(12345))
    idx = np.sort(rng.choice(w.n, size=min(NSAMPLE, w.n), replace=False))
    out = dict(
        workload=wname, n=w.n, box=w.box.tolist(), a=a, h=h, order=order, levels=int(r["levels"]),
        grid=[int(x) for x in r["n1"]], energy=r["energy"], sample=idx.tolist(),
        forces=r["F"][idx].tolist(), potential=r["u"][idx].tolist(), dE_dc6=r["dE_dc6"][idx].tolist(),
        force_rms=float(np.sqrt(np.mean(np.sum(r["F"] ** 2, axis=1)))),
        grid_sums=[float(q.sum()) for q in r["q"]],
        oracle_seconds=dt,
        source="oracle.mls (FP64 numpy) on the seeded workload; written by tests/golden/make_golden.py",
    )
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{name}: E={r['energy']:.15e} oracle {dt:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(SPECS):
        make(nm)
