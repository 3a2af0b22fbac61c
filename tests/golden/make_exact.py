"""Write exact periodic r^-6 forces for a sample of atoms (Ewald, oracle only).

The discretisation error of MLS (its output against the exact periodic sum,
Sec. II.A.1) is a property of a, h, the order and the density, not of the
system size (Sec. III.D); it is measured on a 32,000-atom cube with the
parameters of the 1M-atom workload.  The exact sum of a million atoms is out of
reach of a numpy Ewald, so the stored values cover this smaller cube.  Only
``oracle.exact`` is called; the atoms are the seeded cube of
``paper_1308_4005_amd.workloads``.

    python tests/golden/make_exact.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402
from paper_1308_4005_amd import workloads as W  # noqa: E402

N, RHO, SEED, NSAMPLE, BETA = 32000, 0.8, 31, 512, 0.25


def main():
    w = W.cube(N, RHO, seed=SEED)
    rng = np.random.Generator(np.random.PCG64(12345))
    idx = np.sort(rng.choice(w.n, size=NSAMPLE, replace=False))
    xi = np.sqrt(w.c6)
    t0 = time.time()
    u, g = exact.ewald_field(w.pos, xi, w.box, beta=BETA, targets=idx, chunk=64)
    dt = time.time() - t0
    F = xi[idx, None] * g
    out = dict(workload=f"cube{N // 1000}k", n=w.n, density=RHO, seed=SEED, box=w.box.tolist(),
               sample=idx.tolist(), forces=F.tolist(), potential=u.tolist(), beta=BETA,
               exact_seconds=dt,
               source="oracle.exact.ewald_field (FP64 Ewald, tol 1e-16) at the sampled atoms; "
                      "written by tests/golden/make_exact.py")
    path = os.path.join(HERE, f"cube{N // 1000}k_exact.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"exact forces of {NSAMPLE} atoms in {dt:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    main()
