"""Write bicgstab_counts_20cube.json: the iteration counts the oracle's
unpreconditioned BiCGStab (§3.1.2) needs to reach a 1e-6 relative residual on
the 20^3 instance-1 scatterer problem, for the unperturbed source and for 30
seeded perturbations f (1 + 1e-15 g), g standard normal.

Unpreconditioned BiCGStab on this indefinite operator amplifies rounding
differences by a large factor per iteration, so the count to tolerance is a
spread of values rather than one number; the GPU's count is compared with
this spread (within 2 of its range).  Calls only the oracle and the seeded
input generators.  Run: python tests/golden/make_bicgstab_counts.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2405_12380_amd import inputs as I  # noqa: E402
from oracle import operator as op_or, meta as meta_or  # noqa: E402

N, INSTANCE, TOL, PERTURB, COUNT, SEED = 20, 1, 1e-6, 1e-15, 30, 0


def main():
    C = I.config2(INSTANCE, n=(N, N, N))
    s = op_or.coefficient(C["ksq"], C["alpha"])

    def count(f):
        return int(meta_or.krylov_meta("bicgstab", f, np.zeros_like(f), s, C["mask"], 50, TOL, 5000)[1]["iters"])

    counts = [count(C["f"])]
    g = np.random.default_rng(SEED)
    for _ in range(COUNT):
        counts.append(count(C["f"] * (1 + PERTURB * g.standard_normal(C["f"].shape))))
    out = dict(problem=f"config2 instance {INSTANCE}, {N}^3", tol=TOL, perturbation=PERTURB, seed=SEED,
               unperturbed=counts[0], counts=counts, min=min(counts), max=max(counts))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bicgstab_counts_20cube.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path, out["min"], out["max"])


if __name__ == "__main__":
    main()
