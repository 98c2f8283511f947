"""Writes config1_targets.json: the 1D 5-moment workload's target moments.

Calls only the oracle (``oracle.workloads.config1_targets``) on the seeded
candidates of ``mem_inputs.config1_candidates``: per cell n ~ U(0.5, 2),
v ~ N(0, 1), T ~ U(0.5, 2) and the standardised Maxwellian's He_3 / He_4
multipliers perturbed by N(0, 0.05) (the He_4 one negative); candidates with
more than 1e-10 of their mass beyond |x| > 6 are skipped; the targets are the
64-node Gauss--Hermite moments (FP64) of the first 1024 kept densities, in the
gauge (v, sqrt T) of each cell.  The bench's 1D leg reads this file (it may not
call the oracle); the parity test recomputes the same targets itself.

Usage:
    python tests/golden/make_config1_targets.py
"""

import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mem_inputs  # noqa: E402
from oracle import workloads  # noqa: E402

CELLS = 1024


def main():
    M, g, b = workloads.config1_targets(mem_inputs.config1_candidates(4096), CELLS)
    with open(os.path.abspath(__file__), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out = dict(description="1D 5-moment MaxEnt targets (FP64, 64-node Gauss-Hermite) of "
                           "perturbed-multiplier densities, in each cell's gauge (v, sqrt T)",
               script="tests/golden/make_config1_targets.py", script_sha256=sha,
               cells=CELLS, M=M.tolist(), g=g.tolist(), beta_generating=b.tolist())
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_targets.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: {CELLS} cells")


if __name__ == "__main__":
    main()
