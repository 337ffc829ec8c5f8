"""Writes helix_L20_d4.json: the oracle's folding statistic for the paper's alpha-helix
deck (Fig. 3b) in its own box, L = 20 (24 000 beads).

For each seed the deck is stepped 4000 times at dt = 0.02 by the FP64 oracle, and the mean
i -> i+4 distance of the 60-bead chain is averaged over the samples at steps 2250, 2500, ...,
4000.  The GPU test compares its own ensemble of the same seeds against these values; running
the oracle there would take minutes per seed.

Run from the repository root:  python tests/golden/make_helix_L20.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1804_06205_amd import analysis as A  # noqa: E402
from paper_1804_06205_amd import workloads as W  # noqa: E402

SEEDS = tuple(range(21, 33))
BLOCK, NBLOCKS, FIRST_SAMPLED = 250, 16, 8


def late_d4(seed):
    w = W.helix(L=20.0, seed=seed)
    st = oracle.State.from_workload(w)
    out = []
    for blk in range(NBLOCKS):
        st.step(BLOCK)
        if blk >= FIRST_SAMPLED:
            out.append(A.helix_profile(st.pos, w.L)["d4"])
    return float(np.mean(out))


def main():
    oracle.lib()
    vals = {}
    for s in SEEDS:
        t = time.time()
        vals[str(s)] = late_d4(s)
        print(f"seed {s}: d4 {vals[str(s)]:.4f} ({time.time() - t:.0f} s)", flush=True)
    v = np.array(list(vals.values()))
    doc = {
        "_source": "Written by tests/golden/make_helix_L20.py, which calls only the FP64 oracle. "
                   "Deck: workloads.helix(L=20, seed) (Fig. 3b), 4000 steps at dt = 0.02; value: "
                   "mean i->i+4 distance of the chain averaged over steps 2250..4000 every 250.",
        "block": BLOCK, "nblocks": NBLOCKS, "first_sampled_block": FIRST_SAMPLED,
        "late_d4": vals,
        "mean": float(v.mean()),
        "seed_sd": float(v.std(ddof=1)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "helix_L20_d4.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(f"mean {doc['mean']:.4f} sd {doc['seed_sd']:.4f} -> {path}")


if __name__ == "__main__":
    main()
