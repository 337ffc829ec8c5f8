"""The paper's alpha-helix deck (Fig. 3b; 60 skeletal beads, modified Morse 1-3 and
1-5 terms, dt = 0.02) on the GPU against the oracle.

Trajectories of a chaotic system part ways after a few hundred steps, so what is compared is the
ensemble statistic the model is about: the mean i -> i+4 distance of the chain, which falls from
~1.07 (random walk) to ~0.5 as the 1-5 terms fold it, averaged over steps 2000-4000.

* L = 10, four seeds, both sides run here.  The per-seed spread of that average is 0.033 (oracle,
  8 seeds), so the two four-seed means differ by about 0.023 at one sigma; the bar is 0.08.
* L = 20 (the deck's own box, 24 000 beads), twelve seeds against the oracle's values stored in
  tests/golden/helix_L20_d4.json by tests/golden/make_helix_L20.py (the oracle takes ~45 s per
  seed there).  The bar is four sigma of the difference of two twelve-seed means, from the stored
  per-seed spread.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1804_06205_amd import analysis as A
from paper_1804_06205_amd import dpd
from paper_1804_06205_amd import workloads as W

pytestmark = pytest.mark.gpu

SEEDS = (21, 22, 23, 24)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dpd.lib()
    oracle.lib()


def _late_d4_gpu(w, block=250, nblocks=16, first=8):
    out = []
    with dpd.System.from_workload(w) as g:
        for blk in range(nblocks):
            g.step(block)
            if blk >= first:
                out.append(A.helix_profile(g.get_state(force=False)[0], w.L)["d4"])
    return float(np.mean(out))


def _late_d4_oracle(w):
    st = oracle.State.from_workload(w)
    out = []
    for blk in range(16):
        st.step(250)
        if blk >= 8:
            out.append(A.helix_profile(st.pos, w.L)["d4"])
    return float(np.mean(out))


def test_helix_deck_folds_like_the_oracle():
    ws = [W.helix(L=10.0, seed=s) for s in SEEDS]
    d4_0 = np.mean([A.helix_profile(w.pos, w.L)["d4"] for w in ws])
    g = np.array([_late_d4_gpu(w) for w in ws])
    o = np.array([_late_d4_oracle(w) for w in ws])
    print(f"d4 initial {d4_0:.3f}; GPU {g.round(3)} mean {g.mean():.3f}; "
          f"oracle {o.round(3)} mean {o.mean():.3f}", flush=True)
    assert d4_0 > 0.9
    assert g.mean() < 0.65 and o.mean() < 0.65          # both fold
    assert abs(g.mean() - o.mean()) < 0.08


def test_helix_deck_in_its_own_box_folds_like_the_oracle():
    path = os.path.join(os.path.dirname(__file__), "golden", "helix_L20_d4.json")
    with open(path) as f:
        gold = json.load(f)
    seeds = sorted(int(k) for k in gold["late_d4"])
    o = np.array([gold["late_d4"][str(s)] for s in seeds])
    g = np.array([_late_d4_gpu(W.helix(L=20.0, seed=s), gold["block"], gold["nblocks"],
                               gold["first_sampled_block"]) for s in seeds])
    bar = 4.0 * gold["seed_sd"] * math.sqrt(2.0 / len(seeds))
    print(f"L=20 d4: GPU mean {g.mean():.4f} (sd {g.std(ddof=1):.4f}); oracle mean "
          f"{o.mean():.4f} (sd {gold['seed_sd']:.4f}); bar {bar:.4f}", flush=True)
    assert g.mean() < 0.65 and o.mean() < 0.65
    assert abs(g.mean() - o.mean()) < bar
