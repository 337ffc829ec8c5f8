"""Host-side statistics of read-back states.

Chain geometry of the paper's alpha-helix model (the protein section, Figs. 3-5): in a helix the
1-5 Morse term pulls bead i towards bead i+4, so the mean distances between beads i and i+k
(k = 2, 3, 4) and the share of i -> i+4 contacts near the 1-5 rest length track the chain's
folding.  These work on positions from dpd_get_state (tag order) and take no part in stepping.
"""
from __future__ import annotations

import numpy as np


def chain_distances(pos, L, first: int, nbeads: int, k: int) -> np.ndarray:
    """Minimum-image distances |x_i - x_{i+k}| along the chain of tags
    [first, first + nbeads)."""
    x = np.asarray(pos, dtype=np.float64)[first:first + nbeads]
    L = np.asarray(L, dtype=np.float64)
    d = x[k:] - x[:-k]
    d -= L * np.rint(d / L)
    return np.sqrt((d * d).sum(axis=1))


def helix_profile(pos, L, first: int = 0, nbeads: int = 60, contact=(0.45, 0.75)) -> dict:
    """Mean i -> i+2, i+3, i+4 distances and the fraction of i -> i+4 distances
    inside `contact` (around the 1-5 rest length 0.6 of the helix deck)."""
    d2 = chain_distances(pos, L, first, nbeads, 2)
    d3 = chain_distances(pos, L, first, nbeads, 3)
    d4 = chain_distances(pos, L, first, nbeads, 4)
    return {"d2": float(d2.mean()), "d3": float(d3.mean()), "d4": float(d4.mean()),
            "contact14": float(np.mean((d4 > contact[0]) & (d4 < contact[1])))}
