"""Host-side chain statistics against closed forms."""
import math

import numpy as np

from paper_1804_06205_amd import analysis as A


def test_ideal_helix_distances():
    # Beads on a helix of radius R, turn angle t and rise p per bead:
    # |x_i - x_{i+k}|^2 = 2 R^2 (1 - cos(k t)) + (k p)^2.
    R, t, p, n = 0.35, 2 * math.pi / 3.6, 0.15, 60
    i = np.arange(n)
    pos = np.stack([R * np.cos(i * t), R * np.sin(i * t), i * p], axis=1) + 5.0
    prof = A.helix_profile(pos, (20.0, 20.0, 20.0), 0, n)
    for k in (2, 3, 4):
        exp = math.sqrt(2 * R * R * (1 - math.cos(k * t)) + (k * p) ** 2)
        assert abs(prof[f"d{k}"] - exp) < 1e-12
    d4 = math.sqrt(2 * R * R * (1 - math.cos(4 * t)) + (4 * p) ** 2)
    assert prof["contact14"] == (1.0 if 0.45 < d4 < 0.75 else 0.0)


def test_minimum_image_across_the_box():
    pos = np.array([[0.1, 0.0, 0.0], [9.9, 0.0, 0.0], [9.5, 0.0, 0.0]])
    d = A.chain_distances(pos, (10.0, 10.0, 10.0), 0, 3, 1)
    np.testing.assert_allclose(d, [0.2, 0.4], atol=1e-12)
    d2 = A.chain_distances(pos, (10.0, 10.0, 10.0), 0, 3, 2)
    np.testing.assert_allclose(d2, [0.6], atol=1e-12)
