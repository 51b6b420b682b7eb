"""Host-side pins of the operator-quality helpers (Sec. 7): minimal-image distances against brute
force, and the decay fit on an exact exponential profile.  The defect measures themselves are
checked on the GPU against dense oracle matrices (tests/test_gpu_quality.py)."""

import numpy as np

from paper_1701_00726_amd import quality


def test_distances_brute_force():
    L = (4, 6, 2, 8)
    r = quality.distances(L)
    for t in range(L[3]):
        for z in range(L[2]):
            for y in range(L[1]):
                for x in range(L[0]):
                    s = x + L[0] * (y + L[1] * (z + L[2] * t))
                    want = min(
                        np.sqrt((x - L[0] * a) ** 2 + (y - L[1] * b) ** 2 + (z - L[2] * c) ** 2 + (t - L[3] * d) ** 2)
                        for a in (0, 1) for b in (0, 1) for c in (0, 1) for d in (0, 1))
                    assert abs(r[s] - want) < 1e-12


def test_decay_rate_recovers_exponential():
    L = (8, 8, 8, 16)
    r = quality.distances(L)
    mag = 3.0 * np.exp(-0.7 * r)
    assert abs(quality.decay_rate(r, mag) - 0.7) < 1e-10
