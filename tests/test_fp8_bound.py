"""An approximate e4m3 cross term cannot certify the masked-L2 optimum: on a
small RGB image, the rigorous bound of the e4m3 filter (per-patch scales)
leaves most of the dictionary inside even the exact optimum, so a
certificate would send every target to the float32 scan. CPU only (exact
emulation of e4m3 rounding in float64)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import fp8_bound_emulation as fe  # noqa: E402

from paper_1712_06326_amd import synth  # noqa: E402


def test_e4m3_rounding_matches_hand_values():
    x = np.array([0.0, 1.0, 1.0625, 1.125, 1.1875, 17.0, 19.0, 448.0, 2.0 ** -9, 3 * 2.0 ** -10,
                  -3.3])
    want = np.array([0.0, 1.0, 1.0, 1.125, 1.25, 16.0, 20.0, 448.0, 2.0 ** -9, 2.0 ** -8, -3.25])
    assert np.array_equal(fe.e4m3(x), want)


def test_e4m3_bound_lists_most_of_the_dictionary():
    d = synth.small_image(96, 110, 3, 41)
    counts, n, ratios = fe.listed_counts(d["volume"], d["mask"], 9, 6)
    assert np.all(counts > 0.3 * n), (counts, n)
    assert np.median(ratios) > 0.5
