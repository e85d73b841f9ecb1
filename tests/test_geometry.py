"""Pins of the detector geometry reading (36 sectors x 152 pad rows).

Closed forms: pad totals, exact fixed-point tables, pitch range, and the
agreement of the generator's and the oracle's independent geometry code.
"""
import math
from fractions import Fraction

import numpy as np

import oracle
import tpcsynth


def test_pad_totals_closed_form():
    npads, xfx, pfx = oracle.geometry()
    assert npads[0] == 66 and npads[151] == 138
    assert int(npads.sum()) == 15504
    assert 36 * int(npads.sum()) == 558144
    assert np.all(np.diff(npads) >= 0)


def test_fixed_point_rows_exact():
    npads, xfx, pfx = oracle.geometry()
    for r in range(152):
        x = Fraction(85) + Fraction(160 * r, 151)
        exact = x * 65536
        # round half up of an exact rational
        assert xfx[r] == math.floor(exact + Fraction(1, 2))
        assert xfx[r] < 2 ** 24  # exact in FP32
        n = Fraction(66) + Fraction(72 * r, 151)
        assert npads[r] == math.floor(n + Fraction(1, 2))


def test_pitch_range_and_tiling():
    npads, xfx, pfx = oracle.geometry()
    pitch = pfx / 65536.0
    assert 0.454 <= pitch.min() <= 0.455 and 0.625 <= pitch.max() <= 0.627
    x = 85.0 + np.arange(152) * 160.0 / 151.0
    # the pad plane spans the full +-10 degree sector to within the rounding
    assert np.all(np.abs(npads * pitch - 2 * x * math.tan(math.radians(10))) <= npads * 2.0 ** -17)


def test_generator_geometry_matches_oracle():
    x, pitch, npads_g = tpcsynth.geometry()
    npads, xfx, pfx = oracle.geometry()
    assert np.array_equal(npads, npads_g)
    assert np.all(np.abs(x * 65536 - xfx) <= 0.5)
    assert np.all(np.abs(pitch * 65536 - pfx) <= 0.5)
