"""Measured arithmetic ceilings (mp_measure_rate) on the GPU: plausible magnitudes and the
ordering the operation counts imply."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_rates_are_plausible():
    from paper_2412_17510_amd import mp
    fma = mp.mp_measure_rate(0)
    # binary64 FMA lane-instructions per second: within (5 %, 110 %] of 256 CUs x 64 lanes x 2.4 GHz
    assert 0.05 * 39.3e12 < fma <= 1.1 * 39.3e12
    dd, td, qd = (mp.mp_measure_rate(K) for K in (2, 3, 4))
    # DD's step is ~20 binary64 instructions, TD's and QD's ~200
    assert fma / 40 < dd < fma / 10
    assert fma / 400 < td < fma / 100 and fma / 400 < qd < fma / 100
    assert dd > 5 * td and dd > 5 * qd


def test_measure_rate_rejects_bad_kind():
    from paper_2412_17510_amd import mp
    with pytest.raises(Exception):
        mp.mp_measure_rate(1)
