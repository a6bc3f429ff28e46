"""The interval formulas of the distributional tests against the worked
examples of Newcombe (Statistics in Medicine 17, 1998): single proportions
(the score interval without continuity correction) and a difference of two
independent proportions (the hybrid score method)."""
import pytest

from stats_util import newcombe_diff, wilson


@pytest.mark.parametrize("k,n,lo,hi", [(81, 263, 0.2553, 0.3662), (15, 148, 0.0624, 0.1605),
                                       (0, 20, 0.0, 0.1611), (1, 29, 0.0061, 0.1718)])
def test_wilson_worked_examples(k, n, lo, hi):
    a, b = wilson(k, n)
    assert a == pytest.approx(lo, abs=5e-5) and b == pytest.approx(hi, abs=5e-5)


def test_newcombe_difference_worked_example():
    a, b = newcombe_diff(56, 70, 48, 80)
    assert a == pytest.approx(0.0524, abs=5e-5) and b == pytest.approx(0.3339, abs=5e-5)


def test_difference_interval_symmetry_and_zero():
    a, b = newcombe_diff(300, 1000, 300, 1000)
    assert a < 0 < b and a == pytest.approx(-b, abs=1e-12)
    c, d = newcombe_diff(48, 80, 56, 70)
    e, f = newcombe_diff(56, 70, 48, 80)
    assert c == pytest.approx(-f) and d == pytest.approx(-e)
