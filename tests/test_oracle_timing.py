"""Host logic of the oracle's timing helpers (no oracle runs)."""
import pytest

from oracle.timing import fit_rows, fitted_time


def test_fit_recovers_a_per_call_plus_per_row_cost():
    fixed, per_row, H = 1.25, 0.004, 1080
    t = lambda n: fixed + per_row * n
    assert fitted_time(t(1), 1, t(67), 67, H) == pytest.approx(t(H), rel=1e-12)
    # a sample that is the whole level returns its own measured time
    assert fitted_time(t(3), 3, t(H), H, H) == pytest.approx(t(H), rel=1e-12)


def test_fit_clamps_noise_to_non_negative_parts():
    # the larger call measured faster than the smaller one: no negative cost
    assert fitted_time(2.0, 1, 1.9, 8, 135) == pytest.approx(2.0)
    # degenerate row counts fall back to scaling the single measurement
    assert fitted_time(1.0, 4, 1.0, 4, 40) == pytest.approx(10.0)


@pytest.mark.parametrize("H", [48, 135, 270, 540, 1080])
def test_fit_rows_are_in_range_and_distinct(H):
    small, big = fit_rows(H)
    assert small == [H // 2]
    assert len(big) == max(3, H // 16)
    assert big == sorted(set(big)) and big[0] == 0 and big[-1] == H - 1
