"""Host logic of the probe-mode count rule (Section II, after Eq. 6): add
modes while each carries at least 1% of the total intensity."""
import pytest

from paper_1808_10375_amd import modes


def test_mode_fractions_sum_to_one_and_keep_ratios():
    f = modes.mode_fractions([4.0, 2.0, 1.0, 1.0])
    assert f == [0.5, 0.25, 0.125, 0.125]
    assert modes.mode_fractions([0.0, 0.0]) == [0.0, 0.0]


def test_search_stops_at_the_first_mode_under_one_percent():
    weights = [1.0, 0.3, 0.05, 0.004, 0.002]   # shares of the 4th: 0.3%
    calls = []

    def run(m):
        calls.append(m)
        return weights[:m]

    m, hist = modes.choose_mode_count(run, max_modes=5)
    assert m == 3 and calls == [1, 2, 3, 4]
    assert [h[0] for h in hist] == [1, 2, 3, 4]
    assert min(hist[-1][1]) < 0.01 <= min(hist[-2][1])


def test_search_keeps_the_maximum_when_every_mode_counts():
    m, hist = modes.choose_mode_count(lambda k: [1.0] * k, max_modes=4)
    assert m == 4 and len(hist) == 4


def test_threshold_and_bad_runs():
    # a 2% mode passes the paper's 1% but not a 5% threshold
    run = lambda k: [1.0, 0.02][:k]   # noqa: E731
    assert modes.choose_mode_count(run, 2)[0] == 2
    assert modes.choose_mode_count(run, 2, threshold=0.05)[0] == 1
    with pytest.raises(ValueError):
        modes.choose_mode_count(lambda k: [1.0], 2)
    with pytest.raises(ValueError):
        modes.choose_mode_count(run, 0)
