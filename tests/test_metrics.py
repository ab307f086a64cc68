"""Matching, scores and ESS (host metrics), pinned by hand-built cases and
the closed-form ESS of an AR(1) chain, n (1 - rho) / (1 + rho)."""
import numpy as np
import pytest

from paper_1612_00595_amd import metrics as M
from paper_1612_00595_amd.chromh import as_events


def ev(rows):
    rows = np.array(rows, dtype=np.float64).reshape(-1, 3)
    return as_events(rows[:, 0], rows[:, 1], rows[:, 2], np.full(len(rows), 3.0))


def test_identical_sets_match_perfectly():
    t = ev([[0.1, 0.2, 10], [0.5, 0.5, 300], [0.9, 0.1, 700]])
    r = M.match(t, t)
    assert (r.precision, r.recall, r.f1, r.location_error) == (1.0, 1.0, 1.0, 0.0)
    assert sorted(r.pairs) == [(0, 0), (1, 1), (2, 2)]


def test_thresholds_are_strict_in_space_and_time():
    t = ev([[0.5, 0.5, 100]])
    assert len(M.match(t, ev([[0.5 + 0.119, 0.5, 100]])).pairs) == 1
    assert len(M.match(t, ev([[0.5 + 0.121, 0.5, 100]])).pairs) == 0
    assert len(M.match(t, ev([[0.5, 0.5, 111.9]])).pairs) == 1
    assert len(M.match(t, ev([[0.5, 0.5, 112.1]])).pairs) == 0
    r = M.match(t, ev([[0.56, 0.58, 105]]))
    assert r.location_error == pytest.approx(0.1)


def test_greedy_visits_true_events_by_onset_time():
    # one inferred event between two true ones: the earlier true event takes it
    t = ev([[0.60, 0.5, 200], [0.50, 0.5, 100]])
    i = ev([[0.55, 0.5, 150]])
    r = M.match(t, i, time_thresh=60.0)
    assert r.pairs == [(1, 0)]
    assert r.precision == 1.0 and r.recall == 0.5


def test_closest_uses_the_larger_normalised_separation():
    t = ev([[0.5, 0.5, 100]])
    i = ev([[0.5, 0.5, 110], [0.55, 0.5, 101]])   # 10/12 vs max(0.05/0.12, 1/12)
    assert M.match(t, i).pairs == [(0, 1)]


def test_duplicates_cost_precision_and_empty_sets():
    t = ev([[0.5, 0.5, 100]])
    r = M.match(t, ev([[0.5, 0.5, 100], [0.51, 0.5, 101]]))
    assert (r.precision, r.recall) == (0.5, 1.0)
    assert r.f1 == pytest.approx(2 / 3)
    e = ev([])
    assert (M.match(e, e).precision, M.match(e, e).recall) == (1.0, 1.0)
    r = M.match(e, t)
    assert (r.precision, r.recall) == (0.0, 1.0)
    r = M.match(t, e)
    assert (r.precision, r.recall) == (1.0, 0.0)


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9, 0.98])
def test_ess_of_ar1_chain(rho):
    rng = np.random.default_rng(1)
    n = 200_000
    z = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = z[0] / np.sqrt(1 - rho ** 2)
    for q in range(1, n):
        x[q] = rho * x[q - 1] + z[q]
    want = n * (1 - rho) / (1 + rho)
    assert M.ess(x) == pytest.approx(want, rel=0.12)


def test_ess_degenerate_chains():
    assert M.ess(np.ones(1000)) == 1.0
    assert M.ess(np.arange(3.0)) == 3.0


def test_bootstrap_ci_covers_the_mean():
    v = np.random.default_rng(2).normal(5.0, 1.0, 400)
    mean, lo, hi = M.bootstrap_ci(v)
    assert lo < mean < hi
    assert hi - lo == pytest.approx(2 * 1.96 / np.sqrt(400), rel=0.25)


def test_location_ess_of_synthetic_chains():
    rng = np.random.default_rng(3)
    truth = ev([[0.3, 0.3, 100], [0.7, 0.6, 500]])
    n, rho = 4000, 0.8
    states = []
    ax = np.zeros(2)
    ay = np.zeros(2)
    for q in range(n):
        ax = rho * ax + 0.01 * rng.standard_normal(2)
        ay = rho * ay + 0.01 * rng.standard_normal(2)
        states.append(ev([[0.3 + ax[0], 0.3 + ay[0], 100], [0.7 + ax[1], 0.6 + ay[1], 500]]))
    e, k = M.location_ess(states, truth, burn_frac=0.0)
    assert k == 2
    assert e == pytest.approx(n * (1 - rho) / (1 + rho), rel=0.3)
