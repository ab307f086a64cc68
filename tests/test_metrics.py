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


def _dense_match(true_ev, inf_ev, dt, tt):
    """The matching rule written out over every pair (the definition)."""
    tx, ty, tn = (np.asarray(true_ev[f], dtype=float) for f in ("x", "y", "t"))
    ix, iy, inn = (np.asarray(inf_ev[f], dtype=float) for f in ("x", "y", "t"))
    taken = np.zeros(len(ix), dtype=bool)
    pairs = []
    for a in np.lexsort((np.arange(len(tx)), tn)):
        best, bi = np.inf, -1
        for b in range(len(ix)):
            if taken[b]:
                continue
            d = np.hypot(ix[b] - tx[a], iy[b] - ty[a])
            s = max(d / dt, abs(inn[b] - tn[a]) / tt)
            if s < best:
                best, bi = s, b
        if bi >= 0:
            d = np.hypot(ix[bi] - tx[a], iy[bi] - ty[a])
            if d < dt and abs(inn[bi] - tn[a]) < tt:
                pairs.append((int(a), bi))
                taken[bi] = True
    return pairs


def test_match_equals_the_pairwise_definition():
    """Random clustered sets (many near-ties, events at the thresholds'
    edges, duplicated onsets): the windowed matcher gives the pairs the
    all-pairs rule gives."""
    rng = np.random.default_rng(7)
    for trial in range(40):
        nt, ni = rng.integers(0, 30), rng.integers(0, 40)
        tx = rng.random(nt); ty = rng.random(nt); tn = np.round(rng.random(nt) * 80)
        base = rng.integers(0, max(nt, 1), ni)
        ix = (tx[base] if nt else rng.random(ni)) + rng.normal(0, 0.08, ni)
        iy = (ty[base] if nt else rng.random(ni)) + rng.normal(0, 0.08, ni)
        inn = (tn[base] if nt else rng.random(ni) * 80) + np.round(rng.normal(0, 8, ni))
        if trial % 5 == 0 and ni:  # exactly at the time threshold
            inn[0] = (tn[base[0]] if nt else 0.0) + 12.0
        tru = {"x": tx, "y": ty, "t": tn}
        inf = {"x": ix, "y": iy, "t": inn}
        want = _dense_match(tru, inf, 0.12, 12.0)
        assert M.match(tru, inf).pairs == want, trial
        for go in (M._match_dense, M._match_windowed):
            if len(tx) and len(ix):
                pairs, dists = [], []
                go(tx, ty, tn, ix, iy, inn, 0.12, 12.0, pairs, dists)
                assert pairs == want, (trial, go.__name__)


def test_match_states_equals_match_per_state():
    """The side-by-side matching of many states (padding, ties, states left
    empty, blocks split across the states) against `match` state by state."""
    rng = np.random.default_rng(11)
    nt = 25
    tru = {"x": rng.random(nt), "y": rng.random(nt), "t": np.round(rng.random(nt) * 200)}
    states = []
    for q in range(60):
        n = 0 if q % 17 == 0 else int(rng.integers(1, 40))
        base = rng.integers(0, nt, n)
        states.append({"x": tru["x"][base] + rng.normal(0, 0.06, n),
                       "y": tru["y"][base] + rng.normal(0, 0.06, n),
                       "t": tru["t"][base] + np.round(rng.normal(0, 6, n))})
    for chunk in (1 << 22, 3000):
        idx = M.match_states(tru, states, chunk_elems=chunk)
        for q, st in enumerate(states):
            got = [(a, int(idx[q, a])) for a in np.lexsort((np.arange(nt), tru["t"]))
                   if idx[q, a] >= 0]
            assert sorted(got) == sorted(M.match(tru, st).pairs), (chunk, q)
