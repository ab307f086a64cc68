"""Pins of the oracle's geometry, partition, likelihood and simulator.

Every check here compares the oracle with something other than itself:
values worked by hand from the paper's Figure 1, closed forms of the signal
model, scipy's Gaussian density, Monte Carlo geometry, or distribution tests
of simulated traces.
"""
import os

import numpy as np
import pytest
from scipy import stats

from paper_1612_00595_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def model_of(spec, orc):
    return orc.make_model(**spec.asdict())


# ------------------------------------------------------------- geometry

def test_fig1_travel_times(orc):
    rows = np.loadtxt(os.path.join(HERE, "golden", "fig1_travel_times.txt"))
    for t, x, xs, want in rows:
        got = orc.arrival_time(x, 0.0, t, xs, 0.0, 2.0)
        assert got == want


def test_region_axis_boundaries(orc):
    # region i covers [off + (i-1) w, off + i w); indices clamp to [0, g]
    assert orc.region_axis(0.0, 0.0, 0.25, 4) == 1
    assert orc.region_axis(np.nextafter(0.25, 0), 0.0, 0.25, 4) == 1
    assert orc.region_axis(0.25, 0.0, 0.25, 4) == 2
    assert orc.region_axis(np.nextafter(1.0, 0), 0.0, 0.25, 4) == 4
    assert orc.region_axis(0.05, 0.1, 0.2, 5) == 0
    assert orc.region_axis(0.1, 0.1, 0.2, 5) == 1
    assert orc.region_axis(0.35, 0.1, 0.2, 5) == 2
    assert orc.region_axis(5.0, 0.1, 0.2, 5) == 5


def test_small_static_partition_has_four_colours(orc):
    m = model_of(W.SMALL.model, orc)
    rc, nrx, nry, p, nc, color = orc.partition_and_color(m, 4, 4, 0.0, 0.0, 0)
    assert rc == 0 and (nrx, nry, p, nc) == (5, 5, 2, 4)
    assert orc.coloring_violations(m, 4, 4, 0.0, 0.0, 1) > 0
    # colour (i mod 2) + 2 (k mod 2), grid indexed [k, i]
    grid = color.reshape(5, 5)
    assert grid[1, 1] == 3 and grid[1, 2] == 2 and grid[2, 1] == 1 and grid[2, 2] == 0
    # a longer reach breaks the 2x2 pattern of 0.25-wide regions
    m2 = orc.make_model(**dict(W.SMALL.model.asdict(), rc=0.21))
    assert orc.coloring_violations(m2, 4, 4, 0.0, 0.0, 2) > 0
    rc, *_rest = orc.partition_and_color(m2, 4, 4, 0.0, 0.0, 0)
    assert rc == 0 and _rest[2] == 3


def test_dynamic_period_holds_for_all_offsets(orc):
    spec = W.ModelSpec(nsx=12, nsy=12, N=100, lam=10.0)
    m = model_of(spec, orc)
    rng = np.random.default_rng(0)
    fails2 = 0
    for _ in range(200):
        ox, oy = rng.random(2) * 0.2
        rc, nrx, nry, p, nc, color = orc.partition_and_color(m, 12, 12, ox, oy, 1)
        assert rc == 0 and p == 3 and nc == 9
        assert orc.coloring_violations(m, 12, 12, ox, oy, 3) == 0
        fails2 += orc.coloring_violations(m, 12, 12, ox, oy, 2) > 0
    assert fails2 >= 180


def test_coloring_invariant_monte_carlo(orc):
    """Independent of the rectangle-distance code: draw points in pairs of
    same-coloured regions and check that no station detects both."""
    spec = W.ModelSpec(nsx=8, nsy=8, N=100)
    m = model_of(spec, orc)
    rng = np.random.default_rng(7)
    st = (np.arange(8) + 0.5) * 0.2
    sx, sy = np.meshgrid(st, st)
    sx, sy = sx.ravel(), sy.ravel()
    for trial in range(20):
        ox, oy = rng.random(2) * 0.2
        rc, nrx, nry, p, nc, color = orc.partition_and_color(m, 8, 8, ox, oy, 1)
        pts = rng.random((20000, 2)) * 1.6
        # bias half the points onto region boundaries, where conflicts would appear
        edge = rng.integers(0, 9, size=(10000, 2)) * 0.2 + np.array([ox, oy])
        pts[:10000] = np.clip(edge + rng.normal(0, 0.003, (10000, 2)), 0, np.nextafter(1.6, 0))
        reg = np.array([orc.region_axis(x, ox, 0.2, 8) + 9 * orc.region_axis(y, oy, 0.2, 8)
                        for x, y in pts])
        col = color[reg]
        d = np.hypot(pts[:, None, 0] - sx[None], pts[:, None, 1] - sy[None])
        det = d < 0.19
        for j in range(64):
            who = np.nonzero(det[:, j])[0]
            for c in np.unique(col[who]):
                regs = np.unique(reg[who][col[who] == c])
                assert len(regs) == 1, (trial, j, c, regs)


# ------------------------------------------------------------ likelihood

def test_single_term_is_gaussian_logpdf(orc):
    for s, e in [(0.0, 0.0), (0.3, 0.0), (-1.2, 2.5), (4.0, 25.0), (1e-3, 1e-9)]:
        want = stats.norm.logpdf(s, loc=0.0, scale=np.sqrt(0.01 + e))
        assert orc.single_term(0.1, s, e) == pytest.approx(want, rel=1e-13, abs=1e-13)


def test_loglik_without_events_is_noise_density(orc):
    spec = W.ModelSpec(nsx=3, nsy=2, N=50)
    m = model_of(spec, orc)
    s = np.random.default_rng(3).normal(0, 0.2, (6, 50))
    want = stats.norm.logpdf(s, 0.0, 0.1).sum()
    assert orc.loglik(m, s, orc.events_array(0)) == pytest.approx(want, rel=1e-12)


def test_loglik_is_gaussian_with_model_variance(orc):
    spec = W.ModelSpec(nsx=3, nsy=3, N=400, lam=5.0)
    m = model_of(spec, orc)
    tr = W.truth_events(spec, 11, n=6)
    ev = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    s = np.random.default_rng(4).normal(0, 0.5, (9, 400))
    E = orc.event_variance(m, ev)
    want = stats.norm.logpdf(s, 0.0, np.sqrt(0.01 + E)).sum()
    assert orc.loglik(m, s, ev) == pytest.approx(want, rel=1e-12)


def test_envelope_closed_forms(orc):
    """One event at one station: support [ceil(a), ceil(a) + ts), value at
    onset A^2 exp(-2 f / decay), constant ratio exp(-2 / decay) between
    successive samples, and the geometric-series total."""
    spec = W.ModelSpec(nsx=1, nsy=1, N=400)
    m = model_of(spec, orc)
    x, y, t, mag = 0.1 + 0.06, 0.1 + 0.08, 37.3, 3.0
    ev = orc.as_events([x], [y], [t], [mag])
    E = orc.event_variance(m, ev)[0]
    d = 0.1  # 3-4-5 triangle: hypot(0.06, 0.08)
    a = t + d / 0.05
    n0 = int(np.ceil(a))
    assert n0 == 40
    nz = np.nonzero(E)[0]
    assert nz[0] == n0 and nz[-1] == n0 + 127
    A2 = (mag * np.exp(-d / 0.2)) ** 2
    f = n0 - a
    assert E[n0] == pytest.approx(A2 * np.exp(-2 * f / 20.0), rel=1e-12)
    r = E[n0 + 1:n0 + 128] / E[n0:n0 + 127]
    assert np.allclose(r, np.exp(-0.1), rtol=1e-12)
    total = A2 * np.exp(-2 * f / 20.0) * (1 - np.exp(-0.1) ** 128) / (1 - np.exp(-0.1))
    assert E.sum() == pytest.approx(total, rel=1e-12)


def test_detection_cutoff_and_additivity(orc):
    spec = W.ModelSpec(nsx=2, nsy=1, N=300)
    m = model_of(spec, orc)
    # station (0.1, 0.1): an event at distance 0.19 (cutoff) adds nothing
    far = orc.as_events([0.1 + 0.19], [0.1], [10.0], [5.0])
    E = orc.event_variance(m, far)
    assert E[0].sum() == 0.0 and E[1].sum() > 0.0
    near = orc.as_events([0.1 + 0.18999], [0.1], [10.0], [5.0])
    assert orc.event_variance(m, near)[0].sum() > 0.0
    # independent signals: variances add
    e1 = orc.as_events([0.12], [0.1], [10.0], [3.0])
    e2 = orc.as_events([0.2], [0.15], [60.0], [2.5])
    both = np.concatenate([e1, e2])
    assert np.allclose(orc.event_variance(m, both),
                       orc.event_variance(m, e1) + orc.event_variance(m, e2),
                       rtol=1e-14, atol=0)
    # an arrival after the end of the trace leaves the trace untouched
    late = orc.as_events([0.1], [0.1], [299.5], [4.0])
    assert orc.event_variance(m, late)[0][:299].sum() == 0.0


# ------------------------------------------------------------- simulator

def test_simulator_is_gaussian_with_model_variance(orc):
    spec = W.ModelSpec(nsx=3, nsy=3, N=300, lam=4.0)
    m = model_of(spec, orc)
    tr = W.truth_events(spec, 21, n=5)
    ev = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    v = 0.01 + orc.event_variance(m, ev)
    reps = np.stack([orc.simulate(m, ev, seed) for seed in range(120)])
    z = reps / np.sqrt(v)[None]
    assert stats.kstest(z.ravel()[::7], "norm").pvalue > 1e-3
    # per-sample variance: mean of z^2 over replicates is chi2(120)/120
    chi = (z ** 2).sum(axis=0).ravel()
    p = stats.chi2.sf(chi, 120)
    assert stats.kstest(p, "uniform").pvalue > 1e-3
    # the seeds give different noise, the same seed the same trace
    assert not np.array_equal(reps[0], reps[1])
    assert np.array_equal(reps[3], orc.simulate(m, ev, 3))
