"""Pins of the oracle's line model: the paper's own 1-D world (Section 3 as
printed) partitioned in onset time (Section 4.1).

- Figure 1's two events at the four stations: the variance each event adds
  is its constant signal variance exactly on [ceil(a), ceil(a) + t_s), with a
  the hand-worked arrival times of ``golden/fig1_travel_times.txt``;
- the log-likelihood of one event reduces to two Gaussian log densities (in
  and out of the boxcar), evaluated with scipy;
- the colouring check against brute force over onsets and locations: with
  l = 60, tau_max = 50 and t_s = 10 two colours separate the regions at
  every offset, with t_s = 11 they do not;
- every move's local likelihood change equals two full recomputations;
- with the likelihood off the chain samples the prior (Poisson count, uniform
  location and onset) under the static and the shifted time partition;
- on a small world the chromatic schedules (static and dynamic) agree with
  the serial chain in the posterior count and onset histogram;
- on a lattice line world the serial, chromatic-static and
  chromatic-dynamic chains match the brute-force enumerated posterior and
  the naive parallel schedule (Algorithm 3) does not.
"""
import dataclasses
import math
import os
from collections import Counter

import numpy as np
import pytest
from scipy import stats

from paper_1612_00595_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_travel_times.txt")


def line_model(orc, **kw):
    spec = dataclasses.replace(W.PAPER1D_MODEL, **kw)
    return spec, orc.make_model(**spec.asdict())


def line_sampler(orc, **kw):
    return orc.make_sampler(**dict(W.PAPER1D_SAMPLER.asdict(), **kw))


def fig1():
    rows = np.loadtxt(GOLDEN, comments="#")
    return rows  # event_t event_x station_x arrival


def test_fig1_windows_and_boxcar(orc):
    spec, m = line_model(orc)
    rows = fig1()
    for t, x in {(r[0], r[1]) for r in rows}:
        ev = orc.as_events([x], [0.0], [t], [spec.mmin])
        E = orc.event_variance(m, ev)
        for j, sx in enumerate(spec.sta_x):
            a = rows[(rows[:, 0] == t) & (rows[:, 1] == x) & (rows[:, 2] == sx)][0, 3]
            n0 = math.ceil(a)
            want = np.zeros(spec.N)
            want[n0:min(n0 + spec.ts, spec.N)] = spec.mmin ** 2
            assert np.array_equal(E[j], want), (t, x, sx)


def test_single_event_loglik_closed_form(orc):
    spec, m = line_model(orc)
    rows = fig1()
    rng = np.random.default_rng(4)
    s = rng.normal(0.0, 1.5, (spec.nsta, spec.N))
    t, x = rows[0, 0], rows[0, 1]
    ev = orc.as_events([x], [0.0], [t], [spec.mmin])
    want = 0.0
    for j in range(spec.nsta):
        a = rows[(rows[:, 0] == t) & (rows[:, 2] == spec.sta_x[j])][0, 3]
        inside = np.zeros(spec.N, dtype=bool)
        inside[math.ceil(a):math.ceil(a) + spec.ts] = True
        sd = np.where(inside, math.hypot(spec.sigma, spec.mmin), spec.sigma)
        want += stats.norm.logpdf(s[j], 0.0, sd).sum()
    assert orc.loglik(m, s, ev) == pytest.approx(want, rel=1e-12)
    # prior: Poisson count times uniform location and onset
    assert orc.logprior(m, ev) == pytest.approx(
        -spec.lam + math.log(spec.lam) - math.log(spec.xmax) - math.log(spec.N), rel=1e-14)


def _touched(spec, x, t):
    """Samples an event at (x, t) touches at any station: set of (j, n)."""
    out = set()
    for j, sx in enumerate(spec.sta_x):
        n0 = math.ceil(t + abs(x - sx) / spec.vel)
        out.update((j, n) for n in range(max(n0, 0), min(n0 + spec.ts, spec.N)))
    return out


def _brute_conflict(spec, gx, off, p):
    """Whether two same-coloured regions have events touching a common
    sample, over a grid of onsets (each region's ends approached from
    inside) and locations (including both ends of the line)."""
    w = spec.N / gx
    xs = np.concatenate([np.linspace(0, spec.xmax, 21)[:-1], [np.nextafter(spec.xmax, 0)]])
    cover = []
    for i in range(gx + 1):
        t0, t1 = max(off + (i - 1) * w, 0.0), min(off + i * w, float(spec.N))
        if not t1 > t0:
            cover.append(set())
            continue
        ts = np.concatenate([np.linspace(t0, t1, 13)[:-1], [np.nextafter(t1, t0)]])
        cov = set()
        for t in ts:
            for x in xs:
                cov |= _touched(spec, x, t)
        cover.append(cov)
    for a in range(gx + 1):
        for b in range(a + 1, gx + 1):
            if a % p == b % p and cover[a] & cover[b]:
                return True
    return False


@pytest.mark.parametrize("ts,expect_ok", [(10, True), (11, False)])
def test_colouring_check_against_brute_force(orc, ts, expect_ok):
    spec, m = line_model(orc, ts=ts)
    assert orc.line_tau_max(m) == pytest.approx(50.0)
    rng = np.random.default_rng(9)
    offs = [0.0] + list(rng.random(12) * 60.0)
    for off in offs:
        viol = orc.coloring_violations(m, 4, 0, off, 0.0, 2)
        brute = _brute_conflict(spec, 4, off, 2)
        if viol == 0:
            assert not brute, off
        if expect_ok:
            assert viol == 0, off
    if not expect_ok:
        # the conflict is real: an event ending region 1 and one opening region 3
        assert _brute_conflict(spec, 4, 0.0, 2)
        rc, *_ = orc.partition_and_color(m, 4, 0, 0.0, 0.0, 1)
        assert rc == 0  # a dynamic partition then takes three colours
        assert orc.partition_and_color(m, 4, 0, 0.0, 0.0, 1)[3] == 3
    else:
        rc, nrx, nry, p, nc, col = orc.partition_and_color(m, 4, 0, 0.0, 0.0, 0)
        assert (rc, nrx, nry, p, nc) == (0, 5, 1, 2, 2)
        assert list(col) == [0, 1, 0, 1, 0]


@pytest.mark.parametrize("dynamic", [0, 1])
def test_line_delta_equals_full_recompute(orc, dynamic):
    spec, m = line_model(orc)
    sp = line_sampler(orc, dynamic=dynamic)
    tr = W.truth_events(spec, 3)
    truth = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    s = orc.simulate(m, truth, 103)
    ch = orc.Chain(m, sp, s, seed=1)
    st = W.random_state(spec, 77, 14)
    ch.set_events(orc.as_events(st["x"], st["y"], st["t"], st["m"]))
    ch.begin_sweep(2)
    X = ch.events()
    base = orc.loglik(m, s, X)
    rng = np.random.default_rng(5)
    checked = {t: 0 for t in range(4)}
    for trial in range(120):
        mtype = trial % 4
        r = int(X["region"][rng.integers(len(X))])
        own = np.nonzero(X["region"] == r)[0]
        idx = int(rng.integers(len(own))) if mtype != orc.BIRTH else -1
        if mtype == orc.BIRTH:
            p = orc.events_array(1)[0]
            p["x"], p["t"] = rng.random() * spec.xmax, X["t"][own[0]] + rng.normal(0, 3)
            p["m"], p["id"] = spec.mmin, 10**9 + trial
        else:
            p = X[own[idx]].copy()
            if mtype == orc.LOC:
                p["x"] += rng.normal(0, 4.0)
            elif mtype == orc.TIME:
                p["t"] += rng.normal(0, 3.0)
        p["x"] = np.clip(p["x"], 0, spec.xmax - 1e-9)
        p["t"] = np.clip(p["t"], 0, spec.N - 1e-9)
        d = ch.delta(r, mtype, idx, p)
        X2 = X.copy()
        if mtype == orc.BIRTH:
            X2 = np.concatenate([X2, p.reshape(1)])
        elif mtype == orc.DEATH:
            X2 = np.delete(X2, own[idx])
        else:
            X2[own[idx]] = p
        assert d == pytest.approx(orc.loglik(m, s, X2) - base, rel=1e-9, abs=1e-8), mtype
        checked[mtype] += 1
    assert min(checked.values()) >= 25


@pytest.mark.parametrize("dynamic", [0, 1])
def test_line_prior_only_samples_the_prior(orc, dynamic):
    spec, m = line_model(orc, lam=12.0)
    sp = line_sampler(orc, prior_only=1, dynamic=dynamic, k=6, ploc=0.3, pt=0.3, sxy=20.0,
                      st=30.0)
    ch = orc.Chain(m, sp, np.zeros((spec.nsta, spec.N)), seed=2)
    counts, xs, ts = [], [], []
    for sw in range(12100):
        assert ch.sweep(sw) == 0
        if sw >= 100 and sw % 4 == 0:
            ev = ch.events()
            counts.append(len(ev))
            if sw % 20 == 0:
                xs.append(ev["x"]); ts.append(ev["t"])
                assert np.all(ev["y"] == 0.0) and np.all(ev["m"] == spec.mmin)
    counts = np.array(counts)
    nb = 20
    bm = counts[: len(counts) // nb * nb].reshape(nb, -1).mean(axis=1)
    se = bm.std(ddof=1) / np.sqrt(nb)
    assert abs(counts.mean() - spec.lam) < 4 * se + 0.2, (counts.mean(), se)
    assert 0.75 * spec.lam < counts.var() < 1.3 * spec.lam
    x, t = np.concatenate(xs), np.concatenate(ts)
    assert stats.kstest(x / spec.xmax, "uniform").pvalue > 1e-3
    assert stats.kstest(t / spec.N, "uniform").pvalue > 1e-3


def _posterior(orc, spec, m, s, gx, dynamic, sweeps, k):
    sp = line_sampler(orc, gx=gx, dynamic=dynamic, k=k)
    ch = orc.Chain(m, sp, s, seed=11)
    counts, hist = [], np.zeros(24)
    for sw in range(sweeps):
        assert ch.sweep(sw) == 0
        if sw >= sweeps // 10:
            ev = ch.events()
            counts.append(len(ev))
            hist += np.bincount((ev["t"] // 10).astype(int), minlength=24)[:24]
    return np.array(counts, dtype=float), hist / hist.sum()


def test_line_chromatic_agrees_with_serial(orc):
    """A small, weakly identified world (Poisson mean 3, signal variance
    1.5) whose posterior keeps events moving: serial (one region) against
    static and dynamic chromatic (four regions, two colours) at equal moves
    per sweep, in the posterior count and the onset histogram."""
    spec, m = line_model(orc, lam=3.0, mmin=math.sqrt(1.5))
    tr = W.truth_events(spec, 21)
    truth = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    s = orc.simulate(m, truth, 121)
    serial = _posterior(orc, spec, m, s, 1, 0, 4000, 160)
    for name, dyn in (("static", 0), ("dynamic", 1)):
        other = _posterior(orc, spec, m, s, 4, dyn, 4000, 40)
        nb = 10
        se = [c[: len(c) // nb * nb].reshape(nb, -1).mean(1).std(ddof=1) / math.sqrt(nb)
              for c in (serial[0], other[0])]
        dc = abs(serial[0].mean() - other[0].mean())
        tv = 0.5 * np.abs(serial[1] - other[1]).sum()
        assert dc < 4 * math.hypot(*se) + 0.05 and tv < 0.08, (name, dc, se, tv)


# ------------------------------------------------------------- lattice
# Two stations at the ends of a line of length 8, wave speed 1 (tau_max = 8),
# t_s = 4, 48 samples, four onset regions of 12 (two colours).  Sites: 4
# locations x 8 onsets.  One true event at x = 7, t = 15: its arrival at the
# far station can also be explained from the previous region, so regions of
# different colours compete for the same samples.

def line_lattice(orc, **kw):
    m = orc.make_model(nsx=2, nsy=1, ds=1.0, N=48, sigma=1.0, atten=1.0, vel=1.0, decay=1.0,
                       ts=4, rc=0.5, lam=1.0, mmin=math.sqrt(3.0), mrate=1.0, line=1, xmax=8.0,
                       sta_x=(0.0, 8.0))
    d = dict(gx=4, gy=0, dynamic=0, k=16, cap=64, pb=0.25, pd=0.25, ploc=0.25, pt=0.25, pm=0.0,
             lattice=1, kx=4, ky=1, kt=8, km=1, hm=0.0)
    d.update(kw)
    return m, orc.make_sampler(**d)


@pytest.fixture(scope="module")
def line_exact(orc):
    m, sp = line_lattice(orc)
    e = orc.lattice_site(m, sp, 3 * sp.kt + 2)
    assert (e["x"], e["y"], e["t"], e["m"]) == (7.0, 0.0, 15.0, math.sqrt(3.0))
    truth = orc.as_events([e["x"]], [e["y"]], [e["t"]], [e["m"]])
    s = orc.simulate(m, truth, 4)
    sites, logw = orc.enumerate_posterior(m, sp, s, 6)
    p = np.exp(logw - logw.max())
    p /= p.sum()
    exact = {tuple(int(v) for v in row if v >= 0): pi for row, pi in zip(sites, p)}
    return s, exact


def _line_tv(orc, s, exact, sweeps, **kw):
    m, sp = line_lattice(orc, **kw)
    ch = orc.Chain(m, sp, s, seed=11)
    cnt = Counter()
    for sw in range(sweeps):
        assert ch.sweep(sw) == 0
        if sw >= 500:
            ev = ch.events()
            assert np.all(ev["m"] == m.mmin) and np.all(ev["y"] == 0.0)
            cnt[tuple(sorted(int(e["x"] // 2.0) * 8 + int(e["t"] // 6.0) for e in ev))] += 1
    tot = sum(cnt.values())
    keys = set(cnt) | set(exact)
    return 0.5 * sum(abs(cnt.get(k, 0) / tot - exact.get(k, 0.0)) for k in keys)


def test_line_enumeration_is_normalised_and_truncation_negligible(line_exact):
    _, exact = line_exact
    assert sum(exact.values()) == pytest.approx(1.0)
    assert sum(v for k, v in exact.items() if len(k) == 6) < 1e-6


@pytest.mark.slow
@pytest.mark.parametrize("name,kw", [
    ("serial", dict(gx=1)),
    ("chromatic-static", dict()),
    ("chromatic-dynamic", dict(dynamic=1)),
])
def test_line_chain_matches_enumerated_posterior(orc, line_exact, name, kw):
    s, exact = line_exact
    tv = _line_tv(orc, s, exact, 20000, **kw)
    assert tv < 0.05, (name, tv)


@pytest.mark.slow
def test_line_naive_parallel_does_not_match_posterior(orc, line_exact):
    s, exact = line_exact
    tv = _line_tv(orc, s, exact, 20000, schedule=1)
    assert tv > 0.08, tv
