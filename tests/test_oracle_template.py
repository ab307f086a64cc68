"""Pins of the oracle's mean-template likelihood (the alternative reading of
Section 3's signal model: each event adds a deterministic waveform to the
mean, the noise is Gaussian with variance sigma^2).

- one event's waveform: support [ceil(a), ceil(a) + t_s), onset value
  A e^{-(ceil(a) - a)/decay} with A = m e^{-d/atten}, constant ratio
  e^{-1/decay} between samples, nothing at stations beyond the cutoff;
- the log-likelihood of a trace equal to the mean plus a constant c is the
  closed form -N_s N (log(2 pi sigma^2) + c^2 / sigma^2) / 2, whatever the
  events;
- the simulator's standardised residuals (s - mean) / sigma are N(0, 1);
- a birth changes the log-likelihood by sum g (r - g / 2) / sigma^2 over its
  samples (r the residual before the move, g the new waveform), and every
  move's local change equals two full recomputations;
- on a lattice instance the serial and chromatic chains match the
  brute-force enumerated posterior.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

from paper_1612_00595_amd import workloads as W

from test_oracle_sampler import lattice_instance, site_of  # noqa: F401  (lattice helpers)


def tmodel(orc, **kw):
    spec = dataclasses.replace(W.SMALL.model, tmpl=1, **kw)
    return spec, orc.make_model(**spec.asdict())


def test_single_event_waveform(orc):
    spec, m = tmodel(orc)
    ev = orc.as_events([0.47], [0.52], [300.25], [2.5])
    Emean = orc.event_variance(m, ev)
    hit = 0
    for j in range(spec.nsta):
        sx = (j % spec.nsx + 0.5) * spec.ds
        sy = (j // spec.nsx + 0.5) * spec.ds
        d = math.hypot(0.47 - sx, 0.52 - sy)
        row = Emean[j]
        if d >= spec.rc:
            assert not row.any(), j
            continue
        hit += 1
        a = orc.arrival_time(0.47, 0.52, 300.25, sx, sy, spec.vel)
        n0 = math.ceil(a)
        nz = np.nonzero(row)[0]
        assert nz[0] == n0 and nz[-1] == n0 + spec.ts - 1
        A = 2.5 * math.exp(-d / spec.atten)
        assert row[n0] == pytest.approx(A * math.exp(-(n0 - a) / spec.decay), rel=1e-13)
        ratio = row[n0 + 1:n0 + spec.ts] / row[n0:n0 + spec.ts - 1]
        assert np.allclose(ratio, math.exp(-1.0 / spec.decay), rtol=1e-12)
    assert hit >= 1


@pytest.mark.parametrize("c", [0.0, 0.037])
def test_loglik_closed_form_at_the_mean(orc, c):
    spec, m = tmodel(orc)
    st = W.random_state(spec, 5, 12)
    ev = orc.as_events(st["x"], st["y"], st["t"], st["m"])
    s = orc.event_variance(m, ev) + c
    want = -0.5 * spec.nsta * spec.N * (math.log(2 * math.pi * spec.sigma ** 2) +
                                        c * c / spec.sigma ** 2)
    assert orc.loglik(m, s, ev) == pytest.approx(want, rel=1e-12)


def test_simulator_residuals_are_standard_normal(orc):
    spec, m = tmodel(orc)
    tr = W.truth_events(spec, 7)
    ev = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    mean = orc.event_variance(m, ev)
    z = (orc.simulate(m, ev, 77) - mean) / spec.sigma
    assert stats.kstest(z.ravel(), "norm").pvalue > 1e-3
    # the signal is in the mean: samples inside waveforms are shifted, not wider
    inside = mean > 0.05
    assert inside.sum() > 500
    assert abs(z[inside].std() - 1.0) < 0.08


def test_birth_delta_is_the_residual_formula(orc):
    spec, m = tmodel(orc)
    sp = orc.make_sampler(**W.SMALL.sampler.asdict())
    tr = W.truth_events(spec, 3)
    truth = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    s = orc.simulate(m, truth, 103)
    ch = orc.Chain(m, sp, s, seed=1)
    st = W.random_state(spec, 77, 10)
    X0 = orc.as_events(st["x"], st["y"], st["t"], st["m"])
    ch.set_events(X0)
    ch.begin_sweep(0)
    X = ch.events()
    r = s - orc.event_variance(m, X)
    rng = np.random.default_rng(2)
    for trial in range(20):
        p = orc.events_array(1)[0]
        p["x"], p["y"] = rng.random() * spec.Lx, rng.random() * spec.Ly
        p["t"], p["m"], p["id"] = rng.random() * spec.N, 2.0 + rng.exponential(), 10**9 + trial
        region = 0  # the move's region only selects the event list; births add p
        g = orc.event_variance(m, p.reshape(1))
        want = float(np.sum(g * (r - g / 2.0)) / spec.sigma ** 2)
        got = ch.delta(region, orc.BIRTH, -1, p)
        assert got == pytest.approx(want, rel=1e-9, abs=1e-9)


def test_template_delta_equals_full_recompute(orc):
    spec, m = tmodel(orc)
    sp = orc.make_sampler(**W.SMALL.sampler.asdict())
    tr = W.truth_events(spec, 3)
    truth = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    s = orc.simulate(m, truth, 103)
    ch = orc.Chain(m, sp, s, seed=1)
    st = W.random_state(spec, 77, 40)
    ch.set_events(orc.as_events(st["x"], st["y"], st["t"], st["m"]))
    ch.begin_sweep(3)
    X = ch.events()
    base = orc.loglik(m, s, X)
    rng = np.random.default_rng(5)
    for trial in range(100):
        mtype = trial % 5
        r = int(X["region"][rng.integers(len(X))])
        own = np.nonzero(X["region"] == r)[0]
        idx = int(rng.integers(len(own))) if mtype != orc.BIRTH else -1
        if mtype == orc.BIRTH:
            p = orc.events_array(1)[0]
            p["x"], p["y"] = X["x"][own[0]] + rng.normal(0, 0.03), X["y"][own[0]] + rng.normal(0, 0.03)
            p["t"], p["m"], p["id"] = rng.random() * spec.N, 2 + rng.exponential(), 10**9 + trial
        else:
            p = X[own[idx]].copy()
            if mtype == orc.LOC:
                p["x"] += rng.normal(0, 0.02)
                p["y"] += rng.normal(0, 0.02)
            elif mtype == orc.TIME:
                p["t"] = np.clip(p["t"] + rng.normal(0, 3), 0, spec.N - 1e-9)
            elif mtype == orc.MAG:
                p["m"] += rng.normal(0, 0.3)
        p["x"] = np.clip(p["x"], 0, spec.Lx - 1e-9)
        p["y"] = np.clip(p["y"], 0, spec.Ly - 1e-9)
        X2 = X.copy()
        if mtype == orc.BIRTH:
            X2 = np.concatenate([X2, p.reshape(1)])
        elif mtype == orc.DEATH:
            X2 = np.delete(X2, own[idx])
        else:
            X2[own[idx]] = p
        assert ch.delta(r, mtype, idx, p) == pytest.approx(orc.loglik(m, s, X2) - base, rel=1e-9,
                                                          abs=1e-7), mtype


@pytest.fixture(scope="module")
def template_exact(orc):
    m, sp = lattice_instance(orc)
    m.tmpl = 1
    m.sigma = 0.3
    site = (1 * sp.kt + 0) * sp.km + 1
    e = orc.lattice_site(m, sp, site)
    truth = orc.as_events([e["x"]], [e["y"]], [e["t"]], [e["m"]])
    s = orc.simulate(m, truth, 3)
    sites, logw = orc.enumerate_posterior(m, sp, s, 7)
    p = np.exp(logw - logw.max())
    p /= p.sum()
    return s, {tuple(int(v) for v in row if v >= 0): pi for row, pi in zip(sites, p)}


@pytest.mark.slow
@pytest.mark.parametrize("name,kw", [("serial", dict(gx=1)), ("chromatic-static", dict()),
                                     ("chromatic-dynamic", dict(dynamic=1))])
def test_template_chain_matches_enumerated_posterior(orc, template_exact, name, kw):
    from collections import Counter
    s, exact = template_exact
    assert sum(exact.values()) == pytest.approx(1.0)
    assert sum(v for k, v in exact.items() if len(k) == 7) < 1e-6
    m, sp = lattice_instance(orc, **kw)
    m.tmpl = 1
    m.sigma = 0.3
    ch = orc.Chain(m, sp, s, seed=11)
    cnt = Counter()
    for sw in range(30000):
        assert ch.sweep(sw) == 0
        if sw >= 500:
            cnt[tuple(sorted(site_of(e, m, sp) for e in ch.events()))] += 1
    tot = sum(cnt.values())
    keys = set(cnt) | set(exact)
    tv = 0.5 * sum(abs(cnt.get(k, 0) / tot - exact.get(k, 0.0)) for k in keys)
    top = max(exact.values())
    assert top < 0.95  # a posterior with several live states
    assert tv < 0.03, (name, tv)
