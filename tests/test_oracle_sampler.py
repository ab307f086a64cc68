"""Pins of the oracle sampler.

- the local log-likelihood change of every move type equals the difference of
  two full recomputations;
- with the likelihood off the chain's stationary law is the prior: Poisson
  count, uniform location and onset, exponential magnitude (this pins the
  birth/death factors and the magnitude prior ratio);
- on a lattice instance with two stations, chain histograms match the
  brute-force enumerated posterior for the serial, chromatic-static and
  chromatic-dynamic schedules, and the naive parallel schedule of Algorithm 3
  does not (Section 4.2: it breaks the factor graph).
"""
from collections import Counter

import numpy as np
import pytest
from scipy import stats

from paper_1612_00595_amd import workloads as W


def small_setup(orc, seed=0, nev=30, **model_kw):
    spec = W.ModelSpec(**dict(W.SMALL.model.asdict(), **model_kw))
    m = orc.make_model(**spec.asdict())
    sp = orc.make_sampler(**W.SMALL.sampler.asdict())
    tr = W.truth_events(spec, seed)
    truth = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    s = orc.simulate(m, truth, seed + 100)
    return spec, m, sp, s, truth


@pytest.mark.parametrize("dynamic", [0, 1])
def test_delta_equals_full_recompute(orc, dynamic):
    spec, m, sp, s, truth = small_setup(orc, seed=3)
    sp.dynamic = dynamic
    if dynamic:
        sp.gx = sp.gy = 5
    ch = orc.Chain(m, sp, s, seed=1)
    st = W.random_state(spec, 77, 40)
    ch.set_events(orc.as_events(st["x"], st["y"], st["t"], st["m"]))
    ch.begin_sweep(3)
    lay = ch.layout()
    rng = np.random.default_rng(5)
    X = ch.events()
    base = orc.loglik(m, s, X)
    checked = {t: 0 for t in range(5)}
    for trial in range(150):
        mtype = trial % 5
        r = int(X["region"][rng.integers(len(X))])
        own = np.nonzero(X["region"] == r)[0]
        idx = int(rng.integers(len(own))) if mtype != orc.BIRTH else -1
        if mtype == orc.BIRTH:
            p = orc.events_array(1)[0]
            p["x"], p["y"] = X["x"][own[0]] + rng.normal(0, 0.03), X["y"][own[0]] + rng.normal(0, 0.03)
            p["t"], p["m"] = rng.random() * spec.N, 2 + rng.exponential()
            p["id"] = 10**9 + trial
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
        d = ch.delta(r, mtype, idx, p)
        X2 = X.copy()
        if mtype == orc.BIRTH:
            X2 = np.concatenate([X2, p.reshape(1)])
        elif mtype == orc.DEATH:
            X2 = np.delete(X2, own[idx])
        else:
            X2[own[idx]] = p
        full = orc.loglik(m, s, X2) - base
        assert d == pytest.approx(full, rel=1e-9, abs=1e-7), (mtype, d, full, lay)
        checked[mtype] += 1
    assert min(checked.values()) >= 25


def _prior_run(orc, dynamic, sweeps, lam=20.0):
    spec = W.ModelSpec(**dict(W.SMALL.model.asdict(), lam=lam))
    m = orc.make_model(**spec.asdict())
    sp = orc.make_sampler(**dict(W.SMALL.sampler.asdict(), prior_only=1, dynamic=dynamic,
                                 gx=5 if dynamic else 4, gy=5 if dynamic else 4, k=8))
    s = np.zeros((spec.nsta, spec.N))
    ch = orc.Chain(m, sp, s, seed=2)
    counts, xs, ys, ts, ms = [], [], [], [], []
    for sw in range(sweeps):
        assert ch.sweep(sw) == 0
        if sw >= 100 and sw % 5 == 0:
            ev = ch.events()
            counts.append(len(ev))
            if sw % 25 == 0:
                xs.append(ev["x"]); ys.append(ev["y"]); ts.append(ev["t"]); ms.append(ev["m"])
    return spec, np.array(counts), [np.concatenate(a) for a in (xs, ys, ts, ms)]


@pytest.mark.parametrize("dynamic", [0, 1])
def test_prior_only_chain_samples_the_prior(orc, dynamic):
    spec, counts, (x, y, t, m) = _prior_run(orc, dynamic, 6100)
    lam = spec.lam
    # Poisson(lam): mean and variance both lam (batch-means standard error)
    nb = 20
    bm = counts[: len(counts) // nb * nb].reshape(nb, -1).mean(axis=1)
    se = bm.std(ddof=1) / np.sqrt(nb)
    assert abs(counts.mean() - lam) < 4 * se + 0.3, (counts.mean(), se)
    assert 0.75 * lam < counts.var() < 1.3 * lam
    # the count histogram against the Poisson pmf
    hist = np.bincount(counts, minlength=60)[:60] / len(counts)
    pmf = stats.poisson.pmf(np.arange(60), lam)
    assert 0.5 * np.abs(hist - pmf).sum() < 0.08
    assert stats.kstest(x / spec.Lx, "uniform").pvalue > 1e-3
    assert stats.kstest(y / spec.Ly, "uniform").pvalue > 1e-3
    assert stats.kstest(t / spec.N, "uniform").pvalue > 1e-3
    assert stats.kstest(m - 2.0, "expon").pvalue > 1e-3


# ------------------------------------------------------------- lattice

def lattice_instance(orc, schedule=0, dynamic=0, gx=2, k=16):
    m = orc.make_model(nsx=2, nsy=1, ds=0.2, N=48, sigma=0.1, atten=0.2, vel=0.05,
                       decay=8.0, ts=24, rc=0.19, lam=1.0, mmin=0.4, mrate=1.0)
    sp = orc.make_sampler(gx=gx, gy=1, dynamic=dynamic, k=k, cap=64, pb=0.25, pd=0.25,
                          ploc=0.2, pt=0.15, pm=0.15, lattice=1, kx=4, ky=1, kt=2, km=2,
                          hm=0.05, schedule=schedule)
    return m, sp


def site_of(ev, m, sp):
    hx = 0.4 / sp.kx
    ht = m.N / sp.kt
    ix = int(np.floor(ev["x"] / hx))
    it = int(np.floor(ev["t"] / ht))
    im = int(np.floor((ev["m"] - m.mmin) / sp.hm))
    return (ix * sp.ky * sp.kt + it) * sp.km + im


@pytest.fixture(scope="module")
def lattice_exact(orc):
    m, sp = lattice_instance(orc)
    # one true event at x = 0.15: it reaches both stations, so its signal is
    # seen from both sides of the region boundary at x = 0.2
    site = (1 * sp.kt + 0) * sp.km + 1
    e = orc.lattice_site(m, sp, site)
    truth = orc.as_events([e["x"]], [e["y"]], [e["t"]], [e["m"]])
    s = orc.simulate(m, truth, 3)
    sites, logw = orc.enumerate_posterior(m, sp, s, 7)
    p = np.exp(logw - logw.max())
    p /= p.sum()
    exact = {tuple(int(v) for v in row if v >= 0): pi for row, pi in zip(sites, p)}
    return s, exact


def lattice_tv(orc, s, exact, sweeps, **kw):
    m, sp = lattice_instance(orc, **kw)
    ch = orc.Chain(m, sp, s, seed=11)
    cnt = Counter()
    for sw in range(sweeps):
        assert ch.sweep(sw) == 0
        if sw >= 500:
            cnt[tuple(sorted(site_of(e, m, sp) for e in ch.events()))] += 1
    tot = sum(cnt.values())
    keys = set(cnt) | set(exact)
    return 0.5 * sum(abs(cnt.get(k, 0) / tot - exact.get(k, 0.0)) for k in keys)


def test_enumeration_is_normalised_and_truncation_negligible(lattice_exact):
    _, exact = lattice_exact
    assert sum(exact.values()) == pytest.approx(1.0)
    tail = sum(v for k, v in exact.items() if len(k) == 7)
    assert tail < 1e-6


@pytest.mark.parametrize("name,kw", [
    ("serial", dict(gx=1)),
    ("chromatic-static", dict()),
    ("chromatic-dynamic", dict(dynamic=1)),
])
def test_chain_matches_enumerated_posterior(orc, lattice_exact, name, kw):
    s, exact = lattice_exact
    tv = lattice_tv(orc, s, exact, 30000, **kw)
    assert tv < 0.03, (name, tv)


def test_naive_parallel_does_not_match_posterior(orc, lattice_exact):
    s, exact = lattice_exact
    tv = lattice_tv(orc, s, exact, 30000, schedule=1)
    assert tv > 0.1, tv
