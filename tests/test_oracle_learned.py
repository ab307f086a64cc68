"""Pins of the oracle's learned birth proposal (the independence proposal
mixed with the prior birth, with its density in the acceptance ratio):

- the region density with one component reduces to a product of scipy's
  truncated normals;
- with components of disjoint support, draws pick anchors and components
  with probability (w_a / W_R) pi_k, land on mean + sd * (truncated
  normals), and the density at a draw is that one component's share;
- the 16-wide draw records carry uniforms and [-4, 4]-truncated normals;
- prior-only chains with learned births still sample the Poisson prior
  (the posterior is the prior whatever the proposal, so any error in the
  proposal density or the birth/death factors shows up here).
"""
import numpy as np
import pytest
from scipy import stats

from paper_1612_00595_amd import workloads as W


def _chain(orc, spec, sampler_kw, seed=2):
    m = orc.make_model(**spec.asdict())
    sp = orc.make_sampler(**sampler_kw)
    s = np.zeros((spec.nsta, spec.N))
    return m, sp, orc.Chain(m, sp, s, seed=seed)


def _static(gx, gy, **kw):
    d = dict(W.SMALL.sampler.asdict(), gx=gx, gy=gy, dynamic=0)
    d.update(kw)
    return d


def test_draw_records_of_sixteen(orc):
    recs = np.array([orc.move_draws16(3, 1, sw, r, j)
                     for sw in range(40) for r in range(10) for j in range(16)])
    base = np.array([orc.move_draws(3, 1, sw, r, j)
                     for sw in range(40) for r in range(10) for j in range(16)])
    assert np.array_equal(recs[:, :8], base)
    for c in (8, 9, 10):
        assert stats.kstest(recs[:, c], "uniform").pvalue > 1e-3
    z = recs[:, 11:14].ravel()
    assert np.all(np.abs(z) <= 4.0)
    assert stats.kstest(z, stats.truncnorm(-4, 4).cdf).pvalue > 1e-3
    assert np.all(recs[:, 14:] == 0)


def test_single_component_density_is_truncated_normal_product(orc):
    spec = W.ModelSpec(nsx=3, nsy=3, N=1000)
    m, sp, ch = _chain(orc, spec, _static(3, 3))
    T, w, n_tau = W.random_mixture_table(spec, 4)
    # every anchor: one live component (weight 1) with the same mean and sds
    T[:, :, 6] = -np.inf
    T[:, 0, 6] = 0.0
    T[:, :, 7] = 1.0
    T[:, :, 0:6] = [0.33, 0.29, 400.0, 0.04, 0.03, 7.0]
    assert ch.set_learned(T, w, n_tau) == 0
    assert ch.begin_sweep(0) == 0
    r = 2 * ch.layout()["nrx"] + 2        # region of the centre station
    rng = np.random.default_rng(0)
    for _ in range(200):
        x, y, t = 0.33 + rng.uniform(-0.2, 0.2), 0.29 + rng.uniform(-0.15, 0.15), \
            400.0 + rng.uniform(-35, 35)
        want = (stats.truncnorm(-4, 4, 0.33, 0.04).pdf(x) * stats.truncnorm(-4, 4, 0.29, 0.03).pdf(y)
                * stats.truncnorm(-4, 4, 400.0, 7.0).pdf(t))
        assert ch.learned_q(r, x, y, t) == pytest.approx(want, rel=1e-11, abs=1e-300)


def test_draws_follow_the_mixture(orc):
    """Components with disjoint supports: each draw identifies its anchor and
    component, whose frequencies must be (w_a / W_R) pi_k."""
    spec = W.ModelSpec(nsx=2, nsy=2, N=67 + 32 * 9)
    m, sp, ch = _chain(orc, spec, _static(1, 1))
    T, w, n_tau = W.random_mixture_table(spec, 5)
    nc = spec.nsta * n_tau * 8
    gap = spec.N / nc
    T[..., 2] = (np.arange(nc).reshape(-1, 8) + 0.5) * gap
    T[..., 5] = gap / 10.0
    T[..., 0] = 0.2
    T[..., 1] = 0.2
    T[..., 3:5] = 0.01
    assert ch.set_learned(T, w, n_tau) == 0
    assert ch.begin_sweep(0) == 0
    r = 1 * ch.layout()["nrx"] + 1         # the one region holding all 4 stations
    rng = np.random.default_rng(1)
    n = 30000
    counts = np.zeros(nc)
    pi = np.diff(np.concatenate([np.zeros((len(T), 1)), T[..., 7]], axis=1), axis=1)
    share = (w[:, None] / w.sum()) * pi
    for q in range(n):
        d = np.zeros(16)
        d[8:11] = rng.random(3)
        d[11:14] = stats.truncnorm(-4, 4).rvs(3, random_state=rng)
        x, y, t = ch.learned_draw(r, d)
        c = int(t // gap)
        counts[c] += 1
        a, k = divmod(c, 8)
        assert x == T[a, k, 0] + T[a, k, 3] * d[11]
        assert y == T[a, k, 1] + T[a, k, 4] * d[12]
        assert t == T[a, k, 2] + T[a, k, 5] * d[13]
        if q < 300:
            want = share[a, k] * np.prod([stats.truncnorm(-4, 4, T[a, k, u], T[a, k, 3 + u]).pdf(v)
                                          for u, v in enumerate((x, y, t))])
            assert ch.learned_q(r, x, y, t) == pytest.approx(want, rel=1e-10)
    expect = share.ravel() * n
    # pool sparse cells, then chi-square
    order = np.argsort(expect)
    e, o = expect[order], counts[order]
    cuts = np.searchsorted(np.cumsum(e), np.arange(1, int(e.sum() // 50)) * 50.0)
    eb = np.add.reduceat(e, np.unique(np.concatenate([[0], cuts])))
    ob = np.add.reduceat(o, np.unique(np.concatenate([[0], cuts])))
    chi2 = np.sum((ob - eb) ** 2 / eb)
    assert stats.chi2(len(eb) - 1).sf(chi2) > 1e-4


def _log_ratio_stat(orc, ch, spec, sp, pts):
    """log(1/2 + 1/2 q_R(x) area_R N) at each point, R its region in the
    chain's current partition."""
    lay = ch.layout()
    wx, wy = spec.Lx / sp.gx, spec.Ly / sp.gy
    out = np.empty(len(pts))
    for q, (x, y, t) in enumerate(pts):
        i = orc.region_axis(x, lay["offx"], wx, sp.gx)
        k = orc.region_axis(y, lay["offy"], wy, sp.gy)
        x0, x1 = max(lay["offx"] + (i - 1) * wx, 0.0), min(lay["offx"] + i * wx, spec.Lx)
        y0, y1 = max(lay["offy"] + (k - 1) * wy, 0.0), min(lay["offy"] + k * wy, spec.Ly)
        qv = ch.learned_q(k * lay["nrx"] + i, x, y, t)
        out[q] = np.log(0.5 + 0.5 * qv * (x1 - x0) * (y1 - y0) * spec.N)
    return out


@pytest.mark.parametrize("dynamic", [0, 1])
def test_prior_only_with_learned_births_samples_the_prior(orc, dynamic):
    spec = W.SMALL.model
    kw = dict(W.SMALL.sampler.asdict(), prior_only=1, dynamic=dynamic,
              gx=5 if dynamic else 4, gy=5 if dynamic else 4, k=8)
    m, sp, ch = _chain(orc, spec, kw)
    # components about a fifth of a region wide and 60 samples long: the
    # learned part of the birth density is then of the order of the prior's
    # over much of each region, where a wrong ratio shifts the count most
    T, w, n_tau = W.random_mixture_table(spec, 6)
    T[..., 3:5] = 0.05
    T[..., 5] = 60.0
    assert ch.set_learned(T, w, n_tau) == 0
    rng = np.random.default_rng(7)
    counts, xs, ys, ts, ms, h_ev, h_uni = [], [], [], [], [], [], []
    log = np.zeros((sp.gx + 1) * (sp.gy + 1) * sp.k * 4)
    acc_birth = 0
    for sw in range(16100):
        log[:] = -1
        assert ch.sweep(sw, log=log) == 0
        lg = log.reshape(-1, 4)
        acc_birth += int(np.sum((lg[:, 0] == 0) & (lg[:, 1] == 2)))
        if sw >= 100 and sw % 5 == 0:
            ev = ch.events()
            counts.append(len(ev))
            if sw % 50 == 0:
                xs.append(ev["x"]); ys.append(ev["y"]); ts.append(ev["t"]); ms.append(ev["m"])
                h_ev.append(_log_ratio_stat(orc, ch, spec, sp, np.stack([ev["x"], ev["y"], ev["t"]], 1)))
                u = rng.random((len(ev), 3)) * [spec.Lx, spec.Ly, spec.N]
                h_uni.append(_log_ratio_stat(orc, ch, spec, sp, u))
    counts = np.array(counts)
    x, y, t, mm = (np.concatenate(a) for a in (xs, ys, ts, ms))
    lam = spec.lam
    nb = 20
    bm = counts[: len(counts) // nb * nb].reshape(nb, -1).mean(axis=1)
    se = bm.std(ddof=1) / np.sqrt(nb)
    assert abs(counts.mean() - lam) < 4.5 * se, (counts.mean(), se)
    assert 0.8 * lam < counts.var() < 1.25 * lam
    assert stats.kstest(x / spec.Lx, "uniform").pvalue > 1e-3
    assert stats.kstest(y / spec.Ly, "uniform").pvalue > 1e-3
    assert stats.kstest(t / spec.N, "uniform").pvalue > 1e-3
    assert stats.kstest(mm - 2.0, "expon").pvalue > 1e-3
    # events of the stationary chain are uniform, so their proposal log
    # ratio has the same law as at uniform points (snapshots 50 sweeps
    # apart, treated as independent; a wrong ratio over- or under-weights
    # the places where the proposal is dense)
    he, hu = np.concatenate(h_ev), np.concatenate(h_uni)
    z = (he.mean() - hu.mean()) / np.sqrt(he.var() / len(he) + hu.var() / len(hu))
    assert abs(z) < 4.0, (he.mean(), hu.mean(), z)
    assert stats.ks_2samp(he, hu).pvalue > 1e-4
    assert acc_birth > 1000
