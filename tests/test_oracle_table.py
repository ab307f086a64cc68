"""Pins of three oracle functions that the GPU parity tests lean on:

* ``oracle.mdn.mixture_table`` (the learned proposal's mixture table): log
  weights and cumulative weights against scipy's softmax, the clamps of the
  means and sds at their exact boundary values, the anchor -> (station,
  window) indexing on a non-square grid, and the density the table describes
  against ``mixture_nll`` on the same head row (scipy's normal densities on
  one side, the training loss on the other), which ties the two readings of
  the head's column layout together;
* ``oracle.mdn.anchor_weight`` composed with the oracle's envelope features:
  hand values for constant and single-spike traces, after BF16 rounding;
* the grid branch of the oracle's log prior (Section 3's event prior as a
  set density): scipy's Poisson, uniform and exponential densities for 0, 1
  and 2 events.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

from oracle import mdn as D
from paper_1612_00595_amd import workloads as W


def head(rows, rng, mean_scale=0.5, logsd=(-1.0, -1.0, -2.0)):
    """Head outputs [rows][64] with means and log sds inside the clamps."""
    o = np.zeros((rows, 64))
    for k in range(D.N_K):
        o[:, 7 * k] = rng.normal(0, 1.0, rows)
        o[:, 7 * k + 1:7 * k + 4] = rng.uniform(-mean_scale, mean_scale, (rows, 3))
        o[:, 7 * k + 4:7 * k + 7] = np.asarray(logsd) + rng.uniform(-0.3, 0.3, (rows, 3))
    return o


def test_mixture_table_weights_against_softmax():
    rng = np.random.default_rng(11)
    o = head(6, rng)
    o[0, 0:56:7] = 0.75                         # equal logits
    T = D.mixture_table(o, nsx=4, ds=0.2, n_tau=3)
    assert np.allclose(T[0, :, 6], -math.log(8.0), rtol=0, atol=1e-15)
    assert np.allclose(T[0, :, 7], np.arange(1, 9) / 8.0, rtol=0, atol=1e-15)
    for r in range(1, 6):
        pi = special.softmax(o[r, 0:56:7])
        assert np.allclose(np.exp(T[r, :, 6]), pi, rtol=1e-13, atol=0)
        assert np.allclose(T[r, :, 7], np.cumsum(pi), rtol=1e-13, atol=0)
        assert T[r, 7, 7] == pytest.approx(1.0, abs=1e-14)


def test_mixture_table_clamps_at_exact_boundaries():
    ds, nsx, n_tau = 0.2, 3, 5
    o = np.zeros((1, 64))
    # component 0: far beyond every clamp on the high side; 1: on the low
    # side; 2: exactly on the mean bounds; 3: inside
    o[0, 1:4] = (5.0, 7.0, 10.0)
    o[0, 4:7] = (10.0, 10.0, 10.0)
    o[0, 8:11] = (-5.0, -7.0, -10.0)
    o[0, 11:14] = (-10.0, -10.0, -10.0)
    o[0, 15:18] = (2.0, -2.0, 3.0)
    o[0, 22:25] = (1.5, -0.25, 0.5)
    o[0, 25:28] = (math.log(0.1), math.log(0.2), math.log(0.25))
    a = 7                                       # station 1 = (ix 1, iy 0), window 2
    T = D.mixture_table(o, nsx=nsx, ds=ds, n_tau=n_tau, first=a)[0]
    sx, sy, tau = 1.5 * ds, 0.5 * ds, 64.0
    assert tuple(T[0, :3]) == pytest.approx((sx + 2 * ds, sy + 2 * ds, tau + 96), abs=1e-15)
    assert tuple(T[0, 3:6]) == pytest.approx((1.5 * ds, 1.5 * ds, 32.0), rel=1e-15)
    assert tuple(T[1, :3]) == pytest.approx((sx - 2 * ds, sy - 2 * ds, tau - 32), abs=1e-15)
    assert tuple(T[1, 3:6]) == pytest.approx((0.025 * ds, 0.025 * ds, 0.5), rel=1e-14)
    assert tuple(T[2, :3]) == pytest.approx((sx + 2 * ds, sy - 2 * ds, tau + 96), abs=1e-15)
    assert tuple(T[3, :3]) == pytest.approx((sx + 1.5 * ds, sy - 0.25 * ds, tau + 16),
                                            abs=1e-15)
    assert tuple(T[3, 3:6]) == pytest.approx((0.1 * ds, 0.2 * ds, 0.25 * 32), rel=1e-14)


def test_mixture_table_anchor_indexing_row_major():
    # a 3 x 2 station grid (not square, so a transposed index shows) with
    # five windows per station: anchor a is station a // 5, window a % 5
    ds, nsx, n_tau = 0.25, 3, 5
    o = np.zeros((30, 64))
    T = D.mixture_table(o, nsx=nsx, ds=ds, n_tau=n_tau)
    for a in range(30):
        st, win = divmod(a, n_tau)
        ix, iy = st % nsx, st // nsx
        assert T[a, 0, 0] == pytest.approx((ix + 0.5) * ds, abs=1e-15)
        assert T[a, 0, 1] == pytest.approx((iy + 0.5) * ds, abs=1e-15)
        assert T[a, 0, 2] == 32.0 * win
    # the same rows through `first`
    T2 = D.mixture_table(o[16:22], nsx=nsx, ds=ds, n_tau=n_tau, first=16)
    assert np.array_equal(T2, T[16:22])


def test_mixture_table_density_equals_training_density():
    """The absolute-unit mixture the table describes, evaluated with scipy,
    equals the training loss's mixture on the relative target
    ((x - sx) / ds, (y - sy) / ds, (t - tau) / 32) up to that change of
    variables' Jacobian ds * ds * 32."""
    rng = np.random.default_rng(5)
    ds, nsx, n_tau = 0.2, 4, 6
    rows = 10
    o = head(rows, rng)
    first = 9
    T = D.mixture_table(o, nsx=nsx, ds=ds, n_tau=n_tau, first=first)
    for r in range(rows):
        a = first + r
        st = a // n_tau
        sx, sy, tau = (st % nsx + 0.5) * ds, (st // nsx + 0.5) * ds, 32.0 * (a % n_tau)
        for _ in range(4):
            xi = np.array([sx + rng.normal(0, 0.5) * ds, sy + rng.normal(0, 0.5) * ds,
                           tau + rng.normal(0, 0.5) * 32])
            logq = special.logsumexp([T[r, k, 6] + np.sum(stats.norm.logpdf(
                xi, T[r, k, 0:3], T[r, k, 3:6])) for k in range(D.N_K)])
            z = np.array([[(xi[0] - sx) / ds, (xi[1] - sy) / ds, (xi[2] - tau) / 32.0]])
            nll, _ = D.mixture_nll(o[r:r + 1], z)
            assert logq == pytest.approx(-nll[0] - math.log(ds * ds * 32.0), rel=1e-11, abs=1e-11)


def test_anchor_weight_hand_values(orc):
    spec = W.ModelSpec(nsx=3, nsy=3, N=100)
    m = orc.make_model(**spec.asdict())
    sig2 = spec.sigma ** 2
    # constant trace 0.3: every present feature is ln(1 + 0.09 / 0.01) =
    # ln 10, which BF16 rounds to 2.296875 (spacing 2^-6 on [2, 4))
    s = np.full((9, 100), 0.3)
    f_bf = D.to_bf16(np.log(sig2 + 0.09) - np.log(sig2))
    assert f_bf == 2.296875
    centre = D.to_bf16(D.anchor_features(m, s, 2, 4 * 2))
    assert D.anchor_weight(centre) == pytest.approx(1e-3 + (2.296875 - 1.0), rel=1e-15)
    corner = D.to_bf16(D.anchor_features(m, s, 2, 0))          # 4 of 9 stations on the grid
    assert D.anchor_weight(corner) == pytest.approx(1e-3 + 4 / 9 * (2.296875 - 1.0), rel=1e-15)
    # a quiet constant trace (features ln 1.5 < 1) carries only the floor
    s = np.full((9, 100), math.sqrt(0.005))
    assert D.anchor_weight(D.to_bf16(D.anchor_features(m, s, 2, 4 * 2))) == 1e-3
    # one spike of 2.0 on the centre station: four features ln(1 + 1 / 0.01)
    # = ln 101 -> BF16 4.625 (spacing 2^-5 on [4, 8)); the other 572 are 0
    s = np.zeros((9, 100))
    s[4, 40] = 2.0
    spike = D.to_bf16(D.anchor_features(m, s, 2, 4 * 2 + 1))
    assert np.count_nonzero(spike) == 4 and np.all(spike[spike != 0] == 4.625)
    assert D.anchor_weight(spike) == pytest.approx(1e-3 + 4 * 3.625 / 576, rel=1e-15)


def grid_model(orc, lam=20.0, mrate=1.0):
    spec = W.ModelSpec(nsx=5, nsy=4, N=1000, lam=lam, mrate=mrate)
    return spec, orc.make_model(**spec.asdict())


@pytest.mark.parametrize("lam,mrate", [(20.0, 1.0), (3.5, 2.5)])
def test_grid_logprior_against_scipy(orc, lam, mrate):
    """Section 3's prior: Poisson(lambda) count, uniform location on the
    domain, uniform onset on [0, N), exponential magnitude above mag_min; as a
    set density the n events carry n! orderings, so the density is the
    ordered one times n!."""
    spec, m = grid_model(orc, lam, mrate)
    Lx, Ly = spec.nsx * spec.ds, spec.nsy * spec.ds
    rng = np.random.default_rng(3)
    for n in (0, 1, 2):
        x = rng.uniform(0, Lx, n)
        y = rng.uniform(0, Ly, n)
        t = rng.uniform(0, spec.N, n)
        mag = spec.mmin + rng.exponential(1 / mrate, n)
        ev = orc.as_events(x, y, t, mag)
        want = stats.poisson.logpmf(n, lam) + special.gammaln(n + 1)
        want += np.sum(stats.uniform.logpdf(x, 0, Lx) + stats.uniform.logpdf(y, 0, Ly)
                       + stats.uniform.logpdf(t, 0, spec.N)
                       + stats.expon.logpdf(mag, loc=spec.mmin, scale=1 / mrate))
        assert orc.logprior(m, ev) == pytest.approx(want, rel=1e-13, abs=1e-12)


def test_grid_logprior_differences_are_the_birth_factors(orc):
    """Adding an event changes the log prior by ln(lambda p(e)): the quantity
    whose region-restricted form is the birth factor of the moves."""
    spec, m = grid_model(orc)
    a = orc.as_events([0.3], [0.5], [100.0], [2.7])
    b = orc.as_events([0.3, 0.9], [0.5, 0.1], [100.0, 450.0], [2.7, 3.1])
    dl = orc.logprior(m, b) - orc.logprior(m, a)
    want = math.log(spec.lam) - math.log(spec.nsx * spec.ds * spec.nsy * spec.ds) \
        - math.log(spec.N) + stats.expon.logpdf(3.1, loc=spec.mmin, scale=1 / spec.mrate)
    assert dl == pytest.approx(want, rel=1e-13)
