"""Pins of the network oracle (numpy FP64): mixture density against scipy,
backpropagation against finite differences, GELU against the normal CDF,
BF16 rounding against torch, envelope features against closed forms, and
the training-pair targets' distribution."""
import numpy as np
import pytest
from scipy import stats

from oracle import mdn as D
from paper_1612_00595_amd import workloads as W


def random_params(rng, scale=0.08):
    lay, n = D.param_layout()
    return D.unflatten(rng.normal(0, scale, n))


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 101)
    assert np.allclose(D.gelu(z), z * stats.norm.cdf(z), rtol=1e-13, atol=1e-15)
    h = 1e-6
    assert np.allclose(D.gelu_grad(z), (D.gelu(z + h) - D.gelu(z - h)) / (2 * h), atol=1e-8)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).normal(0, 3, 5000).astype(np.float32)
    x[:3] = [1.00390625, 1.01171875, -2.0]  # ties to even
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(D.to_bf16(x), want.astype(np.float64))


def test_mixture_nll_matches_scipy():
    rng = np.random.default_rng(1)
    M = 20
    o = rng.normal(0, 1, (M, 64))
    z = rng.normal(0, 1, (M, 3))
    loss, _ = D.mixture_nll(o, z)
    for m in range(M):
        logit = o[m, 0:56:7]
        pi = np.exp(logit - logit.max()) / np.exp(logit - logit.max()).sum()
        dens = 0.0
        for k in range(8):
            s = np.clip(o[m, 7 * k + 4:7 * k + 7], D.SLO, D.SHI)
            dens += pi[k] * np.prod(stats.norm.pdf(z[m], o[m, 7 * k + 1:7 * k + 4], np.exp(s)))
        assert loss[m] == pytest.approx(-np.log(dens), rel=1e-10)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(2)
    P = random_params(rng)
    X = rng.normal(0, 1, (3, D.N_IN))
    Z = rng.normal(0, 0.7, (3, 3))
    _, _, G = D.loss_and_grads(P, X, Z, bf16=False)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"):
        flat = P[name].ravel()
        idx = rng.choice(flat.size, 12, replace=False)
        if name in ("W4", "b4"):  # only the 56 live outputs carry gradient
            live = np.arange(flat.size) // (P[name].shape[1] if name == "W4" else 1) < 56
            idx = rng.choice(np.nonzero(live)[0], 12, replace=False)
        for q in idx:
            keep = flat[q]
            flat[q] = keep + h
            lp, _, _ = D.loss_and_grads(P, X, Z, bf16=False)
            flat[q] = keep - h
            lm, _, _ = D.loss_and_grads(P, X, Z, bf16=False)
            flat[q] = keep
            fd = (lp - lm) / (2 * h)
            an = G[name].ravel()[q]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-8), (name, q)


def test_envelope_features_closed_forms(orc):
    spec = W.ModelSpec(nsx=3, nsy=3, N=100)
    m = orc.make_model(**spec.asdict())
    s = np.full((9, 100), 0.3)
    f = D.anchor_features(m, s, 2, 4 * 2 + 0).reshape(9, 64)     # centre station
    assert np.allclose(f, np.log(0.01 + 0.09) - np.log(0.01), rtol=1e-14)
    # corner station 0: the block's row and column beyond the grid are 0
    f = D.anchor_features(m, s, 2, 0).reshape(3, 3, 64)
    assert np.all(f[0, :, :] == 0) and np.all(f[:, 0, :] == 0)
    assert np.allclose(f[1:, 1:], np.log(0.01 + 0.09) - np.log(0.01), rtol=1e-14)
    s = np.zeros((9, 100))
    s[4, 40] = 2.0                       # centre station, window of tau = 32
    f = D.anchor_features(m, s, 2, 4 * 2 + 1).reshape(9, 64)
    spike = np.log(0.01 + 4.0 / 4) - np.log(0.01)
    assert np.allclose(f[4, 5:9], spike) and np.allclose(f[4, :5], 0) and np.allclose(f[4, 9:], 0)
    assert np.allclose(np.delete(f, 4, axis=0), 0)


def edge_class_of(F):
    """(ex, ey) of pairs from which block rows / columns are all zero."""
    z = np.all(F.reshape(-1, 3, 3, 64) == 0, axis=3)         # [pair, row, col]
    ex = np.where(z[:, :, 0].all(1), -1, np.where(z[:, :, 2].all(1), 1, 0))
    ey = np.where(z[:, 0, :].all(1), -1, np.where(z[:, 2, :].all(1), 1, 0))
    return ex, ey


def test_training_pair_targets_and_edge_classes(orc):
    m = orc.make_model(**W.SMALL.model.asdict())
    F, T = D.pairs(m, 9, 0, 1600)
    ex, ey = edge_class_of(F)
    # class 0 with probability 1/2, each of the 8 edge classes 1/16
    cls = (ey + 1) * 3 + (ex + 1)
    obs = np.bincount(cls, minlength=9)
    expect = np.full(9, 1600 / 16)
    expect[4] = 800
    assert stats.chisquare(obs, expect).pvalue > 1e-3
    # targets: uniform over the part of the +-1 spacing box inside the domain
    for axis, e in ((0, ex), (1, ey)):
        for side, lo, hi in ((0, -1.0, 1.0), (-1, -0.5, 1.0), (1, -1.0, 0.5)):
            v = T[e == side, axis]
            assert stats.kstest((v - lo) / (hi - lo), "uniform").pvalue > 1e-3
    assert stats.kstest((T[:, 2] * 32 + 16) / 80, "uniform").pvalue > 1e-3
    # a target that arrives well inside the window (t < 48) leaves the
    # strongest station envelope far above the noise level
    inside = T[:, 2] * 32 < 48
    assert inside.sum() > 800 and np.all(F[inside].max(1) > np.log(1 + 30))


def test_training_pair_noise_is_chi_square(orc):
    # with vanishing magnitudes a feature sample of a present station is pure
    # noise: the mean of four squared N(0, sigma^2) draws, so 4 (exp(f) - 1)
    # ~ chi2 with 4 dof; the first sample of each station is independent of
    # every other one
    spec = W.ModelSpec(nsx=5, nsy=5, N=1000, mmin=1e-7, mrate=1e7)
    m = orc.make_model(**spec.asdict())
    F, _ = D.pairs(m, 3, 100, 300)
    G = F.reshape(-1, 64)
    G = G[~np.all(G == 0, axis=1)]
    for col in (0, 1):
        x = 4 * (np.exp(G[:, col]) - 1)
        assert stats.kstest(x, stats.chi2(4).cdf).pvalue > 1e-3
