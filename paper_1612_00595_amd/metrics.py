"""Evaluation of inferred event sets (host side, numpy).

Matching and scores follow the evaluation of Section 5: true events are
visited in turn, each is joined to the closest still-unmatched inferred
event if the two are closer than a distance threshold and a time threshold,
and matched events leave the pool.  Location error is the mean distance over
matches, precision the matched share of inferred events, recall the matched
share of true events.  The paper's thresholds are 12 units of its 1-D world
(x_max = 100); on the unit-spaced 2-D domain here they read 0.12 in space and
12 samples in time.  "Closest" is the larger of the two normalised
separations, and true events are visited in increasing onset time.

Effective sample size uses Geyer's initial monotone sequence estimator
(Geyer, "Practical Markov chain Monte Carlo", Statistical Science 1992):
autocovariances are summed in adjacent pairs while the pair sums stay
positive, each pair sum clipped to the smallest before it.
"""
from __future__ import annotations

import dataclasses

import numpy as np

DIST_THRESH = 0.12
TIME_THRESH = 12.0
PAPER_DIST_THRESH = 12.0   # the 1-D world of the paper, in its own units


@dataclasses.dataclass
class MatchResult:
    pairs: list            # (true index, inferred index)
    precision: float
    recall: float
    f1: float
    location_error: float  # mean spatial distance over matches (nan if none)


DENSE_PAIRS = 1 << 17   # up to this many true x inferred pairs, all separations at once


def match(true_ev, inf_ev, dist_thresh: float = DIST_THRESH,
          time_thresh: float = TIME_THRESH) -> MatchResult:
    """Greedy bipartite matching of true to inferred events (Section 5): in
    onset order (ties by index) each true event is joined to its closest
    still-unmatched inferred event -- closeness being the larger of the two
    separations, each over its threshold -- when that one lies within both
    thresholds; among equally close ones the lowest index wins.

    Small sets take all separations at once; large ones examine only the
    inferred events inside each true event's time window (found by binary
    search in onset order), which selects the same event: the closest one is
    within the thresholds exactly when some unmatched event is."""
    tx, ty, tt = (np.asarray(true_ev[f], dtype=np.float64) for f in ("x", "y", "t"))
    ix, iy, it = (np.asarray(inf_ev[f], dtype=np.float64) for f in ("x", "y", "t"))
    nt, ni = len(tx), len(ix)
    pairs, dists = [], []
    if nt and ni:
        go = _match_dense if nt * ni <= DENSE_PAIRS else _match_windowed
        go(tx, ty, tt, ix, iy, it, dist_thresh, time_thresh, pairs, dists)
    m = len(pairs)
    precision = m / ni if ni else 1.0
    recall = m / nt if nt else 1.0
    f1 = 2 * precision * recall / (precision + recall) if precision + recall > 0 else 0.0
    err = float(np.mean(dists)) if dists else float("nan")
    return MatchResult(pairs, precision, recall, f1, err)


def _match_dense(tx, ty, tt, ix, iy, it, dt, tw, pairs, dists):
    D = np.hypot(ix[None, :] - tx[:, None], iy[None, :] - ty[:, None])
    T = np.abs(it[None, :] - tt[:, None])
    S = np.maximum(D / dt, T / tw)            # taken inferred events get +inf
    for a in np.lexsort((np.arange(len(tx)), tt)):
        b = int(np.argmin(S[a]))
        if not np.isfinite(S[a, b]):
            break                              # no inferred event left
        if D[a, b] < dt and T[a, b] < tw:
            pairs.append((int(a), b))
            dists.append(float(D[a, b]))
            S[:, b] = np.inf


def _match_windowed(tx, ty, tt, ix, iy, it, dt, tw, pairs, dists):
    order = np.argsort(it, kind="stable")
    its = it[order]
    taken = np.zeros(len(ix), dtype=bool)
    pad = 1e-9 * (1.0 + tw + float(np.max(np.abs(its))))
    for a in np.lexsort((np.arange(len(tx)), tt)):
        lo = int(np.searchsorted(its, tt[a] - tw - pad, "left"))
        hi = int(np.searchsorted(its, tt[a] + tw + pad, "right"))
        cand = order[lo:hi]
        cand = cand[~taken[cand]]
        if len(cand) == 0:
            continue
        D = np.hypot(ix[cand] - tx[a], iy[cand] - ty[a])
        T = np.abs(it[cand] - tt[a])
        S = np.maximum(D / dt, T / tw)
        k = np.nonzero(S == S.min())[0]
        k = k[np.argmin(cand[k])]              # the lowest index among the closest
        if D[k] < dt and T[k] < tw:
            b = int(cand[k])
            pairs.append((int(a), b))
            dists.append(float(D[k]))
            taken[b] = True


def autocovariance(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64) - np.mean(x)
    n = len(x)
    f = np.fft.rfft(x, 2 * n)
    acov = np.fft.irfft(f * np.conj(f))[:n] / n
    return acov


def ess(x: np.ndarray) -> float:
    """Effective sample size of a scalar chain (Geyer's initial monotone
    sequence).  A constant chain has ESS 1."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 4:
        return float(n)
    g = autocovariance(x)
    if g[0] <= 0.0:
        return 1.0
    npair = (n - 1) // 2
    gamma = g[0:2 * npair:2] + g[1:2 * npair + 1:2]  # Gamma_m = g(2m) + g(2m+1)
    pos = np.nonzero(gamma <= 0.0)[0]
    if len(pos):
        gamma = gamma[:pos[0]]
    if len(gamma) == 0:
        return float(n)
    gamma = np.minimum.accumulate(gamma)
    tau = -1.0 + 2.0 * np.sum(gamma) / g[0]  # integrated autocorrelation time
    tau = max(tau, 1.0 / n)
    return float(min(n / tau, n))


def bootstrap_ci(values, n_boot: int = 2000, level: float = 0.95, seed: int = 0):
    """Percentile bootstrap confidence interval of the mean (Section 5 reports
    95% bootstrap intervals over worlds and runs)."""
    v = np.asarray(values, dtype=np.float64)
    rng = np.random.default_rng(seed)
    means = v[rng.integers(0, len(v), size=(n_boot, len(v)))].mean(axis=1)
    lo, hi = np.quantile(means, [(1 - level) / 2, 1 - (1 - level) / 2])
    return float(v.mean()), float(lo), float(hi)


def match_states(true_ev, states, dist_thresh: float = DIST_THRESH,
                 time_thresh: float = TIME_THRESH, chunk_elems: int = 1 << 22) -> np.ndarray:
    """The matching of `match` applied to many inferred sets at once (the
    states of one chain against one truth): entry [s, a] is the index of the
    event of states[s] joined to true event a, or -1.  The states are padded
    to a common length and matched side by side with all separations at
    once, a few states per block."""
    tx, ty, tt = (np.asarray(true_ev[f], dtype=np.float64) for f in ("x", "y", "t"))
    nt, ns = len(tx), len(states)
    out = np.full((ns, nt), -1, dtype=np.int64)
    if nt == 0 or ns == 0:
        return out
    lens = np.array([len(ev["x"]) for ev in states])
    nmax = int(lens.max()) if ns else 0
    if nmax == 0:
        return out
    P = {f: np.full((ns, nmax), np.nan) for f in ("x", "y", "t")}
    for q, ev in enumerate(states):
        for f in P:
            P[f][q, :lens[q]] = ev[f]
    order = np.lexsort((np.arange(nt), tt))
    step = max(1, chunk_elems // (nt * nmax))
    for s0 in range(0, ns, step):
        sl = slice(s0, min(ns, s0 + step))
        D = np.hypot(P["x"][sl, None, :] - tx[None, :, None], P["y"][sl, None, :] - ty[None, :, None])
        T = np.abs(P["t"][sl, None, :] - tt[None, :, None])
        S = np.maximum(D / dist_thresh, T / time_thresh)
        S[np.isnan(S)] = np.inf                 # padding, like a taken event
        r = np.arange(S.shape[0])
        for a in order:
            b = np.argmin(S[:, a, :], axis=1)
            ok = np.isfinite(S[r, a, b]) & (D[r, a, b] < dist_thresh) & (T[r, a, b] < time_thresh)
            rs, bs = r[ok], b[ok]
            out[s0 + rs, a] = bs
            S[rs, :, bs] = np.inf
    return out


def location_ess(snapshots, truth, burn_frac: float = 0.25, min_matched: float = 0.9):
    """Event-location ESS of a chain: after burn-in, each recorded state is
    matched to the truth; every true event matched in at least `min_matched`
    of the states contributes the series of its matched x and y (gaps filled
    with the previous value) and min(ESS(x), ESS(y)).  Returns the median over
    those events (nan if none) and their count."""
    states = snapshots[int(len(snapshots) * burn_frac):]
    nt = len(truth["x"])
    if nt == 0 or not states:
        return float("nan"), 0
    xs = np.full((len(states), nt), np.nan)
    ys = np.full((len(states), nt), np.nan)
    idx = match_states(truth, states)
    for s, ev in enumerate(states):
        a = np.nonzero(idx[s] >= 0)[0]
        xs[s, a] = np.asarray(ev["x"])[idx[s, a]]
        ys[s, a] = np.asarray(ev["y"])[idx[s, a]]
    out = []
    for a in range(nt):
        ok = ~np.isnan(xs[:, a])
        if ok.mean() < min_matched:
            continue
        sx, sy = _ffill(xs[:, a]), _ffill(ys[:, a])
        out.append(min(ess(sx), ess(sy)))
    return (float(np.median(out)) if out else float("nan")), len(out)


def _ffill(v: np.ndarray) -> np.ndarray:
    ok = ~np.isnan(v)
    first = int(np.nonzero(ok)[0][0])
    last = np.maximum.accumulate(np.where(ok, np.arange(len(v)), first))
    return v[last]                     # each gap takes the value before it
