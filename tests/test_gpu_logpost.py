"""Exact refresh and the full log-probability (Section 3's joint density of
events and signals) on the GPU, against the oracle: the log-likelihood and
log prior of given event sets, the scheduled refresh inside replayed sweep
graphs with its log-probability records, and the drift of the in-place
variance over a long run.

Bars: log-likelihood and log prior within 1e-12 relative of the oracle's
(fp64 sums in a different order); the refreshed variance within 1e-12 of
sigma^2 + E of the oracle's direct sum; after 2000 incremental sweeps the
in-place variance within 1e-9 of an exact refresh (the replay bar).
"""
import dataclasses

import numpy as np
import pytest

from gpu_cases import LogCheck, compare_events, compare_logs, dynamic_small, instance, say

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_1612_00595_amd import chromh, workloads as W  # noqa: E402

DEV = "cuda:0"


def _with(w, **kw):
    return dataclasses.replace(w, sampler=dataclasses.replace(w.sampler, **kw))


def _close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(b), 1.0)


@pytest.mark.parametrize("name", ["grid", "grid-template", "line", "line-latent"])
def test_log_posterior_of_an_event_set_matches_oracle(name):
    if name.startswith("grid"):
        w = dynamic_small()
        if name == "grid-template":
            w = dataclasses.replace(w, model=dataclasses.replace(w.model, tmpl=1))
    else:
        w = W.PAPER1D_LATENT if name == "line-latent" else W.PAPER1D
    m, sp, truth, s = instance(w)
    st = W.random_state(w.model, 5, 40 if w.model.line else 200)
    ev = O.as_events(st["x"], st["y"], st["t"], st["m"], st["id"], da=st.get("da"))
    say("log posterior", name, "events", len(ev))
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=1)
    gpu.write_events(0, ev)
    lp = gpu.log_posterior()[0]
    ll_ref, pr_ref = O.loglik(m, s, ev), O.logprior(m, ev)
    assert _close(lp[0], ll_ref), (lp[0], ll_ref)
    assert _close(lp[1], pr_ref), (lp[1], pr_ref)
    assert lp[2] == lp[0] + lp[1]
    # the empty world: only -lambda and the noise
    gpu.write_events(0, O.events_array(0))
    lp0 = gpu.log_posterior()[0]
    assert _close(lp0[1], -w.model.lam)
    assert _close(lp0[0], O.loglik(m, s, O.events_array(0)))
    gpu.close()


def test_log_posterior_of_a_batch_matches_oracle():
    specs = [W.ModelSpec(nsx=6, nsy=6, N=2000, lam=60.0), W.ModelSpec(nsx=9, nsy=5, N=2500, lam=70.0),
             W.PAPER1D.model]
    samplers = [W.SamplerSpec(gx=m.nsx, gy=m.nsy, dynamic=1) for m in specs[:2]]
    samplers.append(dataclasses.replace(W.PAPER1D.sampler, dynamic=1, k=samplers[0].k))
    traces, states = [], []
    for q, m in enumerate(specs):
        om = O.make_model(**m.asdict())
        tr = W.truth_events(m, 40 + q)
        s = O.simulate(om, O.as_events(tr["x"], tr["y"], tr["t"], tr["m"]), 500 + q)
        traces.append(torch.from_numpy(s).to(DEV))
        st = W.random_state(m, 70 + q, 30)
        states.append(O.as_events(st["x"], st["y"], st["t"], st["m"], st["id"]))
    say("log posterior of a batch of three uneven worlds")
    b = chromh.Batch(specs, samplers, traces, [1, 2, 3])
    for q in range(3):
        b.write_events(q, states[q])
    lp = b.log_posterior()
    for q, m in enumerate(specs):
        om = O.make_model(**m.asdict())
        s = traces[q].cpu().numpy()
        assert _close(lp[q, 0], O.loglik(om, s, states[q])), q
        assert _close(lp[q, 1], O.logprior(om, states[q])), q
    b.close()


@pytest.mark.parametrize("block", [64, 256, chromh.SPEC4])
def test_scheduled_refresh_in_replay_matches_oracle(block):
    """refresh_every = 3 in a replayed dynamic run: events bit-exact against
    the oracle, the log-probability records at every third sweep equal the
    oracle's log-likelihood and log prior of that sweep's events, and the
    variance after a refresh sweep is the exact one."""
    w = _with(dynamic_small(), refresh_every=3)
    m, sp, truth, s = instance(w)
    nsw = 7
    feed = W.feed_draws(w.sampler, nsw, seed=17)
    R, k = w.sampler.nreg, w.sampler.k
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=3,
                                  block=block)
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    rec = gpu.set_logprob(0, nsw)
    glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
    gpu.set_log(glog, 0)
    ref = O.Chain(m, sp, s, seed=3)
    rlog = np.full((nsw, R, k, 4), -1.0)
    acc = LogCheck()
    say("scheduled refresh, form", block)
    for sw in range(nsw):
        assert ref.sweep(sw, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
        gpu.run_sweeps(sw, 1)
        ev = ref.events()
        compare_events(gpu.read_events(0), ev, f"sweep {sw}")
        assert compare_logs(glog[sw].cpu().numpy(), rlog[sw], feed[sw], acc, f"sweep {sw}")
        row = rec[sw, 0].cpu().numpy()
        if (sw + 1) % 3 == 0:
            assert _close(row[0], O.loglik(m, s, ev)), sw
            assert _close(row[1], O.logprior(m, ev)), sw
            Er = O.event_variance(m, ev)
            assert np.all(np.abs(gpu.read_variance(0) - Er) <= 1e-12 * (0.01 + Er)), sw
        else:
            assert np.all(np.isnan(row)), sw
    assert acc.evaluated > 2000
    gpu.close()


def test_scheduled_refresh_in_graph_replays_of_a_batch():
    """The refresh inside graph-replayed sweeps of several chains: records
    only at refresh sweeps, each equal to a direct log-posterior of the
    chain's state right after that sweep."""
    w = _with(dynamic_small(), refresh_every=2)
    m, sp, truth, s = instance(w)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), chains=3,
                                  seed=8)
    rec = gpu.set_logprob(4, 4)
    gpu.run_sweeps(0, 6)                   # refreshes after sweeps 1, 3, 5
    lp5 = gpu.log_posterior()              # the state after sweep 5
    gpu.run_sweeps(6, 2)
    r = rec.cpu().numpy()
    assert np.all(np.isnan(r[0])) and np.all(np.isnan(r[2]))      # sweeps 4, 6
    assert np.all(np.isfinite(r[1])) and np.all(np.isfinite(r[3]))  # sweeps 5, 7
    for c in range(3):
        assert _close(r[1, c, 0], lp5[c, 0]) and _close(r[1, c, 1], lp5[c, 1]), c
    gpu.close()


def test_in_place_variance_drift_over_2000_sweeps():
    """The 5x5-station, 1000-sample fp64 workload for its full 2000 sweeps
    without a scheduled refresh: the in-place variance then still equals an
    exact refresh within 1e-9 relative to sigma^2 + E."""
    w = W.SMALL
    m, sp, truth, s = instance(w)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=0)
    say("drift run", w.name, w.sweeps, "sweeps")
    gpu.run_sweeps(0, w.sweeps)
    E_inc = gpu.read_variance(0)
    st = gpu.read_stats(0)
    assert st[:, 2].sum() > 10000              # many accepted rewrites of E
    gpu.refresh(write_variance=True, loglik=False)
    E_ref = gpu.read_variance(0)
    err = np.abs(E_inc - E_ref) / (0.01 + E_ref)
    say("max relative drift", err.max())
    assert err.max() <= 1e-9
    gpu.close()
