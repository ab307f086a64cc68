"""GPU parity of the naive parallel schedule (Algorithm 3, the paper's negative
control) against the oracle's: every region in one phase, each evaluating
against the phase-start state of the others plus its own changes, the
variance recomputed from the merged events afterwards.  Replayed sweeps
(events bit-exact after every sweep, log-likelihood changes within 1e-4,
the same decisions outside the tie band) on the paper's line world and on a
small grid world, batches, and the limits the schedule has."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1612_00595_amd import workloads as W  # noqa: E402

from gpu_cases import LogCheck, compare_events, compare_logs, instance, say  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def naive(w: W.Workload, **kw) -> W.Workload:
    return dataclasses.replace(w, name=w.name + "-naive",
                               sampler=dataclasses.replace(w.sampler, schedule=1, **kw))


def small_grid(tmpl=0) -> W.Workload:
    model = W.ModelSpec(nsx=3, nsy=3, N=200, lam=6.0, tmpl=tmpl)
    sampler = W.SamplerSpec(gx=3, gy=3, dynamic=0, k=16)
    return W.Workload(name="s3x3-n200-static3x3-f64", model=model, sampler=sampler,
                      trace_dtype="f64", sweeps=10, seed=4)


def _replay(w, nsw, feed_seed=71):
    from paper_1612_00595_amd import chromh
    m, sp, truth, s = instance(w)
    feed = W.feed_draws(w.sampler, nsw, seed=feed_seed)
    R, k = w.sampler.nreg, w.sampler.k
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), chains=1,
                                  seed=3)
    assert gpu.ncolors == 1
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
    gpu.set_log(glog, 0)
    ref = O.Chain(m, sp, s, seed=3)
    rlog = np.full((nsw, R, k, 4), -1.0)
    acc = LogCheck()
    for sw in range(nsw):
        assert ref.begin_sweep(sw) == 0
        assert ref.phase(sw, 0, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
        gpu.sweep_color(sw, 0)
        compare_events(gpu.read_events(0), ref.events(), f"sweep {sw}")
        if not compare_logs(glog[sw].cpu().numpy(), rlog[sw], feed[sw], acc, f"sweep {sw}"):
            say("decision tie at sweep", sw, "- stopping the bit-exact comparison")
            break
    ev = ref.events()
    E = gpu.read_variance(0)
    Er = O.event_variance(m, ev)
    if w.model.tmpl:
        Er = s - Er
        assert np.max(np.abs(E - Er)) <= 1e-10 * np.abs(s).max()
    else:
        assert np.all(np.abs(E - Er) <= 1e-9 * (w.model.sigma ** 2 + Er))
    return acc, ev


@pytest.mark.parametrize("dynamic", [0, 1])
def test_naive_replay_parity_line_world(dynamic):
    w = naive(W.PAPER1D, dynamic=dynamic)
    say("naive replay", w.name, "dynamic", dynamic)
    acc, ev = _replay(w, 10)
    say("moves", acc.moves, "evaluated", acc.evaluated)
    assert acc.evaluated > 10000 and len(ev) > 0


@pytest.mark.parametrize("tmpl", [0, 1])
def test_naive_replay_parity_small_grid(tmpl):
    w = naive(small_grid(tmpl))
    say("naive replay", w.name, "template", tmpl)
    acc, ev = _replay(w, 12)
    assert acc.evaluated > 500 and len(ev) > 0


def test_naive_batch_matches_single_runs():
    from paper_1612_00595_amd import chromh
    spec = W.PAPER1D_MODEL
    sampler = dataclasses.replace(W.PAPER1D_SAMPLER, schedule=1)
    traces = []
    for q in range(4):
        tr = W.truth_events(spec, 80 + q)
        traces.append(chromh.simulate(spec, chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"]),
                                      800 + q, "f64", DEV))
    b = chromh.Batch([spec] * 4, [sampler] * 4, traces, [5, 6, 7, 8])
    b.run_sweeps(0, 5)
    torch.cuda.synchronize()
    for q in range(4):
        one = chromh.ChromaticSampler(spec, sampler, traces[q], chains=1, seed=5 + q)
        one.run_sweeps(0, 5)
        ref = one.read_events(0)
        compare_events(b.read_events(q), ref, f"world {q}")
        assert np.array_equal(b.read_counters(q), one.read_counters(0))
        one.close()
    b.close()


def test_naive_limits_are_checked():
    from paper_1612_00595_amd import chromh
    w = naive(W.SMALL)  # 25 stations x 1000 samples: no private copy fits
    s = torch.zeros((w.model.nsta, w.model.N), dtype=torch.float64, device=DEV)
    with pytest.raises(chromh.CmhError):
        chromh.ChromaticSampler(w.model, w.sampler, s, seed=1)
    w2 = naive(W.PAPER1D)
    s2 = torch.zeros((w2.model.nsta, w2.model.N), dtype=torch.float64, device=DEV)
    with pytest.raises(chromh.CmhError):
        chromh.ChromaticSampler(w2.model, w2.sampler, s2, seed=1, block=256)
