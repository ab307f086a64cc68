"""GPU parity of the mean-template likelihood (each event adds a waveform to
the trace's mean; the state holds the residual) against the oracle, through
the C-ABI: the simulator, replayed sweeps (events bit-exact after every
colour phase, log-likelihood changes and log alpha within 1e-4, the same
decisions outside the tie band), the residual and the log-likelihood after
the run, batches, and the paper's line world under templates."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1612_00595_amd import workloads as W  # noqa: E402

from gpu_cases import (LogCheck, compare_events, compare_logs, dynamic_small,  # noqa: E402
                       instance, say)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def templ(w: W.Workload) -> W.Workload:
    return dataclasses.replace(w, name=w.name + "-tmpl",
                               model=dataclasses.replace(w.model, tmpl=1))


def test_template_simulator_matches_oracle():
    from paper_1612_00595_amd import chromh
    w = templ(W.SMALL)
    m = O.make_model(**w.model.asdict())
    tr = W.truth_events(w.model, 3)
    truth = O.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    ref = O.simulate(m, truth, 55)
    say("template simulate small f64/f32")
    g64 = chromh.simulate(w.model, truth, 55, "f64", DEV).cpu().numpy()
    assert np.allclose(g64, ref, rtol=1e-12, atol=1e-14)
    g32 = chromh.simulate(w.model, truth, 55, "f32", DEV).cpu().numpy()
    r32 = ref.astype(np.float32)
    assert np.all(np.abs(g32 - r32) <= np.spacing(np.abs(r32)))


def _replay(w, nsw, block, feed_seed=77):
    from paper_1612_00595_amd import chromh
    m, sp, truth, s = instance(w)
    feed = W.feed_draws(w.sampler, nsw, seed=feed_seed)
    R, k = w.sampler.nreg, w.sampler.k
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), chains=1,
                                  seed=3, block=block)
    # the empty world's residual is the trace itself
    r0 = gpu.read_variance(0)
    assert np.array_equal(r0, s.astype(np.float64))
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
    gpu.set_log(glog, 0)
    ref = O.Chain(m, sp, s, seed=3)
    rlog = np.full((nsw, R, k, 4), -1.0)
    acc = LogCheck()
    for sw in range(nsw):
        assert ref.begin_sweep(sw) == 0
        for c in range(gpu.ncolors):
            assert ref.phase(sw, c, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
            gpu.sweep_color(sw, c)
            compare_events(gpu.read_events(0), ref.events(), f"sweep {sw} colour {c}")
        if not compare_logs(glog[sw].cpu().numpy(), rlog[sw], feed[sw], acc, f"sweep {sw}"):
            say("decision tie at sweep", sw, "- stopping the bit-exact comparison")
            break
    return gpu, ref, m, s, acc


def _check_state(gpu, ref, m, s):
    ev = ref.events()
    assert len(ev) > 0
    resid = s.astype(np.float64) - O.event_variance(m, ev)
    got = gpu.read_variance(0)
    scale = np.abs(s).max()
    assert np.max(np.abs(got - resid)) <= 1e-10 * scale
    ll = gpu.refresh(write_variance=False, loglik=True)[0]
    assert ll == pytest.approx(O.loglik(m, s, ev), rel=1e-10)


@pytest.mark.parametrize("block", [64, 256, 1024 + 256])
def test_template_replay_parity_small_static(block):
    w = templ(W.SMALL)
    say("template replay", w.name, "block", block)
    gpu, ref, m, s, acc = _replay(w, 12, block)
    say("moves", acc.moves, "evaluated", acc.evaluated, "ties", acc.ties, "max rel", acc.max_rel)
    assert acc.evaluated > 1000
    _check_state(gpu, ref, m, s)


@pytest.mark.parametrize("block", [64, 256, 1024 + 512])
def test_template_replay_parity_dynamic(block):
    w = templ(dynamic_small())
    say("template replay", w.name, "block", block)
    gpu, ref, m, s, acc = _replay(w, 8, block)
    assert acc.evaluated > 5000
    _check_state(gpu, ref, m, s)


def test_template_replay_parity_line_world():
    w = templ(dataclasses.replace(W.PAPER1D, sampler=dataclasses.replace(W.PAPER1D.sampler,
                                                                         dynamic=1)))
    say("template replay", w.name)
    gpu, ref, m, s, acc = _replay(w, 6, 64)
    assert acc.evaluated > 5000
    _check_state(gpu, ref, m, s)


def test_template_batch_matches_single_runs():
    from paper_1612_00595_amd import chromh
    specs = [dataclasses.replace(W.ModelSpec(nsx=6, nsy=6, N=2000, lam=60.0), tmpl=1),
             dataclasses.replace(W.ModelSpec(nsx=9, nsy=5, N=2500, lam=70.0), tmpl=1)]
    samplers = [W.SamplerSpec(gx=mm.nsx, gy=mm.nsy, dynamic=1) for mm in specs]
    traces = []
    for q, mm in enumerate(specs):
        tr = W.truth_events(mm, 40 + q)
        traces.append(chromh.simulate(mm, chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"]),
                                      500 + q, "f32", DEV))
    b = chromh.Batch(specs, samplers, traces, [11, 12], block=64)
    b.run_sweeps(0, 6)
    torch.cuda.synchronize()
    for q, mm in enumerate(specs):
        one = chromh.ChromaticSampler(mm, samplers[q], traces[q], chains=1, seed=11 + q,
                                      block=256)
        one.run_sweeps(0, 6)
        ref = one.read_events(0)
        assert len(ref) > 0
        compare_events(b.read_events(q), ref, f"instance {q}")
        assert np.array_equal(b.read_counters(q), one.read_counters(0))
        one.close()
    b.close()


def test_template_learned_births_are_rejected():
    from paper_1612_00595_amd import chromh
    w = templ(W.SMALL)
    s = torch.zeros((w.model.nsta, w.model.N), dtype=torch.float64, device=DEV)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, s, seed=1)
    T, wts, ntau = W.random_mixture_table(W.SMALL.model, 1)
    with pytest.raises(chromh.CmhError):
        gpu.set_learned(torch.from_numpy(T).to(DEV), torch.from_numpy(wts).to(DEV), ntau)
    gpu.run_sweeps(0, 2)
    torch.cuda.synchronize()
