"""GPU parity of the line model (the paper's 1-D world, Section 3 as printed,
partitioned in onset time, Section 4.1) against the oracle, through the
C-ABI: the simulator, replayed sweeps at the paper's k = 500 moves per region
(events bit-exact after every colour phase, log-likelihood changes and log
alpha within 1e-4, the same decisions outside the tie band, variance and
log-likelihood after the run), prior-only stationarity, and batches of
worlds that follow their single runs exactly."""
import dataclasses

import numpy as np
import pytest
from scipy import stats

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


def test_line_simulator_matches_oracle():
    from paper_1612_00595_amd import chromh
    spec = W.PAPER1D_MODEL
    m = O.make_model(**spec.asdict())
    for seed in (3, 4, 5):
        tr = W.truth_events(spec, seed)
        truth = O.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
        say("line simulate seed", seed, "events", len(truth))
        ref = O.simulate(m, truth, 70 + seed)
        g64 = chromh.simulate(spec, truth, 70 + seed, "f64", DEV).cpu().numpy()
        assert np.allclose(g64, ref, rtol=1e-12, atol=1e-15)
        g32 = chromh.simulate(spec, truth, 70 + seed, "f32", DEV).cpu().numpy()
        r32 = ref.astype(np.float32)
        assert np.all(np.abs(g32 - r32) <= np.spacing(np.abs(r32)))


def _line_replay(w, nsw, block, feed_seed=31):
    from paper_1612_00595_amd import chromh
    m, sp, truth, s = instance(w)
    feed = W.feed_draws(w.sampler, nsw, seed=feed_seed)
    R, k = w.sampler.nreg, w.sampler.k
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), chains=1,
                                  seed=3, block=block)
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
    gpu.set_log(glog, 0)
    ref = O.Chain(m, sp, s, seed=3)
    rlog = np.full((nsw, R, k, 4), -1.0)
    acc = LogCheck()
    for sw in range(nsw):
        assert ref.begin_sweep(sw) == 0
        assert ref.layout()["ncolors"] == gpu.ncolors
        for c in range(gpu.ncolors):
            assert ref.phase(sw, c, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
            gpu.sweep_color(sw, c)
            compare_events(gpu.read_events(0), ref.events(), f"sweep {sw} colour {c}")
        if not compare_logs(glog[sw].cpu().numpy(), rlog[sw], feed[sw], acc, f"sweep {sw}"):
            say("decision tie at sweep", sw, "- stopping the bit-exact comparison")
            break
    return gpu, ref, m, s, acc


@pytest.mark.parametrize("dynamic", [0, 1])
@pytest.mark.parametrize("block", [64, 256, 1024 + 256])
def test_line_replay_parity(block, dynamic):
    w = dataclasses.replace(W.PAPER1D, sampler=dataclasses.replace(W.PAPER1D.sampler,
                                                                   dynamic=dynamic))
    say("line replay", w.name, "dynamic", dynamic, "block", block)
    gpu, ref, m, s, acc = _line_replay(w, 10, block)
    say("moves", acc.moves, "evaluated", acc.evaluated, "ties", acc.ties, "max rel", acc.max_rel)
    assert acc.evaluated > 10000
    ev = ref.events()
    assert len(ev) > 0
    E = gpu.read_variance(0)
    Er = O.event_variance(m, ev)
    assert np.all(np.abs(E - Er) <= 1e-9 * (w.model.sigma ** 2 + Er))
    ll = gpu.refresh(write_variance=False, loglik=True)[0]
    assert ll == pytest.approx(O.loglik(m, s, ev), rel=1e-10)


def test_line_prior_only_gpu_samples_the_prior():
    from paper_1612_00595_amd import chromh
    spec = dataclasses.replace(W.PAPER1D_MODEL, lam=12.0)
    sampler = dataclasses.replace(W.PAPER1D_SAMPLER, prior_only=1, dynamic=1, k=6, sxy=20.0,
                                  st=30.0)
    s = torch.zeros((spec.nsta, spec.N), dtype=torch.float64, device=DEV)
    chains = 8
    gpu = chromh.ChromaticSampler(spec, sampler, s, chains=chains, seed=21)
    say("line prior-only: 8 chains x 6000 sweeps")
    gpu.run_sweeps(0, 100)
    counts, xs, ts = [[] for _ in range(chains)], [], []
    for blk in range(1, 120):
        gpu.run_sweeps(50 * blk + 50, 50)
        for c in range(chains):
            ev = gpu.read_events(c)
            counts[c].append(len(ev))
            xs.append(ev["x"]); ts.append(ev["t"])
            assert np.all(ev["y"] == 0.0) and np.all(ev["m"] == spec.mmin)
    cnt = np.array(counts, dtype=float)
    se = cnt.std() / np.sqrt(cnt.size)
    say("count mean", cnt.mean(), "se", se, "var", cnt.var())
    assert abs(cnt.mean() - spec.lam) < 4.5 * se
    assert 0.8 * spec.lam < cnt.var() < 1.25 * spec.lam
    x, t = np.concatenate(xs), np.concatenate(ts)
    assert stats.kstest(x / spec.xmax, "uniform").pvalue > 1e-3
    assert stats.kstest(t / spec.N, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("block", [64, 256])
def test_line_batch_of_worlds_matches_single_runs(block):
    from paper_1612_00595_amd import chromh
    spec, sampler = W.PAPER1D_MODEL, dataclasses.replace(W.PAPER1D_SAMPLER, dynamic=1)
    n = 6
    traces, specs, samplers, seeds = [], [], [], []
    for q in range(n):
        tr = W.truth_events(spec, 60 + q)
        truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
        traces.append(chromh.simulate(spec, truth, 600 + q, "f64", DEV))
        specs.append(spec); samplers.append(sampler); seeds.append(90 + q)
    say("line batch of", n, "worlds, block", block)
    b = chromh.Batch(specs, samplers, traces, seeds, block=block)
    b.run_sweeps(0, 5)
    torch.cuda.synchronize()
    for q in range(n):
        one = chromh.ChromaticSampler(spec, sampler, traces[q], chains=1, seed=seeds[q],
                                      block=256)
        one.run_sweeps(0, 5)
        ref = one.read_events(0)
        compare_events(b.read_events(q), ref, f"world {q}")
        assert np.array_equal(b.read_counters(q), one.read_counters(0))
        one.close()
    b.close()


def test_line_learned_births_are_rejected():
    from paper_1612_00595_amd import chromh
    spec = W.PAPER1D_MODEL
    s = torch.zeros((spec.nsta, spec.N), dtype=torch.float64, device=DEV)
    gpu = chromh.ChromaticSampler(spec, W.PAPER1D_SAMPLER, s, seed=1)
    T = torch.zeros((spec.nsta * 5, 8, 8), dtype=torch.float64, device=DEV)
    w = torch.ones(spec.nsta * 5, dtype=torch.float64, device=DEV)
    with pytest.raises(chromh.CmhError):
        gpu.set_learned(T, w, 5)
    gpu.run_sweeps(0, 2)
    torch.cuda.synchronize()
