"""GPU parity of the learned birth proposal against the oracle: 16-wide draw
records, the mixture-table builder, replayed sweeps with learned births
(events bit-exact after every colour phase, log alpha within 1e-4, the same
decisions outside the tie band), prior-only stationarity of the GPU chains
with learned births drawn from the device generator, and learned births per
instance of a batch."""
import numpy as np
import pytest
from scipy import stats

torch = pytest.importorskip("torch")

import oracle as O
from oracle import mdn as D
from paper_1612_00595_amd import workloads as W

from gpu_cases import LogCheck, compare_events, compare_logs, dynamic_small, instance, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_00595_amd import chromh  # noqa: F401


def test_move_draws16_match_oracle():
    from paper_1612_00595_amd import chromh
    for seed, chain, sweep, region in [(0, 0, 0, 0), (7, 3, 11, 4224), (2**31, 31, 499, 17)]:
        say("draws16", seed, chain, sweep, region)
        g = chromh.move_draws(seed, chain, sweep, region, 0, 300, width=16)
        r = np.array([O.move_draws16(seed, chain, sweep, region, j) for j in range(300)])
        for c in (0, 1, 2, 3, 8, 9, 10, 14, 15):   # integer-derived or zero: exact
            assert np.array_equal(g[:, c], r[:, c]), c
        assert np.allclose(g, r, rtol=1e-14, atol=1e-15)


def test_mixture_table_matches_oracle():
    from paper_1612_00595_amd import chromh
    spec = dynamic_small().model
    na, ntau = chromh.anchor_count(spec)
    rng = np.random.default_rng(3)
    first, rows = 1000, 777
    head = rng.normal(0, 2.0, (rows, 64)).astype(np.float32)
    head[:, 56:] = 0
    say("mixture table rows", rows)
    T = chromh.mixture_table(spec, torch.from_numpy(head).to(DEV), first).cpu().numpy()
    R = D.mixture_table(head, spec.nsx, spec.ds, ntau, first)
    assert np.allclose(T, R, rtol=1e-13, atol=1e-13)
    assert np.allclose(T[:, -1, 7], 1.0, atol=1e-12)


def _learned_replay(w, nsw, block, table_seed, feed_seed=55, p_learned=0.5):
    from paper_1612_00595_amd import chromh
    m, sp, truth, s = instance(w)
    T, wts, ntau = W.random_mixture_table(w.model, table_seed, near=truth)
    feed = W.feed_draws(w.sampler, nsw, seed=feed_seed, learned=True)
    R, k = w.sampler.nreg, w.sampler.k
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), chains=1,
                                  seed=3, block=block)
    gpu.set_learned(torch.from_numpy(T).to(DEV), torch.from_numpy(wts).to(DEV), ntau, p_learned)
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
    gpu.set_log(glog, 0)
    ref = O.Chain(m, sp, s, seed=3)
    assert ref.set_learned(T, wts, ntau, p_learned) == 0
    rlog = np.full((nsw, R, k, 4), -1.0)
    acc = LogCheck()
    births = 0
    for sw in range(nsw):
        assert ref.begin_sweep(sw) == 0
        for c in range(gpu.ncolors):
            assert ref.phase(sw, c, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
            gpu.sweep_color(sw, c)
            compare_events(gpu.read_events(0), ref.events(), f"sweep {sw} colour {c}")
        gl = glog[sw].cpu().numpy()
        births += int(np.sum((rlog[sw][..., 0] == 0) & (rlog[sw][..., 1] == 2)))
        if not compare_logs(gl, rlog[sw], feed[sw], acc, f"sweep {sw}"):
            say("decision tie at sweep", sw, "- stopping the bit-exact comparison")
            break
    return acc, births


@pytest.mark.parametrize("block", [64, 128, 256, 1024 + 256])
def test_learned_replay_parity_small_static(block):
    say("learned replay", W.SMALL.name, "block", block)
    acc, births = _learned_replay(W.SMALL, 12, block, table_seed=11)
    say("moves", acc.moves, "evaluated", acc.evaluated, "accepted births", births)
    assert acc.evaluated > 1000 and births > 20


def test_learned_replay_parity_dynamic():
    w = dynamic_small()
    say("learned replay", w.name)
    acc, births = _learned_replay(w, 6, 256, table_seed=12)
    say("moves", acc.moves, "evaluated", acc.evaluated, "accepted births", births)
    assert acc.evaluated > 3000 and births > 50


def test_learned_feed_width_is_checked():
    from paper_1612_00595_amd import chromh
    w = W.SMALL
    m, sp, truth, s = instance(w)
    T, wts, ntau = W.random_mixture_table(w.model, 1)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=3)
    gpu.set_learned(torch.from_numpy(T).to(DEV), torch.from_numpy(wts).to(DEV), ntau)
    gpu.set_feed(torch.from_numpy(W.feed_draws(w.sampler, 1, seed=1)).to(DEV), 0)
    with pytest.raises(chromh.CmhError):
        gpu.sweep_color(0, 0)
    gpu.set_feed(None, 0)
    gpu.set_learned(None, None, 0)
    gpu.run_sweeps(0, 2)
    torch.cuda.synchronize()


def test_learned_prior_only_gpu_samples_the_prior():
    """Prior-only chains with learned births from the device generator
    (graph-replayed sweeps, 8 chains): the event count is Poisson(20) and
    the events are uniform / Exp(1) + 2, as in the oracle's test."""
    from paper_1612_00595_amd import chromh
    spec = W.SMALL.model
    sampler = W.SamplerSpec(**dict(W.SMALL.sampler.asdict(), prior_only=1, k=8))
    T, wts, ntau = W.random_mixture_table(spec, 6)
    T[..., 3:5] = 0.05
    T[..., 5] = 60.0
    s = torch.zeros((spec.nsta, spec.N), dtype=torch.float64, device=DEV)
    chains = 8
    gpu = chromh.ChromaticSampler(spec, sampler, s, chains=chains, seed=21)
    gpu.set_learned(torch.from_numpy(T).to(DEV), torch.from_numpy(wts).to(DEV), ntau)
    say("prior-only learned: 8 chains x 6000 sweeps")
    counts = [[] for _ in range(chains)]
    xs, ys, ts, ms = [], [], [], []
    gpu.run_sweeps(0, 100)
    for blk in range(1, 60):
        gpu.run_sweeps(100 * blk, 100)
        for c in range(chains):
            ev = gpu.read_events(c)
            counts[c].append(len(ev))
            xs.append(ev["x"]); ys.append(ev["y"]); ts.append(ev["t"]); ms.append(ev["m"])
    cnt = np.array(counts, dtype=float)         # [chain, snapshot], snapshots 100 sweeps apart
    lam = spec.lam
    se = cnt.std() / np.sqrt(cnt.size)
    say("count mean", cnt.mean(), "se", se, "var", cnt.var())
    assert abs(cnt.mean() - lam) < 4.5 * se
    assert 0.8 * lam < cnt.var() < 1.25 * lam
    x, y, t, mm = (np.concatenate(a) for a in (xs, ys, ts, ms))
    assert stats.kstest(x / spec.Lx, "uniform").pvalue > 1e-3
    assert stats.kstest(y / spec.Ly, "uniform").pvalue > 1e-3
    assert stats.kstest(t / spec.N, "uniform").pvalue > 1e-3
    assert stats.kstest(mm - 2.0, "expon").pvalue > 1e-3
    st = gpu.read_stats(0)
    say("birth attempts / accepted", st[0, 0], st[0, 2])
    assert st[0, 2] > 10000


@pytest.mark.parametrize("block", [64, 256, 1024 + 256])
def test_learned_births_in_a_batch_match_single_runs(block):
    """Instances of an uneven batch carry their own learned tables (one stays
    plain); each follows its one-chain run with the same table bit for bit."""
    from paper_1612_00595_amd import chromh
    specs = [W.ModelSpec(nsx=5, nsy=5, N=1000, lam=20.0), W.ModelSpec(nsx=6, nsy=6, N=1200, lam=30.0),
             W.ModelSpec(nsx=4, nsy=4, N=900, lam=14.0)]
    samplers = [W.SamplerSpec(gx=m.nsx, gy=m.nsy, dynamic=1) for m in specs]
    traces, tables = [], []
    for q, m in enumerate(specs):
        tr = W.truth_events(m, 70 + q)
        truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
        traces.append(chromh.simulate(m, truth, 700 + q, "f64", DEV))
        T, wts, ntau = W.random_mixture_table(m, 10 + q, near=O.as_events(tr["x"], tr["y"],
                                                                            tr["t"], tr["m"]))
        tables.append((torch.from_numpy(T).to(DEV), torch.from_numpy(wts).to(DEV), ntau))
    say("learned batch of", len(specs), "instances (instance 1 plain)")
    b = chromh.Batch(specs, samplers, traces, [31, 32, 33], block=block)
    for q in (0, 2):
        b.set_learned_instance(q, *tables[q], p_learned=0.5)
    b.run_sweeps(0, 12)
    torch.cuda.synchronize()
    for q, m in enumerate(specs):
        one = chromh.ChromaticSampler(m, samplers[q], traces[q], chains=1, seed=31 + q, block=block)
        if q != 1:
            one.set_learned(*tables[q], p_learned=0.5)
        one.run_sweeps(0, 12)
        compare_events(b.read_events(q), one.read_events(0), f"instance {q}")
        assert np.array_equal(b.read_counters(q), one.read_counters(0))
        one.close()
    st = b.read_stats(0)
    assert st[0, 2] > 0
    # back to plain births for instance 0: it then matches a plain single run
    b.set_learned_instance(0, None, None, 0)
    b.close()


@pytest.mark.parametrize("block", [64, 256, 1024 + 256])
def test_region_with_too_many_stations_is_reported(block):
    """A region holding more than 16 stations cannot take learned births:
    the learned-birth kernel and every sweep form report it and the run ends
    in CMH_ESTATE (10 x 10 stations in 2 x 2 regions: about 25 per region)."""
    import dataclasses
    from paper_1612_00595_amd import chromh
    m = W.ModelSpec(nsx=10, nsy=10, N=1000, lam=10.0)
    sp = dataclasses.replace(W.SMALL.sampler, gx=2, gy=2)
    tr = W.truth_events(m, 3)
    trace = chromh.simulate(m, chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"]), 30,
                            "f64", DEV)
    T, wts, ntau = W.random_mixture_table(m, 4)
    say("learned births with 25 stations per region, form", block)
    gpu = chromh.ChromaticSampler(m, sp, trace, chains=1, seed=5, block=block)
    gpu.set_learned(torch.from_numpy(T).to(DEV), torch.from_numpy(wts).to(DEV), ntau, 0.5)
    with pytest.raises(chromh.CmhError, match="more stations"):
        gpu.run_sweeps(0, 1)
        torch.cuda.synchronize()
        gpu.read_events(0)
    gpu.close()
