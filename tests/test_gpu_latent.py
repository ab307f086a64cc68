"""GPU parity of latent arrival times (Section 3's arrival density) on the line
model, with the arrival-time move and the joint two-event move, against the
oracle through the C-ABI: the 16-wide draw records, the simulator with
per-event offsets, replayed sweeps (events with their offsets bit-exact after
every colour phase, log-likelihood changes and log alpha within 1e-4, the same
decisions outside the tie band) on the paper's world and on a two-station
world where the joint move is often accepted, batches, prior-only
stationarity, and the limits of the mode."""
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


def two_station() -> W.Workload:
    model = dataclasses.replace(W.PAPER1D_LATENT_MODEL, nsx=2, sta_x=(0.0, 100.0), lam=10.0)
    sampler = dataclasses.replace(W.PAPER1D_LATENT_SAMPLER, gx=2, pj=0.3, pa=0.1, ploc=0.15,
                                  pt=0.15, k=200)
    return W.Workload(name="line2-x100-n240-latent", model=model, sampler=sampler,
                      trace_dtype="f64", sweeps=10, seed=8)


def test_latent_draw_records_match_oracle():
    from paper_1612_00595_amd import chromh
    for seed, chain, sweep, region in [(0, 0, 0, 0), (7, 3, 11, 4), (2**31, 31, 499, 17)]:
        say("latent draws", seed, chain, sweep, region)
        g = chromh.move_draws_arrivals(seed, chain, sweep, region, 0, 300)
        r = np.array([O.move_draws_arr(seed, chain, sweep, region, j) for j in range(300)])
        assert np.array_equal(g[:, :4], r[:, :4])
        assert np.allclose(g[:, 4:], r[:, 4:], rtol=1e-14, atol=1e-14)


def test_latent_simulator_matches_oracle():
    from paper_1612_00595_amd import chromh
    spec = W.PAPER1D_LATENT_MODEL
    m = O.make_model(**spec.asdict())
    for seed in (3, 4):
        tr = W.truth_events(spec, seed)
        truth = O.as_events(tr["x"], tr["y"], tr["t"], tr["m"], da=tr["da"])
        assert np.any(truth["da"] != 0.0)
        say("latent simulate seed", seed, "events", len(truth))
        ref = O.simulate(m, truth, 70 + seed)
        g64 = chromh.simulate(spec, truth, 70 + seed, "f64", DEV).cpu().numpy()
        assert np.allclose(g64, ref, rtol=1e-12, atol=1e-15)


def _early_arrivals(model, ev) -> int:
    """Events of ev with an arrival at least one sample before the trace."""
    n = 0
    for e in ev:
        a = [e["t"] + abs(e["x"] - sx) / model.vel + e["da"][j] for j, sx in enumerate(model.sta_x)]
        n += min(np.ceil(a)) < 0
    return n


def _replay(w, nsw, feed_seed=41, block=0, inst=None, early=None, start=None):
    from paper_1612_00595_amd import chromh
    m, sp, truth, s = instance(w) if inst is None else inst
    feed = W.feed_draws(w.sampler, nsw, seed=feed_seed, latent=True)
    R, k = w.sampler.nreg, w.sampler.k
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), chains=1,
                                  seed=3, block=block)
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
    gpu.set_log(glog, 0)
    ref = O.Chain(m, sp, s, seed=3)
    if start is not None:  # both chains start from the same events
        gpu.write_events(0, start)
        assert ref.set_events(start) == 0
    rlog = np.full((nsw, R, k, 4), -1.0)
    acc = LogCheck()
    for sw in range(nsw):
        assert ref.begin_sweep(sw) == 0
        assert ref.layout()["ncolors"] == gpu.ncolors
        for c in range(gpu.ncolors):
            assert ref.phase(sw, c, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
            gpu.sweep_color(sw, c)
            compare_events(gpu.read_events(0), ref.events(), f"sweep {sw} colour {c}")
            if early is not None:
                early.append(_early_arrivals(w.model, ref.events()))
        if not compare_logs(glog[sw].cpu().numpy(), rlog[sw], feed[sw], acc, f"sweep {sw}"):
            say("decision tie at sweep", sw, "- stopping the bit-exact comparison")
            break
    types = rlog[..., 0]
    status = rlog[..., 1]
    return gpu, ref, m, s, acc, types, status


def _check_state(gpu, ref, m, s, w):
    ev = ref.events()
    assert len(ev) > 0
    E = gpu.read_variance(0)
    Er = O.event_variance(m, ev)
    assert np.all(np.abs(E - Er) <= 1e-9 * (w.model.sigma ** 2 + Er))
    ll = gpu.refresh(write_variance=False, loglik=True)[0]
    assert ll == pytest.approx(O.loglik(m, s, ev), rel=1e-10)


@pytest.mark.parametrize("dynamic", [0, 1])
@pytest.mark.parametrize("block", [64, 256])
def test_latent_replay_parity_paper_world(block, dynamic):
    w = dataclasses.replace(W.PAPER1D_LATENT, sampler=dataclasses.replace(
        W.PAPER1D_LATENT.sampler, dynamic=dynamic))
    say("latent replay", w.name, "dynamic", dynamic, "block", block)
    gpu, ref, m, s, acc, types, status = _replay(w, 8, block=block)
    acc_arr = int(((types == O.ARR) & (status == 2)).sum())
    say("moves", acc.moves, "evaluated", acc.evaluated, "ties", acc.ties, "max rel", acc.max_rel,
        "arrival moves accepted", acc_arr, "joint valid", int(((types == O.JOINT) & (status > 0)).sum()))
    assert gpu.ncolors == 3
    assert acc.evaluated > 10000 and acc_arr > 50
    _check_state(gpu, ref, m, s, w)


@pytest.mark.parametrize("block", [64, 256])
def test_latent_replay_parity_joint_moves(block):
    w = two_station()
    say("latent replay", w.name, "block", block)
    gpu, ref, m, s, acc, types, status = _replay(w, 10, block=block)
    joint_acc = int(((types == O.JOINT) & (status == 2)).sum())
    say("moves", acc.moves, "evaluated", acc.evaluated, "joint accepted", joint_acc)
    assert joint_acc >= 20
    _check_state(gpu, ref, m, s, w)
    st = gpu.read_stats(0)
    assert st[6, 2] >= 20 and st[5, 2] > 0


def early_world():
    """The paper's line with a wide offset prior (sd 3, so offsets reach 12
    samples) and true events at the very start of the trace whose arrivals
    at the nearest stations precede the first sample."""
    model = dataclasses.replace(W.PAPER1D_LATENT_MODEL, arr_sd=3.0)
    return W.Workload(name="line4-x100-n240-latent-sd3-early", model=model,
                      sampler=W.PAPER1D_LATENT_SAMPLER, trace_dtype="f64", sweeps=8, seed=2)


def early_instance(w):
    m = O.make_model(**w.model.asdict())
    sp = O.make_sampler(**w.sampler.asdict())
    da = np.zeros((4, 8))
    da[0, :4] = [-9.0, 2.0, -3.0, 1.0]
    da[1, :4] = [4.0, -10.0, 0.5, -1.0]
    da[2, :4] = [-11.0, -6.0, 0.0, 3.0]
    truth = O.as_events([0.5, 34.0, 2.0, 70.0], [0.0] * 4, [0.3, 1.5, 4.0, 120.0],
                        [w.model.mmin] * 4, da=da)
    return m, sp, truth, O.simulate(m, truth, 1000 + w.seed)


def test_latent_refresh_with_arrivals_before_the_trace():
    from paper_1612_00595_amd import chromh
    w = early_world()
    m, sp, truth, s = early_instance(w)
    assert _early_arrivals(w.model, truth) >= 3
    say("latent refresh, arrivals before the trace")
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), chains=1, seed=3)
    gpu.write_events(0, truth)
    gpu.refresh(write_variance=True, loglik=False)
    E = gpu.read_variance(0)
    Er = O.event_variance(m, gpu.read_events(0))
    assert np.array_equal(E, Er)
    ll = gpu.refresh(write_variance=False, loglik=True)[0]
    assert ll == pytest.approx(O.loglik(m, s, truth), rel=1e-10)


@pytest.mark.parametrize("block", [64, 256])
def test_latent_replay_parity_arrivals_before_the_trace(block):
    """Footprints whose windows start before the first sample: the runs are
    cut at sample 0, exactly as the oracle's windows."""
    w = early_world()
    say("latent replay, arrivals before the trace, block", block)
    early = []
    inst = early_instance(w)
    gpu, ref, m, s, acc, types, status = _replay(w, 8, block=block, inst=inst, early=early,
                                                 start=inst[2])
    say("moves", acc.moves, "evaluated", acc.evaluated, "states with early arrivals",
        sum(1 for q in early if q), "of", len(early))
    assert acc.evaluated > 5000
    assert sum(1 for q in early if q) >= len(early) // 2
    _check_state(gpu, ref, m, s, w)


@pytest.mark.parametrize("tmpl,dtype,block", [(1, "f64", 256), (0, "f32", 256), (1, "f32", 64)])
def test_latent_replay_parity_template_and_f32(tmpl, dtype, block):
    w = W.PAPER1D_LATENT
    w = dataclasses.replace(w, name=w.name + f"-t{tmpl}-{dtype}", trace_dtype=dtype,
                            model=dataclasses.replace(w.model, tmpl=tmpl),
                            sampler=dataclasses.replace(w.sampler, dynamic=1))
    say("latent replay", w.name)
    gpu, ref, m, s, acc, types, status = _replay(w, 6, block=block)
    say("moves", acc.moves, "evaluated", acc.evaluated, "ties", acc.ties)
    assert acc.evaluated > 5000
    ev = ref.events()
    assert len(ev) > 0
    got = gpu.read_variance(0)
    Er = O.event_variance(m, ev)
    if tmpl:
        assert np.max(np.abs(got - (s.astype(np.float64) - Er))) <= 1e-10 * np.abs(s).max()
    else:
        assert np.all(np.abs(got - Er) <= 1e-9 * (w.model.sigma ** 2 + Er))
    ll = gpu.refresh(write_variance=False, loglik=True)[0]
    assert ll == pytest.approx(O.loglik(m, s, ev), rel=1e-10)


def test_latent_graph_replay_matches_eager():
    from paper_1612_00595_amd import chromh
    w = dataclasses.replace(W.PAPER1D_LATENT, sampler=dataclasses.replace(
        W.PAPER1D_LATENT.sampler, dynamic=1))
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    a = chromh.ChromaticSampler(w.model, w.sampler, trace, seed=4)
    b = chromh.ChromaticSampler(w.model, w.sampler, trace, seed=4)
    say("latent graph replay vs eager")
    a.run_sweeps(0, 2)
    torch.cuda.synchronize()
    a.run_sweeps(2, 3)
    for sw in range(5):
        for c in range(b.ncolors):
            b.sweep_color(sw, c)
    compare_events(a.read_events(0), b.read_events(0), "after 5 sweeps")
    assert np.array_equal(a.read_variance(0), b.read_variance(0))
    assert np.array_equal(a.read_stats(0), b.read_stats(0))
    assert a.read_stats(0)[6, 0] > 0 and a.read_stats(0)[5, 2] > 0
    a.close()
    b.close()


@pytest.mark.parametrize("block", [64, 256])
def test_latent_batch_matches_single_runs(block):
    from paper_1612_00595_amd import chromh
    spec = W.PAPER1D_LATENT_MODEL
    sampler = dataclasses.replace(W.PAPER1D_LATENT_SAMPLER, dynamic=1)
    n = 5
    traces, seeds = [], []
    for q in range(n):
        tr = W.truth_events(spec, 60 + q)
        truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"], da=tr["da"])
        traces.append(chromh.simulate(spec, truth, 600 + q, "f64", DEV))
        seeds.append(90 + q)
    say("latent batch of", n, "worlds")
    b = chromh.Batch([spec] * n, [sampler] * n, traces, seeds, block=block)
    b.run_sweeps(0, 5)
    torch.cuda.synchronize()
    for q in range(n):
        one = chromh.ChromaticSampler(spec, sampler, traces[q], chains=1, seed=seeds[q],
                                      block=256 if block == 64 else 64)
        one.run_sweeps(0, 5)
        ref = one.read_events(0)
        compare_events(b.read_events(q), ref, f"world {q}")
        assert np.array_equal(b.read_counters(q), one.read_counters(0))
        one.close()
    b.close()


def test_latent_prior_only_gpu_samples_the_prior():
    from paper_1612_00595_amd import chromh
    w = two_station()
    spec = dataclasses.replace(w.model, lam=12.0)
    sampler = dataclasses.replace(w.sampler, prior_only=1, dynamic=1, k=8, pb=0.2, pd=0.2,
                                  ploc=0.15, pt=0.15, pa=0.15, pj=0.15, sa=2.0)
    s = torch.zeros((spec.nsta, spec.N), dtype=torch.float64, device=DEV)
    chains = 8
    gpu = chromh.ChromaticSampler(spec, sampler, s, chains=chains, seed=21)
    say("latent prior-only: 8 chains x 6000 sweeps")
    gpu.run_sweeps(0, 100)
    counts, xs, ts, das = [[] for _ in range(chains)], [], [], []
    for blk in range(1, 120):
        gpu.run_sweeps(50 * blk + 50, 50)
        for c in range(chains):
            ev = gpu.read_events(c)
            counts[c].append(len(ev))
            xs.append(ev["x"]); ts.append(ev["t"]); das.append(ev["da"][:, :spec.nsx])
    cnt = np.array(counts, dtype=float)
    se = cnt.std() / np.sqrt(cnt.size)
    st = sum(gpu.read_stats(c) for c in range(chains))
    say("count mean", cnt.mean(), "se", se, "var", cnt.var(), "joint att/valid/acc", st[6])
    assert abs(cnt.mean() - spec.lam) < 4.5 * se
    assert 0.8 * spec.lam < cnt.var() < 1.25 * spec.lam
    x, t, da = np.concatenate(xs), np.concatenate(ts), np.concatenate(das)
    assert stats.kstest(x / spec.xmax, "uniform").pvalue > 1e-3
    assert stats.kstest(t / spec.N, "uniform").pvalue > 1e-3
    for j in range(spec.nsx):
        assert stats.kstest(da[:, j] / spec.arr_sd, stats.truncnorm(-4, 4).cdf).pvalue > 1e-3
    assert st[6, 2] > 0.02 * st[6, 0]


def test_latent_limits_are_checked():
    from paper_1612_00595_amd import chromh
    w = W.PAPER1D_LATENT
    s = torch.zeros((w.model.nsta, w.model.N), dtype=torch.float64, device=DEV)
    with pytest.raises(chromh.CmhError):  # only the wave and 256-thread latency forms
        chromh.ChromaticSampler(w.model, w.sampler, s, seed=1, block=128)
    with pytest.raises(chromh.CmhError):  # nor the naive schedule
        chromh.ChromaticSampler(w.model, dataclasses.replace(w.sampler, schedule=1), s, seed=1)
    g = dataclasses.replace(W.SMALL.model, arr_sd=1.0)
    with pytest.raises(chromh.CmhError):  # the grid model has no latent arrivals
        chromh.ChromaticSampler(g, W.SMALL.sampler,
                                torch.zeros((g.nsta, g.N), dtype=torch.float64, device=DEV))
    with pytest.raises(chromh.CmhError):  # the moves need latent arrivals
        chromh.ChromaticSampler(W.PAPER1D_MODEL, w.sampler, s, seed=1)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, s, seed=1)
    ev = chromh.as_events([50.0], [0.0], [100.0], [w.model.mmin], da=[[0, 0, 4.5, 0, 0, 0, 0, 0]])
    with pytest.raises(chromh.CmhError):  # an offset beyond 4 sd
        gpu.write_events(0, ev)
    ev["da"][0, 2] = 3.9
    gpu.write_events(0, ev)
    back = gpu.read_events(0)
    assert np.array_equal(back["da"], ev["da"])
    gpu.close()
