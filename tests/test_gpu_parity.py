"""GPU parity tests: the HIP path against the FP64 oracle, through the C-ABI.

Bars (from the method's contract): region binning, colouring and event
bookkeeping bit-exact; in replay mode (the same draws fed to both sides)
log-likelihood changes within 1e-4 relative (floor 1 nat) and decisions
identical wherever |log u - log alpha| > 1e-6; event variance within 1e-9
relative to the model variance sigma^2 + E.
"""
import numpy as np
import pytest

from gpu_cases import LogCheck, compare_events, compare_logs, dynamic_small, instance, say

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_1612_00595_amd import chromh, workloads as W  # noqa: E402

DEV = "cuda:0"


def _variance_close(Eg, Er, sigma2=0.01, rel=1e-9):
    return np.all(np.abs(Eg - Er) <= rel * (sigma2 + Er))


# ---------------------------------------------------------------- draws

def test_move_draws_match_oracle():
    for seed, chain, sweep, region in [(0, 0, 0, 0), (7, 3, 11, 4224), (2**31, 31, 499, 17)]:
        say("draws", seed, chain, sweep, region)
        g = chromh.move_draws(seed, chain, sweep, region, 0, 300)
        r = np.array([O.move_draws(seed, chain, sweep, region, j) for j in range(300)])
        assert np.array_equal(g[:, :4], r[:, :4])     # integer-derived uniforms: exact
        assert np.allclose(g[:, 4:], r[:, 4:], rtol=1e-14, atol=1e-15)


# ------------------------------------------------------------ simulator

def test_simulator_matches_oracle_small():
    w = W.SMALL
    m = O.make_model(**w.model.asdict())
    tr = W.truth_events(w.model, 3)
    truth = O.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    ref = O.simulate(m, truth, 55)
    say("simulate small f64/f32")
    g64 = chromh.simulate(w.model, truth, 55, "f64", DEV).cpu().numpy()
    assert np.allclose(g64, ref, rtol=1e-12, atol=1e-15)
    g32 = chromh.simulate(w.model, truth, 55, "f32", DEV).cpu().numpy()
    r32 = ref.astype(np.float32)
    ulp = np.spacing(np.abs(r32))
    assert np.all(np.abs(g32 - r32) <= ulp)


def test_simulator_matches_oracle_full_size_sampled():
    w = W.LARGE
    m = O.make_model(**w.model.asdict())
    tr = W.truth_events(w.model, w.seed)
    truth = O.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
    say("simulate", w.name, "events", len(truth))
    g = chromh.simulate(w.model, truth, 123, "f32", DEV)
    rows = np.random.default_rng(0).choice(w.model.nsta, 24, replace=False)
    for j in rows:
        ref = O.simulate_rows(m, truth, 123, int(j), 1)[0].astype(np.float32)
        got = g[int(j)].cpu().numpy()
        assert np.all(np.abs(got - ref) <= np.spacing(np.abs(ref))), j
    assert torch.isfinite(g).all()
    del g


# ------------------------------------------------------------- replay

def _replay(w, nsw, block, feed_seed=77, compare_each_phase=True):
    m, sp, truth, s = instance(w)
    feed = W.feed_draws(w.sampler, nsw, seed=feed_seed)
    R, k = w.sampler.nreg, w.sampler.k
    trace = torch.from_numpy(s).to(DEV)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=1, seed=3, block=block)
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
    gpu.set_log(glog, 0)
    ref = O.Chain(m, sp, s, seed=3)
    rlog = np.full((nsw, R, k, 4), -1.0)
    acc = LogCheck()
    for sw in range(nsw):
        assert ref.begin_sweep(sw) == 0
        lay = ref.layout()
        assert lay["ncolors"] == gpu.ncolors
        for c in range(gpu.ncolors):
            assert ref.phase(sw, c, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
            if block == chromh.PERSIST:  # one launch runs the whole sweep
                continue
            gpu.sweep_color(sw, c)
            if compare_each_phase:
                compare_events(gpu.read_events(0), ref.events(), f"sweep {sw} colour {c}")
        if block == chromh.PERSIST:
            gpu.run_sweeps(sw, 1)
            compare_events(gpu.read_events(0), ref.events(), f"sweep {sw}")
        if not compare_logs(glog[sw].cpu().numpy(), rlog[sw], feed[sw], acc, f"sweep {sw}"):
            say("decision tie at sweep", sw, "- stopping the bit-exact comparison")
            return gpu, ref, m, s, acc
    compare_events(gpu.read_events(0), ref.events(), "final")
    return gpu, ref, m, s, acc


@pytest.mark.parametrize("block", [64, 128, 256, 512, chromh.SPEC2, chromh.SPEC4, chromh.SPEC8])
def test_replay_parity_small_static(block):
    say("replay", W.SMALL.name, "block", block)
    gpu, ref, m, s, acc = _replay(W.SMALL, 12, block)
    assert acc.evaluated > 1000
    ev = ref.events()
    assert _variance_close(gpu.read_variance(0), O.event_variance(m, ev))
    ll = gpu.refresh(write_variance=False, loglik=True)[0]
    assert ll == pytest.approx(O.loglik(m, s, ev), rel=1e-10)
    say("moves", acc.moves, "evaluated", acc.evaluated, "ties", acc.ties, "max rel", acc.max_rel)


@pytest.mark.parametrize("block", [64, 256, chromh.SPEC4, chromh.SPEC8, chromh.PERSIST])
def test_replay_parity_dynamic(block):
    w = dynamic_small()
    say("replay", w.name, "block", block)
    gpu, ref, m, s, acc = _replay(w, 8, block)
    assert acc.evaluated > 5000
    assert _variance_close(gpu.read_variance(0), O.event_variance(m, ref.events()))


def test_replay_parity_full_size_large():
    """The 64x64-station, 144000-sample workload at full size: two sweeps (nine
    colour phases each) from the empty world, every workgroup size the sweep
    may be launched with, against the oracle on the same fp32 trace."""
    w = W.LARGE
    nsw = 2
    say("instance", w.name)
    m, sp, truth, s = instance(w)
    feed = W.feed_draws(w.sampler, nsw, seed=99)
    R, k = w.sampler.nreg, w.sampler.k
    ref = O.Chain(m, sp, s, seed=3)
    rlog = np.full((nsw, R, k, 4), -1.0)
    say("oracle sweeps")
    for sw in range(nsw):
        assert ref.sweep(sw, feed=np.ascontiguousarray(feed[sw]), log=rlog[sw]) == 0
    rev = ref.events()
    say("oracle events", len(rev))
    trace = torch.from_numpy(s).to(DEV)
    fd = torch.from_numpy(feed).to(DEV)
    rows = np.random.default_rng(1).choice(w.model.nsta, 48, replace=False)
    Er = {int(j): O.event_variance_rows(m, rev, int(j), 1)[0] for j in rows}
    for block in (64, 128, 256, 512, chromh.SPEC4, chromh.SPEC8, chromh.PERSIST):
        say("gpu sweep block", block)
        gpu = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=1, seed=3, block=block)
        gpu.set_feed(fd, 0)
        glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
        gpu.set_log(glog, 0)
        gpu.run_sweeps(0, nsw)
        compare_events(gpu.read_events(0), rev, f"block {block}")
        acc = LogCheck()
        for sw in range(nsw):
            assert compare_logs(glog[sw].cpu().numpy(), rlog[sw], feed[sw], acc,
                                f"block {block} sweep {sw}")
        assert acc.evaluated > 20000
        for j in rows:
            assert _variance_close(gpu.read_variance(0, int(j), 1)[0], Er[int(j)]), j
        gpu.close()
        del gpu, glog
        torch.cuda.empty_cache()


def test_replay_parity_full_size_at_steady_state():
    """The 64x64-station workload at the posterior's event count: a state
    from 300 Philox sweeps is written into fresh samplers of every form and
    into the oracle, then both replay two fed sweeps.  Most accepted moves
    there are location, onset and magnitude changes of distinct events, so
    the speculative forms commit several moves per round; every form must
    still give the oracle's chain."""
    w = W.LARGE
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    first, nsw = 300, 2
    say("burn-in to sweep", first)
    base = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=1, seed=3,
                                   block=chromh.SPEC4)
    base.run_sweeps(0, first)
    ev = base.read_events(0)
    base.close()
    say("state events", len(ev))
    assert len(ev) > 15000
    feed = W.feed_draws(w.sampler, nsw, seed=41)
    R, k = w.sampler.nreg, w.sampler.k
    ref = O.Chain(m, sp, s, seed=3)
    assert ref.set_events(O.as_events(ev["x"], ev["y"], ev["t"], ev["m"], ev["id"])) == 0
    rlog = np.full((nsw, R, k, 4), -1.0)
    for q in range(nsw):
        assert ref.sweep(first + q, feed=np.ascontiguousarray(feed[q]), log=rlog[q]) == 0
    rev = ref.events()
    fd = torch.from_numpy(feed).to(DEV)
    for block in (64, 256, chromh.SPEC2, chromh.SPEC4, chromh.SPEC8):
        say("gpu form", block)
        gpu = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=1, seed=3, block=block)
        gpu.write_events(0, ev)
        gpu.set_feed(fd, first)
        glog = torch.full((nsw, R, k, 4), -1.0, dtype=torch.float64, device=DEV)
        gpu.set_log(glog, first)
        gpu.run_sweeps(first, nsw)
        acc = LogCheck()
        exact = True
        for q in range(nsw):
            if not compare_logs(glog[q].cpu().numpy(), rlog[q], feed[q], acc,
                                f"form {block} sweep {first + q}"):
                exact = False  # a decision inside the tie band: the chains may part here
                say("decision tie in sweep", first + q)
                break
        if exact:
            compare_events(gpu.read_events(0), rev, f"form {block}")
        assert acc.evaluated > 30000
        say("evaluated", acc.evaluated, "ties", acc.ties, "max rel", acc.max_rel)
        gpu.close()
        del gpu, glog
        torch.cuda.empty_cache()


# ------------------------------------------------------ state and replays

def test_refresh_matches_oracle():
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    st = W.random_state(w.model, 5, 300)
    ev = O.as_events(st["x"], st["y"], st["t"], st["m"], st["id"])
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=1)
    gpu.write_events(0, ev)
    assert _variance_close(gpu.read_variance(0), O.event_variance(m, ev), rel=1e-12)
    ll = gpu.refresh(write_variance=False, loglik=True)[0]
    assert ll == pytest.approx(O.loglik(m, s, ev), rel=1e-12)
    back = gpu.read_events(0)
    order = np.argsort(back["id"])
    for f in ("x", "y", "t", "m", "id"):
        assert np.array_equal(back[f][order], ev[f])


def test_incremental_variance_matches_exact_refresh():
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=2)
    gpu.run_sweeps(0, 20)
    E_inc = gpu.read_variance(0)
    gpu.refresh(write_variance=True, loglik=False)
    E_ref = gpu.read_variance(0)
    assert len(gpu.read_events(0)) > 50
    assert _variance_close(E_inc, E_ref)


def test_graph_replay_matches_eager():
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    a = chromh.ChromaticSampler(w.model, w.sampler, trace, seed=4, block=128)
    b = chromh.ChromaticSampler(w.model, w.sampler, trace, seed=4, block=128)
    a.run_sweeps(0, 2)
    torch.cuda.synchronize()
    a.run_sweeps(2, 2)
    mid = a.read_events(0)
    a.run_sweeps(4, 3)
    for sw in range(7):
        for c in range(b.ncolors):
            b.sweep_color(sw, c)
        if sw == 3:
            compare_events(b.read_events(0), mid, "after 4 sweeps")
    compare_events(a.read_events(0), b.read_events(0), "after 7 sweeps")
    assert np.array_equal(a.read_variance(0), b.read_variance(0))
    assert np.array_equal(a.read_stats(0), b.read_stats(0))


def test_chain_zero_of_a_batch_equals_a_single_chain():
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    many = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=4, seed=9)
    one = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=1, seed=9)
    many.run_sweeps(0, 5)
    one.run_sweeps(0, 5)
    compare_events(many.read_events(0), one.read_events(0), "chain 0")
    assert np.array_equal(many.read_variance(0), one.read_variance(0))
    assert not np.array_equal(many.read_events(1)["x"][:5], many.read_events(0)["x"][:5])


def test_philox_mode_tracks_the_oracle():
    """Without a feed both sides draw from their own Philox4x32-10; the
    transcendental conversions may differ in the last bit, so event values are
    compared to 1e-12 and ids, regions and counts exactly."""
    w = W.SMALL
    m, sp, truth, s = instance(w)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=21)
    ref = O.Chain(m, sp, s, seed=21)
    for sw in range(6):
        ref.sweep(sw)
        gpu.run_sweeps(sw, 1)
        a, b = gpu.read_events(0), ref.events()
        assert np.array_equal(a["id"], b["id"]) and np.array_equal(a["region"], b["region"])
        for f in ("x", "y", "t", "m"):
            assert np.allclose(a[f], b[f], rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------- statistics

@pytest.mark.parametrize("block", [256, chromh.SPEC4])
def test_prior_only_gpu_chain_samples_the_prior(block):
    from scipy import stats
    w = W.SMALL
    spec = W.SamplerSpec(**dict(w.sampler.asdict(), prior_only=1, k=8))
    trace = torch.zeros((w.model.nsta, w.model.N), dtype=torch.float64, device=DEV)
    gpu = chromh.ChromaticSampler(w.model, spec, trace, seed=2, block=block)
    gpu.run_sweeps(0, 100)
    counts, xs, ms = [], [], []
    for q in range(600):
        gpu.run_sweeps(100 + 5 * q, 5)
        ev = gpu.read_events(0)
        counts.append(len(ev))
        if q % 5 == 0:
            xs.append(ev["x"]); ms.append(ev["m"])
    counts = np.array(counts)
    lam = w.model.lam
    assert abs(counts.mean() - lam) < 1.0
    assert 0.75 * lam < counts.var() < 1.3 * lam
    assert stats.kstest(np.concatenate(xs) / w.model.Lx, "uniform").pvalue > 1e-3
    assert stats.kstest(np.concatenate(ms) - 2.0, "expon").pvalue > 1e-3
    st = gpu.read_stats(0)
    assert st[:, 0].sum() == (100 + 600 * 5) * 16 * spec.k


# ------------------------------------------------------------ error paths

@pytest.mark.parametrize("block", [256, chromh.SPEC4])
def test_capacity_overflow_is_reported(block):
    w = W.SMALL
    spec = W.SamplerSpec(**dict(w.sampler.asdict(), cap=2))
    m, sp, truth, s = instance(w)
    feed = W.feed_draws(spec, 1, seed=1)
    feed[..., 0] = 0.01      # every move a birth
    feed[..., 7] = -1e300    # every birth accepted
    gpu = chromh.ChromaticSampler(w.model, spec, torch.from_numpy(s).to(DEV), seed=1, block=block)
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 0)
    gpu.run_sweeps(0, 1)
    with pytest.raises(chromh.CmhError) as e:
        gpu.read_events(0)
    assert e.value.code == -3
    with pytest.raises(chromh.CmhError) as e:
        gpu.run_sweeps(1, 1)
    assert e.value.code == -6


def test_nan_trace_is_reported():
    w = W.SMALL
    trace = torch.full((w.model.nsta, w.model.N), float("nan"), dtype=torch.float64, device=DEV)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, trace, seed=1)
    gpu.run_sweeps(0, 1)
    with pytest.raises(chromh.CmhError) as e:
        gpu.read_events(0)
    assert e.value.code == -5


def test_feed_range_is_checked():
    w = W.SMALL
    m, sp, truth, s = instance(w)
    feed = W.feed_draws(w.sampler, 2, seed=1)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV), seed=1)
    gpu.set_feed(torch.from_numpy(feed).to(DEV), 5)
    with pytest.raises(chromh.CmhError) as e:
        gpu.sweep_color(4, 0)
    assert e.value.code == -1
    gpu.sweep_color(5, 0)
