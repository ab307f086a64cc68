"""Batches of uneven instances: every instance sampled inside a batch follows
exactly the chain it follows when sampled alone with the same seed (events
bit-identical), the batch's statistics are the instances' own, and mixing
instance sizes and colour counts works."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1612_00595_amd import workloads as W

from gpu_cases import compare_events, say

pytestmark = pytest.mark.gpu


def _instances():
    specs = [W.ModelSpec(nsx=6, nsy=6, N=2000, lam=60.0),
             W.ModelSpec(nsx=10, nsy=10, N=3000, lam=150.0),
             W.ModelSpec(nsx=8, nsy=12, N=1500, lam=120.0),
             W.ModelSpec(nsx=9, nsy=5, N=2500, lam=70.0)]
    samplers = [W.SamplerSpec(gx=m.nsx, gy=m.nsy, dynamic=1) for m in specs]
    return specs, samplers


@pytest.mark.parametrize("block", [64, 256, 1024 + 256, 2048 + 64])
def test_batch_instances_match_single_runs(block):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_00595_amd import chromh
    specs, samplers = _instances()
    seeds = [11, 12, 13, 14]
    traces = []
    for q, m in enumerate(specs):
        tr = W.truth_events(m, 40 + q)
        truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
        traces.append(chromh.simulate(m, truth, 500 + q, "f32", "cuda"))
    say("batch of", len(specs), "instances")
    b = chromh.Batch(specs, samplers, traces, seeds, block=block)
    b.run_sweeps(0, 6)
    torch.cuda.synchronize()
    for q, m in enumerate(specs):
        # the latency form alone: every batch form against it
        one = chromh.ChromaticSampler(m, samplers[q], traces[q], chains=1, seed=seeds[q],
                                      block=256)
        one.run_sweeps(0, 6)
        got, ref = b.read_events(q), one.read_events(0)
        say("instance", q, "events", len(ref))
        assert len(ref) > 0
        compare_events(got, ref, f"instance {q}")
        assert np.array_equal(b.read_counters(q), one.read_counters(0))
        one.close()
    # recording inside the batch graph
    rec = b.set_record(6, 2, 2048)
    b.run_sweeps(6, 2)
    torch.cuda.synchronize()
    for q in range(len(specs)):
        st = chromh.ChromaticSampler.recorded_states(rec[1:2], q)[0]
        assert len(st) == len(b.read_events(q))
    b.close()


def test_tuning_while_running_keeps_the_chain():
    """cmh_tune_running runs each kernel form on sweeps of the batch itself:
    the batch's instances end exactly where a batch run in one fixed form
    ends after the same sweeps, before and after two more sweeps in the
    chosen form."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_00595_amd import chromh
    specs, samplers = _instances()
    seeds = [21, 22, 23, 24]
    traces = []
    for q, m in enumerate(specs):
        tr = W.truth_events(m, 60 + q)
        truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
        traces.append(chromh.simulate(m, truth, 700 + q, "f32", "cuda"))
    say("tuning a batch of", len(specs), "instances while it runs")
    a = chromh.Batch(specs, samplers, traces, seeds)
    nxt = a.tune_running(0, 1)
    # seven forms and the persistent one (dynamic partitions), 1 + 1 sweeps each
    assert nxt == 16
    assert a.block in (64, 128, 256, 512, 1024 + 128, 1024 + 256, 1024 + 512, 2048 + 64)
    ref = chromh.Batch(specs, samplers, traces, seeds, block=256)
    ref.run_sweeps(0, nxt)
    torch.cuda.synchronize()
    for q in range(len(specs)):
        compare_events(a.read_events(q), ref.read_events(q), f"instance {q} after tuning")
        assert np.array_equal(a.read_counters(q), ref.read_counters(q))
    a.run_sweeps(nxt, 2)
    ref.run_sweeps(nxt, 2)
    torch.cuda.synchronize()
    for q in range(len(specs)):
        compare_events(a.read_events(q), ref.read_events(q), f"instance {q} after two more")
    a.close()
    ref.close()
    # latent arrivals on dynamic partitions: the wave and 256-thread forms
    # only (the persistent kernel has no arrival moves)
    import dataclasses
    m = W.PAPER1D_LATENT_MODEL
    sp = dataclasses.replace(W.PAPER1D_LATENT_SAMPLER, dynamic=1)
    tr = W.truth_events(m, 5)
    trace = chromh.simulate(m, chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"], da=tr["da"]),
                            75, "f64", "cuda")
    say("tuning a latent-arrival chain while it runs")
    one = chromh.ChromaticSampler(m, sp, trace, chains=2, seed=9)
    nxt = one.tune_running(0, 1)
    assert nxt == 4 and one.block in (64, 256)
    ref = chromh.ChromaticSampler(m, sp, trace, chains=2, seed=9, block=256)
    ref.run_sweeps(0, nxt)
    torch.cuda.synchronize()
    for c in range(2):
        compare_events(one.read_events(c), ref.read_events(c), f"latent chain {c}")
    one.close()
    ref.close()


def test_batch_rejects_mixed_settings():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_00595_amd import chromh
    specs, samplers = _instances()
    samplers[1] = W.SamplerSpec(gx=10, gy=10, dynamic=0)
    traces = [torch.zeros((m.nsta, m.N), dtype=torch.float32, device="cuda") for m in specs]
    with pytest.raises(chromh.CmhError):
        chromh.Batch(specs, samplers, traces, [1, 2, 3, 4])


def test_persistent_wait_timeout_is_reported():
    """The persistent form's colour-counter wait is bounded: with the limit
    forced to zero (debug bit 2) an item whose slot has not finished its
    lower colours gives up at once, every wave still exits, and the run
    ends in CMH_ESTATE with the state poisoned."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import dataclasses

    from paper_1612_00595_amd import chromh
    specs, samplers = _instances()
    samplers = [dataclasses.replace(sp, debug=4) for sp in samplers]
    traces = [0.1 * torch.ones((m.nsta, m.N), dtype=torch.float32, device="cuda") for m in specs]
    b = chromh.Batch(specs, samplers, traces, [1, 2, 3, 4], block=chromh.PERSIST)
    b.run_sweeps(0, 3)
    with pytest.raises(chromh.CmhError) as e:
        b.read_events(0)
    assert e.value.code == -6
    b.close()
