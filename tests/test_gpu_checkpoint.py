"""Checkpoint and resume through the C-ABI: N sweeps, save, N more sweeps
must equal loading the checkpoint into a fresh state and running the same N
sweeps, bit for bit (events, arrival offsets, event variance, counters), for
several chains of a dynamic grid, the line model with latent arrivals, and a
batch of uneven instances; a checkpoint of another shape is refused."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1612_00595_amd import workloads as W  # noqa: E402

from gpu_cases import compare_events, dynamic_small, instance, say  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check_resume(make, chains, n1, n2):
    a = make()
    a.run_sweeps(0, n1)
    ck = a.save()
    a.run_sweeps(n1, n2)
    b = make()
    b.load(ck)
    b.run_sweeps(n1, n2)
    torch.cuda.synchronize()
    for c in range(chains):
        compare_events(b.read_events(c), a.read_events(c), f"chain {c}")
        assert np.array_equal(b.read_counters(c), a.read_counters(c))
    fresh = make()  # without the checkpoint the same sweeps give another state
    fresh.run_sweeps(n1, n2)
    assert any(len(fresh.read_events(c)) != len(a.read_events(c)) or
               not np.array_equal(fresh.read_events(c)["x"], a.read_events(c)["x"])
               for c in range(chains))
    return a, b


def test_resume_dynamic_grid_chains():
    from paper_1612_00595_amd import chromh
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    say("checkpoint: 3 chains of", w.name)
    a, b = _check_resume(lambda: chromh.ChromaticSampler(w.model, w.sampler, trace, chains=3,
                                                         seed=8, block=1024 + 256), 3, 5, 4)
    for c in range(3):
        assert np.array_equal(a.read_variance(c), b.read_variance(c))


def test_resume_persistent_form():
    from paper_1612_00595_amd import chromh
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    say("checkpoint: persistent form, 3 chains of", w.name)
    a, b = _check_resume(lambda: chromh.ChromaticSampler(w.model, w.sampler, trace, chains=3,
                                                         seed=8, block=chromh.PERSIST), 3, 5, 4)
    for c in range(3):
        assert np.array_equal(a.read_variance(c), b.read_variance(c))


@pytest.mark.parametrize("dynamic", [0, 1])
def test_resume_latent_line_world(dynamic):
    from paper_1612_00595_amd import chromh
    w = dataclasses.replace(W.PAPER1D_LATENT, sampler=dataclasses.replace(
        W.PAPER1D_LATENT.sampler, dynamic=dynamic, k=100))
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    say("checkpoint: latent line world, dynamic", dynamic)
    a, b = _check_resume(lambda: chromh.ChromaticSampler(w.model, w.sampler, trace, chains=2,
                                                         seed=5), 2, 7, 6)
    assert np.any(a.read_events(0)["da"] != 0.0)


def test_resume_uneven_batch():
    from paper_1612_00595_amd import chromh
    specs = [W.ModelSpec(nsx=6, nsy=6, N=2000, lam=60.0), W.ModelSpec(nsx=9, nsy=5, N=2500, lam=70.0),
             W.ModelSpec(nsx=5, nsy=5, N=1500, lam=30.0)]
    samplers = [W.SamplerSpec(gx=m.nsx, gy=m.nsy, dynamic=1) for m in specs]
    traces = []
    for q, m in enumerate(specs):
        tr = W.truth_events(m, 40 + q)
        traces.append(chromh.simulate(m, chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"]),
                                      500 + q, "f32", DEV))
    say("checkpoint: uneven batch of 3")
    _check_resume(lambda: chromh.Batch(specs, samplers, traces, [1, 2, 3], block=64), 3, 5, 5)


def test_checkpoint_of_another_shape_is_refused():
    from paper_1612_00595_amd import chromh
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    a = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=2, seed=8)
    ck = a.save()
    b = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=3, seed=8)
    with pytest.raises(chromh.CmhError):
        b.load(ck)
    w2 = W.SMALL
    m2, sp2, truth2, s2 = instance(w2)
    c = chromh.ChromaticSampler(w2.model, w2.sampler, torch.from_numpy(s2).to(DEV), chains=2,
                                seed=8)
    with pytest.raises(chromh.CmhError):
        c.load(ck)
    bad = ck.copy()
    bad[0] ^= 0xFF
    with pytest.raises(chromh.CmhError):
        a.load(bad)
    with pytest.raises(chromh.CmhError):
        a.load(ck[:100])


def _slot_fields(w, latent=False):
    """Byte offsets of one slot's fields inside a checkpoint of a
    single-instance state (header of 24 bytes, then per slot a 24-byte shape
    record, x, y, t, m, id, counts, offsets, [arrival offsets], variance,
    counters)."""
    R, cap = w.sampler.nreg, w.sampler.cap
    n = R * cap
    o = {"x": 24, "y": 24 + 8 * n, "t": 24 + 16 * n, "m": 24 + 24 * n, "id": 24 + 32 * n,
         "cnt": 24 + 40 * n}
    o["off"] = o["cnt"] + 4 * R
    o["E"] = o["off"] + 16 + (64 * n if latent else 0)
    o["stats"] = o["E"] + 8 * w.model.nsta * w.model.N
    o["end"] = o["stats"] + 8 * 23
    return o, R, cap


def test_corrupt_checkpoint_is_refused_before_any_write():
    """A record whose counts, events, offsets or variance no state of this
    shape can hold is refused on the host (CMH_EINVAL) and the state keeps
    what it had; nothing corrupt ever reaches a sweep."""
    from paper_1612_00595_amd import chromh
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    a = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=1, seed=8)
    a.run_sweeps(0, 4)
    ck = a.save()
    before = a.read_events(0)
    stats_before = a.read_counters(0)
    o, R, cap = _slot_fields(w)
    base = 24                                     # the state header
    assert ck.nbytes == base + o["end"]
    f = lambda name: base + o[name]               # noqa: E731
    cnt = ck[f("cnt"):f("cnt") + 4 * R].view(np.int32)
    r_full = int(np.argmax(cnt))
    assert cnt[r_full] > 0
    say("corrupt checkpoints: region", r_full, "holds", int(cnt[r_full]))

    def refused(mutate, why):
        bad = ck.copy()
        mutate(bad)
        with pytest.raises(chromh.CmhError) as e:
            a.load(bad)
        assert why in str(e.value), str(e.value)

    def set_i32(buf, off, v):
        buf[off:off + 4] = np.frombuffer(np.int32(v).tobytes(), np.uint8)

    def set_f64(buf, off, v):
        buf[off:off + 8] = np.frombuffer(np.float64(v).tobytes(), np.uint8)

    refused(lambda b: set_i32(b, f("cnt") + 4 * r_full, cap + 1), "count")
    refused(lambda b: set_i32(b, f("cnt") + 4 * r_full, -1), "count")
    slot0 = r_full * cap
    refused(lambda b: set_f64(b, f("x") + 8 * slot0, -0.5), "support")
    refused(lambda b: set_f64(b, f("t") + 8 * slot0, float(w.model.N)), "support")
    refused(lambda b: set_f64(b, f("m") + 8 * slot0, np.nan), "support")
    # an event moved to the far corner stays in the domain but not in its region
    x0 = float(ck[f("x") + 8 * slot0:f("x") + 8 * slot0 + 8].view(np.float64)[0])
    far = w.model.Lx - 1e-9 if x0 < w.model.Lx / 2 else 1e-9
    refused(lambda b: set_f64(b, f("x") + 8 * slot0, far), "region")
    refused(lambda b: set_f64(b, f("off"), 0.25), "offset")
    refused(lambda b: set_f64(b, f("off") + 8, -0.01), "offset")
    refused(lambda b: set_f64(b, f("E") + 8 * 17, np.inf), "variance")
    refused(lambda b: set_f64(b, f("E") + 8 * 17, -1.0), "variance")
    if cnt[r_full] > 1:
        def dup_id(b):
            b[f("id") + 8 * (slot0 + 1):f("id") + 8 * (slot0 + 2)] = \
                b[f("id") + 8 * slot0:f("id") + 8 * (slot0 + 1)]
        refused(dup_id, "ids")
    compare_events(a.read_events(0), before, "after refused loads")
    assert np.array_equal(a.read_counters(0), stats_before)
    a.load(ck)                                    # the intact record still loads
    a.run_sweeps(4, 2)
    torch.cuda.synchronize()
