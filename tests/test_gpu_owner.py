"""The debug owner check through the C-ABI (sampler.debug bit 0): every
sample a move reads or writes is tagged with its (sweep, colour, region), and
a tag of another region of the same colour phase latches CMH_ERACE.  With the
colouring of Section 4.1 the check stays silent and changes nothing (events
and counters bit-identical to a run without it) on grids, the line, latent
arrivals, templates and a batch, in every kernel form; with a period forced
past the independence check (bit 1), one the oracle counts violations for,
it reports the breach."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1612_00595_amd import workloads as W  # noqa: E402

from gpu_cases import compare_events, dynamic_small, instance, say  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ERACE = -7


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _with(w, **kw):
    return dataclasses.replace(w, sampler=dataclasses.replace(w.sampler, **kw))


def _cases():
    small_t = dataclasses.replace(W.SMALL, model=dataclasses.replace(W.SMALL.model, tmpl=1))
    return [
        ("grid-dynamic", dynamic_small(), 64, 2),
        ("grid-dynamic", dynamic_small(), 256, 2),
        ("grid-dynamic", dynamic_small(), 1024 + 256, 2),
        ("grid-dynamic", dynamic_small(), 2048 + 64, 3),
        ("grid-static", W.SMALL, 128, 1),
        ("grid-template", small_t, 256, 1),
        ("grid-template", small_t, 1024 + 512, 1),
        ("line-static", W.PAPER1D, 64, 1),
        ("line-dynamic", _with(W.PAPER1D, dynamic=1), 256, 1),
        ("line-dynamic", _with(W.PAPER1D, dynamic=1), 1024 + 256, 1),
        ("latent-dynamic", _with(W.PAPER1D_LATENT, dynamic=1, k=200), 64, 1),
        ("latent-static", _with(W.PAPER1D_LATENT, k=200), 256, 1),
    ]


@pytest.mark.parametrize("name,w,block,chains", _cases(),
                         ids=[f"{c[0]}-{c[2]}" for c in _cases()])
def test_owner_check_is_silent_and_changes_nothing(name, w, block, chains):
    from paper_1612_00595_amd import chromh
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to(DEV)
    say("owner check", name, "block", block, "chains", chains)
    runs = []
    for debug in (0, 1):
        g = chromh.ChromaticSampler(w.model, _with(w, debug=debug).sampler, trace, chains=chains,
                                    seed=4, block=block)
        g.run_sweeps(0, 6)
        runs.append(g)
    plain, checked = runs
    for c in range(chains):
        a, b = plain.read_events(c), checked.read_events(c)
        assert len(a) > 0
        compare_events(b, a, f"chain {c}")
        assert np.array_equal(plain.read_counters(c), checked.read_counters(c))


def test_owner_check_batch_of_uneven_worlds():
    from paper_1612_00595_amd import chromh
    specs = [W.ModelSpec(nsx=6, nsy=6, N=2000, lam=60.0), W.ModelSpec(nsx=9, nsy=5, N=2500, lam=70.0),
             W.PAPER1D.model]
    samplers = [W.SamplerSpec(gx=m.nsx, gy=m.nsy, dynamic=1) for m in specs[:2]]
    samplers.append(dataclasses.replace(W.PAPER1D.sampler, dynamic=1, k=samplers[0].k))
    traces = []
    for q, m in enumerate(specs):
        tr = W.truth_events(m, 40 + q)
        traces.append(chromh.simulate(m, chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"]),
                                      500 + q, "f32", DEV))
    say("owner check: batch of three uneven worlds")
    runs = []
    for debug in (0, 1):
        b = chromh.Batch(specs, [dataclasses.replace(x, debug=debug) for x in samplers], traces,
                         [1, 2, 3], block=64)
        b.run_sweeps(0, 5)
        runs.append(b)
    for q in range(3):
        compare_events(runs[1].read_events(q), runs[0].read_events(q), f"instance {q}")
        assert np.array_equal(runs[1].read_counters(q), runs[0].read_counters(q))


@pytest.mark.parametrize("world,block", [
    ("grid", 64), ("grid", 256), ("grid", 1024 + 256),
    pytest.param("grid", 2048 + 64, marks=pytest.mark.skip(
        reason="the persistent form on this static partition did not finish on the device "
               "once, cause not found; the library now refuses static partitions for it")),
    ("line", 64), ("line", 256)])
def test_owner_check_reports_a_forced_breach(world, block):
    """Period 1 puts neighbouring regions in one colour (the oracle counts
    the dependent pairs); forced past the check, the run must end in
    CMH_ERACE at the next synchronising call."""
    from paper_1612_00595_amd import chromh
    w = W.SMALL if world == "grid" else W.PAPER1D
    m, sp, truth, s = instance(w)
    gy = 0 if w.model.line else w.sampler.gy
    assert O.coloring_violations(m, w.sampler.gx, gy, 0.0, 0.0, 1) > 0
    say("owner check: forced period 1 on", w.name, "block", block)
    g = chromh.ChromaticSampler(w.model, _with(w, period=1, debug=3).sampler,
                                torch.from_numpy(s).to(DEV), chains=1, seed=4, block=block)
    assert g.ncolors == 1
    g.run_sweeps(0, 4)
    with pytest.raises(chromh.CmhError) as err:
        g.read_events(0)
    assert err.value.code == ERACE
    with pytest.raises(chromh.CmhError):  # poisoned from then on
        g.read_events(0)
