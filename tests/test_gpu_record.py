"""Device-side sample recording: the states written after each sweep inside
the replayed sweep graphs equal the event tables read back after that sweep
(dynamic partition, several chains), and truncation keeps the count."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1612_00595_amd import workloads as W

from gpu_cases import compare_events, dynamic_small, instance, say

pytestmark = pytest.mark.gpu


def _sorted(ev):
    return np.sort(np.stack([ev["x"], ev["y"], ev["t"], ev["m"]], 1), axis=0)


def test_recorded_states_match_read_back():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_00595_amd import chromh
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    chains = 3
    say("record", w.name, "chains", chains)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to("cuda"),
                                  chains=chains, seed=4)
    gpu.run_sweeps(0, 5)
    rec = gpu.set_record(5, 6, 400)
    small = None
    for sw in range(5, 11):
        gpu.run_sweeps(sw, 1)
        torch.cuda.synchronize()
        for c in range(chains):
            got = chromh.ChromaticSampler.recorded_states(rec[sw - 5:sw - 4], c)[0]
            ref = gpu.read_events(c)
            assert len(got) == len(ref) > 0
            # recorded in region order, id order within a region: same multiset
            assert np.array_equal(_sorted(got), _sorted(ref)), (sw, c)
    n_last = int(rec[-1, 0, 0])
    # truncation: the count stays, only max_events events are written
    gpu.set_record(11, 1, 3)
    small = gpu._rec
    gpu.run_sweeps(11, 1)
    torch.cuda.synchronize()
    assert int(small[0, 0, 0]) == len(gpu.read_events(0))
    assert len(chromh.ChromaticSampler.recorded_states(small, 0)[0]) == min(3, int(small[0, 0, 0]))
    gpu.set_record(0, 0, 0)
    gpu.run_sweeps(12, 2)
    torch.cuda.synchronize()
    assert n_last > 0


def test_kernel_stamps_from_graph_replays():
    """Stamps taken by the sweep kernels inside replayed graphs: one span per
    colour and stamped sweep, positive, together no longer than the sweeps'
    wall time, none outside the stamped range, and the chain itself is the
    unstamped one."""
    import time

    import numpy as np

    from paper_1612_00595_amd import chromh
    w = dynamic_small()
    m, sp, truth, s = instance(w)
    trace = torch.from_numpy(s).to("cuda:0")
    for block in (64, 256, chromh.SPEC4, chromh.PERSIST):
        say("stamps, form", block)
        a = chromh.ChromaticSampler(w.model, w.sampler, trace, seed=5, block=block)
        b = chromh.ChromaticSampler(w.model, w.sampler, trace, seed=5, block=block)
        st = a.set_stamps(3, 4)
        a.run_sweeps(0, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a.run_sweeps(3, 4)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        a.run_sweeps(7, 2)                 # past the range: no stamps
        spans = chromh.ChromaticSampler.stamp_seconds(st)
        assert spans.shape == (4, a.ncolors)
        if block == chromh.PERSIST:  # one launch per sweep, stamped as colour 0
            assert np.all(spans[:, 1:] < 0)
            spans = spans[:, :1]
        assert np.all(spans > 0) and np.all(spans < 0.1)
        assert spans.sum() <= el
        b.run_sweeps(0, 9)
        compare_events(a.read_events(0), b.read_events(0), f"form {block}")
        assert np.array_equal(a.read_variance(0), b.read_variance(0))
        a.close()
        b.close()
