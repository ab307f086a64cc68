"""Chains inside the full-size batched states against the oracle: chains 0
and 31 of the 32-chain, 32x32-station, 36000-sample state, and the smallest
and largest instances of the 256-instance uneven batch, each followed for two
sweeps by an oracle chain of the same key on the same trace.

Both sides draw from their own Philox4x32-10 streams (key (seed, chain)); the
integer-derived draws are identical, the transcendental conversions may
differ in the last bit, so event values are compared to 1e-12 relative and
ids, regions and counts exactly, as in the single-chain Philox test.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_1612_00595_amd import workloads as W

from gpu_cases import instance, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SWEEPS = 2


def _compare(a, b, where):
    assert len(a) == len(b), f"{where}: {len(a)} events on the GPU, {len(b)} in the oracle"
    assert np.array_equal(a["id"], b["id"]) and np.array_equal(a["region"], b["region"]), where
    for f in ("x", "y", "t", "m"):
        assert np.allclose(a[f], b[f], rtol=1e-12, atol=1e-12), (where, f)


def _oracle_chain(w, m, sp, s, seed, chain):
    ref = O.Chain(m, sp, s, seed=seed, chain=chain)
    for sw in range(SWEEPS):
        assert ref.sweep(sw) == 0
    return ref.events()


@pytest.mark.parametrize("block", [64, 1024 + 256, 2048 + 64])
def test_chains_of_the_32_chain_state_follow_the_oracle(block):
    from paper_1612_00595_amd import chromh
    w = W.CHAINS32
    m, sp, truth, s = instance(w)
    say("32 chains of", w.name, "form", block)
    gpu = chromh.ChromaticSampler(w.model, w.sampler, torch.from_numpy(s).to(DEV),
                                  chains=w.chains, seed=w.seed, block=block)
    gpu.run_sweeps(0, SWEEPS)
    for c in (0, w.chains - 1):
        ref = _oracle_chain(w, m, sp, s, w.seed, c)
        say("chain", c, "events", len(ref))
        assert len(ref) > 100
        _compare(gpu.read_events(c), ref, f"chain {c}")
    gpu.close()


@pytest.mark.parametrize("block", [64, 2048 + 64])
def test_instances_of_the_uneven_batch_follow_the_oracle(block):
    """The whole 256-instance batch runs; the smallest and the largest
    instance get traces from the oracle's side (seeded normals through the
    model variance), the others seeded normals of the noise level, which do
    not reach the compared instances (instances are independent)."""
    from paper_1612_00595_amd import chromh
    ws = W.uneven_batch(256)
    size = [w.model.nsta * w.model.N for w in ws]
    pick = (int(np.argmin(size)), int(np.argmax(size)))
    gen = torch.Generator(device=DEV)
    gen.manual_seed(77)
    traces, host = [], {}
    for q, w in enumerate(ws):
        if q in pick:
            m, sp, truth, s = instance(w)
            host[q] = (m, sp, s)
            traces.append(torch.from_numpy(s).to(DEV))
        else:
            traces.append(0.1 * torch.randn((w.model.nsta, w.model.N), generator=gen,
                                            dtype=torch.float32, device=DEV))
    say("uneven batch of", len(ws), "instances; compared:", [ws[q].name for q in pick])
    b = chromh.Batch([w.model for w in ws], [w.sampler for w in ws], traces,
                     [w.seed for w in ws], block=block)
    b.run_sweeps(0, SWEEPS)
    for q in pick:
        m, sp, s = host[q]
        ref = _oracle_chain(ws[q], m, sp, s, ws[q].seed, 0)
        say("instance", q, ws[q].name, "events", len(ref))
        assert len(ref) > 10
        _compare(b.read_events(q), ref, f"instance {q}")
    b.close()
