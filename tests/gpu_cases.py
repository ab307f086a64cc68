"""Instances and comparison helpers shared by the GPU parity tests.

Inputs come from paper_1612_00595_amd.workloads (truth events, replay
draws, noise) and from the oracle (traces); nothing flows from the GPU into
the oracle.
"""
from __future__ import annotations

import dataclasses
import sys

import numpy as np

import oracle as O
from paper_1612_00595_amd import workloads as W


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def instance(w: W.Workload, trace_seed: int = 1000):
    """(oracle model, oracle sampler, truth events, trace as numpy) for a
    workload; fp64 traces by the oracle simulator, fp32 traces by the oracle
    from seeded standard normals."""
    m = O.make_model(**w.model.asdict())
    sp = O.make_sampler(**w.sampler.asdict())
    tr = W.truth_events(w.model, w.seed)
    truth = O.as_events(tr["x"], tr["y"], tr["t"], tr["m"], tr["id"], da=tr.get("da"))
    if w.trace_dtype == "f64":
        s = O.simulate(m, truth, trace_seed + w.seed)
    else:
        rng = np.random.Generator(np.random.PCG64(trace_seed + w.seed))
        z = rng.standard_normal((w.model.nsta, w.model.N), dtype=np.float32)
        s = O.trace_from_noise_f32(m, truth, z)
    return m, sp, truth, s


def dynamic_small() -> W.Workload:
    """10x10 stations, 3000 fp32 samples, shifted 10x10 regions."""
    model = W.ModelSpec(nsx=10, nsy=10, N=3000, lam=150.0)
    sampler = W.SamplerSpec(gx=10, gy=10, dynamic=1, k=16)
    return W.Workload(name="s10x10-n3000-dyn10x10-f32", model=model, sampler=sampler,
                      trace_dtype="f32", sweeps=10, seed=5)


def compare_events(a: np.ndarray, b: np.ndarray, where: str):
    assert len(a) == len(b), f"{where}: {len(a)} events on the GPU, {len(b)} in the oracle"
    for f in ("id", "region", "x", "y", "t", "m", "da"):
        if not np.array_equal(a[f], b[f]):
            bad = np.nonzero(a[f] != b[f])[0][:5]
            raise AssertionError(f"{where}: field {f} differs at {bad}: {a[f][bad]} vs {b[f][bad]}")


@dataclasses.dataclass
class LogCheck:
    moves: int = 0
    evaluated: int = 0
    ties: int = 0
    max_rel: float = 0.0


def compare_logs(g: np.ndarray, r: np.ndarray, feed: np.ndarray, acc: LogCheck, where: str):
    """Move logs [regions, k, 4]: type and validity identical, log-likelihood
    changes within 1e-4 relative (floor 1 nat), decisions identical wherever
    |log u - log alpha| > 1e-6.  Returns False when a decision differs inside
    that band (the chains may then part, which the contract allows)."""
    written = r[..., 1] >= 0
    assert np.array_equal(g[..., 1] >= 0, written), f"{where}: different moves logged"
    live = r[..., 1] > 0
    assert np.array_equal(g[..., 0][written], r[..., 0][written]), f"{where}: move types differ"
    assert np.array_equal(g[..., 1] > 0, live), f"{where}: validity differs"
    acc.moves += int(np.sum(r[..., 1] >= 0))
    if not live.any():
        return True
    dg, dr = g[..., 2][live], r[..., 2][live]
    rel = np.abs(dg - dr) / np.maximum(np.abs(dr), 1.0)
    acc.max_rel = max(acc.max_rel, float(rel.max()))
    assert rel.max() <= 1e-4, f"{where}: delta relative error {rel.max()}"
    ag, ar = g[..., 3][live], r[..., 3][live]
    rel_a = np.abs(ag - ar) / np.maximum(np.abs(ar), 1.0)
    assert rel_a.max() <= 1e-4, f"{where}: log alpha relative error {rel_a.max()}"
    lnu = feed[..., 7][live]
    la = r[..., 3][live]
    tie = np.abs(lnu - la) <= 1e-6
    same = (g[..., 1][live] == r[..., 1][live])
    acc.evaluated += int(live.sum())
    acc.ties += int(tie.sum())
    assert np.all(same | tie), f"{where}: decision differs outside the tie band"
    return bool(np.all(same))
