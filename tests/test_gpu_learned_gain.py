"""What the trained network gains over the plain sampler (the learned birth
proposal enters the MH ratio with its density, so both chains target the same
posterior; the gain can only be in how fast they get there).

The network is trained on the GPU by the library's own kernels on fresh
simulator pairs (fixed seeds); then on the same seeded 5x5-station worlds the
same chains run with prior births only and with learned births mixed 50/50.
Criterion, fixed in advance: the learned chains' mean F1 (Section 5's
matching) after a quarter of the sweeps is at least the plain chains' mean F1
after all of them, and the same holds per unit of GPU time (a learned sweep
costs more than a plain one).
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1612_00595_amd import workloads as W

from gpu_cases import say

pytestmark = pytest.mark.gpu

PAIRS = 2_000_000
WORLDS = (100, 101, 102, 103)
CHAINS = 16
SWEEPS = 400


def _run(w, trace, tr_ev, seed, table=None):
    from paper_1612_00595_amd import chromh, metrics as M
    smp = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=CHAINS, seed=seed)
    if table is not None:
        smp.set_learned(*table, 0.5)
    rec = smp.set_record(0, SWEEPS + 1, 256)
    smp.run_sweeps(0, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.run_sweeps(1, SWEEPS)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    f1 = {q: [] for q in (SWEEPS // 4, SWEEPS)}
    for c in range(CHAINS):
        states = chromh.ChromaticSampler.recorded_states(rec[1:], c)
        for q in f1:
            f1[q].append(M.match(tr_ev, states[q - 1]).f1)
    smp.close()
    return {q: float(np.mean(v)) for q, v in f1.items()}, el / SWEEPS


def test_learned_births_reach_the_plain_f1_in_a_quarter_of_the_sweeps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_00595_amd import chromh, learned
    w = W.SMALL
    say("training on", PAIRS, "simulator pairs")
    tr = learned.train(w.model, pairs=PAIRS, batch=8192, lr=1e-3, seed=0)
    say("held-out loss", tr.held_out, "in", round(tr.seconds, 2), "s")
    plain, learn, t_plain, t_learn = [], [], [], []
    for seed in WORLDS:
        tr_ev = W.truth_events(w.model, seed)
        truth = chromh.as_events(tr_ev["x"], tr_ev["y"], tr_ev["t"], tr_ev["m"])
        trace = chromh.simulate(w.model, truth, 1000 + seed, w.trace_dtype, "cuda")
        table = learned.anchor_table(tr.net, w.model, trace)
        fp, tp = _run(w, trace, tr_ev, seed)
        fl, tl = _run(w, trace, tr_ev, seed, table)
        say("world", seed, "plain F1", fp, "learned F1", fl, "ms/sweep", tp * 1e3, tl * 1e3)
        plain.append(fp); learn.append(fl); t_plain.append(tp); t_learn.append(tl)
    q = SWEEPS // 4
    p_end = np.mean([f[SWEEPS] for f in plain])
    l_q = np.mean([f[q] for f in learn])
    say("plain F1 after", SWEEPS, "sweeps", p_end, "; learned after", q, "sweeps", l_q)
    assert l_q >= p_end
    # per unit of GPU time: the learned chains' time to that F1 against the
    # plain chains' whole run
    assert q * np.mean(t_learn) < SWEEPS * np.mean(t_plain)
