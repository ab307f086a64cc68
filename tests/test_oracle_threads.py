"""The oracle's colour phases on several host threads (the regions of one
colour are conditionally independent given the others, Section 4.1, which is
the parallelism the paper's own implementation used) give the same chain, bit
for bit, as the serial loop: plain, dynamic, learned births, the line model
with latent arrivals, and the naive schedule."""
import dataclasses

import numpy as np
import pytest

from paper_1612_00595_amd import workloads as W


def _run(orc, w, threads, sweeps, learned=False):
    m = orc.make_model(**w.model.asdict())
    sp = orc.make_sampler(**w.sampler.asdict())
    tr = W.truth_events(w.model, w.seed)
    truth = orc.as_events(tr["x"], tr["y"], tr["t"], tr["m"], da=tr.get("da"))
    s = orc.simulate(m, truth, 500 + w.seed)
    ch = orc.Chain(m, sp, s, seed=3)
    ch.set_threads(threads)
    if learned:
        T, wts, ntau = W.random_mixture_table(w.model, 2, near=truth)
        assert ch.set_learned(T, wts, ntau, 0.5) == 0
    for sw in range(sweeps):
        assert ch.sweep(sw) == 0
    return ch.events(), ch.overflows()


@pytest.mark.parametrize("case", ["small", "dynamic", "learned", "latent", "naive"])
def test_threaded_phases_give_the_same_chain(orc, case):
    learned = False
    if case == "small":
        w = W.SMALL
    elif case == "dynamic":
        w = dataclasses.replace(W.SMALL, sampler=dataclasses.replace(W.SMALL.sampler, dynamic=1,
                                                                     gx=5, gy=5))
    elif case == "learned":
        w, learned = W.SMALL, True
    elif case == "latent":
        w = dataclasses.replace(W.PAPER1D_LATENT, sampler=dataclasses.replace(
            W.PAPER1D_LATENT.sampler, dynamic=1, k=100))
    else:
        w = dataclasses.replace(W.PAPER1D, sampler=dataclasses.replace(W.PAPER1D.sampler,
                                                                       schedule=1, k=100))
    a, oa = _run(orc, w, 1, 30, learned)
    b, ob = _run(orc, w, 4, 30, learned)
    assert len(a) > 0 and oa == ob
    for f in ("id", "region", "x", "y", "t", "m", "da"):
        assert np.array_equal(a[f], b[f]), f
