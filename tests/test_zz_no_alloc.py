"""The no-allocation simulator entry point (cmh_simulate_noalloc): called
through the C-ABI, its traces equal those of cmh_simulate (the workspace
form, same kernels) element for element, on two calls in a row, the second
with a smaller input; a truth layout beyond its scratch is refused."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1612_00595_amd import workloads as W

from gpu_cases import say

pytestmark = pytest.mark.gpu


def _noalloc(chromh, model, truth, seed, dtype):
    truth = np.ascontiguousarray(truth, dtype=chromh.EVENT_DTYPE)
    m = chromh.model_struct(model)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    trace = torch.full((model.nsta, model.N), float("nan"), dtype=tdt, device="cuda")
    torch.cuda.synchronize()
    rc = chromh.lib().cmh_simulate_noalloc(C.byref(m), chromh._ptr(truth), len(truth), seed,
                                           C.c_void_p(trace.data_ptr()),
                                           chromh.CMH_F32 if dtype == "f32" else chromh.CMH_F64,
                                           None)
    return rc, trace


def test_noalloc_simulator_matches_the_workspace_form():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_00595_amd import chromh
    big = W.ModelSpec(nsx=32, nsy=32, N=36000, lam=5000.0)
    small = W.SMALL.model
    for model, seed, dtype in ((big, 2, "f32"), (small, 5, "f64")):
        tr = W.truth_events(model, seed)
        truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"], tr["id"])
        say("no-alloc simulate", model.nsx, "x", model.nsy, model.N, "samples,", len(truth),
            "events", dtype)
        rc, got = _noalloc(chromh, model, truth, 1000 + seed, dtype)
        assert rc == 0, chromh.lib().cmh_last_error()
        ref = chromh.simulate(model, truth, 1000 + seed, dtype, "cuda")
        assert torch.equal(got, ref)
    # a layout beyond the scratch: refused before any device work
    huge = W.ModelSpec(nsx=256, nsy=256, N=1000, lam=1.0)
    tr = W.truth_events(huge, 1, n=200000)
    truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"], tr["id"])
    rc, got = _noalloc(chromh, huge, truth, 1, "f32")
    assert rc == -1
    assert b"scratch" in chromh.lib().cmh_last_error()
    assert torch.isnan(got).all()
