"""CPU checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments on the host, and its partition and
colouring (a pure host function) agree bit for bit with the oracle."""
import ctypes as C
import dataclasses
import os
import re

import numpy as np
import pytest

from paper_1612_00595_amd import chromh, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "chromh.h")).read()
    return sorted(set(re.findall(r"\b(cmh_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for core in ("cmh_partition_and_color", "cmh_init_state", "cmh_sweep_color",
                 "cmh_run_sweeps", "cmh_read_events"):
        assert core in names
    assert set(names) == set(chromh.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    L = chromh.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_host_validation_errors():
    L = chromh.lib()
    m = chromh.model_struct(W.SMALL.model)
    s = chromh.sampler_struct(W.SMALL.sampler)
    nbytes = C.c_size_t()
    assert L.cmh_state_bytes(C.byref(m), C.byref(s), 1, C.byref(nbytes)) == 0
    assert nbytes.value > 25 * 1000 * 8
    bad = chromh.model_struct(W.SMALL.model)
    bad.r_c = 0.25  # must stay below the station spacing
    assert L.cmh_state_bytes(C.byref(bad), C.byref(s), 1, C.byref(nbytes)) == -1
    assert b"r_c" in L.cmh_last_error()
    bad = chromh.sampler_struct(W.SMALL.sampler)
    bad.p_mag = 0.5  # probabilities no longer sum to one
    assert L.cmh_state_bytes(C.byref(m), C.byref(bad), 1, C.byref(nbytes)) == -1
    bad = chromh.sampler_struct(W.SMALL.sampler)
    bad.region_capacity = 65
    assert L.cmh_state_bytes(C.byref(m), C.byref(bad), 1, C.byref(nbytes)) == -1
    bad = chromh.sampler_struct(W.SMALL.sampler)
    bad.block = 96
    assert L.cmh_state_bytes(C.byref(m), C.byref(bad), 1, C.byref(nbytes)) == -1
    # the speculative forms: 2, 4 or 8 waves per region, not with latent
    # arrivals or the naive schedule
    for block, want in ((chromh.SPEC2, 0), (chromh.SPEC4, 0), (chromh.SPEC8, 0),
                        (chromh.BLOCK_SPEC + 64, -1), (chromh.BLOCK_SPEC + 1024, -1)):
        sb = chromh.sampler_struct(W.SMALL.sampler, block)
        assert L.cmh_state_bytes(C.byref(m), C.byref(sb), 1, C.byref(nbytes)) == want, block
    lm = chromh.model_struct(W.PAPER1D_LATENT.model)
    sb = chromh.sampler_struct(W.PAPER1D_LATENT.sampler, chromh.SPEC4)
    assert L.cmh_state_bytes(C.byref(lm), C.byref(sb), 1, C.byref(nbytes)) == -1
    sb = chromh.sampler_struct(dataclasses.replace(W.SMALL.sampler, schedule=1), chromh.SPEC4)
    assert L.cmh_state_bytes(C.byref(m), C.byref(sb), 1, C.byref(nbytes)) == -1
    assert L.cmh_state_bytes(C.byref(m), C.byref(s), 0, C.byref(nbytes)) == -1
    # a static period that leaves dependent regions in one colour
    bad = chromh.sampler_struct(W.SMALL.sampler)
    bad.period = 1
    assert L.cmh_state_bytes(C.byref(m), C.byref(bad), 1, C.byref(nbytes)) == -4
    h = C.c_void_p()
    assert L.cmh_init_state(C.byref(m), C.byref(s), None, 0, 1, 0, None, 0, None,
                            C.byref(h)) == -1
    assert L.cmh_destroy(None) == 0
    nxt = C.c_int64()
    assert L.cmh_tune_running(None, 0, 1, None, C.byref(nxt)) == -1
    # the training loop: refused before any device work for a model without
    # training pairs, zero steps, Adam steps from 0, or missing buffers
    lm = chromh.model_struct(W.PAPER1D.model)
    args = (None, 0, 0, 8, 1024, 1, C.c_float(1e-3), None, None, None, None, 0, None)
    assert L.cmh_mdn_train(None, C.byref(lm), *args[1:]) == -1
    assert b"grid model" in L.cmh_last_error()
    assert L.cmh_mdn_train(None, C.byref(m), 0, 0, 0, 1024, 1, C.c_float(1e-3), None, None, None,
                           None, 0, None) == -1
    assert L.cmh_mdn_train(None, C.byref(m), 0, 0, 4, 1024, 0, C.c_float(1e-3), None, None, None,
                           None, 0, None) == -1
    assert L.cmh_mdn_train(None, C.byref(m), 0, 0, 4, 1024, 1, C.c_float(1e-3), None, None, None,
                           None, 0, None) == -1
    assert b"NULL" in L.cmh_last_error()


@pytest.mark.parametrize("side,grid,dynamic", [(5, 4, 0), (5, 5, 1), (12, 12, 1), (8, 3, 0),
                                               (16, 16, 1)])
def test_partition_matches_oracle(orc, side, grid, dynamic):
    spec = W.ModelSpec(nsx=side, nsy=side, N=100)
    om = orc.make_model(**spec.asdict())
    rng = np.random.default_rng(side * 100 + grid)
    L = side * 0.2
    w = L / grid
    offs = [(0.0, 0.0)] + ([tuple(rng.random(2) * w) for _ in range(25)] if dynamic else [])
    for ox, oy in offs:
        got = chromh.partition_and_color(spec, grid, grid, ox, oy, dynamic)
        rc, *want = orc.partition_and_color(om, grid, grid, ox, oy, dynamic)
        assert rc == 0
        assert got[:4] == tuple(want[:4])
        assert np.array_equal(got[4], want[4])


@pytest.mark.parametrize("ts,gx,dynamic", [(10, 4, 0), (10, 4, 1), (11, 4, 0), (11, 4, 1),
                                           (10, 8, 1), (3, 12, 0)])
def test_line_partition_matches_oracle(orc, ts, gx, dynamic):
    """The line model's time partition and colours (host code of the library)
    against the oracle's, at shifted and unshifted onset offsets."""
    import dataclasses
    spec = dataclasses.replace(W.PAPER1D_MODEL, ts=ts)
    om = orc.make_model(**spec.asdict())
    w = spec.N / gx
    rng = np.random.default_rng(ts * 100 + gx)
    offs = [0.0] + ([float(v) for v in rng.random(25) * w] if dynamic else [])
    for off in offs:
        got = chromh.partition_and_color(spec, gx, 0, off, 0.0, dynamic)
        rc, *want = orc.partition_and_color(om, gx, 0, off, 0.0, dynamic)
        assert rc == 0
        assert got[:4] == tuple(want[:4])
        assert np.array_equal(got[4], want[4])


def test_line_model_validation():
    import dataclasses
    spec = W.PAPER1D_MODEL
    with pytest.raises(chromh.CmhError):  # a second region axis
        chromh.partition_and_color(spec, 4, 1, 0.0, 0.0, 0)
    with pytest.raises(chromh.CmhError):  # more than 8 stations on a line
        chromh.partition_and_color(dataclasses.replace(spec, nsx=9), 4, 0, 0.0, 0.0, 0)
    with pytest.raises(chromh.CmhError):  # offset outside [0, w)
        chromh.partition_and_color(spec, 4, 0, 60.0, 0.0, 1)


def test_owner_check_validation_and_workspace(orc):
    """The debug owner check: its bits, its modes, its workspace (8 bytes per
    sample per chain), and the unchecked period that only it may request."""
    L = chromh.lib()
    m = chromh.model_struct(W.SMALL.model)
    nb = C.c_size_t()
    sizes = {}
    for debug in (0, 1):
        s = chromh.sampler_struct(W.SMALL.sampler)
        s.debug = debug
        assert L.cmh_state_bytes(C.byref(m), C.byref(s), 3, C.byref(nb)) == 0
        sizes[debug] = nb.value
    assert sizes[1] - sizes[0] >= 3 * W.SMALL.model.nsta * W.SMALL.model.N * 8
    assert sizes[1] - sizes[0] <= 3 * W.SMALL.model.nsta * W.SMALL.model.N * 8 + 4096

    def rc(**kw):
        s = chromh.sampler_struct(W.SMALL.sampler)
        for k, v in kw.items():
            setattr(s, k, v)
        return L.cmh_state_bytes(C.byref(m), C.byref(s), 1, C.byref(nb))

    assert rc(debug=8) == -1
    assert rc(debug=4) == 0                 # persistent-form waits give up at once
    assert rc(block=chromh.PERSIST) == -1   # static partition: refused
    s2 = chromh.sampler_struct(W.SamplerSpec(gx=5, gy=5, dynamic=1), chromh.PERSIST)
    assert L.cmh_state_bytes(C.byref(m), C.byref(s2), 1, C.byref(nb)) == 0
    assert rc(debug=2, period=1) == -1      # unchecked period without the owner check
    assert rc(debug=3, period=0) == -1      # unchecked, but no period given
    assert rc(debug=1, schedule=1, block=64) == -1  # naive regions share samples by design
    # period 1 puts neighbouring regions in one colour: refused, unless forced
    om = orc.make_model(**W.SMALL.model.asdict())
    assert orc.coloring_violations(om, W.SMALL.sampler.gx, W.SMALL.sampler.gy, 0.0, 0.0, 1) > 0
    assert rc(period=1) == -4
    assert rc(debug=1, period=1) == -4
    assert rc(debug=3, period=1) == 0
    assert chromh.ERRORS[-7] == "ERACE"
