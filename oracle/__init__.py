"""FP64 CPU oracle of the chromatic Metropolis-Hastings sampler.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; the product path never touches it.
It shares no code with the GPU library (``paper_1612_00595_amd``); both sides
receive their inputs from ``paper_1612_00595_amd.workloads``, which holds only
seeded generators and workload constants.

The C sources (``orc_model.c``, ``orc_sampler.c``) carry the citations of the
paper's sections, equations and algorithms; this module only marshals numpy
arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SOURCES = ["orc_model.c", "orc_sampler.c"]

BIRTH, DEATH, LOC, TIME, MAG, ARR, JOINT = range(7)
ARR_TRUNC = 4.0  # the arrival-time jitter is truncated at this many sds
SCHED_CHROMATIC, SCHED_NAIVE = 0, 1

EVENT_DTYPE = np.dtype([("x", "<f8"), ("y", "<f8"), ("t", "<f8"), ("m", "<f8"),
                        ("id", "<u8"), ("region", "<i4"), ("_pad", "<i4"),
                        ("da", "<f8", (8,))])


class Model(C.Structure):
    _fields_ = [("nsx", C.c_int32), ("nsy", C.c_int32), ("ds", C.c_double),
                ("N", C.c_int64), ("sigma", C.c_double), ("atten", C.c_double),
                ("vel", C.c_double), ("decay", C.c_double), ("ts", C.c_int32),
                ("_pad0", C.c_int32), ("rc", C.c_double), ("lam", C.c_double),
                ("mmin", C.c_double), ("mrate", C.c_double), ("line", C.c_int32),
                ("tmpl", C.c_int32), ("xmax", C.c_double), ("sta_x", C.c_double * 8),
                ("arr_sd", C.c_double)]


class Sampler(C.Structure):
    _fields_ = [("gx", C.c_int32), ("gy", C.c_int32), ("dynamic", C.c_int32),
                ("period", C.c_int32), ("k", C.c_int32), ("cap", C.c_int32),
                ("pb", C.c_double), ("pd", C.c_double), ("ploc", C.c_double),
                ("pt", C.c_double), ("pm", C.c_double), ("sxy", C.c_double),
                ("st", C.c_double), ("sm", C.c_double), ("prior_only", C.c_int32),
                ("schedule", C.c_int32), ("lattice", C.c_int32), ("kx", C.c_int32),
                ("ky", C.c_int32), ("kt", C.c_int32), ("km", C.c_int32),
                ("_pad1", C.c_int32), ("hm", C.c_double), ("pa", C.c_double),
                ("pj", C.c_double), ("sa", C.c_double)]


def build(force: bool = True) -> str:
    """Compile liborc.so with gcc (plain C, FP64, no FMA contraction)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH) and all(
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(s) for s in srcs):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-fopenmp",
           "-shared", "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_u01.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_move_draws.argtypes = [C.c_uint32] * 5 + [P]
        L.orc_offset.argtypes = [C.c_uint32] * 3 + [C.c_double, C.c_double, P, P]
        L.orc_region_axis.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_region_axis.restype = C.c_int32
        L.orc_partition_and_color.argtypes = [P, C.c_int32, C.c_int32, C.c_double,
                                              C.c_double, C.c_int32, P, P, P, P, P]
        L.orc_partition_and_color.restype = C.c_int32
        L.orc_coloring_violations.argtypes = [P, C.c_int32, C.c_int32, C.c_double,
                                              C.c_double, C.c_int32]
        L.orc_coloring_violations.restype = C.c_int64
        L.orc_line_tau_max.argtypes = [P]
        L.orc_line_tau_max.restype = C.c_double
        L.orc_arrival_time.argtypes = [C.c_double] * 6 + [P]
        L.orc_arrival_time.restype = C.c_double
        L.orc_event_variance.argtypes = [P, P, C.c_int64, P]
        L.orc_event_variance_rows.argtypes = [P, P, C.c_int64, C.c_int64, C.c_int64, P]
        L.orc_loglik.argtypes = [P, P, P, C.c_int64]
        L.orc_loglik.restype = C.c_double
        L.orc_logprior.argtypes = [P, P, C.c_int64]
        L.orc_logprior.restype = C.c_double
        L.orc_single_term.argtypes = [C.c_double] * 3
        L.orc_single_term.restype = C.c_double
        L.orc_simulate.argtypes = [P, P, C.c_int64, C.c_uint32, P]
        L.orc_simulate_rows.argtypes = [P, P, C.c_int64, C.c_uint32, C.c_int64, C.c_int64, P]
        L.orc_trace_from_noise_f32.argtypes = [P, P, C.c_int64, P, P]
        L.orc_chain_new.argtypes = [P, P, P, C.c_uint32, C.c_uint32]
        L.orc_chain_new.restype = P
        L.orc_chain_new_f32.argtypes = [P, P, P, C.c_uint32, C.c_uint32]
        L.orc_chain_new_f32.restype = P
        L.orc_chain_free.argtypes = [P]
        L.orc_chain_begin_sweep.argtypes = [P, C.c_int64]
        L.orc_chain_begin_sweep.restype = C.c_int32
        L.orc_chain_phase.argtypes = [P, C.c_int64, C.c_int32, P, P]
        L.orc_chain_phase.restype = C.c_int32
        L.orc_chain_sweep.argtypes = [P, C.c_int64, P, P]
        L.orc_chain_sweep.restype = C.c_int32
        L.orc_chain_set_threads.argtypes = [P, C.c_int32]
        L.orc_chain_count.argtypes = [P]
        L.orc_chain_count.restype = C.c_int64
        L.orc_chain_events.argtypes = [P, P, C.c_int64]
        L.orc_chain_events.restype = C.c_int64
        L.orc_chain_set_events.argtypes = [P, P, C.c_int64]
        L.orc_chain_set_events.restype = C.c_int32
        L.orc_chain_layout.argtypes = [P] * 7
        L.orc_chain_overflows.argtypes = [P]
        L.orc_chain_overflows.restype = C.c_int64
        L.orc_chain_delta.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, P]
        L.orc_chain_delta.restype = C.c_double
        L.orc_chain_set_learned.argtypes = [P, P, P, C.c_int32, C.c_double]
        L.orc_chain_set_learned.restype = C.c_int32
        L.orc_move_draws16.argtypes = [C.c_uint32] * 5 + [P]
        L.orc_move_draws_arr.argtypes = [C.c_uint32] * 5 + [P]
        L.orc_line_fit.argtypes = [P, P, P, P]
        L.orc_chain_learned_q.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_chain_learned_q.restype = C.c_double
        L.orc_chain_learned_draw.argtypes = [P, C.c_int32, P, P]
        L.orc_chain_learned_draw.restype = C.c_int32
        L.orc_lattice_nsites.argtypes = [P, P]
        L.orc_lattice_nsites.restype = C.c_int64
        L.orc_lattice_site.argtypes = [P, P, C.c_int64, P]
        L.orc_enumerate.argtypes = [P, P, P, C.c_int32, P, P, C.c_int64]
        L.orc_enumerate.restype = C.c_int64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_model(**kw) -> Model:
    m = Model()
    m.nsx = kw["nsx"]; m.nsy = kw["nsy"]; m.ds = kw["ds"]; m.N = kw["N"]
    m.sigma = kw["sigma"]; m.atten = kw["atten"]; m.vel = kw["vel"]; m.decay = kw["decay"]
    m.ts = kw["ts"]; m.rc = kw["rc"]; m.lam = kw["lam"]; m.mmin = kw["mmin"]
    m.mrate = kw["mrate"]
    m.line = kw.get("line", 0)
    m.tmpl = kw.get("tmpl", 0)
    m.xmax = kw.get("xmax", 0.0)
    m.arr_sd = kw.get("arr_sd", 0.0)
    sx = tuple(kw.get("sta_x", ()))
    assert len(sx) <= 8
    for j, v in enumerate(sx):
        m.sta_x[j] = v
    return m


def make_sampler(**kw) -> Sampler:
    s = Sampler()
    for name, _ in Sampler._fields_:
        if name.startswith("_"):
            continue
        if name in kw:
            setattr(s, name, kw[name])
    return s


def events_array(n: int = 0) -> np.ndarray:
    return np.zeros(n, dtype=EVENT_DTYPE)


def as_events(x, y, t, m, ids=None, da=None) -> np.ndarray:
    ev = events_array(len(x))
    ev["x"], ev["y"], ev["t"], ev["m"] = x, y, t, m
    ev["id"] = np.arange(len(x), dtype=np.uint64) if ids is None else ids
    if da is not None:
        ev["da"] = da
    return ev


# ---------------------------------------------------------------- wrappers

def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def u01(w0: int, w1: int) -> float:
    return lib().orc_u01(w0, w1)


def move_draws(seed, chain, sweep, region, j) -> np.ndarray:
    out = np.zeros(8)
    lib().orc_move_draws(seed, chain, sweep, region, j, _ptr(out))
    return out


def move_draws16(seed, chain, sweep, region, j) -> np.ndarray:
    out = np.zeros(16)
    lib().orc_move_draws16(seed, chain, sweep, region, j, _ptr(out))
    return out


def move_draws_arr(seed, chain, sweep, region, j) -> np.ndarray:
    out = np.zeros(16)
    lib().orc_move_draws_arr(seed, chain, sweep, region, j, _ptr(out))
    return out


def line_fit(model: Model, arrivals) -> tuple[float, float]:
    a = np.zeros(8)
    a[:model.nsx] = arrivals
    x, t = C.c_double(), C.c_double()
    lib().orc_line_fit(C.byref(model), _ptr(a), C.byref(x), C.byref(t))
    return x.value, t.value


def offset(seed, chain, sweep, wx, wy):
    dx, dy = C.c_double(), C.c_double()
    lib().orc_offset(seed, chain, sweep, wx, wy, C.byref(dx), C.byref(dy))
    return dx.value, dy.value


def region_axis(x, off, w, g) -> int:
    return lib().orc_region_axis(x, off, w, g)


def partition_and_color(model: Model, gx, gy, offx, offy, dynamic):
    nrx, nry, p, nc = (C.c_int32() for _ in range(4))
    color = np.zeros((gx + 1) * (1 if model.line else gy + 1), dtype=np.int32)
    rc = lib().orc_partition_and_color(C.byref(model), gx, gy, offx, offy, dynamic,
                                       C.byref(nrx), C.byref(nry), C.byref(p), C.byref(nc),
                                       _ptr(color))
    return rc, nrx.value, nry.value, p.value, nc.value, color


def coloring_violations(model: Model, gx, gy, offx, offy, period) -> int:
    return lib().orc_coloring_violations(C.byref(model), gx, gy, offx, offy, period)


def line_tau_max(model: Model) -> float:
    return lib().orc_line_tau_max(C.byref(model))


def arrival_time(x, y, t, sx, sy, vel) -> float:
    return lib().orc_arrival_time(x, y, t, sx, sy, vel, None)


def event_variance(model: Model, ev: np.ndarray) -> np.ndarray:
    ev = np.ascontiguousarray(ev, dtype=EVENT_DTYPE)
    E = np.zeros((model.nsx * model.nsy, model.N))
    lib().orc_event_variance(C.byref(model), _ptr(ev), len(ev), _ptr(E))
    return E


def event_variance_rows(model: Model, ev: np.ndarray, j0: int, nrows: int) -> np.ndarray:
    ev = np.ascontiguousarray(ev, dtype=EVENT_DTYPE)
    E = np.zeros((nrows, model.N))
    lib().orc_event_variance_rows(C.byref(model), _ptr(ev), len(ev), j0, nrows, _ptr(E))
    return E


def loglik(model: Model, s: np.ndarray, ev: np.ndarray) -> float:
    s = np.ascontiguousarray(s, dtype=np.float64)
    ev = np.ascontiguousarray(ev, dtype=EVENT_DTYPE)
    return lib().orc_loglik(C.byref(model), _ptr(s), _ptr(ev), len(ev))


def logprior(model: Model, ev: np.ndarray) -> float:
    ev = np.ascontiguousarray(ev, dtype=EVENT_DTYPE)
    return lib().orc_logprior(C.byref(model), _ptr(ev), len(ev))


def single_term(sigma, s, e) -> float:
    return lib().orc_single_term(sigma, s, e)


def simulate(model: Model, truth: np.ndarray, seed: int) -> np.ndarray:
    truth = np.ascontiguousarray(truth, dtype=EVENT_DTYPE)
    s = np.zeros((model.nsx * model.nsy, model.N))
    lib().orc_simulate(C.byref(model), _ptr(truth), len(truth), seed, _ptr(s))
    return s


def simulate_rows(model: Model, truth: np.ndarray, seed: int, j0: int, nrows: int) -> np.ndarray:
    truth = np.ascontiguousarray(truth, dtype=EVENT_DTYPE)
    s = np.zeros((nrows, model.N))
    lib().orc_simulate_rows(C.byref(model), _ptr(truth), len(truth), seed, j0, nrows, _ptr(s))
    return s


def trace_from_noise_f32(model: Model, truth: np.ndarray, z: np.ndarray) -> np.ndarray:
    truth = np.ascontiguousarray(truth, dtype=EVENT_DTYPE)
    z = np.ascontiguousarray(z, dtype=np.float32)
    assert z.size == model.nsx * model.nsy * model.N
    out = np.empty_like(z)
    lib().orc_trace_from_noise_f32(C.byref(model), _ptr(truth), len(truth), _ptr(z), _ptr(out))
    return out


class Chain:
    """One oracle chain.  The trace array is kept alive by the object; a
    float32 trace is read as is (each sample widened to binary64)."""

    def __init__(self, model: Model, sampler: Sampler, s: np.ndarray, seed: int, chain: int = 0):
        self.model, self.sampler = model, sampler
        if s.dtype == np.float32:
            self.s = np.ascontiguousarray(s)
            self._h = lib().orc_chain_new_f32(C.byref(model), C.byref(sampler), _ptr(self.s),
                                              seed, chain)
        else:
            self.s = np.ascontiguousarray(s, dtype=np.float64)
            self._h = lib().orc_chain_new(C.byref(model), C.byref(sampler), _ptr(self.s), seed,
                                          chain)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_chain_free(self._h)
            self._h = None

    def begin_sweep(self, sweep: int) -> int:
        return lib().orc_chain_begin_sweep(self._h, sweep)

    def phase(self, sweep, color, feed=None, log=None) -> int:
        return lib().orc_chain_phase(self._h, sweep, color,
                                     None if feed is None else _ptr(feed),
                                     None if log is None else _ptr(log))

    def sweep(self, sweep, feed=None, log=None) -> int:
        return lib().orc_chain_sweep(self._h, sweep, None if feed is None else _ptr(feed),
                                     None if log is None else _ptr(log))

    def count(self) -> int:
        return lib().orc_chain_count(self._h)

    def set_threads(self, threads: int):
        """Run the regions of each colour phase on `threads` host threads."""
        lib().orc_chain_set_threads(self._h, threads)

    def events(self) -> np.ndarray:
        n = self.count()
        out = events_array(n)
        lib().orc_chain_events(self._h, _ptr(out), n)
        return out

    def set_events(self, ev: np.ndarray) -> int:
        ev = np.ascontiguousarray(ev, dtype=EVENT_DTYPE)
        return lib().orc_chain_set_events(self._h, _ptr(ev), len(ev))

    def layout(self):
        a, b, c, d = (C.c_int32() for _ in range(4))
        ox, oy = C.c_double(), C.c_double()
        lib().orc_chain_layout(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d),
                               C.byref(ox), C.byref(oy))
        return dict(nrx=a.value, nry=b.value, period=c.value, ncolors=d.value,
                    offx=ox.value, offy=oy.value)

    def overflows(self) -> int:
        return lib().orc_chain_overflows(self._h)

    def set_learned(self, table, weights, n_tau: int, p_learned: float = 0.5) -> int:
        """Learned births from a mixture table [nsta * n_tau][8][8] and anchor
        weights [nsta * n_tau] (both kept alive here); table None: off."""
        if table is None:
            self._ltab = self._lw = None
            return lib().orc_chain_set_learned(self._h, None, None, 0, 0.0)
        self._ltab = np.ascontiguousarray(table, dtype=np.float64)
        self._lw = np.ascontiguousarray(weights, dtype=np.float64)
        return lib().orc_chain_set_learned(self._h, _ptr(self._ltab), _ptr(self._lw), n_tau,
                                           p_learned)

    def learned_q(self, region, x, y, t) -> float:
        return lib().orc_chain_learned_q(self._h, region, x, y, t)

    def learned_draw(self, region, d16) -> np.ndarray:
        d = np.ascontiguousarray(d16, dtype=np.float64)
        out = np.zeros(3)
        rc = lib().orc_chain_learned_draw(self._h, region, _ptr(d), _ptr(out))
        assert rc == 0
        return out

    def delta(self, region, mtype, idx, proposed) -> float:
        p = np.ascontiguousarray(proposed, dtype=EVENT_DTYPE).reshape(1)
        return lib().orc_chain_delta(self._h, region, mtype, idx, _ptr(p))


def lattice_nsites(model: Model, sampler: Sampler) -> int:
    return lib().orc_lattice_nsites(C.byref(model), C.byref(sampler))


def lattice_site(model: Model, sampler: Sampler, site: int) -> np.ndarray:
    out = events_array(1)
    lib().orc_lattice_site(C.byref(model), C.byref(sampler), site, _ptr(out))
    return out[0]


def enumerate_posterior(model: Model, sampler: Sampler, s: np.ndarray, nmax: int):
    """All multisets of <= nmax lattice sites and their log weights."""
    from math import comb
    S = lattice_nsites(model, sampler)
    cap = sum(comb(S + n - 1, n) for n in range(nmax + 1))
    sites = np.zeros((cap, max(nmax, 1)), dtype=np.int32)
    logw = np.zeros(cap)
    s = np.ascontiguousarray(s, dtype=np.float64)
    n = lib().orc_enumerate(C.byref(model), C.byref(sampler), _ptr(s), nmax, _ptr(sites),
                            _ptr(logw), cap)
    assert n == cap
    return sites[:, :nmax], logw
