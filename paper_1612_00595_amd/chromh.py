"""Python binding of libchromh.so (include/chromh.h).

Argument marshalling only: every step of the sampler runs in the HIP
library.  PyTorch provides device memory (traces, workspaces, feed and log
arrays) and the stream.  If the library is missing the import of a function
here raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .workloads import ModelSpec, SamplerSpec

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchromh.so")

CMH_F32, CMH_F64 = 0, 1
ERRORS = {-1: "EINVAL", -2: "EHIP", -3: "ECAP", -4: "ECOLOR", -5: "ENAN", -6: "ESTATE",
          -7: "ERACE"}

EVENT_DTYPE = np.dtype([("x", "<f8"), ("y", "<f8"), ("t", "<f8"), ("m", "<f8"),
                        ("id", "<u8"), ("region", "<i4"), ("_pad", "<i4"),
                        ("da", "<f8", (8,))])
N_STATS = 23


class CmhModel(C.Structure):
    _fields_ = [("nsx", C.c_int32), ("nsy", C.c_int32), ("ds", C.c_double),
                ("n_samples", C.c_int64), ("sigma", C.c_double), ("atten", C.c_double),
                ("velocity", C.c_double), ("env_decay", C.c_double), ("t_s", C.c_int32),
                ("_pad0", C.c_int32), ("r_c", C.c_double), ("lam", C.c_double),
                ("mag_min", C.c_double), ("mag_rate", C.c_double), ("line", C.c_int32),
                ("template_mean", C.c_int32), ("x_max", C.c_double),
                ("station_x", C.c_double * 8), ("arrival_sd", C.c_double)]


class CmhSampler(C.Structure):
    _fields_ = [("grid_x", C.c_int32), ("grid_y", C.c_int32), ("dynamic", C.c_int32),
                ("period", C.c_int32), ("moves_per_region", C.c_int32),
                ("region_capacity", C.c_int32), ("p_birth", C.c_double),
                ("p_death", C.c_double), ("p_loc", C.c_double), ("p_time", C.c_double),
                ("p_mag", C.c_double), ("step_xy", C.c_double), ("step_t", C.c_double),
                ("step_m", C.c_double), ("prior_only", C.c_int32), ("block", C.c_int32),
                ("schedule", C.c_int32), ("debug", C.c_int32), ("p_arrival", C.c_double),
                ("p_joint", C.c_double), ("step_arrival", C.c_double),
                ("refresh_every", C.c_int32), ("_pad0", C.c_int32)]


class CmhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


EXPORTS = ["cmh_last_error", "cmh_partition_and_color", "cmh_state_bytes", "cmh_init_state",
           "cmh_sweep_color", "cmh_run_sweeps", "cmh_read_events", "cmh_write_events",
           "cmh_set_feed", "cmh_set_log", "cmh_refresh", "cmh_read_variance", "cmh_read_stats",
           "cmh_get_block", "cmh_autotune", "cmh_tune_running", "cmh_time_phases", "cmh_destroy", "cmh_simulate_bytes", "cmh_simulate",
           "cmh_move_draws", "cmh_move_draws_arrivals", "cmh_mdn_sizes", "cmh_mdn_param_bytes", "cmh_mdn_init",
           "cmh_mdn_set_params", "cmh_mdn_get_params", "cmh_mdn_work_bytes", "cmh_mdn_forward",
           "cmh_mdn_infer",
           "cmh_mdn_gradients", "cmh_mdn_train_step", "cmh_mdn_train", "cmh_mdn_pairs",
           "cmh_anchor_count",
           "cmh_anchor_features", "cmh_mixture_table", "cmh_learned_bytes",
           "cmh_set_learned", "cmh_set_record", "cmh_batch_bytes", "cmh_batch_init",
           "cmh_batch_learned_bytes", "cmh_batch_set_learned", "cmh_checkpoint_bytes", "cmh_save",
           "cmh_load", "cmh_set_stamps", "cmh_stamp_rate", "cmh_log_posterior", "cmh_set_logprob",
           "cmh_simulate_noalloc"]

_lib = None


def lib():
    """Loads libchromh.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1612_00595_amd.build` (HIP, gfx950)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U32, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    sig = {
        "cmh_last_error": ([], C.c_char_p),
        "cmh_partition_and_color": ([P, I32, I32, D, D, I32, P, P, P, P, P], I32),
        "cmh_state_bytes": ([P, P, I32, P], I32),
        "cmh_init_state": ([P, P, P, I32, I32, U32, P, C.c_size_t, P, P], I32),
        "cmh_sweep_color": ([P, I64, I32, P], I32),
        "cmh_run_sweeps": ([P, I64, I64, P], I32),
        "cmh_read_events": ([P, I32, P, I64, P], I32),
        "cmh_write_events": ([P, I32, P, I64], I32),
        "cmh_set_feed": ([P, P, I64, I64, I32], I32),
        "cmh_set_log": ([P, P, I64, I64], I32),
        "cmh_refresh": ([P, I32, P, P], I32),
        "cmh_read_variance": ([P, I32, I64, I64, P], I32),
        "cmh_read_stats": ([P, I32, P], I32),
        "cmh_get_block": ([P, P], I32),
        "cmh_autotune": ([P, I64, I32, P], I32),
        "cmh_tune_running": ([P, I64, I32, P, P], I32),
        "cmh_time_phases": ([P, I64, I64, P, P], I32),
        "cmh_set_stamps": ([P, P, I64, I64], I32),
        "cmh_simulate_noalloc": ([P, P, I64, U32, P, I32, P], I32),
        "cmh_log_posterior": ([P, I32, P, P], I32),
        "cmh_set_logprob": ([P, P, I64, I64], I32),
        "cmh_stamp_rate": ([I32, P], I32),
        "cmh_destroy": ([P], I32),
        "cmh_simulate_bytes": ([P, P, I64, P], I32),
        "cmh_simulate": ([P, P, I64, U32, P, I32, P, C.c_size_t, P], I32),
        "cmh_move_draws": ([U32, U32, U32, U32, U32, I32, I32, P, P], I32),
        "cmh_move_draws_arrivals": ([U32, U32, U32, U32, U32, I32, P, P], I32),
        "cmh_learned_bytes": ([P, I32, P], I32),
        "cmh_set_record": ([P, P, I64, I64, I32], I32),
        "cmh_batch_bytes": ([I32, P, P, P], I32),
        "cmh_batch_init": ([I32, P, P, P, I32, P, P, C.c_size_t, P, P], I32),
        "cmh_set_learned": ([P, P, P, I32, D, P, C.c_size_t, P], I32),
        "cmh_batch_learned_bytes": ([P, I32, I32, P], I32),
        "cmh_checkpoint_bytes": ([P, P], I32),
        "cmh_save": ([P, P, C.c_size_t], I32),
        "cmh_load": ([P, P, C.c_size_t], I32),
        "cmh_batch_set_learned": ([P, I32, P, P, I32, D, P, C.c_size_t, P], I32),
        "cmh_mdn_sizes": ([P, P], I32),
        "cmh_mdn_param_bytes": ([P], I32),
        "cmh_mdn_init": ([P, U32, P], I32),
        "cmh_mdn_set_params": ([P, P, P], I32),
        "cmh_mdn_get_params": ([P, P], I32),
        "cmh_mdn_work_bytes": ([I32, P], I32),
        "cmh_mdn_forward": ([P, P, I32, P, P, C.c_size_t, P], I32),
        "cmh_mdn_infer": ([P, P, I32, P, P], I32),
        "cmh_mdn_gradients": ([P, P, P, I32, P, P, P, C.c_size_t, P], I32),
        "cmh_mdn_train_step": ([P, P, P, I32, I32, C.c_float, P, P, C.c_size_t, P], I32),
        "cmh_mdn_pairs": ([P, U32, I64, I32, P, P, P], I32),
        "cmh_mdn_train": ([P, P, U32, I64, I32, I32, I32, C.c_float, P, P, P, P, C.c_size_t, P],
                          I32),
        "cmh_anchor_count": ([P, P, P], I32),
        "cmh_anchor_features": ([P, P, I32, I64, I32, P, P, P], I32),
        "cmh_mixture_table": ([P, P, I64, I32, P, P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(rc: int):
    if rc != 0:
        raise CmhError(rc, lib().cmh_last_error().decode())


def model_struct(spec: ModelSpec) -> CmhModel:
    m = CmhModel()
    m.nsx, m.nsy, m.ds, m.n_samples = spec.nsx, spec.nsy, spec.ds, spec.N
    m.sigma, m.atten, m.velocity, m.env_decay = spec.sigma, spec.atten, spec.vel, spec.decay
    m.t_s, m.r_c, m.lam = spec.ts, spec.rc, spec.lam
    m.mag_min, m.mag_rate = spec.mmin, spec.mrate
    m.line, m.x_max, m.template_mean = spec.line, spec.xmax, spec.tmpl
    m.arrival_sd = spec.arr_sd
    if len(spec.sta_x) > 8:
        raise ValueError("at most 8 stations on a line")
    for j, v in enumerate(spec.sta_x):
        m.station_x[j] = v
    return m


# sweep-kernel forms beyond the workgroup sizes 64/128/256/512: the
# speculative form with 2, 4 or 8 waves per region (include/chromh.h)
BLOCK_SPEC = 1024
SPEC2, SPEC4, SPEC8 = BLOCK_SPEC + 128, BLOCK_SPEC + 256, BLOCK_SPEC + 512
# the one-wave-per-region form as one persistent launch per sweep
PERSIST = 2048 + 64


def sampler_struct(spec: SamplerSpec, block: int = 0) -> CmhSampler:
    s = CmhSampler()
    s.grid_x, s.grid_y, s.dynamic, s.period = spec.gx, spec.gy, spec.dynamic, spec.period
    s.moves_per_region, s.region_capacity = spec.k, spec.cap
    s.p_birth, s.p_death, s.p_loc, s.p_time, s.p_mag = spec.pb, spec.pd, spec.ploc, spec.pt, spec.pm
    s.step_xy, s.step_t, s.step_m = spec.sxy, spec.st, spec.sm
    s.prior_only, s.block, s.schedule = spec.prior_only, block, spec.schedule
    s.debug = spec.debug
    s.p_arrival, s.p_joint, s.step_arrival = spec.pa, spec.pj, spec.sa
    s.refresh_every = spec.refresh_every
    return s


def _ptr(a) -> C.c_void_p:
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream=None) -> C.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def as_events(x, y, t, m, ids=None, da=None) -> np.ndarray:
    ev = np.zeros(len(x), dtype=EVENT_DTYPE)
    ev["x"], ev["y"], ev["t"], ev["m"] = x, y, t, m
    ev["id"] = np.arange(len(x), dtype=np.uint64) if ids is None else ids
    if da is not None:
        ev["da"] = da
    return ev


def partition_and_color(model: ModelSpec, gx: int, gy: int, offx: float, offy: float,
                        dynamic: int):
    nrx, nry, p, nc = (C.c_int32() for _ in range(4))
    colors = np.zeros((gx + 1) * (gy + 1), dtype=np.int32)
    m = model_struct(model)
    check(lib().cmh_partition_and_color(C.byref(m), gx, gy, offx, offy, dynamic, C.byref(nrx),
                                        C.byref(nry), C.byref(p), C.byref(nc), _ptr(colors)))
    return nrx.value, nry.value, p.value, nc.value, colors


def simulate(model: ModelSpec, truth: np.ndarray, seed: int, dtype: str = "f32",
             device="cuda", stream=None):
    """Trace [stations, N] on the device, sampled from the model given truth."""
    import torch
    truth = np.ascontiguousarray(truth, dtype=EVENT_DTYPE)
    m = model_struct(model)
    nbytes = C.c_size_t()
    check(lib().cmh_simulate_bytes(C.byref(m), _ptr(truth), len(truth), C.byref(nbytes)))
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=device)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    trace = torch.empty((model.nsta, model.N), dtype=tdt, device=device)
    check(lib().cmh_simulate(C.byref(m), _ptr(truth), len(truth), seed, _ptr(trace),
                             CMH_F32 if dtype == "f32" else CMH_F64, _ptr(ws), ws.numel(),
                             _stream(stream)))
    del ws
    return trace


def move_draws(seed: int, chain: int, sweep: int, region: int, j0: int, count: int,
               device="cuda", width: int = 8) -> np.ndarray:
    import torch
    out = torch.empty((count, width), dtype=torch.float64, device=device)
    check(lib().cmh_move_draws(seed, chain, sweep, region, j0, count, width, _ptr(out),
                               _stream()))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def move_draws_arrivals(seed: int, chain: int, sweep: int, region: int, j0: int, count: int,
                        device="cuda") -> np.ndarray:
    """Latent-arrival draw records [count, 16] computed on the device."""
    import torch
    out = torch.empty((count, 16), dtype=torch.float64, device=device)
    check(lib().cmh_move_draws_arrivals(seed, chain, sweep, region, j0, count, _ptr(out),
                                        _stream()))
    torch.cuda.synchronize()
    return out.cpu().numpy()


class ChromaticSampler:
    """Chains of the chromatic MH sampler sharing one device trace."""

    def __init__(self, model: ModelSpec, sampler: SamplerSpec, trace, chains: int = 1,
                 seed: int = 0, block: int = 0, stream=None):
        import torch
        if not (trace.is_cuda and trace.dim() == 2 and trace.is_contiguous()):
            raise ValueError("trace must be a contiguous 2-D device tensor [stations, samples]")
        if trace.dtype not in (torch.float32, torch.float64):
            raise ValueError("trace must be float32 or float64")
        self.model, self.sampler, self.chains = model, sampler, chains
        self.trace = trace
        self._m = model_struct(model)
        self._s = sampler_struct(sampler, block)
        nbytes = C.c_size_t()
        check(lib().cmh_state_bytes(C.byref(self._m), C.byref(self._s), chains, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=trace.device)
        h = C.c_void_p()
        check(lib().cmh_init_state(C.byref(self._m), C.byref(self._s), _ptr(trace),
                                   CMH_F64 if trace.dtype == torch.float64 else CMH_F32, chains,
                                   seed, _ptr(self.workspace), self.workspace.numel(),
                                   _stream(stream), C.byref(h)))
        self._h = h
        _, _, self.period, self.ncolors, _ = partition_and_color(
            model, sampler.gx, sampler.gy, 0.0, 0.0, sampler.dynamic) \
            if sampler.period == 0 else (0, 0, sampler.period,
                                         sampler.period ** (1 if model.line else 2), None)
        if sampler.schedule == 1:  # naive: every region in one phase
            self.ncolors = 1
        self._feed = None
        self._log = None

    # -- sweeps --------------------------------------------------------
    def sweep_color(self, sweep: int, color: int, stream=None):
        check(lib().cmh_sweep_color(self._h, sweep, color, _stream(stream)))

    def run_sweeps(self, first: int, n: int, stream=None):
        check(lib().cmh_run_sweeps(self._h, first, n, _stream(stream)))

    def autotune(self, first: int, n_trial: int = 3, stream=None) -> int:
        check(lib().cmh_autotune(self._h, first, n_trial, _stream(stream)))
        return self.block

    def tune_running(self, first: int, n_trial: int = 3, stream=None) -> int:
        """Tunes the kernel form on sweeps of the run itself (first, first +
        1, ...; every form gives the same chain); returns the next sweep."""
        nxt = C.c_int64()
        check(lib().cmh_tune_running(self._h, first, n_trial, _stream(stream), C.byref(nxt)))
        return nxt.value

    @property
    def block(self) -> int:
        b = C.c_int32()
        check(lib().cmh_get_block(self._h, C.byref(b)))
        return b.value

    # -- replay --------------------------------------------------------
    def _check_buffer(self, t, last: int, name: str):
        import torch
        want = (self.sampler.nreg, self.sampler.k, last)
        if (t.dim() != 4 or tuple(t.shape[1:]) != want or t.dtype != torch.float64
                or not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 device tensor "
                             f"[n_sweeps, {want[0]}, {want[1]}, {want[2]}]")

    def set_feed(self, feed, first: int):
        """feed: float64 device tensor [n_sweeps, regions, k, 8] ([.., 16]
        with learned births or latent arrivals), or None."""
        if feed is not None:
            self._check_buffer(feed, feed.shape[-1] if feed.dim() == 4 else 8, "feed")
            if feed.shape[-1] not in (8, 16):
                raise ValueError("feed records are 8 or 16 wide")
        self._feed = feed
        if feed is None:
            check(lib().cmh_set_feed(self._h, None, 0, 0, 8))
        else:
            check(lib().cmh_set_feed(self._h, _ptr(feed), first, feed.shape[0], feed.shape[-1]))

    def set_learned(self, table, weights, n_tau: int, p_learned: float = 0.5, stream=None):
        """Learned births from a float64 device table [n_stations * n_tau, 8, 8]
        and anchor weights [n_stations * n_tau] (kept alive here); None: off."""
        import torch
        if table is None:
            check(lib().cmh_set_learned(self._h, None, None, 0, 0.0, None, 0, _stream(stream)))
            self._learned = None
            return
        na = self.model.nsta * n_tau
        if (tuple(table.shape) != (na, 8, 8) or table.dtype != torch.float64 or not table.is_cuda
                or not table.is_contiguous()):
            raise ValueError(f"table must be a contiguous float64 device tensor [{na}, 8, 8]")
        if (tuple(weights.shape) != (na,) or weights.dtype != torch.float64 or not weights.is_cuda
                or not weights.is_contiguous()):
            raise ValueError(f"weights must be a contiguous float64 device tensor [{na}]")
        nb = C.c_size_t()
        check(lib().cmh_learned_bytes(self._h, n_tau, C.byref(nb)))
        work = torch.empty(nb.value, dtype=torch.uint8, device=self.trace.device)
        check(lib().cmh_set_learned(self._h, _ptr(table), _ptr(weights), n_tau, p_learned,
                                    _ptr(work), work.numel(), _stream(stream)))
        self._learned = (table, weights, work)

    def set_record(self, first: int, n: int, max_events: int, stream=None):
        """Record every chain's state after sweeps first .. first + n - 1 into
        a device buffer [n, chains, 1 + 4 max_events] (returned); n = 0 stops."""
        import torch
        if n == 0:
            check(lib().cmh_set_record(self._h, None, 0, 0, 0))
            self._rec = None
            return None
        rec = torch.zeros((n, self.chains, 1 + 4 * max_events), dtype=torch.float64,
                          device=self.trace.device)
        check(lib().cmh_set_record(self._h, _ptr(rec), first, n, max_events))
        self._rec = rec
        return rec

    @staticmethod
    def recorded_states(rec, chain: int) -> list:
        """Event arrays (fields x, y, t, m) of one chain from a record buffer."""
        r = rec[:, chain].cpu().numpy() if hasattr(rec, "cpu") else rec[:, chain]
        maxe = (r.shape[1] - 1) // 4
        out = []
        for row in r:
            n = min(int(row[0]), maxe)
            ev = np.zeros(n, dtype=EVENT_DTYPE)
            v = row[1:1 + 4 * n].reshape(n, 4)
            ev["x"], ev["y"], ev["t"], ev["m"] = v[:, 0], v[:, 1], v[:, 2], v[:, 3]
            out.append(ev)
        return out

    def set_log(self, log, first: int):
        """log: float64 device tensor [n_sweeps, regions, k, 4] (or None)."""
        if log is not None:
            self._check_buffer(log, 4, "log")
        self._log = log
        if log is None:
            check(lib().cmh_set_log(self._h, None, 0, 0))
        else:
            check(lib().cmh_set_log(self._h, _ptr(log), first, log.shape[0]))

    # -- state ---------------------------------------------------------
    def read_events(self, chain: int = 0) -> np.ndarray:
        n = C.c_int64()
        rc = lib().cmh_read_events(self._h, chain, None, 0, C.byref(n))
        if rc not in (0, -1):
            check(rc)
        out = np.zeros(n.value, dtype=EVENT_DTYPE)
        check(lib().cmh_read_events(self._h, chain, _ptr(out), len(out), C.byref(n)))
        return out

    def save(self) -> np.ndarray:
        """A checkpoint of every chain (host bytes); resume with load() on a
        sampler made the same way, then continue at the next sweep index."""
        nb = C.c_size_t()
        check(lib().cmh_checkpoint_bytes(self._h, C.byref(nb)))
        buf = np.empty(nb.value, dtype=np.uint8)
        check(lib().cmh_save(self._h, _ptr(buf), buf.nbytes))
        return buf

    def load(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        check(lib().cmh_load(self._h, _ptr(buf), buf.nbytes))

    def write_events(self, chain: int, ev: np.ndarray):
        ev = np.ascontiguousarray(ev, dtype=EVENT_DTYPE)
        check(lib().cmh_write_events(self._h, chain, _ptr(ev), len(ev)))

    def refresh(self, write_variance: bool = True, loglik: bool = True, stream=None):
        out = np.zeros(self.chains) if loglik else None
        check(lib().cmh_refresh(self._h, 1 if write_variance else 0,
                                None if out is None else _ptr(out), _stream(stream)))
        return out

    def read_variance(self, chain: int = 0, station0: int = 0, nsta: int | None = None):
        nsta = self.model.nsta - station0 if nsta is None else nsta
        out = np.zeros((nsta, self.model.N))
        check(lib().cmh_read_variance(self._h, chain, station0, nsta, _ptr(out)))
        return out

    def read_stats(self, chain: int = 0) -> np.ndarray:
        """[7, 3] attempted / evaluated / accepted moves per move type (rows 5
        and 6: the arrival-time and joint moves of latent arrivals)."""
        c = self.read_counters(chain)
        return np.concatenate([c[:15], c[17:23]]).reshape(7, 3)

    def read_counters(self, chain: int = 0) -> np.ndarray:
        """All 23 counters: the move table of types 0..4, footprint samples
        evaluated and rewritten, then the table of the latent-arrival moves
        (types 5 and 6)."""
        out = np.zeros(N_STATS, dtype=np.uint64)
        check(lib().cmh_read_stats(self._h, chain, _ptr(out)))
        return out

    def time_phases(self, first: int, n: int, stream=None) -> np.ndarray:
        """Milliseconds per colour phase (summed over n sweeps), then re-layout."""
        out = np.zeros(self.ncolors + 1, dtype=np.float32)
        check(lib().cmh_time_phases(self._h, first, n, _stream(stream), _ptr(out)))
        return out

    def log_posterior(self, write_variance: bool = False, stream=None) -> np.ndarray:
        """[chains][3]: log-likelihood, log prior and their sum for every
        chain (instance, in a batch), from an exact recomputation."""
        out = np.zeros((self.chains, 3))
        check(lib().cmh_log_posterior(self._h, 1 if write_variance else 0, _ptr(out),
                                      _stream(stream)))
        return out

    def set_logprob(self, first: int, n: int):
        """Device records [n][chains][2] (log-likelihood, log prior) taken by
        the scheduled refresh after sweeps first .. first + n - 1 (NaN where
        no refresh ran); returns the buffer (n <= 0 switches recording off)."""
        import torch
        if n <= 0:
            check(lib().cmh_set_logprob(self._h, None, 0, 0))
            self._lp = None
            return None
        buf = torch.full((n, self.chains, 2), float("nan"), dtype=torch.float64,
                         device=self.trace.device)
        torch.cuda.synchronize(self.trace.device)
        check(lib().cmh_set_logprob(self._h, C.c_void_p(buf.data_ptr()), first, n))
        self._lp = buf
        return buf

    def set_stamps(self, first: int, n: int):
        """Sweep-kernel time stamps for sweeps first .. first + n - 1 into a
        device buffer [n][colours][2] (start minimum, end maximum of the
        steady clock); returns it (None, 0, 0 switches stamping off)."""
        import torch
        if n <= 0:
            check(lib().cmh_set_stamps(self._h, None, 0, 0))
            self._stamps = None
            return None
        buf = torch.zeros((n, self.ncolors, 2), dtype=torch.int64, device=self.trace.device)
        buf[..., 0] = -1  # all ones: the minimum's identity
        torch.cuda.synchronize(self.trace.device)
        check(lib().cmh_set_stamps(self._h, C.c_void_p(buf.data_ptr()), first, n))
        self._stamps = buf
        return buf

    @staticmethod
    def stamp_seconds(buf) -> np.ndarray:
        """Kernel spans [n][colours] in seconds from a stamp buffer."""
        hz = C.c_int64()
        check(lib().cmh_stamp_rate(0, C.byref(hz)))
        a = buf.cpu().numpy().view(np.uint64)
        return (a[..., 1].astype(np.float64) - a[..., 0].astype(np.float64)) / hz.value

    def close(self):
        if getattr(self, "_h", None):
            lib().cmh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- learned proposal

class MDN:
    """The mixture-density network of the learned birth proposal, with its
    parameters (FP32 master + Adam moments + BF16 copies) in device memory."""

    def __init__(self, device="cuda", seed: int | None = 0):
        import torch
        n, nh = C.c_int64(), C.c_int64()
        check(lib().cmh_mdn_sizes(C.byref(n), C.byref(nh)))
        self.n_params = n.value
        nb = C.c_size_t()
        check(lib().cmh_mdn_param_bytes(C.byref(nb)))
        self.device = device
        self.params = torch.zeros(nb.value, dtype=torch.uint8, device=device)
        self._work = None
        self._rows = 0
        if seed is not None:
            check(lib().cmh_mdn_init(_ptr(self.params), seed, _stream()))

    def work(self, rows: int):
        import torch
        if self._work is None or rows > self._rows:
            nb = C.c_size_t()
            check(lib().cmh_mdn_work_bytes(rows, C.byref(nb)))
            self._work = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            self._rows = rows
        return self._work

    def set_params(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.n_params
        check(lib().cmh_mdn_set_params(_ptr(self.params), _ptr(flat), _stream()))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        check(lib().cmh_mdn_get_params(_ptr(self.params), _ptr(out)))
        return out

    def forward(self, X):
        """X: bfloat16 device tensor [rows, 576] -> float32 [rows, 64]."""
        import torch
        rows = X.shape[0]
        out = torch.empty((rows, 64), dtype=torch.float32, device=self.device)
        w = self.work(rows)
        check(lib().cmh_mdn_forward(_ptr(self.params), _ptr(X), rows, _ptr(out), _ptr(w),
                                    w.numel(), _stream()))
        return out

    def infer(self, X):
        """The head outputs of forward() from the fused inference kernel."""
        import torch
        rows = X.shape[0]
        out = torch.empty((rows, 64), dtype=torch.float32, device=self.device)
        check(lib().cmh_mdn_infer(_ptr(self.params), _ptr(X), rows, _ptr(out), _stream()))
        return out

    def gradients(self, X, Z):
        import torch
        rows = X.shape[0]
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        loss = torch.empty(rows, dtype=torch.float32, device=self.device)
        w = self.work(rows)
        check(lib().cmh_mdn_gradients(_ptr(self.params), _ptr(X), _ptr(Z), rows, _ptr(grad),
                                      _ptr(loss), _ptr(w), w.numel(), _stream()))
        return loss, grad

    def train_step(self, X, Z, step: int, lr: float, loss=None):
        rows = X.shape[0]
        w = self.work(rows)
        check(lib().cmh_mdn_train_step(_ptr(self.params), _ptr(X), _ptr(Z), rows, step, lr,
                                       None if loss is None else _ptr(loss), _ptr(w), w.numel(),
                                       _stream()))

    def train(self, model: ModelSpec, seed: int, first_pair: int, steps: int, rows: int,
              step0: int, lr: float, pairs, loss=None):
        """steps Adam steps on fresh simulator pairs in one library call (see
        cmh_mdn_train); pairs = (X bf16 [rows, 576], Z f32 [rows, 3]) buffers."""
        import torch
        X, Z = pairs
        if X.shape != (rows, 576) or Z.shape != (rows, 3) or X.dtype != torch.bfloat16 \
                or Z.dtype != torch.float32 or not (X.is_contiguous() and Z.is_contiguous()):
            raise ValueError("pairs must be contiguous bf16 [rows, 576] and f32 [rows, 3]")
        if loss is not None and (loss.numel() < rows or loss.dtype != torch.float32):
            raise ValueError("loss must be f32 with at least rows elements")
        w = self.work(rows)
        m = model_struct(model)
        check(lib().cmh_mdn_train(_ptr(self.params), C.byref(m), seed, first_pair, steps, rows,
                                  step0, lr, _ptr(X), _ptr(Z), None if loss is None else _ptr(loss),
                                  _ptr(w), w.numel(), _stream()))


def mdn_pairs(model: ModelSpec, seed: int, first: int, count: int, device="cuda", out=None):
    """Training pairs from the forward simulator: (bf16 [count, 576], f32 [count, 3]),
    written into out = (X, Z) when given."""
    import torch
    if out is None:
        X = torch.empty((count, 576), dtype=torch.bfloat16, device=device)
        Z = torch.empty((count, 3), dtype=torch.float32, device=device)
    else:
        X, Z = out
        if X.shape != (count, 576) or Z.shape != (count, 3) or X.dtype != torch.bfloat16 \
                or Z.dtype != torch.float32 or not (X.is_contiguous() and Z.is_contiguous()):
            raise ValueError("out must be contiguous bf16 [count, 576] and f32 [count, 3]")
    m = model_struct(model)
    check(lib().cmh_mdn_pairs(C.byref(m), seed, first, count, _ptr(X), _ptr(Z), _stream()))
    return X, Z


def anchor_count(model: ModelSpec):
    na, nt = C.c_int32(), C.c_int32()
    m = model_struct(model)
    check(lib().cmh_anchor_count(C.byref(m), C.byref(na), C.byref(nt)))
    return na.value, nt.value


def anchor_features(model: ModelSpec, trace, first: int = 0, count: int | None = None):
    """(bf16 [count, 576], f64 [count]) features and weights of anchors
    first .. first + count - 1 of a device trace (all anchors by default)."""
    import torch
    na, _ = anchor_count(model)
    count = na - first if count is None else count
    X = torch.empty((count, 576), dtype=torch.bfloat16, device=trace.device)
    wts = torch.empty(count, dtype=torch.float64, device=trace.device)
    m = model_struct(model)
    check(lib().cmh_anchor_features(C.byref(m), _ptr(trace),
                                    CMH_F64 if trace.dtype == torch.float64 else CMH_F32,
                                    first, count, _ptr(X), _ptr(wts), _stream()))
    return X, wts


def mixture_table(model: ModelSpec, head, first: int = 0):
    """Binary64 mixture table [rows, 8, 8] of anchors first .. from head
    outputs [rows, 64] (device float32)."""
    import torch
    rows = head.shape[0]
    T = torch.empty((rows, 8, 8), dtype=torch.float64, device=head.device)
    m = model_struct(model)
    check(lib().cmh_mixture_table(C.byref(m), _ptr(head), first, rows, _ptr(T), _stream()))
    return T


class Batch(ChromaticSampler):
    """Independent instances of uneven size sampled together: each colour
    phase is one launch over that colour's regions of every instance.
    Readers take the instance index where a chain index is expected."""

    def __init__(self, models, samplers, traces, seeds, block: int = 0, stream=None):
        import torch
        n = len(models)
        if not (len(samplers) == len(traces) == len(seeds) == n):
            raise ValueError("models, samplers, traces and seeds must have equal lengths")
        dt = traces[0].dtype
        for tr, m in zip(traces, models):
            if not (tr.is_cuda and tr.dim() == 2 and tr.is_contiguous() and tr.dtype == dt
                    and tuple(tr.shape) == (m.nsta, m.N)):
                raise ValueError("traces must be contiguous device tensors [stations, samples] "
                                 "of one dtype")
        self.models, self.samplers = list(models), list(samplers)
        self.model, self.sampler = models[0], samplers[0]
        self.chains = n
        self.traces = list(traces)
        self.trace = traces[0]
        ms = (CmhModel * n)(*[model_struct(m) for m in models])
        ss = (CmhSampler * n)(*[sampler_struct(sp, block) for sp in samplers])
        self._ms, self._ss = ms, ss
        nbytes = C.c_size_t()
        check(lib().cmh_batch_bytes(n, ms, ss, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=traces[0].device)
        ptrs = (C.c_void_p * n)(*[tr.data_ptr() for tr in traces])
        sd = (C.c_uint32 * n)(*seeds)
        h = C.c_void_p()
        check(lib().cmh_batch_init(n, ms, ss, ptrs, CMH_F64 if dt == torch.float64 else CMH_F32,
                                   sd, _ptr(self.workspace), self.workspace.numel(),
                                   _stream(stream), C.byref(h)))
        self._h = h
        self.ncolors = max(
            partition_and_color(m, sp.gx, sp.gy, 0.0, 0.0, sp.dynamic)[3] if sp.period == 0
            else sp.period ** (1 if m.line else 2) for m, sp in zip(models, samplers))
        if samplers[0].schedule == 1:
            self.ncolors = 1
        self._feed = None
        self._log = None
        self._learned_q = {}

    def set_learned_instance(self, q: int, table, weights, n_tau: int, p_learned: float = 0.5,
                             stream=None):
        """Learned births for instance q from its own float64 device table
        [n_stations_q * n_tau, 8, 8] and weights [n_stations_q * n_tau] (kept
        alive here); None: plain births again."""
        import torch
        if table is None:
            check(lib().cmh_batch_set_learned(self._h, q, None, None, 0, 0.0, None, 0,
                                              _stream(stream)))
            self._learned_q.pop(q, None)
            return
        na = self.models[q].nsta * n_tau
        for t, shape in ((table, (na, 8, 8)), (weights, (na,))):
            if (tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_cuda
                    or not t.is_contiguous()):
                raise ValueError(f"table and weights must be contiguous float64 device tensors "
                                 f"[{na}, 8, 8] and [{na}]")
        nb = C.c_size_t()
        check(lib().cmh_batch_learned_bytes(self._h, q, n_tau, C.byref(nb)))
        work = torch.empty(nb.value, dtype=torch.uint8, device=self.trace.device)
        check(lib().cmh_batch_set_learned(self._h, q, _ptr(table), _ptr(weights), n_tau,
                                          p_learned, _ptr(work), work.numel(), _stream(stream)))
        self._learned_q[q] = (table, weights, work)
