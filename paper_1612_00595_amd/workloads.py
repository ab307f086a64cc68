"""Workload definitions and seeded input generators.

This module is the only one that both the GPU path and the CPU oracle draw
their inputs from.  It holds workload constants and numpy random generators
and none of the method's arithmetic: no likelihood, no proposal rule, no
acceptance ratio.

Workloads follow the paper's toy seismic model (Section 3) in the 2-D,
attenuating form Section 4.1 names as the natural case for spatial
partitioning; the paper evaluates only on synthetic worlds sampled from its
own model (Section 5), so every input here is synthetic by construction.

Physical constants shared by the grid workloads: stations on a cell-centred
grid of spacing 0.2, amplitude m exp(-d / 0.2), onset-delayed exponential
envelope of decay 20 samples, arrival t + d / 0.05, noise sigma 0.1,
detection cutoff 0.19, signal duration 128 samples, magnitude 2 + Exp(1).
Larger workloads keep the station spacing and grow the domain, so that an
event still reaches at most four stations.  The line workload is the paper's
own 1-D world (Section 3 as printed, partitioned in time as in Section 4.1).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

BIRTH, DEATH, LOC, TIME, MAG = range(5)


@dataclass(frozen=True)
class ModelSpec:
    nsx: int = 5
    nsy: int = 5
    ds: float = 0.2
    N: int = 1000
    sigma: float = 0.1
    atten: float = 0.2
    vel: float = 0.05
    decay: float = 20.0
    ts: int = 128
    rc: float = 0.19
    lam: float = 20.0
    mmin: float = 2.0
    mrate: float = 1.0
    line: int = 0              # 1: stations on a line, events (x, t), time partition
    tmpl: int = 0              # 1: mean-template likelihood (waveforms add to the mean)
    xmax: float = 0.0          # line: locations on [0, xmax)
    sta_x: tuple = ()          # line: station positions (at most 8)
    arr_sd: float = 0.0        # line: arrival-time jitter sd (latent arrivals when > 0)

    @property
    def Lx(self) -> float:
        return self.xmax if self.line else self.nsx * self.ds

    @property
    def Ly(self) -> float:
        return 1.0 if self.line else self.nsy * self.ds

    @property
    def nsta(self) -> int:
        return self.nsx * self.nsy

    def asdict(self) -> dict:
        return dataclasses.asdict(self)


@dataclass(frozen=True)
class SamplerSpec:
    gx: int = 4
    gy: int = 4
    dynamic: int = 0
    period: int = 0
    k: int = 16
    cap: int = 64
    pb: float = 0.2
    pd: float = 0.2
    ploc: float = 0.2
    pt: float = 0.2
    pm: float = 0.2
    sxy: float = 0.02
    st: float = 1.0
    sm: float = 0.2
    prior_only: int = 0
    schedule: int = 0
    lattice: int = 0
    kx: int = 0
    ky: int = 0
    kt: int = 0
    km: int = 0
    hm: float = 0.0
    pa: float = 0.0            # latent arrivals: arrival-time move probability
    pj: float = 0.0            # latent arrivals: joint two-event move probability
    sa: float = 0.0            # latent arrivals: arrival step
    debug: int = 0             # library only: bit 0 owner check, bit 1 unchecked period
    refresh_every: int = 0     # library only: exact variance refresh every this many sweeps

    @property
    def nreg(self) -> int:
        return (self.gx + 1) * (self.gy + 1)

    def asdict(self) -> dict:
        return dataclasses.asdict(self)


@dataclass(frozen=True)
class Workload:
    name: str
    model: ModelSpec
    sampler: SamplerSpec
    trace_dtype: str          # "f64" or "f32"
    chains: int = 1
    sweeps: int = 100
    seed: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


# 5x5 stations on [0,1]^2, 1000-sample fp64 traces, Poisson mean 20 events,
# 4x4 static regions (2x2 colour pattern), 2000 sweeps, seed 0.
SMALL = Workload(
    name="s5x5-n1000-static4x4-f64",
    model=ModelSpec(nsx=5, nsy=5, N=1000, lam=20.0),
    sampler=SamplerSpec(gx=4, gy=4, dynamic=0),
    trace_dtype="f64", chains=1, sweeps=2000, seed=0)

# 64x64 stations, 144000-sample fp32 traces (2.36 GB), Poisson mean 20000,
# 64x64 regions whose offset is redrawn every sweep, 500 sweeps, one chain.
LARGE = Workload(
    name="s64x64-n144000-dyn64x64-f32",
    model=ModelSpec(nsx=64, nsy=64, N=144000, lam=20000.0),
    sampler=SamplerSpec(gx=64, gy=64, dynamic=1),
    trace_dtype="f32", chains=1, sweeps=500, seed=1)

# 32 independent chains of one 32x32-station instance, 36000-sample fp32
# traces, Poisson mean 5000, dynamic 32x32 regions, all chains in one launch.
CHAINS32 = Workload(
    name="s32x32-n36000-dyn32x32-f32-c32",
    model=ModelSpec(nsx=32, nsy=32, N=36000, lam=5000.0),
    sampler=SamplerSpec(gx=32, gy=32, dynamic=1),
    trace_dtype="f32", chains=32, sweeps=500, seed=2)

# The paper's own world (Section 3 as printed, Section 5's setting): four
# stations at x = 0, 33, 66, 100 on a line of length x_max = 100, wave speed
# 2, T = 240 unit samples, Poisson mean 8 events, each an iid Gaussian signal
# of variance 4 over 10 samples on background variance 1 at every station;
# four regions of onset time (l = 60 >= tau_max + t_s = 50 + 10, so two
# colours, as in Section 4.1), k = 500 moves per region per phase (Section 5).
PAPER1D_MODEL = ModelSpec(nsx=4, nsy=1, ds=1.0, N=240, sigma=1.0, atten=1.0, vel=2.0,
                          decay=1.0, ts=10, rc=0.5, lam=8.0, mmin=2.0, mrate=1.0, line=1,
                          xmax=100.0, sta_x=(0.0, 33.0, 66.0, 100.0))
PAPER1D_SAMPLER = SamplerSpec(gx=4, gy=0, dynamic=0, k=500, cap=64, pb=0.2, pd=0.2, ploc=0.3,
                              pt=0.3, pm=0.0, sxy=2.0, st=1.0, sm=0.0)
PAPER1D = Workload(name="line4-x100-n240-t4-k500", model=PAPER1D_MODEL, sampler=PAPER1D_SAMPLER,
                   trace_dtype="f64", chains=1, sweeps=200, seed=5)

# The same world with Section 3's latent arrival times: every arrival is the
# mean travel time plus a Gaussian offset of sd 1 sample (truncated at 4 sd),
# and the sampler adds the arrival-time move and the joint two-event move.
# The jitter bound widens each region's reach by 4 samples on both sides, so
# the four regions need three colours.
PAPER1D_LATENT_MODEL = dataclasses.replace(PAPER1D_MODEL, arr_sd=1.0)
PAPER1D_LATENT_SAMPLER = dataclasses.replace(PAPER1D_SAMPLER, pb=0.15, pd=0.15, ploc=0.25,
                                             pt=0.25, pa=0.1, pj=0.1, sa=1.0)
PAPER1D_LATENT = Workload(name="line4-x100-n240-t4-k500-latent", model=PAPER1D_LATENT_MODEL,
                          sampler=PAPER1D_LATENT_SAMPLER, trace_dtype="f64", chains=1,
                          sweeps=200, seed=6)

WORKLOADS = {w.name: w for w in (SMALL, LARGE, CHAINS32, PAPER1D, PAPER1D_LATENT)}


def truncated_normals(rng, shape, bound: float = 4.0) -> np.ndarray:
    """Standard normals redrawn until |z| <= bound."""
    z = rng.standard_normal(shape)
    bad = np.abs(z) > bound
    while bad.any():
        z[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(z) > bound
    return z


def uneven_batch(count: int = 256, seed: int = 1000) -> list:
    """Instances of uneven size served together (seeds seed .. seed + count -
    1): station grid side n uniform on 8..32 (n x n stations, n x n dynamic
    regions of one spacing), samples 64 * round(U[4000, 36000] / 64), fp32
    traces.  The Poisson mean is the instance's station count times a
    log-uniform density of 100/64 .. 5000/1024 events per station, so that it
    spans 100 (8 x 8) to 5000 (32 x 32) while every region keeps about the
    same number of events."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for q in range(count):
        n = int(rng.integers(8, 33))
        N = 64 * int(round(rng.uniform(4000, 36000) / 64))
        rho = (100 / 64) * ((5000 / 1024) / (100 / 64)) ** rng.uniform()
        lam = float(round(rho * n * n))
        out.append(Workload(name=f"u{q}-s{n}x{n}-n{N}", model=ModelSpec(nsx=n, nsy=n, N=N, lam=lam),
                            sampler=SamplerSpec(gx=n, gy=n, dynamic=1), trace_dtype="f32",
                            seed=seed + q))
    return out


def scaled(w: Workload, *, side: int, N: int, lam: float, name: str | None = None,
           **sampler_kw) -> Workload:
    """Same physics on a smaller station grid (used by tests)."""
    model = dataclasses.replace(w.model, nsx=side, nsy=side, N=N, lam=lam)
    sampler = dataclasses.replace(w.sampler, gx=side, gy=side, **sampler_kw) \
        if w.sampler.dynamic else dataclasses.replace(w.sampler, **sampler_kw)
    return dataclasses.replace(w, name=name or f"{w.name}-scaled{side}", model=model,
                               sampler=sampler)


# ------------------------------------------------------------------ inputs

def truth_events(model: ModelSpec, seed: int, n: int | None = None):
    """Events from the prior: Poisson(lam) count, uniform location and onset,
    magnitude mmin + Exp(mrate).  Returns a dict of float64 arrays and ids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n is None:
        n = int(rng.poisson(model.lam))
    if model.line:  # locations on [0, xmax), y = 0, the fixed amplitude
        x = np.minimum(rng.random(n) * model.xmax, np.nextafter(model.xmax, 0.0))
        t = np.minimum(rng.random(n) * model.N, np.nextafter(float(model.N), 0.0))
        da = np.zeros((n, 8))
        if model.arr_sd > 0:  # latent arrivals: offsets from their truncated prior
            da[:, :model.nsx] = model.arr_sd * truncated_normals(rng, (n, model.nsx))
        return dict(x=x, y=np.zeros(n), t=t, m=np.full(n, model.mmin),
                    id=np.arange(n, dtype=np.uint64), da=da)
    x = np.minimum(rng.random(n) * model.Lx, np.nextafter(model.Lx, 0.0))
    y = np.minimum(rng.random(n) * model.Ly, np.nextafter(model.Ly, 0.0))
    t = np.minimum(rng.random(n) * model.N, np.nextafter(float(model.N), 0.0))
    m = model.mmin + rng.standard_exponential(n) / model.mrate
    return dict(x=x, y=y, t=t, m=m, id=np.arange(n, dtype=np.uint64))


def feed_draws(sampler: SamplerSpec, nsweeps: int, seed: int, learned: bool = False,
               latent: bool = False) -> np.ndarray:
    """Per-move random draws for replay runs, shape [nsweeps, regions, k, 8]:
    [0..3] uniforms on [0,1), [4] Exp(1), [5],[6] standard normals, [7] log of
    a uniform on (0,1].  With learned births the records are 16 wide: [8..10]
    uniforms on [0,1), [11..13] standard normals truncated to [-4, 4],
    [14], [15] zero.  With latent arrivals they are 16 wide too: [8..15]
    standard normals truncated to [-4, 4].  Both the GPU path and the oracle
    consume the same array, so their proposals coincide bit for bit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nsweeps, sampler.nreg, sampler.k)
    out = np.zeros(shape + ((16,) if learned or latent else (8,)), dtype=np.float64)
    out[..., 0:4] = rng.random(shape + (4,))
    out[..., 4] = rng.standard_exponential(shape)
    out[..., 5:7] = rng.standard_normal(shape + (2,))
    out[..., 7] = np.log1p(-rng.random(shape))
    if learned:
        out[..., 8:11] = rng.random(shape + (3,))
        z = rng.standard_normal(shape + (3,))
        bad = np.abs(z) > 4.0
        while bad.any():
            z[bad] = rng.standard_normal(int(bad.sum()))
            bad = np.abs(z) > 4.0
        out[..., 11:14] = z
    if latent:
        out[..., 8:16] = truncated_normals(rng, shape + (8,))
    return out


def random_mixture_table(model: ModelSpec, seed: int, sd_scale: float = 1.0, near=None):
    """An arbitrary learned-proposal table for every anchor (station s,
    window i; anchor index s * n_tau + i): ([anchors][8][8] with rows (mean
    x, y, t, sd x, y, t, log weight, cumulative weight), weights
    [anchors], n_tau).  Means lie near the anchor's station and window; sds
    are log-uniform over the network's clamp ranges times sd_scale.  With
    `near` (events with fields x, y, t), component 0 of every anchor whose
    station lies within 1.5 spacings of an event and whose window starts at
    most 64 samples before it is moved onto that event with small sds, and
    the anchor's weight raised, so that such proposals often land."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_tau = (model.N - 67) // 32 + 1
    na = model.nsta * n_tau
    st = np.repeat(np.arange(model.nsta), n_tau)
    tau = 32.0 * np.tile(np.arange(n_tau), model.nsta)
    sx = ((st % model.nsx) + 0.5) * model.ds
    sy = ((st // model.nsx) + 0.5) * model.ds
    T = np.zeros((na, 8, 8))
    T[..., 0] = sx[:, None] + model.ds * rng.uniform(-1.5, 1.5, (na, 8))
    T[..., 1] = sy[:, None] + model.ds * rng.uniform(-1.5, 1.5, (na, 8))
    T[..., 2] = tau[:, None] + rng.uniform(-32.0, 96.0, (na, 8))
    T[..., 3] = sd_scale * np.exp(rng.uniform(np.log(0.005), np.log(0.3), (na, 8)))
    T[..., 4] = sd_scale * np.exp(rng.uniform(np.log(0.005), np.log(0.3), (na, 8)))
    T[..., 5] = sd_scale * np.exp(rng.uniform(np.log(0.5), np.log(32.0), (na, 8)))
    pi = rng.dirichlet(np.ones(8), na)
    T[..., 6] = np.log(pi)
    T[..., 7] = np.cumsum(pi, axis=1)
    w = 1e-3 + rng.exponential(1.0, na)
    if near is not None:
        for e in near:
            ix, iy = int(e["x"] // model.ds), int(e["y"] // model.ds)
            for jy in range(max(iy - 1, 0), min(iy + 2, model.nsy)):
                for jx in range(max(ix - 1, 0), min(ix + 2, model.nsx)):
                    if np.hypot((jx + 0.5) * model.ds - e["x"],
                                (jy + 0.5) * model.ds - e["y"]) > 1.5 * model.ds:
                        continue
                    for i in range(max(int(np.ceil((e["t"] - 64.0) / 32.0)), 0),
                                   min(int(e["t"] // 32.0), n_tau - 1) + 1):
                        a = (jy * model.nsx + jx) * n_tau + i
                        T[a, 0, 0:3] = [e["x"], e["y"], e["t"]] + rng.normal(0, [0.01, 0.01, 1.0])
                        T[a, 0, 3:6] = [0.02, 0.02, 2.0]
                        w[a] += 20.0
    return T, w, n_tau


def random_state(model: ModelSpec, seed: int, n: int):
    """An arbitrary event set (for likelihood-difference tests)."""
    return truth_events(model, seed, n=n)
