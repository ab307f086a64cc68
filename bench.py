#!/usr/bin/env python3
"""Benchmark of the chromatic MH region sweep on one MI355X.

A step is one full sweep (the partition re-layout plus every colour phase)
of the sampler over the synthetic instance of the 64x64-station,
144000-sample fp32 workload with Poisson mean 20000 events and shifted 64x64
regions.  The instance lives in HBM before timing starts (the trace is
generated on the device by the library's forward simulator).

Prints one JSON line: proposals/s (attempted MH moves per second) with a
roofline block for the sweep kernel (algorithmic bytes per launch over its
average HIP-event-timed duration) and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MH proposals/s + event-location ESS/s per GPU, learned vs plain at equal F1"
TIME_THRESH_1D = 12.0   # Section 5's matching threshold in time, the paper's own units


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--burn-in", type=int, default=-1,
                    help="sweeps before the warm-up; -1: as many as make the timed sweeps the "
                         "last of the workload's stated run (500 sweeps for the main line)")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--block", type=int, default=0, help="sweep workgroup size, 0 = autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-parallel", action="store_true",
                    help="skip the oracle on all host threads (context for the CPU baseline)")
    ap.add_argument("--traffic", default=os.path.join(
                        ROOT, "profiles", "k_sweep_spec-s64x64-n144000-dyn64x64-f32.traffic.json"),
                    help="JSON with rocprofv3 FETCH_SIZE/WRITE_SIZE bytes per sweep-kernel launch; "
                         "used only while the kernel source hash it records is current")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 32-chain workload measured next to the main one")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the batch of uneven instances")
    ap.add_argument("--uneven-count", type=int, default=256)
    ap.add_argument("--uneven-steps", type=int, default=10)
    ap.add_argument("--uneven-block", type=int, default=64,
                    help="sweep kernel form for the uneven batch (64: one wave per region)")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the per-kernel rates (refresh, simulator, features, network)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain study on the 5x5-station worlds")
    ap.add_argument("--learned-worlds", type=int, default=50)
    ap.add_argument("--learned-sweeps", type=int, default=1000)
    ap.add_argument("--learned-chains", type=int, default=8)
    ap.add_argument("--learned-block", type=int, default=0,
                    help="sweep kernel form of the learned study's batches (0: tuned while running)")
    ap.add_argument("--learned-pairs", type=int, default=10_000_000)
    ap.add_argument("--no-template", action="store_true",
                    help="skip the mean-template likelihood on the main workload's shape")
    ap.add_argument("--no-paper-world", action="store_true",
                    help="skip the paper's own 1-D experiment (50 worlds x 5 runs)")
    ap.add_argument("--no-paper-latent", action="store_true",
                    help="skip the paper's world with latent arrival times")
    ap.add_argument("--paper-worlds", type=int, default=50)
    ap.add_argument("--paper-runs", type=int, default=5)
    ap.add_argument("--paper-sweeps", type=int, default=100)
    ap.add_argument("--no-small-full", action="store_true",
                    help="skip the 5x5-station workload run in full on the GPU and by the oracle")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic for calibrating hardware byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """(threads this process may use, CPU model name)."""
    n = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


def cpu_baseline(w, state, budget_s: float, threads: int = 1):
    """The oracle as it stands on the same instance and the same chain: the
    GPU's trace and its events after the timed sweeps (state = (trace,
    events, next sweep)), the same seed, then sweeps until budget_s.
    threads > 1 runs the regions of each colour phase across that many host
    threads (the paper's own CPU parallelism; the chain is the same)."""
    import numpy as np

    import oracle as O

    trace, events, first = state
    m = O.make_model(**w.model.asdict())
    sp = O.make_sampler(**w.sampler.asdict())
    ch = O.Chain(m, sp, trace, seed=w.seed)
    ev = O.as_events(events["x"], events["y"], events["t"], events["m"], events["id"])
    assert ch.set_events(ev) == 0
    ch.set_threads(threads)
    R, k = w.sampler.nreg, w.sampler.k
    logbuf = np.full((R, k, 4), -1.0)
    moves, evaluated, sweeps, t0 = 0, 0, 0, time.perf_counter()
    while True:
        logbuf[...] = -1.0
        assert ch.sweep(first + sweeps, log=logbuf) == 0
        moves += int(np.sum(logbuf[..., 1] >= 0))
        evaluated += int(np.sum(logbuf[..., 1] >= 1))
        sweeps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    how = "single thread" if threads == 1 else \
        f"{threads} threads over the regions of each colour phase"
    return dict(value=moves / el, unit="proposals/s", cores=threads,
                kind="oracle" if threads == 1 else "oracle-threads",
                evaluated_per_s=evaluated / el,
                sample=f"{w.name}: oracle sweeps {first}..{first + sweeps - 1} ({sweeps} sweeps, "
                       f"{moves} proposals, {el:.1f} s) continuing the GPU chain from its state "
                       f"after the timed sweeps ({len(events)} events) on the same trace, {how}")


def small_full(dev):
    """The 5x5-station, 1000-sample fp64 workload run as stated (2000 sweeps
    from the empty world, seed 0) twice on the same simulated instance: on
    the GPU (one chain, graph-replayed sweeps; the kernel form tuned on its
    first sweeps and graph construction included) and by the oracle on one
    host thread; each run's final state is scored against the truth."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1612_00595_amd import chromh, metrics as M, workloads as W
    w = W.SMALL
    tr = W.truth_events(w.model, w.seed)
    truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"], tr["id"])
    trace = chromh.simulate(w.model, truth, 1000 + w.seed, w.trace_dtype, dev)
    smp = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=1, seed=w.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the kernel form tuned on the run's first sweeps (every form gives the
    # same chain), inside the timed run
    first = smp.tune_running(0, 2)
    smp.run_sweeps(first, w.sweeps - first)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    st = smp.read_counters(0)
    gpu_moves = int(st[:15].reshape(5, 3)[:, 0].sum())
    f1_gpu = M.match(tr, smp.read_events(0)).f1
    block = smp.block
    smp.close()
    m = O.make_model(**w.model.asdict())
    sp = O.make_sampler(**w.sampler.asdict())
    ch = O.Chain(m, sp, trace.cpu().numpy(), seed=w.seed)
    t0 = time.perf_counter()
    for sw in range(w.sweeps):
        assert ch.sweep(sw) == 0
    t_cpu = time.perf_counter() - t0
    f1_cpu = M.match(tr, ch.events()).f1
    out = {"workload": w.name, "sweeps": w.sweeps, "proposals": gpu_moves, "block": block,
           "gpu_seconds": t_gpu, "oracle_seconds": t_cpu, "oracle_cores": 1,
           "gpu_over_oracle": t_cpu / t_gpu, "f1_gpu": f1_gpu, "f1_oracle": f1_cpu}
    log(f"[bench] {w.name} in full ({w.sweeps} sweeps): GPU {t_gpu:.2f} s, oracle {t_cpu:.2f} s "
        f"on one host thread; final F1 {f1_gpu:.3f} (GPU), {f1_cpu:.3f} (oracle)")
    return out


# network FLOPs per row: forward 2 (576*256 + 2*256*256 + 256*64) multiply-adds
# (the head padded to 64), training about three times that (forward, input
# gradients, weight gradients)
MDN_FWD_FLOP = 2 * (576 * 256 + 2 * 256 * 256 + 256 * 64)
MDN_TRAIN_FLOP = 3 * MDN_FWD_FLOP
BF16_PEAK_TFLOPS = 2500.0
F1_EVERY = 50


LEARNED_MAX_EVENTS = 96   # recorded events per chain and sweep (the worlds hold ~20)
TUNE_MIN_SWEEPS = 50      # runs at least this long tune their kernel form on their first sweeps


def learned_study(args, dev):
    """The learned birth proposal against the plain sampler on 5x5-station,
    1000-sample worlds (seeds 100, 101, ...): the network trained on fresh
    simulator pairs, then every (world, chain) of a mode as one instance of a
    single batch (one launch per colour for all of them), with and without
    learned births (each world's own anchor table), every state recorded on
    the device; F1 of the final states, F1 against sweeps, and event-location
    ESS after a quarter of burn-in."""
    import numpy as np
    import torch

    from paper_1612_00595_amd import chromh, learned, metrics as M, workloads as W
    w = W.SMALL
    log(f"[bench] training the proposal network on {args.learned_pairs} simulator pairs")
    tr = learned.train(w.model, pairs=args.learned_pairs, batch=8192, lr=1e-3, seed=0)
    train_tflops = tr.pairs * MDN_TRAIN_FLOP / tr.seconds / 1e12
    nw, nc = args.learned_worlds, args.learned_chains
    out = {"workload": w.name + " worlds", "worlds": nw, "chains": nc,
           "sweeps": args.learned_sweeps, "batch_instances": nw * nc,
           "train": {"pairs": tr.pairs, "batch": 8192, "seconds": tr.seconds,
                     "held_out_nll": tr.held_out, "achieved_TFLOPs": train_tflops,
                     "mfma_frac": train_tflops / BF16_PEAK_TFLOPS}}
    truths, traces, tables = [], [], []
    infer_s = 0.0
    for wi in range(nw):
        seed = 100 + wi
        tr_ev = W.truth_events(w.model, seed)
        truths.append(tr_ev)
        truth = chromh.as_events(tr_ev["x"], tr_ev["y"], tr_ev["t"], tr_ev["m"])
        traces.append(chromh.simulate(w.model, truth, 1000 + seed, w.trace_dtype, dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tables.append(learned.anchor_table(tr.net, w.model, traces[-1]))
        torch.cuda.synchronize()
        infer_s += time.perf_counter() - t0
    q_of = [(wi, c) for wi in range(nw) for c in range(nc)]
    per = {}
    checkpoints = list(range(F1_EVERY - 1, args.learned_sweeps, F1_EVERY))
    for mode in ("plain", "learned"):
        def make(form):
            b = chromh.Batch([w.model] * len(q_of), [w.sampler] * len(q_of),
                             [traces[wi] for wi, c in q_of],
                             [(100 + wi) * 1000 + c for wi, c in q_of], block=form)
            if mode == "learned":
                for q, (wi, c) in enumerate(q_of):
                    T, wt, ntau = tables[wi]
                    b.set_learned_instance(q, T, wt, ntau, 0.5)
            return b
        b = make(args.learned_block)
        S = args.learned_sweeps
        rec = b.set_record(0, S + 1, LEARNED_MAX_EVENTS)
        # each mode runs in the form that is fastest for it, tuned on the run's
        # first sweeps (every form gives the same chain), which also build the
        # graphs outside the timed region
        first = 1
        if args.learned_block or S < TUNE_MIN_SWEEPS:
            b.run_sweeps(0, 1)
        else:
            first = b.tune_running(0, 2)
        torch.cuda.synchronize()
        c0 = [b.read_counters(q) for q in range(len(q_of))]
        t0 = time.perf_counter()
        b.run_sweeps(first, S + 1 - first)
        torch.cuda.synchronize()
        # seconds and proposals of S sweeps at the timed sweeps' rate
        scale = S / (S + 1 - first)
        el = (time.perf_counter() - t0) * scale
        st = sum(b.read_counters(q) - c0[q] for q in range(len(q_of))) * scale
        recc = rec[1:].cpu().numpy()
        b.set_record(0, 0, 0)
        block = b.block
        b.close()
        del rec
        f1 = np.zeros((nw, nc))
        ess = np.full((nw, nc), np.nan)
        curve = np.zeros((nw, len(checkpoints)))
        for q, (wi, c) in enumerate(q_of):
            states = chromh.ChromaticSampler.recorded_states(recc, q)
            f1[wi, c] = M.match(truths[wi], states[-1]).f1
            curve[wi] += [M.match(truths[wi], states[k]).f1 for k in checkpoints]
            e, k = M.location_ess(states, truths[wi])
            if k:
                ess[wi, c] = e
        del recc
        tab = st[:15].reshape(5, 3).astype(float)
        per[mode] = dict(seconds=el, f1=f1, ess=ess, curve=curve / nc, block=block,
                         proposals=float(tab[:, 0].sum()),
                         acc=(tab[:, 2] / np.maximum(tab[:, 0], 1)).tolist())
        torch.cuda.empty_cache()
    for mode in ("plain", "learned"):
        r = per[mode]
        # worlds are the independent units: the interval is over world means
        mean, lo, hi = M.bootstrap_ci(r["f1"].mean(axis=1))
        ess_chain = float(np.nanmean(r["ess"]))
        out[mode] = {"f1": mean, "f1_ci95": [lo, hi],
                     # ESS/s per GPU: mean ESS per chain times the chains that run together
                     "ess_per_s": ess_chain * len(q_of) / r["seconds"],
                     "ess_per_sweep_chain": ess_chain / args.learned_sweeps,
                     "proposals_per_s": r["proposals"] / r["seconds"],
                     "ms_per_sweep": r["seconds"] * 1e3 / args.learned_sweeps,
                     "block": r["block"],
                     "acceptance_birth_death_loc_time_mag": np.round(r["acc"], 4).tolist()}
    pl, le = out["plain"], out["learned"]
    out["ess_per_s_ratio"] = le["ess_per_s"] / pl["ess_per_s"]
    # F1 against wall time (mean over worlds and chains, every F1_EVERY
    # sweeps): when the learned chains first reach the plain chains' final F1
    cp = per["plain"]["curve"].mean(axis=0)
    cl = per["learned"]["curve"].mean(axis=0)
    sw = np.arange(F1_EVERY, args.learned_sweeps + 1, F1_EVERY)
    hit = np.nonzero(cl >= cp[-1])[0] if len(cp) else []
    out["f1_curve"] = {"sweeps": sw.tolist(), "plain": cp.round(4).tolist(),
                       "learned": cl.round(4).tolist()}
    if len(hit):
        t_l = sw[hit[0]] * le["ms_per_sweep"]
        t_p = args.learned_sweeps * pl["ms_per_sweep"]
        out["time_to_plain_final_f1"] = {"learned_ms": float(t_l), "plain_ms": float(t_p),
                                         "speedup": float(t_p / t_l)}
    out["equal_f1"] = bool(abs(le["f1"] - pl["f1"]) <= 0.02 or
                           (le["f1_ci95"][0] <= pl["f1_ci95"][1]
                            and pl["f1_ci95"][0] <= le["f1_ci95"][1]))
    na = w.model.nsta * ((w.model.N - 67) // 32 + 1)
    out["inference"] = {"anchors_per_world": na, "seconds_per_world": infer_s / nw}
    log(f"[bench] learned study ({len(q_of)} chains in one batch): F1 plain {pl['f1']:.3f} "
        f"learned {le['f1']:.3f}; ESS/s plain {pl['ess_per_s']:.4g} learned "
        f"{le['ess_per_s']:.4g}; {pl['ms_per_sweep']:.3f} / {le['ms_per_sweep']:.3f} ms per "
        f"sweep; training {tr.seconds:.2f} s ({train_tflops:.1f} TFLOP/s)")
    del traces, tables
    return out, tr.net


def paper_world_study(args, dev, latent: bool = False):
    """Section 5's experiment on the paper's own 1-D world (four stations on
    a line, T = 240, Section 4.1's time partition): worlds from the model
    (seeds 2000, 2001, ...), several runs each, under the paper's four
    schedules, each run as one batch of every (world, run) chain: serial MH
    (one region, 2000 moves per sweep), naive parallel MH (Algorithm 3: four
    onset regions in one phase), chromatic static and chromatic dynamic (four
    onset regions, two colours), k = 500 moves per region per phase, so the
    same 2000 moves per sweep.  Every state is recorded on the device; precision,
    recall, F1 and location error (Section 5's matching, 12 units in space and
    time) against sweeps and wall time, and 95% bootstrap intervals over worlds
    of the final values.  The oracle runs the same schedules on two worlds for
    the CPU rate.

    latent: the same world with Section 3's latent arrival times (offsets of
    sd 1 sample, truncated at 4 sd) and the arrival-time and joint moves; the
    four onset regions then need three colours, and the naive schedule is not
    part of the mode."""
    import dataclasses

    import numpy as np
    import torch

    import oracle as O
    from paper_1612_00595_amd import chromh, metrics as M, workloads as W
    wl = W.PAPER1D_LATENT if latent else W.PAPER1D
    spec, base = wl.model, wl.sampler
    scheds = {"serial": dataclasses.replace(base, gx=1, k=2000)}
    if not latent:
        scheds["naive"] = dataclasses.replace(base, schedule=1)
    scheds["chromatic_static"] = base
    scheds["chromatic_dynamic"] = dataclasses.replace(base, dynamic=1)
    nw, nr, S = args.paper_worlds, args.paper_runs, args.paper_sweeps
    truths, traces = [], []
    for wi in range(nw):
        tr = W.truth_events(spec, 2000 + wi)
        truths.append(tr)
        traces.append(chromh.simulate(spec, chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"],
                                                             da=tr["da"]),
                                      3000 + wi, "f64", dev))
    every = 5
    out = {"workload": wl.name + " worlds", "worlds": nw, "runs": nr, "sweeps": S,
           "moves_per_sweep": 2000, "match_thresholds": [M.PAPER_DIST_THRESH, TIME_THRESH_1D],
           "true_events_mean": float(np.mean([len(t["x"]) for t in truths]))}
    n = nw * nr

    def batch(sp, block):
        return chromh.Batch([spec] * n, [sp] * n, [traces[q // nr] for q in range(n)],
                            [7919 * (q // nr) + q % nr for q in range(n)], block=block)

    for name, sp in scheds.items():
        b = batch(sp, 0)
        rec = b.set_record(0, S + 1, 64)
        # the kernel form, tuned on the run's first sweeps (every form gives
        # the same chain), which also build the graphs outside the timed region
        if S >= TUNE_MIN_SWEEPS:
            first = b.tune_running(0, 2)
        else:
            b.run_sweeps(0, 1)
            first = 1
        block = b.block
        torch.cuda.synchronize()
        c0 = sum(b.read_counters(q) for q in range(n))
        t0 = time.perf_counter()
        b.run_sweeps(first, S + 1 - first)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d = sum(b.read_counters(q) for q in range(n)) - c0
        proposals = float(d[:15].reshape(5, 3)[:, 0].sum())
        pts = list(range(every - 1, S, every))
        P = np.zeros((n, len(pts))); Rc = np.zeros_like(P); F = np.zeros_like(P)
        E = np.full_like(P, np.nan)
        recc = rec[1:].cpu().numpy()
        for q in range(n):
            states = chromh.ChromaticSampler.recorded_states(recc, q)
            for a, sw in enumerate(pts):
                r = M.match(truths[q // nr], states[sw], dist_thresh=M.PAPER_DIST_THRESH,
                            time_thresh=TIME_THRESH_1D)
                P[q, a], Rc[q, a], F[q, a], E[q, a] = r.precision, r.recall, r.f1, \
                    r.location_error
        b.close()
        ms = el * 1e3 / (S + 1 - first)

        def final(v):
            per_world = np.nanmean(v[:, -1].reshape(nw, nr), axis=1)
            mean, lo, hi = M.bootstrap_ci(per_world[np.isfinite(per_world)])
            return [mean, lo, hi]
        if latent:  # arrival-time and joint moves: attempted, valid, accepted
            proposals += float(d[17:23].reshape(2, 3)[:, 0].sum())
        out[name] = {
            "ms_per_sweep": ms, "proposals_per_s": proposals / el, "block": block,
            "final_precision_ci95": final(P), "final_recall_ci95": final(Rc),
            "final_f1_ci95": final(F), "final_location_error_ci95": final(E),
            "curve": {"sweeps": [p + 1 for p in pts],
                      "ms": [(p + 1) * ms for p in pts],
                      "precision": P.mean(0).round(4).tolist(),
                      "recall": Rc.mean(0).round(4).tolist(),
                      "f1": F.mean(0).round(4).tolist(),
                      "location_error": np.nanmean(E, 0).round(3).tolist()}}
        if latent:
            out[name]["arrival_moves"] = [int(v) for v in d[17:20]]
            out[name]["joint_moves"] = [int(v) for v in d[20:23]]
        log(f"[bench] paper world{' (latent arrivals)' if latent else ''}, {name} (block {block}): "
            f"{ms:.3f} ms/sweep for {n} chains, {proposals / el:.4g} proposals/s, "
            f"final F1 {out[name]['final_f1_ci95'][0]:.3f}")
    # the oracle: the same schedules, two worlds, one run each
    osw = max(S // 5, 4)
    m = O.make_model(**spec.asdict())
    orc = {}
    for name, sp in scheds.items():
        t0, moves = time.perf_counter(), 0
        for wi in range(2):
            s = O.simulate(m, O.as_events(truths[wi]["x"], truths[wi]["y"], truths[wi]["t"],
                                          truths[wi]["m"], da=truths[wi]["da"]), 3000 + wi)
            ch = O.Chain(m, O.make_sampler(**sp.asdict()), s, seed=7919 * wi)
            for sw in range(osw):
                assert ch.sweep(sw) == 0
            moves += osw * 2000
        el = time.perf_counter() - t0
        orc[name] = {"proposals_per_s": moves / el, "ms_per_sweep": el * 1e3 / (2 * osw)}
    out["cpu_baseline"] = dict(orc, kind="oracle", cores=1,
                               sample=f"2 worlds x 1 run x {osw} sweeps per schedule")
    st, se = out["chromatic_static"], out["serial"]
    out["per_chain_sweep_speedup_static_vs_serial"] = se["ms_per_sweep"] / st["ms_per_sweep"]
    out["gpu_vs_oracle_proposals"] = {k: out[k]["proposals_per_s"] / orc[k]["proposals_per_s"]
                                      for k in scheds}
    return out


UNEVEN_SWEEPS = 200   # the uneven batch's run: timed sweeps end here


def uneven_burn_in(args) -> int:
    return args.burn_in if args.burn_in >= 0 else \
        max(0, UNEVEN_SWEEPS - args.warmup - args.uneven_steps)


UNEVEN_RECORD = 32        # sweeps recorded after the timed ones for the per-instance report
UNEVEN_ESS_MAX_LAMBDA = 400.0   # location ESS for instances up to this Poisson mean


def uneven_study(args, dev, block: int, net=None):
    """Many independent instances of uneven size in one batch (every colour
    phase one launch over all instances' regions of that colour): proposals/s
    over graph-replayed sweeps and the algorithmic bytes the sweeps moved.
    net: learned births (p = 0.5) from the trained network, each instance's
    anchor table built from its own trace (features, fused network
    inference, mixture table).  After the timed sweeps UNEVEN_RECORD more are
    recorded on the device for a per-instance report: precision, recall and
    F1 of the last state, and event-location ESS/s (ESS over the recorded
    sweeps per second of the batch's sweep time) for the instances of
    Poisson mean up to UNEVEN_ESS_MAX_LAMBDA."""
    import numpy as np
    import torch

    from paper_1612_00595_amd import chromh, learned, metrics as M, workloads as W
    ws = W.uneven_batch(args.uneven_count)
    traces, models, samplers, seeds, truths = [], [], [], [], []
    for w in ws:
        tr = W.truth_events(w.model, w.seed)
        truths.append(tr)
        truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"])
        traces.append(chromh.simulate(w.model, truth, 1000 + w.seed, "f32", dev))
        models.append(w.model)
        samplers.append(w.sampler)
        seeds.append(w.seed)
    b = chromh.Batch(models, samplers, traces, seeds, block=block)
    anchors, t_tables = 0, 0.0
    if net is not None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q, (m, trc) in enumerate(zip(models, traces)):
            T, wt, ntau = learned.anchor_table(net, m, trc)
            anchors += m.nsta * ntau
            b.set_learned_instance(q, T, wt, ntau, 0.5)
        torch.cuda.synchronize()
        t_tables = time.perf_counter() - t0
    bu = uneven_burn_in(args)
    b.run_sweeps(0, bu + args.warmup)
    torch.cuda.synchronize()
    c0 = [b.read_counters(q) for q in range(len(ws))]
    t0 = time.perf_counter()
    b.run_sweeps(bu + args.warmup, args.uneven_steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c1 = [b.read_counters(q) for q in range(len(ws))]
    d = sum(x - y for x, y in zip(c1, c0))
    mv = d[:15].reshape(5, 3)
    proposals = int(mv[:, 0].sum())
    nbytes = int(d[15]) * 12 + int(d[16]) * 8
    out = {"workload": f"{len(ws)} uneven instances (sides 8..32, 4000..36000 fp32 samples, "
                       f"Poisson means 100..5000)" + (", learned births (p = 0.5)" if net else ""),
           "instances": len(ws), "stations": int(sum(m.nsta for m in models)),
           "regions": int(sum(sp.nreg for sp in samplers)),
           "poisson_mean_events": float(sum(m.lam for m in models)),
           "value": proposals / el, "unit": "proposals/s",
           "ms_per_step": el * 1e3 / args.uneven_steps,
           "burn_in_sweeps": bu,
           "algorithmic_GBps_whole_sweep": nbytes / el / 1e9,
           "frac_whole_sweep": nbytes / el / 1e9 / HBM_PEAK_GBS, "block": block,
           "births_attempted_valid_accepted": [int(v) for v in mv[0]],
           "deaths_attempted_valid_accepted": [int(v) for v in mv[1]]}
    if net is not None:
        out.update(anchors=int(anchors), tables_seconds=t_tables)
    # the per-instance report (untimed)
    first = bu + args.warmup + args.uneven_steps
    rec = b.set_record(first, UNEVEN_RECORD, 8192)
    b.run_sweeps(first, UNEVEN_RECORD)
    torch.cuda.synchronize()
    recc = rec.cpu().numpy()
    b.set_record(0, 0, 0)
    sweep_s = el / args.uneven_steps
    per = {"lam": [], "precision": [], "recall": [], "f1": [], "ess_per_s": []}
    for q, w in enumerate(ws):
        states = chromh.ChromaticSampler.recorded_states(recc, q)
        r = M.match(truths[q], states[-1])
        per["lam"].append(w.model.lam)
        per["precision"].append(round(r.precision, 4))
        per["recall"].append(round(r.recall, 4))
        per["f1"].append(round(r.f1, 4))
        e = None
        if w.model.lam <= UNEVEN_ESS_MAX_LAMBDA:
            ess, k = M.location_ess(states, truths[q], burn_frac=0.0)
            e = ess / (UNEVEN_RECORD * sweep_s) if k else None
        per["ess_per_s"].append(e)
    out["per_instance"] = per
    f1 = np.array(per["f1"])
    out["f1_mean_ci95"] = list(M.bootstrap_ci(f1))
    out["precision_mean"] = float(np.mean(per["precision"]))
    out["recall_mean"] = float(np.mean(per["recall"]))
    es = [v for v in per["ess_per_s"] if v is not None]
    out["ess_per_s_median"] = float(np.median(es)) if es else None
    log(f"[bench] uneven batch{' with learned births' if net else ''}: {out['value']:.4g} "
        f"proposals/s, {out['ms_per_step']:.2f} ms/sweep, "
        f"{out['algorithmic_GBps_whole_sweep']:.1f} GB/s algorithmic; mean F1 "
        f"{out['f1_mean_ci95'][0]:.3f}, median ESS/s {out['ess_per_s_median']}")
    b.close()
    del traces, b, rec
    torch.cuda.empty_cache()
    return out


def compare_uneven(plain, learn):
    """Per-instance learned against plain: F1 difference and the ratio of
    location ESS/s where both chains have one."""
    import numpy as np
    pl, le = plain["per_instance"], learn["per_instance"]
    df1 = np.array(le["f1"]) - np.array(pl["f1"])
    ratios = [b / a for a, b in zip(pl["ess_per_s"], le["ess_per_s"])
              if a is not None and b is not None and a > 0]
    return {"f1_learned_minus_plain_mean": float(df1.mean()),
            "f1_learned_minus_plain_quartiles": np.quantile(df1, [0.25, 0.5, 0.75]).round(4).tolist(),
            "ess_per_s_ratio_quartiles": (np.quantile(ratios, [0.25, 0.5, 0.75]).round(3).tolist()
                                          if ratios else None),
            "instances_with_ess": len(ratios),
            "proposals_per_s_ratio": learn["value"] / plain["value"]}


def kernel_rates(dev):
    """The other rows of the path, each against its own roofline, on the
    32x32-station, 36000-sample instance: the forward simulator, the exact
    refresh (variance and log-likelihood), the anchor features of every
    window, the network's forward pass over them and the mixture table.
    Durations from HIP events on the stream the library launches on."""
    import torch

    from paper_1612_00595_amd import chromh, workloads as W
    w = W.CHAINS32
    m = w.model
    samples = m.nsta * m.N
    tr = W.truth_events(m, w.seed)
    truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"])

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3, out

    out = {"workload": w.name.replace("-c32", "") + " (one chain)"}
    t, trace = timed(lambda: chromh.simulate(m, truth, 1000 + w.seed, "f32", dev), 2)
    out["simulate"] = {"seconds": t, "GBps_written": samples * 4 / t / 1e9,
                       "bound": "fp64 alu (Philox, Box-Muller per sample)"}
    smp = chromh.ChromaticSampler(m, w.sampler, trace, chains=1, seed=w.seed, block=64)
    smp.run_sweeps(0, 20)
    t, _ = timed(lambda: smp.refresh(write_variance=True, loglik=True))
    out["refresh"] = {"seconds": t, "GBps": samples * 12 / t / 1e9,
                      "frac": samples * 12 / t / 1e9 / HBM_PEAK_GBS,
                      "bytes_per_sample": 12, "bound": "hbm (4 B trace read, 8 B variance written)"}
    smp.close()
    na, ntau = chromh.anchor_count(m)
    t, (X, wts) = timed(lambda: chromh.anchor_features(m, trace), 2)
    out["anchor_features"] = {"anchors": na, "seconds": t, "anchors_per_s": na / t,
                              "GBps_written": na * (576 * 2 + 8) / t / 1e9}
    net = chromh.MDN(seed=1)
    chunk = 1 << 18

    def forward_all():
        return torch.cat([net.forward(X[q:q + chunk]) for q in range(0, na, chunk)])

    t, head = timed(forward_all, 2)
    out["mdn_forward"] = {"rows": na, "seconds": t, "TFLOPs": na * MDN_FWD_FLOP / t / 1e12,
                          "mfma_frac": na * MDN_FWD_FLOP / t / 1e12 / BF16_PEAK_TFLOPS,
                          "bound": "mfma (bf16, fp32 accumulate)",
                          "kind": "layer by layer (training path: pre-activations kept)"}
    # the fused inference kernel the anchor tables use: activations stay in
    # LDS, one launch over every anchor
    t, head = timed(lambda: net.infer(X), 2)
    out["mdn_infer"] = {"rows": na, "seconds": t, "TFLOPs": na * MDN_FWD_FLOP / t / 1e12,
                        "mfma_frac": na * MDN_FWD_FLOP / t / 1e12 / BF16_PEAK_TFLOPS,
                        "bound": "mfma (bf16, fp32 accumulate)", "kind": "fused, one kernel"}
    t, _ = timed(lambda: chromh.mixture_table(m, head), 2)
    out["mixture_table"] = {"rows": na, "seconds": t, "rows_per_s": na / t}
    log(f"[bench] kernels: refresh {out['refresh']['GBps']:.0f} GB/s, simulate "
        f"{out['simulate']['GBps_written']:.0f} GB/s written, features {na / out['anchor_features']['seconds']:.3g} "
        f"anchors/s, network forward {out['mdn_forward']['TFLOPs']:.1f} TFLOP/s, fused inference "
        f"{out['mdn_infer']['TFLOPs']:.1f} TFLOP/s")
    del X, wts, head, trace, net
    return out


def stream_peaks(dev, gib: int = 4):
    """The device's own streaming rates, for context beside the spec peak:
    a device-to-device copy (read + write counted) and a fill (write only)
    of `gib` GiB, timed with HIP events on the current stream."""
    import torch
    n = gib << 28  # float32 elements
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn, nbytes in (("copy", lambda: dst.copy_(src), 8 * n),
                             ("fill", lambda: dst.fill_(2.0), 4 * n)):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(3):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_GBps"] = nbytes * 3 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


def burn_in_for(w, warmup: int, steps: int) -> int:
    """Sweeps run before the warm-up so that the timed sweeps are the last of
    the workload's stated run length (the chain starts from the empty world;
    its event count only reaches the posterior's level after a few hundred
    sweeps)."""
    return max(0, w.sweeps - warmup - steps)


def measure(smp, w, warmup: int, steps: int, burn_in: int = 0, tune: bool = False):
    """Proposals/s over `steps` graph-replayed sweeps that follow `burn_in`
    + `warmup` untimed ones, and from those same sweeps the sweep kernel's
    launch spans (device steady-clock stamps taken by the kernel's own
    workgroups inside the replayed graphs) and the algorithmic bytes they
    moved (the kernels' own counts of footprint samples read and
    rewritten).  tune: choose the kernel form after the burn-in, on the
    state the timed sweeps start from."""
    import numpy as np
    import torch

    from paper_1612_00595_amd import chromh
    if burn_in:
        smp.run_sweeps(0, burn_in)
    if tune:
        smp.autotune(burn_in, 3)
    first = burn_in + warmup
    stamps = smp.set_stamps(first, steps)  # before the sweep graphs are built
    smp.run_sweeps(burn_in, warmup)
    torch.cuda.synchronize()
    c0 = sum(smp.read_counters(c) for c in range(w.chains))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.run_sweeps(first, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = sum(smp.read_counters(c) for c in range(w.chains))
    spans = chromh.ChromaticSampler.stamp_seconds(stamps)
    smp.set_stamps(0, 0)
    el = t1 - t0
    d = c1 - c0
    tab = d[:15].reshape(5, 3)
    if w.model.arr_sd > 0:
        tab = np.concatenate([tab, d[17:23].reshape(2, 3)])
    proposals, evaluated, accepted = (int(v) for v in tab.sum(0))
    # colours without regions launch nothing: their stamps stay (max, 0)
    live = spans > 0
    kernel_s = float(spans[live].sum())
    # the variance model reads the trace and E per footprint sample; the
    # mean-template model reads only its residual
    tb = 0 if w.model.tmpl else (4 if w.trace_dtype == "f32" else 8)
    nbytes = int(d[15]) * (tb + 8) + int(d[16]) * 8
    launches = int(live.sum())
    return dict(elapsed=el, proposals=proposals, evaluated=evaluated, accepted=accepted,
                value=proposals / el, first=first, launches=launches,
                avg_launch_s=kernel_s / max(launches, 1), kernel_s=kernel_s,
                bytes_per_launch=nbytes / max(launches, 1),
                achieved=nbytes / kernel_s / 1e9 if kernel_s > 0 else 0.0,
                span_ms_per_sweep=spans.clip(min=0).sum(1).round(4).tolist(),
                acceptance=(tab[:, 2] / np.maximum(tab[:, 0], 1)).round(4).tolist(),
                events_after=[len(smp.read_events(c)) for c in range(min(w.chains, 4))])


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sampler's "
              "multi-GPU sharding is a design, not a build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1612_00595_amd import chromh, workloads as W

    w = W.WORKLOADS[args.workload] if args.workload else W.LARGE
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tr = W.truth_events(w.model, w.seed)
    truth = chromh.as_events(tr["x"], tr["y"], tr["t"], tr["m"], tr["id"])
    log(f"[bench] simulating {w.name}: {w.model.nsta} stations x {w.model.N} samples, "
        f"{len(truth)} true events")
    trace = chromh.simulate(w.model, truth, 1000 + w.seed, w.trace_dtype, dev)
    smp = chromh.ChromaticSampler(w.model, w.sampler, trace, chains=w.chains, seed=w.seed,
                                  block=args.block)
    burn = args.burn_in if args.burn_in >= 0 else burn_in_for(w, args.warmup, args.steps)
    res = measure(smp, w, args.warmup, args.steps, burn, tune=args.block == 0)
    el, value = res["elapsed"], res["value"]
    avg_s, bytes_per_launch, achieved = res["avg_launch_s"], res["bytes_per_launch"], res["achieved"]
    log(f"[bench] sweep kernel form {smp.block}, {smp.ncolors} colours; sweeps "
        f"{res['first']}..{res['first'] + args.steps - 1} timed after {burn} of burn-in")
    log(f"[bench] {args.steps} sweeps in {el * 1e3:.1f} ms: {value:.4g} proposals/s "
        f"({res['evaluated'] / el:.4g} evaluated), events {res['events_after']}")
    traffic = None
    if args.traffic and os.path.exists(args.traffic) and w is W.LARGE:
        import hashlib
        t = json.load(open(args.traffic))
        srcs = [os.path.join(ROOT, "paper_1612_00595_amd", "csrc", f)
                for f in ("cmh_kernels.hip", "cmh_common.hpp")]
        digest = hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()
        if t.get("source_sha256") == digest and t.get("block") == smp.block:
            traffic = t.get("bytes_per_launch")
    log(f"[bench] sweep kernel: {avg_s * 1e6:.1f} us/launch (device stamps), "
        f"{bytes_per_launch / 1e6:.3f} MB/launch algorithmic, {achieved:.1f} GB/s; "
        f"{res['kernel_s'] / el * 100:.1f} % of the timed region in the sweep kernel")
    # the chain's trace and state at the end of the timed sweeps: the CPU
    # oracle continues from exactly there
    cpu_state = None
    if not args.no_cpu_baseline:
        cpu_state = (trace.cpu().numpy(), smp.read_events(0), res["first"] + args.steps)

    # the exact refresh (variance written, log-likelihood summed) on the same
    # full-size instance: 12 B per sample streamed
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    smp.refresh(write_variance=True, loglik=True)
    torch.cuda.synchronize()
    e0.record()
    smp.refresh(write_variance=True, loglik=True)
    e1.record()
    torch.cuda.synchronize()
    t_ref = e0.elapsed_time(e1) * 1e-3
    refresh_large = {"workload": w.name, "seconds": t_ref,
                     "GBps": w.model.nsta * w.model.N * 12 / t_ref / 1e9,
                     "frac": w.model.nsta * w.model.N * 12 / t_ref / 1e9 / HBM_PEAK_GBS,
                     "bytes_per_sample": 12, "bound": "hbm"}
    peaks = stream_peaks(dev)
    refresh_large["frac_of_measured_copy"] = refresh_large["GBps"] / peaks["copy_GBps"]
    log(f"[bench] refresh on {w.name}: {refresh_large['GBps']:.0f} GB/s; device copy "
        f"{peaks['copy_GBps']:.0f} GB/s, fill {peaks['fill_GBps']:.0f} GB/s")
    nev = len(smp.read_events(0))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "stations": w.model.nsta,
            "samples": w.model.N,
            "trace_dtype": w.trace_dtype,
            "regions": f"{w.sampler.gx + 1}x{w.sampler.gy + 1}",
            "dynamic_offsets": bool(w.sampler.dynamic),
            "colours": smp.ncolors,
            "moves_per_region": w.sampler.k,
            "chains": w.chains,
            "poisson_mean_events": w.model.lam,
            "burn_in_sweeps": burn,
            "timed_sweeps": [res["first"], res["first"] + args.steps - 1],
            "events_after_run": nev,
            "block": smp.block,
        },
        "proposals": {
            "attempted": res["proposals"], "evaluated": res["evaluated"],
            "rejected_without_delta": res["proposals"] - res["evaluated"],
            "accepted": res["accepted"],
            "evaluated_per_s": res["evaluated"] / el,
            "acceptance_birth_death_loc_time_mag": res["acceptance"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "sweep colour phase (form %d)" % smp.block,
            "avg_launch_us": avg_s * 1e6,
            "launches": res["launches"],
            "duration_source": "device steady-clock stamps of the timed sweeps",
            "kernel_share_of_step": res["kernel_s"] / el,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "measured_stream_GBps": peaks,
        },
    }
    block = smp.block
    smp.close()
    del trace
    torch.cuda.empty_cache()
    if not args.no_batched:
        wb = W.CHAINS32
        trb = W.truth_events(wb.model, wb.seed)
        truthb = chromh.as_events(trb["x"], trb["y"], trb["t"], trb["m"], trb["id"])
        traceb = chromh.simulate(wb.model, truthb, 1000 + wb.seed, wb.trace_dtype, dev)
        sb = chromh.ChromaticSampler(wb.model, wb.sampler, traceb, chains=wb.chains,
                                     seed=wb.seed, block=args.block)
        kb = max(args.steps // 5, 5)
        bb = args.burn_in if args.burn_in >= 0 else burn_in_for(wb, args.warmup, kb)
        rb = measure(sb, wb, args.warmup, kb, bb, tune=args.block == 0)
        log(f"[bench] {wb.name}: {rb['value']:.4g} proposals/s (form {sb.block}), sweep kernel "
            f"{rb['avg_launch_s'] * 1e6:.1f} us/launch, {rb['achieved']:.1f} GB/s algorithmic")
        out["batched"] = {
            "workload": wb.name, "chains": wb.chains, "value": rb["value"],
            "unit": "proposals/s", "ms_per_step": rb["elapsed"] * 1e3 / kb,
            "burn_in_sweeps": bb, "timed_sweeps": [rb["first"], rb["first"] + kb - 1],
            "sweep_kernel_us": rb["avg_launch_s"] * 1e6,
            "kernel_share_of_step": rb["kernel_s"] / rb["elapsed"],
            "algorithmic_bytes_per_launch": rb["bytes_per_launch"],
            "achieved_GBps": rb["achieved"], "frac": rb["achieved"] / HBM_PEAK_GBS,
            "rejected_without_delta": rb["proposals"] - rb["evaluated"],
            "acceptance_birth_death_loc_time_mag": rb["acceptance"],
            "block": sb.block,
        }
        sb.close()
        del traceb
        torch.cuda.empty_cache()
    if not args.no_template:
        # the mean-template likelihood on the main workload's shape: the
        # state is the residual (8 B read per footprint sample, no trace)
        wt = dataclasses.replace(w, name=w.name + "-template",
                                 model=dataclasses.replace(w.model, tmpl=1))
        trt = chromh.simulate(wt.model, truth, 1000 + wt.seed, wt.trace_dtype, dev)
        st_ = chromh.ChromaticSampler(wt.model, wt.sampler, trt, chains=1, seed=wt.seed,
                                      block=block)
        rt = measure(st_, wt, args.warmup, args.steps, burn)
        log(f"[bench] {wt.name}: {rt['value']:.4g} proposals/s, sweep kernel "
            f"{rt['avg_launch_s'] * 1e6:.1f} us/launch, {rt['achieved']:.1f} GB/s algorithmic")
        out["template"] = {
            "workload": wt.name, "value": rt["value"], "unit": "proposals/s",
            "ms_per_step": rt["elapsed"] * 1e3 / args.steps, "block": block,
            "burn_in_sweeps": burn, "timed_sweeps": [rt["first"], rt["first"] + args.steps - 1],
            "sweep_kernel_us": rt["avg_launch_s"] * 1e6,
            "algorithmic_bytes_per_launch": rt["bytes_per_launch"],
            "bytes_per_sample": "8 read (residual) + 8 written on accept",
            "achieved_GBps": rt["achieved"], "frac": rt["achieved"] / HBM_PEAK_GBS,
            "events_after_run": len(st_.read_events(0))}
        st_.close()
        del trt
        torch.cuda.empty_cache()
    if not args.no_kernels:
        out["kernels"] = kernel_rates(dev)
        out["kernels"]["refresh_full_size"] = refresh_large
        torch.cuda.empty_cache()
    if not args.no_uneven:
        out["uneven"] = uneven_study(args, dev, args.uneven_block)
        torch.cuda.empty_cache()
    if not args.no_learned:
        out["learned"], net = learned_study(args, dev)
        if not args.no_uneven:
            out["uneven_learned"] = uneven_study(args, dev, args.uneven_block, net)
            out["uneven_learned"]["vs_plain"] = compare_uneven(out["uneven"],
                                                                out["uneven_learned"])
        del net
        torch.cuda.empty_cache()
    if not args.no_paper_world:
        out["paper_world"] = paper_world_study(args, dev)
    if not args.no_paper_latent:
        out["paper_world_latent"] = paper_world_study(args, dev, latent=True)
        torch.cuda.empty_cache()
    if not args.no_small_full:
        out["small_full"] = small_full(dev)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w, cpu_state, args.cpu_seconds)
        threads, cpu_model = host_cpu()
        out["cpu_baseline"]["cpu_model"] = cpu_model
        if not args.no_cpu_parallel and threads > 1:
            # context, not the baseline: the oracle's colour phases across
            # the host's cores (the parallelism of the paper's own runs)
            out["cpu_parallel"] = cpu_baseline(w, cpu_state, args.cpu_seconds, threads)
            out["cpu_parallel"]["cpu_model"] = cpu_model
            log(f"[bench] oracle on {threads} host threads: "
                f"{out['cpu_parallel']['value']:.4g} proposals/s")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
