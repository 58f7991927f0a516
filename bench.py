#!/usr/bin/env python3
"""Throughput of the dynamic-bonding hot path on one MI355X.

Workload: 12,500 random 40-nt strands paired into 6,250 pre-hybridized duplexes
of the 2-bead/nucleotide model (1,000,000 beads, density 0.5, box 125.99 sigma),
WCA pairs, harmonic bonds, straight backbone and rung angles, cis stacking
dihedrals, Langevin thermostat on a 0.5 -> 1.5 temperature ramp over 1e5 steps,
bond sweep (create within 1.5 sigma with p = 0.5, kill beyond 2.0 sigma, at most
one hybridization bond per bead) every 10 steps.  Inputs are synthetic and
seeded (synth.c3).

One step = one pass of the whole hot path (cell-list upkeep, fused force +
integrate kernel, and on every 10th step the sweep).  Prints one JSON line.
``value`` is the mixed-precision path (FP32 force arithmetic, FP64 positions,
differences, accumulation and integration); the plain FP64 path is measured in
the same run and reported under ``fp64``.
"""
import argparse
import json
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_EVERY = 7

# HBM traffic of the step kernel from hardware counters (rocprofv3 --pmc FETCH_SIZE,
# then WRITE_SIZE), recorded with a hash of the kernel sources it was taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_c3_1M_traffic.txt")
KERNEL_SOURCES = ["kernels_force.hip", "cell_scan.h", "db_device.h", "db_internal.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1108_4214_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_counters():
    """the counter record of the step kernel (key -> text), or None if absent or taken on other sources"""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return kv


def recorded_traffic():
    """bytes per launch from the counters, or None if absent or taken on other sources"""
    kv = recorded_counters()
    return float(kv["traffic_bytes_per_launch"]) if kv else None


# VALU issue of the chip: 256 CUs x 4 SIMDs, one wavefront instruction of 64 lanes per
# 4 cycles on a 16-lane SIMD, at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4.0   # wavefront instructions per second


def valu_issue_frac(launch_us):
    """share of the chip's VALU issue the step kernel uses: its VALU instruction count
    per launch (SQ_INSTS_VALU, recorded with the traffic) over the live launch time"""
    kv = recorded_counters()
    if not kv or "valu_insts_per_launch" not in kv or not launch_us > 0:
        return None
    return float(kv["valu_insts_per_launch"]) / (launch_us * 1e-6) / VALU_ISSUE_PEAK


def copy_probe():
    """a plain device copy of 256 MiB, three times: the reference that scales the
    FETCH_SIZE / WRITE_SIZE counters"""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def algorithmic_bytes_per_bead_step(b, a, d, every):
    """Bytes the method must move per bead and step: position and velocity read and
    written in FP64 (96), the bead type (1), one read of every bond (2 ids + 2 types,
    10 B), angle (3 ids + type, 13 B) and dihedral (4 ids + type, 17 B) counted once,
    plus the sweep's read of positions, types, counts and bonds amortised over its
    interval."""
    per_step = 97.0 + 10.0 * b + 13.0 * a + 17.0 * d
    sweep = (25.0 + 10.0 * b) / every if every > 0 else 0.0
    return per_step, per_step + sweep


def run_gpu(w, precision, steps, warmup, skin=None, permute_every=None):
    import torch

    import paper_1108_4214_amd as pk

    s = w.system
    g = pk.System(s.n, s.L, w.seed, precision)
    if skin is not None:
        pk.db_tune(g.ctx, skin, permute_every or 1)
    g.configure(s, w.ff, w.rules)
    g.step(warmup)
    torch.cuda.synchronize()
    pk.db_step_kernel_time(g.ctx)          # reset the tally
    # events around every 7th step launch: each event pair idles the GPU for a few
    # microseconds, and 7 is prime to the usual block lengths
    pk.db_profile(g.ctx, PROFILE_EVERY)
    st0 = g.stats()
    # the timed steps in five equal chunks (each a multiple of the sweep cadence for
    # the default 1,000 steps, so the blocks are the same), each timed too: the
    # median of the five is reported beside the whole
    nchunk = 5 if steps >= 5 else 1
    sizes = [steps // nchunk] * nchunk
    sizes[-1] += steps - sum(sizes)
    chunk_rates = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in sizes:
        tc = time.perf_counter()
        g.step(k)
        torch.cuda.synchronize()
        chunk_rates.append(s.n * k / (time.perf_counter() - tc))
    t1 = time.perf_counter()
    pk.db_profile(g.ctx, 0)
    kern_us, launches = pk.db_step_kernel_time(g.ctx)
    st1 = g.stats()
    tiles = pk.db_tile_stats(g.ctx)
    nb, na, nd = g.counts()
    out = {
        "seconds": t1 - t0,
        "bead_steps_per_s": s.n * steps / (t1 - t0),
        "chunk_bead_steps_per_s": chunk_rates,
        "median_of_chunks": statistics.median(chunk_rates),
        "ms_per_step": 1e3 * (t1 - t0) / steps,
        "step_kernel_us": kern_us,
        "step_kernel_launches": launches,
        "sweeps": st1["sweeps"] - st0["sweeps"],
        "rebuilds": st1["rebuilds"] - st0["rebuilds"],
        "rollbacks": st1["rollbacks"] - st0["rollbacks"],
        "bonds_created": st1["cum_bonds_created"] - st0["cum_bonds_created"],
        "bonds_killed": st1["cum_bonds_killed"] - st0["cum_bonds_killed"],
        "bonds_broken": st1["cum_bonds_broken"] - st0["cum_bonds_broken"],
        "bonds_converted": st1["cum_bonds_converted"] - st0["cum_bonds_converted"],
        "topology_per_bead": [nb / s.n, na / s.n, nd / s.n],
        "tiles": tiles,
    }
    g.close()
    return out


def run_batch(steps, warmup, precision=1):
    """The replica ladder: 64 uneven replicas advanced together (one launch per
    kernel for all of them) against the same replicas stepped one after another;
    the batch with its blocks' step launches replayed from HIP graphs; and the batch
    after the autotuner (skin, reorder cadence, kernel shape, graphs)."""
    import torch

    import paper_1108_4214_amd as pk
    import synth

    ws = synth.c4()

    def replicas():
        return [pk.System(w.system.n, w.system.L, w.seed, precision).configure(w.system, w.ff, w.rules) for w in ws]

    def timed(g, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(k)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    reps = replicas()
    ntot = sum(g.n for g in reps)
    b = pk.Batch(reps)
    for g in reps:
        g.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in reps:
        g.step(steps)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    b.step(warmup)
    bat_s = timed(b, steps)
    b.close()
    out = {}
    for label, graph in (("graph", 1),):
        bg = pk.Batch(reps)
        pk.db_graph(bg.ctx, graph)
        bg.step(warmup)
        t = timed(bg, steps)
        out[label] = {"value": ntot * steps / t, "ms_per_step": 1e3 * t / steps}
        bg.close()
    bt = pk.Batch(reps)
    skin, perm = pk.db_autotune(bt.ctx, 40)
    shape = pk.db_get_shape(bt.ctx)
    t = timed(bt, steps)
    out["tuned"] = {"value": ntot * steps / t, "ms_per_step": 1e3 * t / steps, "skin": skin,
                    "permute_every": perm, **shape}
    bt.close()
    for g in reps:
        g.close()
    return {"workload": f"{len(ws)} replicas of 2k-50k beads (log-uniform), {ntot} beads, duplexes at rho=0.5, "
                        "T_r = 0.6 + 0.8 r/63, sweep every 10 steps",
            "beads": ntot, "replicas": len(ws), "steps": steps,
            "value": ntot * steps / bat_s, "unit": "bead-steps/s", "ms_per_step": 1e3 * bat_s / steps,
            "sequential_value": ntot * steps / seq_s, "sequential_ms_per_step": 1e3 * seq_s / steps,
            "speedup": seq_s / bat_s, **out}


def run_small(steps, warmup):
    """Launch-bound sizes: the 40-bead pair of 10-nt strands and the 80,000-bead box,
    mixed precision, launches one by one against blocks replayed from HIP graphs."""
    import torch

    import paper_1108_4214_amd as pk
    import synth

    res = {}
    for name, w in (("40 beads", synth.c1()), ("80000 beads", synth.c2())):
        r = {}
        for graph in (0, 1):
            g = pk.System(w.system.n, w.system.L, w.seed, 1)
            pk.db_graph(g.ctx, graph)
            g.configure(w.system, w.ff, w.rules)
            g.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            r["graph" if graph else "launches"] = {"value": w.system.n * steps / t, "ms_per_step": 1e3 * t / steps}
            g.close()
        res[name] = r
    return res


def run_leg(w, description, steps, warmup):
    """One more workload, mixed and FP64, reported beside the headline."""
    mixed = run_gpu(w, 1, steps, warmup)
    fp64 = run_gpu(w, 0, steps, warmup)
    b, a, d = mixed["topology_per_bead"]
    kernel_bytes, step_bytes = algorithmic_bytes_per_bead_step(b, a, d, w.rules.every)
    n = w.system.n

    def frac(r):
        return kernel_bytes * n / (r["step_kernel_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS if r["step_kernel_us"] > 0 else None

    return {"workload": description, "value": mixed["bead_steps_per_s"], "unit": "bead-steps/s",
            "ms_per_step": mixed["ms_per_step"], "step_kernel_us": mixed["step_kernel_us"],
            "hbm_roofline_frac": frac(mixed), "bytes_per_bead_step": kernel_bytes,
            "path_roofline_frac": step_bytes * mixed["bead_steps_per_s"] / (HBM_PEAK_GBS * 1e9),
            "fp64": {"value": fp64["bead_steps_per_s"], "ms_per_step": fp64["ms_per_step"],
                     "step_kernel_us": fp64["step_kernel_us"], "hbm_roofline_frac": frac(fp64),
                     "path_roofline_frac": step_bytes * fp64["bead_steps_per_s"] / (HBM_PEAK_GBS * 1e9)},
            "mixed_detail": mixed, "fp64_detail": fp64}


def run_c5(steps, warmup):
    """The stress workload: 4,000,000 beads at density 0.85, a sweep before every
    step (creation at p = 0.9, conversion of stretched hybridization bonds to the
    weak type, kills), NVE at dt = 0.002.  Every timed step does topology work.  The
    run stays within 200 steps of the lattice start: with the angle and dihedral
    patterns, strained rungs reach near-collinear dihedrals after about 550 steps."""
    import synth

    steps, warmup = min(steps, 150), min(warmup, 50)
    return run_leg(synth.c5(), "100000 x 20-nt random strands, 2-bead model, 4000000 beads, rho=0.85, sweep every "
                   "step (create p=0.9, convert hybridization->weak beyond 1.8, kill), NVE dt=0.002, "
                   f"steps {warmup + 1}..{warmup + steps} from the lattice start", steps, warmup)


def run_dpd(steps, warmup):
    """The paper's own dynamics (section 3): DPD conservative, dissipative and
    random pair forces at density 3 with the hybridization sweep."""
    import synth

    return run_leg(synth.dpd_c3(), "2500 x 20-bp duplexes (2-bead model, 200000 beads) in 800000 DPD solvent beads, "
                   "1000000 beads, rho=3, a=25, gamma=100, T=1, dt=0.01, sweep every 10 steps", steps, warmup)


def run_dna1(steps, warmup):
    """The paper's 1-bead DNA model (section 3 wells, angles and stacking
    dihedrals; Fig. 2 rule table, a sweep every step) in DPD solvent."""
    import synth

    return run_leg(synth.dna1_c3(), "5000 x 20-bp duplexes of the paper's 1-bead model (200000 beads) in 800000 "
                   "DPD solvent beads, 1000000 beads, rho=3, Fig. 2 rules (sweep every step, paircheck14), "
                   "section 3 wells, angles and dihedrals, DPD a=25, gamma=100, T=1, dt=0.01", steps, warmup)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_accuracy(ramp_steps=100000, ramp_every=5000, nve_steps=10000, nve_every=1000, warm_steps=2000):
    """Mixed precision against FP64 on the GPU: force error on the 80,000-bead case, the
    hybridized fraction along the whole 1M-bead temperature ramp, and NVE energy drift
    on the 4M-bead stress case (energy minus the topology-energy ledger, which takes
    out the jumps of bond events)."""
    import numpy as np
    import torch

    import paper_1108_4214_amd as pk
    import synth

    out = {}
    w = synth.c2()
    f = {}
    for prec in (0, 1):
        g = pk.System(w.system.n, w.system.L, w.seed, prec).configure(w.system, w.ff, w.rules)
        f[prec] = g.forces()
        g.close()
    out["c2_force_rel_l2_mixed_vs_fp64"] = float(np.linalg.norm(f[1] - f[0]) / np.linalg.norm(f[0]))
    log(f"accuracy: 80k-bead force error {out['c2_force_rel_l2_mixed_vs_fp64']:.3e}")

    w = synth.c3()
    h0 = int(np.sum(w.system.bonds[:, 2] == synth.H_BOND))
    curves = {}
    for prec in (1, 0):
        g = pk.System(w.system.n, w.system.L, w.seed, prec).configure(w.system, w.ff, w.rules)
        pts = []
        t0 = time.perf_counter()
        for k in range(0, ramp_steps + 1, ramp_every):
            if k:
                g.step(ramp_every)
            st = g.stats()
            nh = h0 + st["cum_bonds_created"] - st["cum_bonds_killed"] - st["cum_bonds_broken"]
            T = w.ff.T0 + (w.ff.T1 - w.ff.T0) * min(k, w.ff.ramp_steps) / w.ff.ramp_steps
            pts.append([k, round(T, 4), nh / h0])
            log(f"accuracy: ramp {'mixed' if prec else 'fp64'} step {k} T {T:.3f} hybridized {nh / h0:.4f}")
        torch.cuda.synchronize()
        curves["mixed" if prec else "fp64"] = {"points": pts, "seconds": time.perf_counter() - t0}
        g.close()
    out["c3_hybridized_fraction"] = {"columns": ["step", "T", "fraction"], **curves}

    w = synth.c5()
    # bond rules only (creation, conversion, kill, maxbond): with the angle and dihedral
    # patterns, the strained rungs formed across the packed lattice drive both paths alike
    # into the near-collinear configurations where the dihedral force diverges (~550 steps)
    rules = synth.RuleSet(every=w.rules.every, rules=[r for r in w.rules.rules if r[0] not in ("angle", "dihedral")])
    s5 = synth.System(L=w.system.L, x=w.system.x, v=w.system.v, type=w.system.type, reactive=w.system.reactive,
                      bonds=w.system.bonds)
    drift = {}
    for prec in (1, 0):
        g = pk.System(s5.n, s5.L, w.seed, prec).configure(s5, w.ff, rules)
        # Langevin warm-up (T = 1, gamma = 1): the first sweeps bond most bases of the
        # lattice and release the strain of the new angles as heat
        pk.db_langevin(g.ctx, 1.0, 1.0, w.ff.dt)
        g.step(warm_steps)
        pk.db_langevin(g.ctx, 1.0, 0.0, w.ff.dt)
        pk.db_track_topology_energy(g.ctx, 1)
        du0 = g.stats()["du_topo_cum"]
        e0 = g.energy()
        c0 = float(np.sum(e0[:5]))
        series = []
        for k in range(nve_every, nve_steps + 1, nve_every):
            g.step(nve_every)
            e = g.energy()
            st = g.stats()
            series.append([k, (float(np.sum(e[:5])) - (st["du_topo_cum"] - du0) - c0) / abs(c0)])
            log(f"accuracy: NVE {'mixed' if prec else 'fp64'} step {k} drift {series[-1][1]:.3e}")
        drift["mixed" if prec else "fp64"] = {"relative_drift": series,
                                              "bonds_created": g.stats()["cum_bonds_created"],
                                              "bonds_converted": g.stats()["cum_bonds_converted"]}
        g.close()
    out["c5_nve_drift"] = {"columns": ["step", "(E - E0 - dU_topo) / |E0|"], "dt": w.ff.dt,
                           "rules": "bond rules of the stress case (create, convert, kill, maxbond); no angle or "
                                    "dihedral patterns",
                           "warmup": f"{warm_steps} Langevin steps (T = 1, gamma = 1)", **drift}
    return out


def _oracle_shard(args):
    """Worker of the CPU baseline: one single-threaded oracle advancing one shard box
    of the workload; returns (beads, steps, start, end) on the monotonic clock."""
    k, n_shards, steps, barrier = args
    sys.path.insert(0, ROOT)
    import oracle
    import synth
    w = synth.c3_shard(k, n_shards)
    o = oracle.Oracle.from_system(w.system, w.ff, w.rules, seed=w.seed)
    barrier.wait()
    t0 = time.monotonic()
    o.step(steps)
    t1 = time.monotonic()
    return w.system.n, steps, t0, t1


def host_cores():
    """cores this process may run on, capped at the GPU's share of its host (16)"""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(steps):
    """The oracle on all host cores: one single-threaded oracle process per core,
    each advancing its own shard box of the 1M-bead workload's recipe (same density,
    duplexes, force field and rules); throughput = all bead-steps over the span from
    the first start to the last end."""
    import multiprocessing as mp

    cores = host_cores()
    ctx = mp.get_context("spawn")   # the parent holds the GPU: no fork
    with ctx.Manager() as m:
        barrier = m.Barrier(cores)
        with ctx.Pool(cores) as pool:
            res = pool.map(_oracle_shard, [(k, cores, steps, barrier) for k in range(cores)])
    beads = sum(r[0] for r in res)
    span = max(r[3] for r in res) - min(r[2] for r in res)
    cpu_s = sum(r[3] - r[2] for r in res)
    return {"value": beads * steps / span, "unit": "bead-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} single-threaded oracle processes, one per host core, each advancing its own "
                      f"box of {beads // cores} beads (1/{cores} of the 1,000,000-bead recipe: pre-hybridized "
                      f"40-bp duplexes at rho=0.5, same force field and rules) {steps} steps with "
                      f"{steps // 10} sweeps; {beads} beads in all, {span:.1f} s wall, {cpu_s:.1f} s of CPU work"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skin", type=float, default=None)
    ap.add_argument("--permute-every", type=int, default=None)
    ap.add_argument("--no-batch", action="store_true", help="skip the replica-ladder measurement")
    ap.add_argument("--no-dpd", action="store_true", help="skip the DPD-solution measurement")
    ap.add_argument("--no-dna1", action="store_true", help="skip the 1-bead DNA model measurement")
    ap.add_argument("--no-c5", action="store_true", help="skip the 4M-bead stress measurement")
    ap.add_argument("--accuracy", action="store_true",
                    help="also report mixed-vs-FP64 accuracy: force error, hybridized-fraction ramp, NVE drift")
    ap.add_argument("--leg", choices=["dpd", "dna1", "batch", "c5", "small"], default=None,
                    help="run only this extra workload and print its JSON (for profiling it alone)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for the traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (single-GPU build: a large box "
              "would shard by spatial domains, which this build does not run)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.leg is not None:
        legs = {"dpd": lambda: run_dpd(args.steps, args.warmup), "dna1": lambda: run_dna1(args.steps, args.warmup),
                "c5": lambda: run_c5(args.steps, args.warmup),
                "small": lambda: run_small(max(200, args.steps), min(args.warmup, 50)),
                "batch": lambda: run_batch(max(100, args.steps // 4), min(args.warmup, 50))}
        out = legs[args.leg]()
        if args.copy_probe:
            copy_probe()
        print(json.dumps({"leg": args.leg, **out}), flush=True)
        return
    w = synth.c3()
    every = w.rules.every
    mixed = run_gpu(w, 1, args.steps, args.warmup, args.skin, args.permute_every)
    log(f"bench: mixed {mixed['ms_per_step']:.4f} ms/step")
    fp64 = run_gpu(w, 0, args.steps, args.warmup, args.skin, args.permute_every)
    log(f"bench: fp64 {fp64['ms_per_step']:.4f} ms/step")
    b, a, d = mixed["topology_per_bead"]
    kernel_bytes, step_bytes = algorithmic_bytes_per_bead_step(b, a, d, every)
    n = w.system.n
    achieved = kernel_bytes * n / (mixed["step_kernel_us"] * 1e-6) / 1e9 if mixed["step_kernel_us"] > 0 else 0.0
    tb = recorded_traffic()
    # measured HBM bytes per launch over the same live launch time: GB/s, comparable with achieved
    traffic = tb / (mixed["step_kernel_us"] * 1e-6) / 1e9 if (tb is not None and mixed["step_kernel_us"] > 0) else None
    line = {
        "metric": "bead-steps/s at 1M beads incl. bond sweep; mixed vs FP64 on same GPU",
        "value": mixed["bead_steps_per_s"],
        "unit": "bead-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        # the timed steps were also timed in five equal chunks: their median rate
        "median_of_5_chunks": mixed["median_of_chunks"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "12500 x 40-nt strands in 6250 pre-hybridized duplexes, 2-bead model, "
                               "1000000 beads, rho=0.5, T ramp 0.5->1.5 over 1e5 steps, sweep every 10 steps",
                   "beads": n, "sweep_every": every, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_bytes_per_launch": tb,
                     "kernel": "k_step<float> (fused pair + bonded + Langevin + velocity Verlet)",
                     "bytes_per_bead_step": kernel_bytes, "beads_per_launch": n,
                     "launch_us": mixed["step_kernel_us"], "launches_timed": mixed["step_kernel_launches"],
                     # the kernel is bound by VALU issue, not HBM: its share of the chip's issue rate
                     "valu_issue_frac": valu_issue_frac(mixed["step_kernel_us"])},
        "path_roofline_frac": step_bytes * mixed["bead_steps_per_s"] / (HBM_PEAK_GBS * 1e9),
        "fp64": {"value": fp64["bead_steps_per_s"], "ms_per_step": fp64["ms_per_step"],
                 "step_kernel_us": fp64["step_kernel_us"],
                 "roofline_frac": kernel_bytes * n / (fp64["step_kernel_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
                 if fp64["step_kernel_us"] > 0 else None},
        "mixed_detail": mixed,
        "fp64_detail": fp64,
    }
    if args.copy_probe:
        copy_probe()
    if args.accuracy:
        line["accuracy"] = run_accuracy()
    if not args.no_batch:
        line["batch"] = run_batch(max(100, args.steps // 4), min(args.warmup, 50))
        log("bench: replica ladder done")
    if not args.no_dpd:
        line["dpd"] = run_dpd(args.steps, args.warmup)
        log("bench: DPD solution done")
    if not args.no_dna1:
        line["dna1"] = run_dna1(args.steps, args.warmup)
        log("bench: 1-bead model done")
    if not args.no_batch:
        line["small"] = run_small(max(200, args.steps), min(args.warmup, 50))
        log("bench: launch-bound sizes done")
    if not args.no_c5:
        line["c5"] = run_c5(args.steps, args.warmup)
        log("bench: 4M-bead stress case done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_steps)
        log("bench: CPU oracle done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
