"""Benchmark: electron-moves/sec of the particle-by-particle VMC hot path on one GPU.

One step = one sweep (every electron of every walker proposes once, the
orbital gather plus the sequential move chain) followed by the local-energy
measurement of every walker.  With ``--moves all`` a step is one all-electron
move per walker instead of the sweep (throughput still counted in electrons
proposed).  Inputs are seeded synthetic workloads from ``qmc_inputs`` and are
resident in HBM before the timed region starts.

Prints one JSON line (see the keys below).  ``--gpus N`` with N > 1 exits:
this build measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "electron-moves/sec (1 GPU) mixed vs FP64; p50/p99 sweep latency served"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
MFMA_FP32_TFLOPS = 157.3    # MI355X dense FP32 matrix peak
MFMA_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
VALU_FP64_TFLOPS = 78.6     # MI355X FP64 vector peak (256 CUs x 4 SIMDs x 16 FMA lanes x 2 x 2.4 GHz)
# FP64 FLOPs of one orbital's value, gradient and Laplacian at one point: per stencil row (16 of
# them) three z sums of 1 multiply + 3 fused multiply-adds and five accumulations in 6 fused
# multiply-adds, i.e. 33 FLOPs (a multiply-add counts 2)
GATHER_FLOPS_PER_ORBITAL = 16 * (3 * (1 + 2 * 3) + 2 * 6)
BOX_CPU_SHARE = 16          # host threads a one-GPU machine grants a process


def describe(wl) -> str:
    tb = "FP32" if wl.coefs.dtype.itemsize == 4 else "FP64"
    j = []
    if wl.j1:
        j.append("J1")
    if wl.j2:
        j.append("J2 " + wl.j2["kind"])
    if getattr(wl, "j3", None):
        j.append("J3 e-e-I")
    return (f"{wl.name}: {wl.n_elec} electrons ({wl.n_up}+{wl.n_dn}), {wl.n_orb} orbitals on "
            f"{wl.grid[0]}x{wl.grid[1]}x{wl.grid[2]} {tb} B-spline table, {wl.n_ions} ions, "
            f"{'+'.join(j) or 'no Jastrow'}, {wl.n_walkers} walkers, sigma {wl.sigma}, "
            f"{'Ewald Coulomb' if wl.hamiltonian == 'coulomb' else 'kinetic only'}, "
            f"{wl.precision}, " + (("all-electron drift-diffusion moves" if wl.drift else "all-electron moves")
                                   if getattr(wl, "all_electron", False)
                                   else f"delay rank {wl.delay_rank}"))


def source_hash(files) -> str:
    """First 16 hex digits of the SHA-256 of the given repository files, in order: the key that
    ties a committed counter record to the kernel sources it was measured on."""
    m = hashlib.sha256()
    for p in files:
        with open(os.path.join(ROOT, p), "rb") as f:
            m.update(f.read())
    return m.hexdigest()[:16]


def measured_traffic(wl, kernel: str = "gather"):
    """HBM bytes per launch of the gather (or of the move chain, kernel="chain") from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs, scaled by a plain copy's counter readings;
    None where none was taken or once the kernel's sources have changed."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_{wl.name}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if source_hash(d["source_files"]) != d["source_sha256_16"]:
        return None
    return d["traffic_bytes_per_dispatch"]


def host_description():
    """Host cores and CPU model, for the CPU baseline."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "affinity_cpus": affinity}


def cpu_baseline(wl, target_s: float = 12.0):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: one walker per
    thread, as many threads as the process may use on a one-GPU machine (its share of the host)."""
    import oracle
    host = host_description()
    threads = max(1, min(host["affinity_cpus"], BOX_CPU_SHARE))
    osys = oracle.OracleSystem(wl)
    # calibrate with one sweep of one walker per thread
    ids = list(range(threads))
    t0 = time.perf_counter()
    osys.run(ids, 1, measure_every=1, bits=False, threads=threads)
    t1 = time.perf_counter() - t0
    sweeps = max(1, min(400, int(target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    osys.run(ids, sweeps, measure_every=1, bits=False, threads=threads)
    dt = time.perf_counter() - t0
    moves = len(ids) * wl.n_elec * sweeps
    return {"value": moves / dt, "unit": "electron-moves/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(ids)} walkers x {sweeps} sweeps (+ measurement every sweep) of "
                      f"{wl.name}, {moves} moves in {dt:.2f} s, one walker per thread",
            "host": host, "threads_rule": f"min(cpus this process may use, {BOX_CPU_SHARE}): the "
                                          "share of the host a one-GPU box grants"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed384",
                    help="mixed384 (default: the mixed-precision headline, with FP64 beside it) | solid128 | heg14")
    ap.add_argument("--delay", type=int, default=None,
                    help="delay rank K (1 = Sherman-Morrison; 4..64 = delayed updates); "
                         "default: autotuned before the timed region")
    ap.add_argument("--mode", default="single", choices=["single", "batched", "served", "copy", "dmc"],
                    help="single: one system (default); batched: the four uneven systems in fused "
                         "launches; served: a Poisson request stream with continuous batching; copy: "
                         "a plain 1 GiB device copy (x3), the reference for HBM counter readings")
    ap.add_argument("--requests", type=int, default=200, help="served: requests of each trace")
    ap.add_argument("--sweep-scale", type=float, default=0.02, help="served: scale of each request's sweeps")
    ap.add_argument("--no-served", action="store_true",
                    help="single: skip the served block (the 200-arrival trace) of the headline line")
    ap.add_argument("--dmc-every", type=int, default=4,
                    help="served: every k-th request is a DMC run (0: VMC only)")
    ap.add_argument("--no-graph", action="store_true", help="batched/served: no HIP graph replay")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gather-lanes", type=int, default=None,
                    help="gather lanes per proposal, log2 (default: autotuned before the timed region)")
    ap.add_argument("--no-compare", action="store_true",
                    help="mixed384: skip the FP64 runs of the same system beside the mixed one")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--moves", default="pbyp", choices=["pbyp", "all", "drift", "pdrift"],
                    help="single: particle-by-particle sweeps (default), one all-electron move per "
                         "walker per step (plain or drift-diffusion), or particle-by-particle "
                         "drift-diffusion sweeps (pdrift; FP64, the table's values stored in FP64)")
    ap.add_argument("--j3", type=float, default=None,
                    help="single: add a three-body e-e-I Jastrow term of this coefficient scale "
                         "(orders 2 and 2, cutoff L/2) to the workload")
    ap.add_argument("--ae-sigma", type=float, default=None,
                    help="all-electron proposal width (default: the workload's sigma / sqrt(N))")
    ap.add_argument("--pipelined", action="store_true",
                    help="single: pipelined steps (qmc_run_steps: a step's measurement on a side "
                         "stream beside the next step's proposals; the default)")
    ap.add_argument("--serial", action="store_true",
                    help="single: the sweep and measurement calls in turn (every kernel alone; at 384 "
                         "electrons about 2%% fewer moves/s than the pipelined steps, and the gather "
                         "alone instead of beside the measurement)")
    args = ap.parse_args(argv)
    if args.serial and args.pipelined:
        ap.error("--serial and --pipelined exclude each other")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(walkers would be sharded across GPUs with one energy reduction per block).",
              file=sys.stderr)
        return 2

    import torch

    import qmc_inputs as qi
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.mode == "batched":
        return bench_batched(args)
    if args.mode == "served":
        return bench_served(args)
    if args.mode == "copy":
        return copy_reference()
    if args.mode == "dmc":
        return bench_dmc(args)
    wl = qi.WORKLOADS[args.workload]()
    if args.j3 is not None:
        import dataclasses
        wl = dataclasses.replace(wl, j3=qi.j3_params(2, 2, wl.L / 2, wl.seed, A=args.j3))
        args.no_compare = True
    ae = args.moves in ("all", "drift")
    if ae:
        # one move displaces all N electrons: a width sigma / sqrt(N) keeps the mean squared
        # displacement of the walker that of one particle-by-particle move
        import dataclasses
        import math
        wl = dataclasses.replace(wl, all_electron=True, drift=args.moves == "drift",
                                 sigma=args.ae_sigma or wl.sigma / math.sqrt(wl.n_elec))
        args.no_compare = True
    pdrift = args.moves == "pdrift"
    if pdrift:
        import dataclasses

        import numpy as np
        wl = dataclasses.replace(wl, drift=True, precision="fp64", coefs=np.asarray(wl.coefs, dtype=np.float64),
                                 delay_rank=1, recompute_period=0, name=wl.name.replace("_mixed", "") + "_pdrift")
        args.no_compare = True
        args.delay = 1
        args.gather_lanes = -1
    r = run_single(wl, args.steps, args.warmup, args.delay, args.gather_lanes, serial=args.serial)
    if r["delay_rank"] is not None:
        wl.delay_rank = r["delay_rank"]
    W, N = r["walkers"], wl.n_elec
    kt = r["kt"]
    g_ms, g_n = kt["chain"] if pdrift else kt["gather"]   # drift sweeps read the table inside the chain
    avg_gather_s = g_ms / max(g_n, 1) / 1e3
    launches = ("alone (sweep and measurement calls in turn)" if args.serial else
                "beside the previous step's local-energy kernels (--pipelined: shared compute units)")
    g_roof = gather_roofline(wl, W, N, avg_gather_s,
                             ("k_chain_drift (the whole sweep: the table reads of every move's row happen "
                              "inside the chain, which is latency-bound)") if pdrift else
                             "k_gather_ordered (tricubic B-spline VGL of every orbital at every proposal, "
                             "in table order) with k_propose and the bucket sort", launches)
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "electron-moves/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": describe(wl), "walkers": W, "electrons": N, "orbitals": wl.n_orb,
                   "grid": list(wl.grid), "delay_rank": r["delay_rank"],
                   "gather_lanes_log2": r["gather_lanes_log2"],
                   "step": (f"1 all-electron {'drift-diffusion ' if wl.drift else ''}move per walker "
                            "(N electrons proposed at once, FP64 determinants at R') + local energy")
                           if ae else
                           ("1 drift-diffusion sweep (N moves per walker, each row evaluated in the chain) "
                            "+ local energy" if pdrift else "1 sweep (N moves per walker) + local energy"),
                   "steps_run": "sweep and measurement calls in turn" if args.serial else
                   "pipelined (a step's measurement beside the next step's proposals)"},
        "roofline": g_roof,
        "kernels_ms_per_step": {k: v[0] / r["steps"] for k, v in kt.items()},
        "kernels_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
        "rebuilds_in_timed_steps": r["rebuilds"],
        "acceptance_last_step": r["acceptance"],
        "sweep_only_moves_per_s": r["sweep_only_moves_per_s"],
        "mean_local_energy": r["mean_local_energy"],
    }
    line["roofline_gather"] = g_roof
    if not ae and not pdrift:
        # the dominant kernel of the timed steps takes the roofline entry
        line["roofline_chain"] = chain_roofline(wl, r)
        if kt["chain"][0] > kt["gather"][0]:
            line["roofline"] = dict(line["roofline_chain"], dominant="move chain: the longest kernel of a step")
    headline = args.workload == "mixed384" and wl.precision == "mixed" and not ae and args.j3 is None
    if headline and not args.no_compare:
        line.update(fp64_beside(wl, r, serial=args.serial))
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    if headline and not args.no_served:
        line["served"] = served_block(args)
    print(json.dumps(line), flush=True)
    return 0


def run_single(wl, steps: int, warmup: int, delay, lanes=None, serial: bool = False):
    """Steps of (sweep + local energy) of one system; the delay rank is autotuned when not given
    (the trial sweeps are ordinary sweeps, before the timed region)."""
    import torch

    from paper_1802_06922_amd import KERNEL_CHAIN, KERNEL_GATHER, KERNEL_MEASURE, KERNEL_REBUILD, System
    if wl.recompute_period > 0 and steps % wl.recompute_period and not wl.all_electron:
        # the timed window holds whole rebuild periods, so it pays for every FP64 rebuild
        steps = (steps // wl.recompute_period + 1) * wl.recompute_period
    if delay is not None:
        wl.delay_rank = delay
    print(f"[bench] building {wl.name}", file=sys.stderr, flush=True)
    s = System(wl)
    if lanes is None:
        lanes_log2, _ = s.autotune_gather(trial_sweeps=3)
    else:
        s.set_gather_lanes(lanes)
        lanes_log2 = lanes
    if wl.all_electron:
        K = None   # no update chain: every accepted move installs fresh inverses
    elif delay is None:
        K, _ = s.autotune_delay(ranks=(1, 8, 16, 32, 64), trial_sweeps=3)
        print(f"[bench] {wl.name}: delay rank {K}, gather lanes 2^{lanes_log2} (autotuned)",
              file=sys.stderr, flush=True)
    else:
        K = delay
    W, N = s.W, wl.n_elec
    # every step's energies stay on the device; steps run pipelined (qmc_run_steps: a step's
    # measurement beside the next step's proposals)
    energies = torch.empty((max(steps, warmup, 1), W, 4), dtype=torch.float64, device="cuda")
    def run(n, out):
        if serial:
            for k in range(n):
                s.sweep(1)
                s.measure(out=out[k])
        else:
            s.run_steps(n, out)

    if warmup:
        run(warmup, energies[:warmup])
    torch.cuda.synchronize()
    s.set_timing(True)
    for k in (KERNEL_GATHER, KERNEL_CHAIN, KERNEL_MEASURE, KERNEL_REBUILD):
        s.kernel_timing(k, reset=True)
    print(f"[bench] {wl.name}: timing {steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps, energies[:steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = {name: s.kernel_timing(k) for name, k in
          (("gather", KERNEL_GATHER), ("chain", KERNEL_CHAIN), ("measure", KERNEL_MEASURE))}
    rebuild = s.kernel_timing(KERNEL_REBUILD)
    e_host = energies[steps - 1].cpu().numpy()
    acceptance = float(s.accept_log().mean())
    pos_host = s.get_walkers()[0]
    s.close()
    moves = W * N * steps
    sweep_ms = (kt["gather"][0] + kt["chain"][0]) / steps
    return {"value": moves / dt, "ms_per_step": dt / steps * 1e3, "kt": kt, "walkers": W, "steps": steps,
            "rebuilds": {"launches": rebuild[1], "ms_per_launch": rebuild[0] / max(rebuild[1], 1)},
            "delay_rank": K, "gather_lanes_log2": lanes_log2, "acceptance": acceptance, "sweep_only_moves_per_s": moves / (sweep_ms * steps / 1e3) if sweep_ms > 0 else None,
            "mean_local_energy": float(e_host.sum(axis=1).mean()), "energies": e_host, "positions": pos_host}


def gather_roofline(wl, W, N, avg_s, kernel, launches=None):
    """The gather against the FP64 vector peak.  Evaluated in table order, its table reads are
    served by the caches (the HBM fetch per launch is a small fraction of the table bytes it
    reads), and the FP64 sums of every orbital set its pace: algorithmic FLOPs per launch =
    GATHER_FLOPS_PER_ORBITAL x n_orb x W N.  The table bytes each launch reads (64 n_orb b per
    proposal) are reported beside, with their rate and the measured HBM traffic."""
    b = wl.coefs.dtype.itemsize
    flops = float(GATHER_FLOPS_PER_ORBITAL) * wl.n_orb * W * N
    table_bytes = 64 * wl.n_orb * b * W * N
    achieved = flops / avg_s / 1e12 if avg_s > 0 else 0.0
    out = {"bound": "alu", "achieved": achieved, "peak": VALU_FP64_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved / VALU_FP64_TFLOPS, "traffic": measured_traffic(wl), "kernel": kernel,
           "flops_per_launch": flops, "avg_launch_ms": avg_s * 1e3,
           "table_bytes_per_launch": table_bytes,
           "table_read_rate_GBs": table_bytes / avg_s / 1e9 if avg_s > 0 else 0.0,
           "hbm_peak_GBs": HBM_PEAK_GBS}
    if launches:
        out["launches"] = launches
    return out


def chain_roofline(wl, r):
    """The move chain against the matrix-core peak of its precision.  Its matrix-core work per
    launch: per walker and spin block of n electrons, the window products Y = V B0 (2 n^3 over
    a sweep) and the rank-m flushes (2 n^2 per accepted move), i.e. 2 W sum_spin n^3 (1 + a) at
    acceptance a; the inverse itself moves 2 n^2 b bytes per spin and walker when the chain
    keeps it on chip for the sweep (read once, written once), and the proposals' value rows
    n^2 b more."""
    kt = r["kt"]
    c_ms, c_n = kt["chain"]
    avg_s = c_ms / max(c_n, 1) / 1e3
    W, a = r["walkers"], r["acceptance"]
    b = wl.coefs.dtype.itemsize
    n3 = wl.n_up ** 3 + wl.n_dn ** 3
    flops = 2.0 * W * n3 * (1.0 + a) if r["delay_rank"] and r["delay_rank"] > 1 else 0.0
    peak = MFMA_FP32_TFLOPS if b == 4 else MFMA_FP64_TFLOPS
    achieved = flops / avg_s / 1e12 if avg_s > 0 else 0.0
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": measured_traffic(wl, "chain"),
            "kernel": "move chain (ratios, Jastrow, decisions, delayed-update products)",
            "flops_per_launch": flops, "avg_launch_ms": avg_s * 1e3, "delay_rank": r["delay_rank"],
            "inverse_bytes_per_launch": 2 * W * (wl.n_up ** 2 + wl.n_dn ** 2) * b,
            "row_bytes_per_launch": W * (wl.n_up ** 2 + wl.n_dn ** 2) * b,
            "note": "sequential per walker (each move depends on the previous decision): the matrix "
                    "cores are busy only in the window products and flushes"}


def fp64_beside(mixed_wl, rm, agree_sweeps: int = 8, serial: bool = True):
    """The same 384-electron system in FP64 (the FP32-valued table stored in FP64, FP64 updates,
    no guard) with its autotuned delay rank, and the plain FP64 sweep (Sherman-Morrison, rank 1),
    for as many steps as the mixed run.  Then the agreement of the two precisions: fresh mixed
    and FP64 systems (same seeds) run sweep for sweep with a measurement after each; the mixed
    path must take the FP64 decisions, and its local energies are compared one to one."""
    import dataclasses

    import numpy as np

    from paper_1802_06922_amd import System
    steps = rm["steps"]
    fp64 = dataclasses.replace(mixed_wl, precision="fp64", coefs=mixed_wl.coefs.astype(np.float64),
                               recompute_period=0, name="solid384_fp64")
    plain = dataclasses.replace(fp64, name="solid384_fp64_plain")
    out = {}
    for tag, wl, K in (("fp64", fp64, None), ("fp64_plain", plain, 1)):
        r = run_single(wl, steps, 1, K, serial=serial)
        out[tag] = {"moves_per_s": r["value"], "ms_per_step": r["ms_per_step"], "delay_rank": r["delay_rank"],
                    "steps": r["steps"],
                    "kernels_ms_per_step": {k: v[0] / r["steps"] for k, v in r["kt"].items()}}
    out["mixed_over_fp64"] = rm["value"] / out["fp64"]["moves_per_s"]
    out["mixed_over_fp64_plain"] = rm["value"] / out["fp64_plain"]["moves_per_s"]
    print(f"[bench] mixed vs FP64 agreement: {agree_sweeps} sweeps of both", file=sys.stderr, flush=True)
    sm, sf = System(mixed_wl), System(dataclasses.replace(fp64, delay_rank=16))
    same, rel = True, []
    for _ in range(agree_sweeps):
        sm.sweep(1)
        sf.sweep(1)
        same = same and bool(np.array_equal(sm.accept_log(), sf.accept_log()))
        em, ef = sm.measure(), sf.measure()
        rel.append(np.abs(em - ef) / np.maximum(np.abs(ef), 1.0))
    sm.close()
    sf.close()
    rel = np.concatenate(rel)
    out["mixed_vs_fp64_agreement"] = {
        "sweeps": agree_sweeps, "same_decisions": same,
        "components": "kinetic, e-e, e-I, I-I of every walker after every sweep",
        "max_rel_energy_difference": float(rel.max()), "p99": float(np.percentile(rel, 99)),
        "median": float(np.median(rel))}
    return out


def bench_dmc(args) -> int:
    """Diffusion Monte Carlo steps (drift-diffusion all-electron move of every slot, local
    energies, branching on the device) on the workload's walker slots; value = electrons of
    the walkers alive at each step, per second."""
    import dataclasses
    import math

    import torch

    import qmc_inputs as qi
    from paper_1802_06922_amd import KERNEL_CHAIN, KERNEL_GATHER, KERNEL_MEASURE, KERNEL_REBUILD, System
    wl = qi.WORKLOADS[args.workload]()
    wl = dataclasses.replace(wl, all_electron=True, drift=True,
                             sigma=args.ae_sigma or wl.sigma / math.sqrt(wl.n_elec))
    print(f"[bench] building {wl.name} (DMC)", file=sys.stderr, flush=True)
    s = System(wl)
    if args.gather_lanes is None:
        lanes_log2, _ = s.autotune_gather(trial_sweeps=3)
    else:
        s.set_gather_lanes(args.gather_lanes)
        lanes_log2 = args.gather_lanes
    W, N = s.W, wl.n_elec
    target = W * 7 // 8
    s.dmc_init(target, feedback=1.0)
    stats = torch.zeros((max(args.steps, args.warmup, 1), 6), dtype=torch.float64, device="cuda")
    if args.warmup:
        s.dmc_steps(args.warmup, stats[:args.warmup])
    torch.cuda.synchronize()
    _, _, _, pop0 = s.dmc_state()
    s.set_timing(True)
    for k in (KERNEL_GATHER, KERNEL_CHAIN, KERNEL_MEASURE, KERNEL_REBUILD):
        s.kernel_timing(k, reset=True)
    print(f"[bench] {wl.name}: timing {args.steps} DMC steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.dmc_steps(args.steps, stats[:args.steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = {name: s.kernel_timing(k) for name, k in
          (("gather", KERNEL_GATHER), ("move", KERNEL_CHAIN), ("measure", KERNEL_MEASURE),
           ("branch", KERNEL_REBUILD))}
    st = stats[:args.steps].cpu().numpy()
    s.close()
    moved = pop0 + st[:-1, 2].sum()   # walkers alive at the start of each timed step
    g_ms, g_n = kt["gather"]
    avg_gather_s = g_ms / max(g_n, 1) / 1e3
    line = {
        "metric": METRIC + "; DMC mode",
        "value": moved * N / dt,
        "unit": "electron-moves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if wl.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": describe(wl), "slots": W, "target_population": target, "electrons": N,
                   "tau": wl.sigma ** 2, "feedback_hartree": 1.0, "gather_lanes_log2": lanes_log2,
                   "step": "1 DMC step: drift-diffusion all-electron move of every slot (fixed node), "
                           "local energies, weights, branching and copies on the device"},
        "roofline": gather_roofline(wl, W, N, avg_gather_s,
                                    "k_gather_ordered (tricubic B-spline VGL of every orbital at every "
                                    "proposal, in table order) with k_propose and the bucket sort"),
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "population": {"start": pop0, "min": float(st[:, 2].min()), "max": float(st[:, 2].max())},
        "mixed_estimate_last": float(st[-1, 0]),
        "dropped_copies": float(st[:, 4].sum()),
        "node_crossings_rejected": float(st[:, 5].sum()),
    }
    print(json.dumps(line), flush=True)
    return 0


def copy_reference() -> int:
    """A plain device copy of known size: each of the three copies reads and writes 1 GiB."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_per_copy": n * 4, "copies": 3}), flush=True)
    return 0


def bench_batched(args) -> int:
    """Four uneven FP32 systems (32/96/192/512 electrons, grids 24..64^3, 256 walkers each),
    delay rank autotuned per system, advanced together by fused launches replayed as a graph."""
    import torch

    import qmc_inputs as qi
    from paper_1802_06922_amd import Batch, System

    wls = qi.batched_systems(n_walkers=256)
    systems, tuned = [], []
    for wl in wls:
        print(f"[bench] building {wl.name}", file=sys.stderr, flush=True)
        s = System(wl)
        tl, gms = s.autotune_gather(trial_sweeps=3)
        K, ms = s.autotune_delay(ranks=(8, 16, 32, 64), trial_sweeps=3)
        tuned.append({"system": wl.name, "delay_rank": K, "chain_ms": ms, "gather_lanes_log2": tl,
                      "gather_ms": gms})
        systems.append(s)
    b = Batch(systems, graph=not args.no_graph)
    for _ in range(args.warmup):
        b.sweep(1, measure=True)
    b.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(args.steps, measure=True)
    gpu_ms, n = b.timing(reset=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    moves = sum(wl.n_walkers * wl.n_elec for wl in wls) * args.steps
    b.close()
    table_bytes = sum(64 * wl.n_orb * 4 * wl.n_walkers * wl.n_elec for wl in wls)
    line = {
        "metric": METRIC, "value": moves / dt, "unit": "electron-moves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "four uneven solid-like systems (32/96/192/512 electrons, grids "
                               "24/32/48/64^3 FP32, 256 walkers each) in fused launches"
                               + ("" if args.no_graph else ", sweeps replayed as a HIP graph"),
                   "tuned": tuned, "step": "1 sweep of every system + local energies"},
        "gpu_ms_per_step": gpu_ms / max(n, 1),
        "spline_bytes_per_step": table_bytes,
        "spline_hbm_fraction_of_step": table_bytes / (gpu_ms / max(n, 1) / 1e3) / 1e9 / HBM_PEAK_GBS,
    }
    print(json.dumps(line), flush=True)
    return 0


def served_block(args):
    """Served request streams: Poisson arrivals of requests with electron counts log-uniform in
    [32, 1024], grids 32..64^3, 64..1024 walkers, 100..1000 sweeps scaled by --sweep-scale, each
    with its own table; every --dmc-every-th request is a DMC run (as many steps), the others VMC
    runs.  First at 20 requests/s (far above one GPU's capacity), then at 0.8 x the capacity
    measured in that run; p50/p99 per-sweep latency for both, throughput of each."""
    import dataclasses

    import qmc_inputs as qi
    from paper_1802_06922_amd import serve

    log = lambda m: print(m, file=sys.stderr, flush=True)
    print(f"[bench] served: {args.requests} requests, sweeps x{args.sweep_scale}", file=sys.stderr, flush=True)
    trace = qi.served_trace(n_requests=args.requests, rate_per_s=20.0, seed=0)
    reqs = serve.build_requests(trace, sweep_scale=args.sweep_scale, table_pool=True, log=None,
                                dmc_every=args.dmc_every)
    srv = serve.Server(graph=not args.no_graph)
    st = srv.run(reqs, log=None)
    print(f"[bench] served at 20/s: {st['requests']} requests in {st['wall_s']:.1f} s", file=sys.stderr, flush=True)
    capacity = st["requests"] / st["wall_s"]
    # the same requests again, arriving at 0.8 x the measured capacity
    rate = 0.8 * capacity
    slow = qi.served_trace(n_requests=args.requests, rate_per_s=rate, seed=0)
    reqs2 = [dataclasses.replace(r, arrival_s=e["arrival_s"], system=None, done_sweeps=0, latencies_ms=[],
                                 gpu_ms=[], energy=None, final_pos=None, stats=None, stream=None, status="queued",
                                 error="")
             for r, e in zip(sorted(reqs, key=lambda r: r.rid), slow)]
    st2 = srv.run(reqs2, log=None)
    print(f"[bench] served at {rate:.2f}/s: {st2['requests']} requests in {st2['wall_s']:.1f} s", file=sys.stderr,
          flush=True)
    return {
        "workload": f"served stream: {args.requests} Poisson arrivals, N log-uniform [32, 1024], grids "
                    f"32..64^3, 64..1024 walkers, 100..1000 sweeps x{args.sweep_scale}, each request its own "
                    "FP32 table" + (f", every {args.dmc_every}th request a DMC run" if args.dmc_every else ""),
        "hbm_budget_bytes": srv.budget, "dmc_requests": st["dmc_requests"],
        "overload_20_per_s": {"p50_sweep_latency_ms": st["p50_sweep_ms"], "p99_sweep_latency_ms": st["p99_sweep_ms"],
                              "moves_per_s": st["moves_per_s"], "requests": st["requests"],
                              "rejected": st["rejected"], "failed": st["failed"], "wall_s": st["wall_s"],
                              "mean_queue_s": st["mean_queue_s"], "capacity_requests_per_s": capacity},
        "at_0.8_capacity": {"rate_per_s": rate, "p50_sweep_latency_ms": st2["p50_sweep_ms"],
                            "p99_sweep_latency_ms": st2["p99_sweep_ms"], "moves_per_s": st2["moves_per_s"],
                            "requests": st2["requests"], "wall_s": st2["wall_s"],
                            "mean_queue_s": st2["mean_queue_s"]},
    }


def bench_served(args) -> int:
    """The served streams alone (--mode served): value = aggregate electron-moves/s at 20/s."""
    sv = served_block(args)
    st = sv["overload_20_per_s"]
    line = {
        "metric": METRIC, "value": st["moves_per_s"], "unit": "electron-moves/s", "n_gpus": 1,
        "steps": st["requests"], "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic", "config": {"workload": sv["workload"]}, "served": sv,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
