"""Serving loop: continuous batching of VMC and DMC requests on one GPU.

Requests (each a VMC run, or a DMC run, with its own system, table, walker
count and sweep or step count) arrive on a trace.  A request is admitted as soon as its device memory
(``qmc_estimate_device_bytes``) fits the HBM budget next to the requests
already resident; its walkers, inverses and table then stay on the GPU until
it finishes.  Every iteration advances all resident requests by one sweep
with one fused batch launch (``qmc_batch_*``), so requests that arrive while
others run join at the next sweep boundary and their work overlaps on the
device.  A DMC request (drift-diffusion all-electron moves, branching on the
device) advances one step per iteration on its own stream, issued before the
fused VMC sweep so that the two overlap.  A request's results do not depend on
which other requests share the GPU: every walker runs the same per-walker
arithmetic in any batch, and a DMC population is private to its request.

Per-sweep latency of a request = wall time between its consecutive sweep
completions (the first one counted from its admission), so host work between
sweeps (admission, batch rebuild) is included; p50/p99 are pooled over all
(request, sweep) pairs.  The GPU time of each batch sweep (HIP events) is kept
beside it.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import time
from collections import deque
from typing import Optional

import numpy as np

from . import qmc


def delay_rank_for(wl, cap: int = 32) -> int:
    """Delay rank of a request: the largest one (at most ``cap``) whose chain fits one workgroup's
    LDS.  It depends on the system only, so a request computes the same alone and in any mix."""
    return min(cap, qmc.max_delay_rank(wl))


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    wl: object
    n_sweeps: int
    est_bytes: int = 0
    system: Optional[object] = None
    done_sweeps: int = 0
    admitted_s: float = 0.0
    finished_s: float = 0.0
    latencies_ms: list = dataclasses.field(default_factory=list)
    gpu_ms: list = dataclasses.field(default_factory=list)
    last_done_s: float = 0.0
    energy: Optional[np.ndarray] = None   # VMC: last energies [W][4]; DMC: per-step statistics [steps][6]
    final_pos: Optional[np.ndarray] = None
    kind: str = "vmc"                     # "vmc" or "dmc" (the workload makes drift-diffusion moves)
    dmc_target: int = 0                   # DMC: target population (slots alive at the start)
    dmc_feedback: float = 1.0             # DMC: E_T feedback constant (hartree)
    stats: Optional[object] = None        # DMC: device tensor [steps][6] of per-step statistics
    stream: Optional[object] = None       # DMC: the request's own stream
    table_fn: Optional[object] = None     # makes the request's table when it is prepared (wl.coefs None)
    status: str = "queued"                # "done"; "rejected" (can never fit the budget); "failed"
    error: str = ""                       # why a request was rejected or failed


class Server:
    """Continuous batching on one GPU.  Admitted requests are prepared (device allocation, table
    upload, walker initialisation) by host threads on their own stream while the resident
    requests keep sweeping; a prepared request joins the batch at the next sweep boundary."""

    def __init__(self, hbm_budget_bytes: Optional[int] = None, reserve_bytes: int = 8 << 30,
                 graph: bool = False, prep_threads: int = 2):
        import torch
        self.torch = torch
        gpu = torch.cuda.is_available()
        budget = torch.cuda.mem_get_info()[0] - reserve_bytes if gpu else 0
        if hbm_budget_bytes is not None:
            budget = min(budget, hbm_budget_bytes) if gpu else hbm_budget_bytes
        self.budget = max(0, int(budget))
        self.graph = graph
        self.stream = torch.cuda.Stream() if gpu else None
        self.prep_threads = prep_threads

    def run(self, requests, time_scale: float = 1.0, log=None):
        """Serve ``requests`` (list of Request, arrival times in seconds); returns a stats dict."""
        torch = self.torch
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        queue: deque = deque()
        preparing: list = []
        active: list = []
        finished: list = []
        used = 0
        batch = None
        dirty = True
        n_sweep_iters = 0
        # every stream is made here, by the serving thread, never by a preparation thread while
        # the serving thread may be capturing a sweep graph
        gpu = torch.cuda.is_available()
        prep_streams = [torch.cuda.Stream() if gpu else None for _ in range(self.prep_threads)]
        t0 = time.perf_counter()

        def prepare(r, k):
            wl = r.wl
            if wl.coefs is None:   # the request's own table, made while others sweep
                wl = dataclasses.replace(wl, coefs=r.table_fn())
            if r.kind == "dmc":
                # a DMC request keeps its own stream (made at admission): its steps overlap the
                # fused VMC sweeps
                with torch.cuda.stream(r.stream):
                    s = qmc.System(wl, stream=r.stream)
                    s.dmc_init(r.dmc_target, feedback=r.dmc_feedback)
                    r.stats = torch.zeros((r.n_sweeps, 6), dtype=torch.float64, device="cuda")
                    return s
            with torch.cuda.stream(prep_streams[k]):
                return qmc.System(wl, stream=prep_streams[k])

        with cf.ThreadPoolExecutor(max_workers=self.prep_threads) as pool, torch.cuda.stream(self.stream):
            n_sub = 0
            while pending or queue or preparing or active:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival_s * time_scale <= now:
                    queue.append(pending.popleft())
                while queue:   # admission by device memory (first come, first served)
                    r = queue[0]
                    if r.est_bytes > self.budget or r.est_bytes <= 0:
                        # can never fit (or has no valid size): refused, the others go on
                        queue.popleft()
                        r.status = "rejected"
                        r.error = (f"needs {r.est_bytes} bytes of device memory, the whole budget is "
                                   f"{self.budget}")
                        r.finished_s = time.perf_counter() - t0
                        finished.append(r)
                        if log:
                            log(f"[serve] reject {r.rid}: {r.error}")
                        continue
                    if used + r.est_bytes > self.budget:
                        break
                    queue.popleft()
                    used += r.est_bytes
                    if r.kind == "dmc" and gpu:
                        r.stream = torch.cuda.Stream()
                    preparing.append((r, pool.submit(prepare, r, n_sub % self.prep_threads)))
                    n_sub += 1
                # prepared requests join at this sweep boundary (and the loop waits for one
                # when nothing else can run)
                if preparing and not active:
                    cf.wait([f for _, f in preparing], return_when=cf.FIRST_COMPLETED)
                still_prep = []
                for r, f in preparing:
                    if f.done():
                        try:
                            r.system = f.result()
                        except Exception as ex:   # this request fails alone; its memory is released
                            used -= r.est_bytes
                            r.status = "failed"
                            r.error = str(ex)
                            r.finished_s = time.perf_counter() - t0
                            finished.append(r)
                            if log:
                                log(f"[serve] request {r.rid} failed in preparation: {ex}")
                            continue
                        r.admitted_s = time.perf_counter() - t0
                        r.last_done_s = r.admitted_s
                        active.append(r)
                        dirty = dirty or r.kind == "vmc"
                        if log:
                            log(f"[serve] t={r.admitted_s:.3f}s admit {r.rid} N={r.wl.n_elec} "
                                f"W={r.wl.n_walkers} sweeps={r.n_sweeps} ({len(active)} resident)")
                    else:
                        still_prep.append((r, f))
                preparing = still_prep
                if not active:
                    if pending and not queue and not preparing:
                        time.sleep(max(0.0, pending[0].arrival_s * time_scale - (time.perf_counter() - t0)))
                    continue
                vmc = [r for r in active if r.kind == "vmc"]
                if dirty:
                    if batch is not None:
                        batch.close()
                    batch = (qmc.Batch([r.system for r in vmc], stream=self.stream, graph=self.graph)
                             if vmc else None)
                    dirty = False
                for r in active:   # DMC steps first, on their own streams
                    if r.kind == "dmc":
                        r.system.dmc_steps(1, r.stats[r.done_sweeps:r.done_sweeps + 1])
                ms = 0.0
                if batch is not None:
                    batch.sweep(1, measure=True)
                    ms, _ = batch.timing(reset=True)     # synchronises: this sweep's GPU time
                for r in active:
                    if r.kind == "dmc":
                        r.stream.synchronize()
                done = time.perf_counter() - t0
                n_sweep_iters += 1
                still = []
                for r in active:
                    r.latencies_ms.append((done - r.last_done_s) * 1e3)
                    r.gpu_ms.append(ms)
                    r.last_done_s = done
                    r.done_sweeps += 1
                    if r.done_sweeps >= r.n_sweeps:
                        if r.kind == "dmc":
                            r.energy = r.stats.cpu().numpy()
                            r.stats = None
                        else:
                            r.energy = r.system.last_energies()
                        r.final_pos = r.system.get_walkers()[0]
                        r.status = "done"
                        r.finished_s = time.perf_counter() - t0
                        r.system.close()
                        r.system = None
                        used -= r.est_bytes
                        finished.append(r)
                        dirty = dirty or r.kind == "vmc"
                    else:
                        still.append(r)
                active = still
        if batch is not None:
            batch.close()
        wall = time.perf_counter() - t0
        refused = [r for r in finished if r.status != "done"]
        finished = [r for r in finished if r.status == "done"]
        lat = np.array([x for r in finished for x in r.latencies_ms])
        def moves_of(r):
            if r.kind == "dmc":   # electrons of the walkers alive at each step
                alive = r.dmc_target + float(np.sum(r.energy[:-1, 2]))
                return alive * r.wl.n_elec
            return r.wl.n_walkers * r.wl.n_elec * r.n_sweeps

        moves = sum(moves_of(r) for r in finished)
        return {
            "requests": len(finished),
            "wall_s": wall,
            "moves": moves,
            "moves_per_s": moves / wall if wall > 0 else 0.0,
            "gpu_sweep_ms_p50": float(np.percentile([x for r in finished for x in r.gpu_ms], 50))
            if lat.size else None,
            "sweep_iterations": n_sweep_iters,
            "p50_sweep_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_sweep_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_queue_s": float(np.mean([r.admitted_s - r.arrival_s * time_scale for r in finished]))
            if finished else None,
            "dmc_requests": sum(r.kind == "dmc" for r in finished),
            "rejected": sum(r.status == "rejected" for r in refused),
            "failed": sum(r.status == "failed" for r in refused),
            "finished": finished,
            "refused": refused,
        }


def build_requests(trace, sweep_scale: float = 1.0, max_workers: int = 8, table_pool: bool = False,
                   log=None, dmc_every: int = 0):
    """Requests for a trace of ``qmc_inputs.served_trace`` entries, each a solid-like mixed-precision
    system with its own table.  Tables are generated on the host before serving starts: per
    request with seed = its id, or, with ``table_pool``, from one orbital bank per grid size
    (seed = grid, as many orbitals as the largest request of that grid): a request takes a cyclic
    window of the bank's orbitals, translated periodically on the grid and with signs, all drawn
    from its own seed (``qmc_inputs.request_table``).  A translated window of a stationary random
    field is again a draw of that field, so every request still has random smooth orbitals of its
    own, and a long trace needs only a few filtered tables.  With ``dmc_every`` = k > 0 every k-th
    request is a DMC run instead (drift-diffusion moves with sigma 0.3 / sqrt(N), 7/8 of its walkers
    as the target population, feedback 1 hartree, as many steps as the request's sweeps)."""
    import qmc_inputs as qi

    pool: dict = {}
    if table_pool:
        grids = sorted({e["grid"] for e in trace})
        need = {g: max(e["n_elec"] // 2 for e in trace if e["grid"] == g) for g in grids}
        with cf.ThreadPoolExecutor(max_workers=max_workers) as ex:
            tabs = list(ex.map(lambda g: qi.solid_table(need[g], g, seed=g, dtype=np.float32), grids))
        pool = dict(zip(grids, tabs))
        if log:
            log(f"[serve] orbital banks: grids {grids}")

    def make(e):
        wl = qi.solid(e["n_elec"], 4 if table_pool else e["grid"], n_walkers=e["n_walkers"], n_sweeps=1,
                      precision="mixed", table_dtype=np.float32, delay_rank=16, recompute_period=64,
                      seed=e["seed"], name=f"req{e['id']}")
        table_fn = None
        if table_pool:
            g = e["grid"]
            wl.grid = (g, g, g)
            wl.coefs = None
            table_fn = (lambda bank=pool[g], n=wl.n_orb, sd=e["seed"]: qi.request_table(bank, n, sd))
        wl.delay_rank = delay_rank_for(wl)
        n = max(1, int(round(e["n_sweeps"] * sweep_scale)))
        dmc = dmc_every > 0 and e["id"] % dmc_every == dmc_every - 1
        if dmc:
            wl = dataclasses.replace(wl, all_electron=True, drift=True, sigma=0.3 / np.sqrt(wl.n_elec))
        r = Request(rid=e["id"], arrival_s=e["arrival_s"], wl=wl, n_sweeps=n, kind="dmc" if dmc else "vmc",
                    dmc_target=max(1, wl.n_walkers * 7 // 8) if dmc else 0, table_fn=table_fn)
        r.est_bytes = qmc.estimate_device_bytes(wl, wl.n_walkers)
        if log:
            log(f"[serve] request {r.rid}: N={wl.n_elec} grid={e['grid']} W={wl.n_walkers} "
                f"sweeps={n} K={wl.delay_rank} {r.est_bytes / 2**30:.2f} GiB")
        return r

    with cf.ThreadPoolExecutor(max_workers=max_workers) as ex:
        reqs = list(ex.map(make, trace))
    if log:
        log(f"[serve] built {len(reqs)} requests")
    return reqs
