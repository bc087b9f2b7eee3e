"""Benchmark of the coupled LBM-DEM step on one MI355X.

Default workload: the dense suspension of 24,000 spheres of diameter 12 in a
512^3 lattice (periodic in x and y, walls in z, ~16 % solids, density ratio 2,
gravity 2e-6, viscosity 0.02), FP32 population storage, and the same inputs
with FP16 storage reported beside it.  A step is one full pass of Alg. 1 on
the GPU: fused stream-collide sweep, DEM sub-cycles, mapping update with
reconstruction, boundary values and momentum-exchange partials of the next
step.

Prints one JSON line: MLUPS over all cells; the roofline of the dominant
kernel (the sweep, HBM bound; algorithmic bytes = 19 loads + 19 stores of the
stored PDF type + 1 flag byte per cell; duration from HIP events around every
sweep launch on the domain's stream); the coupled step's algorithmic GB/s and
fraction of the HBM peak; and the oracle timed on one pinned host core on a
bounded sample of the same workload.  Other workloads: --workload
sphere_wall | dense | dense512 | settling_32 | serve.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "coupled-step MLUPS & % HBM roofline; batched solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def _gpu_params(wl, storage):
    from paper_2003_01490_amd import lbmdem as L

    keys = {f[0] for f in L.Config._fields_}
    p = {k: v for k, v in wl.params.items() if k in keys}
    p["storage"] = storage
    p["max_radius"] = float(max(wl.R))
    p["max_spheres"] = max(len(wl.R), 1)
    return L.default_config(**p)


def make_workload(name, seed):
    from paper_2003_01490_amd import workloads as W

    if name == "sphere_wall":
        return W.sphere_wall(seed)
    if name == "dense":
        return W.dense(seed, n=384, count=10000, steps=1000)
    if name == "dense512":
        return W.dense(seed, n=512, count=24000, steps=1000)
    if name == "settling_32":
        return W.settling_32(seed)
    raise SystemExit(f"unknown workload {name}")


def sweep_source_sha() -> str:
    """SHA-256 over the sources the sweep kernel is built from."""
    import hashlib

    h = hashlib.sha256()
    for name in ("sweep.hip", "collide.hpp", "internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2003_01490_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_record(workload: str, storage: str):
    """HBM bytes per sweep launch measured with hardware counters (profiles/),
    valid only while the sweep source is the one that was measured."""
    import glob
    import hashlib
    import re

    sha = sweep_source_sha()
    tag = {"f64": "FP64", "f32": "FP32", "f16": "FP16"}[storage]
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "pmc_traffic_*.md"))):
        for block in re.findall(r"```json\n(.*?)\n```", open(f).read(), re.S):
            rec = json.loads(block)
            if rec.get("sweep_src_sha256") == sha and rec.get("workload", "").split(" ")[0] == workload \
                    and rec["workload"].endswith(tag):
                return rec["bytes_per_launch"], os.path.relpath(f, ROOT)
    return None, None


def cpu_sample(name, wl, seed):
    """Workload the oracle is timed on: the same one where a few steps take
    seconds; for the dense suspensions its 96^3 sub-problem at the same solid
    fraction (the oracle's brute-force mapping visits every cell for every
    sphere)."""
    from paper_2003_01490_amd import workloads as W

    if name.startswith("dense"):
        return W.dense(seed, n=96, count=156), "96^3 sub-problem with 156 spheres D=12 (same solid fraction)"
    return wl, "the same workload"


def cpu_baseline(wl, steps):
    """The oracle, single-threaded, on `steps` coupled steps of the given
    lattice and spheres, with this process pinned to one host core while it
    runs.  Returns MLUPS, seconds, the core."""
    import oracle as O

    keys = {f[0] for f in O.RefConfig._fields_}
    cfg = O.make_config(**{k: v for k, v in wl.params.items() if k in keys})
    d = O.RefDomain(cfg)
    if len(wl.R):
        d.add_spheres(wl.x, wl.R, wl.rho, u=wl.u, w=wl.w)
    if wl.ramp:
        r = wl.ramp
        d.set_mode(0, O.MODE_PRESCRIBED, r["u_target"], r["c_acc"], r["t_st"], r["release_gap"])
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        d.step(steps)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, set(allowed))
    n = wl.params["nx"] * wl.params["ny"] * wl.params["nz"]
    return n * steps / dt / 1e6, dt, core


def cpu_model() -> str:
    """The host CPU: lscpu's model name, with family, model and stepping from
    /proc/cpuinfo (a virtualised host may report only a generic name)."""
    name = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                name = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    k, v = (t.strip() for t in line.split(":", 1))
                    if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                        info[k] = v
                if not line.strip() and info:
                    break
    except OSError:
        pass
    name = name or info.get("model name") or platform.processor() or "unknown"
    if "cpu family" in info:
        name += f" (family {info['cpu family']}, model {info.get('model', '?')}, stepping {info.get('stepping', '?')})"
    return name


def _oracle_request_sample(req, steps, core):
    """Seconds per coupled step of the oracle on one serving request (its
    first `steps` steps), in a process pinned to one host core."""
    import oracle as O
    from paper_2003_01490_amd import workloads as W

    if core is not None:
        os.sched_setaffinity(0, {core})
    wl = W.serve_workload(req)
    keys = {f[0] for f in O.RefConfig._fields_}
    d = O.RefDomain(O.make_config(**{k: v for k, v in wl.params.items() if k in keys}))
    d.add_spheres(wl.x, wl.R, wl.rho)
    r = wl.ramp
    d.set_mode(0, O.MODE_PRESCRIBED, r["u_target"], r["c_acc"], r["t_st"], r["release_gap"])
    t0 = time.perf_counter()
    d.step(steps)
    return (time.perf_counter() - t0) / steps


def serve_oracle_sample(reqs, steps, procs):
    """The oracle on the 8 smallest requests: each alone on one pinned core,
    then all 8 at once in `procs` processes on distinct cores (aggregate)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    small = sorted(reqs, key=lambda r: r["L"][0] * r["L"][1] * r["L"][2])[:8]
    cores = sorted(os.sched_getaffinity(0))
    alone = [_oracle_request_sample(r, steps, cores[-1]) for r in small]
    os.sched_setaffinity(0, set(cores))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=procs, mp_context=ctx) as ex:
        futs = [ex.submit(_oracle_request_sample, r, steps, cores[k % len(cores)]) for k, r in enumerate(small)]
        together = [f.result() for f in futs]
    wall = time.perf_counter() - t0
    return small, alone, together, wall


def serve_bench(args):
    """Serving stream: independent sphere-wall requests with Poisson arrivals,
    each run until its sphere rebounds (first apex after the wall contact) or a
    step cap, FP32 storage.  Continuous batching: arrived requests are admitted
    while their footprints fit the pool budget, all admitted domains advance
    together in chunks of steps, stopped ones are retired at once and the next
    arrivals take their place.  Runs with the pool capped (--pool-gb) and,
    with --serve-uncapped, with the whole free device memory as the pool.
    Baseline: first-come-first-served, one request at a time.  With
    --serve-baseline run, each request is stepped alone in arrival order;
    with --serve-baseline measured (for streams too long to replay), each
    request's alone cost is measured over a bounded sample (set-up plus
    --solo-steps steps) and scaled to the steps the batched run needed (a
    domain's trajectory is the same alone and in a batch), and the queue is
    replayed from those service times.  The oracle is timed on the 8 smallest
    requests over --cpu-steps steps each, alone and 8 at once in 8
    processes, and scaled to their step counts.
    """
    import numpy as np

    from paper_2003_01490_amd import workloads as W

    reqs = W.serve_requests(args.seed, args.requests, rate=args.rate)
    oracle_part = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the worker processes are fresh interpreters
        oracle_part = serve_oracle_sample(reqs, args.cpu_steps or 20, 8)

    import torch

    from paper_2003_01490_amd import lbmdem as L

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    bytes_per_cell = 2 * 19 * 4 + 1

    def make(req):
        wl = W.serve_workload(req)
        cfg = _gpu_params(wl, L.STORE_F32)
        dom = L.Domain(cfg, device=dev, stream=stream)
        dom.add_spheres(wl.x, wl.R, wl.rho)
        r = wl.ramp
        dom.set_mode(0, L.PRESCRIBED, r["u_target"], r["c_acc"], r["t_st"], r["release_gap"])
        dom.set_stop_rule(L.STOP_REBOUND, args.max_steps)
        return dom

    def footprint(req):
        return L.footprint_bytes(_gpu_params(W.serve_workload(req), L.STORE_F32))

    def summary(done, wall, busy_ms=None):
        lat = np.array([d["latency"] for d in done])
        cells = sum(d["cells"] * d["steps"] for d in done)
        out = {"solves_per_s": round(len(done) / wall, 4), "wall_s": round(wall, 3),
               "p50_s": round(float(np.percentile(lat, 50)), 3), "p99_s": round(float(np.percentile(lat, 99)), 3),
               "aggregate_GBps": round(cells * bytes_per_cell / wall / 1e9, 1),
               "aggregate_MLUPS": round(cells / wall / 1e6, 1),
               "rebounds": int(sum(d["stopped_by_rule"] for d in done)),
               "capped": int(sum(not d["stopped_by_rule"] for d in done))}
        if busy_ms is not None:
            out["gpu_busy"] = round(busy_ms / 1e3 / wall, 4)
        return out

    def run_batched(pool, tag):
        batch = L.Batch(stream, pool)
        pending = sorted(reqs, key=lambda r: r["arrival"])
        active, done, used = {}, [], 0
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        busy, timeline, peak = 0.0, [], 0
        t0 = time.perf_counter()
        last_log = -1.0
        while pending or active:
            now = time.perf_counter() - t0
            while pending and pending[0]["arrival"] <= now:
                fp = footprint(pending[0])
                if used + fp > pool and active:
                    break
                req = pending.pop(0)
                dom = make(req)
                slot = batch.admit(dom)
                active[slot] = (req, dom, fp)
                used += fp
            if not active:
                time.sleep(max(0.0, pending[0]["arrival"] - (time.perf_counter() - t0)))
                continue
            peak = max(peak, len(active))
            ev0.record(stream)
            batch.step(args.chunk)
            ev1.record(stream)
            fin = batch.done()
            busy += ev0.elapsed_time(ev1)
            st = batch.status()
            for slot in fin:
                req, dom, fp = active.pop(slot)
                steps = st[slot][0]
                batch.retire(slot)
                done.append(dict(id=req["id"], latency=time.perf_counter() - t0 - req["arrival"], steps=steps,
                                 cells=dom.N, stopped_by_rule=steps < args.max_steps))
                dom.close()
                used -= fp
            t = time.perf_counter() - t0
            if t - last_log >= 1.0:
                last_log = t
                waiting = sum(1 for r in pending if r["arrival"] <= t)
                timeline.append([round(t, 2), len(active), waiting, len(done), round(used / 2 ** 30, 2)])
                print(f"[serve {tag}] t {t:7.2f}s in flight {len(active):3d} waiting {waiting:3d} "
                      f"done {len(done):3d} pool {used / 2 ** 30:6.1f} GiB", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        batch.close()
        res = summary(done, wall, busy)
        res["pool_GiB"] = round(pool / 2 ** 30, 1)
        res["peak_in_flight"] = peak
        res["in_flight_log"] = {"columns": ["t_s", "in_flight", "waiting", "done", "pool_used_GiB"],
                                "rows": timeline}
        return res, done

    def whole_device():
        free, _ = torch.cuda.mem_get_info(dev)
        return int(free * 0.9)

    if args.pool_gb > 0:
        capped, done = run_batched(int(args.pool_gb * 2 ** 30), f"{args.pool_gb:g}GiB")
    else:  # no budget: the whole free device memory
        capped, done = run_batched(whole_device(), "uncapped")
    uncapped = None
    if args.serve_uncapped and args.pool_gb > 0:
        uncapped, _ = run_batched(whole_device(), "uncapped")
    steps_of = {d["id"]: d["steps"] for d in done}

    base = None
    if args.serve_baseline == "run":
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        done_b, busy_b = [], 0.0
        t0 = time.perf_counter()
        for req in sorted(reqs, key=lambda r: r["arrival"]):
            now = time.perf_counter() - t0
            if req["arrival"] > now:
                time.sleep(req["arrival"] - now)
            dom = make(req)
            while True:
                ev0.record(stream)
                dom.step(args.chunk)
                ev1.record(stream)
                steps, stopped = dom.progress()
                busy_b += ev0.elapsed_time(ev1)
                if stopped:
                    break
            done_b.append(dict(id=req["id"], latency=time.perf_counter() - t0 - req["arrival"], steps=steps,
                               cells=dom.N, stopped_by_rule=steps < args.max_steps))
            dom.close()
            print(f"[serve-fifo] t {time.perf_counter() - t0:7.2f}s done {len(done_b):3d}", file=sys.stderr,
                  flush=True)
        base = summary(done_b, time.perf_counter() - t0, busy_b)
        base["kind"] = "replayed one at a time in arrival order"
    elif args.serve_baseline == "measured":
        service = {}
        for k, req in enumerate(reqs):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            dom = make(req)
            dom.step(1)
            dom.sync()
            t1 = time.perf_counter()
            dom.step(args.solo_steps)
            dom.sync()
            t2 = time.perf_counter()
            dom.close()
            service[req["id"]] = (t1 - t0) + (t2 - t1) / args.solo_steps * (steps_of[req["id"]] - 1)
            if k % 64 == 63:
                print(f"[serve-fifo] measured {k + 1} requests alone", file=sys.stderr, flush=True)
        clock, done_b = 0.0, []
        for req in sorted(reqs, key=lambda r: r["arrival"]):
            clock = max(clock, req["arrival"]) + service[req["id"]]
            n = int(np.prod(req["L"]))
            done_b.append(dict(id=req["id"], latency=clock - req["arrival"], steps=steps_of[req["id"]], cells=n,
                               stopped_by_rule=steps_of[req["id"]] < args.max_steps))
        base = summary(done_b, clock)
        base["kind"] = (f"one at a time in arrival order, each request's cost measured alone (set-up, first "
                        f"step, {args.solo_steps} timed steps) and scaled to its step count")

    cells = np.array([np.prod(r["L"]) for r in reqs])
    St = np.array([r["St"] for r in reqs])
    result = {
        "metric": METRIC,
        "value": capped["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": int(sum(d["steps"] for d in done)),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving stream: {args.requests} sphere-wall requests, Poisson arrivals "
                               f"{args.rate}/s, edges U{{48..192}}, D U[6,24], St logU[1,1000] "
                               f"(median {np.median(St):.1f}), rho_r U[1.5,8], u_s 0.02, stop at rebound "
                               f"or {args.max_steps} steps, FP32 storage",
                   "pool_GiB": capped["pool_GiB"], "chunk_steps": args.chunk, "seed": args.seed,
                   "mean_cells": int(cells.mean()), "parallelism": "single GPU"},
        "batched": capped,
        "batched_uncapped": uncapped,
        "fifo_one_at_a_time": base,
    }
    if base:
        result["speedup_vs_fifo"] = round(capped["solves_per_s"] / base["solves_per_s"], 3)
    if oracle_part:
        import oracle

        small, alone, together, wall = oracle_part
        ids = [r["id"] for r in small]
        solve_alone = [t * steps_of[i] for t, i in zip(alone, ids)]
        solve_together = [t * steps_of[i] for t, i in zip(together, ids)]
        result["cpu_baseline"] = {
            "value": round(1.0 / float(np.mean(solve_alone)), 6),
            "unit": "solves/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the 8 smallest requests ({min(np.prod(r['L']) for r in small)}.."
                      f"{max(np.prod(r['L']) for r in small)} cells), {args.cpu_steps or 20} steps each on one "
                      f"pinned core, scaled to the steps each needed on the GPU",
            "per_request_s": [round(v, 1) for v in solve_alone],
            "aggregate_P_processes": {"P": 8, "solves_per_s": round(8.0 / float(np.max(solve_together)), 6),
                                      "per_request_s": [round(v, 1) for v in solve_together]},
            "cpu": cpu_model(),
            "build": "gcc " + " ".join(oracle.BUILD_FLAGS),
        }
    print(json.dumps(result))


def run_domain(wl, storage_name, args, dev, profile_breakdown=True):
    """One domain of the workload at one storage precision: warm-up, the timed
    steps (HIP events around every sweep launch), a per-kernel-group breakdown
    from extra steps, then the domain is closed."""
    import torch

    from paper_2003_01490_amd import lbmdem as L

    storage = {"f64": L.STORE_F64, "f32": L.STORE_F32, "f16": L.STORE_F16}[storage_name]
    cfg = _gpu_params(wl, storage)
    cfg.overlap = args.overlap
    if args.map_kernel is not None:
        cfg.map_kernel = args.map_kernel
    # step graphs need a stream of their own (not the null stream)
    dom = L.Domain(cfg, device=dev, stream=torch.cuda.Stream(device=dev) if args.graph else None)
    try:
        if args.graph:
            dom.set_graph(True)
        dom.add_spheres(wl.x, wl.R, wl.rho, u=wl.u, w=wl.w)
        if wl.ramp:
            r = wl.ramp
            dom.set_mode(0, L.PRESCRIBED, r["u_target"], r["c_acc"], r["t_st"], r["release_gap"])
        print(f"[bench] workload {wl.name} lattice {cfg.nx}x{cfg.ny}x{cfg.nz} spheres {len(wl.R)} "
              f"storage {storage_name}", file=sys.stderr, flush=True)
        dom.step(args.warmup)
        dom.sync()
        if args.copy_probe_mib:
            nb = args.copy_probe_mib << 20
            a = torch.empty(nb, dtype=torch.uint8, device=dev)
            b = torch.empty(nb, dtype=torch.uint8, device=dev)
            for _ in range(3):
                L.device_copy(b, a, nb, dom.stream)
            torch.cuda.synchronize()
            del a, b
        # timed region: HIP events around every sweep launch only (level 1);
        # with step graphs the timed steps replay the graph untimed and the
        # sweep is timed over as many further steps launched directly
        dom.set_profiling(0 if args.graph else 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dom.step(args.steps)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        dom.sync()
        if args.graph:
            dom.set_profiling(1)
            dom.step(args.steps)
            dom.sync()
        sweep_ms, sweep_n = dom.profile(0)
        brk = {}
        if profile_breakdown:
            dom.set_profiling(2)
            dom.step(min(args.steps, 50))
            dom.sync()
            # kernel groups: the sweep; the DEM with the mapping's claims or bins
            # (beside the sweep); reconstruction, mapping update and boundary pass
            brk = {k: dom.profile(j) for j, k in enumerate(("sweep", "dem_map_prepare", "recon_remap_bc"))}
        dom.set_profiling(0)
        ncell = cfg.nx * cfg.ny * cfg.nz
        nfluid = int((dom.field("flags") <= 1).sum())
        sweep_avg_s = sweep_ms / max(sweep_n, 1) / 1e3
        bytes_per_step = dom.sweep_bytes()
        s0 = dom.sphere(0)
        return {
            "cfg": cfg, "ncell": ncell, "nfluid": nfluid, "elapsed": elapsed,
            "ms_per_step": elapsed / args.steps * 1e3,
            "mlups": ncell * args.steps / elapsed / 1e6,
            "mflups_fluid": nfluid * args.steps / elapsed / 1e6,
            "sweep_avg_s": sweep_avg_s, "bytes_per_step": bytes_per_step,
            "breakdown": {k: round(ms / max(n, 1) * 1e3, 3) for k, (ms, n) in brk.items()},
            "sphere0": {"z": float(s0["x"][2]), "uz": float(s0["u"][2]), "mode": s0["mode"]},
        }
    finally:
        dom.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="dense512")
    ap.add_argument("--storage", default=None, choices=["f64", "f32", "f16"],
                    help="population storage (default f32, with the f16 form of the dense "
                         "workloads reported beside it)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="coupled steps of the oracle sample (default: about 15 s of CPU work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=512, help="serving stream: number of requests")
    ap.add_argument("--rate", type=float, default=50.0, help="serving stream: arrivals per second")
    ap.add_argument("--pool-gb", type=float, default=48.0,
                    help="serving stream: pool budget (GiB; 0: the whole free device memory)")
    ap.add_argument("--max-steps", type=int, default=20000, help="serving stream: step cap per request")
    ap.add_argument("--chunk", type=int, default=100, help="serving stream: steps per batch call")
    ap.add_argument("--serve-baseline", default="measured", choices=["off", "run", "measured"],
                    help="serving stream: first-come-first-served baseline, replayed or from measured costs")
    ap.add_argument("--solo-steps", type=int, default=200,
                    help="serving stream: timed steps per request for the measured baseline")
    ap.add_argument("--serve-uncapped", action="store_true",
                    help="serving stream: also run with the whole free device memory as the pool")
    ap.add_argument("--map-kernel", type=int, default=None, choices=[0, 1, 2, 3],
                    help="particle-link boundary pass (default: the configuration's automatic choice)")
    ap.add_argument("--overlap", type=int, default=1, choices=[0, 1],
                    help="run the DEM beside the sweep on a second stream (1, default) or after it (0)")
    ap.add_argument("--graph", action="store_true",
                    help="replay one captured step graph per step (lbmdem_set_graph)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs the path on one GPU; --gpus must be 1 (how the "
                                   "path would shard over several GPUs is described in the design notes)"}))
        raise SystemExit(2)
    if args.workload == "serve":
        serve_bench(args)
        return

    import torch

    storage = args.storage or "f32"
    second = None if args.storage or not args.workload.startswith("dense") else "f16"
    wl = make_workload(args.workload, args.seed)
    dev = torch.device("cuda:0")
    main_run = run_domain(wl, storage, args, dev)
    other = run_domain(wl, second, args, dev, profile_breakdown=False) if second else None
    cfg = main_run["cfg"]
    achieved = main_run["bytes_per_step"] / main_run["sweep_avg_s"] / 1e9
    coupled = main_run["bytes_per_step"] / (main_run["ms_per_step"] / 1e3) / 1e9
    traffic, traffic_src = traffic_record(args.workload, storage)

    result = {
        "metric": METRIC,
        "value": round(main_run["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": storage,
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name} {cfg.nx}x{cfg.ny}x{cfg.nz}, {len(wl.R)} sphere(s) D={2 * wl.R[0]:g}, "
                        f"{storage.upper()} population storage",
            "lattice": [cfg.nx, cfg.ny, cfg.nz],
            "spheres": len(wl.R),
            "n_sub": cfg.n_sub,
            "collision": "TRT+aB",
            "seed": args.seed,
            "overlap": bool(args.overlap),
            "step_graph": bool(args.graph),
            "map_kernel": cfg.map_kernel,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_sweep (fused stream-collide)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_source": traffic_src,
            "bytes_per_launch": main_run["bytes_per_step"],
            "avg_launch_us": round(main_run["sweep_avg_s"] * 1e6, 3),
        },
        "coupled_step": {
            "bytes_per_step": main_run["bytes_per_step"],
            "achieved_GBps": round(coupled, 1),
            "frac": round(coupled / HBM_PEAK_GBS, 4),
        },
        "mflups_fluid": round(main_run["mflups_fluid"], 2),
        "kernel_avg_us": main_run["breakdown"],
        "sphere_final": main_run["sphere0"],
    }
    if other:
        o_coupled = other["bytes_per_step"] / (other["ms_per_step"] / 1e3) / 1e9
        o_sweep = other["bytes_per_step"] / other["sweep_avg_s"] / 1e9
        result[f"{second}_form"] = {
            "MLUPS": round(other["mlups"], 2), "ms_per_step": round(other["ms_per_step"], 5),
            "sweep_GBps": round(o_sweep, 1), "sweep_frac": round(o_sweep / HBM_PEAK_GBS, 4),
            "coupled_GBps": round(o_coupled, 1), "coupled_frac": round(o_coupled / HBM_PEAK_GBS, 4),
            "bytes_per_step": other["bytes_per_step"],
        }
    if wl.meta:
        result["config"]["params"] = {k: (round(v, 6) if isinstance(v, float) else v)
                                      for k, v in wl.meta.items()}
    if not args.no_cpu_baseline:
        import oracle

        swl, what = cpu_sample(args.workload, wl, args.seed)
        steps = args.cpu_steps or (20 if args.workload.startswith("dense") else 8)
        mlups_cpu, dt, core = cpu_baseline(swl, steps)
        sn = (swl.params["nx"], swl.params["ny"], swl.params["nz"])
        result["cpu_baseline"] = {
            "value": round(mlups_cpu, 4),
            "unit": "MLUPS",
            "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} coupled steps of {what} ({sn[0]}x{sn[1]}x{sn[2]}) from its initial state "
                      f"({dt:.1f} s, one thread pinned to host core {core})",
            "cpu": cpu_model(),
            "build": "gcc " + " ".join(oracle.BUILD_FLAGS),
        }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
