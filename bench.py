"""Benchmark of the MCLG hot path on one MI355X.

One step = one fused stream + Monte Carlo collide pass over every site of the
workload (D1Q3, L = 2^24, rho = 50, u0 = 0.1, C = 10, lambda = 1, Poisson
initial state, seed 2).  Prints one JSON line with site updates per second,
the HBM roofline of the fused kernel, and the oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--extra]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_SITE_UPDATE = 12     # 3 x uint16 read + 3 x uint16 written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_collide_L16M.json")
# the sources the D1Q3 step kernel is compiled from
KERNEL_SRCS = [os.path.join(ROOT, "paper_1706_01094_amd", "csrc", f)
               for f in ("kernels.hip", "rng.h", "device.h")]


# the D2Q9 step kernel: its sources and its counted VALU instructions per site
D2Q9_SRCS = [os.path.join(ROOT, "paper_1706_01094_amd", "csrc", f)
             for f in ("kernels_d2q9.hip", "rng.h", "device.h", "d2q9.h")]
D2Q9_VALU_FILE = os.path.join(ROOT, "profiles", "valu_d2q9_4096x4096.json")
# VALU issue of MI355X: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD
# every 4 cycles (16 lanes wide), 2.4 GHz
VALU_PEAK_G = 256 * 4 / 4 * 2.4


def kernel_hash(paths=None) -> str:
    h = hashlib.sha256()
    for path in paths or KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(budget_s: float = 15.0) -> dict:
    """The oracle (single-threaded C) on a bounded sample of the workload:
    the first 2^20 sites' worth of lattice (its own periodic lattice of that
    length, same rho, u0, seed), stepped until ~budget_s of CPU time."""
    import oracle as O
    import synth
    w = synth.PLAIN_LARGE
    L = 1 << 20
    sim = O.OracleSim([L], w["seed"], C=10, n_max=255)
    sim.init_poisson(0, w["rho"], w["u0"])
    sim.step(1)  # builds the table blocks this density visits
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        sim.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    sim.close()
    return {"value": steps * L / dt, "unit": "site updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle on a periodic L=2^20 lattice of the same workload "
                      f"(rho=50, u0=0.1, C=10), {steps} steps timed after 1 warm-up step"}


def run_plain(args, torch, M):
    import synth
    w = synth.PLAIN_LARGE
    L = w["L"]
    lat = M.Lattice(L, w["seed"], C=10, lam=(1, 1), n_max=255, rho=w["rho"], u0=w["u0"])
    if args.schedule:
        g, t, b = (int(v) for v in args.schedule.split(","))
        lat.set_schedule(g, t, b)
    stream = lat.stream
    cov, lds_bytes = lat.lds_coverage()
    run_plain.lds = {"expected_lds_fraction": round(cov, 5), "lds_bytes": lds_bytes}
    lat.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    if args.graph:
        chunk = 100
        done = 0
        while done + chunk <= args.steps:
            lat.step_graph(chunk)
            done += chunk
        lat.step(args.steps - done)
    else:
        lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    rc = lat.check()
    if rc != 0:
        raise SystemExit(f"device error {rc}")
    run_plain.stats = plain_statistics(lat, args.stat_logs)
    lat.close()
    return L, gpu_ms, wall


def plain_statistics(lat, logs: int) -> dict:
    """After the timed steps: per-velocity mean and variance/mean of the
    occupation numbers every 100 steps (exact int64 sums on the device), the
    check that the state stays Poisson distributed around f^eq."""
    out = {"every": 100, "t": [], "mean": [], "var_over_mean": []}
    for _ in range(logs):
        lat.step(100)
        m = lat.moments()[0]
        n = float(m["sites"])
        mean = [m["sum_n"][i] / n for i in range(3)]
        var = [m["sum_n2"][i] / n - mean[i] ** 2 for i in range(3)]
        out["t"].append(int(m["t"]))
        out["mean"].append([round(v, 5) for v in mean])
        out["var_over_mean"].append([round(var[i] / mean[i], 5) for i in range(3)])
    return out


def run_probe(args, torch, M):
    """Roofline probe: the headline workload at L = 2^27 (768 MiB of state,
    larger than the 256 MB Infinity Cache), so the state streams from HBM."""
    import synth
    w = synth.PLAIN_LARGE
    L = 1 << 27
    lat = M.Lattice(L, w["seed"], C=10, lam=(1, 1), n_max=255, rho=w["rho"], u0=w["u0"])
    lat.step(5)
    torch.cuda.synchronize()
    e0, e1 = _events(torch, lat.stream)
    e0.record(lat.stream)
    lat.step(args.probe_steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.probe_steps
    rc = lat.check()
    lat.close()
    if rc != 0:
        raise SystemExit(f"device error {rc} in the roofline probe")
    return {"workload": "d1q3_L128M_rho50_u0.1", "L": L, "steps": args.probe_steps,
            "ms_per_step": ms, "site_updates_per_s": L / (ms / 1e3),
            "achieved_GBps": BYTES_PER_SITE_UPDATE * L / (ms / 1e3) / 1e9,
            "frac": BYTES_PER_SITE_UPDATE * L / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def _events(torch, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    return e0, e1


def run_batched(args, torch, M):
    """1024 independent replicas of uneven L and density: plain per-replica
    launches vs one batched launch per step vs captured HIP graphs."""
    import synth
    from paper_1706_01094_amd import autotune
    man = synth.replica_manifest()
    sites = int(man["L"].sum())
    lat = M.Lattice(man["L"], synth.BATCHED["seed"], rho=man["rho"], u0=man["u0"],
                    replica_id=man["replica_id"])
    tuned = autotune.tune(man["L"], man["rho"], man["u0"], replica_id=man["replica_id"],
                          steps=10, use_cache=False)
    lat.set_schedule(*tuned["schedule"])
    out = {"workload": "d1q3_1024_replicas", "replicas": len(man["L"]), "sites": sites,
           "schedule": list(tuned["schedule"]),
           "autotune_trials": [[*t["schedule"], round(t.get("seconds_per_step", -1) * 1e6, 1)]
                               for t in tuned["trials"]]}
    lat.step(args.batched_warmup)
    torch.cuda.synchronize()
    for mode in ("batched", "graph"):
        e0, e1 = _events(torch, lat.stream)
        e0.record(lat.stream)
        if mode == "batched":
            lat.step(args.batched_steps)
        else:
            chunk = 100
            for _ in range(args.batched_steps // chunk):
                lat.step_graph(chunk)
            lat.step(args.batched_steps % chunk)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[mode] = {"steps": args.batched_steps, "ms": ms,
                     "site_updates_per_s": sites * args.batched_steps / (ms / 1e3)}
    # plain: one launch per replica per step
    n = len(man["L"])
    e0, e1 = _events(torch, lat.stream)
    t0 = time.perf_counter()
    e0.record(lat.stream)
    for _ in range(args.plain_steps):
        for r in range(n):
            lat.step_replica(r, 1)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    out["plain_per_replica"] = {"steps": args.plain_steps, "launches": args.plain_steps * n,
                                "ms": ms, "wall_s": wall,
                                "site_updates_per_s": sites * args.plain_steps / (ms / 1e3)}
    out["batched_vs_plain"] = out["batched"]["site_updates_per_s"] / \
        out["plain_per_replica"]["site_updates_per_s"]
    out["graph_vs_plain"] = out["graph"]["site_updates_per_s"] / \
        out["plain_per_replica"]["site_updates_per_s"]
    if lat.check() != 0:
        raise SystemExit("device error in the batched run")
    m = lat.moments()
    out["t"] = int(m[0]["t"])
    lat.close()
    return out


def _serve(M, torch, jobs, arena_bytes, max_slots, seed, k, time_limit):
    """Real-time driver: jobs are submitted when their arrival time has
    passed; the server advances all resident jobs k steps per tick."""
    srv = M.Server(arena_bytes, max_slots, seed)
    t0 = time.perf_counter()
    nxt = 0
    done = {}
    work = 0
    while len(done) < len(jobs):
        now = time.perf_counter() - t0
        if now > time_limit:
            break
        while nxt < len(jobs) and jobs[nxt]["arrival"] <= now:
            j = jobs[nxt]
            srv.submit(j["job_id"], j["L"], j["steps"], j["rho"], j["u0"])
            nxt += 1
        q, r, _ = srv.stats()
        if q == 0 and r == 0:
            if nxt < len(jobs):
                time.sleep(max(0.0, min(0.01, jobs[nxt]["arrival"] - now)))
            continue
        srv.tick(k)
        tnow = time.perf_counter() - t0
        for jid, m in srv.poll():
            done[jid] = tnow
    q, r, used = srv.stats()
    srv.close()
    lat = sorted(done[j["job_id"]] - j["arrival"] for j in jobs if j["job_id"] in done)
    work = sum(j["L"] * j["steps"] for j in jobs if j["job_id"] in done)
    span = max(done.values()) - jobs[0]["arrival"] if done else 0.0
    pct = (lambda f: lat[min(len(lat) - 1, int(f * len(lat)))] if lat else None)
    return {"jobs": len(jobs), "completed": len(done), "queued_at_end": q, "resident_at_end": r,
            "p50_latency_s": pct(0.5), "p99_latency_s": pct(0.99),
            "site_updates_per_s": work / span if span > 0 else 0.0,
            "span_s": span, "site_updates": work}


def run_served(args, torch, M, capacity):
    """Poisson arrivals (200 jobs/s) of jobs with L log-uniform in
    [2^12, 2^24], steps U{100..5000}, rho U{5..100}; 200 GB arena."""
    import synth
    cfg = synth.SERVED
    out = {"workload": "d1q3_served_200_per_s", "arena_bytes": cfg["budget"]}
    jobs = synth.job_trace(args.serve_window)
    offered = sum(j["L"] * j["steps"] for j in jobs) / args.serve_window
    out["trace"] = {"window_s": args.serve_window, "jobs": len(jobs),
                    "offered_site_updates_per_s": offered}
    out["overloaded"] = _serve(M, torch, jobs, cfg["budget"], 8192, cfg["seed"], 50,
                               args.serve_limit)
    # sustainable rate: 0.8 x measured batched capacity
    mean_work = offered / cfg["rate"]
    rate = 0.8 * capacity / mean_work
    jobs2 = synth.job_trace(args.serve_window * 2, rate=rate, seed=cfg["seed"] + 1)
    out["sustainable"] = {"rate_jobs_per_s": rate, "jobs": len(jobs2),
                          **_serve(M, torch, jobs2, cfg["budget"], 8192, cfg["seed"], 50,
                                   args.serve_limit)}
    return out


def run_wave(args, torch, M):
    """Decaying density wave, L = 2^22, 5000 steps, int64 Fourier projection
    (Eq. (A)) every 10 steps."""
    import numpy as np
    import synth
    w = synth.DENSITY_WAVE
    L = w["L"]
    counts = synth.density_wave_counts()
    tw = synth.twiddles(L, 1)
    lat = M.Lattice(L, w["seed"], counts=counts)
    twd = torch.as_tensor(tw).to(lat.device)
    den = float(np.sum(tw[1].astype(np.float64) ** 2))
    amp = []
    e0, e1 = _events(torch, lat.stream)
    t0 = time.perf_counter()
    e0.record(lat.stream)
    for _ in range(w["steps"] // w["log_every"]):
        lat.step(w["log_every"])
        m = lat.moments(twd, 1)[0]
        amp.append(m["fourier"][0][1] / den)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat.close()
    return {"workload": "d1q3_L4M_wave_rho40", "steps": w["steps"], "logs": len(amp),
            "wall_s": wall, "site_updates_per_s_incl_logging": L * w["steps"] / wall,
            "amplitude_first": amp[0], "amplitude_last": amp[-1]}


def run_d2q9(args, torch, M):
    """D2Q9 (the paper's second lattice): 4096 x 4096 sites, Poisson start at
    rho = 36, u = 0, C = 10, the lambda_c of the paper's D2Q9 equilibrium run;
    every site runs the literal sub-collision loop (ALU-bound)."""
    Lx = Ly = 4096
    lat = M.Lattice9(Lx, Ly, 9, C=10, rho=36.0, ux=0.0, uy=0.0)
    lat.step(args.d2q9_warmup)
    e0, e1 = _events(torch, lat.stream)
    e0.record(lat.stream)
    lat.step(args.d2q9_steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rc = lat.check()
    m = lat.moments()[0]
    lat.close()
    sites = Lx * Ly
    rate = sites * args.d2q9_steps / (ms / 1e3)
    out = {"workload": "d2q9_4096x4096_rho36_u0", "C": 10, "lambda9": "15/128, 1/4 x6, 1/8, 18/144",
           "steps": args.d2q9_steps, "ms_per_step": ms / args.d2q9_steps,
           "site_updates_per_s": rate, "hbm_GBps": 36.0 * rate / 1e9,
           "check": rc, "mass_per_site": m["sum_N"] / sites, "roofline": None}
    # ALU roofline: VALU wave instructions per site (one lane per site) from
    # the committed counter run, valid while the kernel's sources are the same
    try:
        with open(D2Q9_VALU_FILE) as f:
            v = json.load(f)
    except (OSError, ValueError):
        v = {}
    if v.get("kernel_sha256_16") == kernel_hash(D2Q9_SRCS):
        achieved = v["valu_insts_per_wave"] * rate / 64 / 1e9
        out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_G,
                           "unit": "G VALU wave-instructions/s", "frac": achieved / VALU_PEAK_G,
                           "valu_insts_per_wave": v["valu_insts_per_wave"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10_000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--schedule", default="", help="groups,threads,lds_bytes")
    ap.add_argument("--graph", action="store_true", help="launch steps from captured HIP graphs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the plain headline (skip batched, served, density wave)")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--batched-warmup", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--probe-steps", type=int, default=200)
    ap.add_argument("--stat-logs", type=int, default=10)
    ap.add_argument("--serve-window", type=float, default=2.0)
    ap.add_argument("--serve-limit", type=float, default=60.0)
    ap.add_argument("--d2q9-steps", type=int, default=50)
    ap.add_argument("--d2q9-warmup", type=int, default=5)
    ap.add_argument("--d2q9-only", action="store_true", help="only the D2Q9 measurement")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 1024-replica batched measurement")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run 8 device-to-device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.empty(args.copy_probe // 4, dtype=torch.int32, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 8}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the lattice and replica work of this build "
              "runs on a single MI355X (sharding across GPUs is described in DESIGN.md).",
              file=sys.stderr)
        raise SystemExit(2)
    import torch
    from paper_1706_01094_amd import mclg as M
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")

    if args.d2q9_only:
        print(json.dumps({"d2q9": run_d2q9(args, torch, M)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": run_batched(args, torch, M)}), flush=True)
        return
    L, gpu_ms, wall = run_plain(args, torch, M)
    ms_per_step = gpu_ms / args.steps
    value = L * args.steps / (gpu_ms / 1e3)
    achieved = BYTES_PER_SITE_UPDATE * L / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic()
    out = {
        "metric": "site updates/s (stream+MC collide, D1Q3), % HBM peak; batched vs plain",
        "value": value,
        "unit": "site updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "d1q3_L16M_rho50_u0.1", "L": L, "rho": 50.0, "u0": 0.1, "C": 10,
                   "lambda": 1, "n_max": 255, "seed": 2, "launch": "graph" if args.graph else "plain",
                   "schedule": args.schedule or "default", **getattr(run_plain, "lds", {})},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "statistics": getattr(run_plain, "stats", None),
    }
    if not args.no_extra:
        extra = {}
        extra["roofline_probe"] = run_probe(args, torch, M)
        torch.cuda.empty_cache()
        extra["batched"] = run_batched(args, torch, M)
        extra["density_wave"] = run_wave(args, torch, M)
        torch.cuda.empty_cache()
        extra["served"] = run_served(args, torch, M, extra["batched"]["batched"]["site_updates_per_s"])
        torch.cuda.empty_cache()
        extra["d2q9"] = run_d2q9(args, torch, M)
        out["extra"] = extra
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
