"""Benchmark of the MCLG hot path on one MI355X.

One step = one fused stream + Monte Carlo collide pass over every site of the
workload (D1Q3, L = 2^24, rho = 50, u0 = 0.1, C = 10, lambda = 1, Poisson
initial state, seed 2).  Prints one JSON line with site updates per second,
the HBM roofline of the fused kernel, and the oracle timed on the host; the
other workloads (an HBM-resident lattice, the 1024-replica batch, the
density wave, the served trace, D2Q9, and the headline lattice at lower
densities and without collisions, which shows what bounds its step) follow
under "extra".

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extra] [--no-cpu]
    python bench.py --only plain|probe|batched|wave|served|d2q9|moments|bound
    python bench.py --copy-probe BYTES     (counter calibration: device copies)
"""
from __future__ import annotations

import argparse
import ctypes as ct
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_SITE_UPDATE = 12     # 3 x uint16 read + 3 x uint16 written
INFINITY_CACHE_BYTES = 256 << 20
PROFILES = os.path.join(ROOT, "profiles")
# HBM traffic of the step kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# per workload (valid while the kernel's sources are unchanged)
TRAFFIC_FILES = {
    "plain": os.path.join(PROFILES, "traffic_stream_collide_L16M.json"),
    "probe": os.path.join(PROFILES, "traffic_stream_collide_L128M.json"),
    "batched": os.path.join(PROFILES, "traffic_stream_collide_1024_replicas.json"),
    "probe_blocked": os.path.join(PROFILES, "traffic_stream_collide_L128M_tiles.json"),
    "batched_blocked": os.path.join(PROFILES, "traffic_stream_collide_1024_replicas_blocked.json"),
}
TRAFFIC_FILE = TRAFFIC_FILES["plain"]
# the sources the D1Q3 step kernel is compiled from
KERNEL_SRCS = [os.path.join(ROOT, "paper_1706_01094_amd", "csrc", f)
               for f in ("kernels.hip", "rng.h", "device.h", "mom3_sum.h", "moments.h")]

# the D2Q9 step kernel: its sources and its counted VALU instructions per site
D2Q9_SRCS = [os.path.join(ROOT, "paper_1706_01094_amd", "csrc", f)
             for f in ("kernels_d2q9.hip", "rng.h", "device.h", "d2q9.h")]
D2Q9_VALU_FILE = os.path.join(PROFILES, "valu_d2q9_4096x4096.json")
# VALU issue of MI355X: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD
# every 4 cycles (16 lanes wide), 2.4 GHz
VALU_PEAK_G = 256 * 4 / 4 * 2.4


def kernel_hash(paths=None) -> str:
    h = hashlib.sha256()
    for path in paths or KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counter_record(which: str, steps_per_launch: int = 1):
    """The committed rocprofv3 counter record of this workload, if it was
    taken on the current kernel source with launches of the same number of
    steps."""
    try:
        with open(TRAFFIC_FILES[which]) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    return d if d.get("steps_per_launch", 1) == steps_per_launch else None


def measured_traffic(which: str = "plain", steps_per_launch: int = 1):
    """Memory-side bytes per launch from the committed counter runs, or None."""
    d = _counter_record(which, steps_per_launch)
    return None if d is None else d.get("bytes_per_launch")


def valu_issue_frac(which: str, seconds_per_launch: float, steps_per_launch: int = 1):
    """The step launch's VALU issue time (its counted VALU wave instructions
    at the 614.4 G/s issue peak) over its measured duration, or None."""
    d = _counter_record(which, steps_per_launch)
    if d is None or "sq_insts_valu_per_dispatch" not in d:
        return None
    return d["sq_insts_valu_per_dispatch"] / (VALU_PEAK_G * 1e9) / seconds_per_launch


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = None
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(budget_s: float = 15.0) -> dict:
    """The oracle (single-threaded C) on a bounded sample of the workload:
    a periodic lattice of 2^20 sites of the same density, velocity and seed,
    stepped until ~budget_s of CPU time."""
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
                      f"(rho=50, u0=0.1, C=10), {steps} steps timed after 1 warm-up step",
            "host": host_info()}


def _events(torch, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    return e0, e1


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
    info = {"expected_lds_fraction": round(cov, 5), "lds_bytes": lds_bytes,
            "state_bytes": 6 * L,
            "state_resident_in": "infinity cache (96 MiB of 256 MB)"
            if 6 * L <= INFINITY_CACHE_BYTES else "hbm"}
    K = args.blocked if not args.graph else 1
    if K > 1:
        lat.set_blocked(K)  # K steps per launch (temporal blocking)
    info["steps_per_launch"] = max(1, K)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = _events(torch, stream)
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
    if K > 1 and args.single_steps:
        # the same lattice with one step per launch, for comparison
        lat.set_blocked(1)
        lat.step(20)
        torch.cuda.synchronize()
        e0, e1 = _events(torch, stream)
        e0.record(stream)
        lat.step(args.single_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1) / args.single_steps
        info["single_step_launches"] = {
            "steps": args.single_steps, "ms_per_step": ms1,
            "site_updates_per_s": L / (ms1 / 1e3),
            "frac": BYTES_PER_SITE_UPDATE * L / (ms1 / 1e3) / 1e9 / HBM_PEAK_GBS}
    stats = plain_statistics(lat, args.stat_logs)
    lat.close()
    return L, gpu_ms, wall, info, stats


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

    def timed(steps):
        torch.cuda.synchronize()
        e0, e1 = _events(torch, lat.stream)
        e0.record(lat.stream)
        lat.step(steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # one step per launch: the kernel streams the state from HBM at every step
    ms = timed(args.probe_steps)
    blocked = None
    K = args.probe_blocked
    if K > 1:
        # several steps per launch in tiles (their copies go between the L2s
        # and the Infinity Cache): the state is read and written once per launch
        lat.set_blocked(K)
        lat.step(K)
        n = max(1, args.probe_steps // K) * K
        bms = timed(n)
        ach = BYTES_PER_SITE_UPDATE * L / (bms / 1e3) / 1e9
        btr = measured_traffic("probe_blocked", K)
        blocked = {"steps_per_launch": K, "steps": n, "ms_per_step": bms,
                   "site_updates_per_s": L / (bms / 1e3), "achieved_GBps": ach,
                   "frac": ach / HBM_PEAK_GBS,
                   "traffic_per_launch": btr,
                   "traffic_over_algorithmic": None if btr is None else
                   btr / (BYTES_PER_SITE_UPDATE * L * K),
                   "valu_issue_frac": valu_issue_frac("probe_blocked", bms * K / 1e3, K)}
    rc = lat.check()
    lat.close()
    if rc != 0:
        raise SystemExit(f"device error {rc} in the roofline probe")
    achieved = BYTES_PER_SITE_UPDATE * L / (ms / 1e3) / 1e9
    traffic = measured_traffic("probe")
    return {"workload": "d1q3_L128M_rho50_u0.1", "L": L, "steps": args.probe_steps,
            "state_resident_in": "hbm (768 MiB)",
            "ms_per_step": ms, "site_updates_per_s": L / (ms / 1e3),
            "achieved_GBps": achieved, "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_over_algorithmic": None if traffic is None else
            traffic / (BYTES_PER_SITE_UPDATE * L),
            "valu_issue_frac": valu_issue_frac("probe", ms / 1e3),
            "blocked": blocked}


def sk_twiddles(torch, Ls, n_modes: int, device):
    """int32 twiddles of S(k) for every replica, built on the device: replica
    r's block is [2 n_modes][L_r] with rows round(2^24 cos(2 pi m x / L_r)),
    round(2^24 sin(...)), m = 1..n_modes (input data of the moments call)."""
    Ls = [int(v) for v in Ls]
    total = sum(Ls)
    out = torch.empty(2 * n_modes * total, dtype=torch.int32, device=device)
    L_t = torch.tensor(Ls, dtype=torch.int64, device=device)
    rep = torch.repeat_interleave(torch.arange(len(Ls), device=device), L_t)
    dense = torch.cumsum(L_t, 0) - L_t
    x = torch.arange(total, dtype=torch.int64, device=device) - dense[rep]
    Lr = L_t[rep]
    base = 2 * n_modes * dense[rep] + x
    for m in range(1, n_modes + 1):
        ph = (2.0 * torch.pi) * ((m * x) % Lr).to(torch.float64) / Lr.to(torch.float64)
        s = float(1 << 24)
        out[base + (2 * (m - 1)) * Lr] = torch.round(s * torch.cos(ph)).to(torch.int32)
        out[base + (2 * (m - 1) + 1) * Lr] = torch.round(s * torch.sin(ph)).to(torch.int32)
    return out


def batched_observables(lat, torch, man, samples: int, every: int) -> dict:
    """After the timed steps: exact int64 per-replica sums every `every`
    steps -- mean and variance of n_i (Poisson: var/mean = 1) and the static
    structure factor S(k) = <|sum_x N(x) e^(i k x)|^2> / L for k = 2 pi m / L,
    m = 1..8, over all replicas (an ideal gas gives S(k) = rho)."""
    import numpy as np
    n_modes = 8
    tw = sk_twiddles(torch, man["L"], n_modes, lat.device)
    L = man["L"].astype(np.float64)
    rho = man["rho"]
    vm = []
    sk = np.zeros((samples, len(L), n_modes))
    for k in range(samples):
        lat.step(every)
        ms = lat.moments(tw, n_modes)
        v = np.zeros(3)
        for r, m in enumerate(ms):
            mean = np.array(m["sum_n"], dtype=np.float64) / L[r]
            var = np.array(m["sum_n2"], dtype=np.float64) / L[r] - mean ** 2
            v += var / mean
            f = np.array(m["fourier"][:n_modes], dtype=np.float64) / float(1 << 24)
            sk[k, r] = (f[:, 0] ** 2 + f[:, 1] ** 2) / L[r] / rho[r]
        vm.append(v / len(ms))
    del tw
    # the long-wavelength modes change little between samples, so the
    # standard error is taken over the independent replicas (each replica's
    # mean over its samples)
    per_rep = sk.mean(0)
    return {"samples": samples, "every": every, "replicas": len(man["L"]),
            "var_over_mean": [round(float(x), 5) for x in np.array(vm).mean(0)],
            "S_k_over_rho": [round(float(x), 4) for x in per_rep.mean(0)],
            "S_k_over_rho_se": [round(float(x), 4) for x in per_rep.std(0, ddof=1) /
                                np.sqrt(per_rep.shape[0])]}


def run_batched(args, torch, M):
    """1024 independent replicas of uneven L and density: plain per-replica
    launches vs one batched launch per step vs captured HIP graphs."""
    import synth
    from paper_1706_01094_amd import autotune
    man = synth.replica_manifest()
    sites = int(man["L"].sum())
    lat = M.Lattice(man["L"], synth.BATCHED["seed"], rho=man["rho"], u0=man["u0"],
                    replica_id=man["replica_id"])
    if args.batched_schedule == "auto":
        tuned = autotune.tune(man["L"], man["rho"], man["u0"], replica_id=man["replica_id"],
                              steps=10, use_cache=False)
    else:  # a given schedule (profiling runs: no tuning launches)
        tuned = {"schedule": tuple(int(v) for v in args.batched_schedule.split(",")),
                 "trials": []}
    lat.set_schedule(*tuned["schedule"])
    out = {"workload": "d1q3_1024_replicas", "replicas": len(man["L"]), "sites": sites,
           "state_bytes": int(lat.state_bytes), "schedule": list(tuned["schedule"]),
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
        rate = sites * args.batched_steps / (ms / 1e3)
        out[mode] = {"steps": args.batched_steps, "ms": ms, "us_per_step":
                     1e3 * ms / args.batched_steps, "site_updates_per_s": rate,
                     "hbm_frac": BYTES_PER_SITE_UPDATE * rate / 1e9 / HBM_PEAK_GBS}
    # several steps per launch: each block advances whole replicas, K steps
    # on copies in the caches (the state is read and written once per launch)
    K = args.batched_blocked
    out["blocked"] = None
    if K > 1:
        try:
            lat.set_blocked(K)
        except M.MclgError as e:  # (a schedule other than 1024 threads)
            out["blocked"] = {"refused": str(e)}
        else:
            lat.step(K)
            nb = max(1, args.batched_steps // K) * K
            torch.cuda.synchronize()
            e0, e1 = _events(torch, lat.stream)
            e0.record(lat.stream)
            lat.step(nb)
            e1.record(lat.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            rate = sites * nb / (ms / 1e3)
            btr = measured_traffic("batched_blocked", K)
            out["blocked"] = {"steps_per_launch": K, "steps": nb, "ms": ms,
                              "us_per_step": 1e3 * ms / nb, "site_updates_per_s": rate,
                              "hbm_frac": BYTES_PER_SITE_UPDATE * rate / 1e9 / HBM_PEAK_GBS,
                              "traffic_per_launch": btr,
                              "traffic_over_algorithmic": None if btr is None else
                              btr / (BYTES_PER_SITE_UPDATE * sites * K),
                              "valu_issue_frac": valu_issue_frac("batched_blocked",
                                                                 ms / 1e3 * K / nb, K)}
            lat.set_blocked(1)
    traffic = measured_traffic("batched")
    out["traffic"] = traffic
    out["traffic_over_algorithmic"] = None if traffic is None else \
        traffic / (BYTES_PER_SITE_UPDATE * sites)
    out["valu_issue_frac"] = valu_issue_frac("batched", out["batched"]["us_per_step"] / 1e6)
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
    if args.batched_samples:
        out["observables"] = batched_observables(lat, torch, man, args.batched_samples, 100)
    out["t"] = int(lat.moments()[0]["t"])
    lat.close()
    return out


def run_wave(args, torch, M):
    """Decaying density wave, L = 2^22, 5000 steps, the int64 Fourier
    projection of the density every 10 steps, logged on the device (one
    mclg_step_log call writes the 500 records into a device array; the host
    reads them once).  A(t) is Eq. (A)'s least-squares
    amplitude of the profile N(x) against sin(2 pi x / L)."""
    import numpy as np
    import synth
    w = synth.DENSITY_WAVE
    L = w["L"]
    counts = synth.density_wave_counts()
    tw = synth.twiddles(L, 1)
    K = args.wave_blocked
    words = ct.sizeof(M.mclg_moments_t) // 8
    # a throwaway lattice warms the launch paths; the timed run starts at t = 0
    warm = M.Lattice(L, w["seed"], counts=counts)
    if K > 1:
        warm.set_blocked(K)
    twd = torch.as_tensor(tw).to(warm.device)
    junk = torch.zeros((2 * max(1, K // w["log_every"]), words), dtype=torch.int64,
                       device=warm.device)
    warm.stream.wait_stream(torch.cuda.current_stream(warm.device))
    warm.step_log(w["log_every"], junk.shape[0], junk, twd, 1)
    warm.stream.synchronize()
    warm.close()
    del warm
    lat = M.Lattice(L, w["seed"], counts=counts)
    if K > 1:
        lat.set_blocked(K)  # launches of K steps, each summing the logs in it
    logs = w["steps"] // w["log_every"]
    rec = torch.zeros((logs, words), dtype=torch.int64, device=lat.device)
    lat.stream.wait_stream(torch.cuda.current_stream(lat.device))
    torch.cuda.synchronize()
    e0, e1 = _events(torch, lat.stream)
    t0 = time.perf_counter()
    e0.record(lat.stream)
    # the whole run: 500 intervals of 10 steps, each followed by the moments
    # of the state it reaches
    lat.step_log(w["log_every"], logs, rec, twd, 1)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    host = rec.cpu().numpy()
    lat.close()
    # field offsets (in int64 words) of the record
    off_sin = (M.mclg_moments_t.fourier.offset // 8) + 1
    off_t = M.mclg_moments_t.t.offset // 8
    # Eq. (A): A = sum_x sin(2 pi x / L) N(x) / sum_x sin^2(2 pi x / L); the
    # twiddles are s(x) = round(2^24 sin), so A = 2^24 sum N s / sum s^2
    ss = float(np.sum(tw[1].astype(np.float64) ** 2))
    amp = host[:, off_sin].astype(np.float64) * float(1 << 24) / ss
    return {"workload": "d1q3_L4M_wave_rho40", "steps": w["steps"], "logs": logs,
            "steps_per_launch": max(1, K), "gpu_ms": ms, "wall_s": wall,
            "site_updates_per_s_incl_logging": L * w["steps"] / (ms / 1e3),
            "amplitude_expected_initial": w["rho"] * w["amp"],
            "amplitude_first": float(amp[0]), "amplitude_last": float(amp[-1]),
            "t_first": int(host[0, off_t]), "t_last": int(host[-1, off_t])}


def _serve(M, torch, jobs, arena_bytes, max_slots, seed, k, window, time_limit):
    """Real-time driver: jobs are submitted when their arrival time has
    passed; the server advances all resident jobs k steps per tick."""
    srv = M.Server(arena_bytes, max_slots, seed)
    t0 = time.perf_counter()
    nxt = 0
    done = {}
    backlog = None
    while len(done) < len(jobs):
        now = time.perf_counter() - t0
        if now > time_limit:
            break
        while nxt < len(jobs) and jobs[nxt]["arrival"] <= now:
            j = jobs[nxt]
            srv.submit(j["job_id"], j["L"], j["steps"], j["rho"], j["u0"])
            nxt += 1
        q, r, _ = srv.stats()
        if backlog is None and now >= window:
            backlog = {"queued": int(q), "resident": int(r), "completed": len(done)}
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
            "backlog_at_window_end": backlog,
            "p50_latency_s": pct(0.5), "p99_latency_s": pct(0.99),
            "site_updates_per_s": work / span if span > 0 else 0.0,
            "span_s": span, "site_updates": work}


def run_served(args, torch, M, capacity):
    """Poisson arrivals (200 jobs/s) of jobs with L log-uniform in
    [2^12, 2^24], steps U{100..5000}, rho U{5..100}; 200 GB arena.  The
    offered work exceeds the device's capacity by design, so latency grows
    with the arrival window; a second trace arrives at 0.8 x the measured
    batched capacity."""
    import synth
    cfg = synth.SERVED
    out = {"workload": "d1q3_served_200_per_s", "arena_bytes": cfg["budget"]}
    jobs = synth.job_trace(args.serve_window)
    offered = sum(j["L"] * j["steps"] for j in jobs) / args.serve_window
    out["trace"] = {"window_s": args.serve_window, "jobs": len(jobs),
                    "offered_site_updates_per_s": offered}
    out["overloaded"] = _serve(M, torch, jobs, cfg["budget"], 8192, cfg["seed"], 50,
                               args.serve_window, args.serve_limit)
    mean_work = offered / cfg["rate"]
    rate = 0.8 * capacity / mean_work
    jobs2 = synth.job_trace(args.serve_window, rate=rate, seed=cfg["seed"] + 1)
    out["sustainable"] = {"rate_jobs_per_s": rate, "window_s": args.serve_window,
                          "jobs": len(jobs2),
                          **_serve(M, torch, jobs2, cfg["budget"], 8192, cfg["seed"], 50,
                                   args.serve_window, args.serve_limit)}
    return out


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


def run_bound(args, torch, M):
    """What bounds the blocked step: the headline lattice (L = 2^24, `--blocked`
    steps per launch) at the headline density, at lower densities (fewer
    misses of the LDS image) and with no collisions at all (C = 0: the
    kernel only streams the blocks' copies), each timed over `--bound-steps`
    steps after one warm-up launch."""
    import synth
    w = synth.PLAIN_LARGE
    L, K = w["L"], max(2, args.blocked)
    out = {"L": L, "steps_per_launch": K, "cases": []}
    for C, rho, u0 in ((10, w["rho"], w["u0"]), (10, 20.0, 0.0), (10, 5.0, 0.0), (0, w["rho"], w["u0"])):
        lat = M.Lattice(L, w["seed"], C=C, lam=(1, 1), n_max=255, rho=rho, u0=u0)
        lat.set_blocked(K)
        lat.step(K)
        n = max(1, args.bound_steps // K) * K
        torch.cuda.synchronize()
        e0, e1 = _events(torch, lat.stream)
        e0.record(lat.stream)
        lat.step(n)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        out["cases"].append({"C": C, "rho": rho, "u0": u0, "steps": n, "us_per_step": ms * 1e3,
                             "site_updates_per_s": L / (ms / 1e3),
                             "frac": BYTES_PER_SITE_UPDATE * L / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                             "check": lat.check()})
        lat.close()
    return out


def run_moments(args, torch, M):
    """The moment kernels alone (for kernel traces): exact moments of the
    L = 2^24 lattice (no modes), of the L = 2^22 density wave (one mode), and
    of the 4096 x 4096 D2Q9 lattice, 20 calls each."""
    import synth
    out = {}
    w = synth.PLAIN_LARGE
    lat = M.Lattice(w["L"], w["seed"], rho=w["rho"], u0=w["u0"])
    t0 = time.perf_counter()
    for _ in range(20):
        lat.moments()
    out["d1q3_L16M"] = {"calls": 20, "wall_ms_per_call": (time.perf_counter() - t0) * 50}
    lat.close()
    wv = synth.DENSITY_WAVE
    lat = M.Lattice(wv["L"], wv["seed"], counts=synth.density_wave_counts())
    twd = torch.as_tensor(synth.twiddles(wv["L"], 1)).to(lat.device)
    t0 = time.perf_counter()
    for _ in range(20):
        lat.moments(twd, 1)
    out["d1q3_L4M_one_mode"] = {"calls": 20, "wall_ms_per_call": (time.perf_counter() - t0) * 50}
    lat.close()
    lat = M.Lattice9(4096, 4096, 9, C=10, rho=36.0, ux=0.0, uy=0.0)
    t0 = time.perf_counter()
    for _ in range(20):
        lat.moments()
    out["d2q9_4096x4096"] = {"calls": 20, "wall_ms_per_call": (time.perf_counter() - t0) * 50}
    lat.close()
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
                    help="only the plain headline (skip the other workloads)")
    ap.add_argument("--only", default="",
                    choices=["", "plain", "probe", "batched", "wave", "served", "d2q9", "moments",
                             "bound"],
                    help="run one workload and print its result")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--batched-warmup", type=int, default=20)
    ap.add_argument("--batched-schedule", default="auto",
                    help="'auto' (autotuned) or groups,threads,lds_bytes")
    ap.add_argument("--batched-samples", type=int, default=10,
                    help="S(k) and var/mean samples after the timed batched steps")
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--probe-steps", type=int, default=200)
    ap.add_argument("--stat-logs", type=int, default=10)
    ap.add_argument("--blocked", type=int, default=256,
                    help="steps per launch of the L = 2^24 workload (temporal blocking; 1: off)")
    ap.add_argument("--single-steps", type=int, default=2000,
                    help="steps of the one-step-per-launch comparison of the blocked run")
    ap.add_argument("--batched-blocked", type=int, default=128,
                    help="steps per launch of the batched run's blocked variant (1: off)")
    ap.add_argument("--probe-blocked", type=int, default=128,
                    help="steps per launch of the L = 2^27 probe's blocked run, in tiles "
                         "(1: off)")
    ap.add_argument("--wave-blocked", type=int, default=250,
                    help="steps per launch of the density wave (each launch sums the logs "
                         "that fall in it; 1: off)")
    ap.add_argument("--serve-window", type=float, default=10.0)
    ap.add_argument("--serve-limit", type=float, default=120.0)
    ap.add_argument("--bound-steps", type=int, default=1024,
                    help="steps per case of --only bound")
    ap.add_argument("--d2q9-steps", type=int, default=50)
    ap.add_argument("--d2q9-warmup", type=int, default=5)
    ap.add_argument("--d2q9-only", action="store_true", help="same as --only d2q9")
    ap.add_argument("--batched-only", action="store_true", help="same as --only batched")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run 8 device-to-device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.d2q9_only:
        args.only = "d2q9"
    if args.batched_only:
        args.only = "batched"
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
        print("bench.py measures one GPU only: the lattice and replica work runs on a "
              "single MI355X; sharding a lattice or a batch across GPUs is not implemented.",
              file=sys.stderr)
        raise SystemExit(2)
    import torch
    from paper_1706_01094_amd import mclg as M
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")

    legs = {"probe": run_probe, "batched": run_batched, "wave": run_wave,
            "d2q9": run_d2q9, "moments": run_moments, "bound": run_bound}
    if args.only in legs:
        print(json.dumps({args.only: legs[args.only](args, torch, M)}), flush=True)
        return
    if args.only == "served":
        cap = run_batched(args, torch, M)["batched"]["site_updates_per_s"]
        print(json.dumps({"served": run_served(args, torch, M, cap)}), flush=True)
        return
    L, gpu_ms, wall, info, stats = run_plain(args, torch, M)
    ms_per_step = gpu_ms / args.steps
    value = L * args.steps / (gpu_ms / 1e3)
    achieved = BYTES_PER_SITE_UPDATE * L / (ms_per_step / 1e3) / 1e9
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
                   "schedule": args.schedule or "default", **info},
        # the dominant kernel's launches: K steps each (12 B per site update
        # algorithmic, K L site updates per launch); traffic per launch
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "steps_per_launch": info["steps_per_launch"],
                     "traffic": measured_traffic("plain", info["steps_per_launch"]),
                     "valu_issue_frac": valu_issue_frac(
                         "plain", ms_per_step * info["steps_per_launch"] / 1e3,
                         info["steps_per_launch"])},
        "statistics": stats,
    }
    if args.only == "plain":
        args.no_extra = True
    if not args.no_extra:
        extra = {}
        extra["roofline_probe"] = run_probe(args, torch, M)
        torch.cuda.empty_cache()
        extra["bound"] = run_bound(args, torch, M)
        torch.cuda.empty_cache()
        extra["batched"] = run_batched(args, torch, M)
        torch.cuda.empty_cache()
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
