"""Benchmark: batched parametric source iteration with synthetic acceleration on one MI355X.

One step = one batched solve (Alg. 1 with the ROMSAD switch of Alg. 2 by default) of the
parametric lattice batch: 256 instances, 128 x 128 Q1 mesh, 64 directions on the unit circle,
per-block sigma_s ~ U[0.5, 50], sigma_a ~ U[0.001, 1], FP32 sweep / FP64 corrections,
relative tolerance 1e-6.  Inputs are seeded synthetic materials resident in HBM before timing.
The sweep schedule is the autotuner's measured pick for this workload.

Further legs (reported beside the headline value, never as it):
  - plain single-instance GPU SI-DSA on the same instances (the comparison baseline), and the
    same batch solved by batched SI-DSA (what ROMSAD saves apart from batching);
  - the paper's Krylov baseline (DSA-preconditioned GMRES) on part of the batch;
  - the f-form sweep (rte_sweep writing the FP32 angular flux) against the HBM roofline;
  - the single-instance checkerboard (128^2, 64 directions): plain SI and SI-DSA in FP64 and
    mixed precision, with the mixed results' error against a tight FP64 solution;
  - the large multiscale instance (512^2, 256 directions): ROMSAD with a rank-40 ROM from 64
    training solves, then SI-DSA alone, and the f-form sweep at that size;
  - a served stream: seeded Poisson arrivals of lattice requests with meshes {64,128,256}^2 and
    {32,64,128} directions, ROMSAD with a correction ROM per (mesh, directions) key, continuous
    batching; solves/s and p50/p99 latency, and the same requests replayed through the plain
    single-instance GPU SI-DSA;
  - the CPU oracle on bounded samples of the batch (with the oracle's own ROM from the same 32
    training solves), the checkerboard, the multiscale instance and the stream.

Prints one JSON line.  The sweep kernel's roofline comes from HIP events recorded by the library
around every sweep launch inside the timed region.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic work of one cell-direction update of the 2D sweep: 16 flops for the inflow
# right-hand side, 32 for the 4 x 4 solve with the inverse held per (direction, material), 8 for
# the outflow traces, 8 for the density accumulation.  The kernel holds the solve's
# sigma_t-dependent coefficients per (direction, material) and folds the divisions into them:
# 58 flops per update (its per-cell closed form, for media of more than 16 materials, costs 88);
# that figure is reported beside it.
SWEEP_FLOPS_PER_CD = 64
SWEEP_FLOPS_PER_CD_KERNEL = 58
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}     # MI355X published vector peaks (FP32, FP64)
PEAK_HBM_GBS = 8000.0
METRIC = "cell-dir updates/s; solves/s + p50/p99 latency @1e-6 vs plain GPU SI-DSA"
# HBM traffic of the sweep kernel measured with rocprofv3 counters (FETCH_SIZE, WRITE_SIZE),
# valid only while the kernel source is the one the counters were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep2d_c2_batch_traffic.json")
# the sources the sweep kernel is compiled from (its own file and the shared layout header)
SWEEP_SRCS = [os.path.join(ROOT, "paper_2402_10488_amd", "csrc", n)
              for n in ("sweep.hip", "rte_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_rom(P_train_plane, P_test, rte, problems, args):
    from paper_2402_10488_amd import offline
    t0 = time.perf_counter()
    rom_arrays = offline.build_correction_rom(P_train_plane, r=args.rank, window=args.window,
                                              eps_train=args.eps_train)
    Rm = rte.Rom(P_test, rom_arrays.U_rho, rom_arrays.U_iso, rom_arrays.A0, rom_arrays.A,
                 rom_arrays.eps_pod, rom_arrays.eps_train)
    log(f"[bench] correction ROM r={args.rank} window={args.window} built on the GPU in "
        f"{time.perf_counter() - t0:.1f}s (eps_pod={rom_arrays.eps_pod:.3e})")
    return Rm, rom_arrays


class OracleRomJob:
    """The oracle's correction ROM of the batch's training instances (the same 32 seeds the GPU
    ROM is built from), built on the host by a pool of oracle processes in the background while
    the GPU legs run, and saved as an .npz file for the CPU baseline's oracle processes."""

    def __init__(self, args, procs):
        import subprocess
        import tempfile
        self.dir = tempfile.mkdtemp(prefix="rte_oracle_rom_")
        self.path = os.path.join(self.dir, "c2_rom.npz")
        cfg = {"spec": ["c2_training", [args.n_train, args.n, args.nphi]], "n_train": args.n_train,
               "window": args.window, "eps_train": args.eps_train, "rank": args.rank,
               "procs": procs, "out": self.path}
        env = dict(os.environ, OMP_NUM_THREADS=str(procs), OPENBLAS_NUM_THREADS=str(procs),
                   MKL_NUM_THREADS=str(procs))
        self.t0 = time.perf_counter()
        self.proc = subprocess.Popen([sys.executable, "-m", "oracle.pool", "build-rom",
                                      json.dumps(cfg)], cwd=ROOT, env=env,
                                     stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        self.seconds = None

    def wait(self, timeout_s=900.0):
        import subprocess
        t_end = time.perf_counter() + timeout_s
        while True:
            try:
                out, _ = self.proc.communicate(timeout=20.0)
                break
            except subprocess.TimeoutExpired:
                if time.perf_counter() > t_end:
                    raise
                log(f"[bench] waiting for the oracle ROM ({time.perf_counter() - self.t0:.0f}s)")
        self.seconds = time.perf_counter() - self.t0
        if self.proc.returncode != 0 or not os.path.exists(self.path):
            raise RuntimeError(f"oracle ROM build failed: {out[-2000:]}")
        return self.path

    def close(self):
        import shutil
        if self.proc.poll() is None:
            self.proc.kill()
        shutil.rmtree(self.dir, ignore_errors=True)


def cpu_baseline(args, mode, rom_path):
    """The oracle as it stands, timed on the host on bounded samples of the batch: one instance
    on one core, and one instance per host core started together."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import rte_workloads as W
    from oracle.problem import discretize
    from oracle.sisa import sisa
    from oracle import pool as opool
    plane = W.c2_lattice([20000], n=args.n, n_phi=args.nphi)
    d = discretize(plane, 0)
    rom = opool.load_rom(rom_path) if mode == "romsad" else None
    t0 = time.perf_counter()
    res = sisa(d, "romsad" if mode == "romsad" else mode, eps=args.eps, rom=rom, theta=args.theta)
    dt = time.perf_counter() - t0
    cd = d.nc * d.nv * res.n_sweep
    rom_note = (f"; the oracle's ROM (rank {args.rank}, window {args.window}) from the same "
                f"{args.n_train} training solves as the GPU's, built untimed") if mode == "romsad" else ""
    one = {"value": cd / dt, "cores": 1, "solves_per_s": 1.0 / dt,
           "sample": f"1 instance (seed 20000) of the {args.n}x{args.n} lattice, {args.nphi} "
                     f"directions, {mode}, FP64, tol {args.eps:g}: {res.n_sweep} sweeps in "
                     f"{dt:.1f}s{rom_note}"}
    k = host_cores() if args.cpu_cores <= 0 else args.cpu_cores
    if k <= 1:
        return dict(one, unit="cell-dir updates/s", kind="oracle")
    allc = cpu_all_cores(args, mode, k, rom_path)
    return {"value": allc["value"], "unit": "cell-dir updates/s", "cores": k, "kind": "oracle",
            "sample": f"{k} instances (seeds 20000-{20000 + k - 1}) of the {args.n}x{args.n} "
                      f"lattice, {args.nphi} directions, {mode}, FP64, tol {args.eps:g}, one oracle "
                      f"process per host core started together: {sum(allc['sweeps'])} sweeps in "
                      f"{allc['wall_s']:.1f}s wall{rom_note}",
            "solves_per_s": allc["solves_per_s"], "mean_sweeps": float(np.mean(allc["sweeps"])),
            "one_core": one}


# One oracle instance per host process, for the all-cores CPU baseline: builds its inputs and
# loads the oracle's ROM untimed, reports "ready", waits for a line on stdin, then times its
# solve.  Runs the oracle only (numpy/scipy and the oracle's C sweep); it never touches the GPU.
CPU_WORKER = r"""
import json, sys, time
cfg = json.loads(sys.argv[1])
sys.path.insert(0, cfg["root"])
import rte_workloads as W
from oracle.problem import discretize
from oracle.sisa import sisa
from oracle import pool
plane = W.c2_lattice([cfg["seed"]], n=cfg["n"], n_phi=cfg["nphi"])
d = discretize(plane, 0)
rom = pool.load_rom(cfg["rom"]) if cfg["mode"] == "romsad" else None
print("ready", flush=True)
sys.stdin.readline()
t0 = time.perf_counter()
res = sisa(d, cfg["mode"], eps=cfg["eps"], rom=rom, theta=cfg["theta"])
dt = time.perf_counter() - t0
print(json.dumps({"cd": d.nc * d.nv * res.n_sweep, "n_sweep": res.n_sweep, "s": dt}), flush=True)
"""


def host_cores():
    """Host cores this process may use, capped at 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_all_cores(args, mode, k, rom_path, timeout_s=300.0):
    """k oracle processes, one instance each (seeds 20000 .. 20000 + k - 1), started together
    once every process has built its inputs: aggregate cell-direction updates/s over the wall
    time from the start signal to the last finish."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = []
    try:
        for i in range(k):
            cfg = {"root": ROOT, "seed": 20000 + i, "n": args.n, "nphi": args.nphi,
                   "mode": "romsad" if mode == "romsad" else mode, "eps": args.eps,
                   "theta": args.theta, "rom": rom_path}
            procs.append(subprocess.Popen([sys.executable, "-c", CPU_WORKER, json.dumps(cfg)],
                                          stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                                          text=True, env=env))
        for p in procs:
            if p.stdout.readline().strip() != "ready":
                raise RuntimeError("oracle worker failed before its solve")
        t0 = time.perf_counter()
        for p in procs:
            p.stdin.write("go\n")
            p.stdin.flush()
        res = [json.loads(p.stdout.readline()) for p in procs]
        wall = time.perf_counter() - t0
        for p in procs:
            p.wait(timeout=timeout_s)
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
    cd = sum(r["cd"] for r in res)
    return {"value": cd / wall, "wall_s": wall, "solves_per_s": k / wall,
            "sweeps": [r["n_sweep"] for r in res]}


def cpu_c1(args):
    """The oracle on the single-instance checkerboard, one core: SI-DSA, FP64, tol 1e-8."""
    import rte_workloads as W
    from oracle.problem import discretize
    from oracle.sisa import sisa
    d = discretize(W.c1_checkerboard(), 0)
    t0 = time.perf_counter()
    res = sisa(d, "si_dsa", eps=1e-8)
    dt = time.perf_counter() - t0
    return {"value": d.nc * d.nv * res.n_sweep / dt, "unit": "cell-dir updates/s", "cores": 1,
            "kind": "oracle", "solves_per_s": 1.0 / dt,
            "sample": f"the 128x128 checkerboard, 64 directions, si_dsa, FP64, tol 1e-8: "
                      f"{res.n_sweep} sweeps in {dt:.1f}s (one core)"}


def cpu_c4(args):
    """The oracle's transport sweep of the 512^2, 256-direction multiscale instance, one core
    (a whole solve takes hundreds of sweeps: one sweep is the bounded sample)."""
    import rte_workloads as W
    from oracle.problem import discretize
    d = discretize(W.c4_multiscale(), 0)
    rho = np.zeros(d.ndof)
    t0 = time.perf_counter()
    d.sweep(rho)
    dt = time.perf_counter() - t0
    return {"value": d.nc * d.nv / dt, "unit": "cell-dir updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 sweep of the 512x512, 256-direction multiscale instance "
                      f"({d.nc * d.nv} cell-direction updates) in {dt:.1f}s (one core)"}


def cpu_c3(args, budget_s=20.0):
    """The oracle replaying the stream's requests first come, first served on one core (SI-DSA,
    FP64: the oracle has no per-key ROMs), until about budget_s seconds of work."""
    import rte_workloads as W
    from oracle.problem import discretize
    from oracle.sisa import sisa
    reqs = W.c3_requests(args.serve_requests + args.serve_warmup)[args.serve_warmup:]
    t0 = time.perf_counter()
    cd, n = 0, 0
    for r in reqs:
        d = discretize(W.c2_lattice([r.seed], n=r.n, n_phi=r.n_phi, left_inflow=True), 0)
        res = sisa(d, "si_dsa", eps=args.eps)
        cd += d.nc * d.nv * res.n_sweep
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": cd / dt, "unit": "cell-dir updates/s", "cores": 1, "kind": "oracle",
            "solves_per_s": n / dt,
            "sample": f"the first {n} timed requests of the stream, first come first served, "
                      f"si_dsa (no ROM), FP64, tol {args.eps:g}, in {dt:.1f}s (one core)"}


def sweep_source_hash():
    h = hashlib.sha256()
    for path in SWEEP_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(launch_cd):
    """HBM bytes per launch from the committed counter summary, scaled to this launch's work
    (None when the summary is absent or the kernel changed since the counters were taken)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sweep_src_sha256_16") != sweep_source_hash():
        return None
    return t["hbm_bytes_per_cd"] * launch_cd


def f_form_leg(P, rte, reps=5):
    """rte_sweep writing the FP32 angular flux of the whole batch: HBM roofline of the f-form."""
    import torch
    f = torch.empty(rte.f_shape(P), dtype=torch.float32, device="cuda")
    rho = torch.rand((P.B, P.ndof), dtype=torch.float64, device="cuda")
    ws = P.workspace("si", None, "mixed")
    rte.sweep(P, rho, f_out=f, precision="mixed", ws=ws)
    torch.cuda.synchronize()
    rte.profile_enable(True)
    for _ in range(reps):
        rte.sweep(P, rho, f_out=f, precision="mixed", ws=ws)
    torch.cuda.synchronize()
    ms, n = rte.profile_read("sweep2d")
    rte.profile_enable(False)
    ms /= max(n, 1)
    cd = P.B * P.ncell * P.n_dir
    # algorithmic bytes: the FP32 angular flux (4 dofs x 4 B per cell-direction) plus the sweep
    # input block read once (source and sigma_t in two diagonal layouts, 10 x 4 B per cell)
    nbytes = cd * 16 + P.B * P.ncell * 40
    gbs = nbytes / (ms * 1e-3) / 1e9
    del f
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "traffic": None, "kernel": "sweep2d_kernel (f-form)",
            "avg_launch_ms": ms, "bytes_per_launch": nbytes,
            "cell_dir_updates_per_s": cd / (ms * 1e-3)}


def residual_inf(P, rte, rho):
    """Per-instance R = |rho - (L rho + b_bar)|_inf / |rho|_inf after convergence: one FP64 sweep
    of the converged density (the residual the paper tabulates next to every method)."""
    import torch
    rs = torch.empty_like(rho)
    rte.sweep(P, rho, rho_star_out=rs, precision="fp64")
    d = (rs - rho).abs().amax(dim=1) / rho.abs().amax(dim=1)
    return d.cpu().numpy()


def pgmres_leg(args, plane, rte, problems, romsad_solves_per_s):
    """The paper's Krylov baseline on the first instances of the batch: DSA-preconditioned
    GMRES(25) to a preconditioned relative residual of eps, FP64 (same diffusion CG)."""
    import torch
    k = min(args.pgmres_instances, plane.B)
    sub = plane.subset(range(k))
    Pg = problems.plane_problem(sub)
    ws = Pg.pgmres_workspace(25)
    rho = torch.zeros((Pg.B, Pg.ndof), dtype=torch.float64, device="cuda")
    rte.pgmres_solve(Pg, rho, tol=args.eps, restart=25, cg_rtol=args.cg_rtol, ws=ws)   # warm
    rho.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = rte.pgmres_solve(Pg, rho, tol=args.eps, restart=25, cg_rtol=args.cg_rtol, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sps = Pg.B / dt
    R = residual_inf(Pg, rte, rho)
    return {"instances": Pg.B, "solves_per_s": sps, "mean_sweeps": float(r.n_sweep.mean()),
            "residual_inf_median": float(np.median(R)), "residual_inf_max": float(R.max()),
            "mean_iterations": float(r.iterations.mean()), "not_converged": int((r.inst_status != 0).sum()),
            "romsad_batch_vs_pgmres": romsad_solves_per_s / sps, "precision": "fp64",
            "note": "ratio of the headline batch's solves/s (mixed) to PGMRES solves/s (FP64) on "
                    "the first instances of the same batch"}


SERVE_KEYS = [(n, p) for n in (64, 128, 256) for p in (32, 64, 128)]


def serve_capacity(n, n_phi, batch_mcd=256, lo=16, hi=64):
    """Slots of a key's pool: about batch_mcd million cell-direction updates per batched sweep,
    lo..hi slots."""
    return int(min(hi, max(lo, (batch_mcd << 20) // (n * n * n_phi))))


def serving_leg(args, rte):
    """Seeded Poisson stream through per-key slot pools (continuous batching), ROMSAD at eps."""
    import torch
    import rte_workloads as W
    from paper_2402_10488_amd import offline, serving
    t0 = time.perf_counter()
    roms = {}
    for (n, p) in SERVE_KEYS:
        train = W.c3_training(n, p, args.serve_train)
        roms[(n, p)] = offline.build_correction_rom(train, r=args.rank, window=args.window,
                                                    eps_train=args.eps_train)
        torch.cuda.empty_cache()
    t_rom = time.perf_counter() - t0
    cap = {k: serve_capacity(*k, args.serve_batch_mcd, args.serve_min_slots, args.serve_max_slots)
           for k in SERVE_KEYS}
    pools = {k: serving.KeyPool(k[0], k[1], cap[k], "romsad", roms[k],
                                precision=args.precision, eps=args.eps, theta=args.theta,
                                cg_rtol=args.cg_rtol, iters_per_round=args.serve_iters_per_round,
                                graph_cg_iters=args.serve_graph_cg_iters)
             for k in SERVE_KEYS}
    budget = int(args.serve_budget_gib * 2**30)
    n_all = args.serve_requests + args.serve_warmup

    def stream_at(rate):
        """The request stream (seeded draws) with Poisson arrivals at ``rate`` (inf: all at 0)."""
        reqs = W.c3_requests(n_all, rate=rate if np.isfinite(rate) else 1.0)
        out = [serving.lattice_request(i, r.arrival, r.n, r.n_phi, r.seed) for i, r in enumerate(reqs)]
        warm, timed = out[:args.serve_warmup], out[args.serve_warmup:]
        t_start = timed[0].arrival
        timed = [serving.Request(k, (r.arrival - t_start) if np.isfinite(rate) else 0.0, r.n,
                                 r.n_phi, r.sigma_t, r.sigma_s, r.G, r.g, r.psi)
                 for k, r in enumerate(timed)]
        return warm, timed

    log(f"[bench] serving: nine key ROMs built in {t_rom:.1f}s")
    warm, saturated = stream_at(float("inf"))
    if warm:
        serving.Server(pools, budget).run([serving.Request(k, 0.0, r.n, r.n_phi, r.sigma_t,
                                                           r.sigma_s, r.G, r.g, r.psi)
                                           for k, r in enumerate(warm)])
    # capacity: every request queued at t = 0 (closed loop, the pools stay full)
    srv = serving.Server(pools, budget)
    if args.trace_gap > 0:                 # idle gaps that bracket the stream in a kernel trace
        torch.cuda.synchronize()
        time.sleep(args.trace_gap)
        log(f"[bench] serving stream starts at monotonic {time.monotonic_ns()} ns")
    tw = time.perf_counter()
    res_sat = srv.run(saturated)
    sat = serving.latency_summary(res_sat, time.perf_counter() - tw)
    if args.trace_gap > 0:
        log(f"[bench] serving stream ends at monotonic {time.monotonic_ns()} ns")
        time.sleep(args.trace_gap)
    log(f"[bench] serving saturated: {json.dumps(sat)}")
    # latency: open-loop Poisson arrivals at a rate below capacity
    rate = args.serve_rate if args.serve_rate > 0 else 0.8 * sat["solves_per_s"]
    _, timed = stream_at(rate)
    srv = serving.Server(pools, budget)
    tw = time.perf_counter()
    res = srv.run(timed)
    out = serving.latency_summary(res, time.perf_counter() - tw)
    out.update({"rate_req_per_s": rate, "saturated": sat, "keys": len(SERVE_KEYS),
                "capacity": {f"{k[0]}x{k[0]}/{k[1]}": cap[k] for k in SERVE_KEYS},
                "budget_gib": args.serve_budget_gib, "peak_resident_gib": srv.budget.peak / 2**30,
                "rom_build_s": t_rom, "rom_rank": args.rank, "rom_train": args.serve_train,
                "graph_cg_iters": args.serve_graph_cg_iters,
                "iters_per_round": args.serve_iters_per_round})
    # the same requests, one at a time, through the plain single-instance GPU SI-DSA (FCFS).  A
    # request's cost spans a factor of 64 between keys, so the plain rate of the mix is estimated
    # per key: the first serve_baseline requests of every key in the stream are timed alone
    # (after one warm-up solve of that key), and the mix's mean time per request weights each
    # key's mean by its share of the stream.
    if args.serve_baseline > 0:
        from paper_2402_10488_amd import quadrature
        share = {k: sum(1 for q in timed if (q.n, q.n_phi) == k) / len(timed) for k in SERVE_KEYS}
        per_key = {}
        for k in SERVE_KEYS:
            reqs = [q for q in timed if (q.n, q.n_phi) == k][:args.serve_baseline + 1]
            vx, vy, w = quadrature.chebyshev_circle(k[1])
            times = []
            for j, q in enumerate(reqs):
                dev = lambda a: torch.as_tensor(np.ascontiguousarray(a[None]), device="cuda")
                Pi = rte.Problem(2, q.n, q.n, vx, w, dev(q.sigma_t), dev(q.sigma_s), dev(q.G),
                                 dev(q.g), dirs_y=vy)
                wsi = Pi.workspace("si_dsa", None, args.precision, 500)
                ri = torch.zeros((1, Pi.ndof), dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                tb = time.perf_counter()
                rte.sisa_solve(Pi, ri, mode="si_dsa", eps=args.eps, max_iter=500,
                               cg_rtol=args.cg_rtol, precision=args.precision, ws=wsi)
                torch.cuda.synchronize()
                if j > 0:                                 # the first solve of a key warms up
                    times.append(time.perf_counter() - tb)
            per_key[f"{k[0]}x{k[0]}/{k[1]}"] = {"mean_ms": 1e3 * float(np.mean(times)),
                                                 "share": share[k], "timed": len(times)}
        mean_t = sum(share[k] * per_key[f"{k[0]}x{k[0]}/{k[1]}"]["mean_ms"] * 1e-3
                     for k in SERVE_KEYS)
        base = 1.0 / mean_t
        out.update({"plain_gpu_si_dsa_solves_per_s": base,
                    "plain_gpu_si_dsa_per_key": per_key,
                    "plain_gpu_si_dsa_requests_timed": sum(v["timed"] for v in per_key.values()),
                    "served_vs_plain_gpu_si_dsa": sat["solves_per_s"] / base,
                    "served_vs_plain_note": "saturated served solves/s over the plain rate of the "
                                            "same mix (per-key means weighted by the keys' shares)"})
    return out


def solve_timed(rte, P, rho, reps=1, **kw):
    """Warm-up solve, then ``reps`` timed solves from rho = 0: (result, seconds per solve)."""
    import torch
    rho.zero_()
    rte.sisa_solve(P, rho, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rho.zero_()
        r = rte.sisa_solve(P, rho, **kw)
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) / reps


def split_leg(args, plane, rte, problems, rom_arrays, tuning, ref_n_sweep, headline_ms):
    """The headline batch solved as ``args.split`` sub-batches at once, each with its own problem
    handle, workspace and stream in its own host thread (rte_sisa_solve_multi), with the
    headline's sweep schedule, so every instance's result equals its result in the headline
    solve (checked on the sweep counts).  While one sub-batch's host polls or its kernels leave
    gaps, another's run."""
    import torch
    K = args.split
    B = plane.B
    bounds = [B * k // K for k in range(K + 1)]
    subs = []
    for k in range(K):
        sub = plane.subset(range(bounds[k], bounds[k + 1]))
        Pk = problems.plane_problem(sub, dg=tuning["dg"], wpb=tuning["wpb"],
                                   bands=tuning["bands"])
        Rk = (rte.Rom(Pk, rom_arrays.U_rho, rom_arrays.U_iso, rom_arrays.A0, rom_arrays.A,
                      rom_arrays.eps_pod, rom_arrays.eps_train) if rom_arrays is not None else None)
        psik = problems.plane_psi(sub) if rom_arrays is not None else None
        rhok = torch.zeros((Pk.B, Pk.ndof), dtype=torch.float64, device="cuda")
        subs.append((Pk, Rk, psik, rhok, Pk.workspace(args.mode, Rk, args.precision, 500)))
    streams = [torch.cuda.Stream() for _ in range(K)]
    kw = dict(mode=args.mode, eps=args.eps, max_iter=500, theta=args.theta, cg_rtol=args.cg_rtol,
              precision=args.precision, poll_every=args.poll_every)

    def step():
        for s_ in subs:
            s_[3].zero_()
        torch.cuda.synchronize()
        return rte.sisa_solve_multi([s_[0] for s_ in subs], [s_[3] for s_ in subs], streams,
                                    roms=[s_[1] for s_ in subs], psis=[s_[2] for s_ in subs],
                                    wss=[s_[4] for s_ in subs], **kw)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.split_steps):
        res = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.split_steps
    n_sweep = np.concatenate([r.n_sweep for r in res])
    cd = float(n_sweep.sum()) * plane.nx * plane.ny * subs[0][0].n_dir
    del subs
    torch.cuda.empty_cache()
    return {"parts": K, "steps": args.split_steps, "value": cd / dt, "unit": "cell-dir updates/s",
            "ms_per_step": dt * 1e3, "solves_per_s": B / dt, "vs_headline": headline_ms / (dt * 1e3),
            "sweep_counts_equal_headline": bool(np.array_equal(n_sweep, ref_n_sweep)),
            "note": "the same batch, schedule and results as the headline, as concurrent "
                    "sub-batches on their own streams; reported beside the headline, which stays "
                    "the single-stream solve the roofline object measures"}


def si_dsa_batch_leg(args, P, rte, romsad_solves_per_s, romsad_sweeps):
    """The headline batch solved by batched SI-DSA (same precision, schedule and CG tolerance):
    the ROMSAD batch's gain over it is the correction ROM's alone, apart from batching."""
    import torch
    ws = P.workspace("si_dsa", None, args.precision, 500)
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    r, dt = solve_timed(rte, P, rho, reps=args.batch_dsa_steps, mode="si_dsa", eps=args.eps,
                        max_iter=500, cg_rtol=args.cg_rtol, precision=args.precision, ws=ws)
    del ws
    return {"solves_per_s": P.B / dt, "ms_per_batch": dt * 1e3,
            "cell_dir_updates_per_s": float(r.n_sweep.sum()) * P.ncell * P.n_dir / dt,
            "mean_sweeps": float(r.n_sweep.mean()), "steps": args.batch_dsa_steps,
            "romsad_batch_vs_si_dsa_batch": romsad_solves_per_s / (P.B / dt),
            "romsad_sweeps_saved": 1.0 - romsad_sweeps / float(r.n_sweep.mean())}


def f_gbs(P, rte, reps=3):
    """Average ms and algorithmic GB/s of the FP32 f-form sweep of P's batch."""
    import torch
    f = torch.empty(rte.f_shape(P), dtype=torch.float32, device="cuda")
    rho = torch.rand((P.B, P.ndof), dtype=torch.float64, device="cuda")
    ws = P.workspace("si", None, "mixed")
    rte.sweep(P, rho, f_out=f, precision="mixed", ws=ws)
    torch.cuda.synchronize()
    rte.profile_enable(True)
    for _ in range(reps):
        rte.sweep(P, rho, f_out=f, precision="mixed", ws=ws)
    torch.cuda.synchronize()
    ms, n = rte.profile_read("sweep2d")
    rte.profile_enable(False)
    ms /= max(n, 1)
    nbytes = P.B * P.ncell * P.n_dir * 16 + P.B * P.ncell * 40
    del f, ws
    return ms, nbytes / (ms * 1e-3) / 1e9


def c1_leg(args, rte, problems):
    """The 128^2 checkerboard with 64 directions, one instance: plain SI and SI-DSA in FP64
    (tol 1e-8) and mixed precision (tol 1e-6), each against a tight FP64 solution."""
    import torch
    import rte_workloads as W
    plane = W.c1_checkerboard()
    P = problems.plane_problem(plane)
    rho = torch.zeros((1, P.ndof), dtype=torch.float64, device="cuda")
    rte.sisa_solve(P, rho, mode="si_dsa", eps=1e-12, max_iter=500, cg_rtol=1e-13,
                   precision="fp64")
    ref = rho.clone()
    scale = float(ref.abs().max())
    out = {}
    for prec, eps in (("fp64", 1e-8), ("mixed", 1e-6)):
        for mode in ("si", "si_dsa"):
            r, dt = solve_timed(rte, P, rho, reps=3, mode=mode, eps=eps, max_iter=10000,
                                cg_rtol=args.cg_rtol, precision=prec)
            ns = int(r.n_sweep[0])
            out[f"{mode}_{prec}"] = {"ms": dt * 1e3, "n_sweep": ns, "tol": eps,
                                     "cell_dir_updates_per_s": ns * P.ncell * P.n_dir / dt,
                                     "error_vs_tight_fp64": float((rho - ref).abs().max()) / scale}
    ms, gbs = f_gbs(P, rte)
    out["f_form_sweep"] = {"ms": ms, "GB_s": gbs, "frac": gbs / PEAK_HBM_GBS,
                           "note": "one instance: 16.8 MB of angular flux per sweep, too little "
                                   "to fill the device"}
    out["workload"] = "128x128 Q1 checkerboard, 64 directions, one instance"
    return out


def c4_leg(args, rte, problems, log_fn):
    """The 512^2 multiscale checkerboard with 256 directions: ROMSAD with a rank-40 correction ROM
    from 64 FP64 training solves (window 3, FP32 snapshot columns), then SI-DSA alone; mixed
    precision, tol 1e-6; and the FP32 f-form sweep at this size."""
    import torch
    import rte_workloads as W
    from paper_2402_10488_amd import offline
    plane = W.c4_multiscale()
    P = problems.plane_problem(plane)
    t0 = time.perf_counter()
    ra = offline.build_correction_rom(W.c4_training(args.c4_train), r=40, window=3, eps_train=1e-8,
                                      cg_rtol=1e-10, snapshot_dtype="fp32", chunk=8,
                                      train_max_iter=2000, log=lambda m: log_fn(f"[bench] c4 ROM: {m}"))
    t_rom = time.perf_counter() - t0
    torch.cuda.empty_cache()
    log_fn(f"[bench] c4 ROM: {args.c4_train} training solves, eps_pod {ra.eps_pod:.3e}, {t_rom:.0f}s")
    Rm = rte.Rom(P, ra.U_rho, ra.U_iso, ra.A0, ra.A, ra.eps_pod, ra.eps_train, ra.b_inflow)
    psi = problems.plane_psi(plane)
    rho = torch.zeros((1, P.ndof), dtype=torch.float64, device="cuda")
    out = {"workload": "512x512 Q1 multiscale checkerboard, 256 directions, one instance",
           "rom_rank": 40, "rom_train": args.c4_train, "rom_build_s": t_rom,
           "eps_pod": float(ra.eps_pod)}
    for mode in ("romsad", "si_dsa"):
        log_fn(f"[bench] c4 {mode} solve")
        r, dt = solve_timed(rte, P, rho, reps=1, mode=mode, rom=Rm if mode == "romsad" else None,
                            psi=psi if mode == "romsad" else None, eps=args.eps, theta=args.theta,
                            max_iter=2000, cg_rtol=args.cg_rtol, precision=args.precision)
        ns = int(r.n_sweep[0])
        kinds = r.kind[0, :max(ns - 1, 0)]
        out[mode] = {"ms": dt * 1e3, "n_sweep": ns, "status": int(r.status),
                     "romsa_corrections": int((kinds == 2).sum()),
                     "dsa_corrections": int((kinds == 1).sum()),
                     "cell_dir_updates_per_s": ns * P.ncell * P.n_dir / dt}
    out["romsad_vs_si_dsa"] = out["si_dsa"]["ms"] / out["romsad"]["ms"]
    ms, gbs = f_gbs(P, rte)
    out["f_form_sweep"] = {"ms": ms, "GB_s": gbs, "frac": gbs / PEAK_HBM_GBS}
    del Rm, rho
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="romsad", choices=["si", "si_dsa", "romsad"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nphi", type=int, default=64)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--rank", type=int, default=20)
    ap.add_argument("--window", type=int, default=3)
    ap.add_argument("--theta", type=int, default=5)
    ap.add_argument("--n-train", type=int, default=32)
    ap.add_argument("--eps-train", type=float, default=1e-10)
    ap.add_argument("--cg-rtol", type=float, default=1e-3)
    ap.add_argument("--graph-cg-iters", type=int, default=0,
                    help="> 0: every outer iteration of the timed solves is one HIP graph launch "
                         "with this many diffusion CG iterations per correction")
    ap.add_argument("--poll-every", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's static schedule rule instead of the measured pick")
    ap.add_argument("--baseline-instances", type=int, default=4)
    ap.add_argument("--batch-dsa-steps", type=int, default=2,
                    help="timed solves of the batch by batched SI-DSA (0: skip the leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="oracle processes of the CPU baseline (0: the host's cores, at most 16)")
    ap.add_argument("--no-f-form", action="store_true")
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--c4-train", type=int, default=64)
    ap.add_argument("--pgmres-instances", type=int, default=64,
                    help="instances of the batch solved by DSA-preconditioned GMRES (0: skip)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="copy a buffer of this size before timing (HBM counter calibration)")
    ap.add_argument("--trace-gap", type=float, default=0.0,
                    help="seconds of GPU idle before and after the timed steps, so that a kernel "
                         "trace of the run can cut out the timed region (outside the clock)")
    ap.add_argument("--split", type=int, default=2,
                    help="sub-batches of the headline batch solved at once for the split leg "
                         "(0 or 1: no split leg)")
    ap.add_argument("--split-steps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-warmup", type=int, default=40)
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="open-loop arrival rate (requests/s); 0: 0.8 x the measured capacity")
    ap.add_argument("--serve-train", type=int, default=32)
    ap.add_argument("--serve-batch-mcd", type=int, default=1024,
                    help="a key's slots: about this many million cell-direction updates per sweep")
    ap.add_argument("--serve-min-slots", type=int, default=32)
    ap.add_argument("--serve-max-slots", type=int, default=256)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-baseline", type=int, default=3,
                    help="requests of every key timed alone through plain single-instance SI-DSA")
    ap.add_argument("--serve-graph-cg-iters", type=int, default=0,
                    help="> 0: the slot pools run each outer iteration as one HIP graph launch")
    ap.add_argument("--serve-iters-per-round", type=int, default=2,
                    help="outer iterations of a slot pool between retire/admit rounds")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described, not built)"}))
        sys.exit(2)

    import torch
    import rte_workloads as W
    from paper_2402_10488_amd import autotune, rte, problems

    if args.copy_calibration_gib > 0:
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counter readings give the
        # scale of those counters (bytes moved = known size)
        n = int(args.copy_calibration_gib * 2**30) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
        torch.cuda.empty_cache()

    t_bench = time.perf_counter()
    plane = W.c2_batch(args.batch, args.n, args.nphi)
    tune = None
    if args.no_autotune:
        P = problems.plane_problem(plane)
    else:
        P0 = problems.plane_problem(plane)
        r0 = torch.rand((P0.B, P0.ndof), dtype=torch.float64, device="cuda")
        tune = autotune.tune(P0, r0, args.precision)
        log(f"[bench] sweep schedule: dg={tune['dg']} wpb={tune['wpb']} bands={tune['bands']} "
            f"({'cached' if tune['cached'] else 'measured'}: {tune['candidates']})")
        del r0, P0
        P = problems.plane_problem(plane, dg=tune["dg"], wpb=tune["wpb"], bands=tune["bands"])
    psi = problems.plane_psi(plane)
    Rm, rom_arrays = None, None
    if args.mode == "romsad":
        train = W.c2_training(args.n_train, args.n, args.nphi)
        Rm, rom_arrays = build_rom(train, P, rte, problems, args)
    max_iter = 500
    ws = P.workspace(args.mode, Rm, args.precision, max_iter)
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    log(f"[bench] workload {plane.name}: B={P.B} ndof={P.ndof} n_dir={P.n_dir} tuning={P.tuning()} "
        f"workspace={ws.numel() / 2**30:.2f} GiB graph_cg_iters={args.graph_cg_iters}")

    def step():
        rho.zero_()
        return rte.sisa_solve(P, rho, mode=args.mode, rom=Rm, psi=psi, eps=args.eps,
                              max_iter=max_iter, theta=args.theta, cg_rtol=args.cg_rtol,
                              precision=args.precision, ws=ws, poll_every=args.poll_every,
                              graph_cg_iters=args.graph_cg_iters)

    for w in range(args.warmup):
        r = step()
        log(f"[bench] warmup {w}: n_sweep mean {r.n_sweep.mean():.2f} max {r.n_sweep.max()}")
    torch.cuda.synchronize()
    if args.trace_gap > 0:
        time.sleep(args.trace_gap)
    # HIP events around every sweep launch time the dominant kernel inside the timed region (in
    # graph mode the events cannot sit inside the graph: one extra untimed eager step gives them)
    rte.profile_enable(args.graph_cg_iters <= 0)
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    if args.trace_gap > 0:
        time.sleep(args.trace_gap)
    if args.graph_cg_iters > 0:
        rte.profile_enable(True)
        rho.zero_()
        rte.sisa_solve(P, rho, mode=args.mode, rom=Rm, psi=psi, eps=args.eps, max_iter=max_iter,
                       theta=args.theta, cg_rtol=args.cg_rtol, precision=args.precision, ws=ws,
                       poll_every=args.poll_every)
        torch.cuda.synchronize()
    sweep_ms, sweep_n = rte.profile_read("sweep2d")
    dsa_ms, dsa_n = rte.profile_read("dsa")
    rom_ms, rom_n = rte.profile_read("rom")
    red_ms, red_n = rte.profile_read("reduce")
    rte.profile_enable(False)
    bad = [int(r.status) for r in results if r.status != rte.RTE_OK]
    R_batch = residual_inf(P, rte, rho)
    dsa_corrections = sum(int((r.kind == 1).sum()) for r in results)
    cg_per_correction = (sum(r.cg_iterations for r in results) / dsa_corrections
                         if dsa_corrections else None)
    sweeps = np.array([r.n_sweep for r in results])
    cd_total = float(sweeps.sum()) * P.ncell * P.n_dir
    solves = P.B * args.steps
    value = cd_total / elapsed
    # the sweep's own work per launch: the cell-direction updates of the timed steps over the
    # launches that made them (eager), or of the extra step (graph mode)
    cd_timed_sweeps = cd_total if args.graph_cg_iters <= 0 else float(sweeps[-1].sum()) * P.ncell * P.n_dir
    launch_ms = sweep_ms / max(sweep_n, 1)
    launch_cd = cd_timed_sweeps / max(sweep_n, 1)
    achieved = launch_cd * SWEEP_FLOPS_PER_CD / (launch_ms * 1e-3) / 1e12
    achieved_kf = launch_cd * SWEEP_FLOPS_PER_CD_KERNEL / (launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = measured_traffic(launch_cd)
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f}s; sweeps/instance mean {sweeps.mean():.2f}; "
        f"sweep kernel {sweep_ms:.1f} ms over {sweep_n} launches; dsa {dsa_ms:.1f} ms ({dsa_n}); "
        f"rom {rom_ms:.1f} ms ({rom_n}); reduce {red_ms:.1f} ms ({red_n})")

    split = None
    if args.split > 1 and args.graph_cg_iters <= 0:
        log(f"[bench] the batch as {args.split} concurrent sub-batches")
        split = split_leg(args, plane, rte, problems, rom_arrays, P.tuning(), results[-1].n_sweep,
                          elapsed / args.steps * 1e3)
        log(f"[bench] split: {json.dumps(split)}")

    # plain single-instance GPU SI-DSA (same library, batch of one, same precision)
    base = {}
    if args.baseline_instances > 0:
        t_base, n_base = 0.0, 0
        for b in range(args.baseline_instances):
            Pi = problems.plane_problem(plane.instance(b))
            wsi = Pi.workspace("si_dsa", None, args.precision, max_iter)
            ri = torch.zeros((1, Pi.ndof), dtype=torch.float64, device="cuda")
            rb, dt = solve_timed(rte, Pi, ri, reps=1, mode="si_dsa", eps=args.eps,
                                 max_iter=max_iter, cg_rtol=args.cg_rtol,
                                 precision=args.precision, ws=wsi)
            t_base += dt
            n_base += 1
        base_solves = n_base / t_base
        base = {"plain_gpu_si_dsa_solves_per_s": base_solves,
                "batch_vs_plain_gpu_si_dsa": (solves / elapsed) / base_solves,
                "plain_instances_timed": n_base}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-dir updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sweep/projections + f64 corrections" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"parametric 4x4 block lattice, {args.batch} instances, "
                               f"{args.n}x{args.n} Q1, {args.nphi} directions, {args.mode}, "
                               f"tol {args.eps:g}",
                   "batch": args.batch, "mesh": args.n, "n_dir": args.nphi, "mode": args.mode,
                   "precision": args.precision, "rank": args.rank if Rm else None,
                   "theta": args.theta, "cg_rtol": args.cg_rtol, "tuning": P.tuning(),
                   "graph_cg_iters": args.graph_cg_iters, "poll_every": args.poll_every},
        "solves_per_s": solves / elapsed,
        "mean_sweeps_per_solve": float(sweeps.mean()),
        "residual_inf_median": float(np.median(R_batch)),
        "residual_inf_max": float(R_batch.max()),
        "dsa_corrections_per_solve": dsa_corrections / solves,
        "cg_iterations_per_dsa_correction": cg_per_correction,
        "status_not_ok_steps": bad,
        "batch_latency_ms": {"p50": elapsed / args.steps * 1e3, "p99": elapsed / args.steps * 1e3,
                             "note": "all instances of a step arrive together and return together"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "sweep2d_kernel", "avg_launch_ms": launch_ms,
                     "flops_per_cd": SWEEP_FLOPS_PER_CD,
                     "achieved_kernel_flops": achieved_kf,
                     "flops_per_cd_kernel": SWEEP_FLOPS_PER_CD_KERNEL,
                     "cd_per_launch": launch_cd},
        "time_split_ms": {"sweep": sweep_ms, "reduce": red_ms, "dsa": dsa_ms, "rom": rom_ms,
                          "total": elapsed * 1e3,
                          "note": "event-timed groups of the timed steps" if args.graph_cg_iters <= 0
                                  else "event-timed groups of one extra kernel-by-kernel step"},
    }
    if tune is not None:
        out["autotune"] = {"pick": {"dg": tune["dg"], "wpb": tune["wpb"], "bands": tune["bands"]},
                           "ms": tune["ms"],
                           "cached": tune["cached"], "candidates_ms": tune["candidates"]}
    out.update(base)
    if split is not None:
        out["split"] = split
    if args.batch_dsa_steps > 0 and args.mode == "romsad":
        out["si_dsa_batch"] = si_dsa_batch_leg(args, P, rte, solves / elapsed, float(sweeps.mean()))
        log(f"[bench] batched si_dsa: {json.dumps(out['si_dsa_batch'])}")
    if args.pgmres_instances > 0:
        out["pgmres"] = pgmres_leg(args, plane, rte, problems, solves / elapsed)
        log(f"[bench] pgmres: {json.dumps(out['pgmres'])}")
    if not args.no_f_form:
        out["roofline_f_form"] = f_form_leg(P, rte)
        log(f"[bench] f-form sweep: {out['roofline_f_form']['achieved']:.0f} GB/s")
    del ws
    torch.cuda.empty_cache()
    if not args.no_c1:
        out["c1"] = c1_leg(args, rte, problems)
        log(f"[bench] c1: {json.dumps(out['c1'])}")
    # the oracle's ROM for the CPU baseline builds on the host while the large GPU legs run
    rom_job = None
    if not args.no_cpu_baseline and args.mode == "romsad":
        rom_job = OracleRomJob(args, max(1, host_cores() - 2))
    try:
        if not args.no_c4:
            out["c4"] = c4_leg(args, rte, problems, log)
            log(f"[bench] c4: {json.dumps(out['c4'])}")
        rom_path = None
        if rom_job is not None:
            rom_path = rom_job.wait()
            log(f"[bench] oracle ROM for the CPU baseline built in {rom_job.seconds:.0f}s")
        if args.serve_requests > 0:
            out["serving"] = serving_leg(args, rte)
            log(f"[bench] serving: {json.dumps(out['serving'])}")
        if not args.no_cpu_baseline:
            log("[bench] CPU oracle baselines")
            out["cpu_baseline"] = cpu_baseline(args, args.mode, rom_path)
            log(f"[bench] cpu baseline: {json.dumps(out['cpu_baseline'])}")
            extra = {}
            if not args.no_c1:
                extra["c1"] = cpu_c1(args)
                log(f"[bench] cpu c1: {json.dumps(extra['c1'])}")
            if not args.no_c4:
                extra["c4"] = cpu_c4(args)
                log(f"[bench] cpu c4: {json.dumps(extra['c4'])}")
            if args.serve_requests > 0:
                extra["c3"] = cpu_c3(args)
                log(f"[bench] cpu c3: {json.dumps(extra['c3'])}")
            out["cpu_baseline_other"] = extra
    finally:
        if rom_job is not None:
            rom_job.close()
    out["bench_wall_s"] = time.perf_counter() - t_bench
    print(json.dumps(out))


if __name__ == "__main__":
    main()
