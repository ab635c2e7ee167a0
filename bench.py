"""Benchmark: batched parametric source iteration with synthetic acceleration on one MI355X.

One step = one batched solve (Alg. 1 with the ROMSAD switch of Alg. 2 by default) of the
parametric lattice batch: 256 instances, 128 x 128 Q1 mesh, 64 directions on the unit circle,
per-block sigma_s ~ U[0.5, 50], sigma_a ~ U[0.001, 1], FP32 sweep / FP64 corrections,
relative tolerance 1e-6.  Inputs are seeded synthetic materials resident in HBM before timing.

Prints one JSON line (see the "metric" field).  The dominant kernel's roofline comes from HIP
events recorded by the library around every sweep launch inside the timed region.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic work of one cell-direction update of the 2D sweep (see the sweep kernel header):
# 16 flops right-hand side, 56 flops closed-form Q1 cell solve, 8 flops outflow traces,
# 8 flops FP64 density accumulation
SWEEP_FLOPS_PER_CD = 88
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}     # MI355X published vector peaks (FP32, FP64)


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


def cpu_baseline(args, mode, rom_arrays):
    """The oracle as it stands, timed on the host on a bounded sample (one instance)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import rte_workloads as W
    from oracle.problem import discretize
    from oracle.sisa import sisa
    from oracle import rom as orom
    plane = W.c2_lattice([20000], n=args.n, n_phi=args.nphi)
    d = discretize(plane, 0)
    rom = None
    if mode == "romsad":
        # the oracle builds its own correction ROM from a small training sample (untimed)
        train = W.c2_lattice([30000 + i for i in range(args.cpu_train)], n=args.n, n_phi=args.nphi)
        discs = [discretize(train, b) for b in range(train.B)]
        rom = orom.build_correction_rom(discs, orom.plane_affine(discs[0]), orom.plane_psi,
                                        window=args.window, r=args.rank, eps_train=args.eps_train)
    t0 = time.perf_counter()
    res = sisa(d, "romsad" if mode == "romsad" else mode, eps=args.eps, rom=rom, theta=args.theta)
    dt = time.perf_counter() - t0
    cd = d.nc * d.nv * res.n_sweep
    return {"value": cd / dt, "unit": "cell-dir updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 instance (seed 20000) of the {args.n}x{args.n} lattice, {args.nphi} "
                      f"directions, {mode}, FP64, tol {args.eps:g}: {res.n_sweep} sweeps in "
                      f"{dt:.1f}s; oracle ROM from {args.cpu_train} training solves"
                      if mode == "romsad" else
                      f"1 instance (seed 20000) of the {args.n}x{args.n} lattice, {args.nphi} "
                      f"directions, {mode}, FP64, tol {args.eps:g}: {res.n_sweep} sweeps in {dt:.1f}s",
            "solves_per_s": 1.0 / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
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
    ap.add_argument("--cg-rtol", type=float, default=1e-10)
    ap.add_argument("--baseline-instances", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-train", type=int, default=4)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described, not built)"}))
        sys.exit(2)

    import torch
    import rte_workloads as W
    from paper_2402_10488_amd import rte, problems

    plane = W.c2_batch(args.batch, args.n, args.nphi)
    P = problems.plane_problem(plane)
    psi = problems.plane_psi(plane)
    Rm, rom_arrays = None, None
    if args.mode == "romsad":
        train = W.c2_training(args.n_train, args.n, args.nphi)
        Rm, rom_arrays = build_rom(train, P, rte, problems, args)
    max_iter = 500
    ws = P.workspace(args.mode, Rm, args.precision, max_iter)
    rho = torch.zeros((P.B, P.ndof), dtype=torch.float64, device="cuda")
    log(f"[bench] workload {plane.name}: B={P.B} ndof={P.ndof} n_dir={P.n_dir} tuning={P.tuning()} "
        f"workspace={ws.numel() / 2**30:.2f} GiB")

    def step():
        rho.zero_()
        return rte.sisa_solve(P, rho, mode=args.mode, rom=Rm, psi=psi, eps=args.eps,
                              max_iter=max_iter, theta=args.theta, cg_rtol=args.cg_rtol,
                              precision=args.precision, ws=ws)

    for w in range(args.warmup):
        r = step()
        log(f"[bench] warmup {w}: n_sweep mean {r.n_sweep.mean():.2f} max {r.n_sweep.max()}")
    torch.cuda.synchronize()
    rte.profile_enable(True)
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    sweep_ms, sweep_n = rte.profile_read("sweep2d")
    dsa_ms, dsa_n = rte.profile_read("dsa")
    rom_ms, rom_n = rte.profile_read("rom")
    red_ms, red_n = rte.profile_read("reduce")
    rte.profile_enable(False)
    bad = [int(r.status) for r in results if r.status != rte.RTE_OK]
    sweeps = np.array([r.n_sweep for r in results])
    cd_total = float(sweeps.sum()) * P.ncell * P.n_dir
    solves = P.B * args.steps
    value = cd_total / elapsed
    achieved = cd_total * SWEEP_FLOPS_PER_CD / (sweep_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f}s; sweeps/instance mean {sweeps.mean():.2f}; "
        f"sweep kernel {sweep_ms:.1f} ms over {sweep_n} launches; dsa {dsa_ms:.1f} ms ({dsa_n}); "
        f"rom {rom_ms:.1f} ms ({rom_n}); reduce {red_ms:.1f} ms ({red_n})")

    # plain single-instance GPU SI-DSA (same library, batch of one, FP64? no: same precision)
    base = {}
    if args.baseline_instances > 0:
        t_base, n_base = 0.0, 0
        for b in range(args.baseline_instances):
            Pi = problems.plane_problem(plane.instance(b))
            wsi = Pi.workspace("si_dsa", None, args.precision, max_iter)
            ri = torch.zeros((1, Pi.ndof), dtype=torch.float64, device="cuda")
            rte.sisa_solve(Pi, ri, mode="si_dsa", eps=args.eps, max_iter=max_iter,
                           cg_rtol=args.cg_rtol, precision=args.precision, ws=wsi)   # warm
            ri.zero_()
            torch.cuda.synchronize()
            tb = time.perf_counter()
            rb = rte.sisa_solve(Pi, ri, mode="si_dsa", eps=args.eps, max_iter=max_iter,
                                cg_rtol=args.cg_rtol, precision=args.precision, ws=wsi)
            torch.cuda.synchronize()
            t_base += time.perf_counter() - tb
            n_base += 1
        base_solves = n_base / t_base
        base = {"plain_gpu_si_dsa_solves_per_s": base_solves,
                "served_vs_plain_gpu_si_dsa": (solves / elapsed) / base_solves,
                "plain_instances_timed": n_base}

    out = {
        "metric": "cell-direction updates/s (batched parametric ROMSAD solves)",
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
                   "theta": args.theta, "tuning": P.tuning()},
        "solves_per_s": solves / elapsed,
        "mean_sweeps_per_solve": float(sweeps.mean()),
        "status_not_ok_steps": bad,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "sweep2d_kernel", "avg_launch_ms": sweep_ms / max(sweep_n, 1),
                     "flops_per_cd": SWEEP_FLOPS_PER_CD},
        "time_split_ms": {"sweep": sweep_ms, "reduce": red_ms, "dsa": dsa_ms, "rom": rom_ms,
                          "total": elapsed * 1e3},
    }
    out.update(base)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, args.mode, rom_arrays)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
