"""Oracle: the CPU oracle over many instances in a pool of worker processes.

Test infrastructure only -- never imported by the product path.

The workers are started with the 'spawn' method, so they share nothing with a parent that has
initialised the GPU; they import the oracle and the seeded generators only.  Each worker rebuilds
its instance from the generator's arguments, so only small arguments and results cross the
process boundary; snapshot columns go through a memory-mapped file.  The arithmetic is the
oracle's own (correction_snapshots, correction_rom_from_snapshots, sisa); the pool only runs
independent instances side by side.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def pool_size(limit=16):
    """Worker count: the host's cores, at most ``limit`` (the CPU share of a one-GPU host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def make_pool(n=None, initializer=None, initargs=()):
    """A spawn pool whose workers run single-threaded BLAS (the pool supplies the parallelism)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        return ctx.Pool(n or pool_size(), initializer=_init, initargs=(initializer, initargs))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


_STATE = {}


def _init(fn, args):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    if fn is not None:
        fn(*args)


def _plane(spec):
    import rte_workloads as W
    name, args = spec
    return getattr(W, name)(*args)


# ---- correction-ROM snapshots (Sec. 3.2.1) ------------------------------------------------
def _snapshot_job(job):
    from oracle.problem import discretize
    from oracle.rom import correction_snapshots
    spec, b, window, eps_train, path, shape, col0 = job
    d = discretize(_plane(spec), b)
    cols = correction_snapshots([d], window, eps_train)
    mm = np.memmap(path, dtype=np.float64, mode="r+", shape=shape)
    mm[:, col0:col0 + cols.shape[1]] = cols
    mm.flush()
    del mm
    return b, cols.shape[1]


def correction_snapshots_parallel(spec, n_train, window, eps_train, n_rows, workdir, pool,
                                  log=None):
    """delta F of the correction ROM over the training instances 0..n_train-1 of the plane
    description ``spec`` = (generator name in rte_workloads, args), ``window`` columns each (every
    training solve here takes more sweeps than the window); returns the [n_rows, n_cols] array.
    log (optional) is called with a line as training solves finish."""
    path = os.path.join(workdir, "snapshots.f64")
    shape = (n_rows, n_train * window)
    np.memmap(path, dtype=np.float64, mode="w+", shape=shape).flush()
    jobs = [(spec, b, window, eps_train, path, shape, b * window) for b in range(n_train)]
    got = []
    for item in pool.imap_unordered(_snapshot_job, jobs):
        got.append(item)
        if log and (len(got) % 8 == 0 or len(got) == n_train):
            log(f"training solves finished: {len(got)} of {n_train}")
    assert all(n == window for _, n in got), got
    return np.array(np.memmap(path, dtype=np.float64, mode="r", shape=shape))


# ---- Alg. 1 / Alg. 2 on test instances ----------------------------------------------------
def _set_rom(rom):
    _STATE["rom"] = rom


def _solve_job(job):
    from oracle.problem import discretize
    from oracle.sisa import sisa
    spec, b, mode, eps, theta = job
    d = discretize(_plane(spec), b)
    res = sisa(d, mode, eps=eps, rom=_STATE.get("rom"), theta=theta)
    return b, res.n_sweep, list(res.kinds), list(res.changes), res.rho, res.converged


def solve_instances(spec, ids, mode, eps, theta=5, rom=None, n=None):
    """Oracle sisa() of every listed instance, in a pool; returns {b: (n_sweep, kinds, changes,
    rho, converged)} and the pool's worker count."""
    workers = n or pool_size()
    with make_pool(workers, _set_rom, (rom,)) as pool:
        out = pool.map(_solve_job, [(spec, b, mode, eps, theta) for b in ids], chunksize=1)
    return {b: (ns, kinds, ch, rho, conv) for b, ns, kinds, ch, rho, conv in out}, workers


def build_correction_rom_parallel(spec, n_train, window, eps_train, r=None, workdir=None, n=None,
                                  eps_pod=None, log=None):
    """The oracle's correction ROM (Sec. 3.2.1) of training instances 0..n_train-1 of ``spec``:
    snapshot columns from a pool, then the POD (rank r, or eq. (pod_truncation) with eps_pod) and
    reduced operators of correction_rom_from_snapshots on the medium's affine split."""
    import tempfile
    from oracle import rom as orom
    from oracle.problem import discretize
    d0 = discretize(_plane(spec), 0)
    with tempfile.TemporaryDirectory(dir=workdir) as tmp:
        with make_pool(n) as pool:
            dF = correction_snapshots_parallel(spec, n_train, window, eps_train,
                                               d0.nv * d0.ndof, tmp, pool, log)
    return orom.correction_rom_from_snapshots(dF, d0, orom.plane_affine(d0), orom.plane_psi,
                                              r=r, eps_pod=eps_pod, eps_train=eps_train, log=log)


def build_roms_parallel(spec, n_train, window, eps_train, eps_pod=None, r_c=None, r_p=None,
                        workdir=None, n=None, log=None):
    """The oracle's correction ROM (Sec. 3.2.1) and parametric ROM (Sec. 3.1) of training
    instances 0..n_train-1 of ``spec`` from one pool run of the training solves.  The first column
    of every instance's window is f - f^(0) = f, the converged angular flux, so those columns are
    the parametric snapshots; each ROM is then the POD of its columns (rank r_c / r_p, or eq.
    (pod_truncation) with eps_pod) and its reduced operators, as build_correction_rom and
    build_parametric_rom form them."""
    import tempfile
    from oracle import rom as orom
    from oracle.problem import discretize
    d0 = discretize(_plane(spec), 0)
    with tempfile.TemporaryDirectory(dir=workdir) as tmp:
        with make_pool(n) as pool:
            dF = correction_snapshots_parallel(spec, n_train, window, eps_train,
                                               d0.nv * d0.ndof, tmp, pool, log)
    affine = orom.plane_affine(d0)
    F = np.ascontiguousarray(dF[:, ::window])
    U, sv, _ = np.linalg.svd(F, full_matrices=False)
    del F
    rp = orom.pod_rank(sv, eps_pod) if r_p is None else min(r_p, U.shape[1])
    Ur = np.ascontiguousarray(U[:, :rp])
    del U
    if log:
        log(f"parametric POD: rank {rp} of {n_train} solutions")
    A0, At, As, U_rho, _ = orom.reduced_operators(d0, Ur, affine, log)
    prom = orom.ParametricROM(Ur, U_rho, A0, At, As, sv, orom.plane_psi)
    crom = orom.correction_rom_from_snapshots(dF, d0, affine, orom.plane_psi, r=r_c,
                                              eps_pod=eps_pod, eps_train=eps_train, log=log)
    if log:
        log(f"correction POD: rank {crom.r} of {dF.shape[1]} columns")
    return crom, prom


def save_rom(path, rom):
    """A correction ROM's arrays to an .npz file (no pickled objects)."""
    np.savez(path, dU_rho=rom.dU_rho, dU_iso=rom.dU_iso, A0=rom.A0, At=np.stack(rom.At),
             As=np.stack(rom.As), sv=rom.sv, eps_pod=rom.eps_pod, eps_train=rom.eps_train)


def load_rom(path):
    """The correction ROM saved by save_rom, on the block-lattice affine parameters."""
    from oracle import rom as orom
    z = np.load(path, allow_pickle=False)
    return orom.CorrectionROM(z["dU_rho"], z["dU_iso"], z["A0"], list(z["At"]), list(z["As"]),
                              z["sv"], float(z["eps_pod"]), float(z["eps_train"]), orom.plane_psi)


def _main(argv):
    """python -m oracle.pool build-rom '<json>': builds a correction ROM of a generator's training
    instances in a pool and saves it (cfg: spec, n_train, window, eps_train, rank, procs, out)."""
    import json
    if len(argv) != 3 or argv[1] != "build-rom":
        raise SystemExit("usage: python -m oracle.pool build-rom '<json config>'")
    cfg = json.loads(argv[2])
    spec = (cfg["spec"][0], tuple(cfg["spec"][1]))
    rom = build_correction_rom_parallel(spec, cfg["n_train"], cfg["window"], cfg["eps_train"],
                                        r=cfg["rank"], n=cfg.get("procs"))
    save_rom(cfg["out"], rom)
    print("saved", cfg["out"], flush=True)


if __name__ == "__main__":
    _main(sys.argv)
