"""Measured choice of the 2D sweep schedule, cached per (device, mesh, directions, batch, precision).

The sweep kernel gives every wavefront one (instance, quadrant, group of dg directions), puts wpb
wavefronts of a band in a workgroup and runs `bands` mesh bands of it at once.  Which schedule is
fastest depends on the batch size, the direction count and the precision (registers per lane grow
with dg; the number of wavefronts in flight falls with it; more bands in flight shorten the
pipeline of a single large instance).  The tuner times every schedule the library runs on the workload itself
(rte_tune_sweep: HIP events around the sweeps, on the device) and keeps the fastest.  The choice
is stored in a JSON file, so a workload is timed once per device; later problems of the same shape
read it back.
"""
import json
import os
import tempfile

CANDIDATES = tuple((dg, w, nb) for dg in (1, 2, 4, 8) for w in (1, 2, 4) for nb in (1, 2, 4))
CACHE_ENV = "RTE_TUNE_CACHE"
VERSION = 2


def default_cache_path():
    """$RTE_TUNE_CACHE, else ~/.cache/paper_2402_10488_amd/sweep_tuning.json."""
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2402_10488_amd",
                        "sweep_tuning.json")


def workload_key(device, nx, ny, n_dir, batch, precision, f_form=False):
    return f"{device}|{nx}x{ny}|dirs{n_dir}|B{batch}|{precision}|{'f' if f_form else 'rho'}"


def load(path):
    """The cached table ({} when the file is missing, unreadable or of another version)."""
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    if not isinstance(data, dict) or data.get("version") != VERSION:
        return {}
    table = data.get("entries")
    return table if isinstance(table, dict) else {}


def store(path, table):
    """Writes the table atomically (a concurrent reader sees the old or the new file)."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".sweep_tuning.")
    try:
        with os.fdopen(fd, "w") as f:
            json.dump({"version": VERSION, "entries": table}, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise


def select(times):
    """The fastest schedule among {(dg, wpb, bands): ms} with ms > 0 (ties: the smaller tuple);
    None if no candidate ran."""
    valid = {k: v for k, v in times.items() if v is not None and v > 0}
    if not valid:
        return None
    return min(valid, key=lambda k: (valid[k], k))


def device_name():
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "")
    return f"{props.name}:{arch}:{props.multi_processor_count}cu"


def tune(problem, rho_in, precision="mixed", f_out=None, path=None, refresh=False, timer=None,
         device=None, candidates=CANDIDATES):
    """The schedule for ``problem``'s workload: read from the cache, or timed and stored.

    timer(candidates) -> milliseconds per sweep for each candidate (default: rte_tune_sweep on
    rho_in).  Returns {"dg", "wpb", "bands", "ms", "candidates": {"dg,wpb,bands": ms}, "cached",
    "key"}."""
    path = path or default_cache_path()
    device = device or device_name()
    key = workload_key(device, problem.nx, problem.ny, problem.n_dir, problem.B, precision,
                       f_out is not None)
    table = load(path)
    if not refresh and key in table:
        return dict(table[key], cached=True, key=key)
    if timer is None:
        from . import rte
        timer = lambda c: rte.tune_sweep(problem, c, rho_in, precision, f_out)
    ms = [float(t) for t in timer(list(candidates))]
    times = dict(zip(candidates, ms))
    pick = select(times)
    if pick is None:
        raise RuntimeError(f"no sweep schedule ran for {key}")
    entry = {"dg": int(pick[0]), "wpb": int(pick[1]), "bands": int(pick[2]), "ms": times[pick],
             "candidates": {",".join(map(str, c)): t for c, t in times.items()}}
    table = load(path)               # another process may have added entries meanwhile
    table[key] = entry
    try:
        store(path, table)
    except OSError:
        pass                         # an unwritable cache only costs a new measurement next time
    return dict(entry, cached=False, key=key)
