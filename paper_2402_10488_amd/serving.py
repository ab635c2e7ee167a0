"""Continuous-batching serving loop for parametric solve requests on one GPU.

Requests carry a mesh (n x n Q1), a direction count and lattice materials with a left inflow.
They are grouped by key (n, n_phi).  Each key owns a slot pool:
  - a Problem of capacity S instances whose device material rows are rewritten on admission;
  - a resumable Session (rte_sisa_begin / rte_sisa_admit / rte_sisa_iterate) on its own stream;
  - optionally a correction ROM (ROMSAD), shared by every slot of the key.
A dispatcher releases requests at their arrival times.  Each key's worker thread
  - admits queued requests into free slots while the device-memory budget allows (the footprint
    of a request is its slot's share of the pool's workspace, materials and state);
  - runs outer iterations of all running slots;
  - retires every slot whose solve stopped (copying its rho out).
So requests join and leave a batch between iterations.  The workers run concurrently on their own
streams (the library calls release the GIL), so the kernels of different keys overlap on the
device.  A request's result does not depend on when it was admitted or what shares its batch:
every slot follows Alg. 1 from its own start.

This module only schedules; every step of a solve runs in the library's kernels.
"""
import queue
import threading
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional

import numpy as np

from . import quadrature
from .rte import Problem, Rom, Session


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the stream
    n: int                    # mesh is n x n
    n_phi: int                # directions on the unit circle
    sigma_t: np.ndarray       # [n, n]
    sigma_s: np.ndarray       # [n, n]
    G: np.ndarray             # [n, n]
    g: np.ndarray             # [4] isotropic inflow per side (left, right, bottom, top)
    psi: Optional[np.ndarray] = None   # affine parameters of the request (ROMSAD)


@dataclass
class Result:
    rid: int
    key: tuple
    arrival: float
    admitted: float
    finished: float
    n_sweep: int
    status: int
    rho: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class MemoryBudget:
    """Device bytes that resident requests may hold together."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.used = 0
        self.peak = 0
        self._lock = threading.Lock()

    def try_reserve(self, nbytes: int) -> bool:
        with self._lock:
            if self.used + nbytes > self.capacity:
                return False
            self.used += nbytes
            self.peak = max(self.peak, self.used)
            return True

    def release(self, nbytes: int):
        with self._lock:
            self.used -= nbytes


class KeyPool:
    """Slot pool of one (mesh, directions) key."""

    def __init__(self, n: int, n_phi: int, capacity: int, mode: str, rom_arrays=None,
                 precision="mixed", eps=1e-6, max_iter=500, theta=5, cg_rtol=1e-10,
                 iters_per_round=1, keep_rho=False, graph_cg_iters=0):
        import torch
        self.key = (n, n_phi)
        self.S = capacity
        self.mode = mode
        self.iters_per_round = iters_per_round
        self.keep_rho = keep_rho
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            ones = torch.ones((capacity, n, n), dtype=torch.float64, device="cuda")
            self.sigma_t = ones.clone()
            self.sigma_s = 0.5 * ones
            self.G = torch.zeros_like(ones)
            self.g = torch.zeros((capacity, 4), dtype=torch.float64, device="cuda")
            vx, vy, w = quadrature.chebyshev_circle(n_phi)
            self.P = Problem(2, n, n, vx, w, self.sigma_t, self.sigma_s, self.G, self.g, dirs_y=vy)
            self.rom, self.psi = None, None
            if mode == "romsad":
                assert rom_arrays is not None, "ROMSAD needs the key's correction ROM"
                self.rom = Rom(self.P, rom_arrays.U_rho, rom_arrays.U_iso, rom_arrays.A0,
                               rom_arrays.A, rom_arrays.eps_pod, rom_arrays.eps_train)
                m = rom_arrays.A.shape[0]
                self.psi = torch.zeros((capacity, m), dtype=torch.float64, device="cuda")
            self.session = Session(self.P, mode, self.rom, self.psi, eps=eps, max_iter=max_iter,
                                   theta=theta, cg_rtol=cg_rtol, precision=precision,
                                   poll_every=iters_per_round, stream=self.stream,
                                   graph_cg_iters=graph_cg_iters)
        self.stream.synchronize()
        total = self.session.ws.numel() + 8 * (4 * capacity * n * n + 4 * capacity)
        total += 8 * self.session.rho.numel()
        self.slot_bytes = int(total // capacity)
        self.free = list(range(capacity))[::-1]
        self.slot_req: Dict[int, tuple] = {}     # slot -> (request, admission time)

    def admit(self, reqs: List[Request], t0: float) -> List[int]:
        """Write the requests' materials into free slots and start them; returns the slots."""
        import torch
        slots = [self.free.pop() for _ in reqs]
        with torch.cuda.stream(self.stream):
            idx = torch.as_tensor(slots, device="cuda")
            st = np.stack([r.sigma_t for r in reqs])
            ss = np.stack([r.sigma_s for r in reqs])
            G = np.stack([r.G for r in reqs])
            g = np.stack([r.g for r in reqs])
            self.sigma_t[idx] = torch.as_tensor(st, device="cuda")
            self.sigma_s[idx] = torch.as_tensor(ss, device="cuda")
            self.G[idx] = torch.as_tensor(G, device="cuda")
            self.g[idx] = torch.as_tensor(g, device="cuda")
            if self.psi is not None:
                self.psi[idx] = torch.as_tensor(np.stack([r.psi for r in reqs]), device="cuda")
            self.session.rho[idx] = 0.0
            self.session.admit(slots)        # synchronises the stream
        now = time.perf_counter() - t0
        for s, r in zip(slots, reqs):
            self.slot_req[s] = (r, now)
        return slots

    def step(self, t0: float) -> List[Result]:
        """One round of outer iterations; returns the requests that finished in it."""
        import torch
        before = self.session.active.copy()
        active = self.session.iterate(self.iters_per_round)
        done = [s for s in np.nonzero((before == 1) & (active == 0))[0]]
        now = time.perf_counter() - t0
        out = []
        for s in done:
            r, adm = self.slot_req.pop(int(s))
            rho = None
            if self.keep_rho:
                with torch.cuda.stream(self.stream):
                    rho = self.session.rho[int(s)].cpu().numpy()
            out.append(Result(r.rid, self.key, r.arrival, adm, now,
                              int(self.session.n_sweep[s]), int(self.session.status[s]), rho))
            self.free.append(int(s))
        return out

    @property
    def running(self) -> int:
        return len(self.slot_req)


class Server:
    """Runs a request stream through per-key slot pools with continuous batching."""

    def __init__(self, pools: Dict[tuple, KeyPool], budget_bytes: int):
        self.pools = pools
        self.budget = MemoryBudget(budget_bytes)
        for k, p in pools.items():
            if p.slot_bytes > budget_bytes:
                raise ValueError(f"one request of key {k} needs {p.slot_bytes} bytes, more than "
                                 f"the budget of {budget_bytes}")

    def run(self, requests: List[Request], time_scale: float = 1.0,
            on_result: Optional[Callable[[Result], None]] = None) -> List[Result]:
        """Serve ``requests`` (released at arrival * time_scale seconds) until all finished."""
        queues = {k: queue.Queue() for k in self.pools}
        results: List[Result] = []
        lock = threading.Lock()
        n_total = len(requests)
        errors = []
        t0 = time.perf_counter()
        counts = {k: sum(1 for r in requests if (r.n, r.n_phi) == k) for k in self.pools}

        def worker(key):
            pool = self.pools[key]
            pending: List[Request] = []
            left = counts[key]
            try:
                while left > 0:
                    block = pool.running == 0 and not pending
                    try:
                        while True:
                            item = queues[key].get(block=block, timeout=0.5 if block else None)
                            pending.append(item)
                            block = False
                    except queue.Empty:
                        pass
                    take = []
                    while (pending and len(take) < len(pool.free)
                           and self.budget.try_reserve(pool.slot_bytes)):
                        take.append(pending.pop(0))
                    if take:
                        pool.admit(take, t0)
                    if not pool.running:
                        if pending:                 # waiting for memory held by other keys
                            time.sleep(1e-3)
                        continue
                    if pool.running:
                        fin = pool.step(t0)
                        for _ in fin:
                            self.budget.release(pool.slot_bytes)
                        left -= len(fin)
                        with lock:
                            results.extend(fin)
                        if on_result:
                            for r in fin:
                                on_result(r)
            except BaseException as e:      # surfaced to the caller after the join
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(k,), daemon=True) for k in self.pools
                   if counts[k] > 0]
        for th in threads:
            th.start()
        for r in sorted(requests, key=lambda r: r.arrival):
            delay = r.arrival * time_scale - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            queues[(r.n, r.n_phi)].put(r)
            if errors:
                break
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        assert len(results) == n_total, (len(results), n_total)
        return sorted(results, key=lambda r: r.rid)


def lattice_request(rid: int, arrival: float, n: int, n_phi: int, seed: int) -> Request:
    """A request drawn like the parametric lattice with a left inflow (seeded materials)."""
    import rte_workloads as W
    pl = W.c2_lattice([seed], n=n, n_phi=n_phi, left_inflow=True)
    psi = np.concatenate([pl.block_sigma_t[0], pl.block_sigma_s[0]])
    return Request(rid, arrival, n, n_phi, pl.sigma_t[0], pl.sigma_s[0], pl.G[0], pl.g[0], psi)


def latency_summary(results: List[Result], wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    cd = sum(r.n_sweep * r.key[0] ** 2 * r.key[1] for r in results)
    return {"requests": len(results), "wall_s": wall, "solves_per_s": len(results) / wall,
            "cell_dir_updates_per_s": cd / wall,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_sweeps": float(np.mean([r.n_sweep for r in results])),
            "not_converged": int(sum(r.status != 0 for r in results))}
