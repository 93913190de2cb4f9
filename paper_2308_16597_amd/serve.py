"""Serving many independent simulations on one GPU.

A request is one particle-laden thermal channel (its own lattice size,
particle count and diameter, Rayleigh number and step count).  The server
keeps every admitted run resident in one device arena of a fixed byte
budget, admits queued requests first-come first-served while their
footprint (`lbm_bytes_required`) fits, and advances all resident runs
together with `lbm_step_many` (batched step kernels over a run table, one
captured graph per 6-step cycle of an unchanged set of runs), in chunks of
at most `chunk` steps.  A request completes when its last step has run and
its particle state has been read back; its latency is completion minus
arrival on the host's monotonic clock, queueing included.
"""
import bisect
import ctypes
import math
import time

import numpy as np

from . import lbm, params

# Smallest viscosity a request may use (relaxation time 0.53); a request
# whose Rayleigh number asks for less runs at this viscosity and is marked
# "Ra capped".  Below it the hot plumes are under-resolved on these lattices:
# at 1/300 (relaxation time 0.51) a 129^2 channel at Ra 8e7 overshoots T = 1
# by 100 % and diverges within 1750 steps, in FP64 as in every storage form.
NU_MIN = 0.01
ALIGN = 1 << 16


def request_params(req, storage=lbm.STORE["shift_bf16"], streaming=lbm.STREAMING["two_sets"]):
    """lbm_params of one request: hot particles (T = 1) in a cold channel,
    parameters from (H = ny, Ra, Pr 0.7, d, density ratio 1.5) at Ma 0.1."""
    phys = params.from_dimensionless(req["ny"], req["Ra"], 0.7, req["d"], 1.5)
    capped = phys["nu"] < NU_MIN
    nu = max(phys["nu"], NU_MIN)
    p = lbm.lbm_params_default(
        nx=req["nx"], ny=req["ny"], storage=storage, rho0=1.0, nu=nu, alpha=nu / 0.7,
        gravity=phys["gravity"], beta=phys["beta"], T_ref=0.0, wall_T=(0.0, 0.0), T_fluid0=0.0,
        particle_T=1.0, rho_ratio=1.5, repulsion=1, rep_eps=1e-3, rep_range=3.0, T_shift=0.0,
        max_particles=max(req["n"], 1), max_diameter=req["d"], streaming=streaming)
    return p, capped


class FirstFit:
    """First-fit sub-allocation of [0, nbytes) in 64 KiB aligned pieces."""

    def __init__(self, nbytes):
        self.nbytes = int(nbytes)
        self.free = [(0, self.nbytes)]   # sorted (offset, size), adjacent pieces merged

    def alloc(self, n):
        n = (int(n) + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, size - n)
                return off, n
        return None

    def release(self, off, n):
        i = bisect.bisect(self.free, (off, n))
        self.free.insert(i, (off, n))
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def used(self):
        return self.nbytes - sum(s for _, s in self.free)


class Arena(FirstFit):
    """One device buffer of the budget's size, sub-allocated first fit."""

    def __init__(self, nbytes):
        import torch
        super().__init__(nbytes)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        self.base = self.buf.data_ptr()


class Server:
    """`streaming`: "two_sets" or "in_place" (one population set per run, so
    about twice the runs fit the budget)."""

    def __init__(self, budget_bytes, storage="shift_bf16", chunk=120, gap=3.0, streaming="two_sets"):
        import torch
        self.storage = lbm.STORE[storage]
        self.streaming = lbm.STREAMING[streaming]
        self.arena = Arena(budget_bytes)
        self.chunk = int(chunk)
        self.gap = gap
        self.stream = torch.cuda.Stream()

    def footprint(self, req):
        p, _ = request_params(req, self.storage, self.streaming)
        return lbm.lbm_bytes_required(p)

    def run(self, requests, arrivals, progress=None):
        """Serve `requests` arriving at `arrivals` (seconds from the start).
        Returns one record per request (arrival, admit, done, latency in
        seconds, status).  `progress(n_done, n_total)` is called after every
        32 completions."""
        order = np.argsort(arrivals, kind="stable")
        pending = [int(i) for i in order]
        queue, active, records = [], [], {}
        sptr = self.stream.cuda_stream
        t0 = time.perf_counter()
        nxt = reported = 0
        while nxt < len(pending) or queue or active:
            now = time.perf_counter() - t0
            while nxt < len(pending) and arrivals[pending[nxt]] <= now:
                queue.append(pending[nxt])
                nxt += 1
            while queue:   # first come, first served while the footprint fits
                i = queue[0]
                req = requests[i]
                p, capped = request_params(req, self.storage, self.streaming)
                need = lbm.lbm_bytes_required(p)
                rc = lbm.lbm_check_budget(p, self.arena.nbytes)
                if rc != lbm.LBM_OK:   # invalid, or larger than the whole budget (LBM_EBUDGET)
                    queue.pop(0)
                    why = "over budget" if rc == lbm.LBM_EBUDGET else "invalid parameters"
                    records[i] = dict(rid=req["rid"], status=f"rejected: {why}", arrival=arrivals[i])
                    continue
                got = self.arena.alloc(need)
                if got is None:
                    break
                queue.pop(0)
                sim = lbm.Sim(p, arena=(self.arena.base + got[0], got[1]), stream=sptr)
                try:
                    if req["n"] > 0:
                        sim.seed_particles(req["n"], req["d"], self.gap, req["seed"])
                except lbm.LbmError as e:
                    sim.close()
                    self.arena.release(*got)
                    records[i] = dict(rid=req["rid"], status=f"seeding failed: {e}", arrival=arrivals[i])
                    continue
                active.append(dict(i=i, sim=sim, left=int(req["steps"]), mem=got, capped=capped,
                                   admit=time.perf_counter() - t0))
            if not active:
                if nxt < len(pending):
                    time.sleep(max(0.0, arrivals[pending[nxt]] - (time.perf_counter() - t0)))
                continue
            counts = [min(a["left"], self.chunk) for a in active]
            lbm.step_many([a["sim"] for a in active], counts, ctypes.c_void_p(sptr))
            self.stream.synchronize()
            still = []
            for a, c in zip(active, counts):
                a["left"] -= c
                status = "ok"
                try:   # device errors of the run (a failed run is retired at once)
                    a["sim"].sync()
                except lbm.LbmError as e:
                    status = f"unstable: {e}"
                if a["left"] > 0 and status == "ok":
                    still.append(a)
                    continue
                req = requests[a["i"]]
                if status == "ok":
                    try:
                        a["result"] = a["sim"].particles()
                    except lbm.LbmError as e:
                        status = f"unstable: {e}"
                done = time.perf_counter() - t0
                a["sim"].close()
                self.arena.release(*a["mem"])
                records[a["i"]] = dict(rid=req["rid"], status=status, arrival=float(arrivals[a["i"]]),
                                       admit=a["admit"], done=done, latency=done - float(arrivals[a["i"]]),
                                       nodes=req["nx"] * req["ny"], steps=req["steps"] - a["left"],
                                       ra_capped=a["capped"], particles=a.get("result"))
            if progress is not None and len(records) >= reported + 32:
                reported = len(records)
                progress(reported, len(requests))
            active = still
        return [records[i] for i in range(len(requests))]


def percentile_nearest_rank(values, q):
    """Nearest-rank percentile: the ceil(q n)-th smallest value."""
    v = sorted(values)
    k = max(1, math.ceil(q * len(v)))
    return v[k - 1]


def summarize(records, wall):
    """Completed requests' latency percentiles (nearest rank), throughput
    over the wall time, and the same for the requests that ran at their
    requested Rayleigh number and for those whose viscosity was raised to
    NU_MIN ("Ra capped"), separately."""
    ok = [r for r in records if r["status"] == "ok"]

    def part(rs):
        lat = [r["latency"] for r in rs]
        lups = sum(r["nodes"] * r["steps"] for r in rs)
        return dict(completed=len(rs),
                    p50_s=percentile_nearest_rank(lat, 0.50) if lat else None,
                    p99_s=percentile_nearest_rank(lat, 0.99) if lat else None,
                    mlups=lups / wall / 1e6 if wall > 0 else None)

    out = dict(requests=len(records), failed=len(records) - len(ok), wall_s=wall,
               req_per_s=len(ok) / wall if wall > 0 else None,
               ra_capped=sum(1 for r in ok if r.get("ra_capped")))
    out.update(part(ok))
    out["uncapped"] = part([r for r in ok if not r.get("ra_capped")])
    out["capped"] = part([r for r in ok if r.get("ra_capped")])
    return out
