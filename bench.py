"""Benchmark: MLUPS of the coupled flow + thermal step with 4800 particles.

Workload (default "paper_scale"): 4000 x 4000 periodic-x channel between
cold walls, 4800 hot circular particles of diameter 20 seeded uniformly at
random (seed 2, surface gaps >= 3 = the repulsion range), density ratio 1.5,
Pr 0.7, Ra 1e8, links
recollected every step, FP64.  One step = link collection, bounce-back and
momentum exchange, particle update, solid map, refilling and the fused
stream-collide over the whole lattice.  MLUPS counts every lattice node,
solid included (mesh size x steps / time).

Prints one JSON line.  Besides the throughput it carries:
  roofline     the fused stream-collide kernel (the dominant one), timed with
               HIP events around it on the library's stream in steps run as
               the timed ones (particle kernels concurrent on a second
               stream); achieved = algorithmic bytes per launch (every node
               reads and writes its 9 + 5 populations) / mean launch time,
               against 8 TB/s.
  cpu_baseline the CPU oracle (single thread, FP64) on a bounded sample of
               the same workload, timed on this host.
  paper_workload  the paper's own benchmark case (Sec. 2.6.3: closed 4000^2
               cavity, 60 x 80 hot particles of diameter 40, Pr 5, Gr_p 60,
               rho_p/rho_f = 1.1), a short timed run beside the paper's
               single-GPU figure for it (other hardware: context).  With
               --workload e4_cavity that case is the headline itself.
  serving      256 seeded requests (lattices 128..1024 on a side, aspect 1
               or 2, 5..400 particles of diameter 8..24, Ra 1e5..1e8, 500..5000
               steps, BF16 storage) served from a 2 GiB device budget: first
               all at t = 0 (closed loop, giving the capacity), then with
               Poisson arrivals at 0.8 x that capacity; p50/p99 latency
               (completion - arrival, queueing included), requests/s, MLUPS.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (coupled flow+thermal) at 4000², 4800 particles; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
STORE_BYTES = {"f64": 8, "f32": 4, "shift_f32": 4, "shift_f16": 2, "shift_bf16": 2}
STORE_DTYPE = {"f64": "f64", "f32": "f32", "shift_f32": "f32", "shift_f16": "f32 (f16 storage)",
               "shift_bf16": "f32 (bf16 storage)"}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2308_16597_amd", "csrc", f)
                  for f in ("lattice.hip", "lattice.h", "launch.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, storage, streaming="two_sets"):
    """HBM bytes per launch of the stream-collide kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    tag = "" if streaming == "two_sets" else "_in_place"
    path = os.path.join(ROOT, "profiles", f"stream_collide_{workload}_{storage}{tag}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def place(run, rows):
    """Particles of a workload into a run (library or oracle): rows of 7
    values are circles, rows of 8 ellipses."""
    rows = np.asarray(rows)
    (run.set_particles_ellipse if rows.shape[1] == 8 else run.set_particles)(rows)


def cpu_baseline(workload, steps):
    """The CPU oracle on `steps` steps of the same workload (one thread)."""
    import lbm_inputs
    from oracle import Oracle
    from paper_2308_16597_amd import params
    kw = params.workload_params(workload)
    w = params.WORKLOADS[workload]
    okw = {k: v for k, v in kw.items() if k not in ("storage", "max_particles", "max_diameter")}
    rows = lbm_inputs.workload_particles(w)
    orc = Oracle(**okw)
    place(orc, rows)
    orc.step(1)  # first touch of the oracle's arrays, not timed
    t0 = time.perf_counter()
    orc.step(steps)
    dt = time.perf_counter() - t0
    orc.close()
    return dict(value=round(params.mlups(w["nx"] * w["ny"], steps, dt), 4), unit="MLUPS", cores=1,
                kind="oracle",
                sample=f"steps 2..{steps + 1} of the {w['nx']}x{w['ny']} workload with {w['n']} "
                       f"particles (FP64, one thread): {dt:.1f} s")


def describe(name, storage):
    """One-line description of a named workload."""
    from paper_2308_16597_amd import params
    w = params.WORKLOADS[name]
    geom = "closed cavity" if w.get("closed") else "periodic-x channel"
    if "lattice" in w:
        lat = w["lattice"]
        phys = (f"nu={lat['nu']:g}, alpha={lat['alpha']:g}, g={lat['gravity']:g}, "
                f"beta={lat['beta']:g} (Pr={lat['nu'] / lat['alpha']:g})")
    else:
        phys = f"Pr={w['Pr']}, Ra={w['Ra']:g}"
    layout = w.get("layout")
    where = (f"{w['rows']}x{w['cols']} grid" if layout == "grid" else
             "ring cluster" if layout == "rings" else "random")
    shape = f"ellipses {w['d']:g}x{w['d_minor']:g}" if "d_minor" in w else f"d={w['d']:g}"
    return (f"{name}: {w['nx']}x{w['ny']} {geom}, {w['n']} hot particles {shape} ({where}), "
            f"rho_p/rho_f={w['rho_ratio']}, {phys}, {storage} storage, links rebuilt every step")


def paper_workload(steps, warmup, storage):
    """The paper's own benchmark case (closed 4000^2 cavity, 60 x 80
    particles of diameter 40, 6000 steps there), timed over `steps` steps
    after `warmup`, beside the paper's figure for it."""
    import torch
    import lbm_inputs
    from paper_2308_16597_amd import lbm, params
    name = "e4_cavity"
    w = params.WORKLOADS[name]
    sim = lbm.Sim(lbm.lbm_params_default(**params.workload_params(name, lbm.STORE[storage])))
    place(sim, lbm_inputs.workload_particles(w))
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    links = sim.stats()["links"]
    sim.close()
    v = params.mlups(w["nx"] * w["ny"], steps, dt)
    log(f"[bench] {name}: {steps} steps in {dt:.3f} s: {v:.1f} MLUPS")
    return dict(workload=describe(name, storage), steps=steps, warmup=warmup, mlups=round(v, 2),
                ms_per_step=round(dt / steps * 1e3, 5), links_per_step=links,
                paper_mlups=1750, ratio_to_paper=round(v / 1750.0, 3),
                paper_hardware="NVIDIA A100 40 GB (named for the paper's cluster), precision not stated")


def serving(n_req, budget_gib, chunk, streaming="two_sets"):
    import lbm_inputs
    from paper_2308_16597_amd import serve
    reqs = lbm_inputs.serving_requests(n_req, seed=4)
    srv = serve.Server(int(budget_gib * (1 << 30)), storage="shift_bf16", chunk=chunk, streaming=streaming)
    t0 = time.perf_counter()
    prog = lambda k, n: log(f"[bench] serving: {k}/{n} requests done")  # noqa: E731
    closed = srv.run(reqs, np.zeros(n_req), prog)
    closed_sum = serve.summarize(closed, time.perf_counter() - t0)
    log(f"[bench] serving closed loop: {closed_sum}")
    lam = 0.8 * closed_sum["req_per_s"]
    arr = lbm_inputs.poisson_arrivals(n_req, lam, seed=4)
    t0 = time.perf_counter()
    opened = srv.run(reqs, arr, prog)
    s = serve.summarize(opened, time.perf_counter() - t0)
    log(f"[bench] serving open loop at {lam:.2f} req/s: {s}")
    return dict(requests=n_req, budget_gib=budget_gib, storage="shift_bf16", chunk_steps=chunk,
                streaming=streaming,
                closed_loop=dict(wall_s=round(closed_sum["wall_s"], 3),
                                 req_per_s=round(closed_sum["req_per_s"], 3),
                                 mlups=round(closed_sum["mlups"], 1), failed=closed_sum["failed"]),
                arrival_rate_req_per_s=round(lam, 3),
                p50_s=round(s["p50_s"], 4), p99_s=round(s["p99_s"], 4),
                req_per_s=round(s["req_per_s"], 3), mlups=round(s["mlups"], 1),
                completed=s["completed"], failed=s["failed"], ra_capped=s["ra_capped"])


def copy_probe(nbytes, reps=5):
    """Plain device-to-device copies of a known size: the reference that the
    hardware byte counters of the stream-collide kernel are scaled by."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy probe: {reps} copies of {a.numel() * 8} bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="paper_scale")
    ap.add_argument("--storage", default="f64", choices=sorted(STORE_BYTES))
    ap.add_argument("--streaming", default="two_sets", choices=["two_sets", "in_place"],
                    help="population layout: two sets (pull) or one set in place (AA pattern)")
    ap.add_argument("--phase-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-paper-workload", action="store_true",
                    help="skip the short timed run of the paper's closed-cavity case")
    ap.add_argument("--paper-steps", type=int, default=600)
    ap.add_argument("--addressing", default="indirect", choices=["indirect", "direct"],
                    help="link pass by indirect (default) or direct addressing (the ablation)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run plain copies of this many bytes (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-budget-gib", type=float, default=2.0)
    ap.add_argument("--serve-chunk", type=int, default=120)
    ap.add_argument("--serve-streaming", default="two_sets", choices=["two_sets", "in_place"])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the lattice would shard as y-slabs with a three-row halo)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    from paper_2308_16597_amd import lbm, params

    w = params.WORKLOADS[args.workload]
    nx, ny = w["nx"], w["ny"]
    p = lbm.lbm_params_default(**params.workload_params(args.workload, lbm.STORE[args.storage]),
                               streaming=args.streaming)
    log(f"[bench] {args.workload} {nx}x{ny} n={w['n']} d={w['d']} storage={args.storage}")
    import lbm_inputs
    sim = lbm.Sim(p)
    place(sim, lbm_inputs.workload_particles(w))
    if args.addressing != "indirect":
        sim.set_addressing(args.addressing)
    sim.step(args.warmup)
    sim.sync()
    log(f"[bench] warmup {args.warmup} steps done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mlups = params.mlups(nx * ny, args.steps, dt)
    log(f"[bench] timed {args.steps} steps in {dt:.3f} s: {mlups:.1f} MLUPS")

    phases = sim.time_phases(args.phase_steps)
    stats = sim.stats()
    owner = sim.fields()["owner"]
    n_fluid = int((owner < 0).sum())
    es = STORE_BYTES[args.storage]
    alg_bytes = nx * ny * 28 * es
    lat_ms = phases["lattice_overlapped"]   # as the kernel runs in the timed steps
    achieved = alg_bytes / (lat_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, args.storage, args.streaming)
    log(f"[bench] phases (ms/step): {phases}")

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(mlups / 1750.0, 4) if args.workload == "e4_cavity" else None,
        "dtype": STORE_DTYPE[args.storage],
        "data": "synthetic",
        "config": {
            "workload": describe(args.workload, args.storage)
                        + ("" if args.addressing == "indirect" else ", direct link addressing")
                        + ("" if args.streaming == "two_sets" else ", in-place (AA) streaming"),
            "nx": nx, "ny": ny, "particles": w["n"], "diameter": w["d"], "storage": args.storage,
            "streaming": args.streaming, "device_bytes": lbm.lbm_bytes_required(p),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stream_collide" if args.streaming == "two_sets" else "k_stream_collide_aa",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": alg_bytes,
            "launch_ms": round(lat_ms, 5),
            "launch_ms_alone": round(phases["lattice"], 5),
        },
        "phases_ms": {k: round(v, 5) for k, v in phases.items()},
        # context only: the paper's single-GPU figure, other hardware and workload
        "paper_context": {"mlups": 1750, "hardware": "NVIDIA A100 40 GB (named for the paper's cluster)",
                          "precision": "not stated",
                          "workload": "closed cavity 4000^2, 4800 particles d=40, 6000 steps"},
        "links_per_step": stats["links"],
        "fluid_nodes": n_fluid,
    }
    sim.close()
    del sim
    if args.workload == "paper_scale" and not args.no_paper_workload:
        out["paper_workload"] = paper_workload(args.paper_steps, 20, args.storage)
    if not args.no_serve:
        out["serving"] = serving(args.serve_requests, args.serve_budget_gib, args.serve_chunk,
                                 args.serve_streaming)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
