"""Benchmark: MLUPS of the coupled flow + thermal step with 4800 particles.

Workload (default "paper_scale"): 4000 x 4000 periodic-x channel between
cold walls, 4800 hot circular particles of diameter 20 seeded uniformly at
random (seed 2, surface gaps >= 3 = the repulsion range), density ratio 1.5,
Pr 0.7, Ra 1e8, links
recollected every step, FP64.  One step = link collection, bounce-back and
momentum exchange, particle update, solid map, refilling and the fused
stream-collide over the whole lattice.  MLUPS counts every lattice node,
solid included (mesh size x steps / time).

Timing: after the warm-up steps, the timed calls of `--steps` steps are
rehearsed once untimed (so every step graph they replay is captured before
timing starts), then each of `--repeats` calls is timed between full
synchronisations; the value is the median.  The defaults (50 + 5 x 200 +
5 x 200 steps) keep the run near the workload's nominal 2000 steps.

Prints one JSON line.  Besides the throughput it carries:
  roofline     the fused stream-collide kernel (the dominant one), timed with
               HIP events around it on the library's stream in steps run as
               the timed ones (particle kernels concurrent on a second
               stream); achieved = algorithmic bytes per launch (every node
               reads and writes its 9 + 5 populations) / mean launch time,
               against 8 TB/s; beside it a plain copy of the same 14 arrays
               with the same grid (the copy ceiling).
  step_roofline  the step's MLUPS against the MLUPS of moving the
               algorithmic bytes at 8 TB/s.
  forms        the same workload in the other storage forms (FP32, FP16 and
               BF16 deviations): step MLUPS and the lattice kernel's fraction.
  cpu_baseline the CPU oracle (single thread, FP64) on a bounded sample of
               the same workload (`--cpu-steps` steps after one untimed) and
               all 200 steps of the small 256^2 workload, timed on this host,
               with its CPU model and core counts.
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


def padded_bytes(nx, ny, es):
    """Bytes a copy of the 14 population arrays moves: rows padded to a
    multiple of 64 nodes, each value read and written."""
    return ((nx + 63) // 64 * 64) * ny * 28 * es


def place(run, rows):
    """Particles of a workload into a run (library or oracle): rows of 7
    values are circles, rows of 8 ellipses."""
    rows = np.asarray(rows)
    (run.set_particles_ellipse if rows.shape[1] == 8 else run.set_particles)(rows)


def cpu_info():
    """Host CPU model, logical CPUs of the host and CPUs this process may use."""
    model = "unknown"
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
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def oracle_mlups(workload, steps, untimed=1):
    """MLUPS of the CPU oracle (one thread, FP64) over `steps` steps of a
    named workload, after `untimed` first-touch steps."""
    import lbm_inputs
    from oracle import Oracle
    from paper_2308_16597_amd import params
    kw = params.workload_params(workload)
    w = params.WORKLOADS[workload]
    okw = {k: v for k, v in kw.items() if k not in ("storage", "max_particles", "max_diameter")}
    orc = Oracle(**okw)
    place(orc, lbm_inputs.workload_particles(w))
    if untimed:
        orc.step(untimed)
    t0 = time.perf_counter()
    orc.step(steps)
    dt = time.perf_counter() - t0
    orc.close()
    return params.mlups(w["nx"] * w["ny"], steps, dt), dt


def cpu_baseline(workload, steps, small_steps):
    """The CPU oracle on this host (one thread): `steps` steps of the timed
    workload (the value) and `small_steps` steps of the small 256^2
    workload, with the CPU model and core counts."""
    from paper_2308_16597_amd import params
    w = params.WORKLOADS[workload]
    model, ncpu, usable = cpu_info()
    v, dt = oracle_mlups(workload, steps)
    out = dict(value=round(v, 4), unit="MLUPS", cores=1, kind="oracle",
               sample=f"steps 2..{steps + 1} of the {w['nx']}x{w['ny']} workload with {w['n']} "
                      f"particles (FP64, one thread, after one untimed first-touch step): {dt:.1f} s",
               cpu_model=model, host_cpus=ncpu, usable_cpus=usable, threads=1)
    if small_steps > 0 and workload != "small":
        ws = params.WORKLOADS["small"]
        vs, dts = oracle_mlups("small", small_steps, untimed=0)
        out["small"] = dict(value=round(vs, 4), unit="MLUPS", steps=small_steps, seconds=round(dts, 2),
                            workload=f"{ws['nx']}x{ws['ny']} channel, {ws['n']} particles d={ws['d']:g}, "
                                     f"steps 1..{small_steps}")
    return out


def timed_repeats(sim, steps, repeats):
    """Device seconds of `repeats` calls of sim.step(steps), each bracketed
    by a full synchronisation, after one untimed rehearsal of the same calls
    (which captures the step graph of every step state a call starts from,
    so no capture falls in a timed call) and a return to the starting step
    state.  Returns the list of times."""
    import torch
    for _ in range(repeats):
        sim.step(steps)
    pad = (-repeats * steps) % 6   # the step state repeats every 6 steps
    if pad:
        sim.step(pad)
    sim.sync()
    out = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    if pad:
        sim.step(pad)
    return out


def form_line(workload, storage, steps, warmup, repeats, phase_steps):
    """Throughput of one precision form on the workload: step MLUPS (median
    of `repeats` timed calls of `steps` steps), the lattice kernel's HBM
    fraction in the overlapped steps and alone, and the copy ceiling."""
    import lbm_inputs
    from paper_2308_16597_amd import lbm, params
    w = params.WORKLOADS[workload]
    nx, ny = w["nx"], w["ny"]
    sim = lbm.Sim(lbm.lbm_params_default(**params.workload_params(workload, lbm.STORE[storage])))
    place(sim, lbm_inputs.workload_particles(w))
    sim.step(warmup)
    sim.sync()
    dts = timed_repeats(sim, steps, repeats)
    dt = float(np.median(dts))
    ph = sim.time_phases(phase_steps)
    copy_ms = sim.time_copy(10)
    sim.close()
    es = STORE_BYTES[storage]
    alg = nx * ny * 28 * es
    roof = HBM_PEAK_GBS * 1e9 / (28 * es) / 1e6
    v = params.mlups(nx * ny, steps, dt)
    frac = lambda ms: round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)  # noqa: E731
    line = dict(storage=storage, dtype=STORE_DTYPE[storage], mlups=round(v, 1),
                ms_per_step=round(dt / steps * 1e3, 5), repeats_mlups=[round(params.mlups(nx * ny, steps, t), 1) for t in dts],
                roofline_mlups=round(roof, 1), step_frac=round(v / roof, 4),
                lattice_frac=frac(ph["lattice_overlapped"]), lattice_frac_alone=frac(ph["lattice"]),
                lattice_ms=round(ph["lattice_overlapped"], 5), link_pass_ms=round(ph["links"], 5),
                copy_ms=round(copy_ms, 5),
                copy_frac=round(padded_bytes(nx, ny, es) / (copy_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    log(f"[bench] form {storage}: {line}")
    return line


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
    dt = timed_repeats(sim, steps, 1)[0]
    links = sim.stats()["links"]
    sim.close()
    v = params.mlups(w["nx"] * w["ny"], steps, dt)
    log(f"[bench] {name}: {steps} steps in {dt:.3f} s: {v:.1f} MLUPS")
    return dict(workload=describe(name, storage), steps=steps, warmup=warmup, mlups=round(v, 2),
                ms_per_step=round(dt / steps * 1e3, 5), links_per_step=links,
                paper_mlups=1750, ratio_to_paper=round(v / 1750.0, 3),
                paper_hardware="NVIDIA A100 40 GB (named for the paper's cluster), precision not stated")


def serving(n_req, budget_gib, chunk, streaming="two_sets", storage="shift_bf16"):
    import lbm_inputs
    from paper_2308_16597_amd import serve
    reqs = lbm_inputs.serving_requests(n_req, seed=4)
    srv = serve.Server(int(budget_gib * (1 << 30)), storage=storage, chunk=chunk, streaming=streaming)
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
    r4 = lambda v: None if v is None else round(v, 4)  # noqa: E731
    sub = lambda d: dict(completed=d["completed"], p50_s=r4(d["p50_s"]), p99_s=r4(d["p99_s"]),  # noqa: E731
                         mlups=None if d["mlups"] is None else round(d["mlups"], 1))
    return dict(requests=n_req, budget_gib=budget_gib, storage=storage, chunk_steps=chunk,
                streaming=streaming,
                accuracy=("FP16 deviations: eps_T 6e-3, eps_u 8e-4 against the FP64 oracle after 2000 steps"
                          if storage == "shift_f16" else
                          "throughput form: BF16 deviations lose small temperature increments "
                          "(eps_T 0.39 against the FP64 oracle after 2000 steps)"
                          if storage == "shift_bf16" else "see the precision forms"),
                closed_loop=dict(wall_s=round(closed_sum["wall_s"], 3),
                                 req_per_s=round(closed_sum["req_per_s"], 3),
                                 mlups=round(closed_sum["mlups"], 1), failed=closed_sum["failed"]),
                arrival_rate_req_per_s=round(lam, 3),
                p50_s=r4(s["p50_s"]), p99_s=r4(s["p99_s"]),
                req_per_s=round(s["req_per_s"], 3), mlups=round(s["mlups"], 1),
                completed=s["completed"], failed=s["failed"], ra_capped=s["ra_capped"],
                uncapped=sub(s["uncapped"]), capped=sub(s["capped"]))


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
    ap.add_argument("--steps", type=int, default=200,
                    help="steps per timed call; with the warm-up, the rehearsal and 5 repeats the default run "
                         "covers about the workload's nominal 2000 steps (its settling particles keep "
                         "accelerating: past about 12 000 steps one moves more than half a node per step)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="paper_scale")
    ap.add_argument("--storage", default="f64", choices=sorted(STORE_BYTES))
    ap.add_argument("--streaming", default="two_sets", choices=["two_sets", "in_place"],
                    help="population layout: two sets (pull) or one set in place (AA pattern)")
    ap.add_argument("--phase-steps", type=int, default=100)
    ap.add_argument("--repeats", type=int, default=5, help="timed calls of --steps steps; the median counts")
    ap.add_argument("--cpu-steps", type=int, default=5,
                    help="oracle steps timed on the headline workload (one thread)")
    ap.add_argument("--cpu-small-steps", type=int, default=200,
                    help="oracle steps timed on the small 256^2 workload")
    ap.add_argument("--forms", default="f32,shift_f16,shift_bf16",
                    help="other storage forms timed beside the headline one (comma list, '' for none)")
    ap.add_argument("--form-steps", type=int, default=120)
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
    ap.add_argument("--serve-storage", default="shift_bf16,shift_f16",
                    help="storage forms of the served runs, one serving pass each (the first is 'serving')")
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

    dts = timed_repeats(sim, args.steps, args.repeats)
    dt = float(np.median(dts))
    mlups = params.mlups(nx * ny, args.steps, dt)
    log(f"[bench] timed {args.repeats} x {args.steps} steps: "
        f"{[round(params.mlups(nx * ny, args.steps, t), 1) for t in dts]} MLUPS; median {mlups:.1f}")

    phases = sim.time_phases(args.phase_steps)
    copy_ms = sim.time_copy(10)
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
        "repeats": args.repeats,
        "repeats_mlups": [round(params.mlups(nx * ny, args.steps, t), 2) for t in dts],
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
            # a plain copy of the same 14 arrays (rows padded to 64 nodes)
            "copy_ceiling_ms": round(copy_ms, 5),
            "copy_ceiling_frac": round(padded_bytes(nx, ny, es) / (copy_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "step_roofline": {
            "mlups_at_peak": round(HBM_PEAK_GBS * 1e9 / (28 * es) / 1e6, 1),
            "frac": round(mlups / (HBM_PEAK_GBS * 1e9 / (28 * es) / 1e6), 4),
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
    forms = [f for f in args.forms.split(",") if f and f != args.storage]
    if forms:
        out["forms"] = {f: form_line(args.workload, f, args.form_steps, 20, args.repeats, 50) for f in forms}
    if args.workload == "paper_scale" and not args.no_paper_workload:
        out["paper_workload"] = paper_workload(args.paper_steps, 20, args.storage)
    if not args.no_serve:
        forms_s = [f for f in args.serve_storage.split(",") if f]
        for k, f in enumerate(forms_s):
            out["serving" if k == 0 else f"serving_{f}"] = serving(
                args.serve_requests, args.serve_budget_gib, args.serve_chunk, args.serve_streaming, f)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps (+ {args.cpu_small_steps} on 256^2)")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_steps, args.cpu_small_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
