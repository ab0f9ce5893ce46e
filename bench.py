"""Benchmark of the fused MRTLB-VANSE step on one MI355X.

Workload (the channel configuration the throughput metric is quoted on):
a single 4096 x 4096 D2Q9 channel, half-way bounce-back walls at y = 0 and
y = H, periodic in x, body force G = 1e-7 along x (F^B = phi G), phi a tanh
step from 0.4 to 1.0 (width 2 cells) at mid-channel plus seeded smoothed
noise of amplitude 0.05 (sigma = 8 cells), kappa = 0.5, s_nu = 0.8 and the
other rates 1.2, FP32 arithmetic and FP32 storage (of the deviations from the
rest state).  A "step" is one time step of the whole lattice; the plain step
runs two time steps per launch of its two-step kernel (the populations cross
HBM once per two steps).

Prints ONE JSON line (rank 0).  `value` is MLUPS (million lattice-node
updates per second) over the median of `--windows` timed windows of exactly
`--steps` steps each, inputs resident in HBM.  The `roofline` object prices
the step kernel against the 8 TB/s HBM peak.  `achieved` is the bytes one
launch must move through HBM -- each stored population read once and
written once, phi read once: 76 B per node in FP32, whether the launch
advances the node by one step or by two -- over the launch duration, timed
with HIP events on the stream the kernel is launched on; `frac` is that
over the peak.  `effective_gbs` counts the node updates' algorithmic bytes
instead (76 B per update, two updates per node and launch for the two-step
kernel), which exceeds the HBM peak when two updates share one pass.
`traffic` is the HBM bytes one launch actually moves (rocprofv3 FETCH_SIZE +
WRITE_SIZE, calibrated on the copy kernel, read from the committed record
when it was taken on the current kernel code), `traffic_frac` that rate
over the peak.  `gpu_state` holds rocm-smi clock, power and temperature
readings before the warmup and after the timed windows, and `settle` the
untimed stepping between the warmup and the timed windows that lets the
shader clock rise.  `cpu_baseline` times the FP64
CPU oracle on a bounded sample of the same workload.
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

NX = NY = 4096
G = 1e-7
KAPPA = 0.5
RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)
PRECISION = "f32s"  # FP32 arithmetic, FP32 storage of the deviations (76 B per node update)
TILING = (256, 69)  # single-step launches: threads per workgroup, rows per workgroup
STEPS_PER_PASS = 2  # time steps per launch of the plain step
HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS + %HBM peak (D2Q9 MRT-VANSE); batched solves/s + p99 latency"
BYTES_PER_NODE = {"f64": 9 * 8 * 2 + 8, "f32": 9 * 4 * 2 + 4, "f32s": 9 * 4 * 2 + 4,
                  "f16s": 9 * 2 * 2 + 4}
KERNEL_SOURCES = ["paper_2409_02964_amd/csrc/step_kernel.hpp",
                  "paper_2409_02964_amd/csrc/step2_kernel.hpp",
                  "paper_2409_02964_amd/build.py"]  # (its compiler flags)
PROFILE_PREFIX = os.path.join(ROOT, "profiles", "step2_f32s_channel4096")
TRAFFIC_FILE = PROFILE_PREFIX + "_traffic.json"


def kernel_hash() -> str:
    """Hash of the step kernels' code: the sources with comments and
    whitespace removed, so that the traffic record follows code changes only."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        src = open(os.path.join(ROOT, p)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, when
    they were taken on the current kernel source; else None."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def gpu_clocks():
    """Clock, power and temperature readings of the GPU from rocm-smi (a
    short dict; the error text if the tool is not usable)."""
    import subprocess
    if "rocprofiler" in os.environ.get("LD_PRELOAD", ""):
        return {"skipped": "under a profiler"}
    try:
        out = subprocess.run(["rocm-smi", "--showclocks", "--showpower", "--showtemp", "--json"],
                             capture_output=True, text=True, timeout=20)
        rec = json.loads(out.stdout)
    except (OSError, ValueError, subprocess.SubprocessError) as e:
        return {"error": str(e)[:200]}
    keep = {}
    for card, vals in rec.items():
        if not isinstance(vals, dict):
            continue
        for k, v in vals.items():
            kl = k.lower()
            if any(w in kl for w in ("sclk", "mclk", "fclk", "power", "junction", "memory")):
                keep[f"{card}:{k}"] = v
        break
    return keep


def cpu_baseline(steps: int, single_steps: int = 3):
    """The FP64 oracle on the same channel: `steps` full-lattice steps on up
    to 16 OpenMP threads (the reported value), and `single_steps` on one."""
    import numpy as np
    from oracle import oracle as O
    from paper_2409_02964_amd import workloads as W
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    phi = W.channel_phi(NX, NY, seed=2409)

    def run(threads, n):
        used = O.set_threads(threads)
        o = O.Oracle(NX, NY, phi, kappa=KAPPA, rates=RATES, g=(G, 0.0), bc_y="wall")
        o.init_equilibrium()
        t0 = time.perf_counter()
        o.step(n)
        dt = time.perf_counter() - t0
        assert np.isfinite(o.f[:, ::512, ::512]).all()
        return used, dt

    out = {}
    if single_steps > 0:
        _, dt1 = run(1, single_steps)
        out["single_thread"] = dict(value=round(NX * NY * single_steps / dt1 / 1e6, 2),
                                    sample=f"{single_steps} full steps, 1 thread ({dt1:.1f} s)")
    cores, dt = run(max(1, min(16, avail)), steps)
    return dict(value=NX * NY * steps / dt / 1e6, unit="MLUPS", cores=cores, kind="oracle",
                sample=f"{steps} full steps of the {NX}x{NY} channel, FP64, {cores} OpenMP "
                       f"threads ({dt:.1f} s)", host_cpus=os.cpu_count(), affinity=avail, **out)


def small_bench(steps: int = 1000, graph_steps: int = 100):
    """The 64 x 64 periodic-wave workload (phi = 0.75 + 0.2 sin cos, G = 1e-6,
    FP64, the parity case): far too small to fill the GPU, so bound by the
    latency of a launch and of the row sweep; timed with one launch per step
    and with the step loop captured in hipGraphs (a one-lattice batch)."""
    import torch
    from paper_2409_02964_amd import workloads as W
    from paper_2409_02964_amd.vanse import Batch, Lattice

    n = 64
    lat = Lattice(n, n, precision="f64")
    lat.set_params(KAPPA, RATES).set_body_force(1e-6, 0.0).set_void_fraction(W.periodic_wave(n, n))
    lat.init_equilibrium(1.0)
    lat.step(50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    tl = lat.tiling()  # the single-lattice launch shape, so only the launch path differs
    b = Batch([lat], threads=tl["threads"], rows=tl["rows"], graph_steps=graph_steps)
    b.step(graph_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    b.close()
    return {"workload": f"periodic wave {n}x{n}, FP64, {steps} steps",
            "plain_us_per_step": round(t_plain / steps * 1e6, 2),
            "plain_mlups": round(n * n * steps / t_plain / 1e6, 1),
            "graph_us_per_step": round(t_graph / steps * 1e6, 2),
            "graph_mlups": round(n * n * steps / t_graph / 1e6, 1), "graph_steps": graph_steps}


def batched_bench(steps: int, baseline_steps: int, graph_steps: int = 100):
    """Batched workload: 256 independent periodic lattices, sides log-uniform
    in [32, 512] (seed 4), phi = 0.6 + 0.3 sin(2 pi kx x/L) sin(2 pi ky y/L),
    |G| ~ U[1e-7, 1e-5] along x, FP32, `steps` steps, one launch per step (or
    per two steps) over all lattices (autotuned launch shape, hipGraph-captured
    loop).  The comparison is the plain path with one launch per lattice per
    step."""
    import torch
    from paper_2409_02964_amd import workloads as W
    from paper_2409_02964_amd.vanse import Batch, Lattice, autotune_batch

    specs = W.batch_lattices(256, seed=4)

    def build():
        lats = []
        for sp in specs:
            lat = Lattice(sp["L"], sp["L"], precision=PRECISION)
            lat.set_params(KAPPA, RATES).set_body_force(sp["g"], 0.0).set_void_fraction(sp["phi"])
            lat.init_equilibrium(1.0)
            lats.append(lat)
        return lats

    nodes = sum(sp["L"] ** 2 for sp in specs)
    lats = build()
    best, _ = autotune_batch(lats, candidates=[(128, 16), (256, 0), (64, 16), (128, 0, 2),
                                               (128, 24, 2), (128, 32, 2), (128, 40, 2), (128, 48, 2),
                                               (128, 64, 2), (256, 48, 2), (64, 24, 2),
                                               (64, 32, 2), (64, 40, 2), (64, 64, 2)],
                             steps=40, repeats=3)
    for lat in lats:
        lat.init_equilibrium(1.0)
    b = Batch(lats, threads=best[0], rows=best[1], graph_steps=graph_steps, steps_per_pass=best[2])
    b.step(graph_steps)
    torch.cuda.synchronize()
    for lat in lats:
        lat.init_equilibrium(1.0)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    b.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    t_batch = ev0.elapsed_time(ev1) / 1e3
    # plain path: one launch per lattice per step (timed on fewer steps)
    for lat in lats:
        lat.init_equilibrium(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(baseline_steps):
        for lat in lats:
            lat.step(1)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) * steps / baseline_steps
    return {"workload": "256 periodic lattices, L log-uniform 32..512 (seed 4), FP32, "
                        f"{steps} steps", "lattices": len(specs), "nodes": nodes,
            "steps": steps, "steps_per_launch": best[2], "threads": best[0],
            "rows": b.tiles()["rows"],
            "tiles": b.tiles()["tiles"], "graph_steps": graph_steps,
            "solves_per_s": round(len(specs) / t_batch, 2),
            "mlups": round(nodes * steps / t_batch / 1e6, 1),
            "plain_one_launch_per_lattice_solves_per_s": round(len(specs) / t_plain, 2),
            "plain_mlups": round(nodes * steps / t_plain / 1e6, 1),
            "speedup": round(t_plain / t_batch, 2)}


def served_bench(count: int, rate: float, budget_gib: float, precision: str = "f16s",
                 tol: float = 1e-8, steps_per_pass: int = 1,
                 modes=("continuous_batching", "one_at_a_time")):
    """Served workload: `count` solve requests with Poisson arrivals at `rate`
    per second, periodic lattices with sides log-uniform in [64, 2048] and
    tanh-edged inclusions (phi in [0.35, 1]), G = 1e-6, drag 2e-3 + 1e-2 (1 -
    phi), FP32 arithmetic with FP16 shifted storage, run to a residual of 1e-8
    or 20000 steps, admitted by device memory within `budget_gib`, one time
    step per launch.  Compared with the same server restricted to one solve
    at a time (FIFO, one lattice per launch).  With FP16 storage the residual
    floor (about 4e-4) lies above 1e-8, so every request runs to the cap;
    `precision` and `tol` give the variant whose requests retire on their
    residual (FP32-shifted storage, floor about 2e-7, tolerance 1e-6).
    `steps_per_pass` 2 serves with two time steps per launch; `modes` picks
    the servers run."""
    from paper_2409_02964_amd import workloads as W
    from paper_2409_02964_amd.serve import SolveServer, summarize
    reqs = W.served_requests(count, rate, seed=5)
    budget = int(budget_gib * (1 << 30))
    names = {"f16s": "FP16 shifted", "f32s": "FP32 shifted", "f32": "FP32", "f64": "FP64"}
    out = {"workload": f"{count} requests, Poisson {rate}/s, L log-uniform 64..2048, inclusions, "
                       f"{names[precision]} storage, residual {tol:g} or 20000 steps",
           "memory_budget_gib": budget_gib}
    for name, kw in (("continuous_batching", {}), ("one_at_a_time", {"max_active": 1})):
        if name not in modes:
            continue
        srv = SolveServer(budget, precision=precision, chunk=500, max_steps=20000, tol=tol,
                          steps_per_pass=steps_per_pass, **kw)
        t0 = time.perf_counter()
        done = srv.run(reqs)
        out[name] = summarize(done, time.perf_counter() - t0)
        out[name]["max_active"] = max(a for _, a, _, _ in srv.log)
        out[name]["steps_per_launch"] = srv.steps_per_pass
    return out


def precision_ladder(n: int, steps: int, out_md: str = None, quiet: bool = False):
    """Precision ladder on an n x n channel (the benchmark channel's
    generator: walls, tanh phi step + noise, seed 2409, G = 1e-7): the FP64
    oracle against the GPU in FP64, FP32, FP32-shifted and FP16-shifted
    storage after `steps` steps; writes a short report to `out_md` (if
    given) and returns the rows.  quiet: no progress lines."""
    import math
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_2409_02964_amd import workloads as W
    from paper_2409_02964_amd.vanse import Lattice

    def rel(a, b):
        return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))

    phi = W.channel_phi(n, n, seed=2409)
    o = O.Oracle(n, n, phi, kappa=KAPPA, rates=RATES, g=(G, 0.0), bc_y="wall").init_equilibrium()
    t0 = time.perf_counter()
    chunk = max(1, steps // 20)
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        o.step(k)
        done += k
        if not quiet:
            print(f"oracle {n}x{n}: {done}/{steps} steps, {time.perf_counter() - t0:.0f} s", flush=True)
    t_oracle = time.perf_counter() - t0
    ref = o.macroscopic()
    rows = []
    for prec, spp in (("f64", 1), ("f32", 1), ("f32s", 1), ("f16s", 1), ("f64", 2), ("f32", 2),
                      ("f32s", 2), ("f16s", 2)):
        lat = Lattice(n, n, precision=prec, bc_y="wall")
        lat.set_params(KAPPA, RATES).set_body_force(G, 0.0).set_void_fraction(phi)
        if spp == 2:
            lat.set_steps_per_pass(2)
        lat.init_equilibrium(1.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        m = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
        eu = math.sqrt(float(np.sum((m["ux"] - ref["ux"]) ** 2 + (m["uy"] - ref["uy"]) ** 2))
                       / float(np.sum(ref["ux"] ** 2 + ref["uy"] ** 2)))
        rows.append((prec, spp, BYTES_PER_NODE[prec], eu, rel(m["p"], ref["p"]),
                     rel(m["p"] - m["p"].mean(), ref["p"] - ref["p"].mean()),
                     n * n * steps / dt / 1e6))
        if not quiet:
            print(f"{prec}, {spp} step(s) per launch: rel-L2 u {eu:.3e}", flush=True)
        lat.close()
    if out_md is None:
        return rows, t_oracle
    threads = os.environ.get("OMP_NUM_THREADS", str(os.cpu_count()))
    lines = [f"# Precision ladder: {n}x{n} channel, {steps} steps", "",
             "Command (from the repository root):", "", "```",
             f"python bench.py --precision-ladder {n} --ladder-steps {steps}", "```", "",
             f"Workload: walls in y, G = {G} (F^B = phi G), phi = tanh step 0.4 -> 1.0 + smoothed "
             f"noise 0.05 (seed 2409), kappa = {KAPPA}, s_nu = 0.8, other rates 1.2, rho0 = 1, "
             "from rest.  Reference: the FP64 CPU oracle "
             f"({t_oracle:.0f} s on {threads} OpenMP threads).", "",
             "| storage | steps/launch | bytes/node | rel-L2(u) | rel-L2(p) | rel-L2(p - <p>) | MLUPS |",
             "|---|---|---|---|---|---|---|"]
    for prec, spp, b, eu, ep, epd, ml in rows:
        lines.append(f"| {prec} | {spp} | {b} | {eu:.3e} | {ep:.3e} | {epd:.3e} | {ml:.0f} |")
    lines += ["", "f64: FP64 arithmetic and storage; f32: FP32 arithmetic and storage of f; "
              "f32s: FP32 arithmetic, FP32 storage of the deviations from the rest state; "
              "f16s: FP32 arithmetic, FP16 storage of the deviations scaled by 2^12.  Two steps "
              "per launch keep the intermediate state in LDS in the arithmetic type (one "
              "storage rounding per two steps).  The MLUPS column is a single wall-clock run "
              "of this size (the populations of the smaller formats fit in the 256 MB "
              "last-level cache)."]
    open(out_md, "w").write("\n".join(lines) + "\n")
    return rows, t_oracle


def summarize_profile(prof_dir: str, prefix: str, commands: str) -> None:
    """Turn rocprofv3 CSV output (a kernel-trace --stats run in prof_dir/trace,
    --pmc FETCH_SIZE in prof_dir/fetch, --pmc WRITE_SIZE in prof_dir/write,
    optionally request counts by size in prof_dir/ea_rd and prof_dir/ea_wr and
    SQ instruction counters in prof_dir/sq) into a short text summary and the
    traffic record this benchmark reports.

    The counters are scaled by what they read for the same-pattern copy
    kernel, whose bytes are known exactly (9 planes read, 9 written)."""
    import csv
    import glob
    from collections import defaultdict

    def one(pattern):
        hits = glob.glob(os.path.join(prof_dir, pattern), recursive=True)
        if not hits:
            raise SystemExit(f"no {pattern} under {prof_dir}")
        return hits[0]

    stats = list(csv.DictReader(open(one("trace/**/*kernel_stats.csv"))))
    counters = {}
    for kind, name in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        per = defaultdict(list)
        for r in csv.DictReader(open(one(f"{kind}/**/*counter_collection.csv"))):
            if r["Counter_Name"] == name:
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        counters[name] = {k: sum(v) / len(v) for k, v in per.items()}

    def pick(d, key):
        ks = [k for k in d if key in k]
        if not ks:
            raise SystemExit(f"kernel {key} not in profile")
        return d[ks[0]]

    nodes = NX * NY
    copy_bytes = 9 * 4 * nodes  # per direction, FP32
    f_copy = pick(counters["FETCH_SIZE"], "stream_copy") * 1024
    w_copy = pick(counters["WRITE_SIZE"], "stream_copy") * 1024
    f_scale, w_scale = copy_bytes / f_copy, copy_bytes / w_copy
    kname = "vanse_step2_kernel" if STEPS_PER_PASS == 2 else "vanse_step_kernel"
    f_step = pick(counters["FETCH_SIZE"], kname) * 1024 * f_scale
    w_step = pick(counters["WRITE_SIZE"], kname) * 1024 * w_scale
    alg = BYTES_PER_NODE[PRECISION] * nodes * STEPS_PER_PASS
    step_ns = float(pick({r["Name"]: r["AverageNs"] for r in stats}, kname))
    copy_ns = float(pick({r["Name"]: r["AverageNs"] for r in stats}, "stream_copy"))
    rec = {"kernel_hash": kernel_hash(), "bytes_per_launch": int(f_step + w_step),
           "fetch_bytes": int(f_step), "write_bytes": int(w_step),
           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
           "algorithmic_bytes": alg, "steps_per_launch": STEPS_PER_PASS, "kernel": kname,
           "step_avg_ns": step_ns, "copy_avg_ns": copy_ns}
    lines = [f"# rocprofv3: {kname} ({STEPS_PER_PASS} time steps per launch), {NX}x{NY} "
             f"{PRECISION} channel (walls)", "",
             "Commands (from the repository root; outputs under gpurun_out/prof):", "",
             "```", commands.strip(), "```", "",
             "## Kernel statistics (--kernel-trace --stats)", "",
             "| kernel | calls | average ns | min ns | max ns |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:8]:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                     f"{r['MinNs']} | {r['MaxNs']} |")
    lines += ["", "## HBM traffic per dispatch (--pmc FETCH_SIZE, then --pmc WRITE_SIZE)", "",
              "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|"]
    for k in sorted(counters["FETCH_SIZE"]):
        if "step_kernel" in k or "step2_kernel" in k or "stream_copy" in k:
            lines.append(f"| {k[:90]} | {counters['FETCH_SIZE'][k]:.0f} | "
                         f"{counters['WRITE_SIZE'].get(k, float('nan')):.0f} |")
    comp = BYTES_PER_NODE[PRECISION] * nodes
    lines += ["", f"Calibration with the same-pattern copy ({copy_bytes} B read and written per "
              f"dispatch): FETCH x {f_scale:.4f}, WRITE x {w_scale:.4f}.", "",
              f"Step kernel ({STEPS_PER_PASS} node updates per node per launch): "
              f"{f_step / 1e6:.1f} MB read + {w_step / 1e6:.1f} MB written = "
              f"{(f_step + w_step) / 1e6:.1f} MB per launch; the launch must move {comp / 1e6:.1f} MB "
              f"(each population read and written once, phi read once: "
              f"{(f_step + w_step) / comp:.3f}x); the node updates' algorithmic bytes are "
              f"{alg / 1e6:.1f} MB.  Average duration {step_ns / 1e3:.1f} us -> "
              f"{comp / step_ns:.0f} GB/s of required bytes ({comp / step_ns / HBM_PEAK_GBS:.3f} of "
              f"the peak), {(f_step + w_step) / step_ns:.0f} GB/s measured, "
              f"{alg / step_ns:.0f} GB/s over both updates; copy {copy_bytes * 2 / copy_ns:.0f} GB/s."]

    def pmc(kind):
        per = defaultdict(lambda: defaultdict(list))
        hits = glob.glob(os.path.join(prof_dir, f"{kind}/**/*counter_collection.csv"), recursive=True)
        if not hits:
            return None
        for r in csv.DictReader(open(hits[0])):
            per[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in per.items()}

    # Cross-check of the calibration: HBM read and write requests by size
    ea_rd, ea_wr = pmc("ea_rd"), pmc("ea_wr")
    if ea_rd and ea_wr:
        lines += ["", "## Cross-check: memory requests by size (--pmc TCC_EA0_RDREQ_32B_sum "
                  "TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_sum, then "
                  "TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum)", "",
                  "| kernel | read requests 32/64/128 B (all) | bytes read | write requests "
                  "(64 B) | bytes written | expected |", "|---|---|---|---|---|---|"]
        for key, expect in (("stream_copy", copy_bytes), (kname, None)):
            r = pick(ea_rd, key)
            w = pick(ea_wr, key)
            rd = (32 * r["TCC_EA0_RDREQ_32B_sum"] + 64 * r["TCC_EA0_RDREQ_64B_sum"]
                  + 128 * r["TCC_EA0_RDREQ_128B_sum"])
            # a write request carries 64 B, or 32 B when it is not a 64-byte one
            wb = 64 * w["TCC_EA0_WRREQ_64B_sum"] + 32 * (w["TCC_EA0_WRREQ_sum"] - w["TCC_EA0_WRREQ_64B_sum"])
            rec["ea_read_bytes" if key == kname else "copy_ea_read_bytes"] = int(rd)
            rec["ea_write_bytes" if key == kname else "copy_ea_write_bytes"] = int(wb)
            lines.append(f"| {key} | {r['TCC_EA0_RDREQ_32B_sum']:.0f} / {r['TCC_EA0_RDREQ_64B_sum']:.0f}"
                         f" / {r['TCC_EA0_RDREQ_128B_sum']:.0f} ({r['TCC_EA0_RDREQ_sum']:.0f}) | "
                         f"{rd / 1e6:.1f} MB | {w['TCC_EA0_WRREQ_sum']:.0f} "
                         f"({w['TCC_EA0_WRREQ_64B_sum']:.0f}) | {wb / 1e6:.1f} MB | "
                         + (f"{expect / 1e6:.1f} MB each way |" if expect else "— |"))
        rd_scale = copy_bytes / rec["copy_ea_read_bytes"]
        lines += ["", f"Step kernel by request sizes: {rec['ea_read_bytes'] / 1e6:.1f} MB read + "
                  f"{rec['ea_write_bytes'] / 1e6:.1f} MB written = "
                  f"{(rec['ea_read_bytes'] + rec['ea_write_bytes']) / 1e6:.1f} MB.  The copy's reads "
                  f"count x {1 / rd_scale:.3f} of its bytes by request size; scaled the same way "
                  f"the step kernel reads {rec['ea_read_bytes'] * rd_scale / 1e6:.1f} MB, against "
                  f"{f_step / 1e6:.1f} MB from the calibrated FETCH_SIZE (writes: "
                  f"{rec['ea_write_bytes'] / 1e6:.1f} against {w_step / 1e6:.1f} MB)."]
    # Instruction mix and wave states
    sq = pmc("sq")
    if sq:
        q = pick(sq, kname)
        waves = q.get("SQ_WAVES", float("nan"))
        lines += ["", "## Instruction mix of the step kernel (--pmc " + " ".join(sorted(q)) + ")", "",
                  "| counter | per dispatch | per wave |", "|---|---|---|"]
        for c in sorted(q):
            lines.append(f"| {c} | {q[c]:.4g} | {q[c] / waves:.4g} |")
        rec["sq"] = {c: q[c] for c in sorted(q)}
    json.dump(rec, open(prefix + "_traffic.json", "w"), indent=1)
    open(prefix + "_rocprof.md", "w").write("\n".join(lines) + "\n")
    print(json.dumps(rec))


def summarize_variants(prof_dir: str, out_md: str) -> None:
    """profiles/ summary of a `rocprofv3 --kernel-trace --stats` run of
    `bench.py --variants`: the step kernels' statistics from prof_dir's
    kernel_stats CSV and the HIP-event timings the run printed (prof_dir/
    variants.log)."""
    import csv
    import glob
    hits = glob.glob(os.path.join(prof_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not hits:
        raise SystemExit(f"no kernel_stats.csv under {prof_dir}")
    stats = [r for r in csv.DictReader(open(hits[0])) if "step" in r["Name"] and "kernel" in r["Name"]]
    recs = []
    for ln in open(os.path.join(prof_dir, "variants.log")):
        if ln.startswith("{"):
            recs.append(json.loads(ln))
    cmd = open(os.path.join(prof_dir, "commands.txt")).read().strip()
    lines = ["# rocprofv3: every step-kernel variant, 4096x4096 channel (walls)", "",
             "Command (from the repository root; outputs under gpurun_out/prof_var):", "",
             "```", cmd, "```", "",
             "The benchmark channel's field, forcing and rates, with: a cylinder-and-grain solid "
             "mask (`solid_mask`, seed 5), a force field 1e-7 N(0,1) smoothed over 8 cells, a drag "
             "beta = 1e-3 + 1e-2 (1 - phi), a moving phi without phi(t+1) (d_t phi = 0), model B, "
             "an upper wall at u = 1e-3, and an upper velocity row at u = 1e-3.  Per variant: 4 "
             "untimed steps, half a second of untimed stepping (the shader clock rises under "
             "load), then the timed steps.", "",
             "## Kernel statistics (--kernel-trace --stats)", "",
             "| kernel | calls | average µs | min µs | max µs |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: float(r["AverageNs"])):
        lines.append(f"| {r['Name'][:110]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    lines += ["", "## The same runs timed with HIP events (bench.py --variants)", "",
              "| variant | storage | steps/launch | µs per step | GLUPS |", "|---|---|---|---|---|"]
    for r in recs:
        lines.append(f"| {r['variant']} | {r['storage']} | {r['steps_per_launch']} | "
                     f"{r['us_per_step']} | {r['glups']} |")
    lines += ["", "Calls include the untimed settling steps; the kernel trace adds a little to "
              "each launch."]
    open(out_md, "w").write("\n".join(lines) + "\n")


# Kernel variants timed by --variants: (name, storage, steps per launch, options)
VARIANTS = [
    ("plain", "f32s", 1, {}),
    ("plain", "f32s", 2, {}),
    ("plain", "f16s", 1, {}),
    ("plain", "f16s", 2, {}),
    ("plain", "f64", 1, {}),
    ("plain", "f64", 2, {}),
    ("force field", "f32s", 1, {"force": True}),
    ("force field", "f32s", 2, {"force": True}),
    ("drag", "f32s", 2, {"drag": True}),
    ("moving phi, force field, drag", "f32s", 1, {"dynamic": True, "force": True, "drag": True}),
    ("moving phi, drag", "f32s", 2, {"dynamic": True, "drag": True}),
    ("moving phi, force field, drag", "f32s", 2, {"dynamic": True, "force": True, "drag": True}),
    ("solid nodes", "f32s", 1, {"mask": True}),
    ("solid nodes", "f32s", 2, {"mask": True}),
    ("solid nodes", "f64", 1, {"mask": True}),
    ("solid nodes", "f64", 2, {"mask": True}),
    ("a solid disc of radius 256", "f32s", 1, {"mask": "disc"}),
    ("a solid disc of radius 256", "f32s", 2, {"mask": "disc"}),
    ("a solid disc of radius 256, drag", "f32s", 2, {"mask": "disc", "drag": True}),
    ("solid nodes, force field, drag", "f32s", 1, {"mask": True, "force": True, "drag": True}),
    ("solid nodes, force field, drag", "f32s", 2, {"mask": True, "force": True, "drag": True}),
    ("solid nodes, moving phi", "f32s", 1, {"mask": True, "dynamic": True}),
    ("walls in x (a closed box)", "f32s", 1, {"xwalls": True}),
    ("model B", "f32s", 1, {"model_b": True}),
    ("model B", "f32s", 2, {"model_b": True}),
    ("model B, drag", "f32s", 2, {"model_b": True, "drag": True}),
    ("Appendix B equilibrium", "f32s", 1, {"eq2": True}),
    ("Appendix B equilibrium", "f32s", 2, {"eq2": True}),
    ("moving walls, drag", "f32s", 1, {"wall_u": 1e-3, "drag": True}),
    ("model B, solid nodes", "f32s", 1, {"model_b": True, "mask": True}),
    ("model B, solid nodes", "f32s", 2, {"model_b": True, "mask": True}),
    ("Appendix B equilibrium, solid nodes", "f32s", 2, {"eq2": True, "mask": True}),
    ("velocity rows (Couette), drag", "f32s", 1, {"vel_rows": 1e-3, "drag": True}),
]


def variants_bench(steps: int, settle_s: float = 0.5):
    """Every kernel variant on the 4096 x 4096 benchmark channel: `steps`
    steps each (after 4 untimed, and untimed stepping for `settle_s` seconds
    so that the shader clock has risen), timed with HIP events on the launch
    stream; prints one JSON line per variant and a markdown table."""
    import numpy as np
    import torch
    from paper_2409_02964_amd import workloads as W
    from paper_2409_02964_amd.vanse import Lattice
    phi = W.channel_phi(NX, NY, seed=2409)
    masks = {True: W.solid_mask(NX, NY, seed=5), "disc": W.cylinder_channel(NX, NY, radius=256.0)}
    fx = 1e-7 * W.smoothed_noise(NX, NY, 8.0, seed=1)
    beta = 1e-3 + 1e-2 * (1 - phi)
    rows = []
    for name, prec, spp, o in VARIANTS:
        lat = Lattice(NX, NY, precision=prec, bc_y="wall", mask=bool(o.get("mask", False)),
                      bc_x="wall" if o.get("xwalls") else "periodic",
                      dynamic_phi=o.get("dynamic", False), force_field=o.get("force", False),
                      drag=o.get("drag", False))
        lat.set_params(KAPPA, RATES).set_body_force(G, 0.0, True)
        if o.get("mask"):
            lat.set_mask(masks[o["mask"]])
        if o.get("model_b"):
            lat.set_scheme("B", 3)
        if o.get("eq2"):
            lat.set_scheme("A", 2)
        if o.get("wall_u"):
            lat.set_wall_velocity(0.0, o["wall_u"])
        if o.get("vel_rows"):
            lat.set_velocity_rows(None, o["vel_rows"])
        lat.set_void_fraction(phi)
        if o.get("force"):
            lat.set_force_field(fx, np.zeros_like(fx))
        if o.get("drag"):
            lat.set_drag(beta)
        lat.set_steps_per_pass(spp).init_equilibrium(1.0)
        stream = torch.cuda.current_stream()
        lat.step(4, stream)
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        while time.perf_counter() - t_s < settle_s:
            lat.step(10, stream)
            torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(steps, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / steps * 1e3
        rec = {"variant": name, "storage": prec, "steps_per_launch": spp,
               "us_per_step": round(us, 1), "glups": round(NX * NY / us / 1e3, 1)}
        print(json.dumps(rec), flush=True)
        rows.append(rec)
        lat.close()
    print("| variant | storage | steps/launch | µs per step | GLUPS |")
    print("|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['variant']} | {r['storage']} | {r['steps_per_launch']} | {r['us_per_step']} | {r['glups']} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of --steps steps each; the median is reported")
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed stepping after the warmup, for the GPU clock to rise")
    ap.add_argument("--precision", default=PRECISION, choices=sorted(BYTES_PER_NODE))
    ap.add_argument("--threads", type=int, default=TILING[0])
    ap.add_argument("--rows", type=int, default=TILING[1])
    ap.add_argument("--steps-per-pass", type=int, default=STEPS_PER_PASS, choices=(1, 2),
                    help="time steps per launch of the plain step (2: the two-step kernel)")
    ap.add_argument("--fused-rows", type=int, default=0,
                    help="rows per workgroup of the two-step kernel (0: one full round)")
    ap.add_argument("--sol-steps", type=int, default=200,
                    help="launches of the same-pattern copy kernel (0: skip)")
    ap.add_argument("--cpu-steps", type=int, default=100,
                    help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=2000,
                    help="steps of the batched 256-lattice workload (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests of the served workload (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-sweep", default="",
                    help="further arrival rates (comma list) of the served workload")
    ap.add_argument("--small-steps", type=int, default=1000,
                    help="steps of the 64x64 FP64 workload, plain and graph-captured (0: skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=2.0)
    ap.add_argument("--summarize-variants", metavar="DIR",
                    help="summarize a rocprofv3 kernel trace of --variants in DIR into profiles/")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="summarize rocprofv3 CSVs in DIR/{trace,fetch,write} into profiles/")
    ap.add_argument("--precision-ladder", type=int, metavar="N", default=0,
                    help="run the precision ladder on an N x N channel and write profiles/")
    ap.add_argument("--ladder-steps", type=int, default=5000)
    ap.add_argument("--ladder-n", type=int, default=1024,
                    help="side of the precision ladder in the benchmark line (0: skip)")
    ap.add_argument("--bench-ladder-steps", type=int, default=2000,
                    help="steps of the precision ladder in the benchmark line")
    ap.add_argument("--variants", type=int, metavar="STEPS", default=0,
                    help="time every kernel variant on the benchmark channel (STEPS steps each)")
    args = ap.parse_args()
    if args.variants:
        variants_bench(args.variants)
        return
    if args.summarize_variants:
        summarize_variants(args.summarize_variants,
                           os.path.join(ROOT, "profiles", "variants_channel4096_rocprof.md"))
        return
    if args.precision_ladder:
        n = args.precision_ladder
        precision_ladder(n, args.ladder_steps,
                         os.path.join(ROOT, "profiles", f"precision_ladder_channel{n}.md"))
        return
    if args.summarize_profile:
        cmds = open(os.path.join(args.summarize_profile, "commands.txt")).read()
        summarize_profile(args.summarize_profile, PROFILE_PREFIX, cmds)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_02964_amd import workloads as W
    from paper_2409_02964_amd.vanse import Lattice

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    phi = W.channel_phi(NX, NY, seed=2409)
    lat = Lattice(NX, NY, precision=args.precision, bc_y="wall", device=dev)
    lat.set_params(KAPPA, RATES).set_body_force(G, 0.0, True)
    lat.set_void_fraction(phi)
    lat.set_tiling(args.threads, args.rows)
    spp = args.steps_per_pass
    lat.set_steps_per_pass(spp, args.fused_rows)
    lat.init_equilibrium(1.0)
    stream = torch.cuda.current_stream(dev)

    gpu_clock_before = gpu_clocks()  # idle, before the warmup
    lat.step(args.warmup, stream)
    torch.cuda.synchronize(dev)
    # The GPU idles at a low shader clock and raises it under sustained load
    # (rocm-smi showed 1.2 GHz before and 1.7 GHz after a few milliseconds of
    # stepping): keep stepping, untimed, until the load has lasted
    # --settle-s seconds, so that short timed windows see the clock that a
    # long run does.
    t_settle = time.perf_counter()
    settle_steps = 0
    while time.perf_counter() - t_settle < args.settle_s:
        lat.step(20, stream)
        torch.cuda.synchronize(dev)
        settle_steps += 20
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # `windows` timed windows of exactly K steps each, back to back on the
    # same lattice; the line reports the median window (the spread is kept)
    window_ms = []
    t0 = time.perf_counter()
    for _ in range(max(1, args.windows)):
        torch.cuda.synchronize(dev)
        ev0.record(stream)
        lat.step(args.steps, stream)
        ev1.record(stream)
        torch.cuda.synchronize(dev)
        window_ms.append(ev0.elapsed_time(ev1))
    wall = time.perf_counter() - t0
    gpu_clock_after = gpu_clocks()
    gpu_ms = sorted(window_ms)[len(window_ms) // 2]
    obs = lat.observe(stream, raise_on_diverged=False)

    # speed-of-light reference: the step's memory pattern without arithmetic
    sol = None
    if args.sol_steps > 0:
        lat.stream_copy(10, stream)
        torch.cuda.synchronize(dev)
        ev0.record(stream)
        lat.stream_copy(args.sol_steps, stream)
        ev1.record(stream)
        torch.cuda.synchronize(dev)
        copy_ms = ev0.elapsed_time(ev1) / args.sol_steps
        sol_bytes = (BYTES_PER_NODE[args.precision] - (8 if args.precision == "f64" else 4))
        sol = round(sol_bytes * NX * NY / (copy_ms / 1e3) / 1e9, 1)

    nodes = NX * NY
    sec = gpu_ms / 1e3
    mlups = nodes * args.steps / sec / 1e6
    per_step_ms = gpu_ms / max(args.steps, 1)
    bpn = BYTES_PER_NODE[args.precision]
    ft = lat.fused_tiling()
    per_launch = 2 if ft["active"] else 1
    launch_s = per_step_ms * per_launch / 1e3
    # The HBM bytes a launch must move: every stored population read once
    # and written once, and phi read once -- whether the launch advances the
    # node by one step or by two (the intermediate state stays on chip).
    compulsory = bpn * nodes
    achieved = compulsory / launch_s / 1e9
    # the node updates' algorithmic bytes (76 B per update) over the launch:
    # above the HBM peak when one pass carries two updates
    effective = bpn * nodes * per_launch / launch_s / 1e9
    traffic = (measured_traffic()
               if args.precision == PRECISION and per_launch == STEPS_PER_PASS else None)
    tl = lat.tiling()

    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(per_step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"D2Q9 MRT-VANSE channel {NX}x{NY}, walls in y, G=1e-7, "
                               "phi tanh 0.4->1.0 + smoothed noise 0.05 (seed 2409), kappa=0.5, "
                               "s_nu=0.8, other rates 1.2",
                   "nx": NX, "ny": NY, "storage": args.precision, "steps_per_launch": per_launch,
                   "threads": 512 if per_launch == 2 else tl["threads"],
                   "rows": ft["rows"] if per_launch == 2 else tl["rows"],
                   "workgroups": ft["workgroups"] if per_launch == 2 else tl["workgroups"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "vanse_step2_kernel" if per_launch == 2 else "vanse_step_kernel",
                     "launch_us": round(launch_s * 1e6, 2),
                     "bytes_per_launch": compulsory,
                     "node_updates_per_launch": per_launch * nodes,
                     # the updates' algorithmic bytes over the launch
                     # (76 B per node update, two updates per node)
                     "effective_gbs": round(effective, 1),
                     "effective_frac": round(effective / HBM_PEAK_GBS, 4),
                     # HBM bytes the counters measured for one launch
                     "traffic_gbs": round(traffic / launch_s / 1e9, 1) if traffic else None,
                     "traffic_frac": (round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic else None),
                     "traffic_source": (os.path.relpath(TRAFFIC_FILE, ROOT) if traffic else None),
                     "same_pattern_copy_gbs": sol},
        "windows_ms_per_step": [round(w / max(args.steps, 1), 4) for w in window_ms],
        "settle": {"seconds": args.settle_s, "steps": settle_steps},
        "gpu_state": {"before": gpu_clock_before, "after": gpu_clock_after},
        "wall_s": round(wall, 3),
        "final_umax": obs["umax"],
        "nonfinite": obs["nonfinite"],
    }
    if args.small_steps > 0:
        line["small"] = small_bench(args.small_steps)
    if args.batch_steps > 0:
        line["batched"] = batched_bench(args.batch_steps, max(1, args.batch_steps // 10))
    if args.serve_requests > 0:
        line["served"] = served_bench(args.serve_requests, args.serve_rate, args.serve_budget_gib)
        # requests that retire on their residual take about 4000 steps: at
        # the base rate the GPU idles between arrivals, so this line offers
        # four times as many per second
        line["served_to_residual"] = served_bench(args.serve_requests, 4 * args.serve_rate,
                                                  args.serve_budget_gib, "f32s", 1e-6)
        # the served workload as specified, two time steps per launch: the
        # large requests, which set the p99, gain; the small ones lose
        line["served_two_steps_per_launch"] = served_bench(
            args.serve_requests, args.serve_rate, args.serve_budget_gib, steps_per_pass=2,
            modes=("continuous_batching",))
        extra = [float(r) for r in args.serve_sweep.split(",") if r.strip()] if args.serve_sweep else []
        if extra:
            line["served_sweep"] = {str(r): served_bench(args.serve_requests, r, args.serve_budget_gib)
                                    for r in extra}
    if args.ladder_n > 0:
        # the precision ladder of the 2048^2, 5000-step channel workload at a
        # quarter of its nodes and 2000 steps, so that the oracle's reference
        # run takes about half a minute (the full size: --precision-ladder 2048)
        from oracle import oracle as O
        O.set_threads(max(1, min(16, len(os.sched_getaffinity(0)))))
        rows, t_or = precision_ladder(args.ladder_n, args.bench_ladder_steps, quiet=True)
        line["precision_ladder"] = {
            "workload": f"channel {args.ladder_n}x{args.ladder_n} (the benchmark channel's "
                        f"generator), {args.bench_ladder_steps} steps from rest, against the FP64 oracle "
                        f"({t_or:.0f} s)",
            "rows": [{"storage": p, "steps_per_launch": spp, "bytes_per_node": b,
                      "rel_l2_u": float(f"{eu:.3e}"), "rel_l2_p": float(f"{ep:.3e}"),
                      "rel_l2_p_minus_mean": float(f"{epd:.3e}")}
                     for p, spp, b, eu, ep, epd, _ in rows]}
    if args.cpu_steps > 0:
        line["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
