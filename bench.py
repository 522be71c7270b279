"""Benchmark: the explicit RD step on one MI355X.

Default workload: the moving-front precipitation problem on a 384x384x512
grid (3 species, FP32 fields, dt = 0.005), the largest configuration: one step
= A + B -> C with the Cahn-Hilliard term M Lap(mu), mu = C^3 - C - kappa
Lap(C), in one fused pass (the chemical potential computed in LDS) over 75.5 M
cells x 3 species.  Prints ONE JSON line with Gcell-updates/s, the step
kernel's HBM-roofline fraction (timed with HIP events on the stream the
kernel runs on) and the FP64 CPU oracle timed on a bounded sample of the same
workload, on the host's cores and on one thread.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic HBM bytes per cell-update: one read and one write of every
# stored species (FP32 fields: 4 B each way).  The front model's two-pass
# form additionally writes and reads the FP32 chemical potential (8 B/cell)
# and reads C twice; its one-pass form moves the plain bytes.
def alg_bytes_per_cell(name: str, storage: str, one_pass: bool = False) -> int:
    ns = {"brusselator256": 2, "diffusion64": 1, "diffusion512": 1, "front384": 3,
          "pollutant512": 4, "t1_diffusion192": 1, "t1_turing192": 2, "t1_front192": 3,
          "t1_atmos192": 1}[name]
    es = 4 if storage == "f32" else 2
    b = 2 * ns * es
    if name in ("front384", "t1_front192") and not one_pass:
        b += 8 + es          # mu written (4) and read (4) + C read again by pass 1
    return b


def with_stencil(w, stencil: int):
    """The workload on the 19-point Laplacian of Eqs. (3)-(4) when asked:
    every species keeps its x coefficient on all three axes."""
    if stencil == 7:
        return w
    w.spec.stencil = stencil
    w.spec.K = [[k[0]] * 3 for k in w.spec.K]
    w.name = w.name + "_19pt"
    return w


def profile_name(args) -> str:
    return args.workload + ("_19pt" if getattr(args, "stencil", 7) == 19 else "")


def kernel_source_digest() -> str:
    """Digest of the kernel and engine sources (the one compiled into the
    library)."""
    from paper_1004_0480_amd import build
    return build.source_digest()


KERNEL_NAMES = {1: "direct_kernel", 2: "tiled_kernel", 3: "block_kernel", 4: "lds_kernel", 5: "lds2_kernel",
                6: "fch_kernel", 7: "tr_kernel"}


def measured_traffic(name: str, digest: str, kernel: int = 0):
    """The committed rocprofv3 PMC summary of this workload on the kind of
    kernel the plan runs, if it was taken on the current kernel sources;
    else None."""
    path = os.path.join(PROFILES, "%s_%s_pmc.json" % (name, KERNEL_NAMES.get(kernel, "?")))
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != digest:
        return None
    names = rec.get("kernel")
    names = names if isinstance(names, list) else [names]
    if kernel and not all(KERNEL_NAMES.get(kernel, "?") in str(n) for n in names):
        return None
    return rec


def cpu_sample(w, max_cells: int):
    """The workload itself, or its lowest z planes when the grid has more than
    max_cells cells (same physics and boundary rules; the top face of the
    sample takes the grid's top rule).  Returns (workload, description)."""
    from paper_1004_0480_amd import workloads as W
    nz, ny, nx = w.shape
    if w.cells <= max_cells:
        return w, "whole grid"
    kz = max(1, max_cells // (ny * nx))
    spec = w.spec.copy()
    if spec.wind is not None:
        spec.wind = spec.wind[:kz].copy()
    if spec.sources is not None and len(spec.sources[0]):
        keep = spec.sources[0] < kz * ny * nx
        spec.sources = tuple(a[keep] for a in spec.sources)
    sub = W.Workload(w.name, (kz, ny, nx), spec, [f[:kz].copy() for f in w.fields], w.steps, w.seed)
    return sub, "the lowest %d of %d z planes" % (kz, nz)


def cpu_baseline(w, budget_s: float = 12.0, threads: int = 0, max_cells: int = 1 << 27):
    """The FP64 oracle as it stands, on all host cores (or `threads` of them;
    the paper's CPU baseline is one thread), on a bounded sample (the whole
    grid or its lowest planes, a few steps) of the same workload."""
    import oracle
    before = oracle.threads()
    if threads > 0:
        oracle.set_threads(threads)
    try:
        ws, where = cpu_sample(w, max_cells)
        t0 = time.perf_counter()
        oracle.run(ws.spec, ws.fields, 1)
        one = time.perf_counter() - t0
        steps = int(max(1, min(20, budget_s // max(one, 1e-3))))
        t0 = time.perf_counter()
        oracle.run(ws.spec, ws.fields, steps)
        dt = time.perf_counter() - t0
        nthr = oracle.threads()
    finally:
        oracle.set_threads(before)
    return {"value": ws.cells * steps / dt / 1e9, "unit": "Gcell-updates/s",
            "cores": nthr, "kind": "oracle",
            "sample": "%s %dx%dx%d (%s), %d FP64 steps, %s"
                      % (w.name, ws.shape[2], ws.shape[1], ws.shape[0], where, steps,
                         "one thread" if nthr == 1 else "OpenMP over z, %d threads" % nthr)}


COPY_PROBE_BYTES = 2 * 256 * 1024 * 1024    # copy-ceiling probe: bytes read (and written)


def copy_ceiling(torch, stream, nbytes: int, reps: int = 10):
    from paper_1004_0480_amd import rd
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    with torch.cuda.stream(stream):
        rd.copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            rd.copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, stream)
        e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


# ------------------------------------------------ profile summaries (rocprofv3)

STEP_KERNELS = ("rdk::block_kernel", "rdk::tiled_kernel", "rdk::direct_kernel", "rdk::lds_kernel",
                "rdk::lds2_kernel", "rdk::fch_kernel", "rdk::tr_kernel")


def _counter_rows(d: str):
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no *counter_collection.csv under %s" % d)
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter: str, match):
    vals = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter and match(r["Kernel_Name"])]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def _step_kernels(rows):
    """Step kernels of the run: every kernel family that runs once per step
    (the most frequent dispatch count among them)."""
    names = {}
    for r in rows:
        if any(k in r["Kernel_Name"] for k in STEP_KERNELS):
            names[r["Kernel_Name"]] = names.get(r["Kernel_Name"], 0) + 1
    if not names:
        raise SystemExit("no step kernel dispatches in the counter output")
    top = max(names.values())
    return sorted(n for n, c in names.items() if c == top)


def pmc_summary(args):
    """profiles/<workload>_pmc.json from two rocprofv3 --pmc runs of this
    script (FETCH_SIZE, then WRITE_SIZE).  Both counters are read in KiB per
    dispatch and scaled by what they read for the copy kernel of the same run,
    which moves a known number of bytes each way.  A step of several passes
    sums its kernels."""
    from paper_1004_0480_amd import workloads as W
    fetch_rows, write_rows = _counter_rows(args.pmc_summary[0]), _counter_rows(args.pmc_summary[1])
    knames = _step_kernels(fetch_rows)
    is_copy = lambda n: n.startswith("rdk::copy_kernel")
    f_c, _ = _per_dispatch(fetch_rows, "FETCH_SIZE", is_copy)
    w_c, _ = _per_dispatch(write_rows, "WRITE_SIZE", is_copy)
    if None in (f_c, w_c):
        raise SystemExit("missing counter values for the copy kernel")
    copy_bytes = float(COPY_PROBE_BYTES)
    rs, ws = copy_bytes / (f_c * 1024.0), copy_bytes / (w_c * 1024.0)
    per_kernel, rd_b, wr_b = [], 0.0, 0.0
    for k in knames:
        f_k, nf = _per_dispatch(fetch_rows, "FETCH_SIZE", lambda n: n == k)
        w_k, nw = _per_dispatch(write_rows, "WRITE_SIZE", lambda n: n == k)
        if None in (f_k, w_k):
            raise SystemExit("missing counter values for %s" % k)
        per_kernel.append({"kernel": k, "dispatches": {"FETCH_SIZE": nf, "WRITE_SIZE": nw},
                           "fetch_kib_raw": f_k, "write_kib_raw": w_k,
                           "hbm_read_bytes": f_k * 1024.0 * rs, "hbm_write_bytes": w_k * 1024.0 * ws})
        rd_b += f_k * 1024.0 * rs
        wr_b += w_k * 1024.0 * ws
    cells = int(np.prod(W.DEFAULT_SHAPES[args.workload]))
    # one launch set reads and writes every field once: one step, or two for
    # the two-step (temporally blocked) kernel
    spl = 2 if any("rdk::lds2_kernel" in k for k in knames) else 1
    one_pass = any("rdk::fch_kernel" in k for k in knames)
    bpc = alg_bytes_per_cell(args.workload, args.storage, one_pass)
    alg = bpc * cells
    rec = {"kernel": knames[0] if len(knames) == 1 else knames,
           "workload": "%s %s, %s storage, %d-point Laplacian" % (args.workload, W.DEFAULT_SHAPES[args.workload],
                                                                  args.storage, args.stencil),
           "source_digest": kernel_source_digest(), "command": args.pmc_command,
           "per_kernel": per_kernel, "steps_per_launch": spl,
           "calibration": "copy_kernel moving %d bytes each way in the same run" % COPY_PROBE_BYTES,
           "copy_fetch_kib_raw": f_c, "copy_write_kib_raw": w_c, "read_scale": rs, "write_scale": ws,
           "hbm_read_bytes_per_launch_set": rd_b, "hbm_write_bytes_per_launch_set": wr_b,
           "hbm_bytes_per_launch": (rd_b + wr_b) if len(knames) == 1 else None,
           "hbm_bytes_per_step": (rd_b + wr_b) / spl,
           "alg_bytes_per_cell": bpc, "algorithmic_bytes_per_launch_set": alg,
           "traffic_over_algorithmic": (rd_b + wr_b) / alg}
    kind = next((v for v in KERNEL_NAMES.values() if v in knames[0]), "kernel")
    out = os.path.join(PROFILES, "%s_%s_pmc.json" % (profile_name(args), kind))
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def counter_summary(args):
    """profiles/<workload>_<kernel>_counters.md from one rocprofv3 --pmc run
    of this script: every counter of the run per dispatch of the step
    kernel(s), and per wave where the run counted waves (SQ_WAVES)."""
    from paper_1004_0480_amd import workloads as W
    rows = _counter_rows(args.counter_summary)
    knames = _step_kernels(rows)
    counters = sorted({r["Counter_Name"] for r in rows})
    lines = ["# rocprofv3 counters: %s step kernel (MI355X)" % profile_name(args), "",
             "Workload: %s, grid (z, y, x) = %s, %s storage, %d-point Laplacian; kernel sources %s."
             % (args.workload, W.DEFAULT_SHAPES[args.workload], args.storage, args.stencil,
                kernel_source_digest()),
             "", "Command:", "", "```", args.counter_command, "```", ""]
    for k in knames:
        lines += ["Kernel `%s`:" % k[:160], "", "| counter | per dispatch | per wave | dispatches |", "|---|---|---|---|"]
        waves, _ = _per_dispatch(rows, "SQ_WAVES", lambda n: n == k)
        for c in counters:
            v, n = _per_dispatch(rows, c, lambda n: n == k)
            if v is None:
                continue
            lines.append("| %s | %.6g | %s | %d |" % (c, v, "%.4g" % (v / waves) if waves else "-", n))
        lines.append("")
    kind = next((v for v in KERNEL_NAMES.values() if v in knames[0]), "kernel")
    out = os.path.join(PROFILES, "%s_%s_counters.md" % (profile_name(args), kind))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(args):
    """profiles/<workload>_kernel_trace.md from a rocprofv3 --kernel-trace
    --stats run of this script: the per-kernel table and the step kernel's
    bandwidth at its traced average duration."""
    import csv
    import glob
    from paper_1004_0480_amd import workloads as W
    files = glob.glob(os.path.join(args.trace_summary, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no *kernel_stats.csv under %s" % args.trace_summary)
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    cells = int(np.prod(W.DEFAULT_SHAPES[args.workload]))
    one_pass = any("rdk::fch_kernel" in r["Name"] for r in rows)
    bpc = alg_bytes_per_cell(args.workload, args.storage, one_pass)
    lines = ["# rocprofv3 kernel trace: %s step kernel (MI355X)" % profile_name(args), "",
             "Workload: %s, grid (z, y, x) = %s, %s storage, %d-point Laplacian."
             % (args.workload, W.DEFAULT_SHAPES[args.workload], args.storage, args.stencil),
             "", "Command:", "", "```", args.trace_command, "```", "",
             "| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    steps = []
    for r in rows:
        name = r["Name"]
        avg = float(r["AverageNs"]) / 1e3
        lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %.2f%% |" % (
            name[:100], r["Calls"], avg, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
        if any(k in name for k in STEP_KERNELS):
            steps.append((name, avg, int(r["Calls"])))
    lines.append("")
    # the step's kernels: every step-kernel family with the largest call
    # count (the passes of a multi-pass step), their averages summed
    top = max((c for _, _, c in steps), default=0)
    passes = [(n, t) for n, t, c in steps if c == top]
    step = (passes[0][0], sum(t for _, t in passes)) if passes else None
    if step:
        gbs = bpc * cells / (step[1] * 1e-6) / 1e9
        what = "Step kernel `%s`" % step[0][:80] if len(passes) == 1 else \
            "The step's %d passes (`%s` ...)" % (len(passes), step[0][:60])
        lines += ["%s: %d B/cell algorithmic x %d cells = %.1f MB per step; at the traced"
                  % (what, bpc, cells, bpc * cells / 1e6),
                  "average %.2f us per step that is %.0f GB/s, %.1f%% of the 8 TB/s HBM peak."
                  % (step[1], gbs, 100.0 * gbs / HBM_PEAK_GBS)]
    kind = next((v for v in KERNEL_NAMES.values() if step and v in step[0]), "kernel")
    out = os.path.join(PROFILES, "%s_%s_trace.md" % (profile_name(args), kind))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def serve_bench(args):
    """Served batch: 4096 requests (cubes of 32-128, diffusion or Brusselator,
    200-2000 steps).  A saturating run (all requests at t=0) measures the
    capacity; the served run then draws Poisson arrivals at 80% of it."""
    import torch
    from paper_1004_0480_amd import serve as S
    from paper_1004_0480_amd import workloads as W
    trace = W.make_trace(args.requests, seed=4)
    out = {"metric": "Gcell-updates/s (served batch)", "unit": "Gcell-updates/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic", "vs_baseline": None, "modes": {}}
    for storage in (["f32", "bf16"] if args.storage == "both" else [args.storage]):
        res = {}
        for phase in ("capacity", "served"):
            if phase == "capacity":
                arr = [0.0] * len(trace)
            else:
                arr = S.poisson_arrivals(trace, 0.8 * res["capacity"]["requests_per_s"])
            ex = S.GpuExecutor(storage, max_resident=args.max_resident, hbm_budget=args.hbm_budget)
            print("bench: serve %s %s (%d requests)" % (storage, phase, len(trace)),
                  file=sys.stderr, flush=True)
            rep = S.serve(trace, arr, ex, args.max_resident, args.hbm_budget, args.chunk, min_run=args.min_run,
                          depth=args.ticks_in_flight, admit_per_tick=args.admit_per_tick)
            ex.close()
            torch.cuda.synchronize()
            summ = rep.summary()
            summ["requests_per_s"] = len(trace) / rep.makespan
            res[phase] = summ
            print("bench: %s" % json.dumps(summ), file=sys.stderr, flush=True)
        out["modes"][storage] = res
    first = out["modes"][next(iter(out["modes"]))]["served"]
    out.update({"value": first["gcell_updates_per_s"], "p50_latency_s": first["p50_latency_s"],
                "p99_latency_s": first["p99_latency_s"], "dtype": next(iter(out["modes"])),
                "config": {"workload": "served batch", "requests": len(trace),
                           "edges": list(W.SERVE_EDGES), "steps": [200, 2000],
                           "max_resident": args.max_resident, "hbm_budget": args.hbm_budget,
                           "chunk": args.chunk, "min_run": args.min_run, "ticks_in_flight": args.ticks_in_flight,
                           "admit_per_tick": args.admit_per_tick,
                           "arrival_rate": "0.8 x measured capacity"}})
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="front384",
                    choices=["brusselator256", "diffusion512", "front384", "pollutant512", "diffusion64",
                             "t1_diffusion192", "t1_turing192", "t1_front192", "t1_atmos192", "serve"])
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16", "both"])
    ap.add_argument("--rounding", default="nearest", choices=["nearest", "stochastic"],
                    help="rounding of BF16 stores (stochastic needs --storage bf16)")
    ap.add_argument("--integrator", default="euler", choices=["euler", "rk2", "rk3"],
                    help="forward Euler (Eq. (5)) or the SSP Runge-Kutta step of order 2 or 3")
    ap.add_argument("--stencil", type=int, default=7, choices=[7, 19],
                    help="Laplacian: 7-point, or the 19-point form of Eqs. (3)-(4) (x coefficient on every axis)")
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--max-resident", type=int, default=512)
    ap.add_argument("--hbm-budget", type=int, default=16 << 30)
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--admit-per-tick", type=int, default=128,
                    help="served batch: requests admitted between two ticks at most (0: no limit)")
    ap.add_argument("--ticks-in-flight", type=int, default=2,
                    help="served batch: ticks the host keeps queued before it waits for the oldest")
    ap.add_argument("--min-run", type=int, default=1,
                    help="served batch: steps a tick runs at least (finished grids sit out the rest)")
    ap.add_argument("--graph-chunk", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads for the CPU baseline (0 = all host cores; the paper used 1)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--plan", default=None,
                    help="JSON plan (kernel, vx, ry, waves, cz) to use instead of autotuning")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/<workload>_pmc.json from rocprofv3 --pmc outputs")
    ap.add_argument("--pmc-command", default="", help="the profiling command, recorded in the summary")
    ap.add_argument("--trace-summary", metavar="STATS_DIR",
                    help="write profiles/<workload>_kernel_trace.md from rocprofv3 --stats output")
    ap.add_argument("--trace-command", default="", help="the profiling command, recorded in the summary")
    ap.add_argument("--counter-summary", metavar="PMC_DIR",
                    help="write profiles/<workload>_<kernel>_counters.md from a rocprofv3 --pmc run")
    ap.add_argument("--counter-command", default="", help="the profiling command, recorded in the summary")
    args = ap.parse_args()
    if args.pmc_summary:
        return pmc_summary(args)
    if args.counter_summary:
        return counter_summary(args)
    if args.trace_summary:
        return trace_summary(args)
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (there is no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    if args.workload == "serve":
        return serve_bench(args)

    import torch
    from paper_1004_0480_amd import rd
    from paper_1004_0480_amd import workloads as W

    w = with_stencil(W.make_workload(args.workload), args.stencil)
    w.spec.integrator = args.integrator
    stream = torch.cuda.Stream()
    print("bench: %s %s storage=%s stencil=%d steps=%d warmup=%d" % (w.name, w.shape, args.storage, args.stencil,
                                                                     args.steps, args.warmup),
          file=sys.stderr, flush=True)
    g = rd.Grid.from_workload(w, storage=args.storage, stream=stream)
    if args.rounding != "nearest":
        g.set_rounding(args.rounding, 1)
    if args.plan:
        plan = json.loads(args.plan)
    elif args.no_autotune:
        plan = g.plan()
    else:
        plan = g.autotune(40)
    chunk = args.graph_chunk if args.graph_chunk >= 2 else 0
    plan["graph_chunk"] = chunk - (chunk & 1)
    g.set_plan(**plan)
    plan = g.plan()
    print("bench: plan %s" % plan, file=sys.stderr, flush=True)

    g.step(args.warmup)
    g.sync()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    g.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = w.cells * args.steps / (ms * 1e-3) / 1e9

    # sanity: the fields stayed finite
    for s in range(w.spec.ns):
        g.reduce(s)

    passes = g.passes()
    bpc = alg_bytes_per_cell(args.workload, args.storage, one_pass=passes == 1)
    steps_per_launch = 2 if plan.get("kernel") == 5 else 1     # two-step (temporally blocked) plan
    # a Runge-Kutta step runs 2 or 3 Euler stages; every stage after the first
    # also reads the current state once per species (its combination is
    # fused into the store)
    stages = {"euler": 1, "rk2": 2, "rk3": 3}[args.integrator]
    es = 4 if args.storage == "f32" else 2
    rk_bytes = (stages - 1) * w.spec.ns * es
    # dominant kernel: the step kernel.  A launch reads and writes every field
    # once (for one step, or two with a two-step plan); with one pass its
    # average launch duration is the event-timed time of the steps it covers.
    # A step of several passes is reported per step (all its kernels).
    launch_ms = ms_per_step * steps_per_launch
    achieved = bpc * w.cells / (launch_ms * 1e-3) / 1e9
    if stages > 1:      # reported per step over all its kernels
        achieved = (stages * bpc + rk_bytes) * w.cells / (ms_per_step * 1e-3) / 1e9
    digest = kernel_source_digest()
    pmc = measured_traffic(profile_name(args), digest, plan.get("kernel", 0))
    traffic = None
    if pmc is not None and stages == 1 and pmc.get("steps_per_launch", 1) == steps_per_launch:
        traffic = pmc.get("hbm_bytes_per_launch") if passes == 1 else pmc.get("hbm_bytes_per_step")
    ceiling = copy_ceiling(torch, stream, COPY_PROBE_BYTES)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "per": ("step (%d fused Runge-Kutta stages)" % stages if stages > 1
                    else "launch" if passes == 1 else "step (%d kernels)" % passes),
            "steps_per_launch": steps_per_launch,
            "kernel_avg_ms": launch_ms if passes == 1 and stages == 1 else None,
            "alg_bytes_per_cell": stages * bpc + rk_bytes, "copy_ceiling_GBs": ceiling,
            "frac_of_copy_ceiling": achieved / ceiling, "source_digest": digest}
    out = {
        "metric": "Gcell-updates/s", "value": value, "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "storage_dtype": args.storage, "data": "synthetic",
        "config": {"workload": w.name, "grid_xyz": [w.shape[2], w.shape[1], w.shape[0]],
                   "species": w.spec.ns, "storage": args.storage, "stencil": w.spec.stencil,
                   "integrator": args.integrator, "rounding": args.rounding, "dt": w.spec.dt,
                   "plan": plan, "wall_s": wall},
        "roofline": roof,
    }
    g.close()
    if not args.no_cpu_baseline:
        print("bench: CPU oracle, all host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, threads=args.cpu_threads)
        # the paper's CPU baseline ran on one thread: the same oracle on one
        # host thread, on a smaller sample of the same grid
        print("bench: CPU oracle, one thread", file=sys.stderr, flush=True)
        out["cpu_baseline_single_thread"] = cpu_baseline(w, threads=1, max_cells=1 << 23)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
