"""Throughput of the LLG + cavity stepper on one MI355X.

Workload (default): the field sweep -- 64 YIG spheres of diameter 32 cells on
32^3 grids at 5 nm, FFT demag on 64^3 padded grids, one uniform cavity mode,
Dormand-Prince 5(4) at tol 1e-6 -- advanced as one batch.  A step is one
attempted DP45 step of every instance (six stage evaluations, each with its
demag convolution).

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line: cell-updates/s (grid cells x accepted steps / wall
time of the timed region, inputs resident in HBM), the roofline of the
dominant kernel (HIP-event timing of each launch), the batched-vs-plain
speedup, and the oracle timed on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LLG+cavity cell-updates/s and % HBM peak; batched-vs-plain sweep speedup; adjoint/fwd"
HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (packed FP32 instructions included)
FP32_PEAK_TFLOPS = 157.3
# the ceiling of code built without packed FP32 instructions, as these
# kernels are: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
VALU_UNPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# trace sampling of the timed sweep (every instance records a and m^- every
# 10 ps, room for a 100 ns run)
SWEEP_DT_SAMPLE = 10e-12
SWEEP_MAX_SAMPLES = 10001


def yz_flops_per_item(ny, nz, py, pz):
    """Algorithmic flops of one (instance, kx) item of the y-z convolution:
    the radix-2 count 5 P log2 P per line for the forward and inverse y
    transforms of the nz nonzero rows and the forward and inverse z
    transforms of every ky column, three components each, plus 30 flops per
    (ky, kz) point for the symmetric 3x3 kernel times the three components."""
    import math

    def fft(n):
        return 5.0 * n * math.log2(n)
    return 2 * 3 * nz * fft(py) + 2 * 3 * py * fft(pz) + 30.0 * py * pz


def yz_planes(nx):
    """(instance, kx) planes of the y-z convolution in complex-plane units:
    the planes kx = 0 and Px/2 of the x transform of real rows are real, and
    a real plane's transforms count half those of a complex one."""
    return padded(nx) // 2


def padded(n):
    p = 1
    while p < 2 * n:
        p *= 2
    return p


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--plain-instances", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--streams", type=int, default=0,
                    help="run the sweep batch as this many concurrent sub-batches instead of timing 1..3 "
                         "in the tuner (profiler runs use it to keep the plain run's choice)")
    ap.add_argument("--no-afm", action="store_true")
    ap.add_argument("--no-paper-sweep", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=1024)
    ap.add_argument("--afm-steps", type=int, default=20)
    ap.add_argument("--no-film", action="store_true")
    ap.add_argument("--film-steps", type=int, default=100)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for rocprofv3 --pmc: a marker copy, the per-kernel profile phase, a marker copy")
    ap.add_argument("--probe", choices=("sweep", "film", "afm"), default="sweep",
                    help="workload of --pmc-probe and --leg-trace")
    ap.add_argument("--leg-trace", action="store_true",
                    help="for rocprofv3 --kernel-trace: the --probe workload's timed steps and its per-kernel "
                         "profile phase between marker kernels, one JSON line")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("KERNEL_TRACE_CSV", "BENCH_JSON", "COMMAND"),
                    help="write the per-phase kernel time summary of a rocprofv3 --kernel-trace run (markdown)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "PROBE_JSON"),
                    help="write the HBM-traffic summary of two --pmc runs of --pmc-probe (markdown, stdout)")
    ap.add_argument("--command", default=None, help="command line quoted in a summary (--summarize-pmc)")
    return ap.parse_args()


# ----------------------------------------------------------------- HBM traffic
# The roofline's "traffic" entry comes from two rocprofv3 counter runs of
# --pmc-probe (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).  Each counter is
# scaled by what it reads for a plain elementwise copy of known size (the
# marker), and the result is stored with a hash of the kernel sources and the
# FFT tile choice; it is reported only while both still match.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_sweep_64x32cubed_dp45.md")
MARKER_ELEMS = 1 << 26          # float32 elements of the marker copy (256 MiB read + 256 MiB written)


def source_hash():
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2603_03706_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(src, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "paper_2603_03706_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def tile_key(tuning):
    if not tuning:
        return None
    # the per-kernel profile runs the whole batch with the first part's choices
    return [{k: t.get(k) for k in ("grid", "Wx", "x_stage", "path", "Wy", "TW", "TK")}
            for t in tuning if t.get("part", 0) == 0]


def profile_name(kernel):
    """Name used by the library's launch profiler for a demangled kernel name."""
    import re
    k = kernel.split("(")[0].replace("void ", "").strip()
    m = re.match(r"mmk::k_(stage|final)<(\d+), (\d+)>", k)
    if m:
        return f"{m.group(1)}_{'rk4' if m.group(2) == '0' else 'dp45'}_{m.group(3)}" \
            if not (m.group(1) == "stage" and m.group(2) == "0" and m.group(3) == "0") else "stage_rk4_start"
    if k.startswith(("mmk::k_fft_yzr<", "mmk::k_fft_yz8<", "mmk::k_fft_yzx<")):
        return "fft_yz_convolve"
    m = re.match(r"mmk::k_fft_ysx<\d+, (-?\d+)>", k)
    if m:
        return "fft_y_forward" if m.group(1) == "-1" else "fft_y_inverse"
    table = {"mmk::k_fft_yz": "fft_yz_convolve", "mmk::k_fft_zc": "fft_z_convolve",
             "mmk::k_fft_y<-1>": "fft_y_forward", "mmk::k_fft_y<1>": "fft_y_inverse"}
    if k in table:
        return table[k]
    if k.startswith("mmk::k_fft_xf"):
        return "fft_x_forward"
    if k.startswith("mmk::k_fft_xi"):
        return "fft_x_inverse"
    return None


WORKLOADS = {
    "sweep": "field sweep, 64 x 32^3 spheres, FFT demag on 64^3, DP45 tol 1e-6",
    "film": "multimode film, 128 x 128 x 32 cells at 5 nm, FFT demag on 256 x 256 x 64, 4 profiled modes, "
            "DP45 tol 1e-6",
    "afm": "AFM batch, 32 instances of 64^2 x 16 .. 256^2 x 16 at 2 nm, 2 sublattices, no demag, DP45 tol 1e-6",
}


def leg_batch(name, tol, instances=64):
    """Contexts and batch of one benchmark workload (see WORKLOADS)."""
    from paper_2603_03706_amd import mmcav, workloads as W
    if name == "sweep":
        return build_batch(instances, tol)
    insts = [W.multimode_film()] if name == "film" else [W.afm_instance(k) for k in range(32)]
    ctxs = [mmcav.Context.from_instance(i) for i in insts]
    return insts, ctxs, mmcav.Batch(ctxs)


def leg_trace(args):
    """The --probe workload for a kernel trace: tuned batch, warm-up, the
    timed steps between two marker kernels, then the per-kernel profile
    phase between two more; one JSON line with the bench fields the trace
    summary quotes."""
    import torch
    insts, ctxs, batch = leg_batch(args.probe, args.tol, args.instances)
    tuning = batch.tune()
    cells = sum(i.cells * i.sublattices for i in insts)
    dt, acc = timed_steps(batch, ctxs, args.steps, args.tol, args.warmup, marks=True)
    mark()
    prof = batch.profile(args.profile_steps, args.tol)
    mark()
    kernels = []
    for p in prof:
        avg_ms = p["total_ms"] / max(1, p["launches"])
        kernels.append({"name": p["name"], "launches": p["launches"], "avg_us": avg_ms * 1e3,
                        "bytes_per_launch": p["bytes_per_launch"],
                        "GBps": p["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0})
    kernels.sort(key=lambda k: -k["avg_us"] * k["launches"])
    print(json.dumps({"probe": args.probe, "steps": args.steps, "ms_per_step": dt / args.steps * 1e3,
                      "value": cells / len(insts) * acc / dt, "unit": "cell-updates/s",
                      "config": {"streams": batch.streams(), "fft_tiles": tile_key(tuning)}, "kernels": kernels}))


def stream_copy(gib=1.0, reps=20):
    """Achievable HBM bandwidth: an elementwise float32 copy of `gib` GiB
    (read + write counted), the median of `reps` timed copies."""
    import torch
    n = int(gib * (1 << 30) / 4)
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    times.sort()
    t = times[len(times) // 2]
    return {"bytes": 8 * n, "seconds": t, "GBps": 8 * n / t / 1e9}


def mark():
    """A tiny elementwise kernel between two synchronisations: marks phase
    boundaries (timed steps, per-kernel profile) in a kernel trace."""
    import torch
    torch.cuda.synchronize()
    torch.mul(torch.ones(1024, device="cuda"), 2.0)
    torch.cuda.synchronize()


def summarize_trace(trace_csv, bench_json, command):
    """Per-kernel durations of a rocprofv3 kernel trace of the benchmark,
    split by the phase markers: the timed steps and the profile phase (whose
    averages are the ones the JSON line's kernels and roofline use)."""
    import csv
    rows = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    marks = [i for i, r in enumerate(rows) if "MulFunctor" in r[2]]
    if len(marks) < 4:
        raise SystemExit(f"{trace_csv}: expected four phase markers, found {len(marks)}")
    with open(bench_json) as f:
        out = json.loads(f.read().strip().splitlines()[-1])
    bench_us = {k["name"]: k["avg_us"] for k in out.get("kernels", [])}

    def table(lo, hi, with_bench):
        per = {}
        for s0, s1, k in rows[lo + 1:hi]:
            per.setdefault(k.split("(")[0], []).append((s1 - s0) / 1e3)
        tot = sum(sum(v) for v in per.values())
        extra = " avg us in the JSON line |" if with_bench else ""
        print("| kernel | calls | avg us | total ms | % of phase kernel time |" + extra)
        print("|---|---|---|---|---|" + ("---|" if with_bench else ""))
        for k in sorted(per, key=lambda k: -sum(per[k])):
            v = per[k]
            b = bench_us.get(profile_name(k) or "", None)
            col = (f" {'' if b is None else f'{b:.1f}'} |") if with_bench else ""
            print(f"| `{k}` | {len(v)} | {sum(v) / len(v):.1f} | {sum(v) / 1e3:.3f} | {100 * sum(v) / tot:.1f} |" + col)
        span = (rows[hi][0] - rows[lo][1]) / 1e3
        print(f"\nPhase wall time between the markers: {span / 1e3:.2f} ms; summed kernel time {tot / 1e3:.2f} ms.\n")

    print(f"# Kernel time: {WORKLOADS[out.get('probe', 'sweep')]}\n")
    print("Command (from the repository root, one MI355X):\n")
    print("```\n" + command + "\n```\n")
    print(f"Bench line of this run: {out['ms_per_step']:.4f} ms per step, value {out['value']:.4g} "
          f"{out['unit']}, {out['config'].get('streams')} concurrent sub-batches, FFT tiles "
          f"{json.dumps(out['config'].get('fft_tiles'))}.\n")
    print(f"## Timed steps ({out['steps']} DP45 steps of the batch, graphs on the sub-batch streams)\n")
    print("Kernels of different sub-batches overlap here, so a kernel's duration includes the "
          "time it shares the device.\n")
    table(marks[0], marks[1], False)
    print(f"## Per-kernel profile phase (whole batch, eager launches, one kernel at a time)\n")
    print("The JSON line's kernel table and roofline are measured in this phase with HIP events on the "
          "library stream; the last column repeats them. The event pair around a launch adds a few "
          "microseconds of dispatch overhead to each figure, so the JSON line's durations are the "
          "larger ones and its achieved rates the smaller ones.\n")
    table(marks[2], marks[3], True)


def pmc_probe(args):
    """Between two marker copies: the per-kernel profile phase of the
    benchmark (the whole batch, eager launches).  The FFT strategy is fixed
    to the one the tuner picks on this workload (two-pass exchange y-z kernel, x
    passes in the stage kernels) rather than timed again, since counter
    collection distorts the tuner's timings."""
    import torch
    insts, ctxs, batch = leg_batch(args.probe, args.tol, args.instances)
    if args.probe == "sweep":
        batch.set_fft_path("xch")
        batch.set_fft_x("stage")
        nx = insts[0].grid[0]
        tuning = [{"grid": list(insts[0].grid), "Wx": max(1, min(16, 1024 // padded(nx))), "x_stage": True,
                   "path": "xch", "Wy": None, "TW": None, "TK": None}]
    else:
        # the film's and the AFM batch's choices are timed here too (their
        # summaries are for reading, not for the JSON line's traffic)
        tuning = tile_key(batch.tune(streams=False))
        tuning = tuning if tuning else None
    batch.step(3, args.tol)
    src = torch.ones(MARKER_ELEMS, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    batch.profile(args.profile_steps, args.tol)
    torch.cuda.synchronize()
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"probe": args.probe, "tiles": tile_key(tuning) if args.probe == "sweep" else tuning,
                      "sources": source_hash(), "steps": args.profile_steps, "marker_bytes": 4 * MARKER_ELEMS}))


def read_counters(path):
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    rows.sort()
    marks = [i for i, (d, k, c, v) in enumerate(rows) if "MulFunctor" in k]
    if len(marks) < 2:
        raise SystemExit(f"{path}: expected two marker dispatches, found {len(marks)}")
    lo, hi = marks[0], marks[-1]
    per = {}
    for d, k, c, v in rows[lo + 1:hi]:
        per.setdefault(k, []).append(v)
    return rows[lo][3], rows[hi][3], per


def summarize_pmc(fetch_csv, write_csv, probe_json, args_command=None):
    with open(probe_json) as f:
        probe = json.loads(f.read().strip().splitlines()[-1])
    mb = probe["marker_bytes"]
    f0, f1, fetch = read_counters(fetch_csv)
    w0, w1, write = read_counters(write_csv)
    ff = mb / (0.5 * (f0 + f1) * 1024.0)
    fw = mb / (0.5 * (w0 + w1) * 1024.0)
    name = probe.get("probe", "sweep")
    print(f"# HBM traffic per launch: {WORKLOADS[name]}\n")
    print("Commands (from the repository root, one MI355X; each counter in a run of its own):\n")
    print("```")
    if args_command:
        print(args_command)
    else:
        print(f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch_{name} -o fetch -- "
              f"python3 bench.py --pmc-probe --probe {name} > gpurun_out/probe_{name}.json")
        print(f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write_{name} -o write -- "
              f"python3 bench.py --pmc-probe --probe {name}")
        print(f"python3 bench.py --summarize-pmc gpurun_out/pmc_fetch_{name}/fetch_counter_collection.csv "
              f"gpurun_out/pmc_write_{name}/write_counter_collection.csv gpurun_out/probe_{name}.json")
    print("```\n")
    print(f"Calibration: an elementwise float32 copy of {mb} bytes (read {mb}, write {mb}) reads "
          f"FETCH_SIZE {f0:.0f} / {f1:.0f} KiB and WRITE_SIZE {w0:.0f} / {w1:.0f} KiB; scale factors "
          f"{ff:.4f} (fetch) and {fw:.4f} (write).\n")
    print(f"Kernels between the two markers (the per-kernel profile phase: {probe['steps']} eager DP45 steps "
          f"of the whole batch; tiles {json.dumps(probe.get('tiles'))}), per dispatch:\n")
    print("| kernel | dispatches | FETCH KiB | WRITE KiB | HBM bytes (scaled) |")
    print("|---|---|---|---|---|")
    out = {}
    for k in sorted(fetch, key=lambda k: -sum(fetch[k])):
        name = profile_name(k)
        fv = sum(fetch[k]) / len(fetch[k])
        wv = sum(write.get(k, [0.0])) / max(1, len(write.get(k, [])))
        b = fv * 1024.0 * ff + wv * 1024.0 * fw
        print(f"| `{k.split('(')[0]}` | {len(fetch[k])} | {fv:.0f} | {wv:.0f} | {b:.4g} |")
        if name:
            out[name] = b
    print("\nMachine-readable (kernel sources, FFT tiles, scaled bytes per launch):\n")
    print("```")
    print("traffic-json: " + json.dumps({"sources": probe["sources"], "tiles": probe["tiles"], "bytes": out}))
    print("```")


def tile_fields(kernel, tiles):
    """The part of the FFT tile choice that shapes `kernel`'s launches."""
    if tiles is None:
        return None
    if kernel.startswith("fft_x_"):
        keys = ("grid", "Wx", "x_stage")
    elif kernel.startswith("fft_"):
        keys = ("grid", "path", "TK", "Wy", "TW")
    else:
        keys = ("grid", "x_stage")
    out = []
    for t in tiles:
        d = {k: t.get(k) for k in keys}
        if kernel.startswith("fft_") and not kernel.startswith("fft_x_"):
            if d["path"] != "fused":
                d.pop("TK")
            if d["path"] != "split":
                d.pop("Wy")
            if d["path"] not in ("split", "splitx"):
                d.pop("TW")
        out.append(d)
    return out


def stored_traffic(kernel, tiles):
    """Scaled HBM bytes per launch of `kernel` from the stored counter summary,
    or None when the kernel sources, or the tiles of that kernel, changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("traffic-json: "):
                    rec = json.loads(line[len("traffic-json: "):])
                    if rec["sources"] == source_hash() and \
                            tile_fields(kernel, rec["tiles"]) == tile_fields(kernel, tiles):
                        return rec["bytes"].get(kernel)
    except OSError:
        pass
    return None


def build_batch(n, tol):
    from paper_2603_03706_amd import mmcav, workloads as W
    insts = [W.sweep_sphere(k, count=n) for k in range(n)]
    ctxs = [mmcav.Context.from_instance(inst) for inst in insts]
    for c in ctxs:
        c.set_sampling(SWEEP_DT_SAMPLE, SWEEP_MAX_SAMPLES)
    return insts, ctxs, mmcav.Batch(ctxs)


def timed_steps(batch, ctxs, steps, tol, warmup=0, marks=False):
    """Wall time of exactly `steps` attempted steps of an open run.  The run
    is begun (run parameters, run-start derivative, step graphs captured and
    uploaded), `warmup` untimed steps are run, the device is drained, and the
    clock runs around the next `steps` steps of the same run (graph launches
    only) and a device synchronisation; counts and statistics are read back
    outside the clock.  Returns (seconds, accepted instance-steps of the
    timed steps)."""
    import torch
    batch.begin(tol)
    batch.advance(warmup)
    a0, _ = batch.counts()
    torch.cuda.synchronize()
    if marks:
        mark()
    t0 = time.perf_counter()
    batch.advance(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if marks:
        mark()
    a1, _ = batch.counts()
    batch.end()
    return dt, a1 - a0


def plain_rate(insts, k, steps, warmup, tol):
    """Per-instance time of sequential plain runs (one instance per launch
    sequence), averaged over k instances."""
    from paper_2603_03706_amd import mmcav
    total = 0.0
    acc = 0
    for inst in insts[:k]:
        c = mmcav.Context.from_instance(inst)
        b = mmcav.Batch([c])
        dt, n = timed_steps(b, [c], steps, tol, warmup)
        total += dt
        acc += n
        b.close()
        c.close()
    return total / k, acc / k


def adjoint_ratio(steps, every):
    """Adjoint cost on the multimode film (128 x 128 x 32, 4 profiled modes,
    FFT demag), RK4 at 0.5 ps: plain forward run vs recorded run vs adjoint
    (checkpoint every `every` steps).  The cavity starts empty and mode 1 is
    driven by the Gaussian pulse of Sec. IV A (sigma 20 ps, centre 0.1 ns);
    the loss is |a_1(T)|^2 + |a_3(T)|^2 (mode 3 is reached only through the
    magnet)."""
    import numpy as np
    import torch
    from paper_2603_03706_amd import mmcav, workloads as W
    inst = W.adjoint_film()
    inst.a0 = np.zeros(4, complex)
    inst.drive_amp = np.array([2e8, 0, 0, 0], complex)
    inst.drive_t0 = np.full(4, 0.1e-9)
    inst.drive_sigma = np.full(4, 20e-12)
    T = steps * inst.dt0
    c = mmcav.Context.from_instance(inst)
    start = c.get_state()                     # t = 0, initial m and a
    c.run(10 * inst.dt0)                      # warm-up (graph capture, first launch)
    c.set_state(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run(T)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    c.set_state(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run_record(T, every)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    a = c.get_a()
    dl = np.zeros(4, complex)
    dl[0] = 2 * a[0]
    dl[2] = 2 * a[2]
    t0 = time.perf_counter()
    g = c.adjoint(dl)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    c.close()
    return {"workload": f"multimode film 128x128x32, 4 profiled modes, FFT demag, RK4 dt 0.5 ps, {steps} steps, "
                        f"checkpoint every {every}, mode 1 driven by the Sec. IV A pulse, "
                        "loss |a_1(T)|^2 + |a_3(T)|^2",
            "forward_s": t_fwd, "record_s": t_rec, "adjoint_s": t_adj,
            "adjoint_over_forward": t_adj / t_fwd, "record_plus_adjoint_over_forward": (t_rec + t_adj) / t_fwd,
            "loss": float(abs(a[0]) ** 2 + abs(a[2]) ** 2),
            "grad_g": [float(v) for v in g["g"]], "grad_alpha": float(g["alpha"]),
            "grad_u_norm": float(np.linalg.norm(g["u"]))}


def afm_batch(steps, tol):
    """AFM batch: 32 two-sublattice instances of 64^2x16 .. 256^2x16 at 2 nm,
    DP45: batched steps vs the same instances stepped one after another."""
    import torch
    from paper_2603_03706_amd import mmcav, workloads as W
    insts = [W.afm_instance(k) for k in range(32)]
    ctxs = [mmcav.Context.from_instance(i) for i in insts]
    b = mmcav.Batch(ctxs)
    b.tune()
    streams = b.streams()
    dt, acc = timed_steps(b, ctxs, steps, tol, 10)
    cells = sum(i.cells * 2 for i in insts)
    b.close()
    plain = 0.0
    for inst, c in zip(insts, ctxs):
        pb = mmcav.Batch([c])
        d, _ = timed_steps(pb, [c], steps, tol, 2)
        plain += d
        pb.close()
    for c in ctxs:
        c.close()
    return {"workload": "AFM batch: 32 instances, 64^2x16 .. 256^2x16, 2 sublattices, 2 nm, DP45 tol 1e-6",
            "sublattice_cells": cells, "streams": streams, "batched_s": dt, "plain_sequential_s": plain,
            "batched_vs_plain": plain / dt, "batched_cell_updates_per_s": cells * acc / len(insts) / dt}


def paper_sweep():
    """The anticrossing protocol of Sec. IV A on the device: 41 bias fields
    from 164 to 194 mT on the 8x8x1 geometry of Sec. IV (Table I, Sim 1), a
    Gaussian pulse, RK4 at 1 ps for 16 ns, all fields in one batch.  The
    paper ran this through its operator-split Python loop at about 4.4 ms
    per co-simulation step (Sec. III C); that figure is context for a
    different path, not a target."""
    import time
    import numpy as np
    import torch
    from paper_2603_03706_amd import mmcav, workloads as W
    insts = [W.paper_sim1(B0=b) for b in np.linspace(0.164, 0.194, 41)]
    ctxs = [mmcav.Context.from_instance(i) for i in insts]
    b = mmcav.Batch(ctxs)
    b.run(insts[0].dt0)                      # first step: graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(insts[0].T - insts[0].dt0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = [c.stats()["accepted"] - 1 for c in ctxs]
    b.close()
    for c in ctxs:
        c.close()
    fs = sum(steps)
    return {"workload": "anticrossing sweep of Sec. IV A: 41 fields 164-194 mT, 8x8x1 at 10 nm, "
                        "Gaussian pulse, RK4 1 ps for 16 ns, one batch",
            "instances": len(insts), "field_steps": fs, "wall_s": wall,
            "us_per_field_step": wall / fs * 1e6, "paper_cosim_ms_per_step": 4.4}


def film_rate(steps, tol):
    """Multimode film: 128 x 128 x 32 cells at 5 nm (524,288), FFT demag on
    256 x 256 x 64, four profiled modes, DP45 at tol, from m = +z with
    a_1(0) = 1: cell-updates/s of one instance."""
    import torch
    from paper_2603_03706_amd import mmcav, workloads as W
    inst = W.multimode_film()
    c = mmcav.Context.from_instance(inst)
    b = mmcav.Batch([c])
    b.tune()
    dt, acc = timed_steps(b, [c], steps, tol, 20)
    b.close()
    c.close()
    return {"workload": "multimode film 128x128x32 at 5 nm, FFT demag on 256x256x64, 4 profiled modes, "
                        f"DP45 tol {tol:g}", "cells": inst.cells, "steps": steps, "accepted": acc,
            "ms_per_step": dt / steps * 1e3, "cell_updates_per_s": inst.cells * acc / dt}


def oracle_rate(inst, seconds, tol):
    """Accepted steps of the oracle on one instance, DP45 from its initial
    state, in about `seconds` of host time: (accepted, rejected, seconds)."""
    import torch
    from tests.helpers import oracle_for
    st = oracle_for(inst)
    t0 = time.perf_counter()
    with torch.no_grad():
        st._dp_first()
        # advance in small slices until the time budget is used
        while time.perf_counter() - t0 < seconds:
            st.run(5e-13, tol)
    return st.accepted, st.rejected, time.perf_counter() - t0


def cpu_baseline(inst, seconds, tol):
    """The oracle, as it stands, on the host cores: one sweep instance for
    about `seconds` with one torch thread per core this process may run on
    (its CPU affinity), then for a third of that on one thread."""
    import torch
    cores = len(os.sched_getaffinity(0))
    prev = torch.get_num_threads()
    torch.set_num_threads(cores)
    try:
        acc, rej, dt = oracle_rate(inst, seconds, tol)
        torch.set_num_threads(1)
        acc1, _, dt1 = oracle_rate(inst, seconds / 3.0, tol)
    finally:
        torch.set_num_threads(prev)
    cells = inst.cells
    return {"value": cells * acc / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one 32^3 sphere instance (17,256 magnetic cells, FFT demag on 64^3), DP45 tol {tol:g}, "
                      f"{acc} accepted steps ({rej} rejected) in {dt:.1f} s from t = 0",
            "one_core": {"value": cells * acc1 / dt1, "cores": 1,
                         "sample": f"the same instance, {acc1} accepted steps in {dt1:.1f} s on one thread"}}


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args_command=args.command)
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the batched form would shard instances across GPUs, which is not built here.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_03706_amd import mmcav
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.pmc_probe:
        pmc_probe(args)
        return
    if args.leg_trace:
        leg_trace(args)
        return

    insts, ctxs, batch = build_batch(args.instances, args.tol)
    cells = sum(i.cells for i in insts)
    tuning = None
    if args.streams:
        batch.set_streams(args.streams)
    if not args.no_tune:
        tuning = batch.tune(streams=not args.streams)
        print(f"[bench] fft tuning: {json.dumps(tuning)}", file=sys.stderr, flush=True)
    print(f"[bench] {len(insts)} instances, {cells} cells; warmup {args.warmup} steps, then {args.steps} "
          "timed steps", file=sys.stderr, flush=True)
    dt, acc = timed_steps(batch, ctxs, args.steps, args.tol, args.warmup, marks=True)
    rate = cells / len(insts) * acc / dt
    st0 = ctxs[0].stats()
    print(f"[bench] {dt:.3f} s, {acc} accepted instance-steps, dt now {st0['dt']:.3e} s", file=sys.stderr, flush=True)

    roof = None
    kernels = []
    if not args.no_profile:
        mark()
        prof = batch.profile(args.profile_steps, args.tol)
        mark()
        for p in prof:
            avg_ms = p["total_ms"] / max(1, p["launches"])
            gbs = p["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
            kernels.append({"name": p["name"], "launches": p["launches"], "avg_us": avg_ms * 1e3,
                            "total_ms": p["total_ms"], "bytes_per_launch": p["bytes_per_launch"],
                            "GBps": gbs})
        kernels.sort(key=lambda k: -k["total_ms"])
        top = kernels[0]
        traffic = stored_traffic(top["name"], tile_key(tuning))
        hbm = {"achieved": round(top["GBps"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(top["GBps"] / HBM_PEAK_GBS, 4)}
        if top["name"] == "fft_yz_convolve":
            # bound by FP32 vector issue (rocprofv3 SQ counters: VALU busy
            # about 80 %, HBM about 15 %): priced against the VALU peak
            nx, ny, nz = insts[0].grid
            flops = len(insts) * yz_planes(nx) * yz_flops_per_item(ny, nz, padded(ny), padded(nz))
            tf = flops / (top["avg_us"] * 1e-6) / 1e12
            roof = {"bound": "alu", "achieved": round(tf, 2), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(tf / FP32_PEAK_TFLOPS, 4),
                    "unpacked_fp32_peak": round(VALU_UNPACKED_PEAK_TFLOPS, 1),
                    "frac_of_unpacked_peak": round(tf / VALU_UNPACKED_PEAK_TFLOPS, 4),
                    "flops_per_launch": flops, "hbm": hbm}
        else:
            roof = {"bound": "hbm", **hbm}
        roof.update({"traffic": None if traffic is None else round(traffic), "kernel": top["name"],
                     "avg_us": round(top["avg_us"], 2), "bytes_per_launch": top["bytes_per_launch"]})
        print(f"[bench] profile: {json.dumps(kernels)}", file=sys.stderr, flush=True)

    stream = None
    if not args.no_stream:
        # the achievable HBM bandwidth on this GPU, beside the 8 TB/s peak
        stream = stream_copy()
        if roof is not None:
            roof["hbm"]["achievable"] = round(stream["GBps"], 1)
        print(f"[bench] stream copy: {json.dumps(stream)}", file=sys.stderr, flush=True)

    speedup = None
    if not args.no_plain:
        k = min(args.plain_instances, len(insts))
        t_plain, acc_plain = plain_rate(insts, k, args.steps, args.warmup, args.tol)
        batched_per_step = dt / args.steps
        plain_per_step_all = t_plain / args.steps * len(insts)
        speedup = plain_per_step_all / batched_per_step
        print(f"[bench] plain: {t_plain / args.steps * 1e3:.3f} ms/step per instance ({k} measured), "
              f"batched {batched_per_step * 1e3:.3f} ms/step for {len(insts)}", file=sys.stderr, flush=True)

    adj = None
    if not args.no_adjoint:
        print("[bench] adjoint leg", file=sys.stderr, flush=True)
        adj = adjoint_ratio(args.adjoint_steps, 256)
        print(f"[bench] adjoint: {json.dumps(adj)}", file=sys.stderr, flush=True)
    afm = None
    if not args.no_afm:
        print("[bench] AFM batch leg", file=sys.stderr, flush=True)
        afm = afm_batch(args.afm_steps, args.tol)
        print(f"[bench] afm: {json.dumps(afm)}", file=sys.stderr, flush=True)

    film = None
    if not args.no_film:
        print("[bench] film leg", file=sys.stderr, flush=True)
        film = film_rate(args.film_steps, args.tol)
        print(f"[bench] film: {json.dumps(film)}", file=sys.stderr, flush=True)

    sweep41 = None
    if not args.no_paper_sweep:
        print("[bench] paper sweep leg", file=sys.stderr, flush=True)
        sweep41 = paper_sweep()
        print(f"[bench] paper sweep: {json.dumps(sweep41)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(insts[0], args.cpu_seconds, args.tol)

    out = {
        "metric": METRIC,
        "value": rate,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"field sweep: {len(insts)} YIG spheres (diameter 32 cells) on 32^3 grids at 5 nm, "
                               f"FFT demag on 64^3, 1 uniform mode, DP45 tol {args.tol:g}, batched",
                   "instances": len(insts), "grid": [32, 32, 32], "method": "dp45", "tol": args.tol,
                   "accepted_fraction": acc / (args.steps * len(insts)),
                   "streams": batch.streams(),
                   "fft_tiles": tile_key(tuning)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched_vs_plain": speedup,
        "adjoint_over_forward": None if adj is None else adj["adjoint_over_forward"],
        "adjoint": adj,
        "afm_batch": afm,
        "film": film,
        "paper_sweep": sweep41,
        "stream_copy": stream,
        "kernels": kernels,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
