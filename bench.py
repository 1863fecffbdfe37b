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
    return ap.parse_args()


def build_batch(n, tol):
    from paper_2603_03706_amd import mmcav, workloads as W
    insts = [W.sweep_sphere(k, count=n) for k in range(n)]
    ctxs = [mmcav.Context.from_instance(inst) for inst in insts]
    return insts, ctxs, mmcav.Batch(ctxs)


def accepted(ctxs):
    return sum(c.stats()["accepted"] for c in ctxs)


def timed_steps(batch, ctxs, steps, tol):
    import torch
    torch.cuda.synchronize()
    a0 = accepted(ctxs)
    t0 = time.perf_counter()
    batch.step(steps, tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, accepted(ctxs) - a0


def plain_rate(insts, k, steps, warmup, tol):
    """Per-instance time of sequential plain runs (one instance per launch
    sequence), averaged over k instances."""
    from paper_2603_03706_amd import mmcav
    total = 0.0
    acc = 0
    for inst in insts[:k]:
        c = mmcav.Context.from_instance(inst)
        b = mmcav.Batch([c])
        b.step(warmup, tol)
        dt, n = timed_steps(b, [c], steps, tol)
        total += dt
        acc += n
        b.close()
        c.close()
    return total / k, acc / k


def cpu_baseline(inst, seconds, tol):
    """The oracle, as it stands, on the host cores: one sweep instance,
    DP45 from the same initial state, for about `seconds` of CPU work."""
    import torch
    from tests.helpers import oracle_for
    st = oracle_for(inst)
    cores = torch.get_num_threads()
    t0 = time.perf_counter()
    with torch.no_grad():
        st._dp_first()
        # advance in small slices until the time budget is used
        while time.perf_counter() - t0 < seconds:
            st.run(5e-13, tol)
    dt = time.perf_counter() - t0
    cells = inst.cells
    return {"value": cells * st.accepted / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one 32^3 sphere instance (17,256 magnetic cells, FFT demag on 64^3), DP45 tol {tol:g}, "
                      f"{st.accepted} accepted steps ({st.rejected} rejected) in {dt:.1f} s from t = 0"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the batched form would shard instances across GPUs, which is not built here.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_03706_amd import mmcav
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    insts, ctxs, batch = build_batch(args.instances, args.tol)
    cells = sum(i.cells for i in insts)
    print(f"[bench] {len(insts)} instances, {cells} cells; warmup {args.warmup} steps", file=sys.stderr, flush=True)
    batch.step(args.warmup, args.tol)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    dt, acc = timed_steps(batch, ctxs, args.steps, args.tol)
    rate = cells / len(insts) * acc / dt
    st0 = ctxs[0].stats()
    print(f"[bench] {dt:.3f} s, {acc} accepted instance-steps, dt now {st0['dt']:.3e} s", file=sys.stderr, flush=True)

    roof = None
    kernels = []
    if not args.no_profile:
        prof = batch.profile(args.profile_steps, args.tol)
        for p in prof:
            avg_ms = p["total_ms"] / max(1, p["launches"])
            gbs = p["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
            kernels.append({"name": p["name"], "launches": p["launches"], "avg_us": avg_ms * 1e3,
                            "total_ms": p["total_ms"], "bytes_per_launch": p["bytes_per_launch"],
                            "GBps": gbs})
        kernels.sort(key=lambda k: -k["total_ms"])
        top = kernels[0]
        roof = {"bound": "hbm", "achieved": round(top["GBps"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(top["GBps"] / HBM_PEAK_GBS, 4), "traffic": None, "kernel": top["name"],
                "avg_us": round(top["avg_us"], 2), "bytes_per_launch": top["bytes_per_launch"]}
        print(f"[bench] profile: {json.dumps(kernels)}", file=sys.stderr, flush=True)

    speedup = None
    if not args.no_plain:
        k = min(args.plain_instances, len(insts))
        t_plain, acc_plain = plain_rate(insts, k, args.steps, args.warmup, args.tol)
        batched_per_step = dt / args.steps
        plain_per_step_all = t_plain / args.steps * len(insts)
        speedup = plain_per_step_all / batched_per_step
        print(f"[bench] plain: {t_plain / args.steps * 1e3:.3f} ms/step per instance ({k} measured), "
              f"batched {batched_per_step * 1e3:.3f} ms/step for {len(insts)}", file=sys.stderr, flush=True)

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
                   "accepted_fraction": acc / (args.steps * len(insts))},
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched_vs_plain": speedup,
        "adjoint_over_forward": None,
        "kernels": kernels,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
