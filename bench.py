#!/usr/bin/env python3
"""States integrated per second per global step on one MI355X.

A step is one pass of the whole hot path over the batch: every state of the
workload integrated over one global time step with Radau IIA, once for each
global step size of the workload (1e-6 s and 1e-4 s for the default
262,144-state PaSR-like H2/CO-like workload).  Inputs are resident in HBM
before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 64 FP64 FMA/clk x 2 flops x 2.4 GHz

KERNEL_SOURCES = {"radau_group_kernel": ["rk_group.hip", "rk_internal.h"],
                  "radau_lane_kernel": ["rk_kernels.hip", "rk_internal.h"]}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per dispatch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_dispatch", "source_sha256_16"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_1607_03884_amd", "csrc", f), "rb").read())
    if fields.get("source_sha256_16") != h.hexdigest()[:16] or "traffic_bytes_per_dispatch" not in fields:
        return None
    return float(fields["traffic_bytes_per_dispatch"])


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--variant", default="wave", help="lane | wave | mixed")
    ap.add_argument("--binning", type=int, default=0, help="cost bins of the work queue (0 = input order)")
    ap.add_argument("--autotune", type=int, default=1, help="1: let the library tune bins and grid per dt")
    ap.add_argument("--compare", default="lane,mixed",
                    help="other variants timed (1 warmup + 1 step each) for the comparison fields")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, run one plain 512 MiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: states are independent and the multi-GPU path "
              "(sharding states across GPUs) is not part of this build; run with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1607_03884_amd import Mechanism, configs, gen
    from paper_1607_03884_amd.flops import Costs

    wl = configs.WORKLOADS[args.workload]
    path = configs.mech_path(wl.mech)
    mech_def = gen.make_mechanism(configs.MECHS[wl.mech])
    states = configs.states_for(wl)
    n = len(states)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    y = torch.from_numpy(gen.to_soa(states)).to(dev)
    out = torch.empty_like(y)
    mech = Mechanism(path)
    mech.set_option("variant", args.variant)
    mech.set_option("binning", args.binning)
    mech.set_option("autotune", args.autotune)
    stream = torch.cuda.current_stream()
    print(f"[bench] {wl.name}: {n} states, mechanism {wl.mech} (K={mech.K}, R={mech.R}), dts {wl.dts}", flush=True)

    for _ in range(args.warmup):
        for dt in wl.dts:
            mech.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
    torch.cuda.synchronize()
    print("[bench] warmup done", flush=True)

    events = {dt: [] for dt in wl.dts}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for dt in wl.dts:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            mech.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
            b.record(stream)
            events[dt].append((a, b))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec_per_step = (t1 - t0) / args.steps
    kernel_ms = {dt: float(np.mean([a.elapsed_time(b) for a, b in events[dt]])) for dt in wl.dts}
    print(f"[bench] timed {args.steps} steps: {sec_per_step * 1e3:.2f} ms/step", flush=True)

    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 536870912 bytes read, 536870912 bytes written", flush=True)
        del src, dst

    # counters of one (identical, deterministic) launch per dt, outside the timed region
    costs = Costs.of(mech_def)
    per_dt = {}
    gpu_out = {}
    tot_flops = tot_ms = 0.0
    for dt in wl.dts:
        mech.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
        st = mech.stats()
        fl = costs.flops(st)
        gpu_out[dt] = out.cpu().numpy().T.copy()
        tot_flops += fl["flops"]
        tot_ms += kernel_ms[dt]
        per_dt[f"{dt:g}"] = {"states_per_s": n / (kernel_ms[dt] * 1e-3), "kernel_ms": kernel_ms[dt],
                             "bins": st["nbins_used"], "grid": st["grid_used"], "fp32_fallback": st["fp32_fallback"],
                             "steps_per_state": st["steps"] / n, "max_steps": st["max_steps"],
                             "newton_per_step": st["newton_iters"] / max(st["steps"], 1),
                             "jac_evals": st["jac_evals"], "lu_factor": st["lu_factor"],
                             "failed": st["n_failed"], "D64_mean": st["d_mean64"], "D32_mean": st["d_mean32"],
                             "gflop": fl["flops"] / 1e9, "gtrans": fl["transcendentals"] / 1e9}
    achieved = tot_flops / (tot_ms * 1e-3) / 1e12
    kname = {"lane": "radau_lane_kernel", "wave": "radau_group_kernel"}.get(args.variant, args.variant)
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(kname, wl.name),
                "kernel": kname, "flops_per_launch": tot_flops / len(wl.dts)}

    # the other variants, same inputs, for the comparison fields (not the headline value)
    compare = {}
    for var in [v for v in args.compare.split(",") if v and v != args.variant]:
        other = Mechanism(path)
        other.set_option("variant", var)
        other.set_option("autotune", args.autotune if var != "lane" else 0)
        rate = {}
        for dt in wl.dts:
            other.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            other.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            rate[f"{dt:g}"] = n / (a.elapsed_time(b) * 1e-3)
        compare[var] = {"states_per_s": rate,
                        "per_step_states_per_s": n * len(wl.dts) / sum(n / r for r in rate.values())}
        other.close()
        print(f"[bench] compared {var}: {compare[var]['per_step_states_per_s']:.0f} states/s", flush=True)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        m_or = oracle.Mech(path)
        sample = states[:min(args.cpu_sample, n)]
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        c0 = time.perf_counter()
        worst = 0.0
        for dt in wl.dts:
            ref, res = m_or.integrate(sample, dt, configs.ATOL, configs.RTOL, nthreads=threads)
            g = gpu_out[dt][:len(sample)]
            relT = np.abs(g[:, 0] - ref[:, 0]) / ref[:, 0]
            Yr = ref[:, 1:mech.K + 1]
            mask = Yr > 1e-8
            relY = np.where(mask, np.abs(g[:, 1:mech.K + 1] - Yr) / np.where(mask, Yr, 1.0), 0.0)
            worst = max(worst, float(relT.max()), float(relY.max()))
        c1 = time.perf_counter()
        cpu = {"value": len(sample) * len(wl.dts) / (c1 - c0), "unit": "states/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {len(sample)} states of the {n}-state set (same PaSR-like mix), each dt"}
        parity = {"max_rel_err_vs_oracle": worst, "sample": len(sample), "tol": 1e-5}

    value = n * len(wl.dts) / sec_per_step
    line = {
        "metric": "states integrated/s per global step (dt=1e-6,1e-4 s)",
        "value": value, "unit": "states/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: synthetic {wl.mech} ({mech.K} species, {mech.R} reversible reactions), "
                               f"{n} PaSR-like states, one global step at each of {list(wl.dts)} s",
                   "n_states": n, "dts": list(wl.dts), "atol": configs.ATOL, "rtol": configs.RTOL,
                   "variant": args.variant, "autotune": args.autotune, "binning": args.binning,
                   "path": "mixed FP32 factors" if args.variant == "mixed" else "plain FP64"},
        "per_dt": per_dt,
        "compare": compare,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
