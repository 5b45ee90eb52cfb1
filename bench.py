#!/usr/bin/env python3
"""States integrated per second per global step on one MI355X.

A step is one pass of the whole hot path over the batch: every state of the
workload integrated over one global time step with Radau IIA, once for each
global step size of the workload (1e-6 s and 1e-4 s for the default
262,144-state PaSR-like H2/CO-like workload).  Inputs are resident in HBM
before timing starts.  Prints one JSON line.

Forms (same library, same inputs):
  plain          FP64 factors, one 16-lane group (N <= 16) or wavefront per
                 state, persistent queue in input order, no predictor
  binned         plain + autotuned cost bins of the work queue (proxy key)
  learned        binned + the MLP first-step predictor; bins keyed by the
                 predicted step counts
  learned_mixed  learned with FP32 iteration-matrix factors (FP64 residuals)
  mixed          binned with FP32 factors
  lane           one state per lane (the paper's per-thread pattern)
  block          one 512-lane block per state, FP32 factors, 16 proxy cost bins (N = 57..153;
                 the only cooperative form for the 150-species workload)
The headline form (--form) is timed over --steps steps; the others get one
warm-up and one timed step each for the comparison block.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 64 FP64 FMA/clk x 2 flops x 2.4 GHz

KERNEL_SOURCES = {"radau_group_kernel": ["rk_group_impl.h", "rk_group16.hip", "rk_internal.h"],
                  "radau_block_kernel": ["rk_block.hip", "rk_group_impl.h", "rk_internal.h"],
                  "radau_lane_kernel": ["rk_kernels.hip", "rk_internal.h"]}

FORMS = {
    "plain": dict(variant="wave", binning=0, autotune=0, predictor=False),
    "binned": dict(variant="wave", binning=0, autotune=1, predictor=False),
    "learned": dict(variant="wave", binning=0, autotune=1, predictor=True),
    "learned_mixed": dict(variant="mixed", binning=0, autotune=1, predictor=True),
    "mixed": dict(variant="mixed", binning=0, autotune=1, predictor=False),
    "lane": dict(variant="lane", binning=0, autotune=0, predictor=False),
    "block": dict(variant="block", binning=16, autotune=0, predictor=False),
}


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


def max_rel_err(got, ref, K):
    import numpy as np
    relT = np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
    Yr = ref[:, 1:K + 1]
    mask = Yr > 1e-8
    relY = np.where(mask, np.abs(got[:, 1:K + 1] - Yr) / np.where(mask, Yr, 1.0), 0.0)
    return float(max(relT.max(initial=0.0), relY.max(initial=0.0)))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--form", default="learned", choices=sorted(FORMS))
    ap.add_argument("--compare", default="plain,binned,learned_mixed,mixed,lane",
                    help="other forms timed (1 warm-up + 1 step each) for the comparison block")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dt", type=float, default=None,
                    help="only this global step size (profiling runs; the headline uses every dt)")
    ap.add_argument("--n-states", type=int, default=None,
                    help="only the first N states of the workload (a bounded sample of a large workload)")
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

    from paper_1607_03884_amd import Mechanism, configs, gen, predictor
    from paper_1607_03884_amd.flops import Costs

    wl = configs.WORKLOADS[args.workload]
    if args.dt is not None:
        if not any(abs(args.dt - d) <= 1e-12 * d for d in wl.dts):
            print(f"--dt must be one of {wl.dts}", file=sys.stderr)
            return 2
        wl = dataclasses.replace(wl, dts=(args.dt,))
    path = configs.mech_path(wl.mech)
    mech_def = gen.make_mechanism(configs.MECHS[wl.mech])
    costs = Costs.of(mech_def)
    states = configs.states_for(wl)
    if args.n_states is not None:
        states = states[:max(1, args.n_states)]
    n = len(states)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    y = torch.from_numpy(gen.to_soa(states)).to(dev)
    out = torch.empty_like(y)
    stream = torch.cuda.current_stream()
    have_pred = all(os.path.exists(predictor.path_for(wl.mech, dt)) for dt in wl.dts)

    def make(form):
        f = FORMS[form]
        if f["predictor"] and not have_pred:
            return None
        m = Mechanism(path)
        for k in ("variant", "binning", "autotune"):
            m.set_option(k, f[k])
        if f["predictor"]:
            for dt in wl.dts:
                m.set_option("predictor", predictor.path_for(wl.mech, dt))
        return m

    def launch(m, dt):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        m.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
        b.record(stream)
        return a, b

    def launch_stats(m, dt, ms):
        """counters of one (deterministic) launch, outside any timed region"""
        m.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
        st = m.stats()
        fl = costs.flops(st)
        tf = fl["flops"] / (ms * 1e-3) / 1e12
        return st, fl, {"states_per_s": n / (ms * 1e-3), "kernel_ms": ms, "bins": st["nbins_used"],
                        "grid": st["grid_used"], "steps_per_state": st["steps"] / n, "max_steps": st["max_steps"],
                        "newton_per_step": st["newton_iters"] / max(st["steps"], 1),
                        "newton_fail": st["newton_fail"], "rejected": st["rejected"],
                        "jac_evals": st["jac_evals"], "lu_factor": st["lu_factor"], "failed": st["n_failed"],
                        "fp32_fallback": st["fp32_fallback"], "predictor_kept": st["predictor_kept"],
                        "predictor_fallback": st["predictor_fallback"], "D64_mean": st["d_mean64"],
                        "D32_mean": st["d_mean32"], "gflop": fl["flops"] / 1e9,
                        "gtrans": fl["transcendentals"] / 1e9, "tflops": tf,
                        "fp64_frac": tf / FP64_VECTOR_PEAK_TFLOPS}

    form = args.form
    if configs.MECHS[wl.mech].n_species + 1 > 56 and FORMS[form]["variant"] in ("wave", "mixed"):
        print(f"[bench] {wl.mech} has more than 56 unknowns: headline form 'block'", flush=True)
        form = "block"
    if FORMS[form]["predictor"] and not have_pred:
        print(f"[bench] no predictor files for {wl.mech}; headline form falls back to 'binned'", flush=True)
        form = "binned"
    mech = make(form)
    print(f"[bench] {wl.name}: {n} states, mechanism {wl.mech} (K={mech.K}, R={mech.R}), dts {wl.dts}, "
          f"form {form}", flush=True)

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
            events[dt].append(launch(mech, dt))
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

    per_dt, gpu_out = {}, {}
    tot_flops = tot_ms = 0.0
    for dt in wl.dts:
        st, fl, rec = launch_stats(mech, dt, kernel_ms[dt])
        gpu_out[dt] = out.cpu().numpy().T.copy()
        tot_flops += fl["flops"]
        tot_ms += kernel_ms[dt]
        per_dt[f"{dt:g}"] = rec
        print(f"[bench] statistics launch dt={dt:g} done", flush=True)
    achieved = tot_flops / (tot_ms * 1e-3) / 1e12
    kname = {"lane": "radau_lane_kernel", "block": "radau_block_kernel"}.get(FORMS[form]["variant"],
                                                                             "radau_group_kernel")
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(kname, wl.name),
                "kernel": kname, "flops_per_launch": tot_flops / len(wl.dts),
                "note": "launch time includes the predictor network and bin sort (separate small kernels)"}

    # the paper's convention: the same step with the states copied in from
    # pinned host memory before and back after (not the headline value)
    host_in = torch.from_numpy(gen.to_soa(states)).pin_memory()
    host_out = torch.empty_like(host_in).pin_memory()
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for dt in wl.dts:
        y.copy_(host_in, non_blocking=True)
        mech.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
        host_out.copy_(out, non_blocking=True)
    torch.cuda.synchronize()
    print("[bench] host-copy step done", flush=True)
    pcie = {"states_per_s": n * len(wl.dts) / (time.perf_counter() - p0),
            "note": "one step with H2D copy of y before and D2H copy of y_out after each dt (pinned host memory)"}
    del host_in, host_out

    compare = {}
    for other in [v for v in args.compare.split(",") if v and v != form]:
        m = make(other)
        if m is None:
            continue
        recs, tot = {}, 0.0
        for dt in wl.dts:
            m.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
            a, b = launch(m, dt)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            tot += ms
            _, _, recs[f"{dt:g}"] = launch_stats(m, dt, ms)
        m.close()
        compare[other] = {"per_step_states_per_s": n * len(wl.dts) / (tot * 1e-3), "per_dt": recs}
        print(f"[bench] compared {other}: {compare[other]['per_step_states_per_s']:.0f} states/s", flush=True)

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import predict as opred
        m_or = oracle.Mech(path)
        sample = states[:min(args.cpu_sample, n)]
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        c0 = time.perf_counter()
        cold = {dt: m_or.integrate(sample, dt, configs.ATOL, configs.RTOL, nthreads=threads)[0] for dt in wl.dts}
        c1 = time.perf_counter()
        cpu = {"value": len(sample) * len(wl.dts) / (c1 - c0), "unit": "states/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {len(sample)} states of the {n}-state set (same PaSR-like mix), each dt"}
        parity = {"sample": len(sample), "tol": 1e-5,
                  "vs_oracle_cold": max(max_rel_err(gpu_out[dt][:len(sample)], cold[dt], mech.K) for dt in wl.dts)}
        if FORMS[form]["predictor"]:
            worst = 0.0
            for dt in wl.dts:
                pr = opred.load(predictor.path_for(wl.mech, dt))
                h, z, _ = opred.warm_start(pr, sample, configs.ATOL, configs.RTOL, dt)
                ref, _ = m_or.integrate_warm(sample, dt, h, z, configs.ATOL, configs.RTOL, nthreads=threads)
                worst = max(worst, max_rel_err(gpu_out[dt][:len(sample)], ref, mech.K))
            parity["vs_oracle_same_start"] = worst
            parity["note"] = ("the learned form is judged against the oracle started from the same "
                              "prediction; vs_oracle_cold is the deviation from a cold-started oracle")

    value = n * len(wl.dts) / sec_per_step
    fdesc = FORMS[form]
    line = {
        "metric": "states integrated/s per global step (dt=1e-6,1e-4 s), learned+FP32-LU vs plain FP64",
        "value": value, "unit": "states/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: synthetic {wl.mech} ({mech.K} species, {mech.R} reversible reactions), "
                               f"{n} PaSR-like states" + (f" (first {n} of {wl.n_states})" if n < wl.n_states else "")
                               + f", one global step at each of {list(wl.dts)} s",
                   "n_states": n, "dts": list(wl.dts), "atol": configs.ATOL, "rtol": configs.RTOL,
                   "form": form, "variant": fdesc["variant"], "autotune": fdesc["autotune"],
                   "predictor": fdesc["predictor"],
                   "factors": "FP32 (FP64 residuals)" if fdesc["variant"] in ("mixed", "block") else "FP64"},
        "per_dt": per_dt,
        "compare": compare,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "pcie_inclusive": pcie,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
