#!/usr/bin/env python3
"""States integrated per second per global step on one MI355X.

A step is one pass of the whole hot path over the batch: every state of the
workload integrated over one global time step with Radau IIA, once for each
global step size of the workload.  The default workload is the 53-species
PaSR-like set (131,072 states, global steps 1e-6 s and 1e-4 s) with the
learned predictor; inputs are resident in HBM before timing starts.  Prints
one JSON line.

Forms (same library, same inputs):
  learned        headline: FP32 iteration-matrix factors with FP64 residuals
                 (variant "mixed"), persistent queue ordered by autotuned bins
                 of the MLP's predicted step counts, cold starts (the network
                 orders the queue and nothing else, so results are bitwise those
                 of the mixed variant and are compared with the cold oracle)
  plain          FP64 factors, one 16-lane group (N <= 16) or wavefront per
                 state, persistent queue in input order, no predictor
  binned         plain + autotuned proxy-key cost bins
  mixed          FP32 factors + autotuned proxy-key cost bins
  learned_fp64   the learned form with FP64 factors
  learned_warm   the learned form plus the predicted first step size and
                 stage values as warm start (a different step sequence:
                 compared with the oracle started from the same prediction,
                 its deviation from the cold oracle reported)
  lane           one state per lane (the paper's per-thread pattern)
  block          one 512-lane block per state, FP32 factors, 16 proxy cost
                 bins (N = 57..153; the cooperative form for 150 species)
  block_fp64     block with FP64-accurate solves (three to six refinement
                 sweeps per solve from the first step)
  block_learned  block with its queue binned by the MLP's predicted step
                 counts (cold starts)
  block_learned_warm  block_learned plus the predicted first step size and
                 stage values as warm start (as learned_warm)
  rodas3         the Rosenbrock method Rodas3 on the wavefront kernels (FP64,
                 autotuned proxy bins): the semi-implicit alternative the
                 paper recommends; it solves the same ODE to the same
                 tolerances but follows its own steps, so its cold-oracle
                 figure is the difference of two methods
The headline form (--form) is timed over --steps steps; each comparison form
gets one timed step (after a warm-up call when it autotunes).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 64 FP64 FMA/clk x 2 flops x 2.4 GHz

# source files whose text decides each kernel's code, launch shape and table
# layouts (counter summaries carry their hash and are ignored once any of them
# changes): the kernel's own sources, the shared device structures, and the
# host code that builds the device tables and launches it
_COMMON = ["rk_internal.h", "rk_api.cpp"]
KERNEL_SOURCES = {"radau_group_kernel16": ["rk_group_impl.h", "rk_group16.hip", "rk_group.hip"] + _COMMON,
                  "radau_group_kernel64": ["rk_group_impl.h", "rk_group64.hip", "rk_group.hip"] + _COMMON,
                  "radau_block_kernel": ["rk_block.hip", "rk_group_impl.h"] + _COMMON,
                  "radau_lane_kernel": ["rk_kernels.hip"] + _COMMON}

FORMS = {
    "learned": dict(variant="mixed", binning=0, autotune=1, predictor="bins"),
    "plain": dict(variant="wave", binning=0, autotune=0, predictor=None),
    "binned": dict(variant="wave", binning=0, autotune=1, predictor=None),
    "mixed": dict(variant="mixed", binning=0, autotune=1, predictor=None),
    "learned_fp64": dict(variant="wave", binning=0, autotune=1, predictor="bins"),
    "learned_warm": dict(variant="mixed", binning=0, autotune=1, predictor="both"),
    "lane": dict(variant="lane", binning=0, autotune=0, predictor=None),
    "block": dict(variant="block", binning=16, autotune=0, predictor=None),
    "block_fp64": dict(variant="block", binning=16, autotune=0, predictor=None, block_solves="fp64_accurate"),
    "block_learned": dict(variant="block", binning=16, autotune=0, predictor="bins"),
    "block_learned_warm": dict(variant="block", binning=16, autotune=0, predictor="both"),
    "rodas3": dict(variant="wave", binning=0, autotune=1, predictor=None, method="rodas3"),
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_1607_03884_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per dispatch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_dispatch", "source_sha256_16"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    if fields.get("source_sha256_16") != source_hash(kernel) or "traffic_bytes_per_dispatch" not in fields:
        return None
    return float(fields["traffic_bytes_per_dispatch"])


def max_rel_err(got, ref, K):
    import numpy as np
    relT = np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
    Yr = ref[:, 1:K + 1]
    mask = Yr > 1e-8
    relY = np.where(mask, np.abs(got[:, 1:K + 1] - Yr) / np.where(mask, Yr, 1.0), 0.0)
    return float(max(relT.max(initial=0.0), relY.max(initial=0.0)))


def eq1_error(got, truth, K, atol, rtol):
    """Eq. (1) per state against a tight-tolerance run: the weighted 2-norm as
    printed and its RMS form; the maximum over states of each."""
    import numpy as np
    N = K + 1
    w = atol + np.abs(truth[:, :N]) * rtol
    e = (got[:, :N] - truth[:, :N]) / w
    two = np.sqrt((e * e).sum(axis=1))
    return {"two_norm_max": float(two.max()), "rms_max": float((two / np.sqrt(N)).max())}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--form", default=None, choices=sorted(FORMS),
                    help="headline form (default: learned; block for N > 56)")
    ap.add_argument("--compare", default=None,
                    help="other forms timed once each (default: plain,learned_warm; "
                         "block_fp64 for N > 56); empty string for none")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dt", type=float, default=None,
                    help="only this global step size (profiling runs; the headline uses every dt)")
    ap.add_argument("--n-states", type=int, default=None,
                    help="only the first N states of the workload (a bounded sample of a large workload)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, run one plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--jac-ratio", action="store_true",
                    help="instead of the headline: the runtime ratio of Radau IIA with the first-order "
                         "finite-difference Jacobian to the analytical one (paper Sec. 3.4), GPU lane and wave "
                         "kernels and the CPU oracle; prints one JSON line")
    ap.add_argument("--ratio-variants", default="lane,wave",
                    help="GPU variants of --jac-ratio (the lane kernel is slow for large mechanisms)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: states are independent and the multi-GPU path "
              "(sharding states across GPUs) is not implemented; run with --gpus 1.", file=sys.stderr)
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
    big = configs.MECHS[wl.mech].n_species + 1 > 56
    form = args.form or ("block" if big else "learned")
    compare_arg = args.compare if args.compare is not None else ("block_fp64" if big else "plain,learned_warm")
    path = configs.mech_path(wl.mech)
    mech_def = gen.make_mechanism(configs.MECHS[wl.mech])
    costs = Costs.of(mech_def)
    states = configs.states_for(wl)
    if args.n_states is not None:
        states = states[:max(1, args.n_states)]
    n = len(states)
    K = mech_def.K
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    y = torch.from_numpy(gen.to_soa(states)).to(dev)
    out = torch.empty_like(y)
    stream = torch.cuda.current_stream()
    have_pred = all(os.path.exists(predictor.path_for(wl.mech, dt)) for dt in wl.dts)

    def make(fname):
        f = FORMS[fname]
        if f["predictor"] and not have_pred:
            return None
        m = Mechanism(path)
        for k in ("variant", "binning", "autotune"):
            m.set_option(k, f[k])
        for key in ("block_solves", "method"):
            if key in f:
                m.set_option(key, f[key])
        if f["predictor"]:
            for dt in wl.dts:
                m.set_option("predictor", predictor.path_for(wl.mech, dt))
            m.set_option("predictor_use", f["predictor"])
        return m

    def launch(m, dt):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        m.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
        b.record(stream)
        return a, b

    def record(st, ms):
        """counters of a (deterministic) launch and its algorithmic rate"""
        fl = costs.flops(st)
        tf = fl["flops"] / (ms * 1e-3) / 1e12
        return fl, {"states_per_s": n / (ms * 1e-3), "kernel_ms": ms, "bins": st["nbins_used"],
                    "grid": st["grid_used"], "steps_per_state": st["steps"] / n, "max_steps": st["max_steps"],
                    "newton_per_step": st["newton_iters"] / max(st["steps"], 1),
                    "newton_fail": st["newton_fail"], "rejected": st["rejected"],
                    "jac_evals": st["jac_evals"], "lu_factor": st["lu_factor"], "failed": st["n_failed"],
                    "fp32_fallback": st["fp32_fallback"], "predictor_kept": st["predictor_kept"],
                    "predictor_fallback": st["predictor_fallback"], "D64_mean": st["d_mean64"],
                    "D32_mean": st["d_mean32"], "D64_queue_mean": st["d_mean64_queue"],
                    "gflop": fl["flops"] / 1e9, "gtrans": fl["transcendentals"] / 1e9, "tflops": tf,
                    "fp64_frac": tf / FP64_VECTOR_PEAK_TFLOPS}

    if args.jac_ratio:
        return jac_ratio(args, wl, states, y, out, stream, path)
    if FORMS[form]["predictor"] and not have_pred:
        print(f"[bench] no predictor files for {wl.mech}; headline form falls back to 'mixed'", flush=True)
        form = "mixed"
    mech = make(form)
    print(f"[bench] {wl.name}: {n} states, mechanism {wl.mech} (K={mech.K}, R={mech.R}), dts {wl.dts}, "
          f"form {form}", flush=True)

    for _ in range(args.warmup):
        for dt in wl.dts:
            mech.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
            torch.cuda.synchronize()
            print(f"[bench] warm-up dt={dt:g} done", flush=True)

    events = {dt: [] for dt in wl.dts}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
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

    # statistics and outputs of one launch per dt (integration is deterministic)
    per_dt, gpu_out, steps_of = {}, {}, {}
    tot_flops = tot_ms = 0.0
    for dt in wl.dts:
        mech.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
        st = mech.stats(per_state=True)
        fl, rec = record(st, kernel_ms[dt])
        gpu_out[dt] = out.cpu().numpy().T.copy()
        steps_of[dt] = st["per_state_steps"].copy()
        tot_flops += fl["flops"]
        tot_ms += kernel_ms[dt]
        per_dt[f"{dt:g}"] = rec
        print(f"[bench] statistics launch dt={dt:g} done", flush=True)
    achieved = tot_flops / (tot_ms * 1e-3) / 1e12
    variant = FORMS[form]["variant"]
    if variant == "lane":
        kname = "radau_lane_kernel"
    elif variant == "block":
        kname = "radau_block_kernel"
    else:
        kname = "radau_group_kernel16" if mech.N <= 16 else "radau_group_kernel64"
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(kname, wl.name),
                "kernel": kname, "flops_per_launch": tot_flops / len(wl.dts),
                "note": "algorithmic FP64-vector flops (flop model x per-state counters) over the whole "
                        "radau_integrate call per dt; the call's predictor and bin-sort kernels take ~0.02 %"}

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

    # parity sample: the 1 % costliest states (by step count) and a seeded draw
    rng = np.random.default_rng(4242)
    draw = np.sort(rng.choice(n, min(args.cpu_sample, n), replace=False))
    costly = np.unique(np.concatenate([np.argsort(steps_of[dt], kind="stable")[-max(1, n // 100):]
                                       for dt in wl.dts]))
    pick = np.unique(np.concatenate([draw, costly]))

    compare, cmp_out = {}, {}
    for other in [v for v in compare_arg.split(",") if v and v != form]:
        m = make(other)
        if m is None:
            continue
        recs, tot = {}, 0.0
        cmp_out[other] = {}
        for dt in wl.dts:
            if FORMS[other]["autotune"]:
                m.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)   # tunes, warms
            a, b = launch(m, dt)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            tot += ms
            _, recs[f"{dt:g}"] = record(m.stats(), ms)
            cmp_out[other][dt] = out.cpu().numpy().T[pick].copy()
        m.close()
        compare[other] = {"per_step_states_per_s": n * len(wl.dts) / (tot * 1e-3), "per_dt": recs}
        print(f"[bench] compared {other}: {compare[other]['per_step_states_per_s']:.0f} states/s", flush=True)

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import predict as opred
        m_or = oracle.Mech(path)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        sample = states[draw]
        c0 = time.perf_counter()
        cold_draw = {dt: m_or.integrate(sample, dt, configs.ATOL, configs.RTOL, nthreads=threads)[0]
                     for dt in wl.dts}
        c1 = time.perf_counter()
        cpu = {"value": len(sample) * len(wl.dts) / (c1 - c0), "unit": "states/s", "cores": threads,
               "kind": "oracle", "cpu": cpu_model(),
               "sample": f"{len(sample)} states drawn uniformly (seed 4242) from the {n}-state set, each dt"}
        print(f"[bench] CPU oracle: {cpu['value']:.0f} states/s on {threads} threads", flush=True)
        # the cold oracle on the whole parity sample (the costliest states added, untimed)
        rest = np.setdiff1d(pick, draw)
        cold = {}
        for dt in wl.dts:
            r = m_or.integrate(states[rest], dt, configs.ATOL, configs.RTOL, nthreads=threads)[0] if len(rest) \
                else np.zeros((0, K + 2))
            full = np.zeros((n, K + 2))
            full[draw] = cold_draw[dt]
            full[rest] = r
            cold[dt] = full[pick]
        parity = {"sample": int(len(pick)), "costliest_included": int(len(costly)), "tol": 1e-5,
                  "vs_oracle_cold": max(max_rel_err(gpu_out[dt][pick], cold[dt], K) for dt in wl.dts),
                  "per_form_vs_oracle_cold": {
                      f: max(max_rel_err(cmp_out[f][dt], cold[dt], K) for dt in wl.dts) for f in cmp_out}}
        warm_forms = [f for f in [form] + list(cmp_out) if FORMS[f]["predictor"] in ("both", "h0", "z0")]
        if warm_forms:
            # warm-started forms: also against the oracle started from the same prediction
            for f in warm_forms:
                worst = 0.0
                print(f"[bench] same-start oracle for {f}", flush=True)
                for dt in wl.dts:
                    pr = opred.load(predictor.path_for(wl.mech, dt))
                    h, z, _ = opred.warm_start(pr, states[pick], configs.ATOL, configs.RTOL, dt)
                    ref, _ = m_or.integrate_warm(states[pick], dt, h, z, configs.ATOL, configs.RTOL,
                                                 nthreads=threads)
                    got = gpu_out[dt][pick] if f == form else cmp_out[f][dt]
                    worst = max(worst, max_rel_err(got, ref, K))
                parity.setdefault("vs_oracle_same_start", {})[f] = worst
            # Eq. (1) against a tight-tolerance oracle run on a small sub-sample
            # (fewer states for the large mechanism: the tight run is slow there)
            sub = pick[:256 if K + 1 <= 56 else 16]
            print(f"[bench] tight-tolerance oracle on {len(sub)} states", flush=True)
            idx = np.searchsorted(pick, sub)
            truth_err = {}
            for dt in wl.dts:
                truth = m_or.integrate(states[sub], dt, 1e-20, 1e-13, nthreads=threads)[0]
                rec = {"oracle_cold": eq1_error(cold[dt][idx], truth, K, configs.ATOL, configs.RTOL),
                       form: eq1_error(gpu_out[dt][sub], truth, K, configs.ATOL, configs.RTOL)}
                for f in cmp_out:
                    rec[f] = eq1_error(cmp_out[f][dt][idx], truth, K, configs.ATOL, configs.RTOL)
                truth_err[f"{dt:g}"] = rec
            parity["eq1_vs_tight_oracle"] = {"sample": int(len(sub)), "atol": 1e-20, "rtol": 1e-13,
                                             "per_dt": truth_err}
        print("[bench] parity done", flush=True)

    value = n * len(wl.dts) / sec_per_step
    fdesc = FORMS[form]
    factors = "FP32 (FP64 residuals)" if fdesc["variant"] in ("mixed", "block") else "FP64"
    line = {
        "metric": "states integrated/s per global step (dt=1e-6,1e-4 s), learned+FP32-LU vs plain FP64",
        "value": value, "unit": "states/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: synthetic {wl.mech} ({mech.K} species, {mech.R} reversible reactions), "
                               f"{n} PaSR-like states" + (f" (first {n} of {wl.n_states})" if n < wl.n_states else "")
                               + f", one global step at each of {list(wl.dts)} s; form {form}: factors {factors}, "
                               + ("queue bins of predicted step counts, cold starts" if fdesc["predictor"] == "bins"
                                  else f"predictor {fdesc['predictor']}"),
                   "n_states": n, "dts": list(wl.dts), "atol": configs.ATOL, "rtol": configs.RTOL,
                   "form": form, "variant": fdesc["variant"], "autotune": fdesc["autotune"],
                   "predictor": fdesc["predictor"], "factors": factors},
        "per_dt": per_dt,
        "compare": compare,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "pcie_inclusive": pcie,
    }
    if "plain" in compare:
        line["vs_plain_fp64"] = {"headline_states_per_s": value,
                                 "plain_states_per_s": compare["plain"]["per_step_states_per_s"],
                                 "per_dt_ratio": {k: per_dt[k]["states_per_s"] / compare["plain"]["per_dt"][k][
                                     "states_per_s"] for k in per_dt}}
    print(json.dumps(line), flush=True)
    mech.close()
    return 0


def jac_ratio(args, wl, states, y, out, stream, path) -> int:
    """R_FD / R_AJ: runtime with the forward-difference Jacobian over runtime
    with the analytical one, per global step size (the paper's Fig. 6 ratio),
    for the lane-per-state kernel (the paper's per-thread pattern), the
    wavefront-cooperative kernel and the CPU oracle."""
    import numpy as np
    import torch
    from paper_1607_03884_amd import Mechanism, configs
    n = len(states)
    res = {"n_states": n, "gpu": {}, "cpu": {}}
    for variant in [v for v in args.ratio_variants.split(",") if v]:
        for jac in ("analytical", "fd"):
            m = Mechanism(path)
            m.set_option("variant", variant)
            m.set_option("jacobian", jac)
            for dt in wl.dts:
                m.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)   # warm-up
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                m.integrate(y, dt, configs.ATOL, configs.RTOL, y_out=out, stream=stream)
                b.record(stream)
                torch.cuda.synchronize()
                st = m.stats()
                res["gpu"].setdefault(variant, {}).setdefault(f"{dt:g}", {})[jac] = {
                    "ms": a.elapsed_time(b), "f_evals_per_state": st["f_evals"] / n,
                    "jac_evals_per_state": st["jac_evals"] / n, "steps_per_state": st["steps"] / n}
                print(f"[bench] {variant} {jac} dt={dt:g}: {a.elapsed_time(b):.1f} ms", flush=True)
            m.close()
    for variant, per in res["gpu"].items():
        for dtk, r in per.items():
            r["ratio_fd_over_aj"] = r["fd"]["ms"] / r["analytical"]["ms"]
    if not args.no_cpu_baseline:
        import oracle
        from oracle import default_opts
        m_or = oracle.Mech(path)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        rng = np.random.default_rng(4242)
        sample = states[np.sort(rng.choice(n, min(args.cpu_sample, n), replace=False))]
        for dt in wl.dts:
            t = {}
            for jac, fd in (("analytical", 0), ("fd", 1)):
                c0 = time.perf_counter()
                m_or.integrate(sample, dt, configs.ATOL, configs.RTOL, opts=default_opts(fd_jac=fd), nthreads=threads)
                t[jac] = time.perf_counter() - c0
            res["cpu"][f"{dt:g}"] = {"s": t, "ratio_fd_over_aj": t["fd"] / t["analytical"]}
            print(f"[bench] CPU oracle dt={dt:g}: FD/AJ {t['fd'] / t['analytical']:.2f}", flush=True)
        res["cpu_sample"] = f"{len(sample)} states drawn uniformly (seed 4242), {threads} threads, {cpu_model()}"
    print(json.dumps({"metric": "runtime ratio, finite-difference / analytical Jacobian (Radau IIA)",
                      "workload": f"{wl.name}: {wl.mech}, {n} states, dts {list(wl.dts)}", "fd_jacobian_ratio": res}),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
