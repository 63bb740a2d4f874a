#!/usr/bin/env python3
"""Throughput of the level-scheduled SpTRSV with equation rewriting on one
MI355X.

One step = one solve of each of the three large synthetic systems (3D 7-point
stencil on 128^3, random banded n=1e6 / bandwidth 200, power-law n=4e6 with a
20k-row serial tail), FP64, one right-hand side each, with every input
already resident in HBM.  The rewrite (host analysis) happens before the
timed region, once per matrix, as a factorisation would.  Reported:

  value        solves/s over the timed steps (3 solves per step)
  roofline     algorithmic bytes of the rewritten solves / their measured
               time, against 8 TB/s HBM
  plain        the same kernel on the plain level-set schedule (no rewrite)
  cpu_baseline the serial FP64 CPU oracle on the host, on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))
from gate import TOL, errors  # noqa: E402  (floored componentwise error, see tests/gate.py)

HBM_PEAK_GBS = 8000.0

# Rewrite policy per workload (threshold rule of the paper's thin-level
# rewriting with GPU-sized parameters; see the design doc for how they were chosen).
POLICIES = {
    "stencil3d_128": {"kind": "threshold", "max_width": 4, "max_depth": 64, "max_fill": 0.25},
    "banded_1m": {"kind": "threshold", "max_width": 4, "max_depth": 64, "max_fill": 0.25},
    "powerlaw_4m": {"kind": "threshold", "max_width": 4, "max_depth": 64, "max_fill": 0.25},
}
LARGE = ["stencil3d_128", "banded_1m", "powerlaw_4m"]
SMALL = ["stencil2d_100"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["large", "small"], default="large")
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solve is not sharded across GPUs "
              "(see DESIGN.md, 'How it would shard'); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2103_11445_amd as sp
    import workloads

    sp.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    names = LARGE if args.workload == "large" else SMALL

    systems, plans, plain, bs, xs, host = {}, {}, {}, {}, {}, {}
    for name in names:
        t0 = time.perf_counter()
        s = workloads.config(name)
        t1 = time.perf_counter()
        pol = dict(POLICIES.get(name, {"kind": "threshold"}))
        kind = pol.pop("kind")
        p = sp.Plan(s.row_ptr, s.col_idx, s.val)
        t2 = time.perf_counter()
        p.rewrite(kind, **pol)
        t3 = time.perf_counter()
        p.upload()
        t4 = time.perf_counter()
        systems[name], plans[name] = s, p
        host[name] = {"generate_s": t1 - t0, "analyse_s": t2 - t1, "rewrite_s": t3 - t2,
                      "upload_s": t4 - t3}
        if not args.no_plain:
            plain[name] = sp.Plan(s.row_ptr, s.col_idx, s.val).upload()
        bs[name] = torch.from_numpy(s.b).to(dev)
        xs[name] = torch.empty_like(bs[name])
        info = p.info()
        log(f"[setup] {name}: n={info['n']} nnz={info['nnz']} levels {info['levels']} -> "
            f"{info['levels_rw']} (stages {info['stages']}), entries {info['nnz']} -> "
            f"{info['nnz_rw'] + info['nnz_m']}, tiles {info['tiles']}, host {host[name]}")

    stream = torch.cuda.current_stream()

    def run(plan_set, steps, tag):
        ev = {n: [] for n in names}
        for _ in range(args.warmup):
            for n in names:
                plan_set[n].solve(bs[n], xs[n])
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(steps):
            for n in names:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                plan_set[n].solve(bs[n], xs[n])
                b.record(stream)
                ev[n].append((a, b))
        end.record(stream)
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(end)
        per = {n: float(np.mean([a.elapsed_time(b) for a, b in ev[n]])) for n in names}
        status = {n: plan_set[n].check() for n in names}
        errs = {}
        for n in names:
            s = systems[n]
            ref = refs.setdefault(n, None)
            if ref is None:
                import oracle
                ref = oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
                refs[n] = ref
            errs[n] = errors(xs[n].cpu().numpy(), ref)
        log(f"[{tag}] {steps} steps, {total_ms / steps:.3f} ms/step, per-solve ms "
            f"{ {n: round(v, 4) for n, v in per.items()} }, (strict, floored) err {errs}, status {status}")
        return total_ms, per, errs, status

    refs = {}
    log("[timed] rewritten plans")
    total_ms, per, errs, status = run(plans, args.steps, "rewritten")
    plain_res = None
    if not args.no_plain:
        ps = args.plain_steps or max(2, args.steps // 4)
        log("[timed] plain level-set plans")
        plain_res = run(plain, ps, "plain")

    ms_per_step = total_ms / args.steps
    solves = len(names)
    value = solves * 1000.0 / ms_per_step
    bytes_rw = {n: plans[n].info()["bytes_rw"] for n in names}
    bytes_plain = {n: plans[n].info()["bytes"] for n in names}
    kern_ms = sum(per.values())
    achieved = sum(bytes_rw.values()) / (kern_ms * 1e-3) / 1e9
    matrices = {}
    for n in names:
        i = plans[n].info()
        m = {
            "n": i["n"], "nnz": i["nnz"], "levels": i["levels"], "stages": i["stages"],
            "levels_rw": i["levels_rw"], "entries_rw": i["nnz_rw"] + i["nnz_m"],
            "flops": i["flops"], "flops_rw": i["flops_rw"],
            "ms_per_solve": per[n], "solves_per_s": 1000.0 / per[n],
            "plan_gbps": bytes_rw[n] / (per[n] * 1e-3) / 1e9,
            "effective_gbps": bytes_plain[n] / (per[n] * 1e-3) / 1e9,
            "max_rel_err_strict": errs[n][0], "max_rel_err_floored": errs[n][1],
            "device_status": status[n],
            "policy": POLICIES.get(n), **{k: round(v, 3) for k, v in host[n].items()},
        }
        if plain_res is not None:
            m["plain_ms_per_solve"] = plain_res[1][n]
            m["plain_max_rel_err_floored"] = plain_res[2][n][1]
            m["speedup_vs_plain"] = plain_res[1][n] / per[n]
        matrices[n] = m
    ok = all(e[1] <= TOL for e in errs.values()) and not any(status.values())
    if plain_res is not None:
        ok = ok and all(e[1] <= TOL for e in plain_res[2].values()) and not any(plain_res[3].values())

    cpu = None
    if not args.no_cpu:
        import oracle
        cores = 1
        t_total, count = 0.0, 0
        t0 = time.perf_counter()
        while t_total < args.cpu_seconds:
            for n in names:
                s = systems[n]
                oracle.solve(s.row_ptr, s.col_idx, s.val, s.b)
                count += 1
            t_total = time.perf_counter() - t0
        cpu = {"value": count / t_total, "unit": "solves/s", "cores": cores, "kind": "oracle",
               "sample": f"serial FP64 oracle forward substitution, the same {solves} systems "
                         f"cycled {count // solves} times ({t_total:.1f} s)"}

    out = {
        "metric": "SpTRSV solves/s + achieved HBM GB/s vs plain level-set, rel err <=1e-10",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "stencil3d_128 + banded_1m + powerlaw_4m, FP64 CSR, 1 RHS"
                   if args.workload == "large" else "stencil2d_100, FP64 CSR, 1 RHS",
                   "solves_per_step": solves},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": cpu,
        "parity_ok": ok,
        "plain_levelset": None if plain_res is None else {
            "solves_per_s": solves * 1000.0 * (args.plain_steps or max(2, args.steps // 4)) / plain_res[0],
            "speedup_of_rewrite": (plain_res[0] / (args.plain_steps or max(2, args.steps // 4))) / ms_per_step,
        },
        "matrices": matrices,
    }
    print(json.dumps(out), flush=True)
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
