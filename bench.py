#!/usr/bin/env python3
"""Benchmark of the SamBaTen batch update on one MI355X.

Workload (dense FP32): an existing 500 x 500 x 500 tensor from a rank-10
U[0,1) CP model plus 1% Gaussian noise, then update batches of 50 frontal
slices; sampling factor s = 5, r = 10 repetitions, 30 ALS sweeps per summary.
Inputs are synthetic (seeded generator), resident in HBM before timing; the
model starts from the generator's factors (normalised).

A step is one update (sampling, gather, CP-ALS on the r summaries, matching,
row solve, append) of one 50-slice batch.  The timed region is exactly
--steps consecutive updates of one tensor; `value` is updated slices per
second over it.  Both schedules of the library are timed: "batched" (every
launch covers all repetitions, two summary passes per ALS sweep) gives
`value`; "plain" (one launch sequence per repetition, three passes per sweep)
is reported beside it.  Per-update latency p50/p99 comes from --latency-runs
repetitions of the whole sequence.

The roofline entry is the dominant kernel (by summed device time), timed live
with HIP events on the launch stream, with its algorithmic bytes (summary
elements read once + factor rows + outputs) per launch.  cpu_baseline times
the CPU FP64 oracle on one update of the same workload.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(I=500, J=500, K0=500, Kn=50, R=10, s=5, r=10, iters=30, seed=2, noise=0.01)
HBM_PEAK_GBS = 8000.0


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def run_path(sbt, torch, Xd, model, schedule, steps, warmup, latency_runs, profile):
    w = WORKLOAD
    I, J, K0, Kn = w["I"], w["J"], w["K0"], w["Kn"]
    cfg = sbt.make_config(w["R"], w["r"], w["iters"], w["s"], w["seed"],
                          precision=sbt.SBT_P_F32, schedule=schedule,
                          k_capacity=K0 + steps * Kn, max_batch=Kn)

    def batch(b):
        return Xd[K0 + b * Kn:K0 + (b + 1) * Kn]

    def fresh():
        return sbt.Tensor.init_dense(cfg, Xd[:K0], I, J, K0, factors=model)

    # untimed warmup on a throwaway tensor
    T = fresh()
    for b in range(min(warmup, steps)):
        T.update_batch_dense(batch(b), Kn)
    T.close()
    torch.cuda.synchronize()

    # timed region: exactly `steps` updates
    T = fresh()
    if profile:
        T.profile_enable(True)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for b in range(steps):
        ts = time.perf_counter()
        T.update_batch_dense(batch(b), Kn)  # returns when the update is complete
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = {}
    if profile:
        for kind, name in ((sbt.SBT_K_MTTKRP_C, "mttkrp_contract_c"),
                           (sbt.SBT_K_MTTKRP_AB, "mttkrp_third_mode"),
                           (sbt.SBT_K_ROW_SOLVE, "row_solve"),
                           (sbt.SBT_K_GATHER, "gather"), (sbt.SBT_K_UPDATE, "update")):
            n, ms, by = T.profile_read(kind)
            prof[name] = dict(launches=n, total_ms=ms, alg_bytes=by)
        T.profile_enable(False)
    fit = T.fit()
    T.close()
    # extra untimed sequences for latency percentiles
    for _ in range(max(0, latency_runs - 1)):
        T = fresh()
        torch.cuda.synchronize()
        for b in range(steps):
            ts = time.perf_counter()
            T.update_batch_dense(batch(b), Kn)
            lat.append(time.perf_counter() - ts)
        T.close()
    return dict(slices_per_s=steps * Kn / wall, wall_s=wall, ms_per_step=1e3 * wall / steps,
                p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99),
                latency_samples=len(lat), fit=fit, profile=prof)


# HIP kernel behind each timed launch kind of the batched FP32 schedule
KERNEL_OF = {"mttkrp_contract_c": "pw_kernel<float, 12, 1>",
             "mttkrp_third_mode": "p3_kernel<float, 12, 4, false>",
             "row_solve": "p3_kernel<float, 12, 4, true>",
             "gather": "gather_dense_kernel<float, float>"}


def cpu_baseline(X, model, updates=2):
    """The CPU FP64 oracle on the first `updates` updates of the same workload."""
    from oracle import sambaten as osb
    w = WORKLOAD
    K0, Kn = w["K0"], w["Kn"]
    cfg = osb.Config(rank=w["R"], reps=w["r"], als_iters=w["iters"], sample_factor=w["s"],
                     seed=w["seed"], k_capacity=K0 + updates * Kn)
    ora = osb.OracleTensor(cfg, osb.DENSE, (w["I"], w["J"], K0), X0=X[:, :, :K0],
                           factors=model)
    t0 = time.perf_counter()
    for b in range(updates):
        ora.update(X[:, :, K0 + b * Kn:K0 + (b + 1) * Kn])
    dt = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return dict(value=round(updates * Kn / dt, 3), unit="slices/s", cores=int(threads),
                kind="oracle",
                sample=f"the first {updates} updates ({Kn} slices each, r={w['r']}, "
                       f"{w['iters']} ALS sweeps) of the same workload, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--latency-runs", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic that calibrates hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the update on a single MI355X "
              "(no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1709_00668_amd import sambaten as sbt
    sbt.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = WORKLOAD
    steps = args.steps
    I, J, K0, Kn = w["I"], w["J"], w["K0"], w["Kn"]
    gen = synth.DenseCP(I, J, K0 + steps * Kn, w["R"], seed=w["seed"], noise=w["noise"],
                        dtype=np.float32)
    X = gen.slices(0, K0 + steps * Kn)
    Xd = torch.from_numpy(np.ascontiguousarray(X.transpose(2, 1, 0))).cuda()
    model = gen.true_model_prefix(K0)
    print(f"# data ready: {X.shape} fp32, {X.nbytes / 1e9:.2f} GB on device", file=sys.stderr,
          flush=True)

    res = {}
    res["batched"] = run_path(sbt, torch, Xd, model, sbt.SBT_SCHED_BATCHED, steps, args.warmup,
                              args.latency_runs, profile=True)
    print(f"# batched: {res['batched']['slices_per_s']:.1f} slices/s", file=sys.stderr,
          flush=True)
    if not args.no_plain:
        res["plain"] = run_path(sbt, torch, Xd, model, sbt.SBT_SCHED_PLAIN, steps, args.warmup,
                                args.latency_runs, profile=False)
        print(f"# plain: {res['plain']['slices_per_s']:.1f} slices/s", file=sys.stderr,
              flush=True)

    # dominant kernel by summed device time
    prof = res["batched"]["profile"]
    kernels = {k: v for k, v in prof.items() if k != "update" and v["launches"]}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    d = kernels[dom]
    avg_ms = d["total_ms"] / d["launches"]
    bytes_per_launch = d["alg_bytes"] / d["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", kernel=KERNEL_OF.get(dom, dom), step=dom,
                    achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    avg_launch_us=round(avg_ms * 1e3, 2),
                    alg_bytes_per_launch=int(bytes_per_launch),
                    share_of_update_time=round(d["total_ms"] / prof["update"]["total_ms"], 3))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(X, model)

    b = res["batched"]
    line = {
        "metric": "updated slices/sec (batched path; p50/p99 update latency and the plain "
                  "path alongside, at equal fit)",
        "value": round(b["slices_per_s"], 2),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(b["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense FP32 500x500x500 + 50-slice batches, rank 10, "
                               "s=5, r=10, 30 ALS sweeps",
                   "I": I, "J": J, "K0": K0, "batch": Kn, "rank": w["R"], "s": w["s"],
                   "r": w["r"], "als_iters": w["iters"]},
        "p50_ms": round(b["p50_ms"], 3),
        "p99_ms": round(b["p99_ms"], 3),
        "latency_samples": b["latency_samples"],
        "fit": round(b["fit"], 6),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "plain" in res:
        p = res["plain"]
        line["plain"] = {"value": round(p["slices_per_s"], 2), "unit": "slices/s",
                         "p50_ms": round(p["p50_ms"], 3), "p99_ms": round(p["p99_ms"], 3),
                         "fit": round(p["fit"], 6)}
        line["batched_over_plain"] = round(b["slices_per_s"] / p["slices_per_s"], 3)
    line["kernels"] = {k: {"launches": v["launches"], "avg_us": round(1e3 * v["total_ms"] /
                                                                      max(1, v["launches"]), 2),
                           "GB_s": round(v["alg_bytes"] / max(1e-12, v["total_ms"] * 1e-3) / 1e9,
                                         1)}
                       for k, v in prof.items()}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
