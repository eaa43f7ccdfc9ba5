#!/usr/bin/env python3
"""Benchmark of the SamBaTen batch update on one MI355X.

Workloads (--workload; all inputs seeded and synthetic, resident in HBM
before timing, the model starting from the generator's factors):

  dense2000   (default; the largest single-GPU workload) dense FP32 2000 x 2000
              x 1000, rank-20 U[0,1) CP model plus 1% Gaussian noise generated on
              the GPU, batches of 100 slices, s = 5, r = 10, 30 sweeps: batched
              BF16 (matrix cores) = `value`, batched FP32 and plain FP32 beside it.
  dense500    dense FP32 500 x 500 x 500, rank-10 U[0,1) CP model plus 1% noise,
              update batches of 50 frontal slices; s = 5, r = 10, 30 ALS sweeps.
              `value` is the batched FP32 schedule; the plain FP32 schedule and
              the batched BF16 (matrix-core) path run on the same batches.
  getrank400  GetRank on rank-deficient updates (Sec. 3.2; Q3 of Sec. 4): dense
              FP32 400 x 400 x 400 of true rank 3 (N(0,1) factors, nearly
              orthogonal components) with a rank-5 model (the three generating
              components and two small ones the data do not hold), batches of
              50, s = 2, r = 4: the
              update with GetRank (`value`) and without, factor match score of
              each against the generating components.
  getrank_sparse  the same on COO summaries: 2000 x 2000 x 400 of true rank 3
              whose factor columns are nonzero on 5% of their rows (about
              5.7e5 nonzeros in the initial block, 5.6e4 per batch), a rank-5
              model, batches of 40, s = 2, r = 4.
  dense4d     dense FP32 order-4 120 x 120 x 120 x 120 (the last mode grows),
              rank-10 U[0,1) CP model plus 1% noise, batches of 12 slices; s = 4
              on every mode, r = 10, 30 ALS sweeps.  `value` is the FP32 path; the
              FP64 path beside it; recompute: CP-ALS of the whole grown tensor.
  coo4d       order-4 COO 500 x 500 x 500 x 100 with 1e7 nonzeros (Zipf 1.1
              popularity over every leading mode, rank-10 nonnegative model),
              batches of 10 slices with 1e6 nonzeros, s = 4 per mode, r = 10,
              30 sweeps, from the model of the GPU's initial CP-ALS.
  sparse100k  COO 100000^3 with about 1e8 nonzeros (Zipf 1.1 popularity,
              rank-10 nonnegative model), batches of 1000 slices with about
              1e6 nonzeros, s = 10, r = 10, 30 sweeps.
  serve16     16 resident dense tensors of random shapes and ranks, 512 update
              requests of 5-100 slices through the serving loop (4 slots):
              closed loop (all requests queued at once: `value`), then open
              loop with Poisson arrivals at 80% of the closed-loop request
              rate (p50/p99 of completion minus arrival), and the same
              requests one at a time on one slot for comparison.  Tensor data
              are generated on the GPU (CP model plus 1% noise); a request of
              K slices appends the first K of its tensor's 100-slice pool.

A step is one update (importance, sampling, summaries, CP-ALS on the r
summaries, matching, row solve, append) of one batch.  The timed region is
exactly --steps consecutive updates of one tensor, after --warmup updates of a
throwaway copy; `value` is updated slices per second over it.  Per-update
latency p50/p99 comes from --latency-runs repetitions of the whole sequence.

roofline: the dominant kernel (by summed device time over the timed updates),
timed with HIP events recorded on the stream it runs on (every fifth timed
launch carries an event pair, so the timing costs the update little), with its algorithmic
bytes per launch (summary elements read once, factor rows, outputs written
once) against 8 TB/s; `traffic` comes from hardware counters of the same
kernel when a committed measurement of the current kernel sources exists.
cpu_baseline (dense workloads): the CPU FP64 oracle on the first update of the
same data (its repetitions and BLAS on the host threads), and
vs_oracle_first_update: the fit of every GPU path after that same update
against the oracle's (|dfit|) and the relative error of its new rows of C.
recompute (dense workloads):
CP-ALS of the whole grown tensor on the GPU and the relative fitness of the
incremental result against it (Sec. 4.2); fms_truth: the factor match score
(Sec. 4.4, on the GPU) of the final model against the generating components.
getrank_full_rank_data (dense workloads, --getrank-runs > 0): the batched FP32
update with GetRank (Sec. 3.2) on every summary of this full-rank data.
persistent (dense and sparse workloads): the main path with persistent summaries (samples of the first update kept, warm-started summary
CP-ALS; the old part of each summary kept, so only the new slices are read).

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload dense2000]
"""

import argparse
import hashlib
import json
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "dense500": dict(kind="dense", I=500, J=500, K0=500, Kn=50, R=10, s=5, r=10, iters=30,
                     seed=2, noise=0.01,
                     desc="dense FP32 500x500x500 + 50-slice batches, rank 10, s=5, r=10, "
                          "30 ALS sweeps"),
    "dense2000": dict(kind="dense", I=2000, J=2000, K0=1000, Kn=100, R=20, s=5, r=10,
                      iters=30, seed=5, noise=0.01, device_data=True,
                      desc="dense 2000x2000x1000 + 100-slice batches, rank 20, s=5, r=10, "
                           "30 ALS sweeps, BF16 summaries on the matrix cores"),
    "serve16": dict(kind="serve", tensors=16, requests=512, seed=4, s=5, r=10, iters=30,
                    slots=4, load=0.8,
                    desc="serving: 16 resident dense FP32 tensors (I, J uniform in [200, 2000], "
                         "K0 in [100, 1000], rank 5-20), 512 update requests of 5-100 slices, "
                         "s=5, r=10, 30 ALS sweeps, 4 concurrent slots"),
    "getrank400": dict(kind="getrank", I=400, J=400, K0=400, Kn=50, R=5, R_true=3, s=2, r=4,
                       iters=30, seed=7, noise=0.01,
                       desc="GetRank (Sec. 3.2): dense FP32 400x400x400 of true rank 3 "
                            "(N(0,1) factors) with a rank-5 model, 50-slice batches, s=2, r=4, "
                            "30 ALS sweeps; the update with and without GetRank"),
    "getrank_sparse": dict(kind="getrank", fmt="coo", I=2000, J=2000, K0=400, Kn=40, R=5,
                           R_true=3, s=2, r=4, iters=30, seed=8, support=0.05, noise=1e-3,
                           desc="GetRank (Sec. 3.2) on COO summaries: 2000x2000x400 sparse "
                                "tensor of true rank 3 (factor columns nonzero on 5% of their "
                                "rows) with a rank-5 model, 40-slice batches, s=2, r=4, 30 ALS "
                                "sweeps; the update with and without GetRank"),
    "dense4d": dict(kind="nd", dims=(120, 120, 120), K0=120, Kn=12, R=10, s=4, r=10, iters=30,
                    seed=6, noise=0.01,
                    desc="dense FP32 order-4 120x120x120x120 + 12-slice batches along the last "
                         "mode, rank 10, s=4 per mode, r=10, 30 ALS sweeps"),
    "coo4d": dict(kind="nd_coo", dims=(500, 500, 500), K0=100, Kn=10, R=10, s=4, r=10,
                  iters=30, seed=9, nnz0=10_000_000, nnz_b=1_000_000,
                  desc="sparse COO order-4 500x500x500x100 with 1e7 nonzeros (Zipf 1.1 "
                       "popularity per leading mode) + 10-slice batches of 1e6, rank 10, s=4 "
                       "per mode, r=10, 30 ALS sweeps, fitted initial model"),
    "sparse100k": dict(kind="coo", I=100000, J=100000, K0=100000, Kn=1000, R=10, s=10,
                       r=10, iters=30, seed=3, nnz0=100_000_000, nnz_b=1_000_000,
                       desc="sparse COO 100000^3 with 1e8 nonzeros + 1000-slice batches of "
                            "1e6 nonzeros, rank 10, s=10, r=10, 30 ALS sweeps"),
}
HBM_PEAK_GBS = 8000.0
# the timed updates record kernel events on every PROF_EVERY-th timed launch:
# an event pair on every launch costs about a tenth of a 500^3 update
PROF_EVERY = 5
MFMA_BF16_PEAK_TFS = 2500.0

KIND_NAMES = ("mttkrp_contract_c", "mttkrp_third_mode", "row_solve", "gather", "coo_mttkrp",
              "update")


# launch shapes of the matrix-core path, in the library's choice order: rows
# tiles per wavefront of pass W, K steps in flight of the mode-3 pass, slice
# groups per gathering thread
PW_TILES, P3_STEPS, GATHER_GROUPS = (4, 2, 1), (2, 1, 4), (8, 4, 16)
# the launch-shape table the benchmark loads (decided on MI355X by a run of
# this script with --tune-save)
TILE_CACHE = os.path.join(ROOT, "paper_1709_00668_amd", "tiles_gfx950.txt")


def tuned_shapes(sbt, R, n12, r, store_prec=1):
    """Shapes the tuner holds for a summary shape: {0: gather, 1: pass W,
    2: mode 3} -> choice (a kernel missing from the dict runs shape 0)."""
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "shapes.txt")
        sbt.autotune_save(path)
        rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    got = {}
    for a in rows:
        k, sh, c = int(a[1]), [int(x) for x in a[2:6]], int(a[6])
        if k in (1, 2) and sh == [R, n12, r, 0]:
            got[k] = c
        elif k == 0 and sh == [store_prec, n12, r, 0]:
            got[k] = c
    return got


def kernel_of(step, path, R, coo_row_nnz=0.0, n1_third=0, tiles=None):
    """HIP kernel behind a timed launch kind (coo_row_nnz: summary entries per
    row, which picks the sparse kernel's lanes per unit; n1_third: first extent
    of the order-N third-mode view, which picks the fused pass's vector width;
    tiles: the tuner's launch shapes of the matrix-core path)."""
    tiles = tiles or {}
    rp = (R + 3) // 4 * 4
    v3 = 4 if n1_third % 4 == 0 and rp <= 16 else (2 if n1_third % 2 == 0 else 1)
    ul = 64 if coo_row_nnz >= 128.0 else 32
    nt = 1 if R <= 16 else 2
    table = {
        "f32": {"mttkrp_contract_c": f"pw_kernel<float, {rp}>",
                "mttkrp_third_mode": f"p3_kernel<float, {rp}, 4, false>",
                "row_solve": f"p3_kernel<float, {rp}, 4, true>",
                "gather": "gather_dense_kernel<float, float>"},
        "bf16": {"mttkrp_contract_c": f"pw_mfma_kernel<{nt}, {PW_TILES[tiles.get(1, 0)]}>",
                 "mttkrp_third_mode": f"p3_mfma_kernel<{nt}, {P3_STEPS[tiles.get(2, 0)]}>",
                 "row_solve": f"p3_mfma_kernel<{nt}, 2> + mode3_finish_kernel",
                 "gather": f"gather_mfma_kernel<float, {GATHER_GROUPS[tiles.get(0, 0)]}>"},
        "coo": {"coo_mttkrp": f"coo_units_kernel<{rp}, {ul}>", "gather": "summary_emit_kernel"},
        "nd_f32": {"mttkrp_contract_c": f"p1s_kernel<float, {rp}, 1>",
                   "mttkrp_third_mode": f"p3_kernel<float, {rp}, {v3}, false>",
                   "row_solve": f"p3_kernel<float, {rp}, {v3}, false>",
                   "gather": "gather_nd_kernel<float, float>"},
    }
    return table.get(path, {}).get(step, step)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def timed_sequence(sbt, torch, fresh, apply_batch, steps, warmup, latency_runs, Kn, truth=None,
                   first=None):
    """Warm-up on a throwaway tensor, then exactly `steps` timed updates with the
    per-kind launch timing on; extra untimed sequences for latency samples.
    truth: the generating model of the grown tensor, scored by FMS (GPU).
    first: a dict that receives the fit and the factors after the first update
    (taken on the warm-up tensor, outside the timed region)."""
    kinds = {"mttkrp_contract_c": sbt.SBT_K_MTTKRP_C, "mttkrp_third_mode": sbt.SBT_K_MTTKRP_AB,
             "row_solve": sbt.SBT_K_ROW_SOLVE, "gather": sbt.SBT_K_GATHER,
             "coo_mttkrp": sbt.SBT_K_COO_MTTKRP, "update": sbt.SBT_K_UPDATE}
    T = fresh()
    for b in range(max(min(warmup, steps), 1 if first is not None else 0)):
        apply_batch(T, b)
        if b == 0 and first is not None:
            first["fit"] = T.fit()
            first["factors"] = T.get_factors()
    T.close()
    torch.cuda.synchronize()
    T = fresh()
    T.profile_enable(True, every=PROF_EVERY)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for b in range(steps):
        ts = time.perf_counter()
        apply_batch(T, b)  # returns when the update is complete
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = {}
    for name in KIND_NAMES:
        n, ms, by = T.profile_read(kinds[name])
        prof[name] = dict(launches=n, total_ms=ms, alg_bytes=by)
    T.profile_enable(False)
    fit = T.fit()
    extra = {}
    if truth is not None:
        extra["fms_truth"] = T.fms(*truth)
        extra["factors"] = T.get_factors()
    T.close()
    for _ in range(max(0, latency_runs - 1)):
        T = fresh()
        torch.cuda.synchronize()
        for b in range(steps):
            ts = time.perf_counter()
            apply_batch(T, b)
            lat.append(time.perf_counter() - ts)
        T.close()
    return dict(slices_per_s=steps * Kn / wall, wall_s=wall, ms_per_step=1e3 * wall / steps,
                p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99),
                latency_samples=len(lat), fit=fit, profile=prof, **extra)


def run_dense(sbt, torch, w, Xd, model, precision, schedule, steps, warmup, latency_runs,
              truth=None, getrank_runs=0, persist=False, first=None):
    I, J, K0, Kn = w["I"], w["J"], w["K0"], w["Kn"]
    cfg = sbt.make_config(w["R"], w["r"], w["iters"], w["s"], w["seed"], precision=precision,
                          schedule=schedule, k_capacity=K0 + steps * Kn, max_batch=Kn,
                          getrank_runs=getrank_runs, persist_summaries=persist)

    def fresh():
        return sbt.Tensor.init_dense(cfg, Xd[:K0], I, J, K0, factors=model)

    def apply_batch(T, b):
        T.update_batch_dense(Xd[K0 + b * Kn:K0 + (b + 1) * Kn], Kn)

    return timed_sequence(sbt, torch, fresh, apply_batch, steps, warmup, latency_runs, Kn,
                          truth=truth, first=first)


CSRC = os.path.join(ROOT, "paper_1709_00668_amd", "csrc")


def _header_defs(text):
    """The definitions a kernel can depend on in a header: comments and
    function declarations removed, whitespace collapsed."""
    text = re.sub(r"//[^\n]*", "", text)
    text = re.sub(r"\b(?:hipError_t|bool|int|size_t|int64_t)\s+\w+\([^;{}]*\)\s*;", "", text)
    return " ".join(text.split())


def kernel_digest(kernel, read=None):
    """Digest of the source file that defines `kernel` (its launch code lives
    there too) and of the definitions in the shared device headers (`.hpp`;
    declarations of other launchers do not count, nor does the host-only
    `autotune.h`, which no kernel source includes): a counter measurement of
    the kernel stays valid while this digest does.  `read(name)` returns a
    source file's text (default: the working tree)."""
    if read is None:
        def read(name):
            with open(os.path.join(CSRC, name)) as f:
                return f.read()
    base = re.match(r"\w+", kernel).group(0)
    pat = re.compile(r"\bvoid\s+" + re.escape(base) + r"\s*\(")
    names = sorted(os.listdir(CSRC))
    home = [n for n in names if n.endswith(".hip") and pat.search(read(n))]
    h = hashlib.sha256()
    for name in home:
        h.update(name.encode() + b"\0" + read(name).encode())
    for name in [n for n in names if n.endswith(".hpp")]:
        h.update(name.encode() + b"\0" + _header_defs(read(name)).encode())
    return h.hexdigest()[:16] if home else None


def committed_traffic(kernel, key):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (profiles/<workload>_traffic.md) taken on the same workload, step count and
    warmup (`key`, so the same launches) and on the kernel's current sources
    (per-kernel digest column)."""
    name = key.split("@")[0]
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"workload key: `([^`]+)`", text)
    if not m or m.group(1) != key:
        return None
    want = kernel_digest(kernel)
    for line in text.splitlines():
        cells = [c.strip().strip("`") for c in line.split("|")]
        if len(cells) > 4 and cells[1] == kernel:
            if cells[-2] != want:
                return None
            try:
                return int(float(cells[-3]))
            except ValueError:
                return None
    return None


def roofline_of(prof, path, R, key, summary_rows=0, n1_third=0, every=PROF_EVERY, tiles=None):
    kernels = {k: v for k, v in prof.items() if k != "update" and v["launches"]}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    d = kernels[dom]
    avg_ms = d["total_ms"] / d["launches"]
    bytes_per_launch = d["alg_bytes"] / d["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    # sparse: 12 B per summary entry; entries per row over all repetitions' rows
    row_nnz = bytes_per_launch / 12.0 / summary_rows if summary_rows else 0.0
    kname = kernel_of(dom, path, R, row_nnz, n1_third, tiles)
    return dict(bound="hbm", kernel=kname, step=dom, achieved=round(achieved, 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=committed_traffic(kname, key),
                avg_launch_us=round(avg_ms * 1e3, 2), alg_bytes_per_launch=int(bytes_per_launch),
                timed_every=every,
                share_of_update_time=round(every * d["total_ms"] / prof["update"]["total_ms"], 3))


def kernels_table(prof):
    return {k: {"launches": v["launches"],
                "avg_us": round(1e3 * v["total_ms"] / max(1, v["launches"]), 2),
                "GB_s": round(v["alg_bytes"] / max(1e-12, v["total_ms"] * 1e-3) / 1e9, 1)}
            for k, v in prof.items() if v["launches"]}


def path_summary(res):
    return {"value": round(res["slices_per_s"], 2), "unit": "slices/s",
            "ms_per_step": round(res["ms_per_step"], 3), "p50_ms": round(res["p50_ms"], 3),
            "p99_ms": round(res["p99_ms"], 3), "fit": round(res["fit"], 6)}


def host_threads():
    """Host threads the oracle may use: the machine's CPU share (OMP_NUM_THREADS
    there), at most 16."""
    return max(1, min(16, int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)))


def oracle_first_update(w, X, model, log):
    """The CPU FP64 oracle on the first update of the same data: X is the host
    (I, J, K0 + Kn) tensor; its r repetitions (independent, Sec. 3.1) and its
    blocks of slices run on the host threads.  Returns (cpu_baseline entry,
    oracle fit after the update, oracle C rows of the new slices)."""
    from oracle import sambaten as osb
    K0, Kn = w["K0"], w["Kn"]
    threads = host_threads()
    cfg = osb.Config(rank=w["R"], reps=w["r"], als_iters=w["iters"], sample_factor=w["s"],
                     seed=w["seed"], k_capacity=K0 + Kn, workers=threads)
    t0 = time.perf_counter()
    ora = osb.OracleTensor(cfg, osb.DENSE, (w["I"], w["J"], K0), X0=X[:, :, :K0],
                           factors=model)
    log(f"# oracle: importance of the {K0} initial slices ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    ora.update(X[:, :, K0:K0 + Kn])
    dt = time.perf_counter() - t0
    log(f"# oracle: first update in {dt:.1f} s")
    t0 = time.perf_counter()
    fit = ora.fit()
    log(f"# oracle: fit {fit:.6f} over {K0 + Kn} slices ({time.perf_counter() - t0:.1f} s)")
    cpu = dict(value=round(Kn / dt, 3), unit="slices/s", cores=threads, kind="oracle",
               fit_after=round(fit, 6), seconds=round(dt, 2),
               sample=f"the first update ({Kn} slices, all r={w['r']} repetitions, "
                      f"{w['iters']} ALS sweeps) of the same data, repetitions and BLAS on "
                      f"{threads} host threads")
    return cpu, fit, ora.C[K0:K0 + Kn].copy()


def base_line(args, w, b, dtype):
    cfg = {"workload": w["desc"]}
    for k in ("I", "J", "K0", "Kn", "R", "s", "r", "iters"):
        cfg[{"Kn": "batch", "R": "rank", "iters": "als_iters"}.get(k, k)] = w[k]
    return {
        "metric": "updated slices/sec (p50/p99 update latency, the plain schedule and the "
                  "other precision alongside, at equal fit)",
        "value": round(b["slices_per_s"], 2),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(b["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": cfg,
        "p50_ms": round(b["p50_ms"], 3),
        "p99_ms": round(b["p99_ms"], 3),
        "latency_samples": b["latency_samples"],
        "fit": round(b["fit"], 6),
    }


def bench_dense(args, sbt, torch, synth, log):
    name = args.workload
    w = WORKLOADS[name]
    steps = args.steps
    I, J, K0, Kn = w["I"], w["J"], w["K0"], w["Kn"]
    K = K0 + steps * Kn
    gen = synth.DenseCP(I, J, K, w["R"], seed=w["seed"], noise=w["noise"], dtype=np.float32)
    t0 = time.perf_counter()
    if w.get("device_data"):
        # generated on the GPU (a tensor of this size takes minutes on the host);
        # the oracle reads the same bytes copied back
        Xd = torch.empty((K, J, I), dtype=torch.float32, device="cuda")  # column-major (I,J,K)
        gen.fill_device(torch, Xd)
        torch.cuda.synchronize()
        Xkji = None
    else:
        Xkji = np.empty((K, J, I), dtype=np.float32)  # memory = column-major (I, J, K)
        gen.fill_slices_kji(Xkji, 0, K)
        Xd = torch.from_numpy(Xkji).cuda()
    log(f"# data ready: {I}x{J}x{K} fp32, {4 * I * J * K / 1e9:.2f} GB on device "
        f"({time.perf_counter() - t0:.1f} s)")
    model = gen.true_model_prefix(K0)
    truth = gen.true_model_prefix(K)  # generating components of the grown tensor
    main_prec = sbt.SBT_P_F32 if name == "dense500" else sbt.SBT_P_BF16
    order = [("batched_f32", sbt.SBT_P_F32, sbt.SBT_SCHED_BATCHED),
             ("batched_bf16", sbt.SBT_P_BF16, sbt.SBT_SCHED_BATCHED)]
    if main_prec == sbt.SBT_P_BF16:
        order.reverse()
    if not args.no_plain:
        order.append(("plain_f32", sbt.SBT_P_F32, sbt.SBT_SCHED_PLAIN))
    runs, firsts = {}, {}
    for key, prec, sched in order:
        main = prec == main_prec and sched == sbt.SBT_SCHED_BATCHED
        lr = args.latency_runs if main else max(1, min(args.latency_runs, 2))
        # the state after the first update, for the comparison with the oracle
        first = None if args.no_cpu_baseline else firsts.setdefault(key, {})
        runs[key] = run_dense(sbt, torch, w, Xd, model, prec, sched, steps, args.warmup, lr,
                              truth=truth if main else None, first=first)
        log(f"# {key}: {runs[key]['slices_per_s']:.1f} slices/s, fit {runs[key]['fit']:.6f}"
            + (f" (after the first update {first['fit']:.6f})" if first else ""))
    main = "batched_f32" if main_prec == sbt.SBT_P_F32 else "batched_bf16"
    b = runs[main]
    path = "f32" if main == "batched_f32" else "bf16"
    line = base_line(args, w, b, path)
    n12 = -(-I // w["s"]) * -(-J // w["s"])
    tiles = tuned_shapes(sbt, w["R"], n12, w["r"]) if path == "bf16" else None
    line["roofline"] = roofline_of(b["profile"], path, w["R"],
                                   f"{name}@steps{steps}w{args.warmup}", tiles=tiles)
    if path == "bf16":
        line["launch_shapes"] = {
            "source": args.tune_cache or "online",
            "pw_mfma_row_tiles": PW_TILES[tiles.get(1, 0)],
            "p3_mfma_steps_in_flight": P3_STEPS[tiles.get(2, 0)],
            "gather_slice_groups": GATHER_GROUPS[tiles.get(0, 0)]}
        # useful matrix-core work of the mode-3 pass: 2 |Z| R flops per summary
        pr = b["profile"]["mttkrp_third_mode"]
        if pr["launches"]:
            Kp_mean = (w["K0"] + Kn * (steps - 1) / 2.0) / w["s"] + Kn
            flops = 2.0 * w["r"] * (I / w["s"]) * (J / w["s"]) * Kp_mean * w["R"]
            tfs = flops / (pr["total_ms"] / pr["launches"] * 1e-3) / 1e12
            line["roofline"]["mfma_useful_tflops"] = round(tfs, 2)
            line["roofline"]["mfma_frac"] = round(tfs / MFMA_BF16_PEAK_TFS, 5)
    if not args.no_recompute:
        # the paper's baseline for accuracy (Sec. 4.2): CP-ALS recomputed on the whole grown
        # tensor (on the GPU), and relative fitness = ||X - X_sambaten|| / ||X - X_recomputed||
        cfg = sbt.make_config(w["R"], w["r"], w["iters"], w["s"], w["seed"],
                              precision=sbt.SBT_P_F32, k_capacity=K + 1, max_batch=Kn,
                              init_iters=args.recompute_iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = sbt.Tensor.init_dense(cfg, Xd, I, J, K)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fr = T.fit()
        fms_rt = T.fms(*truth)
        fms_sr = T.fms(*b["factors"])
        T.close()
        line["recompute"] = {"fit": round(fr, 6), "seconds": round(dt, 4),
                             "als_sweeps": args.recompute_iters,
                             "relative_fitness": round((1.0 - b["fit"]) / max(1e-12, 1.0 - fr), 4),
                             "fms_vs_sambaten": round(fms_sr, 4),
                             "fms_truth": round(fms_rt, 4)}
        log(f"# recompute CP-ALS: fit {fr:.6f} in {dt:.2f} s, FMS vs truth {fms_rt:.4f}")
    if "fms_truth" in b:
        line["fms_truth"] = round(b["fms_truth"], 4)
    if args.getrank_runs > 0:
        # GetRank (Sec. 3.2) on every summary: ranks 1..R, getrank_runs CP runs each.  This
        # data is full rank R, where core consistency picks much lower ranks: a timing of
        # the GetRank path, not an accuracy result (the rank-deficient workload is that)
        g = run_dense(sbt, torch, w, Xd, model, sbt.SBT_P_F32, sbt.SBT_SCHED_BATCHED, steps,
                      min(args.warmup, 1), 1, truth=truth, getrank_runs=args.getrank_runs)
        line["getrank_full_rank_data"] = dict(path_summary(g), runs=args.getrank_runs,
                                              fms_truth=round(g["fms_truth"], 4))
        log(f"# getrank: {g['slices_per_s']:.1f} slices/s, fit {g['fit']:.6f}")
    if not args.no_persist:
        # persistent summaries: the first update's samples kept, warm-started summary CP-ALS
        first = None if args.no_cpu_baseline else firsts.setdefault("persistent", {})
        p = run_dense(sbt, torch, w, Xd, model, main_prec, sbt.SBT_SCHED_BATCHED, steps,
                      args.warmup, 1, truth=truth, persist=True, first=first)
        line["persistent"] = dict(path_summary(p), fms_truth=round(p["fms_truth"], 4))
        log(f"# persistent summaries: {p['slices_per_s']:.1f} slices/s, fit {p['fit']:.6f}")
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the first update of the same data, and every GPU path's fit and new
        # rows after that update against it
        t0 = time.perf_counter()
        if Xkji is None:
            Xkji = Xd[:K0 + Kn].cpu().numpy()
        Xh = Xkji.transpose(2, 1, 0)[:, :, :K0 + Kn]   # (I, J, K) column-major view
        log(f"# host copy of the first {K0 + Kn} slices ({time.perf_counter() - t0:.1f} s)")
        cpu, fit_o, cnew_o = oracle_first_update(w, Xh, model, log)
        par = {"oracle_fit": round(fit_o, 6), "paths": {}}
        for key, f in firsts.items():
            cnew = f["factors"][2][K0:K0 + Kn]
            par["paths"][key] = {
                "fit": round(f["fit"], 6), "abs_dfit": float(f"{abs(f['fit'] - fit_o):.3g}"),
                "c_new_rel_err": float(f"{np.linalg.norm(cnew - cnew_o) / np.linalg.norm(cnew_o):.3g}")}
        par["max_abs_dfit"] = max(v["abs_dfit"] for v in par["paths"].values())
        line["vs_oracle_first_update"] = par
        log(f"# |dfit| against the oracle after the first update: "
            + ", ".join(f"{k} {v['abs_dfit']:.2e}" for k, v in par["paths"].items()))
    line["cpu_baseline"] = cpu
    for key in runs:
        if key != main:
            line[key] = path_summary(runs[key])
    if "plain_f32" in runs:
        line["over_plain_f32"] = round(b["slices_per_s"] / runs["plain_f32"]["slices_per_s"], 3)
    line["kernels"] = kernels_table(b["profile"])
    return line


def bench_getrank(args, sbt, torch, synth, log):
    """Rank-deficient updates (Sec. 3.2, Q3 of Sec. 4): the data hold R_true < R
    components, the model R (the generating components of the initial block
    and R - R_true small components the data do not hold).  The update
    with GetRank (one CP run per candidate rank, threshold 90) against the one
    without, on the same batches: factor match score against the generating
    components (padded with zero components to rank R: those pairs score 0, so
    R_true / R is the best possible score) and fit.  Dense FP32 tensors, or
    COO tensors of sparse support (fmt "coo")."""
    w = WORKLOADS[args.workload]
    coo = w.get("fmt") == "coo"
    steps = args.steps
    I, J, K0, Kn, R = w["I"], w["J"], w["K0"], w["Kn"], w["R"]
    K = K0 + steps * Kn
    pad = R - w["R_true"]
    if coo:
        gen = synth.SparseSupportCP(I, J, K, w["R_true"], w["seed"], support=w["support"],
                                    noise=w["noise"])
        idx0, v0 = gen.entries(0, K0)
        batches = [gen.entries(K0 + b * Kn, K0 + (b + 1) * Kn) for b in range(steps)]
        cols0, vd0 = sbt.coo_to_device(idx0, v0)
        bdev = [sbt.coo_to_device(ix, v) for ix, v in batches]
        nnz_total = len(v0) + sum(len(v) for _, v in batches)
        log(f"# data ready: {len(v0)} + {steps} x ~{len(batches[0][1])} nonzeros")
        Fn = [np.linalg.norm(M, axis=0) for M in gen.F]
        A, B, C = (M / n for M, n in zip(gen.F, Fn))
        lam = Fn[0] * Fn[1] * Fn[2]
        A0, B0, C0, lam0 = A, B, C[:K0], lam
    else:
        gen = synth.DenseCP(I, J, K, w["R_true"], seed=w["seed"], noise=w["noise"],
                            dtype=np.float32, factors="normal")
        Xd = torch.empty((K, J, I), dtype=torch.float32, device="cuda")
        gen.fill_device(torch, Xd)
        torch.cuda.synchronize()
        A, B, C, lam = gen.true_model_prefix(K)
        A0, B0, C0, lam0 = gen.true_model_prefix(K0)
    truth = (np.hstack([A, np.zeros((I, pad))]), np.hstack([B, np.zeros((J, pad))]),
             np.hstack([C, np.zeros((K, pad))]), np.concatenate([lam, np.zeros(pad)]))
    # the model: the generating components of the initial block and R - R_true
    # components that the data do not hold (random unit columns, weight 1% of the
    # smallest true one): an R-component model whose updates have rank R_true
    g = np.random.default_rng(np.random.SeedSequence([w["seed"], 31]))
    extra = [g.standard_normal((n, pad)) for n in (I, J, K0)]
    extra = [M / np.linalg.norm(M, axis=0) for M in extra]
    model = (np.hstack([A0, extra[0]]), np.hstack([B0, extra[1]]), np.hstack([C0, extra[2]]),
             np.concatenate([lam0, np.full(pad, 0.01 * lam0.min())]))

    def make_cfg(runs):
        if coo:
            return sbt.make_config(R, w["r"], w["iters"], w["s"], w["seed"], fmt=sbt.SBT_COO,
                                   precision=sbt.SBT_P_F32, k_capacity=K, max_batch=Kn,
                                   nnz_capacity=nnz_total, getrank_runs=runs)
        return sbt.make_config(R, w["r"], w["iters"], w["s"], w["seed"],
                               precision=sbt.SBT_P_F32, k_capacity=K, max_batch=Kn,
                               getrank_runs=runs)

    def run(runs, first):
        if not coo:
            return run_dense(sbt, torch, w, Xd, model, sbt.SBT_P_F32, sbt.SBT_SCHED_BATCHED,
                             steps, args.warmup, 1, truth=truth, getrank_runs=runs,
                             first=first)
        cfg = make_cfg(runs)

        def fresh():
            return sbt.Tensor.init_coo(cfg, cols0, vd0, len(v0), I, J, K0, model)

        def apply_batch(T, b):
            c, v = bdev[b]
            T.update_batch_coo(c, v, int(v.numel()), Kn)

        return timed_sequence(sbt, torch, fresh, apply_batch, steps, args.warmup, 1, Kn,
                              truth=truth, first=first)

    if coo:
        T0 = sbt.Tensor.init_coo(make_cfg(0), cols0, vd0, len(v0), I, J, K0, model)
    else:
        T0 = sbt.Tensor.init_dense(make_cfg(0), Xd[:K0], I, J, K0, factors=model)
    init_fit = T0.fit()
    T0.close()
    log(f"# rank-{R} model of rank-{w['R_true']} data: fit {init_fit:.6f}")
    out, firsts = {}, {}
    for name, runs in (("without", 0), ("with", 1)):
        first = None if args.no_cpu_baseline else firsts.setdefault(name, {})
        res = run(runs, first)
        out[name] = dict(path_summary(res), fms_truth=round(res["fms_truth"], 4))
        log(f"# {name} GetRank: {res['slices_per_s']:.1f} slices/s, fit {res['fit']:.6f}, "
            f"FMS vs truth {res['fms_truth']:.4f}")
    config = {"workload": w["desc"], "I": I, "J": J, "K0": K0, "batch": Kn, "rank": R,
              "true_rank": w["R_true"], "s": w["s"], "r": w["r"], "als_iters": w["iters"],
              "getrank_runs": 1, "getrank_threshold": 90.0}
    if coo:
        config["nnz0"] = len(v0)
        config["nnz_batch"] = int(np.mean([len(v) for _, v in batches]))
    line = {
        "metric": "updated slices/sec with GetRank on rank-deficient data (factor match score "
                  "against the generating components and fit, with and without GetRank)",
        "value": out["with"]["value"], "unit": "slices/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": out["with"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": config,
        "fms_truth_best_possible": round(w["R_true"] / R, 4),
        "with_getrank": out["with"], "without_getrank": out["without"],
        "initial_fit": round(init_fit, 6), "roofline": None, "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle with GetRank on the first update of the same data
        from oracle import sambaten as osb
        ocfg = osb.Config(rank=R, reps=w["r"], als_iters=w["iters"], sample_factor=w["s"],
                          seed=w["seed"], k_capacity=K0 + Kn, getrank_runs=1,
                          nnz_capacity=(len(v0) + len(batches[0][1])) if coo else None,
                          workers=host_threads())
        if coo:
            ora = osb.OracleTensor(ocfg, osb.COO, (I, J, K0), coo0=(idx0, v0), factors=model)
            t0 = time.perf_counter()
            d = ora.update(coo=(batches[0][0], batches[0][1], Kn), debug=True)
        else:
            Xh = Xd[:K0 + Kn].cpu().numpy().transpose(2, 1, 0)
            ora = osb.OracleTensor(ocfg, osb.DENSE, (I, J, K0), X0=Xh[:, :, :K0],
                                   factors=model)
            t0 = time.perf_counter()
            d = ora.update(Xh[:, :, K0:K0 + Kn], debug=True)
        dt = time.perf_counter() - t0
        fo = ora.fit()
        line["cpu_baseline"] = {"value": round(Kn / dt, 3), "unit": "slices/s",
                                "cores": host_threads(), "kind": "oracle",
                                "sample": f"the first update with GetRank ({Kn} slices, "
                                          f"r={w['r']}) of the same data, {dt:.1f} s",
                                "fit_after": round(fo, 6),
                                "rnew": [int(r["Rnew"]) for r in d["reps"]]}
        f = firsts["with"]
        line["vs_oracle_first_update"] = {"abs_dfit": float(f"{abs(f['fit'] - fo):.3g}")}
        log(f"# oracle with GetRank: R_new {line['cpu_baseline']['rnew']}, fit {fo:.6f} "
            f"(GPU {f['fit']:.6f})")
    return line


def cpu_baseline_nd(w, X, model, updates):
    """The CPU FP64 N-mode oracle on the first `updates` updates of the workload."""
    from oracle import nmode
    K0, Kn = w["K0"], w["Kn"]
    N = len(w["dims"]) + 1
    cfg = nmode.Config(rank=w["R"], reps=w["r"], als_iters=w["iters"], sample_factor=w["s"],
                       seed=w["seed"], order=N, k_capacity=K0 + updates * Kn)
    ora = nmode.OracleTensorN(cfg, X[..., :K0], factors=model[0], lam=model[1])
    t0 = time.perf_counter()
    for b in range(updates):
        ora.update(X[..., K0 + b * Kn:K0 + (b + 1) * Kn])
    dt = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return dict(value=round(updates * Kn / dt, 3), unit="slices/s", cores=int(threads),
                kind="oracle", sample=f"the first {updates} update(s) ({Kn} slices each, "
                                      f"r={w['r']}, {w['iters']} ALS sweeps) of the same "
                                      f"workload, {dt:.1f} s")


def bench_nd(args, sbt, torch, synth, log):
    name = args.workload
    w = WORKLOADS[name]
    steps = args.steps
    dims, K0, Kn, R = tuple(w["dims"]), w["K0"], w["Kn"], w["R"]
    N = len(dims) + 1
    K = K0 + steps * Kn
    slice_n = int(np.prod(dims))
    t0 = time.perf_counter()
    gen = synth.DenseCPN(dims + (K,), R, seed=w["seed"], noise=w["noise"], dtype=np.float32)
    X = gen.slices(0, K)
    Xd = torch.from_numpy(X.ravel(order="F")).cuda()  # memory = column-major
    log(f"# data ready: {'x'.join(map(str, dims + (K,)))} fp32, {X.nbytes / 1e9:.2f} GB "
        f"({time.perf_counter() - t0:.1f} s)")
    model = gen.true_model_prefix(K0)

    def run(prec, lr):
        cfg = sbt.make_config(R, w["r"], w["iters"], 1, w["seed"], precision=prec,
                              k_capacity=K, max_batch=Kn)
        Xp = Xd.double() if prec == sbt.SBT_P_F64 else Xd  # BF16 summaries: FP32 store

        def fresh():
            return sbt.TensorN.init_dense_nd(cfg, Xp[:K0 * slice_n], dims + (K0,), w["s"],
                                             factors=model[0], lam=model[1])

        def apply_batch(T, b):
            T.update_batch_dense(Xp[(K0 + b * Kn) * slice_n:(K0 + (b + 1) * Kn) * slice_n], Kn)

        return timed_sequence(sbt, torch, fresh, apply_batch, steps, args.warmup, lr, Kn)

    b = run(sbt.SBT_P_F32, args.latency_runs)
    log(f"# nd fp32: {b['slices_per_s']:.1f} slices/s, fit {b['fit']:.6f}")
    f64 = run(sbt.SBT_P_F64, max(1, min(args.latency_runs, 2)))
    log(f"# nd fp64: {f64['slices_per_s']:.1f} slices/s, fit {f64['fit']:.6f}")
    bf = run(sbt.SBT_P_BF16, max(1, min(args.latency_runs, 2)))
    log(f"# nd bf16 summaries: {bf['slices_per_s']:.1f} slices/s, fit {bf['fit']:.6f}")
    cfg = {"workload": w["desc"], "dims": list(dims), "K0": K0, "batch": Kn, "rank": R,
           "s": w["s"], "r": w["r"], "als_iters": w["iters"]}
    line = {
        "metric": "updated slices/sec (p50/p99 update latency, the FP64 and BF16-summary "
                  "paths alongside)",
        "value": round(b["slices_per_s"], 2), "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(b["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": cfg, "p50_ms": round(b["p50_ms"], 3),
        "p99_ms": round(b["p99_ms"], 3), "latency_samples": b["latency_samples"],
        "fit": round(b["fit"], 6),
    }
    n0 = -(-dims[0] // w["s"])
    line["roofline"] = roofline_of(b["profile"], "nd_f32", R,
                                   f"{name}@steps{steps}w{args.warmup}", n1_third=n0)
    if not args.no_recompute:
        # relative fitness against CP-ALS recomputed on the whole grown tensor (Sec. 4.2)
        cfg_r = sbt.make_config(R, w["r"], w["iters"], 1, w["seed"], precision=sbt.SBT_P_F32,
                                k_capacity=K + 1, max_batch=Kn, init_iters=args.recompute_iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = sbt.TensorN.init_dense_nd(cfg_r, Xd, dims + (K,), w["s"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fr = T.fit()
        T.close()
        line["recompute"] = {"fit": round(fr, 6), "seconds": round(dt, 4),
                             "als_sweeps": args.recompute_iters,
                             "relative_fitness": round((1.0 - b["fit"]) / max(1e-12, 1.0 - fr),
                                                       4)}
        log(f"# recompute CP-ALS: fit {fr:.6f} in {dt:.2f} s")
    # the oracle takes about 2 s per update of this workload on 8 host cores: three
    # times --cpu-updates updates make a sample of about 10 s
    line["cpu_baseline"] = None if args.no_cpu_baseline else \
        cpu_baseline_nd(w, X, model, max(1, min(3 * args.cpu_updates, steps)))
    line["fp64"] = path_summary(f64)
    line["bf16"] = path_summary(bf)
    line["bf16"]["kernels"] = kernels_table(bf["profile"])
    line["kernels"] = kernels_table(b["profile"])
    return line


def bench_nd_coo(args, sbt, torch, synth, log):
    """Order-N COO tensors: the update of the N-mode COO path (FP32 values, FP64
    arithmetic) from a model fitted by its own initial CP-ALS on the GPU."""
    name = args.workload
    w = WORKLOADS[name]
    steps = args.steps
    dims, K0, Kn, R = tuple(w["dims"]), w["K0"], w["Kn"], w["R"]
    K = K0 + steps * Kn
    t0 = time.perf_counter()
    gen = synth.SparseCPN(dims + (K,), R, seed=w["seed"])
    c0, v0 = gen.slices(0, K0, w["nnz0"], 0)
    batches = [gen.slices(K0 + b * Kn, K0 + (b + 1) * Kn, w["nnz_b"], b + 1)
               for b in range(steps)]

    def to_dev(cols, v):
        return [torch.from_numpy(c).cuda() for c in cols], torch.from_numpy(v).cuda()

    d0 = to_dev(c0, v0)
    bdev = [to_dev(c, v) for c, v in batches]
    nnz_total = len(v0) + sum(len(v) for _, v in batches)
    log(f"# data ready: {len(v0)} + {steps} x ~{w['nnz_b']} nonzeros "
        f"({time.perf_counter() - t0:.1f} s)")
    cfg = sbt.make_config(R, w["r"], w["iters"], 1, w["seed"], fmt=sbt.SBT_COO,
                          precision=sbt.SBT_P_F32, k_capacity=K, max_batch=Kn,
                          nnz_capacity=nnz_total, init_iters=max(1, args.coo_init_iters))
    # the initial decomposition: CP-ALS of the initial block on the GPU, run once
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T0 = sbt.TensorN.init_coo_nd(cfg, d0[0], d0[1], dims + (K0,), w["s"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    Us, lam = T0.get_factors_nd()
    init = {"fit": round(T0.fit(), 6), "seconds": round(dt, 3), "als_sweeps": cfg.init_iters}
    T0.close()
    log(f"# initial CP-ALS of {len(v0)} nonzeros: fit {init['fit']:.6f} in {dt:.2f} s")

    def fresh():
        return sbt.TensorN.init_coo_nd(cfg, d0[0], d0[1], dims + (K0,), w["s"], factors=Us,
                                       lam=lam)

    def apply_batch(T, b):
        T.update_batch_coo_nd(bdev[b][0], bdev[b][1], Kn)

    res = timed_sequence(sbt, torch, fresh, apply_batch, steps, args.warmup, args.latency_runs,
                         Kn)
    log(f"# nd coo: {res['slices_per_s']:.1f} slices/s, fit {res['fit']:.6f}")
    cfgl = {"workload": w["desc"], "dims": list(dims), "K0": K0, "batch": Kn, "rank": R,
            "s": w["s"], "r": w["r"], "als_iters": w["iters"], "nnz0": len(v0),
            "nnz_batch": w["nnz_b"]}
    line = {
        "metric": "updated slices/sec (p50/p99 update latency)",
        "value": round(res["slices_per_s"], 2), "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": cfgl, "p50_ms": round(res["p50_ms"], 3),
        "p99_ms": round(res["p99_ms"], 3), "latency_samples": res["latency_samples"],
        "fit": round(res["fit"], 6), "initial_cp_als": init,
    }
    prof = res["profile"]
    kinds = {k: v for k, v in prof.items() if k != "update" and v["launches"]}
    dom = max(kinds, key=lambda k: kinds[k]["total_ms"])
    d = kinds[dom]
    avg_ms = d["total_ms"] / d["launches"]
    by = d["alg_bytes"] / d["launches"]
    kname = {"coo_mttkrp": "mttkrp_coo_nd_kernel", "gather": "summary_emit_nd_kernel"}.get(dom,
                                                                                           dom)
    line["roofline"] = dict(bound="hbm", kernel=kname, step=dom,
                            achieved=round(by / (avg_ms * 1e-3) / 1e9, 1), peak=HBM_PEAK_GBS,
                            unit="GB/s", frac=round(by / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            traffic=committed_traffic(kname, f"{name}@steps{steps}w{args.warmup}"),
                            avg_launch_us=round(avg_ms * 1e3, 2), alg_bytes_per_launch=int(by),
                            timed_every=PROF_EVERY,
                            share_of_update_time=round(PROF_EVERY * d["total_ms"] /
                                                       prof["update"]["total_ms"], 3))
    # the N-mode oracle works on dense arrays: a tensor of 1.25e10 entries per
    # hundred slices is out of its reach
    line["cpu_baseline"] = None
    line["kernels"] = kernels_table(prof)
    return line


def bench_sparse(args, sbt, torch, synth, log):
    name = args.workload
    w = dict(WORKLOADS[name])
    nnz0, nnzb = int(w["nnz0"] * args.nnz_scale), int(w["nnz_b"] * args.nnz_scale)
    steps = args.steps
    I, J, K0, Kn = w["I"], w["J"], w["K0"], w["Kn"]
    t0 = time.perf_counter()
    gen = synth.SparseCP(I, J, K0 + steps * Kn, w["R"], seed=w["seed"])
    cache = None
    if args.data_cache:
        os.makedirs(args.data_cache, exist_ok=True)
        cache = os.path.join(args.data_cache, f"sparse_{w['seed']}_{nnz0}_{nnzb}_{steps}.npz")
    if cache and os.path.exists(cache):
        # the generator's output of an earlier run (same seed, counts and steps)
        z = np.load(cache)
        idx0, v0 = z["idx0"], z["v0"]
        batches = [(z[f"idx{b + 1}"], z[f"v{b + 1}"]) for b in range(steps)]
        gen.last_mean = float(z["last_mean"])
    else:
        idx0, v0 = gen.slices(0, K0, nnz0, block_id=0)
        mean0 = gen.last_mean
        batches = [gen.slices(K0 + b * Kn, K0 + (b + 1) * Kn, nnzb, block_id=b + 1)
                   for b in range(steps)]
        gen.last_mean = mean0
        if cache:
            arrs = {"idx0": idx0, "v0": v0, "last_mean": np.float64(mean0)}
            for b, (ix, v) in enumerate(batches):
                arrs[f"idx{b + 1}"], arrs[f"v{b + 1}"] = ix, v
            np.savez(cache, **arrs)
    model = synth.sparse_model(gen, K0, gen.last_mean)  # the generator's (replaced below)
    cols0, vd0 = sbt.coo_to_device(idx0, v0)
    bdev = [sbt.coo_to_device(ix, v) for ix, v in batches]
    nnz_total = len(v0) + sum(len(v) for _, v in batches)
    log(f"# data ready: {len(v0)} + {steps} x ~{nnzb} nonzeros "
        f"({time.perf_counter() - t0:.1f} s)")
    cfg = sbt.make_config(w["R"], w["r"], w["iters"], w["s"], w["seed"], fmt=sbt.SBT_COO,
                          precision=sbt.SBT_P_F32, k_capacity=K0 + steps * Kn, max_batch=Kn,
                          nnz_capacity=nnz_total, init_iters=max(1, args.coo_init_iters))
    init = None
    if args.coo_init_iters > 0:
        # the initial decomposition is CP-ALS of the initial block on the GPU (run once;
        # every timed tensor starts from its factors)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T0 = sbt.Tensor.init_coo(cfg, cols0, vd0, len(v0), I, J, K0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        model = T0.get_factors()
        init = {"fit": round(T0.fit(), 6), "seconds": round(dt, 3),
                "als_sweeps": args.coo_init_iters}
        T0.close()
        log(f"# initial CP-ALS of {len(v0)} nonzeros: fit {init['fit']:.6f} in {dt:.2f} s")

    def fresh():
        return sbt.Tensor.init_coo(cfg, cols0, vd0, len(v0), I, J, K0, model)

    def apply_batch(T, b):
        c, v = bdev[b]
        T.update_batch_coo(c, v, int(v.numel()), Kn)

    res = timed_sequence(sbt, torch, fresh, apply_batch, steps, args.warmup,
                         args.latency_runs, Kn)
    log(f"# coo: {res['slices_per_s']:.1f} slices/s, fit {res['fit']:.6f}")
    line = base_line(args, w, res, "f32")
    line["config"]["nnz0"] = len(v0)
    line["config"]["nnz_batch"] = nnzb
    line["initial_cp_als"] = init
    line["roofline"] = roofline_of(res["profile"], "coo", w["R"],
                                   f"{name}@{args.nnz_scale:g}@steps{steps}w{args.warmup}",
                                   summary_rows=w["r"] * -(-w["I"] // w["s"]))
    line["cpu_baseline"] = None
    if not args.no_recompute:
        # CP-ALS recomputed on the whole grown tensor (Sec. 4.2): an update with s = 1 and
        # r = 1 whose batch is every slice after the first K0 has the whole tensor as its
        # one summary, so that summary's CP-ALS (--recompute-iters sweeps from U[0,1)
        # factors) is the recompute; its fit comes from a tensor holding all nonzeros
        Kall = K0 + steps * Kn
        cols_all = [torch.cat([bdev[b][0][m] for b in range(steps)]) for m in range(3)]
        cols_all[2] = torch.cat([bdev[b][0][2] + b * Kn for b in range(steps)])
        v_all = torch.cat([bdev[b][1] for b in range(steps)])
        cfg_r = sbt.make_config(w["R"], 1, args.recompute_iters, 1, w["seed"], fmt=sbt.SBT_COO,
                                precision=sbt.SBT_P_F32, k_capacity=Kall, max_batch=Kall - K0,
                                nnz_capacity=nnz_total)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = sbt.Tensor.init_coo(cfg_r, cols0, vd0, len(v0), I, J, K0, model)
        T.update_batch_coo(cols_all, v_all, int(v_all.numel()), Kall - K0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = (T.last_rep(0, sbt.SBT_REP_AP, I), T.last_rep(0, sbt.SBT_REP_BP, J),
               T.last_rep(0, sbt.SBT_REP_CP, Kall), T.last_rep(0, sbt.SBT_REP_LAMP, 1)[0])
        T.close()
        cols_full = [torch.cat([cols0[m], cols_all[m] + (K0 if m == 2 else 0)])
                     for m in range(3)]
        cfg_f = sbt.make_config(w["R"], 1, 1, 1, w["seed"], fmt=sbt.SBT_COO,
                                precision=sbt.SBT_P_F32, k_capacity=Kall + 1, max_batch=1,
                                nnz_capacity=nnz_total)
        T = sbt.Tensor.init_coo(cfg_f, cols_full, torch.cat([vd0, v_all]), nnz_total, I, J, Kall,
                                rec)
        fr = T.fit()
        T.close()
        line["recompute"] = {"fit": round(fr, 6), "seconds": round(dt, 4),
                             "als_sweeps": args.recompute_iters,
                             "relative_fitness": round((1.0 - res["fit"]) / max(1e-12, 1.0 - fr),
                                                       4)}
        log(f"# recompute CP-ALS: fit {fr:.6f} in {dt:.2f} s")
    if not args.no_persist:
        # persistent summaries: the first update's samples kept; each later
        # update scans only its batch for the new slices' entries
        cfg_p = sbt.make_config(w["R"], w["r"], w["iters"], w["s"], w["seed"], fmt=sbt.SBT_COO,
                                precision=sbt.SBT_P_F32, k_capacity=K0 + steps * Kn,
                                max_batch=Kn, nnz_capacity=nnz_total, persist_summaries=True)

        def fresh_p():
            return sbt.Tensor.init_coo(cfg_p, cols0, vd0, len(v0), I, J, K0, model)

        p = timed_sequence(sbt, torch, fresh_p, apply_batch, steps, args.warmup, 1, Kn)
        line["persistent"] = path_summary(p)
        log(f"# coo persistent summaries: {p['slices_per_s']:.1f} slices/s, fit {p['fit']:.6f}")
    line["kernels"] = kernels_table(res["profile"])
    return line


def bench_serve(args, sbt, torch, synth, log):
    w = WORKLOADS["serve16"]
    nt, nreq = w["tensors"], args.serve_requests or w["requests"]
    g = np.random.default_rng(np.random.SeedSequence([w["seed"], 21]))
    Is = g.integers(200, 2001, nt)
    Js = g.integers(200, 2001, nt)
    K0s = g.integers(100, 1001, nt)
    Rs = g.integers(5, 21, nt)
    who = g.integers(0, nt, nreq)
    kns = g.integers(5, 101, nreq)
    grow = np.bincount(who, weights=kns, minlength=nt).astype(np.int64)
    pool_slices = 100
    dev = torch.device("cuda")

    def gen_tensor(i):
        """(X0 + 100-slice pool) on the device as (K, J, I) float32, and the
        model of X0 (unit columns, lambda)."""
        I, J, K0, R = int(Is[i]), int(Js[i]), int(K0s[i]), int(Rs[i])
        gf = np.random.default_rng(np.random.SeedSequence([w["seed"], 22, i]))
        A, B, C = gf.random((I, R)), gf.random((J, R)), gf.random((K0 + pool_slices, R))
        H = (A.T @ A) * (B.T @ B) * (C.T @ C)
        sigma = 0.01 * np.sqrt(H.sum() / (I * J * (K0 + pool_slices)))
        At = torch.from_numpy(A.T.copy()).float().to(dev)      # (R, I)
        Bd = torch.from_numpy(B).float().to(dev)               # (J, R)
        Cd = torch.from_numpy(C).float().to(dev)               # (K, R)
        X = torch.empty((K0 + pool_slices, J, I), dtype=torch.float32, device=dev)
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(w["seed"]) * 1000 + i)
        for k0 in range(0, K0 + pool_slices, 64):
            k1 = min(K0 + pool_slices, k0 + 64)
            blk = torch.matmul(Bd[None, :, :] * Cd[k0:k1, None, :], At)   # (k, J, I)
            blk += sigma * torch.randn(blk.shape, generator=gen, device=dev)
            X[k0:k1] = blk
        nA, nB, nC = (np.linalg.norm(M, axis=0) for M in (A, B, C[:K0]))
        model = (A / nA, B / nB, C[:K0] / nC, nA * nB * nC)
        return X, model

    def fresh_tensors():
        out = []
        for i in range(nt):
            X, model = gen_tensor(i)
            K0 = int(K0s[i])
            cfg = sbt.make_config(int(Rs[i]), w["r"], w["iters"], w["s"], w["seed"] + i,
                                  precision=sbt.SBT_P_F32, k_capacity=K0 + int(grow[i]),
                                  max_batch=pool_slices)
            T = sbt.Tensor.init_dense(cfg, X[:K0], int(Is[i]), int(Js[i]), K0, factors=model)
            pool = X[K0:].clone()
            del X
            torch.cuda.empty_cache()  # hand the generation buffer back for the next store
            out.append((T, pool))
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return out

    max_batch_bytes = int((Is * Js).max()) * pool_slices * 4

    def run(slots, arrivals):
        made = fresh_tensors()
        srv = sbt.Server(slots, slots * max_batch_bytes)
        tickets = []
        t0 = time.perf_counter()
        for q in range(nreq):
            if arrivals is not None:
                d = arrivals[q] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
            T, pool = made[who[q]]
            tickets.append(srv.submit_dense(T, pool[:int(kns[q])], int(kns[q])))
        srv.drain()
        wall = time.perf_counter() - t0
        lat, bad = [], 0
        for tk in tickets:
            state, res, ts, tb, te = srv.poll(tk)
            bad += res != sbt.SBT_OK
            lat.append(te - ts)
        fits = [T.fit() for T, _ in made]
        factors = [T.get_factors() for T, _ in made]
        srv.close()
        for T, pool in made:
            T.close()
        del made
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return dict(slices_per_s=float(kns.sum()) / wall, wall_s=wall,
                    req_per_s=nreq / wall, p50_ms=1e3 * percentile(lat, 50),
                    p99_ms=1e3 * percentile(lat, 99), failed=int(bad),
                    fit_min=float(min(fits)), fit_mean=float(np.mean(fits)), fits=fits,
                    factors=factors)

    def replay(i, fit_gpu, factors_gpu):
        """Tensor i's requests replayed in arrival order through the FP64 oracle on
        the same data (copied from the GPU): its fit and model against the served
        tensor's."""
        from oracle import sambaten as osb
        X, model = gen_tensor(i)
        K0 = int(K0s[i])
        Xh = X.cpu().numpy().transpose(2, 1, 0)  # (I, J, K0 + pool) column-major view
        del X
        torch.cuda.empty_cache()
        ocfg = osb.Config(rank=int(Rs[i]), reps=w["r"], als_iters=w["iters"],
                          sample_factor=w["s"], seed=w["seed"] + i,
                          k_capacity=K0 + int(grow[i]), workers=host_threads())
        t0 = time.perf_counter()
        ora = osb.OracleTensor(ocfg, osb.DENSE, (int(Is[i]), int(Js[i]), K0),
                               X0=Xh[:, :, :K0], factors=model)
        nup = 0
        for q in range(nreq):
            if who[q] == i:
                ora.update(Xh[:, :, K0:K0 + int(kns[q])])
                nup += 1
        fo = ora.fit()
        C = factors_gpu[2]
        return {"tensor": int(i), "I": int(Is[i]), "J": int(Js[i]), "K0": K0,
                "rank": int(Rs[i]), "updates": nup, "slices_added": int(grow[i]),
                "gpu_fit": round(fit_gpu, 6), "oracle_fit": round(fo, 6),
                "abs_dfit": float(f"{abs(fit_gpu - fo):.3g}"),
                "c_rel_err": float(f"{np.linalg.norm(C - ora.C) / np.linalg.norm(ora.C):.3g}"),
                "seconds": round(time.perf_counter() - t0, 1)}

    closed = run(w["slots"], None)
    log(f"# serve closed loop: {closed['slices_per_s']:.1f} slices/s, "
        f"{closed['req_per_s']:.1f} req/s")
    replays = []
    if not args.no_cpu_baseline:
        # the lowest-fit served tensors of moderate size, replayed through the oracle
        order = np.argsort(closed["fits"])
        size = Is * Js * (K0s + grow)
        for i in [int(i) for i in order if size[i] <= args.serve_replay_max][:2]:
            rp = replay(i, closed["fits"][i], closed["factors"][i])
            replays.append(rp)
            log(f"# oracle replay of tensor {i} ({rp['updates']} requests): fit gpu "
                f"{rp['gpu_fit']:.6f} oracle {rp['oracle_fit']:.6f}")
    rate = w["load"] * closed["req_per_s"]
    arrivals = synth.poisson_arrivals(nreq, rate, w["seed"])
    opened = run(w["slots"], arrivals)
    log(f"# serve open loop at {rate:.1f} req/s: p50 {opened['p50_ms']:.1f} ms, "
        f"p99 {opened['p99_ms']:.1f} ms")
    single = run(1, None)
    log(f"# one slot: {single['slices_per_s']:.1f} slices/s")
    line = {
        "metric": "updated slices/sec (p50/p99 update latency under Poisson arrivals, one slot "
                  "alongside, at equal fit)",
        "value": round(closed["slices_per_s"], 2), "unit": "slices/s", "n_gpus": 1,
        "steps": nreq, "warmup": 0, "ms_per_step": round(1e3 * closed["wall_s"] / nreq, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "tensors": nt, "requests": nreq, "s": w["s"],
                   "r": w["r"], "als_iters": w["iters"], "slots": w["slots"],
                   "slices": int(kns.sum())},
        "p50_ms": round(closed["p50_ms"], 3), "p99_ms": round(closed["p99_ms"], 3),
        "open_loop": {"rate_req_per_s": round(rate, 3), "p50_ms": round(opened["p50_ms"], 3),
                      "p99_ms": round(opened["p99_ms"], 3),
                      "slices_per_s": round(opened["slices_per_s"], 2)},
        "one_slot": {"value": round(single["slices_per_s"], 2),
                     "p50_ms": round(single["p50_ms"], 3), "p99_ms": round(single["p99_ms"], 3)},
        "fit_min": round(closed["fit_min"], 6), "fit_mean": round(closed["fit_mean"], 6),
        "oracle_replay": replays,
        "failed_requests": closed["failed"] + opened["failed"] + single["failed"],
        "roofline": None, "cpu_baseline": None,
    }
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--latency-runs", type=int, default=10)
    ap.add_argument("--workload", default="dense2000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-updates", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-recompute", action="store_true",
                    help="skip the CP-ALS recompute of the grown tensor (relative fitness)")
    ap.add_argument("--recompute-iters", type=int, default=100)
    ap.add_argument("--no-persist", action="store_true",
                    help="dense and sparse: skip the persistent-summary variant")
    ap.add_argument("--getrank-runs", type=int, default=0,
                    help="dense: also time the update with GetRank on this full-rank data, "
                         "this many CP runs per candidate rank (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests of the serving workload (default: the workload's 512)")
    ap.add_argument("--serve-replay-max", type=float, default=4e8,
                    help="serving: replay through the oracle the two lowest-fit tensors with "
                         "at most this many entries at their final size")
    ap.add_argument("--coo-init-iters", type=int, default=30,
                    help="sparse: CP-ALS sweeps of the initial decomposition on the GPU "
                         "(0: start from the generator's model)")
    ap.add_argument("--data-cache", default="",
                    help="sparse: keep the generated nonzeros in this folder and reuse them")
    ap.add_argument("--nnz-scale", type=float, default=1.0,
                    help="scale the nonzero counts of the sparse workload")
    ap.add_argument("--tune-cache", default=os.path.relpath(TILE_CACHE, ROOT),
                    help="launch-shape table to load before the run (\"\": none, every "
                         "shape is then decided online by timing the first launches)")
    ap.add_argument("--tune-save", default="",
                    help="write the launch-shape table to this file after the run")
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
    if args.tune_cache and os.path.exists(os.path.join(ROOT, args.tune_cache)):
        sbt.autotune_load(os.path.join(ROOT, args.tune_cache))
    else:
        args.tune_cache = ""  # none: every launch shape is decided online

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if WORKLOADS[args.workload]["kind"] == "coo":
        line = bench_sparse(args, sbt, torch, synth, log)
    elif WORKLOADS[args.workload]["kind"] == "nd":
        line = bench_nd(args, sbt, torch, synth, log)
    elif WORKLOADS[args.workload]["kind"] == "nd_coo":
        line = bench_nd_coo(args, sbt, torch, synth, log)
    elif WORKLOADS[args.workload]["kind"] == "serve":
        line = bench_serve(args, sbt, torch, synth, log)
    elif WORKLOADS[args.workload]["kind"] == "getrank":
        line = bench_getrank(args, sbt, torch, synth, log)
    else:
        line = bench_dense(args, sbt, torch, synth, log)
    if args.tune_save:
        sbt.autotune_save(args.tune_save)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
