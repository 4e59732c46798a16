#!/usr/bin/env python3
"""Benchmark of LBG codebook design on one MI355X.

One step = one complete LBG run (Algorithm 1: centroid of the training set,
then split / Lloyd iterations until N codevectors) on the 16-image workload:
16 synthetic 512 x 512 pictures (seeds 0..15), 4 x 4 blocks -> M = 262,144
training vectors of dimension L = 16, split from the global mean to N = 256,
stop when the relative distortion change is <= 1e-3.  The training matrix is
resident in HBM before the timed region starts.

Prints one JSON line.  ``value`` is vector-codeword distances per second over
the whole job (sum over every allocation of M * n, divided by the wall time
of the timed steps).  ``roofline`` reports the allocation kernel (the
dominant one) against the FP32 matrix-core peak, from its own HIP-event
durations inside the timed steps; ``cpu_baseline`` times the FP64 CPU oracle
on a bounded sample of the same workload on this host's cores.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

HERE = os.path.dirname(os.path.abspath(__file__))
# Sources of the allocation kernel: counters taken on an older build of them
# are not reported.
ASSIGN_SOURCES = ("paper_0910_4711_amd/csrc/assign_common.h",
                  "paper_0910_4711_amd/csrc/assign.hip")
TRAFFIC_FILE = "profiles/assign_fp32_img16x512x512_b4_traffic.txt"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload():
    import synth
    cfg = synth.CONFIG1
    X = synth.image_training_set(cfg["seeds"], cfg["W"], cfg["H"], cfg["b"])
    return cfg, X


def assign_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ASSIGN_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per allocation launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a plain copy of known size), or None when the summary is
    missing or was taken on other kernel sources."""
    path = os.path.join(HERE, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != assign_source_hash():
        return None
    try:
        return dict(bytes=float(kv["traffic_bytes_per_launch"]),
                    fetch=float(kv["fetch_bytes_per_launch"]),
                    write=float(kv["write_bytes_per_launch"]),
                    algorithmic=float(kv["algorithmic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))


def _instances_worker(args):
    import synth
    n, base, scale, lo = args
    return synth.batched_instances(n, base_seed=base, scale=scale)


def form_batched(args):
    """Batched form: 512 independent LBG instances (M_i ~ U{2048..65536},
    L_i in {16, 64}, N_i in {16..256}, Gaussian-mixture data) trained by
    lbg_train_batched (one persistent allocation launch per round, hipGraph
    rounds, autotuned queue) versus one lbg_train per instance on the same
    GPU.  Prints one JSON line."""
    import concurrent.futures as cf
    import torch
    import paper_0910_4711_amd as P
    n_inst = args.instances
    chunks = [(16, 10_000 + k, args.scale, k) for k in range(0, n_inst, 16)]
    t0 = time.perf_counter()
    inst = []
    with cf.ProcessPoolExecutor(max_workers=min(16, len(chunks))) as ex:
        for k, part in zip(range(0, n_inst, 16), ex.map(_instances_worker, chunks)):
            inst.extend(part[: max(0, min(16, n_inst - k))])
    log(f"generated {len(inst)} instances in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    Xs = [torch.from_numpy(X).to(dev) for X, _ in inst]
    Ns = [N for _, N in inst]
    side = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize(dev)
    with torch.cuda.stream(side):
        res, st0 = P.train_batched(Xs, Ns)  # warm-up (runs the autotuner once)
    side.synchronize()
    log(f"warm-up done (autotuned grab={st0['grab']} grid={st0['grid']}, "
        f"{st0['ms_tune']:.1f} ms of candidate timing)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        with torch.cuda.stream(side):
            res, st = P.train_batched(Xs, Ns)
    side.synchronize()
    t_b = (time.perf_counter() - t0) / args.steps
    dist = st["total_distances"]
    # one lbg_train per instance, same data, same GPU
    ws = None
    for X, N in zip(Xs[:2], Ns[:2]):
        P.train(X, N)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    D_single = []
    for X, N in zip(Xs, Ns):
        C, idx, D, _ = P.train(X, N)
        D_single.append(D)
    torch.cuda.synchronize(dev)
    t_s = time.perf_counter() - t0
    same = sum(1 for r, d in zip(res, D_single) if r[2] == d)
    out = {
        "metric": "batched LBG vector-codeword distances/s",
        "value": dist / t_b,
        "unit": "distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "ms_per_step": t_b * 1e3,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched{len(inst)}_gmm_M2048-65536_L16-64_N16-256",
                   "instances": len(inst), "sum_M": int(sum(x.shape[0] for x in Xs)),
                   "grab": st["grab"], "grid": st["grid"], "graph": st["graph"],
                   "rounds": st["rounds"]},
        "per_instance_launches": {"value": dist / t_s, "ms_total": t_s * 1e3},
        "speedup_vs_per_instance": t_s / t_b,
        "identical_D_to_per_instance": f"{same}/{len(inst)}",
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(X, N, images):
    """The FP64 oracle, as it stands, on the first ``images`` pictures' rows
    with all host cores; distances/s of the full LBG run."""
    import oracle
    rows_per_image = X.shape[0] // 16
    S = X[: images * rows_per_image]
    cores = len(os.sched_getaffinity(0))
    oracle.load()
    t0 = time.perf_counter()
    r = oracle.train(S, N, nthreads=cores)
    t = time.perf_counter() - t0
    dist = int(S.shape[0]) * int(sum(int(n) * (int(i) + 1)
                                     for n, i in zip(r["level_n"], r["level_iters"])))
    return dict(value=dist / t, unit="distances/s", cores=cores, kind="oracle",
                sample=f"full LBG to N={N} on the first {images} of 16 images "
                       f"(M={S.shape[0]}, L={S.shape[1]}), FP64, {t:.2f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-images", type=int, default=16,
                    help="images of the workload the CPU oracle baseline runs on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, metavar="MIB", default=0,
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--form", choices=["batched"], default=None,
                    help="benchmark one of the forms instead of the main workload")
    ap.add_argument("--instances", type=int, default=512, help="instances of --form batched")
    ap.add_argument("--scale", type=float, default=1.0, help="row-count scale of --form batched")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.form == "batched":
        if args.gpus != 1:
            sys.exit("bench.py: the forms run on one GPU")
        form_batched(args)
        return
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on exactly one GPU; --gpus {args.gpus} "
              "is not supported (the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0910_4711_amd as P

    cfg, X = workload()
    M, L = X.shape
    N = cfg["N"]
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    ws = torch.empty(P.load().lbg_workspace_size(P.OP_TRAIN, M, L, N, P.FP32),
                     dtype=torch.uint8, device=dev)
    log(f"workload {cfg['name']}: M={M} L={L} N={N}; device {torch.cuda.get_device_name(dev)}")

    # A dedicated (default-priority) stream: the library replays its Lloyd
    # iterations as hipGraphs on non-default streams.
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize(dev)
    for i in range(args.warmup):
        with torch.cuda.stream(stream):
            P.train(Xd, N, workspace=ws, timing=True)
        stream.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize(dev)
    tot = dict(dist=0, ms_assign=0.0, ms_update=0.0, ms_split=0.0, assigns=0, updates=0,
               fallback=0)
    last = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        with torch.cuda.stream(stream):
            C, idx, D, st = P.train(Xd, N, workspace=ws, timing=True)
        tot["dist"] += st["total_distances"]
        tot["ms_assign"] += st["ms_assign"]
        tot["ms_update"] += st["ms_update"]
        tot["ms_split"] += st["ms_split"]
        tot["assigns"] += st["total_assigns"]
        tot["updates"] += st["total_updates"]
        tot["fallback"] += st["fallback_rows"]
        last = (D, st)
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.4f} s")

    D, st = last
    traffic = measured_traffic()
    flops = 2.0 * L * tot["dist"]  # 2L flops per vector-codeword distance
    assign_s = tot["ms_assign"] / 1e3
    achieved_tf = flops / assign_s / 1e12
    upd_bytes = tot["updates"] * M * (4 * L + 4)  # X rows + cell index per update
    upd_gbs = upd_bytes / (tot["ms_update"] / 1e3) / 1e9 if tot["ms_update"] > 0 else None

    out = {
        "metric": "LBG iteration vector-codeword distances/s",
        "value": tot["dist"] / elapsed,
        "unit": "distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": cfg["name"],
            "M": M, "L": L, "N": N, "thr": 1e-3, "eps_split": 0.01,
            "images": len(cfg["seeds"]), "image_size": [cfg["H"], cfg["W"]], "block": cfg["b"],
            "precision": "fp32 (exact allocation)",
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved_tf,
            "peak": PEAK_FP32_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tf / PEAK_FP32_MFMA_TFLOPS,
            "traffic": traffic["bytes"] if traffic else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
            "kernel": "allocation: assign_kernel<Fp32Screen<16>, vector loads>",
            "launches": tot["assigns"],
            "avg_launch_us": tot["ms_assign"] / tot["assigns"] * 1e3,
            "flops_per_launch_avg": flops / tot["assigns"],
        },
        "update": {
            "bound": "hbm",
            "achieved_gbs": upd_gbs,
            "peak_gbs": PEAK_HBM_GBS,
            "frac": (upd_gbs / PEAK_HBM_GBS) if upd_gbs else None,
            "avg_update_us": tot["ms_update"] / max(1, tot["updates"]) * 1e3,
        },
        "per_step": {
            "assigns": tot["assigns"] // args.steps,
            "updates": tot["updates"] // args.steps,
            "ms_assign": tot["ms_assign"] / args.steps,
            "ms_update": tot["ms_update"] / args.steps,
            "ms_split": tot["ms_split"] / args.steps,
            "fallback_rows": tot["fallback"] // args.steps,
            "level_iters": st["level_iters"],
            "D": D,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle) ...")
        out["cpu_baseline"] = cpu_baseline(X, N, args.cpu_images)
        log(f"cpu baseline done: {out['cpu_baseline']['sample']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
