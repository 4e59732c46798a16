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
durations inside the timed region: the first ``--event-steps`` timed steps
(default 1) record an event pair around every allocation and update (their
recording cost is part of the measured wall time); ``cpu_baseline`` times
the FP64 CPU oracle on a bounded sample of the same workload on this host's
cores.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

HERE = os.path.dirname(os.path.abspath(__file__))
# Sources of the allocation kernels: counters taken on an older build of them
# are not reported.
BF16_SOURCES = ("paper_0910_4711_amd/csrc/assign_common.h",
                "paper_0910_4711_amd/csrc/assign_bf16.hip")
FP32_SOURCES = ("paper_0910_4711_amd/csrc/assign_common.h",
                "paper_0910_4711_amd/csrc/assign.hip")
TRAFFIC_FILE_BF16 = "profiles/assign_bf16_img256x1024x1024_b8_N1024_traffic.txt"
TRAFFIC_FILE_FP32 = "profiles/assign_fp32_img256x1024x1024_b8_N1024_traffic.txt"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload():
    import synth
    cfg = synth.CONFIG1
    X = synth.image_training_set(cfg["seeds"], cfg["W"], cfg["H"], cfg["b"])
    return cfg, X


def source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(traffic_file, sources):
    """HBM bytes per allocation launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a plain copy of known size), or None when the summary is
    missing or was taken on other kernel sources."""
    path = os.path.join(HERE, traffic_file)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash(sources):
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
    # one more run with an event pair around every round's allocation and
    # update (direct launches): the kernels' own rooflines
    with torch.cuda.stream(side):
        res_t, st_t = P.train_batched(Xs, Ns, timing=True)
    side.synchronize()
    Ls = [x.shape[1] for x in Xs]
    Ms = [x.shape[0] for x in Xs]
    flops = sum(2.0 * L * r[3]["distances"] for L, r in zip(Ls, res_t))
    upd_bytes = sum(r[3]["n_update"] * M * (4.0 * L + 4.0) for M, L, r in zip(Ms, Ls, res_t))
    tf = flops / (st_t["ms_assign"] * 1e-3) / 1e12
    gbs = upd_bytes / (st_t["ms_update"] * 1e-3) / 1e9
    # per-instance roofline: each instance's allocations take at least the
    # longer of its flops at the FP32 MFMA peak (2L per distance, the
    # arithmetic the allocation resolves) and its bytes at the HBM peak (X
    # read and idx written per allocation); its updates at least their bytes
    # at the HBM peak.  The bound is the sum over instances.
    t_alloc = 0.0
    t_upd = 0.0
    for M, L, r in zip(Ms, Ls, res_t):
        info = r[3]
        f_i = 2.0 * L * info["distances"]
        b_i = info["n_assign"] * M * (4.0 * L + 4.0)
        t_alloc += max(f_i / (PEAK_FP32_MFMA_TFLOPS * 1e12), b_i / (PEAK_HBM_GBS * 1e9))
        t_upd += info["n_update"] * M * (4.0 * L + 4.0) / (PEAK_HBM_GBS * 1e9)
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
    # the batched single steps on the final codebooks: one allocation (with
    # D) and one update of every instance, against the single calls
    Cs = [r[0] for r in res]
    ab = P.assign_batched(Xs, Cs)  # warm-up
    ub = P.update_batched(Xs, ab[0], Cs)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    ib, Db = P.assign_batched(Xs, Cs)
    t_ab = time.perf_counter() - t0
    t0 = time.perf_counter()
    ub = P.update_batched(Xs, ib, Cs)
    t_ub = time.perf_counter() - t0
    t0 = time.perf_counter()
    single_ab = [P.assign_distortion(X, C, P.FP32) for X, C in zip(Xs, Cs)]
    torch.cuda.synchronize(dev)
    t_as = time.perf_counter() - t0
    t0 = time.perf_counter()
    single_ub = [P.update(X, i1[0], C) for X, i1, C in zip(Xs, single_ab, Cs)]
    torch.cuda.synchronize(dev)
    t_us = time.perf_counter() - t0
    steps_same = sum(1 for a, b, c, d in zip(ib, Db, single_ab, ub[0])
                     if torch.equal(a, c[0]) and float(b.item()) == float(c[2].item()))
    upd_same = sum(1 for a, b in zip(ub[0], single_ub) if torch.equal(a, b[0]))
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
        "allocation_roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_FP32_MFMA_TFLOPS,
                                "unit": "TFLOP/s", "frac": tf / PEAK_FP32_MFMA_TFLOPS,
                                "ms_all_rounds": st_t["ms_assign"],
                                "per_instance_bound_ms": t_alloc * 1e3,
                                "frac_per_instance": t_alloc * 1e3 / st_t["ms_assign"],
                                "per_instance_basis": "sum_i max(2 L_i distances_i / FP32 MFMA "
                                                      "peak, n_assign_i M_i (4 L_i + 4) / HBM peak)"},
        "update_roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                            "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                            "ms_all_rounds": st_t["ms_update"],
                            "algorithmic_bytes": upd_bytes,
                            "per_instance_bound_ms": t_upd * 1e3,
                            "frac_per_instance": t_upd * 1e3 / st_t["ms_update"]},
        "per_instance_launches": {"value": dist / t_s, "ms_total": t_s * 1e3},
        "speedup_vs_per_instance": t_s / t_b,
        "identical_D_to_per_instance": f"{same}/{len(inst)}",
        "batched_single_steps": {
            "assign_batched_ms": t_ab * 1e3, "assign_distortion_per_instance_ms": t_as * 1e3,
            "update_batched_ms": t_ub * 1e3, "update_per_instance_ms": t_us * 1e3,
            "identical_allocation_and_D": f"{steps_same}/{len(inst)}",
            "identical_update": f"{upd_same}/{len(inst)}"},
    }
    print(json.dumps(out), flush=True)


def _image_blocks_worker(args):
    import synth
    seed, W, H, b = args
    return synth.blocks(synth.image(seed, W, H), b)


def _image_set_parallel(seeds, W, H, b):
    import concurrent.futures as cf
    with cf.ProcessPoolExecutor(max_workers=16) as ex:
        parts = list(ex.map(_image_blocks_worker, [(s_, W, H, b) for s_ in seeds]))
    return np.concatenate(parts).astype(np.float32)


def _events_ms(fn, stream, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) / reps


def form_precision(args):
    """Precision form at the 8x8-block workload: M = 4,194,304 vectors of
    L = 64 from 256 synthetic 1024 x 1024 images, N = 1024 initial
    codevectors = distinct training vectors, 10 Lloyd iterations in exact FP32
    and with the BF16 screen + FP32 top-2 rescore; errors against the FP64
    oracle on a 65,536-vector subsample."""
    import torch
    import oracle
    import synth
    import paper_0910_4711_amd as P
    cfg = synth.CONFIG2
    n_img = args.images if args.images else len(cfg["seeds"])
    t0 = time.perf_counter()
    X = _image_set_parallel(tuple(range(n_img)), cfg["W"], cfg["H"], cfg["b"])
    M, L = X.shape
    N = cfg["N"]
    log(f"generated M={M} L={L} in {time.perf_counter() - t0:.1f} s")
    C0 = X[synth.distinct_rows(X, N, 1000)]
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    C0d = torch.from_numpy(np.ascontiguousarray(C0)).to(dev)
    stream = torch.cuda.Stream(device=dev)
    out = {"metric": "precision form: allocation vector-codeword distances/s, BF16 screen + "
                     "FP32 top-2 rescore vs exact FP32",
           "unit": "distances/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": f"img{n_img}x1024x1024_b8_M{M}_L{L}_N{N}_10iters",
                      "M": M, "L": L, "N": N, "iterations": 10}}
    runs = {}
    for prec in (P.FP32, P.BF16_RESCORE):
        name = "fp32" if prec == P.FP32 else "bf16"
        with torch.cuda.stream(stream):
            P.train(Xd, N, C_init=C0d, fixed_iters=10, precision=prec)  # warm-up
        stream.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            C, idx, D, st = P.train(Xd, N, C_init=C0d, fixed_iters=10, precision=prec,
                                    timing=True)
        stream.synchronize()
        wall = time.perf_counter() - t0
        dist = st["total_distances"]
        flops = 2.0 * L * dist
        ms_a = st["ms_assign"]
        peak = PEAK_FP32_MFMA_TFLOPS if prec == P.FP32 else 2500.0
        tf = flops / (ms_a * 1e-3) / 1e12
        runs[name] = (C, idx, D, st)
        out[name] = {"distances_per_s_assign": dist / (ms_a * 1e-3),
                     "assign_ms_total": ms_a, "update_ms_total": st["ms_update"],
                     "wall_ms": wall * 1e3, "assigns": st["total_assigns"],
                     "roofline": {"bound": "mfma", "achieved": tf, "peak": peak,
                                  "unit": "TFLOP/s", "frac": tf / peak,
                                  "peak_basis": ("FP32 MFMA peak for the 2L FP32 flops per "
                                                 "distance; the exact kernel screens with BF16 "
                                                 "hi/mid/lo parts (25 v_mfma_f32_32x32x16_bf16 "
                                                 "per 32x32 tile at L = 64), so frac can exceed 1"
                                                 if prec == P.FP32 else
                                                 "BF16 MFMA peak, 2L flops per distance")},
                     "update_GBs": (st["total_updates"] * M * (4 * L + 4)
                                    / (st["ms_update"] * 1e-3) / 1e9
                                    if st["ms_update"] > 0 else None),
                     "D": D}
    out["value"] = out["bf16"]["distances_per_s_assign"]
    out["speedup_bf16_vs_fp32_assign"] = (out["fp32"]["assign_ms_total"]
                                          / out["bf16"]["assign_ms_total"])
    # Per-step errors: the same FP32 codebook (the exact run's final one) into
    # one BF16 and one FP32 allocation + update; allocation errors against the
    # FP64 oracle on a 65,536-vector subsample.
    Cref = runs["fp32"][0]
    idx_b, mind_b = P.assign(Xd, Cref, P.BF16_RESCORE)
    idx_f, _ = P.assign(Xd, Cref, P.FP32)
    Cb1, _ = P.update(Xd, idx_b, Cref)
    Cf1, _ = P.update(Xd, idx_f, Cref)
    D_b = float(P.distortion(Xd, Cref, idx_b).item())
    D_f = float(P.distortion(Xd, Cref, idx_f).item())
    torch.cuda.synchronize()
    rows = np.random.default_rng(1001).choice(M, min(M, 65536), replace=False)
    rows.sort()
    Ch = Cref.cpu().numpy().astype(np.float64)
    idx_o, d1, d2 = oracle.assign(X[rows], Ch)
    ib = idx_b.cpu().numpy()[rows]
    xx = (X[rows].astype(np.float64) ** 2).sum(1)
    wrong = ib != idx_o
    near = (d2 - d1) < 1e-6 * xx
    dsel = ((X[rows].astype(np.float64) - Ch[ib]) ** 2).sum(1)

    def rel_rows(A, B):
        A = A.cpu().numpy().astype(np.float64)
        B = B.cpu().numpy().astype(np.float64)
        return np.linalg.norm(A - B, axis=1) / np.maximum(np.linalg.norm(B, axis=1), 1e-30)

    r1 = rel_rows(Cb1, Cf1)
    r10 = rel_rows(runs["bf16"][0], runs["fp32"][0])
    out["bf16_errors"] = {
        "per_step": {
            "subsample_rows": int(rows.size),
            "assign_mismatch_rate_vs_fp64_oracle": float(wrong.mean()),
            "assign_mismatch_outside_tie_band": int((wrong & ~near).sum()),
            "rescored_distance_excess_rel_max": float(((dsel - d1) / np.maximum(d1, 1e-30)).max()),
            "codebook_rel_vs_exact_update_max": float(r1.max()),
            "codebook_rel_vs_exact_update_median": float(np.median(r1)),
            "D_rel_vs_exact": abs(D_b - D_f) / D_f,
        },
        "after_10_iterations": {
            "codebook_rel_vs_exact_run_max": float(r10.max()),
            "codebook_rel_vs_exact_run_median": float(np.median(r10)),
            "D_rel_vs_exact_run": abs(runs["bf16"][2] - runs["fp32"][2]) / runs["fp32"][2],
        },
    }
    print(json.dumps(out), flush=True)


def form_differentiation(args):
    """Differentiation form: D = mean_m min_k ||x_m - c_k||^2 with X
    [1,048,576 x 64] from a 512-component diagonal Gaussian mixture and C
    [4096 x 64] distinct training vectors: forward (allocation + FP64
    distortion) and backward (dD/dX, dD/dC) through the autograd function."""
    import torch
    import synth
    import paper_0910_4711_amd as P
    M, L, K, N = 1_048_576, 64, 512, 4096
    t0 = time.perf_counter()
    X = synth.gmm_diag(20000, M, L, K)
    C = np.ascontiguousarray(X[synth.distinct_rows(X, N, 20001)])
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev).requires_grad_(True)
    Cd = torch.from_numpy(C).to(dev).requires_grad_(True)
    stream = torch.cuda.Stream(device=dev)

    def fwd():
        return P.Distortion.apply(Xd, Cd)

    def fwd_bwd():
        Xd.grad = None
        Cd.grad = None
        fwd().backward()

    for _ in range(2):
        with torch.cuda.stream(stream):
            fwd_bwd()
    stream.synchronize()
    ms_f = _events_ms(fwd, stream, args.steps)
    ms_fb = _events_ms(fwd_bwd, stream, args.steps)
    ms_b = ms_fb - ms_f
    dist = M * N
    tf = 2.0 * L * dist / (ms_f * 1e-3) / 1e12
    # matrix-core work the screen issues: 6 L/16 + 1 products of 32x32x16 per
    # 32 x 32 tile of distances
    bf16_tf = (6 * (L // 16) + 1) * 32 * 32 * 16 * 2 / 1024 * dist / (ms_f * 1e-3) / 1e12
    bwd_bytes = M * L * 4 * 2 + M * 4 + M * L * 4 + N * L * 4  # read X (twice), idx; write gX, gC
    out = {"metric": "differentiation form: forward vector-codeword distances/s",
           "value": dist / (ms_f * 1e-3), "unit": "distances/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"gmmdiag512_M{M}_L{L}_N{N}", "M": M, "L": L, "N": N},
           "forward_ms": ms_f, "backward_ms": ms_b,
           "forward_roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_FP32_MFMA_TFLOPS,
                                "unit": "TFLOP/s", "frac": tf / PEAK_FP32_MFMA_TFLOPS,
                                "peak_basis": "FP32 MFMA peak for the 2L FP32 flops per "
                                              "distance the allocation resolves; the screen "
                                              "runs on exact three-part BF16 splits (25 "
                                              "v_mfma_f32_32x32x16_bf16 per 32x32 tile at "
                                              "L = 64), so this FP32-equivalent rate can "
                                              "exceed the FP32 peak",
                                "bf16_mfma_issued_tflops": bf16_tf,
                                "bf16_mfma_frac": bf16_tf / PEAK_BF16_MFMA_TFLOPS},
           "backward_roofline": {"bound": "hbm", "achieved": bwd_bytes / (ms_b * 1e-3) / 1e9,
                                 "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": bwd_bytes / (ms_b * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                 "algorithmic_bytes": bwd_bytes}}
    print(json.dumps(out), flush=True)


def _image_worker(args):
    import synth
    seed, W, H = args
    return synth.image(seed, W, H)


def form_codec(args):
    """Codec form: the encoder/decoder half of VQ with the benchmark
    workload's codebook (LBG on the 16 training pictures, 4 x 4 blocks, N =
    256), applied to 64 other synthetic 512 x 512 pictures (seeds
    1000..1063, M = 1,048,576 blocks): pictures -> block vectors
    (lbg_image_blocks), encoder (nearest codevector, lbg_encode), decoder
    straight into pictures (lbg_decode_image); PSNR from the distortion and
    the rate log2(N)/L."""
    import concurrent.futures as cf
    import torch
    import paper_0910_4711_amd as P
    cfg, Xtrain = workload()
    N, b, W, H = cfg["N"], cfg["b"], cfg["W"], cfg["H"]
    L = b * b
    seeds = list(range(1000, 1064))
    with cf.ProcessPoolExecutor(max_workers=16) as ex:
        pics = np.stack(list(ex.map(_image_worker, [(s_, W, H) for s_ in seeds])))
    nimg = len(seeds)
    M = nimg * (H // b) * (W // b)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        C, _, _, _ = P.train(torch.from_numpy(Xtrain).to(dev), N)
        img = torch.from_numpy(pics.astype(np.float32)).to(dev)
        X = P.image_blocks(img, b)
        idx = P.encode(X, C)
        rec = P.decode_image(idx, C, nimg, H, W, b)
        D = P.distortion(X, C, idx)
    stream.synchronize()
    psnr = P.psnr(D, L)
    ms_blocks = _events_ms(lambda: P.image_blocks(img, b), stream, args.steps)
    ms_enc = _events_ms(lambda: P.encode(X, C), stream, args.steps)
    ms_dec = _events_ms(lambda: P.decode_image(idx, C, nimg, H, W, b), stream, args.steps)

    def pipeline():
        x = P.image_blocks(img, b)
        return P.decode_image(P.encode(x, C), C, nimg, H, W, b)

    ms_all = _events_ms(pipeline, stream, args.steps)
    pixels = nimg * H * W
    dec_bytes = M * 4 + M * L * 4 + N * L * 4  # indices, pictures written, codebook once
    blk_bytes = 2 * M * L * 4                  # pictures read, vectors written
    dec_gbs = dec_bytes / (ms_dec * 1e-3) / 1e9
    blk_gbs = blk_bytes / (ms_blocks * 1e-3) / 1e9
    enc_tf = 2.0 * L * M * N / (ms_enc * 1e-3) / 1e12
    out = {"metric": "codec form: picture pixels coded and decoded/s",
           "value": pixels / (ms_all * 1e-3), "unit": "pixels/s", "n_gpus": 1,
           "steps": args.steps, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"code{nimg}x{H}x{W}_b{b}_M{M}_L{L}_N{N}",
                      "codebook": cfg["name"], "pictures": nimg, "M": M, "L": L, "N": N},
           "psnr_db": psnr, "rate_bits_per_sample": P.rate(N, L), "D": float(D.item()),
           "ms": {"image_blocks": ms_blocks, "encode": ms_enc, "decode_image": ms_dec,
                  "pipeline": ms_all},
           "decode_roofline": {"bound": "hbm", "achieved": dec_gbs, "peak": PEAK_HBM_GBS,
                               "unit": "GB/s", "frac": dec_gbs / PEAK_HBM_GBS,
                               "algorithmic_bytes": dec_bytes,
                               "kernel": "block_rows_kernel<1, 128, 0> (decoder)"},
           "image_blocks_roofline": {"bound": "hbm", "achieved": blk_gbs,
                                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                     "frac": blk_gbs / PEAK_HBM_GBS,
                                     "algorithmic_bytes": blk_bytes,
                                     "kernel": "block_rows_kernel<1, 128, 1, true> (pictures to blocks, stores staged through LDS)"},
           "encode": {"distances_per_s": M * N / (ms_enc * 1e-3), "tflops": enc_tf,
                      "frac_fp32_mfma": enc_tf / PEAK_FP32_MFMA_TFLOPS}}
    print(json.dumps(out), flush=True)


def lscpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_precision(X, C0, iters):
    """The FP64 oracle, as it stands, on the 65,536-row subsample of the
    precision workload (rows from default_rng(1001), without replacement):
    the same 1,024 starting codevectors and the same number of Lloyd
    iterations, on all host cores and on one thread (the paper's sequential
    baseline).  Distances/s = rows * N * allocations / wall time."""
    import oracle
    oracle.load()
    rows = np.random.default_rng(1001).choice(X.shape[0], min(X.shape[0], 65536), replace=False)
    rows.sort()
    S = np.ascontiguousarray(X[rows])
    N = C0.shape[0]
    cores = len(os.sched_getaffinity(0))
    out = {}
    for name, nt in (("all_cores", cores), ("one_thread", 1)):
        t0 = time.perf_counter()
        oracle.train(S, N, C_init=C0.astype(np.float64), fixed_iters=iters, nthreads=nt)
        t = time.perf_counter() - t0
        out[name] = dict(value=S.shape[0] * N * (iters + 1) / t, threads=nt, seconds=t)
    return dict(value=out["all_cores"]["value"], unit="distances/s", cores=cores,
                kind="oracle", cpu_model=lscpu_model(),
                one_thread=out["one_thread"],
                speedup_all_cores_vs_one_thread=out["one_thread"]["seconds"]
                / out["all_cores"]["seconds"],
                sample=f"{iters} Lloyd iterations ({iters + 1} allocations) from the same "
                       f"{N} starting codevectors on the {S.shape[0]}-row subsample "
                       f"(default_rng(1001)) of the M = {X.shape[0]} workload, FP64; "
                       f"{out['all_cores']['seconds']:.2f} s on {cores} threads, "
                       f"{out['one_thread']['seconds']:.2f} s on one thread")


def paper_experiment(cores):
    """The paper's own experiment (Sec. 5, Figs. 3 and 4), shape only, on the
    FP64 oracle: full LBG runs on 2,000 synthetic training vectors (a
    16-component Gaussian mixture) of dimension k; wall time against the
    codebook size N = 8..128 sequentially and on 4 threads, and against the
    thread count at N = 128.  Only the allocation loop of the oracle runs on
    several threads (static chunks of vectors, as Algorithm 1 hands them
    out).  Each time is the median of three runs."""
    import oracle
    import synth

    def timed(X, N, nt):
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.train(X, N, nthreads=nt)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    fig3 = []
    for k in (2, 10):
        X = synth.gmm(40_000 + k, 2000, k, 16)
        for N in (8, 16, 32, 64, 128):
            t1, t4 = timed(X, N, 1), timed(X, N, 4)
            fig3.append({"k": k, "N": N, "seconds_1_thread": t1, "seconds_4_threads": t4,
                         "speedup_4": t1 / t4})
    X = synth.gmm(40_010, 2000, 10, 16)
    fig4 = []
    t1 = None
    for nt in sorted({1, 2, 4, 8, cores}):
        if nt > cores:
            continue
        t = timed(X, 128, nt)
        t1 = t if nt == 1 else t1
        fig4.append({"threads": nt, "seconds": t, "speedup": t1 / t})
    return {"what": "paper Sec. 5 experiment on the FP64 oracle (shape only; the paper's "
                    "data and figure values are not given): M = 2000 synthetic vectors",
            "time_vs_codebook_size": fig3, "time_vs_threads_N128_k10": fig4}


PAPER_CONTEXT = {
    "source": "paper Sec. 4 (profiling) and Sec. 5; hardware unstated, no absolute timings",
    "share_of_sequential_time_in_allocation": "70-75%",
    "share_of_sequential_time_in_update": "10-15%",
    "amdahl_speedup_4_threads_serial_fraction_0.15": 2.76,
}


def run_lbg_steps(P, Xd, N, steps, warmup, stream, event_steps=1, **kw):
    """Warm-up, then ``steps`` timed lbg_train calls (the first
    ``event_steps`` of them with an event pair around every allocation and
    update).  Returns (wall seconds of the timed steps, totals, event sums,
    last stats, last result)."""
    import torch
    for _ in range(warmup):
        with torch.cuda.stream(stream):
            P.train(Xd, N, timing=True, **kw)
        stream.synchronize()
    torch.cuda.synchronize()
    tot = dict(dist=0, assigns=0, updates=0, fallback=0)
    ev = dict(steps=0, dist=0, ms_assign=0.0, ms_update=0.0, assigns=0, updates=0)
    n_ev = max(1, min(event_steps, steps))
    last = None
    t0 = time.perf_counter()
    for i in range(steps):
        timed = i < n_ev
        with torch.cuda.stream(stream):
            C, idx, D, st = P.train(Xd, N, timing=timed, **kw)
        tot["dist"] += st["total_distances"]
        tot["assigns"] += st["total_assigns"]
        tot["updates"] += st["total_updates"]
        tot["fallback"] += st["fallback_rows"]
        if timed:
            ev["steps"] += 1
            ev["dist"] += st["total_distances"]
            ev["assigns"] += st["total_assigns"]
            ev["updates"] += st["total_updates"]
            ev["ms_assign"] += st["ms_assign"]
            ev["ms_update"] += st["ms_update"]
        last = (C, idx, D, st)
    stream.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, tot, ev, last


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline form (no exact-form, 16-picture or error legs)")
    ap.add_argument("--event-steps", type=int, default=1,
                    help="timed steps that record HIP events around every kernel")
    ap.add_argument("--copy-calibration", type=int, metavar="MIB", default=0,
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--form", choices=["batched", "precision", "differentiation", "codec",
                                       "config1"],
                    default=None, help="benchmark one of the forms instead of the main workload")
    ap.add_argument("--precision", choices=["bf16", "fp32"], default=None,
                    help="only this precision form of the main workload (profiling runs)")
    ap.add_argument("--images", type=int, default=0,
                    help="images of the main / precision workload (default: all 256)")
    ap.add_argument("--instances", type=int, default=512, help="instances of --form batched")
    ap.add_argument("--scale", type=float, default=1.0, help="row-count scale of --form batched")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on exactly one GPU; --gpus {args.gpus} "
              "is not supported (the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.form:
        {"batched": form_batched, "precision": form_precision,
         "differentiation": form_differentiation, "codec": form_codec,
         "config1": form_config1}[args.form](args)
        return

    import torch
    import synth
    import paper_0910_4711_amd as P

    cfg = synth.CONFIG2
    n_img = args.images if args.images else len(cfg["seeds"])
    t0 = time.perf_counter()
    X = _image_set_parallel(tuple(range(n_img)), cfg["W"], cfg["H"], cfg["b"])
    M, L = X.shape
    N = cfg["N"]
    iters = 10
    C0 = np.ascontiguousarray(X[synth.distinct_rows(X, N, 1000)])
    log(f"generated M={M} L={L} in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    C0d = torch.from_numpy(C0).to(dev)
    lib = P.load()
    ws = torch.empty(max(lib.lbg_workspace_size(P.OP_TRAIN, M, L, N, prec) for prec in
                         (P.FP32, P.BF16_RESCORE)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    log(f"workload {cfg['name']}: M={M} L={L} N={N}, {iters} Lloyd iterations per step; "
        f"device {torch.cuda.get_device_name(dev)}")

    forms = {}
    want = [args.precision] if args.precision else ["bf16", "fp32"]
    if args.no_extras and not args.precision:
        want = ["bf16"]
    for name in want:
        prec = P.BF16_RESCORE if name == "bf16" else P.FP32
        el, tot, ev, last = run_lbg_steps(P, Xd, N, args.steps, args.warmup, stream,
                                          args.event_steps, C_init=C0d, fixed_iters=iters,
                                          precision=prec, workspace=ws)
        log(f"{name}: timed {args.steps} steps in {el:.4f} s")
        forms[name] = (el, tot, ev, last)

    def roofline(name):
        el, tot, ev, last = forms[name]
        flops = 2.0 * L * ev["dist"]  # 2L flops per vector-codeword distance
        a_s = ev["ms_assign"] / 1e3
        ach = flops / a_s / 1e12
        upd_bytes = ev["updates"] * M * (4 * L + 4)
        upd_gbs = upd_bytes / (ev["ms_update"] / 1e3) / 1e9 if ev["ms_update"] > 0 else None
        if name == "bf16":
            kern = ("bf16v2_kernel<64, vector loads> (BF16 screen, codebook resident in LDS, "
                    "8 waves per CU, two 32-vector tiles per wave; FP32 top-2 rescore)")
            peak, basis = PEAK_BF16_MFMA_TFLOPS, "BF16 dense MFMA peak, 2L flops per distance"
            tr = measured_traffic(TRAFFIC_FILE_BF16, BF16_SOURCES)
        else:
            kern = "assign_kernel<Bf16x3Screen<64>, vector loads, 4 waves> (exact)"
            peak, basis = PEAK_BF16_MFMA_TFLOPS, ("BF16 dense MFMA peak (the exact screen "
                                                  "contracts BF16 parts), 2L flops per distance")
            tr = measured_traffic(TRAFFIC_FILE_FP32, FP32_SOURCES)
        r = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
             "frac": ach / peak,
             "traffic": tr["bytes"] if tr else None,
             "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                             "copy-calibrated)",
             "algorithmic_bytes_per_launch": M * (4 * L + 4) + N * L * 4,
             "kernel": kern, "peak_basis": basis,
             "frac_of_fp32_mfma_peak": ach / PEAK_FP32_MFMA_TFLOPS,
             "launches": ev["assigns"], "event_steps": ev["steps"],
             "avg_launch_us": ev["ms_assign"] / ev["assigns"] * 1e3,
             "flops_per_launch": flops / ev["assigns"]}
        u = {"bound": "hbm", "achieved_gbs": upd_gbs, "peak_gbs": PEAK_HBM_GBS,
             "frac": (upd_gbs / PEAK_HBM_GBS) if upd_gbs else None,
             "avg_update_us": ev["ms_update"] / max(1, ev["updates"]) * 1e3,
             "algorithmic_bytes_per_update": M * (4 * L + 4)}
        return r, u

    head = "bf16" if "bf16" in forms else "fp32"
    el, tot, ev, last = forms[head]
    rl, upd = roofline(head)
    out = {
        "metric": "LBG iteration vector-codeword distances/s (BF16 screen + FP32 top-2 "
                  "rescore; exact FP32-accurate form and its ratio beside it)",
        "value": tot["dist"] / el,
        "unit": "distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if head == "bf16" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"img{n_img}x1024x1024_b8_M{M}_L{L}_N{N}_10iters",
            "M": M, "L": L, "N": N, "images": n_img, "image_size": [1024, 1024], "block": 8,
            "init": "1024 distinct training vectors, default_rng(1000) permutation",
            "lloyd_iterations_per_step": iters,
            "precision": ("BF16 distances with FP32 accumulation, top-2 rescored in FP32"
                          if head == "bf16" else "exact (FP32-accurate screen, FP64 certificate)"),
        },
        "roofline": rl,
        "update": upd,
        "per_step": {"assigns": tot["assigns"] // args.steps,
                     "updates": tot["updates"] // args.steps,
                     "ms_assign": ev["ms_assign"] / ev["steps"],
                     "ms_update": ev["ms_update"] / ev["steps"],
                     "D": last[2]},
        "paper_context": PAPER_CONTEXT,
    }
    if "fp32" in forms and head != "fp32":
        el2, tot2, ev2, last2 = forms["fp32"]
        rl2, upd2 = roofline("fp32")
        out["fp32_exact"] = {"value": tot2["dist"] / el2, "ms_per_step": el2 / args.steps * 1e3,
                             "roofline": rl2, "update": upd2,
                             "fallback_rows_per_step": tot2["fallback"] // args.steps,
                             "D": last2[2]}
        out["speedup_vs_fp32_exact"] = (tot["dist"] / el) / (tot2["dist"] / el2)
        out["bf16_errors"] = bf16_errors(P, X, Xd, last2[0], last[0], last[2], last2[2], C0d, iters)
    if not args.no_extras and not args.precision:
        out["config1"] = config1_line(P, max(3, args.steps // 2), 2, stream)
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle) ...")
        out["cpu_baseline"] = cpu_baseline_precision(X, C0, iters)
        log(f"cpu baseline done: {out['cpu_baseline']['sample']}")
        if not args.no_extras:
            out["cpu_baseline"]["paper_experiment"] = paper_experiment(
                out["cpu_baseline"]["cores"])
    print(json.dumps(out), flush=True)


def bf16_errors(P, X, Xd, C_exact, C_bf16, D_bf16, D_exact, C0d=None, iters=10):
    """Errors of the BF16 form: per step (the exact run's final codebook into
    one BF16 and one exact allocation + update; allocations against the FP64
    oracle on the 65,536-row subsample), along the BF16 run (every one of its
    steps against the exact step from the same codebook) and after the 10
    iterations."""
    import torch
    import oracle
    M = X.shape[0]
    idx_b, _ = P.assign(Xd, C_exact, P.BF16_RESCORE)
    idx_f, _ = P.assign(Xd, C_exact, P.FP32)
    Cb1, _ = P.update(Xd, idx_b, C_exact)
    Cf1, _ = P.update(Xd, idx_f, C_exact)
    D_b = float(P.distortion(Xd, C_exact, idx_b).item())
    D_f = float(P.distortion(Xd, C_exact, idx_f).item())
    torch.cuda.synchronize()
    rows = np.random.default_rng(1001).choice(M, min(M, 65536), replace=False)
    rows.sort()
    Ch = C_exact.cpu().numpy().astype(np.float64)
    idx_o, d1, d2 = oracle.assign(X[rows], Ch)
    ib = idx_b.cpu().numpy()[rows]
    xx = (X[rows].astype(np.float64) ** 2).sum(1)
    wrong = ib != idx_o
    near = (d2 - d1) < 1e-6 * xx

    def rel_rows(A, B):
        A = A.cpu().numpy().astype(np.float64)
        B = B.cpu().numpy().astype(np.float64)
        return np.linalg.norm(A - B, axis=1) / np.maximum(np.linalg.norm(B, axis=1), 1e-30)

    r1 = rel_rows(Cb1, Cf1)
    r10 = rel_rows(C_bf16, C_exact)
    # along the BF16 trajectory: step t of the BF16 run (allocation in BF16,
    # exact update) against the exact step from the same codebook C_t
    along = []
    if C0d is not None:
        Ct = C0d.clone()
        for _ in range(iters):
            ib_t, _ = P.assign(Xd, Ct, P.BF16_RESCORE)
            if_t, _ = P.assign(Xd, Ct, P.FP32)
            Cb_t, _ = P.update(Xd, ib_t, Ct)
            Cf_t, _ = P.update(Xd, if_t, Ct)
            r = rel_rows(Cb_t, Cf_t)
            along.append({"codebook_rel_max": float(r.max()),
                          "codebook_rel_median": float(np.median(r)),
                          "allocation_mismatch_rate_vs_exact":
                              float((ib_t != if_t).float().mean().item())})
            Ct = Cb_t
    return {
        "per_step": {
            "subsample_rows": int(rows.size),
            "assign_mismatch_rate_vs_fp64_oracle": float(wrong.mean()),
            "assign_mismatch_outside_tie_band": int((wrong & ~near).sum()),
            "codebook_rel_vs_exact_update_max": float(r1.max()),
            "codebook_rel_vs_exact_update_median": float(np.median(r1)),
            "D_rel_vs_exact": abs(D_b - D_f) / D_f,
        },
        "per_step_along_bf16_run": {
            "steps": along,
            "codebook_rel_max_over_steps": max((a["codebook_rel_max"] for a in along),
                                               default=None),
        },
        "after_10_iterations": {
            "codebook_rel_vs_exact_run_max": float(r10.max()),
            "codebook_rel_vs_exact_run_median": float(np.median(r10)),
            "D_rel_vs_exact_run": abs(D_bf16 - D_exact) / D_exact,
        },
    }


def config1_line(P, steps, warmup, stream):
    """Full LBG runs on the 16-picture workload (M = 262,144, L = 16, split
    to N = 256, stop at relative change 1e-3), exact form."""
    import torch
    cfg, X = workload()
    M, L = X.shape
    N = cfg["N"]
    Xd = torch.from_numpy(X).to("cuda:0")
    el, tot, ev, last = run_lbg_steps(P, Xd, N, steps, warmup, stream, 1)
    flops = 2.0 * L * ev["dist"]
    ach = flops / (ev["ms_assign"] / 1e3) / 1e12
    upd_bytes = ev["updates"] * M * (4 * L + 4)
    return {"workload": cfg["name"], "value": tot["dist"] / el, "unit": "distances/s",
            "steps": steps, "ms_per_step": el / steps * 1e3,
            "assign_tflops": ach, "assign_frac_fp32_mfma_peak": ach / PEAK_FP32_MFMA_TFLOPS,
            "assign_frac_bf16_mfma_peak": ach / PEAK_BF16_MFMA_TFLOPS,
            "avg_assign_us": ev["ms_assign"] / ev["assigns"] * 1e3,
            "avg_update_us": ev["ms_update"] / max(1, ev["updates"]) * 1e3,
            "update_frac_hbm": upd_bytes / (ev["ms_update"] / 1e3) / 1e9 / PEAK_HBM_GBS,
            "level_iters": last[3]["level_iters"], "D": last[2]}


def form_config1(args):
    """The 16-picture workload alone (full LBG runs): one JSON line, with the
    oracle timed on the same runs."""
    import torch
    import oracle
    import paper_0910_4711_amd as P
    stream = torch.cuda.Stream(device="cuda:0")
    out = config1_line(P, args.steps, args.warmup, stream)
    if not args.no_cpu_baseline:
        cfg, X = workload()
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        r = oracle.train(X, cfg["N"], nthreads=cores)
        t = time.perf_counter() - t0
        dist = X.shape[0] * int(sum(int(n) * (int(i) + 1)
                                    for n, i in zip(r["level_n"], r["level_iters"])))
        out["cpu_baseline"] = dict(value=dist / t, unit="distances/s", cores=cores,
                                   kind="oracle", cpu_model=lscpu_model(),
                                   sample=f"full LBG to N={cfg['N']} on M={X.shape[0]}, "
                                          f"FP64, {t:.2f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
