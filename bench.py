"""Benchmark: whole hot path on one MI355X.

Workload (the configuration the metric is quoted on): 2D annulus r in [0.3, 1], K = [[1, .5],
[.5, 2]], 128 + 128 boundary arcs, 1024 observation points, N = 1e5 walks per point, eps = 1e-4,
FP32 walk geometry with FP64 exit test / binning, then FP64 SVD of the 1024 x 192 Gamma_1 block and
the TSVD reconstruction (discrepancy principle) of u_1.  One step = zero counts + walk kernel +
assembly + SVD + reconstruction; inputs are resident in HBM.  Steps are pipelined over two CU
partitions (two streams with CU masks): the walk kernel of step i + 1 runs on most CUs while the
SVD and reconstruction of step i run on the rest; ms_per_step is the interval between step
completions, and the latency of one step alone (a captured HIP graph) is reported beside it.

Prints one JSON line (rank 0).  Extra fields: the walk kernel alone (HIP events on its stream), the
FP64 walk path, the roofline of the walk kernel, the CPU oracle baseline and serving latency.
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

# Algorithmic 32-bit VALU operations per sphere step of the 2D FP32 annulus walk, counted from the
# method (an FMA counts once): Philox4x32-10 = 10 rounds x (2 mul-lo + 2 mul-hi + 4 xor) = 80 ops
# per block, one block per 4 steps -> 20; uniform from 24 bits 3; direction cos, sin 2; shrunken
# radius 1; x += r S U 6; annulus distance 8; exit / band / cap tests and step count 4.  Per walk:
# FP64 projection onto the boundary + arc index + histogram 30.
OPS_PER_STEP_2D_FP32 = 20 + 3 + 2 + 1 + 6 + 8 + 4
OPS_PER_WALK = 30
# Algorithmic HBM bytes per launch of the workload: observation points (2 x f64 each) read once,
# the 1024 x 256 uint32 count rows written once, 8 statistics words.
ALGO_BYTES_PER_POINT = 16 + 256 * 4
# HBM traffic measured with rocprofv3 counters (FETCH_SIZE, WRITE_SIZE) for the walk kernel of this
# workload, with the hash of the kernel sources it was measured on; reported only while they match.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "walk_kernel_f32_annulus_1024x1e5_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2409_03686_amd", "csrc", f) for f in ("walk_kernel.hip", "wos_device.hpp")]
# MI355X VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one lane-op per lane per clock).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(shape):
    """(bytes per launch, detail) from the committed counter summary, or (None, reason)."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None, "no counter summary"
    rec = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    try:
        if rec.get("kernel_sources_sha256") != kernel_sources_hash():
            return None, "kernel changed since the counters were taken"
        if rec.get("launch_shape") != f"{shape[0]},{shape[1]},{ITEM_MODES[shape[2]]}":
            return None, "counters were taken at another launch shape"
        f, w = float(rec["fetch_bytes_per_launch"]), float(rec["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None, "counter summary unreadable"
    return f + w, {"fetch_bytes": f, "write_bytes": w}


ITEM_MODES = ("auto", "block", "wave", "point")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--walks", type=int, default=100_000)
    p.add_argument("--spectral-cus", type=int, default=8,
                   help="CUs of the spectral stream (SVD + reconstruction); the walk kernel gets the rest")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--autotune", action="store_true",
                   help="time every walk launch shape first (its launches then appear in kernel traces)")
    p.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    p.add_argument("--serve-seconds", type=float, default=3.0)
    p.add_argument("--serve-svd", type=int, default=1, choices=(0, 1),
                   help="serving SVD: 0 full (cooperative Jacobi), 1 truncated (plain kernels, overlapping)")
    p.add_argument("--serve-rate", type=float, default=200.0)
    p.add_argument("--serve-radius", default="mapped", choices=("mapped", "dist"),
                   help="step radius of the serving requests: each kind's mapped radius, or r = dist (the "
                        "cube's exact radius only)")
    p.add_argument("--serve-only", action="store_true", help="only the serving measurement (for profiling)")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target wall time of the CPU sample")
    p.add_argument("--items", choices=("auto", "block", "wave", "point"), default="auto",
                   help="who owns the walk work: the library's choice, a block per item, a wave per item, "
                        "or a block per point")
    p.add_argument("--kernel-only", action="store_true",
                   help="for counter collection: one 1 GiB device copy (calibration), then the FP32 walk "
                        "kernel of the workload --steps times")
    return p.parse_args()


def cpu_baseline(inst, target_s):
    """The oracle (FP64 walks + LAPACK SVD + TSVD) on a sample of the same workload: every point,
    the first n walks, n chosen so the walks take about target_s seconds on all host cores."""
    from oracle import linalg as ol
    from oracle import walks as ow
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ow.build_instance(inst, walk_end=64, threads=cores)
    cal = time.perf_counter() - t0
    n = int(max(64, min(inst.n_walks, 64 * target_s / max(cal, 1e-3))))
    t0 = time.perf_counter()
    counts, st, _ = ow.build_instance(inst, walk_end=n, threads=cores)
    t_walk = time.perf_counter() - t0
    t0 = time.perf_counter()
    sigma = ow.element_measures(inst.geom)
    out = ol.assemble(counts, n, inst.geom.gamma1_mask, sigma, uD=inst.uD, u0=inst.u0)
    U, s, Vt = ol.svd(out["B"])
    g1 = inst.geom.gamma1_mask.astype(bool)
    ol.reconstruct(U, s, Vt, sigma[g1], out["q"], kind=ol.TSVD_DISCREPANCY, delta=inst.noise_delta, tau=1.1)
    t_lin = time.perf_counter() - t0
    walks = st["walks"]
    return {"value": walks / (t_walk + t_lin), "unit": "walks/s", "cores": cores, "kind": "oracle",
            "sample": f"all {inst.x_obs.shape[0]} points x first {n} walks (of {inst.n_walks}), FP64 walks + "
                      f"LAPACK SVD + TSVD; walks {t_walk:.2f} s, linear algebra {t_lin:.3f} s",
            "steps_per_s": st["steps"] / t_walk}


def _requests(wos, insts, arrivals):
    """wos_request / wos_result arrays for the instances (host buffers kept alive in `keep`)."""
    import ctypes as C
    reqs, res, keep = [], [], []
    for inst, t in zip(insts, arrivals):
        r = wos.WosRequest()
        gs = wos.geometry(inst.geom)
        r.geom = gs
        r.walk = wos.walk_params_of(inst)
        x = np.ascontiguousarray(inst.x_obs)
        m = np.ascontiguousarray(inst.geom.gamma1_mask)
        uD, u0 = np.ascontiguousarray(inst.uD), np.ascontiguousarray(inst.u0)
        r.x_obs_host = x.ctypes.data_as(C.POINTER(C.c_double))
        r.n_obs = x.shape[0]
        r.gamma1_mask_host = m.ctypes.data_as(C.POINTER(C.c_uint8))
        r.uD_host = uD.ctypes.data_as(C.POINTER(C.c_double))
        r.u0_host = u0.ctypes.data_as(C.POINTER(C.c_double))
        r.reg = wos.reg_params(wos.WOS_TSVD_DISCREPANCY, noise_delta=inst.noise_delta, tau=1.1)
        r.arrival_s = float(t)
        u1 = np.zeros(int(m.sum()))
        o = wos.WosResult()
        o.u1_host = u1.ctypes.data_as(C.POINTER(C.c_double))
        keep += [gs, x, m, uD, u0, u1]
        reqs.append(r)
        res.append(o)
    return reqs, res, keep


def _serve(ctx, wos, insts, arrivals, svd_mode):
    reqs, res, keep = _requests(wos, insts, arrivals)
    t0 = time.perf_counter()
    out = wos.wos_serve(ctx, reqs, res, hbm_budget_bytes=32 << 30, max_inflight=16, svd_mode=svd_mode)
    wall = time.perf_counter() - t0
    ok = [o for o in out if o.status == 0]
    lat = np.array([o.t_done - o.t_arrive for o in ok]) if ok else np.zeros(1)
    # reconstruction error of each completed request: max |u1 - u| / max |u| on Gamma_1
    errs = []
    for k, (inst, o) in enumerate(zip(insts, out)):
        if o.status == 0 and inst.u_exact_g1 is not None:
            u1 = keep[6 * k + 5]
            errs.append(float(np.abs(u1 - inst.u_exact_g1).max() / max(np.abs(inst.u_exact_g1).max(), 1e-300)))
    return {"requests": len(out), "completed": len(ok), "median_rel_err_u1": float(np.median(errs)) if errs else None,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "walks_per_s": sum(o.walks for o in ok) / wall,
            "steps_per_s": sum(o.steps for o in ok) / wall, "wall_s": wall}


def serving(ctx, wos, wi, seconds, rate=200.0, svd_mode=1, radius="mapped"):
    """Request serving on the heterogeneous-instance generator (kinds, conductivities, sizes and walk
    budgets drawn per request; 1-5 % noise; random harmonic data of degree <= 6): each request is
    build H + FP64 SVD + TSVD reconstruction, host buffers in and out.  Capacity = requests per
    second with every request queued at t = 0; then open-loop Poisson arrivals at `rate` for
    `seconds`, and, when that load exceeds the capacity, at 0.8 x capacity as well.  Step radius: each
    kind's mapped radius (the same exit law as r = dist, shorter walks), or r = dist."""
    arr = wi.cfg5_arrivals(rate=rate, duration_s=seconds, seed=5)
    rng = np.random.default_rng(5)
    mapped = radius == "mapped"
    insts = [wi.random_instance(rng, i, mapped_radii=mapped) for i in range(len(arr))]
    cap = _serve(ctx, wos, insts, np.zeros(len(insts)), svd_mode)
    capacity = cap["completed"] / cap["wall_s"]
    offered = _serve(ctx, wos, insts, arr, svd_mode)
    mean_walks = float(np.mean([i.x_obs.shape[0] * i.n_walks for i in insts]))
    out = {"svd_mode": svd_mode, "radius": radius, "capacity_req_s": capacity, "capacity_walks_per_s": cap["walks_per_s"],
           "capacity_steps_per_s": cap["steps_per_s"], "mean_walks_per_request": mean_walks,
           "offered_rate_req_s": rate, "utilisation": rate / capacity, "at_offered_rate": offered}
    if rate >= capacity:
        r8 = 0.8 * capacity
        arr8 = wi.cfg5_arrivals(rate=r8, duration_s=seconds, seed=5)
        while len(insts) < len(arr8):
            insts.append(wi.random_instance(rng, len(insts), mapped_radii=mapped))
        out["at_0.8_capacity"] = dict(_serve(ctx, wos, insts[:len(arr8)], arr8, svd_mode), rate_req_s=r8)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import wos_inputs as wi
    from paper_2409_03686_amd import wos

    torch.cuda.set_device(0)
    inst = wi.cfg2_annulus(n_walks=a.walks, precision=wi.FP32_GEOM_FP64_EXIT)
    if a.serve_only:
        ctx = wos.wos_create(0)
        print(json.dumps({"serve_only": True, "serving": serving(ctx, wos, wi, a.serve_seconds, a.serve_rate, a.serve_svd,
                                                                 a.serve_radius)}))
        wos.wos_destroy(ctx)
        return
    items = {"auto": wos.WOS_ITEMS_AUTO, "block": wos.WOS_ITEMS_BLOCK, "wave": wos.WOS_ITEMS_WAVE,
             "point": wos.WOS_ITEMS_POINT}[a.items]
    if a.kernel_only:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ctx = wos.wos_create(0)
        wos.wos_set_tuning(ctx, 2, -1, inst.precision, 256, 16, items)
        x = wos.device_inputs(inst)
        for _ in range(a.steps):
            wos.run_measure(ctx, inst, x_dev=x)
        torch.cuda.synchronize()
        wos.wos_destroy(ctx)
        print(json.dumps({"kernel_only": True, "steps": a.steps, "copy_bytes": 2 * src.numel() * 8}))
        return
    g = inst.geom
    M = g.n_elem
    n_obs = inst.x_obs.shape[0]
    n1 = int(g.gamma1_mask.sum())
    ctx = wos.wos_create(0)
    dev = "cuda"
    x = wos.device_inputs(inst)
    counts = torch.zeros((n_obs, M), dtype=torch.int32, device=dev)
    stats = torch.zeros(wos.WOS_STATS_WORDS, dtype=torch.int64, device=dev)
    uD = torch.as_tensor(inst.uD, device=dev)
    u0 = torch.as_tensor(inst.u0, device=dev)
    u1 = torch.zeros(n1, dtype=torch.float64, device=dev)
    pred = torch.zeros(n_obs, dtype=torch.float64, device=dev)
    rank = torch.zeros(1, dtype=torch.int32, device=dev)
    sigma = wos.wos_element_measures(g)
    h = wos.wos_svd_create(ctx, n_obs, M, g.gamma1_mask, sigma)
    reg = wos.reg_params(wos.WOS_TSVD_DISCREPANCY, noise_delta=inst.noise_delta, tau=1.1)
    job = wos.measure_job(g, wos.walk_params_of(inst), x, n_obs, counts, stats)
    # launch shape (threads per block, walks per lane): the library default, or the autotuner's
    # choice on a walk sub-range
    tuned = (256, 16, items)
    for prec in (wi.FP32_GEOM_FP64_EXIT, wi.FP64):
        wos.wos_set_tuning(ctx, 2, -1, prec, *tuned)
    if a.autotune:
        tuned = tuple(wos.wos_autotune(ctx, job, max(1, inst.n_walks // 5)))
        log(f"autotuned walk launch shape: block {tuned[0]}, walks per lane {tuned[1]}, items {tuned[2]}")
    # --- timed region: the path pipelined over two CU partitions.  Step i runs its walk kernel on
    # the walk stream and its spectral step (assembly, SVD, reconstruction) on the spectral stream,
    # where it overlaps the walk kernel of step i + 1; buffers alternate between two sets, and a
    # set is reused only after the spectral step that read it has finished.
    walk_s, spec_s = wos.wos_streams_create(ctx, a.spectral_cus)
    sw, ss = torch.cuda.ExternalStream(walk_s), torch.cuda.ExternalStream(spec_s)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    sets = []
    for b in range(2):
        c_b = counts if b == 0 else torch.zeros_like(counts)
        st_b = stats if b == 0 else torch.zeros_like(stats)
        h_b = h if b == 0 else wos.wos_svd_create(ctx, n_obs, M, g.gamma1_mask, sigma)
        sets.append({"counts": c_b, "stats": st_b, "h": h_b, "u1": u1 if b == 0 else torch.zeros_like(u1),
                     "pred": pred if b == 0 else torch.zeros_like(pred),
                     "rank": rank if b == 0 else torch.zeros_like(rank)})
    wp = wos.walk_params_of(inst)
    spec_done = [None, None]
    walk_ev = []

    def step(i, timed):
        S = sets[i % 2]
        if spec_done[i % 2] is not None:
            sw.wait_event(spec_done[i % 2])
        with torch.cuda.stream(sw):
            S["counts"].zero_()
            S["stats"].zero_()
        if timed:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sw)
        wos.wos_build_measure(ctx, g, wp, x, n_obs, S["counts"], S["stats"], None, walk_s)
        walked = torch.cuda.Event()
        walked.record(sw)
        if timed:
            e1.record(sw)
            walk_ev.append((e0, e1))
        ss.wait_event(walked)
        wos.wos_svd(ctx, S["h"], S["counts"], inst.n_walks, spec_s)
        wos.wos_reconstruct(ctx, S["h"], S["counts"], inst.n_walks, uD, u0, reg, S["u1"], S["pred"], S["rank"],
                            None, spec_s)
        done = torch.cuda.Event()
        done.record(ss)
        spec_done[i % 2] = done

    log(f"pipelined path on {n_cu - a.spectral_cus} + {a.spectral_cus} CUs; warmup")
    for i in range(a.warmup):
        step(i, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(a.warmup + i, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    walk_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in walk_ev]))
    walks_step = n_obs * inst.n_walks
    steps_step, lane_slots, fp64_evals = 0, 0, 0
    for S in sets:
        st = wos.stats_dict(S["stats"])
        assert st["walks"] == walks_step, st
        steps_step = st["steps"]
        lane_slots = st["lane_slots"]
        fp64_evals = st["fp64_evals"]
    last = sets[(a.warmup + a.steps - 1) % 2]
    ms_step = elapsed / a.steps * 1e3
    u1_h = last["u1"].cpu().numpy()
    err = float(np.abs(u1_h - inst.u_exact_g1).max() / np.abs(inst.u_exact_g1).max())
    rank_used = int(last["rank"].item())
    log(f"timed {a.steps} pipelined steps: {ms_step:.2f} ms/step; walk kernel {walk_ms:.3f} ms")

    # --- one step at a time (latency): the whole path of one instance as one captured HIP graph
    plan = wos.wos_plan_create(ctx, job, h, uD, u0, reg, u1, pred, rank)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        wos.wos_plan_launch(plan, stream)
    torch.cuda.synchronize()
    lat = []
    for _ in range(5):
        t1 = time.perf_counter()
        wos.wos_plan_launch(plan, stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    latency_ms = float(np.median(lat))

    # the walk kernel alone on the whole device: HIP events on the launch stream
    def time_walks(precision, reps, radius_mode=None):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w = wos.walk_params_of(inst, precision=precision, radius_mode=radius_mode)
        ms = []
        for r in range(reps + 1):
            counts.zero_()
            stats.zero_()
            ev0.record(stream)
            wos.wos_build_measure(ctx, g, w, x, n_obs, counts, stats, None, stream)
            ev1.record(stream)
            ev1.synchronize()
            if r:
                ms.append(ev0.elapsed_time(ev1))
        return float(np.mean(ms)), wos.stats_dict(stats)

    # the spectral step alone (assemble + SVD) on the last step's counts, HIP events on the stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    svd_ms = []
    for r in range(4):
        ev0.record(stream)
        wos.wos_svd(ctx, h, counts, inst.n_walks, stream)
        ev1.record(stream)
        ev1.synchronize()
        if r:
            svd_ms.append(ev0.elapsed_time(ev1))
    sweeps, svd_err, method = wos.wos_svd_info(h, stream)
    svd_info = {"ms": float(np.mean(svd_ms)), "sweeps": sweeps, "error_flag": svd_err,
                "method": "gram" if method == wos.WOS_SVD_GRAM else "hestenes"}
    full_ms, st32 = time_walks(wi.FP32_GEOM_FP64_EXIT, 3)
    walk64_ms, st64 = time_walks(wi.FP64, 3)
    # the same workload with the mapped-bound radius (a larger inscribed ellipsoid per step, same exit
    # law): walk kernel alone, and the reconstruction from its counts
    mb_ms, stmb = time_walks(wi.FP32_GEOM_FP64_EXIT, 3, radius_mode=wos.WOS_RADIUS_MAPPED_BOUND)
    wos.wos_svd(ctx, h, counts, inst.n_walks, stream)
    wos.wos_reconstruct(ctx, h, counts, inst.n_walks, uD, u0, reg, u1, pred, rank, None, stream)
    err_mb = float(np.abs(u1.cpu().numpy() - inst.u_exact_g1).max() / np.abs(inst.u_exact_g1).max())
    mapped_bound = {"fp32_ms": mb_ms, "fp32_walks_per_s": walks_step / (mb_ms * 1e-3),
                    "mean_steps_per_walk": stmb["steps"] / walks_step,
                    "woe_bound_mean_steps_per_walk": st32["steps"] / walks_step,
                    "escapes": stmb["escapes"], "max_rel_err_u1": err_mb, "rank": int(rank.item())}
    log(f"mapped-bound radius: walk kernel {mb_ms:.3f} ms, {mapped_bound['mean_steps_per_walk']:.2f} steps/walk")
    ops = steps_step * OPS_PER_STEP_2D_FP32 + walks_step * OPS_PER_WALK
    achieved = ops / (walk_ms * 1e-3)
    traffic, traffic_detail = measured_traffic(tuned)
    walk_cus = n_cu - a.spectral_cus
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
            "frac": achieved / VALU_PEAK_OPS, "traffic": traffic, "traffic_detail": traffic_detail,
            "algorithmic_bytes": n_obs * ALGO_BYTES_PER_POINT,
            "kernel": "walk_kernel<float,2,annulus>", "avg_ms": walk_ms, "cus": walk_cus,
            "frac_of_partition": achieved / (VALU_PEAK_OPS * walk_cus / n_cu),
            "whole_device": {"avg_ms": full_ms, "frac": ops / (full_ms * 1e-3) / VALU_PEAK_OPS},
            "ops_per_step": OPS_PER_STEP_2D_FP32, "ops_per_walk": OPS_PER_WALK,
            "simd_efficiency": steps_step / max(lane_slots, 1),
            "launch_shape": {"block": tuned[0], "walks_per_lane": tuned[1], "items": ITEM_MODES[tuned[2]]}}

    out = {
        "metric": "walks/s (whole path: walks + SVD + TSVD reconstruction)",
        "value": walks_step * a.steps / elapsed,
        "unit": "walks/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "dtype_detail": "f32 walk geometry; f64 exit test, binning, SVD and reconstruction",
        "data": "synthetic",
        "config": {"workload": "annulus r in [0.3,1], K=[[1,.5],[.5,2]], 128+128 arcs, 1024 points uniform "
                               "by area, N=1e5 walks/point, eps=1e-4, FP32 geometry + FP64 exit; FP64 SVD of "
                               "the 1024x192 Gamma_1 block; TSVD (discrepancy) reconstruction of u_1",
                   "n_obs": n_obs, "n_walks": inst.n_walks, "n_elem": M, "eps": inst.eps},
        "sphere_steps_per_s": steps_step * a.steps / elapsed,
        "pipeline": {"walk_cus": walk_cus, "spectral_cus": a.spectral_cus, "buffer_sets": 2,
                     "step_latency_ms": latency_ms},
        "walk_kernel": {"fp32_ms": full_ms, "fp32_walks_per_s": walks_step / (full_ms * 1e-3),
                        "fp32_steps_per_s": st32["steps"] / (full_ms * 1e-3),
                        "fp64_ms": walk64_ms, "fp64_walks_per_s": walks_step / (walk64_ms * 1e-3),
                        "fp64_steps_per_s": st64["steps"] / (walk64_ms * 1e-3),
                        "fp32_fp64_evals": st32["fp64_evals"], "escapes": st32["escapes"] + st64["escapes"]},
        "svd": svd_info,
        "reconstruction": {"rank": rank_used, "max_rel_err_u1": err},
        "mapped_bound_radius": mapped_bound,
        "roofline": roof,
    }
    if not a.no_serve:
        log("serving runs")
        out["serving"] = serving(ctx, wos, wi, a.serve_seconds, a.serve_rate, a.serve_svd, a.serve_radius)
    if not a.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(inst, a.cpu_seconds)
    wos.wos_plan_destroy(plan)
    torch.cuda.synchronize()
    wos.wos_streams_destroy(ctx, walk_s, spec_s)
    for S in sets:
        wos.wos_svd_destroy(ctx, S["h"])
    wos.wos_destroy(ctx)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
