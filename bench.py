"""Benchmark: the whole hot path on one MI355X.

Workload (default, --workload cube): the unit cube [0,1]^3 with K = Q diag(1, 3, 10) Q^T (Q Haar,
seed 1), each face split into 24 x 24 patches (3456 cells; Gamma_1 = the faces x = 1, y = 1, z = 1,
1728 cells), 4096 observation points on the 16^3 interior grid, N = 1e5 walks per point
(4.1e8 walks per step), eps = 1e-4; FP32 walk geometry with the exact mapped radius (the largest
ellipsoid x + r S B(0, 1) inside the cube) and the FP64 exit test and binning; then the FP64 SVD of
the 4096 x 1728 Gamma_1 block and the TSVD reconstruction (discrepancy principle) of u_1 from data
with 1 % noise.  One step = zero counts + walk kernel + assembly + SVD + reconstruction; the timed
steps are pipelined over two CU partitions (the walks of step i + 1 on 128 CUs beside the
assembly, SVD and reconstruction of step i on the other 128, two buffer sets), and the steps run
one after the other on one stream are reported beside them (--no-pipeline makes those the
headline); the points and data are resident in HBM.  --workload annulus: the 2D annulus (1024 x
1e5 walks, 1024 x 192 block), pipelined the same way with 8 spectral CUs.

Prints one JSON line.  `roofline` is that of the step's dominant kernel (the device-wide Jacobi of
the SVD on the cube), measured live with HIP events on its stream; the walk kernel's roofline, the
plain FP64 walk path, the r = dist (walk-on-ellipsoids bound) chain, the serving loop and the CPU
oracle baseline are reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walks/s & sphere-steps/s (FP32 vs FP64 WoS, ε=1e-4); p50/p99 solve latency"

# Algorithmic 32-bit VALU operations per sphere step, counted from the method (an FMA counts once).
# 2D FP32 annulus: Philox4x32-10 = 10 rounds x (2 mul-lo + 2 mul-hi + 4 xor) = 80 ops per block, one
# block per 4 steps -> 20; uniform 3; cos, sin 2; shrunken radius 1; x += r S U 6; annulus
# distance 8; exit / band / cap tests and step count 4.
OPS_PER_STEP_2D_FP32 = 20 + 3 + 2 + 1 + 6 + 8 + 4
# 3D FP32 box with the exact mapped radius: Philox 80 ops per block, one block per 2 steps -> 40;
# two uniforms (shift, convert, scale) 6; direction z = 1 - 2 u, (1 - z)(1 + z), clamp, sqrt, cos,
# sin, two products 10; mapped radius min_a min(x_a - lo_a, hi_a - x_a) / |S e_a|, per axis two
# differences, their min, one product and the running min: 15; shrink 1; x += r S U 12; distance to
# the six faces 11; exit / band tests and step count 5.
OPS_PER_STEP_3D_FP32 = 40 + 6 + 10 + 15 + 1 + 12 + 11 + 5
# Per walk: FP64 projection onto the boundary, cell index and LDS histogram (2D arc 30; 3D box
# face selection and patch index 40).
OPS_PER_WALK_2D, OPS_PER_WALK_3D = 30, 40
# MI355X 32-bit VALU peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6e12 lane-ops/s (the published
# FP32 vector rate, 157.3 TFLOP/s, counts an FMA as two flops; here an FMA is one op).  Integer
# 32 x 32 -> 64 multiplies (Philox) and transcendentals issue at a quarter of that rate.
VALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
# MI355X FP64 vector peak (published): 78.6 TFLOP/s (one FP64 FMA per lane per clock).
FP64_PEAK_FLOPS = 78.6e12

# HBM traffic from rocprofv3 counters (FETCH_SIZE, WRITE_SIZE) per launch of a kernel, with the hash
# of the sources it was measured on; reported only while they match.
SRC = os.path.join(ROOT, "paper_2409_03686_amd", "csrc")
TRAFFIC = {
    "jacobi": (os.path.join(ROOT, "profiles", "grid_jacobi_cube_4096x1728_traffic.txt"),
               [os.path.join(SRC, "linalg_kernels.hip")]),
    "walk_cube": (os.path.join(ROOT, "profiles", "walk_kernel_f32_cube_4096x1e5_traffic.txt"),
                  [os.path.join(SRC, f) for f in ("walk_kernel.hip", "wos_device.hpp")]),
}


def sources_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(which):
    """(bytes per launch, detail) from a committed counter summary, or (None, reason)."""
    path, files = TRAFFIC[which]
    if not os.path.exists(path):
        return None, "no counter summary"
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    try:
        if rec.get("sources_sha256") != sources_hash(files):
            return None, "kernel sources changed since the counters were taken"
        f, w = float(rec["fetch_bytes_per_launch"]), float(rec["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None, "counter summary unreadable"
    return f + w, {"fetch_bytes": f, "write_bytes": w}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--workload", choices=("cube", "annulus"), default="cube")
    p.add_argument("--steps", type=int, default=None, help="timed steps (default: cube 10, annulus 100)")
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--spectral-cus", type=int, default=None,
                   help="CUs of the spectral stream (assembly + SVD + reconstruction) in the pipelined step; the "
                        "walk kernel gets the rest (default: cube 128, annulus 8)")
    p.add_argument("--no-pipeline", action="store_true",
                   help="cube: time the steps one after the other on one stream instead of pipelined")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    p.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch measurement")
    p.add_argument("--no-mesh", action="store_true", help="skip the triangle-mesh measurement")
    p.add_argument("--mesh-only", action="store_true", help="only the triangle-mesh measurement (for profiling)")
    p.add_argument("--serve-seconds", type=float, default=10.0)
    p.add_argument("--serve-svd", type=int, default=1, choices=(0, 1, 2),
                   help="serving SVD: 0 full (cooperative Jacobi), 1 truncated (plain kernels, overlapping), "
                        "2 truncated and certified (full SVD for a rank beyond its certified triplets)")
    p.add_argument("--serve-rate", type=float, default=200.0)
    p.add_argument("--serve-radius", default="mapped", choices=("mapped", "dist"),
                   help="step radius of the serving requests: each kind's mapped radius, or r = dist (the "
                        "cube's exact radius only)")
    p.add_argument("--serve-only", action="store_true", help="only the serving measurement (for profiling)")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target wall time of the CPU sample")
    p.add_argument("--kernel-only", action="store_true",
                   help="for counter collection: one 1 GiB device copy (calibration), the workload's walk kernel "
                        "in FP64 and in FP32, then the SVD --steps times")
    return p.parse_args()


# ----------------------------------------------------------------------------------------- CPU

def cpu_baseline_cube(inst, target_s):
    """The oracle (FP64 walks + LAPACK SVD + TSVD) on a sample of the cube workload: every 16th point x
    the first n walks (n chosen so the walks take about target_s seconds on all host cores), then
    LAPACK's SVD and the TSVD of a full-size 4096 x 1728 block built from those rows (each sampled row
    stands for the 16 it represents).  Walks/s per step = walks per step / (walks per step / the
    sample's walk rate + the linear algebra time)."""
    from oracle import linalg as ol
    from oracle import walks as ow
    cores = len(os.sched_getaffinity(0))
    rows = np.arange(0, inst.x_obs.shape[0], 16)
    kw = dict(seed=inst.seed, radius_mode=inst.radius_mode, point_ids=rows, threads=cores)
    t0 = time.perf_counter()
    ow.build_measure(inst.geom, inst.K, inst.x_obs[rows], inst.eps, walk_end=16, **kw)
    cal = time.perf_counter() - t0
    n = int(max(16, min(inst.n_walks, 16 * target_s / max(cal, 1e-3))))
    t0 = time.perf_counter()
    counts, st, _ = ow.build_measure(inst.geom, inst.K, inst.x_obs[rows], inst.eps, walk_end=n, **kw)
    t_walk = time.perf_counter() - t0
    rate = st["walks"] / t_walk
    full = np.repeat(counts, 16, axis=0)
    sigma = ow.element_measures(inst.geom)
    t0 = time.perf_counter()
    out = ol.assemble(full, n, inst.geom.gamma1_mask, sigma, uD=inst.uD, u0=inst.u0)
    U, s, Vt = ol.svd(out["B"])
    g1 = inst.geom.gamma1_mask.astype(bool)
    ol.reconstruct(U, s, Vt, sigma[g1], out["q"], kind=ol.TSVD_DISCREPANCY, delta=inst.noise_delta, tau=1.1)
    t_lin = time.perf_counter() - t0
    walks_step = inst.x_obs.shape[0] * inst.n_walks
    t_step = walks_step / rate + t_lin
    return {"value": walks_step / t_step, "unit": "walks/s", "cores": cores, "kind": "oracle",
            "sample": f"every 16th point ({len(rows)}) x first {n} walks (of {inst.n_walks}), FP64 walks "
                      f"{t_walk:.2f} s ({rate:.3e} walks/s); LAPACK SVD + TSVD of the full 4096 x 1728 block "
                      f"{t_lin:.2f} s; per step {t_step:.1f} s extrapolated",
            "steps_per_s": st["steps"] / t_walk, "linear_algebra_s": t_lin}


def cpu_baseline_annulus(inst, target_s):
    """The oracle on a sample of the annulus workload: every point, the first n walks, then LAPACK's
    SVD + TSVD of the sample's block."""
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


# ----------------------------------------------------------------------------------------- serving

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
    errs = []
    for k, (inst, o) in enumerate(zip(insts, out)):
        if o.status == 0 and inst.u_exact_g1 is not None:
            u1 = keep[6 * k + 5]
            errs.append(float(np.abs(u1 - inst.u_exact_g1).max() / max(np.abs(inst.u_exact_g1).max(), 1e-300)))
    return {"requests": len(out), "completed": len(ok), "svd_fallbacks": sum(o.svd_fallback for o in ok),
            "median_rel_err_u1": float(np.median(errs)) if errs else None,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "walks_per_s": sum(o.walks for o in ok) / wall,
            "steps_per_s": sum(o.steps for o in ok) / wall, "wall_s": wall}, keep


def _oracle_errors(wos, insts, keep, n_sample=20):
    """The oracle's reconstruction error on sampled served requests: the same noisy data, the oracle's
    own walks (FP64, the request's Philox keys) and LAPACK's SVD with the same discrepancy rule; the
    served error beside it.  Requests small enough for the host (at most 2e7 walks) are sampled."""
    from oracle import linalg as ol
    from oracle import walks as ow
    cores = len(os.sched_getaffinity(0))
    idx = [k for k, i in enumerate(insts) if i.x_obs.shape[0] * i.n_walks <= 2e7][:n_sample]
    rows = []
    for k in idx:
        inst = insts[k]
        counts, _, _ = ow.build_instance(inst, threads=cores)
        sigma = ow.element_measures(inst.geom)
        g1 = inst.geom.gamma1_mask.astype(bool)
        out = ol.assemble(counts, inst.n_walks, inst.geom.gamma1_mask, sigma, uD=inst.uD, u0=inst.u0)
        U, s, Vt = ol.svd(out["B"])
        u1r, rr, _ = ol.reconstruct(U, s, Vt, sigma[g1], out["q"], kind=ol.TSVD_DISCREPANCY,
                                    delta=inst.noise_delta, tau=1.1)
        ue = inst.u_exact_g1
        served = keep[6 * k + 5]
        rows.append((float(np.abs(u1r - ue).max() / np.abs(ue).max()),
                     float(np.abs(served - ue).max() / np.abs(ue).max())))
    if not rows:
        return None
    o = np.array(rows)
    return {"requests": len(rows), "median_rel_err_u1_oracle": float(np.median(o[:, 0])),
            "median_rel_err_u1_served": float(np.median(o[:, 1])),
            "per_request": [{"oracle": a, "served": b} for a, b in rows]}


def serving(ctx, wos, wi, seconds, rate=200.0, svd_mode=1, radius="mapped", oracle_sample=True):
    """Request serving on the heterogeneous-instance generator (kinds, conductivities, sizes and walk
    budgets drawn per request; 1-5 % noise; random harmonic data of degree <= 6): each request is
    build H + FP64 SVD + TSVD reconstruction, host buffers in and out.  Capacity = requests per
    second with every request queued at t = 0; then open-loop Poisson arrivals at `rate` for
    `seconds`, and, when that load exceeds the capacity, at 0.8 x capacity as well."""
    arr = wi.cfg5_arrivals(rate=rate, duration_s=seconds, seed=5)
    rng = np.random.default_rng(5)
    mapped = radius == "mapped"
    insts = [wi.random_instance(rng, i, mapped_radii=mapped) for i in range(len(arr))]
    cap, _ = _serve(ctx, wos, insts, np.zeros(len(insts)), svd_mode)
    capacity = cap["completed"] / cap["wall_s"]
    offered, keep = _serve(ctx, wos, insts, arr, svd_mode)
    mean_walks = float(np.mean([i.x_obs.shape[0] * i.n_walks for i in insts]))
    out = {"svd_mode": svd_mode, "radius": radius, "duration_s": seconds, "capacity_req_s": capacity,
           "capacity_walks_per_s": cap["walks_per_s"], "capacity_steps_per_s": cap["steps_per_s"],
           "mean_walks_per_request": mean_walks, "offered_rate_req_s": rate, "utilisation": rate / capacity,
           "at_offered_rate": offered}
    if oracle_sample:
        out["oracle_error_sample"] = _oracle_errors(wos, insts, keep)
    if rate >= capacity:
        r8 = 0.8 * capacity
        arr8 = wi.cfg5_arrivals(rate=r8, duration_s=seconds, seed=5)
        while len(insts) < len(arr8):
            insts.append(wi.random_instance(rng, len(insts), mapped_radii=mapped))
        out["at_0.8_capacity"] = dict(_serve(ctx, wos, insts[:len(arr8)], arr8, svd_mode)[0], rate_req_s=r8)
    return out


# ----------------------------------------------------------------------------------------- batch

def bench_batch(ctx, wos, wi, torch, reps=3):
    """The 64-instance heterogeneous batch at its full walk budgets: disks, ellipses, L-shapes,
    annuli, balls and cubes with random conductivities (condition numbers 1-20), 32-2048 points,
    64-2048 cells and 1e3-1e5 walks per point, FP32 geometry with each kind's mapped radius.  Each
    (dimension, kind) is autotuned on a sample, then the whole batch (one persistent launch per
    dimension) is captured as one HIP graph and replayed `reps` times, timed with HIP events."""
    insts = wi.cfg4_batch()
    stream = torch.cuda.current_stream()
    jobs, keep = [], []
    for inst in insts:
        M = wos.wos_element_count(inst.geom)
        x = wos.device_inputs(inst)
        cnt = torch.zeros((x.shape[0], M), dtype=torch.int32, device="cuda")
        stt = torch.zeros(wos.WOS_STATS_WORDS, dtype=torch.int64, device="cuda")
        keep += [x, cnt, stt]
        jobs.append(wos.measure_job(inst.geom, wos.walk_params_of(inst), x, x.shape[0], cnt, stt))
    walks = sum(i.x_obs.shape[0] * i.n_walks for i in insts)
    tuned = {}
    t0 = time.perf_counter()
    for inst, job in zip(insts, jobs):
        key = (inst.geom.dim, wi.KIND_NAMES[inst.geom.kind])
        if key not in tuned:
            block, wpl, items = wos.wos_autotune(ctx, job, 2000)
            tuned[key] = {"block": block, "walks_per_lane": wpl, "items": items}
    tune_s = time.perf_counter() - t0
    plan = wos.wos_plan_create_batch(ctx, jobs)
    wos.wos_plan_launch(plan, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(stream)
        wos.wos_plan_launch(plan, stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    wos.wos_plan_destroy(plan)
    sts = [wos.stats_dict(keep[3 * k + 2]) for k in range(len(insts))]
    assert all(st["walks"] == i.x_obs.shape[0] * i.n_walks for st, i in zip(sts, insts))
    steps = sum(st["steps"] for st in sts)
    steps_2d = sum(st["steps"] for st, i in zip(sts, insts) if i.geom.dim == 2)
    walks_2d = sum(i.x_obs.shape[0] * i.n_walks for i in insts if i.geom.dim == 2)
    ops = (steps_2d * OPS_PER_STEP_2D_FP32 + (steps - steps_2d) * OPS_PER_STEP_3D_FP32
           + walks_2d * OPS_PER_WALK_2D + (walks - walks_2d) * OPS_PER_WALK_3D)
    lane_slots = sum(st["lane_slots"] for st in sts)
    return {"instances": len(insts), "walks": walks, "sphere_steps": steps, "ms_per_launch": ms,
            "walks_per_s": walks / (ms * 1e-3), "sphere_steps_per_s": steps / (ms * 1e-3),
            "launch": "one HIP graph: zero-fill + one persistent walk launch per dimension", "replays": reps,
            "autotune_s": tune_s, "tuning": {f"{d}D {k}": v for (d, k), v in tuned.items()},
            "roofline": {"bound": "alu", "achieved": ops / (ms * 1e-3) / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                         "unit": "Tops/s", "frac": ops / (ms * 1e-3) / VALU_PEAK_OPS,
                         "ops": "approximate: every 2D step priced at the annulus count, every 3D step at the box "
                                "count, per walk the arc / face binning counts",
                         "simd_efficiency": steps / max(lane_slots, 1)}}


# ----------------------------------------------------------------------------------------- cube

def bench_mesh(ctx, wos, wi, torch, box_steps_per_s, walks=10_000, reps=2):
    """The cube workload's domain as a closed triangle mesh (each of the 3456 patches two triangles:
    6912 triangles, the same cells), its 4096 points and K, 1e4 walks per point: the walk kernel with
    the BVH nearest-triangle search at r = dist in FP32 and FP64, beside the box kind's closed-form
    distance at r = dist (the same chain), and in FP32 with the mapped-exact radius (a second search
    over the mapped triangles each step)."""
    inst = wi.cfg3_cube(n_walks=walks)
    g = inst.geom
    gm = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.box_mesh(np.array(g.params[:3]), np.array(g.params[3:6]),
                                                                 g.layout[0]))
    M = gm.n_elem
    n_obs = inst.x_obs.shape[0]
    x = wos.device_inputs(inst)
    counts = torch.zeros((n_obs, M), dtype=torch.int32, device="cuda")
    stats = torch.zeros(wos.WOS_STATS_WORDS, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    mi = wi.Instance(gm, inst.K, inst.x_obs, walks, eps=inst.eps, seed=inst.seed)
    out = {"geometry": f"cube surface as {gm.n_tri} triangles (two per patch, the same {M} cells)",
           "walks_per_point": walks, "radius": "r = dist (fp32, fp64); mapped exact (fp32_mapped_exact)"}
    for name, prec, rm in (("fp32", wi.FP32_GEOM_FP64_EXIT, wos.WOS_RADIUS_WOE_BOUND),
                           ("fp64", wi.FP64, wos.WOS_RADIUS_WOE_BOUND),
                           ("fp32_mapped_exact", wi.FP32_GEOM_FP64_EXIT, wos.WOS_RADIUS_MAPPED_EXACT)):
        w = wos.walk_params_of(mi, precision=prec, radius_mode=rm)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            counts.zero_()
            stats.zero_()
            ev0.record()
            wos.wos_build_measure(ctx, gm, w, x, n_obs, counts, stats, None, stream)
            ev1.record()
            ev1.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        st = wos.stats_dict(stats)
        t = float(np.mean(ms))
        out[name] = {"ms": t, "walks_per_s": st["walks"] / (t * 1e-3), "steps_per_s": st["steps"] / (t * 1e-3),
                     "steps_per_walk": st["steps"] / st["walks"], "escapes": st["escapes"]}
    if box_steps_per_s is not None:
        out["box_kind_r_dist_fp32_steps_per_s"] = box_steps_per_s
        out["fp32_step_cost_vs_box_kind"] = box_steps_per_s / out["fp32"]["steps_per_s"]
    log(f"mesh: FP32 {out['fp32']['ms']:.0f} ms, FP64 {out['fp64']['ms']:.0f} ms, FP32 mapped exact "
        f"{out['fp32_mapped_exact']['ms']:.0f} ms for {n_obs} x {walks} walks")
    return out


def bench_cube(a, wos, wi, torch):
    inst = wi.cfg3_cube(precision=wi.FP32_GEOM_FP64_EXIT)
    g = inst.geom
    M = g.n_elem
    n_obs = inst.x_obs.shape[0]
    n1 = int(g.gamma1_mask.sum())
    steps = a.steps or 10
    ctx = wos.wos_create(0)
    dev = "cuda"
    stream = torch.cuda.current_stream()
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
    wp = wos.walk_params_of(inst)
    if a.kernel_only:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        wos.wos_build_measure(ctx, g, wos.walk_params_of(inst, precision=wi.FP64), x, n_obs, counts, stats, None,
                              stream)
        counts.zero_()
        wos.wos_build_measure(ctx, g, wp, x, n_obs, counts, stats, None, stream)
        for _ in range(steps):
            wos.wos_svd(ctx, h, counts, inst.n_walks, stream)
        torch.cuda.synchronize()
        wos.wos_svd_destroy(ctx, h)
        wos.wos_destroy(ctx)
        print(json.dumps({"kernel_only": True, "workload": "cube", "steps": steps, "copy_bytes": 2 * src.numel() * 8}))
        return

    def step():
        counts.zero_()
        stats.zero_()
        wos.wos_build_measure(ctx, g, wp, x, n_obs, counts, stats, None, stream)
        wos.wos_svd(ctx, h, counts, inst.n_walks, stream)
        wos.wos_reconstruct(ctx, h, counts, inst.n_walks, uD, u0, reg, u1, pred, rank, None, stream)

    log(f"cube: {a.warmup} warmup steps")
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    log(f"cube: {steps} timed steps")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / steps * 1e3
    st = wos.stats_dict(stats)
    walks_step = n_obs * inst.n_walks
    assert st["walks"] == walks_step, st
    err = float(np.abs(u1.cpu().numpy() - inst.u_exact_g1).max() / np.abs(inst.u_exact_g1).max())
    rank_used = int(rank.item())
    log(f"cube: {ms_step:.1f} ms/step one after the other")
    seq = {"ms_per_step": ms_step, "walks_per_s": walks_step * steps / elapsed}

    # Steps pipelined over two CU partitions: the walks of step i + 1 on one, the assembly, SVD and
    # reconstruction of step i on the other (128 CUs by default: the device-wide Jacobi needs its
    # 108 workgroups resident, one per CU), two buffer sets, each reused only after the spectral
    # step that read it has finished.
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    spec_cus = a.spectral_cus or 128
    pipe = None
    if not a.no_pipeline:
        walk_s, spec_s = wos.wos_streams_create(ctx, spec_cus)
        sw, ss = torch.cuda.ExternalStream(walk_s), torch.cuda.ExternalStream(spec_s)
        sets = [{"counts": torch.zeros((n_obs, M), dtype=torch.int32, device=dev),
                 "stats": torch.zeros(wos.WOS_STATS_WORDS, dtype=torch.int64, device=dev),
                 "h": wos.wos_svd_create(ctx, n_obs, M, g.gamma1_mask, sigma),
                 "u1": torch.zeros(n1, dtype=torch.float64, device=dev),
                 "pred": torch.zeros(n_obs, dtype=torch.float64, device=dev),
                 "rank": torch.zeros(1, dtype=torch.int32, device=dev)} for _ in range(2)]
        spec_done = [None, None]

        def pstep(i):
            S = sets[i % 2]
            if spec_done[i % 2] is not None:
                sw.wait_event(spec_done[i % 2])
            with torch.cuda.stream(sw):
                S["counts"].zero_()
                S["stats"].zero_()
            wos.wos_build_measure(ctx, g, wp, x, n_obs, S["counts"], S["stats"], None, walk_s)
            walked = torch.cuda.Event()
            walked.record(sw)
            ss.wait_event(walked)
            wos.wos_svd(ctx, S["h"], S["counts"], inst.n_walks, spec_s)
            wos.wos_reconstruct(ctx, S["h"], S["counts"], inst.n_walks, uD, u0, reg, S["u1"], S["pred"], S["rank"],
                                None, spec_s)
            done = torch.cuda.Event()
            done.record(ss)
            spec_done[i % 2] = done

        log(f"cube: pipelined steps ({n_cu - spec_cus} walk CUs, {spec_cus} spectral CUs)")
        for i in range(a.warmup):
            pstep(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            pstep(a.warmup + i)
        torch.cuda.synchronize()
        elapsed_p = time.perf_counter() - t0
        last = sets[(a.warmup + steps - 1) % 2]
        st_p = wos.stats_dict(last["stats"])
        assert st_p["walks"] == walks_step, st_p
        err_p = float(np.abs(last["u1"].cpu().numpy() - inst.u_exact_g1).max() / np.abs(inst.u_exact_g1).max())
        del sw, ss, spec_done
        torch.cuda.synchronize()
        wos.wos_streams_destroy(ctx, walk_s, spec_s)
        for S in sets:
            wos.wos_svd_destroy(ctx, S["h"])
        pipe = {"walk_cus": n_cu - spec_cus, "spectral_cus": spec_cus, "buffer_sets": 2,
                "ms_per_step": elapsed_p / steps * 1e3, "max_rel_err_u1": err_p, "rank": int(last["rank"].item())}
        log(f"cube: {pipe['ms_per_step']:.1f} ms/step pipelined")

    # the step's parts, one at a time, with HIP events on the launch stream
    def time_walks(precision, reps, radius_mode=None):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w = wos.walk_params_of(inst, precision=precision, radius_mode=radius_mode)
        ms = []
        for r in range(reps):
            counts.zero_()
            stats.zero_()
            ev0.record(stream)
            wos.wos_build_measure(ctx, g, w, x, n_obs, counts, stats, None, stream)
            ev1.record(stream)
            ev1.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        return float(np.mean(ms)), wos.stats_dict(stats)

    walk_ms, st32 = time_walks(wi.FP32_GEOM_FP64_EXIT, 3)
    jac, svd_tot, nrot = [], [], 0
    for _ in range(3):
        wos.wos_svd(ctx, h, counts, inst.n_walks, stream)
        jm, tm, nrot = wos.wos_svd_timing(h)
        jac.append(jm)
        svd_tot.append(tm)
    jac_ms, svd_ms = float(np.mean(jac)), float(np.mean(svd_tot))
    sweeps, svd_err, method = wos.wos_svd_info(h, stream)
    gs, ge, check, resid = wos.wos_svd_gram_check(h, stream)
    _, s_ptr, _, _, _, k = wos.wos_svd_factors(h)
    s_host = wos.device_to_numpy(s_ptr, k, np.float64)
    log(f"cube: walk kernel {walk_ms:.2f} ms, SVD {svd_ms:.1f} ms (Jacobi {jac_ms:.1f} ms, {sweeps} sweeps)")
    walk64_ms, st64 = time_walks(wi.FP64, 2)
    woe_ms, stwoe = time_walks(wi.FP32_GEOM_FP64_EXIT, 2, radius_mode=wos.WOS_RADIUS_WOE_BOUND)
    log(f"cube: FP64 walks {walk64_ms:.1f} ms, r = dist walks {woe_ms:.1f} ms")

    # one step alone (latency): the whole path of one instance as one captured HIP graph
    job = wos.measure_job(g, wp, x, n_obs, counts, stats)
    plan = wos.wos_plan_create(ctx, job, h, uD, u0, reg, u1, pred, rank)
    for _ in range(2):
        wos.wos_plan_launch(plan, stream)
    torch.cuda.synchronize()
    lat = []
    for _ in range(3):
        t1 = time.perf_counter()
        wos.wos_plan_launch(plan, stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    wos.wos_plan_destroy(plan)
    latency_ms = float(np.median(lat))

    # roofline of the dominant kernel (the device-wide Jacobi of the SVD): algorithmic FP64 flops =
    # every pair visit's dot product (2 flops per row) + every applied rotation (6 flops per row)
    ncol = n1
    npx = ((ncol + 63) // 64) * 64  # rows of the factor X
    flops = gs * (ncol * (ncol - 1) // 2) * 2.0 * npx + nrot * 6.0 * npx
    achieved = flops / (jac_ms * 1e-3)
    traffic, traffic_detail = measured_traffic("jacobi")
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_PEAK_FLOPS / 1e12, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_FLOPS, "traffic": traffic, "traffic_detail": traffic_detail,
            "algorithmic_bytes": 2 * 8 * npx * npx,
            "kernel": "gram_jacobi_grid_kernel<7,8,256> (one-sided Jacobi of the 1728 x 1728 Cholesky factor)",
            "avg_ms": jac_ms, "sweeps": gs, "rotations": nrot, "flops_per_launch": flops,
            "note": "FP64 vector arithmetic (plane rotations), peak = FP64 vector rate"}
    ops = st32["steps"] * OPS_PER_STEP_3D_FP32 + walks_step * OPS_PER_WALK_3D
    wtraffic, wtraffic_detail = measured_traffic("walk_cube")
    roof_walk = {"bound": "alu", "achieved": ops / (walk_ms * 1e-3) / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                 "unit": "Tops/s", "frac": ops / (walk_ms * 1e-3) / VALU_PEAK_OPS, "traffic": wtraffic,
                 "traffic_detail": wtraffic_detail, "algorithmic_bytes": n_obs * (24 + M * 4),
                 "kernel": "walk_kernel<float,3,box>", "avg_ms": walk_ms, "ops_per_step": OPS_PER_STEP_3D_FP32,
                 "ops_per_walk": OPS_PER_WALK_3D, "simd_efficiency": st32["steps"] / max(st32["lane_slots"], 1)}
    t_step = pipe["ms_per_step"] if pipe else ms_step
    out = {
        "metric": METRIC,
        "value": walks_step / (t_step * 1e-3),
        "unit": "walks/s",
        "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": t_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "dtype_detail": "f32 walk geometry; f64 exit test, binning, SVD and reconstruction",
        "data": "synthetic",
        "config": {"workload": "cube [0,1]^3, K = Q diag(1,3,10) Q^T (Haar Q, seed 1), 24x24 patches per face "
                               "(3456 cells, Gamma_1 = faces x=1, y=1, z=1), 4096 points on the 16^3 grid, "
                               "N=1e5 walks/point, eps=1e-4, FP32 geometry (exact mapped radius) + FP64 exit; "
                               "FP64 SVD of the 4096x1728 Gamma_1 block; TSVD (discrepancy) reconstruction of "
                               "u_1 from 1 % noisy data",
                   "n_obs": n_obs, "n_walks": inst.n_walks, "n_elem": M, "eps": inst.eps},
        "sphere_steps_per_s": st["steps"] / (t_step * 1e-3),
        "pipeline": pipe, "sequential": seq,
        "step": {"walk_kernel_ms": walk_ms, "svd_ms": svd_ms, "jacobi_ms": jac_ms,
                 "latency_one_step_graph_ms": latency_ms},
        "walk_kernel": {"fp32_ms": walk_ms, "fp32_walks_per_s": walks_step / (walk_ms * 1e-3),
                        "fp32_steps_per_s": st32["steps"] / (walk_ms * 1e-3),
                        "fp32_steps_per_walk": st32["steps"] / walks_step,
                        "fp64_ms": walk64_ms, "fp64_walks_per_s": walks_step / (walk64_ms * 1e-3),
                        "fp64_steps_per_s": st64["steps"] / (walk64_ms * 1e-3),
                        "fp32_fp64_evals": st32["fp64_evals"], "escapes": st32["escapes"] + st64["escapes"],
                        "woe_bound_fp32_ms": woe_ms, "woe_bound_walks_per_s": walks_step / (woe_ms * 1e-3),
                        "woe_bound_steps_per_walk": stwoe["steps"] / walks_step},
        "svd": {"ms": svd_ms, "sweeps": sweeps, "error_flag": svd_err,
                "method": "gram" if method == wos.WOS_SVD_GRAM else "hestenes", "gram_check": check,
                "residual_certificate_rel_s1": resid / s_host[0], "s_min_over_s1": float(s_host[-1] / s_host[0])},
        "reconstruction": {"rank": rank_used, "max_rel_err_u1": err},
        "roofline": roof,
        "roofline_walk_kernel": roof_walk,
    }
    return ctx, inst, out, h


# ----------------------------------------------------------------------------------------- annulus

def bench_annulus(a, wos, wi, torch):
    inst = wi.cfg2_annulus(precision=wi.FP32_GEOM_FP64_EXIT)
    g = inst.geom
    M = g.n_elem
    n_obs = inst.x_obs.shape[0]
    n1 = int(g.gamma1_mask.sum())
    steps = a.steps or 100
    ctx = wos.wos_create(0)
    dev = "cuda"
    x = wos.device_inputs(inst)
    sigma = wos.wos_element_measures(g)
    reg = wos.reg_params(wos.WOS_TSVD_DISCREPANCY, noise_delta=inst.noise_delta, tau=1.1)
    wp = wos.walk_params_of(inst)
    # steps pipelined over two CU partitions: step i's walks on the walk stream, its spectral step
    # (assembly, SVD, reconstruction) on the spectral stream beside step i + 1's walks; two buffer
    # sets, a set reused only after the spectral step that read it has finished
    spec_cus = a.spectral_cus or 8
    walk_s, spec_s = wos.wos_streams_create(ctx, spec_cus)
    sw, ss = torch.cuda.ExternalStream(walk_s), torch.cuda.ExternalStream(spec_s)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    sets = []
    for _ in range(2):
        sets.append({"counts": torch.zeros((n_obs, M), dtype=torch.int32, device=dev),
                     "stats": torch.zeros(wos.WOS_STATS_WORDS, dtype=torch.int64, device=dev),
                     "h": wos.wos_svd_create(ctx, n_obs, M, g.gamma1_mask, sigma),
                     "u1": torch.zeros(n1, dtype=torch.float64, device=dev),
                     "pred": torch.zeros(n_obs, dtype=torch.float64, device=dev),
                     "rank": torch.zeros(1, dtype=torch.int32, device=dev)})
    uD = torch.as_tensor(inst.uD, device=dev)
    u0 = torch.as_tensor(inst.u0, device=dev)
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

    for i in range(a.warmup):
        step(i, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(a.warmup + i, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    walk_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in walk_ev]))
    walks_step = n_obs * inst.n_walks
    st = wos.stats_dict(sets[0]["stats"])
    last = sets[(a.warmup + steps - 1) % 2]
    err = float(np.abs(last["u1"].cpu().numpy() - inst.u_exact_g1).max() / np.abs(inst.u_exact_g1).max())
    jm, tm, _ = wos.wos_svd_timing(last["h"])
    # release the torch wrappers of the partition's streams and events before the streams go
    del sw, ss, walk_ev, spec_done
    torch.cuda.synchronize()
    wos.wos_streams_destroy(ctx, walk_s, spec_s)
    ops = st["steps"] * OPS_PER_STEP_2D_FP32 + walks_step * OPS_PER_WALK_2D
    walk_cus = n_cu - spec_cus
    out = {
        "metric": METRIC, "value": walks_step * steps / elapsed, "unit": "walks/s",
        "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "dtype_detail": "f32 walk geometry; f64 exit test, binning, SVD and reconstruction", "data": "synthetic",
        "config": {"workload": "annulus r in [0.3,1], K=[[1,.5],[.5,2]], 128+128 arcs, 1024 points uniform "
                               "by area, N=1e5 walks/point, eps=1e-4, FP32 geometry + FP64 exit; FP64 SVD of "
                               "the 1024x192 Gamma_1 block; TSVD (discrepancy) reconstruction of u_1",
                   "n_obs": n_obs, "n_walks": inst.n_walks, "n_elem": M, "eps": inst.eps},
        "sphere_steps_per_s": st["steps"] * steps / elapsed,
        "pipeline": {"walk_cus": walk_cus, "spectral_cus": spec_cus, "buffer_sets": 2},
        "svd": {"ms": tm, "jacobi_ms": jm}, "reconstruction": {"max_rel_err_u1": err},
        "roofline": {"bound": "alu", "achieved": ops / (walk_ms * 1e-3) / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": ops / (walk_ms * 1e-3) / VALU_PEAK_OPS, "traffic": None,
                     "kernel": "walk_kernel<float,2,annulus>", "avg_ms": walk_ms, "cus": walk_cus,
                     "ops_per_step": OPS_PER_STEP_2D_FP32, "ops_per_walk": OPS_PER_WALK_2D},
    }
    for S in sets:
        wos.wos_svd_destroy(ctx, S["h"])
    return ctx, inst, out, None


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import wos_inputs as wi
    from paper_2409_03686_amd import wos

    torch.cuda.set_device(0)
    if a.mesh_only:
        ctx = wos.wos_create(0)
        print(json.dumps({"mesh_only": True, "mesh": bench_mesh(ctx, wos, wi, torch, None, reps=1)}))
        wos.wos_destroy(ctx)
        return
    if a.serve_only:
        ctx = wos.wos_create(0)
        print(json.dumps({"serve_only": True, "serving": serving(ctx, wos, wi, a.serve_seconds, a.serve_rate,
                                                                 a.serve_svd, a.serve_radius, oracle_sample=False)}))
        wos.wos_destroy(ctx)
        return
    if a.workload == "cube":
        res = bench_cube(a, wos, wi, torch)
    else:
        res = bench_annulus(a, wos, wi, torch)
    if res is None:
        return
    ctx, inst, out, h = res
    if not a.no_batch:
        log("64-instance batch at full walk budgets")
        out["batch"] = bench_batch(ctx, wos, wi, torch)
    if not a.no_mesh and a.workload == "cube":
        log("cube as a triangle mesh")
        wk = out["walk_kernel"]
        box_sps = wk["woe_bound_steps_per_walk"] * wk["woe_bound_walks_per_s"]
        out["mesh"] = bench_mesh(ctx, wos, wi, torch, box_sps)
    if not a.no_serve:
        log(f"serving runs ({a.serve_seconds:.0f} s of arrivals)")
        out["serving"] = serving(ctx, wos, wi, a.serve_seconds, a.serve_rate, a.serve_svd, a.serve_radius)
    if not a.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = (cpu_baseline_cube if a.workload == "cube" else cpu_baseline_annulus)(inst, a.cpu_seconds)
    torch.cuda.synchronize()
    if h is not None:
        wos.wos_svd_destroy(ctx, h)
    wos.wos_destroy(ctx)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
