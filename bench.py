#!/usr/bin/env python
"""Benchmark of the ray-traced SRP hot path on one MI355X.

Workload: the seeded procedural ~50k-triangle spacecraft (49,644 triangles,
9 tree nodes, 8 hinge DOF, 6 materials), 1024 x 1024 rays per evaluation,
2 specular bounces.  One step = one pass of the whole hot path over one
batch: per-item hinge angles (articulation slots), window pass, persistent
trace with the fixed-visibility adjoint, fixed-order reduction; i.e.
srp_eval_grad_batch over `--batch` attitudes (Fibonacci sun directions, root
hinges drawn in [-90, 90] deg).  Inputs are resident on the device before
the timed region; results and gradients stay on the device.

Also measured (reported beside the headline value): the same batch forward
only (srp_eval_batch), and the plain path (srp_set_panel_angles + srp_eval
per item, a host round trip per evaluation, as a propagator stage does).

Prints one JSON line.
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

PEAK_LANE_OPS = 256 * 64 * 2.4e9     # CUs x lanes x clock: one VALU lane-op per lane per cycle
BOX_OPS, TRI_OPS = 10, 30             # algorithmic lane-ops per ray-box / ray-triangle test
TRAFFIC = os.path.join(ROOT, "profiles", "k_trace_grad_traffic.json")


def source_digest(paths):
    """SHA-256 of the code in `paths` (relative to the repository root) with
    // comments, trailing blanks and empty lines removed: a comment edit does
    not invalidate counters taken on the same code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for src in paths:
        with open(os.path.join(ROOT, src), encoding="utf-8") as f:
            for line in f:
                code = re.sub(r"//.*$", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(schedule):
    """HBM bytes per launch of the adjoint trace kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None when the kernel sources have
    changed since those counters were taken or this run's schedule (patches per
    chunk, blocks per CU: the gradient partials are per chunk) is not the one
    they were taken with."""
    try:
        with open(TRAFFIC) as f:
            rec = json.load(f)
        if source_digest(rec["sources"]) != rec["code_sha256"] or rec.get("schedule") != schedule:
            return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_config(srp, torch, name, stream, steps, oracle_sample=True):
    """Throughput of one of the other batch workloads: the box-wing at 128^2
    (c1, 1,024 attitudes), the 32,768-evaluation SPAD table at 512^2 (c3), the
    uneven 64-scene batch (c4), the 1M-triangle batch of 256 attitudes at
    2048^2 with the adjoint (c5).  Autotuned, one warm-up call, `steps` timed
    calls (a call runs as consecutive sub-batches when its workspace would
    pass 16 GiB); ray and test counts from one counting call.  With
    oracle_sample, the oracle is timed on a seeded subsample of the items
    (forward only) and their forces are compared with the batch's."""
    import synth
    grad = False
    if name == "c1":
        mesh = synth.box_wing()
        sc = srp.Scene(mesh)
        E, n, B = 1024, 128, 0
        dirs = synth.fibonacci_dirs(E)
        rng = np.random.default_rng(1001)
        angles = rng.uniform(-np.pi / 2, np.pi / 2, size=(E, mesh.n_dof))
        items = [(sc, angles[k], dirs[k], n) for k in range(E)]
        meshes = [mesh] * E
        sample = list(np.random.default_rng(11).choice(E, 64, replace=False))
        desc = f"box-wing ({mesh.n_tris} tris), {E} attitudes, {n}x{n} rays, B={B}"
    elif name == "c3":
        mesh, dirs, angles, n, B = synth.c3_spad()
        sc = srp.Scene(mesh)
        items = [(sc, angles[k], dirs[k], n) for k in range(len(dirs))]
        meshes = [mesh] * len(items)
        sample = list(np.random.default_rng(13).choice(len(items), 64, replace=False))
        desc = f"SPAD table: {mesh.n_tris}-triangle spacecraft, {len(dirs)} attitudes, {n}x{n} rays, B={B}"
    elif name == "c4":
        specs, B = synth.c4_uneven()
        scenes = [srp.Scene(m) for m, _, _, _ in specs]
        items = [(scenes[k], a, s_, n_) for k, (m, a, s_, n_) in enumerate(specs)]
        tris = [m.n_tris for m, _, _, _ in specs]
        meshes = [m for m, _, _, _ in specs]
        sample = [k for k in range(len(specs)) if specs[k][3] <= 512]   # every scene at N <= 512
        desc = (f"uneven batch: {len(specs)} scenes of {min(tris)}..{max(tris)} triangles, "
                f"grids {min(x[3] for x in specs)}..{max(x[3] for x in specs)}, B={B}")
    elif name == "c5":
        mesh, dirs, angles, n, B = synth.c5_batch()
        sc = srp.Scene(mesh)
        items = [(sc, angles[k], dirs[k], n) for k in range(len(dirs))]
        meshes = [mesh] * len(items)
        sample = list(np.random.default_rng(15).choice(len(items), 4, replace=False))
        grad = True
        desc = (f"greebled spacecraft ({mesh.n_tris} tris, {mesh.n_dof} hinge DOF), {len(dirs)} attitudes, "
                f"{n}x{n} rays, B={B}, forward + adjoint")
    else:
        raise SystemExit(f"unknown workload {name}")
    plain_items = [(s_, a, srp.params(d, n_, B)) for s_, a, d, n_ in items]
    entries = srp.Batch(plain_items)   # marshalled once
    E = len(entries)
    cnt = srp.results_to_numpy(srp.eval_batch([(s_, a, srp.params(d, n_, B, count=True)) for s_, a, d, n_ in items]))
    rays = int(cnt["n_rays"].sum() + cnt["n_secondary"].sum())
    work = BOX_OPS * int(cnt["n_box_tests"].sum()) + TRI_OPS * int(cnt["n_tri_tests"].sum())
    tune = srp.autotune(entries, grad=grad)
    run = (lambda: srp.eval_grad_batch(entries, None, None, stream)) if grad else (lambda: srp.eval_batch(entries, None, stream))
    out = run()
    torch.cuda.synchronize()
    srp.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms, launches = srp.profile_read()
    launch_ms, _ = srp.profile_read_launch()
    srp.profile(False)
    res = srp.results_to_numpy(out[0] if grad else out)
    assert (res["status"] == 0).all()
    kern = ms / 1e3 / steps   # the ray-tracing kernels of one call (of all its sub-batches)
    dev = launch_ms / 1e3 / steps   # its whole launches: upload, every kernel, result copy
    rec = {"workload": desc, "evals": E}
    if name == "c4":
        # the uneven batch as a captured graph (upload, window, trace, reduction), replayed
        plan = srp.Plan(plain_items)
        ref = res.tobytes()
        pout = plan.launch(stream)
        torch.cuda.synchronize()
        assert srp.results_to_numpy(pout).tobytes() == ref, "plan replay differs from the direct batch"
        t0 = time.perf_counter()
        for _ in range(steps):
            pout = plan.launch(stream)
        torch.cuda.synchronize()
        dt_plan = (time.perf_counter() - t0) / steps
        assert srp.results_to_numpy(pout).tobytes() == ref
        plan.close()
        _log(f"{name} (graph replays): {E / dt_plan:.1f} evals/s, {dt_plan * 1e3:.2f} ms per replay "
             f"(direct call {dt * 1e3:.2f} ms)")
        rec.update(path="srp_plan (captured graph replay); kernel_ms from a profiled direct call of the same batch",
                   evals_per_s=round(E / dt_plan, 2), grays_per_s=round(rays / dt_plan / 1e9, 3),
                   ms_per_call=round(dt_plan * 1e3, 3), direct_ms_per_call=round(dt * 1e3, 3))
    else:
        rec.update(path="srp_eval_grad_batch" if grad else "srp_eval_batch",
                   evals_per_s=round(E / dt, 2), grays_per_s=round(rays / dt / 1e9, 3), ms_per_call=round(dt * 1e3, 3))
    _log(f"{name}: {E / dt:.1f} evals/s, {rays / dt / 1e9:.2f} Grays/s, kernels {kern * 1e3:.2f} ms of "
        f"{dt * 1e3:.2f} ms per call ({launches // steps} launches; whole launches {dev * 1e3:.2f} ms)")
    rec.update(rays_per_call=rays, kernel_ms=round(kern * 1e3, 3), launches_per_call=launches // steps,
               device_ms=round(dev * 1e3, 3), device_share=round(dev / dt, 3),
               device_ms_definition="HIP events around each launch of a direct call: staging upload, articulation, "
               "window, trace, reduction kernels and result copy; device_share = device_ms / ms of the direct call",
               lane_op_frac=round(work / kern / PEAK_LANE_OPS, 4),
               tests_per_ray=round((int(cnt["n_box_tests"].sum()) + int(cnt["n_tri_tests"].sum())) / rays, 2),
               schedule={"patches_per_chunk": tune[0], "blocks_per_cu": tune[1]})
    if oracle_sample:
        # the FP64 oracle (its own hierarchy) on a seeded subsample of the items, forward
        # only, timed on the host's cores; then each item's parity by the tests' policy:
        # its single recorded evaluation (bitwise the batch item) against the oracle's
        # hits (raw), against oracle physics on the GPU's hits (visibility matched), and
        # the primary rays whose hits differ outside the edge band
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import compare_eval
        t0 = time.perf_counter()
        o_rays, orcs = 0, []
        for k in sample:
            _, a, d, n_ = items[k]
            o = oracle.eval_srp(meshes[k], d, n_, bounces=B, angles=a, record=True)
            o_rays += o.n_rays + o.n_secondary
            orcs.append(o)
        dt_o = time.perf_counter() - t0
        f_err, f_vm, outside, band = [], [], 0, []
        for k, o in zip(sample, orcs):
            sc_k, a, d, n_ = items[k]
            sc_k.set_angles(a)
            single = srp.eval(sc_k, d, n_, bounces=B, record=True)
            assert np.array_equal(single["force"], res[k]["force"]), (name, k)
            rep = compare_eval(meshes[k], a, d, n_, B, single, o)
            f_err.append(rep["f_err"])
            f_vm.append(rep["f_err_vis_matched"])
            outside += rep["primary_outside_band"]
            band.append(rep["edge_band_fraction"])
        rec["oracle"] = {"evals_per_s": round(len(sample) / dt_o, 4), "grays_per_s": round(o_rays / dt_o / 1e9, 6),
                         "cores": oracle.threads(), "sample": f"items {sorted(int(k) for k in sample)} of {E}, "
                         f"forward only (FP64, oracle BVH)",
                         "max_rel_force_err": max(f_err), "max_rel_force_err_vis_matched": max(f_vm),
                         "primary_ids_differing_outside_edge_band": outside, "edge_band_fraction": max(band)}
        _log(f"{name} oracle: {len(sample) / dt_o:.3f} evals/s on {oracle.threads()} threads ({len(sample)} items); "
             f"max rel force err {max(f_err):.2e}, visibility matched {max(f_vm):.2e}, "
             f"ids differing outside the edge band {outside}")
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--bounces", type=int, default=2)
    ap.add_argument("--plain", type=int, default=16, help="evaluations timed on the plain path")
    ap.add_argument("--cpu-samples", type=int, default=2, help="batch items the oracle times (0: skip)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (profiling runs)")
    ap.add_argument("--schedule", default="", help="PPC,BPC: fixed patches per chunk and blocks per CU "
                    "for both launches (implies --no-tune; profiling runs)")
    ap.add_argument("--spad", type=int, default=1, help="SPAD vs direct propagation measurement (0: skip)")
    ap.add_argument("--spad-steps", type=int, default=400, help="RK4 steps of the SPAD comparison orbit")
    ap.add_argument("--p2", type=int, default=1,
                    help="20-revolution propagation timing (0: skip, 1: fixed panels, 2: also tracking panels)")
    ap.add_argument("--p2-revs", type=int, default=20)
    ap.add_argument("--configs", default="c1,c3,c4,c5",
                    help="also time these other workloads, comma-separated from c1,c3,c4,c5 ('' to skip)")
    ap.add_argument("--p2-rtol", type=float, default=1e-9)
    ap.add_argument("--c2-prop-steps", type=int, default=1440,
                    help="RK4 steps of 60 s of the headline workload's propagation leg (0: skip)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run a device copy of this many MiB (calibrates memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this SRP path has no multi-GPU mode "
              "(batches shard with no collective; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2608_07307_amd as srp
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731

    mesh, dirs, angles, _, _ = synth.c2_batch(args.batch)
    scene = srp.Scene(mesh)
    B, N, E = args.bounces, args.n, args.batch
    entries = [(scene, angles[k], srp.params(dirs[k], N, B)) for k in range(E)]
    stride = srp.grad_size(scene)
    out = torch.empty(E * srp.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    grad = torch.zeros((E, stride), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    log(f"workload: T={mesh.n_tris} N={N} B={B} batch={E}")

    # algorithmic work of one launch: box and triangle tests (counting variant, same inputs)
    cnt_entries = [(scene, angles[k], srp.params(dirs[k], N, B, count=True)) for k in range(E)]
    cres = srp.results_to_numpy(srp.eval_batch(cnt_entries))
    n_box, n_tri = int(cres["n_box_tests"].sum()), int(cres["n_tri_tests"].sum())
    rays_primary = int(cres["n_rays"].sum())
    rays_total = rays_primary + int(cres["n_secondary"].sum())
    work = BOX_OPS * n_box + TRI_OPS * n_tri
    log(f"counts per batch: box {n_box:.3e} tri {n_tri:.3e} rays {rays_total:.3e} "
        f"(tests/ray {(n_box + n_tri) / rays_total:.1f})")

    if args.copy_mb:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings calibrate the counters
        src = torch.ones(args.copy_mb * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)          # one elementwise kernel: reads and writes copy_mb MiB
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_mb} MiB read + {args.copy_mb} MiB written")

    # schedule: the autotuner picks tiles per chunk and blocks per CU (untimed)
    tune = (0, 0, 0.0)
    if args.schedule:
        ppc, bpc = (int(x) for x in args.schedule.split(","))
        srp.set_schedule(ppc, bpc)
        tune = (ppc, bpc, 0.0)
        log(f"schedule fixed: patches/chunk {ppc}, blocks/CU {bpc}")
    elif not args.no_tune:
        tune = srp.autotune(entries, grad=True)
        log(f"autotune (forward+adjoint): patches/chunk {tune[0]}, blocks/CU {tune[1]}, {tune[2]:.3f} ms")
        tune_fwd = srp.autotune(entries, grad=False)
        log(f"autotune (forward): patches/chunk {tune_fwd[0]}, blocks/CU {tune_fwd[1]}, {tune_fwd[2]:.3f} ms")

    # headline: batched forward + adjoint
    for _ in range(args.warmup):
        srp.eval_grad_batch(entries, out, grad, stream)
    torch.cuda.synchronize()
    srp.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        srp.eval_grad_batch(entries, out, grad, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    trace_ms, launches = srp.profile_read()
    srp.profile(False)
    dt = (t1 - t0) / args.steps
    res = srp.results_to_numpy(out)
    assert (res["status"] == 0).all()
    value = E / dt
    kern_s = trace_ms / 1e3 / max(launches, 1)
    log(f"batched+adjoint: {dt * 1e3:.3f} ms/step, {value:.1f} evals/s, trace kernel {kern_s * 1e3:.3f} ms")

    # batched forward only
    for _ in range(args.warmup):
        srp.eval_batch(entries, out, stream)
    torch.cuda.synchronize()
    srp.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        srp.eval_batch(entries, out, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fwd_ms, fwd_launches = srp.profile_read()
    srp.profile(False)
    fwd_dt = (t1 - t0) / args.steps
    fwd = srp.results_to_numpy(out)
    log(f"batched forward: {fwd_dt * 1e3:.3f} ms/step, {E / fwd_dt:.1f} evals/s")

    # plain: set angles + blocking eval per item
    P = min(args.plain, E)
    for k in range(min(2, P)):
        scene.set_angles(angles[k])
        srp.eval(scene, dirs[k], N, bounces=B)
    t0 = time.perf_counter()
    plain_f = []
    for k in range(P):
        scene.set_angles(angles[k])
        plain_f.append(srp.eval(scene, dirs[k], N, bounces=B)["force"])
    t1 = time.perf_counter()
    plain_eps = P / (t1 - t0)
    log(f"plain: {plain_eps:.1f} evals/s")
    for k in range(P):
        assert np.array_equal(plain_f[k], fwd[k]["force"]), "plain and batched results differ"

    # the paper's ray-traced setting (256^2 window, two secondary levels, 16 diffuse
    # rays per emitting hit), batched forward over the same attitudes
    _, _, _, dN, dB, dK = synth.diffuse_batch(E)
    d_entries = [(scene, angles[k], srp.params(dirs[k], dN, dB, diffuse=dK)) for k in range(E)]
    dc = srp.results_to_numpy(srp.eval_batch(
        [(scene, angles[k], srp.params(dirs[k], dN, dB, count=True, diffuse=dK)) for k in range(E)]))
    d_work = BOX_OPS * int(dc["n_box_tests"].sum()) + TRI_OPS * int(dc["n_tri_tests"].sum())
    d_rays = int(dc["n_rays"].sum() + dc["n_secondary"].sum())
    if args.schedule:
        srp.set_schedule(0, 0)   # the fixed schedule is the headline batch's; this batch takes its own
    elif not args.no_tune:
        srp.autotune(d_entries, grad=False)
    for _ in range(args.warmup):
        srp.eval_batch(d_entries, out, stream)
    torch.cuda.synchronize()
    srp.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        srp.eval_batch(d_entries, out, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d_ms, d_launches = srp.profile_read()
    srp.profile(False)
    d_dt = (t1 - t0) / args.steps
    d_kern = d_ms / 1e3 / max(d_launches, 1)
    assert (srp.results_to_numpy(out)["status"] == 0).all()
    # one evaluation at a time, as a propagator calls it (srp_eval: host round trip
    # and result readback included; the scene at the first attitude's angles)
    scene.set_angles(angles[0])
    for k in range(3):
        srp.eval(scene, dirs[k], dN, bounces=dB, diffuse=dK)
    n_single = min(E, 32)
    t0 = time.perf_counter()
    for k in range(n_single):
        srp.eval(scene, dirs[k], dN, bounces=dB, diffuse=dK)
    single_ms = (time.perf_counter() - t0) / n_single * 1e3
    paper_setting = {
        "workload": f"same mesh and {E} attitudes, {dN}x{dN} rays, {dB} secondary levels, "
                    f"{dK} diffuse rays per emitting hit, batched forward",
        "evals_per_s": round(E / d_dt, 3),
        "grays_per_s": round(d_rays / d_dt / 1e9, 4),
        "rays_per_batch": d_rays,
        "kernel_ms": round(d_kern * 1e3, 4),
        "lane_op_frac": round(d_work / d_kern / PEAK_LANE_OPS, 4),
        "single_eval_ms": round(single_ms, 4),
    }
    log(f"paper setting (N={dN}, B={dB}, K={dK}): {E / d_dt:.1f} evals/s, {d_rays / d_dt / 1e9:.2f} Grays/s; "
        f"one evaluation {single_ms:.3f} ms")

    # SPAD (precomputed table + interpolation) against direct ray tracing during
    # propagation: the paper's 20 x 10 grids (plain and shifted by 5 deg) built at
    # the ray-traced setting, one revolution of the circular orbit C (0.388 AU)
    # with the attitude inertially fixed (hinges at the first attitude's angles)
    spad = None
    if args.spad:
        AU, MU_SUN, P1AU, MASS = 1.495978707e11, 1.32712440018e20, 4.56e-6, 1000.0
        deg = np.pi / 180
        grids = {"20x10": srp.spad_grid(20, 10, -180 * deg, -90 * deg, 18 * deg, 18 * deg),
                 "20x10S": srp.spad_grid(20, 10, -175 * deg, -85 * deg, 18 * deg, 18 * deg)}
        srp.spad_build(scene, grids["20x10"], dN, bounces=dB, angles=angles[0], diffuse=dK)   # warm-up
        torch.cuda.synchronize()
        tabs, build_ms = {}, {}
        for name, G in grids.items():
            t0 = time.perf_counter()
            tabs[name] = srp.spad_build(scene, G, dN, bounces=dB, pressure=P1AU, angles=angles[0], diffuse=dK)
            build_ms[name] = (time.perf_counter() - t0) * 1e3
        a = 0.388 * AU
        y0 = np.array([a, 0, 0, 0, np.sqrt(MU_SUN / a), 0])
        steps = args.spad_steps
        h = 2 * np.pi * np.sqrt(a ** 3 / MU_SUN) / steps
        t0 = time.perf_counter()
        direct, st = srp.propagate(scene, y0, 0.0, h, steps, MU_SUN, MASS, P1AU, AU, dN, bounces=dB,
                                   angles0=angles[0], diffuse=dK)
        direct_s = time.perf_counter() - t0
        sep, spad_s = {}, {}
        for name, G in grids.items():
            t0 = time.perf_counter()
            tr = srp.propagate_spad(G, tabs[name], P1AU, y0, 0.0, h, steps, MU_SUN, MASS, P1AU, AU)
            spad_s[name] = time.perf_counter() - t0
            sep[name] = float(np.linalg.norm(tr[-1, 1:4] - direct[-1, 1:4]) / 1e3)
        # the N-plate model of the same craft (plates of the articulated mesh, no
        # shadowing, no secondary rays) over the same revolution
        plates = srp.nplate_from_scene(scene, angles[0])
        t0 = time.perf_counter()
        tr = srp.propagate_nplate(plates, y0, 0.0, h, steps, MU_SUN, MASS, P1AU, AU)
        nplate_s = time.perf_counter() - t0
        sep["nplate"] = float(np.linalg.norm(tr[-1, 1:4] - direct[-1, 1:4]) / 1e3)
        kep = srp.propagate_spad(grids["20x10"], 0.0 * tabs["20x10"], P1AU, y0, 0.0, h, steps, MU_SUN, MASS,
                                 P1AU, AU)
        # interpolation error per evaluation along the orbit plane (elevation 0, 1 deg steps)
        az = np.arange(360) * deg
        S = np.stack([np.cos(az), np.sin(az), np.zeros_like(az)], 1)
        ref_f = srp.results_to_numpy(srp.eval_batch(
            [(scene, angles[0], srp.params(S[k], dN, dB, P1AU, diffuse=dK)) for k in range(360)]))["force"].copy()
        scale = float(np.linalg.norm(ref_f, axis=1).mean())
        interp_err = {name: round(float(np.sqrt(np.mean([np.sum((srp.spad_interp(G, tabs[name], S[k])[:3] - ref_f[k]) ** 2)
                                                          for k in range(360)])) / scale), 5)
                      for name, G in grids.items()}
        interp_err["nplate"] = round(float(np.sqrt(np.mean([np.sum((srp.nplate_eval(plates, S[k], P1AU)["force"]
                                                                   - ref_f[k]) ** 2) for k in range(360)])) / scale), 5)
        # the paper's four orbits (Sec. 6.1 table: a in AU, e; angles zero), one
        # revolution from perihelion each, adaptive RK7(8): ray-traced SRP per
        # stage against the SPAD tables and the N-plate model, each integrated
        # with the same step control
        orbit_set = {"C": (0.388, 0.0), "E(S)": (0.388, 0.881), "E(M)": (0.437, 0.786), "E(L)": (0.557, 0.682)}
        per_orbit = {}
        for oname, (a_au, ecc) in orbit_set.items():
            ao = a_au * AU
            rp = ao * (1 - ecc)
            yo = np.array([rp, 0, 0, 0, np.sqrt(MU_SUN * (1 + ecc) / rp), 0])
            To = 2 * np.pi * np.sqrt(ao ** 3 / MU_SUN)
            oo = srp.rk78_opts(To / 100, True, args.p2_rtol, [args.p2_rtol * AU] * 3 + [args.p2_rtol * 1e5] * 3)
            t0 = time.perf_counter()
            dtr, dst = srp.propagate_rk78(scene, yo, 0.0, To, oo, MU_SUN, MASS, P1AU, AU, dN, bounces=dB,
                                          angles0=angles[0], diffuse=dK)
            d_s = time.perf_counter() - t0
            end = dtr[-1, 1:4]
            ends = {name: srp.propagate_spad_rk78(G, tabs[name], P1AU, yo, 0.0, To, oo, MU_SUN, MASS, P1AU,
                                                  AU)[-1, 1:4] for name, G in grids.items()}
            ends["nplate"] = srp.propagate_nplate_rk78(plates, yo, 0.0, To, oo, MU_SUN, MASS, P1AU, AU)[-1, 1:4]
            two_body = srp.propagate_nplate_rk78(plates[:0], yo, 0.0, To, oo, MU_SUN, MASS, P1AU, AU)[-1, 1:4]
            per_orbit[oname] = {
                "direct_s": round(d_s, 3), "direct_evals": dst["n_evals"], "steps": len(dtr) - 1,
                "final_separation_km": {k: round(float(np.linalg.norm(v - end) / 1e3), 3) for k, v in ends.items()},
                "srp_displacement_km": round(float(np.linalg.norm(two_body - end) / 1e3), 3)}
            log(f"orbit {oname}: direct {d_s:.2f} s ({dst['n_evals']} evaluations), separations (km) "
                f"{per_orbit[oname]['final_separation_km']}, SRP displacement "
                f"{per_orbit[oname]['srp_displacement_km']} km")
        spad = {
            "workload": f"{mesh.n_tris}-triangle spacecraft, {dN}x{dN} rays, {dB} secondary levels, {dK} diffuse "
                        f"rays; orbit C (a = 0.388 AU, e = 0), one revolution, {steps} RK4 steps, "
                        f"mass {MASS:.0f} kg, fixed attitude",
            "table_nodes": 200,
            "n_plates": len(plates),
            "table_build_ms": {k: round(v, 3) for k, v in build_ms.items()},
            "direct_ms_per_step": round(direct_s / steps * 1e3, 4),
            "direct_evals": st["n_evals"],
            "spad_us_per_step": {k: round(v / steps * 1e6, 3) for k, v in spad_s.items()},
            "nplate_us_per_step": round(nplate_s / steps * 1e6, 3),
            "interp_rms_rel_err_el0": interp_err,
            "final_separation_km": {k: round(v, 4) for k, v in sep.items()},
            "srp_displacement_km": round(float(np.linalg.norm(kep[-1, 1:4] - direct[-1, 1:4]) / 1e3), 3),
            "orbits_one_revolution_rk78": per_orbit,
        }
        log(f"SPAD: table {build_ms['20x10']:.1f} ms, direct {direct_s / steps * 1e3:.2f} ms/step, "
            f"SPAD {spad_s['20x10'] / steps * 1e6:.1f} us/step, separation 20x10 {sep['20x10']:.3f} km, "
            f"20x10S {sep['20x10S']:.3f} km, N-plate {sep['nplate']:.3f} km (SRP displacement {spad['srp_displacement_km']} km); "
            f"interpolation rms error {interp_err}")

    # 20 revolutions of the paper's reference orbit (a = 0.557 AU, e = 0.682,
    # perihelion start) with adaptive RK7(8) and one ray-traced evaluation per
    # stage at the paper's ray-traced setting; the same span with the SPAD
    # tables; with --p2 2 also with sun-tracking panels
    p2 = None
    if args.p2 and spad is not None:
        a2, e2 = 0.557 * AU, 0.682
        rp = a2 * (1 - e2)
        y2 = np.array([rp, 0, 0, 0, np.sqrt(MU_SUN * (1 + e2) / rp), 0])
        T2 = 2 * np.pi * np.sqrt(a2 ** 3 / MU_SUN)
        opts = srp.rk78_opts(T2 / 100, True, args.p2_rtol, [args.p2_rtol * AU] * 3 + [args.p2_rtol * 1e5] * 3)
        p2 = {"workload": f"reference orbit a = 0.557 AU, e = 0.682, {args.p2_revs} revolutions from perihelion, "
                          f"adaptive RK7(8) (rtol {args.p2_rtol:g}), {dN}x{dN} rays, {dB} secondary levels, "
                          f"{dK} diffuse rays, mass {MASS:.0f} kg"}
        runs = [("fixed_panels", False)] + ([("tracking_panels", True)] if args.p2 > 1 else [])
        finals = {}
        for name, track in runs:
            t0 = time.perf_counter()
            tr2, st2 = srp.propagate_rk78(scene, y2, 0.0, args.p2_revs * T2, opts, MU_SUN, MASS, P1AU, AU, dN,
                                          bounces=dB, track_sun=track, angles0=angles[0], diffuse=dK)
            dt2 = time.perf_counter() - t0
            finals[name] = tr2[-1, 1:4]
            p2[name] = {"total_s": round(dt2, 3), "steps": len(tr2) - 1, "srp_evals": st2["n_evals"],
                        "ms_per_eval": round(dt2 / st2["n_evals"] * 1e3, 4),
                        "srp_share": round(st2["srp_seconds"] / dt2, 4)}
            log(f"P2 {name}: {args.p2_revs} revolutions in {dt2:.2f} s, {len(tr2) - 1} steps, "
                f"{st2['n_evals']} evaluations")
        sep2 = {}
        for name, G in grids.items():
            t0 = time.perf_counter()
            tr2 = srp.propagate_spad_rk78(G, tabs[name], P1AU, y2, 0.0, args.p2_revs * T2, opts, MU_SUN, MASS,
                                          P1AU, AU)
            p2[f"spad_{name}_s"] = round(time.perf_counter() - t0, 4)
            sep2[name] = float(np.linalg.norm(tr2[-1, 1:4] - finals["fixed_panels"]) / 1e3)
        t0 = time.perf_counter()
        tr2 = srp.propagate_nplate_rk78(plates, y2, 0.0, args.p2_revs * T2, opts, MU_SUN, MASS, P1AU, AU)
        p2["nplate_s"] = round(time.perf_counter() - t0, 4)
        sep2["nplate"] = float(np.linalg.norm(tr2[-1, 1:4] - finals["fixed_panels"]) / 1e3)
        p2["final_separation_km"] = {(k if k == "nplate" else f"spad_{k}"): round(v, 3) for k, v in sep2.items()}
        if "tracking_panels" in finals:
            p2["final_separation_km"]["tracking_vs_fixed_panels"] = round(
                float(np.linalg.norm(finals["tracking_panels"] - finals["fixed_panels"]) / 1e3), 3)
        log(f"P2 separations (km): {p2['final_separation_km']}")

    # the propagation leg of the headline workload: 1,000 kg on the circular 1 AU
    # orbit, attitude inertially fixed, RK4 at 60 s steps for one day (4 SRP
    # evaluations per step at the headline's 1024^2 rays and 2 bounces), the
    # wing roots tracking the Sun at every stage
    c2prop = None
    if args.c2_prop_steps > 0:
        AU, MU_SUN, MASS, P0 = 1.495978707e11, 1.32712440018e20, 1000.0, 1361.0 / 299792458.0
        y0 = np.array([AU, 0.0, 0.0, 0.0, np.sqrt(MU_SUN / AU), 0.0])
        srp.propagate(scene, y0, 0.0, 60.0, 2, MU_SUN, MASS, P0, AU, N, bounces=B, track_sun=True)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr, st = srp.propagate(scene, y0, 0.0, 60.0, args.c2_prop_steps, MU_SUN, MASS, P0, AU, N, bounces=B,
                               track_sun=True)
        prop_s = time.perf_counter() - t0
        kep = srp.propagate_nplate(srp.nplate_from_scene(scene)[:0], y0, 0.0, 60.0, args.c2_prop_steps, MU_SUN,
                                   MASS, P0, AU)   # no plates: two-body RK4 on the same steps
        c2prop = {
            "workload": f"{mesh.n_tris}-triangle spacecraft, 1000 kg, circular 1 AU orbit, RK4, 60 s steps, "
                        f"{args.c2_prop_steps} steps ({args.c2_prop_steps * 60 / 86400:.3g} day), {N}x{N} rays, "
                        f"{B} bounces, sun-tracking wing roots, one srp_eval per stage",
            "steps": args.c2_prop_steps, "evals": st["n_evals"], "total_s": round(prop_s, 3),
            "ms_per_eval": round(prop_s / st["n_evals"] * 1e3, 4),
            "srp_share": round(st["srp_seconds"] / prop_s, 4),
            "srp_displacement_m": round(float(np.linalg.norm(tr[-1, 1:4] - kep[-1, 1:4])), 3)}
        log(f"c2 propagation: {args.c2_prop_steps} RK4 steps, {st['n_evals']} evaluations in {prop_s:.2f} s "
            f"({c2prop['ms_per_eval']} ms each), SRP displacement {c2prop['srp_displacement_m']} m")

    # oracle on a bounded sample (CPU baseline and parity of the sampled items)
    cpu = None
    parity = None
    if args.cpu_samples > 0:
        import oracle
        errs, gerrs = [], {"rho_s": [], "rho_d": [], "theta": []}
        g_host = grad.cpu().numpy()
        M, J = mesh.n_mats, mesh.n_dof
        t0 = time.perf_counter()
        fds, orcs = [], []
        for k in range(args.cpu_samples):
            o = oracle.eval_srp(mesh, dirs[k], N, bounces=B, angles=angles[k], record=True)
            orcs.append(o)
            fds.append(oracle.fd_gradients(mesh, dirs[k], N, B, o.grid, o.ids, angles=angles[k]))
            errs.append(float(np.linalg.norm(res[k]["force"] - o.force) / np.linalg.norm(o.force)))
        t1 = time.perf_counter()
        for k, fd in enumerate(fds):
            blocks = {"rho_s": g_host[k, :3 * M].reshape(M, 3), "rho_d": g_host[k, 3 * M:6 * M].reshape(M, 3),
                      "theta": g_host[k, 6 * M:6 * M + 3 * J].reshape(J, 3)}
            for key, gk in blocks.items():
                gerrs[key].append(float(np.abs(gk - fd[key]).max() / np.abs(fd[key]).max()))
        # primary ids of the sampled items (their single recorded evaluations, bitwise the
        # batch's) against the oracle's: rays that differ must lie in the edge band
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import classify_primary
        band, mism, outside = [], 0, 0
        for k, o in enumerate(orcs):
            scene.set_angles(angles[k])
            single = srp.eval(scene, dirs[k], N, bounces=B, record=True)
            assert np.array_equal(single["force"], res[k]["force"])
            m_, out_, frac_ = classify_primary(mesh, angles[k], o.grid, N, o.ids[:, 0], single["ids"][:, 0])
            band.append(frac_)
            mism += m_
            outside += out_
        orc_tests = sum(o.n_box_tests + o.n_tri_tests for o in orcs) / sum(o.n_rays + o.n_secondary for o in orcs)
        cpu = {"value": round(args.cpu_samples / (t1 - t0), 4), "unit": "evals/s",
               "cores": oracle.threads(), "kind": "oracle",
               "sample": f"{args.cpu_samples} of the {E} batch items: FP64 forward (oracle BVH) + "
                         f"central-difference gradient ({2 * (2 * mesh.n_mats + mesh.n_dof)} "
                         f"fixed-visibility re-shades), {N}x{N} rays, B={B}"}
        parity = {"max_rel_force_err": max(errs), "items_checked": args.cpu_samples,
                  "primary_ids_differing": mism, "primary_ids_differing_outside_edge_band": outside,
                  "edge_band_fraction": max(band),
                  "edge_band_definition": "fraction of primary rays whose GPU and oracle hits differ inside the "
                                          "edge band (image-plane distance to an edge of either triangle, or "
                                          "depth difference, <= 1e-6 L)",
                  "max_rel_grad_err": {k: max(v) for k, v in gerrs.items()},
                  "grad_err_definition": "per block: max |adjoint - oracle central difference (h = 1e-4, "
                                         "oracle's own hits)| / max |oracle central difference|"}
        cpu["oracle_bvh_tests_per_ray"] = round(orc_tests, 2)
        log(f"oracle: {cpu['value']} evals/s on {cpu['cores']} threads; parity {max(errs):.2e}; "
            f"edge band {max(band):.2e}; oracle BVH {orc_tests:.1f} tests/ray")

    achieved = work / kern_s / 1e12
    peak = PEAK_LANE_OPS / 1e12
    vp = srp.valu_peak()
    log(f"measured FMA-loop peak: {vp['lane_fma_per_s'] / 1e12:.2f} T lane-FMA/s at {vp['shader_ghz']:.3f} GHz "
        f"on {vp['n_cu']} CUs")
    line = {
        "metric": "SRP evals/sec and Grays/s at 1024^2 rays, batched+adjoint vs plain, at 1e-5 rel force err",
        "value": round(value, 3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"procedural ~50k-triangle spacecraft ({mesh.n_tris} tris, 9 nodes, 8 DOF, "
                        f"6 materials), {N}x{N} rays, {B} bounces, batch of {E} attitudes, "
                        f"forward + fixed-visibility adjoint per step",
            "batch": E, "n": N, "bounces": B, "triangles": mesh.n_tris,
            "schedule": {"patches_per_chunk": tune[0], "blocks_per_cu": tune[1]},
        },
        "grays_per_s": round(rays_total * args.steps / (dt * args.steps) / 1e9, 4),
        "grays_per_s_primary": round(rays_primary / dt / 1e9, 4),
        "batched_forward_evals_per_s": round(E / fwd_dt, 3),
        "batched_forward_grays_per_s": round(rays_total / fwd_dt / 1e9, 4),
        "plain_evals_per_s": round(plain_eps, 3),
        "paper_setting": paper_setting,
        "spad": spad,
        "p2": p2,
        "c2_propagation": c2prop,
        "parity": parity,
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 4),
            "peak": round(peak, 4),
            "unit": "Tlane-op/s",
            "frac": round(achieved / peak, 4),
            "peak_definition": "256 CUs x 64 lanes x 2.4 GHz: one non-packed VALU lane-op per lane per cycle",
            "frac_vs_packed_peak": round(achieved / (2 * peak), 4),
            "packed_peak_definition": "157.3 TFLOP/s FP32 = 78.6 T packed lane-FMA/s (packed FP32 is not used here)",
            "measured_peak": {"lane_fma_per_s_T": round(vp["lane_fma_per_s"] / 1e12, 4),
                              "shader_ghz": round(vp["shader_ghz"], 4), "n_cu": vp["n_cu"],
                              "frac": round(achieved * 1e12 / vp["lane_fma_per_s"], 4),
                              "how": "srp_valu_peak: 8 waves per SIMD, 8 independent v_fma_f32 chains per lane"},
            "tests_per_ray": round((n_box + n_tri) / rays_total, 2),
            "traffic": measured_traffic({"patches_per_chunk": tune[0], "blocks_per_cu": tune[1]}),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_source": "not measured by this run: the committed counter record "
                              "profiles/k_trace_grad_traffic.json, used only while its kernel-code digest "
                              "and schedule match this run (null otherwise)",
            "kernel": "k_trace<GRAD> (forward + adjoint)",
            "work_per_launch": {"box_tests": n_box, "tri_tests": n_tri,
                                "lane_ops": work, "ops_per_box": BOX_OPS, "ops_per_tri": TRI_OPS},
            "kernel_ms": round(kern_s * 1e3, 4),
            "forward_kernel_ms": round(fwd_ms / max(fwd_launches, 1), 4),
        },
        "cpu_baseline": cpu,
    }
    if args.configs:
        line["configs"] = {c: time_config(srp, torch, c, stream, max(1, min(args.steps, 3)), args.cpu_samples > 0)
                           for c in args.configs.split(",") if c}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
