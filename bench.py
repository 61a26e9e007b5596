#!/usr/bin/env python3
"""Throughput of the geometric PLIC VoF flux path on one MI355X.

One step = the whole path on the 128^3 hex mesh of the deformation test
(eq. 4.6, T = 3, sphere r = 0.15 at (0.35, 0.35, 0.35), Co 0.5, dt = 1/512):
backtrack, flux polyhedra, flux correction, PLIC planes, clipping and the
conservative update, for all 6.3M faces and 2.1M cells.  Inputs are resident
in HBM when the timed region starts.

Prints one JSON line: face-fluxes/s (faces with F != 0 per step, each built,
corrected and given its phase volume) over the whole run to T (1536 steps,
timed from alpha^0 in segments that show the rate along the run), run as the
library runs them (each step one captured HIP graph); the advection error E_g
and alpha's range at the end; per-kernel durations and the dominant kernel's
roofline figure from HIP events around every kernel over 20 steps from the
middle of the run, launched kernel by kernel; a sampled parity check of an
extra step against the oracle; and the oracle's own rate on a bounded sample
of the same steps (CPU baseline).  --workload batched / served run the
batched and served forms against the plain per-mesh / per-request loop.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "face-fluxes/s at 1e-12 rel vol err; batched/served vs plain, p50/p99 lat"
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E

# Estimates of the FP64 work per unit, used only where no counter summary of
# the current kernel sources is committed (profiles/fp64_counters_*.md).
FLUX_FLOPS_PER_QUAD_FACE = 400.0     # sweep, exact volume cubic, branch, ~2 Newton steps
FLUX_BYTES_PER_FACE = 52.0           # CSR 20, F0 8, lambda 8, V_alpha 8, bytes 3, points ~5
CLIP_FLOPS_PER_PAIR = 1000.0         # plane tests, clips and volume of one (tet, cell) pair
PLANE_FLOPS_PER_CELL = 20000.0       # NAG gradient + ~12 fill-level evaluations x 24 tets


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# bench kernel name -> device function whose HBM traffic was counted
KERNEL_FUNCS = {"flux": "k_flux", "clip": "k_clip_fast", "clip_general": "k_clip_general",
                "plane": "k_plane", "update": "k_update", "point_prep": "k_point_prep",
                "cell_class": "k_cell_class", "face_sum": "k_face_sum"}
WORKLOAD = ["deform3d"]  # set from the command line
# peak VALU issue: a wave64 instruction occupies a 16-lane SIMD for 4 cycles
# (the FP64 rate: 256 CUs x 4 SIMDs x 16 FMA lanes x 2 flops x 2.4 GHz = 78.6
# TFLOP/s); 256 x 4 x 2.4e9 / 4 wave instructions per second
PEAK_VALU_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def kernel_source_hash():
    """sha256 prefix of the device sources, as recorded beside the counters."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_1305_3417_amd", "csrc", "*"))):
        if path.endswith((".hip", ".hpp", ".h")):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_record(prefix, tag):
    """The JSON line `tag` of profiles/<prefix>_<workload>_<n>.md when it was
    taken on the current kernel sources, else None."""
    path = os.path.join(ROOT, "profiles", f"{prefix}_{WORKLOAD[0]}_{WORKLOAD[1]}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        line = next((ln for ln in fh if ln.startswith(tag + ":")), None)
    if line is None:
        return None
    rec = json.loads(line.split(":", 1)[1])
    return rec if rec.get("source_sha256_16") == kernel_source_hash() else None


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE
    summary of the profiled window (copy-calibrated), or None when it was taken
    on other kernel sources."""
    rec = _profile_record("hbm_traffic", "traffic-json")
    return None if rec is None else rec["bytes_per_launch"].get(KERNEL_FUNCS.get(kernel, ""))


def recorded_flops(kernel, unit):
    """(executed FP64 flops per unit, VALU wave instructions per launch) of
    `kernel` from the committed counter summary of the profiled window, or
    None when it was taken on other kernel sources."""
    rec = _profile_record("fp64_counters", "flops-json")
    if rec is None or not rec.get("window_units_per_step"):
        return None
    f = KERNEL_FUNCS.get(kernel, "")
    n = rec["window_units_per_step"].get(unit)
    if f not in rec["flops_per_launch"] or not n:
        return None
    return rec["flops_per_launch"][f] / n, rec.get("valu_insts_per_launch", {}).get(f)


CPU_SAMPLE_SECONDS = 10.0   # oracle steps are run until this much host time has passed
CPU_SAMPLE_MAX_STEPS = 16


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, alpha, step):
    """Whole steps of the oracle (reconstruction, correction of every face,
    phase volumes, update) on the same mesh, from the same state, on the host
    cores: consecutive steps until about CPU_SAMPLE_SECONDS have passed on all
    threads, then one step on one thread."""
    import numpy as np

    import oracle
    o = oracle.Oracle(w.mesh)
    o.set_velocity(w.U0c, w.F0)
    n_flux = int(np.count_nonzero(w.F0))
    threads = oracle.set_threads(0)
    a = alpha
    n = 0
    t0 = time.perf_counter()
    while n < CPU_SAMPLE_MAX_STEPS and step + n < len(w.dt):
        a = o.step(a, w.dt[step + n], w.scale[step + n])["alpha"]
        n += 1
        if time.perf_counter() - t0 >= CPU_SAMPLE_SECONDS:
            break
    t = time.perf_counter() - t0
    one = None
    if step + n < len(w.dt):
        oracle.set_threads(1)
        t1 = time.perf_counter()
        o.step(a, w.dt[step + n], w.scale[step + n])
        one = n_flux / (time.perf_counter() - t1)
        oracle.set_threads(threads)
    return {"value": n * n_flux / t, "unit": "face-fluxes/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "one_thread_value": one,
            "sample": f"{n} whole steps ({n_flux} flux faces each) of the same {w.name} case "
                      f"from mid-run (step {step}) on {threads} threads, {t:.1f} s; then one "
                      f"step on one thread"}


def parity_check(vof, mesh, w, step, n_sample=2000, seed=5):
    """One extra (untimed) step from the current state, checked on sampled
    faces against the oracle: lambda and V_alpha within 1e-12 of
    max(|F| dt, gross swept volume, 1e-2 max(V_owner, d_f^3))."""
    import numpy as np

    import oracle
    alpha = vof.vof_read_alpha(mesh)
    vof.vof_advect(mesh, w.dt[step:step + 1], w.scale[step:step + 1])
    lam = vof.vof_read_face(mesh, vof.VOF_FACE_LAMBDA)
    vph = vof.vof_read_face(mesh, vof.VOF_FACE_VPHASE)
    kind = vof.vof_read_face(mesh, vof.VOF_FACE_KIND)
    status = vof.vof_read_face(mesh, vof.VOF_FACE_STATUS)
    rng = np.random.default_rng(seed)
    geo = np.flatnonzero(kind == 3)
    flux = np.flatnonzero(w.F0 != 0)
    faces = np.unique(np.concatenate([rng.choice(geo, min(n_sample, geo.size), replace=False),
                                      rng.choice(flux, n_sample, replace=False)]))
    o = oracle.Oracle(w.mesh)
    V, _, S, _ = o.geometry()
    Up = o.set_velocity(w.U0c, w.F0)
    st_off, st_cells = o.stencil()
    need = np.unique(np.concatenate([st_cells[st_off[f]:st_off[f + 1]] for f in faces]))
    o.reconstruct_subset(alpha, need)
    r = o.faces_subset(w.dt[step], w.scale[step], alpha, faces)
    sdt = abs(w.scale[step] * w.dt[step])
    # gross swept volume |S_f| max|s dt U_p|: FP64 evaluations of the signed
    # polyhedron volume agree to a few eps of it
    m = w.mesh
    n = np.diff(m.face_offsets)
    sp = np.linalg.norm(Up, axis=1)[m.face_points]
    mx = np.zeros(m.n_faces)
    np.maximum.at(mx, np.repeat(np.arange(m.n_faces), n), sp)
    G = (np.linalg.norm(S, axis=1) * mx * sdt)[faces]
    T = np.abs(w.F0[faces] * sdt)
    ok = (w.F0[faces] != 0) & (r["status"] == 0)
    # rounding floor of a polyhedron's tetrahedra: their edges are as long as
    # the face (diameter d_f) however short the sweep; max(V_owner, d_f^3)
    face_of = np.repeat(np.arange(m.n_faces), n)
    P = m.points[m.face_points]
    ctr = np.zeros((m.n_faces, 3))
    np.add.at(ctr, face_of, P)
    ctr /= n[:, None]
    rad = np.zeros(m.n_faces)
    np.maximum.at(rad, face_of, np.linalg.norm(P - ctr[face_of], axis=1))
    floor = np.maximum(V[m.owner], (2.0 * rad) ** 3)[faces]
    # the oracle's volume at the GPU's lambda against F dt, relative to
    # max(|F dt|, G) (lambda is ill-conditioned where V' is small)
    sub = faces[ok][::4]
    res = [abs(o.flux_volume(f, w.dt[step], w.scale[step], lam[f]) - w.F0[f] * w.scale[step]
               * w.dt[step]) for f in sub]
    ref = np.maximum(np.maximum(T[ok][::4], G[ok][::4]), 1e-2 * floor[ok][::4])
    lam_err = float((np.asarray(res) / ref).max())
    tol = 1e-12 * np.maximum(np.maximum(T, G), 1e-2 * floor)
    ratio = float((np.abs(vph[faces] - r["vphase"]) / tol).max())
    flags_equal = bool(np.array_equal(status[faces], r["status"].astype(np.uint8)))
    return {"faces": int(faces.size), "geometric": int(min(n_sample, geo.size)),
            "max_volume_residual_at_gpu_lambda": lam_err, "max_vphase_err_over_tol": ratio,
            "flags_equal": flags_equal,
            "ok": bool(lam_err < 1e-12 and ratio <= 1.0 and flags_equal)}


def _make_instance(i, count, seed, n_lo, n_hi, steps):
    import workloads as W
    return W.batch_instances(count, seed, (n_lo, n_hi), steps, first=i, stop=i + 1)[0]


def generate_instances(count, seed, n_range, steps, workers):
    """The batched workload's instances, built in parallel host processes."""
    import multiprocessing as mp
    args = [(i, count, seed, n_range[0], n_range[1], steps) for i in range(count)]
    out = [None] * count
    t0 = time.perf_counter()
    # largest first: the pool's tail is then made of small instances
    order = sorted(range(count), key=lambda i: -_instance_size_hint(i, seed, n_range))
    with mp.get_context("fork").Pool(workers) as pool:
        for k, (i, w) in enumerate(zip(order, pool.imap(_make_star, [args[i] for i in order]))):
            out[i] = w
            if (k + 1) % 32 == 0 or k + 1 == count:
                log(f"[bench] generated {k + 1}/{count} instances ({time.perf_counter() - t0:.0f} s)")
    return out


def _make_star(a):
    return _make_instance(*a)


def _instance_size_hint(i, seed, n_range):
    import numpy as np
    return int(np.random.default_rng([seed, i]).integers(n_range[0], n_range[1] + 1))


def run_batched(args):
    """The batched form against the plain per-instance loop on the batched
    workload: 256 hex meshes N^3, N ~ U{16..96} (odd instances refined once
    around their sphere), random sphere and rigid rotation, 100 steps each at
    cell Courant number 0.5.  Both runs start from alpha^0 on the same
    resident meshes; every mesh's final alpha must be bitwise the same."""
    import numpy as np
    import torch

    import paper_1305_3417_amd as vof

    count, steps = args.instances, args.steps
    workers = max(1, min(16, (os.cpu_count() or 1)))
    log(f"[bench] generating {count} instances with {workers} processes")
    ws = generate_instances(count, 3417, (args.n_min, args.n_max), steps, workers)
    ctx = vof.vof_context_create(0)
    meshes = []
    t0 = time.perf_counter()
    for k, w in enumerate(ws):
        m = vof.upload_mesh(ctx, w.mesh)
        vof.vof_set_alpha(m, w.alpha0)
        vof.vof_set_velocity(m, w.U0c, w.F0)
        meshes.append(m)
        if (k + 1) % 32 == 0 or k + 1 == count:
            log(f"[bench] uploaded {k + 1}/{count} meshes ({time.perf_counter() - t0:.0f} s, "
                f"{sum(x.info.device_bytes for x in meshes) / 2**30:.1f} GiB)")
    dt = np.stack([w.dt[:steps] for w in ws])
    sc = np.stack([w.scale[:steps] for w in ws])
    flux_faces = sum(int(np.count_nonzero(w.F0)) for w in ws)
    cells = sum(w.mesh.n_cells for w in ws)

    def reset():
        for w, m in zip(ws, meshes):
            vof.vof_set_alpha(m, w.alpha0)
        torch.cuda.synchronize()

    def geo_total():
        return sum(vof.vof_get_stats(m)["geometric_faces"] for m in meshes)

    # plain loop: one vof_advect per mesh, each its own captured step graph
    Wm = args.warmup
    for w, m in zip(ws, meshes):
        vof.vof_advect(m, w.dt[:Wm], w.scale[:Wm])
    for m in meshes:
        vof.vof_synchronize(m)
    reset()
    log(f"[bench] plain loop: {count} meshes x {steps} steps")
    t0 = time.perf_counter()
    for w, m in zip(ws, meshes):
        vof.vof_advect(m, w.dt[:steps], w.scale[:steps])
    for m in meshes:
        vof.vof_synchronize(m)
    t_plain = time.perf_counter() - t0
    geo_plain = geo_total()
    a_plain = [vof.vof_read_alpha(m) for m in meshes]
    log(f"[bench] plain loop {t_plain:.3f} s")

    b = vof.vof_batch_create(ctx, meshes)
    tune = None
    if args.autotune:
        reset()
        tune = vof.vof_autotune(b, dt[:, :args.tune_steps], sc[:, :args.tune_steps],
                                args.tune_cache)
        log(f"[bench] autotuned {tune}")
    reset()
    vof.vof_batch_advect(b, dt[:, :Wm], sc[:, :Wm])   # captures the batch step
    vof.vof_batch_synchronize(b)
    reset()
    log(f"[bench] batched: {count} meshes x {steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vof.vof_batch_advect(b, dt, sc)
    vof.vof_batch_synchronize(b)
    t_batch = time.perf_counter() - t0
    geo_batch = geo_total()
    diff = {ws[i].name + f"#{i}": float(np.abs(vof.vof_read_alpha(m) - a).max())
            for i, (m, a) in enumerate(zip(meshes, a_plain))}
    diff = {k: v for k, v in diff.items() if v != 0.0 or not np.isfinite(v)}
    same = not diff
    log(f"[bench] batched {t_batch:.3f} s, alpha bitwise equal to the plain loop: {same}"
        + ("" if same else f" (differing meshes: {diff})"))
    cfg = vof.vof_batch_get_config(b).as_dict()

    parity = None
    if not args.no_parity:
        import oracle
        small = sorted(range(count), key=lambda i: ws[i].mesh.n_cells)[:2]
        errs = {}
        for i in small:
            o = oracle.Oracle(ws[i].mesh)
            o.set_velocity(ws[i].U0c, ws[i].F0)
            a, _, _, _ = o.advect(ws[i].alpha0, ws[i].dt[:steps], ws[i].scale[:steps])
            errs[ws[i].name] = float(np.abs(a - a_plain[i]).max())
        parity = {"oracle_max_abs_alpha_err": errs, "ok": max(errs.values()) < 1e-10}
        log(f"[bench] parity {parity}")

    v_batch = flux_faces * steps / t_batch
    v_plain = flux_faces * steps / t_plain
    out = {
        "metric": METRIC, "value": v_batch, "unit": "face-fluxes/s", "n_gpus": 1,
        "steps": steps, "warmup": Wm, "ms_per_step": t_batch * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {count} hex meshes N^3, N ~ U{{{args.n_min}.."
                               f"{args.n_max}}} (odd instances refined 2:1 around the sphere), "
                               f"sphere r ~ U[0.1, 0.2], random rigid rotation, cell Courant "
                               f"0.5, {steps} steps, seed 3417",
                   "instances": count, "cells": int(cells), "flux_faces_per_step": flux_faces,
                   "parallelism": "single GPU"},
        "form": "batched",
        "plain_loop": {"value": v_plain, "seconds": t_plain, "ms_per_step": t_plain * 1e3 / steps},
        "batched_over_plain": v_batch / v_plain,
        "seconds": t_batch,
        "alpha_bitwise_equal_to_plain": bool(same),
        "geometric_faces": {"plain": int(geo_plain), "batched": int(geo_batch)},
        "cell_updates_per_s": cells * steps / t_batch,
        "launch_config": cfg, "autotune": tune,
        "device_gib": sum(x.info.device_bytes for x in meshes) / 2**30,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    b.close()
    for m in meshes:
        m.close()
    vof.vof_context_destroy(ctx)


SERVED_HEX_N = (22, 32, 45, 64, 90, 126)      # 1.1e4 .. 2.0e6 cells, log-spaced
SERVED_TET_N = (12, 17, 24, 34, 49, 69)       # 6 N^3: 1.0e4 .. 2.0e6 cells
SERVED_SPHERES = 4                            # alpha0 draws per mesh


def _served_template(args):
    kind, n, seed = args
    import numpy as np

    import workloads as W
    tpl = W.deformation_template(kind, n)
    rng = np.random.default_rng([seed, n, 0 if kind == "hex" else 1])
    # alpha0 of a few random spheres (r ~ U[0.1, 0.2], centre ~ U[0.3, 0.7]^3)
    alphas = [W.served_request(tpl, rng, 1)[0] for _ in range(SERVED_SPHERES)]
    return tpl, alphas


def run_served(args):
    """The served form against the plain per-request loop: a Poisson stream of
    advection requests (deformation field, eq. 4.6) on hex and jittered-tet
    meshes of 1e4 to 2e6 cells (log-spaced), K ~ U{10..200} steps each, state
    admitted by a fixed HBM budget.  Both serve the same requests at the same
    arrival times; every served result must equal its plain result bitwise.
    A second pass submits every request at once (saturation): capacity."""
    import multiprocessing as mp
    import threading

    import numpy as np
    import torch

    import paper_1305_3417_amd as vof

    seed, nreq = 5, args.requests
    workers = max(1, min(16, (os.cpu_count() or 1)))
    specs = [("hex", n, seed) for n in SERVED_HEX_N] + [("tets", n, seed) for n in SERVED_TET_N]
    log(f"[bench] generating {len(specs)} meshes and {SERVED_SPHERES} spheres each "
        f"({workers} processes)")
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        made = pool.map(_served_template, sorted(specs, key=lambda s: -s[1]))
    by = {(t.meta["kind"], t.meta["n"]): (t, al) for t, al in made}
    tpls = [by[(k, n)] for k, n, _ in specs]
    log(f"[bench] generated in {time.perf_counter() - t0:.0f} s")
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(nreq):
        kind = int(rng.integers(2))           # hex or tets, even odds
        i = kind * len(SERVED_HEX_N) + int(rng.integers(len(SERVED_HEX_N)))
        K = int(rng.integers(10, 201))
        sph = int(rng.integers(SERVED_SPHERES))
        reqs.append((i, sph, K))
    gaps = rng.exponential(1.0, size=nreq)    # Poisson arrivals, scaled by the rate below
    ctx = vof.vof_context_create(0)
    meshes = [vof.upload_mesh(ctx, t.mesh) for t, _ in tpls]
    nflux = [int(np.count_nonzero(t.F0)) for t, _ in tpls]
    sched = {}

    def schedule(i, K):
        if (i, K) not in sched:
            t = tpls[i][0]
            dt = float(t.dt[0])
            tt = (np.arange(K) + 0.5) * dt
            sched[(i, K)] = (np.full(K, dt), np.cos(np.pi * tt / t.meta["T"]))
        return sched[(i, K)]

    def plain(r):
        i, sph, K = r
        t, al = tpls[i]
        dt, sc = schedule(i, K)
        vof.vof_set_alpha(meshes[i], al[sph])
        vof.vof_set_velocity(meshes[i], t.U0c, t.F0)
        vof.vof_advect(meshes[i], dt, sc)
        return vof.vof_read_alpha(meshes[i])

    # plain service time of every request (one warm pass over the meshes first)
    for i in range(len(tpls)):
        plain((i, 0, 10))
    torch.cuda.synchronize()
    work = sum(nflux[i] * K for i, _, K in reqs)
    # plain per-request loop at the offered rate: completion_k =
    # max(arrival_k, completion_{k-1}) + service_k, run for real in arrival order
    def run_plain(arrivals):
        out, lat = [], []
        t_start = time.perf_counter()
        for r, ta in zip(reqs, arrivals):
            now = time.perf_counter() - t_start
            if ta > now:
                time.sleep(ta - now)
            out.append(plain(r))
            lat.append(time.perf_counter() - t_start - ta)
        span = time.perf_counter() - t_start - arrivals[0]
        return out, np.array(lat), span

    zero = np.zeros(nreq)
    log(f"[bench] plain loop, all {nreq} requests at once")
    a_plain, lat_sat, span_plain_sat = run_plain(zero)
    cap_plain = work / span_plain_sat
    rate = args.rate if args.rate else 0.7 * nreq / span_plain_sat   # requests per second
    arrivals = np.cumsum(gaps / rate) - gaps[0] / rate
    log(f"[bench] plain capacity {cap_plain:.3e} face-fluxes/s; offered rate {rate:.1f} "
        f"requests/s")
    log(f"[bench] plain loop, Poisson arrivals")
    _, lat_plain, span_plain = run_plain(arrivals)

    def run_served_once(arr):
        srv = vof.vof_server_create(ctx, args.budget_gib << 30)
        jobs = [None] * nreq
        t_start = time.perf_counter()

        def submit():
            for k, (r, ta) in enumerate(zip(reqs, arr)):
                now = time.perf_counter() - t_start
                if ta > now:
                    time.sleep(ta - now)
                i, sph, K = r
                t, al = tpls[i]
                dt, sc = schedule(i, K)
                jobs[k] = vof.vof_server_submit(srv, meshes[i], al[sph], t.U0c, t.F0, dt, sc)
        th = threading.Thread(target=submit)
        th.start()
        th.join()
        res = [vof.vof_server_wait(j) for j in jobs]
        span = time.perf_counter() - t_start - arr[0]
        st = vof.vof_server_get_stats(srv)
        srv.close()
        return [a for a, _ in res], np.array([l for _, l in res]), span, st

    log(f"[bench] served, all {nreq} requests at once (budget {args.budget_gib} GiB)")
    a_srv_sat, lat_srv_sat, span_srv_sat, st_sat = run_served_once(zero)
    log(f"[bench] served, Poisson arrivals")
    a_srv, lat_srv, span_srv, st = run_served_once(arrivals)
    same = sum(np.array_equal(x, y) for x, y in zip(a_plain, a_srv))
    same_sat = sum(np.array_equal(x, y) for x, y in zip(a_plain, a_srv_sat))
    log(f"[bench] served results bitwise equal to plain: {same}/{nreq} (Poisson), "
        f"{same_sat}/{nreq} (all at once)")
    cap_srv = work / span_srv_sat
    pct = lambda a, q: float(np.percentile(a, q))  # noqa: E731
    out = {
        "metric": METRIC, "value": cap_srv, "unit": "face-fluxes/s", "n_gpus": 1,
        "steps": int(sum(K for _, _, K in reqs)), "warmup": 1,
        "ms_per_step": span_srv_sat * 1e3 / max(st_sat["ticks"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served: {nreq} requests, deformation field (eq. 4.6, T=3), "
                               f"hex N^3 N in {list(SERVED_HEX_N)} and jittered tets 6 N^3 N in "
                               f"{list(SERVED_TET_N)} (1e4..2e6 cells, even odds), random sphere "
                               f"r ~ U[0.1,0.2] ({SERVED_SPHERES} per mesh), K ~ U{{10..200}}, "
                               f"cell Courant 0.5, seed {seed}, HBM budget {args.budget_gib} GiB",
                   "requests": nreq, "face_flux_work": work, "parallelism": "single GPU"},
        "form": "served",
        "saturated": {"served_face_fluxes_per_s": cap_srv, "plain_face_fluxes_per_s": cap_plain,
                      "served_over_plain": cap_srv / cap_plain,
                      "served_s": span_srv_sat, "plain_s": span_plain_sat,
                      "server_stats": st_sat},
        "poisson": {"rate_requests_per_s": rate, "offered_load_of_plain_capacity": 0.7,
                    "served": {"p50_ms": pct(lat_srv, 50) * 1e3, "p99_ms": pct(lat_srv, 99) * 1e3,
                               "face_fluxes_per_s": work / span_srv, "span_s": span_srv},
                    "plain": {"p50_ms": pct(lat_plain, 50) * 1e3,
                              "p99_ms": pct(lat_plain, 99) * 1e3,
                              "face_fluxes_per_s": work / span_plain, "span_s": span_plain},
                    "server_stats": st},
        "bitwise_equal_to_plain": {"poisson": int(same), "saturated": int(same_sat),
                                   "of": nreq},
    }
    print(json.dumps(out), flush=True)
    for m in meshes:
        m.close()
    vof.vof_context_destroy(ctx)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the whole run; batched 100)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=None,
                    help="mesh is n^3 hexahedra (default 128), or n^3 cubes of six jittered "
                         "tetrahedra for tets (default 80)")
    ap.add_argument("--workload",
                    choices=["deform3d", "shear3d", "tets", "disc2d", "batched", "served"],
                    default="deform3d",
                    help="deform3d (eq. 4.6, fixed dt; the headline case), disc2d (the "
                         "64x64x1 layer of the 2D translation, 50 steps), shear3d "
                         "(eq. 4.5, adaptive Courant dt), tets (slotted sphere rotating "
                         "on jittered tetrahedra), batched (many meshes per launch against "
                         "the plain per-mesh loop) or served (a request stream against the "
                         "plain per-request loop)")
    ap.add_argument("--requests", type=int, default=400, help="served: number of requests")
    ap.add_argument("--rate", type=float, default=None,
                    help="served: arrivals per second (default 0.7 x the plain loop's "
                         "measured capacity)")
    ap.add_argument("--budget-gib", type=int, default=96, help="served: HBM budget")
    ap.add_argument("--instances", type=int, default=256, help="batched: number of meshes")
    ap.add_argument("--n-min", type=int, default=16, help="batched: smallest N")
    ap.add_argument("--n-max", type=int, default=96, help="batched: largest N")
    ap.add_argument("--autotune", action="store_true",
                    help="batched: pick the launch configuration by timing candidates")
    ap.add_argument("--tune-steps", type=int, default=6)
    ap.add_argument("--tune-cache", default=None,
                    help="batched: JSON cache of tuned configurations")
    ap.add_argument("--window-only", action="store_true",
                    help="only advance to the middle of the run (captured steps) and launch "
                         "the profiled window's steps kernel by kernel, then print the work "
                         "counted in it (for rocprofv3 counter runs)")
    ap.add_argument("--band-wisps", action="store_true",
                    help="run the step with the narrow band and wisp redistribution "
                         "(Section 2.3) after the update")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (read BYTES, write BYTES) "
                         "three times: the reference kernel for scaling HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the flux path is measured on one GPU's share of the mesh)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1305_3417_amd as vof
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 8, "bytes_written": n * 8,
                          "launches": 3}), flush=True)
        return
    if args.workload == "served":
        run_served(args)
        return
    if args.workload == "batched":
        if args.steps is None:
            args.steps = 100
        run_batched(args)
        return
    WORKLOAD[0] = args.workload
    if args.n is None:
        args.n = {"tets": 80, "disc2d": 64}.get(args.workload, 128)
    WORKLOAD.append(args.n)
    Wm = args.warmup
    log(f"[bench] generating {args.workload} {args.n}^3")
    make = {"deform3d": W.deform3d, "shear3d": W.shear3d, "tets": W.rotate_tets,
            "disc2d": W.disc2d}[args.workload]
    w = make(args.n)  # the whole run: to T, or one revolution
    K = w.n_steps if args.steps is None else min(args.steps, w.n_steps)
    if args.workload == "tets" and args.steps is None:
        K = min(K, 2000)  # a revolution is ~26k steps at Courant 0.5 on these slivers
    P = min(K, 20)   # profiled steps, from the middle of the timed run
    mid = K // 2
    ctx = vof.vof_context_create(0)
    log("[bench] uploading mesh")
    mesh = vof.upload_mesh(ctx, w.mesh)
    if args.band_wisps:
        p = vof.vof_get_params(mesh)
        p.narrow_band, p.wisps = 1, 1
        vof.vof_set_params(mesh, p)
    vof.vof_set_velocity(mesh, w.U0c, w.F0)
    vof.vof_set_alpha(mesh, w.alpha0)
    if args.window_only:
        vof.vof_advect(mesh, w.dt[:mid], w.scale[:mid])
        vof.vof_synchronize(mesh)
        vof.vof_profile_enable(mesh, True)
        sp0 = vof.vof_get_stats(mesh)
        vof.vof_advect(mesh, w.dt[mid:mid + P], w.scale[mid:mid + P])
        vof.vof_synchronize(mesh)
        sp1 = vof.vof_get_stats(mesh)
        prof = {k: v for k, v in vof.vof_read_profile(mesh).items() if v[1] > 0}
        print(json.dumps({"window": [mid, mid + P], "workload": args.workload, "n": args.n,
                          "per_step": {k: (sp1[k] - sp0[k]) / P for k in
                                       ("face_fluxes", "geometric_faces", "interface_cells",
                                        "clip_pairs", "general_tets")},
                          "kernels_us": {k: v[0] / v[1] * 1e3 for k, v in prof.items()}}),
              flush=True)
        return
    log(f"[bench] warmup {Wm} steps")
    vof.vof_advect(mesh, w.dt[:max(Wm, 1)], w.scale[:max(Wm, 1)])
    vof.vof_synchronize(mesh)
    vof.vof_set_alpha(mesh, w.alpha0)     # the timed run starts from alpha^0 again
    # timed region: steps 0 .. K-1 as the library runs them (one captured graph
    # per step, replayed on the library's stream), in segments whose times give
    # the rate along the run
    nseg = 1 if args.workload == "disc2d" else min(K, 24)  # 50 steps of ~0.1 ms: one segment
    bounds = np.linspace(0, K, nseg + 1).astype(int)
    log(f"[bench] timing {K} steps ({nseg} segments)")
    seg_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    for a, b in zip(bounds[:-1], bounds[1:]):
        vof.vof_advect(mesh, w.dt[a:b], w.scale[a:b])
        vof.vof_synchronize(mesh)
        now = time.perf_counter()
        seg_ms.append((now - last) * 1e3 / (b - a))
        last = now
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st1 = vof.vof_get_stats(mesh)
    face_fluxes = st1["face_fluxes"]
    geo = st1["geometric_faces"]
    value = face_fluxes / elapsed
    log(f"[bench] {elapsed * 1e3 / K:.3f} ms/step, {value:.3e} face-fluxes/s")
    a_end = vof.vof_read_alpha(mesh)
    V = W.generated_volumes(w.mesh)
    m0 = float((w.alpha0 * V).sum())
    e_g = float((V * np.abs(a_end - w.alpha0)).sum())
    run = {"steps": int(K), "t_end": float(np.sum(w.dt[:K])),
           "segments": [{"steps": [int(a), int(b)], "ms_per_step": float(t)}
                        for a, b, t in zip(bounds[:-1], bounds[1:], seg_ms)],
           "alpha_min": st1["alpha_min"], "alpha_max": st1["alpha_max"],
           "unreached_faces_per_step": st1["unreached_faces"] / K,
           "geometric_faces_per_step": geo / K,
           "mass_plus_outflow_rel_err": abs(st1["mass"] + st1["ledger"] - m0) / m0,
           "E_g_at_end": e_g}
    if args.workload == "deform3d" and K == w.n_steps and args.n == 128:
        run["E_g_paper_table4_128_co05"] = 1.30304e-3   # context: same method, other setup
    log(f"[bench] run: {run}")

    # per-kernel durations over P steps from the middle of the run, launched
    # kernel by kernel, each bracketed by HIP events on the library's stream
    vof.vof_set_alpha(mesh, w.alpha0)
    vof.vof_advect(mesh, w.dt[:mid], w.scale[:mid])
    vof.vof_synchronize(mesh)
    vof.vof_profile_enable(mesh, True)
    vof.vof_read_profile(mesh)
    sp0 = vof.vof_get_stats(mesh)
    tp0 = time.perf_counter()
    vof.vof_advect(mesh, w.dt[mid:mid + P], w.scale[mid:mid + P])
    vof.vof_synchronize(mesh)
    prof_elapsed = time.perf_counter() - tp0
    prof = {k: v for k, v in vof.vof_read_profile(mesh).items() if v[1] > 0}
    vof.vof_profile_enable(mesh, False)
    sp1 = vof.vof_get_stats(mesh)
    log("[bench] per-kernel: " + ", ".join(f"{k} {v[0] / max(v[1], 1) * 1e3:.1f}us"
                                           for k, v in prof.items()))

    # dominant kernel and its roofline figure: algorithmic flops per launch
    # (per-unit figure x units per launch, counted over the profiled steps)
    # over its average duration
    dom = max(prof, key=lambda k: prof[k][0])
    dom_ms, dom_n = prof[dom]
    avg_s = dom_ms / dom_n / 1e3
    units = {"flux": ((sp1["face_fluxes"] - sp0["face_fluxes"]) / P, FLUX_FLOPS_PER_QUAD_FACE,
                      "face-fluxes", "face_fluxes"),
             "clip": ((sp1["clip_pairs"] - sp0["clip_pairs"]) / P, CLIP_FLOPS_PER_PAIR,
                      "overlapping (tet, cell) pairs", "clip_pairs"),
             "plane": ((sp1["interface_cells"] - sp0["interface_cells"]) / P,
                       PLANE_FLOPS_PER_CELL, "interface cells", "interface_cells")}
    roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": None, "traffic": recorded_traffic(dom),
            "avg_launch_us": avg_s * 1e6, "profiled_steps": P, "profiled_from_step": mid}
    if dom in units:
        n_units, estimate, what, key = units[dom]
        measured = recorded_flops(dom, key)
        # executed FP64 flops counted on the same window (rocprofv3 FP64
        # instruction counters x active lanes) when taken on these sources,
        # else the per-unit estimate
        per_unit = measured[0] if measured else estimate
        achieved = n_units * per_unit / avg_s / 1e12
        at_estimate = n_units * estimate / avg_s / 1e12
        roof.update({"achieved": achieved, "frac": achieved / PEAK_FP64_TFLOPS,
                     "units_per_launch": n_units, "flop_per_unit": per_unit,
                     "flop_per_unit_source": "rocprofv3 FP64 counters" if measured
                     else "estimate", "flop_per_unit_estimate": estimate,
                     "achieved_at_estimate": at_estimate,
                     "frac_at_estimate": at_estimate / PEAK_FP64_TFLOPS, "unit_kind": what})
        if measured and measured[1]:
            issue = measured[1] / avg_s
            roof["valu_issue"] = {"wave_insts_per_s": issue, "peak": PEAK_VALU_WAVE_INSTS,
                                  "frac": issue / PEAK_VALU_WAVE_INSTS}
    step_after = mid + P

    parity = None
    if not args.no_parity:
        log("[bench] parity check of one extra step against the oracle")
        parity = parity_check(vof, mesh, w, step_after)
        log(f"[bench] parity {parity}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] oracle CPU baseline")
        a = vof.vof_read_alpha(mesh)
        cpu = cpu_baseline(w, a, step_after + 1)
        log(f"[bench] cpu {cpu}")
    out = {
        "metric": METRIC, "value": value, "unit": "face-fluxes/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": {
                       "deform3d": f"deform3d hex {args.n}^3 (eq. 4.6, T=3, sphere r=0.15 at "
                                   f"(0.35,0.35,0.35), Co 0.5, dt=1/{4 * args.n})",
                       "shear3d": f"shear3d hex {args.n}^3 (eq. 4.5, T=3, u_max=1, R=0.5, "
                                  f"sphere r=0.15 at (0.5,0.75,0.25), adaptive Courant dt at "
                                  f"Co 0.5)",
                       "tets": f"tets {args.n}^3 cubes x 6 jittered Kuhn tetrahedra (slotted "
                               f"sphere r=0.15 at (0.5,0.75,0.5), rotation about z, "
                               f"omega=2 pi, cell Courant 0.5, dt=1/{w.meta.get('steps_per_rev')}"
                               f")",
                       "disc2d": f"disc2d hex {args.n}x{args.n}x1 layer (disc r=0.15 at "
                                 f"(0.5,0.75), U=(1,0.5,0), Co 0.5, dt=0.5h/sqrt(1.25))",
                       }[args.workload]
                               + f", steps 0..{K - 1} of {w.n_steps} (timed from alpha^0)",
                   "cells": int(w.mesh.n_cells), "faces": int(w.mesh.n_faces),
                   "band_wisps": bool(args.band_wisps),
                   "parallelism": "single GPU"},
        "cell_updates_per_s": w.mesh.n_cells * K / elapsed,
        "geometric_faces_per_step": geo / K,
        "general_clip_tets_per_step": st1["general_tets"] / K,
        "wisps_per_step": st1["wisps"] / K,
        "face_fluxes_per_step": face_fluxes / K,
        "run": run,
        "kernels_us": {k: v[0] / max(v[1], 1) * 1e3 for k, v in prof.items()},
        "profiled_ms_per_step": prof_elapsed * 1e3 / P,
        "roofline": roof,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    vof.vof_mesh_destroy(mesh)
    vof.vof_context_destroy(ctx)


if __name__ == "__main__":
    main()
