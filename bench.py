#!/usr/bin/env python3
"""Throughput of the Heun-integrated stochastic LLG step on one MI355X.

Workload: periodic bcc block of 160^3 cells (8,192,000 spins) with first
(J1 = 7.05e-21 J, 8 per site) and second (J2 = 3.0e-21 J, 6 per site)
neighbours, mu_s = 2.22 muB, k_u = 5.65e-25 J along z, T = 300 K,
lambda = 0.05, dt = 1e-16 s, spins starting along +z, noise seed 4.  A step
is one full Heun step over the whole system: thermal noise, exchange
gather, anisotropy, Zeeman, predictor, corrector, renormalisation, and the
FP64 reductions of m and E.  Inputs are resident in HBM before timing.

Prints one JSON line: FP32 spin-steps/s as `value`, with the FP64 run, the
FP32-vs-FP64 difference, the roofline of the step kernels, the serving
workload's p50/p99 latency and the single-threaded CPU oracle beside it.
"""
import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-steps/s (Heun sLLG) FP32 vs FP64 at 1 GPU; p50/p99 latency of batched sweeps"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1310_6143_amd", "csrc")
# committed rocprofv3 counter summaries, each tied to the sources of the
# kernels it measured (and, for the fused step, to the work-item shape)
COUNTER_FILES = {
    "two_launch": (os.path.join(ROOT, "profiles", "bcc160_step_hbm_counters.md"),
                   ["kernels.hip", "device_common.hpp"]),
    "fused": (os.path.join(ROOT, "profiles", "bcc160_fused_step_counters.md"),
              ["fused.hip", "device_common.hpp"]),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_spin_step(w_bytes, mean_degree):
    """Bytes the method itself must move per spin and step: read S once,
    write S once (6w), read the neighbour structure once (4 B row offset plus
    4 B per neighbour entry); the thermal noise is generated, not read."""
    return 6 * w_bytes + 4 + 4 * mean_degree


def kernel_hash(kind):
    h = hashlib.sha256()
    for name in COUNTER_FILES[kind][1]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_value(kind, key, shape=None):
    """A machine-readable value of the committed rocprofv3 counter summary
    of `kind`, or None when it is missing, the kernels changed since it was
    taken, or (fused step) it was taken at another work-item shape."""
    path = COUNTER_FILES[kind][0]
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    if shape is not None:    # values per work-item shape: key[tx,ty,planes,threads]
        key = re.escape(f"{key}[{','.join(str(x) for x in shape)}]")
    v = re.search(rf"^{key}:\s*([0-9.eE+]+)", text, re.M)
    if not h or not v or h.group(1) != kernel_hash(kind):
        return None
    return float(v.group(1))


def run_gpu(w, precision, steps, warmup, torch, launch=None, autotune=False, fused=1, fused_shape=None):
    import paper_1310_6143_amd as sl

    t0 = time.time()
    sysm = sl.from_workload(w, precision=precision, check_symmetry=False)
    sysm.set_option("fused", fused)
    if fused_shape and sysm.get_option("lattice") == 2:
        for key, v in zip(("fused_tile_x", "fused_tile_y", "fused_planes", "fused_threads"), fused_shape):
            sysm.set_option(key, v)
    log(f"precision {'fp32' if precision == sl.FP32 else 'fp64'}: set-up {time.time() - t0:.1f} s")
    st = torch.cuda.Stream()
    # device buffers first, so that nothing allocates (and leaves the GPU
    # idle) between the autotuner's trial steps, the warmup and the timing
    m_w = torch.empty((max(warmup, 1), 3), dtype=torch.float64, device="cuda")
    E_w = torch.empty(max(warmup, 1), dtype=torch.float64, device="cuda")
    m_dev = torch.empty((steps, 3), dtype=torch.float64, device="cuda")
    E_dev = torch.empty(steps, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    if launch:
        sysm.set_option("xcd_remap", launch[0])
        sysm.set_option("grid_scale_pct", launch[1])
        if len(launch) > 2:
            sysm.set_option("tile_order", launch[2])
        choice = {k: sysm.get_option(k) for k in ("xcd_remap", "grid_scale_pct", "graph_steps", "tile_order")}
    elif autotune and not fused_shape:
        # also brings the GPU out of its idle clocks before the timed steps
        tuned_us, choice = sysm.autotune(25, stream=st)
        log(f"  autotune: {tuned_us:.1f} us/step with {choice}")
    else:   # the library's default launch shape (the one the counter summary was taken at)
        choice = {k: sysm.get_option(k) for k in ("xcd_remap", "grid_scale_pct", "graph_steps", "tile_order")}
    if warmup:
        sysm.integrate_dev(warmup, m_w, E_w, stream=st)
    st.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(st)
    sysm.integrate_dev(steps, m_dev, E_dev, stream=st)
    ev1.record(st)
    st.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1)
    m = m_dev.cpu().numpy()
    E = E_dev.cpu().numpy()
    if not np.all(np.isfinite(E)):
        raise SystemExit("non-finite energy in the timed run")
    fused_on = sysm.get_option("fused_active")
    shape = [sysm.get_option(k) for k in ("fused_tile_x", "fused_tile_y", "fused_planes", "fused_threads")]
    sysm.close()
    log(f"  {steps} steps in {ms:.2f} ms (events), {wall * 1e3:.2f} ms (wall); fused {fused_on} shape {shape}")
    choice = dict(choice, fused=int(fused_on), fused_shape=shape if fused_on else None)
    return {"ms": ms, "wall_s": wall, "m": m, "E": E, "launch": choice}


def run_serving(args):
    """The serving workload: Poisson arrivals of independent simple-cubic
    requests admitted by HBM budget into the continuous-batching server."""
    import paper_1310_6143_amd as sl
    from spin_systems import serving_requests, sc_request_system

    reqs = serving_requests(n_requests=args.serving_requests)
    t0 = time.time()
    systems = [sc_request_system(r["L"], r["temperature"], r["H"], r["n_steps"], r["seed"]) for r in reqs]
    log(f"serving: {len(reqs)} requests prepared in {time.time() - t0:.1f} s")
    total = float(sum(w.n * w.n_steps for w in systems))
    with sl.Server(hbm_budget=args.serving_budget << 20, max_active=512, chunk_steps=args.serving_chunk,
                   precision=sl.FP32) as srv:
        # warm the server (graph capture, allocator) with one small request
        srv.wait(srv.submit(sc_request_system(8, 300.0, [0, 0, 0], 64, 1)), 60)
        tickets = []
        start = srv.clock()
        for r, w in zip(reqs, systems):
            delay = start + r["arrival_s"] - srv.clock()
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(w, n_avg=w.n_steps // 2))
        res = [srv.wait(t, 600) for t in tickets]
        stats = srv.stats()
    bad = [r for r in res if r["state"] != "done"]
    if bad:
        raise SystemExit(f"{len(bad)} serving requests did not complete")
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    return {
        "workload": "512 requests, Poisson arrivals at 200/s, periodic sc L^3 with L~U{8..48}, "
                    "T~U[0,1200] K, |H|~U[0,2] T, 2000..20000 steps, FP32",
        "requests": len(res),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "spin_steps_per_s": total / span,
        "busy_spin_steps_per_s": stats["spin_steps"] / max(stats["busy_seconds"], 1e-9),
        "total_spin_steps": total,
        "makespan_s": span,
        "chunks": int(stats["chunks"]),
        "launch_tuning": {"compositions_tuned": int(stats["tuned_compositions"]),
                          "last_shape": {"xcd_remap": int(stats["last_xcd_remap"]),
                                         "tile_order": int(stats["last_tile_order"])}},
    }


def run_sweep(kind, precision, args):
    """Full sweep workloads.  film: M(T) heating ramp 0..1500 K in 50 K steps
    with 5000 + 5000 steps per point and continuation (bcc 64x64x16 film).
    sphere: hysteresis H_z = -5..5 T in 0.1 T steps, 2000 steps per point
    (1000 + 1000 averaged), fcc particle of radius 8 nm at 10 K."""
    import paper_1310_6143_amd as sl
    from spin_systems import bcc_film, fcc_nanoparticle

    if kind == "film":
        w = bcc_film()
        pts = w.extra["temperatures"]
        n_eq, n_avg = w.extra["n_eq"], w.extra["n_avg"]
    else:
        w = fcc_nanoparticle()
        pts = np.stack([np.zeros_like(w.extra["fields_z"]), np.zeros_like(w.extra["fields_z"]),
                        w.extra["fields_z"]], axis=1)
        n_eq, n_avg = 1000, 1000
    if args.sweep_points:
        pts = pts[: args.sweep_points]
    sysm = sl.from_workload(w, precision=precision)
    sysm.integrate(10, record=False)              # first use: upload, graph capture
    t0 = time.perf_counter()
    if kind == "film":
        rows = sysm.sweep_temperature(pts, n_eq, n_avg, 10)
    else:
        rows = sysm.sweep_field(pts, n_eq, n_avg, 10)
    dt = time.perf_counter() - t0
    sysm.close()
    steps = len(pts) * (n_eq + n_avg)
    return {"spin_steps_per_s": w.n * steps / dt, "seconds": dt, "n_spins": w.n, "steps": steps,
            "points": [{"x": (float(r["T"]) if kind == "film" else float(r["H"][2])),
                        "m_abs": r["m_abs"], "m_abs_se": r["m_abs_se"], "m_z": float(r["m"][2]),
                        "E": r["E"], "E_se": r["E_se"]} for r in rows]}


def run_mc(precision, args):
    """Monte Carlo M(T) of the paper's simple-cubic test system (21,952 spins,
    J = 6.0e-21 J/link, periodic): heating 50..1000 K in 50 K steps with
    continuation, 5000 equilibration + 5000 averaging steps per point
    (the paper uses 50,000 each), records every step; then the Monte Carlo
    step rate of the 8,192,000-spin bcc block (50 steps with records)."""
    import paper_1310_6143_amd as sl
    from spin_systems import bcc_block, sc_reference

    w = sc_reference(L=28, temperature=50.0, seed=1)
    temps = np.arange(50.0, 1001.0, 50.0)
    n_eq = n_avg = args.mc_steps
    sysm = sl.from_workload(w, precision=precision)
    sysm.mc(10, record=False)                       # first use: upload
    rows = []
    t0 = time.perf_counter()
    for T in temps:
        sysm.set_conditions(float(T), (0.0, 0.0, 0.0))
        r = sysm.mc_average(n_eq, n_avg, 10)
        rows.append({"x": float(T), "m_abs": r["m_abs"], "m_abs_se": r["m_abs_se"], "E": r["E"],
                     "E_se": r["E_se"], "acceptance": r["acceptance"]})
    dt = time.perf_counter() - t0
    sysm.close()
    steps = len(temps) * (n_eq + n_avg)
    blk = bcc_block(cells=args.cells)

    def block_rate(colouring):
        # colouring 1: the greedy colouring visits the declared lattice by
        # basis site and cell parity (four equal classes on this lattice);
        # 0: in ascending site order (ten unequal classes)
        g = sl.from_workload(blk, precision=precision, check_symmetry=False)
        g.set_option("mc_colouring", colouring)
        classes = g.get_option("mc_colours")
        g.mc(2)   # sllg_mc returns once its steps are done
        t1 = time.perf_counter()
        _, _, acc = g.mc(50)
        dt_blk = time.perf_counter() - t1
        t2 = time.perf_counter()
        g.mc(50, record=False)
        dt_sweep = time.perf_counter() - t2
        g.close()
        return {"n_spins": blk.n, "colour_classes": classes, "mc_steps": 50, "trials_per_s": blk.n * 50 / dt_blk,
                "ms_per_mc_step": dt_blk * 1e3 / 50, "ms_per_sweep_without_record": dt_sweep * 1e3 / 50,
                "acceptance": float(acc.sum()) / (blk.n * 50)}

    return {"spin_steps_per_s": w.n * steps / dt, "seconds": dt, "n_spins": w.n, "steps": steps,
            "points": rows, "block": block_rate(1), "block_ascending_colouring": block_rate(0)}


def run_sw(precision, args, n_angles=1024):
    """Quasi-static Stoner-Wohlfarth loops ("Angular variation of the
    Coercivity"): n_angles uncoupled spins (H_k = 2 k_u/mu_s = 1 T, easy axes
    at 0.05..89.95 degrees from the field), field along z from +1.5 to -1.5
    H_k in steps of 0.01 H_k, relaxed at each point to a torque of 1e-6 T
    (FP64; 2e-5 T in FP32, whose Heun updates stall below that), torque
    checked every 64 steps (one captured graph of steps between checks).
    Switching fields against the astroid."""
    import paper_1310_6143_amd as sl
    from spin_systems import MU_B, GAMMA, Workload
    from spin_systems.lattice import Lattice

    psi = np.radians(np.linspace(0.05, 89.95, n_angles))
    axes = np.stack([np.sin(psi), np.zeros(n_angles), np.cos(psi)], axis=1)
    lat = Lattice("uncoupled", np.zeros((n_angles, 3)), np.zeros(n_angles + 1, dtype=np.int64),
                  np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.uint8))
    mu = 1.5 * MU_B
    w = Workload(name="Stoner-Wohlfarth", lattice=lat, J=np.array([0.0]), mu_s=np.full(n_angles, mu),
                 k_u=np.full(n_angles, mu / 2), easy_axis=axes, alpha=1.0, gamma=GAMMA, dt=2e-13,
                 temperature=0.0, H=np.array([0.0, 0.0, 1.5]), seed=0, n_steps=0,
                 S0=np.tile([0.0, 0.0, 1.0], (n_angles, 1)))
    h = np.round(np.arange(150, -151, -1) * 0.01, 10)
    tol = 1e-6 if precision == sl.FP64 else 2e-5
    sysm = sl.from_workload(w, precision=precision)
    sysm.relax(tol, 200_000, check_every=64)            # first use: upload, graph capture
    # per point, to read every spin's projection on its easy axis
    t0 = time.perf_counter()
    proj = np.empty((h.size, n_angles))
    steps = np.empty(h.size, dtype=np.int64)
    for k in range(h.size):
        _, st = sysm.hysteresis(np.array([[0.0, 0.0, h[k]]]), tol, 200_000, check_every=64)
        steps[k] = st[0]
        proj[k] = (sysm.get_spins() * axes).sum(1)
    dt = time.perf_counter() - t0
    sysm.close()
    sw = h[np.argmax(proj < 0, axis=0)]
    h_sw = (np.cos(psi) ** (2 / 3) + np.sin(psi) ** (2 / 3)) ** -1.5
    miss = (sw < -h_sw - 0.0101) | (sw > -h_sw + 1e-6)
    return {"seconds": dt, "angles": n_angles, "field_points": int(h.size), "steps": int(steps.sum()),
            "unconverged_points": int((steps < 0).sum()), "torque_tol_T": tol,
            "angle_field_points_per_s": n_angles * h.size / dt,
            "switching_fields_off_the_astroid": int(miss.sum())}


def run_demag(precision, args):
    """Macrocell demagnetising field.  (1) All-pairs field update throughput:
    simple-cubic slab 128 x 128 x 32 atoms (a = 0.25 nm) in macrocells of 2
    atoms per edge: 65,536 cells, 4.3e9 pair terms per update.  (2) The
    paper's prolate-ellipsoid test: fcc (a = 0.354 nm), mu_s = 1.5 muB,
    H_k = 1 T along the long axis z, diameter 10 nm, height 20 nm,
    macrocells of 2 unit cells updated every 100 steps; LLG step rate with
    and without the field, and the easy-axis switching field with and
    without it (field 0.5 degree off z; each probe starts from +z, relaxes
    to 1e-4 T at T = 0 and is read as switched when m_z < 0; bisection to
    0.01 T)."""
    import paper_1310_6143_amd as sl
    from spin_systems import MU_B, GAMMA, Workload, fcc_ellipsoid, simple_cubic, with_demag

    def wl(lat, J, mu, ku, dt):
        n = lat.n
        return Workload(name="demag", lattice=lat, J=np.array([J]), mu_s=np.full(n, mu), k_u=np.full(n, ku),
                        easy_axis=np.tile([0.0, 0.0, 1.0], (n, 1)), alpha=1.0, gamma=GAMMA, dt=dt,
                        temperature=0.0, H=np.zeros(3), seed=5, n_steps=0, S0=np.tile([0.0, 0.0, 1.0], (n, 1)))

    out = {}
    slab = with_demag(wl(simple_cubic((128, 128, 32), (False, False, False)), 1e-21, 1.5 * MU_B, 0.0, 1e-16),
                      0.25, 0.5, every=1)
    S = np.random.default_rng(1).standard_normal((slab.lattice.n, 3))
    slab.S0 = S / np.linalg.norm(S, axis=1, keepdims=True)
    g = sl.from_workload(slab, precision=precision)
    g.demag_field()                                    # first use: upload
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        g.demag_field()
    dt = (time.perf_counter() - t0) / reps
    g.close()
    cells = 64 * 64 * 16
    pairs = cells * (cells - 1)
    out["update"] = {"cells": cells, "pair_terms": pairs, "seconds": dt, "pair_terms_per_s": pairs / dt,
                     "flops_per_pair": 31, "achieved_TFLOPs": 31 * pairs / dt / 1e12,
                     "note": "wall time of sllg_demag_field (update, copy of the cell fields, per-atom expansion)"}
    if args.demag_update_only:
        return out

    mu = 1.5 * MU_B
    lat = fcc_ellipsoid(0.354, (5.0, 5.0, 10.0))
    M = mu / (0.354e-9 ** 3 / 4)
    MU0 = 4e-7 * np.pi

    def system(demag):
        w = wl(lat, 1e-21, mu, mu / 2, 1e-15)
        return with_demag(w, 0.354, 0.708, every=100) if demag else w

    rates = {}
    for demag in (False, True):
        g = sl.from_workload(system(demag), precision=precision)
        g.integrate(200, record=False)
        t0 = time.perf_counter()
        g.integrate(2000, record=False)
        rates["with" if demag else "without"] = 2000 / (time.perf_counter() - t0)
        g.close()

    psi = np.radians(0.5)
    d = np.array([np.sin(psi), 0.0, np.cos(psi)])

    def switches(g, h):
        g.set_spins(np.tile([0.0, 0.0, 1.0], (lat.n, 1)))
        g.set_conditions(0.0, tuple(-h * d))
        try:
            g.relax(1e-4, 300_000, check_every=100)
        except sl.SllgError:
            pass                                        # still moving: read the state reached
        return g.get_spins()[:, 2].mean() < 0

    hc = {}
    for demag in (False, True):
        g = sl.from_workload(system(demag), precision=precision)
        lo, hi = 0.5, 2.5
        while hi - lo > 0.01:
            mid = 0.5 * (lo + hi)
            sw = switches(g, mid)
            log(f"  ellipsoid {'with' if demag else 'without'} demag: h = {mid:.4f} T "
                f"{'switches' if sw else 'holds'}")
            if sw:
                hi = mid
            else:
                lo = mid
        g.close()
        hc["with" if demag else "without"] = 0.5 * (lo + hi)
    Nz_o = (2 / np.sqrt(3) * np.log(2 + np.sqrt(3)) - 1) / 3
    out["ellipsoid"] = {
        "atoms": int(lat.n), "steps_per_s_without": rates["without"], "steps_per_s_with_demag": rates["with"],
        "switching_field_T_without": hc["without"], "switching_field_T_with": hc["with"],
        "rise_T": hc["with"] - hc["without"],
        "osborn_rise_T": ((1 - Nz_o) / 2 - Nz_o) * MU0 * M, "paper_rise_T": 0.33, "paper_expected_T": 0.37,
    }
    return out


def sweep_main(args):
    import paper_1310_6143_amd as sl

    kind = args.workload
    if kind == "demag":
        r32 = run_demag(sl.FP32, args)
        out = {
            "metric": "demagnetising-field pair terms/s (all-pairs macrocell update)",
            "value": r32["update"]["pair_terms_per_s"], "unit": "pair-terms/s", "n_gpus": 1, "steps": 5,
            "warmup": 1, "ms_per_step": r32["update"]["seconds"] * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "65,536 macrocells (sc slab 128x128x32 atoms, 2-atom cells); prolate "
                                   "fcc ellipsoid 10 x 20 nm with macrocells of 2 unit cells"},
            "roofline": {"bound": "alu", "achieved": r32["update"]["achieved_TFLOPs"], "peak": 157.3,
                         "unit": "TFLOP/s", "frac": r32["update"]["achieved_TFLOPs"] / 157.3, "traffic": None},
            "fp32": r32,
        }
        if not args.no_fp64:
            out["fp64"] = run_demag(sl.FP64, args)
        print(json.dumps(out))
        return
    if kind == "sw":
        r32 = run_sw(sl.FP32, args)
        out = {
            "metric": "relaxed (angle, field) points/s (quasi-static Stoner-Wohlfarth loops)",
            "value": r32["angle_field_points_per_s"], "unit": "points/s", "n_gpus": 1,
            "steps": r32["steps"], "warmup": 1, "ms_per_step": r32["seconds"] * 1e3 / max(r32["steps"], 1),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "1024 uncoupled spins, easy axes 0.05..89.95 deg from the field, "
                                   "H = +1.5..-1.5 H_k in 0.01 H_k steps, relaxed to the torque tolerance"},
            "fp32": r32,
        }
        if not args.no_fp64:
            out["fp64"] = run_sw(sl.FP64, args)
        print(json.dumps(out))
        return
    if kind == "mc":
        r32 = run_mc(sl.FP32, args)
        out = {
            "metric": "spin trials/s (Monte Carlo, Hinzke-Nowak moves)", "value": r32["spin_steps_per_s"],
            "unit": "spin-trials/s", "n_gpus": 1, "steps": r32["steps"], "warmup": 10,
            "ms_per_step": r32["seconds"] * 1e3 / r32["steps"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"Monte Carlo M(T), sc 28^3 (21,952 spins), 50..1000 K in 50 K steps, "
                                   f"{args.mc_steps} + {args.mc_steps} steps per point"},
            "fp32": r32,
        }
        if not args.no_fp64:
            out["fp64"] = run_mc(sl.FP64, args)
        print(json.dumps(out))
        return
    r32 = run_sweep(kind, sl.FP32, args)
    out = {
        "metric": METRIC, "value": r32["spin_steps_per_s"], "unit": "spin-steps/s", "n_gpus": 1,
        "steps": r32["steps"], "warmup": 10, "ms_per_step": r32["seconds"] * 1e3 / r32["steps"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("M(T) ramp, bcc 64x64x16 film (131,072 spins), 0..1500 K in 50 K steps, "
                                "5000 + 5000 steps per point, lambda = 1" if kind == "film" else
                                "hysteresis sweep, fcc sphere R = 8 nm (196,053 spins), H_z = -5..5 T in "
                                "0.1 T steps, 2000 steps per point, T = 10 K")},
        "fp32": r32,
    }
    if not args.no_fp64:
        r64 = run_sweep(kind, sl.FP64, args)
        out["fp64"] = r64
        dm = [abs(a["m_abs"] - b["m_abs"]) for a, b in zip(r32["points"], r64["points"])]
        se = [np.hypot(a["m_abs_se"], b["m_abs_se"]) for a, b in zip(r32["points"], r64["points"])]
        out["fp32_vs_fp64"] = {"max_abs_dM_over_Ms": float(max(dm)),
                               "max_dM_in_combined_se": float(max(d / s if s > 0 else 0.0 for d, s in zip(dm, se)))}
    print(json.dumps(out))


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(w, n_steps):
    """The FP64 oracle on one host thread: a bounded sample of the benchmark
    block (n_steps steps of every spin, records every step), and the whole
    4096-spin simple-cubic reference run (1000 steps at 300 K)."""
    import oracle
    from spin_systems import sc_reference

    sysm = oracle.System(w)
    S = np.ascontiguousarray(w.S0.copy())
    t0 = time.perf_counter()
    sysm.integrate(S, 0, n_steps, record=True)
    dt = time.perf_counter() - t0
    ref = sc_reference(L=16, temperature=300.0, n_steps=1000, seed=42)
    S_ref = np.ascontiguousarray(ref.S0.copy())
    t1 = time.perf_counter()
    oracle.System(ref).integrate(S_ref, 0, 1000, record=True)
    dt_ref = time.perf_counter() - t1
    model = cpu_model()
    return {
        "value": w.n * n_steps / dt,
        "unit": "spin-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n_steps} Heun steps (with per-step m and E) of the full {w.n}-spin block, "
                  f"FP64 oracle on one thread of {model} ({os.cpu_count()} host threads)",
        "seconds": dt,
        "cpu_model": model,
        "sc4096_1000_steps": {"seconds": dt_ref, "spin_steps_per_s": ref.n * 1000 / dt_ref,
                              "run": "simple-cubic 16^3 = 4096 spins, T = 300 K, seed 42, 1000 Heun steps "
                                     "with per-step m and E, the whole run"},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cells", type=int, default=160)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--only-fp64", action="store_true", help="time only the FP64 run (profiling)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-budget", type=int, default=16384, help="MiB")
    ap.add_argument("--serving-chunk", type=int, default=64)
    ap.add_argument("--workload", default="block",
                    choices=["block", "dmi", "lr", "film", "sphere", "mc", "sw", "demag"],
                    help="block: 8.19M-spin bcc step throughput (default); dmi: the same block with "
                         "exchange tensors and cubic anisotropy; lr: long-range exchange (388 partners); "
                         "film: full M(T) ramp; "
                         "sphere: full hysteresis sweep; mc: Monte Carlo M(T) of the sc test system "
                         "and the Monte Carlo step rate of the block; sw: quasi-static "
                         "Stoner-Wohlfarth loops at 1024 angles; demag: macrocell demagnetising field")
    ap.add_argument("--mc-steps", type=int, default=5000, help="equilibration (= averaging) steps per "
                    "temperature for --workload mc")
    ap.add_argument("--sweep-points", type=int, default=0, help="limit the sweep to its first points")
    ap.add_argument("--demag-update-only", action="store_true",
                    help="demag workload: time the field update only (skip the ellipsoid)")
    ap.add_argument("--launch", default="", help="fixed launch shape 'xcd_remap,grid_scale_pct[,tile_order]' "
                    "instead of the library default")
    ap.add_argument("--no-autotune", action="store_true", help="run the library's default launch shape "
                    "instead of timing the candidate shapes first (sllg_autotune) and running the fastest")
    ap.add_argument("--no-fused", action="store_true", help="run the two-launch step even where the "
                    "lattice allows the fused one")
    ap.add_argument("--fused-shape", default="", help="fused work-item shape 'tile_x,tile_y,planes,threads' "
                    "instead of the library's choice")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run a plain device copy of this many MiB (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU path of this library is a design "
              "only (independent requests shard by rank; one large system needs a halo exchange "
              "that is not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy << 18          # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 5
        print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 6, "ms_per_copy": ms,
                          "read_plus_write_GBs": 2 * n * 4 / (ms / 1e3) / 1e9}))
        return

    if args.workload not in ("block", "dmi", "lr"):
        sweep_main(args)
        return

    from spin_systems import bcc_block, long_range_sc, with_tensor_exchange

    t0 = time.time()
    dmi = args.workload == "dmi"
    lr = args.workload == "lr"
    if lr:    # long-range exchange: 388 partners per site, 16 radial types
        w = long_range_sc(L=64, r_cut=4.5)
        args.no_serving = True
    else:
        w = bcc_block(cells=args.cells)
    if dmi:   # the general kernel variant: 14 directed exchange tensors and cubic anisotropy
        w = with_tensor_exchange(w, D=(1.2e-21, 0.5e-21), dmi="bulk", k_c=4e-24)
        args.no_serving = True
    deg = w.lattice.nnz / w.n
    log(f"workload: {w.n} spins, {w.lattice.nnz} neighbour entries, built in {time.time() - t0:.1f} s")

    import paper_1310_6143_amd as sl

    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    fshape = tuple(int(v) for v in args.fused_shape.split(",")) if args.fused_shape else None
    fused = 0 if args.no_fused else 1
    if args.only_fp64:
        r64 = run_gpu(w, sl.FP64, args.steps, args.warmup, torch, launch, not args.no_autotune, fused, fshape)
        print(json.dumps({"fp64_ms_per_step": r64["ms"] / args.steps}))
        return
    r32 = run_gpu(w, sl.FP32, args.steps, args.warmup, torch, launch, not args.no_autotune, fused, fshape)
    r64 = None if args.no_fp64 else run_gpu(w, sl.FP64, args.steps, args.warmup, torch, launch, not args.no_autotune,
                                            fused, fshape)

    n = w.n
    ms_step = r32["ms"] / args.steps
    value = n * args.steps / (r32["ms"] / 1e3)
    b_alg = algorithmic_bytes_per_spin_step(4, deg)
    achieved = b_alg * n / (ms_step / 1e3) / 1e9
    fused_on = bool(r32["launch"].get("fused"))
    kind = "fused" if fused_on else "two_launch"
    shape = r32["launch"].get("fused_shape") if fused_on else None
    traffic = None if (dmi or lr) else profile_value(kind, "fp32_hbm_bytes_per_step", shape)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"periodic sc 64^3 ({n} spins), every pair within 4.5 lattice constants linked "
                         "(388 partners, 16 radial types, J = 6e-21 J exp(-(r - 1))), T=300 K, alpha=0.1, "
                         "dt=1e-16 s; FP32 spins, FP64 m/E reductions every step") if lr else
                        (f"periodic bcc {args.cells}^3 cells, J1+J2 14-entry CSR, {n} spins, T=300 K, "
                         "alpha=0.05, dt=1e-16 s, seed 4; FP32 spins, FP64 m/E reductions every step"
                         + ("; exchange tensors per bond direction (14 types: J plus bulk "
                            "Dzyaloshinskii-Moriya D1 = 1.2e-21 J, D2 = 0.5e-21 J) and cubic "
                            "anisotropy k_c = 4e-24 J" if dmi else "")),
            "n_spins": n,
            "neighbour_entries": int(w.lattice.nnz),
            "launch_shape": r32["launch"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic * n,
            "kernel": ("fused Heun step k_fused (one launch per step)" if fused_on else
                       "Heun step (predictor + corrector launches)"),
            "algorithmic_bytes_per_spin_step": b_alg,
            "traffic_GBs": None if traffic is None else traffic * n / (ms_step / 1e3) / 1e9,
            "traffic_frac": None if traffic is None else traffic * n / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
            "valu_busy": None if (dmi or lr) else (
                {"k_fused": profile_value("fused", "fp32_fused_valu_busy", shape)} if fused_on else
                {"predictor": profile_value("two_launch", "fp32_predictor_valu_busy"),
                 "corrector": profile_value("two_launch", "fp32_corrector_valu_busy")}),
        },
    }
    if lr:
        # 388 links x 3 FMAs x 2 passes = 12 z flops per spin-step of exchange arithmetic alone
        flops = 12.0 * deg * n / (ms_step / 1e3)
        out["roofline"] = {"bound": "alu", "achieved": flops / 1e12, "peak": 157.3, "unit": "TFLOP/s",
                           "frac": flops / 1e12 / 157.3, "traffic": None,
                           "kernel": "Heun step (predictor + corrector launches)",
                           "flops_per_spin_step": 12.0 * deg,
                           "hbm_view_GBs_at_B_alg": achieved}
    if r64 is not None:
        ms64 = r64["ms"] / args.steps
        b64 = algorithmic_bytes_per_spin_step(8, deg)
        fused64 = bool(r64["launch"].get("fused"))
        shape64 = r64["launch"].get("fused_shape") if fused64 else None
        traffic64 = None if (dmi or lr or not fused64) else profile_value("fused", "fp64_hbm_bytes_per_step", shape64)
        out["fp64"] = {
            "value": n * args.steps / (r64["ms"] / 1e3),
            "ms_per_step": ms64,
            "roofline_achieved_GBs": b64 * n / (ms64 / 1e3) / 1e9,
            "roofline_frac": b64 * n / (ms64 / 1e3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_spin_step": b64,
            "kernel": ("fused Heun step k_fused<double> (one launch per step)" if fused64 else
                       "Heun step (predictor + corrector launches)"),
            "launch_shape": r64["launch"],
            "traffic": None if traffic64 is None else traffic64 * n,
        }
        dm = np.abs(r32["m"] - r64["m"]).max()
        dE = (np.abs(r32["E"] - r64["E"]) / np.abs(r64["E"])).max()
        out["fp32_vs_fp64"] = {"max_abs_dm": float(dm), "max_rel_dE": float(dE),
                               "steps_compared": args.steps}
    if not args.no_serving:
        out["serving"] = run_serving(args)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: {args.cpu_steps} oracle steps on {n} spins")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
