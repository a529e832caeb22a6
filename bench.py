"""Benchmark of the ESP long-range pipeline on one MI355X.

Workload: water-like boxes of 3000 rigid three-site molecules (9,000 atoms,
O -0.8476 / H +0.4238), cubic L = 31.0, grid 32^3, P = 6, tolerance 1e-4, with
seeded uniform centres and random orientations. A step evaluates potentials,
forces and energies of a batch of B such boxes (B = 128 by default) with the
FP32 batched plan, replayed as one HIP graph; inputs are resident in HBM.
The FP64 plain single-system path on one box is timed beside it, the pipeline
phases are timed with HIP events on the plan's stream, and the CPU reference
five-step method is timed on one box for the CPU baseline.

Prints ONE JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_VALU_TFLOPS = 78.6   # non-packed FP32 FMA: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
PEAK_FP64_VALU_TFLOPS = 78.6


def _rel_rms(a, b):
    """sqrt(sum |a - b|^2 / sum |b|^2): agreement of two runs of the library."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def algorithmic_cost(phase, N, n, P, deg, prec):
    """Algorithmic HBM bytes and flops of one launch of a phase for one system
    of N particles on an n^3 grid (formulas in the design notes)."""
    rb = 8 if prec == 64 else 4
    g = n ** 3                       # grid points
    spec = n * n * (n // 2 + 1)      # half-spectrum modes
    if phase == "spread":
        b = N * 4 * rb + g * rb                     # sorted (u, q) in, grid out
        f = N * (2 * 3 * P * deg + P + P * P + P ** 3)       # Horner FMAs + weight products
    elif phase == "gather":
        b = N * (4 * rb + 4 + 4 * rb) + g * rb      # sorted in, perm, phi+F out, grid in
        f = N * (2 * 3 * P * 2 * deg + 2 * (2 * P ** 3 + 3 * P * P + 4 * P))
    elif phase in ("fft_zy", "fft_yz"):
        b = g * rb + spec * 2 * rb
        f = 2.5 * spec * 2 * math.log2(n * n)      # ~5 N log2 N per complex transform pair
    elif phase == "fft_x_scale":
        b = 2 * spec * 2 * rb
        f = 2 * 5 * spec * math.log2(n) + 8 * spec
    elif phase == "bin":
        b = N * (4 * rb + 4)
        f = N * 10
    elif phase == "scatter":
        b = N * (4 * rb + 4 + 4 * rb + 4)
        f = N * 10
    elif phase == "zero":
        b = n * n * (n + 2) * rb
        f = 0
    else:
        b, f = 0, 0
    return b, f


# LDS: 128 bytes per clock per CU (32 banks x 4 B) -> 16 lanes of 64-bit atomics
# or 32 lanes of 32-bit reads per clock per CU, over 256 CUs at 2.4 GHz.
PEAK_LDS_U64_ATOMICS_GOPS = 16 * 256 * 2.4
PEAK_LDS_F32_READS_GOPS = 32 * 256 * 2.4

PHASE_KERNEL = {"hist": "k_hist<float>", "scan": "k_scan", "scatter": "k_scatter<float>",
                "spread": "k_spread<float, {P}>", "fft_zy": "k_fwd_zy<float, {n}>",
                "fft_x_scale": "k_fft_x<float, {n}>", "fft_yz": "k_inv_yz<float, {n}>",
                "gather": "k_gather<float, {P}>", "finalize": "k_finalize"}


def measured_traffic(phase, n, P):
    """HBM bytes per dispatch of the phase's main kernel from the committed
    rocprofv3 counter summary, or None when the kernel sources changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "esp_fp32_water9k_b128_hbm_traffic.md")
    try:
        txt = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", txt, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    for f, h in rec["source_sha256_16"].items():
        src = os.path.join(ROOT, "paper_2505_09727_amd", "csrc", f)
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != h:
            return None
    return rec["hbm_bytes_per_dispatch"].get(PHASE_KERNEL.get(phase, "").format(n=n, P=P))


def roofline(phase, ms, B, N, n, P, deg):
    """Roofline record of one phase launch over the batch (algorithmic bytes
    and flops from algorithmic_cost, measured launch time ms)."""
    b1, f1 = algorithmic_cost(phase, N, n, P, deg, 32)
    bytes_launch, flops_launch = B * b1, B * f1
    t = ms / 1e3
    gbs, tfl = bytes_launch / t / 1e9, flops_launch / t / 1e12
    if flops_launch / (PEAK_FP32_VALU_TFLOPS * 1e12) > bytes_launch / (PEAK_HBM_GBS * 1e9):
        r = dict(kernel=phase, bound="alu", achieved=tfl, peak=PEAK_FP32_VALU_TFLOPS, unit="TFLOP/s",
                 frac=tfl / PEAK_FP32_VALU_TFLOPS, hbm_achieved_GBs=gbs, hbm_frac=gbs / PEAK_HBM_GBS)
    else:
        r = dict(kernel=phase, bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s",
                 frac=gbs / PEAK_HBM_GBS, alu_achieved_TFLOPs=tfl)
    tr = measured_traffic(phase, n, P)
    r["traffic"] = tr
    r["avg_launch_ms"] = ms
    r["algorithmic_bytes_per_launch"] = bytes_launch
    r["algorithmic_flops_per_launch"] = flops_launch
    if phase == "spread":
        ops = B * N * P ** 3 / t / 1e9
        r["lds_u64_atomics"] = dict(achieved_Gops=ops, peak_Gops=PEAK_LDS_U64_ATOMICS_GOPS,
                                    frac=ops / PEAK_LDS_U64_ATOMICS_GOPS)
    if phase == "gather":
        ops = B * N * P ** 3 / t / 1e9
        r["lds_f32_reads"] = dict(achieved_Gops=ops, peak_Gops=PEAK_LDS_F32_READS_GOPS,
                                  frac=ops / PEAK_LDS_F32_READS_GOPS)
    return r


def _one_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _oracle_box(args):
    """One evaluation of the reference five-step on one box (a pool job)."""
    from oracle.fivestep import five_step
    pos, q, L, nf, P, c, rc, c1 = args
    five_step(pos, q, L, nf, P, c, rc, c1)
    return len(q)


def _host():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpus_available": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(boxes, L, prm, budget_s=12.0, max_workers=16):
    """The reference five-step (FP64, exact window, matrix DFT) on the host's
    cores: independent boxes of the batch, one per worker process (one thread
    each), in rounds until about budget_s seconds have passed."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    host = _host()
    workers = max(1, min(max_workers, host["cpus_available"]))
    jobs = [(b[0], b[1], L, prm.nf, prm.P, prm.c, prm.rc, prm.c1) for b in boxes]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_one_thread) as ex:
        list(ex.map(_oracle_box, jobs[:workers]))  # imports and first-touch outside the timed window
        t0 = time.perf_counter()
        done, k = 0, 0
        while True:
            batch = [jobs[(k + i) % len(jobs)] for i in range(workers)]
            k += workers
            done += sum(ex.map(_oracle_box, batch))
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    return dict(value=done / el, unit="particle-steps/s", cores=workers, kind="oracle",
                sample=f"{done // len(boxes[0][1])} evaluations of 9000-atom boxes of the batch by the FP64 "
                       f"reference five-step (exact window, matrix DFT), {workers} worker processes of one "
                       f"thread each, {el:.1f} s",
                host=host)


def serving_run(seconds, rate, budget_gb, seed=5):
    """Poisson request stream through the continuous-batching server."""
    import threading
    import workloads as W
    from paper_2505_09727_amd.esp import Server, esp_warm_tables
    reqs = W.request_stream(duration_s=seconds, rate_hz=rate, seed=seed)
    systems = []
    for r in reqs:
        pos, q, L = r.system()
        systems.append((pos.astype(np.float32), q.astype(np.float32), L))
    # deployment step, outside the timed stream: parameter classes of every
    # grid size at the stream's tolerances
    tw = time.perf_counter()
    esp_warm_tables(sorted({r.tol for r in reqs}), 144)
    warm_s = time.perf_counter() - tw
    srv = Server(hbm_budget_bytes=int(budget_gb * (1 << 30)))
    t0 = time.perf_counter()
    late = [0.0]

    def feed():
        for r, (pos, q, L) in zip(reqs, systems):
            dt = r.t_arrival - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            else:
                late[0] = max(late[0], -dt)
            srv.submit(pos, q, L, r.tol, nsteps=r.steps, drift=0.01, seed=r.seed, tag=r.rid)

    th = threading.Thread(target=feed)
    th.start()
    th.join()
    srv.wait(600)
    wall = time.perf_counter() - t0
    res = srv.poll(len(reqs) + 16)
    st = srv.stats()
    srv.close()
    offered = sum(r.n_atoms * r.steps for r in reqs) / seconds
    return {
        "workload": f"Poisson arrivals at {rate:.0f}/s for {seconds} s ({len(reqs)} requests), N log-uniform "
                    f"1000-200000 (water 1 g/cm^3 or +-1 melt), tol in {{1e-3,1e-4,1e-5}}, 10 steps each with "
                    f"0.01 drift, FP32, HBM budget {budget_gb} GiB",
        "requests": len(reqs), "completed": st["completed"], "failed": st["failed"],
        "particle_steps_per_s": st["particle_steps"] / st["span_s"] if st["span_s"] > 0 else None,
        "offered_particle_steps_per_s": offered,
        "p50_latency_ms": st["p50_latency_s"] * 1e3, "p99_latency_ms": st["p99_latency_s"] * 1e3,
        "max_latency_ms": st["max_latency_s"] * 1e3, "scheduler_iterations": st["iterations"],
        "peak_hbm_bytes": st["bytes_peak"], "submit_lag_max_ms": late[0] * 1e3, "wall_s": wall,
        "scheduler_s": {"build": st["build_s"], "admit": st["admit_s"], "step": st["step_s"],
                        "busy": st["busy_s"]},
        "statuses_ok": sum(1 for r in res if r["status"] == 0),
        "table_warmup_s": warm_s,
    }


def _time_plan(plan, ext, pos, q, phi, F, steps):
    """Mean ms per step of `steps` enqueued steps on the plan's stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ext)
    for _ in range(steps):
        plan.longrange_async(pos, q, phi, F)
    e1.record(ext)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def ik_run(pos, q, L, B, N, steps, F_ad):
    """The same batch with forces by spectral derivatives (ik): cost beside
    the AD route, force difference and net force."""
    import torch
    from paper_2505_09727_amd.esp import Plan
    dev = torch.device("cuda:0")
    plan = Plan([L] * B, [N] * B, 1e-4, force_method=1)
    phi = torch.empty(B * N, dtype=torch.float32, device=dev)
    F = torch.empty((B * N, 3), dtype=torch.float32, device=dev)
    ext = torch.cuda.ExternalStream(plan.stream)
    plan.set_graph(True)
    for _ in range(3):
        plan.longrange_async(pos, q, phi, F)
    ms = _time_plan(plan, ext, pos, q, phi, F, steps)
    plan.longrange(pos, q, phi, F)
    Fik = F.cpu().double().numpy()
    plan.close()
    F0 = Fik[:N]
    net = np.abs(F0.sum(axis=0)).max() / (N * np.sqrt(np.mean(F0 ** 2)))
    net_ad = np.abs(F_ad[:N].sum(axis=0)).max() / (N * np.sqrt(np.mean(F_ad[:N] ** 2)))
    return {"particle_steps_per_s": B * N / (ms / 1e3), "ms_per_step": ms,
            "rel_rms_F_ik_vs_ad": _rel_rms(Fik, F_ad),
            "net_force_rel": {"ik": float(net), "ad": float(net_ad)}}


def _pairs_within(pos, L, rc, chunk=512):
    """Ordered pairs (i, j), j != i, closer than rc over nearest images."""
    n, cnt = len(pos), 0
    for s in range(0, n, chunk):
        d = pos[s:s + chunk, None, :] - pos[None, :, :]
        d -= L * np.round(d / L)
        r2 = np.einsum("abk,abk->ab", d, d)
        cnt += int(np.count_nonzero(r2 < rc * rc)) - min(chunk, n - s)
    return cnt


def local_run(pos, q, L, B, N, steps, box0, reps):
    """The same batch with the local part of the split on the device (full
    Coulomb phi, F, E): cost beside the long-range step, and the local phase's
    time and ALU roofline."""
    import ctypes as C
    import torch
    from paper_2505_09727_amd.esp import Plan, esp_local_coeffs, lib
    dev = torch.device("cuda:0")
    plan = Plan([L] * B, [N] * B, 1e-4, local=1)
    phi = torch.empty(B * N, dtype=torch.float32, device=dev)
    F = torch.empty((B * N, 3), dtype=torch.float32, device=dev)
    ext = torch.cuda.ExternalStream(plan.stream)
    plan.set_graph(True)
    for _ in range(3):
        plan.longrange_async(pos, q, phi, F)
    ms = _time_plan(plan, ext, pos, q, phi, F, steps)
    nph = lib().esp_num_phases()
    msp = (C.c_double * nph)()
    st = lib().esp_plan_profile(plan._h, C.c_void_p(pos.data_ptr()), C.c_void_p(q.data_ptr()),
                                C.c_void_p(phi.data_ptr()), C.c_void_p(F.data_ptr()), reps, msp)
    assert st == 0, lib().esp_last_error()
    phases = {lib().esp_phase_name(i).decode(): msp[i] for i in range(nph)}
    p = plan.params[0]
    plan.close()
    pos0 = box0[0].astype(np.float32).astype(np.float64)
    pairs = _pairs_within(pos0, L, p.rc)
    deg = esp_local_coeffs(p)[0].shape[1] - 1
    fpp = 27 + 4 * deg
    flops = B * pairs * fpp
    t = phases["local"] / 1e3
    tfl = flops / t / 1e12
    return {"particle_steps_per_s": B * N / (ms / 1e3), "ms_per_step": ms, "phases_ms": phases,
            "roofline_local": {"kernel": "k_cellsort + k_local", "bound": "alu", "achieved": tfl,
                               "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": tfl / PEAK_FP32_VALU_TFLOPS,
                               "traffic": None, "avg_launch_ms": phases["local"],
                               "algorithmic_flops_per_launch": flops, "pairs_per_particle": pairs / N,
                               "flops_per_pair": fpp, "rc": p.rc},
            "what": "full Coulomb (long-range + local part within rc) on the same batch"}


FFT_SIZES = (8, 12, 16, 18, 24, 32, 36, 48, 54, 64, 72, 96, 108, 128, 144)


# The smallest grid at which the classical method (P = 5, alpha = log(1/tol),
# the ESP cutoff) reaches a full-Coulomb force error of 1e-4 against Ewald on
# the 9000-atom water-like box (L = 31); the device tests check it.
CLASSICAL_GRID_WATER9K = 48


def classical_run(pos, q, L, B, N, steps, ms_esp, ms_esp_full, tol=1e-4):
    """The classical method (Gaussian split, B-spline window of order 5, the
    ESP cutoff) on the same batch at the smallest grid that meets the
    tolerance (eq. cemparameters' grid pushed up for aliasing), beside ESP."""
    import torch
    from paper_2505_09727_amd.esp import Plan, esp_plan_query
    dev = torch.device("cuda:0")
    p0 = esp_plan_query(L, N, tol, method=1)
    p_esp = esp_plan_query(L, N, tol)
    chosen = CLASSICAL_GRID_WATER9K
    out = {"P": p0.P, "alpha": p0.c, "rc": p0.rc, "grid_formula": p0.nf, "grid": chosen, "grid_esp": p_esp.nf,
           "grid_ratio_R": (chosen / p_esp.nf) ** 3}
    for local, key in ((0, "longrange"), (1, "full_coulomb")):
        plan = Plan([L] * B, [N] * B, tol, method=1, nf=chosen, local=local)
        phi = torch.empty(B * N, dtype=torch.float32, device=dev)
        F = torch.empty((B * N, 3), dtype=torch.float32, device=dev)
        ext = torch.cuda.ExternalStream(plan.stream)
        plan.set_graph(True)
        for _ in range(3):
            plan.longrange_async(pos, q, phi, F)
        ms = _time_plan(plan, ext, pos, q, phi, F, steps)
        plan.close()
        ref = ms_esp if local == 0 else ms_esp_full
        out[key] = {"ms_per_step": ms, "particle_steps_per_s": B * N / (ms / 1e3),
                    "esp_ms_per_step": ref, "esp_speedup": (ms / ref) if ref else None}
    return out


def nacl_run(steps=200):
    """The 512-ion rock-salt crystal (a = 5.64 A, 4 x 4 x 4 cells, perturbed by
    U(-0.1, 0.1) A, n = 16, P = 6, tol 1e-4): launch-latency bound, so
    microseconds per step in FP64 and FP32 (autotuned, graph replay), and the exact
    lattice's Madelung constant from the FP64 potentials with the local part."""
    import torch
    import workloads as W
    from paper_2505_09727_amd.esp import Plan
    dev = torch.device("cuda:0")
    cfg = W.NACL
    out = {"workload": "512-ion rock-salt crystal, L = 22.56, n = 16, P = 6, tol 1e-4"}
    pos, q, L = W.nacl_crystal(cells=cfg["cells"], a=cfg["a"], perturb=0.1, seed=1)
    for prec, dt in ((64, torch.float64), (32, torch.float32)):
        plan = Plan(L, len(q), cfg["tol"], nf=cfg["n"], P=cfg["P"], precision=prec)
        tp = torch.tensor(pos, dtype=dt, device=dev)
        tq = torch.tensor(q, dtype=dt, device=dev)
        ph = torch.empty(len(q), dtype=dt, device=dev)
        F = torch.empty((len(q), 3), dtype=dt, device=dev)
        ext = torch.cuda.ExternalStream(plan.stream)
        plan.autotune(tp, tq, ph, F, reps=5)
        plan.set_graph(True)
        for _ in range(5):
            plan.longrange_async(tp, tq, ph, F)
        out[f"fp{prec}_us_per_step"] = 1e3 * _time_plan(plan, ext, tp, tq, ph, F, steps)
        out[f"fp{prec}_fft_passes"] = plan.params[0].fft_passes
        plan.close()
    pos0, q0, _ = W.nacl_crystal(cells=cfg["cells"], a=cfg["a"])
    plan = Plan(L, len(q0), cfg["tol"], nf=cfg["n"], P=cfg["P"], precision=64, local=1)
    tp = torch.tensor(pos0, dtype=torch.float64, device=dev)
    tq = torch.tensor(q0, dtype=torch.float64, device=dev)
    ph = torch.empty(len(q0), dtype=torch.float64, device=dev)
    F = torch.empty((len(q0), 3), dtype=torch.float64, device=dev)
    E = plan.longrange(tp, tq, ph, F)[0]
    plan.close()
    r0 = cfg["a"] / 2
    out["madelung_from_energy"] = -E * 4 * math.pi * r0 / (len(q0) / 2)
    out["madelung_reference"] = 1.747565
    return out


def box_run(steps, B=128, n_mol=3000, tol=1e-4):
    """Orthorhombic boxes: a batch of water-like boxes of the 9000-atom
    workload's volume and density with the membrane system's aspect ratio
    (10.79 : 10.18 : 9.55, Methods, experimental design), timed beside the
    cubic batch, and with the local part."""
    import torch
    import workloads as W
    from paper_2505_09727_amd.esp import Plan
    dev = torch.device("cuda:0")
    ratios = np.array([10.79, 10.18, 9.55])
    box = ratios * (31.0 ** 3 / np.prod(ratios)) ** (1.0 / 3.0)
    boxes = [W.water_box(n_mol, box, seed=2000 + b) for b in range(B)]
    N = 3 * n_mol
    pos = torch.tensor(np.concatenate([b[0] for b in boxes]), dtype=torch.float32, device=dev)
    q = torch.tensor(np.concatenate([b[1] for b in boxes]), dtype=torch.float32, device=dev)
    plan = Plan([box[0]] * B, [N] * B, tol, per_system=[{"Ly": box[1], "Lz": box[2]}] * B)
    p = plan.params[0]
    phi = torch.empty(B * N, dtype=torch.float32, device=dev)
    F = torch.empty((B * N, 3), dtype=torch.float32, device=dev)
    ext = torch.cuda.ExternalStream(plan.stream)
    plan.set_graph(True)
    for _ in range(3):
        plan.longrange_async(pos, q, phi, F)
    ms = _time_plan(plan, ext, pos, q, phi, F, steps)
    plan.close()
    full = Plan([box[0]] * B, [N] * B, tol, per_system=[{"Ly": box[1], "Lz": box[2], "local": 1}] * B)
    ext = torch.cuda.ExternalStream(full.stream)
    full.set_graph(True)
    for _ in range(3):
        full.longrange_async(pos, q, phi, F)
    ms_full = _time_plan(full, ext, pos, q, phi, F, steps)
    full.close()
    return {"box": [float(x) for x in box], "grid": p.nf, "P": p.P, "rc": p.rc,
            "particle_steps_per_s": B * N / (ms / 1e3), "ms_per_step": ms, "full_coulomb_ms_per_step": ms_full,
            "workload": f"batch of {B} orthorhombic water-like boxes, {N} atoms each, FP32, tol {tol}"}


def cell_run(steps, B=128, n_mol=3000, tol=1e-4):
    """Triclinic cells: a batch of water-like rhombic dodecahedra (square xy
    face) of the 9000-atom workload's volume and density, timed beside the
    cubic batch, and with the local part."""
    import torch
    import workloads as W
    from paper_2505_09727_amd.esp import Plan
    dev = torch.device("cuda:0")
    H = W.rhombic_dodecahedron(31.0 ** 3)
    cell = (H[0, 0], H[1, 1], H[2, 2], H[0, 1], H[0, 2], H[1, 2])
    tilt = {"Ly": cell[1], "Lz": cell[2], "xy": cell[3], "xz": cell[4], "yz": cell[5]}
    cells = [W.water_cell(n_mol, H, seed=3000 + b) for b in range(B)]
    N = 3 * n_mol
    pos = torch.tensor(np.concatenate([c[0] for c in cells]), dtype=torch.float32, device=dev)
    q = torch.tensor(np.concatenate([c[1] for c in cells]), dtype=torch.float32, device=dev)
    plan = Plan([cell[0]] * B, [N] * B, tol, per_system=[tilt] * B)
    p = plan.params[0]
    phi = torch.empty(B * N, dtype=torch.float32, device=dev)
    F = torch.empty((B * N, 3), dtype=torch.float32, device=dev)
    ext = torch.cuda.ExternalStream(plan.stream)
    plan.set_graph(True)
    for _ in range(3):
        plan.longrange_async(pos, q, phi, F)
    ms = _time_plan(plan, ext, pos, q, phi, F, steps)
    plan.close()
    full = Plan([cell[0]] * B, [N] * B, tol, per_system=[dict(tilt, local=1)] * B)
    ext = torch.cuda.ExternalStream(full.stream)
    full.set_graph(True)
    for _ in range(3):
        full.longrange_async(pos, q, phi, F)
    ms_full = _time_plan(full, ext, pos, q, phi, F, steps)
    full.close()
    return {"cell": [float(v) for v in cell], "grid": p.nf, "P": p.P, "rc": p.rc,
            "particle_steps_per_s": B * N / (ms / 1e3), "ms_per_step": ms, "full_coulomb_ms_per_step": ms_full,
            "workload": f"batch of {B} rhombic-dodecahedron water-like cells, {N} atoms each, FP32, tol {tol}"}


def ensemble_run(steps, seed=4):
    """256 water-like boxes at 1 g/cm^3 with log-uniform sizes in one FP32 plan
    (autotuned bin edges, graph replay) against the FP64 plain path run one
    system at a time."""
    import torch
    import workloads as W
    from collections import Counter
    from paper_2505_09727_amd.esp import Plan
    dev = torch.device("cuda:0")
    systems = W.ensemble(n_sys=256, seed=seed)
    Ls = [s[2] for s in systems]
    Ns = [len(s[1]) for s in systems]
    off = np.cumsum([0] + Ns)
    Ntot = int(off[-1])
    pos = torch.tensor(np.concatenate([s[0] for s in systems]), dtype=torch.float32, device=dev)
    q = torch.tensor(np.concatenate([s[1] for s in systems]), dtype=torch.float32, device=dev)
    phi = torch.empty(Ntot, dtype=torch.float32, device=dev)
    F = torch.empty((Ntot, 3), dtype=torch.float32, device=dev)
    plan = Plan(Ls, Ns, 1e-4)
    default_tiles = Counter(p.tile for p in plan.params)
    grids = sorted({p.nf for p in plan.params})
    ext = torch.cuda.ExternalStream(plan.stream)
    plan.set_graph(True)
    for _ in range(3):
        plan.longrange_async(pos, q, phi, F)
    ms_default = _time_plan(plan, ext, pos, q, phi, F, steps)
    t0 = time.perf_counter()
    tiles = plan.autotune(pos, q, phi, F, reps=3)
    tune_s = time.perf_counter() - t0
    one_block_fft = sum(1 for p in plan.params if p.fft_passes == 1)
    for _ in range(3):
        plan.longrange_async(pos, q, phi, F)
    ms = _time_plan(plan, ext, pos, q, phi, F, steps)
    plan.longrange(pos, q, phi, F)
    F32 = F.cpu().double().numpy()
    plan.close()
    # FP64 plain, one single-system plan after another
    ms64, errs = 0.0, []
    for s, (ps, qs, L) in enumerate(systems):
        p64 = Plan(L, len(qs), 1e-4, precision=64)
        tp = torch.tensor(ps, dtype=torch.float64, device=dev)
        tq = torch.tensor(qs, dtype=torch.float64, device=dev)
        ph = torch.empty(len(qs), dtype=torch.float64, device=dev)
        Fs = torch.empty((len(qs), 3), dtype=torch.float64, device=dev)
        e64 = torch.cuda.ExternalStream(p64.stream)
        p64.longrange_async(tp, tq, ph, Fs)
        ms64 += _time_plan(p64, e64, tp, tq, ph, Fs, 3)
        errs.append(_rel_rms(F32[off[s]:off[s + 1]], Fs.cpu().numpy()))
        p64.close()
    return {
        "workload": f"256 water-like boxes at 1 g/cm^3, atoms log-uniform in [500, 20000] (total {Ntot}), "
                    f"grids {grids[0]}^3..{grids[-1]}^3, tol 1e-4, FP32 batched plan, HIP graph replay",
        "particle_steps_per_s": Ntot / (ms / 1e3), "ms_per_step": ms,
        "ms_per_step_default_tiles": ms_default, "autotune_s": tune_s,
        "tiles_default": dict(default_tiles), "tiles_autotuned": dict(Counter(tiles)),
        "systems_on_one_block_fft": one_block_fft,
        "fp64_plain": {"particle_steps_per_s": Ntot / (ms64 / 1e3), "ms_per_sweep": ms64,
                       "what": "256 single-system FP64 plans run one after another"},
        "speedup_vs_fp64_plain": ms64 / ms,
        "rel_rms_F_fp32_vs_fp64": {"median": float(np.median(errs)), "max": float(np.max(errs))},
    }


def large_run(steps, serve_steps=100):
    """300,000-atom water-like box (L = 100, tol 1e-5): FP32 plan vs FP64 plain
    on the same positions, and 100 served steps with 0.01 drift (device
    resident, one request)."""
    import torch
    import workloads as W
    from paper_2505_09727_amd.esp import Plan, Server
    dev = torch.device("cuda:0")
    cfg = W.WATER_300K
    pos, q = W.water_box(cfg["n_mol"], cfg["L"], seed=cfg["seed"])
    L, N, tol = cfg["L"], len(q), cfg["tol"]
    out = {"workload": f"{N} atoms (water-like), L={L}, tol {tol}"}
    res = {}
    for prec, dt in ((32, torch.float32), (64, torch.float64)):
        plan = Plan(L, N, tol, precision=prec)
        tp = torch.tensor(pos, dtype=dt, device=dev)
        tq = torch.tensor(q, dtype=dt, device=dev)
        ph = torch.empty(N, dtype=dt, device=dev)
        Fs = torch.empty((N, 3), dtype=dt, device=dev)
        ext = torch.cuda.ExternalStream(plan.stream)
        if prec == 32:
            plan.set_graph(True)
        for _ in range(3):
            plan.longrange_async(tp, tq, ph, Fs)
        ms = _time_plan(plan, ext, tp, tq, ph, Fs, steps)
        E = plan.longrange(tp, tq, ph, Fs)
        p = plan.params[0]
        res[prec] = dict(ms=ms, F=Fs.cpu().double().numpy(), E=float(E[0]))
        out[f"fp{prec}"] = {"particle_steps_per_s": N / (ms / 1e3), "ms_per_step": ms,
                            "grid": p.nf, "P": p.P, "tile": p.tile}
        plan.close()
    # the same box with the local part (full Coulomb), FP32
    plan = Plan(L, N, tol, local=1)
    tp = torch.tensor(pos, dtype=torch.float32, device=dev)
    tq = torch.tensor(q, dtype=torch.float32, device=dev)
    ph = torch.empty(N, dtype=torch.float32, device=dev)
    Fs = torch.empty((N, 3), dtype=torch.float32, device=dev)
    ext = torch.cuda.ExternalStream(plan.stream)
    plan.set_graph(True)
    for _ in range(3):
        plan.longrange_async(tp, tq, ph, Fs)
    msl = _time_plan(plan, ext, tp, tq, ph, Fs, steps)
    plan.close()
    out["fp32_full_coulomb"] = {"particle_steps_per_s": N / (msl / 1e3), "ms_per_step": msl}
    out["speedup_fp32_vs_fp64_plain"] = res[64]["ms"] / res[32]["ms"]
    out["rel_rms_F_fp32_vs_fp64"] = _rel_rms(res[32]["F"], res[64]["F"])
    out["rel_E_fp32_vs_fp64"] = abs(res[32]["E"] - res[64]["E"]) / abs(res[64]["E"])
    srv = Server()
    t0 = time.perf_counter()
    srv.submit(pos.astype(np.float32), q.astype(np.float32), L, tol, nsteps=serve_steps, drift=0.01, seed=3)
    srv.wait(300)
    wall = time.perf_counter() - t0
    r = srv.poll()
    srv.close()
    out["served_drift"] = {"steps": serve_steps, "wall_s": wall, "particle_steps_per_s": N * serve_steps / wall,
                           "E_first": r[0]["E_first"] if r else None, "E_last": r[0]["E_last"] if r else None,
                           "what": "one request, positions resident, seeded 0.01 drift per step, "
                                   "wall time incl. upload and planning"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-reps", type=int, default=20)
    ap.add_argument("--serve-seconds", type=float, default=0.5, help="length of the served arrival stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 256-system ensemble section")
    ap.add_argument("--no-ik", action="store_true", help="skip the ik-forces section")
    ap.add_argument("--no-large", action="store_true", help="skip the 300,000-atom section")
    ap.add_argument("--no-local", action="store_true", help="skip the full-Coulomb (local part) section")
    ap.add_argument("--no-classical", action="store_true", help="skip the classical-method (PME) comparison")
    ap.add_argument("--no-box", action="store_true", help="skip the orthorhombic-box section")
    ap.add_argument("--no-nacl", action="store_true", help="skip the 512-ion crystal section")
    ap.add_argument("--no-cell", action="store_true", help="skip the triclinic-cell section")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB 10 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_mib > 0:
        import torch
        x = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda:0").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": x.numel() * 4, "copy_bytes_written_per_launch": y.numel() * 4,
                          "launches": 10}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; sharding across GPUs is designed but not "
                                   "implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2505_09727_amd.esp import Plan, lib
    import ctypes as C

    dev = torch.device("cuda:0")
    B, L, n_mol, tol = args.batch, 31.0, 3000, 1e-4
    boxes = [W.water_box(n_mol, L, seed=1000 + b) for b in range(B)]
    N = 3 * n_mol
    pos = torch.tensor(np.concatenate([b[0] for b in boxes]), dtype=torch.float32, device=dev).contiguous()
    q = torch.tensor(np.concatenate([b[1] for b in boxes]), dtype=torch.float32, device=dev)
    phi = torch.empty(B * N, dtype=torch.float32, device=dev)
    F = torch.empty((B * N, 3), dtype=torch.float32, device=dev)
    E_dev = torch.empty(B, dtype=torch.float64, device=dev)

    plan = Plan([L] * B, [N] * B, tol)
    prm = plan.params[0]
    if not args.no_graph:
        plan.set_graph(True)
    ext = torch.cuda.ExternalStream(plan.stream)
    for _ in range(args.warmup):
        plan.longrange_async(pos, q, phi, F, E_dev)
    plan.sync()
    torch.cuda.synchronize()
    # timed region: K steps on the plan's stream, bracketed by events
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    evs[0].record(ext)
    for k in range(args.steps):
        plan.longrange_async(pos, q, phi, F, E_dev)
        evs[k + 1].record(ext)
    evs[-1].synchronize()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps
    value = B * N * args.steps / (total_ms / 1e3)
    plan.longrange(pos, q, phi, F)  # one synchronous call: its forces feed the comparisons below

    F_all = F.double().cpu().numpy()
    F0 = F_all[:N]

    # per-phase timing (HIP events between phases on the plan's stream)
    nph = lib().esp_num_phases()
    ms = (C.c_double * nph)()
    st = lib().esp_plan_profile(plan._h, C.c_void_p(pos.data_ptr()), C.c_void_p(q.data_ptr()),
                                C.c_void_p(phi.data_ptr()), C.c_void_p(F.data_ptr()), args.profile_reps, ms)
    assert st == 0, lib().esp_last_error()
    phases = {lib().esp_phase_name(i).decode(): ms[i] for i in range(nph)}
    dom = max(phases, key=phases.get)
    roof = roofline(dom, phases[dom], B, N, prm.nf, prm.P, prm.degree)
    kernels = {ph: roofline(ph, phases[ph], B, N, prm.nf, prm.P, prm.degree)
               for ph in ("spread", "gather", "fft_zy", "fft_x_scale", "fft_yz")}
    plan.close()

    # FP64 plain single-system path on one box (same workload shape)
    p64 = Plan(L, N, tol, precision=64)
    pos64 = pos[:N].double().contiguous()
    q64 = q[:N].double().contiguous()
    phi64 = torch.empty(N, dtype=torch.float64, device=dev)
    F64 = torch.empty((N, 3), dtype=torch.float64, device=dev)
    ext64 = torch.cuda.ExternalStream(p64.stream)
    for _ in range(5):
        p64.longrange_async(pos64, q64, phi64, F64)
    p64.sync()
    k64 = max(10, args.steps // 4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ext64)
    for _ in range(k64):
        p64.longrange_async(pos64, q64, phi64, F64)
    e1.record(ext64)
    e1.synchronize()
    ms64 = e0.elapsed_time(e1) / k64
    fp64 = dict(value=N / (ms64 / 1e3), unit="particle-steps/s", ms_per_step=ms64,
                rel_rms_F_fp32_vs_fp64=_rel_rms(F0, F64.cpu().numpy()))
    p64.close()

    cpu = None if args.no_cpu_baseline else cpu_baseline(boxes, L, prm)
    serving = serving_run(args.serve_seconds, args.serve_rate, args.serve_budget_gb) if args.serve_seconds > 0 else None
    ik = None if args.no_ik else ik_run(pos, q, L, B, N, max(10, args.steps // 4), F_all)
    full = None if args.no_local else local_run(pos, q, L, B, N, max(10, args.steps // 4), boxes[0],
                                                   args.profile_reps)
    classical = None
    if not args.no_classical:
        classical = classical_run(pos, q, L, B, N, max(10, args.steps // 4), ms_per_step,
                                  full["ms_per_step"] if full else None)
    ortho = None if args.no_box else box_run(max(10, args.steps // 4))
    tric = None if args.no_cell else cell_run(max(10, args.steps // 4))
    nacl = None if args.no_nacl else nacl_run()
    ensemble = None if args.no_ensemble else ensemble_run(max(10, args.steps // 4))
    large = None if args.no_large else large_run(max(10, args.steps // 10))

    out = {
        "metric": "long-range particle-steps/s at 1e-4 force err (FP32 batched vs FP64 plain); p50/p99 latency",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch of {B} water-like boxes, 9000 atoms each (3000 rigid 3-site molecules), "
                               f"L=31.0, grid 32^3, P={prm.P}, tol 1e-4, FP32, HIP graph replay",
                   "batch": B, "atoms_per_system": N, "grid": prm.nf, "P": prm.P, "degree": prm.degree,
                   "c": prm.c, "c1": prm.c1, "rc": prm.rc, "tol": tol, "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "what": "per batched step"},
        "wall_s_timed_region": t_wall,
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": value / fp64["value"],
        "phases_ms": phases,
        "roofline": roof,
        "kernel_rooflines": kernels,
        "cpu_baseline": cpu,
        "serving": serving,
        "ik_forces": ik,
        "full_coulomb": full,
        "classical_method": classical,
        "orthorhombic": ortho,
        "triclinic": tric,
        "nacl_512": nacl,
        "ensemble": ensemble,
        "large_system": large,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
