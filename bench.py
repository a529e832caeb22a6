"""Benchmark of the ESP long-range pipeline on one MI355X.

Headline workload (the batched FP32 configuration at tol 1e-4): an ensemble
of 256 independent water-like boxes at 1 g/cm^3 (O -0.8476 / H +0.4238 rigid
three-site molecules), atom counts log-uniform in [500, 20000] (seeded),
each with its own side and grid (16^3 .. 48^3), P = 6. A step evaluates
potentials, forces and energies of all 256 systems with one FP32 batched
plan (autotuned bin edges), replayed as one HIP graph on the caller's
stream; inputs are resident in HBM. The FP64 plain path, one single-system
plan per box, is timed beside it, the phases are timed with HIP events on
the plan's stream, and the CPU reference five-step method is timed on the
host's cores on a sample of the same systems.

Per-configuration records follow under "configs": the 512-ion crystal (C1),
the 9000-atom water box alone and as a batch of 128 (C2), the 300,000-atom
box (C3), the ensemble itself (C4) and the served request stream (C5), each
with its own roofline record and CPU baseline where one applies.

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


def algorithmic_cost(phase, N, n, P, deg, prec, g=None):
    """Algorithmic HBM bytes and flops of one launch of a phase for one system
    of N particles on an n^3 grid (or, for spread and gather, N particles over
    g grid points in all). FMAs count 2 flops. Window weights are
    Horner polynomials of degree deg (3 P deg FMAs per particle for the
    values, 3 P (deg - 1) more for the derivatives); the spread forms the P^3
    products by P^2 + P^3 multiplies; the gather contracts the P^3
    neighbourhood for the value and three derivatives in 2 P^3 + 3 P^2 + 4 P
    FMAs. The grid is written (spread) or read (gather) once."""
    rb = 8 if prec == 64 else 4
    if g is None:
        g = n ** 3                   # grid points
    spec = n * n * (n // 2 + 1)      # half-spectrum modes
    if phase == "spread":
        b = N * 4 * rb + g * rb                     # sorted (u, q) in, grid out
        f = 2 * N * (3 * P * deg + P * P + P ** 3)
    elif phase == "gather":
        b = N * (4 * rb + 4 + 4 * rb) + g * rb      # sorted in, perm, phi+F out, grid in
        f = 2 * N * (3 * P * deg + 3 * P * (deg - 1) + 2 * P ** 3 + 3 * P * P + 4 * P)
    elif phase in ("fft_zy", "fft_yz"):
        b = g * rb + spec * 2 * rb
        f = 2.5 * spec * 2 * math.log2(n * n)      # ~5 N log2 N per complex transform pair
    elif phase == "fft_x_scale":
        b = 2 * spec * 2 * rb
        f = 2 * 5 * spec * math.log2(n) + 8 * spec
    elif phase == "hist":
        b = N * (4 * rb + 4)
        f = N * 10
    elif phase == "scatter":
        b = N * (4 * rb + 4 + 4 * rb + 4)
        f = N * 10
    else:
        b, f = 0, 0
    return b, f


# LDS: 128 bytes per clock per CU (32 banks x 4 B) -> 16 lanes of 64-bit atomics
# or 32 lanes of 32-bit reads per clock per CU, over 256 CUs at 2.4 GHz.
PEAK_LDS_U64_ATOMICS_GOPS = 16 * 256 * 2.4
PEAK_LDS_F32_READS_GOPS = 32 * 256 * 2.4
PEAK_LDS_U32_ATOMICS_GOPS = 32 * 256 * 2.4

PHASE_KERNEL = {"hist": "k_hist<float>", "scan": "k_scan", "scatter": "k_scatter<float>",
                "spread": "k_spread<float, {P}>", "fft_zy": "k_fwd_zy<float, {n}>",
                "fft_x_scale": "k_fft_x<float, {n}>", "fft_yz": "k_inv_yz<float, {n}>",
                "gather": "k_gather<float, {P}, {BT}>", "finalize": "k_finalize"}
# threads per gather block: 256 in launches of at least 4 bins per compute unit
GATHER_MANY_BINS = 4 * 256


def measured_traffic(profile, kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter
    summary profiles/<profile>_hbm_traffic.md, or None when it is missing or
    the kernel sources changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{profile}_hbm_traffic.md")
    try:
        txt = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", txt, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    for f, h in rec["source_sha256_16"].items():
        src = os.path.join(ROOT, "paper_2505_09727_amd", "csrc", f)
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != h:
            return None
    return rec["hbm_bytes_per_dispatch"].get(kernel)


def roofline(phase, ms, systems, prec=32, profile=None, points=None, blocks=None):
    """Roofline record of one launch of a phase over the systems it covers
    (list of (N, n, P, degree)); algorithmic bytes and flops from
    algorithmic_cost, ms the measured launch time. With `points`, systems is
    one entry (particles of the launch, n of its first system, P, degree) and
    points the grid points of all its systems (spread and gather)."""
    bytes_launch = flops_launch = 0
    atoms = p3 = 0
    for (N, n, P, deg) in systems:
        b1, f1 = algorithmic_cost(phase, N, n, P, deg, prec, g=points)
        bytes_launch += b1
        flops_launch += f1
        atoms += N
        p3 += N * P ** 3
    peak_alu = PEAK_FP64_VALU_TFLOPS if prec == 64 else PEAK_FP32_VALU_TFLOPS
    t = ms / 1e3
    gbs, tfl = bytes_launch / t / 1e9, flops_launch / t / 1e12
    if flops_launch / (peak_alu * 1e12) > bytes_launch / (PEAK_HBM_GBS * 1e9):
        r = dict(kernel=phase, bound="alu", achieved=tfl, peak=peak_alu, unit="TFLOP/s",
                 frac=tfl / peak_alu, hbm_achieved_GBs=gbs, hbm_frac=gbs / PEAK_HBM_GBS)
    else:
        r = dict(kernel=phase, bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s",
                 frac=gbs / PEAK_HBM_GBS, alu_achieved_TFLOPs=tfl)
    P0, n0 = systems[0][2], systems[0][1]
    bt = 256 if (blocks or 0) >= GATHER_MANY_BINS else 512
    kname = PHASE_KERNEL.get(phase, phase).format(P=P0, n=n0, BT=bt).replace("float", "double" if prec == 64 else "float")
    r["kernel_symbol"] = kname
    # a kernel launched more than once per step (one launch per pipeline
    # lane) has its traffic recorded per launch, keyed by its block count
    r["traffic"] = measured_traffic(profile, kname if blocks is None else f"{kname}#{blocks}") if profile else None
    r["avg_launch_ms"] = ms
    r["algorithmic_bytes_per_launch"] = bytes_launch
    r["algorithmic_flops_per_launch"] = flops_launch
    r["particles_per_launch"] = atoms
    if phase == "spread" and prec == 32:
        ops = p3 / t / 1e9
        if P0 <= 6:  # 32-bit fixed-point accumulators
            r["lds_u32_atomics"] = dict(achieved_Gops=ops, peak_Gops=PEAK_LDS_U32_ATOMICS_GOPS,
                                        frac=ops / PEAK_LDS_U32_ATOMICS_GOPS)
        else:
            r["lds_u64_atomics"] = dict(achieved_Gops=ops, peak_Gops=PEAK_LDS_U64_ATOMICS_GOPS,
                                        frac=ops / PEAK_LDS_U64_ATOMICS_GOPS)
    if phase == "gather" and prec == 32:
        ops = p3 / t / 1e9
        r["lds_f32_reads"] = dict(achieved_Gops=ops, peak_Gops=PEAK_LDS_F32_READS_GOPS,
                                  frac=ops / PEAK_LDS_F32_READS_GOPS)
    return r


def profile_phases(plan, pos, q, phi, F, reps):
    """Mean ms of each pipeline phase (esp_plan_profile: HIP events between
    the phases on the plan's stream)."""
    import ctypes as C
    from paper_2505_09727_amd.esp import lib
    nph = lib().esp_num_phases()
    ms = (C.c_double * nph)()
    st = lib().esp_plan_profile(plan._h, C.c_void_p(pos.data_ptr()), C.c_void_p(q.data_ptr()),
                                C.c_void_p(phi.data_ptr()), C.c_void_p(F.data_ptr()), reps, ms)
    assert st == 0, lib().esp_last_error()
    return {lib().esp_phase_name(i).decode(): ms[i] for i in range(nph)}


# Phases launched once per step whatever the systems' grid sizes (the FFT
# phases launch once per grid size): the dominant of these is the roofline
# record's kernel.
SINGLE_LAUNCH = ("hist", "spread", "gather")


def dominant_roofline(phases, systems, prec=32, profile=None):
    ph = max(SINGLE_LAUNCH, key=lambda k: phases.get(k, 0.0))
    return roofline(ph, phases[ph], systems, prec, profile)


def launch_rooflines(plan, pos, q, phi, F, reps, systems, profile, prec=32):
    """Per-launch rooflines of the spread and the gather (a plan with several
    pipeline lanes launches each once per (lane, P)): every launch timed on
    its own with HIP events (esp_plan_profile_launches). Returns {phase:
    [record per launch]}; the records carry launches_per_step."""
    P0, deg0, n0 = systems[0][2], systems[0][3], systems[0][1]
    out = {}
    for ph in ("spread", "gather"):
        ls = plan.profile_launches(pos, q, phi, F, reps, ph)
        recs = []
        for k, L in enumerate(ls):
            r = roofline(ph, L["ms"], [(L["particles"], n0, P0, deg0)], prec, profile, points=L["points"],
                         blocks=L["blocks"])
            r["launch"] = k
            r["launches_per_step"] = len(ls)
            r["blocks"] = L["blocks"]
            recs.append(r)
        out[ph] = recs
    return out


def dominant_launch_roofline(phases, launches):
    """The roofline record of the dominant kernel: among hist (one launch),
    spread and gather, the phase with the longest time per step; for spread
    and gather its longest launch."""
    ph = max(SINGLE_LAUNCH, key=lambda k: phases.get(k, 0.0))
    if ph in launches and launches[ph]:
        return max(launches[ph], key=lambda r: r["avg_launch_ms"])
    return None


def _one_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _oracle_job(args):
    """One evaluation of the reference five-step on one system (a pool job)."""
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


def cpu_baseline(jobs, what, budget_s=12.0, max_workers=16):
    """The reference five-step (FP64, exact window, matrix DFT) on the host's
    cores: jobs (systems with their parameters) in worker processes of one
    thread each, in rounds of one job per worker until about budget_s seconds
    have passed (at least one round). Returns particle-steps/s."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    host = _host()
    workers = max(1, min(max_workers, host["cpus_available"]))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_one_thread) as ex:
        # imports and first touch outside the timed window (the smallest jobs)
        warm = sorted(jobs, key=lambda j: len(j[1]))[:workers]
        list(ex.map(_oracle_job, warm))
        t0 = time.perf_counter()
        done, evals, k = 0, 0, 0
        while True:
            batch = [jobs[(k + i) % len(jobs)] for i in range(workers)]
            k += workers
            done += sum(ex.map(_oracle_job, batch))
            evals += len(batch)
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    return dict(value=done / el, unit="particle-steps/s", cores=workers, kind="oracle",
                sample=f"{evals} evaluations ({done} particle-steps) of {what} by the FP64 reference five-step "
                       f"(exact window, matrix DFT), {workers} worker processes of one thread each, {el:.1f} s",
                host=host)


def _job(pos, q, L, p):
    return (pos, q, L, p.nf, p.P, p.c, p.rc, p.c1)


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
    # grid size at the stream's tolerances, and one tiny request (two
    # opposite charges) per (grid size, tolerance), so that every kernel
    # variant the stream uses has run once
    tw = time.perf_counter()
    tols = sorted({r.tol for r in reqs})
    esp_warm_tables(tols, 144)
    warm_s = time.perf_counter() - tw
    srv = Server(hbm_budget_bytes=int(budget_gb * (1 << 30)))
    pair = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]], np.float32)
    qpair = np.array([1.0, -1.0], np.float32)
    for n in (8, 12, 16, 18, 24, 32, 36, 48, 54, 64, 72, 96, 108, 128, 144):
        for tol in tols:
            srv.submit(pair, qpair, 1.25 * n, tol, nsteps=2, drift=0.01, seed=1)
    srv.wait(120)
    srv.poll(1024)
    srv.close()
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
        "offered_rate_hz": rate,
        "scheduler_busy_frac": st["busy_s"] / st["span_s"] if st["span_s"] > 0 else None,
    }


def _time_plan(plan, ext, pos, q, phi, F, steps):
    """Mean ms per step of `steps` enqueued steps on the plan's stream, made
    torch's current stream so that the binding adds no cross-stream fences."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(ext):
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


def nacl_run(args, steps=200):
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
        # the plan on the caller's stream: no cross-stream fences per step
        plan, st = _stream_plan(L, len(q), cfg["tol"], nf=cfg["n"], P=cfg["P"], precision=prec)
        with torch.cuda.stream(st):
            tp = torch.tensor(pos, dtype=dt, device=dev)
            tq = torch.tensor(q, dtype=dt, device=dev)
            ph = torch.empty(len(q), dtype=dt, device=dev)
            F = torch.empty((len(q), 3), dtype=dt, device=dev)
            plan.autotune(tp, tq, ph, F, reps=5)
        plan.set_graph(True)
        _time_on(st, plan, tp, tq, ph, F, 5)
        out[f"fp{prec}_us_per_step"] = 1e3 * _time_on(st, plan, tp, tq, ph, F, steps)
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
    if not args.no_cpu_baseline:
        from paper_2505_09727_amd.esp import esp_plan_query
        p = esp_plan_query(L, len(q), cfg["tol"], nf=cfg["n"], P=cfg["P"])
        out["cpu_baseline"] = cpu_baseline([_job(pos, q, L, p)], "the perturbed 512-ion crystal", args.cpu_seconds)
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


def _stream_plan(*args, **kw):
    """A plan on a fresh torch stream (the caller's stream, esp_params.stream)."""
    import torch
    from paper_2505_09727_amd.esp import Plan
    st = torch.cuda.Stream()
    return Plan(*args, stream=st, **kw), st


def _time_on(stream, plan, pos, q, phi, F, steps, E_dev=None):
    """Mean ms per step of `steps` enqueued steps on the plan's (torch) stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(steps):
            plan.longrange_async(pos, q, phi, F, E_dev)
        e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def ensemble_headline(args, seed=4):
    """The 256-system ensemble: timed region of the headline (W warm-up and K
    timed steps of the FP32 batched plan, autotuned, graph replay, on the
    caller's stream), phase times, roofline, FP64 plain path, CPU baseline."""
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
    plan, st = _stream_plan(Ls, Ns, 1e-4)
    with torch.cuda.stream(st):
        pos = torch.tensor(np.concatenate([s[0] for s in systems]), dtype=torch.float32, device=dev)
        q = torch.tensor(np.concatenate([s[1] for s in systems]), dtype=torch.float32, device=dev)
        phi = torch.empty(Ntot, dtype=torch.float32, device=dev)
        F = torch.empty((Ntot, 3), dtype=torch.float32, device=dev)
        E_dev = torch.empty(len(systems), dtype=torch.float64, device=dev)
    default_tiles = Counter(p.tile for p in plan.params)
    grids = sorted({p.nf for p in plan.params})
    plan.set_graph(not args.no_graph)
    _time_on(st, plan, pos, q, phi, F, 3)  # capture and first replays, untimed
    ms_default = _time_on(st, plan, pos, q, phi, F, 20)
    t0 = time.perf_counter()
    tiles = plan.autotune(pos, q, phi, F, reps=5)
    tune_s = time.perf_counter() - t0
    one_block_fft = sum(1 for p in plan.params if p.fft_passes == 1)
    # timed region: W untimed warm-up steps, then exactly K steps between
    # synchronisations, with HIP events on the plan's stream around each step
    with torch.cuda.stream(st):
        for _ in range(args.warmup):
            plan.longrange_async(pos, q, phi, F, E_dev)
        plan.sync()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t_wall = time.perf_counter()
        evs[0].record(st)
        for k in range(args.steps):
            plan.longrange_async(pos, q, phi, F, E_dev)
            evs[k + 1].record(st)
        evs[-1].synchronize()
        torch.cuda.synchronize()
        t_wall = time.perf_counter() - t_wall
        E = plan.batch_longrange(pos, q, phi, F)   # waits; checks every system's neutrality
    step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    total_ms = evs[0].elapsed_time(evs[-1])
    F32 = F.cpu().double().numpy()
    phases = profile_phases(plan, pos, q, phi, F, args.profile_reps)
    sysl = [(N, p.nf, p.P, p.degree) for N, p in zip(Ns, plan.params)]
    kernels = launch_rooflines(plan, pos, q, phi, F, args.profile_reps, sysl, "esp_fp32_ensemble256")
    roof = dominant_launch_roofline(phases, kernels)
    if roof is None:
        roof = dominant_roofline(phases, sysl, 32, "esp_fp32_ensemble256")
        if roof["kernel"] == "hist":
            roof["kernel_symbol"] = "k_bin_small<float>"
    prm = list(plan.params)
    plan.close()
    # FP64 plain, one single-system plan after another
    ms64, errs, errs_w = 0.0, [], []
    for s, (ps, qs, L) in enumerate(systems):
        p64, s64 = _stream_plan(L, len(qs), 1e-4, precision=64)
        with torch.cuda.stream(s64):
            tp = torch.tensor(ps, dtype=torch.float64, device=dev)
            tq = torch.tensor(qs, dtype=torch.float64, device=dev)
            ph = torch.empty(len(qs), dtype=torch.float64, device=dev)
            Fs = torch.empty((len(qs), 3), dtype=torch.float64, device=dev)
            p64.longrange_async(tp, tq, ph, Fs)
        ms64 += _time_on(s64, p64, tp, tq, ph, Fs, 3)
        F64 = Fs.cpu().numpy()
        errs.append(_rel_rms(F32[off[s]:off[s + 1]], F64))
        errs_w.append(float(np.max(np.linalg.norm(F32[off[s]:off[s + 1]] - F64, axis=1))
                            / np.sqrt(np.mean(np.sum(F64 ** 2, axis=1)))))
        p64.close()
    cpu = None
    if not args.no_cpu_baseline:
        order = np.argsort(Ns)   # every size class in the sample: sizes spread over the jobs
        jobs = [_job(systems[i][0], systems[i][1], systems[i][2], prm[i]) for i in order[::4]]
        cpu = cpu_baseline(jobs, "ensemble systems (every fourth by size, 500-20,000 atoms)", args.cpu_seconds)
    value = Ntot * args.steps / (total_ms / 1e3)
    rec = {
        "workload": f"256 water-like boxes at 1 g/cm^3, atoms log-uniform in [500, 20000] (total {Ntot}), "
                    f"grids {grids[0]}^3..{grids[-1]}^3, P=6, tol 1e-4, FP32 batched plan (one launch per "
                    f"phase), autotuned bin edges, HIP graph replay on the caller's stream",
        "systems": len(systems), "atoms_total": Ntot, "grids": grids,
        "particle_steps_per_s": value, "ms_per_step": total_ms / args.steps,
        "latency_ms_per_step": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "wall_s_timed_region": t_wall,
        "ms_per_step_default_tiles": ms_default, "autotune_s": tune_s,
        "tiles_default": dict(default_tiles), "tiles_autotuned": dict(Counter(tiles)),
        "systems_on_one_block_fft": one_block_fft,
        "phases_ms": phases, "roofline": roof, "kernel_rooflines": kernels,
        "fp64_plain": {"particle_steps_per_s": Ntot / (ms64 / 1e3), "ms_per_sweep": ms64,
                       "what": "256 single-system FP64 plans run one after another"},
        "speedup_vs_fp64_plain": ms64 / (total_ms / args.steps),
        "fp32_vs_fp64_forces": {"rel_rms_median": float(np.median(errs)), "rel_rms_max": float(np.max(errs)),
                                "worst_particle_over_rms_max": float(np.max(errs_w))},
        "energies_finite": bool(np.all(np.isfinite(E))),
        "cpu_baseline": cpu,
    }
    return value, total_ms / args.steps, rec


def water9k_run(args):
    """The 9000-atom water box: FP32 and FP64 single-system plans, and a batch
    of 128 such boxes (FP32, graph replay) with its phases, roofline and the
    CPU baseline on boxes of the batch. Returns the record and the batch's
    device arrays for the sections that reuse them."""
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    B, L, n_mol, tol = args.batch, 31.0, 3000, 1e-4
    N = 3 * n_mol
    out = {"workload": "water-like box, 3000 rigid 3-site molecules (9000 atoms), L = 31.0, grid 32^3, P = 6, tol 1e-4"}
    box0 = W.water_box(n_mol, L, seed=W.WATER_9K["seed"])
    single = {}
    for prec, dt in ((32, torch.float32), (64, torch.float64)):
        plan, st = _stream_plan(L, N, tol, precision=prec)
        with torch.cuda.stream(st):
            tp = torch.tensor(box0[0], dtype=dt, device=dev)
            tq = torch.tensor(box0[1], dtype=dt, device=dev)
            ph = torch.empty(N, dtype=dt, device=dev)
            Fs = torch.empty((N, 3), dtype=dt, device=dev)
        plan.autotune(tp, tq, ph, Fs, reps=5)
        plan.set_graph(True)
        _time_on(st, plan, tp, tq, ph, Fs, 10)
        ms = _time_on(st, plan, tp, tq, ph, Fs, max(20, args.steps // 2))
        with torch.cuda.stream(st):
            plan.longrange(tp, tq, ph, Fs)
        single[prec] = Fs.cpu().double().numpy()
        p = plan.params[0]
        out[f"single_fp{prec}"] = {"particle_steps_per_s": N / (ms / 1e3), "ms_per_step": ms, "tile": p.tile,
                                   "fft_passes": p.fft_passes}
        plan.close()
    out["single_fp32_vs_fp64"] = {"rel_rms_F": _rel_rms(single[32], single[64]),
                                  "speedup": out["single_fp64"]["ms_per_step"] / out["single_fp32"]["ms_per_step"]}
    boxes = [W.water_box(n_mol, L, seed=1000 + b) for b in range(B)]
    plan, st = _stream_plan([L] * B, [N] * B, tol)
    with torch.cuda.stream(st):
        pos = torch.tensor(np.concatenate([b[0] for b in boxes]), dtype=torch.float32, device=dev)
        q = torch.tensor(np.concatenate([b[1] for b in boxes]), dtype=torch.float32, device=dev)
        phi = torch.empty(B * N, dtype=torch.float32, device=dev)
        F = torch.empty((B * N, 3), dtype=torch.float32, device=dev)
    prm = plan.params[0]
    plan.set_graph(True)
    _time_on(st, plan, pos, q, phi, F, 10)
    ms = _time_on(st, plan, pos, q, phi, F, args.steps)
    with torch.cuda.stream(st):
        plan.batch_longrange(pos, q, phi, F)
    F_all = F.cpu().double().numpy()
    phases = profile_phases(plan, pos, q, phi, F, args.profile_reps)
    sysl = [(N, prm.nf, prm.P, prm.degree)] * B
    kernels = launch_rooflines(plan, pos, q, phi, F, args.profile_reps, sysl, "esp_fp32_water9k_b128")
    roof = dominant_launch_roofline(phases, kernels)
    if roof is None:
        roof = dominant_roofline(phases, sysl, 32, "esp_fp32_water9k_b128")
        if roof["kernel"] == "hist":
            roof["kernel_symbol"] = "k_bin_small<float>"
    kernels.update({ph: roofline(ph, phases[ph], sysl, 32, "esp_fp32_water9k_b128")
                    for ph in ("fft_zy", "fft_x_scale", "fft_yz")})
    plan.close()
    torch.cuda.synchronize()
    out["batch128_fp32"] = {"batch": B, "particle_steps_per_s": B * N / (ms / 1e3), "ms_per_step": ms,
                            "tile": prm.tile, "phases_ms": phases, "roofline": roof, "kernel_rooflines": kernels,
                            "speedup_vs_single_fp64": out["single_fp64"]["ms_per_step"] * B / ms}
    out["roofline"] = roof
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(
        [_job(b[0], b[1], L, prm) for b in boxes], "9000-atom boxes of the batch", args.cpu_seconds)
    out["params"] = {"grid": prm.nf, "P": prm.P, "degree": prm.degree, "c": prm.c, "c1": prm.c1, "rc": prm.rc}
    return out, (pos, q, L, B, N, boxes, F_all)


def large_run(args, serve_steps=100):
    """300,000-atom water-like box (L = 100, tol 1e-5, n = 96, P = 8): FP32 plan
    vs FP64 plain on the same positions, phases and roofline of the FP32
    plan, the CPU baseline, the local part, and 100 served steps with 0.01
    drift (device resident, one request)."""
    import torch
    import workloads as W
    from paper_2505_09727_amd.esp import Server
    dev = torch.device("cuda:0")
    cfg = W.WATER_300K
    pos, q = W.water_box(cfg["n_mol"], cfg["L"], seed=cfg["seed"])
    L, N, tol = cfg["L"], len(q), cfg["tol"]
    steps = max(10, args.steps // 4)
    out = {"workload": f"{N} atoms (100,000 water-like molecules), L={L}, grid 96^3, P=8, tol {tol}"}
    res = {}
    for prec, dt in ((32, torch.float32), (64, torch.float64)):
        plan, st = _stream_plan(L, N, tol, precision=prec)
        with torch.cuda.stream(st):
            tp = torch.tensor(pos, dtype=dt, device=dev)
            tq = torch.tensor(q, dtype=dt, device=dev)
            ph = torch.empty(N, dtype=dt, device=dev)
            Fs = torch.empty((N, 3), dtype=dt, device=dev)
        plan.set_graph(True)
        _time_on(st, plan, tp, tq, ph, Fs, 3)
        ms = _time_on(st, plan, tp, tq, ph, Fs, steps)
        with torch.cuda.stream(st):
            E = plan.longrange(tp, tq, ph, Fs)
        p = plan.params[0]
        res[prec] = dict(ms=ms, F=Fs.cpu().double().numpy(), E=float(E[0]))
        rec = {"particle_steps_per_s": N / (ms / 1e3), "ms_per_step": ms, "grid": p.nf, "P": p.P,
               "degree": p.degree, "tile": p.tile}
        if prec == 32:
            phases = profile_phases(plan, tp, tq, ph, Fs, args.profile_reps)
            rec["phases_ms"] = phases
            out["roofline"] = dominant_roofline(phases, [(N, p.nf, p.P, p.degree)], 32, "esp_fp32_water300k")
            prm32 = p
        out[f"fp{prec}"] = rec
        plan.close()
    if not args.no_local:
        plan, st = _stream_plan(L, N, tol, local=1)
        with torch.cuda.stream(st):
            tp = torch.tensor(pos, dtype=torch.float32, device=dev)
            tq = torch.tensor(q, dtype=torch.float32, device=dev)
            ph = torch.empty(N, dtype=torch.float32, device=dev)
            Fs = torch.empty((N, 3), dtype=torch.float32, device=dev)
        plan.set_graph(True)
        _time_on(st, plan, tp, tq, ph, Fs, 3)
        msl = _time_on(st, plan, tp, tq, ph, Fs, steps)
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
    if not args.no_cpu_baseline:
        # one evaluation of the whole box per worker (about 20-30 s each)
        out["cpu_baseline"] = cpu_baseline([_job(pos, q, L, prm32)], "the 300,000-atom box", 1.0,
                                           max_workers=args.cpu_workers_large)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=128, help="boxes in the 9000-atom batch")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of each CPU-baseline sample")
    ap.add_argument("--cpu-workers-large", type=int, default=16,
                    help="worker processes of the 300,000-atom CPU baseline (one box each)")
    ap.add_argument("--profile-reps", type=int, default=20)
    ap.add_argument("--serve-seconds", type=float, default=0.5, help="length of the served arrival stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-loads", type=str, default="1,1.5,2",
                    help="offered loads as multiples of --serve-rate (the saturation curve)")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--only-headline", action="store_true", help="the ensemble only (profiling runs)")
    ap.add_argument("--only-large", action="store_true",
                    help="the 300,000-atom box only, long-range FP32 and FP64 (profiling runs; no headline value)")
    ap.add_argument("--no-ik", action="store_true", help="skip the ik-forces section")
    ap.add_argument("--no-large", action="store_true", help="skip the 300,000-atom section")
    ap.add_argument("--no-local", action="store_true", help="skip the full-Coulomb (local part) sections")
    ap.add_argument("--no-classical", action="store_true", help="skip the classical-method (PME) comparison")
    ap.add_argument("--no-box", action="store_true", help="skip the orthorhombic-box section")
    ap.add_argument("--no-nacl", action="store_true", help="skip the 512-ion crystal section")
    ap.add_argument("--no-cell", action="store_true", help="skip the triclinic-cell section")
    ap.add_argument("--no-water9k", action="store_true", help="skip the 9000-atom box section")
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
    if args.only_headline or args.only_large:
        args.no_cpu_baseline = args.no_water9k = args.no_nacl = True
        args.no_ik = args.no_local = args.no_classical = args.no_box = args.no_cell = True
        args.serve_seconds = 0
        args.no_large = args.only_headline

    import torch
    torch.cuda.synchronize()
    configs = {}
    if args.only_large:
        value, ms_per_step, ens = None, None, None
    else:
        value, ms_per_step, ens = ensemble_headline(args)
        print(f"# ensemble: {value:.3e} particle-steps/s, {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)
        configs["C4_ensemble"] = ens
    extras = {}
    if not args.no_water9k:
        w9, (pos, q, L, B, N, boxes, F_all) = water9k_run(args)
        configs["C2_water9k"] = w9
        print("# water9k done", file=sys.stderr, flush=True)
        ms_b = w9["batch128_fp32"]["ms_per_step"]
        if not args.no_ik:
            extras["ik_forces"] = ik_run(pos, q, L, B, N, max(10, args.steps // 4), F_all)
        full = None
        if not args.no_local:
            full = local_run(pos, q, L, B, N, max(10, args.steps // 4), boxes[0], args.profile_reps)
            extras["full_coulomb"] = full
        if not args.no_classical:
            extras["classical_method"] = classical_run(pos, q, L, B, N, max(10, args.steps // 4), ms_b,
                                                       full["ms_per_step"] if full else None)
        del pos, q, F_all
        print("# water9k extras done", file=sys.stderr, flush=True)
    if not args.no_box:
        extras["orthorhombic"] = box_run(max(10, args.steps // 4))
    if not args.no_cell:
        extras["triclinic"] = cell_run(max(10, args.steps // 4))
    if not args.no_nacl:
        configs["C1_nacl512"] = nacl_run(args)
        print("# nacl done", file=sys.stderr, flush=True)
    if not args.no_large:
        configs["C3_water300k"] = large_run(args)
        print("# water300k done", file=sys.stderr, flush=True)
    if args.serve_seconds > 0:
        runs = [serving_run(args.serve_seconds, args.serve_rate * float(m), args.serve_budget_gb)
                for m in args.serve_loads.split(",")]
        # the highest offered load the server keeps up with: served within 5%
        # of offered, with every request completed
        kept_up = [r for r in runs if r["completed"] == r["requests"] and r["particle_steps_per_s"]
                   and r["particle_steps_per_s"] >= 0.95 * r["offered_particle_steps_per_s"]]
        configs["C5_serving"] = dict(runs[0], load_curve=[
            {k: r[k] for k in ("offered_rate_hz", "offered_particle_steps_per_s", "particle_steps_per_s",
                               "p50_latency_ms", "p99_latency_ms", "max_latency_ms", "scheduler_busy_frac")}
            for r in runs], max_sustained_rate_hz=max((r["offered_rate_hz"] for r in kept_up), default=None))

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
        "config": {"workload": ens["workload"], "systems": ens["systems"], "atoms_total": ens["atoms_total"],
                   "grids": ens["grids"], "P": 6, "tol": 1e-4, "parallelism": "single GPU"} if ens else None,
        "latency_ms": {"p50": ens["latency_ms_per_step"]["p50"], "p99": ens["latency_ms_per_step"]["p99"],
                       "what": "per batched step of all 256 systems (request latency: configs.C5_serving)"}
        if ens else None,
        "wall_s_timed_region": ens["wall_s_timed_region"] if ens else None,
        "fp64_plain": ens["fp64_plain"] if ens else None,
        "speedup_vs_fp64_plain": ens["speedup_vs_fp64_plain"] if ens else None,
        "phases_ms": ens["phases_ms"] if ens else None,
        "roofline": ens["roofline"] if ens else None,
        "cpu_baseline": ens["cpu_baseline"] if ens else None,
        "configs": configs,
        "extras": extras,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
