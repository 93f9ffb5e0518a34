#!/usr/bin/env python
"""Benchmark of one block-eigensolver step (the whole hot path) on one MI355X.

One step = degree-m Chebyshev filter (m H applications, each: stick/plane FFTs with V(r),
projector GEMMs, fused update) + W = H Y + [S | H_s] = Y^H [Y | W] + FP64 generalised
eigensolve + rotation + residual norms.  Default workload: Si512 (4x4x4 diamond cells,
a = 10.26 bohr), E_cut = 20 Ha, 1088 bands, degree 10, mixed precision (FP32 complex FFTs
and GEMMs, FP64 eigensolve and residuals); the FP64 form of the same step is timed beside
it and one step of each from the same block gives the eigenvalue difference.

Prints one JSON line.  Inputs are synthetic and seeded; they are resident in device memory
before the timed region starts.
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
# bf16 split products: Gram / projected matrices (4 terms), projectors and rotations (3 terms)
DEFAULT_MIXED_FLAGS = 2 | 4 | 8
PEAK_BF16_TFLOPS = 2516.6
PEAK_VALU_FP32_TFLOPS = 157.3  # FP32 vector ALU (256 CUs at 2.4 GHz)
METRIC = "eig-steps/sec & HΨ band-apps/sec, mixed vs FP64 @|Δε|≤1e-5 Ha; p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def phase_work(name: str, info, nb: int, m: int, steps: int, real_bytes: int, n1a: int = 0):
    """Algorithmic work of a phase over the timed region: (amount, kind) with kind 'flop' or 'byte'."""
    npw, nproj, nst = int(info.npw), int(info.nproj), int(info.nst)
    n1, n2, n3 = (int(x) for x in info.fft_n)
    nr = n1 * n2 * n3
    cb = 2 * real_bytes
    happs = steps * (m + 1)  # H applications of nb bands in the timed steps
    bands = happs * nb
    if name == "proj" or name == "nl":
        return 8.0 * npw * nproj * nb * happs, "flop"
    if name == "gram":
        # S = Y^H Y (Hermitian: one triangle, 4 N_pw N_b^2) and H_s = Y^H W (8 N_pw N_b^2)
        return 12.0 * npw * nb * nb * steps, "flop"
    if name == "rotate":
        return 8.0 * npw * nb * nb * 2 * steps, "flop"
    if name == "sticks_inv" or name == "sticks_fwd":
        return float(bands) * (npw + nst * n3) * cb, "byte"
    if name == "plane":
        return float(bands) * (2.0 * nst * n3 * cb + nr * real_bytes), "byte"
    if name == "pencil_yinv" or name == "pencil_yfwd":
        return float(bands) * (nst * n3 + n3 * n2 * n1a) * cb, "byte"
    if name == "pencil_x":
        return float(bands) * (2.0 * n3 * n2 * n1a * cb + nr * real_bytes), "byte"
    if name == "resid":
        return 2.0 * npw * nb * cb * steps, "byte"
    return None, None


# flops the kernels execute per algorithmic flop: the Gram kernel forms all of S, except that its
# pipelined form (blocks of 256 x 128 entries, used from nb x 2 nb >= 2^20 entries on) skips the
# blocks of S wholly below the diagonal
EXECUTED_PER_ALGORITHMIC = {"gram": 16.0 / 12.0}


def gram_executed_per_algorithmic(nb: int) -> float:
    if nb * 2 * nb < (1 << 20):
        return 16.0 / 12.0
    tm, tn = -(-nb // 256), -(-(2 * nb) // 128)
    skipped = sum(1 for i in range(tm) for j in range(tn) if (j + 1) * 128 <= nb and i * 256 > j * 128 + 127)
    return 16.0 / 12.0 * (tm * tn - skipped) / (tm * tn)


def measured_traffic(workload, flags, phase):
    """HBM bytes per launch of a phase from the committed counter summary (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, scaled by the copy-kernel calibration), or None when the summary does not cover this
    workload or the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_mixed_hbm_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    src = os.path.join(ROOT, d["source"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != d["source_sha256"]:
            return None
    if d.get("mixed_flags") != flags or phase not in d["kernels"]:
        return None
    k = d["kernels"][phase]
    return 1024.0 * (k["FETCH_SIZE_KiB"] * d["scale"]["FETCH_SIZE"] + k["WRITE_SIZE_KiB"] * d["scale"]["WRITE_SIZE"])


def phase_table(stats, info, nb, m, steps, real_bytes, n1a, nterm, fp64=False, mixed_flags=0):
    """Per-phase rates over the timed steps and the roofline entry of the longest phase."""
    mfma_peak = PEAK_MFMA_TFLOPS["fp64" if fp64 else "fp32"]
    phases = {}
    dom, dom_ms = None, -1.0
    for name, st in stats.items():
        if st["launches"] == 0:
            continue
        amount, kind = phase_work(name, info, nb, m, steps, real_bytes, n1a)
        entry = {"launches": st["launches"], "ms_total": round(st["ms"], 3),
                 "ms_per_launch": round(st["ms"] / st["launches"], 4)}
        if amount is not None:
            if kind == "flop":
                entry["tflops"] = round(amount / (st["ms"] * 1e-3) / 1e12, 2)
                if name in nterm:
                    ratio = EXECUTED_PER_ALGORITHMIC.get(name, 1.0)
                    if name == "gram" and (mixed_flags & 14) == 14:
                        ratio = gram_executed_per_algorithmic(nb)
                    ex = entry["tflops"] * nterm[name] * ratio
                    entry["dtype"] = "bf16x%d" % nterm[name]
                    entry["tflops_bf16_executed"] = round(ex, 2)
                    entry["frac_peak"] = round(entry["tflops"] / PEAK_BF16_TFLOPS, 4)
                    entry["frac_peak_executed"] = round(ex / PEAK_BF16_TFLOPS, 4)
                else:
                    entry["dtype"] = "fp64" if fp64 else "fp32"
                    entry["frac_peak"] = round(entry["tflops"] / mfma_peak, 4)
            else:
                entry["gbs"] = round(amount / (st["ms"] * 1e-3) / 1e9, 1)
                entry["frac_peak"] = round(entry["gbs"] / PEAK_HBM_GBS, 4)
            if st["ms"] > dom_ms:
                dom, dom_ms = name, st["ms"]
        phases[name] = entry
    if dom is None:
        return phases, None, None
    d = phases[dom]
    amount, kind = phase_work(dom, info, nb, m, steps, real_bytes, n1a)
    per_launch = amount / stats[dom]["launches"]
    if kind == "flop":
        peak = PEAK_BF16_TFLOPS if dom in nterm else mfma_peak
        roofline = {"bound": "mfma", "kernel": dom, "achieved": d["tflops"], "peak": peak, "unit": "TFLOP/s",
                    "frac": d["frac_peak"], "traffic": None, "algorithmic_per_launch": per_launch,
                    "avg_launch_ms": d["ms_per_launch"]}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": d["frac_peak"], "traffic": None, "algorithmic_per_launch": per_launch,
                    "avg_launch_ms": d["ms_per_launch"]}
    return phases, dom, roofline


def occupied_angle(Xa, Xb, nocc, npw):
    """Largest principal angle (radians) between the spans of the first nocc columns of two
    blocks (rows of the (nb, ld) tensors), each orthonormal."""
    import torch

    A = Xa[:nocc, :npw].to(torch.complex128)
    B = Xb[:nocc, :npw].to(torch.complex128).t().contiguous()
    M = torch.mm(A.conj(), B)
    s = torch.linalg.svdvals(M.cpu()).numpy()
    return float(np.arccos(min(1.0, float(s.min()))))


def accuracy_at_convergence(pw, synth, torch, workload, mflags, degree, tol_mixed=5e-5, tol_fp64=1e-9):
    """Mixed and FP64 solves of one cell from the same seeded block, compared at convergence:
    eigenvalue differences, per-cluster principal angles with the Davis-Kahan bound beside them
    (residuals of the mixed span from an FP64 Rayleigh-Ritz on it), and the FP64 polish (FP64 steps
    started from the converged mixed block)."""
    from paper_2406_10765_amd import accuracy as acc

    cell = synth.make_cell(workload)
    nb, nocc = cell.nbands, cell.nocc
    hm = pw.Handle(cell, pw.PW_MIXED, flags=mflags)
    h64 = pw.Handle(cell, pw.PW_FP64)
    if not np.array_equal(hm.gvectors(), h64.gvectors()):
        raise RuntimeError("mixed and FP64 handles order the plane waves differently")
    X0 = hm.random_block(nb, synth.SEED_X0 + synth.WORKLOADS[workload]["index"])
    t0 = time.perf_counter()
    Xm = X0.clone()
    em, rm, sm, cm = hm.solve(Xm, nocc, tol_mixed, degree, 200)
    t_m = time.perf_counter() - t0
    t0 = time.perf_counter()
    X64 = X0.to(torch.complex128)
    e64, r64, s64, c64 = h64.solve(X64, nocc, tol_fp64, degree, 400)
    t_64 = time.perf_counter() - t0
    # FP64 Rayleigh-Ritz on span X_m: same span, FP64 Ritz values and exact residuals
    Y = Xm.to(torch.complex128)
    erep, rrep, _ = h64.eig_step(Y, 0, b=1.0)
    t0 = time.perf_counter()
    Xp = Y.clone()
    ep, rp, sp, cp = h64.solve(Xp, nocc, tol_fp64, degree, 400)
    t_p = time.perf_counter() - t0
    A64, Am, Ap = h64.to_host(X64), h64.to_host(Y), h64.to_host(Xp)
    rows_m = acc.cluster_report(Am, erep, rrep, A64, e64, r64, nocc)
    rows_p = acc.cluster_report(Ap, ep, rp, A64, e64, r64, nocc)
    worst = sorted(rows_m, key=lambda r: -r[2])[:8]
    out = {
        "workload": workload, "mixed_flags": mflags, "degree": degree, "nocc": nocc, "clusters": len(rows_m),
        "mixed": {"tol": tol_mixed, "steps": sm, "converged": bool(cm), "seconds": round(t_m, 3),
                  "max_resid_occ": float(rm[:nocc].max())},
        "fp64": {"tol": tol_fp64, "steps": s64, "converged": bool(c64), "seconds": round(t_64, 3),
                 "max_resid_occ": float(r64[:nocc].max())},
        "max_abs_deig_occ_mixed_vs_fp64_Ha": float(np.abs(em[:nocc] - e64[:nocc]).max()),
        "max_abs_deig_occ_mixed_span_fp64_rr_Ha": float(np.abs(erep[:nocc] - e64[:nocc]).max()),
        "max_cluster_angle_rad": float(max(r[2] for r in rows_m)),
        "max_davis_kahan_bound": float(max(r[3] for r in rows_m)),
        "angles_within_bound": bool(all(r[2] <= r[3] * (1 + 1e-9) + 1e-15 for r in rows_m)),
        "worst_clusters": [{"bands": [lo, hi], "angle_rad": float(a), "davis_kahan_bound": float(b)}
                           for lo, hi, a, b in worst],
        "polish": {"fp64_steps": sp, "converged": bool(cp), "seconds": round(t_p, 3),
                   "fp64_steps_from_scratch": s64,
                   "max_abs_deig_occ_Ha": float(np.abs(ep[:nocc] - e64[:nocc]).max()),
                   "max_cluster_angle_rad": float(max(r[2] for r in rows_p)),
                   "max_davis_kahan_bound": float(max(r[3] for r in rows_p))},
        "what": "both forms converged from the same seeded block (occupied residuals <= tol); angles per "
                "cluster of FP64 eigenvalues (gap < 1e-3 Ha) against the FP64 block; the bound adds the "
                "Davis-Kahan bounds ||R||_F / delta of both blocks; polish = FP64 steps from the mixed block",
    }
    del hm, h64, X0, Xm, X64, Y, Xp
    torch.cuda.empty_cache()
    return out


def device_info(torch, minfo):
    p = torch.cuda.get_device_properties(0)
    out = {"name": p.name, "arch": getattr(p, "gcnArchName", None), "hbm_gib": round(p.total_memory / 2**30, 1),
           "hip": torch.version.hip, "cus": p.multi_processor_count,
           "arena_gib_mixed": round(minfo.footprint_bytes / 2**30, 2)}
    try:  # current clocks as the SMI tool reports them (a child process; absent tools are skipped)
        import subprocess
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        card = next(iter(json.loads(r.stdout).values()))
        out["clocks"] = {k: v for k, v in card.items() if "clock" in k.lower()}
    except Exception:
        out["clocks"] = None
    return out


def run_steps(h, X, m, steps, bounds, b, keep_first=False, times=None):
    """steps eig-steps on X; each returns after its host outputs are written, so the wall time
    between returns is the step time (appended to times when given)."""
    import torch

    eig = res = first = None
    t_prev = time.perf_counter()
    for i in range(steps):
        eig, res, bnd = h.eig_step(X, m, bounds[0], bounds[1], b)
        if times is not None:
            t_now = time.perf_counter()
            times.append(t_now - t_prev)
            t_prev = t_now
        bounds = (bnd[0], bnd[1])
        if i == 0:
            first = eig.copy()
        if steps > 1:
            log(f"  step {i + 1}/{steps} done")
            t_prev = time.perf_counter()
    torch.cuda.synchronize()
    if keep_first:
        return eig, res, bounds, first
    return eig, res, bounds


def cpu_baseline(cell, nb: int, m: int, sample_bands: int = 32):
    """Time the oracle on a bounded sample and extrapolate to one step."""
    import scipy.linalg
    from oracle import pw_oracle as O
    from paper_2406_10765_amd import synth

    cores = len(os.sched_getaffinity(0))
    O.FFT_WORKERS = cores
    try:
        from threadpoolctl import threadpool_limits

        limiter = threadpool_limits(limits=cores)
    except Exception:  # pragma: no cover
        limiter = None
    t0 = time.time()
    model = O.model_from_cell(cell)
    t_model = time.time() - t0
    X = synth.initial_block(model.miller, cell.L, sample_bands, 5)
    t0 = time.time()
    W = O.apply_h(model, X)
    t_apply = time.time() - t0
    t0 = time.time()
    S = X.conj().T @ X
    Hs = X.conj().T @ W
    C = np.eye(sample_bands, dtype=complex)
    _ = X @ C
    _ = W @ C
    t_rr = time.time() - t0
    rng = np.random.default_rng(1)
    A = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
    A = A @ A.conj().T + nb * np.eye(nb)
    Bm = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
    Bm = 0.5 * (Bm + Bm.conj().T)
    t0 = time.time()
    scipy.linalg.eigh(Bm, A)
    t_eig = time.time() - t0
    step = (m + 1) * (nb / sample_bands) * t_apply + (nb / sample_bands) ** 2 * t_rr + t_eig
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return {
        "value": 1.0 / step,
        "unit": "eig-steps/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle H application on {sample_bands} of {nb} bands ({t_apply:.2f} s) and the "
                   f"Rayleigh-Ritz products on that block ({t_rr:.2f} s), extrapolated linearly in bands "
                   f"(quadratically for the products) to one degree-{m} step, plus a timed FP64 "
                   f"generalised eigensolve of size {nb} ({t_eig:.2f} s); model build {t_model:.1f} s not counted"),
        "extrapolated_step_s": step,
    }


def validate_cpu_baseline(workload: str, m: int, sample_bands: int = 32):
    """The extrapolation of cpu_baseline next to one fully timed oracle step of the same cell (all
    bands, degree m, from a seeded block), on the same cores: the check of the extrapolation."""
    from oracle import pw_oracle as O
    from paper_2406_10765_amd import synth

    cell = synth.make_cell(workload)
    nb = cell.nbands
    est = cpu_baseline(cell, nb, m, sample_bands)
    cores = est["cores"]
    O.FFT_WORKERS = cores
    model = O.model_from_cell(cell)
    hop = lambda Y: O.apply_h(model, Y)
    X0 = synth.initial_block(model.miller, cell.L, nb, 6)
    s0 = O.eig_step(hop, X0, 0, 0.0, 0.0, 1.0)
    b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=3)
    t0 = time.time()
    O.eig_step(hop, s0.X, m, s0.a_lo, s0.a, b)
    full = time.time() - t0
    return {"workload": workload, "bands": nb, "degree": m, "cores": cores,
            "extrapolated_step_s": est["extrapolated_step_s"], "timed_step_s": full,
            "ratio_extrapolated_over_timed": est["extrapolated_step_s"] / full, "sample": est["sample"]}


def peak_in_flight(intervals):
    ev = sorted([(a, 1) for a, _ in intervals] + [(d, -1) for _, d in intervals], key=lambda e: (e[0], e[1]))
    cur = peak = 0
    for _, dlt in ev:
        cur += dlt
        peak = max(peak, cur)
    return peak


def rspace_leg(pw, synth, torch, cell, m, steps):
    """The localized projector family on the bench cell, filtered with the reciprocal-space projector
    GEMMs (bf16 planes, the headline's flags) and with the real-space projectors (PW_FLAG_RSPACE_KB;
    the other products as in the headline), from the same block and bounds: ms per step, per-phase
    times, and the occupied eigenvalues of the first degree-m step of each.  Radius 5.5 sigma: the
    truncation then changes H X by less than FP32 rounding does (4.7e-8 relative on Si64)."""
    nb = cell.nbands
    R = 5.5 * cell.pseudo.beta_sigma
    seed = synth.SEED_X0 + 17
    out = {"radius_bohr": R, "projectors": "PW_PROJ_LOCALIZED",
           "what": "degree-%d filter steps, the same cell with the localized projectors applied by the "
                   "reciprocal-space GEMMs and in real space" % m}
    eigs = {}
    b = bounds = None
    routes = (("gspace", DEFAULT_MIXED_FLAGS, 0.0),
              ("rspace", (DEFAULT_MIXED_FLAGS & ~pw.PW_FLAG_BF16_KB) | pw.PW_FLAG_RSPACE_KB, R))
    for name, flags, rad in routes:
        h = pw.Handle(cell, pw.PW_MIXED, flags=flags, proj_form=pw.PW_PROJ_LOCALIZED, rs_radius=rad)
        if b is None:
            b = h.spectrum_bound(20, 1)
        X = h.random_block(nb, seed)
        _, _, bnd = h.eig_step(X, 0, b=b)
        if bounds is None:
            bounds = (bnd[0], bnd[1])
        e1, _, _ = h.eig_step(X, m, bounds[0], bounds[1], b)
        eigs[name] = e1
        run_steps(h, X, m, 1, bounds, b)
        torch.cuda.synchronize()
        ts = []
        t0 = time.perf_counter()
        run_steps(h, X, m, steps, bounds, b, times=ts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        h.reset_stats()
        h.set_timing(True)
        run_steps(h, X, m, 1, bounds, b)
        st = h.stats()
        h.set_timing(False)
        out[name] = {"ms_per_step": round(1000.0 * dt / steps, 2), "flags": flags,
                     "footprint_gb": round(h.info.footprint_bytes / 1e9, 2),
                     "phases_ms_per_step": {k: round(v["ms"], 3) for k, v in st.items() if v["launches"]},
                     "phases_launches_per_step": {k: v["launches"] for k, v in st.items() if v["launches"]}}
        log(f"{name} (localized projectors): {out[name]['ms_per_step']:.1f} ms/step")
        del h, X
        torch.cuda.empty_cache()
    out["max_abs_deig_occ_Ha"] = float(np.abs(eigs["gspace"][: cell.nocc] - eigs["rspace"][: cell.nocc]).max())
    out["speedup"] = round(out["gspace"]["ms_per_step"] / out["rspace"]["ms_per_step"], 3)
    # algorithmic work of the real-space passes: 16 flop (four real projectors times one complex
    # value) per ball point and band in each of the two passes; the ball points are counted on the
    # grid (nearest image), and the passes' time is the projection phase plus what the D P
    # addition adds to the plane phase
    n = np.asarray(pw.plan(cell, pw.PW_MIXED).fft_n)
    h = np.asarray(cell.L, float) / n
    nball = 0
    for t in np.asarray(cell.tau, float):
        t = np.mod(t, cell.L)
        ax = [np.arange(int(np.ceil((t[i] - R) / h[i])), int(np.floor((t[i] + R) / h[i])) + 1) * h[i] - t[i]
              for i in range(3)]
        d2 = ax[0][:, None, None] ** 2 + ax[1][None, :, None] ** 2 + ax[2][None, None, :] ** 2
        nball += int((d2 <= R * R).sum())
    r, g = out["rspace"]["phases_ms_per_step"], out["gspace"]["phases_ms_per_step"]
    t_ms = r.get("proj", 0.0) + r.get("plane", 0.0) - g.get("plane", 0.0)
    nl_apps = out["gspace"]["phases_launches_per_step"].get("nl", 0)
    flop = 2 * 16.0 * nball * nb * nl_apps
    out["ball_points"] = nball
    out["alu"] = {"flop_per_h_application": 2 * 16.0 * nball * nb, "h_applications_per_step": nl_apps,
                  "ms_per_step": round(t_ms, 2),
                  "tflops": round(flop / (t_ms * 1e-3) / 1e12, 2) if t_ms > 0 else None,
                  "peak_tflops": PEAK_VALU_FP32_TFLOPS,
                  "what": "both real-space passes against the FP32 vector peak (the GEMMs of the other route: "
                          "2 x 8 N_pw N_proj N_b flop per H application on the matrix cores)"}
    out["alu"]["frac"] = round(out["alu"]["tflops"] / PEAK_VALU_FP32_TFLOPS, 4) if out["alu"]["tflops"] else None
    return out


def serving_leg(n, rate, slots, flags, degree):
    """Poisson stream of eigen-solves (mixed precision) through the request loop."""
    import threading

    from paper_2406_10765_amd import pw, synth

    mix = synth.serving_mix(n, rate)
    srv = pw.Server(48 << 30, max_slots=slots)
    tickets = [None] * n
    t_base = srv.clock() + 0.5

    def client():
        for i, m in enumerate(mix):
            t = t_base + m["t_arrive"]
            while srv.clock() < t:
                time.sleep(min(0.002, max(0.0, t - srv.clock())))
            c = m["cell"]
            tickets[i] = srv.submit(c, pw.PW_MIXED, flags, seed=m["seed"], tol=1e-4, max_steps=200,
                                    degree=degree, nconv=c.nocc, t_arrive=t)

    th = threading.Thread(target=client)
    th.start()
    res = [None] * n
    while any(r is None for r in res):
        for i, m in enumerate(mix):
            if res[i] is None and tickets[i] is not None:
                res[i] = srv.poll(tickets[i], m["cell"].nbands)
        time.sleep(0.002)
    th.join()
    srv.close()
    lat = np.array([r["t_done"] - r["t_arrive"] for r in res])
    wait = np.array([r["t_admit"] - r["t_arrive"] for r in res])
    t0 = min(r["t_arrive"] for r in res)
    t1 = max(r["t_done"] for r in res)
    band_apps = sum((1 + (r["steps"] - 1) * (degree + 1) + r["steps"]) * m["cell"].nbands for r, m in zip(res, mix))
    by, svc = {}, {}
    for r, m in zip(res, mix):
        key = "%s_ecut%d" % (m["name"], int(m["cell"].ecut))
        by.setdefault(m["name"], []).append(r["t_done"] - r["t_arrive"])
        svc.setdefault(key, []).append(r["t_done"] - r["t_admit"])
    return {
        "requests": n, "rate_req_s": rate, "slots": slots,
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_queue_wait_s": float(wait.mean()),
        "throughput_req_s": n / (t1 - t0), "band_apps_per_sec": band_apps / (t1 - t0),
        "makespan_s": t1 - t0,
        "peak_in_flight": peak_in_flight([(r["t_admit"], r["t_done"]) for r in res]),
        "converged": int(sum(r["status"] == 0 for r in res)),
        "not_converged": [{"cell": m["name"], "ecut_ha": float(m["cell"].ecut), "seed": int(m["seed"]),
                           "status": int(r["status"]), "steps": int(r["steps"]), "message": r.get("message", "")}
                          for r, m in zip(res, mix) if r["status"] != 0],
        "retried_steps": [{"cell": m["name"], "ecut_ha": float(m["cell"].ecut), "seed": int(m["seed"]),
                           "status": int(r["status"]), "message": r.get("message", "")}
                          for r, m in zip(res, mix) if r.get("retried", 0) > 0],
        "mean_steps": float(np.mean([r["steps"] for r in res])),
        "p50_latency_by_cell_s": {k: float(np.percentile(v, 50)) for k, v in sorted(by.items())},
        "mean_service_by_cell_s": {k: float(np.mean(v)) for k, v in sorted(svc.items())},
    }


def serving_solve_phases(flags, degree):
    """One request of each serving cell and cutoff solved alone on the device (pw_solve, as the
    request loop runs it: seeded block, Lanczos bound, a degree-0 step, then degree-m steps to
    tol 1e-4 on the occupied bands): wall time of an untimed solve after a warm-up one, and the
    per-phase times (HIP events, phases serialised) of a third."""
    import torch

    from paper_2406_10765_amd import pw, synth

    out = {}
    for name, nc in synth.SERVING_CELLS.items():
        for ec in (10.0, 15.0, 20.0):
            cell = synth.silicon_cell(nc, ec, disp_seed=synth.SEED_REQUEST)
            h = pw.Handle(cell, pw.PW_MIXED, flags=flags)
            try:
                npw = h.info.npw
                walls = []
                for rep in range(3):
                    X = h.random_block(cell.nbands, synth.SEED_REQUEST)
                    if rep == 2:
                        h.set_timing(True)
                        h.reset_stats()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, _, steps, ok = h.solve(X, cell.nocc, 1e-4, degree=degree)
                    torch.cuda.synchronize()
                    walls.append(time.perf_counter() - t0)
                st = h.stats()
            finally:
                h.close()
            key = "%s_ecut%d" % (name, int(ec))
            out[key] = {"nbands": cell.nbands, "npw": int(npw), "steps": int(steps), "converged": bool(ok),
                        "wall_ms": round(1e3 * walls[1], 2), "timed_ms": round(1e3 * walls[2], 2),
                        "phases_ms": {k: round(v["ms"], 2) for k, v in st.items() if v["launches"]}}
            log(f"serving solve {key}: {steps} steps, {1e3 * walls[1]:.1f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="si512")
    ap.add_argument("--degree", type=int, default=10)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-lobpcg", action="store_true", help="skip the LOBPCG step timing")
    ap.add_argument("--no-rspace", action="store_true", help="skip the real-space projector comparison")
    ap.add_argument("--rspace-only", action="store_true",
                    help="run only the real-space projector comparison on the workload (for traces)")
    ap.add_argument("--rspace-apply", action="store_true",
                    help="two real-space H applications of the workload's block and exit (for counter runs)")
    ap.add_argument("--flags", type=int, default=None,
                    help="mixed-precision product flags (bit 2: bf16 Gram, 4: bf16 projectors, 8: bf16 rotation)")
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests in the serving mix (0 = skip; the recipe has 200)")
    ap.add_argument("--serving-rate", type=float, default=20.0)
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--serving-solve-phases", action="store_true",
                    help="per-phase times of one request of each serving cell and cutoff, solved alone, and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--accuracy-workload", default="si64",
                    help="cell of the mixed-vs-FP64 comparison at convergence ('none' to skip)")
    ap.add_argument("--validate-cpu-baseline", default=None, metavar="WORKLOAD",
                    help="CPU only: time one full oracle step of WORKLOAD beside the extrapolation and exit")
    ap.add_argument("--filter-only", action="store_true",
                    help="set up the workload, run one degree-m filter step and exit (for counter runs)")
    args = ap.parse_args()
    if args.validate_cpu_baseline:
        print(json.dumps({"cpu_baseline_validation": validate_cpu_baseline(args.validate_cpu_baseline,
                                                                           args.degree)}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2406_10765_amd import pw, synth

    torch.cuda.set_device(0)
    if args.serving_solve_phases:
        mflags = DEFAULT_MIXED_FLAGS if args.flags is None else args.flags
        print(json.dumps({"serving_solve_phases": serving_solve_phases(mflags, args.degree)}), flush=True)
        return
    if args.serving_only:
        mflags = DEFAULT_MIXED_FLAGS if args.flags is None else args.flags
        print(json.dumps({"serving": serving_leg(args.serving_requests, args.serving_rate, args.serving_slots,
                                                 mflags, args.degree)}), flush=True)
        return
    if args.rspace_apply:
        cell = synth.make_cell(args.workload)
        h = pw.Handle(cell, pw.PW_MIXED, flags=pw.PW_FLAG_RSPACE_KB | 2 | 8, proj_form=pw.PW_PROJ_LOCALIZED,
                      rs_radius=5.5 * cell.pseudo.beta_sigma)
        X = h.random_block(cell.nbands, synth.SEED_X0 + 17)
        HX = torch.empty_like(X)
        for i in range(2):
            h.apply_h(X, HX)
            torch.cuda.synchronize()
            log(f"real-space H application {i + 1} done")
        return
    if args.rspace_only:
        cell = synth.make_cell(args.workload)
        print(json.dumps({"rspace_projectors": rspace_leg(pw, synth, torch, cell, args.degree, args.steps)}),
              flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one copy kernel")
        del src, dst
    cell = synth.make_cell(args.workload)
    nb, m = cell.nbands, args.degree
    if args.filter_only:
        mflags = DEFAULT_MIXED_FLAGS if args.flags is None else args.flags
        hm = pw.Handle(cell, pw.PW_MIXED, flags=mflags)
        b = hm.spectrum_bound(20, 1)
        X = hm.random_block(nb, synth.SEED_X0 + synth.WORKLOADS[args.workload]["index"])
        eig, res, bnd = hm.eig_step(X, 0, b=b)
        eig, res, bnd = hm.eig_step(X, m, bnd[0], bnd[1], b)
        torch.cuda.synchronize()
        log(f"filter step done: lowest eigenvalue {eig[0]:.6f}")
        return

    # ---- mixed precision (the headline) --------------------------------------------------
    t0 = time.time()
    mflags = DEFAULT_MIXED_FLAGS if args.flags is None else args.flags
    dev_bytes = torch.cuda.get_device_properties(0).total_memory
    minfo = pw.plan(cell, pw.PW_MIXED, flags=mflags)
    ldp = (minfo.npw + 15) // 16 * 16
    big = minfo.footprint_bytes + 2 * nb * ldp * 8 > 0.9 * dev_bytes
    if big:
        # band-blocked steps of minutes: report each filter block as it completes
        os.environ["PW_PROGRESS"] = "1"
    hm = pw.Handle(cell, pw.PW_MIXED, flags=mflags)
    G = hm.gvectors()
    n1a = 2 * int(np.abs(G[:, 0]).max()) + 1
    b = hm.spectrum_bound(20, 1)
    X = hm.random_block(nb, synth.SEED_X0 + synth.WORKLOADS[args.workload]["index"])
    eig, res, bnd = hm.eig_step(X, 0, b=b)
    bounds = (bnd[0], bnd[1])
    log(f"setup and first (degree 0) step {time.time() - t0:.1f}s  npw={hm.npw} nb={nb} b={b:.4f} "
        f"fused_planes={hm.info.fused_planes} filter_block={hm.info.filter_block}")
    eig, res, bounds = run_steps(hm, X, m, args.warmup, bounds, b)
    # snapshot of the block the timed steps start from (the FP64 form starts from it too)
    snap = None
    if not args.no_fp64:
        snap = X.cpu() if big else X.clone()
    bounds_m = bounds
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_times = []
    eig, res, bounds, eig_first = run_steps(hm, X, m, args.steps, bounds, b, keep_first=True, times=step_times)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # phase times from further steps with per-launch events (the FFT part then runs on the
    # caller's stream instead of beside the projection, so each phase is timed alone)
    hm.reset_stats()
    hm.set_timing(True)
    run_steps(hm, X, m, args.steps, bounds, b)
    stats = hm.stats()
    hm.set_timing(False)
    ms_step = 1000.0 * dt / args.steps
    value = 1000.0 / ms_step
    band_apps = (m + 1) * nb / (ms_step / 1000.0)
    log(f"mixed: {ms_step:.1f} ms/step, max resid(occ) {res[:cell.nocc].max():.2e}")
    # H applications alone (N_b / pw_apply_h time), and the mixed block after one step from the
    # snapshot (for the subspace angle against the FP64 form)
    apply_rate = None
    density = None
    x1_mixed = None
    if not big:
        HX = torch.empty_like(X)
        hm.apply_h(X, HX)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            hm.apply_h(X, HX)
        torch.cuda.synchronize()
        apply_rate = nb * reps / (time.perf_counter() - t0)
        del HX
        # charge density of the block (doubly occupied lowest bands), timed alone
        occ = np.where(np.arange(nb) < cell.nocc, 2.0, 0.0)
        rho = hm.density(X, occ)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            hm.density(X, occ, rho)
        torch.cuda.synchronize()
        t_rho = (time.perf_counter() - t0) / reps
        density = {"ms_per_call": round(1000.0 * t_rho, 3), "bands": nb, "band_per_sec": nb / t_rho,
                   "x_read_gbs": nb * hm.npw * 8 / t_rho / 1e9,
                   "electrons": float(rho.sum().item()) / float(np.prod(hm.info.fft_n)),
                   "what": "rho(r) = sum_n f_n |psi_n(r)|^2 on the FFT grid, f = 2 for the lowest %d bands "
                           "(electrons = sum_r rho / N_r for the unnormalised transform)" % cell.nocc}
        del rho
        if snap is not None:
            x1_mixed = snap.clone()
            hm.eig_step(x1_mixed, m, bounds_m[0], bounds_m[1], b)

    # bf16 split terms executed per real product, by phase
    nterm = {}
    if mflags & 4:
        nterm["proj"] = nterm["nl"] = 3
    if mflags & 2:
        nterm["gram"] = 4
    if mflags & 8:
        nterm["rotate"] = 3
    phases, dom, roofline = phase_table(stats, hm.info, nb, m, args.steps, 4, n1a, nterm, mixed_flags=mflags)
    if roofline is not None:
        roofline["traffic"] = measured_traffic(args.workload, mflags, dom)
        if roofline["traffic"] is not None:
            roofline["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"

    # ---- LOBPCG and PPCG steps on the same cell ----------------------------------------------
    # LOBPCG: three H applications and a Rayleigh-Ritz of size 3 N_b (the kept part of the span
    # when [X R P] is numerically dependent); PPCG: three H applications of N_b columns and a
    # Rayleigh-Ritz of size N_b plus one 3 x 3 problem per column.
    lobpcg = None
    ppcg = None
    if not big and not args.no_lobpcg:
        try:
            hl = pw.Handle(cell, pw.PW_MIXED, flags=mflags | pw.PW_FLAG_LOBPCG)
            Xl = (snap if snap is not None else X).clone()
            Pl = hl.empty_block(nb)
            hl.lobpcg_step(Xl, Pl, False)
            times, kept, failures = [], [], 0
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = {}
                try:
                    el, rl = hl.lobpcg_step(Xl, Pl, True, info)
                except pw.PWError as exc:
                    failures += 1
                    log(f"lobpcg step failed: {exc}")
                    continue
                times.append(time.perf_counter() - t0)
                kept.append(info.get("kept"))
            if times:
                lobpcg = {"ms_per_step": [round(1000.0 * t, 2) for t in times],
                          "rayleigh_ritz_basis": 3 * nb, "rayleigh_ritz_kept": kept,
                          "restarts_without_directions": failures,
                          "max_resid_occ_input": float(rl[: cell.nocc].max()),
                          "what": "mixed-precision LOBPCG steps with search directions, from the filter's "
                                  "starting block after one step without them"}
                log(f"lobpcg: ms/step {lobpcg['ms_per_step']}, Rayleigh-Ritz kept {kept} of {3 * nb}")
            Xl.copy_((snap if snap is not None else X))
            hl.ppcg_step(Xl, Pl, False)
            ptimes, pres = [], None
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ep, pres = hl.ppcg_step(Xl, Pl, True)
                ptimes.append(time.perf_counter() - t0)
            ppcg = {"ms_per_step": [round(1000.0 * t, 2) for t in ptimes],
                    "max_resid_occ_input": float(pres[: cell.nocc].max()),
                    "what": "mixed-precision PPCG steps with search directions, from the filter's starting "
                            "block after one step without them"}
            log(f"ppcg: ms/step {ppcg['ms_per_step']}")
            del hl, Xl, Pl
            torch.cuda.empty_cache()
        except Exception as exc:  # a failed side measurement must not lose the headline line
            lobpcg = {"error": str(exc)}
            log(f"lobpcg/ppcg measurement failed: {exc}")

    # ---- real-space projectors (localized family): reciprocal-space GEMMs vs real space ------
    rspace = None
    if not big and not args.no_rspace and pw.plan(cell, pw.PW_MIXED).fft_n[0] == 128:
        try:
            rspace = rspace_leg(pw, synth, torch, cell, m, args.steps)
            log(f"rspace: {rspace['rspace']['ms_per_step']:.1f} vs gspace {rspace['gspace']['ms_per_step']:.1f} "
                f"ms/step, one-step |de| {rspace['max_abs_deig_occ_Ha']:.2e} Ha")
        except Exception as exc:  # a failed side measurement must not lose the headline line
            rspace = {"error": str(exc)}
            log(f"rspace measurement failed: {exc}")

    # ---- FP64 form from the same block and bounds -----------------------------------------
    fp64 = None
    accuracy = None
    info = hm.info
    del hm, X
    torch.cuda.empty_cache()
    x64_bytes = nb * ldp * 16
    fp64_flags = 0
    if pw.plan(cell, pw.PW_FP64).footprint_bytes + x64_bytes > 0.9 * dev_bytes:
        fp64_flags = pw.PW_FLAG_BETA_OTF  # projectors generated in the GEMMs (no table)
    fp64_need = pw.plan(cell, pw.PW_FP64, flags=fp64_flags).footprint_bytes + x64_bytes
    if args.no_fp64:
        pass
    elif fp64_need > 0.9 * dev_bytes:
        log(f"fp64 form skipped: needs {fp64_need / 1e9:.0f} GB")
        fp64 = {"skipped": "needs %.0f GB of device memory" % (fp64_need / 1e9)}
    else:
        hd = pw.Handle(cell, pw.PW_FP64, flags=fp64_flags)
        Xd = hd.empty_block(nb)
        chunk = 256
        for c0 in range(0, nb, chunk):
            Xd[c0:c0 + chunk].copy_(snap[c0:c0 + chunk].to("cuda", non_blocking=False))
        del snap
        steps64 = 1 if big else args.fp64_steps
        angle = None
        if not big:
            # warm the FP64 handle (solver workspace) on a copy, untimed; this is also one FP64
            # step from the snapshot, compared with the mixed one by principal angles
            Xw = Xd.clone()
            ew, _, _ = hd.eig_step(Xw, m, bounds_m[0], bounds_m[1], b)
            if x1_mixed is not None:
                # the occupied bands, extended to the end of the cluster (gaps < 1e-3 Ha) that
                # holds the last of them, so that the span is well defined
                n_eff = cell.nocc
                while n_eff < nb and ew[n_eff] - ew[n_eff - 1] < 1e-3:
                    n_eff += 1
                angle = {"rad": occupied_angle(x1_mixed, Xw, n_eff, hd.npw), "bands": n_eff}
                del x1_mixed
            del Xw
        # the largest cells take minutes per FP64 step: one step, timed per phase as it runs
        hd.reset_stats()
        hd.set_timing(big)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e64, r64, bd, e64_first = run_steps(hd, Xd, m, steps64, bounds_m, b, keep_first=True)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        if not big:
            hd.reset_stats()
            hd.set_timing(True)
            run_steps(hd, Xd, m, 1, bd, b)
        st64 = hd.stats()
        hd.set_timing(False)
        ms64 = 1000.0 * dt64 / steps64
        phase_steps64 = steps64 if big else 1
        ph64, dom64, roof64 = phase_table(st64, hd.info, nb, m, phase_steps64, 8, n1a, {}, fp64=True)
        fp64 = {"value": 1000.0 / ms64, "unit": "eig-steps/s", "ms_per_step": round(ms64, 2), "steps": steps64,
                "band_apps_per_sec": (m + 1) * nb / (ms64 / 1000.0),
                "generated_projectors": bool(fp64_flags & pw.PW_FLAG_BETA_OTF),
                "roofline": roof64, "phases": ph64}
        nocc = cell.nocc
        accuracy = {"max_abs_deig_occ_mixed_vs_fp64_Ha": float(np.abs(eig_first[:nocc] - e64_first[:nocc]).max()),
                    "max_principal_angle_occ": angle,
                    "bands_compared": nocc, "what": "first timed degree-%d step of each form, same block and bounds" % m}
        del hd, Xd
        torch.cuda.empty_cache()
        log(f"fp64: {ms64:.1f} ms/step; one-step |de| mixed vs fp64 = {accuracy['max_abs_deig_occ_mixed_vs_fp64_Ha']:.2e}")

    accuracy_converged = None
    if args.accuracy_workload != "none":
        try:
            accuracy_converged = accuracy_at_convergence(pw, synth, torch, args.accuracy_workload, mflags, m)
            a = accuracy_converged
            log(f"accuracy at convergence ({a['workload']}): |de| {a['max_abs_deig_occ_mixed_vs_fp64_Ha']:.2e} Ha, "
                f"max cluster angle {a['max_cluster_angle_rad']:.2e} (bound {a['max_davis_kahan_bound']:.2e}); "
                f"after FP64 polish ({a['polish']['fp64_steps']} steps vs {a['fp64']['steps']}): "
                f"|de| {a['polish']['max_abs_deig_occ_Ha']:.2e}, angle {a['polish']['max_cluster_angle_rad']:.2e}")
        except Exception as exc:  # a failed side measurement must not lose the headline line
            accuracy_converged = {"error": str(exc)}
            log(f"accuracy study failed: {exc}")

    serving = None
    if args.serving_requests > 0:
        serving = serving_leg(args.serving_requests, args.serving_rate, args.serving_slots, mflags, m)
        log(f"serving: p50 {serving['p50_latency_s']:.3f}s p99 {serving['p99_latency_s']:.3f}s "
            f"throughput {serving['throughput_req_s']:.2f} req/s, converged {serving['converged']}/{serving['requests']}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cell, nb, m)
        log(f"cpu baseline: {cpu['extrapolated_step_s']:.1f} s/step (extrapolated), {cpu['cores']} cores")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "eig-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": round(1000.0 * float(np.median(step_times)), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+bf16x3" if mflags & (pw.PW_FLAG_BF16_ALL) else "c64",
        "dtype_note": "complex FP32 data and FFTs; projector, rotation and Gram products as split-bf16 MFMA "
                      "(3 and 4 terms, FP32 accumulation, FP64 split-K sums) per the flags; FP64 eigensolve and "
                      "residual norms",
        "data": "synthetic",
        "config": {"workload": f"{args.workload.capitalize()}: {cell.natoms} Si atoms ({'x'.join(str(int(round(L / synth.A0_BOHR))) for L in cell.L)} diamond cells, a=10.26 bohr), "
                               f"Ecut {cell.ecut:g} Ha, Gamma point, {G.shape[0]} plane waves, {nb} bands, "
                               f"degree-{m} Chebyshev-filtered Rayleigh-Ritz step, mixed precision",
                   "npw": int(G.shape[0]), "nbands": nb, "degree": m, "ecut_ha": cell.ecut,
                   "fft_grid": list(int(x) for x in pw.plan(cell, pw.PW_MIXED).fft_n), "precision": "mixed",
                   "mixed_flags": mflags},
        "band_apps_per_sec": band_apps,
        "apply_h_band_apps_per_sec": apply_rate,
        "density": density,
        "lobpcg": lobpcg, "ppcg": ppcg, "rspace_projectors": rspace,
        "device": device_info(torch, minfo),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": fp64,
        "accuracy": accuracy,
        "accuracy_converged": accuracy_converged,
        "phases": phases,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
