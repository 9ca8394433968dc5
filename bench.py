#!/usr/bin/env python3
"""Benchmark of the domain-wall multigrid hot path on one MI355X.

Metric: MG-preconditioned domain-wall solves per second to a true FP64
relative residual of 1e-10 on a 256^2 x Ls 16 lattice (beta 6, m_f 0.01,
M5 = -1) with the 2-level hierarchy (4x4 aggregates, 16 null vectors, coarse
Ls 2), mixed precision (FP32 fine level, BF16 coarse links on the matrix
cores, FP64 coarsest Krylov vectors, FP64 outer defect correction).  The
coarsest level runs restarted GCR(6) on hat-A to 0.5 by default.  Rows beside
the headline: the paper's parameter table throughout (coarse Ls 4, coarsest
CGNR to 0.05), coarse Ls 4 with GCR, three levels, 8 null vectors.

A step is one full solve (K-cycle preconditioned flexible GCR inside the FP64
defect correction) of one right-hand side already resident in HBM.  The
hierarchy setup is done once before timing and reported separately.  Beside
the headline: 16 right-hand sides in one solve, the three-level hierarchy,
the plain FP64 solve of the same algorithm, the fine-stencil bandwidth rows
and the oracle on the host.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0   # dense matrix-core BF16 peak of MI355X
METRIC = "DWF solves/s to 1e-10 at 256\u00b2\u00d7Ls16, mixed vs FP64; D_dw stencil HBM GB/s"

WORKLOADS = {
    # metric workload: 256^2 x 16, 2-level 4x4 aggregates with 16 null vectors, coarse Ls 2
    "dwf256_ls16_mg2": dict(L=256, Ls=16, beta=6.0, sweeps=200, m=0.01, M5=-1.0, cfg=6, gauge_cfg=4,
                            nvec=[16], block=[(4, 4)], Ls_coarse=[2]),
    # same lattice, the three-level aggregation of the paper's parameter table, coarse Ls 2
    "dwf256_ls16_mg3": dict(L=256, Ls=16, beta=6.0, sweeps=200, m=0.01, M5=-1.0, cfg=6, gauge_cfg=4,
                            nvec=[8, 12], block=[(4, 4), (2, 2)], Ls_coarse=[2, 2]),
    # 128^2 x 16 precision form
    "dwf128_ls16_mg2": dict(L=128, Ls=16, beta=6.0, sweeps=200, m=0.01, M5=-1.0, cfg=2, gauge_cfg=2,
                            nvec=[16], block=[(4, 4)], Ls_coarse=[4]),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_params(dwfmg, wl, mixed, nev=0, m_setup=None, setup_iters=None, coarsest_f32=False, **eig):
    n = len(wl["nvec"])
    if mixed:
        link = [dwfmg.P_BF16] * n
        # FP32 Krylov vectors on the intermediate levels, FP64 on the coarsest (its solve is
        # kept in FP64); coarsest_f32 (a reported variant) puts the coarsest in FP32 too
        vec = [dwfmg.P_F32] * (n - 1) + [dwfmg.P_F32 if coarsest_f32 else dwfmg.P_F64]
        fine = dwfmg.P_F32
    else:
        link = [dwfmg.P_F64] * n
        vec = [dwfmg.P_F64] * n
        fine = dwfmg.P_F64
    extra = {}
    if m_setup is not None:
        extra["m_setup"] = m_setup
    if setup_iters is not None:
        extra["setup_iters"] = setup_iters
    return dwfmg.MGParams(nvec=list(wl["nvec"]), block=list(wl["block"]), Ls_coarse=list(wl["Ls_coarse"]),
                          link_prec=link, vec_prec=vec, fine_prec=fine, coarsest_nev=nev, **extra, **eig)


def null_starts(inputs, wl, torch):
    starts = []
    L, n = wl["L"], 2
    for l, nv in enumerate(wl["nvec"]):
        starts.append(torch.from_numpy(inputs.gaussian_field((nv, L, L, n), inputs.null_start_seed(wl["cfg"], l))).cuda())
        L //= wl["block"][l][0]
        n = 2 * nv
    return starts


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(kernel_src, algorithmic_bytes, summary="coarse_stencil_traffic.json"):
    """HBM traffic per launch of a kernel from its committed rocprofv3 counter
    summary, or None when the kernel source or the launch shape changed since
    it was taken."""
    p = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_sha256_16") != source_hash(kernel_src) or d.get("algorithmic_bytes") != algorithmic_bytes:
        return None
    return d.get("bytes_per_launch")


def _oracle_unit_costs(O, inputs, U_np, L, Ls, m, M5, nv, block, Lsc):
    """Seconds of one oracle D_DW apply on the fine lattice and one on the coarse
    lattice of a hierarchy of this shape (prolongator from Gaussian vectors)."""
    psi = inputs.gaussian_field((Ls, L, L, 2), 1)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        O.dwf(U_np, psi, m, M5)
    t_fine = (time.perf_counter() - t0) / reps
    bx, by = block
    V = inputs.gaussian_field((L, L, 2, 1, nv), 2)
    P = O.Prolongator(V=O.block_orthonormalize(V, (by, bx)), block=(by, bx))
    S = O.galerkin(O.wilson_stencil(U_np), P)
    ec = inputs.gaussian_field((Lsc, L // by, L // bx, 2 * nv), 3)
    t0 = time.perf_counter()
    for _ in range(reps):
        O.stencil_dwf(S, ec, m, M5)
    t_coarse = (time.perf_counter() - t0) / reps
    return t_fine, t_coarse


def cpu_baseline(wl, stats, U_np, coarsest):
    """The oracle, untuned, on the host.

    A whole oracle solve at the metric size does not fit a bounded sample (its
    setup alone relaxes 16 null vectors for 250 CG steps at 256^2), so the
    figure is a calibrated model:
      1. a real oracle multigrid solve, timed end to end (setup excluded, as on
         the GPU), at 32^2 x Ls 8 (beta 6, m 0.01; 4x4 aggregates, 8 null
         vectors, coarse Ls 4, the paper's K-cycle with coarsest CGNR), with its
         fine and coarse D_DW applications counted;
      2. the model (applications x the oracle's unit cost per application) at
         that size, and the ratio actual / model (the vector algebra and the
         interpreter overhead the model leaves out);
      3. at the metric size: the GPU solve's application counts x the oracle's
         unit costs at 256^2 x 16 (fine) and 64^2 x 2 x 32 dof (coarse), times
         that ratio.
    Steps 1-3 run with the host's default thread pool and again on one thread."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import dwf_oracle as O
    from paper_2004_07732_amd import inputs

    if len(wl["nvec"]) != 1:
        return None
    L, Ls, m, M5 = wl["L"], wl["Ls"], wl["m"], wl["M5"]
    nv, block, Lsc = wl["nvec"][0], wl["block"][0], wl["Ls_coarse"][0]
    # the GPU solve's counts: fine D_DW-type applications, coarse D_DW-type applications
    # (one coarsest GCR iteration applies A-hat = D_PV-hat^dag D_DW-hat: two; CGNR: four, plus
    # one A-hat^dag per call)
    fine_D = float(stats.fine_applies)
    if coarsest["coarsest_solver"] == 0:
        coarse_D = 4.0 * stats.level_iters[0] + 2.0 * stats.level_calls[0]
    else:
        coarse_D = 2.0 * stats.level_iters[0]
    # calibration problem (config 1 of the scope table)
    Lc, Lsc1, mc = 32, 8, 0.01
    gc = inputs.metropolis_u1(Lc, Lc, 6.0, 200, inputs.gauge_seed(1, Lc))
    bc = inputs.gaussian_field((Lsc1, Lc, Lc, 2), inputs.rhs_seed(1, Lc, 0))
    startc = [inputs.gaussian_field((8, Lc, Lc, 2), inputs.null_start_seed(1, 0))]

    def run(threads):
        lim = {} if threads is None else {"limits": threads}
        with threadpool_limits(**lim):
            used = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
            mg = O.MG(gc.U, Lsc1, mc, M5, O.MGParams(levels=[O.LevelParams(nvec=8, block=(4, 4), Ls=4)]), startc)
            counts = {"fine": 0, "coarse": 0}
            dwf0, sdwf0 = O.dwf, O.stencil_dwf

            def dwf_c(*a, **k):
                counts["fine"] += 1
                return dwf0(*a, **k)

            def sdwf_c(*a, **k):
                counts["coarse"] += 1
                return sdwf0(*a, **k)
            O.dwf, O.stencil_dwf = dwf_c, sdwf_c
            try:
                t0 = time.perf_counter()
                xc, _ = mg.solve(bc, 1e-10)
                t_actual = time.perf_counter() - t0
            finally:
                O.dwf, O.stencil_dwf = dwf0, sdwf0
            res = float(np.linalg.norm(bc - O.dwf(gc.U, xc, mc, M5)) / np.linalg.norm(bc))
            tf1, tc1 = _oracle_unit_costs(O, inputs, gc.U, Lc, Lsc1, mc, M5, 8, (4, 4), 4)
            model1 = counts["fine"] * tf1 + counts["coarse"] * tc1
            ratio = t_actual / model1
            tf, tc = _oracle_unit_costs(O, inputs, U_np, L, Ls, m, M5, nv, block, Lsc)
            t_solve = (fine_D * tf + coarse_D * tc) * ratio
            return {"threads": used, "solves_per_s": 1.0 / t_solve, "t_solve_s": t_solve,
                    "calibration": {"actual_s": t_actual, "model_s": model1, "ratio": ratio, "residual": res,
                                    "fine_applies": counts["fine"], "coarse_applies": counts["coarse"]},
                    "unit_s": {"fine_dw": tf, "coarse_dw": tc}}

    all_threads = run(None)
    one_thread = run(1)
    d_bytes = 2 * Ls * L * L * 2 * 16 + 2 * L * L * 16
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    a = all_threads
    return {"value": a["solves_per_s"], "unit": "solves/s", "cores": a["threads"], "kind": "oracle",
            "cpu_model": cpu_model, "host_cpus": os.cpu_count(),
            "oracle_dw_GB_s": d_bytes / a["unit_s"]["fine_dw"] / 1e9,
            "one_thread": {"value": one_thread["solves_per_s"], "calibration": one_thread["calibration"]},
            "calibration": a["calibration"], "unit_s": a["unit_s"],
            "sample": (f"a real oracle MG solve at 32^2 x 8 (4x4 aggregates, 8 null vectors, coarse Ls 4, "
                       f"coarsest CGNR) took {a['calibration']['actual_s']:.2f} s = "
                       f"{a['calibration']['ratio']:.2f} x its application model; at {L}^2 x {Ls}: "
                       f"{fine_D:.0f} fine and {coarse_D:.0f} coarse D_DW applications of the GPU solve x the "
                       f"oracle's unit costs ({a['unit_s']['fine_dw']:.3f} s, {a['unit_s']['coarse_dw']:.4f} s) "
                       f"x that ratio = {a['t_solve_s']:.0f} s per solve")}


def coarse_stencil_bytes(nsites, n, Ls_c, ncol, link_bytes, vec_bytes, link_blocks=5):
    """Algorithmic bytes of one coarse D_DW launch: per coarse site the five
    (2 nvec)^2 link blocks of the stencil (site term and four hops) once, and
    every vector entry read once and written once.  With link_blocks = 3: the
    bytes the kernel stores and reads from memory (the site term and the two
    forward hops; the backward hops are the sigma_3-adjoints of the neighbours'
    forward hops, re-read through the caches)."""
    return nsites * (link_blocks * n * n * link_bytes + 2 * Ls_c * ncol * n * vec_bytes)


def coarse_a_bytes(launch_bytes, nsites, n, Ls_c, ncol, vec_bytes):
    """Algorithmic bytes of one coarse A-hat = D_PV-hat^dag D_DW-hat: two stencil
    launches of `launch_bytes` each, less what the narrower intermediate saves: with
    FP64 vectors (16 B complex) the D_DW-hat output is written and read back as FP32
    (8 B complex), which the stencil's FP32 accumulation makes exact."""
    return 2 * launch_bytes - 2 * nsites * Ls_c * ncol * n * (vec_bytes - 8)


def coarse_mfma_per_launch(nsites, n, Ls_c, ncol, tw=None):
    """Matrix-core products (16x16x32, BF16) one coarse launch issues.  A wave owns
    16 output rows of one site and a tile of up to TW (slice, column) pairs (TW = 2,
    4 or 8; by default the heuristic one for Ls_c * ncol; several tiles only at
    TW = 8, whichever workgroups take them); per tile it issues one product per 16
    complex inner entries of the five blocks and per half (hi, lo) of the split
    vector."""
    C = Ls_c * ncol
    if tw is None:
        tw = 2 if C <= 2 else (4 if C <= 4 else 8)
    ntile = 1 if tw < 8 else -(-C // 8)
    return nsites * (n // 16) * ntile * 2 * (5 * n // 16)


GRAM_STEPS = 6   # longest smoother cycle the library runs in the Gram form


def smoother_model_passes(ns, ks):
    """Fine-vector passes of one post-smoothing call.
    Gram form (cycles of at most GRAM_STEPS steps): the initial residual straight into the
    first direction (subtract: 3, norm: 1); per step j < kc - 1 of a cycle the multi-dot
    (j + 2) and the next direction (j + 2 read, 1 written); the cycle's last step the
    multi-dot (kc + 1) and the pass that updates z and the starting residual (2 kc + 1
    read, 2 written): kc^2 + 5 kc + 1 per cycle.
    Orthogonalising form: the initial residual (subtract: 3, copy: 2, norm: 1); per step
    the multi-dot (j + 2) and the fused update (j + 2 read; w and r written, and the next
    direction except after the cycle's last step); per cycle the solution update
    (kc + 2), with the restart copy (2 more) on every cycle but the last."""
    if ns <= 0:
        return 0
    ks = ks if 0 < ks < ns else ns
    gram = ks <= GRAM_STEPS
    passes, done = (4 if gram else 6), 0
    while done < ns:
        kc = min(ks, ns - done)
        if gram:
            passes += kc * kc + 5 * kc + 1
        else:
            passes += kc * kc + 6 * kc - 1 + kc + 2
        done += kc
        if done < ns and not gram:
            passes += 2
    return passes


def solve_model_bytes(fine_applies, coarse_iters, k, L, Ls, coarse_a, coarse_vec_bytes,
                      kcycles=0, smooth_iters=0, smooth_restart=0):
    """HBM bytes of one solve by a model (a lower bound): the fine FP32 stencils
    (vector read and written, links once per apply), one coarse A-hat per coarsest
    iteration (`coarse_a` bytes, coarse_a_bytes), the coarsest GCR(k)
    vector algebra per restart cycle of k iterations and, for `kcycles` K-cycles,
    the post-smoother's FP32 vector algebra (smoother_model_passes).  The coarsest
    cycle: in the Gram form (k <= GRAM_STEPS) the multi-dot (j + 2) and the next
    direction (j + 3) at each step but the last, whose multi-dot (k + 1) is followed
    by the pass that updates x and the starting residual (2 k + 3): k^2 + 5 k + 1
    passes; in the orthogonalising form the multi-dot (j + 2) and the fused update
    (j + 2 read, 3 written, 2 after the last direction), then the solution update
    and restart (k + 4): k^2 + 7 k + 3.  The outer flexible GCR's vector algebra is
    not counted."""
    fine_apply = 2 * Ls * L * L * 2 * 8 + 2 * L * L * 8
    fine_vec = Ls * L * L * 2 * 8
    cycle = k * k + 5 * k + 1 if k <= GRAM_STEPS else k * k + 7 * k + 3
    return (fine_applies * fine_apply + coarse_iters * coarse_a
            + coarse_iters * cycle / k * coarse_vec_bytes
            + kcycles * smoother_model_passes(smooth_iters, smooth_restart) * fine_vec)


def timed(mg, b, steps, warmup, tol=1e-10):
    """Seconds per solve over `steps` solves after `warmup` untimed ones: the
    mean over the whole bracketed interval and the median of the per-solve
    times (each solve is synchronous: it returns after the true residual is
    known).  Returns (mean, median, stats, x)."""
    import statistics

    import torch
    st = x = None
    for _ in range(warmup):
        x, st = mg.solve(b, tol)
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        x, st = mg.solve(b, tol)
        times.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    mean = (time.perf_counter() - t0) / max(steps, 1)
    return mean, statistics.median(times), st, x


ROW_SAMPLES = 5   # timed solves per row beside the headline (median reported)


def stats_dict(st):
    return {"residual": st.true_rel_residual, "outer_steps": st.outer_steps, "fine_iters": st.fine_iters,
            "fine_applies": st.fine_applies, "coarse_iters": st.level_iters, "coarse_calls": st.level_calls}


# the HBM-bound fine stencil shape: 512^2 x Ls 32 x 4 rhs, FP32 (about 1.08 GB per apply)
FINE_HBM_SHAPE = (512, 32, 4)


def stencil_rows(dwfmg, inputs, torch, m, M5):
    """Fine D_DW bandwidth: (ii) 512^2 x 32 x 4 rhs FP32 (about 1.08 GB per apply,
    far above the 256 MB last-level cache) is the HBM figure; (i) 256^2 x 16
    one rhs FP32 / FP64 and (iii) 256^2 x 16 x 16 rhs FP32 beside it; and the
    bandwidth of a plain 2 GiB device copy as the measured peak.  Each figure is
    50 back-to-back applies replayed from one HIP graph, timed with events."""
    def one(L, Ls, nr, dtype, seed):
        U = torch.from_numpy(inputs.links_from_theta(inputs.random_theta(L, L, seed))).cuda().to(dtype)
        psi = torch.randn((nr, Ls, L, L, 2), dtype=dtype, device="cuda")
        out = torch.empty_like(psi)
        for _ in range(3):   # the first call times the launch configurations
            dwfmg.dwf_apply(U, psi, m, M5, out=out)
        torch.cuda.synchronize()
        # the applies are replayed from a HIP graph, so that host launch overhead
        # (larger than the kernel at the one-rhs 256^2 shape) is not timed
        reps = 50
        graph, cap = torch.cuda.CUDAGraph(), torch.cuda.Stream()
        with torch.cuda.graph(graph, stream=cap):
            for _ in range(reps):
                dwfmg.dwf_apply(U, psi, m, M5, out=out)
        graph.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        t_ms = e0.elapsed_time(e1) / reps
        del graph
        esz = psi.element_size()
        sbytes = 2 * psi.numel() * esz + U.numel() * esz
        return {"shape": f"{L}^2 x {Ls} x {nr} rhs", "dtype": str(dtype).replace("torch.", ""), "us": t_ms * 1e3,
                "bytes": sbytes, "GB_s": sbytes / (t_ms * 1e-3) / 1e9}
    rows = {"ii_hbm": one(*FINE_HBM_SHAPE, torch.complex64, 8_000_000),
            "i_fp32": one(256, 16, 1, torch.complex64, 8_000_001),
            "i_fp64": one(256, 16, 1, torch.complex128, 8_000_002),
            "iii_fp32_16rhs": one(256, 16, 16, torch.complex64, 8_000_003)}
    # measured copy bandwidth: the library's streaming copy kernel over 2 GiB (read 2 GiB +
    # write 2 GiB), median of five runs of ten copies
    copy_gbs = sorted(dwfmg.copy_bandwidth(2 ** 31, 10) for _ in range(5))[2]
    torch.cuda.empty_cache()
    for r in rows.values():
        r["frac_nominal"] = r["GB_s"] / PEAK_HBM_GBS
        r["frac_measured_copy"] = r["GB_s"] / copy_gbs
    rows["copy_2GiB_GB_s"] = copy_gbs
    rows["ii_hbm"]["traffic"] = stored_traffic(
        os.path.join(ROOT, "paper_2004_07732_amd", "csrc", "fine_stencil.hip"), rows["ii_hbm"]["bytes"],
        "fine_stencil_traffic.json")
    return rows


def fine_a_rows(dwfmg, inputs, torch, mg, L, Ls):
    """Level-0 A = D_PV^dag D_DW of the headline hierarchy (FP32) for 1 and 16 columns:
    HIP-event time per application (median of three runs of 100) with the two stencil
    launches pinned and with each fused tile shape at each chunk length the timed choice
    considers; algorithmic bytes of A as one operator (psi read once, out written once, the
    links once)."""
    out = {}
    for ncol in (1, 16):
        x = torch.from_numpy(inputs.gaussian_field((ncol, Ls, L, L, 2), 9_000_000 + ncol)).cuda()
        def t_of(shape, chunk):
            dwfmg.dwf_fine_a_config(shape, chunk)
            return sorted(mg.time_op(0, dwfmg.MG_OP_A, x, ncol, iters=100) for _ in range(3))[1] * 1e3
        try:
            two = t_of(dwfmg.FINE_A_TWO, 1)
            fused = min((t_of(sh, c), sh, c) for sh in (dwfmg.FINE_A_16x16, dwfmg.FINE_A_32x8, dwfmg.FINE_A_16x8)
                        for c in sorted({Ls, (Ls + 1) // 2, (Ls + 3) // 4, 4, 2}))
        finally:
            dwfmg.dwf_fine_a_config(dwfmg.FINE_A_AUTO)
        nbytes = ncol * Ls * L * L * 32 + 2 * L * L * 8
        out[f"{ncol}rhs"] = {"shape": f"{L}^2 x {Ls} x {ncol} rhs", "dtype": "complex64", "bytes": nbytes,
                            "two_launch_us": two, "fused_us": fused[0], "fused_tile": ["16x16", "32x8", "16x8"][fused[1] - 1],
                            "fused_chunk": fused[2], "two_launch_GB_s": nbytes / (two * 1e-6) / 1e9,
                            "fused_GB_s": nbytes / (fused[0] * 1e-6) / 1e9,
                            "chosen": "fused" if fused[0] * 1.03 < two else "two launches"}
        log(f"[bench] fine A {ncol} rhs: two launches {two:.1f} us, fused {fused[0]:.1f} us "
            f"({out[f'{ncol}rhs']['fused_tile']}, chunk {fused[2]})")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dwf256_ls16_mg2", choices=sorted(WORKLOADS))
    ap.add_argument("--coarsest", choices=["cgnr", "gcr"], default="gcr",
                    help="coarsest-level solver: restarted GCR on A (default) or CGNR on A^dag A as in the paper")
    ap.add_argument("--coarsest-restart", type=int, default=6)
    ap.add_argument("--coarsest-tol", type=float, default=None,
                    help="coarsest relative tolerance (default 0.25 with GCR, 0.05 with CGNR)")
    ap.add_argument("--nev", type=int, default=0,
                    help="deflate the coarsest CGNR with this many eigenvectors of its normal operator")
    ap.add_argument("--eig-degree", type=int, default=None, help="Chebyshev degree of the Lanczos acceleration")
    ap.add_argument("--eig-maxit", type=int, default=None)
    ap.add_argument("--eig-tol", type=float, default=None)
    ap.add_argument("--m-setup", type=float, default=None, help="mass of the setup relaxation's Wilson kernel")
    ap.add_argument("--setup-iters", type=int, default=None, help="CG iterations per null vector (max)")
    ap.add_argument("--smooth-iters", type=int, default=20,
                    help="post-smoothing GCR steps per K-cycle (default 20; the paper's parameter table has 8)")
    ap.add_argument("--smooth-restart", type=int, default=5,
                    help="restart length of the post-smoothing GCR (default 5; 0: none, the paper's smoother)")
    ap.add_argument("--nvec", type=int, nargs="+", default=None, help="override the workload's null vectors per level")
    ap.add_argument("--ls-coarse", type=int, nargs="+", default=None, help="override the coarse Ls per level")
    ap.add_argument("--fine-a", choices=["auto", "two", "fused"], default="auto",
                    help="the solver's fine A: timed choice (default), the two stencil launches, or the fused launch "
                         "(16x16 tiles, chunk Ls); a profiler's per-launch overhead can tip the timed choice, so "
                         "profiled runs pin the choice the unprofiled benchmark makes")
    ap.add_argument("--quick", action="store_true", help="only the headline solve and its roofline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stencil", action="store_true", help="skip the fine-stencil bandwidth rows")
    ap.add_argument("--counters", nargs="?", const="coarse", choices=["coarse", "coarse16", "fine"], default=None,
                    help="only run one kernel (21 launches: the dominant coarse stencil; with 'coarse16' the "
                         "same stencil on 16 right-hand sides; with 'fine' the fine stencil at 512^2 x 32 x 4 rhs "
                         "FP32 in a fixed launch configuration) next to a plain 256 MiB copy, for rocprofv3 --pmc "
                         "runs; prints no benchmark line")
    args = ap.parse_args()

    if args.counters:
        # the counter runs time one fixed launch configuration: no tuning dispatches
        os.environ["DWF_AUTOTUNE"] = "0"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the library has no "
              f"multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2004_07732_amd import dwfmg, inputs

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.fine_a == "two":
        dwfmg.dwf_fine_a_config(dwfmg.FINE_A_TWO)
    elif args.fine_a == "fused":
        dwfmg.dwf_fine_a_config(dwfmg.FINE_A_16x16, 4096 - 1)
    wl = dict(WORKLOADS[args.workload])
    if args.nvec:
        wl["nvec"] = list(args.nvec)
    if args.ls_coarse:
        wl["Ls_coarse"] = list(args.ls_coarse)
    L, Ls, m, M5 = wl["L"], wl["Ls"], wl["m"], wl["M5"]
    log(f"[bench] workload {args.workload}: generating gauge field {L}^2 beta {wl['beta']}")
    g = inputs.metropolis_u1(L, L, wl["beta"], wl["sweeps"], inputs.gauge_seed(wl["gauge_cfg"], L))
    U = torch.from_numpy(g.U).cuda()
    b = torch.from_numpy(inputs.gaussian_field((1, Ls, L, L, 2), inputs.rhs_seed(wl["cfg"], L, 0))).cuda()
    starts = null_starts(inputs, wl, torch)

    def coarsest(kind, tol=None):
        d = {"coarsest_solver": dwfmg.COARSEST_GCR if kind == "gcr" else dwfmg.COARSEST_CGNR,
             "coarsest_restart": args.coarsest_restart}
        d["coarsest_tol"] = tol if tol is not None else (0.5 if kind == "gcr" else 0.05)
        return d

    head = coarsest(args.coarsest, args.coarsest_tol)
    if args.m_setup is not None:
        head["m_setup"] = args.m_setup
    if args.setup_iters is not None:
        head["setup_iters"] = args.setup_iters
    head["smooth_iters"] = args.smooth_iters
    head["smooth_restart"] = args.smooth_restart
    for k, v in (("eig_degree", args.eig_degree), ("eig_maxit", args.eig_maxit), ("eig_tol", args.eig_tol)):
        if v is not None:
            head[k] = v

    if args.counters == "fine":
        Lf, Lsf, nrf = FINE_HBM_SHAPE
        Uf = torch.from_numpy(inputs.links_from_theta(inputs.random_theta(Lf, Lf, 8_000_000))).cuda()
        Uf = Uf.to(torch.complex64)
        psi = torch.randn((nrf, Lsf, Lf, Lf, 2), dtype=torch.complex64, device="cuda")
        out = torch.empty_like(psi)
        # one fixed configuration (64 x 8 tiles, 8 slices per thread; among the tuner's
        # equally fast choices at this shape) so that separate profiler runs see the same kernel
        dwfmg.dwf_fine_config(dwfmg.FINE_TILE_64x8, 8)
        dwfmg.dwf_apply(Uf, psi, m, M5, out=out)
        torch.cuda.synchronize()
        log("[bench] fine stencil: 21 launches follow")
        for _ in range(21):
            dwfmg.dwf_apply(Uf, psi, m, M5, out=out)
        a = torch.ones(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        bcopy = torch.empty_like(a)
        for _ in range(5):
            bcopy.copy_(a)
        torch.cuda.synchronize()
        log("[bench] counters run done: 21 fine stencil launches, 5 copies of 256 MiB")
        return

    if args.counters:
        nc = 16 if args.counters == "coarse16" else 1
        mg = dwfmg.MG(U, Ls, m, M5, make_params(dwfmg, wl, True, **head), starts, max_nrhs=nc)
        c = mg.info(1)
        xin = torch.from_numpy(inputs.gaussian_field((nc, c["Ls"], c["Ly"], c["Lx"], c["n"]), 5)).cuda()
        mg.time_op(1, dwfmg.MG_OP_DW, xin, nc, iters=20)
        a = torch.ones(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        bcopy = torch.empty_like(a)
        for _ in range(5):
            bcopy.copy_(a)
        torch.cuda.synchronize()
        tw, tpb = mg.coarse_config(1, nc)
        log(f"[bench] counters run done: 21 coarse launches on {nc} rhs (tile width {tw}, {tpb} tiles per "
            f"workgroup), 5 copies of 256 MiB")
        return

    # ---------------------------------------------------------------- headline: mixed precision, 1 rhs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = dwfmg.MG(U, Ls, m, M5, make_params(dwfmg, wl, True, args.nev, **head), starts,
                  max_nrhs=1 if args.quick else 16)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.2f} s")
    if args.nev:
        di = mg.deflation_info()
        log(f"[bench] deflation: nev {di['nev']}, {di['iters']} Lanczos steps, worst residual "
            f"{di['worst_residual']:.1e}, lambda {di['lambdas'][0]:.3e} .. {di['lambdas'][-1]:.3e}")
    t_step, t_median, stats, x_head = timed(mg, b, args.steps, args.warmup)
    mixed_sps = 1.0 / t_step
    log(f"[bench] headline: {t_step * 1e3:.1f} ms/solve (median {t_median * 1e3:.1f}), residual "
        f"{stats.true_rel_residual:.2e}, fine iters {stats.fine_iters}, coarse iters {stats.level_iters} "
        f"calls {stats.level_calls}")
    # the last timed solution's true residual, recomputed by the oracle's FP64 operator
    oracle_residual = None
    if not args.no_cpu_baseline:
        from oracle import dwf_oracle as O
        bn, xn = b[0].cpu().numpy(), x_head[0].cpu().numpy()
        oracle_residual = float(np.linalg.norm(bn - O.dwf(g.U, xn, m, M5)) / np.linalg.norm(bn))
        log(f"[bench] headline residual recomputed by the oracle: {oracle_residual:.2e}")

    # ---------------------------------------------------------------- dominant kernel: coarse stencil
    c = mg.info(1)
    xin = torch.from_numpy(inputs.gaussian_field((1, c["Ls"], c["Ly"], c["Lx"], c["n"]), 5)).cuda()
    # median of five runs of 200 back-to-back launches (HIP events on the stream they run on)
    t_coarse_ms = sorted(mg.time_op(1, dwfmg.MG_OP_DW, xin, 1, iters=200) for _ in range(5))[2]
    n, nsites, Lsc = c["n"], c["Lx"] * c["Ly"], c["Ls"]
    link_bytes = 4  # bfloat16 complex
    vec_bytes = 16 if make_params(dwfmg, wl, True, args.nev).vec_prec[0] == dwfmg.P_F64 else 8
    coarse_bytes = coarse_stencil_bytes(nsites, n, Lsc, 1, link_bytes, vec_bytes)
    stored_bytes = coarse_stencil_bytes(nsites, n, Lsc, 1, link_bytes, vec_bytes, link_blocks=3)
    achieved = coarse_bytes / (t_coarse_ms * 1e-3) / 1e9
    traffic = stored_traffic(os.path.join(ROOT, "paper_2004_07732_amd", "csrc", "coarse_mfma.hip"), stored_bytes)
    log(f"[bench] coarse stencil {t_coarse_ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic (5 link blocks), "
        f"{stored_bytes / (t_coarse_ms * 1e-3) / 1e9:.0f} GB/s on the 3 stored blocks")
    # the coarse A = D_PV-hat^dag D_DW-hat as the solve applies it (with FP64 vectors its
    # intermediate in FP32): median of five runs of 200 applications
    t_a_ms = sorted(mg.time_op(1, dwfmg.MG_OP_A, xin, 1, iters=200) for _ in range(5))[2]
    a_bytes = coarse_a_bytes(coarse_bytes, nsites, n, Lsc, 1, vec_bytes)
    a_stored = coarse_a_bytes(stored_bytes, nsites, n, Lsc, 1, vec_bytes)
    coarse_a = {"us_per_application": t_a_ms * 1e3, "launches": 2, "algorithmic_bytes": a_bytes,
                "GB_s": a_bytes / (t_a_ms * 1e-3) / 1e9, "frac": a_bytes / (t_a_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                "stored_bytes": a_stored,
                "frac_stored_bytes": a_stored / (t_a_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    log(f"[bench] coarse A {t_a_ms * 1e3:.1f} us per application (two launches), "
        f"{coarse_a['GB_s']:.0f} GB/s algorithmic = {coarse_a['frac']:.3f}")
    tw, tpb = mg.coarse_config(1, 1)
    mfma_per_launch = coarse_mfma_per_launch(nsites, n, Lsc, 1, tw)
    issued_tf = mfma_per_launch * 16 * 16 * 32 * 2 / (t_coarse_ms * 1e-3) / 1e12
    useful_tf = nsites * Lsc * 5 * n * n * 8 / (t_coarse_ms * 1e-3) / 1e12
    coarse_mfma = {"tile_width": tw, "tiles_per_workgroup": tpb, "mfma_per_launch": mfma_per_launch,
                   "issued_TFLOP_s": issued_tf,
                   "algorithmic_TFLOP_s": useful_tf, "peak_bf16_TFLOP_s": PEAK_BF16_TFLOPS,
                   "frac_issued": issued_tf / PEAK_BF16_TFLOPS, "frac_algorithmic": useful_tf / PEAK_BF16_TFLOPS}
    solve_bytes = (solve_model_bytes(stats.fine_applies, stats.level_iters[0], args.coarsest_restart, L, Ls,
                                     coarse_a_bytes(coarse_bytes, nsites, n, Lsc, 1, vec_bytes),
                                     nsites * Lsc * n * vec_bytes, kcycles=stats.level_calls[0],
                                     smooth_iters=args.smooth_iters, smooth_restart=args.smooth_restart)
                   if args.coarsest == "gcr" and len(wl["nvec"]) == 1 else None)
    solve_roofline = None
    if solve_bytes is not None:
        gbs = solve_bytes / t_step / 1e9
        solve_roofline = {"bound": "hbm", "model_bytes": solve_bytes, "achieved": gbs, "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "lower_bound": True}
        log(f"[bench] coarse matrix cores {issued_tf:.0f} TFLOP/s issued ({issued_tf / PEAK_BF16_TFLOPS:.3f}); "
            f"whole solve {solve_bytes / 1e9:.0f} GB modelled, {gbs:.0f} GB/s = {gbs / PEAK_HBM_GBS:.3f}")

    rows = {}
    if not args.quick:
        # 16 right-hand sides in one solve on the same hierarchy
        b16 = torch.from_numpy(np.stack([inputs.gaussian_field((Ls, L, L, 2), inputs.rhs_seed(wl["cfg"], L, j))
                                         for j in range(16)])).cuda()
        _, t16, st16, _ = timed(mg, b16, ROW_SAMPLES, 1)
        rows["batched_16rhs"] = {"solves_per_s": 16.0 / t16, "ms_per_batch": t16 * 1e3, "samples": ROW_SAMPLES,
                                 **stats_dict(st16)}
        log(f"[bench] 16 rhs: {t16 * 1e3:.1f} ms per batch, {16.0 / t16:.3f} solves/s, "
            f"residual {st16.true_rel_residual:.2e}")
        del b16
    # the solver's fine A = D_PV^dag D_DW: two stencil launches against the fused launch (the
    # timed choice's best fused configuration), 1 and 16 columns, FP32
    fine_a = {}
    if not args.quick:
        fine_a = fine_a_rows(dwfmg, inputs, torch, mg, L, Ls)
    mg.close()

    if not args.quick:
        def variant(name, wlv, **kw):
            mgv = dwfmg.MG(U, Ls, m, M5, make_params(dwfmg, wlv, True, **kw), null_starts(inputs, wlv, torch))
            _, tv, stv, _ = timed(mgv, b, ROW_SAMPLES, 1)
            rows[name] = {"solves_per_s": 1.0 / tv, "samples": ROW_SAMPLES,
                          "mg": {"nvec": wlv["nvec"], "block": wlv["block"], "Ls_coarse": wlv["Ls_coarse"],
                                 "smooth_iters": kw.get("smooth_iters", 8), "smooth_restart": kw.get("smooth_restart", 0)},
                          "coarsest": {k: v for k, v in kw.items() if k.startswith("coarsest")}, **stats_dict(stv)}
            if kw.get("pv_poly") is not None:
                rows[name]["pv_poly"] = list(kw["pv_poly"])
            log(f"[bench] {name}: {tv * 1e3:.1f} ms/solve, fine applies {stv.fine_applies}")
            mgv.close()
        wl4 = dict(wl, Ls_coarse=[4] * len(wl["nvec"]))
        # the paper's parameter table throughout: coarse Ls 4, coarsest CGNR to 0.05, 8 post-smoothing steps
        variant("paper_table_cgnr_Ls4", wl4, **coarsest("cgnr"))
        # the headline hierarchy with the paper's smoother (8 steps, one GCR cycle) and coarsest GCR(6) to 0.25
        variant("smoother8_gcr025", wl, **coarsest("gcr", 0.25))
        # coarse Ls 4 with the headline's coarsest GCR
        variant("gcr_Ls4", wl4, **head)
        # three-level hierarchy (4x4 / 8 vectors, then 2x2 / 12 vectors), headline coarsest settings
        variant("three_level", dict(WORKLOADS["dwf256_ls16_mg3"]), **head)
        # the fastest shape measured: 8 null vectors, coarse Ls 2
        variant("nvec8_Ls2", dict(wl, nvec=[8], Ls_coarse=[2]), **head)
        # the headline with the coarsest Krylov vectors in FP32 as well (below the FP64
        # coarsest solve of the precision form; same FP64 true residual)
        variant("coarsest_fp32", wl, coarsest_f32=True, **head)
        # the polynomial correction of the PV preconditioning (App. A): minimax weighting of
        # degree 2 over [1, 25], the free-field range of D_PV D_PV^dag
        variant("pv_poly_cheb2", wl, pv_poly=dwfmg.pv_poly_chebyshev(2, 1.0, 25.0), **head)

    if not args.quick:
        # the paper's solver comparison: Krylov solves of the same system without multigrid (FP64)
        bf = b[0].contiguous()
        for name, meth, ell in (("krylov_cgnr", dwfmg.KRYLOV_CGNR, 0), ("krylov_bicgstab6", dwfmg.KRYLOV_BICGSTAB, 6)):
            tks = []
            for _ in range(ROW_SAMPLES):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, sk = dwfmg.dwf_krylov_solve(U, bf, m, M5, method=meth, ell=max(ell, 1), tol=1e-10, maxit=200000,
                                               check=False)
                tks.append(time.perf_counter() - t0)
            tk = sorted(tks)[len(tks) // 2]
            rows[name] = {"solves_per_s": 1.0 / tk, "samples": ROW_SAMPLES, "iterations": sk.fine_iters,
                          "fine_applies": sk.fine_applies, "residual": sk.true_rel_residual, "status": sk.status}
            log(f"[bench] {name}: {tk * 1e3:.1f} ms, {sk.fine_iters} iterations, {sk.fine_applies} applications, "
                f"residual {sk.true_rel_residual:.2e}")

    # ---------------------------------------------------------------- plain FP64 solve (same algorithm)
    fp64 = None
    if not args.no_fp64 and not args.quick:
        mg64 = dwfmg.MG(U, Ls, m, M5, make_params(dwfmg, wl, False, **head), starts)
        _, t64, st64, _ = timed(mg64, b, ROW_SAMPLES, 1)
        fp64 = {"solves_per_s": 1.0 / t64, "samples": ROW_SAMPLES, **stats_dict(st64)}
        log(f"[bench] fp64 solve {t64 * 1e3:.1f} ms")
        mg64.close()

    stencil = None
    if not args.no_stencil and not args.quick:
        stencil = stencil_rows(dwfmg, inputs, torch, m, M5)
        log(f"[bench] fine stencil {json.dumps(stencil)}")

    cpu = None
    if not args.no_cpu_baseline and not args.quick:
        log("[bench] timing the oracle on the host")
        cpu = cpu_baseline(wl, stats, g.U, head)
        log(f"[bench] oracle baseline: {json.dumps(cpu)}")

    res = {
        "metric": METRIC,
        "value": mixed_sps,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 / mixed_sps,
        "median_ms_per_step": t_median * 1e3,
        "oracle_residual": oracle_residual,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": f"{L}x{L}", "Ls": Ls, "nrhs": 1, "beta": wl["beta"],
                   "m_f": m, "M5": M5, "tol": 1e-10,
                   "mg": {"nvec": wl["nvec"], "block": wl["block"], "Ls_coarse": wl["Ls_coarse"],
                          "coarsest_solver": args.coarsest, "coarsest_tol": head["coarsest_tol"],
                          "coarsest_restart": args.coarsest_restart if args.coarsest == "gcr" else None,
                          "coarsest_nev": args.nev, "m_setup": head.get("m_setup", 0.0),
                          "setup_iters": head.get("setup_iters", 250), "smooth_iters": head.get("smooth_iters", 8),
                          "smooth_restart": head.get("smooth_restart", 0)},
                   "precision": "fine FP32, coarse links BF16 (FP32 arithmetic), coarsest vectors FP64, "
                                "outer defect correction FP64"},
        "roofline": {"bound": "hbm", "kernel": "coarse_mfma_kernel (coarse D_DW apply, level 1)",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "algorithmic_bytes": coarse_bytes, "us_per_launch": t_coarse_ms * 1e3,
                     "stored_bytes": stored_bytes,
                     "frac_stored_bytes": stored_bytes / (t_coarse_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "frac_counter_bytes": (traffic / (t_coarse_ms * 1e-3) / 1e9 / PEAK_HBM_GBS) if traffic else None},
        "cpu_baseline": cpu,
        "coarse_mfma": coarse_mfma,
        "coarse_A": coarse_a,
        "solve_roofline": solve_roofline,
        "fp64": fp64,
        "mixed_vs_fp64": (mixed_sps / fp64["solves_per_s"]) if fp64 else None,
        "rows": rows,
        "fine_stencil": stencil,
        "fine_a": fine_a,
        "setup_s": setup_s,
        "solve": stats_dict(stats),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
