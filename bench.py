#!/usr/bin/env python3
"""Benchmark of the domain-wall multigrid hot path on one MI355X.

Metric: MG-preconditioned domain-wall solves per second to a true FP64
relative residual of 1e-10 on a 256^2 x Ls 16 lattice (beta 6, m_f 0.01,
M5 = -1), mixed precision (FP32 fine level, BF16 coarse links, FP64 outer
defect correction and FP64 coarse Krylov vectors), next to the plain FP64
solve and the fine-stencil HBM bandwidth.

A step is one full solve (K-cycle preconditioned flexible GCR inside the FP64
defect correction) of one right-hand side already resident in HBM.  The
hierarchy setup is done once before timing and reported separately.  Prints
one JSON line.
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

WORKLOADS = {
    # metric workload: 256^2 x 16, 2-level 4x4 aggregates with 16 null vectors
    "dwf256_ls16_mg2": dict(L=256, Ls=16, beta=6.0, sweeps=200, m=0.01, M5=-1.0, cfg=6, gauge_cfg=4,
                            nvec=[16], block=[(4, 4)], Ls_coarse=[4]),
    # same lattice, the paper's three-level parameter table
    "dwf256_ls16_mg3": dict(L=256, Ls=16, beta=6.0, sweeps=200, m=0.01, M5=-1.0, cfg=6, gauge_cfg=4,
                            nvec=[8, 12], block=[(4, 4), (2, 2)], Ls_coarse=[4, 4]),
    # 128^2 x 16 precision form
    "dwf128_ls16_mg2": dict(L=128, Ls=16, beta=6.0, sweeps=200, m=0.01, M5=-1.0, cfg=2, gauge_cfg=2,
                            nvec=[16], block=[(4, 4)], Ls_coarse=[4]),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_params(dwfmg, wl, mixed, nev=0, **eig):
    n = len(wl["nvec"])
    if mixed:
        link = [dwfmg.P_BF16] * n
        vec = [dwfmg.P_F32] * (n - 1) + [dwfmg.P_F64]
        fine = dwfmg.P_F32
    else:
        link = [dwfmg.P_F64] * n
        vec = [dwfmg.P_F64] * n
        fine = dwfmg.P_F64
    return dwfmg.MGParams(nvec=list(wl["nvec"]), block=list(wl["block"]), Ls_coarse=list(wl["Ls_coarse"]),
                          link_prec=link, vec_prec=vec, fine_prec=fine, coarsest_nev=nev, **eig)


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


def stored_traffic(kernel_src):
    """HBM traffic of the dominant kernel from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    p = os.path.join(ROOT, "profiles", "coarse_stencil_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_sha256_16") != source_hash(kernel_src):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(wl, stats, U_np):
    """The oracle, untuned, on the host: unit costs of its operator applications
    on the same lattice and hierarchy shape, combined with the operation counts
    of one GPU solve (a lower bound on the oracle's solve time: the Krylov
    vector algebra is not counted)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import dwf_oracle as O
    from paper_2004_07732_amd import inputs

    L, Ls, m, M5 = wl["L"], wl["Ls"], wl["m"], wl["M5"]
    with threadpool_limits(limits=1):
        psi = inputs.gaussian_field((Ls, L, L, 2), 1)
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            O.pv_dag_dw(U_np, psi, m, M5)
        tA = (time.perf_counter() - t0) / reps
        # coarse operator of the same shape (prolongator from Gaussian vectors)
        nv, (bx, by), Lsc = wl["nvec"][0], wl["block"][0], wl["Ls_coarse"][0]
        V = inputs.gaussian_field((L, L, 2, 1, nv), 2)
        P = O.Prolongator(V=O.block_orthonormalize(V, (by, bx)), block=(by, bx))
        S = O.galerkin(O.wilson_stencil(U_np), P)
        ec = inputs.gaussian_field((Lsc, L // by, L // bx, 2 * nv), 3)
        t0 = time.perf_counter()
        O.stencil_dwf(S, O.stencil_dwf(S, ec, m, M5), 1.0, M5, dagger=True)
        tAc = time.perf_counter() - t0
    fine_A = stats.fine_applies / 2.0
    # one CGNR iteration applies A and A^dagger; each call adds one A^dagger
    coarse_A = 2.0 * stats.level_iters[0] + stats.level_calls[0] if len(wl["nvec"]) == 1 else None
    if coarse_A is None:
        return None
    t_solve = fine_A * tA + coarse_A * tAc
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle unit costs on the host: D_PV^dag D_DW at {L}^2 x {Ls} = {tA:.3f} s, "
                       f"coarse hat-A at {L // bx}^2 x {Lsc} x {2 * nv} dof = {tAc:.3f} s; "
                       f"times the counts of one GPU solve ({fine_A:.0f} fine A, {coarse_A:.0f} coarse A); "
                       f"Krylov vector algebra not counted")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dwf256_ls16_mg2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stencil", action="store_true", help="skip the fine-stencil bandwidth run")
    ap.add_argument("--nev", type=int, default=0,
                    help="deflate the coarsest solve with this many eigenvectors of its normal operator")
    ap.add_argument("--eig-degree", type=int, default=None, help="Chebyshev filter degree of the eigensolver")
    ap.add_argument("--eig-maxit", type=int, default=None)
    ap.add_argument("--eig-tol", type=float, default=None)
    ap.add_argument("--coarsest", choices=["cgnr", "gcr"], default="cgnr",
                    help="coarsest-level solver: CGNR on A^dag A (as in the paper) or restarted GCR on A")
    ap.add_argument("--coarsest-restart", type=int, default=16)
    ap.add_argument("--coarsest-tol", type=float, default=None, help="coarsest relative tolerance (default 0.05)")
    ap.add_argument("--counters", action="store_true",
                    help="only run the dominant kernel (20 launches) next to a plain 256 MiB copy, for "
                         "rocprofv3 --pmc runs; prints no benchmark line")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (this build has no "
              f"multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2004_07732_amd import dwfmg, inputs

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    wl = WORKLOADS[args.workload]
    L, Ls, m, M5 = wl["L"], wl["Ls"], wl["m"], wl["M5"]
    log(f"[bench] workload {args.workload}: generating gauge field {L}^2 beta {wl['beta']}")
    g = inputs.metropolis_u1(L, L, wl["beta"], wl["sweeps"], inputs.gauge_seed(wl["gauge_cfg"], L))
    U = torch.from_numpy(g.U).cuda()
    b = torch.from_numpy(inputs.gaussian_field((1, Ls, L, L, 2), inputs.rhs_seed(wl["cfg"], L, 0))).cuda()
    starts = null_starts(inputs, wl, torch)

    if args.counters:
        mg = dwfmg.MG(U, Ls, m, M5, make_params(dwfmg, wl, True), starts)
        c = mg.info(1)
        xin = torch.from_numpy(inputs.gaussian_field((1, c["Ls"], c["Ly"], c["Lx"], c["n"]), 5)).cuda()
        mg.time_op(1, dwfmg.MG_OP_DW, xin, 1, iters=20)
        a = torch.ones(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        bcopy = torch.empty_like(a)
        for _ in range(5):
            bcopy.copy_(a)
        torch.cuda.synchronize()
        log("[bench] counters run done: 21 coarse launches, 5 copies of 256 MiB")
        return

    # ---------------------------------------------------------------- mixed-precision solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eig = {k: v for k, v in (("eig_degree", args.eig_degree), ("eig_maxit", args.eig_maxit),
                             ("eig_tol", args.eig_tol)) if v is not None}
    eig["coarsest_solver"] = dwfmg.COARSEST_GCR if args.coarsest == "gcr" else dwfmg.COARSEST_CGNR
    eig["coarsest_restart"] = args.coarsest_restart
    if args.coarsest_tol is not None:
        eig["coarsest_tol"] = args.coarsest_tol
    mg = dwfmg.MG(U, Ls, m, M5, make_params(dwfmg, wl, True, args.nev, **eig), starts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.2f} s")
    if args.nev:
        di = mg.deflation_info()
        log(f"[bench] deflation: nev {di['nev']}, {di['iters']} filtered iterations, worst residual "
            f"{di['worst_residual']:.1e}, lambda {di['lambdas'][0]:.3e} .. {di['lambdas'][-1]:.3e}")
    for i in range(args.warmup):
        x, st = mg.solve(b, 1e-10)
        log(f"[bench] warmup {i}: {st.solve_ms:.1f} ms, residual {st.true_rel_residual:.2e}, "
            f"fine iters {st.fine_iters}, coarse iters {st.level_iters}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        x, st = mg.solve(b, 1e-10)
        log(f"[bench] step {i}: {st.solve_ms:.1f} ms, residual {st.true_rel_residual:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mixed_sps = args.steps / elapsed
    stats = st

    # ---------------------------------------------------------------- dominant kernel: coarse stencil
    c = mg.info(1)
    xin = torch.from_numpy(inputs.gaussian_field((1, c["Ls"], c["Ly"], c["Lx"], c["n"]), 5)).cuda()
    t_coarse_ms = mg.time_op(1, dwfmg.MG_OP_DW, xin, 1, iters=200)
    n, nsites, Lsc = c["n"], c["Lx"] * c["Ly"], c["Ls"]
    link_bytes = 4  # bfloat16 complex
    vec_bytes = 16 if make_params(dwfmg, wl, True).vec_prec[0] == dwfmg.P_F64 else 8
    coarse_bytes = nsites * (5 * n * n * link_bytes + 2 * Lsc * n * vec_bytes)
    achieved = coarse_bytes / (t_coarse_ms * 1e-3) / 1e9
    traffic = stored_traffic(os.path.join(ROOT, "paper_2004_07732_amd", "csrc", "coarse_mfma.hip"))
    log(f"[bench] coarse stencil {t_coarse_ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic")
    mg.close()

    # ---------------------------------------------------------------- plain FP64 solve
    fp64 = None
    if not args.no_fp64:
        mg64 = dwfmg.MG(U, Ls, m, M5, make_params(dwfmg, wl, False), starts)
        x64, st64 = mg64.solve(b, 1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x64, st64 = mg64.solve(b, 1e-10)
        torch.cuda.synchronize()
        fp64 = {"solves_per_s": 1.0 / (time.perf_counter() - t0), "residual": st64.true_rel_residual,
                "fine_iters": st64.fine_iters, "coarse_iters": st64.level_iters[0]}
        log(f"[bench] fp64 solve {1e3 / fp64['solves_per_s']:.1f} ms")
        mg64.close()

    # ---------------------------------------------------------------- fine stencil bandwidth
    stencil = None
    if not args.no_stencil:
        Ls2, L2, nr = 32, 512, 4
        U2 = torch.from_numpy(inputs.links_from_theta(inputs.random_theta(L2, L2, 8_000_000))).cuda().to(torch.complex64)
        psi = (torch.randn((nr, Ls2, L2, L2, 2), dtype=torch.complex64, device="cuda"))
        out = torch.empty_like(psi)
        for _ in range(3):
            dwfmg.dwf_apply(U2, psi, m, M5, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 50
        e0.record()
        for _ in range(reps):
            dwfmg.dwf_apply(U2, psi, m, M5, out=out)
        e1.record()
        torch.cuda.synchronize()
        t_ms = e0.elapsed_time(e1) / reps
        sbytes = 2 * psi.numel() * 8 + U2.numel() * 8
        stencil = {"workload": f"{L2}^2 x {Ls2} x {nr} rhs FP32", "us": t_ms * 1e3,
                   "GB_s": sbytes / (t_ms * 1e-3) / 1e9, "frac_of_peak": sbytes / (t_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        log(f"[bench] fine stencil {stencil}")
        del psi, out

    # ---------------------------------------------------------------- CPU baseline (oracle)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        cpu = cpu_baseline(wl, stats, g.U)

    res = {
        "metric": "DWF solves/s to 1e-10 at 256^2xLs16, mixed vs FP64; D_dw stencil HBM GB/s",
        "value": mixed_sps,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 / mixed_sps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": f"{L}x{L}", "Ls": Ls, "nrhs": 1, "beta": wl["beta"],
                   "m_f": m, "M5": M5, "tol": 1e-10,
                   "mg": {"nvec": wl["nvec"], "block": wl["block"], "Ls_coarse": wl["Ls_coarse"],
                          "coarsest_nev": args.nev, "coarsest_solver": args.coarsest},
                   "precision": "fine FP32, coarse links BF16 (FP32 arithmetic), coarse vectors FP64, "
                                "outer defect correction FP64"},
        "roofline": {"bound": "hbm", "kernel": "coarse_kernel (coarse D_DW apply, level 1)",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "algorithmic_bytes": coarse_bytes, "us_per_launch": t_coarse_ms * 1e3},
        "cpu_baseline": cpu,
        "fp64": fp64,
        "mixed_vs_fp64": (mixed_sps / fp64["solves_per_s"]) if fp64 else None,
        "fine_stencil": stencil,
        "setup_s": setup_s,
        "solve": {"residual": stats.true_rel_residual, "outer_steps": stats.outer_steps,
                  "fine_iters": stats.fine_iters, "fine_applies": stats.fine_applies,
                  "coarse_iters": stats.level_iters, "coarse_calls": stats.level_calls},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
