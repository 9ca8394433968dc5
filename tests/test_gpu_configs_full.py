"""The large combined form and the batched form at full size.

Large combined form: 512^2 x Ls 32, beta 10, m_f 0.001, 16
seeded Gaussian right-hand sides, 3-level multigrid (4x4 aggregates with 16
null vectors, then 2x2 with 24), BF16 matrix-core coarse levels, FP64 outer
residual and FP64 coarsest vectors, to a relative residual of 1e-10.

The oracle cannot solve this system in reasonable time, so the check is on
sampled outputs it can compute one by one: the true residual
|b_j - D_DW x_j| / |b_j| of sampled right-hand sides j, recomputed with the
oracle's own FP64 operator from the GPU's x_j."""
import sys

import numpy as np
import pytest
import torch

from oracle import dwf_oracle as O
from paper_2004_07732_amd import inputs

pytestmark = pytest.mark.gpu

dwfmg = pytest.importorskip("paper_2004_07732_amd.dwfmg")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_large_combined_form_16_rhs():
    L, Ls, m, M5, beta, nrhs, cfg = 512, 32, 0.001, -1.0, 10.0, 16, 5
    g = inputs.metropolis_u1(L, L, beta, 500, inputs.gauge_seed(cfg, L))
    say(f"[C5] gauge field ready: acceptance {g.acceptance:.3f}")
    U = torch.from_numpy(g.U).cuda()
    b = torch.empty((nrhs, Ls, L, L, 2), dtype=torch.complex128, device="cuda")
    for j in range(nrhs):
        b[j] = torch.from_numpy(inputs.gaussian_field((Ls, L, L, 2), inputs.rhs_seed(cfg, L, j)))
    say("[C5] right-hand sides ready")
    starts = [torch.from_numpy(inputs.gaussian_field((16, L, L, 2), inputs.null_start_seed(cfg, 0))).cuda(),
              torch.from_numpy(inputs.gaussian_field((24, L // 4, L // 4, 32), inputs.null_start_seed(cfg, 1))).cuda()]
    p = dwfmg.MGParams(nvec=[16, 24], block=[(4, 4), (2, 2)], Ls_coarse=[2, 2], link_prec=[dwfmg.P_BF16] * 2,
                       vec_prec=[dwfmg.P_F32, dwfmg.P_F64], fine_prec=dwfmg.P_F32,
                       coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=8, coarsest_tol=0.25, max_iters=20000)
    mg = dwfmg.MG(U, Ls, m, M5, p, starts)
    say("[C5] hierarchy ready, solving 16 rhs")
    x, st = mg.solve(b, 1e-10)
    say(f"[C5] solve: {st.solve_ms / 1e3:.1f} s, fine iters {st.fine_iters}, fine applies {st.fine_applies}, "
        f"levels {st.level_iters} / {st.level_calls}, residual {st.true_rel_residual:.2e}")
    assert st.status == dwfmg.DWF_OK and st.true_rel_residual <= 1e-10
    for j in (0, nrhs - 1):
        xj = x[j].cpu().numpy()
        bj = b[j].cpu().numpy()
        res = np.linalg.norm(bj - O.dwf(g.U, xj, m, M5)) / np.linalg.norm(bj)
        say(f"[C5] rhs {j}: oracle residual {res:.2e}")
        assert res <= 1e-10


def test_batched_form_64_rhs_three_lattices():
    """Batched form at full size: 64 seeded Gaussian right-hand sides over
    16 x 64^2, 32 x 128^2 and 16 x 256^2 (Ls 16, beta 3, m_f 0.005), one
    hierarchy per lattice with FP16 matrix-core coarse links, solved together
    by mg_solve_batch to 1e-10; sampled right-hand sides checked with the
    oracle's operator."""
    Ls, m, M5, beta, cfg = 16, 0.005, -1.0, 3.0, 3
    cases = [(64, 16), (128, 32), (256, 16)]
    mgs, bs, fields = [], [], []
    for k, (L, nr) in enumerate(cases):
        g = inputs.metropolis_u1(L, L, beta, 200, inputs.gauge_seed(cfg, L))
        starts = [torch.from_numpy(inputs.gaussian_field((16, L, L, 2), inputs.null_start_seed(cfg, 0) + k)).cuda()]
        p = dwfmg.MGParams(nvec=[16], block=[(4, 4)], Ls_coarse=[2], link_prec=[dwfmg.P_F16],
                           vec_prec=[dwfmg.P_F64], fine_prec=dwfmg.P_F32, coarsest_solver=dwfmg.COARSEST_GCR,
                           coarsest_restart=8, coarsest_tol=0.25, max_iters=20000)
        mgs.append(dwfmg.MG(torch.from_numpy(g.U).cuda(), Ls, m, M5, p, starts))
        b = torch.empty((nr, Ls, L, L, 2), dtype=torch.complex128, device="cuda")
        for j in range(nr):
            b[j] = torch.from_numpy(inputs.gaussian_field((Ls, L, L, 2), inputs.rhs_seed(cfg, L, j)))
        bs.append(b)
        fields.append(g.U)
    say("[C3] three hierarchies ready, solving 64 rhs")
    xs, sts = dwfmg.solve_batch(mgs, bs, 1e-10)
    for (L, nr), U, b, x, st in zip(cases, fields, bs, xs, sts):
        say(f"[C3] L={L} nrhs={nr}: {st.solve_ms / 1e3:.1f} s, fine iters {st.fine_iters}, "
            f"coarse {st.level_iters[0]} in {st.level_calls[0]} calls, residual {st.true_rel_residual:.2e}")
        assert st.status == dwfmg.DWF_OK and st.true_rel_residual <= 1e-10
        j = nr - 1
        bj = b[j].cpu().numpy()
        res = np.linalg.norm(bj - O.dwf(U, x[j].cpu().numpy(), m, M5)) / np.linalg.norm(bj)
        assert res <= 1e-10


@pytest.mark.parametrize("nrhs", [1, 16])
def test_headline_configuration(nrhs):
    """The benchmark's own configuration at full size: 256^2 x Ls 16, beta 6,
    m_f 0.01, 2 levels (4x4 aggregates, 16 null vectors, coarse Ls 2), FP32 fine
    level, BF16 matrix-core coarse links, FP64 coarse vectors, coarsest GCR(8) to
    0.25, FP64 defect correction to 1e-10; the oracle recomputes the residual of
    sampled right-hand sides."""
    L, Ls, m, M5, cfg = 256, 16, 0.01, -1.0, 6
    g = inputs.metropolis_u1(L, L, 6.0, 200, inputs.gauge_seed(4, L))
    b = torch.empty((nrhs, Ls, L, L, 2), dtype=torch.complex128, device="cuda")
    for j in range(nrhs):
        b[j] = torch.from_numpy(inputs.gaussian_field((Ls, L, L, 2), inputs.rhs_seed(cfg, L, j)))
    starts = [torch.from_numpy(inputs.gaussian_field((16, L, L, 2), inputs.null_start_seed(cfg, 0))).cuda()]
    p = dwfmg.MGParams(nvec=[16], block=[(4, 4)], Ls_coarse=[2], link_prec=[dwfmg.P_BF16], vec_prec=[dwfmg.P_F64],
                       fine_prec=dwfmg.P_F32, coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=8,
                       coarsest_tol=0.25)
    mg = dwfmg.MG(torch.from_numpy(g.U).cuda(), Ls, m, M5, p, starts)
    x, st = mg.solve(b, 1e-10)
    say(f"[headline] nrhs {nrhs}: {st.solve_ms:.0f} ms, fine iters {st.fine_iters}, residual {st.true_rel_residual:.2e}")
    assert st.status == dwfmg.DWF_OK and st.true_rel_residual <= 1e-10
    for j in sorted({0, nrhs - 1}):
        bj = b[j].cpu().numpy()
        res = np.linalg.norm(bj - O.dwf(g.U, x[j].cpu().numpy(), m, M5)) / np.linalg.norm(bj)
        assert res <= 1e-10
