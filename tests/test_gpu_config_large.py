"""Large combined form at full size: 512^2 x Ls 32, beta 10, m_f 0.001, 16
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
