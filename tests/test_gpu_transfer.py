"""Transfer variants of Sec. 4.1 on the GPU: the bulk transfer (the 2-d
prolongator on every slice) against the oracle, MG solves with either
transfer, and the local colinearity / oblique projector diagnostics computed
from the library's level operators against the oracle's definitions."""
import numpy as np
import pytest
import torch

from oracle import dwf_oracle as O
from paper_2004_07732_amd import inputs

pytestmark = pytest.mark.gpu

dwfmg = pytest.importorskip("paper_2004_07732_amd.dwfmg")
DEV = "cuda"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def pair(L, Ls, m, levels, seed, transfer, beta=6.0, **kw):
    """GPU and oracle hierarchies from the same field and null-vector starts;
    levels: list of (nvec, block, Ls_coarse)."""
    U = inputs.metropolis_u1(L, L, beta, 30, seed).U
    starts, Lc, n = [], L, 2
    for li, (nv, (bx, by), _) in enumerate(levels):
        starts.append(inputs.gaussian_field((nv, Lc, Lc, n), seed + 10 + li))
        Lc //= bx
        n = 2 * nv
    code = {"wall": dwfmg.TRANSFER_WALL, "bulk": dwfmg.TRANSFER_BULK, "slice1": dwfmg.TRANSFER_SLICE1}[transfer]
    params = dwfmg.MGParams(nvec=[l[0] for l in levels], block=[l[1] for l in levels],
                            Ls_coarse=[l[2] for l in levels], link_prec=[dwfmg.P_F64] * len(levels),
                            vec_prec=[dwfmg.P_F64] * len(levels), fine_prec=dwfmg.P_F64, setup_iters=0, transfer=code,
                            **kw)
    mg = dwfmg.MG(T(U), Ls, m, -1.0, params, [T(s) for s in starts], max_nrhs=2)
    op = O.MGParams(levels=[O.LevelParams(nvec=l[0], block=(l[1][1], l[1][0]), Ls=l[2], setup_iters=0)
                            for l in levels], transfer=transfer,
                    smooth_iters=params.smooth_iters, coarsest_tol=params.coarsest_tol,
                    coarsest_maxit=params.coarsest_maxit)
    return U, mg, O.MG(U, Ls, m, -1.0, op, starts)


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("transfer", ["bulk", "slice1"])
def test_transfer_variant_parity(level, transfer):
    """Bulk transfer and the literal-slice toggle against the oracle on both levels."""
    Lsc = (4, 4) if transfer == "bulk" else (3, 2)
    U, mg, omg = pair(16, 4, 0.05, [(4, (4, 4), Lsc[0]), (2, (2, 2), Lsc[1])], 900, transfer)
    f, c = mg.info(level), mg.info(level + 1)
    r = inputs.gaussian_field((2, f["Ls"], f["Ly"], f["Lx"], f["n"]), 901)
    e = inputs.gaussian_field((2, c["Ls"], c["Ly"], c["Lx"], c["n"]), 902)
    got_r = mg.level_op(level, dwfmg.MG_OP_RESTRICT, T(r), 2, out_shape=e.shape).cpu().numpy()
    got_e = mg.level_op(level, dwfmg.MG_OP_PROLONG, T(e), 2, out_shape=r.shape).cpu().numpy()
    assert rel(got_r, omg.restrict(level, r)) < 1e-13
    assert rel(got_e, omg.prolong(level, e)) < 1e-13


def test_bulk_transfer_requires_full_coarse_ls():
    U = inputs.metropolis_u1(16, 16, 6.0, 10, 903).U
    s = inputs.gaussian_field((4, 16, 16, 2), 904)
    p = dwfmg.MGParams(nvec=[4], block=[(4, 4)], Ls_coarse=[2], transfer=dwfmg.TRANSFER_BULK, setup_iters=0)
    with pytest.raises(dwfmg.DwfError):
        dwfmg.MG(T(U), 4, 0.05, -1.0, p, [T(s)])


@pytest.mark.parametrize("transfer", ["wall", "bulk", "slice1"])
def test_diagnostics_match_oracle(transfer):
    """Local colinearity |(1 - P R) v| and oblique projector |(1 - P hat-A^{-1} R A) v|
    for low right eigenvectors v of the fine A (dense eigensolve) and a random
    vector: from the library's level operators (restrict, prolong, A, and a
    K-cycle without smoothing and with an exact coarsest solve, which is
    P hat-A^{-1} R) against the oracle's definitions."""
    L, Ls, m = 8, 4, 0.05
    U, mg, omg = pair(L, Ls, m, [(2, (4, 4), Ls)], 910, transfer, beta=10.0, smooth_iters=0,
                      coarsest_tol=1e-14, coarsest_maxit=20000)
    shape = (Ls, L, L, 2)
    A = O.assemble(lambda v: omg.A(0, v), shape)
    w, vr = np.linalg.eig(A)
    order = np.argsort(np.abs(w))[:4]
    vecs = [vr[:, i].reshape(shape) for i in order] + [inputs.gaussian_field(shape, 911)]
    c = mg.info(1)
    cshape = (c["Ls"], c["Ly"], c["Lx"], c["n"])
    Ahat = O.assemble(lambda e: omg.A(1, e), cshape)
    inv = lambda rc: np.linalg.solve(Ahat, rc.reshape(-1)).reshape(cshape)
    for v in vecs:
        v = v / np.linalg.norm(v)
        vt = T(v[None])
        pr = mg.level_op(0, dwfmg.MG_OP_PROLONG,
                         mg.level_op(0, dwfmg.MG_OP_RESTRICT, vt, 1, out_shape=(1,) + cshape), 1,
                         out_shape=(1,) + shape)
        col_gpu = float(torch.linalg.vector_norm(vt - pr))
        Av = mg.level_op(0, dwfmg.MG_OP_A, vt, 1)
        kc = mg.level_op(0, dwfmg.MG_OP_KCYCLE, Av, 1)
        obl_gpu = float(torch.linalg.vector_norm(vt - kc))
        col_o = omg.local_colinearity(v)
        obl_o = omg.oblique_projector(v, inv)
        assert abs(col_gpu - col_o) <= 1e-10 * max(1.0, col_o)
        assert abs(obl_gpu - obl_o) <= 1e-8 * max(1.0, obl_o), (obl_gpu, obl_o)


def test_bulk_and_wall_transfer_solves():
    """Both transfers precondition the solve to 1e-10 at 64^2 x 8 (coarse L^_s = L_s = 8,
    relaxed null vectors); the counts are printed for the comparison of Sec. 4.1."""
    L, Ls, m, M5 = 64, 8, 0.02, -1.0
    U = inputs.metropolis_u1(L, L, 6.0, 100, 921).U
    b = inputs.gaussian_field((1, Ls, L, L, 2), 920)
    start = inputs.gaussian_field((8, L, L, 2), 922)
    counts = {}
    for transfer, code in (("wall", dwfmg.TRANSFER_WALL), ("bulk", dwfmg.TRANSFER_BULK)):
        p = dwfmg.MGParams(nvec=[8], block=[(4, 4)], Ls_coarse=[Ls], transfer=code)
        mg = dwfmg.MG(T(U), Ls, m, M5, p, [T(start)])
        x, st = mg.solve(T(b), 1e-10)
        res = np.linalg.norm(b[0] - O.dwf(U, x[0].cpu().numpy(), m, M5)) / np.linalg.norm(b[0])
        assert res <= 1e-10
        counts[transfer] = (st.fine_iters, st.fine_applies, st.level_iters[0])
    print(f"64^2 x 8, L^_s 8: wall {counts['wall']}, bulk {counts['bulk']} (fine iters, fine applies, coarse iters)")


def test_bulk_transfer_at_fifth_extent_16():
    """The bulk transfer keeps L^_s = L_s = 16 on the coarse level, beyond one pass
    of the coarse kernels' slice loop; the solve reaches 1e-10 like the wall transfer."""
    L, Ls, m, M5 = 32, 16, 0.02, -1.0
    U = inputs.metropolis_u1(L, L, 6.0, 100, 931).U
    b = inputs.gaussian_field((1, Ls, L, L, 2), 930)
    start = inputs.gaussian_field((8, L, L, 2), 932)
    counts = {}
    for transfer, code in (("wall", dwfmg.TRANSFER_WALL), ("bulk", dwfmg.TRANSFER_BULK)):
        p = dwfmg.MGParams(nvec=[8], block=[(4, 4)], Ls_coarse=[Ls], transfer=code)
        mg = dwfmg.MG(T(U), Ls, m, M5, p, [T(start)])
        x, st = mg.solve(T(b), 1e-10)
        res = np.linalg.norm(b[0] - O.dwf(U, x[0].cpu().numpy(), m, M5)) / np.linalg.norm(b[0])
        assert res <= 1e-10
        counts[transfer] = (st.fine_iters, st.fine_applies, st.level_iters[0])
    print(f"32^2 x 16, L^_s 16: wall {counts['wall']}, bulk {counts['bulk']} (fine iters, fine applies, coarse iters)")


def test_wall_transfer_coarse_ls_sweep():
    """Sec. 4.2: with the wall-only transfer the coarse fifth extent is free.  Every
    L^_s from 2 to 32 preconditions the 32^2 x 16 solve to 1e-10 (mixed precision,
    BF16 coarse links); the counts are printed."""
    L, Ls, m, M5 = 32, 16, 0.02, -1.0
    U = inputs.metropolis_u1(L, L, 6.0, 100, 941).U
    b = inputs.gaussian_field((1, Ls, L, L, 2), 940)
    start = inputs.gaussian_field((8, L, L, 2), 942)
    counts = {}
    for Lsc in (2, 4, 8, 12, 16, 32):
        # the mixed-precision form: BF16 coarse links on the matrix cores
        p = dwfmg.MGParams(nvec=[8], block=[(4, 4)], Ls_coarse=[Lsc], link_prec=[dwfmg.P_BF16],
                           vec_prec=[dwfmg.P_F64], fine_prec=dwfmg.P_F32)
        mg = dwfmg.MG(T(U), Ls, m, M5, p, [T(start)])
        x, st = mg.solve(T(b), 1e-10)
        res = np.linalg.norm(b[0] - O.dwf(U, x[0].cpu().numpy(), m, M5)) / np.linalg.norm(b[0])
        assert res <= 1e-10, (Lsc, res)
        counts[Lsc] = (st.fine_iters, st.level_iters[0])
    print(f"32^2 x 16 wall transfer, L^_s -> (fine iters, coarse iters): {counts}")


def test_coarse_ls_limits():
    L, Ls = 8, 4
    U = inputs.metropolis_u1(L, L, 6.0, 10, 951).U
    start = inputs.gaussian_field((2, L, L, 2), 952)
    for bad in (1, 33):
        with pytest.raises(dwfmg.DwfError):
            dwfmg.MG(T(U), Ls, 0.05, -1.0, dwfmg.MGParams(nvec=[2], block=[(4, 4)], Ls_coarse=[bad]), [T(start)])


def test_literal_slice1_reading_against_the_wall_pair():
    """The reading of the transfer's "s = 1" (slice 1 of the chirally permuted basis,
    i.e. P- psi_1 + P+ psi_Ls) against the literal unpermuted slice 1 (a test toggle):
    both are run on the same 32^2 x 16 problem and the counts printed.  The wall pair
    must reach 1e-10; the literal slice is reported as it comes out (converged with its
    residual at tol, or stopped at the iteration cap)."""
    L, Ls, m, M5 = 32, 16, 0.02, -1.0
    U = inputs.metropolis_u1(L, L, 6.0, 100, 961).U
    b = inputs.gaussian_field((1, Ls, L, L, 2), 960)
    start = inputs.gaussian_field((8, L, L, 2), 962)
    out = {}
    for name, code in (("wall pair", dwfmg.TRANSFER_WALL), ("literal slice 1", dwfmg.TRANSFER_SLICE1)):
        p = dwfmg.MGParams(nvec=[8], block=[(4, 4)], Ls_coarse=[4], transfer=code, max_iters=300)
        mg = dwfmg.MG(T(U), Ls, m, M5, p, [T(start)])
        x, st = mg.solve(T(b), 1e-10, check=False)
        res = np.linalg.norm(b[0] - O.dwf(U, x[0].cpu().numpy(), m, M5)) / np.linalg.norm(b[0])
        out[name] = (st.status, st.fine_iters, st.level_iters[0], res)
        if st.status == 0:
            assert res <= 1e-10
    print(f"32^2 x 16, L^_s 4 (status, fine iters, coarse iters, true residual): {out}")
    assert out["wall pair"][0] == 0
