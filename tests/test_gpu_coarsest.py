"""Coarsest-level variants: deflation (Ritz values of the coarsest normal
operator against a dense eigensolve of the oracle's coarsest operator;
deflated solves against undeflated ones) and restarted GCR on the coarsest A
in place of CGNR (same solution to the outer tolerance)."""
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


def hierarchy(L, Ls, m, levels, seed, oracle=False, **kw):
    U = inputs.metropolis_u1(L, L, 6.0, 30, seed).U
    starts, Lc, n = [], L, 2
    for li, (nv, (bx, by), _) in enumerate(levels):
        starts.append(inputs.gaussian_field((nv, Lc, Lc, n), seed + 10 + li))
        Lc //= bx
        n = 2 * nv
    params = dwfmg.MGParams(nvec=[l[0] for l in levels], block=[l[1] for l in levels],
                            Ls_coarse=[l[2] for l in levels], link_prec=[dwfmg.P_F64] * len(levels),
                            vec_prec=[dwfmg.P_F64] * len(levels), setup_iters=0, **kw)
    mg = dwfmg.MG(T(U), Ls, m, -1.0, params, [T(s) for s in starts], max_nrhs=4)
    omg = None
    if oracle:
        op = O.MGParams(levels=[O.LevelParams(nvec=l[0], block=(l[1][1], l[1][0]), Ls=l[2], setup_iters=0)
                                for l in levels])
        omg = O.MG(U, Ls, m, -1.0, op, starts)
    return U, mg, omg


@pytest.mark.parametrize("levels", [[(4, (4, 4), 4)], [(4, (4, 4), 3), (2, (2, 2), 2)]])
def test_ritz_values_match_dense_spectrum(levels):
    """The nev Ritz values equal the nev smallest eigenvalues of hat-A^dag hat-A,
    from numpy's dense Hermitian eigensolver on the oracle's coarsest operator."""
    nev = 12
    _, mg, omg = hierarchy(16, 4, 0.05, levels, 700, oracle=True, coarsest_nev=nev, eig_tol=1e-9, eig_maxit=300)
    info = mg.deflation_info()
    assert info["nev"] == nev and info["worst_residual"] <= 1e-9
    lc = len(levels)
    c = mg.info(lc)
    shape = (c["Ls"], c["Ly"], c["Lx"], c["n"])
    A = O.assemble(lambda v: omg.A(lc, v), shape)
    lam = np.linalg.eigvalsh(A.conj().T @ A)[:nev]
    got = np.array(info["lambdas"])
    assert np.all(np.diff(got) >= 0)
    np.testing.assert_allclose(got, lam, rtol=1e-9, atol=0)


def test_deflation_off_reports_nothing():
    _, mg, _ = hierarchy(16, 4, 0.05, [(4, (4, 4), 4)], 701)
    info = mg.deflation_info()
    assert info["nev"] == 0 and info["lambdas"] == []


@pytest.mark.parametrize("nrhs,solver", [(1, "cgnr"), (3, "cgnr"), (1, "gcr"), (3, "gcr")])
def test_deflated_solve_same_answer_fewer_coarse_iterations(nrhs, solver):
    """Deflation only changes the coarsest start vector: both solves meet the
    tolerance, agree with each other, and the deflated one needs fewer coarsest
    iterations (CGNR on A^dag A, or restarted GCR on A)."""
    levels = [(4, (4, 4), 4)]
    L, Ls, m = 32, 8, 0.01
    b = T(inputs.gaussian_field((nrhs, Ls, L, L, 2), 702))
    kw = {} if solver == "cgnr" else dict(coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=6, coarsest_tol=0.25)
    res = {}
    for nev in (0, 48):
        _, mg, _ = hierarchy(L, Ls, m, levels, 703, coarsest_nev=nev, eig_tol=1e-3, **kw)
        x, st = mg.solve(b, tol=1e-10)
        assert st.true_rel_residual <= 1e-10
        res[nev] = (x.cpu().numpy(), st)
    x0, s0 = res[0]
    x1, s1 = res[48]
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-8
    it0 = s0.level_iters[0] / max(s0.level_calls[0], 1)
    it1 = s1.level_iters[0] / max(s1.level_calls[0], 1)
    print(f"{solver} coarsest iterations per call: {it0:.1f} undeflated, {it1:.1f} with 48 eigenvectors")
    assert it1 < 0.8 * it0, (it0, it1)


def test_deflation_requires_fp64_coarsest_vectors():
    U = inputs.metropolis_u1(16, 16, 6.0, 10, 704).U
    s = inputs.gaussian_field((4, 16, 16, 2), 705)
    p = dwfmg.MGParams(nvec=[4], block=[(4, 4)], Ls_coarse=[4], link_prec=[dwfmg.P_F32], vec_prec=[dwfmg.P_F32],
                       setup_iters=0, coarsest_nev=8)
    with pytest.raises(dwfmg.DwfError):
        dwfmg.MG(T(U), 4, 0.05, -1.0, p, [T(s)])


@pytest.mark.parametrize("nrhs", [1, 2])
def test_coarsest_gcr_solve_matches_cgnr_solve(nrhs):
    """Restarted GCR on the coarsest A instead of CGNR on A^dag A: a different
    (flexible) preconditioner, the same solution of D_DW x = b to 1e-10."""
    levels = [(4, (4, 4), 4)]
    L, Ls, m = 32, 8, 0.01
    b = T(inputs.gaussian_field((nrhs, Ls, L, L, 2), 706))
    xs = {}
    for solver in (dwfmg.COARSEST_CGNR, dwfmg.COARSEST_GCR):
        _, mg, _ = hierarchy(L, Ls, m, levels, 707, coarsest_solver=solver, coarsest_restart=12)
        x, st = mg.solve(b, tol=1e-10)
        assert st.true_rel_residual <= 1e-10
        assert st.level_calls[0] > 0 and st.level_iters[0] > 0
        xs[solver] = x.cpu().numpy()
    x0, x1 = xs[dwfmg.COARSEST_CGNR], xs[dwfmg.COARSEST_GCR]
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-8


@pytest.mark.parametrize("restart", [5, 6])
def test_coarsest_gcr_restart_lengths(restart):
    """Odd and even restart lengths (the stop flags of the last fused step sit in one or
    the other of the two flag buffers, and restarts continue from the recursive residual):
    both precondition the solve to the 1e-10 true residual for two right-hand sides."""
    levels = [(4, (4, 4), 4)]
    L, Ls, m = 32, 8, 0.01
    b = T(inputs.gaussian_field((2, Ls, L, L, 2), 710))
    _, mg, _ = hierarchy(L, Ls, m, levels, 711, coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=restart)
    x, st = mg.solve(b, tol=1e-10)
    assert st.true_rel_residual <= 1e-10
    assert st.level_calls[0] > 0 and st.level_iters[0] > 0


def test_coarsest_gcr_three_levels():
    levels = [(4, (4, 4), 3), (4, (2, 2), 2)]
    b = T(inputs.gaussian_field((1, 8, 32, 32, 2), 708))
    _, mg, _ = hierarchy(32, 8, 0.02, levels, 709, coarsest_solver=dwfmg.COARSEST_GCR)
    x, st = mg.solve(b, tol=1e-10)
    assert st.true_rel_residual <= 1e-10 and st.level_calls[1] > 0


def test_coarsest_parameter_errors():
    U = inputs.metropolis_u1(16, 16, 6.0, 10, 710).U
    s = inputs.gaussian_field((4, 16, 16, 2), 711)
    for kw in (dict(coarsest_solver=7), dict(coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=0),
               dict(coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=17)):
        p = dwfmg.MGParams(nvec=[4], block=[(4, 4)], Ls_coarse=[4], link_prec=[dwfmg.P_F64], vec_prec=[dwfmg.P_F64],
                           setup_iters=0, **kw)
        with pytest.raises(dwfmg.DwfError):
            dwfmg.MG(T(U), 4, 0.05, -1.0, p, [T(s)])
