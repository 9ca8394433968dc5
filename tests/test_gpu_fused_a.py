"""The solver's fine operator A = D_PV^dag D_DW(m) (eq. NormalExp) in one fused launch:
LDS tiles of the input with a two-site margin, the intermediate D_DW(m) psi evaluated
on every tile and its one-site ring and never stored.  Checked against the oracle's A
(FP64) and against the two separate stencil launches (FP32), for every fused tile
shape, slice chunks from 1 to Ls, several columns, lattices of one or several tiles,
Ls = 2 (both fifth-dimension wraps in every chunk), and in solves."""
import numpy as np
import pytest
import torch

from oracle import dwf_oracle as O
from paper_2004_07732_amd import inputs

pytestmark = pytest.mark.gpu

dwfmg = pytest.importorskip("paper_2004_07732_amd.dwfmg")


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(autouse=True)
def automatic_choice_afterwards():
    yield
    dwfmg.dwf_fine_a_config(dwfmg.FINE_A_AUTO)


def field(Lx, Ly, seed):
    theta = inputs.random_theta(Lx, Ly, seed) if Lx != Ly else None
    if theta is not None:
        return inputs.links_from_theta(theta)
    return inputs.metropolis_u1(Lx, Ly, 6.0, 10, seed).U


def hierarchy(U, Ls, m, M5, fine_prec, ncol, seed):
    Ly, Lx = U.shape[1], U.shape[2]
    starts = [T(inputs.gaussian_field((4, Ly, Lx, 2), seed))]
    p = dwfmg.MGParams(nvec=[4], block=[(4, 4)], Ls_coarse=[2], link_prec=[dwfmg.P_F64], vec_prec=[dwfmg.P_F64],
                       fine_prec=fine_prec, setup_iters=0)
    return dwfmg.MG(T(U), Ls, m, M5, p, starts, max_nrhs=ncol)


LATTICES = [(32, 32, 8, 1), (16, 16, 2, 2), (48, 32, 5, 1), (32, 16, 16, 3)]


@pytest.mark.parametrize("Lx,Ly,Ls,ncol", LATTICES)
@pytest.mark.parametrize("chunk", [1, 2, 3, 64])
def test_fused_a_fp64_matches_the_oracle(Lx, Ly, Ls, ncol, chunk):
    """FP64 fields (tiles of 16 x 8, the shape whose LDS fits FP64) against the oracle's
    D_PV^dag D_DW(m) to 1e-13."""
    m, M5 = 0.05, -1.0
    U = field(Lx, Ly, 8100 + Lx + Ls)
    mg = hierarchy(U, Ls, m, M5, dwfmg.P_F64, ncol, 8200)
    x = inputs.gaussian_field((ncol, Ls, Ly, Lx, 2), 8300 + chunk)
    dwfmg.dwf_fine_a_config(dwfmg.FINE_A_16x8, chunk)
    got = mg.level_op(0, dwfmg.MG_OP_A, T(x), ncol).cpu().numpy()
    for c in range(ncol):
        assert rel(got[c], O.pv_dag_dw(U, x[c], m, M5)) < 1e-13
    mg.close()


@pytest.mark.parametrize("Lx,Ly,Ls,ncol", LATTICES)
@pytest.mark.parametrize("shape", ["16x16", "32x8", "16x8"])
@pytest.mark.parametrize("chunk", [1, 3, 64])
def test_fused_a_fp32_matches_two_launches_and_the_oracle(Lx, Ly, Ls, ncol, shape, chunk):
    """FP32 fields: the fused launch against the two stencil launches (the same arithmetic
    per site; FMA contraction may differ, so a bar of 2e-7 relative, about two FP32
    roundings of the result) and against the oracle on the FP32-rounded input (1e-6).
    A shape that does not tile the lattice falls back to the timed choice."""
    m, M5 = 0.01, -1.0
    U = field(Lx, Ly, 8400 + Lx + Ls)
    mg = hierarchy(U, Ls, m, M5, dwfmg.P_F32, ncol, 8500)
    x = inputs.gaussian_field((ncol, Ls, Ly, Lx, 2), 8600 + chunk).astype(np.complex64).astype(np.complex128)
    dwfmg.dwf_fine_a_config(dwfmg.FINE_A_TWO)
    two = mg.level_op(0, dwfmg.MG_OP_A, T(x), ncol).cpu().numpy()
    code = {"16x16": dwfmg.FINE_A_16x16, "32x8": dwfmg.FINE_A_32x8, "16x8": dwfmg.FINE_A_16x8}[shape]
    dwfmg.dwf_fine_a_config(code, chunk)
    got = mg.level_op(0, dwfmg.MG_OP_A, T(x), ncol).cpu().numpy()
    assert np.isfinite(got).all()
    assert rel(got, two) < 2e-7
    for c in range(ncol):
        assert rel(got[c], O.pv_dag_dw(U, x[c], m, M5)) < 1e-6
    mg.close()


def test_fused_a_config_arguments():
    with pytest.raises(dwfmg.DwfError):
        dwfmg.dwf_fine_a_config(4, 1)
    with pytest.raises(dwfmg.DwfError):
        dwfmg.dwf_fine_a_config(dwfmg.FINE_A_16x16, 0)
    with pytest.raises(dwfmg.DwfError):
        dwfmg.dwf_fine_a_config(-2, 1)
    dwfmg.dwf_fine_a_config(dwfmg.FINE_A_TWO, 0)   # chunk ignored


@pytest.mark.parametrize("shape,chunk", [(1, 4), (2, 8)])   # FINE_A_16x16, FINE_A_32x8
def test_mixed_solve_with_the_fused_a(shape, chunk):
    """A mixed-precision MG solve (FP32 fine level) with the fused A pinned, to the 1e-10
    true residual recomputed by the oracle, in the same number of iterations as with the
    two launches (within one)."""
    L, Ls, m, M5 = 32, 8, 0.01, -1.0
    g = inputs.metropolis_u1(L, L, 6.0, 60, 8700)
    starts = [T(inputs.gaussian_field((8, L, L, 2), 8701))]
    b = inputs.gaussian_field((2, Ls, L, L, 2), 8702)
    p = dwfmg.MGParams(nvec=[8], block=[(4, 4)], Ls_coarse=[2], link_prec=[dwfmg.P_BF16], vec_prec=[dwfmg.P_F32],
                       fine_prec=dwfmg.P_F32, coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=6, coarsest_tol=0.5,
                       smooth_iters=20, smooth_restart=5)
    its = {}
    for pin in (dwfmg.FINE_A_TWO, shape):
        dwfmg.dwf_fine_a_config(pin, chunk)
        mg = dwfmg.MG(T(g.U), Ls, m, M5, p, starts, max_nrhs=2)
        x, st = mg.solve(T(b), 1e-10)
        for c in range(2):
            r = np.linalg.norm(b[c] - O.dwf(g.U, x[c].cpu().numpy(), m, M5)) / np.linalg.norm(b[c])
            assert r <= 1e-10
        its[pin] = st.fine_iters
        mg.close()
    assert abs(its[shape] - its[dwfmg.FINE_A_TWO]) <= 1


def test_fused_a_full_size_headline_shape():
    """256^2 x 16, one column, FP32: every fused shape with the chunk lengths the timed
    choice considers, against the two launches, and the automatic choice (whatever it
    is) against the oracle on the rounded input."""
    L, Ls, m, M5 = 256, 16, 0.01, -1.0
    g = inputs.metropolis_u1(L, L, 6.0, 20, 8800)
    mg = hierarchy(g.U, Ls, m, M5, dwfmg.P_F32, 1, 8801)
    x = inputs.gaussian_field((1, Ls, L, L, 2), 8802).astype(np.complex64).astype(np.complex128)
    dwfmg.dwf_fine_a_config(dwfmg.FINE_A_TWO)
    two = mg.level_op(0, dwfmg.MG_OP_A, T(x), 1).cpu().numpy()
    for shape in (dwfmg.FINE_A_16x16, dwfmg.FINE_A_32x8, dwfmg.FINE_A_16x8):
        for chunk in (16, 8, 4, 2):
            dwfmg.dwf_fine_a_config(shape, chunk)
            got = mg.level_op(0, dwfmg.MG_OP_A, T(x), 1).cpu().numpy()
            assert rel(got, two) < 2e-7, (shape, chunk)
    dwfmg.dwf_fine_a_config(dwfmg.FINE_A_AUTO)
    got = mg.level_op(0, dwfmg.MG_OP_A, T(x), 1).cpu().numpy()
    assert rel(got[0], O.pv_dag_dw(g.U, x[0], m, M5)) < 1e-6
    mg.close()
