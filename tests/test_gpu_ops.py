"""GPU parity of the fine-level operators and utilities against the FP64 oracle.

Bars: FP64 operator applies within 1e-13 relative (2-norm); index and gauge
work bit-exact; FP32 applies report their error against FP64 (bounded by a
few FP32 ulps times the stencil size)."""
import numpy as np
import pytest
import torch

from oracle import dwf_oracle as O
from paper_2004_07732_amd import inputs

pytestmark = pytest.mark.gpu

dwfmg = pytest.importorskip("paper_2004_07732_amd.dwfmg")
DEV = "cuda"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gauge(L0, L1, seed, beta=6.0, sweeps=30):
    if L0 % 2 == 0 and L1 % 2 == 0:
        return inputs.metropolis_u1(L0, L1, beta, sweeps, seed).U
    return inputs.links_from_theta(inputs.random_theta(L0, L1, seed))


# shapes span several 256-thread blocks, ragged tails, extents 1 and 2, odd sizes
SHAPES = [(24, 20, 6, 2), (13, 7, 5, 1), (1, 8, 4, 1), (2, 2, 3, 3), (64, 64, 8, 1), (40, 24, 16, 4)]


@pytest.mark.parametrize("Lx,Ly,Ls,nrhs", SHAPES)
@pytest.mark.parametrize("dagger", [False, True])
def test_dwf_fp64_parity(Lx, Ly, Ls, nrhs, dagger):
    U = gauge(Lx, Ly, 100 + Lx)
    psi = inputs.gaussian_field((nrhs, Ls, Ly, Lx, 2), 200 + Ls)
    m, M5 = 0.03, -1.05
    got = dwfmg.dwf_apply(torch.from_numpy(U).to(DEV), torch.from_numpy(psi).to(DEV), m, M5, dagger=dagger)
    want = O.dwf(U, psi, m, M5, dagger=dagger)
    assert rel(got.cpu().numpy(), want) < 1e-13


# lattices where every tile shape fits (128 x 16), where one tile is the whole
# lattice so the halo ring wraps onto the tile itself (64 x 8, 128 x 4), and
# chunks that leave ragged last chunks or a single slice per thread
FINE_CFG_CASES = [((128, 16, 6, 2), (1, 2, 4, 6)), ((64, 8, 5, 1), (1, 2, 5)), ((128, 4, 3, 1), (1, 2, 3))]
FINE_SHAPES = ["FINE_ROW", "FINE_TILE_64x8", "FINE_TILE_32x16", "FINE_TILE_128x4"]


@pytest.mark.parametrize("case", range(len(FINE_CFG_CASES)))
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_fine_launch_configs_bitwise(case, dtype):
    """Every launch configuration of the fine stencil (row kernel, LDS-tiled
    shapes, chunk lengths) gives the same bits, and those match the oracle."""
    (Lx, Ly, Ls, nrhs), chunks = FINE_CFG_CASES[case]
    U = gauge(Lx, Ly, 300 + Lx + Ly)
    psi = inputs.gaussian_field((nrhs, Ls, Ly, Lx, 2), 310 + Ls)
    m, M5 = 0.02, -1.0
    Ut, pt = torch.from_numpy(U).to(DEV).to(dtype), torch.from_numpy(psi).to(DEV).to(dtype)
    try:
        for dagger in (False, True):
            want = O.dwf(U, psi, m, M5, dagger=dagger)
            ref = None
            for shape in FINE_SHAPES:
                for c in chunks:
                    dwfmg.dwf_fine_config(getattr(dwfmg, shape), c)
                    got = dwfmg.dwf_apply(Ut, pt, m, M5, dagger=dagger)
                    torch.cuda.synchronize()
                    if ref is None:
                        ref = got.clone()
                        err = rel(got.cpu().numpy().astype(np.complex128), want)
                        assert err < (1e-13 if dtype == torch.complex128 else 2e-6), err
                    assert torch.equal(got, ref), (shape, c, dagger)
    finally:
        dwfmg.dwf_fine_config(dwfmg.FINE_AUTO)


def test_fine_config_argument_errors():
    for shape, chunk in ((7, 1), (-2, 1), (0, 0), (1, 4096)):
        with pytest.raises(dwfmg.DwfError):
            dwfmg.dwf_fine_config(shape, chunk)
    dwfmg.dwf_fine_config(dwfmg.FINE_AUTO)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_pv_modes_fp64_parity(mode):
    Lx, Ly, Ls, nrhs, m, M5 = 32, 24, 8, 2, 0.01, -1.0
    U = gauge(Lx, Ly, 7)
    psi = inputs.gaussian_field((nrhs, Ls, Ly, Lx, 2), 8)
    got = dwfmg.dwf_pv_apply(torch.from_numpy(U).to(DEV), torch.from_numpy(psi).to(DEV), m, M5, mode=mode)
    want = {0: lambda: O.pv(U, psi, M5), 1: lambda: O.pv(U, psi, M5, dagger=True),
            2: lambda: O.pv_dag_dw(U, psi, m, M5), 3: lambda: O.pv_dag_dw_dagger(U, psi, m, M5)}[mode]()
    assert rel(got.cpu().numpy(), want) < 1e-13


def test_pv_inverse_mode_against_a_dense_solve():
    """DWF_PVINV_DW: D_PV^-1 D_DW psi (the exactly preconditioned operator of Sec. 2.2)
    against LU on the assembled D_PV of a small lattice, and on a larger one the
    defining property D_PV out = D_DW psi with the oracle's operators."""
    Lx, Ly, Ls, m, M5 = 8, 6, 4, 0.05, -1.0
    U = gauge(Lx, Ly, 11)
    psi = inputs.gaussian_field((2, Ls, Ly, Lx, 2), 12)
    got = dwfmg.dwf_pv_apply(torch.from_numpy(U).to(DEV), torch.from_numpy(psi).to(DEV), m, M5,
                             mode=dwfmg.DWF_PVINV_DW).cpu().numpy()
    shape = (Ls, Ly, Lx, 2)
    Dpv = O.assemble(lambda v: O.pv(U, v, M5), shape)
    for r in range(2):
        want = np.linalg.solve(Dpv, O.dwf(U, psi[r], m, M5).reshape(-1)).reshape(shape)
        assert rel(got[r], want) < 1e-10
    Lx, Ly, Ls = 32, 24, 8
    U = gauge(Lx, Ly, 13)
    psi = inputs.gaussian_field((1, Ls, Ly, Lx, 2), 14)
    got = dwfmg.dwf_pv_apply(torch.from_numpy(U).to(DEV), torch.from_numpy(psi).to(DEV), m, M5,
                             mode=dwfmg.DWF_PVINV_DW).cpu().numpy()
    rhs = O.dwf(U, psi[0], m, M5)
    assert rel(O.pv(U, got[0], M5), rhs) < 1e-11
    with pytest.raises(dwfmg.DwfError):
        dwfmg.dwf_pv_apply(torch.from_numpy(U).to(DEV).to(torch.complex64),
                           torch.from_numpy(psi).to(DEV).to(torch.complex64), m, M5, mode=dwfmg.DWF_PVINV_DW)


def test_dwf_full_size_fp64_and_fp32():
    """The 256^2 x Ls 16 operator of the solve benchmark, FP64 and FP32."""
    L, Ls, m, M5 = 256, 16, 0.01, -1.0
    U = inputs.metropolis_u1(L, L, 6.0, 20, 40256).U
    psi = inputs.gaussian_field((1, Ls, L, L, 2), 6256000)
    want = O.dwf(U, psi, m, M5)
    Ud, pd = torch.from_numpy(U).to(DEV), torch.from_numpy(psi).to(DEV)
    assert rel(dwfmg.dwf_apply(Ud, pd, m, M5).cpu().numpy(), want) < 1e-13
    got32 = dwfmg.dwf_apply(Ud.to(torch.complex64), pd.to(torch.complex64), m, M5).cpu().numpy()
    err32 = rel(got32.astype(np.complex128), want)
    print(f"FP32 D_DW relative error vs FP64 oracle: {err32:.2e}")
    assert err32 < 2e-7


@pytest.mark.parametrize("dagger", [False, True])
def test_dwf_bandwidth_shape_fp32_every_rhs(dagger):
    """512^2 x Ls 32 x 4 rhs (the stencil-bandwidth workload), FP32; the
    oracle recomputes every right-hand side in full from the same FP32 inputs."""
    L, Ls, nrhs, m, M5 = 512, 32, 4, 0.01, -1.0
    U = inputs.links_from_theta(inputs.random_theta(L, L, 8_000_000))
    psi = inputs.gaussian_field((nrhs, Ls, L, L, 2), 8_000_001).astype(np.complex64)
    got = dwfmg.dwf_apply(torch.from_numpy(U.astype(np.complex64)).to(DEV), torch.from_numpy(psi).to(DEV), m, M5,
                          dagger=dagger).cpu().numpy()
    U64 = U.astype(np.complex64).astype(np.complex128)
    for j in range(nrhs):
        want = O.dwf(U64, psi[j].astype(np.complex128), m, M5, dagger=dagger)
        err = rel(got[j].astype(np.complex128), want)
        assert err < 2e-7, f"rhs {j}: {err:.2e}"


@pytest.mark.parametrize("dagger", [False, True])
def test_wilson2d_parity(dagger):
    Lx, Ly, n = 20, 12, 3
    U = gauge(Lx, Ly, 9)
    psi = inputs.gaussian_field((n, Ly, Lx, 2), 10)
    got = dwfmg.dwf_wilson_apply(torch.from_numpy(U).to(DEV), torch.from_numpy(psi).to(DEV), -0.3, dagger=dagger)
    assert rel(got.cpu().numpy(), O.wilson(U, psi, -0.3, dagger=dagger)) < 1e-13


def test_gamma5R_bit_exact():
    psi = inputs.gaussian_field((3, 5, 6, 7, 2), 11)
    got = dwfmg.dwf_gamma5R(torch.from_numpy(psi).to(DEV)).cpu().numpy()
    assert np.array_equal(got, O.Gamma5(psi))
    got32 = dwfmg.dwf_gamma5R(torch.from_numpy(psi.astype(np.complex64)).to(DEV)).cpu().numpy()
    assert np.array_equal(got32, O.Gamma5(psi.astype(np.complex64).astype(np.complex128)).astype(np.complex64))


def test_gauge_transform_bit_exact_and_covariance():
    Lx, Ly, Ls = 24, 16, 4
    U = gauge(Lx, Ly, 12)
    g = inputs.random_phases((Ly, Lx), 13)
    psi = inputs.gaussian_field((2, Ls, Ly, Lx, 2), 14)
    Ug, psig = dwfmg.dwf_gauge_transform(torch.from_numpy(U).to(DEV), torch.from_numpy(g).to(DEV),
                                         torch.from_numpy(psi).to(DEV))
    assert np.array_equal(Ug.cpu().numpy(), O.gauge_transform_links(U, g))
    assert np.array_equal(psig.cpu().numpy(), O.gauge_transform_field(psi, g))
    # covariance of the GPU operator: D(U^g) g psi = g D(U) psi
    lhs = dwfmg.dwf_apply(Ug, psig, 0.02, -1.0).cpu().numpy()
    rhs = O.gauge_transform_field(O.dwf(U, psi, 0.02, -1.0), g)
    assert rel(lhs, rhs) < 1e-13


def test_pack_unpack_bit_exact():
    x = inputs.gaussian_field((1000, 3), 15)
    xd = torch.from_numpy(x).to(DEV)
    p = dwfmg.dwf_pack(xd)
    assert np.array_equal(p.cpu().numpy(), x.astype(np.complex64))
    assert np.array_equal(dwfmg.dwf_unpack(p).cpu().numpy(), x.astype(np.complex64).astype(np.complex128))


def test_force_parity():
    Lx, Ly, Ls, nrhs = 16, 12, 4, 2
    U = gauge(Lx, Ly, 16)
    X = inputs.gaussian_field((nrhs, Ls, Ly, Lx, 2), 17)
    Y = inputs.gaussian_field((nrhs, Ls, Ly, Lx, 2), 18)
    F = dwfmg.dwf_force(torch.from_numpy(U).to(DEV), torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV))
    want = O.force(U, X, Y)
    assert np.max(np.abs(F.cpu().numpy() - want)) < 1e-12 * np.max(np.abs(want))


def test_argument_errors_on_device():
    U = torch.ones((2, 4, 4), dtype=torch.complex128, device=DEV)
    psi = torch.ones((1, 4, 4, 4, 2), dtype=torch.complex128, device=DEV)
    with pytest.raises(dwfmg.DwfError) as e:
        dwfmg.dwf_apply(U, psi, 0.1, -1.0, out=psi)
    assert e.value.code == dwfmg.DWF_EINVAL
    with pytest.raises(ValueError):
        dwfmg.dwf_apply(U, psi.to(torch.complex64), 0.1, -1.0)


def test_links_from_theta():
    """U = exp(i theta) on the device against numpy's cos / sin of the same angles
    (the generator's links), to a couple of ulp."""
    theta = inputs.metropolis_u1(32, 16, 6.0, 20, 19).theta
    U = dwfmg.dwf_links_from_theta(torch.from_numpy(theta).to(DEV)).cpu().numpy()
    want = inputs.links_from_theta(theta)
    assert np.max(np.abs(U - want)) < 4e-16
