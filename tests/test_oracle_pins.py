"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form
printed in (or derived from) the paper, an exact invariant, a special case that
reduces to a library routine (dense LU / eigenvalues / SVD), or an exact
statistical result for the input generator.
"""
import math

import numpy as np
import pytest
import scipy.special

from oracle import dwf_oracle as O
from paper_2004_07732_amd import inputs

RNG = np.random.default_rng(1234)


def cgauss(shape, seed):
    return inputs.gaussian_field(shape, seed)


def hot_links(Lx, Ly, seed):
    return inputs.links_from_theta(inputs.random_theta(Lx, Ly, seed))


def plane_wave(Lx, Ly, p):
    yy, xx = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    return np.exp(1j * (p[0] * xx + p[1] * yy))


def wilson_momentum(p, M):
    """Free Wilson kernel in momentum space, M + sum_mu (1 - cos p + i gamma sin p)
    (Sec. 2.2, free-field limit; App. A)."""
    out = M * O.IDENT2
    for mu in (0, 1):
        out = out + (1 - math.cos(p[mu])) * O.IDENT2 + 1j * math.sin(p[mu]) * O.GAMMA[mu]
    return out


# ----------------------------------------------------------------------------- free field
@pytest.mark.parametrize("M", [0.0, -1.0, 0.37])
def test_free_wilson_plane_waves(M):
    Lx, Ly = 6, 4
    U = np.ones((2, Ly, Lx), dtype=np.complex128)
    for kx in range(Lx):
        for ky in range(Ly):
            p = (2 * math.pi * kx / Lx, 2 * math.pi * ky / Ly)
            chi = cgauss((2,), 100 * kx + ky)
            psi = plane_wave(Lx, Ly, p)[..., None] * chi
            got = O.wilson(U, psi, M)
            want = plane_wave(Lx, Ly, p)[..., None] * (wilson_momentum(p, M) @ chi)
            assert np.max(np.abs(got - want)) < 1e-14


def test_constant_field_shifts_momentum():
    """U_mu = e^{i phi_mu}: a plane wave of momentum p sees p + phi (derived from
    the gauge coupling of the Wilson operator, Sec. 2)."""
    Lx, Ly = 5, 4
    phi = (0.3, -1.1)
    U = np.stack([np.full((Ly, Lx), np.exp(1j * phi[0])), np.full((Ly, Lx), np.exp(1j * phi[1]))])
    p = (2 * math.pi * 2 / Lx, 2 * math.pi * 1 / Ly)
    chi = cgauss((2,), 7)
    psi = plane_wave(Lx, Ly, p)[..., None] * chi
    got = O.wilson(U, psi, -0.4)
    want = plane_wave(Lx, Ly, p)[..., None] * (wilson_momentum((p[0] + phi[0], p[1] + phi[1]), -0.4) @ chi)
    assert np.max(np.abs(got - want)) < 1e-14


def free_dw_block(p, Ls, m, M5, dagger=False):
    """2Ls x 2Ls momentum-space domain-wall matrix of eq. DWoperator (spin fastest)."""
    Dw = wilson_momentum(p, M5) + O.IDENT2
    if dagger:
        Dw = Dw.conj().T
    up, dn = (O.P_MINUS, O.P_PLUS) if not dagger else (O.P_PLUS, O.P_MINUS)
    M = np.zeros((Ls, 2, Ls, 2), dtype=np.complex128)
    for s in range(Ls):
        M[s, :, s, :] += Dw
        fac_up = -m if s == Ls - 1 else 1.0
        fac_dn = -m if s == 0 else 1.0
        M[s, :, (s + 1) % Ls, :] += fac_up * up
        M[s, :, (s - 1) % Ls, :] += fac_dn * dn
    return M.reshape(2 * Ls, 2 * Ls)


def test_free_dwf_plane_waves():
    Lx, Ly, Ls, m, M5 = 4, 6, 5, 0.07, -1.05
    U = np.ones((2, Ly, Lx), dtype=np.complex128)
    for (kx, ky) in [(0, 0), (1, 0), (3, 5), (2, 3)]:
        p = (2 * math.pi * kx / Lx, 2 * math.pi * ky / Ly)
        chi = cgauss((Ls, 2), kx * 10 + ky)
        pw = plane_wave(Lx, Ly, p)
        psi = pw[None, :, :, None] * chi[:, None, None, :]
        for dag in (False, True):
            got = O.dwf(U, psi, m, M5, dagger=dag)
            want_chi = (free_dw_block(p, Ls, m, M5, dagger=dag) @ chi.reshape(-1)).reshape(Ls, 2)
            want = pw[None, :, :, None] * want_chi[:, None, None, :]
            assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("Ls,m", [(4, 0.01), (8, 0.1), (5, 0.3), (16, 0.01)])
def test_p0_spectrum_closed_form(Ls, m):
    """Free field, M5 = -1, zero momentum: the eigenvalues of D_DW are
    m^{1/Ls} exp(i(2n+1)pi/Ls), each twice (Sec. 2.1, free-limit spectrum)."""
    Lx = Ly = 4
    U = np.ones((2, Ly, Lx), dtype=np.complex128)
    # isometry onto constant-in-x fields
    Q = np.zeros((Ls, Ly, Lx, 2, Ls * 2), dtype=np.complex128)
    for s in range(Ls):
        for a in range(2):
            Q[s, :, :, a, 2 * s + a] = 1.0 / math.sqrt(Lx * Ly)
    Qf = Q.reshape(-1, 2 * Ls)
    cols = O.dwf(U, np.moveaxis(Q, -1, 0), m, -1.0)
    B = Qf.conj().T @ cols.reshape(2 * Ls, -1).T
    ev = np.linalg.eigvals(B)
    want = np.array([m ** (1.0 / Ls) * np.exp(1j * (2 * n + 1) * math.pi / Ls) for n in range(Ls)] * 2)
    assert _match_sets(ev, want) < 1e-13
    # D_PV^{-1} D_DW on the same block: m twice, 1 with multiplicity 2(Ls-1)
    cols_pv = O.pv(U, np.moveaxis(Q, -1, 0), -1.0)
    Bpv = Qf.conj().T @ cols_pv.reshape(2 * Ls, -1).T
    ev2 = np.linalg.eigvals(np.linalg.solve(Bpv, B))
    want2 = np.array([m, m] + [1.0] * (2 * Ls - 2))
    assert _match_sets(ev2, want2) < 1e-10


def _match_sets(a, b):
    """Max distance of a greedy one-to-one matching of two eigenvalue lists."""
    a = list(np.asarray(a))
    worst = 0.0
    for v in np.asarray(b):
        d = [abs(v - w) for w in a]
        i = int(np.argmin(d))
        worst = max(worst, d[i])
        a.pop(i)
    return worst


def test_free_pv_normal_bounded_by_one():
    """Free field, M5 = -1: the squared singular values of D_PV are
    1 + (sum a)^2 - sum a^2 + 2 (sum a)(1 + cos p5), a_mu = 2 sin^2(p_mu/2),
    p5 = pi(2n+1)/Ls, each twice (App. A, free Pauli-Villars normal operator)."""
    Lx, Ly, Ls = 4, 6, 4
    U = np.ones((2, Ly, Lx), dtype=np.complex128)
    D = O.assemble(lambda v: O.pv(U, v, -1.0), (Ls, Ly, Lx, 2))
    sv2 = np.sort(np.linalg.svd(D, compute_uv=False) ** 2)
    want = []
    for kx in range(Lx):
        for ky in range(Ly):
            a = [2 * math.sin(math.pi * kx / Lx) ** 2, 2 * math.sin(math.pi * ky / Ly) ** 2]
            for n in range(Ls):
                p5 = math.pi * (2 * n + 1) / Ls
                v = 1 + sum(a) ** 2 - sum(x * x for x in a) + 2 * sum(a) * (1 + math.cos(p5))
                want += [v, v]
    want = np.sort(want)
    assert np.max(np.abs(sv2 - want)) < 1e-12
    assert sv2.min() > 1 - 1e-12


# ----------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("m", [0.01, 1.0])
def test_gamma5_hermiticity_and_adjoint(m):
    """Gamma5 D Gamma5 = D^dag with Gamma5 = gamma5 R (Sec. 2.1), and the dagger
    flag is the true adjoint: <chi, D psi> = <D^dag chi, psi>."""
    Lx, Ly, Ls, M5 = 6, 4, 6, -1.0
    U = hot_links(Lx, Ly, 5)
    psi = cgauss((2, Ls, Ly, Lx, 2), 11)
    chi = cgauss((2, Ls, Ly, Lx, 2), 12)
    Dpsi = O.dwf(U, psi, m, M5)
    Ddchi = O.dwf(U, chi, m, M5, dagger=True)
    assert abs(np.vdot(chi, Dpsi) - np.vdot(Ddchi, psi)) < 1e-12 * np.linalg.norm(chi) * np.linalg.norm(Dpsi)
    lhs = O.Gamma5(O.dwf(U, O.Gamma5(psi), m, M5))
    rhs = O.dwf(U, psi, m, M5, dagger=True)
    assert np.max(np.abs(lhs - rhs)) < 1e-14
    # dense: the dagger matrix is the conjugate transpose
    Us = hot_links(4, 4, 6)
    D = O.assemble(lambda v: O.dwf(Us, v, m, M5), (4, 4, 4, 2))
    Dd = O.assemble(lambda v: O.dwf(Us, v, m, M5, dagger=True), (4, 4, 4, 2))
    assert np.max(np.abs(Dd - D.conj().T)) < 1e-15


def test_normal_operator_is_square_of_gamma5_form():
    """D^dag D = (Gamma5 D)^2 (Sec. 2.1)."""
    Lx, Ly, Ls, m, M5 = 4, 4, 4, 0.05, -1.0
    U = hot_links(Lx, Ly, 9)
    psi = cgauss((Ls, Ly, Lx, 2), 3)
    g5d = lambda v: O.Gamma5(O.dwf(U, v, m, M5))
    lhs = O.dwf(U, O.dwf(U, psi, m, M5), m, M5, dagger=True)
    assert np.max(np.abs(lhs - g5d(g5d(psi)))) < 1e-13


def test_gauge_covariance():
    """D(U^g)(g psi) = g D(U) psi for a random U(1) rotation g."""
    Lx, Ly, Ls = 6, 4, 4
    U = hot_links(Lx, Ly, 21)
    g = inputs.random_phases((Ly, Lx), 22)
    psi = cgauss((Ls, Ly, Lx, 2), 23)
    Ug = O.gauge_transform_links(U, g)
    for dag in (False, True):
        lhs = O.dwf(Ug, O.gauge_transform_field(psi, g), 0.02, -1.0, dagger=dag)
        rhs = O.gauge_transform_field(O.dwf(U, psi, 0.02, -1.0, dagger=dag), g)
        assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_chiral_permutation_is_unitary_and_moves_walls():
    Ls = 5
    P = O.assemble(lambda v: O.chiral_permute(v), (Ls, 1, 1, 2))
    assert np.max(np.abs(P.conj().T @ P - np.eye(2 * Ls))) < 1e-15
    Pd = O.assemble(lambda v: O.chiral_permute_dagger(v), (Ls, 1, 1, 2))
    assert np.max(np.abs(Pd - P.conj().T)) < 1e-15
    psi = cgauss((Ls, 1, 1, 2), 1)
    w = O.chiral_permute_dagger(psi)[0]
    want = O.spin_mul(O.P_MINUS, psi[0]) + O.spin_mul(O.P_PLUS, psi[-1])
    assert np.max(np.abs(w - want)) == 0.0


# ----------------------------------------------------------------------------- spectra
def metropolis_links(L, beta, sweeps, seed):
    return inputs.metropolis_u1(L, L, beta, sweeps, seed).U


@pytest.mark.parametrize("Ls", [4, 6])
def test_pv_inverse_dw_spectrum(Ls):
    """D_PV^{-1} D_DW: exactly (Ls-1) 2V eigenvalues equal to 1 (eq. DWFmatrix);
    the other 2V lie in the disk of centre (1+m)/2, radius (1-m)/2 for even Ls
    and equal the eigenvalues of the overlap operator
    D_ov = (1+m)/2 + (1-m)/2 gamma5 eps_L[H], H = gamma5 D_W(M5)/(2 + D_W(M5))
    (eq. Overlap, App. B).  READING: eps_L = ((1+H)^L - (1-H)^L)/((1+H)^L + (1-H)^L),
    the sign that tends to sign(H) as L grows."""
    L, m, M5 = 4, 0.1, -1.0
    U = metropolis_links(L, 2.0, 20, 77)
    shape = (Ls, L, L, 2)
    D = O.assemble(lambda v: O.dwf(U, v, m, M5), shape)
    Dpv = O.assemble(lambda v: O.pv(U, v, M5), shape)
    ev = np.linalg.eigvals(np.linalg.solve(Dpv, D))
    V2 = 2 * L * L
    near1 = np.abs(ev - 1.0) < 1e-8
    assert near1.sum() >= (Ls - 1) * V2
    rest = ev[np.argsort(np.abs(ev - 1.0))[(Ls - 1) * V2:]]
    # overlap operator, dense 2V x 2V
    Dw = O.assemble(lambda v: O.wilson(U, v, M5), (L, L, 2))
    g5 = np.kron(np.eye(L * L), O.GAMMA5)
    I = np.eye(V2)
    H = g5 @ Dw @ np.linalg.inv(2 * I + Dw)
    Ap = np.linalg.matrix_power(I + H, Ls)
    Am = np.linalg.matrix_power(I - H, Ls)
    eps = (Ap - Am) @ np.linalg.inv(Ap + Am)
    Dov = 0.5 * (1 + m) * I + 0.5 * (1 - m) * g5 @ eps
    ev_ov = np.linalg.eigvals(Dov)
    assert _match_sets(rest, ev_ov) < 1e-8
    assert np.all(np.abs(rest - 0.5 * (1 + m)) <= 0.5 * (1 - m) + 1e-10)


def test_pv_dag_dw_right_half_plane():
    """spec(D_PV^dag D_DW) lies in Re(lambda) > 0 for m > 0 (App. B)."""
    L, Ls, m, M5 = 4, 4, 0.02, -1.0
    U = metropolis_links(L, 1.0, 10, 5)
    A = O.assemble(lambda v: O.pv_dag_dw(U, v, m, M5), (Ls, L, L, 2))
    ev = np.linalg.eigvals(A)
    assert ev.real.min() > 0.0


def test_dense_lu_vs_cgnr():
    """The domain-wall solve: dense LU (LAPACK) against the oracle's CGNR."""
    L, Ls, m, M5 = 4, 4, 0.05, -1.0
    U = metropolis_links(L, 3.0, 20, 8)
    shape = (Ls, L, L, 2)
    D = O.assemble(lambda v: O.dwf(U, v, m, M5), shape)
    b = cgauss(shape, 44)
    x_lu = np.linalg.solve(D, b.reshape(-1)).reshape(shape)
    x_cg, it = O.cgnr(lambda v: O.dwf(U, v, m, M5), lambda v: O.dwf(U, v, m, M5, dagger=True), b, 1e-14, 5000)
    assert np.linalg.norm(x_cg - x_lu) / np.linalg.norm(x_lu) < 1e-10


def _textbook_bicgstab(A, b, iters):
    """van der Vorst's BiCGStab (1992) written out independently, for the ell = 1 pin."""
    x = np.zeros_like(b)
    r = b.copy()
    rt = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for _ in range(iters):
        rho_new = np.vdot(rt, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A @ p
        alpha = rho_new / np.vdot(rt, v)
        s_ = r - alpha * v
        t = A @ s_
        omega = np.vdot(t, s_) / np.vdot(t, t)
        x = x + alpha * p + omega * s_
        r = s_ - omega * t
        rho = rho_new
    return x


def _random_nonnormal(n, seed):
    rng = np.random.default_rng(seed)
    A = 3.0 * np.eye(n) + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


@pytest.mark.parametrize("ell", [1, 2, 4, 6])
def test_bicgstab_l_solves_and_keeps_its_residual(ell):
    """BiCGStab(ell) solves a non-normal complex system (LAPACK solution), and its
    recursively updated residual is the true residual b - A x (a wrong update of
    x, r or u breaks the identity)."""
    A, b = _random_nonnormal(80, 3)
    x, cyc, ap = O.bicgstab_l(lambda v: A @ v, b, ell, 1e-12, 400)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10
    assert ap == 2 * ell * cyc
    # stop exactly when the true residual crosses the tolerance (within rounding)
    res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert res <= 1.5e-12


def test_bicgstab_1_is_textbook_bicgstab():
    """ell = 1 is van der Vorst's BiCGStab: the iterates agree step by step."""
    A, b = _random_nonnormal(50, 4)
    for k in (1, 3, 6):
        x1, _, _ = O.bicgstab_l(lambda v: A @ v, b, 1, 0.0, k)
        xt = _textbook_bicgstab(A, b, k)
        assert np.linalg.norm(x1 - xt) / np.linalg.norm(xt) < 1e-12


def _bicgstab_l_lstsq(A, b, ell, cycles):
    """BiCGStab(ell) with the minimal-residual step done as a dense least-squares
    problem: gamma = argmin |r_0 - sum_j gamma_j r_j| over the BiCG residuals
    r_j = A r_(j-1), then x += sum gamma_j r_(j-1), r_0 -= sum gamma_j r_j,
    u_0 -= sum gamma_j u_j.  Independent of the recurrences the oracle uses."""
    x = np.zeros_like(b)
    rt = b.copy()
    u = [np.zeros_like(b) for _ in range(ell + 1)]
    r = [np.zeros_like(b) for _ in range(ell + 1)]
    r[0] = b.copy()
    rho0 = alpha = omega = 1.0 + 0j
    for _ in range(cycles):
        rho0 = -omega * rho0
        for j in range(ell):
            rho1 = np.vdot(rt, r[j])
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = A @ u[j]
            alpha = rho0 / np.vdot(rt, u[j + 1])
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = A @ r[j]
            x = x + alpha * u[0]
        R = np.stack(r[1:], axis=1)
        gam = np.linalg.lstsq(R, r[0], rcond=None)[0]
        omega = gam[-1]
        x = x + sum(gam[j - 1] * r[j - 1] for j in range(1, ell + 1))
        r[0] = r[0] - R @ gam
        u[0] = u[0] - sum(gam[j - 1] * u[j] for j in range(1, ell + 1))
    return x


@pytest.mark.parametrize("ell", [2, 4])
def test_bicgstab_l_minimal_residual_step(ell):
    """The Gram-Schmidt recurrences of the minimal-residual step give the same
    iterates as solving that least-squares problem directly."""
    A, b = _random_nonnormal(50, 6)
    for k in (1, 2, 3):
        x1, _, _ = O.bicgstab_l(lambda v: A @ v, b, ell, 0.0, k)
        x2 = _bicgstab_l_lstsq(A, b, ell, k)
        assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-10


def test_fig1_baselines_solve_the_domain_wall_system():
    """The two baselines of the paper's comparison reach the true residual of
    D_DW x = b: CGNR on D_DW, and BiCGStab(6) on D_PV^dag D_DW x = D_PV^dag b
    (same x, since D_PV is invertible); both against dense LU."""
    L, Ls, m, M5 = 4, 4, 0.05, -1.0
    U = metropolis_links(L, 3.0, 20, 8)
    shape = (Ls, L, L, 2)
    D = O.assemble(lambda v: O.dwf(U, v, m, M5), shape)
    b = cgauss(shape, 45)
    x_lu = np.linalg.solve(D, b.reshape(-1)).reshape(shape)
    x1, it, ap = O.cgnr_true(lambda v: O.dwf(U, v, m, M5), lambda v: O.dwf(U, v, m, M5, dagger=True), b,
                             1e-12, 5000)
    assert ap == 2 * it + 1
    assert np.linalg.norm(b - O.dwf(U, x1, m, M5)) / np.linalg.norm(b) <= 1e-12
    assert np.linalg.norm(x1 - x_lu) / np.linalg.norm(x_lu) < 1e-8
    bp = O.pv(U, b, M5, dagger=True)
    x2, cyc, ap2 = O.bicgstab_l(lambda v: O.pv_dag_dw(U, v, m, M5), bp, 6, 1e-12, 500)
    assert np.linalg.norm(x2 - x_lu) / np.linalg.norm(x_lu) < 1e-8


# ----------------------------------------------------------------------------- coarse level
def make_prolongator(L, block, nvec, nc, seed):
    """Orthonormalised random prolongator on an L x L lattice."""
    V = cgauss((L, L, 2, nc, nvec), seed)
    return O.Prolongator(V=O.block_orthonormalize(V, block), block=block)


def dense_prolongator(P):
    Ly, Lx = P.V.shape[:2]
    cY, cX = P.coarse_shape
    return O.assemble(lambda e: O.prolong2d(P, e), (cY, cX, 2 * P.nvec))


@pytest.mark.parametrize("L,block,nvec", [(4, (4, 4), 3), (8, (4, 4), 4), (8, (2, 4), 3), (12, (4, 4), 5), (4, (2, 2), 4)])
def test_galerkin_equals_dense_product(L, block, nvec):
    """hat-D_W = P^dag D_W P (Sec. 2.3) for coarse extents 1, 2 and 3, and the
    projection keeps gamma5: gamma5 P = P sigma3, P^dag P = 1 (eq. gamma5)."""
    U = hot_links(L, L, 31)
    P = make_prolongator(L, block, nvec, 1, 32)
    Pd = dense_prolongator(P)
    assert np.max(np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1]))) < 1e-14
    g5 = np.kron(np.eye(L * L), O.GAMMA5)
    cY, cX = P.coarse_shape
    s3 = np.kron(np.eye(cY * cX), np.diag(O.chirality(nvec)))
    assert np.max(np.abs(g5 @ Pd - Pd @ s3)) == 0.0
    for M in (0.0, -0.3):
        Dw = O.assemble(lambda v: O.wilson(U, v, M), (L, L, 2))
        S = O.galerkin(O.wilson_stencil(U), P)
        Dc = O.assemble(lambda e: O.stencil_apply(S, e, shift_mass=M), (cY, cX, 2 * nvec))
        assert np.max(np.abs(Dc - Pd.conj().T @ Dw @ Pd)) < 1e-13
        Dcd = O.assemble(lambda e: O.stencil_apply(S, e, shift_mass=M, dagger=True), (cY, cX, 2 * nvec))
        assert np.max(np.abs(Dcd - Dc.conj().T)) < 1e-14
        assert np.max(np.abs(s3 @ Dc @ s3 - Dc.conj().T)) < 1e-13


def test_second_level_galerkin_and_stencil_form():
    """A coarse level built on a coarse stencil (3-level hierarchies) is again
    the dense Galerkin product; the fine D_W in stencil form equals D_W."""
    L = 8
    U = hot_links(L, L, 41)
    Sf = O.wilson_stencil(U)
    psi = cgauss((L, L, 2), 1)
    assert np.max(np.abs(O.stencil_apply(Sf, psi, shift_mass=-0.2) - O.wilson(U, psi, -0.2))) < 1e-14
    P1 = make_prolongator(L, (2, 2), 3, 1, 42)
    S1 = O.galerkin(Sf, P1)
    P2 = make_prolongator(4, (2, 2), 2, 3, 43)
    S2 = O.galerkin(S1, P2)
    D1 = O.assemble(lambda e: O.stencil_apply(S1, e), (4, 4, 6))
    P2d = dense_prolongator(P2)
    D2 = O.assemble(lambda e: O.stencil_apply(S2, e), (2, 2, 4))
    assert np.max(np.abs(D2 - P2d.conj().T @ D1 @ P2d)) < 1e-13


def test_full_rank_coarse_kernel_is_unitarily_similar():
    """nvec equal to the block dimension makes P unitary, so spec hat-D_W = spec D_W."""
    L = 4
    U = hot_links(L, L, 51)
    P = make_prolongator(L, (2, 2), 4, 1, 52)
    S = O.galerkin(O.wilson_stencil(U), P)
    Dc = O.assemble(lambda e: O.stencil_apply(S, e, shift_mass=-1.0), (2, 2, 8))
    Dw = O.assemble(lambda v: O.wilson(U, v, -1.0), (L, L, 2))
    assert _match_sets(np.linalg.eigvals(Dc), np.linalg.eigvals(Dw)) < 1e-10


def test_coarse_dw_is_projected_dw_when_Ls_kept():
    """With hat-Ls = Ls, hat-D_DW = (1 x P)^dag D_DW (1 x P) (Sec. 2.3)."""
    L, Ls, m, M5 = 4, 3, 0.05, -1.0
    U = hot_links(L, L, 61)
    P = make_prolongator(L, (2, 2), 2, 1, 62)
    S = O.galerkin(O.wilson_stencil(U), P)
    Pd = dense_prolongator(P)
    big = np.kron(np.eye(Ls), Pd)
    for dag in (False, True):
        D = O.assemble(lambda v: O.dwf(U, v, m, M5, dagger=dag), (Ls, L, L, 2))
        Dc = O.assemble(lambda e: O.stencil_dwf(S, e, m, M5, dagger=dag), (Ls, 2, 2, 4))
        assert np.max(np.abs(Dc - big.conj().T @ D @ big)) < 1e-13


def test_wall_transfer_adjoint_and_identity():
    """Restriction is the adjoint of prolongation; Restr(Prol(e)) = e on the
    coarse wall subspace; the bulk of a prolonged field is exactly zero
    (eq. TruncProjectInterpolate)."""
    L, Ls, Lsc, nvec = 8, 6, 4, 3
    P = make_prolongator(L, (4, 4), nvec, 1, 71)
    chir = np.array([1.0, -1.0])
    r = cgauss((Ls, L, L, 2), 72)
    e = cgauss((Lsc, 2, 2, 2 * nvec), 73)
    Pe = O.prolong_wall(P, e, chir, Ls)
    Rr = O.restrict_wall(P, r, chir, Lsc)
    assert abs(np.vdot(Pe, r) - np.vdot(e, Rr)) < 1e-12 * np.linalg.norm(r) * np.linalg.norm(e)
    assert np.all(Pe[1:Ls - 1] == 0)
    assert np.all(Pe[0][..., 0] == 0) and np.all(Pe[-1][..., 1] == 0)
    # wall subspace: P- on coarse slice 1, P+ on the last coarse slice
    s3 = O.chirality(nvec)
    ew = np.zeros_like(e)
    ew[0] = e[0] * (s3 < 0)
    ew[-1] = e[-1] * (s3 > 0)
    back = O.restrict_wall(P, O.prolong_wall(P, ew, chir, Ls), chir, Lsc)
    assert np.max(np.abs(back - ew)) < 1e-14


def test_slice1_transfer_against_the_wall_transfer():
    """The literal-slice toggle: adjoint pair, R P = 1 on coarse slice 1, support on
    slice 1 only, and on a field that lives on slice 1 with chirality - only it is
    exactly the wall transfer (which takes chirality - from slice 1 and
    chirality + from slice Ls); with chirality + on slice 1 the two differ."""
    L, Ls, Lsc, nvec = 8, 6, 4, 3
    P = make_prolongator(L, (4, 4), nvec, 1, 74)
    chir = np.array([1.0, -1.0])
    r = cgauss((Ls, L, L, 2), 75)
    e = cgauss((Lsc, 2, 2, 2 * nvec), 76)
    Pe = O.prolong_slice1(P, e, Ls)
    Rr = O.restrict_slice1(P, r, Lsc)
    assert abs(np.vdot(Pe, r) - np.vdot(e, Rr)) < 1e-12 * np.linalg.norm(r) * np.linalg.norm(e)
    assert np.all(Pe[1:] == 0) and np.all(Rr[1:] == 0)
    e1 = np.zeros_like(e)
    e1[0] = e[0]
    assert np.max(np.abs(O.restrict_slice1(P, O.prolong_slice1(P, e1, Ls), Lsc) - e1)) < 1e-14
    r2 = r.copy()
    r2[1:] = cgauss((Ls - 1, L, L, 2), 77)       # other slices do not enter
    assert np.array_equal(O.restrict_slice1(P, r2, Lsc), Rr)
    rm = np.zeros_like(r)
    rm[0][..., 1] = r[0][..., 1]                  # chirality - on slice 1
    assert np.max(np.abs(O.restrict_slice1(P, rm, Lsc) - O.restrict_wall(P, rm, chir, Lsc))) < 1e-14
    rp = np.zeros_like(r)
    rp[0][..., 0] = r[0][..., 0]                  # chirality + on slice 1: the wall transfer ignores it
    assert np.linalg.norm(O.restrict_wall(P, rp, chir, Lsc)) == 0.0
    assert np.linalg.norm(O.restrict_slice1(P, rp, Lsc)) > 0.1 * np.linalg.norm(rp)


def test_bulk_transfer_adjoint_identity_and_range():
    """The bulk transfer of Sec. 4.1: R P = 1 (P^dag P = 1 per slice), P is the
    adjoint of R, and a field in the range of P has zero local colinearity."""
    L, nc, nvec, Ls = 8, 1, 3, 4
    P = make_prolongator(L, (4, 4), nvec, nc, 60)
    ec = cgauss((Ls, 2, 2, 2 * nvec), 61)
    r = cgauss((Ls, L, L, 2 * nc), 62)
    assert np.allclose(O.restrict_bulk(P, O.prolong_bulk(P, ec)), ec, atol=1e-13)
    lhs = np.vdot(O.prolong_bulk(P, ec), r)
    rhs = np.vdot(ec, O.restrict_bulk(P, r))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    v = O.prolong_bulk(P, ec)
    assert np.linalg.norm(v - O.prolong_bulk(P, O.restrict_bulk(P, v))) < 1e-12 * np.linalg.norm(v)


@pytest.mark.parametrize("transfer", ["wall", "bulk"])
def test_mg_solve_with_either_transfer(transfer):
    """Both transfers give a working preconditioner: the MG solve reaches the
    tolerance and agrees with LU (L^_s = L_s for the bulk transfer)."""
    L, Ls, m, M5 = 8, 4, 0.05, -1.0
    U = metropolis_links(L, 3.0, 20, 9)
    shape = (Ls, L, L, 2)
    b = cgauss(shape, 63)
    starts = [cgauss((4, L, L, 2), 64)]
    params = O.MGParams(levels=[O.LevelParams(nvec=4, block=(4, 4), Ls=Ls, setup_iters=20)], transfer=transfer)
    mg = O.MG(U, Ls, m, M5, params, starts)
    x, it = mg.solve(b, 1e-10)
    D = O.assemble(lambda v: O.dwf(U, v, m, M5), shape)
    x_lu = np.linalg.solve(D, b.reshape(-1)).reshape(shape)
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-8


def test_oblique_projector_annihilates_galerkin_range():
    """With the bulk transfer and the exact Galerkin product R A P as hat-A, the
    oblique projector 1 - P (R A P)^{-1} R A vanishes on the range of P: a check
    of the composition order in the diagnostic."""
    L, Ls, m, M5 = 8, 4, 0.05, -1.0
    U = metropolis_links(L, 3.0, 20, 10)
    starts = [cgauss((2, L, L, 2), 65)]
    params = O.MGParams(levels=[O.LevelParams(nvec=2, block=(4, 4), Ls=Ls, setup_iters=10)], transfer="bulk")
    mg = O.MG(U, Ls, m, M5, params, starts)
    cshape = (Ls, 2, 2, 4)
    RAP = O.assemble(lambda e: mg.restrict(0, mg.A(0, mg.prolong(0, e))), cshape)
    inv = lambda rc: np.linalg.solve(RAP, rc.reshape(-1)).reshape(cshape)
    v = mg.prolong(0, cgauss(cshape, 66))
    assert mg.oblique_projector(v, inv) < 1e-10 * np.linalg.norm(v)
    w = cgauss((Ls, L, L, 2), 67)
    assert mg.oblique_projector(w, inv) > 1e-3 * np.linalg.norm(w)


def test_kcycle_with_exact_coarse_solve():
    """With no smoothing and an (essentially) exact coarsest solve the K-cycle
    preconditioner is Prol . hat-A^{-1} . Restr (Sec. 2.3 summary)."""
    L, Ls, m, M5 = 4, 4, 0.1, -1.0
    U = metropolis_links(L, 3.0, 10, 3)
    params = O.MGParams(levels=[O.LevelParams(nvec=2, block=(2, 2), Ls=2, setup_iters=20)],
                        smooth_iters=0, coarsest_tol=1e-14, coarsest_maxit=5000)
    starts = [cgauss((2, L, L, 2), 91)]
    mg = O.MG(U, Ls, m, M5, params, starts)
    r = cgauss((Ls, L, L, 2), 92)
    got = mg.kcycle(0, r)
    Ac = O.assemble(lambda v: mg.A(1, v), (2, 2, 2, 4))
    rc = mg.restrict(0, r)
    ec = np.linalg.solve(Ac, rc.reshape(-1)).reshape(rc.shape)
    want = mg.prolong(0, ec)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-11


@pytest.mark.parametrize("levels", [1, 2])
def test_mg_solve_meets_tolerance_and_matches_lu(levels):
    L, Ls, m, M5 = 8, 4, 0.05, -1.0
    U = metropolis_links(L, 4.0, 30, 12)
    lp = [O.LevelParams(nvec=4, block=(2, 2), Ls=4, setup_iters=50)]
    if levels == 2:
        lp.append(O.LevelParams(nvec=3, block=(2, 2), Ls=2, setup_iters=50))
    params = O.MGParams(levels=lp)
    starts = [cgauss((4, L, L, 2), 1)]
    if levels == 2:
        starts.append(cgauss((3, 4, 4, 8), 2))
    mg = O.MG(U, Ls, m, M5, params, starts)
    b = cgauss((Ls, L, L, 2), 3)
    x, it = mg.solve(b, 1e-10)
    res = np.linalg.norm(b - O.dwf(U, x, m, M5)) / np.linalg.norm(b)
    assert res <= 1e-10
    D = O.assemble(lambda v: O.dwf(U, v, m, M5), (Ls, L, L, 2))
    x_lu = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-7


def test_setup_relaxation_reduces_normal_residual():
    L = 8
    U = metropolis_links(L, 6.0, 30, 13)
    B = lambda v: O.wilson(U, O.wilson(U, v, 0.0, dagger=True), 0.0)
    v0 = cgauss((L, L, 2), 4)
    v, it = O.cg_homogeneous(B, v0, 1e-4, 250)
    assert it == 250 or np.linalg.norm(B(v)) <= 1e-4 * np.linalg.norm(B(v0))


# ----------------------------------------------------------------------------- force
def test_force_matches_finite_differences():
    """dS/dtheta for S = phi^dag (D^dag D)^{-1} phi against central differences
    of dense solves (h = 1e-5)."""
    L, Ls, m, M5 = 4, 4, 0.1, -1.0
    theta = inputs.random_theta(L, L, 3) * 0.3
    phi = cgauss((Ls, L, L, 2), 5)
    shape = (Ls, L, L, 2)

    def S_of(th):
        U = inputs.links_from_theta(th)
        D = O.assemble(lambda v: O.dwf(U, v, m, M5), shape)
        y = np.linalg.solve(D.conj().T, phi.reshape(-1))
        return float(np.vdot(y, y).real)

    U = inputs.links_from_theta(theta)
    D = O.assemble(lambda v: O.dwf(U, v, m, M5), shape)
    Y = np.linalg.solve(D.conj().T, phi.reshape(-1)).reshape(shape)
    X = np.linalg.solve(D, Y.reshape(-1)).reshape(shape)
    F = O.force(U, X, Y)
    h = 1e-5
    for (mu, y, x) in [(0, 0, 0), (1, 2, 3), (0, 3, 1), (1, 1, 1)]:
        tp = theta.copy(); tp[mu, y, x] += h
        tm = theta.copy(); tm[mu, y, x] -= h
        fd = (S_of(tp) - S_of(tm)) / (2 * h)
        assert abs(fd - F[mu, y, x]) < 1e-6 * max(1.0, abs(fd))


# ----------------------------------------------------------------------------- inputs
def test_metropolis_plaquette_matches_exact_result():
    """For the 2-d U(1) plaquette action the mean plaquette is I1(beta)/I0(beta)
    (up to finite-volume corrections that vanish like exp(-V)); the input
    generator must sample it."""
    beta = 6.0
    g = inputs.metropolis_u1(32, 32, beta, 300, 99)
    th = g.theta
    plaq = th[0] + np.roll(th[1], -1, axis=1) - np.roll(th[0], -1, axis=0) - th[1]
    mean = np.cos(plaq).mean()
    exact = scipy.special.i1(beta) / scipy.special.i0(beta)
    assert abs(mean - exact) < 0.01
    assert 0.2 < g.acceptance < 0.95


# ----------------------------------------------------------------------------- polynomial PV correction
def test_pv_poly_order_zero_is_the_paper_operator():
    """c = (1): the polynomial-corrected operator is A = D_PV^dag D_DW (Sec. 2.3)."""
    U = hot_links(6, 4, 41)
    psi = cgauss((5, 4, 6, 2), 42)
    assert np.array_equal(O.pv_poly_dw(U, psi, 0.05, -1.0, [1.0]), O.pv_dag_dw(U, psi, 0.05, -1.0))
    assert np.array_equal(O.pv_poly_dw(U, psi, 0.05, -1.0, [1.0], dagger=True),
                          O.pv_dag_dw_dagger(U, psi, 0.05, -1.0))


def test_pv_poly_free_plane_waves():
    """Free field: on chi e^{ip.x} the operator acts as the momentum-space product
    M_PV^dag p(M_PV M_PV^dag) M_DW (and M_DW^dag p(.) M_PV for the adjoint), with
    the 2 Ls x 2 Ls blocks of eq. DWoperator at momentum p."""
    Lx, Ly, Ls, m, M5 = 4, 6, 4, 0.03, -1.0
    U = np.ones((2, Ly, Lx), dtype=np.complex128)
    c = [0.7, -0.2, 0.05]
    for (kx, ky) in [(0, 0), (1, 2), (3, 5)]:
        p = (2 * math.pi * kx / Lx, 2 * math.pi * ky / Ly)
        Mdw = free_dw_block(p, Ls, m, M5)
        Mpv = free_dw_block(p, Ls, 1.0, M5)
        X = Mpv @ Mpv.conj().T
        P = sum(ck * np.linalg.matrix_power(X, k) for k, ck in enumerate(c))
        chi = cgauss((Ls, 2), 50 + kx * 10 + ky)
        pw = plane_wave(Lx, Ly, p)
        psi = pw[None, :, :, None] * chi[:, None, None, :]
        for dag, M in ((False, Mpv.conj().T @ P @ Mdw), (True, Mdw.conj().T @ P @ Mpv)):
            got = O.pv_poly_dw(U, psi, m, M5, c, dagger=dag)
            want = pw[None, :, :, None] * (M @ chi.reshape(-1)).reshape(Ls, 2)[:, None, None, :]
            assert np.max(np.abs(got - want)) < 1e-12


def test_pv_poly_neumann_truncation_gains_two_powers_of_momentum():
    """App. A: truncating the expansion of (1 + A_PV)^{-1}, A_PV = D_PV D_PV^dag - 1,
    after one more term corrects D_PV^{-1} ~ D_PV^dag p(D_PV D_PV^dag) by another two
    powers of p; the second-order coefficients are the printed (2, -1)."""
    assert np.array_equal(O.pv_poly_neumann(0), [1.0])
    assert np.array_equal(O.pv_poly_neumann(1), [2.0, -1.0])
    Ls, M5 = 8, -1.0

    def err(q, c):
        Mpv = free_dw_block((q, 0.5 * q), Ls, 1.0, M5)
        X = Mpv @ Mpv.conj().T
        P = sum(ck * np.linalg.matrix_power(X, k) for k, ck in enumerate(c))
        return np.linalg.norm(Mpv.conj().T @ P - np.linalg.inv(Mpv), 2)

    for order in (0, 1, 2):
        c = O.pv_poly_neumann(order)
        slope = math.log2(err(0.1, c) / err(0.05, c))
        assert abs(slope - 2 * (order + 1)) < 0.1, (order, slope)


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_pv_poly_chebyshev_is_minimax_and_positive(order):
    """The weighted coefficients: 1 - x p(x) equioscillates with the bound
    1 / T_n((b + a)/(b - a)), n = order + 1, on [a, b] (the Chebyshev minimax
    property), so x p(x) stays in (0, 2) there."""
    lo, hi = 1.0, 25.0
    c = O.pv_poly_chebyshev(order, lo, hi)
    x = np.linspace(lo, hi, 200001)
    xp = x * np.polynomial.polynomial.polyval(x, c)
    bound = 1.0 / math.cosh((order + 1) * math.acosh((hi + lo) / (hi - lo)))
    dev = np.abs(1.0 - xp)
    assert dev.max() <= bound * (1 + 1e-9)
    assert dev.max() >= bound * (1 - 1e-6)
    assert np.all(xp > 0) and np.all(xp < 2)
    # the extremes alternate in sign at order + 2 points
    ext = np.linspace(0, 1, order + 2) * math.pi
    xe = 0.5 * (hi + lo) - 0.5 * (hi - lo) * np.cos(ext)
    re = 1.0 - xe * np.polynomial.polynomial.polyval(xe, c)
    assert np.allclose(np.abs(re), bound, rtol=1e-9)
    assert np.all(np.sign(re[1:]) == -np.sign(re[:-1]))


def test_second_order_truncation_is_not_positive_on_the_free_spectrum():
    """App. A warns that 2 - D_PV D_PV^dag is not positive definite: on the free
    field (M5 = -1) the squared singular values of D_PV reach past 2 (towards 25),
    while the minimax polynomial on [1, 25] keeps x p(x) > 0 over all of them."""
    Lx, Ly, Ls = 8, 8, 8
    sig2 = []
    for kx in range(Lx):
        for ky in range(Ly):
            a = [2 * math.sin(math.pi * kx / Lx) ** 2, 2 * math.sin(math.pi * ky / Ly) ** 2]
            for n in range(Ls):
                p5 = math.pi * (2 * n + 1) / Ls
                sig2.append(1 + sum(a) ** 2 - sum(v * v for v in a) + 2 * sum(a) * (1 + math.cos(p5)))
    sig2 = np.array(sig2)
    assert sig2.min() >= 1 - 1e-12 and sig2.max() < 25
    assert np.any(2 - sig2 < 0)
    c = O.pv_poly_chebyshev(1, 1.0, 25.0)
    assert np.all(sig2 * np.polynomial.polynomial.polyval(sig2, c) > 0)
