"""Plain FP64 CPU oracle for the domain-wall multigrid hot path.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library itself never does, and it shares no code with the library.

Everything is complex128 numpy.  Each function cites the passage of the paper
(Brower, Clark, Howarth, Weinberg, "Multigrid for Chiral Lattice Fermions:
Domain Wall", arXiv:2004.07732) that defines it.

Conventions (readings of the paper where it is silent are marked READING):
  * 2-d periodic lattice, ``d = 2``; fields ``psi[..., y, x, spin]``;
    links ``U[mu, y, x]`` with mu=0 the x direction.
  * READING: gamma_1 = sigma_1, gamma_2 = sigma_2, gamma_5 = sigma_3, so that
    P_+ = diag(1, 0) and P_- = diag(0, 1).
  * 5-d fields ``psi[..., s, y, x, spin]`` with s = 0..Ls-1 standing for the
    paper's s = 1..Ls.
  * READING: M5 is the paper's signed bulk mass (negative in the domain-wall
    regime; the free-field optimum is -1).
  * A generic 2-d nearest-neighbour operator on sites with ``n`` dof is held
    in "stencil form" ``(diag[y, x, n, n], hop[h, y, x, n, n])`` with hop
    directions h = (+x, -x, +y, -y):
        (S psi)(x) = diag(x) psi(x) + sum_h hop_h(x) psi(x + h).
    Coarse operators (Galerkin products) are stored this way.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

# ----------------------------------------------------------------------------
# Dirac algebra (Sec. 2, Wilson operator and P_pm below the domain-wall matrix)
# ----------------------------------------------------------------------------
SIGMA1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMA3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
GAMMA = (SIGMA1, SIGMA2)          # gamma_mu, mu = 0 (x), 1 (y)
GAMMA5 = SIGMA3
IDENT2 = np.eye(2, dtype=np.complex128)
P_PLUS = 0.5 * (IDENT2 + GAMMA5)  # P_+ = (1 + gamma_5)/2
P_MINUS = 0.5 * (IDENT2 - GAMMA5)  # P_- = (1 - gamma_5)/2

# hop direction table: (mu, sign) for h = 0..3
HOPS = ((0, +1), (0, -1), (1, +1), (1, -1))
_SITE_AXIS = {0: -1, 1: -2}        # axis of x / y in a [..., y, x] site array


def spin_mul(mat: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Multiply every 2-spinor of ``psi[..., 2]`` by the 2x2 matrix ``mat``."""
    return np.einsum("ab,...b->...a", mat, psi)


def shift(f: np.ndarray, mu: int, sign: int, site_axes_from_end: int = 1) -> np.ndarray:
    """Return g with g(x) = f(x + sign*mu_hat) on the periodic lattice.

    ``site_axes_from_end`` is the number of trailing non-site axes (1 for a
    spinor index, 1 for a coarse dof index, 0 for a scalar field).
    """
    axis = _SITE_AXIS[mu] - site_axes_from_end
    return np.roll(f, -sign, axis=axis)


# ----------------------------------------------------------------------------
# Wilson operator (Sec. 2, the Wilson discretization D_W(U, m))
# ----------------------------------------------------------------------------
def wilson(U: np.ndarray, psi: np.ndarray, M: float, dagger: bool = False) -> np.ndarray:
    """D_W(M) psi, or its adjoint, for psi[..., y, x, 2].

    D_W(M)psi(x) = (d + M) psi(x)
                   - sum_mu [ (1-gamma_mu)/2 U_mu(x) psi(x+mu)
                              + (1+gamma_mu)/2 U_mu(x-mu)^* psi(x-mu) ].
    The adjoint is the conjugate transpose of that matrix: the two spin
    projectors trade places and the links stay where they are.
    """
    d = 2
    out = (d + M) * psi
    for mu in (0, 1):
        fwd_proj = 0.5 * (IDENT2 - GAMMA[mu])
        bwd_proj = 0.5 * (IDENT2 + GAMMA[mu])
        if dagger:
            fwd_proj, bwd_proj = bwd_proj, fwd_proj
        link_fwd = U[mu][..., None]                                   # U_mu(x)
        link_bwd = np.conj(shift(U[mu], mu, -1, site_axes_from_end=0))[..., None]  # U_mu(x-mu)^*
        out = out - spin_mul(fwd_proj, link_fwd * shift(psi, mu, +1))
        out = out - spin_mul(bwd_proj, link_bwd * shift(psi, mu, -1))
    return out


# ----------------------------------------------------------------------------
# Shamir domain-wall operator (Sec. 2, eq. DWoperator) and Pauli-Villars
# ----------------------------------------------------------------------------
def s_hop(psi: np.ndarray, m: float, proj_up: np.ndarray, proj_dn: np.ndarray,
          spin_axis_mul: Callable) -> np.ndarray:
    """Fifth-dimension part of the domain-wall matrix.

    Row s of eq. DWoperator couples slice s to slice s+1 through P_- and to
    slice s-1 through P_+, with the corner blocks -m P_+ (row 1, column Ls) and
    -m P_- (row Ls, column 1).  ``proj_up`` multiplies psi_{s+1}, ``proj_dn``
    multiplies psi_{s-1}; the slice axis is axis -4 of a fine field or the
    equivalent axis of a coarse field (the caller passes ``spin_axis_mul``).
    """
    up = np.roll(psi, -1, axis=-4).copy()   # psi_{s+1}
    up[..., -1, :, :, :] *= -m              # psi_{Ls+1} := -m psi_1
    dn = np.roll(psi, +1, axis=-4).copy()   # psi_{s-1}
    dn[..., 0, :, :, :] *= -m               # psi_0 := -m psi_Ls
    return spin_axis_mul(proj_up, up) + spin_axis_mul(proj_dn, dn)


def dwf(U: np.ndarray, psi: np.ndarray, m: float, M5: float, dagger: bool = False) -> np.ndarray:
    """Shamir D_DW(m) psi for psi[..., Ls, y, x, 2] (eq. DWoperator).

    Diagonal blocks D_W(M5) + 1; the adjoint is the conjugate transpose of the
    block matrix: D_W -> D_W^dagger and the roles of P_+ and P_- in the
    fifth-dimension hop are exchanged (the corners keep their -m).
    """
    diag = wilson(U, psi, M5, dagger=dagger) + psi
    if not dagger:
        return diag + s_hop(psi, m, P_MINUS, P_PLUS, spin_mul)
    return diag + s_hop(psi, m, P_PLUS, P_MINUS, spin_mul)


def pv(U: np.ndarray, psi: np.ndarray, M5: float, dagger: bool = False) -> np.ndarray:
    """Pauli-Villars operator D_PV = D_DW(1) (Sec. 2.2)."""
    return dwf(U, psi, 1.0, M5, dagger=dagger)


def pv_dag_dw(U: np.ndarray, psi: np.ndarray, m: float, M5: float) -> np.ndarray:
    """A = D_PV^dagger D_DW(m), the approximate PV-preconditioned operator
    (Sec. 2.3, eq. NormalExp and the K-cycle summary)."""
    return pv(U, dwf(U, psi, m, M5), M5, dagger=True)


def pv_dag_dw_dagger(U: np.ndarray, psi: np.ndarray, m: float, M5: float) -> np.ndarray:
    """A^dagger = D_DW(m)^dagger D_PV."""
    return dwf(U, pv(U, psi, M5), m, M5, dagger=True)


def pv_normal(U: np.ndarray, psi: np.ndarray, M5: float) -> np.ndarray:
    """X = D_PV D_PV^dagger, the operator whose inverse the PV preconditioning
    of Sec. 2.3 truncates to 1 (eq. NormalExp)."""
    return pv(U, pv(U, psi, M5, dagger=True), M5)


def pv_poly_dw(U: np.ndarray, psi: np.ndarray, m: float, M5: float, c, dagger: bool = False) -> np.ndarray:
    """Polynomial correction of the PV preconditioning (the remark after
    eq. NormalExp and the expansion at the end of App. A): (D_PV D_PV^dag)^{-1}
    is replaced by p(X) = sum_k c_k X^k instead of by 1, giving
        A_p = D_PV^dagger p(X) D_DW(m),     c = (1): A of the paper;
        A_p^dagger = D_DW(m)^dagger p(X) D_PV   (p(X) is Hermitian for real c).
    The powers of X are summed term by term."""
    w = pv(U, psi, M5) if dagger else dwf(U, psi, m, M5)
    y = np.zeros_like(w)
    Xk = w
    for k, ck in enumerate(c):
        if k > 0:
            Xk = pv_normal(U, Xk, M5)
        y = y + ck * Xk
    return dwf(U, y, m, M5, dagger=True) if dagger else pv(U, y, M5, dagger=True)


def pv_poly_neumann(order: int):
    """c_k of the expansion of (1 + A_PV)^{-1}, A_PV = X - 1, truncated after
    A_PV^order and rewritten in powers of X (App. A): order 0 gives (1), order 1
    the paper's (2, -1)."""
    c = np.zeros(order + 1)
    for j in range(order + 1):          # (-1)^j (X - 1)^j
        for k in range(j + 1):
            c[k] += (-1) ** j * math.comb(j, k) * (-1) ** (j - k)
    return c


def pv_poly_chebyshev(order: int, lam_min: float, lam_max: float):
    """c_k of the polynomial p of degree `order` that minimises max |1 - x p(x)|
    over [lam_min, lam_max]: 1 - x p(x) = T_{n}(t(x)) / T_{n}(t(0)), n = order + 1,
    t(x) = (lam_max + lam_min - 2 x) / (lam_max - lam_min).  READING: the paper
    asks for the coefficients to be weighted over the whole spectrum (App. A)
    without fixing a weighting; this minimax choice keeps x p(x) in (0, 2) on
    the interval, so A_p stays in the right half plane where A is."""
    from numpy.polynomial import chebyshev as npc
    from numpy.polynomial import polynomial as npp
    n = order + 1
    a = (lam_max + lam_min) / (lam_max - lam_min)
    b = -2.0 / (lam_max - lam_min)
    tn = npc.cheb2poly([0.0] * n + [1.0])      # T_n(t) as a power series in t
    r = np.zeros(1)
    for coef in tn[::-1]:                       # Horner in t = a + b x
        r = npp.polyadd(npp.polymul(r, [a, b]), [coef])
    r = r / r[0]                                # r(x) = 1 - x p(x), r(0) = 1
    return -np.asarray(r[1:], dtype=np.float64)


def gamma5_field(psi: np.ndarray) -> np.ndarray:
    return spin_mul(GAMMA5, psi)


def reflect_s(psi: np.ndarray) -> np.ndarray:
    """R: slice s -> slice Ls+1-s (Sec. 2.1, the reflection in the extra dimension)."""
    return psi[..., ::-1, :, :, :].copy()


def Gamma5(psi: np.ndarray) -> np.ndarray:
    """Gamma_5 = gamma_5 R (Sec. 2.1)."""
    return gamma5_field(reflect_s(psi))


def chiral_permute(chi: np.ndarray, chir: Optional[np.ndarray] = None) -> np.ndarray:
    """Apply the chiral permutation matrix calP of Sec. 2.2 to chi[..., s, ...].

    Row s (< Ls) holds P_- at column s and P_+ at column s+1; row Ls holds P_+
    at column 1 and P_- at column Ls.  ``chir`` is the chirality (+1/-1) of each
    dof of the site (default: the fine spin, gamma_5 = sigma_3).
    """
    pp, pm = _chiral_masks(chi, chir)
    nxt = np.roll(chi, -1, axis=-4)      # chi_{s+1}, and chi_1 for row Ls
    return pm * chi + pp * nxt


def chiral_permute_dagger(psi: np.ndarray, chir: Optional[np.ndarray] = None) -> np.ndarray:
    """calP^dagger: (calP^dagger Psi)_s = P_- Psi_s + P_+ Psi_{s-1}, with
    Psi_0 read as Psi_Ls.  Slice 1 of the result is the wall field
    P_- Psi_1 + P_+ Psi_Ls of Sec. 2.2."""
    pp, pm = _chiral_masks(psi, chir)
    prv = np.roll(psi, +1, axis=-4)
    return pm * psi + pp * prv


def _chiral_masks(f: np.ndarray, chir: Optional[np.ndarray]):
    if chir is None:
        chir = np.array([1.0, -1.0])
    chir = np.asarray(chir, dtype=np.float64)
    assert f.shape[-1] == chir.shape[0]
    pp = (chir > 0).astype(np.float64)
    pm = (chir < 0).astype(np.float64)
    return pp, pm


# ----------------------------------------------------------------------------
# Gauge transformation and fermion force
# ----------------------------------------------------------------------------
def cmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Complex product with the real arithmetic spelled out: re = ar*br - ai*bi,
    im = ar*bi + ai*br, each product and sum rounded on its own (no fusion)."""
    ar, ai = np.real(a), np.imag(a)
    br, bi = np.real(b), np.imag(b)
    out = np.empty(np.broadcast(a, b).shape, dtype=np.complex128)
    out.real = ar * br - ai * bi
    out.imag = ar * bi + ai * br
    return out


def gauge_transform_links(U: np.ndarray, g: np.ndarray) -> np.ndarray:
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^*, evaluated as (g(x) U) g(x+mu)^*."""
    out = np.empty_like(U)
    for mu in (0, 1):
        out[mu] = cmul(cmul(g, U[mu]), np.conj(shift(g, mu, +1, site_axes_from_end=0)))
    return out


def gauge_transform_field(psi: np.ndarray, g: np.ndarray) -> np.ndarray:
    """psi^g(x) = g(x) psi(x) for every slice, spin and rhs."""
    return cmul(g[..., None], psi)


def force(U: np.ndarray, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """dS/dtheta_mu(x) for S = phi^dag (D^dag D)^{-1} phi, D = D_DW(m).

    With Y = D^{-dag} phi and X = D^{-1} Y one has dS = -2 Re(Y^dag dD X), and
    only the Wilson hops of D depend on theta (U = e^{i theta}, Sec. 2):
      F_mu(x) = 2 Re sum_s [ i U_mu(x) Y_s(x)^dag (1-gamma_mu)/2 X_s(x+mu)
                           - i U_mu(x)^* Y_s(x+mu)^dag (1+gamma_mu)/2 X_s(x) ].
    X and Y are [..., Ls, y, x, 2]; leading axes are summed.  Returns F[mu, y, x].
    """
    F = np.zeros(U.shape, dtype=np.float64)
    for mu in (0, 1):
        pm = 0.5 * (IDENT2 - GAMMA[mu])
        pp = 0.5 * (IDENT2 + GAMMA[mu])
        t1 = np.einsum("...a,...a->...", np.conj(Y), spin_mul(pm, shift(X, mu, +1)))
        t2 = np.einsum("...a,...a->...", np.conj(shift(Y, mu, +1)), spin_mul(pp, X))
        t1 = t1.reshape((-1,) + U.shape[1:]).sum(axis=0)
        t2 = t2.reshape((-1,) + U.shape[1:]).sum(axis=0)
        F[mu] = 2.0 * np.real(1j * U[mu] * t1 - 1j * np.conj(U[mu]) * t2)
    return F


def action(U, phi, m, M5, solve) -> float:
    """S = phi^dag (D^dag D)^{-1} phi = |D^{-dag} phi|^2 (used by gradient checks)."""
    Y = solve_dagger(U, phi, m, M5, solve)
    return float(np.vdot(Y, Y).real)


def solve_dagger(U, phi, m, M5, solve):
    """Y = D^{-dag} phi via Gamma5 D^{-1} Gamma5 phi (Gamma5-hermiticity, Sec. 2.1)."""
    return Gamma5(solve(Gamma5(phi)))


# ----------------------------------------------------------------------------
# Generic 2-d stencils (coarse Wilson kernels, Sec. 2.3 "Wilson kernel MG projection")
# ----------------------------------------------------------------------------
@dataclass
class Stencil:
    """2-d nearest-neighbour operator: diag[y, x, n, n], hop[4, y, x, n, n]."""
    diag: np.ndarray
    hop: np.ndarray
    chir: np.ndarray          # chirality (+1/-1) of each of the n dof (sigma_3)

    @property
    def n(self) -> int:
        return self.diag.shape[-1]

    @property
    def shape2d(self):
        return self.diag.shape[:2]


def stencil_apply(S: Stencil, psi: np.ndarray, shift_mass: float = 0.0,
                  dagger: bool = False) -> np.ndarray:
    """(S + shift_mass*I) psi, or its adjoint, for psi[..., y, x, n].

    The adjoint is the conjugate transpose of the sparse matrix: the block on
    site x from site x+h is hop_h(x); its transpose lives on site x+h and
    reaches x = (x+h) - h, i.e. (S^dag psi)(x) = diag(x)^dag psi(x)
    + sum_h hop_h(x-h)^dag psi(x-h).
    """
    if not dagger:
        out = np.einsum("yxab,...yxb->...yxa", S.diag, psi) + shift_mass * psi
        for h, (mu, sgn) in enumerate(HOPS):
            out = out + np.einsum("yxab,...yxb->...yxa", S.hop[h], shift(psi, mu, sgn))
        return out
    out = np.einsum("yxba,...yxb->...yxa", np.conj(S.diag), psi) + shift_mass * psi
    for h, (mu, sgn) in enumerate(HOPS):
        hop_back = shift(S.hop[h], mu, -sgn, site_axes_from_end=2)     # hop_h(x - h)
        out = out + np.einsum("yxba,...yxb->...yxa", np.conj(hop_back), shift(psi, mu, -sgn))
    return out


def wilson_stencil(U: np.ndarray) -> Stencil:
    """Stencil form of the fine D_W(0): diag = d*1, hop_{+mu}(x) =
    -(1-gamma_mu)/2 U_mu(x), hop_{-mu}(x) = -(1+gamma_mu)/2 U_mu(x-mu)^* (Sec. 2)."""
    Ly, Lx = U.shape[1:]
    diag = np.broadcast_to(2.0 * IDENT2, (Ly, Lx, 2, 2)).copy()
    hop = np.zeros((4, Ly, Lx, 2, 2), dtype=np.complex128)
    for h, (mu, sgn) in enumerate(HOPS):
        if sgn > 0:
            hop[h] = -0.5 * (IDENT2 - GAMMA[mu])[None, None] * U[mu][..., None, None]
        else:
            ub = np.conj(shift(U[mu], mu, -1, site_axes_from_end=0))
            hop[h] = -0.5 * (IDENT2 + GAMMA[mu])[None, None] * ub[..., None, None]
    return Stencil(diag=diag, hop=hop, chir=np.array([1.0, -1.0]))


def stencil_dwf(S: Stencil, psi: np.ndarray, m: float, M5: float,
                dagger: bool = False) -> np.ndarray:
    """Coarse D_DW(m) (eq. coarsenDW): diagonal blocks D_W(M5) + 1 built on the
    stencil S (which holds the kernel at zero mass), fifth-dimension hops
    through hat-P_pm = (1 pm sigma_3)/2, the same -m corners.  For psi[..., Ls, y, x, n]."""
    pp, pm = _chiral_masks(psi, S.chir)
    diag = stencil_apply(S, psi, shift_mass=M5 + 1.0, dagger=dagger)
    proj = lambda P, f: P * f      # hat-P_pm are diagonal in this basis
    if not dagger:
        return diag + s_hop(psi, m, pm, pp, proj)
    return diag + s_hop(psi, m, pp, pm, proj)


# ----------------------------------------------------------------------------
# Prolongator, Galerkin product, wall transfer (Sec. 2.3)
# ----------------------------------------------------------------------------
@dataclass
class Prolongator:
    """Block aggregation prolongator of one level.

    ``V[y, x, c, j, k]``: fine site (y, x), chirality c (0: +, 1: -), internal
    dof j of that chirality (nc of them), coarse vector k (nvec of them).
    Fine dof index is c*nc + j; coarse dof index is c*nvec + k.
    """
    V: np.ndarray
    block: tuple             # (by, bx)

    @property
    def nc(self):
        return self.V.shape[3]

    @property
    def nvec(self):
        return self.V.shape[4]

    @property
    def coarse_shape(self):
        Ly, Lx = self.V.shape[:2]
        return (Ly // self.block[0], Lx // self.block[1])


def _block_view(f: np.ndarray, block, lead: int):
    """Reshape [..., y, x, rest...] -> [..., Y, by, X, bx, rest...]."""
    by, bx = block
    shp = f.shape
    Ly, Lx = shp[lead], shp[lead + 1]
    return f.reshape(shp[:lead] + (Ly // by, by, Lx // bx, bx) + shp[lead + 2:])


def prolong2d(P: Prolongator, ec: np.ndarray) -> np.ndarray:
    """P e: fine[x][c][j] = sum_k V[x][c][j][k] e[X(x)][c][k] (ec[..., Y, X, 2*nvec])."""
    by, bx = P.block
    nv, nc = P.nvec, P.nc
    lead = ec.shape[:-3]
    e = ec.reshape(lead + ec.shape[-3:-1] + (2, nv))
    e = np.repeat(np.repeat(e, by, axis=-4), bx, axis=-3)   # broadcast coarse -> fine sites
    out = np.einsum("yxcjk,...yxck->...yxcj", P.V, e)
    return out.reshape(lead + out.shape[-4:-2] + (2 * nc,))


def restrict2d(P: Prolongator, r: np.ndarray) -> np.ndarray:
    """P^dagger r: coarse[X][c][k] = sum_{x in X} sum_j V[x][c][j][k]^* r[x][c][j]."""
    nv, nc = P.nvec, P.nc
    lead = r.shape[:-3]
    rf = r.reshape(lead + r.shape[-3:-1] + (2, nc))
    t = np.einsum("yxcjk,...yxcj->...yxck", np.conj(P.V), rf)
    nl = len(lead)
    tb = _block_view(t, P.block, nl)
    out = tb.sum(axis=(nl + 1, nl + 3))
    return out.reshape(lead + out.shape[nl:nl + 2] + (2 * nv,))


def restrict_bulk(P: Prolongator, r: np.ndarray) -> np.ndarray:
    """Sec. 4.1's alternative to the boundary-only transfer: the 2-d restriction
    repeated on every slice, coarse slice s from fine slice s (L^_s = L_s)."""
    return restrict2d(P, r)


def prolong_bulk(P: Prolongator, ec: np.ndarray) -> np.ndarray:
    """Adjoint of restrict_bulk: the 2-d prolongation on every slice."""
    return prolong2d(P, ec)


def chirality(n_per_chir: int) -> np.ndarray:
    """sigma_3 on a site with chirality-major dof ordering."""
    return np.concatenate([np.ones(n_per_chir), -np.ones(n_per_chir)])


def block_orthonormalize(V: np.ndarray, block) -> np.ndarray:
    """Per block and per chirality, classical Gram-Schmidt applied twice to
    the columns k = 0..nvec-1 in order, giving P^dagger P = 1 (Sec. 2.3,
    "normalization convention of the restrictor")."""
    Ly, Lx, _, nc, nv = V.shape
    by, bx = block
    Vb = V.reshape(Ly // by, by, Lx // bx, bx, 2, nc, nv)
    Vb = Vb.transpose(0, 2, 4, 1, 3, 5, 6).reshape(Ly // by, Lx // bx, 2, by * bx * nc, nv).copy()
    for k in range(nv):
        v = Vb[..., k]
        for _ in range(2):
            if k > 0:
                Q = Vb[..., :k]
                coeff = np.einsum("...ik,...i->...k", np.conj(Q), v)
                v = v - np.einsum("...ik,...k->...i", Q, coeff)
        nrm = np.sqrt(np.einsum("...i,...i->...", np.conj(v), v).real)
        Vb[..., k] = v / nrm[..., None]
    Vb = Vb.reshape(Ly // by, Lx // bx, 2, by, bx, nc, nv).transpose(0, 3, 1, 4, 2, 5, 6)
    return Vb.reshape(Ly, Lx, 2, nc, nv).copy()


def fine_to_chiral_columns(v: np.ndarray, chir: np.ndarray) -> np.ndarray:
    """Chiral doubling (Sec. 3.1): P_+ v_k and P_- v_k as the columns of the
    two chiralities.  v[k, y, x, n] -> V[y, x, 2, n/2, nvec] (dof chirality-major)."""
    nv, Ly, Lx, n = v.shape
    nc = n // 2
    assert np.all(chir[:nc] > 0) and np.all(chir[nc:] < 0)
    V = v.reshape(nv, Ly, Lx, 2, nc).transpose(1, 2, 3, 4, 0)
    return V.copy()


def galerkin(S: Stencil, P: Prolongator) -> Stencil:
    """Coarse kernel hat-D = P^dagger S P (Sec. 2.3, "Wilson kernel MG projection").

    Term by term: a hop of type h from fine site x to x+h contributes
    V(x)^dagger hop_h(x) V(x+h) to the coarse block (X(x), X(x+h)).  It lands
    in the coarse diagonal when x+h lies in the same aggregate and in the
    coarse hop of type h otherwise; the test is on the fine local coordinate
    (a forward hop leaves the aggregate exactly when x_mu mod b_mu = b_mu - 1),
    which stays right for coarse extents 1 and 2 with periodic wrap.
    """
    Ly, Lx = S.shape2d
    by, bx = P.block
    cY, cX = Ly // by, Lx // bx
    nv = P.nvec
    n = 2 * nv
    # W[y, x, a, b]: fine dof a -> coarse dof b, block-diagonal in chirality
    W = np.zeros((Ly, Lx, S.n, n), dtype=np.complex128)
    nc = P.nc
    W[:, :, :nc, :nv] = P.V[:, :, 0]
    W[:, :, nc:, nv:] = P.V[:, :, 1]
    WH = np.conj(W).swapaxes(-1, -2)

    def block_sum(f):  # f[y, x, n, n] -> [Y, X, n, n]
        return f.reshape(cY, by, cX, bx, n, n).sum(axis=(1, 3))

    cdiag = block_sum(WH @ S.diag @ W)
    chop = np.zeros((4, cY, cX, n, n), dtype=np.complex128)
    yy, xx = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    for h, (mu, sgn) in enumerate(HOPS):
        coord = xx if mu == 0 else yy
        b = bx if mu == 0 else by
        leaves = (coord % b == b - 1) if sgn > 0 else (coord % b == 0)
        Wn = shift(W, mu, sgn, site_axes_from_end=2)          # W(x + h)
        term = WH @ S.hop[h] @ Wn
        inside = np.where(leaves[..., None, None], 0.0, term)
        outside = np.where(leaves[..., None, None], term, 0.0)
        cdiag = cdiag + block_sum(inside)
        chop[h] = block_sum(outside)
    return Stencil(diag=cdiag, hop=chop, chir=chirality(nv))


def restrict_wall(P: Prolongator, r: np.ndarray, chir_f: np.ndarray, Ls_c: int) -> np.ndarray:
    """Wall-only restriction (eq. TruncProjectInterpolate) of r[..., Ls, y, x, n].

    In the permuted chiral basis (Sec. 2.2) both walls sit on slice 1:
    the coarse residual is P^dagger (calP^dagger r)_1 on coarse slice 1 and zero
    elsewhere, expressed back in the unpermuted coarse basis with hat-calP.
    READING: "the boundary at s = 1" is slice 1 of the permuted basis.
    """
    w = chiral_permute_dagger(r, chir_f)[..., 0, :, :, :]
    wc = restrict2d(P, w)
    lead = r.shape[:-4]
    chat = np.zeros(lead + (Ls_c,) + wc.shape[-3:], dtype=np.complex128)
    chat[..., 0, :, :, :] = wc
    return chiral_permute(chat, chirality(P.nvec))


def prolong_wall(P: Prolongator, ec: np.ndarray, chir_f: np.ndarray, Ls_f: int) -> np.ndarray:
    """Wall-only prolongation (eq. TruncProjectInterpolate): e = calP [P (hat-calP^dagger e)_1, 0, ..., 0]."""
    w = chiral_permute_dagger(ec, chirality(P.nvec))[..., 0, :, :, :]
    wf = prolong2d(P, w)
    lead = ec.shape[:-4]
    perm = np.zeros(lead + (Ls_f,) + wf.shape[-3:], dtype=np.complex128)
    perm[..., 0, :, :, :] = wf
    return chiral_permute(perm, chir_f)


def restrict_slice1(P: Prolongator, r: np.ndarray, Ls_c: int) -> np.ndarray:
    """The other reading of eq. TruncProjectInterpolate's "s = 1", kept as a
    test toggle: both chiralities of the unpermuted fine slice 1, restricted by
    the 2-d P^dagger onto the unpermuted coarse slice 1, zero elsewhere (no
    chiral permutation on either level)."""
    wc = restrict2d(P, r[..., 0, :, :, :])
    chat = np.zeros(r.shape[:-4] + (Ls_c,) + wc.shape[-3:], dtype=np.complex128)
    chat[..., 0, :, :, :] = wc
    return chat


def prolong_slice1(P: Prolongator, ec: np.ndarray, Ls_f: int) -> np.ndarray:
    """Adjoint of restrict_slice1: P applied to coarse slice 1 onto fine slice 1."""
    wf = prolong2d(P, ec[..., 0, :, :, :])
    e = np.zeros(ec.shape[:-4] + (Ls_f,) + wf.shape[-3:], dtype=np.complex128)
    e[..., 0, :, :, :] = wf
    return e


# ----------------------------------------------------------------------------
# Krylov solvers (Sec. 3, Table kcycle)
# ----------------------------------------------------------------------------
def vdot(a, b):
    return complex(np.vdot(a, b))


def norm(a):
    return math.sqrt(float(np.vdot(a, a).real))


def cg_homogeneous(apply_B, v0, tol, maxit):
    """CG on B v = 0 from v0 (setup relaxation, Sec. 3.1 and Table kcycle).
    Stops at |B v_j| <= tol |B v_0| or after maxit iterations; returns (v, iters)."""
    v = v0.copy()
    r = -apply_B(v)
    p = r.copy()
    rr = vdot(r, r).real
    rr0 = rr
    it = 0
    while it < maxit and rr > tol * tol * rr0:
        Bp = apply_B(p)
        alpha = rr / vdot(p, Bp).real
        v = v + alpha * p
        r = r - alpha * Bp
        rr_new = vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return v, it


def cgnr(apply_A, apply_Adag, b, tol, maxit, x0=None):
    """CG on the normal equations A^dagger A x = A^dagger b (Table kcycle, coarsest level).
    READING: stop when |A^dagger (b - A x)| <= tol |A^dagger b| (the residual of
    the normal system the CG runs on) or after maxit iterations."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    z = apply_Adag(r)
    p = z.copy()
    zz = vdot(z, z).real
    zz0 = vdot(apply_Adag(b), apply_Adag(b)).real if x0 is not None else zz
    it = 0
    while it < maxit and zz > tol * tol * zz0:
        w = apply_A(p)
        alpha = zz / vdot(w, w).real
        x = x + alpha * p
        r = r - alpha * w
        z = apply_Adag(r)
        zz_new = vdot(z, z).real
        p = z + (zz_new / zz) * p
        zz = zz_new
        it += 1
    return x, it


def cgnr_true(apply_A, apply_Adag, b, tol, maxit):
    """CG on the normal equations A^dagger A x = A^dagger b without multigrid (Sec. 3,
    Fig. iterationscompare: "CGNR on D_DW^dagger D_DW"), keeping the residual
    r = b - A x of the original system.  READING: the figure's tolerance 1e-10 is
    on |b - A x| / |b|, the stopping rule of the multigrid solve it is compared
    with.  Returns (x, iterations, applications of A or A^dagger)."""
    x = np.zeros_like(b)
    r = b.copy()
    bb = vdot(b, b).real
    z = apply_Adag(r)
    p = z.copy()
    zz = vdot(z, z).real
    it, applies = 0, 1
    while it < maxit and vdot(r, r).real > tol * tol * bb:
        w = apply_A(p)
        alpha = zz / vdot(w, w).real
        x = x + alpha * p
        r = r - alpha * w
        z = apply_Adag(r)
        zz_new = vdot(z, z).real
        p = z + (zz_new / zz) * p
        zz = zz_new
        it += 1
        applies += 2
    return x, it, applies


def bicgstab_l(apply_A, b, ell, tol, maxit, x0=None):
    """BiCGStab(ell) (Sleijpen & Fokkema, ETNA 1, 1993) on A x = b, as the paper
    applies it to A = D_PV^dagger D_DW (Sec. 3, Fig. iterationscompare, ell = 6;
    valid because that operator has its spectrum in the right half-plane,
    appendix).  Each cycle runs ell BiCG steps, which build the Krylov
    directions u_0..u_ell and residuals r_0..r_ell, then one minimal-residual
    step that minimises |r_0 - sum_j gamma_j r_j| over gamma_1..gamma_ell by
    modified Gram-Schmidt on r_1..r_ell.  Complex inner products are
    (a, b) = a^H b; the shadow residual is the initial residual.  Stops when the
    recursively updated |r| <= tol |b| (checked after every cycle) or after
    maxit cycles.  Returns (x, cycles, applications of A)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r0 = b - apply_A(x) if x0 is not None else b.copy()
    applies = 1 if x0 is not None else 0
    rt = r0.copy()                       # shadow residual
    u = [np.zeros_like(b) for _ in range(ell + 1)]
    r = [np.zeros_like(b) for _ in range(ell + 1)]
    r[0] = r0
    rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
    bb = vdot(b, b).real
    cycles = 0
    while cycles < maxit and vdot(r[0], r[0]).real > tol * tol * bb:
        rho0 = -omega * rho0
        # BiCG part
        for j in range(ell):
            rho1 = vdot(rt, r[j])
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = apply_A(u[j])
            gamma = vdot(rt, u[j + 1])
            alpha = rho0 / gamma
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = apply_A(r[j])
            x = x + alpha * u[0]
            applies += 2
        # MR part: modified Gram-Schmidt on r_1..r_ell
        tau = np.zeros((ell + 1, ell + 1), dtype=np.complex128)
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1, dtype=np.complex128)      # gamma'
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = vdot(r[i], r[j]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = vdot(r[j], r[j]).real
            gp[j] = vdot(r[j], r[0]) / sigma[j]
        g = np.zeros(ell + 1, dtype=np.complex128)       # gamma
        g[ell] = gp[ell]
        omega = g[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        gpp = np.zeros(ell + 1, dtype=np.complex128)     # gamma''
        for j in range(1, ell):
            gpp[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        x = x + g[1] * r[0]
        r[0] = r[0] - gp[ell] * r[ell]
        u[0] = u[0] - g[ell] * u[ell]
        for j in range(1, ell):
            u[0] = u[0] - g[j] * u[j]
            x = x + gpp[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
        cycles += 1
    return x, cycles, applies


def gcr(apply_A, b, tol, maxit, restart, precond=None, x0=None):
    """Flexible GCR with restarts (Table kcycle): directions p_j = M(r_j),
    q_j = A p_j orthonormalised against the previous q's by modified
    Gram-Schmidt, x += alpha p_j, r -= alpha q_j with alpha = <q_j, r>.
    Stops when |r| <= tol |b| or after maxit iterations.  Returns (x, iters)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    bnorm = norm(b)
    it = 0
    if bnorm == 0.0:
        return x, 0
    while it < maxit and norm(r) > tol * bnorm:
        ps, qs = [], []
        for _ in range(restart):
            if it >= maxit or norm(r) <= tol * bnorm:
                break
            p = precond(r) if precond is not None else r.copy()
            q = apply_A(p)
            for pi, qi in zip(ps, qs):
                beta = vdot(qi, q)
                q = q - beta * qi
                p = p - beta * pi
            qn = norm(q)
            q = q / qn
            p = p / qn
            alpha = vdot(q, r)
            x = x + alpha * p
            r = r - alpha * q
            ps.append(p)
            qs.append(q)
            it += 1
        if it < maxit and norm(r) > tol * bnorm:
            r = b - apply_A(x)      # true residual before the next cycle
    return x, it


# ----------------------------------------------------------------------------
# Multigrid hierarchy and K-cycle (Sec. 2.3 summary, Sec. 3.1, Table kcycle)
# ----------------------------------------------------------------------------
@dataclass
class LevelParams:
    nvec: int
    block: tuple                   # (by, bx)
    Ls: int                        # extent of the fifth dimension on the coarse level
    setup_iters: int = 250
    setup_tol: float = 1e-4


@dataclass
class MGParams:
    levels: List[LevelParams]
    m_setup: float = 0.0           # READING: mass of the setup Wilson kernel
    outer_restart: int = 16
    smooth_iters: int = 8          # post-smoothing GCR steps (pre-smoothing 0)
    smooth_restart: int = 0        # restart length of the smoothing GCR (0: one cycle of smooth_iters)
    inter_maxit: int = 16
    inter_tol: float = 0.25
    inter_restart: int = 16
    coarsest_tol: float = 0.05
    coarsest_maxit: int = 1024
    transfer: str = "wall"         # "wall": eq. TruncProjectInterpolate; "bulk": Sec. 4.1's alternative;
                                   # "slice1": the literal unpermuted slice 1 (test toggle)


@dataclass
class Level:
    """One level: its fifth extent, kernel (fine: U; coarse: Stencil),
    chirality of a site's dof and (except on the coarsest) the prolongator
    to the next level."""
    Ls: int
    U: Optional[np.ndarray] = None
    S: Optional[Stencil] = None
    P: Optional[Prolongator] = None
    chir: np.ndarray = field(default_factory=lambda: np.array([1.0, -1.0]))

    def dw(self, psi, m, M5, dagger=False):
        if self.U is not None:
            return dwf(self.U, psi, m, M5, dagger=dagger)
        return stencil_dwf(self.S, psi, m, M5, dagger=dagger)

    def wilson2d(self, psi, M, dagger=False):
        if self.U is not None:
            return wilson(self.U, psi, M, dagger=dagger)
        return stencil_apply(self.S, psi, shift_mass=M, dagger=dagger)

    def kernel_stencil(self):
        return wilson_stencil(self.U) if self.U is not None else self.S


class MG:
    """The domain-wall multigrid of Sec. 2.3 built on an oracle hierarchy."""

    def __init__(self, U, Ls, m, M5, params: MGParams, null_starts):
        """``null_starts[l]``: Gaussian starting vectors of level l's setup,
        shape [nvec, y, x, n] on level l's 2-d lattice."""
        self.m, self.M5, self.params = m, M5, params
        self.levels: List[Level] = [Level(Ls=Ls, U=U)]
        self.setup_iters = []
        for li, lp in enumerate(params.levels):
            lev = self.levels[-1]
            Bop = lambda v, lev=lev: lev.wilson2d(lev.wilson2d(v, params.m_setup, dagger=True),
                                                   params.m_setup)
            vs = []
            its = []
            for k in range(lp.nvec):
                v, it = cg_homogeneous(Bop, null_starts[li][k], lp.setup_tol, lp.setup_iters)
                vs.append(v)
                its.append(it)
            self.setup_iters.append(its)
            V = fine_to_chiral_columns(np.stack(vs), lev.chir)
            V = block_orthonormalize(V, lp.block)
            lev.P = Prolongator(V=V, block=tuple(lp.block))
            S = galerkin(lev.kernel_stencil(), lev.P)
            self.levels.append(Level(Ls=lp.Ls, S=S, chir=S.chir))

    # operators
    def A(self, l, psi):
        lev = self.levels[l]
        return lev.dw(lev.dw(psi, self.m, self.M5), 1.0, self.M5, dagger=True)

    def Adag(self, l, psi):
        lev = self.levels[l]
        return lev.dw(lev.dw(psi, 1.0, self.M5), self.m, self.M5, dagger=True)

    def restrict(self, l, r):
        lev = self.levels[l]
        if self.params.transfer == "bulk":
            return restrict_bulk(lev.P, r)
        if self.params.transfer == "slice1":
            return restrict_slice1(lev.P, r, self.levels[l + 1].Ls)
        return restrict_wall(lev.P, r, lev.chir, self.levels[l + 1].Ls)

    def prolong(self, l, e):
        lev = self.levels[l]
        if self.params.transfer == "bulk":
            return prolong_bulk(lev.P, e)
        if self.params.transfer == "slice1":
            return prolong_slice1(lev.P, e, lev.Ls)
        return prolong_wall(lev.P, e, lev.chir, lev.Ls)

    def local_colinearity(self, v):
        """Sec. 4.1: |(1 - P R) v| for the level-0 transfer (wall or bulk)."""
        return norm(v - self.prolong(0, self.restrict(0, v)))

    def oblique_projector(self, v, coarse_inverse):
        """Sec. 4.1: |(1 - P hat-A^{-1} R A) v| with A = D_PV^dag D_DW on level 0 and
        hat-A its coarse counterpart; `coarse_inverse` applies hat-A^{-1} exactly."""
        return norm(v - self.prolong(0, coarse_inverse(self.restrict(0, self.A(0, v)))))

    def coarse_solve(self, l, rc):
        """Approximate solve of level l's A (l >= 1) for the K-cycle."""
        p = self.params
        if l == len(self.levels) - 1:
            x, it = cgnr(lambda v: self.A(l, v), lambda v: self.Adag(l, v), rc,
                         p.coarsest_tol, p.coarsest_maxit)
            return x
        x, it = gcr(lambda v: self.A(l, v), rc, p.inter_tol, p.inter_maxit, p.inter_restart,
                    precond=lambda r: self.kcycle(l, r))
        return x

    def kcycle(self, l, r):
        """M(r) on level l: coarse-grid correction on the wall, then post-smoothing
        (0 pre-, 8 post-smoothing GCR steps on A, Table kcycle)."""
        e = self.coarse_solve(l + 1, self.restrict(l, r))
        z0 = self.prolong(l, e)
        if self.params.smooth_iters == 0:
            return z0
        rs = r - self.A(l, z0)
        ks = self.params.smooth_restart or self.params.smooth_iters
        zs, _ = gcr(lambda v: self.A(l, v), rs, 0.0, self.params.smooth_iters, ks)
        return z0 + zs

    def solve(self, b, tol, maxit=10000):
        """x with |b - D_DW x| <= tol |b|: flexible GCR on D_PV^dag D_DW x = D_PV^dag b
        with the K-cycle as preconditioner (Sec. 2.3 summary)."""
        lev = self.levels[0]
        rhs = lev.dw(b, 1.0, self.M5, dagger=True)
        x = np.zeros_like(b)
        total = 0
        bnorm = norm(b)
        while True:
            rtrue = b - lev.dw(x, self.m, self.M5)
            if norm(rtrue) <= tol * bnorm or total >= maxit:
                return x, total
            rA = lev.dw(rtrue, 1.0, self.M5, dagger=True)
            # stop the inner solve at the A-residual that the stopping rule needs
            inner = 0.5 * tol * bnorm / norm(rhs)
            e, it = gcr(lambda v: self.A(0, v), rA, inner * norm(rhs) / norm(rA),
                        maxit - total, self.params.outer_restart,
                        precond=lambda r: self.kcycle(0, r))
            x = x + e
            total += it


def assemble(op: Callable, shape) -> np.ndarray:
    """Dense matrix of a linear operator acting on arrays of ``shape``
    (columns are the images of the unit vectors)."""
    N = int(np.prod(shape))
    eye = np.eye(N, dtype=np.complex128).reshape((N,) + tuple(shape))
    cols = op(eye).reshape(N, -1)
    return cols.T.copy()
