"""Python binding of libdwfmg.so (argument marshalling only).

Every function takes torch tensors that live on the GPU, checks their dtype,
shape and contiguity, and passes raw device pointers and the current HIP stream
to the C ABI declared in include/dwfmg.h.  All arithmetic happens in the HIP
library; if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwfmg.so")

DWF_OK = 0
DWF_NOT_CONVERGED = 1
DWF_EINVAL = -1
DWF_EHIP = -2
DWF_EBREAKDOWN = -3
DWF_ENAN = -4
DWF_ENOSETUP = -5
DWF_EUNSUPPORTED = -6
DWF_ESCRATCH = -7

DWF_DAGGER = 1
DWF_PREC_F32 = 2
DWF_PV_SOURCE = 4

DWF_PV, DWF_PV_DAG, DWF_PVDAG_DW, DWF_PVDAG_DW_DAG, DWF_PVINV_DW = 0, 1, 2, 3, 4
P_F64, P_F32, P_BF16, P_F16 = 0, 1, 2, 3
MAX_LEVELS = 3

MG_OP_DW, MG_OP_DW_DAG, MG_OP_PV, MG_OP_PV_DAG, MG_OP_A = 0, 1, 2, 3, 4
MG_OP_WILSON, MG_OP_WILSON_DAG, MG_OP_RESTRICT, MG_OP_PROLONG, MG_OP_KCYCLE = 5, 6, 7, 8, 9
COARSEST_CGNR, COARSEST_GCR = 0, 1
KRYLOV_CGNR, KRYLOV_BICGSTAB = 0, 1
TRANSFER_WALL, TRANSFER_BULK, TRANSFER_SLICE1 = 0, 1, 2
PV_POLY_MAX = 3
FINE_AUTO, FINE_ROW, FINE_TILE_64x8, FINE_TILE_32x16, FINE_TILE_128x4 = -1, 0, 1, 2, 3
FINE_A_AUTO, FINE_A_TWO, FINE_A_16x16, FINE_A_32x8, FINE_A_16x8 = -1, 0, 1, 2, 3


class DwfError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libdwfmg.so (built in-tree by `python -m paper_2004_07732_amd.build`)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              f"(python -m paper_2004_07732_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.dwf_apply.argtypes = [vp, vp, vp, i, i, i, i, d, d, i, vp]
        L.dwf_pv_apply.argtypes = [vp, vp, vp, i, i, i, i, d, d, i, i, vp]
        L.dwf_pv_apply_noalloc.argtypes = [vp, vp, vp, i, i, i, i, d, d, i, i, vp]
        L.dwf_pv_apply_noalloc_max_bytes.argtypes = []
        L.dwf_pv_apply_noalloc_max_bytes.restype = sz
        L.dwf_fine_config.argtypes = [i, i]
        L.dwf_fine_a_config.argtypes = [i, i]
        L.dwf_fine_a_chosen.argtypes = [i, i, i, i, i, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.dwf_pv_poly_apply.argtypes = [vp, vp, vp, i, i, i, i, d, d, ctypes.POINTER(d), i, i, vp]
        L.dwf_pv_poly_chebyshev.argtypes = [i, d, d, ctypes.POINTER(d)]
        L.dwf_wilson_apply.argtypes = [vp, vp, vp, i, i, i, d, i, vp]
        L.dwf_gamma5R.argtypes = [vp, vp, i, i, i, i, i, vp]
        L.dwf_gauge_transform.argtypes = [vp, vp, vp, vp, vp, i, i, i, i, vp]
        L.dwf_pack.argtypes = [vp, vp, sz, vp]
        L.dwf_unpack.argtypes = [vp, vp, sz, vp]
        L.dwf_force.argtypes = [vp, vp, vp, vp, i, i, i, i, vp]
        L.dwf_links_from_theta.argtypes = [vp, vp, i, i, vp]
        L.dwf_mg_default_params.argtypes = [ctypes.POINTER(CParams), i]
        L.dwf_mg_default_params.restype = None
        L.mg_workspace_bytes.argtypes = [i, i, i, i, ctypes.POINTER(CParams)]
        L.mg_workspace_bytes.restype = sz
        L.mg_setup.argtypes = [ctypes.POINTER(vp), vp, i, i, i, d, d, ctypes.POINTER(CParams),
                               ctypes.POINTER(vp), i, vp, sz, vp]
        L.mg_solve.argtypes = [vp, vp, vp, i, d, i, ctypes.POINTER(CStats), vp]
        L.mg_level_op.argtypes = [vp, i, i, vp, vp, i, d, vp]
        L.mg_export.argtypes = [vp, i, vp, vp, vp]
        L.mg_time_op.argtypes = [vp, i, i, vp, i, i, ctypes.POINTER(d), vp]
        L.dwf_norm2.argtypes = [vp, sz, i, vp, vp]
        L.dwf_copy_bandwidth.argtypes = [vp, vp, sz, i, ctypes.POINTER(d), vp]
        L.mg_solve_batch.argtypes = [i, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(i), d, i, ctypes.POINTER(CStats), vp]
        L.mg_update_links.argtypes = [vp, vp, vp]
        L.mg_level_info.argtypes = [vp, i] + [ctypes.POINTER(i)] * 5
        L.mg_coarse_config.argtypes = [vp, i, i, i, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.mg_deflation_info.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(d), vp]
        L.dwf_krylov_solve.argtypes = [vp, vp, vp, i, i, i, d, d, i, i, d, i, ctypes.POINTER(CStats), vp]
        L.mg_destroy.argtypes = [vp]
        L.dwf_release_scratch.argtypes = []
        L.dwf_strerror.argtypes = [i]
        L.dwf_strerror.restype = ctypes.c_char_p
        for name in ("dwf_apply", "dwf_pv_apply", "dwf_pv_apply_noalloc", "dwf_fine_config", "dwf_fine_a_config",
                     "dwf_fine_a_chosen", "dwf_pv_poly_apply", "dwf_pv_poly_chebyshev",
                     "dwf_wilson_apply", "dwf_gamma5R", "dwf_gauge_transform",
                     "dwf_pack", "dwf_unpack", "dwf_force", "dwf_links_from_theta", "mg_setup", "mg_solve", "mg_level_op", "mg_export",
                     "mg_time_op", "dwf_norm2", "dwf_copy_bandwidth", "mg_update_links", "mg_solve_batch",
                     "mg_level_info", "mg_coarse_config", "mg_deflation_info", "mg_destroy", "dwf_release_scratch",
                     "dwf_krylov_solve"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().dwf_strerror(code).decode()
    except ImportError:
        return str(code)


def _check(code: int, what: str, soft_ok: bool = False) -> int:
    if code == DWF_OK or (soft_ok and code > 0):
        return code
    raise DwfError(code, what)


class CParams(ctypes.Structure):
    _fields_ = [
        ("nlevels", ctypes.c_int),
        ("nvec", ctypes.c_int * MAX_LEVELS),
        ("block", (ctypes.c_int * 2) * MAX_LEVELS),
        ("Ls_coarse", ctypes.c_int * MAX_LEVELS),
        ("link_prec", ctypes.c_int * MAX_LEVELS),
        ("vec_prec", ctypes.c_int * MAX_LEVELS),
        ("fine_prec", ctypes.c_int),
        ("m_setup", ctypes.c_double),
        ("setup_iters", ctypes.c_int),
        ("setup_tol", ctypes.c_double),
        ("outer_restart", ctypes.c_int),
        ("smooth_iters", ctypes.c_int),
        ("smooth_restart", ctypes.c_int),
        ("inter_maxit", ctypes.c_int),
        ("inter_tol", ctypes.c_double),
        ("inter_restart", ctypes.c_int),
        ("coarsest_maxit", ctypes.c_int),
        ("coarsest_tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("max_iters", ctypes.c_int),
        ("max_outer", ctypes.c_int),
        ("coarsest_nev", ctypes.c_int),
        ("eig_degree", ctypes.c_int),
        ("eig_maxit", ctypes.c_int),
        ("eig_tol", ctypes.c_double),
        ("coarsest_solver", ctypes.c_int),
        ("coarsest_restart", ctypes.c_int),
        ("transfer", ctypes.c_int),
        ("pv_poly_order", ctypes.c_int),
        ("pv_poly", ctypes.c_double * (PV_POLY_MAX + 1)),
        ("stagnation_ratio", ctypes.c_double),
    ]


class CStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("outer_steps", ctypes.c_int),
        ("fine_iters", ctypes.c_int),
        ("fine_applies", ctypes.c_longlong),
        ("level_iters", ctypes.c_longlong * MAX_LEVELS),
        ("level_calls", ctypes.c_longlong * MAX_LEVELS),
        ("true_rel_residual", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("escalations", ctypes.c_int),
    ]


@dataclass
class MGParams:
    """K-cycle parameters (defaults: the paper's parameter table, Table kcycle)."""
    nvec: List[int] = field(default_factory=lambda: [8, 12])
    block: List[tuple] = field(default_factory=lambda: [(4, 4), (2, 2)])   # (bx, by)
    Ls_coarse: List[int] = field(default_factory=lambda: [4, 4])
    link_prec: List[int] = field(default_factory=lambda: [P_F64, P_F64])
    vec_prec: List[int] = field(default_factory=lambda: [P_F64, P_F64])
    fine_prec: int = P_F64
    m_setup: float = 0.0
    setup_iters: int = 250
    setup_tol: float = 1e-4
    outer_restart: int = 16
    smooth_iters: int = 8
    smooth_restart: int = 0        # restart length of the post-smoothing GCR (0: none)
    inter_maxit: int = 16
    inter_tol: float = 0.25
    inter_restart: int = 16
    coarsest_maxit: int = 1024
    coarsest_tol: float = 0.05
    inner_tol: float = 0.0
    max_iters: int = 10000
    max_outer: int = 20
    coarsest_nev: int = 0          # coarsest-level deflation (0: off, as in Table kcycle)
    eig_degree: int = 0            # Chebyshev degree of the Lanczos acceleration (0: automatic)
    eig_maxit: int = 40            # thick-restart cycles
    eig_tol: float = 1e-3
    coarsest_solver: int = COARSEST_CGNR   # CGNR on A^dag A (Table 2), or COARSEST_GCR: GCR on A
    coarsest_restart: int = 16
    transfer: int = 0              # TRANSFER_WALL (the paper's method), TRANSFER_BULK (Sec. 4.1) or
                                   # TRANSFER_SLICE1 (the literal-slice reading, a test toggle)
    pv_poly: Optional[List[float]] = None   # c_0..c_K of the PV polynomial on the fine level (None: A itself)
    stagnation_ratio: float = 0.9  # outer step stagnates above this residual ratio: promote 16-bit coarse links

    @property
    def nlevels(self) -> int:
        return len(self.nvec)

    def to_c(self) -> CParams:
        c = CParams()
        lib().dwf_mg_default_params(ctypes.byref(c), self.nlevels)
        c.nlevels = self.nlevels
        for l in range(self.nlevels):
            c.nvec[l] = self.nvec[l]
            c.block[l][0], c.block[l][1] = self.block[l]
            c.Ls_coarse[l] = self.Ls_coarse[l]
            c.link_prec[l] = self.link_prec[l]
            c.vec_prec[l] = self.vec_prec[l]
        for name in ("fine_prec", "m_setup", "setup_iters", "setup_tol", "outer_restart", "smooth_iters", "smooth_restart",
                     "inter_maxit", "inter_tol", "inter_restart", "coarsest_maxit", "coarsest_tol", "inner_tol",
                     "max_iters", "max_outer", "coarsest_nev", "eig_degree", "eig_maxit", "eig_tol",
                     "coarsest_solver", "coarsest_restart", "transfer", "stagnation_ratio"):
            setattr(c, name, getattr(self, name))
        if self.pv_poly is not None:
            coef = [float(v) for v in self.pv_poly]
            if not 1 <= len(coef) <= PV_POLY_MAX + 1:
                raise ValueError(f"pv_poly takes 1..{PV_POLY_MAX + 1} coefficients")
            c.pv_poly_order = len(coef) - 1
            for k, v in enumerate(coef):
                c.pv_poly[k] = v
        return c


@dataclass
class SolveStats:
    status: int
    outer_steps: int
    fine_iters: int
    fine_applies: int
    level_iters: List[int]
    level_calls: List[int]
    true_rel_residual: float
    solve_ms: float
    escalations: int = 0


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, name: str, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _prec(t: torch.Tensor):
    if t.dtype == torch.complex128:
        return 0
    if t.dtype == torch.complex64:
        return DWF_PREC_F32
    raise ValueError(f"unsupported dtype {t.dtype}")


def _fine_dims(U: torch.Tensor, psi: torch.Tensor):
    if U.dim() != 3 or U.shape[0] != 2:
        raise ValueError("U must be [2, Ly, Lx]")
    Ly, Lx = U.shape[1], U.shape[2]
    if psi.dim() == 4:
        psi = psi.unsqueeze(0)
    if psi.dim() != 5 or tuple(psi.shape[2:]) != (Ly, Lx, 2):
        raise ValueError("fields must be [nrhs, Ls, Ly, Lx, 2]")
    return Lx, Ly, psi.shape[1], psi.shape[0]


# ----------------------------------------------------------------------------- operators
def dwf_apply(U, psi, m_f, M5, dagger=False, out=None, stream=None):
    """out = D_DW(m_f) psi (or its adjoint); U [2,Ly,Lx], psi [nrhs,Ls,Ly,Lx,2] (or without nrhs)."""
    _need(U, "U", psi.dtype)
    _need(psi, "psi")
    Lx, Ly, Ls, nrhs = _fine_dims(U, psi)
    out = torch.empty_like(psi) if out is None else out
    _need(out, "out", psi.dtype, psi.shape)
    flags = _prec(psi) | (DWF_DAGGER if dagger else 0)
    _check(lib().dwf_apply(_ptr(U), _ptr(psi), _ptr(out), Lx, Ly, Ls, nrhs, float(m_f), float(M5), flags,
                           _stream(stream)), "dwf_apply")
    return out


def dwf_pv_poly_apply(U, psi, m_f, M5, c, dagger=False, out=None, stream=None):
    """out = D_PV^dag p(D_PV D_PV^dag) D_DW psi, p(X) = sum_k c[k] X^k (or the adjoint)."""
    _need(U, "U", psi.dtype)
    _need(psi, "psi")
    Lx, Ly, Ls, nrhs = _fine_dims(U, psi)
    out = torch.empty_like(psi) if out is None else out
    _need(out, "out", psi.dtype, psi.shape)
    coef = (ctypes.c_double * len(c))(*[float(v) for v in c])
    flags = _prec(psi) | (DWF_DAGGER if dagger else 0)
    _check(lib().dwf_pv_poly_apply(_ptr(U), _ptr(psi), _ptr(out), Lx, Ly, Ls, nrhs, float(m_f), float(M5), coef,
                                   len(c) - 1, flags, _stream(stream)), "dwf_pv_poly_apply")
    return out


def pv_poly_chebyshev(order, lam_min=1.0, lam_max=25.0):
    """Coefficients of the degree-`order` polynomial p minimising max |1 - x p(x)| on [lam_min, lam_max]."""
    coef = (ctypes.c_double * (order + 1))()
    _check(lib().dwf_pv_poly_chebyshev(int(order), float(lam_min), float(lam_max), coef), "dwf_pv_poly_chebyshev")
    return list(coef)


def dwf_fine_config(shape, chunk=1):
    """Pin the fine stencil's launch configuration for the process (FINE_ROW or a
    FINE_TILE_* shape, `chunk` slices per thread); FINE_AUTO restores the tuned choice."""
    _check(lib().dwf_fine_config(int(shape), int(chunk)), "dwf_fine_config")


def dwf_fine_a_config(shape, chunk=1):
    """Pin the launch configuration of the solver's fine A = D_PV^dag D_DW: FINE_A_TWO
    (two stencil launches) or a fused FINE_A_* tile shape with `chunk` output slices per
    workgroup; FINE_A_AUTO restores the timed choice."""
    _check(lib().dwf_fine_a_config(int(shape), int(chunk)), "dwf_fine_a_config")


def dwf_fine_a_chosen(Lx, Ly, Ls, nrhs, f32=True):
    """(shape, chunk) the timed choice picked for the fine A at this shape, or None."""
    sh, ch = ctypes.c_int(), ctypes.c_int()
    code = lib().dwf_fine_a_chosen(DWF_PREC_F32 if f32 else 0, int(Lx), int(Ly), int(Ls), int(nrhs),
                                   ctypes.byref(sh), ctypes.byref(ch))
    return (sh.value, ch.value) if code == DWF_OK else None


def dwf_pv_apply(U, psi, m_f, M5, mode=DWF_PVDAG_DW, out=None, stream=None):
    """Pauli-Villars forms: DWF_PV, DWF_PV_DAG, DWF_PVDAG_DW (A), DWF_PVDAG_DW_DAG (A^dagger),
    DWF_PVINV_DW (D_PV^-1 D_DW by an inner CGNR solve to 1e-12, complex128 only)."""
    _need(U, "U", psi.dtype)
    _need(psi, "psi")
    Lx, Ly, Ls, nrhs = _fine_dims(U, psi)
    out = torch.empty_like(psi) if out is None else out
    _need(out, "out", psi.dtype, psi.shape)
    _check(lib().dwf_pv_apply(_ptr(U), _ptr(psi), _ptr(out), Lx, Ly, Ls, nrhs, float(m_f), float(M5), int(mode),
                              _prec(psi), _stream(stream)), "dwf_pv_apply")
    return out


def dwf_pv_apply_noalloc(U, psi, m_f, M5, mode=DWF_PVDAG_DW, out=None, stream=None):
    """dwf_pv_apply without device allocation (modes DWF_PV .. DWF_PVDAG_DW_DAG): the
    intermediate field lives in the library's static per-GPU array (see
    noalloc_max_bytes()); calls that overlap on one GPU race."""
    _need(U, "U", psi.dtype)
    _need(psi, "psi")
    Lx, Ly, Ls, nrhs = _fine_dims(U, psi)
    out = torch.empty_like(psi) if out is None else out
    _need(out, "out", psi.dtype, psi.shape)
    _check(lib().dwf_pv_apply_noalloc(_ptr(U), _ptr(psi), _ptr(out), Lx, Ly, Ls, nrhs, float(m_f), float(M5),
                                      int(mode), _prec(psi), _stream(stream)), "dwf_pv_apply_noalloc")
    return out


def noalloc_max_bytes() -> int:
    """Size of the static scratch array of dwf_pv_apply_noalloc (bytes per GPU)."""
    return int(lib().dwf_pv_apply_noalloc_max_bytes())


def dwf_wilson_apply(U, psi, M, dagger=False, out=None, stream=None):
    """out = D_W(M) psi on 2-d fields psi [nrhs, Ly, Lx, 2]."""
    _need(U, "U", psi.dtype)
    _need(psi, "psi")
    Ly, Lx = U.shape[1], U.shape[2]
    p = psi if psi.dim() == 4 else psi.unsqueeze(0)
    if tuple(p.shape[1:]) != (Ly, Lx, 2):
        raise ValueError("psi must be [nrhs, Ly, Lx, 2]")
    out = torch.empty_like(psi) if out is None else out
    _need(out, "out", psi.dtype, psi.shape)
    flags = _prec(psi) | (DWF_DAGGER if dagger else 0)
    _check(lib().dwf_wilson_apply(_ptr(U), _ptr(psi), _ptr(out), Lx, Ly, p.shape[0], float(M), flags,
                                  _stream(stream)), "dwf_wilson_apply")
    return out


def dwf_gamma5R(psi, out=None, stream=None):
    """Gamma_5 = gamma_5 R on psi [nrhs, Ls, Ly, Lx, 2]."""
    _need(psi, "psi")
    p = psi if psi.dim() == 5 else psi.unsqueeze(0)
    out = torch.empty_like(psi) if out is None else out
    _need(out, "out", psi.dtype, psi.shape)
    _check(lib().dwf_gamma5R(_ptr(psi), _ptr(out), p.shape[3], p.shape[2], p.shape[1], p.shape[0], _prec(psi),
                             _stream(stream)), "dwf_gamma5R")
    return out


def dwf_gauge_transform(U, g, psi=None, stream=None):
    """Returns (U^g, psi^g) (psi^g is None when psi is None); complex128."""
    _need(U, "U", torch.complex128)
    _need(g, "g", torch.complex128, U.shape[1:])
    Ly, Lx = U.shape[1], U.shape[2]
    Ug = torch.empty_like(U)
    psig = None
    Ls = nrhs = 1
    if psi is not None:
        _need(psi, "psi", torch.complex128)
        p = psi if psi.dim() == 5 else psi.unsqueeze(0)
        Ls, nrhs = p.shape[1], p.shape[0]
        psig = torch.empty_like(psi)
    _check(lib().dwf_gauge_transform(_ptr(U), _ptr(g), _ptr(psi), _ptr(Ug), _ptr(psig), Lx, Ly, Ls, nrhs,
                                     _stream(stream)), "dwf_gauge_transform")
    return Ug, psig


def dwf_pack(x, stream=None):
    """complex128 -> complex64."""
    _need(x, "x", torch.complex128)
    out = torch.empty(x.shape, dtype=torch.complex64, device=x.device)
    _check(lib().dwf_pack(_ptr(x), _ptr(out), x.numel(), _stream(stream)), "dwf_pack")
    return out


def dwf_unpack(x, stream=None):
    """complex64 -> complex128."""
    _need(x, "x", torch.complex64)
    out = torch.empty(x.shape, dtype=torch.complex128, device=x.device)
    _check(lib().dwf_unpack(_ptr(x), _ptr(out), x.numel(), _stream(stream)), "dwf_unpack")
    return out


def dwf_force(U, X, Y, stream=None):
    """F[mu, y, x] = dS/dtheta_mu(x) for S = phi^dag (D^dag D)^-1 phi, given Y = D^-dag phi, X = D^-1 Y."""
    _need(U, "U", torch.complex128)
    _need(X, "X", torch.complex128)
    _need(Y, "Y", torch.complex128, X.shape)
    Lx, Ly, Ls, nrhs = _fine_dims(U, X)
    F = torch.empty(U.shape, dtype=torch.float64, device=U.device)
    _check(lib().dwf_force(_ptr(U), _ptr(X), _ptr(Y), _ptr(F), Lx, Ly, Ls, nrhs, _stream(stream)), "dwf_force")
    return F


def dwf_links_from_theta(theta, stream=None):
    """U = exp(i theta) for theta [2, Ly, Lx] float64; returns a complex128 tensor."""
    _need(theta, "theta", torch.float64)
    if theta.dim() != 3 or theta.shape[0] != 2:
        raise ValueError("theta must be [2, Ly, Lx]")
    U = torch.empty(theta.shape, dtype=torch.complex128, device=theta.device)
    _check(lib().dwf_links_from_theta(_ptr(theta), _ptr(U), theta.shape[2], theta.shape[1], _stream(stream)),
           "dwf_links_from_theta")
    return U


def dwf_norm2(x, stream=None):
    """Per-column |x_c|^2 (first axis = columns), FP64, deterministic; returns a CUDA float64 tensor."""
    _need(x, "x", torch.complex128)
    ncol = x.shape[0] if x.dim() > 1 else 1
    out = torch.empty(ncol, dtype=torch.float64, device=x.device)
    _check(lib().dwf_norm2(_ptr(x), x.numel() // ncol, ncol, _ptr(out), _stream(stream)), "dwf_norm2")
    return out


def copy_bandwidth(nbytes: int = 2 ** 31, iters: int = 10, device="cuda", stream=None) -> float:
    """GB/s (read + write) of the library's streaming copy over `nbytes`."""
    src = torch.empty(nbytes, dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    src.fill_(1)
    out = ctypes.c_double()
    _check(lib().dwf_copy_bandwidth(_ptr(src), _ptr(dst), nbytes, int(iters), ctypes.byref(out), _stream(stream)),
           "dwf_copy_bandwidth")
    return out.value


def release_scratch():
    _check(lib().dwf_release_scratch(), "dwf_release_scratch")


# ----------------------------------------------------------------------------- multigrid
def _stats(st: "CStats") -> "SolveStats":
    return SolveStats(st.status, st.outer_steps, st.fine_iters, st.fine_applies, list(st.level_iters),
                      list(st.level_calls), st.true_rel_residual, st.solve_ms, st.escalations)


def dwf_krylov_solve(U, b, m_f, M5, method=KRYLOV_BICGSTAB, ell=6, tol=1e-10, maxit=1_000_000, x=None,
                     stream=None, check=True):
    """Solve D_DW x = b without multigrid (CGNR on D_DW, or BiCGStab(ell) on
    D_PV^dagger D_DW); U [2, Ly, Lx] and b [Ls, Ly, Lx, 2] complex128.
    Returns (x, SolveStats) with fine_iters = iterations / cycles and
    fine_applies = applications of D_DW, D_DW^dagger, D_PV^dagger."""
    _need(U, "U", torch.complex128)
    _need(b, "b", torch.complex128)
    if b.dim() != 4 or b.shape[-1] != 2 or tuple(U.shape) != (2, b.shape[1], b.shape[2]):
        raise ValueError("b must be [Ls, Ly, Lx, 2] matching U [2, Ly, Lx]")
    x = torch.empty_like(b) if x is None else x
    _need(x, "x", torch.complex128, b.shape)
    st = CStats()
    Ls, Ly, Lx = b.shape[0], b.shape[1], b.shape[2]
    code = lib().dwf_krylov_solve(_ptr(U), _ptr(b), _ptr(x), Lx, Ly, Ls, float(m_f), float(M5), int(method), int(ell),
                                  float(tol), int(maxit), ctypes.byref(st), _stream(stream))
    if check:
        _check(code, "dwf_krylov_solve", soft_ok=False)
    return x, _stats(st)


def workspace_bytes(Lx: int, Ly: int, Ls: int, params: "MGParams", max_nrhs: int = 1) -> int:
    """Device bytes a hierarchy needs (mg_workspace_bytes); 0 for invalid arguments."""
    cp = params.to_c()
    return int(lib().mg_workspace_bytes(int(Lx), int(Ly), int(Ls), int(max_nrhs), ctypes.byref(cp)))


def solve_batch(mgs: Sequence["MG"], bs: Sequence[torch.Tensor], tol: float = 1e-10, stream=None,
                check: bool = True, pv_source: bool = False):
    """Solve several lattices at once (mg_solve_batch): returns ([x_i], [stats_i])."""
    n = len(mgs)
    if n != len(bs) or n == 0:
        raise ValueError("one right-hand-side tensor per hierarchy is required")
    xs, nr = [], []
    for mg, b in zip(mgs, bs):
        _need(b, "b", torch.complex128)
        bb = b if b.dim() == 5 else b.unsqueeze(0)
        if tuple(bb.shape[1:]) != (mg.Ls, mg.Ly, mg.Lx, 2):
            raise ValueError("b has the wrong shape for its hierarchy")
        xs.append(torch.empty_like(b))
        nr.append(bb.shape[0])
    VP = ctypes.c_void_p * n
    st = (CStats * n)()
    code = lib().mg_solve_batch(n, VP(*[m._h.value for m in mgs]), VP(*[b.data_ptr() for b in bs]),
                                VP(*[x.data_ptr() for x in xs]), (ctypes.c_int * n)(*nr), float(tol),
                                DWF_PV_SOURCE if pv_source else 0, st, _stream(stream))
    if check:
        _check(code, "mg_solve_batch")
    return xs, [_stats(s) for s in st]


class MG:
    """Domain-wall multigrid hierarchy on one GPU (mg_setup / mg_solve).

    All device memory of the hierarchy lives in one torch tensor (`workspace`,
    mg_workspace_bytes of it) unless the caller passes one; solves take
    right-hand sides in groups of at most `max_nrhs`."""

    def __init__(self, U: torch.Tensor, Ls: int, m_f: float, M5: float, params: MGParams,
                 null_starts: Sequence[torch.Tensor], stream=None, max_nrhs: int = 1,
                 workspace: Optional[torch.Tensor] = None):
        _need(U, "U", torch.complex128)
        if len(null_starts) < params.nlevels:
            raise ValueError("one null-vector start tensor per coarse level is required")
        for k, t in enumerate(null_starts):
            _need(t, f"null_starts[{k}]", torch.complex128)
        self.Lx, self.Ly, self.Ls = U.shape[2], U.shape[1], Ls
        self.m_f, self.M5, self.params = m_f, M5, params
        self._starts = list(null_starts)
        arr = (ctypes.c_void_p * MAX_LEVELS)(*([t.data_ptr() for t in null_starts] +
                                              [None] * (MAX_LEVELS - len(null_starts))))
        self._h = ctypes.c_void_p()
        self._cp = params.to_c()
        self.max_nrhs = int(max_nrhs)
        need = lib().mg_workspace_bytes(self.Lx, self.Ly, Ls, self.max_nrhs, ctypes.byref(self._cp))
        if need == 0:
            raise DwfError(DWF_EINVAL, "mg_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=U.device)
        _need(workspace, "workspace")
        self.workspace = workspace
        _check(lib().mg_setup(ctypes.byref(self._h), _ptr(U), self.Lx, self.Ly, Ls, float(m_f), float(M5),
                              ctypes.byref(self._cp), arr, self.max_nrhs, _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream)), "mg_setup")

    def solve(self, b: torch.Tensor, tol: float = 1e-10, x: Optional[torch.Tensor] = None, stream=None,
              check: bool = True, pv_source: bool = False):
        """x with |b - D_DW x| <= tol |b| for every rhs (pv_source: D_DW x = D_PV b);
        b [nrhs, Ls, Ly, Lx, 2] complex128."""
        _need(b, "b", torch.complex128)
        bb = b if b.dim() == 5 else b.unsqueeze(0)
        if tuple(bb.shape[1:]) != (self.Ls, self.Ly, self.Lx, 2):
            raise ValueError("b has the wrong shape")
        x = torch.empty_like(b) if x is None else x
        _need(x, "x", torch.complex128, b.shape)
        st = CStats()
        code = lib().mg_solve(self._h, _ptr(b), _ptr(x), bb.shape[0], float(tol), DWF_PV_SOURCE if pv_source else 0,
                              ctypes.byref(st), _stream(stream))
        stats = _stats(st)
        if check:
            _check(code, "mg_solve")
        return x, stats

    def update_links(self, U: torch.Tensor, stream=None):
        """Swap in a new fine gauge field; the coarse levels stay as preconditioner."""
        _need(U, "U", torch.complex128, (2, self.Ly, self.Lx))
        _check(lib().mg_update_links(self._h, _ptr(U), _stream(stream)), "mg_update_links")

    def info(self, level: int):
        vals = [ctypes.c_int() for _ in range(5)]
        _check(lib().mg_level_info(self._h, level, *[ctypes.byref(v) for v in vals]), "mg_level_info")
        Lx, Ly, Ls, n, nvec = (v.value for v in vals)
        return dict(Lx=Lx, Ly=Ly, Ls=Ls, n=n, nvec=nvec)

    def coarse_config(self, level: int = 1, ncol: int = 1, dagger: bool = False):
        """(tile width, tiles per workgroup) of the matrix-core coarse stencil on `level`."""
        tw, tpb = ctypes.c_int(), ctypes.c_int()
        _check(lib().mg_coarse_config(self._h, int(level), int(ncol), 1 if dagger else 0, ctypes.byref(tw),
                                      ctypes.byref(tpb)), "mg_coarse_config")
        return tw.value, tpb.value

    def deflation_info(self):
        """Coarsest-level deflation space: dict(nev, iters, worst_residual, lambdas) with
        the Ritz values of hat-A^dag hat-A in ascending order (empty when deflation is off)."""
        nev, iters, worst = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().mg_deflation_info(self._h, ctypes.byref(nev), ctypes.byref(iters), ctypes.byref(worst), None),
               "mg_deflation_info")
        lam = (ctypes.c_double * max(nev.value, 1))()
        _check(lib().mg_deflation_info(self._h, None, None, None, ctypes.cast(lam, ctypes.c_void_p)),
               "mg_deflation_info")
        return dict(nev=nev.value, iters=iters.value, worst_residual=worst.value, lambdas=list(lam)[:nev.value])

    def level_op(self, level: int, op: int, inp: torch.Tensor, ncol: int, mass: float = 0.0, out_shape=None,
                 stream=None) -> torch.Tensor:
        _need(inp, "in", torch.complex128)
        out = torch.empty(out_shape if out_shape is not None else inp.shape, dtype=torch.complex128,
                          device=inp.device)
        _check(lib().mg_level_op(self._h, level, op, _ptr(inp), _ptr(out), ncol, float(mass), _stream(stream)),
               "mg_level_op")
        return out

    def time_op(self, level: int, op: int, inp: torch.Tensor, ncol: int, iters: int = 50, stream=None) -> float:
        """Mean milliseconds of one application of a level operator (HIP events on `stream`)."""
        _need(inp, "in", torch.complex128)
        ms = ctypes.c_double()
        _check(lib().mg_time_op(self._h, level, op, _ptr(inp), ncol, iters, ctypes.byref(ms), _stream(stream)),
               "mg_time_op")
        return ms.value

    def export(self, level: int, stream=None):
        """(V[y,x,c,j,k], diag[Y,X,n,n], hop[4,Y,X,n,n]) of level -> level+1, complex128."""
        f = self.info(level)
        c = self.info(level + 1)
        nc = f["n"] // 2
        V = torch.empty((f["Ly"], f["Lx"], 2, nc, f["nvec"]), dtype=torch.complex128, device="cuda")
        n = c["n"]
        K = torch.empty((5, c["Ly"], c["Lx"], n, n), dtype=torch.complex128, device="cuda")
        _check(lib().mg_export(self._h, level, _ptr(V), _ptr(K), _stream(stream)), "mg_export")
        return V, K[0], K[1:]

    def close(self):
        if self._h:
            lib().mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
