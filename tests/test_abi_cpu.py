"""Host-side checks that need no GPU: the C-ABI library loads and exports every
symbol that include/dwfmg.h declares, and the Python parameter mirror matches
the paper's parameter table."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwfmg.h")
LIB = os.path.join(ROOT, "paper_2004_07732_amd", "libdwfmg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^(?:int|void|size_t|const char\s*\*)\s+\**\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libdwf():
    if not os.path.exists(LIB):
        from paper_2004_07732_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dwf_apply", "dwf_pv_apply", "mg_setup", "mg_solve", "mg_destroy", "dwf_force",
              "dwf_gauge_transform", "dwf_pack", "dwf_unpack", "dwf_gamma5R", "dwf_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol(libdwf):
    missing = [n for n in declared_functions() if not hasattr(libdwf, n)]
    assert not missing, missing


def test_strerror_and_defaults_without_gpu(libdwf):
    libdwf.dwf_strerror.restype = ctypes.c_char_p
    assert libdwf.dwf_strerror(0) == b"ok"
    assert b"invalid" in libdwf.dwf_strerror(-1)
    from paper_2004_07732_amd import dwfmg
    c = dwfmg.MGParams().to_c()
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "kcycle_params.json")))
    assert c.setup_iters == golden["setup"]["max_iterations"]
    assert c.setup_tol == golden["setup"]["tolerance_per_null_vector"]
    assert c.nvec[0] == golden["setup"]["nvec_level1"] and c.nvec[1] == golden["setup"]["nvec_coarser"]
    assert tuple(c.block[0]) == tuple(golden["setup"]["block_level1"])
    assert tuple(c.block[1]) == tuple(golden["setup"]["block_coarser"])
    assert c.outer_restart == golden["level1"]["gcr_restart"]
    assert c.smooth_iters == golden["level1"]["post_smooth"]
    assert c.inter_maxit == golden["level2"]["max_iterations"]
    assert c.inter_tol == golden["level2"]["tolerance"]
    assert c.Ls_coarse[0] == golden["level2"]["Ls_coarse"]
    assert c.coarsest_tol == golden["level3"]["tolerance"]
    assert c.coarsest_maxit == golden["level3"]["max_iterations"]


def test_argument_errors_are_reported_before_any_device_work(libdwf):
    """Null pointers and impossible sizes are rejected on the host (no GPU touched)."""
    vp = ctypes.c_void_p
    libdwf.dwf_apply.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, vp]
    assert libdwf.dwf_apply(None, None, None, 4, 4, 4, 1, 0.1, -1.0, 0, None) == -1
    assert libdwf.dwf_apply(1, 2, 3, 0, 4, 4, 1, 0.1, -1.0, 0, None) == -1
    assert libdwf.dwf_apply(1, 2, 3, 4, 4, 4, 1, float("nan"), -1.0, 0, None) == -1
    libdwf.mg_solve.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_double, vp, vp]
    assert libdwf.mg_solve(None, 1, 2, 1, 1e-10, None, None) == -5
    # dwf_pv_apply: unknown mode; the exact D_PV^-1 D_DW mode has no FP32 form (DWF_EUNSUPPORTED)
    libdwf.dwf_pv_apply.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, vp]
    assert libdwf.dwf_pv_apply(1, 2, 3, 4, 4, 4, 1, 0.1, -1.0, 5, 0, None) == -1
    assert libdwf.dwf_pv_apply(1, 2, 3, 4, 4, 4, 1, 0.1, -1.0, 4, 2, None) == -6


@pytest.mark.parametrize("order,lo,hi", [(0, 1.0, 25.0), (1, 1.0, 25.0), (2, 1.0, 30.0), (3, 0.5, 12.0)])
def test_pv_poly_chebyshev_coefficients_match_the_oracle(libdwf, order, lo, hi):
    """The library's minimax coefficients (host code, a three-term recurrence)
    against the oracle's (numpy's Chebyshev-to-power-series conversion)."""
    import numpy as np
    from oracle import dwf_oracle as O
    d = ctypes.c_double
    libdwf.dwf_pv_poly_chebyshev.argtypes = [ctypes.c_int, d, d, ctypes.POINTER(d)]
    c = (d * (order + 1))()
    assert libdwf.dwf_pv_poly_chebyshev(order, lo, hi, c) == 0
    want = O.pv_poly_chebyshev(order, lo, hi)
    assert np.allclose(np.array(c[:]), want, rtol=1e-12, atol=1e-15)


def test_pv_poly_arguments_rejected_on_the_host(libdwf):
    d, vp, i = ctypes.c_double, ctypes.c_void_p, ctypes.c_int
    libdwf.dwf_pv_poly_chebyshev.argtypes = [i, d, d, ctypes.POINTER(d)]
    c = (d * 8)()
    assert libdwf.dwf_pv_poly_chebyshev(4, 1.0, 25.0, c) == -1
    assert libdwf.dwf_pv_poly_chebyshev(1, 25.0, 1.0, c) == -1
    assert libdwf.dwf_pv_poly_chebyshev(1, 0.0, 1.0, c) == -1
    libdwf.dwf_pv_poly_apply.argtypes = [vp, vp, vp, i, i, i, i, d, d, ctypes.POINTER(d), i, i, vp]
    one = (d * 1)(1.0)
    assert libdwf.dwf_pv_poly_apply(1, 2, 3, 4, 4, 4, 1, 0.1, -1.0, one, 4, 0, None) == -1
    assert libdwf.dwf_pv_poly_apply(1, 2, 3, 4, 4, 4, 1, 0.1, -1.0, None, 0, 0, None) == -1
    nan = (d * 1)(float("nan"))
    assert libdwf.dwf_pv_poly_apply(1, 2, 3, 4, 4, 4, 1, 0.1, -1.0, nan, 0, 0, None) == -1


def _headline_params(dwfmg, **kw):
    p = dwfmg.MGParams(nvec=[16], block=[(4, 4)], Ls_coarse=[2], link_prec=[dwfmg.P_BF16], vec_prec=[dwfmg.P_F64],
                       fine_prec=dwfmg.P_F32, coarsest_solver=dwfmg.COARSEST_GCR, coarsest_restart=6,
                       coarsest_tol=0.25)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_workspace_bytes_on_the_host(libdwf):
    """mg_workspace_bytes needs no device: it lays the hierarchy out in counting
    mode.  At 256^2 x Ls 16 (16 null vectors, 4x4 aggregates, coarse Ls 2) the
    layout holds at least the operators: FP64 + BF16 coarse links (5 FP64
    blocks of 32^2 and 3 BF16 blocks per coarse site), FP64 + FP32
    prolongator, FP64 + FP32 fine links."""
    from paper_2004_07732_amd import dwfmg
    L, Ls = 256, 16
    p = _headline_params(dwfmg)
    b1 = dwfmg.workspace_bytes(L, L, Ls, p, 1)
    b16 = dwfmg.workspace_bytes(L, L, Ls, p, 16)
    sites_c = (L // 4) ** 2
    floor = (sites_c * 5 * 32 * 32 * 16 + sites_c * 3 * 32 * 32 * 4 + L * L * 2 * 16 * 24 + 2 * L * L * 24)
    assert floor < b1 < b16 < 64 * b1
    # the fine FP32 solve buffers grow with the column count: at least 16 of the outer GCR's
    # 2 x 16 directions per extra column (16.8 MB per FP32 fine vector)
    assert b16 - b1 >= 15 * 32 * (L * L * Ls * 2 * 8)
    # deflation adds its space (nev coarsest vectors of 64^2 x 2 x 32 FP64) and eigensolver buffers
    pc = _headline_params(dwfmg, coarsest_solver=dwfmg.COARSEST_CGNR, coarsest_nev=32)
    assert dwfmg.workspace_bytes(L, L, Ls, pc, 1) - dwfmg.workspace_bytes(
        L, L, Ls, _headline_params(dwfmg, coarsest_solver=dwfmg.COARSEST_CGNR), 1) >= 32 * sites_c * 2 * 32 * 16
    # invalid arguments give 0
    assert dwfmg.workspace_bytes(L, L, Ls, p, 0) == 0
    assert dwfmg.workspace_bytes(L, 250, Ls, p, 1) == 0
    assert dwfmg.workspace_bytes(L, L, 1, p, 1) == 0


def test_smoother_restart_parameters_on_the_host(libdwf):
    """Post-smoothing steps: at most 16 in one GCR cycle; with a restart length of
    1..16, up to 64 steps, and the smoother's direction buffers hold one cycle
    (24 steps in cycles of 6 need less memory than 16 steps in one cycle).  The
    stagnation ratio lies in [0, 1)."""
    from paper_2004_07732_amd import dwfmg
    L, Ls = 64, 8
    ok = lambda **kw: dwfmg.workspace_bytes(L, L, Ls, _headline_params(dwfmg, **kw), 1)
    assert ok(smooth_iters=16) > 0
    assert ok(smooth_iters=17) == 0
    assert ok(smooth_iters=24, smooth_restart=6) > 0
    assert ok(smooth_iters=64, smooth_restart=16) > 0
    assert ok(smooth_iters=65, smooth_restart=16) == 0
    assert ok(smooth_iters=16, smooth_restart=17) == 0
    assert ok(smooth_iters=16, smooth_restart=-1) == 0
    fine_vec = L * L * Ls * 2 * 8     # one FP32 fine vector
    assert ok(smooth_iters=16) - ok(smooth_iters=24, smooth_restart=6) >= 2 * 10 * fine_vec
    # the stagnation ratio: 0 (off) up to below 1
    assert ok(stagnation_ratio=0.0) > 0 and ok(stagnation_ratio=0.9) > 0
    assert ok(stagnation_ratio=1.0) == 0 and ok(stagnation_ratio=-0.5) == 0
    # a restart at least as long as the steps is no restart
    assert ok(smooth_iters=8, smooth_restart=8) == ok(smooth_iters=8) == ok(smooth_iters=8, smooth_restart=12)


def _span(src, header):
    """(start, end) of the brace-matched definition whose header matches `header`."""
    m = re.search(header, src, flags=re.M)
    assert m, header
    i = src.index("{", m.end() - 1)
    depth, j = 1, i + 1
    while depth:
        depth += {"{": 1, "}": -1}.get(src[j], 0)
        j += 1
    return m.start(), j


def test_device_allocation_only_where_documented():
    """After mg_setup no path of a hierarchy allocates device memory: the only
    hipMalloc / hipFree calls in the library are the workspace that mg_setup
    makes when the caller passes none (and its release), the library-owned
    scratch of dwf_pv_apply / dwf_pv_poly_apply / dwf_norm2 (acquire / drop),
    and the work vectors of dwf_krylov_solve (documented per call in the header).
    The allocation-free entry point and everything a solve runs allocate nothing."""
    allowed = {
        "mg.hip": [r"^int Hierarchy::setup\(", r"^Hierarchy::~Hierarchy\(\)"],
        "abi.hip": [r"^void\* acquire\(", r"^void drop\("],
        "krylov.hip": [r"^struct Work \{"],
    }
    csrc = os.path.join(ROOT, "paper_2004_07732_amd", "csrc")
    seen = set()
    for fn in sorted(os.listdir(csrc)):
        if not fn.endswith((".hip", ".hpp")):
            continue
        src = open(os.path.join(csrc, fn)).read()
        spans = [_span(src, h) for h in allowed.get(fn, [])]
        for m in re.finditer(r"\bhip(Malloc|Free|MallocManaged|ExtMallocWithFlags|MallocAsync|MallocPitch)\s*\(", src):
            inside = [k for k, (a, b) in enumerate(spans) if a <= m.start() < b]
            line = src.count("\n", 0, m.start()) + 1
            assert inside, f"{fn}:{line}: device allocation outside the documented places"
            seen.add((fn, inside[0]))
    assert ("mg.hip", 0) in seen and ("abi.hip", 0) in seen
