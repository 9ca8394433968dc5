// Allocation-free variant of the Pauli-Villars products (dwf_pv_apply_noalloc,
// declared in include/dwfmg.h), for callers that cannot allocate device memory.
//
// The intermediate field lives in a static device array, one copy per GPU,
// held until the process ends.  The array's name is only a host-side stand-in
// for the device copy: host code passes kernels the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept.
#include <cmath>
#include <mutex>

#include "../../include/dwfmg.h"
#include "kernels.hpp"

using namespace dwf;

namespace {

constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device
void* noalloc_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_noalloc_ptr[dev] = p;
    }
    return g_noalloc_ptr[dev];
}

inline int status_of(hipError_t e) { return e == hipSuccess ? DWF_OK : DWF_EHIP; }

template <typename R>
int pv_apply_noalloc_t(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, double m,
                       double M5, int mode, hipStream_t st) {
    auto u = reinterpret_cast<const cpx<R>*>(U);
    auto in = reinterpret_cast<const cpx<R>*>(psi);
    auto o = reinterpret_cast<cpx<R>*>(out);
    if (mode == DWF_PV || mode == DWF_PV_DAG)
        return status_of(fine_dw_untimed<R>(u, in, o, Lx, Ly, Ls, nrhs, 1.0, M5, mode == DWF_PV_DAG, st));
    const size_t bytes = sizeof(cpx<R>) * 2 * (size_t)Lx * Ly * Ls * nrhs;
    if (bytes > kNoAllocBytes) return DWF_ESCRATCH;
    auto t = reinterpret_cast<cpx<R>*>(noalloc_scratch());
    if (!t) return DWF_EHIP;
    // the first stencil overwrites every entry of the intermediate field, so
    // nothing has to be cleared between calls
    const double m1 = (mode == DWF_PVDAG_DW) ? m : 1.0, m2 = (mode == DWF_PVDAG_DW) ? 1.0 : m;
    if (fine_dw_untimed<R>(u, in, t, Lx, Ly, Ls, nrhs, m1, M5, false, st) != hipSuccess) return DWF_EHIP;
    return status_of(fine_dw_untimed<R>(u, t, o, Lx, Ly, Ls, nrhs, m2, M5, true, st));
}

}  // namespace

extern "C" {

int dwf_pv_apply_noalloc(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, double m_f,
                         double M5, int mode, int flags, void* stream) {
    if (!U || !psi || !out || psi == out) return DWF_EINVAL;
    if (Lx < 1 || Ly < 1 || Ls < 1 || nrhs < 1 || (long long)Lx * Ly >= (1LL << 30) ||
        (long long)Lx * Ly * Ls * nrhs >= (1LL << 40))
        return DWF_EINVAL;
    if (!std::isfinite(m_f) || !std::isfinite(M5) || mode < DWF_PV || mode > DWF_PVINV_DW) return DWF_EINVAL;
    if (mode == DWF_PVINV_DW) return DWF_EUNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (flags & DWF_PREC_F32) return pv_apply_noalloc_t<float>(U, psi, out, Lx, Ly, Ls, nrhs, m_f, M5, mode, st);
    return pv_apply_noalloc_t<double>(U, psi, out, Lx, Ly, Ls, nrhs, m_f, M5, mode, st);
}

size_t dwf_pv_apply_noalloc_max_bytes(void) { return kNoAllocBytes; }

}  // extern "C"
