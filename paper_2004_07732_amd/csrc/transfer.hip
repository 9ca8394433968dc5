// Wall-only restriction and prolongation (eq. TruncProjectInterpolate).
//
// Both walls sit on slice 1 of the permuted chiral basis of Sec. 2.2, whose
// slice 1 is P_- r_1 + P_+ r_Ls.  Because the prolongator keeps chirality
// (gamma_5 P = P sigma_3), the transfer splits by chirality:
//   restriction : rc_1 = hatP_- P^dag r_1 (from the - components of fine slice 1),
//                 rc_Lsc = hatP_+ P^dag r_Ls (from the + components of slice Ls),
//                 every other coarse entry zero;
//   prolongation: e_1 = P hatP_- ec_1, e_Ls = P hatP_+ ec_Lsc, bulk zero.
// Prolongator layout V[site][c][j][k]: chirality c, internal dof j of the
// fine site (nc per chirality), coarse vector k (nvec per chirality).
#include "kernels.hpp"

namespace dwf {

// one thread per (column, coarse site, coarse dof a); writes all Lsc slices
template <typename T>
__global__ void k_restrict_wall(const cpx<T>* __restrict__ V, const cpx<T>* __restrict__ r,
                                cpx<T>* __restrict__ rc, TransferGeom g, int ncol) {
    const int nf = 2 * g.nc, ncd = 2 * g.nvec;
    const int cX = g.Lx / g.bx, cY = g.Ly / g.by;
    const int csites = cX * cY;
    const long long total = (long long)ncol * csites * ncd;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int a = (int)(t % ncd);
    const int cs = (int)((t / ncd) % csites);
    const int col = (int)(t / ((long long)ncd * csites));
    const int c = a / g.nvec, k = a - c * g.nvec;
    const int X = cs % cX, Y = cs / cX;
    const int V2 = g.Lx * g.Ly;
    // chirality - comes from fine slice 1, chirality + from fine slice Ls (the
    // literal toggle takes both from fine slice 1)
    const int sf = (c == 1 || g.literal) ? 0 : g.Ls - 1;
    const cpx<T>* rs = r + ((size_t)col * g.Ls + sf) * V2 * nf;
    cpx<double> acc = {0.0, 0.0};
    for (int by = 0; by < g.by; ++by)
        for (int bx = 0; bx < g.bx; ++bx) {
            const int site = (Y * g.by + by) * g.Lx + X * g.bx + bx;
            for (int j = 0; j < g.nc; ++j) {
                const cpx<T> v = V[(((size_t)site * 2 + c) * g.nc + j) * g.nvec + k];
                const cpx<T> x = rs[(size_t)site * nf + c * g.nc + j];
                acc.re += (double)v.re * x.re + (double)v.im * x.im;
                acc.im += (double)v.re * x.im - (double)v.im * x.re;
            }
        }
    cpx<T>* out = rc + (size_t)col * g.Lsc * csites * ncd;
    const int swall = (c == 1 || g.literal) ? 0 : g.Lsc - 1;
    for (int s = 0; s < g.Lsc; ++s) {
        cpx<T> v = {T(0), T(0)};
        if (s == swall) v = {(T)acc.re, (T)acc.im};
        out[((size_t)s * csites + cs) * ncd + a] = v;
    }
}

// one thread per (column, fine site, fine dof); writes all Ls slices
template <typename T>
__global__ void k_prolong_wall(const cpx<T>* __restrict__ V, const cpx<T>* __restrict__ ec,
                               cpx<T>* __restrict__ e, TransferGeom g, int ncol) {
    const int nf = 2 * g.nc, ncd = 2 * g.nvec;
    const int cX = g.Lx / g.bx, cY = g.Ly / g.by;
    const int csites = cX * cY;
    const int V2 = g.Lx * g.Ly;
    const long long total = (long long)ncol * V2 * nf;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int af = (int)(t % nf);
    const int site = (int)((t / nf) % V2);
    const int col = (int)(t / ((long long)nf * V2));
    const int c = af / g.nc, j = af - c * g.nc;
    const int x = site % g.Lx, y = site / g.Lx;
    const int cs = (y / g.by) * cX + x / g.bx;
    const int swall_c = (c == 1 || g.literal) ? 0 : g.Lsc - 1;
    const cpx<T>* ev = ec + (((size_t)col * g.Lsc + swall_c) * csites + cs) * ncd + c * g.nvec;
    const cpx<T>* vrow = V + (((size_t)site * 2 + c) * g.nc + j) * g.nvec;
    cpx<double> acc = {0.0, 0.0};
    for (int k = 0; k < g.nvec; ++k) {
        const cpx<T> v = vrow[k], x = ev[k];
        acc.re += (double)v.re * x.re - (double)v.im * x.im;
        acc.im += (double)v.re * x.im + (double)v.im * x.re;
    }
    cpx<T>* out = e + (size_t)col * g.Ls * V2 * nf;
    const int swall_f = (c == 1 || g.literal) ? 0 : g.Ls - 1;
    for (int s = 0; s < g.Ls; ++s) {
        cpx<T> v = {T(0), T(0)};
        if (s == swall_f) v = {(T)acc.re, (T)acc.im};
        out[((size_t)s * V2 + site) * nf + af] = v;
    }
}

// Bulk transfer (Sec. 4.1, the alternative to the boundary-only transfer): the
// 2-d prolongator repeated on every slice, coarse slice s <-> fine slice s
// (requires Lsc == Ls).  Restriction: rc_s = P^dag r_s; prolongation: e_s = P ec_s.
template <typename T>
__global__ void k_restrict_bulk(const cpx<T>* __restrict__ V, const cpx<T>* __restrict__ r,
                                cpx<T>* __restrict__ rc, TransferGeom g, int ncol) {
    const int nf = 2 * g.nc, ncd = 2 * g.nvec;
    const int cX = g.Lx / g.bx, cY = g.Ly / g.by;
    const int csites = cX * cY;
    const long long total = (long long)ncol * g.Ls * csites * ncd;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int a = (int)(t % ncd);
    const int cs = (int)((t / ncd) % csites);
    const long long cslab = t / ((long long)ncd * csites);   // col * Ls + s
    const int c = a / g.nvec, k = a - c * g.nvec;
    const int X = cs % cX, Y = cs / cX;
    const int V2 = g.Lx * g.Ly;
    const cpx<T>* rs = r + (size_t)cslab * V2 * nf;
    cpx<double> acc = {0.0, 0.0};
    for (int by = 0; by < g.by; ++by)
        for (int bx = 0; bx < g.bx; ++bx) {
            const int site = (Y * g.by + by) * g.Lx + X * g.bx + bx;
            for (int j = 0; j < g.nc; ++j) {
                const cpx<T> v = V[(((size_t)site * 2 + c) * g.nc + j) * g.nvec + k];
                const cpx<T> x = rs[(size_t)site * nf + c * g.nc + j];
                acc.re += (double)v.re * x.re + (double)v.im * x.im;
                acc.im += (double)v.re * x.im - (double)v.im * x.re;
            }
        }
    rc[((size_t)cslab * csites + cs) * ncd + a] = {(T)acc.re, (T)acc.im};
}

template <typename T>
__global__ void k_prolong_bulk(const cpx<T>* __restrict__ V, const cpx<T>* __restrict__ ec,
                               cpx<T>* __restrict__ e, TransferGeom g, int ncol) {
    const int nf = 2 * g.nc, ncd = 2 * g.nvec;
    const int cX = g.Lx / g.bx, cY = g.Ly / g.by;
    const int csites = cX * cY;
    const int V2 = g.Lx * g.Ly;
    const long long total = (long long)ncol * g.Ls * V2 * nf;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int af = (int)(t % nf);
    const int site = (int)((t / nf) % V2);
    const long long cslab = t / ((long long)nf * V2);         // col * Ls + s
    const int c = af / g.nc, j = af - c * g.nc;
    const int x = site % g.Lx, y = site / g.Lx;
    const int cs = (y / g.by) * cX + x / g.bx;
    const cpx<T>* ev = ec + ((size_t)cslab * csites + cs) * ncd + c * g.nvec;
    const cpx<T>* vrow = V + (((size_t)site * 2 + c) * g.nc + j) * g.nvec;
    cpx<double> acc = {0.0, 0.0};
    for (int k = 0; k < g.nvec; ++k) {
        const cpx<T> v = vrow[k], xx = ev[k];
        acc.re += (double)v.re * xx.re - (double)v.im * xx.im;
        acc.im += (double)v.re * xx.im + (double)v.im * xx.re;
    }
    e[((size_t)cslab * V2 + site) * nf + af] = {(T)acc.re, (T)acc.im};
}

template <typename T>
hipError_t restrict_bulk(const cpx<T>* V, const cpx<T>* r, cpx<T>* rc, const TransferGeom& g, int ncol, hipStream_t st) {
    if (g.Lsc != g.Ls) return hipErrorInvalidValue;
    const long long total = (long long)ncol * g.Ls * (g.Lx / g.bx) * (g.Ly / g.by) * 2 * g.nvec;
    hipLaunchKernelGGL(k_restrict_bulk<T>, dim3(grid_for(total)), dim3(kBlock), 0, st, V, r, rc, g, ncol);
    return hipGetLastError();
}
template <typename T>
hipError_t prolong_bulk(const cpx<T>* V, const cpx<T>* ec, cpx<T>* e, const TransferGeom& g, int ncol, hipStream_t st) {
    if (g.Lsc != g.Ls) return hipErrorInvalidValue;
    const long long total = (long long)ncol * g.Ls * g.Lx * g.Ly * 2 * g.nc;
    hipLaunchKernelGGL(k_prolong_bulk<T>, dim3(grid_for(total)), dim3(kBlock), 0, st, V, ec, e, g, ncol);
    return hipGetLastError();
}

template <typename T>
hipError_t restrict_wall(const cpx<T>* V, const cpx<T>* r, cpx<T>* rc, const TransferGeom& g, int ncol, hipStream_t st) {
    const long long total = (long long)ncol * (g.Lx / g.bx) * (g.Ly / g.by) * 2 * g.nvec;
    hipLaunchKernelGGL(k_restrict_wall<T>, dim3(grid_for(total)), dim3(kBlock), 0, st, V, r, rc, g, ncol);
    return hipGetLastError();
}
template <typename T>
hipError_t prolong_wall(const cpx<T>* V, const cpx<T>* ec, cpx<T>* e, const TransferGeom& g, int ncol, hipStream_t st) {
    const long long total = (long long)ncol * g.Lx * g.Ly * 2 * g.nc;
    hipLaunchKernelGGL(k_prolong_wall<T>, dim3(grid_for(total)), dim3(kBlock), 0, st, V, ec, e, g, ncol);
    return hipGetLastError();
}

template hipError_t restrict_wall<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, const TransferGeom&, int, hipStream_t);
template hipError_t restrict_wall<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, const TransferGeom&, int, hipStream_t);
template hipError_t prolong_wall<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, const TransferGeom&, int, hipStream_t);
template hipError_t prolong_wall<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, const TransferGeom&, int, hipStream_t);
template hipError_t restrict_bulk<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, const TransferGeom&, int, hipStream_t);
template hipError_t restrict_bulk<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, const TransferGeom&, int, hipStream_t);
template hipError_t prolong_bulk<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, const TransferGeom&, int, hipStream_t);
template hipError_t prolong_bulk<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, const TransferGeom&, int, hipStream_t);

}  // namespace dwf
