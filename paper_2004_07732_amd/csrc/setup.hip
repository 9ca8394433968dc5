// Multigrid setup kernels (Sec. 2.3 and Sec. 3.1): chiral doubling of the
// relaxed near-null vectors, block Gram-Schmidt (P^dagger P = 1 per aggregate
// and chirality, so gamma_5 P = P sigma_3), and the Galerkin coarse kernel
// P^dagger D_W P in stencil form.  All in FP64.
//
// Galerkin term by term: a hop of type h from fine site x to x+h contributes
// V(x)^dag H_h(x) V(x+h) to the coarse diagonal block when x+h stays in the
// aggregate, and to the coarse hop of type h otherwise.  "Leaves the aggregate"
// is decided on the fine local coordinate (x_mu mod b_mu == b_mu - 1 for a
// forward hop), which stays correct for coarse extents 1 and 2 with periodic wrap.
#include "kernels.hpp"

namespace dwf {

namespace {
__device__ __forceinline__ int hop_nbr(int x, int y, int Lx, int Ly, int h) {
    switch (h) {
        case 1: x = (x + 1 == Lx) ? 0 : x + 1; break;
        case 2: x = (x == 0) ? Lx - 1 : x - 1; break;
        case 3: y = (y + 1 == Ly) ? 0 : y + 1; break;
        case 4: y = (y == 0) ? Ly - 1 : y - 1; break;
        default: break;
    }
    return y * Lx + x;
}
__device__ __forceinline__ bool hop_leaves(int lx, int ly, int bx, int by, int h) {
    switch (h) {
        case 1: return lx == bx - 1;
        case 2: return lx == 0;
        case 3: return ly == by - 1;
        case 4: return ly == 0;
        default: return false;
    }
}
// spin part of the fine Wilson hop of type h, without the -1/2 and the link:
// +x: (1 - s1), -x: (1 + s1), +y: (1 - s2), -y: (1 + s2)
__device__ __forceinline__ cpx<double> hop_spin(int h, int a, int b) {
    if (a == b) return {1.0, 0.0};
    switch (h) {
        case 1: return {-1.0, 0.0};
        case 2: return {1.0, 0.0};
        case 3: return (a == 0) ? cpx<double>{0.0, 1.0} : cpx<double>{0.0, -1.0};
        case 4: return (a == 0) ? cpx<double>{0.0, -1.0} : cpx<double>{0.0, 1.0};
        default: return {0.0, 0.0};
    }
}
}  // namespace

// ------------------------------------------------------------ chiral doubling
__global__ void k_chiral_columns(const cpx<double>* v, cpx<double>* V, int nsites, int nc, int nvec) {
    const long long total = (long long)nsites * 2 * nc * nvec;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int k = (int)(t % nvec);
    const long long r = t / nvec;          // (site*2 + c)*nc + j
    const int cj = (int)(r % (2 * nc));
    const int site = (int)(r / (2 * nc));
    V[t] = v[((size_t)k * nsites + site) * 2 * nc + cj];
}
hipError_t chiral_columns(const cpx<double>* v, cpx<double>* V, int nsites, int nc, int nvec, hipStream_t st) {
    const long long total = (long long)nsites * 2 * nc * nvec;
    hipLaunchKernelGGL(k_chiral_columns, dim3(grid_for(total)), dim3(kBlock), 0, st, v, V, nsites, nc, nvec);
    return hipGetLastError();
}

// ------------------------------------------------------------ block Gram-Schmidt
// One workgroup per (aggregate, chirality).  The aggregate's columns are held
// in LDS as Q[e][k], e = (local y, local x, j).  Classical Gram-Schmidt twice:
// thread i < k computes the coefficient <q_i, v_k> serially over e (fixed
// order), then every thread updates its elements.
__global__ void __launch_bounds__(kBlock)
k_block_orth(cpx<double>* V, int Lx, int Ly, int nc, int nvec, int bx, int by, int* bad) {
    extern __shared__ unsigned char smem_raw[];
    cpx<double>* Q = reinterpret_cast<cpx<double>*>(smem_raw);
    __shared__ cpx<double> coef[64];
    __shared__ double nrm2, nrm2_0;
    const int cX = Lx / bx;
    const int agg = blockIdx.x;
    const int c = blockIdx.y;
    const int X = agg % cX, Y = agg / cX;
    const int Lb = bx * by * nc;
    auto vidx = [&](int e, int k) -> size_t {
        const int j = e % nc, l = e / nc;
        const int lx = l % bx, ly = l / bx;
        const int site = (Y * by + ly) * Lx + X * bx + lx;
        return (((size_t)site * 2 + c) * nc + j) * nvec + k;
    };
    for (int t = threadIdx.x; t < Lb * nvec; t += blockDim.x) {
        const int e = t / nvec, k = t - e * nvec;
        Q[t] = V[vidx(e, k)];
    }
    __syncthreads();
    for (int k = 0; k < nvec; ++k) {
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int e = 0; e < Lb; ++e) s += Q[e * nvec + k].re * Q[e * nvec + k].re + Q[e * nvec + k].im * Q[e * nvec + k].im;
            nrm2_0 = s;
        }
        __syncthreads();
        for (int pass = 0; pass < 2 && k > 0; ++pass) {
            if (threadIdx.x < k) {
                const int i = threadIdx.x;
                cpx<double> s = {0.0, 0.0};
                for (int e = 0; e < Lb; ++e) {
                    const cpx<double> p = cjmul(Q[e * nvec + i], Q[e * nvec + k]);
                    s.re += p.re;
                    s.im += p.im;
                }
                coef[i] = s;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < Lb; e += blockDim.x) {
                cpx<double> v = Q[e * nvec + k];
                for (int i = 0; i < k; ++i) {
                    const cpx<double> t = cmul(coef[i], Q[e * nvec + i]);
                    v.re -= t.re;
                    v.im -= t.im;
                }
                Q[e * nvec + k] = v;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int e = 0; e < Lb; ++e) s += Q[e * nvec + k].re * Q[e * nvec + k].re + Q[e * nvec + k].im * Q[e * nvec + k].im;
            nrm2 = s;
            if (!(s > 1e-24 * nrm2_0) || !(s > 0.0)) bad[0] = 1;
        }
        __syncthreads();
        const double inv = (nrm2 > 0.0) ? 1.0 / sqrt(nrm2) : 0.0;
        for (int e = threadIdx.x; e < Lb; e += blockDim.x) {
            Q[e * nvec + k].re *= inv;
            Q[e * nvec + k].im *= inv;
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < Lb * nvec; t += blockDim.x) {
        const int e = t / nvec, k = t - e * nvec;
        V[vidx(e, k)] = Q[t];
    }
}

hipError_t block_orthonormalize(cpx<double>* V, int Lx, int Ly, int nc, int nvec, int bx, int by,
                                int* bad, hipStream_t st) {
    const size_t shm = (size_t)bx * by * nc * nvec * sizeof(cpx<double>);
    if (shm > 64 * 1024 || nvec > 64) return hipErrorInvalidValue;
    dim3 grid((Lx / bx) * (Ly / by), 2);
    hipLaunchKernelGGL(k_block_orth, grid, dim3(kBlock), shm, st, V, Lx, Ly, nc, nvec, bx, by, bad);
    return hipGetLastError();
}

// ------------------------------------------------------------ Galerkin, level 0
// Output column layout: links[((X*5 + d)*n + b)*n + a] = block_d[a][b], n = 2 nvec.
__global__ void k_galerkin_fine(const cpx<double>* U, const cpx<double>* V, cpx<double>* links,
                                int Lx, int Ly, int nvec, int bx, int by) {
    const int n = 2 * nvec;
    const int cX = Lx / bx, cY = Ly / by;
    const long long total = (long long)cX * cY * 5 * n * n;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int a = (int)(t % n);
    const int b = (int)((t / n) % n);
    const int d = (int)((t / ((long long)n * n)) % 5);
    const int cs = (int)(t / (5LL * n * n));
    const int ca = a / nvec, ka = a - ca * nvec;
    const int cb = b / nvec, kb = b - cb * nvec;
    const int X = cs % cX, Y = cs / cX;
    const int V2 = Lx * Ly;
    cpx<double> acc = {0.0, 0.0};
    for (int ly = 0; ly < by; ++ly)
        for (int lx = 0; lx < bx; ++lx) {
            const int x = X * bx + lx, y = Y * by + ly;
            const int site = y * Lx + x;
            const cpx<double> va = V[((size_t)site * 2 + ca) * nvec + ka];
            if (d == 0 && ca == cb) {
                // site-diagonal term d * 1 of D_W(0)
                const cpx<double> vb = V[((size_t)site * 2 + cb) * nvec + kb];
                const cpx<double> p = cjmul(va, vb);
                acc.re += 2.0 * p.re;
                acc.im += 2.0 * p.im;
            }
            for (int h = 1; h <= 4; ++h) {
                const bool leaves = hop_leaves(lx, ly, bx, by, h);
                if ((d == 0 && leaves) || (d != 0 && (d != h || !leaves))) continue;
                const int nbs = hop_nbr(x, y, Lx, Ly, h);
                cpx<double> link;
                switch (h) {
                    case 1: link = U[site]; break;
                    case 2: link = conj(U[hop_nbr(x, y, Lx, Ly, 2)]); break;
                    case 3: link = U[V2 + site]; break;
                    default: link = conj(U[V2 + hop_nbr(x, y, Lx, Ly, 4)]); break;
                }
                const cpx<double> spin = hop_spin(h, ca, cb);
                const cpx<double> vb = V[((size_t)nbs * 2 + cb) * nvec + kb];
                const cpx<double> hv = cmul(cmul(spin, link), vb);
                const cpx<double> p = cjmul(va, hv);
                acc.re -= 0.5 * p.re;
                acc.im -= 0.5 * p.im;
            }
        }
    links[(((size_t)cs * 5 + d) * n + b) * n + a] = acc;
}

hipError_t galerkin_fine(const cpx<double>* U, const cpx<double>* V, cpx<double>* links,
                         int Lx, int Ly, int nvec, int bx, int by, hipStream_t st) {
    const int n = 2 * nvec;
    const long long total = (long long)(Lx / bx) * (Ly / by) * 5 * n * n;
    hipLaunchKernelGGL(k_galerkin_fine, dim3(grid_for(total)), dim3(kBlock), 0, st, U, V, links, Lx, Ly, nvec, bx, by);
    return hipGetLastError();
}

// ------------------------------------------------------------ Galerkin, level >= 1
__global__ void k_galerkin_coarse(const cpx<double>* S, const cpx<double>* V, cpx<double>* links,
                                  int Lx, int Ly, int nc, int nvec, int bx, int by) {
    const int n = 2 * nvec, nf = 2 * nc;
    const int cX = Lx / bx, cY = Ly / by;
    const long long total = (long long)cX * cY * 5 * n * n;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int a = (int)(t % n);
    const int b = (int)((t / n) % n);
    const int d = (int)((t / ((long long)n * n)) % 5);
    const int cs = (int)(t / (5LL * n * n));
    const int ca = a / nvec, ka = a - ca * nvec;
    const int cb = b / nvec, kb = b - cb * nvec;
    const int X = cs % cX, Y = cs / cX;
    cpx<double> acc = {0.0, 0.0};
    for (int ly = 0; ly < by; ++ly)
        for (int lx = 0; lx < bx; ++lx) {
            const int x = X * bx + lx, y = Y * by + ly;
            const int site = y * Lx + x;
            for (int h = 0; h <= 4; ++h) {
                const bool leaves = hop_leaves(lx, ly, bx, by, h);
                if ((d == 0 && leaves) || (d != 0 && (d != h || !leaves))) continue;
                const int nbs = hop_nbr(x, y, Lx, Ly, h);
                const cpx<double>* blk = S + ((size_t)site * 5 + h) * nf * nf;   // blk[col][row]
                for (int j = 0; j < nc; ++j) {
                    const cpx<double> va = V[(((size_t)site * 2 + ca) * nc + j) * nvec + ka];
                    const int row = ca * nc + j;
                    cpx<double> s = {0.0, 0.0};
                    for (int jp = 0; jp < nc; ++jp) {
                        const int colf = cb * nc + jp;
                        const cpx<double> vb = V[(((size_t)nbs * 2 + cb) * nc + jp) * nvec + kb];
                        cfma(s, blk[(size_t)colf * nf + row], vb);
                    }
                    const cpx<double> p = cjmul(va, s);
                    acc.re += p.re;
                    acc.im += p.im;
                }
            }
        }
    links[(((size_t)cs * 5 + d) * n + b) * n + a] = acc;
}

hipError_t galerkin_coarse(const cpx<double>* S, const cpx<double>* V, cpx<double>* links,
                           int Lx, int Ly, int nc, int nvec, int bx, int by, hipStream_t st) {
    const int n = 2 * nvec;
    const long long total = (long long)(Lx / bx) * (Ly / by) * 5 * n * n;
    hipLaunchKernelGGL(k_galerkin_coarse, dim3(grid_for(total)), dim3(kBlock), 0, st, S, V, links, Lx, Ly, nc, nvec, bx, by);
    return hipGetLastError();
}

// ------------------------------------------------------------ storage conversion
__global__ void k_links_f32(const cpx<double>* in, cpx<float>* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = {(float)in[i].re, (float)in[i].im};
}
__global__ void k_links_bf16(const cpx<double>* in, cbf16* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t re = f32_to_bf16_bits((float)in[i].re), im = f32_to_bf16_bits((float)in[i].im);
        out[i].v = re | (im << 16);
    }
}
__global__ void k_links_f16(const cpx<double>* in, cf16* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = {(_Float16)(float)in[i].re, (_Float16)(float)in[i].im};
}
__global__ void k_links_f64(const cpx<double>* in, cpx<double>* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

hipError_t convert_links(const cpx<double>* in, void* out, int prec, size_t n, hipStream_t st) {
    unsigned g = grid_for((long long)n);
    if (g > 8192) g = 8192;
    switch (prec) {
        case P_F64: hipLaunchKernelGGL(k_links_f64, dim3(g), dim3(kBlock), 0, st, in, (cpx<double>*)out, n); break;
        case P_F32: hipLaunchKernelGGL(k_links_f32, dim3(g), dim3(kBlock), 0, st, in, (cpx<float>*)out, n); break;
        case P_BF16: hipLaunchKernelGGL(k_links_bf16, dim3(g), dim3(kBlock), 0, st, in, (cbf16*)out, n); break;
        case P_F16: hipLaunchKernelGGL(k_links_f16, dim3(g), dim3(kBlock), 0, st, in, (cf16*)out, n); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// column layout -> stencil form: diag[site][i][k], then hop[h][site][i][k]
__global__ void k_export_links(const cpx<double>* links, cpx<double>* out, int nsites, int n) {
    const long long total = (long long)nsites * 5 * n * n;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int k = (int)(t % n);
    const int i = (int)((t / n) % n);
    const int site = (int)((t / ((long long)n * n)) % nsites);
    const int d = (int)(t / ((long long)n * n * nsites));
    out[t] = links[(((size_t)site * 5 + d) * n + k) * n + i];
}
hipError_t export_links(const cpx<double>* links, cpx<double>* out, int nsites, int n, hipStream_t st) {
    const long long total = (long long)nsites * 5 * n * n;
    hipLaunchKernelGGL(k_export_links, dim3(grid_for(total)), dim3(kBlock), 0, st, links, out, nsites, n);
    return hipGetLastError();
}

}  // namespace dwf
