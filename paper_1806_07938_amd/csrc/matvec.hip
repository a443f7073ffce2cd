// The fused 2RBT product y = W_s (Sigma_ss + Sigma_eta) W_s^T x (§2.E, Sigma_ss
// zeta equation; §2.F masks), one launch per phase.
//
// The two-dimensional transform of every channel is split into a row pass
// (along x, real input -> half spectrum f2 in [0, L/2]) and a column pass
// (along y).  The column pass owns one f2 column of all C = 2G channels, so
// it also does the per-frequency products summed over input channels and the
// inverse column transform; the inverse row pass then returns to the n x n
// grid, restricted to valid subapertures, and adds the noise term.
//
//   row_fwd : T[f2][c][a]  = sum_{b<n} x_c[a][b] exp(-2 pi i f2 b / L)         (S1, F along x)
//   col_pass: X[c][f1]     = sum_{a<n} T[f2][c][a] exp(-2 pi i f1 a / L)        (F along y)
//             Y[p][f1]     = sum_q M_pq(f1, f2) X[q][f1]                        (products, summed)
//             U[f2][p][a]  = sum_{f1<L} Y[p][f1] exp(+2 pi i f1 a / L), a < n  (F^-1 along y, S2 rows)
//   row_inv : y_p[a][b]    = L^-2 sum_{f2} w(f2) Re(U[f2][p][a] exp(+2 pi i f2 b / L)),
//             w = 1 for f2 = 0 and f2 = L/2, else 2 (real output)               (F^-1 along x, S2, W_s)
//             out = y + sigma^2 x (+ the x-y noise covariance times the other
//             slope of the subaperture when Sigma_eta has 2x2 blocks, §2.F)
//
// Inputs are only nonzero on the n x n top-left corner of the L x L embedding
// and only that corner of the output is read (pruned transforms).
#include "tt_internal.h"

template <typename R>
__global__ void k_row_fwd(const R* __restrict__ x, const int* __restrict__ vmap, const cplx<R>* __restrict__ tw,
                          cplx<R>* __restrict__ T, int n, int C, int L, int Lh, int n_vs) {
    __shared__ R xs[512];
    __shared__ cplx<R> tws[1024];
    const int row = blockIdx.x;
    const int c = row / n, a = row % n;
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
        const int v = vmap[a * n + b];
        xs[b] = v >= 0 ? x[(long)c * n_vs + v] : R(0);
    }
    for (int k = threadIdx.x; k < L; k += blockDim.x) tws[k] = tw[k];
    __syncthreads();
    for (int f2 = threadIdx.x; f2 < Lh; f2 += blockDim.x) {
        R re = 0, im = 0;
        int m = 0;
        for (int b = 0; b < n; ++b) {
            const cplx<R> w = tws[m];
            re += xs[b] * w.x;
            im -= xs[b] * w.y;
            m += f2;
            if (m >= L) m -= L;
        }
        T[((long)f2 * C + c) * n + a] = cplx<R>{re, im};
    }
}

template <typename R>
__global__ void k_col_pass(const cplx<R>* __restrict__ T, const R* __restrict__ M, const cplx<R>* __restrict__ tw,
                           cplx<R>* __restrict__ U, int n, int G, int L, int Lh) {
    extern __shared__ char smem_raw[];
    cplx<R>* sm = reinterpret_cast<cplx<R>*>(smem_raw);
    const int C = 2 * G;
    const int P = 3 * G * G;
    cplx<R>* tws = sm;
    cplx<R>* Tc = tws + L;
    cplx<R>* Xh = Tc + C * n;
    cplx<R>* Yh = Xh + C * L;
    const int f2 = blockIdx.x;
    for (int k = threadIdx.x; k < L; k += blockDim.x) tws[k] = tw[k];
    for (int k = threadIdx.x; k < C * n; k += blockDim.x) Tc[k] = T[(long)f2 * C * n + k];
    __syncthreads();
    // forward column transform
    for (int idx = threadIdx.x; idx < C * L; idx += blockDim.x) {
        const int c = idx / L, f1 = idx % L;
        R re = 0, im = 0;
        int m = 0;
        for (int a = 0; a < n; ++a) {
            const cplx<R> t = Tc[c * n + a];
            const cplx<R> w = tws[m];
            re += t.x * w.x + t.y * w.y;
            im += t.y * w.x - t.x * w.y;
            m += f1;
            if (m >= L) m -= L;
        }
        Xh[idx] = cplx<R>{re, im};
    }
    __syncthreads();
    // per-frequency products summed over input channels (Hermitian packed M)
    for (int idx = threadIdx.x; idx < C * L; idx += blockDim.x) {
        const int p = idx / L, f1 = idx % L;
        const R* Mf = M + ((long)f2 * L + f1) * P;
        const int g = p >> 1, pp = p & 1;
        R re = 0, im = 0;
        for (int q = 0; q < C; ++q) {
            const int h = q >> 1, comp = pp + (q & 1);
            R mr, mi;
            if (g == h) {
                mr = Mf[3 * g + comp];
                mi = 0;
            } else if (g < h) {
                const int s = 3 * G + 6 * (g * (2 * G - g - 1) / 2 + (h - g - 1)) + 2 * comp;
                mr = Mf[s];
                mi = Mf[s + 1];
            } else {
                const int s = 3 * G + 6 * (h * (2 * G - h - 1) / 2 + (g - h - 1)) + 2 * comp;
                mr = Mf[s];
                mi = -Mf[s + 1];
            }
            const cplx<R> xv = Xh[q * L + f1];
            re += mr * xv.x - mi * xv.y;
            im += mr * xv.y + mi * xv.x;
        }
        Yh[idx] = cplx<R>{re, im};
    }
    __syncthreads();
    // inverse column transform, rows a < n only
    for (int idx = threadIdx.x; idx < C * n; idx += blockDim.x) {
        const int p = idx / n, a = idx % n;
        R re = 0, im = 0;
        int m = 0;
        for (int f1 = 0; f1 < L; ++f1) {
            const cplx<R> y = Yh[p * L + f1];
            const cplx<R> w = tws[m];
            re += y.x * w.x - y.y * w.y;
            im += y.x * w.y + y.y * w.x;
            m += a;
            if (m >= L) m -= L;
        }
        U[((long)f2 * C + p) * n + a] = cplx<R>{re, im};
    }
}

template <typename R>
__global__ void k_row_inv(const cplx<R>* __restrict__ U, const cplx<R>* __restrict__ tw, const int* __restrict__ vmap,
                          const R* __restrict__ x, const R* __restrict__ noise, const R* __restrict__ nxy,
                          R* __restrict__ y, double* __restrict__ part, int n, int C, int L, int Lh, int n_vs) {
    __shared__ cplx<R> Us[513];
    __shared__ cplx<R> tws[1024];
    __shared__ double red[256];
    const int row = blockIdx.x;
    const int c = row / n, a = row % n;
    for (int f2 = threadIdx.x; f2 < Lh; f2 += blockDim.x) Us[f2] = U[((long)f2 * C + c) * n + a];
    for (int k = threadIdx.x; k < L; k += blockDim.x) tws[k] = tw[k];
    __syncthreads();
    const R inv = R(1) / (R(L) * R(L));
    const bool even = (L % 2) == 0;
    double acc_dot = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
        const int v = vmap[a * n + b];
        if (v < 0) continue;
        R s = Us[0].x;
        int m = b;
        for (int f2 = 1; f2 < Lh; ++f2) {
            const cplx<R> u = Us[f2];
            const cplx<R> w = tws[m];
            const R wt = (even && 2 * f2 == L) ? R(1) : R(2);
            s += wt * (u.x * w.x - u.y * w.y);
            m += b;
            if (m >= L) m -= L;
        }
        const long i = (long)c * n_vs + v;
        R out = s * inv + noise[i] * x[i];
        // 2x2 noise blocks: x-y covariance of this subaperture times the other slope
        if (nxy) out += nxy[(long)(c >> 1) * n_vs + v] * x[(long)(c ^ 1) * n_vs + v];
        y[i] = out;
        acc_dot += (double)x[i] * (double)out;
    }
    if (part) {
        red[threadIdx.x] = acc_dot;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[row] = red[0];
    }
}

namespace {

size_t col_pass_lds(const tt_ctx& c, size_t elem) { return elem * ((size_t)c.L + (size_t)c.C * c.n + 2ull * c.C * c.L); }

template <typename R>
__global__ void k_copy_vec(const R* __restrict__ a, R* __restrict__ b, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = a[i];
}

tt_status mode_project(tt_ctx& c, float* v) { return modes_project_f32(c, v); }
tt_status mode_project(tt_ctx& c, double* v) { return modes_project_f64(c, v); }

// With mode removal (§2.F) the product is M A M x: the input is projected into
// tmp first (the partial dot products are then (M x).A(M x) = x.(M A M x)) and
// the output after.
template <typename R>
tt_status matvec_t(tt_ctx& c, const R* x, R* y, double* part, const R* M, const cplx<R>* tw, cplx<R>* T,
                   cplx<R>* U, const R* noise, const R* nxy, R* tmp) {
    const int rows = c.C * c.n;
    if (c.modes) {
        hipLaunchKernelGGL(k_copy_vec<R>, dim3(cdiv(c.n_slopes, 256)), dim3(256), 0, c.stream, x, tmp,
                           (long)c.n_slopes);
        TT_CHECK(mode_project(c, tmp));
        x = tmp;
    }
    hipLaunchKernelGGL(k_row_fwd<R>, dim3(rows), dim3(128), 0, c.stream, x, c.vmap.p, tw, T, c.n, c.C, c.L, c.Lh,
                       c.n_vs);
    TT_HIP(hipGetLastError());
    const size_t lds = col_pass_lds(c, sizeof(cplx<R>));
    hipLaunchKernelGGL(k_col_pass<R>, dim3(c.Lh), dim3(256), lds, c.stream, T, M, tw, U, c.n, c.G, c.L, c.Lh);
    TT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_row_inv<R>, dim3(rows), dim3(128), 0, c.stream, U, tw, c.vmap.p, x, noise, nxy, y, part,
                       c.n, c.C, c.L, c.Lh, c.n_vs);
    TT_HIP(hipGetLastError());
    if (c.modes) TT_CHECK(mode_project(c, y));
    return TT_OK;
}

}  // namespace

tt_status matvec_prepare(tt_ctx& c) {
    // dynamic LDS of the column pass above the default limit
    const size_t l32 = col_pass_lds(c, sizeof(c32)), l64 = col_pass_lds(c, sizeof(c64));
    if (l64 > 160 * 1024) {
        tt_set_error("system too large for the column pass: " + std::to_string(l64) + " bytes of LDS");
        return TT_INVALID_ARG;
    }
    TT_HIP(hipFuncSetAttribute((const void*)k_col_pass<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l32));
    TT_HIP(hipFuncSetAttribute((const void*)k_col_pass<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l64));
    return TT_OK;
}

tt_status matvec_f32(tt_ctx& c, const float* x, float* y, double* part) {
    return matvec_t<float>(c, x, y, part, c.M32.p, c.tw32.p, c.T32.p, c.U32.p, c.noise32.p,
                           c.has_nxy ? c.nxy32.p : nullptr, c.mtmp32.p);
}

// the FP32 product with caller-chosen transform work buffers (tt_matvec_noalloc)
tt_status matvec_f32_into(tt_ctx& c, const float* x, float* y, c32* T, c32* U, float* tmp) {
    return matvec_t<float>(c, x, y, nullptr, c.M32.p, c.tw32.p, T, U, c.noise32.p, c.has_nxy ? c.nxy32.p : nullptr,
                           tmp);
}

tt_status matvec_f64(tt_ctx& c, const double* x, double* y, double* part) {
    return matvec_t<double>(c, x, y, part, c.M64.p, c.tw64.p, c.T64.p, c.U64.p, c.noise64.p,
                            c.has_nxy ? c.nxy64.p : nullptr, c.mtmp64.p);
}

// exported for the projection: forward row pass of float data with another padding
tt_status row_fwd_f32(const float* x, const int* vmap, const c32* tw, c32* T, int n, int C, int L, int n_vs,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_row_fwd<float>, dim3(C * n), dim3(128), 0, s, x, vmap, tw, T, n, C, L, L / 2 + 1, n_vs);
    TT_HIP(hipGetLastError());
    return TT_OK;
}
