// Projection to the target direction:
//
//   phi = W_phi sum_k I'_k S2 F^-1 { sum_q Xi'~_{q,k} . F[S1 zeta_q] }
//
// (§2.E LGS phase-slope equation with a common grid size n'; §2.D new phase
// grids and bilinear interpolation; §2.F W_phi).  One forward transform per
// slope channel at padding L' >= n' + n - 1, per layer the products summed over
// channels, one inverse transform per layer restricted to the n' x n' grid,
// then bilinear interpolation from the layer grid (spacing s_k d, centred on
// the target ray) to the valid phase points, summed over layers.
//
// Readings: n' = ceil(n / min_k s_k) + 1 by default; grids centred on the
// direction; standard bilinear weights, nodes outside a grid contribute zero.
// With natural guide stars (s_k = 1 for every layer) the layer spectra are
// summed at set-up: one inverse transform and one interpolation in all (the
// NGS phase-slope product of §2.E).
#include "tt_internal.h"
#include "vk_math.h"

tt_status table_spectra(const double* d_tables, long ntab, int m, int off, int L, DevBuf<c64>& S, hipStream_t s);
tt_status row_fwd_f32(const float* x, const int* vmap, const c32* tw, c32* T, int n, int C, int L, int n_vs,
                      hipStream_t s);

namespace {

__global__ void k_pack_proj(const c64* __restrict__ S, c32* __restrict__ spec, int ntab, int L, int Lh) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;   // i = f * ntab + tab, f = f2 * L + f1
    if (i >= (long)L * Lh * ntab) return;
    const int tab = (int)(i % ntab);
    const long f = i / ntab;
    const int f2 = (int)(f / L), f1 = (int)(f % L);
    const c64 v = S[((long)tab * Lh + f2) * L + f1];
    spec[i] = c32{(float)v.x, (float)v.y};
}

// Natural guide stars: every layer uses the same grid and interpolation, so the
// per-layer spectra are summed over layers (the NGS phase-slope product of
// §2.E: one inverse transform instead of one per layer).
__global__ void k_pack_proj_sum(const c64* __restrict__ S, c32* __restrict__ spec, int K, int C, int L, int Lh) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;   // i = f * C + q, f = f2 * L + f1
    if (i >= (long)L * Lh * C) return;
    const int q = (int)(i % C);
    const long f = i / C;
    const int f2 = (int)(f / L), f1 = (int)(f % L);
    double re = 0.0, im = 0.0;
    for (int k = 0; k < K; ++k) {
        const c64 v = S[(((long)k * C + q) * Lh + f2) * L + f1];
        re += v.x;
        im += v.y;
    }
    spec[i] = c32{(float)re, (float)im};
}

__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// per f2 column: forward column DFT of the C channels, per-layer products, inverse to n' rows
__global__ void k_proj_col(const c32* __restrict__ T, const c32* __restrict__ spec, const c32* __restrict__ tw,
                           c32* __restrict__ W, int n, int C, int K, int np, int L, int Lh) {
    extern __shared__ char smem_raw[];
    c32* tws = reinterpret_cast<c32*>(smem_raw);
    c32* Tc = tws + L;
    c32* Xh = Tc + C * n;
    c32* Ph = Xh + C * L;
    const int f2 = blockIdx.x;
    for (int k = threadIdx.x; k < L; k += blockDim.x) tws[k] = tw[k];
    for (int k = threadIdx.x; k < C * n; k += blockDim.x) Tc[k] = T[(long)f2 * C * n + k];
    __syncthreads();
    for (int idx = threadIdx.x; idx < C * L; idx += blockDim.x) {
        const int c = idx / L, f1 = idx % L;
        float re = 0, im = 0;
        int m = 0;
        for (int a = 0; a < n; ++a) {
            const c32 t = Tc[c * n + a];
            const c32 w = tws[m];
            re += t.x * w.x + t.y * w.y;
            im += t.y * w.x - t.x * w.y;
            m += f1;
            if (m >= L) m -= L;
        }
        Xh[idx] = c32{re, im};
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < K * L; idx += blockDim.x) {
        const int k = idx / L, f1 = idx % L;
        const c32* sp = spec + (((long)f2 * L + f1) * K + k) * C;
        float re = 0, im = 0;
        for (int q = 0; q < C; ++q) {
            const c32 s = sp[q];
            const c32 x = Xh[q * L + f1];
            re += s.x * x.x - s.y * x.y;
            im += s.x * x.y + s.y * x.x;
        }
        Ph[idx] = c32{re, im};
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < K * np; idx += blockDim.x) {
        const int k = idx / np, a = idx % np;
        float re = 0, im = 0;
        int m = 0;
        for (int f1 = 0; f1 < L; ++f1) {
            const c32 y = Ph[k * L + f1];
            const c32 w = tws[m];
            re += y.x * w.x - y.y * w.y;
            im += y.x * w.y + y.y * w.x;
            m += a;
            if (m >= L) m -= L;
        }
        W[((long)f2 * K + k) * np + a] = c32{re, im};
    }
}

// inverse row transform of every layer, n' x n' outputs
__global__ void k_proj_row_inv(const c32* __restrict__ W, const c32* __restrict__ tw, float* __restrict__ out,
                               int K, int np, int L, int Lh) {
    __shared__ c32 Ws[513];
    __shared__ c32 tws[1024];
    const int row = blockIdx.x;   // k * np + i'
    const int k = row / np, a = row % np;
    for (int f2 = threadIdx.x; f2 < Lh; f2 += blockDim.x) Ws[f2] = W[((long)f2 * K + k) * np + a];
    for (int i = threadIdx.x; i < L; i += blockDim.x) tws[i] = tw[i];
    __syncthreads();
    const float inv = 1.0f / ((float)L * (float)L);
    const bool even = (L % 2) == 0;
    for (int b = threadIdx.x; b < np; b += blockDim.x) {
        float s = Ws[0].x;
        int m = b;
        for (int f2 = 1; f2 < Lh; ++f2) {
            const c32 u = Ws[f2];
            const c32 w = tws[m];
            const float wt = (even && 2 * f2 == L) ? 1.0f : 2.0f;
            s += wt * (u.x * w.x - u.y * w.y);
            m += b;
            if (m >= L) m -= L;
        }
        out[(long)row * np + b] = s * inv;
    }
}

// bilinear interpolation to the valid phase points, summed over layers
__global__ void k_interp(const float* __restrict__ layer, const int* __restrict__ vphi, const double* __restrict__ sk,
                         float* __restrict__ phi, int n_vphi, int n, int np, int K, double d) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_vphi) return;
    const int flat = vphi[m];
    const int i = flat / (n + 1), j = flat % (n + 1);
    const double rx = (j - 0.5 * n) * d, ry = (i - 0.5 * n) * d;
    const double c = 0.5 * (np - 1);
    double acc = 0.0;
    for (int k = 0; k < K; ++k) {
        const double fx = rx / (sk[k] * d) + c, fy = ry / (sk[k] * d) + c;
        const int j0 = (int)floor(fx), i0 = (int)floor(fy);
        const double tx = fx - j0, ty = fy - i0;
        const float* g = layer + (long)k * np * np;
        const double wts[4] = {(1 - tx) * (1 - ty), tx * (1 - ty), (1 - tx) * ty, tx * ty};
        const int di[4] = {0, 0, 1, 1}, dj[4] = {0, 1, 0, 1};
        for (int t = 0; t < 4; ++t) {
            const int ii = i0 + di[t], jj = j0 + dj[t];
            if (ii >= 0 && ii < np && jj >= 0 && jj < np && wts[t] != 0.0) acc += wts[t] * (double)g[ii * np + jj];
        }
    }
    phi[m] = (float)acc;
}

size_t proj_col_lds(int L, int C, int n, int K) {
    return sizeof(c32) * ((size_t)L + (size_t)C * n + (size_t)C * L + (size_t)K * L);
}

}  // namespace

tt_status projection_setup(tt_ctx& c, const tt_target* t) {
    Projection& P = c.proj;
    P.on = false;
    TT_REQUIRE(std::isfinite(t->beta_x) && std::isfinite(t->beta_y), "non-finite target direction");
    double smin = 1.0;
    std::vector<double> sk(c.n_layer, 1.0);
    // natural guide stars: all layers share one grid; their spectra are summed
    const bool ngs_sum = !c.lgs;
    if (c.lgs)
        for (int k = 0; k < c.n_layer; ++k) {
            sk[k] = 1.0 - c.h[k] / c.h_lgs;
            smin = std::min(smin, sk[k]);
        }
    int np = t->n_prime;
    if (np <= 0) np = (int)std::ceil(c.n / smin - 1e-12) + 1;
    TT_REQUIRE(np >= 2 && np <= 1024, "n_prime out of range");
    int L = t->pad_L;
    if (L <= 0) {
        L = np + c.n - 1;
        L += L & 1;
    }
    TT_REQUIRE(L >= np + c.n - 1 && L <= 1024, "projection pad_L must be in [n'+n-1, 1024]");
    TT_REQUIRE(L / 2 + 1 <= 513 && c.n <= 512, "projection too large");
    const size_t lds = proj_col_lds(L, c.C, c.n, ngs_sum ? 1 : c.n_layer);
    if (lds > 160 * 1024) {
        tt_set_error("projection needs " + std::to_string(lds) + " bytes of LDS per column (> 160 KiB)");
        return TT_INVALID_ARG;
    }
    P.beta_x = t->beta_x;
    P.beta_y = t->beta_y;
    P.np = np;
    P.Lp = L;
    P.Lph = L / 2 + 1;
    P.n_layer = ngs_sum ? 1 : c.n_layer;
    const int K = c.n_layer, C = c.C;
    const int m = np + c.n - 1;
    // phase-slope tables (FP64) and their spectra
    DevBuf<double> tab;
    TT_CHECK(tab.alloc((size_t)K * C * m * m));
    TT_CHECK(gen_phase_tables_launch(c, np, tab.p, c.stream));
    DevBuf<c64> S;
    TT_CHECK(table_spectra(tab.p, (long)K * C, m, np - 1, L, S, c.stream));
    tab.release();
    const long nspec = (long)L * P.Lph * P.n_layer * C;
    TT_CHECK(P.spec.alloc(nspec));
    if (ngs_sum)
        hipLaunchKernelGGL(k_pack_proj_sum, dim3(cdiv(nspec, 256)), dim3(256), 0, c.stream, S.p, P.spec.p, K, C, L,
                           P.Lph);
    else
        hipLaunchKernelGGL(k_pack_proj, dim3(cdiv(nspec, 256)), dim3(256), 0, c.stream, S.p, P.spec.p, K * C, L,
                           P.Lph);
    TT_HIP(hipGetLastError());
    TT_HIP(hipStreamSynchronize(c.stream));
    S.release();
    // valid phase points: corners of valid subapertures
    std::vector<int> vphi;
    const int n = c.n;
    for (int i = 0; i <= n; ++i)
        for (int j = 0; j <= n; ++j) {
            bool ok = false;
            for (int di = -1; di <= 0 && !ok; ++di)
                for (int dj = -1; dj <= 0 && !ok; ++dj) {
                    const int a = i + di, b = j + dj;
                    if (a >= 0 && a < n && b >= 0 && b < n && c.valid[a * n + b]) ok = true;
                }
            if (ok) vphi.push_back(i * (n + 1) + j);
        }
    P.n_vphi = (int)vphi.size();
    TT_CHECK(P.vphi.upload(vphi.data(), vphi.size(), c.stream));
    TT_CHECK(c.proj.T.alloc((size_t)P.Lph * C * n));
    TT_CHECK(c.proj.Xw.alloc((size_t)P.Lph * P.n_layer * np));
    TT_CHECK(c.proj.layer_out.alloc((size_t)P.n_layer * np * np));
    TT_CHECK(build_twiddles(L, P.twp, nullptr, c.stream));
    if (ngs_sum) sk.assign(1, 1.0);
    TT_CHECK(P.sk.upload(sk.data(), sk.size(), c.stream));
    TT_CHECK(P.z32.alloc(c.n_slopes));
    TT_HIP(hipFuncSetAttribute((const void*)k_proj_col, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    TT_HIP(hipStreamSynchronize(c.stream));
    P.on = true;
    return TT_OK;
}

tt_status projection_apply(tt_ctx& c, const double* zeta, float* phi) {
    Projection& P = c.proj;
    const int K = P.n_layer, C = c.C, n = c.n;
    hipLaunchKernelGGL(k_d2f, dim3(cdiv(c.n_slopes, 256)), dim3(256), 0, c.stream, zeta, P.z32.p,
                       (long)c.n_slopes);
    TT_HIP(hipGetLastError());
    if (c.modes) TT_CHECK(modes_project_f32(c, P.z32.p));   // zeta_MW = M_s zeta_W (§2.F)
    TT_CHECK(row_fwd_f32(P.z32.p, c.vmap.p, P.twp.p, P.T.p, n, C, P.Lp, c.n_vs, c.stream));
    const size_t lds = proj_col_lds(P.Lp, C, n, K);
    hipLaunchKernelGGL(k_proj_col, dim3(P.Lph), dim3(256), lds, c.stream, P.T.p, P.spec.p, P.twp.p, P.Xw.p, n, C, K,
                       P.np, P.Lp, P.Lph);
    TT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_proj_row_inv, dim3(K * P.np), dim3(128), 0, c.stream, P.Xw.p, P.twp.p, P.layer_out.p, K,
                       P.np, P.Lp, P.Lph);
    TT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_interp, dim3(cdiv(P.n_vphi, 128)), dim3(128), 0, c.stream, P.layer_out.p, P.vphi.p,
                       P.sk.p, phi, P.n_vphi, n, P.np, K, c.d);
    TT_HIP(hipGetLastError());
    if (c.modes) TT_CHECK(modes_project_phase(c, phi));      // M_phi (§2.F)
    return TT_OK;
}
