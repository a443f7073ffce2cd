// Spectra of the embedded covariance tables, float64 (§2.E: the FFT of
// the unique-element vector is computed offline).
//
// A table t(U, V), U, V in [-off, m-1-off] (U column lag, V row lag), is
// embedded reflected into an L x L array, K[(-V) mod L, (-U) mod L] = t(U, V),
// so that the circular convolution of K with the shuffled input reproduces
// sum_b Theta[a, b] x_b (reading of the garbled shuffle rules of §2.E: the
// two-dimensional circulant embedding with any L >= rows + cols - 1).  Its
// half spectrum, f1 in [0, L), f2 in [0, L/2],
//
//   K~(f1, f2) = sum_{U,V} t(U, V) exp(+2 pi i (f1 V + f2 U) / L),
//
// is computed as a row DFT over U followed by a column DFT over V, with
// twiddles exp(2 pi i m / L), m = (f U) mod L, taken from an exact-index table.
//
// Slope-slope spectra are packed per frequency as the Hermitian
// 2G x 2G matrix of the fused product (§2.E, Sigma_ss zeta equation):
//   sensor g with itself: 3 reals (xx, xy, yy) -- the tables are even, so the
//   spectra are real; sensors g < h: 3 complex (xx, xy = yx, yy); the blocks
//   below the diagonal are the conjugates (Theta^{hg}_{qp}(lag) = Theta^{gh}_{pq}(-lag)).
#include "tt_internal.h"

namespace {

// G[tab][row][f2] = sum_U t[tab][row][U] exp(+2 pi i f2 (U - off) / L)
__global__ void tab_rowdft(const double* __restrict__ t, c64* __restrict__ G, const c64* __restrict__ tw,
                           int m, int off, int L, int Lh) {
    const int row = blockIdx.x % m;
    const long tab = blockIdx.x / m;
    const double* src = t + (tab * m + row) * (long)m;
    for (int f2 = threadIdx.x; f2 < Lh; f2 += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int u = 0; u < m; ++u) {
            int k = (int)(((long)f2 * (u - off)) % L);
            if (k < 0) k += L;
            const c64 w = tw[k];
            re += src[u] * w.x;
            im += src[u] * w.y;
        }
        G[(tab * m + row) * (long)Lh + f2] = c64{re, im};
    }
}

// S[tab][f2][f1] = sum_V G[tab][V][f2] exp(+2 pi i f1 (V - off) / L)
__global__ void tab_coldft(const c64* __restrict__ G, c64* __restrict__ S, const c64* __restrict__ tw,
                           int m, int off, int L, int Lh) {
    const int f2 = blockIdx.x % Lh;
    const long tab = blockIdx.x / Lh;
    for (int f1 = threadIdx.x; f1 < L; f1 += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int v = 0; v < m; ++v) {
            int k = (int)(((long)f1 * (v - off)) % L);
            if (k < 0) k += L;
            const c64 w = tw[k];
            const c64 g = G[(tab * m + v) * (long)Lh + f2];
            re += g.x * w.x - g.y * w.y;
            im += g.x * w.y + g.y * w.x;
        }
        S[(tab * Lh + f2) * (long)L + f1] = c64{re, im};
    }
}

// Pack slope-slope spectra into M[(f2 L + f1) P + slot] (FP64 and FP32 copies).
__global__ void pack_slope(const c64* __restrict__ S, double* __restrict__ M64, float* __restrict__ M32,
                           int G, int L, int Lh) {
    const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;   // f = f2 * L + f1
    if (f >= (long)L * Lh) return;
    const int f2 = (int)(f / L), f1 = (int)(f % L);
    const int P = 3 * G * G;
    int tabpair = 0;
    for (int g = 0; g < G; ++g) {
        for (int h = g; h < G; ++h, ++tabpair) {
            for (int comp = 0; comp < 3; ++comp) {
                const long tab = (long)tabpair * 3 + comp;
                const c64 v = S[(tab * Lh + f2) * (long)L + f1];
                if (g == h) {
                    const int slot = 3 * g + comp;
                    M64[f * P + slot] = v.x;
                    M32[f * P + slot] = (float)v.x;
                } else {
                    const int px = g * (2 * G - g - 1) / 2 + (h - g - 1);
                    const int slot = 3 * G + 6 * px + 2 * comp;
                    M64[f * P + slot] = v.x;
                    M64[f * P + slot + 1] = v.y;
                    M32[f * P + slot] = (float)v.x;
                    M32[f * P + slot + 1] = (float)v.y;
                }
            }
        }
    }
}

}  // namespace

tt_status build_twiddles(int L, DevBuf<c32>& t32, DevBuf<c64>* t64, hipStream_t s) {
    // exp(+2 pi i k / L) stored as (cos, sin); kernels conjugate where needed.
    std::vector<c64> h64(L);
    std::vector<c32> h32(L);
    for (int k = 0; k < L; ++k) {
        // reduce to the first half-turn for a symmetric, exactly periodic table
        const double a = 2.0 * M_PI * (double)k / (double)L;
        h64[k] = c64{std::cos(a), std::sin(a)};
        if (4 * k == L) h64[k] = c64{0.0, 1.0};
        if (2 * k == L) h64[k] = c64{-1.0, 0.0};
        if (4 * k == 3 * L) h64[k] = c64{0.0, -1.0};
        h32[k] = c32{(float)h64[k].x, (float)h64[k].y};
    }
    TT_CHECK(t32.upload(h32.data(), L, s));
    if (t64) TT_CHECK(t64->upload(h64.data(), L, s));
    TT_HIP(hipStreamSynchronize(s));
    return TT_OK;
}

// Generic: spectra of `ntab` tables of side m with lag offset `off` into S (complex, [tab][f2][f1]).
tt_status table_spectra(const double* d_tables, long ntab, int m, int off, int L, DevBuf<c64>& S,
                        hipStream_t s) {
    const int Lh = L / 2 + 1;
    DevBuf<c32> tw32;
    DevBuf<c64> tw64;
    TT_CHECK(build_twiddles(L, tw32, &tw64, s));
    DevBuf<c64> Gb;
    TT_CHECK(Gb.alloc((size_t)ntab * m * Lh));
    TT_CHECK(S.alloc((size_t)ntab * Lh * L));
    hipLaunchKernelGGL(tab_rowdft, dim3((unsigned)(ntab * m)), dim3(128), 0, s, d_tables, Gb.p, tw64.p, m,
                       off, L, Lh);
    TT_HIP(hipGetLastError());
    hipLaunchKernelGGL(tab_coldft, dim3((unsigned)(ntab * Lh)), dim3(256), 0, s, Gb.p, S.p, tw64.p, m, off,
                       L, Lh);
    TT_HIP(hipGetLastError());
    TT_HIP(hipStreamSynchronize(s));
    return TT_OK;
}

tt_status build_slope_spectra(tt_ctx& c, const tt_kernels& k) {
    const int m = 2 * k.n - 1;
    const long ntab = (long)n_pairs_incl(k.n_gs) * 3;
    DevBuf<c64> S;
    TT_CHECK(table_spectra(k.tables.p, ntab, m, k.n - 1, c.L, S, c.stream));
    const size_t nf = (size_t)c.L * c.Lh;
    TT_CHECK(c.M64.alloc(nf * packed_reals(c.G)));
    TT_CHECK(c.M32.alloc(nf * packed_reals(c.G)));
    hipLaunchKernelGGL(pack_slope, dim3(cdiv(nf, 256)), dim3(256), 0, c.stream, S.p, c.M64.p, c.M32.p, c.G, c.L,
                       c.Lh);
    TT_HIP(hipGetLastError());
    TT_HIP(hipStreamSynchronize(c.stream));
    return TT_OK;
}
