// The 2RBT product y = W_s (Sigma_ss + Sigma_eta) W_s^T x (§2.E, with the
// §2.F masks) of many independent systems in one launch per phase: every
// system keeps its own spectra, sizes and work buffers, and one call streams
// the per-frequency spectra of all of them once.  This is the form in which the
// product is bound by HBM bandwidth (the spectra of a few dozen 74x74 systems
// exceed the last-level cache), as opposed to the latency-bound single-system
// product inside the persistent solver.
//
// Phases (the transform conventions of the single-system product):
//   row_fwd : T[f2][c][a] = sum_{b<n} x_c[a][b] w_L^{f2 b},        w_L = exp(-2 pi i / L)
//   col     : column work item (system, f2, h), h < S, owns the frequencies
//             f1 = S k + h, k < m = L / S.  As the input column is zero for
//             a >= n and m >= n,
//               X[S k + h] = sum_{a<n} (T[f2][c][a] w_L^{h a}) w_m^{k a},
//             an m-point DFT of the twisted column: a radix-2 FFT in LDS when m
//             is a power of two, the plain sum otherwise.  Products with the
//             spectra of these m frequencies (Y_p = sum_q M_pq X_q, Hermitian
//             packing), then this item's share of the inverse column transform
//               U_h[f2][p][a] = w_L^{-h a} sum_k Y_p[k] w_m^{-k a},  a < n.
//   row_inv : y_p[a][b] = L^-2 sum_{f2} wt(f2) Re(sum_h U_h[f2][p][a] w_L^{-f2 b}) + noise,
//             restricted to the valid subapertures (S2, W_s).
//
// S = 2 when every L of the batch is even (then L >= 2n gives m >= n), else 1.
// The two items of one column are given workgroup numbers 8 apart, which the
// dispatcher places on the same XCD at nearly the same time, so the column of
// T and the cache lines shared by neighbouring frequencies are read from HBM
// once.  The spectra of an item are prefetched into registers with coalesced
// loads while the forward transform runs, then stored to LDS with a padded
// stride of 3G^2 + 1 floats per frequency (conflict-free reads when the lanes
// of a wave take consecutive frequencies).
#include "tt_internal.h"

#include <algorithm>

namespace {

constexpr int BT = 256;     // threads of a column work item
constexpr int NPF = 64;     // spectra floats prefetched per thread and round
constexpr int TMAX = 8;     // (frequency, sensor) product tasks per thread at most

struct BSys {
    const float* x;
    float* y;
    const int* vmap;
    const c32* tw;     // L twiddles exp(-2 pi i k / L) as (cos, sin)
    c32* T;            // [Lh][C][n]
    c32* U;            // [Lh][S][C][n]
    const float* M;    // [Lh][L][3G^2]
    const float* noise;
    const float* nxy;  // NULL unless the noise has 2x2 blocks
    int n, G, L, n_vs;
    int row0, col0;    // first flat row (C n per system) and column (L/2 + 1 per system)
};

// largest b with start(b) <= idx (starts increase with b)
__device__ inline int find_sys(const BSys* __restrict__ d, int count, int idx, bool by_row) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int st = by_row ? d[mid].row0 : d[mid].col0;
        if (st <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_brow_fwd(const BSys* __restrict__ sys, int count) {
    __shared__ float xs[512];
    __shared__ c32 tws[1024];
    const BSys s = sys[find_sys(sys, count, blockIdx.x, true)];
    const int row = blockIdx.x - s.row0;
    const int n = s.n, L = s.L, Lh = L / 2 + 1, C = 2 * s.G;
    const int c = row / n, a = row % n;
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
        const int v = s.vmap[a * n + b];
        xs[b] = v >= 0 ? s.x[(long)c * s.n_vs + v] : 0.f;
    }
    for (int k = threadIdx.x; k < L; k += blockDim.x) tws[k] = s.tw[k];
    __syncthreads();
    for (int f2 = threadIdx.x; f2 < Lh; f2 += blockDim.x) {
        float re = 0.f, im = 0.f;
        int m = 0;
        for (int b = 0; b < n; ++b) {
            const c32 w = tws[m];
            re += xs[b] * w.x;
            im -= xs[b] * w.y;
            m += f2;
            if (m >= L) m -= L;
        }
        s.T[((long)f2 * C + c) * n + a] = c32{re, im};
    }
}

__device__ inline c32 cmul(c32 a, c32 b) { return c32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline c32 cmulc(c32 a, c32 b) { return c32{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a conj(b)

// Workgroup barrier for LDS traffic only: the spectra loads in flight stay in
// flight (a full __syncthreads would also wait for them).
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// the spectra are read through a global-address-space pointer so that the
// loads are counted apart from LDS traffic
typedef const __attribute__((address_space(1))) float* gfloat_ptr;

__device__ inline int bitrev(int v, int bits) {
    return bits ? (int)(__builtin_bitreverse32((unsigned)v) >> (32 - bits)) : 0;
}

// in-place radix-2 decimation-in-time transform of C arrays of length m
// (input in bit-reversed order, output in natural order); twiddles w_L^{j L/(2hs)}
template <bool INV>
__device__ void fft_inplace(c32* A, const c32* tws, int C, int m, int L) {
    const int half = m >> 1;
    for (int hs = 1; hs < m; hs <<= 1) {
        const int step = L / (2 * hs);
        for (int bf = threadIdx.x; bf < C * half; bf += BT) {
            const int c = bf / half, r = bf - c * half;
            const int grp = r / hs, j = r - grp * hs;
            const int i0 = c * m + grp * 2 * hs + j, i1 = i0 + hs;
            const c32 w = tws[j * step];
            const c32 u = A[i0];
            const c32 v = INV ? cmul(A[i1], w) : cmulc(A[i1], w);
            A[i0] = c32{u.x + v.x, u.y + v.y};
            A[i1] = c32{u.x - v.x, u.y - v.y};
        }
        lds_barrier();
    }
}

__global__ __launch_bounds__(BT) void k_bcol(const BSys* __restrict__ sys, int count, int total_cols, int S) {
    extern __shared__ __align__(16) char smem_raw[];
    // column work item: workgroups 8 apart share an XCD
    const int id = blockIdx.x, xcd = id & 7, slot = id >> 3;
    const int col = (slot / S) * 8 + xcd, h = slot % S;
    if (col >= total_cols) return;
    const BSys s = sys[find_sys(sys, count, col, false)];
    const int f2 = col - s.col0;
    const int n = s.n, G = s.G, C = 2 * G, L = s.L, m = L / S, P = 3 * G * G, Pst = P + 1;
    const bool fft = (m & (m - 1)) == 0;
    int bits = 0;
    while ((1 << bits) < m) ++bits;

    float* Ms = reinterpret_cast<float*>(smem_raw);
    const size_t ms_bytes = (((size_t)m * Pst * sizeof(float)) + 15) & ~size_t(15);
    c32* A = reinterpret_cast<c32*>(smem_raw + ms_bytes);     // C x m
    c32* B = A + (size_t)C * m;                               // C x m (plain-sum transforms only)
    c32* tws = fft ? B : B + (size_t)C * m;                   // L twiddles

    // twisted input column, zero-padded to m (bit-reversed positions for the FFT)
    for (int i = threadIdx.x; i < L; i += BT) tws[i] = s.tw[i];
    __syncthreads();
    const c32* Tc = s.T + (size_t)f2 * C * n;
    for (int idx = threadIdx.x; idx < C * m; idx += BT) {
        const int c = idx / m, a = idx - c * m;
        c32 v = c32{0.f, 0.f};
        if (a < n) {
            v = Tc[c * n + a];
            if (h) v = cmulc(v, tws[(h * a) % L]);
        }
        A[c * m + (fft ? bitrev(a, bits) : a)] = v;
    }
    __syncthreads();

    // spectra of this item: float j < m P is entry w = j mod P of frequency
    // k = j / P, i.e. of row S k + h of the column block: offset j + (S - 1) P k + h P.
    // First round prefetched into registers here, consumed after the forward
    // transform (the loads overlap it); an out-of-range lane reads the last
    // entry of the item and discards it.
    const gfloat_ptr Mcol = (gfloat_ptr)(s.M + (size_t)f2 * L * P);
    const int Q = m * P;
    const int dk = BT / P, dw = BT - dk * P;
    const int k0 = threadIdx.x / P, w0 = threadIdx.x - k0 * P;
    float pf[NPF];
    {
        int k = k0, w = w0;
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            const int j = threadIdx.x + i * BT;
            const int off = j < Q ? (S * k + h) * P + w : (S * (m - 1) + h) * P + P - 1;
            pf[i] = Mcol[off];
            w += dw;
            const int cy = w >= P;
            w -= cy ? P : 0;
            k += dk + cy;
        }
    }

    // forward column transform of the C channels
    c32* X = A;
    if (fft) {
        fft_inplace<false>(A, tws, C, m, L);
    } else {
        for (int idx = threadIdx.x; idx < C * m; idx += BT) {
            const int c = idx / m, k = idx - c * m;
            const c32* in = A + c * m;
            float re = 0.f, im = 0.f;
            int e = 0;
            const int de = (S * k) % L;
            for (int a = 0; a < n; ++a) {
                const c32 t = in[a], w = tws[e];
                re += t.x * w.x + t.y * w.y;
                im += t.y * w.x - t.x * w.y;
                e += de;
                if (e >= L) e -= L;
            }
            B[idx] = c32{re, im};
        }
        X = B;
    }

    // spectra to LDS (first round from the prefetch, then round by round)
    for (int base = 0; base < Q; base += NPF * BT) {
        const int kb = (base + threadIdx.x) / P, wb = (base + threadIdx.x) - kb * P;
        int k = kb, w = wb;
        if (base) {
#pragma unroll
            for (int i = 0; i < NPF; ++i) {
                const int j = base + threadIdx.x + i * BT;
                const int off = j < Q ? (S * k + h) * P + w : (S * (m - 1) + h) * P + P - 1;
                pf[i] = Mcol[off];
                w += dw;
                const int cy = w >= P;
                w -= cy ? P : 0;
                k += dk + cy;
            }
            k = kb;
            w = wb;
        }
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            const int j = base + threadIdx.x + i * BT;
            if (j < Q) Ms[k * Pst + w] = pf[i];
            w += dw;
            const int cy = w >= P;
            w -= cy ? P : 0;
            k += dk + cy;
        }
    }
    __syncthreads();

    // per-frequency products summed over the input channels: task (k, g) gives
    // the x and y outputs of sensor g at frequency k
    c32 yx[TMAX], yy[TMAX];
#pragma unroll
    for (int it = 0; it < TMAX; ++it) {
        const int task = threadIdx.x + it * BT;
        yx[it] = yy[it] = c32{0.f, 0.f};
        if (task < m * G) {
            const int g = task / m, k = task - g * m;
            const float* Mf = Ms + k * Pst;
            c32 ax = c32{0.f, 0.f}, ay = c32{0.f, 0.f};
            for (int hh = 0; hh < G; ++hh) {
                const c32 xh = X[(2 * hh) * m + k], yh = X[(2 * hh + 1) * m + k];
                c32 mxx, mxy, myy;
                if (hh == g) {
                    mxx = c32{Mf[3 * g], 0.f};
                    mxy = c32{Mf[3 * g + 1], 0.f};
                    myy = c32{Mf[3 * g + 2], 0.f};
                } else {
                    const int lo = g < hh ? g : hh, hi = g < hh ? hh : g;
                    const int sl = 3 * G + 6 * (lo * (2 * G - lo - 1) / 2 + (hi - lo - 1));
                    const float sg = g < hh ? 1.f : -1.f;  // M_gh = conj(M_hg) for g > h
                    mxx = c32{Mf[sl], sg * Mf[sl + 1]};
                    mxy = c32{Mf[sl + 2], sg * Mf[sl + 3]};
                    myy = c32{Mf[sl + 4], sg * Mf[sl + 5]};
                }
                const c32 p0 = cmul(mxx, xh), p1 = cmul(mxy, yh), p2 = cmul(mxy, xh), p3 = cmul(myy, yh);
                ax.x += p0.x + p1.x;
                ax.y += p0.y + p1.y;
                ay.x += p2.x + p3.x;
                ay.y += p2.y + p3.y;
            }
            yx[it] = ax;
            yy[it] = ay;
        }
    }
    __syncthreads();
    c32* Y = A;   // the twisted input is no longer needed (FFT: X is A itself, read above)
#pragma unroll
    for (int it = 0; it < TMAX; ++it) {
        const int task = threadIdx.x + it * BT;
        if (task < m * G) {
            const int g = task / m, k = task - g * m;
            const int pos = fft ? bitrev(k, bits) : k;
            Y[(2 * g) * m + pos] = yx[it];
            Y[(2 * g + 1) * m + pos] = yy[it];
        }
    }
    __syncthreads();

    // this item's share of the inverse column transform, rows a < n
    c32* Uo = s.U + ((size_t)f2 * S + h) * C * n;
    if (fft) {
        fft_inplace<true>(Y, tws, C, m, L);
        for (int idx = threadIdx.x; idx < C * n; idx += BT) {
            const int p = idx / n, a = idx - p * n;
            c32 v = Y[p * m + a];
            if (h) v = cmul(v, tws[(h * a) % L]);
            Uo[idx] = v;
        }
    } else {
        for (int idx = threadIdx.x; idx < C * n; idx += BT) {
            const int p = idx / n, a = idx - p * n;
            const c32* yv = Y + p * m;
            float re = 0.f, im = 0.f;
            int e = (h * a) % L;
            const int de = (S * a) % L;
            for (int k = 0; k < m; ++k) {
                const c32 y = yv[k], w = tws[e];
                re += y.x * w.x - y.y * w.y;
                im += y.x * w.y + y.y * w.x;
                e += de;
                if (e >= L) e -= L;
            }
            Uo[idx] = c32{re, im};
        }
    }
}

__global__ void k_brow_inv(const BSys* __restrict__ sys, int count, int S) {
    __shared__ c32 Us[513];
    __shared__ c32 tws[1024];
    const BSys s = sys[find_sys(sys, count, blockIdx.x, true)];
    const int row = blockIdx.x - s.row0;
    const int n = s.n, L = s.L, Lh = L / 2 + 1, C = 2 * s.G;
    const int c = row / n, a = row % n;
    for (int f2 = threadIdx.x; f2 < Lh; f2 += blockDim.x) {
        c32 u = c32{0.f, 0.f};
        for (int h = 0; h < S; ++h) {
            const c32 v = s.U[(((long)f2 * S + h) * C + c) * n + a];
            u.x += v.x;
            u.y += v.y;
        }
        Us[f2] = u;
    }
    for (int k = threadIdx.x; k < L; k += blockDim.x) tws[k] = s.tw[k];
    __syncthreads();
    const float inv = 1.f / ((float)L * (float)L);
    const bool even = (L % 2) == 0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
        const int v = s.vmap[a * n + b];
        if (v < 0) continue;
        float acc = Us[0].x;
        int m = b;
        for (int f2 = 1; f2 < Lh; ++f2) {
            const c32 u = Us[f2], w = tws[m];
            const float wt = (even && 2 * f2 == L) ? 1.f : 2.f;
            acc += wt * (u.x * w.x - u.y * w.y);
            m += b;
            if (m >= L) m -= L;
        }
        const long i = (long)c * s.n_vs + v;
        float out = acc * inv + s.noise[i] * s.x[i];
        if (s.nxy) out += s.nxy[(long)(c >> 1) * s.n_vs + v] * s.x[(long)(c ^ 1) * s.n_vs + v];
        s.y[i] = out;
    }
}

size_t col_lds(int n, int G, int L, int S) {
    const int m = L / S, C = 2 * G, P = 3 * G * G;
    const bool fft = (m & (m - 1)) == 0;
    const size_t ms = (((size_t)m * (P + 1) * sizeof(float)) + 15) & ~size_t(15);
    (void)n;
    return ms + (size_t)C * m * sizeof(c32) * (fft ? 1 : 2) + (size_t)L * sizeof(c32);
}

}  // namespace

// Host side of tt_matvec_batch (see include/tt.h).
tt_status matvec_batch(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y,
                       float* phase_ms) {
    TT_REQUIRE(count >= 0, "count must be >= 0");
    if (count == 0) return TT_OK;
    TT_REQUIRE(systems && d_x && d_y, "NULL argument");
    tt_ctx& c0 = *systems[0];
    for (int i = 0; i < count; ++i) {
        TT_REQUIRE(systems[i] && d_x[i] && d_y[i], "NULL system or vector");
        TT_REQUIRE((const void*)d_x[i] != (const void*)d_y[i], "d_x and d_y must not alias");
        if (!systems[i]->ready) {
            tt_set_error("tt_matvec_batch: no system set on context " + std::to_string(i));
            return TT_NOT_READY;
        }
        TT_REQUIRE(systems[i]->device == c0.device, "all contexts of a batch must be on one device");
        TT_REQUIRE(!systems[i]->modes, "mode removal is not supported in a batch (use tt_matvec)");
    }
    {
        std::vector<const tt_ctx*> sorted(systems, systems + count);
        std::sort(sorted.begin(), sorted.end());
        TT_REQUIRE(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(),
                   "a context appears twice in the batch");
    }
    int S = 2;
    for (int i = 0; i < count; ++i)
        if (systems[i]->L % 2) S = 1;
    size_t lds = 0;
    for (int i = 0; i < count; ++i) {
        const tt_ctx& c = *systems[i];
        TT_REQUIRE((long)(c.L / S) * c.G <= (long)TMAX * BT,
                   "system too large for the batched product: (L / S) * n_gs must be <= " +
                       std::to_string(TMAX * BT));
        lds = std::max(lds, col_lds(c.n, c.G, c.L, S));
    }
    TT_REQUIRE(lds <= 160 * 1024, "system too large for the batched product: " + std::to_string(lds) +
                                      " bytes of LDS per column item");
    TT_HIP(hipSetDevice(c0.device));

    std::vector<BSys> d(count);
    int rows = 0, cols = 0;
    for (int i = 0; i < count; ++i) {
        tt_ctx& c = *systems[i];
        const size_t ucount = (size_t)c.Lh * S * c.C * c.n;
        if (c.bU32.n < ucount) TT_CHECK(c.bU32.alloc(ucount));
        d[i] = BSys{d_x[i], d_y[i], c.vmap.p, c.tw32.p, c.T32.p, c.bU32.p, c.M32.p, c.noise32.p,
                    c.has_nxy ? c.nxy32.p : nullptr, c.n, c.G, c.L, c.n_vs, rows, cols};
        rows += c.C * c.n;
        cols += c.Lh;
    }
    const size_t bytes = sizeof(BSys) * (size_t)count;
    if (c0.bdesc.n < bytes) TT_CHECK(c0.bdesc.alloc(bytes));
    c0.bdesc_host.assign(reinterpret_cast<const unsigned char*>(d.data()),
                         reinterpret_cast<const unsigned char*>(d.data()) + bytes);
    TT_HIP(hipMemcpyAsync(c0.bdesc.p, c0.bdesc_host.data(), bytes, hipMemcpyHostToDevice, c0.stream));
    const BSys* dd = reinterpret_cast<const BSys*>(c0.bdesc.p);

    TT_HIP(hipFuncSetAttribute((const void*)k_bcol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const unsigned col_grid = (unsigned)(cdiv(cols, 8) * 8 * S);
    if (phase_ms && !c0.bev[0])
        for (auto& e : c0.bev) TT_HIP(hipEventCreate(&e));
    if (phase_ms) TT_HIP(hipEventRecord(c0.bev[0], c0.stream));
    hipLaunchKernelGGL(k_brow_fwd, dim3(rows), dim3(128), 0, c0.stream, dd, count);
    TT_HIP(hipGetLastError());
    if (phase_ms) TT_HIP(hipEventRecord(c0.bev[1], c0.stream));
    hipLaunchKernelGGL(k_bcol, dim3(col_grid), dim3(BT), lds, c0.stream, dd, count, cols, S);
    TT_HIP(hipGetLastError());
    if (phase_ms) TT_HIP(hipEventRecord(c0.bev[2], c0.stream));
    hipLaunchKernelGGL(k_brow_inv, dim3(rows), dim3(128), 0, c0.stream, dd, count, S);
    TT_HIP(hipGetLastError());
    if (phase_ms) {
        TT_HIP(hipEventRecord(c0.bev[3], c0.stream));
        TT_HIP(hipEventSynchronize(c0.bev[3]));
        for (int k = 0; k < 3; ++k) TT_HIP(hipEventElapsedTime(&phase_ms[k], c0.bev[k], c0.bev[k + 1]));
    }
    return TT_OK;
}
