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
//             a >= n and w_m^{k a} depends on a mod m only,
//               X[S k + h] = sum_{a<n} (T[f2][c][a] w_L^{h a}) w_m^{k (a mod m)},
//             an m-point DFT of the twisted column: an FFT in LDS when m is a
//             power of two (radix-2 decimation in frequency, output in
//             bit-reversed order), the plain sum otherwise.  Products with the
//             spectra of these m frequencies (Y_p = sum_q M_pq X_q, Hermitian
//             packing), then this item's share of the inverse column transform
//               U_h[f2][p][a] = w_L^{-h a} sum_k Y_p[k] w_m^{-k a},  a < n.
//   row_inv : y_p[a][b] = L^-2 sum_{f2} wt(f2) Re(sum_h U_h[f2][p][a] w_L^{-f2 b}) + noise,
//             restricted to the valid subapertures (S2, W_s).
//
// S = 2 when every L of the batch is even (then L >= 2n gives m >= n), else 1;
// the preconditioner (C^2 reals per frequency, twice the LDS) takes S = 4 when
// every L is a multiple of 4: then m = L / 4 may be below n (never below n / 2)
// and the column is folded, entry a going to a mod m with the same twist, and
// the inverse share of row a is read at a mod m.
// The two items of one column get item numbers 8 apart, which land on the same
// XCD at nearly the same time, so the column of T and the cache lines shared
// by neighbouring frequencies are read from HBM once.  Column workgroups are
// persistent over their items: the spectra and input column of the next item
// load into registers (coalesced) during the current item's products and
// inverse transform, and are stored to LDS with a padded stride of 3G^2 + 1
// floats per frequency (conflict-free reads when the lanes of a wave take
// consecutive frequencies).  The row phases are FFTs of length L as well when
// L is a power of two.
#include "tt_internal.h"

#include <algorithm>
#include <cstring>
#include <type_traits>

namespace {

constexpr int BT = 512;     // threads of a column work item (two items per CU, four waves per SIMD)
constexpr int NPF = 8;      // spectra vectors (VEC floats each) prefetched per thread and round
constexpr int TMAX = 4;     // (frequency, sensor) product tasks per thread at most
constexpr int TPF = 2;      // entries of the input column prefetched per thread

struct BSys {
    const float* x;
    float* y;
    const int* vmap;
    const c32* tw;     // L twiddles exp(-2 pi i k / L) as (cos, sin)
    c32* T;            // [Lh][C][n]
    c32* U;            // [Lh][S][C][n]
    const float* M;    // [Lh][L][3G^2]
    const unsigned short* Mh;   // the same in FP16 / BF16 (half-precision storage), or null
    const float* Mhs;           // [Lh][L] factor restoring each frequency's FP16 values (1 for BF16)
    const float* Mt;            // power-of-two L: M slot-major, [Lh][P][L], frequencies bit-reversed (k_bcolt)
    const unsigned short* Mht;  // the same for Mh
    const float* Mhst;          // and for Mhs, [Lh][L] bit-reversed
    const float* noise;
    const float* nxy;  // NULL unless the noise has 2x2 blocks
    int n, G, L, n_vs;
    int col0;          // first flat column of this system (L/2 + 1 columns per system)
};

__device__ inline c32 cmul(c32 a, c32 b) { return c32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline c32 cmulc(c32 a, c32 b) { return c32{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a conj(b)

// Workgroup barrier for LDS traffic only: the spectra loads in flight stay in
// flight (a full __syncthreads would also wait for them).
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }


// Global memory through global-address-space pointers: loads and stores are
// then counted apart from LDS traffic (a generic access would make every LDS
// wait also wait for it).
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ inline c32 gload(const c32* p) {
    const f2v t = *(const __attribute__((address_space(1))) f2v*)p;
    return c32{t.x, t.y};
}
__device__ inline void gstore(c32* p, c32 v) { *(__attribute__((address_space(1))) f2v*)p = f2v{v.x, v.y}; }

__device__ inline int bitrev(int v, int bits) {
    return bits ? (int)(__builtin_bitreverse32((unsigned)v) >> (32 - bits)) : 0;
}

__device__ inline c32 cadd(c32 a, c32 b) { return c32{a.x + b.x, a.y + b.y}; }
__device__ inline c32 csub(c32 a, c32 b) { return c32{a.x - b.x, a.y - b.y}; }
__device__ inline c32 mul_mi(c32 a) { return c32{a.y, -a.x}; }   // a (-i)
__device__ inline c32 mul_pi(c32 a) { return c32{-a.y, a.x}; }   // a (+i)

// Forward transform of C arrays of length m = 2^bits in place: radix-2
// decimation in frequency, natural-order input, bit-reversed output.  Two
// stages per pass (half spans H and H/2 on the four entries j, j + H/2, j + H,
// j + 3H/2 of a block of 2H), a last single stage when bits is odd.  Entries at
// or beyond nin are zero and are not read (first pass only).
// LDS index of entry i of an FFT buffer: with PAD one element of padding
// follows every 16, which spreads the strided accesses of the short-span
// passes over the banks
template <bool PAD>
__device__ __forceinline__ int pidx(int i) { return PAD ? i + (i >> 4) : i; }

struct NoHook {
    __device__ void operator()() const {}
};

// hook() runs after every pass (the column kernel issues direct loads there)
template <int NT, bool PAD, typename Hook = NoHook>
__device__ void fft_dif(c32* A, const c32* tws, int C, int bits, int L, int nin, Hook hook = Hook()) {
    const int m = 1 << bits;
    int H = m >> 1, lH = bits - 1;
    bool first = true;
    while (H >= 2) {
        const int q = H >> 1, lq = lH - 1;
        const int nb = C << (bits - 2);
        const int step = L >> (lH + 1);                 // w_{2H}^j = conj(tws[j step])
        for (int b = threadIdx.x; b < nb; b += NT) {
            const int c = b >> (bits - 2), r = b & ((m >> 2) - 1);
            const int j = r & (q - 1);
            const int p0 = ((r >> lq) << (lH + 1)) + j;
            const int i0 = pidx<PAD>((c << bits) + p0), i1 = pidx<PAD>((c << bits) + p0 + q);
            const int i2 = pidx<PAD>((c << bits) + p0 + H), i3 = pidx<PAD>((c << bits) + p0 + H + q);
            const c32 z = c32{0.f, 0.f};
            const c32 x0 = (!first || p0 < nin) ? A[i0] : z;
            const c32 x1 = (!first || p0 + q < nin) ? A[i1] : z;
            const c32 x2 = (!first || p0 + H < nin) ? A[i2] : z;
            const c32 x3 = (!first || p0 + H + q < nin) ? A[i3] : z;
            const c32 w1 = tws[j * step], w2 = tws[2 * j * step];
            const c32 t0 = cadd(x0, x2), t2 = cmulc(csub(x0, x2), w1);
            const c32 t1 = cadd(x1, x3), t3 = mul_mi(cmulc(csub(x1, x3), w1));
            A[i0] = cadd(t0, t1);
            A[i1] = cmulc(csub(t0, t1), w2);
            A[i2] = cadd(t2, t3);
            A[i3] = cmulc(csub(t2, t3), w2);
        }
        lds_barrier();
        hook();
        H >>= 2;
        lH -= 2;
        first = false;
    }
    if (H == 1) {
        for (int b = threadIdx.x; b < (C << (bits - 1)); b += NT) {
            const int i0 = 2 * b, p = i0 & (m - 1);
            const int j0 = pidx<PAD>(i0), j1 = pidx<PAD>(i0 + 1);
            const c32 z = c32{0.f, 0.f};
            const c32 u = (!first || p < nin) ? A[j0] : z;
            const c32 v = (!first || p + 1 < nin) ? A[j1] : z;
            A[j0] = cadd(u, v);
            A[j1] = csub(u, v);
        }
        lds_barrier();
        hook();
    }
}

// Inverse transform (unnormalised, exponent +) of C arrays of length m = 2^bits
// in place: radix-2 decimation in time, bit-reversed input, natural output; a
// first single stage when bits is odd, then two stages per pass (half spans h
// and 2h on the entries j, j + h, j + 2h, j + 3h of a block of 4h).
template <int NT, bool PAD, typename Hook = NoHook>
__device__ void fft_dit_inv(c32* A, const c32* tws, int C, int bits, int L, Hook hook = Hook()) {
    const int m = 1 << bits;
    int h = 1, lh = 0;
    if (bits & 1) {
        for (int b = threadIdx.x; b < (C << (bits - 1)); b += NT) {
            const int j0 = pidx<PAD>(2 * b), j1 = pidx<PAD>(2 * b + 1);
            const c32 u = A[j0], v = A[j1];
            A[j0] = cadd(u, v);
            A[j1] = csub(u, v);
        }
        lds_barrier();
        hook();
        h = 2;
        lh = 1;
    }
    while (h < m) {
        const int nb = C << (bits - 2);
        const int sa = L >> (lh + 1), sb = L >> (lh + 2);   // w_{2h}^j = tws[j sa], w_{4h}^j = tws[j sb]
        for (int b = threadIdx.x; b < nb; b += NT) {
            const int c = b >> (bits - 2), r = b & ((m >> 2) - 1);
            const int j = r & (h - 1);
            const int p0 = ((r >> lh) << (lh + 2)) + j;
            const int i0 = pidx<PAD>((c << bits) + p0), i1 = pidx<PAD>((c << bits) + p0 + h);
            const int i2 = pidx<PAD>((c << bits) + p0 + 2 * h), i3 = pidx<PAD>((c << bits) + p0 + 3 * h);
            const c32 wa = tws[j * sa], wb = tws[j * sb];
            const c32 x0 = A[i0], x1 = cmul(A[i1], wa), x2 = A[i2], x3 = cmul(A[i3], wa);
            const c32 t0 = cadd(x0, x1), t1 = csub(x0, x1), t2 = cadd(x2, x3), t3 = csub(x2, x3);
            const c32 u2 = cmul(t2, wb), u3 = mul_pi(cmul(t3, wb));
            A[i0] = cadd(t0, u2);
            A[i1] = cadd(t1, u3);
            A[i2] = csub(t0, u2);
            A[i3] = csub(t1, u3);
        }
        lds_barrier();
        hook();
        h <<= 2;
        lh += 2;
    }
}

// spectra of item (f2, h) of a system, in vectors of VEC floats (VEC = 4 when
// P = 3 G^2 is a multiple of 4, else 1): vector j < m P / VEC is vector
// w = j mod (P / VEC) of frequency k = j / (P / VEC), i.e. of row S k + h of the
// column block.  One round covers NPF vectors per thread.
template <int VEC> struct vecf;
template <> struct vecf<1> { typedef float t; };
template <> struct vecf<4> { typedef float t __attribute__((ext_vector_type(4))); };
template <int VEC>
using gvec_ptr = const __attribute__((address_space(1))) typename vecf<VEC>::t*;

// An empty use of a loaded value on every path: the wait for its load is then
// placed here, by count, whether or not the value is used afterwards (a value
// used under a branch only leaves its load pending on the other path, and a
// later reuse of its registers would then wait for every memory operation).
template <typename T>
__device__ __forceinline__ void keep(const T& v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void keep(const c32& v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }

template <int VEC>
__device__ __forceinline__ void spectra_load(typename vecf<VEC>::t (&pf)[NPF], const float* Mcol, int base, int Q,
                                             int P, int S, int h) {
    const int Pv = P / VEC;
    const int dk = BT / Pv, dw = BT - dk * Pv;
    int k = (base + (int)threadIdx.x) / Pv, w = (base + (int)threadIdx.x) - k * Pv;
    const gvec_ptr<VEC> g = (gvec_ptr<VEC>)Mcol;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
        // unconditional (an in-range vector past the end of the round): no branch
        // between the loads, so the waits on them count exactly
        const bool ok = base + (int)threadIdx.x + i * BT < Q;
        pf[i] = g[ok ? (S * k + h) * Pv + w : h * Pv];
        w += dw;
        const int cy = w >= Pv;
        w -= cy ? Pv : 0;
        k += dk + cy;
    }
}

// the same round into LDS, frequency k at row k (P + 1) floats (padded stride),
// or at row bitrev(k) when rbits >= 0 (the order of the forward FFT's output)
template <int VEC>
__device__ __forceinline__ void spectra_store(const typename vecf<VEC>::t (&pf)[NPF], float* Ms, int base, int Q,
                                              int P, int rbits) {
    const int Pv = P / VEC;
    const int dk = BT / Pv, dw = BT - dk * Pv;
    int k = (base + (int)threadIdx.x) / Pv, w = (base + (int)threadIdx.x) - k * Pv;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
        keep(pf[i]);
        if (base + (int)threadIdx.x + i * BT < Q) {
            float* d = Ms + (rbits >= 0 ? bitrev(k, rbits) : k) * (P + 1) + w * VEC;
            if constexpr (VEC == 4) {
                d[0] = pf[i].x;
                d[1] = pf[i].y;
                d[2] = pf[i].z;
                d[3] = pf[i].w;
            } else {
                d[0] = pf[i];
            }
        }
        w += dw;
        const int cy = w >= Pv;
        w -= cy ? Pv : 0;
        k += dk + cy;
    }
}

// Half-precision spectra (HALF = 1: FP16 scaled per frequency, 2: BF16): the
// raw 16-bit values of a round are kept in registers with the factor of their
// frequency and decoded when stored to LDS (FP32 from there on).
template <int VEC> struct vech;
template <> struct vech<1> { typedef unsigned short t; };
typedef unsigned u2v __attribute__((ext_vector_type(2)));
template <> struct vech<4> { typedef u2v t; };
template <int VEC>
using ghvec_ptr = const __attribute__((address_space(1))) typename vech<VEC>::t*;

template <int VEC>
__device__ __forceinline__ void spectra_load_h(typename vech<VEC>::t (&pf)[NPF], float (&pfs)[NPF],
                                               const unsigned short* Mcol, const float* scol, int base, int Q, int P,
                                               int S, int h) {
    const int Pv = P / VEC;
    const int dk = BT / Pv, dw = BT - dk * Pv;
    int k = (base + (int)threadIdx.x) / Pv, w = (base + (int)threadIdx.x) - k * Pv;
    const ghvec_ptr<VEC> g = (ghvec_ptr<VEC>)Mcol;
    const __attribute__((address_space(1))) float* gs = (const __attribute__((address_space(1))) float*)scol;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
        const bool ok = base + (int)threadIdx.x + i * BT < Q;
        pf[i] = g[ok ? (S * k + h) * Pv + w : h * Pv];
        pfs[i] = gs[ok ? S * k + h : h];
        w += dw;
        const int cy = w >= Pv;
        w -= cy ? Pv : 0;
        k += dk + cy;
    }
}

template <int HALF>
__device__ __forceinline__ float half_dec(unsigned short b) {
    if constexpr (HALF == 1) return (float)__builtin_bit_cast(_Float16, b);
    else return __uint_as_float((unsigned)b << 16);
}

template <int VEC, int HALF>
__device__ __forceinline__ void spectra_store_h(const typename vech<VEC>::t (&pf)[NPF], const float (&pfs)[NPF],
                                                float* Ms, int base, int Q, int P, int rbits) {
    const int Pv = P / VEC;
    const int dk = BT / Pv, dw = BT - dk * Pv;
    int k = (base + (int)threadIdx.x) / Pv, w = (base + (int)threadIdx.x) - k * Pv;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
        keep(pf[i]);
        keep(pfs[i]);
        if (base + (int)threadIdx.x + i * BT < Q) {
            float* d = Ms + (rbits >= 0 ? bitrev(k, rbits) : k) * (P + 1) + w * VEC;
            const float sc = pfs[i];
            if constexpr (VEC == 4) {
                d[0] = half_dec<HALF>((unsigned short)(pf[i].x & 0xffffu)) * sc;
                d[1] = half_dec<HALF>((unsigned short)(pf[i].x >> 16)) * sc;
                d[2] = half_dec<HALF>((unsigned short)(pf[i].y & 0xffffu)) * sc;
                d[3] = half_dec<HALF>((unsigned short)(pf[i].y >> 16)) * sc;
            } else {
                d[0] = half_dec<HALF>(pf[i]) * sc;
            }
        }
        w += dw;
        const int cy = w >= Pv;
        w -= cy ? Pv : 0;
        k += dk + cy;
    }
}

// (row, column) of the flat index threadIdx.x + i BT of a rows x len array,
// advanced without division
struct Walk {
    int r, c, dr, dc, len;
    __device__ Walk(int len_) : len(len_) {
        r = (int)threadIdx.x / len_;
        c = (int)threadIdx.x - r * len_;
        dr = BT / len_;
        dc = BT - dr * len_;
    }
    __device__ void next() {
        c += dc;
        const int cy = c >= len;
        c -= cy ? len : 0;
        r += dr + cy;
    }
};

// w_16^j, j < 8 (exponent -): (cos, -sin) of j pi / 8
__device__ __forceinline__ c32 w16(int j) {
    constexpr float C1 = 0.92387953251128674f, S1 = 0.38268343236508977f, R = 0.70710678118654752f;
    switch (j) {
        case 0: return c32{1.f, 0.f};
        case 1: return c32{C1, -S1};
        case 2: return c32{R, -R};
        case 3: return c32{S1, -C1};
        case 4: return c32{0.f, -1.f};
        case 5: return c32{-S1, -C1};
        case 6: return c32{-R, -R};
        default: return c32{-C1, -S1};
    }
}

// orders the LDS accesses of the lanes of one wave (the hardware keeps a
// wave's LDS operations in order; this keeps the compiler from moving them)
__device__ __forceinline__ void wave_lds_order() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// w_16^j, j < 16
__device__ __forceinline__ c32 w16f(int j) {
    const c32 w = w16(j & 7);
    return (j & 8) ? c32{-w.x, -w.y} : w;
}

template <bool INV>
__device__ __forceinline__ void dft4(c32& a0, c32& a1, c32& a2, c32& a3) {
    const c32 s02 = cadd(a0, a2), d02 = csub(a0, a2), s13 = cadd(a1, a3), d13 = csub(a1, a3);
    const c32 r = INV ? mul_pi(d13) : mul_mi(d13);
    a0 = cadd(s02, s13);
    a1 = cadd(d02, r);
    a2 = csub(s02, s13);
    a3 = csub(d02, r);
}

// 16-point DFT in registers, natural order in and out (n = 4 n1 + n2,
// k = k1 + 4 k2: 4-point DFTs over n1, twiddles w_16^{n2 k1}, 4-point DFTs
// over n2); INV: exponent +
template <bool INV>
__device__ __forceinline__ void dft16(c32 (&a)[16]) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);   // slot 4 k1 + n2
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) {
            const c32 w = w16f(n2 * k1);
            a[4 * k1 + n2] = INV ? cmulc(a[4 * k1 + n2], w) : cmul(a[4 * k1 + n2], w);
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);   // slot 4 k1 + k2
    c32 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = t[i];
}

// 256-point DFT of one row by the 16 lanes q of a group of one wave: the row
// at R in the padded layout pidx (entry i at i + i / 16), natural order in and
// out; n = 16 n1 + q, k = k1 + 16 k2: 16-point DFTs over n1 in registers,
// twiddles w_256^{q k1} (tws: the 256 twiddles of exp(+2 pi i k / 256)), a
// transpose through R, 16-point DFTs over q.  INV: exponent +.
template <bool INV>
__device__ __forceinline__ void fft256_group(c32* R, const c32* tws, int q) {
    c32 a[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) a[n1] = R[17 * n1 + q];   // pidx(16 n1 + q)
    dft16<INV>(a);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) a[k1] = INV ? cmul(a[k1], tws[q * k1]) : cmulc(a[k1], tws[q * k1]);
    wave_lds_order();
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) R[17 * k1 + q] = a[k1];   // C_q[k1] at pidx(16 k1 + q)
    wave_lds_order();
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = R[17 * q + j];   // lane q as k1: C_j[q]
    dft16<INV>(a);
    wave_lds_order();
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) R[q + 17 * k2] = a[k2];   // Z[q + 16 k2] at pidx(q + 16 k2)
}

constexpr int RS256 = 272;   // row stride of the L = 256 row transforms (pidx(255) = 270)

// Row phases: grid (row tile, system).  A workgroup takes consecutive rows a
// of one channel c, so that for every f2 its entries of T and U are contiguous
// in memory; tiles beyond a system's channels exit.  When L is a power of two
// the row transforms are FFTs of length L (the passes of the column phase; the
// forward one reads only the n nonzero inputs, the inverse one takes the half
// spectrum weighted by 1 or 2 and keeps the real part), else plain sums.
constexpr int RBT = 256;
constexpr int RLDS = 33792;   // bytes of row data per workgroup

__host__ __device__ inline bool is_pow2(int v) { return (v & (v - 1)) == 0; }
__host__ __device__ inline int row_tile_fwd(int L) { return is_pow2(L) ? (RLDS / 8 / L < 16 ? RLDS / 8 / L : 16) : 16; }
__host__ __device__ inline int row_tile_inv(int L) { return is_pow2(L) ? (RLDS / 8 / L < 16 ? RLDS / 8 / L : 16) : 8; }

// L = 256: a workgroup takes 16 consecutive rows a of one channel c, each row
// transformed by 16 lanes of one wave (fft256_group: no workgroup barrier
// inside the transform).  Each real row is transformed on its own (a complex
// transform with zero imaginary part): packing two channels into the real and
// imaginary parts of one transform would halve the work but leaks each
// channel's rounding into the other (errors of order u |X_other|, not
// u |X_own|), which stalls CG on the least damped systems.
static_assert(16 * RS256 * sizeof(c32) + 256 * sizeof(c32) <= RLDS + 1024 * sizeof(c32), "row LDS");

__global__ __launch_bounds__(RBT) void k_brow_fwd(const BSys* __restrict__ sys) {
    __shared__ __align__(16) char lds[RLDS + 1024 * sizeof(c32)];
    c32* tws = reinterpret_cast<c32*>(lds + RLDS);
    const BSys s = sys[blockIdx.y];
    const int n = s.n, L = s.L, Lh = L / 2 + 1, C = 2 * s.G;
    if (L == 256) {
        const int tiles16 = (n + 15) / 16, c = blockIdx.x / tiles16, a0 = (blockIdx.x - c * tiles16) * 16;
        if (c >= C) return;
        c32* A = reinterpret_cast<c32*>(lds);   // 16 rows of RS256
        c32* tw = A + 16 * RS256;
        for (int k = threadIdx.x; k < 256; k += RBT) tw[k] = s.tw[k];
        const int r = threadIdx.x >> 4, q = threadIdx.x & 15, a = a0 + r;
        c32* R = A + r * RS256;
        const float* xc = s.x + (long)c * s.n_vs;
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const int b = 16 * n1 + q;
            float v = 0.f;
            if (a < n && b < n) {
                const int vi = s.vmap[a * n + b];
                if (vi >= 0) v = xc[vi];
            }
            R[17 * n1 + q] = c32{v, 0.f};   // pidx(b)
        }
        __syncthreads();   // the twiddles
        fft256_group<false>(R, tw, q);
        __syncthreads();
        const int rows = min(16, n - a0);
        for (int idx = threadIdx.x; idx < Lh * 16; idx += RBT) {
            const int f = idx >> 4, rr = idx & 15;
            if (rr < rows) s.T[((long)f * C + c) * n + a0 + rr] = A[rr * RS256 + f + (f >> 4)];
        }
        return;
    }
    const int rt = row_tile_fwd(L), tiles = (n + rt - 1) / rt;
    const int c = blockIdx.x / tiles, a0 = (blockIdx.x - c * tiles) * rt;
    if (c >= C) return;
    const int rows = min(rt, n - a0);
    for (int k = threadIdx.x; k < L; k += RBT) tws[k] = s.tw[k];
    if (is_pow2(L)) {
        int bits = 0;
        while ((1 << bits) < L) ++bits;
        c32* A = reinterpret_cast<c32*>(lds);   // rows x L
        for (int i = threadIdx.x; i < rows * n; i += RBT) {
            const int r = i / n, b = i - r * n;
            const int v = s.vmap[(a0 + r) * n + b];
            A[r * L + b] = c32{v >= 0 ? s.x[(long)c * s.n_vs + v] : 0.f, 0.f};
        }
        __syncthreads();
        fft_dif<RBT, false>(A, tws, rows, bits, L, n);   // bit-reversed output
        for (int idx = threadIdx.x; idx < Lh * rt; idx += RBT) {
            const int f2 = idx / rt, r = idx - f2 * rt;
            if (r < rows) s.T[((long)f2 * C + c) * n + a0 + r] = A[r * L + bitrev(f2, bits)];
        }
        return;
    }
    float* xs = reinterpret_cast<float*>(lds);   // rows x (n + 1)
    const int ld = n + 1;
    for (int i = threadIdx.x; i < rows * n; i += RBT) {
        const int r = i / n, b = i - r * n;
        const int v = s.vmap[(a0 + r) * n + b];
        xs[r * ld + b] = v >= 0 ? s.x[(long)c * s.n_vs + v] : 0.f;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < Lh * rt; idx += RBT) {
        const int f2 = idx / rt, r = idx - f2 * rt;
        if (r >= rows) continue;
        float re = 0.f, im = 0.f;
        int m = 0;
        for (int b = 0; b < n; ++b) {
            const c32 w = tws[m];
            re += xs[r * ld + b] * w.x;
            im -= xs[r * ld + b] * w.y;
            m += f2;
            if (m >= L) m -= L;
        }
        s.T[((long)f2 * C + c) * n + a0 + r] = c32{re, im};
    }
}

__global__ __launch_bounds__(RBT) void k_brow_inv(const BSys* __restrict__ sys, int S) {
    __shared__ __align__(16) char lds[RLDS + 1024 * sizeof(c32)];
    c32* tws = reinterpret_cast<c32*>(lds + RLDS);
    const BSys s = sys[blockIdx.y];
    const int n = s.n, L = s.L, Lh = L / 2 + 1, C = 2 * s.G;
    if (L == 256) {
        const int tiles16 = (n + 15) / 16, c = blockIdx.x / tiles16, a0 = (blockIdx.x - c * tiles16) * 16;
        if (c >= C) return;
        c32* A = reinterpret_cast<c32*>(lds);   // 16 rows of RS256
        c32* tw = A + 16 * RS256;
        for (int k = threadIdx.x; k < 256; k += RBT) tw[k] = s.tw[k];
        const int rows = min(16, n - a0);
        // Z[f] = U_c[f] and Z[L - f] = conj U_c[f] (the S column shares summed; real part only at f = 0
        // and L / 2): the Hermitian extension, whose transform is real
        for (int idx = threadIdx.x; idx < Lh * 16; idx += RBT) {
            const int f = idx >> 4, rr = idx & 15;
            c32 u = c32{0.f, 0.f};
            if (rr < rows)
                for (int h = 0; h < S; ++h) {
                    const c32 v = s.U[(((long)f * S + h) * C + c) * n + a0 + rr];
                    u.x += v.x;
                    u.y += v.y;
                }
            c32* Rr = A + rr * RS256;
            if (f == 0 || f == 128) {
                Rr[f + (f >> 4)] = c32{u.x, 0.f};
            } else {
                const int fc = 256 - f;
                Rr[f + (f >> 4)] = u;
                Rr[fc + (fc >> 4)] = c32{u.x, -u.y};
            }
        }
        __syncthreads();
        const int r = threadIdx.x >> 4, q = threadIdx.x & 15, a = a0 + r;
        c32* R = A + r * RS256;
        fft256_group<true>(R, tw, q);
        // outputs b = q + 16 k of row a: written by this lane group (one wave, in order)
        if (a < n) {
            const float inv = 1.f / (256.f * 256.f);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int b = q + 16 * k;
                if (b >= n) break;
                const int v = s.vmap[a * n + b];
                if (v < 0) continue;
                const long i = (long)c * s.n_vs + v;
                float out = R[b + k].x * inv;   // pidx(b) = b + b / 16
                if (s.noise) out += s.noise[i] * s.x[i];
                if (s.nxy) out += s.nxy[(long)(c >> 1) * s.n_vs + v] * s.x[(long)(c ^ 1) * s.n_vs + v];
                s.y[i] = out;
            }
        }
        return;
    }
    const int rt = row_tile_inv(L), tiles = (n + rt - 1) / rt;
    const int c = blockIdx.x / tiles, a0 = (blockIdx.x - c * tiles) * rt;
    if (c >= C) return;
    const int rows = min(rt, n - a0);
    for (int k = threadIdx.x; k < L; k += RBT) tws[k] = s.tw[k];
    const float inv = 1.f / ((float)L * (float)L);
    const bool even = (L % 2) == 0;
    // the S column shares summed: U[f2][a0 + r], contiguous in r
    auto share = [&](int f2, int r) {
        c32 u = c32{0.f, 0.f};
        for (int h = 0; h < S; ++h) {
            const c32 v = s.U[(((long)f2 * S + h) * C + c) * n + a0 + r];
            u.x += v.x;
            u.y += v.y;
        }
        return u;
    };
    if (is_pow2(L)) {
        int bits = 0;
        while ((1 << bits) < L) ++bits;
        c32* A = reinterpret_cast<c32*>(lds);   // rows x L, bit-reversed input
        for (int idx = threadIdx.x; idx < L * rt; idx += RBT) {
            const int f = idx / rt, r = idx - f * rt;
            if (r >= rows) continue;
            c32 u = c32{0.f, 0.f};
            if (f < Lh) {
                u = share(f, r);
                const float wt = (f == 0 || (even && 2 * f == L)) ? 1.f : 2.f;
                u.x *= wt;
                u.y *= wt;
            }
            A[r * L + bitrev(f, bits)] = u;
        }
        __syncthreads();
        fft_dit_inv<RBT, false>(A, tws, rows, bits, L);
        for (int idx = threadIdx.x; idx < rows * n; idx += RBT) {
            const int r = idx / n, b = idx - r * n;
            const int v = s.vmap[(a0 + r) * n + b];
            if (v < 0) continue;
            const long i = (long)c * s.n_vs + v;
            float out = A[r * L + b].x * inv;
            if (s.noise) out += s.noise[i] * s.x[i];
            if (s.nxy) out += s.nxy[(long)(c >> 1) * s.n_vs + v] * s.x[(long)(c ^ 1) * s.n_vs + v];
            s.y[i] = out;
        }
        return;
    }
    c32* Us = reinterpret_cast<c32*>(lds);   // Lh x rt
    for (int idx = threadIdx.x; idx < Lh * rt; idx += RBT) {
        const int f2 = idx / rt, r = idx - f2 * rt;
        Us[idx] = r < rows ? share(f2, r) : c32{0.f, 0.f};
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < rows * n; idx += RBT) {
        const int r = idx / n, b = idx - r * n;
        const int v = s.vmap[(a0 + r) * n + b];
        if (v < 0) continue;
        float acc = Us[r].x;
        int m = b;
        for (int f2 = 1; f2 < Lh; ++f2) {
            const c32 u = Us[f2 * rt + r], w = tws[m];
            const float wt = (even && 2 * f2 == L) ? 1.f : 2.f;
            acc += wt * (u.x * w.x - u.y * w.y);
            m += b;
            if (m >= L) m -= L;
        }
        const long i = (long)c * s.n_vs + v;
        float out = acc * inv;
        if (s.noise) out += s.noise[i] * s.x[i];
        if (s.nxy) out += s.nxy[(long)(c >> 1) * s.n_vs + v] * s.x[(long)(c ^ 1) * s.n_vs + v];
        s.y[i] = out;
    }
}

// x and y outputs of sensor g at position k: sum over the sensors hh of the
// 2x2 blocks M_{g hh} (Hermitian packing: real diagonal blocks, pairs g < hh
// stored once, M_{g hh} = conj(M_{hh g}) for g > hh) times X_hh
__device__ __forceinline__ void sensor_products(const float* Ms, const c32* X, int m, int P, int G, int g, int k,
                                                bool pad, c32& yx, c32& yy) {
    const float* Mf = Ms + k * (P + 1);
    c32 ax = c32{0.f, 0.f}, ay = c32{0.f, 0.f};
    for (int hh = 0; hh < G; ++hh) {
        const int ix = (2 * hh) * m + k, iy = ix + m;
        const c32 xh = X[pad ? pidx<true>(ix) : ix], yh = X[pad ? pidx<true>(iy) : iy];
        c32 mxx, mxy, myy;
        if (hh == g) {
            mxx = c32{Mf[3 * g], 0.f};
            mxy = c32{Mf[3 * g + 1], 0.f};
            myy = c32{Mf[3 * g + 2], 0.f};
        } else {
            const int lo = g < hh ? g : hh, hi = g < hh ? hh : g;
            const int o = 3 * G + 6 * (lo * (2 * G - lo - 1) / 2 + (hi - lo - 1));
            const float sg = g < hh ? 1.f : -1.f;
            mxx = c32{Mf[o], sg * Mf[o + 1]};
            mxy = c32{Mf[o + 2], sg * Mf[o + 3]};
            myy = c32{Mf[o + 4], sg * Mf[o + 5]};
        }
        ax = cadd(ax, cadd(cmul(mxx, xh), cmul(mxy, yh)));
        ay = cadd(ay, cadd(cmul(mxy, xh), cmul(myy, yh)));
    }
    yx = ax;
    yy = ay;
}

// Entry (a, b) of the general Hermitian C x C matrix of one frequency packed
// in C^2 reals: slot a = Re H[a][a]; for a < b, slots C + 2k and C + 2k + 1 =
// Re, Im H[a][b] with k = a C - a (a + 1) / 2 + b - a - 1; H[b][a] = conj H[a][b].
__device__ __forceinline__ c32 herm_entry(const float* Mf, int C, int a, int b) {
    if (a == b) return c32{Mf[a], 0.f};
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int k = lo * C - lo * (lo + 1) / 2 + hi - lo - 1;
    const float im = Mf[C + 2 * k + 1];
    return c32{Mf[C + 2 * k], a < b ? im : -im};
}

// outputs 2g and 2g + 1 at position k of Y = H X (the block-circulant
// preconditioner's per-frequency matrices)
__device__ __forceinline__ void herm_products(const float* Ms, const c32* X, int m, int P, int C, int g, int k,
                                              bool pad, c32& y0, c32& y1) {
    const float* Mf = Ms + k * (P + 1);
    c32 a0 = c32{0.f, 0.f}, a1 = c32{0.f, 0.f};
    for (int q = 0; q < C; ++q) {
        const int iq = q * m + k;
        const c32 xq = X[pad ? pidx<true>(iq) : iq];
        a0 = cadd(a0, cmul(herm_entry(Mf, C, 2 * g, q), xq));
        a1 = cadd(a1, cmul(herm_entry(Mf, C, 2 * g + 1, q), xq));
    }
    y0 = a0;
    y1 = a1;
}

// Column work items q = 0, 1, ...: xcd = q mod 8, slot = q / 8, column
// (slot / S) 8 + xcd, share h = slot mod S.  Workgroup b takes q = b, b + grid,
// ... (grid a multiple of 8): all its items are on its own XCD, and the sibling
// item q + 8 is processed by workgroup b + 8 at the same time.  The spectra of
// the next item load under the products and inverse transform of the current.
// PACK 0: the slope-slope spectra (3 G^2 reals per frequency); PACK 1: the
// preconditioner's general Hermitian spectra (C^2 reals per frequency)
// HALF: spectra stored in FP32 (0), FP16 scaled per frequency (1) or BF16 (2);
// the products are FP32 either way.
template <int VEC, int PACK, int HALF>
__global__ __launch_bounds__(BT, 2) void k_bcol(const BSys* __restrict__ sys, const int* __restrict__ col_sys,
                                                 int total_cols, int S, int Lmax) {
    extern __shared__ __align__(16) char smem_raw[];
    const int sh = S == 4 ? 2 : S - 1, hm = S - 1;   // S is 1, 2 or 4
    int q = blockIdx.x;
    int col = ((q >> 3) >> sh) * 8 + (q & 7), h = (q >> 3) & hm;
    if (col >= total_cols) return;
    c32* tws = reinterpret_cast<c32*>(smem_raw);   // twiddles of the current L
    char* work = smem_raw + (((size_t)Lmax * sizeof(c32) + 15) & ~size_t(15));

    // this item's spectra and input column, prefetched; the system of the next
    // item is looked up one item ahead
    typename vecf<VEC>::t pf[NPF];
    typename vech<VEC>::t pfh[NPF];
    float pfs[NPF];
    c32 tp[TPF];
    int si = col_sys[col];
    {
        const BSys& s0 = sys[si];
        const int f20 = col - s0.col0, P0 = PACK ? 4 * s0.G * s0.G : 3 * s0.G * s0.G, Cn0 = 2 * s0.G * s0.n;
#pragma unroll
        for (int i = 0; i < TPF; ++i) {
            const int idx = threadIdx.x + i * BT;
            tp[i] = gload(s0.T + (size_t)f20 * Cn0 + (idx < Cn0 ? idx : 0));
        }
        if constexpr (HALF)
            spectra_load_h<VEC>(pfh, pfs, s0.Mh + (size_t)f20 * s0.L * P0, s0.Mhs + (size_t)f20 * s0.L, 0,
                                (s0.L >> sh) * P0 / VEC, P0, S, h);
        else
            spectra_load<VEC>(pf, s0.M + (size_t)f20 * s0.L * P0, 0, (s0.L >> sh) * P0 / VEC, P0, S, h);
    }
    int qn = q + gridDim.x;
    int coln = ((qn >> 3) >> sh) * 8 + (qn & 7);
    int sin_ = coln < total_cols ? col_sys[coln] : 0;
    int prevL = -1;
    while (true) {
        const BSys& s = sys[si];
        const int f2 = col - s.col0;
        const int n = s.n, G = s.G, C = 2 * G, L = s.L, m = L >> sh, P = PACK ? C * C : 3 * G * G, Q = m * P;
        const bool fft = (m & (m - 1)) == 0;
        int bits = 0;
        while ((1 << bits) < m) ++bits;
        float* Ms = reinterpret_cast<float*>(work);
        c32* A = reinterpret_cast<c32*>(work + ((((size_t)m * (P + 1) * sizeof(float)) + 15) & ~size_t(15)));
        c32* B = A + (size_t)C * m;   // plain-sum transforms only (the FFT buffer A is padded, pidx)
        // next item: its system's fields are read now, used after this item's forward transform
        const bool more = coln < total_cols;
        const int hn = (qn >> 3) & hm;
        const BSys& sn = sys[sin_];
        const float* Mn = sn.M;
        const unsigned short* Mnh = sn.Mh;
        const float* Mnhs = sn.Mhs;
        const c32* Tn = sn.T;
        const int Ln = sn.L, Gn = sn.G, nn = sn.n, f2n = coln - sn.col0;

        __syncthreads();   // the previous item's last LDS reads are done
        if (L != prevL) {
            for (int i = threadIdx.x; i < L; i += BT) tws[i] = gload(s.tw + i);
            prevL = L;
            __syncthreads();
        }
        // twisted input column folded to length m: entry a < n goes to a mod m
        // (m >= n / 2, so at most two terms: those with a >= m are added in a
        // second pass); entries from min(n, m) on are zero and never read
        {
            const c32* Tc = s.T + (size_t)f2 * C * n;
            auto fold = [&](c32 v, int c, int a, bool add) {
                int hw = h * a;   // < 2L
                if (hw >= L) hw -= L;
                if (h) v = cmulc(v, tws[hw]);   // w_L^{h a}
                const int i = c * m + (add ? a - m : a);
                const int li = fft ? pidx<true>(i) : i;
                A[li] = add ? cadd(A[li], v) : v;
            };
            for (int pass = 0; pass < (n > m ? 2 : 1); ++pass) {
                if (pass) __syncthreads();
                Walk wk(n);
#pragma unroll
                for (int i = 0; i < TPF; ++i, wk.next()) {
                    const int idx = threadIdx.x + i * BT;
                    keep(tp[i]);
                    if (idx < C * n && (wk.c >= m) == (pass == 1)) fold(tp[i], wk.r, wk.c, pass == 1);
                }
                for (int idx = threadIdx.x + TPF * BT; idx < C * n; idx += BT, wk.next())
                    if ((wk.c >= m) == (pass == 1)) fold(gload(Tc + idx), wk.r, wk.c, pass == 1);
            }
        }
        __syncthreads();

        // forward column transform of the C channels
        c32* X = A;
        if (fft) {
            fft_dif<BT, true>(A, tws, C, bits, L, n < m ? n : m);   // X at bit-reversed positions
        } else {
            Walk wk(m);
            for (int idx = threadIdx.x; idx < C * m; idx += BT, wk.next()) {
                const c32* in = A + wk.r * m;
                float re = 0.f, im = 0.f;
                int e = 0;
                const int de = (S * wk.c) % L;
                for (int a = 0; a < (n < m ? n : m); ++a) {
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

        // this item's spectra to LDS: first round from the registers, then round by round
        const int rbits = fft ? bits : -1;
        if constexpr (HALF) {
            const unsigned short* Mcol = s.Mh + (size_t)f2 * L * P;
            const float* scol = s.Mhs + (size_t)f2 * L;
            spectra_store_h<VEC, HALF>(pfh, pfs, Ms, 0, Q / VEC, P, rbits);
            for (int base = NPF * BT; base < Q / VEC; base += NPF * BT) {
                spectra_load_h<VEC>(pfh, pfs, Mcol, scol, base, Q / VEC, P, S, h);
                spectra_store_h<VEC, HALF>(pfh, pfs, Ms, base, Q / VEC, P, rbits);
            }
        } else {
            const float* Mcol = s.M + (size_t)f2 * L * P;
            spectra_store<VEC>(pf, Ms, 0, Q / VEC, P, rbits);
            for (int base = NPF * BT; base < Q / VEC; base += NPF * BT) {
                spectra_load<VEC>(pf, Mcol, base, Q / VEC, P, S, h);
                spectra_store<VEC>(pf, Ms, base, Q / VEC, P, rbits);
            }
        }
        __syncthreads();

        // the next item's spectra and input column start loading, and the system
        // of the item after it is looked up
        int sinn = 0, qnn = qn + gridDim.x;
        const int colnn = ((qnn >> 3) >> sh) * 8 + (qnn & 7);
        if (more) {
            const int Pn = PACK ? 4 * Gn * Gn : 3 * Gn * Gn, Cnn = 2 * Gn * nn;
            // the input column first: the next item's first step waits for it alone
#pragma unroll
            for (int i = 0; i < TPF; ++i) {
                const int idx = threadIdx.x + i * BT;
                tp[i] = gload(Tn + (size_t)f2n * Cnn + (idx < Cnn ? idx : 0));
            }
            if constexpr (HALF)
                spectra_load_h<VEC>(pfh, pfs, Mnh + (size_t)f2n * Ln * Pn, Mnhs + (size_t)f2n * Ln, 0,
                                    (Ln >> sh) * Pn / VEC, Pn, S, hn);
            else
                spectra_load<VEC>(pf, Mn + (size_t)f2n * Ln * Pn, 0, (Ln >> sh) * Pn / VEC, Pn, S, hn);
            if (colnn < total_cols) sinn = col_sys[colnn];
        }

        // per-frequency products summed over the input channels: task (g, k) gives
        // the x and y outputs of sensor g at position k (frequency k, or bitrev(k)
        // after the FFT: spectra rows and X share that order)
        c32 yx[TMAX], yy[TMAX];
        {
            Walk wk(m);
            const bool wave_uniform = (m & 63) == 0;   // the 64 tasks of a wave share g
#pragma unroll
            for (int it = 0; it < TMAX; ++it, wk.next()) {
                const int task = threadIdx.x + it * BT;
                yx[it] = yy[it] = c32{0.f, 0.f};
                if (task < m * G) {
                    if constexpr (PACK == 0) {
                        if (wave_uniform)
                            sensor_products(Ms, X, m, P, G, __builtin_amdgcn_readfirstlane(wk.r), wk.c, fft, yx[it],
                                            yy[it]);
                        else
                            sensor_products(Ms, X, m, P, G, wk.r, wk.c, fft, yx[it], yy[it]);
                    } else {
                        if (wave_uniform)
                            herm_products(Ms, X, m, P, C, __builtin_amdgcn_readfirstlane(wk.r), wk.c, fft, yx[it],
                                          yy[it]);
                        else
                            herm_products(Ms, X, m, P, C, wk.r, wk.c, fft, yx[it], yy[it]);
                    }
                }
            }
        }
        __syncthreads();
        c32* Y = A;   // the twisted input is no longer needed (FFT: X is A itself, read above)
        {
            Walk wk(m);
#pragma unroll
            for (int it = 0; it < TMAX; ++it, wk.next()) {
                const int task = threadIdx.x + it * BT;
                if (task < m * G) {
                    const int ix = (2 * wk.r) * m + wk.c, iy = ix + m;
                    Y[fft ? pidx<true>(ix) : ix] = yx[it];
                    Y[fft ? pidx<true>(iy) : iy] = yy[it];
                }
            }
        }
        __syncthreads();

        // this item's share of the inverse column transform, rows a < n
        c32* Uo = s.U + ((size_t)f2 * S + h) * C * n;
        if (fft) {
            fft_dit_inv<BT, true>(Y, tws, C, bits, L);
            Walk wk(n);
            for (int idx = threadIdx.x; idx < C * n; idx += BT, wk.next()) {
                const int a = wk.c;   // V at a mod m, a < n <= 2m
                c32 v = Y[pidx<true>(wk.r * m + (a < m ? a : a - m))];
                if (h) {
                    int hw = h * a;
                    if (hw >= L) hw -= L;
                    v = cmul(v, tws[hw]);   // w_L^{-h a}
                }
                gstore(Uo + idx, v);
            }
        } else {
            Walk wk(n);
            for (int idx = threadIdx.x; idx < C * n; idx += BT, wk.next()) {
                const int a = wk.c;
                const c32* yv = Y + wk.r * m;
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
                gstore(Uo + idx, c32{re, im});
            }
        }
        if (!more) break;
        q = qn;
        col = coln;
        h = hn;
        si = sin_;
        qn = qnn;
        coln = colnn;
        sin_ = sinn;
    }
}

// ---------------------------------------------------------------------------
// Column transforms of length m in {64, 128} by single waves: m = 8 Q, each
// channel taken by Q lanes of one wave (Q = 8 or 16), eight points a lane.
// Forward, with n = Q n1 + q and k = k1 + 8 k2:
//   X[k1 + 8 k2] = sum_q w_Q^{q k2} [w_m^{q k1} sum_{n1} x[Q n1 + q] w_8^{n1 k1}],
// an 8-point DFT in registers (lane q), a twiddle, a transpose through the
// channel's own LDS buffer (written and read by lanes of one wave, in order:
// no workgroup barrier), and the Q-point DFTs over q: in registers for Q = 8;
// for Q = 16 as two 8-point halves (even and odd q) in a lane pair combined by
// one radix-2 step across the pair (DPP swap).  Input in natural order, output
// at bit-reversed positions, both in the padded layout pidx; the inverse runs
// the same steps backwards (exponent +, unnormalised).

// 8-point DFT in registers, natural order in and out; INV: exponent +
template <bool INV>
__device__ __forceinline__ void dft8(c32 (&a)[8]) {
    constexpr float R = 0.70710678118654752f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const c32 u = cadd(a[i], a[i + 4]), v = csub(a[i], a[i + 4]);
        a[i] = u;
        a[i + 4] = v;
    }
    // twiddles w_8^i on the second half: (1 - i) R, -i, (-1 - i) R (forward; conjugates inverse)
    a[5] = INV ? c32{(a[5].x - a[5].y) * R, (a[5].x + a[5].y) * R} : c32{(a[5].x + a[5].y) * R, (a[5].y - a[5].x) * R};
    a[6] = INV ? mul_pi(a[6]) : mul_mi(a[6]);
    a[7] = INV ? c32{(-a[7].x - a[7].y) * R, (a[7].x - a[7].y) * R} : c32{(a[7].y - a[7].x) * R, -(a[7].x + a[7].y) * R};
#pragma unroll
    for (int b = 0; b < 8; b += 4)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const c32 u = cadd(a[b + i], a[b + i + 2]), v = csub(a[b + i], a[b + i + 2]);
            a[b + i] = u;
            a[b + i + 2] = i ? (INV ? mul_pi(v) : mul_mi(v)) : v;
        }
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
        const c32 u = cadd(a[i], a[i + 1]), v = csub(a[i], a[i + 1]);
        a[i] = u;
        a[i + 1] = v;
    }
    // bit-reversed to natural order
    c32 t = a[1];
    a[1] = a[4];
    a[4] = t;
    t = a[3];
    a[3] = a[6];
    a[6] = t;
}

// value of the partner lane (lane ^ 1)
__device__ __forceinline__ c32 swap_pair(c32 v) {
    return c32{__int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.x), 0xB1, 0xF, 0xF, false)),
               __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.y), 0xB1, 0xF, 0xF, false))};
}

// Padded index pidx(i) = i + i / 16 of the entries a wave-transform lane
// touches, written as one base per lane plus compile-time offsets (for
// i = Q n1 + q and i = Q k1 + j with q, j < Q, and for the bit-reversed output
// positions), so that the compiler keeps one address register per pattern.
__device__ __forceinline__ int rev3(int v) { return ((v & 1) << 2) | (v & 2) | ((v >> 2) & 1); }

// Forward transform of C channels of length M into the channel buffers;
// threads t < C M / 8 take part (the others return at once), there is no
// workgroup barrier inside.  The input x[i] of channel c comes from in(c, i)
// (the caller folds and twists it there, from wherever it is staged).
template <int M, typename In>
__device__ __forceinline__ void fft_wave_fwd(c32* A, const c32* tws, int C, int L, In in) {
    constexpr int Q = M / 8, LQ = Q == 16 ? 4 : 3, MP = M + M / 16;
    const int t = threadIdx.x;
    if (t >= C * Q) return;
    const int q = t & (Q - 1), step = L / M;
    c32* Ac = A + (t >> LQ) * MP;
    // pidx(Q n1 + q): Q = 16: 17 n1 + q; Q = 8: 8 n1 + n1 / 2 + q
    auto row = [](int n1) { return Q == 16 ? 17 * n1 : 8 * n1 + (n1 >> 1); };
    c32 a[8];
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) a[n1] = in(t >> LQ, Q * n1 + q);   // x[Q n1 + q] of channel t / Q
    dft8<false>(a);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) a[k1] = cmulc(a[k1], tws[((q * k1) & (M - 1)) * step]);   // w_M^{q k1}
    wave_lds_order();
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) Ac[q + row(k1)] = a[k1];   // transposed: pidx(Q k1 + q)
    wave_lds_order();
    if constexpr (Q == 8) {
        const int k1 = q, rb = rev3(k1);
        c32* Ar = Ac + row(k1);   // pidx(8 k1 + j) = row(k1) + j
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = Ar[j];
        dft8<false>(a);
        wave_lds_order();
        // X[k1 + 8 k2] at bitrev6 = 8 rev3(k1) + rev3(k2): pidx = 8 rb + rb / 2 + rev3(k2)
        c32* Ao = Ac + 8 * rb + (rb >> 1);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) Ao[rev3(k2)] = a[k2];
    } else {
        const int k1 = q >> 1, e = q & 1, rb = rev3(k1);
        c32* Ar = Ac + 17 * k1 + e;   // pidx(16 k1 + 2 j + e) = 17 k1 + 2 j + e
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = Ar[2 * j];
        dft8<false>(a);   // e = 0: E[j], e = 1: O[j] (even / odd q)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (e) a[j] = cmul(a[j], w16(j));
            const c32 r = swap_pair(a[j]);
            a[j] = e ? csub(r, a[j]) : cadd(a[j], r);   // X[k1 + 8 (j + 8 e)] = E + w O, E - w O
        }
        wave_lds_order();
        // bitrev7(k1 + 8 j + 64 e) = 16 rev3(k1) + 2 rev3(j) + e: pidx = 17 rb + 2 rev3(j) + e
        c32* Ao = Ac + 17 * rb + e;
#pragma unroll
        for (int j = 0; j < 8; ++j) Ao[2 * rev3(j)] = a[j];
    }
}

// Inverse transform (exponent +, unnormalised) of C channels of length M,
// bit-reversed positions in; output x[a] of channel c goes to out(c, a, x)
// from the registers of the lane that computes it (natural order in the
// channel's buffer when out is WriteBack); as fft_wave_fwd.
struct WriteBack {
    c32* A;
    int mp;   // channel stride of the padded buffer
    __device__ void operator()(int c, int a, c32 v) const { A[c * mp + a + (a >> 4)] = v; }
};

template <int M, typename Out>
__device__ __forceinline__ void fft_wave_inv(c32* A, const c32* tws, int C, int L, Out out) {
    constexpr int Q = M / 8, LQ = Q == 16 ? 4 : 3, MP = M + M / 16;
    const int t = threadIdx.x;
    if (t >= C * Q) return;
    const int q = t & (Q - 1), step = L / M;
    c32* Ac = A + (t >> LQ) * MP;
    auto row = [](int n1) { return Q == 16 ? 17 * n1 : 8 * n1 + (n1 >> 1); };
    c32 a[8];
    if constexpr (Q == 8) {
        const int k1 = q, rb = rev3(k1);
        const c32* Ai = Ac + 8 * rb + (rb >> 1);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) a[k2] = Ai[rev3(k2)];   // X[k1 + 8 k2]
        dft8<true>(a);   // Z_{k1}[j], j < 8
#pragma unroll
        for (int j = 1; j < 8; ++j) a[j] = cmul(a[j], tws[((j * k1) & (M - 1)) * step]);   // w_M^{-j k1}
        wave_lds_order();
        c32* Ar = Ac + row(k1);
#pragma unroll
        for (int j = 0; j < 8; ++j) Ar[j] = a[j];
    } else {
        const int k1 = q >> 1, e = q & 1, rb = rev3(k1);
        const c32* Ai = Ac + 17 * rb + e;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = Ai[2 * rev3(j)];   // A = X[k1 + 8 j] (e = 0), B = X[k1 + 8 j + 64] (e = 1)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const c32 r = swap_pair(a[j]);
            a[j] = e ? cmulc(csub(r, a[j]), w16(j)) : cadd(a[j], r);   // A + B; (A - B) w_16^{-j}
        }
        dft8<true>(a);   // Z_{k1}[2 j + e]
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int zq = 2 * j + e;
            if (zq) a[j] = cmul(a[j], tws[((zq * k1) & (M - 1)) * step]);   // w_M^{-q k1}
        }
        wave_lds_order();
        c32* Ar = Ac + 17 * k1 + e;
#pragma unroll
        for (int j = 0; j < 8; ++j) Ar[2 * j] = a[j];
    }
    wave_lds_order();
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) a[k1] = Ac[q + row(k1)];   // Z_{k1}[q]
    dft8<true>(a);
    wave_lds_order();
    const int c = t >> LQ;
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) out(c, Q * n1 + q, a[n1]);   // x[Q n1 + q]
}

// ---------------------------------------------------------------------------
// Column kernel for batches whose every L is a power of two.  There the
// spectra of a column are kept slot-major with the column's L frequencies in
// bit-reversed order ([Lh][P][L], built once per system by k_slot_major), so
// the m frequencies S k + h of item h are one contiguous run of every slot
// row, at bitrev_s(h) m, already in the order of the m-point FFT's output.
// An item's spectra (P runs of m values) go from HBM to LDS by direct loads
// (global_load_lds_dwordx4: each lane moves 16 bytes, one wave fills 1 KB of
// LDS), issued by every wave as soon as the previous item's products are
// done: they land under that item's inverse transform and this item's input
// fold and forward transform, with no registers held and no copy through the
// vector ALU.  The products read value j of position p at j m + p (the lanes
// of a wave on consecutive positions: no bank conflicts).  The input column of
// the next item loads into registers during this item's forward transform;
// one wait on all vector memory operations before the products covers both.
constexpr unsigned WAIT_VM0 = 0x0F70;   // s_waitcnt vmcnt(0), lgkmcnt and expcnt not waited

__device__ __forceinline__ int bitrev_split(int h, int sh) {   // bit reversal of h < 2^sh, sh <= 2
    return sh == 2 ? (((h & 1) << 1) | (h >> 1)) : h;
}

template <int HALF>
__device__ __forceinline__ float sdec(const void* M, int i) {
    if constexpr (HALF == 0) return static_cast<const float*>(M)[i];
    else return half_dec<HALF>(static_cast<const unsigned short*>(M)[i]);
}

// sensor_products on the slot-major LDS layout: value j of position p at j m + p
template <int HALF>
__device__ __forceinline__ void sensor_products_t(const void* Ms, const c32* X, int m, int G, int g, int p, c32& yx,
                                                  c32& yy) {
    c32 ax = c32{0.f, 0.f}, ay = c32{0.f, 0.f};
    for (int hh = 0; hh < G; ++hh) {
        const c32 xh = X[pidx<true>(2 * hh * m + p)], yh = X[pidx<true>((2 * hh + 1) * m + p)];
        c32 mxx, mxy, myy;
        if (hh == g) {
            mxx = c32{sdec<HALF>(Ms, 3 * g * m + p), 0.f};
            mxy = c32{sdec<HALF>(Ms, (3 * g + 1) * m + p), 0.f};
            myy = c32{sdec<HALF>(Ms, (3 * g + 2) * m + p), 0.f};
        } else {
            const int lo = g < hh ? g : hh, hi = g < hh ? hh : g;
            const int b = (3 * G + 6 * (lo * (2 * G - lo - 1) / 2 + (hi - lo - 1))) * m + p;
            const float sg = g < hh ? 1.f : -1.f;
            mxx = c32{sdec<HALF>(Ms, b), sg * sdec<HALF>(Ms, b + m)};
            mxy = c32{sdec<HALF>(Ms, b + 2 * m), sg * sdec<HALF>(Ms, b + 3 * m)};
            myy = c32{sdec<HALF>(Ms, b + 4 * m), sg * sdec<HALF>(Ms, b + 5 * m)};
        }
        ax = cadd(ax, cadd(cmul(mxx, xh), cmul(mxy, yh)));
        ay = cadd(ay, cadd(cmul(mxy, xh), cmul(myy, yh)));
    }
    yx = ax;
    yy = ay;
}

// herm_entry / herm_products on the slot-major LDS layout
template <int HALF>
__device__ __forceinline__ c32 herm_entry_t(const void* Ms, int m, int p, int C, int a, int b) {
    if (a == b) return c32{sdec<HALF>(Ms, a * m + p), 0.f};
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int k = lo * C - lo * (lo + 1) / 2 + hi - lo - 1;
    const float im = sdec<HALF>(Ms, (C + 2 * k + 1) * m + p);
    return c32{sdec<HALF>(Ms, (C + 2 * k) * m + p), a < b ? im : -im};
}

template <int HALF>
__device__ __forceinline__ void herm_products_t(const void* Ms, const c32* X, int m, int C, int g, int p, c32& y0,
                                                c32& y1) {
    c32 a0 = c32{0.f, 0.f}, a1 = c32{0.f, 0.f};
    for (int q = 0; q < C; ++q) {
        const c32 xq = X[pidx<true>(q * m + p)];
        a0 = cadd(a0, cmul(herm_entry_t<HALF>(Ms, m, p, C, 2 * g, q), xq));
        a1 = cadd(a1, cmul(herm_entry_t<HALF>(Ms, m, p, C, 2 * g + 1, q), xq));
    }
    y0 = a0;
    y1 = a1;
}

__device__ __forceinline__ c32 cfma(c32 acc, c32 a, c32 b) {   // acc + a b
    return c32{acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ c32 cfmac(c32 acc, c32 a, c32 b) {  // acc + conj(a) b
    return c32{acc.x + a.x * b.x + a.y * b.y, acc.y + a.x * b.y - a.y * b.x};
}

// Pins the accumulators updated so far: the products that feed them are issued
// before it, so the spectra values they read do not stay live past it (the
// compiler would otherwise load far ahead and run out of registers).
__device__ __forceinline__ void pin4(c32& a, c32& b, c32& c, c32& d) {
    asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(b.x), "+v"(b.y), "+v"(c.x), "+v"(c.y), "+v"(d.x), "+v"(d.y)::"memory");
}
__device__ __forceinline__ void pin2(c32& a, c32& b) {
    asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(b.x), "+v"(b.y)::"memory");
}

// Slope spectra, two lanes per position (adjacent lanes of one wave): lane e
// gives the outputs of component e (x: 0, y: 1) of every sensor.  Of a 2x2
// block it reads the two values its rows need, at slots o + 2e and o + 2 + 2e
// (xx, xy for e = 0; xy, yy for e = 1; real blocks (g, g): 3g + e, 3g + 1 + e),
// so every offset is one per-lane base plus an immediate.  X is read by both
// lanes before either writes (in program order, one wave: no barrier).
template <int G, int M, int HALF>
__device__ __forceinline__ void products_pos2(const void* Ms, c32* A, int p, int e, float f) {
    constexpr int MP = M + M / 16, NP = G * (G - 1) / 2;
    c32* Ap = A + (p + (p >> 4));
    c32 x[2 * G], y[G];
#pragma unroll
    for (int c = 0; c < 2 * G; ++c) x[c] = Ap[c * MP];
    const int pe = p + 2 * e * M;   // value j of this lane's rows at j M + pe (real blocks: j M + p + e M)
    auto v = [&](int j) { return sdec<HALF>(Ms, j * M + pe); };
    auto vd = [&](int j) { return sdec<HALF>(Ms, j * M + p + e * M); };
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const float s0 = vd(3 * g), s1 = vd(3 * g + 1);
        const c32 a = x[2 * g], b = x[2 * g + 1];
        y[g] = c32{s0 * a.x + s1 * b.x, s0 * a.y + s1 * b.y};
        if (g & 1) pin2(y[g - 1], y[g]);
    }
    float cur[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) cur[i] = v(3 * G + i);
    int lo = 0, hi = 1;
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        float nxt[4];
        if (t + 1 < NP) {
#pragma unroll
            for (int i = 0; i < 4; ++i) nxt[i] = v(3 * G + 6 * (t + 1) + i);
        }
        const c32 ma = c32{cur[0], cur[1]}, mb = c32{cur[2], cur[3]};
        y[lo] = cfma(cfma(y[lo], ma, x[2 * hi]), mb, x[2 * hi + 1]);
        y[hi] = cfmac(cfmac(y[hi], ma, x[2 * lo]), mb, x[2 * lo + 1]);
        pin2(y[lo], y[hi]);
        if (t + 1 < NP) {
#pragma unroll
            for (int i = 0; i < 4; ++i) cur[i] = nxt[i];
        }
        if (++hi == G) {
            ++lo;
            hi = lo + 1;
        }
    }
    wave_lds_order();
#pragma unroll
    for (int g = 0; g < G; ++g) Ap[(2 * g + e) * MP] = HALF == 1 ? c32{y[g].x * f, y[g].y * f} : y[g];
}

// All C outputs of position p for the preconditioner's general Hermitian C x C
// blocks (C^2 reals; the C (C - 1) / 2 entries above the diagonal in storage
// order), one thread per position, in place: X_c read from and Y_c written to
// pidx(c M + p) = c (M + M / 16) + pidx(p) (M a multiple of 16); G and M
// compile-time, so every LDS offset is an immediate.  f: the FP16 factor.
template <int C, int M, int HALF>
__device__ __forceinline__ void products_pos_herm(const void* Ms, c32* A, int p, float f) {
    constexpr int MP = M + M / 16, NE = C * (C - 1) / 2;
    c32* Ap = A + (p + (p >> 4));
    c32 x[C], y[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = Ap[c * MP];
    auto v = [&](int j) { return sdec<HALF>(Ms, j * M + p); };
#pragma unroll
    for (int a = 0; a < C; ++a) {
        const float d = v(a);
        y[a] = c32{d * x[a].x, d * x[a].y};
    }
    int a = 0, b = 1;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const c32 hv = c32{v(C + 2 * k), v(C + 2 * k + 1)};
        y[a] = cfma(y[a], hv, x[b]);
        y[b] = cfmac(y[b], hv, x[a]);
        pin2(y[a], y[b]);
        if (++b == C) {
            ++a;
            b = a + 1;
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) Ap[c * MP] = HALF == 1 ? c32{y[c].x * f, y[c].y * f} : y[c];
}

// products of every position of an item, one thread per position, for G in
// [4, 6] and m in {64, 128} (the columns of L = 256 split in 2 or 4, and of
// L = 128 split in 2); false for other sizes, the caller then uses tasks (with
// G >= 7 the accumulators of one position no longer fit the registers of four
// waves per SIMD)
template <int PACK, int HALF>
__device__ __forceinline__ bool products_fixed(const void* Ms, c32* A, const float* fac, int m, int G) {
    if ((m != 64 && m != 128) || G < 4 || G > 6) return false;
    if constexpr (PACK == 0) {   // two lanes per position
        const int p = threadIdx.x >> 1, e = threadIdx.x & 1;
        if (p < m) {
            const float f = HALF == 1 ? fac[p] : 1.f;
#define TT_POS(g, mm) \
    if (G == g && m == mm) products_pos2<g, mm, HALF>(Ms, A, p, e, f);
            TT_POS(4, 64) TT_POS(5, 64) TT_POS(6, 64) TT_POS(4, 128) TT_POS(5, 128) TT_POS(6, 128)
#undef TT_POS
        }
    } else {
        for (int p = threadIdx.x; p < m; p += BT) {
            const float f = HALF == 1 ? fac[p] : 1.f;
#define TT_POS(g, mm) \
    if (G == g && m == mm) products_pos_herm<2 * g, mm, HALF>(Ms, A, p, f);
            TT_POS(4, 64) TT_POS(5, 64) TT_POS(6, 64) TT_POS(4, 128) TT_POS(5, 128) TT_POS(6, 128)
#undef TT_POS
        }
    }
    return true;
}

// One direct load: 16 bytes from g (per lane) to LDS at lds + 16 lane (lds
// uniform over the wave).  Written as inline assembly so that the compiler
// neither adds waits on it (it would make every later LDS access and workgroup
// barrier wait for the whole transfer) nor reorders memory accesses across it;
// the kernel waits for it explicitly (vmcnt) before reading the spectra.
typedef __attribute__((address_space(3))) char lchar;
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const void* g, const void* lds) {
    const unsigned a = __builtin_amdgcn_readfirstlane((unsigned)(size_t)(const lchar*)lds);
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(a), "v"(g) : "memory", "m0");
}
#pragma clang diagnostic pop

// s_waitcnt vmcnt(min(k, 15)) for a wave-uniform k: the wait of a wave for its
// own direct loads older than its last k vector-memory instructions (memory
// instructions of a wave complete in order)
__device__ __forceinline__ void wait_vm_le(int k) {
    switch (k < 15 ? k : 15) {
#define TT_W(i) \
    case i: asm volatile("s_waitcnt vmcnt(" #i ")" ::: "memory"); break;
        TT_W(0) TT_W(1) TT_W(2) TT_W(3) TT_W(4) TT_W(5) TT_W(6) TT_W(7)
        TT_W(8) TT_W(9) TT_W(10) TT_W(11) TT_W(12) TT_W(13) TT_W(14)
#undef TT_W
        default: asm volatile("s_waitcnt vmcnt(15)" ::: "memory"); break;
    }
}

// LDS (bytes from the start of dynamic shared memory): twiddles at 0, the
// transform buffer at offA, the FP16 factors at offF, the input column at offT,
// the spectra at offM; the host sizes each region for the largest system of the
// batch, so the direct loads of the next item never reach the buffers the
// current item still uses.
template <int PACK, int HALF>
__global__ __launch_bounds__(BT, 4) void k_bcolt(const BSys* __restrict__ sys, const int* __restrict__ col_sys,
                                                  int total_cols, int S, int offA, int offF, int offT, int offM) {
    extern __shared__ __align__(16) char smem_raw[];
    typedef typename std::conditional<HALF != 0, unsigned short, float>::type E;
    constexpr int PER = 16 / (int)sizeof(E);   // values per lane of one direct load
    const int sh = S == 4 ? 2 : S - 1, hm = S - 1;   // S is 1, 2 or 4
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    int q = blockIdx.x;
    int col = ((q >> 3) >> sh) * 8 + (q & 7), h = (q >> 3) & hm;
    if (col >= total_cols) return;
    c32* tws = reinterpret_cast<c32*>(smem_raw);
    c32* A = reinterpret_cast<c32*>(smem_raw + offA);
    float* fac = reinterpret_cast<float*>(smem_raw + offF);
    c32* Tst = reinterpret_cast<c32*>(smem_raw + offT);
    char* Ms = smem_raw + offM;

    // Direct loads of item (column cl, share hh) of system s, issued by the
    // waves dw0 .. BT / 64 - 1 (with the single-wave transforms dw0 is the first
    // wave without a channel: those waves issue the whole item at once, under
    // the others' inverse transform; otherwise every wave issues, a few rounds
    // between the passes of the transforms):
    // * first the input column T[f2][c][a] (C n complex, 16 bytes a lane) to
    //   the staging buffer Tst, which the next fold reads: each issuing wave
    //   waits for its share at the top of the next item (its loads issued
    //   after those are counted, dafter) and the workgroup barrier there
    //   publishes it;
    // * then P runs of m values of the spectra, chunk c of the item landing at
    //   Ms + 16 c, round by round (one load per wave per round: chunk
    //   (r nd + w - dw0) 64 + lane, the same position nd 64 / cpr rows on,
    //   nd = BT / 64 - dw0), waited for before the products.
    // The state is uniform but for one byte offset per lane.
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const char* dbase = nullptr;
    unsigned doff = 0, dstep = 0;
    int dround = 0, dchunks = 0, dw0 = 0, dnd = BT / 64, dafter = 0;
    auto dma_begin = [&](const BSys& s, int cl, int hh, int first_wave) {
        const int f2 = cl - s.col0, L = s.L, m = L >> sh, P = PACK ? 4 * s.G * s.G : 3 * s.G * s.G;
        const int run = bitrev_split(hh, sh) * m, lcpr = __builtin_ctz(m / PER);
        dw0 = ((BT / 64 - first_wave) * 64) % (m / PER) ? 0 : first_wave;   // whole rows per round
        dnd = BT / 64 - dw0;
        dafter = 0;
        if (wave_u < dw0) {
            dchunks = 0;
        } else {
            const int t = (wave_u - dw0) * 64 + lane;
            const int Cn = 2 * s.G * s.n, tch = Cn / 2;   // 16-byte chunks of the input column
            const char* tsrc = (const char*)(s.T + (size_t)f2 * Cn);
            for (int c = t; c - lane < tch; c += dnd * 64)
                if (c < tch) dma16(tsrc + 16 * (size_t)c, (const char*)Tst + 16 * (size_t)c);
            const int j0 = t >> lcpr, pp = (t - (j0 << lcpr)) * PER;
            dbase = (const char*)((HALF ? (const E*)s.Mht : (const E*)s.Mt) + ((size_t)f2 * P * L + run));
            doff = (unsigned)(((size_t)j0 * L + pp) * sizeof(E));
            dstep = (unsigned)((size_t)((dnd * 64) >> lcpr) * L * sizeof(E));
            dchunks = P * m / PER;
            if constexpr (HALF == 1) {   // the m factors of these frequencies
                const float* fs = s.Mhst + ((size_t)f2 * L + run);
                for (int c = t; c - lane < m / 4; c += dnd * 64) {
                    if (c < m / 4) dma16(fs + 4 * c, fac + 4 * (size_t)c);
                    ++dafter;
                }
            }
        }
        dround = 0;
    };
    auto dma_rounds = [&](int k) {
        for (int i = 0; i < k; ++i) {
            const int cw = (dround * dnd + wave_u - dw0) * 64;   // first chunk of this wave's load in this round
            if (wave_u < dw0 || cw >= dchunks) return;
            if (cw + lane < dchunks) dma16(dbase + doff + (size_t)dround * dstep, Ms + (size_t)cw * 16);
            ++dround;
            ++dafter;
        }
    };
    auto hook = [&]() { dma_rounds(2); };

    int si = col_sys[col];
    dma_begin(sys[si], col, h, 0);
    dma_rounds(1 << 20);
    int qn = q + gridDim.x;
    int coln = ((qn >> 3) >> sh) * 8 + (qn & 7);
    int sin_ = coln < total_cols ? col_sys[coln] : 0;
    int prevL = -1;
    while (true) {
        const BSys& s = sys[si];
        const int f2 = col - s.col0;
        const int n = s.n, G = s.G, C = 2 * G, L = s.L, m = L >> sh;
        int bits = 0;
        while ((1 << bits) < m) ++bits;
        const bool more = coln < total_cols;
        const int hn = (qn >> 3) & hm;
        const BSys& sn = sys[sin_];
        int sinn = 0, qnn = qn + gridDim.x;
        const int colnn = ((qnn >> 3) >> sh) * 8 + (qnn & 7);
        if (more && colnn < total_cols) sinn = col_sys[colnn];

        if (wave_u >= dw0) wait_vm_le(dafter);   // this wave's share of the input column has landed
        __syncthreads();   // ... every wave's; the previous item's last reads of A and of the twiddles are done
        if (L != prevL) {
            for (int i = threadIdx.x; i < L; i += BT) tws[i] = gload(s.tw + i);
            prevL = L;
            __syncthreads();
        }
        // twisted input column folded to length m: x[i] = sum over a = i, i + m (< n) of T[c][a] w_L^{h a}
        // (m >= n / 2: at most two terms)
        auto twisted = [&](int c, int a) {
            c32 v = Tst[c * n + a];
            if (h) {
                int hw = h * a;   // < 2L
                if (hw >= L) hw -= L;
                v = cmulc(v, tws[hw]);   // w_L^{h a}
            }
            return v;
        };
        // X at bit-reversed positions; the waves without a channel issue their direct loads meanwhile
        if (m == 128 || m == 64) {
            auto in = [&](int c, int i) {
                c32 v = c32{0.f, 0.f};
                if (i < n) v = twisted(c, i);
                if (i + m < n) v = cadd(v, twisted(c, i + m));
                return v;
            };
            if (m == 128) fft_wave_fwd<128>(A, tws, C, L, in);
            else fft_wave_fwd<64>(A, tws, C, L, in);
        } else {
            for (int pass = 0; pass < (n > m ? 2 : 1); ++pass) {
                if (pass) __syncthreads();
                Walk wk(n);
                for (int idx = threadIdx.x; idx < C * n; idx += BT, wk.next())
                    if ((wk.c >= m) == (pass == 1)) {
                        const c32 v = twisted(wk.r, wk.c);
                        const int li = pidx<true>(wk.r * m + (pass ? wk.c - m : wk.c));
                        A[li] = pass ? cadd(A[li], v) : v;
                    }
            }
            dma_rounds(2);
            __syncthreads();
            fft_dif<BT, true>(A, tws, C, bits, L, n < m ? n : m, hook);
        }
        dma_rounds(1 << 20);                     // the rest of this item's spectra
        __builtin_amdgcn_s_waitcnt(WAIT_VM0);   // this wave's direct loads are done
        __syncthreads();                         // ... and every other wave's

        // per-frequency products: one thread per position (in place) for the usual sizes, else
        // task (g, p) gives the x and y outputs of sensor g at position p
        c32 yx[TMAX], yy[TMAX];
        const bool fixed = products_fixed<PACK, HALF>(Ms, A, fac, m, G);
        if (!fixed) {
            Walk wk(m);
            const bool wave_uniform = (m & 63) == 0;   // the 64 tasks of a wave share g
#pragma unroll
            for (int it = 0; it < TMAX; ++it, wk.next()) {
                const int task = threadIdx.x + it * BT;
                yx[it] = yy[it] = c32{0.f, 0.f};
                if (task < m * G) {
                    const int g = wave_uniform ? __builtin_amdgcn_readfirstlane(wk.r) : wk.r;
                    if constexpr (PACK == 0) sensor_products_t<HALF>(Ms, A, m, G, g, wk.c, yx[it], yy[it]);
                    else herm_products_t<HALF>(Ms, A, m, C, g, wk.c, yx[it], yy[it]);
                    if constexpr (HALF == 1) {
                        const float f = fac[wk.c];
                        yx[it] = c32{yx[it].x * f, yx[it].y * f};
                        yy[it] = c32{yy[it].x * f, yy[it].y * f};
                    }
                }
            }
        }
        __syncthreads();   // every read of the spectra, of X and of the input column is done
        if (more) {
            const int fw = (m == 64 || m == 128) ? (C * (m / 8) + 63) / 64 : 0;   // waves of the wave transforms
            dma_begin(sn, coln, hn, fw < BT / 64 ? fw : 0);
            dma_rounds(dw0 ? (1 << 20) : 2);
        }
        if (!fixed) {
            Walk wk(m);
#pragma unroll
            for (int it = 0; it < TMAX; ++it, wk.next()) {
                const int task = threadIdx.x + it * BT;
                if (task < m * G) {
                    const int ix = (2 * wk.r) * m + wk.c;
                    A[pidx<true>(ix)] = yx[it];
                    A[pidx<true>(ix + m)] = yy[it];
                }
            }
            __syncthreads();
        }

        // this item's share of the inverse column transform, rows a < n (V at a mod m, a < n <= 2m)
        c32* Uo = s.U + ((size_t)f2 * S + h) * C * n;
        auto store_u = [&](int c, int a, c32 v) {
            if (h) {
                int hw = h * a;
                if (hw >= L) hw -= L;
                v = cmul(v, tws[hw]);   // w_L^{-h a}
            }
            gstore(Uo + c * n + a, v);
        };
        if (PACK == 0 && (m == 128 || m == 64)) {
            // straight from the transform's registers: entry i gives rows i and i + m
            auto out = [&](int c, int i, c32 v) {
                if (i < n) store_u(c, i, v);
                if (i + m < n) store_u(c, i + m, v);
            };
            if (m == 128) fft_wave_inv<128>(A, tws, C, L, out);
            else fft_wave_inv<64>(A, tws, C, L, out);
            dma_rounds(4);
        } else {
            if (m == 128 || m == 64) {
                if (m == 128) fft_wave_inv<128>(A, tws, C, L, WriteBack{A, 128 + 8});
                else fft_wave_inv<64>(A, tws, C, L, WriteBack{A, 64 + 4});
                dma_rounds(4);
                __syncthreads();
            } else {
                fft_dit_inv<BT, true>(A, tws, C, bits, L, hook);
            }
            Walk wk(n);
            for (int idx = threadIdx.x; idx < C * n; idx += BT, wk.next())
                store_u(wk.r, wk.c, A[pidx<true>(wk.r * m + (wk.c < m ? wk.c : wk.c - m))]);
        }
        dma_rounds(2);
        if (!more) break;
        q = qn;
        col = coln;
        h = hn;
        si = sin_;
        qn = qnn;
        coln = colnn;
        sin_ = sinn;
    }
}

// dst[((f2 P + j) L + r] = src[(f2 L + bitrev(r)) P + j]: one system's spectra
// [Lh][L][P] to the slot-major bit-reversed layout (P = 1: the factors)
template <typename T>
__global__ void k_slot_major(const T* __restrict__ src, T* __restrict__ dst, int Lh, int L, int P, int bits) {
    const long total = (long)Lh * P * L;
    for (long d = blockIdx.x * (long)blockDim.x + threadIdx.x; d < total; d += (long)gridDim.x * blockDim.x) {
        const int r = (int)(d % L);
        const long fj = d / L;
        const int j = (int)(fj % P);
        const long f2 = fj / P;
        dst[d] = src[(f2 * L + bitrev(r, bits)) * P + j];
    }
}

// FP32 spectra rows (one frequency each, P reals) -> FP16 or BF16 storage.
// FP16: each row is multiplied by the power of two 2^(15 - e) that brings its
// largest magnitude m = f 2^e (f in [0.5, 1)) to [2^14, 2^15) and stored with
// the factor 2^(e - 15) that restores it (exact powers of two); every stored
// value is then within u m of the exact one, u = 2^-11.  BF16 keeps the FP32
// exponent range and is stored unscaled (factor 1), u = 2^-8.  Round to nearest
// even.  With ndiag > 0 the row is the general Hermitian packing of a C x C
// positive definite block (the preconditioner, C = ndiag, diagonal in slots
// 0 .. C-1): its diagonal is first raised by d = s m' with s = 1.5 C u and
// m' = m / (1 - s), which exceeds the Frobenius norm (<= sqrt(2) C u m') of the
// rounding error of the raised block, so the stored block is still positive
// definite: the preconditioner stays symmetric positive definite.
__global__ void k_to_half(const float* __restrict__ M, unsigned short* __restrict__ Mh, float* __restrict__ fac,
                          long rows, int P, int kind, int ndiag) {
    const float u = kind == TT_PREC_F16 ? 0x1p-11f : 0x1p-8f;
    for (long r = blockIdx.x; r < rows; r += gridDim.x) {
        const float* src = M + r * P;
        float m = 0.0f;
        for (int i = threadIdx.x; i < P; i += 64) m = fmaxf(m, fabsf(src[i]));
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        float shift = 0.0f;
        if (ndiag > 0) {
            const float sfac = 1.5f * (float)ndiag * u;
            shift = sfac * m / (1.0f - sfac);
            m += shift;
        }
        float up = 1.0f, back = 1.0f;
        if (kind == TT_PREC_F16 && m > 0.0f) {
            int e;
            frexpf(m, &e);
            up = ldexpf(1.0f, 15 - e);
            back = ldexpf(1.0f, e - 15);
        }
        for (int i = threadIdx.x; i < P; i += 64) {
            const float v = (src[i] + (i < ndiag ? shift : 0.0f)) * up;
            unsigned short b;
            if (kind == TT_PREC_F16) {
                b = __builtin_bit_cast(unsigned short, (_Float16)v);
            } else {
                const unsigned uu = __float_as_uint(v);
                b = (unsigned short)((uu + 0x7fffu + ((uu >> 16) & 1u)) >> 16);
            }
            Mh[r * P + i] = b;
        }
        if (threadIdx.x == 0) fac[r] = back;
    }
}

tt_status ensure_half(tt_ctx& c, int op, int kind) {
    if (c.mh_kind[op] == kind) return TT_OK;
    const int P = op ? c.C * c.C : packed_reals(c.G);
    const long rows = (long)c.Lh * c.L;
    TT_CHECK(c.Mh[op].alloc((size_t)rows * P));
    TT_CHECK(c.Mhs[op].alloc((size_t)rows));
    hipLaunchKernelGGL(k_to_half, dim3((unsigned)std::min<long>(rows, 65535)), dim3(64), 0, c.stream,
                       op ? c.Minv32.p : c.M32.p, c.Mh[op].p, c.Mhs[op].p, rows, P, kind, op ? c.C : 0);
    TT_HIP(hipGetLastError());
    c.mh_kind[op] = kind;
    return TT_OK;
}

// The context whose spectra of operator op a context uses: a view reads its
// base's (unless it built its own preconditioner), and so do the copies made
// from them, which are then built once for the base and all its views.
tt_ctx& spectra_owner(tt_ctx& c, int op) {
    tt_ctx* b = c.view_of;
    if (b && (op ? b->Minv32.p == c.Minv32.p : b->M32.p == c.M32.p)) return *b;
    return c;
}

// the slot-major bit-reversed copies read by k_bcolt (power-of-two L), built on first use
tt_status ensure_slot_major(tt_ctx& c, int op, int half_kind) {
    const int P = op ? c.C * c.C : packed_reals(c.G);
    int bits = 0;
    while ((1 << bits) < c.L) ++bits;
    const size_t vals = (size_t)c.Lh * c.L * P;
    const unsigned grid = (unsigned)std::min<size_t>((vals + 255) / 256, 65535);
    if (!half_kind && !c.mt_ready[op]) {
        TT_CHECK(c.Mt32[op].alloc(vals));
        hipLaunchKernelGGL(k_slot_major<float>, dim3(grid), dim3(256), 0, c.stream, op ? c.Minv32.p : c.M32.p,
                           c.Mt32[op].p, c.Lh, c.L, P, bits);
        TT_HIP(hipGetLastError());
        c.mt_ready[op] = true;
    }
    if (half_kind && c.mht_kind[op] != half_kind) {
        TT_CHECK(ensure_half(c, op, half_kind));
        TT_CHECK(c.Mht[op].alloc(vals));
        TT_CHECK(c.Mhst[op].alloc((size_t)c.Lh * c.L));
        hipLaunchKernelGGL(k_slot_major<unsigned short>, dim3(grid), dim3(256), 0, c.stream, c.Mh[op].p, c.Mht[op].p,
                           c.Lh, c.L, P, bits);
        TT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_slot_major<float>, dim3((unsigned)std::min<size_t>((c.Lh * (size_t)c.L + 255) / 256, 65535)),
                           dim3(256), 0, c.stream, c.Mhs[op].p, c.Mhst[op].p, c.Lh, c.L, 1, bits);
        TT_HIP(hipGetLastError());
        c.mht_kind[op] = half_kind;
    }
    return TT_OK;
}

// LDS of one column item past the twiddles: spectra (padded), transform buffer(s)
size_t col_work_lds(int G, int L, int S, int pack) {
    const int m = L / S, C = 2 * G, P = pack ? C * C : 3 * G * G;
    const bool fft = (m & (m - 1)) == 0;
    const size_t ms = (((size_t)m * (P + 1) * sizeof(float)) + 15) & ~size_t(15);
    return ms + (fft ? ((size_t)C * m + (size_t)C * m / 16 + 1) * sizeof(c32) : (size_t)C * m * sizeof(c32) * 2);
}

}  // namespace

// Host side of tt_matvec_batch (see include/tt.h), op 0, and of the batched
// block-circulant preconditioner u = W_s S2 F^-1 (M_+ + sigma^2)^-1 F S1 W_s^T r,
// op 1 (spectra built by precond_build; no noise term).
// Frequency splits S a batch admits: S divides every L, and with S = 4 the
// folded column length L / 4 must reach n / 2 (one fold).
bool split_ok(tt_ctx* const* systems, int count, int S) {
    for (int i = 0; i < count; ++i) {
        const tt_ctx& c = *systems[i];
        if (c.L % S) return false;
        if (S == 4 && 2 * (c.L / 4) < c.n) return false;
    }
    return true;
}

tt_status batch_apply(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y, int op,
                      float* phase_ms, int precision, int S_force, HostMirror<unsigned char>* desc) {
    TT_REQUIRE(count >= 0 && count <= 65535, "count must be in [0, 65535]");
    TT_REQUIRE(precision == TT_PREC_F32 || precision == TT_PREC_F16 || precision == TT_PREC_BF16,
               "spectra precision must be TT_PREC_F32, TT_PREC_F16 or TT_PREC_BF16");
    const int half = precision == TT_PREC_F16 ? 1 : precision == TT_PREC_BF16 ? 2 : 0;
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
        TT_REQUIRE(op == 0 || systems[i]->pc_ready, "preconditioner spectra not built");
    }
    {
        std::vector<const tt_ctx*> sorted(systems, systems + count);
        std::sort(sorted.begin(), sorted.end());
        TT_REQUIRE(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(),
                   "a context appears twice in the batch");
    }
    int S = op ? 4 : 2;
    for (int i = 0; i < count; ++i) {
        if (systems[i]->L % 4) S = std::min(S, 2);
        if (systems[i]->L % 2) S = 1;
    }
    if (S_force) {
        TT_REQUIRE(S_force == 1 || S_force == 2 || S_force == 4, "frequency split must be 1, 2 or 4");
        TT_REQUIRE(split_ok(systems, count, S_force), "frequency split not admitted by the batch");
        S = S_force;
    } else if (c0.tuned_S[op] && c0.tuned_for[op].size() == (size_t)count &&
               std::equal(systems, systems + count, c0.tuned_for[op].begin())) {
        S = c0.tuned_S[op];   // chosen by tt_tune_batch for this batch
    }
    // k_bcolt (spectra slot-major, direct loads to LDS) when every L is a power of
    // two and an item's run of one spectra row is at least 16 bytes; else k_bcol
    const int ebytes = half ? 2 : 4;
    bool slot = true;
    for (int i = 0; i < count; ++i)
        if (!is_pow2(systems[i]->L) || (systems[i]->L / S) * ebytes < 16) slot = false;
    size_t work = 0, a_max = 0, f_max = 0, t_max = 0, m_max = 0;
    int Lmax = 0, fwd_tiles = 0, inv_tiles = 0;
    auto a16 = [](size_t b) { return (b + 15) & ~size_t(15); };
    for (int i = 0; i < count; ++i) {
        const tt_ctx& c = *systems[i];
        TT_REQUIRE((long)(c.L / S) * c.G <= (long)TMAX * BT,
                   "system too large for the batched product: (L / S) * n_gs must be <= " +
                       std::to_string(TMAX * BT));
        const size_t m = (size_t)(c.L / S), P = op ? (size_t)c.C * c.C : (size_t)packed_reals(c.G);
        work = std::max(work, col_work_lds(c.G, c.L, S, op));
        a_max = std::max(a_max, a16(((size_t)c.C * m + (size_t)c.C * m / 16 + 1) * sizeof(c32)));
        f_max = std::max(f_max, half == 1 ? a16(m * sizeof(float)) : size_t(0));
        m_max = std::max(m_max, a16(P * m * ebytes));
        t_max = std::max(t_max, a16((size_t)c.C * c.n * sizeof(c32)));
        Lmax = std::max(Lmax, c.L);
        fwd_tiles = std::max(fwd_tiles, c.C * (int)cdiv(c.n, row_tile_fwd(c.L)));
        inv_tiles = std::max(inv_tiles, c.C * (int)cdiv(c.n, row_tile_inv(c.L)));
    }
    const size_t off_a = a16((size_t)Lmax * sizeof(c32)), off_f = off_a + a_max, off_t = off_f + f_max,
                 off_m = off_t + t_max;
    const size_t lds = slot ? off_m + m_max : off_a + work;
    TT_REQUIRE(lds <= 160 * 1024, "system too large for the batched product: " + std::to_string(lds) +
                                      " bytes of LDS per column item");
    TT_HIP(hipSetDevice(c0.device));

    // descriptors, then the system of every flat column; uploaded only when
    // they differ from the last upload of this first context
    std::vector<BSys> d(count);
    int cols = 0;
    for (int i = 0; i < count; ++i) {
        tt_ctx& c = *systems[i];
        // column shares sized for the largest split, so a later call with another
        // split never moves the buffer a captured launch writes
        const size_t ucount = (size_t)c.Lh * 4 * c.C * c.n;
        if (c.bU32.n < ucount) TT_CHECK(c.bU32.alloc(ucount));
        // the half and slot-major copies are built once, on the owning system's stream; the kernels run on
        // the first one's
        tt_ctx& o = spectra_owner(c, op);
        const bool build = slot ? (half ? o.mht_kind[op] != precision : !o.mt_ready[op])
                                : (half && o.mh_kind[op] != precision);
        if (build) {
            TT_CHECK(slot ? ensure_slot_major(o, op, half ? precision : 0) : ensure_half(o, op, precision));
            if (o.stream != c0.stream) TT_HIP(hipStreamSynchronize(o.stream));
        }
        d[i] = BSys{d_x[i], d_y[i], c.vmap.p, c.tw32.p, c.T32.p, c.bU32.p, op ? c.Minv32.p : c.M32.p,
                    half ? o.Mh[op].p : nullptr, half ? o.Mhs[op].p : nullptr,
                    (slot && !half) ? o.Mt32[op].p : nullptr, (slot && half) ? o.Mht[op].p : nullptr,
                    (slot && half) ? o.Mhst[op].p : nullptr,
                    op ? nullptr : c.noise32.p, (!op && c.has_nxy) ? c.nxy32.p : nullptr, c.n, c.G, c.L, c.n_vs,
                    cols};
        cols += c.Lh;
    }
    const size_t dbytes = ((sizeof(BSys) * (size_t)count) + 15) & ~size_t(15);
    std::vector<unsigned char> hb(dbytes + sizeof(int) * (size_t)cols, 0);
    std::memcpy(hb.data(), d.data(), sizeof(BSys) * (size_t)count);
    {
        int* cs = reinterpret_cast<int*>(hb.data() + dbytes);
        for (int i = 0, k = 0; i < count; ++i)
            for (int f2 = 0; f2 < systems[i]->Lh; ++f2) cs[k++] = i;
    }
    HostMirror<unsigned char>& mir = desc ? *desc : c0.bdesc[op];
    DevBuf<unsigned char>& db = mir.dev;
    std::vector<unsigned char>& dh = mir.host;
    if (db.n < hb.size()) {
        TT_CHECK(db.alloc(hb.size()));
        dh.clear();
    }
    if (dh != hb) {
        dh.swap(hb);
        TT_HIP(hipMemcpyAsync(db.p, dh.data(), dh.size(), hipMemcpyHostToDevice, c0.stream));
    }
    const BSys* dd = reinterpret_cast<const BSys*>(db.p);
    const int* col_sys = reinterpret_cast<const int*>(db.p + dbytes);

    // persistent column items: as many workgroups as fit at once (a multiple of 8);
    // spectra in float4 when every 3 G^2 is a multiple of 4
    bool vec4 = true;
    for (int i = 0; i < count; ++i)
        if (!op && (3 * systems[i]->G * systems[i]->G) % 4) vec4 = false;   // C^2 is always a multiple of 4
    typedef void (*ColKernel)(const BSys*, const int*, int, int, int);
    static const ColKernel table[2][2][3] = {
        {{k_bcol<1, 0, 0>, k_bcol<1, 0, 1>, k_bcol<1, 0, 2>}, {k_bcol<1, 0, 0>, k_bcol<1, 0, 1>, k_bcol<1, 0, 2>}},
        {{k_bcol<4, 0, 0>, k_bcol<4, 0, 1>, k_bcol<4, 0, 2>}, {k_bcol<4, 1, 0>, k_bcol<4, 1, 1>, k_bcol<4, 1, 2>}}};
    typedef void (*SlotKernel)(const BSys*, const int*, int, int, int, int, int, int);
    static const SlotKernel slot_table[2][3] = {{k_bcolt<0, 0>, k_bcolt<0, 1>, k_bcolt<0, 2>},
                                                {k_bcolt<1, 0>, k_bcolt<1, 1>, k_bcolt<1, 2>}};
    const ColKernel kc = table[(op || vec4) ? 1 : 0][op ? 1 : 0][half];
    const SlotKernel ks = slot_table[op ? 1 : 0][half];
    const void* kcol = slot ? (const void*)ks : (const void*)kc;
    TT_HIP(hipFuncSetAttribute(kcol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    TT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kcol, BT, lds));
    const long items = (long)cdiv(cols, 8) * 8 * S;
    const long fit = std::max(8L, (long)std::max(per_cu, 1) * std::max(c0.num_cu, 1) / 8 * 8);
    const unsigned col_grid = (unsigned)std::min(items, fit);
    if (phase_ms && !c0.bev[0])
        for (auto& e : c0.bev) TT_HIP(hipEventCreate(&e));
    if (phase_ms) TT_HIP(hipEventRecord(c0.bev[0], c0.stream));
    hipLaunchKernelGGL(k_brow_fwd, dim3(fwd_tiles, count), dim3(RBT), 0, c0.stream, dd);
    TT_HIP(hipGetLastError());
    if (phase_ms) TT_HIP(hipEventRecord(c0.bev[1], c0.stream));
    if (slot)
        hipLaunchKernelGGL(ks, dim3(col_grid), dim3(BT), lds, c0.stream, dd, col_sys, cols, S, (int)off_a, (int)off_f,
                           (int)off_t, (int)off_m);
    else
        hipLaunchKernelGGL(kc, dim3(col_grid), dim3(BT), lds, c0.stream, dd, col_sys, cols, S, Lmax);
    TT_HIP(hipGetLastError());
    if (phase_ms) TT_HIP(hipEventRecord(c0.bev[2], c0.stream));
    hipLaunchKernelGGL(k_brow_inv, dim3(inv_tiles, count), dim3(RBT), 0, c0.stream, dd, S);
    TT_HIP(hipGetLastError());
    if (phase_ms) {
        TT_HIP(hipEventRecord(c0.bev[3], c0.stream));
        TT_HIP(hipEventSynchronize(c0.bev[3]));
        for (int k = 0; k < 3; ++k) TT_HIP(hipEventElapsedTime(&phase_ms[k], c0.bev[k], c0.bev[k + 1]));
    }
    return TT_OK;
}

// Autotuner of the batched column kernel: times the product (op 0) or the
// block-circulant preconditioner (op 1) of this batch with every frequency
// split S in {1, 2, 4} the batch admits (LDS limits included) on seeded
// vectors, 2 warm-up and 5 timed calls each (HIP events, the three phases
// summed), and keeps the fastest for later calls with exactly these systems in
// this order.  ms[0..2]: mean call time for S = 1, 2, 4 (-1: not admitted).
tt_status tune_batch(tt_ctx* const* systems, int count, int op, int precision, int* best_S, float* ms) {
    TT_REQUIRE(count >= 1 && systems, "NULL or empty batch");
    TT_REQUIRE(op == 0 || op == 1, "op must be 0 (product) or 1 (preconditioner)");
    tt_ctx& c0 = *systems[0];
    TT_HIP(hipSetDevice(c0.device));
    std::vector<DevBuf<float>> xs(count), ys(count);
    std::vector<const float*> px(count);
    std::vector<float*> py(count);
    for (int i = 0; i < count; ++i) {
        TT_REQUIRE(systems[i] && systems[i]->ready, "system without a configured system");
        const size_t n = (size_t)systems[i]->n_slopes;
        TT_CHECK(xs[i].alloc(n));
        TT_CHECK(ys[i].alloc(n));
        std::vector<float> h(n);
        uint32_t st = 0x9E3779B9u ^ (uint32_t)i;
        for (auto& v : h) {   // xorshift32, uniform in [-1, 1)
            st ^= st << 13;
            st ^= st >> 17;
            st ^= st << 5;
            v = (float)((double)st / 2147483648.0 - 1.0);
        }
        TT_HIP(hipMemcpy(xs[i].p, h.data(), n * sizeof(float), hipMemcpyHostToDevice));
        px[i] = xs[i].p;
        py[i] = ys[i].p;
    }
    const int cand[3] = {1, 2, 4};
    int best = 0;
    float best_ms = 0.0f;
    for (int k = 0; k < 3; ++k) {
        float t = -1.0f;
        if (split_ok(systems, count, cand[k])) {
            float ph[3];
            tt_status s = TT_OK;
            for (int r = 0; r < 2 && s == TT_OK; ++r)
                s = batch_apply(systems, count, px.data(), py.data(), op, nullptr, precision, cand[k]);
            double sum = 0.0;
            for (int r = 0; r < 5 && s == TT_OK; ++r) {
                s = batch_apply(systems, count, px.data(), py.data(), op, ph, precision, cand[k]);
                sum += (double)ph[0] + ph[1] + ph[2];
            }
            if (s == TT_OK) t = (float)(sum / 5.0);
            else if (s != TT_INVALID_ARG) return s;   // an LDS or size limit only excludes the candidate
        }
        if (ms) ms[k] = t;
        if (t > 0.0f && (best == 0 || t < best_ms)) {
            best = cand[k];
            best_ms = t;
        }
    }
    TT_REQUIRE(best > 0, "no frequency split fits this batch");
    c0.tuned_S[op] = best;
    c0.tuned_for[op].assign(systems, systems + count);
    if (best_S) *best_S = best;
    return TT_OK;
}

tt_status matvec_batch(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y,
                       float* phase_ms, int precision) {
    return batch_apply(systems, count, d_x, d_y, 0, phase_ms, precision);
}
