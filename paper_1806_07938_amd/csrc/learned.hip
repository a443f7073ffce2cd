// Learned preconditioner (the paper leaves preconditioning of its Toeplitz
// system open, §2.G and the conclusion): P = K^T K, K a four-layer linear
// convolutional network over the C = 2 n_gs slope maps of the n x n
// subaperture grid (3 x 3 kernels, C -> H -> H -> H -> C, zero padding, no
// bias), restricted to the valid subapertures on input and output (§2.F).
// The weights are masked so that K is lower triangular in the order (pixel
// in row-major order, then channel): no tap on the next row or the next pixel
// of the row, and the centre tap W[o][i] only when deg(o) >= deg(i) (input and
// output channel c has degree c, hidden channel h degree h mod C).  The
// diagonal of K is then d = diag(D_4 D_3 D_2 D_1) at every valid subaperture
// (D_l the centre taps) and log|det K| = n_vs sum_c log|d_c|, which makes
// Kaporin's condition number of P A computable:
//   J = N log(t / N) - 2 n_vs sum_c log|d_c|,  t = mean_b (K r_b).(K e_b),
// N = C n_vs, over pairs (r_b = A e_b, e_b ~ N(0, I)): e_b is the exact
// solution of A e = r_b and E[(K r).(K e)] = tr(K A K^T).  Training minimises
// J with Adam on FP32 master weights; the network computes with the weights
// rounded to bfloat16.
//
// Convolutions run on the matrix cores (v_mfma_f32_16x16x16bf16_1k) as
// implicit products: output channels are the M rows, 16 consecutive pixels of
// one grid row the N columns, and K = (tap, input channel) with the channel
// fastest.  The weights are bfloat16 operands; each activation is split into
// two bfloat16 terms (hi = bf16(x), lo = bf16(x - hi), x represented to
// 2^-16 relative), both multiplied, FP32 accumulation.  The adjoint layers
// (K^T and back-propagation) use the same kernel with the flipped, transposed
// weights.  The weight gradient is a reduction over all pixels of the batch:
// FP32 on the vector units, per-workgroup partials summed in a fixed order.
#include "cg_common.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

constexpr int NL = 4;          // layers
constexpr int WGR = 256;       // threads of the weight-gradient and reduction kernels
constexpr int NPART = 256;     // workgroups (partials) of the reductions

__device__ __host__ inline unsigned short bf16_rne(float x) {
    const unsigned u = __builtin_bit_cast(unsigned, x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_to_f32(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

int rup(int a, int b) { return (a + b - 1) / b * b; }

// ---------------------------------------------------------------------------
// convolution: out[b][o][y][x] = sum_{i, ky, kx} W[o][i][ky][kx] in[b][i][y + ky - 1][x + kx - 1]
// W as a bfloat16 operand [16 MT rows][KP], k = (ky 3 + kx) cinp + i, zero padded.
// A block of CR waves covers 16 pixels (x0 .. x0 + 15) of CR consecutive rows
// of map b, one row per wave, all output channels.  The CR + 2 input rows it
// reads (one column of halo on each side) are staged once in LDS as hi / lo
// bfloat16, channel fastest, and so is the weight operand.
// ---------------------------------------------------------------------------
struct ConvArgs {
    const float* in;            // [B][cin][n][n]
    float* out;                 // [B][cout][n][n]
    const unsigned short* w;    // [16 MT][KP]
    const int* vmap;            // n*n valid index or -1 (zero those outputs), or null
    // Optional vector ends of the network (one launch fewer at each end):
    // vin[b] (C n_vs valid slopes, channel-major) replaces in as map b, read
    // through imap (n*n valid index or -1); vout[b] receives the valid outputs
    // of map b in place of out (vmap required).
    const int* imap;
    const float* const* vin;
    float* const* vout;
    int n, cin, cinp, cout, KP, n_vs;
};

constexpr int CMAXP = 32;      // largest padded channel count
constexpr int TW = 18;         // tile width: 16 pixels + halo
constexpr int CR = 4;          // grid rows (waves) per block
constexpr int KPMAX = 9 * CMAXP;
constexpr int NT = 64 * CR;                                   // threads of a convolution block
constexpr int NST = ((CR + 2) * TW * CMAXP + NT - 1) / NT;    // staged inputs per thread
template <int MT>
constexpr int NWV = (16 * MT * KPMAX / 8 + NT - 1) / NT;      // 16-byte weight words per thread

template <int MT, bool VIN>
__global__ __launch_bounds__(64 * CR) void k_conv(ConvArgs a) {
    __shared__ __align__(16) unsigned short th[(CR + 2) * TW * CMAXP];
    __shared__ __align__(16) unsigned short tl[(CR + 2) * TW * CMAXP];
    __shared__ __align__(16) unsigned short ws[16 * MT * KPMAX];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int x0 = blockIdx.x * 16, y0 = blockIdx.y * CR, b = blockIdx.z;
    const int n = a.n, cinp = a.cinp;
    const float* inb = a.in ? a.in + (long)b * a.cin * n * n : nullptr;
    // Every global load of the staging is issued before the first one is
    // used (addresses clamped to the map's first element where the position
    // is padding), so the block waits for one memory round trip, not one per
    // element.
    const int total = (CR + 2) * TW * cinp;
    const int nwv = 16 * MT * a.KP / 8;
    const uint4* wsrc = reinterpret_cast<const uint4*>(a.w);
    float v[NST];
    int kv[NST];
    uint4 wv[NWV<MT>];
#pragma unroll
    for (int j = 0; j < NST; ++j) {
        const int idx = tid + NT * j;
        const int col = idx % TW;
        const int r = (idx / TW) % (CR + 2);
        const int c = idx / ((CR + 2) * TW);
        const int yy = y0 - 1 + r, xx = x0 - 1 + col;
        const bool ok = idx < total && c < a.cin && yy >= 0 && yy < n && xx >= 0 && xx < n;
        if constexpr (VIN) {   // the position's index in the valid-slope vector, or -1
            const int k = a.imap[ok ? yy * n + xx : 0];
            kv[j] = ok && k >= 0 ? c * a.n_vs + k : -1;
        } else {
            const float t = inb[ok ? ((long)c * n + yy) * n + xx : 0];
            v[j] = ok ? t : 0.0f;
        }
    }
#pragma unroll
    for (int j = 0; j < NWV<MT>; ++j) {
        const int i = tid + NT * j;
        wv[j] = wsrc[i < nwv ? i : 0];
    }
    if constexpr (VIN) {
        const float* vb = a.vin[b];
#pragma unroll
        for (int j = 0; j < NST; ++j) {
            const float t = vb[kv[j] >= 0 ? kv[j] : 0];
            v[j] = kv[j] >= 0 ? t : 0.0f;
        }
    }
    // (keeps the weight loads here: otherwise the compiler sinks each into
    // its conditional store below and waits for it there, one at a time)
#pragma unroll
    for (int j = 0; j < NWV<MT>; ++j) asm volatile("" : "+v"(wv[j].x), "+v"(wv[j].y), "+v"(wv[j].z), "+v"(wv[j].w));
#pragma unroll
    for (int j = 0; j < NST; ++j) {
        const int idx = tid + NT * j;
        if (idx < total) {
            const int col = idx % TW;
            const int r = (idx / TW) % (CR + 2);
            const int c = idx / ((CR + 2) * TW);
            const unsigned short hi = bf16_rne(v[j]);
            const unsigned short lo = bf16_rne(v[j] - bf16_to_f32(hi));
            th[(r * TW + col) * cinp + c] = hi;
            tl[(r * TW + col) * cinp + c] = lo;
        }
    }
    {
        uint4* dst = reinterpret_cast<uint4*>(ws);
#pragma unroll
        for (int j = 0; j < NWV<MT>; ++j) {
            const int i = tid + NT * j;
            if (i < nwv) dst[i] = wv[j];
        }
    }
    __syncthreads();
    const int y = y0 + wave;
    if (y >= n) return;
    const int kq = lane >> 4, lc = lane & 15;
    f32x4 acc[MT];
    for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nk = a.KP / 16;
#pragma unroll 3
    for (int s = 0; s < nk; ++s) {
        const int k0 = 16 * s + 4 * kq;
        const int tap = k0 / cinp, c0 = k0 - tap * cinp;
        i16x4 bh = {0, 0, 0, 0}, bl = {0, 0, 0, 0};
        if (tap < 9) {
            const int ky = tap / 3, kx = tap - 3 * ky;
            const int o = ((wave + ky) * TW + lc + kx) * cinp + c0;
            bh = *reinterpret_cast<const i16x4*>(&th[o]);
            bl = *reinterpret_cast<const i16x4*>(&tl[o]);
        }
        for (int m = 0; m < MT; ++m) {
            const i16x4 av = *reinterpret_cast<const i16x4*>(&ws[(16 * m + lc) * a.KP + k0]);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bh, acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bl, acc[m], 0, 0, 0);
        }
    }
    const int x = x0 + lc;
    if (x >= n) return;
    if (a.vout) {
        const int k = a.vmap[y * n + x];
        if (k < 0) return;
        float* vb = a.vout[b];
        for (int m = 0; m < MT; ++m)
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * m + 4 * kq + v;
                if (o < a.cout) vb[(long)o * a.n_vs + k] = acc[m][v];
            }
        return;
    }
    const bool keep = !a.vmap || a.vmap[y * n + x] >= 0;
    float* outb = a.out + (long)b * a.cout * n * n;
    for (int m = 0; m < MT; ++m)
        for (int v = 0; v < 4; ++v) {
            const int o = 16 * m + 4 * kq + v;
            if (o < a.cout) outb[((long)o * n + y) * n + x] = keep ? acc[m][v] : 0.0f;
        }
}

// valid-slope vectors -> maps (zeros at invalid subapertures); map b reads vec[b]
__global__ void k_scatter(const float* const* __restrict__ vec, const int* __restrict__ vmap, float* __restrict__ maps,
                          int C, int n, int n_vs) {
    const int b = blockIdx.y;
    const float* v = vec[b];
    const long per = (long)C * n * n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (long)gridDim.x * blockDim.x) {
        const int pix = (int)(i % (n * n));
        const int c = (int)(i / (n * n));
        const int k = vmap[pix];
        maps[(long)b * per + i] = k >= 0 ? v[(long)c * n_vs + k] : 0.0f;
    }
}

// masked FP32 master weights -> bfloat16 operands of the forward and adjoint
// convolutions of one layer:
//   forward  wf[o][(ky 3 + kx) cinp + i]          = W[o][i][ky][kx]
//   adjoint  wa[i][(ky 3 + kx) coutp + o]         = W[o][i][2 - ky][2 - kx]
__global__ void k_prep_weights(const float* __restrict__ w, const float* __restrict__ mask, unsigned short* wf,
                               unsigned short* wa, int cout, int cin, int cinp, int coutp, int KPf, int KPa,
                               int rowsf, int rowsa) {
    const int tot_f = rowsf * KPf, tot_a = rowsa * KPa;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot_f + tot_a; i += gridDim.x * blockDim.x) {
        if (i < tot_f) {
            const int o = i / KPf, k = i % KPf;
            const int tap = k / cinp, c = k % cinp;
            float v = 0.0f;
            if (o < cout && tap < 9 && c < cin) {
                const int j = ((o * cin + c) * 9) + tap;
                v = w[j] * mask[j];
            }
            wf[i] = bf16_rne(v);
        } else {
            const int ii = i - tot_f;
            const int c = ii / KPa, k = ii % KPa;
            const int tap = k / coutp, o = k % coutp;
            float v = 0.0f;
            if (c < cin && tap < 9 && o < cout) {
                const int j = ((o * cin + c) * 9) + (8 - tap);
                v = w[j] * mask[j];
            }
            wa[ii] = bf16_rne(v);
        }
    }
}

// ---------------------------------------------------------------------------
// training kernels
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = WGR / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// partial sums of sum_b sum_i a[b][i] a[B + b][i] (output maps already masked)
__global__ __launch_bounds__(WGR) void k_pair_dot(const float* __restrict__ h4, long per, int B,
                                                  double* __restrict__ part) {
    __shared__ double red[WGR];
    double v = 0.0;
    const long tot = (long)B * per;
    for (long i = (long)blockIdx.x * WGR + threadIdx.x; i < tot; i += (long)NPART * WGR)
        v += (double)h4[i] * (double)h4[tot + i];
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

struct TrainScalars {
    double t, J, logdet, scale;
    int bad, pad;
};

// t, J, the log-determinant and the upstream scale N / (t B); one block
__global__ __launch_bounds__(WGR) void k_objective(const double* __restrict__ part, const unsigned short* __restrict__ wf,
                                                   int C, int H, int KP0, int KP1, int KP3, int B, int n_vs,
                                                   long woff1, long woff2, long woff3, TrainScalars* S) {
    __shared__ double red[WGR];
    __shared__ double D[32 * 32], T[32 * 32];
    double v = 0.0;
    for (int i = threadIdx.x; i < NPART; i += WGR) v += part[i];
    const double tsum = block_sum(v, red);
    // centre taps (tap 4) of the bfloat16 forward operands, D = D_4 D_3 D_2 D_1
    // layer 0: [H][KP0], cinp = C (C even multiple of 2; padded to 4 below)
    const int cp0 = (C + 3) / 4 * 4;
    const int hp = (H + 3) / 4 * 4;
    for (int i = threadIdx.x; i < H * C; i += WGR) {
        const int o = i / C, c = i % C;
        D[i] = bf16_to_f32(wf[(long)o * KP0 + 4 * cp0 + c]);
    }
    __syncthreads();
    for (int l = 1; l < 3; ++l) {
        const unsigned short* wl = wf + (l == 1 ? woff1 : woff2);
        for (int i = threadIdx.x; i < H * C; i += WGR) {
            const int o = i / C, c = i % C;
            double s = 0.0;
            for (int k = 0; k < H; ++k) s += (double)bf16_to_f32(wl[(long)o * KP1 + 4 * hp + k]) * D[k * C + c];
            T[i] = s;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < H * C; i += WGR) D[i] = T[i];
        __syncthreads();
    }
    double ld = 0.0;
    int bad = 0;
    if (threadIdx.x == 0) {
        const unsigned short* w3 = wf + woff3;
        for (int c = 0; c < C; ++c) {
            double s = 0.0;
            for (int k = 0; k < H; ++k) s += (double)bf16_to_f32(w3[(long)c * KP3 + 4 * hp + k]) * D[k * C + c];
            if (!(s != 0.0) || !isfinite(s)) bad = 1;
            ld += log(fabs(s));
        }
        const double N = (double)C * n_vs;
        const double t = tsum / B;
        if (!(t > 0.0) || !isfinite(t)) bad = 1;
        S->t = t;
        S->logdet = (double)n_vs * ld;
        S->J = N * log(t / N) - 2.0 * (double)n_vs * ld;
        S->scale = N / (t * B);
        S->bad = bad;
    }
}

// upstream gradient of J at the outputs: branch r gets scale * (K e), branch e scale * (K r)
__global__ void k_upstream(const float* __restrict__ h4, float* __restrict__ g4, long per, int B,
                           const TrainScalars* __restrict__ S) {
    const float sc = (float)S->scale;
    const long tot = (long)B * per;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        g4[i] = sc * h4[tot + i];
        g4[tot + i] = sc * h4[i];
    }
}

// weight-gradient partials of one layer: gw[o][i][ky][kx] = sum_{b,y,x} g[b][o][y][x] h[b][i][y+ky-1][x+kx-1]
// over the rows (b, y) of this workgroup (b < nb maps); thread entry (o, i) keeps
// the 9 taps; the rows are staged in LDS (g row, three h rows with halo).
__global__ __launch_bounds__(WGR) void k_wgrad(const float* __restrict__ h, const float* __restrict__ g, int nb, int n,
                                               int cin, int cout, float* __restrict__ part) {
    extern __shared__ float sm[];
    float* gs = sm;                    // [cout][n]
    float* hs = sm + cout * n;         // [cin][3][n + 2]
    const int pairs = cin * cout;   // at most 4 WGR
    float acc[4][9];
    for (int q = 0; q < 4; ++q)
        for (int t = 0; t < 9; ++t) acc[q][t] = 0.0f;
    const int rows = nb * n;
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int b = row / n, y = row % n;
        __syncthreads();
        for (int i = threadIdx.x; i < cout * n; i += WGR) {
            const int o = i / n, x = i % n;
            gs[i] = g[(((long)b * cout + o) * n + y) * n + x];
        }
        for (int i = threadIdx.x; i < cin * 3 * (n + 2); i += WGR) {
            const int xx = i % (n + 2) - 1;
            const int r = (i / (n + 2)) % 3;
            const int c = i / (3 * (n + 2));
            const int yy = y - 1 + r;
            hs[i] = (yy >= 0 && yy < n && xx >= 0 && xx < n) ? h[(((long)b * cin + c) * n + yy) * n + xx] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + q * WGR;
            if (e >= pairs) continue;
            const int o = e / cin, c = e % cin;
            const float* gr = gs + o * n;
            const float* h0 = hs + (c * 3 + 0) * (n + 2);
            const float* h1 = h0 + (n + 2);
            const float* h2 = h1 + (n + 2);
            float a0 = h0[0], a1 = h0[1], b0 = h1[0], b1 = h1[1], d0 = h2[0], d1 = h2[1];
            for (int x = 0; x < n; ++x) {
                const float gv = gr[x];
                const float a2 = h0[x + 2], b2 = h1[x + 2], d2 = h2[x + 2];
                acc[q][0] += gv * a0;
                acc[q][1] += gv * a1;
                acc[q][2] += gv * a2;
                acc[q][3] += gv * b0;
                acc[q][4] += gv * b1;
                acc[q][5] += gv * b2;
                acc[q][6] += gv * d0;
                acc[q][7] += gv * d1;
                acc[q][8] += gv * d2;
                a0 = a1; a1 = a2; b0 = b1; b1 = b2; d0 = d1; d1 = d2;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + q * WGR;
        if (e >= pairs) continue;
        for (int t = 0; t < 9; ++t) part[(long)blockIdx.x * pairs * 9 + (long)e * 9 + t] = acc[q][t];
    }
}

// grad[j] = sum_p part[p][j] (fixed order), masked; then the log-determinant term
__global__ void k_wgrad_reduce(const float* __restrict__ part, int np, int cnt, const float* __restrict__ mask,
                               float* __restrict__ grad) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int p = 0; p < np; ++p) s += part[(long)p * cnt + j];
        grad[j] = (float)(s * mask[j]);
    }
}

// the gradient of -2 n_vs sum_c log|d_c| w.r.t. the centre taps:
// -2 n_vs (D_4..D_{l+1})^T diag(1/d) (D_{l-1}..D_1)^T, added to the centre tap
// entries of grad (masked).  One block; matrices from the bfloat16 weights.
__global__ __launch_bounds__(WGR) void k_logdet_grad(const float* __restrict__ w, const float* __restrict__ mask,
                                                     float* __restrict__ grad, int C, int H, int n_vs, long o1,
                                                     long o2, long o3) {
    __shared__ double Dl[4][32 * 32];   // centre taps of each layer (bf16 values), [out][in]
    __shared__ double P[32 * 32], Q[32 * 32], T[32 * 32];
    __shared__ double dinv[32];
    const int co[4] = {H, H, H, C}, ci[4] = {C, H, H, H};
    const long off[4] = {0, o1, o2, o3};
    for (int l = 0; l < 4; ++l)
        for (int i = threadIdx.x; i < co[l] * ci[l]; i += WGR) {
            const long j = off[l] + (long)i * 9 + 4;
            Dl[l][i] = (double)bf16_to_f32(bf16_rne(w[j] * mask[j]));
        }
    __syncthreads();
    // d = diag(D3 D2 D1 D0): T = D0 (H x C), then left products
    for (int i = threadIdx.x; i < H * C; i += WGR) T[i] = Dl[0][i];
    __syncthreads();
    for (int l = 1; l < 3; ++l) {
        for (int i = threadIdx.x; i < H * C; i += WGR) {
            const int o = i / C, c = i % C;
            double s = 0.0;
            for (int k = 0; k < H; ++k) s += Dl[l][o * H + k] * T[k * C + c];
            P[i] = s;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < H * C; i += WGR) T[i] = P[i];
        __syncthreads();
    }
    for (int c = threadIdx.x; c < C; c += WGR) {
        double s = 0.0;
        for (int k = 0; k < H; ++k) s += Dl[3][c * H + k] * T[k * C + c];
        dinv[c] = 1.0 / s;
    }
    __syncthreads();
    for (int l = 0; l < 4; ++l) {
        // above = D_3 .. D_{l+1} (C x co[l]); below = D_{l-1} .. D_0 (ci[l] x C)
        // P <- above (starts as the C x C identity), Q <- below (likewise)
        for (int i = threadIdx.x; i < C * C; i += WGR) P[i] = (i / C == i % C) ? 1.0 : 0.0;
        __syncthreads();
        for (int k2 = 3; k2 > l; --k2) {
            // T = P (C x co[k2]) D_k2 (co[k2] x ci[k2])
            for (int i = threadIdx.x; i < C * ci[k2]; i += WGR) {
                const int r = i / ci[k2], c = i % ci[k2];
                double s = 0.0;
                for (int k = 0; k < co[k2]; ++k) s += P[r * co[k2] + k] * Dl[k2][k * ci[k2] + c];
                T[i] = s;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < C * ci[k2]; i += WGR) P[i] = T[i];
            __syncthreads();
        }
        // now P = D_3 .. D_{l+1} as C x co[l] (ci[l+1] = co[l])
        for (int i = threadIdx.x; i < C * C; i += WGR) Q[i] = (i / C == i % C) ? 1.0 : 0.0;
        __syncthreads();
        for (int k2 = 0; k2 < l; ++k2) {
            for (int i = threadIdx.x; i < co[k2] * C; i += WGR) {
                const int r = i / C, c = i % C;
                double s = 0.0;
                for (int k = 0; k < ci[k2]; ++k) s += Dl[k2][r * ci[k2] + k] * Q[k * C + c];
                T[i] = s;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < co[k2] * C; i += WGR) Q[i] = T[i];
            __syncthreads();
        }
        // grad centre of layer l [a][b] += -2 n_vs sum_c P[c][a] dinv[c] Q[b][c]
        for (int i = threadIdx.x; i < co[l] * ci[l]; i += WGR) {
            const int a = i / ci[l], b = i % ci[l];
            double s = 0.0;
            for (int c = 0; c < C; ++c) s += P[c * co[l] + a] * dinv[c] * Q[b * C + c];
            const long j = off[l] + (long)i * 9 + 4;
            grad[j] += (float)(-2.0 * n_vs * s * mask[j]);
        }
        __syncthreads();
    }
}

// Adam (Kingma & Ba, Algorithm 1), masked; lr already includes the schedule
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, const float* __restrict__ mask, int cnt, float lr, float bc1,
                       float bc2, const TrainScalars* __restrict__ S) {
    if (S->bad) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += gridDim.x * blockDim.x) {
        const float gj = g[j];
        const float mj = 0.9f * m[j] + 0.1f * gj;
        const float vj = 0.999f * v[j] + 0.001f * gj * gj;
        m[j] = mj;
        v[j] = vj;
        const float upd = lr * (mj / bc1) / (sqrtf(vj / bc2) + 1e-8f);
        w[j] = (w[j] - upd) * mask[j];
    }
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals
// ---------------------------------------------------------------------------
struct u4 { unsigned x, y, z, w; };
__device__ __host__ inline u4 philox(u4 c, unsigned k0, unsigned k1) {
    const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)M0 * c.x;
        const unsigned long long p1 = (unsigned long long)M1 * c.z;
        const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
        const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
        c = u4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// e[i] ~ N(0, 1): counter (i / 4, stream, 0, 0) under the key (seed), Box-Muller on two words
__global__ void k_normal(float* __restrict__ e, long cnt, unsigned stream, unsigned k0, unsigned k1) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (cnt + 1) / 2;
         i += (long)gridDim.x * blockDim.x) {
        const u4 r = philox(u4{(unsigned)i, (unsigned)(i >> 32), stream, 0x4e4f524du}, k0, k1);
        const float u1 = ((float)(r.x >> 8) + 1.0f) * (1.0f / 16777216.0f);   // (0, 1]
        const float u2 = (float)(r.y >> 8) * (1.0f / 16777216.0f);            // [0, 1)
        const float rad = sqrtf(-2.0f * logf(u1));
        float s, c;
        sincosf(6.283185307179586f * u2, &s, &c);
        e[2 * i] = rad * c;
        if (2 * i + 1 < cnt) e[2 * i + 1] = rad * s;
    }
}

// batch b draws pair index hash(step, b) mod npairs; pointers to its r and e
__global__ void k_pick(const float* const* __restrict__ R, const float* const* __restrict__ E, int npairs, int B,
                       unsigned step, unsigned k0, unsigned k1, float** __restrict__ sel) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const u4 r = philox(u4{step, (unsigned)b, 0x50494b43u, 0u}, k0, k1);
    const int j = (int)(((unsigned long long)r.x * (unsigned)npairs) >> 32);
    sel[b] = const_cast<float*>(R[j]);
    sel[B + b] = const_cast<float*>(E[j]);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct tt_learned {
    int device = 0;
    int C = 0, H = 0;
    int cin[NL], cout[NL], cinp[NL], coutp[NL], KPf[NL], KPa[NL], rowsf[NL], rowsa[NL];
    long woff[NL + 1];          // FP32 weights [o][i][3][3] of the layers, concatenated
    long wfoff[NL + 1];         // bfloat16 forward operands
    long waoff[NL + 1];         // bfloat16 adjoint operands
    DevBuf<float> w, mask, am, av, grad;
    DevBuf<unsigned short> wf, wa;
    int step = 0;
    unsigned long long seed = 0;
    // work buffers (grown on demand)
    DevBuf<float> maps;         // activations and gradients
    DevBuf<float> wpart;        // weight-gradient partials
    DevBuf<double> dpart;
    DevBuf<TrainScalars> ts;
    DevBuf<float*> ptrs;            // pointer tables of the batched vectors
    std::vector<float*> ptrs_host;  // what ptrs holds (an application re-uploads only on change)
    hipStream_t stream = nullptr;
};

namespace {

std::vector<float> host_masks(const tt_learned& L) {
    std::vector<float> m((size_t)L.woff[NL], 0.0f);
    for (int l = 0; l < NL; ++l) {
        const int co = L.cout[l], ci = L.cin[l];
        auto deg_in = [&](int c) { return l == 0 ? c : c % L.C; };
        auto deg_out = [&](int o) { return l == NL - 1 ? o : o % L.C; };
        for (int o = 0; o < co; ++o)
            for (int c = 0; c < ci; ++c)
                for (int t = 0; t < 9; ++t) {
                    const int ky = t / 3, kx = t % 3;
                    float v = 1.0f;
                    if (ky == 2 || (ky == 1 && kx == 2)) v = 0.0f;
                    if (ky == 1 && kx == 1) v = deg_out(o) >= deg_in(c) ? 1.0f : 0.0f;
                    m[(size_t)L.woff[l] + ((size_t)o * ci + c) * 9 + t] = v;
                }
    }
    return m;
}

tt_status prep_weights(tt_learned& L, hipStream_t s) {
    for (int l = 0; l < NL; ++l) {
        const int tot = L.rowsf[l] * L.KPf[l] + L.rowsa[l] * L.KPa[l];
        hipLaunchKernelGGL(k_prep_weights, dim3(cdiv(tot, 256)), dim3(256), 0, s, L.w.p + L.woff[l],
                           L.mask.p + L.woff[l], L.wf.p + L.wfoff[l], L.wa.p + L.waoff[l], L.cout[l], L.cin[l],
                           L.cinp[l], L.coutp[l], L.KPf[l], L.KPa[l], L.rowsf[l], L.rowsa[l]);
    }
    TT_HIP(hipGetLastError());
    return TT_OK;
}

// out = conv(in) with layer l's forward (adj = false) or adjoint operand, B maps
tt_status conv(const tt_learned& L, int l, bool adj, const float* in, float* out, int B, int n, const int* vmap,
               hipStream_t s, const int* imap = nullptr, const float* const* vin = nullptr,
               float* const* vout = nullptr, int n_vs = 0) {
    ConvArgs a;
    a.in = in;
    a.out = out;
    a.vmap = vmap;
    a.imap = imap;
    a.vin = vin;
    a.vout = vout;
    a.n_vs = n_vs;
    a.n = n;
    if (!adj) {
        a.w = L.wf.p + L.wfoff[l];
        a.cin = L.cin[l];
        a.cinp = L.cinp[l];
        a.cout = L.cout[l];
        a.KP = L.KPf[l];
    } else {
        a.w = L.wa.p + L.waoff[l];
        a.cin = L.cout[l];
        a.cinp = L.coutp[l];
        a.cout = L.cin[l];
        a.KP = L.KPa[l];
    }
    if (a.KP > KPMAX || a.cinp > CMAXP) {
        tt_set_error("convolution layer too wide");
        return TT_INVALID_ARG;
    }
    const dim3 grid(cdiv(n, 16), cdiv(n, CR), B);
    if (a.cout <= 16) {
        if (vin)
            hipLaunchKernelGGL((k_conv<1, true>), grid, dim3(64 * CR), 0, s, a);
        else
            hipLaunchKernelGGL((k_conv<1, false>), grid, dim3(64 * CR), 0, s, a);
    } else {
        if (vin)
            hipLaunchKernelGGL((k_conv<2, true>), grid, dim3(64 * CR), 0, s, a);
        else
            hipLaunchKernelGGL((k_conv<2, false>), grid, dim3(64 * CR), 0, s, a);
    }
    TT_HIP(hipGetLastError());
    return TT_OK;
}

tt_status grow(DevBuf<float>& b, size_t n) { return b.n >= n ? TT_OK : b.alloc(n); }

}  // namespace

// Work-buffer need of an application to B maps of n x n.
static size_t apply_floats(const tt_learned& L, int B, int n) { return (size_t)2 * B * std::max(L.C, L.H) * n * n; }

// z_b = K^T K r_b for B vectors of one geometry (vmap / vidx of ctx), on stream s.
tt_status learned_apply_batch(tt_learned& L, const tt_ctx& c, const float* const* d_r, float* const* d_z, int B,
                              hipStream_t s, HostMirror<float*>* table) {
    TT_REQUIRE(c.C == L.C, "the network's channel count differs from the system's 2 n_gs");
    TT_CHECK(grow(L.maps, apply_floats(L, B, c.n)));
    DevBuf<float*>& tdev = table ? table->dev : L.ptrs;
    std::vector<float*>& thost = table ? table->host : L.ptrs_host;
    if (tdev.n < (size_t)(2 * B + 2)) {
        TT_CHECK(tdev.alloc((size_t)2 * B + 2));
        thost.clear();
    }
    const int n = c.n;
    const size_t half = (size_t)B * std::max(L.C, L.H) * n * n;
    float* m0 = L.maps.p;
    float* m1 = L.maps.p + half;
    std::vector<float*> hp(2 * B);
    for (int b = 0; b < B; ++b) {
        hp[b] = const_cast<float*>(d_r[b]);
        hp[B + b] = d_z[b];
    }
    if (hp != thost) {
        thost = hp;
        TT_HIP(hipMemcpyAsync(tdev.p, thost.data(), sizeof(float*) * 2 * B, hipMemcpyHostToDevice, s));
    }
    // the first layer reads the vectors through the valid map, the last one
    // writes the valid outputs to the vectors
    TT_CHECK(conv(L, 0, false, nullptr, m1, B, n, nullptr, s, c.vmap.p, tdev.p, nullptr, c.n_vs));
    TT_CHECK(conv(L, 1, false, m1, m0, B, n, nullptr, s));
    TT_CHECK(conv(L, 2, false, m0, m1, B, n, nullptr, s));
    TT_CHECK(conv(L, 3, false, m1, m0, B, n, c.vmap.p, s));   // K r on the valid subapertures
    TT_CHECK(conv(L, 3, true, m0, m1, B, n, nullptr, s));
    TT_CHECK(conv(L, 2, true, m1, m0, B, n, nullptr, s));
    TT_CHECK(conv(L, 1, true, m0, m1, B, n, nullptr, s));
    TT_CHECK(conv(L, 0, true, m1, nullptr, B, n, c.vmap.p, s, nullptr, nullptr, tdev.p + B, c.n_vs));
    return TT_OK;
}

namespace {

// One training step on B pairs given by device pointers sel[0..B) (r) and
// sel[B..2B) (e), geometry of ctx; lr is this step's rate.  Leaves the
// scalars of the step in L.ts.
tt_status train_step_ptrs(tt_learned& L, const tt_ctx& c, int B, float lr, hipStream_t s) {
    const int n = c.n, C = L.C, H = L.H;
    const long npix = (long)n * n;
    // layout: x0 [2B][C], h1..h3 [2B][H], h4 [2B][C], g4 [2B][C], g3..g1 [2B][H]
    const size_t szC = (size_t)2 * B * C * npix, szH = (size_t)2 * B * H * npix;
    TT_CHECK(grow(L.maps, 3 * szC + 6 * szH));
    float* x0 = L.maps.p;
    float* h1 = x0 + szC;
    float* h2 = h1 + szH;
    float* h3 = h2 + szH;
    float* h4 = h3 + szH;
    float* g4 = h4 + szC;
    float* g3 = g4 + szC;
    float* g2 = g3 + szH;
    float* g1 = g2 + szH;
    const unsigned gx = std::min<unsigned>(cdiv((size_t)C * npix, 256), 1024);
    hipLaunchKernelGGL(k_scatter, dim3(gx, 2 * B), dim3(256), 0, s, L.ptrs.p, c.vmap.p, x0, C, n, c.n_vs);
    TT_HIP(hipGetLastError());
    TT_CHECK(conv(L, 0, false, x0, h1, 2 * B, n, nullptr, s));
    TT_CHECK(conv(L, 1, false, h1, h2, 2 * B, n, nullptr, s));
    TT_CHECK(conv(L, 2, false, h2, h3, 2 * B, n, nullptr, s));
    TT_CHECK(conv(L, 3, false, h3, h4, 2 * B, n, c.vmap.p, s));
    if (L.dpart.n < NPART) TT_CHECK(L.dpart.alloc(NPART));
    if (L.ts.n < 1) TT_CHECK(L.ts.alloc(1));
    const long per = (long)C * npix;
    hipLaunchKernelGGL(k_pair_dot, dim3(NPART), dim3(WGR), 0, s, h4, per, B, L.dpart.p);
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(WGR), 0, s, L.dpart.p, L.wf.p, C, H, L.KPf[0], L.KPf[1], L.KPf[3],
                       B, c.n_vs, L.wfoff[1], L.wfoff[2], L.wfoff[3], L.ts.p);
    hipLaunchKernelGGL(k_upstream, dim3(std::min<unsigned>(cdiv((size_t)B * per, 256), 2048)), dim3(256), 0, s, h4,
                       g4, per, B, L.ts.p);
    TT_HIP(hipGetLastError());
    TT_CHECK(conv(L, 3, true, g4, g3, 2 * B, n, nullptr, s));
    TT_CHECK(conv(L, 2, true, g3, g2, 2 * B, n, nullptr, s));
    TT_CHECK(conv(L, 1, true, g2, g1, 2 * B, n, nullptr, s));
    // weight gradients of the four layers
    const float* hin[NL] = {x0, h1, h2, h3};
    const float* gout[NL] = {g1, g2, g3, g4};
    size_t maxcnt = 0;
    for (int l = 0; l < NL; ++l) maxcnt = std::max(maxcnt, (size_t)(L.woff[l + 1] - L.woff[l]));
    const int nparts = NPART;
    TT_CHECK(grow(L.wpart, maxcnt * nparts));
    for (int l = 0; l < NL; ++l) {
        const int ci = L.cin[l], co = L.cout[l];
        const size_t lds = sizeof(float) * ((size_t)co * n + (size_t)ci * 3 * (n + 2));
        TT_REQUIRE(lds <= 64 * 1024, "grid too large for the weight-gradient kernel");
        TT_REQUIRE(ci * co <= 4 * WGR, "layer too wide for the weight-gradient kernel");
        hipLaunchKernelGGL(k_wgrad, dim3(nparts), dim3(WGR), lds, s, hin[l], gout[l], 2 * B, n, ci, co, L.wpart.p);
        const int cnt = (int)(L.woff[l + 1] - L.woff[l]);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(cdiv(cnt, 256)), dim3(256), 0, s, L.wpart.p, nparts, cnt,
                           L.mask.p + L.woff[l], L.grad.p + L.woff[l]);
    }
    hipLaunchKernelGGL(k_logdet_grad, dim3(1), dim3(WGR), 0, s, L.w.p, L.mask.p, L.grad.p, C, H, c.n_vs, L.woff[1],
                       L.woff[2], L.woff[3]);
    L.step++;
    const float bc1 = 1.0f - powf(0.9f, (float)L.step), bc2 = 1.0f - powf(0.999f, (float)L.step);
    const int nw = (int)L.woff[NL];
    hipLaunchKernelGGL(k_adam, dim3(cdiv(nw, 256)), dim3(256), 0, s, L.w.p, L.am.p, L.av.p, L.grad.p, L.mask.p, nw,
                       lr, bc1, bc2, L.ts.p);
    TT_HIP(hipGetLastError());
    return prep_weights(L, s);
}

tt_status require_dev(int dev) {
    TT_HIP(hipSetDevice(dev));
    return TT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
tt_status learned_create(tt_learned** out, int device, int n_gs, int hidden, unsigned long long seed) {
    TT_REQUIRE(out, "out is NULL");
    *out = nullptr;
    TT_REQUIRE(n_gs >= 1 && n_gs <= 16, "n_gs must be in [1, 16]");
    TT_REQUIRE(hidden >= 2 * n_gs && hidden <= 32 && hidden % 4 == 0,
               "hidden must be a multiple of 4 in [2 n_gs, 32]");
    int ndev = 0;
    TT_HIP(hipGetDeviceCount(&ndev));
    TT_REQUIRE(device >= 0 && device < ndev, "device index out of range");
    TT_CHECK(require_dev(device));
    tt_learned* L = new tt_learned();
    L->device = device;
    L->C = 2 * n_gs;
    L->H = hidden;
    L->seed = seed;
    const int ins[NL] = {L->C, L->H, L->H, L->H}, outs[NL] = {L->H, L->H, L->H, L->C};
    L->woff[0] = L->wfoff[0] = L->waoff[0] = 0;
    for (int l = 0; l < NL; ++l) {
        L->cin[l] = ins[l];
        L->cout[l] = outs[l];
        L->cinp[l] = rup(ins[l], 4);
        L->coutp[l] = rup(outs[l], 4);
        L->KPf[l] = rup(9 * L->cinp[l], 16);
        L->KPa[l] = rup(9 * L->coutp[l], 16);
        L->rowsf[l] = rup(outs[l], 16);
        L->rowsa[l] = rup(ins[l], 16);
        L->woff[l + 1] = L->woff[l] + (long)outs[l] * ins[l] * 9;
        L->wfoff[l + 1] = L->wfoff[l] + (long)L->rowsf[l] * L->KPf[l];
        L->waoff[l + 1] = L->waoff[l] + (long)L->rowsa[l] * L->KPa[l];
    }
    const size_t nw = (size_t)L->woff[NL];
    tt_status st = TT_OK;
    if ((st = L->w.alloc(nw)) != TT_OK || (st = L->mask.alloc(nw)) != TT_OK || (st = L->am.alloc(nw)) != TT_OK ||
        (st = L->av.alloc(nw)) != TT_OK || (st = L->grad.alloc(nw)) != TT_OK ||
        (st = L->wf.alloc((size_t)L->wfoff[NL])) != TT_OK || (st = L->wa.alloc((size_t)L->waoff[NL])) != TT_OK) {
        delete L;
        return st;
    }
    // initial weights: identity-like centre taps (hidden channel h and output c
    // carry input channel h mod C, so K = I) plus small seeded noise
    std::vector<float> m = host_masks(*L);
    std::vector<float> w(nw, 0.0f);
    for (int l = 0; l < NL; ++l) {
        const int co = L->cout[l], ci = L->cin[l];
        const float sd = 0.1f / std::sqrt(9.0f * ci);
        for (int o = 0; o < co; ++o)
            for (int c = 0; c < ci; ++c)
                for (int t = 0; t < 9; ++t) {
                    const size_t j = (size_t)L->woff[l] + ((size_t)o * ci + c) * 9 + t;
                    const u4 r = philox(u4{(unsigned)j, (unsigned)l, 0x494e4954u, 0u}, (unsigned)seed,
                                        (unsigned)(seed >> 32));
                    const float u1 = ((float)(r.x >> 8) + 1.0f) * (1.0f / 16777216.0f);
                    const float u2 = (float)(r.y >> 8) * (1.0f / 16777216.0f);
                    float v = sd * std::sqrt(-2.0f * std::log(u1)) * std::cos(6.283185307179586f * u2);
                    bool eye;
                    if (l == 0) eye = (o % L->C) == c && o < L->C;
                    else if (l == NL - 1) eye = o == c;
                    else eye = o == c;
                    if (t == 4 && eye) v += 1.0f;
                    w[j] = v * m[j];
                }
    }
    hipStream_t s = nullptr;
    std::vector<float> zero(nw, 0.0f);
    if (hipMemcpy(L->w.p, w.data(), nw * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L->mask.p, m.data(), nw * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L->am.p, zero.data(), nw * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L->av.p, zero.data(), nw * 4, hipMemcpyHostToDevice) != hipSuccess) {
        delete L;
        tt_set_error("tt_learned_create: weight upload failed");
        return TT_HIP_ERROR;
    }
    if ((st = prep_weights(*L, s)) != TT_OK || hipDeviceSynchronize() != hipSuccess) {
        delete L;
        return st == TT_OK ? TT_HIP_ERROR : st;
    }
    *out = L;
    return TT_OK;
}

tt_status learned_destroy(tt_learned* L) {
    if (!L) return TT_OK;
    (void)hipSetDevice(L->device);
    (void)hipDeviceSynchronize();
    delete L;
    return TT_OK;
}

int learned_channels(const tt_learned* L) { return L ? L->C : 0; }

size_t learned_weight_count(const tt_learned* L) { return L ? (size_t)L->woff[NL] : 0; }

tt_status learned_get_weights(const tt_learned* L, float* host, size_t count) {
    TT_REQUIRE(L && host, "NULL argument");
    TT_REQUIRE(count == (size_t)L->woff[NL], "count must equal the network's weight count");
    TT_CHECK(require_dev(L->device));
    TT_HIP(hipDeviceSynchronize());
    TT_HIP(hipMemcpy(host, L->w.p, count * sizeof(float), hipMemcpyDeviceToHost));
    return TT_OK;
}

tt_status learned_set_weights(tt_learned* L, const float* host, size_t count) {
    TT_REQUIRE(L && host, "NULL argument");
    TT_REQUIRE(count == (size_t)L->woff[NL], "count must equal the network's weight count");
    TT_CHECK(require_dev(L->device));
    std::vector<float> m = host_masks(*L);
    std::vector<float> w(host, host + count);
    for (size_t j = 0; j < count; ++j) {
        TT_REQUIRE(std::isfinite(w[j]), "non-finite weight");
        w[j] *= m[j];
    }
    TT_HIP(hipDeviceSynchronize());
    TT_HIP(hipMemcpy(L->w.p, w.data(), count * 4, hipMemcpyHostToDevice));
    std::vector<float> zero(count, 0.0f);
    TT_HIP(hipMemcpy(L->am.p, zero.data(), count * 4, hipMemcpyHostToDevice));
    TT_HIP(hipMemcpy(L->av.p, zero.data(), count * 4, hipMemcpyHostToDevice));
    L->step = 0;
    TT_CHECK(prep_weights(*L, nullptr));
    TT_HIP(hipDeviceSynchronize());
    return TT_OK;
}

tt_status learned_apply(tt_learned* L, tt_ctx* c, const float* d_r, float* d_z) {
    TT_REQUIRE(L && c && d_r && d_z, "NULL argument");
    TT_REQUIRE(d_r != d_z, "d_r and d_z must not alias");
    if (!c->ready) {
        tt_set_error("tt_learned_apply: no system set");
        return TT_NOT_READY;
    }
    TT_REQUIRE(c->device == L->device, "network and context on different devices");
    TT_CHECK(require_dev(c->device));
    const float* r[1] = {d_r};
    float* z[1] = {d_z};
    return learned_apply_batch(*L, *c, r, z, 1, c->stream);
}

// One training step on caller pairs (device arrays R, E: batch x n_slopes,
// row-major); J, t at the weights used (host, after a wait).
tt_status learned_train_step(tt_learned* L, tt_ctx* c, const float* d_R, const float* d_E, int batch, double lr,
                             double* J, double* t) {
    TT_REQUIRE(L && c && d_R && d_E, "NULL argument");
    TT_REQUIRE(batch >= 1 && batch <= 4096, "batch must be in [1, 4096]");
    TT_REQUIRE(lr > 0 && std::isfinite(lr), "lr must be positive");
    if (!c->ready) {
        tt_set_error("tt_learned_train_step: no system set");
        return TT_NOT_READY;
    }
    TT_REQUIRE(c->C == L->C, "the network's channel count differs from the system's 2 n_gs");
    TT_REQUIRE(c->device == L->device, "network and context on different devices");
    TT_CHECK(require_dev(c->device));
    const hipStream_t s = c->stream;
    if (L->ptrs.n < (size_t)(2 * batch)) TT_CHECK(L->ptrs.alloc((size_t)2 * batch));
    L->ptrs_host.clear();
    std::vector<float*> hp(2 * batch);
    for (int b = 0; b < batch; ++b) {
        hp[b] = const_cast<float*>(d_R + (size_t)b * c->n_slopes);
        hp[batch + b] = const_cast<float*>(d_E + (size_t)b * c->n_slopes);
    }
    L->ptrs_host = hp;
    TT_HIP(hipMemcpyAsync(L->ptrs.p, L->ptrs_host.data(), sizeof(float*) * 2 * batch, hipMemcpyHostToDevice, s));
    TT_CHECK(train_step_ptrs(*L, *c, batch, (float)lr, s));
    TrainScalars h{};
    TT_HIP(hipMemcpyAsync(&h, L->ts.p, sizeof(h), hipMemcpyDeviceToHost, s));
    TT_HIP(hipStreamSynchronize(s));
    if (J) *J = h.J;
    if (t) *t = h.t;
    if (h.bad) {
        tt_set_error("tt_learned_train_step: non-positive trace estimate or a zero diagonal of K; step skipped");
        return TT_BREAKDOWN;
    }
    return TT_OK;
}

// Training on pairs drawn by the library: n_pairs vectors e ~ N(0, I) (Philox
// under the network's seed), spread over the systems in turn, r = A_j e by the
// FP32 product of system j; steps Adam steps on batches of `batch` pairs chosen
// by a counter-based hash, step size lr with cosine decay to lr / 100.
tt_status learned_train(tt_learned* L, tt_ctx* const* systems, int count, int n_pairs, int steps, int batch,
                        double lr, double* J_first, double* J_last, double* ms) {
    TT_REQUIRE(L && systems, "NULL argument");
    TT_REQUIRE(count >= 1 && count <= 1024, "count must be in [1, 1024]");
    TT_REQUIRE(n_pairs >= count && n_pairs <= 1 << 22, "n_pairs must be in [count, 2^22]");
    TT_REQUIRE(steps >= 1 && batch >= 1 && batch <= 4096, "steps >= 1 and batch in [1, 4096]");
    TT_REQUIRE(lr > 0 && std::isfinite(lr), "lr must be positive");
    const tt_ctx& c0 = *systems[0];
    for (int i = 0; i < count; ++i) {
        TT_REQUIRE(systems[i], "NULL system");
        const tt_ctx& c = *systems[i];
        if (!c.ready) {
            tt_set_error("tt_learned_train: no system set on context " + std::to_string(i));
            return TT_NOT_READY;
        }
        TT_REQUIRE(c.device == L->device, "network and contexts on different devices");
        TT_REQUIRE(c.C == L->C, "the network's channel count differs from a system's 2 n_gs");
        TT_REQUIRE(c.n == c0.n && c.n_vs == c0.n_vs, "all systems must share the grid and the valid subapertures");
        TT_REQUIRE(!c.modes, "mode removal is not supported");
    }
    {
        std::vector<int> v0(c0.n * c0.n), v(c0.n * c0.n);
        TT_CHECK(require_dev(c0.device));
        TT_HIP(hipMemcpy(v0.data(), c0.vmap.p, v0.size() * sizeof(int), hipMemcpyDeviceToHost));
        for (int i = 1; i < count; ++i) {
            TT_HIP(hipMemcpy(v.data(), systems[i]->vmap.p, v.size() * sizeof(int), hipMemcpyDeviceToHost));
            TT_REQUIRE(v == v0, "all systems must share the valid subapertures");
        }
    }
    const hipStream_t s = c0.stream;
    for (int i = 0; i < count; ++i) TT_HIP(hipStreamSynchronize(systems[i]->stream));
    const size_t N = (size_t)c0.n_slopes;
    DevBuf<float> E, R;
    TT_CHECK(E.alloc(N * (size_t)n_pairs));
    TT_CHECK(R.alloc(N * (size_t)n_pairs));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TT_HIP(hipEventCreate(&e0));
    TT_HIP(hipEventCreate(&e1));
    TT_HIP(hipEventRecord(e0, s));
    const unsigned k0 = (unsigned)L->seed, k1 = (unsigned)(L->seed >> 32);
    hipLaunchKernelGGL(k_normal, dim3(4096), dim3(256), 0, s, E.p, (long)(N * (size_t)n_pairs), 0x50414952u, k0, k1);
    TT_HIP(hipGetLastError());
    TT_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < n_pairs; ++p) {
        tt_ctx& c = *systems[p % count];
        TT_CHECK(matvec_f32(c, E.p + (size_t)p * N, R.p + (size_t)p * N, nullptr));
        if (c.stream != s && (p % count) == count - 1) TT_HIP(hipStreamSynchronize(c.stream));
    }
    for (int i = 0; i < count; ++i) TT_HIP(hipStreamSynchronize(systems[i]->stream));
    // pair pointer tables for the sampler
    DevBuf<const float*> tabR, tabE;
    TT_CHECK(tabR.alloc((size_t)n_pairs));
    TT_CHECK(tabE.alloc((size_t)n_pairs));
    {
        std::vector<const float*> hr(n_pairs), he(n_pairs);
        for (int p = 0; p < n_pairs; ++p) {
            hr[p] = R.p + (size_t)p * N;
            he[p] = E.p + (size_t)p * N;
        }
        TT_HIP(hipMemcpy(tabR.p, hr.data(), sizeof(float*) * n_pairs, hipMemcpyHostToDevice));
        TT_HIP(hipMemcpy(tabE.p, he.data(), sizeof(float*) * n_pairs, hipMemcpyHostToDevice));
    }
    if (L->ptrs.n < (size_t)(2 * batch)) TT_CHECK(L->ptrs.alloc((size_t)2 * batch));
    L->ptrs_host.clear();   // k_pick writes the table
    std::vector<double> Js;
    Js.reserve(steps);
    DevBuf<TrainScalars> hist;
    TT_CHECK(hist.alloc((size_t)steps));
    for (int st = 0; st < steps; ++st) {
        const double cosf_ = 0.5 * (1.0 + std::cos(M_PI * st / std::max(1, steps)));
        const float lr_t = (float)(lr * (0.01 + 0.99 * cosf_));
        hipLaunchKernelGGL(k_pick, dim3(cdiv(batch, 64)), dim3(64), 0, s, tabR.p, tabE.p, n_pairs, batch,
                           (unsigned)(L->step + 1), k0, k1, L->ptrs.p);
        TT_CHECK(train_step_ptrs(*L, c0, batch, lr_t, s));
        TT_HIP(hipMemcpyAsync(hist.p + st, L->ts.p, sizeof(TrainScalars), hipMemcpyDeviceToDevice, s));
    }
    TT_HIP(hipEventRecord(e1, s));
    TT_HIP(hipEventSynchronize(e1));
    float t_ms = 0.0f;
    TT_HIP(hipEventElapsedTime(&t_ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::vector<TrainScalars> h(steps);
    TT_HIP(hipMemcpy(h.data(), hist.p, sizeof(TrainScalars) * steps, hipMemcpyDeviceToHost));
    if (J_first) *J_first = h[0].J;
    if (J_last) {
        const int k = std::max(1, steps / 10);
        double a = 0.0;
        for (int i = steps - k; i < steps; ++i) a += h[i].J;
        *J_last = a / k;
    }
    if (ms) *ms = t_ms;
    int nbad = 0;
    for (auto& x : h) nbad += x.bad;
    if (nbad == steps) {
        tt_set_error("tt_learned_train: every step had a non-positive trace estimate or a zero diagonal");
        return TT_BREAKDOWN;
    }
    return TT_OK;
}

// ---------------------------------------------------------------------------
// exported entry points (no exception crosses the ABI)
// ---------------------------------------------------------------------------
#define TT_LGUARD(expr)                                            \
    do {                                                           \
        try {                                                      \
            return (expr);                                         \
        } catch (const std::exception& e) {                        \
            tt_set_error(std::string("exception: ") + e.what());   \
            return TT_OUT_OF_MEMORY;                               \
        } catch (...) {                                            \
            tt_set_error("unknown exception");                     \
            return TT_HIP_ERROR;                                   \
        }                                                          \
    } while (0)

extern "C" {

tt_status tt_learned_create(tt_learned** out, int device, int n_gs, int hidden, unsigned long long seed) {
    TT_LGUARD(learned_create(out, device, n_gs, hidden, seed));
}

tt_status tt_learned_destroy(tt_learned* net) { return learned_destroy(net); }

tt_status tt_learned_weight_count(const tt_learned* net, size_t* count) {
    TT_REQUIRE(net && count, "NULL argument");
    *count = learned_weight_count(net);
    return TT_OK;
}

tt_status tt_learned_get_weights(const tt_learned* net, float* host, size_t count) {
    TT_LGUARD(learned_get_weights(net, host, count));
}

tt_status tt_learned_set_weights(tt_learned* net, const float* host, size_t count) {
    TT_LGUARD(learned_set_weights(net, host, count));
}

tt_status tt_learned_apply(tt_learned* net, tt_ctx* ctx, const float* d_r, float* d_z) {
    TT_LGUARD(learned_apply(net, ctx, d_r, d_z));
}

tt_status tt_learned_train_step(tt_learned* net, tt_ctx* ctx, const float* d_R, const float* d_E, int batch,
                                double lr, double* objective, double* trace) {
    TT_LGUARD(learned_train_step(net, ctx, d_R, d_E, batch, lr, objective, trace));
}

tt_status tt_learned_train(tt_learned* net, tt_ctx* const* systems, int count, const tt_train_opts* opts,
                           tt_train_info* info) {
    TT_REQUIRE(opts, "opts is NULL");
    double jf = 0, jl = 0, ms = 0;
    tt_status st;
    try {
        st = learned_train(net, systems, count, opts->n_pairs, opts->steps, opts->batch, opts->lr, &jf, &jl, &ms);
    } catch (const std::exception& e) {
        tt_set_error(std::string("exception: ") + e.what());
        return TT_OUT_OF_MEMORY;
    }
    if (info) {
        info->objective_first = jf;
        info->objective_last = jl;
        info->ms = ms;
    }
    return st;
}

tt_status tt_set_learned(tt_ctx* ctx, tt_learned* net) {
    TT_REQUIRE(ctx, "NULL context");
    if (net) {
        TT_REQUIRE(net->device == ctx->device, "network and context on different devices");
        if (ctx->ready) TT_REQUIRE(net->C == ctx->C, "the network's channel count differs from the system's 2 n_gs");
    }
    ctx->learned = net;
    return TT_OK;
}

}  // extern "C"
