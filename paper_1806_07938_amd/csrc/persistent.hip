// Persistent solver (TT_SOLVER_PERSISTENT): one cooperative launch runs the
// iterations until convergence, a residual-replacement point, the iteration
// cap or a breakdown.  Rows a3-a8 of the hot path in one kernel, for three
// iterations (KIND):
//
// K_CG: the single-reduction rearrangement of CG (Chronopoulos & Gear,
// J. Comput. Appl. Math. 25 (1989)), both inner products of an iteration
// after one matrix-vector product with the residual:
//   w_i = A r_i,  gamma_i = r_i.r_i,  delta_i = r_i.w_i,
//   beta_i = gamma_i / gamma_{i-1} (0 at a start),
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})  (gamma_i/delta_i at a start),
//   p_i = r_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}   (s_i = A p_i),
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i;
// in exact arithmetic the iterates of textbook CG (§2.G).
// K_PCG: the same preconditioned by the block-circulant inverse (see
// row_pc_update; four phases per iteration).
// K_MINRES: Paige-Saunders MINRES (see row_mr), the paper's Toeplitz solver.
// After an FP64 residual replacement every iteration restarts from scratch.
//
// The product A r is the fused 2RBT product of §2.E, split in two phases
// separated by grid barriers:
//   row phase    (rows (c, a) of the n x n grids, a few consecutive rows per
//                block, one lane per grid point with the vectors in
//                registers): inverse row transform of the gathered column-phase
//                output -> w = A r (+ Sigma_eta r); vector updates; forward row
//                transform of the new vector -> T[f2][c][a]; partial sums;
//   column phase (block = one f2 column and one of S ranges of f1):
//                forward column transform of the C channels, per-frequency
//                Hermitian products summed over input channels, partial inverse
//                column transform -> U[f2][part][c][a], and the partial of
//                r.(Sigma_ss r) by Parseval: r.C r = L^-2 sum_f w(f2) Re(X~^H Y~),
//                valid because r vanishes outside the n x n corner.
// The column transforms are dense contractions and run on the matrix cores
// (col_mf: FP32, or FP16 / BF16 operands for the TT_PREC_F16 / BF16 forms);
// the FP64 form uses the VALU.  Each block keeps its transform tiles (its f1
// range of the column DFT matrix as operand fragments, the row DFT matrix)
// and its share of the packed spectra in LDS for the whole launch when they
// fit, so an iteration reads no spectra from memory; the preconditioned
// solver stages the slope or preconditioner spectra per column phase.  With
// 2x2 noise blocks (§2.F) the x and y rows of a subaperture share a block.
//
// Barrier: two-level counters (per XCD, then global), see grid_sync.  Every
// poll has a 2 s wall-clock limit and honours an abort word, so every wave
// exits.  All blocks sum the partial arrays in the same order and take the same
// decision at the top of every iteration.
#include "cg_common.h"

#include <algorithm>
#include <cstring>

namespace {

constexpr int PT = 512;                                  // threads per block
enum { K_CG = 0, K_PCG = 1, K_MINRES = 2 };              // iteration of the persistent kernel
constexpr unsigned long long SPIN_TICKS = 200000000ull;  // 2 s of the 100 MHz wall clock

template <typename R>
struct PArgs {
    int n, C, G, L, Lh, n_vs, S, Lrm, nrows, nwg;
    int it0, max_iter, first;
    double gprev, aprev, gmax;
    const int* vmap;
    const R* M;              // packed spectra [f2][f1][3G^2]
    const R* Mi;             // preconditioner spectra [f2][f1][C^2] (general Hermitian packing), or null
    const cplx<R>* Fa;       // [S][n][Lrm]  exp(-2 pi i f1 a / L), f1 = f1a(part) + j
    const cplx<R>* Fb;       // [S][Lrm][n]  the same values, a fastest
    const cplx<R>* Gr;       // [Lh][n]      exp(+2 pi i f2 b / L)
    const R* noise;
    const R* nxy;            // x-y noise covariance [g][v] (2x2 noise blocks, §2.F), or null
    R *x, *r, *p, *s;
    cplx<R>* T;              // [f2][c][a]
    cplx<R>* U;              // [f2][part][c][a]
    double* part;            // [2][nwg][4]: partial r.r, sigma^2 r.r, r.C r (Parseval)
    int vreg;                // CG vectors held in registers (rows per block * n <= threads)
    int rbv;                 // rows per block at a time
    const uint2* FAm;        // [S][TKf][4][Lrm] forward column-transform operand fragments (MF > 0)
    const uint2* FBm;        // [S][TKi][4][n]   inverse column-transform operand fragments (MF > 0)
    int MTf, TKf, MTi, TKi;  // output row tiles and K steps of the two column transforms
    CgScalars* S_;
    PScalars* P;
    unsigned* bar;           // barrier words: [0] top counter, [16] abort, [32 + 32 g] group counters
};

// Two-level grid barrier.  Blocks are dispatched round-robin over the 8 XCDs,
// so block i joins group i % 8, the blocks sharing one L2.  Every wave first
// drains its own memory operations (s_waitcnt 0: its stores are in the L2 of
// its XCD, the L1 being write-through); thread 0 of every block then
// increments its group counter.  The last arriver of a group issues one agent
// release fence (write-back of that L2) and increments the top counter; every
// block polls the top counter with relaxed loads (2 s wall-clock limit and the
// abort word, both checked every 64th poll) and finishes with an agent acquire
// fence.  One L2 write-back per XCD
// instead of one per block.  Counters grow monotonically within a launch
// (reset before it).  A stale read would show up as a failed FP64 true-residual
// check after the launch, never as a silently accepted result.
constexpr unsigned NGRP = 8;

__device__ bool grid_sync(unsigned* bar, unsigned nwg, unsigned& epoch, int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    ++epoch;
    if (threadIdx.x == 0) {
        unsigned* top = bar;
        unsigned* abort_w = bar + 16;
        unsigned* grp = bar + 32;
        const unsigned g = blockIdx.x % NGRP;
        const unsigned ng = nwg < NGRP ? nwg : NGRP;
        const unsigned gsz = (nwg - g + NGRP - 1) / NGRP;
        const unsigned old = __hip_atomic_fetch_add(&grp[g * 32], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == epoch * gsz - 1u) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        int ok = 1;
        const unsigned long long t0 = wall_clock64();
        unsigned spins = 0;
        // one load per poll; the abort word and the time limit every 64th poll
        while (__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch * ng) {
            if ((++spins & 63u) == 0u) {
                if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > SPIN_TICKS) {
                    __hip_atomic_store(abort_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Sum over the block with wave shuffles and one LDS pass; every lane gets the
// same value, and the order of additions is fixed, so every block reduces
// identical inputs to bit-identical results.
__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct D3 {
    double a, b, c;
};

__device__ D3 block_sum3(D3 v, double* red) {
    v.a = wave_sum(v.a);
    v.b = wave_sum(v.b);
    v.c = wave_sum(v.c);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        red[w * 3] = v.a;
        red[w * 3 + 1] = v.b;
        red[w * 3 + 2] = v.c;
    }
    __syncthreads();
    D3 r{0.0, 0.0, 0.0};
    for (int i = 0; i < PT / 64; ++i) {
        r.a += red[i * 3];
        r.b += red[i * 3 + 1];
        r.c += red[i * 3 + 2];
    }
    return r;
}

template <typename R>
struct Tiles {
    const cplx<R>* Fa;    // VALU column transforms
    const cplx<R>* Fb;
    const uint2* FAm;     // matrix-core column transforms: this block's fragments
    const uint2* FBm;
    const cplx<R>* Gr;
    R* Ms;             // resident: [slot][Lrm]; else null
    const R* Mg;       // global: M + f2 L P (used when Ms is null)
    cplx<R>* work;
};

template <typename R>
__device__ inline R mval(const Tiles<R>& t, int slot, int j, int Lrm, int f1a, int P) {
    return t.Ms ? t.Ms[slot * Lrm + j] : t.Mg[(long)(f1a + j) * P + slot];
}

// Hermitian block (g, h) of the per-frequency matrix at local frequency j:
// (xx, xy = yx, yy) as complex values.
template <typename R>
__device__ inline void mblock(const Tiles<R>& t, int g, int h, int j, int G, int Lrm, int f1a, cplx<R>* m3) {
    const int P = 3 * G * G;
    if (g == h) {
        for (int k = 0; k < 3; ++k) m3[k] = cplx<R>{mval(t, 3 * g + k, j, Lrm, f1a, P), R(0)};
    } else {
        const int lo = g < h ? g : h, hi = g < h ? h : g;
        const int base = 3 * G + 6 * (lo * (2 * G - lo - 1) / 2 + (hi - lo - 1));
        const R sg = g < h ? R(1) : R(-1);
        for (int k = 0; k < 3; ++k)
            m3[k] = cplx<R>{mval(t, base + 2 * k, j, Lrm, f1a, P), sg * mval(t, base + 2 * k + 1, j, Lrm, f1a, P)};
    }
}

// State of one lane's grid point when the CG vectors live in registers.
template <typename R>
struct Lane {
    long gi;   // slope index, or -1 (no point / invalid subaperture)
    R x, r, p, s, nz;
    R u;       // preconditioned residual P r (preconditioned solver)
    R nxy;     // x-y noise covariance of this subaperture (0 without 2x2 noise blocks)
};

// Grid row index -> (channel c, subaperture row a): row = c n + a, or, with
// 2x2 noise blocks (pair set), row = (g n + a) 2 + p with c = 2 g + p, so that
// with an even number of rows per block both slopes of a subaperture are in
// the same block.
__device__ inline void row_ca(int row, int n, bool pair, int& c, int& ra) {
    if (!pair) {
        c = row / n;
        ra = row - c * n;
        return;
    }
    const int g = row / (2 * n), rem = row - g * 2 * n;
    ra = rem >> 1;
    c = 2 * g + (rem & 1);
}

// The same vector value of the other slope (x <-> y) of this lane's
// subaperture, through a block exchange buffer: lanes (k, b) and (k ^ 1, b).
template <typename R>
__device__ inline R partner_value(R mine, int nrk, int n) {
    __shared__ R xch[PT];
    if ((int)threadIdx.x < nrk * n) xch[threadIdx.x] = mine;
    __syncthreads();
    R other = 0;
    if ((int)threadIdx.x < nrk * n) {
        const int k = threadIdx.x / n, b = threadIdx.x % n;
        if ((k ^ 1) < nrk) other = xch[(k ^ 1) * n + b];
    }
    __syncthreads();
    return other;
}

// x-y noise part of w.Sigma_eta w for this lane's value w: nxy w w_partner.
template <typename R>
__device__ inline double xy_noise_term(const Lane<R>& v, R w, int nrk, int n) {
    const R wp = partner_value(v.gi >= 0 ? w : R(0), nrk, n);
    return v.gi >= 0 ? (double)v.nxy * (double)w * (double)wp : 0.0;
}

// Us[k][f2] = sum over f1 ranges of the column-phase outputs of row k
template <typename R>
__device__ void gather_u(const PArgs<R>& a, cplx<R>* Us, int base, int stride, int nrk) {
    const int n = a.n, Lh = a.Lh, C = a.C, S = a.S;
    for (int i = threadIdx.x; i < nrk * Lh; i += PT) {
        const int k = i / Lh, f2 = i % Lh;
        const int row = base + k * stride;
        int c, ra;
        row_ca(row, n, a.nxy != nullptr, c, ra);
        const cplx<R>* u = a.U + ((long)f2 * S * C + c) * n + ra;
        // the first (up to) four ranges loaded together, then summed in order
        cplx<R> q[4];
#pragma unroll
        for (int part = 0; part < 4; ++part) q[part] = part < S ? u[(long)part * C * n] : cplx<R>{0, 0};
        R ux = q[0].x, uy = q[0].y;
#pragma unroll
        for (int part = 1; part < 4; ++part)
            if (part < S) {
                ux += q[part].x;
                uy += q[part].y;
            }
        for (int part = 4; part < S; ++part) {
            const cplx<R> w = u[(long)part * C * n];
            ux += w.x;
            uy += w.y;
        }
        Us[k * Lh + f2] = cplx<R>{ux, uy};
    }
}

// sum_{f2} w(f2) Re(us[f2] exp(+2 pi i f2 b / L)), w = 1 at f2 = 0 and L/2, else 2
template <typename R>
__device__ inline R inv_row(const cplx<R>* us, const cplx<R>* Gr, int n, int b, int L, int Lh) {
    const int fend = (L % 2 == 0) ? Lh - 1 : Lh;
    R s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int f2 = 1;
    for (; f2 + 3 < fend; f2 += 4) {
        const cplx<R> u0 = us[f2], u1 = us[f2 + 1], u2 = us[f2 + 2], u3 = us[f2 + 3];
        const cplx<R> w0 = Gr[f2 * n + b], w1 = Gr[(f2 + 1) * n + b], w2 = Gr[(f2 + 2) * n + b],
                      w3 = Gr[(f2 + 3) * n + b];
        s0 += u0.x * w0.x - u0.y * w0.y;
        s1 += u1.x * w1.x - u1.y * w1.y;
        s2 += u2.x * w2.x - u2.y * w2.y;
        s3 += u3.x * w3.x - u3.y * w3.y;
    }
    for (; f2 < fend; ++f2) {
        const cplx<R> u0 = us[f2], w0 = Gr[f2 * n + b];
        s0 += u0.x * w0.x - u0.y * w0.y;
    }
    R nyq = 0;
    if (L % 2 == 0 && Lh > 1) {
        const cplx<R> u0 = us[Lh - 1], w0 = Gr[(Lh - 1) * n + b];
        nyq = u0.x * w0.x - u0.y * w0.y;
    }
    return us[0].x + R(2) * ((s0 + s1) + (s2 + s3)) + nyq;
}

// T[f2][c][a] = sum_b xr[b] exp(-2 pi i f2 b / L)
template <typename R>
__device__ void fwd_rows(const PArgs<R>& a, const cplx<R>* Gr, const R* xs, int base, int stride, int nrk) {
    const int n = a.n, Lh = a.Lh, C = a.C;
    for (int i = threadIdx.x; i < nrk * Lh; i += PT) {
        const int k = i / Lh, f2 = i % Lh;
        const int row = base + k * stride;
        int c, ra;
        row_ca(row, n, a.nxy != nullptr, c, ra);
        const R* xr = xs + k * n;
        const cplx<R>* g = Gr + f2 * n;
        R r0 = 0, i0 = 0, r1 = 0, i1 = 0;
        int b = 0;
        for (; b + 1 < n; b += 2) {
            const cplx<R> w0 = g[b], w1 = g[b + 1];
            r0 += xr[b] * w0.x;
            i0 -= xr[b] * w0.y;
            r1 += xr[b + 1] * w1.x;
            i1 -= xr[b + 1] * w1.y;
        }
        if (b < n) {
            r0 += xr[b] * g[b].x;
            i0 -= xr[b] * g[b].y;
        }
        a.T[((long)f2 * C + c) * n + ra] = cplx<R>{r0 + r1, i0 + i1};
    }
}

// Row phase, CG vectors in registers (one lane per grid point of the block's rows).
template <typename R>
__device__ void row_phase_reg(const PArgs<R>& a, const Tiles<R>& t, Lane<R>& v, int nrk, bool update, R alpha,
                              R beta, int par, double* red) {
    const int n = a.n, Lh = a.Lh, L = a.L;
    cplx<R>* Us = t.work;   // filled by gather_u before the call when update is set
    R* xs = reinterpret_cast<R*>(Us + a.rbv * Lh);
    __syncthreads();
    double g = 0.0, sg = 0.0;
    // 2x2 noise blocks: the other slope's residual for the noise term of A r
    R rp = 0;
    if (update && a.nxy) rp = partner_value(v.gi >= 0 ? v.r : R(0), nrk, n);
    R rn = 0;
    if ((int)threadIdx.x < nrk * n) {
        const int k = threadIdx.x / n, b = threadIdx.x % n;
        if (v.gi >= 0) {
            if (update) {
                const R inv = R(1) / (R(L) * R(L));
                const R wv = inv_row(Us + k * Lh, t.Gr, n, b, L, Lh) * inv + v.nz * v.r + v.nxy * rp;
                v.p = v.r + beta * v.p;
                v.s = wv + beta * v.s;
                v.x += alpha * v.p;
                v.r = v.r - alpha * v.s;
            }
            rn = v.r;
            g = (double)rn * (double)rn;
            sg = (double)v.nz * g;
        }
        xs[k * n + b] = rn;
    }
    __syncthreads();
    if (a.nxy) sg += xy_noise_term(v, rn, nrk, n);
    fwd_rows(a, t.Gr, xs, blockIdx.x * a.rbv, 1, nrk);
    const D3 tot = block_sum3(D3{g, sg, 0.0}, red);
    if (threadIdx.x == 0) {
        a.part[((long)par * a.nwg + blockIdx.x) * 4 + 0] = tot.a;
        a.part[((long)par * a.nwg + blockIdx.x) * 4 + 1] = tot.b;
    }
}

// Preconditioned solver, row phases (CG vectors in registers).  The
// iteration is the single-reduction form of preconditioned CG:
//   u_i = P r_i,  w_i = A u_i,  gamma_i = r_i.u_i,  delta_i = u_i.w_i,
//   beta_i = gamma_i / gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1},
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i,
// with four phases per iteration: row (update, forward transform of r), column
// with the preconditioner spectra (partial gamma by Parseval), row (u = P r,
// partial sigma^2 u.u, forward transform of u), column with the slope spectra
// (partial u.C u by Parseval).
//
// Update phase: w = A u from the gathered column outputs (Us), vector updates,
// forward row transform of the new residual; partial r.r in slot 0.
template <typename R>
__device__ void row_pc_update(const PArgs<R>& a, const Tiles<R>& t, Lane<R>& v, int nrk, R alpha, R beta, int par,
                              double* red) {
    const int n = a.n, Lh = a.Lh, L = a.L;
    cplx<R>* Us = t.work;   // filled by gather_u before the call
    R* xs = reinterpret_cast<R*>(Us + a.rbv * Lh);
    __syncthreads();
    double g = 0.0;
    R up = 0;   // 2x2 noise blocks: the other slope's u
    if (a.nxy) up = partner_value(v.u, nrk, n);
    if ((int)threadIdx.x < nrk * n) {
        const int k = threadIdx.x / n, b = threadIdx.x % n;
        R rn = 0;
        if (v.gi >= 0) {
            const R inv = R(1) / (R(L) * R(L));
            const R wv = inv_row(Us + k * Lh, t.Gr, n, b, L, Lh) * inv + v.nz * v.u + v.nxy * up;
            v.p = v.u + beta * v.p;
            v.s = wv + beta * v.s;
            v.x += alpha * v.p;
            v.r = v.r - alpha * v.s;
            rn = v.r;
            g = (double)rn * (double)rn;
        }
        xs[k * n + b] = rn;
    }
    __syncthreads();
    fwd_rows(a, t.Gr, xs, blockIdx.x * a.rbv, 1, nrk);
    const D3 tot = block_sum3(D3{g, 0.0, 0.0}, red);
    if (threadIdx.x == 0) a.part[((long)par * a.nwg + blockIdx.x) * 4 + 0] = tot.a;
}

// Preconditioner phase: u = P r from the column outputs of the preconditioner
// spectra (no noise term: it is inside P), forward row transform of u; partial
// sigma^2 u.u in slot 1.
template <typename R>
__device__ void row_pc_precond(const PArgs<R>& a, const Tiles<R>& t, Lane<R>& v, int nrk, int par, double* red) {
    const int n = a.n, Lh = a.Lh, L = a.L;
    cplx<R>* Us = t.work;
    R* xs = reinterpret_cast<R*>(Us + a.rbv * Lh);
    __syncthreads();
    gather_u(a, Us, blockIdx.x * a.rbv, 1, nrk);
    __syncthreads();
    double sg = 0.0;
    R un = 0;
    if ((int)threadIdx.x < nrk * n) {
        const int k = threadIdx.x / n, b = threadIdx.x % n;
        if (v.gi >= 0) {
            const R inv = R(1) / (R(L) * R(L));
            un = inv_row(Us + k * Lh, t.Gr, n, b, L, Lh) * inv;
            sg = (double)v.nz * (double)un * (double)un;
        }
        v.u = un;
        xs[k * n + b] = un;
    }
    __syncthreads();
    if (a.nxy) sg += xy_noise_term(v, un, nrk, n);
    fwd_rows(a, t.Gr, xs, blockIdx.x * a.rbv, 1, nrk);
    const D3 tot = block_sum3(D3{sg, 0.0, 0.0}, red);
    if (threadIdx.x == 0) a.part[((long)par * a.nwg + blockIdx.x) * 4 + 1] = tot.a;
}

// MINRES (Paige-Saunders; the paper's solver for its Toeplitz system, §2.G),
// CG vectors in registers with the lane fields read as
//   r: q_j = beta_j v_j, the Lanczos vector before normalisation,
//   p: v_{j-1},  s: d_{j-2},  u: d_{j-3}  (direction vectors of the solution).
// At the top of iteration j the partial sums give beta_j = ||q_j|| and
// alpha_j = v_j.A v_j = q_j.A q_j / beta_j^2, and the Givens QR step j-1 of
// the tridiagonal matrix (scalars identical in every block) gives tau, delta2,
// eps, gamma2 and the residual norm phi_{j-1}.  This row phase then applies
// the solution update of step j-1 (qr set), normalises v_j, forms
// A v_j = (C q_j + sigma^2 q_j) / beta_j from the gathered column outputs, and
// the next Lanczos vector q_{j+1} = A v_j - alpha_j v_j - beta_j v_{j-1};
// partial ||q||^2 and sigma^2 ||q||^2 in slots 0 and 1 (the CG layout), and the
// forward row transform of q_{j+1} for the column phase's q.C q.
template <typename R>
__device__ inline void mr_update(Lane<R>& v, bool qr, R tau, R delta2, R eps, R igamma2) {
    if (qr) {
        const R d = (v.p - delta2 * v.s - eps * v.u) * igamma2;
        v.x += tau * d;
        v.u = v.s;
        v.s = d;
    }
}

template <typename R>
__device__ void row_mr(const PArgs<R>& a, const Tiles<R>& t, Lane<R>& v, int nrk, bool qr, R tau, R delta2, R eps,
                       R igamma2, R alpha, R beta, int par, double* red) {
    const int n = a.n, Lh = a.Lh, L = a.L;
    cplx<R>* Us = t.work;   // filled by gather_u before the call
    R* xs = reinterpret_cast<R*>(Us + a.rbv * Lh);
    __syncthreads();
    double g = 0.0, sg = 0.0;
    R qp = 0;   // 2x2 noise blocks: the other slope's q
    if (a.nxy) qp = partner_value(v.gi >= 0 ? v.r : R(0), nrk, n);
    R qn = 0;
    if ((int)threadIdx.x < nrk * n) {
        const int k = threadIdx.x / n, b = threadIdx.x % n;
        if (v.gi >= 0) {
            mr_update(v, qr, tau, delta2, eps, igamma2);
            const R ib = R(1) / beta;
            const R inv = R(1) / (R(L) * R(L));
            const R vj = v.r * ib;
            const R avj = (inv_row(Us + k * Lh, t.Gr, n, b, L, Lh) * inv + v.nz * v.r + v.nxy * qp) * ib;
            qn = avj - alpha * vj - beta * v.p;
            v.p = vj;
            v.r = qn;
            g = (double)qn * (double)qn;
            sg = (double)v.nz * g;
        }
        xs[k * n + b] = qn;
    }
    __syncthreads();
    if (a.nxy) sg += xy_noise_term(v, qn, nrk, n);
    fwd_rows(a, t.Gr, xs, blockIdx.x * a.rbv, 1, nrk);
    const D3 tot = block_sum3(D3{g, sg, 0.0}, red);
    if (threadIdx.x == 0) {
        a.part[((long)par * a.nwg + blockIdx.x) * 4 + 0] = tot.a;
        a.part[((long)par * a.nwg + blockIdx.x) * 4 + 1] = tot.b;
    }
}

// Row phase with the CG vectors in global memory (systems with more rows per block).
template <typename R>
__device__ void row_phase_mem(const PArgs<R>& a, const Tiles<R>& t, bool update, R alpha, R beta, int par,
                              double* red) {
    const int n = a.n, Lh = a.Lh, L = a.L;
    cplx<R>* Us = t.work;
    R* xs = reinterpret_cast<R*>(Us + a.rbv * Lh);
    double g = 0.0, sg = 0.0;
    for (int base = blockIdx.x; base < a.nrows; base += a.rbv * a.nwg) {
        int nrk = 0;
        while (nrk < a.rbv && base + nrk * a.nwg < a.nrows) ++nrk;
        __syncthreads();
        if (update) {
            gather_u(a, Us, base, a.nwg, nrk);
            __syncthreads();
        }
        for (int i = threadIdx.x; i < nrk * n; i += PT) {
            const int k = i / n, b = i % n;
            const int row = base + k * a.nwg;
            int c, ra;
            row_ca(row, n, a.nxy != nullptr, c, ra);
            const int vv = a.vmap[ra * n + b];
            R rn = 0;
            if (vv >= 0) {
                const long gi = (long)c * a.n_vs + vv;
                const R ro = a.r[gi];
                if (update) {
                    const R inv = R(1) / (R(L) * R(L));
                    const R wv = inv_row(Us + k * Lh, t.Gr, n, b, L, Lh) * inv + a.noise[gi] * ro;
                    const R pv = ro + beta * a.p[gi];
                    const R sv = wv + beta * a.s[gi];
                    a.p[gi] = pv;
                    a.s[gi] = sv;
                    a.x[gi] += alpha * pv;
                    rn = ro - alpha * sv;
                    a.r[gi] = rn;
                } else {
                    rn = ro;
                }
                g += (double)rn * (double)rn;
                sg += (double)a.noise[gi] * (double)rn * (double)rn;
            }
            xs[k * n + b] = rn;
        }
        __syncthreads();
        fwd_rows(a, t.Gr, xs, base, a.nwg, nrk);
    }
    const D3 tot = block_sum3(D3{g, sg, 0.0}, red);
    if (threadIdx.x == 0) {
        a.part[((long)par * a.nwg + blockIdx.x) * 4 + 0] = tot.a;
        a.part[((long)par * a.nwg + blockIdx.x) * 4 + 1] = tot.b;
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

// Column transforms on the matrix cores.  Both are real products
//   forward  X (Lr x 2C) = A (Lr x 2n) B (2n x 2C):  A[j][(a,e)] = (Re, Im) F[f1a+j][a],
//            B[(a,0)][2c+f] = (Re T, Im T)[f],  B[(a,1)][2c+f] = (-Im T, Re T)[f],  T = T[c][a]
//   inverse  U (n x 2C) = A' (n x 2Lr) B' (2Lr x 2C): A'[a][(j,e)] = (Re, Im) F[f1a+j][a],
//            B'[(j,0)][2p+f] = (Re Y, Im Y)[f],  B'[(j,1)][2p+f] = (Im Y, -Re Y)[f],  Y = Y[p][j]
// so that column 2c (2p) of the result is the real and column 2c+1 the
// imaginary part of X_c = sum_a F[.][a] T[c][a]  (U_p = sum_j Y[p][j] conj F[j][a]).
// One 16 x 16 output tile per wave at a time; the K index (a, e) (or (j, e)) is
// taken in an order that lets a lane read one complex operand per K step pair:
//   MF = 1, FP32, v_mfma_f32_16x16x4f32: lane (kq = l/16, lc = l%16) supplies
//       A[lc][k], B[k][lc] with k = (4t + kq, e) at the two steps (t, e = 0, 1);
//   MF = 2, 3, FP16 / BF16 operands, v_mfma_f32_16x16x16{f16,bf16_1k}: lane
//       supplies the 4 K values (8t + 2kq, e), (8t + 2kq + 1, e), e = 0, 1.
// The result element v of lane l is row 4 kq + v, column lc of the tile.
// The constant operand (A, A') is precomputed per K step in this lane order
// (uint2 per lane per step: one complex FP32, or four 16-bit values) as
// [t][kq][row], zero outside the transform, rows past the last output row not
// stored; a wave reads 4 runs of 16 consecutive 8-byte words per step.  FP16 / BF16 data operands are multiplied by sc, a power of two that
// brings the block's largest magnitude to [2^13, 2^14); results are multiplied
// by 1/sc, both exact.
__device__ inline unsigned short bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);   // round to nearest even
}

template <int MF>
__device__ inline f32x4 mfma_k16(uint2 av, float b0, float b1, float b2, float b3, float sc, f32x4 acc) {
    if constexpr (MF == 2) {
        const f16x4 A = __builtin_bit_cast(f16x4, av);
        const f16x4 B = {(_Float16)(b0 * sc), (_Float16)(b1 * sc), (_Float16)(b2 * sc), (_Float16)(b3 * sc)};
        return __builtin_amdgcn_mfma_f32_16x16x16f16(A, B, acc, 0, 0, 0);
    } else {
        const i16x4 A = __builtin_bit_cast(i16x4, av);
        const i16x4 B = {(short)bf16_bits(b0 * sc), (short)bf16_bits(b1 * sc), (short)bf16_bits(b2 * sc),
                         (short)bf16_bits(b3 * sc)};
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc, 0, 0, 0);
    }
}

// power of two bringing a largest magnitude (float bits, >= 0) to [2^13, 2^14)
__device__ inline float mf_scale(int mbits) {
    const int e = (mbits >> 23) & 0xff;
    if (mbits <= 0 || e == 0xff) return 1.0f;
    int se = 267 - e;
    se = se < 1 ? 1 : (se > 253 ? 253 : se);
    return __uint_as_float((unsigned)se << 23);
}

// One K step of a column transform: operands already loaded (av: constant
// side; w0, w1: data-side complex values, masked), accumulated into acc.
//   fwd (INV = false): B = ((Re, Im)[f], (-Im, Re)[f]) of w
//   inv (INV = true):  B = ((Re, Im)[f], (Im, -Re)[f]) of w
template <int MF, bool INV>
__device__ inline f32x4 col_step(uint2 av, cplx<float> w0, cplx<float> w1, int f, float sc, f32x4 acc) {
    const float p0 = f ? w0.y : w0.x;
    const float q0 = INV ? (f ? -w0.x : w0.y) : (f ? w0.x : -w0.y);
    if constexpr (MF == 1) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.x), p0, acc, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.y), q0, acc, 0, 0, 0);
    } else {
        const float p1 = f ? w1.y : w1.x;
        const float q1 = INV ? (f ? -w1.x : w1.y) : (f ? w1.x : -w1.y);
        return mfma_k16<MF>(av, p0, q0, p1, q1, sc, acc);
    }
}

// data-side operand(s) of K step t for this lane: index k0 (and k0 + 1) of
// the row src, masked to zero outside [0, kmax) or for an unused column
template <int MF>
__device__ inline void col_load(const cplx<float>* src, int t, int kq, int kmax, bool colok, cplx<float>& w0,
                                cplx<float>& w1) {
    const int k0 = MF == 1 ? 4 * t + kq : 8 * t + 2 * kq;
    w0 = src[k0 < kmax ? k0 : 0];
    if (!(colok && k0 < kmax)) w0 = cplx<float>{0.f, 0.f};
    if constexpr (MF != 1) {
        w1 = src[k0 + 1 < kmax ? k0 + 1 : 0];
        if (!(colok && k0 + 1 < kmax)) w1 = cplx<float>{0.f, 0.f};
    }
}

// One output tile per wave at a time: the K loop runs in groups of 4 steps
// (all loads of a group issued before its products, on two accumulators) and
// a remainder of single steps.  INV selects the inverse transform.
template <int MF, bool INV>
__device__ void col_mf(const uint2* FR, int rowsA, const cplx<float>* src, int srcstride, int kmax, float* dst,
                       int dststride, int rmax, int C, int MT, int TK, float sc) {
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, kq = l >> 4, lc = l & 15;
    const int NT = (2 * C + 15) / 16;
    const float isc = 1.0f / sc;
    for (int tp = wave; tp < MT * NT; tp += PT / 64) {
        const int mt = tp % MT, nt = tp / MT;
        const int c = nt * 8 + (lc >> 1), f = lc & 1;
        const bool cv = c < C;
        const cplx<float>* sp = src + (cv ? c : 0) * srcstride;
        // constant operand: [t][kq][row] words, rows >= rowsA are zero (not stored)
        const int arow = mt * 16 + lc;
        const bool aok = arow < rowsA;
        const uint2* fr = FR + kq * rowsA + (aok ? arow : 0);
        const int ts = 4 * rowsA;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
        int t = 0;
        for (; t + 4 <= TK; t += 4) {
            uint2 av[4];
            cplx<float> w0[4], w1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = fr[(t + u) * ts];
                if (!aok) av[u] = uint2{0u, 0u};
                col_load<MF>(sp, t + u, kq, kmax, cv, w0[u], w1[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; u += 2) {
                acc0 = col_step<MF, INV>(av[u], w0[u], w1[u], f, sc, acc0);
                acc1 = col_step<MF, INV>(av[u + 1], w0[u + 1], w1[u + 1], f, sc, acc1);
            }
        }
        for (; t < TK; ++t) {
            cplx<float> w0, w1;
            col_load<MF>(sp, t, kq, kmax, cv, w0, w1);
            uint2 av = fr[t * ts];
            if (!aok) av = uint2{0u, 0u};
            acc0 = col_step<MF, INV>(av, w0, w1, f, sc, acc0);
        }
        if (cv)
            for (int v = 0; v < 4; ++v) {
                const int row = mt * 16 + 4 * kq + v;
                const float r = acc0[v] + acc1[v];
                if (row < rmax) dst[2 * (c * dststride + row) + f] = MF == 1 ? r : r * isc;
            }
    }
}

// forward: Xh[c][j] = sum_a F[f1a+j][a] Tc[c][a], j < Lr
template <int MF>
__device__ inline void col_fwd_mf(const uint2* FA, const cplx<float>* Tc, cplx<float>* Xh, int n, int C, int Lr,
                                  int Lrm, int MT, int TK, float sc) {
    col_mf<MF, false>(FA, Lrm, Tc, n, n, reinterpret_cast<float*>(Xh), Lrm, Lr, C, MT, TK, sc);
}

// inverse (partial over this f1 range): Uo[p][a] = sum_j Yh[p][j] conj F[f1a+j][a], a < n
template <int MF>
__device__ inline void col_inv_mf(const uint2* FB, const cplx<float>* Yh, cplx<float>* Uo, int n, int C, int Lr,
                                  int Lrm, int MT, int TK, float sc) {
    col_mf<MF, true>(FB, n, Yh, Lrm, Lr, reinterpret_cast<float*>(Uo), n, n, C, MT, TK, sc);
}

// largest |value| over the block, as float bits, accumulated into *slot
__device__ inline void block_max_bits(float m, int* slot) {
    int b = (int)__float_as_uint(m);
    for (int o = 32; o > 0; o >>= 1) {
        const int q = __shfl_xor(b, o);
        b = q > b ? q : b;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(slot, b);
}

// General Hermitian per-frequency matrix (preconditioner spectra, C^2 reals
// per frequency: slot a = Re H[a][a]; for a < b, slots C + 2k, C + 2k + 1 =
// Re, Im H[a][b] with k = a C - a(a+1)/2 + b - a - 1) at local frequency j.
template <typename R>
__device__ inline cplx<R> hval(const R* Hs, const R* Hg, int a, int b, int j, int C, int Lrm) {
    const int C2 = C * C;
    auto val = [&](int slot) { return Hs ? Hs[slot * Lrm + j] : Hg[(long)j * C2 + slot]; };
    if (a == b) return cplx<R>{val(a), R(0)};
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int k = lo * C - lo * (lo + 1) / 2 + (hi - lo - 1);
    const R im = val(C + 2 * k + 1);
    return cplx<R>{val(C + 2 * k), a < b ? im : -im};
}

// MF: column transforms on the VALU (0) or on the matrix cores with FP32 (1),
// FP16 (2) or BF16 (3) operands and FP32 accumulation.  GEN: the products use
// the general Hermitian spectra gsrc (preconditioner) instead of the packed
// slope spectra.  gsrc: global spectra of this phase, [f2][f1][reals]; when
// stage is set they are first copied to the block's LDS spectra region (in the
// same loop as the T loads); slot: partial-sum slot of the Parseval term.
template <typename R, int MF, bool GEN>
__device__ void col_phase(const PArgs<R>& a, const Tiles<R>& t, int par, double* red, int* s_mx, const R* gsrc,
                          bool stage, int slot) {
    const int n = a.n, L = a.L, C = a.C, G = a.G, S = a.S, Lrm = a.Lrm;
    double accd = 0.0;
    if (blockIdx.x < a.Lh * S) {
        const int f2 = blockIdx.x / S, part = blockIdx.x % S;
        const int f1a = (int)((long)part * L / S), f1b = (int)((long)(part + 1) * L / S);
        const int Lr = f1b - f1a;
        cplx<R>* Tc = t.work;          // [C][n]
        cplx<R>* Xh = Tc + C * n;      // [C][Lrm]
        cplx<R>* Yh = Xh + C * Lrm;    // [C][Lrm]
        if (MF >= 2 && threadIdx.x == 0) s_mx[0] = s_mx[1] = 0;
        __syncthreads();
        const int Pn = GEN ? C * C : 3 * G * G;
        const R* gcol = gsrc + ((long)f2 * L + f1a) * Pn;   // this block's spectra, [j][reals]
        {
            R m = 0;
            // the column's C n inputs, up to four per thread and pass with every
            // load issued before the first store (one memory round trip a pass)
            const cplx<R>* Tg = a.T + (long)f2 * C * n;
            for (int i0 = 0; i0 < C * n; i0 += 4 * PT) {
                cplx<R> q[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * PT + threadIdx.x;
                    q[u] = Tg[i < C * n ? i : 0];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) asm volatile("" : "+v"(q[u].x), "+v"(q[u].y));
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * PT + threadIdx.x;
                    if (i < C * n) {
                        Tc[i] = q[u];
                        if constexpr (MF >= 2) m = fmaxf(m, fmaxf(fabsf(q[u].x), fabsf(q[u].y)));
                    }
                }
            }
            if (stage) {   // this block's spectra, [j][reals] -> [reals][j], the same way
                const int tot = Pn * Lr;
                for (int i0 = 0; i0 < tot; i0 += 16 * PT) {
                    R g[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int i = i0 + u * PT + threadIdx.x;
                        g[u] = gcol[i < tot ? i : 0];
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) asm volatile("" : "+v"(g[u]));
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int i = i0 + u * PT + threadIdx.x;
                        if (i < tot) t.Ms[(i % Pn) * Lrm + i / Pn] = g[u];
                    }
                }
            }
            if constexpr (MF >= 2) block_max_bits(m, s_mx);
        }
        __syncthreads();
        // forward column transform: matrix cores, or two channels per lane on the VALU
        if constexpr (MF > 0) {
            col_fwd_mf<MF>(t.FAm, Tc, Xh, n, C, Lr, Lrm, a.MTf, a.TKf, MF >= 2 ? mf_scale(s_mx[0]) : 1.0f);
        } else {
        for (int i = threadIdx.x; i < (C / 2) * Lr; i += PT) {
            const int cp = i / Lr, j = i % Lr;
            const cplx<R>* t0 = Tc + (2 * cp) * n;
            const cplx<R>* t1 = t0 + n;
            R a0r = 0, a0i = 0, a1r = 0, a1i = 0, b0r = 0, b0i = 0, b1r = 0, b1i = 0;
            int ra = 0;
            for (; ra + 1 < n; ra += 2) {
                const cplx<R> f = t.Fa[ra * Lrm + j], g = t.Fa[(ra + 1) * Lrm + j];
                const cplx<R> u0 = t0[ra], u1 = t1[ra], w0 = t0[ra + 1], w1 = t1[ra + 1];
                a0r += u0.x * f.x - u0.y * f.y;
                a0i += u0.x * f.y + u0.y * f.x;
                a1r += u1.x * f.x - u1.y * f.y;
                a1i += u1.x * f.y + u1.y * f.x;
                b0r += w0.x * g.x - w0.y * g.y;
                b0i += w0.x * g.y + w0.y * g.x;
                b1r += w1.x * g.x - w1.y * g.y;
                b1i += w1.x * g.y + w1.y * g.x;
            }
            if (ra < n) {
                const cplx<R> f = t.Fa[ra * Lrm + j];
                const cplx<R> u0 = t0[ra], u1 = t1[ra];
                a0r += u0.x * f.x - u0.y * f.y;
                a0i += u0.x * f.y + u0.y * f.x;
                a1r += u1.x * f.x - u1.y * f.y;
                a1i += u1.x * f.y + u1.y * f.x;
            }
            Xh[(2 * cp) * Lrm + j] = cplx<R>{a0r + b0r, a0i + b0i};
            Xh[(2 * cp + 1) * Lrm + j] = cplx<R>{a1r + b1r, a1i + b1i};
        }
        }
        __syncthreads();
        // per-frequency products, x and y outputs of one sensor per lane
        const double wt2 = ((f2 == 0) || ((L % 2) == 0 && 2 * f2 == L)) ? 1.0 : 2.0;
        R ym = 0;
        for (int i = threadIdx.x; i < G * Lr; i += PT) {
            const int g = i / Lr, j = i % Lr;
            R y0r = 0, y0i = 0, y1r = 0, y1i = 0;
            if constexpr (GEN) {
                const R* Hs = t.Ms;
                const R* Hg = gcol;
                for (int b = 0; b < C; ++b) {
                    const cplx<R> xb = Xh[b * Lrm + j];
                    const cplx<R> h0 = hval(Hs, Hg, 2 * g, b, j, C, Lrm), h1 = hval(Hs, Hg, 2 * g + 1, b, j, C, Lrm);
                    y0r += h0.x * xb.x - h0.y * xb.y;
                    y0i += h0.x * xb.y + h0.y * xb.x;
                    y1r += h1.x * xb.x - h1.y * xb.y;
                    y1i += h1.x * xb.y + h1.y * xb.x;
                }
            } else
            for (int h = 0; h < G; ++h) {
                cplx<R> m3[3];
                mblock(t, g, h, j, G, Lrm, f1a, m3);
                const cplx<R> xa = Xh[(2 * h) * Lrm + j], xb = Xh[(2 * h + 1) * Lrm + j];
                y0r += m3[0].x * xa.x - m3[0].y * xa.y + m3[1].x * xb.x - m3[1].y * xb.y;
                y0i += m3[0].x * xa.y + m3[0].y * xa.x + m3[1].x * xb.y + m3[1].y * xb.x;
                y1r += m3[1].x * xa.x - m3[1].y * xa.y + m3[2].x * xb.x - m3[2].y * xb.y;
                y1i += m3[1].x * xa.y + m3[1].y * xa.x + m3[2].x * xb.y + m3[2].y * xb.x;
            }
            Yh[(2 * g) * Lrm + j] = cplx<R>{y0r, y0i};
            Yh[(2 * g + 1) * Lrm + j] = cplx<R>{y1r, y1i};
            const cplx<R> x0 = Xh[(2 * g) * Lrm + j], x1 = Xh[(2 * g + 1) * Lrm + j];
            accd += wt2 * ((double)x0.x * y0r + (double)x0.y * y0i + (double)x1.x * y1r + (double)x1.y * y1i);
            if constexpr (MF >= 2) ym = fmaxf(ym, fmaxf(fmaxf(fabsf(y0r), fabsf(y0i)), fmaxf(fabsf(y1r), fabsf(y1i))));
        }
        if constexpr (MF >= 2) block_max_bits(ym, s_mx + 1);
        __syncthreads();
        // partial inverse column transform over this f1 range
        cplx<R>* Uo = a.U + (((long)f2 * S + part) * C) * n;
        if constexpr (MF > 0) {
            col_inv_mf<MF>(t.FBm, Yh, Uo, n, C, Lr, Lrm, a.MTi, a.TKi, MF >= 2 ? mf_scale(s_mx[1]) : 1.0f);
        } else {
        for (int i = threadIdx.x; i < (C / 2) * n; i += PT) {
            const int pp = i / n, ra = i % n;
            const cplx<R>* y0 = Yh + (2 * pp) * Lrm;
            const cplx<R>* y1 = y0 + Lrm;
            R a0r = 0, a0i = 0, a1r = 0, a1i = 0, b0r = 0, b0i = 0, b1r = 0, b1i = 0;
            int j = 0;
            for (; j + 1 < Lr; j += 2) {
                const cplx<R> f = t.Fb[j * n + ra], g = t.Fb[(j + 1) * n + ra];   // conj: inverse twiddles
                const cplx<R> u0 = y0[j], u1 = y1[j], w0 = y0[j + 1], w1 = y1[j + 1];
                a0r += u0.x * f.x + u0.y * f.y;
                a0i += u0.y * f.x - u0.x * f.y;
                a1r += u1.x * f.x + u1.y * f.y;
                a1i += u1.y * f.x - u1.x * f.y;
                b0r += w0.x * g.x + w0.y * g.y;
                b0i += w0.y * g.x - w0.x * g.y;
                b1r += w1.x * g.x + w1.y * g.y;
                b1i += w1.y * g.x - w1.x * g.y;
            }
            if (j < Lr) {
                const cplx<R> f = t.Fb[j * n + ra];
                const cplx<R> u0 = y0[j], u1 = y1[j];
                a0r += u0.x * f.x + u0.y * f.y;
                a0i += u0.y * f.x - u0.x * f.y;
                a1r += u1.x * f.x + u1.y * f.y;
                a1i += u1.y * f.x - u1.x * f.y;
            }
            Uo[(2 * pp) * n + ra] = cplx<R>{a0r + b0r, a0i + b0i};
            Uo[(2 * pp + 1) * n + ra] = cplx<R>{a1r + b1r, a1i + b1i};
        }
        }
    }
    const D3 tot = block_sum3(D3{accd, 0.0, 0.0}, red);
    if (threadIdx.x == 0) a.part[((long)par * a.nwg + blockIdx.x) * 4 + slot] = tot.a / ((double)a.L * (double)a.L);
}

// KIND: K_CG, K_PCG (preconditioned CG, four phases per iteration, see
// row_pc_update) or K_MINRES (see row_mr).
template <typename R, bool RES, int MF, int KIND>
__global__ void __launch_bounds__(PT) k_cg_persistent(PArgs<R> a) {
    constexpr bool PC = KIND == K_PCG;
    constexpr bool MR = KIND == K_MINRES;
    // The FP64 preconditioned kernel is built without the 2x2 noise blocks (the
    // present gfx950 compiler rejects that instantiation; the host refuses it).
    if constexpr (PC && sizeof(R) == 8) a.nxy = nullptr;
    extern __shared__ __align__(16) char smem_raw[];
    __shared__ double red[3 * PT / 64];
    __shared__ int s_flag;
    __shared__ int s_mx[2];
    const int n = a.n, Lh = a.Lh, Lrm = a.Lrm, S = a.S, L = a.L, P = 3 * a.G * a.G;
    const bool colunit = blockIdx.x < Lh * S;
    const int f2 = colunit ? blockIdx.x / S : 0, part = colunit ? blockIdx.x % S : 0;
    const int f1a = (int)((long)part * L / S), f1b = (int)((long)(part + 1) * L / S);
    const long fragA = (long)a.TKf * 4 * a.Lrm, fragB = (long)a.TKi * 4 * a.n;
    Tiles<R> t;
    t.Mg = a.M + (long)f2 * L * P;
    t.Fa = t.Fb = nullptr;
    t.FAm = t.FBm = nullptr;
    if constexpr (RES) {
        char* q = smem_raw;
        if constexpr (MF > 0) {
            uint2* FAm = reinterpret_cast<uint2*>(q);
            uint2* FBm = FAm + fragA;
            const uint2* fa = a.FAm + part * fragA;
            const uint2* fb = a.FBm + part * fragB;
            for (int i = threadIdx.x; i < fragA; i += PT) FAm[i] = fa[i];
            for (int i = threadIdx.x; i < fragB; i += PT) FBm[i] = fb[i];
            t.FAm = FAm;
            t.FBm = FBm;
            q = reinterpret_cast<char*>(FBm + fragB);
        } else {
            cplx<R>* Fa = reinterpret_cast<cplx<R>*>(q);
            cplx<R>* Fb = Fa + n * Lrm;
            const cplx<R>* fa = a.Fa + (long)part * n * Lrm;
            const cplx<R>* fb = a.Fb + (long)part * Lrm * n;
            for (int i = threadIdx.x; i < n * Lrm; i += PT) {
                Fa[i] = fa[i];
                Fb[i] = fb[i];
            }
            t.Fa = Fa;
            t.Fb = Fb;
            q = reinterpret_cast<char*>(Fb + Lrm * n);
        }
        cplx<R>* Gr = reinterpret_cast<cplx<R>*>(q);
        R* Ms = reinterpret_cast<R*>(Gr + Lh * n);
        for (int i = threadIdx.x; i < Lh * n; i += PT) Gr[i] = a.Gr[i];
        const int Lr = f1b - f1a;
        if (colunit && !PC)   // resident for the launch (the preconditioned solver stages per phase)
            for (int i = threadIdx.x; i < P * Lr; i += PT) {
                const int slot = i / Lr, j = i % Lr;
                Ms[slot * Lrm + j] = t.Mg[(long)(f1a + j) * P + slot];
            }
        t.Gr = Gr;
        t.Ms = Ms;
        // spectra region: the slope spectra, or (preconditioned) whichever spectra
        // the current column phase staged, the larger general packing included
        const int Preg = PC ? (P > a.C * a.C ? P : a.C * a.C) : P;
        t.work = reinterpret_cast<cplx<R>*>(Ms + (((long)Preg * Lrm + 3) & ~3L));   // 16-byte aligned
        __syncthreads();
    } else {
        if constexpr (MF > 0) {
            t.FAm = a.FAm + part * fragA;
            t.FBm = a.FBm + part * fragB;
        } else {
            t.Fa = a.Fa + (long)part * n * Lrm;
            t.Fb = a.Fb + (long)part * Lrm * n;
        }
        t.Gr = a.Gr;
        t.Ms = nullptr;
        t.work = reinterpret_cast<cplx<R>*>(smem_raw);
    }
    // lanes of the register-resident CG vectors
    Lane<R> v{-1, 0, 0, 0, 0, 0, 0, 0};
    int nrk = 0;
    if (a.vreg) {
        // a block owns the consecutive rows blockIdx.x * rbv + k, k < nrk
        nrk = a.nrows - (int)blockIdx.x * a.rbv;
        nrk = nrk < 0 ? 0 : (nrk > a.rbv ? a.rbv : nrk);
        if ((int)threadIdx.x < nrk * n) {
            const int k = threadIdx.x / n, b = threadIdx.x % n;
            const int row = blockIdx.x * a.rbv + k;
            int c, ra;
            row_ca(row, n, a.nxy != nullptr, c, ra);
            const int vv = a.vmap[ra * n + b];
            if (vv >= 0) {
                v.gi = (long)c * a.n_vs + vv;
                if (a.nxy) v.nxy = a.nxy[(long)(c >> 1) * a.n_vs + vv];
                v.x = a.x[v.gi];
                v.r = a.r[v.gi];
                v.p = a.p[v.gi];
                v.s = a.s[v.gi];
                v.nz = a.noise[v.gi];
            }
        }
    }
    unsigned epoch = 0;
    int it = a.it0;
    if (a.vreg) row_phase_reg<R>(a, t, v, nrk, false, R(0), R(0), it & 1, red);
    else row_phase_mem<R>(a, t, false, R(0), R(0), it & 1, red);
    if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
    if constexpr (PC) {
        col_phase<R, MF, true>(a, t, it & 1, red, s_mx, a.Mi, RES, 3);
        if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
        row_pc_precond<R>(a, t, v, nrk, it & 1, red);
        if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
        col_phase<R, MF, false>(a, t, it & 1, red, s_mx, a.M, RES, 2);
    } else {
        col_phase<R, MF, false>(a, t, it & 1, red, s_mx, a.M, false, 2);
    }
    if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
    double gprev = a.gprev, aprev = a.aprev;
    bool first = a.first != 0;
    const double tol2 = a.S_->tol2, drop2 = a.S_->drop2;
    // MINRES: Givens QR state (every launch starts a fresh Lanczos process)
    double mr_c = -1.0, mr_s = 0.0, mr_d1 = 0.0, mr_eps = 0.0, mr_phi = 0.0, mr_alpha = 0.0;
    int mr_k = 0;   // Lanczos vectors normalised so far in this launch
    while (true) {
        const int par = it & 1;
        // The loads of the partial sums and of this block's column-phase outputs
        // (for the next row phase) are issued together: one memory round trip.
        D3 pv{0.0, 0.0, 0.0};
        if (a.nwg <= PT) {
            if ((int)threadIdx.x < a.nwg) {
                const double* q = a.part + ((long)par * a.nwg + threadIdx.x) * 4;
                pv = PC ? D3{q[0], q[1] + q[2], q[3]} : D3{q[0], q[1], q[2]};
            }
        } else {
            for (int i = threadIdx.x; i < a.nwg; i += PT) {
                const double* q = a.part + ((long)par * a.nwg + i) * 4;
                pv.a += q[0];
                pv.b += PC ? q[1] + q[2] : q[1];
                pv.c += PC ? q[3] : q[2];
            }
        }
        if (a.vreg) gather_u(a, t.work, blockIdx.x * a.rbv, 1, nrk);
        const D3 tot = block_sum3(pv, red);
        // rr: r.r (stopping rule); CG: gm = r.r, dl = r.A r;  PCG: gm = r.P r, dl = u.A u
        const double g = tot.a;
        const double gm = PC ? tot.c : tot.a;
        const double dl = PC ? tot.b : tot.c + tot.b;
        int st = ST_RUN;
        double alpha = 0.0, beta = 0.0;
        // MINRES scalars of this iteration (see row_mr)
        bool mr_qr = false;
        double mr_tau = 0.0, mr_delta2 = 0.0, mr_epsk = 0.0, mr_ig = 0.0, mr_rr = 0.0;
        if constexpr (MR) {
            beta = sqrt(g);          // beta_j = ||q_j||
            alpha = dl / g;          // alpha_j = q_j.A q_j / ||q_j||^2
            mr_qr = mr_k >= 1;
            bool bad = !isfinite(g) || !isfinite(dl);
            if (mr_qr) {             // Givens QR step j-1: alpha_{j-1} = mr_alpha, beta_j
                mr_delta2 = mr_c * mr_d1 + mr_s * mr_alpha;
                const double gamma1 = mr_s * mr_d1 - mr_c * mr_alpha;
                const double eps_next = mr_s * beta, d1_next = -mr_c * beta;
                const double gamma2 = sqrt(gamma1 * gamma1 + beta * beta);
                bad = bad || !(gamma2 > 0.0);
                mr_epsk = mr_eps;
                mr_c = gamma1 / gamma2;
                mr_s = beta / gamma2;
                mr_tau = mr_c * mr_phi;
                mr_phi = mr_s * mr_phi;
                mr_ig = 1.0 / gamma2;
                mr_eps = eps_next;
                mr_d1 = d1_next;
            } else {
                mr_phi = beta;       // phi_0 = beta_1 = ||r||
            }
            mr_alpha = alpha;
            mr_rr = mr_phi * mr_phi; // residual norm^2 of the current iterate
            if (bad || !isfinite(mr_rr)) st = ST_BREAK;
            else if (mr_rr <= tol2) st = ST_CONV;
            else if (drop2 > 0.0 && mr_rr < drop2 * a.gmax) st = ST_REFINE;
            else if (it >= a.max_iter) st = ST_CAP;
            else if (!(g > 0.0)) st = ST_BREAK;
        } else {
        if (!isfinite(g) || !isfinite(dl) || !isfinite(gm)) st = ST_BREAK;
        else if (g <= tol2) st = ST_CONV;
        else if (drop2 > 0.0 && g < drop2 * a.gmax) st = ST_REFINE;
        else if (it >= a.max_iter) st = ST_CAP;
        }
        if (!MR && st == ST_RUN) {
            if (first) {
                beta = 0.0;
                alpha = gm / dl;
            } else {
                beta = gm / gprev;
                alpha = gm / (dl - beta * gm / aprev);
            }
            if (!(alpha > 0.0) || !isfinite(alpha)) st = ST_BREAK;
        }
        if (st != ST_RUN) {
            // MINRES: the solution update of the QR step just taken
            if (MR && a.vreg && v.gi >= 0 && st != ST_BREAK)
                mr_update(v, mr_qr, (R)mr_tau, (R)mr_delta2, (R)mr_epsk, (R)mr_ig);
            if (a.vreg && v.gi >= 0) {
                a.x[v.gi] = v.x;
                a.r[v.gi] = v.r;
                a.p[v.gi] = v.p;
                a.s[v.gi] = v.s;
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                a.P->gamma_prev = gprev;
                a.P->alpha_prev = aprev;
                a.P->gamma = gm;
                a.P->delta = dl;
                a.P->first = first ? 1 : 0;
                a.S_->state = st;
                a.S_->iter = it;
                a.S_->rr[it & 1] = MR ? mr_rr : g;
            }
            return;
        }
        if constexpr (PC) {
            row_pc_update<R>(a, t, v, nrk, (R)alpha, (R)beta, (it + 1) & 1, red);
        } else if constexpr (MR) {
            row_mr<R>(a, t, v, nrk, mr_qr, (R)mr_tau, (R)mr_delta2, (R)mr_epsk, (R)mr_ig, (R)alpha, (R)beta,
                      (it + 1) & 1, red);
            ++mr_k;
        } else {
            if (a.vreg) row_phase_reg<R>(a, t, v, nrk, true, (R)alpha, (R)beta, (it + 1) & 1, red);
            else row_phase_mem<R>(a, t, true, (R)alpha, (R)beta, (it + 1) & 1, red);
        }
        gprev = gm;
        aprev = alpha;
        first = false;
        ++it;
        if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
        if constexpr (PC) {
            col_phase<R, MF, true>(a, t, it & 1, red, s_mx, a.Mi, RES, 3);
            if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
            row_pc_precond<R>(a, t, v, nrk, it & 1, red);
            if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
            col_phase<R, MF, false>(a, t, it & 1, red, s_mx, a.M, RES, 2);
        } else {
            col_phase<R, MF, false>(a, t, it & 1, red, s_mx, a.M, false, 2);
        }
        if (!grid_sync(a.bar, a.nwg, epoch, &s_flag)) return;
    }
}

// Fragment tiles and K steps of the matrix-core column transforms (MF > 0).
struct FragShape {
    int MTf = 0, TKf = 0, MTi = 0, TKi = 0, rowsA = 0, rowsB = 0;
    long a_words() const { return (long)TKf * 4 * rowsA; }
    long b_words() const { return (long)TKi * 4 * rowsB; }
};

FragShape frag_shape(int MF, int n, int Lrm) {
    FragShape f;
    if (MF == 0) return f;
    const int kstep = MF == 1 ? 4 : 8;   // K values (a or j) per lane step pair / per step
    f.MTf = (Lrm + 15) / 16;
    f.TKf = (n + kstep - 1) / kstep;
    f.MTi = (n + 15) / 16;
    f.TKi = (Lrm + kstep - 1) / kstep;
    f.rowsA = Lrm;   // forward: output rows j < Lrm
    f.rowsB = n;     // inverse: output rows a < n
    return f;
}

// LDS bytes: resident tiles (if RES) + work region (max of column and row needs)
template <typename R>
size_t lds_bytes(const tt_ctx& c, int Lrm, int rbv, bool res, int MF, bool pc) {
    const size_t cs = sizeof(cplx<R>);
    const size_t colw = cs * ((size_t)c.C * c.n + 2ull * c.C * Lrm);
    const size_t roww = cs * (size_t)rbv * c.Lh + sizeof(R) * (size_t)rbv * c.n;
    size_t b = std::max(colw, roww);
    if (res) {
        const FragShape fs = frag_shape(MF, c.n, Lrm);
        b += MF > 0 ? 8 * (size_t)(fs.a_words() + fs.b_words()) : cs * 2ull * c.n * Lrm;
        const size_t reals = pc ? std::max((size_t)packed_reals(c.G), (size_t)c.C * c.C) : (size_t)packed_reals(c.G);
        b += cs * (size_t)c.Lh * c.n + sizeof(R) * ((reals * Lrm + 3) & ~(size_t)3);
    }
    return b;
}

// IEEE binary16 and bfloat16 bit patterns, round to nearest even (host).
uint16_t half_bits(double v) {
    const uint16_t sgn = std::signbit(v) ? 0x8000 : 0;
    double x = std::fabs(v);
    if (x == 0.0) return sgn;
    if (x >= 65520.0) return sgn | 0x7c00;
    int e = 0;
    std::frexp(x, &e);                       // x = m 2^e, m in [0.5, 1)
    if (e - 1 < -14) {                       // subnormal: multiples of 2^-24
        const double q = std::nearbyint(std::ldexp(x, 24));
        return sgn | (uint16_t)q;            // q = 1024 is the smallest normal
    }
    double q = std::nearbyint(std::ldexp(x, 11 - e) - 1024.0);   // 10 mantissa bits
    int E = e - 1 + 15;
    if (q >= 1024.0) {
        q = 0.0;
        ++E;
    }
    if (E >= 31) return sgn | 0x7c00;
    return sgn | (uint16_t)(E << 10) | (uint16_t)q;
}

uint16_t bf16_bits_host(double v) {
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Operand fragments of the matrix-core column transforms for every f1 range,
// in the lane order of col_fwd_mf / col_inv_mf; zero outside the transform.
void build_frags(int MF, int n, int L, int S, int Lrm, const std::vector<double>& co, const std::vector<double>& si,
                 std::vector<uint2>& FA, std::vector<uint2>& FB) {
    const FragShape fs = frag_shape(MF, n, Lrm);
    FA.assign((size_t)S * fs.a_words(), uint2{0u, 0u});
    FB.assign((size_t)S * fs.b_words(), uint2{0u, 0u});
    auto enc = [MF](double v) -> uint32_t {
        if (MF == 1) {
            const float f = (float)v;
            uint32_t u;
            std::memcpy(&u, &f, 4);
            return u;
        }
        return MF == 2 ? half_bits(v) : bf16_bits_host(v);
    };
    for (int part = 0; part < S; ++part) {
        const int f1a = (int)((long)part * L / S), Lr = (int)((long)(part + 1) * L / S) - f1a;
        // (Re, Im) exp(-2 pi i f1 a / L) at local frequency j, encoded; zero outside
        auto F = [&](int j, int a, uint32_t* re, uint32_t* im) {
            *re = *im = 0u;
            if (j < Lr && a < n) {
                const int m = (int)(((long)(f1a + j) * a) % L);
                *re = enc(co[m]);
                *im = enc(-si[m]);
            }
        };
        for (int pass = 0; pass < 2; ++pass) {
            const int rows = pass == 0 ? fs.rowsA : fs.rowsB, TK = pass == 0 ? fs.TKf : fs.TKi;
            uint2* out = (pass == 0 ? FA.data() : FB.data()) + (size_t)part * TK * 4 * rows;
            for (int t = 0; t < TK; ++t)
                for (int kq = 0; kq < 4; ++kq)
                    for (int row = 0; row < rows; ++row) {
                        uint2& w = out[((size_t)t * 4 + kq) * rows + row];
                        if (MF == 1) {
                            const int k = 4 * t + kq;
                            if (pass == 0) F(row, k, &w.x, &w.y);   // j = row, a = k
                            else F(k, row, &w.x, &w.y);             // j = k, a = row
                        } else {
                            const int k0 = 8 * t + 2 * kq;
                            uint32_t r0, i0, r1, i1;
                            if (pass == 0) {
                                F(row, k0, &r0, &i0);
                                F(row, k0 + 1, &r1, &i1);
                            } else {
                                F(k0, row, &r0, &i0);
                                F(k0 + 1, row, &r1, &i1);
                            }
                            w.x = r0 | (i0 << 16);
                            w.y = r1 | (i1 << 16);
                        }
                    }
        }
    }
}

// Host-built transform tiles for the persistent kernel (exact twiddle indices):
// the VALU tiles (Fa, Fb), the row tiles (Gr) and, for MF > 0, the fragments.
template <typename R>
tt_status build_tiles(tt_ctx& c, int S, int Lrm, int MF) {
    const int n = c.n, L = c.L, Lh = c.Lh;
    std::vector<double> co(L), si(L);
    for (int k = 0; k < L; ++k) {
        const double ang = 2.0 * M_PI * (double)k / (double)L;
        co[k] = std::cos(ang);
        si[k] = std::sin(ang);
    }
    std::vector<cplx<R>> fa((size_t)S * n * Lrm, cplx<R>{0, 0}), fb((size_t)S * Lrm * n, cplx<R>{0, 0}),
        gr((size_t)Lh * n);
    for (int part = 0; part < S; ++part) {
        const int f1a = (int)((long)part * L / S), f1b = (int)((long)(part + 1) * L / S);
        for (int j = 0; j < f1b - f1a; ++j)
            for (int a = 0; a < n; ++a) {
                const int m = (int)(((long)(f1a + j) * a) % L);
                const cplx<R> v{(R)co[m], (R)(-si[m])};   // exp(-2 pi i f1 a / L)
                fa[((size_t)part * n + a) * Lrm + j] = v;
                fb[((size_t)part * Lrm + j) * n + a] = v;
            }
    }
    for (int f2 = 0; f2 < Lh; ++f2)
        for (int b = 0; b < n; ++b) {
            const int m = (int)(((long)f2 * b) % L);
            gr[(size_t)f2 * n + b] = cplx<R>{(R)co[m], (R)si[m]};   // exp(+2 pi i f2 b / L)
        }
    const size_t sc = sizeof(cplx<R>);
    TT_CHECK(c.tFa.alloc(fa.size() * sc / sizeof(c64) + 1));
    TT_CHECK(c.tFb.alloc(fb.size() * sc / sizeof(c64) + 1));
    TT_CHECK(c.tGr.alloc(gr.size() * sc / sizeof(c64) + 1));
    TT_HIP(hipMemcpyAsync(c.tFa.p, fa.data(), fa.size() * sc, hipMemcpyHostToDevice, c.stream));
    TT_HIP(hipMemcpyAsync(c.tFb.p, fb.data(), fb.size() * sc, hipMemcpyHostToDevice, c.stream));
    TT_HIP(hipMemcpyAsync(c.tGr.p, gr.data(), gr.size() * sc, hipMemcpyHostToDevice, c.stream));
    if (MF > 0) {
        std::vector<uint2> FA, FB;
        build_frags(MF, n, L, S, Lrm, co, si, FA, FB);
        TT_CHECK(c.tFAm.alloc(FA.size() + 1));
        TT_CHECK(c.tFBm.alloc(FB.size() + 1));
        TT_HIP(hipMemcpyAsync(c.tFAm.p, FA.data(), FA.size() * sizeof(uint2), hipMemcpyHostToDevice, c.stream));
        TT_HIP(hipMemcpyAsync(c.tFBm.p, FB.data(), FB.size() * sizeof(uint2), hipMemcpyHostToDevice, c.stream));
    }
    TT_HIP(hipStreamSynchronize(c.stream));   // the host vectors are released on return
    return TT_OK;
}

template <typename R, bool RES, int MF, int KIND>
tt_status launch(tt_ctx& c, PArgs<R>& a, size_t lds, float* ms) {
    TT_HIP(hipMemsetAsync(c.bar.p, 0, c.bar.n * sizeof(unsigned), c.stream));
    void* args[] = {&a};
    TT_HIP(hipEventRecord(c.ev0, c.stream));
    TT_HIP(hipLaunchCooperativeKernel((const void*)k_cg_persistent<R, RES, MF, KIND>, dim3(a.nwg), dim3(PT), args,
                                      (unsigned)lds, c.stream));
    TT_HIP(hipEventRecord(c.ev1, c.stream));
    TT_HIP(hipEventSynchronize(c.ev1));
    TT_HIP(hipEventElapsedTime(ms, c.ev0, c.ev1));
    unsigned ab = 0;
    TT_HIP(hipMemcpy(&ab, a.bar + 16, sizeof(ab), hipMemcpyDeviceToHost));
    if (ab != 0u) {
        tt_set_error("persistent solver: grid barrier timed out");
        return TT_HIP_ERROR;
    }
    return TT_OK;
}

// the recurrences stopped on a non-positive or non-finite step with finite
// residual norms (an inexact operator), not on non-finite data
inline bool finite_breakdown(const CgScalars& h) { return std::isfinite(h.rr[h.iter & 1]) && std::isfinite(h.rr_true); }

template <typename R, bool RES, int MF, int KIND>
tt_status run_persistent(tt_ctx& c, const float* s, double* zeta, const tt_solve_opts& o, tt_solve_info& info,
                         PArgs<R>& a, size_t lds, CgScalars& h) {
    const bool f32 = sizeof(R) == 4;
    TT_HIP(hipFuncSetAttribute((const void*)k_cg_persistent<R, RES, MF, KIND>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    int per_cu = 0;
    TT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_cg_persistent<R, RES, MF, KIND>, PT, lds));
    if (per_cu < 1) {
        tt_set_error("persistent solver does not fit on a compute unit");
        return TT_INVALID_ARG;
    }
    int it = 0, first = 1;
    double gprev = 0.0, aprev = 0.0, gmax = h.rr_true;
    int code = TT_OK;
    bool have_true = false;
    while (true) {
        a.it0 = it;
        a.first = first;
        a.gprev = gprev;
        a.aprev = aprev;
        a.gmax = gmax;
        float ms = 0.f;
        TT_CHECK((launch<R, RES, MF, KIND>(c, a, lds, &ms)));
        info.kernel_ms += ms;
        info.kernel_launches++;
        TT_HIP(hipMemcpy(&h, cg_scalars(c), sizeof(h), hipMemcpyDeviceToHost));
        it = h.iter;
        if (h.state == ST_BREAK) {
            // With FP16 / BF16 column transforms the inner operator is inexact
            // and not exactly symmetric, which can end the recurrences early;
            // the last iterate is kept (the failed step is not applied), so the
            // solve continues from the FP64 true residual while that keeps
            // falling (by 10% or more per restart), and otherwise ends with
            // TT_NOT_CONVERGED.
            if (MF < 2 || !finite_breakdown(h)) {
                code = TT_BREAKDOWN;
                break;
            }
            const double prev = gmax;
            TT_CHECK(cg_true_residual(c, s, f32, &h));
            have_true = true;
            info.refinements++;
            if (h.rr_true <= h.tol2) break;
            if (!(h.rr_true < 0.81 * prev) || it >= o.max_iter) {
                // no further progress: the last iterate is returned
                code = std::isfinite(h.rr_true) ? TT_NOT_CONVERGED : TT_BREAKDOWN;
                break;
            }
            TT_CHECK(cg_copy_r64_to_r32(c));
            TT_CHECK(cg_fill_zero(c, (float*)a.p, nullptr));
            TT_CHECK(cg_fill_zero(c, (float*)a.s, nullptr));
            gmax = h.rr_true;
            first = 1;
            gprev = aprev = 0.0;
            continue;
        }
        if (h.state == ST_CAP) {
            code = TT_NOT_CONVERGED;
            break;
        }
        // ST_CONV or ST_REFINE: certify / replace with the FP64 true residual
        TT_CHECK(cg_true_residual(c, s, f32, &h));
        have_true = true;
        info.refinements++;
        if (h.rr_true <= h.tol2) break;
        if (it >= o.max_iter) {
            code = TT_NOT_CONVERGED;
            break;
        }
        if (f32) TT_CHECK(cg_copy_r64_to_r32(c));
        // restart the recurrences from the replaced residual
        TT_CHECK(cg_fill_zero(c, f32 ? (float*)a.p : nullptr, f32 ? nullptr : (double*)a.p));
        TT_CHECK(cg_fill_zero(c, f32 ? (float*)a.s : nullptr, f32 ? nullptr : (double*)a.s));
        gmax = h.rr_true;
        first = 1;
        gprev = aprev = 0.0;
    }
    return cg_finish(c, s, zeta, f32, have_true, info, code);
}

template <typename R, int MF, int KIND>
tt_status run_mode(tt_ctx& c, const float* s, double* zeta, const tt_solve_opts& o, tt_solve_info& info,
                   PArgs<R>& a, size_t lds, bool res, CgScalars& h) {
    if (res) return run_persistent<R, true, MF, KIND>(c, s, zeta, o, info, a, lds, h);
    return run_persistent<R, false, MF, KIND>(c, s, zeta, o, info, a, lds, h);
}

// MF: column-transform mode (0 VALU, 1 FP32, 2 FP16, 3 BF16 matrix cores);
// kind: K_CG, K_PCG (block-circulant preconditioner, Mi: its spectra), K_MINRES
template <typename R>
tt_status solve_persistent_t(tt_ctx& c, const float* s, const double* x0, double* zeta, const tt_solve_opts& o,
                             tt_solve_info& info, R* x, R* r, R* p, R* sv, const R* M, const R* noise, int MF,
                             int kind, const R* Mi) {
    const bool pc = kind == K_PCG;
    const bool f32 = sizeof(R) == 4;
    info = tt_solve_info{};
    TT_CHECK(cg_setup(c, s, x0, o, f32));
    TT_CHECK(cg_fill_zero(c, f32 ? (float*)p : nullptr, f32 ? nullptr : (double*)p));
    TT_CHECK(cg_fill_zero(c, f32 ? (float*)sv : nullptr, f32 ? nullptr : (double*)sv));
    CgScalars h;
    TT_HIP(hipMemcpyAsync(&h, cg_scalars(c), sizeof(h), hipMemcpyDeviceToHost, c.stream));
    TT_HIP(hipStreamSynchronize(c.stream));
    if (h.bnorm2 == 0.0 || h.rr_true <= h.tol2) return cg_finish(c, s, zeta, f32, true, info, TT_OK);

    // launch shape: one block per compute unit; the f1 axis split so that the
    // Lh x S column units cover the blocks
    const int nwg = c.num_cu;
    int S = std::max(1, nwg / std::max(c.Lh, 1));
    S = std::min(S, std::max(1, c.L / 8));
    const int Lrm = (c.L + S - 1) / S;
    // every column unit (f2, f1 range) is owned by one block for the whole launch
    if (c.Lh * S > nwg) {
        tt_set_error("persistent solver: pad_L / 2 + 1 frequency columns exceed the compute units; use "
                     "TT_SOLVER_KERNELS or TT_SOLVER_BATCHED");
        return TT_INVALID_ARG;
    }
    const size_t lim = 160 * 1024 - 512;   // minus the static LDS (reduction scratch and flags)
    // rows per block: all of a block's rows at once when they fit the threads
    const int rows_per_block = (c.C * c.n + nwg - 1) / nwg;
    // with 2x2 noise blocks, rows per block rounded up to even: the x and y rows
    // of a subaperture row stay together
    const int rpb2 = c.has_nxy ? (rows_per_block + 1) / 2 * 2 : rows_per_block;
    const bool vreg = rpb2 * c.n <= PT;
    const int rbv = vreg ? rpb2 : std::max(1, std::min(4, PT / std::max(c.n, 1)));
    if (kind == K_PCG && c.has_nxy && !f32) {
        tt_set_error("2x2 noise blocks with the preconditioned solver need TT_PREC_F32");
        return TT_INVALID_ARG;
    }
    if ((kind != K_CG || c.has_nxy) && !vreg) {
        tt_set_error("preconditioned CG / MINRES / 2x2 noise blocks: a block's grid rows must fit its threads "
                     "(n * ceil(2 n_gs n / CUs), rounded up to even, <= 512)");
        return TT_INVALID_ARG;
    }
    const bool res = lds_bytes<R>(c, Lrm, rbv, true, MF, pc) <= lim;
    const size_t lds = lds_bytes<R>(c, Lrm, rbv, res, MF, pc);
    if (lds > lim) {
        tt_set_error("persistent solver: system too large for LDS");
        return TT_INVALID_ARG;
    }
    if (c.tile_S != S || c.tile_elem != (int)sizeof(R) || c.tile_mf != MF) {
        c.tile_S = 0;   // rebuilt below; left invalid if the build fails
        TT_CHECK(build_tiles<R>(c, S, Lrm, MF));
        c.tile_S = S;
        c.tile_elem = (int)sizeof(R);
        c.tile_mf = MF;
    }
    if (c.pU.n < (size_t)c.Lh * S * c.C * c.n) TT_CHECK(c.pU.alloc((size_t)c.Lh * S * c.C * c.n));
    if (c.ppart.n < 8 * (size_t)nwg) TT_CHECK(c.ppart.alloc(8 * (size_t)nwg));
    if (c.bar.n < 32 + 32 * NGRP) TT_CHECK(c.bar.alloc(32 + 32 * NGRP));

    PArgs<R> a{};
    a.nwg = nwg;
    a.S = S;
    a.Lrm = Lrm;
    a.n = c.n;
    a.C = c.C;
    a.G = c.G;
    a.L = c.L;
    a.Lh = c.Lh;
    a.n_vs = c.n_vs;
    a.nrows = c.C * c.n;
    a.max_iter = o.max_iter;
    a.vmap = c.vmap.p;
    a.M = M;
    a.Mi = Mi;
    a.Fa = reinterpret_cast<const cplx<R>*>(c.tFa.p);
    a.Fb = reinterpret_cast<const cplx<R>*>(c.tFb.p);
    a.Gr = reinterpret_cast<const cplx<R>*>(c.tGr.p);
    const FragShape fs = frag_shape(MF, c.n, Lrm);
    a.FAm = reinterpret_cast<const uint2*>(c.tFAm.p);
    a.FBm = reinterpret_cast<const uint2*>(c.tFBm.p);
    a.MTf = fs.MTf;
    a.TKf = fs.TKf;
    a.MTi = fs.MTi;
    a.TKi = fs.TKi;
    a.noise = noise;
    a.nxy = c.has_nxy ? reinterpret_cast<const R*>(f32 ? (const void*)c.nxy32.p : (const void*)c.nxy64.p) : nullptr;
    a.x = x;
    a.r = r;
    a.p = p;
    a.s = sv;
    a.T = reinterpret_cast<cplx<R>*>(f32 ? (void*)c.T32.p : (void*)c.T64.p);
    a.U = reinterpret_cast<cplx<R>*>(c.pU.p);
    a.part = c.ppart.p;
    a.vreg = vreg ? 1 : 0;
    a.rbv = rbv;
    a.S_ = cg_scalars(c);
    a.P = p_scalars(c);
    a.bar = c.bar.p;
    if constexpr (sizeof(R) == 4) {
        if (pc) return run_mode<R, 1, K_PCG>(c, s, zeta, o, info, a, lds, res, h);
        if (kind == K_MINRES) return run_mode<R, 1, K_MINRES>(c, s, zeta, o, info, a, lds, res, h);
        switch (MF) {
            case 2: return run_mode<R, 2, K_CG>(c, s, zeta, o, info, a, lds, res, h);
            case 3: return run_mode<R, 3, K_CG>(c, s, zeta, o, info, a, lds, res, h);
            default: return run_mode<R, 1, K_CG>(c, s, zeta, o, info, a, lds, res, h);
        }
    } else {
        if (pc) return run_mode<R, 0, K_PCG>(c, s, zeta, o, info, a, lds, res, h);
        if (kind == K_MINRES) return run_mode<R, 0, K_MINRES>(c, s, zeta, o, info, a, lds, res, h);
        return run_mode<R, 0, K_CG>(c, s, zeta, o, info, a, lds, res, h);
    }
}

}  // namespace

tt_status solve_persistent(tt_ctx& c, const float* s, const double* x0, double* zeta, const tt_solve_opts& o,
                           tt_solve_info& info) {
    if (!c.ev0) {
        TT_HIP(hipEventCreate(&c.ev0));
        TT_HIP(hipEventCreate(&c.ev1));
    }
    const bool pc = o.preconditioner == TT_PRECOND_CIRCULANT;
    if (pc) TT_CHECK(precond_build(c));
    const int kind = o.method == TT_METHOD_MINRES ? K_MINRES : pc ? K_PCG : K_CG;
    if (o.precision == TT_PREC_F64)
        return solve_persistent_t<double>(c, s, x0, zeta, o, info, c.x64.p, c.r64.p, c.p64.p, c.q64.p, c.M64.p,
                                          c.noise64.p, 0, kind, c.Minv64.p);
    // FP32 vectors and products; the column transforms on the matrix cores
    // with FP32, FP16 or BF16 operands
    const int MF = o.precision == TT_PREC_F16 ? 2 : o.precision == TT_PREC_BF16 ? 3 : 1;
    return solve_persistent_t<float>(c, s, x0, zeta, o, info, c.x32.p, c.r32.p, c.p32.p, c.q32.p, c.M32.p,
                                     c.noise32.p, MF, kind, c.Minv32.p);
}
