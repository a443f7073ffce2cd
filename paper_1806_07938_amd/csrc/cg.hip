// Conjugate gradients for W_s (Sigma_ss + Sigma_eta) W_s^T zeta = s (§2.C first
// step, §2.G), one launch per phase (TT_SOLVER_KERNELS), with the FP64 residual
// replacement that certifies the tolerance.
//
// Iteration j (textbook CG):
//   q = A p                                   (fused 2RBT product, matvec.hip)
//   alpha = rr_j / (p . q);  x += alpha p;  r -= alpha q
//   rr_{j+1} = r . r;  beta = rr_{j+1} / rr_j;  p = r + beta p
// Dot products accumulate in FP64 per block and are summed in a fixed order by
// every block that needs them, so all blocks take the same decision.
//
// Residual replacement (FP32 precision): x is kept as x64 + x32.  When the
// recursive residual has dropped by `refine_drop` since the last replacement,
// or meets the tolerance, x64 += x32, x32 = 0 and r is replaced by the true
// residual s - A x64 computed with the FP64 operator; CG then continues from
// the same search direction with beta = rr_true / rr_j.  The tolerance is
// certified on that FP64 true residual.
#include "tt_internal.h"

tt_status matvec_prepare(tt_ctx& c);

#include "cg_common.h"

namespace {

constexpr int NT = 256;

__device__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Fixed-order sum of np partials, identical in every block.
__device__ double sum_partials(const double* __restrict__ part, int np, double* red) {
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
    return block_sum(v, red);
}

template <typename Ta, typename Tb>
__global__ void k_dot_partial(const Ta* __restrict__ a, const Tb* __restrict__ b, long n, double* __restrict__ part) {
    __shared__ double red[NT];
    double v = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        v += (double)a[i] * (double)b[i];
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// init: S->bnorm2 = sum(part_s), S->rr[0] = S->rr_max = S->rr_true = sum(part_r)
__global__ void k_init_scalars(const double* part_s, const double* part_r, int np, CgScalars* S, double tol,
                               double drop) {
    __shared__ double red[NT];
    const double b = sum_partials(part_s, np, red);
    const double r = sum_partials(part_r, np, red);
    if (threadIdx.x == 0) {
        S->bnorm2 = b;
        S->tol2 = tol * tol * b;
        S->drop2 = drop * drop;
        S->rr[0] = S->rr[1] = r;
        S->rr_max = r;
        S->rr_true = r;
        S->pAp = 0.0;
        S->state = ST_RUN;
        S->iter = 0;
    }
}

__global__ void k_resid(const float* __restrict__ s, const double* __restrict__ q, double* __restrict__ r, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        r[i] = (double)s[i] - q[i];
}

__global__ void k_copy_f2d(const float* __restrict__ a, double* __restrict__ b, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

__global__ void k_copy_d2f(const double* __restrict__ a, float* __restrict__ b, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

__global__ void k_fold_x(double* __restrict__ x64, float* __restrict__ x32, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        x64[i] += (double)x32[i];
        x32[i] = 0.0f;
    }
}

template <typename R>
__global__ void k_fill(R* __restrict__ a, R v, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) a[i] = v;
}

template <typename R>
__global__ void k_copy(const R* __restrict__ a, R* __restrict__ b, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = a[i];
}

// after a replacement: rr_true = sum(part); p = r + (rr_true / rr_j) p; restart bookkeeping
template <typename R>
__global__ void k_restart(R* __restrict__ p, const R* __restrict__ r, const double* __restrict__ part, int np,
                          CgScalars* S, long n, int it) {
    __shared__ double red[NT];
    const double rt = sum_partials(part, np, red);
    const double beta = rt / S->rr[(it - 1) & 1];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = r[i] + (R)beta * p[i];
}

__global__ void k_restart_scalars(const double* __restrict__ part, int np, CgScalars* S, int it) {
    __shared__ double red[NT];
    const double rt = sum_partials(part, np, red);
    if (threadIdx.x == 0) {
        S->rr[it & 1] = rt;
        S->rr_max = rt;
        S->rr_true = rt;
        S->state = ST_RUN;
    }
}

__global__ void k_set_true(const double* __restrict__ part, int np, CgScalars* S) {
    __shared__ double red[NT];
    const double rt = sum_partials(part, np, red);
    if (threadIdx.x == 0) S->rr_true = rt;
}

template <typename R>
__global__ void k_update_xr(R* __restrict__ x, R* __restrict__ r, const R* __restrict__ p, const R* __restrict__ q,
                            const double* __restrict__ partA, int nA, double* __restrict__ partB, CgScalars* S,
                            long n, int it) {
    __shared__ double red[NT];
    if (S->state != ST_RUN) return;
    const double pAp = sum_partials(partA, nA, red);
    const double rr = S->rr[it & 1];
    const double alpha = rr / pAp;
    if (!(pAp > 0.0) || !isfinite(alpha)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S->state = ST_BREAK;
            S->pAp = pAp;
        }
        return;
    }
    const R a = (R)alpha;
    double v = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        x[i] += a * p[i];
        const R ri = r[i] - a * q[i];
        r[i] = ri;
        v += (double)ri * (double)ri;
    }
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) partB[blockIdx.x] = s;
    if (blockIdx.x == 0 && threadIdx.x == 0) S->pAp = pAp;
}

template <typename R>
__global__ void k_update_p(R* __restrict__ p, const R* __restrict__ r, const double* __restrict__ partB, int nB,
                           CgScalars* S, long n, int it, int max_iter) {
    __shared__ double red[NT];
    if (S->state != ST_RUN) return;
    const double rn = sum_partials(partB, nB, red);
    const double ro = S->rr[it & 1];
    const bool conv = rn <= S->tol2;
    const bool refine = S->drop2 > 0.0 && rn < S->drop2 * S->rr_max;
    const bool cap = it + 1 >= max_iter;
    const bool bad = !isfinite(rn);
    if (conv || refine || cap || bad) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S->rr[(it + 1) & 1] = rn;
            S->iter = it + 1;
            S->state = bad ? ST_BREAK : conv ? ST_CONV : refine ? ST_REFINE : ST_CAP;
        }
        return;
    }
    const R beta = (R)(rn / ro);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S->rr[(it + 1) & 1] = rn;
        S->iter = it + 1;
    }
}

unsigned vec_blocks(long n) { return std::min<unsigned>(cdiv(n, NT), 1024u); }

// r64 = s - A x64 (FP64 operator, scratch aux64); S->rr_true = r64.r64; partials left in part
tt_status true_residual(tt_ctx& c, const float* s, CgScalars* S) {
    const long n = c.n_slopes;
    TT_CHECK(matvec_f64(c, c.x64.p, c.aux64.p, nullptr));
    hipLaunchKernelGGL(k_resid, dim3(vec_blocks(n)), dim3(NT), 0, c.stream, s, c.aux64.p, c.r64.p, n);
    // mode removal: the residual of the mode-removed system is M (s - M A M x)
    if (c.modes) TT_CHECK(modes_project_f64(c, c.r64.p));
    hipLaunchKernelGGL((k_dot_partial<double, double>), dim3(vec_blocks(n)), dim3(NT), 0, c.stream, c.r64.p,
                       c.r64.p, n, c.part.p);
    hipLaunchKernelGGL(k_set_true, dim3(1), dim3(NT), 0, c.stream, c.part.p, (int)vec_blocks(n), S);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

}  // namespace

tt_status cg_alloc(tt_ctx& c) {
    const size_t n = c.n_slopes;
    TT_CHECK(c.x32.alloc(n));
    TT_CHECK(c.r32.alloc(n));
    TT_CHECK(c.p32.alloc(n));
    TT_CHECK(c.q32.alloc(n));
    TT_CHECK(c.x64.alloc(n));
    TT_CHECK(c.r64.alloc(n));
    TT_CHECK(c.p64.alloc(n));
    TT_CHECK(c.q64.alloc(n));
    TT_CHECK(c.aux64.alloc(n));
    const size_t np = std::max<size_t>((size_t)c.C * c.n, 1024) + 1024;
    TT_CHECK(c.part.alloc(np * 2));
    TT_CHECK(c.scal.alloc(64));
    TT_CHECK(c.bar.alloc(64));
    TT_HIP(hipMemsetAsync(c.bar.p, 0, 64 * sizeof(unsigned), c.stream));
    return matvec_prepare(c);
}

// Shared set-up of both solver kinds: scalars, x64, r64 (and FP32 copies).
tt_status cg_setup(tt_ctx& c, const float* s, const double* x0, const tt_solve_opts& o, bool f32) {
    const long n = c.n_slopes;
    CgScalars* S = reinterpret_cast<CgScalars*>(c.scal.p);
    const unsigned nb = vec_blocks(n);
    double* part_s = c.part.p;
    double* part_r = c.part.p + 1024;
    if (c.modes) {
        // ||M s||^2 in FP64 (the norm of the mode-removed right-hand side)
        hipLaunchKernelGGL(k_copy_f2d, dim3(nb), dim3(NT), 0, c.stream, s, c.aux64.p, n);
        TT_CHECK(modes_project_f64(c, c.aux64.p));
        hipLaunchKernelGGL((k_dot_partial<double, double>), dim3(nb), dim3(NT), 0, c.stream, c.aux64.p, c.aux64.p,
                           n, part_s);
    } else {
        hipLaunchKernelGGL((k_dot_partial<float, float>), dim3(nb), dim3(NT), 0, c.stream, s, s, n, part_s);
    }
    if (x0) {
        hipLaunchKernelGGL(k_copy<double>, dim3(nb), dim3(NT), 0, c.stream, x0, c.x64.p, n);
        TT_CHECK(matvec_f64(c, c.x64.p, c.aux64.p, nullptr));
        hipLaunchKernelGGL(k_resid, dim3(nb), dim3(NT), 0, c.stream, s, c.aux64.p, c.r64.p, n);
    } else {
        hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(NT), 0, c.stream, c.x64.p, 0.0, n);
        hipLaunchKernelGGL(k_copy_f2d, dim3(nb), dim3(NT), 0, c.stream, s, c.r64.p, n);
    }
    if (c.modes) TT_CHECK(modes_project_f64(c, c.r64.p));   // residual in the range of M
    hipLaunchKernelGGL((k_dot_partial<double, double>), dim3(nb), dim3(NT), 0, c.stream, c.r64.p, c.r64.p, n,
                       part_r);
    const double drop = f32 ? (o.refine_drop > 0 ? o.refine_drop : 1e-3) : 0.0;
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(NT), 0, c.stream, part_s, part_r, (int)nb, S, o.tol, drop);
    if (f32) {
        hipLaunchKernelGGL(k_copy_d2f, dim3(nb), dim3(NT), 0, c.stream, c.r64.p, c.r32.p, n);
        hipLaunchKernelGGL(k_copy<float>, dim3(nb), dim3(NT), 0, c.stream, c.r32.p, c.p32.p, n);
        hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(NT), 0, c.stream, c.x32.p, 0.0f, n);
    } else {
        hipLaunchKernelGGL(k_copy<double>, dim3(nb), dim3(NT), 0, c.stream, c.r64.p, c.p64.p, n);
    }
    TT_HIP(hipGetLastError());
    return TT_OK;
}

// Replacement step shared by both solver kinds (host-driven): returns true in
// *converged when the FP64 true residual meets the tolerance.
tt_status cg_replace(tt_ctx& c, const float* s, bool f32, int it, bool* converged, CgScalars* hS) {
    const long n = c.n_slopes;
    CgScalars* S = reinterpret_cast<CgScalars*>(c.scal.p);
    const unsigned nb = vec_blocks(n);
    if (f32) hipLaunchKernelGGL(k_fold_x, dim3(nb), dim3(NT), 0, c.stream, c.x64.p, c.x32.p, n);
    TT_CHECK(true_residual(c, s, S));
    TT_HIP(hipMemcpyAsync(hS, S, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
    TT_HIP(hipStreamSynchronize(c.stream));
    *converged = hS->rr_true <= hS->tol2;
    if (*converged) return TT_OK;
    // restart from the true residual, same search direction
    if (f32) {
        hipLaunchKernelGGL(k_copy_d2f, dim3(nb), dim3(NT), 0, c.stream, c.r64.p, c.r32.p, n);
        hipLaunchKernelGGL(k_restart<float>, dim3(nb), dim3(NT), 0, c.stream, c.p32.p, c.r32.p, c.part.p, (int)nb, S,
                           n, it);
    } else {
        hipLaunchKernelGGL(k_restart<double>, dim3(nb), dim3(NT), 0, c.stream, c.p64.p, c.r64.p, c.part.p, (int)nb,
                           S, n, it);
    }
    hipLaunchKernelGGL(k_restart_scalars, dim3(1), dim3(NT), 0, c.stream, c.part.p, (int)nb, S, it);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

tt_status cg_finish(tt_ctx& c, const float* s, double* zeta, bool f32, bool have_true, tt_solve_info& info,
                    int status_code) {
    const long n = c.n_slopes;
    CgScalars* S = reinterpret_cast<CgScalars*>(c.scal.p);
    const unsigned nb = vec_blocks(n);
    if (!have_true) {
        if (f32) hipLaunchKernelGGL(k_fold_x, dim3(nb), dim3(NT), 0, c.stream, c.x64.p, c.x32.p, n);
        TT_CHECK(true_residual(c, s, S));
    }
    hipLaunchKernelGGL(k_copy<double>, dim3(nb), dim3(NT), 0, c.stream, c.x64.p, zeta, n);
    TT_HIP(hipGetLastError());
    CgScalars h;
    TT_HIP(hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    TT_HIP(hipStreamSynchronize(c.stream));
    info.iterations = h.iter;
    info.rel_residual = h.bnorm2 > 0 ? std::sqrt(h.rr_true / h.bnorm2) : 0.0;
    info.recursive_residual = h.bnorm2 > 0 ? std::sqrt(h.rr[h.iter & 1] / h.bnorm2) : 0.0;
    if (status_code == TT_OK && !(h.rr_true <= h.tol2)) status_code = TT_NOT_CONVERGED;
    info.status = status_code;
    return TT_OK;
}

tt_status solve_kernels(tt_ctx& c, const float* s, const double* x0, double* zeta, const tt_solve_opts& o,
                        tt_solve_info& info) {
    const bool f32 = o.precision == TT_PREC_F32;
    const long n = c.n_slopes;
    CgScalars* S = reinterpret_cast<CgScalars*>(c.scal.p);
    const unsigned nb = vec_blocks(n);
    const int rows = c.C * c.n;
    double* partA = c.part.p;
    double* partB = c.part.p + rows;
    info = tt_solve_info{};
    TT_CHECK(cg_setup(c, s, x0, o, f32));
    CgScalars h;
    TT_HIP(hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    TT_HIP(hipStreamSynchronize(c.stream));
    if (h.bnorm2 == 0.0 || h.rr_true <= h.tol2) {
        return cg_finish(c, s, zeta, f32, true, info, TT_OK);
    }
    int it = 0;
    const int chunk = 32;
    int code = TT_OK;
    bool have_true = false;
    while (true) {
        for (int i = 0; i < chunk && it + i < o.max_iter; ++i) {
            const int j = it + i;
            if (f32) {
                TT_CHECK(matvec_f32(c, c.p32.p, c.q32.p, partA));
                hipLaunchKernelGGL(k_update_xr<float>, dim3(nb), dim3(NT), 0, c.stream, c.x32.p, c.r32.p, c.p32.p,
                                   c.q32.p, partA, rows, partB, S, n, j);
                hipLaunchKernelGGL(k_update_p<float>, dim3(nb), dim3(NT), 0, c.stream, c.p32.p, c.r32.p, partB,
                                   (int)nb, S, n, j, o.max_iter);
            } else {
                TT_CHECK(matvec_f64(c, c.p64.p, c.q64.p, partA));
                hipLaunchKernelGGL(k_update_xr<double>, dim3(nb), dim3(NT), 0, c.stream, c.x64.p, c.r64.p, c.p64.p,
                                   c.q64.p, partA, rows, partB, S, n, j);
                hipLaunchKernelGGL(k_update_p<double>, dim3(nb), dim3(NT), 0, c.stream, c.p64.p, c.r64.p, partB,
                                   (int)nb, S, n, j, o.max_iter);
            }
        }
        TT_HIP(hipGetLastError());
        TT_HIP(hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, c.stream));
        TT_HIP(hipStreamSynchronize(c.stream));
        it = h.iter;
        if (h.state == ST_BREAK) {
            code = TT_BREAKDOWN;
            break;
        }
        if (h.state == ST_CAP || (h.state == ST_RUN && it >= o.max_iter)) {
            code = TT_NOT_CONVERGED;
            break;
        }
        if (h.state == ST_REFINE || h.state == ST_CONV) {
            bool conv = false;
            if (!f32) {
                // FP64: the recursive residual is checked against the true one
                TT_CHECK(cg_replace(c, s, false, it, &conv, &h));
            } else {
                TT_CHECK(cg_replace(c, s, true, it, &conv, &h));
            }
            info.refinements++;
            if (conv) {
                have_true = true;
                break;
            }
            if (it >= o.max_iter) {
                have_true = true;
                code = TT_NOT_CONVERGED;
                break;
            }
        }
    }
    return cg_finish(c, s, zeta, f32, have_true, info, code);
}

tt_status cg_true_residual(tt_ctx& c, const float* s, bool f32, CgScalars* hS) {
    const long n = c.n_slopes;
    CgScalars* S = cg_scalars(c);
    if (f32) hipLaunchKernelGGL(k_fold_x, dim3(vec_blocks(n)), dim3(NT), 0, c.stream, c.x64.p, c.x32.p, n);
    TT_CHECK(true_residual(c, s, S));
    TT_HIP(hipMemcpyAsync(hS, S, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
    TT_HIP(hipStreamSynchronize(c.stream));
    return TT_OK;
}

tt_status cg_fill_zero(tt_ctx& c, float* a32, double* a64) {
    const long n = c.n_slopes;
    if (a32) hipLaunchKernelGGL(k_fill<float>, dim3(vec_blocks(n)), dim3(NT), 0, c.stream, a32, 0.0f, n);
    if (a64) hipLaunchKernelGGL(k_fill<double>, dim3(vec_blocks(n)), dim3(NT), 0, c.stream, a64, 0.0, n);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

tt_status cg_copy_r64_to_r32(tt_ctx& c) {
    const long n = c.n_slopes;
    hipLaunchKernelGGL(k_copy_d2f, dim3(vec_blocks(n)), dim3(NT), 0, c.stream, c.r64.p, c.r32.p, n);
    TT_HIP(hipGetLastError());
    return TT_OK;
}
