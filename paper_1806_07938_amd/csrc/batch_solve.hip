// Frames of many systems solved together (TT_SOLVER_BATCHED): conjugate
// gradients (§2.G, row a8) run in lockstep over every system still iterating,
// each iteration's products by one batched 2RBT product (batch.hip) and the
// vector updates by kernels over all systems at once; the FP64 residual
// replacement and certification of row a10 are those of the single-system
// path (cg.hip), per system, between chunks of iterations.
//
// Per system the recurrences are exactly those of TT_SOLVER_KERNELS in FP32:
//   q = A p;  alpha = rr_j / (p . q);  x += alpha p;  r -= alpha q;
//   rr_{j+1} = r . r;  beta = rr_{j+1} / rr_j;  p = r + beta p,
// with FP64 dot products summed in a fixed order.  The iteration index of a
// system within a chunk is its count at the chunk's start plus the step, so no
// kernel reads a counter that another block of the same launch writes.
#include "cg_common.h"

#include <algorithm>

tt_status cg_replace(tt_ctx& c, const float* s, bool f32, int it, bool* converged, CgScalars* hS);

namespace {

constexpr int VT = 256;   // threads of a vector block
constexpr int VB = 64;    // vector blocks per system

struct BVec {
    float* x;
    float* r;
    float* p;
    const float* q;
    double* partA;   // VB partials of p . q
    double* partB;   // VB partials of r . r
    CgScalars* S;
    long n;
    int it0;         // iterations done at the start of the chunk
    int pad;
};

__device__ double vblock_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ double vsum_partials(const double* __restrict__ part, double* red) {
    double v = 0.0;
    for (int i = threadIdx.x; i < VB; i += VT) v += part[i];
    return vblock_sum(v, red);
}

// grid (VB, systems): partA = p . q of this block's share
__global__ __launch_bounds__(VT) void k_bdot(const BVec* __restrict__ vs) {
    __shared__ double red[VT];
    const BVec d = vs[blockIdx.y];
    if (d.S->state != ST_RUN) return;
    double v = 0.0;
    for (long i = (long)blockIdx.x * VT + threadIdx.x; i < d.n; i += (long)VB * VT)
        v += (double)d.p[i] * (double)d.q[i];
    const double s = vblock_sum(v, red);
    if (threadIdx.x == 0) d.partA[blockIdx.x] = s;
}

__global__ __launch_bounds__(VT) void k_bupdate_xr(const BVec* __restrict__ vs, int step) {
    __shared__ double red[VT];
    const BVec d = vs[blockIdx.y];
    CgScalars* S = d.S;
    if (S->state != ST_RUN) return;
    const int it = d.it0 + step;
    const double pAp = vsum_partials(d.partA, red);
    const double alpha = S->rr[it & 1] / pAp;
    if (!(pAp > 0.0) || !isfinite(alpha)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S->state = ST_BREAK;
            S->pAp = pAp;
        }
        return;
    }
    const float a = (float)alpha;
    double v = 0.0;
    for (long i = (long)blockIdx.x * VT + threadIdx.x; i < d.n; i += (long)VB * VT) {
        d.x[i] += a * d.p[i];
        const float ri = d.r[i] - a * d.q[i];
        d.r[i] = ri;
        v += (double)ri * (double)ri;
    }
    const double s = vblock_sum(v, red);
    if (threadIdx.x == 0) d.partB[blockIdx.x] = s;
    if (blockIdx.x == 0 && threadIdx.x == 0) S->pAp = pAp;
}

__global__ __launch_bounds__(VT) void k_bupdate_p(const BVec* __restrict__ vs, int step, int max_iter) {
    __shared__ double red[VT];
    const BVec d = vs[blockIdx.y];
    CgScalars* S = d.S;
    if (S->state != ST_RUN) return;
    const int it = d.it0 + step;
    const double rn = vsum_partials(d.partB, red);
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
    const float beta = (float)(rn / ro);
    for (long i = (long)blockIdx.x * VT + threadIdx.x; i < d.n; i += (long)VB * VT) d.p[i] = d.r[i] + beta * d.p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S->rr[(it + 1) & 1] = rn;
        S->iter = it + 1;
    }
}

// the solver scalars of every system, gathered for one copy to the host
__global__ void k_bgather(const BVec* __restrict__ vs, int count, CgScalars* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = *vs[i].S;
}

}  // namespace

// Lockstep FP32 CG over systems[0..count) (contexts already validated: ready,
// distinct, one device, no mode removal); infos[i] and zeta[i] as tt_solve_frame.
// Returns TT_OK, or the first runtime error; per-system outcomes are in
// infos[i].status.
tt_status solve_batched(tt_ctx* const* systems, int count, const float* const* d_s, const double* const* d_x0,
                        double* const* d_zeta, const tt_solve_opts& o, tt_solve_info* infos) {
    if (count == 0) return TT_OK;
    tt_ctx& c0 = *systems[0];
    std::vector<CgScalars> h(count);
    std::vector<int> have_true(count, 0), done(count, 0), code(count, TT_OK), refinements(count, 0);
    for (int i = 0; i < count; ++i) {
        tt_ctx& c = *systems[i];
        TT_CHECK(cg_setup(c, d_s[i], d_x0 ? d_x0[i] : nullptr, o, true));
        TT_HIP(hipMemcpyAsync(&h[i], c.scal.p, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
        TT_HIP(hipStreamSynchronize(c.stream));
        if (h[i].bnorm2 == 0.0 || h[i].rr_true <= h[i].tol2) {
            done[i] = 1;
            have_true[i] = 1;
        }
    }
    DevBuf<BVec> dvec;
    DevBuf<CgScalars> dS;
    TT_CHECK(dvec.alloc((size_t)count));
    TT_CHECK(dS.alloc((size_t)count));
    std::vector<BVec> hv;
    std::vector<tt_ctx*> act;
    std::vector<int> idx;
    std::vector<const float*> px;
    std::vector<float*> qy;
    const int chunk = 16;
    while (true) {
        act.clear();
        idx.clear();
        hv.clear();
        px.clear();
        qy.clear();
        for (int i = 0; i < count; ++i) {
            if (done[i]) continue;
            tt_ctx& c = *systems[i];
            act.push_back(&c);
            idx.push_back(i);
            hv.push_back(BVec{c.x32.p, c.r32.p, c.p32.p, c.q32.p, c.part.p, c.part.p + VB, cg_scalars(c),
                              (long)c.n_slopes, h[i].iter, 0});
            px.push_back(c.p32.p);
            qy.push_back(c.q32.p);
        }
        const int na = (int)act.size();
        if (na == 0) break;
        TT_HIP(hipMemcpyAsync(dvec.p, hv.data(), sizeof(BVec) * na, hipMemcpyHostToDevice, c0.stream));
        for (int k = 0; k < chunk; ++k) {
            TT_CHECK(matvec_batch(act.data(), na, px.data(), qy.data(), nullptr));
            hipLaunchKernelGGL(k_bdot, dim3(VB, na), dim3(VT), 0, c0.stream, dvec.p);
            hipLaunchKernelGGL(k_bupdate_xr, dim3(VB, na), dim3(VT), 0, c0.stream, dvec.p, k);
            hipLaunchKernelGGL(k_bupdate_p, dim3(VB, na), dim3(VT), 0, c0.stream, dvec.p, k, o.max_iter);
        }
        hipLaunchKernelGGL(k_bgather, dim3(cdiv(na, 64)), dim3(64), 0, c0.stream, dvec.p, na, dS.p);
        TT_HIP(hipGetLastError());
        std::vector<CgScalars> g(na);
        TT_HIP(hipMemcpyAsync(g.data(), dS.p, sizeof(CgScalars) * na, hipMemcpyDeviceToHost, c0.stream));
        TT_HIP(hipStreamSynchronize(c0.stream));
        for (int a = 0; a < na; ++a) {
            const int i = idx[a];
            tt_ctx& c = *systems[i];
            h[i] = g[a];
            const int it = h[i].iter;
            if (h[i].state == ST_BREAK) {
                code[i] = TT_BREAKDOWN;
                done[i] = 1;
            } else if (h[i].state == ST_CAP || (h[i].state == ST_RUN && it >= o.max_iter)) {
                code[i] = TT_NOT_CONVERGED;
                done[i] = 1;
            } else if (h[i].state == ST_REFINE || h[i].state == ST_CONV) {
                bool conv = false;
                TT_CHECK(cg_replace(c, d_s[i], true, it, &conv, &h[i]));
                refinements[i]++;
                if (conv) {
                    have_true[i] = 1;
                    done[i] = 1;
                } else if (it >= o.max_iter) {
                    have_true[i] = 1;
                    code[i] = TT_NOT_CONVERGED;
                    done[i] = 1;
                } else {
                    // restarted: its scalars on the device are current again
                    TT_HIP(hipMemcpyAsync(&h[i], c.scal.p, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
                    TT_HIP(hipStreamSynchronize(c.stream));
                }
            }
        }
    }
    for (int i = 0; i < count; ++i) {
        tt_ctx& c = *systems[i];
        tt_solve_info inf{};
        TT_CHECK(cg_finish(c, d_s[i], d_zeta[i], true, have_true[i] != 0, inf, code[i]));
        inf.refinements = refinements[i];
        if (infos) infos[i] = inf;
    }
    return TT_OK;
}
