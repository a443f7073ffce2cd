// Frames of many systems solved together (TT_SOLVER_BATCHED): conjugate
// gradients (§2.G) run in lockstep over every system still iterating,
// each iteration's products by one batched 2RBT product (batch.hip) and the
// vector updates by kernels over all systems at once; the FP64 residual
// replacement and the certification of the tolerance are those of the single-system
// path (cg.hip), per system, between chunks of iterations.
//
// Plain CG, per system the recurrences of TT_SOLVER_KERNELS in FP32:
//   q = A p;  alpha = rr_j / (p . q);  x += alpha p;  r -= alpha q;
//   rr_{j+1} = r . r;  beta = rr_{j+1} / rr_j;  p = r + beta p.
// Preconditioned by the block-circulant inverse P (batched as the product):
//   q = A p;  alpha = ru_j / (p . q);  x += alpha p;  r -= alpha q;  u = P r;
//   ru_{j+1} = r . u;  beta = ru_{j+1} / ru_j;  p = u + beta p,
// restarted from p = u = P r at every residual replacement; the stopping and
// replacement tests use r . r as in plain CG.
// Preconditioned by the learned network (TT_PRECOND_LEARNED), flexible CG:
// the same with beta = r_{j+1} . (u_{j+1} - u_j) / ru_j (Polak-Ribiere), u_j
// kept between iterations; a system whose r . u is not positive or finite, or
// whose recursive residual has made no new minimum for 256 iterations, falls
// back to plain CG (u = r) from its FP64 true residual.  FP64 dot products are summed in
// a fixed order.  The iteration index of a system within a chunk is its count
// at the chunk's start plus the step, and the scalars of iteration j + 1 go to
// the other parity slot, so no kernel reads a value another block of the same
// launch writes.
#include "cg_common.h"

#include <algorithm>
#include <memory>

tt_status cg_replace(tt_ctx& c, const float* s, bool f32, int it, bool* converged, CgScalars* hS);

namespace {

constexpr int VT = 256;   // threads of a vector block
constexpr int VB = 64;    // vector blocks per system

struct BVec {
    float* x;
    float* r;
    float* p;
    const float* q;
    const float* u;  // P r (preconditioned)
    float* uo;       // the previous u (flexible CG)
    double* partA;   // VB partials of p . q
    double* partB;   // VB partials of r . r
    double* partC;   // VB partials of r . u
    double* partD;   // VB partials of r . uo (flexible CG)
    CgScalars* S;
    long n;
    int it0;         // iterations done at the start of the chunk
    int flex;        // flexible CG (Polak-Ribiere beta)
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

// grid (VB, systems): partC = r . u of this block's share (running systems, or
// every system that has not stopped for good when starting)
__global__ __launch_bounds__(VT) void k_bdot_ru(const BVec* __restrict__ vs, int starting) {
    __shared__ double red[VT];
    const BVec d = vs[blockIdx.y];
    const int st = d.S->state;
    if (starting ? (st == ST_BREAK || st == ST_CAP) : st != ST_RUN) return;
    double v = 0.0, w = 0.0;
    for (long i = (long)blockIdx.x * VT + threadIdx.x; i < d.n; i += (long)VB * VT) {
        v += (double)d.r[i] * (double)d.u[i];
        if (d.flex && !starting) w += (double)d.r[i] * (double)d.uo[i];
    }
    const double s = vblock_sum(v, red);
    if (threadIdx.x == 0) d.partC[blockIdx.x] = s;
    if (d.flex && !starting) {
        const double t = vblock_sum(w, red);
        if (threadIdx.x == 0) d.partD[blockIdx.x] = t;
    }
}

// (re)start of preconditioned CG at iteration it0: p = u, ru = r . u, and the
// replacement bookkeeping (rr of this iteration = the FP64 true residual)
__global__ __launch_bounds__(VT) void k_bpc_start(const BVec* __restrict__ vs) {
    __shared__ double red[VT];
    const BVec d = vs[blockIdx.y];
    CgScalars* S = d.S;
    if (S->state == ST_BREAK || S->state == ST_CAP) return;
    const double ru = vsum_partials(d.partC, red);
    if (!(ru > 0.0) || !isfinite(ru)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) S->state = ST_BREAK;
        return;
    }
    for (long i = (long)blockIdx.x * VT + threadIdx.x; i < d.n; i += (long)VB * VT) {
        d.p[i] = d.u[i];
        if (d.flex) d.uo[i] = d.u[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S->ru[d.it0 & 1] = ru;
        S->rr[d.it0 & 1] = S->rr_true;
        S->rr_max = S->rr_true;
        S->state = ST_RUN;
    }
}

template <bool PC>
__global__ __launch_bounds__(VT) void k_bupdate_xr(const BVec* __restrict__ vs, int step) {
    __shared__ double red[VT];
    const BVec d = vs[blockIdx.y];
    CgScalars* S = d.S;
    if (S->state != ST_RUN) return;
    const int it = d.it0 + step;
    const double pAp = vsum_partials(d.partA, red);
    const double alpha = (PC ? S->ru[it & 1] : S->rr[it & 1]) / pAp;
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

__global__ __launch_bounds__(VT) void k_bupdate_p_pc(const BVec* __restrict__ vs, int step, int max_iter) {
    __shared__ double red[VT];
    const BVec d = vs[blockIdx.y];
    CgScalars* S = d.S;
    if (S->state != ST_RUN) return;
    const int it = d.it0 + step;
    const double rn = vsum_partials(d.partB, red);
    const double run = vsum_partials(d.partC, red);
    const bool conv = rn <= S->tol2;
    const bool refine = S->drop2 > 0.0 && rn < S->drop2 * S->rr_max;
    const bool cap = it + 1 >= max_iter;
    const bool bad = !isfinite(rn) || !(run > 0.0) || !isfinite(run);
    if (conv || refine || cap || bad) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S->rr[(it + 1) & 1] = rn;
            S->iter = it + 1;
            S->state = bad ? ST_BREAK : conv ? ST_CONV : refine ? ST_REFINE : ST_CAP;
        }
        return;
    }
    const double rdo = d.flex ? vsum_partials(d.partD, red) : 0.0;
    const float beta = (float)((run - rdo) / S->ru[it & 1]);
    for (long i = (long)blockIdx.x * VT + threadIdx.x; i < d.n; i += (long)VB * VT) {
        d.p[i] = d.u[i] + beta * d.p[i];
        if (d.flex) d.uo[i] = d.u[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S->rr[(it + 1) & 1] = rn;
        S->ru[(it + 1) & 1] = run;
        S->iter = it + 1;
    }
}

// u = r (plain CG in the preconditioned recurrences), for the systems that fell back
__global__ __launch_bounds__(VT) void k_bcopy_ru(const BVec* __restrict__ vs, const int* __restrict__ which,
                                                int starting) {
    const BVec d = vs[which[blockIdx.y]];
    const int st = d.S->state;
    if (starting ? (st == ST_BREAK || st == ST_CAP) : st != ST_RUN) return;
    float* u = const_cast<float*>(d.u);
    for (long i = (long)blockIdx.x * VT + threadIdx.x; i < d.n; i += (long)VB * VT) u[i] = d.r[i];
}

// a system that falls back to plain CG resumes iterating
__global__ void k_resume(CgScalars* S) { S->state = ST_RUN; }

// the solver scalars of every system, gathered for one copy to the host
__global__ void k_bgather(const BVec* __restrict__ vs, int count, CgScalars* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = *vs[i].S;
}


// u = P r for the systems act[0..na) (their BVec at dvec[0..na), on stream st):
// the block-circulant inverse batched (mode TT_PRECOND_CIRCULANT), or the
// learned network (TT_PRECOND_LEARNED) batched over runs of systems sharing the
// network and the valid subapertures, with u = r for the systems in fb (those
// fallen back to plain CG, indices into act, uploaded at dfb).
struct PcPlan {
    int mode = 0;
    int prec = TT_PREC_F32;                  // storage precision of the block-circulant spectra
    std::vector<std::pair<int, int>> runs;   // learned: [begin, end) of act sharing a network and geometry
    std::vector<int> fb;                     // fallen back: indices into act
    DevBuf<int> dfb;
};

tt_status plan_precond(PcPlan& plan, tt_ctx* const* act, int na, const std::vector<int>& fallback_of_act,
                       hipStream_t st) {
    plan.runs.clear();
    plan.fb.clear();
    if (plan.mode != TT_PRECOND_LEARNED) return TT_OK;
    int a = 0;
    while (a < na) {
        if (fallback_of_act[a]) {
            plan.fb.push_back(a++);
            continue;
        }
        int b = a + 1;
        while (b < na && !fallback_of_act[b] && act[b]->learned == act[a]->learned && act[b]->n == act[a]->n &&
               act[b]->valid == act[a]->valid)
            ++b;
        plan.runs.push_back({a, b});
        a = b;
    }
    if (!plan.fb.empty()) {
        if (plan.dfb.n < plan.fb.size()) TT_CHECK(plan.dfb.alloc(std::max<size_t>(plan.fb.size(), 64)));
        TT_HIP(hipMemcpyAsync(plan.dfb.p, plan.fb.data(), sizeof(int) * plan.fb.size(), hipMemcpyHostToDevice, st));
    }
    return TT_OK;
}

// desc / tables: the descriptor and pointer tables the launches read (null: the
// shared defaults; a caller capturing the launches passes its own, one table
// per run of the learned network)
tt_status apply_precond(const PcPlan& plan, tt_ctx* const* act, int na, const float* const* pr, float* const* pu,
                        const BVec* dvec, int starting, hipStream_t st, HostMirror<unsigned char>* desc = nullptr,
                        std::vector<std::unique_ptr<HostMirror<float*>>>* tables = nullptr) {
    if (plan.mode == TT_PRECOND_CIRCULANT) return batch_apply(act, na, pr, pu, 1, nullptr, plan.prec, 0, desc);
    while (tables && tables->size() < plan.runs.size()) tables->emplace_back(new HostMirror<float*>());
    for (size_t r = 0; r < plan.runs.size(); ++r) {
        const auto& run = plan.runs[r];
        TT_CHECK(learned_apply_batch(*act[run.first]->learned, *act[run.first], pr + run.first, pu + run.first,
                                     run.second - run.first, st, tables ? (*tables)[r].get() : nullptr));
    }
    if (!plan.fb.empty()) {
        hipLaunchKernelGGL(k_bcopy_ru, dim3(VB, (unsigned)plan.fb.size()), dim3(VT), 0, st, dvec, plan.dfb.p,
                           starting);
        TT_HIP(hipGetLastError());
    }
    return TT_OK;
}

// Preconditioned start of the systems in vs (count of them, on stream st):
// u = P r, ru = r . u, p = u.
tt_status pc_start(const PcPlan& plan, tt_ctx* const* act, int na, const std::vector<const float*>& pr,
                   const std::vector<float*>& pu, const BVec* dvec, hipStream_t st) {
    TT_CHECK(apply_precond(plan, act, na, pr.data(), pu.data(), dvec, 1, st));
    hipLaunchKernelGGL(k_bdot_ru, dim3(VB, na), dim3(VT), 0, st, dvec, 1);
    hipLaunchKernelGGL(k_bpc_start, dim3(VB, na), dim3(VT), 0, st, dvec);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

BVec bvec_of(tt_ctx& c, int it0, bool flex) {
    return BVec{c.x32.p,      c.r32.p,          c.p32.p,          c.q32.p,          c.bu32.p,      c.bu_old32.p,
                c.part.p,     c.part.p + VB,    c.part.p + 2 * VB, c.part.p + 3 * VB, cg_scalars(c), (long)c.n_slopes,
                it0,          flex ? 1 : 0};
}

}  // namespace

// Lockstep FP32 CG (plain, preconditioned by the block-circulant inverse, or
// flexible with the learned preconditioner) over systems[0..count) (contexts
// already validated: ready, distinct, one device, no mode removal); infos[i]
// and zeta[i] as tt_solve_frame.  Returns TT_OK, or the first runtime error;
// per-system outcomes are in infos[i].status.
tt_status solve_batched(tt_ctx* const* systems, int count, const float* const* d_s, const double* const* d_x0,
                        double* const* d_zeta, const tt_solve_opts& o, tt_solve_info* infos) {
    if (count == 0) return TT_OK;
    const int mode = o.preconditioner;
    const bool pc = mode != TT_PRECOND_NONE;
    const bool flex = mode == TT_PRECOND_LEARNED;
    constexpr int STALL = 256;   // learned: iterations without a new minimum of r.r before the fallback
    std::vector<CgScalars> h(count);
    std::vector<int> have_true(count, 0), done(count, 0), code(count, TT_OK), refinements(count, 0);
    std::vector<int> fallback(count, 0), fb_iter(count, -1), best_it(count, 0);
    std::vector<double> best_rr(count, 0.0);
    for (int i = 0; i < count; ++i) {
        tt_ctx& c = *systems[i];
        if (mode == TT_PRECOND_CIRCULANT) TT_CHECK(precond_build(c));
        if (pc && c.bu32.n < (size_t)c.n_slopes) TT_CHECK(c.bu32.alloc(c.n_slopes));
        if (flex && c.bu_old32.n < (size_t)c.n_slopes) TT_CHECK(c.bu_old32.alloc(c.n_slopes));
        TT_CHECK(cg_setup(c, d_s[i], d_x0 ? d_x0[i] : nullptr, o, true));
        TT_HIP(hipMemcpyAsync(&h[i], c.scal.p, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
        TT_HIP(hipStreamSynchronize(c.stream));
        best_rr[i] = h[i].rr_true;
        best_it[i] = h[i].iter;
        if (h[i].bnorm2 == 0.0 || h[i].rr_true <= h[i].tol2) {
            done[i] = 1;
            have_true[i] = 1;
        }
    }
    DevBuf<BVec> dvec, d1;
    DevBuf<CgScalars> dS;
    TT_CHECK(dvec.alloc((size_t)count));
    TT_CHECK(d1.alloc(1));
    TT_CHECK(dS.alloc((size_t)count));
    std::vector<BVec> hv;
    std::vector<tt_ctx*> act;
    std::vector<int> idx, fb_act;
    std::vector<const float*> px, pr;
    std::vector<float*> qy, pu;
    PcPlan plan, plan1;
    plan.mode = plan1.mode = mode;
    plan.prec = plan1.prec = o.precision;   // FP16 / BF16: the preconditioner's spectra only
    auto gather_active = [&]() {
        for (int i = 0; i < count; ++i)   // iteration cap reached (max_iter 0 included)
            if (!done[i] && h[i].iter >= o.max_iter) {
                code[i] = TT_NOT_CONVERGED;
                done[i] = 1;
            }
        act.clear();
        idx.clear();
        hv.clear();
        px.clear();
        qy.clear();
        pr.clear();
        pu.clear();
        fb_act.clear();
        for (int i = 0; i < count; ++i) {
            if (done[i]) continue;
            tt_ctx& c = *systems[i];
            act.push_back(&c);
            idx.push_back(i);
            hv.push_back(bvec_of(c, h[i].iter, flex));
            px.push_back(c.p32.p);
            qy.push_back(c.q32.p);
            pr.push_back(c.r32.p);
            pu.push_back(c.bu32.p);
            fb_act.push_back(fallback[i]);
        }
    };
    // restart system i from its FP64 true residual: r = r64, p = u = P r (u = r
    // after a fallback); refreshes h[i]
    auto restart = [&](int i, int it) -> tt_status {
        tt_ctx& c = *systems[i];
        TT_CHECK(cg_copy_r64_to_r32(c));
        tt_ctx* one[1] = {&c};
        const BVec b1 = bvec_of(c, it, flex);
        TT_HIP(hipMemcpyAsync(d1.p, &b1, sizeof(BVec), hipMemcpyHostToDevice, c.stream));
        std::vector<int> f1(1, fallback[i]);
        if (fallback[i]) hipLaunchKernelGGL(k_resume, dim3(1), dim3(1), 0, c.stream, cg_scalars(c));
        TT_CHECK(plan_precond(plan1, one, 1, f1, c.stream));
        TT_CHECK(pc_start(plan1, one, 1, {c.r32.p}, {c.bu32.p}, d1.p, c.stream));
        TT_HIP(hipMemcpyAsync(&h[i], c.scal.p, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
        TT_HIP(hipStreamSynchronize(c.stream));
        return TT_OK;
    };
    // the batched launches go to the stream of the first system still iterating
    // (batch_apply uses it too)
    if (pc) {   // p = u = P r for every system that iterates
        gather_active();
        const int na = (int)act.size();
        if (na > 0) {
            const hipStream_t st = act[0]->stream;
            TT_HIP(hipMemcpyAsync(dvec.p, hv.data(), sizeof(BVec) * na, hipMemcpyHostToDevice, st));
            TT_CHECK(plan_precond(plan, act.data(), na, fb_act, st));
            TT_CHECK(pc_start(plan, act.data(), na, pr, pu, dvec.p, st));
            TT_HIP(hipStreamSynchronize(st));
            if (flex) {   // a network that is not positive on the right-hand side: plain CG from the start
                std::vector<CgScalars> g(na);
                hipLaunchKernelGGL(k_bgather, dim3(cdiv(na, 64)), dim3(64), 0, st, dvec.p, na, dS.p);
                TT_HIP(hipMemcpyAsync(g.data(), dS.p, sizeof(CgScalars) * na, hipMemcpyDeviceToHost, st));
                TT_HIP(hipStreamSynchronize(st));
                for (int a = 0; a < na; ++a) {
                    const int i = idx[a];
                    h[i] = g[a];
                    if (h[i].state == ST_BREAK) {
                        fallback[i] = 1;
                        fb_iter[i] = h[i].iter;
                        TT_CHECK(cg_true_residual(*systems[i], d_s[i], true, &h[i]));
                        TT_CHECK(restart(i, h[i].iter));
                    }
                }
            }
        }
    }
    const int chunk = 16;
    // HIP graph of one chunk (opts.graph): captured at the second chunk with an
    // unchanged set of iterating systems (the first one, launched eagerly, has
    // uploaded every descriptor and grown every buffer the chunk uses) and
    // replayed while the set stays the same; the per-chunk descriptors (the
    // iteration indices) are uploaded before each replay.
    hipGraphExec_t gexec = nullptr;
    std::vector<int> g_idx, g_seen;
    // the tables the chunk's launches read, owned by this solve: the restarts of
    // single systems between chunks use the shared ones and cannot overwrite them
    HostMirror<unsigned char> gdesc[2];
    std::vector<std::unique_ptr<HostMirror<float*>>> gtab;
    struct GraphGuard {
        hipGraphExec_t* e;
        ~GraphGuard() {
            if (*e) (void)hipGraphExecDestroy(*e);
        }
    } gguard{&gexec};
    while (true) {
        gather_active();
        const int na = (int)act.size();
        if (na == 0) break;
        const hipStream_t st = act[0]->stream;
        TT_HIP(hipMemcpyAsync(dvec.p, hv.data(), sizeof(BVec) * na, hipMemcpyHostToDevice, st));
        if (pc) TT_CHECK(plan_precond(plan, act.data(), na, fb_act, st));
        bool replay = false, capture = false;
        if (o.graph) {
            if (gexec && g_idx == idx && fb_act == g_seen) {
                replay = true;
            } else {
                if (gexec) {
                    TT_HIP(hipGraphExecDestroy(gexec));
                    gexec = nullptr;
                }
                capture = !g_idx.empty() && g_idx == idx && fb_act == g_seen;
                g_idx = idx;
                g_seen = fb_act;
            }
        }
        // graph mode: the chunk runs on a capturable stream of the first system
        // (the context's own stream may be the null stream), ordered after the
        // uploads above and before the gather below by events
        hipStream_t run_st = st;
        struct StreamSwap {
            tt_ctx* c;
            hipStream_t orig;
            ~StreamSwap() {
                if (c) c->stream = orig;
            }
        } swap{nullptr, st};
        if (o.graph) {
            tt_ctx& c0 = *act[0];
            if (!c0.gstream) TT_HIP(hipStreamCreateWithFlags(&c0.gstream, hipStreamNonBlocking));
            for (auto& e : c0.gev)
                if (!e) TT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            TT_HIP(hipEventRecord(c0.gev[0], st));
            TT_HIP(hipStreamWaitEvent(c0.gstream, c0.gev[0], 0));
            run_st = c0.gstream;
            swap.c = &c0;
            c0.stream = run_st;   // batch_apply launches on the first system's stream
        }
        if (capture) TT_HIP(hipStreamBeginCapture(run_st, hipStreamCaptureModeRelaxed));
        // a failure while capturing ends the capture before it is returned
        struct CaptureGuard {
            hipStream_t s;
            bool on;
            ~CaptureGuard() {
                if (on) {
                    hipGraph_t g = nullptr;
                    if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
                }
            }
        } cguard{run_st, capture};
        HostMirror<unsigned char>* d0 = o.graph ? &gdesc[0] : nullptr;
        HostMirror<unsigned char>* d1 = o.graph ? &gdesc[1] : nullptr;
        std::vector<std::unique_ptr<HostMirror<float*>>>* tabs = o.graph ? &gtab : nullptr;
        for (int k = 0; k < chunk && !replay; ++k) {
            TT_CHECK(batch_apply(act.data(), na, px.data(), qy.data(), 0, nullptr, TT_PREC_F32, 0, d0));
            hipLaunchKernelGGL(k_bdot, dim3(VB, na), dim3(VT), 0, run_st, dvec.p);
            if (pc) {
                hipLaunchKernelGGL(k_bupdate_xr<true>, dim3(VB, na), dim3(VT), 0, run_st, dvec.p, k);
                TT_CHECK(apply_precond(plan, act.data(), na, pr.data(), pu.data(), dvec.p, 0, run_st, d1, tabs));
                hipLaunchKernelGGL(k_bdot_ru, dim3(VB, na), dim3(VT), 0, run_st, dvec.p, 0);
                hipLaunchKernelGGL(k_bupdate_p_pc, dim3(VB, na), dim3(VT), 0, run_st, dvec.p, k, o.max_iter);
            } else {
                hipLaunchKernelGGL(k_bupdate_xr<false>, dim3(VB, na), dim3(VT), 0, run_st, dvec.p, k);
                hipLaunchKernelGGL(k_bupdate_p, dim3(VB, na), dim3(VT), 0, run_st, dvec.p, k, o.max_iter);
            }
        }
        if (capture) {
            hipGraph_t graph = nullptr;
            cguard.on = false;
            TT_HIP(hipStreamEndCapture(run_st, &graph));
            const hipError_t e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            TT_HIP(e);
            replay = true;
        }
        if (replay) TT_HIP(hipGraphLaunch(gexec, run_st));
        if (o.graph) {
            tt_ctx& c0 = *act[0];
            c0.stream = st;
            swap.c = nullptr;
            TT_HIP(hipEventRecord(c0.gev[1], run_st));
            TT_HIP(hipStreamWaitEvent(st, c0.gev[1], 0));
        }
        hipLaunchKernelGGL(k_bgather, dim3(cdiv(na, 64)), dim3(64), 0, st, dvec.p, na, dS.p);
        TT_HIP(hipGetLastError());
        std::vector<CgScalars> g(na);
        TT_HIP(hipMemcpyAsync(g.data(), dS.p, sizeof(CgScalars) * na, hipMemcpyDeviceToHost, st));
        TT_HIP(hipStreamSynchronize(st));
        for (int a = 0; a < na; ++a) {
            const int i = idx[a];
            tt_ctx& c = *systems[i];
            h[i] = g[a];
            const int it = h[i].iter;
            // learned preconditioner: fall back to plain CG on a breakdown of the
            // flexible recurrences or a stall of the recursive residual
            if (flex && !fallback[i]) {
                const double rr = h[i].rr[it & 1];
                if (h[i].state == ST_RUN && rr < best_rr[i]) {
                    best_rr[i] = rr;
                    best_it[i] = it;
                }
                const bool stall = h[i].state == ST_RUN && it - best_it[i] >= STALL;
                if (h[i].state == ST_BREAK || stall) {
                    fallback[i] = 1;
                    fb_iter[i] = it;
                    TT_CHECK(cg_true_residual(c, d_s[i], true, &h[i]));
                    refinements[i]++;
                    if (h[i].rr_true <= h[i].tol2) {
                        have_true[i] = 1;
                        done[i] = 1;
                        continue;
                    }
                    TT_CHECK(restart(i, it));
                    if (h[i].state == ST_BREAK) {
                        code[i] = TT_BREAKDOWN;
                        done[i] = 1;
                    }
                    continue;
                }
            }
            if (h[i].state == ST_BREAK) {
                code[i] = TT_BREAKDOWN;
                done[i] = 1;
            } else if (h[i].state == ST_CAP || (h[i].state == ST_RUN && it >= o.max_iter)) {
                code[i] = TT_NOT_CONVERGED;
                done[i] = 1;
            } else if (h[i].state == ST_REFINE || h[i].state == ST_CONV) {
                bool conv = false;
                if (pc) {
                    TT_CHECK(cg_true_residual(c, d_s[i], true, &h[i]));
                    conv = h[i].rr_true <= h[i].tol2;
                } else {
                    TT_CHECK(cg_replace(c, d_s[i], true, it, &conv, &h[i]));
                }
                refinements[i]++;
                if (conv) {
                    have_true[i] = 1;
                    done[i] = 1;
                } else if (it >= o.max_iter) {
                    have_true[i] = 1;
                    code[i] = TT_NOT_CONVERGED;
                    done[i] = 1;
                } else {
                    if (pc) {   // restart from the true residual: r = r64, p = u = P r
                        TT_CHECK(restart(i, it));
                        if (flex) {   // the replacement is a new minimum of the residual
                            best_rr[i] = h[i].rr_true;
                            best_it[i] = it;
                        }
                    } else {
                        // restarted: its scalars on the device are current again
                        TT_HIP(hipMemcpyAsync(&h[i], c.scal.p, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
                        TT_HIP(hipStreamSynchronize(c.stream));
                    }
                    if (h[i].state == ST_BREAK) {
                        if (flex && !fallback[i]) {
                            fallback[i] = 1;
                            fb_iter[i] = it;
                            TT_CHECK(restart(i, it));
                        }
                        if (h[i].state == ST_BREAK) {
                            code[i] = TT_BREAKDOWN;
                            done[i] = 1;
                        }
                    }
                }
            }
        }
    }
    for (int i = 0; i < count; ++i) {
        tt_ctx& c = *systems[i];
        tt_solve_info inf{};
        TT_CHECK(cg_finish(c, d_s[i], d_zeta[i], true, have_true[i] != 0, inf, code[i]));
        inf.refinements = refinements[i];
        inf.fallback = fb_iter[i];
        if (infos) infos[i] = inf;
    }
    return TT_OK;
}
