// Covariance generation in float64 on the device (App. A.2 / A.3).
//
// Slope-slope tables (App. A.2 Hudgin-like slope-slope equations, or the App.
// A.3 Fried equations, §2.D cone scaling): for every unordered guide-star pair g <= h, component c in
// {xx, xy (= yx), yy} and subaperture lag (U, V) in [-(n-1), n-1]^2 (U column,
// V row, of the second slope relative to the first)
//
//   t(U, V) = sum_k w_k Hud_c(Delta_k; delta_k),
//   Delta_k = s_k (U d, V d) + h_k (alpha_h - alpha_g),  delta_k = s_k d,
//   xx(D) = 1/2[-2 D(D) + D(D + delta x) + D(D - delta x)],  yy with y,
//   xy(D) = 1/2[D(D + delta(x+y)/2) - D(D + delta(-x+y)/2)
//               - D(D + delta(x-y)/2) + D(D - delta(x+y)/2)]
//
// (reading of the printed xy sign: "+" on the last term, which the product of
// the two phase differences gives and which makes xy(0) = 0).
//
// Phase-slope tables of the projection (App. A.2 Hudgin phase-slope equation
// on the per-layer grids of §2.D): for layer k, channel q = (g, p) and lag
// (U, V) in [-(n'-1), n-1]^2 (subaperture index minus grid index)
//
//   t'(U, V) = w_k 1/2 [D(Delta - delta e_p/2) - D(Delta + delta e_p/2)],
//   Delta = s_k d (U + (n'-n)/2, V + (n'-n)/2) + h_k (alpha_g - beta).
#include "tt_internal.h"
#include "vk_math.h"

namespace {

__constant__ double c_trap_a[vk::NTRAP];
__constant__ double c_trap_b[vk::NTRAP];

tt_status upload_trap(hipStream_t s) {
    static const vk::Trap t = vk::make_trap();
    TT_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_trap_a), t.a, sizeof(t.a), 0, hipMemcpyHostToDevice, s));
    TT_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_trap_b), t.b, sizeof(t.b), 0, hipMemcpyHostToDevice, s));
    return TT_OK;
}

__device__ inline double Dfun(double dx, double dy, const vk::Params& p) {
    return vk::structure(dx, dy, p, c_trap_a, c_trap_b);
}

struct GenArgs {
    int n, G, K, model;
    double d;
    vk::Params vk;
    const double* gs;   // 2G
    const double* h;    // K
    const double* w;    // K
    const double* s;    // K cone factors
};

__global__ void gen_slope_tables(GenArgs a, double* __restrict__ out, long total) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int m = 2 * a.n - 1;
    const int U = (int)(idx % m) - (a.n - 1);
    const int V = (int)((idx / m) % m) - (a.n - 1);
    const int comp = (int)((idx / ((long)m * m)) % 3);
    int pair = (int)(idx / (3L * m * m));
    int g = 0;
    while (pair >= a.G - g) { pair -= a.G - g; ++g; }
    const int hh = g + pair;
    const double bx = a.gs[2 * hh] - a.gs[2 * g];
    const double by = a.gs[2 * hh + 1] - a.gs[2 * g + 1];
    double acc = 0.0;
    for (int k = 0; k < a.K; ++k) {
        const double sk = a.s[k];
        const double dx = sk * U * a.d + a.h[k] * bx;
        const double dy = sk * V * a.d + a.h[k] * by;
        const double del = sk * a.d;
        double v;
        if (a.model == TT_MODEL_FRIED) {
            // App. A.3: 1/8 [-4 D + 2 F1 - 2 F2 + F3 + F4] (xx), [-4 D - 2 F1 + 2 F2 + F3 + F4] (yy),
            // 1/8 (F3 - F4) (xy = yx), slopes in rad
            const double F3 = Dfun(dx + del, dy + del, a.vk) + Dfun(dx - del, dy - del, a.vk);
            const double F4 = Dfun(dx + del, dy - del, a.vk) + Dfun(dx - del, dy + del, a.vk);
            if (comp == 1) {
                v = 0.125 * (F3 - F4);
            } else {
                const double F1 = Dfun(dx + del, dy, a.vk) + Dfun(dx - del, dy, a.vk);
                const double F2 = Dfun(dx, dy + del, a.vk) + Dfun(dx, dy - del, a.vk);
                const double sg = comp == 0 ? 1.0 : -1.0;
                v = 0.125 * (-4.0 * Dfun(dx, dy, a.vk) + sg * (2.0 * F1 - 2.0 * F2) + F3 + F4);
            }
        } else if (comp == 0) {
            v = 0.5 * (-2.0 * Dfun(dx, dy, a.vk) + Dfun(dx + del, dy, a.vk) + Dfun(dx - del, dy, a.vk));
        } else if (comp == 2) {
            v = 0.5 * (-2.0 * Dfun(dx, dy, a.vk) + Dfun(dx, dy + del, a.vk) + Dfun(dx, dy - del, a.vk));
        } else {
            const double e = 0.5 * del;
            v = 0.5 * (Dfun(dx + e, dy + e, a.vk) - Dfun(dx - e, dy + e, a.vk)
                       - Dfun(dx + e, dy - e, a.vk) + Dfun(dx - e, dy - e, a.vk));
        }
        acc += a.w[k] * v;
    }
    out[idx] = acc;
}

struct PhaseArgs {
    int n, np, G, K, model;
    double d, bx, by;
    vk::Params vk;
    const double* gs;
    const double* h;
    const double* w;
    const double* s;
};

__global__ void gen_phase_tables(PhaseArgs a, double* __restrict__ out, long total) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int m = a.np + a.n - 1;
    const int U = (int)(idx % m) - (a.np - 1);
    const int V = (int)((idx / m) % m) - (a.np - 1);
    const int q = (int)((idx / ((long)m * m)) % (2 * a.G));
    const int k = (int)(idx / ((long)m * m * 2 * a.G));
    const int g = q >> 1, p = q & 1;
    const double sk = a.s[k];
    const double off = 0.5 * (a.np - a.n);
    const double dx = sk * a.d * (U + off) + a.h[k] * (a.gs[2 * g] - a.bx);
    const double dy = sk * a.d * (V + off) + a.h[k] * (a.gs[2 * g + 1] - a.by);
    const double e = 0.5 * sk * a.d;
    double v;
    if (a.model == TT_MODEL_FRIED) {
        // App. A.3: 1/4 (-F5 + F6 + F7 - F8) (x), 1/4 (-F5 - F6 + F7 + F8) (y)
        const double F5 = Dfun(dx + e, dy + e, a.vk), F6 = Dfun(dx - e, dy + e, a.vk);
        const double F7 = Dfun(dx - e, dy - e, a.vk), F8 = Dfun(dx + e, dy - e, a.vk);
        v = p == 0 ? 0.25 * (-F5 + F6 + F7 - F8) : 0.25 * (-F5 - F6 + F7 + F8);
    } else if (p == 0) {
        v = 0.5 * (Dfun(dx - e, dy, a.vk) - Dfun(dx + e, dy, a.vk));
    } else {
        v = 0.5 * (Dfun(dx, dy - e, a.vk) - Dfun(dx, dy + e, a.vk));
    }
    out[idx] = a.w[k] * v;
}

std::vector<double> cone_factors(const std::vector<double>& h, bool lgs, double h_lgs) {
    std::vector<double> s(h.size(), 1.0);
    if (lgs)
        for (size_t k = 0; k < h.size(); ++k) s[k] = 1.0 - h[k] / h_lgs;
    return s;
}

}  // namespace

double vk_host_bracket(double x) {
    static const vk::Trap t = vk::make_trap();
    const vk::Params p = vk::make_params(1.0, 1.0);
    return vk::bracket(x, p, t.a, t.b);
}

tt_status gen_tables_launch(const tt_kernels& k, double* d_out, hipStream_t s) {
    TT_CHECK(upload_trap(s));
    DevBuf<double> gs, h, w, sc;
    TT_CHECK(gs.upload(k.gs.data(), k.gs.size(), s));
    TT_CHECK(h.upload(k.h.data(), k.h.size(), s));
    TT_CHECK(w.upload(k.w.data(), k.w.size(), s));
    const std::vector<double> cf = cone_factors(k.h, k.lgs, k.h_lgs);
    TT_CHECK(sc.upload(cf.data(), cf.size(), s));
    GenArgs a;
    a.model = k.model;
    a.n = k.n;
    a.G = k.n_gs;
    a.K = k.n_layer;
    a.d = k.d;
    a.vk = vk::make_params(k.r0, k.L0);
    a.gs = gs.p;
    a.h = h.p;
    a.w = w.p;
    a.s = sc.p;
    const long total = (long)k.count;
    hipLaunchKernelGGL(gen_slope_tables, dim3(cdiv(total, 256)), dim3(256), 0, s, a, d_out, total);
    TT_HIP(hipGetLastError());
    TT_HIP(hipStreamSynchronize(s));   // temporaries are released on return
    return TT_OK;
}

tt_status gen_phase_tables_launch(const tt_ctx& c, int np, double* d_out, hipStream_t s) {
    TT_CHECK(upload_trap(s));
    DevBuf<double> gs, h, w, sc;
    TT_CHECK(gs.upload(c.gs.data(), c.gs.size(), s));
    TT_CHECK(h.upload(c.h.data(), c.h.size(), s));
    TT_CHECK(w.upload(c.w.data(), c.w.size(), s));
    const std::vector<double> cf = cone_factors(c.h, c.lgs, c.h_lgs);
    TT_CHECK(sc.upload(cf.data(), cf.size(), s));
    PhaseArgs a;
    a.model = c.model;
    a.n = c.n;
    a.np = np;
    a.G = c.G;
    a.K = c.n_layer;
    a.d = c.d;
    a.bx = c.proj.beta_x;
    a.by = c.proj.beta_y;
    a.vk = vk::make_params(c.r0, c.L0);
    a.gs = gs.p;
    a.h = h.p;
    a.w = w.p;
    a.s = sc.p;
    const long m = np + c.n - 1;
    const long total = (long)c.n_layer * 2 * c.G * m * m;
    hipLaunchKernelGGL(gen_phase_tables, dim3(cdiv(total, 256)), dim3(256), 0, s, a, d_out, total);
    TT_HIP(hipGetLastError());
    TT_HIP(hipStreamSynchronize(s));
    return TT_OK;
}
