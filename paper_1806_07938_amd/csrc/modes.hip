// Low-order mode removal (§2.F "Mode removal"): per sensor, the projector
// M_s,i = I - Z_s,i Z_s,i^+ that removes tip, tilt and focus from the valid
// slopes, and M_phi removing the same modes from the reconstructed phase.
// With it the system is (M_s W_s)(Sigma_ss + Sigma_eta)(M_s W_s)^T zeta =
// M_s s (zeta in the range of M_s) and phi = M_phi W_phi Sigma_phi_s zeta.
//
// Modes on the valid slopes of one sensor (2 n_vs x 3, Hudgin slopes of the
// phase modes x, y and x^2 + y^2, up to scale): tip (x slopes 1, y slopes 0),
// tilt (0, 1), focus (x, y) with (x, y) the subaperture centre in units of d.
// On the valid phase points: x, y, x^2 + y^2 at the corners.  Z^+ = (Z^T Z)^-1
// Z^T; the 3 x 3 Gram inverses are formed on the host in FP64.
#include "tt_internal.h"

namespace {

constexpr int NTM = 256;

__device__ inline double msum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = NTM / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

struct Gram3 {
    double g[9];   // (Z^T Z)^-1, row-major
};

// v <- v - Z (Z^T Z)^-1 Z^T v for the slopes of sensor blockIdx.x
template <typename R>
__global__ void k_project_slopes(R* __restrict__ v, const float* __restrict__ pos, Gram3 gi, int n_vs) {
    __shared__ double red[NTM];
    R* vx = v + (long)blockIdx.x * 2 * n_vs;
    R* vy = vx + n_vs;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int i = threadIdx.x; i < n_vs; i += NTM) {
        const double a = vx[i], b = vy[i];
        t0 += a;
        t1 += b;
        t2 += pos[2 * i] * a + pos[2 * i + 1] * b;
    }
    t0 = msum(t0, red);
    t1 = msum(t1, red);
    t2 = msum(t2, red);
    const double c0 = gi.g[0] * t0 + gi.g[1] * t1 + gi.g[2] * t2;
    const double c1 = gi.g[3] * t0 + gi.g[4] * t1 + gi.g[5] * t2;
    const double c2 = gi.g[6] * t0 + gi.g[7] * t1 + gi.g[8] * t2;
    for (int i = threadIdx.x; i < n_vs; i += NTM) {
        vx[i] = (R)((double)vx[i] - c0 - c2 * pos[2 * i]);
        vy[i] = (R)((double)vy[i] - c1 - c2 * pos[2 * i + 1]);
    }
}

// phi <- phi - Z_phi (Z_phi^T Z_phi)^-1 Z_phi^T phi, modes x, y, x^2 + y^2
__global__ void k_project_phase(float* __restrict__ phi, const float* __restrict__ pos, Gram3 gi, int m) {
    __shared__ double red[NTM];
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int i = threadIdx.x; i < m; i += NTM) {
        const double x = pos[2 * i], y = pos[2 * i + 1], p = phi[i];
        t0 += x * p;
        t1 += y * p;
        t2 += (x * x + y * y) * p;
    }
    t0 = msum(t0, red);
    t1 = msum(t1, red);
    t2 = msum(t2, red);
    const double c0 = gi.g[0] * t0 + gi.g[1] * t1 + gi.g[2] * t2;
    const double c1 = gi.g[3] * t0 + gi.g[4] * t1 + gi.g[5] * t2;
    const double c2 = gi.g[6] * t0 + gi.g[7] * t1 + gi.g[8] * t2;
    for (int i = threadIdx.x; i < m; i += NTM) {
        const double x = pos[2 * i], y = pos[2 * i + 1];
        phi[i] = (float)((double)phi[i] - c0 * x - c1 * y - c2 * (x * x + y * y));
    }
}

// inverse of a symmetric positive definite 3 x 3 matrix (cofactors)
bool inv3(const double a[9], double out[9]) {
    const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
    const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    out[0] = c00 / det;
    out[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    out[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    out[3] = c01 / det;
    out[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    out[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    out[6] = c02 / det;
    out[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    out[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    return true;
}

Gram3 to_gram(const std::vector<double>& g) {
    Gram3 r;
    for (int i = 0; i < 9; ++i) r.g[i] = g[i];
    return r;
}

}  // namespace

tt_status modes_setup(tt_ctx& c) {
    const int n = c.n;
    // slopes: subaperture centres of the valid subapertures (units of d)
    std::vector<float> pos;
    double sx = 0, sy = 0, sr = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (c.valid[i * n + j]) {
                const double x = j - 0.5 * (n - 1), y = i - 0.5 * (n - 1);
                pos.push_back((float)x);
                pos.push_back((float)y);
                sx += (float)x;
                sy += (float)y;
                sr += (double)(float)x * (float)x + (double)(float)y * (float)y;
            }
    const double nv = (double)c.n_vs;
    const double G[9] = {nv, 0.0, sx, 0.0, nv, sy, sx, sy, sr};
    std::vector<double> gi(9);
    TT_REQUIRE(inv3(G, gi.data()), "tip/tilt/focus are not independent on the valid subapertures");
    TT_CHECK(c.mode_pos.upload(pos.data(), pos.size(), c.stream));
    c.mode_ginv = gi;
    // phase: the valid phase points (units of d)
    c.mode_phase_ginv.clear();
    if (c.proj.on) {
        std::vector<int> vphi(c.proj.n_vphi);
        TT_HIP(hipMemcpyAsync(vphi.data(), c.proj.vphi.p, vphi.size() * sizeof(int), hipMemcpyDeviceToHost, c.stream));
        TT_HIP(hipStreamSynchronize(c.stream));
        std::vector<float> pp;
        double A[9] = {0};
        for (int f : vphi) {
            const double x = (float)(f % (n + 1) - 0.5 * n), y = (float)(f / (n + 1) - 0.5 * n);
            pp.push_back((float)x);
            pp.push_back((float)y);
            const double z[3] = {x, y, x * x + y * y};
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) A[r * 3 + q] += z[r] * z[q];
        }
        std::vector<double> pg(9);
        TT_REQUIRE(inv3(A, pg.data()), "tip/tilt/focus are not independent on the valid phase points");
        TT_CHECK(c.mode_phase_pos.upload(pp.data(), pp.size(), c.stream));
        c.mode_phase_ginv = pg;
    }
    TT_HIP(hipStreamSynchronize(c.stream));
    return TT_OK;
}

tt_status modes_project_f32(tt_ctx& c, float* v) {
    hipLaunchKernelGGL(k_project_slopes<float>, dim3(c.G), dim3(NTM), 0, c.stream, v, c.mode_pos.p,
                       to_gram(c.mode_ginv), c.n_vs);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

tt_status modes_project_f64(tt_ctx& c, double* v) {
    hipLaunchKernelGGL(k_project_slopes<double>, dim3(c.G), dim3(NTM), 0, c.stream, v, c.mode_pos.p,
                       to_gram(c.mode_ginv), c.n_vs);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

tt_status modes_project_phase(tt_ctx& c, float* phi) {
    if (c.mode_phase_ginv.empty()) return TT_OK;
    hipLaunchKernelGGL(k_project_phase, dim3(1), dim3(NTM), 0, c.stream, phi, c.mode_phase_pos.p,
                       to_gram(c.mode_phase_ginv), c.proj.n_vphi);
    TT_HIP(hipGetLastError());
    return TT_OK;
}
