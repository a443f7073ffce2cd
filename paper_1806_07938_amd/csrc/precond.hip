// Block-circulant preconditioner of the masked 2RBT system (set-up, FP64).
//
// The embedded block-circulant operator of the product (§2.E) is
// F^-1 diag_f(M(f)) F with M(f) the C x C Hermitian matrix of the channel
// spectra at frequency f.  The preconditioner is the restriction to the valid
// subapertures of the inverse of its positive part plus the noise variance,
//
//   P r = W_s S2 F^-1 [ (M_+(f) + sigma^2 I)^-1 F[S1 W_s^T r] ],
//
// M_+ having the negative eigenvalues of M set to zero (a circulant
// embedding of a covariance need not be positive semi-definite).  It is
// symmetric positive definite and is applied with the same transforms as the
// product.  (The paper leaves preconditioning open, §2.G.)
//
// Per frequency, H = M(f) = A + iB is eigen-decomposed through the real
// symmetric 2C x 2C matrix [[A, -B], [B, A]] (cyclic Jacobi rotations, FP64),
// whose eigenvalues are those of H, each twice; for any real function g,
// g([[A, -B], [B, A]]) = [[Re g(H), -Im g(H)], [Im g(H), Re g(H)]].
//
// (M_+ + sigma^2)^-1 is not block-symmetric like M (its x-y entries differ
// from its y-x entries and same-sensor blocks are complex), so it is stored
// in the general Hermitian packing of C^2 reals per frequency:
//   slot a            Re H[a][a]                               (a < C)
//   slot C + 2k, +1   Re, Im H[a][b], k = a C - a(a+1)/2 + b - a - 1   (a < b)
#include "tt_internal.h"

#include <algorithm>
#include <thread>

namespace {

// Cyclic Jacobi eigen-decomposition of a real symmetric m x m matrix (row-major,
// overwritten); V receives the eigenvectors as columns, w the eigenvalues.
void jacobi_eigen(int m, double* a, double* V, double* w) {
    for (int i = 0; i < m * m; ++i) V[i] = 0.0;
    for (int i = 0; i < m; ++i) V[i * m + i] = 1.0;
    double scale = 0.0;
    for (int i = 0; i < m * m; ++i) scale += a[i] * a[i];
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) off += a[p * m + q] * a[p * m + q];
        if (off <= 1e-32 * scale || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = a[p * m + q];
                if (apq == 0.0) continue;
                // tan of the angle that zeroes a[p][q]: the smaller root of t^2 + 2 theta t - 1 = 0
                const double theta = (a[q * m + q] - a[p * m + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {   // columns p, q
                    const double akp = a[k * m + p], akq = a[k * m + q];
                    a[k * m + p] = c * akp - s * akq;
                    a[k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {   // rows p, q
                    const double apk = a[p * m + k], aqk = a[q * m + k];
                    a[p * m + k] = c * apk - s * aqk;
                    a[q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double vkp = V[k * m + p], vkq = V[k * m + q];
                    V[k * m + p] = c * vkp - s * vkq;
                    V[k * m + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < m; ++i) w[i] = a[i * m + i];
}

// (M_+ + sigma^2)^-1 of one frequency: packed slope spectra (3 G^2 reals) in,
// general Hermitian packing (C^2 reals) out.
void invert_one(int G, const double* Mp, double sigma2, double* out, std::vector<double>& work) {
    const int C = 2 * G, m = 2 * C;
    work.assign(3 * (size_t)m * m + m, 0.0);
    double* S = work.data();
    double* V = S + m * m;
    double* Q = V + m * m;
    double* w = Q + m * m;
    // H[a][b] = re + i im, written into S = [[Re, -Im], [Im, Re]]
    auto put = [&](int a, int b, double re, double im) {
        S[a * m + b] = re;
        S[(a + C) * m + (b + C)] = re;
        S[(a + C) * m + b] = im;
        S[a * m + (b + C)] = -im;
    };
    for (int g = 0; g < G; ++g) {
        const double xx = Mp[3 * g], xy = Mp[3 * g + 1], yy = Mp[3 * g + 2];
        put(2 * g, 2 * g, xx, 0.0);
        put(2 * g, 2 * g + 1, xy, 0.0);
        put(2 * g + 1, 2 * g, xy, 0.0);
        put(2 * g + 1, 2 * g + 1, yy, 0.0);
    }
    for (int g = 0; g < G; ++g)
        for (int h = g + 1; h < G; ++h) {
            const int px = g * (2 * G - g - 1) / 2 + (h - g - 1);
            const double* v = Mp + 3 * G + 6 * px;   // xx, xy (= yx), yy as (re, im)
            const int comp[2][2] = {{0, 1}, {1, 2}};
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q) {
                    const double re = v[2 * comp[p][q]], im = v[2 * comp[p][q] + 1];
                    put(2 * g + p, 2 * h + q, re, im);
                    put(2 * h + q, 2 * g + p, re, -im);
                }
        }
    jacobi_eigen(m, S, V, w);
    for (int i = 0; i < m; ++i) w[i] = 1.0 / (std::max(w[i], 0.0) + sigma2);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < C; ++j) {   // only the first C columns are needed
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += V[i * m + k] * w[k] * V[j * m + k];
            Q[i * m + j] = acc;
        }
    // Re g(H) = Q[0:C][0:C], Im g(H) = Q[C:2C][0:C]
    for (int a = 0; a < C; ++a) {
        out[a] = Q[a * m + a];
        for (int b = a + 1; b < C; ++b) {
            const int k = a * C - a * (a + 1) / 2 + (b - a - 1);
            out[C + 2 * k] = 0.5 * (Q[a * m + b] + Q[b * m + a]);                  // Re H[a][b]
            out[C + 2 * k + 1] = 0.5 * (Q[(a + C) * m + b] - Q[(b + C) * m + a]);  // Im H[a][b]
        }
    }
}

}  // namespace

double precond_noise(const tt_ctx& c) {
    double s = 0.0;
    for (double v : c.host_noise) s += v;
    return c.host_noise.empty() ? 0.0 : s / (double)c.host_noise.size();
}

tt_status precond_build(tt_ctx& c) {
    if (c.pc_ready) return TT_OK;
    const size_t nf = (size_t)c.L * c.Lh, P = packed_reals(c.G), C2 = (size_t)c.C * c.C;
    std::vector<double> M(nf * P), out(nf * C2);
    TT_HIP(hipMemcpyAsync(M.data(), c.M64.p, M.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    TT_HIP(hipStreamSynchronize(c.stream));
    const double sigma2 = precond_noise(c);
    if (!(sigma2 > 0.0)) {
        tt_set_error("the circulant preconditioner needs a positive mean noise variance");
        return TT_INVALID_ARG;
    }
    const unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t)
        pool.emplace_back([&, t]() {
            std::vector<double> work;
            for (size_t f = t; f < nf; f += nt) invert_one(c.G, M.data() + f * P, sigma2, out.data() + f * C2, work);
        });
    for (auto& th : pool) th.join();
    std::vector<float> out32(out.size());
    for (size_t i = 0; i < out.size(); ++i) out32[i] = (float)out[i];
    TT_CHECK(c.Minv64.alloc(out.size()));
    TT_CHECK(c.Minv32.alloc(out32.size()));
    TT_HIP(hipMemcpyAsync(c.Minv64.p, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    TT_HIP(hipMemcpyAsync(c.Minv32.p, out32.data(), out32.size() * sizeof(float), hipMemcpyHostToDevice, c.stream));
    TT_HIP(hipStreamSynchronize(c.stream));
    c.pc_ready = true;
    return TT_OK;
}
