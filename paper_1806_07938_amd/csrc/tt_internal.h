// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tt.h"

// ---------------------------------------------------------------------------
// error handling (no exception crosses the C ABI)
// ---------------------------------------------------------------------------
void tt_set_error(const std::string& msg);

#define TT_REQUIRE(cond, msg)                                   \
    do {                                                        \
        if (!(cond)) {                                          \
            tt_set_error(std::string(__func__) + ": " + (msg)); \
            return TT_INVALID_ARG;                              \
        }                                                       \
    } while (0)

#define TT_HIP(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            tt_set_error(std::string(#call) + " failed: " + hipGetErrorString(e_));         \
            return e_ == hipErrorOutOfMemory ? TT_OUT_OF_MEMORY : TT_HIP_ERROR;             \
        }                                                                                   \
    } while (0)

#define TT_CHECK(expr)                   \
    do {                                 \
        tt_status s_ = (expr);           \
        if (s_ != TT_OK) return s_;      \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers owned by the library
// ---------------------------------------------------------------------------
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    bool own = true;   // false: a view of another buffer (a context view shares its base's system)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p && own) (void)hipFree(p);
        p = nullptr;
        n = 0;
        own = true;
    }
    void share(const DevBuf& o) {
        release();
        p = o.p;
        n = o.n;
        own = false;
    }
    tt_status alloc(size_t count) {
        release();
        if (count == 0) return TT_OK;
        hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            tt_set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? TT_OUT_OF_MEMORY : TT_HIP_ERROR;
        }
        n = count;
        return TT_OK;
    }
    tt_status upload(const T* host, size_t count, hipStream_t s) {
        TT_CHECK(alloc(count));
        if (count) TT_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
        return TT_OK;
    }
};

// Device copy of a host table that a launch reads (descriptors, pointer
// tables), re-uploaded only when the host table changes.  A caller that replays
// captured launches keeps its own: another call with different contents then
// cannot overwrite (or reallocate) what the captured launches read.
template <typename T>
struct HostMirror {
    DevBuf<T> dev;
    std::vector<T> host;
};

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename R> struct cplx { R x, y; };
using c32 = cplx<float>;
using c64 = cplx<double>;

// ---------------------------------------------------------------------------
// generated covariance tables (App. A.2 / A.3, §2.D cone scaling)
// ---------------------------------------------------------------------------
struct tt_kernels {
    int device = 0;
    int n = 0, n_gs = 0, pad_L = 0, model = 0;
    double D = 0, d = 0, h_lgs = 0;
    bool lgs = false;
    std::vector<double> gs;            // 2 n_gs
    std::vector<unsigned char> valid;  // n*n
    int n_layer = 0;
    std::vector<double> h, w;
    double r0 = 0, L0 = 0;
    DevBuf<double> tables;             // [pair(g<=h)][comp][2n-1][2n-1]
    size_t count = 0;
};

// number of unordered pairs g <= h and their row-major index
inline int n_pairs_incl(int G) { return G * (G + 1) / 2; }
inline int pair_incl(int g, int h, int G) { return g * G - g * (g - 1) / 2 + (h - g); }

// packed per-frequency Hermitian matrix: 3 reals per sensor (xx, xy, yy), then
// for g < h (row-major) 3 complex (xx, xy = yx, yy): 3 G^2 reals in total.
inline int packed_reals(int G) { return 3 * G * G; }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Projection {
    bool on = false;
    int np = 0, Lp = 0, Lph = 0, n_vphi = 0, n_layer = 0;
    double beta_x = 0, beta_y = 0;
    DevBuf<c32> spec;        // [f2][f1][layer][channel] complex, FP32
    DevBuf<int> vphi;        // n_vphi: flat phase-point index i*(n+1)+j
    DevBuf<double> sk;       // per-layer cone factors s_k
    DevBuf<float> z32;       // zeta rounded to FP32
    DevBuf<c32> twp;         // Lp twiddles
    DevBuf<c32> T, Xw;       // work: row transforms [f2][C][n]; per-layer column outputs [f2][layer][n']
    DevBuf<float> layer_out; // [layer][n'][n']
};

struct tt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 0;

    // system
    bool ready = false;
    int n = 0, G = 0, C = 0, L = 0, Lh = 0, n_vs = 0, n_slopes = 0, n_layer = 0;
    int model = 0;            // tt_gradient_model of the system
    DevBuf<float> M32;        // [Lh][L][3G^2]
    DevBuf<double> M64;
    DevBuf<int> vmap;         // n*n: valid index v or -1
    DevBuf<int> vidx;         // n_vs: flat index of valid subaperture v
    DevBuf<float> noise32;    // n_slopes
    DevBuf<double> noise64;
    DevBuf<float> nxy32;      // x-y noise covariance per sensor and valid subaperture [g][v] (§2.F), if set
    DevBuf<double> nxy64;
    bool has_nxy = false;
    bool modes = false;       // tip/tilt/focus removal (§2.F), see modes.hip
    DevBuf<float> mode_pos;   // (x, y) of the valid subapertures, units of d
    std::vector<double> mode_ginv;         // (Z^T Z)^-1 of one sensor's slope modes
    DevBuf<float> mode_phase_pos;          // (x, y) of the valid phase points
    std::vector<double> mode_phase_ginv;   // (Z^T Z)^-1 of the phase modes (empty: no target)
    DevBuf<float> mtmp32;     // projected input of the product with mode removal
    DevBuf<double> mtmp64;
    DevBuf<c32> tw32;         // L twiddles exp(-2 pi i k / L) as (cos, sin)
    DevBuf<c64> tw64;

    // matvec work buffers
    DevBuf<c32> T32, U32;     // [Lh][C][n]
    DevBuf<c64> T64, U64;

    // solver work buffers
    DevBuf<float> x32, r32, p32, q32;   // q = A p
    DevBuf<double> x64, r64, p64, q64, aux64;
    DevBuf<double> ppart;               // persistent solver partial sums
    DevBuf<c64> pU;                     // persistent solver column outputs [f2][split][C][n]
    DevBuf<c64> tFa, tFb, tGr;          // persistent solver transform tiles
    DevBuf<c32> tFAm, tFBm;             // persistent solver matrix-core operand fragments (8 bytes each)
    int tile_S = 0, tile_elem = 0;      // split and element size the tiles were built for
    int tile_mf = -1;                   // column-transform mode the fragments were built for
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t gstream = nullptr;      // batched solver's graph chunks (a capturable stream), made on first use
    hipEvent_t gev[2] = {nullptr, nullptr};
    DevBuf<c32> bU32;                   // batched product: column shares [Lh][S][C][n]
    DevBuf<float> bu32;                 // batched preconditioned CG: u = P r
    HostMirror<unsigned char> bdesc[2]; // batched product / preconditioner: per-system descriptors
                                        // (kept by the first context of a call)
    hipEvent_t bev[4] = {nullptr, nullptr, nullptr, nullptr};   // batched product phase timing
    DevBuf<unsigned short> Mh[2];       // batched operators: slope / preconditioner spectra in FP16 or BF16
    DevBuf<float> Mhs[2];               // their per-frequency factors [Lh][L]
    int mh_kind[2] = {0, 0};            // tt_precision the half copies hold (0: none)
    // batched operators on a power-of-two L: the same spectra slot-major, [Lh][P][L], the L frequencies of
    // every column in bit-reversed order (the order of the column FFT's output); FP32, or FP16 / BF16 with
    // the factors [Lh][L] in that order.  Built on first use by the batched column kernel.
    DevBuf<float> Mt32[2];
    DevBuf<unsigned short> Mht[2];
    DevBuf<float> Mhst[2];
    bool mt_ready[2] = {false, false};
    int mht_kind[2] = {0, 0};
    int tuned_S[2] = {0, 0};            // batched product / preconditioner: frequency split chosen by
    std::vector<const tt_ctx*> tuned_for[2];   // tt_tune_batch for this exact batch (this context first)
    DevBuf<float> Minv32;               // circulant preconditioner spectra [Lh][L][C^2] (general Hermitian packing)
    DevBuf<double> Minv64;
    bool pc_ready = false;              // Minv built for the current system
    DevBuf<double> part;                // per-block partial sums
    DevBuf<double> scal;                // solver scalars (see cg.hip)
    DevBuf<unsigned int> bar;           // grid barrier counters
    std::vector<double> host_noise;

    tt_learned* learned = nullptr;      // attached learned preconditioner (not owned)
    tt_ctx* view_of = nullptr;          // a view: the context whose system it shares
    int n_views = 0;                    // live views of this context
    DevBuf<float> bu_old32;             // flexible PCG: the previous u = P r
    Projection proj;
    // copy of the geometry the system was built from (for the projection)
    double d = 0, h_lgs = 0;
    bool lgs = false;
    std::vector<double> gs, h, w;
    double r0 = 0, L0 = 0;
    std::vector<unsigned char> valid;

    tt_ctx() = default;
    tt_ctx(const tt_ctx&) = delete;
    tt_ctx& operator=(const tt_ctx&) = delete;
    ~tt_ctx() {
        for (hipEvent_t e : {ev0, ev1, bev[0], bev[1], bev[2], bev[3], gev[0], gev[1]})
            if (e) (void)hipEventDestroy(e);
        if (gstream) (void)hipStreamDestroy(gstream);
    }
};

// ---------------------------------------------------------------------------
// module entry points (host side)
// ---------------------------------------------------------------------------
// vonkarman.hip
tt_status gen_tables_launch(const tt_kernels& k, double* d_out, hipStream_t s);
tt_status gen_phase_tables_launch(const tt_ctx& c, int np, double* d_out, hipStream_t s);
double vk_host_bracket(double x);   // host copy of the device bracket (diagnostics)

// spectra.hip
tt_status build_slope_spectra(tt_ctx& c, const tt_kernels& k);
tt_status build_twiddles(int L, DevBuf<c32>& t32, DevBuf<c64>* t64, hipStream_t s);
tt_status table_spectra(const double* d_tables, long ntab, int m, int off, int L, DevBuf<c64>& S, hipStream_t s);

// matvec.hip
tt_status matvec_f32(tt_ctx& c, const float* x, float* y, double* part);
tt_status matvec_f64(tt_ctx& c, const double* x, double* y, double* part);

// batch.hip
tt_status matvec_batch(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y,
                       float* phase_ms, int precision);
tt_status batch_apply(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y, int op,
                      float* phase_ms, int precision = TT_PREC_F32,   // op 0: the product, op 1: the block-circulant
                      int S_force = 0,                                // preconditioner; spectra storage precision;
                      HostMirror<unsigned char>* desc = nullptr);     // frequency split (0: tuned or default);
                                                                      // descriptor table (null: the first system's)
tt_status tune_batch(tt_ctx* const* systems, int count, int op, int precision, int* best_S, float* ms);

// cg.hip
tt_status cg_alloc(tt_ctx& c);
tt_status solve_kernels(tt_ctx& c, const float* s, const double* x0, double* zeta,
                        const tt_solve_opts& o, tt_solve_info& info);
tt_status solve_persistent(tt_ctx& c, const float* s, const double* x0, double* zeta,
                           const tt_solve_opts& o, tt_solve_info& info);

// batch_solve.hip: lockstep FP32 CG over several systems (TT_SOLVER_BATCHED)
tt_status solve_batched(tt_ctx* const* systems, int count, const float* const* d_s, const double* const* d_x0,
                        double* const* d_zeta, const tt_solve_opts& o, tt_solve_info* infos);

// precond.hip
tt_status precond_build(tt_ctx& c);   // Minv32 / Minv64 of the current system (once per system)
double precond_noise(const tt_ctx& c);

// modes.hip
tt_status modes_setup(tt_ctx& c);
tt_status modes_project_f32(tt_ctx& c, float* v);
tt_status modes_project_f64(tt_ctx& c, double* v);
tt_status modes_project_phase(tt_ctx& c, float* phi);

// project.hip
tt_status projection_setup(tt_ctx& c, const tt_target* t);
tt_status projection_apply(tt_ctx& c, const double* zeta, float* phi);

// learned.hip: the learned preconditioner P = K^T K
tt_status learned_apply_batch(tt_learned& L, const tt_ctx& c, const float* const* d_r, float* const* d_z, int B,
                              hipStream_t s, HostMirror<float*>* table = nullptr);   // null: the network's table
int learned_channels(const tt_learned* L);

// noalloc.hip: device scratch of tt_matvec_noalloc (address looked up once per device)
void noalloc_init(int device);
size_t noalloc_scratch_bytes();

// pupil.hip: the valid-subaperture rule (tt_pupil_mask)
tt_status pupil_rule(int n, double D, double obstruction, unsigned char* out, int* n_valid);

// launch-shape helper
inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }
