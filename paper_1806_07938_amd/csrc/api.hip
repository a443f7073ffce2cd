// C entry points (include/tt.h).  Argument validation, ownership and the
// order of the set-up steps live here; the arithmetic is in the other units.
#include <algorithm>
#include <cstring>

#include "tt_internal.h"

tt_status matvec_prepare(tt_ctx& c);

namespace {
thread_local std::string g_last_error;

bool finite_all(const double* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

tt_status use_device(int dev) {
    TT_HIP(hipSetDevice(dev));
    return TT_OK;
}

#define TT_GUARD(expr)                                    \
    do {                                                  \
        try {                                             \
            return (expr);                                \
        } catch (const std::exception& e) {               \
            tt_set_error(std::string("exception: ") + e.what()); \
            return TT_OUT_OF_MEMORY;                      \
        } catch (...) {                                   \
            tt_set_error("unknown exception");            \
            return TT_HIP_ERROR;                          \
        }                                                 \
    } while (0)

tt_status create_impl(tt_ctx** out, int device, void* stream) {
    TT_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    TT_HIP(hipGetDeviceCount(&ndev));
    TT_REQUIRE(device >= 0 && device < ndev, "device index out of range");
    TT_CHECK(use_device(device));
    tt_ctx* c = new tt_ctx();
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        tt_set_error("hipGetDeviceProperties failed");
        return TT_HIP_ERROR;
    }
    c->num_cu = prop.multiProcessorCount;
    noalloc_init(device);   // scratch address of tt_matvec_noalloc on this device
    *out = c;
    return TT_OK;
}

// A context sharing the system of `base` (spectra, maps, noise, twiddles, and
// the block-circulant preconditioner spectra if built) with its own stream,
// solver vectors and transform buffers.
tt_status view_impl(tt_ctx** out, tt_ctx* base, void* stream) {
    TT_REQUIRE(out && base, "NULL argument");
    *out = nullptr;
    if (!base->ready) {
        tt_set_error("tt_create_view: the base context has no system");
        return TT_NOT_READY;
    }
    TT_REQUIRE(!base->view_of, "the base is itself a view (take a view of its base)");
    TT_REQUIRE(!base->modes, "mode removal is not supported on views");
    TT_CHECK(use_device(base->device));
    tt_ctx* c = new tt_ctx();
    c->device = base->device;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    c->num_cu = base->num_cu;
    c->n = base->n;
    c->G = base->G;
    c->C = base->C;
    c->L = base->L;
    c->Lh = base->Lh;
    c->n_vs = base->n_vs;
    c->n_slopes = base->n_slopes;
    c->n_layer = base->n_layer;
    c->model = base->model;
    c->d = base->d;
    c->h_lgs = base->h_lgs;
    c->lgs = base->lgs;
    c->gs = base->gs;
    c->h = base->h;
    c->w = base->w;
    c->r0 = base->r0;
    c->L0 = base->L0;
    c->valid = base->valid;
    c->host_noise = base->host_noise;
    c->M32.share(base->M32);
    c->M64.share(base->M64);
    c->vmap.share(base->vmap);
    c->vidx.share(base->vidx);
    c->noise32.share(base->noise32);
    c->noise64.share(base->noise64);
    c->has_nxy = base->has_nxy;
    if (base->has_nxy) {
        c->nxy32.share(base->nxy32);
        c->nxy64.share(base->nxy64);
    }
    c->tw32.share(base->tw32);
    c->tw64.share(base->tw64);
    if (base->pc_ready) {
        c->Minv32.share(base->Minv32);
        c->Minv64.share(base->Minv64);
        c->pc_ready = true;
    }
    c->learned = base->learned;
    const size_t tsz = (size_t)c->Lh * c->C * c->n;
    tt_status st = TT_OK;
    if ((st = c->T32.alloc(tsz)) != TT_OK || (st = c->U32.alloc(tsz)) != TT_OK || (st = c->T64.alloc(tsz)) != TT_OK ||
        (st = c->U64.alloc(tsz)) != TT_OK || (st = cg_alloc(*c)) != TT_OK ||
        (st = hipStreamSynchronize(c->stream) == hipSuccess ? TT_OK : TT_HIP_ERROR) != TT_OK) {
        delete c;
        return st;
    }
    c->view_of = base;
    base->n_views++;
    c->ready = true;
    *out = c;
    return TT_OK;
}

tt_status generate_impl(tt_ctx* c, const tt_geometry* g, const tt_atmosphere* a, tt_kernels** out) {
    TT_REQUIRE(c && g && a && out, "NULL argument");
    *out = nullptr;
    TT_REQUIRE(g->n >= 1 && g->n <= 512, "n must be in [1, 512]");
    TT_REQUIRE(g->n_gs >= 1 && g->n_gs <= 16, "n_gs must be in [1, 16]");
    TT_REQUIRE(g->pad_L >= 2 * g->n - 1 && g->pad_L <= 1024, "pad_L must be in [2n-1, 1024]");
    TT_REQUIRE(g->gradient_model == TT_MODEL_HUDGIN || g->gradient_model == TT_MODEL_FRIED,
               "unsupported gradient model");
    TT_REQUIRE(std::isfinite(g->D) && g->D > 0, "D must be positive");
    TT_REQUIRE(g->gs_xy, "gs_xy is required");
    TT_REQUIRE(finite_all(g->gs_xy, 2 * g->n_gs), "non-finite guide-star direction");
    // W_s: the caller's mask, or the valid-subaperture rule (§2.F) with the obstruction
    std::vector<unsigned char> mask((size_t)g->n * g->n);
    if (g->valid) {
        for (int i = 0; i < g->n * g->n; ++i) mask[i] = g->valid[i] ? 1 : 0;
    } else {
        TT_CHECK(pupil_rule(g->n, g->D, g->obstruction, mask.data(), nullptr));
    }
    int nv = 0;
    for (int i = 0; i < g->n * g->n; ++i) nv += mask[i] != 0;
    TT_REQUIRE(nv > 0, "no valid subaperture");
    TT_REQUIRE(a->n_layer >= 1 && a->n_layer <= 256, "n_layer must be in [1, 256]");
    TT_REQUIRE(a->h && a->w, "h and w are required");
    TT_REQUIRE(finite_all(a->h, a->n_layer) && finite_all(a->w, a->n_layer), "non-finite layer data");
    TT_REQUIRE(std::isfinite(a->r0) && a->r0 > 0 && std::isfinite(a->L0) && a->L0 > 0, "r0 and L0 must be positive");
    const bool lgs = std::isfinite(g->h_lgs) && g->h_lgs > 0;
    for (int k = 0; k < a->n_layer; ++k) {
        TT_REQUIRE(a->h[k] >= 0, "negative layer altitude");
        if (lgs) TT_REQUIRE(a->h[k] < g->h_lgs, "layer at or above the LGS altitude");
    }
    TT_CHECK(use_device(c->device));
    tt_kernels* k = new tt_kernels();
    k->device = c->device;
    k->n = g->n;
    k->n_gs = g->n_gs;
    k->pad_L = g->pad_L;
    k->model = g->gradient_model;
    k->D = g->D;
    k->d = g->D / g->n;
    k->h_lgs = g->h_lgs;
    k->lgs = lgs;
    k->gs.assign(g->gs_xy, g->gs_xy + 2 * g->n_gs);
    k->valid = mask;
    k->n_layer = a->n_layer;
    k->h.assign(a->h, a->h + a->n_layer);
    k->w.assign(a->w, a->w + a->n_layer);
    k->r0 = a->r0;
    k->L0 = a->L0;
    const long m = 2 * g->n - 1;
    k->count = (size_t)n_pairs_incl(g->n_gs) * 3 * m * m;
    tt_status st = k->tables.alloc(k->count);
    if (st == TT_OK) st = gen_tables_launch(*k, k->tables.p, c->stream);
    if (st != TT_OK) {
        delete k;
        return st;
    }
    *out = k;
    return TT_OK;
}

tt_status set_system_impl(tt_ctx* c, const tt_kernels* k, const double* noise_var, double noise_scalar,
                          const tt_target* target) {
    TT_REQUIRE(c && k, "NULL argument");
    TT_REQUIRE(k->device == c->device, "kernels were generated on another device");
    TT_REQUIRE(!c->view_of, "a view shares its base's system and cannot set one");
    TT_REQUIRE(c->n_views == 0, "the context has live views sharing its system (destroy them first)");
    TT_CHECK(use_device(c->device));
    c->ready = false;
    c->proj.on = false;
    c->tile_S = 0;
    c->pc_ready = false;
    c->mh_kind[0] = c->mh_kind[1] = 0;
    c->mt_ready[0] = c->mt_ready[1] = false;
    c->mht_kind[0] = c->mht_kind[1] = 0;
    c->has_nxy = false;
    c->modes = false;
    c->n = k->n;
    c->G = k->n_gs;
    c->C = 2 * k->n_gs;
    c->L = k->pad_L;
    c->Lh = k->pad_L / 2 + 1;
    c->n_layer = k->n_layer;
    c->model = k->model;
    c->d = k->d;
    c->h_lgs = k->h_lgs;
    c->lgs = k->lgs;
    c->gs = k->gs;
    c->h = k->h;
    c->w = k->w;
    c->r0 = k->r0;
    c->L0 = k->L0;
    c->valid = k->valid;
    // W_s index maps
    std::vector<int> vmap((size_t)c->n * c->n, -1), vidx;
    for (int i = 0; i < c->n * c->n; ++i)
        if (k->valid[i]) {
            vmap[i] = (int)vidx.size();
            vidx.push_back(i);
        }
    c->n_vs = (int)vidx.size();
    c->n_slopes = c->C * c->n_vs;
    // noise
    std::vector<double> nz(c->n_slopes, noise_scalar);
    if (noise_var) nz.assign(noise_var, noise_var + c->n_slopes);
    for (double v : nz) TT_REQUIRE(std::isfinite(v), "non-finite noise variance");
    std::vector<float> nz32(nz.begin(), nz.end());
    TT_CHECK(c->vmap.upload(vmap.data(), vmap.size(), c->stream));
    TT_CHECK(c->vidx.upload(vidx.data(), vidx.size(), c->stream));
    TT_CHECK(c->noise64.upload(nz.data(), nz.size(), c->stream));
    TT_CHECK(c->noise32.upload(nz32.data(), nz32.size(), c->stream));
    TT_HIP(hipStreamSynchronize(c->stream));
    c->host_noise = nz;
    TT_CHECK(build_twiddles(c->L, c->tw32, &c->tw64, c->stream));
    TT_CHECK(build_slope_spectra(*c, *k));
    const size_t tsz = (size_t)c->Lh * c->C * c->n;
    TT_CHECK(c->T32.alloc(tsz));
    TT_CHECK(c->U32.alloc(tsz));
    TT_CHECK(c->T64.alloc(tsz));
    TT_CHECK(c->U64.alloc(tsz));
    TT_CHECK(cg_alloc(*c));
    if (target) TT_CHECK(projection_setup(*c, target));
    TT_HIP(hipStreamSynchronize(c->stream));
    c->ready = true;
    return TT_OK;
}

// Solve options with their defaults, checked against the context.
tt_status parse_opts(const tt_ctx* c, const tt_solve_opts* opts, tt_solve_opts& o) {
    o.tol = 1e-6;
    o.max_iter = 20000;
    o.precision = TT_PREC_F32;
    o.solver = TT_SOLVER_PERSISTENT;
    o.refine_drop = 1e-3;
    o.preconditioner = TT_PRECOND_NONE;
    o.method = TT_METHOD_CG;
    o.graph = 0;
    if (opts) o = *opts;
    TT_REQUIRE(std::isfinite(o.tol) && o.tol >= 0, "tol must be >= 0");
    TT_REQUIRE(o.max_iter >= 0, "max_iter must be >= 0");
    TT_REQUIRE(o.precision == TT_PREC_F32 || o.precision == TT_PREC_F64 || o.precision == TT_PREC_F16 ||
                   o.precision == TT_PREC_BF16,
               "unknown precision");
    TT_REQUIRE(o.solver == TT_SOLVER_PERSISTENT || o.solver == TT_SOLVER_KERNELS || o.solver == TT_SOLVER_BATCHED,
               "unknown solver");
    TT_REQUIRE(o.solver == TT_SOLVER_PERSISTENT || (o.precision != TT_PREC_F16 && o.precision != TT_PREC_BF16) ||
                   (o.solver == TT_SOLVER_BATCHED && o.preconditioner == TT_PRECOND_CIRCULANT),
               "TT_PREC_F16 / TT_PREC_BF16 need TT_SOLVER_PERSISTENT, or TT_SOLVER_BATCHED with "
               "TT_PRECOND_CIRCULANT");
    TT_REQUIRE(std::isfinite(o.refine_drop) && o.refine_drop >= 0 && o.refine_drop < 1, "refine_drop in [0, 1)");
    TT_REQUIRE(o.preconditioner == TT_PRECOND_NONE || o.preconditioner == TT_PRECOND_CIRCULANT ||
                   o.preconditioner == TT_PRECOND_LEARNED,
               "unknown preconditioner");
    if (o.preconditioner == TT_PRECOND_LEARNED) {
        TT_REQUIRE(o.solver == TT_SOLVER_BATCHED && o.precision == TT_PREC_F32 && o.method == TT_METHOD_CG,
                   "TT_PRECOND_LEARNED needs TT_SOLVER_BATCHED, TT_PREC_F32 and TT_METHOD_CG");
        if (!c->learned) {
            tt_set_error("TT_PRECOND_LEARNED: no network attached (tt_set_learned)");
            return TT_NOT_READY;
        }
        TT_REQUIRE(learned_channels(c->learned) == c->C,
                   "the attached network's channel count differs from the system's 2 n_gs");
    }
    TT_REQUIRE(o.preconditioner != TT_PRECOND_CIRCULANT || o.solver == TT_SOLVER_BATCHED ||
                   (o.solver == TT_SOLVER_PERSISTENT && (o.precision == TT_PREC_F32 || o.precision == TT_PREC_F64)),
               "TT_PRECOND_CIRCULANT needs TT_SOLVER_PERSISTENT with TT_PREC_F32 or TT_PREC_F64, or "
               "TT_SOLVER_BATCHED");
    TT_REQUIRE(o.method == TT_METHOD_CG || o.method == TT_METHOD_MINRES, "unknown method");
    TT_REQUIRE(o.method == TT_METHOD_CG ||
                   (o.solver == TT_SOLVER_PERSISTENT && o.preconditioner == TT_PRECOND_NONE &&
                    (o.precision == TT_PREC_F32 || o.precision == TT_PREC_F64)),
               "TT_METHOD_MINRES needs TT_SOLVER_PERSISTENT, TT_PREC_F32 or TT_PREC_F64 and no preconditioner");
    TT_REQUIRE(o.solver != TT_SOLVER_BATCHED || o.precision != TT_PREC_F64, "TT_SOLVER_BATCHED computes in FP32");
    TT_REQUIRE(!c->modes || o.solver == TT_SOLVER_KERNELS, "mode removal needs TT_SOLVER_KERNELS");
    return TT_OK;
}

// context and output checks shared by tt_solve_frame and tt_solve_batch
tt_status check_frame(const tt_ctx* c, const float* s, const double* zeta, const float* phi) {
    TT_REQUIRE(c && s && zeta, "NULL argument");
    if (!c->ready) {
        tt_set_error("tt_solve_frame: no system set");
        return TT_NOT_READY;
    }
    if (phi && !c->proj.on) {
        tt_set_error("tt_solve_frame: d_phi given but no target was set");
        return TT_NOT_READY;
    }
    return TT_OK;
}

// after the iterations: mode removal projects the solution (the system is
// (M_s W_s)(Sigma_ss + Sigma_eta)(M_s W_s)^T zeta = M_s s, products projected on
// both sides and every residual projected), then the projection phi
tt_status finish_frame(tt_ctx* c, double* zeta, float* phi) {
    if (c->modes) {
        TT_CHECK(modes_project_f64(*c, zeta));
        TT_HIP(hipStreamSynchronize(c->stream));
    }
    if (phi) {
        TT_CHECK(projection_apply(*c, zeta, phi));
        TT_HIP(hipStreamSynchronize(c->stream));
    }
    return TT_OK;
}

tt_status solve_impl(tt_ctx* c, const float* s, const double* x0, double* zeta, float* phi, const tt_solve_opts* opts,
                     tt_solve_info* info) {
    TT_CHECK(check_frame(c, s, zeta, phi));
    tt_solve_opts o;
    TT_CHECK(parse_opts(c, opts, o));
    TT_CHECK(use_device(c->device));
    tt_solve_info inf{};
    inf.fallback = -1;
    if (o.solver == TT_SOLVER_PERSISTENT)
        TT_CHECK(solve_persistent(*c, s, x0, zeta, o, inf));
    else if (o.solver == TT_SOLVER_KERNELS)
        TT_CHECK(solve_kernels(*c, s, x0, zeta, o, inf));
    else
        TT_CHECK(solve_batched(&c, 1, &s, x0 ? &x0 : nullptr, &zeta, o, &inf));
    TT_CHECK(finish_frame(c, zeta, phi));
    if (info) *info = inf;
    if (inf.status != TT_OK)
        tt_set_error(std::string("tt_solve_frame: ") + tt_status_string((tt_status)inf.status) + " after " +
                     std::to_string(inf.iterations) + " iterations, FP64 relative residual " +
                     std::to_string(inf.rel_residual));
    return (tt_status)inf.status;
}

}  // namespace

void tt_set_error(const std::string& msg) { g_last_error = msg; }

static tt_status batch_impl(tt_ctx* const* systems, int count, const float* const* d_s, const double* const* d_x0,
                         double* const* d_zeta, float* const* d_phi, const tt_solve_opts* opts, tt_solve_info* infos) {
    TT_REQUIRE(count >= 0, "count must be >= 0");
    TT_REQUIRE(count == 0 || (systems && d_s && d_zeta), "NULL argument");
    for (int i = 0; i < count; ++i)
        for (int j = 0; j < i; ++j) TT_REQUIRE(systems[i] != systems[j], "a context appears twice in the batch");
    bool breakdown = false, notconv = false;
    tt_solve_opts o;
    if (count > 0) TT_CHECK(parse_opts(systems[0], opts, o));
    if (count > 0 && o.solver == TT_SOLVER_BATCHED) {
        // all systems iterate together (solve_batched); options checked for each
        for (int i = 0; i < count; ++i) {
            TT_CHECK(check_frame(systems[i], d_s[i], d_zeta[i], d_phi ? d_phi[i] : nullptr));
            tt_solve_opts oi;
            TT_CHECK(parse_opts(systems[i], opts, oi));
        }
        TT_CHECK(use_device(systems[0]->device));
        std::vector<tt_solve_info> inf((size_t)count);
        TT_CHECK(solve_batched(systems, count, d_s, d_x0, d_zeta, o, inf.data()));
        for (int i = 0; i < count; ++i) {
            TT_CHECK(finish_frame(systems[i], d_zeta[i], d_phi ? d_phi[i] : nullptr));
            if (infos) infos[i] = inf[i];
            if (inf[i].status == TT_BREAKDOWN) breakdown = true;
            else if (inf[i].status == TT_NOT_CONVERGED) notconv = true;
            if (inf[i].status != TT_OK)
                tt_set_error(std::string("tt_solve_batch: frame ") + std::to_string(i) + ": " +
                             tt_status_string((tt_status)inf[i].status) + " after " +
                             std::to_string(inf[i].iterations) + " iterations");
        }
        return breakdown ? TT_BREAKDOWN : notconv ? TT_NOT_CONVERGED : TT_OK;
    }
    for (int i = 0; i < count; ++i) {
        const tt_status st = solve_impl(systems[i], d_s[i], d_x0 ? d_x0[i] : nullptr, d_zeta[i],
                                        d_phi ? d_phi[i] : nullptr, opts, infos ? &infos[i] : nullptr);
        if (st == TT_BREAKDOWN) breakdown = true;
        else if (st == TT_NOT_CONVERGED) notconv = true;
        else if (st != TT_OK) return st;
    }
    return breakdown ? TT_BREAKDOWN : notconv ? TT_NOT_CONVERGED : TT_OK;
}

extern "C" {

tt_status tt_create(tt_ctx** out, int device, void* stream) { TT_GUARD(create_impl(out, device, stream)); }

tt_status tt_destroy(tt_ctx* ctx) {
    if (!ctx) return TT_OK;
    if (ctx->n_views > 0) {
        tt_set_error("tt_destroy: the context still has " + std::to_string(ctx->n_views) + " live views");
        return TT_INVALID_ARG;
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->view_of) ctx->view_of->n_views--;
    delete ctx;
    return TT_OK;
}

tt_status tt_create_view(tt_ctx** out, tt_ctx* base, void* stream) { TT_GUARD(view_impl(out, base, stream)); }

tt_status tt_generate_kernels(tt_ctx* ctx, const tt_geometry* geom, const tt_atmosphere* atm, tt_kernels** out) {
    TT_GUARD(generate_impl(ctx, geom, atm, out));
}

tt_status tt_kernels_destroy(tt_kernels* k) {
    if (!k) return TT_OK;
    (void)hipSetDevice(k->device);
    delete k;
    return TT_OK;
}

tt_status tt_kernels_copy(const tt_kernels* k, double* host_out, size_t count) {
    TT_REQUIRE(k && host_out, "NULL argument");
    TT_REQUIRE(count == k->count, "count must equal n_gs(n_gs+1)/2 * 3 * (2n-1)^2");
    TT_HIP(hipSetDevice(k->device));
    TT_HIP(hipMemcpy(host_out, k->tables.p, count * sizeof(double), hipMemcpyDeviceToHost));
    return TT_OK;
}

tt_status tt_set_system(tt_ctx* ctx, const tt_kernels* k, const double* noise_var, double noise_scalar,
                        const tt_target* target) {
    TT_GUARD(set_system_impl(ctx, k, noise_var, noise_scalar, target));
}

tt_status tt_set_noise_xy(tt_ctx* c, const double* cov_xy) {
    TT_REQUIRE(c, "NULL context");
    if (!c->ready) {
        tt_set_error("tt_set_noise_xy: no system set");
        return TT_NOT_READY;
    }
    TT_REQUIRE(!c->view_of && c->n_views == 0, "the noise of a system shared with views cannot change");
    TT_CHECK(use_device(c->device));
    if (!cov_xy) {
        c->has_nxy = false;
        return TT_OK;
    }
    const size_t m = (size_t)c->G * c->n_vs;
    for (size_t i = 0; i < m; ++i) {
        const size_t g = i / c->n_vs, v = i % c->n_vs;
        const double vx = c->host_noise[(2 * g) * c->n_vs + v], vy = c->host_noise[(2 * g + 1) * c->n_vs + v];
        TT_REQUIRE(std::isfinite(cov_xy[i]) && vx > 0 && vy > 0 && cov_xy[i] * cov_xy[i] < vx * vy,
                   "every 2x2 noise block must be positive definite");
    }
    std::vector<float> c32(cov_xy, cov_xy + m);
    TT_CHECK(c->nxy64.upload(cov_xy, m, c->stream));
    TT_CHECK(c->nxy32.upload(c32.data(), m, c->stream));
    TT_HIP(hipStreamSynchronize(c->stream));
    c->has_nxy = true;
    return TT_OK;
}

tt_status tt_set_mode_removal(tt_ctx* c, int on) {
    TT_REQUIRE(c, "NULL context");
    if (!c->ready) {
        tt_set_error("tt_set_mode_removal: no system set");
        return TT_NOT_READY;
    }
    TT_REQUIRE(!c->view_of && c->n_views == 0, "mode removal is not supported with views");
    TT_CHECK(use_device(c->device));
    if (!on) {
        c->modes = false;
        return TT_OK;
    }
    TT_CHECK(modes_setup(*c));
    TT_CHECK(c->mtmp32.alloc(c->n_slopes));
    TT_CHECK(c->mtmp64.alloc(c->n_slopes));
    c->modes = true;
    return TT_OK;
}

tt_status tt_get_system_info(const tt_ctx* c, tt_system_info* out) {
    TT_REQUIRE(c && out, "NULL argument");
    if (!c->ready) {
        tt_set_error("tt_get_system_info: no system set");
        return TT_NOT_READY;
    }
    tt_system_info s{};
    s.n = c->n;
    s.n_gs = c->G;
    s.pad_L = c->L;
    s.n_vs = c->n_vs;
    s.n_slopes = c->n_slopes;
    s.n_layer = c->n_layer;
    s.n_vphi = c->proj.on ? c->proj.n_vphi : 0;
    s.n_prime = c->proj.on ? c->proj.np : 0;
    s.proj_pad_L = c->proj.on ? c->proj.Lp : 0;
    s.spectra_bytes_f32 = c->M32.n * sizeof(float);
    s.spectra_bytes_f64 = c->M64.n * sizeof(double);
    s.proj_spectra_bytes = c->proj.on ? c->proj.spec.n * sizeof(c32) : 0;
    *out = s;
    return TT_OK;
}

tt_status tt_matvec(tt_ctx* c, const float* d_x, float* d_y) {
    TT_REQUIRE(c && d_x && d_y, "NULL argument");
    TT_REQUIRE(d_x != d_y, "d_x and d_y must not alias");
    if (!c->ready) {
        tt_set_error("tt_matvec: no system set");
        return TT_NOT_READY;
    }
    TT_HIP(hipSetDevice(c->device));
    return matvec_f32(*c, d_x, d_y, nullptr);
}

tt_status tt_matvec_f64(tt_ctx* c, const double* d_x, double* d_y) {
    TT_REQUIRE(c && d_x && d_y, "NULL argument");
    TT_REQUIRE(d_x != d_y, "d_x and d_y must not alias");
    if (!c->ready) {
        tt_set_error("tt_matvec_f64: no system set");
        return TT_NOT_READY;
    }
    TT_HIP(hipSetDevice(c->device));
    return matvec_f64(*c, d_x, d_y, nullptr);
}

tt_status tt_matvec_batch(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y,
                          float* phase_ms) {
    TT_GUARD(matvec_batch(systems, count, d_x, d_y, phase_ms, TT_PREC_F32));
}

tt_status tt_tune_batch(tt_ctx* const* systems, int count, int op, int precision, int* best_split,
                        float* ms_per_split) {
    TT_GUARD(tune_batch(systems, count, op, precision, best_split, ms_per_split));
}

tt_status tt_matvec_batch_prec(tt_ctx* const* systems, int count, const float* const* d_x, float* const* d_y,
                               int precision, int split, float* phase_ms) {
    TT_REQUIRE(split == 0 || split == 1 || split == 2 || split == 4, "split must be 0, 1, 2 or 4");
    TT_GUARD(batch_apply(systems, count, d_x, d_y, 0, phase_ms, precision, split));
}

tt_status tt_solve_frame(tt_ctx* ctx, const float* d_s, const double* d_x0, double* d_zeta, float* d_phi,
                         const tt_solve_opts* opts, tt_solve_info* info) {
    TT_GUARD(solve_impl(ctx, d_s, d_x0, d_zeta, d_phi, opts, info));
}

tt_status tt_solve_batch(tt_ctx* const* systems, int count, const float* const* d_s, const double* const* d_x0,
                         double* const* d_zeta, float* const* d_phi, const tt_solve_opts* opts, tt_solve_info* infos) {
    TT_GUARD(batch_impl(systems, count, d_s, d_x0, d_zeta, d_phi, opts, infos));
}

tt_status tt_project(tt_ctx* c, const double* d_zeta, float* d_phi) {
    TT_REQUIRE(c && d_zeta && d_phi, "NULL argument");
    if (!c->ready || !c->proj.on) {
        tt_set_error("tt_project: no system or no target set");
        return TT_NOT_READY;
    }
    TT_HIP(hipSetDevice(c->device));
    return projection_apply(*c, d_zeta, d_phi);
}

const char* tt_status_string(tt_status s) {
    switch (s) {
        case TT_OK: return "TT_OK";
        case TT_INVALID_ARG: return "TT_INVALID_ARG";
        case TT_HIP_ERROR: return "TT_HIP_ERROR";
        case TT_OUT_OF_MEMORY: return "TT_OUT_OF_MEMORY";
        case TT_NOT_CONVERGED: return "TT_NOT_CONVERGED";
        case TT_BREAKDOWN: return "TT_BREAKDOWN";
        case TT_NOT_READY: return "TT_NOT_READY";
    }
    return "TT_UNKNOWN_STATUS";
}

const char* tt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
