// Solver state shared by the two solver kinds (cg.hip, persistent.hip).
#pragma once
#include "tt_internal.h"

struct CgScalars {
    double rr[2];     // r.r of the current iterate, slot (iteration & 1)
    double rr_max;    // r.r at the last replacement
    double tol2;      // tol^2 ||s||^2
    double drop2;     // refine_drop^2 (0: no replacement trigger)
    double bnorm2;    // ||s||^2
    double rr_true;   // last FP64 true residual
    double pAp;       // last p.Ap
    int state;        // 0 running, 1 replacement due, 2 recursive residual converged,
                      // 3 breakdown, 4 iteration cap
    int iter;         // iterations done
    double ru[2];     // r.u = r.P r, slot (iteration & 1) (preconditioned CG, batched solver)
};

enum { ST_RUN = 0, ST_REFINE = 1, ST_CONV = 2, ST_BREAK = 3, ST_CAP = 4 };

// State of the single-reduction CG recurrences kept across persistent launches.
struct PScalars {
    double gamma_prev;   // r.r of the previous iterate
    double alpha_prev;   // previous step length
    double gamma;        // r.r at exit
    double delta;        // r.Ar at exit
    int first;           // no iteration done since the start (beta = 0 next)
    int pad;
};

inline CgScalars* cg_scalars(tt_ctx& c) { return reinterpret_cast<CgScalars*>(c.scal.p); }
inline PScalars* p_scalars(tt_ctx& c) { return reinterpret_cast<PScalars*>(c.scal.p + 32); }

tt_status cg_setup(tt_ctx& c, const float* s, const double* x0, const tt_solve_opts& o, bool f32);
tt_status cg_true_residual(tt_ctx& c, const float* s, bool f32, CgScalars* host_out);
tt_status cg_finish(tt_ctx& c, const float* s, double* zeta, bool f32, bool have_true, tt_solve_info& info,
                    int status_code);
tt_status cg_fill_zero(tt_ctx& c, float* a32, double* a64);
tt_status cg_copy_r64_to_r32(tt_ctx& c);
