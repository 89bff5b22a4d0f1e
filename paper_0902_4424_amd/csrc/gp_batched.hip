// Batched entry points.  Shared K in bf16 runs on the matrix cores
// (gp_batched_shared.hip); other cases run as a sequence of single-problem
// solves on the caller's stream.  Every problem keeps its own steplength,
// threshold and line-search state.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "gp_internal.hpp"
#include "gp_l1.h"

using namespace gpl1;

namespace {
int check_targets(gp_handle h, const gp_opts& o, int64_t B) {
    if (!o.f_targets) return GP_OK_TOL;
    for (int64_t b = 0; b < B; ++b)
        if (std::isnan(o.f_targets[b])) return fail(h, GP_E_ARG, "opts.f_targets holds a NaN");
    return GP_OK_TOL;
}

int severity(int s) {            // errors first, then unfinished, then finished
    if (s < 0) return 100 - s;
    if (s == GP_BACKTRACK_LIMIT) return 4;
    if (s == GP_MAX_ITER) return 3;
    return 1;
}
}  // namespace

extern "C" int gp_l1_solve_batched_shared(gp_handle h, gp_dtype kdtype, const void* K, int64_t n, int64_t p,
                                          int64_t ldk, const void* Y, int64_t ldy, int64_t B,
                                          const double* rho, const void* X0, int64_t ldx, double tol,
                                          void* X_out, const gp_opts* opts, gp_result* res, void* stream) {
    if (!h) return GP_E_ARG;
    if (B < 0) return fail(h, GP_E_ARG, "B must be >= 0");
    if (B == 0) return GP_OK_TOL;
    if (!res || !rho || !Y || !X_out) return fail(h, GP_E_ARG, "null pointer argument");
    if (ldy < n || ldx < p) return fail(h, GP_E_ARG, "ldy must be >= n and ldx >= p");
    if (n <= 0 || p <= 0 || ldk < p) return fail(h, GP_E_ARG, "bad matrix shape");
    if (!K) return fail(h, GP_E_ARG, "null K");
    if (!(tol >= 0.0)) return fail(h, GP_E_ARG, "tol must be >= 0");
    for (int64_t b = 0; b < B; ++b)
        if (!(rho[b] >= 0.0) || !std::isfinite(rho[b])) return fail(h, GP_E_ARG, "rho must be finite and >= 0");
    gp_opts o;
    if (opts) o = *opts; else gp_opts_default(&o);
    int rc0 = check_opts(h, o);
    if (rc0) return rc0;
    rc0 = check_targets(h, o, B);
    if (rc0) return rc0;
    for (int64_t b = 0; b < B; ++b) { std::memset(&res[b], 0, sizeof(gp_result)); res[b].status = GP_E_ARG; }
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    // the matrix-core path for bf16 and FP32 K; other cases run one problem at a time
    int rcm = solve_batched_shared_mfma(h, kdtype, K, n, p, ldk, Y, ldy, B, rho, X0, ldx, tol, X_out, o, res,
                                        (hipStream_t)stream);
    if (rcm != GP_E_UNSUPPORTED) return rcm;
    const size_t vsz = kdtype == GP_F64 ? 8 : 4;
    int worst = GP_OK_TOL;
    for (int64_t b = 0; b < B; ++b) {
        const char* yb = (const char*)Y + (size_t)b * ldy * vsz;
        const char* x0b = X0 ? (const char*)X0 + (size_t)b * ldx * vsz : nullptr;
        char* xb = (char*)X_out + (size_t)b * ldx * vsz;
        gp_opts ob = o;
        if (o.f_targets) ob.f_target = o.f_targets[b];
        int rc = gp_l1_solve(h, kdtype, K, n, p, ldk, yb, rho[b], x0b, tol, xb, &ob, &res[b], stream);
        if (rc == GP_E_ARG || rc == GP_E_HIP || rc == GP_E_NOMEM || rc == GP_E_UNSUPPORTED) return rc;
        if (severity(rc) > severity(worst)) worst = rc;
    }
    return worst;
}

extern "C" int gp_l1_solve_batched_var(gp_handle h, gp_dtype kdtype, const gp_instance* inst, int64_t B,
                                       double tol, const gp_opts* opts, gp_result* res, void* stream) {
    if (!h) return GP_E_ARG;
    if (B < 0) return fail(h, GP_E_ARG, "B must be >= 0");
    if (B == 0) return GP_OK_TOL;
    if (!inst || !res) return fail(h, GP_E_ARG, "null pointer argument");
    if (kdtype != GP_F64 && kdtype != GP_F32 && kdtype != GP_BF16) return fail(h, GP_E_ARG, "bad dtype");
    if (!(tol >= 0.0)) return fail(h, GP_E_ARG, "tol must be >= 0");
    for (int64_t b = 0; b < B; ++b) {
        const gp_instance& I = inst[b];
        if (I.n <= 0 || I.p <= 0 || I.ldk < I.p || !I.K || !I.y || !I.x_out)
            return fail(h, GP_E_ARG, "instance " + std::to_string(b) + ": bad shape or null pointer");
        if (!(I.rho >= 0.0) || !std::isfinite(I.rho))
            return fail(h, GP_E_ARG, "instance " + std::to_string(b) + ": rho must be finite and >= 0");
        if (I.n > ((int64_t)1 << 31) || I.p > ((int64_t)1 << 31))
            return fail(h, GP_E_UNSUPPORTED, "instance too large");
    }
    gp_opts o;
    if (opts) o = *opts; else gp_opts_default(&o);
    int rc0 = check_opts(h, o);
    if (rc0) return rc0;
    rc0 = check_targets(h, o, B);
    if (rc0) return rc0;
    if (o.x0_fallback) return fail(h, GP_E_UNSUPPORTED, "opts.x0_fallback is not available for uneven batches");
    for (int64_t b = 0; b < B; ++b) { std::memset(&res[b], 0, sizeof(gp_result)); res[b].status = GP_E_ARG; }
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    int rcl = solve_batched_var_lockstep(h, kdtype, inst, B, tol, o, res, (hipStream_t)stream);
    if (rcl != GP_E_UNSUPPORTED) return rcl;
    int worst = GP_OK_TOL;
    for (int64_t b = 0; b < B; ++b) {
        const gp_instance& I = inst[b];
        gp_opts ob = o;
        if (o.f_targets) ob.f_target = o.f_targets[b];
        int rc = gp_l1_solve(h, kdtype, I.K, I.n, I.p, I.ldk, I.y, I.rho, I.x0, tol, I.x_out, &ob, &res[b],
                             stream);
        if (rc == GP_E_ARG || rc == GP_E_HIP || rc == GP_E_NOMEM || rc == GP_E_UNSUPPORTED) return rc;
        if (severity(rc) > severity(worst)) worst = rc;
    }
    return worst;
}
