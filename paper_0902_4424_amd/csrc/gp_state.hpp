// Device-resident solver state for one problem of
//     min ||K x - y||^2  s.t.  ||x||_1 <= rho
// solved by gradient projection along d = P(x - alpha g) - x with Armijo
// backtracking (Algorithm 1, Section 3) and the adaptive Barzilai-Borwein
// alternation of Algorithm 2.  All scalars are double.  The state lives in
// device memory and is read and written only by the kernels, so an iteration
// needs no host round trip.
//
// Ownership of the fields between kernels (a kernel never reads a field that
// another workgroup of the same launch writes):
//   projection kernel (one workgroup): commits pending updates, runs the
//       steplength rule, writes gd/dd/stationary status;
//   update kernel, workgroup 0: writes lam, f_new, k_new, pending flags and
//       the stopping request; all its workgroups read only committed fields.
// Stop protocol: the update kernel raises `stop_req`; the next projection
// kernel (one workgroup) turns it into `live = 0`, and the multi-workgroup
// kernels test only `live`, which no workgroup of theirs writes.
#pragma once
#include <stdint.h>

namespace gpl1 {

constexpr int MAX_M = 16;       // line-search memory
constexpr int MAX_RING = 4;     // alpha^(2) window: M_alpha <= 3

enum Status : int32_t {
    ST_OK_TOL = 0, ST_STATIONARY = 1, ST_MAX_ITER = 2, ST_TARGET = 3,
    ST_BACKTRACK = 4, ST_NONFINITE = -2
};

struct GPParams {
    double theta, beta, amin, amax, tau1, f_target, tol, rho;
    int32_t M, Malpha, max_iter, bt_cap;
    int32_t x0_fallback;       // start from 0 when f(P(x0)) >= f(0) = ||y||^2
    // host-mapped word the update kernel posts its progress to (updates
    // completed, bit 31 once a stop is requested), or NULL
    uint32_t* progress;
    // ring of per-update records (GP_TRACE_FIELDS doubles each), or NULL
    double* trace;
    int32_t trace_cap;
};

struct GPState {
    GPParams prm;
    // committed iterate scalars
    double f;                  // f(x^k)
    double fhist[MAX_M];       // ring of the last M objective values
    int32_t nhist, hpos;
    int32_t k;                 // accepted updates so far
    double alpha, tau;         // steplength for the next projection, SS threshold
    double a2v[MAX_RING];      // alpha^(2) values with their iteration index
    int32_t a2k[MAX_RING];
    int32_t na2;
    int32_t rule;              // last SS branch: 0 alpha_max, 1 BB1, 2 window min
    // written by the projection kernel
    double gd, dd, dmax, mu;
    double pm, pt;             // the iteration's projection: m = max|v| and t = mu - m
    int32_t hmode;             // h = sgn(v) max((|v| - m) - t, 0) (0), h = v (1, inside), h = 0 (2, rho = 0)
    // written by the update kernel (block 0)
    double lam, f_new, rel;
    int32_t k_new, pending, ss_pending, nb;
    int32_t backtracks;
    int32_t status, done, projected, x0_rejected;
    int32_t live, stop_req;
    int32_t michelot_iters;    // diagnostics: passes of the last threshold search
    int32_t michelot_total;    // diagnostics: passes summed over the iterations
    // final results
    double l1, gmax;
    // exact check of an objective target (see gp_verify.hpp)
    double f_target0;          // the caller's target (prm.f_target may be lowered below it)
    double f_exact;            // f recomputed in double at the last check
    int32_t tcheck;            // 1: a stop at the target passed the check
    int32_t reopened;          // checks that failed and reopened the problem
    int32_t reproj;            // uneven batches: reopened, needs a projection before its next sweep
    int32_t nactive;           // the last threshold search's active set size (-1: inside the ball)
};

}  // namespace gpl1
