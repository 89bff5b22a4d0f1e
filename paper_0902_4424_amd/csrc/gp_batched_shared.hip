// Batched GPSS: B problems min ||K x_b - y_b||^2 s.t. ||x_b||_1 <= rho_b that
// share one K (bf16 or FP32).  The two matrix products of an iteration become
// GEMMs on the bf16 matrix cores (gp_gemm.hpp):
//     Q = K D          (n x B, D = [d_1 .. d_B], the projected directions)
//     W = K^T Q        (p x B, W = K^T K D: the gradient change, since
//                       g_b(x + lam d) = g_b + 2 lam K^T K d_b)
// with D and Q split into three bf16 planes each, so the products carry FP32
// accuracy.  K^T is a transposed bf16 copy made once per call so that both
// GEMMs read their left operand with the reduction index contiguous.  An
// FP32 K is kept as three bf16 planes Kh + Km + Kl as well; a product is then
// Kh (Dh + Dm + Dl) + Km (Dh + Dm) + Kl Dh, formed in one GEMM pass that
// stages all six planes (the dropped plane products are below 2^-24 of the
// result).
//
// Everything per problem (projection and threshold search, the steplength
// rule of Algorithm 2, the closed-form Armijo backtracking of Algorithm 1,
// vector updates, stopping) runs in workgroups that each own one problem, so
// all per-problem scalars stay on the device and finished problems are
// frozen by their own flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gp_gemm.hpp"
#include "gp_internal.hpp"
#include "gp_kernels.hpp"
#include "gp_l1.h"
#include "gp_verify.hpp"

using namespace gpl1;

namespace gpl1 {

constexpr int BS_T = 1024;          // threads of the per-problem workgroups
constexpr int BS_PAD = 128;         // GEMM tile: M, N padding
constexpr int NSPL = 3;             // bf16 planes per FP32 operand

enum BsRowMode : int32_t { BR_REFRESH = 0, BR_ITER = 1 };
enum BsColMode : int32_t { BC_INIT = 0, BC_ITER = 1, BC_ITER_NOPROJ = 2, BC_REFRESH_PROJ = 3, BC_PROJ_ONLY = 4 };
// P.done values: 0 running, 1 stopped, 2 stopped with a target (to be
// checked), 3 reopened by the check (needs a projection before it runs on)

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// v = hi + mid + lo with each part a bf16 (hi = bf16(v), mid = bf16(v - hi),
// lo = bf16(v - hi - mid), remainders formed in double).
__device__ __forceinline__ void split3(double v, uint16_t* planes, int64_t pstride, int64_t idx) {
    const uint16_t h = f32_to_bf16_rne((float)v);
    const double r1 = v - (double)bf16_bits_to_f32(h);
    const uint16_t mmid = f32_to_bf16_rne((float)r1);
    const double r2 = r1 - (double)bf16_bits_to_f32(mmid);
    const uint16_t l = f32_to_bf16_rne((float)r2);
    planes[idx] = h;
    planes[pstride + idx] = mmid;
    planes[2 * pstride + idx] = l;
}

// Padded copies of K: Kp (npad x ppad, row-major) and Kt (ppad x npad).
__global__ void k_bs_pack(const uint16_t* __restrict__ K, int64_t n, int64_t p, int64_t ldk,
                          uint16_t* __restrict__ Kp, int64_t ldkp, uint16_t* __restrict__ Kt, int64_t ldkt) {
    __shared__ uint16_t tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 256 threads: 64 x 4
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, j = j0 + tx;
        const uint16_t v = (i < n && j < p) ? K[i * ldk + j] : (uint16_t)0;
        tile[r][tx] = v;
        Kp[i * ldkp + j] = v;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t j = j0 + r, i = i0 + tx;
        Kt[j * ldkt + i] = tile[tx][r];
    }
}

// FP32 K: padded copies as three bf16 planes each (plane strides kps, kts).
__global__ void k_bs_pack_f32(const float* __restrict__ K, int64_t n, int64_t p, int64_t ldk,
                              uint16_t* __restrict__ Kp, int64_t ldkp, int64_t kps, uint16_t* __restrict__ Kt,
                              int64_t ldkt, int64_t kts) {
    __shared__ float tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 256 threads: 64 x 4
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, j = j0 + tx;
        const float v = (i < n && j < p) ? K[i * ldk + j] : 0.f;
        tile[r][tx] = v;
        split3((double)v, Kp, kps, i * ldkp + j);
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t j = j0 + r, i = i0 + tx;
        split3((double)tile[tx][r], Kt, kts, j * ldkt + i);
    }
}

struct BsPtrs {
    GPState* st; int32_t* done;
    double *X, *G, *R, *Y, *Qv;              // B x p (X, G) and B x n (R, Y, Qv), ld = p / n
    uint16_t *Dsp, *Qsp;                      // GEMM right operands: 3 planes of Bpad x ppad / npad
    const float *Qpart, *Wpart;               // GEMM partial outputs
    int64_t n, p, npad, ppad, plD, plQ;       // plane strides of Dsp / Qsp
    int S1, S2;                               // split-K chunks of the two GEMMs
    int64_t sQ, sW;                           // partial strides (elements)
    const int32_t* list;                      // problems of the launch's workgroups (NULL: 0..B-1)
};

// ---------------------------------------------------------------------------
// init: state, x0 (projected if outside the ball), y; X split for K X
// ---------------------------------------------------------------------------
template <int NV>
__global__ __launch_bounds__(BS_T) void k_bs_init(BsPtrs P, GPParams prm, const double* __restrict__ rho,
                                                  const double* __restrict__ ftarget,
                                                  const void* __restrict__ Y, int64_t ldy,
                                                  const void* __restrict__ X0, int64_t ldx, int f64v) {
    __shared__ double lds[3 * (BS_T / WAVE)];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int64_t n = P.n, p = P.p;
    double* x = P.X + b * p;
    double* y = P.Y + b * n;
    for (int64_t i = tid; i < n; i += BS_T)
        y[i] = f64v ? ((const double*)Y)[b * ldy + i] : (double)((const float*)Y)[b * ldy + i];
    double vr[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * BS_T + tid) + (e & 1);
        double v = 0.0;
        if (X0 && j < p) v = f64v ? ((const double*)X0)[b * ldx + j] : (double)((const float*)X0)[b * ldx + j];
        vr[e] = v;
    }
    double m, t;
    bool inside;
    int passes;
    const double rb = rho[b];
    l1_threshold_regs<BS_T, NV>(vr, p, rb, -1.0, lds, m, t, inside, passes);
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * BS_T + tid) + (e & 1);
        if (j < p) {
            const double h = l1_hval(vr[e], m, t, inside, rb);
            x[j] = h;
            split3(h, P.Dsp, P.plD, b * P.ppad + j);
        }
    }
    if (tid == 0) {
        // written in place (a local copy of the state would go to scratch)
        GPState* sp = P.st + b;
        __builtin_memset(sp, 0, sizeof(GPState));
        sp->prm = prm;
        sp->prm.rho = rb;
        if (ftarget) sp->prm.f_target = ftarget[b];
        sp->f_target0 = sp->prm.f_target;
        sp->tau = prm.tau1;
        sp->alpha = prm.amax;
        sp->status = ST_MAX_ITER;
        sp->projected = inside ? 0 : 1;
        sp->live = 1;
        P.done[b] = 0;
    }
}

// ---------------------------------------------------------------------------
// row side: t = sum of the K-products; refresh (r = t - y) or the line search
// ---------------------------------------------------------------------------
// RPT > 0: n <= RPT * T, and an iteration keeps each thread's q_i and r_i in
// registers between the dots and the update; RPT = 0 parks q in Qv instead.
template <int T, int RPT>
__global__ __launch_bounds__(T) void k_bs_rows(BsPtrs P, int mode) {
    __shared__ double lds[3 * (T / WAVE)];
    __shared__ double sh[4];
    const int b = P.list ? P.list[blockIdx.x] : (int)blockIdx.x, tid = threadIdx.x;
    GPState* st = P.st + b;
    if (P.done[b]) return;
    const int64_t n = P.n;
    double* r = P.R + b * n;
    const double* y = P.Y + b * n;
    double* qv = P.Qv + b * n;
    auto tval = [&](int64_t i) {
        double s = 0.0;
        for (int c = 0; c < P.S1; ++c) s += (double)P.Qpart[c * P.sQ + b * P.npad + i];
        return s;
    };
    if (mode == BR_REFRESH) {
        // first pass with the x0 test: also ||y||^2 = f(0)
        const bool fb = st->prm.x0_fallback && st->k == 0 && st->nhist == 0;
        double acc[2] = {0.0, 0.0}, none[1] = {0.0};
        for (int64_t i = tid; i < n; i += T) {
            const double ri = tval(i) - y[i];
            r[i] = ri;
            acc[0] += ri * ri;
            acc[1] += y[i] * y[i];
            split3(ri, P.Qsp, P.plQ, b * P.npad + i);
        }
        block_reduce<T, 2, 1>(acc, none, lds);
        const bool reject = fb && !(acc[0] < acc[1]);
        if (reject) {
            // P(x0) is no better than 0: start from x = 0, r = -y
            for (int64_t i = tid; i < n; i += T) {
                r[i] = -y[i];
                split3(-y[i], P.Qsp, P.plQ, b * P.npad + i);
            }
            double* x = P.X + b * P.p;
            for (int64_t j = tid; j < P.p; j += T) x[j] = 0.0;
        }
        if (tid == 0) {
            const double f = reject ? acc[1] : acc[0];
            if (reject) st->x0_rejected = 1;
            if (st->k == 0 && st->nhist == 0) {
                st->hpos = 0;
                st->fhist[0] = f;
                st->nhist = 1;
            } else {
                st->fhist[st->hpos] = f;
            }
            st->f = f;
            if (!isfinite(f)) { st->status = ST_NONFINITE; st->done = 1; P.done[b] = 1; }
        }
        return;
    }
    // iteration: q = K d, its dots, the Armijo step, then r, x updates
    double acc[2] = {0.0, 0.0}, none[1] = {0.0};
    double qreg[RPT > 0 ? RPT : 1], rreg[RPT > 0 ? RPT : 1];
    if constexpr (RPT > 0) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int64_t i = tid + (int64_t)k * T;
            qreg[k] = rreg[k] = 0.0;
            if (i < n) {
                qreg[k] = tval(i);
                rreg[k] = r[i];
                acc[0] += qreg[k] * qreg[k];
                acc[1] += rreg[k] * qreg[k];
            }
        }
    } else {
        for (int64_t i = tid; i < n; i += T) {
            const double qi = tval(i);
            qv[i] = qi;
            acc[0] += qi * qi;
            acc[1] += r[i] * qi;
        }
    }
    block_reduce<T, 2, 1>(acc, none, lds);
    if (tid == 0) {
        const GPParams& Pm = st->prm;
        const double qq = acc[0], rq = acc[1], f = st->f, gd = st->gd;
        double fmax = f;
        const int nh = st->nhist < Pm.M ? st->nhist : Pm.M;
        for (int i = 0; i < nh; ++i) fmax = fmax > st->fhist[(st->hpos - i + MAX_M) % MAX_M]
                                              ? fmax : st->fhist[(st->hpos - i + MAX_M) % MAX_M];
        double lam = 1.0;
        int nb = 0;
        bool fail = false;
        for (;;) {
            const double inc = lam * (2.0 * rq + lam * qq);
            if (inc <= (fmax - f) + Pm.beta * lam * gd) break;
            if (++nb > Pm.bt_cap) { fail = true; break; }
            lam *= Pm.theta;
        }
        sh[0] = lam;
        sh[1] = fail ? 1.0 : 0.0;
        if (fail) {
            st->status = ST_BACKTRACK;
            st->done = 1;
            P.done[b] = st->f_target0 >= 0.0 ? 2 : 1;   // with a target: to be checked
        } else {
            const double fn = f + lam * (2.0 * rq + lam * qq);
            st->lam = lam;
            st->nb = nb;
            st->backtracks += nb;
            st->rel = (f - fn) / f;
            st->f = fn;
            st->k += 1;
            st->hpos = (st->hpos + 1) % MAX_M;
            st->fhist[st->hpos] = fn;
            if (st->nhist < MAX_M) st->nhist++;
            st->ss_pending = 1;
            int stop = 0;
            if (!isfinite(fn)) { st->status = ST_NONFINITE; stop = 1; }
            else if (Pm.f_target >= 0.0 && fn <= Pm.f_target) { st->status = ST_TARGET; stop = 2; }
            else if (Pm.tol > 0.0 && st->rel < Pm.tol) { st->status = ST_OK_TOL; stop = 1; }
            else if (st->k >= Pm.max_iter) { st->status = ST_MAX_ITER; stop = 1; }
            // a problem with a target is checked whatever ended it (2)
            if (stop) { st->done = 1; P.done[b] = (st->f_target0 >= 0.0 && stop != 0 && isfinite(fn)) ? 2 : 1; }
        }
    }
    __syncthreads();
    if (sh[1] != 0.0) return;
    const double lam = sh[0];
    if constexpr (RPT > 0) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int64_t i = tid + (int64_t)k * T;
            if (i < n) {
                r[i] = rreg[k] + lam * qreg[k];
                split3(qreg[k], P.Qsp, P.plQ, b * P.npad + i);
            }
        }
    } else {
        for (int64_t i = tid; i < n; i += T) {
            const double qi = qv[i];
            r[i] += lam * qi;
            split3(qi, P.Qsp, P.plQ, b * P.npad + i);
        }
    }
    // the p-space part of the step (x += lam d) is applied by the column
    // kernel, which reads x anyway
}

// ---------------------------------------------------------------------------
// column side: the accepted step (x += lam d with d = h - x, g += 2 lam w from
// W = K^T Q), the steplength rule, the projection, the next direction
// d = P(x - alpha g) - x and its dots, d split for the next K D.  Every
// thread keeps its elements of x and g in registers (pairs of neighbours), so
// each vector is read and written once per iteration.  h is not stored: the
// projection leaves (alpha, m, t, mode) in the problem's state, and the next
// launch recomputes h from the x and g it reads with the same operations.
// Modes: BC_INIT (g = 2 W at x0, then alpha_0 and the first projection);
// BC_ITER (step, rule, projection); BC_ITER_NOPROJ (step and rule only, x
// split for the residual refresh that follows); BC_REFRESH_PROJ (g = 2 W at
// the current x, then the projection).
// ---------------------------------------------------------------------------
template <int T, int NV>
__global__ __launch_bounds__(T) void k_bs_cols(BsPtrs P, int mode) {
    __shared__ double lds[3 * (T / WAVE)];
    __shared__ double sh[4];
    const int b = P.list ? P.list[blockIdx.x] : (int)blockIdx.x, tid = threadIdx.x;
    GPState* st = P.st + b;
    const int64_t p = P.p;
    double* x = P.X + b * p;
    double* g = P.G + b * p;
    const bool iter = mode == BC_ITER || mode == BC_ITER_NOPROJ;
    const int step_pending = iter ? st->ss_pending : 0;
    const int col_done = mode == BC_PROJ_ONLY ? 0 : P.done[b];
    if (col_done && !step_pending) return;
    auto wval = [&](int64_t j) {
        double sw = 0.0;
        for (int c = 0; c < P.S2; ++c) sw += (double)P.Wpart[c * P.sW + b * P.ppad + j];
        return sw;
    };
    // slot e <-> element j = 2*((e/2)*T + tid) + (e&1)
    double xr[NV], gr[NV];
    if (step_pending) {
        const double lam = st->lam;
        // the last projection's scalars, read before the rule below replaces alpha
        const ProjH ph = proj_h_params(st);
        double acc[2] = {0.0, 0.0}, none[1] = {0.0};
#pragma unroll
        for (int e = 0; e < NV; e += 2) {
            const int64_t j = 2 * ((e / 2) * T + tid);
            double xo[2] = {0.0, 0.0}, go[2] = {0.0, 0.0}, w[2] = {0.0, 0.0};
            if (j + 1 < p) {      // 16-byte loads for the pair
                const double2 x2 = *reinterpret_cast<const double2*>(x + j);
                const double2 g2 = *reinterpret_cast<const double2*>(g + j);
                xo[0] = x2.x; xo[1] = x2.y; go[0] = g2.x; go[1] = g2.y;
                w[0] = wval(j);
                w[1] = wval(j + 1);
            } else if (j < p) {
                xo[0] = x[j]; go[0] = g[j];
                w[0] = wval(j);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double dj = proj_h(xo[u], go[u], ph) - xo[u];   // the last h, recomputed
                xr[e + u] = xo[u] + lam * dj;
                gr[e + u] = go[u] + 2.0 * lam * w[u];
                acc[0] += dj * w[u];                             // d'w
                acc[1] += w[u] * w[u];                           // w'w
            }
        }
        block_reduce<T, 2, 1>(acc, none, lds);
        if (tid == 0) {
            // s = lam d, z = 2 lam w: s's = lam^2 d'd, s'z = 2 lam^2 d'w,
            // z'z = 4 lam^2 w'w (equation (5)), then Algorithm 2
            const double l2 = lam * lam;
            ss_update(st, st->k, l2 * st->dd, 2.0 * l2 * acc[0], 4.0 * l2 * acc[1]);
            st->ss_pending = 0;
        }
#pragma unroll
        for (int e = 0; e < NV; e += 2) {
            const int64_t j = 2 * ((e / 2) * T + tid);
            if (j + 1 < p) {
                *reinterpret_cast<double2*>(x + j) = make_double2(xr[e], xr[e + 1]);
                *reinterpret_cast<double2*>(g + j) = make_double2(gr[e], gr[e + 1]);
            } else if (j < p) {
                x[j] = xr[e];
                g[j] = gr[e];
            }
            if (mode == BC_ITER_NOPROJ) {
                if (j < p) split3(xr[e], P.Dsp, P.plD, b * P.ppad + j);
                if (j + 1 < p) split3(xr[e + 1], P.Dsp, P.plD, b * P.ppad + j + 1);
            }
        }
    } else if (mode == BC_PROJ_ONLY) {
        // a problem reopened by the target check: its step and steplength are
        // applied, x and g are current
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int64_t j = 2 * ((e / 2) * T + tid) + (e & 1);
            xr[e] = j < p ? x[j] : 0.0;
            gr[e] = j < p ? g[j] : 0.0;
        }
    } else {
        // BC_INIT / BC_REFRESH_PROJ: fresh gradient at the current x
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int64_t j = 2 * ((e / 2) * T + tid) + (e & 1);
            xr[e] = j < p ? x[j] : 0.0;
            gr[e] = j < p ? 2.0 * wval(j) : 0.0;
            if (j < p) g[j] = gr[e];
        }
    }
    if (col_done || mode == BC_ITER_NOPROJ) return;
    __syncthreads();
    if (tid == 0) { sh[0] = st->alpha; sh[1] = st->mu; sh[2] = st->prm.rho; }
    __syncthreads();
    const double rho = sh[2];
    double vr[NV];
    double m, t;
    bool inside;
    int passes;
    double alpha;
    if (mode == BC_INIT) {
        // alpha_0 = max{alpha_min, min{1/||P(x0 - grad f(x0))||_inf, alpha_max}}
#pragma unroll
        for (int e = 0; e < NV; ++e) vr[e] = xr[e] - gr[e];
        l1_threshold_regs<T, NV>(vr, p, rho, -1.0, lds, m, t, inside, passes);
        double hm = 0.0;
#pragma unroll
        for (int e = 0; e < NV; ++e) hm = fmax(hm, fabs(l1_hval(vr[e], m, t, inside, rho)));
        hm = block_max<T>(hm, lds);
        alpha = hm > 0.0 ? clamp_alpha(1.0 / hm, st->prm) : st->prm.amax;
        __syncthreads();
        if (tid == 0) st->alpha = alpha;
    } else {
        alpha = sh[0];
    }
    const double mu_prev = mode == BC_INIT ? 0.0 : sh[1];
#pragma unroll
    for (int e = 0; e < NV; ++e) vr[e] = fma(-alpha, gr[e], xr[e]);   // as proj_h forms it
    // warm start from the previous threshold when it lies below max|v|
    double mloc = 0.0;
#pragma unroll
    for (int e = 0; e < NV; ++e) mloc = fmax(mloc, fabs(vr[e]));
    mloc = block_max<T>(mloc, lds);
    const double start = (mu_prev > 0.0 && mu_prev < mloc) ? mu_prev - mloc : -1.0;
    l1_threshold_regs<T, NV>(vr, p, rho, start, lds, m, t, inside, passes);
    double sums[2] = {0.0, 0.0}, mx[1] = {0.0};
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int64_t j = 2 * ((e / 2) * T + tid) + (e & 1);
        if (j < p) {
            const double h = l1_hval(vr[e], m, t, inside, rho);
            const double dj = h - xr[e];
            split3(dj, P.Dsp, P.plD, b * P.ppad + j);
            sums[0] += gr[e] * dj;
            sums[1] += dj * dj;
            mx[0] = fmax(mx[0], fabs(dj));
        }
    }
    block_reduce<T, 2, 1>(sums, mx, lds);
    if (tid == 0) {
        if (!isfinite(m)) { st->status = ST_NONFINITE; st->done = 1; P.done[b] = 1; return; }
        st->gd = sums[0];
        st->dd = sums[1];
        st->dmax = mx[0];
        st->mu = inside ? 0.0 : m + t;
        // what the next launch needs to recompute h (alpha is already st->alpha)
        st->pm = m;
        st->pt = t;
        st->hmode = inside ? 1 : (rho > 0.0 ? 0 : 2);
        st->michelot_total += passes;
        if (mx[0] == 0.0 || !(sums[0] < 0.0)) {
            st->status = ST_STATIONARY;
            st->done = 1;
            P.done[b] = st->f_target0 >= 0.0 ? 2 : 1;   // with a target: to be checked
        } else if (mode == BC_PROJ_ONLY) {
            st->done = 0;
            P.done[b] = 0;
        }
    }
}

// Target check of the problems listed in `cand`: f = ||K x - y||^2 in double
// from the caller's K (widened exactly), y and x narrowed to float as
// returned.  The checked problems' iterates are not sparse enough to skip
// columns (GP keeps old entries whenever lambda < 1), so this is a batched
// product in double: a workgroup owns 64 rows of K, 64 checked problems and
// one of `ns` column chunks, stages K and x tiles of 32 columns in LDS (each K
// element read once for the 64 problems), and every thread accumulates 4 rows
// x 4 problems.  dot[(s * nc + c) * n + i] = sum over chunk s of K_ij x_cj.
constexpr int CV_T = 256, CV_R = 64, CV_C = 64, CV_J = 32;

template <typename TK> __device__ __forceinline__ double cv_widen(TK v);
template <> __device__ __forceinline__ double cv_widen<float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double cv_widen<uint16_t>(uint16_t v) { return (double)bf16_bits_to_f32(v); }

template <typename TK>
__global__ __launch_bounds__(CV_T) void k_bs_check_tiles(const TK* __restrict__ K, int64_t ldk, int64_t n,
                                                         int64_t p, const double* __restrict__ X,
                                                         const int32_t* __restrict__ cand, int nc, int64_t jchunk,
                                                         double* __restrict__ dot) {
    __shared__ double ks[CV_J][CV_R + 1];
    __shared__ double xs[CV_J][CV_C + 1];
    const int tid = threadIdx.x, tr = tid % 16, tc = tid / 16;
    const int64_t i0 = (int64_t)blockIdx.x * CV_R;
    const int c0 = (int)blockIdx.y * CV_C;
    const int64_t jb = (int64_t)blockIdx.z * jchunk;
    const int64_t je = jb + jchunk < p ? jb + jchunk : p;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int64_t j0 = jb; j0 < je; j0 += CV_J) {
        __syncthreads();
        for (int e = tid; e < CV_R * CV_J; e += CV_T) {
            const int r = e / CV_J, jj = e % CV_J;
            const int64_t i = i0 + r, j = j0 + jj;
            ks[jj][r] = (i < n && j < je) ? cv_widen<TK>(K[i * ldk + j]) : 0.0;
        }
        for (int e = tid; e < CV_C * CV_J; e += CV_T) {
            const int cc = e / CV_J, jj = e % CV_J;
            const int c = c0 + cc;
            const int64_t j = j0 + jj;
            xs[jj][cc] = (c < nc && j < je) ? (double)(float)X[(int64_t)cand[c] * p + j] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int jj = 0; jj < CV_J; ++jj) {
            double kr[4], xc[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) kr[a] = ks[jj][tr + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) xc[b] = xs[jj][tc + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(kr[a], xc[b], acc[a][b]);
        }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int c = c0 + tc + 16 * b;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int64_t i = i0 + tr + 16 * a;
            if (i < n && c < nc) dot[((int64_t)blockIdx.z * nc + c) * n + i] = acc[a][b];
        }
    }
}

// One workgroup per checked problem: r_i = (sum of the chunks' dots) - y_i,
// f = sum r_i^2 (fixed order), then the decision: P.done 1 (kept) or 3
// (reopened), kout[c] = iterations.
__global__ __launch_bounds__(256) void k_bs_check_decide(BsPtrs P, const double* __restrict__ dot, int ns, int nc,
                                                         const int32_t* __restrict__ cand,
                                                         int32_t* __restrict__ kout) {
    __shared__ double lds[256 / WAVE];
    const int c = blockIdx.x, b = cand[c];
    const int64_t n = P.n;
    const double* y = P.Y + (int64_t)b * n;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        double t = 0.0;
        for (int sidx = 0; sidx < ns; ++sidx) t += dot[((int64_t)sidx * nc + c) * n + i];
        const double d = t - y[i];
        acc += d * d;
    }
    const double f = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) {
        GPState* st = P.st + b;
        P.done[b] = target_decide(st, f) ? 1 : 3;
        kout[c] = st->k;
    }
}

// Column chunks of the check for nc problems: about 512 workgroups in all,
// at most 16 chunks, whole tiles of 32 columns per chunk.
void check_split(int64_t n, int64_t p, int nc, int* ns, int64_t* jchunk) {
    const int64_t wg = ((n + CV_R - 1) / CV_R) * ((nc + CV_C - 1) / CV_C);
    int64_t want = (512 + wg - 1) / wg;
    const int64_t tiles = (p + CV_J - 1) / CV_J;
    want = std::max<int64_t>(1, std::min<int64_t>({want, 16, tiles}));
    const int64_t tpc = (tiles + want - 1) / want;
    *jchunk = tpc * CV_J;
    *ns = (int)((p + *jchunk - 1) / *jchunk);
}

// results: ||x||_1, ||g||_inf and x out in the vector dtype
__global__ __launch_bounds__(BS_T) void k_bs_finish(BsPtrs P, void* __restrict__ Xout, int64_t ldx, int f64v) {
    __shared__ double lds[3 * (BS_T / WAVE)];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int64_t p = P.p;
    const double* x = P.X + b * p;
    const double* g = P.G + b * p;
    double s[1] = {0.0}, mx[1] = {0.0};
    for (int64_t j = tid; j < p; j += BS_T) {
        s[0] += fabs(x[j]);
        mx[0] = fmax(mx[0], fabs(g[j]));
        if (f64v) ((double*)Xout)[b * ldx + j] = x[j];
        else ((float*)Xout)[b * ldx + j] = (float)x[j];
    }
    block_reduce<BS_T, 1, 1>(s, mx, lds);
    if (tid == 0) {
        P.st[b].l1 = s[0];
        P.st[b].gmax = mx[0];
    }
}

namespace {

// Column-kernel shape: 256 threads up to p = 2048 and 512 threads up to
// p = 8192, 1024 beyond; each thread holds its elements in at most 16
// register slots, and up to p = 4096 in at most 8 (512 x 8 needs 102
// registers, four waves per SIMD, against 180 and two for 256 x 16), so that
// several problems share a CU and one problem's reductions overlap another's
// loads.
int bs_cols_t(int64_t p) {
    if ((p + 255) / 256 <= 8) return 256;
    if ((p + 511) / 512 <= 16) return 512;
    return 1024;
}

int bs_nv_t(int64_t p, int T) {
    const int64_t per = (p + T - 1) / T;
    if (per <= 2) return 2;
    if (per <= 4) return 4;
    if (per <= 8) return 8;
    if (per <= 16) return 16;
    return 0;
}

int bs_nv(int64_t p) {
    const int64_t per = (p + BS_T - 1) / BS_T;
    if (per <= 2) return 2;
    if (per <= 4) return 4;
    if (per <= 8) return 8;
    if (per <= 16) return 16;
    return 0;
}

#define GPL1_BS_NV_SWITCH(nv, STMT) \
    switch (nv) {                   \
        case 2: { constexpr int NVc = 2; STMT; } break;   \
        case 4: { constexpr int NVc = 4; STMT; } break;   \
        case 8: { constexpr int NVc = 8; STMT; } break;   \
        case 16: { constexpr int NVc = 16; STMT; } break; \
    }

// the (threads, slots) shapes of k_bs_cols that are compiled
#define GPL1_BS_COLS_SHAPES(X) \
    X(256, 2) X(256, 4) X(256, 8) X(512, 4) X(512, 8) X(512, 16) X(1024, 2) X(1024, 4) X(1024, 8) X(1024, 16)
// the (threads, rows per thread in registers; 0 = q parked in memory) shapes
// of k_bs_rows that are compiled
#define GPL1_BS_ROWS_SHAPES(X) \
    X(256, 4) X(256, 8) X(256, 0) X(512, 2) X(512, 4) X(512, 0) X(1024, 1) X(1024, 2) X(1024, 4) X(1024, 0)

// rows per thread of the row kernel with T threads: the smallest compiled
// register count that holds n, else 0
int rows_rpt(int64_t n, int T) {
    const int64_t per = (n + T - 1) / T;
    static const int opts256[] = {4, 8}, opts512[] = {2, 4}, opts1024[] = {1, 2, 4};
    const int* o = T == 256 ? opts256 : T == 512 ? opts512 : opts1024;
    const int no = T == 1024 ? 3 : 2;
    for (int i = 0; i < no; ++i)
        if (per <= o[i]) return o[i];
    return 0;
}

void launch_rows(int T, int rpt, int64_t B, hipStream_t s, const BsPtrs& P, int mode) {
#define GPL1_BS_ROWS(TT, RR) \
    if (T == TT && rpt == RR) { hipLaunchKernelGGL((k_bs_rows<TT, RR>), dim3((unsigned)B), dim3(TT), 0, s, P, mode); return; }
    GPL1_BS_ROWS_SHAPES(GPL1_BS_ROWS)
#undef GPL1_BS_ROWS
}

bool cols_shape_ok(int T, int nv) {
#define GPL1_BS_OK(TT, NN) \
    if (T == TT && nv == NN) return true;
    GPL1_BS_COLS_SHAPES(GPL1_BS_OK)
#undef GPL1_BS_OK
    return false;
}

void launch_cols(int T, int nv, int64_t B, hipStream_t s, const BsPtrs& P, int mode) {
#define GPL1_BS_COLS(TT, NN) \
    if (T == TT && nv == NN) { hipLaunchKernelGGL((k_bs_cols<TT, NN>), dim3((unsigned)B), dim3(TT), 0, s, P, mode); return; }
    GPL1_BS_COLS_SHAPES(GPL1_BS_COLS)
#undef GPL1_BS_COLS
}

int64_t rup(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

int severity(int s) {
    if (s < 0) return 100 - s;
    if (s == GP_BACKTRACK_LIMIT) return 4;
    if (s == GP_MAX_ITER) return 3;
    return 1;
}

}  // namespace

// The MFMA path; returns GP_E_UNSUPPORTED (nothing launched) if the shape or
// dtype does not fit it.
int solve_batched_shared_mfma(gp_handle h, gp_dtype kdtype, const void* K, int64_t n, int64_t p, int64_t ldk,
                              const void* Y, int64_t ldy, int64_t B, const double* rho, const void* X0,
                              int64_t ldx, double tol, void* X_out, const gp_opts& o, gp_result* res,
                              hipStream_t s) {
    if (kdtype != GP_BF16 && kdtype != GP_F32) return GP_E_UNSUPPORTED;
    const int nK = kdtype == GP_F32 ? 3 : 1;   // bf16 planes of K
    const int nv = bs_nv(p);
    const int ct = o.batch_cols_t ? o.batch_cols_t : bs_cols_t(p), cnv = bs_nv_t(p, ct);
    if (nv == 0 || B > (1 << 20)) return GP_E_UNSUPPORTED;
    if (!cols_shape_ok(ct, cnv)) {
        if (o.batch_cols_t)
            return fail(h, GP_E_ARG, "opts.batch_cols_t = " + std::to_string(ct) + " has no column-kernel shape for p = " +
                                         std::to_string(p));
        return GP_E_UNSUPPORTED;
    }
    const int rt = o.batch_rows_t ? o.batch_rows_t : 256, rrpt = rows_rpt(n, rt);
    const int64_t npad = rup(n, BS_PAD), ppad = rup(p, BS_PAD), bpad = rup(B, BS_PAD);
    // split-K chunks (multiples of 32 dividing the padded size) per GEMM:
    // about 1024 (512 with 256-row tiles), or the tuned size
    const bool tile256 = nK == 1 && o.batch_gemm_tile == 256;
    auto chunk_of = [&](int64_t kd) {
        int64_t c = std::min<int64_t>(kd, o.batch_splitk > 0 ? o.batch_splitk : (tile256 ? 512 : 1024));
        while (kd % c) c -= 32;
        return c;
    };
    const int64_t kc1 = chunk_of(ppad), kc2 = chunk_of(npad);
    const int S1 = (int)(ppad / kc1), S2 = (int)(npad / kc2);
    const int64_t kpl = npad * ppad;           // elements of one K plane

    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = off; off += (bytes + 255) / 256 * 256; return o2; };
    const size_t o_st = take(sizeof(GPState) * B), o_done = take(sizeof(int32_t) * B);
    const size_t o_X = take(8 * B * p), o_G = take(8 * B * p);
    const size_t o_R = take(8 * B * n), o_Y = take(8 * B * n), o_Qv = take(8 * B * n);
    const size_t o_Kp = take(2 * nK * kpl), o_Kt = take(2 * nK * kpl);
    // GEMM right operands and outputs get one extra row (index bpad) that
    // stays zero: the column list of a compacted batch is padded with it
    const int64_t brows = bpad + 1;
    const size_t o_Dsp = take(2 * NSPL * brows * ppad), o_Qsp = take(2 * NSPL * brows * npad);
    const size_t o_Qp = take(4 * (size_t)S1 * brows * npad), o_Wp = take(4 * (size_t)S2 * brows * ppad);
    const size_t o_rho = take(8 * B), o_ft = take(8 * B), o_list = take(4 * bpad);
    const size_t o_cand = take(4 * B), o_kout = take(4 * B);
    // target check: the dots of every (column chunk, checked problem, row),
    // for the largest chunk count x problem count a check can need
    size_t check_elems = 0;
    if (o.f_target >= 0.0 || o.f_targets) {
        for (int64_t g = 1; g <= (B + CV_C - 1) / CV_C; ++g) {
            int ns;
            int64_t jchunk;
            const int nc = (int)std::min<int64_t>(B, g * CV_C);
            check_split(n, p, nc, &ns, &jchunk);
            check_elems = std::max(check_elems, (size_t)ns * nc * n);
        }
    }
    const size_t o_check = take(8 * check_elems);
    int rc = ensure_workspace(h, off);
    if (rc) return rc;
    if (o.graph && (rc = graph_stream(h, s, &s))) return rc;
    char* ws = (char*)h->ws;
    BsPtrs P;
    P.st = (GPState*)(ws + o_st);
    P.done = (int32_t*)(ws + o_done);
    P.X = (double*)(ws + o_X); P.G = (double*)(ws + o_G);
    P.R = (double*)(ws + o_R); P.Y = (double*)(ws + o_Y); P.Qv = (double*)(ws + o_Qv);
    uint16_t* Kp = (uint16_t*)(ws + o_Kp);
    uint16_t* Kt = (uint16_t*)(ws + o_Kt);
    P.Dsp = (uint16_t*)(ws + o_Dsp); P.Qsp = (uint16_t*)(ws + o_Qsp);
    float* Qpart = (float*)(ws + o_Qp);
    float* Wpart = (float*)(ws + o_Wp);
    P.Qpart = Qpart; P.Wpart = Wpart;
    P.n = n; P.p = p; P.npad = npad; P.ppad = ppad;
    P.plD = brows * ppad; P.plQ = brows * npad;
    P.S1 = S1; P.S2 = S2;
    P.sQ = brows * npad; P.sW = brows * ppad;
    P.list = nullptr;
    int32_t* dlist = (int32_t*)(ws + o_list);
    int32_t* dcand = (int32_t*)(ws + o_cand);
    int32_t* dkout = (int32_t*)(ws + o_kout);
    double* dcheck = (double*)(ws + o_check);
    const bool check_target = o.f_target >= 0.0 || o.f_targets != nullptr;
    double* drho = (double*)(ws + o_rho);
    double* dft = o.f_targets ? (double*)(ws + o_ft) : nullptr;

    hipError_t e = hipMemcpyAsync(drho, rho, 8 * B, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && dft) e = hipMemcpyAsync(dft, o.f_targets, 8 * B, hipMemcpyHostToDevice, s);
    // zero padding of the GEMM operands (rows beyond n, p and columns beyond B)
    if (e == hipSuccess) e = hipMemsetAsync(P.Dsp, 0, 2 * NSPL * brows * ppad, s);
    if (e == hipSuccess) e = hipMemsetAsync(P.Qsp, 0, 2 * NSPL * brows * npad, s);
    if (e != hipSuccess) return hip_fail(h, e, "batched set-up");
    if (nK == 1)
        hipLaunchKernelGGL(k_bs_pack, dim3((unsigned)(ppad / 64), (unsigned)(npad / 64)), dim3(256), 0, s,
                           (const uint16_t*)K, n, p, ldk, Kp, ppad, Kt, npad);
    else
        hipLaunchKernelGGL(k_bs_pack_f32, dim3((unsigned)(ppad / 64), (unsigned)(npad / 64)), dim3(256), 0, s,
                           (const float*)K, n, p, ldk, Kp, ppad, kpl, Kt, npad, kpl);
    GPParams prm = make_params(o, 0.0, tol);
    prm.x0_fallback = (o.x0_fallback && X0) ? 1 : 0;
    const int f64v = 0;
    GPL1_BS_NV_SWITCH(nv, hipLaunchKernelGGL(k_bs_init<NVc>, dim3((unsigned)B), dim3(BS_T), 0, s, P, prm, drho,
                                             dft, Y, ldy, X0, ldx, f64v));
    // bf16 K: one plane times the three planes of the right operand; FP32 K:
    // the six plane products of k_gemm_bf16_planes<3, 3> in one pass
    // Active set: after each status poll the problems still running are
    // listed (padded to the tile with the zero row), and the GEMMs and the
    // per-problem kernels cover only them.
    int64_t live = B;
    auto gemm_planes = [&](const uint16_t* A0, int64_t lda, int64_t M, const uint16_t* Bpl, int64_t ldb,
                           int64_t plB, int S, int64_t kc, float* Cp, int64_t ldc, int64_t cs) {
        const dim3 grid((unsigned)(M / GM_BM), (unsigned)(rup(live, GM_BN) / GM_BN), (unsigned)S);
        if (nK == 1 && (grid.y == 1 || o.batch_gemm_tile == 64))
            // 64-column tiles (same bits): always when asked, else once one
            // 128-column tile is left, where they keep the chip busy
            hipLaunchKernelGGL(k_gemm_bf16_n64<NSPL>, dim3(grid.x, grid.y * (unsigned)(GM_BN / GM3_BN), grid.z),
                               dim3(GM_T), 0, s, A0, lda, Bpl, ldb, plB, (int)kc, Cp, ldc, cs, P.list);
        else if (tile256)
            hipLaunchKernelGGL(k_gemm_bf16_m256<NSPL>, dim3((unsigned)((M + GM2_BM - 1) / GM2_BM), grid.y, grid.z),
                               dim3(GM2_T), 0, s, A0, lda, Bpl, ldb, plB, (int)kc, Cp, ldc, cs, P.list, M);
        else if (nK == 1 && o.batch_gemm_depth == 2)
            hipLaunchKernelGGL(k_gemm_bf16_d2<NSPL>, grid, dim3(GM_T), 0, s, A0, lda, Bpl, ldb, plB, (int)kc, Cp, ldc,
                               cs, P.list);
        else if (nK == 1)
            hipLaunchKernelGGL(k_gemm_bf16<NSPL>, grid, dim3(GM_T), 0, s, A0, lda, Bpl, ldb, plB, (int)kc, Cp, ldc, cs,
                               P.list);
        else
            hipLaunchKernelGGL((k_gemm_bf16_planes<3, 3>), grid, dim3(GM_T), 0, s, A0, lda, kpl, Bpl, ldb, plB,
                               (int)kc, Cp, ldc, cs, P.list);
    };
    auto gemm1 = [&]() {   // Qpart = K * (Dsp planes)
        gemm_planes(Kp, ppad, npad, P.Dsp, ppad, P.plD, S1, kc1, Qpart, npad, P.sQ);
    };
    auto gemm2 = [&]() {   // Wpart = K^T * (Qsp planes)
        gemm_planes(Kt, npad, ppad, P.Qsp, npad, P.plQ, S2, kc2, Wpart, ppad, P.sW);
    };
    auto rows = [&](int mode) {
        launch_rows(rt, rrpt, live, s, P, mode);
    };
    auto cols = [&](int mode) {
        launch_cols(ct, cnv, live, s, P, mode);
    };
    // r = K x - y, g = 2 K^T r, alpha_0, first direction
    gemm1();
    rows(BR_REFRESH);
    gemm2();
    cols(BC_INIT);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "batched init launch");

    // target check of the problems that stopped at their target (P.done 2)
    auto launch_verify = [&](int nc) {
        int ns;
        int64_t jchunk;
        check_split(n, p, nc, &ns, &jchunk);
        const dim3 g((unsigned)((n + CV_R - 1) / CV_R), (unsigned)((nc + CV_C - 1) / CV_C), (unsigned)ns);
        if (nK == 1)
            hipLaunchKernelGGL(k_bs_check_tiles<uint16_t>, g, dim3(CV_T), 0, s, (const uint16_t*)K, ldk, n, p,
                               (const double*)P.X, dcand, nc, jchunk, dcheck);
        else
            hipLaunchKernelGGL(k_bs_check_tiles<float>, g, dim3(CV_T), 0, s, (const float*)K, ldk, n, p,
                               (const double*)P.X, dcand, nc, jchunk, dcheck);
        hipLaunchKernelGGL(k_bs_check_decide, dim3((unsigned)nc), dim3(256), 0, s, P, dcheck, ns, nc, dcand, dkout);
    };
    // status flags and the active list go through the handle's pinned buffer,
    // so the copies are plain DMA and the list upload needs no wait of its own
    if ((rc = ensure_pinned(h, 4 * (size_t)(B + bpad)))) return rc;
    int32_t* hdone = (int32_t*)h->pin;
    int32_t* hlist = hdone + B;
    std::vector<int32_t> hcand, hk;
    // a problem that is never stopped has done exactly `it` iterations; one
    // reopened by a target check at iteration k needs max_iter - k more
    int it = 0, it_cap = o.max_iter;
    auto iteration = [&](int i) {
        const bool refresh = o.refresh_every > 0 && (i + 1) % o.refresh_every == 0 && i + 1 < it_cap;
        gemm1();
        rows(BR_ITER);
        gemm2();
        if (refresh) {
            cols(BC_ITER_NOPROJ);
            gemm1();
            rows(BR_REFRESH);
            gemm2();
            cols(BC_REFRESH_PROJ);
        } else {
            cols(BC_ITER);
        }
    };
    // graph replay: chunks of gch iterations starting at multiples of gch
    // (the refresh that the plain schedule puts at their end included),
    // captured again whenever the running problems change the launch sizes
    const int gch = o.refresh_every > 0 ? o.refresh_every : o.chunk;
    int64_t glive = -1;
    while (it < it_cap) {
        if (o.graph && it % gch == 0 && it + gch < it_cap) {
            if (glive != live) {
                const int base = it;
                if ((rc = capture_graph(h, s, &h->gexec_b, [&]() {
                         for (int k = 0; k < gch; ++k) iteration(base + k);
                     })))
                    return rc;
                glive = live;
            }
            e = hipGraphLaunch(h->gexec_b, s);
            if (e != hipSuccess) return hip_fail(h, e, "batched graph launch");
            it += gch;
        } else {
            const int end = o.graph ? std::min(it_cap, (it / gch + 1) * gch) : std::min(it_cap, it + o.chunk);
            for (; it < end; ++it) iteration(it);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(h, e, "batched iteration launch");
        e = hipMemcpyAsync(hdone, P.done, 4 * B, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "batched status poll");
        if (check_target) {
            hcand.clear();
            for (int64_t b = 0; b < B; ++b)
                if (hdone[(size_t)b] == 2) hcand.push_back((int32_t)b);
            const int nc = (int)hcand.size();
            if (nc > 0) {
                e = hipMemcpyAsync(dcand, hcand.data(), 4 * nc, hipMemcpyHostToDevice, s);
                if (e != hipSuccess) return hip_fail(h, e, "batched target check");
                launch_verify(nc);
                hk.resize((size_t)nc);
                e = hipGetLastError();
                if (e == hipSuccess) e = hipMemcpyAsync(hdone, P.done, 4 * B, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipMemcpyAsync(hk.data(), dkout, 4 * nc, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_fail(h, e, "batched target check");
                // reopened problems: a fresh projection, then they run on
                int nr = 0;
                for (int c = 0; c < nc; ++c) {
                    const int32_t b = hcand[(size_t)c];
                    if (hdone[(size_t)b] != 3) continue;
                    hcand[(size_t)nr++] = b;
                    hdone[(size_t)b] = 0;
                    it_cap = std::max(it_cap, it + (o.max_iter - hk[(size_t)c]));
                }
                if (nr > 0) {
                    e = hipMemcpyAsync(dcand, hcand.data(), 4 * nr, hipMemcpyHostToDevice, s);
                    if (e != hipSuccess) return hip_fail(h, e, "batched target check");
                    BsPtrs Pr = P;
                    Pr.list = dcand;
                    launch_cols(ct, cnv, nr, s, Pr, BC_PROJ_ONLY);
                    e = hipGetLastError();
                    if (e == hipSuccess) e = hipStreamSynchronize(s);   // hcand is reused at the next poll
                    if (e != hipSuccess) return hip_fail(h, e, "batched target check");
                }
            }
        }
        int64_t nlive = 0;
        for (int64_t b = 0; b < B; ++b)
            if (!hdone[(size_t)b]) hlist[(size_t)nlive++] = (int32_t)b;
        if (nlive == 0) break;
        if (nlive != live) {
            // compact: later launches cover the listed problems only
            for (int64_t k = nlive; k < rup(nlive, GM_BN); ++k) hlist[(size_t)k] = (int32_t)bpad;
            // (hlist is next written after the next poll's synchronisation)
            e = hipMemcpyAsync(dlist, hlist, 4 * rup(nlive, GM_BN), hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(h, e, "batched active set");
            live = nlive;
            P.list = dlist;
        }
    }
    hipLaunchKernelGGL(k_bs_finish, dim3((unsigned)B), dim3(BS_T), 0, s, P, X_out, ldx, f64v);
    std::vector<GPState> hst((size_t)B);
    e = hipMemcpyAsync(hst.data(), P.st, sizeof(GPState) * B, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "batched final sync");
    int worst = GP_OK_TOL;
    for (int64_t b = 0; b < B; ++b) {
        fill_result(hst[(size_t)b], &res[b]);
        if (severity(res[b].status) > severity(worst)) worst = res[b].status;
    }
    return worst;
}

}  // namespace gpl1
