// Kernels of one GPSS iteration on MI355X.  Per iteration three launches:
//
//   k_proj   (1 workgroup)  : steplength rule (Algorithm 2), v = x - alpha g,
//                             threshold search for P_Omega, h = P(v)
//                             (Algorithm 1, projection).  Stores the float
//                             copy of d = h - x and the scalars from which
//                             the other kernels recompute h (proj_h).
//   k_fused  (G workgroups) : d = h - x (Algorithm 1, direction), then one
//                             read of K serves both products: every workgroup
//                             owns a slab of rows, forms q_i = K_i d for its
//                             rows and, while that slab of K is still in
//                             registers, adds K_i^T q_i into a private
//                             p-vector.  Output: q (n), G partial vectors of
//                             w = K^T K d, and per-workgroup partial dots g'd,
//                             d'd, ||d||_inf over a slice of the columns.
//   k_update (many)         : stationarity test (d = 0 or g'd >= 0),
//                             closed-form Armijo backtracking from
//                             (f, g'd, r'q, q'q), x += lam d, r += lam q,
//                             g += 2 lam w (the new gradient 2 K^T r), and the
//                             dots d'w, w'w that Algorithm 2 needs next.
//
// With f quadratic, f(x + lam d) = f + 2 lam r'q + lam^2 q'q with r = Kx - y
// and q = Kd, so every backtracking trial is a scalar formula, and
// grad f(x + lam d) = g + 2 lam K^T K d, so the new gradient needs K^T q only.
#pragma once

#include <type_traits>

#include "gp_device.hpp"
#include "gp_state.hpp"

namespace gpl1 {

enum ProjMode : int32_t { PM_ITER = 0, PM_INIT_X0 = 1, PM_ALPHA0 = 2, PM_PLAIN = 3 };
enum UpdMode : int32_t { UM_ITER = 0, UM_REFRESH = 1 };

constexpr int PROJ_T = 1024;
constexpr int UPD_T = 256;
constexpr int UPD_COLS = 32;   // columns per p-part workgroup of k_update
constexpr int UPD_ROWS = 256;  // rows per n-part workgroup of k_update
constexpr int TRACE_FIELDS = 10;   // doubles per record of the per-update trace
constexpr int SPART = 8;       // doubles per fused-kernel workgroup in spart:
                               // t't, t'r, g'd, d'd, ||d||_inf

// ---------------------------------------------------------------------------
// The state is staged through LDS: one coalesced load by the workgroup
// instead of a chain of dependent global loads by one thread.
// ---------------------------------------------------------------------------
static_assert(sizeof(GPState) % 4 == 0, "state is copied as 32-bit words");
constexpr int STATE_WORDS = (int)(sizeof(GPState) / 4);

__device__ __forceinline__ void state_load(GPState& dst, const GPState* src) {
    for (int i = threadIdx.x; i < STATE_WORDS; i += blockDim.x)
        reinterpret_cast<uint32_t*>(&dst)[i] = reinterpret_cast<const uint32_t*>(src)[i];
}
__device__ __forceinline__ void state_store(GPState* dst, const GPState& src) {
    for (int i = threadIdx.x; i < STATE_WORDS; i += blockDim.x)
        reinterpret_cast<uint32_t*>(dst)[i] = reinterpret_cast<const uint32_t*>(&src)[i];
}

// ---------------------------------------------------------------------------
// scalar logic (thread 0 of a workgroup)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double clamp_alpha(double a, const GPParams& P) {
    return fmax(P.amin, fmin(a, P.amax));
}

// Make the update of the previous launch visible in the committed fields.
__device__ __forceinline__ void commit_pending(GPState* st) {
    if (!st->pending) return;
    if (st->k_new != st->k) {               // a new iterate: push f into the ring
        st->hpos = (st->hpos + 1) % MAX_M;
        st->fhist[st->hpos] = st->f_new;
        if (st->nhist < MAX_M) st->nhist++;
    } else {                                // same iterate, f recomputed (refresh)
        st->fhist[st->hpos] = st->f_new;
        if (st->nhist == 0) st->nhist = 1;  // f(x^0): the first value of the window
    }
    st->f = st->f_new;
    st->k = st->k_new;
    st->pending = 0;
}

// Algorithm 2 for iteration k >= 1 from s's, s'z, z'z of the last step.
// Readings: if s'z <= 0 the threshold is kept and no alpha^(2) is recorded;
// the ratio test and the window minimum use the clamped values; the window
// holds the recorded alpha^(2) of iterations max(1, k - M_alpha) .. k.
__device__ __forceinline__ void ss_update(GPState* st, int k, double ss, double sz, double zz) {
    const GPParams& P = st->prm;
    if (!(sz > 0.0)) {
        st->alpha = P.amax;
        st->rule = 0;
        return;
    }
    const double a1 = clamp_alpha(ss / sz, P);
    const double a2 = zz > 0.0 ? clamp_alpha(sz / zz, P) : P.amax;
    const int first = k - P.Malpha > 1 ? k - P.Malpha : 1;
    int m = 0;
    for (int i = 0; i < st->na2; ++i) {
        if (st->a2k[i] >= first) {
            st->a2k[m] = st->a2k[i];
            st->a2v[m] = st->a2v[i];
            ++m;
        }
    }
    if (m == MAX_RING) {                    // cannot happen for M_alpha <= 3
        for (int i = 1; i < MAX_RING; ++i) { st->a2k[i - 1] = st->a2k[i]; st->a2v[i - 1] = st->a2v[i]; }
        --m;
    }
    st->a2k[m] = k;
    st->a2v[m] = a2;
    st->na2 = m + 1;
    if (a2 / a1 <= st->tau) {
        double a = st->a2v[0];
        for (int i = 1; i < st->na2; ++i) a = fmin(a, st->a2v[i]);
        st->alpha = a;
        st->tau *= 0.9;
        st->rule = 2;
    } else {
        st->alpha = a1;
        st->tau *= 1.1;
        st->rule = 1;
    }
}

// The projection's scalar step in an iteration: commit_pending, then (when the
// last update left its dots) ss_update, with the same arithmetic.  Every field
// it reads is loaded up front and the alpha^(2) window is kept in registers,
// so the single thread that runs it waits for LDS once instead of once per
// dependent access.
__device__ __forceinline__ void iter_rule(GPState& S, bool need_ss, double dw, double ww) {
    const int pending = S.pending, k_new = S.k_new, k0 = S.k, hpos0 = S.hpos, nhist0 = S.nhist;
    const double f_new = S.f_new, lam = S.lam, dd = S.dd, tau = S.tau;
    const double amin = S.prm.amin, amax = S.prm.amax;
    const int Malpha = S.prm.Malpha, na2 = S.na2;
    int a2k[MAX_RING];
    double a2v[MAX_RING];
#pragma unroll
    for (int i = 0; i < MAX_RING; ++i) { a2k[i] = S.a2k[i]; a2v[i] = S.a2v[i]; }

    int k = k0;
    if (pending) {
        int hpos = hpos0;
        if (k_new != k0) {                  // a new iterate: push f into the ring
            hpos = (hpos0 + 1) % MAX_M;
            S.hpos = hpos;
            S.nhist = nhist0 < MAX_M ? nhist0 + 1 : nhist0;
        } else if (nhist0 == 0) {           // f(x^0): the first value of the window
            S.nhist = 1;
        }
        S.fhist[hpos] = f_new;
        S.f = f_new;
        S.k = k_new;
        S.pending = 0;
        k = k_new;
    }
    if (!need_ss) return;
    S.ss_pending = 0;
    // s = lam d, z = 2 lam w (w = K^T K d): s's = lam^2 d'd, s'z = 2 lam^2 d'w,
    // z'z = 4 lam^2 w'w (equation (5))
    const double l2 = lam * lam;
    const double ss = l2 * dd, sz = 2.0 * l2 * dw, zz = 4.0 * l2 * ww;
    if (!(sz > 0.0)) {
        S.alpha = amax;
        S.rule = 0;
        return;
    }
    const double a1 = fmax(amin, fmin(ss / sz, amax));
    const double a2 = zz > 0.0 ? fmax(amin, fmin(sz / zz, amax)) : amax;
    const int first = k - Malpha > 1 ? k - Malpha : 1;
    // keep the recorded entries of iterations >= first, in order
    int nk[MAX_RING] = {}, m = 0;
    double nv[MAX_RING] = {};
#pragma unroll
    for (int i = 0; i < MAX_RING; ++i) {
        const bool keep = i < na2 && a2k[i] >= first;
#pragma unroll
        for (int o = 0; o < MAX_RING; ++o)
            if (keep && m == o) { nk[o] = a2k[i]; nv[o] = a2v[i]; }
        m += keep ? 1 : 0;
    }
    if (m == MAX_RING) {                    // cannot happen for M_alpha <= 3
#pragma unroll
        for (int o = 0; o + 1 < MAX_RING; ++o) { nk[o] = nk[o + 1]; nv[o] = nv[o + 1]; }
        --m;
    }
#pragma unroll
    for (int o = 0; o < MAX_RING; ++o)
        if (o == m) { nk[o] = k; nv[o] = a2; }
    const int nn = m + 1;
#pragma unroll
    for (int o = 0; o < MAX_RING; ++o) { S.a2k[o] = nk[o]; S.a2v[o] = nv[o]; }
    S.na2 = nn;
    if (a2 / a1 <= tau) {
        double a = nv[0];
#pragma unroll
        for (int o = 1; o < MAX_RING; ++o)
            if (o < nn) a = fmin(a, nv[o]);
        S.alpha = a;
        S.tau = tau * 0.9;
        S.rule = 2;
    } else {
        S.alpha = a1;
        S.tau = tau * 1.1;
        S.rule = 1;
    }
}

// ---------------------------------------------------------------------------
// k_proj: projection onto the l1 ball by a parallel threshold search.
//
// With b_i = |v_i| - m (m = max|v|), the threshold t = mu - m solves
// phi(t) = sum max(b_i - t, 0) = rho.  phi is convex, piecewise linear and
// decreasing, and a Newton step from any t,
//     A = {i : b_i > t},  t <- (sum_A b_i - rho) / |A|,
// lands at or left of the root (the tangent of a convex function lies below
// it).  From the left the same step is Michelot's: the sets A shrink
// monotonically and the pass whose set does not change gives the exact
// threshold.  So the search may start anywhere with t < 0: in the iteration
// it starts from the previous iteration's threshold, which usually leaves
// one or two passes.  Every pass is one workgroup reduction of (count, sum)
// over values held in registers (VPT per thread; VPT = 0 streams from vbuf).
// ---------------------------------------------------------------------------
// Threshold of the projection for values held in registers (slot e of
// thread tid is element 2*((e/2)*T + tid) + (e&1), elements >= p are
// ignored).  Returns m = max|v|, inside = (||v||_1 <= rho), and t = mu - m
// (see the k_proj comment for the method).  `start` < 0 is a first guess of
// t (e.g. from the previous iteration); any value is valid.  Every thread of
// the workgroup must call it.
template <int T, int NV>
__device__ __forceinline__ void l1_threshold_regs(const double (&vr)[NV], int64_t p, double rho, double start,
                                                  double* lds, double& m, double& t, bool& inside,
                                                  int& passes) {
    const int tid = threadIdx.x;
    __shared__ __align__(16) double slots[4 * (T / WAVE)];   // the passes' reductions (one barrier each)
    double Sm_s[1] = {0.0}, Sm_m[1] = {0.0};
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const double a = fabs(vr[e]);
        Sm_s[0] += a;
        Sm_m[0] = fmax(Sm_m[0], a);
    }
    block_reduce<T, 1, 1>(Sm_s, Sm_m, lds);
    const double Sv = Sm_s[0];
    m = Sm_m[0];
    inside = Sv <= rho;
    t = 0.0;
    passes = 0;
    if (inside || !(rho > 0.0) || !isfinite(Sv)) return;
    t = start < 0.0 ? fmax(-rho, start) : fmax(-rho, (Sv - rho) / (double)p - m);
    if (!(t < 0.0)) t = -rho;
    int cprev = -1;
    bool first = true;
    for (;;) {
        int c = 0;
        double sum = 0.0;
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int j = 2 * ((e / 2) * T + tid) + (e & 1);
            const double b = fabs(vr[e]) - m;
            const bool a = j < p && b > t;
            c += wave_count(a);
            if (a) sum += b;
        }
        block_sum2_alt<T>(c, sum, slots, passes);
        ++passes;
        if (c == cprev || passes >= (1 << 20)) break;
        cprev = c;
        const double tn = (sum - rho) / (double)c;
        t = first ? tn : fmax(t, tn);
        first = false;
    }
}

// h = sgn(v) max((|v| - m) - t, 0); inside: h = v; rho == 0: h = 0.
__device__ __forceinline__ double l1_hval(double vj, double m, double t, bool inside, double rho) {
    if (inside) return vj;
    if (!(rho > 0.0)) return 0.0;
    const double a = fmax((fabs(vj) - m) - t, 0.0);
    return vj < 0.0 ? -a : a;
}

// Scalars with which the iteration's projection formed h, read once by the
// kernels that use h after it.
struct ProjH {
    double alpha, m, t;
    int mode;
};
__device__ __forceinline__ ProjH proj_h_params(const GPState* st) {
    return ProjH{st->alpha, st->pm, st->pt, st->hmode};
}
// h_j of the iteration's projection, recomputed from x_j and g_j with the
// projection's own operations (so the same bits): v = x - alpha g as one
// fused multiply-add, then the shifted soft threshold.
__device__ __forceinline__ double proj_h(double xj, double gj, const ProjH& P) {
    const double v = fma(-P.alpha, gj, xj);
    if (P.mode == 1) return v;
    if (P.mode == 2) return 0.0;
    const double a = fmax((fabs(v) - P.m) - P.t, 0.0);
    return v < 0.0 ? -a : a;
}

template <int VPT, int T>
__global__ __launch_bounds__(T) void k_proj(GPState* __restrict__ st, int mode, int64_t p,
                                                 double* __restrict__ x, const double* __restrict__ g,
                                                 double* __restrict__ dout,
                                                 const double* __restrict__ upart, int GU,
                                                 double* __restrict__ vbuf, float* __restrict__ d32) {
    constexpr int NV = VPT > 0 ? VPT : 1;
    constexpr int PU = 8;   // streamed form (VPT = 0): elements per thread per round
    static_assert(NV <= 32, "the sign mask of the shifted slots has 32 bits");
    __shared__ double lds[3 * (T / WAVE)];
    __shared__ __align__(16) double slots[4 * (T / WAVE)];   // the threshold passes' reductions
    __shared__ double sh_alpha, sh_mu;
    __shared__ GPState S;
    const int tid = threadIdx.x;
    // x and g are requested first so that their latency overlaps the state
    // load and the steplength rule; v = x - alpha g is formed once alpha is
    // known (up to 32 slots per thread and 16384 per workgroup, where x and
    // g fit in the registers that T threads leave per lane; beyond that both
    // are read after the steplength rule).  g is not read in the modes that
    // have none.
    constexpr bool PREF = VPT > 0 && VPT <= 32 && VPT * T <= 16384;
    // x kept per thread in LDS (slot e of thread tid at e*T + tid) for the
    // float copy of d at the end, instead of a second read from memory
    __shared__ double xkeep[PREF ? NV * T : 1];
    const bool use_g = mode == PM_ITER || mode == PM_ALPHA0;
    const bool keep_x = PREF && d32 != nullptr;
    double vr[NV], gr[PREF ? NV : 1];
    // the partial dots of the last update, requested with x and g
    double dots[2] = {0.0, 0.0};
    if (mode == PM_ITER)
        for (int i = tid; i < GU; i += T) { dots[0] += upart[4 * i]; dots[1] += upart[4 * i + 1]; }
    if (PREF) {
#pragma unroll
        for (int e = 0; e < NV; e += 2) {
            const int j = 2 * ((e / 2) * T + tid);   // p < 2^31: 32-bit offsets
            if (NV > 1 && j + 1 < p) {
                const double2 x2 = *reinterpret_cast<const double2*>(x + j);
                double2 g2 = make_double2(0.0, 0.0);
                if (use_g) g2 = *reinterpret_cast<const double2*>(g + j);
                vr[e] = x2.x;
                vr[e + 1] = x2.y;
                gr[PREF ? e : 0] = g2.x;
                gr[PREF ? e + 1 : 0] = g2.y;
            } else {
                vr[e] = j < p ? x[j] : 0.0;
                gr[PREF ? e : 0] = (j < p && use_g) ? g[j] : 0.0;
                if (NV > 1) { vr[e + 1] = 0.0; gr[PREF ? e + 1 : 0] = 0.0; }
            }
        }
        if (keep_x) {
#pragma unroll
            for (int e = 0; e < NV; ++e) xkeep[PREF ? e * T + tid : 0] = vr[e];
        }
    }
    state_load(S, st);
    __syncthreads();
    if (S.done || S.stop_req) {
        if (tid == 0) st->live = 0;
        return;
    }

    // -- steplength (Algorithm 2) from the partial dots of the last update --
    if (mode == PM_ITER) {
        const int need_ss = S.ss_pending;
        double none[1] = {0.0};
        if (need_ss) block_reduce<T, 2, 1>(dots, none, lds);
        if (tid == 0) {
            iter_rule(S, need_ss != 0, dots[0], dots[1]);
            sh_alpha = S.alpha;
            sh_mu = S.mu;
        }
    } else if (tid == 0) {
        commit_pending(&S);
        sh_alpha = mode == PM_ALPHA0 ? 1.0 : 0.0;
        sh_mu = 0.0;
    }
    __syncthreads();
    const double alpha = sh_alpha;
    const double mu_prev = sh_mu;
    const double rho = S.prm.rho;

    // -- v = x - alpha g ---------------------------------------------------
    // Register slot e holds element j = 2*((e/2)*T + tid) + (e&1): each
    // thread owns pairs of neighbours, read with 16-byte loads.
    double Sm_s[1] = {0.0}, Sm_m[1] = {0.0};
    if (VPT > 0) {
        if (PREF) {
            if (use_g) {
#pragma unroll
                for (int e = 0; e < NV; ++e) vr[e] = fma(-alpha, gr[PREF ? e : 0], vr[e]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < NV; e += 2) {
                const int j = 2 * ((e / 2) * T + tid);
                if (NV > 1 && j + 1 < p) {
                    const double2 x2 = *reinterpret_cast<const double2*>(x + j);
                    double2 g2 = make_double2(0.0, 0.0);
                    if (use_g) g2 = *reinterpret_cast<const double2*>(g + j);
                    vr[e] = fma(-alpha, g2.x, x2.x);
                    vr[e + 1] = fma(-alpha, g2.y, x2.y);
                } else {
                    vr[e] = j < p ? (use_g ? fma(-alpha, g[j], x[j]) : x[j]) : 0.0;
                    if (NV > 1) vr[e + 1] = 0.0;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const double a = fabs(vr[e]);
            Sm_s[0] += a;
            Sm_m[0] = fmax(Sm_m[0], a);
        }
    } else {
        // PU loads per operand in flight per thread (one L2 round trip per
        // PU elements instead of per element), summed in the same j order
        int64_t j = tid;
        for (; j + (PU - 1) * T < p; j += PU * T) {
            double xv[PU], gv[PU];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                xv[u] = x[j + u * T];
                gv[u] = use_g ? g[j + u * T] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const double vj = use_g ? fma(-alpha, gv[u], xv[u]) : xv[u];
                vbuf[j + u * T] = vj;
                Sm_s[0] += fabs(vj);
                Sm_m[0] = fmax(Sm_m[0], fabs(vj));
            }
        }
        for (; j < p; j += T) {
            const double vj = use_g ? fma(-alpha, g[j], x[j]) : x[j];
            vbuf[j] = vj;
            Sm_s[0] += fabs(vj);
            Sm_m[0] = fmax(Sm_m[0], fabs(vj));
        }
    }
    block_reduce<T, 1, 1>(Sm_s, Sm_m, lds);
    const double Sv = Sm_s[0], m = Sm_m[0];
    if (!isfinite(Sv)) {
        if (tid == 0) { S.status = ST_NONFINITE; S.done = 1; S.live = 0; }
        __syncthreads();
        state_store(st, S);
        return;
    }

    // -- threshold --------------------------------------------------------
    const bool inside = Sv <= rho;
    double t = 0.0;     // mu - m
    int passes = 0;
    int nact = inside ? -1 : 0;   // the final pass's active set
    // Outside the ball the register slots are turned into b = |v| - m once
    // (-inf for slots past p) with the signs kept in `neg`, so that a pass is
    // one compare and one add per slot.
    const bool shifted = VPT > 0 && !inside && rho > 0.0;
    uint32_t neg = 0;
    if (shifted) {
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int j = 2 * ((e / 2) * T + tid) + (e & 1);
            if (vr[e] < 0.0) neg |= 1u << e;
            vr[e] = j < p ? fabs(vr[e]) - m : -INFINITY;
        }
    }
    if (!inside && rho > 0.0) {
        // start: the previous threshold if it lies below m, else the lower
        // bound max(-rho, mean bound); any start with t < 0 is valid
        const double tw = mu_prev - m;
        t = (mode == PM_ITER && mu_prev > 0.0 && tw < 0.0) ? fmax(-rho, tw)
                                                           : fmax(-rho, (Sv - rho) / (double)p - m);
        if (!(t < 0.0)) t = -rho;
        int cprev = -1;
        bool first = true;
        for (;;) {
            int c = 0;
            double sum = 0.0;
            if (VPT > 0) {
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const bool a = vr[e] > t;
                    c += wave_count(a);
                    if (a) sum += vr[e];
                }
            } else {
                int64_t j = tid;
                for (; j + (PU - 1) * T < p; j += PU * T) {
                    double b[PU];
#pragma unroll
                    for (int u = 0; u < PU; ++u) b[u] = fabs(vbuf[j + u * T]) - m;
#pragma unroll
                    for (int u = 0; u < PU; ++u)
                        if (b[u] > t) { ++c; sum += b[u]; }
                }
                for (; j < p; j += T) {
                    const double b = fabs(vbuf[j]) - m;
                    if (b > t) { ++c; sum += b; }
                }
                c = wave_sum(c);
            }
            block_sum2_alt<T>(c, sum, slots, passes);
            ++passes;
            // c >= 1: the largest entry has b = 0 > t.  After the first
            // (Newton) step t is kept monotone, so the sets are nested in
            // floating point too and the loop ends within p + 1 passes.
            if (c == cprev || passes >= (1 << 20)) {
                nact = c;
                break;
            }
            cprev = c;
            const double tn = (sum - rho) / (double)c;
            t = first ? tn : fmax(t, tn);
            first = false;
        }
    }
    // h_i = sgn(v_i) max(b_i - t, 0);  rho == 0 gives h = 0.  hval takes a
    // value of v (the vbuf path), hreg register slot e (v itself, or b with
    // its sign in `neg` once shifted)
    auto hval = [&](double vj) -> double {
        if (inside) return vj;
        if (!(rho > 0.0)) return 0.0;
        const double a = fmax((fabs(vj) - m) - t, 0.0);
        return vj < 0.0 ? -a : a;
    };
    auto hreg = [&](int e) -> double {
        if (!shifted) return hval(vr[e]);
        const double a = fmax(vr[e] - t, 0.0);
        return ((neg >> e) & 1u) ? -a : a;
    };

    // -- outputs ------------------------------------------------------------
    if (mode == PM_ITER) {
        // h = P(x - alpha g).  Only the float copy of d = h - x is stored (for
        // the products); the kernels that need h itself recompute it from x,
        // g and (alpha, m, t, mode) with the same operations (proj_h).
        if (keep_x && shifted) {
            // the usual case, without branches: x from LDS, h from the
            // shifted slots (slots past p hold b = -inf and give h = 0)
            auto hs = [&](int e) {
                const double a = fmax(vr[e] - t, 0.0);
                return ((neg >> e) & 1u) ? -a : a;
            };
            if ((int64_t)NV * T == p) {
#pragma unroll
                for (int e = 0; e < NV; e += 2) {
                    const int j = 2 * ((e / 2) * T + tid);
                    const double h0 = hs(e), h1 = hs(e + 1);
                    const double x0 = xkeep[PREF ? e * T + tid : 0], x1 = xkeep[PREF ? (e + 1) * T + tid : 0];
                    *reinterpret_cast<float2*>(d32 + j) = make_float2((float)(h0 - x0), (float)(h1 - x1));
                }
            } else {
#pragma unroll
                for (int e = 0; e < NV; e += 2) {
                    const int j = 2 * ((e / 2) * T + tid);
                    const double h0 = hs(e), h1 = hs(e + 1);
                    const double x0 = xkeep[PREF ? e * T + tid : 0], x1 = xkeep[PREF ? (e + 1) * T + tid : 0];
                    if (j + 1 < p) *reinterpret_cast<float2*>(d32 + j) = make_float2((float)(h0 - x0), (float)(h1 - x1));
                    else if (j < p) d32[j] = (float)(h0 - x0);
                }
            }
        } else if (d32 && VPT > 0) {
#pragma unroll
            for (int e = 0; e < NV; e += 2) {
                const int j = 2 * ((e / 2) * T + tid);
                if (NV > 1 && j + 1 < p) {
                    const double h0 = hreg(e), h1 = hreg(e + 1);
                    if (keep_x) {
                        const double x0 = xkeep[PREF ? e * T + tid : 0], x1 = xkeep[PREF ? (e + 1) * T + tid : 0];
                        *reinterpret_cast<float2*>(d32 + j) = make_float2((float)(h0 - x0), (float)(h1 - x1));
                    } else {
                        const double2 x2 = *reinterpret_cast<const double2*>(x + j);
                        *reinterpret_cast<float2*>(d32 + j) = make_float2((float)(h0 - x2.x), (float)(h1 - x2.y));
                    }
                } else if (j < p) {
                    d32[j] = (float)(hreg(e) - (keep_x ? xkeep[PREF ? e * T + tid : 0] : x[j]));
                }
            }
        } else if (d32) {
            int64_t j = tid;
            for (; j + (PU - 1) * T < p; j += PU * T) {
                double vv[PU], xv[PU];
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    vv[u] = vbuf[j + u * T];
                    xv[u] = x[j + u * T];
                }
#pragma unroll
                for (int u = 0; u < PU; ++u) d32[j + u * T] = (float)(hval(vv[u]) - xv[u]);
            }
            for (; j < p; j += T) d32[j] = (float)(hval(vbuf[j]) - x[j]);
        }
        if (tid == 0) {
            S.mu = inside ? 0.0 : m + t;
            S.pm = m;
            S.pt = t;
            S.hmode = inside ? 1 : (rho > 0.0 ? 0 : 2);
            S.michelot_iters = passes;
            S.michelot_total += passes;
            S.nactive = nact;
            S.live = 1;
        }
    } else if (mode == PM_ALPHA0) {
        double hmax = 0.0;
        if (VPT > 0) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int j = 2 * ((e / 2) * T + tid) + (e & 1);
                if (j < p) hmax = fmax(hmax, fabs(hreg(e)));
            }
        } else {
            int64_t j = tid;
            for (; j + (PU - 1) * T < p; j += PU * T) {
                double vv[PU];
#pragma unroll
                for (int u = 0; u < PU; ++u) vv[u] = vbuf[j + u * T];
#pragma unroll
                for (int u = 0; u < PU; ++u) hmax = fmax(hmax, fabs(hval(vv[u])));
            }
            for (; j < p; j += T) hmax = fmax(hmax, fabs(hval(vbuf[j])));
        }
        hmax = block_max<T>(hmax, lds);
        if (tid == 0) {
            // alpha_0 = max{alpha_min, min{1/||P(x0 - grad f(x0))||_inf, alpha_max}}
            S.alpha = hmax > 0.0 ? clamp_alpha(1.0 / hmax, S.prm) : S.prm.amax;
            S.live = 1;
        }
    } else {   // PM_INIT_X0 (in place on x) and PM_PLAIN (into dout)
        double* out = mode == PM_INIT_X0 ? x : dout;
        if (VPT > 0) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int j = 2 * ((e / 2) * T + tid) + (e & 1);
                if (j < p) out[j] = hreg(e);
            }
        } else {
            int64_t j = tid;
            for (; j + (PU - 1) * T < p; j += PU * T) {
                double vv[PU];
#pragma unroll
                for (int u = 0; u < PU; ++u) vv[u] = vbuf[j + u * T];
#pragma unroll
                for (int u = 0; u < PU; ++u) out[j + u * T] = hval(vv[u]);
            }
            for (; j < p; j += T) out[j] = hval(vbuf[j]);
        }
        if (tid == 0) {
            S.mu = inside ? 0.0 : (rho > 0.0 ? m + t : m);
            S.michelot_iters = passes;
            if (mode == PM_INIT_X0) S.projected = inside ? 0 : 1;
            S.live = 1;
        }
    }
    __syncthreads();
    state_store(st, S);
}

// ---------------------------------------------------------------------------
// k_fused: t = K v (- y), and partial w = K^T t, reading K once.
//
// Workgroup b owns rows [b*R, min(n, (b+1)*R)).  Thread `tid` owns the column
// chunks col = (c*T + tid)*VEC, c < CPT, so each row is read with coalesced
// 16-byte loads.  For a block of RB rows: per-thread partial dots, a wave
// butterfly, one LDS exchange -> every thread holds t_i for the block, then
// w_j += K_ij t_i on the registers that still hold the row block.  The next
// row block is loaded before the current one is reduced.
// ---------------------------------------------------------------------------
template <typename TK, typename ACC, int T, int CPT, int RB>
struct FusedBlock {
    static constexpr int VEC = KTraits<TK>::VEC;
    static constexpr int NW = T / WAVE;

    // BRANCHLESS (rows aligned to the chunk size and p a multiple of VEC, so
    // every chunk lies wholly before p or wholly past it): each chunk is one
    // load from a valid address with no branch around it (rows past r1 read
    // row r1 - 1, chunks past p read column 0), so the compiler's waits can
    // count the loads still in flight and the next row blocks keep loading
    // while one is reduced.  A chunk past p multiplies the zeros of the
    // direction, so the dots are the same, and the partial w it forms there
    // lies in columns past p, which no reader uses; rows past r1 are skipped
    // by process.  Otherwise chunks outside the block read as zero.
    template <bool ALIGNED, bool BRANCHLESS = false>
    __device__ __forceinline__ static void load(KVec<TK> (&buf)[RB][CPT], const TK* K, int64_t ldk,
                                                int64_t p, int64_t row0, int64_t r1) {
        if constexpr (BRANCHLESS) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int64_t row = row0 + r < r1 ? row0 + r : r1 - 1;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int64_t col = ((int64_t)c * T + threadIdx.x) * VEC;
                    const TK* src = K + row * ldk + (col < p ? col : 0);
                    if constexpr (std::is_same<TK, bf16x4_t>::value)
                        buf[r][c].raw = *reinterpret_cast<const uint2*>(src);
                    else
                        buf[r][c].raw = *reinterpret_cast<const uint4*>(src);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int64_t row = row0 + r;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int64_t col = ((int64_t)c * T + threadIdx.x) * VEC;
                    if (row < r1 && col < p) load_kvec<TK, ALIGNED>(K + row * ldk, col, p, buf[r][c]);
                    else buf[r][c].clear();
                }
            }
        }
    }

    // Reduce one block of RB rows and fold it into w.  Row values live in
    // LDS (stage: y_i and r_i staged in, t_i buffered out) so that no global
    // access sits on the per-row path: vmcnt is in order, and waiting for a
    // scalar load would also wait for the prefetched rows of K.
    // With `wl` (LDS, thread-private slots) the partial w is accumulated there
    // instead of in registers.
    __device__ __forceinline__ static void process(const KVec<TK> (&buf)[RB][CPT], const ACC (&dv)[CPT][VEC],
                                                   ACC (&w)[CPT][VEC], double (*red)[RB][NW], int bi,
                                                   int64_t row0, int64_t r1, int kl, const double* s_y,
                                                   const double* s_r, double* s_t, double& tt, double& tr,
                                                   ACC* wl = nullptr) {
        const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
        double part[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            ACC s = 0;
#pragma unroll
            for (int c = 0; c < CPT; ++c)
#pragma unroll
                for (int e = 0; e < VEC; ++e) s += (ACC)buf[r][c].get(e) * dv[c][e];
            part[r] = wave_sum((double)s);
        }
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < RB; ++r) red[bi][r][wid] = part[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int64_t row = row0 + r;
            if (row < r1) {
                double t = 0.0;
#pragma unroll
                for (int i = 0; i < NW; ++i) t += red[bi][r][i];
                t -= s_y[kl + r];
                if (threadIdx.x == 0) {
                    s_t[kl + r] = t;
                    tt += t * t;
                    tr += t * s_r[kl + r];
                }
                const ACC ta = (ACC)t;
                if (wl) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        ACC* wp = wl + ((int64_t)c * T + threadIdx.x) * VEC;
#pragma unroll
                        for (int e = 0; e < VEC; ++e) wp[e] += (ACC)buf[r][c].get(e) * ta;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < CPT; ++c)
#pragma unroll
                        for (int e = 0; e < VEC; ++e) w[c][e] += (ACC)buf[r][c].get(e) * ta;
                }
            }
        }
    }
};

// The vector multiplied is u = v - vsub (vsub may be NULL): in an iteration
// v = h and vsub = x give the direction d; on a refresh v = x.  With g given,
// workgroup b also returns g'd, d'd and ||d||_inf over its column slice.
// Body of the fused pass for workgroup `wg` of `ngroups` (the slab index and
// slab count of one problem); `wrow` and `sp` are this workgroup's partial
// vector and partial dots.
template <typename TK, typename ACC, int T, int CPT, int RB, int NB, bool ALIGNED, bool WL = false>
__device__ __forceinline__ void fused_body(const TK* __restrict__ K, int64_t n, int64_t p, int64_t ldk,
                                           int64_t rows_per_wg, const double* __restrict__ v,
                                           const double* __restrict__ vsub, const double* __restrict__ g,
                                           const double* __restrict__ ysub, const double* __restrict__ rvec,
                                           double* __restrict__ tout, ACC* __restrict__ wrow, int64_t ldw,
                                           double* __restrict__ sp, int interleave, int64_t wg, int64_t ngroups,
                                           const float* __restrict__ v32 = nullptr, ProjH ph = ProjH{}) {
    using FB = FusedBlock<TK, ACC, T, CPT, RB>;
    // h_j: given (v), or, with v NULL in an iteration, recomputed from
    // x = vsub and g as the projection formed it
    auto hval_at = [&](int64_t j) -> double { return v ? v[j] : proj_h(vsub[j], g[j], ph); };
    constexpr int VEC = FB::VEC;
    constexpr int NW = FB::NW;
    constexpr int FCH = 256;    // rows staged per chunk (a multiple of RB)
    static_assert(FCH % RB == 0, "row blocks must not straddle a chunk");
    __shared__ double red[2][RB][NW];
    __shared__ double lds3[3 * NW];
    __shared__ double s_y[FCH], s_r[FCH], s_t[FCH];
    const int tid = threadIdx.x;

    // Row blocks of this workgroup: a contiguous slab [r0, r1), or, with
    // `interleave`, blocks b, b + G, b + 2G, ... so that at any moment the
    // whole grid streams one compact window of K.
    const int64_t r0 = wg * rows_per_wg;
    const int64_t first = interleave ? wg * RB : r0;
    const int64_t step = interleave ? ngroups * RB : RB;
    const int64_t lim = interleave ? n : (r0 + rows_per_wg < n ? r0 + rows_per_wg : n);
    // NB register buffers of RB rows each: NB - 1 row blocks are in flight
    // while one is reduced
    KVec<TK> A[RB][CPT], B[RB][CPT], C[NB > 2 ? RB : 1][CPT];
    // start streaming K before the vector loads so their latencies overlap
    if (first < lim) FB::template load<ALIGNED>(A, K, ldk, p, first, lim);
    if (NB > 2 && first + step < lim) FB::template load<ALIGNED>(B, K, ldk, p, first + step, lim);

    ACC dv[CPT][VEC], w[CPT][VEC];
    // WL: the partial w lives in LDS (thread-private float4/double2 slots),
    // which frees its registers for wide workgroups
    __shared__ __attribute__((aligned(16))) ACC wls[WL ? CPT * T * VEC : 1];
    ACC* wl = WL ? wls : nullptr;
    // the multiplied vector: its float copy when the caller has one (ACC is
    // float then, so the products are the same), else v - vsub in double
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t col = ((int64_t)c * T + tid) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int64_t j = col + e;
            if (v32) dv[c][e] = j < p ? (ACC)v32[j] : (ACC)0;
            else dv[c][e] = j < p ? (ACC)(vsub ? hval_at(j) - vsub[j] : v[j]) : (ACC)0;
            w[c][e] = 0;
            if constexpr (WL) wls[((int64_t)c * T + tid) * VEC + e] = 0;
        }
    }
    double tt = 0.0, tr = 0.0;
    int bi = 0;
    // Staging of y_i, r_i and the outputs t_i, CH rows at a time.  `kl` is
    // the index of a row block within the current chunk; a chunk boundary
    // flushes t and loads the next chunk (one wait per CH rows).
    int64_t chunk_first = -1;   // first row block (in units of step) of the staged chunk
    int kl = 0;
    auto stage = [&](int64_t blk) {
        // rows of row-block index bb: first + bb*step + r, r < RB
        __syncthreads();
        if (chunk_first >= 0) {
            for (int i = tid; i < FCH; i += T) {
                const int64_t bb = chunk_first + i / RB;
                const int64_t row = first + bb * step + i % RB;
                if (row < lim && i < kl) tout[row] = s_t[i];
            }
        }
        chunk_first = blk;
        for (int i = tid; i < FCH; i += T) {
            const int64_t bb = blk + i / RB;
            const int64_t row = first + bb * step + i % RB;
            const bool ok = row < lim;
            s_y[i] = (ok && ysub) ? ysub[row] : 0.0;
            s_r[i] = (ok && rvec) ? rvec[row] : 0.0;
        }
        kl = 0;
        __syncthreads();
    };
    int64_t blk = 0;    // row-block counter
    auto run = [&](const KVec<TK> (&buf)[RB][CPT], int64_t row) {
        if (kl == FCH || chunk_first < 0) stage(blk);
        FB::process(buf, dv, w, red, bi, row, lim, kl, s_y, s_r, s_t, tt, tr, wl);
        bi ^= 1;
        kl += RB;
        ++blk;
    };
    // the next row block's loads.  Branch-free for 2-byte K with three
    // buffers, issued even past the last block (rows clamped, never reduced):
    // the bf16 pass is limited by how long each row waits, and measured
    // 35.4 -> 33.8 us per launch at 4096 x 16384; the FP32 pass streams at
    // the memory system's pace either way, and the extra loads past the last
    // block cost it about 1 %, so it keeps its guarded loads
    constexpr bool BRANCHLESS = ALIGNED && NB > 2 && sizeof(TK) == 2;
    auto prefetch = [&](KVec<TK> (&buf)[RB][CPT], int64_t row) {
        if constexpr (BRANCHLESS)
            FB::template load<true, true>(buf, K, ldk, p, row < lim ? row : lim - 1, lim);
        else if (row < lim)
            FB::template load<ALIGNED>(buf, K, ldk, p, row, lim);
    };
    if constexpr (NB > 2) {
        for (int64_t row = first; row < lim; row += 3 * step) {
            prefetch(C, row + 2 * step);
            run(A, row);
            if (row + step >= lim) break;
            prefetch(A, row + 3 * step);
            run(B, row + step);
            if (row + 2 * step >= lim) break;
            prefetch(B, row + 4 * step);
            run(C, row + 2 * step);
        }
    } else {
        for (int64_t row = first; row < lim; row += 2 * step) {
            prefetch(B, row + step);
            run(A, row);
            if (row + step >= lim) break;
            prefetch(A, row + 2 * step);
            run(B, row + step);
        }
    }
    // flush the last chunk of outputs
    __syncthreads();
    if (chunk_first >= 0) {
        for (int i = tid; i < FCH; i += T) {
            const int64_t bb = chunk_first + i / RB;
            const int64_t row = first + bb * step + i % RB;
            if (row < lim && i < kl) tout[row] = s_t[i];
        }
    }
    // direction dots over this workgroup's column slice
    double dsum[2] = {0.0, 0.0}, dmx[1] = {0.0};
    if (g) {
        const int64_t cs = (p + ngroups - 1) / ngroups;
        const int64_t c0 = wg * cs;
        const int64_t c1 = c0 + cs < p ? c0 + cs : p;
        for (int64_t j = c0 + tid; j < c1; j += T) {
            const double dj = hval_at(j) - vsub[j];
            dsum[0] += g[j] * dj;
            dsum[1] += dj * dj;
            dmx[0] = fmax(dmx[0], fabs(dj));
        }
        block_reduce<T, 2, 1>(dsum, dmx, lds3);
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t col = ((int64_t)c * T + tid) * VEC;
        if (col < ldw) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) wrow[col + e] = WL ? wls[((int64_t)c * T + tid) * VEC + e] : w[c][e];
        }
    }
    if (tid == 0) {
        sp[0] = tt;
        sp[1] = tr;
        sp[2] = dsum[0];
        sp[3] = dsum[1];
        sp[4] = dmx[0];
    }
}

template <typename TK, typename ACC, int T, int CPT, int RB, int NB, bool ALIGNED, bool WL = false>
__global__ __launch_bounds__(T) void k_fused(const GPState* __restrict__ st, const TK* __restrict__ K,
                                                int64_t n, int64_t p, int64_t ldk, int64_t rows_per_wg,
                                                const double* __restrict__ v, const double* __restrict__ vsub,
                                                const double* __restrict__ g, const double* __restrict__ ysub,
                                                const double* __restrict__ rvec, double* __restrict__ tout,
                                                ACC* __restrict__ wpart, int64_t ldw,
                                                double* __restrict__ spart, int interleave,
                                                const float* __restrict__ v32) {
    if (!st->live) return;
    const ProjH ph = v ? ProjH{} : proj_h_params(st);
    fused_body<TK, ACC, T, CPT, RB, NB, ALIGNED, WL>(K, n, p, ldk, rows_per_wg, v, vsub, g, ysub, rvec, tout,
                                                 wpart + (int64_t)blockIdx.x * ldw, ldw,
                                                 spart + (int64_t)SPART * blockIdx.x, interleave,
                                                 (int64_t)blockIdx.x, (int64_t)gridDim.x, v32, ph);
}

// ---------------------------------------------------------------------------
// The update kernel's progress report to the host (when the solve has a
// host-mapped word): updates completed, bit 31 once a stop is requested.  A
// system-scope store, so the host sees it without a synchronisation; the word
// only paces how far ahead the host enqueues, the state stays authoritative.
__device__ __forceinline__ void post_progress(const GPParams& P, int32_t k, bool stop) {
    if (P.progress)
        __hip_atomic_store(P.progress, (uint32_t)k | (stop ? 0x80000000u : 0u), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}

// k_update: line search and vector updates (see file comment).
// Grid: nbp workgroups over columns (UPD_COLS each), then workgroups over rows.
// ---------------------------------------------------------------------------
template <typename ACC>
__global__ __launch_bounds__(UPD_T) void k_update(GPState* __restrict__ st, int mode,
                                                  const double* __restrict__ spart, int GF,
                                                  const ACC* __restrict__ wpart, int64_t ldw, int64_t p,
                                                  int64_t n, int nbp, double* __restrict__ x,
                                                  double* __restrict__ g,
                                                  double* __restrict__ r, const double* __restrict__ tq,
                                                  double* __restrict__ upart) {
    constexpr int T = UPD_T;
    constexpr int VU = 16 / (int)sizeof(ACC);   // columns per vector load
    constexpr int CQ = UPD_COLS / VU;           // column vectors per workgroup
    constexpr int NG = T / CQ;                  // partial groups
    using V16 = typename std::conditional<VU == 4, float4, double2>::type;
    __shared__ double red[NG][UPD_COLS];
    __shared__ GPState S;
    __shared__ double sh5[5];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const bool colwg = (int)blockIdx.x < nbp;
    // Everything this workgroup reads that does not depend on the state is
    // requested before the state, so the latencies overlap: the first eight
    // partial vectors per thread, this thread's x, h, g (or r, q) entries,
    // and the fused kernel's partial dots.
    const int cq = tid % CQ, grp = tid / CQ;
    const int64_t c0 = (int64_t)blockIdx.x * UPD_COLS;
    const ACC* src = wpart + c0 + cq * VU;
    V16 w8[8];
    const bool pre8 = colwg && grp + 7 * NG < GF;
    if (pre8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) w8[u] = *reinterpret_cast<const V16*>(src + (int64_t)(grp + u * NG) * ldw);
    }
    const int64_t jc = c0 + tid;
    const bool colj = colwg && tid < UPD_COLS && jc < p;
    double xj = 0.0, gj = 0.0;
    if (colj) {
        xj = x[jc];
        if (mode == UM_ITER) gj = g[jc];
    }
    const int64_t ir = (int64_t)(blockIdx.x - nbp) * UPD_ROWS + tid;
    const bool rowi = !colwg && ir < n;
    double ri = 0.0, qi = 0.0;
    if (rowi) {
        qi = tq[ir];
        if (mode == UM_ITER) ri = r[ir];
    }
    // (q'q, r'q, g'd, d'd, ||d||_inf) or (r'r) from the fused kernel's
    // partials, fixed order
    if (tid < WAVE) {
        double a = 0.0, b = 0.0, c = 0.0, e = 0.0, mx = 0.0;
        for (int i = lane; i < GF; i += WAVE) {
            const double* sp = spart + (int64_t)SPART * i;
            a += sp[0]; b += sp[1]; c += sp[2]; e += sp[3]; mx = fmax(mx, sp[4]);
        }
        a = wave_sum(a);
        b = wave_sum(b);
        c = wave_sum(c);
        e = wave_sum(e);
        mx = wave_max(mx);
        if (lane == 0) { sh5[0] = a; sh5[1] = b; sh5[2] = c; sh5[3] = e; sh5[4] = mx; }
    }
    state_load(S, st);
    __syncthreads();
    if (!S.live) return;
    const double qq = sh5[0], rq = sh5[1], gd = sh5[2], dd = sh5[3], dmax = sh5[4];
    if (mode == UM_ITER && (dmax == 0.0 || !(gd < 0.0))) {
        // h == x, or no descent left at working precision: stationary
        if (blockIdx.x == 0 && tid == 0) {
            st->gd = gd;
            st->dd = dd;
            st->dmax = dmax;
            st->status = ST_STATIONARY;
            st->stop_req = 1;
            post_progress(S.prm, S.k, true);
        }
        return;
    }

    double lam = 1.0;
    int nb = 0;
    bool fail = false;
    if (mode == UM_ITER) {
        // Armijo with memory M: f(x + lam d) <= f_max + beta lam g'd, where
        // f(x + lam d) - f = lam (2 r'q + lam q'q) exactly for this f.
        const GPParams& P = S.prm;
        const double f = S.f;
        double fmax = f;
        const int nh = S.nhist < P.M ? S.nhist : P.M;
        for (int i = 0; i < nh; ++i) fmax = fmax > S.fhist[(S.hpos - i + MAX_M) % MAX_M]
                                              ? fmax : S.fhist[(S.hpos - i + MAX_M) % MAX_M];
        for (;;) {
            const double inc = lam * (2.0 * rq + lam * qq);
            if (inc <= (fmax - f) + P.beta * lam * gd) break;
            if (++nb > P.bt_cap) { fail = true; break; }
            lam *= P.theta;
        }
        if (fail) {
            if (blockIdx.x == 0 && tid == 0) {
                st->status = ST_BACKTRACK;
                st->stop_req = 1;
                post_progress(S.prm, S.k, true);
            }
            return;
        }
    }

    if (colwg) {
        // ---- columns: w_j = sum of the fused kernel's partials ----
        double acc[VU];
#pragma unroll
        for (int e = 0; e < VU; ++e) acc[e] = 0.0;
        int gi = grp;
        // eight partial vectors in flight per thread, summed in index order
        // (the first eight were requested at the start)
        if (pre8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const ACC* pw = reinterpret_cast<const ACC*>(&w8[u]);
#pragma unroll
                for (int e = 0; e < VU; ++e) acc[e] += (double)pw[e];
            }
            gi += 8 * NG;
        }
        for (; gi + 7 * NG < GF; gi += 8 * NG) {
            V16 wn[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) wn[u] = *reinterpret_cast<const V16*>(src + (int64_t)(gi + u * NG) * ldw);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const ACC* pw = reinterpret_cast<const ACC*>(&wn[u]);
#pragma unroll
                for (int e = 0; e < VU; ++e) acc[e] += (double)pw[e];
            }
        }
        for (; gi < GF; gi += NG) {
            const V16 w1 = *reinterpret_cast<const V16*>(src + (int64_t)gi * ldw);
            const ACC* pw = reinterpret_cast<const ACC*>(&w1);
#pragma unroll
            for (int e = 0; e < VU; ++e) acc[e] += (double)pw[e];
        }
#pragma unroll
        for (int e = 0; e < VU; ++e) red[grp][cq * VU + e] = acc[e];
        __syncthreads();
        double dw = 0.0, ww = 0.0;
        if (tid < WAVE) {
            double w = 0.0;
            if (tid < UPD_COLS) {
#pragma unroll
                for (int i = 0; i < NG; ++i) w += red[i][tid];
            }
            if (colj) {
                if (mode == UM_ITER) {
                    // h_j as the projection formed it
                    const double dj = proj_h(xj, gj, ProjH{S.alpha, S.pm, S.pt, S.hmode}) - xj;
                    x[jc] = xj + lam * dj;
                    g[jc] = gj + 2.0 * lam * w;
                    dw = dj * w;
                    ww = w * w;
                } else {
                    g[jc] = 2.0 * w;
                }
            }
            dw = wave_sum(dw);
            ww = wave_sum(ww);
            if (tid == 0) {
                upart[4 * blockIdx.x] = dw;
                upart[4 * blockIdx.x + 1] = ww;
                upart[4 * blockIdx.x + 2] = 0.0;
                upart[4 * blockIdx.x + 3] = 0.0;
            }
        }
    } else {
        // ---- rows: r += lam q, or r = K x - y on a refresh ----
        if (rowi) r[ir] = mode == UM_ITER ? ri + lam * qi : qi;
        if (tid == 0) {
            upart[4 * blockIdx.x] = 0.0;
            upart[4 * blockIdx.x + 1] = 0.0;
            upart[4 * blockIdx.x + 2] = 0.0;
            upart[4 * blockIdx.x + 3] = 0.0;
        }
    }

    if (blockIdx.x == 0 && tid == 0) {
        const GPParams& P = S.prm;
        if (mode == UM_ITER) {
            const double f = S.f;
            const double fn = f + lam * (2.0 * rq + lam * qq);
            st->lam = lam;
            st->gd = gd;
            st->dd = dd;
            st->dmax = dmax;
            st->nb = nb;
            st->backtracks = S.backtracks + nb;
            st->f_new = fn;
            st->k_new = S.k + 1;
            st->pending = 1;
            st->ss_pending = 1;
            const double rel = (f - fn) / f;
            st->rel = rel;
            bool stop = true;
            if (!isfinite(fn)) st->status = ST_NONFINITE;
            else if (P.f_target >= 0.0 && fn <= P.f_target) st->status = ST_TARGET;
            else if (P.tol > 0.0 && rel < P.tol) st->status = ST_OK_TOL;
            else if (S.k + 1 >= P.max_iter) st->status = ST_MAX_ITER;
            else stop = false;
            if (stop) st->stop_req = 1;
            if (P.trace) {
                double* rec = P.trace + (int64_t)(S.k % P.trace_cap) * TRACE_FIELDS;
                rec[0] = S.k + 1;
                rec[1] = fn;
                rec[2] = S.alpha;
                rec[3] = lam;
                rec[4] = nb;
                rec[5] = S.tau;
                rec[6] = S.k == 0 ? -1 : S.rule;
                rec[7] = S.mu;
                rec[8] = S.nactive;
                rec[9] = S.michelot_iters;
            }
            post_progress(P, S.k + 1, stop);
        } else {
            st->f_new = qq;              // sum of t_i^2 = ||K x - y||^2
            if (!S.pending) st->k_new = S.k;
            st->pending = 1;
            if (!isfinite(qq)) { st->status = ST_NONFINITE; st->stop_req = 1; }
        }
    }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void init_state(GPState* st, const GPParams& prm) {
    GPState s = {};
    s.prm = prm;
    s.f_target0 = prm.f_target;
    s.live = 1;
    s.tau = prm.tau1;
    s.alpha = prm.amax;
    s.status = ST_MAX_ITER;
    s.hpos = 0;
    s.nhist = 0;
    *st = s;
}

static __global__ void k_init_state(GPState* st, GPParams prm) { init_state(st, prm); }

// Start of a solve in one launch: the state, y and x0 widened to double
// (x = 0 without x0).
template <typename TV>
__global__ void k_setup(GPState* __restrict__ st, GPParams prm, const TV* __restrict__ y, double* __restrict__ y64,
                        int64_t n, const TV* __restrict__ x0, double* __restrict__ x, int64_t p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y64[i] = (double)y[i];
    if (i < p) x[i] = x0 ? (double)x0[i] : 0.0;
    if (i == 0) init_state(st, prm);
}

template <typename TV>
__global__ void k_to_f64(const TV* __restrict__ in, double* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in ? (double)in[i] : 0.0;
}

template <typename TV>
__global__ void k_from_f64(const double* __restrict__ in, TV* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (TV)in[i];
}

// End of a solve: commit the last update, ||x||_1 and ||g||_inf for the
// result, and x narrowed into the caller's output.  Launched after every
// chunk of iterations; it does nothing unless the solve has stopped (done or
// stop_req) or `force` is set (the iteration budget is spent), so the host's
// status poll after a chunk already finds the finished result.
template <typename TV>
__global__ __launch_bounds__(PROJ_T) void k_finish(GPState* __restrict__ st, const double* __restrict__ x,
                                                   const double* __restrict__ g, int64_t p, int force,
                                                   TV* __restrict__ x_out) {
    __shared__ double lds[PROJ_T / WAVE];
    __shared__ int go;
    if (threadIdx.x == 0) go = force || st->done || st->stop_req;
    __syncthreads();
    if (!go) return;
    double l1 = 0.0, gm = 0.0;
    for (int64_t j = threadIdx.x; j < p; j += PROJ_T) {
        const double xj = x[j];
        l1 += fabs(xj);
        gm = fmax(gm, fabs(g[j]));
        x_out[j] = (TV)xj;
    }
    l1 = block_sum<PROJ_T>(l1, lds);
    gm = block_max<PROJ_T>(gm, lds);
    if (threadIdx.x == 0) {
        commit_pending(st);
        st->l1 = l1;
        st->gmax = gm;
        st->done = 1;
        st->live = 0;
    }
}

}  // namespace gpl1
