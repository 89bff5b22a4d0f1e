// Kernels of one GPSS iteration on MI355X.  Per iteration three launches:
//
//   k_proj   (1 workgroup)  : steplength rule (Algorithm 2), v = x - alpha g,
//                             threshold search for P_Omega, d = P(v) - x and
//                             the dots g'd, d'd (Algorithm 1, projection and
//                             direction).
//   k_fused  (G workgroups) : one read of K serves both products: every
//                             workgroup owns a slab of rows, forms q_i = K_i d
//                             for its rows and, while that slab of K is still
//                             in registers, adds K_i^T q_i into a private
//                             p-vector.  Output: q (n) and G partial vectors of
//                             w = K^T K d.
//   k_update (many)         : closed-form Armijo backtracking from
//                             (f, g'd, r'q, q'q), x += lam d, r += lam q,
//                             g += 2 lam w (the new gradient 2 K^T r), and the
//                             dots d'w, w'w that Algorithm 2 needs next.
//
// With f quadratic, f(x + lam d) = f + 2 lam r'q + lam^2 q'q with r = Kx - y
// and q = Kd, so every backtracking trial is a scalar formula, and
// grad f(x + lam d) = g + 2 lam K^T K d, so the new gradient needs K^T q only.
#pragma once

#include "gp_device.hpp"
#include "gp_state.hpp"

namespace gpl1 {

enum ProjMode : int32_t { PM_ITER = 0, PM_INIT_X0 = 1, PM_ALPHA0 = 2, PM_PLAIN = 3 };
enum UpdMode : int32_t { UM_ITER = 0, UM_REFRESH = 1 };

constexpr int PROJ_T = 1024;
constexpr int UPD_T = 256;
constexpr int UPD_COLS = 64;   // columns per p-part workgroup of k_update
constexpr int UPD_ROWS = 256;  // rows per n-part workgroup of k_update

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

// ---------------------------------------------------------------------------
// k_proj: projection onto the l1 ball by a parallel threshold search.
//
// With b_i = |v_i| - m (m = max|v|), the threshold t = mu - m solves
// sum max(b_i - t, 0) = rho.  Starting from a lower bound t_0 <= t
// (t_0 = max(-rho, (sum b - rho)/p): mu >= m - rho because the largest entry
// of P(v) is at most rho, and mu >= the mean-based bound because all entries
// could be active), each pass takes A = {b_i > t} and sets
// t = (sum_A b - rho)/|A|.  The sets shrink monotonically and the pass whose
// set is unchanged gives the exact threshold (Michelot's method).  Every pass
// is one workgroup reduction of (count, sum) over values held in registers.
// VPT = values per thread kept in registers; VPT = 0 streams them from vbuf.
// ---------------------------------------------------------------------------
template <int VPT>
__global__ __launch_bounds__(PROJ_T) void k_proj(GPState* __restrict__ st, int mode, int64_t p,
                                                 double* __restrict__ x, const double* __restrict__ g,
                                                 double* __restrict__ dout,
                                                 const double* __restrict__ upart, int GU,
                                                 double* __restrict__ vbuf) {
    constexpr int T = PROJ_T;
    constexpr int NV = VPT > 0 ? VPT : 1;
    __shared__ double lds[2 * (T / WAVE)];
    __shared__ double sh_alpha;
    const int tid = threadIdx.x;
    if (st->done || st->stop_req) {
        if (tid == 0) st->live = 0;
        return;
    }

    // -- steplength (Algorithm 2) from the partial dots of the last update --
    if (mode == PM_ITER) {
        const int need_ss = st->ss_pending;          // uniform read before any write
        double dw = 0.0, ww = 0.0;
        if (need_ss) {
            for (int i = tid; i < GU; i += T) { dw += upart[4 * i]; ww += upart[4 * i + 1]; }
            dw = block_sum<T>(dw, lds);
            ww = block_sum<T>(ww, lds);
        }
        if (tid == 0) {
            commit_pending(st);
            if (need_ss) {
                // s = lam d, z = 2 lam w (w = K^T K d): s's = lam^2 d'd,
                // s'z = 2 lam^2 d'w, z'z = 4 lam^2 w'w (equation (5))
                const double l2 = st->lam * st->lam;
                ss_update(st, st->k, l2 * st->dd, 2.0 * l2 * dw, 4.0 * l2 * ww);
                st->ss_pending = 0;
            }
            sh_alpha = st->alpha;
        }
    } else if (tid == 0) {
        commit_pending(st);
        sh_alpha = mode == PM_ALPHA0 ? 1.0 : 0.0;
    }
    __syncthreads();
    const double alpha = sh_alpha;
    const double rho = st->prm.rho;

    // -- v = x - alpha g ---------------------------------------------------
    double v[NV];
    double S = 0.0, m = 0.0;
    auto vload = [&](int64_t j) -> double {
        if (mode == PM_ITER || mode == PM_ALPHA0) return x[j] - alpha * g[j];
        return x[j];
    };
    if (VPT > 0) {
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int64_t j = (int64_t)e * T + tid;
            v[e] = j < p ? vload(j) : 0.0;
            S += fabs(v[e]);
            m = fmax(m, fabs(v[e]));
        }
    } else {
        for (int64_t j = tid; j < p; j += T) {
            const double vj = vload(j);
            vbuf[j] = vj;
            S += fabs(vj);
            m = fmax(m, fabs(vj));
        }
    }
    S = block_sum<T>(S, lds);
    m = block_max<T>(m, lds);
    if (!isfinite(S)) {
        if (tid == 0) { st->status = ST_NONFINITE; st->done = 1; st->live = 0; }
        return;
    }

    // -- threshold --------------------------------------------------------
    const bool inside = S <= rho;
    double t = 0.0;     // mu - m
    int passes = 0;
    if (!inside && rho > 0.0) {
        double sb = 0.0;
        if (VPT > 0) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int64_t j = (int64_t)e * T + tid;
                if (j < p) sb += fabs(v[e]) - m;
            }
        } else {
            for (int64_t j = tid; j < p; j += T) sb += fabs(vbuf[j]) - m;
        }
        sb = block_sum<T>(sb, lds);
        t = fmax(-rho, (sb - rho) / (double)p);
        int cprev = -1;
        for (;;) {
            int c = 0;
            double s = 0.0;
            if (VPT > 0) {
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const int64_t j = (int64_t)e * T + tid;
                    const double b = fabs(v[e]) - m;
                    if (j < p && b > t) { ++c; s += b; }
                }
            } else {
                for (int64_t j = tid; j < p; j += T) {
                    const double b = fabs(vbuf[j]) - m;
                    if (b > t) { ++c; s += b; }
                }
            }
            block_sum2<T>(c, s, lds);
            ++passes;
            // c >= 1: the largest entry has b = 0 > t.  Keeping t monotone
            // makes the sets nested in floating point too, so c never grows
            // and the loop ends after at most p + 1 passes.
            if (c == cprev || passes >= (1 << 20)) break;
            cprev = c;
            t = fmax(t, (s - rho) / (double)c);
        }
    }
    // h_i = sgn(v_i) max(b_i - t, 0);  rho == 0 gives h = 0
    auto hval = [&](double vj) -> double {
        if (inside) return vj;
        if (!(rho > 0.0)) return 0.0;
        const double a = fmax((fabs(vj) - m) - t, 0.0);
        return vj < 0.0 ? -a : a;
    };

    // -- outputs ------------------------------------------------------------
    if (mode == PM_ITER) {
        double gd = 0.0, dd = 0.0, dmax = 0.0;
        auto emit = [&](int64_t j, double vj) {
            const double dj = hval(vj) - x[j];
            dout[j] = dj;
            gd += g[j] * dj;
            dd += dj * dj;
            dmax = fmax(dmax, fabs(dj));
        };
        if (VPT > 0) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int64_t j = (int64_t)e * T + tid;
                if (j < p) emit(j, v[e]);
            }
        } else {
            for (int64_t j = tid; j < p; j += T) emit(j, vbuf[j]);
        }
        gd = block_sum<T>(gd, lds);
        dd = block_sum<T>(dd, lds);
        dmax = block_max<T>(dmax, lds);
        if (tid == 0) {
            st->gd = gd;
            st->dd = dd;
            st->dmax = dmax;
            st->mu = inside ? 0.0 : m + t;
            st->michelot_iters = passes;
            // h == x, or no descent left at working precision: stationary
            if (dmax == 0.0 || !(gd < 0.0)) { st->status = ST_STATIONARY; st->done = 1; st->live = 0; }
            else st->live = 1;
        }
    } else if (mode == PM_ALPHA0) {
        double hmax = 0.0;
        if (VPT > 0) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int64_t j = (int64_t)e * T + tid;
                if (j < p) hmax = fmax(hmax, fabs(hval(v[e])));
            }
        } else {
            for (int64_t j = tid; j < p; j += T) hmax = fmax(hmax, fabs(hval(vbuf[j])));
        }
        hmax = block_max<T>(hmax, lds);
        if (tid == 0) {
            // alpha_0 = max{alpha_min, min{1/||P(x0 - grad f(x0))||_inf, alpha_max}}
            st->alpha = hmax > 0.0 ? clamp_alpha(1.0 / hmax, st->prm) : st->prm.amax;
            st->live = 1;
        }
    } else {   // PM_INIT_X0 (in place on x) and PM_PLAIN (into dout)
        double* out = mode == PM_INIT_X0 ? x : dout;
        if (VPT > 0) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int64_t j = (int64_t)e * T + tid;
                if (j < p) out[j] = hval(v[e]);
            }
        } else {
            for (int64_t j = tid; j < p; j += T) out[j] = hval(vbuf[j]);
        }
        if (tid == 0) {
            st->mu = inside ? 0.0 : (rho > 0.0 ? m + t : m);
            st->michelot_iters = passes;
            if (mode == PM_INIT_X0) st->projected = inside ? 0 : 1;
            st->live = 1;
        }
    }
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

    template <bool ALIGNED>
    __device__ __forceinline__ static void load(KVec<TK> (&buf)[RB][CPT], const TK* K, int64_t ldk,
                                                int64_t p, int64_t row0, int64_t r1) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int64_t row = row0 + r;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int64_t col = ((int64_t)c * T + threadIdx.x) * VEC;
                if (row < r1 && col < p) load_kvec<TK, ALIGNED>(K + row * ldk, col, p, buf[r][c]);
                else buf[r][c].raw = make_uint4(0u, 0u, 0u, 0u);
            }
        }
    }

    __device__ __forceinline__ static void process(const KVec<TK> (&buf)[RB][CPT], const ACC (&dv)[CPT][VEC],
                                                   ACC (&w)[CPT][VEC], double (*red)[RB][NW], int bi,
                                                   int64_t row0, int64_t r1, const double* ysub,
                                                   const double* rvec, double* tout, double& tt,
                                                   double& tr) {
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
                if (ysub) t -= ysub[row];
                if (threadIdx.x == 0) {
                    tout[row] = t;
                    tt += t * t;
                    if (rvec) tr += t * rvec[row];
                }
                const ACC ta = (ACC)t;
#pragma unroll
                for (int c = 0; c < CPT; ++c)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) w[c][e] += (ACC)buf[r][c].get(e) * ta;
            }
        }
    }
};

template <typename TK, typename ACC, int T, int CPT, int RB, bool ALIGNED>
__global__ __launch_bounds__(T) void k_fused(const GPState* __restrict__ st, const TK* __restrict__ K,
                                                int64_t n, int64_t p, int64_t ldk, int64_t rows_per_wg,
                                                const double* __restrict__ v, const double* __restrict__ ysub,
                                                const double* __restrict__ rvec, double* __restrict__ tout,
                                                ACC* __restrict__ wpart, int64_t ldw,
                                                double* __restrict__ spart) {
    using FB = FusedBlock<TK, ACC, T, CPT, RB>;
    constexpr int VEC = FB::VEC;
    constexpr int NW = FB::NW;
    __shared__ double red[2][RB][NW];
    if (!st->live) return;
    const int tid = threadIdx.x;

    ACC dv[CPT][VEC], w[CPT][VEC];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t col = ((int64_t)c * T + tid) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            dv[c][e] = col + e < p ? (ACC)v[col + e] : (ACC)0;
            w[c][e] = 0;
        }
    }
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r1 = r0 + rows_per_wg < n ? r0 + rows_per_wg : n;
    double tt = 0.0, tr = 0.0;
    KVec<TK> A[RB][CPT], B[RB][CPT];
    int bi = 0;
    if (r0 < r1) FB::template load<ALIGNED>(A, K, ldk, p, r0, r1);
    for (int64_t row = r0; row < r1; row += 2 * RB) {
        if (row + RB < r1) FB::template load<ALIGNED>(B, K, ldk, p, row + RB, r1);
        FB::process(A, dv, w, red, bi, row, r1, ysub, rvec, tout, tt, tr);
        bi ^= 1;
        if (row + RB >= r1) break;
        if (row + 2 * RB < r1) FB::template load<ALIGNED>(A, K, ldk, p, row + 2 * RB, r1);
        FB::process(B, dv, w, red, bi, row + RB, r1, ysub, rvec, tout, tt, tr);
        bi ^= 1;
    }
    ACC* wrow = wpart + (int64_t)blockIdx.x * ldw;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t col = ((int64_t)c * T + tid) * VEC;
        if (col < ldw) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) wrow[col + e] = w[c][e];
        }
    }
    if (tid == 0) {
        spart[2 * blockIdx.x] = tt;
        spart[2 * blockIdx.x + 1] = tr;
    }
}

// ---------------------------------------------------------------------------
// k_update: line search and vector updates (see file comment).
// Grid: nbp workgroups over columns (UPD_COLS each), then workgroups over rows.
// ---------------------------------------------------------------------------
template <typename ACC>
__global__ __launch_bounds__(UPD_T) void k_update(GPState* __restrict__ st, int mode,
                                                  const double* __restrict__ spart, int GF,
                                                  const ACC* __restrict__ wpart, int64_t ldw, int64_t p,
                                                  int64_t n, int nbp, double* __restrict__ x,
                                                  double* __restrict__ g, const double* __restrict__ d,
                                                  double* __restrict__ r, const double* __restrict__ tq,
                                                  double* __restrict__ upart) {
    constexpr int T = UPD_T;
    constexpr int VU = 16 / (int)sizeof(ACC);   // columns per vector load
    constexpr int CQ = UPD_COLS / VU;           // column vectors per workgroup
    constexpr int NG = T / CQ;                  // partial groups
    __shared__ double red[NG][UPD_COLS];
    __shared__ double sh[4];
    if (!st->live) return;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);

    // (q'q, r'q) or (r'r) from the fused kernel's partials, fixed order
    if (tid < WAVE) {
        double a = 0.0, b = 0.0;
        for (int i = lane; i < GF; i += WAVE) { a += spart[2 * i]; b += spart[2 * i + 1]; }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) { sh[0] = a; sh[1] = b; }
    }
    __syncthreads();
    const double qq = sh[0], rq = sh[1];

    double lam = 1.0;
    int nb = 0;
    bool fail = false;
    if (mode == UM_ITER) {
        // Armijo with memory M: f(x + lam d) <= f_max + beta lam g'd, where
        // f(x + lam d) - f = lam (2 r'q + lam q'q) exactly for this f.
        const GPParams& P = st->prm;
        const double f = st->f;
        double fmax = f;
        const int nh = st->nhist < P.M ? st->nhist : P.M;
        for (int i = 0; i < nh; ++i) fmax = fmax > st->fhist[(st->hpos - i + MAX_M) % MAX_M]
                                              ? fmax : st->fhist[(st->hpos - i + MAX_M) % MAX_M];
        const double gd = st->gd;
        for (;;) {
            const double inc = lam * (2.0 * rq + lam * qq);
            if (inc <= (fmax - f) + P.beta * lam * gd) break;
            if (++nb > P.bt_cap) { fail = true; break; }
            lam *= P.theta;
        }
        if (fail) {
            if (blockIdx.x == 0 && tid == 0) { st->status = ST_BACKTRACK; st->stop_req = 1; }
            return;
        }
    }

    if ((int)blockIdx.x < nbp) {
        // ---- columns: w_j = sum of the fused kernel's partials ----
        const int cq = tid % CQ, grp = tid / CQ;
        const int64_t c0 = (int64_t)blockIdx.x * UPD_COLS;
        double acc[VU];
#pragma unroll
        for (int e = 0; e < VU; ++e) acc[e] = 0.0;
        for (int gi = grp; gi < GF; gi += NG) {
            const ACC* src = wpart + (int64_t)gi * ldw + c0 + cq * VU;
            if constexpr (VU == 4) {
                const float4 w4 = *reinterpret_cast<const float4*>(src);
                acc[0] += w4.x; acc[1] += w4.y; acc[2] += w4.z; acc[3] += w4.w;
            } else {
                const double2 w2 = *reinterpret_cast<const double2*>(src);
                acc[0] += w2.x; acc[1] += w2.y;
            }
        }
#pragma unroll
        for (int e = 0; e < VU; ++e) red[grp][cq * VU + e] = acc[e];
        __syncthreads();
        double dw = 0.0, ww = 0.0;
        if (tid < UPD_COLS) {
            double w = 0.0;
#pragma unroll
            for (int i = 0; i < NG; ++i) w += red[i][tid];
            const int64_t j = c0 + tid;
            if (j < p) {
                if (mode == UM_ITER) {
                    const double dj = d[j];
                    x[j] += lam * dj;
                    g[j] += 2.0 * lam * w;
                    dw = dj * w;
                    ww = w * w;
                } else {
                    g[j] = 2.0 * w;
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
        const int64_t i = (int64_t)(blockIdx.x - nbp) * UPD_ROWS + tid;
        if (i < n) r[i] = mode == UM_ITER ? r[i] + lam * tq[i] : tq[i];
        if (tid == 0) {
            upart[4 * blockIdx.x] = 0.0;
            upart[4 * blockIdx.x + 1] = 0.0;
            upart[4 * blockIdx.x + 2] = 0.0;
            upart[4 * blockIdx.x + 3] = 0.0;
        }
    }

    if (blockIdx.x == 0 && tid == 0) {
        const GPParams& P = st->prm;
        if (mode == UM_ITER) {
            const double f = st->f;
            const double fn = f + lam * (2.0 * rq + lam * qq);
            st->lam = lam;
            st->nb = nb;
            st->backtracks += nb;
            st->f_new = fn;
            st->k_new = st->k + 1;
            st->pending = 1;
            st->ss_pending = 1;
            const double rel = (f - fn) / f;
            st->rel = rel;
            if (!isfinite(fn)) { st->status = ST_NONFINITE; st->stop_req = 1; }
            else if (P.f_target >= 0.0 && fn <= P.f_target) { st->status = ST_TARGET; st->stop_req = 1; }
            else if (P.tol > 0.0 && rel < P.tol) { st->status = ST_OK_TOL; st->stop_req = 1; }
            else if (st->k + 1 >= P.max_iter) { st->status = ST_MAX_ITER; st->stop_req = 1; }
        } else {
            st->f_new = qq;              // sum of t_i^2 = ||K x - y||^2
            if (!st->pending) st->k_new = st->k;
            st->pending = 1;
            if (!isfinite(qq)) { st->status = ST_NONFINITE; st->stop_req = 1; }
        }
    }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_init_state(GPState* st, GPParams prm) {
    GPState s = {};
    s.prm = prm;
    s.live = 1;
    s.tau = prm.tau1;
    s.alpha = prm.amax;
    s.status = ST_MAX_ITER;
    s.hpos = 0;
    s.nhist = 0;
    *st = s;
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

// Commit the last update and compute ||x||_1 and ||g||_inf for the result.
__global__ __launch_bounds__(PROJ_T) void k_finish(GPState* __restrict__ st, const double* __restrict__ x,
                                                   const double* __restrict__ g, int64_t p) {
    __shared__ double lds[PROJ_T / WAVE];
    double l1 = 0.0, gm = 0.0;
    for (int64_t j = threadIdx.x; j < p; j += PROJ_T) {
        l1 += fabs(x[j]);
        gm = fmax(gm, fabs(g[j]));
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
