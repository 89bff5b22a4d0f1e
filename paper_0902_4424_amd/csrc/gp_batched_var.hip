// Batched GPSS over independent problems of different sizes.
//
// All problems advance in lockstep, three launches per sweep:
//   k_bv_fused  : a work list of (problem, slab of rows) items; each item
//                 runs the fused pass of the plain solver (q = K d for its
//                 rows and a partial p-vector of K^T q from the same read of
//                 K), so the HBM stream is spread over thousands of
//                 workgroups whatever the mix of sizes;
//   k_bv_update : one workgroup per problem: closed-form Armijo backtracking
//                 (Algorithm 1), x, r, g updates, the dots of equation (5)
//                 and the steplength rule of Algorithm 2;
//   k_bv_proj   : one workgroup per problem: projection onto the l1 ball
//                 (threshold search in registers), direction d = P(v) - x
//                 and its dots, stationarity.
// A problem that has stopped is skipped by all three (its own flag).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gp_internal.hpp"
#include "gp_kernels.hpp"
#include "gp_l1.h"
#include "gp_verify.hpp"

using namespace gpl1;

namespace gpl1 {

constexpr int BV_T = 1024;   // per-problem workgroups
constexpr int BV_FT = 256;   // fused-pass workgroups
constexpr int BV_ROWS = 64;  // rows per work item unless tuned (32: the same, 256: 30 % slower)
constexpr int BV_RB = 1;     // rows per block in the fused pass (2 measured the same, 4 slower)
constexpr int BV_NB = 2;     // register buffers (3 measured the same)

struct VarInst {
    const void* K;
    const void* yin;
    const void* x0in;
    void* xout;
    int64_t n, p, ldk;
    double rho;
    double *x, *g, *d, *r, *q, *y;   // FP64 per-problem vectors
    int64_t item0, nitems, ldw;      // work items (slabs) and partial stride
    float* wpart;                    // nitems x ldw partial vectors (float accumulation)
    double* wpart64;                 // same for FP64 K
    double* spart;                   // nitems x SPART partial dots
    double ftarget;                  // this problem's f_target
    int32_t aligned;                 // rows 16-byte aligned
    int32_t aligned8;                // rows 8-byte aligned (bf16: read as 4-element chunks)
    int32_t item_rows;               // rows of K per work item
    int32_t waves;                   // 1: the wave-per-row fused pass (narrow float or bf16 problems)
    int64_t nparts;                  // partial vectors and dots: nitems, or BV_NW per item with `waves`
};

struct VarItem { int32_t inst, slab; };

template <int NV>
__global__ __launch_bounds__(BV_T) void k_bv_init(const VarInst* __restrict__ I, GPState* __restrict__ st,
                                                  GPParams prm, int f64v) {
    __shared__ double lds[3 * (BV_T / WAVE)];
    const int b = blockIdx.x, tid = threadIdx.x;
    const VarInst D = I[b];
    for (int64_t i = tid; i < D.n; i += BV_T)
        D.y[i] = f64v ? ((const double*)D.yin)[i] : (double)((const float*)D.yin)[i];
    double vr[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * BV_T + tid) + (e & 1);
        double v = 0.0;
        if (D.x0in && j < D.p) v = f64v ? ((const double*)D.x0in)[j] : (double)((const float*)D.x0in)[j];
        vr[e] = v;
    }
    double m, t;
    bool inside;
    int passes;
    l1_threshold_regs<BV_T, NV>(vr, D.p, D.rho, -1.0, lds, m, t, inside, passes);
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * BV_T + tid) + (e & 1);
        if (j < D.p) D.x[j] = l1_hval(vr[e], m, t, inside, D.rho);
    }
    if (tid == 0) {
        // written in place (a local copy of the state would go to scratch)
        GPState* sp = st + b;
        __builtin_memset(sp, 0, sizeof(GPState));
        sp->prm = prm;
        sp->prm.rho = D.rho;
        sp->prm.f_target = D.ftarget;
        sp->f_target0 = D.ftarget;
        sp->tau = prm.tau1;
        sp->alpha = prm.amax;
        sp->status = ST_MAX_ITER;
        sp->projected = inside ? 0 : 1;
        sp->live = 1;
    }
}

// fused pass on one work item; v = x (refresh, with y subtracted) or d
template <typename TK, typename ACC, int CPT>
__device__ __forceinline__ void bv_item(const VarItem& it, const VarInst& D, int refresh) {
    ACC* wp;
    if constexpr (sizeof(ACC) == 8) wp = (ACC*)D.wpart64;
    else wp = (ACC*)D.wpart;
    ACC* wrow = wp + (int64_t)it.slab * D.ldw;
    double* sp = D.spart + (int64_t)SPART * it.slab;
    const double* v = refresh ? D.x : D.d;
    const double* ys = refresh ? D.y : nullptr;
    const double* rs = refresh ? nullptr : D.r;
    if (D.aligned) {
        fused_body<TK, ACC, BV_FT, CPT, BV_RB, BV_NB, true>((const TK*)D.K, D.n, D.p, D.ldk, D.item_rows, v, nullptr,
                                                             nullptr, ys, rs, D.q, wrow, D.ldw, sp, 0, it.slab,
                                                             D.nitems);
        return;
    }
    if constexpr (std::is_same<TK, bf16_t>::value) {
        // 8-byte aligned bf16 rows (odd n with p = 4n, say): four-element
        // chunks keep every wave's loads contiguous; twice the chunks cover
        // the same columns
        if (D.aligned8) {
            fused_body<bf16x4_t, ACC, BV_FT, 2 * CPT, BV_RB, BV_NB, true>(
                (const bf16x4_t*)D.K, D.n, D.p, D.ldk, D.item_rows, v, nullptr, nullptr, ys, rs, D.q, wrow, D.ldw, sp,
                0, it.slab, D.nitems);
            return;
        }
    }
    fused_body<TK, ACC, BV_FT, CPT, BV_RB, BV_NB, false>((const TK*)D.K, D.n, D.p, D.ldk, D.item_rows, v, nullptr,
                                                          nullptr, ys, rs, D.q, wrow, D.ldw, sp, 0, it.slab,
                                                          D.nitems);
}

// Work item of a narrow problem, whose rows fit CW chunks of one wave (at most
// BV_NARROW columns): each wave takes every fourth row of the item and
// reduces its row dots within the wave, so no row waits for a barrier (in the
// workgroup-wide pass a row of a few KB spends most of its time in the
// cross-wave reduction), and each wave leaves a partial vector and partial
// dots of its own (partial row 4 * slab + wave), which the update kernel adds
// with the others in index order.  Same outputs otherwise as bv_item: t_i =
// K_i v (minus y_i on a refresh) for the item's rows.
constexpr int BV_NW = BV_FT / WAVE;
constexpr int BV_NARROW = 1024;   // widest p of the wave-per-row pass
template <typename TK, int CW, bool ALIGNED>
__device__ __forceinline__ void bv_item_waves(const VarItem& it, const VarInst& D, int refresh) {
    constexpr int VEC = KTraits<TK>::VEC;
    static_assert(CW * WAVE * VEC <= BV_NARROW, "narrow items only");
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t p = D.p, ldk = D.ldk;
    const TK* K = (const TK*)D.K;
    const double* v = refresh ? D.x : D.d;
    const int64_t r0 = (int64_t)it.slab * D.item_rows;
    const int64_t r1 = r0 + D.item_rows < D.n ? r0 + D.item_rows : D.n;
    float dv[CW][VEC], w[CW][VEC];
#pragma unroll
    for (int c = 0; c < CW; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int64_t j = ((int64_t)c * WAVE + lane) * VEC + e;
            dv[c][e] = j < p ? (float)v[j] : 0.0f;
            w[c][e] = 0.0f;
        }
    // rows past the item reload its last row (issued unconditionally so the
    // waits count exactly, never used); y_i (subtracted on a refresh) or r_i
    // (for t'r in an iteration) comes with each row
    auto rowc = [&](int64_t r) { return r < r1 ? r : r1 - 1; };
    const double* yv = refresh ? D.y : D.r;
    auto load = [&](KVec<TK> (&buf)[CW], double& yr, int64_t row) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int64_t col = ((int64_t)c * WAVE + lane) * VEC;
            if (col < p) load_kvec<TK, ALIGNED>(K + row * ldk, col, p, buf[c]);
            else buf[c].clear();
        }
        yr = yv[row];
    };
    double tt = 0.0, tr = 0.0;
    auto proc = [&](const KVec<TK> (&buf)[CW], double yr, int64_t row) {
        float sdot = 0.0f;
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int e = 0; e < VEC; ++e) sdot += buf[c].get(e) * dv[c][e];
        const double t = wave_sum((double)sdot) - (refresh ? yr : 0.0);
        if (lane == 0) {
            D.q[row] = t;
            tt += t * t;
            if (!refresh) tr += t * yr;
        }
        const float ta = (float)t;
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int e = 0; e < VEC; ++e) w[c][e] += buf[c].get(e) * ta;
    };
    KVec<TK> A[CW], B[CW];
    double ya = 0.0, yb = 0.0;
    int64_t row = r0 + wv;
    if (row < r1) {
        load(A, ya, row);
        for (; row < r1; row += 2 * BV_NW) {
            load(B, yb, rowc(row + BV_NW));
            proc(A, ya, row);
            if (row + BV_NW >= r1) break;
            load(A, ya, rowc(row + 2 * BV_NW));
            proc(B, yb, row + BV_NW);
        }
    }
    const int64_t part = (int64_t)it.slab * BV_NW + wv;
    float* wrow = D.wpart + part * D.ldw;
#pragma unroll
    for (int c = 0; c < CW; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int64_t j = ((int64_t)c * WAVE + lane) * VEC + e;
            if (j < D.ldw) wrow[j] = w[c][e];
        }
    if (lane == 0) {
        double* sp = D.spart + SPART * part;
        sp[0] = tt;
        sp[1] = tr;
        sp[2] = 0.0;
        sp[3] = 0.0;
        sp[4] = 0.0;
    }
}

// the wave-per-row item with the fewest chunks that cover p
template <typename TK>
__device__ __forceinline__ void bv_item_narrow(const VarItem& it, const VarInst& D, int refresh) {
    constexpr int VEC = KTraits<TK>::VEC;
    const int64_t p = D.p;
    if (p <= WAVE * VEC) bv_item_waves<TK, 1, true>(it, D, refresh);
    else if (p <= 2 * WAVE * VEC) bv_item_waves<TK, 2, true>(it, D, refresh);
    else if constexpr (VEC == 4) bv_item_waves<TK, 4, true>(it, D, refresh);
}

// CPT column chunks per thread cover the widest problem of the batch; an
// item of a narrower problem runs with the fewest chunks that cover its own p
// (the chunks past p hold zeros either way, so the sums are the same).  WAVES:
// compiled with the wave-per-row pass for the problems marked `waves` (it
// needs more registers than the one-chunk workgroup pass, so a batch whose
// widest problem needs one chunk uses it only if every problem is narrow)
template <typename TK, typename ACC, int CPT, bool WAVES>
__global__ __launch_bounds__(BV_FT) void k_bv_fused(const VarInst* __restrict__ I, const VarItem* __restrict__ items,
                                                    const GPState* __restrict__ st, int refresh) {
    const VarItem it = items[blockIdx.x];
    if (st[it.inst].done) return;
    const VarInst D = I[it.inst];
    if constexpr (WAVES && sizeof(ACC) == 4) {
        if (D.waves) {
            if constexpr (std::is_same<TK, bf16_t>::value) {
                if (!D.aligned) { bv_item_narrow<bf16x4_t>(it, D, refresh); return; }
            }
            bv_item_narrow<TK>(it, D, refresh);
            return;
        }
    }
    constexpr int64_t COLS1 = (int64_t)BV_FT * KTraits<TK>::VEC;   // columns of one chunk per thread
    if constexpr (CPT >= 4) {
        if (D.p <= COLS1) { bv_item<TK, ACC, 1>(it, D, refresh); return; }
        if (D.p <= 2 * COLS1) { bv_item<TK, ACC, 2>(it, D, refresh); return; }
    } else if constexpr (CPT == 2) {
        if (D.p <= COLS1) { bv_item<TK, ACC, 1>(it, D, refresh); return; }
    }
    bv_item<TK, ACC, CPT>(it, D, refresh);
}

// line search, updates, steplength rule (iteration) or r, g, f (refresh)
template <typename ACC, int T>
__global__ __launch_bounds__(T) void k_bv_update(const VarInst* __restrict__ I, GPState* __restrict__ st_all,
                                                    int refresh) {
    __shared__ double lds[3 * (T / WAVE)];
    __shared__ double sh[4];
    // the problem's state, loaded by all threads at once together with the
    // partial dots (one round trip instead of the scalar thread's dependent
    // reads), updated in LDS and stored back at the end
    __shared__ GPState S;
    const int b = blockIdx.x, tid = threadIdx.x;
    GPState* st = st_all + b;
    state_load(S, st);
    const VarInst D = I[b];
    const ACC* wp;
    if constexpr (sizeof(ACC) == 8) wp = (const ACC*)D.wpart64;
    else wp = (const ACC*)D.wpart;
    // partial dots of the items, fixed order
    double a[2] = {0.0, 0.0}, none[1] = {0.0};
    for (int64_t i = tid; i < D.nparts; i += T) {
        a[0] += D.spart[SPART * i];
        a[1] += D.spart[SPART * i + 1];
    }
    block_reduce<T, 2, 1>(a, none, lds);   // (its barriers also publish S)
    if (S.done) return;
    const double tt = a[0], tr = a[1];
    auto wsum = [&](int64_t j) {
        double s = 0.0;
        for (int64_t c = 0; c < D.nparts; ++c) s += (double)wp[c * D.ldw + j];
        return s;
    };
    if (refresh) {
        for (int64_t i = tid; i < D.n; i += T) D.r[i] = D.q[i];
        for (int64_t j = tid; j < D.p; j += T) D.g[j] = 2.0 * wsum(j);
        if (tid == 0) {
            if (S.k == 0 && S.nhist == 0) { S.hpos = 0; S.nhist = 1; }
            S.fhist[S.hpos] = tt;
            S.f = tt;
            if (!isfinite(tt)) { S.status = ST_NONFINITE; S.done = 1; }
        }
        __syncthreads();
        state_store(st, S);
        return;
    }
    if (tid == 0) {
        const GPParams& P = S.prm;
        const double qq = tt, rq = tr, f = S.f, gd = S.gd;
        double fmax = f;
        const int nh = S.nhist < P.M ? S.nhist : P.M;
        for (int i = 0; i < nh; ++i) fmax = fmax > S.fhist[(S.hpos - i + MAX_M) % MAX_M]
                                              ? fmax : S.fhist[(S.hpos - i + MAX_M) % MAX_M];
        double lam = 1.0;
        int nb = 0;
        bool fail = false;
        for (;;) {
            const double inc = lam * (2.0 * rq + lam * qq);
            if (inc <= (fmax - f) + P.beta * lam * gd) break;
            if (++nb > P.bt_cap) { fail = true; break; }
            lam *= P.theta;
        }
        sh[0] = lam;
        sh[1] = fail ? 1.0 : 0.0;
        if (fail) {
            S.status = ST_BACKTRACK;
            S.done = 1;
        } else {
            const double fn = f + lam * (2.0 * rq + lam * qq);
            S.lam = lam;
            S.nb = nb;
            S.backtracks += nb;
            S.rel = (f - fn) / f;
            S.f = fn;
            S.k += 1;
            S.hpos = (S.hpos + 1) % MAX_M;
            S.fhist[S.hpos] = fn;
            if (S.nhist < MAX_M) S.nhist++;
        }
    }
    __syncthreads();
    if (sh[1] != 0.0) {
        state_store(st, S);
        return;
    }
    const double lam = sh[0];
    for (int64_t i = tid; i < D.n; i += T) D.r[i] += lam * D.q[i];
    double dots[2] = {0.0, 0.0};
    // JU columns per thread at a time; the items' partial values of those
    // columns are requested eight items at a time (clamped indices, values
    // masked) and added in item order, as wsum does
    constexpr int JU = 4, CU = 8;
    for (int64_t j0 = tid; j0 < D.p; j0 += (int64_t)T * JU) {
        double w[JU];
#pragma unroll
        for (int u = 0; u < JU; ++u) w[u] = 0.0;
        for (int64_t c0 = 0; c0 < D.nparts; c0 += CU) {
            ACC v[JU][CU];
#pragma unroll
            for (int u = 0; u < JU; ++u) {
                const int64_t j = j0 + (int64_t)u * T;
                const int64_t jc = j < D.p ? j : 0;
#pragma unroll
                for (int cc = 0; cc < CU; ++cc) {
                    const int64_t c = c0 + cc < D.nparts ? c0 + cc : 0;
                    v[u][cc] = wp[c * D.ldw + jc];
                }
            }
#pragma unroll
            for (int u = 0; u < JU; ++u)
#pragma unroll
                for (int cc = 0; cc < CU; ++cc)
                    if (c0 + cc < D.nparts) w[u] += (double)v[u][cc];
        }
        double dj[JU], xj[JU], gj[JU];
#pragma unroll
        for (int u = 0; u < JU; ++u) {
            const int64_t j = j0 + (int64_t)u * T;
            const int64_t jc = j < D.p ? j : 0;
            dj[u] = D.d[jc];
            xj[u] = D.x[jc];
            gj[u] = D.g[jc];
        }
#pragma unroll
        for (int u = 0; u < JU; ++u) {
            const int64_t j = j0 + (int64_t)u * T;
            if (j < D.p) {
                D.x[j] = xj[u] + lam * dj[u];
                D.g[j] = gj[u] + 2.0 * lam * w[u];
                dots[0] += dj[u] * w[u];
                dots[1] += w[u] * w[u];
            }
        }
    }
    block_reduce<T, 2, 1>(dots, none, lds);
    if (tid == 0) {
        const GPParams& P = S.prm;
        // s = lam d, z = 2 lam w: equation (5), then Algorithm 2
        const double l2 = lam * lam;
        ss_update(&S, S.k, l2 * S.dd, 2.0 * l2 * dots[0], 4.0 * l2 * dots[1]);
        const double fn = S.f;
        int stop = 0;
        if (!isfinite(fn)) { S.status = ST_NONFINITE; stop = 1; }
        else if (P.f_target >= 0.0 && fn <= P.f_target) { S.status = ST_TARGET; stop = 1; }
        else if (P.tol > 0.0 && S.rel < P.tol) { S.status = ST_OK_TOL; stop = 1; }
        else if (S.k >= P.max_iter) { S.status = ST_MAX_ITER; stop = 1; }
        if (stop) S.done = 1;
    }
    __syncthreads();
    state_store(st, S);
}

// projection (alpha0 first on init), direction and its dots
// `reproj`: only the problems that a target check reopened (their step and
// steplength are applied; the direction is missing)
template <int T, int NV>
__global__ __launch_bounds__(T) void k_bv_proj(const VarInst* __restrict__ I, GPState* __restrict__ st_all,
                                                  int init, int reproj) {
    __shared__ double lds[3 * (T / WAVE)];
    __shared__ double sh[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    GPState* st = st_all + b;
    if (st->done || (reproj && !st->reproj)) return;
    const VarInst D = I[b];
    const int64_t p = D.p;
    const double rho = D.rho;
    double vr[NV];
    double m, t;
    bool inside;
    int passes;
    // x and g of this thread's slots, requested together (clamped indices,
    // values masked) and kept for the output loop while they fit the
    // registers (else read again where used)
    constexpr bool KEEP = T <= 256 || NV <= 8;
    double xr[KEEP ? NV : 1], gr[KEEP ? NV : 1];
    auto xval = [&](int e, int j) { return KEEP ? xr[KEEP ? e : 0] : D.x[j]; };
    auto gval = [&](int e, int j) { return KEEP ? gr[KEEP ? e : 0] : D.g[j]; };
    if constexpr (KEEP) {
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int j = 2 * ((e / 2) * T + tid) + (e & 1);
            const int jc = j < p ? j : 0;
            xr[e] = D.x[jc];
            gr[e] = D.g[jc];
        }
    }
    if (tid == 0) { sh[0] = st->alpha; sh[1] = st->mu; }
    __syncthreads();
    double alpha = sh[0];
    if (init) {
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int j = 2 * ((e / 2) * T + tid) + (e & 1);
            vr[e] = j < p ? xval(e, j) - gval(e, j) : 0.0;
        }
        l1_threshold_regs<T, NV>(vr, p, rho, -1.0, lds, m, t, inside, passes);
        double hm = 0.0;
#pragma unroll
        for (int e = 0; e < NV; ++e) hm = fmax(hm, fabs(l1_hval(vr[e], m, t, inside, rho)));
        hm = block_max<T>(hm, lds);
        alpha = hm > 0.0 ? clamp_alpha(1.0 / hm, st->prm) : st->prm.amax;
        __syncthreads();
        if (tid == 0) st->alpha = alpha;
    }
    const double mu_prev = init ? 0.0 : sh[1];
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * T + tid) + (e & 1);
        vr[e] = j < p ? xval(e, j) - alpha * gval(e, j) : 0.0;
    }
    double mloc = 0.0;
#pragma unroll
    for (int e = 0; e < NV; ++e) mloc = fmax(mloc, fabs(vr[e]));
    mloc = block_max<T>(mloc, lds);
    const double start = (mu_prev > 0.0 && mu_prev < mloc) ? mu_prev - mloc : -1.0;
    l1_threshold_regs<T, NV>(vr, p, rho, start, lds, m, t, inside, passes);
    double sums[2] = {0.0, 0.0}, mx[1] = {0.0};
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * T + tid) + (e & 1);
        if (j < p) {
            const double dj = l1_hval(vr[e], m, t, inside, rho) - xval(e, j);
            D.d[j] = dj;
            sums[0] += gval(e, j) * dj;
            sums[1] += dj * dj;
            mx[0] = fmax(mx[0], fabs(dj));
        }
    }
    block_reduce<T, 2, 1>(sums, mx, lds);
    if (tid == 0) {
        st->gd = sums[0];
        st->dd = sums[1];
        st->dmax = mx[0];
        st->mu = inside ? 0.0 : m + t;
        st->michelot_total += passes;
        st->reproj = 0;
        if (!isfinite(m)) { st->status = ST_NONFINITE; st->done = 1; }
        else if (mx[0] == 0.0 || !(sums[0] < 0.0)) { st->status = ST_STATIONARY; st->done = 1; }
    }
}

__global__ __launch_bounds__(BV_T) void k_bv_finish(const VarInst* __restrict__ I, GPState* __restrict__ st_all,
                                                    int f64v) {
    __shared__ double lds[3 * (BV_T / WAVE)];
    const int b = blockIdx.x, tid = threadIdx.x;
    const VarInst D = I[b];
    double s[1] = {0.0}, mx[1] = {0.0};
    for (int64_t j = tid; j < D.p; j += BV_T) {
        s[0] += fabs(D.x[j]);
        mx[0] = fmax(mx[0], fabs(D.g[j]));
        if (f64v) ((double*)D.xout)[j] = D.x[j];
        else ((float*)D.xout)[j] = (float)D.x[j];
    }
    block_reduce<BV_T, 1, 1>(s, mx, lds);
    if (tid == 0) {
        st_all[b].l1 = s[0];
        st_all[b].gmax = mx[0];
    }
}

namespace {
int bv_nv(int64_t p) {
    const int64_t per = (p + BV_T - 1) / BV_T;
    if (per <= 2) return 2;
    if (per <= 4) return 4;
    if (per <= 8) return 8;
    if (per <= 16) return 16;
    return 0;
}
int severity(int s) {
    if (s < 0) return 100 - s;
    if (s == GP_BACKTRACK_LIMIT) return 4;
    if (s == GP_MAX_ITER) return 3;
    return 1;
}
#define GPL1_BV_NV_SWITCH(nv, STMT) \
    switch (nv) {                   \
        case 2: { constexpr int NVc = 2; STMT; } break;   \
        case 4: { constexpr int NVc = 4; STMT; } break;   \
        case 8: { constexpr int NVc = 8; STMT; } break;   \
        case 16: { constexpr int NVc = 16; STMT; } break; \
    }

template <typename TK, typename ACC, bool WAVES>
void launch_bv_fused_w(int cpt, hipStream_t s, unsigned nitems, const VarInst* I, const VarItem* items,
                       const GPState* st, int refresh) {
    switch (cpt) {
        case 1:
            hipLaunchKernelGGL((k_bv_fused<TK, ACC, 1, WAVES>), dim3(nitems), dim3(BV_FT), 0, s, I, items, st, refresh);
            break;
        case 2:
            hipLaunchKernelGGL((k_bv_fused<TK, ACC, 2, WAVES>), dim3(nitems), dim3(BV_FT), 0, s, I, items, st, refresh);
            break;
        case 4:
            hipLaunchKernelGGL((k_bv_fused<TK, ACC, 4, WAVES>), dim3(nitems), dim3(BV_FT), 0, s, I, items, st, refresh);
            break;
    }
}
template <typename TK, typename ACC>
void launch_bv_fused(int cpt, bool waves, hipStream_t s, unsigned nitems, const VarInst* I, const VarItem* items,
                     const GPState* st, int refresh) {
    if (waves) launch_bv_fused_w<TK, ACC, true>(cpt, s, nitems, I, items, st, refresh);
    else launch_bv_fused_w<TK, ACC, false>(cpt, s, nitems, I, items, st, refresh);
}
}  // namespace

// Returns GP_E_UNSUPPORTED (nothing launched) when the sizes do not fit.
int solve_batched_var_lockstep(gp_handle h, gp_dtype kdtype, const gp_instance* inst, int64_t B, double tol,
                               const gp_opts& o, gp_result* res, hipStream_t s) {
    const int esz = kdtype == GP_F64 ? 8 : kdtype == GP_F32 ? 4 : 2;
    const int vec = 16 / esz;
    int64_t maxp = 0;
    for (int64_t b = 0; b < B; ++b) maxp = std::max(maxp, inst[b].p);
    int cpt = 0;
    for (int c : {1, 2, 4})
        if ((int64_t)BV_FT * c * vec >= maxp) { cpt = c; break; }
    const int nv = bv_nv(maxp);
    const int pnv = maxp <= 512 ? 2 : maxp <= 1024 ? 4 : maxp <= 2048 ? 8 : 16;   // slots at 256 threads
    if (cpt == 0 || nv == 0) return GP_E_UNSUPPORTED;
    const bool f64v = kdtype == GP_F64;

    // workspace: states, descriptors, items, vectors, partials
    std::vector<VarInst> hI((size_t)B);
    std::vector<VarItem> hitems;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = off; off += (bytes + 255) / 256 * 256; return o2; };
    const size_t o_st = take(sizeof(GPState) * B);
    const size_t o_I = take(sizeof(VarInst) * B);
    std::vector<size_t> ox((size_t)B), ow((size_t)B), osp((size_t)B);
    int64_t total_items = 0;
    for (int64_t b = 0; b < B; ++b) {
        const gp_instance& S = inst[b];
        VarInst& D = hI[(size_t)b];
        D.K = S.K; D.yin = S.y; D.x0in = S.x0; D.xout = S.x_out;
        D.n = S.n; D.p = S.p; D.ldk = S.ldk; D.rho = S.rho;
        D.ftarget = o.f_targets ? o.f_targets[b] : o.f_target;
        D.item_rows = o.var_item_rows > 0 ? o.var_item_rows : BV_ROWS;
        D.nitems = (S.n + D.item_rows - 1) / D.item_rows;
        D.item0 = total_items;
        D.ldw = (S.p + 63) / 64 * 64;
        // whole chunks for the fused pass: rows aligned to the chunk and p a
        // multiple of it
        D.aligned = (S.ldk % vec == 0) && (S.p % vec == 0) && (((uintptr_t)S.K) % 16 == 0);
        D.aligned8 = (S.ldk * esz % 8 == 0) && (S.p * esz % 8 == 0) && (((uintptr_t)S.K) % 8 == 0);
        // narrow problems of float or bf16 K with 16-byte aligned rows (or
        // 8-byte aligned bf16 rows) run the wave-per-row pass
        D.waves = (o.var_wave_rows >= 0 && !f64v && S.p <= BV_NARROW &&
                   (D.aligned || (kdtype == GP_BF16 && D.aligned8))) ? 1 : 0;
        for (int64_t i = 0; i < D.nitems; ++i) hitems.push_back(VarItem{(int32_t)b, (int32_t)i});
        total_items += D.nitems;
        ox[(size_t)b] = take(8 * (3 * S.p + 3 * S.n));
        D.nparts = D.waves ? BV_NW * D.nitems : D.nitems;
        ow[(size_t)b] = take((size_t)(f64v ? 8 : 4) * D.nparts * D.ldw);
        osp[(size_t)b] = take(8 * SPART * D.nparts);
    }
    const size_t o_items = take(sizeof(VarItem) * hitems.size());
    // target check: a descriptor per problem; candidates, item ranges, row
    // items and partial sums for as many rows as the whole batch has
    const bool check_target = o.f_target >= 0.0 || o.f_targets != nullptr;
    int64_t vrows = 0;
    for (int64_t b = 0; b < B; ++b) vrows += (inst[b].n + VR_ROWS - 1) / VR_ROWS;
    const size_t o_vp = take(check_target ? sizeof(VerProb) * B : 0);
    const size_t o_vc = take(check_target ? sizeof(int32_t) * (2 * B + 1) : 0);
    const size_t o_vi = take(check_target ? sizeof(VerItem) * vrows : 0);
    const size_t o_vs = take(check_target ? sizeof(double) * vrows : 0);
    int rc = ensure_workspace(h, off);
    if (rc) return rc;
    if (o.graph && (rc = graph_stream(h, s, &s))) return rc;
    char* ws = (char*)h->ws;
    for (int64_t b = 0; b < B; ++b) {
        VarInst& D = hI[(size_t)b];
        double* base = (double*)(ws + ox[(size_t)b]);
        D.x = base; D.g = base + D.p; D.d = base + 2 * D.p;
        D.r = base + 3 * D.p; D.q = D.r + D.n; D.y = D.q + D.n;
        D.wpart = f64v ? nullptr : (float*)(ws + ow[(size_t)b]);
        D.wpart64 = f64v ? (double*)(ws + ow[(size_t)b]) : nullptr;
        D.spart = (double*)(ws + osp[(size_t)b]);
    }
    // the kernel with the wave-per-row pass: when some problem uses it, and,
    // while the workgroup pass of the batch's widest problem needs fewer
    // registers than the wave pass (bf16 K with one column chunk per thread,
    // float K with up to two), only if every problem does (the problems keep
    // the workgroup pass otherwise)
    int64_t nwaves = 0;
    for (int64_t b = 0; b < B; ++b) nwaves += hI[(size_t)b].waves;
    const bool kwaves = nwaves > 0 && (cpt >= (kdtype == GP_BF16 ? 2 : 4) || nwaves == B);
    if (!kwaves)
        for (int64_t b = 0; b < B; ++b) {
            hI[(size_t)b].waves = 0;
            hI[(size_t)b].nparts = hI[(size_t)b].nitems;   // (their partials were sized for the waves)
        }
    // longest rows first so that big items start early
    std::stable_sort(hitems.begin(), hitems.end(), [&](const VarItem& a, const VarItem& c) {
        return hI[(size_t)a.inst].p > hI[(size_t)c.inst].p;
    });
    GPState* st = (GPState*)(ws + o_st);
    VarInst* dI = (VarInst*)(ws + o_I);
    VarItem* ditems = (VarItem*)(ws + o_items);
    VerProb* dvp = (VerProb*)(ws + o_vp);
    int32_t* dvc = (int32_t*)(ws + o_vc);
    VerItem* dvi = (VerItem*)(ws + o_vi);
    double* dvs = (double*)(ws + o_vs);
    std::vector<VerProb> hvp;
    if (check_target) {
        hvp.resize((size_t)B);
        for (int64_t b = 0; b < B; ++b) {
            const VarInst& D = hI[(size_t)b];
            hvp[(size_t)b] = VerProb{D.K, D.ldk, D.n, D.p, D.x, D.y, f64v ? 0 : 1, D.aligned};
        }
    }
    hipError_t e = hipMemcpyAsync(dI, hI.data(), sizeof(VarInst) * B, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ditems, hitems.data(), sizeof(VarItem) * hitems.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && check_target)
        e = hipMemcpyAsync(dvp, hvp.data(), sizeof(VerProb) * B, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(h, e, "batched-var set-up");
    const GPParams prm = make_params(o, 0.0, tol);
    const unsigned nit = (unsigned)hitems.size();
    auto fused = [&](int refresh) {
        if (kdtype == GP_F64) launch_bv_fused<double, double>(cpt, false, s, nit, dI, ditems, st, refresh);
        else if (kdtype == GP_F32) launch_bv_fused<float, float>(cpt, kwaves, s, nit, dI, ditems, st, refresh);
        else launch_bv_fused<bf16_t, float>(cpt, kwaves, s, nit, dI, ditems, st, refresh);
    };
    auto update = [&](int refresh) {
        if (f64v) hipLaunchKernelGGL((k_bv_update<double, BV_T>), dim3((unsigned)B), dim3(BV_T), 0, s, dI, st, refresh);
        else hipLaunchKernelGGL((k_bv_update<float, BV_T>), dim3((unsigned)B), dim3(BV_T), 0, s, dI, st, refresh);
    };
    auto proj = [&](int init, int reproj) {
        // 256 threads (several problems per CU) when the largest p fits 16 slots of each
        if (maxp <= 256 * 16) {
            GPL1_BV_NV_SWITCH(pnv, hipLaunchKernelGGL((k_bv_proj<256, NVc>), dim3((unsigned)B), dim3(256), 0, s, dI,
                                                      st, init, reproj));
        } else {
            GPL1_BV_NV_SWITCH(nv, hipLaunchKernelGGL((k_bv_proj<BV_T, NVc>), dim3((unsigned)B), dim3(BV_T), 0, s,
                                                     dI, st, init, reproj));
        }
    };
    GPL1_BV_NV_SWITCH(nv, hipLaunchKernelGGL(k_bv_init<NVc>, dim3((unsigned)B), dim3(BV_T), 0, s, dI, st, prm,
                                             f64v ? 1 : 0));
    fused(1);
    update(1);
    proj(1, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "batched-var init launch");
    // the states are polled into the handle's pinned buffer (plain DMA)
    if ((rc = ensure_pinned(h, sizeof(GPState) * (size_t)B))) return rc;
    GPState* hst = (GPState*)h->pin;
    std::vector<int32_t> hvc;
    std::vector<VerItem> hvi;
    // a problem that is never stopped has done exactly `it` iterations; one
    // reopened by a target check at iteration k needs max_iter - k more
    int it = 0, it_cap = o.max_iter;
    auto read_states = [&]() -> int {
        hipError_t pe = hipMemcpyAsync(hst, st, sizeof(GPState) * B, hipMemcpyDeviceToHost, s);
        if (pe == hipSuccess) pe = hipStreamSynchronize(s);
        return pe == hipSuccess ? 0 : hip_fail(h, pe, "batched-var status poll");
    };
    auto sweep = [&](int i) {
        fused(0);
        update(0);
        if (o.refresh_every > 0 && (i + 1) % o.refresh_every == 0 && i + 1 < it_cap) {
            fused(1);
            update(1);
        }
        proj(0, 0);
    };
    // graph replay: chunks of gch sweeps starting at multiples of gch (the
    // launch sizes never change here, so one capture serves the call)
    const int gch = o.refresh_every > 0 ? o.refresh_every : o.chunk;
    bool captured = false;
    while (it < it_cap) {
        if (o.graph && it % gch == 0 && it + gch < it_cap) {
            if (!captured) {
                const int base = it;
                if ((rc = capture_graph(h, s, &h->gexec_b, [&]() {
                         for (int k = 0; k < gch; ++k) sweep(base + k);
                     })))
                    return rc;
                captured = true;
            }
            e = hipGraphLaunch(h->gexec_b, s);
            if (e != hipSuccess) return hip_fail(h, e, "batched-var graph launch");
            it += gch;
        } else {
            const int end = o.graph ? std::min(it_cap, (it / gch + 1) * gch) : std::min(it_cap, it + o.chunk);
            for (; it < end; ++it) sweep(it);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(h, e, "batched-var iteration launch");
        if ((rc = read_states())) return rc;
        if (check_target) {
            // problems stopped at their target and not yet checked
            hvc.clear();
            hvi.clear();
            std::vector<int32_t> first;
            for (int64_t b = 0; b < B; ++b) {
                const GPState& S = hst[(size_t)b];
                if (!(S.done && S.f_target0 >= 0.0 && target_checkable(S.status) && !S.tcheck)) continue;
                hvc.push_back((int32_t)b);
                first.push_back((int32_t)hvi.size());
                const int64_t nb = (hI[(size_t)b].n + VR_ROWS - 1) / VR_ROWS;
                for (int64_t k = 0; k < nb; ++k) hvi.push_back(VerItem{(int32_t)b, (int32_t)k});
            }
            const int nc = (int)hvc.size();
            if (nc > 0) {
                first.push_back((int32_t)hvi.size());
                hvc.insert(hvc.end(), first.begin(), first.end());   // [cand | first]
                e = hipMemcpyAsync(dvc, hvc.data(), sizeof(int32_t) * hvc.size(), hipMemcpyHostToDevice, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(dvi, hvi.data(), sizeof(VerItem) * hvi.size(), hipMemcpyHostToDevice, s);
                if (e != hipSuccess) return hip_fail(h, e, "batched-var target check");
                const unsigned ni = (unsigned)hvi.size();
                if (kdtype == GP_F64)
                    hipLaunchKernelGGL(k_verify_rows<double>, dim3(ni), dim3(VR_T), 0, s, dvp, dvi, dvs);
                else if (kdtype == GP_F32)
                    hipLaunchKernelGGL(k_verify_rows<float>, dim3(ni), dim3(VR_T), 0, s, dvp, dvi, dvs);
                else
                    hipLaunchKernelGGL(k_verify_rows<bf16_t>, dim3(ni), dim3(VR_T), 0, s, dvp, dvi, dvs);
                hipLaunchKernelGGL(k_verify_decide, dim3((unsigned)((nc + 63) / 64)), dim3(64), 0, s, st, dvc,
                                   dvc + nc, nc, dvs, 1);
                proj(0, 1);   // a direction for the reopened problems
                e = hipGetLastError();
                if (e != hipSuccess) return hip_fail(h, e, "batched-var target check");
                std::vector<int32_t> kb((size_t)nc);
                for (int c = 0; c < nc; ++c) kb[(size_t)c] = hst[(size_t)hvc[(size_t)c]].k;
                if ((rc = read_states())) return rc;   // hvc and hvi were copied before this sync
                for (int c = 0; c < nc; ++c)
                    if (!hst[(size_t)hvc[(size_t)c]].done) it_cap = std::max(it_cap, it + (o.max_iter - kb[(size_t)c]));
            }
        }
        bool all = true;
        for (int64_t b = 0; b < B && all; ++b) all = hst[(size_t)b].done != 0;
        if (all) break;
    }
    hipLaunchKernelGGL(k_bv_finish, dim3((unsigned)B), dim3(BV_T), 0, s, dI, st, f64v ? 1 : 0);
    e = hipMemcpyAsync(hst, st, sizeof(GPState) * B, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "batched-var final sync");
    int worst = GP_OK_TOL;
    for (int64_t b = 0; b < B; ++b) {
        fill_result(hst[(size_t)b], &res[b]);
        if (severity(res[b].status) > severity(worst)) worst = res[b].status;
    }
    return worst;
}

}  // namespace gpl1
