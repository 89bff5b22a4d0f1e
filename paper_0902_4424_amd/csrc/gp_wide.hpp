// The K pass of wide problems: p beyond the columns one workgroup of the
// fused kernel holds in registers at full speed.
//
// The fused kernel keeps a whole row of the direction in each workgroup's
// registers, so that the row block of K it reads for q_i = K_i d can serve
// K_i^T q_i while still in registers.  A wider problem cuts the columns into
// panels of WIDE_T * wide_cpt * VEC columns.  q_i then sums over panels that no single
// workgroup holds, so the pass takes two launches over K:
//
//   k_wide_t (slabs x panels) : partial dots of every panel,
//                               tpart[c * n + i] = sum_{j in panel c} K_ij u_j;
//   k_wide_w (slabs x panels) : t_i = sum_c tpart[c * n + i] (- y_i), in a
//                               fixed order, the same bits in every panel;
//                               then the panel's columns of the slab's partial
//                               w = K^T t, written where the fused kernel
//                               writes them.
//
// The outputs are those of the fused kernel (t, the G partial vectors of w,
// the per-slab dots t't, t'r, g'd, d'd, ||d||_inf), so the update kernel and
// every caller work unchanged.  K is read twice per pass: twice the fused
// kernel's bytes.
#pragma once

#include "gp_kernels.hpp"

namespace gpl1 {

constexpr int WIDE_T = 512;
constexpr int WIDE_RB = 1;

// 16-byte column chunks per thread: 32 columns for float and bf16 K (with 64
// bf16 columns per thread the pass measured 2-16 % slower), 16 for double.
template <typename TK>
constexpr int wide_cpt() {
    return sizeof(TK) == 2 ? 4 : 8;
}
// Columns of one panel.
template <typename TK>
constexpr int64_t wide_panel() {
    return (int64_t)WIDE_T * wide_cpt<TK>() * KTraits<TK>::VEC;
}

// The multiplied vector u over panel columns [c0, c0 + PW), as the fused
// kernel forms it (float copy of d, else h - x, else v).
template <typename TK, typename ACC, int T, int CPT>
__device__ __forceinline__ void wide_direction(ACC (&dv)[CPT][KTraits<TK>::VEC], int64_t c0, int64_t p,
                                               const double* v, const double* vsub, const double* g,
                                               const float* v32, const ProjH& ph) {
    constexpr int VEC = KTraits<TK>::VEC;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int64_t j = c0 + ((int64_t)c * T + threadIdx.x) * VEC + e;
            ACC u = 0;
            if (j < p) {
                if (v32) u = (ACC)v32[j];
                else if (vsub) u = (ACC)((v ? v[j] : proj_h(vsub[j], g[j], ph)) - vsub[j]);
                else u = (ACC)v[j];
            }
            dv[c][e] = u;
        }
    }
}

template <typename TK, typename ACC, int T, int CPT, int RB, bool ALIGNED>
__global__ __launch_bounds__(T) void k_wide_t(const GPState* __restrict__ st, const TK* __restrict__ K, int64_t n,
                                              int64_t p, int64_t ldk, int64_t rows_per_wg,
                                              const double* __restrict__ v, const double* __restrict__ vsub,
                                              const double* __restrict__ g, const float* __restrict__ v32,
                                              double* __restrict__ tpart) {
    if (!st->live) return;
    using FB = FusedBlock<TK, ACC, T, CPT, RB>;
    constexpr int VEC = FB::VEC;
    constexpr int NW = FB::NW;
    constexpr int64_t PW = (int64_t)T * CPT * VEC;
    const ProjH ph = v ? ProjH{} : proj_h_params(st);
    const int64_t c0 = (int64_t)blockIdx.y * PW;
    const int64_t pw = p - c0 < PW ? p - c0 : PW;
    const TK* Kp = K + c0;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r1 = r0 + rows_per_wg < n ? r0 + rows_per_wg : n;
    double* out = tpart + (int64_t)blockIdx.y * n;

    ACC dv[CPT][VEC];
    wide_direction<TK, ACC, T, CPT>(dv, c0, p, v, vsub, g, v32, ph);
    __shared__ double red[2][RB][NW];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    int bi = 0;
    // one barrier per row block: red is double-buffered, and a wave can only
    // overwrite a buffer after every wave has passed the next block's barrier
    auto dots = [&](const KVec<TK> (&buf)[RB][CPT], int64_t row) {
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
        if (threadIdx.x < RB && row + threadIdx.x < r1) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < NW; ++i) t += red[bi][threadIdx.x][i];
            out[row + threadIdx.x] = t;
        }
        bi ^= 1;
    };
    KVec<TK> A[RB][CPT], B[RB][CPT];
    if (r0 < r1) FB::template load<ALIGNED>(A, Kp, ldk, pw, r0, r1);
    for (int64_t row = r0; row < r1; row += 2 * RB) {
        if (row + RB < r1) FB::template load<ALIGNED>(B, Kp, ldk, pw, row + RB, r1);
        dots(A, row);
        if (row + RB >= r1) break;
        if (row + 2 * RB < r1) FB::template load<ALIGNED>(A, Kp, ldk, pw, row + 2 * RB, r1);
        dots(B, row + RB);
    }
}

template <typename TK, typename ACC, int T, int CPT, int RB, bool ALIGNED>
__global__ __launch_bounds__(T) void k_wide_w(const GPState* __restrict__ st, const TK* __restrict__ K, int64_t n,
                                              int64_t p, int64_t ldk, int64_t rows_per_wg, int np,
                                              const double* __restrict__ tpart, const double* __restrict__ v,
                                              const double* __restrict__ vsub, const double* __restrict__ g,
                                              const double* __restrict__ ysub, const double* __restrict__ rvec,
                                              double* __restrict__ tout, ACC* __restrict__ wpart, int64_t ldw,
                                              double* __restrict__ spart) {
    if (!st->live) return;
    using FB = FusedBlock<TK, ACC, T, CPT, RB>;
    constexpr int VEC = FB::VEC;
    constexpr int NW = FB::NW;
    constexpr int64_t PW = (int64_t)T * CPT * VEC;
    constexpr int FCH = 256;   // rows of t staged at a time
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * PW;
    const int64_t pw = p - c0 < PW ? p - c0 : PW;
    const TK* Kp = K + c0;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r1 = r0 + rows_per_wg < n ? r0 + rows_per_wg : n;
    // the panel-0 workgroup of each slab writes t and the slab's dots
    const bool lead = blockIdx.y == 0;

    ACC w[CPT][VEC];
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) w[c][e] = 0;
    __shared__ double s_t[FCH];
    double tt = 0.0, tr = 0.0;
    KVec<TK> A[RB][CPT], B[RB][CPT];
    auto fold = [&](const KVec<TK> (&buf)[RB][CPT], int64_t row, int64_t cb, int64_t ce) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (row + r < ce) {
                const ACC ta = (ACC)s_t[row + r - cb];
#pragma unroll
                for (int c = 0; c < CPT; ++c)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) w[c][e] += (ACC)buf[r][c].get(e) * ta;
            }
        }
    };
    for (int64_t cb = r0; cb < r1; cb += FCH) {
        const int64_t ce = cb + FCH < r1 ? cb + FCH : r1;
        // the chunk's first rows of K load while t is formed
        FB::template load<ALIGNED>(A, Kp, ldk, pw, cb, ce);
        __syncthreads();   // the previous chunk's t is no longer read
        for (int64_t i = tid; i < ce - cb; i += T) {
            const int64_t row = cb + i;
            double t = 0.0;
            for (int c = 0; c < np; ++c) t += tpart[(int64_t)c * n + row];
            if (ysub) t -= ysub[row];
            s_t[i] = t;
            if (lead) {
                tout[row] = t;
                tt += t * t;
                if (rvec) tr += t * rvec[row];
            }
        }
        __syncthreads();
        for (int64_t row = cb; row < ce; row += 2 * RB) {
            if (row + RB < ce) FB::template load<ALIGNED>(B, Kp, ldk, pw, row + RB, ce);
            fold(A, row, cb, ce);
            if (row + RB >= ce) break;
            if (row + 2 * RB < ce) FB::template load<ALIGNED>(A, Kp, ldk, pw, row + 2 * RB, ce);
            fold(B, row + RB, cb, ce);
        }
    }
    ACC* wrow = wpart + (int64_t)blockIdx.x * ldw + c0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t col = ((int64_t)c * T + tid) * VEC;
        if (c0 + col < ldw) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) wrow[col + e] = w[c][e];
        }
    }
    if (!lead) return;
    // direction dots over this slab's slice of the columns, as the fused
    // kernel takes them
    double sums[4] = {tt, tr, 0.0, 0.0}, dmx[1] = {0.0};
    if (g) {
        const ProjH ph = v ? ProjH{} : proj_h_params(st);
        const int64_t G = gridDim.x;
        const int64_t cs = (p + G - 1) / G;
        const int64_t j0 = (int64_t)blockIdx.x * cs;
        const int64_t j1 = j0 + cs < p ? j0 + cs : p;
        for (int64_t j = j0 + tid; j < j1; j += T) {
            const double dj = (v ? v[j] : proj_h(vsub[j], g[j], ph)) - vsub[j];
            sums[2] += g[j] * dj;
            sums[3] += dj * dj;
            dmx[0] = fmax(dmx[0], fabs(dj));
        }
    }
    __shared__ double lds5[5 * NW];
    block_reduce<T, 4, 1>(sums, dmx, lds5);
    if (tid == 0) {
        double* sp = spart + (int64_t)SPART * blockIdx.x;
        sp[0] = sums[0];
        sp[1] = sums[1];
        sp[2] = sums[2];
        sp[3] = sums[3];
        sp[4] = dmx[0];
    }
}

}  // namespace gpl1
