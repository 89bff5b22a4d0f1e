// Exact check of an objective target.
//
// The iteration tracks f(x) = ||K x - y||^2 as f + lam (2 r'q + lam q'q) with
// products of FP32 accuracy, so a stop on "f <= f_target" is only as exact as
// those products.  When the tracked f of a problem meets its target, the
// stop is a candidate: f is recomputed in double from the stored K, y and
// the x the caller receives (narrowed to the vector dtype), and
//   * f_exact <= the caller's target: the stop stands and the result reports
//     f_exact;
//   * otherwise the problem is reopened with its device target lowered by
//     twice the difference between f_exact and the tracked f, and iterates on.
// A problem with a target that stops for another reason (stationary, tol,
// budget, failed line search) is checked as well: it reports f_exact, with
// status ST_TARGET if that meets the target.
#pragma once

#include "gp_device.hpp"
#include "gp_state.hpp"

namespace gpl1 {

constexpr int VR_T = 256;       // threads of a row-check workgroup (four waves)
constexpr int VR_ROWS = 16;     // rows per work item (four per wave)
constexpr int VR_TILE = 2048;   // columns of x staged in LDS at a time

// One problem of a check: K row-major (ldk), x and y as double copies on the
// device; `narrow` rounds each x_j to float first (the vector dtype the
// caller receives for float and bf16 K); `aligned`: rows 16-byte aligned.
struct VerProb {
    const void* K;
    int64_t ldk, n, p;
    const double* x;
    const double* y;
    int32_t narrow, aligned;
};
struct VerItem { int32_t prob, blk; };   // rows [blk * VR_ROWS, (blk + 1) * VR_ROWS) of problem prob

template <typename TK> __device__ __forceinline__ double kelem(const TK* row, int64_t j);
template <> __device__ __forceinline__ double kelem<double>(const double* row, int64_t j) { return row[j]; }
template <> __device__ __forceinline__ double kelem<float>(const float* row, int64_t j) { return (double)row[j]; }
template <> __device__ __forceinline__ double kelem<bf16_t>(const bf16_t* row, int64_t j) {
    return (double)bf16_to_float(reinterpret_cast<const uint16_t*>(row)[j]);
}

// part[item] = sum over the item's rows of (K_i x - y_i)^2, every product and
// sum in double (K and x widen exactly).  Fixed order: per lane along the
// columns, a wave butterfly per row, waves in index order.
template <typename TK>
__global__ __launch_bounds__(VR_T) void k_verify_rows(const VerProb* __restrict__ probs,
                                                      const VerItem* __restrict__ items,
                                                      double* __restrict__ part) {
    constexpr int NWV = VR_T / WAVE;
    constexpr int RPW = VR_ROWS / NWV;
    constexpr int VEC = KTraits<TK>::VEC;
    static_assert(VR_TILE % (WAVE * VEC) == 0, "a tile is a whole number of wave-wide chunks");
    __shared__ double xs[VR_TILE];
    __shared__ double wpost[NWV];
    const VerItem it = items[blockIdx.x];
    const VerProb P = probs[it.prob];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int64_t i0 = (int64_t)it.blk * VR_ROWS + (int64_t)wid * RPW;
    double acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = 0.0;
    for (int64_t c0 = 0; c0 < P.p; c0 += VR_TILE) {
        const int cw = (int)(P.p - c0 < VR_TILE ? P.p - c0 : VR_TILE);
        __syncthreads();
        for (int j = threadIdx.x; j < VR_TILE; j += VR_T) {
            double v = j < cw ? P.x[c0 + j] : 0.0;
            if (P.narrow) v = (double)(float)v;
            xs[j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int64_t i = i0 + r;
            if (i >= P.n) break;
            const TK* row = (const TK*)P.K + i * P.ldk + c0;
            double a = acc[r];
            if (P.aligned) {
                // c0 is a multiple of the tile, so the tile's row start keeps
                // the row's 16-byte alignment; chunks past cw read as zero
                for (int jj = lane * VEC; jj < cw; jj += WAVE * VEC) {
                    KVec<TK> kv;
                    load_kvec<TK, true>(row, jj, cw, kv);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) a = fma((double)kv.get(e), xs[jj + e], a);
                }
            } else {
                for (int jj = lane; jj < cw; jj += WAVE) a = fma(kelem<TK>(row, jj), xs[jj], a);
            }
            acc[r] = a;
        }
    }
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int64_t i = i0 + r;
        const double t = wave_sum(acc[r]);
        if (i < P.n) {
            const double d = t - P.y[i];
            s += d * d;
        }
    }
    if (lane == 0) wpost[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) tot += wpost[w];
        part[blockIdx.x] = tot;
    }
}

// Which stops of a problem with a target are checked: the target stop, and
// the stops that end the run for another reason (stationary, tol, budget, a
// line search that found no decrease at working precision, x unchanged),
// where the check may find the target met after all.
__device__ __host__ __forceinline__ bool target_checkable(int status) {
    return status == ST_TARGET || status == ST_STATIONARY || status == ST_OK_TOL || status == ST_MAX_ITER ||
           status == ST_BACKTRACK;
}

// Descriptor, row items and index arrays of a single problem's check,
// written on the device (no host buffer to keep alive).
static __global__ void k_verify_setup_single(VerProb* vp, VerItem* items, int32_t* idx, int nitems, VerProb prob) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *vp = prob;
        idx[0] = 0;          // the checked problem
        idx[1] = 0;          // its items: [0, nitems)
        idx[2] = nitems;
    }
    if (i < nitems) items[i] = VerItem{0, i};
}

// The decision for a stopped problem with a target, given f_exact.  The
// result reports f_exact.  f_exact <= the caller's target: the status becomes
// ST_TARGET.  Otherwise a target stop is reopened (returns 0: status back to
// ST_MAX_ITER, device target lowered; the caller clears its own stop flags)
// and any other stop keeps its status.  Returns 1 when the stop stands.
__device__ __forceinline__ int target_decide(GPState* st, double f_exact) {
    st->f_exact = f_exact;
    if (f_exact <= st->f_target0 || st->status != ST_TARGET) {
        if (f_exact <= st->f_target0) st->status = ST_TARGET;
        st->f = f_exact;
        st->tcheck = 1;
        return 1;
    }
    // the tracked f undershot by f_exact - f (> 0, since f <= target < f_exact)
    const double lowered = st->f_target0 - 2.0 * (f_exact - st->f);
    st->prm.f_target = fmax(0.0, fmin(st->prm.f_target, lowered));
    st->status = ST_MAX_ITER;
    st->reopened += 1;
    return 0;
}

// Sum the partial sums of checked problem c (items first[c] .. first[c+1]-1,
// in order) and decide.  The single-problem solver (mode 0) reopens by
// clearing its stop flags; an uneven batch (mode 1) marks the problem for a
// fresh projection before its next sweep.  One thread per checked problem.
static __global__ void k_verify_decide(GPState* __restrict__ st_all, const int32_t* __restrict__ cand,
                                const int32_t* __restrict__ first, int nc, const double* __restrict__ part,
                                int mode) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    GPState* st = st_all + cand[c];
    double f = 0.0;
    for (int i = first[c]; i < first[c + 1]; ++i) f += part[i];
    if (target_decide(st, f)) return;
    st->done = 0;
    if (mode == 0) {
        st->stop_req = 0;
        st->live = 1;
    } else {
        st->reproj = 1;
    }
}

}  // namespace gpl1
