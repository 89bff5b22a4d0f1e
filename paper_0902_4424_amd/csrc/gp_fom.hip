// The paper's fully specified comparison methods (Section 2) on the same
// device passes as GPSS:
//
//   ISTA  (item 1):  x <- S_{tau lam}[x + tau K^T (y - K x)]
//   FISTA (item 2, equation (3)):  x^(k+1) = T(z^(k)),
//         z^(k) = x^(k) + ((t_k - 1) / t_(k+1)) (x^(k) - x^(k-1)), t_0 = 1,
//         t_(k+1) = (1 + sqrt(1 + 4 t_k^2)) / 2, T the ISTA step
//   PSD   (item 5):  x <- P_Omega[x + beta r], r = K^T (y - K x),
//         beta = ||r||^2 / ||K r||^2
//
// Each K^T (y - K v) is one launch of the fused pass (t = K v - y and K^T t
// from one read of K, row slabs with partial vectors), followed by a column
// kernel that sums the partial vectors in a fixed order and applies the
// method's elementwise step.  PSD needs K r as well (a second fused pass on
// r) and the threshold search of the l1-ball projection (one workgroup, the
// values in registers).  The soft threshold S_t[v] = sgn(v) max(|v| - t, 0)
// is the projection's shrinkage with a fixed threshold (Section 2).
// ISTA and FISTA minimise the penalised functional (1),
// F(x) = ||K x - y||^2 + 2 lam ||x||_1; PSD problem (2).
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

enum FomStep : int32_t { FS_ISTA = 0, FS_FISTA = 1, FS_PSD_R = 2 };

__device__ __forceinline__ double soft(double v, double t) {
    const double a = fmax(fabs(v) - t, 0.0);
    return v < 0.0 ? -a : a;
}

// Column kernel: w_j = sum of the fused pass's partial vectors (K^T (K v - y)
// summed in index order), then
//   FS_ISTA : x_j <- S_thr(x_j - tau w_j)
//   FS_FISTA: x_new = S_thr(z_j - tau w_j), z_j <- x_new + c (x_new - x_j), x_j <- x_new
//   FS_PSD_R: r_j = -w_j, and the partial sums of r_j^2 (one per workgroup)
// (K^T (y - K v) = -w).  UPD_COLS columns per workgroup.
template <typename ACC>
__global__ __launch_bounds__(UPD_T) void k_fom_cols(GPState* __restrict__ st, int step,
                                                    const ACC* __restrict__ wpart, int64_t ldw, int GF, int64_t p,
                                                    double* __restrict__ x, double* __restrict__ z,
                                                    double* __restrict__ r, double* __restrict__ rpart, double thr,
                                                    double tau, double c) {
    constexpr int T = UPD_T;
    constexpr int VU = 16 / (int)sizeof(ACC);   // columns per vector load
    constexpr int CQ = UPD_COLS / VU;           // column vectors per workgroup
    constexpr int NG = T / CQ;                  // groups of partial vectors
    using V16 = typename std::conditional<VU == 4, float4, double2>::type;
    __shared__ double red[NG][UPD_COLS];
    if (!st->live) return;
    const int tid = threadIdx.x, cq = tid % CQ, grp = tid / CQ;
    const int64_t c0 = (int64_t)blockIdx.x * UPD_COLS;
    const ACC* src = wpart + c0 + cq * VU;
    double acc[VU];
#pragma unroll
    for (int e = 0; e < VU; ++e) acc[e] = 0.0;
    int gi = grp;
    for (; gi + 3 * NG < GF; gi += 4 * NG) {
        V16 wn[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) wn[u] = *reinterpret_cast<const V16*>(src + (int64_t)(gi + u * NG) * ldw);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
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
    if (tid >= WAVE) return;
    double rr = 0.0;
    const int64_t j = c0 + tid;
    if (tid < UPD_COLS && j < p) {
        double w = 0.0;
#pragma unroll
        for (int i = 0; i < NG; ++i) w += red[i][tid];
        if (step == FS_ISTA) {
            x[j] = soft(x[j] - tau * w, thr);
        } else if (step == FS_FISTA) {
            const double xo = x[j];
            const double xn = soft(z[j] - tau * w, thr);
            x[j] = xn;
            z[j] = xn + c * (xn - xo);
        } else {
            r[j] = -w;
            rr = w * w;
        }
    }
    if (step == FS_PSD_R) {
        rr = wave_sum(rr);
        if (tid == 0) rpart[blockIdx.x] = rr;
    } else if (blockIdx.x == 0 && tid == 0) {
        st->k += 1;
    }
}

// PSD step: beta = ||r||^2 / ||K r||^2 from the column kernel's partial sums
// and the second fused pass's t't, then x <- P_Omega(x + beta r) by the
// threshold search of the projection (values in registers, NV per thread).
// r = 0 or K r = 0 ends the run (stationary).
template <int T, int NV>
__global__ __launch_bounds__(T) void k_fom_psd_proj(GPState* __restrict__ st, double* __restrict__ x,
                                                    const double* __restrict__ r, int64_t p,
                                                    const double* __restrict__ rpart, int nr,
                                                    const double* __restrict__ spart, int GF) {
    __shared__ double lds[3 * (T / WAVE)];
    __shared__ int live;
    const int tid = threadIdx.x;
    if (tid == 0) live = st->live;
    __syncthreads();
    if (!live) return;
    double s[2] = {0.0, 0.0}, none[1] = {0.0};
    for (int i = tid; i < nr; i += T) s[0] += rpart[i];
    for (int i = tid; i < GF; i += T) s[1] += spart[SPART * i];
    block_reduce<T, 2, 1>(s, none, lds);
    const double rr = s[0], kk = s[1];
    if (!(rr > 0.0) || !(kk > 0.0)) {
        if (tid == 0) {
            st->status = isfinite(rr) && isfinite(kk) ? ST_STATIONARY : ST_NONFINITE;
            st->live = 0;
            st->stop_req = 1;
        }
        return;
    }
    const double beta = rr / kk;
    const double rho = st->prm.rho;
    double vr[NV];
    double mloc = 0.0;
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int64_t j = 2 * ((e / 2) * T + tid) + (e & 1);
        vr[e] = j < p ? fma(beta, r[j], x[j]) : 0.0;
        mloc = fmax(mloc, fabs(vr[e]));
    }
    mloc = block_max<T>(mloc, lds);
    const double mu_prev = st->mu;
    const double start = (mu_prev > 0.0 && mu_prev < mloc) ? mu_prev - mloc : -1.0;
    double m, t;
    bool inside;
    int passes;
    l1_threshold_regs<T, NV>(vr, p, rho, start, lds, m, t, inside, passes);
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int64_t j = 2 * ((e / 2) * T + tid) + (e & 1);
        if (j < p) x[j] = l1_hval(vr[e], m, t, inside, rho);
    }
    if (tid == 0) {
        if (!isfinite(m)) {
            st->status = ST_NONFINITE;
            st->live = 0;
            st->stop_req = 1;
            return;
        }
        st->k += 1;
        st->lam = beta;
        st->mu = inside ? 0.0 : m + t;
        st->michelot_total += passes;
    }
}

// PSD past the register projection's width: every workgroup forms beta from
// the same partial sums in the same order, then v = x + beta r into `v`; the
// projection kernel's streamed form (PM_PLAIN) writes P_Omega(v) into x next.
// r = 0 or K r = 0 requests the stop, which that kernel turns into live = 0.
__global__ __launch_bounds__(256) void k_fom_psd_v(GPState* __restrict__ st, const double* __restrict__ x,
                                                   const double* __restrict__ r, int64_t p,
                                                   const double* __restrict__ rpart, int nr,
                                                   const double* __restrict__ spart, int GF,
                                                   double* __restrict__ v) {
    __shared__ double lds[3 * (256 / WAVE)];
    __shared__ int live;
    const int tid = threadIdx.x;
    if (tid == 0) live = st->live;
    __syncthreads();
    if (!live) return;
    double s[2] = {0.0, 0.0}, none[1] = {0.0};
    for (int i = tid; i < nr; i += 256) s[0] += rpart[i];
    for (int i = tid; i < GF; i += 256) s[1] += spart[SPART * i];
    block_reduce<256, 2, 1>(s, none, lds);
    const double rr = s[0], kk = s[1];
    if (!(rr > 0.0) || !(kk > 0.0)) {
        if (blockIdx.x == 0 && tid == 0) {
            st->status = isfinite(rr) && isfinite(kk) ? ST_STATIONARY : ST_NONFINITE;
            st->stop_req = 1;
        }
        return;
    }
    const double beta = rr / kk;
    for (int64_t j = (int64_t)blockIdx.x * 256 + tid; j < p; j += (int64_t)gridDim.x * 256)
        v[j] = fma(beta, r[j], x[j]);
    if (blockIdx.x == 0 && tid == 0) {
        st->k += 1;
        st->lam = beta;
    }
}

// End of a run: x narrowed into the caller's output and ||x||_1 of the
// returned values.
template <typename TV>
__global__ __launch_bounds__(1024) void k_fom_finish(GPState* __restrict__ st, const double* __restrict__ x,
                                                     int64_t p, TV* __restrict__ x_out) {
    __shared__ double lds[1024 / WAVE];
    double l1 = 0.0;
    for (int64_t j = threadIdx.x; j < p; j += 1024) {
        const TV v = (TV)x[j];
        x_out[j] = v;
        l1 += fabs((double)v);
    }
    l1 = block_sum<1024>(l1, lds);
    if (threadIdx.x == 0) {
        st->l1 = l1;
        st->done = 1;
    }
}

// Objective of the returned x: f = ||K x - y||^2 from the rows' FP64 partial
// sums (fixed order), plus 2 lam ||x||_1 for the penalised methods.
static __global__ void k_fom_objective(GPState* __restrict__ st, const double* __restrict__ part, int nitems,
                                       double lam2) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double f = 0.0;
    for (int i = 0; i < nitems; ++i) f += part[i];
    st->f = f + lam2 * st->l1;
    st->f_exact = f;
}

namespace {
int fom_nv(int64_t p) {
    const int64_t per = (p + 1023) / 1024;
    for (int v : {2, 4, 8, 16, 32})
        if (per <= v) return v;
    return 0;
}
}  // namespace

}  // namespace gpl1

extern "C" int gp_fom_solve(gp_handle h, int32_t method, gp_dtype kdtype, const void* K, int64_t n, int64_t p,
                            int64_t ldk, const void* y, double param, double tau, const void* x0, int32_t iters,
                            void* x_out, const gp_opts* opts, gp_result* res, void* stream) {
    if (!h) return GP_E_ARG;
    h->err.clear();
    if (!res) return fail(h, GP_E_ARG, "res must not be NULL");
    std::memset(res, 0, sizeof(*res));
    res->status = GP_E_ARG;
    gp_opts o;
    if (opts) o = *opts; else gp_opts_default(&o);
    if (method != GP_ISTA && method != GP_FISTA && method != GP_PSD) return fail(h, GP_E_ARG, "unknown method");
    if (kdtype != GP_F64 && kdtype != GP_F32 && kdtype != GP_BF16) return fail(h, GP_E_ARG, "bad dtype");
    if (n <= 0 || p <= 0) return fail(h, GP_E_ARG, "n and p must be positive");
    if (ldk < p) return fail(h, GP_E_ARG, "ldk must be >= p");
    if (!(param >= 0.0) || !std::isfinite(param))
        return fail(h, GP_E_ARG, "lambda (ISTA, FISTA) or rho (PSD) must be finite and >= 0");
    if (tau == 0.0) tau = 1.0;
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(h, GP_E_ARG, "tau must be finite and > 0");
    if (iters < 0) return fail(h, GP_E_ARG, "iters must be >= 0");
    if (o.chunk < 1) return fail(h, GP_E_ARG, "opts.chunk must be >= 1");
    if (!K || !y || !x_out) return fail(h, GP_E_ARG, "null pointer argument");
    if (n > ((int64_t)1 << 31)) return fail(h, GP_E_UNSUPPORTED, "n too large");
    // PSD projects in registers (up to 32 values per thread of one workgroup);
    // ISTA and FISTA take any p
    // PSD projects in registers up to 32 values per thread of one workgroup,
    // beyond that through the projection kernel's streamed form
    const int nv = fom_nv(p);
    Plan P = plan_single(kdtype, n, p, o);
    if (P.cfg < 0)
        return fail(h, GP_E_UNSUPPORTED, "p = " + std::to_string(p) + " exceeds the fused kernel's column capacity");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    int rc = ensure_workspace(h, P.bytes);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)h->ws;
    GPState* st = (GPState*)(ws + P.o_state);
    double* x = (double*)(ws + P.o_x);
    double* zr = (double*)(ws + P.o_g);      // FISTA: z; PSD: r
    double* vb = (double*)(ws + P.o_vbuf);
    double* t = (double*)(ws + P.o_q);       // K v - y of the last pass
    double* y64 = (double*)(ws + P.o_y);
    double* spart = (double*)(ws + P.o_spart);
    double* rpart = (double*)(ws + P.o_upart);
    void* wpart = ws + P.o_wpart;
    const bool f64v = kdtype == GP_F64;
    const int vec = 16 / esize(kdtype);
    const bool aligned = (ldk % vec == 0) && (p % vec == 0) && (((uintptr_t)K) % 16 == 0);   // as in gp_l1_solve

    gp_opts po = o;
    po.max_iter = iters;
    po.f_target = -1.0;
    GPParams prm = make_params(po, method == GP_PSD ? param : 0.0, 0.0);
    {
        const unsigned sg = (unsigned)((std::max(n, p) + 255) / 256);
        if (f64v)
            hipLaunchKernelGGL(k_setup<double>, dim3(sg), dim3(256), 0, s, st, prm, (const double*)y, y64, n,
                               (const double*)x0, x, p);
        else
            hipLaunchKernelGGL(k_setup<float>, dim3(sg), dim3(256), 0, s, st, prm, (const float*)y, y64, n,
                               (const float*)x0, x, p);
    }
    // PSD starts from P_Omega(x0) (x0 in Omega, Algorithm 1's requirement)
    if (method == GP_PSD && x0) {
        hipLaunchKernelGGL((k_proj<0, 1024>), dim3(1), dim3(1024), 0, s, st, (int)PM_INIT_X0, p, x,
                           (const double*)nullptr, (double*)nullptr, (const double*)nullptr, 0, vb, (float*)nullptr);
    }
    if (method == GP_FISTA) {
        e = hipMemcpyAsync(zr, x, 8 * p, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(h, e, "fista set-up");
    }
    // FISTA momentum factors c_k = (t_k - 1) / t_(k+1), t_0 = 1 (equation (3))
    std::vector<double> cf;
    if (method == GP_FISTA) {
        cf.resize((size_t)iters + 2);
        double tk = 1.0;
        for (size_t k = 0; k < cf.size(); ++k) {
            const double tn = (1.0 + std::sqrt(1.0 + 4.0 * tk * tk)) / 2.0;
            cf[k] = (tk - 1.0) / tn;
            tk = tn;
        }
    }
    FusedArgs fa_x{st, K, n, p, ldk, P.rows, x, nullptr, nullptr, y64, nullptr, t, wpart, P.ldw, spart,
                   o.fused_interleave, nullptr};
    FusedArgs fa_z{st, K, n, p, ldk, P.rows, zr, nullptr, nullptr, y64, nullptr, t, wpart, P.ldw, spart,
                   o.fused_interleave, nullptr};
    FusedArgs fa_r{st, K, n, p, ldk, P.rows, zr, nullptr, nullptr, nullptr, nullptr, t, wpart, P.ldw, spart,
                   o.fused_interleave, nullptr};
    fa_x.tpart = fa_z.tpart = fa_r.tpart = (double*)(ws + P.o_tpart);
    fa_x.np = fa_z.np = fa_r.np = P.np;
    const unsigned nbp = (unsigned)P.nbp;
    auto cols = [&](int step, double thr, double c) {
        if (f64v)
            hipLaunchKernelGGL(k_fom_cols<double>, dim3(nbp), dim3(UPD_T), 0, s, st, step, (const double*)wpart,
                               P.ldw, (int)P.G, p, x, zr, zr, rpart, thr, tau, c);
        else
            hipLaunchKernelGGL(k_fom_cols<float>, dim3(nbp), dim3(UPD_T), 0, s, st, step, (const float*)wpart,
                               P.ldw, (int)P.G, p, x, zr, zr, rpart, thr, tau, c);
    };
    double* vd = (double*)(ws + P.o_d);      // PSD past 32768 columns: v = x + beta r
    auto psd_proj = [&]() {
        if (nv == 0) {
            const unsigned gb = (unsigned)std::min<int64_t>((p + 255) / 256, 1024);
            hipLaunchKernelGGL(k_fom_psd_v, dim3(gb), dim3(256), 0, s, st, (const double*)x, (const double*)zr, p,
                               (const double*)rpart, (int)nbp, (const double*)spart, (int)P.G, vd);
            hipLaunchKernelGGL((k_proj<0, 1024>), dim3(1), dim3(1024), 0, s, st, (int)PM_PLAIN, p, vd,
                               (const double*)nullptr, x, (const double*)nullptr, 0, vb, (float*)nullptr);
            return;
        }
        switch (nv) {
#define GPL1_FOM_PROJ(V) \
    case V: \
        hipLaunchKernelGGL((k_fom_psd_proj<1024, V>), dim3(1), dim3(1024), 0, s, st, x, (const double*)zr, p, \
                           (const double*)rpart, (int)nbp, (const double*)spart, (int)P.G); \
        break;
            GPL1_FOM_PROJ(2) GPL1_FOM_PROJ(4) GPL1_FOM_PROJ(8) GPL1_FOM_PROJ(16) GPL1_FOM_PROJ(32)
#undef GPL1_FOM_PROJ
        }
    };
    const double thr = tau * param;
    int it = 0;
    while (it < iters) {
        const int end = std::min(iters, it + o.chunk);
        for (; it < end; ++it) {
            if (method == GP_ISTA) {
                launch_fused(kdtype, P.cfg, aligned, s, P.G, fa_x);
                cols(FS_ISTA, thr, 0.0);
            } else if (method == GP_FISTA) {
                launch_fused(kdtype, P.cfg, aligned, s, P.G, fa_z);
                cols(FS_FISTA, thr, cf[(size_t)it + 1]);
            } else {
                launch_fused(kdtype, P.cfg, aligned, s, P.G, fa_x);
                cols(FS_PSD_R, 0.0, 0.0);
                launch_fused(kdtype, P.cfg, aligned, s, P.G, fa_r);
                psd_proj();
            }
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(h, e, "iteration launch");
        if (method == GP_PSD && it < iters) {
            // PSD may stop early (r = 0 or K r = 0): poll between chunks
            e = hipMemcpyAsync(h->host_state, st, sizeof(GPState), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(h, e, "status poll");
            if (!h->host_state->live) break;
        }
    }
    // the returned x and its objective, with K x - y in double
    if (f64v) hipLaunchKernelGGL(k_fom_finish<double>, dim3(1), dim3(1024), 0, s, st, x, p, (double*)x_out);
    else hipLaunchKernelGGL(k_fom_finish<float>, dim3(1), dim3(1024), 0, s, st, x, p, (float*)x_out);
    VerProb* vprob = (VerProb*)(ws + P.o_vprob);
    VerItem* vitems = (VerItem*)(ws + P.o_vitem);
    double* vpart = (double*)(ws + P.o_vpart);
    int32_t* vidx = (int32_t*)(ws + P.o_vidx);
    const VerProb vp{K, ldk, n, p, x, y64, f64v ? 0 : 1,
                     ((ldk * esize(kdtype)) % 16 == 0 && ((uintptr_t)K) % 16 == 0) ? 1 : 0};
    hipLaunchKernelGGL(k_verify_setup_single, dim3((unsigned)((P.nvitems + 255) / 256)), dim3(256), 0, s, vprob,
                       vitems, vidx, P.nvitems, vp);
    launch_verify_rows(kdtype, s, P.nvitems, vprob, vitems, vpart);
    hipLaunchKernelGGL(k_fom_objective, dim3(1), dim3(64), 0, s, st, vpart, P.nvitems,
                       method == GP_PSD ? 0.0 : 2.0 * param);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h->host_state, st, sizeof(GPState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "final sync");
    const GPState& S = *h->host_state;
    res->status = S.status == ST_STATIONARY ? GP_STATIONARY : S.status == ST_NONFINITE ? GP_E_NONFINITE : GP_MAX_ITER;
    res->iters = S.k;
    res->f = S.f;
    res->l1norm = S.l1;
    res->projected_x0 = S.projected;
    res->proj_passes = S.michelot_total;
    if (!std::isfinite(S.f) && res->status >= 0) res->status = GP_E_NONFINITE;
    if (res->status < 0) return fail(h, res->status, "non-finite value in the run");
    return res->status;
}
