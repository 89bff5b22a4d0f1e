// Unrolled soft-thresholding network (learned warm start for GPSS).
//
//   c = We y,  u_1 = c,  x_t = S_{theta_t}(u_t),  u_t = c + S x_{t-1} (t >= 2)
//
// Forward and backward products run on the bf16 matrix cores through the
// GEMM of gp_gemm.hpp: Cpart[j][i] = sum_k A[i][k] * B[j][k] with A in bf16
// (one plane) and B as three bf16 planes.  Products weight x activation use
// the bf16 weights as A and split activations as B (FP32-accurate); the
// weight gradients use one activation as a bf16 A operand (bf16-accurate, the
// usual mixed-precision choice).
//
// Layouts (all padded to multiples of 128 with zeros; pp = padded p, np =
// padded n, bp = padded batch):
//   masters (FP32, in the layout the gradient GEMMs produce):
//     WeT [np][pp]  WeT[a][i] = We[i][a]        ST [pp][pp]  ST[j][i] = S[i][j]
//   bf16 working copies: We_bf [pp][np] = We, S_bf [pp][pp] = S, St_bf = S^T
//   activations: U, X [layers][bp][pp] (FP32), planes of the GEMM operands.
// The gradient of S is one GEMM over all layers: the reduction index runs
// over (layer, sample) pairs of dU_t and x_{t-1} laid out side by side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gp_gemm.hpp"
#include "gp_internal.hpp"
#include "gp_kernels.hpp"
#include "gp_l1.h"

using namespace gpl1;

struct gp_lista_s {
    gp_handle h = nullptr;
    int64_t n = 0, p = 0, np = 0, pp = 0;
    int32_t L = 0;
    int64_t step = 0;
    // persistent
    float *WeT = nullptr, *ST = nullptr, *th = nullptr;            // masters
    float *mWe = nullptr, *vWe = nullptr, *mS = nullptr, *vS = nullptr, *mth = nullptr, *vth = nullptr;
    uint16_t *We_bf = nullptr, *S_bf = nullptr, *St_bf = nullptr;
    float *gWeT = nullptr, *gST = nullptr, *gth = nullptr;          // gradients (master layouts)
    bool bf_valid = false;
    void* persist = nullptr;
    // per batch size
    void* act = nullptr;
    size_t act_bytes = 0;
    int64_t act_bp = 0;
    int fwd_planes = 3;   // bf16 planes of the activations in gp_lista_forward
};

namespace gpl1 {

constexpr int LI_PAD = 128;
constexpr int LI_T = 256;

__device__ __forceinline__ uint16_t li_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float li_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ void li_split3(float v, uint16_t* pl, int64_t ps, int64_t idx) {
    const uint16_t h = li_bf16(v);
    const float r1 = v - li_f32(h);
    const uint16_t m = li_bf16(r1);
    const float r2 = r1 - li_f32(m);
    pl[idx] = h;
    pl[ps + idx] = m;
    pl[2 * ps + idx] = li_bf16(r2);
}

// out planes[j][i] (ld_out) from src[i][j] (ld_src), rows i < ri, cols j < cj
// (zeros elsewhere in the tile); nplanes = 1 or 3.  64 x 64 tiles.
__global__ void k_li_transpose_split(const float* __restrict__ src, int64_t ld_src, int64_t ri, int64_t cj,
                                     uint16_t* __restrict__ out, int64_t ld_out, int64_t pstride,
                                     int nplanes, int64_t out_col_off) {
    __shared__ float tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, j = j0 + tx;
        tile[r][tx] = (i < ri && j < cj) ? src[i * ld_src + j] : 0.f;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t j = j0 + r, i = i0 + tx;
        const float v = tile[tx][r];
        const int64_t idx = j * ld_out + out_col_off + i;
        if (nplanes == 3) li_split3(v, out, pstride, idx);
        else out[idx] = li_bf16(v);
    }
}

// planes[r][c] (ld_out) from src[r][c] (ld_src), r < rows, c < cols
__global__ void k_li_split_rows(const float* __restrict__ src, int64_t ld_src, int64_t rows, int64_t cols,
                                uint16_t* __restrict__ out, int64_t ld_out, int64_t pstride) {
    const int64_t r = blockIdx.y;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x)
        li_split3(r < rows ? src[r * ld_src + c] : 0.f, out, pstride, r * ld_out + c);
}

// bf16 working copies from the masters
__global__ void k_li_weights_bf16(const float* __restrict__ ST, int64_t pp, uint16_t* __restrict__ St_bf) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < pp * pp) St_bf[idx] = li_bf16(ST[idx]);
}

// forward epilogue of layer t: u = sum of partials (+ c), x = S_theta(u)
__global__ void k_li_fwd_act(const float* __restrict__ part, int S, int64_t pstride_part, int64_t ld,
                             int64_t B, int64_t p, float* __restrict__ C, int first, float* __restrict__ U,
                             float* __restrict__ X, const float* __restrict__ th, int t,
                             uint16_t* __restrict__ Xpl, int64_t plstride) {
    const int64_t b = blockIdx.y;
    if (b >= B) return;
    const float theta = th[t];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t idx = b * ld + i;
        float u = 0.f;
        for (int s = 0; s < S; ++s) u += part[s * pstride_part + idx];
        if (first) C[idx] = u;
        else u += C[idx];
        U[idx] = u;
        const float a = fabsf(u) - theta;
        const float x = a > 0.f ? copysignf(a, u) : 0.f;
        X[idx] = x;
        if (Xpl) li_split3(x, Xpl, plstride, idx);
    }
}

// loss and dX of the last layer: dX = (x - x*)/B; per-block loss partials
__global__ void k_li_loss(const float* __restrict__ X, int64_t ld, const float* __restrict__ Xs, int64_t ldx,
                          int64_t B, int64_t p, float* __restrict__ dX, double* __restrict__ lpart) {
    __shared__ double lds[3 * (LI_T / WAVE)];
    const int64_t b = blockIdx.y;
    double acc[1] = {0.0}, none[1] = {0.0};
    if (b < B) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x) {
            const float e = X[b * ld + i] - Xs[b * ldx + i];
            dX[b * ld + i] = e / (float)B;
            acc[0] += (double)e * e;
        }
    }
    block_reduce<LI_T, 1, 1>(acc, none, lds);
    if (threadIdx.x == 0) lpart[blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
}

// backward through S_theta of layer t: dU = dX 1[|u| > theta]; dtheta partial
// = -sum dX sgn(u) 1[...]; dC += dU (= dU at the last layer); dU planes for
// the dX of the layer below
__global__ void k_li_bwd_act(const float* __restrict__ dX, const float* __restrict__ U, int64_t ld, int64_t B,
                             int64_t p, const float* __restrict__ th, int t, float* __restrict__ dU,
                             float* __restrict__ dC, int first, uint16_t* __restrict__ dUpl, int64_t plstride,
                             double* __restrict__ tpart) {
    __shared__ double lds[3 * (LI_T / WAVE)];
    const int64_t b = blockIdx.y;
    const float theta = th[t];
    double acc[1] = {0.0}, none[1] = {0.0};
    if (b < B) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x) {
            const int64_t idx = b * ld + i;
            const float u = U[idx];
            const bool on = fabsf(u) > theta;
            const float g = on ? dX[idx] : 0.f;
            dU[idx] = g;
            if (on) acc[0] -= (double)dX[idx] * (u > 0.f ? 1.0 : -1.0);
            dC[idx] = first ? g : dC[idx] + g;
            if (dUpl) li_split3(g, dUpl, plstride, idx);
        }
    }
    block_reduce<LI_T, 1, 1>(acc, none, lds);
    if (threadIdx.x == 0) tpart[blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
}

// dst[c * ldd + r] = src[r * lds + c] for r < rows, c < cols
__global__ void k_li_transpose_f32(const float* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                                   float* __restrict__ dst, int64_t ldd) {
    const int64_t r = blockIdx.y;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x)
        dst[c * ldd + r] = src[r * lds + c];
}

__global__ void k_li_sum_parts(const float* __restrict__ part, int S, int64_t pstride, int64_t count,
                               float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int c = 0; c < S; ++c) s += part[c * pstride + i];
    out[i] = s;
}

// fixed-order sum of block partials (one workgroup)
__global__ void k_li_reduce(const double* __restrict__ part, int64_t count, double* __restrict__ out) {
    __shared__ double lds[3 * (LI_T / WAVE)];
    double acc[1] = {0.0}, none[1] = {0.0};
    for (int64_t i = threadIdx.x; i < count; i += LI_T) acc[0] += part[i];
    block_reduce<LI_T, 1, 1>(acc, none, lds);
    if (threadIdx.x == 0) *out = acc[0];
}

// Adam on an FP32 master with its gradient (same layout)
__global__ void k_li_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps,
                          float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ISTA initialisation: WeT[a][i] = K[a][i]/L (We = K^T/L); ST = I - G/L with
// G = K^T K from a GEMM (symmetric, so its [j][i] layout is ST's); theta = lam/L
__global__ void k_li_init_we(const float* __restrict__ K, int64_t ldk, int64_t n, int64_t p, float* __restrict__ WeT,
                             int64_t pp, double invL) {
    const int64_t a = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x)
        WeT[a * pp + i] = a < n ? (float)((double)K[a * ldk + i] * invL) : 0.f;
}
// Gram: three partial planes of pp x pp, summed in double
__global__ void k_li_init_s(const float* __restrict__ Gram, int64_t pp, int64_t p, float* __restrict__ ST, double invL) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pp; i += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        if (i < p && j < p) {
            const int64_t idx = j * pp + i;
            const double g = (double)Gram[idx] + (double)Gram[pp * pp + idx] + (double)Gram[2 * pp * pp + idx];
            v = (float)((i == j ? 1.0 : 0.0) - g * invL);
        }
        ST[j * pp + i] = v;
    }
}
__global__ void k_li_fill(float* __restrict__ x, int64_t count, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) x[i] = v;
}

// per-sample projection of the network output (one workgroup per sample)
template <int NV>
__global__ __launch_bounds__(1024) void k_li_project(const float* __restrict__ X, int64_t ld, int64_t p,
                                                     const double* __restrict__ rho, float* __restrict__ out,
                                                     int64_t ldo) {
    __shared__ double lds[3 * (1024 / WAVE)];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    double vr[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * 1024 + tid) + (e & 1);
        vr[e] = j < p ? (double)X[b * ld + j] : 0.0;
    }
    double m, t;
    bool inside;
    int passes;
    const double rb = rho[b];
    l1_threshold_regs<1024, NV>(vr, p, rb, -1.0, lds, m, t, inside, passes);
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const int j = 2 * ((e / 2) * 1024 + tid) + (e & 1);
        if (j < p) out[b * ldo + j] = (float)l1_hval(vr[e], m, t, inside, rb);
    }
}

}  // namespace gpl1

namespace {

int64_t rup(int64_t a, int64_t m) { return (a + m - 1) / m * m; }
// reduction chunk for a padded Kd (multiple of 128): 1, 2 or 4 chunks, so
// the partial buffer never needs more than 4 output planes
int64_t kchunk_for(int64_t kd) {
    const int64_t S = kd <= 1024 ? 1 : kd <= 2048 ? 2 : 4;
    return kd / S;
}

// Cpart = A * Bplanes^T (see gp_gemm.hpp); M, N multiples of 128, Kd of 32
void gemm(hipStream_t s, const uint16_t* A, int64_t lda, int64_t M, const uint16_t* Bp, int64_t ldb, int64_t pstride,
          int64_t N, int64_t Kd, int64_t kchunk, float* C, int64_t ldc, int64_t cstride, int nsplit = 3) {
    const dim3 grid((unsigned)(M / GM_BM), (unsigned)(N / GM_BN), (unsigned)(Kd / kchunk));
    if (nsplit == 3)
        hipLaunchKernelGGL(k_gemm_bf16<3>, grid, dim3(GM_T), 0, s, A, lda, Bp, ldb, pstride, (int)kchunk, C, ldc, cstride, nullptr);
    else if (nsplit == 2)
        hipLaunchKernelGGL(k_gemm_bf16<2>, grid, dim3(GM_T), 0, s, A, lda, Bp, ldb, pstride, (int)kchunk, C, ldc, cstride, nullptr);
    else
        hipLaunchKernelGGL(k_gemm_bf16<1>, grid, dim3(GM_T), 0, s, A, lda, Bp, ldb, pstride, (int)kchunk, C, ldc, cstride, nullptr);
}

struct Act {
    int64_t bp;
    float *U, *X, *C, *dX, *dU, *dC, *part;
    uint16_t *Ypl, *YTpl, *Xpl, *dUpl, *dUT, *XT, *dCT;
    double *lpart, *tpart, *scal;
    int64_t part_elems;
};

int act_layout(gp_lista net, int64_t B, Act& a, bool alloc) {
    const int64_t pp = net->pp, np = net->np, L = net->L;
    const int64_t bp = rup(std::max<int64_t>(B, 1), LI_PAD);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = off; off += (bytes + 255) / 256 * 256; return o2; };
    const size_t fl = 4 * (size_t)bp * pp;
    const size_t oU = take(fl * L), oX = take(fl * L), oC = take(fl), odX = take(fl), odU = take(fl), odC = take(fl);
    const int64_t part_elems = std::max<int64_t>({4 * bp * pp, pp * pp, np * pp});
    const size_t opart = take(4 * (size_t)part_elems);
    const size_t oYpl = take(2 * 3 * (size_t)bp * np), oYTpl = take(2 * 3 * (size_t)np * bp);
    const size_t oXpl = take(2 * 3 * (size_t)bp * pp), odUpl = take(2 * 3 * (size_t)bp * pp);
    const int64_t kcat = std::max<int64_t>(1, (L - 1) * bp);
    const size_t odUT = take(2 * (size_t)pp * kcat), oXT = take(2 * 3 * (size_t)pp * kcat), odCT = take(2 * (size_t)pp * bp);
    const int64_t nblk = std::max<int64_t>((pp + 255) / 256 * bp, bp);   // partials of the elementwise kernels
    const size_t olp = take(8 * nblk), otp = take(8 * nblk * L), osc = take(8 * (L + 4));
    if (alloc) {
        if (bp != net->act_bp && off <= net->act_bytes) {
            // a new layout over the old buffer: padding rows and columns must read as zeros
            if (hipMemset(net->act, 0, net->act_bytes) != hipSuccess) return GP_E_HIP;
        }
        net->act_bp = bp;
        if (off > net->act_bytes) {
            if (net->act) (void)hipFree(net->act);
            net->act = nullptr;
            net->act_bytes = 0;
            if (hipMalloc(&net->act, off) != hipSuccess) { (void)hipGetLastError(); return GP_E_NOMEM; }
            net->act_bytes = off;
            if (hipMemset(net->act, 0, off) != hipSuccess) return GP_E_HIP;
        }
    }
    char* base = (char*)net->act;
    a.bp = bp;
    a.U = (float*)(base + oU); a.X = (float*)(base + oX); a.C = (float*)(base + oC);
    a.dX = (float*)(base + odX); a.dU = (float*)(base + odU); a.dC = (float*)(base + odC);
    a.part = (float*)(base + opart); a.part_elems = part_elems;
    a.Ypl = (uint16_t*)(base + oYpl); a.YTpl = (uint16_t*)(base + oYTpl); a.Xpl = (uint16_t*)(base + oXpl);
    a.dUpl = (uint16_t*)(base + odUpl); a.dUT = (uint16_t*)(base + odUT); a.XT = (uint16_t*)(base + oXT);
    a.dCT = (uint16_t*)(base + odCT);
    a.lpart = (double*)(base + olp); a.tpart = (double*)(base + otp); a.scal = (double*)(base + osc);
    return GP_OK_TOL;
}

void refresh_bf16(gp_lista net, hipStream_t s) {
    if (net->bf_valid) return;
    const int64_t pp = net->pp, np = net->np;
    // We_bf[i][a] = WeT[a][i]; S_bf[i][j] = ST[j][i]; St_bf = bf16(ST)
    hipLaunchKernelGGL(k_li_transpose_split, dim3((unsigned)(pp / 64), (unsigned)(np / 64)), dim3(256), 0, s,
                       net->WeT, pp, np, pp, net->We_bf, np, (int64_t)0, 1, (int64_t)0);
    hipLaunchKernelGGL(k_li_transpose_split, dim3((unsigned)(pp / 64), (unsigned)(pp / 64)), dim3(256), 0, s,
                       net->ST, pp, pp, pp, net->S_bf, pp, (int64_t)0, 1, (int64_t)0);
    hipLaunchKernelGGL(k_li_weights_bf16, dim3((unsigned)((pp * pp + 255) / 256)), dim3(256), 0, s, net->ST, pp,
                       net->St_bf);
    net->bf_valid = true;
}

// forward pass; keeps U, X of every layer in `a`
void forward(gp_lista net, const float* Y, int64_t ldy, int64_t B, Act& a, hipStream_t s, int planes = 3) {
    const int64_t pp = net->pp, np = net->np, bp = a.bp;
    const int64_t plY = bp * np, plX = bp * pp;
    refresh_bf16(net, s);
    hipLaunchKernelGGL(k_li_split_rows, dim3((unsigned)((np + 255) / 256), (unsigned)bp), dim3(256), 0, s, Y, ldy,
                       B, net->n, a.Ypl, np, plY);
    // c = We y
    const int64_t kc1 = kchunk_for(np);
    const int S1 = (int)(np / kc1);
    gemm(s, net->We_bf, np, pp, a.Ypl, np, plY, bp, np, kc1, a.part, pp, bp * pp, planes);
    const dim3 eg((unsigned)((pp + 255) / 256), (unsigned)bp);
    hipLaunchKernelGGL(k_li_fwd_act, eg, dim3(256), 0, s, a.part, S1, bp * pp, pp, B, net->p, a.C, 1, a.U, a.X,
                       net->th, 0, net->L > 1 ? a.Xpl : nullptr, plX);
    const int64_t kc2 = kchunk_for(pp);
    const int S2 = (int)(pp / kc2);
    for (int t = 1; t < net->L; ++t) {
        gemm(s, net->S_bf, pp, pp, a.Xpl, pp, plX, bp, pp, kc2, a.part, pp, bp * pp, planes);
        hipLaunchKernelGGL(k_li_fwd_act, eg, dim3(256), 0, s, a.part, S2, bp * pp, pp, B, net->p, a.C, 0,
                           a.U + t * bp * pp, a.X + t * bp * pp, net->th, t,
                           t + 1 < net->L ? a.Xpl : nullptr, plX);
    }
}

// loss, gradients into a.part-free buffers: returns loss; grads: gWeT (np x pp
// layout [a][i]), gST ([j][i]), gth[L] (device)
int backward(gp_lista net, const float* Y, int64_t ldy, const float* Xs, int64_t ldx, int64_t B, Act& a,
             float* gWeT, float* gST, float* gth, double* loss_host, hipStream_t s) {
    const int64_t pp = net->pp, np = net->np, bp = a.bp, L = net->L;
    const int64_t plX = bp * pp, kcat = std::max<int64_t>(1, (L - 1) * bp);
    const dim3 eg((unsigned)((pp + 255) / 256), (unsigned)bp);
    const int64_t nblk = (int64_t)eg.x * eg.y;
    hipLaunchKernelGGL(k_li_loss, eg, dim3(LI_T), 0, s, a.X + (L - 1) * bp * pp, pp, Xs, ldx, B, net->p, a.dX,
                       a.lpart);
    hipLaunchKernelGGL(k_li_reduce, dim3(1), dim3(LI_T), 0, s, a.lpart, nblk, a.scal);
    const int64_t kc2 = kchunk_for(pp);
    const int S2 = (int)(pp / kc2);
    for (int t = (int)L - 1; t >= 0; --t) {
        hipLaunchKernelGGL(k_li_bwd_act, eg, dim3(LI_T), 0, s, a.dX, a.U + t * bp * pp, pp, B, net->p, net->th, t,
                           a.dU, a.dC, t == L - 1 ? 1 : 0, t > 0 ? a.dUpl : nullptr, plX, a.tpart + t * nblk);
        if (t > 0) {
            // dU_t^T and x_{t-1}^T side by side for the gradient of S
            hipLaunchKernelGGL(k_li_transpose_split, dim3((unsigned)(pp / 64), (unsigned)(bp / 64)), dim3(256), 0, s,
                               a.dU, pp, B, net->p, a.dUT, kcat, (int64_t)0, 1, (int64_t)(t - 1) * bp);
            hipLaunchKernelGGL(k_li_transpose_split, dim3((unsigned)(pp / 64), (unsigned)(bp / 64)), dim3(256), 0, s,
                               a.X + (t - 1) * bp * pp, pp, B, net->p, a.XT, kcat, pp * kcat, 3,
                               (int64_t)(t - 1) * bp);
            // dx_{t-1} = S^T dU_t
            gemm(s, net->St_bf, pp, pp, a.dUpl, pp, plX, bp, pp, kc2, a.part, pp, bp * pp);
            hipLaunchKernelGGL(k_li_sum_parts, dim3((unsigned)((bp * pp + 255) / 256)), dim3(256), 0, s, a.part, S2,
                               bp * pp, bp * pp, a.dX);
        }
    }
    for (int t = 0; t < L; ++t)
        hipLaunchKernelGGL(k_li_reduce, dim3(1), dim3(LI_T), 0, s, a.tpart + t * nblk, nblk, a.scal + 1 + t);
    // gradient of S: [j][i] = sum over (t, b) dU_t[b][i] x_{t-1}[b][j]
    if (L > 1) {
        gemm(s, a.dUT, kcat, pp, a.XT, kcat, pp * kcat, pp, kcat, kcat, gST, pp, pp * pp);
    } else {
        (void)hipMemsetAsync(gST, 0, 4 * pp * pp, s);
    }
    // gradient of We: [a][i] = sum_b dC[b][i] y[b][a]
    hipLaunchKernelGGL(k_li_transpose_split, dim3((unsigned)(pp / 64), (unsigned)(bp / 64)), dim3(256), 0, s, a.dC,
                       pp, B, net->p, a.dCT, bp, (int64_t)0, 1, (int64_t)0);
    hipLaunchKernelGGL(k_li_transpose_split, dim3((unsigned)(np / 64), (unsigned)(bp / 64)), dim3(256), 0, s, Y, ldy,
                       B, net->n, a.YTpl, bp, np * bp, 3, (int64_t)0);
    gemm(s, a.dCT, bp, pp, a.YTpl, bp, np * bp, np, bp, bp, gWeT, pp, np * pp);
    std::vector<double> sc((size_t)(L + 1));
    hipError_t e = hipMemcpyAsync(sc.data(), a.scal, 8 * (L + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return GP_E_HIP;
    if (loss_host) *loss_host = 0.5 * sc[0] / (double)B;
    std::vector<float> gt((size_t)L);
    for (int t = 0; t < L; ++t) gt[(size_t)t] = (float)sc[(size_t)(1 + t)];
    e = hipMemcpyAsync(gth, gt.data(), 4 * L, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GP_OK_TOL : GP_E_HIP;
}

int check_batch(gp_lista net, int64_t B) {
    if (!net) return GP_E_ARG;
    if (B <= 0 || B > (1 << 16)) return fail(net->h, GP_E_ARG, "batch size must be in 1..65536");
    return GP_OK_TOL;
}

}  // namespace

extern "C" {

int gp_lista_create(gp_handle h, gp_lista* out, int64_t n, int64_t p, int32_t layers) {
    if (!h || !out) return GP_E_ARG;
    *out = nullptr;
    if (n <= 0 || p <= 0 || n > (1 << 16) || p > (1 << 16)) return fail(h, GP_E_ARG, "n, p must be in 1..65536");
    if (layers < 1 || layers > 32) return fail(h, GP_E_ARG, "layers must be in 1..32");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    gp_lista net = new (std::nothrow) gp_lista_s();
    if (!net) return GP_E_NOMEM;
    net->h = h;
    net->n = n; net->p = p; net->L = layers;
    net->np = rup(n, LI_PAD); net->pp = rup(p, LI_PAD);
    const int64_t np = net->np, pp = net->pp;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = off; off += (bytes + 255) / 256 * 256; return o2; };
    const size_t oW = take(4 * np * pp), oS = take(4 * pp * pp), oth = take(4 * 64);
    const size_t omW = take(4 * np * pp), ovW = take(4 * np * pp), omS = take(4 * pp * pp), ovS = take(4 * pp * pp);
    const size_t omt = take(4 * 64), ovt = take(4 * 64);
    const size_t oWb = take(2 * pp * np), oSb = take(2 * pp * pp), oStb = take(2 * pp * pp);
    const size_t ogW = take(4 * np * pp), ogS = take(4 * pp * pp), ogt = take(4 * 64);
    if (hipMalloc(&net->persist, off) != hipSuccess) { (void)hipGetLastError(); delete net; return GP_E_NOMEM; }
    if (hipMemset(net->persist, 0, off) != hipSuccess) { (void)hipFree(net->persist); delete net; return GP_E_HIP; }
    char* b = (char*)net->persist;
    net->WeT = (float*)(b + oW); net->ST = (float*)(b + oS); net->th = (float*)(b + oth);
    net->mWe = (float*)(b + omW); net->vWe = (float*)(b + ovW); net->mS = (float*)(b + omS); net->vS = (float*)(b + ovS);
    net->mth = (float*)(b + omt); net->vth = (float*)(b + ovt);
    net->We_bf = (uint16_t*)(b + oWb); net->S_bf = (uint16_t*)(b + oSb); net->St_bf = (uint16_t*)(b + oStb);
    net->gWeT = (float*)(b + ogW); net->gST = (float*)(b + ogS); net->gth = (float*)(b + ogt);
    *out = net;
    return GP_OK_TOL;
}

int gp_lista_destroy(gp_lista net) {
    if (!net) return GP_OK_TOL;
    (void)hipSetDevice(net->h->device);
    if (net->persist) (void)hipFree(net->persist);
    if (net->act) (void)hipFree(net->act);
    delete net;
    return GP_OK_TOL;
}

int gp_lista_init_from_K(gp_lista net, const float* K, int64_t ldk, double L, double lam, void* stream) {
    if (!net) return GP_E_ARG;
    gp_handle h = net->h;
    if (!K || ldk < net->p) return fail(h, GP_E_ARG, "K must be n x p with ldk >= p");
    if (!(L > 0.0) || !std::isfinite(L) || !(lam >= 0.0)) return fail(h, GP_E_ARG, "need L > 0 and lam >= 0");
    hipStream_t s = (hipStream_t)stream;
    const int64_t pp = net->pp, np = net->np;
    hipLaunchKernelGGL(k_li_init_we, dim3((unsigned)((pp + 255) / 256), (unsigned)np), dim3(256), 0, s, K, ldk,
                       net->n, net->p, net->WeT, pp, 1.0 / L);
    // Gram G = K^T K to FP32 accuracy: K^T as three bf16 planes h + m + l;
    // G = h (h + m + l) + m (h + m) + l h (the dropped products are below
    // 2^-24 relative), three GEMMs into three partial planes of one-time scratch
    const int64_t kpl = pp * np;
    void* scr = nullptr;
    if (hipMalloc(&scr, 2 * 3 * (size_t)kpl + 4 * 3 * (size_t)pp * pp) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, GP_E_NOMEM, "init scratch");
    }
    uint16_t* ktp = (uint16_t*)scr;
    float* G3 = (float*)(ktp + 3 * kpl);
    hipLaunchKernelGGL(k_li_transpose_split, dim3((unsigned)(pp / 64), (unsigned)(np / 64)), dim3(256), 0, s, K, ldk,
                       net->n, net->p, ktp, np, kpl, 3, (int64_t)0);
    for (int a = 0; a < 3; ++a)
        gemm(s, ktp + a * kpl, np, pp, ktp, np, kpl, pp, np, np, G3 + a * pp * pp, pp, pp * pp, 3 - a);
    hipLaunchKernelGGL(k_li_init_s, dim3((unsigned)((pp + 255) / 256), (unsigned)pp), dim3(256), 0, s, G3, pp,
                       net->p, net->ST, 1.0 / L);
    hipLaunchKernelGGL(k_li_fill, dim3(1), dim3(64), 0, s, net->th, (int64_t)net->L, (float)(lam / L));
    (void)hipMemsetAsync(net->mWe, 0, 4 * np * pp, s);
    (void)hipMemsetAsync(net->vWe, 0, 4 * np * pp, s);
    (void)hipMemsetAsync(net->mS, 0, 4 * pp * pp, s);
    (void)hipMemsetAsync(net->vS, 0, 4 * pp * pp, s);
    (void)hipMemsetAsync(net->mth, 0, 4 * 64, s);
    (void)hipMemsetAsync(net->vth, 0, 4 * 64, s);
    net->step = 0;
    net->bf_valid = false;
    hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(scr);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "network init");
    return GP_OK_TOL;
}

int gp_lista_set_weights(gp_lista net, const float* We, const float* S, const float* theta, void* stream) {
    if (!net || !We || !S || !theta) return GP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t pp = net->pp;
    // WeT[a][i] = We[i][a] (We is p x n), ST[j][i] = S[i][j]
    hipLaunchKernelGGL(k_li_transpose_f32, dim3((unsigned)((net->n + 255) / 256), (unsigned)net->p), dim3(256), 0, s,
                       We, net->n, net->p, net->n, net->WeT, pp);
    hipLaunchKernelGGL(k_li_transpose_f32, dim3((unsigned)((net->p + 255) / 256), (unsigned)net->p), dim3(256), 0, s,
                       S, net->p, net->p, net->p, net->ST, pp);
    hipError_t e = hipMemcpyAsync(net->th, theta, 4 * net->L, hipMemcpyDeviceToDevice, s);
    net->bf_valid = false;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GP_OK_TOL : hip_fail(net->h, e, "set weights");
}

int gp_lista_get_weights(gp_lista net, float* We, float* S, float* theta, void* stream) {
    if (!net || !We || !S || !theta) return GP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t pp = net->pp;
    // We[i][a] = WeT[a][i]: rows a < n, cols i < p of WeT -> dst (p x n, ld n)
    hipLaunchKernelGGL(k_li_transpose_f32, dim3((unsigned)((net->p + 255) / 256), (unsigned)net->n), dim3(256), 0, s,
                       net->WeT, pp, net->n, net->p, We, net->n);
    hipLaunchKernelGGL(k_li_transpose_f32, dim3((unsigned)((net->p + 255) / 256), (unsigned)net->p), dim3(256), 0, s,
                       net->ST, pp, net->p, net->p, S, net->p);
    hipError_t e = hipMemcpyAsync(theta, net->th, 4 * net->L, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GP_OK_TOL : hip_fail(net->h, e, "get weights");
}

int gp_lista_set_forward_planes(gp_lista net, int32_t planes) {
    if (!net) return GP_E_ARG;
    if (planes < 1 || planes > 3) return fail(net->h, GP_E_ARG, "planes must be 1, 2 or 3");
    net->fwd_planes = planes;
    return GP_OK_TOL;
}

int gp_lista_save(gp_lista net, const char* path) {
    if (!net) return GP_E_ARG;
    gp_handle h = net->h;
    if (!path) return fail(h, GP_E_ARG, "null path");
    const int64_t n = net->n, p = net->p, pp = net->pp;
    std::vector<float> W((size_t)(n * p)), S((size_t)(p * p)), th((size_t)net->L);
    hipError_t e = hipSetDevice(h->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy2D(W.data(), 4 * p, net->WeT, 4 * pp, 4 * p, n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy2D(S.data(), 4 * p, net->ST, 4 * pp, 4 * p, p, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(th.data(), net->th, 4 * net->L, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "weights to host");
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(h, GP_E_ARG, std::string("cannot open ") + path);
    const int32_t hdr32[2] = {net->L, 0};
    const int64_t hdr64[2] = {n, p};
    bool ok = std::fwrite("GPLISTA1", 1, 8, f) == 8 && std::fwrite(hdr64, 8, 2, f) == 2 &&
              std::fwrite(hdr32, 4, 2, f) == 2 && std::fwrite(W.data(), 4, W.size(), f) == W.size() &&
              std::fwrite(S.data(), 4, S.size(), f) == S.size() && std::fwrite(th.data(), 4, th.size(), f) == th.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? GP_OK_TOL : fail(h, GP_E_ARG, std::string("write failed: ") + path);
}

int gp_lista_load(gp_lista net, const char* path) {
    if (!net) return GP_E_ARG;
    gp_handle h = net->h;
    if (!path) return fail(h, GP_E_ARG, "null path");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(h, GP_E_ARG, std::string("cannot open ") + path);
    char tag[8];
    int64_t hdr64[2];
    int32_t hdr32[2];
    bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, "GPLISTA1", 8) == 0 &&
              std::fread(hdr64, 8, 2, f) == 2 && std::fread(hdr32, 4, 2, f) == 2;
    if (!ok || hdr64[0] != net->n || hdr64[1] != net->p || hdr32[0] != net->L) {
        std::fclose(f);
        return fail(h, GP_E_ARG, "not a network file of this shape");
    }
    const int64_t n = net->n, p = net->p, pp = net->pp;
    std::vector<float> W((size_t)(n * p)), S((size_t)(p * p)), th((size_t)net->L);
    ok = std::fread(W.data(), 4, W.size(), f) == W.size() && std::fread(S.data(), 4, S.size(), f) == S.size() &&
         std::fread(th.data(), 4, th.size(), f) == th.size();
    std::fclose(f);
    if (!ok) return fail(h, GP_E_ARG, "truncated network file");
    hipError_t e = hipSetDevice(h->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy2D(net->WeT, 4 * pp, W.data(), 4 * p, 4 * p, n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy2D(net->ST, 4 * pp, S.data(), 4 * p, 4 * p, p, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(net->th, th.data(), 4 * net->L, hipMemcpyHostToDevice);
    // a fresh Adam state
    const int64_t np = net->np;
    if (e == hipSuccess) e = hipMemset(net->mWe, 0, 4 * np * pp);
    if (e == hipSuccess) e = hipMemset(net->vWe, 0, 4 * np * pp);
    if (e == hipSuccess) e = hipMemset(net->mS, 0, 4 * pp * pp);
    if (e == hipSuccess) e = hipMemset(net->vS, 0, 4 * pp * pp);
    if (e == hipSuccess) e = hipMemset(net->mth, 0, 4 * 64);
    if (e == hipSuccess) e = hipMemset(net->vth, 0, 4 * 64);
    if (e != hipSuccess) return hip_fail(h, e, "weights to device");
    net->step = 0;
    net->bf_valid = false;
    return GP_OK_TOL;
}

int gp_lista_forward(gp_lista net, const float* Y, int64_t ldy, int64_t B, const double* rho, float* X_out,
                     int64_t ldx, void* stream) {
    int rc = check_batch(net, B);
    if (rc) return rc;
    gp_handle h = net->h;
    if (!Y || !X_out || ldy < net->n || ldx < net->p) return fail(h, GP_E_ARG, "bad Y / X_out");
    if (rho)
        for (int64_t b = 0; b < B; ++b)
            if (!(rho[b] >= 0.0) || !std::isfinite(rho[b])) return fail(h, GP_E_ARG, "rho must be finite and >= 0");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    // large batches run in slices of 1024 samples
    for (int64_t b0 = 0; b0 < B; b0 += 1024) {
        const int64_t bs = std::min<int64_t>(1024, B - b0);
        Act a;
        rc = act_layout(net, bs, a, true);
        if (rc) return fail(h, rc, "activation allocation failed");
        forward(net, Y + b0 * ldy, ldy, bs, a, s, net->fwd_planes);
        const float* XL = a.X + (int64_t)(net->L - 1) * a.bp * net->pp;
        if (rho) {
            std::vector<double> r((size_t)bs);
            for (int64_t b = 0; b < bs; ++b) r[(size_t)b] = rho[b0 + b];
            double* d_r = a.lpart;   // lpart holds at least bp >= bs doubles
            e = hipMemcpyAsync(d_r, r.data(), 8 * bs, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(h, e, "rho upload");
            const int64_t per = (net->p + 1023) / 1024;
            const int nv = per <= 2 ? 2 : per <= 4 ? 4 : per <= 8 ? 8 : per <= 16 ? 16 : 0;
            if (!nv) return fail(h, GP_E_UNSUPPORTED, "p too large for the projection of the network output");
            switch (nv) {
                case 2: hipLaunchKernelGGL(k_li_project<2>, dim3((unsigned)bs), dim3(1024), 0, s, XL, net->pp, net->p, d_r, X_out + b0 * ldx, ldx); break;
                case 4: hipLaunchKernelGGL(k_li_project<4>, dim3((unsigned)bs), dim3(1024), 0, s, XL, net->pp, net->p, d_r, X_out + b0 * ldx, ldx); break;
                case 8: hipLaunchKernelGGL(k_li_project<8>, dim3((unsigned)bs), dim3(1024), 0, s, XL, net->pp, net->p, d_r, X_out + b0 * ldx, ldx); break;
                case 16: hipLaunchKernelGGL(k_li_project<16>, dim3((unsigned)bs), dim3(1024), 0, s, XL, net->pp, net->p, d_r, X_out + b0 * ldx, ldx); break;
            }
        } else {
            e = hipMemcpy2DAsync(X_out + b0 * ldx, 4 * ldx, XL, 4 * net->pp, 4 * net->p, bs, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(h, e, "output copy");
        }
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "forward");
    }
    return GP_OK_TOL;
}

int gp_lista_gradients(gp_lista net, const float* Y, int64_t ldy, const float* Xstar, int64_t ldx, int64_t B,
                       float* dWe, float* dS, float* dtheta, double* loss_out, void* stream) {
    int rc = check_batch(net, B);
    if (rc) return rc;
    gp_handle h = net->h;
    if (B > 1024) return fail(h, GP_E_ARG, "gradients take at most 1024 samples per call");
    if (!Y || !Xstar || !dWe || !dS || !dtheta) return fail(h, GP_E_ARG, "null pointer");
    if (ldy < net->n || ldx < net->p) return fail(h, GP_E_ARG, "bad leading dimension");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    Act a;
    rc = act_layout(net, B, a, true);
    if (rc) return fail(h, rc, "activation allocation failed");
    const int64_t pp = net->pp;
    forward(net, Y, ldy, B, a, s);
    rc = backward(net, Y, ldy, Xstar, ldx, B, a, net->gWeT, net->gST, net->gth, loss_out, s);
    if (rc) return fail(h, rc, "gradient pass failed");
    hipLaunchKernelGGL(k_li_transpose_f32, dim3((unsigned)((net->p + 255) / 256), (unsigned)net->n), dim3(256), 0, s,
                       net->gWeT, pp, net->n, net->p, dWe, net->n);
    hipLaunchKernelGGL(k_li_transpose_f32, dim3((unsigned)((net->p + 255) / 256), (unsigned)net->p), dim3(256), 0, s,
                       net->gST, pp, net->p, net->p, dS, net->p);
    e = hipMemcpyAsync(dtheta, net->gth, 4 * net->L, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GP_OK_TOL : hip_fail(h, e, "gradient copy");
}

int gp_lista_train_step(gp_lista net, const float* Y, int64_t ldy, const float* Xstar, int64_t ldx, int64_t B,
                        double lr, double* loss_out, void* stream) {
    int rc = check_batch(net, B);
    if (rc) return rc;
    gp_handle h = net->h;
    if (B > 1024) return fail(h, GP_E_ARG, "a training step takes at most 1024 samples");
    if (!Y || !Xstar) return fail(h, GP_E_ARG, "null pointer");
    if (ldy < net->n || ldx < net->p) return fail(h, GP_E_ARG, "bad leading dimension");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(h, GP_E_ARG, "lr must be positive");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    Act a;
    rc = act_layout(net, B, a, true);
    if (rc) return fail(h, rc, "activation allocation failed");
    const int64_t pp = net->pp, np = net->np;
    forward(net, Y, ldy, B, a, s);
    rc = backward(net, Y, ldy, Xstar, ldx, B, a, net->gWeT, net->gST, net->gth, loss_out, s);
    if (rc) return fail(h, rc, "training step failed");
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)net->step), c2 = 1.f - powf(b2, (float)net->step);
    hipLaunchKernelGGL(k_li_adam, dim3((unsigned)((np * pp + 255) / 256)), dim3(256), 0, s, net->WeT, net->gWeT,
                       net->mWe, net->vWe, np * pp, (float)lr, b1, b2, eps, c1, c2);
    hipLaunchKernelGGL(k_li_adam, dim3((unsigned)((pp * pp + 255) / 256)), dim3(256), 0, s, net->ST, net->gST,
                       net->mS, net->vS, pp * pp, (float)lr, b1, b2, eps, c1, c2);
    hipLaunchKernelGGL(k_li_adam, dim3(1), dim3(64), 0, s, net->th, net->gth, net->mth, net->vth, (int64_t)net->L,
                       (float)lr, b1, b2, eps, c1, c2);
    net->bf_valid = false;
    e = hipStreamSynchronize(s);
    return e == hipSuccess ? GP_OK_TOL : hip_fail(h, e, "training step");
}

}  // extern "C"
