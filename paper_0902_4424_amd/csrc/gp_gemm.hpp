// bf16 MFMA GEMM for the batched (shared K) solver on gfx950.
//
//   Cpart[s][j][i] = sum_{k in chunk s} A[i][k] * (sum_t Bt[t][j][k])
//
// A is M x Kd bf16, row-major (k contiguous).  The right operand is given as
// NSPLIT planes, each N x Kd bf16 with k contiguous per column j; their sum
// represents an FP32 matrix to about 8 * NSPLIT bits (x = hi + mid + lo, each
// part rounded to bf16 from the remainder), and every bf16 x bf16 product is
// exact in the FP32 accumulator, so the result carries FP32-level accuracy
// while running on the bf16 matrix cores.  The reduction dimension is split
// into chunks of `kchunk` (grid.z); each chunk writes FP32 partial sums that
// the caller adds in double.
//
// Shapes are padded by the host: M and N multiples of 128, Kd and kchunk
// multiples of 32, leading dimensions multiples of 8 (16-byte rows), padding
// filled with zeros.  No bounds checks are needed inside.
//
// Tiling: a 256-thread workgroup computes a 128 x 128 tile; its four waves
// each own a 64 x 64 sub-tile = 4 x 4 MFMA 16x16x32 blocks.  Each k-step of
// 32 stages the A tile and the NSPLIT B tiles in LDS (rows padded to 40
// elements against bank conflicts), double buffered with one barrier per
// step; the next step's global loads are in registers while the current
// step's MFMAs run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpl1 {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int GM_BM = 128, GM_BN = 128, GM_BK = 32, GM_LDS_ROW = 40, GM_T = 256;

template <int NSPLIT>
__global__ __launch_bounds__(GM_T) void k_gemm_bf16(const uint16_t* __restrict__ A, int64_t lda,
                                                    const uint16_t* __restrict__ Bp, int64_t ldb,
                                                    int64_t pstride, int kchunk,
                                                    float* __restrict__ Cpart, int64_t ldc,
                                                    int64_t cstride) {
    static_assert(NSPLIT >= 1 && NSPLIT <= 3, "one to three bf16 planes");
    constexpr int TILE = GM_BM * GM_LDS_ROW;               // elements of one staged tile
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][(1 + NSPLIT) * TILE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t m0 = (int64_t)blockIdx.x * GM_BM;
    const int64_t n0 = (int64_t)blockIdx.y * GM_BN;
    const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
    const int nsteps = kchunk / GM_BK;

    // global -> register staging: each tile is 128 rows x 4 chunks of 8
    // elements = 512 chunks, two per thread
    // (written out without loops so that the staging values stay in registers)
    uint4 ra0, ra1, rb00, rb01, rb10, rb11, rb20, rb21;
    const int c0_ = tid, c1_ = tid + GM_T;
    const int row0_ = c0_ >> 2, kc0_ = (c0_ & 3) * 8, row1_ = c1_ >> 2, kc1_ = (c1_ & 3) * 8;
    const uint16_t* a0p = A + (m0 + row0_) * lda + k_begin + kc0_;
    const uint16_t* a1p = A + (m0 + row1_) * lda + k_begin + kc1_;
    const uint16_t* b0p = Bp + (n0 + row0_) * ldb + k_begin + kc0_;
    const uint16_t* b1p = Bp + (n0 + row1_) * ldb + k_begin + kc1_;
#define GPL1_LD(p_, off_) (*reinterpret_cast<const uint4*>((p_) + (off_)))
#define GPL1_GEMM_GLOAD(step_)                                                  \
    {                                                                           \
        const int64_t ko_ = (int64_t)(step_) * GM_BK;                           \
        ra0 = GPL1_LD(a0p, ko_);                                                \
        ra1 = GPL1_LD(a1p, ko_);                                                \
        rb00 = GPL1_LD(b0p, ko_);                                               \
        rb01 = GPL1_LD(b1p, ko_);                                               \
        if constexpr (NSPLIT > 1) {                                             \
            rb10 = GPL1_LD(b0p, pstride + ko_);                                 \
            rb11 = GPL1_LD(b1p, pstride + ko_);                                 \
        }                                                                       \
        if constexpr (NSPLIT > 2) {                                             \
            rb20 = GPL1_LD(b0p, 2 * pstride + ko_);                             \
            rb21 = GPL1_LD(b1p, 2 * pstride + ko_);                             \
        }                                                                       \
    }
#define GPL1_ST(buf_, t_, row_, kc_, v_) \
    (*reinterpret_cast<uint4*>(&lds[buf_][(t_) * TILE + (row_) * GM_LDS_ROW + (kc_)]) = (v_))
#define GPL1_GEMM_LSTORE(buf_)                                                  \
    {                                                                           \
        GPL1_ST(buf_, 0, row0_, kc0_, ra0);                                     \
        GPL1_ST(buf_, 0, row1_, kc1_, ra1);                                     \
        GPL1_ST(buf_, 1, row0_, kc0_, rb00);                                    \
        GPL1_ST(buf_, 1, row1_, kc1_, rb01);                                    \
        if constexpr (NSPLIT > 1) {                                             \
            GPL1_ST(buf_, 2, row0_, kc0_, rb10);                                \
            GPL1_ST(buf_, 2, row1_, kc1_, rb11);                                \
        }                                                                       \
        if constexpr (NSPLIT > 2) {                                             \
            GPL1_ST(buf_, 3, row0_, kc0_, rb20);                                \
            GPL1_ST(buf_, 3, row1_, kc1_, rb21);                                \
        }                                                                       \
    }

    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    GPL1_GEMM_GLOAD(0)
    GPL1_GEMM_LSTORE(0)
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;   // fragment row/col and k offset of this lane
    for (int step = 0; step < nsteps; ++step) {
        const int cur = step & 1;
        if (step + 1 < nsteps) GPL1_GEMM_GLOAD(step + 1)
        bf16x8_t af[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8_t*>(&lds[cur][(wm * 64 + i * 16 + fr) * GM_LDS_ROW + fk]);
#pragma unroll
        for (int t = 0; t < NSPLIT; ++t) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bf16x8_t bfr = *reinterpret_cast<const bf16x8_t*>(
                    &lds[cur][(1 + t) * TILE + (wn * 64 + j * 16 + fr) * GM_LDS_ROW + fk]);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr, acc[i][j], 0, 0, 0);
            }
        }
        if (step + 1 < nsteps) {
            GPL1_GEMM_LSTORE(cur ^ 1)
            __syncthreads();
        }
    }
    // lane holds C[m = (lane/16)*4 + r][n = lane%16] of each 16x16 block:
    // four consecutive m of one column -> one 16-byte store into [j][i]
    float* out = Cpart + (int64_t)blockIdx.z * cstride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t m = m0 + wm * 64 + i * 16 + (lane >> 4) * 4;
            const int64_t nn = n0 + wn * 64 + j * 16 + (lane & 15);
            *reinterpret_cast<float4*>(out + nn * ldc + m) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        }
#undef GPL1_GEMM_GLOAD
#undef GPL1_GEMM_LSTORE
#undef GPL1_LD
#undef GPL1_ST
}

}  // namespace gpl1
