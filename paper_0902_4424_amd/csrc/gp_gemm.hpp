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
// filled with zeros.  No bounds checks are needed inside.  With `nmap`, row
// n of the right operand and of the output is nmap[n] (so a grid over a list
// of columns reads and writes only those; the host pads the list to the tile
// size with the index of a zero row).
//
// Tiling: a 256-thread workgroup computes a 128 x 128 tile; its four waves
// each own a 64 x 64 sub-tile = 4 x 4 MFMA 16x16x32 blocks.  Each k-step of
// 32 stages the A tile and the NSPLIT B tiles in LDS (64-byte rows whose
// 16-byte chunks are XOR-swizzled by the row against bank conflicts; the
// other variants below pad rows to 40 elements instead), double buffered
// with one barrier per step; the next step's global loads are in registers
// while the current step's MFMAs run.
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
                                                    int64_t cstride, const int32_t* __restrict__ nmap) {
    static_assert(NSPLIT >= 1 && NSPLIT <= 3, "one to three bf16 planes");
    // staged tiles: rows of 32 elements (64 bytes) with the 16-byte chunk kc
    // of row r stored at chunk kc ^ ((r >> 2) & 3), so that the staging
    // stores of a wave (sixteen rows of four chunks) and the fragment reads
    // (sixteen rows, one chunk each) spread over the banks without padding
    constexpr int TILE = GM_BM * GM_BK;                    // elements of one staged tile
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
    const int64_t bn0_ = nmap ? nmap[n0 + row0_] : n0 + row0_;
    const int64_t bn1_ = nmap ? nmap[n0 + row1_] : n0 + row1_;
    const uint16_t* b0p = Bp + bn0_ * ldb + k_begin + kc0_;
    const uint16_t* b1p = Bp + bn1_ * ldb + k_begin + kc1_;
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
#define GPL1_ST(buf_, t_, row_, kc_, v_)                                                                       \
    (*reinterpret_cast<uint4*>(&lds[buf_][(t_) * TILE + (row_) * GM_BK + ((((kc_) >> 3) ^ (((row_) >> 2) & 3)) << 3)]) = \
         (v_))
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
    const int fks = ((fk >> 3) ^ ((fr >> 2) & 3)) << 3;   // its chunk in the swizzled rows
    for (int step = 0; step < nsteps; ++step) {
        const int cur = step & 1;
        if (step + 1 < nsteps) GPL1_GEMM_GLOAD(step + 1)
        bf16x8_t af[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8_t*>(&lds[cur][(wm * 64 + i * 16 + fr) * GM_BK + fks]);
#pragma unroll
        for (int t = 0; t < NSPLIT; ++t) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bf16x8_t bfr = *reinterpret_cast<const bf16x8_t*>(
                    &lds[cur][(1 + t) * TILE + (wn * 64 + j * 16 + fr) * GM_BK + fks]);
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
            const int64_t nl = n0 + wn * 64 + j * 16 + (lane & 15);
            const int64_t nn = nmap ? nmap[nl] : nl;
            *reinterpret_cast<float4*>(out + nn * ldc + m) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        }
#undef GPL1_GEMM_GLOAD
#undef GPL1_GEMM_LSTORE
#undef GPL1_LD
#undef GPL1_ST
}

// k_gemm_bf16 with the global loads issued two k-steps ahead: two sets of
// staging registers (S and T) alternate, so a step's tiles have about two
// steps of matrix-core work to arrive instead of one.  That is what a grid of
// one workgroup per CU needs when the operands come from the Infinity Cache
// rather than L2.  Same arguments, tiling and output as k_gemm_bf16.
template <int NSPLIT>
__global__ __launch_bounds__(GM_T) void k_gemm_bf16_d2(const uint16_t* __restrict__ A, int64_t lda,
                                                       const uint16_t* __restrict__ Bp, int64_t ldb,
                                                       int64_t pstride, int kchunk,
                                                       float* __restrict__ Cpart, int64_t ldc,
                                                       int64_t cstride, const int32_t* __restrict__ nmap) {
    static_assert(NSPLIT >= 1 && NSPLIT <= 3, "one to three bf16 planes");
    constexpr int TILE = GM_BM * GM_LDS_ROW;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][(1 + NSPLIT) * TILE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t m0 = (int64_t)blockIdx.x * GM_BM;
    const int64_t n0 = (int64_t)blockIdx.y * GM_BN;
    const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
    const int nsteps = kchunk / GM_BK;
    const int c0_ = tid, c1_ = tid + GM_T;
    const int row0_ = c0_ >> 2, kc0_ = (c0_ & 3) * 8, row1_ = c1_ >> 2, kc1_ = (c1_ & 3) * 8;
    const uint16_t* a0p = A + (m0 + row0_) * lda + k_begin + kc0_;
    const uint16_t* a1p = A + (m0 + row1_) * lda + k_begin + kc1_;
    const int64_t bn0_ = nmap ? nmap[n0 + row0_] : n0 + row0_;
    const int64_t bn1_ = nmap ? nmap[n0 + row1_] : n0 + row1_;
    const uint16_t* b0p = Bp + bn0_ * ldb + k_begin + kc0_;
    const uint16_t* b1p = Bp + bn1_ * ldb + k_begin + kc1_;
    // two staging sets, named one by one so that they stay in VGPRs
    uint4 Sa0, Sa1, Sb00, Sb01, Sb10, Sb11, Sb20, Sb21;
    uint4 Ta0, Ta1, Tb00, Tb01, Tb10, Tb11, Tb20, Tb21;
#define GPL1_D2_LD(p_, off_) (*reinterpret_cast<const uint4*>((p_) + (off_)))
#define GPL1_D2_GLOAD(X_, step_)                                                \
    {                                                                           \
        const int64_t ko_ = (int64_t)(step_) * GM_BK;                           \
        X_##a0 = GPL1_D2_LD(a0p, ko_);                                          \
        X_##a1 = GPL1_D2_LD(a1p, ko_);                                          \
        X_##b00 = GPL1_D2_LD(b0p, ko_);                                         \
        X_##b01 = GPL1_D2_LD(b1p, ko_);                                         \
        if constexpr (NSPLIT > 1) {                                             \
            X_##b10 = GPL1_D2_LD(b0p, pstride + ko_);                           \
            X_##b11 = GPL1_D2_LD(b1p, pstride + ko_);                           \
        }                                                                       \
        if constexpr (NSPLIT > 2) {                                             \
            X_##b20 = GPL1_D2_LD(b0p, 2 * pstride + ko_);                       \
            X_##b21 = GPL1_D2_LD(b1p, 2 * pstride + ko_);                       \
        }                                                                       \
    }
#define GPL1_D2_ST(buf_, t_, row_, kc_, v_) \
    (*reinterpret_cast<uint4*>(&lds[buf_][(t_) * TILE + (row_) * GM_LDS_ROW + (kc_)]) = (v_))
#define GPL1_D2_LSTORE(buf_, X_)                                                \
    {                                                                           \
        GPL1_D2_ST(buf_, 0, row0_, kc0_, X_##a0);                               \
        GPL1_D2_ST(buf_, 0, row1_, kc1_, X_##a1);                               \
        GPL1_D2_ST(buf_, 1, row0_, kc0_, X_##b00);                              \
        GPL1_D2_ST(buf_, 1, row1_, kc1_, X_##b01);                              \
        if constexpr (NSPLIT > 1) {                                             \
            GPL1_D2_ST(buf_, 2, row0_, kc0_, X_##b10);                          \
            GPL1_D2_ST(buf_, 2, row1_, kc1_, X_##b11);                          \
        }                                                                       \
        if constexpr (NSPLIT > 2) {                                             \
            GPL1_D2_ST(buf_, 3, row0_, kc0_, X_##b20);                          \
            GPL1_D2_ST(buf_, 3, row1_, kc1_, X_##b21);                          \
        }                                                                       \
    }
// one k-step: every fragment of the step is read from LDS first, then the
// 16 * NSPLIT MFMAs issue back to back (the scheduling barriers keep the
// compiler from interleaving reads and waits between them)
#define GPL1_D2_COMPUTE(buf_)                                                   \
    {                                                                           \
        bf16x8_t af[4], bfr[NSPLIT][4];                                         \
        _Pragma("unroll") for (int i = 0; i < 4; ++i)                           \
            af[i] = *reinterpret_cast<const bf16x8_t*>(&lds[buf_][(wm * 64 + i * 16 + fr) * GM_LDS_ROW + fk]); \
        _Pragma("unroll") for (int t = 0; t < NSPLIT; ++t)                      \
        _Pragma("unroll") for (int j = 0; j < 4; ++j)                           \
            bfr[t][j] = *reinterpret_cast<const bf16x8_t*>(                     \
                &lds[buf_][(1 + t) * TILE + (wn * 64 + j * 16 + fr) * GM_LDS_ROW + fk]); \
        __builtin_amdgcn_sched_group_barrier(0x100, 4 + 4 * NSPLIT, 0);         \
        _Pragma("unroll") for (int t = 0; t < NSPLIT; ++t)                      \
        _Pragma("unroll") for (int j = 0; j < 4; ++j)                           \
        _Pragma("unroll") for (int i = 0; i < 4; ++i)                           \
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[t][j], acc[i][j], 0, 0, 0); \
        __builtin_amdgcn_sched_group_barrier(0x008, 16 * NSPLIT, 0);            \
    }

    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    // Every load is issued unconditionally (steps past the end re-read the
    // last one), so the count of loads in flight is the same on every path
    // and the wait before storing one set leaves the other set in flight.
    const int last = nsteps - 1;
    GPL1_D2_GLOAD(S, 0)
    GPL1_D2_LSTORE(0, S)
    GPL1_D2_GLOAD(S, 1 < last ? 1 : last)
    GPL1_D2_GLOAD(T, 2 < last ? 2 : last)
    __syncthreads();
    // buffer 0 holds even steps, buffer 1 odd ones; S carries odd steps, T even ones
    for (int step = 0; step < nsteps; step += 2) {
        GPL1_D2_COMPUTE(0)
        if (step + 1 >= nsteps) break;
        GPL1_D2_LSTORE(1, S)
        __syncthreads();
        GPL1_D2_GLOAD(S, step + 3 < last ? step + 3 : last)
        GPL1_D2_COMPUTE(1)
        if (step + 2 >= nsteps) break;
        GPL1_D2_LSTORE(0, T)
        __syncthreads();
        GPL1_D2_GLOAD(T, step + 4 < last ? step + 4 : last)
    }
    float* out = Cpart + (int64_t)blockIdx.z * cstride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t m = m0 + wm * 64 + i * 16 + (lane >> 4) * 4;
            const int64_t nl = n0 + wn * 64 + j * 16 + (lane & 15);
            const int64_t nn = nmap ? nmap[nl] : nl;
            *reinterpret_cast<float4*>(out + nn * ldc + m) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        }
#undef GPL1_D2_GLOAD
#undef GPL1_D2_LSTORE
#undef GPL1_D2_LD
#undef GPL1_D2_ST
#undef GPL1_D2_COMPUTE
}

// Both operands as bf16 planes: A = sum_a A_a (NA planes, stride apstride),
// B = sum_t B_t (NB planes), and only the plane products with a + t < NB are
// formed: for NA = NB = 3 that is A_h (B_h + B_m + B_l) + A_m (B_h + B_m) +
// A_l B_h, an FP32-accurate product of two FP32 matrices (the dropped plane
// products are below 2^-24 of the result) in one pass that stages every
// plane once.  Same tiling, padding rules and output layout as k_gemm_bf16.
// LDS holds the (NA + NB) tiles of one k-step (48 KiB for 3 + 3, so two
// workgroups fit a CU); the next step waits in registers, two barriers a step.
template <int NA, int NB>
__global__ __launch_bounds__(GM_T) void k_gemm_bf16_planes(const uint16_t* __restrict__ A, int64_t lda,
                                                           int64_t apstride, const uint16_t* __restrict__ Bp,
                                                           int64_t ldb, int64_t bpstride, int kchunk,
                                                           float* __restrict__ Cpart, int64_t ldc,
                                                           int64_t cstride, const int32_t* __restrict__ nmap) {
    static_assert(NA >= 1 && NA <= 3 && NB >= 1 && NB <= 3 && NA <= NB, "one to three planes each");
    constexpr int TILE = GM_BM * GM_BK;   // swizzled 64-byte rows, as in k_gemm_bf16
    constexpr int NT = NA + NB;
    __shared__ __attribute__((aligned(16))) uint16_t lds[1][NT * TILE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t m0 = (int64_t)blockIdx.x * GM_BM;
    const int64_t n0 = (int64_t)blockIdx.y * GM_BN;
    const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
    const int nsteps = kchunk / GM_BK;

    // two 16-byte chunks per thread per tile (rows row0_/row1_, k offsets kc0_/kc1_)
    const int c0_ = tid, c1_ = tid + GM_T;
    const int row0_ = c0_ >> 2, kc0_ = (c0_ & 3) * 8, row1_ = c1_ >> 2, kc1_ = (c1_ & 3) * 8;
    const uint16_t* a0p = A + (m0 + row0_) * lda + k_begin + kc0_;
    const uint16_t* a1p = A + (m0 + row1_) * lda + k_begin + kc1_;
    const int64_t bn0_ = nmap ? nmap[n0 + row0_] : n0 + row0_;
    const int64_t bn1_ = nmap ? nmap[n0 + row1_] : n0 + row1_;
    const uint16_t* b0p = Bp + bn0_ * ldb + k_begin + kc0_;
    const uint16_t* b1p = Bp + bn1_ * ldb + k_begin + kc1_;
    // staging registers for the next k-step (its loads are in flight while
    // the current step is multiplied), named one by one so that they stay in
    // VGPRs
    uint4 r0a00, r0a01, r0a10, r0a11, r0a20, r0a21, r0b00, r0b01, r0b10, r0b11, r0b20, r0b21;
#define GPL1_PL_LD(p_, off_) (*reinterpret_cast<const uint4*>((p_) + (off_)))
#define GPL1_PL_GLOAD(S_, step_)                                                \
    {                                                                           \
        const int64_t ko_ = (int64_t)(step_) * GM_BK;                           \
        S_##a00 = GPL1_PL_LD(a0p, ko_);                                         \
        S_##a01 = GPL1_PL_LD(a1p, ko_);                                         \
        if constexpr (NA > 1) {                                                 \
            S_##a10 = GPL1_PL_LD(a0p, apstride + ko_);                          \
            S_##a11 = GPL1_PL_LD(a1p, apstride + ko_);                          \
        }                                                                       \
        if constexpr (NA > 2) {                                                 \
            S_##a20 = GPL1_PL_LD(a0p, 2 * apstride + ko_);                      \
            S_##a21 = GPL1_PL_LD(a1p, 2 * apstride + ko_);                      \
        }                                                                       \
        S_##b00 = GPL1_PL_LD(b0p, ko_);                                         \
        S_##b01 = GPL1_PL_LD(b1p, ko_);                                         \
        if constexpr (NB > 1) {                                                 \
            S_##b10 = GPL1_PL_LD(b0p, bpstride + ko_);                          \
            S_##b11 = GPL1_PL_LD(b1p, bpstride + ko_);                          \
        }                                                                       \
        if constexpr (NB > 2) {                                                 \
            S_##b20 = GPL1_PL_LD(b0p, 2 * bpstride + ko_);                      \
            S_##b21 = GPL1_PL_LD(b1p, 2 * bpstride + ko_);                      \
        }                                                                       \
    }
#define GPL1_PL_ST(u_, row_, kc_, v_)                                                                          \
    (*reinterpret_cast<uint4*>(&lds[0][(u_) * TILE + (row_) * GM_BK + ((((kc_) >> 3) ^ (((row_) >> 2) & 3)) << 3)]) = \
         (v_))
#define GPL1_PL_LSTORE(S_)                                                      \
    {                                                                           \
        GPL1_PL_ST(0, row0_, kc0_, S_##a00);                                    \
        GPL1_PL_ST(0, row1_, kc1_, S_##a01);                                    \
        if constexpr (NA > 1) {                                                 \
            GPL1_PL_ST(1, row0_, kc0_, S_##a10);                                \
            GPL1_PL_ST(1, row1_, kc1_, S_##a11);                                \
        }                                                                       \
        if constexpr (NA > 2) {                                                 \
            GPL1_PL_ST(2, row0_, kc0_, S_##a20);                                \
            GPL1_PL_ST(2, row1_, kc1_, S_##a21);                                \
        }                                                                       \
        GPL1_PL_ST(NA, row0_, kc0_, S_##b00);                                   \
        GPL1_PL_ST(NA, row1_, kc1_, S_##b01);                                   \
        if constexpr (NB > 1) {                                                 \
            GPL1_PL_ST(NA + 1, row0_, kc0_, S_##b10);                           \
            GPL1_PL_ST(NA + 1, row1_, kc1_, S_##b11);                           \
        }                                                                       \
        if constexpr (NB > 2) {                                                 \
            GPL1_PL_ST(NA + 2, row0_, kc0_, S_##b20);                           \
            GPL1_PL_ST(NA + 2, row1_, kc1_, S_##b21);                           \
        }                                                                       \
    }
    // one k-step on the tiles in LDS
#define GPL1_PL_COMPUTE()                                                       \
    {                                                                           \
        _Pragma("unroll") for (int a = 0; a < NA; ++a) {                        \
            bf16x8_t af[4];                                                     \
            _Pragma("unroll") for (int i = 0; i < 4; ++i)                       \
                af[i] = *reinterpret_cast<const bf16x8_t*>(                     \
                    &lds[0][a * TILE + (wm * 64 + i * 16 + fr) * GM_BK + fks]); \
            _Pragma("unroll") for (int t = 0; t + a < NB; ++t)                  \
            _Pragma("unroll") for (int j = 0; j < 4; ++j) {                     \
                const bf16x8_t bfr = *reinterpret_cast<const bf16x8_t*>(        \
                    &lds[0][(NA + t) * TILE + (wn * 64 + j * 16 + fr) * GM_BK + fks]); \
                _Pragma("unroll") for (int i = 0; i < 4; ++i)                   \
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr, acc[i][j], 0, 0, 0); \
            }                                                                   \
        }                                                                       \
    }

    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int fks = ((fk >> 3) ^ ((fr >> 2) & 3)) << 3;   // its chunk in the swizzled rows
    GPL1_PL_GLOAD(r0, 0)
    GPL1_PL_LSTORE(r0)
    __syncthreads();
    for (int step = 0; step < nsteps; ++step) {
        if (step + 1 < nsteps) GPL1_PL_GLOAD(r0, step + 1)
        GPL1_PL_COMPUTE()
        if (step + 1 < nsteps) {
            __syncthreads();          // every wave is done reading this step's tiles
            GPL1_PL_LSTORE(r0)
            __syncthreads();
        }
    }
    float* out = Cpart + (int64_t)blockIdx.z * cstride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t m = m0 + wm * 64 + i * 16 + (lane >> 4) * 4;
            const int64_t nl = n0 + wn * 64 + j * 16 + (lane & 15);
            const int64_t nn = nmap ? nmap[nl] : nl;
            *reinterpret_cast<float4*>(out + nn * ldc + m) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        }
#undef GPL1_PL_GLOAD
#undef GPL1_PL_LSTORE
#undef GPL1_PL_LD
#undef GPL1_PL_ST
#undef GPL1_PL_COMPUTE
}

}  // namespace gpl1

namespace gpl1 {

// k_gemm_bf16 with 256-row tiles: 512 threads, eight waves (four along M,
// two along N, each the 64 x 64 sub-tile of k_gemm_bf16 with the same
// accumulation order, so the results are bitwise those of k_gemm_bf16 for the
// same kchunk).  Each staged B tile serves twice the rows, which cuts the
// bytes a workgroup fetches per matrix-core operation by about 1.6 times (the
// three B planes are most of them); a grid needs about half the kchunk of
// k_gemm_bf16 to fill the chip.  M need not be a multiple of 256: the rows of
// the last tile past M read row M - 1 and are not stored.
constexpr int GM2_T = 512, GM2_BM = 256;
template <int NSPLIT>
__global__ __launch_bounds__(GM2_T) void k_gemm_bf16_m256(const uint16_t* __restrict__ A, int64_t lda,
                                                         const uint16_t* __restrict__ Bp, int64_t ldb,
                                                         int64_t pstride, int kchunk,
                                                         float* __restrict__ Cpart, int64_t ldc,
                                                         int64_t cstride, const int32_t* __restrict__ nmap,
                                                         int64_t M) {
    static_assert(NSPLIT >= 1 && NSPLIT <= 3, "one to three bf16 planes");
    constexpr int TA = GM2_BM * GM_LDS_ROW, TB = GM_BN * GM_LDS_ROW;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][TA + NSPLIT * TB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 3, wn = wave >> 2;
    const int64_t m0 = (int64_t)blockIdx.x * GM2_BM;
    const int64_t n0 = (int64_t)blockIdx.y * GM_BN;
    const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
    const int nsteps = kchunk / GM_BK;
    // staging: the A tile is 256 rows x 4 chunks of 8 (two per thread), each
    // B plane 128 rows x 4 chunks (one per thread)
    const int rowA0 = tid >> 2, rowA1 = (tid + GM2_T) >> 2, kc_ = (tid & 3) * 8;
    const int rowB = tid >> 2;
    const int64_t ga0 = m0 + rowA0 < M ? m0 + rowA0 : M - 1;
    const int64_t ga1 = m0 + rowA1 < M ? m0 + rowA1 : M - 1;
    const uint16_t* a0p = A + ga0 * lda + k_begin + kc_;
    const uint16_t* a1p = A + ga1 * lda + k_begin + kc_;
    const int64_t bn = nmap ? nmap[n0 + rowB] : n0 + rowB;
    const uint16_t* bp = Bp + bn * ldb + k_begin + kc_;
    uint4 ra0, ra1, rb0, rb1, rb2;
#define GPL1_M2_LD(p_, off_) (*reinterpret_cast<const uint4*>((p_) + (off_)))
#define GPL1_M2_GLOAD(step_)                                                    \
    {                                                                           \
        const int64_t ko_ = (int64_t)(step_) * GM_BK;                           \
        ra0 = GPL1_M2_LD(a0p, ko_);                                             \
        ra1 = GPL1_M2_LD(a1p, ko_);                                             \
        rb0 = GPL1_M2_LD(bp, ko_);                                              \
        if constexpr (NSPLIT > 1) rb1 = GPL1_M2_LD(bp, pstride + ko_);          \
        if constexpr (NSPLIT > 2) rb2 = GPL1_M2_LD(bp, 2 * pstride + ko_);      \
    }
#define GPL1_M2_ST(buf_, off_, v_) (*reinterpret_cast<uint4*>(&lds[buf_][(off_)]) = (v_))
#define GPL1_M2_LSTORE(buf_)                                                    \
    {                                                                           \
        GPL1_M2_ST(buf_, rowA0 * GM_LDS_ROW + kc_, ra0);                        \
        GPL1_M2_ST(buf_, rowA1 * GM_LDS_ROW + kc_, ra1);                        \
        GPL1_M2_ST(buf_, TA + rowB * GM_LDS_ROW + kc_, rb0);                    \
        if constexpr (NSPLIT > 1) GPL1_M2_ST(buf_, TA + TB + rowB * GM_LDS_ROW + kc_, rb1);       \
        if constexpr (NSPLIT > 2) GPL1_M2_ST(buf_, TA + 2 * TB + rowB * GM_LDS_ROW + kc_, rb2);   \
    }
    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    GPL1_M2_GLOAD(0)
    GPL1_M2_LSTORE(0)
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int step = 0; step < nsteps; ++step) {
        const int cur = step & 1;
        if (step + 1 < nsteps) GPL1_M2_GLOAD(step + 1)
        bf16x8_t af[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8_t*>(&lds[cur][(wm * 64 + i * 16 + fr) * GM_LDS_ROW + fk]);
#pragma unroll
        for (int t = 0; t < NSPLIT; ++t) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bf16x8_t bfr = *reinterpret_cast<const bf16x8_t*>(
                    &lds[cur][TA + t * TB + (wn * 64 + j * 16 + fr) * GM_LDS_ROW + fk]);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr, acc[i][j], 0, 0, 0);
            }
        }
        if (step + 1 < nsteps) {
            GPL1_M2_LSTORE(cur ^ 1)
            __syncthreads();
        }
    }
    float* out = Cpart + (int64_t)blockIdx.z * cstride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t m = m0 + wm * 64 + i * 16 + (lane >> 4) * 4;
            const int64_t nl = n0 + wn * 64 + j * 16 + (lane & 15);
            const int64_t nn = nmap ? nmap[nl] : nl;
            if (m < M)
                *reinterpret_cast<float4*>(out + nn * ldc + m) =
                    make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        }
#undef GPL1_M2_GLOAD
#undef GPL1_M2_LSTORE
#undef GPL1_M2_LD
#undef GPL1_M2_ST
}

// k_gemm_bf16 with 64-column tiles, for a right operand of at most one
// 128-column tile (the last problems of a batch): twice the workgroups, each
// with half the work, where the 128-column grid would leave half the chip
// idle.  Four waves of 64 x 32 sub-tiles (4 x 2 MFMA blocks); every output
// element sees the same MFMAs in the same order as in k_gemm_bf16 (k-steps in
// turn, planes in turn within a step), so the results are bitwise those of
// k_gemm_bf16 for the same kchunk.  Same arguments; N (the column list) is
// padded to 64.
constexpr int GM3_BN = 64;
template <int NSPLIT>
__global__ __launch_bounds__(GM_T) void k_gemm_bf16_n64(const uint16_t* __restrict__ A, int64_t lda,
                                                        const uint16_t* __restrict__ Bp, int64_t ldb,
                                                        int64_t pstride, int kchunk,
                                                        float* __restrict__ Cpart, int64_t ldc,
                                                        int64_t cstride, const int32_t* __restrict__ nmap) {
    static_assert(NSPLIT >= 1 && NSPLIT <= 3, "one to three bf16 planes");
    constexpr int TA = GM_BM * GM_BK, TB = GM3_BN * GM_BK;   // swizzled rows, as in k_gemm_bf16
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][TA + NSPLIT * TB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t m0 = (int64_t)blockIdx.x * GM_BM;
    const int64_t n0 = (int64_t)blockIdx.y * GM3_BN;
    const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
    const int nsteps = kchunk / GM_BK;
    // staging: the A tile is 128 rows x 4 chunks of 8 (two per thread), each
    // B plane 64 rows x 4 chunks (one per thread)
    const int rowA0 = tid >> 2, rowA1 = (tid + GM_T) >> 2, kc_ = (tid & 3) * 8;
    const int rowB = tid >> 2;
    const uint16_t* a0p = A + (m0 + rowA0) * lda + k_begin + kc_;
    const uint16_t* a1p = A + (m0 + rowA1) * lda + k_begin + kc_;
    const int64_t bn = nmap ? nmap[n0 + rowB] : n0 + rowB;
    const uint16_t* bp = Bp + bn * ldb + k_begin + kc_;
    uint4 ra0, ra1, rb0, rb1, rb2;
#define GPL1_N3_LD(p_, off_) (*reinterpret_cast<const uint4*>((p_) + (off_)))
#define GPL1_N3_GLOAD(step_)                                                    \
    {                                                                           \
        const int64_t ko_ = (int64_t)(step_) * GM_BK;                           \
        ra0 = GPL1_N3_LD(a0p, ko_);                                             \
        ra1 = GPL1_N3_LD(a1p, ko_);                                             \
        rb0 = GPL1_N3_LD(bp, ko_);                                              \
        if constexpr (NSPLIT > 1) rb1 = GPL1_N3_LD(bp, pstride + ko_);          \
        if constexpr (NSPLIT > 2) rb2 = GPL1_N3_LD(bp, 2 * pstride + ko_);      \
    }
#define GPL1_N3_SWZ(row_) ((row_) * GM_BK + ((((kc_) >> 3) ^ (((row_) >> 2) & 3)) << 3))
#define GPL1_N3_ST(buf_, off_, v_) (*reinterpret_cast<uint4*>(&lds[buf_][(off_)]) = (v_))
#define GPL1_N3_LSTORE(buf_)                                                    \
    {                                                                           \
        GPL1_N3_ST(buf_, GPL1_N3_SWZ(rowA0), ra0);                              \
        GPL1_N3_ST(buf_, GPL1_N3_SWZ(rowA1), ra1);                              \
        GPL1_N3_ST(buf_, TA + GPL1_N3_SWZ(rowB), rb0);                          \
        if constexpr (NSPLIT > 1) GPL1_N3_ST(buf_, TA + TB + GPL1_N3_SWZ(rowB), rb1);             \
        if constexpr (NSPLIT > 2) GPL1_N3_ST(buf_, TA + 2 * TB + GPL1_N3_SWZ(rowB), rb2);         \
    }
    f32x4_t acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    GPL1_N3_GLOAD(0)
    GPL1_N3_LSTORE(0)
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int fks = ((fk >> 3) ^ ((fr >> 2) & 3)) << 3;   // its chunk in the swizzled rows
    for (int step = 0; step < nsteps; ++step) {
        const int cur = step & 1;
        if (step + 1 < nsteps) GPL1_N3_GLOAD(step + 1)
        bf16x8_t af[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8_t*>(&lds[cur][(wm * 64 + i * 16 + fr) * GM_BK + fks]);
#pragma unroll
        for (int t = 0; t < NSPLIT; ++t) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const bf16x8_t bfr = *reinterpret_cast<const bf16x8_t*>(
                    &lds[cur][TA + t * TB + (wn * 32 + j * 16 + fr) * GM_BK + fks]);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr, acc[i][j], 0, 0, 0);
            }
        }
        if (step + 1 < nsteps) {
            GPL1_N3_LSTORE(cur ^ 1)
            __syncthreads();
        }
    }
    float* out = Cpart + (int64_t)blockIdx.z * cstride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t m = m0 + wm * 64 + i * 16 + (lane >> 4) * 4;
            const int64_t nl = n0 + wn * 32 + j * 16 + (lane & 15);
            const int64_t nn = nmap ? nmap[nl] : nl;
            *reinterpret_cast<float4*>(out + nn * ldc + m) =
                make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        }
#undef GPL1_N3_GLOAD
#undef GPL1_N3_LSTORE
#undef GPL1_N3_LD
#undef GPL1_N3_ST
#undef GPL1_N3_SWZ
}

}  // namespace gpl1
