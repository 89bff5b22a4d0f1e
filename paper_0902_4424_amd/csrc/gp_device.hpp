// Device helpers shared by the solver kernels: K element decoding, 16-byte
// vector loads, and deterministic wave / workgroup reductions for 64-wide
// CDNA wavefronts.
//
// Determinism: every reduction below combines values in a fixed order that
// does not depend on scheduling, so two runs on the same inputs give
// bit-identical scalars.  The xor butterfly leaves the same value in every
// lane because IEEE addition is commutative.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpl1 {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// K storage types.  bf16 is carried as raw uint16 bits.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };

template <typename TK> struct KTraits;
template <> struct KTraits<double> { using acc = double; static constexpr int VEC = 2; };
template <> struct KTraits<float>  { using acc = float;  static constexpr int VEC = 4; };
template <> struct KTraits<bf16_t> { using acc = float;  static constexpr int VEC = 8; };

__device__ __forceinline__ float bf16_to_float(uint32_t bits16) {
    return __uint_as_float(bits16 << 16);
}

template <typename TK, typename ACC>
__device__ __forceinline__ ACC load_elem(const TK* p);
template <> __device__ __forceinline__ double load_elem<double, double>(const double* p) { return *p; }
template <> __device__ __forceinline__ float load_elem<float, float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float load_elem<bf16_t, float>(const bf16_t* p) {
    return bf16_to_float(reinterpret_cast<const uint16_t*>(p)[0]);
}

// A 16-byte chunk of one row of K, decoded to the accumulation type.
template <typename TK> struct KVec {
    using ACC = typename KTraits<TK>::acc;
    static constexpr int VEC = KTraits<TK>::VEC;
    uint4 raw;
    __device__ __forceinline__ ACC get(int e) const;
};
template <> __device__ __forceinline__ double KVec<double>::get(int e) const {
    uint32_t lo = e == 0 ? raw.x : raw.z;
    uint32_t hi = e == 0 ? raw.y : raw.w;
    return __hiloint2double((int)hi, (int)lo);
}
template <> __device__ __forceinline__ float KVec<float>::get(int e) const {
    uint32_t w = e == 0 ? raw.x : e == 1 ? raw.y : e == 2 ? raw.z : raw.w;
    return __uint_as_float(w);
}
template <> __device__ __forceinline__ float KVec<bf16_t>::get(int e) const {
    uint32_t w = (e >> 1) == 0 ? raw.x : (e >> 1) == 1 ? raw.y : (e >> 1) == 2 ? raw.z : raw.w;
    return (e & 1) ? __uint_as_float(w & 0xffff0000u) : __uint_as_float(w << 16);
}

// Load VEC consecutive elements K[row][col .. col+VEC) into `out`.
// ALIGNED: the row start is 16-byte aligned (ldk % VEC == 0, base aligned);
// then a full chunk is one 16-byte load.  Elements at col >= p read as 0.
template <typename TK, bool ALIGNED>
__device__ __forceinline__ void load_kvec(const TK* rowp, int64_t col, int64_t p, KVec<TK>& out) {
    constexpr int VEC = KTraits<TK>::VEC;
    if (ALIGNED && col + VEC <= p) {
        out.raw = *reinterpret_cast<const uint4*>(rowp + col);
        return;
    }
    // ragged tail or unaligned rows: element loads, zero beyond p
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    const int esz = (int)sizeof(TK);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        if (col + e < p) {
            if (esz == 8) {
                uint64_t b = reinterpret_cast<const uint64_t*>(rowp)[col + e];
                w[e * 2] = (uint32_t)b;
                w[e * 2 + 1] = (uint32_t)(b >> 32);
            } else if (esz == 4) {
                w[e] = reinterpret_cast<const uint32_t*>(rowp)[col + e];
            } else {
                uint32_t b = reinterpret_cast<const uint16_t*>(rowp)[col + e];
                w[e >> 1] |= (e & 1) ? (b << 16) : b;
            }
        }
    }
    out.raw = make_uint4(w[0], w[1], w[2], w[3]);
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) v = fmax(v, __shfl_xor(v, m, WAVE));
    return v;
}

// Workgroup sum of one double per thread.  `lds` holds T/64 doubles.  Every
// thread receives the same value (wave partials added in wave order).
template <int T>
__device__ __forceinline__ double block_sum(double v, double* lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < T / WAVE; ++i) s += lds[i];
    return s;
}

template <int T>
__device__ __forceinline__ double block_max(double v, double* lds) {
    v = wave_max(v);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = lds[0];
#pragma unroll
    for (int i = 1; i < T / WAVE; ++i) s = fmax(s, lds[i]);
    return s;
}

// Sum of (count, value) pairs in one pass (two LDS slots per wave).
template <int T>
__device__ __forceinline__ void block_sum2(int& c, double& v, double* lds) {
    c = wave_sum(c);
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) { lds[2 * wid] = (double)c; lds[2 * wid + 1] = v; }
    __syncthreads();
    double cs = 0.0, vs = 0.0;
#pragma unroll
    for (int i = 0; i < T / WAVE; ++i) { cs += lds[2 * i]; vs += lds[2 * i + 1]; }
    c = (int)cs;
    v = vs;
}

}  // namespace gpl1
