// Device helpers shared by the solver kernels: K element decoding, 16-byte
// vector loads, and deterministic wave / workgroup reductions for 64-wide
// CDNA wavefronts.
//
// Determinism: every reduction below combines values in a fixed order that
// does not depend on scheduling, so two runs on the same inputs give
// bit-identical scalars.  The symmetric lane pairings leave the same value in
// every lane because IEEE addition is commutative.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace gpl1 {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// K storage types.  bf16 is carried as raw uint16 bits.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };
// bf16 K whose rows are 8-byte but not 16-byte aligned, read four elements
// (8 bytes) per chunk so that a wave's loads stay contiguous
struct bf16x4_t { uint16_t bits; };

template <typename TK> struct KTraits;
template <> struct KTraits<double>   { using acc = double; static constexpr int VEC = 2; };
template <> struct KTraits<float>    { using acc = float;  static constexpr int VEC = 4; };
template <> struct KTraits<bf16_t>   { using acc = float;  static constexpr int VEC = 8; };
template <> struct KTraits<bf16x4_t> { using acc = float;  static constexpr int VEC = 4; };

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
    __device__ __forceinline__ void clear() { raw = make_uint4(0u, 0u, 0u, 0u); }
};
// An 8-byte chunk of four bf16 elements.
template <> struct KVec<bf16x4_t> {
    static constexpr int VEC = 4;
    uint2 raw;
    __device__ __forceinline__ float get(int e) const {
        const uint32_t w = (e >> 1) == 0 ? raw.x : raw.y;
        return (e & 1) ? __uint_as_float(w & 0xffff0000u) : __uint_as_float(w << 16);
    }
    __device__ __forceinline__ void clear() { raw = make_uint2(0u, 0u); }
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
    if constexpr (std::is_same<TK, bf16x4_t>::value) {
        // four bf16; ALIGNED: the row start is 8-byte aligned (ldk % 4 == 0)
        if (ALIGNED && col + 4 <= p) {
            out.raw = *reinterpret_cast<const uint2*>(rowp + col);
            return;
        }
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (col + e < p) {
                const uint32_t b = reinterpret_cast<const uint16_t*>(rowp)[col + e];
                w[e >> 1] |= (e & 1) ? (b << 16) : b;
            }
        }
        out.raw = make_uint2(w[0], w[1]);
    } else {
        constexpr int VEC = KTraits<TK>::VEC;
        if (ALIGNED && col + VEC <= p) {
            out.raw = *reinterpret_cast<const uint4*>(rowp + col);
            return;
        }
        if (!ALIGNED && col + VEC <= p) {
            // rows that are not 16-byte aligned: the widest loads the address
            // allows (the alignment is the row's, the same in every lane)
            const uintptr_t a = reinterpret_cast<uintptr_t>(rowp + col);
            if ((a & 7) == 0) {
                const uint2 lo = reinterpret_cast<const uint2*>(rowp + col)[0];
                const uint2 hi = reinterpret_cast<const uint2*>(rowp + col)[1];
                out.raw = make_uint4(lo.x, lo.y, hi.x, hi.y);
                return;
            }
            if ((a & 3) == 0) {
                const uint32_t* q = reinterpret_cast<const uint32_t*>(rowp + col);
                out.raw = make_uint4(q[0], q[1], q[2], q[3]);
                return;
            }
        }
        // ragged tail or 2-byte aligned rows: element loads, zero beyond p
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
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
// Wave reductions with DPP lane permutes (VALU, no LDS round trip):
// quad_perm xor 1 and xor 2, row_half_mirror and row_mirror leave the sum of
// each 16-lane row in all of its lanes; the four row sums are then read with
// v_readlane and added in a fixed order, so every lane holds the same total.
// Requires all 64 lanes active.
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7-i within 8
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15-i within 16

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = dpp_i<CTRL>(__double2loint(v));
    const int hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<DPP_XOR1>(v);
    v += dpp_d<DPP_XOR2>(v);
    v += dpp_d<DPP_HALF_MIRROR>(v);
    v += dpp_d<DPP_MIRROR>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<DPP_XOR1>(v);
    v += dpp_f<DPP_XOR2>(v);
    v += dpp_f<DPP_HALF_MIRROR>(v);
    v += dpp_f<DPP_MIRROR>(v);
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (a + b) + (c + d);
}
__device__ __forceinline__ int wave_sum(int v) {
    v += dpp_i<DPP_XOR1>(v);
    v += dpp_i<DPP_XOR2>(v);
    v += dpp_i<DPP_HALF_MIRROR>(v);
    v += dpp_i<DPP_MIRROR>(v);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<DPP_XOR1>(v));
    v = fmax(v, dpp_d<DPP_XOR2>(v));
    v = fmax(v, dpp_d<DPP_HALF_MIRROR>(v));
    v = fmax(v, dpp_d<DPP_MIRROR>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Sum (maximum) over groups of N neighbouring lanes, N in {1, 2, 4, 8, 16}:
// the first log2(N) steps of the wave_sum butterfly; every lane of a group
// holds the group's result.
template <int N>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "groups of 1 to 16 lanes");
    if (N > 1) v += dpp_d<DPP_XOR1>(v);
    if (N > 2) v += dpp_d<DPP_XOR2>(v);
    if (N > 4) v += dpp_d<DPP_HALF_MIRROR>(v);
    if (N > 8) v += dpp_d<DPP_MIRROR>(v);
    return v;
}
template <int N>
__device__ __forceinline__ double group_max(double v) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "groups of 1 to 16 lanes");
    if (N > 1) v = fmax(v, dpp_d<DPP_XOR1>(v));
    if (N > 2) v = fmax(v, dpp_d<DPP_XOR2>(v));
    if (N > 4) v = fmax(v, dpp_d<DPP_HALF_MIRROR>(v));
    if (N > 8) v = fmax(v, dpp_d<DPP_MIRROR>(v));
    return v;
}

// The workgroup reductions below post one value per wave into LDS and then
// combine the T/64 posts lane-parallel: lane l of every wave reads post
// l mod T/64 and a group butterfly over the first T/64 lanes forms the total,
// which lane 0 hands to the whole wave.  Every thread receives the same value.

// Workgroup sum of one double per thread.  `lds` holds T/64 doubles.
template <int T>
__device__ __forceinline__ double block_sum(double v, double* lds) {
    constexpr int NWV = T / WAVE;
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    return readlane_d(group_sum<NWV>(lds[lane & (NWV - 1)]), 0);
}

template <int T>
__device__ __forceinline__ double block_max(double v, double* lds) {
    constexpr int NWV = T / WAVE;
    v = wave_max(v);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    return readlane_d(group_max<NWV>(lds[lane & (NWV - 1)]), 0);
}

// NS sums and NM maxima in one pass (one LDS exchange).  `lds` holds
// (NS + NM) * T/64 doubles.
template <int T, int NS, int NM>
__device__ __forceinline__ void block_reduce(double (&s)[NS], double (&mx)[NM], double* lds) {
    constexpr int NWV = T / WAVE;
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
#pragma unroll
    for (int i = 0; i < NS; ++i) s[i] = wave_sum(s[i]);
#pragma unroll
    for (int i = 0; i < NM; ++i) mx[i] = wave_max(mx[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) lds[i * NWV + wid] = s[i];
#pragma unroll
        for (int i = 0; i < NM; ++i) lds[(NS + i) * NWV + wid] = mx[i];
    }
    __syncthreads();
    const int l = lane & (NWV - 1);
#pragma unroll
    for (int i = 0; i < NS; ++i) s[i] = readlane_d(group_sum<NWV>(lds[i * NWV + l]), 0);
#pragma unroll
    for (int i = 0; i < NM; ++i) mx[i] = readlane_d(group_max<NWV>(lds[(NS + i) * NWV + l]), 0);
}

// Number of lanes of the wave for which `pred` holds (the same in every
// lane).  Call from uniform control flow.
__device__ __forceinline__ int wave_count(bool pred) {
    return __builtin_popcountll(__builtin_amdgcn_ballot_w64(pred));
}

// Workgroup sum of (count, value) pairs for a loop of reductions with one
// barrier each.  `c` is a wave's count (the same in all its lanes, e.g. from
// wave_count), `v` a value per lane.  Successive calls alternate between two
// slot sets of `slots` (4 * T/64 doubles, used by nothing else), so a wave
// writing the slots of call k + 1 never meets a wave still reading those of
// call k - 1 (it passed call k's barrier first).
template <int T>
__device__ __forceinline__ void block_sum2_alt(int& c, double& v, double* slots, int parity) {
    constexpr int NWV = T / WAVE;
    // the count is formed here, not sunk into the posting lane's branch
    // (which would keep every ballot mask of the caller alive until then)
    asm volatile("" ::"s"(c));
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    double* sl = slots + (parity & 1) * 2 * NWV;
    if (lane == 0) { sl[2 * wid] = (double)c; sl[2 * wid + 1] = v; }
    __syncthreads();
    const int l = lane & (NWV - 1);
    const double2 cv = *reinterpret_cast<const double2*>(sl + 2 * l);
    c = (int)readlane_d(group_sum<NWV>(cv.x), 0);
    v = readlane_d(group_sum<NWV>(cv.y), 0);
}

}  // namespace gpl1
