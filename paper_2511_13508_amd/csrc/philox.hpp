// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), usable from host and
// device code.  Key = (seed, stream tag), counter = four 64-bit words.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlpt {

// stream tags (second key word)
constexpr uint64_t kTagGraph = 0x4752415048ULL;  // "GRAPH"
constexpr uint64_t kTagInit = 0x494E4954ULL;     // "INIT"
constexpr uint64_t kTagPair = 0x50414952ULL;     // "PAIR"
constexpr uint64_t kTagMove = 0x4D4F5645ULL;     // "MOVE"
constexpr uint64_t kTagSwap = 0x53574150ULL;     // "SWAP"

struct Philox4 {
    uint64_t v[4];
};

__host__ __device__ inline uint64_t mul_hi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline Philox4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1) {
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL;
    constexpr uint64_t kMulB = 0xCA5A826395121157ULL;
    constexpr uint64_t kBumpA = 0x9E3779B97F4A7C15ULL;
    constexpr uint64_t kBumpB = 0xBB67AE8584CAA73BULL;
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
    for (int r = 0; r < 10; ++r) {
        const uint64_t hA = mul_hi64(kMulA, c0), lA = kMulA * c0;
        const uint64_t hB = mul_hi64(kMulB, c2), lB = kMulB * c2;
        const uint64_t n0 = hB ^ c1 ^ k0;
        const uint64_t n2 = hA ^ c3 ^ k1;
        c0 = n0;
        c1 = lB;
        c2 = n2;
        c3 = lA;
        k0 += kBumpA;
        k1 += kBumpB;
    }
    Philox4 out;
    out.v[0] = c0;
    out.v[1] = c1;
    out.v[2] = c2;
    out.v[3] = c3;
    return out;
}

// uniform in [0, 1): top 53 bits (double) or top 24 bits (float), exact.
template <typename R>
__host__ __device__ inline R uniform01(uint64_t w);
template <>
__host__ __device__ inline double uniform01<double>(uint64_t w) {
    return (double)(w >> 11) * 0x1.0p-53;
}
template <>
__host__ __device__ inline float uniform01<float>(uint64_t w) {
    return (float)(uint32_t)(w >> 40) * 0x1.0p-24f;
}

// index in [0, n) from the top 32 bits
__host__ __device__ inline int32_t index_below(uint64_t w, int32_t n) {
    return (int32_t)(((w >> 32) * (uint64_t)n) >> 32);
}

}  // namespace rlpt
