// Definitions the kernels see (limits, descriptors, complex types, the exact
// bucket arithmetic).  Host-only state lives in mr1l_internal.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mr1l {

// ---------------------------------------------------------------- limits
constexpr int kMaxL = 64;          // lattices per function (singleton masks: two uint32 words)
constexpr int kMaxD = 64;          // lattice dimensions
__host__ __device__ constexpr int mask_words(int L) { return (L + 31) >> 5; }   // uint32 words per mask
constexpr int kMaxCap = 8192;      // detected-list capacity per function
constexpr int kFftThreads = 1024;  // threads of a DFT workgroup
constexpr int kLdsBytes = 163840;  // LDS of one gfx950 workgroup
constexpr int kTabTw = 256;        // LDS twiddles of the four-step sub-transforms
constexpr int kTabCh = 384;        // LDS two-level chirp table entries of the four-step

// Largest transform held whole in LDS (re and im planes).
template <typename T> constexpr int lds_max_n() { return kLdsBytes / (2 * (int)sizeof(T)); }

// ---------------------------------------------------------------- descriptors
// One lattice (f, l) of the batch.
struct LatDesc {
    int64_t node_off;   // O_{f,l}
    int32_t M;          // prime lattice size
    int32_t mid;        // index of the distinct-size tables (MDesc)
    int32_t func;       // function f
    float inv_m;        // 1/M rounded down (fast modulo)
    uint32_t off32;     // multiple of M added before the fast modulo
    int64_t z_off;      // offset of z_{f,l} in the z tables
};

// Tables shared by every lattice of one size M, for the DFT schedule in use.
struct MDesc {
    int64_t spec_off;   // kernel spectrum (N complex) in the spectrum table
    int64_t chirp_off;  // two-level chirp table e^{-pi i r / M}, r < 2M
    int32_t chirp_shift;// log2 of the low table size S
    int32_t chirp_nlo;  // S
    int64_t tw_N;       // twiddle table e^{-2 pi i m / N}, m < N
    int32_t N;          // Bluestein length >= 2M - 1
    int32_t N1, N2;     // four-step split N = N1 N2 (N2 == 1: whole transform in LDS)
};

// ---------------------------------------------------------------- complex
template <typename T> struct cplx { T x, y; };
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };

// ---------------------------------------------------------------- exact hash
// Fast path: valid when every |k_u| <= kb (host-proved bound per function):
// sum_u k_u z_u fits int32, every product fits the 24-bit multiplier, and the
// float-reciprocal quotient of (s + off32) / M is exact or one too small.
__device__ __forceinline__ uint32_t fast_mod(uint32_t s, uint32_t m, float inv_m)
{
    uint32_t q = (uint32_t)((float)s * inv_m);
    uint32_t r = s - __umul24(q, m);
    return r >= m ? r - m : r;
}

// Exact bucket of any int64 frequency (coordinates strided by `stride`).
__device__ __forceinline__ int32_t exact_bucket(const int64_t *k, int64_t stride, int d,
                                                const int64_t *z, int64_t m)
{
    int64_t acc = 0;
    for (int u = 0; u < d; ++u) {
        int64_t ku = k[(int64_t)u * stride] % m;       // |ku| < m
        if (ku < 0) ku += m;
        acc = (acc + (ku * z[u]) % m) % m;            // ku, z < m < 2^23
    }
    return (int32_t)acc;
}

}  // namespace mr1l
