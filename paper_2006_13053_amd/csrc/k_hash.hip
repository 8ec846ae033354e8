// Candidate hashing, the non-zero vote and bucket occupancy.
//
// Bucket of candidate k in lattice l (Section 2.2, rearrangement step of
// Algorithm 1; non-negative representative of Section 2.1):
//     h_l(k) = (sum_u k_u z_{l,u}) mod M_l.
// Vote of Algorithms 1/2 with the threshold test of Remark 2.3 (the
// non-zero bitmap comes from the DFT epilogue):
//     v(k) = #{l : bitmap bit O_l + h_l(k) set},  k detected iff v(k) >= vote_min.
//
// The candidate stream is structure-of-arrays int64 (one coalesced 8-byte
// column per coordinate) and is read exactly once.  Exactness: when every
// |k_u| <= kb_f (a per-function bound the host derives from d and the
// lattice sizes) the dot product is formed with 24-bit multiply-adds in
// 32-bit integers, offset by a multiple of M to make it non-negative, and
// reduced with a float reciprocal whose quotient is provably exact or one
// too small; any other candidate takes the exact 64-bit path.  Both give
// the same bucket.
#include "mr1l_internal.h"

namespace mr1l {

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return MR1L_OK;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

int launch_fill_bytes(void *p, int64_t nbytes, hipStream_t s)
{
    // all library buffers are 4-byte multiples
    return launch_fill_u32(reinterpret_cast<uint32_t *>(p), nbytes / 4, 0u, s);
}

// ------------------------------------------------------------------ helpers
// Function owning global candidate index i (set_off ascending, F + 1 entries).
__device__ __forceinline__ int func_of(const int64_t *set_off, int F, int64_t i)
{
    int lo = 0, hi = F;   // set_off[lo] <= i < set_off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (set_off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ vote
constexpr int kVoteThreads = 512;
constexpr int kVoteCPT = 1;                   // candidates per thread
constexpr int kVoteLdsWords = 20480;          // 80 KiB: two workgroups per CU

// Each workgroup owns a contiguous, tile-aligned range of the concatenated
// candidate sets; the current function's bitmap words sit in LDS (reloaded at
// function boundaries).  Thread t of a tile handles candidates 2t and 2t + 1.
template <int D, bool LDSB, int CPT, bool DOT2>
__global__ __launch_bounds__(kVoteThreads) void k_vote(
    const int64_t *__restrict__ freq, int64_t n_total, const int64_t *__restrict__ set_off, int F,
    int L, int d_rt, const LatDesc *__restrict__ lat, const int32_t *__restrict__ z32,
    const int64_t *__restrict__ z64, const uint32_t *__restrict__ vrec, int rs, const int32_t *__restrict__ kbound,
    const uint32_t *__restrict__ bitmap, int vote_min, int64_t cap,
    int64_t *__restrict__ det_cnt, int64_t *__restrict__ det_idx, uint8_t *__restrict__ votes, int aligned)
{
    const int d = D > 0 ? D : d_rt;
    constexpr int DM = D > 0 ? D : kMaxD;
    extern __shared__ __align__(16) uint32_t bits[];
    __shared__ int s_f;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    constexpr int TILE = kVoteThreads * CPT;
    const int64_t ntiles = (n_total + TILE - 1) / TILE;
    const int64_t tper = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * tper * TILE;
    const int64_t end = min(n_total, beg + tper * TILE);
    const bool want_votes = votes != nullptr;
    int cur_f = -1;
    int64_t f_lo = 0, f_hi = 0;
    int64_t word0 = 0;

    for (int64_t t0 = beg; t0 < end; t0 += TILE) {
        const int64_t tend = min(end, t0 + TILE);
        int64_t seg = t0;
        while (seg < tend) {
            if (!(seg >= f_lo && seg < f_hi)) {
                if (tid == 0) s_f = func_of(set_off, F, seg);
                __syncthreads();
                cur_f = s_f;
                __syncthreads();   // s_f is rewritten at the next function change
                f_lo = set_off[cur_f];
                f_hi = set_off[cur_f + 1];
                const LatDesc l0 = lat[cur_f * L];
                const LatDesc lL = lat[cur_f * L + L - 1];
                word0 = l0.node_off >> 5;
                if (LDSB) {
                    const int64_t wN = ((lL.node_off + lL.M - 1) >> 5) - word0 + 1;
                    for (int64_t w = tid; w < wN; w += kVoteThreads) bits[w] = bitmap[word0 + w];
                    __syncthreads();
                }
            }
            if (f_hi <= seg) break;   // inconsistent offsets: stop instead of spinning
            const int64_t sEnd = min(tend, f_hi);
            const int f = __builtin_amdgcn_readfirstlane(cur_f);
            const int64_t c0 = t0 + CPT * tid;
            bool val[CPT];
            int32_t lo[CPT][DM];
            bool fast[CPT];
            const int32_t kb = kbound[f];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                val[c] = (c0 + c >= seg) && (c0 + c < sEnd);
                fast[c] = true;
            }
            // coalesced loads of the thread's candidates, one column per coordinate
#pragma unroll
            for (int u = 0; u < DM; ++u) {
                if (u < d) {
                    const int64_t *row = freq + (int64_t)u * n_total;
                    int64_t k[CPT];
                    if constexpr (CPT == 2) {
                        if (aligned && val[0] && val[1]) {
                            const longlong2 vv = *reinterpret_cast<const longlong2 *>(row + c0);
                            k[0] = vv.x;
                            k[1] = vv.y;
                        } else {
                            k[0] = val[0] ? row[c0] : 0;
                            k[1] = val[1] ? row[c0 + 1] : 0;
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < CPT; ++c) k[c] = val[c] ? __builtin_nontemporal_load(row + c0 + c) : 0;
                    }
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        lo[c][u] = (int32_t)k[c];
                        fast[c] = fast[c] && (k[c] >= -kb) && (k[c] <= kb);
                    }
                }
            }
            int v[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) v[c] = 0;
            const LatDesc *lf = lat + f * L;
            // fast path for candidates within the 24-bit bound (all but adversarial inputs)
            bool act[CPT], any = false;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                act[c] = val[c] && fast[c];
                any = any || act[c];
            }
            if (__any(any)) {   // wave-uniform, so the record loads stay scalar
                // one contiguous record per lattice (wave-uniform); the next record is
                // loaded while the current lattice is hashed (record L is a padding copy)
                constexpr int ZW = DOT2 ? (DM + 1) / 2 : DM;
                const int zw = DOT2 ? (d + 1) / 2 : d;
                // constant address space: uniform loads of the read-only records go through
                // the scalar cache
                typedef const __attribute__((address_space(4))) uint32_t *crec_t;
                crec_t rec = (crec_t)(uintptr_t)(vrec + (int64_t)f * (L + 1) * rs);
                uint32_t kp[CPT][(DM + 1) / 2];
                if constexpr (DOT2) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c)
#pragma unroll
                        for (int j = 0; j < (DM + 1) / 2; ++j) {
                            const uint32_t a = (2 * j < d) ? ((uint32_t)lo[c][2 * j] & 0xffffu) : 0u;
                            const uint32_t b = (2 * j + 1 < d) ? ((uint32_t)lo[c][2 * j + 1] << 16) : 0u;
                            kp[c][j] = a | b;
                        }
                }
                uint32_t zc[ZW + 4];
#pragma unroll
                for (int u = 0; u < ZW; ++u) zc[u] = (u < zw) ? rec[u] : 0u;
#pragma unroll
                for (int u = 0; u < 4; ++u) zc[ZW + u] = rec[zw + u];
                for (int l = 0; l < L; ++l) {
                    rec += rs;
                    uint32_t zn[ZW + 4];
#pragma unroll
                    for (int u = 0; u < ZW; ++u) zn[u] = (u < zw) ? rec[u] : 0u;
#pragma unroll
                    for (int u = 0; u < 4; ++u) zn[ZW + u] = rec[zw + u];
                    const uint32_t off32 = zc[ZW], Mm = zc[ZW + 1], bbase = zc[ZW + 3];
                    const float inv_m = __uint_as_float(zc[ZW + 2]);
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        uint32_t s = off32;
                        if constexpr (DOT2) {
                            typedef short v2s __attribute__((ext_vector_type(2)));
#pragma unroll
                            for (int j = 0; j < ZW; ++j)
                                if (j < zw)
                                    s = (uint32_t)__builtin_amdgcn_sdot2(__builtin_bit_cast(v2s, kp[c][j]),
                                                                         __builtin_bit_cast(v2s, zc[j]), (int)s,
                                                                         false);
                        } else {
#pragma unroll
                            for (int u = 0; u < DM; ++u)
                                if (u < d) s += (uint32_t)__mul24(lo[c][u], (int32_t)zc[u]);
                        }
                        const uint32_t g = bbase + fast_mod(s, Mm, inv_m);
                        uint32_t word;
                        if constexpr (LDSB) word = bits[g >> 5];
                        else word = bitmap[word0 + (g >> 5)];
                        // bit g mod 32 (the extract uses the low five bits of the offset)
                        v[c] += act[c] ? (int)__builtin_amdgcn_ubfe(word, g, 1) : 0;
                    }
#pragma unroll
                    for (int u = 0; u < ZW + 4; ++u) zc[u] = zn[u];
                    if (!want_votes && l >= L - vote_min) {
                        // leave once every candidate of the wave has reached vote_min or can no longer
                        // (no candidate can be hopeless before lattice L - vote_min)
                        const int rest = L - 1 - l;
                        bool decided = true;
#pragma unroll
                        for (int c = 0; c < CPT; ++c)
                            decided = decided && (!act[c] || v[c] >= vote_min || v[c] + rest < vote_min);
                        if (__all(decided)) break;
                    }
                }
            }
            // exact 64-bit path for candidates beyond the bound (rare, divergent)
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                if (val[c] && !fast[c]) {
                    for (int l = 0; l < L; ++l) {
                        const LatDesc ld = lf[l];
                        const int32_t h = exact_bucket(freq + c0 + c, n_total, d, z64 + ld.z_off, ld.M);
                        const int64_t g = ld.node_off + h;
                        uint32_t word;
                        if constexpr (LDSB) word = bits[(g >> 5) - word0];
                        else word = bitmap[g >> 5];
                        v[c] += (word >> (g & 31)) & 1u;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                if (want_votes && val[c]) votes[c0 + c] = (uint8_t)v[c];
                const bool det = val[c] && v[c] >= vote_min;
                const uint64_t bal = __ballot(det);
                if (bal) {
                    const int cnt = __popcll(bal);
                    const int first = __ffsll((unsigned long long)bal) - 1;
                    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
                    unsigned long long base = 0;
                    if (lane == first)
                        base = atomicAdd((unsigned long long *)(det_cnt + f), (unsigned long long)cnt);
                    base = __shfl(base, first);
                    if (det && (int64_t)(base + rank) < cap) det_idx[f * cap + base + rank] = c0 + c - f_lo;
                }
            }
            seg = sEnd;
        }
    }
}

#define MR1L_VOTE_LAUNCH(Dv, LD, D2)                                                                 \
    hipLaunchKernelGGL((k_vote<Dv, LD, kVoteCPT, D2>), grid, blk, LD ? shm : 0, p.stream, freq, n_total,  \
                       set_off, p.F, p.L, p.d, p.d_lat, p.d_z32, p.d_z64, p.d_vrec, p.vrec_stride, p.d_kb, bitmap,         \
                       vote_min, cap, n_det, det_idx, votes, aligned)
#define MR1L_VOTE_DISPATCH(Dv)                                          \
    case Dv:                                                            \
        if (lds) {                                                      \
            if (p.dot2) MR1L_VOTE_LAUNCH(Dv, true, true);               \
            else MR1L_VOTE_LAUNCH(Dv, true, false);                     \
        } else {                                                        \
            if (p.dot2) MR1L_VOTE_LAUNCH(Dv, false, true);              \
            else MR1L_VOTE_LAUNCH(Dv, false, false);                    \
        }                                                               \
        break;

int vote_init_attrs()
{
#define MR1L_VOTE_ATTR(Dv)                                                                        \
    MR1L_HIP(hipFuncSetAttribute((const void *)k_vote<Dv, true, kVoteCPT, true>,                       \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kVoteLdsWords * 4));      \
    MR1L_HIP(hipFuncSetAttribute((const void *)k_vote<Dv, true, kVoteCPT, false>,                      \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kVoteLdsWords * 4));
    MR1L_VOTE_ATTR(0) MR1L_VOTE_ATTR(1) MR1L_VOTE_ATTR(2) MR1L_VOTE_ATTR(3) MR1L_VOTE_ATTR(4)
    MR1L_VOTE_ATTR(5) MR1L_VOTE_ATTR(6) MR1L_VOTE_ATTR(7) MR1L_VOTE_ATTR(8) MR1L_VOTE_ATTR(9)
    MR1L_VOTE_ATTR(10) MR1L_VOTE_ATTR(12) MR1L_VOTE_ATTR(16) MR1L_VOTE_ATTR(20) MR1L_VOTE_ATTR(25)
    MR1L_VOTE_ATTR(30)
#undef MR1L_VOTE_ATTR
    return MR1L_OK;
}

int vote_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq,
             const uint32_t *bitmap, int32_t vote_min, int64_t cap, int64_t *n_det, int64_t *det_idx,
             uint8_t *votes)
{
    // n_det is zero-filled by the caller (outside the timed vote stage)
    if (n_total <= 0) return MR1L_OK;
    // LDS bitmap when every function's lattice bits fit
    int64_t maxw = 0;
    for (int f = 0; f < p.F; ++f) {
        const LatDesc &a = p.lat[(size_t)f * p.L], &b = p.lat[(size_t)f * p.L + p.L - 1];
        maxw = std::max<int64_t>(maxw, ((b.node_off + b.M - 1) >> 5) - (a.node_off >> 5) + 1);
    }
    const bool lds = maxw <= kVoteLdsWords;
    const size_t shm = lds ? (size_t)maxw * 4 : 0;
    const int aligned = ((reinterpret_cast<uintptr_t>(freq) & 15) == 0 && (n_total & 1) == 0) ? 1 : 0;
    const int64_t tiles = (n_total + kVoteThreads * kVoteCPT - 1) / (kVoteThreads * kVoteCPT);
    // one co-resident workgroup per slot: no partial second round of workgroups
    int per_cu = 0;
    const void *kfn = lds ? (const void *)k_vote<10, true, kVoteCPT, true> : (const void *)k_vote<10, false, kVoteCPT, true>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kVoteThreads, shm) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int64_t gridn = std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)num_cus() * per_cu));
    dim3 grid((unsigned)gridn), blk(kVoteThreads);
    switch (p.d) {
        MR1L_VOTE_DISPATCH(1)
        MR1L_VOTE_DISPATCH(2)
        MR1L_VOTE_DISPATCH(3)
        MR1L_VOTE_DISPATCH(4)
        MR1L_VOTE_DISPATCH(5)
        MR1L_VOTE_DISPATCH(6)
        MR1L_VOTE_DISPATCH(7)
        MR1L_VOTE_DISPATCH(8)
        MR1L_VOTE_DISPATCH(9)
        MR1L_VOTE_DISPATCH(10)
        MR1L_VOTE_DISPATCH(12)
        MR1L_VOTE_DISPATCH(16)
        MR1L_VOTE_DISPATCH(20)
        MR1L_VOTE_DISPATCH(25)
        MR1L_VOTE_DISPATCH(30)
    default:
        MR1L_VOTE_DISPATCH(0)
    }
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

// ------------------------------------------------------------------ hash + count
// hash[l * n_total + i] and counts[O_{f,l} + h] over a candidate set; counts is
// zero-filled first and accumulated with global atomics (order-independent).
__global__ __launch_bounds__(256) void k_hash_count(
    const int64_t *__restrict__ freq, int64_t n_total, const int64_t *__restrict__ set_off, int F, int L,
    int d, const LatDesc *__restrict__ lat, const int32_t *__restrict__ z32, const int64_t *__restrict__ z64,
    const int32_t *__restrict__ kbound, int32_t *__restrict__ hash, int32_t *__restrict__ counts)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int f = func_of(set_off, F, i);
        const int32_t kb = kbound[f];
        int32_t lo[kMaxD];
        bool fast = true;
        for (int u = 0; u < d; ++u) {
            const int64_t k = freq[(int64_t)u * n_total + i];
            lo[u] = (int32_t)k;
            fast = fast && (k >= -kb) && (k <= kb);
        }
        for (int l = 0; l < L; ++l) {
            const LatDesc ld = lat[f * L + l];
            int32_t h;
            if (fast) {
                uint32_t s = ld.off32;
                for (int u = 0; u < d; ++u) s += (uint32_t)__mul24(lo[u], z32[ld.z_off + u]);
                h = (int32_t)fast_mod(s, (uint32_t)ld.M, ld.inv_m);
            } else {
                h = exact_bucket(freq + i, n_total, d, z64 + ld.z_off, ld.M);
            }
            if (hash) hash[(int64_t)l * n_total + i] = h;
            if (counts) atomicAdd(counts + ld.node_off + h, 1);
        }
    }
}

int hash_count_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq, int32_t *hash,
                   int32_t *counts)
{
    if (counts) {
        int rc = launch_fill_u32(reinterpret_cast<uint32_t *>(counts), p.nodes, 0u, p.stream);
        if (rc) return rc;
    }
    if (n_total <= 0) return MR1L_OK;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_total + 255) / 256, (int64_t)num_cus() * 16));
    hipLaunchKernelGGL(k_hash_count, dim3((unsigned)blocks), dim3(256), 0, p.stream, freq, n_total, set_off,
                       p.F, p.L, p.d, p.d_lat, p.d_z32, p.d_z64, p.d_kb, hash, counts);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

}  // namespace mr1l
