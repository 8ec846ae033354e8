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
constexpr int kVoteThreads = 256;
constexpr int kVoteLdsWords = 16384;   // 64 KiB of bitmap words per workgroup

// Candidate range of this workgroup: contiguous share of [0, n_total).
template <int D, bool VOTES, bool LDS_BITS>
__global__ __launch_bounds__(kVoteThreads) void k_vote(
    const int64_t *__restrict__ freq, int64_t n_total, const int64_t *__restrict__ set_off, int F,
    int L, int d_rt, const LatDesc *__restrict__ lat, const int32_t *__restrict__ z32,
    const int64_t *__restrict__ z64, const int32_t *__restrict__ kbound,
    const uint32_t *__restrict__ bitmap, int vote_min, int64_t cap, int64_t *__restrict__ det_cnt,
    int64_t *__restrict__ det_idx, uint8_t *__restrict__ votes)
{
    const int d = D > 0 ? D : d_rt;
    __shared__ uint32_t bits[LDS_BITS ? kVoteLdsWords : 1];
    __shared__ int s_f;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t per = (n_total + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * per;
    const int64_t end = min(n_total, beg + per);
    int cur_f = -1;
    int64_t f_lo = 0, f_hi = 0;      // candidate range of cur_f
    int64_t word0 = 0;               // first bitmap word of cur_f

    for (int64_t t0 = beg; t0 < end; t0 += kVoteThreads) {
        // function segments inside this tile
        int64_t seg = t0;
        const int64_t tend = min(end, t0 + kVoteThreads);
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
                if (LDS_BITS) {
                    const int64_t wN = ((lL.node_off + lL.M - 1) >> 5) - word0 + 1;
                    for (int64_t w = tid; w < wN; w += kVoteThreads) bits[w] = bitmap[word0 + w];
                    __syncthreads();
                }
            }
            if (f_hi <= seg) break;   // inconsistent offsets: stop instead of spinning
            const int64_t sEnd = min(tend, f_hi);
            // thread tid handles candidate t0 + tid if it lies in [seg, sEnd)
            const int64_t ci = t0 + tid;
            const bool valid = (ci >= seg) && (ci < sEnd);
            const int f = __builtin_amdgcn_readfirstlane(cur_f);
            int v = 0;
            if (valid) {
                int32_t lo[D > 0 ? D : kMaxD];
                bool fast = true;
                const int32_t kb = kbound[f];
#pragma unroll
                for (int u = 0; u < (D > 0 ? D : kMaxD); ++u) {
                    if (u < d) {
                        const int64_t k = freq[(int64_t)u * n_total + ci];
                        lo[u] = (int32_t)k;
                        fast = fast && (k >= -kb) && (k <= kb);
                    }
                }
                const LatDesc *lf = lat + f * L;
                if (fast) {
                    for (int l = 0; l < L; ++l) {
                        const LatDesc ld = lf[l];
                        const int32_t *zl = z32 + ld.z_off;
                        uint32_t s = ld.off32;
#pragma unroll
                        for (int u = 0; u < (D > 0 ? D : kMaxD); ++u)
                            if (u < d) s += (uint32_t)__mul24(lo[u], zl[u]);
                        const uint32_t h = fast_mod(s, (uint32_t)ld.M, ld.inv_m);
                        const int64_t g = ld.node_off + h;
                        uint32_t word;
                        if (LDS_BITS) word = bits[(g >> 5) - word0];
                        else word = bitmap[g >> 5];
                        v += (word >> (g & 31)) & 1u;
                        if (!VOTES) {
                            // cannot reach vote_min any more: leave the loop
                            const bool hopeless = (v + (L - 1 - l)) < vote_min;
                            const bool done = v >= vote_min;
                            if (__all(hopeless || done)) break;
                        }
                    }
                } else {
                    for (int l = 0; l < L; ++l) {
                        const LatDesc ld = lf[l];
                        const int32_t h = exact_bucket(freq + ci, n_total, d, z64 + ld.z_off, ld.M);
                        const int64_t g = ld.node_off + h;
                        v += (bitmap[g >> 5] >> (g & 31)) & 1u;
                    }
                }
                if (VOTES) votes[ci] = (uint8_t)v;
            }
            // ordered compaction is done later by a sort; here: wave-aggregated append
            const bool det = valid && v >= vote_min;
            const uint64_t bal = __ballot(det);
            if (bal) {
                const int cnt = __popcll(bal);
                const int first = __ffsll((unsigned long long)bal) - 1;
                const int rank = __popcll(bal & ((1ull << lane) - 1ull));
                unsigned long long base = 0;
                if (lane == first) base = atomicAdd((unsigned long long *)(det_cnt + f), (unsigned long long)cnt);
                base = __shfl(base, first);
                if (det && (int64_t)(base + rank) < cap) det_idx[f * cap + base + rank] = ci - f_lo;
            }
            seg = sEnd;
        }
    }
}

#define MR1L_VOTE_DISPATCH(Dv)                                                                    \
    case Dv:                                                                                      \
        if (votes) {                                                                              \
            if (lds) hipLaunchKernelGGL((k_vote<Dv, true, true>), grid, blk, 0, p.stream, ARGS);  \
            else hipLaunchKernelGGL((k_vote<Dv, true, false>), grid, blk, 0, p.stream, ARGS);     \
        } else {                                                                                  \
            if (lds) hipLaunchKernelGGL((k_vote<Dv, false, true>), grid, blk, 0, p.stream, ARGS); \
            else hipLaunchKernelGGL((k_vote<Dv, false, false>), grid, blk, 0, p.stream, ARGS);    \
        }                                                                                         \
        break;

int vote_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq,
             const uint32_t *bitmap, int32_t vote_min, int64_t cap, int64_t *n_det, int64_t *det_idx,
             uint8_t *votes)
{
    int rc = launch_fill_bytes(n_det, sizeof(int64_t) * p.F, p.stream);
    if (rc) return rc;
    if (n_total <= 0) return MR1L_OK;
    // LDS bitmap when every function's lattice bits fit 64 KiB
    int64_t maxw = 0;
    for (int f = 0; f < p.F; ++f) {
        const LatDesc &a = p.lat[(size_t)f * p.L], &b = p.lat[(size_t)f * p.L + p.L - 1];
        maxw = std::max<int64_t>(maxw, ((b.node_off + b.M - 1) >> 5) - (a.node_off >> 5) + 1);
    }
    const bool lds = maxw <= kVoteLdsWords;
    const int64_t want = (n_total + kVoteThreads - 1) / kVoteThreads;
    const int64_t gridn = std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cus() * 8));
    dim3 grid((unsigned)gridn), blk(kVoteThreads);
#define ARGS freq, n_total, set_off, p.F, p.L, p.d, p.d_lat, p.d_z32, p.d_z64, p.d_kb, bitmap, vote_min, \
             cap, n_det, det_idx, votes
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
#undef ARGS
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
