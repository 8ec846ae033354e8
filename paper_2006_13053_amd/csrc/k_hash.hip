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

// Each workgroup owns a contiguous, tile-aligned range of the concatenated
// candidate sets (one candidate per thread and tile).  When they fit, the
// current function's bitmap words sit in LDS (reloaded at function
// boundaries).  The lattice records (offset, -M, reciprocal, bit base, z
// words) are wave-uniform and come through the scalar cache; the record of
// lattice l + 1 is loaded while lattice l is hashed (record L is a padding
// copy).  Lanes without a fast-path candidate start their count far below
// zero, which makes them count as decided in the early exit.
// Waves per SIMD the register allocation aims at: 8 (four 512-thread workgroups per
// CU, as a 40 KiB LDS bitmap allows; the SGPRs beyond 78 go to VGPR lanes) for the
// dimensions where that needs no VGPR spills, else whatever the registers give.
template <int D> constexpr int vote_waves() { return (D >= 1 && D <= 4) || (D >= 7 && D <= 10) ? 8 : 1; }

template <int D, bool LDSB, bool DOT2>
__global__ __launch_bounds__(kVoteThreads) __attribute__((amdgpu_waves_per_eu(vote_waves<D>())))
void k_vote(
    const int64_t *__restrict__ freq, int64_t n_total, const int64_t *__restrict__ set_off, int F,
    int L, int d_rt, const LatDesc *__restrict__ lat, const int64_t *__restrict__ z64,
    const uint32_t *__restrict__ vrec, int rs, int32_t kb_min,
    const uint32_t *__restrict__ bitmap, int64_t bm_words, int vote_min, int64_t cap,
    int64_t *__restrict__ det_cnt, int64_t *__restrict__ det_idx, uint8_t *__restrict__ votes,
    int32_t *__restrict__ cstage)
{
    // D > 0: exactly D coordinates; D < 0: runtime d <= -D; D == 0: runtime d <= kMaxD
    const int d = D > 0 ? D : d_rt;
    constexpr int DM = D > 0 ? D : (D < 0 ? -D : kMaxD);
    constexpr int ZW = DOT2 ? (DM + 1) / 2 : DM;   // z words of a record
    const int zw = DOT2 ? (d + 1) / 2 : d;
    extern __shared__ __align__(16) uint32_t lds[];
    const int recw = (L + 1) * rs;                  // rs is a multiple of 4
    uint32_t *bits = lds;
    // In LDS each lattice's bits start on a word (re-aligned when the function's bitmap
    // is loaded), so bucket h of lattice l is bit h mod 32 of the word at byte
    // base_l + 4 (h >> 5); base_l (record word 3) plus the bitmap's LDS base is a
    // scalar sum, and the per-lane address needs one shift and one shift-add
    typedef __attribute__((address_space(3))) const uint32_t lds_u32;
    const uint32_t lds_byte0 = LDSB ? (uint32_t)(uintptr_t)(lds_u32 *)bits : 0u;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t ntiles = (n_total + kVoteThreads - 1) / kVoteThreads;
    const int64_t tper = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * tper * kVoteThreads;
    const int64_t end = min(n_total, beg + tper * kVoteThreads);
    const bool want_votes = votes != nullptr;
    // no candidate can be hopeless before lattice L - vote_min
    const int L1 = want_votes ? L : max(0, min(L, L - vote_min));
    int f = 0;
    int64_t f_lo = 0, f_hi = 0, word0 = 0;

    // the coordinates of the next tile are loaded while the current one is hashed
    int64_t kn[DM];
    // buffer loads: one descriptor per coordinate row, based at the tile and bounded by
    // the row's end (lanes past the last candidate read 0), plus the lane's byte
    // offset; the descriptors come from scalar adds, not per-lane 64-bit addresses
    auto load_tile = [&](int64_t t) {
        // (t past the last candidate: an empty range, every lane reads 0)
        const int nrec = (int)max<int64_t>(0, min<int64_t>((n_total - t) * 8, (int64_t)0x7ffffff8));
        const char *b = reinterpret_cast<const char *>(freq + t);
#pragma unroll
        for (int u = 0; u < DM; ++u) {
            if (u < d) {
                const __amdgpu_buffer_rsrc_t r =
                    __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(b), (short)0, nrec, 0x00020000);
                typedef int v2i __attribute__((ext_vector_type(2)));
                const v2i x = __builtin_amdgcn_raw_buffer_load_b64(r, tid * 8, 0, 2);   // nontemporal
                kn[u] = (int64_t)(((uint64_t)(uint32_t)x.y << 32) | (uint32_t)x.x);
            }
            b += n_total * 8;
        }
    };
    if (beg < end) load_tile(beg);
    for (int64_t t0 = beg; t0 < end; t0 += kVoteThreads) {
        // this tile's candidate: within the fast bound of every function of the batch
        // (kb_min; beyond it the exact path decides), low words, packed pairs
        // |k_u| <= kb_min for every u, in 32-bit operations (64-bit compares cost more):
        // the high word is the sign of the low word (bad collects the differences) and
        // lo_u + kb_min, unsigned, is at most 2 kb_min (big collects the largest)
        int32_t lo[DM];
        uint32_t bad = 0u, big = 0u;
#pragma unroll
        for (int u = 0; u < DM; ++u) {
            if (u < d) {
                lo[u] = (int32_t)kn[u];
                bad |= (uint32_t)(kn[u] >> 32) ^ (uint32_t)(lo[u] >> 31);
                big = max(big, (uint32_t)lo[u] + (uint32_t)kb_min);
            }
        }
        const bool fast = (bad == 0u) & (big <= 2u * (uint32_t)kb_min);
        uint32_t kp[ZW];
        if constexpr (DOT2) {
#pragma unroll
            for (int j = 0; j < ZW; ++j) {
                // the low halves of a pair in one byte permute (bytes 0, 1 of the first,
                // then bytes 0, 1 of the second); an odd last coordinate pairs with 0
                const uint32_t a0 = (2 * j < d) ? (uint32_t)lo[2 * j] : 0u;
                const uint32_t a1 = (2 * j + 1 < d) ? (uint32_t)lo[2 * j + 1] : 0u;
                kp[j] = __builtin_amdgcn_perm(a1, a0, 0x05040100u);
            }
        }
        // the next tile's loads, issued unconditionally (past the range they read zeros) so
        // that they can land in the registers of the coordinates used above, no copies
        load_tile(t0 + kVoteThreads);
        const int64_t tend = min(end, t0 + kVoteThreads);
        int64_t seg = t0;
        while (seg < tend) {
            if (!(seg >= f_lo && seg < f_hi)) {
                // the workgroup walks its range in order: past the first lookup, the next
                // function is f + 1 (or a later one when sets are empty), one scalar load
                // instead of a binary search, which made many small functions expensive
                int fn;
                if (f_hi > 0 && seg >= f_hi) {
                    fn = f + 1;
                    while (fn + 1 < F && set_off[fn + 1] <= seg) ++fn;
                } else {
                    fn = func_of(set_off, F, seg);
                }
                // every lane searches the same offsets, so f is uniform
                f = __builtin_amdgcn_readfirstlane(fn);
                f_lo = set_off[f];
                f_hi = set_off[f + 1];
                const LatDesc l0 = lat[f * L];
                word0 = l0.node_off >> 5;
                __syncthreads();   // every wave is done with the previous function's tables
                if (LDSB) {
                    // lattice l's M_l bits from bit node_off of the bitmap, to words from
                    // sum_{l' < l} ceil(M_l' / 32) on (a funnel shift of two words)
                    int wbase = 0;
                    for (int l = 0; l < L; ++l) {
                        const LatDesc ll = lat[f * L + l];
                        const int nw = (ll.M + 31) >> 5;
                        const int64_t g0 = ll.node_off >> 5;
                        const uint32_t sh = (uint32_t)(ll.node_off & 31);
                        for (int w = tid; w < nw; w += kVoteThreads) {
                            const uint32_t lo = bitmap[g0 + w];
                            const uint32_t hi = g0 + w + 1 < bm_words ? bitmap[g0 + w + 1] : 0u;
                            bits[wbase + w] = __builtin_amdgcn_alignbit(hi, lo, sh);
                        }
                        wbase += nw;
                    }
                }
                __syncthreads();
            }
            if (f_hi <= seg) break;   // inconsistent offsets: stop instead of spinning
            const int64_t sEnd = min(tend, f_hi);
            const int64_t c = t0 + tid;
            // the lanes of [seg, sEnd), tested on tile offsets (32-bit)
            const bool val = (tid >= (int)(seg - t0)) && (tid < (int)(sEnd - t0));
            const bool act = val && fast;
            int v = act ? 0 : -(1 << 20);
            if (__any(act)) {
                // uniform records through the scalar cache (constant address space)
                typedef const __attribute__((address_space(4))) uint32_t *crec_t;
                const crec_t rp = (crec_t)(uintptr_t)(vrec + (int64_t)f * recw);
                constexpr int RW = 4 + ZW;
                uint32_t ra[RW], rb[RW];
#pragma unroll
                for (int j = 0; j < RW; ++j) ra[j] = (j < 4 + zw) ? rp[j] : 0u;
                // hash lattice l with record `cur` while record l + 1 is loaded into `nxt`
                auto step = [&](const uint32_t (&r)[RW], uint32_t (&nxt)[RW], int l) {
#pragma unroll
                    for (int j = 0; j < RW; ++j) nxt[j] = (j < 4 + zw) ? rp[(l + 1) * rs + j] : 0u;
                    uint32_t s = r[0];
                    if constexpr (DOT2) {
                        typedef short v2s __attribute__((ext_vector_type(2)));
#pragma unroll
                        for (int j = 0; j < ZW; ++j)
                            if (j < zw)
                                s = (uint32_t)__builtin_amdgcn_sdot2(__builtin_bit_cast(v2s, kp[j]),
                                                                     __builtin_bit_cast(v2s, r[4 + j]), (int)s, false);
                    } else {
#pragma unroll
                        for (int u = 0; u < DM; ++u)
                            if (u < d) s += (uint32_t)__mul24(lo[u], (int32_t)r[4 + u]);
                    }
                    // s < 2^32 and s / M < 2^20: the float quotient is exact or one too small
                    const int32_t negM = (int32_t)r[1];
                    const uint32_t q = (uint32_t)((float)s * __uint_as_float(r[2]));
                    uint32_t h = (uint32_t)(__mul24((int32_t)q, negM) + (int32_t)s);   // in [0, 2M)
                    h = min(h, h + (uint32_t)negM);
                    uint32_t word, g;
                    if constexpr (LDSB) {
                        const uint32_t wb = (uint32_t)__builtin_amdgcn_readfirstlane(r[3] + lds_byte0);
                        // the word index hidden from the optimiser, so that the address stays
                        // one shift-add instead of a shift, a mask and an add
                        uint32_t hw = h >> 5;
                        asm("" : "+v"(hw));
                        word = *(lds_u32 *)(uintptr_t)(wb + (hw << 2));
                        g = h;
                    } else {
                        g = r[3] + h;
                        word = bitmap[word0 + (g >> 5)];
                    }
                    v += (int)__builtin_amdgcn_ubfe(word, g, 1);   // bit g mod 32
                };
                // undecided after lattice l: vote_min - rest <= v < vote_min
                auto decided = [&](int l) {
                    const int rest = L - 1 - l;
                    return __all((uint32_t)(v - vote_min + rest) >= (uint32_t)rest);
                };
                // two lattices per iteration, so the record buffers alternate without copies
                int l = 0;
                for (; l + 1 < L1; l += 2) {
                    step(ra, rb, l);
                    step(rb, ra, l + 1);
                }
                if (l < L1) {
                    step(ra, rb, l);
#pragma unroll
                    for (int j = 0; j < RW; ++j) ra[j] = rb[j];
                    ++l;
                }
                while (l < L) {
                    step(ra, rb, l);
                    if (decided(l) || ++l == L) break;
                    step(rb, ra, l);
                    if (decided(l)) break;
                    ++l;
                }
            }
            // exact 64-bit path for candidates beyond the bound (rare, divergent)
            if (val && !fast) {
                v = 0;
                const LatDesc *lf = lat + f * L;
                for (int l = 0; l < L; ++l) {
                    const LatDesc ld = lf[l];
                    const int32_t h = exact_bucket(freq + c, n_total, d, z64 + ld.z_off, ld.M);
                    uint32_t word;
                    int bit;
                    if constexpr (LDSB) {
                        word = bits[(vrec[(int64_t)f * recw + l * rs + 3] >> 2) + (h >> 5)];
                        bit = h & 31;
                    } else {
                        const int64_t g = ld.node_off + h;
                        word = bitmap[g >> 5];
                        bit = (int)(g & 31);
                    }
                    v += (word >> bit) & 1u;
                }
            }
            if (want_votes && val) votes[c] = (uint8_t)max(v, 0);
            const bool det = val && v >= vote_min;
            const uint64_t bal = __ballot(det);
            if (bal) {
                const int cnt = __popcll(bal);
                const int first = __ffsll((unsigned long long)bal) - 1;
                const int rank = __popcll(bal & ((1ull << lane) - 1ull));
                unsigned long long base = 0;
                if (lane == first) base = atomicAdd((unsigned long long *)(det_cnt + f), (unsigned long long)cnt);
                base = __shfl(base, first);
                const int64_t pos = (int64_t)(base + rank);
                if (det && pos < cap) {
                    det_idx[f * cap + pos] = c - f_lo;
                    // short lists: the detected candidate's coordinates as hashed here (the
                    // packed pairs or the low words), at its append position, so that the
                    // bucket pass reads a compact list instead of the candidate set
                    if (cstage) {
                        int32_t *cs = cstage + (f * cap + pos) * (int64_t)zw;
                        if (!fast) {
                            cs[0] = INT32_MIN;   // beyond the fast bound: the exact path rereads it
                        } else if constexpr (DOT2) {
#pragma unroll
                            for (int j = 0; j < ZW; ++j)
                                if (j < zw) cs[j] = (int32_t)kp[j];
                        } else {
#pragma unroll
                            for (int u = 0; u < DM; ++u)
                                if (u < d) cs[u] = lo[u];
                        }
                    }
                }
            }
            seg = sEnd;
        }
    }
}

#define MR1L_VOTE_LAUNCH(Dv, LD, D2)                                                                       \
    hipLaunchKernelGGL((k_vote<Dv, LD, D2>), grid, blk, shm, p.stream, freq, n_total, set_off, p.F, p.L, p.d, \
                       p.d_lat, p.d_z64, p.d_vrec, p.vrec_stride, kb_min, bitmap, bm_words, vote_min, cap, n_det,   \
                       det_idx, votes, cstage)
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
#define MR1L_VOTE_ATTR(Dv)                                                                              \
    MR1L_HIP(hipFuncSetAttribute((const void *)k_vote<Dv, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                 kVoteLdsWords * 4));                                                    \
    MR1L_HIP(hipFuncSetAttribute((const void *)k_vote<Dv, true, false>,                                  \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kVoteLdsWords * 4));
    MR1L_VOTE_ATTR(0) MR1L_VOTE_ATTR(1) MR1L_VOTE_ATTR(2) MR1L_VOTE_ATTR(3) MR1L_VOTE_ATTR(4)
    MR1L_VOTE_ATTR(5) MR1L_VOTE_ATTR(6) MR1L_VOTE_ATTR(7) MR1L_VOTE_ATTR(8) MR1L_VOTE_ATTR(9)
    MR1L_VOTE_ATTR(10) MR1L_VOTE_ATTR(12) MR1L_VOTE_ATTR(16) MR1L_VOTE_ATTR(20) MR1L_VOTE_ATTR(25)
    MR1L_VOTE_ATTR(30) MR1L_VOTE_ATTR(-16) MR1L_VOTE_ATTR(-32)
#undef MR1L_VOTE_ATTR
    return MR1L_OK;
}

int vote_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq,
             const uint32_t *bitmap, int32_t vote_min, int64_t cap, int64_t *n_det, int64_t *det_idx,
             uint8_t *votes, int32_t *cstage)
{
    // n_det is zero-filled by the caller (outside the timed vote stage)
    if (n_total <= 0) return MR1L_OK;
    // LDS bitmap copy (each lattice's bits from a word boundary) when every function's
    // fits; the records were built for the same choice
    const int64_t bm_words = (p.nodes + 31) / 32;
    const bool lds = p.vote_lds;
    const size_t shm = lds ? (size_t)p.vote_lds_words * 4 : 0;
    int32_t kb_min = INT32_MAX;
    for (int32_t k : p.kb) kb_min = std::min(kb_min, k);
    const int64_t tiles = (n_total + kVoteThreads - 1) / kVoteThreads;
    // one co-resident workgroup per slot: no partial second round of workgroups
    int per_cu = 0;
    const void *kfn = lds ? (const void *)k_vote<10, true, true> : (const void *)k_vote<10, false, true>;
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
        // other dimensions: the coordinate registers sized for d <= 16, d <= 32 or any d
        switch (p.d <= 16 ? -16 : p.d <= 32 ? -32 : 0) {
            MR1L_VOTE_DISPATCH(-16)
            MR1L_VOTE_DISPATCH(-32)
        default:
            MR1L_VOTE_DISPATCH(0)
        }
    }
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

// ------------------------------------------------------------------ hash + count
// hash[l * n_total + i] and counts[O_{f,l} + h] over a candidate set; counts is
// zero-filled first and accumulated with global atomics (order-independent).
template <int DM>   // d <= DM: the coordinates stay in registers
__global__ __launch_bounds__(256) void k_hash_count(
    const int64_t *__restrict__ freq, int64_t n_total, const int64_t *__restrict__ set_off, int F, int L,
    int d, const LatDesc *__restrict__ lat, const int32_t *__restrict__ z32, const int64_t *__restrict__ z64,
    const int32_t *__restrict__ kbound, int32_t *__restrict__ hash, int32_t *__restrict__ counts)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int f = func_of(set_off, F, i);
        const int32_t kb = kbound[f];
        int32_t lo[DM];
        bool fast = true;
#pragma unroll
        for (int u = 0; u < DM; ++u) {
            if (u < d) {
                const int64_t k = freq[(int64_t)u * n_total + i];
                lo[u] = (int32_t)k;
                fast = fast & (k >= -kb) & (k <= kb);
            }
        }
        for (int l = 0; l < L; ++l) {
            const LatDesc ld = lat[f * L + l];
            int32_t h;
            if (fast) {
                uint32_t s = ld.off32;
#pragma unroll
                for (int u = 0; u < DM; ++u)
                    if (u < d) s += (uint32_t)__mul24(lo[u], z32[ld.z_off + u]);
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
#define MR1L_HC(DM)                                                                                          \
    hipLaunchKernelGGL(k_hash_count<DM>, dim3((unsigned)blocks), dim3(256), 0, p.stream, freq, n_total, set_off, \
                       p.F, p.L, p.d, p.d_lat, p.d_z32, p.d_z64, p.d_kb, hash, counts)
    if (p.d <= 16) MR1L_HC(16);
    else if (p.d <= 32) MR1L_HC(32);
    else MR1L_HC(kMaxD);
#undef MR1L_HC
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

}  // namespace mr1l
