// After the vote: ordered detected set, singleton masks, coefficients and the
// output limitation.
//
//  k_sort_det    detected set of each function in ascending candidate order
//                (one workgroup per function, bitonic sort in registers, lane
//                shuffles and, for the longest distances only, LDS).
//  k_det_hash_staged / k_det_hash  buckets h_l(k) of every detected candidate,
//                one thread per candidate: short lists from the coordinates the
//                vote staged, long ones from the candidate set.
//  k_singleton   whether each bucket holds one or several detected candidates,
//                one workgroup per lattice with two LDS bitmaps; bit l of
//                mask[q] is set when candidate q is alone in its bucket (the
//                sets of Remark 2.9).
//  k_combine     medians of the real and imaginary parts of the L lattice
//                values (eq. (2.10); even L: mean of the two middle order
//                statistics; order by value, ties by lattice index) and the
//                singleton average of Remark 2.9, plus the weights of the
//                coefficient as a real-linear map of the lattice values.
//  k_limit       Algorithm 4: |p| >= theta, descending modulus, ties by
//                ascending candidate index, first s~ (the same block sort).
//  k_adjoint_scatter  transpose of the gather/combination: coefficient
//                gradients into buckets (the inverse lattice DFT follows).
#include <algorithm>

#include "mr1l_internal.h"

namespace mr1l {

constexpr int kSortThreads = 1024;
constexpr int64_t kTailBlocks = 4;    // least workgroups per function of the per-entry tail kernels
constexpr int64_t kTailGrid = 256;    // workgroups the whole grid of such a kernel aims at (one per CU)

// Workgroups per function of a per-entry tail kernel whose lists need `need` workgroups at
// most: the kernels loop over a function's entries, so a few per function suffice when there
// are many functions, while a single long list still spreads over the whole chip
static unsigned tail_blocks(int64_t need, int F, int64_t scale = 1)
{
    const int64_t per_f = std::max<int64_t>(kTailBlocks * scale, kTailGrid * scale / std::max(F, 1));
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, per_f));
}

__device__ __forceinline__ int64_t n_of(const int64_t *n_det, int f, int64_t cap)
{
    const int64_t n = n_det[f];
    return n < cap ? n : cap;
}

// ------------------------------------------------------------------ block sort
// Bitonic sort of P = 2^p (key, value) pairs ascending by key, ties by value, held E
// per thread in registers: thread t holds positions tE .. tE + E - 1 (threads t < P/E
// take part; E <= P <= E x blockDim.x).  Compare-exchange partners closer than E sit
// in the same thread, those closer than 64 E in the same wave (exchanged by lane
// shuffles); only the stages with larger distances go through LDS (lk, lv: P entries
// each, value e of thread t at e P/E + t), with two barriers each.  Every thread of
// the block must call it.
__device__ __forceinline__ bool kv_gt(uint64_t ka, int32_t va, uint64_t kb, int32_t vb)
{
    return ka > kb || (ka == kb && va > vb);
}

template <int E>
__device__ __forceinline__ void block_bitonic(uint64_t (&k)[E], int32_t (&v)[E], int P, uint64_t *lk, int32_t *lv)
{
    const int t = threadIdx.x, na = P / E;
    const bool act = t < na;
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 64 * E) {
                // the partner of position tE + e is (t ^ m)E + e (m = j / E): value e of
                // every thread sits at lk[e na + t], so a wave's lanes touch consecutive words
                const int m = j / E;
                if (act)
#pragma unroll
                    for (int e = 0; e < E; ++e) { lk[e * na + t] = k[e]; lv[e * na + t] = v[e]; }
                __syncthreads();
                if (act)
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int p = t * E + e;
                        const uint64_t kb = lk[e * na + (t ^ m)];
                        const int32_t vb = lv[e * na + (t ^ m)];
                        const bool gt = kv_gt(k[e], v[e], kb, vb);
                        if ((((p & j) == 0) == ((p & kk) == 0)) ? gt : !gt) { k[e] = kb; v[e] = vb; }
                    }
                __syncthreads();
            } else if (j >= E) {
                const int m = j / E;
                const bool lower = (t & m) == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const uint64_t kb = __shfl_xor(k[e], m);
                    const int32_t vb = __shfl_xor(v[e], m);
                    const bool asc = ((t * E + e) & kk) == 0;
                    const bool gt = kv_gt(k[e], v[e], kb, vb);
                    if (act && ((lower == asc) ? gt : !gt)) { k[e] = kb; v[e] = vb; }
                }
            } else {
#pragma unroll
                for (int jj = E / 2; jj >= 1; jj >>= 1)
                    if (jj == j)
#pragma unroll
                        for (int e = 0; e < E; ++e)
                            if ((e & jj) == 0) {
                                const int e2 = e | jj;
                                const bool asc = ((t * E + e) & kk) == 0;
                                if (kv_gt(k[e], v[e], k[e2], v[e2]) == asc) {
                                    const uint64_t tk = k[e]; k[e] = k[e2]; k[e2] = tk;
                                    const int32_t tv = v[e]; v[e] = v[e2]; v[e2] = tv;
                                }
                            }
            }
        }
    }
}

__device__ __forceinline__ int sort_len(int n, int E)
{
    int P = E;
    while (P < n) P <<= 1;
    return P;
}

// ------------------------------------------------------------------ sort detected
// Dynamic LDS: max(pow2ceil(cap) x 12, kSortBitmapBytes) bytes.  A function whose
// candidate set has at most 8 x (that many) members takes the ordered compaction of a
// bitmap over its set in LDS (one bit per detected candidate, then per-thread counts,
// a block scan and the emission: O(|I_f| / 32 + n) work); larger sets take the block
// sort, E = pow2ceil(cap) / kSortThreads values per thread, at least 1.
constexpr int kSortBitmapBytes = 128 * 1024;

__device__ __forceinline__ int block_excl_scan(int v, int *wsum)
{
    // inclusive scan within the wave, then the waves' totals
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int k = 0; k < nw; ++k) {
            const int t = wsum[k];
            wsum[k] = acc;
            acc += t;
        }
    }
    __syncthreads();
    return wsum[w] + x - v;
}

// perm (or NULL): [F][cap] append position of the entry at each place of the ordered list.
template <int E>
__global__ __launch_bounds__(kSortThreads) void k_sort_det(const int64_t *__restrict__ n_det, int64_t cap,
                                                           int64_t *__restrict__ det_idx,
                                                           const int64_t *__restrict__ set_off, int64_t n_total,
                                                           int region_bytes, uint32_t *__restrict__ mask, int mw,
                                                           int32_t *__restrict__ perm)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wsum[kSortThreads / 64];
    __shared__ int offs[kSortThreads];
    const int f = blockIdx.x, t = threadIdx.x;
    const int64_t fb = (int64_t)f * cap;
    // the function's singleton masks start cleared (the singleton pass only sets bits)
    for (int64_t i = t; i < cap * mw; i += kSortThreads) mask[fb * mw + i] = 0u;
    const int n = (int)n_of(n_det, f, cap);
    if (n == 0) return;
    int64_t *src = det_idx + fb;
    if (n == 1) {
        if (perm && t == 0) perm[fb] = 0;
        return;
    }
    const int64_t nset = set_off ? set_off[f + 1] - set_off[f] : n_total;
    if (nset <= (int64_t)region_bytes * 8) {
        // each entry's place in the ordered list from a bitmap over the function's set: the
        // bits before it in its word plus the counts of the words before (a block scan over
        // per-thread runs of words); entry p is held by thread p mod kSortThreads
        int64_t cv[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = t + kSortThreads * e;
            cv[e] = p < n ? src[p] : -1;
        }
        uint32_t *bm = reinterpret_cast<uint32_t *>(smem);
        const int nw = (int)((nset + 31) >> 5);
        for (int w = t; w < nw; w += kSortThreads) bm[w] = 0u;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (cv[e] >= 0) atomicOr(bm + (cv[e] >> 5), 1u << (cv[e] & 31));
        __syncthreads();
        // thread t owns words [t c, t c + c)
        const int c = (nw + kSortThreads - 1) / kSortThreads, w0 = min(nw, t * c), w1 = min(nw, w0 + c);
        int cnt = 0;
        for (int w = w0; w < w1; ++w) cnt += __popc(bm[w]);
        offs[t] = block_excl_scan(cnt, wsum);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (cv[e] < 0) continue;
            const int w = (int)(cv[e] >> 5), own = w / c;
            int r = offs[own];
            for (int x = own * c; x < w; ++x) r += __popc(bm[x]);
            r += __popc(bm[w] & ((1u << (cv[e] & 31)) - 1u));
            src[r] = cv[e];
            if (perm) perm[fb + r] = t + kSortThreads * e;
        }
        return;
    }
    const int P = sort_len(n, E);
    uint64_t *lk = reinterpret_cast<uint64_t *>(smem);
    int32_t *lv = reinterpret_cast<int32_t *>(lk + P);
    uint64_t k[E];
    int32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = t * E + e;
        k[e] = (p < n) ? (uint64_t)src[p] : ~0ull;   // indices are non-negative
        v[e] = p;                                    // the entry's append position
    }
    block_bitonic<E>(k, v, P, lk, lv);
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (t * E + e < n) {
            src[t * E + e] = (int64_t)k[e];
            if (perm) perm[fb + t * E + e] = v[e];
        }
}

// ------------------------------------------------------------------ hashes of detected
// Fast path (every |k_u| within the function's bound kb): 24-bit multiply-adds in 32-bit
// integers and the float-reciprocal modulo; else the exact 64-bit reduction.  Both give
// the same bucket.
//
// Long lists: one thread per detected candidate: its d coordinates are read once (adjacent threads
// hold adjacent entries of the ascending list) and hashed into all L lattices of its
// function, with L running sums in registers; the lattice records and z words are
// workgroup-uniform (scalar loads).  The chunk's buckets go through LDS in output order
// ([entry][lattice]) so that the stores are contiguous.  Dynamic LDS: 256 L int32.
constexpr int kDetHashThreads = 256;
constexpr int kDetHashBatch = 8;

template <int LM>
__global__ __launch_bounds__(kDetHashThreads) void k_det_hash(
    const int64_t *__restrict__ freq, int64_t n_total, const int64_t *__restrict__ set_off, int L, int d,
    const LatDesc *__restrict__ lat, const int32_t *__restrict__ z32, const int64_t *__restrict__ z64,
    const int32_t *__restrict__ kbound, const int64_t *__restrict__ n_det, int64_t cap,
    const int64_t *__restrict__ det_idx, int32_t *__restrict__ det_hash)
{
    extern __shared__ int32_t hs[];
    const int f = blockIdx.y, t = threadIdx.x;
    const int64_t n = n_of(n_det, f, cap);
    const int64_t base = set_off[f];
    const int32_t kb = kbound[f];
    const LatDesc *lf = lat + (int64_t)f * L;
    for (int64_t q0 = (int64_t)blockIdx.x * kDetHashThreads; q0 < n; q0 += (int64_t)gridDim.x * kDetHashThreads) {
        const int64_t q = q0 + t;
        if (q < n) {
            const int64_t ci = base + det_idx[(int64_t)f * cap + q];
            uint32_t acc[LM];
#pragma unroll
            for (int l = 0; l < LM; ++l) acc[l] = l < L ? lf[l].off32 : 0u;
            bool fast = true;
            // the coordinates in batches whose loads are all in flight together
            for (int u0 = 0; u0 < d; u0 += kDetHashBatch) {
                int64_t kv[kDetHashBatch];
#pragma unroll
                for (int j = 0; j < kDetHashBatch; ++j)
                    kv[j] = u0 + j < d ? freq[(int64_t)(u0 + j) * n_total + ci] : 0;
#pragma unroll
                for (int j = 0; j < kDetHashBatch; ++j) {
                    if (u0 + j < d) {
                        fast = fast & (kv[j] >= -kb) & (kv[j] <= kb);
                        const int32_t k32 = (int32_t)kv[j];
#pragma unroll
                        for (int l = 0; l < LM; ++l)
                            if (l < L) acc[l] += (uint32_t)__mul24(k32, z32[lf[l].z_off + u0 + j]);
                    }
                }
            }
#pragma unroll
            for (int l = 0; l < LM; ++l)
                if (l < L)
                    hs[t * L + l] = fast ? (int32_t)fast_mod(acc[l], (uint32_t)lf[l].M, lf[l].inv_m)
                                         : exact_bucket(freq + ci, n_total, d, z64 + lf[l].z_off, lf[l].M);
        }
        __syncthreads();
        const int64_t cnt = min<int64_t>(kDetHashThreads, n - q0) * L;
        int32_t *dst = det_hash + ((int64_t)f * cap + q0) * L;
        for (int64_t i = t; i < cnt; i += kDetHashThreads) dst[i] = hs[i];
        __syncthreads();
    }
}

// Short lists: one thread per entry of the ordered list, from the coordinates the vote
// staged at the entry's append position (perm): W = ceil(d/2) packed 16-bit pairs or d low
// words, read once, hashed into all L lattices with the 32-bit fast path (valid: the vote
// staged only candidates within the batch's fast bound, which no function's exceeds); an
// entry marked INT32_MIN takes the exact path from the candidate set.  Buckets staged in
// LDS for contiguous stores, as above.
template <int LM>
__global__ __launch_bounds__(kDetHashThreads) void k_det_hash_staged(
    const int64_t *__restrict__ freq, int64_t n_total, const int64_t *__restrict__ set_off, int L, int d,
    int packed, const LatDesc *__restrict__ lat, const int32_t *__restrict__ z32, const int64_t *__restrict__ z64,
    const int64_t *__restrict__ n_det, int64_t cap, const int64_t *__restrict__ det_idx,
    const int32_t *__restrict__ cstage, const int32_t *__restrict__ perm, int32_t *__restrict__ det_hash)
{
    extern __shared__ int32_t hs[];
    const int f = blockIdx.y, t = threadIdx.x;
    const int64_t n = n_of(n_det, f, cap);
    const int64_t fb = (int64_t)f * cap;
    const int W = packed ? (d + 1) / 2 : d;
    const LatDesc *lf = lat + (int64_t)f * L;
    for (int64_t q0 = (int64_t)blockIdx.x * kDetHashThreads; q0 < n; q0 += (int64_t)gridDim.x * kDetHashThreads) {
        const int64_t q = q0 + t;
        if (q < n) {
            const int32_t *cs = cstage + (fb + perm[fb + q]) * W;
            if (cs[0] != INT32_MIN) {
                uint32_t acc[LM];
#pragma unroll
                for (int l = 0; l < LM; ++l) acc[l] = l < L ? lf[l].off32 : 0u;
                for (int w = 0; w < W; ++w) {
                    const int32_t x = cs[w];
                    const int nu = packed ? min(2, d - 2 * w) : 1;
                    for (int h = 0; h < nu; ++h) {
                        const int u = packed ? 2 * w + h : w;
                        const int32_t k = packed ? (int32_t)(int16_t)(x >> (16 * h)) : x;
#pragma unroll
                        for (int l = 0; l < LM; ++l)
                            if (l < L) acc[l] += (uint32_t)__mul24(k, z32[lf[l].z_off + u]);
                    }
                }
#pragma unroll
                for (int l = 0; l < LM; ++l)
                    if (l < L) hs[t * L + l] = (int32_t)fast_mod(acc[l], (uint32_t)lf[l].M, lf[l].inv_m);
            } else {
                const int64_t ci = set_off[f] + det_idx[fb + q];
                for (int l = 0; l < L; ++l)
                    hs[t * L + l] = exact_bucket(freq + ci, n_total, d, z64 + lf[l].z_off, lf[l].M);
            }
        }
        __syncthreads();
        const int64_t cnt = min<int64_t>(kDetHashThreads, n - q0) * L;
        int32_t *dst = det_hash + (fb + q0) * L;
        for (int64_t i = t; i < cnt; i += kDetHashThreads) dst[i] = hs[i];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ singletons
// One workgroup per lattice (f, l).  Two LDS bitmaps over the buckets: the first
// atomicOr of a bucket's bit in `once` returns it clear, every later one sets the
// bit in `twice`; a detected candidate is alone in its bucket exactly when the
// bucket's `twice` bit stays clear.  Buckets beyond one LDS span are handled in
// further passes over the detected set.
constexpr int kSingleWords = 20480;   // words per bitmap: 2 x 80 KiB of LDS at most

__global__ __launch_bounds__(256) void k_singleton(const LatDesc *__restrict__ lat, int L,
                                                   const int64_t *__restrict__ n_det, int64_t cap,
                                                   const int32_t *__restrict__ det_hash,
                                                   uint32_t *__restrict__ mask, int words)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *once = reinterpret_cast<uint32_t *>(smem);
    uint32_t *twice = once + words;
    int l = blockIdx.x, f = blockIdx.y;
    if ((gridDim.x * gridDim.y) % 8 == 0) {
        // the L workgroups of a function on one XCD (workgroups are dealt to the 8 XCDs in
        // turn): they read the same bucket rows and set bits in the same mask words
        const int G = gridDim.x * gridDim.y, w = blockIdx.y * gridDim.x + blockIdx.x;
        const int i = (w & 7) * (G >> 3) + (w >> 3);
        f = i / gridDim.x;
        l = i - f * gridDim.x;
    }
    const int n = (int)n_of(n_det, f, cap);
    if (n == 0) return;
    const int M = lat[f * L + l].M;
    const int32_t *hh = det_hash + (int64_t)f * cap * L;
    const int span = words * 32;
    for (int c0 = 0; c0 < M; c0 += span) {
        const int c1 = min(M, c0 + span);
        const int nw = (c1 - c0 + 31) >> 5;
        for (int i = threadIdx.x; i < nw; i += blockDim.x) { once[i] = 0u; twice[i] = 0u; }
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int h = hh[(int64_t)q * L + l];
            if (h >= c0 && h < c1) {
                const int r = h - c0;
                const uint32_t bit = 1u << (r & 31);
                if (atomicOr(once + (r >> 5), bit) & bit) atomicOr(twice + (r >> 5), bit);
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int h = hh[(int64_t)q * L + l];
            if (h >= c0 && h < c1) {
                const int r = h - c0;
                if (!((twice[r >> 5] >> (r & 31)) & 1u))
                    atomicOr(mask + ((int64_t)f * cap + q) * mask_words(L) + (l >> 5), 1u << (l & 31));
            }
        }
        __syncthreads();
    }
}

// Long detected lists (global bitmaps once / twice per lattice, zeroed first):
// workgroup (chunk, l, f) counts its chunk of the detected set in LDS bitmaps as
// above, then merges them word by word.  A bucket ends in `twice` when one chunk
// saw it twice, or when it was already in `once` from another chunk.
constexpr int kSingleThreads = 1024;
constexpr int kSingleLoads = 8;

__global__ __launch_bounds__(kSingleThreads) void k_single_count(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ n_det, int64_t cap,
    const int32_t *__restrict__ det_hash, int chunks, int64_t wl, uint32_t *__restrict__ g_once,
    uint32_t *__restrict__ g_twice, int words)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *once = reinterpret_cast<uint32_t *>(smem);
    uint32_t *twice = once + words;
    const int l = blockIdx.y, f = blockIdx.z;
    const int64_t n = n_of(n_det, f, cap);
    const int64_t per = (n + chunks - 1) / chunks;
    const int64_t q0 = (int64_t)blockIdx.x * per, q1 = min(n, q0 + per);
    if (q0 >= q1) return;
    const int M = lat[f * L + l].M;
    const int32_t *hh = det_hash + (int64_t)f * cap * L;
    uint32_t *go = g_once + ((int64_t)f * L + l) * wl;
    uint32_t *gt = g_twice + ((int64_t)f * L + l) * wl;
    const int span = words * 32;
    for (int c0 = 0; c0 < M; c0 += span) {
        const int c1 = min(M, c0 + span);
        const int nw = (c1 - c0 + 31) >> 5;
        for (int i = threadIdx.x; i < nw; i += blockDim.x) { once[i] = 0u; twice[i] = 0u; }
        __syncthreads();
        // kSingleLoads buckets in flight per thread (the loop is latency-bound otherwise)
        for (int64_t qb = q0 + threadIdx.x; qb < q1; qb += (int64_t)kSingleLoads * blockDim.x) {
            int hv[kSingleLoads];
#pragma unroll
            for (int k = 0; k < kSingleLoads; ++k) {
                const int64_t q = qb + (int64_t)k * blockDim.x;
                hv[k] = q < q1 ? hh[q * L + l] : -1;
            }
#pragma unroll
            for (int k = 0; k < kSingleLoads; ++k) {
                const int h = hv[k];
                if (h >= c0 && h < c1) {
                    const int r = h - c0;
                    const uint32_t bit = 1u << (r & 31);
                    if (atomicOr(once + (r >> 5), bit) & bit) atomicOr(twice + (r >> 5), bit);
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nw; i += blockDim.x) {
            const uint32_t o = once[i];
            if (o) {
                const uint32_t prev = atomicOr(go + (c0 >> 5) + i, o);
                const uint32_t t = twice[i] | (prev & o);
                if (t) atomicOr(gt + (c0 >> 5) + i, t);
            }
        }
        __syncthreads();
    }
}

// The same with the lattices in groups: workgroup (chunk, group, f) counts its chunk for
// the group's lattices [l0, l0 + ng), each in its own pair of LDS bitmaps (sw words per
// lattice, sw >= ceil(M / 32) for every lattice), so that each entry's buckets of the
// group are read together, once per workgroup (a chunk's rows were read by L workgroups,
// spread over the chip, before).
__global__ __launch_bounds__(kSingleThreads) void k_single_count_grp(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ n_det, int64_t cap,
    const int32_t *__restrict__ det_hash, int chunks, int gs, int sw, int64_t wl, uint32_t *__restrict__ g_once,
    uint32_t *__restrict__ g_twice)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *once = reinterpret_cast<uint32_t *>(smem);
    uint32_t *twice = once + gs * sw;
    const int f = blockIdx.z, l0 = blockIdx.y * gs, ng = min(gs, L - l0);
    const int64_t n = n_of(n_det, f, cap);
    const int64_t per = (n + chunks - 1) / chunks;
    const int64_t q0 = (int64_t)blockIdx.x * per, q1 = min(n, q0 + per);
    if (q0 >= q1) return;
    for (int i = threadIdx.x; i < ng * sw; i += blockDim.x) { once[i] = 0u; twice[i] = 0u; }
    __syncthreads();
    const int32_t *hh = det_hash + (int64_t)f * cap * L + l0;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const int32_t *hq = hh + q * L;
        for (int j0 = 0; j0 < ng; j0 += kSingleLoads) {
            int hv[kSingleLoads];
#pragma unroll
            for (int k = 0; k < kSingleLoads; ++k) hv[k] = j0 + k < ng ? hq[j0 + k] : 0;
#pragma unroll
            for (int k = 0; k < kSingleLoads; ++k) {
                if (j0 + k < ng) {
                    const int wi = (j0 + k) * sw + (hv[k] >> 5);
                    const uint32_t bit = 1u << (hv[k] & 31);
                    if (atomicOr(once + wi, bit) & bit) atomicOr(twice + wi, bit);
                }
            }
        }
    }
    __syncthreads();
    for (int j = 0; j < ng; ++j) {
        const int nw = (lat[f * L + l0 + j].M + 31) >> 5;
        uint32_t *go = g_once + ((int64_t)f * L + l0 + j) * wl;
        uint32_t *gt = g_twice + ((int64_t)f * L + l0 + j) * wl;
        for (int i = threadIdx.x; i < nw; i += blockDim.x) {
            const uint32_t o = once[j * sw + i];
            if (o) {
                const uint32_t prev = atomicOr(go + i, o);
                const uint32_t t = twice[j * sw + i] | (prev & o);
                if (t) atomicOr(gt + i, t);
            }
        }
    }
}

// One thread per detected candidate: its singleton mask over all lattices from the
// merged `twice` bitmaps, written whole (no atomics).
__global__ __launch_bounds__(256) void k_single_mask(const LatDesc *__restrict__ lat, int L,
                                                     const int64_t *__restrict__ n_det, int64_t cap,
                                                     const int32_t *__restrict__ det_hash, int64_t wl,
                                                     const uint32_t *__restrict__ g_twice,
                                                     uint32_t *__restrict__ mask)
{
    const int f = blockIdx.y;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_of(n_det, f, cap)) return;
    const int32_t *hq = det_hash + ((int64_t)f * cap + q) * L;
    const uint32_t *gt = g_twice + (int64_t)f * L * wl;
    uint32_t w[2] = {0u, 0u};
    for (int l = 0; l < L; ++l) {
        const int h = hq[l];
        if (!((gt[(int64_t)l * wl + (h >> 5)] >> (h & 31)) & 1u)) w[l >> 5] |= 1u << (l & 31);
    }
    const int W = mask_words(L);
    for (int k = 0; k < W; ++k) mask[((int64_t)f * cap + q) * W + k] = w[k];
}

// ------------------------------------------------------------------ combine
// Median position(s) by rank: rank_l = #{m : (v_m, m) < (v_l, l)}.  Entries
// L..LMAX-1 hold +infinity, which never ranks below a lattice value, so the
// counting needs no bounds tests.
template <typename T, int LMAX>
__device__ __forceinline__ void median_sel(const T *v, int L, T &med, int &s0, int &s1)
{
    const int want0 = (L - 1) / 2, want1 = L / 2;
    s0 = 0; s1 = 0;
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
        int rank = 0;
#pragma unroll
        for (int m = 0; m < LMAX; ++m) {
            if (m < l) rank += v[m] <= v[l];
            else if (m > l) rank += v[m] < v[l];
        }
        if (l < L) {
            if (rank == want0) s0 = l;
            if (rank == want1) s1 = l;
        }
    }
    T a = 0, b = 0;
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
        if (l == s0) a = v[l];
        if (l == s1) b = v[l];
    }
    med = (L & 1) ? a : T(0.5) * (a + b);
}

// Writes the median, the post-processed coefficient (mean of the lattice values
// over the singleton lattices of mask mk, when post-processing is on and there
// is one) and the real weights of the coefficient as a linear map of the
// lattice values.
template <typename T>
__device__ __forceinline__ void combine_store(int L, int64_t e, uint64_t mk, T mr, T mi, T sum_r, T sum_i,
                                              int r0, int r1, int i0, int i1, int postproc,
                                              typename cvec<T>::type *__restrict__ det_coef,
                                              typename cvec<T>::type *__restrict__ det_med,
                                              double *__restrict__ det_w)
{
    using V = typename cvec<T>::type;
    const int na = __popcll(mk);
    V med; med.x = mr; med.y = mi;
    if (det_med) det_med[e] = med;
    V out = med;
    const bool avg = postproc && na > 0;
    if (avg) {
        out.x = sum_r / (T)na;
        out.y = sum_i / (T)na;
    }
    det_coef[e] = out;
    if (det_w) {
        double *w = det_w + e * L * 2;
        for (int l = 0; l < L; ++l) {
            double wr = 0.0, wi = 0.0;
            if (avg) {
                if ((mk >> l) & 1ull) { wr = 1.0 / na; wi = 1.0 / na; }
            } else if (L & 1) {
                wr = (l == r0) ? 1.0 : 0.0;
                wi = (l == i0) ? 1.0 : 0.0;
            } else {
                wr = 0.5 * ((l == r0) + (l == r1));
                wi = 0.5 * ((l == i0) + (l == i1));
            }
            w[2 * l] = wr;
            w[2 * l + 1] = wi;
        }
    }
}

__device__ __forceinline__ uint64_t load_mask(const uint32_t *__restrict__ mask, int64_t e, int L)
{
    const int W = mask_words(L);
    uint64_t mk = mask[e * W];
    if (W > 1) mk |= (uint64_t)mask[e * W + 1] << 32;
    return mk;
}

// Up to LMAX <= 40 lattices: the values stay in registers.  TW (long lists): the
// singleton mask is formed here from the merged `twice` bitmaps and the buckets already
// loaded for the gather, and written whole, instead of being read.
template <typename T, int LMAX, bool TW>
__global__ __launch_bounds__(256) void k_combine(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ n_det, int64_t cap,
    const int32_t *__restrict__ det_hash, uint32_t *__restrict__ mask,
    const typename cvec<T>::type *__restrict__ ghat, int postproc,
    typename cvec<T>::type *__restrict__ det_coef, typename cvec<T>::type *__restrict__ det_med,
    double *__restrict__ det_w, const uint32_t *__restrict__ g_twice, int64_t wl)
{
    using V = typename cvec<T>::type;
    int f = blockIdx.y, bx = blockIdx.x;
    if ((gridDim.x * gridDim.y) % 8 == 0) {
        // workgroups are dealt to the 8 XCDs in turn; renumbered so that each XCD takes a
        // contiguous range of (function, block) pairs, i.e. the lattice values of few
        // functions, which its L2 then holds (whenever the count is a multiple of 8; the
        // host rounds it up for long lists)
        const int G = gridDim.x * gridDim.y, w = blockIdx.y * gridDim.x + blockIdx.x;
        const int i = (w & 7) * (G >> 3) + (w >> 3);
        f = i / gridDim.x;
        bx = i - f * gridDim.x;
    }
    const int64_t n = n_of(n_det, f, cap);
    for (int64_t q = bx * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = (int64_t)f * cap + q;
    T vr[LMAX], vi[LMAX];
    int32_t hl[TW ? LMAX : 1];
    const T inf = __builtin_inf();
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
        vr[l] = inf; vi[l] = inf;
        if (l < L) {
            const int32_t h = det_hash[e * L + l];
            if constexpr (TW) hl[l] = h;
            const V g = ghat[lat[f * L + l].node_off + h];
            vr[l] = g.x; vi[l] = g.y;
        }
    }
    T mr, mi;
    int r0, r1, i0, i1;
    median_sel<T, LMAX>(vr, L, mr, r0, r1);
    median_sel<T, LMAX>(vi, L, mi, i0, i1);
    uint64_t mk = 0;
    if constexpr (TW) {
        const uint32_t *gt = g_twice + (int64_t)f * L * wl;
#pragma unroll
        for (int l = 0; l < LMAX; ++l)
            if (l < L && !((gt[(int64_t)l * wl + (hl[l] >> 5)] >> (hl[l] & 31)) & 1u)) mk |= 1ull << l;
        const int W = mask_words(L);
        mask[e * W] = (uint32_t)mk;
        if (W > 1) mask[e * W + 1] = (uint32_t)(mk >> 32);
    } else {
        mk = load_mask(mask, e, L);
    }
    T sr = 0, si = 0;
#pragma unroll
    for (int l = 0; l < LMAX; ++l)
        if (l < L && ((mk >> l) & 1ull)) { sr += vr[l]; si += vi[l]; }
    combine_store<T>(L, e, mk, mr, mi, sr, si, r0, r1, i0, i1, postproc, det_coef, det_med, det_w);
    }
}

// 41..64 lattices: each lane keeps its values in its own column of an LDS array
// ([lattice][lane], one wavefront per block) and indexes it freely; no lane reads
// another lane's column, so no barrier is needed.  Same ranks as median_sel.
template <typename T>
__global__ __launch_bounds__(64) void k_combine_wide(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ n_det, int64_t cap,
    const int32_t *__restrict__ det_hash, const uint32_t *__restrict__ mask,
    const typename cvec<T>::type *__restrict__ ghat, int postproc,
    typename cvec<T>::type *__restrict__ det_coef, typename cvec<T>::type *__restrict__ det_med,
    double *__restrict__ det_w)
{
    using V = typename cvec<T>::type;
    __shared__ T cr[kMaxL][64], ci[kMaxL][64];
    const int f = blockIdx.y, t = threadIdx.x;
    const int64_t n = n_of(n_det, f, cap);
    for (int64_t q = blockIdx.x * (int64_t)64 + t; q < n; q += (int64_t)gridDim.x * 64) {
    const int64_t e = (int64_t)f * cap + q;
    for (int l = 0; l < L; ++l) {
        const V g = ghat[lat[f * L + l].node_off + det_hash[e * L + l]];
        cr[l][t] = g.x;
        ci[l][t] = g.y;
    }
    const int w0 = (L - 1) / 2, w1 = L / 2;
    int r0 = 0, r1 = 0, i0 = 0, i1 = 0;
    for (int l = 0; l < L; ++l) {
        const T a = cr[l][t], b = ci[l][t];
        int rr = 0, ri = 0;
        for (int m = 0; m < L; ++m) {
            const T am = cr[m][t], bm = ci[m][t];
            rr += (am < a) || (am == a && m < l);
            ri += (bm < b) || (bm == b && m < l);
        }
        if (rr == w0) r0 = l;
        if (rr == w1) r1 = l;
        if (ri == w0) i0 = l;
        if (ri == w1) i1 = l;
    }
    const T mr = (L & 1) ? cr[r0][t] : T(0.5) * (cr[r0][t] + cr[r1][t]);
    const T mi = (L & 1) ? ci[i0][t] : T(0.5) * (ci[i0][t] + ci[i1][t]);
    const uint64_t mk = load_mask(mask, e, L);
    T sr = 0, si = 0;
    for (int l = 0; l < L; ++l)
        if ((mk >> l) & 1ull) { sr += cr[l][t]; si += ci[l][t]; }
    combine_store<T>(L, e, mk, mr, mi, sr, si, r0, r1, i0, i1, postproc, det_coef, det_med, det_w);
    }
}

// ------------------------------------------------------------------ limit (Algorithm 4)
// Dynamic LDS: pow2ceil(cap) x 12 bytes (the sort's exchange arrays).
template <typename T>
__device__ __forceinline__ uint64_t limit_key(typename cvec<T>::type c, T th2, bool &pass)
{
    const T m2 = c.x * c.x + c.y * c.y;
    pass = m2 >= th2;
    return pass ? ~(uint64_t)__double_as_longlong((double)m2) : ~0ull;   // m2 >= 0: bits are monotonic
}

// The entries with |p| >= theta are first compacted to the front of the LDS arrays
// (a block scan keeps them in list order), so the sort runs over pow2ceil(#passing)
// pairs only; the others would sort after them anyway.
template <typename T, int E>
__global__ __launch_bounds__(kSortThreads) void k_limit(
    const int64_t *__restrict__ n_det, int64_t cap, const int64_t *__restrict__ det_idx,
    const typename cvec<T>::type *__restrict__ det_coef, T th2, int64_t s_cap, int64_t *__restrict__ n_out,
    int64_t *__restrict__ out_idx, typename cvec<T>::type *__restrict__ out_coef, int32_t *__restrict__ out_pos)
{
    using V = typename cvec<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wsum[kSortThreads / 64];
    __shared__ int npass;
    const int f = blockIdx.x, t = threadIdx.x;
    const int n = (int)n_of(n_det, f, cap);
    const int Pn = sort_len(n, E);
    uint64_t *lk = reinterpret_cast<uint64_t *>(smem);
    int32_t *lv = reinterpret_cast<int32_t *>(lk + Pn);
    const V *dc = det_coef + (int64_t)f * cap;
    uint64_t k[E];
    int32_t v[E];
    bool ps[E];
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = t * E + e;
        ps[e] = false;
        k[e] = ~0ull;
        if (p < n) k[e] = limit_key<T>(dc[p], th2, ps[e]);
        cnt += ps[e];
    }
    int o = block_excl_scan(cnt, wsum);
    if (t == kSortThreads - 1) npass = o + cnt;
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (ps[e]) {
            lk[o] = k[e];
            lv[o] = t * E + e;
            ++o;
        }
    __syncthreads();
    const int np = npass;
    const int P = sort_len(np, E);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = t * E + e;
        k[e] = p < np ? lk[p] : ~0ull;
        v[e] = p < np ? lv[p] : INT32_MAX;
    }
    __syncthreads();   // the sort's exchanges reuse the arrays
    block_bitonic<E>(k, v, P, lk, lv);
    const int64_t no = min((int64_t)np, s_cap);
    if (t == 0) n_out[f] = no;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int o2 = t * E + e;
        if (o2 < no) {
            const int q = v[e];
            out_idx[(int64_t)f * s_cap + o2] = det_idx[(int64_t)f * cap + q];
            out_coef[(int64_t)f * s_cap + o2] = dc[q];
            if (out_pos) out_pos[(int64_t)f * s_cap + o2] = q;
        }
    }
}

// ------------------------------------------------------------------ global sort (large lists)
// Detected lists longer than one workgroup's LDS sort (cap > 8192) are ordered by a
// bitonic sort of (key, position) pairs in global memory, one segment of P = 2^e
// pairs per function, ascending by (key, position).  Stages with a partner
// distance of at most kGsortLocal / 2 run inside one workgroup's LDS.
constexpr int kGsortLocal = 2048;   // pairs per workgroup in the LDS stages

__device__ __forceinline__ void gs_cmpswap(uint64_t &ka, int32_t &pa, uint64_t &kb, int32_t &pb, bool asc)
{
    const bool gt = (ka > kb) || (ka == kb && pa > pb);
    if (gt == asc) {
        const uint64_t tk = ka; ka = kb; kb = tk;
        const int32_t tp = pa; pa = pb; pb = tp;
    }
}

// One stage (k, j) with j >= kGsortLocal / 2 over every segment.
__global__ __launch_bounds__(256) void k_gsort_global(uint64_t *__restrict__ key, int32_t *__restrict__ pos,
                                                      int64_t P, int64_t k, int64_t j)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= P / 2) return;
    const int64_t base = (int64_t)blockIdx.y * P;
    const int64_t i = 2 * t - (t & (j - 1));   // lower element of the pair
    const int64_t x = base + i, y = x + j;
    uint64_t ka = key[x], kb = key[y];
    int32_t pa = pos[x], pb = pos[y];
    gs_cmpswap(ka, pa, kb, pb, (i & k) == 0);
    key[x] = ka; key[y] = kb;
    pos[x] = pa; pos[y] = pb;
}

// All stages of merge size k with j < kGsortLocal, or (k0 == 0) the whole sort
// up to merge size kGsortLocal, on blocks of kGsortLocal pairs in LDS.
__global__ __launch_bounds__(kGsortLocal / 2) void k_gsort_local(uint64_t *__restrict__ key,
                                                                 int32_t *__restrict__ pos, int64_t P, int64_t k0)
{
    __shared__ uint64_t sk[kGsortLocal];
    __shared__ int32_t sp[kGsortLocal];
    const int64_t base = (int64_t)blockIdx.y * P + (int64_t)blockIdx.x * kGsortLocal;
    const int n = (int)min((int64_t)kGsortLocal, P);
    for (int i = threadIdx.x; i < n; i += blockDim.x) { sk[i] = key[base + i]; sp[i] = pos[base + i]; }
    __syncthreads();
    const int64_t off = (int64_t)blockIdx.x * kGsortLocal;   // position of the block in its segment
    const int64_t kfirst = k0 ? k0 : 2;
    const int64_t klast = k0 ? k0 : (int64_t)n;
    for (int64_t k = kfirst; k <= klast; k <<= 1) {
        for (int64_t j = (k0 ? min(k0, (int64_t)n) : k) >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
                const int i = 2 * t - (t & ((int)j - 1));
                gs_cmpswap(sk[i], sp[i], sk[i + j], sp[i + j], ((off + i) & k) == 0);
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) { key[base + i] = sk[i]; pos[base + i] = sp[i]; }
}

// Sorts F segments of P (a power of two) pairs.
int gsort_run(Plan &p, uint64_t *key, int32_t *pos, int64_t P)
{
    if (P <= 1) return MR1L_OK;
    const int64_t lb = std::min<int64_t>(P, kGsortLocal);
    const dim3 gl((unsigned)(P / lb), (unsigned)p.F);
    hipLaunchKernelGGL(k_gsort_local, gl, dim3(kGsortLocal / 2), 0, p.stream, key, pos, P, (int64_t)0);
    MR1L_LAUNCH_CHECK();
    for (int64_t k = 2 * kGsortLocal; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j >= kGsortLocal; j >>= 1) {
            const dim3 g((unsigned)((P / 2 + 255) / 256), (unsigned)p.F);
            hipLaunchKernelGGL(k_gsort_global, g, dim3(256), 0, p.stream, key, pos, P, k, j);
            MR1L_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_gsort_local, gl, dim3(kGsortLocal / 2), 0, p.stream, key, pos, P, k);
        MR1L_LAUNCH_CHECK();
    }
    return MR1L_OK;
}

// Ascending order of a long detected list without a sort: the detected candidates
// set their bits in a bitmap over the concatenated candidate sets, and an ordered
// compaction of each function's range of bits writes them back in index order
// (counts per block of 1024 words, a scan of the counts, then the emission).
constexpr int kFlagWordsPerBlock = 1024;   // 256 threads x 4 words

// The vote appends each wave's detections as an ascending run, so the entries of a word
// mostly sit in adjacent lanes: each lane ORs in the bits of the lanes after it that hit
// the same word (a suffix OR over 32 lanes), and only the first lane of each such group
// issues the atomic.  Lanes of one group that are not adjacent still set their own word.
__global__ __launch_bounds__(256) void k_flag_det(const int64_t *__restrict__ n_det, int64_t cap,
                                                  const int64_t *__restrict__ det_idx,
                                                  const int64_t *__restrict__ set_off, uint32_t *__restrict__ flags)
{
    const int f = blockIdx.y;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = q < n_of(n_det, f, cap);
    const int64_t c = act ? set_off[f] + det_idx[(int64_t)f * cap + q] : -64;
    const int64_t w = c >> 5;   // lanes past the list: word -2, never a real one
    uint32_t b = act ? 1u << (c & 31) : 0u;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
        const uint32_t nb = __shfl_down(b, o);
        const int64_t nw = __shfl_down(w, o);
        if (lane + o < 64 && nw == w) b |= nb;
    }
    const int64_t pw = __shfl_up(w, 1);
    if (act && (lane == 0 || pw != w)) atomicOr(flags + w, b);
}

// bits of word w that belong to the candidate range [lo, hi)
__device__ __forceinline__ uint32_t flag_word(const uint32_t *flags, int64_t w, int64_t lo, int64_t hi)
{
    const int64_t b0 = w * 32;
    if (b0 + 32 <= lo || b0 >= hi) return 0u;
    uint32_t v = flags[w];
    if (lo > b0) v &= ~0u << (lo - b0);
    if (hi < b0 + 32) v &= (1u << (hi - b0)) - 1u;
    return v;
}

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        const int a = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += a;
        __syncthreads();
    }
    const int incl = sh[tid];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void k_flag_count(const int64_t *__restrict__ set_off,
                                                    const uint32_t *__restrict__ flags, int nx,
                                                    int32_t *__restrict__ cnt)
{
    __shared__ int sh[256];
    const int f = blockIdx.y;
    const int64_t lo = set_off[f], hi = set_off[f + 1];
    const int64_t wb = (lo >> 5) + (int64_t)blockIdx.x * kFlagWordsPerBlock + threadIdx.x * 4;
    int c = 0;
    for (int k = 0; k < 4; ++k) c += __popc(flag_word(flags, wb + k, lo, hi));
    const int before = block_exclusive_scan(c, sh);
    if (threadIdx.x == blockDim.x - 1) cnt[(int64_t)f * nx + blockIdx.x] = before + c;
}

__global__ __launch_bounds__(64) void k_flag_scan(int nx, int32_t *__restrict__ cnt)
{
    if (threadIdx.x != 0) return;
    int32_t *c = cnt + (int64_t)blockIdx.x * nx;
    int acc = 0;
    for (int x = 0; x < nx; ++x) {
        const int v = c[x];
        c[x] = acc;
        acc += v;
    }
}

__global__ __launch_bounds__(256) void k_flag_emit(const int64_t *__restrict__ set_off,
                                                   const uint32_t *__restrict__ flags, int nx,
                                                   const int32_t *__restrict__ off, int64_t cap,
                                                   int64_t *__restrict__ det_idx)
{
    __shared__ int sh[256];
    const int f = blockIdx.y;
    const int64_t lo = set_off[f], hi = set_off[f + 1];
    const int64_t wb = (lo >> 5) + (int64_t)blockIdx.x * kFlagWordsPerBlock + threadIdx.x * 4;
    uint32_t v[4];
    int c = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = flag_word(flags, wb + k, lo, hi);
        c += __popc(v[k]);
    }
    int64_t r = off[(int64_t)f * nx + blockIdx.x] + block_exclusive_scan(c, sh);
    for (int k = 0; k < 4; ++k) {
        uint32_t b = v[k];
        while (b) {
            const int j = __ffs(b) - 1;
            b &= b - 1;
            if (r < cap) det_idx[(int64_t)f * cap + r] = (wb + k) * 32 + j - lo;
            ++r;
        }
    }
}

// Algorithm 4 keys of a long list: ~bits(|p|^2) for |p|^2 >= theta^2 (ascending key =
// descending modulus), the position as tie-break; others sort last.
template <typename T>
__global__ __launch_bounds__(256) void k_limit_keys(const int64_t *__restrict__ n_det, int64_t cap,
                                                    const typename cvec<T>::type *__restrict__ det_coef, T th2,
                                                    int64_t P, uint64_t *__restrict__ key, int32_t *__restrict__ pos)
{
    using V = typename cvec<T>::type;
    const int f = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= P) return;
    uint64_t k = ~0ull;
    int32_t ps = INT32_MAX;
    if (i < n_of(n_det, f, cap)) {
        const V c = det_coef[(int64_t)f * cap + i];
        const T m2 = c.x * c.x + c.y * c.y;
        if (m2 >= th2) {
            k = ~(uint64_t)__double_as_longlong((double)m2);
            ps = (int32_t)i;
        }
    }
    key[(int64_t)f * P + i] = k;
    pos[(int64_t)f * P + i] = ps;
}

template <typename T>
__global__ __launch_bounds__(256) void k_limit_emit(int64_t cap,
                                                    const int64_t *__restrict__ det_idx,
                                                    const typename cvec<T>::type *__restrict__ det_coef, int64_t P,
                                                    const int32_t *__restrict__ pos, int64_t s_cap,
                                                    int64_t *__restrict__ n_out, int64_t *__restrict__ out_idx,
                                                    typename cvec<T>::type *__restrict__ out_coef,
                                                    int32_t *__restrict__ out_pos)
{
    const int f = blockIdx.y;
    const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    // the passing entries sort first (their positions are below INT32_MAX): the
    // output length is the first failing position among the first s~
    const int32_t *pf = pos + (int64_t)f * P;
    int64_t lo = 0, hi = min(P, s_cap);
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (pf[mid] != INT32_MAX) lo = mid + 1; else hi = mid;
    }
    const int64_t no = lo;
    if (o == 0) n_out[f] = no;
    if (o >= no) return;
    const int32_t q = pf[o];
    out_idx[(int64_t)f * s_cap + o] = det_idx[(int64_t)f * cap + q];
    out_coef[(int64_t)f * s_cap + o] = det_coef[(int64_t)f * cap + q];
    if (out_pos) out_pos[(int64_t)f * s_cap + o] = q;
}

// ------------------------------------------------------------------ adjoint scatter
template <typename T>
__global__ __launch_bounds__(256) void k_adjoint_scatter(
    const LatDesc *__restrict__ lat, int L, int64_t cap, int64_t s_cap, const int64_t *__restrict__ n_out,
    const int32_t *__restrict__ out_pos, const int32_t *__restrict__ det_hash, const double *__restrict__ det_w,
    const typename cvec<T>::type *__restrict__ grad, T *__restrict__ gbar)
{
    const int f = blockIdx.y;
    const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (o >= n_out[f]) return;
    const auto g = grad[(int64_t)f * s_cap + o];
    const int64_t e = (int64_t)f * cap + out_pos[(int64_t)f * s_cap + o];
    for (int l = 0; l < L; ++l) {
        const double wr = det_w[(e * L + l) * 2], wi = det_w[(e * L + l) * 2 + 1];
        if (wr == 0.0 && wi == 0.0) continue;
        const int64_t node = lat[f * L + l].node_off + det_hash[e * L + l];
        if (wr != 0.0) unsafeAtomicAdd(gbar + 2 * node, (T)(wr * (double)g.x));
        if (wi != 0.0) unsafeAtomicAdd(gbar + 2 * node + 1, (T)(wi * (double)g.y));
    }
}

// ------------------------------------------------------------------ selection (long lists)
// Algorithm 4 on a long list keeps at most s~ entries: the s~-th smallest key of the
// function (keys as k_limit_keys writes them, failing entries ~0) is found by an
// 8-round radix selection, 8 bits per round from the top (per-block LDS histograms of
// the keys that match the prefix found so far, then the digit where the cumulative
// count reaches the remaining rank); an ordered compaction then keeps the entries
// below it and, among those equal to it, the first ones by position, so only
// min(s~, #passing) pairs are sorted.
struct SelState {
    uint64_t prefix, mask;
    int64_t kk;    // rank still to reach among the keys matching the prefix
    int64_t pad;   // after the scan: the number of keys below the threshold
};

__global__ void k_sel_init(int F, const int64_t *__restrict__ n_det, int64_t cap, int64_t s_cap,
                           SelState *__restrict__ st, uint32_t *__restrict__ hist)
{
    const int f = blockIdx.x;
    if (f >= F) return;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[(int64_t)f * 256 + i] = 0u;
    if (threadIdx.x == 0) {
        st[f].prefix = 0;
        st[f].mask = 0;
        st[f].kk = min(s_cap, n_of(n_det, f, cap));
    }
}

__global__ __launch_bounds__(256) void k_sel_hist(const int64_t *__restrict__ n_det, int64_t cap, int64_t P,
                                                  const uint64_t *__restrict__ key, int shift,
                                                  const SelState *__restrict__ st, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    const int f = blockIdx.y;
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t n = n_of(n_det, f, cap);
    const uint64_t pre = st[f].prefix, msk = st[f].mask;
    // the keys share their top digits in the first rounds: the lanes of a wave with
    // the same digit add their count with one atomic (one pass per distinct digit)
    if (st[f].kk > 0) {
        const int lane = threadIdx.x & 63;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63);
        for (int64_t w0 = i0; w0 < n; w0 += stride) {   // whole waves take part
            const int64_t i = w0 + lane;
            uint64_t k = 0;
            bool m = false;
            if (i < n) {
                k = key[(int64_t)f * P + i];
                m = (k & msk) == pre;
            }
            const uint32_t dg = (uint32_t)(k >> shift) & 255u;
            uint64_t act = __ballot(m);
            while (act) {
                const int leader = __ffsll((unsigned long long)act) - 1;
                const uint32_t dl = (uint32_t)__shfl((int)dg, leader);
                const uint64_t same = __ballot(m && dg == dl);
                if (lane == leader) atomicAdd(&h[dl], (uint32_t)__popcll(same));
                act &= ~same;
            }
        }
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd(hist + (int64_t)f * 256 + threadIdx.x, c);
}

// one workgroup of 256 threads per function: the digit whose cumulative count first
// reaches the remaining rank (a block scan of the 256 bins), then the bins cleared
__global__ __launch_bounds__(256) void k_sel_pick(int shift, SelState *__restrict__ st, uint32_t *__restrict__ hist)
{
    __shared__ int wsum[kSortThreads / 64];
    __shared__ int pick;
    const int f = blockIdx.x, t = threadIdx.x;
    uint32_t *h = hist + (int64_t)f * 256;
    const int64_t kk = st[f].kk;
    const int c = (int)h[t];
    const int below = block_excl_scan(c, wsum);
    if (t == 0) pick = 255;
    __syncthreads();
    if (kk > 0 && (int64_t)below < kk && (int64_t)below + c >= kk) pick = t;   // exactly one thread
    __syncthreads();
    h[t] = 0u;
    if (t == pick && kk > 0) {
        st[f].kk = kk - below;
        st[f].prefix |= (uint64_t)t << shift;
        st[f].mask |= (uint64_t)255u << shift;
    }
}

// per block of kSortThreads entries: how many keys are below the threshold T and how
// many equal it (equal ones only when T is a passing key)
__global__ __launch_bounds__(kSortThreads) void k_sel_count(const int64_t *__restrict__ n_det, int64_t cap, int64_t P,
                                                            const uint64_t *__restrict__ key,
                                                            const SelState *__restrict__ st, int nb,
                                                            int32_t *__restrict__ cnt)
{
    __shared__ int wsum[kSortThreads / 64];
    const int f = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)kSortThreads + threadIdx.x;
    const int64_t n = n_of(n_det, f, cap);
    const uint64_t T = st[f].prefix;
    int lt = 0, eq = 0;
    if (i < n) {
        const uint64_t k = key[(int64_t)f * P + i];
        lt = k < T;
        eq = (k == T) && (T != ~0ull);
    }
    const int a = block_excl_scan(lt, wsum);
    __syncthreads();
    const int b = block_excl_scan(eq, wsum);
    if (threadIdx.x == kSortThreads - 1) {
        cnt[((int64_t)f * nb + blockIdx.x) * 2] = a + lt;
        cnt[((int64_t)f * nb + blockIdx.x) * 2 + 1] = b + eq;
    }
}

// exclusive offsets of the blocks' counts (one workgroup per function, kSortThreads
// blocks' counts at a time); n_sel[f] = the number of pairs kept
__global__ __launch_bounds__(kSortThreads) void k_sel_scan(int nb, const SelState *__restrict__ st,
                                                           int32_t *__restrict__ cnt, int64_t *__restrict__ n_sel)
{
    __shared__ int wsum[kSortThreads / 64];
    __shared__ int64_t tot[2];
    const int f = blockIdx.x, t = threadIdx.x;
    int32_t *c = cnt + (int64_t)f * nb * 2;
    if (t == 0) { tot[0] = 0; tot[1] = 0; }
    __syncthreads();
    for (int x0 = 0; x0 < nb; x0 += kSortThreads) {
        const int x = x0 + t;
        const int ca = x < nb ? c[2 * x] : 0, cb = x < nb ? c[2 * x + 1] : 0;
        const int ea = block_excl_scan(ca, wsum);
        __syncthreads();
        const int eb = block_excl_scan(cb, wsum);
        const int64_t ba = tot[0], bb = tot[1];
        if (x < nb) {
            c[2 * x] = (int32_t)(ba + ea);
            c[2 * x + 1] = (int32_t)(bb + eb);
        }
        __syncthreads();
        if (t == kSortThreads - 1) { tot[0] = ba + ea + ca; tot[1] = bb + eb + cb; }
        __syncthreads();
    }
    if (t == 0) {
        const bool pass_t = st[f].prefix != ~0ull;
        n_sel[f] = tot[0] + (pass_t ? min(st[f].kk, tot[1]) : 0);
    }
}

// the kept pairs, in position order: keys below T first, then the first kk equal to T
__global__ __launch_bounds__(kSortThreads) void k_sel_emit(const int64_t *__restrict__ n_det, int64_t cap, int64_t P,
                                                           const uint64_t *__restrict__ key,
                                                           const int32_t *__restrict__ pos,
                                                           const SelState *__restrict__ st, int nb,
                                                           const int32_t *__restrict__ cnt, int64_t S,
                                                           uint64_t *__restrict__ okey, int32_t *__restrict__ opos)
{
    __shared__ int wsum[kSortThreads / 64];
    const int f = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)kSortThreads + threadIdx.x;
    const int64_t n = n_of(n_det, f, cap);
    const uint64_t T = st[f].prefix;
    const int64_t kk = st[f].kk;
    uint64_t k = ~0ull;
    int lt = 0, eq = 0;
    if (i < n) {
        k = key[(int64_t)f * P + i];
        lt = k < T;
        eq = (k == T) && (T != ~0ull);
    }
    const int a = block_excl_scan(lt, wsum);
    __syncthreads();
    const int b = block_excl_scan(eq, wsum);
    const int32_t *c = cnt + ((int64_t)f * nb + blockIdx.x) * 2;
    if (lt) {
        const int64_t o = c[0] + a;
        okey[(int64_t)f * S + o] = k;
        opos[(int64_t)f * S + o] = pos[(int64_t)f * P + i];
    } else if (eq) {
        const int64_t r = c[1] + b;
        if (r < kk) {
            const int64_t o = st[f].pad + r;   // after all keys below T
            okey[(int64_t)f * S + o] = k;
            opos[(int64_t)f * S + o] = pos[(int64_t)f * P + i];
        }
    }
}

// number of keys below the threshold (the kept entries equal to it go after them)
__global__ void k_sel_below(int F, int nb, SelState *__restrict__ st, const int64_t *__restrict__ n_sel)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const bool pass_t = st[f].prefix != ~0ull;
    // n_sel = below + min(kk, equal) when T passes, else below
    st[f].pad = n_sel[f] - (pass_t ? st[f].kk : 0);
}

// Algorithm 4's order over the kept pairs of each function (at most E x kSortThreads),
// one workgroup per function; dynamic LDS pow2ceil(S) x 12 bytes.
template <typename T, int E>
__global__ __launch_bounds__(kSortThreads) void k_limit_sel(int64_t cap, const int64_t *__restrict__ det_idx,
                                                            const typename cvec<T>::type *__restrict__ det_coef,
                                                            const int64_t *__restrict__ n_sel, int64_t S,
                                                            const uint64_t *__restrict__ skey,
                                                            const int32_t *__restrict__ spos, int64_t s_cap,
                                                            int64_t *__restrict__ n_out, int64_t *__restrict__ out_idx,
                                                            typename cvec<T>::type *__restrict__ out_coef,
                                                            int32_t *__restrict__ out_pos)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int f = blockIdx.x, t = threadIdx.x;
    const int np = (int)n_sel[f];
    const int P = sort_len(np, E);
    uint64_t *lk = reinterpret_cast<uint64_t *>(smem);
    int32_t *lv = reinterpret_cast<int32_t *>(lk + P);
    uint64_t k[E];
    int32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = t * E + e;
        k[e] = p < np ? skey[(int64_t)f * S + p] : ~0ull;
        v[e] = p < np ? spos[(int64_t)f * S + p] : INT32_MAX;
    }
    block_bitonic<E>(k, v, P, lk, lv);
    const int64_t no = min((int64_t)np, s_cap);
    if (t == 0) n_out[f] = no;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int o = t * E + e;
        if (o < no) {
            const int q = v[e];
            out_idx[(int64_t)f * s_cap + o] = det_idx[(int64_t)f * cap + q];
            out_coef[(int64_t)f * s_cap + o] = det_coef[(int64_t)f * cap + q];
            if (out_pos) out_pos[(int64_t)f * s_cap + o] = q;
        }
    }
}

// ------------------------------------------------------------------ host
// g_twice (long lists): the merged `twice` bitmaps, wl words per lattice, from which the
// singleton masks are formed (by the combine kernel itself up to 40 lattices).
template <typename T>
static int combine_launch(Plan &p, const int64_t *n_det, int64_t cap, int64_t nmax, const int32_t *det_hash,
                          uint32_t *mask, const void *ghat, int postproc, void *det_coef, void *det_med,
                          double *det_w, int64_t scale, const uint32_t *g_twice, int64_t wl)
{
    using V = typename cvec<T>::type;
    // a bounded number of workgroups per function (the kernels loop): most functions' lists
    // are far shorter than the capacity, and launching a workgroup per 256 entries of it
    // cost more than the work; long lists (scale > 1) need more waves in flight, since
    // every entry gathers L scattered lattice values
    dim3 grid(tail_blocks((nmax + 255) / 256, p.F, scale), (unsigned)p.F), blk(256);
    if (g_twice) grid.x = (grid.x + 7) & ~7u;   // the long-list kernel's XCD renumbering
#define MR1L_COMB(LM)                                                                                          \
    if (g_twice)                                                                                               \
        hipLaunchKernelGGL((k_combine<T, LM, true>), grid, blk, 0, p.stream, p.d_lat, p.L, n_det, cap, det_hash, \
                           mask, (const V *)ghat, postproc, (V *)det_coef, (V *)det_med, det_w, g_twice, wl);    \
    else                                                                                                       \
        hipLaunchKernelGGL((k_combine<T, LM, false>), grid, blk, 0, p.stream, p.d_lat, p.L, n_det, cap,         \
                           det_hash, mask, (const V *)ghat, postproc, (V *)det_coef, (V *)det_med, det_w,       \
                           nullptr, (int64_t)0)
    if (p.L <= 8) MR1L_COMB(8);
    else if (p.L <= 12) MR1L_COMB(12);
    else if (p.L <= 16) MR1L_COMB(16);
    else if (p.L <= 20) MR1L_COMB(20);
    else if (p.L <= 24) MR1L_COMB(24);
    else if (p.L <= 32) MR1L_COMB(32);
    else if (p.L <= 40) MR1L_COMB(40);
    else {
        if (g_twice) {
            hipLaunchKernelGGL(k_single_mask, dim3((unsigned)((nmax + 255) / 256), (unsigned)p.F), dim3(256), 0,
                               p.stream, p.d_lat, p.L, n_det, cap, det_hash, wl, g_twice, mask);
            MR1L_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_combine_wide<T>, dim3(tail_blocks((nmax + 63) / 64, p.F, 4), (unsigned)p.F), dim3(64), 0, p.stream,
                           p.d_lat, p.L, n_det, cap, det_hash, mask, (const V *)ghat, postproc, (V *)det_coef,
                           (V *)det_med, det_w);
    }
#undef MR1L_COMB
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

template <int E>
static int sort_attrs()
{
    // dynamic LDS at the largest capacity (static LDS comes on top of it)
    const void *ks[] = {(const void *)k_sort_det<E>, (const void *)k_limit<double, E>, (const void *)k_limit<float, E>,
                        (const void *)k_limit_sel<double, E>, (const void *)k_limit_sel<float, E>};
    for (const void *k : ks)
        MR1L_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     std::max(kMaxCap * 12, kSortBitmapBytes)));
    return MR1L_OK;
}

int extract_init_attrs()
{
    const std::pair<const void *, int> ks[] = {
        {(const void *)k_singleton, 2 * kSingleWords * (int)sizeof(uint32_t)},
        {(const void *)k_single_count, 2 * kSingleWords * (int)sizeof(uint32_t)},
        {(const void *)k_single_count_grp, 2 * kSingleWords * (int)sizeof(uint32_t)}};
    for (const auto &k : ks) MR1L_HIP(hipFuncSetAttribute(k.first, hipFuncAttributeMaxDynamicSharedMemorySize, k.second));
    int rc = sort_attrs<1>();
    if (!rc) rc = sort_attrs<2>();
    if (!rc) rc = sort_attrs<4>();
    if (!rc) rc = sort_attrs<8>();
    return rc;
}

static int64_t pow2ceil(int64_t n)
{
    int64_t P = 1;
    while (P < n) P <<= 1;
    return P;
}

// Values per thread of the block sorts for capacity cap <= kMaxCap: pow2ceil(cap) /
// kSortThreads, at least 1.
static int sort_e(int64_t cap)
{
    return (int)std::max<int64_t>(1, pow2ceil(std::max<int64_t>(cap, 1)) / kSortThreads);
}
#define MR1L_BY_E(E_, X)           \
    switch (E_) {                  \
    case 1: X(1); break;           \
    case 2: X(2); break;           \
    case 4: X(4); break;           \
    default: X(8); break;          \
    }

// Register arrays of the per-candidate kernels sized to the next of 8, 12, ..., 64 lattices.
#define MR1L_BY_L(L_, X)                         \
    if ((L_) <= 8) X(8);                         \
    else if ((L_) <= 12) X(12);                  \
    else if ((L_) <= 16) X(16);                  \
    else if ((L_) <= 20) X(20);                  \
    else if ((L_) <= 24) X(24);                  \
    else if ((L_) <= 32) X(32);                  \
    else if ((L_) <= 40) X(40);                  \
    else X(64);

static int grow_sort(Plan &p, int64_t P)
{
    const int64_t bytes = p.F * P * 12;
    if (p.gsort_bytes >= bytes && p.d_gsort) return MR1L_OK;
    if (p.capturing) return fail(MR1L_E_ARG, "lists longer than 8192 cannot be recorded in a graph");
    p.gsort_bytes = 0;
    const int rc = plan_regrow(p, (void **)&p.d_gsort, (size_t)bytes);
    if (rc) return rc;
    p.gsort_bytes = bytes;
    return MR1L_OK;
}

// Algorithm 4 on a long list (sort buffers sized for P >= every function's count,
// nmax the longest count): lists that fit one workgroup take the block sort; longer
// ones keep min(s~, #passing) pairs by a radix selection and sort only those (in one
// workgroup when they fit it, else by the global sort).
static int limit_short(Plan &p, const int64_t *n_det, int64_t cap, const int64_t *det_idx, const void *det_coef,
                       double theta, int64_t s_cap, int64_t *n_out, int64_t *out_idx, void *out_coef, int32_t *out_pos,
                       int64_t nmax);

static int limit_long(Plan &p, const int64_t *n_det, int64_t cap, const int64_t *det_idx, const void *det_coef,
                      double theta, int64_t s_cap, int64_t *n_out, int64_t *out_idx, void *out_coef,
                      int32_t *out_pos, int64_t P, int64_t nmax)
{
    if (nmax <= kMaxCap)
        return limit_short(p, n_det, cap, det_idx, det_coef, theta, s_cap, n_out, out_idx, out_coef, out_pos, nmax);
    const int64_t F = p.F;
    const int64_t S = pow2ceil(std::min(s_cap, nmax));   // kept pairs per function, padded
    const int nb = (int)((nmax + kSortThreads - 1) / kSortThreads);
    // sort buffers [F][P] keys + positions, then [F][S] kept pairs, the histograms, the
    // selection states, the block counts and the kept counts
    const int64_t b_keys = F * P * 12, b_kept = F * S * 12, b_hist = F * 256 * 4;
    const int64_t b_st = F * (int64_t)sizeof(SelState), b_cnt = F * nb * 8, b_nsel = F * 8;
    const int64_t bytes = b_keys + b_kept + b_hist + b_st + b_cnt + b_nsel + 64;
    if (p.gsort_bytes < bytes || !p.d_gsort) {
        if (p.capturing) return fail(MR1L_E_ARG, "lists longer than 8192 cannot be recorded in a graph");
        p.gsort_bytes = 0;
        if (int rc = plan_regrow(p, (void **)&p.d_gsort, (size_t)bytes)) return rc;
        p.gsort_bytes = bytes;
    }
    unsigned char *base = (unsigned char *)p.d_gsort;
    uint64_t *skey = (uint64_t *)base;
    int32_t *spos = (int32_t *)(skey + F * P);
    uint64_t *kkey = (uint64_t *)(base + b_keys);
    int32_t *kpos = (int32_t *)(kkey + F * S);
    uint32_t *hist = (uint32_t *)(base + b_keys + b_kept);
    SelState *st = (SelState *)(base + ((b_keys + b_kept + b_hist + 15) & ~int64_t(15)));
    int32_t *cnt = (int32_t *)((unsigned char *)st + b_st);
    int64_t *nsel = (int64_t *)(((uintptr_t)((unsigned char *)cnt + b_cnt) + 7) & ~(uintptr_t)7);
    int rc = MR1L_OK;
    const dim3 gp((unsigned)((P + 255) / 256), (unsigned)F);
    if (p.dtype == MR1L_C128)
        hipLaunchKernelGGL(k_limit_keys<double>, gp, dim3(256), 0, p.stream, n_det, cap, (const double2 *)det_coef,
                           theta * theta, P, skey, spos);
    else
        hipLaunchKernelGGL(k_limit_keys<float>, gp, dim3(256), 0, p.stream, n_det, cap, (const float2 *)det_coef,
                           (float)(theta * theta), P, skey, spos);
    MR1L_LAUNCH_CHECK();
    // the threshold: the s~-th smallest key of each function
    hipLaunchKernelGGL(k_sel_init, dim3((unsigned)F), dim3(256), 0, p.stream, (int)F, n_det, cap, s_cap, st, hist);
    MR1L_LAUNCH_CHECK();
    const dim3 gh((unsigned)std::min<int64_t>((nmax + 255) / 256, std::max<int64_t>(1, 1024 / F + 1)), (unsigned)F);
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist, gh, dim3(256), 0, p.stream, n_det, cap, P, skey, shift, st, hist);
        MR1L_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sel_pick, dim3((unsigned)F), dim3(256), 0, p.stream, shift, st, hist);
        MR1L_LAUNCH_CHECK();
    }
    // the kept pairs in position order
    const dim3 gb((unsigned)nb, (unsigned)F);
    hipLaunchKernelGGL(k_sel_count, gb, dim3(kSortThreads), 0, p.stream, n_det, cap, P, skey, st, nb, cnt);
    MR1L_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_scan, dim3((unsigned)F), dim3(kSortThreads), 0, p.stream, nb, st, cnt, nsel);
    MR1L_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_below, dim3((unsigned)((F + 63) / 64)), dim3(64), 0, p.stream, (int)F, nb, st, nsel);
    MR1L_LAUNCH_CHECK();
    if (S > kMaxCap) {
        // padding sorts last: keys ~0, positions INT32_MAX
        if ((rc = launch_fill_u32((uint32_t *)kkey, F * S * 2, 0xffffffffu, p.stream))) return rc;
        if ((rc = launch_fill_u32((uint32_t *)kpos, F * S, 0x7fffffffu, p.stream))) return rc;
    }
    hipLaunchKernelGGL(k_sel_emit, gb, dim3(kSortThreads), 0, p.stream, n_det, cap, P, skey, spos, st, nb, cnt, S,
                       kkey, kpos);
    MR1L_LAUNCH_CHECK();
    if (S <= kMaxCap) {
        const size_t lds = (size_t)S * 12;
#define MR1L_LSD(E)                                                                                               \
    hipLaunchKernelGGL((k_limit_sel<double, E>), dim3((unsigned)F), dim3(kSortThreads), lds, p.stream, cap, det_idx, \
                       (const double2 *)det_coef, nsel, S, kkey, kpos, s_cap, n_out, out_idx, (double2 *)out_coef,   \
                       out_pos)
#define MR1L_LSF(E)                                                                                              \
    hipLaunchKernelGGL((k_limit_sel<float, E>), dim3((unsigned)F), dim3(kSortThreads), lds, p.stream, cap, det_idx, \
                       (const float2 *)det_coef, nsel, S, kkey, kpos, s_cap, n_out, out_idx, (float2 *)out_coef,    \
                       out_pos)
        if (p.dtype == MR1L_C128) MR1L_BY_E(sort_e(S), MR1L_LSD)
        else MR1L_BY_E(sort_e(S), MR1L_LSF)
#undef MR1L_LSD
#undef MR1L_LSF
        MR1L_LAUNCH_CHECK();
        return MR1L_OK;
    }
    if ((rc = gsort_run(p, kkey, kpos, S))) return rc;
    const dim3 ge((unsigned)((s_cap + 255) / 256), (unsigned)F);
    if (p.dtype == MR1L_C128)
        hipLaunchKernelGGL(k_limit_emit<double>, ge, dim3(256), 0, p.stream, cap, det_idx, (const double2 *)det_coef,
                           S, kpos, s_cap, n_out, out_idx, (double2 *)out_coef, out_pos);
    else
        hipLaunchKernelGGL(k_limit_emit<float>, ge, dim3(256), 0, p.stream, cap, det_idx, (const float2 *)det_coef,
                           S, kpos, s_cap, n_out, out_idx, (float2 *)out_coef, out_pos);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

// the longest of the F detected lists (one synchronisation) and sort buffers of its
// power-of-two size
static int long_list_size(Plan &p, const int64_t *n_det, int64_t cap, int64_t &nmax, int64_t &P,
                          const int64_t *set_off = nullptr, std::vector<int64_t> *so = nullptr)
{
    if (p.capturing) return fail(MR1L_E_ARG, "lists longer than 8192 cannot be recorded in a graph");
    std::vector<int64_t> nd((size_t)p.F);
    MR1L_HIP(hipMemcpyAsync(nd.data(), n_det, nd.size() * sizeof(int64_t), hipMemcpyDeviceToHost, p.stream));
    if (so) {
        so->resize((size_t)p.F + 1);
        MR1L_HIP(hipMemcpyAsync(so->data(), set_off, so->size() * sizeof(int64_t), hipMemcpyDeviceToHost, p.stream));
    }
    MR1L_HIP(hipStreamSynchronize(p.stream));
    nmax = 0;
    for (int64_t v : nd) nmax = std::max(nmax, std::min(v, cap));
    P = pow2ceil(std::max<int64_t>(nmax, 1));
    return grow_sort(p, P);
}

// Algorithm 4 on lists of at most nmax <= kMaxCap entries (cap is the lists' stride):
// one workgroup per function.
static int limit_short(Plan &p, const int64_t *n_det, int64_t cap, const int64_t *det_idx, const void *det_coef,
                       double theta, int64_t s_cap, int64_t *n_out, int64_t *out_idx, void *out_coef, int32_t *out_pos,
                       int64_t nmax)
{
    const size_t pc = (size_t)pow2ceil(std::max<int64_t>(nmax, 1));
#define MR1L_LD(E)                                                                                                 \
    hipLaunchKernelGGL((k_limit<double, E>), dim3(p.F), dim3(kSortThreads), pc * 12, p.stream, n_det, cap, det_idx, \
                       (const double2 *)det_coef, theta * theta, s_cap, n_out, out_idx, (double2 *)out_coef, out_pos)
#define MR1L_LF(E)                                                                                                \
    hipLaunchKernelGGL((k_limit<float, E>), dim3(p.F), dim3(kSortThreads), pc * 12, p.stream, n_det, cap, det_idx, \
                       (const float2 *)det_coef, (float)(theta * theta), s_cap, n_out, out_idx, (float2 *)out_coef,  \
                       out_pos)
    if (p.dtype == MR1L_C128) MR1L_BY_E(sort_e(nmax), MR1L_LD)
    else MR1L_BY_E(sort_e(nmax), MR1L_LF)
#undef MR1L_LD
#undef MR1L_LF
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

int extract_tail_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq, const void *ghat,
                     const mr1l_extract_opts &o, const mr1l_extract_out &out, int32_t *det_hash, double *det_w,
                     uint32_t *det_mask, void *det_med, int32_t *out_pos, const int32_t *cstage, int32_t *perm)
{
    const int64_t cap = o.cap;
    const bool large = cap > kMaxCap;
    int64_t nmax = cap, P = 1;
    int rc = MR1L_OK;
    if (!large) {
        const size_t sb = std::max<size_t>((size_t)pow2ceil(std::max<int64_t>(cap, 1)) * 12, kSortBitmapBytes);
#define MR1L_SD(E) \
    hipLaunchKernelGGL(k_sort_det<E>, dim3(p.F), dim3(kSortThreads), sb, p.stream, out.n_det, cap, out.det_idx, \
                       set_off, n_total, (int)sb, det_mask, mask_words(p.L), perm)
        MR1L_BY_E(sort_e(cap), MR1L_SD)
#undef MR1L_SD
        MR1L_LAUNCH_CHECK();
    } else {
        // the buffer sizes come from the detected counts and the set offsets
        std::vector<int64_t> so;
        if ((rc = long_list_size(p, out.n_det, cap, nmax, P, set_off, &so))) return rc;
        if (nmax > 0) {
            // ascending order by an ordered compaction of the detected candidates' bits
            int64_t wmax = 1;
            for (int f = 0; f < p.F; ++f)
                wmax = std::max<int64_t>(wmax, ((so[f + 1] + 31) >> 5) - (so[f] >> 5));
            const int nx = (int)((wmax + kFlagWordsPerBlock - 1) / kFlagWordsPerBlock);
            const int64_t fwords = (n_total + 31) / 32 + 1;
            const int64_t bytes = fwords * 4 + (int64_t)p.F * nx * 4;
            if (p.dflag_bytes < bytes || !p.d_dflag) {
                p.dflag_bytes = 0;
                if ((rc = plan_regrow(p, (void **)&p.d_dflag, (size_t)bytes))) return rc;
                p.dflag_bytes = bytes;
            }
            uint32_t *flags = p.d_dflag;
            int32_t *cnt = (int32_t *)(p.d_dflag + fwords);
            if ((rc = launch_fill_u32(flags, fwords, 0u, p.stream))) return rc;
            hipLaunchKernelGGL(k_flag_det, dim3((unsigned)((nmax + 255) / 256), (unsigned)p.F), dim3(256), 0, p.stream,
                               out.n_det, cap, out.det_idx, set_off, flags);
            MR1L_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_flag_count, dim3((unsigned)nx, (unsigned)p.F), dim3(256), 0, p.stream, set_off, flags,
                               nx, cnt);
            MR1L_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_flag_scan, dim3((unsigned)p.F), dim3(64), 0, p.stream, nx, cnt);
            MR1L_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_flag_emit, dim3((unsigned)nx, (unsigned)p.F), dim3(256), 0, p.stream, set_off, flags,
                               nx, cnt, cap, out.det_idx);
            MR1L_LAUNCH_CHECK();
        }
    }
    if (!large && !cstage) return fail(MR1L_E_ARG, "short lists need the staged coordinates");
    if (nmax > 0 && !large) {
        dim3 gq(tail_blocks((nmax + kDetHashThreads - 1) / kDetHashThreads, p.F, 4), (unsigned)p.F);
        const size_t hb = (size_t)kDetHashThreads * p.L * sizeof(int32_t);
#define MR1L_DS(LM)                                                                                               \
    hipLaunchKernelGGL(k_det_hash_staged<LM>, gq, dim3(kDetHashThreads), hb, p.stream, freq, n_total, set_off, p.L, \
                       p.d, (int)p.dot2, p.d_lat, p.d_z32, p.d_z64, out.n_det, cap, out.det_idx, cstage, perm,      \
                       det_hash)
        MR1L_BY_L(p.L, MR1L_DS)
#undef MR1L_DS
        MR1L_LAUNCH_CHECK();
    } else if (nmax > 0) {
        dim3 gq(tail_blocks((nmax + kDetHashThreads - 1) / kDetHashThreads, p.F, 4), (unsigned)p.F);
        const size_t hb = (size_t)kDetHashThreads * p.L * sizeof(int32_t);
#define MR1L_DH(LM)                                                                                          \
    hipLaunchKernelGGL(k_det_hash<LM>, gq, dim3(kDetHashThreads), hb, p.stream, freq, n_total, set_off, p.L, \
                       p.d, p.d_lat, p.d_z32, p.d_z64, p.d_kb, out.n_det, cap, out.det_idx, det_hash)
        MR1L_BY_L(p.L, MR1L_DH)
#undef MR1L_DH
        MR1L_LAUNCH_CHECK();
    }
    if (large) {   // (short lists: k_sort_det cleared the masks)
        rc = launch_fill_u32(det_mask, (int64_t)p.F * cap * mask_words(p.L), 0u, p.stream);
        if (rc) return rc;
    }
    int64_t maxM = 1;
    for (int64_t m : p.M) maxM = std::max(maxM, m);
    const int words = (int)std::min<int64_t>(kSingleWords, (maxM + 31) / 32);
    const uint32_t *tw = nullptr;   // merged `twice` bitmaps of the long-list path
    int64_t twl = 0;
    if (!large || nmax <= kMaxCap) {
        hipLaunchKernelGGL(k_singleton, dim3(p.L, p.F), dim3(256), 2 * (size_t)words * sizeof(uint32_t), p.stream,
                           p.d_lat, p.L, out.n_det, cap, det_hash, det_mask, words);
        MR1L_LAUNCH_CHECK();
    } else {
        // long lists: chunks of the detected set per lattice, merged in global bitmaps
        const int64_t wl = (maxM + 31) / 32;
        const int64_t bytes = 2 * (int64_t)p.F * p.L * wl * (int64_t)sizeof(uint32_t);
        if (p.single_bytes < bytes || !p.d_single) {
            p.single_bytes = 0;
            if ((rc = plan_regrow(p, (void **)&p.d_single, (size_t)bytes))) return rc;
            p.single_bytes = bytes;
        }
        uint32_t *g_once = p.d_single, *g_twice = p.d_single + (int64_t)p.F * p.L * wl;
        if ((rc = launch_fill_u32(p.d_single, 2 * (int64_t)p.F * p.L * wl, 0u, p.stream))) return rc;
        if (wl <= kSingleWords) {
            // as many lattices per workgroup as the LDS holds; about one workgroup per CU
            const int gs = (int)std::min<int64_t>(p.L, kSingleWords / wl);
            const int groups = (p.L + gs - 1) / gs;
            const int64_t by_cus = std::max<int64_t>(1, (int64_t)num_cus() / ((int64_t)groups * p.F));
            const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(by_cus, (nmax + 4095) / 4096));
            hipLaunchKernelGGL(k_single_count_grp, dim3((unsigned)chunks, (unsigned)groups, (unsigned)p.F),
                               dim3(kSingleThreads), 2 * (size_t)gs * wl * sizeof(uint32_t), p.stream, p.d_lat, p.L,
                               out.n_det, cap, det_hash, chunks, gs, (int)wl, wl, g_once, g_twice);
        } else {
            const int64_t by_cus =
                std::max<int64_t>(1, 2 * (int64_t)num_cus() / std::max<int64_t>(1, (int64_t)p.L * p.F));
            const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(by_cus, (nmax + 4095) / 4096));
            hipLaunchKernelGGL(k_single_count, dim3((unsigned)chunks, (unsigned)p.L, (unsigned)p.F),
                               dim3(kSingleThreads), 2 * (size_t)words * sizeof(uint32_t), p.stream, p.d_lat, p.L,
                               out.n_det, cap, det_hash, chunks, wl, g_once, g_twice, words);
        }
        MR1L_LAUNCH_CHECK();
        tw = g_twice;
        twl = wl;
    }
    const int64_t ncomb = std::max<int64_t>(nmax, 1);
    if (p.dtype == MR1L_C128)
        rc = combine_launch<double>(p, out.n_det, cap, ncomb, det_hash, det_mask, ghat, o.postproc, out.det_coef,
                                    det_med, det_w, large ? 16 : 1, tw, twl);
    else
        rc = combine_launch<float>(p, out.n_det, cap, ncomb, det_hash, det_mask, ghat, o.postproc, out.det_coef,
                                   det_med, det_w, large ? 16 : 1, tw, twl);
    if (rc) return rc;
    if (!large) {
        return limit_short(p, out.n_det, cap, out.det_idx, out.det_coef, o.theta, o.s_cap, out.n_out, out.out_idx,
                           out.out_coef, out_pos, cap);
    }
    return limit_long(p, out.n_det, cap, out.det_idx, out.det_coef, o.theta, o.s_cap, out.n_out, out.out_idx,
                      out.out_coef, out_pos, P, nmax);
}

int limit_run(Plan &p, const int64_t *n_det, int64_t cap, const int64_t *det_idx, const void *det_coef, double theta,
              int64_t s_cap, int64_t *n_out, int64_t *out_idx, void *out_coef)
{
    if (cap < 1 || cap > kMaxCapLarge) return fail(MR1L_E_ARG, "capacity must be in [1, 2^24]");
    if (cap > kMaxCap) {
        int64_t nmax = 0, P = 1;
        const int rc = long_list_size(p, n_det, cap, nmax, P);
        return rc ? rc
                  : limit_long(p, n_det, cap, det_idx, det_coef, theta, s_cap, n_out, out_idx, out_coef, nullptr, P, nmax);
    }
    return limit_short(p, n_det, cap, det_idx, det_coef, theta, s_cap, n_out, out_idx, out_coef, nullptr, cap);
}

int adjoint_run(Plan &p, int64_t cap, int64_t s_cap, const int64_t *n_out, const int32_t *out_pos,
                const int32_t *det_hash, const double *det_w, const void *grad_out, void *grad_f)
{
    const size_t esz = p.dtype == MR1L_C128 ? 16 : 8;
    int rc = launch_fill_bytes(p.d_nodes_scratch, (int64_t)(p.nodes * esz), p.stream);
    if (rc) return rc;
    dim3 grid((unsigned)((s_cap + 255) / 256), (unsigned)p.F), blk(256);
    if (p.dtype == MR1L_C128)
        hipLaunchKernelGGL(k_adjoint_scatter<double>, grid, blk, 0, p.stream, p.d_lat, p.L, cap, s_cap, n_out,
                           out_pos, det_hash, det_w, (const double2 *)grad_out, (double *)p.d_nodes_scratch);
    else
        hipLaunchKernelGGL(k_adjoint_scatter<float>, grid, blk, 0, p.stream, p.d_lat, p.L, cap, s_cap, n_out,
                           out_pos, det_hash, det_w, (const float2 *)grad_out, (float *)p.d_nodes_scratch);
    MR1L_LAUNCH_CHECK();
    return fft_run(p, p.d_nodes_scratch, grad_f, 0.0, nullptr, FFT_INV, 1.0);
}

}  // namespace mr1l
