// Samples of a sparse trigonometric polynomial (eq. (2.2)) at rank-1 lattice
// nodes x_j = j z_l / M_l mod 1 (eq. (2.1)), with optional fixed anchor
// coordinates x'_u = a_u / 2^32 for u >= d (the embedding of Algorithm 3).
//
// For term k: k . x_j = (j h_l(k) mod M_l) / M_l + (sum_{u>=d} k_u a_u mod 2^32) / 2^32,
// both reduced exactly in integers.  The anchor factor is folded into the
// coefficient once per term.
//   direct  one thread per node sums all terms of its function; the phase
//           e^{2 pi i r / M} comes from a two-level table (r = hi S + lo) in LDS.
//   bucket  the aliasing formula eq. (2.4): coefficients are summed into the
//           buckets h_l(k) (in LDS per lattice, component and chunk of terms when
//           one lattice's buckets fit, else by global atomics), then
//           f_l[j] = sum_h B[h] e^{2 pi i j h / M} is an inverse lattice DFT
//           (scaled by M).
#include <mutex>
#include <string>

#include "mr1l_internal.h"

namespace mr1l {

__device__ __forceinline__ int func_of_terms(const int64_t *off, int F, int64_t i)
{
    int lo = 0, hi = F;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Per term: anchored coefficient and buckets in all lattices of its function.
// PLANAR writes the coefficients as a real plane followed by an imaginary plane
// (for the LDS bucket accumulation), else interleaved.  When all lanes of a wave
// hold terms of one function (the usual case), its lattice records and generating
// vectors are wave-uniform and come through scalar loads.  DM bounds d at compile
// time so that the coordinates stay in registers (DM = 16 covers d <= 16).
template <typename T, bool PLANAR, int DM>
__global__ __launch_bounds__(256) void k_term_prep(
    const int64_t *__restrict__ freq, int64_t n_terms, const int64_t *__restrict__ term_off, int F, int L, int d,
    int d_poly, const LatDesc *__restrict__ lat, const int32_t *__restrict__ z32, const int64_t *__restrict__ z64,
    const int32_t *__restrict__ kbound, const typename cvec<T>::type *__restrict__ coef,
    const uint32_t *__restrict__ anchor, typename cvec<T>::type *__restrict__ cterm, int32_t *__restrict__ thash)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_terms;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int f = func_of_terms(term_off, F, t);
        auto c = coef[t];
        if (d_poly > d) {
            uint32_t acc = 0;
            for (int u = d; u < d_poly; ++u)
                acc += (uint32_t)freq[(int64_t)u * n_terms + t] * anchor[(int64_t)f * (d_poly - d) + (u - d)];
            double sn, cs;
            sincospi((double)acc * 4.656612873077392578125e-10, &sn, &cs);  // acc / 2^31
            const T cr = c.x, ci = c.y;
            c.x = (T)(cr * cs - ci * sn);
            c.y = (T)(cr * sn + ci * cs);
        }
        if constexpr (PLANAR) {
            T *pl = reinterpret_cast<T *>(cterm);
            pl[t] = c.x;
            pl[n_terms + t] = c.y;
        } else {
            cterm[t] = c;
        }
        const int32_t kb = kbound[f];
        int32_t lo[DM];
        bool fast = true;
#pragma unroll
        for (int u = 0; u < DM; ++u) {
            if (u < d) {
                const int64_t k = freq[(int64_t)u * n_terms + t];
                lo[u] = (int32_t)k;
                fast = fast & (k >= -kb) & (k <= kb);
            }
        }
        auto hash_all = [&](int ff) {
            for (int l = 0; l < L; ++l) {
                const LatDesc ld = lat[ff * L + l];
                int32_t h;
                if (fast) {
                    uint32_t s = ld.off32;
#pragma unroll
                    for (int u = 0; u < DM; ++u)
                        if (u < d) s += (uint32_t)__mul24(lo[u], z32[ld.z_off + u]);
                    h = (int32_t)fast_mod(s, (uint32_t)ld.M, ld.inv_m);
                } else {
                    h = exact_bucket(freq + t, n_terms, d, z64 + ld.z_off, ld.M);
                }
                thash[(int64_t)l * n_terms + t] = h;
            }
        };
        const int fu = __builtin_amdgcn_readfirstlane(f);
        if (__all(f == fu)) hash_all(fu);
        else hash_all(f);
    }
}

constexpr int kTermTile = 256;
constexpr int kPhaseTab = 4096;   // entries of the two-level phase table (both levels)

template <typename T>
__global__ __launch_bounds__(256) void k_sample_direct(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ term_off, int64_t n_terms,
    const typename cvec<T>::type *__restrict__ cterm, const int32_t *__restrict__ thash,
    typename cvec<T>::type *__restrict__ out)
{
    using V = typename cvec<T>::type;
    __shared__ V tab[kPhaseTab];
    __shared__ int32_t sh[kTermTile];
    __shared__ V sc[kTermTile];
    const int li = blockIdx.y;
    const LatDesc ld = lat[li];
    const int f = li / L, l = li - f * L;
    const int M = ld.M;
    // two-level table of e^{2 pi i r / M}: S = 2^shift >= sqrt(M)
    int shift = 0;
    while ((1 << (2 * shift)) < M) ++shift;
    const int S = 1 << shift;
    const int nhi = (M + S - 1) / S;
    for (int i = threadIdx.x; i < S + nhi; i += blockDim.x) {
        const int64_t r = i < S ? i : (int64_t)(i - S) * S;
        double sn, cs;
        sincospi(2.0 * (double)r / (double)M, &sn, &cs);
        V v; v.x = (T)cs; v.y = (T)sn;
        tab[i] = v;
    }
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t0 = term_off[f], t1 = term_off[f + 1];
    const double invM = 1.0 / (double)M;
    T ar = 0, ai = 0;
    for (int64_t tb = t0; tb < t1; tb += kTermTile) {
        __syncthreads();
        const int cnt = (int)min<int64_t>(kTermTile, t1 - tb);
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            sh[i] = thash[(int64_t)l * n_terms + tb + i];
            sc[i] = cterm[tb + i];
        }
        __syncthreads();
        if (j < M) {
            for (int i = 0; i < cnt; ++i) {
                // r = (j h) mod M, j h < 2^46 is exact in double
                const double pr = (double)j * (double)sh[i];
                int64_t q = (int64_t)(pr * invM);
                int64_t r = (int64_t)pr - q * M;
                if (r < 0) r += M;
                if (r >= M) r -= M;
                const V a = tab[r & (S - 1)], b = tab[S + (r >> shift)];
                const T er = a.x * b.x - a.y * b.y, ei = a.x * b.y + a.y * b.x;
                const V c = sc[i];
                ar += c.x * er - c.y * ei;
                ai += c.x * ei + c.y * er;
            }
        }
    }
    if (j < M) {
        V o; o.x = ar; o.y = ai;
        out[ld.node_off + j] = o;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sample_scatter(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ term_off, int F, int64_t n_terms,
    const typename cvec<T>::type *__restrict__ cterm, const int32_t *__restrict__ thash, T *__restrict__ buckets)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_terms;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int f = func_of_terms(term_off, F, t);
        const auto c = cterm[t];
        for (int l = 0; l < L; ++l) {
            const int64_t node = lat[f * L + l].node_off + thash[(int64_t)l * n_terms + t];
            unsafeAtomicAdd(buckets + 2 * node, c.x);
            unsafeAtomicAdd(buckets + 2 * node + 1, c.y);
        }
    }
}

// Bucket sums of one lattice and one component (real or imaginary) in LDS: a
// workgroup takes one chunk of its function's terms (planar coefficients), adds
// them into an LDS copy of the M_l buckets, then adds the copy into the global
// buckets.  Global atomics drop from two per term and lattice to one per bucket
// and chunk.
constexpr int kLdsScatterThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kLdsScatterThreads) void k_sample_lds(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ term_off, int64_t n_terms, int chunks,
    const T *__restrict__ cplane, const int32_t *__restrict__ thash, T *__restrict__ buckets)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *acc = reinterpret_cast<T *>(smem);
    const int comp = blockIdx.y & 1;
    const int li = blockIdx.y >> 1;
    const int f = li / L, l = li - f * L;
    const LatDesc ld = lat[li];
    const int M = ld.M;
    for (int i = threadIdx.x; i < M; i += blockDim.x) acc[i] = T(0);
    __syncthreads();
    const int64_t t0 = term_off[f], t1 = term_off[f + 1];
    const int64_t per = (t1 - t0 + chunks - 1) / chunks;
    const int64_t b = min(t1, t0 + (int64_t)blockIdx.x * per), e = min(t1, b + per);
    const T *cv = cplane + (int64_t)comp * n_terms;
    const int32_t *hh = thash + (int64_t)l * n_terms;
    constexpr int U = 4;   // loads in flight per thread
    int64_t t = b + threadIdx.x;
    for (; t + (U - 1) * (int64_t)kLdsScatterThreads < e; t += U * (int64_t)kLdsScatterThreads) {
        int32_t h[U];
        T v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            h[q] = __builtin_nontemporal_load(hh + t + q * kLdsScatterThreads);
            v[q] = __builtin_nontemporal_load(cv + t + q * kLdsScatterThreads);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) unsafeAtomicAdd(acc + h[q], v[q]);
    }
    for (; t < e; t += kLdsScatterThreads) unsafeAtomicAdd(acc + hh[t], cv[t]);
    __syncthreads();
    if (b >= e) return;
    T *out = buckets + 2 * ld.node_off + comp;
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
        const T v = acc[i];
        if (v != T(0)) unsafeAtomicAdd(out + 2 * (int64_t)i, v);
    }
}

int sample_init_attrs()
{
    MR1L_HIP(hipFuncSetAttribute((const void *)k_sample_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes));
    MR1L_HIP(hipFuncSetAttribute((const void *)k_sample_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes));
    return MR1L_OK;
}

template <typename T>
static int sample_impl(Plan &p, int32_t d_poly, const int64_t *term_off, int64_t n_terms, const int64_t *freq,
                       const void *coef, const uint32_t *anchor, void *f, int32_t mode, void *cterm,
                       int32_t *thash)
{
    using V = typename cvec<T>::type;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_terms + 255) / 256, (int64_t)num_cus() * 16));
    int32_t maxM = 0;
    for (auto m : p.M) maxM = std::max<int32_t>(maxM, (int32_t)m);
    // bucket sums in LDS when one lattice's buckets (one component) fit and the
    // functions have many terms per bucket chunk
    const int units = p.F * p.L * 2;
    const int64_t per_f = n_terms / std::max(1, p.F);
    const bool lds = mode == 2 && units <= 65535 && (int64_t)maxM * (int64_t)sizeof(T) <= kLdsBytes &&
                     per_f >= 8 * (int64_t)maxM;
    if (n_terms > 0) {
#define MR1L_PREP(PL, DM)                                                                                        \
    hipLaunchKernelGGL((k_term_prep<T, PL, DM>), dim3((unsigned)blocks), dim3(256), 0, p.stream, freq, n_terms, \
                       term_off, p.F, p.L, p.d, d_poly, p.d_lat, p.d_z32, p.d_z64, p.d_kb, (const V *)coef, anchor, \
                       (V *)cterm, thash)
        if (lds) {
            if (p.d <= 16) MR1L_PREP(true, 16);
            else MR1L_PREP(true, kMaxD);
        } else {
            if (p.d <= 16) MR1L_PREP(false, 16);
            else MR1L_PREP(false, kMaxD);
        }
#undef MR1L_PREP
        MR1L_LAUNCH_CHECK();
    }
    if (mode == 1) {
        dim3 grid((unsigned)((maxM + 255) / 256), (unsigned)(p.F * p.L));
        hipLaunchKernelGGL(k_sample_direct<T>, grid, dim3(256), 0, p.stream, p.d_lat, p.L, term_off, n_terms,
                           (const V *)cterm, thash, (V *)f);
        MR1L_LAUNCH_CHECK();
        return MR1L_OK;
    }
    int rc = launch_fill_bytes(p.d_nodes_scratch, p.nodes * (int64_t)sizeof(V), p.stream);
    if (rc) return rc;
    if (n_terms > 0 && lds) {
        // chunks per (lattice, component): one round of workgroups over the CUs,
        // at least 2 M terms per chunk
        const int64_t by_cus = std::max<int64_t>(1, num_cus() / std::max(1, units));
        const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(by_cus, per_f / (2 * (int64_t)maxM)));
        hipLaunchKernelGGL(k_sample_lds<T>, dim3((unsigned)chunks, (unsigned)units), dim3(kLdsScatterThreads),
                           (size_t)maxM * sizeof(T), p.stream, p.d_lat, p.L, term_off, n_terms, chunks,
                           (const T *)cterm, thash, (T *)p.d_nodes_scratch);
        MR1L_LAUNCH_CHECK();
    } else if (n_terms > 0) {
        hipLaunchKernelGGL(k_sample_scatter<T>, dim3((unsigned)blocks), dim3(256), 0, p.stream, p.d_lat, p.L,
                           term_off, p.F, n_terms, (const V *)cterm, thash, (T *)p.d_nodes_scratch);
        MR1L_LAUNCH_CHECK();
    }
    return fft_run(p, p.d_nodes_scratch, f, 0.0, nullptr, FFT_INV, -1.0);   // times M
}

static int resolve_mode(const Plan &p, int64_t n_terms, int32_t mode)
{
    // direct when a function has few terms per node; buckets otherwise
    if (mode == 0) mode = (n_terms / std::max(1, p.F) > 2048) ? 2 : 1;
    return mode;
}

int sample_run_with(Plan &p, int32_t d_poly, const int64_t *term_off, int64_t n_terms, const int64_t *freq,
                    const void *coef, const uint32_t *anchor, void *f, int32_t mode, void *cterm, int32_t *thash)
{
    mode = resolve_mode(p, n_terms, mode);
    if (p.dtype == MR1L_C128)
        return sample_impl<double>(p, d_poly, term_off, n_terms, freq, coef, anchor, f, mode, cterm, thash);
    return sample_impl<float>(p, d_poly, term_off, n_terms, freq, coef, anchor, f, mode, cterm, thash);
}

// Term scratch of the allocation-free sampler: one array per device, held from the
// library's load until the process ends.  Host code never uses the array's name as
// an address (in host code it is a stand-in, not device memory): each device's
// address comes from hipGetSymbolAddress, once per device, at plan creation.
constexpr int64_t kStaticScratchBytes = int64_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

int sample_static_scratch(void **out)
{
    int dev = 0;
    MR1L_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MR1L_E_ARG, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MR1L_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MR1L_OK;
}

// The sampler with its term scratch (anchored coefficients, then the buckets, each
// from a 256-byte boundary) in the device's static array: no allocation.  Every call
// on a device shares the array, so calls that overlap on one device race.
int sample_run_noalloc(Plan &p, int32_t d_poly, const int64_t *term_off, int64_t n_terms, const int64_t *freq,
                       const void *coef, const uint32_t *anchor, void *f, int32_t mode)
{
    if (!p.d_static_scratch) return fail(MR1L_E_ARG, "the plan has no static scratch address");
    const int64_t esz = p.dtype == MR1L_C128 ? 16 : 8;
    const int64_t nt = std::max<int64_t>(1, n_terms);
    const int64_t cbytes = (nt * esz + 255) / 256 * 256;
    const int64_t need = cbytes + nt * 4 * (int64_t)p.L;
    if (need > kStaticScratchBytes)
        return fail(MR1L_E_CAPACITY, "n_terms too large for the static term scratch: needs " + std::to_string(need) +
                                         " bytes, at most " + std::to_string(kStaticScratchBytes) + " (n_terms * (" +
                                         std::to_string(esz) + " + 4 L) plus alignment)");
    unsigned char *base = static_cast<unsigned char *>(p.d_static_scratch);
    return sample_run_with(p, d_poly, term_off, n_terms, freq, coef, anchor, f, mode, base,
                           reinterpret_cast<int32_t *>(base + cbytes));
}

// The term scratch (anchored coefficients and buckets) belongs to the plan and grows
// with the largest call, outside graph capture only.
int sample_run(Plan &p, int32_t d_poly, const int64_t *term_off, int64_t n_terms, const int64_t *freq,
               const void *coef, const uint32_t *anchor, void *f, int32_t mode)
{
    const int64_t esz = p.dtype == MR1L_C128 ? 16 : 8;
    int rc = grow_scratch(p, &p.d_cterm, std::max<int64_t>(1, n_terms) * esz, p.cterm_bytes);
    if (rc) return rc;
    rc = grow_scratch(p, (void **)&p.d_thash, std::max<int64_t>(1, n_terms) * 4 * p.L, p.thash_bytes);
    if (rc) return rc;
    return sample_run_with(p, d_poly, term_off, n_terms, freq, coef, anchor, f, mode, p.d_cterm, p.d_thash);
}

}  // namespace mr1l
