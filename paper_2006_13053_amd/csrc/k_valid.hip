// Validation of a candidate set against the lattice sizes: M must lie in P^Gamma
// (Section 2.1), i.e. the candidates stay pairwise distinct modulo M.  Every
// prime above the expansion N_Gamma of the set (its largest coordinate range)
// qualifies; for smaller sizes the reduced vectors k mod M are compared exactly
// through an open-addressing table of candidate indices.
#include <algorithm>
#include <vector>

#include "mr1l_internal.h"

namespace mr1l {

// Per function and coordinate: minimum and maximum over the function's candidates.
__global__ __launch_bounds__(256) void k_minmax(const int64_t *__restrict__ freq, int64_t n_total, int d,
                                                int64_t lo, int64_t hi, int64_t *__restrict__ mm)
{
    for (int u = 0; u < d; ++u) {
        long long a = LLONG_MAX, b = LLONG_MIN;
        for (int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < hi;
             i += (int64_t)gridDim.x * blockDim.x) {
            const long long k = freq[(int64_t)u * n_total + i];
            a = min(a, k);
            b = max(b, k);
        }
        for (int o = 32; o > 0; o >>= 1) {
            a = min(a, (long long)__shfl_xor(a, o));
            b = max(b, (long long)__shfl_xor(b, o));
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMin((long long *)(mm + 2 * u), a);
            atomicMax((long long *)(mm + 2 * u + 1), b);
        }
    }
}

__device__ __forceinline__ int64_t floor_mod(int64_t k, int64_t m)
{
    const int64_t r = k % m;
    return r < 0 ? r + m : r;
}

// Inserts candidates [lo, hi) into the table (index + 1, 0 = empty); a candidate
// whose reduced vector equals that of one already present sets *dup.
__global__ __launch_bounds__(256) void k_inject(const int64_t *__restrict__ freq, int64_t n_total, int d,
                                                int64_t lo, int64_t hi, int64_t M, uint32_t *__restrict__ table,
                                                uint32_t tmask, int32_t *__restrict__ dup)
{
    for (int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < hi;
         i += (int64_t)gridDim.x * blockDim.x) {
        // 64-bit multiplicative hash of the reduced vector (any hash works: equality is checked)
        uint64_t h = 0x9E3779B97F4A7C15ull;
        for (int u = 0; u < d; ++u) {
            h ^= (uint64_t)floor_mod(freq[(int64_t)u * n_total + i], M);
            h *= 0xBF58476D1CE4E5B9ull;
            h ^= h >> 29;
        }
        uint32_t slot = (uint32_t)h & tmask;
        const uint32_t me = (uint32_t)(i - lo) + 1u;
        for (uint32_t probe = 0; probe <= tmask; ++probe) {
            const uint32_t old = atomicCAS(table + slot, 0u, me);
            if (old == 0u) break;
            const int64_t j = lo + (int64_t)old - 1;
            bool same = true;
            for (int u = 0; u < d && same; ++u)
                same = floor_mod(freq[(int64_t)u * n_total + i], M) == floor_mod(freq[(int64_t)u * n_total + j], M);
            if (same) {
                atomicExch(dup, 1);
                break;
            }
            slot = (slot + 1) & tmask;
        }
    }
}

int check_injective_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq, int32_t *ok)
{
    std::vector<int64_t> off(p.F + 1, 0);
    if (set_off) {
        MR1L_HIP(hipMemcpyAsync(off.data(), set_off, (p.F + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, p.stream));
        MR1L_HIP(hipStreamSynchronize(p.stream));
    } else {
        off[1] = n_total;
    }
    for (int f = 0; f < p.F; ++f)
        if (off[f] < 0 || off[f] > off[f + 1] || off[f + 1] > n_total)
            return fail(MR1L_E_ARG, "set_off must be non-decreasing within [0, n_total]");
    int64_t nmax = 0;
    for (int f = 0; f < p.F; ++f) nmax = std::max(nmax, off[f + 1] - off[f]);
    if (nmax >= (int64_t(1) << 31) - 1) return fail(MR1L_E_OVERFLOW, "candidate set too large for the check");
    int64_t *d_mm = nullptr;
    uint32_t *d_tab = nullptr;
    int32_t *d_dup = nullptr;
    int rc = MR1L_OK;
    auto fin = [&](int r) {
        (void)hipStreamSynchronize(p.stream);
        if (d_mm) (void)hipFree(d_mm);
        if (d_tab) (void)hipFree(d_tab);
        if (d_dup) (void)hipFree(d_dup);
        return r;
    };
    if (hipMalloc(&d_mm, 2 * (size_t)p.d * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&d_dup, sizeof(int32_t)) != hipSuccess)
        return fin(fail(MR1L_E_NOMEM, "allocation for the injectivity check failed"));
    uint32_t tsize = 1;
    while ((int64_t)tsize < 2 * std::max<int64_t>(nmax, 1)) tsize <<= 1;
    bool any_bad = false;
    for (int f = 0; f < p.F && rc == MR1L_OK; ++f) {
        const int64_t lo = off[f], hi = off[f + 1];
        bool good = true;
        if (hi - lo > 1) {
            std::vector<int64_t> mm(2 * (size_t)p.d);
            for (int u = 0; u < p.d; ++u) { mm[2 * u] = INT64_MAX; mm[2 * u + 1] = INT64_MIN; }
            if (hipMemcpy(d_mm, mm.data(), mm.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
                return fin(fail(MR1L_E_HIP, "copy for the injectivity check failed"));
            const int64_t blocks = std::min<int64_t>((hi - lo + 255) / 256, 4096);
            hipLaunchKernelGGL(k_minmax, dim3((unsigned)blocks), dim3(256), 0, p.stream, freq, n_total, p.d, lo, hi,
                               d_mm);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(mm.data(), d_mm, mm.size() * sizeof(int64_t), hipMemcpyDeviceToHost, p.stream) !=
                    hipSuccess ||
                hipStreamSynchronize(p.stream) != hipSuccess)
                return fin(fail(MR1L_E_HIP, "minimum/maximum pass failed"));
            // expansion N_Gamma (saturating: ranges beyond 2^62 compare as huge)
            int64_t expn = 0;
            for (int u = 0; u < p.d; ++u) {
                const __int128 r = (__int128)mm[2 * u + 1] - (__int128)mm[2 * u];
                expn = std::max<int64_t>(expn, r > ((__int128)1 << 62) ? (int64_t(1) << 62) : (int64_t)r);
            }
            std::vector<int64_t> sizes;
            for (int l = 0; l < p.L; ++l) sizes.push_back(p.M[(size_t)f * p.L + l]);
            std::sort(sizes.begin(), sizes.end());
            sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
            for (int64_t M : sizes) {
                if (M > expn) continue;   // every prime above N_Gamma lies in P^Gamma
                if (!d_tab && hipMalloc(&d_tab, (size_t)tsize * sizeof(uint32_t)) != hipSuccess)
                    return fin(fail(MR1L_E_NOMEM, "allocation of the injectivity table failed"));
                uint32_t ts = 1;
                while ((int64_t)ts < 2 * (hi - lo)) ts <<= 1;
                if ((rc = launch_fill_u32(d_tab, ts, 0u, p.stream)) || (rc = launch_fill_u32((uint32_t *)d_dup, 1, 0u, p.stream)))
                    return fin(rc);
                hipLaunchKernelGGL(k_inject, dim3((unsigned)blocks), dim3(256), 0, p.stream, freq, n_total, p.d, lo, hi,
                                   M, d_tab, ts - 1, d_dup);
                int32_t dup = 0;
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(&dup, d_dup, sizeof(int32_t), hipMemcpyDeviceToHost, p.stream) != hipSuccess ||
                    hipStreamSynchronize(p.stream) != hipSuccess)
                    return fin(fail(MR1L_E_HIP, "injectivity pass failed"));
                if (dup) { good = false; break; }
            }
        }
        if (ok) ok[f] = good ? 1 : 0;
        any_bad = any_bad || !good;
    }
    rc = fin(MR1L_OK);
    if (any_bad) return fail(MR1L_E_NOT_INJECTIVE, "a candidate set is not injective modulo a lattice size");
    return rc;
}

}  // namespace mr1l
