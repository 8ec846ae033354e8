// Worst-case aliasing diagnostic of Section 4.1.1 (Table 4.1).  The method is run
// on the counting polynomial of eq. (4.1) (all-ones coefficients on the support I);
// every lattice value at a bucket of k is then the number of support members that
// share k's bucket, so the detected set and the medians of one extract pass classify
// each candidate as a potential false positive (PFP) or potential false negative
// (PFN).  This kernel turns one extract pass into per-function counts.
#include "mr1l_internal.h"

namespace mr1l {

template <typename T>
__global__ __launch_bounds__(256) void k_pfpn(int64_t cap, const int64_t *__restrict__ n_active,
                                              const int64_t *__restrict__ n_det, const int64_t *__restrict__ det_idx,
                                              const T *__restrict__ det_med, const T *__restrict__ det_coef,
                                              double theta2, int64_t *__restrict__ counts)
{
    __shared__ int acc[3];   // PFN, PFP after post-processing, support-order violations
    if (threadIdx.x < 3) acc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t f = blockIdx.x;
    const int64_t na = n_active[f], nd = n_det[f];
    const int64_t m = nd < cap ? nd : cap;
    int pfn = 0, post = 0, bad = 0;
    for (int64_t c = threadIdx.x; c < m; c += blockDim.x) {
        const int64_t k = det_idx[f * cap + c];
        if (c < na && k != c) bad = 1;   // the support must come first and be detected whole
        if (k < na) {
            // medians of integer counts are integers or half-integers: > 1 means >= 1.5
            if ((double)det_med[2 * (f * cap + c)] > 1.25) ++pfn;
        } else {
            const double re = det_coef[2 * (f * cap + c)], im = det_coef[2 * (f * cap + c) + 1];
            if (re * re + im * im >= theta2) ++post;
        }
    }
    if (pfn) atomicAdd(&acc[0], pfn);
    if (post) atomicAdd(&acc[1], post);
    if (bad) atomicOr(&acc[2], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t flags = 0;
        // a truncated list keeps an unspecified subset of the detected set: the support
        // is then only checked to fit
        if (nd > cap) flags |= 1;
        else if (acc[2] || nd < na) flags |= 2;
        if (na > cap) flags |= 2;
        counts[4 * f + 0] = nd - na;
        counts[4 * f + 1] = acc[0];
        counts[4 * f + 2] = acc[1];
        counts[4 * f + 3] = flags;
    }
}

int pfpn_run(Plan &p, int64_t cap, const int64_t *n_active, const int64_t *n_det, const int64_t *det_idx,
             const void *det_med, const void *det_coef, double theta, int64_t *counts)
{
    if (p.F <= 0) return MR1L_OK;
    const double t2 = theta * theta;
    if (p.dtype == MR1L_C128)
        hipLaunchKernelGGL(k_pfpn<double>, dim3((unsigned)p.F), dim3(256), 0, p.stream, cap, n_active, n_det, det_idx,
                           (const double *)det_med, (const double *)det_coef, t2, counts);
    else
        hipLaunchKernelGGL(k_pfpn<float>, dim3((unsigned)p.F), dim3(256), 0, p.stream, cap, n_active, n_det, det_idx,
                           (const float *)det_med, (const float *)det_coef, t2, counts);
    if (hipGetLastError() != hipSuccess) return fail(MR1L_E_HIP, "launch of the PFP/PFN count failed");
    return MR1L_OK;
}

}  // namespace mr1l
