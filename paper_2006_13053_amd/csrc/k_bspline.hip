// Samples of sums of tensor products of periodic B-splines (the test function
// eq. (4.3) of Section 4.2.3) at rank-1 lattice nodes with fixed anchors:
//   f(x) = sum_j prod_{u in S_j} N_{m_j}(x_u),
//   N_m(x) = C_m sum_k sinc(pi k / m)^m (-1)^k e^{2 pi i k x}.
// The series is m B_m(m x) on [0, 1) for the cardinal B-spline B_m of order m
// with knots 0, 1, ..., m (its Fourier transform is sinc(pi xi)^m e^{-pi i xi m}),
// so N_m(x) = C_m m B_m(m x) with C_m = (m B_2m(m))^{-1/2} for unit L2 norm
// (the autocorrelation of B_m is B_2m shifted by m).  B_m is evaluated with the
// Cox-de Boor recursion in double.
#include <cmath>
#include <vector>

#include "mr1l_internal.h"

namespace mr1l {

constexpr int kBsMaxOrder = 16;
constexpr int kBsMaxProd = 16;

struct BsDesc {
    int32_t n;                    // products
    int32_t d_poly;               // coordinates of the function
    int32_t order[kBsMaxProd];
    double scale[kBsMaxProd];     // C_m m
};

// B_m(y) for 0 <= y < m: values B_k(t + r), r < k, of the piece containing y.
__device__ __forceinline__ double cardinal_bspline(int m, double y)
{
    const int i = min(max((int)floor(y), 0), m - 1);
    const double t = y - i;
    double v[kBsMaxOrder];
#pragma unroll
    for (int r = 0; r < kBsMaxOrder; ++r) v[r] = r == 0 ? 1.0 : 0.0;
#pragma unroll
    for (int k = 2; k <= kBsMaxOrder; ++k) {
        if (k <= m) {
            const double inv = 1.0 / (k - 1);
#pragma unroll
            for (int r = kBsMaxOrder - 1; r >= 0; --r) {
                if (r < k) {
                    const double a = (r < k - 1) ? v[r] : 0.0;
                    const double b = (r >= 1) ? v[r > 0 ? r - 1 : 0] : 0.0;
                    v[r] = ((t + r) * a + (k - t - r) * b) * inv;
                }
            }
        }
    }
    double out = 0.0;
#pragma unroll
    for (int r = 0; r < kBsMaxOrder; ++r)
        if (r == i) out = v[r];
    return out;
}

template <typename T>
__global__ __launch_bounds__(256) void k_sample_bspline(const LatDesc *__restrict__ lat, int L, int d,
                                                        const int64_t *__restrict__ z64, BsDesc bs,
                                                        const uint64_t *__restrict__ dims,
                                                        const uint32_t *__restrict__ anchor,
                                                        typename cvec<T>::type *__restrict__ out)
{
    using V = typename cvec<T>::type;
    const int li = blockIdx.y;
    const LatDesc ld = lat[li];
    const int f = li / L;
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= ld.M) return;
    const int na = bs.d_poly - d;
    double acc = 0.0;
    for (int q = 0; q < bs.n; ++q) {
        uint64_t mask = dims[(int64_t)f * bs.n + q];
        const int m = bs.order[q];
        double prod = 1.0;
        while (mask) {
            const int u = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            double x;
            if (u < d) x = (double)((j * z64[ld.z_off + u]) % ld.M) / (double)ld.M;   // j z < 2^46
            else x = (double)anchor[(int64_t)f * na + (u - d)] * 2.3283064365386962890625e-10;   // a / 2^32
            prod *= bs.scale[q] * cardinal_bspline(m, m * x);
        }
        acc += prod;
    }
    V o;
    o.x = (T)acc;
    o.y = (T)0;
    out[ld.node_off + j] = o;
}

// Host: B_m(y) by the same recursion (for the normalising constants).
static double host_bspline(int m, double y)
{
    if (y < 0.0 || y >= m) return 0.0;
    const int i = std::min((int)std::floor(y), m - 1);
    const double t = y - i;
    std::vector<double> v((size_t)m, 0.0);
    v[0] = 1.0;
    for (int k = 2; k <= m; ++k)
        for (int r = k - 1; r >= 0; --r) {
            const double a = (r < k - 1) ? v[(size_t)r] : 0.0;
            const double b = (r >= 1) ? v[(size_t)r - 1] : 0.0;
            v[(size_t)r] = ((t + r) * a + (k - t - r) * b) / (k - 1);
        }
    return v[(size_t)i];
}

int bspline_sample_run(Plan &p, int32_t d_poly, int32_t n_prod, const int32_t *order, const uint64_t *dims,
                       const uint32_t *anchor, void *f)
{
    if (d_poly < p.d || d_poly > 64) return fail(MR1L_E_ARG, "d_poly must be in [d, 64]");
    if (n_prod < 1 || n_prod > kBsMaxProd) return fail(MR1L_E_ARG, "n_prod must be in [1, 16]");
    if (!order || !dims || !f) return fail(MR1L_E_ARG, "null argument");
    if (d_poly > p.d && !anchor) return fail(MR1L_E_ARG, "anchors required when d_poly > d");
    BsDesc bs{};
    bs.n = n_prod;
    bs.d_poly = d_poly;
    for (int q = 0; q < n_prod; ++q) {
        const int m = order[q];
        if (m < 1 || m > kBsMaxOrder) return fail(MR1L_E_ARG, "B-spline order must be in [1, 16]");
        bs.order[q] = m;
        bs.scale[q] = m / std::sqrt(m * host_bspline(2 * m, (double)m));   // C_m m
    }
    const int64_t nd = (int64_t)p.F * n_prod;
    for (int64_t i = 0; i < nd; ++i)
        if (d_poly < 64 && (dims[i] >> d_poly)) return fail(MR1L_E_ARG, "dims names a coordinate >= d_poly");
    if (p.bs_bytes < nd * 8) {
        if (p.capturing) return fail(MR1L_E_ARG, "size the B-spline sampler before graph capture");
        p.bs_bytes = 0;
        if (int rc = plan_regrow(p, (void **)&p.d_bs_dims, (size_t)nd * 8)) return rc;
        p.bs_bytes = nd * 8;
    }
    MR1L_HIP(hipMemcpyAsync(p.d_bs_dims, dims, (size_t)nd * 8, hipMemcpyHostToDevice, p.stream));
    int32_t maxM = 1;
    for (int64_t m : p.M) maxM = std::max<int32_t>(maxM, (int32_t)m);
    const dim3 grid((unsigned)((maxM + 255) / 256), (unsigned)(p.F * p.L));
    if (p.dtype == MR1L_C128)
        hipLaunchKernelGGL(k_sample_bspline<double>, grid, dim3(256), 0, p.stream, p.d_lat, p.L, p.d, p.d_z64, bs,
                           (const uint64_t *)p.d_bs_dims, anchor, (double2 *)f);
    else
        hipLaunchKernelGGL(k_sample_bspline<float>, grid, dim3(256), 0, p.stream, p.d_lat, p.L, p.d, p.d_z64, bs,
                           (const uint64_t *)p.d_bs_dims, anchor, (float2 *)f);
    MR1L_LAUNCH_CHECK();
    // the host copy of dims may be released by the caller after return
    MR1L_HIP(hipStreamSynchronize(p.stream));
    return MR1L_OK;
}

}  // namespace mr1l
