// Least-squares coefficients on the detected set (Remark 2.9, least-squares
// variant): the coefficients c_k, k in the detected set I~, of the trigonometric
// polynomial that best fits the samples already taken on the fixed lattices.
// By Parseval on each lattice and the aliasing formula eq. (2.4),
//   sum_l sum_j |sum_k c_k e^{2 pi i j k.z_l / M_l} - f_l[j]|^2
//     = sum_l M_l sum_h |sum_{k : h_l(k) = h} c_k - ghat_l[h]|^2,
// so the normal equations are G c = b with
//   (G c)_k = sum_l M_l (sum of c over k's bucket of lattice l),
//   b_k     = sum_l M_l ghat_l[h_l(k)],
// a real symmetric positive semi-definite system solved by conjugate gradients.
//
//  k_lsq_mark / k_lsq_min / k_lsq_rep  per (candidate, lattice): the smallest
//      detected index sharing the bucket, or -1 when the candidate is alone in it
//      (bit l of its singleton mask);
//  k_lsq_cg  one workgroup per function: CG iterations with the bucket sums of
//      one lattice at a time in LDS.
#include <climits>

#include "mr1l_internal.h"

namespace mr1l {

constexpr int kLsqThreads = 1024;

__device__ __forceinline__ int64_t n_kept(const int64_t *n_det, int f, int64_t cap)
{
    const int64_t n = n_det[f];
    return n < cap ? n : cap;
}

__device__ __forceinline__ bool alone(const uint32_t *__restrict__ mask, int64_t e, int L, int l)
{
    return (mask[e * mask_words(L) + (l >> 5)] >> (l & 31)) & 1u;
}

__global__ __launch_bounds__(256) void k_lsq_mark(const LatDesc *__restrict__ lat, int L,
                                                  const int64_t *__restrict__ n_det, int64_t cap,
                                                  const int32_t *__restrict__ det_hash,
                                                  const uint32_t *__restrict__ mask, int32_t *__restrict__ owner)
{
    const int f = blockIdx.y;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t q = t / L;
    const int l = (int)(t - q * L);
    if (q >= n_kept(n_det, f, cap)) return;
    const int64_t e = (int64_t)f * cap + q;
    if (!alone(mask, e, L, l)) owner[lat[f * L + l].node_off + det_hash[e * L + l]] = INT_MAX;
}

__global__ __launch_bounds__(256) void k_lsq_min(const LatDesc *__restrict__ lat, int L,
                                                 const int64_t *__restrict__ n_det, int64_t cap,
                                                 const int32_t *__restrict__ det_hash,
                                                 const uint32_t *__restrict__ mask, int32_t *__restrict__ owner)
{
    const int f = blockIdx.y;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t q = t / L;
    const int l = (int)(t - q * L);
    if (q >= n_kept(n_det, f, cap)) return;
    const int64_t e = (int64_t)f * cap + q;
    if (!alone(mask, e, L, l)) atomicMin(owner + lat[f * L + l].node_off + det_hash[e * L + l], (int32_t)q);
}

__global__ __launch_bounds__(256) void k_lsq_rep(const LatDesc *__restrict__ lat, int L,
                                                 const int64_t *__restrict__ n_det, int64_t cap,
                                                 const int32_t *__restrict__ det_hash,
                                                 const uint32_t *__restrict__ mask,
                                                 const int32_t *__restrict__ owner, int32_t *__restrict__ rep)
{
    const int f = blockIdx.y;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t q = t / L;
    const int l = (int)(t - q * L);
    if (q >= n_kept(n_det, f, cap)) return;
    const int64_t e = (int64_t)f * cap + q;
    rep[e * L + l] = alone(mask, e, L, l) ? -1 : owner[lat[f * L + l].node_off + det_hash[e * L + l]];
}

// Sum of two doubles over the workgroup, returned to every thread (identical values:
// every thread adds the per-wave partials in the same order).
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red)
{
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
    __syncthreads();
    a = 0.0; b = 0.0;
    for (int i = 0; i < nw; ++i) { a += red[2 * i]; b += red[2 * i + 1]; }
    __syncthreads();
}

// Group sums of one lattice: in LDS (GS = false) or, for lists longer than the
// LDS holds, in global memory, where every access is an atomic at device scope
// so that the workgroup's threads see each other's sums after a barrier.
template <bool GS, typename T>
__device__ __forceinline__ void gsum_zero(T *a)
{
    if (GS) __hip_atomic_store(a, (T)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *a = (T)0;
}
template <bool GS, typename T>
__device__ __forceinline__ T gsum_load(const T *a)
{
    if (GS) return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *a;
}

// out = G v over the function's n detected candidates (entries owned by thread
// q mod blockDim).  s: group sums of one lattice, indexed by representative.
template <typename T, bool GS>
__device__ void apply_g(const LatDesc *__restrict__ lf, int L, int n, int64_t base,
                        const int32_t *__restrict__ rep, const typename cvec<T>::type *v,
                        typename cvec<T>::type *out, typename cvec<T>::type *s)
{
    using V = typename cvec<T>::type;
    for (int q = threadIdx.x; q < n; q += blockDim.x) { out[base + q].x = 0; out[base + q].y = 0; }
    for (int l = 0; l < L; ++l) {
        const T w = (T)lf[l].M;
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int rp = rep[(base + q) * L + l];
            if (rp >= 0) { gsum_zero<GS>(&s[rp].x); gsum_zero<GS>(&s[rp].y); }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int rp = rep[(base + q) * L + l];
            if (rp >= 0) {
                const V a = v[base + q];
                unsafeAtomicAdd(&s[rp].x, a.x);
                unsafeAtomicAdd(&s[rp].y, a.y);
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int rp = rep[(base + q) * L + l];
            V a;
            if (rp >= 0) { a.x = gsum_load<GS>(&s[rp].x); a.y = gsum_load<GS>(&s[rp].y); }
            else a = v[base + q];
            V o = out[base + q];
            o.x += w * a.x;
            o.y += w * a.y;
            out[base + q] = o;
        }
        __syncthreads();
    }
}

template <typename T, bool GS>
__global__ __launch_bounds__(kLsqThreads) void k_lsq_cg(
    const LatDesc *__restrict__ lat, int L, const int64_t *__restrict__ n_det, int64_t cap,
    const int32_t *__restrict__ det_hash, const int32_t *__restrict__ rep,
    const typename cvec<T>::type *__restrict__ ghat, int max_iter, double tol2, typename cvec<T>::type *x,
    typename cvec<T>::type *r, typename cvec<T>::type *pv, typename cvec<T>::type *ap,
    typename cvec<T>::type *gsums, double *__restrict__ resid, int32_t *__restrict__ iters)
{
    using V = typename cvec<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    V *s = GS ? gsums + (int64_t)blockIdx.x * cap : reinterpret_cast<V *>(smem);
    __shared__ double red[2 * (kLsqThreads / 64)];
    const int f = blockIdx.x;
    const int n = (int)n_kept(n_det, f, cap);
    const int64_t base = (int64_t)f * cap;
    const LatDesc *lf = lat + (int64_t)f * L;
    // b into r
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        double br = 0.0, bi = 0.0;
        for (int l = 0; l < L; ++l) {
            const V g = ghat[lf[l].node_off + det_hash[(base + q) * L + l]];
            br += (double)lf[l].M * (double)g.x;
            bi += (double)lf[l].M * (double)g.y;
        }
        r[base + q].x = (T)br;
        r[base + q].y = (T)bi;
    }
    apply_g<T, GS>(lf, L, n, base, rep, x, ap, s);
    double bb = 0.0, rr = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        V b = r[base + q];
        bb += (double)b.x * b.x + (double)b.y * b.y;
        const V a = ap[base + q];
        b.x -= a.x;
        b.y -= a.y;
        r[base + q] = b;
        pv[base + q] = b;
        rr += (double)b.x * b.x + (double)b.y * b.y;
    }
    block_sum2(bb, rr, red);
    int it = 0;
    while (it < max_iter && rr > tol2 * bb) {
        apply_g<T, GS>(lf, L, n, base, rep, pv, ap, s);
        double pap = 0.0, unused = 0.0;
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const V p = pv[base + q], a = ap[base + q];
            pap += (double)p.x * a.x + (double)p.y * a.y;
        }
        block_sum2(pap, unused, red);
        if (!(pap > 0.0)) break;
        const double alpha = rr / pap;
        double rn = 0.0;
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const V p = pv[base + q], a = ap[base + q];
            V xv = x[base + q], rv = r[base + q];
            xv.x += (T)(alpha * p.x);
            xv.y += (T)(alpha * p.y);
            rv.x -= (T)(alpha * a.x);
            rv.y -= (T)(alpha * a.y);
            x[base + q] = xv;
            r[base + q] = rv;
            rn += (double)rv.x * rv.x + (double)rv.y * rv.y;
        }
        block_sum2(rn, unused, red);
        const double beta = rn / rr;
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const V rv = r[base + q];
            V p = pv[base + q];
            p.x = (T)(rv.x + beta * p.x);
            p.y = (T)(rv.y + beta * p.y);
            pv[base + q] = p;
        }
        rr = rn;
        ++it;
    }
    if (threadIdx.x == 0) {
        if (resid) resid[f] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        if (iters) iters[f] = it;
    }
}

int lsq_init_attrs()
{
    MR1L_HIP(hipFuncSetAttribute((const void *)k_lsq_cg<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kMaxCap * 16));
    MR1L_HIP(hipFuncSetAttribute((const void *)k_lsq_cg<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kMaxCap * 8));
    return MR1L_OK;
}

int lsq_run(Plan &p, int64_t cap, const int64_t *n_det, const int32_t *det_hash, const uint32_t *det_mask,
            const void *ghat, int32_t max_iter, double tol, void *coef, double *resid, int32_t *iters,
            int32_t *rep, void *vecs)
{
    const int L = p.L;
    const size_t esz = p.dtype == MR1L_C128 ? 16 : 8;
    int32_t *owner = (int32_t *)p.d_nodes_scratch;   // [nodes] int32 view of the node scratch
    dim3 g((unsigned)((cap * L + 255) / 256), (unsigned)p.F), b(256);
    hipLaunchKernelGGL(k_lsq_mark, g, b, 0, p.stream, p.d_lat, L, n_det, cap, det_hash, det_mask, owner);
    MR1L_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_lsq_min, g, b, 0, p.stream, p.d_lat, L, n_det, cap, det_hash, det_mask, owner);
    MR1L_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_lsq_rep, g, b, 0, p.stream, p.d_lat, L, n_det, cap, det_hash, det_mask, owner, rep);
    MR1L_LAUNCH_CHECK();
    const bool gs = cap > kMaxCap;   // group sums in global memory
    const size_t shm = gs ? 0 : (size_t)cap * esz;
    const int64_t stride = p.F * cap;
    const dim3 grid((unsigned)p.F), blk(kLsqThreads);
    if (p.dtype == MR1L_C128) {
        double2 *v = (double2 *)vecs;
        if (gs)
            hipLaunchKernelGGL((k_lsq_cg<double, true>), grid, blk, 0, p.stream, p.d_lat, L, n_det, cap, det_hash,
                               rep, (const double2 *)ghat, max_iter, tol * tol, (double2 *)coef, v, v + stride,
                               v + 2 * stride, v + 3 * stride, resid, iters);
        else
            hipLaunchKernelGGL((k_lsq_cg<double, false>), grid, blk, shm, p.stream, p.d_lat, L, n_det, cap, det_hash,
                               rep, (const double2 *)ghat, max_iter, tol * tol, (double2 *)coef, v, v + stride,
                               v + 2 * stride, v + 3 * stride, resid, iters);
    } else {
        float2 *v = (float2 *)vecs;
        if (gs)
            hipLaunchKernelGGL((k_lsq_cg<float, true>), grid, blk, 0, p.stream, p.d_lat, L, n_det, cap, det_hash,
                               rep, (const float2 *)ghat, max_iter, tol * tol, (float2 *)coef, v, v + stride,
                               v + 2 * stride, v + 3 * stride, resid, iters);
        else
            hipLaunchKernelGGL((k_lsq_cg<float, false>), grid, blk, shm, p.stream, p.d_lat, L, n_det, cap, det_hash,
                               rep, (const float2 *)ghat, max_iter, tol * tol, (float2 *)coef, v, v + stride,
                               v + 2 * stride, v + 3 * stride, resid, iters);
    }
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

}  // namespace mr1l
