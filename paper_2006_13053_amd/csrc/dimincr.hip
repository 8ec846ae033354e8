// Dimension-incremental driver: Algorithm 3 with Algorithm 4 as the detection
// method (Section 3.2.2).
//
// Step 1 (optional; otherwise every I^(t) is the whole range [-N, N]): all
// d x r one-dimensional problems run as one batched plan of composite size
// K = 2N + 1 -- the polynomial with coordinate t moved first, anchors for the
// others, samples on the grid l / K, the normalised DFT, and Algorithm 4 over
// the K frequencies [-N, N] keeping the s_local largest; I^(t) is the union
// over the r repetitions.
//
// Per step t = 2..d and repetition i = 1..r~:
//   J_t = I^(1..t-1) x I^(t)                  (k_cartesian, lexicographic)
//   L   = eq. (4.2) on |J_t|, every lattice of size M
//   draws from SplitMix64 stream (seed, t, i): anchors, then generating vectors
//   samples on the t-dimensional lattices with the anchors fixed (Step 2b)
//   mr1l_fft + mr1l_extract with s~ (Step 2c)
//   union of the detected tuples (Step 2d): a bitmap over J compacted in ascending
//   order (J is lexicographic, so the union is sorted and has no repeats)
// The rt repetitions of a step are the rt functions of one batched plan; J, the
// union and the next step's tuples stay on the device (one transfer per step).
#include "mr1l_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>

namespace mr1l {

// SplitMix64 (Steele, Lea, Flood 2014): output n of seed S is the finaliser of
// S + n * 0x9E3779B97F4A7C15.
static uint64_t splitmix(uint64_t seed, uint64_t n)
{
    uint64_t x = seed + n * 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

// Step 2 streams: n = ((t*64 + i) << 24) + c + 1; Step 1 streams add 2^62.
struct Stream {
    uint64_t seed, base, c = 0;
    Stream(uint64_t s, int t, int i, bool step1 = false)
        : seed(s), base((step1 ? (uint64_t(1) << 62) : 0u) + (((uint64_t)t * 64u + (uint64_t)i) << 24)) {}
    uint64_t next() { return splitmix(seed, base + (c++) + 1u); }
    int64_t below(int64_t m) { return (int64_t)(((unsigned __int128)next() * (uint64_t)m) >> 64); }
};

// J = prev x set, lexicographic: J[u][a * K + b] = prev[u][a] (u < tm1), set[b].
__global__ void k_cartesian(const int64_t *__restrict__ prev, int64_t nprev, int tm1,
                            const int64_t *__restrict__ set, int64_t K, int64_t *__restrict__ J)
{
    const int64_t nJ = nprev * K;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nJ; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = q / K, b = q - a * K;
        for (int u = 0; u < tm1; ++u) J[(int64_t)u * nJ + q] = prev[(int64_t)u * nprev + a];
        J[(int64_t)tm1 * nJ + q] = set[b];
    }
}

// Step 1 lists for Algorithm 4: entry q of problem f is the frequency q - N with
// the DFT value at index (q - N) mod K.
template <typename T>
__global__ void k_line_gather(int F, int64_t K, int64_t N, const typename cvec<T>::type *__restrict__ ghat,
                              int64_t *__restrict__ det_idx, typename cvec<T>::type *__restrict__ det_coef,
                              int64_t *__restrict__ n_det)
{
    const int f = blockIdx.y;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < K; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t h = (q + N + 1) % K;   // (q - N) mod K
        det_idx[(int64_t)f * K + q] = q;
        det_coef[(int64_t)f * K + q] = ghat[(int64_t)f * K + h];
        if (q == 0) n_det[f] = K;
    }
}

// J = prev x set, lexicographic, written rt times (one copy per repetition's
// function): J[u][f nJ + a K + b] = prev[u][a] (u < tm1), set[b].
__global__ void k_cartesian_rep(const int64_t *__restrict__ prev, int64_t nprev, int64_t prev_stride, int tm1,
                                const int64_t *__restrict__ set, int64_t K, int rt, int64_t *__restrict__ J)
{
    const int64_t nJ = nprev * K, tot = nJ * rt;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < tot; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = g % nJ;
        const int64_t a = q / K, b = q - a * K;
        for (int u = 0; u < tm1; ++u) J[(int64_t)u * tot + g] = prev[(int64_t)u * prev_stride + a];
        J[(int64_t)tm1 * tot + g] = set[b];
    }
}

// rows x n int64 values, each row written rt times side by side: dst[r][f n + j] = src[r][j].
__global__ void k_replicate(const int64_t *__restrict__ src, int rows, int64_t n, int rt, int64_t *__restrict__ dst)
{
    const int64_t tot = (int64_t)rows * n * rt;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < tot; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = g / (n * rt), rem = g - r * n * rt, j = rem % n;
        dst[g] = src[r * n + j];
    }
}

// Step 2d union: the output lists of the rt repetitions (indices into the same J) set
// bits of one bitmap over J; the bitmap's set bits in ascending order are the union,
// already lexicographic and without repeats (J is built in lexicographic order).
__global__ void k_union_mark(const int64_t *__restrict__ n_out, const int64_t *__restrict__ out_idx, int64_t s_cap,
                             int rt, uint32_t *__restrict__ bits)
{
    const int f = blockIdx.y;
    const int64_t n = min(n_out[f], s_cap);
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = out_idx[(int64_t)f * s_cap + q];
        atomicOr(bits + (j >> 5), 1u << (j & 31));
    }
}

constexpr int kUnionWords = 256;   // bitmap words per counting block (one per thread)

__device__ __forceinline__ int union_block_scan(int v, int *sh)
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
    return sh[tid] - v;
}

__global__ __launch_bounds__(kUnionWords) void k_union_count(const uint32_t *__restrict__ bits, int64_t nwords,
                                                             int32_t *__restrict__ cnt)
{
    __shared__ int sh[kUnionWords];
    const int64_t w = (int64_t)blockIdx.x * kUnionWords + threadIdx.x;
    const int c = w < nwords ? __popc(bits[w]) : 0;
    const int before = union_block_scan(c, sh);
    if (threadIdx.x == blockDim.x - 1) cnt[blockIdx.x] = before + c;
}

// exclusive offsets of the counting blocks; stat[0] = the union's size
__global__ void k_union_scan(int nb, int32_t *__restrict__ cnt, int64_t *__restrict__ stat)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    for (int x = 0; x < nb; ++x) {
        const int v = cnt[x];
        cnt[x] = (int32_t)acc;
        acc += v;
    }
    stat[0] = acc;
}

// the union's tuples: column u of J at each set bit, in ascending order, to prev_out
// (SoA [t][cap_prev]; entries beyond cap_prev are counted but not written)
__global__ __launch_bounds__(kUnionWords) void k_union_emit(const uint32_t *__restrict__ bits, int64_t nwords,
                                                            const int32_t *__restrict__ off,
                                                            const int64_t *__restrict__ J, int64_t Jstride, int t,
                                                            int64_t cap_prev, int64_t *__restrict__ prev_out)
{
    __shared__ int sh[kUnionWords];
    const int64_t w = (int64_t)blockIdx.x * kUnionWords + threadIdx.x;
    uint32_t b = w < nwords ? bits[w] : 0u;
    int64_t r = off[blockIdx.x] + union_block_scan(__popc(b), sh);
    while (b) {
        const int j = __ffs(b) - 1;
        b &= b - 1;
        const int64_t q = w * 32 + j;
        if (r < cap_prev)
            for (int u = 0; u < t; ++u) prev_out[(int64_t)u * cap_prev + r] = J[(int64_t)u * Jstride + q];
        ++r;
    }
}

// A device buffer of the driver, grown on demand; blocks go back to the library's cache
// once the driver's stream is done with them.
template <typename P> struct DevBuf {
    hipStream_t s;
    P *p = nullptr;
    int64_t n = 0;
    explicit DevBuf(hipStream_t st) : s(st) {}
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf()
    {
        if (!p) return;
        (void)hipStreamSynchronize(s);
        dev_free(p);
    }
    int need(int64_t cnt)
    {
        if (cnt <= n) return MR1L_OK;
        if (p) {
            MR1L_HIP(hipStreamSynchronize(s));
            dev_free(p);
        }
        p = nullptr;
        n = 0;
        if (int rc = dev_alloc((void **)&p, sizeof(P) * (size_t)std::max<int64_t>(cnt, 1))) return rc;
        n = cnt;
        return MR1L_OK;
    }
};

struct PlanHolder {
    mr1l_plan p = nullptr;
    ~PlanHolder() { if (p) mr1l_plan_destroy(p); }
};

}  // namespace mr1l

using namespace mr1l;

extern "C" int mr1l_dimincr(const mr1l_dimincr_params *prm, mr1l_sample_fn fn, void *user,
                            const int64_t *poly_freq, const void *poly_coef, int64_t poly_s, int64_t cap,
                            int64_t *n_out, int64_t *freq_out, void *coef_out, int64_t *total_samples, void *stream)
{
    if (!prm || !n_out || !freq_out || !coef_out) return fail(MR1L_E_ARG, "null argument");
    const mr1l_dimincr_params P = *prm;
    if (P.d < 2 || P.d > kMaxD) return fail(MR1L_E_ARG, "d must be in [2, 64]");
    if (P.N < 0 || P.s < 1 || P.s_local < P.s || P.r < 1) return fail(MR1L_E_ARG, "invalid N, s, s_local or r");
    if (P.dtype != MR1L_C128 && P.dtype != MR1L_C64) return fail(MR1L_E_ARG, "invalid dtype");
    const bool bsp = !fn && P.bs_n > 0;
    if (P.bs_n < 0 || P.bs_n > 16) return fail(MR1L_E_ARG, "bs_n must be in [0, 16]");
    if (!fn && !bsp && (poly_s < 0 || (poly_s > 0 && (!poly_freq || !poly_coef))))
        return fail(MR1L_E_ARG, "built-in sampler needs the polynomial");
    if (cap < P.s) return fail(MR1L_E_CAPACITY, "cap below s");
    const hipStream_t st = (hipStream_t)stream;
    const int d = P.d;
    const int64_t K = 2 * P.N + 1;
    const size_t esz = P.dtype == MR1L_C128 ? 16 : 8;
    *n_out = 0;
    int64_t samples = 0;

    DevBuf<int64_t> dprev{st}, dJ{st}, n_det{st}, det_idx{st}, n_o{st}, out_idx{st}, dset{st};
    DevBuf<unsigned char> fbuf{st}, gbuf{st}, det_coef{st}, out_coef{st};
    DevBuf<uint32_t> bitmap{st};
    int rc;

    // single-coordinate sets I^(t), t = 1..d
    std::vector<std::vector<int64_t>> I1(d);
    if (!P.step1) {
        for (int t = 0; t < d; ++t)
            for (int64_t a = 0; a < K; ++a) I1[t].push_back(a - P.N);
    } else {
        if (fn) return fail(MR1L_E_ARG, "Step 1 needs the built-in sampler");
        if (K > kMaxCap) return fail(MR1L_E_ARG, "Step 1 needs 2N + 1 <= 8192");
        if (!bsp && poly_s < 1) return fail(MR1L_E_ARG, "Step 1 needs a non-empty polynomial");
        // the polynomial on the host, then one copy per (t, i) with coordinate t first
        // (for the B-spline function: its coordinate masks with bit t moved to bit 0)
        const int64_t ps = bsp ? 0 : poly_s;
        std::vector<int64_t> hf((size_t)d * ps);
        std::vector<unsigned char> hc((size_t)ps * esz);
        if (ps > 0) {
            MR1L_HIP(hipMemcpyAsync(hf.data(), poly_freq, hf.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
            MR1L_HIP(hipMemcpyAsync(hc.data(), poly_coef, hc.size(), hipMemcpyDeviceToHost, st));
            MR1L_HIP(hipStreamSynchronize(st));
        }
        const int F1 = d * P.r;
        const int64_t T1 = (int64_t)F1 * ps;
        std::vector<int64_t> rf((size_t)d * T1), toff(F1 + 1);
        std::vector<unsigned char> rcf((size_t)T1 * esz);
        std::vector<uint32_t> anc1((size_t)F1 * (d - 1));
        std::vector<uint64_t> bdims((size_t)F1 * std::max(1, P.bs_n));
        for (int f = 0; f < F1; ++f) {
            const int t = f / P.r + 1, i = f % P.r + 1;
            toff[f] = (int64_t)f * ps;
            for (int q = 0; q < (bsp ? P.bs_n : 0); ++q) {
                uint64_t m = (P.bs_dims[q] >> (t - 1)) & 1u;
                int row = 1;
                for (int u = 0; u < d; ++u)
                    if (u != t - 1) m |= ((P.bs_dims[q] >> u) & 1u) << (row++);
                bdims[(size_t)f * P.bs_n + q] = m;
            }
            for (int64_t q = 0; q < ps; ++q) {
                const int64_t col = (int64_t)f * poly_s + q;
                rf[col] = hf[(size_t)(t - 1) * poly_s + q];
                int row = 1;
                for (int u = 0; u < d; ++u)
                    if (u != t - 1) rf[(size_t)(row++) * T1 + col] = hf[(size_t)u * poly_s + q];
            }
            std::memcpy(rcf.data() + (size_t)f * poly_s * esz, hc.data(), (size_t)poly_s * esz);
            Stream rs(P.seed, t, i, true);
            for (int j = 0; j < d - 1; ++j) anc1[(size_t)f * (d - 1) + j] = (uint32_t)(rs.next() >> 32);
        }
        toff[F1] = T1;
        DevBuf<int64_t> drf{st}, dtoff{st};
        DevBuf<unsigned char> drc{st};
        DevBuf<uint32_t> danc1{st};
        if ((rc = drf.need(std::max<int64_t>(1, (int64_t)rf.size()))) || (rc = dtoff.need(F1 + 1)) ||
            (rc = drc.need(std::max<int64_t>(1, (int64_t)rcf.size()))) || (rc = danc1.need((int64_t)anc1.size())))
            return rc;
        if (ps > 0) {
            MR1L_HIP(hipMemcpyAsync(drf.p, rf.data(), rf.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
            MR1L_HIP(hipMemcpyAsync(drc.p, rcf.data(), rcf.size(), hipMemcpyHostToDevice, st));
        }
        MR1L_HIP(hipMemcpyAsync(dtoff.p, toff.data(), toff.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        MR1L_HIP(hipMemcpyAsync(danc1.p, anc1.data(), anc1.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        std::vector<int64_t> M1(F1, K), z1(F1, 1);
        PlanHolder p1;
        if ((rc = plan_create_impl(&p1.p, 1, F1, 1, M1.data(), z1.data(), P.dtype, stream, false))) return rc;
        const int64_t nodes1 = (int64_t)F1 * K;
        if ((rc = fbuf.need(nodes1 * esz)) || (rc = gbuf.need(nodes1 * esz)) || (rc = n_det.need(F1)) ||
            (rc = det_idx.need(nodes1)) || (rc = det_coef.need(nodes1 * esz)) || (rc = n_o.need(F1)) ||
            (rc = out_idx.need((int64_t)F1 * P.s_local)) || (rc = out_coef.need((int64_t)F1 * P.s_local * esz)))
            return rc;
        if (bsp) {
            if ((rc = bspline_sample_run(plan_of(p1.p), d, P.bs_n, P.bs_order, bdims.data(), danc1.p, fbuf.p)))
                return rc;
        } else if ((rc = mr1l_sample(p1.p, d, dtoff.p, T1, drf.p, drc.p, danc1.p, fbuf.p, 1))) {
            return rc;
        }
        if ((rc = mr1l_fft(p1.p, fbuf.p, gbuf.p, P.theta, nullptr))) return rc;
        const dim3 gg((unsigned)std::min<int64_t>((K + 255) / 256, 64), (unsigned)F1);
        if (P.dtype == MR1L_C128)
            hipLaunchKernelGGL(k_line_gather<double>, gg, dim3(256), 0, st, F1, K, P.N, (const double2 *)gbuf.p,
                               det_idx.p, (double2 *)det_coef.p, n_det.p);
        else
            hipLaunchKernelGGL(k_line_gather<float>, gg, dim3(256), 0, st, F1, K, P.N, (const float2 *)gbuf.p,
                               det_idx.p, (float2 *)det_coef.p, n_det.p);
        MR1L_LAUNCH_CHECK();
        if ((rc = limit_run(plan_of(p1.p), n_det.p, K, det_idx.p, det_coef.p, P.theta, P.s_local, n_o.p, out_idx.p,
                            out_coef.p)))
            return rc;
        std::vector<int64_t> hn(F1), hi((size_t)F1 * P.s_local);
        MR1L_HIP(hipMemcpyAsync(hn.data(), n_o.p, F1 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        MR1L_HIP(hipMemcpyAsync(hi.data(), out_idx.p, hi.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        MR1L_HIP(hipStreamSynchronize(st));
        samples += nodes1;
        for (int t = 0; t < d; ++t) {
            std::vector<char> in(K, 0);
            for (int i = 0; i < P.r; ++i) {
                const int f = t * P.r + i;
                for (int64_t q = 0; q < hn[f]; ++q) in[hi[(size_t)f * P.s_local + q]] = 1;
            }
            for (int64_t a = 0; a < K; ++a)
                if (in[a]) I1[t].push_back(a - P.N);
        }
    }

    // Step 2 on the device: per step t, the rt repetitions are the rt functions of one
    // batched plan (their own lattices and anchors, the same candidate set J in rt
    // copies), sampled, transformed and detected together; their union and the next
    // step's tuples stay on the device, and one transfer per step brings the union's
    // size and the detected counts to the host.
    int64_t nprev = (int64_t)I1[0].size();
    if (nprev == 0) {
        if (total_samples) *total_samples = samples;
        return MR1L_OK;   // nothing detected: the result is empty
    }
    int64_t prev_stride = nprev;   // columns of the SoA tuples in dprev
    if ((rc = dprev.need(nprev))) return rc;
    MR1L_HIP(hipMemcpyAsync(dprev.p, I1[0].data(), nprev * sizeof(int64_t), hipMemcpyHostToDevice, st));
    DevBuf<int64_t> dnext{st}, dstat{st}, dstage{st}, drf{st};
    DevBuf<unsigned char> drc{st};
    DevBuf<uint32_t> dbits{st};
    DevBuf<int32_t> dcnt{st};
    std::vector<int64_t> hst;   // a step's small host tables (uploaded in one copy)
    std::vector<uint64_t> bdims;   // B-spline coordinate masks per repetition (uploaded by the sampler)
    int rep_rt = 0;             // repetitions the replicated polynomial in drf/drc holds
    bool long_lists = false;    // a step overflowed the short-list capacity: later steps take the long path

    for (int t = 2; t <= d; ++t) {
        const int rt = (t < d) ? P.r : 1;
        const int64_t s_t = (t < d) ? P.s_local : P.s;
        const std::vector<int64_t> &It = I1[t - 1];
        const int64_t Kt = (int64_t)It.size();
        const int64_t nJ = nprev * Kt;
        if (nJ == 0) {
            *n_out = 0;
            if (total_samples) *total_samples = samples;
            return MR1L_OK;
        }
        const int32_t L = mr1l_num_lattices(nJ, P.c, P.delta);
        if (L < 1 || L > kMaxL) return fail(MR1L_E_ARG, "eq. (4.2) lattice count out of range");
        const int64_t nJr = nJ * rt;
        // draws of every repetition: anchors, then generating vectors
        std::vector<uint32_t> anc((size_t)rt * std::max(1, d - t), 0u);
        std::vector<int64_t> z((size_t)rt * L * t);
        for (int i = 1; i <= rt; ++i) {
            Stream rs(P.seed, t, i);
            for (int u = t; u < d; ++u) anc[(size_t)(i - 1) * (d - t) + (u - t)] = (uint32_t)(rs.next() >> 32);
            for (int l = 0; l < L; ++l)
                for (int u = 0; u < t; ++u) z[((size_t)(i - 1) * L + l) * t + u] = rs.below(P.M);
        }
        std::vector<int64_t> Ms((size_t)rt * L, P.M);
        PlanHolder plan;
        if ((rc = mr1l_plan_create(&plan.p, t, rt, L, Ms.data(), z.data(), P.dtype, stream))) return rc;
        // the step's small tables in one upload: I^(t), the sets' offsets, the terms'
        // offsets and the anchors (hst lives until the step's synchronisation)
        const int64_t na = (int64_t)anc.size(), o_so = Kt, o_to = o_so + rt + 1, o_an = o_to + rt + 1;
        hst.assign((size_t)(o_an + (na + 1) / 2), 0);
        std::copy(It.begin(), It.end(), hst.begin());
        for (int f = 0; f <= rt; ++f) {
            hst[o_so + f] = (int64_t)f * nJ;
            hst[o_to + f] = (int64_t)f * poly_s;
        }
        std::memcpy(hst.data() + o_an, anc.data(), (size_t)na * sizeof(uint32_t));
        if ((rc = dJ.need(nJr * t)) || (rc = dstage.need((int64_t)hst.size()))) return rc;
        MR1L_HIP(hipMemcpyAsync(dstage.p, hst.data(), hst.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        const int64_t *d_set = dstage.p, *d_setoff = dstage.p + o_so, *d_toff = dstage.p + o_to;
        const uint32_t *d_anc = d > t ? (const uint32_t *)(dstage.p + o_an) : nullptr;
        // J in rt copies
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((nJr + 255) / 256, 4096));
        hipLaunchKernelGGL(k_cartesian_rep, dim3((unsigned)blocks), dim3(256), 0, st, dprev.p, nprev, prev_stride,
                           t - 1, d_set, Kt, rt, dJ.p);
        MR1L_LAUNCH_CHECK();

        // samples of every repetition (Step 2b)
        const int64_t nodes_f = (int64_t)L * P.M, nodes = nodes_f * rt;
        if ((rc = fbuf.need(nodes * esz)) || (rc = gbuf.need(nodes * esz)) || (rc = bitmap.need((nodes + 31) / 32)))
            return rc;
        if (fn) {
            for (int i = 0; i < rt; ++i)
                if (fn(user, t, L, Ms.data() + (size_t)i * L, z.data() + (size_t)i * L * t,
                       anc.data() + (size_t)i * std::max(1, d - t), fbuf.p + (size_t)i * nodes_f * esz, stream) != 0)
                    return fail(MR1L_E_ARG, "sampling callback failed");
        } else if (bsp) {
            bdims.assign((size_t)rt * P.bs_n, 0u);
            for (int i = 0; i < rt; ++i)
                for (int q = 0; q < P.bs_n; ++q) bdims[(size_t)i * P.bs_n + q] = P.bs_dims[q];
            if ((rc = bspline_sample_run(plan_of(plan.p), d, P.bs_n, P.bs_order, bdims.data(), d_anc, fbuf.p)))
                return rc;
        } else {
            // the polynomial's terms once per repetition (kept while rt stays the same)
            if (rt != rep_rt) {
                const int64_t cw = (int64_t)esz / 8;   // int64 words per coefficient
                if ((rc = drf.need(std::max<int64_t>(1, (int64_t)d * poly_s * rt))) ||
                    (rc = drc.need(std::max<int64_t>(1, poly_s * rt) * (int64_t)esz)))
                    return rc;
                if (poly_s > 0) {
                    const int64_t rb =
                        std::max<int64_t>(1, std::min<int64_t>(((int64_t)d * poly_s * rt + 255) / 256, 4096));
                    hipLaunchKernelGGL(k_replicate, dim3((unsigned)rb), dim3(256), 0, st, poly_freq, d, poly_s, rt,
                                       drf.p);
                    MR1L_LAUNCH_CHECK();
                    hipLaunchKernelGGL(k_replicate, dim3((unsigned)rb), dim3(256), 0, st, (const int64_t *)poly_coef,
                                       1, poly_s * cw, rt, (int64_t *)drc.p);
                    MR1L_LAUNCH_CHECK();
                }
                rep_rt = rt;
            }
            if ((rc = mr1l_sample(plan.p, d, d_toff, poly_s * rt, drf.p, drc.p, d_anc, fbuf.p, 1))) return rc;
        }
        samples += nodes;
        if ((rc = mr1l_fft(plan.p, fbuf.p, gbuf.p, P.theta, bitmap.p))) return rc;

        // Algorithm 4 on every repetition (Step 2c): short lists unless a step overflowed
        if ((rc = n_det.need(rt)) || (rc = n_o.need(rt)) || (rc = out_idx.need((int64_t)rt * s_t)) ||
            (rc = out_coef.need((int64_t)rt * s_t * esz)) || (rc = dstat.need(1 + rt)))
            return rc;
        auto extract = [&](int64_t ecap) -> int {
            int r2;
            if ((r2 = det_idx.need((int64_t)rt * ecap)) || (r2 = det_coef.need((int64_t)rt * ecap * esz))) return r2;
            mr1l_extract_opts o{P.theta, 0, P.postproc, s_t, ecap};
            mr1l_extract_out ex{};
            ex.n_det = n_det.p; ex.det_idx = det_idx.p; ex.det_coef = det_coef.p;
            ex.n_out = n_o.p; ex.out_idx = out_idx.p; ex.out_coef = out_coef.p;
            return mr1l_extract(plan.p, nJr, d_setoff, dJ.p, gbuf.p, bitmap.p, &o, &ex);
        };
        const int64_t long_cap = std::min<int64_t>(kMaxCapLarge, std::max<int64_t>(nJ, s_t));
        int64_t ecap = (long_lists || s_t > kMaxCap) ? long_cap : std::max<int64_t>(kMaxCap, s_t);
        if ((rc = extract(ecap))) return rc;

        if (t < d) {
            // union of the repetitions' outputs (Step 2d), then the next step's tuples
            const int64_t nwords = (nJ + 31) / 32;
            const int nb = (int)((nwords + kUnionWords - 1) / kUnionWords);
            const int64_t cap_prev = std::min<int64_t>(nJ, (int64_t)rt * s_t);
            if ((rc = dbits.need(nwords)) || (rc = dcnt.need(nb)) || (rc = dnext.need(std::max<int64_t>(1, cap_prev * t))))
                return rc;
            auto unite = [&]() -> int {
                int r2 = launch_fill_u32(dbits.p, nwords, 0u, st);
                if (r2) return r2;
                const dim3 gm((unsigned)std::max<int64_t>(1, std::min<int64_t>((s_t + 255) / 256, 64)), (unsigned)rt);
                hipLaunchKernelGGL(k_union_mark, gm, dim3(256), 0, st, n_o.p, out_idx.p, s_t, rt, dbits.p);
                MR1L_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_union_count, dim3((unsigned)nb), dim3(kUnionWords), 0, st, dbits.p, nwords,
                                   dcnt.p);
                MR1L_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_union_scan, dim3(1), dim3(64), 0, st, nb, dcnt.p, dstat.p);
                MR1L_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_union_emit, dim3((unsigned)nb), dim3(kUnionWords), 0, st, dbits.p, nwords,
                                   dcnt.p, dJ.p, nJr, t, cap_prev, dnext.p);
                MR1L_LAUNCH_CHECK();
                MR1L_HIP(hipMemcpyAsync(dstat.p + 1, n_det.p, rt * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
                return MR1L_OK;
            };
            if ((rc = unite())) return rc;
            std::vector<int64_t> hs(1 + rt);
            MR1L_HIP(hipMemcpyAsync(hs.data(), dstat.p, hs.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
            MR1L_HIP(hipStreamSynchronize(st));
            bool over = false;
            for (int f = 0; f < rt; ++f) over = over || hs[1 + f] > ecap;
            if (over) {
                if (ecap >= long_cap) return fail(MR1L_E_CAPACITY, "detected set exceeds the capacity of one step");
                // a list overflowed the short capacity: this step again with the long path
                long_lists = true;
                ecap = long_cap;
                if ((rc = extract(ecap)) || (rc = unite())) return rc;
                MR1L_HIP(hipMemcpyAsync(hs.data(), dstat.p, hs.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
                MR1L_HIP(hipStreamSynchronize(st));
                for (int f = 0; f < rt; ++f)
                    if (hs[1 + f] > ecap) return fail(MR1L_E_CAPACITY, "detected set exceeds the capacity of one step");
            }
            if (hs[0] > cap) return fail(MR1L_E_CAPACITY, "union exceeds cap");
            nprev = hs[0];
            if (nprev == 0) {
                *n_out = 0;
                if (total_samples) *total_samples = samples;
                return MR1L_OK;   // nothing detected: the result is empty
            }
            std::swap(dprev.p, dnext.p);
            std::swap(dprev.n, dnext.n);
            prev_stride = cap_prev;
            continue;
        }

        // t = d: the output list (one repetition) to the host, in lexicographic order
        int64_t h_ndet = 0, h_nout = 0;
        MR1L_HIP(hipMemcpyAsync(&h_ndet, n_det.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        MR1L_HIP(hipMemcpyAsync(&h_nout, n_o.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        MR1L_HIP(hipStreamSynchronize(st));
        if (h_ndet > ecap) {
            if (ecap >= long_cap) return fail(MR1L_E_CAPACITY, "detected set exceeds the capacity of one step");
            ecap = long_cap;
            if ((rc = extract(ecap))) return rc;
            MR1L_HIP(hipMemcpyAsync(&h_ndet, n_det.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            MR1L_HIP(hipMemcpyAsync(&h_nout, n_o.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            MR1L_HIP(hipStreamSynchronize(st));
            if (h_ndet > ecap) return fail(MR1L_E_CAPACITY, "detected set exceeds the capacity of one step");
        }
        std::vector<int64_t> oi(h_nout), hprev((size_t)(t - 1) * nprev);
        std::vector<unsigned char> oc(h_nout * esz);
        if (h_nout > 0) {
            MR1L_HIP(hipMemcpy(oi.data(), out_idx.p, h_nout * sizeof(int64_t), hipMemcpyDeviceToHost));
            MR1L_HIP(hipMemcpy(oc.data(), out_coef.p, h_nout * esz, hipMemcpyDeviceToHost));
            for (int u = 0; u < t - 1; ++u)
                MR1L_HIP(hipMemcpy(hprev.data() + (size_t)u * nprev, dprev.p + (int64_t)u * prev_stride,
                                   nprev * sizeof(int64_t), hipMemcpyDeviceToHost));
        }
        std::vector<int64_t> cur;   // row-major d-tuples
        std::vector<unsigned char> cur_coef = oc;
        for (int64_t q = 0; q < h_nout; ++q) {
            const int64_t a = oi[q] / Kt, b = oi[q] - a * Kt;
            for (int u = 0; u < t - 1; ++u) cur.push_back(hprev[(size_t)u * nprev + a]);
            cur.push_back(It[b]);
        }
        if (P.lsq_iters > 0 && h_nout > 0) {
            // least squares on the output frequencies with this step's samples (Remark 2.9):
            // every output is kept (theta 0, one vote), then CG on the normal equations
            std::vector<int64_t> soa2((size_t)d * h_nout);
            for (int64_t q = 0; q < h_nout; ++q)
                for (int u = 0; u < d; ++u) soa2[(size_t)u * h_nout + q] = cur[(size_t)q * d + u];
            DevBuf<int64_t> dsel{st}, n2{st}, i2{st}, o2n{st}, o2i{st};
            DevBuf<unsigned char> c2{st}, o2c{st};
            DevBuf<double> res{st};
            if ((rc = dsel.need((int64_t)soa2.size())) || (rc = n2.need(1)) || (rc = i2.need(h_nout)) ||
                (rc = c2.need(h_nout * esz)) || (rc = o2n.need(1)) || (rc = o2i.need(h_nout)) ||
                (rc = o2c.need(h_nout * esz)) || (rc = res.need(1)))
                return rc;
            MR1L_HIP(hipMemcpyAsync(dsel.p, soa2.data(), soa2.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
            if ((rc = launch_fill_u32(bitmap.p, (nodes + 31) / 32, 0xffffffffu, st))) return rc;
            mr1l_extract_opts o2{0.0, 1, P.postproc, h_nout, h_nout};
            mr1l_extract_out ex2{};
            ex2.n_det = n2.p; ex2.det_idx = i2.p; ex2.det_coef = c2.p;
            ex2.n_out = o2n.p; ex2.out_idx = o2i.p; ex2.out_coef = o2c.p;
            if ((rc = mr1l_extract(plan.p, h_nout, nullptr, dsel.p, gbuf.p, bitmap.p, &o2, &ex2))) return rc;
            Plan &pp = plan_of(plan.p);
            if ((rc = mr1l_lsq(plan.p, h_nout, n2.p, i2.p, pp.d_ex_hash, pp.d_ex_mask, gbuf.p, P.lsq_iters,
                               1e-14, c2.p, res.p, nullptr, 0.0, 1, nullptr, nullptr, nullptr)))
                return rc;
            // the detected list is every output in ascending position: coefficient q belongs to row q
            std::vector<int64_t> hi2(h_nout);
            MR1L_HIP(hipMemcpyAsync(hi2.data(), i2.p, h_nout * sizeof(int64_t), hipMemcpyDeviceToHost, st));
            std::vector<unsigned char> hc2(h_nout * esz);
            MR1L_HIP(hipMemcpyAsync(hc2.data(), c2.p, h_nout * esz, hipMemcpyDeviceToHost, st));
            MR1L_HIP(hipStreamSynchronize(st));
            for (int64_t q = 0; q < h_nout; ++q)
                std::memcpy(cur_coef.data() + hi2[q] * esz, hc2.data() + q * esz, esz);
        }
        if (h_nout > cap) return fail(MR1L_E_CAPACITY, "union exceeds cap");
        // ascending J index is lexicographic order
        std::vector<int64_t> order(h_nout);
        for (int64_t q = 0; q < h_nout; ++q) order[q] = q;
        std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return oi[x] < oi[y]; });
        for (int64_t q = 0; q < h_nout; ++q) {
            for (int u = 0; u < d; ++u) freq_out[q * d + u] = cur[(size_t)order[q] * d + u];
            std::memcpy((unsigned char *)coef_out + q * esz, cur_coef.data() + order[q] * esz, esz);
        }
        *n_out = h_nout;
    }
    if (total_samples) *total_samples = samples;
    return MR1L_OK;
}
