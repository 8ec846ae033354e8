// Lattice DFTs of prime size M by Bluestein's chirp convolution on the register
// FFT engine (lfft.h): normalised forward transforms (Algorithm 2, first loop), the
// inverse map and the kernel spectra, for the "reg" and "split" DFT schedules.
//
// With w[n] = e^{-pi i n^2 / M} and cw = conj(w),
//   ghat[h] = (w[h] / M) sum_{j<M} (f[j] w[j]) cw[h - j],   h < M,
// a linear convolution of the chirped input with cw on (-M, M).
//
// reg    one length-N transform pair per lattice, N the smallest power of two
//        >= 2M - 1 (up to 16384 in complex128, 32768 in complex64): load the
//        chirped input in the first pass's layout, forward FFT, times the
//        spectrum of cw (the 1/(N M) normalisation folded in), conjugate, FFT,
//        conjugate (the inverse transform), times the chirp.  Small N: several
//        lattices per workgroup.
// split  complex128 lattices too large for one workgroup (M <= 4 * 8192): the
//        input and the output are cut into K blocks of B = ceil(M / K) entries
//        (2B - 1 <= N = 16384).  Output block q is sum_p a_p * c_{q-p}, where a_p
//        is input block p (chirped) and c_s[m] = cw[s B + m], |m| < B, is one of
//        2K - 1 segments of the chirp; each term is a cyclic convolution of length
//        N, so  Y_q = sum_p FFT(a_p) Cs_{q-p}  with the segment spectra Cs_s.  cw
//        is even, so c_{-s}[m] = c_s[-m] (indices mod N) and Cs_{-s}[h] = Cs_s[-h]:
//        only the K spectra s = 0 .. K - 1 are stored.
//        One workgroup per lattice runs K forward and K inverse transforms; the
//        spectra of the first K - 1 blocks wait in a global scratch slot of the
//        workgroup (each thread reads back only what it wrote).
#pragma once

#include "lfft.h"
#include "mr1l_internal.h"

namespace mr1l {

namespace lf {

// Threads of a workgroup holding G transforms of length N with E values per thread.
template <int N, int E, int G> constexpr int wg_threads() { return ((G * (N / E) + 63) / 64) * 64; }

// Entries of the two-level chirp table of size M (S = 2^s >= sqrt(2M) low entries,
// ceil(2M / S) high ones), and their maximum over the sizes a transform of length N
// serves (2M - 1 <= N, or M <= 2N in blocks of at most N / 2 for the split kernel).
constexpr int chirp_entries(int M)
{
    int s = 0;
    while ((1 << (2 * s)) < 2 * M) ++s;
    return (1 << s) + (2 * M + (1 << s) - 1) / (1 << s);
}
constexpr int chirp_max(int Mmax)
{
    int c = 0;
    for (int M = 1; M <= Mmax; ++M) c = chirp_entries(M) > c ? chirp_entries(M) : c;
    return c;
}

// The lattice's chirp table into LDS, by the n threads t < n.
template <typename T>
__device__ __forceinline__ void load_chirp(typename cvec<T>::type *dst, const typename cvec<T>::type *src, int M,
                                           int nlo, int t, int n)
{
    const int nch = nlo + (2 * M + nlo - 1) / nlo;
    for (int i = t; i < nch; i += n) dst[i] = src[i];
}

// Chirp index r = n^2 mod 2M in 32-bit arithmetic (n^2 < 2^31): q from the high half
// of n^2 times floor((2^32 - 1) / 2M), which is at most two below the quotient.
struct ChirpMod {
    uint32_t d, magic;
    __device__ __forceinline__ explicit ChirpMod(int M) : d(2u * (uint32_t)M), magic(0xffffffffu / (2u * (uint32_t)M)) {}
    __device__ __forceinline__ uint32_t operator()(uint32_t n) const
    {
        const uint32_t sq = n * n;
        uint32_t r = sq - __umulhi(sq, magic) * d;
        if (r >= d) r -= d;
        if (r >= d) r -= d;
        return r;
    }
};

// w[n] = e^{-pi i (n^2 mod 2M) / M} from the two-level table of e^{-pi i r / M}
// (r = hi S + lo; entries [0, S) low part, [S, ...) high part).
template <typename T>
__device__ __forceinline__ typename cvec<T>::type chirp_at(const typename cvec<T>::type *tab, int shift, int nlo,
                                                           int n, const ChirpMod &cm)
{
    const uint32_t r = cm((uint32_t)n);
    const auto a = tab[r & (uint32_t)(nlo - 1)];
    const auto b = tab[nlo + (r >> shift)];
    typename cvec<T>::type o;
    o.x = a.x * b.x - a.y * b.y;
    o.y = a.x * b.y + a.y * b.x;
    return o;
}

}  // namespace lf

// ------------------------------------------------------------------ reg kernel
// Workgroup: G groups of N/E threads, group g on lattice blockIdx.x G + g.  LDS: G
// planes of N reals (one component at a time) or 2N (both, BOTH).
template <typename T, int N, int E, int G, bool BOTH, bool SPEC>
__global__ __launch_bounds__((lf::wg_threads<N, E, G>()), (lf::wg_threads<N, E, G>() >= 1024 ? 4 : 4)) void k_blu_reg(
    const int32_t *__restrict__ lats, int nl, const LatDesc *__restrict__ lat, const MDesc *__restrict__ md,
    const typename cvec<T>::type *__restrict__ in, typename cvec<T>::type *__restrict__ out,
    typename cvec<T>::type *__restrict__ spec_tab, const typename cvec<T>::type *__restrict__ chirp_tab,
    const typename cvec<T>::type *__restrict__ tw_tab, uint32_t *__restrict__ bitmap, T th2, int mode, T scale,
    int scale_by_m)
{
    using V = typename cvec<T>::type;
    using S = lf::Shape<N, E>;
    constexpr int NT = S::NT, R0 = S::R0, RL = S::RL;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int g = tid / NT;
    const int li0 = blockIdx.x * G + g;
    const bool act = g < G && li0 < nl;
    const int t = act ? tid - g * NT : 0;
    constexpr int CH = lf::chirp_max((N + 1) / 2);
    constexpr int PL = lf::plane_len<T>(N);
    T *re = reinterpret_cast<T *>(smem) + (size_t)(act ? g : 0) * (BOTH ? 2 * PL : PL);
    T *im = BOTH ? re + PL : re;
    V *ctab = reinterpret_cast<V *>(reinterpret_cast<T *>(smem) + (size_t)G * (BOTH ? 2 * PL : PL)) +
              (act ? g : 0) * CH;
    const LatDesc ld = lat[lats[act ? li0 : 0]];
    const MDesc m = md[ld.mid];
    const int M = ld.M;
    const lf::ChirpMod inv2m(M);
    const V *tw = tw_tab + m.tw_N;
    if (act) lf::load_chirp<T>(ctab, chirp_tab + m.chirp_off, M, m.chirp_nlo, t, NT);
    __syncthreads();
    const T cj = (mode == FFT_INV) ? T(-1) : T(1);
    T xr[E], xi[E];

    // inputs in the first pass's layout: value c R0 + q of thread t is entry
    // t + NT c + q N / R0 of the length-N sequence
    if (act) {
        const V *x = in + ld.node_off;
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int n = lf::in_pos<N, E, R0>(tt, e / R0, e % R0);
            if constexpr (SPEC) {
                // the kernel cw[n] for n < M and cw[N - n] at N - n, 0 < n < M
                const int src = n < M ? n : (n > N - M ? N - n : -1);
                const V w = lf::chirp_at<T>(ctab, m.chirp_shift, m.chirp_nlo, src < 0 ? 0 : src, inv2m);
                xr[e] = src < 0 ? T(0) : w.x;
                xi[e] = src < 0 ? T(0) : -w.y;
            } else {
                const V v = x[n < M ? n : 0];
                const V w = lf::chirp_at<T>(ctab, m.chirp_shift, m.chirp_nlo, n < M ? n : 0, inv2m);
                const T vi = cj * v.y;
                xr[e] = n < M ? v.x * w.x - vi * w.y : T(0);
                xi[e] = n < M ? v.x * w.y + vi * w.x : T(0);
            }
        }
    }
    lf::fft<T, N, E>(re, im, xr, xi, act, t, tw);
    if constexpr (SPEC) {
        if (act) {
            const T s = T(1) / ((T)N * (T)M);
            V *dst = spec_tab + m.spec_off;
            const int tt = lf::opq(t);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int h = tt + NT * (e / RL) + (e % RL) * (N / RL);
                V o;
                o.x = xr[e] * s;
                o.y = xi[e] * s;
                dst[h] = o;
            }
        }
        return;
    }
    // times the spectrum, conjugated: the second transform is an inverse one
    if (act) {
        const V *sp = spec_tab + m.spec_off;
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const V s = sp[tt + NT * (e / RL) + (e % RL) * (N / RL)];
            const T a = xr[e], b = xi[e];
            xr[e] = a * s.x - b * s.y;
            xi[e] = -(a * s.y + b * s.x);
        }
    }
    lf::relayout<T, N, E>(re, im, xr, xi, act, t);
    lf::fft<T, N, E>(re, im, xr, xi, act, t, tw);
    // ghat[h] = conj(conv[h]) w[h] scale for h < M; every lane takes part in the bitmap
    const T sc = scale_by_m ? scale * (T)M : scale;
    V *y = out + ld.node_off;
    const int tt = lf::opq(t);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int h = tt + NT * (e / RL) + (e % RL) * (N / RL);
        const bool ok = act && h < M;
        bool set = false;
        if (ok) {
            const V w = lf::chirp_at<T>(ctab, m.chirp_shift, m.chirp_nlo, h, inv2m);
            const T cr = xr[e], ci = -xi[e];
            const T gr = (cr * w.x - ci * w.y) * sc;
            T gi = (cr * w.y + ci * w.x) * sc;
            if (mode == FFT_INV) gi = -gi;
            V o;
            o.x = gr;
            o.y = gi;
            y[h] = o;
            set = gr * gr + gi * gi >= th2;
        }
        if (mode == FFT_FWD && bitmap) {
            // one lattice per workgroup and whole waves: a wave's lanes hold consecutive nodes
            if constexpr (G == 1 && NT % 64 == 0) bitmap_set_run(bitmap, ld.node_off + h, set);
            else bitmap_set_lanes(bitmap, ld.node_off + h, set);
        }
    }
}

// ------------------------------------------------------------------ split kernels
// One workgroup of N/E threads per lattice (persistent over the list), one LDS plane
// of N reals.  MDesc: N (transform length), N1 = B (block), N2 = K (blocks), spectra
// of the segments s = 0 .. K-1 at spec_off + s N (segment -s is segment s at -h).
// Scratch slot of the workgroup: (K - 1) N complex.

// Segment spectra of one size (one workgroup per size, the segments in turn):
// c_s[m'] = cw[s B + m'] at m' mod N for |m'| < B, transformed, times 1/(N M).
template <typename T, int N, int E>
__global__ __launch_bounds__(N / E) void k_blu_split_spec(
    const int32_t *__restrict__ lats, const LatDesc *__restrict__ lat, const MDesc *__restrict__ md,
    typename cvec<T>::type *__restrict__ spec_tab, const typename cvec<T>::type *__restrict__ chirp_tab,
    const typename cvec<T>::type *__restrict__ tw_tab)
{
    using V = typename cvec<T>::type;
    using S = lf::Shape<N, E>;
    constexpr int NT = S::NT, R0 = S::R0, RL = S::RL;
    extern __shared__ __align__(16) unsigned char smem[];
    T *pl = reinterpret_cast<T *>(smem);
    const int t = threadIdx.x;
    const LatDesc ld = lat[lats[blockIdx.x]];
    const MDesc m = md[ld.mid];
    const int M = ld.M, B = m.N1, K = m.N2;
    const lf::ChirpMod inv2m(M);
    V *ctab = reinterpret_cast<V *>(pl + lf::plane_len<T>(N));
    lf::load_chirp<T>(ctab, chirp_tab + m.chirp_off, M, m.chirp_nlo, t, NT);
    __syncthreads();
    const V *tw = tw_tab + m.tw_N;
    T xr[E], xi[E];
    for (int s = 0; s <= K - 1; ++s) {
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int n = lf::in_pos<N, E, R0>(tt, e / R0, e % R0);
            const int mm = n < B ? n : (n > N - B ? n - N : N);
            const bool nz = mm != N;
            const int64_t src = (int64_t)s * B + (nz ? mm : 0);
            const V w = lf::chirp_at<T>(ctab, m.chirp_shift, m.chirp_nlo, (int)(src < 0 ? -src : src), inv2m);
            xr[e] = nz ? w.x : T(0);
            xi[e] = nz ? -w.y : T(0);
        }
        lf::fft<T, N, E>(pl, pl, xr, xi, true, t, tw);
        const T sc = T(1) / ((T)N * (T)M);
        V *dst = spec_tab + m.spec_off + (int64_t)s * N;
        const int t2 = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            V o;
            o.x = xr[e] * sc;
            o.y = xi[e] * sc;
            dst[t2 + NT * (e / RL) + (e % RL) * (N / RL)] = o;
        }
    }
}

// Forward (FFT_FWD) or inverse (FFT_INV) transforms of lattices cut into K blocks.
template <typename T, int N, int E, int K>
__global__ __launch_bounds__(N / E) void k_blu_split(
    const int32_t *__restrict__ lats, int nl, const LatDesc *__restrict__ lat, const MDesc *__restrict__ md,
    const typename cvec<T>::type *__restrict__ in, typename cvec<T>::type *__restrict__ out,
    const typename cvec<T>::type *__restrict__ spec_tab, const typename cvec<T>::type *__restrict__ chirp_tab,
    const typename cvec<T>::type *__restrict__ tw_tab, uint32_t *__restrict__ bitmap, T th2, int mode, T scale,
    int scale_by_m, typename cvec<T>::type *__restrict__ scratch, int64_t slot_len)
{
    using V = typename cvec<T>::type;
    using S = lf::Shape<N, E>;
    constexpr int NT = S::NT, R0 = S::R0, RL = S::RL;
    extern __shared__ __align__(16) unsigned char smem[];
    T *pl = reinterpret_cast<T *>(smem);
    const int t = threadIdx.x;
    V *slot = scratch + (int64_t)blockIdx.x * slot_len;
    const T cj = (mode == FFT_INV) ? T(-1) : T(1);

    for (int li = blockIdx.x; li < nl; li += gridDim.x) {
        const LatDesc ld = lat[lats[li]];
        const MDesc m = md[ld.mid];
        const int M = ld.M, B = m.N1;
        const lf::ChirpMod inv2m(M);
        V *ctab = reinterpret_cast<V *>(pl + lf::plane_len<T>(N));
        __syncthreads();   // the previous lattice's last reads of the table are done
        lf::load_chirp<T>(ctab, chirp_tab + m.chirp_off, M, m.chirp_nlo, t, NT);
        __syncthreads();
        const V *tw = tw_tab + m.tw_N;
        T xr[E], xi[E];

        // forward transforms of the chirped input blocks; all but the last wait in
        // the slot in register order (value e of thread t at e NT + t)
#pragma unroll 1
        for (int p = 0; p < K; ++p) {
            const V *x = in + ld.node_off;
            const int tt = lf::opq(t);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int n = lf::in_pos<N, E, R0>(tt, e / R0, e % R0);
                const int j = p * B + n;
                const bool ok = n < B && j < M;
                const V v = x[ok ? j : 0];
                const V w = lf::chirp_at<T>(ctab, m.chirp_shift, m.chirp_nlo, ok ? j : 0, inv2m);
                const T vi = cj * v.y;
                xr[e] = ok ? v.x * w.x - vi * w.y : T(0);
                xi[e] = ok ? v.x * w.y + vi * w.x : T(0);
            }
            lf::fft<T, N, E>(pl, pl, xr, xi, true, t, tw);
            if (p < K - 1) {
                V *sl = slot + (int64_t)p * N;
                const int t2 = lf::opq(t);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    V o;
                    o.x = xr[e];
                    o.y = xi[e];
                    sl[e * NT + t2] = o;
                }
            }
        }
        // Y_q = sum_p X_p Cs_{q-p}, element by element: Y_{K-1} stays in the registers,
        // the others replace X_q in the slot; all conjugated for the inverse transforms
        {
            const V *sp = spec_tab + m.spec_off;
            const int tt = lf::opq(t);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int h = tt + NT * (e / RL) + (e % RL) * (N / RL);
                V X[K];
#pragma unroll
                for (int p = 0; p < K - 1; ++p) X[p] = slot[(int64_t)p * N + e * NT + tt];
                X[K - 1].x = xr[e];
                X[K - 1].y = xi[e];
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    T yr = 0, yi = 0;
#pragma unroll
                    for (int p = 0; p < K; ++p) {
                        // Cs_{q-p}[h], or Cs_{p-q}[-h mod N] for q < p
                        const V s = q >= p ? sp[(int64_t)(q - p) * N + h] : sp[(int64_t)(p - q) * N + ((N - h) & (N - 1))];
                        yr += X[p].x * s.x - X[p].y * s.y;
                        yi += X[p].x * s.y + X[p].y * s.x;
                    }
                    if (q == K - 1) {
                        xr[e] = yr;
                        xi[e] = -yi;
                    } else {
                        V o;
                        o.x = yr;
                        o.y = -yi;
                        slot[(int64_t)q * N + e * NT + tt] = o;
                    }
                }
                // keep the loads of later elements from being hoisted over this one
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // inverse transforms, last block first (its values are in the registers)
        const T sc = scale_by_m ? scale * (T)M : scale;
#pragma unroll 1
        for (int q = K - 1; q >= 0; --q) {
            if (q < K - 1) {
                const V *sl = slot + (int64_t)q * N;
                const int tt = lf::opq(t);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const V o = sl[e * NT + tt];
                    xr[e] = o.x;
                    xi[e] = o.y;
                }
            }
            lf::relayout<T, N, E>(pl, pl, xr, xi, true, t);
            lf::fft<T, N, E>(pl, pl, xr, xi, true, t, tw);
            V *y = out + ld.node_off;
            const int tt = lf::opq(t);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int hh = tt + NT * (e / RL) + (e % RL) * (N / RL);
                const int h = q * B + hh;
                const bool ok = hh < B && h < M;
                bool set = false;
                if (ok) {
                    const V w = lf::chirp_at<T>(ctab, m.chirp_shift, m.chirp_nlo, h, inv2m);
                    const T cr = xr[e], ci = -xi[e];
                    const T gr = (cr * w.x - ci * w.y) * sc;
                    T gi = (cr * w.y + ci * w.x) * sc;
                    if (mode == FFT_INV) gi = -gi;
                    V o;
                    o.x = gr;
                    o.y = gi;
                    y[h] = o;
                    set = gr * gr + gi * gi >= th2;
                }
                if (mode == FFT_FWD && bitmap) bitmap_set_run(bitmap, ld.node_off + h, set);
            }
        }
    }
}

// ------------------------------------------------------------------ launch tables
// Whole-transform lengths of the reg schedule and their shapes: E values per thread,
// G lattices per workgroup, both LDS planes at once when G N 2 w <= 64 KiB.
template <typename T, int N> struct RegCfg {
    static constexpr int E = N <= 16384 ? 16 : 32;
    static constexpr int NT = N / E;
    // 256-thread workgroups where one transform has fewer threads; one plane (the two
    // components in turn), so that four workgroups fit a CU's LDS and registers up to
    // 8192 points and the barrier phases of one overlap the others' work
    static constexpr int G = NT >= 256 ? 1 : 256 / NT;
    static constexpr bool BOTH = false;
    static constexpr int PL = lf::plane_len<T>(N);
    static constexpr size_t lds = (size_t)G * PL * (BOTH ? 2 : 1) * sizeof(T) +
                                  (size_t)G * lf::chirp_max((N + 1) / 2) * 2 * sizeof(T);
    static_assert(G >= 1 && lds <= (size_t)kLdsBytes, "reg schedule LDS budget");
};

template <typename T, int N>
static int reg_launch_n(Plan &p, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                        T th2, uint32_t *bitmap, int mode, T sc, int by_m)
{
    using V = typename cvec<T>::type;
    using C = RegCfg<T, N>;
    const int grid = (nl + C::G - 1) / C::G;
    if (mode == FFT_SPEC)
        hipLaunchKernelGGL((k_blu_reg<T, N, C::E, C::G, C::BOTH, true>), dim3((unsigned)grid),
                           dim3(lf::wg_threads<N, C::E, C::G>()), C::lds, p.stream, d_lats, nl, p.d_lat, d_md,
                           (const V *)in, (V *)out, (V *)p.d_spec, (const V *)p.d_chirp, (const V *)p.d_tw, bitmap,
                           th2, mode, sc, by_m);
    else
        hipLaunchKernelGGL((k_blu_reg<T, N, C::E, C::G, C::BOTH, false>), dim3((unsigned)grid),
                           dim3(lf::wg_threads<N, C::E, C::G>()), C::lds, p.stream, d_lats, nl, p.d_lat, d_md,
                           (const V *)in, (V *)out, (V *)p.d_spec, (const V *)p.d_chirp, (const V *)p.d_tw, bitmap,
                           th2, mode, sc, by_m);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

template <typename T>
int reg_launch_t(Plan &p, int N, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                 double theta, uint32_t *bitmap, int mode, double scale, int by_m)
{
    const T th2 = (T)(theta * theta), sc = (T)scale;
    if (nl <= 0) return MR1L_OK;
    switch (N) {
    case 64: return reg_launch_n<T, 64>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 128: return reg_launch_n<T, 128>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 256: return reg_launch_n<T, 256>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 512: return reg_launch_n<T, 512>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 1024: return reg_launch_n<T, 1024>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 2048: return reg_launch_n<T, 2048>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 4096: return reg_launch_n<T, 4096>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 8192: return reg_launch_n<T, 8192>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 16384: return reg_launch_n<T, 16384>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
    case 32768:
        if constexpr (sizeof(T) == 4)
            return reg_launch_n<T, 32768>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
        break;
    default: break;
    }
    return fail(MR1L_E_ARG, "no reg DFT kernel of length " + std::to_string(N));
}

template <typename T>
int reg_attrs_t()
{
    auto set = [](const void *k, size_t b) {
        return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b) == hipSuccess;
    };
#define MR1L_REG_ATTR(NN)                                                                                         \
    if (!set((const void *)k_blu_reg<T, NN, RegCfg<T, NN>::E, RegCfg<T, NN>::G, RegCfg<T, NN>::BOTH, false>,   \
             RegCfg<T, NN>::lds) ||                                                                               \
        !set((const void *)k_blu_reg<T, NN, RegCfg<T, NN>::E, RegCfg<T, NN>::G, RegCfg<T, NN>::BOTH, true>,    \
             RegCfg<T, NN>::lds))                                                                                 \
        return fail(MR1L_E_HIP, "reg DFT kernel attribute");
    MR1L_REG_ATTR(64) MR1L_REG_ATTR(128) MR1L_REG_ATTR(256) MR1L_REG_ATTR(512) MR1L_REG_ATTR(1024)
    MR1L_REG_ATTR(2048) MR1L_REG_ATTR(4096) MR1L_REG_ATTR(8192) MR1L_REG_ATTR(16384)
    if constexpr (sizeof(T) == 4) { MR1L_REG_ATTR(32768) }
#undef MR1L_REG_ATTR
    return MR1L_OK;
}

// split: complex128, N = 16384 with 16 values per thread (1024 threads, one 128 KiB
// plane and the chirp table of M <= 4 N / 2); one launch per block count K (cls).
constexpr int kSplitE = 16;
constexpr size_t kSplitLds = (size_t)lf::plane_len<double>(kSplitLen) * sizeof(double) +
                             (size_t)lf::chirp_max(kSplitMaxK * kSplitLen / 2) * 2 * sizeof(double);

template <typename T, int K>
static int split_launch_k(Plan &p, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                          double theta, uint32_t *bitmap, int mode, double scale, int by_m)
{
    using V = typename cvec<T>::type;
    const int grid = std::min(nl, std::min(p.fft_slots, num_cus()));
    if (grid < 1 || p.fft_slot_len < (int64_t)(K - 1) * kSplitLen) return fail(MR1L_E_ARG, "split DFT without a scratch slot");
    hipLaunchKernelGGL((k_blu_split<T, kSplitLen, kSplitE, K>), dim3((unsigned)grid), dim3(kSplitLen / kSplitE),
                       kSplitLds, p.stream, d_lats, nl, p.d_lat, d_md, (const V *)in, (V *)out,
                       (const V *)p.d_spec, (const V *)p.d_chirp, (const V *)p.d_tw, bitmap, (T)(theta * theta),
                       mode, (T)scale, by_m, (V *)p.d_fft_scratch, p.fft_slot_len);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

template <typename T>
int split_launch_t(Plan &p, int K, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                   double theta, uint32_t *bitmap, int mode, double scale, int by_m)
{
    using V = typename cvec<T>::type;
    if (nl <= 0) return MR1L_OK;
    if constexpr (sizeof(T) != 8) {
        return fail(MR1L_E_ARG, "the split DFT schedule is complex128 only");
    } else {
        if (mode == FFT_SPEC) {
            hipLaunchKernelGGL((k_blu_split_spec<T, kSplitLen, kSplitE>), dim3((unsigned)nl),
                               dim3(kSplitLen / kSplitE), kSplitLds, p.stream, d_lats, p.d_lat,
                               d_md, (V *)p.d_spec, (const V *)p.d_chirp, (const V *)p.d_tw);
            MR1L_LAUNCH_CHECK();
            return MR1L_OK;
        }
        switch (K) {
        case 2: return split_launch_k<T, 2>(p, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);
        case 3: return split_launch_k<T, 3>(p, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);
        case 4: return split_launch_k<T, 4>(p, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);
        default: return fail(MR1L_E_ARG, "split DFT: block count must be 2, 3 or 4");
        }
    }
}

template <typename T>
int split_attrs_t()
{
    if constexpr (sizeof(T) == 8) {
        auto set = [](const void *k) {
            return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSplitLds) == hipSuccess;
        };
        if (!set((const void *)k_blu_split_spec<T, kSplitLen, kSplitE>) ||
            !set((const void *)k_blu_split<T, kSplitLen, kSplitE, 2>) ||
            !set((const void *)k_blu_split<T, kSplitLen, kSplitE, 3>) ||
            !set((const void *)k_blu_split<T, kSplitLen, kSplitE, 4>))
            return fail(MR1L_E_HIP, "split DFT kernel attribute");
    }
    return MR1L_OK;
}

}  // namespace mr1l
