// Lattice DFTs of prime size M with M - 1 = 2^a 5^b (a >= 2, b >= 1) by Rader's
// algorithm, the whole transform in registers: for h != 0,
//   ghat[g^-p] = (1/M) (f[0] + sum_q f[g^q] w^(-g^(q-p))),   w = e^{2 pi i / M},
// a cyclic convolution of length P = M - 1 of a[q] = f[g^q] with
// b[n] = w^(-g^-n) (g a primitive root mod M), done as a length-P DFT of a, a
// product with the precomputed DFT of b (1/P folded in), and a second length-P
// DFT of the conjugate (an inverse DFT is conj(DFT(conj(.)))).  ghat[0] is the
// mean of f.  One workgroup per lattice: each of the P/E active threads holds
// E values in registers through Stockham passes of radix 40 (8 x 5), 20 (4 x 5), 10,
// 5, 4 or 2 (the register FFT engine); between passes the values move through one LDS
// plane of P reals, real and imaginary parts in turn.  Nothing goes through global
// scratch.
#include <complex>
#include <map>
#include <mutex>
#include <vector>

#include "lfft.h"
#include "mr1l_internal.h"

namespace mr1l {

// Values per thread: every supported length P = M - 1 (the prime lattice sizes
// M = 20 2^i 5^j + 1 up to 16001) gets its own kernel on the register FFT engine
// (lfft.h) with E values in each of P / E threads, so the pass sequence and all index
// arithmetic are compile-time constants.  E = 20 (radices 20, 10, 5, 4, 2), except
// P = 16000: E = 40 in 400 threads, passes of radix 40, 40, 10 (two LDS exchanges per
// transform instead of three; 256 VGPRs, seven waves per lattice), 4-5% faster than
// 800 threads of 20.
constexpr int kRaderSizes[] = {40, 100, 400, 640, 1600, 4000, 16000};
template <int P> constexpr int rader_e() { return P == 16000 ? 40 : 20; }

template <int P> constexpr int rader_threads() { return (P / rader_e<P>() + 63) / 64 * 64; }

// mode: FFT_FWD (ghat = (1/M) sum f w^{-jh} times scale, and the non-zero bitmap) or
// FFT_INV (scale (1/M) sum g w^{+jh}, times M when scale_by_m).  One workgroup per
// lattice, one LDS plane of P reals (the two components in turn).
template <typename T, int P>
__global__ __launch_bounds__(rader_threads<P>()) void k_rader(
    const int32_t *__restrict__ lats, const LatDesc *__restrict__ lat, const RaderDesc *__restrict__ rdesc,
    const int32_t *__restrict__ itab, const typename cvec<T>::type *__restrict__ ctab,
    const typename cvec<T>::type *__restrict__ in, typename cvec<T>::type *__restrict__ out,
    uint32_t *__restrict__ bitmap, T th2, int mode, T scale, int scale_by_m)
{
    using V = typename cvec<T>::type;
    using S = lf::Shape<P, rader_e<P>()>;
    constexpr int E = rader_e<P>(), NT = S::NT, NTH = rader_threads<P>(), R0 = S::R0, RL = S::RL;
    extern __shared__ __align__(16) unsigned char smem[];
    T *pl = reinterpret_cast<T *>(smem);
    __shared__ double red[2 * (NTH / 64)];
    const LatDesc ld = lat[lats[blockIdx.x]];
    const RaderDesc *rd = rdesc + ld.mid;
    const int M = P + 1;
    const int tid = threadIdx.x;
    const bool act = tid < NT;
    const int t = act ? tid : 0;   // inactive threads mirror thread 0 (in range), results unused
    const int32_t *pin = itab + rd->perm_in;
    const int32_t *pout = itab + rd->perm_out;
    const V *tw = ctab + rd->tw;
    const V *sp = ctab + rd->spec;
    const T cj = (mode == FFT_INV) ? T(-1) : T(1);
    const V *x = in + ld.node_off;
    T xr[E], xi[E];

    // f[1..P] in natural order, coalesced: value e of thread t is f[1 + t + NT e]; the
    // real parts go to the plane at once, the imaginary parts wait in registers
    T vy[E];
    double sr = 0.0, si = 0.0;
    if (act) {
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const V v = x[1 + tt + NT * e];
            pl[lf::padq<T, E>(tt + NT * e)] = v.x;
            vy[e] = cj * v.y;
            sr += v.x;
            si += vy[e];
        }
    }
    // ghat[0] needs the sum of f
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o);
        si += __shfl_xor(si, o);
    }
    if ((tid & 63) == 0) { red[2 * (tid >> 6)] = sr; red[2 * (tid >> 6) + 1] = si; }
    __syncthreads();
    // a[q] = f[g^q] in the first pass's input layout (q = t + NT c + m P / R0); the
    // gather positions (< P < 2^16) are kept two to a register
    static_assert(E % 2 == 0 && P < 65536, "gather positions are packed in 16-bit pairs");
    uint32_t gpk[E / 2];
    auto gidx = [&](int e) -> int { return (int)((e & 1) ? (gpk[e >> 1] >> 16) : (gpk[e >> 1] & 0xffffu)); };
    if (act) {
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; e += 2)
            gpk[e / 2] = (uint32_t)(pin[lf::in_pos<P, E, R0>(tt, e / R0, e % R0)] - 1) |
                         ((uint32_t)(pin[lf::in_pos<P, E, R0>(tt, (e + 1) / R0, (e + 1) % R0)] - 1) << 16);
#pragma unroll
        for (int e = 0; e < E; ++e) xr[e] = pl[lf::padq<T, E>(gidx(e))];
    }
    __syncthreads();
    if (act) {
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) pl[lf::padq<T, E>(tt + NT * e)] = vy[e];
    }
    __syncthreads();
    if (act)
#pragma unroll
        for (int e = 0; e < E; ++e) xi[e] = pl[lf::padq<T, E>(gidx(e))];
    __syncthreads();

    // forward length-P DFT of a; times the spectrum of b (with 1/P), conjugated; the
    // second DFT is then the inverse one (conjugated result): the cyclic convolution
    lf::fft<T, P, E>(pl, pl, xr, xi, act, t, tw);
    if (act) {
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const V s = sp[tt + NT * (e / RL) + (e % RL) * (P / RL)];
            const T ar = xr[e], ai = xi[e];
            xr[e] = ar * s.x - ai * s.y;
            xi[e] = -(ar * s.y + ai * s.x);
        }
    }
    lf::relayout<T, P, E>(pl, pl, xr, xi, act, t);
    lf::fft<T, P, E>(pl, pl, xr, xi, act, t, tw);

    // ghat[g^-p] = (f[0] + conv[p]) / M (conv[p] = conj of the value at natural p):
    // scattered through the plane into natural order, then complex stores, coalesced
    V f0 = x[0];
    f0.y *= cj;
    const T sc = (scale_by_m ? scale * (T)M : scale) / (T)M;
    if (act) {
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; e += 2)
            gpk[e / 2] = (uint32_t)(pout[tt + NT * (e / RL) + (e % RL) * (P / RL)] - 1) |
                         ((uint32_t)(pout[tt + NT * ((e + 1) / RL) + ((e + 1) % RL) * (P / RL)] - 1) << 16);
#pragma unroll
        for (int e = 0; e < E; ++e) pl[lf::padq<T, E>(gidx(e))] = (f0.x + xr[e]) * sc;
    }
    __syncthreads();
    if (act) {
        const int tt = lf::opq(t);
#pragma unroll
        for (int e = 0; e < E; ++e) xr[e] = pl[lf::padq<T, E>(tt + NT * e)];
    }
    __syncthreads();
    if (act)
#pragma unroll
        for (int e = 0; e < E; ++e) pl[lf::padq<T, E>(gidx(e))] = cj * (f0.y - xi[e]) * sc;
    __syncthreads();
    V *y = out + ld.node_off;
    const int tt = lf::opq(t);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        bool set = false;
        if (act) {
            V o;
            o.x = xr[e];
            o.y = pl[lf::padq<T, E>(tt + NT * e)];
            y[1 + tt + NT * e] = o;
            set = o.x * o.x + o.y * o.y >= th2;
        }
        // every lane takes part: a wave's lanes hold consecutive nodes
        if (mode == FFT_FWD && bitmap) bitmap_set_run(bitmap, ld.node_off + 1 + tt + NT * e, set);
    }
    if (tid == 0) {
        double ar = 0.0, ai = 0.0;
        for (int w = 0; w < NTH / 64; ++w) { ar += red[2 * w]; ai += red[2 * w + 1]; }
        V o;
        o.x = (T)(((double)f0.x + ar) * (double)sc);
        o.y = (T)(cj * ((double)f0.y + ai) * (double)sc);
        y[0] = o;
        if (mode == FFT_FWD && bitmap && o.x * o.x + o.y * o.y >= th2)
            atomicOr(bitmap + (ld.node_off >> 5), 1u << (ld.node_off & 31));
    }
}

// ------------------------------------------------------------------ host
static int64_t powmod(int64_t a, int64_t e, int64_t m)
{
    int64_t r = 1 % m;
    a %= m;
    while (e > 0) {
        if (e & 1) r = (int64_t)((__int128)r * a % m);
        a = (int64_t)((__int128)a * a % m);
        e >>= 1;
    }
    return r;
}

static bool is_prime_host(int64_t n)
{
    if (n < 2) return false;
    for (int64_t q = 2; q * q <= n; ++q)
        if (n % q == 0) return false;
    return true;
}

// Radix list of P = 2^a 5^b for the register layout (a >= 2, b >= 1), or empty.
static std::vector<int> rader_radices(int64_t P)
{
    int a = 0, b = 0;
    int64_t Q = P;
    while (Q % 2 == 0) { Q /= 2; ++a; }
    while (Q % 5 == 0) { Q /= 5; ++b; }
    std::vector<int> r;
    if (Q != 1 || a < 2 || b < 1) return r;
    for (int i = 0; i < a / 2; ++i) r.push_back(4);
    if (a % 2) r.push_back(2);
    for (int i = 0; i < b; ++i) r.push_back(5);
    return r;
}

bool rader_applies(int64_t M, size_t real_bytes)
{
    const int64_t P = M - 1;
    bool listed = false;
    for (int q : kRaderSizes) listed = listed || q == P;
    if (!listed) return false;
    // one LDS plane of P reals
    if ((int64_t)real_bytes * P + 2048 > kLdsBytes) return false;
    if (rader_radices(P).empty()) return false;
    return is_prime_host(M);
}

// Length-n DFT (n = 2^a 5^b) in long double, by recursive decimation in time.
static void dft_ld(std::vector<std::complex<long double>> &x)
{
    const size_t n = x.size();
    if (n == 1) return;
    const size_t r = (n % 2 == 0) ? 2 : 5;
    const size_t m = n / r;
    std::vector<std::vector<std::complex<long double>>> sub(r, std::vector<std::complex<long double>>(m));
    for (size_t s = 0; s < r; ++s)
        for (size_t j = 0; j < m; ++j) sub[s][j] = x[j * r + s];
    for (auto &v : sub) dft_ld(v);
    const long double tp = -6.283185307179586476925286766559005768L / (long double)n;
    for (size_t k = 0; k < n; ++k) {
        std::complex<long double> acc = 0;
        for (size_t s = 0; s < r; ++s) {
            const size_t e = (s * k) % n;
            acc += sub[s][k % m] * std::complex<long double>(cosl(tp * e), sinl(tp * e));
        }
        x[k] = acc;
    }
}

// Appends the tables of size M: permutations (itab) and twiddles and spectrum
// (ctab, interleaved re/im of T).
template <typename T>
static int rader_tables_compute(int64_t M, RaderDesc &rd, std::vector<int32_t> &itab, std::vector<T> &ctab);

// The tables of one size, computed once per process (the recursive long-double DFT
// of the kernel takes tens of milliseconds at M = 16001) and appended to the plan's.
template <typename T>
int rader_tables(int64_t M, RaderDesc &rd, std::vector<int32_t> &itab, std::vector<T> &ctab)
{
    struct Entry {
        RaderDesc rd;
        std::vector<int32_t> itab;
        std::vector<T> ctab;
    };
    static std::mutex mu;
    static std::map<int64_t, Entry> cache;
    const Entry *e;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(M);
        if (it == cache.end()) {
            Entry n;
            rader_tables_compute<T>(M, n.rd, n.itab, n.ctab);
            it = cache.emplace(M, std::move(n)).first;
        }
        e = &it->second;
    }
    rd = e->rd;
    const int64_t ioff = (int64_t)itab.size(), coff = (int64_t)ctab.size() / 2;
    rd.perm_in += ioff;
    rd.perm_out += ioff;
    rd.tw += coff;
    rd.spec += coff;
    itab.insert(itab.end(), e->itab.begin(), e->itab.end());
    ctab.insert(ctab.end(), e->ctab.begin(), e->ctab.end());
    return MR1L_OK;
}

template <typename T>
static int rader_tables_compute(int64_t M, RaderDesc &rd, std::vector<int32_t> &itab, std::vector<T> &ctab)
{
    const int64_t P = M - 1;
    const std::vector<int> rad = rader_radices(P);
    rd = RaderDesc{};
    rd.P = (int32_t)P;
    rd.nthreads = (int32_t)(P / 20);
    for (int r : rad) {
        if (r == 4) rd.n4++;
        else if (r == 2) rd.n2++;
        else rd.n5++;
    }
    // primitive root
    int64_t g = 2;
    for (;; ++g) {
        if (powmod(g, P / 2, M) != 1 && powmod(g, P / 5, M) != 1) break;
    }
    const int64_t ginv = powmod(g, M - 2, M);
    rd.perm_in = (int64_t)itab.size();
    for (int64_t q = 0, v = 1; q < P; ++q, v = v * g % M) itab.push_back((int32_t)v);
    rd.perm_out = (int64_t)itab.size();
    for (int64_t q = 0, v = 1; q < P; ++q, v = v * ginv % M) itab.push_back((int32_t)v);
    rd.tw = (int64_t)ctab.size() / 2;
    const long double tpP = -6.283185307179586476925286766559005768L / (long double)P;
    for (int64_t x = 0; x < P; ++x) {
        ctab.push_back((T)cosl(tpP * x));
        ctab.push_back((T)sinl(tpP * x));
    }
    // spectrum of b[n] = w^(-g^-n), with the 1/P of the inverse DFT
    std::vector<std::complex<long double>> b((size_t)P);
    const long double tpM = -6.283185307179586476925286766559005768L / (long double)M;
    for (int64_t q = 0, v = 1; q < P; ++q, v = v * ginv % M)
        b[(size_t)q] = std::complex<long double>(cosl(tpM * v), sinl(tpM * v));
    dft_ld(b);
    rd.spec = (int64_t)ctab.size() / 2;
    for (int64_t k = 0; k < P; ++k) {
        ctab.push_back((T)(b[(size_t)k].real() / (long double)P));
        ctab.push_back((T)(b[(size_t)k].imag() / (long double)P));
    }
    return MR1L_OK;
}
template int rader_tables<double>(int64_t, RaderDesc &, std::vector<int32_t> &, std::vector<double> &);
template int rader_tables<float>(int64_t, RaderDesc &, std::vector<int32_t> &, std::vector<float> &);

template <typename T, int P>
static int rader_attr()
{
    MR1L_HIP(hipFuncSetAttribute((const void *)k_rader<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 lf::plane_len<T, rader_e<P>()>(P) * (int)sizeof(T)));
    return MR1L_OK;
}

template <typename T, int... Ps>
static int rader_attrs()
{
    int rc = MR1L_OK;
    ((rc = rc ? rc : rader_attr<T, Ps>()), ...);
    return rc;
}

int rader_init_attrs()
{
    int rc = rader_attrs<double, 40, 100, 400, 640, 1600, 4000, 16000>();
    return rc ? rc : rader_attrs<float, 40, 100, 400, 640, 1600, 4000, 16000>();
}

template <typename T, int P>
static int rader_go(Plan &p, const int32_t *d_lats, int nl, const void *in, void *out, T th2, uint32_t *bitmap,
                    int mode, T scale, int by_m)
{
    using V = typename cvec<T>::type;
    constexpr size_t shm = (size_t)lf::plane_len<T, rader_e<P>()>(P) * sizeof(T);
    hipLaunchKernelGGL((k_rader<T, P>), dim3((unsigned)nl), dim3(rader_threads<P>()), shm,
                       p.stream, d_lats, p.d_lat, p.d_rdesc, p.d_ritab, (const V *)p.d_rctab, (const V *)in,
                       (V *)out, bitmap, th2, mode, scale, by_m);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

template <typename T>
static int rader_dispatch(Plan &p, int P, const int32_t *d_lats, int nl, const void *in, void *out, T th2,
                          uint32_t *bitmap, int mode, T scale, int by_m)
{
#define MR1L_RADER(Q) \
    case Q: return rader_go<T, Q>(p, d_lats, nl, in, out, th2, bitmap, mode, scale, by_m);
    switch (P) {
        MR1L_RADER(40) MR1L_RADER(100) MR1L_RADER(400) MR1L_RADER(640) MR1L_RADER(1600) MR1L_RADER(4000)
        MR1L_RADER(16000)
    default: return fail(MR1L_E_ARG, "no Rader kernel for this lattice size");
    }
#undef MR1L_RADER
}

int rader_launch(Plan &p, int P, const int32_t *d_lats, int nl, const void *in, void *out, double theta,
                 uint32_t *bitmap, int mode, double scale, int by_m)
{
    if (nl <= 0) return MR1L_OK;
    if (mode == FFT_SPEC) return MR1L_OK;   // the Rader spectra are built on the host
    if (p.dtype == MR1L_C128)
        return rader_dispatch<double>(p, P, d_lats, nl, in, out, theta * theta, bitmap, mode, scale, by_m);
    return rader_dispatch<float>(p, P, d_lats, nl, in, out, (float)(theta * theta), bitmap, mode, (float)scale, by_m);
}

}  // namespace mr1l
