// Lattice DFTs of prime size M with M - 1 = 2^a 5^b (a >= 2, b >= 1) by Rader's
// algorithm, the whole transform in registers: for h != 0,
//   ghat[g^-p] = (1/M) (f[0] + sum_q f[g^q] w^(-g^(q-p))),   w = e^{2 pi i / M},
// a cyclic convolution of length P = M - 1 of a[q] = f[g^q] with
// b[n] = w^(-g^-n) (g a primitive root mod M), done as a length-P DFT of a, a
// product with the precomputed DFT of b (1/P folded in), and a second length-P
// DFT of the conjugate (an inverse DFT is conj(DFT(conj(.)))).  ghat[0] is the
// mean of f.  One workgroup per lattice: each of the P/20 active threads holds
// 20 values in registers through Stockham passes of radix 20 (4 x 5), 10, 5, 4 or 2; between
// passes the values move through one LDS plane (P reals), real and imaginary
// parts in turn.  Nothing goes through global scratch.
#include <complex>
#include <map>
#include <mutex>
#include <vector>

#include "mr1l_internal.h"

namespace mr1l {

// Values per thread.  Every supported length P = M - 1 (the prime lattice sizes
// M = 20 2^i 5^j + 1 up to P = 20480) gets its own kernel, so that the pass sequence,
// the sub-lengths and all index arithmetic are compile-time constants.  40 values in
// half the threads was slower in double: fewer waves to hide the LDS and barrier
// latency.
constexpr int kRaderE = 20;
constexpr int kRaderSizes[] = {40, 100, 400, 640, 1600, 4000, 16000};

constexpr int rader_log(int P, int b)
{
    int n = 0;
    while (P % b == 0) { P /= b; ++n; }
    return n;
}

// The transform of length P: 20 values in each of P/20 threads, through Stockham
// passes whose radices divide 20: first the factors of P / 20^k that are left
// (10, else fours, a five, a two), then k passes of radix 20, k as large as possible.
template <int P> struct RShape {
    static constexpr int E = kRaderE;
    static constexpr int Tn = P / E;
    static constexpr int threads = (Tn + 63) / 64 * 64;
    static constexpr int n20()
    {
        int k = 0, q = P;
        while (q % 20 == 0) { q /= 20; ++k; }
        return k;
    }
    static constexpr int rest() { int q = P; for (int k = 0; k < n20(); ++k) q /= 20; return q; }
    static constexpr int small_radix(int q) { return q % 10 == 0 ? 10 : q % 4 == 0 ? 4 : q % 5 == 0 ? 5 : 2; }
    static constexpr int nsmall()
    {
        int k = 0;
        for (int q = rest(); q > 1; q /= small_radix(q)) ++k;
        return k;
    }
    static constexpr int NP = nsmall() + n20();
    static constexpr int radix(int i)
    {
        int q = rest();
        for (int k = 0; k < nsmall(); ++k) {
            if (k == i) return small_radix(q);
            q /= small_radix(q);
        }
        return 20;
    }
    static constexpr int sub(int i)   // sub-length before pass i
    {
        int L = 1;
        for (int k = 0; k < i; ++k) L *= radix(k);
        return L;
    }
    static constexpr int R0 = radix(0), RL = radix(NP - 1), Llast = sub(NP - 1);
    static_assert(P % E == 0 && sub(NP) == P && Tn <= 1024, "P = 20 2^i 5^j <= 20480");
};

// Hides a value from the optimiser so that per-pass index arithmetic is not hoisted
// out of the pass sequence (which would hold all passes' indices in registers).
__device__ __forceinline__ int rader_opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// cos and sin of 18 m degrees (W_20^m = cos - i sin), from the exact values of the
// multiples of 18 degrees.
template <typename T> __device__ __forceinline__ constexpr T cos18(int m)
{
    constexpr T c[6] = {(T)1, (T)0.95105651629515357211643933337938214, (T)0.80901699437494742410229341718281906,
                        (T)0.58778525229247312916870595463907277, (T)0.30901699437494742410229341718281906, (T)0};
    m = ((m % 20) + 20) % 20;
    return m <= 5 ? c[m] : m <= 10 ? -c[10 - m] : m <= 15 ? -c[m - 10] : c[20 - m];
}
template <typename T> __device__ __forceinline__ constexpr T sin18(int m) { return cos18<T>(m - 5); }

template <typename T, int R>
__device__ __forceinline__ void dft_small(T *xr, T *xi);

// DFT of length R = R1 R2 (R2 = 5) by the index split n = R2 n1 + n2, k = k1 + R1 k2:
// R2 DFTs of length R1, twiddles W_R^{n2 k1}, R1 DFTs of length R2.
template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_composite(T *xr, T *xi)
{
    constexpr int R = R1 * R2;
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        T ar[R1], ai[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) { ar[n1] = xr[R2 * n1 + n2]; ai[n1] = xi[R2 * n1 + n2]; }
        dft_small<T, R1>(ar, ai);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            const int m = n2 * k1 * (20 / R);
            if (m) {
                const T c = cos18<T>(m), s = sin18<T>(m);   // times c - i s
                const T r = ar[k1] * c + ai[k1] * s;
                ai[k1] = ai[k1] * c - ar[k1] * s;
                ar[k1] = r;
            }
            xr[R2 * k1 + n2] = ar[k1];
            xi[R2 * k1 + n2] = ai[k1];
        }
    }
    T yr[R], yi[R];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        T br[R2], bi[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) { br[n2] = xr[R2 * k1 + n2]; bi[n2] = xi[R2 * k1 + n2]; }
        dft_small<T, R2>(br, bi);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) { yr[k1 + R1 * k2] = br[k2]; yi[k1 + R1 * k2] = bi[k2]; }
    }
#pragma unroll
    for (int p = 0; p < R; ++p) { xr[p] = yr[p]; xi[p] = yi[p]; }
}

template <typename T, int R>
__device__ __forceinline__ void dft_small(T *xr, T *xi)
{
    if constexpr (R == 2) {
        const T ar = xr[0], ai = xi[0];
        xr[0] = ar + xr[1]; xi[0] = ai + xi[1];
        xr[1] = ar - xr[1]; xi[1] = ai - xi[1];
    } else if constexpr (R == 4) {
        const T s0r = xr[0] + xr[2], s0i = xi[0] + xi[2], d0r = xr[0] - xr[2], d0i = xi[0] - xi[2];
        const T s1r = xr[1] + xr[3], s1i = xi[1] + xi[3], d1r = xr[1] - xr[3], d1i = xi[1] - xi[3];
        xr[0] = s0r + s1r; xi[0] = s0i + s1i;
        xr[2] = s0r - s1r; xi[2] = s0i - s1i;
        xr[1] = d0r + d1i; xi[1] = d0i - d1r;   // d0 - i d1
        xr[3] = d0r - d1i; xi[3] = d0i + d1r;   // d0 + i d1
    } else if constexpr (R == 5) {
        const T c1 = (T)0.30901699437494742410229341718281906, c2 = (T)-0.80901699437494742410229341718281906;
        const T s1 = (T)0.95105651629515357211643933337938214, s2 = (T)0.58778525229247312916870595463907277;
        const T t1r = xr[1] + xr[4], t1i = xi[1] + xi[4], t3r = xr[1] - xr[4], t3i = xi[1] - xi[4];
        const T t2r = xr[2] + xr[3], t2i = xi[2] + xi[3], t4r = xr[2] - xr[3], t4i = xi[2] - xi[3];
        const T a1r = xr[0] + c1 * t1r + c2 * t2r, a1i = xi[0] + c1 * t1i + c2 * t2i;
        const T a2r = xr[0] + c2 * t1r + c1 * t2r, a2i = xi[0] + c2 * t1i + c1 * t2i;
        const T b1r = s1 * t3r + s2 * t4r, b1i = s1 * t3i + s2 * t4i;
        const T b2r = s2 * t3r - s1 * t4r, b2i = s2 * t3i - s1 * t4i;
        xr[0] = xr[0] + t1r + t2r; xi[0] = xi[0] + t1i + t2i;
        xr[1] = a1r + b1i; xi[1] = a1i - b1r;   // a1 - i b1
        xr[4] = a1r - b1i; xi[4] = a1i + b1r;   // a1 + i b1
        xr[2] = a2r + b2i; xi[2] = a2i - b2r;   // a2 - i b2
        xr[3] = a2r - b2i; xi[3] = a2i + b2r;   // a2 + i b2
    } else if constexpr (R == 10) {
        dft_composite<T, 2, 5>(xr, xi);
    } else {
        static_assert(R == 20, "radix 2, 4, 5, 10 or 20");
        dft_composite<T, 4, 5>(xr, xi);
    }
}

// One Stockham pass of radix R on sub-length L: butterfly j = tid + Tn c
// (c < E/R) takes the inputs j + m P/R, twiddles them by W_{LR}^{k m} (k = j mod L)
// and leaves the outputs for positions (j / L) L R + k + p L.
template <typename T, int P, int R, int L>
__device__ __forceinline__ void rader_pass(T (&xr)[kRaderE], T (&xi)[kRaderE], int tid,
                                           const typename cvec<T>::type *__restrict__ tw)
{
    using V = typename cvec<T>::type;
    constexpr int E = kRaderE, Tn = P / E, step = P / (L * R);
#pragma unroll
    for (int c = 0; c < E / R; ++c) {
        if constexpr (L > 1) {   // the first pass has no twiddles
            // W^m by products with W^1, restarted from the table at m = 5, 10, 15
            const int k = (tid + Tn * c) % L;
            const V w1 = tw[k * step];
            T wr = w1.x, wi = w1.y;
#pragma unroll
            for (int m = 1; m < R; ++m) {
                if (m % 5 == 0) {
                    const V wm = tw[k * step * m];
                    wr = wm.x;
                    wi = wm.y;
                } else if (m > 1) {
                    const T nr = wr * w1.x - wi * w1.y;
                    wi = wr * w1.y + wi * w1.x;
                    wr = nr;
                }
                const T ar = xr[c * R + m], ai = xi[c * R + m];
                xr[c * R + m] = ar * wr - ai * wi;
                xi[c * R + m] = ar * wi + ai * wr;
            }
        }
        dft_small<T, R>(xr + c * R, xi + c * R);
    }
}

// Output position of value (c, p) of a pass of radix R with sub-length L.
template <int P, int R, int L>
__device__ __forceinline__ int out_pos(int tid, int c, int p)
{
    const int j = tid + (P / kRaderE) * c;
    return (j / L) * L * R + (j % L) + p * L;
}

template <typename T, int P, int R, int L>
__device__ __forceinline__ void put_plane(T *pl, const T (&x)[kRaderE], int tid)
{
#pragma unroll
    for (int c = 0; c < kRaderE / R; ++c)
#pragma unroll
        for (int p = 0; p < R; ++p) pl[out_pos<P, R, L>(tid, c, p)] = x[c * R + p];
}

template <typename T, int P, int R>
__device__ __forceinline__ void get_plane(const T *pl, T (&x)[kRaderE], int tid)
{
#pragma unroll
    for (int c = 0; c < kRaderE / R; ++c)
#pragma unroll
        for (int m = 0; m < R; ++m) x[c * R + m] = pl[tid + (P / kRaderE) * c + m * (P / R)];
}

// Values leave the layout of a pass (radix RO, sub-length LO) for the input layout
// of a pass of radix RI, through the LDS plane, real and imaginary parts in turn.
// Inactive threads (tid >= Tn) take part in the barriers only.
template <typename T, int P, int RO, int LO, int RI>
__device__ __forceinline__ void exchange(T *pl, T (&xr)[kRaderE], T (&xi)[kRaderE], bool act, int tid)
{
    // each access gets its own opaque copy of tid, so the addresses are recomputed
    // instead of being held across the barriers
    if (act) put_plane<T, P, RO, LO>(pl, xr, rader_opaque(tid));
    __syncthreads();
    if (act) get_plane<T, P, RI>(pl, xr, rader_opaque(tid));
    __syncthreads();
    if (act) put_plane<T, P, RO, LO>(pl, xi, rader_opaque(tid));
    __syncthreads();
    if (act) get_plane<T, P, RI>(pl, xi, rader_opaque(tid));
    __syncthreads();
}

// Passes I, I + 1, ... of a length-P DFT (forward sign), the values in the input
// layout of pass I; the outputs end in the layout of the last pass.
template <typename T, int P, int I>
__device__ __forceinline__ void dft_passes(T *pl, T (&xr)[kRaderE], T (&xi)[kRaderE], bool act, int t, int tid,
                                           const typename cvec<T>::type *__restrict__ tw)
{
    using S = RShape<P>;
    if constexpr (I < S::NP) {
        if constexpr (I > 0) exchange<T, P, S::radix(I - 1), S::sub(I - 1), S::radix(I)>(pl, xr, xi, act, tid);
        if (act) rader_pass<T, P, S::radix(I), S::sub(I)>(xr, xi, rader_opaque(t), tw);
        dft_passes<T, P, I + 1>(pl, xr, xi, act, t, tid, tw);
    }
}

// mode: FFT_FWD (ghat = (1/M) sum f w^{-jh} times scale, and the non-zero bitmap) or
// FFT_INV (scale (1/M) sum g w^{+jh}, times M when scale_by_m).
template <typename T, int P>
__global__ __launch_bounds__(RShape<P>::threads) void k_rader(
    const int32_t *__restrict__ lats, const LatDesc *__restrict__ lat, const RaderDesc *__restrict__ rdesc,
    const int32_t *__restrict__ itab, const typename cvec<T>::type *__restrict__ ctab,
    const typename cvec<T>::type *__restrict__ in, typename cvec<T>::type *__restrict__ out,
    uint32_t *__restrict__ bitmap, T th2, int mode, T scale, int scale_by_m)
{
    using V = typename cvec<T>::type;
    using S = RShape<P>;
    constexpr int E = kRaderE, Tn = S::Tn, NT = S::threads, Ll = S::Llast, RL = S::RL;
    extern __shared__ __align__(16) unsigned char smem[];
    T *pl = reinterpret_cast<T *>(smem);
    __shared__ double red[2 * (NT / 64)];
    const LatDesc ld = lat[lats[blockIdx.x]];
    const RaderDesc *rd = rdesc + ld.mid;
    const int M = P + 1;
    const int tid = threadIdx.x;
    const bool act = tid < Tn;
    const int t = act ? tid : 0;   // inactive threads mirror thread 0 (in range), results unused
    const int32_t *pin = itab + rd->perm_in;
    const int32_t *pout = itab + rd->perm_out;
    const V *tw = ctab + rd->tw;
    const V *sp = ctab + rd->spec;
    const T cj = (mode == FFT_INV) ? T(-1) : T(1);
    const V *x = in + ld.node_off;
    T xr[E], xi[E];

    // a[q] = f[g^q]: f[1..M) through the plane in natural order, gathered in the
    // input order of the first pass
    for (int i = tid; i < P; i += NT) pl[i] = x[1 + i].x;
    __syncthreads();
    int gidx[E];
    // first-pass input index of register e = R0 c + m: q = t + Tn c + m P / R0
#pragma unroll
    for (int e = 0; e < E; ++e) gidx[e] = pin[t + Tn * (e / S::R0) + (e % S::R0) * (P / S::R0)] - 1;
#pragma unroll
    for (int e = 0; e < E; ++e) xr[e] = pl[gidx[e]];
    __syncthreads();
    for (int i = tid; i < P; i += NT) pl[i] = cj * x[1 + i].y;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xi[e] = pl[gidx[e]];
    __syncthreads();

    // ghat[0]: the sum of f
    V f0 = x[0];
    f0.y *= cj;
    {
        double sr = 0.0, si = 0.0;
        if (act)
#pragma unroll
            for (int e = 0; e < E; ++e) { sr += xr[e]; si += xi[e]; }
        for (int o = 32; o > 0; o >>= 1) {
            sr += __shfl_xor(sr, o);
            si += __shfl_xor(si, o);
        }
        if ((tid & 63) == 0) { red[2 * (tid >> 6)] = sr; red[2 * (tid >> 6) + 1] = si; }
    }

    // forward length-P DFT of a
    dft_passes<T, P, 0>(pl, xr, xi, act, t, tid, tw);
    // times the spectrum of b (with 1/P), conjugated for the inverse DFT
    if (act) {
        const int tt = rader_opaque(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const V s = sp[out_pos<P, RL, Ll>(tt, e / RL, e % RL)];
            const T ar = xr[e], ai = xi[e];
            xr[e] = ar * s.x - ai * s.y;
            xi[e] = -(ar * s.y + ai * s.x);
        }
    }
    // inverse length-P DFT (conjugated input): the convolution, conjugated
    exchange<T, P, RL, Ll, S::R0>(pl, xr, xi, act, tid);
    dft_passes<T, P, 0>(pl, xr, xi, act, t, tid, tw);
    // ghat[g^-p] = (f[0] + conv[p]) / M at natural index g^-p - 1 of the plane; the
    // real parts go out first (8-byte stores), then the imaginary parts
    const T sc = (scale_by_m ? scale * (T)M : scale) / (T)M;
    {
        const int tt = rader_opaque(t);
#pragma unroll
        for (int e = 0; e < E; ++e) gidx[e] = pout[out_pos<P, RL, Ll>(tt, e / RL, e % RL)] - 1;
    }
    V *y = out + ld.node_off;
    T *yr = reinterpret_cast<T *>(y);
    if (act)
#pragma unroll
        for (int e = 0; e < E; ++e) pl[gidx[e]] = (f0.x + xr[e]) * sc;
    __syncthreads();
    for (int i = tid; i < P; i += NT) yr[2 * (1 + i)] = pl[i];
    __syncthreads();
    if (act)
#pragma unroll
        for (int e = 0; e < E; ++e) pl[gidx[e]] = cj * (f0.y - xi[e]) * sc;   // undo the conjugation
    __syncthreads();
    for (int i = tid; i < P; i += NT) {
        const T gi = pl[i];
        yr[2 * (1 + i) + 1] = gi;
        if (mode == FFT_FWD && bitmap) {
            const T gr = yr[2 * (1 + i)];   // written by this thread above
            bitmap_set_run(bitmap, ld.node_off + 1 + i, gr * gr + gi * gi >= th2);
        }
    }
    if (tid == 0) {
        double sr = 0.0, si = 0.0;
        for (int w = 0; w < NT / 64; ++w) { sr += red[2 * w]; si += red[2 * w + 1]; }
        V o;
        o.x = (T)(((double)f0.x + sr) * (double)sc);
        o.y = (T)(cj * ((double)f0.y + si) * (double)sc);
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
    rd.nthreads = (int32_t)(P / kRaderE);
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
                                 P * (int)sizeof(T)));
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
    hipLaunchKernelGGL((k_rader<T, P>), dim3((unsigned)nl), dim3(RShape<P>::threads), (size_t)P * sizeof(T),
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
