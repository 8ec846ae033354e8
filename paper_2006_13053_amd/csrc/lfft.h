// Register-resident batched FFT engine for the lattice DFTs (Algorithm 2, first
// loop, "using a 1d FFT").
//
// A length-N transform (N a compile-time constant) is held by NT = N / E threads, E
// values each, in registers.  It runs as Stockham passes whose radices divide E; in
// the pass of radix R on sub-length L (L = product of the earlier radices), thread t
// does E / R butterflies j = t + NT c: inputs x[j + m N / R] (m < R) times the
// twiddles W_{LR}^{k m} (k = j mod L), a length-R DFT, outputs at
// (j / L) L R + k + p L (p < R).  Between passes the values move through the
// workgroup's LDS into the next pass's input layout: both components at once when
// the workgroup's LDS budget holds them, else the real and the imaginary parts in
// turn.  The first pass reads its inputs, and the last pass leaves its outputs, in
// rows t + NT c + m N / R of consecutive threads, so the loads and stores of a
// transform are coalesced without a permutation.
//
// Several transforms of one length can share a workgroup (G groups of NT threads;
// every group follows the same barriers).
#pragma once

#include "mr1l_internal.h"

namespace mr1l {
namespace lf {

// cos(2 pi k / 160), k = 0..40 (80-bit evaluation rounded to double).  Every radix
// used here divides 160, so all butterfly constants come from this quadrant.
__host__ __device__ constexpr double cos160(int k)
{
    constexpr double t[41] = {
        1.00000000000000000000e+00, 9.99229036240722934736e-01, 9.96917333733127976206e-01,
        9.93068456954926295657e-01, 9.87688340595137726169e-01, 9.80785280403230449119e-01,
        9.72369920397676601822e-01, 9.62455236453647287648e-01, 9.51056516295153572111e-01,
        9.38191335922484134443e-01, 9.23879532511286756101e-01, 9.08143173825081299238e-01,
        8.91006524188367862380e-01, 8.72496007072797114543e-01, 8.52640164354092221514e-01,
        8.31469612302545237081e-01, 8.09016994374947424104e-01, 7.85316930880744927469e-01,
        7.60405965600030938169e-01, 7.34322509435685535613e-01, 7.07106781186547524382e-01,
        6.78800745532941741381e-01, 6.49448048330183655755e-01, 6.19093949309833986919e-01,
        5.87785252292473129135e-01, 5.55570233019602224757e-01, 5.22498564715948865002e-01,
        4.88621241496954947345e-01, 4.53990499739546791606e-01, 4.18659737537428086628e-01,
        3.82683432365089771696e-01, 3.46117057077492976439e-01, 3.09016994374947424076e-01,
        2.71440449865074253348e-01, 2.33445363855905411768e-01, 1.95090322016128267870e-01,
        1.56434465040230868933e-01, 1.17537397457837644147e-01, 7.84590957278449449780e-02,
        3.92598157590686130645e-02, 0.0};
    k %= 160;
    if (k < 0) k += 160;
    return k <= 40 ? t[k] : k <= 80 ? -t[80 - k] : k <= 120 ? -t[k - 80] : t[160 - k];
}
__host__ __device__ constexpr double sin160(int k) { return cos160(k - 40); }

// (xr + i xi) times e^{-2 pi i k / 160}; exact for multiples of 90 degrees, two
// multiplications for odd multiples of 45 degrees.
template <typename T>
__device__ __forceinline__ void rot(T &xr, T &xi, int k)
{
    k %= 160;
    if (k < 0) k += 160;
    if (k == 0) return;
    if (k == 40) { const T t = xr; xr = xi; xi = -t; return; }
    if (k == 80) { xr = -xr; xi = -xi; return; }
    if (k == 120) { const T t = xr; xr = -xi; xi = t; return; }
    constexpr T h = T(0.70710678118654752440084436210485);
    if (k == 20) { const T r = (xr + xi) * h; xi = (xi - xr) * h; xr = r; return; }
    if (k == 60) { const T r = (xi - xr) * h; xi = -(xr + xi) * h; xr = r; return; }
    if (k == 100) { const T r = -(xr + xi) * h; xi = (xr - xi) * h; xr = r; return; }
    if (k == 140) { const T r = (xr - xi) * h; xi = (xr + xi) * h; xr = r; return; }
    const T c = (T)cos160(k), s = (T)sin160(k);
    const T r = xr * c + xi * s;
    xi = xi * c - xr * s;
    xr = r;
}

// ------------------------------------------------------------------ butterflies
// Forward DFT of length R in place: X[k] = sum_n x[n] e^{-2 pi i n k / R}.
template <typename T, int R> __device__ __forceinline__ void dft(T *xr, T *xi);

// Length R = R1 R2 by n = R2 n1 + n2, k = k1 + R1 k2: R2 DFTs of length R1 over n1,
// twiddles W_R^{n2 k1}, R1 DFTs of length R2 over n2.
template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_comp(T *xr, T *xi)
{
    constexpr int R = R1 * R2;
    T ar[R], ai[R];   // [n2][k1]
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        T br[R1], bi[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) { br[n1] = xr[R2 * n1 + n2]; bi[n1] = xi[R2 * n1 + n2]; }
        dft<T, R1>(br, bi);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            rot(br[k1], bi[k1], n2 * k1 * (160 / R));
            ar[n2 * R1 + k1] = br[k1];
            ai[n2 * R1 + k1] = bi[k1];
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        T cr[R2], ci[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) { cr[n2] = ar[n2 * R1 + k1]; ci[n2] = ai[n2 * R1 + k1]; }
        dft<T, R2>(cr, ci);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) { xr[k1 + R1 * k2] = cr[k2]; xi[k1 + R1 * k2] = ci[k2]; }
    }
}

template <typename T, int R>
__device__ __forceinline__ void dft(T *xr, T *xi)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
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
        const T c1 = (T)cos160(32), c2 = (T)cos160(64), s1 = (T)sin160(32), s2 = (T)sin160(64);
        const T t1r = xr[1] + xr[4], t1i = xi[1] + xi[4], t3r = xr[1] - xr[4], t3i = xi[1] - xi[4];
        const T t2r = xr[2] + xr[3], t2i = xi[2] + xi[3], t4r = xr[2] - xr[3], t4i = xi[2] - xi[3];
        const T a1r = xr[0] + c1 * t1r + c2 * t2r, a1i = xi[0] + c1 * t1i + c2 * t2i;
        const T a2r = xr[0] + c2 * t1r + c1 * t2r, a2i = xi[0] + c2 * t1i + c1 * t2i;
        const T b1r = s1 * t3r + s2 * t4r, b1i = s1 * t3i + s2 * t4i;
        const T b2r = s2 * t3r - s1 * t4r, b2i = s2 * t3i - s1 * t4i;
        xr[0] = xr[0] + t1r + t2r; xi[0] = xi[0] + t1i + t2i;
        xr[1] = a1r + b1i; xi[1] = a1i - b1r;   // a1 - i b1
        xr[4] = a1r - b1i; xi[4] = a1i + b1r;
        xr[2] = a2r + b2i; xi[2] = a2i - b2r;   // a2 - i b2
        xr[3] = a2r - b2i; xi[3] = a2i + b2r;
    } else if constexpr (R == 8) {
        dft_comp<T, 4, 2>(xr, xi);
    } else if constexpr (R == 10) {
        dft_comp<T, 2, 5>(xr, xi);
    } else if constexpr (R == 16) {
        dft_comp<T, 4, 4>(xr, xi);
    } else if constexpr (R == 20) {
        dft_comp<T, 4, 5>(xr, xi);
    } else if constexpr (R == 32) {
        dft_comp<T, 8, 4>(xr, xi);
    } else {
        static_assert(R == 40, "radix 2, 4, 5, 8, 10, 16, 20, 32 or 40");
        dft_comp<T, 8, 5>(xr, xi);
    }
}

// ------------------------------------------------------------------ shape
// The pass plan of a length-N transform with E values per thread: greedy, the
// largest radix that divides both E and what is left of N.
template <int N, int E> struct Shape {
    static constexpr int NT = N / E;
    static constexpr int pick(int q)
    {
        constexpr int cand[] = {40, 32, 20, 16, 10, 8, 5, 4, 2};
        for (int r : cand)
            if (E % r == 0 && q % r == 0) return r;
        return 0;
    }
    static constexpr int count()
    {
        int n = 0;
        for (int q = N; q > 1; q /= pick(q)) {
            if (pick(q) == 0) return -1;
            ++n;
        }
        return n;
    }
    static constexpr int NP = count();
    static constexpr int radix(int i)
    {
        int q = N;
        for (int k = 0; k < i; ++k) q /= pick(q);
        return pick(q);
    }
    static constexpr int sub(int i)   // sub-length before pass i
    {
        int L = 1;
        for (int k = 0; k < i; ++k) L *= radix(k);
        return L;
    }
    static constexpr int R0 = radix(0), RL = radix(NP - 1), LL = sub(NP - 1);
    static_assert(NP > 0 && N % E == 0, "N must factor into radices that divide E");
    static_assert(sub(NP) == N, "radix plan");
};

// Hides a value from the optimiser so that index arithmetic is recomputed where it
// is used instead of being held in registers across the passes.
__device__ __forceinline__ int opq(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Twiddles of a pass of radix R on sub-length L: butterfly c of thread t needs
// W_{LR}^{k m} = e^{-2 pi i k m step / N} (table entry k m step, step = N / (L R),
// k = j mod L, m < R).  Two table entries per butterfly, b = W^k and q = W^{4k}, are loaded ahead
// (before the exchange that precedes the pass, so that their latency overlaps it);
// W^{k m} = q^a b^r for m = 4a + r is formed with a few complex multiplications
// (error a few units of roundoff).
template <typename T, int N, int E, int R, int L> struct Tw {
    using V = typename cvec<T>::type;
    V b[E / R], q[(R > 4) ? E / R : 1];
};

template <typename T, int N, int E, int R, int L>
__device__ __forceinline__ void tw_load(Tw<T, N, E, R, L> &w, int t, const typename cvec<T>::type *__restrict__ tw)
{
    constexpr int NT = N / E, step = N / (L * R);
    if constexpr (L > 1) {
#pragma unroll
        for (int c = 0; c < E / R; ++c) {
            const int k = (t + NT * c) % L;
            w.b[c] = tw[k * step];
            if constexpr (R > 4) w.q[c] = tw[4 * k * step];
        }
    }
}

template <typename T>
__device__ __forceinline__ typename cvec<T>::type cmul(const typename cvec<T>::type &a, const typename cvec<T>::type &b)
{
    typename cvec<T>::type o;
    o.x = a.x * b.x - a.y * b.y;
    o.y = a.x * b.y + a.y * b.x;
    return o;
}

// One pass of radix R on sub-length L: twiddles (none in the first pass, L = 1),
// then the butterflies.
template <typename T, int N, int E, int R, int L>
__device__ __forceinline__ void pass(T (&xr)[E], T (&xi)[E], const Tw<T, N, E, R, L> &w)
{
    using V = typename cvec<T>::type;
#pragma unroll
    for (int c = 0; c < E / R; ++c) {
        if constexpr (L > 1) {
            V br[4];   // b^0 .. b^3
            br[1] = w.b[c];
            br[2] = cmul<T>(br[1], br[1]);
            br[3] = cmul<T>(br[2], br[1]);
            V qa = w.b[c];   // q^a, set for a >= 1
#pragma unroll
            for (int a = 0; a < (R + 3) / 4; ++a) {
                if constexpr (R > 4) {
                    if (a == 1) qa = w.q[c];
                    else if (a > 1) qa = cmul<T>(qa, w.q[c]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 4 * a + r;
                    if (m == 0 || m >= R) continue;
                    const V tw = a == 0 ? br[r] : (r == 0 ? qa : cmul<T>(qa, br[r]));
                    const T ar = xr[c * R + m], ai = xi[c * R + m];
                    xr[c * R + m] = ar * tw.x - ai * tw.y;
                    xi[c * R + m] = ar * tw.y + ai * tw.x;
                }
            }
        }
        dft<T, R>(xr + c * R, xi + c * R);
    }
}

// Position of output p of butterfly c of thread t after a pass of radix R on
// sub-length L.
template <int N, int E, int R, int L>
__device__ __forceinline__ int out_pos(int t, int c, int p)
{
    const int j = t + (N / E) * c;
    return (j / L) * L * R + (j % L) + p * L;
}

// Input position of value (c, m) of thread t for a pass of radix R.
template <int N, int E, int R>
__device__ __forceinline__ int in_pos(int t, int c, int m)
{
    return t + (N / E) * c + m * (N / R);
}

// LDS index of plane entry q: one pad entry after every 16 doubles (32 floats), so
// that the first pass's outputs (stride E entries across the lanes) fall in distinct
// banks; runs of 16 or more consecutive lanes stay conflict-free.  E = 40 (the Rader
// transform of length 16000) takes one pad entry per 8 entries: its first pass's
// stride-40 stores, unpadded, put a half-wave's doubles in two bank pairs (a 16-way
// conflict), and with period 8 the base 40 t of those stores stays a multiple of the
// period, so every offset is an immediate (period 16 gave 5% more time).  With E = 20
// (the other radix-20 transforms) the plane is left unpadded.
template <typename T, int E = 16> constexpr int pad_shift() { return E % 8 ? 30 : E % 16 ? 3 : (sizeof(T) == 8 ? 4 : 5); }
template <typename T, int E = 16> __device__ __forceinline__ int padq(int q) { return q + (q >> pad_shift<T, E>()); }
// Entries of one padded plane of length N.
template <typename T, int E = 16> constexpr int plane_len(int N) { return N + (N >> pad_shift<T, E>()); }

// Plane stores of a pass's outputs and loads of the next pass's inputs.  Every index
// is base(t) + K with K a constant of the unrolled loops (t + NT c splits this way
// because NT and the sub-length are powers of two, one dividing the other); where K
// is a multiple of the pad period the padded index is padq(base) + K + the pad of K,
// so the address is one register plus an immediate offset.
// BAL: base is a multiple of the pad period, so every K gives an immediate offset.
template <typename T, int E, bool BAL = false>
__device__ __forceinline__ int padded(int base, int pbase, int K)
{
    constexpr int sh = pad_shift<T, E>();
    return (sh >= 30 || BAL || K % (1 << sh) == 0) ? pbase + K + (K >> sh) : padq<T, E>(base + K);
}

template <typename T, int N, int E, int RO, int LO>
__device__ __forceinline__ void put_plane(T *pl, const T (&x)[E], int t)
{
    constexpr int NT = N / E;
    constexpr bool A = NT % LO == 0, B = LO % NT == 0;
    constexpr int sh = pad_shift<T, E>();
    // first pass (LO = 1): base = t RO, a multiple of the pad period when RO is
    constexpr bool BAL = A && LO == 1 && sh < 30 && RO % (1 << (sh < 30 ? sh : 0)) == 0;
    const int base = A ? (t / LO) * LO * RO + (t % LO) : t;
    const int pb = padq<T, E>(base);
#pragma unroll
    for (int c = 0; c < E / RO; ++c)
#pragma unroll
        for (int p = 0; p < RO; ++p) {
            if constexpr (A || B) {
                const int qc = (NT * c) / LO, rc = (NT * c) % LO;   // B: NT c = qc LO + rc, rc + t < LO
                const int K = A ? NT * c * RO + p * LO : qc * LO * RO + rc + p * LO;
                pl[padded<T, E, BAL>(base, pb, K)] = x[c * RO + p];
            } else {
                pl[padq<T, E>(out_pos<N, E, RO, LO>(t, c, p))] = x[c * RO + p];
            }
        }
}

template <typename T, int N, int E, int RI>
__device__ __forceinline__ void get_plane(const T *pl, T (&x)[E], int t)
{
    const int pb = padq<T, E>(t);
#pragma unroll
    for (int c = 0; c < E / RI; ++c)
#pragma unroll
        for (int m = 0; m < RI; ++m) x[c * RI + m] = pl[padded<T, E>(t, pb, (N / E) * c + m * (N / RI))];
}

// Values leave the layout of a pass (radix RO, sub-length LO) for the input layout of
// a pass of radix RI through the LDS: planes re and im (im == re: one plane, the two
// components in turn).  Threads that hold no transform (act false) take part in the
// barriers only.
template <typename T, int N, int E, int RO, int LO, int RI>
__device__ __forceinline__ void exchange(T *re, T *im, T (&xr)[E], T (&xi)[E], bool act, int t)
{
    if (re != im) {
        if (act) {
            put_plane<T, N, E, RO, LO>(re, xr, opq(t));
            put_plane<T, N, E, RO, LO>(im, xi, opq(t));
        }
        __syncthreads();
        if (act) {
            get_plane<T, N, E, RI>(re, xr, opq(t));
            get_plane<T, N, E, RI>(im, xi, opq(t));
        }
        __syncthreads();
        return;
    }
    if (act) put_plane<T, N, E, RO, LO>(re, xr, opq(t));
    __syncthreads();
    if (act) get_plane<T, N, E, RI>(re, xr, opq(t));
    __syncthreads();
    if (act) put_plane<T, N, E, RO, LO>(re, xi, opq(t));
    __syncthreads();
    if (act) get_plane<T, N, E, RI>(re, xi, opq(t));
    __syncthreads();
}

// Passes I, I + 1, ... of a forward length-N transform, the values in the input
// layout of pass I; they end in the output layout of the last pass.
template <typename T, int N, int E, int I>
__device__ __forceinline__ void passes(T *re, T *im, T (&xr)[E], T (&xi)[E], bool act, int t,
                                       const typename cvec<T>::type *__restrict__ tw)
{
    using S = Shape<N, E>;
    if constexpr (I < S::NP) {
        constexpr int R = S::radix(I), L = S::sub(I);
        Tw<T, N, E, R, L> w;
        if (act) tw_load<T, N, E, R, L>(w, opq(t), tw);
        if constexpr (I > 0) exchange<T, N, E, S::radix(I - 1), S::sub(I - 1), R>(re, im, xr, xi, act, t);
        if (act) pass<T, N, E, R, L>(xr, xi, w);
        passes<T, N, E, I + 1>(re, im, xr, xi, act, t, tw);
    }
}

// Forward transform of values in the first pass's input layout; the result is in
// the last pass's output layout, X[h] at h = t + NT c + p N / RL for value c RL + p.
template <typename T, int N, int E>
__device__ __forceinline__ void fft(T *re, T *im, T (&xr)[E], T (&xi)[E], bool act, int t,
                                    const typename cvec<T>::type *__restrict__ tw)
{
    passes<T, N, E, 0>(re, im, xr, xi, act, t, tw);
}

// From the last pass's output layout back to the first pass's input layout.
template <typename T, int N, int E>
__device__ __forceinline__ void relayout(T *re, T *im, T (&xr)[E], T (&xi)[E], bool act, int t)
{
    using S = Shape<N, E>;
    exchange<T, N, E, S::RL, S::LL, S::R0>(re, im, xr, xi, act, t);
}

}  // namespace lf
}  // namespace mr1l
