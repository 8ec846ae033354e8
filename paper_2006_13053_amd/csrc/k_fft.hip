// Normalised lattice DFTs (Algorithm 2, first loop) for prime lattice sizes.
//
//   ghat[h] = (1/M) sum_{j<M} f[j] e^{-2 pi i j h / M},  h < M.
//
// M is prime, so the transform is Bluestein's chirp convolution: with
// w[n] = e^{-pi i n^2 / M},
//   ghat[h] = w[h] / M * sum_j (f[j] w[j]) conj(w[h - j]),
// a cyclic convolution of length N >= 2M - 1 (N 5-smooth) evaluated with two
// length-N FFTs and the precomputed spectrum of conj(w) (the 1/(N M)
// normalisation is folded into that spectrum).  The inverse map
// (1/M) sum_h g[h] e^{+2 pi i j h / M} is the conjugate of the forward map of
// the conjugate input.
//
// Length-N FFTs are Stockham autosort passes (radix 8, 4, 2, 5, 3) on re/im
// planes held in the workgroup's LDS; every pass reads its butterflies into
// registers, synchronises, and writes in place.  One workgroup handles one
// lattice.  When N does not fit the LDS (N > 10240 for complex128) the
// transform is split as N = N1 * N2 (four-step): N2 columns of length N1,
// twiddle, N1 rows of length N2, with the intermediate in a per-workgroup
// global scratch slot (it stays in L2/MALL) and the chirp and spectrum
// products fused into the column load and the row store.
#include <algorithm>
#include <cstring>
#include <cmath>
#include <initializer_list>
#include <map>

#include "mr1l_internal.h"

namespace mr1l {

// The thread index laundered through an empty asm: index arithmetic derived from
// it cannot be hoisted out of the batch loops, where it would stay live through
// every Stockham pass and spill.
__device__ __forceinline__ int opaque(int x) { asm volatile("" : "+v"(x)); return x; }

// ------------------------------------------------------------------ radix DFTs
template <typename T>
__device__ __forceinline__ void dft2(T *xr, T *xi)
{
    T ar = xr[0], ai = xi[0];
    xr[0] = ar + xr[1]; xi[0] = ai + xi[1];
    xr[1] = ar - xr[1]; xi[1] = ai - xi[1];
}

template <typename T>
__device__ __forceinline__ void dft3(T *xr, T *xi)
{
    const T c = T(-0.5);
    const T s = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    T sr = xr[1] + xr[2], si = xi[1] + xi[2];
    T dr = xr[1] - xr[2], di = xi[1] - xi[2];
    T br = xr[0] + c * sr, bi = xi[0] + c * si;
    xr[0] = xr[0] + sr; xi[0] = xi[0] + si;
    // forward: y1 = b - i s d, y2 = b + i s d
    xr[1] = br + s * di; xi[1] = bi - s * dr;
    xr[2] = br - s * di; xi[2] = bi + s * dr;
}

template <typename T>
__device__ __forceinline__ void dft4(T *xr, T *xi)
{
    T t0r = xr[0] + xr[2], t0i = xi[0] + xi[2];
    T t1r = xr[0] - xr[2], t1i = xi[0] - xi[2];
    T t2r = xr[1] + xr[3], t2i = xi[1] + xi[3];
    T t3r = xr[1] - xr[3], t3i = xi[1] - xi[3];
    xr[0] = t0r + t2r; xi[0] = t0i + t2i;
    xr[2] = t0r - t2r; xi[2] = t0i - t2i;
    // y1 = t1 - i t3, y3 = t1 + i t3
    xr[1] = t1r + t3i; xi[1] = t1i - t3r;
    xr[3] = t1r - t3i; xi[3] = t1i + t3r;
}

template <typename T>
__device__ __forceinline__ void dft5(T *xr, T *xi)
{
    const T c1 = T(0.30901699437494742410229341718282);   // cos(2 pi / 5)
    const T c2 = T(-0.80901699437494742410229341718282);  // cos(4 pi / 5)
    const T s1 = T(0.95105651629515357211643933337938);   // sin(2 pi / 5)
    const T s2 = T(0.58778525229247312916870595463907);   // sin(4 pi / 5)
    T t1r = xr[1] + xr[4], t1i = xi[1] + xi[4];
    T t2r = xr[2] + xr[3], t2i = xi[2] + xi[3];
    T t3r = xr[1] - xr[4], t3i = xi[1] - xi[4];
    T t4r = xr[2] - xr[3], t4i = xi[2] - xi[3];
    T b1r = xr[0] + c1 * t1r + c2 * t2r, b1i = xi[0] + c1 * t1i + c2 * t2i;
    T b2r = xr[0] + c2 * t1r + c1 * t2r, b2i = xi[0] + c2 * t1i + c1 * t2i;
    T e1r = s1 * t3r + s2 * t4r, e1i = s1 * t3i + s2 * t4i;   // y1 = b1 - i e1
    T e2r = s2 * t3r - s1 * t4r, e2i = s2 * t3i - s1 * t4i;   // y2 = b2 - i e2
    xr[0] = xr[0] + t1r + t2r; xi[0] = xi[0] + t1i + t2i;
    xr[1] = b1r + e1i; xi[1] = b1i - e1r;
    xr[4] = b1r - e1i; xi[4] = b1i + e1r;
    xr[2] = b2r + e2i; xi[2] = b2i - e2r;
    xr[3] = b2r - e2i; xi[3] = b2i + e2r;
}

template <typename T>
__device__ __forceinline__ void dft8(T *xr, T *xi)
{
    const T h = T(0.70710678118654752440084436210485);
    T er[4] = {xr[0], xr[2], xr[4], xr[6]}, ei[4] = {xi[0], xi[2], xi[4], xi[6]};
    T orr[4] = {xr[1], xr[3], xr[5], xr[7]}, oi[4] = {xi[1], xi[3], xi[5], xi[7]};
    dft4(er, ei);
    dft4(orr, oi);
    // twiddles e^{-2 pi i k / 8}: 1, (1 - i)/sqrt2, -i, (-1 - i)/sqrt2
    T w1r = h * (orr[1] + oi[1]), w1i = h * (oi[1] - orr[1]);
    T w2r = oi[2], w2i = -orr[2];
    T w3r = h * (oi[3] - orr[3]), w3i = -h * (orr[3] + oi[3]);
    xr[0] = er[0] + orr[0]; xi[0] = ei[0] + oi[0];
    xr[4] = er[0] - orr[0]; xi[4] = ei[0] - oi[0];
    xr[1] = er[1] + w1r; xi[1] = ei[1] + w1i;
    xr[5] = er[1] - w1r; xi[5] = ei[1] - w1i;
    xr[2] = er[2] + w2r; xi[2] = ei[2] + w2i;
    xr[6] = er[2] - w2r; xi[6] = ei[2] - w2i;
    xr[3] = er[3] + w3r; xi[3] = ei[3] + w3i;
    xr[7] = er[3] - w3r; xi[7] = ei[3] - w3i;
}

template <typename T, int R>
__device__ __forceinline__ void dftR(T *xr, T *xi)
{
    if constexpr (R == 2) dft2(xr, xi);
    else if constexpr (R == 3) dft3(xr, xi);
    else if constexpr (R == 4) dft4(xr, xi);
    else if constexpr (R == 5) dft5(xr, xi);
    else dft8(xr, xi);
}

__device__ __forceinline__ int next_radix(int rem)
{
    if (rem % 8 == 0) return 8;
    if (rem % 4 == 0) return 4;
    if (rem % 2 == 0) return 2;
    if (rem % 5 == 0) return 5;
    return 3;
}

// One Stockham pass of radix R over `batch` transforms of length n stored
// contiguously in the LDS planes.  Butterfly j of transform b reads
// x[b n + jj + r n/R] (jj = j mod n/R), multiplies by e^{-2 pi i r k/(Ns R)}
// (k = jj mod Ns), applies the radix-R DFT and writes
// x[b n + (jj / Ns) Ns R + k + r Ns].
// LDS index of element i of the mixed-radix planes: one pad element after every
// 32 when the planes have room for it (PAD), which spreads the strided Stockham
// writes of the early passes over the banks.
template <bool PAD> __device__ __forceinline__ int pidx(int i) { return PAD ? i + (i >> 5) : i; }
template <int NMAXT, bool PAD> constexpr int mr_plane() { return PAD ? NMAXT + NMAXT / 32 : NMAXT; }

template <typename T, int R, int NT, int NMAXT, bool PAD>
__device__ void stockham_pass(T *re, T *im, int n, int batch, int Ns,
                              const typename cvec<T>::type *__restrict__ tw)
{
    constexpr int BPT = (NMAXT / R + NT - 1) / NT;
    const int nR = n / R;
    const int total = batch * nR;
    const int tstride = n / (Ns * R);
    const int tid0 = opaque((int)threadIdx.x);
    T vr[BPT][R], vi[BPT][R];
    int ob[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int j = tid0 + i * NT;
        ob[i] = -1;
        if (j < total) {
            const int b = j / nR;
            const int jj = j - b * nR;
            const int q = jj / Ns;
            const int k = jj - q * Ns;
            const int base = b * n + jj;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                vr[i][r] = re[pidx<PAD>(base + r * nR)];
                vi[i][r] = im[pidx<PAD>(base + r * nR)];
            }
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const auto w = tw[r * k * tstride];
                    const T xr = vr[i][r], xi = vi[i][r];
                    vr[i][r] = xr * w.x - xi * w.y;
                    vi[i][r] = xr * w.y + xi * w.x;
                }
            }
            dftR<T, R>(vr[i], vi[i]);
            ob[i] = b * n + q * Ns * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        if (ob[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                re[pidx<PAD>(ob[i] + r * Ns)] = vr[i][r];
                im[pidx<PAD>(ob[i] + r * Ns)] = vi[i][r];
            }
        }
    }
    __syncthreads();
}

// Forward FFT (e^{-2 pi i}) of `batch` contiguous length-n transforms in LDS
// (batch * n <= NMAXT) by NT threads; tw = table e^{-2 pi i m / n}, m < n.
// Output in natural order.
template <typename T, int NT, int NMAXT, bool PAD>
__device__ void lds_fft(T *re, T *im, int n, int batch, const typename cvec<T>::type *tw)
{
    int Ns = 1, rem = n;
    while (rem > 1) {
        const int R = next_radix(rem);
        switch (R) {
        case 8: stockham_pass<T, 8, NT, NMAXT, PAD>(re, im, n, batch, Ns, tw); break;
        case 4: stockham_pass<T, 4, NT, NMAXT, PAD>(re, im, n, batch, Ns, tw); break;
        case 2: stockham_pass<T, 2, NT, NMAXT, PAD>(re, im, n, batch, Ns, tw); break;
        case 5: stockham_pass<T, 5, NT, NMAXT, PAD>(re, im, n, batch, Ns, tw); break;
        default: stockham_pass<T, 3, NT, NMAXT, PAD>(re, im, n, batch, Ns, tw); break;
        }
        Ns *= R;
        rem /= R;
    }
}

// ------------------------------------------------------------------ power-of-two passes
// Radix 16 as 4 x 4: X[k1 + 4 k2] = sum_{n2} W16^{n2 k1} W4^{n2 k2} sum_{n1} x[4 n1 + n2] W4^{n1 k1}.
template <typename T>
__device__ __forceinline__ void dft16(T *xr, T *xi)
{
    const T c1 = T(0.92387953251128675612818318939679);   // cos(2 pi / 16)
    const T s1 = T(0.38268343236508977172845998403040);   // sin(2 pi / 16)
    const T h = T(0.70710678118654752440084436210485);
    T ar[4][4], ai[4][4];   // [n2][k1]
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        T tr[4] = {xr[n2], xr[4 + n2], xr[8 + n2], xr[12 + n2]};
        T ti[4] = {xi[n2], xi[4 + n2], xi[8 + n2], xi[12 + n2]};
        dft4(tr, ti);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) { ar[n2][k1] = tr[k1]; ai[n2][k1] = ti[k1]; }
    }
    // twiddles W16^{n2 k1} = e^{-2 pi i m / 16}, m = n2 k1 in {0..9}
    const T wc[10] = {T(1), c1, h, s1, T(0), -s1, -h, -c1, T(-1), -c1};
    const T ws[10] = {T(0), -s1, -h, -c1, T(-1), -c1, -h, -s1, T(0), s1};
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) {
            const int m = n2 * k1;
            const T r = ar[n2][k1], i = ai[n2][k1];
            ar[n2][k1] = r * wc[m] - i * ws[m];
            ai[n2][k1] = r * ws[m] + i * wc[m];
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        T tr[4] = {ar[0][k1], ar[1][k1], ar[2][k1], ar[3][k1]};
        T ti[4] = {ai[0][k1], ai[1][k1], ai[2][k1], ai[3][k1]};
        dft4(tr, ti);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) { xr[k1 + 4 * k2] = tr[k2]; xi[k1 + 4 * k2] = ti[k2]; }
    }
}

// LDS planes of the power-of-two path hold P elements (the workgroup's LDS
// batch) of rows of length 2^logn: element i sits at i + i/32 + i/2^lr, lr =
// max(logn, 5), one pad element after every 32 and one more after every row.
// The row stride becomes odd (column accesses by consecutive lanes fall in
// distinct banks) and the strided Stockham accesses spread over the banks.
__device__ __forceinline__ int padr(int i, int lr) { return i + (i >> 5) + (i >> lr); }
constexpr int p2_plane(int P) { return P + P / 16; }

// One Stockham pass of radix 2^LR over 2^logb transforms of length 2^logn held
// in planes of P elements, by NT threads; the twiddle e^{-2 pi i r k / (Ns R)}
// is entry (r k) << (logN - logNs - LR) of a table e^{-2 pi i j / 2^logN}.
template <typename T, int LR, int NT, int P, typename TW>
__device__ void stockham_p2(T *re, T *im, int logn, int logb, int logNs, TW tw, int logN)
{
    constexpr int R = 1 << LR;
    constexpr int BPT = (P / R + NT - 1) / NT;
    const int lognR = logn - LR;
    const int total = 1 << (logb + lognR);
    const int tsh = logN - logNs - LR;
    const int lr = max(logn, 5);
    const int tid0 = opaque((int)threadIdx.x);
    T vr[BPT][R], vi[BPT][R];
    int ob[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int j = tid0 + i * NT;
        ob[i] = -1;
        if (j < total) {
            const int b = j >> lognR;
            const int jj = j & ((1 << lognR) - 1);
            const int k = jj & ((1 << logNs) - 1);
            const int q = jj >> logNs;
            const int base = (b << logn) + jj;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                vr[i][r] = re[padr(base + (r << lognR), lr)];
                vi[i][r] = im[padr(base + (r << lognR), lr)];
            }
            if (logNs > 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const auto w = tw[(r * k) << tsh];
                    const T xr = vr[i][r], xi = vi[i][r];
                    vr[i][r] = xr * w.x - xi * w.y;
                    vi[i][r] = xr * w.y + xi * w.x;
                }
            }
            if constexpr (R == 16) dft16(vr[i], vi[i]);
            else dftR<T, R>(vr[i], vi[i]);
            ob[i] = (b << logn) + (q << (logNs + LR)) + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        if (ob[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                re[padr(ob[i] + (r << logNs), lr)] = vr[i][r];
                im[padr(ob[i] + (r << logNs), lr)] = vi[i][r];
            }
        }
    }
    __syncthreads();
}

// Radix 16 for float; radix 8 at most for double (a 16-point double butterfly
// does not fit the register budget of the two-per-CU schedules).
template <typename T, int NT, int P, typename TW>
__device__ void lds_fft_p2(T *re, T *im, int logn, int logb, TW tw, int logN)
{
    int logNs = 0, rem = logn;
    while (rem > 0) {
        if (sizeof(T) == 4 && rem >= 4) { stockham_p2<T, 4, NT, P, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 4; rem -= 4; }
        else if (rem >= 3) { stockham_p2<T, 3, NT, P, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 3; rem -= 3; }
        else if (rem == 2) { stockham_p2<T, 2, NT, P, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 2; rem -= 2; }
        else { stockham_p2<T, 1, NT, P, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 1; rem -= 1; }
    }
}

// ------------------------------------------------------------------ chirps
// w[n] = e^{-pi i (n^2 mod 2M) / M} from the two-level table of e^{-pi i r / M}:
// r = hi * S + lo, table = [lo part: S entries][hi part].
template <typename T, typename TAB = const typename cvec<T>::type *>
__device__ __forceinline__ typename cvec<T>::type chirp(TAB tab, int shift, int nlo, int64_t n, int M,
                                                       double inv2m)
{
    // r = n^2 mod 2M: n < M < 2^23, so n^2 < 2^46 is exact in double and the quotient
    // from the reciprocal inv2m = 1 / (2M) is off by at most one
    const int64_t m2 = 2 * (int64_t)M;
    const int64_t sq = n * n;
    int64_t r = sq - (int64_t)floor((double)sq * inv2m) * m2;
    if (r < 0) r += m2;
    if (r >= m2) r -= m2;
    const auto a = tab[r & (int64_t)(nlo - 1)];
    const auto b = tab[nlo + (r >> shift)];
    typename cvec<T>::type o;
    o.x = a.x * b.x - a.y * b.y;
    o.y = a.x * b.y + a.y * b.x;
    return o;
}

// ------------------------------------------------------------------ LDS kernel
// One workgroup of NT threads per lattice with N <= NMAXT, the whole transform in
// the workgroup's LDS (2 NMAXT elements).  mode: FFT_FWD (f -> ghat, bitmap),
// FFT_INV (g -> (1/M) sum g e^{+}) times scale (times M when scale_by_m),
// FFT_SPEC (kernel spectrum of the lattice size, written to the spectrum table).
// Size classes (NT, NMAXT) keep small transforms from holding a whole CU's LDS.
template <typename T, int NT, int NMAXT, bool PAD>
__global__ __launch_bounds__(NT) void k_bluestein_lds(
    const int32_t *__restrict__ lats, const LatDesc *__restrict__ lat, const MDesc *__restrict__ md,
    const typename cvec<T>::type *__restrict__ in, typename cvec<T>::type *__restrict__ out,
    typename cvec<T>::type *__restrict__ spec_tab, const typename cvec<T>::type *__restrict__ chirp_tab,
    const typename cvec<T>::type *__restrict__ tw_tab, uint32_t *__restrict__ bitmap, T th2, int mode,
    T scale, int scale_by_m)
{
    using V = typename cvec<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    T *re = reinterpret_cast<T *>(smem);
    T *im = re + mr_plane<NMAXT, PAD>();
    const LatDesc ld = lat[lats[blockIdx.x]];
    const MDesc m = md[ld.mid];
    const int N = m.N, M = ld.M;
    const double inv2m = 1.0 / (2.0 * (double)M);
    const V *ctab = chirp_tab + m.chirp_off;
    const V *tw = tw_tab + m.tw_N;
    const int tid = threadIdx.x;

    if (mode == FFT_SPEC) {
        // B[n] = conj(w[n]) for n < M, B[N - n] = conj(w[n]) for 0 < n < M
        for (int i = tid; i < N; i += NT) {
            int src = -1;
            if (i < M) src = i;
            else if (i > N - M) src = N - i;
            T xr = 0, xi = 0;
            if (src >= 0) {
                V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, src, M, inv2m);
                xr = w.x; xi = -w.y;
            }
            re[pidx<PAD>(i)] = xr; im[pidx<PAD>(i)] = xi;
        }
        __syncthreads();
        lds_fft<T, NT, NMAXT, PAD>(re, im, N, 1, tw);
        const T s = T(1) / ((T)N * (T)M);
        V *dst = spec_tab + m.spec_off;
        for (int i = tid; i < N; i += NT) {
            V o; o.x = re[pidx<PAD>(i)] * s; o.y = im[pidx<PAD>(i)] * s;
            dst[i] = o;
        }
        return;
    }

    const T cj = (mode == FFT_INV) ? T(-1) : T(1);
    const V *x = in + ld.node_off;
    constexpr int EPT = (NMAXT + NT - 1) / NT;
    {
        T xr[EPT], xi[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = opaque(tid) + k * NT;
            const V v = x[i < M ? i : 0];
            const V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, i < M ? i : 0, M, inv2m);
            const T vi = cj * v.y;
            xr[k] = i < M ? v.x * w.x - vi * w.y : T(0);
            xi[k] = i < M ? v.x * w.y + vi * w.x : T(0);
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = opaque(tid) + k * NT;
            if (i < N) { re[pidx<PAD>(i)] = xr[k]; im[pidx<PAD>(i)] = xi[k]; }
        }
    }
    __syncthreads();
    lds_fft<T, NT, NMAXT, PAD>(re, im, N, 1, tw);
    const V *sp = spec_tab + m.spec_off;
    {
        V sv[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = opaque(tid) + k * NT;
            sv[k] = sp[i < N ? i : 0];
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = opaque(tid) + k * NT;
            if (i < N) {
                T a = re[pidx<PAD>(i)], b = im[pidx<PAD>(i)];
                re[pidx<PAD>(i)] = a * sv[k].x - b * sv[k].y;
                im[pidx<PAD>(i)] = -(a * sv[k].y + b * sv[k].x);   // conjugate: the next FFT is an inverse one
            }
        }
    }
    __syncthreads();
    lds_fft<T, NT, NMAXT, PAD>(re, im, N, 1, tw);
    const T sc = scale_by_m ? scale * (T)M : scale;
    V *y = out + ld.node_off;
    for (int i = tid; i < M; i += NT) {
        V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, i, M, inv2m);
        const T cr = re[pidx<PAD>(i)], ci = -im[pidx<PAD>(i)];     // undo the conjugation
        T gr = (cr * w.x - ci * w.y) * sc;
        T gi = (cr * w.y + ci * w.x) * sc;
        if (mode == FFT_INV) gi = -gi;
        V o; o.x = gr; o.y = gi;
        y[i] = o;
        if (mode == FFT_FWD && bitmap) bitmap_set_run(bitmap, ld.node_off + i, gr * gr + gi * gi >= th2);
    }
}

// ------------------------------------------------------------------ four-step kernel
// Power-of-two N = N1 N2 (N1, N2 <= P, the LDS batch), three phases per lattice
// on one slot of N complex in global scratch (it stays in L2/MALL), in place:
//   A  for a batch of columns n2: length-N1 DFTs over n1 of x[N2 n1 + n2]
//      (x = chirped input), twiddle W_N^{n2 k1}, stored Y[k1][n2];
//   B  for a batch of rows k1: length-N2 DFTs over n2 give X[k1 + N1 k2]; times
//      the kernel spectrum; inverse length-N2 DFTs over k2; twiddle W_N^{-b k1};
//      stored back over the same rows as U[k1][b] -- the forward row stage and
//      the first stage of the inverse transform share the LDS, so the product
//      never leaves the chip;
//   C  for a batch of columns b: inverse length-N1 DFTs over k1 give the
//      convolution at N2 a + b; times the chirp and 1/M (folded into the
//      spectrum); output.
// Inverse DFTs are conj(DFT(conj(.))).  SPEC mode runs A and the forward half of
// B on the chirp sequence and stores the scaled spectrum.  Loads are issued for
// every lane from a clamped, always valid index (the value is discarded where
// the element does not exist), which keeps the partially filled load arrays from
// being carried across loop iterations.  Persistent: workgroup
// w owns scratch slot w and handles lattices w, w + grid, ...  Every phase-C
// load of a lattice completes before the barrier that precedes its last DFT, so
// the next lattice's phase A may overwrite the slot.
template <typename T, bool LTAB, int NT, int LOGP, int WAVES>
__global__ __launch_bounds__(NT, WAVES) void k_bluestein_4step(
    const int32_t *__restrict__ lats, int nlats, const LatDesc *__restrict__ lat,
    const MDesc *__restrict__ md, const typename cvec<T>::type *__restrict__ in,
    typename cvec<T>::type *__restrict__ out, typename cvec<T>::type *__restrict__ spec_tab,
    const typename cvec<T>::type *__restrict__ chirp_tab, const typename cvec<T>::type *__restrict__ tw_tab,
    uint32_t *__restrict__ bitmap, T th2, int mode, T scale, int scale_by_m,
    typename cvec<T>::type *__restrict__ scratch, int64_t slot_len)
{
    using V = typename cvec<T>::type;
    constexpr int P = 1 << LOGP;
    constexpr int EPT = P / NT;     // elements per thread of a full batch
    constexpr int CH = 4;           // loads issued together per thread
    static_assert(EPT % CH == 0, "the LDS batch must hold a multiple of CH elements per thread");
    extern __shared__ __align__(16) unsigned char smem[];
    T *re = reinterpret_cast<T *>(smem);
    T *im = re + p2_plane(P);
    // small tables next to the planes: twiddles of the sub-transforms (W_nt^j, nt =
    // max(N1, N2) <= kTabTw) and the two-level chirp table (<= kTabCh entries)
    V *ltw = reinterpret_cast<V *>(im + p2_plane(P));
    V *lch = ltw + kTabTw;
    V *buf = scratch + (int64_t)blockIdx.x * slot_len;
    const int tid = threadIdx.x;
    const T cj = (mode == FFT_INV) ? T(-1) : T(1);

    for (int li = blockIdx.x; li < nlats; li += gridDim.x) {
        const LatDesc ld = lat[lats[li]];
        const MDesc m = md[ld.mid];
        const int N = m.N, M = ld.M;
        const double inv2m = 1.0 / (2.0 * (double)M);
        const int logN = 31 - __clz(N), logN1 = 31 - __clz(m.N1), logN2 = 31 - __clz(m.N2);
        const V *twN = tw_tab + m.tw_N;
        const V *x = in + ld.node_off;
        const V *sp = spec_tab + m.spec_off;
        // small tables in LDS when they fit (LTAB), else read from the global tables
        const int logNT = LTAB ? max(logN1, logN2) : logN;
        const V *ctab;
        const V *tsub;
        if constexpr (LTAB) {
            const int nch = m.chirp_nlo + (2 * M + m.chirp_nlo - 1) / m.chirp_nlo;
            __syncthreads();
            for (int j = tid; j < (1 << logNT); j += NT) ltw[j] = twN[j << (logN - logNT)];
            for (int j = tid; j < nch; j += NT) lch[j] = chirp_tab[m.chirp_off + j];
            __syncthreads();
            ctab = lch;
            tsub = ltw;
        } else {
            ctab = chirp_tab + m.chirp_off;
            tsub = twN;
        }
        const int logB2 = min(logN2, LOGP - logN1);
        const int logB1 = min(logN1, LOGP - logN2);
        const int B2 = 1 << logB2, B1 = 1 << logB1;
        const int lrA = max(logN1, 5), lrB = max(logN2, 5);   // LDS rows of phases A/C and B

        // ---- phase A: columns.  The raw inputs of a batch are loaded together into
        // LDS, then each thread chirps its own elements (no barrier in between).
        for (int c0 = 0; c0 < (1 << logN2); c0 += B2) {
            const int tot = B2 << logN1;
            if (mode != FFT_SPEC) {
                _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                    V v[CH];
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        const int e = opaque(tid) + (i0 + i) * NT;
                        const int nn = ((e >> logB2) << logN2) + c0 + (e & (B2 - 1));
                        v[i] = x[(e < tot && nn < M) ? nn : 0];
                    }
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        const int e = opaque(tid) + (i0 + i) * NT;
                        if (e < tot) {
                            const int nn = ((e >> logB2) << logN2) + c0 + (e & (B2 - 1));
                            const int q = padr(((e & (B2 - 1)) << logN1) + (e >> logB2), lrA);
                            re[q] = nn < M ? v[i].x : T(0);
                            im[q] = nn < M ? cj * v[i].y : T(0);
                        }
                    }
                }
            }
#pragma unroll 4
            for (int i = 0; i < EPT; ++i) {
                const int e = opaque(tid) + i * NT;
                if (e < tot) {
                    const int b = e & (B2 - 1), n1 = e >> logB2;
                    const int nn = (n1 << logN2) + c0 + b;
                    const int q = padr((b << logN1) + n1, lrA);
                    if (mode == FFT_SPEC) {
                        int src = -1;
                        if (nn < M) src = nn;
                        else if (nn > N - M) src = N - nn;
                        T xr = 0, xi = 0;
                        if (src >= 0) {
                            V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, src, M, inv2m);
                            xr = w.x; xi = -w.y;
                        }
                        re[q] = xr; im[q] = xi;
                    } else if (nn < M) {
                        const V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, nn, M, inv2m);
                        const T vr = re[q], vi = im[q];
                        re[q] = vr * w.x - vi * w.y;
                        im[q] = vr * w.y + vi * w.x;
                    }
                }
            }
            __syncthreads();
            lds_fft_p2<T, NT, P>(re, im, logN1, logB2, tsub, logNT);
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V w[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    w[i] = twN[e < tot ? (c0 + (e & (B2 - 1))) * (e >> logB2) : 0];   // e^{-2 pi i n2 k1 / N}
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    if (e < tot) {
                        const int b = e & (B2 - 1), k1 = e >> logB2;
                        const T a = re[padr((b << logN1) + k1, lrA)], bb = im[padr((b << logN1) + k1, lrA)];
                        V o; o.x = a * w[i].x - bb * w[i].y; o.y = a * w[i].y + bb * w[i].x;
                        buf[((int64_t)k1 << logN2) + c0 + b] = o;
                    }
                }
            }
            __syncthreads();
        }
        // ---- phase B: rows (forward), spectrum, rows (inverse), twiddle, in place
        for (int r0 = 0; r0 < (1 << logN1); r0 += B1) {
            const int tot = B1 << logN2;
            V *row = buf + ((int64_t)r0 << logN2);
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V v[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    v[i] = row[e < tot ? e : 0];
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    if (e < tot) { re[padr(e, lrB)] = v[i].x; im[padr(e, lrB)] = v[i].y; }
                }
            }
            __syncthreads();
            lds_fft_p2<T, NT, P>(re, im, logN2, logB1, tsub, logNT);
            if (mode == FFT_SPEC) {
                const T s = T(1) / ((T)N * (T)M);
                for (int e = opaque(tid); e < tot; e += NT) {
                    const int b = e & (B1 - 1), k2 = e >> logB1;
                    const int k = r0 + b + (k2 << logN1);
                    V o; o.x = re[padr((b << logN2) + k2, lrB)] * s; o.y = im[padr((b << logN2) + k2, lrB)] * s;
                    spec_tab[m.spec_off + k] = o;
                }
                __syncthreads();
                continue;
            }
            // X[k1 + N1 k2] sits at row b = k1 - r0, column k2: times the spectrum, conjugated
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V sv[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;   // b = e mod B1 (fast), k2 = e / B1
                    sv[i] = sp[e < tot ? r0 + (e & (B1 - 1)) + ((e >> logB1) << logN1) : 0];
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    if (e < tot) {
                        const int q = padr(((e & (B1 - 1)) << logN2) + (e >> logB1), lrB);
                        const T a = re[q], bb = im[q];
                        re[q] = a * sv[i].x - bb * sv[i].y;
                        im[q] = -(a * sv[i].y + bb * sv[i].x);
                    }
                }
            }
            __syncthreads();
            lds_fft_p2<T, NT, P>(re, im, logN2, logB1, tsub, logNT);
            // undo the conjugation, twiddle e^{+2 pi i b' k1 / N} (b' = output column), store
            // U[k1][b'] over the rows just read: element e is row b = e / N2, column b' = e mod N2
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V w[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    w[i] = twN[e < tot ? (e & ((1 << logN2) - 1)) * (r0 + (e >> logN2)) : 0];   // b' k1 < N
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    if (e < tot) {
                        const T a = re[padr(e, lrB)], bb = -im[padr(e, lrB)];
                        V o; o.x = a * w[i].x + bb * w[i].y; o.y = bb * w[i].x - a * w[i].y;   // times conj(w)
                        row[e] = o;
                    }
                }
            }
            __syncthreads();
        }
        if (mode == FFT_SPEC) continue;
        // ---- phase C: inverse columns over k1 for a batch of b'
        for (int c0 = 0; c0 < (1 << logN2); c0 += B2) {
            const int tot = B2 << logN1;
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V v[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    v[i] = buf[e < tot ? ((int64_t)(e >> logB2) << logN2) + c0 + (e & (B2 - 1)) : 0];
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = opaque(tid) + (i0 + i) * NT;
                    if (e < tot) {
                        const int q = padr(((e & (B2 - 1)) << logN1) + (e >> logB2), lrA);
                        re[q] = v[i].x; im[q] = -v[i].y;
                    }
                }
            }
            __syncthreads();
            lds_fft_p2<T, NT, P>(re, im, logN1, logB2, tsub, logNT);
            const T sc = scale_by_m ? scale * (T)M : scale;
            for (int e = opaque(tid); e < tot; e += NT) {
                const int b = e & (B2 - 1), a = e >> logB2;   // output n = N2 a + (c0 + b)
                const int h = (a << logN2) + c0 + b;
                bool set = false;
                if (h < M) {
                    const int q = padr((b << logN1) + a, lrA);
                    const T cr = re[q], ci = -im[q];
                    const V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, h, M, inv2m);
                    T gr = (cr * w.x - ci * w.y) * sc;
                    T gi = (cr * w.y + ci * w.x) * sc;
                    if (mode == FFT_INV) gi = -gi;
                    V o; o.x = gr; o.y = gi;
                    out[ld.node_off + h] = o;
                    set = gr * gr + gi * gi >= th2;
                }
                // every lane of the loop takes part (runs of consecutive h per wave)
                if (mode == FFT_FWD && bitmap) bitmap_set_lanes(bitmap, ld.node_off + h, set);
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ host side
const FftSched kSched[kNumSched] = {
    {"lds", 0, kFftThreads, 0, 1, 0, 0, 0},
    {"4step-512x2-ceil", 1, 512, 12, 2, 0, 0, 0},
    {"4step-512x2-floor", 1, 512, 12, 2, 1, 0, 0},
    {"4step-512x1-ceil", 1, 512, 13, 1, 0, 0, 0},
    {"4step-512x1-floor", 1, 512, 13, 1, 1, 0, 0},
    {"4step-1024x1-ceil", 1, 1024, 13, 1, 0, 0, 0},
    {"4step-1024x1-floor", 1, 1024, 13, 1, 1, 0, 0},
    {"4step-256x2-ceil", 1, 256, 12, 2, 0, 0, 0},
    {"4step-256x2-floor", 1, 256, 12, 2, 1, 0, 0},
    {"rader-20", 0, 1024, 0, 1, 0, 1, 0},
    {"reg", 0, 0, 0, 1, 0, 0, 1},
    {"split", 0, kSplitLen / 16, 0, 1, 0, 0, 2},
};

template <typename T, int LOGP, bool LTAB>
constexpr size_t lds_4step()
{
    return 2 * sizeof(T) * p2_plane(1 << LOGP) + (LTAB ? (kTabTw + kTabCh) * 2 * sizeof(T) : 0);
}

template <typename T, bool LTAB, int NT, int LOGP, int WAVES>
static int launch4(Plan &p, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                   T th2, uint32_t *bitmap, int mode, T scale, int by_m, int per_cu)
{
    using V = typename cvec<T>::type;
    static_assert(lds_4step<T, LOGP, LTAB>() <= (size_t)kLdsBytes, "four-step LDS budget");
    const int grid = std::min(nl, std::min(p.fft_slots, per_cu * num_cus()));
    if (grid < 1) return fail(MR1L_E_ARG, "four-step DFT without a scratch slot");
    constexpr size_t shm = lds_4step<T, LOGP, LTAB>();
    hipLaunchKernelGGL((k_bluestein_4step<T, LTAB, NT, LOGP, WAVES>), dim3(grid), dim3(NT), shm, p.stream, d_lats, nl, p.d_lat, d_md, (const V *)in, (V *)out,
                       (V *)p.d_spec, (const V *)p.d_chirp, (const V *)p.d_tw, bitmap, th2, mode, scale, by_m,
                       (V *)p.d_fft_scratch, p.fft_slot_len);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

// One launch of schedule s over the lattices d_lats (their sizes' tables in d_md).
template <typename T, int NT, int NMAXT, bool PAD>
static int launch_lds(Plan &p, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                      T th2, uint32_t *bitmap, int mode, T sc, int by_m)
{
    using V = typename cvec<T>::type;
    constexpr size_t shm = 2 * sizeof(T) * (size_t)mr_plane<NMAXT, PAD>();
    static_assert(shm <= (size_t)kLdsBytes, "LDS transform budget");
    hipLaunchKernelGGL((k_bluestein_lds<T, NT, NMAXT, PAD>), dim3((unsigned)nl), dim3(NT), shm, p.stream, d_lats, p.d_lat,
                       d_md, (const V *)in, (V *)out, (V *)p.d_spec, (const V *)p.d_chirp, (const V *)p.d_tw, bitmap,
                       th2, mode, sc, by_m);
    MR1L_LAUNCH_CHECK();
    return MR1L_OK;
}

template <typename T>
static int launch_sched(Plan &p, int s, int cls, const int32_t *d_lats, int nl, const MDesc *d_md, bool ltab,
                        const void *in, void *out, double theta, uint32_t *bitmap, int mode, double scale,
                        int by_m)
{
    constexpr int LS = sizeof(T) == 8 ? 12 : 13;   // log2 LDS batch of the two-per-CU schedules
    const T th2 = (T)(theta * theta);
    const T sc = (T)scale;
    const int pc = kSched[s].per_cu;
    if (nl <= 0) return MR1L_OK;
    switch (s) {
    case 0:
        if (cls == 0) return launch_lds<T, 128, 1024, true>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
        if (cls == 1) return launch_lds<T, 512, 4096, true>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m);
        return launch_lds<T, kFftThreads, lds_max_n<T>(), false>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc,
                                                                 by_m);
    case 1: case 2:
        return ltab ? launch4<T, true, 512, LS, 4>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc)
                    : launch4<T, false, 512, LS, 4>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc);
    case 3: case 4:
        return ltab ? launch4<T, true, 512, LS + 1, 2>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc)
                    : launch4<T, false, 512, LS + 1, 2>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc);
    case 5: case 6:
        return ltab ? launch4<T, true, 1024, LS + 1, 4>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc)
                    : launch4<T, false, 1024, LS + 1, 4>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc);
    case 7: case 8:
        return ltab ? launch4<T, true, 256, LS, 2>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc)
                    : launch4<T, false, 256, LS, 2>(p, d_lats, nl, d_md, in, out, th2, bitmap, mode, sc, by_m, pc);
    case 9:
        return rader_launch(p, cls, d_lats, nl, in, out, theta, bitmap, mode, scale, by_m);   // cls = M - 1
    case 10:   // cls = transform length
        return sizeof(T) == 8 ? reg_launch_d(p, cls, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m)
                              : reg_launch_f(p, cls, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);
    case 11:
        if (sizeof(T) != 8) return fail(MR1L_E_ARG, "the split DFT schedule is complex128 only");
        return split_launch_d(p, cls, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);   // cls = K
    default:
        return fail(MR1L_E_ARG, "unknown DFT schedule");
    }
}

static int launch_any(Plan &p, int s, int cls, const int32_t *d_lats, int nl, const MDesc *d_md, bool ltab,
                      const void *in, void *out, double theta, uint32_t *bitmap, int mode, double scale, int by_m)
{
    return p.dtype == MR1L_C128
               ? launch_sched<double>(p, s, cls, d_lats, nl, d_md, ltab, in, out, theta, bitmap, mode, scale, by_m)
               : launch_sched<float>(p, s, cls, d_lats, nl, d_md, ltab, in, out, theta, bitmap, mode, scale, by_m);
}

template <typename K> static int allow_lds_one(K k, size_t bytes)
{
    MR1L_HIP(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return MR1L_OK;
}

template <typename T> static int allow_lds()
{
    constexpr int LS = sizeof(T) == 8 ? 12 : 13;
    constexpr size_t e = sizeof(T);
    int rc = MR1L_OK;
    if (!rc) rc = allow_lds_one(k_bluestein_lds<T, 128, 1024, true>, 2 * e * mr_plane<1024, true>());
    if (!rc) rc = allow_lds_one(k_bluestein_lds<T, 512, 4096, true>, 2 * e * mr_plane<4096, true>());
    if (!rc) rc = allow_lds_one(k_bluestein_lds<T, kFftThreads, lds_max_n<T>(), false>, 2 * e * lds_max_n<T>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, true, 512, LS, 4>, lds_4step<T, LS, true>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, false, 512, LS, 4>, lds_4step<T, LS, false>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, true, 512, LS + 1, 2>, lds_4step<T, LS + 1, true>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, false, 512, LS + 1, 2>, lds_4step<T, LS + 1, false>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, true, 1024, LS + 1, 4>, lds_4step<T, LS + 1, true>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, false, 1024, LS + 1, 4>, lds_4step<T, LS + 1, false>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, true, 256, LS, 2>, lds_4step<T, LS, true>());
    if (!rc) rc = allow_lds_one(k_bluestein_4step<T, false, 256, LS, 2>, lds_4step<T, LS, false>());
    return rc;
}

constexpr int64_t kFftForkNodes = int64_t(1) << 20;   // nodes from which DFT groups run concurrently

int fft_run(Plan &p, const void *in, void *out, double theta, uint32_t *bitmap, int mode, double scale)
{
    // mode FFT_INV with scale < 0 means "multiply by M" (used by the sampler)
    int by_m = 0;
    if (mode == FFT_INV && scale < 0) { by_m = 1; scale = -scale; }
    if (bitmap) {
        int rc = launch_fill_u32(bitmap, (p.nodes + 31) / 32, 0u, p.stream);
        if (rc) return rc;
    }
    // Groups that use the scratch slots (four-step, split) run in turn on the plan's
    // stream, the largest first; the others are spread over the auxiliary streams
    // (forked from the plan's stream after the bitmap fill, joined back at the end),
    // so that the tail of one group's launch overlaps the next group's work.
    std::vector<int> order(p.fft_groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    auto uses_scratch = [&](int i) {
        const int s = p.fft_groups[i].sched;
        return kSched[s].four_step || kSched[s].engine == 2;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (uses_scratch(a) != uses_scratch(b)) return uses_scratch(a);
        return p.fft_groups[a].work > p.fft_groups[b].work;
    });
    // (small plans stay on one stream: the cross-stream waits cost more than the
    // overlap gains when each group is a short launch)
    int nfork = 0;
    for (int i : order) nfork += !uses_scratch(i);
    const bool fork = nfork > 1 && p.fft_aux[0] != nullptr && p.nodes >= kFftForkNodes;
    if (fork) MR1L_HIP(hipEventRecord(p.fft_ev[Plan::kFftAux], p.stream));
    bool used[Plan::kFftAux] = {};
    int next = 0;
    for (int i : order) {
        const FftGroup &g = p.fft_groups[i];
        hipStream_t st = p.stream;
        if (fork && !uses_scratch(i)) {
            const int a = next++ % Plan::kFftAux;
            if (!used[a]) MR1L_HIP(hipStreamWaitEvent(p.fft_aux[a], p.fft_ev[Plan::kFftAux], 0));
            used[a] = true;
            st = p.fft_aux[a];
        }
        const hipStream_t keep = p.stream;
        p.stream = st;
        int rc = launch_any(p, g.sched, g.cls, g.d_lats, (int)g.lats.size(), p.d_mdesc, g.ltab, in, out, theta,
                            bitmap, mode, scale, by_m);
        p.stream = keep;
        if (rc) return rc;
    }
    for (int a = 0; a < Plan::kFftAux; ++a)
        if (used[a]) {
            MR1L_HIP(hipEventRecord(p.fft_ev[a], p.fft_aux[a]));
            MR1L_HIP(hipStreamWaitEvent(p.stream, p.fft_ev[a], 0));
        }
    return MR1L_OK;
}

int fft_init_attrs()
{
    int rc = allow_lds<double>();
    if (!rc) rc = allow_lds<float>();
    if (!rc) rc = lfft_attrs_d();
    if (!rc) rc = lfft_attrs_f();
    return rc;
}

// Table entry of size `mid` for the layout of schedule s.
MDesc fft_layout(const Plan &p, int mid, int s)
{
    MDesc m = p.mdesc[mid];
    const MInfo &mi = p.minfo[mid];
    if (kSched[s].engine == 1) {
        m.spec_off = mi.spec_r; m.tw_N = mi.tw_r; m.N = mi.Nr; m.N1 = mi.Nr; m.N2 = 1;
    } else if (kSched[s].engine == 2) {
        m.spec_off = mi.spec_q; m.tw_N = mi.tw_q; m.N = mi.Nq; m.N1 = mi.Bq; m.N2 = mi.Kq;
    } else if (!kSched[s].four_step && !kSched[s].rader) {
        m.spec_off = mi.spec_s; m.tw_N = mi.tw_s; m.N = mi.Ns; m.N1 = mi.Ns; m.N2 = 1;
    } else {
        int k = 0;
        while ((1 << k) < mi.Np) ++k;
        const int kc = (k + 1) / 2, kf = k / 2;
        m.spec_off = mi.spec_p; m.tw_N = mi.tw_p; m.N = mi.Np;
        m.N1 = 1 << (kSched[s].split_floor ? kf : kc);
        m.N2 = mi.Np / m.N1;
    }
    return m;
}

static bool applies(const MInfo &mi, int s)
{
    if (kSched[s].engine == 1) return mi.Nr > 0;
    if (kSched[s].engine == 2) return mi.Nq > 0;
    if (kSched[s].rader) return mi.rader;
    return kSched[s].four_step ? mi.Np > 0 : mi.Ns > 0;
}
bool fft_schedule_applies(const MInfo &mi, int s) { return s >= 0 && s < kNumSched && applies(mi, s); }

// Grow the four-step scratch to `slots` slots of `len` complex (capped at 8 GiB in
// total, at least one slot).  Synchronises the plan's stream before freeing.
static int ensure_scratch(Plan &p, int64_t len, int64_t slots)
{
    const int64_t esz = p.dtype == MR1L_C128 ? 16 : 8;
    len = std::max(len, p.fft_slot_len);
    const int64_t cap = std::max<int64_t>(1, (int64_t(8) << 30) / (len * esz));
    slots = std::min(std::max<int64_t>({slots, (int64_t)p.fft_slots, 1}), cap);
    if (p.d_fft_scratch && len == p.fft_slot_len && slots == p.fft_slots) return MR1L_OK;
    MR1L_HIP(hipStreamSynchronize(p.stream));
    p.fft_slots = 0;
    if (int rc = plan_regrow(p, &p.d_fft_scratch, (size_t)(slots * len * esz))) return rc;
    p.fft_slot_len = len;
    p.fft_slots = (int32_t)slots;
    return MR1L_OK;
}

// Spectrum layout kind of schedule s: 0 whole-LDS, 1 four-step, 2 split, 3 reg, -1
// none (Rader keeps its own tables).
static int spec_kind(int s)
{
    if (kSched[s].rader) return -1;
    if (kSched[s].engine == 1) return 3;
    if (kSched[s].engine == 2) return 2;
    return kSched[s].four_step ? 1 : 0;
}

static int fft_prepare_spectra(Plan &p);

int fft_apply_schedules(Plan &p, bool fresh)
{
    // the device layout table and group lists may be read by queued work
    if (!fresh) MR1L_HIP(hipStreamSynchronize(p.stream));
    for (size_t mid = 0; mid < p.minfo.size(); ++mid) p.mdesc[mid] = fft_layout(p, (int)mid, p.minfo[mid].sched);
    MR1L_HIP(hipMemcpyAsync(p.d_mdesc, p.mdesc.data(), p.mdesc.size() * sizeof(MDesc), hipMemcpyHostToDevice,
                            p.stream));
    p.fft_groups.clear();
    std::map<std::pair<int, int>, size_t> gi;   // (schedule, class) -> group
    int64_t len = 0, slots = 0;
    for (size_t i = 0; i < p.lat.size(); ++i) {
        const MInfo &mi = p.minfo[p.lat[i].mid];
        // one group per size for the Rader kernels (compiled per length M - 1), per
        // transform length for reg
        const int cls = kSched[mi.sched].rader          ? (int)(mi.M - 1)
                        : kSched[mi.sched].engine == 1 ? mi.Nr
                        : kSched[mi.sched].engine == 2 ? mi.Kq
                        : kSched[mi.sched].four_step   ? 0
                                                       : lds_class(mi.Ns);
        auto it = gi.find({mi.sched, cls});
        if (it == gi.end()) {
            it = gi.emplace(std::make_pair(mi.sched, cls), p.fft_groups.size()).first;
            p.fft_groups.emplace_back();
            p.fft_groups.back().sched = mi.sched;
            p.fft_groups.back().cls = cls;
        }
        FftGroup &g = p.fft_groups[it->second];
        g.lats.push_back((int32_t)i);
        g.work += (double)mi.M * std::log2((double)mi.M + 1.0);
        g.ltab = g.ltab && mi.ltab;
        if (kSched[mi.sched].four_step) len = std::max<int64_t>(len, mi.Np);
        if (kSched[mi.sched].engine == 2) len = std::max<int64_t>(len, (int64_t)(mi.Kq - 1) * mi.Nq);
    }
    // every group's lattice list in one device buffer (one copy)
    p.h_glists.clear();
    std::vector<size_t> goff;
    for (const FftGroup &g : p.fft_groups) {
        goff.push_back(p.h_glists.size());
        p.h_glists.insert(p.h_glists.end(), g.lats.begin(), g.lats.end());
    }
    if ((int64_t)p.h_glists.size() > p.glists_cap) {
        p.glists_cap = 0;
        if (int rc = plan_regrow(p, (void **)&p.d_glists, std::max<size_t>(p.h_glists.size(), 1) * sizeof(int32_t)))
            return rc;
        p.glists_cap = (int64_t)p.h_glists.size();
    }
    if (!p.h_glists.empty())
        MR1L_HIP(hipMemcpyAsync(p.d_glists, p.h_glists.data(), p.h_glists.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, p.stream));
    for (size_t k = 0; k < p.fft_groups.size(); ++k) {
        FftGroup &g = p.fft_groups[k];
        g.d_lats = p.d_glists + goff[k];
        if (kSched[g.sched].four_step || kSched[g.sched].engine == 2)
            slots = std::max<int64_t>(slots, std::min<int64_t>((int64_t)g.lats.size(),
                                                               (int64_t)kSched[g.sched].per_cu * num_cus()));
    }
    if (len > 0) {
        const int rc = ensure_scratch(p, len, slots);
        if (rc) return rc;
    }
    return fft_prepare_spectra(p);
}

int fft_time_plan(Plan &p, const void *in, void *out, int reps, float *ms)
{
    int rc = fft_run(p, in, out, 0.0, nullptr, FFT_FWD, 1.0);
    if (rc) return rc;
    hipEvent_t a, b;
    MR1L_HIP(hipEventCreate(&a));
    MR1L_HIP(hipEventCreate(&b));
    MR1L_HIP(hipEventRecord(a, p.stream));
    for (int r = 0; r < reps && rc == MR1L_OK; ++r) rc = fft_run(p, in, out, 0.0, nullptr, FFT_FWD, 1.0);
    MR1L_HIP(hipEventRecord(b, p.stream));
    MR1L_HIP(hipEventSynchronize(b));
    float t = 0.f;
    MR1L_HIP(hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / (float)std::max(reps, 1);
    return rc;
}

// Kernel spectra of the layouts that the sizes' current schedules use and that are
// not computed yet, computed by the DFT kernels themselves (SPEC mode) on one
// representative lattice per size.  The passes' layout tables and representative
// lists go to the plan's spectrum work buffer in one copy; work of an earlier call
// that still reads that buffer has ended (it is only reused after a stream
// synchronisation in fft_apply_schedules, or grown after one here).
static int fft_prepare_spectra(Plan &p)
{
    std::vector<int32_t> rep(p.minfo.size(), -1);
    for (size_t i = 0; i < p.lat.size(); ++i)
        if (rep[p.lat[i].mid] < 0) rep[p.lat[i].mid] = (int32_t)i;
    // (schedule, class): the reg schedule runs one launch per transform length
    std::vector<std::pair<int, int>> passes = {{0, kLdsClasses - 1}, {kDefaultFourStep, 0}, {kSplitSched, 0}};
    {
        std::vector<int> lens;
        for (const MInfo &mi : p.minfo)
            if (mi.Nr && std::find(lens.begin(), lens.end(), mi.Nr) == lens.end()) lens.push_back(mi.Nr);
        for (int n : lens) passes.push_back({kRegSched, n});
    }
    struct Pass {
        int s, cls, n;
        bool ltab;
        size_t md_off, rep_off;
    };
    std::vector<Pass> todo;
    std::vector<MDesc> mds;
    std::vector<int32_t> reps;
    int64_t len = 0, slots = 0;
    for (const auto &sc : passes) {
        const int s = sc.first, kind = spec_kind(s);
        std::vector<MDesc> md(p.mdesc);
        const size_t r0 = reps.size();
        bool ltab = true;
        for (size_t mid = 0; mid < p.minfo.size(); ++mid) {
            const MInfo &mi = p.minfo[mid];
            if (rep[mid] < 0 || spec_kind(mi.sched) != kind || (mi.spec_done >> kind & 1u)) continue;
            if (s == kRegSched && mi.Nr != sc.second) continue;
            md[mid] = fft_layout(p, (int)mid, s);
            reps.push_back(rep[mid]);
            ltab = ltab && mi.ltab;
            len = std::max<int64_t>(len, s == kSplitSched ? (int64_t)(mi.Kq - 1) * mi.Nq : (int64_t)mi.Np);
        }
        const int n = (int)(reps.size() - r0);
        if (n == 0) continue;
        if (kSched[s].four_step || kSched[s].engine == 2)
            slots = std::max<int64_t>(slots, std::min<int64_t>(n, (int64_t)kSched[s].per_cu * num_cus()));
        todo.push_back({s, sc.second, n, ltab, mds.size(), r0});
        mds.insert(mds.end(), md.begin(), md.end());
    }
    if (todo.empty()) return MR1L_OK;
    int rc = MR1L_OK;
    if (slots > 0 && (rc = ensure_scratch(p, len, slots))) return rc;
    const size_t md_bytes = mds.size() * sizeof(MDesc), rep_at = (md_bytes + 255) & ~size_t(255);
    const size_t bytes = rep_at + reps.size() * sizeof(int32_t);
    if ((int64_t)bytes > p.specwork_bytes) {
        MR1L_HIP(hipStreamSynchronize(p.stream));
        p.specwork_bytes = 0;
        if (int rc = plan_regrow(p, &p.d_specwork, bytes)) return rc;
        p.specwork_bytes = (int64_t)bytes;
    }
    p.h_specwork.assign(bytes, 0);
    std::memcpy(p.h_specwork.data(), mds.data(), md_bytes);
    std::memcpy(p.h_specwork.data() + rep_at, reps.data(), reps.size() * sizeof(int32_t));
    MR1L_HIP(hipMemcpyAsync(p.d_specwork, p.h_specwork.data(), bytes, hipMemcpyHostToDevice, p.stream));
    const MDesc *d_md = (const MDesc *)p.d_specwork;
    const int32_t *d_rep = (const int32_t *)((const unsigned char *)p.d_specwork + rep_at);
    for (const Pass &ps : todo) {
        rc = launch_any(p, ps.s, ps.cls, d_rep + ps.rep_off, ps.n, d_md + ps.md_off, ps.ltab, nullptr, nullptr, 0.0,
                        nullptr, FFT_SPEC, 1.0, 0);
        if (rc) return rc;
    }
    for (size_t mid = 0; mid < p.minfo.size(); ++mid) {
        MInfo &mi = p.minfo[mid];
        const int kind = spec_kind(mi.sched);
        if (kind >= 0 && rep[mid] >= 0) mi.spec_done |= 1u << kind;
    }
    return MR1L_OK;
}

}  // namespace mr1l
