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
#include "mr1l_internal.h"

namespace mr1l {

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
template <typename T, int R>
__device__ void stockham_pass(T *re, T *im, int n, int batch, int Ns,
                              const typename cvec<T>::type *__restrict__ tw)
{
    constexpr int NMAX = lds_max_n<T>();
    constexpr int BPT = (NMAX / R + kFftThreads - 1) / kFftThreads;
    const int nR = n / R;
    const int total = batch * nR;
    const int tstride = n / (Ns * R);
    T vr[BPT][R], vi[BPT][R];
    int ob[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int j = threadIdx.x + i * kFftThreads;
        ob[i] = -1;
        if (j < total) {
            const int b = j / nR;
            const int jj = j - b * nR;
            const int q = jj / Ns;
            const int k = jj - q * Ns;
            const int base = b * n + jj;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                vr[i][r] = re[base + r * nR];
                vi[i][r] = im[base + r * nR];
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
                re[ob[i] + r * Ns] = vr[i][r];
                im[ob[i] + r * Ns] = vi[i][r];
            }
        }
    }
    __syncthreads();
}

// Forward FFT (e^{-2 pi i}) of `batch` contiguous length-n transforms in LDS;
// tw = table e^{-2 pi i m / n}, m < n.  Output in natural order.
template <typename T>
__device__ void lds_fft(T *re, T *im, int n, int batch, const typename cvec<T>::type *tw)
{
    int Ns = 1, rem = n;
    while (rem > 1) {
        const int R = next_radix(rem);
        switch (R) {
        case 8: stockham_pass<T, 8>(re, im, n, batch, Ns, tw); break;
        case 4: stockham_pass<T, 4>(re, im, n, batch, Ns, tw); break;
        case 2: stockham_pass<T, 2>(re, im, n, batch, Ns, tw); break;
        case 5: stockham_pass<T, 5>(re, im, n, batch, Ns, tw); break;
        default: stockham_pass<T, 3>(re, im, n, batch, Ns, tw); break;
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

// LDS planes of the power-of-two path hold NMAXP elements with one pad element
// after every 16, which breaks the power-of-two strides of the column accesses
// and of the early Stockham passes (bank conflicts).
constexpr int kFft4Threads = 512;   // two four-step workgroups per CU
constexpr int kTabTw = 256;         // LDS twiddles of the four-step sub-transforms
constexpr int kTabCh = 384;         // LDS two-level chirp table entries
template <typename T> constexpr int p2_max_n() { return sizeof(T) == 8 ? 4096 : 8192; }
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }
template <typename T> constexpr int p2_plane() { return p2_max_n<T>() + p2_max_n<T>() / 16; }

// One Stockham pass of radix 2^LR over 2^logb transforms of length 2^logn; the
// twiddle e^{-2 pi i r k / (Ns R)} is entry (r k) << (logN - logNs - LR) of a
// table e^{-2 pi i j / 2^logN} (logN >= logn; in LDS for the lengths used here).
template <typename T, int LR, typename TW>
__device__ void stockham_p2(T *re, T *im, int logn, int logb, int logNs, TW tw, int logN)
{
    constexpr int R = 1 << LR;
    constexpr int BPT = (p2_max_n<T>() / R + kFft4Threads - 1) / kFft4Threads;
    const int lognR = logn - LR;
    const int total = 1 << (logb + lognR);
    const int tsh = logN - logNs - LR;
    T vr[BPT][R], vi[BPT][R];
    int ob[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int j = threadIdx.x + i * kFft4Threads;
        ob[i] = -1;
        if (j < total) {
            const int b = j >> lognR;
            const int jj = j & ((1 << lognR) - 1);
            const int k = jj & ((1 << logNs) - 1);
            const int q = jj >> logNs;
            const int base = (b << logn) + jj;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                vr[i][r] = re[pad16(base + (r << lognR))];
                vi[i][r] = im[pad16(base + (r << lognR))];
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
                re[pad16(ob[i] + (r << logNs))] = vr[i][r];
                im[pad16(ob[i] + (r << logNs))] = vi[i][r];
            }
        }
    }
    __syncthreads();
}

template <typename T, typename TW>
__device__ void lds_fft_p2(T *re, T *im, int logn, int logb, TW tw, int logN)
{
    int logNs = 0, rem = logn;
    while (rem > 0) {
        // radix 16 for float; radix 8 at most for double, whose 16-point butterfly
        // would not fit the register budget of two workgroups per CU
        if (sizeof(T) == 4 && rem >= 4) { stockham_p2<T, 4, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 4; rem -= 4; }
        else if (sizeof(T) == 8 && rem >= 3) { stockham_p2<T, 3, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 3; rem -= 3; }
        else if (rem == 3) { stockham_p2<T, 3, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 3; rem -= 3; }
        else if (rem == 2) { stockham_p2<T, 2, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 2; rem -= 2; }
        else { stockham_p2<T, 1, TW>(re, im, logn, logb, logNs, tw, logN); logNs += 1; rem -= 1; }
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

template <typename T>
__device__ __forceinline__ void set_bit_if(uint32_t *bitmap, int64_t g, T re, T im, T th2)
{
    if (re * re + im * im >= th2) atomicOr(bitmap + (g >> 5), 1u << (g & 31));
}

// ------------------------------------------------------------------ LDS kernel
// One workgroup per lattice with N <= NMAX.  mode: FFT_FWD (f -> ghat, bitmap),
// FFT_INV (g -> (1/M) sum g e^{+}) times scale (times M when scale_by_m),
// FFT_SPEC (kernel spectrum of the lattice size, written to the spectrum table).
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_bluestein_lds(
    const int32_t *__restrict__ lats, const LatDesc *__restrict__ lat, const MDesc *__restrict__ md,
    const typename cvec<T>::type *__restrict__ in, typename cvec<T>::type *__restrict__ out,
    typename cvec<T>::type *__restrict__ spec_tab, const typename cvec<T>::type *__restrict__ chirp_tab,
    const typename cvec<T>::type *__restrict__ tw_tab, uint32_t *__restrict__ bitmap, T th2, int mode,
    T scale, int scale_by_m)
{
    using V = typename cvec<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    T *re = reinterpret_cast<T *>(smem);
    T *im = re + lds_max_n<T>();
    const LatDesc ld = lat[lats[blockIdx.x]];
    const MDesc m = md[ld.mid];
    const int N = ld.N, M = ld.M;
    const double inv2m = 1.0 / (2.0 * (double)M);
    const V *ctab = chirp_tab + m.chirp_off;
    const V *tw = tw_tab + m.tw_N;
    const int tid = threadIdx.x;

    if (mode == FFT_SPEC) {
        // B[n] = conj(w[n]) for n < M, B[N - n] = conj(w[n]) for 0 < n < M
        for (int i = tid; i < N; i += kFftThreads) {
            int src = -1;
            if (i < M) src = i;
            else if (i > N - M) src = N - i;
            T xr = 0, xi = 0;
            if (src >= 0) {
                V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, src, M, inv2m);
                xr = w.x; xi = -w.y;
            }
            re[i] = xr; im[i] = xi;
        }
        __syncthreads();
        lds_fft<T>(re, im, N, 1, tw);
        const T s = T(1) / ((T)N * (T)M);
        V *dst = spec_tab + m.spec_off;
        for (int i = tid; i < N; i += kFftThreads) {
            V o; o.x = re[i] * s; o.y = im[i] * s;
            dst[i] = o;
        }
        return;
    }

    const T cj = (mode == FFT_INV) ? T(-1) : T(1);
    const V *x = in + ld.node_off;
    constexpr int EPT = (lds_max_n<T>() + kFftThreads - 1) / kFftThreads;
    {
        T xr[EPT], xi[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = tid + k * kFftThreads;
            xr[k] = 0; xi[k] = 0;
            if (i < M) {
                V v = x[i];
                V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, i, M, inv2m);
                const T vi = cj * v.y;
                xr[k] = v.x * w.x - vi * w.y;
                xi[k] = v.x * w.y + vi * w.x;
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = tid + k * kFftThreads;
            if (i < N) { re[i] = xr[k]; im[i] = xi[k]; }
        }
    }
    __syncthreads();
    lds_fft<T>(re, im, N, 1, tw);
    const V *sp = spec_tab + m.spec_off;
    {
        V sv[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = tid + k * kFftThreads;
            if (i < N) sv[k] = sp[i];
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = tid + k * kFftThreads;
            if (i < N) {
                T a = re[i], b = im[i];
                re[i] = a * sv[k].x - b * sv[k].y;
                im[i] = -(a * sv[k].y + b * sv[k].x);   // conjugate: the next FFT is an inverse one
            }
        }
    }
    __syncthreads();
    lds_fft<T>(re, im, N, 1, tw);
    const T sc = scale_by_m ? scale * (T)M : scale;
    V *y = out + ld.node_off;
    for (int i = tid; i < M; i += kFftThreads) {
        V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, i, M, inv2m);
        const T cr = re[i], ci = -im[i];     // undo the conjugation
        T gr = (cr * w.x - ci * w.y) * sc;
        T gi = (cr * w.y + ci * w.x) * sc;
        if (mode == FFT_INV) gi = -gi;
        V o; o.x = gr; o.y = gi;
        y[i] = o;
        if (mode == FFT_FWD && bitmap) set_bit_if<T>(bitmap, ld.node_off + i, gr, gi, th2);
    }
}

// ------------------------------------------------------------------ four-step kernel
// Power-of-two N = N1 N2 (N1, N2 <= NMAXP), three phases per lattice:
//   A  length-N1 DFTs over n1 of x[N2 n1 + n2] (x = chirped input), twiddle
//      W_N^{n2 k1}, stored Y[k1][n2];
//   B  for a batch of k1: length-N2 DFTs over n2 give X[k1 + N1 k2]; times the
//      kernel spectrum; inverse length-N2 DFTs over k2; twiddle W_N^{-b k1};
//      stored U[b][k1] -- the forward row stage and the first stage of the
//      inverse transform share the LDS, so the product never leaves the chip;
//   C  for a batch of b: inverse length-N1 DFTs over k1 give the convolution at
//      N2 a + b; times the chirp and 1/M (folded into the spectrum); output.
// Inverse DFTs are conj(DFT(conj(.))).  SPEC mode runs A and the forward half of B
// on the chirp sequence and stores the scaled spectrum.  Persistent: workgroup w
// owns scratch slot w (2 maxN complex) and handles lattices w, w + grid, ...
template <typename T, bool LTAB>
__global__ __launch_bounds__(kFft4Threads, 4) void k_bluestein_4step(
    const int32_t *__restrict__ lats, int nlats, const LatDesc *__restrict__ lat,
    const MDesc *__restrict__ md, const typename cvec<T>::type *__restrict__ in,
    typename cvec<T>::type *__restrict__ out, typename cvec<T>::type *__restrict__ spec_tab,
    const typename cvec<T>::type *__restrict__ chirp_tab, const typename cvec<T>::type *__restrict__ tw_tab,
    uint32_t *__restrict__ bitmap, T th2, int mode, T scale, int scale_by_m,
    typename cvec<T>::type *__restrict__ scratch, int64_t slot_len)
{
    using V = typename cvec<T>::type;
    constexpr int NMAXP = p2_max_n<T>();
    constexpr int LOGNMAXP = sizeof(T) == 8 ? 12 : 13;
    constexpr int NT = kFft4Threads;
    extern __shared__ __align__(16) unsigned char smem[];
    T *re = reinterpret_cast<T *>(smem);
    T *im = re + p2_plane<T>();
    // small tables next to the planes: twiddles of the sub-transforms (W_nt^j, nt =
    // max(N1, N2) <= kTabTw) and the two-level chirp table (<= kTabCh entries)
    V *ltw = reinterpret_cast<V *>(im + p2_plane<T>());
    V *lch = ltw + kTabTw;
    V *bufY = scratch + (int64_t)blockIdx.x * slot_len;
    V *bufU = bufY + slot_len / 2;
    const int tid = threadIdx.x;
    const T cj = (mode == FFT_INV) ? T(-1) : T(1);
    (void)NMAXP;

    for (int li = blockIdx.x; li < nlats; li += gridDim.x) {
        const LatDesc ld = lat[lats[li]];
        const MDesc m = md[ld.mid];
        const int N = ld.N, M = ld.M;
        const double inv2m = 1.0 / (2.0 * (double)M);
        const int logN = 31 - __clz(N), logN1 = 31 - __clz(ld.N1), logN2 = 31 - __clz(ld.N2);
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
        const int logB2 = min(logN2, LOGNMAXP - logN1);
        const int logB1 = min(logN1, LOGNMAXP - logN2);
        const int B2 = 1 << logB2, B1 = 1 << logB1;

        // ---- phase A: columns.  The raw inputs of a batch are loaded together into
        // LDS, then each thread chirps its own elements (no barrier in between).
        constexpr int EPT = p2_max_n<T>() / NT;   // elements per thread of a full batch
        constexpr int CH = 4;                     // loads issued together per thread
        for (int c0 = 0; c0 < (1 << logN2); c0 += B2) {
            const int tot = B2 << logN1;
            if (mode != FFT_SPEC) {
                _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                    V v[CH];
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        const int e = tid + (i0 + i) * NT;
                        const int nn = ((e >> logB2) << logN2) + c0 + (e & (B2 - 1));
                        if (e < tot && nn < M) v[i] = x[nn];
                    }
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        const int e = tid + (i0 + i) * NT;
                        if (e < tot) {
                            const int nn = ((e >> logB2) << logN2) + c0 + (e & (B2 - 1));
                            const int q = pad16(((e & (B2 - 1)) << logN1) + (e >> logB2));
                            re[q] = nn < M ? v[i].x : T(0);
                            im[q] = nn < M ? cj * v[i].y : T(0);
                        }
                    }
                }
            }
#pragma unroll 4
            for (int i = 0; i < EPT; ++i) {
                const int e = tid + i * NT;
                if (e < tot) {
                    const int b = e & (B2 - 1), n1 = e >> logB2;
                    const int nn = (n1 << logN2) + c0 + b;
                    const int q = pad16((b << logN1) + n1);
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
            lds_fft_p2<T>(re, im, logN1, logB2, tsub, logNT);
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V w[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) w[i] = twN[(c0 + (e & (B2 - 1))) * (e >> logB2)];   // e^{-2 pi i n2 k1 / N}
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) {
                        const int b = e & (B2 - 1), k1 = e >> logB2;
                        const T a = re[pad16((b << logN1) + k1)], bb = im[pad16((b << logN1) + k1)];
                        V o; o.x = a * w[i].x - bb * w[i].y; o.y = a * w[i].y + bb * w[i].x;
                        bufY[((int64_t)k1 << logN2) + c0 + b] = o;
                    }
                }
            }
            __syncthreads();
        }
        // ---- phase B: rows (forward), spectrum, rows (inverse), twiddle
        for (int r0 = 0; r0 < (1 << logN1); r0 += B1) {
            const int tot = B1 << logN2;
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V v[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) v[i] = bufY[((int64_t)r0 << logN2) + e];
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) { re[pad16(e)] = v[i].x; im[pad16(e)] = v[i].y; }
                }
            }
            __syncthreads();
            lds_fft_p2<T>(re, im, logN2, logB1, tsub, logNT);
            if (mode == FFT_SPEC) {
                const T s = T(1) / ((T)N * (T)M);
                for (int e = tid; e < tot; e += NT) {
                    const int b = e & (B1 - 1), k2 = e >> logB1;
                    const int k = r0 + b + (k2 << logN1);
                    V o; o.x = re[pad16((b << logN2) + k2)] * s; o.y = im[pad16((b << logN2) + k2)] * s;
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
                    const int e = tid + (i0 + i) * NT;   // b = e mod B1 (fast), k2 = e / B1
                    if (e < tot) sv[i] = sp[r0 + (e & (B1 - 1)) + ((e >> logB1) << logN1)];
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) {
                        const int q = pad16(((e & (B1 - 1)) << logN2) + (e >> logB1));
                        const T a = re[q], bb = im[q];
                        re[q] = a * sv[i].x - bb * sv[i].y;
                        im[q] = -(a * sv[i].y + bb * sv[i].x);
                    }
                }
            }
            __syncthreads();
            lds_fft_p2<T>(re, im, logN2, logB1, tsub, logNT);
            // undo the conjugation, twiddle e^{+2 pi i b' k1 / N} (b' = output column), store U[b'][k1]
            _Pragma("unroll 1") for (int i0 = 0; i0 < EPT; i0 += CH) {
                V w[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) w[i] = twN[(e >> logB1) * (r0 + (e & (B1 - 1)))];   // b' k1 < N
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) {
                        const int b = e & (B1 - 1), bp = e >> logB1;   // k1 = r0 + b
                        const int q = pad16((b << logN2) + bp);
                        const T a = re[q], bb = -im[q];
                        V o; o.x = a * w[i].x + bb * w[i].y; o.y = bb * w[i].x - a * w[i].y;   // times conj(w)
                        bufU[((int64_t)bp << logN1) + r0 + b] = o;
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
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) v[i] = bufU[((int64_t)c0 << logN1) + e];
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int e = tid + (i0 + i) * NT;
                    if (e < tot) { re[pad16(e)] = v[i].x; im[pad16(e)] = -v[i].y; }
                }
            }
            __syncthreads();
            lds_fft_p2<T>(re, im, logN1, logB2, tsub, logNT);
            const T sc = scale_by_m ? scale * (T)M : scale;
#pragma unroll 4
            for (int e = tid; e < tot; e += NT) {
                const int b = e & (B2 - 1), a = e >> logB2;   // output n = N2 a + (c0 + b)
                const int h = (a << logN2) + c0 + b;
                if (h < M) {
                    const int q = pad16((b << logN1) + a);
                    const T cr = re[q], ci = -im[q];
                    const V w = chirp<T>(ctab, m.chirp_shift, m.chirp_nlo, h, M, inv2m);
                    T gr = (cr * w.x - ci * w.y) * sc;
                    T gi = (cr * w.y + ci * w.x) * sc;
                    if (mode == FFT_INV) gi = -gi;
                    V o; o.x = gr; o.y = gi;
                    out[ld.node_off + h] = o;
                    if (mode == FFT_FWD && bitmap) set_bit_if<T>(bitmap, ld.node_off + h, gr, gi, th2);
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ host side
template <typename T>
static int fft_launch(Plan &p, const void *in, void *out, double theta, uint32_t *bitmap, int mode,
                      double scale, int scale_by_m)
{
    using V = typename cvec<T>::type;
    const T th2 = (T)(theta * theta);
    const size_t shm = kLdsBytes;
    if (!p.lds_lats.empty()) {
        hipLaunchKernelGGL(k_bluestein_lds<T>, dim3((unsigned)p.lds_lats.size()), dim3(kFftThreads), shm,
                           p.stream, p.d_lds_lats, p.d_lat, p.d_mdesc, (const V *)in, (V *)out,
                           (V *)p.d_spec, (const V *)p.d_chirp, (const V *)p.d_tw, bitmap, th2, mode,
                           (T)scale, scale_by_m);
        MR1L_LAUNCH_CHECK();
    }
    if (!p.big_lats.empty()) {
        const int nl = (int)p.big_lats.size();
        const int grid = std::min(nl, p.fft_slots);   // slots: two per CU
        const bool ltab = p.big_ltab;
        const size_t shm4 = 2 * sizeof(T) * p2_plane<T>() + (ltab ? (kTabTw + kTabCh) * 2 * sizeof(T) : 0);
        if (ltab)
            hipLaunchKernelGGL((k_bluestein_4step<T, true>), dim3(grid), dim3(kFft4Threads), shm4, p.stream,
                               p.d_big_lats, nl, p.d_lat, p.d_mdesc, (const V *)in, (V *)out, (V *)p.d_spec,
                               (const V *)p.d_chirp, (const V *)p.d_tw, bitmap, th2, mode, (T)scale, scale_by_m,
                               (V *)p.d_fft_scratch, (int64_t)2 * p.big_maxN);
        else
            hipLaunchKernelGGL((k_bluestein_4step<T, false>), dim3(grid), dim3(kFft4Threads), shm4, p.stream,
                               p.d_big_lats, nl, p.d_lat, p.d_mdesc, (const V *)in, (V *)out, (V *)p.d_spec,
                               (const V *)p.d_chirp, (const V *)p.d_tw, bitmap, th2, mode, (T)scale, scale_by_m,
                               (V *)p.d_fft_scratch, (int64_t)2 * p.big_maxN);
        MR1L_LAUNCH_CHECK();
    }
    return MR1L_OK;
}

template <typename T> static void allow_lds()
{
    (void)hipFuncSetAttribute((const void *)k_bluestein_lds<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        kLdsBytes);
    (void)hipFuncSetAttribute((const void *)k_bluestein_4step<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    (void)hipFuncSetAttribute((const void *)k_bluestein_4step<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
}

int fft_run(Plan &p, const void *in, void *out, double theta, uint32_t *bitmap, int mode, double scale)
{
    // mode FFT_INV with scale < 0 means "multiply by M" (used by the sampler)
    int by_m = 0;
    if (mode == FFT_INV && scale < 0) { by_m = 1; scale = -scale; }
    if (bitmap) {
        int rc = launch_fill_u32(bitmap, (p.nodes + 31) / 32, 0u, p.stream);
        if (rc) return rc;
    }
    if (p.dtype == MR1L_C128) return fft_launch<double>(p, in, out, theta, bitmap, mode, scale, by_m);
    return fft_launch<float>(p, in, out, theta, bitmap, mode, scale, by_m);
}

void fft_init_attrs()
{
    allow_lds<double>();
    allow_lds<float>();
}

int fft_prepare_spectra(Plan &p)
{
    // one lattice per distinct size: run the SPEC mode on representative lattices
    std::vector<int32_t> rep_lds, rep_big;
    std::vector<char> seen(p.mdesc.size(), 0);
    for (size_t i = 0; i < p.lat.size(); ++i) {
        const LatDesc &ld = p.lat[i];
        if (seen[ld.mid]) continue;
        seen[ld.mid] = 1;
        (ld.N2 == 1 ? rep_lds : rep_big).push_back((int32_t)i);
    }
    std::vector<int32_t> save_lds = p.lds_lats, save_big = p.big_lats;
    int32_t *dl = nullptr, *db = nullptr;
    if (!rep_lds.empty()) {
        MR1L_HIP(hipMalloc(&dl, rep_lds.size() * sizeof(int32_t)));
        MR1L_HIP(hipMemcpy(dl, rep_lds.data(), rep_lds.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (!rep_big.empty()) {
        MR1L_HIP(hipMalloc(&db, rep_big.size() * sizeof(int32_t)));
        MR1L_HIP(hipMemcpy(db, rep_big.data(), rep_big.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    int32_t *sl = p.d_lds_lats, *sb = p.d_big_lats;
    p.lds_lats = rep_lds; p.big_lats = rep_big; p.d_lds_lats = dl; p.d_big_lats = db;
    int rc = fft_run(p, nullptr, nullptr, 0.0, nullptr, FFT_SPEC, 1.0);
    p.lds_lats = save_lds; p.big_lats = save_big; p.d_lds_lats = sl; p.d_big_lats = sb;
    if (rc == MR1L_OK) MR1L_HIP(hipStreamSynchronize(p.stream));
    if (dl) (void)hipFree(dl);
    if (db) (void)hipFree(db);
    return rc;
}

}  // namespace mr1l
