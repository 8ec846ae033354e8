/*
 * Reference oracle for the multiple-rank-1-lattice sparse FFT
 * (Kaemmerer, Krahmer, Volkmer, "A sample efficient sparse FFT for arbitrary
 * frequency candidate sets in high dimensions", arXiv:2006.13053).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow CPU statement of what
 * the method computes.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the GPU library, and it never calls it.
 *
 * Conventions (identical to the public C ABI, restated here on purpose):
 *   - frequencies are structure-of-arrays int64, freq[u*n + i] = k_u of the
 *     i-th frequency, u < d;
 *   - lattice l has prime size M[l] and generating vector z[l*d + u];
 *   - lattice-concatenated arrays (samples f, coefficients ghat, counts) use
 *     offsets O_l = sum_{l' < l} M[l'];
 *   - complex numbers are interleaved doubles (re, im).
 *
 * Precision: every sum is accumulated in long double (x87 80-bit on x86-64);
 * every phase is reduced exactly in integers before a trigonometric call,
 * so results are correct to about 1e-18 relative before the final rounding
 * to double.
 *
 * Parity pins: every function below is pinned by the CPU tests (closed forms,
 * invariants, brute force, library special cases and values printed in the
 * paper).  None is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;
static const ld TWO_PI_L = 6.283185307179586476925286766559005768L;

/* ------------------------------------------------------------------ */
/* Section 2.1: lattice sizes are primes (the set P^Gamma).           */
/* Plain trial division; the sizes used are far below 2^40.           */
/* ------------------------------------------------------------------ */
int orc_is_prime(int64_t n)
{
    if (n < 2) return 0;
    if (n < 4) return 1;
    if (n % 2 == 0) return 0;
    for (int64_t q = 3; q <= n / q; q += 2)
        if (n % q == 0) return 0;
    return 1;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Non-negative representative of x mod m (the "Gamma mod M" convention of
 * Section 2.1: h = k - M floor(k / M)). */
static int64_t floor_mod_i128(__int128 x, int64_t m)
{
    __int128 r = x % (__int128)m;
    if (r < 0) r += m;
    return (int64_t)r;
}

/* ------------------------------------------------------------------ */
/* Bucket of frequency k in lattice l: h = (k . z_l) mod M_l.         */
/* Section 2.2, the rearrangement step of Algorithm 1 (second half of  */
/* Section 2.2, before Algorithm 1), with the floor-mod representative */
/* of Section 2.1.  Exact in 128-bit integers.                         */
/* ------------------------------------------------------------------ */
int64_t orc_hash_one(int32_t d, const int64_t *k, int64_t stride,
                     const int64_t *zl, int64_t Ml)
{
    __int128 acc = 0;
    for (int32_t u = 0; u < d; ++u)
        acc += (__int128)k[(int64_t)u * stride] * (__int128)zl[u];
    return floor_mod_i128(acc, Ml);
}

void orc_hash(int32_t d, int64_t n, const int64_t *freq, int32_t L,
              const int64_t *M, const int64_t *z, int32_t *out /* [L][n] */)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t l = 0; l < L; ++l)
            out[(int64_t)l * n + i] =
                (int32_t)orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l]);
}

/* Bucket occupancy cnt_l[h] = #{k in S : h_l(k) = h}.  This is the count
 * behind the singleton sets of Remark 2.9 and the counting polynomial of
 * eq. (4.1) (Section 4.1.1). */
void orc_counts(int32_t d, int64_t n, const int64_t *freq, int32_t L,
                const int64_t *M, const int64_t *z, int32_t *counts /* [sum M] */)
{
    int64_t off = 0;
    for (int32_t l = 0; l < L; ++l) {
        memset(counts + off, 0, sizeof(int32_t) * (size_t)M[l]);
        for (int64_t i = 0; i < n; ++i)
            counts[off + orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l])]++;
        off += M[l];
    }
}

/* ------------------------------------------------------------------ */
/* Samples of the sparse trigonometric polynomial, eq. (2.2), at the   */
/* rank-1 lattice nodes x_j = j z_l / M_l mod 1, eq. (2.1).            */
/*                                                                     */
/* The lattice fixes the first t coordinates; coordinates u >= t are   */
/* fixed anchors x'_u = a_u / 2^32 shared by all nodes (the embedding  */
/* of Algorithm 3, Step 2a).  For t = d there are no anchors.          */
/* Phase of term k at node j:                                          */
/*   k . x_j = (j (k_{<t} . z_l) mod M_l) / M_l                        */
/*           + ((sum_{u>=t} k_u a_u) mod 2^32) / 2^32     (mod 1)      */
/* Both parts are reduced exactly in integers.                         */
/* ------------------------------------------------------------------ */
void orc_sample(int32_t d, int32_t t, int64_t s, const int64_t *freq,
                const double *coef, const uint32_t *anchor /* [d-t] or NULL */,
                int32_t L, const int64_t *M, const int64_t *z /* [L][t] */,
                double *f /* [sum M][2] */)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L + 1));
    off[0] = 0;
    for (int32_t l = 0; l < L; ++l) off[l + 1] = off[l] + M[l];

    /* anchor phase of every term, as a fraction of 2^32 */
    uint32_t *aph = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(s > 0 ? s : 1));
    for (int64_t i = 0; i < s; ++i) {
        uint32_t acc = 0;
        for (int32_t u = t; u < d; ++u)
            acc += (uint32_t)((uint64_t)freq[(int64_t)u * s + i] * (uint64_t)anchor[u - t]);
        aph[i] = acc; /* arithmetic mod 2^32 is exact for the fractional part */
    }

    for (int32_t l = 0; l < L; ++l) {
        const int64_t Ml = M[l];
        int64_t *h = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s > 0 ? s : 1));
        for (int64_t i = 0; i < s; ++i)
            h[i] = orc_hash_one(t, freq + i, s, z + (int64_t)l * t, Ml);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < Ml; ++j) {
            ld re = 0.0L, im = 0.0L;
            for (int64_t i = 0; i < s; ++i) {
                int64_t r = (int64_t)(((__int128)j * h[i]) % Ml);
                ld frac = (ld)r / (ld)Ml + (ld)aph[i] / 4294967296.0L;
                ld ang = TWO_PI_L * frac;
                ld c = cosl(ang), sn = sinl(ang);
                ld cr = coef[2 * i], ci = coef[2 * i + 1];
                re += cr * c - ci * sn;
                im += cr * sn + ci * c;
            }
            f[2 * (off[l] + j)] = (double)re;
            f[2 * (off[l] + j) + 1] = (double)im;
        }
        free(h);
    }
    free(aph);
    free(off);
}

/* Single sample value (used to check large problems node by node). */
void orc_sample_nodes(int32_t d, int32_t t, int64_t s, const int64_t *freq,
                      const double *coef, const uint32_t *anchor,
                      const int64_t *zl /* [t] */, int64_t Ml,
                      int64_t nj, const int64_t *j_list, double *out /* [nj][2] */)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nj; ++q) {
        const int64_t j = j_list[q];
        ld re = 0.0L, im = 0.0L;
        for (int64_t i = 0; i < s; ++i) {
            uint32_t acc = 0;
            for (int32_t u = t; u < d; ++u)
                acc += (uint32_t)((uint64_t)freq[(int64_t)u * s + i] * (uint64_t)anchor[u - t]);
            int64_t h = orc_hash_one(t, freq + i, s, zl, Ml);
            int64_t r = (int64_t)(((__int128)j * h) % Ml);
            ld ang = TWO_PI_L * ((ld)r / (ld)Ml + (ld)acc / 4294967296.0L);
            ld c = cosl(ang), sn = sinl(ang);
            re += (ld)coef[2 * i] * c - (ld)coef[2 * i + 1] * sn;
            im += (ld)coef[2 * i] * sn + (ld)coef[2 * i + 1] * c;
        }
        out[2 * q] = (double)re;
        out[2 * q + 1] = (double)im;
    }
}

/* ------------------------------------------------------------------ */
/* Normalised lattice DFT, Algorithm 2 line 2 (and the lattice rule of */
/* eq. (2.4)):  ghat_l[h] = (1/M_l) sum_j f_l[j] exp(-2 pi i j h / M_l) */
/* computed directly in O(M^2) per lattice; no FFT.  The twiddle index */
/* (j h) mod M is reduced exactly.  sign = -1 is the forward map;      */
/* sign = +1 gives (1/M) sum_j g[j] exp(+2 pi i j h / M), the adjoint  */
/* of the forward map.                                                 */
/* ------------------------------------------------------------------ */
static void dft_one(int64_t Ml, const double *x, double *y, int sign,
                    int64_t nb, const int64_t *bins)
{
    ld *cw = (ld *)malloc(sizeof(ld) * (size_t)Ml);
    ld *sw = (ld *)malloc(sizeof(ld) * (size_t)Ml);
    for (int64_t r = 0; r < Ml; ++r) {
        ld ang = TWO_PI_L * (ld)r / (ld)Ml;
        cw[r] = cosl(ang);
        sw[r] = (ld)sign * sinl(ang);
    }
    const int64_t nout = bins ? nb : Ml;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nout; ++q) {
        const int64_t h = bins ? bins[q] : q;
        ld re = 0.0L, im = 0.0L;
        int64_t r = 0; /* r = (j h) mod M, advanced by h each step */
        for (int64_t j = 0; j < Ml; ++j) {
            ld xr = x[2 * j], xi = x[2 * j + 1];
            re += xr * cw[r] - xi * sw[r];
            im += xr * sw[r] + xi * cw[r];
            r += h;
            if (r >= Ml) r -= Ml;
        }
        y[2 * q] = (double)(re / (ld)Ml);
        y[2 * q + 1] = (double)(im / (ld)Ml);
    }
    free(cw);
    free(sw);
}

void orc_dft(int32_t L, const int64_t *M, const double *f, double *ghat, int32_t sign)
{
    int64_t off = 0;
    for (int32_t l = 0; l < L; ++l) {
        dft_one(M[l], f + 2 * off, ghat + 2 * off, sign, 0, NULL);
        off += M[l];
    }
}

/* Selected bins of one lattice's normalised DFT. */
void orc_dft_bins(int64_t Ml, const double *fl, int64_t nb, const int64_t *bins,
                  double *out, int32_t sign)
{
    dft_one(Ml, fl, out, sign, nb, bins);
}

/* ------------------------------------------------------------------ */
/* Aliasing formula, eq. (2.4): for a trigonometric polynomial with     */
/* frequencies in S, the lattice rule returns in bucket h the sum of    */
/* the coefficients of every k in S with h_l(k) = h.  Written out as    */
/* that sum (long double accumulation, in candidate order).            */
/* ------------------------------------------------------------------ */
void orc_bucket_sums(int32_t d, int64_t n, const int64_t *freq, const double *coef,
                     int32_t L, const int64_t *M, const int64_t *z, double *out /* [sum M][2] */)
{
    int64_t off = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int64_t Ml = M[l];
        ld *acc = (ld *)calloc((size_t)Ml * 2, sizeof(ld));
        for (int64_t i = 0; i < n; ++i) {
            int64_t h = orc_hash_one(d, freq + i, n, z + (int64_t)l * d, Ml);
            acc[2 * h] += (ld)coef[2 * i];
            acc[2 * h + 1] += (ld)coef[2 * i + 1];
        }
        for (int64_t h = 0; h < Ml; ++h) {
            out[2 * (off + h)] = (double)acc[2 * h];
            out[2 * (off + h) + 1] = (double)acc[2 * h + 1];
        }
        free(acc);
        off += Ml;
    }
}

/* ------------------------------------------------------------------ */
/* Remark 2.3: the comparison with zero is a threshold test.           */
/* bucket is "non-zero" iff |ghat|^2 >= theta^2 (in double).           */
/* ------------------------------------------------------------------ */
static int nonzero(const double *g, double theta)
{
    double m2 = g[0] * g[0] + g[1] * g[1];
    return m2 >= theta * theta;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Median of L reals (eq. (2.10)); for even L the mean of the two middle
 * order statistics. */
static double median_of(double *v, int32_t L)
{
    qsort(v, (size_t)L, sizeof(double), cmp_double);
    if (L & 1) return v[L / 2];
    return 0.5 * (v[L / 2 - 1] + v[L / 2]);
}

typedef struct {
    double key;  /* |p|^2 */
    int64_t idx; /* candidate index */
    int64_t pos; /* position in the detected list */
} sel_t;

static int cmp_sel(const void *a, const void *b)
{
    const sel_t *x = (const sel_t *)a, *y = (const sel_t *)b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* ------------------------------------------------------------------ */
/* One call of the method for a fixed lattice configuration:          */
/*   Algorithm 2 (detection with vote threshold vote_min, which is    */
/*   ceil(nu L) of Algorithm 1; nu = 1/2 gives Algorithm 2), the      */
/*   median coefficients of eq. (2.10), the singleton post-processing  */
/*   of Remark 2.9 (optional), and the output limitation of           */
/*   Algorithm 4 (threshold theta, descending modulus, first s_cap).  */
/*                                                                    */
/* Inputs: candidates (d x n SoA), lattices, ghat (already the        */
/* normalised DFT of the samples).  Outputs (caller-allocated):        */
/*   votes[n]               number of lattices with a non-zero bucket  */
/*   det_idx[cap]           detected set, ascending candidate index    */
/*   det_med[cap][2]        median coefficient (eq. (2.10))            */
/*   det_mask[cap]          bit l set iff k is alone among the detected */
/*                          set in its bucket of lattice l (Remark 2.9) */
/*   det_coef[cap][2]       post-processed coefficient (or median)     */
/*   out_idx/out_coef/out_pos[s_cap]  Algorithm 4 output               */
/* Returns |detected|; only the first min(|detected|, cap) entries are */
/* written; *n_out gets the Algorithm 4 output size.                   */
/* ------------------------------------------------------------------ */
int64_t orc_extract(int32_t d, int64_t n, const int64_t *freq, int32_t L,
                    const int64_t *M, const int64_t *z, const double *ghat,
                    double theta, int32_t vote_min, int32_t postproc,
                    int64_t s_cap, int64_t cap,
                    uint8_t *votes, int64_t *det_idx, double *det_med,
                    uint64_t *det_mask, double *det_coef,
                    int64_t *n_out, int64_t *out_idx, double *out_coef,
                    int64_t *out_pos)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L + 1));
    off[0] = 0;
    for (int32_t l = 0; l < L; ++l) off[l + 1] = off[l] + M[l];

    /* Algorithm 2, detection loop: count non-zero buckets per candidate */
    uint8_t *v = votes ? votes : (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int32_t l = 0; l < L; ++l) {
            int64_t h = orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l]);
            c += nonzero(ghat + 2 * (off[l] + h), theta);
        }
        v[i] = (uint8_t)c;
    }
    int64_t ndet = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (v[i] >= vote_min) {
            if (ndet < cap) det_idx[ndet] = i;
            ndet++;
        }
    }
    const int64_t nd = ndet < cap ? ndet : cap;

    /* median of real and imaginary parts, eq. (2.10) */
    double *vals = (double *)malloc(sizeof(double) * (size_t)(nd > 0 ? nd : 1) * (size_t)L * 2);
    int64_t *hh = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nd > 0 ? nd : 1) * (size_t)L);
    for (int64_t q = 0; q < nd; ++q) {
        const int64_t i = det_idx[q];
        double re[64], im[64];
        for (int32_t l = 0; l < L; ++l) {
            int64_t h = orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l]);
            hh[q * L + l] = h;
            re[l] = ghat[2 * (off[l] + h)];
            im[l] = ghat[2 * (off[l] + h) + 1];
            vals[(q * L + l) * 2] = re[l];
            vals[(q * L + l) * 2 + 1] = im[l];
        }
        det_med[2 * q] = median_of(re, L);
        det_med[2 * q + 1] = median_of(im, L);
    }

    /* Remark 2.9: occupancy of every bucket by the detected set */
    int32_t *cnt = (int32_t *)calloc((size_t)off[L] + 1, sizeof(int32_t));
    for (int64_t q = 0; q < nd; ++q)
        for (int32_t l = 0; l < L; ++l) cnt[off[l] + hh[q * L + l]]++;
    for (int64_t q = 0; q < nd; ++q) {
        uint64_t mask = 0;
        ld sr = 0.0L, si = 0.0L;
        int32_t na = 0;
        for (int32_t l = 0; l < L; ++l) {
            if (cnt[off[l] + hh[q * L + l]] == 1) {
                mask |= 1ull << l;
                sr += vals[(q * L + l) * 2];
                si += vals[(q * L + l) * 2 + 1];
                na++;
            }
        }
        if (det_mask) det_mask[q] = mask;
        if (postproc && na > 0) {
            det_coef[2 * q] = (double)(sr / (ld)na);
            det_coef[2 * q + 1] = (double)(si / (ld)na);
        } else {
            det_coef[2 * q] = det_med[2 * q];
            det_coef[2 * q + 1] = det_med[2 * q + 1];
        }
    }

    /* Algorithm 4: keep |p| >= theta, sort by modulus descending (ties by
     * ascending candidate index), keep the first s_cap */
    sel_t *sel = (sel_t *)malloc(sizeof(sel_t) * (size_t)(nd > 0 ? nd : 1));
    int64_t ns = 0;
    for (int64_t q = 0; q < nd; ++q) {
        double m2 = det_coef[2 * q] * det_coef[2 * q] + det_coef[2 * q + 1] * det_coef[2 * q + 1];
        if (m2 >= theta * theta) {
            sel[ns].key = m2;
            sel[ns].idx = det_idx[q];
            sel[ns].pos = q;
            ns++;
        }
    }
    qsort(sel, (size_t)ns, sizeof(sel_t), cmp_sel);
    if (ns > s_cap) ns = s_cap;
    for (int64_t q = 0; q < ns; ++q) {
        out_idx[q] = sel[q].idx;
        out_pos[q] = sel[q].pos;
        out_coef[2 * q] = det_coef[2 * sel[q].pos];
        out_coef[2 * q + 1] = det_coef[2 * sel[q].pos + 1];
    }
    *n_out = ns;

    free(sel);
    free(cnt);
    free(hh);
    free(vals);
    if (!votes) free(v);
    free(off);
    return ndet;
}

/* ------------------------------------------------------------------ */
/* Linear map of the samples onto the extracted coefficients, for a    */
/* fixed support and fixed selections.                                 */
/*                                                                    */
/* With the detected set, the singleton masks of Remark 2.9 and the     */
/* order statistics chosen by the medians of eq. (2.10) held fixed,     */
/*   Re p_q = sum_l wr[q][l] Re ghat_l[h_l(k_q)],                       */
/*   Im p_q = sum_l wi[q][l] Im ghat_l[h_l(k_q)],                       */
/* and ghat_l is the normalised lattice DFT of Algorithm 2 line 2.      */
/* Singleton average: wr = wi = 1/|A_k| on A_k.  Median fallback:       */
/* weight 1 on the lattice holding the median order statistic (order    */
/* by value, ties by lattice index); for even L weight 1/2 on each of   */
/* the two middle order statistics.                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    double v;
    int32_t l;
} vl_t;

static int cmp_vl(const void *a, const void *b)
{
    const vl_t *x = (const vl_t *)a, *y = (const vl_t *)b;
    if (x->v < y->v) return -1;
    if (x->v > y->v) return 1;
    return (x->l > y->l) - (x->l < y->l);
}

void orc_weights(int32_t d, int64_t n, const int64_t *freq, int32_t L,
                 const int64_t *M, const int64_t *z, const double *ghat,
                 int64_t nd, const int64_t *det_idx, const uint64_t *det_mask,
                 int32_t postproc, double *w /* [nd][L][2] */)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L + 1));
    off[0] = 0;
    for (int32_t l = 0; l < L; ++l) off[l + 1] = off[l] + M[l];
    for (int64_t q = 0; q < nd; ++q) {
        double *wq = w + q * L * 2;
        for (int32_t l = 0; l < 2 * L; ++l) wq[l] = 0.0;
        uint64_t mask = det_mask[q];
        int32_t na = 0;
        for (int32_t l = 0; l < L; ++l) na += (int32_t)((mask >> l) & 1u);
        if (postproc && na > 0) {
            for (int32_t l = 0; l < L; ++l)
                if ((mask >> l) & 1u) {
                    wq[2 * l] = 1.0 / na;
                    wq[2 * l + 1] = 1.0 / na;
                }
            continue;
        }
        for (int32_t part = 0; part < 2; ++part) {
            vl_t vs[64];
            for (int32_t l = 0; l < L; ++l) {
                int64_t h = orc_hash_one(d, freq + det_idx[q], n, z + (int64_t)l * d, M[l]);
                vs[l].v = ghat[2 * (off[l] + h) + part];
                vs[l].l = l;
            }
            qsort(vs, (size_t)L, sizeof(vl_t), cmp_vl);
            if (L & 1) {
                wq[2 * vs[L / 2].l + part] = 1.0;
            } else {
                wq[2 * vs[L / 2 - 1].l + part] += 0.5;
                wq[2 * vs[L / 2].l + part] += 0.5;
            }
        }
    }
    free(off);
}

/* Transpose of that real-linear map, applied element by element:
 *   grad_f_l[j] = (1/M_l) sum_{q} e^{+2 pi i j h_l(k_q) / M_l}
 *                          (wr[q][l] Re g_q + i wi[q][l] Im g_q)
 * (the real transpose of Re/Im-weighted gathers of a normalised DFT). */
void orc_adjoint(int32_t d, int64_t n, const int64_t *freq, int32_t L,
                 const int64_t *M, const int64_t *z, int64_t nd,
                 const int64_t *det_idx, const double *w /* [nd][L][2] */,
                 const double *grad /* [nd][2] */, double *grad_f /* [sum M][2] */)
{
    int64_t off = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int64_t Ml = M[l];
        int64_t *h = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nd > 0 ? nd : 1));
        for (int64_t q = 0; q < nd; ++q)
            h[q] = orc_hash_one(d, freq + det_idx[q], n, z + (int64_t)l * d, Ml);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < Ml; ++j) {
            ld re = 0.0L, im = 0.0L;
            for (int64_t q = 0; q < nd; ++q) {
                ld a = (ld)w[(q * L + l) * 2] * (ld)grad[2 * q];
                ld b = (ld)w[(q * L + l) * 2 + 1] * (ld)grad[2 * q + 1];
                int64_t r = (int64_t)(((__int128)j * h[q]) % Ml);
                ld ang = TWO_PI_L * (ld)r / (ld)Ml;
                ld c = cosl(ang), sn = sinl(ang);
                re += a * c - b * sn;
                im += a * sn + b * c;
            }
            grad_f[2 * (off + j)] = (double)(re / (ld)Ml);
            grad_f[2 * (off + j) + 1] = (double)(im / (ld)Ml);
        }
        free(h);
        off += Ml;
    }
}

/* ------------------------------------------------------------------ */
/* Counter-based random numbers: the SplitMix64 generator of Steele,   */
/* Lea and Flood (OOPSLA 2014).  Its n-th output (n >= 1) from seed S  */
/* is mix(S + n * 0x9E3779B97F4A7C15) with the published finaliser     */
/*   z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;                             */
/*   z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31.               */
/* A draw stream (seed, t, i) of the driver reads outputs                */
/*   n = ((t * 64 + i) << 24) + c + 1,  c = 0, 1, 2, ...                */
/* Uniform integer in [0, m): floor(x * m / 2^64) (multiply-shift).     */
/* Uniform 32-bit anchor numerator: x >> 32.                            */
/* ------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t x = seed + n * 0x9E3779B97F4A7C15ULL;
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ULL;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return x;
}

static uint64_t stream_draw(uint64_t seed, int32_t t, int32_t i, uint64_t c)
{
    uint64_t n = ((((uint64_t)t * 64u) + (uint64_t)i) << 24) + c + 1u;
    return orc_splitmix64(seed, n);
}

/* Step 1 of the driver draws from a second family of streams:          */
/*   n = 2^62 + ((t * 64 + i) << 24) + c + 1 (t = coordinate, 1-based).  */
static uint64_t stream1_draw(uint64_t seed, int32_t t, int32_t i, uint64_t c)
{
    uint64_t n = (1ULL << 62) + ((((uint64_t)t * 64u) + (uint64_t)i) << 24) + c + 1u;
    return orc_splitmix64(seed, n);
}

/* ------------------------------------------------------------------ */
/* The test function of eq. (4.3) (Sec. 4.2.3): sums of tensor products */
/* of the periodic B-splines                                            */
/*   N_m(x) = C_m sum_k sinc(pi k / m)^m (-1)^k e^{2 pi i k x}.          */
/* The series equals C_m m B_m(m x) on [0, 1), B_m the cardinal         */
/* B-spline of order m with knots 0..m, evaluated here by its           */
/* truncated-power form                                                 */
/*   B_m(y) = (1/(m-1)!) sum_{j=0}^{m} (-1)^j binom(m, j) (y - j)_+^{m-1}. */
/* C_m makes ||N_m||_2 = 1; by Parseval C_m^-2 = sum_k sinc(pi k/m)^{2m}, */
/* summed directly (terms decay like k^{-2m}).                         */
/* ------------------------------------------------------------------ */
static ld trunc_power_bspline(int32_t m, ld y)
{
    if (y < 0 || y >= m) return 0;
    ld s = 0, binom = 1, fact = 1;
    for (int32_t j = 2; j < m; ++j) fact *= j;
    for (int32_t j = 0; j <= m; ++j) {
        if (y >= j) {
            ld pw = 1;
            for (int32_t e = 0; e < m - 1; ++e) pw *= (y - j);
            s += ((j & 1) ? -binom : binom) * pw;
        }
        binom = binom * (m - j) / (j + 1);
    }
    return s / fact;
}

static ld bspline_norm_const(int32_t m)
{
    static ld cache[33];
    if (m >= 1 && m <= 32 && cache[m] > 0) return cache[m];
    ld acc = 1;   /* k = 0 */
    for (int64_t k = 1; k <= 200000; ++k) {
        const ld x = (ld)3.14159265358979323846264338327950288L * (ld)k / (ld)m;
        const ld sc = sinl(x) / x;
        ld p = 1;
        for (int32_t e = 0; e < 2 * m; ++e) p *= sc;
        acc += 2 * p;
    }
    const ld c = 1 / sqrtl(acc);
    if (m >= 1 && m <= 32) cache[m] = c;
    return c;
}

/* N_m(x) for any real x (period 1). */
ld orc_bspline_periodic(int32_t m, ld x)
{
    x = x - floorl(x);
    return bspline_norm_const(m) * (ld)m * trunc_power_bspline(m, (ld)m * x);
}

/* Samples of f(x) = sum_j prod_{u in S_j} N_{m_j}(x_u) at the nodes of L   */
/* lattices in t coordinates (x_u = j z_u / M mod 1, u < t) with anchors   */
/* x_u = anchor[u - t] / 2^32 (u = t..d_poly-1); dims[j] has bit u set iff */
/* u is in S_j.  f: complex [sum M] (imaginary parts zero).                 */
void orc_sample_bspline(int32_t t, int32_t d_poly, int32_t n_prod, const int32_t *order,
                        const uint64_t *dims, const uint32_t *anchor, int32_t L, const int64_t *M,
                        const int64_t *z, double *f)
{
    for (int32_t q = 0; q < n_prod; ++q) (void)bspline_norm_const(order[q]);   /* fill the cache serially */
    int64_t off = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int64_t Ml = M[l];
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < Ml; ++j) {
            ld acc = 0;
            for (int32_t q = 0; q < n_prod; ++q) {
                ld prod = 1;
                for (int32_t u = 0; u < d_poly; ++u) {
                    if (!((dims[q] >> u) & 1u)) continue;
                    ld x;
                    if (u < t) x = (ld)floor_mod_i128((__int128)j * z[(int64_t)l * t + u], Ml) / (ld)Ml;
                    else x = (ld)anchor[u - t] / 4294967296.0L;
                    prod *= orc_bspline_periodic(order[q], x);
                }
                acc += prod;
            }
            f[2 * (off + j)] = (double)acc;
            f[2 * (off + j) + 1] = 0.0;
        }
        off += Ml;
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 3, Step 1 (single frequency component identification) for  */
/* coordinate t (1-based) over the range [-N, N] (K = 2N + 1):           */
/* r times: anchors x'_j = a_j / 2^32 for j != t (drawn in ascending j  */
/* from stream1 (t, i)), samples p at x_t = l / K, l < K, the           */
/* normalised length-K DFT, and the frequencies k_t in [-N, N] among   */
/* the s_local largest |p~_{t,k_t}| with |p~| >= theta (ties: smaller  */
/* k_t first); I^(t) is the union, returned sorted in set[], size      */
/* returned.  *samples grows by r K.                                   */
/* ------------------------------------------------------------------ */
static int64_t step1_set(int32_t d, int32_t t, int64_t N, int64_t s_poly, const int64_t *poly_freq,
                         const double *poly_coef, int32_t bs_n, const int32_t *bs_order,
                         const uint64_t *bs_dims, int64_t s_local, int32_t r, double theta,
                         uint64_t seed, int64_t *set, int64_t *samples)
{
    const int64_t K = 2 * N + 1;
    /* the polynomial's coordinates with t moved to the front */
    int64_t *pf = (int64_t *)malloc(sizeof(int64_t) * (size_t)d * (size_t)(s_poly > 0 ? s_poly : 1));
    for (int64_t q = 0; q < s_poly; ++q) {
        pf[q] = poly_freq[(int64_t)(t - 1) * s_poly + q];
        int32_t row = 1;
        for (int32_t u = 0; u < d; ++u)
            if (u != t - 1) pf[(int64_t)(row++) * s_poly + q] = poly_freq[(int64_t)u * s_poly + q];
    }
    char *in = (char *)calloc((size_t)K, 1);
    double *f = (double *)malloc(sizeof(double) * 2 * (size_t)K);
    double *g = (double *)malloc(sizeof(double) * 2 * (size_t)K);
    struct key { double m2; int64_t idx; } *keys = malloc(sizeof(struct key) * (size_t)K);
    uint32_t *anc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)d);
    const int64_t one = 1;

    for (int32_t i = 1; i <= r; ++i) {
        uint64_t cnt = 0;
        for (int32_t j = 0; j < d - 1; ++j) anc[j] = (uint32_t)(stream1_draw(seed, t, i, cnt++) >> 32);
        if (bs_n > 0) {
            /* the test function on the line: x_t = l / K, the other coordinates anchored */
            for (int32_t q = 0; q < bs_n; ++q) (void)bspline_norm_const(bs_order[q]);
            for (int64_t l = 0; l < K; ++l) {
                ld acc = 0;
                for (int32_t q = 0; q < bs_n; ++q) {
                    ld prod = 1;
                    for (int32_t u = 0; u < d; ++u) {
                        if (!((bs_dims[q] >> u) & 1u)) continue;
                        const ld x = (u == t - 1) ? (ld)l / (ld)K
                                                  : (ld)anc[u < t - 1 ? u : u - 1] / 4294967296.0L;
                        prod *= orc_bspline_periodic(bs_order[q], x);
                    }
                    acc += prod;
                }
                f[2 * l] = (double)acc;
                f[2 * l + 1] = 0.0;
            }
        } else {
            orc_sample(d, 1, s_poly, pf, poly_coef, anc, 1, &K, &one, f);
        }
        *samples += K;
        orc_dft(1, &K, f, g, -1);
        int64_t nk = 0;
        for (int64_t k = -N; k <= N; ++k) {
            const int64_t h = ((k % K) + K) % K;
            const double m2 = g[2 * h] * g[2 * h] + g[2 * h + 1] * g[2 * h + 1];
            if (m2 >= theta * theta) { keys[nk].m2 = m2; keys[nk].idx = k + N; nk++; }
        }
        /* the s_local largest moduli, ties by smaller frequency (selection by repeated maxima) */
        for (int64_t q = 0; q < s_local && q < nk; ++q) {
            int64_t b = q;
            for (int64_t x = q + 1; x < nk; ++x)
                if (keys[x].m2 > keys[b].m2 || (keys[x].m2 == keys[b].m2 && keys[x].idx < keys[b].idx)) b = x;
            struct key tmp = keys[q]; keys[q] = keys[b]; keys[b] = tmp;
            in[keys[q].idx] = 1;
        }
    }
    int64_t n = 0;
    for (int64_t a = 0; a < K; ++a)
        if (in[a]) set[n++] = a - N;
    free(anc); free(keys); free(g); free(f); free(in); free(pf);
    return n;
}

static int64_t uniform_below(uint64_t x, int64_t m)
{
    return (int64_t)(((unsigned __int128)x * (unsigned __int128)(uint64_t)m) >> 64);
}

/* Number of lattices of eq. (4.2): the smallest odd n with
 *   n >= (1/4) * 4c / ((c - 2) ln(c - 1)) * (ln |J| - ln delta). */
int32_t orc_num_lattices_eq42(int64_t nJ, double c, double delta)
{
    double bound = 0.25 * (4.0 * c / ((c - 2.0) * log(c - 1.0))) * (log((double)nJ) - log(delta));
    int32_t L = (int32_t)ceil(bound);
    if (L < 1) L = 1;
    if ((L & 1) == 0) L++;
    return L;
}

/* Lexicographic comparison of t-tuples stored row-wise. */
static int32_t g_cmp_t;
static int cmp_tuple(const void *a, const void *b)
{
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    for (int32_t u = 0; u < g_cmp_t; ++u) {
        if (x[u] < y[u]) return -1;
        if (x[u] > y[u]) return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 3, Step 2 (coupling of frequency components), with         */
/* Algorithm 4 in the role of Algorithm A, for a sparse trigonometric   */
/* polynomial given by its d x s frequencies and coefficients, or       */
/* (bs_n > 0) the test function of eq. (4.3) given by its products.     */
/* The single-coordinate sets I^(t) come from Step 1 (step1 != 0) or   */
/* are the full one-dimensional range [-N, N]; the output of the t = d  */
/* call is the result (the external Step 3 is not part of this method). */
/*                                                                     */
/* For t = 2..d and i = 1..r~ (r~ = r for t < d, 1 for t = d;           */
/* s~ = s_local for t < d, s for t = d):                                 */
/*   J_t  = I^(1..t-1) x I^(t) (lexicographic order),                   */
/*   L    = eq. (4.2) on |J_t|, every lattice of size Mlat,             */
/*   draws: anchors a_u (u = t..d-1), then z_{l,u} (l < L, u < t),       */
/*   samples at the t-dimensional lattice nodes with anchors,           */
/*   normalised DFT, Algorithm 4 on J_t, union into I^(1..t).           */
/* Output: final tuples out_freq[q*d + u] (row-wise), out_coef[q][2],   */
/* sorted lexicographically; returns the output size, or -1 when a      */
/* capacity is exceeded.  *total_samples gets sum over calls of L*Mlat.  */
/* ------------------------------------------------------------------ */
int64_t orc_dimincr(int32_t d, int64_t N, int64_t s_poly, const int64_t *poly_freq,
                    const double *poly_coef, int32_t bs_n, const int32_t *bs_order,
                    const uint64_t *bs_dims, int64_t s, int64_t s_local, int32_t r,
                    double theta, double c, double delta, int64_t Mlat,
                    int32_t postproc, uint64_t seed, int64_t cap_set, int32_t step1,
                    int64_t *out_freq, double *out_coef, int64_t *total_samples)
{
    const int64_t K = 2 * N + 1;
    int64_t samples = 0;
    /* single-coordinate sets I^(t): Step 1, or the whole range [-N, N] */
    int64_t *I1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)d * (size_t)K);
    int64_t *n1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)d);
    for (int32_t t = 1; t <= d; ++t) {
        if (step1) {
            n1[t - 1] = step1_set(d, t, N, s_poly, poly_freq, poly_coef, bs_n, bs_order, bs_dims, s_local, r,
                                  theta, seed,
                                  I1 + (int64_t)(t - 1) * K, &samples);
        } else {
            for (int64_t a = 0; a < K; ++a) I1[(int64_t)(t - 1) * K + a] = a - N;
            n1[t - 1] = K;
        }
    }
    int64_t nprev = n1[0];               /* |I^(1..t-1)| */
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap_set * (size_t)d);
    for (int64_t a = 0; a < nprev; ++a) prev[a] = I1[a]; /* I^(1) */
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap_set * (size_t)d);
    int64_t nout_final = 0;

    for (int32_t t = 2; t <= d && nprev > 0; ++t) {
        const int32_t rt = (t < d) ? r : 1;
        const int64_t st = (t < d) ? s_local : s;
        const int64_t Kt = n1[t - 1];
        const int64_t *It = I1 + (int64_t)(t - 1) * K;
        const int64_t nJ = nprev * Kt;
        if (nJ == 0) { nprev = 0; break; }
        /* J_t = I^(1..t-1) x I^(t) as SoA [t][nJ], lexicographic */
        int64_t *J = (int64_t *)malloc(sizeof(int64_t) * (size_t)nJ * (size_t)t);
        for (int64_t a = 0; a < nprev; ++a)
            for (int64_t b = 0; b < Kt; ++b) {
                int64_t q = a * Kt + b;
                for (int32_t u = 0; u < t - 1; ++u) J[(int64_t)u * nJ + q] = prev[a * (t - 1) + u];
                J[(int64_t)(t - 1) * nJ + q] = It[b];
            }
        const int32_t L = orc_num_lattices_eq42(nJ, c, delta);
        int64_t *Ms = (int64_t *)malloc(sizeof(int64_t) * (size_t)L);
        for (int32_t l = 0; l < L; ++l) Ms[l] = Mlat;
        const int64_t SM = (int64_t)L * Mlat;
        int64_t ncur = 0;

        for (int32_t i = 1; i <= rt; ++i) {
            uint64_t cnt = 0;
            uint32_t *anc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(d - t + 1));
            for (int32_t u = t; u < d; ++u) anc[u - t] = (uint32_t)(stream_draw(seed, t, i, cnt++) >> 32);
            int64_t *zz = (int64_t *)malloc(sizeof(int64_t) * (size_t)L * (size_t)t);
            for (int32_t l = 0; l < L; ++l)
                for (int32_t u = 0; u < t; ++u)
                    zz[(int64_t)l * t + u] = uniform_below(stream_draw(seed, t, i, cnt++), Mlat);

            double *f = (double *)malloc(sizeof(double) * 2 * (size_t)SM);
            double *g = (double *)malloc(sizeof(double) * 2 * (size_t)SM);
            if (bs_n > 0) orc_sample_bspline(t, d, bs_n, bs_order, bs_dims, anc, L, Ms, zz, f);
            else orc_sample(d, t, s_poly, poly_freq, poly_coef, anc, L, Ms, zz, f);
            samples += SM;
            orc_dft(L, Ms, f, g, -1);

            const int64_t cap = nJ;
            int64_t *det_idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
            double *det_med = (double *)malloc(sizeof(double) * 2 * (size_t)cap);
            uint64_t *det_mask = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cap);
            double *det_coef = (double *)malloc(sizeof(double) * 2 * (size_t)cap);
            int64_t *out_idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(st > 0 ? st : 1));
            int64_t *out_pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(st > 0 ? st : 1));
            double *oc = (double *)malloc(sizeof(double) * 2 * (size_t)(st > 0 ? st : 1));
            int64_t nsel = 0;
            orc_extract(t, nJ, J, L, Ms, zz, g, theta, (L + 1) / 2, postproc, st, cap,
                        NULL, det_idx, det_med, det_mask, det_coef, &nsel, out_idx, oc, out_pos);
            /* Step 2d: union */
            for (int64_t q = 0; q < nsel; ++q) {
                if (ncur >= cap_set) { ncur = -1; break; }
                for (int32_t u = 0; u < t; ++u) cur[ncur * t + u] = J[(int64_t)u * nJ + out_idx[q]];
                ncur++;
            }
            if (t == d && ncur >= 0) {
                for (int64_t q = 0; q < nsel; ++q) {
                    out_coef[2 * q] = oc[2 * q];
                    out_coef[2 * q + 1] = oc[2 * q + 1];
                }
            }
            free(out_idx); free(out_pos); free(oc);
            free(det_idx); free(det_med); free(det_mask); free(det_coef);
            free(f); free(g); free(zz); free(anc);
            if (ncur < 0) break;
        }
        free(Ms);
        free(J);
        if (ncur < 0) { free(prev); free(cur); free(I1); free(n1); return -1; }

        if (t == d) {
            /* sort final tuples (with their coefficients) lexicographically */
            int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncur > 0 ? ncur : 1) * (size_t)(d + 1));
            for (int64_t q = 0; q < ncur; ++q) {
                for (int32_t u = 0; u < d; ++u) rows[q * (d + 1) + u] = cur[q * d + u];
                rows[q * (d + 1) + d] = q;
            }
            g_cmp_t = d;
            qsort(rows, (size_t)ncur, sizeof(int64_t) * (size_t)(d + 1), cmp_tuple);
            double *cc = (double *)malloc(sizeof(double) * 2 * (size_t)(ncur > 0 ? ncur : 1));
            memcpy(cc, out_coef, sizeof(double) * 2 * (size_t)ncur);
            for (int64_t q = 0; q < ncur; ++q) {
                for (int32_t u = 0; u < d; ++u) out_freq[q * d + u] = rows[q * (d + 1) + u];
                int64_t src = rows[q * (d + 1) + d];
                out_coef[2 * q] = cc[2 * src];
                out_coef[2 * q + 1] = cc[2 * src + 1];
            }
            free(cc);
            free(rows);
            nout_final = ncur;
        } else {
            /* I^(1..t): sorted, duplicates removed */
            g_cmp_t = t;
            qsort(cur, (size_t)ncur, sizeof(int64_t) * (size_t)t, cmp_tuple);
            int64_t m = 0;
            for (int64_t q = 0; q < ncur; ++q) {
                if (m > 0 && cmp_tuple(cur + (m - 1) * t, cur + q * t) == 0) continue;
                if (m != q) memmove(cur + m * t, cur + q * t, sizeof(int64_t) * (size_t)t);
                m++;
            }
            int64_t *tmp = prev; prev = cur; cur = tmp;
            nprev = m;
            if (nprev == 0) break;   /* nothing detected: the result is empty */
        }
    }
    free(prev);
    free(cur);
    free(I1);
    free(n1);
    if (total_samples) *total_samples = samples;
    return nout_final;
}

/* ------------------------------------------------------------------ */
/* Worst-case aliasing classification of Section 4.1.1 (Table 4.1).   */
/* The method is applied to the counting polynomial of eq. (4.1):     */
/* all-ones coefficients on the support I.  By the aliasing formula   */
/* eq. (2.4) the lattice-l value at k's bucket is the number of       */
/* members of I in that bucket; its median over the lattices          */
/* (eq. (2.10)) classifies k:                                         */
/*   k in I:      median > 1  ->  potential false negative (PFN);     */
/*   k not in I:  median > 0  ->  potential false positive (PFP).     */
/* The candidates [0, n_active) are I.  The detected set of the       */
/* method is then I together with the PFPs.  In the post-processing   */
/* of Remark 2.9 a PFP is removed iff some lattice puts it alone      */
/* among the detected set in its bucket: such a bucket holds no       */
/* member of I, so the recovered coefficient is zero.                 */
/* cls[i]: bit 0 PFP, bit 1 PFN, bit 2 PFP kept by post-processing.   */
/* ------------------------------------------------------------------ */
void orc_pfpn(int32_t d, int64_t n, const int64_t *freq, int64_t n_active, int32_t L,
              const int64_t *M, const int64_t *z, uint8_t *cls)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L + 1));
    off[0] = 0;
    for (int32_t l = 0; l < L; ++l) off[l + 1] = off[l] + M[l];
    int32_t *cnt = (int32_t *)calloc((size_t)off[L], sizeof(int32_t));
    for (int32_t l = 0; l < L; ++l)
        for (int64_t i = 0; i < n_active; ++i)
            cnt[off[l] + orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l])]++;
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * (size_t)L);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            for (int32_t l = 0; l < L; ++l)
                v[l] = (double)cnt[off[l] + orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l])];
            const double med = median_of(v, L);
            cls[i] = (uint8_t)(i < n_active ? (med > 1.0 ? 2 : 0) : (med > 0.0 ? 1 : 0));
        }
        free(v);
    }
    /* occupancy by the detected set I u PFP */
    int32_t *cd = (int32_t *)calloc((size_t)off[L], sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        if (i >= n_active && !(cls[i] & 1)) continue;
        for (int32_t l = 0; l < L; ++l)
            cd[off[l] + orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l])]++;
    }
    for (int64_t i = n_active; i < n; ++i) {
        if (!(cls[i] & 1)) continue;
        int alone = 0;
        for (int32_t l = 0; l < L && !alone; ++l)
            alone = cd[off[l] + orc_hash_one(d, freq + i, n, z + (int64_t)l * d, M[l])] == 1;
        if (!alone) cls[i] |= 4;
    }
    free(cd);
    free(cnt);
    free(off);
}
