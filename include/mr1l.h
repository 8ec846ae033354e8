/*
 * mr1l.h -- C ABI of the MI355X (gfx950) multiple-rank-1-lattice sparse FFT.
 *
 * Method: Kaemmerer, Krahmer, Volkmer, "A sample efficient sparse FFT for
 * arbitrary frequency candidate sets in high dimensions" (arXiv:2006.13053).
 * The library computes, on one GPU, the step the paper builds everything on:
 * samples of a function on L random rank-1 lattices (eq. (2.1)), one
 * normalised length-M_l DFT per lattice (Algorithm 2, first loop), the bucket
 * h_l(k) = k . z_l mod M_l of every candidate frequency (Section 2.2 and
 * the "Gamma mod M" representative of Section 2.1), the non-zero vote of
 * Algorithms 1 and 2 with the threshold test of Remark 2.3, the median
 * coefficients of eq. (2.10), the singleton ("alias-free") averaging of
 * Remark 2.9, the output limitation of Algorithm 4, the adjoint of the
 * coefficient map, and the dimension-incremental Step 2 of Algorithm 3.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - A plan describes a batch of F >= 1 functions with the same number of
 *    lattice dimensions d and the same number of lattices L per function.
 *    F = 1 is the plain method.  Lattice (f, l) has prime size M[f*L + l]
 *    and generating vector z[(f*L + l)*d + u], 0 <= z < M.
 *  - Nodes.  Samples f, DFT values ghat, bucket counts and the non-zero
 *    bitmap are concatenated over (f, l) in that order: lattice (f, l)
 *    occupies nodes [O_{f,l}, O_{f,l} + M_{f,l}), O the running sum of the
 *    sizes.  mr1l_plan_nodes() returns the total.  Bitmap bit g of node g
 *    lives in word g / 32, bit g % 32.
 *  - Candidate sets are structure-of-arrays int64: freq[u * n_total + i] is
 *    coordinate u of candidate i (u < d).  Function f owns candidates
 *    [set_off[f], set_off[f+1]); set_off is a DEVICE array of F + 1 int64
 *    (may be NULL when F == 1, meaning [0, n_total)).  Indices written by
 *    the library (det_idx, out_idx) are relative to the function's own
 *    range.  Any int64 frequency is hashed exactly.
 *  - Complex arrays are interleaved (re, im) in the plan's dtype:
 *    MR1L_C128 = double, MR1L_C64 = float.
 *  - Every pointer argument marked "dev" is device memory owned by the
 *    caller; "host" is host memory owned by the caller and read before the
 *    call returns.  The plan owns only its tables and scratch.
 *  - Calls are asynchronous on the plan's stream and never synchronise
 *    unless stated; sizes produced on the device (detected counts) stay in
 *    device memory, so a sequence of calls can be captured in a HIP graph.
 *  - Errors are status codes (MR1L_OK = 0, negative on error); no C++
 *    exception crosses the ABI.  mr1l_last_error() returns a message for
 *    the calling thread's last failure.  A plan is not thread-safe; distinct
 *    plans are independent.
 */
#ifndef MR1L_H
#define MR1L_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MR1L_C64 = 1, MR1L_C128 = 2 };

enum {
    MR1L_OK = 0,
    MR1L_E_ARG = -1,          /* invalid argument (size, pointer, range)        */
    MR1L_E_NOT_PRIME = -2,    /* a lattice size is not prime (Section 2.1)     */
    MR1L_E_OVERFLOW = -3,     /* a size would overflow the index types          */
    MR1L_E_NOT_INJECTIVE = -4,/* candidate set not injective mod M (Section 2.1)*/
    MR1L_E_CAPACITY = -5,     /* an output capacity is too small               */
    MR1L_E_NOMEM = -6,        /* device allocation failed                      */
    MR1L_E_HIP = -7           /* a HIP runtime call failed                     */
};

typedef struct mr1l_plan_s *mr1l_plan;

/* Version of the library (major * 10000 + minor * 100 + patch). */
int mr1l_version(void);

/* Message of the calling thread's last error ("" if none). */
const char *mr1l_last_error(void);

/*
 * Create a plan for F functions of d lattice dimensions with L lattices each
 * (the multiple rank-1 lattice configuration of Section 2.1); 1 <= d <= 64,
 * 1 <= F <= 2^20, 1 <= L <= 64.
 *   M     host [F*L]   lattice sizes; each must be a prime (checked with a
 *                      deterministic Miller-Rabin test) with 2 <= M < 2^23.
 *   z     host [F*L*d] generating vectors, 0 <= z < M (checked).
 *   dtype MR1L_C128 or MR1L_C64.
 *   stream hipStream_t (as void*) the plan's calls are ordered on; NULL is
 *          the default stream.
 * The plan precomputes the Bluestein chirps, kernel spectra and twiddle
 * tables of the per-lattice DFTs and the constants of the exact bucket
 * hash, and allocates its scratch.  The tables are uploaded and the spectra
 * computed on `stream` without waiting for it (spectra of another DFT
 * schedule are computed when a size is switched to it).  Returns
 * MR1L_E_NOT_PRIME, MR1L_E_ARG, MR1L_E_NOMEM or MR1L_E_HIP on failure (*out
 * is then NULL).
 */
int mr1l_plan_create(mr1l_plan *out, int32_t d, int32_t F, int32_t L,
                     const int64_t *M, const int64_t *z, int32_t dtype,
                     void *stream);

/*
 * Waits for the plan's stream and releases the plan.  Its device memory
 * goes to a per-device cache of blocks that later plans (and the
 * dimension-incremental driver) reuse, so that a loop creating and
 * destroying plans does not pay hipMalloc/hipFree each time (a request
 * takes a cached block of up to twice its size); the cache holds at most an
 * eighth of the device's memory, and an allocation that fails empties it
 * and retries.
 */
int mr1l_plan_destroy(mr1l_plan p);

/* Frees the cached device blocks of the current device (plans in use keep
 * theirs).  Not to be called while another thread creates or grows a plan
 * on the same device. */
int mr1l_release_cache(void);

/* Total number of nodes (sum of all M); sizes f, ghat, counts. */
int64_t mr1l_plan_nodes(mr1l_plan p);

/* Replace the plan's stream (the next calls are ordered on it, after the
 * work queued so far on the old one). */
int mr1l_plan_set_stream(mr1l_plan p, void *stream);

/* Replace the generating vectors (host [F*L*d], same M), keeping the DFT
 * tables; used when new random lattices of the same sizes are drawn. */
int mr1l_plan_set_z(mr1l_plan p, const int64_t *z);

/*
 * Sample a sparse trigonometric polynomial (eq. (2.2)) at the lattice nodes
 * x_j = j z_l / M_l mod 1 (eq. (2.1)).
 *   d_poly   number of coordinates of the polynomial's frequencies, >= d.
 *            The lattice sets coordinates u < d; coordinates d <= u < d_poly
 *            are fixed anchors x'_u = anchor[f*(d_poly-d) + u-d] / 2^32 for
 *            all nodes of function f (the embedding of Algorithm 3,
 *            Step 2a).
 *   term_off dev [F+1] or NULL (F == 1): function f's terms are
 *            [term_off[f], term_off[f+1]).
 *   n_terms  total number of terms.
 *   freq     dev [d_poly][n_terms] int64;  coef dev [n_terms] complex.
 *   anchor   dev uint32 [F][d_poly-d], or NULL when d_poly == d.
 *   f        dev [nodes] complex output.
 *   mode     0 = automatic, 1 = direct sum over terms per node (exact
 *            integer phases), 2 = bucket sums (eq. (2.4)) followed by an
 *            inverse lattice DFT; for many terms per node.
 */
int mr1l_sample(mr1l_plan p, int32_t d_poly, const int64_t *term_off,
                int64_t n_terms, const int64_t *freq, const void *coef,
                const uint32_t *anchor, void *f, int32_t mode);

/*
 * mr1l_sample for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and results, but the term scratch (anchored
 * coefficients and buckets, n_terms * (w + 4 L) bytes, w = 16 for complex128
 * and 8 for complex64, plus up to 255 bytes of alignment) lives in a static
 * 64 MiB array that the library holds on every device it runs on until the
 * process ends.  The call allocates nothing and does not synchronise.
 *   term_off is required (dev [F+1]), also when F == 1.
 * Errors: MR1L_E_CAPACITY when the term scratch would exceed 64 MiB (nothing is
 * launched), and the argument errors of mr1l_sample.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (several streams or threads) race; order them.
 */
int mr1l_sample_noalloc(mr1l_plan p, int32_t d_poly, const int64_t *term_off,
                        int64_t n_terms, const int64_t *freq, const void *coef,
                        const uint32_t *anchor, void *f, int32_t mode);

/*
 * Samples of a sum of tensor products of periodic B-splines, the kind of test
 * function of eq. (4.3) (Section 4.2.3):
 *   f(x) = sum_{j < n_prod} prod_{u in S_j} N_{m_j}(x_u),
 *   N_m(x) = C_m sum_k sinc(pi k / m)^m (-1)^k e^{2 pi i k x},  ||N_m||_2 = 1,
 * at the plan's lattice nodes, coordinates u < d from the lattice and
 * u >= d fixed anchors x'_u = anchor[f*(d_poly-d) + u-d] / 2^32, as in
 * mr1l_sample.  On [0, 1), N_m(x) = C_m m B_m(m x) with the cardinal B-spline
 * B_m of order m (knots 0..m) and C_m = (m B_2m(m))^{-1/2}.
 *   d_poly   coordinates of the function, d <= d_poly <= 64;
 *   n_prod   1..16 products; order host int32 [n_prod], 1 <= m_j <= 16;
 *   dims     host uint64 [F][n_prod]: bit u set iff coordinate u (in the
 *            order above) belongs to S_j for function f;
 *   anchor   dev uint32 [F][d_poly-d] (NULL when d_poly == d);
 *   f        dev [nodes] complex output (imaginary parts zero).
 * Synchronises the plan's stream before returning (the masks are copied).
 */
int mr1l_sample_bspline(mr1l_plan p, int32_t d_poly, int32_t n_prod,
                        const int32_t *order, const uint64_t *dims,
                        const uint32_t *anchor, void *f);

/*
 * Normalised lattice DFT of Algorithm 2 (first loop):
 *   ghat[O + h] = (1/M) sum_{j<M} f[O + j] exp(-2 pi i j h / M), h < M,
 * for every lattice (Bluestein's chirp transform with LDS-staged Stockham
 * FFTs), and the non-zero test of Remark 2.3 as a bitmap:
 *   bit (O + h) of nz_bitmap = (|ghat[O+h]|^2 >= theta^2).
 *   f, ghat   dev [nodes] complex (may not alias);
 *   nz_bitmap dev uint32 [ceil(nodes/32)] or NULL.
 */
int mr1l_fft(mr1l_plan p, const void *f, void *ghat, double theta,
             uint32_t *nz_bitmap);

/*
 * Buckets and bucket occupancy of a frequency set S:
 *   hash[l * n_total + i] = h_{f,l}(k_i)  (i in function f's range),
 *   counts[O_{f,l} + h]   = #{k in S_f : h_{f,l}(k) = h}
 * (the occupancy behind Remark 2.9 and the counting polynomial of
 * eq. (4.1)).  Either output may be NULL; counts is overwritten.
 */
int mr1l_hash_count(mr1l_plan p, int64_t n_total, const int64_t *set_off,
                    const int64_t *freq, int32_t *hash, int32_t *counts);

/* Options of mr1l_extract. */
typedef struct {
    double theta;      /* threshold of Remark 2.3 and Algorithm 4 (>= 0)      */
    int32_t vote_min;  /* keep k iff #non-zero buckets >= vote_min; 0 means
                          ceil(L/2), i.e. Algorithm 2 (nu = 1/2); otherwise
                          ceil(nu L) of Algorithm 1                          */
    int32_t postproc;  /* 1: singleton averaging of Remark 2.9, median as
                          fall-back; 0: medians of eq. (2.10) only           */
    int64_t s_cap;     /* Algorithm 4 sparsity s~ per function (>= 1)         */
    int64_t cap;       /* detected-list capacity per function, 1..2^24; above
                          8192 the call synchronises its stream once (to size
                          its global-memory buffers: the ordered compaction of
                          the detected set and Algorithm 4's sort) and cannot
                          be graph-captured */
} mr1l_extract_opts;

/* Outputs of mr1l_extract (all dev; optional ones may be NULL). */
typedef struct {
    int64_t *n_det;     /* [F] |detected set| (may exceed cap: then cap of
                           the detected candidates, a subset that depends
                           on the order of the vote pass, are kept, sorted
                           ascending, and the later stages see only them)  */
    int64_t *det_idx;   /* [F][cap] detected candidates, ascending          */
    void *det_coef;     /* [F][cap] coefficient: singleton average, else
                           median (postproc = 1); median (postproc = 0)    */
    void *det_med;      /* [F][cap] median coefficient, eq. (2.10) | NULL   */
    uint32_t *det_mask; /* [F][cap][W], W = ceil(L/32) words: bit l % 32 of
                           word l / 32 set iff the candidate is alone
                           among the detected set in its bucket of lattice
                           l (Remark 2.9) | NULL                           */
    int32_t *det_hash;  /* [F][cap][L] buckets of the detected set | NULL   */
    double *det_w;      /* [F][cap][L][2] real weights (re, im) of the
                           coefficient as a linear map of the lattice
                           values, for the adjoint | NULL                  */
    int64_t *n_out;     /* [F] Algorithm 4 output size (<= s_cap)           */
    int64_t *out_idx;   /* [F][s_cap] candidates by descending modulus      */
    void *out_coef;     /* [F][s_cap] their coefficients                    */
    int32_t *out_pos;   /* [F][s_cap] position in the detected list | NULL  */
    uint8_t *votes;     /* [n_total] number of non-zero buckets | NULL      */
} mr1l_extract_out;

/*
 * One pass of Algorithm 2 (+ Remark 2.9) + Algorithm 4 over the candidate
 * sets, given the DFT values and the non-zero bitmap of mr1l_fft:
 *   1. votes v(k) = #{l : bit h_l(k) of the bitmap is set}; the detected set
 *      is {k : v(k) >= vote_min} in ascending candidate order;
 *   2. occupancy of every bucket by the detected set, singleton masks;
 *   3. coefficients: medians of the real and imaginary parts over the L
 *      lattice values (even L: mean of the two middle order statistics),
 *      and the singleton average when postproc;
 *   4. keep |p| >= theta, order by |p| descending (ties: ascending index),
 *      keep the first s_cap.
 * Hashing and votes are bit-exact for any int64 input.  Returns
 * MR1L_E_ARG for invalid options.  A detected count above cap is reported
 * in n_det (device) and is not an error of the call.
 */
int mr1l_extract(mr1l_plan p, int64_t n_total, const int64_t *set_off,
                 const int64_t *freq, const void *ghat,
                 const uint32_t *nz_bitmap, const mr1l_extract_opts *o,
                 const mr1l_extract_out *out);

/*
 * Adjoint of the coefficient map for a fixed support and fixed selections
 * (the transpose of the real-linear map samples -> out_coef that one
 * mr1l_fft + mr1l_extract computed):
 *   gbar_{f,l}[h] = sum over outputs o of f with bucket h in lattice l of
 *                   w_re * Re(grad[o]) + i w_im * Im(grad[o]),
 *   grad_f[O + j] = (1/M) sum_h gbar[h] exp(+2 pi i j h / M).
 *   cap, s_cap       the values used in the extract call;
 *   n_out, out_pos,
 *   det_hash, det_w  dev outputs of that extract call;
 *   grad_out         dev [F][s_cap] complex (entries o >= n_out ignored);
 *   grad_f           dev [nodes] complex output.
 */
int mr1l_adjoint(mr1l_plan p, int64_t cap, int64_t s_cap,
                 const int64_t *n_out, const int32_t *out_pos,
                 const int32_t *det_hash, const double *det_w,
                 const void *grad_out, void *grad_f);

/*
 * HIP graphs: record the plan's subsequent calls into a graph instead of
 * running them (mr1l_graph_begin), finish and instantiate it
 * (mr1l_graph_end), replay it on the plan's stream (mr1l_graph_launch).
 * Calls recorded this way must not change pointers or sizes between
 * replays.  The library records only kernel launches (no memsets).
 */
typedef struct mr1l_graph_s *mr1l_graph;
int mr1l_graph_begin(mr1l_plan p);
int mr1l_graph_end(mr1l_plan p, mr1l_graph *g);
int mr1l_graph_launch(mr1l_graph g, void *stream);
int mr1l_graph_destroy(mr1l_graph g);

/*
 * Check that every function's candidate set stays injective modulo each of its
 * lattice sizes (the sizes must lie in P^Gamma, Section 2.1).  Every prime
 * above the set's expansion N_Gamma (largest coordinate range) qualifies; for
 * smaller sizes the reduced vectors k mod M are compared exactly.
 *   freq, set_off  as for mr1l_extract;
 *   ok             host [F] or NULL: 1 if function f's set is injective
 *                  modulo all of its sizes, else 0.
 * Returns MR1L_E_NOT_INJECTIVE when some function fails (ok is filled for all
 * functions).  Allocates a temporary table of 4 * pow2ceil(2 |Gamma_f|) bytes
 * when a size needs the exact comparison; synchronises the plan's stream.
 */
int mr1l_check_injective(mr1l_plan p, int64_t n_total, const int64_t *set_off,
                         const int64_t *freq, int32_t *ok);

/*
 * Least-squares coefficients on the detected set (Remark 2.9: with the
 * detected set I~ taken as the frequencies of the polynomial, its
 * coefficients are computed from the samples already taken on the fixed
 * lattices by a least-squares method).  Minimises over c in C^{|I~|}
 *   sum_l sum_{j<M_l} |sum_{k in I~} c_k e^{2 pi i j k.z_l / M_l} - f_l[j]|^2
 *   = sum_l M_l sum_h |sum_{k in I~, h_l(k) = h} c_k - ghat_l[h]|^2
 * (Parseval on each lattice and eq. (2.4)) by conjugate gradients on the
 * normal equations, per function, then applies Algorithm 4 to c.  When the
 * lattices discretise the polynomials on I~ and I~ contains the support, the
 * solution is exact and zero on the false positives.
 *   cap, n_det, det_idx, det_hash, det_mask  dev outputs of the extract call
 *            that found I~ (det_hash and det_mask required; only the first
 *            min(n_det, cap) entries take part); ghat  dev lattice values of
 *            mr1l_fft (the same samples).
 *   max_iter >= 0 CG iterations at most; tol >= 0: stop once the normal-
 *            equation residual is <= tol times the right-hand side.
 *   coef     dev [F][cap] complex, in: the start (e.g. the extract call's
 *            det_coef), out: the least-squares coefficients.
 *   resid    dev double [F] final relative residual | NULL;
 *   iters    dev int32 [F] iterations taken | NULL.
 *   theta, s_cap, n_out, out_idx, out_coef  Algorithm 4 on the solution, as
 *            in mr1l_extract; n_out == NULL skips it.
 * Asynchronous on the plan's stream, except that with cap > 8192 and
 * n_out != NULL it synchronises once (to size the global-memory sort of
 * Algorithm 4, as mr1l_extract does); grows plan scratch of
 * F*cap*(4L + 4*sizeof(complex)) bytes on first use (not during graph
 * capture); MR1L_E_ARG for invalid arguments.
 */
int mr1l_lsq(mr1l_plan p, int64_t cap, const int64_t *n_det,
             const int64_t *det_idx, const int32_t *det_hash,
             const uint32_t *det_mask, const void *ghat, int32_t max_iter,
             double tol, void *coef, double *resid, int32_t *iters,
             double theta, int64_t s_cap, int64_t *n_out, int64_t *out_idx,
             void *out_coef);

/*
 * Worst-case aliasing counts of Section 4.1.1 (Table 4.1).  Run mr1l_sample,
 * mr1l_fft and mr1l_extract (Remark 2.9 post-processing on, vote_min 0) on the
 * counting polynomial of eq. (4.1), all-ones coefficients on the support I,
 * over candidate sets that list I first: candidates [0, n_active[f]) of
 * function f are I, the rest are Gamma \ I.  Every lattice value at a bucket
 * of k then counts the members of I in that bucket, and per function
 *   counts[4f+0] = #PFP: candidates outside I that are detected
 *                  (n_det - n_active, exact also beyond cap),
 *   counts[4f+1] = #PFN: members of I whose median (eq. (2.10)) exceeds 1,
 *   counts[4f+2] = #PFP left after Remark 2.9: detected candidates outside I
 *                  whose post-processed coefficient keeps |p| >= theta,
 *   counts[4f+3] = flags: bit 0 the detected list was truncated (n_det > cap;
 *                  counts[4f+1] and counts[4f+2] then cover the kept
 *                  entries only); bit 1 I was not detected whole in front
 *                  of a complete list, or |I| > cap (a threshold outside
 *                  (0, 1) or a set not listing I first).
 *   cap, n_det, det_idx, det_med, det_coef  the extract call's cap and dev
 *            outputs (det_med required); n_active dev int64 [F];
 *   theta    the extract call's threshold; counts dev int64 [F][4].
 * Asynchronous on the plan's stream; MR1L_E_ARG for NULL buffers or an
 * invalid cap.
 */
int mr1l_pfpn_count(mr1l_plan p, int64_t cap, const int64_t *n_active,
                    const int64_t *n_det, const int64_t *det_idx,
                    const void *det_med, const void *det_coef, double theta,
                    int64_t *counts);

/*
 * DFT schedules and their autotuner.  The lattice DFT of one size M runs under
 * one schedule: 0 = the whole Bluestein transform (5-smooth length) in one
 * workgroup's LDS, valid while that length fits; 1..8 = power-of-two four-step
 * Bluestein transforms differing in workgroup size, LDS batch, workgroups per
 * CU and the split N = N1 N2; 9 = Rader's algorithm with the length-(M-1)
 * convolution in registers, for prime M with M - 1 = 2^a 5^b, a >= 2, b >= 1,
 * (M - 1)/20 <= 1024 and M - 1 reals fitting the LDS (names from
 * mr1l_fft_schedule_name).  Every schedule computes the same transform to
 * within rounding.  A new plan starts each size on the schedule the autotuner
 * chose for (dtype, M) earlier in the process, else on 0 where it applies,
 * else on 9 where it applies, else on the default four-step schedule.
 *
 * mr1l_plan_fft_schedule: sched < 0 returns the schedule of size M in the
 * plan; otherwise sets it (MR1L_E_ARG if M is not a size of the plan or the
 * schedule does not apply to it) and returns it.  Synchronises the plan's
 * stream and may grow the plan's scratch; graphs recorded earlier must be
 * recorded again.
 *
 * mr1l_fft_tune: groups the plan's distinct sizes whose transforms run
 * alike (same power-of-two length and same LDS size class of the 5-smooth
 * length, or none), times each schedule that applies to a group on all of the
 * plan's lattices of that group in one launch (one warm-up run, then the mean
 * of reps runs, HIP events on the plan's stream), keeps the fastest for every
 * size of the group and records it for later plans of this process.  sizes
 * (host [max_sizes] or NULL) receives the distinct sizes in the order used;
 * times_ms (host [max_sizes][mr1l_fft_schedule_count()] or NULL) the mean
 * milliseconds per run of each size's group, -1 where a schedule does not
 * apply.  Allocates and frees two node-sized buffers; synchronises the plan's
 * stream.
 */
int mr1l_fft_schedule_count(void);
const char *mr1l_fft_schedule_name(int32_t sched);
int mr1l_plan_fft_schedule(mr1l_plan p, int64_t M, int32_t sched);
int mr1l_fft_tune(mr1l_plan p, int32_t reps, int32_t max_sizes, int64_t *sizes, float *times_ms);

/* Parameters of the dimension-incremental driver. */
typedef struct {
    int32_t d;         /* spatial dimension of the function                */
    int64_t N;         /* single-coordinate candidate range [-N, N]        */
    int64_t s;         /* sparsity s of the final step                     */
    int64_t s_local;   /* sparsity of the intermediate steps (2 s default) */
    int32_t r;         /* detection repetitions per step t < d             */
    double theta;      /* threshold                                        */
    double c;          /* constant of eq. (4.2) (10.33)                    */
    double delta;      /* failure parameter of eq. (4.2)                   */
    int64_t M;         /* prime lattice size used for every lattice        */
    int32_t postproc;  /* Remark 2.9 averaging on/off                      */
    uint64_t seed;     /* SplitMix64 seed of all random draws               */
    int32_t dtype;     /* MR1L_C128 or MR1L_C64                            */
    int32_t step1;     /* 1: single-coordinate sets from Step 1; 0: [-N, N] */
    int32_t bs_n;      /* > 0: the function is the built-in B-spline test
                          function of mr1l_sample_bspline with bs_n products
                          (orders bs_order, coordinate masks bs_dims over the
                          d coordinates); 0: the sparse polynomial           */
    int32_t bs_order[16];
    uint64_t bs_dims[16];
    int32_t lsq_iters; /* > 0: the final coefficients are the least-squares
                          fit (mr1l_lsq, at most lsq_iters CG iterations) of
                          the output frequencies to the samples of the t = d
                          step's lattices (Remark 2.9, in place of the
                          external Step 3); 0: Algorithm 4's estimates       */
} mr1l_dimincr_params;

/*
 * Sampling callback for the driver: write the samples of the black-box
 * function at the nodes of L lattices in t dimensions with anchors
 * x'_u = anchor[u - t] / 2^32 (u = t..d-1) into the device array f_dev
 * (L*M complex, lattice-major), ordered on `stream`.  Return 0 on success.
 */
typedef int (*mr1l_sample_fn)(void *user, int32_t t, int32_t L,
                              const int64_t *M, const int64_t *z,
                              const uint32_t *anchor, void *f_dev,
                              void *stream);

/*
 * Steps 1 and 2 of Algorithm 3 with Algorithm 4 as the detection method
 * (Section 3.2.2).
 * Step 1 (step1 = 1; built-in sampler only; 2N + 1 <= 8192): for every
 * coordinate t = 1..d and i = 1..r, anchors x'_j = a_j / 2^32 for j != t
 * (ascending j) from the SplitMix64 stream n = 2^62 + ((t*64 + i) << 24)
 * + c + 1, samples at x_t = l / (2N+1), l <= 2N, the normalised length-(2N+1)
 * DFT, and the frequencies k_t in [-N, N] among the s_local largest moduli
 * with |value| >= theta (ties: smaller k_t first); I^(t) is the union over i.
 * With step1 = 0 every I^(t) is the full range [-N, N].
 * Step 2: for t = 2..d and i = 1..r~ (r~ = r for t < d, 1 for t = d),
 * candidates J_t = I^(1..t-1) x I^(t) in lexicographic order, L lattices by
 * eq. (4.2) on |J_t| (smallest odd L >= (c/((c-2) ln(c-1))) (ln|J_t| -
 * ln delta)), every lattice of size M, random anchors and generating
 * vectors drawn from SplitMix64 outputs of the stream (seed, t, i)
 * (n = ((t*64 + i) << 24) + c + 1; anchors u = t..d-1 first, then z_{l,u}
 * for l < L, u < t; integers in [0, m) by floor(x m / 2^64); anchors x >> 32),
 * Algorithm 4 with s~ = s_local (t < d) or s (t = d), and the union of the
 * detected tuples (sorted, without repeats).  The output of the t = d call
 * is the result.
 *   fn/user   sampling callback; if fn is NULL the built-in sampler of the
 *             B-spline test function (bs_n > 0) or of the sparse polynomial
 *             (poly_freq dev [d][poly_s] int64, poly_coef dev [poly_s]
 *             complex) is used.
 *   cap       capacity of freq_out / coef_out and of every intermediate
 *             union (entries).
 *   n_out     host: number of recovered frequencies.
 *   freq_out  host [cap][d] int64, lexicographically sorted;
 *   coef_out  host [cap] complex (dtype of the params).
 *   total_samples host (may be NULL): sum over Step 2 calls of L*M, plus
 *             d*r*(2N+1) with Step 1.
 * Synchronises the stream.  MR1L_E_CAPACITY if a union exceeds cap.
 */
int mr1l_dimincr(const mr1l_dimincr_params *prm, mr1l_sample_fn fn,
                 void *user, const int64_t *poly_freq, const void *poly_coef,
                 int64_t poly_s, int64_t cap, int64_t *n_out,
                 int64_t *freq_out, void *coef_out, int64_t *total_samples,
                 void *stream);

/*
 * Stage timing.  While enabled, every call records a pair of HIP events on
 * the plan's stream around each stage it launches: MR1L_STAGE_FFT (the
 * lattice DFTs), MR1L_STAGE_VOTE (hashing + vote kernel), MR1L_STAGE_TAIL
 * (sort, singleton masks, combine, limit), MR1L_STAGE_SAMPLE.
 * mr1l_profile_read synchronises the stream, adds the elapsed milliseconds
 * of every recorded pair into ms[stage] and the number of pairs into
 * count[stage] (host arrays of MR1L_NSTAGE), and forgets the pairs.  Do not
 * enable it while recording a graph.
 */
enum { MR1L_STAGE_FFT = 0, MR1L_STAGE_VOTE = 1, MR1L_STAGE_TAIL = 2, MR1L_STAGE_SAMPLE = 3,
       MR1L_NSTAGE = 4 };
int mr1l_profile(mr1l_plan p, int32_t enable);
int mr1l_profile_read(mr1l_plan p, double *ms, int64_t *count);

/* Number of lattices of eq. (4.2) for |J| candidates (host helper). */
int32_t mr1l_num_lattices(int64_t nJ, double c, double delta);

#ifdef __cplusplus
}
#endif

#endif /* MR1L_H */
