// Internal declarations of the mr1l library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mr1l.h"
#include "mr1l_device.h"

namespace mr1l {

// detected lists longer than kMaxCap are sorted in global memory (one stream synchronisation)
constexpr int64_t kMaxCapLarge = int64_t(1) << 24;

// LDS words of the vote pass's bitmap copy at most (80 KiB: two or more workgroups per CU)
constexpr int kVoteLdsWords = 20480;

// Non-zero bitmap bits of a wave whose active lanes are a prefix of the wave holding
// consecutive nodes (lane j: node g of lane 0 plus j, as in a loop i = tid, tid + NT, ...
// with NT a multiple of 64): the bits are gathered by a ballot and each 32-bit word the
// wave touches gets one atomicOr, from the lane that starts it.
__device__ __forceinline__ void bitmap_set_run(uint32_t *bitmap, int64_t g, bool set)
{
    const uint64_t b = __ballot(set);
    if (b == 0) return;
    const int lane = (int)(threadIdx.x & 63);
    const int bit = (int)(g & 31);
    if (lane == 0 || bit == 0) {
        const int len = min(64 - lane, 32 - bit);   // lanes in this word, at most 32
        const uint64_t seg = (b >> lane) & ((uint64_t(1) << len) - 1);
        if (seg) atomicOr(bitmap + (g >> 5), (uint32_t)(seg << bit));
    }
}

// The same for any node order, as long as the active lanes are a prefix of the wave:
// lanes whose node follows the previous lane's node within one 32-bit word join that
// lane's run, and each run's first lane sets the run's bits with one atomicOr.
__device__ __forceinline__ void bitmap_set_lanes(uint32_t *bitmap, int64_t g, bool set)
{
    const uint64_t b = __ballot(set);
    if (b == 0) return;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t gp = __shfl_up(g, 1);
    const bool cont = lane > 0 && gp + 1 == g && (g & 31) != 0;
    const uint64_t c = __ballot(cont);
    if (!cont) {
        const uint64_t next = lane == 63 ? 0 : (c >> (lane + 1));   // continuation flags after this lane
        const int len = 1 + __builtin_ctzll(~next);                 // at most 32: runs stop at word ends
        const uint64_t seg = (b >> lane) & ((uint64_t(1) << len) - 1);
        if (seg) atomicOr(bitmap + (g >> 5), (uint32_t)(seg << (g & 31)));
    }
}

// ---------------------------------------------------------------- DFT schedules
// How the Bluestein transform of one lattice runs.  Schedule 0 holds the whole
// 5-smooth-length transform in one workgroup's LDS; the others are power-of-two
// four-step transforms that differ in workgroup size, LDS batch (elements per
// LDS-resident sub-problem), resident workgroups per CU (which sets the register
// budget) and the split N1 = 2^ceil(k/2) or 2^floor(k/2) of N = 2^k.
struct FftSched {
    const char *name;
    int32_t four_step;
    int32_t threads;
    int32_t batch_log2;   // complex128; complex64 uses one more
    int32_t per_cu;
    int32_t split_floor;
    int32_t rader;        // Rader's algorithm in registers (prime M, M - 1 = 2^a 5^b)
    int32_t engine;       // 1: reg (whole transform in registers), 2: split (blocks of one workgroup)
};
constexpr int kNumSched = 12;
extern const FftSched kSched[kNumSched];
constexpr int kDefaultFourStep = 2;
constexpr int kRaderSched = 9;
constexpr int kRegSched = 10;
constexpr int kSplitSched = 11;
// Register-engine lengths: reg takes N = the smallest power of two >= 2M - 1 in
// [64, 16384] (complex128) or [64, 32768] (complex64); split (complex128) cuts M into
// K = ceil(M / 8192) <= 4 blocks transformed at length 16384.
constexpr int kRegMinN = 64;
constexpr int kSplitLen = 16384;
constexpr int kSplitMaxK = 4;

// Lattices launched together: schedule, LDS size class (schedule 0), whether the
// four-step tables fit the LDS, and the lattice list (host and device).
struct FftGroup {
    int32_t sched = 0, cls = 0;
    bool ltab = true;
    double work = 0.0;   // sum of M log M over the group (launch order)
    std::vector<int32_t> lats;
    int32_t *d_lats = nullptr;   // into Plan::d_glists
};
constexpr int kLdsClasses = 3;     // whole-LDS transforms: N <= 1024, <= 4096, <= NMAX
inline int lds_class(int64_t N) { return N <= 1024 ? 0 : (N <= 4096 ? 1 : 2); }

// Rader transform of one prime size M (P = M - 1): register passes and table offsets
// (permutations in the plan's int32 table, twiddles and the spectrum of the
// convolution kernel in its complex table).
struct RaderDesc {
    int32_t P = 0, nthreads = 0;
    int32_t n4 = 0, n2 = 0, n5 = 0, pad = 0;   // passes of radix 4, 2 and 5, in this order
    int64_t perm_in = 0, perm_out = 0, tw = 0, spec = 0;
};

// Per distinct lattice size: both possible layouts of its transform.
struct MInfo {
    int64_t M = 0;
    int32_t Ns = 0;           // 5-smooth length (0: too large for one workgroup's LDS)
    int64_t spec_s = -1, tw_s = -1;
    int32_t Np = 0;           // power-of-two length
    int64_t spec_p = -1, tw_p = -1;
    bool ltab = true;         // four-step tables fit the LDS (M <= 32768, N <= 2^16)
    bool rader = false;       // the Rader schedule applies
    int32_t Nr = 0;           // reg schedule: transform length (0: does not apply)
    int64_t spec_r = -1, tw_r = -1;
    int32_t Nq = 0, Bq = 0, Kq = 0;   // split schedule: transform length, block, blocks (Nq 0: does not apply)
    int64_t spec_q = -1, tw_q = -1;
    int32_t sched = 0;
    bool tuned = false;       // sched came from the autotuner's record
    int32_t nlat = 0;
    uint32_t spec_done = 0;   // spectra computed, bit per layout kind (see fft_spec_kind)
};

// ---------------------------------------------------------------- plan
struct Plan {
    int32_t d = 0, F = 0, L = 0, dtype = MR1L_C128;
    hipStream_t stream = nullptr;
    // DFT groups without scratch run concurrently on these (default priority) streams,
    // forked from and joined back into the plan's stream with the events
    static constexpr int kFftAux = 3;
    hipStream_t fft_aux[kFftAux] = {};   // the device's shared pool (never destroyed)
    hipEvent_t fft_ev[kFftAux + 1] = {};
    // the small device tables (descriptors, z, vote records, twiddles, chirps, Rader
    // tables, counters) in one allocation, uploaded by one copy from h_arena (kept
    // with the plan, so the copy may run after plan creation returns)
    void *d_arena = nullptr;
    std::vector<unsigned char> h_arena;
    std::vector<std::pair<void **, size_t>> arena_fix;
    // the DFT groups' lattice lists, concatenated (host copy kept for the async upload)
    int32_t *d_glists = nullptr;
    int64_t glists_cap = 0;
    std::vector<int32_t> h_glists;
    // spectrum passes: per-pass layout tables and representative lattices
    void *d_specwork = nullptr;
    int64_t specwork_bytes = 0;
    std::vector<unsigned char> h_specwork;
    int64_t nodes = 0;
    std::vector<int64_t> M;          // host [F*L]
    std::vector<int64_t> z;          // host [F*L*d]
    std::vector<LatDesc> lat;        // host copy
    std::vector<MDesc> mdesc;
    std::vector<int32_t> kb;         // per function: fast-hash bound on |k_u|
    // device tables
    LatDesc *d_lat = nullptr;
    MDesc *d_mdesc = nullptr;
    int32_t *d_z32 = nullptr;        // [F*L*d] z as int32
    int64_t *d_z64 = nullptr;        // [F*L*d] z as int64
    int32_t *d_kb = nullptr;         // [F]
    uint32_t *d_z16 = nullptr;       // [F*L][ceil(d/2)] z as packed int16 pairs (M <= 2^15)
    bool dot2 = false;               // every M <= 2^15: 16-bit packed dot products
    // vote records: per function L + 1 records of vrec_stride (a power of two >= 4) words
    //   [off32, -M, inv_m bits, base, z words (packed pairs when dot2, else int32)...]
    // base: with the LDS bitmap copy (vote_lds), the byte offset of the lattice's words,
    // 4 x the words of the function's earlier lattices (each lattice's bits start on a
    // word there); else the bit of bucket 0 relative to the function's first bitmap
    // word.  Record L repeats record L - 1 so the next record can always be loaded.
    uint32_t *d_vrec = nullptr;
    int32_t vrec_stride = 0;
    bool vote_lds = false;           // every function's bitmap fits the vote pass's LDS copy
    int64_t vote_lds_words = 0;      // its words: max over functions of sum_l ceil(M_l / 32)
    void *d_spec = nullptr;          // kernel spectra (dtype complex)
    void *d_chirp = nullptr;         // chirp tables (dtype complex)
    void *d_tw = nullptr;            // twiddle tables (dtype complex)
    int64_t spec_len = 0, chirp_len = 0, tw_len = 0;
    // DFT schedule per distinct size; one launch per group of lattices with the
    // same schedule (and, for schedule 0, the same LDS size class)
    std::vector<MInfo> minfo;
    std::vector<FftGroup> fft_groups;
    // four-step scratch: one in-place slot of slot_len complex per resident workgroup
    void *d_fft_scratch = nullptr;
    int64_t fft_slot_len = 0;
    int32_t fft_slots = 0;
    void *d_nodes_scratch = nullptr; // [nodes] complex (sampler, adjoint)
    void *d_cterm = nullptr;         // sampler: [n_terms] anchored coefficients (complex)
    int64_t cterm_bytes = 0;
    int32_t *d_thash = nullptr;      // sampler: [L][n_terms] buckets of the terms
    int64_t thash_bytes = 0;
    void *d_static_scratch = nullptr; // this device's copy of the library's static term scratch
    std::vector<RaderDesc> rdesc;    // per distinct size (P = 0 where Rader does not apply)
    RaderDesc *d_rdesc = nullptr;
    int32_t *d_ritab = nullptr;      // Rader permutations
    void *d_rctab = nullptr;         // Rader twiddles and spectra (dtype complex)
    int64_t *d_det_tmp = nullptr;    // [F] detected counters
    // persistent scratch of extract when the caller passes NULL outputs
    int64_t ex_cap = 0;
    int32_t *d_ex_hash = nullptr;    // [F][cap][L]
    double *d_ex_w = nullptr;        // [F][cap][L][2]
    uint32_t *d_ex_mask = nullptr;   // [F][cap][mask_words(L)]
    void *d_ex_med = nullptr;        // [F][cap] complex
    int32_t *d_ex_pos = nullptr;     // [F][s_cap]
    int32_t *d_ex_cstage = nullptr;  // short lists: staged coordinates [F][cap][W] and the order
    int64_t cstage_bytes = 0;        //   pass's permutation [F][cap] behind them
    int64_t ex_scap = 0;
    void *d_gsort = nullptr;         // global sort pairs of long detected lists: [F][P] uint64 + [F][P] int32
    int64_t gsort_bytes = 0;
    uint32_t *d_single = nullptr;    // long lists: bucket bitmaps seen once / twice, 2 x [F][L][ceil(maxM/32)]
    int64_t single_bytes = 0;
    uint32_t *d_dflag = nullptr;     // long lists: detected-candidate bitmap over all sets + block counts
    int64_t dflag_bytes = 0;
    void *d_bs_dims = nullptr;       // B-spline sampler: [F][n_prod] coordinate masks
    int64_t bs_bytes = 0;
    void *d_ls = nullptr;            // least squares: [F][cap][L] int32 representatives + 4 [F][cap] complex
    int64_t ls_bytes = 0;
    int64_t *d_setoff_default = nullptr; // [2] = {0, n} for F == 1 calls
    int64_t setoff_n = -1;           // n the default pair holds (-1: unknown)
    int64_t *d_termoff_default = nullptr;
    int64_t termoff_n = -1;
    bool offsets_recorded = false;   // a graph recorded a write of a default pair
    bool capturing = false;
    // stage timing
    bool profiling = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof;
};

// Records an event pair around a stage when the plan is profiling.
struct StageTimer {
    Plan &p;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(Plan &pl, int st) : p(pl), stage(st)
    {
        if (p.profiling && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, p.stream);
    }
    ~StageTimer()
    {
        if (a && b) {
            (void)hipEventRecord(b, p.stream);
            p.prof.push_back({stage, {a, b}});
        }
    }
};

struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
#define MR1L_HIP(call)                                                           \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                    \
            return ::mr1l::fail(MR1L_E_HIP, std::string(#call) + ": " +          \
                                                hipGetErrorString(e_));          \
    } while (0)
#define MR1L_LAUNCH_CHECK() MR1L_HIP(hipGetLastError())

// ---------------------------------------------------------------- launches
int launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
int launch_fill_bytes(void *p, int64_t nbytes, hipStream_t s);  // zero fill

// Device memory through the per-device block cache (devmem.hip).  dev_free takes blocks
// the device is done with (the caller has synchronised the stream that used them).
int dev_alloc(void **ptr, size_t bytes);
void dev_free(void *ptr);
// *ptr replaced by a block of at least `bytes` bytes (contents not kept); the old block
// is released once the plan's stream is done with it.
int plan_regrow(Plan &p, void **ptr, size_t bytes);

// Plan scratch of at least `bytes` bytes in *ptr (capacity in `have`): reallocated when
// smaller, refused while the plan records a graph (a recorded kernel keeps the pointer).
int grow_scratch(Plan &p, void **ptr, int64_t bytes, int64_t &have);

int fft_run(Plan &p, const void *in, void *out, double theta, uint32_t *bitmap,
            int mode, double scale);
// Layouts, groups and (lazily) the spectra of the sizes' current schedules; a plan
// that has run nothing yet (fresh) skips the stream synchronisation.
int fft_apply_schedules(Plan &p, bool fresh = false);
bool fft_schedule_applies(const MInfo &mi, int s);
int tuned_schedule(int32_t dtype, int64_t M);
MDesc fft_layout(const Plan &p, int mid, int s);   // table entry of size mid under schedule s
int fft_time_plan(Plan &p, const void *in, void *out, int reps, float *ms);   // whole-plan forward DFT
Plan &plan_of(mr1l_plan p);   // the plan behind an ABI handle
int plan_create_impl(mr1l_plan *out, int32_t d, int32_t F, int32_t L, const int64_t *M, const int64_t *z,
                     int32_t dtype, void *stream, bool need_prime);
int limit_run(Plan &p, const int64_t *n_det, int64_t cap, const int64_t *det_idx, const void *det_coef, double theta,
              int64_t s_cap, int64_t *n_out, int64_t *out_idx, void *out_coef);
int check_injective_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq, int32_t *ok);
int bspline_sample_run(Plan &p, int32_t d_poly, int32_t n_prod, const int32_t *order, const uint64_t *dims,
                       const uint32_t *anchor, void *f);
bool rader_applies(int64_t M, size_t real_bytes);
template <typename T> int rader_tables(int64_t M, RaderDesc &rd, std::vector<int32_t> &itab, std::vector<T> &ctab);
int rader_init_attrs();
int rader_launch(Plan &p, int P, const int32_t *d_lats, int nl, const void *in, void *out, double theta,
                 uint32_t *bitmap, int mode, double scale, int by_m);
int lsq_init_attrs();
int lsq_run(Plan &p, int64_t cap, const int64_t *n_det, const int32_t *det_hash, const uint32_t *det_mask,
            const void *ghat, int32_t max_iter, double tol, void *coef, double *resid, int32_t *iters,
            int32_t *rep, void *vecs);
int pfpn_run(Plan &p, int64_t cap, const int64_t *n_active, const int64_t *n_det, const int64_t *det_idx,
             const void *det_med, const void *det_coef, double theta, int64_t *counts);
int fft_init_attrs();
int extract_init_attrs();
int vote_init_attrs();

// cstage (or NULL): [F][cap][W] coordinates of every detected candidate at its append
// position as the vote hashed them: W = ceil(d/2) packed 16-bit pairs when p.dot2, else d
// low words; first word INT32_MIN for a candidate beyond the fast bound.
int vote_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq,
             const uint32_t *bitmap, int32_t vote_min, int64_t cap, int64_t *n_det,
             int64_t *det_idx, uint8_t *votes, int32_t *cstage);
int hash_count_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq,
                   int32_t *hash, int32_t *counts);
int extract_tail_run(Plan &p, int64_t n_total, const int64_t *set_off, const int64_t *freq,
                     const void *ghat, const mr1l_extract_opts &o, const mr1l_extract_out &out,
                     int32_t *det_hash, double *det_w, uint32_t *det_mask, void *det_med,
                     int32_t *out_pos, const int32_t *cstage, int32_t *perm);
int sample_init_attrs();
// Address of the static term scratch on the current device (looked up once per device).
int sample_static_scratch(void **out);
int sample_run_noalloc(Plan &p, int32_t d_poly, const int64_t *term_off, int64_t n_terms, const int64_t *freq,
                       const void *coef, const uint32_t *anchor, void *f, int32_t mode);
int sample_run(Plan &p, int32_t d_poly, const int64_t *term_off, int64_t n_terms,
               const int64_t *freq, const void *coef, const uint32_t *anchor, void *f,
               int32_t mode);
// The sampler with caller-provided term scratch: cterm [n_terms] complex, thash [L][n_terms].
int sample_run_with(Plan &p, int32_t d_poly, const int64_t *term_off, int64_t n_terms,
                    const int64_t *freq, const void *coef, const uint32_t *anchor, void *f,
                    int32_t mode, void *cterm, int32_t *thash);
int adjoint_run(Plan &p, int64_t cap, int64_t s_cap, const int64_t *n_out,
                const int32_t *out_pos, const int32_t *det_hash, const double *det_w,
                const void *grad_out, void *grad_f);

enum { FFT_FWD = 0, FFT_INV = 1, FFT_SPEC = 2 };

// reg and split DFT schedules (k_lfft_d.hip, k_lfft_f.hip)
int reg_launch_d(Plan &p, int N, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                 double theta, uint32_t *bitmap, int mode, double scale, int by_m);
int reg_launch_f(Plan &p, int N, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                 double theta, uint32_t *bitmap, int mode, double scale, int by_m);
int split_launch_d(Plan &p, int K, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                   double theta, uint32_t *bitmap, int mode, double scale, int by_m);
int lfft_attrs_d();
int lfft_attrs_f();

// Number of compute units of the current device.
int num_cus();

}  // namespace mr1l
