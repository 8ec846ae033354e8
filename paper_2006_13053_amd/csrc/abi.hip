// C ABI of the library: plan construction and the entry points of mr1l.h.
#include "mr1l_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

namespace mr1l {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int num_cus()
{
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cached = n;
        else
            cached = 256;
    }
    return cached;
}

// ---------------------------------------------------------------- number theory
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m)
{
    return (uint64_t)((unsigned __int128)a * b % m);
}

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for 64-bit integers (first twelve prime bases).
static bool is_prime_u64(uint64_t n)
{
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : small) {
        if (n == p) return true;
        if (n % p == 0) return false;
    }
    uint64_t dd = n - 1;
    int s = 0;
    while ((dd & 1) == 0) { dd >>= 1; ++s; }
    for (uint64_t a : small) {
        uint64_t x = powmod(a, dd, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

static bool smooth235(int64_t n)
{
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

static int64_t next_smooth(int64_t n)
{
    while (!smooth235(n)) ++n;
    return n;
}

// ---------------------------------------------------------------- tables (host, long double)
// The tables of one size are the same in every plan, and their long-double evaluation
// dominates plan creation (the driver creates a plan per step): each is computed once
// per process and kept (entries are never removed, so references stay valid).
template <typename V> struct TableCache {
    std::mutex mu;
    std::map<int64_t, V> map;
    template <typename F> const V &get(int64_t key, F make)
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = map.find(key);
        if (it == map.end()) it = map.emplace(key, make()).first;
        return it->second;
    }
};

template <typename T>
static void push_twiddles(std::vector<T> &tab, int64_t n)
{
    static TableCache<std::vector<T>> cache;
    const std::vector<T> &v = cache.get(n, [n] {
        std::vector<T> t;
        t.reserve(2 * (size_t)n);
        const long double tp = 6.283185307179586476925286766559005768L;
        for (int64_t m = 0; m < n; ++m) {
            long double a = -tp * (long double)m / (long double)n;
            t.push_back((T)cosl(a));
            t.push_back((T)sinl(a));
        }
        return t;
    });
    tab.insert(tab.end(), v.begin(), v.end());
}

// e^{-pi i r / M}: low part r < S, high part r = hi * S
template <typename T>
static void push_chirp(std::vector<T> &tab, int64_t M, int32_t &shift, int32_t &nlo)
{
    shift = 0;
    while ((int64_t(1) << (2 * shift)) < 2 * M) ++shift;
    nlo = 1 << shift;
    const int32_t S = nlo;
    static TableCache<std::vector<T>> cache;
    const std::vector<T> &v = cache.get(M, [M, S] {
        std::vector<T> t;
        const long double pi = 3.141592653589793238462643383279502884L;
        const int64_t nhi = (2 * M + S - 1) / S;
        for (int64_t r = 0; r < S; ++r) {
            long double a = -pi * (long double)r / (long double)M;
            t.push_back((T)cosl(a));
            t.push_back((T)sinl(a));
        }
        for (int64_t h = 0; h < nhi; ++h) {
            long double a = -pi * (long double)(h * S) / (long double)M;
            t.push_back((T)cosl(a));
            t.push_back((T)sinl(a));
        }
        return t;
    });
    tab.insert(tab.end(), v.begin(), v.end());
}

// float reciprocal of M rounded down by at least 2^-21 relative
static float inv_m_down(int64_t M)
{
    const double x = (1.0 / (double)M) * (1.0 - std::ldexp(1.0, -21));
    float f = (float)x;
    while ((double)f > x) f = std::nextafter(f, 0.0f);
    return f;
}

// Largest |k_u| for which the 24-bit hash of every lattice of a function is exact.
static int32_t fast_bound(int d, const int64_t *M, int L)
{
    int64_t kb = (int64_t(1) << 23) - 1;
    kb = std::min<int64_t>(kb, ((int64_t(1) << 19) - 2) / d);
    for (int l = 0; l < L; ++l) {
        const int64_t m = M[l];
        if (m > 1) kb = std::min<int64_t>(kb, ((int64_t(1) << 31) - m - 1) / ((int64_t)d * (m - 1)));
    }
    return (int32_t)std::max<int64_t>(kb, 0);
}

// A table for the plan's arena: copied to the host staging buffer at a 256-byte
// boundary; *dst is pointed at its device copy when the arena is committed.
static void stage(Plan &p, void **dst, const void *src, size_t bytes)
{
    const size_t off = (p.h_arena.size() + 255) & ~size_t(255);
    p.h_arena.resize(off + std::max<size_t>(bytes, 16), 0);
    if (src && bytes) std::memcpy(p.h_arena.data() + off, src, bytes);
    p.arena_fix.push_back({dst, off});
}

static int arena_commit(Plan &p)
{
    {
        const int rc = dev_alloc(&p.d_arena, std::max<size_t>(p.h_arena.size(), 16));
        if (rc) return rc;
    }
    for (auto &f : p.arena_fix) *f.first = (unsigned char *)p.d_arena + f.second;
    p.arena_fix.clear();
    if (!p.h_arena.empty())
        MR1L_HIP(hipMemcpyAsync(p.d_arena, p.h_arena.data(), p.h_arena.size(), hipMemcpyHostToDevice, p.stream));
    return MR1L_OK;
}

constexpr int64_t kFewLattices = 64;

template <typename T>
static int build_tables(Plan &p)
{
    constexpr int NMAX = lds_max_n<T>();
    std::map<int64_t, int32_t> mid_of;
    std::map<int64_t, int64_t> tw_of;
    std::vector<T> tw, ch;
    std::vector<int32_t> ritab;
    std::vector<T> rctab;
    int64_t spec_len = 0;
    auto twoff = [&](int64_t n) -> int64_t {
        auto it = tw_of.find(n);
        if (it != tw_of.end()) return it->second;
        const int64_t off = (int64_t)tw.size() / 2;
        push_twiddles(tw, n);
        tw_of[n] = off;
        return off;
    };
    for (int64_t i = 0; i < (int64_t)p.M.size(); ++i) {
        const int64_t M = p.M[i];
        if (mid_of.count(M)) continue;
        const int32_t mid = (int32_t)p.mdesc.size();
        mid_of[M] = mid;
        MDesc md{};
        MInfo mi;
        mi.M = M;
        // layout of the whole-LDS schedule: 5-smooth N >= 2M - 1 when it fits one workgroup
        const int64_t Ns = next_smooth(std::max<int64_t>(2 * M - 1, 2));
        if (Ns <= NMAX) {
            mi.Ns = (int32_t)Ns;
            mi.spec_s = spec_len;
            spec_len += Ns;
            mi.tw_s = twoff(Ns);
        }
        // layout of the four-step schedules: power-of-two N >= 2M - 1 (at least 4)
        int k = 2;
        while ((int64_t(1) << k) < 2 * M - 1) ++k;
        mi.Np = 1 << k;
        mi.spec_p = spec_len;
        spec_len += mi.Np;
        mi.tw_p = twoff(mi.Np);
        md.chirp_off = (int64_t)ch.size() / 2;
        push_chirp(ch, M, md.chirp_shift, md.chirp_nlo);
        // the sub-transform twiddles (max(N1, N2) entries) and the two-level chirp
        // table go to LDS when they fit their LDS tables
        const int64_t nch = md.chirp_nlo + (2 * M + md.chirp_nlo - 1) / md.chirp_nlo;
        mi.ltab = mi.Np <= kTabTw * kTabTw && nch <= kTabCh;
        // reg: one register-resident transform pair of the power of two N >= 2M - 1
        {
            const int64_t nmax = sizeof(T) == 8 ? 16384 : 32768;
            int64_t n = kRegMinN;
            while (n < 2 * M - 1) n <<= 1;
            if (n <= nmax) {
                mi.Nr = (int32_t)n;
                mi.spec_r = spec_len;
                spec_len += n;
                mi.tw_r = twoff(n);
            }
        }
        // split (complex128, M too large for reg): K blocks of B <= kSplitLen / 2
        if (!mi.Nr && sizeof(T) == 8 && M <= (int64_t)kSplitMaxK * (kSplitLen / 2)) {
            const int64_t K = (M + kSplitLen / 2 - 1) / (kSplitLen / 2);
            mi.Nq = kSplitLen;
            mi.Kq = (int32_t)K;
            mi.Bq = (int32_t)((M + K - 1) / K);
            mi.spec_q = spec_len;
            spec_len += K * kSplitLen;   // segments 0 .. K - 1 (the chirp is even)
            mi.tw_q = twoff(kSplitLen);
        }
        // Rader's algorithm in registers for prime M with M - 1 = 2^a 5^b
        RaderDesc rd{};
        if (rader_applies(M, sizeof(T))) {
            mi.rader = true;
            rader_tables<T>(M, rd, ritab, rctab);
        }
        mi.sched = tuned_schedule(p.dtype, M);
        if (mi.sched >= 0 && !fft_schedule_applies(mi, mi.sched)) mi.sched = -1;
        // untuned: Rader where it applies (half the transform length of Bluestein),
        // else the register transforms, else the whole-LDS transform, else the four-step
        mi.tuned = mi.sched >= 0;
        if (mi.sched < 0)
            mi.sched = mi.rader ? kRaderSched : mi.Nr ? kRegSched : mi.Nq ? kSplitSched : mi.Ns ? 0 : kDefaultFourStep;
        p.mdesc.push_back(md);
        p.minfo.push_back(mi);
        p.rdesc.push_back(rd);
    }
    // A plan of at most kFewLattices lattices runs its DFT as a few latency-bound
    // launches, one per group: its untuned register-transform sizes take the whole-LDS
    // transform instead when they all fit it and that needs fewer launches (three LDS
    // size classes against one register length per power of two).
    if ((int64_t)p.M.size() <= kFewLattices) {
        std::vector<int> reg_n, lds_c;
        bool fit = true;
        for (const MInfo &mi : p.minfo)
            if (!mi.tuned && mi.sched == kRegSched) {
                fit = fit && mi.Ns > 0;
                if (std::find(reg_n.begin(), reg_n.end(), mi.Nr) == reg_n.end()) reg_n.push_back(mi.Nr);
                const int c = mi.Ns > 0 ? lds_class(mi.Ns) : -1;
                if (std::find(lds_c.begin(), lds_c.end(), c) == lds_c.end()) lds_c.push_back(c);
            }
        if (fit && lds_c.size() < reg_n.size())
            for (MInfo &mi : p.minfo)
                if (!mi.tuned && mi.sched == kRegSched) mi.sched = 0;
    }
    p.lat.resize(p.M.size());
    int64_t off = 0;
    bool all16 = true;
    for (auto m : p.M) all16 = all16 && m <= (int64_t(1) << 15);
    for (int f = 0; f < p.F; ++f) {
        int32_t kb = fast_bound(p.d, p.M.data() + (size_t)f * p.L, p.L);
        if (all16) kb = std::min<int32_t>(kb, 32767);   // k_u must fit the 16-bit dot products
        p.kb.push_back(kb);
        for (int l = 0; l < p.L; ++l) {
            const int64_t i = (int64_t)f * p.L + l;
            const int64_t M = p.M[i];
            LatDesc ld{};
            ld.node_off = off;
            ld.M = (int32_t)M;
            ld.mid = mid_of[M];
            p.minfo[ld.mid].nlat += 1;
            ld.func = f;
            ld.inv_m = inv_m_down(M);
            const int64_t S = (int64_t)p.d * kb * (M - 1);
            ld.off32 = (uint32_t)(((S + M - 1) / M) * M);
            ld.z_off = i * p.d;
            p.lat[i] = ld;
            off += M;
        }
    }
    p.nodes = off;
    p.spec_len = spec_len;
    p.tw_len = (int64_t)tw.size() / 2;
    p.chirp_len = (int64_t)ch.size() / 2;
    const size_t esz = 2 * sizeof(T);
    stage(p, (void **)&p.d_rdesc, p.rdesc.data(), p.rdesc.size() * sizeof(RaderDesc));
    if (!ritab.empty()) {
        stage(p, (void **)&p.d_ritab, ritab.data(), ritab.size() * sizeof(int32_t));
        stage(p, &p.d_rctab, rctab.data(), rctab.size() * sizeof(T));
    }
    stage(p, &p.d_tw, tw.data(), tw.size() * sizeof(T));
    stage(p, &p.d_chirp, ch.data(), ch.size() * sizeof(T));
    // the spectra are written by the DFT kernels (only the layouts in use)
    return dev_alloc(&p.d_spec, std::max<size_t>((size_t)spec_len * esz, 16));
}

// Records of the vote pass (see Plan::d_vrec).
static int build_vote_records(Plan &p, std::vector<uint32_t> &vr)
{
    const int zw = p.dot2 ? (p.d + 1) / 2 : p.d;
    int rs = 4;
    while (rs < zw + 4) rs <<= 1;
    p.vrec_stride = rs;
    // the LDS copy: each lattice's bits from a word boundary, when every function fits
    p.vote_lds_words = 0;
    for (int f = 0; f < p.F; ++f) {
        int64_t w = 0;
        for (int l = 0; l < p.L; ++l) w += (p.lat[(size_t)f * p.L + l].M + 31) >> 5;
        p.vote_lds_words = std::max(p.vote_lds_words, w);
    }
    p.vote_lds = p.vote_lds_words <= kVoteLdsWords;
    vr.assign((size_t)p.F * (p.L + 1) * rs, 0u);
    for (int f = 0; f < p.F; ++f) {
        const int64_t word0 = p.lat[(size_t)f * p.L].node_off >> 5;
        uint32_t wbase = 0;   // words of the function's earlier lattices in the LDS layout
        for (int l = 0; l <= p.L; ++l) {
            const int ls = l < p.L ? l : p.L - 1;
            const size_t i = (size_t)f * p.L + ls;
            const LatDesc &ld = p.lat[i];
            uint32_t *r = &vr[((size_t)f * (p.L + 1) + l) * rs];
            r[0] = ld.off32;
            r[1] = (uint32_t)(-(int32_t)ld.M);
            std::memcpy(&r[2], &ld.inv_m, 4);
            r[3] = p.vote_lds ? 4u * (l < p.L ? wbase : wbase - (uint32_t)((ld.M + 31) >> 5))
                              : (uint32_t)(ld.node_off - (word0 << 5));
            for (int u = 0; u < p.d; ++u) {
                const uint32_t zu = (uint32_t)p.z[i * p.d + u];
                if (p.dot2) r[4 + u / 2] |= (zu & 0xffffu) << (16 * (u & 1));
                else r[4 + u] = zu;
            }
            if (l < p.L) wbase += (uint32_t)((ld.M + 31) >> 5);
        }
    }
    return MR1L_OK;
}

static int upload(Plan &p)
{
    stage(p, (void **)&p.d_lat, p.lat.data(), p.lat.size() * sizeof(LatDesc));
    stage(p, (void **)&p.d_mdesc, p.mdesc.data(), p.mdesc.size() * sizeof(MDesc));
    std::vector<int32_t> z32(p.z.begin(), p.z.end());
    stage(p, (void **)&p.d_z32, z32.data(), z32.size() * sizeof(int32_t));
    stage(p, (void **)&p.d_z64, p.z.data(), p.z.size() * sizeof(int64_t));
    // packed 16-bit pairs of z for the dot2 hash (valid when every M <= 2^15)
    p.dot2 = true;
    for (auto m : p.M) p.dot2 = p.dot2 && m <= (int64_t(1) << 15);
    if (p.dot2) {
        const int dh = (p.d + 1) / 2;
        const int64_t nl = (int64_t)p.F * p.L;
        std::vector<uint32_t> z16((size_t)nl * dh, 0u);
        for (int64_t i = 0; i < nl; ++i)
            for (int u = 0; u < p.d; ++u)
                z16[(size_t)i * dh + u / 2] |= (uint32_t)(p.z[(size_t)i * p.d + u] & 0xffff) << (16 * (u & 1));
        stage(p, (void **)&p.d_z16, z16.data(), z16.size() * sizeof(uint32_t));
    }
    {
        std::vector<uint32_t> vr;
        int rc = build_vote_records(p, vr);
        if (rc) return rc;
        stage(p, (void **)&p.d_vrec, vr.data(), vr.size() * sizeof(uint32_t));
    }
    stage(p, (void **)&p.d_kb, p.kb.data(), p.kb.size() * sizeof(int32_t));
    stage(p, (void **)&p.d_det_tmp, nullptr, sizeof(int64_t) * (size_t)p.F);
    stage(p, (void **)&p.d_setoff_default, nullptr, 2 * sizeof(int64_t));
    stage(p, (void **)&p.d_termoff_default, nullptr, 2 * sizeof(int64_t));
    int rc = arena_commit(p);
    if (rc) return rc;
    const size_t esz = p.dtype == MR1L_C128 ? 16 : 8;
    return dev_alloc(&p.d_nodes_scratch, (size_t)std::max<int64_t>(p.nodes, 1) * esz);
}

// The auxiliary DFT streams of the current device: created once per device, shared
// by its plans (work of several plans on one of them runs in turn) and kept until
// the process ends.
static std::mutex g_aux_mu;
static hipStream_t g_aux[64][Plan::kFftAux];

static int aux_streams(hipStream_t *out)
{
    int dev = 0;
    MR1L_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MR1L_E_ARG, "device index beyond the stream pool");
    std::lock_guard<std::mutex> g(g_aux_mu);
    for (int i = 0; i < Plan::kFftAux; ++i) {
        if (!g_aux[dev][i] && hipStreamCreateWithFlags(&g_aux[dev][i], hipStreamNonBlocking) != hipSuccess) {
            g_aux[dev][i] = nullptr;
            return fail(MR1L_E_HIP, "DFT stream creation failed");
        }
        out[i] = g_aux[dev][i];
    }
    return MR1L_OK;
}

static void release(Plan *p)
{
    // (the tables in the arena are not freed one by one)
    void *ptrs[] = {p->d_arena, p->d_spec, p->d_glists, p->d_specwork, p->d_fft_scratch, p->d_nodes_scratch,
                    p->d_cterm, p->d_thash, p->d_ex_hash, p->d_ex_w, p->d_ex_mask, p->d_ex_med, p->d_ex_pos,
                    p->d_ex_cstage,
                    p->d_ls, p->d_gsort, p->d_single, p->d_dflag, p->d_bs_dims};
    (void)hipStreamSynchronize(p->stream);   // the blocks go back to the cache
    for (void *q : ptrs) dev_free(q);
    for (auto &ev : p->fft_ev)
        if (ev) (void)hipEventDestroy(ev);
    delete p;
}

__global__ void k_set_pair(int64_t *dst, int64_t a, int64_t b)
{
    if (threadIdx.x == 0) { dst[0] = a; dst[1] = b; }
}

// {0, n} for a one-function call without offsets.  The pair is rewritten only when n
// changes (cached in `have`), except once a graph has recorded such a write: a replay
// may then have left another n there, so every later call writes it again.
static int default_offsets(Plan &p, int64_t *dst, int64_t n, int64_t &have)
{
    if (!p.capturing && have == n) return MR1L_OK;
    hipLaunchKernelGGL(k_set_pair, dim3(1), dim3(64), 0, p.stream, dst, (int64_t)0, n);
    MR1L_LAUNCH_CHECK();
    if (p.capturing) p.offsets_recorded = true;
    have = p.offsets_recorded ? -1 : n;
    return MR1L_OK;
}

int grow_scratch(Plan &p, void **ptr, int64_t bytes, int64_t &have)
{
    if (have >= bytes && *ptr) return MR1L_OK;
    if (p.capturing) return fail(MR1L_E_ARG, "scratch must be sized before graph capture (run the call once)");
    have = 0;
    const int rc = plan_regrow(p, ptr, (size_t)std::max<int64_t>(bytes, 16));
    if (rc) return rc;
    have = bytes;
    return MR1L_OK;
}

int plan_regrow(Plan &p, void **ptr, size_t bytes)
{
    if (*ptr) {
        MR1L_HIP(hipStreamSynchronize(p.stream));
        dev_free(*ptr);
        *ptr = nullptr;
    }
    return dev_alloc(ptr, bytes);
}

static int grow(Plan &p, void **ptr, int64_t bytes, int64_t &have) { return grow_scratch(p, ptr, bytes, have); }

// Schedules chosen by the autotuner in this process, per (dtype, M); later plans
// start from them.
static std::mutex g_tuned_mu;
static std::map<std::pair<int32_t, int64_t>, int32_t> g_tuned;

int tuned_schedule(int32_t dtype, int64_t M)
{
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto it = g_tuned.find({dtype, M});
    return it == g_tuned.end() ? -1 : it->second;
}

static void record_tuned(int32_t dtype, int64_t M, int32_t s)
{
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[{dtype, M}] = s;
}

}  // namespace mr1l

using namespace mr1l;

struct mr1l_plan_s : public Plan {
    int64_t h_bytes = 0, w_bytes = 0, m_bytes = 0, med_bytes = 0, pos_bytes = 0;
};

struct mr1l_graph_s : public Graph {};

extern "C" {

int mr1l_version(void) { return 10000; }

const char *mr1l_last_error(void) { return g_err.c_str(); }

int mr1l_plan_create(mr1l_plan *out, int32_t d, int32_t F, int32_t L, const int64_t *M, const int64_t *z,
                     int32_t dtype, void *stream)
{
    return plan_create_impl(out, d, F, L, M, z, dtype, stream, true);
}

}  // extern "C"

mr1l::Plan &mr1l::plan_of(mr1l_plan p) { return *p; }

// Plan creation; need_prime = false admits composite sizes (the one-dimensional
// DFT grids of the driver's Step 1; the Bluestein transform holds for any size).
int mr1l::plan_create_impl(mr1l_plan *out, int32_t d, int32_t F, int32_t L, const int64_t *M, const int64_t *z,
                           int32_t dtype, void *stream, bool need_prime)
{
    if (!out) return fail(MR1L_E_ARG, "out is NULL");
    *out = nullptr;
    if (d < 1 || d > kMaxD) return fail(MR1L_E_ARG, "d must be in [1, 64]");
    // F is a grid dimension of the per-function kernels and f * L an int index
    if (F < 1 || F > (1 << 20)) return fail(MR1L_E_ARG, "F must be in [1, 2^20]");
    if (L < 1 || L > kMaxL) return fail(MR1L_E_ARG, "L must be in [1, 64]");
    if (dtype != MR1L_C128 && dtype != MR1L_C64) return fail(MR1L_E_ARG, "dtype must be MR1L_C128 or MR1L_C64");
    if (!M || !z) return fail(MR1L_E_ARG, "M or z is NULL");
    const int64_t nl = (int64_t)F * L;
    for (int64_t i = 0; i < nl; ++i) {
        if (M[i] < 2 || M[i] >= (int64_t(1) << 23))
            return fail(MR1L_E_ARG, "lattice size out of range [2, 2^23): " + std::to_string(M[i]));
        if (need_prime && !is_prime_u64((uint64_t)M[i]))
            return fail(MR1L_E_NOT_PRIME, "lattice size is not prime: " + std::to_string(M[i]));
        for (int u = 0; u < d; ++u) {
            const int64_t v = z[i * d + u];
            if (v < 0 || v >= M[i]) return fail(MR1L_E_ARG, "generating vector entry outside [0, M)");
        }
    }
    // LDS limits of the kernels, once per process (the first plan's device)
    static std::once_flag attrs_once;
    static int attrs_rc = MR1L_OK;
    static std::string attrs_err;
    std::call_once(attrs_once, [] {
        attrs_rc = fft_init_attrs();
        if (!attrs_rc) attrs_rc = extract_init_attrs();
        if (!attrs_rc) attrs_rc = vote_init_attrs();
        if (!attrs_rc) attrs_rc = lsq_init_attrs();
        if (!attrs_rc) attrs_rc = rader_init_attrs();
        if (!attrs_rc) attrs_rc = sample_init_attrs();
        if (attrs_rc) attrs_err = g_err;
    });
    if (attrs_rc) return fail(attrs_rc, "kernel attribute setup failed: " + attrs_err);
    mr1l_plan_s *p = new (std::nothrow) mr1l_plan_s();
    if (!p) return fail(MR1L_E_NOMEM, "host allocation failed");
    p->d = d; p->F = F; p->L = L; p->dtype = dtype;
    p->stream = (hipStream_t)stream;
    p->M.assign(M, M + nl);
    p->z.assign(z, z + nl * d);
    int rc = dtype == MR1L_C128 ? build_tables<double>(*p) : build_tables<float>(*p);
    if (rc == MR1L_OK) rc = upload(*p);
    if (rc == MR1L_OK) rc = sample_static_scratch(&p->d_static_scratch);
    if (rc == MR1L_OK) rc = aux_streams(p->fft_aux);
    for (int i = 0; rc == MR1L_OK && i <= Plan::kFftAux; ++i)
        if (hipEventCreateWithFlags(&p->fft_ev[i], hipEventDisableTiming) != hipSuccess)
            rc = fail(MR1L_E_HIP, "DFT event creation failed");
    if (rc == MR1L_OK) rc = fft_apply_schedules(*p, true);
    if (rc != MR1L_OK) {
        std::string keep = g_err;
        release(p);
        g_err = keep;
        return rc;
    }
    *out = p;
    return MR1L_OK;
}

extern "C" {

int mr1l_plan_destroy(mr1l_plan p)
{
    if (!p) return MR1L_OK;
    (void)hipStreamSynchronize(p->stream);
    release(p);
    return MR1L_OK;
}

int64_t mr1l_plan_nodes(mr1l_plan p) { return p ? p->nodes : -1; }

int mr1l_plan_set_stream(mr1l_plan p, void *stream)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    const hipStream_t ns = (hipStream_t)stream;
    if (ns != p->stream) {
        // work queued on the old stream (the table upload of plan creation among it)
        // comes before anything on the new one
        hipEvent_t ev = nullptr;
        MR1L_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        const hipError_t e1 = hipEventRecord(ev, p->stream);
        const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(ns, ev, 0) : e1;
        (void)hipEventDestroy(ev);
        if (e2 != hipSuccess) return fail(MR1L_E_HIP, std::string("stream ordering failed: ") + hipGetErrorString(e2));
    }
    p->stream = ns;
    return MR1L_OK;
}

int mr1l_plan_set_z(mr1l_plan p, const int64_t *z)
{
    if (!p || !z) return fail(MR1L_E_ARG, "plan or z is NULL");
    const int64_t nl = (int64_t)p->F * p->L;
    for (int64_t i = 0; i < nl; ++i)
        for (int u = 0; u < p->d; ++u)
            if (z[i * p->d + u] < 0 || z[i * p->d + u] >= p->M[i])
                return fail(MR1L_E_ARG, "generating vector entry outside [0, M)");
    p->z.assign(z, z + nl * p->d);
    std::vector<int32_t> z32(p->z.begin(), p->z.end());
    MR1L_HIP(hipMemcpyAsync(p->d_z32, z32.data(), z32.size() * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
    MR1L_HIP(hipMemcpyAsync(p->d_z64, p->z.data(), p->z.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                            p->stream));
    std::vector<uint32_t> z16;
    if (p->dot2) {
        const int dh = (p->d + 1) / 2;
        z16.assign((size_t)nl * dh, 0u);
        for (int64_t i = 0; i < nl; ++i)
            for (int u = 0; u < p->d; ++u)
                z16[(size_t)i * dh + u / 2] |= (uint32_t)(p->z[(size_t)i * p->d + u] & 0xffff) << (16 * (u & 1));
        MR1L_HIP(hipMemcpyAsync(p->d_z16, z16.data(), z16.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                p->stream));
    }
    std::vector<uint32_t> vr;
    (void)build_vote_records(*p, vr);
    MR1L_HIP(hipMemcpyAsync(p->d_vrec, vr.data(), vr.size() * sizeof(uint32_t), hipMemcpyHostToDevice, p->stream));
    MR1L_HIP(hipStreamSynchronize(p->stream));
    return MR1L_OK;
}

int mr1l_sample(mr1l_plan p, int32_t d_poly, const int64_t *term_off, int64_t n_terms, const int64_t *freq,
                const void *coef, const uint32_t *anchor, void *f, int32_t mode)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (d_poly < p->d || d_poly > kMaxD) return fail(MR1L_E_ARG, "d_poly must be in [d, 64]");
    if (n_terms < 0 || (n_terms > 0 && (!freq || !coef)) || !f) return fail(MR1L_E_ARG, "null buffer");
    if (d_poly > p->d && !anchor) return fail(MR1L_E_ARG, "anchors required when d_poly > d");
    if (mode < 0 || mode > 2) return fail(MR1L_E_ARG, "mode must be 0, 1 or 2");
    if (!term_off) {
        if (p->F != 1) return fail(MR1L_E_ARG, "term_off required when F > 1");
        int rc = default_offsets(*p, p->d_termoff_default, n_terms, p->termoff_n);
        if (rc) return rc;
        term_off = p->d_termoff_default;
    }
    if (mode == 1)
        for (auto m : p->M)
            if (m > (int64_t(1) << 22)) mode = 2;
    StageTimer tm(*p, MR1L_STAGE_SAMPLE);
    return sample_run(*p, d_poly, term_off, n_terms, freq, coef, anchor, f, mode);
}

int mr1l_sample_noalloc(mr1l_plan p, int32_t d_poly, const int64_t *term_off, int64_t n_terms, const int64_t *freq,
                        const void *coef, const uint32_t *anchor, void *f, int32_t mode)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (d_poly < p->d || d_poly > kMaxD) return fail(MR1L_E_ARG, "d_poly must be in [d, 64]");
    if (n_terms < 0 || (n_terms > 0 && (!freq || !coef)) || !f) return fail(MR1L_E_ARG, "null buffer");
    if (d_poly > p->d && !anchor) return fail(MR1L_E_ARG, "anchors required when d_poly > d");
    if (mode < 0 || mode > 2) return fail(MR1L_E_ARG, "mode must be 0, 1 or 2");
    if (!term_off) return fail(MR1L_E_ARG, "term_off is required (dev [F+1])");
    if (mode == 1)
        for (auto m : p->M)
            if (m > (int64_t(1) << 22)) mode = 2;
    return sample_run_noalloc(*p, d_poly, term_off, n_terms, freq, coef, anchor, f, mode);
}

int mr1l_fft(mr1l_plan p, const void *f, void *ghat, double theta, uint32_t *nz_bitmap)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (!f || !ghat || f == ghat) return fail(MR1L_E_ARG, "f and ghat must be distinct device buffers");
    if (!(theta >= 0.0)) return fail(MR1L_E_ARG, "theta must be >= 0");
    StageTimer tm(*p, MR1L_STAGE_FFT);
    return fft_run(*p, f, ghat, theta, nz_bitmap, FFT_FWD, 1.0);
}

int mr1l_hash_count(mr1l_plan p, int64_t n_total, const int64_t *set_off, const int64_t *freq, int32_t *hash,
                    int32_t *counts)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (n_total < 0 || (n_total > 0 && !freq)) return fail(MR1L_E_ARG, "invalid candidate set");
    if (!set_off) {
        if (p->F != 1) return fail(MR1L_E_ARG, "set_off required when F > 1");
        int rc = default_offsets(*p, p->d_setoff_default, n_total, p->setoff_n);
        if (rc) return rc;
        set_off = p->d_setoff_default;
    }
    return hash_count_run(*p, n_total, set_off, freq, hash, counts);
}

int mr1l_extract(mr1l_plan p, int64_t n_total, const int64_t *set_off, const int64_t *freq, const void *ghat,
                 const uint32_t *nz_bitmap, const mr1l_extract_opts *o, const mr1l_extract_out *out)
{
    if (!p || !o || !out) return fail(MR1L_E_ARG, "plan, options or outputs NULL");
    if (n_total < 0 || (n_total > 0 && !freq) || !ghat || !nz_bitmap) return fail(MR1L_E_ARG, "null input buffer");
    if (o->cap < 1 || o->cap > kMaxCapLarge) return fail(MR1L_E_ARG, "cap must be in [1, 2^24]");
    if (o->s_cap < 1 || o->s_cap > o->cap) return fail(MR1L_E_ARG, "s_cap must be in [1, cap]");
    if (!(o->theta >= 0.0)) return fail(MR1L_E_ARG, "theta must be >= 0");
    if (o->vote_min < 0 || o->vote_min > p->L) return fail(MR1L_E_ARG, "vote_min must be in [0, L]");
    if (!out->n_det || !out->det_idx || !out->det_coef || !out->n_out || !out->out_idx || !out->out_coef)
        return fail(MR1L_E_ARG, "required output NULL");
    if (!set_off) {
        if (p->F != 1) return fail(MR1L_E_ARG, "set_off required when F > 1");
        int rc = default_offsets(*p, p->d_setoff_default, n_total, p->setoff_n);
        if (rc) return rc;
        set_off = p->d_setoff_default;
    }
    const int32_t vmin = o->vote_min ? o->vote_min : (p->L + 1) / 2;
    const int64_t F = p->F, cap = o->cap, L = p->L;
    const size_t esz = p->dtype == MR1L_C128 ? 16 : 8;
    int32_t *dh = out->det_hash;
    double *dw = out->det_w;
    uint32_t *dm = out->det_mask;
    void *dmed = out->det_med;
    int32_t *dpos = out->out_pos;
    int rc = MR1L_OK;
    if (!dh && (rc = grow(*p, (void **)&p->d_ex_hash, F * cap * L * 4, p->h_bytes))) return rc;
    if (!dh) dh = p->d_ex_hash;
    if (!dm && (rc = grow(*p, (void **)&p->d_ex_mask, F * cap * 4 * mask_words(p->L), p->m_bytes))) return rc;
    if (!dm) dm = p->d_ex_mask;
    if (!dpos && (rc = grow(*p, (void **)&p->d_ex_pos, F * o->s_cap * 4, p->pos_bytes))) return rc;
    if (!dpos) dpos = p->d_ex_pos;
    // short lists: the vote stages each detection's coordinates, the ordering pass records
    // the permutation, and the bucket pass reads them from there
    int32_t *cstage = nullptr, *perm = nullptr;
    if (cap <= kMaxCap) {
        const int64_t W = p->dot2 ? (p->d + 1) / 2 : p->d;
        if ((rc = grow(*p, (void **)&p->d_ex_cstage, F * cap * (W + 1) * 4, p->cstage_bytes))) return rc;
        cstage = p->d_ex_cstage;
        perm = p->d_ex_cstage + F * cap * W;
    }
    (void)dmed;
    (void)esz;
    if ((rc = launch_fill_bytes(out->n_det, (int64_t)sizeof(int64_t) * p->F, p->stream))) return rc;
    {
        StageTimer tm(*p, MR1L_STAGE_VOTE);
        rc = vote_run(*p, n_total, set_off, freq, nz_bitmap, vmin, cap, out->n_det, out->det_idx, out->votes,
                      cstage);
    }
    if (rc) return rc;
    StageTimer tm(*p, MR1L_STAGE_TAIL);
    return extract_tail_run(*p, n_total, set_off, freq, ghat, *o, *out, dh, dw, dm, dmed, dpos, cstage, perm);
}

int mr1l_adjoint(mr1l_plan p, int64_t cap, int64_t s_cap, const int64_t *n_out, const int32_t *out_pos,
                 const int32_t *det_hash, const double *det_w, const void *grad_out, void *grad_f)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (cap < 1 || cap > kMaxCapLarge || s_cap < 1 || s_cap > cap) return fail(MR1L_E_ARG, "invalid cap/s_cap");
    if (!n_out || !out_pos || !det_hash || !det_w || !grad_out || !grad_f)
        return fail(MR1L_E_ARG, "null buffer (out_pos, det_hash and det_w of the extract call are required)");
    return adjoint_run(*p, cap, s_cap, n_out, out_pos, det_hash, det_w, grad_out, grad_f);
}

int mr1l_graph_begin(mr1l_plan p)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (!p->stream) return fail(MR1L_E_ARG, "graph capture needs a non-default stream");
    MR1L_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    p->capturing = true;
    return MR1L_OK;
}

int mr1l_graph_end(mr1l_plan p, mr1l_graph *g)
{
    if (!p || !g) return fail(MR1L_E_ARG, "plan or graph pointer is NULL");
    p->capturing = false;
    mr1l_graph_s *G = new (std::nothrow) mr1l_graph_s();
    if (!G) return fail(MR1L_E_NOMEM, "host allocation failed");
    hipError_t e = hipStreamEndCapture(p->stream, &G->graph);
    if (e != hipSuccess) {
        delete G;
        return fail(MR1L_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(G->graph);
        delete G;
        return fail(MR1L_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    *g = G;
    return MR1L_OK;
}

int mr1l_graph_launch(mr1l_graph g, void *stream)
{
    if (!g) return fail(MR1L_E_ARG, "graph is NULL");
    MR1L_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return MR1L_OK;
}

int mr1l_graph_destroy(mr1l_graph g)
{
    if (!g) return MR1L_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return MR1L_OK;
}

int mr1l_profile(mr1l_plan p, int32_t enable)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (enable && p->capturing) return fail(MR1L_E_ARG, "cannot profile while recording a graph");
    p->profiling = enable != 0;
    return MR1L_OK;
}

int mr1l_profile_read(mr1l_plan p, double *ms, int64_t *count)
{
    if (!p || !ms || !count) return fail(MR1L_E_ARG, "null argument");
    MR1L_HIP(hipStreamSynchronize(p->stream));
    for (auto &e : p->prof) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, e.second.first, e.second.second) == hipSuccess && e.first >= 0 &&
            e.first < MR1L_NSTAGE) {
            ms[e.first] += t;
            count[e.first] += 1;
        }
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    p->prof.clear();
    return MR1L_OK;
}

int32_t mr1l_num_lattices(int64_t nJ, double c, double delta)
{
    if (nJ < 1 || !(c > 2.0) || !(delta > 0.0) || !(delta < 1.0)) return -1;
    // eq. (4.2): a quarter of the Corollary 2.7 count
    const double bound = 0.25 * (4.0 * c / ((c - 2.0) * std::log(c - 1.0))) * (std::log((double)nJ) - std::log(delta));
    int32_t L = (int32_t)std::ceil(bound);
    if (L < 1) L = 1;
    if ((L & 1) == 0) ++L;
    return L;
}

int mr1l_sample_bspline(mr1l_plan p, int32_t d_poly, int32_t n_prod, const int32_t *order, const uint64_t *dims,
                        const uint32_t *anchor, void *f)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    StageTimer tm(*p, MR1L_STAGE_SAMPLE);
    return bspline_sample_run(*p, d_poly, n_prod, order, dims, anchor, f);
}

int mr1l_lsq(mr1l_plan p, int64_t cap, const int64_t *n_det, const int64_t *det_idx, const int32_t *det_hash,
             const uint32_t *det_mask, const void *ghat, int32_t max_iter, double tol, void *coef, double *resid,
             int32_t *iters, double theta, int64_t s_cap, int64_t *n_out, int64_t *out_idx, void *out_coef)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (cap < 1 || cap > kMaxCapLarge) return fail(MR1L_E_ARG, "cap must be in [1, 2^24]");
    if (!n_det || !det_hash || !det_mask || !ghat || !coef) return fail(MR1L_E_ARG, "null input buffer");
    if (max_iter < 0 || !(tol >= 0.0)) return fail(MR1L_E_ARG, "max_iter and tol must be >= 0");
    if (n_out) {
        if (!det_idx || !out_idx || !out_coef) return fail(MR1L_E_ARG, "Algorithm 4 outputs need det_idx, out_idx, out_coef");
        if (s_cap < 1 || s_cap > cap) return fail(MR1L_E_ARG, "s_cap must be in [1, cap]");
        if (!(theta >= 0.0)) return fail(MR1L_E_ARG, "theta must be >= 0");
    }
    const int64_t esz = p->dtype == MR1L_C128 ? 16 : 8;
    const int64_t rep_bytes = ((int64_t)p->F * cap * p->L * 4 + 255) / 256 * 256;
    int rc = grow(*p, &p->d_ls, rep_bytes + 4 * (int64_t)p->F * cap * esz, p->ls_bytes);
    if (rc) return rc;
    rc = lsq_run(*p, cap, n_det, det_hash, det_mask, ghat, max_iter, tol, coef, resid, iters, (int32_t *)p->d_ls,
                 (char *)p->d_ls + rep_bytes);
    if (rc || !n_out) return rc;
    return limit_run(*p, n_det, cap, det_idx, coef, theta, s_cap, n_out, out_idx, out_coef);
}

int mr1l_pfpn_count(mr1l_plan p, int64_t cap, const int64_t *n_active, const int64_t *n_det, const int64_t *det_idx,
                    const void *det_med, const void *det_coef, double theta, int64_t *counts)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (cap < 1 || cap > kMaxCapLarge) return fail(MR1L_E_ARG, "cap must be in [1, 2^24]");
    if (!(theta >= 0.0)) return fail(MR1L_E_ARG, "theta must be >= 0");
    if (!n_active || !n_det || !det_idx || !det_med || !det_coef || !counts)
        return fail(MR1L_E_ARG, "null buffer");
    return pfpn_run(*p, cap, n_active, n_det, det_idx, det_med, det_coef, theta, counts);
}

int mr1l_check_injective(mr1l_plan p, int64_t n_total, const int64_t *set_off, const int64_t *freq, int32_t *ok)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (n_total < 0 || (n_total > 0 && !freq)) return fail(MR1L_E_ARG, "invalid candidate buffer");
    if (!set_off && p->F != 1) return fail(MR1L_E_ARG, "set_off required when F > 1");
    return check_injective_run(*p, n_total, set_off, freq, ok);
}

int mr1l_fft_schedule_count(void) { return kNumSched; }

const char *mr1l_fft_schedule_name(int32_t s) { return (s >= 0 && s < kNumSched) ? kSched[s].name : ""; }

int mr1l_plan_fft_schedule(mr1l_plan p, int64_t M, int32_t sched)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    int mid = -1;
    for (size_t i = 0; i < p->minfo.size(); ++i)
        if (p->minfo[i].M == M) mid = (int)i;
    if (mid < 0) return fail(MR1L_E_ARG, "no lattice of this size in the plan");
    if (sched < 0) return p->minfo[mid].sched;
    if (sched >= kNumSched) return fail(MR1L_E_ARG, "unknown DFT schedule");
    if (!fft_schedule_applies(p->minfo[mid], sched))
        return fail(MR1L_E_ARG, kSched[sched].rader         ? "the Rader schedule needs a prime M with M - 1 = 2^a 5^b"
                                : kSched[sched].engine == 1 ? "the reg schedule needs 2M - 1 <= 16384 (complex128) or 32768"
                                : kSched[sched].engine == 2 ? "the split schedule needs complex128 and 8192 < M <= 32768"
                                                            : "this lattice size does not fit one workgroup's LDS");
    p->minfo[mid].sched = sched;
    const int rc = fft_apply_schedules(*p);
    return rc ? rc : sched;
}

int mr1l_fft_tune(mr1l_plan p, int32_t reps, int32_t max_sizes, int64_t *sizes, float *times_ms)
{
    if (!p) return fail(MR1L_E_ARG, "plan is NULL");
    if (reps < 1 || reps > 1000) return fail(MR1L_E_ARG, "reps must be in [1, 1000]");
    if ((sizes || times_ms) && max_sizes < (int32_t)p->minfo.size())
        return fail(MR1L_E_ARG, "max_sizes is smaller than the number of distinct lattice sizes");
    const size_t esz = p->dtype == MR1L_C128 ? 16 : 8;
    void *in = nullptr, *out = nullptr;
    int rc = MR1L_OK;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(p->stream);
        if (in) (void)hipFree(in);
        if (out) (void)hipFree(out);
    };
    if (hipMalloc(&in, (size_t)std::max<int64_t>(p->nodes, 1) * esz) != hipSuccess ||
        hipMalloc(&out, (size_t)std::max<int64_t>(p->nodes, 1) * esz) != hipSuccess) {
        cleanup();
        return fail(MR1L_E_NOMEM, "allocation of the tuning buffers failed");
    }
    rc = launch_fill_bytes(in, p->nodes * (int64_t)esz, p->stream);
    // Sizes whose transforms run alike (same LDS class of the 5-smooth length, or
    // none, and the same power-of-two length) form a group and get one schedule.
    // Coordinate descent over the groups, largest first: each schedule of a group is
    // timed on the whole plan's DFT (every group launched as it runs afterwards),
    // the others held at their current schedules.
    std::map<std::pair<int, int32_t>, std::vector<int>> gmap;
    for (size_t mid = 0; mid < p->minfo.size(); ++mid) {
        const MInfo &mi = p->minfo[mid];
        gmap[{(mi.Ns ? lds_class(mi.Ns) : kLdsClasses) + (mi.rader ? 16 : 0) + (mi.Nq ? 64 * mi.Kq : 0), mi.Np}]
            .push_back((int)mid);
        if (sizes) sizes[mid] = mi.M;
    }
    std::vector<std::pair<int64_t, std::vector<int>>> groups;   // (lattice count, sizes)
    for (auto &g : gmap) {
        int64_t nl = 0;
        for (int mid : g.second) nl += p->minfo[mid].nlat;
        groups.push_back({nl, g.second});
    }
    std::stable_sort(groups.begin(), groups.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    auto set_group = [&](const std::vector<int> &mids, int s) {
        for (int mid : mids) p->minfo[mid].sched = s;
        return fft_apply_schedules(*p);
    };
    float cur_ms = 0.f;
    if (rc == MR1L_OK) rc = fft_time_plan(*p, in, out, reps, &cur_ms);
    for (size_t gi = 0; gi < groups.size() && rc == MR1L_OK; ++gi) {
        const std::vector<int> &mids = groups[gi].second;
        const int start = p->minfo[mids[0]].sched;
        int best = start;
        float best_ms = cur_ms;
        for (int s = 0; s < kNumSched && rc == MR1L_OK; ++s) {
            float ms = -1.f;
            if (s == start) {
                ms = cur_ms;
            } else if (fft_schedule_applies(p->minfo[mids[0]], s)) {
                rc = set_group(mids, s);
                if (rc == MR1L_OK) rc = fft_time_plan(*p, in, out, reps, &ms);
                if (rc == MR1L_OK && ms < best_ms) { best_ms = ms; best = s; }
            }
            if (times_ms)
                for (int mid : mids) times_ms[mid * kNumSched + s] = ms;
        }
        if (rc == MR1L_OK) rc = set_group(mids, best);
        cur_ms = best_ms;
        for (int mid : mids) record_tuned(p->dtype, p->minfo[mid].M, best);
    }
    cleanup();
    if (rc) return rc;
    return fft_apply_schedules(*p);
}

}  // extern "C"
