// Host side of the thin-disk force solver: validation, planning of the four
// FFT passes for a nested hierarchy, resident kernel spectra, solves,
// batches (one launch per pass and transform length for many hierarchies,
// optionally replayed from a HIP graph), the serving loop and the
// launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <fstream>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "td_fft.hpp"
#include "td_launch.h"
#include "thindisk.h"

using namespace td;

namespace {

thread_local std::string g_err;

td_status fail(td_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define TD_HIP(expr)                                                                       \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return fail(TD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));    \
    } while (0)

// The HIP runtime keeps a per-thread "last error" that the caller's own
// code (PyTorch checks it after every kernel launch) reads.  Entry points
// leave it as they found it: an error the library's own calls raised and
// handled (a query of an unfinished event, an allocation refused and
// retried) is cleared on the way out unless one was already pending.
struct ErrScope {
    bool clean;
    ErrScope() : clean(hipPeekAtLastError() == hipSuccess) {}
    ~ErrScope()
    {
        if (clean) (void)hipGetLastError();
    }
};

#define TD_TRY(expr)                    \
    do {                                \
        td_status _s = (expr);          \
        if (_s != TD_OK) return _s;     \
    } while (0)

int floor_div(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
int ceil_div(int a, int b) { return -floor_div(-a, b); }

int ipow(int b, int e)
{
    int r = 1;
    while (e-- > 0) r *= b;
    return r;
}

int fft_len(int n)
{
    int M = 16;
    while (M < 2 * n) M *= 2;
    return M;
}

size_t elem_size(td_dtype dt) { return dt == TD_F64 ? 16 : 8; }  // complex element

// Launch-shape passes; timing adds a fourth slot for the accumulating
// row-inverse launches.
enum Pass { P_ROWFWD = 0, P_COL = 1, P_ROWINV = 2, NSHAPE = 3, NTIMED = 4 };

// Kernel feeding output component c (0: Fx, 1: Fy) from field f (sigma,
// dsdx, dsdy): I0, Ixx, Ixy for Fx and J0, Jyx, Jyy for Fy.
const int kKernOfHost[2][3] = {{0, 1, 2}, {3, 5, 4}};

// Launch shape of a pass: C sequences (row passes) or C columns x G slots
// (column passes), packed as C | G << 16.
int shape_C(int v) { return v & 0xffff; }
int shape_G(int v) { return std::max(1, v >> 16); }
int pack_shape(int C, int G) { return C | (G << 16); }

// Default launch shapes (from autotuning on gfx950): row FFTs 256 threads;
// the column pass and the row inverse one column / row per workgroup with
// up to 16 slots, 512 threads up to M = 256 and 256 threads beyond, except
// the row inverse at M = 512: two rows of 4 slots (512 threads); LDS
// <= 64 KiB.
int default_shape(int pass, int M, td_dtype dt)
{
    const size_t es = elem_size(dt);
    if (pass == P_ROWFWD) {
        int S = std::max(1, 2048 / M);
        while (S > 1 && lds_bytes(M, S, es) > 64 * 1024) S /= 2;
        return pack_shape(S, 1);
    }
    if (pass == P_ROWINV && M == 512 && lds_bytes(M, 2, es, 4) <= 64 * 1024) return pack_shape(2, 4);
    int S = std::max(1, (M <= 256 ? 4096 : 2048) / M);
    int G = std::min(16, S);
    int C = std::max(1, S / G);
    while (C > 1 && lds_bytes(M, C, es, G) > 64 * 1024) C /= 2;
    while (G > 1 && lds_bytes(M, C, es, G) > 64 * 1024) G /= 2;
    return pack_shape(C, G);
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

// ===========================================================================
// context
// ===========================================================================

struct SpecEntry {
    void* ptr = nullptr;
    size_t bytes = 0;
    int nphase = 0;
};

struct td_context {
    int device = 0;
    int cus = 256;  // compute units of the device
    size_t budget = 0;
    std::atomic<size_t> used{0};
    std::atomic<size_t> spectra_bytes{0};
    std::recursive_mutex mu;
    std::map<int, void*> tw32, tw64;
    // (M, kind, m, dtype, family, aspect)
    std::map<std::tuple<int, int, int, int, int, double>, SpecEntry> spectra;
    std::map<std::tuple<int, int, int>, int> tune;               // (pass, M, dtype) -> shape
    hipStream_t stream = nullptr;                                 // plan-time work
    std::vector<void*> allocs;
    // Scratch of the kernel-spectrum builds (FP64 tables and their row
    // transforms), kept between builds and grown when a longer lattice
    // appears, so that a build frees nothing (hipFree waits for the whole
    // device, flights included).  Used under mu, on `stream` only.
    void* b_table = nullptr;
    size_t b_table_bytes = 0;
    void* b_rows = nullptr;
    size_t b_rows_bytes = 0;
    void* b_small = nullptr;  // pointer table, level table, row jobs
    size_t b_small_bytes = 0;
    // debug mode (td_context_set_debug): non-finite outputs are counted here
    std::atomic<int> debug{0};
    unsigned long long* d_nonfinite = nullptr;
    // per-pass timing (diagnostics)
    bool timing = false;
    int timing_mask = 0;  // launch kinds timed (bit per kind)
    struct Timed { int pass; hipEvent_t a, b; };
    std::deque<Timed> timed;
    std::vector<hipEvent_t> ev_pool;
    double t_ms[NTIMED] = {0, 0, 0, 0};
    int64_t t_n[NTIMED] = {0, 0, 0, 0};
    // Fold the timed launches that have completed into the totals and
    // return their events to the pool (oldest first, stopping at the first
    // still in flight), so that a long timed run reuses a few events
    // instead of creating two per launch.
    void harvest_timed()
    {
        while (!timed.empty() && hipEventQuery(timed.front().b) == hipSuccess) {
            const Timed t = timed.front();
            timed.pop_front();
            float e = 0;
            if (hipEventElapsedTime(&e, t.a, t.b) == hipSuccess) {
                t_ms[t.pass] += e;
                t_n[t.pass] += 1;
            }
            ev_pool.push_back(t.a);
            ev_pool.push_back(t.b);
        }
    }
    hipEvent_t get_event()
    {
        hipEvent_t e = nullptr;
        if (ev_pool.empty()) harvest_timed();
        if (!ev_pool.empty()) {
            e = ev_pool.back();
            ev_pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }

    td_status alloc(size_t bytes, void** out)
    {
        if (budget && used.load() + bytes > budget)
            return fail(TD_ENOMEM, "HBM budget exceeded: need " + std::to_string(bytes) +
                                       " more bytes, " + std::to_string(used.load()) + " of " +
                                       std::to_string(budget) + " in use");
        hipError_t e = hipMalloc(out, bytes ? bytes : 16);
        if (e != hipSuccess) return fail(TD_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        used += bytes;
        return TD_OK;
    }
    void release(void* p, size_t bytes)
    {
        if (p) {
            (void)hipFree(p);
            used -= bytes;
        }
    }
    int shape(int pass, int M, td_dtype dt)
    {
        std::lock_guard<std::recursive_mutex> lk(mu);
        auto it = tune.find(std::make_tuple(pass, M, (int)dt));
        return it != tune.end() ? it->second : default_shape(pass, M, dt);
    }
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

td_status twiddles(td_context* ctx, int M, td_dtype dt, const void** out)
{
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto& tab = dt == TD_F64 ? ctx->tw64 : ctx->tw32;
    auto it = tab.find(M);
    if (it != tab.end()) {
        *out = it->second;
        return TD_OK;
    }
    std::vector<double> h64(2 * (size_t)M, 0.0);
    std::vector<float> h32(2 * (size_t)M, 0.0f);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    // per-pass layout of fft_lds: entry tw_offset(M, NS) + (r-1) NS + k holds
    // exp(-2 pi i r k / (8 NS)) = exp(-2 pi i e / M), e = r k M / (8 NS)
    for (int NS = tw_first_span(M); NS < M; NS *= 8)
        for (int r = 1; r < 8; ++r)
            for (int k = 0; k < NS; ++k) {
                const int idx = tw_offset(M, NS) + (r - 1) * NS + k;
                const long long e = ((long long)r * k * (M / (8 * NS))) % M;
                long double a = two_pi * (long double)e / (long double)M;
                long double c = cosl(a), s = -sinl(a);
                if (4 * e == M) { c = 0; s = -1; }
                if (2 * e == M) { c = -1; s = 0; }
                if (4 * e == 3LL * M) { c = 0; s = 1; }
                if (e == 0) { c = 1; s = 0; }
                h64[2 * idx] = (double)c;
                h64[2 * idx + 1] = (double)s;
                h32[2 * idx] = (float)c;
                h32[2 * idx + 1] = (float)s;
            }
    size_t bytes = (dt == TD_F64 ? sizeof(double) : sizeof(float)) * 2 * (size_t)M;
    void* d = nullptr;
    TD_TRY(ctx->alloc(bytes, &d));
    TD_HIP(hipMemcpy(d, dt == TD_F64 ? (void*)h64.data() : (void*)h32.data(), bytes,
                     hipMemcpyHostToDevice));
    tab[M] = d;
    ctx->allocs.push_back(d);
    *out = d;
    return TD_OK;
}

template <typename Job>
SegTable<Job> single_seg(const Job* jobs, int n, int slot_base, const void* aux, char* ws)
{
    SegTable<Job> s;
    memset(&s, 0, sizeof(s));
    s.nseg = 1;
    s.start[0] = 0;
    s.start[1] = n;
    s.slot_base[0] = slot_base;
    s.jobs[0] = jobs;
    s.aux[0] = aux;
    s.ws[0] = ws;
    return s;
}

// Build (once per context) the kernel spectra of one (M, kind, m, dtype,
// family); family 1 holds the potential tables (P0, Px, Py, zero planes).
// Stored phases: kind 1 -> (0,0); kinds 2/3 -> (kx, ky) in [0, hp)^2 with
// hp = ceil(m/2), the others being mirror images (for odd m the middle
// phase of each axis is its own mirror).  Layout [phase][X][M/2+1][M].
td_status spectra(td_context* ctx, int M, int kind, int m, td_dtype dt, int family,
                  double aspect, const SpecEntry** out)
{
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto key = std::make_tuple(M, kind, m, (int)dt, family, aspect);
    auto it = ctx->spectra.find(key);
    if (it != ctx->spectra.end()) {
        *out = &it->second;
        return TD_OK;
    }
    const int hp = (kind == 1) ? 1 : (m + 1) / 2;
    const int nphase = hp * hp;
    const size_t NCOL = M / 2 + 1;
    const size_t per_phase = 6 * NCOL * (size_t)M;
    const bool quarter = kind == 1;  // one real per frequency, ky <= M/2
    SpecEntry e;
    e.nphase = nphase;
    e.bytes = quarter ? 6 * NCOL * NCOL * elem_size(dt) / 2 : per_phase * nphase * elem_size(dt);
    TD_TRY(ctx->alloc(e.bytes, &e.ptr));
    // FP64 scratch: the six real tables, their row transforms, and the
    // small tables of the row launch (6 plane pointers, the level table of
    // one M x M patch, the row jobs)
    const int C = std::max(1, std::min(shape_C(default_shape(P_ROWFWD, M, TD_F64)), TD_MAX_THREADS / (M / 8)));
    std::vector<RowFwdJob> jobs;
    for (int X = 0; X < 6; ++X)
        for (int r0 = 0; r0 < M; r0 += 2 * C) {
            RowFwdJob j;
            memset(&j, 0, sizeof(j));
            j.lvl = 0;
            j.f = X;
            j.m = 1;
            j.ld = M;
            j.row0 = r0;
            j.nrow = std::min(2 * C, M - r0);
            j.scale = 1.0;
            j.est_scale = 1.0;
            j.lc_lo = 0;
            j.lc_hi = M;
            j.out = (int64_t)(X * NCOL * (size_t)M * 16);
            jobs.push_back(j);
        }
    const size_t tbytes = 6 * (size_t)M * M * sizeof(double);
    const size_t rbytes = per_phase * 16;
    const size_t o_lp = 256, o_jobs = 256 + ((sizeof(LevelPatches) + 255) & ~size_t(255));
    const size_t sbytes = o_jobs + jobs.size() * sizeof(RowFwdJob);
    td_status st = TD_OK;
    if (ctx->b_table_bytes < tbytes || ctx->b_rows_bytes < rbytes || ctx->b_small_bytes < sbytes) {
        // earlier builds on the stream still read the old scratch
        hipError_t he = hipStreamSynchronize(ctx->stream);
        if (he != hipSuccess) st = fail(TD_EDEVICE, hipGetErrorString(he));
        if (st == TD_OK && ctx->b_table_bytes < tbytes) {
            ctx->release(ctx->b_table, ctx->b_table_bytes);
            ctx->b_table = nullptr;
            ctx->b_table_bytes = 0;
            st = ctx->alloc(tbytes, &ctx->b_table);
            if (st == TD_OK) ctx->b_table_bytes = tbytes;
        }
        if (st == TD_OK && ctx->b_rows_bytes < rbytes) {
            ctx->release(ctx->b_rows, ctx->b_rows_bytes);
            ctx->b_rows = nullptr;
            ctx->b_rows_bytes = 0;
            st = ctx->alloc(rbytes, &ctx->b_rows);
            if (st == TD_OK) ctx->b_rows_bytes = rbytes;
        }
        if (st == TD_OK && ctx->b_small_bytes < sbytes) {
            ctx->release(ctx->b_small, ctx->b_small_bytes);
            ctx->b_small = nullptr;
            ctx->b_small_bytes = 0;
            st = ctx->alloc(sbytes, &ctx->b_small);
            if (st == TD_OK) ctx->b_small_bytes = sbytes;
        }
    }
    void* table = ctx->b_table;
    void* rows = ctx->b_rows;
    void* dptr = ctx->b_small;
    void* dlp = (char*)ctx->b_small + o_lp;
    RowFwdJob* djobs = (RowFwdJob*)((char*)ctx->b_small + o_jobs);
    const void* tw64 = nullptr;
    if (st == TD_OK) st = twiddles(ctx, M, TD_F64, &tw64);
    // the small tables, staged once in host memory and copied in stream
    // order (an earlier build's launches may still read the previous ones)
    std::vector<char> hsmall(sbytes, 0);
    {
        void* hp_ptr[6];
        for (int X = 0; X < 6; ++X) hp_ptr[X] = (char*)table + X * (size_t)M * M * sizeof(double);
        memcpy(hsmall.data(), hp_ptr, sizeof(hp_ptr));
        LevelPatches lp;
        memset(&lp, 0, sizeof(lp));
        lp.np = 1;
        lp.pn[0] = M;
        memcpy(hsmall.data() + o_lp, &lp, sizeof(lp));
        memcpy(hsmall.data() + o_jobs, jobs.data(), jobs.size() * sizeof(RowFwdJob));
    }
    if (st == TD_OK) {
        hipError_t he = hipMemcpyAsync(dptr, hsmall.data(), sbytes, hipMemcpyHostToDevice, ctx->stream);
        if (he != hipSuccess) st = fail(TD_EDEVICE, hipGetErrorString(he));
    }
    for (int p = 0; st == TD_OK && p < nphase; ++p) {
        TableJob tj;
        memset(&tj, 0, sizeof(tj));
        tj.M = M;
        tj.kind = kind;
        tj.m = (kind == 1) ? 1 : m;
        tj.kx = p % hp;
        tj.ky = p / hp;
        tj.family = family;
        tj.aspect = aspect;
        tj.out = (double*)table;
        hipError_t he = launch_table(tj, ctx->stream);
        if (he == hipSuccess)
            he = launch_row_fwd<double>(M, C, (int)jobs.size(),
                                        single_seg<RowFwdJob>(djobs, (int)jobs.size(), 0, dlp, (char*)rows),
                                        (const void* const*)dptr, FieldPtrs{}, tw64, false, ctx->stream);
        const int Cs = std::max(1, std::min(shape_C(default_shape(P_ROWINV, M, TD_F64)), TD_MAX_THREADS / (M / 8)));
        void* dst = (char*)e.ptr + (size_t)p * per_phase * elem_size(dt);
        if (he == hipSuccess)
            he = dt == TD_F64
                     ? launch_spec_col<double>(M, Cs, rows, dst, tw64, quarter | (family << 1), ctx->stream)
                     : launch_spec_col<float>(M, Cs, rows, dst, tw64, quarter | (family << 1), ctx->stream);
        if (he != hipSuccess) st = fail(TD_EDEVICE, std::string("kernel-table build: ") + hipGetErrorString(he));
    }
    // the staged small tables must outlive their copy, and the entry is
    // complete for every stream once this returns
    if (st == TD_OK) {
        hipError_t he = hipStreamSynchronize(ctx->stream);
        if (he != hipSuccess) st = fail(TD_EDEVICE, std::string("kernel-table build: ") + hipGetErrorString(he));
    } else {
        (void)hipStreamSynchronize(ctx->stream);
    }
    if (st != TD_OK) {
        ctx->release(e.ptr, e.bytes);
        return st;
    }
    ctx->spectra_bytes += e.bytes;
    auto ins = ctx->spectra.emplace(key, e);
    *out = &ins.first->second;
    return TD_OK;
}

}  // namespace

// ===========================================================================
// hierarchy validation
// ===========================================================================

namespace {

// Level of every patch and the index of each level's first patch; checks
// that patches are grouped by level, level 0 first, with one level-0 patch.
td_status patch_levels(const td_hierarchy* h, int* nlevels)
{
    if (!h || !h->patches) return fail(TD_EINVAL, "hierarchy or patches is NULL");
    if (h->npatches < 1 || h->npatches > TD_MAX_PATCHES)
        return fail(TD_EINVAL, "npatches must be in 1.." + std::to_string(TD_MAX_PATCHES));
    const td_patch* P = h->patches;
    if (P[0].level != 0) return fail(TD_EINVAL, "the first patch must be the level-0 patch");
    std::vector<int> count(1, 1);
    for (int k = 1; k < h->npatches; ++k) {
        const int l = P[k].level, prev = P[k - 1].level;
        if (l != prev && l != prev + 1)
            return fail(TD_EINVAL, "patches must be grouped by level in increasing order");
        if (l == 0) return fail(TD_EINVAL, "exactly one level-0 patch");
        if (l == (int)count.size()) count.push_back(0);
        count[l] += 1;
    }
    if ((int)count.size() > TD_MAX_LEVELS)
        return fail(TD_EINVAL, "at most " + std::to_string(TD_MAX_LEVELS) + " levels");
    for (int c : count)
        if (c > TD_PATCHES_PER_LEVEL)
            return fail(TD_EINVAL, "at most " + std::to_string(TD_PATCHES_PER_LEVEL) + " patches per level");
    *nlevels = (int)count.size();
    return TD_OK;
}

// Bounding rectangle of a level's patches (level cells): origin and size.
void level_window(const td_hierarchy* h, int level, int* ox, int* oy, int* nx, int* ny)
{
    int x0 = INT32_MAX, y0 = INT32_MAX, x1 = INT32_MIN, y1 = INT32_MIN;
    for (int k = 0; k < h->npatches; ++k) {
        const td_patch& p = h->patches[k];
        if (p.level != level) continue;
        x0 = std::min(x0, p.ox);
        y0 = std::min(y0, p.oy);
        x1 = std::max(x1, p.ox + p.n);
        y1 = std::max(y1, p.oy + p.n);
    }
    *ox = x0;
    *oy = y0;
    *nx = x1 - x0;
    *ny = y1 - y0;
}

}  // namespace

extern "C" td_status td_hierarchy_check(const td_hierarchy* h)
{
    ErrScope es_;
    int L = 0;
    TD_TRY(patch_levels(h, &L));
    if (!std::isfinite(h->aspect) || h->aspect < 0 ||
        (h->aspect != 0 && (h->aspect < 1.0 / 64 || h->aspect > 64)))
        return fail(TD_EINVAL, "aspect must be 0 (square cells) or in [1/64, 64]");
    if (h->ratio < 2 || h->ratio > 4)
        return fail(TD_EUNSUPPORTED, "refinement ratio must be 2, 3 or 4");
    if (!(h->h0 > 0) || !std::isfinite(h->h0) || !std::isfinite(h->x0) || !std::isfinite(h->y0))
        return fail(TD_EINVAL, "h0 must be positive and x0, y0, h0 finite");
    const td_patch* P = h->patches;
    if (P[0].ox != 0 || P[0].oy != 0) return fail(TD_EINVAL, "level-0 offsets must be 0");
    const int r = h->ratio;
    if (ipow(r, L - 1) > 16)
        return fail(TD_EUNSUPPORTED, "levels may differ in resolution by at most 16x (ratio^(levels-1) <= 16)");
    for (int k = 0; k < h->npatches; ++k) {
        const td_patch& p = P[k];
        const std::string who = "patch " + std::to_string(k) + " (level " + std::to_string(p.level) + ")";
        if (p.n < 1 || p.n > TD_MAX_N)
            return fail(TD_EINVAL, who + ": n must be in 1.." + std::to_string(TD_MAX_N));
        if (p.ox < 0 || p.oy < 0) return fail(TD_ENEST, who + ": negative offset");
        if (p.level == 0) continue;
        long span = 1;
        for (int l = 0; l < p.level; ++l) span *= r;
        if (span * (long)P[0].n > (1L << 30)) return fail(TD_EINVAL, "hierarchy too deep");
        if (p.n % r || p.ox % r || p.oy % r)
            return fail(TD_EALIGN, who + ": size and offsets must be multiples of the ratio");
        // inside one patch of the level above
        const int px0 = p.ox / r, py0 = p.oy / r, w = p.n / r;
        bool inside = false;
        for (int q = 0; q < h->npatches; ++q) {
            const td_patch& u = P[q];
            inside |= u.level == p.level - 1 && px0 >= u.ox && py0 >= u.oy &&
                      px0 + w <= u.ox + u.n && py0 + w <= u.oy + u.n;
        }
        if (!inside) return fail(TD_ENEST, who + " is not inside a patch of level " + std::to_string(p.level - 1));
        // no overlap with another patch of the same level
        for (int q = 0; q < k; ++q) {
            const td_patch& u = P[q];
            if (u.level == p.level && p.ox < u.ox + u.n && u.ox < p.ox + p.n && p.oy < u.oy + u.n &&
                u.oy < p.oy + p.n)
                return fail(TD_EINVAL, who + " overlaps patch " + std::to_string(q));
        }
    }
    for (int l = 0; l < L; ++l) {
        int ox, oy, nx, ny;
        level_window(h, l, &ox, &oy, &nx, &ny);
        if (nx > TD_MAX_N || ny > TD_MAX_N)
            return fail(TD_EUNSUPPORTED, "level " + std::to_string(l) + ": patches span more than " +
                                             std::to_string(TD_MAX_N) + " cells");
    }
    return TD_OK;
}

extern "C" td_status td_hierarchy_snap(td_hierarchy* h, td_patch* patches, const double* cx,
                                       const double* cy)
{
    ErrScope es_;
    if (!h || !patches || (h->npatches > 1 && (!cx || !cy))) return fail(TD_EINVAL, "NULL argument");
    if (h->npatches < 1 || h->npatches > TD_MAX_LEVELS) return fail(TD_EINVAL, "bad npatches");
    if (h->ratio < 2 || h->ratio > 4) return fail(TD_EUNSUPPORTED, "ratio must be 2, 3 or 4");
    for (int l = 0; l < h->npatches; ++l)
        if (patches[l].level != l) return fail(TD_EINVAL, "snap takes one patch per level, patch l on level l");
    patches[0].ox = patches[0].oy = 0;
    double hh = h->h0;
    const double asp = h->aspect > 0 ? h->aspect : 1.0;
    for (int l = 1; l < h->npatches; ++l) {
        const int r = h->ratio, n = patches[l].n, pn = patches[l - 1].n;
        if (n % r) return fail(TD_EALIGN, "child size must be a multiple of the ratio");
        const int span = n / r;
        if (span > pn) return fail(TD_ENEST, "child wider than its parent");
        const double px0 = h->x0 + patches[l - 1].ox * hh, py0 = h->y0 + patches[l - 1].oy * hh * asp;
        const double ext = n * hh / r;
        long kx = (long)std::floor((cx[l - 1] - ext / 2 - px0) / hh + 0.5);
        long ky = (long)std::floor((cy[l - 1] - ext * asp / 2 - py0) / (hh * asp) + 0.5);
        kx = std::min<long>(std::max<long>(kx, 0), pn - span);
        ky = std::min<long>(std::max<long>(ky, 0), pn - span);
        patches[l].ox = r * (patches[l - 1].ox + (int)kx);
        patches[l].oy = r * (patches[l - 1].oy + (int)ky);
        hh /= r;
    }
    h->patches = patches;
    return TD_OK;
}

// ===========================================================================
// planning
// ===========================================================================

namespace {

// Jobs of one transform length M, on the host and on the device.
struct Group {
    int M = 0;
    const void* tw = nullptr;    // twiddles of length M in the plan's dtype
    int C[NSHAPE] = {1, 1, 1};   // sequences / columns / rows per workgroup
    int G[NSHAPE] = {1, 1, 1};   // slots per column or row
    std::vector<RowFwdJob> rowfwd;
    std::vector<ColJob> col;
    std::vector<ColIn> colins;
    std::vector<ColOut> colouts;
    std::vector<RowInvJob> rinv[2];  // [0] write, [1] accumulate
    int nq[2] = {1, 1};              // row inverse: most outputs per thread and row
    std::vector<RowInvContrib> contribs;
    // device copies
    RowFwdJob* d_rowfwd = nullptr;
    ColJob* d_col = nullptr;
    ColIn* d_colins = nullptr;
    ColOut* d_colouts = nullptr;
    void* d_coltabs = nullptr;  // {d_colins, d_colouts}
    RowInvJob* d_rinv[2] = {nullptr, nullptr};
    RowInvContrib* d_contribs = nullptr;
    RowInvTables* d_rinv_tabs = nullptr;  // {d_contribs, the plan's level tables}
};

// A level's window (bounding rectangle of its patches, level cells) and
// transform length.
struct LevelG {
    int ox, oy, nx, ny, M;
    double h;
};

}  // namespace

struct td_plan {
    td_context* ctx = nullptr;
    bool dry = false;          // host-only planning: no spectra, no device memory
    td_dtype dt = TD_F32;
    int quantity = TD_FORCE;   // TD_FORCE (Fx, Fy) or TD_POTENTIAL (Phi into fx)
    double aspect = 1.0;       // cell height / width
    int ratio = 2;
    int nlevels = 0;
    int npatches = 0;
    std::vector<LevelG> lv;
    std::vector<LevelPatches> lp;          // per level, for the row kernels
    std::vector<int> patch_n;              // side of every patch
    LevelPatches* d_lp = nullptr;
    double x0 = 0, y0 = 0, h0 = 0;
    std::vector<Group> groups;
    void* ws = nullptr;        // workspace for td_solve, allocated on first use
    size_t ws_bytes = 0;
    size_t spectra_bytes = 0;  // resident spectra this plan reads
    size_t job_bytes = 0;
    std::vector<std::pair<void*, size_t>> dev_allocs;
    uint64_t id = 0;
};

namespace {

std::atomic<uint64_t> g_plan_ids{1};

template <typename V>
td_status upload(td_context* ctx, td_plan* p, const std::vector<V>& v, V** out)
{
    *out = nullptr;
    if (v.empty()) return TD_OK;
    const size_t b = v.size() * sizeof(V);
    void* d = nullptr;
    TD_TRY(ctx->alloc(b, &d));
    p->dev_allocs.push_back({d, b});
    p->job_bytes += b;
    TD_HIP(hipMemcpy(d, v.data(), b, hipMemcpyHostToDevice));
    *out = (V*)d;
    return TD_OK;
}

Group& group_for(std::vector<Group>& groups, int M)
{
    for (auto& g : groups)
        if (g.M == M) return g;
    groups.push_back(Group());
    groups.back().M = M;
    return groups.back();
}

// Every polyphase phase (kx, ky) of ratio m, ordered so that the mirror
// images of each stored phase (sx, sy) in [0, ceil(m/2))^2 come one after
// another (two or one of them on an axis whose middle phase, odd m, is its
// own mirror).
std::vector<std::pair<int, int>> phase_order(int m)
{
    std::vector<std::pair<int, int>> out;
    const int hp = (m + 1) / 2;
    for (int sy = 0; sy < hp; ++sy)
        for (int sx = 0; sx < hp; ++sx)
            for (int mir = 0; mir < 4; ++mir) {
                const int kx = (mir & 1) ? m - 1 - sx : sx, ky = (mir & 2) ? m - 1 - sy : sy;
                if (((mir & 1) && kx == sx) || ((mir & 2) && ky == sy)) continue;  // self-mirror
                out.push_back({kx, ky});
            }
    return out;
}

// Stored spectra of phase (kx, ky) within an entry, and the mirror bits
// that map them onto it.
const void* phase_kernels(const SpecEntry* e, int m, int kx, int ky, size_t per_phase_bytes, int* flip)
{
    const int hp = (m + 1) / 2;
    const int sx = std::min(kx, m - 1 - kx), sy = std::min(ky, m - 1 - ky);
    *flip = (kx >= hp ? 1 : 0) | (ky >= hp ? 2 : 0);
    return (const char*)e->ptr + (size_t)(sy * hp + sx) * per_phase_bytes;
}


// Kernel spectra of a plan; a dry (host-only) plan gets a stand-in entry
// whose address is never dereferenced.
td_status plan_spectra(td_plan* P, int M, int kind, int m, const SpecEntry** out)
{
    if (!P->dry) return spectra(P->ctx, M, kind, m, P->dt, P->quantity, P->aspect, out);
    static SpecEntry fake;
    const int hp = kind == 1 ? 1 : (m + 1) / 2;
    fake.ptr = (void*)(uintptr_t)4096;
    fake.nphase = hp * hp;
    fake.bytes = (size_t)hp * hp * 6 * (M / 2 + 1) * (size_t)M * elem_size(P->dt);
    *out = &fake;
    return TD_OK;
}

// Multipliers of a row-forward job reading field f of a level with cell
// width h (height aspect h).  The force tables are dimensionless, in units of
// the cell width: sigma enters as read, a given slope as h * slope (x and y
// alike), an estimated one (a difference per cell) as it is along x and
// divided by the aspect along y.  The potential carries one more length and
// the sign of the Green's function -1/rho, so every multiplier takes a
// further -h (the tables are in units of the pair's finer cell; Case-3
// tables absorb the ratio to a coarser source's h).
void row_scales(const td_plan* P, double h, int f, RowFwdJob* j)
{
    const double q = P->quantity == TD_POTENTIAL ? -h : 1.0;
    j->scale = f == 0 ? q : q * h;
    j->est_scale = f == 2 ? q / P->aspect : q;
}

// The lattice columns lc of a row job whose source column m lc + col_off
// lies inside the source level's window [0, nx): the others read nothing.
void row_columns(RowFwdJob* j, int nx, int ncols)
{
    const int lo = ceil_div(-j->col_off, j->m), hi = ceil_div(nx - j->col_off, j->m);
    j->lc_lo = std::max(0, std::min(lo, ncols));
    j->lc_hi = std::max(j->lc_lo, std::min(hi, ncols));
}

// Emit every job of a plan (workspace addresses as byte offsets) and the
// workspace size in complex elements.
//
// Workspace per lattice t (level t's zero-padded M x M grid):
//   own_in[t]      3 row-pass planes [M/2+1][ny_t] of level t's fields
//   ph_in[s][t]    per finer level s: m^2 phases x 3 row-pass planes
//                  [M/2+1][nr] of the polyphase sub-grids on lattice t
//   own_out[t]     Fx, Fy column outputs [M/2+1][ny_t]
//   c3_out[t][s]   per finer level s: m^2 phases x (Fx, Fy) outputs
//                  [M/2+1][ld] on lattice t for target level s
td_status build_jobs(td_plan* P, size_t* ws_elems, bool emit)
{
    td_context* ctx = P->ctx;
    const int L = P->nlevels, r = P->ratio;
    const size_t es = elem_size(P->dt);
    size_t off = 0;  // complex elements
    auto take = [&](size_t n) {
        size_t o = off;
        off += (n + 31) & ~size_t(31);  // 256-byte aligned sub-buffers for FP32
        return o;
    };
    auto ptr = [&](size_t o) -> int64_t { return (int64_t)(o * es); };
    // ---- workspace layout
    std::vector<size_t> own_in(L), own_out(L);
    std::vector<std::vector<size_t>> ph_in(L, std::vector<size_t>(L)), c3_out(L, std::vector<size_t>(L));
    std::vector<std::vector<int>> ph_nr(L, std::vector<int>(L)), c3_ld(L, std::vector<int>(L));
    for (int l = 0; l < L; ++l) {
        const LevelG& g = P->lv[l];
        const size_t H = g.M / 2 + 1;
        own_in[l] = take(3 * H * g.ny);
        own_out[l] = take(2 * H * g.ny);
    }
    for (int t = 0; t < L; ++t)
        for (int s = t + 1; s < L; ++s) {
            const int m = ipow(r, s - t);
            const LevelG &G = P->lv[t], &S = P->lv[s];
            const size_t H = G.M / 2 + 1;
            const int nr = (S.ny + m - 1) / m + 1;
            ph_nr[s][t] = nr;
            ph_in[s][t] = take((size_t)m * m * 3 * H * nr);
            // coarser source t, finer target s: Case-3 outputs on lattice t
            const int ld = floor_div(S.oy + S.ny - 1, m) - floor_div(S.oy, m) + 1;
            c3_ld[t][s] = ld;
            c3_out[t][s] = take((size_t)m * m * 2 * H * ld);
        }
    *ws_elems = off;
    if (!emit) return TD_OK;

    P->groups.clear();
    for (int l = 0; l < L; ++l) {
        Group& g = group_for(P->groups, P->lv[l].M);
        for (int pass = 0; pass < NSHAPE; ++pass) {
            const int v = ctx->shape(pass, g.M, P->dt);
            g.C[pass] = shape_C(v);
            g.G[pass] = shape_G(v);
        }
    }
    // ---- pass 1: row FFTs of every input plane
    for (int l = 0; l < L; ++l) {
        const LevelG& G = P->lv[l];
        Group& g = group_for(P->groups, G.M);
        const int R = 2 * g.C[P_ROWFWD];
        const size_t H = G.M / 2 + 1, plane = H * G.ny;
        for (int f = 0; f < 3; ++f) {
            for (int r0 = 0; r0 < G.ny; r0 += R) {
                RowFwdJob j;
                memset(&j, 0, sizeof(j));
                j.lvl = l;
                j.f = f;
                j.m = 1;
                j.ld = G.ny;
                j.row0 = r0;
                j.nrow = std::min(R, G.ny - r0);
                row_scales(P, G.h, f, &j);
                row_columns(&j, G.nx, G.M / 2);
                j.out = ptr(own_in[l] + f * plane);
                g.rowfwd.push_back(j);
            }
        }
        // polyphase sub-grids of every finer level s, placed on this lattice
        for (int s = l + 1; s < L; ++s) {
            const LevelG& S = P->lv[s];
            const int m = ipow(r, s - l), nr = ph_nr[s][l];
            for (int ky = 0; ky < m; ++ky)
                for (int kx = 0; kx < m; ++kx) {
                    const int lr_lo = ceil_div(S.oy - ky, m) - G.oy;
                    const int lr_hi = floor_div(S.oy + S.ny - 1 - ky, m) - G.oy;
                    if (lr_hi < lr_lo) continue;
                    const int phase = ky * m + kx;
                    // every stored row is written (rows past the source are
                    // zeros), since the column pass reads all nr of them
                    for (int f = 0; f < 3; ++f) {
                        const size_t in = ph_in[s][l] + ((size_t)phase * 3 + f) * H * nr;
                        for (int r0 = 0; r0 < nr; r0 += R) {
                            RowFwdJob j;
                            memset(&j, 0, sizeof(j));
                            j.lvl = s;
                            j.f = f;
                            j.m = m;
                            j.row_off = m * G.oy + ky - S.oy;
                            j.col_off = m * G.ox + kx - S.ox;
                            j.lr_first = lr_lo;
                            j.ld = nr;
                            j.row0 = r0;
                            j.nrow = std::min(R, nr - r0);
                            row_scales(P, S.h, f, &j);
                            row_columns(&j, S.nx, G.M / 2);
                            j.out = ptr(in);
                            g.rowfwd.push_back(j);
                        }
                    }
                }
        }
    }
    // Row-forward jobs gather the lattice columns [lc_lo, lc_hi) of their
    // source (a level's own rows: its width; a ratio-m phase: 1/m of it),
    // then transform and write the same M/2 + 1 frequencies: the widest
    // gathers run first, so the cheaper phase rows fill the tail.  (Each
    // plane's jobs stay consecutive, in row order.)
    for (auto& g : P->groups)
        std::stable_sort(g.rowfwd.begin(), g.rowfwd.end(), [](const RowFwdJob& a, const RowFwdJob& b) {
            return a.lc_hi - a.lc_lo > b.lc_hi - b.lc_lo;
        });
    // ---- pass 2: column transforms, products and inverse column
    // transforms, per lattice
    const int fam = P->quantity == TD_POTENTIAL ? 8 : 0;  // kernel family bit
    for (int t = 0; t < L; ++t) {
        const LevelG& G = P->lv[t];
        Group& g = group_for(P->groups, G.M);
        const size_t H = G.M / 2 + 1;
        const int C = g.C[P_COL], Gs = g.G[P_COL];
        // (a) the level's own force: same-level kernels on its own fields,
        // Case-2 phase kernels on every finer level's sub-grids
        const int in0 = (int)g.colins.size();
        {
            const SpecEntry* k1 = nullptr;
            TD_TRY(plan_spectra(P, G.M, 1, 1, &k1));
            for (int f = 0; f < 3; ++f)
                g.colins.push_back({ptr(own_in[t] + f * H * G.ny), k1->ptr, G.ny, 0, f, 4 | fam, G.ny, 0});
            // the phase inputs follow, band-limited ones (few enough rows
            // for the band transforms) last
            std::vector<ColIn> wide, band;
            const int band_rows = col_band_rows(G.M, (int)es);
            for (int s = t + 1; s < L; ++s) {
                const LevelG& S = P->lv[s];
                const int m = ipow(r, s - t), nr = ph_nr[s][t];
                const SpecEntry* k2 = nullptr;
                TD_TRY(plan_spectra(P, G.M, 2, m, &k2));
                const size_t per_phase = 6 * H * G.M;
                // the mirror images of one stored phase (adjacent in
                // phase_order) are listed field by field: consecutive inputs,
                // which run side by side in a workgroup's slots or one round
                // apart, then read the same stored kernel columns
                std::vector<ColIn> grp;  // field-0 inputs of one stored phase
                auto flush = [&]() {
                    for (int f = 0; f < 3; ++f)
                        for (ColIn I : grp) {
                            I.in += (int64_t)f * H * nr * es;
                            I.f = f;
                            (I.rows <= band_rows ? band : wide).push_back(I);
                        }
                    grp.clear();
                };
                for (const auto& ph : phase_order(m)) {
                    const int kx = ph.first, ky = ph.second;
                    const int lr_lo = ceil_div(S.oy - ky, m) - G.oy;
                    const int lr_hi = floor_div(S.oy + S.ny - 1 - ky, m) - G.oy;
                    if (lr_hi < lr_lo) continue;
                    const int phase = ky * m + kx;
                    int flip = 0;
                    const void* kern = phase_kernels(k2, m, kx, ky, per_phase * es, &flip);
                    if (!grp.empty() && grp.back().kern != kern) flush();
                    grp.push_back({ptr(ph_in[s][t] + (size_t)phase * 3 * H * nr), kern, nr, lr_lo, 0,
                                   flip | fam, lr_hi - lr_lo + 1, 0});
                }
                flush();
            }
            g.colins.insert(g.colins.end(), wide.begin(), wide.end());
            g.colins.insert(g.colins.end(), band.begin(), band.end());
            const int out0 = (int)g.colouts.size();
            for (int comp = 0; comp < 2; ++comp)
                g.colouts.push_back({ptr(own_out[t] + comp * H * G.ny), nullptr, G.ny, 0, comp, 0});
            const int nin = (int)g.colins.size() - in0;
            for (int kx0 = 0; kx0 < (int)H; kx0 += C)
                g.col.push_back({0, kx0, std::min(C, (int)H - kx0), in0, nin, out0, 2, (int)band.size()});
        }
        // (b) Case-3 phases of this (coarser) level onto every finer target:
        // the level's three own planes (the first inputs above) are
        // transformed again by every job, so a job takes the outputs of all
        // finer targets in a row (up to 256 of them: about the length of
        // the longest own-force job)
        const int c3_out0 = (int)g.colouts.size();
        for (int s = t + 1; s < L; ++s) {
            const LevelG& T = P->lv[s];
            const int m = ipow(r, s - t), ld = c3_ld[t][s];
            const SpecEntry* k3 = nullptr;
            TD_TRY(plan_spectra(P, G.M, 3, m, &k3));
            const size_t per_phase = 6 * H * G.M;
            // mirror images of one stored phase component by component, as
            // the Case-2 inputs above
            std::vector<ColOut> grp;  // component-0 outputs of one stored phase
            auto flush = [&]() {
                for (int comp = 0; comp < 2; ++comp)
                    for (ColOut O : grp) {
                        O.out += (int64_t)comp * H * ld * es;
                        O.comp = comp;
                        g.colouts.push_back(O);
                    }
                grp.clear();
            };
            for (const auto& ph : phase_order(m)) {
                const int kx = ph.first, ky = ph.second;
                const int phase = ky * m + kx;
                int flip = 0;
                const void* kern = phase_kernels(k3, m, kx, ky, per_phase * es, &flip);
                if (!grp.empty() && grp.back().kern != kern) flush();
                grp.push_back({ptr(c3_out[t][s] + (size_t)phase * 2 * H * ld), kern, ld,
                               floor_div(T.oy, m) - G.oy, 0, flip | fam});
            }
            flush();
        }
        const int nout = (int)g.colouts.size() - c3_out0;
        const int chunk = std::max(16 * Gs, 256);
        for (int kx0 = 0; kx0 < (int)H; kx0 += C)
            for (int o0 = 0; o0 < nout; o0 += chunk)
                g.col.push_back({1, kx0, std::min(C, (int)H - kx0), in0, 3, c3_out0 + o0,
                                 std::min(chunk, nout - o0), 0});
    }
    // ---- XCD affinity of the column pass.  Workgroups are dispatched to
    // the eight XCDs round-robin, each with its own L2; every job of one
    // spectral column reads the same stored kernel columns (same lattice,
    // same spectra).  Placing the jobs of column group kx0 / C at list
    // positions congruent to it mod 8 keeps each column's kernel reads in
    // one L2, and each residue's jobs run longest first.
    for (auto& g : P->groups) {
        constexpr int NX = 8;
        std::vector<ColJob> bucket[NX];
        const int C = g.C[P_COL];  // columns per job: kx0 is a multiple of C
        for (const ColJob& j : g.col) bucket[(j.kx0 / C) % NX].push_back(j);
        auto cost = [](const ColJob& j) { return j.kind == 0 ? j.nin : 3 + j.nout; };
        for (auto& b : bucket)
            std::stable_sort(b.begin(), b.end(), [&](const ColJob& a, const ColJob& c) { return cost(a) > cost(c); });
        size_t pos[NX] = {};
        std::vector<ColJob> order;
        order.reserve(g.col.size());
        while (order.size() < g.col.size()) {
            const int x = (int)(order.size() % NX);
            int take = x;
            if (pos[take] == bucket[take].size()) {  // residue exhausted: the fullest other
                take = 0;
                for (int k = 1; k < NX; ++k)
                    if (bucket[k].size() - pos[k] > bucket[take].size() - pos[take]) take = k;
            }
            order.push_back(bucket[take][pos[take]++]);
        }
        g.col.swap(order);
    }
    // ---- pass 4: row inverse, grouped by lattice length
    for (int t = 0; t < L; ++t) {
        const LevelG& T = P->lv[t];
        // contributions: own lattice first, then every coarser source
        struct Ctb { int M; RowInvContrib c; };
        std::vector<Ctb> all;
        {
            RowInvContrib c;
            memset(&c, 0, sizeof(c));
            c.base = ptr(own_out[t]);
            c.phase_stride = 0;
            c.comp_stride = (int64_t)(T.M / 2 + 1) * T.ny;
            c.m = 1;
            c.mshift = 0;
            c.ld = T.ny;
            c.lr_first = 0;
            c.ox_s = T.ox;
            c.oy_s = T.oy;
            all.push_back({T.M, c});
        }
        for (int s = 0; s < t; ++s) {
            const LevelG& S = P->lv[s];
            const int m = ipow(r, t - s), ld = c3_ld[s][t];
            RowInvContrib c;
            memset(&c, 0, sizeof(c));
            c.base = ptr(c3_out[s][t]);
            c.phase_stride = (int64_t)2 * (S.M / 2 + 1) * ld;
            c.comp_stride = (int64_t)(S.M / 2 + 1) * ld;
            c.m = m;
            c.mshift = (m & (m - 1)) ? -1 : ilog2(m);  // -1: not a power of two
            c.ld = ld;
            c.lr_first = floor_div(T.oy, m) - S.oy;
            c.ox_s = S.ox;
            c.oy_s = S.oy;
            all.push_back({S.M, c});
        }
        std::vector<int> Ms;
        for (auto& a : all)
            if (std::find(Ms.begin(), Ms.end(), a.M) == Ms.end()) Ms.push_back(a.M);
        for (size_t gi = 0; gi < Ms.size(); ++gi) {
            const int M = Ms[gi];
            Group& g = group_for(P->groups, M);
            const int c0 = (int)g.contribs.size();
            for (auto& a : all)
                if (a.M == M) g.contribs.push_back(a.c);
            const int nc = (int)g.contribs.size() - c0;
            const int C = g.C[P_ROWINV];
            const int acc = (gi == 0) ? 0 : 1;  // Ms[0] is the own lattice's M
            // at most 2M target columns per job: 16 outputs per thread
            const int xchunk = std::min(T.nx, 2 * M);
            for (int y0 = 0; y0 < T.ny; y0 += C)
            for (int x0 = 0; x0 < T.nx; x0 += xchunk) {
                RowInvJob j;
                memset(&j, 0, sizeof(j));
                j.lvl = t;
                j.nx_t = T.nx;
                j.ny_t = T.ny;
                j.ox_t = T.ox;
                j.oy_t = T.oy;
                j.y0 = y0;
                j.ny = std::min(C, T.ny - y0);
                j.c0 = c0;
                j.nc = nc;
                j.accumulate = acc;
                j.x0 = x0;
                j.nx = std::min(xchunk, T.nx - x0);
                g.rinv[acc].push_back(j);
            }
        }
    }
    for (auto& g : P->groups)
        for (int a = 0; a < 2; ++a) {
            const int per = g.G[P_ROWINV] * (g.M / 8);
            for (auto& j : g.rinv[a]) g.nq[a] = std::max(g.nq[a], (j.nx + per - 1) / per);
        }
    // ---- XCD placement of the row inverse.  Workgroups are dispatched to
    // the eight XCDs round-robin (list position p runs on XCD p mod 8, up to
    // a rotation that is the same for the whole list), each with its own L2.
    // A job reads, per frequency, a few consecutive stored rows of each
    // contribution plane; one cache line holds the rows of 16 m target rows
    // (f32; 8 m in f64) for a coarser source at ratio m.  Each level's jobs
    // are cut into eight contiguous runs of target rows, one per XCD, so a
    // line is fetched by one or two XCDs rather than by all eight, and every
    // XCD gets the same share of every level's work.
    // Within each XCD the levels run longest first (a finer level's rows
    // take more rounds: one item per x-phase of every coarser source), so
    // the short rows of the coarse levels fill the tail.
    for (auto& g : P->groups)
        for (int a = 0; a < 2; ++a) {
            std::vector<RowInvJob>& jobs = g.rinv[a];
            auto items = [&](const RowInvJob& j) {
                int n = 0;
                for (int k = 0; k < j.nc; ++k) n += g.contribs[j.c0 + k].m;
                return n;
            };
            std::vector<std::pair<size_t, size_t>> runs;  // one level's jobs
            for (size_t i = 0; i < jobs.size();) {
                size_t e = i;
                while (e < jobs.size() && jobs[e].lvl == jobs[i].lvl) ++e;
                runs.push_back({i, e});
                i = e;
            }
            std::stable_sort(runs.begin(), runs.end(), [&](const auto& x, const auto& y) {
                return items(jobs[x.first]) > items(jobs[y.first]);
            });
            std::vector<std::vector<RowInvJob>> bins(8);
            for (const auto& run : runs) {
                const size_t n = run.second - run.first;
                for (size_t k = 0; k < n; ++k) bins[k * 8 / n].push_back(jobs[run.first + k]);
            }
            std::vector<RowInvJob> order;
            order.reserve(jobs.size());
            for (size_t r = 0; order.size() < jobs.size(); ++r)
                for (auto& b : bins)
                    if (r < b.size()) order.push_back(b[r]);
            jobs.swap(order);
        }
    return TD_OK;
}

// Host-side bounds proof of every job against the workspace, the kernel
// spectra, the fields and the launch shape, and of the data flow: every
// workspace row a pass reads was written by the pass before.
td_status validate_jobs(td_plan* P)
{
    const size_t es = elem_size(P->dt);
    const int64_t ws = (int64_t)P->ws_bytes;
    auto in_ws = [&](int64_t off, int64_t elems) { return off >= 0 && off + elems * (int64_t)es <= ws; };
    auto bad = [&](const char* what) { return fail(TD_EINVAL, std::string("plan validation: ") + what); };
    // patch tables: patches inside their level's window, covered squares
    // inside the window, pointer slots within the request's table
    if ((int)P->lp.size() != P->nlevels) return bad("level tables");
    for (int l = 0; l < P->nlevels; ++l) {
        const LevelPatches& lp = P->lp[l];
        const LevelG& G = P->lv[l];
        if (lp.np < 1 || lp.np > TD_PATCHES_PER_LEVEL || lp.nc < 0 || lp.nc > TD_PATCHES_PER_LEVEL)
            return bad("level patch counts");
        for (int k = 0; k < lp.np; ++k)
            if (lp.pi0[k] < 0 || lp.pj0[k] < 0 || lp.pn[k] < 1 || lp.pi0[k] + lp.pn[k] > G.nx ||
                lp.pj0[k] + lp.pn[k] > G.ny || lp.pslot[k] < 0 || lp.pslot[k] + 4 >= 5 * P->npatches ||
                lp.pslot[k] % 5 || P->patch_n[lp.pslot[k] / 5] != lp.pn[k])
                return bad("level patch");
        for (int k = 0; k < lp.nc; ++k)
            if (lp.ci0[k] < 0 || lp.cj0[k] < 0 || lp.ci0[k] + lp.cn[k] > G.nx || lp.cj0[k] + lp.cn[k] > G.ny)
                return bad("covered square");
    }
    for (auto& g : P->groups) {
        const int M = g.M, H = M / 2 + 1;
        for (int pass = 0; pass < NSHAPE; ++pass) {
            const int C = g.C[pass], Gs = g.G[pass];
            const size_t lds = pass == P_COL ? col_lds_bytes(M, C, es, Gs) : lds_bytes(M, C, es, Gs);
            if (C < 1 || Gs < 1 || Gs > 16 || C * Gs * (M / 8) > TD_MAX_THREADS ||
                (C & (C - 1)) || (Gs & (Gs - 1)) || lds > TD_MAX_DYN_LDS)
                return bad("launch shape");
        }
        // pass 1: rows written per row-pass plane, and the lattice row of
        // each plane's stored row 0
        std::map<int64_t, std::vector<char>> rows_written;
        std::map<int64_t, int> plane_lr;
        std::map<int64_t, std::array<int, 3>> plane_src;  // level, m, row_off
        for (auto& j : g.rowfwd) {
            if (j.lvl < 0 || j.lvl >= P->nlevels || j.f < 0 || j.f > 2) return bad("row source");
            // lattice columns and rows >= M/2 map past the source level's
            // window (so hold zeros): the row transforms gather only columns
            // < M/2 and the column transforms read only rows < M/2
            if ((int64_t)j.m * (M / 2) + j.col_off < P->lv[j.lvl].nx ||
                (int64_t)j.m * (M / 2) + j.row_off < P->lv[j.lvl].ny)
                return bad("row source reaches the upper half of the lattice");
            if (plane_lr.emplace(j.out, j.lr_first).first->second != j.lr_first)
                return bad("row plane origin");
            {
                const std::array<int, 3> src = {j.lvl, j.m, j.row_off};
                if (plane_src.emplace(j.out, src).first->second != src) return bad("row plane source");
            }
            // slope fields are scaled by their level's cell side, which the
            // row kernel's in-place slope estimate (per-cell differences)
            // takes for granted
            {
                RowFwdJob w;
                row_scales(P, P->lv[j.lvl].h, j.f, &w);
                if (j.scale != w.scale || j.est_scale != w.est_scale) return bad("row scale");
            }
            if (j.row0 < 0 || j.nrow < 1 || j.nrow > 2 * g.C[P_ROWFWD] || j.row0 + j.nrow > j.ld)
                return bad("row range");
            // the columns the gather skips map outside the source window
            if (j.lc_lo < 0 || j.lc_hi < j.lc_lo || j.lc_hi > M / 2 ||
                (j.lc_lo > 0 && (int64_t)j.m * (j.lc_lo - 1) + j.col_off >= 0) ||
                (j.lc_hi < M / 2 && (int64_t)j.m * j.lc_hi + j.col_off < P->lv[j.lvl].nx))
                return bad("row column range");
            if (!in_ws(j.out, (int64_t)H * j.ld)) return bad("row output");
            auto& w = rows_written[j.out];
            if ((int)w.size() < j.ld) w.resize(j.ld, 0);
            for (int r = j.row0; r < j.row0 + j.nrow; ++r) w[r] = 1;
        }
        // pass 2: inputs fully written by pass 1, outputs in range;
        // columns written per output plane
        std::vector<char> in_ok(g.colins.size(), 0);
        for (size_t i = 0; i < g.colins.size(); ++i) {
            const ColIn& I = g.colins[i];
            if (I.ld < 1 || I.lr_first < 0 || I.lr_first + I.ld > M) return bad("col input rows");
            {
                auto pl = plane_lr.find(I.in);
                if (pl == plane_lr.end() || pl->second != I.lr_first) return bad("col input origin");
            }
            // stored rows >= rows map past the source level's window (zeros)
            {
                const auto& src = plane_src.at(I.in);
                if (I.rows < 1 || I.rows > I.ld ||
                    (int64_t)src[1] * (I.lr_first + I.rows) + src[2] < P->lv[src[0]].ny)
                    return bad("col input source rows");
            }
            if (I.f < 0 || I.f > 2 || (I.flip & ~8) < 0 || (I.flip & ~8) > 4 ||
                ((I.flip >> 3) & 1) != (P->quantity == TD_POTENTIAL ? 1 : 0))
                return bad("col input kernel");
            if (!in_ws(I.in, (int64_t)H * I.ld)) return bad("col input plane");
            auto it = rows_written.find(I.in);
            if (it == rows_written.end() || (int)it->second.size() < I.ld) return bad("col reads unwritten rows");
            for (int rr = 0; rr < I.ld; ++rr)
                if (!it->second[rr]) return bad("col reads unwritten rows");
            in_ok[i] = 1;
        }
        for (auto& O : g.colouts) {
            if (O.out_ld < 1 || O.out_lr_first < 0 || O.out_lr_first + O.out_ld > M / 2)
                return bad("col output rows");
            if (!in_ws(O.out, (int64_t)H * O.out_ld)) return bad("col output plane");
            if (O.comp < 0 || O.comp > 1 || (O.flip & ~8) < 0 || (O.flip & ~8) > 3 ||
                (O.kern && ((O.flip >> 3) & 1) != (P->quantity == TD_POTENTIAL ? 1 : 0)))
                return bad("col output kernel");
        }
        std::map<int64_t, std::pair<int, std::vector<char>>> out_written;  // ld, columns
        for (auto& j : g.col) {
            if (j.kx0 < 0 || j.ncol < 1 || j.ncol > g.C[P_COL] || j.kx0 + j.ncol > H) return bad("col columns");
            if (j.in0 < 0 || j.nin < 1 || j.in0 + j.nin > (int)g.colins.size()) return bad("col inputs");
            if (j.out0 < 0 || j.nout < 1 || j.out0 + j.nout > (int)g.colouts.size()) return bad("col outputs");
            if (j.kind == 0) {
                if (j.nout != 2) return bad("col own outputs");
                for (int i = j.in0; i < j.in0 + j.nin; ++i)
                    if (!g.colins[i].kern) return bad("col input kernel");
                // band-limited inputs: a band path for M, and few enough rows
                if (j.nband < 0 || j.nband > j.nin || (j.nband > 0 && col_band_rows(M, (int)es) == 0))
                    return bad("col band inputs");
                for (int i = j.in0 + j.nin - j.nband; i < j.in0 + j.nin; ++i)
                    if (g.colins[i].rows > col_band_rows(M, (int)es)) return bad("col band input rows");
            } else if (j.kind == 1) {
                if (j.nin != 3 || j.nband != 0) return bad("col Case-3 inputs");
                for (int o = j.out0; o < j.out0 + j.nout; ++o)
                    if (!g.colouts[o].kern) return bad("col output kernel");
            } else {
                return bad("col job kind");
            }
            for (int k = j.out0; k < j.out0 + j.nout; ++k) {
                auto& w = out_written[g.colouts[k].out];
                w.first = g.colouts[k].out_ld;
                if ((int)w.second.size() < H) w.second.resize(H, 0);
                for (int cc = j.kx0; cc < j.kx0 + j.ncol; ++cc) w.second[cc] = 1;
            }
        }
        // pass 3 (each contribution's input planes are proven once)
        std::vector<char> contrib_ok(g.contribs.size(), 0);
        for (int a = 0; a < 2; ++a)
            for (auto& j : g.rinv[a]) {
                if (j.lvl < 0 || j.lvl >= P->nlevels || j.nx_t != P->lv[j.lvl].nx ||
                    j.ny_t != P->lv[j.lvl].ny || j.ox_t != P->lv[j.lvl].ox || j.oy_t != P->lv[j.lvl].oy)
                    return bad("rinv level");
                if (j.y0 < 0 || j.ny < 1 || j.ny > g.C[P_ROWINV] || j.y0 + j.ny > j.ny_t) return bad("rinv rows");
                if (j.x0 < 0 || j.nx < 1 || j.x0 + j.nx > j.nx_t || (long)j.nx > 2L * M ||
                    j.nx > (long)g.nq[a] * g.G[P_ROWINV] * (M / 8))
                    return bad("rinv columns");
                if (j.c0 < 0 || j.c0 + j.nc > (int)g.contribs.size()) return bad("rinv contribs");
                if (j.oy_t < 0 || j.ox_t < 0) return bad("rinv offsets");
                for (int k = 0; k < j.nc; ++k) {
                    const RowInvContrib& c = g.contribs[j.c0 + k];
                    if (c.m < 1 || c.m > 16 || (c.mshift >= 0 ? (1 << c.mshift) != c.m : !(c.m & (c.m - 1))))
                        return bad("rinv ratio");
                    // rows and columns reached by this job's targets
                    for (int rr : {j.y0, j.y0 + j.ny - 1}) {
                        const int gg = j.oy_t + rr, Jc = floor_div(gg, c.m);
                        const int sr = Jc - c.oy_s - c.lr_first;
                        if (sr < 0 || sr >= c.ld) return bad("rinv source row");
                    }
                    for (int ii : {j.x0, j.x0 + j.nx - 1}) {
                        const int lc = floor_div(j.ox_t + ii, c.m) - c.ox_s;
                        if (lc < 0 || lc >= M / 2) return bad("rinv source col");
                    }
                    const int64_t last = c.base + ((int64_t)(c.m * c.m - 1) * c.phase_stride +
                                                   c.comp_stride + (int64_t)H * c.ld) * (int64_t)es;
                    if (c.base < 0 || last > ws) return bad("rinv contribution");
                    if (contrib_ok[j.c0 + k]) continue;
                    contrib_ok[j.c0 + k] = 1;
                    // every phase / component plane it reads was written in full
                    for (int p = 0; p < c.m * c.m; ++p)
                        for (int comp = 0; comp < 2; ++comp) {
                            const int64_t plane = c.base + ((int64_t)p * c.phase_stride + comp * c.comp_stride) * (int64_t)es;
                            auto it = out_written.find(plane);
                            if (it == out_written.end() || it->second.first != c.ld) return bad("rinv reads unwritten outputs");
                            for (int cc = 0; cc < H; ++cc)
                                if (!it->second.second[cc]) return bad("rinv reads unwritten outputs");
                        }
                }
            }
    }
    return TD_OK;
}

// Level geometry (sizes, offsets, FFT lengths, covered rectangles).
td_status plan_geometry(td_plan* P, const td_hierarchy* h, td_dtype dt)
{
    int L = 0;
    TD_TRY(patch_levels(h, &L));
    P->dt = dt;
    P->ratio = h->ratio;
    P->nlevels = L;
    P->npatches = h->npatches;
    P->x0 = h->x0;
    P->y0 = h->y0;
    P->h0 = h->h0;
    P->aspect = h->aspect > 0 ? h->aspect : 1.0;
    P->id = g_plan_ids++;
    double hh = h->h0;
    for (int l = 0; l < L; ++l) {
        LevelG g;
        level_window(h, l, &g.ox, &g.oy, &g.nx, &g.ny);
        g.M = fft_len(std::max(g.nx, g.ny));
        g.h = hh;
        LevelPatches lp;
        memset(&lp, 0, sizeof(lp));
        for (int k = 0; k < h->npatches; ++k) {
            const td_patch& q = h->patches[k];
            if (q.level == l) {
                lp.pi0[lp.np] = q.ox - g.ox;
                lp.pj0[lp.np] = q.oy - g.oy;
                lp.pn[lp.np] = q.n;
                lp.pslot[lp.np] = 5 * k;
                lp.np += 1;
            } else if (q.level == l + 1) {
                lp.ci0[lp.nc] = q.ox / h->ratio - g.ox;
                lp.cj0[lp.nc] = q.oy / h->ratio - g.oy;
                lp.cn[lp.nc] = q.n / h->ratio;
                lp.nc += 1;
            }
        }
        P->lv.push_back(g);
        P->lp.push_back(lp);
        hh /= h->ratio;
    }
    for (int k = 0; k < h->npatches; ++k) P->patch_n.push_back(h->patches[k].n);
    return TD_OK;
}

td_status plan_upload(td_plan* P)
{
    td_context* ctx = P->ctx;
    TD_TRY(upload(ctx, P, P->lp, &P->d_lp));
    for (auto& g : P->groups) {
        TD_TRY(upload(ctx, P, g.rowfwd, &g.d_rowfwd));
        TD_TRY(upload(ctx, P, g.col, &g.d_col));
        TD_TRY(upload(ctx, P, g.colins, &g.d_colins));
        TD_TRY(upload(ctx, P, g.colouts, &g.d_colouts));
        {
            const std::vector<const void*> tabs{g.d_colins, g.d_colouts};
            const void** d = nullptr;
            TD_TRY(upload(ctx, P, tabs, &d));
            g.d_coltabs = (void*)d;
        }
        TD_TRY(upload(ctx, P, g.rinv[0], &g.d_rinv[0]));
        TD_TRY(upload(ctx, P, g.rinv[1], &g.d_rinv[1]));
        TD_TRY(upload(ctx, P, g.contribs, &g.d_contribs));
        {
            const std::vector<RowInvTables> tabs{{g.d_contribs, P->d_lp}};
            TD_TRY(upload(ctx, P, tabs, &g.d_rinv_tabs));
        }
    }
    return TD_OK;
}

void plan_free(td_plan* P)
{
    if (!P) return;
    td_context* ctx = P->ctx;
    for (auto& a : P->dev_allocs) ctx->release(a.first, a.second);
    P->dev_allocs.clear();
    if (P->ws) ctx->release(P->ws, P->ws_bytes);
    P->ws = nullptr;
}

// Copy a pointer table to the device through a ring of pinned staging
// buffers; a slot is reused only after its previous copy has completed.
struct Stager {
    static const int RING = 8;
    void** host[RING] = {};
    hipEvent_t ev[RING] = {};
    bool used[RING] = {};
    int next = 0;
    size_t cap = 0;
    td_status init(size_t nptr)
    {
        cap = nptr;
        for (int k = 0; k < RING; ++k) {
            TD_HIP(hipHostMalloc((void**)&host[k], sizeof(void*) * std::max<size_t>(nptr, 1)));
            TD_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
        }
        return TD_OK;
    }
    void destroy()
    {
        for (int k = 0; k < RING; ++k) {
            if (ev[k]) (void)hipEventDestroy(ev[k]);
            if (host[k]) (void)hipHostFree(host[k]);
            ev[k] = nullptr;
            host[k] = nullptr;
        }
    }
    td_status push(void** dev, const std::vector<void*>& v, hipStream_t st)
    {
        const int k = next;
        next = (next + 1) % RING;
        if (used[k]) TD_HIP(hipEventSynchronize(ev[k]));
        memcpy(host[k], v.data(), sizeof(void*) * v.size());
        TD_HIP(hipMemcpyAsync(dev, host[k], sizeof(void*) * v.size(), hipMemcpyHostToDevice, st));
        TD_HIP(hipEventRecord(ev[k], st));
        used[k] = true;
        return TD_OK;
    }
};

}  // namespace

// ===========================================================================
// launching the four passes for a list of (plan, slot base) members
// ===========================================================================

namespace {

struct Member {
    td_plan* plan;
    int slot_base;
    char* ws;
};

template <typename Job>
void push_seg(std::vector<SegTable<Job>>& tabs, std::vector<int>& totals, const Job* jobs, int n,
              int slot_base, const void* aux, char* ws)
{
    if (n <= 0) return;
    if (tabs.empty() || tabs.back().nseg == TD_MAX_SEGS) {
        SegTable<Job> s;
        memset(&s, 0, sizeof(s));
        tabs.push_back(s);
        totals.push_back(0);
    }
    SegTable<Job>& s = tabs.back();
    s.start[s.nseg] = totals.back();
    s.slot_base[s.nseg] = slot_base;
    s.jobs[s.nseg] = jobs;
    s.aux[s.nseg] = aux;
    s.ws[s.nseg] = ws;
    s.nseg += 1;
    totals.back() += n;
    s.start[s.nseg] = totals.back();
}

// The persistent column launches of a fixed member set (a batch): one work
// queue per column launch, in launch order, recorded once by running
// launch_members with `building` set (which launches nothing).
struct QueueRec {
    JobQueue q;
    int grid;
};
struct Queues {
    bool building = false;
    std::vector<QueueRec> recs;
    // while recording: each launch's job order and list starts
    std::vector<std::vector<int32_t>> order, start;
    void* dev = nullptr;  // counters of every launch, then starts and orders
    size_t dev_bytes = 0;
};

// Record one persistent column launch over the jobs of `segs` (in launch
// order).  A job goes to the list of its column group kx0 / C mod TD_NXCD (the
// jobs of one column read the same kernel columns: one L2), unless that
// list already holds its share of the launch's work; then to the least
// loaded list.  Jobs are placed and listed longest first, so that the
// short ones fill the tail.  The grid holds as many workgroups as the
// device runs at once, at most one per job.
void record_col_launch(const td_context* ctx, const std::vector<std::pair<const ColJob*, int>>& segs,
                       bool f64, int M, int C, int G, Queues* qs)
{
    struct Item { int cost, col, idx; };
    std::vector<Item> items;
    int base = 0;
    long long total = 0;
    for (auto& sg : segs) {
        for (int k = 0; k < sg.second; ++k) {
            const ColJob& j = sg.first[k];
            const int cost = j.kind == 0 ? std::max(1, j.nin) : 3 + j.nout;
            items.push_back({cost, (j.kx0 / C) % TD_NXCD, base + k});
            total += cost;
        }
        base += sg.second;
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    const long long share = (total + TD_NXCD - 1) / TD_NXCD;
    std::vector<std::vector<int32_t>> lists(TD_NXCD);
    long long load[TD_NXCD] = {0};
    for (const Item& it : items) {
        int l = it.col;
        if (load[l] + it.cost > share) l = int(std::min_element(load, load + TD_NXCD) - load);
        lists[l].push_back(it.idx);
        load[l] += it.cost;
    }
    std::vector<int32_t> order, start(1, 0);
    for (auto& l : lists) {
        order.insert(order.end(), l.begin(), l.end());
        start.push_back((int32_t)order.size());
    }
    const int per_xcd = std::max(1, ctx->cus / TD_NXCD) * col_resident_blocks(f64, M, C, G);
    const int grid = TD_NXCD * std::max(1, std::min(per_xcd, (base + TD_NXCD - 1) / TD_NXCD));
    qs->order.push_back(std::move(order));
    qs->start.push_back(std::move(start));
    qs->recs.push_back({JobQueue{}, grid});
}

// One launch per (pass, M, <= TD_MAX_SEGS members), in pass order.  With
// `qs`: persistent launches on the batch's recorded queues (or, while
// qs->building, record them and launch nothing).
td_status launch_members(td_context* ctx, td_dtype dt, const std::vector<Member>& mem,
                         void* const* d_ptrs, const FieldPtrs& fp, hipStream_t st,
                         Queues* qs = nullptr)
{
    size_t launch_index = 0;
    std::vector<int> Ms;
    for (auto& m : mem)
        for (auto& g : m.plan->groups)
            if (std::find(Ms.begin(), Ms.end(), g.M) == Ms.end()) Ms.push_back(g.M);
    std::sort(Ms.begin(), Ms.end());
    auto find_group = [](td_plan* p, int M) -> Group* {
        for (auto& g : p->groups)
            if (g.M == M) return &g;
        return nullptr;
    };
    const bool f64 = dt == TD_F64;
    bool timed = false;
    if (ctx->timing && !(qs && qs->building)) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        timed = hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
    }
    // C per (pass, M) must agree across members; members built with other
    // tunings are launched in separate groups.
    for (int pass = 0; pass < NTIMED; ++pass) {
        hipEvent_t ev_a = nullptr, ev_b = nullptr;
        bool any = false;
        for (auto& m : mem)
            for (auto& g : m.plan->groups) {
                const size_t nj = pass == P_ROWFWD ? g.rowfwd.size() : pass == P_COL ? g.col.size()
                                : g.rinv[pass == P_ROWINV ? 0 : 1].size();
                any |= nj > 0;
            }
        if (timed && any && (ctx->timing_mask >> pass) & 1) {
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            ev_a = ctx->get_event();
            ev_b = ctx->get_event();
            if (ev_a) (void)hipEventRecord(ev_a, st);
        }
        for (int M : Ms) {
            const void* tw = nullptr;
            // partition members by C of this pass
            std::map<int, std::vector<std::pair<Group*, const Member*>>> byC;
            for (auto& m : mem) {
                Group* g = find_group(m.plan, M);
                if (!g) continue;
                if (!tw) tw = g->tw;
                const int pi = pass == NSHAPE ? P_ROWINV : pass;
                byC[pack_shape(g->C[pi], g->G[pi])].push_back({g, &m});
            }
            for (auto& kv : byC) {
                const int C = shape_C(kv.first), Gs = shape_G(kv.first);
                hipError_t e = hipSuccess;
                if (pass == P_ROWFWD) {
                    std::vector<SegTable<RowFwdJob>> t;
                    std::vector<int> n;
                    for (auto& gs : kv.second)
                        push_seg(t, n, gs.first->d_rowfwd, (int)gs.first->rowfwd.size(), gs.second->slot_base,
                                 (const void*)gs.second->plan->d_lp, gs.second->ws);
                    if (qs && qs->building) continue;
                    for (size_t i = 0; i < t.size() && e == hipSuccess; ++i)
                        e = f64 ? launch_row_fwd<double>(M, C, n[i], t[i], (const void* const*)d_ptrs, fp, tw, true, st)
                                : launch_row_fwd<float>(M, C, n[i], t[i], (const void* const*)d_ptrs, fp, tw, true, st);
                } else if (pass == P_COL) {
                    std::vector<SegTable<ColJob>> t;
                    std::vector<int> n;
                    // the host job lists of each launch's segments
                    std::vector<std::vector<std::pair<const ColJob*, int>>> host;
                    for (auto& gs : kv.second) {
                        const size_t before = t.size();
                        push_seg(t, n, gs.first->d_col, (int)gs.first->col.size(), gs.second->slot_base,
                                 (const void*)gs.first->d_coltabs, gs.second->ws);
                        if (gs.first->col.empty()) continue;
                        if (t.size() > before) host.emplace_back();
                        host.back().push_back({gs.first->col.data(), (int)gs.first->col.size()});
                    }
                    for (size_t i = 0; i < t.size() && e == hipSuccess; ++i, ++launch_index) {
                        JobQueue q{};
                        int blocks = n[i];
                        if (qs && qs->building) {
                            record_col_launch(ctx, host[i], f64, M, C, Gs, qs);
                            continue;
                        }
                        if (qs) {
                            if (launch_index >= qs->recs.size()) {
                                e = hipErrorInvalidValue;
                                break;
                            }
                            q = qs->recs[launch_index].q;
                            blocks = qs->recs[launch_index].grid;
                        }
                        e = f64 ? launch_col<double>(M, C, Gs, blocks, t[i], tw, st, q)
                                : launch_col<float>(M, C, Gs, blocks, t[i], tw, st, q);
                    }
                } else {
                    const int a = pass == P_ROWINV ? 0 : 1;
                    std::vector<SegTable<RowInvJob>> t;
                    std::vector<int> n;
                    for (auto& gs : kv.second)
                        push_seg(t, n, gs.first->d_rinv[a], (int)gs.first->rinv[a].size(),
                                 gs.second->slot_base, (const void*)gs.first->d_rinv_tabs,
                                 gs.second->ws);
                    if (qs && qs->building) continue;
                    int nq = 1;
                    for (auto& gs : kv.second) nq = std::max(nq, gs.first->nq[a]);
                    for (size_t i = 0; i < t.size() && e == hipSuccess; ++i)
                        e = f64 ? launch_row_inv<double>(M, C, Gs, n[i], t[i], d_ptrs, fp, tw, st, nq)
                                : launch_row_inv<float>(M, C, Gs, n[i], t[i], d_ptrs, fp, tw, st, nq);
                }
                if (e != hipSuccess)
                    return fail(TD_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
            }
        }
        if (ev_a && ev_b) {
            (void)hipEventRecord(ev_b, st);
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            ctx->timed.push_back({pass, ev_a, ev_b});
        }
    }
    return TD_OK;
}

// The 5 field pointers of every patch of a request (sigma, dsdx, dsdy, fx,
// fy) into v[base ...], checked against the patch count, element size and
// quantity of the plan that will run it.
td_status fill_ptrs_for(const td_request& q, int npatches, td_dtype dt, int quantity,
                        void** v, size_t base)
{
    const bool pot = quantity == TD_POTENTIAL;  // fx receives Phi; fy optional
    if (!q.sigma || !q.fx || (!q.fy && !pot))
        return fail(TD_EINVAL, pot ? "sigma and fx are required" : "sigma, fx and fy are required");
    if (q.slopes != TD_SLOPES_GIVEN && q.slopes != TD_SLOPES_ESTIMATE)
        return fail(TD_EINVAL, "slopes must be TD_SLOPES_GIVEN or TD_SLOPES_ESTIMATE");
    if (q.slopes == TD_SLOPES_ESTIMATE && (q.dsdx || q.dsdy))
        return fail(TD_EINVAL, "dsdx and dsdy must be NULL with TD_SLOPES_ESTIMATE");
    const uintptr_t align = dt == TD_F64 ? 8 : 4;
    for (int l = 0; l < npatches; ++l) {
        void* fyl = q.fy ? q.fy[l] : nullptr;
        if (!q.sigma[l] || !q.fx[l] || (!fyl && !pot))
            return fail(TD_EINVAL, "NULL sigma/fx/fy pointer of patch " + std::to_string(l));
        void* f[5] = {(void*)q.sigma[l], q.dsdx ? (void*)q.dsdx[l] : nullptr,
                      q.dsdy ? (void*)q.dsdy[l] : nullptr, q.fx[l], fyl};
        for (int i = 0; i < 5; ++i) {
            if ((uintptr_t)f[i] % align)
                return fail(TD_EINVAL, "field pointer of patch " + std::to_string(l) +
                                           " is not aligned to its element size");
            v[base + 5 * l + i] = f[i];
        }
        // estimated slopes: the slope slots carry the sigma pointer, tagged
        // in bit 0 (clear in every element-aligned pointer)
        if (q.slopes == TD_SLOPES_ESTIMATE)
            v[base + 5 * l + 1] = v[base + 5 * l + 2] = (void*)((uintptr_t)f[0] | 1u);
    }
    return TD_OK;
}

td_status fill_ptrs(const td_request& q, const td_plan& P, std::vector<void*>& v, size_t base)
{
    return fill_ptrs_for(q, P.npatches, P.dt, P.quantity, v.data(), base);
}

// The passes of one plan on one workspace, in pass order, with the field
// pointers in the kernel arguments: no host or device allocation, no
// context lock (twiddles were looked up when the plan was made).
// Debug mode: count the non-finite values a solve wrote to its outputs
// (fx, fy of every patch; v holds the 5 field pointers per patch from
// `base`), on the solve's stream, after its passes.
td_status debug_count(td_context* ctx, const td_plan* P, void* const* v, size_t base, hipStream_t st)
{
    if (!(ctx->debug.load() & TD_DEBUG_NONFINITE) || !ctx->d_nonfinite) return TD_OK;
    for (int k = 0; k < P->npatches; ++k)
        for (int c = 3; c < 5; ++c) {
            const void* p = v[base + 5 * k + c];
            if (!p) continue;
            const int64_t n = (int64_t)P->patch_n[k] * P->patch_n[k];
            TD_HIP(launch_count_nonfinite(P->dt == TD_F64, p, n, ctx->d_nonfinite, st));
        }
    return TD_OK;
}

td_status launch_plan_direct(const td_plan* P, char* ws, const FieldPtrs& fp, hipStream_t st)
{
    const bool f64 = P->dt == TD_F64;
    for (int pass = 0; pass < NTIMED; ++pass)
        for (const Group& g : P->groups) {
            hipError_t e = hipSuccess;
            if (pass == P_ROWFWD) {
                const int n = (int)g.rowfwd.size();
                if (!n) continue;
                const auto t = single_seg<RowFwdJob>(g.d_rowfwd, n, 0, (const void*)P->d_lp, ws);
                e = f64 ? launch_row_fwd<double>(g.M, g.C[P_ROWFWD], n, t, nullptr, fp, g.tw, true, st)
                        : launch_row_fwd<float>(g.M, g.C[P_ROWFWD], n, t, nullptr, fp, g.tw, true, st);
            } else if (pass == P_COL) {
                const int n = (int)g.col.size();
                if (!n) continue;
                const auto t = single_seg<ColJob>(g.d_col, n, 0, (const void*)g.d_coltabs, ws);
                e = f64 ? launch_col<double>(g.M, g.C[P_COL], g.G[P_COL], n, t, g.tw, st)
                        : launch_col<float>(g.M, g.C[P_COL], g.G[P_COL], n, t, g.tw, st);
            } else {
                const int a = pass == P_ROWINV ? 0 : 1;
                const int n = (int)g.rinv[a].size();
                if (!n) continue;
                const auto t = single_seg<RowInvJob>(g.d_rinv[a], n, 0, (const void*)g.d_rinv_tabs, ws);
                e = f64 ? launch_row_inv<double>(g.M, g.C[P_ROWINV], g.G[P_ROWINV], n, t, nullptr, fp, g.tw, st,
                                                 g.nq[a])
                        : launch_row_inv<float>(g.M, g.C[P_ROWINV], g.G[P_ROWINV], n, t, nullptr, fp, g.tw, st,
                                                g.nq[a]);
            }
            if (e != hipSuccess) return fail(TD_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
        }
    return TD_OK;
}

}  // namespace

// ===========================================================================
// public: context
// ===========================================================================

extern "C" td_status td_context_create(int dev, size_t budget, td_context** out)
{
    ErrScope es_;
    if (!out) return fail(TD_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    TD_HIP(hipGetDeviceCount(&ndev));
    if (dev < 0 || dev >= ndev) return fail(TD_EINVAL, "no such HIP device");
    DeviceGuard g(dev);
    hipDeviceProp_t prop;
    TD_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos)
        return fail(TD_EUNSUPPORTED, std::string("built for gfx950, device is ") + prop.gcnArchName);
    TD_HIP(prepare_kernels());
    // the allocation-free solve's device workspace on this device (looked
    // up once per device, with it current)
    {
        void* scratch = nullptr;
        TD_HIP(noalloc_scratch(dev, &scratch));
    }
    auto* c = new td_context();
    c->device = dev;
    c->cus = prop.multiProcessorCount;
    c->budget = budget;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return fail(TD_EDEVICE, hipGetErrorString(e));
    }
    *out = c;
    return TD_OK;
}

extern "C" td_status td_context_destroy(td_context* c)
{
    ErrScope es_;
    if (!c) return fail(TD_EINVAL, "NULL context");
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    for (auto& t : c->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto& kv : c->spectra) c->release(kv.second.ptr, kv.second.bytes);
    c->release(c->b_table, c->b_table_bytes);
    c->release(c->b_rows, c->b_rows_bytes);
    c->release(c->b_small, c->b_small_bytes);
    if (c->d_nonfinite) (void)hipFree(c->d_nonfinite);
    for (auto& kv : c->tw32) (void)hipFree(kv.second);
    for (auto& kv : c->tw64) (void)hipFree(kv.second);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return TD_OK;
}

extern "C" td_status td_context_usage(const td_context* c, size_t* in_use, size_t* spectra)
{
    ErrScope es_;
    if (!c) return fail(TD_EINVAL, "NULL context");
    if (in_use) *in_use = c->used.load();
    if (spectra) *spectra = c->spectra_bytes.load();
    return TD_OK;
}

extern "C" td_status td_context_set_debug(td_context* c, int32_t flags)
{
    ErrScope es_;
    if (!c) return fail(TD_EINVAL, "NULL context");
    if (flags & ~TD_DEBUG_NONFINITE) return fail(TD_EINVAL, "unknown debug flag");
    DeviceGuard g(c->device);
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if ((flags & TD_DEBUG_NONFINITE) && !c->d_nonfinite) {
        TD_HIP(hipMalloc((void**)&c->d_nonfinite, sizeof(unsigned long long)));
        TD_HIP(hipMemset(c->d_nonfinite, 0, sizeof(unsigned long long)));
    }
    c->debug.store(flags);
    return TD_OK;
}

extern "C" td_status td_debug_nonfinite(td_context* c, uint64_t* count)
{
    ErrScope es_;
    if (!c || !count) return fail(TD_EINVAL, "NULL argument");
    *count = 0;
    if (!c->d_nonfinite) return TD_OK;
    DeviceGuard g(c->device);
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    unsigned long long h = 0;
    TD_HIP(hipDeviceSynchronize());
    TD_HIP(hipMemcpy(&h, c->d_nonfinite, sizeof(h), hipMemcpyDeviceToHost));
    TD_HIP(hipMemset(c->d_nonfinite, 0, sizeof(unsigned long long)));
    *count = h;
    return TD_OK;
}

// ===========================================================================
// public: plans and solves
// ===========================================================================

extern "C" td_status td_plan_create(td_context* ctx, const td_hierarchy* h, td_dtype dt,
                                    td_plan** out)
{
    ErrScope es_;
    return td_plan_create_quantity(ctx, h, dt, TD_FORCE, out);
}

extern "C" td_status td_plan_create_quantity(td_context* ctx, const td_hierarchy* h, td_dtype dt,
                                             int32_t quantity, td_plan** out)
{
    ErrScope es_;
    if (!ctx || !out) return fail(TD_EINVAL, "NULL argument");
    *out = nullptr;
    if (dt != TD_F32 && dt != TD_F64) return fail(TD_EINVAL, "dtype must be TD_F32 or TD_F64");
    if (quantity != TD_FORCE && quantity != TD_POTENTIAL)
        return fail(TD_EINVAL, "quantity must be TD_FORCE or TD_POTENTIAL");
    TD_TRY(td_hierarchy_check(h));
    DeviceGuard dg(ctx->device);
    std::unique_ptr<td_plan> P(new td_plan());
    P->ctx = ctx;
    P->quantity = quantity;
    TD_TRY(plan_geometry(P.get(), h, dt));
    size_t elems = 0;
    td_status st = build_jobs(P.get(), &elems, true);
    P->ws_bytes = elems * elem_size(dt);
    // the twiddles of every length, looked up once here: launches then
    // take no context lock (a spectrum build on another thread holds it)
    for (auto& g : P->groups)
        if (st == TD_OK) st = twiddles(ctx, g.M, dt, &g.tw);
    if (st == TD_OK) st = validate_jobs(P.get());
    if (st == TD_OK) st = plan_upload(P.get());
    if (st != TD_OK) {
        plan_free(P.get());
        return st;
    }
    // spectra bytes this plan reads
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        std::vector<const void*> seen;
        for (auto& g : P->groups) {
            for (auto& t : g.colins)
                if (std::find(seen.begin(), seen.end(), t.kern) == seen.end()) seen.push_back(t.kern);
            for (auto& t : g.colouts)
                if (t.kern && std::find(seen.begin(), seen.end(), t.kern) == seen.end()) seen.push_back(t.kern);
        }
        size_t b = 0;
        for (auto& kv : ctx->spectra) {
            const char* lo = (const char*)kv.second.ptr;
            for (const void* p : seen)
                if ((const char*)p >= lo && (const char*)p < lo + kv.second.bytes) {
                    b += kv.second.bytes;
                    break;
                }
        }
        P->spectra_bytes = b;
    }
    *out = P.release();
    return TD_OK;
}

extern "C" td_status td_plan_check(const td_hierarchy* h, td_dtype dt, size_t* workspace_bytes)
{
    ErrScope es_;
    if (dt != TD_F32 && dt != TD_F64) return fail(TD_EINVAL, "dtype must be TD_F32 or TD_F64");
    TD_TRY(td_hierarchy_check(h));
    static td_context host_ctx;  // default launch shapes, no device
    td_plan P;
    P.ctx = &host_ctx;
    P.dry = true;
    TD_TRY(plan_geometry(&P, h, dt));
    size_t elems = 0;
    TD_TRY(build_jobs(&P, &elems, true));
    P.ws_bytes = elems * elem_size(dt);
    TD_TRY(validate_jobs(&P));
    if (workspace_bytes) *workspace_bytes = P.ws_bytes;
    return TD_OK;
}

extern "C" td_status td_plan_footprint(const td_plan* p, size_t* ws, size_t* spec)
{
    ErrScope es_;
    if (!p) return fail(TD_EINVAL, "NULL plan");
    if (ws) *ws = p->ws_bytes + p->job_bytes;
    if (spec) *spec = p->spectra_bytes;
    return TD_OK;
}

extern "C" td_status td_plan_destroy(td_plan* p)
{
    ErrScope es_;
    if (!p) return fail(TD_EINVAL, "NULL plan");
    DeviceGuard g(p->ctx->device);
    plan_free(p);
    delete p;
    return TD_OK;
}

extern "C" td_status td_solve(const td_request* req, void* stream)
{
    ErrScope es_;
    if (!req || !req->plan) return fail(TD_EINVAL, "NULL request or plan");
    td_plan* P = req->plan;
    DeviceGuard g(P->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<void*> v(5 * P->npatches, nullptr);
    TD_TRY(fill_ptrs(*req, *P, v, 0));
    if (!P->ws) TD_TRY(P->ctx->alloc(P->ws_bytes, &P->ws));
    // one solve: the field pointers travel in the kernel arguments
    static_assert(5 * TD_MAX_PATCHES <= TD_KARG_PTRS, "kernel-argument pointer table too small");
    FieldPtrs fp{};
    fp.n = (int32_t)v.size();
    for (size_t i = 0; i < v.size(); ++i) fp.p[i] = v[i];
    std::vector<Member> mem{{P, 0, (char*)P->ws}};
    TD_TRY(launch_members(P->ctx, P->dt, mem, nullptr, fp, st));
    return debug_count(P->ctx, P, v.data(), 0, st);
}

extern "C" td_status td_solve_noalloc(const td_request* req, void* stream)
{
    ErrScope es_;
    if (!req || !req->plan) return fail(TD_EINVAL, "NULL request or plan");
    const td_plan* P = req->plan;
    if (P->ws_bytes > TD_NOALLOC_SCRATCH_BYTES)
        return fail(TD_ENOMEM, "td_solve_noalloc: the plan's workspace (" + std::to_string(P->ws_bytes) +
                                   " bytes) exceeds the fixed scratch of " +
                                   std::to_string((size_t)TD_NOALLOC_SCRATCH_BYTES) + " bytes");
    DeviceGuard g(P->ctx->device);
    void* v[5 * TD_MAX_PATCHES];
    TD_TRY(fill_ptrs_for(*req, P->npatches, P->dt, P->quantity, v, 0));
    void* scratch = nullptr;
    TD_HIP(noalloc_scratch(P->ctx->device, &scratch));
    static_assert(5 * TD_MAX_PATCHES <= TD_KARG_PTRS, "kernel-argument pointer table too small");
    FieldPtrs fp{};
    fp.n = 5 * P->npatches;
    for (int i = 0; i < fp.n; ++i) fp.p[i] = v[i];
    TD_TRY(launch_plan_direct(P, (char*)scratch, fp, (hipStream_t)stream));
    return debug_count(P->ctx, P, v, 0, (hipStream_t)stream);
}

// ===========================================================================
// public: batches
// ===========================================================================

struct td_batch {
    td_context* ctx = nullptr;
    td_dtype dt = TD_F32;
    std::vector<td_plan*> plans;  // borrowed: must outlive the batch
    std::vector<Member> mem;
    size_t nslots = 0;
    void** d_ptrs = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    Stager stager;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
    // the pointer table last copied to d_ptrs, and the stream it went on: a
    // solve on that stream with the same pointers needs no new copy
    std::vector<void*> last_ptrs;
    hipStream_t last_stream = nullptr;
    bool pushed = false;
    // persistent launches (td_batch_set_launch): the recorded work queues
    int launch_mode = TD_LAUNCH_DIRECT;
    Queues queues;
};

namespace {

// Record the batch's column launches and upload their work lists: the
// TD_NXCD counters of every launch (zeroed by a kernel ahead of each
// solve), then per launch the TD_NXCD + 1 list starts and the job order.
td_status build_queues(td_batch* B)
{
    Queues& qs = B->queues;
    qs.building = true;
    td_status s = launch_members(B->ctx, B->dt, B->mem, nullptr, FieldPtrs{}, nullptr, &qs);
    qs.building = false;
    if (s != TD_OK) return s;
    const size_t nl = qs.recs.size();
    size_t words = nl * TD_NXCD + nl * (TD_NXCD + 1);
    for (auto& o : qs.order) words += o.size();
    std::vector<int32_t> host(words, 0);
    size_t at = nl * TD_NXCD;
    std::vector<size_t> st_at(nl), or_at(nl);
    for (size_t i = 0; i < nl; ++i) {
        st_at[i] = at;
        std::copy(qs.start[i].begin(), qs.start[i].end(), host.begin() + at);
        at += TD_NXCD + 1;
        or_at[i] = at;
        std::copy(qs.order[i].begin(), qs.order[i].end(), host.begin() + at);
        at += qs.order[i].size();
    }
    qs.dev_bytes = std::max<size_t>(4, words * sizeof(int32_t));
    TD_TRY(B->ctx->alloc(qs.dev_bytes, &qs.dev));
    TD_HIP(hipMemcpy(qs.dev, host.data(), words * sizeof(int32_t), hipMemcpyHostToDevice));
    int32_t* d = (int32_t*)qs.dev;
    for (size_t i = 0; i < nl; ++i) {
        qs.recs[i].q.counter = (unsigned int*)(d + i * TD_NXCD);
        qs.recs[i].q.start = d + st_at[i];
        qs.recs[i].q.order = d + or_at[i];
    }
    qs.order.clear();
    qs.start.clear();
    return TD_OK;
}

// The batch's launches on stream st: with persistent launches, first zero
// the work-list counters.
td_status batch_launch(td_batch* B, hipStream_t st)
{
    Queues* qs = nullptr;
    if (B->launch_mode == TD_LAUNCH_PERSISTENT && !B->queues.recs.empty()) {
        qs = &B->queues;
        TD_HIP(launch_zero_counters((unsigned int*)qs->dev, (int)(qs->recs.size() * TD_NXCD), st));
    }
    return launch_members(B->ctx, B->dt, B->mem, B->d_ptrs, FieldPtrs{}, st, qs);
}

}  // namespace

extern "C" td_status td_batch_create(td_context* ctx, int32_t count, td_plan* const* plans,
                                     td_batch** out)
{
    ErrScope es_;
    if (!ctx || !plans || !out || count < 1) return fail(TD_EINVAL, "bad batch arguments");
    *out = nullptr;
    DeviceGuard dg(ctx->device);
    std::unique_ptr<td_batch> B(new td_batch());
    B->ctx = ctx;
    B->dt = plans[0] ? plans[0]->dt : TD_F32;
    std::vector<size_t> ws_off;
    for (int k = 0; k < count; ++k) {
        td_plan* p = plans[k];
        if (!p || p->ctx != ctx || p->dt != B->dt)
            return fail(TD_EINVAL, "batch members must be plans of one context and dtype");
        B->plans.push_back(p);
        ws_off.push_back(B->ws_bytes);
        B->mem.push_back({p, (int)B->nslots, nullptr});
        B->nslots += 5 * p->npatches;
        B->ws_bytes += (p->ws_bytes + 255) & ~size_t(255);
    }
    td_status st = ctx->alloc(B->ws_bytes, &B->ws);
    if (st == TD_OK) st = ctx->alloc(sizeof(void*) * B->nslots, (void**)&B->d_ptrs);
    if (st == TD_OK) st = B->stager.init(B->nslots);
    if (st != TD_OK) {
        if (B->ws) ctx->release(B->ws, B->ws_bytes);
        if (B->d_ptrs) ctx->release(B->d_ptrs, sizeof(void*) * B->nslots);
        B->stager.destroy();
        return st;
    }
    for (size_t k = 0; k < B->mem.size(); ++k) B->mem[k].ws = (char*)B->ws + ws_off[k];
    st = build_queues(B.get());
    if (st != TD_OK) {
        ctx->release(B->ws, B->ws_bytes);
        ctx->release(B->d_ptrs, sizeof(void*) * B->nslots);
        B->stager.destroy();
        return st;
    }
    *out = B.release();
    return TD_OK;
}

extern "C" td_status td_batch_set_launch(td_batch* B, int32_t mode)
{
    ErrScope es_;
    if (!B) return fail(TD_EINVAL, "NULL batch");
    if (mode != TD_LAUNCH_DIRECT && mode != TD_LAUNCH_PERSISTENT) return fail(TD_EINVAL, "unknown launch mode");
    if (mode == B->launch_mode) return TD_OK;
    DeviceGuard dg(B->ctx->device);
    // the captured graph holds the old launches
    if (B->exec || B->graph) TD_HIP(hipDeviceSynchronize());
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->launch_mode = mode;
    return TD_OK;
}

extern "C" td_status td_batch_solve(td_batch* B, const td_request* reqs, int use_graph,
                                    void* stream)
{
    ErrScope es_;
    if (!B || !reqs) return fail(TD_EINVAL, "NULL batch or requests");
    DeviceGuard dg(B->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<void*> v(B->nslots, nullptr);
    for (size_t k = 0; k < B->plans.size(); ++k) {
        if (reqs[k].plan != B->plans[k]) return fail(TD_EINVAL, "request plan does not match the batch");
        TD_TRY(fill_ptrs(reqs[k], *B->plans[k], v, B->mem[k].slot_base));
    }
    if (use_graph && !B->exec) {
        // Capture once on a private stream; the pointer-table copy stays
        // outside the graph so every replay reads the current pointers.
        if (!B->graph_stream) TD_HIP(hipStreamCreateWithFlags(&B->graph_stream, hipStreamNonBlocking));
        for (auto& m : B->mem)
            for (auto& g : m.plan->groups) {
                const void* tw = nullptr;
                TD_TRY(twiddles(B->ctx, g.M, B->dt, &tw));
            }
        TD_HIP(hipStreamBeginCapture(B->graph_stream, hipStreamCaptureModeThreadLocal));
        td_status s = batch_launch(B, B->graph_stream);
        hipGraph_t gph = nullptr;
        hipError_t e = hipStreamEndCapture(B->graph_stream, &gph);
        if (s != TD_OK) {
            if (gph) (void)hipGraphDestroy(gph);
            return s;
        }
        if (e != hipSuccess) return fail(TD_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        B->graph = gph;
        TD_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    }
    // d_ptrs is written only here: stream order makes an identical earlier
    // copy on the same stream visible to these launches
    if (!(B->pushed && st == B->last_stream && v == B->last_ptrs)) {
        TD_TRY(B->stager.push(B->d_ptrs, v, st));
        B->last_ptrs = v;
        B->last_stream = st;
        B->pushed = true;
    }
    if (!use_graph) TD_TRY(batch_launch(B, st));
    else TD_HIP(hipGraphLaunch(B->exec, st));
    for (auto& m : B->mem) TD_TRY(debug_count(B->ctx, m.plan, v.data(), m.slot_base, st));
    return TD_OK;
}

extern "C" td_status td_batch_footprint(const td_batch* B, size_t* ws)
{
    ErrScope es_;
    if (!B) return fail(TD_EINVAL, "NULL batch");
    if (ws) *ws = B->ws_bytes;
    return TD_OK;
}

extern "C" td_status td_batch_destroy(td_batch* B)
{
    ErrScope es_;
    if (!B) return fail(TD_EINVAL, "NULL batch");
    DeviceGuard dg(B->ctx->device);
    (void)hipDeviceSynchronize();
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->graph_stream) (void)hipStreamDestroy(B->graph_stream);
    if (B->ws) B->ctx->release(B->ws, B->ws_bytes);
    if (B->d_ptrs) B->ctx->release(B->d_ptrs, sizeof(void*) * B->nslots);
    if (B->queues.dev) B->ctx->release(B->queues.dev, B->queues.dev_bytes);
    B->stager.destroy();
    delete B;
    return TD_OK;
}

// ===========================================================================
// public: serving loop
// ===========================================================================

namespace {

enum TicketState { T_QUEUED = 0, T_RUNNING = 1, T_DONE = 2, T_CANCELLED = 3, T_PLANNING = 4,
                   T_FAILED = 5 };

struct Ticket {
    uint64_t id = 0;
    td_plan* plan = nullptr;
    std::vector<void*> ptrs;  // 5 per patch: sigma, dsdx, dsdy, fx, fy
    double t_submit = 0, t_done = 0;
    int state = T_QUEUED;
    size_t need = 0;
    hipEvent_t inputs = nullptr;  // recorded on the submitter's stream
    td_status error = TD_OK;      // T_FAILED
    std::string message;
    // T_PLANNING: the hierarchy the server plans before admission
    std::vector<td_patch> patches;
    td_hierarchy hier{};
    td_dtype dt = TD_F32;
    int quantity = TD_FORCE;
};

struct Flight {
    td_server* owner = nullptr;
    hipStream_t stream = nullptr;
    void** d_ptrs = nullptr;
    size_t cap = 0;
    Stager stager;
    std::vector<uint64_t> tickets;
    std::vector<std::pair<void*, size_t>> ws;  // workspace blocks bound to the tickets
    bool active = false;
    // set by the host callback after the flight's work (the callback takes
    // no lock a HIP call could be made under: see flight_finished)
    std::atomic<bool> finished{false};
    std::atomic<double> t_finish{0.0};
};

// The server's flights, sized once at creation (callbacks hold pointers).
struct FlightArray {
    std::unique_ptr<Flight[]> p;
    int n = 0;
    Flight* begin() { return p.get(); }
    Flight* end() { return p.get() + n; }
};

}  // namespace

struct td_server {
    td_context* ctx = nullptr;
    int max_inflight = 2, max_batch = 16;
    size_t queue_cap = 1 << 16;
    std::mutex mu;
    std::condition_variable cv_done, cv_plan;
    // wake-ups of the worker: a counter bumped under wake_mu, which is never
    // held across a HIP call (the flights' host callbacks bump it too)
    std::mutex wake_mu;
    std::condition_variable wake_cv;
    std::atomic<uint64_t> wake_seq{0};
    std::deque<uint64_t> queue;   // admitted to the queue, waiting for a flight
    std::deque<uint64_t> planq;   // waiting for the planner
    std::map<uint64_t, Ticket> tickets;
    FlightArray flights;
    std::multimap<size_t, void*> pool;  // idle workspace blocks (held, counted as used)
    std::vector<std::pair<void*, size_t>> pool_all;
    std::vector<hipEvent_t> ev_pool;
    std::map<std::string, td_plan*> plans;  // plans the server made, by hierarchy
    std::thread worker;
    std::vector<std::thread> planners;
    bool stop = false;
    uint64_t next_id = 1;
    uint64_t completed = 0, cancelled = 0, refused = 0, deferred = 0, batches = 0, peak_queue = 0,
             planned = 0, failed = 0;
    std::string worker_error;
};

namespace {

void wake(td_server* S)
{
    {
        std::lock_guard<std::mutex> g(S->wake_mu);
        S->wake_seq.fetch_add(1, std::memory_order_acq_rel);
    }
    S->wake_cv.notify_all();
}

// Host callback at the end of a flight's stream work.  It runs on a HIP
// runtime thread, so it makes no HIP call and takes no lock that another
// thread may hold while inside the HIP runtime (the server mutex is held
// around allocations): the flag is atomic, and the wake-up mutex is only
// ever held for a counter increment or a condition wait.
void flight_finished(void* arg)
{
    Flight* f = static_cast<Flight*>(arg);
    f->t_finish.store(now_s(), std::memory_order_relaxed);
    f->finished.store(true, std::memory_order_release);
    wake(f->owner);
}

// Workspace for one admitted solve: reuse an idle block of a close size, or
// allocate against the context's HBM budget.  Returns nullptr when the
// budget has no room (the request waits); idle blocks that would make room
// are moved to `to_free`, which the caller frees outside the server lock
// (hipFree waits for the device).
void* pool_get(td_server* S, size_t need, size_t* got, std::vector<std::pair<void*, size_t>>& to_free)
{
    auto it = S->pool.lower_bound(need);
    if (it != S->pool.end() && it->first <= 2 * need + (1 << 20)) {
        void* p = it->second;
        *got = it->first;
        S->pool.erase(it);
        return p;
    }
    void* p = nullptr;
    if (S->ctx->alloc(need, &p) == TD_OK) {
        S->pool_all.push_back({p, need});
        *got = need;
        return p;
    }
    // no room: give the idle blocks back (freed by the caller), so that a
    // later attempt can allocate
    for (auto& kv : S->pool) {
        for (auto a = S->pool_all.begin(); a != S->pool_all.end(); ++a)
            if (a->first == kv.second) {
                S->pool_all.erase(a);
                break;
            }
        to_free.push_back({kv.second, kv.first});
    }
    S->pool.clear();
    return nullptr;
}

void fail_ticket(td_server* S, Ticket& T, td_status st, const std::string& msg)
{
    T.state = T_FAILED;
    T.error = st;
    T.message = msg;
    T.t_done = now_s();
    S->failed++;
}

void server_loop(td_server* S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    bool mem_blocked = false;  // the queue head waits for memory a flight holds
    while (true) {
        // wake-ups from here on are seen by the wait at the bottom
        const uint64_t seen = S->wake_seq.load(std::memory_order_acquire);
        // retire finished flights (their host callback has run)
        bool progressed = false;
        for (auto& f : S->flights) {
            if (!f.active || !f.finished.load(std::memory_order_acquire)) continue;
            for (uint64_t id : f.tickets) {
                auto it = S->tickets.find(id);
                if (it != S->tickets.end()) {
                    it->second.state = T_DONE;
                    it->second.t_done = f.t_finish.load(std::memory_order_relaxed);
                    if (it->second.inputs) S->ev_pool.push_back(it->second.inputs);
                    it->second.inputs = nullptr;
                }
                S->completed++;
            }
            for (auto& w : f.ws) S->pool.insert({w.second, w.first});
            f.ws.clear();
            f.tickets.clear();
            f.active = false;
            f.finished.store(false, std::memory_order_relaxed);
            progressed = true;
        }
        if (progressed) {
            mem_blocked = false;
            S->cv_done.notify_all();
        }
        // continuous batching: a free flight slot takes the requests that
        // have arrived so far (FIFO, up to max_batch) that fit in HBM
        Flight* slot = nullptr;
        for (auto& f : S->flights)
            if (!f.active) {
                slot = &f;
                break;
            }
        bool any_active = false;
        for (auto& f : S->flights) any_active |= f.active;
        if (slot && !S->queue.empty() && !mem_blocked) {
            std::vector<uint64_t> pick;
            std::vector<Member> mem;
            std::vector<std::pair<void*, size_t>> blocks, to_free;
            size_t nslots = 0;
            bool waited = false;
            for (auto it = S->queue.begin(); it != S->queue.end() && (int)pick.size() < S->max_batch;) {
                Ticket& T = S->tickets[*it];
                if (T.state == T_CANCELLED) {
                    it = S->queue.erase(it);
                    continue;
                }
                if (!mem.empty() && mem[0].plan->dt != T.plan->dt) {
                    ++it;
                    continue;
                }
                size_t got = 0;
                void* ws = pool_get(S, T.need, &got, to_free);
                if (!ws) {
                    waited = true;
                    ++it;
                    continue;
                }
                blocks.push_back({ws, got});
                mem.push_back({T.plan, (int)nslots, (char*)ws});
                nslots += 5 * T.plan->npatches;
                pick.push_back(*it);
                it = S->queue.erase(it);
            }
            if (waited) S->deferred++;
            if (!to_free.empty()) {
                lk.unlock();
                for (auto& b : to_free) S->ctx->release(b.first, b.second);
                lk.lock();
            }
            if (pick.empty()) {
                if (!to_free.empty()) continue;  // idle blocks were just freed: retry
                if (waited && !any_active) {
                    // nothing runs and nothing idles: the head cannot fit
                    Ticket& T = S->tickets[S->queue.front()];
                    fail_ticket(S, T, TD_ENOMEM, "request workspace does not fit in the HBM budget");
                    S->queue.pop_front();
                    S->cv_done.notify_all();
                } else if (waited) {
                    mem_blocked = any_active;  // wait for a flight to free memory
                }
                continue;
            }
            // the flight holds its requests from here on (drain sees them
            // in flight while the lock is released below)
            slot->active = true;
            slot->finished.store(false, std::memory_order_relaxed);
            slot->tickets = pick;
            slot->ws = blocks;
            // the flight's device pointer table: grown before the launch,
            // so a failure leaves the slot idle and the requests back at the
            // head of the queue
            td_status st = TD_OK;
            if (slot->cap < nslots) {
                // only this thread touches an idle slot; the allocations and
                // frees (which wait for the device, hence for the flights'
                // callbacks, which take the lock) run unlocked
                lk.unlock();
                const size_t cap = std::max<size_t>(nslots, 1024);
                void** d = nullptr;
                Stager stg;
                st = S->ctx->alloc(sizeof(void*) * cap, (void**)&d);
                if (st == TD_OK) {
                    st = stg.init(cap);
                    if (st != TD_OK) {
                        stg.destroy();
                        S->ctx->release(d, sizeof(void*) * cap);
                    }
                }
                if (st == TD_OK) {
                    // the old table's last copies are complete: the slot is idle
                    if (slot->d_ptrs) S->ctx->release(slot->d_ptrs, sizeof(void*) * slot->cap);
                    slot->stager.destroy();
                    slot->d_ptrs = d;
                    slot->stager = stg;
                    slot->cap = cap;
                }
                lk.lock();
            }
            if (st != TD_OK) {
                const std::string why = td_last_error();
                slot->active = false;
                slot->tickets.clear();
                slot->ws.clear();
                for (auto it = pick.rbegin(); it != pick.rend(); ++it) S->queue.push_front(*it);
                for (auto& b : blocks) S->pool.insert({b.second, b.first});
                mem_blocked = any_active;
                if (!any_active) {
                    // cannot make progress: fail the head rather than spin
                    Ticket& T = S->tickets[S->queue.front()];
                    fail_ticket(S, T, st, "flight pointer table: " + why);
                    S->queue.pop_front();
                    S->cv_done.notify_all();
                }
                continue;
            }
            std::vector<void*> v(nslots, nullptr);
            std::vector<hipEvent_t> waits;
            for (size_t k = 0; k < pick.size(); ++k) {
                Ticket& T = S->tickets[pick[k]];
                T.state = T_RUNNING;
                std::copy(T.ptrs.begin(), T.ptrs.end(), v.begin() + mem[k].slot_base);
                if (T.inputs) waits.push_back(T.inputs);
            }
            S->batches++;
            const td_dtype dt = mem[0].plan->dt;
            lk.unlock();
            for (hipEvent_t e : waits)
                if (st == TD_OK && hipStreamWaitEvent(slot->stream, e, 0) != hipSuccess)
                    st = fail(TD_EDEVICE, "hipStreamWaitEvent");
            if (st == TD_OK) st = slot->stager.push(slot->d_ptrs, v, slot->stream);
            if (st == TD_OK) st = launch_members(S->ctx, dt, mem, slot->d_ptrs, FieldPtrs{}, slot->stream);
            for (size_t k = 0; st == TD_OK && k < mem.size(); ++k)
                st = debug_count(S->ctx, mem[k].plan, v.data(), mem[k].slot_base, slot->stream);
            const bool cb = st == TD_OK &&
                            hipLaunchHostFunc(slot->stream, flight_finished, slot) == hipSuccess;
            lk.lock();
            if (!cb) {
                // nothing will call back: finish the flight here, after its
                // stream has drained, with its tickets failed
                if (st == TD_OK) st = fail(TD_EDEVICE, "hipLaunchHostFunc");
                S->worker_error = td_last_error();
                lk.unlock();
                (void)hipStreamSynchronize(slot->stream);
                lk.lock();
                for (uint64_t id : slot->tickets) {
                    Ticket& T = S->tickets[id];
                    fail_ticket(S, T, st, S->worker_error);
                }
                for (auto& w : slot->ws) S->pool.insert({w.second, w.first});
                slot->ws.clear();
                slot->tickets.clear();
                slot->active = false;
                S->cv_done.notify_all();
            }
            continue;
        }
        if (S->stop && S->queue.empty() && S->planq.empty() && !any_active) break;
        if (progressed) continue;  // retired flights may let the queue move
        // sleep until a flight finishes, a request arrives or the server
        // stops (any of which bumps the wake counter)
        lk.unlock();
        {
            std::unique_lock<std::mutex> wk(S->wake_mu);
            S->wake_cv.wait(wk, [&] { return S->wake_seq.load(std::memory_order_acquire) != seen; });
        }
        lk.lock();
    }
}

std::string hierarchy_key(const td_hierarchy& h, td_dtype dt, int quantity)
{
    std::ostringstream o;
    o.precision(17);
    o << (int)dt << ' ' << quantity << ' ' << h.x0 << ' ' << h.y0 << ' ' << h.h0 << ' ' << h.ratio << ' '
      << h.aspect;
    for (int k = 0; k < h.npatches; ++k)
        o << ' ' << h.patches[k].level << ',' << h.patches[k].n << ',' << h.patches[k].ox << ','
          << h.patches[k].oy;
    return o.str();
}

// Plans the hierarchies of tickets submitted without a plan, off the worker
// thread: plan creation builds spectra and uploads job lists on the
// context's own stream and waits only for that stream, so flights keep
// running meanwhile.  Plans are kept per hierarchy for later requests.
void planner_loop(td_server* S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->cv_plan.wait(lk, [&] { return S->stop || !S->planq.empty(); });
        if (S->planq.empty()) {
            if (S->stop) break;
            continue;
        }
        const uint64_t id = S->planq.front();
        S->planq.pop_front();
        auto it = S->tickets.find(id);
        if (it == S->tickets.end() || it->second.state != T_PLANNING) continue;
        td_hierarchy h = it->second.hier;
        std::vector<td_patch> pats = it->second.patches;
        h.patches = pats.data();
        const td_dtype dt = it->second.dt;
        const int quantity = it->second.quantity;
        lk.unlock();
        const std::string key = hierarchy_key(h, dt, quantity);
        td_plan* plan = nullptr;
        td_status st = TD_OK;
        std::string msg;
        {
            std::lock_guard<std::mutex> g(S->mu);
            auto pi = S->plans.find(key);
            if (pi != S->plans.end()) plan = pi->second;
        }
        if (!plan) {
            st = td_plan_create_quantity(S->ctx, &h, dt, quantity, &plan);
            if (st == TD_OK) {
                std::lock_guard<std::mutex> g(S->mu);
                auto ins = S->plans.emplace(key, plan);
                if (!ins.second) {  // another planner made it meanwhile
                    td_plan_destroy(plan);
                    plan = ins.first->second;
                }
            } else {
                msg = td_last_error();
            }
        }
        lk.lock();
        it = S->tickets.find(id);
        if (it == S->tickets.end() || it->second.state != T_PLANNING) continue;  // cancelled
        Ticket& T = it->second;
        if (st != TD_OK) {
            fail_ticket(S, T, st, "planning: " + msg);
            S->cv_done.notify_all();
            continue;
        }
        S->planned++;
        T.plan = plan;
        T.need = (plan->ws_bytes + 255) & ~size_t(255);
        if (S->ctx->budget && T.need > S->ctx->budget) {
            fail_ticket(S, T, TD_ENOMEM, "request workspace exceeds the HBM budget");
            S->cv_done.notify_all();
            continue;
        }
        T.state = T_QUEUED;
        S->queue.push_back(id);
        lk.unlock();
        wake(S);
        lk.lock();
    }
}

// Common tail of the two submit calls: the arrival event on the caller's
// stream, the queue limit, the ticket.
td_status submit_ticket(td_server* S, Ticket&& T, int32_t queue_if_full, void* stream,
                        uint64_t* ticket)
{
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->queue.size() + S->planq.size() >= S->queue_cap && !queue_if_full) {
            S->refused++;
            return fail(TD_EBUSY, "server queue full");
        }
        if (!S->ev_pool.empty()) {
            ev = S->ev_pool.back();
            S->ev_pool.pop_back();
        }
    }
    DeviceGuard dg(S->ctx->device);
    if (!ev) TD_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    // the flight waits for the caller's work on its stream up to this point
    // (the inputs it wrote, the earlier uses of the output buffers)
    if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->ev_pool.push_back(ev);
        return fail(TD_EDEVICE, "hipEventRecord on the submitting stream");
    }
    T.inputs = ev;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        T.id = S->next_id++;
        T.t_submit = now_s();
        *ticket = T.id;
        const bool planning = T.state == T_PLANNING;
        S->tickets[T.id] = std::move(T);
        if (planning) {
            S->planq.push_back(*ticket);
            S->cv_plan.notify_all();
        } else {
            S->queue.push_back(*ticket);
        }
        S->peak_queue = std::max<uint64_t>(S->peak_queue, S->queue.size() + S->planq.size());
    }
    wake(S);
    return TD_OK;
}

}  // namespace

extern "C" td_status td_server_create(td_context* ctx, int32_t max_inflight, int32_t max_batch,
                                      td_server** out)
{
    ErrScope es_;
    if (!ctx || !out || max_inflight < 1 || max_batch < 1 || max_batch > 4096)
        return fail(TD_EINVAL, "bad server arguments");
    DeviceGuard dg(ctx->device);
    std::unique_ptr<td_server> S(new td_server());
    S->ctx = ctx;
    S->max_inflight = max_inflight;
    S->max_batch = max_batch;
    S->flights.p.reset(new Flight[max_inflight]);
    S->flights.n = max_inflight;
    for (auto& f : S->flights) {
        f.owner = S.get();
        hipError_t e = hipStreamCreateWithFlags(&f.stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (auto& g : S->flights)
                if (g.stream) (void)hipStreamDestroy(g.stream);
            return fail(TD_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
    }
    td_server* raw = S.release();
    raw->worker = std::thread(server_loop, raw);
    for (int k = 0; k < 2; ++k) raw->planners.emplace_back(planner_loop, raw);
    *out = raw;
    return TD_OK;
}

extern "C" td_status td_server_set_queue_limit(td_server* S, int32_t max_queued)
{
    ErrScope es_;
    if (!S || max_queued < 1) return fail(TD_EINVAL, "bad server or queue limit");
    std::lock_guard<std::mutex> lk(S->mu);
    S->queue_cap = (size_t)max_queued;
    return TD_OK;
}

extern "C" td_status td_server_submit(td_server* S, const td_request* req, int32_t queue_if_full,
                                      void* hip_stream, uint64_t* ticket)
{
    ErrScope es_;
    if (!S || !req || !req->plan || !ticket) return fail(TD_EINVAL, "NULL argument");
    if (req->plan->ctx != S->ctx) return fail(TD_EINVAL, "plan belongs to another context");
    const td_plan* P = req->plan;
    Ticket T;
    T.plan = req->plan;
    T.ptrs.assign(5 * P->npatches, nullptr);
    TD_TRY(fill_ptrs(*req, *P, T.ptrs, 0));
    T.need = (P->ws_bytes + 255) & ~size_t(255);
    if (S->ctx->budget && T.need > S->ctx->budget) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->refused++;
        return fail(TD_ENOMEM, "request workspace exceeds the HBM budget");
    }
    return submit_ticket(S, std::move(T), queue_if_full, hip_stream, ticket);
}

extern "C" td_status td_server_submit_hierarchy(td_server* S, const td_hierarchy* h, td_dtype dtype,
                                                int32_t quantity, const td_request* req,
                                                int32_t queue_if_full, void* hip_stream,
                                                uint64_t* ticket)
{
    ErrScope es_;
    if (!S || !h || !req || !ticket) return fail(TD_EINVAL, "NULL argument");
    if (req->plan) return fail(TD_EINVAL, "req->plan must be NULL: the server plans the hierarchy");
    if (dtype != TD_F32 && dtype != TD_F64) return fail(TD_EINVAL, "dtype must be TD_F32 or TD_F64");
    if (quantity != TD_FORCE && quantity != TD_POTENTIAL)
        return fail(TD_EINVAL, "quantity must be TD_FORCE or TD_POTENTIAL");
    TD_TRY(td_hierarchy_check(h));
    Ticket T;
    T.state = T_PLANNING;
    T.dt = dtype;
    T.quantity = quantity;
    T.patches.assign(h->patches, h->patches + h->npatches);
    T.hier = *h;
    T.hier.patches = nullptr;
    T.ptrs.assign(5 * h->npatches, nullptr);
    TD_TRY(fill_ptrs_for(*req, h->npatches, dtype, quantity, T.ptrs.data(), 0));
    return submit_ticket(S, std::move(T), queue_if_full, hip_stream, ticket);
}

extern "C" td_status td_server_poll(td_server* S, uint64_t ticket, int32_t* done, double* lat)
{
    ErrScope es_;
    if (!S || !done) return fail(TD_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->worker_error.empty() && S->tickets.count(ticket) &&
        S->tickets[ticket].state == T_RUNNING)
        return fail(TD_EDEVICE, "server: " + S->worker_error);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(TD_EINVAL, "unknown ticket (or already reported done)");
    if (it->second.state == T_FAILED) {
        const td_status st = it->second.error;
        const std::string msg = it->second.message;
        S->tickets.erase(it);
        return fail(st, "request failed: " + msg);
    }
    *done = it->second.state == T_DONE ? 1 : 0;
    if (lat) *lat = *done ? it->second.t_done - it->second.t_submit : 0.0;
    if (*done) S->tickets.erase(it);  // reported once; the map does not grow without bound
    return TD_OK;
}

extern "C" td_status td_server_drain(td_server* S)
{
    ErrScope es_;
    if (!S) return fail(TD_EINVAL, "NULL server");
    wake(S);
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] {
        if (!S->queue.empty() || !S->planq.empty()) return false;
        for (auto& kv : S->tickets)
            if (kv.second.state == T_PLANNING) return false;
        for (auto& f : S->flights)
            if (f.active) return false;
        return true;
    });
    if (!S->worker_error.empty()) return fail(TD_EDEVICE, "server: " + S->worker_error);
    return TD_OK;
}

extern "C" td_status td_server_cancel(td_server* S, uint64_t ticket)
{
    ErrScope es_;
    if (!S) return fail(TD_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end() || (it->second.state != T_QUEUED && it->second.state != T_PLANNING))
        return fail(TD_EINVAL, "ticket unknown or already started");
    if (it->second.inputs) S->ev_pool.push_back(it->second.inputs);
    S->cancelled++;
    S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), ticket), S->queue.end());
    S->planq.erase(std::remove(S->planq.begin(), S->planq.end(), ticket), S->planq.end());
    S->tickets.erase(it);
    S->cv_done.notify_all();
    return TD_OK;
}

extern "C" td_status td_server_stats(const td_server* S, uint64_t* completed, uint64_t* cancelled,
                                     uint64_t* refused, uint64_t* deferred, uint64_t* batches,
                                     uint64_t* peak_queue)
{
    ErrScope es_;
    if (!S) return fail(TD_EINVAL, "NULL server");
    auto* s = const_cast<td_server*>(S);
    std::lock_guard<std::mutex> lk(s->mu);
    if (completed) *completed = s->completed;
    if (cancelled) *cancelled = s->cancelled;
    if (refused) *refused = s->refused;
    if (deferred) *deferred = s->deferred;
    if (batches) *batches = s->batches;
    if (peak_queue) *peak_queue = s->peak_queue;
    return TD_OK;
}

extern "C" td_status td_server_stats2(const td_server* S, uint64_t* planned, uint64_t* failed)
{
    ErrScope es_;
    if (!S) return fail(TD_EINVAL, "NULL server");
    auto* s = const_cast<td_server*>(S);
    std::lock_guard<std::mutex> lk(s->mu);
    if (planned) *planned = s->planned;
    if (failed) *failed = s->failed;
    return TD_OK;
}

extern "C" td_status td_server_destroy(td_server* S)
{
    ErrScope es_;
    if (!S) return fail(TD_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    wake(S);
    S->cv_plan.notify_all();
    for (auto& t : S->planners)
        if (t.joinable()) t.join();
    wake(S);
    if (S->worker.joinable()) S->worker.join();
    DeviceGuard dg(S->ctx->device);
    for (auto& f : S->flights) {
        if (f.stream) (void)hipStreamSynchronize(f.stream);
        if (f.d_ptrs) S->ctx->release(f.d_ptrs, sizeof(void*) * f.cap);
        f.stager.destroy();
        if (f.stream) (void)hipStreamDestroy(f.stream);
    }
    for (auto& kv : S->tickets)
        if (kv.second.inputs) S->ev_pool.push_back(kv.second.inputs);
    for (hipEvent_t e : S->ev_pool) (void)hipEventDestroy(e);
    for (auto& a : S->pool_all) S->ctx->release(a.first, a.second);
    for (auto& kv : S->plans) td_plan_destroy(kv.second);
    delete S;
    return TD_OK;
}

// ===========================================================================
// public: autotuner
// ===========================================================================

namespace {

std::string arch_name(int dev)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    return a.substr(0, a.find(':'));
}

// Minimal reader/writer for the tuning database: one JSON object per line,
// {"arch":"gfx950","dtype":0,"pass":1,"M":512,"C":2,"us":12.3}
void db_load(td_context* ctx, const char* path, const std::string& arch)
{
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // position of the value of "key" (after its colon and any blanks)
        auto value_at = [&](const char* key) -> size_t {
            size_t p = line.find(std::string("\"") + key + "\"");
            if (p == std::string::npos) return std::string::npos;
            p = line.find(':', p + strlen(key) + 2);
            if (p == std::string::npos) return std::string::npos;
            return line.find_first_not_of(" \t", p + 1);
        };
        auto num = [&](const char* key, double* v) {
            const size_t p = value_at(key);
            if (p == std::string::npos) return false;
            *v = atof(line.c_str() + p);
            return true;
        };
        const size_t pa = value_at("arch");
        if (pa == std::string::npos || line.compare(pa, arch.size() + 2, "\"" + arch + "\"") != 0) continue;
        double dt, pass, M, C, G = 1;
        num("G", &G);
        if (num("dtype", &dt) && num("pass", &pass) && num("M", &M) && num("C", &C))
            ctx->tune[std::make_tuple((int)pass, (int)M, (int)dt)] = pack_shape((int)C, (int)G);
    }
}

}  // namespace

extern "C" td_status td_autotune(td_context* ctx, td_dtype dt, int32_t max_M, const char* db_path)
{
    ErrScope es_;
    if (!ctx || max_M < 16) return fail(TD_EINVAL, "bad autotune arguments");
    DeviceGuard dg(ctx->device);
    const std::string arch = arch_name(ctx->device);
    if (db_path) {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        db_load(ctx, db_path, arch);
        bool all = true;
        for (int M = 64; M <= max_M; M *= 2)
            for (int pass = 0; pass < NSHAPE; ++pass)
                all &= ctx->tune.count(std::make_tuple(pass, M, (int)dt)) > 0;
        if (all) return TD_OK;
    }
    std::ofstream db;
    if (db_path) db.open(db_path, std::ios::app);
    hipEvent_t e0, e1;
    TD_HIP(hipEventCreate(&e0));
    TD_HIP(hipEventCreate(&e1));
    td_status result = TD_OK;
    for (int M = 64; M <= max_M && result == TD_OK; M *= 2) {
        // a two-level hierarchy whose lattices have length M exercises all passes
        const int n = M / 2;
        td_patch lv[2] = {{0, n, 0, 0}, {1, n, n / 2, n / 2}};
        td_hierarchy h{-1.0, -1.0, 2.0 / n, 2, 2, lv};
        const size_t es = dt == TD_F64 ? 8 : 4;
        void* bufs[10] = {};
        for (int k = 0; k < 10 && result == TD_OK; ++k) {
            result = ctx->alloc((size_t)n * n * es, &bufs[k]);
            if (result == TD_OK) (void)hipMemset(bufs[k], 0, (size_t)n * n * es);
        }
        for (int pass = 0; pass < NSHAPE && result == TD_OK; ++pass) {
            int bestC = -1;
            double best = 1e30;
            std::vector<int> cands;
            for (int C = 1; C * (M / 8) <= TD_MAX_THREADS; C *= 2)
                for (int Gs = 1; Gs <= (pass == P_ROWFWD ? 1 : 16); Gs *= 2)
                    if (C * Gs * (M / 8) <= TD_MAX_THREADS &&
                        (pass == P_COL ? col_lds_bytes(M, C, elem_size(dt), Gs)
                                       : lds_bytes(M, C, elem_size(dt), Gs)) <= TD_MAX_DYN_LDS)
                        cands.push_back(pack_shape(C, Gs));
            for (int C : cands) {
                {
                    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
                    ctx->tune[std::make_tuple(pass, M, (int)dt)] = C;
                }
                td_plan* p = nullptr;
                if (td_plan_create(ctx, &h, dt, &p) != TD_OK) continue;
                const void* sg[2] = {bufs[0], bufs[1]};
                const void* dx[2] = {bufs[2], bufs[3]};
                const void* dy[2] = {bufs[4], bufs[5]};
                void* fx[2] = {bufs[6], bufs[7]};
                void* fy[2] = {bufs[8], bufs[9]};
                td_request q{p, sg, dx, dy, fx, fy};
                td_status s = TD_OK;
                for (int w = 0; w < 3 && s == TD_OK; ++w) s = td_solve(&q, ctx->stream);
                (void)hipEventRecord(e0, ctx->stream);
                const int reps = 10;
                for (int w = 0; w < reps && s == TD_OK; ++w) s = td_solve(&q, ctx->stream);
                (void)hipEventRecord(e1, ctx->stream);
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                td_plan_destroy(p);
                if (s != TD_OK) continue;
                const double us = 1000.0 * ms / reps;
                if (us < best) {
                    best = us;
                    bestC = C;
                }
            }
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            if (bestC < 0) {
                ctx->tune.erase(std::make_tuple(pass, M, (int)dt));
                continue;
            }
            ctx->tune[std::make_tuple(pass, M, (int)dt)] = bestC;
            if (db.is_open())
                db << "{\"arch\":\"" << arch << "\",\"dtype\":" << (int)dt << ",\"pass\":" << pass
                   << ",\"M\":" << M << ",\"C\":" << shape_C(bestC) << ",\"G\":" << shape_G(bestC)
                   << ",\"us\":" << best << "}\n";
        }
        for (int k = 0; k < 10; ++k)
            if (bufs[k]) ctx->release(bufs[k], (size_t)n * n * es);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return result;
}

// ===========================================================================
// public: diagnostics
// ===========================================================================

extern "C" td_status td_kernel_table(td_context* ctx, int32_t quantity, double aspect, int32_t M,
                                     int32_t kind, int32_t m, int32_t kx, int32_t ky,
                                     double* out_host)
{
    ErrScope es_;
    if (!ctx || !out_host) return fail(TD_EINVAL, "NULL argument");
    if (!std::isfinite(aspect) || aspect < 0 || (aspect != 0 && (aspect < 1.0 / 64 || aspect > 64)))
        return fail(TD_EINVAL, "aspect must be 0 (square cells) or in [1/64, 64]");
    if (quantity != TD_FORCE && quantity != TD_POTENTIAL)
        return fail(TD_EINVAL, "quantity must be TD_FORCE or TD_POTENTIAL");
    if (M < 16 || M > 4096 || (M & (M - 1))) return fail(TD_EINVAL, "M must be a power of two in 16..4096");
    if (kind < 1 || kind > 3) return fail(TD_EINVAL, "kind must be 1, 2 or 3");
    if (kind == 1) m = 1;
    if (m < 1 || kx < 0 || ky < 0 || kx >= m || ky >= m) return fail(TD_EINVAL, "bad m or phase");
    if (kind != 1 && m > 16) return fail(TD_EUNSUPPORTED, "m must be at most 16");
    DeviceGuard dg(ctx->device);
    const size_t bytes = 6 * (size_t)M * M * sizeof(double);
    void* d = nullptr;
    TD_TRY(ctx->alloc(bytes, &d));
    TableJob j;
    memset(&j, 0, sizeof(j));
    j.M = M;
    j.kind = kind;
    j.m = m;
    j.kx = kx;
    j.ky = ky;
    j.family = quantity == TD_POTENTIAL ? 1 : 0;
    j.aspect = aspect > 0 ? aspect : 1.0;
    j.out = (double*)d;
    hipError_t e = launch_table(j, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipMemcpy(out_host, d, bytes, hipMemcpyDeviceToHost);
    ctx->release(d, bytes);
    if (e != hipSuccess) return fail(TD_EDEVICE, hipGetErrorString(e));
    return TD_OK;
}

extern "C" td_status td_timing_enable(td_context* ctx, int enable)
{
    ErrScope es_;
    if (!ctx) return fail(TD_EINVAL, "NULL context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->timing = (enable & ((1 << NTIMED) - 1)) != 0;
    ctx->timing_mask = enable & ((1 << NTIMED) - 1);
    return TD_OK;
}

extern "C" td_status td_timing_read(td_context* ctx, double* ms, int64_t* launches)
{
    ErrScope es_;
    if (!ctx) return fail(TD_EINVAL, "NULL context");
    DeviceGuard dg(ctx->device);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    for (auto& t : ctx->timed) {
        TD_HIP(hipEventSynchronize(t.b));
        float e = 0;
        TD_HIP(hipEventElapsedTime(&e, t.a, t.b));
        ctx->t_ms[t.pass] += e;
        ctx->t_n[t.pass] += 1;
        ctx->ev_pool.push_back(t.a);
        ctx->ev_pool.push_back(t.b);
    }
    ctx->timed.clear();
    for (int p = 0; p < NTIMED; ++p) {
        if (ms) ms[p] = ctx->t_ms[p];
        if (launches) launches[p] = ctx->t_n[p];
        ctx->t_ms[p] = 0;
        ctx->t_n[p] = 0;
    }
    return TD_OK;
}

extern "C" td_status td_plan_traffic(const td_plan* P, int32_t slopes, double* bytes)
{
    ErrScope es_;
    if (!P || !bytes) return fail(TD_EINVAL, "NULL argument");
    if (slopes != TD_SLOPES_GIVEN && slopes != TD_SLOPES_ESTIMATE)
        return fail(TD_EINVAL, "slopes must be TD_SLOPES_GIVEN or TD_SLOPES_ESTIMATE");
    const double cs = (double)elem_size(P->dt), rs = cs / 2;
    for (int p = 0; p < NTIMED; ++p) bytes[p] = 0;
    for (auto& g : P->groups) {
        const int M = g.M, H = M / 2 + 1;
        for (auto& j : g.rowfwd) {
            // source values in range (rows x columns), spectrum rows written
            const LevelG& S = P->lv[j.lvl];
            int cols = 0;
            for (int lc = 0; lc < M; ++lc) {
                const int c = j.m * lc + j.col_off;
                cols += (c >= 0 && c < S.nx) ? 1 : 0;
            }
            int rows = 0;
            for (int r = j.row0; r < j.row0 + j.nrow; ++r) {
                const int sr = j.m * (j.lr_first + r) + j.row_off;
                rows += (sr >= 0 && sr < S.ny) ? 1 : 0;
            }
            // estimated slopes re-read sigma's values (counted with sigma)
            const bool reads = j.f == 0 || slopes == TD_SLOPES_GIVEN;
            bytes[P_ROWFWD] += (reads ? (double)rows * cols * rs : 0.0) + (double)H * j.nrow * cs;
        }
        // col: every input plane (its rows below lattice row M/2), every
        // stored kernel plane it multiplies (real quarter planes for
        // same-level kernels) and every output plane, once per solve
        std::set<int64_t> ins;
        std::set<std::pair<const void*, int>> kerns;
        for (auto& I : g.colins) {
            if (ins.insert(I.in).second)
                bytes[P_COL] += (double)H * std::max(0, std::min(I.ld, M / 2 - I.lr_first)) * cs;
            for (int comp = 0; comp < 2; ++comp)
                if (kerns.insert({I.kern, kKernOfHost[comp][I.f]}).second)
                    bytes[P_COL] += (I.flip & 4) ? (double)H * H * rs : (double)H * M * cs;
        }
        for (auto& O : g.colouts) {
            bytes[P_COL] += (double)H * O.out_ld * cs;
            if (O.kern)
                for (int f = 0; f < 3; ++f)
                    if (kerns.insert({O.kern, kKernOfHost[O.comp][f]}).second)
                        bytes[P_COL] += (double)H * M * cs;
        }
        for (int a = 0; a < 2; ++a)
            for (auto& j : g.rinv[a]) {
                for (int k = 0; k < j.nc; ++k) {
                    const RowInvContrib& c = g.contribs[j.c0 + k];
                    bytes[P_ROWINV + a] += (double)c.m * j.ny * H * 2 * cs;
                }
                bytes[P_ROWINV + a] += (double)j.ny * j.nx * 2 * rs * (a ? 2 : 1);
            }
    }
    return TD_OK;
}

extern "C" const char* td_status_string(td_status s)
{
    switch (s) {
        case TD_OK: return "TD_OK";
        case TD_EINVAL: return "TD_EINVAL";
        case TD_EALIGN: return "TD_EALIGN";
        case TD_ENEST: return "TD_ENEST";
        case TD_ENOMEM: return "TD_ENOMEM";
        case TD_EDEVICE: return "TD_EDEVICE";
        case TD_EBUSY: return "TD_EBUSY";
        case TD_EUNSUPPORTED: return "TD_EUNSUPPORTED";
    }
    return "TD_UNKNOWN";
}

extern "C" const char* td_last_error(void) { return g_err.c_str(); }

extern "C" const char* td_version(void) { return "thindisk-mi355x 0.1 (gfx950)"; }
