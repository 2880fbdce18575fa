// C ABI and host orchestration of the H-matrix build and matvec.
// Every step of the path runs in the device kernels of k_*.hip; this file
// sizes buffers, launches, and reads back the few counters that size the
// next step (one per block-tree level, as in Algorithm 4, and one per pool).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "hmx_internal.h"

using namespace hmx;

namespace {

thread_local std::string g_err;

void set_err(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

struct Fail {
    hmx_status s;
};

// Process-wide cache of device blocks.  Builds allocate and release the same
// large pools again and again (capacity scratch, factor and near-field
// pools); returning them to the driver and mapping them anew each time costs
// seconds on a busy device, so released blocks are kept per device and
// reused best-fit (a block is reused for requests of 3/4 of its size or
// more).  A failed device allocation flushes the cache and retries once.
// Blocks enter the cache only after the work using them has completed (the
// build synchronises its stream before releasing scratch, destroy
// synchronises the device).
struct DeviceCache {
    std::mutex mu;
    std::multimap<size_t, std::pair<int, void*>> blocks;  // size -> (device, ptr)
    size_t cached = 0;
    // every block this library obtained with hipMalloc and has not freed:
    // only these may enter the cache and be freed by it
    std::unordered_set<void*> owned;
};
DeviceCache& cache() {
    static DeviceCache* c = new DeviceCache();  // never destroyed: process lifetime
    return *c;
}

// bytes the library obtained from the driver (cache misses) and cache
// flushes, over the process: a handle's stats report their growth during
// its build
std::atomic<int64_t> g_fresh_bytes{0}, g_flushes{0};

size_t cache_round(size_t bytes) {
    const size_t g = bytes >= ((size_t)64 << 20) ? ((size_t)2 << 20) : 256;
    return (bytes + g - 1) / g * g;
}

// *bytes: requested size in, size of the block handed out on return
hipError_t cache_alloc(void** p, size_t* bytes) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    DeviceCache& c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        for (auto it = c.blocks.lower_bound(*bytes); it != c.blocks.end(); ++it) {
            if (it->first / 4 * 3 > *bytes) break;
            if (it->second.first != dev) continue;
            *p = it->second.second;
            *bytes = it->first;
            c.cached -= it->first;
            c.blocks.erase(it);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, *bytes);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(c.mu);
        (void)hipDeviceSynchronize();
        for (auto& b : c.blocks) {
            c.owned.erase(b.second.second);
            (void)hipFree(b.second.second);
        }
        c.blocks.clear();
        c.cached = 0;
        g_flushes.fetch_add(1);
        e = hipMalloc(p, *bytes);
    }
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(c.mu);
        c.owned.insert(*p);
        g_fresh_bytes.fetch_add((int64_t)*bytes);
    }
    return e;
}

// a block back into the cache; a pointer the library did not allocate is
// never cached (so the cache never frees memory another allocator owns)
void cache_free(void* p, size_t bytes) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    DeviceCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.owned.count(p) == 0) return;
    c.blocks.insert({bytes, {dev, p}});
    c.cached += bytes;
}

// A caller's device allocator (hmx_params.dev_alloc / dev_free / alloc_ctx).
// While one is in scope on this thread (AllocScope: the build, and the
// handle's own later allocations) every device buffer comes from it instead
// of the library's cache.
struct Allocator {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free)(void*, size_t, void*) = nullptr;
    void* ctx = nullptr;
};
thread_local const Allocator* g_user_alloc = nullptr;

struct AllocScope {
    const Allocator* saved;
    explicit AllocScope(const Allocator* a) : saved(g_user_alloc) {
        g_user_alloc = (a && a->alloc) ? a : nullptr;
    }
    ~AllocScope() { g_user_alloc = saved; }
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;
};

// owning device buffer (from the cache, or from the caller's allocator that
// was in scope when it was allocated; it goes back to where it came from)
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    Allocator from{};
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (from.alloc)
                from.free(p, bytes, from.ctx);
            else
                cache_free(p, bytes);
        }
        p = nullptr;
        bytes = 0;
        from = Allocator{};
    }
    // exchange contents with another buffer: pointer, size and owner travel
    // together, so each block still returns to the allocator it came from
    void swap(DevBuf& o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(from, o.from);
    }
    template <typename T>
    T* as() const {
        return (T*)p;
    }
};

// a second stream (default priority, non-blocking) owned for one build
struct AuxStream {
    hipStream_t s = nullptr;
    AuxStream() {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            s = nullptr;  // the classes then run one after the other
        }
    }
    ~AuxStream() {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
    AuxStream(const AuxStream&) = delete;
    AuxStream& operator=(const AuxStream&) = delete;
};

void check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        set_err("%s: %s", what, hipGetErrorString(e));
        // unwinding returns buffers to the cache: wait for in-flight work first
        (void)hipDeviceSynchronize();
        throw Fail{e == hipErrorOutOfMemory ? HMX_ERR_OOM : HMX_ERR_DEVICE};
    }
}

void alloc(DevBuf& b, size_t bytes, const char* what) {
    b.release();
    if (bytes == 0) bytes = 16;
    if (g_user_alloc) {
        bytes = (bytes + 255) / 256 * 256;
        void* q = g_user_alloc->alloc(bytes, g_user_alloc->ctx);
        if (!q) {
            (void)hipDeviceSynchronize();  // in-flight work may still use released blocks
            set_err("device allocation of %zu bytes for %s failed: the caller's allocator "
                    "returned NULL", bytes, what);
            throw Fail{HMX_ERR_OOM};
        }
        b.p = q;
        b.bytes = bytes;
        b.from = *g_user_alloc;
        return;
    }
    bytes = cache_round(bytes);
    hipError_t e = cache_alloc(&b.p, &bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();  // in-flight work may still use released blocks
        b.p = nullptr;
        set_err("device allocation of %zu bytes for %s failed: %s", bytes, what,
                hipGetErrorString(e));
        throw Fail{HMX_ERR_OOM};
    }
    b.bytes = bytes;
}

template <typename T>
T read_scalar(const T* dev, hipStream_t st) {
    T v;
    check(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, st), "readback");
    check(hipStreamSynchronize(st), "stream synchronize");
    return v;
}

// device -> pageable host copy through a pinned staging buffer (large
// readbacks never ask the runtime to pin caller memory).  The staging buffer
// is allocated once and kept for the process: freeing pinned memory waits for
// the whole device, which would serialise the build's concurrent streams.
std::mutex g_stage_mu;
void* g_stage = nullptr;
constexpr size_t kStageBytes = (size_t)32 << 20;

// pinned words the multi-workgroup ACA polls into, one per build in flight
// (the set only grows; each word is reused once its build has finished)
std::mutex g_poll_mu;
std::vector<int*> g_poll_free;

struct PollWord {
    int* p = nullptr;
    PollWord() {
        std::lock_guard<std::mutex> lk(g_poll_mu);
        if (!g_poll_free.empty()) {
            p = g_poll_free.back();
            g_poll_free.pop_back();
            return;
        }
        void* q = nullptr;
        hipError_t e = hipHostMalloc(&q, 64, hipHostMallocDefault);
        if (e != hipSuccess) {
            set_err("pinned poll word allocation failed: %s", hipGetErrorString(e));
            throw Fail{HMX_ERR_OOM};
        }
        p = (int*)q;
    }
    PollWord(const PollWord&) = delete;
    PollWord& operator=(const PollWord&) = delete;
    ~PollWord() {
        std::lock_guard<std::mutex> lk(g_poll_mu);
        g_poll_free.push_back(p);
    }
};

void d2h(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (!g_stage) {
        hipError_t e = hipHostMalloc(&g_stage, kStageBytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            g_stage = nullptr;
            set_err("pinned staging allocation failed: %s", hipGetErrorString(e));
            throw Fail{HMX_ERR_OOM};
        }
    }
    hipError_t r = hipSuccess;
    for (size_t off = 0; off < bytes && r == hipSuccess; off += kStageBytes) {
        const size_t nb = std::min(kStageBytes, bytes - off);
        r = hipMemcpyAsync(g_stage, (const char*)src + off, nb, hipMemcpyDeviceToHost, st);
        if (r == hipSuccess) r = hipStreamSynchronize(st);
        if (r == hipSuccess) memcpy((char*)dst + off, g_stage, nb);
    }
    if (r != hipSuccess) {
        set_err("device to host copy: %s", hipGetErrorString(r));
        throw Fail{HMX_ERR_DEVICE};
    }
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// rank predictor: FP32 parameters, standardisation and Adam state on the
// device, plus work buffers grown on demand
struct hmx_mlp_s {
    DevBuf w, m, v, mean, scale;
    int64_t t = 0;  // Adam steps taken
    DevBuf act, scratch, grad, Xb, yb, loss;
};

// a captured sequence of matvecs (hmx_matvec_graph)
struct hmx_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// The far field without precomputation: the ACA list in chunk order (each
// chunk's column scratch within the budget), per entry its leaf, capacity
// offsets and the ranks of the last matvec, and the apply pieces sorted by
// (chunk, row tile) with their segments
struct NpPlan {
    int64_t nl = 0, npcs = 0, nseg = 0;
    int64_t max_u = 0, max_v = 0, max_nb = 0;
    int big_words = 0, med_words = 0, tiny_words = 0;  // the ACA classes' bitmask words
    DevBuf blocks, lmap, cu, cv, rank, steps, spcs, seg_start, seg_tile;
    std::vector<int64_t> bounds, hcu, hcv, cseg, cls;  // cls: nsplit, nbig, nmed per chunk
};

struct hmx_hmatrix_s {
    int64_t n = 0;
    int d = 0;
    hmx_kernel kern{};
    hmx_params prm{};
    int f64 = 0;
    size_t esz = 4;  // bytes per compute-type value (vectors, ACA scratch)
    int smode = 1;   // factor (U, V) storage mode: 0 F64, 1 F32, 2 BF16
    size_t ssz = 4;  // bytes per stored factor entry
    int nmode = 1;   // near-field storage mode
    size_t nsz = 4;  // bytes per stored near-field entry
    double box[6] = {0, 0, 0, 0, 0, 0};
    int L = 0;
    int64_t nslots = 0;
    int64_t n_adm = 0, n_dense = 0, ntiles = 0, npieces = 0, sum_rank = 0;
    int max_tile = 0;
    int64_t big_adm = 0;  // rows of the largest admissible leaf's clusters
    // batched build: problem p owns indices [offsets[p], offsets[p + 1])
    int32_t nprob = 1;
    bool batched = false;
    int rt_config = -1;  // row-tile kernel configuration (-1: default shape)
    int p1_lanes = 0;    // phase-1 lanes per column group (0: chosen by tile height)
    std::vector<int64_t> offsets;
    int64_t factor_entries = 0, near_entries = 0;
    DevBuf codes, perm, soa64, soa32, node_lo, node_hi, bmin, bmax;
    DevBuf adm, adm_level, adm_ids, dense, dense_level;
    DevBuf tile_of_point, tile_lo;
    DevBuf rank, steps, toff;
    DevBuf pieces, upool, npool, widx, tile_meta, vecpool;
    int64_t upool_entries = 0, npool_entries = 0, ncols_total = 0;
    // phase 1 (t = V^T x) by row tiles: the V pool (pieces of V_b rows per
    // row tile of sigma_b; with the symmetric far field only for leaves that
    // are their own mirror), partial sums per source column, and per t entry
    // the first of its source pieces in pfc
    int sym = 0;       // symmetric far field: the mirror of a leaf reuses its factors
    int Ru = 0, Rv = 0;  // row units of the factor pool and of the V pool
    int64_t ncols_u = 0, ncols_v = 0, nvpieces = 0, vtpool_entries = 0;
    DevBuf partner, vpieces, vtpool, vt_meta, p1rec, pfc, partial;
    int far_np = 0;  // factors recomputed by every matvec
    NpPlan np;
    // the process-wide allocation counters when the handle was created
    int64_t fresh0 = g_fresh_bytes.load(), flush0 = g_flushes.load();
    // rectangular A(Y1 x Y2): the union holds Y1 (rows, [0, nrows)) then Y2
    // (columns, [col0, col0 + ncols)); the row tiles are Y1's leaf clusters,
    // the first ntiles_rows tiles.  Square handles: rows = columns = [0, n).
    bool rect = false;
    int64_t nrows = 0, ncols = 0, col0 = 0, ntiles_rows = 0;
    // work vectors of hmx_matmat (16 right-hand sides, point-major), grown on use
    DevBuf mm_vec, mm_partial;
    int kd = 0;  // the points' dimension for the kernel's normalisation
    hmx_stats stats{};
    // matvec phase tracing (hmx_profile_begin / end)
    std::vector<hipEvent_t> prof_events;
    int32_t prof_max = 0, prof_calls = 0;

    void prof_release() {
        for (auto e : prof_events) (void)hipEventDestroy(e);
        prof_events.clear();
        prof_max = prof_calls = 0;
    }
    ~hmx_hmatrix_s() { prof_release(); }

    int64_t device_bytes() const {
        const DevBuf* all[] = {&codes,   &perm,    &soa64,     &soa32,         &node_lo,
                               &node_hi, &bmin,    &bmax,      &adm,           &adm_level,
                               &adm_ids, &dense,   &dense_level, &tile_of_point, &tile_lo,
                               &rank,    &steps,   &toff,      &pieces,        &upool,
                               &npool,   &widx,    &tile_meta, &vecpool,       &partner,
                               &vpieces, &vtpool,  &vt_meta,   &p1rec,         &pfc,
                               &partial, &np.blocks, &np.lmap, &np.cu,  &np.cv,
                               &np.rank, &np.steps, &np.spcs,  &np.seg_start, &np.seg_tile,
                               &mm_vec,  &mm_partial};
        int64_t s = 0;
        for (auto* b : all) s += (int64_t)b->bytes;
        return s;
    }
};

namespace {

// counts, sizes and the matvec's algorithmic bytes into the handle's stats
void finish_stats(hmx_hmatrix_s* h, std::chrono::steady_clock::time_point t_all) {
    hmx_stats& S = h->stats;
    const size_t esz = h->esz, ssz = h->ssz;
    const int64_t n = h->n;
    S.n = n;
    S.d = h->d;
    S.n_adm = h->n_adm;
    S.n_dense = h->n_dense;
    S.n_tiles = h->ntiles;
    if (!h->prm.aca_only) S.sum_rank = h->sum_rank;
    S.factor_entries = h->factor_entries;
    S.near_entries = h->near_entries;
    S.entry_bytes = (int32_t)ssz;
    S.near_entry_bytes = (int32_t)h->nsz;
    S.tile_config = h->rt_config;
    S.rows = h->nrows;
    S.cols = h->ncols;
    S.alloc_fresh_bytes = g_fresh_bytes.load() - h->fresh0;
    S.alloc_flushes = g_flushes.load() - h->flush0;
    S.phase_ms[7] = ms_since(t_all);
    // algorithmic bytes of one matvec with beta = 0: the near field once,
    // U_b and V_b of every admissible leaf once (with the symmetric far
    // field each stored factor serves twice: as a leaf's U in phase 2 and as
    // its mirror's V in phase 1), the vectors x and z once, perm for gather
    // and scatter, t written and read
    S.matvec_bytes = h->prm.aca_only
                         ? 0.0
                         : (double)h->near_entries * h->nsz +
                               (double)(S.u_entries + S.v_entries) * ssz +
                               (double)n * (2.0 * esz + 8.0) + (double)S.sum_rank * 2.0 * esz;
    S.device_bytes = h->device_bytes();
}

// length scale l of the predictor's features
double kernel_length(const hmx_kernel& k) {
    if (k.kind == HMX_GAUSSIAN) return std::sqrt(k.p0);
    if (k.kind == HMX_MATERN32 || k.kind == HMX_MATERN_NU1) return k.p0;
    return 1.0;
}

// the kernel function as the device kernels take it; the Matern nu = 1
// kernel's normalisation 1 / (2^(beta-1) Gamma(beta)), beta = 1 + d/2
KernelFn kernel_fn(const hmx_kernel& k, int d) {
    KernelFn f{(int)k.kind, k.p0};
    if (k.kind == HMX_MATERN_NU1) {
        const double beta = 1.0 + 0.5 * d;
        f.norm = 1.0 / (std::pow(2.0, beta - 1.0) * std::tgamma(beta));
    }
    return f;
}

// grow a device buffer to at least `bytes`, keeping the first `keep` bytes
void grow(DevBuf& b, size_t bytes, size_t keep, hipStream_t st, const char* what,
          bool exact = false) {
    if (b.p && b.bytes >= bytes) return;
    size_t nb = exact ? bytes : std::max(bytes, b.bytes * 2);
    DevBuf nbuf;
    alloc(nbuf, nb, what);
    if (keep) check(hipMemcpyAsync(nbuf.p, b.p, keep, hipMemcpyDeviceToDevice, st), "grow copy");
    check(hipStreamSynchronize(st), "grow sync");
    b.swap(nbuf);
}

int max_depth(int64_t n, int leaf) {
    int L = 0;
    int64_t s = n;  // largest cluster at depth L is ceil(n / 2^L)
    while (s > leaf) {
        s = (s + 1) / 2;
        ++L;
    }
    return L;
}


// dimensions, kernel, parameters and the storage modes they imply
void init_handle(hmx_hmatrix_s* h, int64_t n, int d, const hmx_kernel& k, const hmx_params& p) {
    h->n = n;
    h->d = d;
    h->kern = k;
    h->prm = p;
    h->f64 = p.compute_dtype == HMX_F64;
    h->esz = h->f64 ? 8 : 4;
    h->smode = p.storage_dtype == HMX_F64 ? 0 : (p.storage_dtype == HMX_F32 ? 1 : 2);
    h->ssz = h->smode == 0 ? 8 : (h->smode == 1 ? 4 : 2);
    h->nmode = p.near_dtype == HMX_F64 ? 0 : (p.near_dtype == HMX_F32 ? 1 : 2);
    h->nsz = h->nmode == 0 ? 8 : (h->nmode == 1 ? 4 : 2);
    if (p.near_recompute) {  // nothing stored: entries evaluated in every product
        h->nmode = 3;
        h->nsz = 0;
    }
    h->sym = p.symmetric_far;
    h->far_np = p.far_recompute;
    h->nrows = h->ncols = n;
    h->kd = d;
}

// validation shared by the single and the batched build
hmx_status check_params(const hmx_params& p) {
    if (p.leaf_size < 1 || !(p.eta >= 0) || !std::isfinite(p.eta) || !(p.aca_eps >= 0) ||
        !(p.aca_eta >= 0 && p.aca_eta < 1) || p.max_rank < 1 || p.max_rank > kMaxRankCap ||
        !(p.sigma2 >= 0) || !std::isfinite(p.sigma2)) {
        set_err("invalid params (leaf %d, eta %g, eps %g, aca_eta %g, max_rank %d, sigma2 %g)",
                p.leaf_size, p.eta, p.aca_eps, p.aca_eta, p.max_rank, p.sigma2);
        return HMX_ERR_INVALID_ARG;
    }
    if (p.compute_dtype != HMX_F64 && p.compute_dtype != HMX_F32) {
        set_err("compute_dtype must be F64 or F32");
        return HMX_ERR_UNSUPPORTED;
    }
    if ((p.compute_dtype == HMX_F64) != (p.storage_dtype == HMX_F64) ||
        (p.storage_dtype != HMX_F64 && p.storage_dtype != HMX_F32 && p.storage_dtype != HMX_BF16)) {
        set_err("storage_dtype must be F64 with F64 compute, F32 or BF16 with F32 compute");
        return HMX_ERR_UNSUPPORTED;
    }
    if (p.near_recompute != 0 && p.near_recompute != 1) {
        set_err("near_recompute must be 0 or 1");
        return HMX_ERR_INVALID_ARG;
    }
    if ((p.dev_alloc == nullptr) != (p.dev_free == nullptr)) {
        set_err("dev_alloc and dev_free must both be set, or neither");
        return HMX_ERR_INVALID_ARG;
    }
    if (p.aca_split_rows < 0) {
        set_err("aca_split_rows must be >= 0 (0: default)");
        return HMX_ERR_INVALID_ARG;
    }
    if (!p.near_recompute) {
        const bool ok = (p.near_dtype == p.storage_dtype) ||
                        (p.storage_dtype == HMX_BF16 && p.near_dtype == HMX_F32);
        if (!ok) {
            set_err("near_dtype must equal storage_dtype, or be F32 with BF16 factors");
            return HMX_ERR_UNSUPPORTED;
        }
    }
    if (p.rank_mode != HMX_RANK_ADAPTIVE && p.rank_mode != HMX_RANK_FIXED &&
        p.rank_mode != HMX_RANK_LEARNED) {
        set_err("unsupported rank mode %d", (int)p.rank_mode);
        return HMX_ERR_UNSUPPORTED;
    }
    if (p.rank_mode == HMX_RANK_LEARNED && !p.mlp) {
        set_err("HMX_RANK_LEARNED needs a rank predictor (params.mlp)");
        return HMX_ERR_INVALID_ARG;
    }
    if (p.aca_only != 0 && p.aca_only != 1) {
        set_err("aca_only must be 0 or 1");
        return HMX_ERR_INVALID_ARG;
    }
    if (p.learned_one_shot != 0 && p.learned_one_shot != 1) {
        set_err("learned_one_shot must be 0 or 1");
        return HMX_ERR_INVALID_ARG;
    }
    if (p.symmetric_far != 0 && p.symmetric_far != 1) {
        set_err("symmetric_far must be 0 or 1");
        return HMX_ERR_INVALID_ARG;
    }
    if (p.far_recompute != 0 && p.far_recompute != 1) {
        set_err("far_recompute must be 0 or 1");
        return HMX_ERR_INVALID_ARG;
    }
    if (p.far_recompute && p.aca_only) {
        set_err("far_recompute and aca_only exclude each other (the build runs no ACA)");
        return HMX_ERR_INVALID_ARG;
    }
    if (p.far_recompute && p.rank_mode == HMX_RANK_LEARNED) {
        set_err("far_recompute supports the adaptive and fixed rank modes");
        return HMX_ERR_UNSUPPORTED;
    }
    return HMX_OK;
}


// phases 1-3: ordering, cluster tree and boxes, block-tree traversal
void stage_partition(hmx_hmatrix_s* h, const void* pts, int pts_f64, hipStream_t st) {
    using clk = std::chrono::steady_clock;
    const int64_t n = h->n;
    const int d = h->d;
    const int leaf = h->prm.leaf_size;
    const double eta = h->prm.eta;
    const int f64 = h->f64;
    hmx_stats& S = h->stats;
    auto t0 = clk::now();

    // ---- 1. global box, Morton codes, stable sort, ordered coordinates ----
    {
        const int nparts = global_box_parts(n);
        DevBuf partial, boxd;
        alloc(partial, (size_t)nparts * 6 * sizeof(double), "box partials");
        alloc(boxd, 6 * sizeof(double), "box");
        check(launch_global_box(pts, pts_f64, n, d, partial.as<double>(), nparts,
                                boxd.as<double>(), st),
              "global box");
        double hb[6];
        check(hipMemcpyAsync(hb, boxd.p, 2 * d * sizeof(double), hipMemcpyDeviceToHost, st),
              "box readback");
        check(hipStreamSynchronize(st), "box sync");
        for (int k = 0; k < 2 * d; ++k)
            if (!std::isfinite(hb[k])) {
                set_err("points contain NaN or infinite coordinates");
                throw Fail{HMX_ERR_INVALID_ARG};
            }
        for (int k = 0; k < 2 * d; ++k) h->box[k] = hb[k];

        alloc(h->codes, n * 8, "morton codes");
        alloc(h->perm, n * 4, "permutation");
        check(launch_morton(pts, pts_f64, n, d, boxd.as<double>(), h->codes.as<uint64_t>(),
                            h->perm.as<uint32_t>(), st),
              "morton");
        DevBuf scratch;
        alloc(scratch, radix_sort_scratch_bytes(n), "sort scratch");
        const int bits = d == 3 ? 63 : 64;
        check(radix_sort_pairs(h->codes.as<uint64_t>(), h->perm.as<uint32_t>(), n, bits,
                               scratch.p, st),
              "radix sort");
        alloc(h->soa64, (size_t)n * d * 8, "coords f64");
        if (!f64) alloc(h->soa32, (size_t)n * d * 4, "coords f32");
        check(launch_gather_coords(pts, pts_f64, n, d, h->perm.as<uint32_t>(),
                                   h->soa64.as<double>(), f64 ? nullptr : h->soa32.as<float>(), st),
              "gather coords");
        check(hipStreamSynchronize(st), "order sync");
    }
    S.phase_ms[0] = ms_since(t0);
    t0 = clk::now();

    // ---- 2. cluster tree, boxes, leaf tiles ----
    h->L = max_depth(n, leaf);
    if (h->L > 29) {
        set_err("cluster tree too deep (%d levels); raise leaf_size", h->L);
        throw Fail{HMX_ERR_UNSUPPORTED};
    }
    h->nslots = (2ll << h->L) - 1;
    alloc(h->node_lo, h->nslots * 4, "node lo");
    alloc(h->node_hi, h->nslots * 4, "node hi");
    for (int l = 0; l <= h->L; ++l)
        check(launch_tree_level(l, n, leaf, h->node_lo.as<int32_t>(), h->node_hi.as<int32_t>(), st),
              "tree level");
    alloc(h->bmin, (size_t)h->nslots * d * 8, "box min");
    alloc(h->bmax, (size_t)h->nslots * d * 8, "box max");
    for (int l = h->L; l >= 0; --l)
        check(launch_box_level(l, d, leaf, h->node_lo.as<int32_t>(), h->node_hi.as<int32_t>(),
                               h->soa64.as<double>(), n, h->bmin.as<double>(),
                               h->bmax.as<double>(), st),
              "box level");
    {
        alloc(h->tile_of_point, n * 4, "tile of point");
        check(hipMemsetAsync(h->tile_of_point.p, 0, n * 4, st), "memset");
        check(launch_mark_leaves(h->L, leaf, h->node_lo.as<int32_t>(), h->node_hi.as<int32_t>(),
                                 h->nslots, h->tile_of_point.as<int32_t>(), st),
              "mark leaves");
        DevBuf scratch, cnt;
        alloc(scratch, tile_scan_scratch_bytes(n), "tile scan");
        alloc(cnt, 8, "tile count");
        // upper bound on tiles for tile_lo: number of slots
        alloc(h->tile_lo, (size_t)(std::min<int64_t>(h->nslots, n) + 1) * 4, "tile lo");
        check(launch_iota_scan_tiles(h->tile_of_point.as<int32_t>(), n, h->tile_lo.as<int32_t>(),
                                     cnt.as<int64_t>(), scratch.p, st),
              "tile scan");
        h->ntiles = read_scalar(cnt.as<int64_t>(), st);
        h->ntiles_rows = h->ntiles;
    }
    {
        // largest leaf cluster = largest tile
        int64_t s = n;
        while (s > leaf) s = (s + 1) / 2;
        h->max_tile = (int)s;
    }
    S.phase_ms[1] = ms_since(t0);
    t0 = clk::now();

    // ---- 3. block cluster tree traversal (Algorithm 4 applied to Algorithm 1) ----
    int64_t big_adm = n;
    {
        DevBuf cur, nxt, scratch, totals;
        alloc(cur, 8, "level 0");
        const int2 root = make_int2(0, 0);
        check(hipMemcpyAsync(cur.p, &root, sizeof root, hipMemcpyHostToDevice, st), "root");
        alloc(totals, 8 * sizeof(int64_t), "totals");
        int64_t ncur = 1;
        int level = 0;
        int64_t cap_adm = 0, cap_dense = 0;
        int min_adm_level = -1;
        while (ncur > 0) {
            if (level >= 64) {
                set_err("block tree deeper than 64 levels");
                throw Fail{HMX_ERR_UNSUPPORTED};
            }
            S.level_sizes[level] = ncur;
            const int64_t nblk = traverse_blocks(ncur);
            if (!scratch.p || scratch.bytes < traverse_scratch_bytes(ncur))
                alloc(scratch, traverse_scratch_bytes(ncur), "traverse scratch");
            int64_t* bc = scratch.as<int64_t>();
            check(launch_traverse_count(cur.as<int2>(), ncur, h->node_lo.as<int32_t>(),
                                        h->node_hi.as<int32_t>(), h->bmin.as<double>(),
                                        h->bmax.as<double>(), d, leaf, eta, bc, st),
                  "traverse count");
            check(launch_traverse_scan(bc, nblk, totals.as<int64_t>(), st), "traverse scan");
            int64_t tot[3];
            check(hipMemcpyAsync(tot, totals.p, 3 * 8, hipMemcpyDeviceToHost, st), "totals");
            check(hipStreamSynchronize(st), "level sync");
            if (tot[0] > 0 && min_adm_level < 0) min_adm_level = level;
            if (h->n_adm + tot[0] > cap_adm) {
                int64_t nc = std::max<int64_t>(2 * cap_adm, h->n_adm + tot[0]);
                grow(h->adm, nc * sizeof(int4), h->n_adm * sizeof(int4), st, "adm leaves");
                grow(h->adm_level, nc * 4, h->n_adm * 4, st, "adm levels");
                grow(h->adm_ids, nc * sizeof(int2), h->n_adm * sizeof(int2), st, "adm node ids");
                cap_adm = nc;
            }
            if (h->n_dense + tot[2] > cap_dense) {
                int64_t nc = std::max<int64_t>(2 * cap_dense, h->n_dense + tot[2]);
                grow(h->dense, nc * sizeof(int4), h->n_dense * sizeof(int4), st, "dense leaves");
                grow(h->dense_level, nc * 4, h->n_dense * 4, st, "dense levels");
                cap_dense = nc;
            }
            const int64_t nnext = 4 * tot[1];
            alloc(nxt, nnext * sizeof(int2), "next level");
            check(launch_traverse_write(cur.as<int2>(), ncur, h->node_lo.as<int32_t>(),
                                        h->node_hi.as<int32_t>(), h->bmin.as<double>(),
                                        h->bmax.as<double>(), d, leaf, eta, bc, level,
                                        nxt.as<int2>(), h->adm.as<int4>(),
                                        h->adm_level.as<int32_t>(), h->adm_ids.as<int2>(),
                                        h->n_adm, h->dense.as<int4>(),
                                        h->dense_level.as<int32_t>(), h->n_dense, nullptr, st),
                  "traverse write");
            h->n_adm += tot[0];
            h->n_dense += tot[2];
            cur.swap(nxt);
            ncur = nnext;
            ++level;
        }
        check(hipStreamSynchronize(st), "traverse sync");
        S.levels = level;
        // largest admissible block side: clusters at the first admissible level
        for (int l = 0; l < std::max(min_adm_level, 0); ++l) big_adm = (big_adm + 1) / 2;
    }
    S.phase_ms[2] = ms_since(t0);
    h->big_adm = big_adm;
}

// how the ACA treats the admissible leaves of a handle: size classes and
// (learned sizing) the predicted targets
struct AcaPlan {
    const int32_t* cls = nullptr;  // per leaf, non-decreasing; < split0: many workgroups,
    int split0 = 0;                // < split: 512-thread class, < split2: 256-thread
    int split = 0, split2 = 0;     // class, else single wave
    int big_words = 2, med_words = 2, tiny_words = 2;  // LDS mask words per class
    const int32_t* rt = nullptr;         // learned targets, or null
};

// clusters of split_rows(h) or more points put their blocks on many
// workgroups each, of kBigRows or more in the 512-thread class; clusters of
// at most kTinyRows points in the single-wave class.  With the chunks
// interleaving the levels, a block of up to 2^17 rows runs as well on one
// 512-thread workgroup beside the other classes as on many workgroups; the
// default keeps the many-workgroup path for blocks whose bitmasks would not
// fit a workgroup's LDS
constexpr int64_t kDefaultSplitRows = (int64_t)1 << 18;
// (one-wave class up to 512 points rather than 256: N = 2^22 3-d ACA
// 3.36 -> 3.16 s, N = 2^20 2-d 38 -> 34.5 ms, the same ranks; the 512-thread
// cut at 4096 or 8192 points makes no measurable difference)
constexpr int64_t kBigRows = 4096;
constexpr int64_t kTinyRows = 512;

// size classes of a single problem by tree level: clusters at level l hold at
// most s_l points (s_0 = n, s_{l+1} = ceil(s_l / 2)); levels whose clusters
// can reach kBigRows points form the 512-thread class
int64_t split_rows(const hmx_hmatrix_s* h) {
    return h->prm.aca_split_rows > 0 ? h->prm.aca_split_rows : kDefaultSplitRows;
}

// the first tree levels of the 512-thread, the 256-thread and the
// single-wave class for a problem of n points (clusters at level l hold at
// most ceil(n / 2^l) points); *s0, *s1, *s2: the largest cluster of each
int4 level_cuts(int64_t n, int64_t split_at, int64_t* s0, int64_t* s1, int64_t* s2) {
    int4 c = make_int4(0, 0, 0, 0);
    int64_t a = n;  // the largest cluster below the many-workgroup levels
    while (a >= split_at) {
        a = (a + 1) / 2;
        ++c.x;
    }
    int64_t b = n;
    while (b >= kBigRows) {
        b = (b + 1) / 2;
        ++c.y;
    }
    int64_t e = b;
    c.z = c.y;
    while (e > kTinyRows) {
        e = (e + 1) / 2;
        ++c.z;
    }
    if (s0) *s0 = a;
    if (s1) *s1 = b;
    if (s2) *s2 = e;
    return c;
}

AcaPlan level_plan(const hmx_hmatrix_s* h) {
    AcaPlan p;
    int64_t s0, s_split, s_split2;
    const int4 c = level_cuts(h->n, split_rows(h), &s0, &s_split, &s_split2);
    p.split0 = c.x;
    p.split = c.y;
    p.split2 = c.z;
    const int64_t big = std::min(h->big_adm, s0);  // the largest single-workgroup block
    const int64_t words = 2 * ((big + 31) / 32);
    if (words * 4 > 64 * 1024) {
        set_err("admissible block of %lld rows exceeds the ACA bitmask capacity", (long long)big);
        throw Fail{HMX_ERR_UNSUPPORTED};
    }
    p.cls = h->adm_level.as<int32_t>();
    p.big_words = (int)std::max<int64_t>(words, 2);
    p.med_words = (int)std::max<int64_t>(2 * ((std::min(s_split, big) + 31) / 32), 2);
    p.tiny_words = (int)std::max<int64_t>(2 * ((std::min(s_split2, big) + 31) / 32), 2);
    return p;
}

// learned sizing: the predictor's target for every admissible leaf
void stage_predict(hmx_hmatrix_s* h, DevBuf& rt, hipStream_t st) {
    alloc(rt, std::max<int64_t>(h->n_adm, 1) * 4, "rank targets");
    const auto tp = std::chrono::steady_clock::now();
    const hmx_mlp_s* mp = h->prm.mlp;
    check(launch_rank_predict(h->adm.as<int4>(), h->adm_ids.as<int2>(), h->n_adm,
                              h->bmin.as<double>(), h->bmax.as<double>(), h->d,
                              kernel_length(h->kern), mp->w.as<float>(), mp->mean.as<float>(),
                              mp->scale.as<float>(), h->prm.max_rank, nullptr, rt.as<int32_t>(),
                              st),
          "rank prediction");
    check(hipStreamSynchronize(st), "prediction sync");
    h->stats.predict_ms += ms_since(tp);
}

// the multi-workgroup ACA of a chunk's largest blocks a.blocks[0 .. a.nsplit):
// tile maps and bitmask offsets built on the host from the blocks' sizes
// (prepared before the other classes start, so that no host wait falls
// inside the concurrent part)
struct SplitBuffers {
    DevBuf drt, dct, drtoff, dctoff, dmoff, masks, state, cpart, rpart, urow, udp, vdp, act;
    std::unique_ptr<PollWord> poll;
    SplitPlan P{};
};

void prepare_split(hmx_hmatrix_s* h, const AcaArgs& a, int f64, hipStream_t st,
                   SplitBuffers& B) {
    const int64_t nb = a.nsplit;
    std::vector<int4> hb(nb);
    d2h(hb.data(), a.blocks, (size_t)nb * sizeof(int4), st);
    const int tile = split_tile();
    std::vector<int2> rt, ct;
    std::vector<int64_t> rtoff(nb + 1), ctoff(nb + 1), moff(nb + 1);
    rtoff[0] = ctoff[0] = moff[0] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int m = hb[b].y - hb[b].x, nc = hb[b].w - hb[b].z;
        for (int t = 0; t * (int64_t)tile < m; ++t) rt.push_back(make_int2((int)b, t));
        for (int t = 0; t * (int64_t)tile < nc; ++t) ct.push_back(make_int2((int)b, t));
        rtoff[b + 1] = (int64_t)rt.size();
        ctoff[b + 1] = (int64_t)ct.size();
        moff[b + 1] = moff[b] + (m + 31) / 32 + (nc + 31) / 32;
    }
    alloc(B.drt, rt.size() * sizeof(int2), "split row tiles");
    alloc(B.dct, ct.size() * sizeof(int2), "split column tiles");
    alloc(B.drtoff, (nb + 1) * 8, "split row tile offsets");
    alloc(B.dctoff, (nb + 1) * 8, "split column tile offsets");
    alloc(B.dmoff, (nb + 1) * 8, "split mask offsets");
    alloc(B.masks, (size_t)moff[nb] * 4, "split masks");
    alloc(B.state, (size_t)nb * split_state_bytes(), "split state");
    alloc(B.cpart, rt.size() * split_colpart_bytes(f64), "split column partials");
    alloc(B.rpart, ct.size() * split_rowpart_bytes(f64), "split row partials");
    alloc(B.urow, (size_t)nb * (kMaxRankCap + 1) * h->esz, "split pivot rows");
    alloc(B.udp, rt.size() * (kMaxRankCap + 1) * 8, "split U products");
    alloc(B.vdp, ct.size() * (kMaxRankCap + 1) * 8, "split V products");
    alloc(B.act, 8, "split active count");
    check(hipMemcpyAsync(B.drt.p, rt.data(), rt.size() * sizeof(int2), hipMemcpyHostToDevice, st),
          "split tiles");
    check(hipMemcpyAsync(B.dct.p, ct.data(), ct.size() * sizeof(int2), hipMemcpyHostToDevice, st),
          "split tiles");
    check(hipMemcpyAsync(B.drtoff.p, rtoff.data(), (nb + 1) * 8, hipMemcpyHostToDevice, st),
          "split offsets");
    check(hipMemcpyAsync(B.dctoff.p, ctoff.data(), (nb + 1) * 8, hipMemcpyHostToDevice, st),
          "split offsets");
    check(hipMemcpyAsync(B.dmoff.p, moff.data(), (nb + 1) * 8, hipMemcpyHostToDevice, st),
          "split offsets");
    check(hipStreamSynchronize(st), "split plan");  // the host vectors go out of scope
    SplitPlan& P = B.P;
    P.nblocks = nb;
    P.nrowtiles = (int64_t)rt.size();
    P.ncoltiles = (int64_t)ct.size();
    P.rowtiles = B.drt.as<int2>();
    P.coltiles = B.dct.as<int2>();
    P.rtoff = B.drtoff.as<int64_t>();
    P.ctoff = B.dctoff.as<int64_t>();
    P.moff = B.dmoff.as<int64_t>();
    P.masks = B.masks.as<uint32_t>();
    P.state = B.state.p;
    P.colpart = B.cpart.p;
    P.rowpart = B.rpart.p;
    P.urow = B.urow.p;
    P.udpart = B.udp.as<double>();
    P.vdpart = B.vdp.as<double>();
    P.active_dev = B.act.as<int>();
    B.poll.reset(new PollWord);
    P.active_host = B.poll->p;
}

// The blocks of a level-sorted list regrouped into nsl chunks that each hold
// the same share of every level, level-sorted within the chunk (so the size
// classes of the ACA run side by side in every chunk): entry i of the chunk
// order is list entry perm[i]; bounds: the chunks' first entries and the end.
// cap and rt (optional per-block int32 arrays) are gathered along.
struct ChunkOrder {
    DevBuf perm, blocks, levels, cap, rt;
    std::vector<int64_t> bounds;
};

void interleave(const int4* blocks, const int32_t* levels, int64_t nb, const int32_t* cap,
                const int32_t* rt, int nsl, hipStream_t st, ChunkOrder& o) {
    DevBuf lb;
    alloc(lb, 2 * 64 * 8, "level bounds");
    check(hipMemsetAsync(lb.p, 0, 2 * 64 * 8, st), "level bounds");
    int64_t* lstart = lb.as<int64_t>();
    int64_t* lend = lstart + 64;
    check(launch_level_bounds(levels, nb, lstart, lend, st), "level bounds");
    int64_t hl[128];
    d2h(hl, lb.p, sizeof hl, st);
    // chunk k: the positions p of each level (c blocks) with
    // floor(p nsl / c) == k, i.e. [ceil(k c / nsl), ceil((k + 1) c / nsl))
    std::vector<int64_t>& bounds = o.bounds;
    bounds.assign(nsl + 1, 0);
    for (int l = 0; l < 64; ++l) {
        const int64_t c = hl[64 + l] - hl[l];
        if (c <= 0) continue;
        for (int k = 0; k < nsl; ++k)
            bounds[k + 1] +=
                ((int64_t)(k + 1) * c + nsl - 1) / nsl - ((int64_t)k * c + nsl - 1) / nsl;
    }
    for (int k = 0; k < nsl; ++k) bounds[k + 1] += bounds[k];
    if (bounds[nsl] != nb) {
        set_err("interleaved chunks cover %lld of %lld blocks", (long long)bounds[nsl],
                (long long)nb);
        throw Fail{HMX_ERR_DEVICE};
    }
    DevBuf keys, sscr;
    alloc(keys, (size_t)nb * 8, "interleave keys");
    alloc(o.perm, (size_t)nb * 4, "interleave order");
    check(launch_interleave_keys(levels, nb, lstart, lend, nsl, keys.as<uint64_t>(),
                                 o.perm.as<uint32_t>(), st),
          "interleave keys");
    int bits = 8;
    while ((1ll << (bits - 8)) < nsl) ++bits;
    alloc(sscr, radix_sort_scratch_bytes(nb), "interleave sort");
    check(radix_sort_pairs(keys.as<uint64_t>(), o.perm.as<uint32_t>(), nb, bits, sscr.p, st),
          "interleave sort");
    keys.release();
    sscr.release();
    alloc(o.blocks, (size_t)nb * sizeof(int4), "interleaved blocks");
    alloc(o.levels, (size_t)nb * 4, "interleaved levels");
    if (cap) alloc(o.cap, (size_t)nb * 4, "interleaved capacities");
    if (rt) alloc(o.rt, (size_t)nb * 4, "interleaved targets");
    check(launch_gather_blocks(o.perm.as<uint32_t>(), nb, blocks, levels, cap, rt,
                               o.blocks.as<int4>(), o.levels.as<int32_t>(),
                               cap ? o.cap.as<int32_t>() : nullptr,
                               rt ? o.rt.as<int32_t>() : nullptr, st),
          "interleave gather");
}

// the ACA arguments every chunk shares
AcaArgs aca_args_base(const hmx_hmatrix_s* h, const AcaPlan& plan) {
    AcaArgs a{};
    const int f64 = h->f64;
    a.soa = f64 ? h->soa64.p : h->soa32.p;
    a.soa64 = h->soa64.as<double>();
    a.n = h->n;
    a.d = h->d;
    a.kern = kernel_fn(h->kern, h->kd);
    a.kmax = h->prm.max_rank;
    a.eps = h->prm.aca_eps;
    a.aca_eta = h->prm.aca_eta;
    a.eps0 = h->prm.aca_eps0 >= 0 ? h->prm.aca_eps0 : (f64 ? 1e-14 : 1e-7);
    a.fixed = h->prm.rank_mode == HMX_RANK_FIXED;
    a.big_words = plan.big_words;
    a.med_words = plan.med_words;
    a.tiny_words = plan.tiny_words;
    return a;
}

// ACA scratch budget of one chunk, in compute-type entries: the caller's, else
// 40% of the device memory that is free now (the library's cached blocks
// count as free)
int64_t aca_budget(const hmx_hmatrix_s* h) {
    int64_t budget_bytes = (int64_t)h->prm.aca_chunk_mb << 20;
    if (h->prm.aca_chunk_mb <= 0) {
        size_t fr = 0, tot = 0;
        check(hipMemGetInfo(&fr, &tot), "memory info");
        size_t cached = 0;
        {
            std::lock_guard<std::mutex> lk(cache().mu);
            cached = cache().cached;
        }
        budget_bytes = std::max<int64_t>((int64_t)((fr + cached) / 10 * 4), (int64_t)1 << 30);
    }
    return std::max<int64_t>(budget_bytes / (int64_t)h->esz, 1);
}

// The far field without precomputation: the ACA list (blocks Lb with levels
// Ll, level-sorted; lmap: the leaf of each entry, null: entry i is leaf i)
// cut into chunks whose k_max column scratch fits the budget, each holding a
// share of every level as in the stored build, and the pieces that each
// chunk's products add to the row tiles, sorted by (chunk, tile)
void np_plan(hmx_hmatrix_s* h, const AcaPlan& plan, const int4* Lb, const int32_t* Ll,
             int64_t nl, const int32_t* lmap, hipStream_t st) {
    NpPlan& P = h->np;
    P.nl = nl;
    P.big_words = plan.big_words;
    P.med_words = plan.med_words;
    P.tiny_words = plan.tiny_words;
    const int kmax = h->prm.max_rank;
    DevBuf scan_scr;
    auto scan = [&](int64_t* data, int64_t cnt) -> int64_t {
        const size_t need = scan_scratch_bytes(cnt + 1) + 64;
        if (!scan_scr.p || scan_scr.bytes < need) alloc(scan_scr, need, "scan scratch");
        check(exclusive_scan_i64(data, cnt, data + cnt, scan_scr.p, st), "scan");
        return read_scalar(data + cnt, st);
    };
    DevBuf ident;
    if (!lmap) {
        alloc(ident, (size_t)nl * 4, "list leaves");
        check(launch_np_iota(ident.as<int32_t>(), nl, st), "list leaves");
        lmap = ident.as<int32_t>();
    }
    DevBuf cc;
    alloc(cc, (size_t)(nl + 1) * 8, "capacity");
    check(launch_extent(Lb, nl, 7, kmax, nullptr, nullptr, cc.as<int64_t>(), st), "extent");
    const int64_t ctot = scan(cc.as<int64_t>(), nl);
    cc.release();
    const int64_t budget = aca_budget(h);
    const int32_t* levels = Ll;
    ChunkOrder o;
    if (ctot > budget) {
        const int nsl = (int)std::min<int64_t>((ctot + ctot / 8 + budget - 1) / budget, 1 << 20);
        interleave(Lb, Ll, nl, lmap, nullptr, nsl, st, o);
        P.blocks.swap(o.blocks);
        P.lmap.swap(o.cap);
        levels = o.levels.as<int32_t>();
        P.bounds = o.bounds;
    } else {
        alloc(P.blocks, (size_t)nl * sizeof(int4), "list blocks");
        alloc(P.lmap, (size_t)nl * 4, "list leaves");
        check(hipMemcpyAsync(P.blocks.p, Lb, (size_t)nl * sizeof(int4), hipMemcpyDeviceToDevice,
                             st),
              "list blocks");
        check(hipMemcpyAsync(P.lmap.p, lmap, (size_t)nl * 4, hipMemcpyDeviceToDevice, st),
              "list leaves");
        P.bounds = {0, nl};
    }
    const int nch = (int)P.bounds.size() - 1;
    const int4* B = P.blocks.as<int4>();
    // k_max columns of U and V per block, offsets in chunk order
    alloc(P.cu, (size_t)(nl + 1) * 8, "U capacity offsets");
    alloc(P.cv, (size_t)(nl + 1) * 8, "V capacity offsets");
    check(launch_extent(B, nl, 0, kmax, nullptr, nullptr, P.cu.as<int64_t>(), st), "extent");
    check(launch_extent(B, nl, 1, kmax, nullptr, nullptr, P.cv.as<int64_t>(), st), "extent");
    scan(P.cu.as<int64_t>(), nl);
    scan(P.cv.as<int64_t>(), nl);
    P.hcu.assign(nch + 1, 0);
    P.hcv.assign(nch + 1, 0);
    for (int k = 0; k <= nch; ++k) {
        check(hipMemcpyAsync(&P.hcu[k], P.cu.as<int64_t>() + P.bounds[k], 8,
                             hipMemcpyDeviceToHost, st),
              "cu");
        check(hipMemcpyAsync(&P.hcv[k], P.cv.as<int64_t>() + P.bounds[k], 8,
                             hipMemcpyDeviceToHost, st),
              "cv");
    }
    // the size classes of every chunk (level-sorted within the chunk)
    DevBuf split;
    alloc(split, (size_t)nch * 3 * 8, "class split");
    check(hipMemsetAsync(split.p, 0, (size_t)nch * 3 * 8, st), "class split");
    const int lv[3] = {plan.split0, plan.split, plan.split2};
    for (int k = 0; k < nch; ++k)
        for (int c = 0; c < 3; ++c)
            check(launch_level_split(levels + P.bounds[k], P.bounds[k + 1] - P.bounds[k], lv[c],
                                     split.as<int64_t>() + 3 * k + c, st),
                  "class split");
    P.cls.assign((size_t)nch * 3, 0);
    d2h(P.cls.data(), split.p, (size_t)nch * 3 * 8, st);
    P.max_u = P.max_v = P.max_nb = 0;
    for (int k = 0; k < nch; ++k) {
        P.max_u = std::max(P.max_u, P.hcu[k + 1] - P.hcu[k]);
        P.max_v = std::max(P.max_v, P.hcv[k + 1] - P.hcv[k]);
        P.max_nb = std::max(P.max_nb, P.bounds[k + 1] - P.bounds[k]);
    }
    alloc(P.rank, (size_t)nl * 4, "list ranks");
    alloc(P.steps, (size_t)nl * 4, "list steps");
    check(hipMemsetAsync(P.rank.p, 0, (size_t)nl * 4, st), "list ranks");
    check(hipMemsetAsync(P.steps.p, 0, (size_t)nl * 4, st), "list steps");
    // apply pieces: (entry, side) per row tile of tau (side 0) and, for a
    // mirrored primary, of sigma (side 1), sorted by (chunk, tile)
    DevBuf cnt;
    alloc(cnt, (size_t)(nl + 1) * 8, "piece counts");
    check(launch_np_piece_count(B, nl, h->sym, h->tile_of_point.as<int32_t>(),
                                cnt.as<int64_t>(), st),
          "piece counts");
    const int64_t npcs = scan(cnt.as<int64_t>(), nl);
    if (npcs >= ((int64_t)1 << 32)) {
        set_err("far_recompute: %lld apply pieces exceed the sort's 2^32", (long long)npcs);
        throw Fail{HMX_ERR_UNSUPPORTED};
    }
    P.npcs = npcs;
    int tbits = 1, cbits = 1;
    while ((1ll << tbits) < h->ntiles) ++tbits;
    while ((1ll << cbits) < nch) ++cbits;
    DevBuf dbounds, keys, vals, pcs, sscr, flags, dcseg;
    alloc(dbounds, (size_t)(nch + 1) * 8, "chunk bounds");
    check(hipMemcpyAsync(dbounds.p, P.bounds.data(), (size_t)(nch + 1) * 8,
                         hipMemcpyHostToDevice, st),
          "chunk bounds");
    alloc(keys, (size_t)npcs * 8, "piece keys");
    alloc(vals, (size_t)npcs * 4, "piece order");
    alloc(pcs, (size_t)npcs * sizeof(int2), "pieces");
    check(launch_np_piece_fill(B, nl, h->sym, h->tile_of_point.as<int32_t>(), cnt.as<int64_t>(),
                               dbounds.as<int64_t>(), nch, tbits, keys.as<uint64_t>(),
                               vals.as<uint32_t>(), pcs.as<int2>(), st),
          "piece fill");
    alloc(sscr, radix_sort_scratch_bytes(npcs), "piece sort");
    check(radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(), npcs, tbits + cbits, sscr.p,
                           st),
          "piece sort");
    sscr.release();
    alloc(flags, (size_t)(npcs + 1) * 8, "segment flags");
    check(launch_np_seg_flags(keys.as<uint64_t>(), npcs, flags.as<int64_t>(), st),
          "segment flags");
    P.nseg = npcs > 0 ? scan(flags.as<int64_t>(), npcs) : 0;
    alloc(P.seg_start, (size_t)(P.nseg + 1) * 8, "segment starts");
    alloc(P.seg_tile, (size_t)std::max<int64_t>(P.nseg, 1) * 4, "segment tiles");
    alloc(P.spcs, (size_t)std::max<int64_t>(npcs, 1) * sizeof(int2), "sorted pieces");
    check(launch_np_seg_fill(keys.as<uint64_t>(), vals.as<uint32_t>(), pcs.as<int2>(),
                             flags.as<int64_t>(), npcs, P.nseg, tbits, P.seg_start.as<int64_t>(),
                             P.seg_tile.as<int32_t>(), P.spcs.as<int2>(), st),
          "segments");
    alloc(dcseg, (size_t)(nch + 1) * 8, "chunk segments");
    check(hipMemsetAsync(dcseg.p, 0, (size_t)(nch + 1) * 8, st), "chunk segments");
    check(launch_np_chunk_segs(keys.as<uint64_t>(), P.seg_start.as<int64_t>(), P.nseg, tbits,
                               nch, dcseg.as<int64_t>(), st),
          "chunk segments");
    P.cseg.assign(nch + 1, 0);
    d2h(P.cseg.data(), dcseg.p, (size_t)(nch + 1) * 8, st);
    check(hipStreamSynchronize(st), "plan sync");
}

// phases 4-5: batched ACA, compaction, the tile-major matrix pool
void stage_factors(hmx_hmatrix_s* h, const AcaPlan& plan, hipStream_t st,
                   std::chrono::steady_clock::time_point t_all) {
    using clk = std::chrono::steady_clock;
    const int64_t n = h->n;
    const int d = h->d;
    const int f64 = h->f64;
    const size_t esz = h->esz;
    const size_t ssz = h->ssz;
    const int smode = h->smode;
    hmx_stats& S = h->stats;
    auto t0 = clk::now();

    const int kmax = h->prm.max_rank;
    DevBuf scan_scr;
    // exclusive scan of data[0..cnt) in place; the total is also stored in
    // data[cnt] (every offset array has cnt + 1 entries) and returned
    auto scan = [&](int64_t* data, int64_t cnt) -> int64_t {
        const size_t need = scan_scratch_bytes(cnt + 1) + 64;
        if (!scan_scr.p || scan_scr.bytes < need) alloc(scan_scr, need, "scan scratch");
        check(exclusive_scan_i64(data, cnt, data + cnt, scan_scr.p, st), "scan");
        return read_scalar(data + cnt, st);
    };

    // ---- 4. batched ACA of the admissible leaves, in chunks ----
    // A pass approximates a list of blocks in chunks: every block gets
    // scratch for its column capacity (k_max, or the predicted target of the
    // learned sizing) within the chunk budget; after the chunk's ACA the
    // factors are compacted to their exact ranks in the storage type (U as
    // the source of the tile-major pool, V as phase 1's operand) and
    // appended to the pools.
    alloc(h->rank, std::max<int64_t>(h->n_adm, 1) * 4, "ranks");
    alloc(h->steps, std::max<int64_t>(h->n_adm, 1) * 4, "steps");
    // F: the exact-rank factors of every approximated leaf (per chunk its U_b
    // then its V_b, column-major, storage type).  rfo[b]: offset of leaf b's
    // row factor (its U_b; with the symmetric far field a mirror's row factor
    // is its primary's V), vfo[b]: offset of V_b (approximated leaves)
    DevBuf F, rfo, vfo;
    // the largest ACA chunk scratch, kept past the ACA: the near-field pool
    // reuses it when it fits (new device memory that was used and released
    // before is cleared by the driver on allocation, tens of GB per second)
    DevBuf aca_keep;
    alloc(rfo, (h->n_adm + 1) * 8, "row factor offsets");
    alloc(vfo, (h->n_adm + 1) * 8, "V offsets");
    int nchunks = 0;
    double aca_ms = 0.0;
    int64_t ftot = 0;
    const bool learned = plan.rt != nullptr;
    const bool aca_only = h->prm.aca_only != 0;
    // The ACA list: every admissible leaf, or with the symmetric far field the
    // primary ones (tau before sigma, or tau = sigma) in their canonical order,
    // which keeps the levels sorted; results return to the leaves at the end
    int64_t nl = h->n_adm;
    DevBuf lst, lblk, llev, lrt, lrank, lsteps, lue, lve;
    const int4* Lb = h->adm.as<int4>();
    const int32_t* Ll = plan.cls;
    const int32_t* Lrt = plan.rt;
    if (h->n_adm > 0 && h->sym) {
        const int64_t na = h->n_adm;
        alloc(h->partner, (size_t)na * 4, "mirror table");
        {
            DevBuf keys, vals, sscr, bad;
            alloc(keys, (size_t)na * 8, "mirror keys");
            alloc(vals, (size_t)na * 4, "mirror order");
            alloc(bad, 8, "mirror check");
            check(hipMemsetAsync(bad.p, 0, 8, st), "mirror check");
            check(launch_mirror_keys(h->adm.as<int4>(), na, keys.as<uint64_t>(),
                                     vals.as<uint32_t>(), st),
                  "mirror keys");
            int bits = 32;
            while (bits < 64 && (1ll << (bits - 32)) <= n) ++bits;
            alloc(sscr, radix_sort_scratch_bytes(na), "mirror sort");
            check(radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(), na, bits, sscr.p, st),
                  "mirror sort");
            check(launch_mirror_find(h->adm.as<int4>(), na, keys.as<uint64_t>(),
                                     vals.as<uint32_t>(), h->partner.as<int32_t>(), bad.as<int>(),
                                     st),
                  "mirror find");
            if (read_scalar(bad.as<int>(), st) != 0) {
                set_err("symmetric far field: an admissible leaf has no mirror in the partition");
                throw Fail{HMX_ERR_DEVICE};
            }
        }
        DevBuf pos;
        alloc(pos, (size_t)(na + 1) * 8, "primary flags");
        check(launch_primary_flags(h->adm.as<int4>(), na, 1, pos.as<int64_t>(), st),
              "primary flags");
        nl = scan(pos.as<int64_t>(), na);
        alloc(lst, (size_t)std::max<int64_t>(nl, 1) * 4, "ACA list");
        alloc(lblk, (size_t)std::max<int64_t>(nl, 1) * sizeof(int4), "ACA list blocks");
        alloc(llev, (size_t)std::max<int64_t>(nl, 1) * 4, "ACA list levels");
        if (Lrt) alloc(lrt, (size_t)std::max<int64_t>(nl, 1) * 4, "ACA list targets");
        check(launch_gather_list(pos.as<int64_t>(), na, h->adm.as<int4>(), plan.cls, Lrt,
                                 lst.as<int32_t>(), lblk.as<int4>(), llev.as<int32_t>(),
                                 Lrt ? lrt.as<int32_t>() : nullptr, st),
              "ACA list");
        Lb = lblk.as<int4>();
        Ll = llev.as<int32_t>();
        if (Lrt) Lrt = lrt.as<int32_t>();
    }
    alloc(lrank, (size_t)std::max<int64_t>(nl, 1) * 4, "list ranks");
    alloc(lsteps, (size_t)std::max<int64_t>(nl, 1) * 4, "list steps");
    alloc(lue, (size_t)(nl + 1) * 8, "list U offsets");
    alloc(lve, (size_t)(nl + 1) * 8, "list V offsets");
    if (h->far_np) {
        // no precomputation: the chunk plan only; the leaves keep rank 0 (no
        // factor pieces in the matrix pool) until a matvec approximates them
        if (nl > 0) np_plan(h, plan, Lb, Ll, nl, h->sym ? lst.as<int32_t>() : nullptr, st);
        nchunks = nl > 0 ? (int)h->np.bounds.size() - 1 : 0;
        check(hipMemsetAsync(h->rank.p, 0, h->rank.bytes, st), "ranks");
        check(hipMemsetAsync(h->steps.p, 0, h->steps.bytes, st), "steps");
        check(hipMemsetAsync(rfo.p, 0, rfo.bytes, st), "row factor offsets");
        check(hipMemsetAsync(vfo.p, 0, vfo.bytes, st), "V offsets");
    } else if (nl > 0) {
        const int64_t budget = aca_budget(h);
        // the single-workgroup classes run beside the multi-workgroup path
        AuxStream auxs[3];
        const hipStream_t aux[3] = {auxs[0].s, auxs[1].s, auxs[2].s};
        const bool have_aux = aux[0] && aux[1] && aux[2];
        AcaArgs a = aca_args_base(h, plan);
        DevBuf split;
        alloc(split, 3 * 8, "class split");

        // one pass over blocks[0..nb): cap = per-block column capacity (null:
        // k_max), rt = one-shot targets (null: adaptive); exact offsets of the
        // blocks' factors in the pools go to ue_all / ve_all
        // (bounds: the chunks' first blocks and the end, when the caller cut
        // the list; each chunk must be level-sorted)
        auto pass = [&](const int4* blocks, const int32_t* levels, int64_t nb, const int32_t* cap,
                        const int32_t* rt, int one_shot, int cap_only, int32_t* rank,
                        int32_t* steps, int64_t* ue_all, int64_t* ve_all,
                        const std::vector<int64_t>* bounds) {
            DevBuf cu, cv, cc, Ucap;
            alloc(cu, (nb + 1) * 8, "U capacity offsets");
            alloc(cv, (nb + 1) * 8, "V capacity offsets");
            alloc(cc, (nb + 1) * 8, "capacity offsets");
            check(launch_extent(blocks, nb, cap ? 3 : 0, kmax, cap, nullptr, cu.as<int64_t>(), st),
                  "extent");
            check(launch_extent(blocks, nb, cap ? 4 : 1, kmax, cap, nullptr, cv.as<int64_t>(), st),
                  "extent");
            check(launch_extent(blocks, nb, cap ? 8 : 7, kmax, cap, nullptr, cc.as<int64_t>(), st),
                  "extent");
            scan(cu.as<int64_t>(), nb);
            scan(cv.as<int64_t>(), nb);
            const int64_t ctot = scan(cc.as<int64_t>(), nb);
            S.aca_capacity += ctot;
            std::vector<int64_t> hb;
            int nch;
            if (bounds) {
                hb = *bounds;
                nch = (int)hb.size() - 1;
            } else {
                // each chunk's capacity is at most step + one block
                nch = (int)std::min<int64_t>((ctot + budget - 1) / budget, 1 << 20);
                nch = std::max(nch, 1);
                const int64_t step = (ctot + nch - 1) / nch;
                DevBuf bnd;
                alloc(bnd, (size_t)(nch + 1) * 8, "chunk bounds");
                check(launch_chunk_bounds(cc.as<int64_t>(), nb, step, nch, bnd.as<int64_t>(), st),
                      "chunk bounds");
                hb.resize(nch + 1);
                d2h(hb.data(), bnd.p, (nch + 1) * 8, st);
            }
            std::vector<int64_t> hcu(nch + 1), hcv(nch + 1);
            int64_t max_u = 0, max_v = 0;
            for (int k = 0; k <= nch; ++k) {
                check(hipMemcpyAsync(&hcu[k], cu.as<int64_t>() + hb[k], 8, hipMemcpyDeviceToHost,
                                     st),
                      "cu");
                check(hipMemcpyAsync(&hcv[k], cv.as<int64_t>() + hb[k], 8, hipMemcpyDeviceToHost,
                                     st),
                      "cv");
            }
            check(hipStreamSynchronize(st), "bounds sync");
            for (int k = 0; k < nch; ++k) {
                max_u = std::max(max_u, hcu[k + 1] - hcu[k]);
                max_v = std::max(max_v, hcv[k + 1] - hcv[k]);
            }
            // a pass with storage for the targets only keeps a reserve behind
            // the chunk's capacity, where blocks that need more columns
            // continue (those it cannot hold are approximated again later)
            const int64_t ovf_cap =
                cap_only ? std::max<int64_t>(std::max(max_u, max_v) / 16,
                                             2 * std::min(h->big_adm, split_rows(h)) * kmax)
                         : 0;
            // U and V scratch in one block: a single large block can serve
            // the near-field pool once the ACA is done (the cache reuses a
            // block for requests of 3/4 of its size or more), so that pool
            // takes no new device memory, which the driver would clear first
            const int64_t ucols = (std::max<int64_t>(max_u + ovf_cap, 1) + 63) / 64 * 64;
            alloc(Ucap, (size_t)(ucols + std::max<int64_t>(max_v + ovf_cap, 1)) * esz,
                  "ACA chunk scratch");
            void* const vcap = (char*)Ucap.p + (size_t)ucols * esz;
            DevBuf ovf_used, moved;
            if (cap_only) {
                alloc(ovf_used, 8, "overflow counter");
                alloc(moved, (size_t)nb * 8, "overflow offsets");
                check(hipMemsetAsync(moved.p, 0xff, (size_t)nb * 8, st), "overflow offsets");
            }
            a.U = Ucap.p;
            a.V = vcap;
            a.one_shot = one_shot;
            a.cap_only = cap_only;
            a.ovf_used = cap_only ? ovf_used.as<unsigned long long>() : nullptr;
            a.ovf_cap = ovf_cap;
            a.ovf_moved = cap_only ? moved.as<int64_t>() : nullptr;
            for (int k = 0; k < nch; ++k) {
                const int64_t b0 = hb[k], nbk = hb[k + 1] - hb[k];
                if (nbk == 0) continue;
                ++nchunks;
                const auto ta = clk::now();
                a.blocks = blocks + b0;
                a.nblocks = nbk;
                a.uoff = cu.as<int64_t>() + b0;
                a.voff = cv.as<int64_t>() + b0;
                a.ubase = hcu[k];
                a.vbase = hcv[k];
                a.rtarget = rt ? rt + b0 : nullptr;
                // the size classes of this chunk (level-sorted within the chunk)
                int64_t cls[3];
                const int lv[3] = {plan.split0, plan.split, plan.split2};
                for (int c = 0; c < 3; ++c)
                    check(launch_level_split(levels + b0, nbk, lv[c], split.as<int64_t>() + c, st),
                          "class split");
                d2h(cls, split.p, sizeof cls, st);
                a.nsplit = cls[0];
                a.nbig = cls[1];
                a.nmed = cls[2];
                a.rank = rank + b0;
                a.steps = steps + b0;
                a.ovf_u0 = hcu[k] + max_u;
                a.ovf_v0 = hcv[k] + max_v;
                a.ovf_moved = cap_only ? moved.as<int64_t>() + b0 : nullptr;
                if (a.ovf_used)
                    check(hipMemsetAsync(a.ovf_used, 0, sizeof(unsigned long long), st),
                          "overflow counter");
                SplitBuffers sb;
                if (a.nsplit > 0) prepare_split(h, a, f64, st, sb);
                check(aca_classes_begin(a, f64, st, have_aux ? aux : nullptr), "aca");
                if (a.nsplit > 0)
                    check(launch_aca_split(a, sb.P, f64, st), "aca (many workgroups per block)");
                check(aca_classes_join(st, have_aux ? aux : nullptr), "aca join");
                if (a.ovf_moved)
                    check(launch_apply_moved(a.ovf_moved, nbk, a.ovf_u0, a.ovf_v0,
                                             cu.as<int64_t>() + b0, cv.as<int64_t>() + b0, st),
                          "overflow offsets");
                check(hipStreamSynchronize(st), "aca sync");  // before sb returns to the cache
                aca_ms += ms_since(ta);
                if (aca_only) continue;
                // exact offsets of this chunk's blocks: chunk-local scans plus the
                // running total; the chunk's U factors, then its V factors
                int64_t* ue = ue_all + b0;
                int64_t* ve = ve_all + b0;
                check(launch_extent(a.blocks, nbk, 3, 0, a.rank, nullptr, ue, st), "extent");
                check(launch_extent(a.blocks, nbk, 4, 0, a.rank, nullptr, ve, st), "extent");
                const int64_t uk = scan(ue, nbk), vk = scan(ve, nbk);
                check(launch_add_const(ue, nbk, ftot, st), "offsets");
                check(launch_add_const(ve, nbk, ftot + uk, st), "offsets");
                // the pool's size extrapolated from the chunks so far (each chunk
                // holds a share of every level), so it grows in one step
                // rather than by doublings that copy tens of GB
                int64_t want = ftot + uk + vk;
                if (nch > 1 && (size_t)want * ssz > F.bytes)
                    want = std::max<int64_t>(
                        want, (int64_t)((double)want / (k + 1) * nch * 1.05) + 1);
                grow(F, (size_t)want * ssz, (size_t)ftot * ssz, st, "factor pool", true);
                check(launch_compact_u(a.blocks, nbk, a.rank, a.uoff, a.ubase, ue, Ucap.p, F.p,
                                       smode, st),
                      "compact U");
                check(launch_compact_v(a.blocks, nbk, a.rank, a.voff, a.vbase, ve, vcap, F.p,
                                       smode, st),
                      "compact V");
                check(hipStreamSynchronize(st), "compact sync");
                ftot += uk + vk;
            }
            if (!aca_only && Ucap.bytes > aca_keep.bytes) aca_keep.swap(Ucap);
        };

        // The level-ordered list cut into chunks by capacity would give each
        // chunk one or two size classes (the largest blocks first, the leaf
        // level last), so the classes, which run concurrently, would rarely
        // overlap.  A list that needs several chunks is reordered so that every
        // chunk holds the same share of every level (level-sorted within the
        // chunk); ranks, steps and pool offsets return to the canonical order.
        auto chunked_pass = [&](const int4* blocks, const int32_t* levels, int64_t nb,
                                const int32_t* cap, const int32_t* rt, int one_shot, int cap_only,
                                int32_t* rank, int32_t* steps, int64_t* ue_all, int64_t* ve_all) {
            DevBuf cc;
            alloc(cc, (nb + 1) * 8, "capacity");
            check(launch_extent(blocks, nb, cap ? 8 : 7, kmax, cap, nullptr, cc.as<int64_t>(), st),
                  "extent");
            const int64_t ctot = scan(cc.as<int64_t>(), nb);
            cc.release();
            if (ctot <= budget) {
                pass(blocks, levels, nb, cap, rt, one_shot, cap_only, rank, steps, ue_all, ve_all,
                     nullptr);
                return;
            }
            // slices of equal shares, with room for the variation of the
            // per-block capacities between slices
            const int nsl = (int)std::min<int64_t>((ctot + ctot / 8 + budget - 1) / budget, 1 << 20);
            ChunkOrder o;
            interleave(blocks, levels, nb, cap, rt, nsl, st, o);
            const std::vector<int64_t>& bounds = o.bounds;
            DevBuf &perm = o.perm, &pb = o.blocks, &pl = o.levels, &pc = o.cap, &pr = o.rt;
            DevBuf prk, pst, pue, pve;
            alloc(prk, (size_t)nb * 4, "interleaved ranks");
            alloc(pst, (size_t)nb * 4, "interleaved steps");
            alloc(pue, (size_t)(nb + 1) * 8, "interleaved U offsets");
            alloc(pve, (size_t)(nb + 1) * 8, "interleaved V offsets");
            // the same targets serve as capacity and as the kernel's target (cap == rt)
            const int32_t* pcap = cap ? (cap == rt ? pr.as<int32_t>() : pc.as<int32_t>()) : nullptr;
            pass(pb.as<int4>(), pl.as<int32_t>(), nb, pcap, rt ? pr.as<int32_t>() : nullptr,
                 one_shot, cap_only, prk.as<int32_t>(), pst.as<int32_t>(), pue.as<int64_t>(),
                 pve.as<int64_t>(), &bounds);
            const int32_t* li = (const int32_t*)perm.p;
            check(launch_scatter_i32(li, nb, prk.as<int32_t>(), rank, 0, st), "interleaved ranks");
            check(launch_scatter_i32(li, nb, pst.as<int32_t>(), steps, 0, st), "interleaved steps");
            if (!aca_only) {
                check(launch_scatter_i64(li, nb, pue.as<int64_t>(), ue_all, st), "interleaved U");
                check(launch_scatter_i64(li, nb, pve.as<int64_t>(), ve_all, st), "interleaved V");
                check(hipMemcpyAsync(ue_all + nb, pue.as<int64_t>() + nb, 8,
                                     hipMemcpyDeviceToDevice, st),
                      "U total");
                check(hipMemcpyAsync(ve_all + nb, pve.as<int64_t>() + nb, 8,
                                     hipMemcpyDeviceToDevice, st),
                      "V total");
            }
            check(hipStreamSynchronize(st), "interleave sync");  // before the buffers return
        };

        int32_t* Lrank = lrank.as<int32_t>();
        int32_t* Lsteps = lsteps.as<int32_t>();
        int64_t* Lue = lue.as<int64_t>();
        int64_t* Lve = lve.as<int64_t>();
        if (!learned) {
            chunked_pass(Lb, Ll, nl, nullptr, nullptr, 0, 0, Lrank, Lsteps, Lue, Lve);
        } else {
            // learned sizing: predicted targets, a pass with storage of that
            // size, then the blocks left unfinished again with k_max columns
            // (sizing form: plain adaptive; one-shot form: the same target
            // steps, the test, then adaptive)
            const int one_shot = h->prm.learned_one_shot;
            const int32_t* rt = Lrt;
            chunked_pass(Lb, Ll, nl, rt, rt, one_shot, 1, Lrank, Lsteps, Lue, Lve);
            DevBuf flag;
            alloc(flag, (nl + 1) * 8, "fallback flags");
            check(launch_over_flags(Lrank, rt, nl, flag.as<int64_t>(), st), "overflow flags");
            S.aca_overflow = scan(flag.as<int64_t>(), nl);
            check(launch_fail_flags(Lrank, nl, flag.as<int64_t>(), st), "fallback flags");
            const int64_t nfb = scan(flag.as<int64_t>(), nl);
            S.aca_fallback = nfb;
            if (nfb > 0) {
                DevBuf list, bfb, lvfb, rtfb, rkfb, stfb, uefb, vefb;
                alloc(list, nfb * 4, "fallback list");
                alloc(bfb, nfb * sizeof(int4), "fallback blocks");
                alloc(lvfb, nfb * 4, "fallback levels");
                alloc(rtfb, nfb * 4, "fallback targets");
                alloc(rkfb, nfb * 4, "fallback ranks");
                alloc(stfb, nfb * 4, "fallback steps");
                alloc(uefb, (nfb + 1) * 8, "fallback U offsets");
                alloc(vefb, (nfb + 1) * 8, "fallback V offsets");
                check(launch_gather_failed(Lrank, flag.as<int64_t>(), nl, Lb, Ll, rt,
                                           list.as<int32_t>(), bfb.as<int4>(),
                                           lvfb.as<int32_t>(), rtfb.as<int32_t>(), st),
                      "fallback gather");
                pass(bfb.as<int4>(), lvfb.as<int32_t>(), nfb, nullptr,
                     one_shot ? rtfb.as<int32_t>() : nullptr, one_shot, 0, rkfb.as<int32_t>(),
                     stfb.as<int32_t>(), uefb.as<int64_t>(), vefb.as<int64_t>(), nullptr);
                const int32_t* li = list.as<int32_t>();
                check(launch_scatter_i32(li, nfb, rkfb.as<int32_t>(), Lrank, 0, st),
                      "fallback ranks");
                check(launch_scatter_i32(li, nfb, stfb.as<int32_t>(), Lsteps, 1, st),
                      "fallback steps");
                if (!aca_only) {
                    check(launch_scatter_i64(li, nfb, uefb.as<int64_t>(), Lue, st),
                          "fallback offsets");
                    check(launch_scatter_i64(li, nfb, vefb.as<int64_t>(), Lve, st),
                          "fallback offsets");
                }
                check(hipStreamSynchronize(st), "fallback sync");
            }
        }
        h->factor_entries = ftot;
        S.phase_ms[3] = aca_ms;
        // the list's results back to the leaves (a mirror takes its
        // primary's rank, and its primary's V as its row factor)
        check(launch_scatter_list(h->sym ? lst.as<int32_t>() : nullptr, nl,
                                  h->sym ? h->partner.as<int32_t>() : nullptr, Lrank, Lsteps,
                                  Lue, Lve, h->rank.as<int32_t>(), h->steps.as<int32_t>(),
                                  aca_only ? nullptr : rfo.as<int64_t>(),
                                  aca_only ? nullptr : vfo.as<int64_t>(), st),
              "ACA results");
        // rank statistics over the leaves, ACA work over the list, on the device
        DevBuf red;
        alloc(red, 6 * sizeof(unsigned long long), "stats");
        unsigned long long* rd = red.as<unsigned long long>();
        check(launch_int_stats(h->rank.as<int32_t>(), h->n_adm, rd, st), "rank stats");
        check(launch_int_stats(Lsteps, nl, rd + 2, st), "step stats");
        check(launch_aca_work(Lb, Lrank, Lsteps, nl, rd + 4, st), "aca work");
        unsigned long long hv[6];
        check(hipMemcpyAsync(hv, rd, sizeof hv, hipMemcpyDeviceToHost, st), "stats readback");
        check(hipStreamSynchronize(st), "stats sync");
        S.max_rank_used = (int32_t)hv[0];
        S.sum_rank = (int64_t)hv[1];
        S.aca_columns = (int64_t)hv[3];
        S.aca_kernel_evals = (int64_t)hv[4];
        S.aca_flops = (double)hv[5];
    }
    if (!F.p) alloc(F, 16, "factor pool");
    S.aca_chunks = nchunks;
    S.phase_ms[4] = ms_since(t0) - S.phase_ms[3];
    lst.release();
    lblk.release();
    llev.release();
    lrt.release();
    lrank.release();
    lsteps.release();
    lue.release();
    lve.release();
    if (aca_only) {
        F.release();
        finish_stats(h, t_all);
        return;
    }
    if (h->n_adm > 0) {  // entries the two phases of a matvec read
        DevBuf ex;
        alloc(ex, (h->n_adm + 1) * 8, "entry counts");
        check(launch_extent(h->adm.as<int4>(), h->n_adm, 3, 0, h->rank.as<int32_t>(), nullptr,
                            ex.as<int64_t>(), st),
              "extent");
        S.u_entries = scan(ex.as<int64_t>(), h->n_adm);
        check(launch_extent(h->adm.as<int4>(), h->n_adm, 4, 0, h->rank.as<int32_t>(), nullptr,
                            ex.as<int64_t>(), st),
              "extent");
        S.v_entries = scan(ex.as<int64_t>(), h->n_adm);
    }
    t0 = clk::now();
    // t offsets, vector pool, column -> leaf map of phase 1
    alloc(h->toff, (h->n_adm + 1) * 8, "t offsets");
    if (h->n_adm > 0) {
        check(launch_extent(h->adm.as<int4>(), h->n_adm, 5, 0, h->rank.as<int32_t>(), nullptr,
                            h->toff.as<int64_t>(), st),
              "extent");
        h->sum_rank = scan(h->toff.as<int64_t>(), h->n_adm);
    }
    alloc(h->vecpool, (size_t)(n + h->sum_rank) * esz, "vector pool");
    S.phase_ms[4] += ms_since(t0);
    t0 = clk::now();

    // ---- 5. tile-major matrix pool: pieces (leaf block x row tile) sorted by
    //         tile, then filled with near-field entries and U rows ----
    {
        const int64_t nb = h->n_adm + h->n_dense;
        DevBuf cnt, unsorted, keys, vals, sscr, psize, pcols;
        alloc(cnt, (nb + 1) * 8, "piece counts");
        check(launch_extent(h->adm.as<int4>(), h->n_adm, 6, 0, h->rank.as<int32_t>(),
                            h->tile_of_point.as<int32_t>(), cnt.as<int64_t>(), st),
              "extent");
        check(launch_extent(h->dense.as<int4>(), h->n_dense, 6, 0, nullptr,
                            h->tile_of_point.as<int32_t>(), cnt.as<int64_t>() + h->n_adm, st),
              "extent");
        h->npieces = scan(cnt.as<int64_t>(), nb);
        alloc(unsorted, h->npieces * sizeof(Piece), "pieces");
        alloc(keys, h->npieces * 8, "piece keys");
        alloc(vals, h->npieces * 4, "piece vals");
        check(launch_piece_fill(h->adm.as<int4>(), h->n_adm, h->rank.as<int32_t>(),
                                h->tile_of_point.as<int32_t>(), h->tile_lo.as<int32_t>(),
                                cnt.as<int64_t>(), h->toff.as<int64_t>(), n, 0,
                                unsorted.as<Piece>(), keys.as<uint64_t>(), vals.as<uint32_t>(), st),
              "piece fill");
        check(launch_piece_fill(h->dense.as<int4>(), h->n_dense, nullptr,
                                h->tile_of_point.as<int32_t>(), h->tile_lo.as<int32_t>(),
                                cnt.as<int64_t>() + h->n_adm, nullptr, 0, 0, unsorted.as<Piece>(),
                                keys.as<uint64_t>(), vals.as<uint32_t>(), st),
              "piece fill");
        int bits = 1;
        while ((1ll << bits) <= h->ntiles) ++bits;
        alloc(sscr, radix_sort_scratch_bytes(h->npieces), "piece sort");
        check(radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(), h->npieces, bits, sscr.p,
                               st),
              "piece sort");
        alloc(h->pieces, h->npieces * sizeof(Piece), "sorted pieces");
        DevBuf psu, psn, pc, pcu;
        alloc(psu, (h->npieces + 1) * 8, "piece sizes");
        alloc(psn, (h->npieces + 1) * 8, "piece sizes");
        alloc(pc, (h->npieces + 1) * 8, "piece columns");
        alloc(pcu, (h->npieces + 1) * 8, "piece columns");
        const int R = rows_per_unit(smode, h->nmode);
        check(launch_piece_gather(unsorted.as<Piece>(), vals.as<uint32_t>(), h->npieces,
                                  h->pieces.as<Piece>(), psu.as<int64_t>(), psn.as<int64_t>(),
                                  pc.as<int64_t>(), pcu.as<int64_t>(), h->tile_lo.as<int32_t>(), R,
                                  h->nmode != 3, st),
              "piece gather");
        h->upool_entries = scan(psu.as<int64_t>(), h->npieces);
        h->npool_entries = scan(psn.as<int64_t>(), h->npieces);
        h->ncols_total = scan(pc.as<int64_t>(), h->npieces);
        h->ncols_u = scan(pcu.as<int64_t>(), h->npieces);
        alloc(h->widx, (size_t)std::max<int64_t>(h->ncols_total, 1) * 8, "column weights");
        check(launch_piece_layout(h->pieces.as<Piece>(), h->npieces, psu.as<int64_t>(),
                                  psn.as<int64_t>(), pc.as<int64_t>(), h->widx.as<int64_t>(), st),
              "piece layout");
        DevBuf tptr;
        alloc(tptr, (h->ntiles + 1) * 8, "tile ptr");
        check(launch_tile_offsets(keys.as<uint64_t>(), h->npieces, h->ntiles, tptr.as<int64_t>(),
                                  st),
              "tile ptr");
        alloc(h->tile_meta, (size_t)(h->ntiles + 1) * 4 * 8, "tile meta");
        check(launch_tile_meta(tptr.as<int64_t>(), h->ntiles, h->npieces, pc.as<int64_t>(),
                               pcu.as<int64_t>(), psu.as<int64_t>(), psn.as<int64_t>(),
                               h->tile_meta.as<int64_t>(), st),
              "tile meta");
        // the factor rows first; the near field's pool is allocated once the
        // exact-rank factors are released (the two never coexist).  It takes
        // over the kept ACA scratch when that block fits it (a block serves
        // requests of 3/4 of its size or more) and the factor rows still fit
        // in the free memory beside it; otherwise the scratch returns to the
        // cache now, where it can serve the factor rows or be released.
        const size_t near_bytes =
            h->nmode == 3 ? 0 : (size_t)std::max<int64_t>(h->npool_entries, 1) * h->nsz;
        const size_t ubytes = (size_t)std::max<int64_t>(h->upool_entries, 1) * ssz;
        bool keep = aca_keep.p && near_bytes > 0 && aca_keep.bytes >= near_bytes &&
                    aca_keep.bytes / 4 * 3 <= near_bytes;
        if (keep && !aca_keep.from.alloc) {
            size_t fr = 0, tot = 0;
            check(hipMemGetInfo(&fr, &tot), "memory info");
            size_t cached = 0;
            {
                std::lock_guard<std::mutex> lk(cache().mu);
                cached = cache().cached;
            }
            keep = fr + cached >= ubytes + ((size_t)4 << 30);
        }
        if (!keep) aca_keep.release();
        alloc(h->upool, ubytes, "factor pool");
        check(launch_piece_data(h->pieces.as<Piece>(), h->npieces, h->tile_lo.as<int32_t>(),
                                h->adm.as<int4>(), h->dense.as<int4>(), rfo.as<int64_t>(), F.p,
                                f64 ? h->soa64.p : h->soa32.p, n, d,
                                kernel_fn(h->kern, h->kd), h->upool.p, nullptr, smode, h->nmode, 1,
                                st),
              "piece data (factors)");
        h->Ru = R;
        // ---- phase-1 sources (t = V^T x by row tiles) ----
        // the V pool: pieces of V_b rows per row tile of sigma_b for every
        // leaf, or (symmetric far field) for the leaves that are their own
        // mirror; the other leaves read their mirror's factor pieces
        const int32_t* prt = h->sym ? h->partner.as<int32_t>() : nullptr;
        const int64_t nadm_pieces = h->n_adm > 0 ? read_scalar(cnt.as<int64_t>() + h->n_adm, st) : 0;
        const int64_t pfc_u = h->sym ? nadm_pieces : 0;  // pfc entries of the factor pieces
        DevBuf cntv;
        alloc(cntv, (h->n_adm + 1) * 8, "V piece counts");
        check(launch_vpiece_count(h->adm.as<int4>(), h->n_adm, h->rank.as<int32_t>(), prt,
                                  h->tile_of_point.as<int32_t>(), cntv.as<int64_t>(), st),
              "V piece counts");
        h->nvpieces = h->n_adm > 0 ? scan(cntv.as<int64_t>(), h->n_adm) : 0;
        alloc(h->pfc, (size_t)std::max<int64_t>(pfc_u + h->nvpieces, 1) * 8, "source columns");
        if (h->sym && nadm_pieces > 0)
            check(launch_pfc(h->pieces.as<Piece>(), vals.as<uint32_t>(), pcu.as<int64_t>(),
                             h->npieces, nadm_pieces, 0, h->pfc.as<int64_t>(), st),
                  "source columns");
        const int64_t vbase = h->sym ? h->ncols_u : 0;  // first source column of the V pool
        h->Rv = rows_per_unit(smode, smode);
        h->ncols_v = 0;
        alloc(h->vt_meta, (size_t)(h->ntiles + 1) * 4 * 8, "V pool tile meta");
        if (h->nvpieces > 0) {
            const int64_t nv = h->nvpieces;
            DevBuf vun, vk, vv, vs, vsz, vcl, vptr;
            alloc(vun, (size_t)nv * sizeof(Piece), "V pieces");
            alloc(vk, (size_t)nv * 8, "V piece keys");
            alloc(vv, (size_t)nv * 4, "V piece vals");
            check(launch_vpiece_fill(h->adm.as<int4>(), h->n_adm, h->rank.as<int32_t>(),
                                     cntv.as<int64_t>(), h->tile_of_point.as<int32_t>(),
                                     h->tile_lo.as<int32_t>(), vun.as<Piece>(), vk.as<uint64_t>(),
                                     vv.as<uint32_t>(), st),
                  "V pieces");
            alloc(vs, radix_sort_scratch_bytes(nv), "V piece sort");
            check(radix_sort_pairs(vk.as<uint64_t>(), vv.as<uint32_t>(), nv, bits, vs.p, st),
                  "V piece sort");
            vs.release();
            alloc(h->vpieces, (size_t)nv * sizeof(Piece), "sorted V pieces");
            alloc(vsz, (size_t)(nv + 1) * 8, "V piece sizes");
            alloc(vcl, (size_t)(nv + 1) * 8, "V piece columns");
            check(launch_vpiece_sizes(vun.as<Piece>(), vv.as<uint32_t>(), nv, h->vpieces.as<Piece>(),
                                      h->tile_lo.as<int32_t>(), h->Rv, vsz.as<int64_t>(),
                                      vcl.as<int64_t>(), st),
                  "V piece sizes");
            h->vtpool_entries = scan(vsz.as<int64_t>(), nv);
            h->ncols_v = scan(vcl.as<int64_t>(), nv);
            check(launch_vpiece_layout(h->vpieces.as<Piece>(), nv, vsz.as<int64_t>(), st),
                  "V piece layout");
            alloc(vptr, (h->ntiles + 1) * 8, "V tile ptr");
            check(launch_tile_offsets(vk.as<uint64_t>(), nv, h->ntiles, vptr.as<int64_t>(), st),
                  "V tile ptr");
            check(launch_tile_meta(vptr.as<int64_t>(), h->ntiles, nv, vcl.as<int64_t>(),
                                   vcl.as<int64_t>(), vsz.as<int64_t>(), vsz.as<int64_t>(),
                                   h->vt_meta.as<int64_t>(), st),
                  "V tile meta");
            alloc(h->vtpool, (size_t)std::max<int64_t>(h->vtpool_entries, 1) * ssz, "V pool");
            check(launch_vpiece_data(h->vpieces.as<Piece>(), nv, h->tile_lo.as<int32_t>(),
                                     h->adm.as<int4>(), vfo.as<int64_t>(), F.p, h->Rv,
                                     h->vtpool.p, smode, st),
                  "V pool");
            check(launch_pfc(h->vpieces.as<Piece>(), vv.as<uint32_t>(), vcl.as<int64_t>(), nv, nv,
                             vbase, h->pfc.as<int64_t>() + pfc_u, st),
                  "V source columns");
            check(hipStreamSynchronize(st), "V pool sync");
        } else {
            check(hipMemsetAsync(h->vt_meta.p, 0, (size_t)(h->ntiles + 1) * 4 * 8, st),
                  "V pool tile meta");
        }
        alloc(h->partial, (size_t)std::max<int64_t>(vbase + h->ncols_v, 1) * esz,
              "phase-1 partial sums");
        // per t entry: where its source pieces start in pfc, and how many
        if (h->n_adm > 0) {
            DevBuf sb, sn;
            alloc(sb, (size_t)h->n_adm * 8, "source bases");
            alloc(sn, (size_t)h->n_adm * 4, "source counts");
            check(launch_p1_source(h->n_adm, prt, cnt.as<int64_t>(), cntv.as<int64_t>(), pfc_u,
                                   sb.as<int64_t>(), sn.as<int32_t>(), st),
                  "phase-1 sources");
            alloc(h->p1rec, (size_t)std::max<int64_t>(h->sum_rank, 1) * sizeof(int4),
                  "phase-1 records");
            check(launch_p1_rec(h->rank.as<int32_t>(), h->toff.as<int64_t>(), sb.as<int64_t>(),
                                sn.as<int32_t>(), h->n_adm, h->p1rec.as<int4>(), st),
                  "phase-1 records");
        } else {
            alloc(h->p1rec, 16, "phase-1 records");
        }
        check(hipStreamSynchronize(st), "pool sync");
        F.release();
        if (keep)
            h->npool.swap(aca_keep);
        else
            alloc(h->npool, (size_t)std::max<int64_t>(h->npool_entries, 1) * h->nsz,
                  "near-field pool");
        if (h->nmode != 3)
            check(launch_piece_data(h->pieces.as<Piece>(), h->npieces, h->tile_lo.as<int32_t>(),
                                    h->adm.as<int4>(), h->dense.as<int4>(), nullptr, nullptr,
                                    f64 ? h->soa64.p : h->soa32.p, n, d,
                                    kernel_fn(h->kern, h->kd), h->upool.p, h->npool.p, smode,
                                    h->nmode, 2, st),
                  "piece data (near field)");
        check(hipStreamSynchronize(st), "near-field sync");
    }
    F.release();
    // near-field entry count (algorithmic, unpadded)
    if (h->n_dense > 0) {
        DevBuf ne;
        alloc(ne, (h->n_dense + 1) * 8, "near entries");
        check(launch_extent(h->dense.as<int4>(), h->n_dense, 2, 0, nullptr, nullptr,
                            ne.as<int64_t>(), st),
              "extent");
        h->near_entries = scan(ne.as<int64_t>(), h->n_dense);
    }
    S.phase_ms[5] = ms_since(t0);
    S.phase_ms[6] = 0.0;

    finish_stats(h, t_all);
}

void build_impl(hmx_hmatrix_s* h, const void* pts, int pts_f64, hipStream_t st) {
    const auto t_all = std::chrono::steady_clock::now();
    stage_partition(h, pts, pts_f64, st);
    AcaPlan plan = h->n_adm > 0 ? level_plan(h) : AcaPlan{};
    DevBuf rt;
    if (h->prm.rank_mode == HMX_RANK_LEARNED && h->n_adm > 0) {
        stage_predict(h, rt, st);
        plan.rt = rt.as<int32_t>();
    }
    stage_factors(h, plan, st, t_all);
}

// Many independent problems as one block-diagonal H-matrix.  Each problem's
// ordering, cluster tree and traversal run on its own points (bit for bit
// what a single build computes); the union then takes the problems' index
// ranges one after another: problem p owns [off_p, off_p + n_p).  Its
// coordinates are scaled by 1 / l_p (l the kernel's length: sqrt(p0) for the
// Gaussian, p0 for Matern-3/2) and padded to three dimensions with zeros,
// so phi with length 1 gives every problem its own kernel.  The admissible
// leaves of all problems are ordered upper-level class first, then the ACA,
// near field and matvec run once over the union.
// The partition of many problems at once (the forest of a batched build):
// the problems' points in one union index space, each problem ordered in its
// own box and clustered in its own tree, and one launch per step for all of
// them: boxes, Morton codes, the sort (by code, then stably by problem),
// every tree level, every box level, and every block-tree level of the
// traversal (one host readback per level for all problems).  Each problem's
// codes, permutation, clusters and leaves are those of its own build; the
// union leaf lists hold them level by level, problem by problem within a
// level, so each problem's leaves keep its canonical order.
void stage_forest(hmx_hmatrix_s* u, int np, const void* const* pts, int pts_f64,
                  const int64_t* n, const int32_t* d, const hmx_kernel* kern, hipStream_t st,
                  bool cross = false) {
    using clk = std::chrono::steady_clock;
    const int64_t N = u->n;
    const int leaf = u->prm.leaf_size;
    const double eta = u->prm.eta;
    hmx_stats& S = u->stats;
    auto t0 = clk::now();
    // per-problem tables (host and device): point offsets, tree depths and
    // slot offsets, dimensions, inverse kernel lengths, inputs
    std::vector<int64_t> pb(np + 1, 0), nb(np + 1, 0);
    std::vector<int32_t> dims(np), depth(np);
    std::vector<double> inv_ell(np);
    std::vector<ForestInput> in(np);
    int Lmax = 0;
    for (int p = 0; p < np; ++p) {
        pb[p + 1] = pb[p] + n[p];
        dims[p] = d[p];
        depth[p] = max_depth(n[p], leaf);
        if (depth[p] > 29) {
            set_err("problem %d: cluster tree too deep (%d levels); raise leaf_size", p,
                    depth[p]);
            throw Fail{HMX_ERR_UNSUPPORTED};
        }
        Lmax = std::max(Lmax, (int)depth[p]);
        nb[p + 1] = nb[p] + ((2ll << depth[p]) - 1);
        inv_ell[p] = 1.0 / kernel_length(kern[p]);
        in[p] = ForestInput{pts[p], d[p]};
    }
    const int64_t nslots = nb[np];
    if (nslots >= (1ll << 31)) {
        set_err("the problems' cluster trees need %lld slots (more than 2^31)",
                (long long)nslots);
        throw Fail{HMX_ERR_UNSUPPORTED};
    }
    DevBuf dpb, dnb, ddims, ddepth, dinv, din;
    alloc(dpb, (np + 1) * 8, "problem offsets");
    alloc(dnb, (np + 1) * 8, "problem slot offsets");
    alloc(ddims, np * 4, "problem dimensions");
    alloc(ddepth, np * 4, "problem tree depths");
    alloc(dinv, np * 8, "problem kernel scales");
    alloc(din, np * sizeof(ForestInput), "problem inputs");
    check(hipMemcpyAsync(dpb.p, pb.data(), (np + 1) * 8, hipMemcpyHostToDevice, st), "tables");
    check(hipMemcpyAsync(dnb.p, nb.data(), (np + 1) * 8, hipMemcpyHostToDevice, st), "tables");
    check(hipMemcpyAsync(ddims.p, dims.data(), np * 4, hipMemcpyHostToDevice, st), "tables");
    check(hipMemcpyAsync(ddepth.p, depth.data(), np * 4, hipMemcpyHostToDevice, st), "tables");
    check(hipMemcpyAsync(dinv.p, inv_ell.data(), np * 8, hipMemcpyHostToDevice, st), "tables");
    check(hipMemcpyAsync(din.p, in.data(), np * sizeof(ForestInput), hipMemcpyHostToDevice, st),
          "tables");
    const int64_t* PB = dpb.as<int64_t>();
    const int64_t* NB = dnb.as<int64_t>();

    // ---- 1. boxes, Morton codes, the sort, ordered coordinates ----
    DevBuf soa;  // unscaled Morton-ordered coordinates, 3 x N (partition and boxes)
    {
        DevBuf P, partial, box;
        alloc(P, (size_t)N * 3 * 8, "union points");
        check(launch_forest_points(din.as<ForestInput>(), np, PB, N, pts_f64, P.as<double>(), st),
              "union points");
        alloc(partial, (size_t)np * forest_box_parts() * 6 * 8, "box partials");
        alloc(box, (size_t)np * 6 * 8, "problem boxes");
        check(launch_forest_box(P.as<double>(), np, PB, ddims.as<int32_t>(),
                                partial.as<double>(), box.as<double>(), st),
              "problem boxes");
        std::vector<double> hb((size_t)np * 6);
        d2h(hb.data(), box.p, hb.size() * 8, st);
        for (int p = 0; p < np; ++p)
            for (int k = 0; k < d[p]; ++k)
                if (!std::isfinite(hb[6 * p + k]) || !std::isfinite(hb[6 * p + 3 + k])) {
                    set_err("problem %d: points contain NaN or infinite coordinates", p);
                    throw Fail{HMX_ERR_INVALID_ARG};
                }
        DevBuf C, keys, sscr;
        alloc(C, (size_t)N * 8, "union codes");
        alloc(keys, (size_t)N * 8, "sort keys");
        alloc(u->perm, (size_t)N * 4, "permutation");
        check(launch_forest_morton(P.as<double>(), N, np, PB, ddims.as<int32_t>(),
                                   box.as<double>(), C.as<uint64_t>(), u->perm.as<uint32_t>(), st),
              "morton");
        check(hipMemcpyAsync(keys.p, C.p, (size_t)N * 8, hipMemcpyDeviceToDevice, st), "keys");
        alloc(sscr, radix_sort_scratch_bytes(N), "sort scratch");
        check(radix_sort_pairs(keys.as<uint64_t>(), u->perm.as<uint32_t>(), N, 64, sscr.p, st),
              "radix sort");
        // stably by problem: every problem's points back in its own range
        int pbits = 1;
        while ((1ll << pbits) < np) ++pbits;
        check(launch_forest_problem_keys(u->perm.as<uint32_t>(), N, np, PB, keys.as<uint64_t>(),
                                         st),
              "problem keys");
        check(radix_sort_pairs(keys.as<uint64_t>(), u->perm.as<uint32_t>(), N, pbits, sscr.p, st),
              "problem sort");
        alloc(u->codes, (size_t)N * 8, "morton codes");
        check(launch_gather_u64(C.as<uint64_t>(), u->perm.as<uint32_t>(), N,
                                u->codes.as<uint64_t>(), st),
              "codes");
        alloc(soa, (size_t)N * 3 * 8, "ordered coordinates");
        check(launch_gather_coords(P.p, 1, N, 3, u->perm.as<uint32_t>(), soa.as<double>(),
                                   nullptr, st),
              "ordered coordinates");
        // the kernel's coordinates: each problem's divided by its kernel length
        alloc(u->soa64, (size_t)N * 3 * 8, "coords f64");
        if (!u->f64) alloc(u->soa32, (size_t)N * 3 * 4, "coords f32");
        check(launch_forest_scale(soa.as<double>(), N, np, PB, dinv.as<double>(),
                                  u->soa64.as<double>(), u->f64 ? nullptr : u->soa32.as<float>(),
                                  st),
              "scaled coordinates");
        check(hipStreamSynchronize(st), "order sync");
    }
    S.phase_ms[0] = ms_since(t0);
    t0 = clk::now();

    // ---- 2. every problem's cluster tree and boxes, level by level ----
    u->nslots = nslots;
    alloc(u->node_lo, nslots * 4, "node lo");
    alloc(u->node_hi, nslots * 4, "node hi");
    for (int l = 0; l <= Lmax; ++l)
        check(launch_forest_tree_level(l, np, PB, NB, ddepth.as<int32_t>(), leaf,
                                       u->node_lo.as<int32_t>(), u->node_hi.as<int32_t>(), st),
              "tree level");
    alloc(u->bmin, (size_t)nslots * 3 * 8, "box min");
    alloc(u->bmax, (size_t)nslots * 3 * 8, "box max");
    for (int l = Lmax; l >= 0; --l)
        check(launch_forest_box_level(l, np, NB, ddepth.as<int32_t>(), leaf,
                                      u->node_lo.as<int32_t>(), u->node_hi.as<int32_t>(),
                                      soa.as<double>(), N, u->bmin.as<double>(),
                                      u->bmax.as<double>(), st),
              "box level");
    soa.release();
    {
        alloc(u->tile_of_point, N * 4, "tile of point");
        check(hipMemsetAsync(u->tile_of_point.p, 0, N * 4, st), "memset");
        check(launch_mark_leaves(0, leaf, u->node_lo.as<int32_t>(), u->node_hi.as<int32_t>(),
                                 nslots, u->tile_of_point.as<int32_t>(), st),
              "mark leaves");
        DevBuf scratch, cnt;
        alloc(scratch, tile_scan_scratch_bytes(N), "tile scan");
        alloc(cnt, 8, "tile count");
        alloc(u->tile_lo, (size_t)(N + 1) * 4, "tile lo");
        check(launch_iota_scan_tiles(u->tile_of_point.as<int32_t>(), N, u->tile_lo.as<int32_t>(),
                                     cnt.as<int64_t>(), scratch.p, st),
              "tile scan");
        u->ntiles = read_scalar(cnt.as<int64_t>(), st);
        u->ntiles_rows = u->ntiles;
        if (cross) {  // the row tiles: the leaf clusters of the first point set
            std::vector<int32_t> tl(u->ntiles + 1);
            d2h(tl.data(), u->tile_lo.p, tl.size() * 4, st);
            u->ntiles_rows = std::lower_bound(tl.begin(), tl.end() - 1, (int32_t)n[0]) - tl.begin();
        }
    }
    u->max_tile = 0;
    for (int p = 0; p < np; ++p) {
        int64_t sz = n[p];
        while (sz > leaf) sz = (sz + 1) / 2;
        u->max_tile = std::max(u->max_tile, (int)sz);
    }
    S.phase_ms[1] = ms_since(t0);
    t0 = clk::now();

    // ---- 3. the block cluster trees, one level of all of them at a time ----
    {
        DevBuf sbase, cur, nxt, scratch, totals;
        alloc(sbase, nslots * 4, "slot bases");
        check(launch_forest_slot_base(NB, np, nslots, sbase.as<int32_t>(), st), "slot bases");
        // one root block per problem, or (two point sets) the one block of
        // the first set's root by the second set's root
        std::vector<int2> roots;
        if (cross)
            roots.push_back(make_int2((int)nb[0], (int)nb[1]));
        else
            for (int p = 0; p < np; ++p) roots.push_back(make_int2((int)nb[p], (int)nb[p]));
        alloc(cur, roots.size() * sizeof(int2), "level 0");
        check(hipMemcpyAsync(cur.p, roots.data(), roots.size() * sizeof(int2),
                             hipMemcpyHostToDevice, st),
              "roots");
        alloc(totals, 8 * sizeof(int64_t), "totals");
        int64_t ncur = (int64_t)roots.size();
        int level = 0;
        int64_t cap_adm = 0, cap_dense = 0;
        while (ncur > 0) {
            if (level >= 64) {
                set_err("block tree deeper than 64 levels");
                throw Fail{HMX_ERR_UNSUPPORTED};
            }
            S.level_sizes[level] = ncur;
            const int64_t nblk = traverse_blocks(ncur);
            if (!scratch.p || scratch.bytes < traverse_scratch_bytes(ncur))
                alloc(scratch, traverse_scratch_bytes(ncur), "traverse scratch");
            int64_t* bc = scratch.as<int64_t>();
            check(launch_traverse_count(cur.as<int2>(), ncur, u->node_lo.as<int32_t>(),
                                        u->node_hi.as<int32_t>(), u->bmin.as<double>(),
                                        u->bmax.as<double>(), 3, leaf, eta, bc, st),
                  "traverse count");
            check(launch_traverse_scan(bc, nblk, totals.as<int64_t>(), st), "traverse scan");
            int64_t tot[3];
            check(hipMemcpyAsync(tot, totals.p, 3 * 8, hipMemcpyDeviceToHost, st), "totals");
            check(hipStreamSynchronize(st), "level sync");
            if (u->n_adm + tot[0] > cap_adm) {
                int64_t nc = std::max<int64_t>(2 * cap_adm, u->n_adm + tot[0]);
                grow(u->adm, nc * sizeof(int4), u->n_adm * sizeof(int4), st, "adm leaves");
                grow(u->adm_level, nc * 4, u->n_adm * 4, st, "adm levels");
                grow(u->adm_ids, nc * sizeof(int2), u->n_adm * sizeof(int2), st, "adm node ids");
                cap_adm = nc;
            }
            if (u->n_dense + tot[2] > cap_dense) {
                int64_t nc = std::max<int64_t>(2 * cap_dense, u->n_dense + tot[2]);
                grow(u->dense, nc * sizeof(int4), u->n_dense * sizeof(int4), st, "dense leaves");
                grow(u->dense_level, nc * 4, u->n_dense * 4, st, "dense levels");
                cap_dense = nc;
            }
            const int64_t nnext = 4 * tot[1];
            alloc(nxt, std::max<int64_t>(nnext, 1) * sizeof(int2), "next level");
            check(launch_traverse_write(cur.as<int2>(), ncur, u->node_lo.as<int32_t>(),
                                        u->node_hi.as<int32_t>(), u->bmin.as<double>(),
                                        u->bmax.as<double>(), 3, leaf, eta, bc, level,
                                        nxt.as<int2>(), u->adm.as<int4>(),
                                        u->adm_level.as<int32_t>(), u->adm_ids.as<int2>(),
                                        u->n_adm, u->dense.as<int4>(),
                                        u->dense_level.as<int32_t>(), u->n_dense,
                                        sbase.as<int32_t>(), st),
                  "traverse write");
            u->n_adm += tot[0];
            u->n_dense += tot[2];
            cur.swap(nxt);
            ncur = nnext;
            ++level;
        }
        check(hipStreamSynchronize(st), "traverse sync");
        S.levels = level;
    }
    if (!u->adm.p) alloc(u->adm, sizeof(int4), "adm leaves");
    if (!u->adm_level.p) alloc(u->adm_level, 4, "adm levels");
    if (!u->adm_ids.p) alloc(u->adm_ids, sizeof(int2), "adm node ids");
    if (!u->dense.p) alloc(u->dense, sizeof(int4), "dense leaves");
    if (!u->dense_level.p) alloc(u->dense_level, 4, "dense levels");
    S.phase_ms[2] = ms_since(t0);
    u->offsets.assign(pb.begin(), pb.end());
}

void batched_impl(hmx_hmatrix_s* u, int np, const void* const* pts, int pts_f64,
                  const int64_t* n, const int32_t* d, const hmx_kernel* kern, hipStream_t st,
                  bool cross = false) {
    const auto t_all = std::chrono::steady_clock::now();
    const bool learned = u->prm.rank_mode == HMX_RANK_LEARNED;
    stage_forest(u, np, pts, pts_f64, n, d, kern, st, cross);
    const int64_t nadm = u->n_adm;
    AcaPlan plan;
    DevBuf cls, rt;
    if (nadm > 0) {
        // size classes: each leaf's from its problem's level cuts; the leaves
        // stably grouped by class (each problem's leaves keep their order)
        std::vector<int4> cuts(np);
        // (two point sets: a block's clusters at level l hold at most
        // ceil(max(n_1, n_2) / 2^l) points on either side)
        const int64_t nmax = cross ? std::max(n[0], n[1]) : 0;
        for (int p = 0; p < np; ++p)
            cuts[p] = level_cuts(cross ? nmax : n[p], split_rows(u), nullptr, nullptr, nullptr);
        std::vector<int64_t> pb(u->offsets);
        DevBuf dcuts, dpb, keys, vals, sscr, big;
        alloc(dcuts, np * sizeof(int4), "class cuts");
        alloc(dpb, (np + 1) * 8, "problem offsets");
        check(hipMemcpyAsync(dcuts.p, cuts.data(), np * sizeof(int4), hipMemcpyHostToDevice, st),
              "class cuts");
        check(hipMemcpyAsync(dpb.p, pb.data(), (np + 1) * 8, hipMemcpyHostToDevice, st),
              "problem offsets");
        alloc(keys, nadm * 8, "class keys");
        alloc(vals, nadm * 4, "class order");
        check(launch_forest_class(u->adm.as<int4>(), u->adm_level.as<int32_t>(), nadm, np,
                                  dpb.as<int64_t>(), dcuts.as<int4>(), keys.as<uint64_t>(),
                                  vals.as<uint32_t>(), st),
              "classes");
        alloc(sscr, radix_sort_scratch_bytes(nadm), "class sort");
        check(radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(), nadm, 2, sscr.p, st),
              "class sort");
        DevBuf a2, l2, i2;
        alloc(a2, nadm * sizeof(int4), "adm leaves");
        alloc(l2, nadm * 4, "adm levels");
        alloc(i2, nadm * sizeof(int2), "adm node ids");
        alloc(cls, nadm * 4, "size classes");
        check(launch_gather_blocks(vals.as<uint32_t>(), nadm, u->adm.as<int4>(),
                                   u->adm_level.as<int32_t>(), nullptr, nullptr, a2.as<int4>(),
                                   l2.as<int32_t>(), nullptr, nullptr, st),
              "class gather");
        check(launch_gather_u64((const uint64_t*)u->adm_ids.p, vals.as<uint32_t>(), nadm,
                                (uint64_t*)i2.p, st),
              "class gather");
        check(launch_narrow_u64(keys.as<uint64_t>(), nadm, cls.as<int32_t>(), st), "classes");
        u->adm.swap(a2);
        u->adm_level.swap(l2);
        u->adm_ids.swap(i2);
        // the largest cluster side of an admissible leaf
        alloc(big, 8, "largest block side");
        check(hipMemsetAsync(big.p, 0, 8, st), "largest block side");
        check(launch_max_side(u->adm.as<int4>(), nadm, big.as<int>(), st), "largest block side");
        u->big_adm = read_scalar(big.as<int>(), st);
        if (learned) {
            alloc(rt, nadm * 4, "rank targets");
            std::vector<double> ell(np);
            std::vector<int32_t> dd(np);
            for (int p = 0; p < np; ++p) {
                ell[p] = kernel_length(kern[p]);
                dd[p] = d[p];
            }
            DevBuf dell, ddim;
            alloc(dell, np * 8, "problem lengths");
            alloc(ddim, np * 4, "problem dimensions");
            check(hipMemcpyAsync(dell.p, ell.data(), np * 8, hipMemcpyHostToDevice, st), "lengths");
            check(hipMemcpyAsync(ddim.p, dd.data(), np * 4, hipMemcpyHostToDevice, st),
                  "dimensions");
            const auto tp = std::chrono::steady_clock::now();
            const hmx_mlp_s* mp = u->prm.mlp;
            check(launch_rank_predict(u->adm.as<int4>(), u->adm_ids.as<int2>(), nadm,
                                      u->bmin.as<double>(), u->bmax.as<double>(), 3, 1.0,
                                      mp->w.as<float>(), mp->mean.as<float>(),
                                      mp->scale.as<float>(), u->prm.max_rank, nullptr,
                                      rt.as<int32_t>(), st, dpb.as<int64_t>(), np,
                                      dell.as<double>(), ddim.as<int32_t>()),
                  "rank prediction");
            check(hipStreamSynchronize(st), "prediction sync");
            u->stats.predict_ms += ms_since(tp);
        }
        check(hipStreamSynchronize(st), "class sync");
        const int64_t big_rows = u->big_adm;
        const int64_t words = 2 * ((big_rows + 31) / 32);
        if (words * 4 > 64 * 1024) {
            set_err("admissible block of %lld rows exceeds the ACA bitmask capacity",
                    (long long)big_rows);
            throw Fail{HMX_ERR_UNSUPPORTED};
        }
        plan.cls = cls.as<int32_t>();
        plan.split0 = 1;
        plan.split = 2;
        plan.split2 = 3;
        plan.big_words = (int)std::max<int64_t>(words, 2);
        plan.med_words =
            (int)std::max<int64_t>(2 * ((std::min(kBigRows - 1, big_rows) + 31) / 32), 2);
        plan.tiny_words =
            (int)std::max<int64_t>(2 * ((std::min(kTinyRows, big_rows) + 31) / 32), 2);
        plan.rt = learned ? rt.as<int32_t>() : nullptr;
    }
    stage_factors(u, plan, st, t_all);
}

}  // namespace


namespace {

const int64_t kP = HMX_MLP_NPARAMS;
// predictor file: magic, then int64 parameter count and Adam step, then FP32
// parameters, standardisation mean and scale, Adam moments m and v
const char kMlpMagic[8] = {'H', 'M', 'X', 'M', 'L', 'P', '0', '1'};

template <typename F>
hmx_status guarded(F&& f) {
    try {
        f();
    } catch (const Fail& e) {
        return e.s;
    } catch (const std::bad_alloc&) {
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    return HMX_OK;
}

// grow a work buffer without keeping its contents (the stream is synchronised
// first: the old block may still be in use by queued work)
void ensure(DevBuf& b, size_t bytes, hipStream_t st, const char* what) {
    if (b.p && b.bytes >= bytes) return;
    check(hipStreamSynchronize(st), "work buffer sync");
    alloc(b, bytes, what);
}

// argument checks shared by hmx_matvec and hmx_matvec_graph
hmx_status matvec_args(hmx_hmatrix_s* h, const void* x, const void* z, hmx_dtype vec_dtype) {
    if (!h || !x || !z) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    if ((vec_dtype == HMX_F64) != (h->f64 == 1) || vec_dtype == HMX_BF16) {
        set_err("vector dtype must equal the compute dtype");
        return HMX_ERR_INVALID_ARG;
    }
    if (h->prm.aca_only) {
        set_err("handle was built with aca_only: no matrix to apply");
        return HMX_ERR_UNSUPPORTED;
    }
    return HMX_OK;
}

// phase 1's tile passes (t = V^T x partial sums per row tile): the factor
// pool (symmetric far field) and the V pool
hipError_t p1_tiles(hmx_hmatrix_s* h, hipStream_t st, int lanes) {
    hipError_t e = hipSuccess;
    if (h->sym && h->ncols_u > 0)
        e = launch_p1_tile(h->ntiles, h->tile_lo.as<int32_t>(), h->tile_meta.as<int64_t>(), 4,
                           h->Ru, h->max_tile, h->upool.p, h->vecpool.p, h->partial.p, 0,
                           h->smode, lanes, st);
    if (e == hipSuccess && h->ncols_v > 0)
        e = launch_p1_tile(h->ntiles, h->tile_lo.as<int32_t>(), h->vt_meta.as<int64_t>(), 4,
                           h->Rv, h->max_tile, h->vtpool.p, h->vecpool.p, h->partial.p,
                           h->sym ? h->ncols_u : 0, h->smode, lanes, st);
    return e;
}

// the three launches of one matvec: gather of x into Morton order, far-field
// phase 1 (t = V^T x), row tiles (near field + U t, scatter to z); ev: four
// events recorded around them, or null
hipError_t matvec_launch(hmx_hmatrix_s* h, const void* x, void* z, double alpha, double beta,
                         hipStream_t st, hipEvent_t* ev, int config) {
    const int f64 = h->f64;
    hipError_t e = ev ? hipEventRecord(ev[0], st) : hipSuccess;
    if (e == hipSuccess)
        e = launch_gather_x(x, h->perm.as<int32_t>() + h->col0, h->ncols,
                            (char*)h->vecpool.p + (size_t)h->col0 * h->esz, f64, st, h->col0);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], st);
    // phase 1 by row tiles: partial sums of every source column, then the t
    // entries; the sources are the factor pool (symmetric far field) and the V pool
    if (e == hipSuccess) e = p1_tiles(h, st, h->p1_lanes);
    if (e == hipSuccess)
        e = launch_p1_reduce(h->p1rec.as<int4>(), h->sum_rank, h->pfc.as<int64_t>(),
                             h->partial.p, h->vecpool.p, h->n, f64, st);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], st);
    if (e == hipSuccess)
        e = launch_rowtile(h->ntiles_rows, h->tile_lo.as<int32_t>(), h->tile_meta.as<int64_t>(),
                           h->widx.as<int64_t>(), h->upool.p, h->npool.p, h->vecpool.p,
                           h->perm.as<int32_t>(), alpha, beta, h->prm.sigma2, z, h->max_tile,
                           h->smode, h->nmode, config, f64 ? h->soa64.p : h->soa32.p, h->n, h->d,
                           kernel_fn(h->kern, h->kd), st);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], st);
    return e;
}


// A matvec without precomputed factors: the near field (and sigma2 x, beta z)
// by the row tiles, then chunk by chunk the ACA of the chunk's blocks into
// the column scratch, t = V^T x per block and z|tile += alpha U t per row
// tile, then the ranks back to the leaves.  Synchronises st.
void np_matvec(hmx_hmatrix_s* h, const void* x, void* z, double alpha, double beta,
               hipStream_t st, hipEvent_t* ev) {
    const int f64 = h->f64;
    const size_t esz = h->esz;
    const int kmax = h->prm.max_rank;
    NpPlan& P = h->np;
    if (ev) check(hipEventRecord(ev[0], st), "event");
    check(matvec_launch(h, x, z, alpha, beta, st, nullptr, h->rt_config), "matvec (near field)");
    if (ev) check(hipEventRecord(ev[1], st), "event");
    if (P.nl > 0) {
        AcaPlan plan{};
        plan.big_words = P.big_words;
        plan.med_words = P.med_words;
        plan.tiny_words = P.tiny_words;
        DevBuf Ucap, tb, t2b;
        const int64_t ucols = (std::max<int64_t>(P.max_u, 1) + 63) / 64 * 64;
        alloc(Ucap, (size_t)(ucols + std::max<int64_t>(P.max_v, 1)) * esz, "ACA chunk scratch");
        void* const vcap = (char*)Ucap.p + (size_t)ucols * esz;
        alloc(tb, (size_t)std::max<int64_t>(P.max_nb, 1) * kmax * esz, "chunk t");
        if (h->sym) alloc(t2b, (size_t)std::max<int64_t>(P.max_nb, 1) * kmax * esz, "chunk t'");
        AuxStream auxs[3];
        const hipStream_t aux[3] = {auxs[0].s, auxs[1].s, auxs[2].s};
        const bool have_aux = aux[0] && aux[1] && aux[2];
        AcaArgs a = aca_args_base(h, plan);
        a.U = Ucap.p;
        a.V = vcap;
        const int4* B = P.blocks.as<int4>();
        const int64_t* cu = P.cu.as<int64_t>();
        const int64_t* cv = P.cv.as<int64_t>();
        int32_t* rank = P.rank.as<int32_t>();
        const int nch = (int)P.bounds.size() - 1;
        for (int k = 0; k < nch; ++k) {
            const int64_t b0 = P.bounds[k], nbk = P.bounds[k + 1] - b0;
            if (nbk == 0) continue;
            a.blocks = B + b0;
            a.nblocks = nbk;
            a.uoff = cu + b0;
            a.voff = cv + b0;
            a.ubase = P.hcu[k];
            a.vbase = P.hcv[k];
            a.rank = rank + b0;
            a.steps = P.steps.as<int32_t>() + b0;
            a.nsplit = P.cls[3 * k];
            a.nbig = P.cls[3 * k + 1];
            a.nmed = P.cls[3 * k + 2];
            SplitBuffers sb;
            if (a.nsplit > 0) prepare_split(h, a, f64, st, sb);
            check(aca_classes_begin(a, f64, st, have_aux ? aux : nullptr), "aca");
            if (a.nsplit > 0)
                check(launch_aca_split(a, sb.P, f64, st), "aca (many workgroups per block)");
            check(aca_classes_join(st, have_aux ? aux : nullptr), "aca join");
            check(launch_np_t(B + b0, nbk, rank + b0, cu + b0, cv + b0, P.hcu[k], P.hcv[k], Ucap.p,
                              vcap, h->vecpool.p, kmax, h->sym, tb.p, h->sym ? t2b.p : nullptr,
                              f64, st),
                  "far field t");
            check(launch_np_apply(P.seg_start.as<int64_t>(), P.seg_tile.as<int32_t>(), P.cseg[k],
                                  P.cseg[k + 1] - P.cseg[k], P.spcs.as<int2>(), B, rank, cu, cv,
                                  P.hcu[k], P.hcv[k], b0, Ucap.p, vcap, tb.p,
                                  h->sym ? t2b.p : nullptr, kmax, h->tile_lo.as<int32_t>(),
                                  h->perm.as<int32_t>(), alpha, z, h->max_tile, f64, st),
                  "far field apply");
            if (a.nsplit > 0) check(hipStreamSynchronize(st), "chunk sync");  // sb returns
        }
        if (ev) check(hipEventRecord(ev[2], st), "event");
        // the ranks of this product back to the leaves (a mirror takes its
        // primary's), and their statistics
        check(launch_scatter_list(P.lmap.as<int32_t>(), P.nl,
                                  h->sym ? h->partner.as<int32_t>() : nullptr, rank,
                                  P.steps.as<int32_t>(), nullptr, nullptr,
                                  h->rank.as<int32_t>(), h->steps.as<int32_t>(), nullptr, nullptr,
                                  st),
              "ranks");
        DevBuf red;
        alloc(red, 2 * sizeof(unsigned long long), "stats");
        check(launch_int_stats(h->rank.as<int32_t>(), h->n_adm, red.as<unsigned long long>(), st),
              "rank stats");
        unsigned long long hv[2];
        check(hipMemcpyAsync(hv, red.p, sizeof hv, hipMemcpyDeviceToHost, st), "stats readback");
        if (ev) check(hipEventRecord(ev[3], st), "event");
        check(hipStreamSynchronize(st), "matvec sync");  // before the scratch returns
        h->stats.max_rank_used = (int32_t)hv[0];
        h->stats.sum_rank = (int64_t)hv[1];
    } else if (ev) {
        check(hipEventRecord(ev[2], st), "event");
        check(hipEventRecord(ev[3], st), "event");
    }
}

// Work space of a CG solve: three n-vectors in the compute type, 8 FP64
// scalars (r.r, p.q, r'.r', b.b, |b - (H + sigma2 I) x|^2) and the dot
// products' block partials.
struct CgWork {
    void *r, *p, *q;
    double* sc;
    double* pa;
};

constexpr size_t kCgScalBytes = 256;

size_t cg_vec_bytes(int64_t n, size_t esz) { return ((size_t)n * esz + 255) / 256 * 256; }

hmx_status cg_args(hmx_hmatrix_s* h, const void* b, const void* x, double rel_tol,
                   int32_t max_iter) {
    if (!h || !b || !x || !(rel_tol >= 0) || max_iter < 0) {
        set_err("invalid argument to the CG solve");
        return HMX_ERR_INVALID_ARG;
    }
    if (h->prm.aca_only) {
        set_err("handle was built with aca_only: no matrix to apply");
        return HMX_ERR_UNSUPPORTED;
    }
    if (h->rect) {
        set_err("a rectangular handle has no linear system to solve");
        return HMX_ERR_UNSUPPORTED;
    }
    return HMX_OK;
}

// Textbook CG (Hestenes-Stiefel) from x = 0 on (H + sigma2 I); every buffer
// of w is overwritten before it is read, so leftover contents do not matter.
hmx_status cg_run(hmx_hmatrix_s* h, const void* b, void* x, double rel_tol, int32_t max_iter,
                  hipStream_t st, const CgWork& w, int32_t* iters, double* rel_res,
                  double* true_rel_res) {
    const int f64 = h->f64;
    const int64_t n = h->n;
    const hmx_dtype vdt = f64 ? HMX_F64 : HMX_F32;
    int32_t it = 0;
    double rr = 0.0, bb = 0.0, res = 0.0;
    hmx_status status = HMX_OK;
    double* sc = w.sc;
    double* pa = w.pa;
    check(launch_fill_zero(x, n, f64, st), "cg init");
    check(launch_copy(w.r, b, n, f64, st), "cg init");
    check(launch_copy(w.p, b, n, f64, st), "cg init");
    check(launch_dot(b, b, n, f64, pa, sc + 3, st), "cg dot");
    check(launch_copy(sc, sc + 3, 1, 1, st), "cg init");  // r.r = b.b
    check(hipMemcpyAsync(&bb, sc + 3, 8, hipMemcpyDeviceToHost, st), "cg readback");
    check(hipStreamSynchronize(st), "cg sync");
    rr = bb;
    if (bb == 0.0) {
        if (iters) *iters = 0;
        if (rel_res) *rel_res = 0.0;
        if (true_rel_res) *true_rel_res = 0.0;
        return HMX_OK;
    }
    res = 1.0;
    status = HMX_ERR_NOT_CONVERGED;
    while (it < max_iter) {
        hmx_status s = hmx_matvec(h, w.p, w.q, vdt, 1.0, 0.0, st);
        if (s != HMX_OK) return s;
        check(launch_dot(w.p, w.q, n, f64, pa, sc + 1, st), "cg dot");
        check(launch_cg_update(x, w.r, w.p, w.q, sc, n, f64, pa, sc + 2, st), "cg update");
        double two[2];
        check(hipMemcpyAsync(two, sc + 1, 16, hipMemcpyDeviceToHost, st), "cg readback");
        check(hipStreamSynchronize(st), "cg sync");
        ++it;
        if (!(two[0] > 0.0)) {
            set_err("CG breakdown at iteration %d: p.Ap = %g", it, two[0]);
            break;  // the step was not taken: x is the last iterate; not converged
        }
        rr = two[1];
        res = sqrt(rr / bb);
        if (res <= rel_tol) {
            status = HMX_OK;
            break;
        }
        check(launch_cg_direction(w.p, w.r, sc, n, f64, st), "cg direction");
        check(launch_copy(sc, sc + 2, 1, 1, st), "cg shift");
    }
    if (status != HMX_OK && it >= max_iter) set_err("CG did not converge in %d iterations", it);
    if (true_rel_res) {
        // r = b - (H + sigma2 I) x
        hmx_status s = hmx_matvec(h, x, w.q, vdt, 1.0, 0.0, st);
        if (s != HMX_OK) return s;
        check(launch_sub(w.r, b, w.q, n, f64, st), "cg residual");
        check(launch_dot(w.r, w.r, n, f64, pa, sc + 4, st), "cg residual");
        double d2 = 0.0;
        check(hipMemcpyAsync(&d2, sc + 4, 8, hipMemcpyDeviceToHost, st), "cg readback");
        check(hipStreamSynchronize(st), "cg sync");
        *true_rel_res = sqrt(d2 / bb);
    }
    if (iters) *iters = it;
    if (rel_res) *rel_res = res;
    return status;
}

// Fixed work space of hmx_cg_solve_noalloc.  In host code `cg_scratch` names
// a host-side stand-in, not the device array: its device address is looked up
// once per device (hipGetSymbolAddress) and only that address is used.
__device__ __align__(256) unsigned char cg_scratch[HMX_CG_NOALLOC_MAX_BYTES];

std::mutex g_cg_scratch_mu;
void* g_cg_scratch_dev[64] = {};

void* cg_scratch_device() {
    int dev = 0;
    check(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= 64) {
        set_err("device ordinal %d out of range", dev);
        throw Fail{HMX_ERR_DEVICE};
    }
    std::lock_guard<std::mutex> lk(g_cg_scratch_mu);
    if (!g_cg_scratch_dev[dev]) {
        void* ptr = nullptr;
        check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(cg_scratch)), "hipGetSymbolAddress(cg_scratch)");
        g_cg_scratch_dev[dev] = ptr;
    }
    return g_cg_scratch_dev[dev];
}
}  // namespace

extern "C" {

const char* hmx_status_string(hmx_status s) {
    switch (s) {
        case HMX_OK: return "ok";
        case HMX_ERR_INVALID_ARG: return "invalid argument";
        case HMX_ERR_OOM: return "out of device memory";
        case HMX_ERR_DEVICE: return "device error";
        case HMX_ERR_NOT_CONVERGED: return "not converged";
        case HMX_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* hmx_last_error(void) { return g_err.c_str(); }

hmx_status hmx_params_default(hmx_params* p) {
    if (!p) {
        set_err("params is NULL");
        return HMX_ERR_INVALID_ARG;
    }
    memset(p, 0, sizeof *p);
    p->leaf_size = 256;
    p->eta = 1.5;
    p->aca_eps = 1e-5;
    p->aca_eta = 0.0;
    p->aca_eps0 = -1.0;
    p->max_rank = 64;
    p->sigma2 = 0.0;
    p->compute_dtype = HMX_F32;
    p->storage_dtype = HMX_F32;
    p->near_dtype = HMX_F32;
    p->rank_mode = HMX_RANK_ADAPTIVE;
    return HMX_OK;
}

hmx_status hmx_build(const void* points, hmx_dtype pts_dtype, int64_t n, int32_t d,
                     const hmx_kernel* kernel, const hmx_params* params, void* stream,
                     hmx_hmatrix* out) {
    if (out) *out = nullptr;
    if (!out || !points || !kernel || !params) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    if (n < 1 || n >= (1ll << 31)) {
        set_err("n = %lld out of range [1, 2^31)", (long long)n);
        return HMX_ERR_INVALID_ARG;
    }
    if (d < 1 || d > 3) {
        set_err("d = %d not in {1,2,3}", d);
        return HMX_ERR_INVALID_ARG;
    }
    if (pts_dtype != HMX_F64 && pts_dtype != HMX_F32) {
        set_err("points must be F64 or F32");
        return HMX_ERR_INVALID_ARG;
    }
    const hmx_params& p = *params;
    {
        const hmx_status ps = check_params(p);
        if (ps != HMX_OK) return ps;
    }
    if (kernel->kind != HMX_GAUSSIAN && kernel->kind != HMX_MATERN32 &&
        kernel->kind != HMX_MATERN_NU1 && kernel->kind != HMX_TEST_CONST &&
        kernel->kind != HMX_TEST_LOWRANK) {
        set_err("unknown kernel kind %d", (int)kernel->kind);
        return HMX_ERR_INVALID_ARG;
    }
    if ((kernel->kind == HMX_GAUSSIAN || kernel->kind == HMX_MATERN32 ||
         kernel->kind == HMX_MATERN_NU1) &&
        !(kernel->p0 > 0 && std::isfinite(kernel->p0))) {
        set_err("kernel parameter p0 must be positive and finite");
        return HMX_ERR_INVALID_ARG;
    }
    hmx_hmatrix_s* h = new (std::nothrow) hmx_hmatrix_s();
    if (!h) {
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    init_handle(h, n, d, *kernel, p);
    const Allocator ua{p.dev_alloc, p.dev_free, p.alloc_ctx};
    AllocScope scope(&ua);
    try {
        build_impl(h, points, pts_dtype == HMX_F64, (hipStream_t)stream);
    } catch (const Fail& f) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        (void)hipGetLastError();
        delete h;
        return f.s;
    } catch (const std::bad_alloc&) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        delete h;
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    *out = h;
    return HMX_OK;
}

hmx_status hmx_build_batched(int32_t nprob, const void* const* points, hmx_dtype pts_dtype,
                             const int64_t* n, const int32_t* d, const hmx_kernel* kernels,
                             const hmx_params* params, void* stream, hmx_hmatrix* out) {
    if (out) *out = nullptr;
    if (!out || !points || !n || !d || !kernels || !params || nprob < 1) {
        set_err("NULL argument or nprob < 1");
        return HMX_ERR_INVALID_ARG;
    }
    if (pts_dtype != HMX_F64 && pts_dtype != HMX_F32) {
        set_err("points must be F64 or F32");
        return HMX_ERR_INVALID_ARG;
    }
    const hmx_params& p = *params;
    {
        const hmx_status ps = check_params(p);
        if (ps != HMX_OK) return ps;
    }
    const hmx_kernel_kind kind = kernels[0].kind;
    if (kind != HMX_GAUSSIAN && kind != HMX_MATERN32) {
        set_err("batched build supports the Gaussian and Matern-3/2 kernels");
        return HMX_ERR_UNSUPPORTED;
    }
    int64_t total = 0;
    for (int32_t q = 0; q < nprob; ++q) {
        if (!points[q] || n[q] < 1 || d[q] < 1 || d[q] > 3) {
            set_err("problem %d: NULL points, n < 1 or d not in {1,2,3}", q);
            return HMX_ERR_INVALID_ARG;
        }
        if (kernels[q].kind != kind) {
            set_err("problem %d: all problems of a batch need the same kernel kind", q);
            return HMX_ERR_INVALID_ARG;
        }
        if (!(kernels[q].p0 > 0 && std::isfinite(kernels[q].p0))) {
            set_err("problem %d: kernel parameter p0 must be positive and finite", q);
            return HMX_ERR_INVALID_ARG;
        }
        total += n[q];
    }
    if (total >= (1ll << 31)) {
        set_err("total points %lld exceed 2^31 - 1", (long long)total);
        return HMX_ERR_INVALID_ARG;
    }
    hmx_hmatrix_s* h = new (std::nothrow) hmx_hmatrix_s();
    if (!h) {
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    init_handle(h, total, 3, hmx_kernel{kind, 1.0, 0.0}, p);
    h->nprob = nprob;
    h->batched = true;
    const Allocator ua{p.dev_alloc, p.dev_free, p.alloc_ctx};
    AllocScope scope(&ua);
    try {
        batched_impl(h, nprob, points, pts_dtype == HMX_F64, n, d, kernels, (hipStream_t)stream);
    } catch (const Fail& f) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        (void)hipGetLastError();
        delete h;
        return f.s;
    } catch (const std::bad_alloc&) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        delete h;
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    *out = h;
    return HMX_OK;
}

hmx_status hmx_build_rect(const void* rows, int64_t n1, const void* cols, int64_t n2,
                          hmx_dtype pts_dtype, int32_t d, const hmx_kernel* kernel,
                          const hmx_params* params, void* stream, hmx_hmatrix* out) {
    if (out) *out = nullptr;
    if (!out || !rows || !cols || !kernel || !params || n1 < 1 || n2 < 1 || d < 1 || d > 3) {
        set_err("NULL argument, n1 < 1, n2 < 1 or d not in {1,2,3}");
        return HMX_ERR_INVALID_ARG;
    }
    if (pts_dtype != HMX_F64 && pts_dtype != HMX_F32) {
        set_err("points must be F64 or F32");
        return HMX_ERR_INVALID_ARG;
    }
    if (n1 + n2 >= (1ll << 31)) {
        set_err("n1 + n2 = %lld exceeds 2^31 - 1", (long long)(n1 + n2));
        return HMX_ERR_INVALID_ARG;
    }
    const hmx_params& p = *params;
    {
        const hmx_status ps = check_params(p);
        if (ps != HMX_OK) return ps;
    }
    if (p.sigma2 != 0.0 || p.symmetric_far) {
        set_err("a rectangular matrix takes no diagonal shift and has no mirror blocks "
                "(sigma2 = 0, symmetric_far = 0)");
        return HMX_ERR_INVALID_ARG;
    }
    const hmx_kernel_kind kind = kernel->kind;
    if (kind != HMX_GAUSSIAN && kind != HMX_MATERN32 && kind != HMX_MATERN_NU1) {
        set_err("rectangular build supports the Gaussian and Matern kernels");
        return HMX_ERR_UNSUPPORTED;
    }
    if (!(kernel->p0 > 0 && std::isfinite(kernel->p0))) {
        set_err("kernel parameter p0 must be positive and finite");
        return HMX_ERR_INVALID_ARG;
    }
    hmx_hmatrix_s* h = new (std::nothrow) hmx_hmatrix_s();
    if (!h) {
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    // the two sets as a forest of two trees (each ordered in its own box,
    // coordinates divided by the kernel length), traversed from the one root
    // block Y1 x Y2
    init_handle(h, n1 + n2, 3, hmx_kernel{kind, 1.0, 0.0}, p);
    h->kd = d;
    h->nprob = 2;
    h->batched = true;
    h->rect = true;
    h->nrows = n1;
    h->ncols = n2;
    h->col0 = n1;
    const void* pts[2] = {rows, cols};
    const int64_t nn[2] = {n1, n2};
    const int32_t dd[2] = {d, d};
    const hmx_kernel kk[2] = {*kernel, *kernel};
    const Allocator ua{p.dev_alloc, p.dev_free, p.alloc_ctx};
    AllocScope scope(&ua);
    try {
        batched_impl(h, 2, pts, pts_dtype == HMX_F64, nn, dd, kk, (hipStream_t)stream, true);
    } catch (const Fail& f) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        (void)hipGetLastError();
        delete h;
        return f.s;
    } catch (const std::bad_alloc&) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        delete h;
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    *out = h;
    return HMX_OK;
}

hmx_status hmx_get_batch(hmx_hmatrix h, int32_t* nprob, int64_t* offsets) {
    if (!h || !nprob) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    *nprob = h->nprob;
    if (offsets) {
        if (h->batched)
            for (int32_t q = 0; q <= h->nprob; ++q) offsets[q] = h->offsets[q];
        else {
            offsets[0] = 0;
            offsets[1] = h->n;
        }
    }
    return HMX_OK;
}

hmx_status hmx_matvec(hmx_hmatrix h, const void* x, void* z, hmx_dtype vec_dtype, double alpha,
                      double beta, void* stream) {
    const hmx_status cs = matvec_args(h, x, z, vec_dtype);
    if (cs != HMX_OK) return cs;
    hipEvent_t* ev = nullptr;
    if (h->prof_calls < h->prof_max) ev = &h->prof_events[4 * h->prof_calls++];
    if (h->far_np) {
        const Allocator ua{h->prm.dev_alloc, h->prm.dev_free, h->prm.alloc_ctx};
        AllocScope scope(&ua);
        return guarded([&] { np_matvec(h, x, z, alpha, beta, (hipStream_t)stream, ev); });
    }
    const hipError_t e = matvec_launch(h, x, z, alpha, beta, (hipStream_t)stream, ev, h->rt_config);
    if (e != hipSuccess) {
        set_err("matvec launch: %s", hipGetErrorString(e));
        return HMX_ERR_DEVICE;
    }
    return HMX_OK;
}

hmx_status hmx_matmat(hmx_hmatrix h, const void* X, int64_t ldx, void* Z, int64_t ldz,
                      int32_t m, hmx_dtype vec_dtype, double alpha, double beta, void* stream) {
    const hmx_status cs = matvec_args(h, X, Z, vec_dtype);
    if (cs != HMX_OK) return cs;
    if (m < 1 || ldx < h->ncols || ldz < h->nrows) {
        set_err("m < 1, ldx < %lld or ldz < %lld", (long long)h->ncols, (long long)h->nrows);
        return HMX_ERR_INVALID_ARG;
    }
    if (h->far_np) {
        set_err("hmx_matmat: a far_recompute handle multiplies one vector at a time");
        return HMX_ERR_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    const Allocator ua{h->prm.dev_alloc, h->prm.dev_free, h->prm.alloc_ctx};
    AllocScope scope(&ua);
    return guarded([&] {
        constexpr int kMaxM = 16;
        const size_t esz = h->esz;
        const int f64 = h->f64;
        ensure(h->mm_vec, (size_t)(h->n + h->sum_rank) * kMaxM * esz, st, "multi-RHS vectors");
        const int64_t np1 = (h->sym ? h->ncols_u : 0) + h->ncols_v;
        ensure(h->mm_partial, (size_t)std::max<int64_t>(np1, 1) * kMaxM * esz, st,
               "multi-RHS partial sums");
        // groups: 16 sides at a time; the rest in one group padded to 8 or 16
        // zero sides when the row tiles run on the matrix cores (stored near
        // field: a padded group costs the same stream of stored entries),
        // else in power-of-two groups; a single remaining side is an
        // ordinary matvec
        const bool cores = h->nmode != 3;
        for (int32_t c0 = 0; c0 < m;) {
            const int32_t left = m - c0;
            const void* Xc = (const char*)X + (size_t)c0 * ldx * esz;
            void* Zc = (char*)Z + (size_t)c0 * ldz * esz;
            if (left == 1) {
                check(matvec_launch(h, Xc, Zc, alpha, beta, st, nullptr, h->rt_config),
                      "multi-RHS (one side)");
                break;
            }
            int M = kMaxM, mr = kMaxM;
            if (left < kMaxM) {
                if (cores) {
                    M = left > 8 ? 16 : 8;
                    mr = left;
                } else {
                    while (M > left) M >>= 1;
                    mr = M;
                }
            }
            check(launch_mm_gather(Xc, ldx, h->perm.as<int32_t>(), h->ncols, h->col0, h->mm_vec.p,
                                   M, mr, f64, st),
                  "multi-RHS gather");
            if (h->sym && h->ncols_u > 0)
                check(launch_mm_p1(M, h->ntiles, h->tile_lo.as<int32_t>(),
                                   h->tile_meta.as<int64_t>(), 4, h->Ru, h->upool.p, h->mm_vec.p,
                                   h->mm_partial.p, 0, h->smode, st),
                      "multi-RHS phase 1");
            if (h->ncols_v > 0)
                check(launch_mm_p1(M, h->ntiles, h->tile_lo.as<int32_t>(),
                                   h->vt_meta.as<int64_t>(), 4, h->Rv, h->vtpool.p, h->mm_vec.p,
                                   h->mm_partial.p, h->sym ? h->ncols_u : 0, h->smode, st),
                      "multi-RHS phase 1");
            check(launch_mm_p1_reduce(M, h->p1rec.as<int4>(), h->sum_rank, h->pfc.as<int64_t>(),
                                      h->mm_partial.p, h->mm_vec.p, h->n, f64, st),
                  "multi-RHS phase 1 sums");
            check(launch_mm_rowtile(M, h->ntiles_rows, h->tile_lo.as<int32_t>(),
                                    h->tile_meta.as<int64_t>(), h->widx.as<int64_t>(),
                                    h->upool.p, h->npool.p, h->mm_vec.p, h->perm.as<int32_t>(),
                                    alpha, beta, h->prm.sigma2, Zc, ldz, h->Ru, h->max_tile,
                                    h->smode, h->nmode, f64 ? h->soa64.p : h->soa32.p, h->n, h->d,
                                    kernel_fn(h->kern, h->kd), mr, st),
                  "multi-RHS row tiles");
            c0 += mr;
        }
    });
}

hmx_status hmx_matvec_batched(int32_t nprob, const hmx_hmatrix* hs, const void* const* x,
                              void* const* z, hmx_dtype vec_dtype, double alpha, double beta,
                              void* stream) {
    if (nprob < 0 || (nprob > 0 && (!hs || !x || !z))) {
        set_err("invalid argument to hmx_matvec_batched");
        return HMX_ERR_INVALID_ARG;
    }
    for (int32_t q = 0; q < nprob; ++q) {  // every argument checked before any launch
        const hmx_status cs = matvec_args(hs[q], x[q], z[q], vec_dtype);
        if (cs != HMX_OK) {
            set_err("problem %d: %s", q, g_err.c_str());
            return cs;
        }
    }
    for (int32_t q = 0; q < nprob; ++q) {
        const hmx_status s = hmx_matvec(hs[q], x[q], z[q], vec_dtype, alpha, beta, stream);
        if (s != HMX_OK) return s;
    }
    return HMX_OK;
}

hmx_status hmx_matvec_graph(hmx_hmatrix h, const void* x, void* z, hmx_dtype vec_dtype,
                            double alpha, double beta, int32_t reps, hmx_graph* out) {
    if (out) *out = nullptr;
    if (!out || reps < 1 || reps > 4096) {
        set_err("NULL output or reps not in [1, 4096]");
        return HMX_ERR_INVALID_ARG;
    }
    const hmx_status cs = matvec_args(h, x, z, vec_dtype);
    if (cs != HMX_OK) return cs;
    if (h->far_np) {
        set_err("far_recompute: the matvec waits for its chunks on the host; no graph");
        return HMX_ERR_UNSUPPORTED;
    }
    hmx_graph_s* g = new (std::nothrow) hmx_graph_s();
    if (!g) {
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        for (int32_t r = 0; r < reps && le == hipSuccess; ++r)
            le = matvec_launch(h, x, z, alpha, beta, cap, nullptr, h->rt_config);
        e = hipStreamEndCapture(cap, &g->graph);  // always ends the capture
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        set_err("matvec graph capture: %s", hipGetErrorString(e));
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        (void)hipGetLastError();
        return HMX_ERR_DEVICE;
    }
    *out = g;
    return HMX_OK;
}

hmx_status hmx_graph_launch(hmx_graph g, void* stream) {
    if (!g) {
        set_err("NULL graph");
        return HMX_ERR_INVALID_ARG;
    }
    const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_err("graph launch: %s", hipGetErrorString(e));
        return HMX_ERR_DEVICE;
    }
    return HMX_OK;
}

hmx_status hmx_graph_destroy(hmx_graph g) {
    if (!g) return HMX_OK;
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return HMX_OK;
}

hmx_status hmx_autotune(hmx_hmatrix h, int32_t reps, void* stream, int32_t* choice,
                        double* times_ms) {
    if (!h || reps < 1 || reps > 1000) {
        set_err("NULL handle or reps not in [1, 1000]");
        return HMX_ERR_INVALID_ARG;
    }
    if (h->prm.aca_only) {
        set_err("handle was built with aca_only: no matrix to apply");
        return HMX_ERR_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const Allocator ua{h->prm.dev_alloc, h->prm.dev_free, h->prm.alloc_ctx};
    AllocScope scope(&ua);
    hmx_status status = guarded([&] {
        DevBuf x, z;
        alloc(x, (size_t)h->n * h->esz, "tuning x");
        alloc(z, (size_t)h->n * h->esz, "tuning z");
        check(launch_fill_zero(x.p, h->n, h->f64, st), "fill");
        check(matvec_launch(h, x.p, z.p, 1.0, 0.0, st, nullptr, -1), "matvec");
        check(hipEventCreate(&e0), "event");
        check(hipEventCreate(&e1), "event");
        double best = INFINITY;
        int bc = -1;
        for (int c = 0; c < kRowtileConfigs; ++c) {
            auto rt = [&] {
                return launch_rowtile(h->ntiles_rows, h->tile_lo.as<int32_t>(),
                                      h->tile_meta.as<int64_t>(), h->widx.as<int64_t>(),
                                      h->upool.p, h->npool.p, h->vecpool.p,
                                      h->perm.as<int32_t>(), 1.0, 0.0, h->prm.sigma2, z.p,
                                      h->max_tile, h->smode, h->nmode, c,
                                      h->f64 ? h->soa64.p : h->soa32.p, h->n, h->d,
                                      kernel_fn(h->kern, h->kd), st);
            };
            check(rt(), "tuning warm-up");
            check(hipEventRecord(e0, st), "event");
            for (int r = 0; r < reps; ++r) check(rt(), "tuning launch");
            check(hipEventRecord(e1, st), "event");
            check(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            const double t = (double)ms / reps;
            if (times_ms) times_ms[c] = t;
            if (t < best) {
                best = t;
                bc = c;
            }
        }
        // phase 1: lanes per column group
        double pbest = INFINITY;
        int pl = 0;
        for (int lanes : {8, 16, 32, 64}) {
            check(p1_tiles(h, st, lanes), "tuning warm-up");
            check(hipEventRecord(e0, st), "event");
            for (int r = 0; r < reps; ++r) check(p1_tiles(h, st, lanes), "tuning launch");
            check(hipEventRecord(e1, st), "event");
            check(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            if (ms < pbest) {
                pbest = ms;
                pl = lanes;
            }
        }
        check(hipStreamSynchronize(st), "tuning sync");
        h->rt_config = bc;
        h->stats.tile_config = bc;
        h->p1_lanes = pl;
    });
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (status == HMX_OK && choice) *choice = h->rt_config;
    return status;
}

hmx_status hmx_set_tile_config(hmx_hmatrix h, int32_t config) {
    if (!h || config < -1 || config >= kRowtileConfigs) {
        set_err("NULL handle or tile config not in [-1, %d)", kRowtileConfigs);
        return HMX_ERR_INVALID_ARG;
    }
    h->rt_config = config;
    h->stats.tile_config = config;
    if (config < 0) h->p1_lanes = 0;  // the defaults of both phases
    return HMX_OK;
}

hmx_status hmx_cg_solve(hmx_hmatrix h, const void* b, void* x, double rel_tol, int32_t max_iter,
                        void* stream, int32_t* iters, double* rel_res, double* true_rel_res) {
    hmx_status s = cg_args(h, b, x, rel_tol, max_iter);
    if (s != HMX_OK) return s;
    const Allocator ua{h->prm.dev_alloc, h->prm.dev_free, h->prm.alloc_ctx};
    AllocScope scope(&ua);
    try {
        DevBuf r, p, q, scal, partial;
        const size_t vb = (size_t)h->n * h->esz;
        alloc(r, vb, "cg r");
        alloc(p, vb, "cg p");
        alloc(q, vb, "cg q");
        alloc(scal, 8 * sizeof(double), "cg scalars");
        alloc(partial, cg_scratch_bytes(), "cg partials");
        CgWork w{r.p, p.p, q.p, scal.as<double>(), partial.as<double>()};
        return cg_run(h, b, x, rel_tol, max_iter, (hipStream_t)stream, w, iters, rel_res,
                      true_rel_res);
    } catch (const Fail& f) {
        return f.s;
    }
}

hmx_status hmx_cg_solve_noalloc(hmx_hmatrix h, const void* b, void* x, double rel_tol,
                                int32_t max_iter, void* stream, int32_t* iters, double* rel_res,
                                double* true_rel_res) {
    hmx_status s = cg_args(h, b, x, rel_tol, max_iter);
    if (s != HMX_OK) return s;
    if (h->far_np) {
        set_err("hmx_cg_solve_noalloc: a far_recompute handle allocates chunk scratch per matvec");
        return HMX_ERR_UNSUPPORTED;
    }
    const size_t vb = cg_vec_bytes(h->n, h->esz);
    if (3 * vb + kCgScalBytes + cg_scratch_bytes() > HMX_CG_NOALLOC_MAX_BYTES) {
        set_err("hmx_cg_solve_noalloc: %lld entries of %zu bytes need %zu bytes of work space, "
                "more than its fixed %zu",
                (long long)h->n, h->esz, 3 * vb + kCgScalBytes + cg_scratch_bytes(),
                (size_t)HMX_CG_NOALLOC_MAX_BYTES);
        return HMX_ERR_INVALID_ARG;
    }
    try {
        char* base = (char*)cg_scratch_device();
        CgWork w{base, base + vb, base + 2 * vb, (double*)(base + 3 * vb),
                 (double*)(base + 3 * vb + kCgScalBytes)};
        return cg_run(h, b, x, rel_tol, max_iter, (hipStream_t)stream, w, iters, rel_res,
                      true_rel_res);
    } catch (const Fail& f) {
        return f.s;
    }
}

hmx_status hmx_get_partition(hmx_hmatrix h, uint64_t* codes, int32_t* perm, int32_t* adm,
                             int64_t* n_adm, int32_t* dense, int64_t* n_dense, void* stream) {
    if (!h) {
        set_err("NULL handle");
        return HMX_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    try {
        if ((adm && (!n_adm || *n_adm < h->n_adm)) || (dense && (!n_dense || *n_dense < h->n_dense))) {
            if (n_adm) *n_adm = h->n_adm;
            if (n_dense) *n_dense = h->n_dense;
            set_err("partition capacity too small");
            return HMX_ERR_INVALID_ARG;
        }
        if (n_adm) *n_adm = h->n_adm;
        if (n_dense) *n_dense = h->n_dense;
        std::vector<uint32_t> pm(h->n);
        d2h(pm.data(), h->perm.p, h->n * 4, st);
        std::vector<uint64_t> sc;
        if (codes) {
            sc.resize(h->n);
            d2h(sc.data(), h->codes.p, h->n * 8, st);
        }
        std::vector<int4> a(h->n_adm), dn(h->n_dense);
        std::vector<int32_t> al(h->n_adm), dl(h->n_dense);
        if (adm && h->n_adm) {
            d2h(a.data(), h->adm.p, h->n_adm * 16, st);
            d2h(al.data(), h->adm_level.p, h->n_adm * 4, st);
        }
        if (dense && h->n_dense) {
            d2h(dn.data(), h->dense.p, h->n_dense * 16, st);
            d2h(dl.data(), h->dense_level.p, h->n_dense * 4, st);
        }
        check(hipStreamSynchronize(st), "sync");
        if (perm)
            for (int64_t k = 0; k < h->n; ++k) perm[k] = (int32_t)pm[k];
        if (codes)
            for (int64_t k = 0; k < h->n; ++k) codes[pm[k]] = sc[k];
        if (adm)
            for (int64_t q = 0; q < h->n_adm; ++q) {
                int32_t* o = adm + 5 * q;
                o[0] = a[q].x; o[1] = a[q].y; o[2] = a[q].z; o[3] = a[q].w; o[4] = al[q];
            }
        if (dense)
            for (int64_t q = 0; q < h->n_dense; ++q) {
                int32_t* o = dense + 5 * q;
                o[0] = dn[q].x; o[1] = dn[q].y; o[2] = dn[q].z; o[3] = dn[q].w; o[4] = dl[q];
            }
    } catch (const Fail& f) {
        return f.s;
    }
    return HMX_OK;
}

hmx_status hmx_get_boxes(hmx_hmatrix h, double* global_box, double* leaf_boxes, void* stream) {
    if (h && h->batched) {
        set_err("batched handle: boxes belong to the individual problems");
        return HMX_ERR_UNSUPPORTED;
    }
    if (!h) {
        set_err("NULL handle");
        return HMX_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    try {
        if (global_box)
            for (int k = 0; k < 2 * h->d; ++k) global_box[k] = h->box[k];
        if (leaf_boxes) {
            const int d = h->d;
            std::vector<int32_t> lo(h->nslots), hi(h->nslots);
            std::vector<double> bmn(h->nslots * d), bmx(h->nslots * d);
            d2h(lo.data(), h->node_lo.p, h->nslots * 4, st);
            d2h(hi.data(), h->node_hi.p, h->nslots * 4, st);
            d2h(bmn.data(), h->bmin.p, h->nslots * d * 8, st);
            d2h(bmx.data(), h->bmax.p, h->nslots * d * 8, st);
            check(hipStreamSynchronize(st), "sync");
            // leaf clusters in Morton order (sorted by lo)
            std::vector<std::pair<int32_t, int64_t>> leaves;
            for (int64_t id = 0; id < h->nslots; ++id)
                if (lo[id] >= 0 && hi[id] - lo[id] <= h->prm.leaf_size) leaves.push_back({lo[id], id});
            std::sort(leaves.begin(), leaves.end());
            const int w = 2 * d + 2;
            for (size_t t = 0; t < leaves.size(); ++t) {
                const int64_t id = leaves[t].second;
                for (int k = 0; k < d; ++k) {
                    leaf_boxes[t * w + k] = bmn[id * d + k];
                    leaf_boxes[t * w + d + k] = bmx[id * d + k];
                }
                leaf_boxes[t * w + 2 * d] = lo[id];
                leaf_boxes[t * w + 2 * d + 1] = hi[id];
            }
        }
    } catch (const Fail& f) {
        return f.s;
    }
    return HMX_OK;
}

hmx_status hmx_get_ranks(hmx_hmatrix h, int32_t* ranks, void* stream) {
    if (!h || !ranks) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    try {
        if (h->n_adm) {
            d2h(ranks, h->rank.p, h->n_adm * 4, st);
        }
    } catch (const Fail& f) {
        return f.s;
    }
    return HMX_OK;
}

hmx_status hmx_get_factors(hmx_hmatrix h, int64_t leaf, double* U, double* V, int32_t* rank,
                           void* stream) {
    if (!h || leaf < 0 || leaf >= h->n_adm || !U || !V || !rank) {
        set_err("invalid argument to hmx_get_factors");
        return HMX_ERR_INVALID_ARG;
    }
    if (h->prm.aca_only || h->far_np) {
        set_err("handle was built with %s: factors were not kept",
                h->far_np ? "far_recompute" : "aca_only");
        return HMX_ERR_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    try {
        int4 bl;
        int32_t r, mirror = (int32_t)leaf;
        check(hipMemcpyAsync(&bl, h->adm.as<int4>() + leaf, 16, hipMemcpyDeviceToHost, st), "blk");
        check(hipMemcpyAsync(&r, h->rank.as<int32_t>() + leaf, 4, hipMemcpyDeviceToHost, st), "r");
        if (h->sym)
            check(hipMemcpyAsync(&mirror, h->partner.as<int32_t>() + leaf, 4,
                                 hipMemcpyDeviceToHost, st),
                  "mirror");
        check(hipStreamSynchronize(st), "sync");
        const int64_t m = bl.y - bl.x, nc = bl.w - bl.z;
        const size_t esz = h->ssz;  // stored entry size
        *rank = r;
        auto to_double = [&](const std::vector<char>& raw, size_t cnt, double* out) {
            for (size_t e = 0; e < cnt; ++e) {
                if (esz == 8) {
                    out[e] = ((const double*)raw.data())[e];
                } else if (esz == 4) {
                    out[e] = ((const float*)raw.data())[e];
                } else {
                    uint32_t u = (uint32_t)((const uint16_t*)raw.data())[e] << 16;
                    float f;
                    memcpy(&f, &u, 4);
                    out[e] = f;
                }
            }
        };
        std::vector<int32_t> tlo(h->ntiles + 1);
        d2h(tlo.data(), h->tile_lo.p, (h->ntiles + 1) * 4, st);
        // the rows of leaf blk's r columns held by its pieces in a row-tile
        // pool (one piece per row tile), into out (len x r, column-major)
        auto rows_of = [&](const DevBuf& dpcs, int64_t npcs, int32_t blk, const DevBuf& pool, int R,
                           int64_t len, double* out) {
            std::vector<Piece> pcs(npcs);
            if (npcs > 0) d2h(pcs.data(), dpcs.p, npcs * sizeof(Piece), st);
            for (const Piece& pc : pcs) {
                if (pc.blk != blk) continue;
                const int mt = tlo[pc.tile + 1] - tlo[pc.tile];
                const int ld = (mt + R - 1) / R * R;
                std::vector<char> col((size_t)ld * r * esz + 1);
                d2h(col.data(), (const char*)pool.p + pc.d_off * esz, (size_t)ld * r * esz, st);
                std::vector<double> cd((size_t)ld * r);
                to_double(col, (size_t)ld * r, cd.data());
                for (int l = 0; l < r; ++l)
                    for (int i = 0; i < mt; ++i)
                        out[(int64_t)l * len + pc.row0 + i] = cd[(size_t)l * ld + i];
            }
        };
        // U: the leaf's factor pieces; V: its V pieces, or (symmetric far
        // field) the factor pieces of its mirror, whose rows are sigma's
        rows_of(h->pieces, h->npieces, (int32_t)leaf, h->upool, h->Ru, m, U);
        if (mirror != (int32_t)leaf)
            rows_of(h->pieces, h->npieces, mirror, h->upool, h->Ru, nc, V);
        else
            rows_of(h->vpieces, h->nvpieces, (int32_t)leaf, h->vtpool, h->Rv, nc, V);
    } catch (const Fail& f) {
        return f.s;
    }
    return HMX_OK;
}

hmx_status hmx_get_stats(hmx_hmatrix h, hmx_stats* s) {
    if (!h || !s) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    *s = h->stats;
    return HMX_OK;
}

hmx_status hmx_profile_begin(hmx_hmatrix h, int32_t max_calls) {
    if (!h || max_calls < 0 || max_calls > (1 << 20)) {
        set_err("invalid argument to hmx_profile_begin");
        return HMX_ERR_INVALID_ARG;
    }
    h->prof_release();
    h->prof_events.resize((size_t)4 * max_calls, nullptr);
    for (auto& e : h->prof_events) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            e = nullptr;
            h->prof_release();
            set_err("hipEventCreate: %s", hipGetErrorString(r));
            return HMX_ERR_DEVICE;
        }
    }
    h->prof_max = max_calls;
    h->prof_calls = 0;
    return HMX_OK;
}

hmx_status hmx_profile_end(hmx_hmatrix h, double* ms, int32_t* calls) {
    if (!h || !ms || !calls) {
        set_err("invalid argument to hmx_profile_end");
        return HMX_ERR_INVALID_ARG;
    }
    ms[0] = ms[1] = ms[2] = 0.0;
    *calls = h->prof_calls;
    hmx_status s = HMX_OK;
    if (h->prof_calls > 0) {
        hipError_t r = hipEventSynchronize(h->prof_events[4 * h->prof_calls - 1]);
        for (int32_t c = 0; c < h->prof_calls && r == hipSuccess; ++c)
            for (int p = 0; p < 3 && r == hipSuccess; ++p) {
                float t = 0.f;
                r = hipEventElapsedTime(&t, h->prof_events[4 * c + p], h->prof_events[4 * c + p + 1]);
                ms[p] += t;
            }
        if (r != hipSuccess) {
            set_err("event timing: %s", hipGetErrorString(r));
            s = HMX_ERR_DEVICE;
        }
    }
    h->prof_release();
    return s;
}

// ---------------------------------------------------------------------------
// rank predictor
// ---------------------------------------------------------------------------


hmx_status hmx_mlp_create(const float* params, hmx_mlp* out) {
    if (out) *out = nullptr;
    if (!out) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    if (mlp_nparams() != kP) {
        set_err("parameter count mismatch");
        return HMX_ERR_DEVICE;
    }
    hmx_mlp_s* m = new (std::nothrow) hmx_mlp_s();
    if (!m) {
        set_err("host allocation failed");
        return HMX_ERR_OOM;
    }
    hmx_status s = guarded([&] {
        alloc(m->w, kP * 4, "mlp weights");
        alloc(m->m, kP * 4, "adam m");
        alloc(m->v, kP * 4, "adam v");
        alloc(m->mean, 8 * 4, "mlp mean");
        alloc(m->scale, 8 * 4, "mlp scale");
        std::vector<float> w(kP, 0.f), mu(8, 0.f), sc(8, 1.f);
        if (params) memcpy(w.data(), params, kP * 4);
        check(hipMemcpy(m->w.p, w.data(), kP * 4, hipMemcpyHostToDevice), "weights");
        check(hipMemset(m->m.p, 0, kP * 4), "adam m");
        check(hipMemset(m->v.p, 0, kP * 4), "adam v");
        check(hipMemcpy(m->mean.p, mu.data(), 32, hipMemcpyHostToDevice), "mean");
        check(hipMemcpy(m->scale.p, sc.data(), 32, hipMemcpyHostToDevice), "scale");
    });
    if (s != HMX_OK) {
        delete m;
        return s;
    }
    *out = m;
    return HMX_OK;
}

hmx_status hmx_mlp_destroy(hmx_mlp m) {
    if (!m) return HMX_OK;
    (void)hipDeviceSynchronize();
    delete m;
    return HMX_OK;
}

hmx_status hmx_mlp_set_params(hmx_mlp m, const float* params, const float* mean,
                              const float* scale) {
    if (!m) {
        set_err("NULL predictor");
        return HMX_ERR_INVALID_ARG;
    }
    return guarded([&] {
        check(hipDeviceSynchronize(), "sync");
        if (params) check(hipMemcpy(m->w.p, params, kP * 4, hipMemcpyHostToDevice), "weights");
        if (mean) check(hipMemcpy(m->mean.p, mean, 32, hipMemcpyHostToDevice), "mean");
        if (scale) check(hipMemcpy(m->scale.p, scale, 32, hipMemcpyHostToDevice), "scale");
        check(hipMemset(m->m.p, 0, kP * 4), "adam m");
        check(hipMemset(m->v.p, 0, kP * 4), "adam v");
        m->t = 0;
    });
}

hmx_status hmx_mlp_get_params(hmx_mlp m, float* params, float* mean, float* scale) {
    if (!m) {
        set_err("NULL predictor");
        return HMX_ERR_INVALID_ARG;
    }
    return guarded([&] {
        check(hipDeviceSynchronize(), "sync");
        if (params) check(hipMemcpy(params, m->w.p, kP * 4, hipMemcpyDeviceToHost), "weights");
        if (mean) check(hipMemcpy(mean, m->mean.p, 32, hipMemcpyDeviceToHost), "mean");
        if (scale) check(hipMemcpy(scale, m->scale.p, 32, hipMemcpyDeviceToHost), "scale");
    });
}

hmx_status hmx_mlp_save(hmx_mlp m, const char* path) {
    if (!m || !path) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    std::vector<float> w(kP), mo(kP), vo(kP), mu(8), sc(8);
    hmx_status s = guarded([&] {
        check(hipDeviceSynchronize(), "sync");
        check(hipMemcpy(w.data(), m->w.p, kP * 4, hipMemcpyDeviceToHost), "weights");
        check(hipMemcpy(mo.data(), m->m.p, kP * 4, hipMemcpyDeviceToHost), "adam m");
        check(hipMemcpy(vo.data(), m->v.p, kP * 4, hipMemcpyDeviceToHost), "adam v");
        check(hipMemcpy(mu.data(), m->mean.p, 32, hipMemcpyDeviceToHost), "mean");
        check(hipMemcpy(sc.data(), m->scale.p, 32, hipMemcpyDeviceToHost), "scale");
    });
    if (s != HMX_OK) return s;
    FILE* f = fopen(path, "wb");
    if (!f) {
        set_err("cannot open %s for writing", path);
        return HMX_ERR_INVALID_ARG;
    }
    const int64_t head[2] = {kP, m->t};
    bool ok = fwrite(kMlpMagic, 1, 8, f) == 8 && fwrite(head, 8, 2, f) == 2 &&
              fwrite(w.data(), 4, kP, f) == (size_t)kP && fwrite(mu.data(), 4, 8, f) == 8 &&
              fwrite(sc.data(), 4, 8, f) == 8 && fwrite(mo.data(), 4, kP, f) == (size_t)kP &&
              fwrite(vo.data(), 4, kP, f) == (size_t)kP;
    ok = (fclose(f) == 0) && ok;
    if (!ok) {
        set_err("writing %s failed", path);
        return HMX_ERR_INVALID_ARG;
    }
    return HMX_OK;
}

hmx_status hmx_mlp_load(const char* path, hmx_mlp* out) {
    if (out) *out = nullptr;
    if (!path || !out) {
        set_err("NULL argument");
        return HMX_ERR_INVALID_ARG;
    }
    FILE* f = fopen(path, "rb");
    if (!f) {
        set_err("cannot open %s", path);
        return HMX_ERR_INVALID_ARG;
    }
    char magic[8];
    int64_t head[2] = {0, 0};
    std::vector<float> w(kP), mo(kP), vo(kP), mu(8), sc(8);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMlpMagic, 8) == 0 &&
              fread(head, 8, 2, f) == 2 && head[0] == kP && head[1] >= 0 &&
              fread(w.data(), 4, kP, f) == (size_t)kP && fread(mu.data(), 4, 8, f) == 8 &&
              fread(sc.data(), 4, 8, f) == 8 && fread(mo.data(), 4, kP, f) == (size_t)kP &&
              fread(vo.data(), 4, kP, f) == (size_t)kP;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the record
    fclose(f);
    if (!ok) {
        set_err("%s is not a rank predictor file of %lld parameters", path, (long long)kP);
        return HMX_ERR_INVALID_ARG;
    }
    hmx_mlp m = nullptr;
    hmx_status s = hmx_mlp_create(w.data(), &m);
    if (s != HMX_OK) return s;
    s = guarded([&] {
        check(hipMemcpy(m->mean.p, mu.data(), 32, hipMemcpyHostToDevice), "mean");
        check(hipMemcpy(m->scale.p, sc.data(), 32, hipMemcpyHostToDevice), "scale");
        check(hipMemcpy(m->m.p, mo.data(), kP * 4, hipMemcpyHostToDevice), "adam m");
        check(hipMemcpy(m->v.p, vo.data(), kP * 4, hipMemcpyHostToDevice), "adam v");
        m->t = head[1];
    });
    if (s != HMX_OK) {
        hmx_mlp_destroy(m);
        return s;
    }
    *out = m;
    return HMX_OK;
}

hmx_status hmx_mlp_fit_normalization(hmx_mlp m, const float* X, int64_t n, void* stream) {
    if (!m || !X || n < 1) {
        set_err("invalid argument to hmx_mlp_fit_normalization");
        return HMX_ERR_INVALID_ARG;
    }
    return guarded([&] {
        check(mlp_norm(X, n, m->mean.as<float>(), m->scale.as<float>(), (hipStream_t)stream),
              "normalization");
    });
}

hmx_status hmx_mlp_forward(hmx_mlp m, const float* X, int64_t B, float* out, void* stream) {
    if (!m || B < 0 || (B > 0 && (!X || !out))) {
        set_err("invalid argument to hmx_mlp_forward");
        return HMX_ERR_INVALID_ARG;
    }
    if (B == 0) return HMX_OK;
    hipStream_t st = (hipStream_t)stream;
    return guarded([&] {
        ensure(m->act, (size_t)B * 193 * 4, st, "activations");
        check(mlp_forward(m->w.as<float>(), m->mean.as<float>(), m->scale.as<float>(), X, B,
                          m->act.as<float>(), st),
              "mlp forward");
        check(hipMemcpyAsync(out, m->act.as<float>() + (size_t)B * 192, (size_t)B * 4,
                             hipMemcpyDeviceToDevice, st),
              "output copy");
    });
}

extern "C++" {
namespace {
// forward + backward on a device batch; loss_dev optional
void mlp_step_grad(hmx_mlp_s* m, const float* X, const float* y, int64_t B, double q,
                   float* grad, double* loss_dev, hipStream_t st) {
    ensure(m->act, (size_t)B * 193 * 4, st, "activations");
    ensure(m->scratch, mlp_grad_scratch_floats(B) * 4, st, "gradient scratch");
    check(mlp_forward(m->w.as<float>(), m->mean.as<float>(), m->scale.as<float>(), X, B,
                      m->act.as<float>(), st),
          "mlp forward");
    check(mlp_backward(m->w.as<float>(), m->mean.as<float>(), m->scale.as<float>(), X, y, B,
                       (float)q, m->act.as<float>(), grad, m->scratch.as<float>(), loss_dev, st),
          "mlp backward");
}
}  // namespace
}  // extern "C++"

hmx_status hmx_mlp_loss_grad(hmx_mlp m, const float* X, const float* y, int64_t B, double q,
                             float* grad, double* loss, void* stream) {
    if (!m || !X || !y || !grad || B < 1 || !(q > 0 && q < 1)) {
        set_err("invalid argument to hmx_mlp_loss_grad");
        return HMX_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    return guarded([&] {
        ensure(m->loss, 8, st, "loss");
        mlp_step_grad(m, X, y, B, q, grad, loss ? m->loss.as<double>() : nullptr, st);
        if (loss) *loss = read_scalar(m->loss.as<double>(), st);
    });
}

hmx_status hmx_mlp_adam(hmx_mlp m, const float* grad, double lr, double beta1, double beta2,
                        double eps, void* stream) {
    if (!m || !grad || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
        !(eps > 0)) {
        set_err("invalid argument to hmx_mlp_adam");
        return HMX_ERR_INVALID_ARG;
    }
    return guarded([&] {
        m->t += 1;
        check(mlp_adam(m->w.as<float>(), m->m.as<float>(), m->v.as<float>(), grad, m->t,
                       (float)lr, (float)beta1, (float)beta2, (float)eps, (hipStream_t)stream),
              "adam");
    });
}

hmx_status hmx_mlp_train(hmx_mlp m, const float* X, const float* y, int64_t n,
                         const int64_t* batch_idx, int64_t B, int32_t steps, double q, double lr,
                         double* losses, void* stream) {
    if (!m || !X || !y || n < 1 || !batch_idx || B < 1 || steps < 0 || !(q > 0 && q < 1) ||
        !(lr >= 0)) {
        set_err("invalid argument to hmx_mlp_train");
        return HMX_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    return guarded([&] {
        ensure(m->Xb, (size_t)B * 8 * 4, st, "batch features");
        ensure(m->yb, (size_t)B * 4, st, "batch targets");
        ensure(m->grad, (size_t)kP * 4, st, "gradient");
        ensure(m->act, (size_t)B * 193 * 4, st, "activations");
        ensure(m->scratch, mlp_grad_scratch_floats(B) * 4, st, "gradient scratch");
        for (int32_t s = 0; s < steps; ++s) {
            check(mlp_gather_batch(X, y, n, batch_idx + (int64_t)s * B, B, m->Xb.as<float>(),
                                   m->yb.as<float>(), st),
                  "batch gather");
            mlp_step_grad(m, m->Xb.as<float>(), m->yb.as<float>(), B, q, m->grad.as<float>(),
                          losses ? losses + s : nullptr, st);
            m->t += 1;
            check(mlp_adam(m->w.as<float>(), m->m.as<float>(), m->v.as<float>(),
                           m->grad.as<float>(), m->t, (float)lr, 0.9f, 0.999f, 1e-8f, st),
                  "adam");
        }
    });
}

hmx_status hmx_block_features(hmx_hmatrix h, float* features, float* ranks, int64_t* n_adm,
                              void* stream) {
    if (!h || !n_adm || (h->n_adm > 0 && !features)) {
        set_err("invalid argument to hmx_block_features");
        return HMX_ERR_INVALID_ARG;
    }
    if (h->batched) {
        set_err("batched handle: features belong to the individual problems");
        return HMX_ERR_UNSUPPORTED;
    }
    if (*n_adm < h->n_adm) {
        set_err("capacity %lld below %lld admissible leaves", (long long)*n_adm,
                (long long)h->n_adm);
        *n_adm = h->n_adm;
        return HMX_ERR_INVALID_ARG;
    }
    *n_adm = h->n_adm;
    return guarded([&] {
        check(launch_features(h->adm.as<int4>(), h->adm_ids.as<int2>(), h->n_adm,
                              h->bmin.as<double>(), h->bmax.as<double>(), h->d,
                              kernel_length(h->kern), h->rank.as<int32_t>(), features, ranks,
                              (hipStream_t)stream),
              "features");
    });
}

hmx_status hmx_rank_predict(hmx_hmatrix h, hmx_mlp m, float* pred, int32_t* target,
                            int64_t* n_adm, void* stream) {
    if (!h || !m || !n_adm || (h->n_adm > 0 && !pred && !target)) {
        set_err("invalid argument to hmx_rank_predict");
        return HMX_ERR_INVALID_ARG;
    }
    if (h->batched) {
        set_err("batched handle: predictions belong to the individual problems");
        return HMX_ERR_UNSUPPORTED;
    }
    if (*n_adm < h->n_adm) {
        set_err("capacity %lld below %lld admissible leaves", (long long)*n_adm,
                (long long)h->n_adm);
        *n_adm = h->n_adm;
        return HMX_ERR_INVALID_ARG;
    }
    *n_adm = h->n_adm;
    return guarded([&] {
        check(launch_rank_predict(h->adm.as<int4>(), h->adm_ids.as<int2>(), h->n_adm,
                                  h->bmin.as<double>(), h->bmax.as<double>(), h->d,
                                  kernel_length(h->kern), m->w.as<float>(), m->mean.as<float>(),
                                  m->scale.as<float>(), h->prm.max_rank, pred, target,
                                  (hipStream_t)stream),
              "rank prediction");
    });
}

hmx_status hmx_destroy(hmx_hmatrix h) {
    if (!h) return HMX_OK;
    (void)hipDeviceSynchronize();
    delete h;
    return HMX_OK;
}

hmx_status hmx_trim(int64_t* released_bytes) {
    DeviceCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    (void)hipDeviceSynchronize();
    int64_t tot = 0;
    for (auto& b : c.blocks) {
        c.owned.erase(b.second.second);
        (void)hipFree(b.second.second);
        tot += (int64_t)b.first;
    }
    c.blocks.clear();
    c.cached = 0;
    if (released_bytes) *released_bytes = tot;
    return HMX_OK;
}

}  // extern "C"
