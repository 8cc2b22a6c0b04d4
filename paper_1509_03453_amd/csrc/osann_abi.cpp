// Host side of the C ABI declared in include/osann.h: argument checks, device
// memory of an index, the launch sequences of the gfx950 kernels, the split
// autotuner of the tiled path and hipGraph replay of repeated searches.
#include "osann.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <atomic>
#include <mutex>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "osann_batch.h"
#include "osann_fixedc.h"
#include "osann_ivf.h"
#include "osann_sparse.h"
#include "osann_kernels.h"
#include "osann_tiled.h"
#include "osann_wht.h"

using namespace osann;

// Scratch of os_ann_search_static: a fixed device array, one copy per GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): it takes the device address from hipGetSymbolAddress once per
// device and uses that.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local int g_err = OS_ANN_OK;
thread_local std::string g_msg;

int fail(int code, const std::string& msg) {
    g_err = code;
    g_msg = msg;
    return code;
}
void clear_error() {
    g_err = OS_ANN_OK;
    g_msg.clear();
}
int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? OS_ANN_ENOMEM : OS_ANN_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define OSANN_HIP(call, what)                              \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, what);   \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int64_t pow2_ceil(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

// Low-precision, 16-row padded copy used by the tiled path (built on first use).
struct LowpCopy {
    bool ready = false;
    int dk = 0, f16 = 0;
    int64_t np = 0;  // padded rows
    uint32_t* poff = nullptr;
    uint32_t* ne_id = nullptr;
    uint32_t* ne_cone = nullptr;
    uint16_t* xl = nullptr;
    float* nrm = nullptr;
    uint32_t* ppos = nullptr;
    uint32_t* prow = nullptr;  // original row of each padded row
    uint32_t* ipos = nullptr;  // padded position of each original row
};

// Graph replay by shape class.  The graphs captured on one stream read and
// write that stream's arena: the search scratch, the staged queries and the
// outputs, sized for the largest class captured there so far.  Calls on one
// stream run in order, so its graphs can share the arena.
struct GraphArena {
    hipStream_t s = nullptr;
    int64_t cap_q = 0;     // query rows the staging and output buffers hold
    int qtype = -1;        // element type the staged rows were last written in
    size_t ws_bytes = 0;
    char* ws = nullptr;
    void* q = nullptr;     // [cap_q][D] elements of up to 4 bytes
    int64_t* oidx = nullptr;
    float* odist = nullptr;
    int64_t* oncand = nullptr;
    int64_t* capped = nullptr;
};
struct GraphEntry {
    std::vector<int64_t> key;  // stream, query class, query type, mode, R, cone budget, budget, capped count
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;         // last replay (the least recently used goes first)
};
constexpr size_t kMaxGraphs = 512;  // per index: a few streams times the classes up to 8192 queries

// The graph cap; OSANN_MAX_GRAPHS (1 .. 4096) lowers it for testing.
size_t max_graphs() {
    if (const char* e = std::getenv("OSANN_MAX_GRAPHS")) {
        const long v = std::atol(e);
        if (v >= 1 && v <= 4096) return (size_t)v;
    }
    return kMaxGraphs;
}

struct os_ann_index {
    int64_t N = 0;
    int32_t D = 0, L = 0, dtype = 0;
    int32_t Dk = 0;  // length of the keys the cones come from (D, or k for a projected table)
    int64_t n_cones = 0, n_sub = 0, n_nonempty = 0;
    int nch = 0, epc = 0;
    int device = 0, num_cu = 256;
    size_t device_bytes = 0;
    uint32_t* row_cone = nullptr;
    uint64_t* row_top = nullptr;
    uint32_t* perm = nullptr;
    uint32_t* sorted_cone = nullptr;
    uint32_t* offsets = nullptr;
    void* planes = nullptr;
    uint8_t* lexsub = nullptr;
    uint8_t* maskord = nullptr;
    uint32_t* binom = nullptr;
    // a build whose closing check is left to the low-precision copy's end:
    // its flags ([0] non-finite, [1] non-empty count) and sort scratch, kept
    // until that synchronisation
    uint32_t* pending_small = nullptr;
    uint32_t* pending_tmp = nullptr;
    std::mutex lowp_mu;
    LowpCopy lp;
    // scratch owned by the index, used when the caller brings no workspace
    std::mutex scratch_mu;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    // events around timed kernel launches: (kernel id, start, stop)
    struct Timed {
        int kernel;
        hipEvent_t start, stop;
    };
    std::mutex time_mu;
    std::vector<Timed> timed;
    // captured search sequences, by shape class, and their per-stream arenas
    std::mutex graph_mu;
    std::vector<GraphEntry> graphs;
    std::vector<GraphArena> arenas;
    uint64_t graph_tick = 0;
    int64_t graph_captures = 0, graph_replays = 0;
    // the tiling of the last tiled search enqueued (kernel 0 query-tile, 1 cone-major)
    std::atomic<int32_t> last_kern{-1}, last_order{-1}, last_groups{0}, last_splits{0};
    // several bases (Section 3.A): one table per basis; this index then owns
    // the tables, the bases and their gathered copies
    int n_rot = 0;
    std::vector<os_ann_index*> sub;
    float* rot = nullptr;            // [R][D][D]
    float* rot_signs = nullptr;      // structured bases: [R][D] signs of H diag(s) (rot unused)
    uint32_t* rot_offsets = nullptr;  // [R][n_cones+1]
    uint32_t* rot_perm = nullptr;     // [R][N]
    uint64_t* xtop = nullptr;         // [R][R][N]
    void** planes_tab = nullptr;      // [R] device copies of the tables' plane pointers
    // PCA front-end (Section 4.B): keys are P (x - mu), k = Dk components
    bool proj = false;
    float* proj_mu = nullptr;  // [D], or null: no centring
    float* proj_P = nullptr;   // [k][D]
    // coarse clusters (ROSANNA+, Section 4.B): buckets are (cluster, cone) =
    // cluster * n_cones + cone; the rows are hashed on their residuals
    int32_t n_groups = 1;       // clusters (1: a plain table)
    float* ivf_cent = nullptr;  // [n_groups][D]
    // sparse table (more than 2^24 cones): offsets are per non-empty cone
    bool sparse = false;
    uint64_t* sp_keys = nullptr;   // [n_nonempty] cone ids, ascending
    uint64_t* sp_hkeys = nullptr;  // [sp_cap] hash slots
    uint32_t* sp_hval = nullptr;   // [sp_cap]
    uint64_t sp_cap = 0;
    uint64_t* sp_filt = nullptr;   // [sp_fbits / 64] filter words
    uint64_t sp_fbits = 0;
    uint64_t* binom64 = nullptr;   // [257][8]
    int32_t nprobe = 0;         // clusters searched per query
};

namespace {

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------
// Freed device blocks are kept per (device, rounded size) and handed out
// again, so that indexes and scratch built and released over and over do
// not pay hipMalloc / hipFree (which waits for the whole device) each time.
// A block enters the cache only once the device has finished with it: every
// caller of dev_free has synchronized first, as hipFree itself would.
struct BlockCache {
    std::mutex mu;
    std::multimap<std::pair<int, size_t>, void*> idle;             // (device, size) -> block
    std::unordered_map<void*, std::pair<int, size_t>> owned;        // block -> (device, size)
    size_t idle_bytes = 0;
};
BlockCache& block_cache() {
    static BlockCache* c = new BlockCache;  // never destroyed: blocks live until the process ends
    return *c;
}

// Caller-supplied allocator (os_ann_set_allocator).  Blocks it hands out are
// recorded with the hook that made them and the stream they were asked for,
// and go back to that hook, never to the idle cache.
struct Hook {
    os_ann_alloc_fn alloc = nullptr;
    os_ann_free_fn free = nullptr;
    void* ctx = nullptr;
};
struct HookedBlock {
    Hook hook;
    void* stream;
};
Hook g_hook;                                         // guarded by block_cache().mu
std::unordered_map<void*, HookedBlock> g_hooked;     // guarded by block_cache().mu
thread_local hipStream_t t_stream = nullptr;         // stream of the calling entry point

// Sets the stream an entry point's allocations are made for, for its scope.
struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s) : prev(t_stream) { t_stream = s; }
    ~StreamScope() { t_stream = prev; }
};
constexpr size_t kIdleMax = size_t(8) << 30;  // idle bytes kept at most (all devices)

size_t block_size(size_t bytes) { return bytes > (size_t(1) << 20) ? align_up(bytes, size_t(2) << 20) : align_up(bytes, 256); }

// Returns the idle blocks of every device to the runtime.
void trim_blocks() {
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> g(c.mu);
    for (auto& kv : c.idle) (void)hipFree(kv.second);
    c.idle.clear();
    c.idle_bytes = 0;
}

hipError_t cached_malloc(void** p, size_t bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t sz = block_size(bytes);
    BlockCache& c = block_cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.idle.find({dev, sz});
        if (it != c.idle.end()) {
            *p = it->second;
            c.idle.erase(it);
            c.idle_bytes -= sz;
            c.owned[*p] = {dev, sz};
            return hipSuccess;
        }
    }
    e = hipMalloc(p, sz);
    if (e == hipErrorOutOfMemory) {  // idle blocks of other sizes may be what is missing
        (void)hipGetLastError();
        trim_blocks();
        e = hipMalloc(p, sz);
    }
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(c.mu);
    c.owned[*p] = {dev, sz};
    return hipSuccess;
}

// The caller has synchronized the device (no kernel still uses p).
void dev_free(void* p) {
    if (!p) return;
    BlockCache& c = block_cache();
    std::unique_lock<std::mutex> g(c.mu);
    auto hk = g_hooked.find(p);
    if (hk != g_hooked.end()) {
        const HookedBlock b = hk->second;
        g_hooked.erase(hk);
        g.unlock();  // the hook may call back into the runtime
        b.hook.free(p, b.stream, b.hook.ctx);
        return;
    }
    auto it = c.owned.find(p);
    if (it == c.owned.end()) {
        (void)hipFree(p);
        return;
    }
    const auto key = it->second;
    c.owned.erase(it);
    if (c.idle_bytes + key.second <= kIdleMax) {
        c.idle.emplace(key, p);
        c.idle_bytes += key.second;
    } else {
        (void)hipFree(p);
    }
}

int dev_alloc(os_ann_index* ix, void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    Hook h;
    {
        std::lock_guard<std::mutex> g(block_cache().mu);
        h = g_hook;
    }
    if (h.alloc) {
        void* q = h.alloc(bytes, static_cast<void*>(t_stream), h.ctx);
        if (!q) return fail(OS_ANN_ENOMEM, std::string(what) + ": the allocator hook returned NULL");
        if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
            h.free(q, static_cast<void*>(t_stream), h.ctx);
            return fail(OS_ANN_ENOMEM, std::string(what) + ": the allocator hook returned a block not aligned to 256 bytes");
        }
        {
            std::lock_guard<std::mutex> g(block_cache().mu);
            g_hooked[q] = {h, static_cast<void*>(t_stream)};
        }
        *p = q;
        if (ix) ix->device_bytes += bytes;
        return OS_ANN_OK;
    }
    hipError_t e = cached_malloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return hip_fail(e, what);
    }
    if (ix) ix->device_bytes += bytes;
    return OS_ANN_OK;
}

void destroy_graph(GraphEntry& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
}

void drop_graphs(os_ann_index* ix) {
    for (auto& g : ix->graphs) destroy_graph(g);
    ix->graphs.clear();
}

void free_arena(os_ann_index* ix, GraphArena& a) {
    void* ptrs[] = {a.ws, a.q, a.oidx, a.odist, a.oncand, a.capped};
    for (void* p : ptrs) dev_free(p);
    ix->device_bytes -= a.ws_bytes + (size_t)a.cap_q * (ix->D * 4 + 20) + 8;
    a = GraphArena{a.s};
}

void release(os_ann_index* ix, bool synced = false) {
    if (!ix) return;
    if (!synced) (void)hipDeviceSynchronize();  // the blocks go back to the cache idle
    for (auto& t : ix->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    drop_graphs(ix);
    for (auto& a : ix->arenas) free_arena(ix, a);
    for (auto* t : ix->sub) release(t, true);
    void* ptrs[] = {ix->row_cone, ix->row_top,  ix->perm,       ix->sorted_cone, ix->offsets,
                    ix->planes,   ix->lexsub,   ix->maskord,    ix->binom,       ix->scratch,
                    ix->lp.poff,  ix->lp.ne_id, ix->lp.ne_cone, ix->lp.xl,       ix->lp.nrm,
                    ix->lp.ppos,  ix->lp.prow,  ix->lp.ipos,  ix->rot,      ix->rot_offsets, ix->rot_perm,   ix->xtop,
                    ix->planes_tab, ix->proj_mu, ix->proj_P, ix->ivf_cent, ix->rot_signs,
                    ix->sp_keys, ix->sp_hkeys, ix->sp_hval, ix->sp_filt, ix->binom64,
                    ix->pending_small, ix->pending_tmp};
    for (void* p : ptrs) dev_free(p);
    delete ix;
}

int check_shape(int64_t N, int32_t D, int32_t L, int64_t* n_cones, bool allow_sparse = false) {
    if (N < 1 || N >= (int64_t(1) << 31)) return fail(OS_ANN_EINVAL, "N must be in [1, 2^31)");
    if (D < 1 || D > kMaxD) return fail(OS_ANN_EINVAL, "D must be in [1, 256]");
    if (L < 1 || L > kMaxL || L > D) return fail(OS_ANN_EINVAL, "L must be in [1, min(D, 7)]");
    const int64_t nc = binom_host(D, L) << L;
    if (nc > kMaxCones && !allow_sparse) return fail(OS_ANN_ENOTSUP, "C(D,L)*2^L exceeds 2^24 cones");
    *n_cones = nc;
    return OS_ANN_OK;
}

bool dtype_ok(int32_t t) { return t == kF32 || t == kF16 || t == kU8; }
bool rerank_ok(int32_t r) { return r == 4 || r == 8 || r == 16; }

// Two words of pinned host memory per calling thread, for the flags a build
// reads back (allocated on first use, held until the process ends).
uint32_t* pinned_flags() {
    thread_local uint32_t* p = nullptr;
    if (!p && hipHostMalloc((void**)&p, 16, hipHostMallocDefault) != hipSuccess) p = nullptr;
    return p;
}

// The screens' dynamic LDS limits: set once per device (the attribute
// belongs to the device, not to an index).
hipError_t screen_lds_once() {
    static std::mutex mu;
    static std::set<int> set_on;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(mu);
    if (set_on.count(dev)) return hipSuccess;
    e = tiled_screen_max_lds();
    if (e == hipSuccess) e = cone_screen_max_lds();
    if (e == hipSuccess) set_on.insert(dev);
    return e;
}

// Builds the low-precision copy once per index.
int ensure_lowp(os_ann_index* ix, hipStream_t s) {
    std::lock_guard<std::mutex> g(ix->lowp_mu);
    LowpCopy& lp = ix->lp;
    if (lp.ready) return OS_ANN_OK;
    const int64_t nc = ix->n_cones;
    lp.dk = (int)align_up((size_t)ix->D, 32);
    lp.f16 = ix->dtype == kF16;
    uint32_t* tmp = nullptr;
    const size_t bytes0 = ix->device_bytes;
    // on failure every block of the copy goes back, so a later call starts afresh
    auto done = [&](int code) {
        if (code != OS_ANN_OK) {
            (void)hipDeviceSynchronize();
            for (void** q : {(void**)&lp.poff, (void**)&lp.ne_id, (void**)&lp.ne_cone, (void**)&lp.xl,
                             (void**)&lp.nrm, (void**)&lp.ppos, (void**)&lp.prow, (void**)&lp.ipos}) {
                dev_free(*q);
                *q = nullptr;
            }
            ix->device_bytes = bytes0;
        }
        dev_free(tmp);
        return code;
    };
    const int64_t scan_words = exclusive_scan_tmp_words(nc);
    int rc = dev_alloc(ix, (void**)&lp.poff, (size_t)(nc + 1) * 4, "poff");
    if (!rc) rc = dev_alloc(ix, (void**)&lp.ne_id, (size_t)(nc + 1) * 4, "ne_id");
    if (!rc) rc = dev_alloc(ix, (void**)&lp.ne_cone, (size_t)nc * 4, "ne_cone");
    if (!rc) rc = dev_alloc(nullptr, (void**)&tmp, (size_t)(2 * nc + scan_words) * 4, "lowp scratch");
    if (rc) return done(rc);
    hipError_t e = launch_lowp_layout(ix->offsets, nc, tmp, tmp + nc, tmp + 2 * nc, lp.poff, lp.ne_id,
                                      lp.ne_cone, s);
    if (e != hipSuccess) return done(hip_fail(e, "low-precision layout"));
    // Each non-empty cone rounds up to a multiple of 16 rows, so the copy
    // holds at most N + 15 min(cones, N) rows.  Where that bound is within a
    // quarter of N it sizes the copy (no wait for the exact count); else the
    // count is read first.
    const int64_t ne_max = std::min<int64_t>(nc, ix->N);
    if (15 * ne_max <= ix->N / 4) {
        lp.np = ix->N + 15 * ne_max;
    } else {
        uint32_t np32 = 0;
        e = hipMemcpyAsync(&np32, lp.poff + nc, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return done(hip_fail(e, "low-precision layout"));
        lp.np = np32;
    }
    const int64_t rows = lp.np + 16;  // at least 16 zero rows past the end
    rc = dev_alloc(ix, (void**)&lp.xl, (size_t)rows * lp.dk * 2, "xl");
    if (!rc) rc = dev_alloc(ix, (void**)&lp.nrm, (size_t)rows * 4, "nrm");
    if (!rc) rc = dev_alloc(ix, (void**)&lp.ppos, (size_t)rows * 4, "ppos");
    if (!rc) rc = dev_alloc(ix, (void**)&lp.prow, (size_t)rows * 4, "prow");
    if (!rc) rc = dev_alloc(ix, (void**)&lp.ipos, (size_t)ix->N * 4, "ipos");
    if (rc) return done(rc);
    e = launch_lowp_rows(ix->planes, ix->dtype, ix->N, ix->D, ix->nch, ix->sorted_cone, ix->offsets, nc, lp.poff,
                         ix->perm, lp.dk, lp.f16, lp.xl, lp.ppos, lp.prow, lp.ipos, lp.nrm, rows, s);
    if (e == hipSuccess) e = screen_lds_once();
    // a build that left its closing check here: its flags come back with
    // this one synchronisation (into pinned memory: the copy is queued
    // behind the build, not staged by the calling thread)
    uint32_t* host_small = pinned_flags();
    if (e == hipSuccess && ix->pending_small && !host_small) e = hipErrorOutOfMemory;
    if (e == hipSuccess && ix->pending_small)
        e = hipMemcpyAsync(host_small, ix->pending_small, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(hip_fail(e, "low-precision copy"));
    if (ix->pending_small) {
        dev_free(ix->pending_small);
        dev_free(ix->pending_tmp);
        ix->pending_small = ix->pending_tmp = nullptr;
        if (host_small[0]) return done(fail(OS_ANN_ENONFINITE, "database holds NaN or infinity"));
        ix->n_nonempty = host_small[1];
    }
    lp.ready = true;
    return done(OS_ANN_OK);
}

// ---------------------------------------------------------------------------
// search plans: byte offsets inside one scratch buffer
// ---------------------------------------------------------------------------
struct SearchPlan {
    int64_t Q = 0;
    int dpad = 0, mode = OS_ANN_MODE_FP32, R = 8;
    bool cones = false;  // fixed-C mode: the budget counts cones per walk
    size_t off_yf = 0, off_order = 0, off_sbit = 0, off_jstop = 0, off_np = 0, off_nc = 0;
    // tiled mode
    int dk = 0, smin = 1, smax = 1, mq = 0, G = 4;  // G: MFMA B groups per wave tile
    int qkey = 0;                                   // query order of the wave tiles (launch_query_key mode)
    int kern = 0;                                   // screen kernel: 0 query tiles x cone splits, 1 cone-major
    bool cone_ok = false;                           // the cone-major screen applies (bitmaps, dk, list memory)
    bool seed = true;                               // the seed pass runs (the tuner may drop it)
    int64_t T = 0, nw = 0;
    bool bitmap = false, fits = true;
    size_t off_ql = 0, off_qcone = 0, off_sort = 0, off_qorder = 0, off_qsorted = 0, off_part = 0,
           off_counter = 0, off_qbits = 0, off_cmin = 0, off_qkey = 0;
    size_t off_yr = 0;  // several bases: query coordinates [R][Q][D]
    size_t off_yk = 0;  // projected table: query keys [Q][Dk]
    // clustered table: per virtual query (query x searched cluster)
    size_t off_vyr = 0, off_vyf = 0, off_vbase = 0, off_vidx = 0, off_vdist = 0;
    int64_t Qv = 0;
    size_t bytes = 0;
};

// Non-empty cones per split for S splits: a multiple of 64 (whole bitmap words).
int64_t split_span(int64_t n_ne, int S) {
    const int64_t per = (n_ne + S - 1) / S;
    return (per + 63) / 64 * 64;
}

// Rows a walk is expected to take: the budget, or in fixed-C mode C cones of
// the mean non-empty bucket size.
int64_t expected_rows(const os_ann_index* ix, int64_t budget, bool cones) {
    if (!cones) return std::min<int64_t>(budget, ix->N);
    const int64_t mean = std::max<int64_t>(1, ix->N / std::max<int64_t>(1, ix->n_nonempty));
    return budget >= ix->N / mean ? ix->N : std::min<int64_t>(ix->N, budget * mean);
}

SearchPlan plan_search(const os_ann_index* ix, int64_t Q, int64_t budget, int mode, int R, bool cones, int G = 0) {
    SearchPlan p;
    p.Q = Q;
    p.mode = mode;
    p.R = R;
    p.cones = cones;
    p.dpad = ix->nch * ix->epc;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at = align_up(at + bytes, 256);
        return here;
    };
    p.off_yf = take((size_t)Q * p.dpad * sizeof(float));
    if (ix->sparse) {  // sparse table: walk state for the one-pass walk and scan
        p.mode = OS_ANN_MODE_FP32;
        p.Qv = Q;
        p.off_order = take((size_t)Q * ix->D);
        p.off_sbit = take((size_t)Q * ix->D);
        p.bytes = at;
        return p;
    }
    if (ix->n_rot > 0) {  // several bases: FP32 scan with per-basis walk state
        const size_t R = (size_t)ix->n_rot;
        p.mode = OS_ANN_MODE_FP32;
        p.off_yr = take(R * (size_t)Q * ix->D * sizeof(float));
        p.off_order = take(R * (size_t)Q * ix->D);
        p.off_sbit = take(R * (size_t)Q * ix->D);
        p.off_jstop = take((size_t)Q * sizeof(uint32_t));
        p.off_nc = take((size_t)Q * sizeof(int64_t));
        p.bytes = at;
        return p;
    }
    // walk state per query, or per (query, searched cluster) on a clustered table
    const int64_t Qw = ix->ivf_cent ? Q * ix->nprobe : Q;
    p.Qv = Qw;
    p.off_order = take((size_t)Qw * ix->Dk);
    p.off_sbit = take((size_t)Qw * ix->Dk);
    p.off_jstop = take((size_t)Qw * sizeof(uint32_t));
    p.off_np = take((size_t)Qw * sizeof(uint32_t));
    if (ix->proj) p.off_yk = take((size_t)Q * ix->Dk * sizeof(float));
    p.off_nc = take((size_t)Qw * sizeof(int64_t));
    if (ix->ivf_cent) {
        p.off_vyr = take((size_t)Qw * ix->D * sizeof(float));
        p.off_vyf = take((size_t)Qw * p.dpad * sizeof(float));
        p.off_vbase = take((size_t)Qw * sizeof(uint32_t));
        p.off_vidx = take((size_t)Qw * sizeof(int64_t));
        p.off_vdist = take((size_t)Qw * sizeof(float));
    }
    if (mode == OS_ANN_MODE_TILED) {
        const int64_t ne = ix->n_nonempty > 0 ? ix->n_nonempty : 1;
        p.dk = (int)align_up((size_t)ix->D, 32);
        p.G = G ? G : tile_groups(R);
        p.mq = 16 * p.G;
        p.T = (Q + p.mq - 1) / p.mq;
        p.nw = (ne + 63) / 64;
        // splits only add parallelism (up to about four wave items for each
        // of the 8 waves a compute unit holds); the tuner picks the count
        p.smin = 1;
        p.fits = tiled_screen_lds() + tiled_screen_static_lds(R, p.G) <= kLdsPerBlock;
        const int64_t want = (32 * (int64_t)ix->num_cu + p.T - 1) / (p.T > 0 ? p.T : 1);
        p.smax = (int)std::min<int64_t>(64, pow2_ceil(std::max<int64_t>(want, 1)));
        while (p.smax > 1 && split_span(ne, p.smax) < 64 * 2) p.smax >>= 1;
        // probed-cone bitmaps pay off once a query probes many cones and stay small
        const int64_t mean_bucket = std::max<int64_t>(1, ix->N / ne);
        const int64_t probes = cones ? std::min<int64_t>(budget, ne) : std::min<int64_t>(budget, ix->N) / mean_bucket + 1;
        const bool bitmap_fits = p.nw <= 512 && (size_t)Q * p.nw * 8 <= ((size_t)1 << 30);
        p.bitmap = probes >= 32 && bitmap_fits;
        // the cone-major screen keeps one top-R list per (query, 64-cone word);
        // OSANN_TILED_KERNEL=cone (testing) takes it at any probe count
        const char* kenv = std::getenv("OSANN_TILED_KERNEL");
        const bool force_cone = kenv && std::string(kenv) == "cone";
        p.cone_ok = (p.bitmap || (force_cone && bitmap_fits)) && cone_screen_ok(p.dk, R) &&
                    (size_t)Q * p.nw * R * 8 <= ((size_t)1 << 30);
        p.off_ql = take((size_t)Q * p.dk * 2);
        p.off_qcone = take((size_t)Q * 4);
        p.off_sort = take((size_t)(4 * Q + radix_hist_words(Q)) * 4);
        p.off_qorder = take((size_t)Q * 4);
        p.off_qkey = take((size_t)Q * 4);
        p.off_qsorted = take((size_t)Q * 4);
        p.off_part = take((size_t)Q * (p.cone_ok ? std::max<int64_t>(p.smax, p.nw) : p.smax) * R * 8);
        p.off_counter = take(256);
        p.off_cmin = take((size_t)Q * R * 4);
        if (p.bitmap || p.cone_ok) p.off_qbits = take((size_t)Q * p.nw * 8);
    }
    p.bytes = at;
    return p;
}

int search_checks(const os_ann_index* ix, const void* queries, int64_t Q, int64_t budget,
                  const os_ann_search_opts* o) {
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    if (Q < 0) return fail(OS_ANN_EINVAL, "Q must be >= 0");
    if (Q >= (int64_t(1) << 31)) return fail(OS_ANN_EINVAL, "Q must be below 2^31");
    if (budget < 1) return fail(OS_ANN_EINVAL, "max_candidates must be >= 1");
    if (Q > 0 && !queries) return fail(OS_ANN_EINVAL, "null queries");
    if (o) {
        if (!dtype_ok(o->query_dtype)) return fail(OS_ANN_EINVAL, "bad query dtype");
        if (o->mode != OS_ANN_MODE_FP32 && o->mode != OS_ANN_MODE_TILED)
            return fail(OS_ANN_EINVAL, "bad mode");
        if (o->mode == OS_ANN_MODE_TILED && !rerank_ok(o->rerank_r ? o->rerank_r : 8))
            return fail(OS_ANN_EINVAL, "rerank_r must be 4, 8 or 16");
        if (o->mode == OS_ANN_MODE_TILED && ix->n_rot > 0)
            return fail(OS_ANN_ENOTSUP, "several bases: FP32 mode only");
        if (o->mode == OS_ANN_MODE_TILED && ix->sparse)
            return fail(OS_ANN_ENOTSUP, "sparse table: FP32 mode only");
        if (o->mode == OS_ANN_MODE_TILED && ix->ivf_cent)
            return fail(OS_ANN_ENOTSUP, "clustered table: FP32 mode only");
    }
    return OS_ANN_OK;
}

// Returns scratch for a plan: the caller's workspace or the index's own.
int get_scratch(os_ann_index* ix, const os_ann_search_opts* o, size_t bytes, char** base) {
    if (o && o->workspace) {
        if (o->workspace_bytes < 0 || (size_t)o->workspace_bytes < bytes)
            return fail(OS_ANN_EINVAL, "workspace smaller than os_ann_workspace_bytes");
        *base = static_cast<char*>(o->workspace);
        return OS_ANN_OK;
    }
    std::lock_guard<std::mutex> g(ix->scratch_mu);
    if (ix->scratch_bytes < bytes) {
        if (ix->scratch) {
            OSANN_HIP(hipDeviceSynchronize(), "scratch resize");
            dev_free(ix->scratch);
            ix->device_bytes -= ix->scratch_bytes;
            ix->scratch = nullptr;
            ix->scratch_bytes = 0;
        }
        const size_t want = align_up(bytes + bytes / 4, 1 << 20);
        int rc = dev_alloc(ix, &ix->scratch, want, "search scratch");
        if (rc) return rc;
        ix->scratch_bytes = want;
    }
    *base = static_cast<char*>(ix->scratch);
    return OS_ANN_OK;
}

// Launches `fn` on stream s, bracketed by HIP events when timing is on.
template <typename F>
hipError_t timed_launch(os_ann_index* ix, bool on, int kernel, hipStream_t s, F&& fn) {
    if (!on) return fn();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        return e;
    }
    std::lock_guard<std::mutex> g(ix->time_mu);
    ix->timed.push_back({kernel, a, b});
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// autotuner of the tiled path: number of cone splits per query tile
// ---------------------------------------------------------------------------
struct Tuner {
    std::mutex mu;
    bool loaded = false;
    std::map<std::string, int> best;

    static const char* path() { return std::getenv("OSANN_TUNE_FILE"); }

    void load_locked() {
        if (loaded) return;
        loaded = true;
        const char* p = path();
        if (!p) return;
        FILE* f = std::fopen(p, "r");
        if (!f) return;
        char key[256];
        int s = 0;
        double ms = 0;
        while (std::fscanf(f, "%255s %d %lf", key, &s, &ms) == 3) best[key] = s;
        std::fclose(f);
    }
    int get(const std::string& k) {
        std::lock_guard<std::mutex> g(mu);
        load_locked();
        auto it = best.find(k);
        return it == best.end() ? 0 : it->second;
    }
    void put(const std::string& k, int s, double ms) {
        std::lock_guard<std::mutex> g(mu);
        load_locked();
        best[k] = s;
        if (const char* p = path()) {
            if (FILE* f = std::fopen(p, "a")) {
                std::fprintf(f, "%s %d %.4f\n", k.c_str(), s, ms);
                std::fclose(f);
            }
        }
    }
};
Tuner g_tuner;

std::string tune_key(const os_ann_index* ix, const SearchPlan& p, int64_t budget) {
    const int64_t qb = pow2_ceil(p.Q);
    const int64_t bb = pow2_ceil(std::min<int64_t>(budget, ix->N));
    char buf[256];
    std::snprintf(buf, sizeof buf, "gfx950:D%d:L%d:t%d:R%d:ne%lld:N%lld:Q%lld:B%lld%s", ix->D, ix->L, ix->dtype,
                  p.R, (long long)ix->n_nonempty, (long long)pow2_ceil(ix->N), (long long)qb, (long long)bb,
                  p.cones ? ":cones" : "");
    return buf;
}

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------
struct Call {
    os_ann_index* ix;
    const void* queries;
    int qtype;
    int64_t Q, budget;
    int64_t* out_idx;
    float* out_dist;
    int64_t* out_ncand;
    int64_t* walks_capped;  // sparse tables: capped walks counted here (may be null)
    char* base;
    SearchPlan p;
    bool timing;
    hipStream_t s;
};

ProbeArgs probe_args(const Call& c) {
    const os_ann_index* ix = c.ix;
    ProbeArgs pa{};
    pa.Y = c.queries;
    pa.qtype = c.qtype;
    pa.Q = c.Q;
    pa.D = ix->Dk;
    pa.L = ix->L;
    pa.offsets = ix->offsets;
    pa.n_cones = ix->n_cones;
    pa.n_sub = ix->n_sub;
    pa.N = ix->N;
    pa.budget = c.budget;
    pa.lexsub = ix->lexsub;
    pa.maskord = ix->maskord;
    pa.binom = ix->binom;
    pa.yf = reinterpret_cast<float*>(c.base + c.p.off_yf);
    pa.dpad = c.p.dpad;
    pa.order = reinterpret_cast<uint8_t*>(c.base + c.p.off_order);
    pa.sbit = reinterpret_cast<uint8_t*>(c.base + c.p.off_sbit);
    pa.jstop = reinterpret_cast<uint32_t*>(c.base + c.p.off_jstop);
    pa.nprobe = reinterpret_cast<uint32_t*>(c.base + c.p.off_np);
    pa.ncand = c.out_ncand ? c.out_ncand : reinterpret_cast<int64_t*>(c.base + c.p.off_nc);
    if (c.p.mode == OS_ANN_MODE_TILED) {
        pa.ql = reinterpret_cast<uint16_t*>(c.base + c.p.off_ql);
        pa.dk = c.p.dk;
        pa.ql_f16 = ix->lp.f16;
        pa.q_cone = reinterpret_cast<uint32_t*>(c.base + c.p.off_qcone);
        if (c.p.bitmap) {
            pa.qbits = reinterpret_cast<uint64_t*>(c.base + c.p.off_qbits);
            pa.nw = c.p.nw;
            pa.ne_id = ix->lp.ne_id;
            pa.n_ne = ix->n_nonempty;
        }
    }
    return pa;
}

// Walk lengths.  Row budget: the probe kernel finds them.  Fixed-C mode
// (Section 3, Table III): the probe kernel only ranks each walk's query (its
// length outputs left out), then the cones kernel takes the first C
// positions and counts the non-empty cones and their rows.
hipError_t launch_walk(const ProbeArgs& pa, bool cones, int64_t take, hipStream_t s) {
    if (!cones) return launch_probe(pa, s);
    ProbeArgs pr = pa;
    pr.jstop = nullptr;
    pr.nprobe = nullptr;
    pr.ncand = nullptr;
    pr.qbits = nullptr;
    hipError_t e = launch_probe(pr, s);
    if (e != hipSuccess) return e;
    ConesArgs ca{};
    ca.Q = pa.Q;
    ca.D = pa.D;
    ca.L = pa.L;
    ca.n_cones = pa.n_cones;
    ca.n_sub = pa.n_sub;
    ca.take = take;
    ca.offsets = pa.offsets;
    ca.cone_base = pa.cone_base;
    ca.lexsub = pa.lexsub;
    ca.maskord = pa.maskord;
    ca.binom = pa.binom;
    ca.order = pa.order;
    ca.sbit = pa.sbit;
    ca.jstop = pa.jstop;
    ca.nprobe = pa.nprobe;
    ca.ncand = pa.ncand;
    ca.qbits = pa.qbits;
    ca.nw = pa.nw;
    ca.ne_id = pa.ne_id;
    return launch_cones(ca, s);
}

hipError_t enqueue_fp32(const Call& c) {
    os_ann_index* ix = c.ix;
    const ProbeArgs pa = probe_args(c);
    hipError_t e;
    if (ix->proj) {
        // the FP32 copy of the queries (all D components), their keys, then
        // the walk on the keys
        ProbeArgs pf{};
        pf.Y = c.queries;
        pf.qtype = c.qtype;
        pf.Q = c.Q;
        pf.D = ix->D;
        pf.L = ix->L;
        pf.yf = pa.yf;
        pf.dpad = pa.dpad;
        ProbeArgs pk = pa;
        float* yk = reinterpret_cast<float*>(c.base + c.p.off_yk);
        pk.Y = yk;
        pk.qtype = kF32;
        pk.yf = nullptr;
        e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s, [&] {
            hipError_t r = launch_probe(pf, c.s);
            if (r == hipSuccess)
                r = launch_project(c.queries, c.qtype, c.Q, ix->D, ix->proj_mu, ix->proj_P, ix->Dk, yk, c.s);
            if (r == hipSuccess) r = launch_walk(pk, c.p.cones, c.budget, c.s);
            return r;
        });
    } else {
        e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s,
                         [&] { return launch_walk(pa, c.p.cones, c.budget, c.s); });
    }
    if (e != hipSuccess) return e;
    ScanArgs sa{};
    sa.planes = ix->planes;
    sa.dtype = ix->dtype;
    sa.N = ix->N;
    sa.D = ix->Dk;  // the walk state's length
    sa.L = ix->L;
    sa.nch = ix->nch;
    sa.yf = pa.yf;
    sa.Q = c.Q;
    sa.order = pa.order;
    sa.sbit = pa.sbit;
    sa.jstop = pa.jstop;
    sa.offsets = ix->offsets;
    sa.n_sub = ix->n_sub;
    sa.lexsub = ix->lexsub;
    sa.maskord = ix->maskord;
    sa.binom = ix->binom;
    sa.perm = ix->perm;
    sa.out_idx = c.out_idx;
    sa.out_dist = c.out_dist;
    sa.waves_per_query = expected_rows(ix, c.budget, c.p.cones) <= 8192 ? 1 : 4;
    return timed_launch(ix, c.timing, OS_ANN_KERNEL_SCAN, c.s, [&] { return launch_scan_fp32(sa, c.s); });
}

hipError_t enqueue_tiled(const Call& c, int S) {
    os_ann_index* ix = c.ix;
    const SearchPlan& p = c.p;
    const ProbeArgs pa = probe_args(c);
    hipError_t e;
    ix->last_kern = p.kern;
    ix->last_order = p.qkey;
    ix->last_groups = p.kern == 1 ? 4 : p.G;
    ix->last_splits = p.kern == 1 ? (int32_t)p.nw : S;
    if (ix->proj) {
        // keyed table: the FP32 and low-precision copies of the full queries,
        // their keys, then the walk on the keys
        ProbeArgs pf{};
        pf.Y = c.queries;
        pf.qtype = c.qtype;
        pf.Q = c.Q;
        pf.D = ix->D;
        pf.L = ix->L;
        pf.yf = pa.yf;
        pf.dpad = pa.dpad;
        pf.ql = pa.ql;
        pf.dk = pa.dk;
        pf.ql_f16 = pa.ql_f16;
        ProbeArgs pk = pa;
        float* yk = reinterpret_cast<float*>(c.base + p.off_yk);
        pk.Y = yk;
        pk.qtype = kF32;
        pk.yf = nullptr;
        pk.ql = nullptr;
        e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s, [&] {
            hipError_t r = launch_probe(pf, c.s);
            if (r == hipSuccess)
                r = launch_project(c.queries, c.qtype, c.Q, ix->D, ix->proj_mu, ix->proj_P, ix->Dk, yk, c.s);
            if (r == hipSuccess) r = launch_walk(pk, c.p.cones, c.budget, c.s);
            return r;
        });
    } else {
        e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s,
                         [&] { return launch_walk(pa, c.p.cones, c.budget, c.s); });
    }
    if (e != hipSuccess) return e;
    uint32_t* qorder = reinterpret_cast<uint32_t*>(c.base + p.off_qorder);
    {
        // wave tiles of queries with equal keys (launch_query_key): own cone
        // and next component (where that fits 32 bits), or sign bits
        const uint32_t* key = pa.q_cone;
        int64_t nb = ix->n_cones;
        const int64_t nb0 = ix->n_cones * 2 * ix->Dk;
        if (ix->L < ix->Dk && (p.qkey == 1 || nb0 <= (int64_t(1) << 32))) {
            uint32_t* kb = reinterpret_cast<uint32_t*>(c.base + p.off_qkey);
            e = launch_query_key(pa.q_cone, pa.order, pa.sbit, c.Q, ix->Dk, ix->L, p.qkey, kb, c.s);
            if (e != hipSuccess) return e;
            key = kb;
            nb = p.qkey == 1 ? (int64_t(1) << query_sign_bits(ix->Dk, c.Q)) : nb0;
        }
        e = launch_sort_by_cone(key, c.Q, nb, reinterpret_cast<uint32_t*>(c.base + p.off_sort), qorder,
                                reinterpret_cast<uint32_t*>(c.base + p.off_qsorted), c.s);
    }
    if (e != hipSuccess) return e;
    uint32_t* counter = reinterpret_cast<uint32_t*>(c.base + p.off_counter);
    e = launch_fill_u32(counter, kXcd, 0u, c.s);
    if (e != hipSuccess) return e;
    uint32_t* cmin = reinterpret_cast<uint32_t*>(c.base + p.off_cmin);
    e = launch_fill_u32(cmin, c.Q * p.R, 0xFFFFFFFFu, c.s);
    if (e != hipSuccess) return e;
    SeedArgs sd{};
    sd.xl = ix->lp.xl;
    sd.nrm = ix->lp.nrm;
    sd.poff = ix->lp.poff;
    sd.dk = ix->lp.dk;
    sd.ql = pa.ql;
    sd.qorder = qorder;
    sd.Q = c.Q;
    sd.cmin = cmin;
    sd.order = pa.order;
    sd.sbit = pa.sbit;
    sd.jstop = pa.jstop;
    sd.lexsub = ix->lexsub;
    sd.maskord = ix->maskord;
    sd.binom = ix->binom;
    sd.n_sub = ix->n_sub;
    sd.n_cones = ix->n_cones;
    sd.D = ix->Dk;  // the walk state's length
    sd.L = ix->L;
    // The seed reads up to sd.rows padded rows from the first cones of each
    // query's walk, one query at a time (no row is shared between queries):
    // keep that near a sixteenth of the budget, 64 .. 192 rows.  Past 192
    // the seed costs more than its tighter bound saves the screen (1e6 x 64
    // Gaussian rows, 1e4 queries, budget 327,680, cone-major screen: 2.01 /
    // 1.98 / 1.98 / 2.00 / 2.04 ms per search at 64 / 128 / 192 / 256 / 512
    // rows).
    const int64_t rows = expected_rows(ix, c.budget, p.cones);
    sd.rows = (int)std::min<int64_t>(192, std::max<int64_t>(64, pow2_ceil(std::max<int64_t>(rows / 16, 1))));
    bool seed = p.seed;
    if (const char* env = std::getenv("OSANN_TILED_SEED_ROWS")) {  // fixed seed size, 0: none (testing)
        const int v = std::atoi(env);
        if (v >= 64 && v <= 1024 && v % 64 == 0) sd.rows = v;
        if (std::string(env) == "0") seed = false;
    }
    // without the seed the class minima start at +inf (a valid bound that
    // discards nothing): the tuner drops it where the screen gains less
    // than the seed costs (many queries, short candidate lists)
    if (seed) e = launch_tiled_seed(sd, p.R, ix->lp.f16, c.s);
    if (e != hipSuccess) return e;
    TiledArgs ta{};
    ta.xl = ix->lp.xl;
    ta.dk = ix->lp.dk;
    ta.nrm = ix->lp.nrm;
    ta.prow = ix->lp.prow;
    ta.poff = ix->lp.poff;
    ta.offsets = ix->offsets;
    ta.ne_id = ix->lp.ne_id;
    ta.ne_cone = ix->lp.ne_cone;
    ta.n_ne = ix->n_nonempty;
    ta.lexsub = ix->lexsub;
    ta.maskord = ix->maskord;
    ta.binom = ix->binom;
    ta.n_sub = ix->n_sub;
    ta.D = ix->Dk;  // the walk state's length (the keys' on a keyed table)
    ta.L = ix->L;
    ta.ql = pa.ql;
    ta.Q = c.Q;
    ta.qorder = qorder;
    ta.order = pa.order;
    ta.sbit = pa.sbit;
    ta.jstop = pa.jstop;
    ta.qbits = pa.qbits;
    ta.nw = p.nw;
    ta.T = p.T;
    ta.S = S;
    ta.span = split_span(ix->n_nonempty > 0 ? ix->n_nonempty : 1, S);
    ta.counter = counter;
    ta.part = reinterpret_cast<uint2*>(c.base + p.off_part);
    ta.cmin = cmin;
    const size_t lds = tiled_screen_lds();
    int occ = tiled_screen_occupancy(p.R, p.G, ix->lp.f16, ix->lp.dk / 32, lds);
    if (occ < 1) occ = 1;
    const int64_t items = p.T * S;  // one wave each, 4 waves per block
    // a multiple of kXcd blocks, so that every chiplet queue has blocks
    const int64_t cap = std::max<int64_t>(kXcd, (int64_t)occ * ix->num_cu / kXcd * kXcd);
    const int blocks = (int)std::min<int64_t>(cap, ((items + 3) / 4 + kXcd - 1) / kXcd * kXcd);
    if (std::getenv("OSANN_VERBOSE"))
        std::fprintf(stderr, "[osann] tiled Q=%lld T=%lld G=%d S=%d span=%lld lds=%zu occ=%d blocks=%d bitmap=%d R=%d\n",
                     (long long)c.Q, (long long)p.T, p.G, S, (long long)ta.span, lds, occ, blocks, (int)p.bitmap, p.R);
    if (p.kern == 1) {
        ta.S = (int)p.nw;  // one list per (query, 64-cone word)
        e = timed_launch(ix, c.timing, OS_ANN_KERNEL_SCREEN, c.s,
                         [&] { return launch_cone_screen(ta, p.R, ix->lp.f16, c.s); });
    } else {
        e = timed_launch(ix, c.timing, OS_ANN_KERNEL_SCREEN, c.s,
                         [&] { return launch_tiled_screen(ta, p.R, p.G, ix->lp.f16, blocks, c.s); });
    }
    if (e != hipSuccess) return e;
    FinishArgs fa{};
    fa.part = ta.part;
    fa.S = ta.S;
    fa.Q = c.Q;
    fa.planes = ix->planes;
    fa.dtype = ix->dtype;
    fa.N = ix->N;
    fa.nch = ix->nch;
    fa.ppos = ix->lp.ppos;
    fa.ipos = ix->lp.ipos;
    fa.yf = pa.yf;
    fa.dpad = p.dpad;
    // the codes hold FP16 rows and uint8 rows exactly (FP32 rows: planes)
    fa.xl = ix->lp.xl;
    fa.dk = ix->lp.dk;
    fa.xl_codes = ix->dtype == kF16 && ix->lp.f16 ? 1 : ix->dtype == kU8 && !ix->lp.f16 ? 2 : 0;
    fa.out_idx = c.out_idx;
    fa.out_dist = c.out_dist;
    return timed_launch(ix, c.timing, OS_ANN_KERNEL_FINISH, c.s, [&] { return launch_tiled_finish(fa, p.R, c.s); });
}

// Plans of the tiled path: the query-tile screen for every tile width and
// the cone-major screen (where the probe bitmaps exist), each for both query
// orders; the default first.
constexpr int kMaxPlans = 8;
int tiled_plans(const os_ann_index* ix, int64_t Q, int64_t budget, int R, bool cones, SearchPlan (&plans)[kMaxPlans]) {
    int n = 0;
    const char* genv = std::getenv("OSANN_TILED_GROUPS");  // fixed tile width (testing)
    const char* oenv = std::getenv("OSANN_TILED_ORDER");   // fixed query order (testing)
    const char* kenv = std::getenv("OSANN_TILED_KERNEL");  // fixed screen kernel (testing): tile | cone
    const int gfix = genv && tile_groups_ok(R, std::atoi(genv)) ? std::atoi(genv) : 0;
    const int ofix = oenv && (std::atoi(oenv) == 0 || std::atoi(oenv) == 1) ? std::atoi(oenv) + 1 : 0;
    const int kfix = kenv ? (std::string(kenv) == "cone" ? 2 : std::string(kenv) == "tile" ? 1 : 0) : 0;
    const SearchPlan def = plan_search(ix, Q, budget, OS_ANN_MODE_TILED, R, cones, gfix);
    for (int qk = 0; qk < 2; ++qk) {
        if (ofix && qk != ofix - 1) continue;
        if (def.cone_ok && kfix != 1) {
            plans[n] = def;
            plans[n].qkey = qk;
            plans[n].fits = true;  // its LDS use depends on dk only (at most 32 KB of queries)
            plans[n].bitmap = true;    // it finds each cone's queries in the bitmaps
            plans[n++].kern = 1;
        }
        if (kfix == 2 && def.cone_ok) continue;
        for (int G : {def.G, def.G == 4 ? 2 : 4}) {
            if (!tile_groups_ok(R, G) || (gfix && G != gfix)) continue;
            plans[n] = plan_search(ix, Q, budget, OS_ANN_MODE_TILED, R, cones, G);
            plans[n++].qkey = qk;
        }
    }
    return n;
}

// Picks the tile width G and split count S of the tiled path and leaves c.p
// as the plan of that G: OSANN_TILED_SPLITS (testing) fixes S with the
// default G; else the cached choice; else both are timed over every
// candidate pair (each computes the same result, so the outputs of the last
// run are valid); else (during capture) the default G and the smallest S.
int choose_tiling(Call& c, const SearchPlan* plans, int n_plans, bool may_time, hipError_t* err) {
    // the choice is cached as (no seed << 24) | (kernel << 20) | (query order << 16) | (G << 12) | S
    *err = hipSuccess;
    c.p = plans[0];
    if (const char* env = std::getenv("OSANN_TILED_SPLITS")) {  // fixed split count (testing)
        const int v = std::atoi(env);
        for (int k = 0; k < n_plans; ++k)
            if (plans[k].kern == 0 && v >= plans[k].smin && v <= plans[k].smax && (v & (v - 1)) == 0) {
                c.p = plans[k];
                return v;
            }
    }
    // testing overrides narrow the candidates: their choices are cached
    // under keys of their own, never as the unrestricted choice
    std::string key = tune_key(c.ix, plans[0], c.budget) + ":KOGSD";
    for (const char* var : {"OSANN_TILED_GROUPS", "OSANN_TILED_ORDER", "OSANN_TILED_KERNEL"})
        if (const char* v = std::getenv(var)) key += std::string(":") + var + "=" + v;
    if (int v = g_tuner.get(key)) {
        for (int k = 0; k < n_plans; ++k) {
            const SearchPlan& pk = plans[k];
            if (!pk.fits || pk.kern != ((v >> 20) & 0xF) || pk.qkey != ((v >> 16) & 0xF)) continue;
            if (pk.kern == 1) {
                c.p = pk;
                c.p.seed = !((v >> 24) & 1);
                return (int)pk.nw;
            }
            if (pk.G == ((v >> 12) & 0xF) && (v & 0xFFF) >= pk.smin && (v & 0xFFF) <= pk.smax) {
                c.p = pk;
                c.p.seed = !((v >> 24) & 1);
                return v & 0xFFF;
            }
        }
    }
    if (!may_time) return c.p.kern == 1 ? (int)c.p.nw : c.p.smin;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int best_k = 0, best_s = plans[0].kern == 1 ? (int)plans[0].nw : plans[0].smin;
    float best_ms = 1e30f;
    const bool timing = c.timing;
    c.timing = false;
    for (int k = 0; k < n_plans && e == hipSuccess; ++k) {
        if (!plans[k].fits) continue;
        c.p = plans[k];
        const int s_lo = c.p.kern == 1 ? (int)c.p.nw : c.p.smin;
        const int s_hi = c.p.kern == 1 ? (int)c.p.nw : c.p.smax;
        for (int s = s_lo; s <= s_hi && e == hipSuccess; s = c.p.kern == 1 ? s_hi + 1 : s << 1) {
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // first run warms caches
                e = hipEventRecord(a, c.s);
                if (e == hipSuccess) e = enqueue_tiled(c, s);
                if (e == hipSuccess) e = hipEventRecord(b, c.s);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                if (e == hipSuccess && rep == 1 && ms < best_ms) {
                    best_ms = ms;
                    best_k = k;
                    best_s = s;
                }
            }
        }
    }
    // the best plan again without the seed pass
    c.p = plans[best_k];
    bool seed = true;
    c.p.seed = false;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = hipEventRecord(a, c.s);
        if (e == hipSuccess) e = enqueue_tiled(c, best_s);
        if (e == hipSuccess) e = hipEventRecord(b, c.s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && rep == 1 && ms < best_ms) {
            best_ms = ms;
            seed = false;
        }
    }
    c.timing = timing;
    c.p = plans[best_k];
    c.p.seed = seed;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    *err = e;
    if (e == hipSuccess)
        g_tuner.put(key,
                    ((seed ? 0 : 1) << 24) | (plans[best_k].kern << 20) | (plans[best_k].qkey << 16) |
                        (plans[best_k].G << 12) | best_s,
                    best_ms);
    return best_s;
}

// Several bases: FP32 queries, coordinates in every basis, interleaved walk
// length, then the scan that analyzes each row once.
hipError_t enqueue_rot(const Call& c) {
    os_ann_index* ix = c.ix;
    const SearchPlan& p = c.p;
    const int R = ix->n_rot;
    ProbeArgs pa{};
    pa.Y = c.queries;
    pa.qtype = c.qtype;
    pa.Q = c.Q;
    pa.D = ix->D;
    pa.L = ix->L;
    pa.yf = reinterpret_cast<float*>(c.base + p.off_yf);
    pa.dpad = p.dpad;
    float* yr = reinterpret_cast<float*>(c.base + p.off_yr);
    hipError_t e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s, [&] {
        hipError_t r = launch_probe(pa, c.s);
        for (int b = 0; b < R && r == hipSuccess; ++b)
            r = ix->rot_signs ? launch_wht(c.queries, c.qtype, c.Q, ix->D, ix->rot_signs + (size_t)b * ix->D,
                                           yr + (size_t)b * c.Q * ix->D, c.s)
                              : launch_rotate(c.queries, c.qtype, c.Q, ix->D, ix->rot + (size_t)b * ix->D * ix->D,
                                              yr + (size_t)b * c.Q * ix->D, c.s);
        return r;
    });
    if (e != hipSuccess) return e;
    RotArgs ra{};
    ra.N = ix->N;
    ra.D = ix->D;
    ra.L = ix->L;
    ra.R = R;
    ra.nch = ix->nch;
    ra.dtype = ix->dtype;
    ra.dpad = p.dpad;
    ra.n_cones = ix->n_cones;
    ra.n_sub = ix->n_sub;
    ra.offsets = ix->rot_offsets;
    ra.perm = ix->rot_perm;
    ra.xtop = ix->xtop;
    ra.planes_tab = reinterpret_cast<const uint4* const*>(ix->planes_tab);
    ra.waves_per_query = expected_rows(ix, c.budget, p.cones) <= 8192 ? 1 : 4;
    ra.lexsub = ix->sub[0]->lexsub;
    ra.maskord = ix->sub[0]->maskord;
    ra.binom = ix->sub[0]->binom;
    ra.Q = c.Q;
    ra.budget = c.budget;
    ra.yr = yr;
    ra.yf = pa.yf;
    ra.order = reinterpret_cast<uint8_t*>(c.base + p.off_order);
    ra.sbit = reinterpret_cast<uint8_t*>(c.base + p.off_sbit);
    ra.kstop = reinterpret_cast<uint32_t*>(c.base + p.off_jstop);
    ra.visited = reinterpret_cast<int64_t*>(c.base + p.off_nc);
    ra.out_idx = c.out_idx;
    ra.out_dist = c.out_dist;
    ra.out_ncand = c.out_ncand;
    e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s, [&] {
        hipError_t r = launch_probe_rot(ra, c.s);
        // fixed-C mode: levels 0..C-1 of every basis
        if (r == hipSuccess && p.cones)
            r = launch_fill_u32(ra.kstop, c.Q, (uint32_t)(std::min<int64_t>(c.budget, ix->n_cones) * R), c.s);
        return r;
    });
    if (e != hipSuccess) return e;
    return timed_launch(ix, c.timing, OS_ANN_KERNEL_SCAN, c.s, [&] { return launch_scan_rot(ra, c.s); });
}

// Clustered table: the FP32 queries, their nprobe nearest clusters and
// residuals, the walk and scan of every (query, cluster) pair as its own
// query with its cluster's bucket base, then the best pair per query.
hipError_t enqueue_ivf(const Call& c) {
    os_ann_index* ix = c.ix;
    const SearchPlan& p = c.p;
    const int np = ix->nprobe;
    ProbeArgs pf{};
    pf.Y = c.queries;
    pf.qtype = c.qtype;
    pf.Q = c.Q;
    pf.D = ix->D;
    pf.L = ix->L;
    pf.yf = reinterpret_cast<float*>(c.base + p.off_yf);
    pf.dpad = p.dpad;
    IvfQueryArgs ia{};
    ia.yf = pf.yf;
    ia.dpad = p.dpad;
    ia.D = ix->D;
    ia.Q = c.Q;
    ia.cent = ix->ivf_cent;
    ia.C = ix->n_groups;
    ia.nprobe = np;
    ia.n_cones = ix->n_cones;
    ia.yr = reinterpret_cast<float*>(c.base + p.off_vyr);
    ia.yfv = reinterpret_cast<float*>(c.base + p.off_vyf);
    ia.cone_base = reinterpret_cast<uint32_t*>(c.base + p.off_vbase);
    ProbeArgs pk{};
    pk.Y = ia.yr;
    pk.qtype = kF32;
    pk.Q = p.Qv;
    pk.D = ix->D;
    pk.L = ix->L;
    pk.offsets = ix->offsets;
    pk.n_cones = ix->n_cones;
    pk.n_sub = ix->n_sub;
    pk.N = INT64_MAX;  // a cluster's walk never takes the whole database
    pk.budget = (c.budget + np - 1) / np;
    pk.lexsub = ix->lexsub;
    pk.maskord = ix->maskord;
    pk.binom = ix->binom;
    pk.order = reinterpret_cast<uint8_t*>(c.base + p.off_order);
    pk.sbit = reinterpret_cast<uint8_t*>(c.base + p.off_sbit);
    pk.jstop = reinterpret_cast<uint32_t*>(c.base + p.off_jstop);
    pk.nprobe = reinterpret_cast<uint32_t*>(c.base + p.off_np);
    pk.ncand = reinterpret_cast<int64_t*>(c.base + p.off_nc);
    pk.cone_base = ia.cone_base;
    hipError_t e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s, [&] {
        hipError_t r = launch_probe(pf, c.s);
        if (r == hipSuccess) r = launch_ivf_queries(ia, c.s);
        if (r == hipSuccess) r = launch_walk(pk, p.cones, c.budget, c.s);
        return r;
    });
    if (e != hipSuccess) return e;
    ScanArgs sa{};
    sa.planes = ix->planes;
    sa.dtype = ix->dtype;
    sa.N = ix->N;
    sa.D = ix->D;
    sa.L = ix->L;
    sa.nch = ix->nch;
    sa.yf = ia.yfv;
    sa.Q = p.Qv;
    sa.order = pk.order;
    sa.sbit = pk.sbit;
    sa.jstop = pk.jstop;
    sa.offsets = ix->offsets;
    sa.n_sub = ix->n_sub;
    sa.lexsub = ix->lexsub;
    sa.maskord = ix->maskord;
    sa.binom = ix->binom;
    sa.perm = ix->perm;
    sa.cone_base = ia.cone_base;
    int64_t* vidx = reinterpret_cast<int64_t*>(c.base + p.off_vidx);
    float* vdist = reinterpret_cast<float*>(c.base + p.off_vdist);
    sa.out_idx = vidx;
    sa.out_dist = vdist;
    sa.waves_per_query = (p.cones ? expected_rows(ix, c.budget, true) : std::min<int64_t>(pk.budget, ix->N)) <= 8192
                             ? 1
                             : 4;
    e = timed_launch(ix, c.timing, OS_ANN_KERNEL_SCAN, c.s, [&] {
        hipError_t r = launch_scan_fp32(sa, c.s);
        if (r == hipSuccess)
            r = launch_ivf_combine(vidx, vdist, pk.ncand, c.Q, np, c.out_idx, c.out_dist, c.out_ncand, c.s);
        return r;
    });
    return e;
}

// Sparse table: the probe kernel ranks the queries (walk state, FP32 copy),
// then one pass walks the cones and scans their rows.
hipError_t enqueue_sparse(const Call& c) {
    os_ann_index* ix = c.ix;
    const SearchPlan& p = c.p;
    ProbeArgs pa{};
    pa.Y = c.queries;
    pa.qtype = c.qtype;
    pa.Q = c.Q;
    pa.D = ix->D;
    pa.L = ix->L;
    pa.N = ix->N;
    pa.yf = reinterpret_cast<float*>(c.base + p.off_yf);
    pa.dpad = p.dpad;
    pa.order = reinterpret_cast<uint8_t*>(c.base + p.off_order);
    pa.sbit = reinterpret_cast<uint8_t*>(c.base + p.off_sbit);
    SparseTable t{};
    t.hkeys = ix->sp_hkeys;
    t.hval = ix->sp_hval;
    t.hmask = ix->sp_cap - 1;
    t.filt = ix->sp_filt;
    t.fmask = ix->sp_fbits - 1;
    t.offsets = ix->offsets;
    t.binom = ix->binom64;
    t.maskord = ix->maskord;
    t.n_sub = ix->n_sub;
    t.n_cones = ix->n_cones;
    t.N = ix->N;
    t.D = ix->D;
    t.L = ix->L;
    hipError_t e = timed_launch(ix, c.timing, OS_ANN_KERNEL_PROBE, c.s, [&] { return launch_probe(pa, c.s); });
    if (e != hipSuccess) return e;
    SparseSearchArgs sa{};
    sa.t = t;
    sa.planes = ix->planes;
    sa.dtype = ix->dtype;
    sa.nch = ix->nch;
    sa.yf = pa.yf;
    sa.dpad = p.dpad;
    sa.order = pa.order;
    sa.sbit = pa.sbit;
    sa.perm = ix->perm;
    sa.Q = c.Q;
    sa.budget = c.budget;
    sa.cones = p.cones ? 1 : 0;
    sa.out_idx = c.out_idx;
    sa.out_dist = c.out_dist;
    sa.out_ncand = c.out_ncand;
    sa.out_capped = reinterpret_cast<unsigned long long*>(c.walks_capped);
    if (c.walks_capped) {  // zeroed by a fill kernel (the sequence stays graph-capturable)
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(c.walks_capped), 2, 0u, c.s);
        if (e != hipSuccess) return e;
    }
    return timed_launch(ix, c.timing, OS_ANN_KERNEL_SCAN, c.s, [&] { return launch_sparse_search(sa, c.s); });
}

hipError_t enqueue(const Call& c, int S) {
    if (c.ix->sparse) return enqueue_sparse(c);
    if (c.ix->n_rot > 0) return enqueue_rot(c);
    if (c.ix->ivf_cent) return enqueue_ivf(c);
    return c.p.mode == OS_ANN_MODE_TILED ? enqueue_tiled(c, S) : enqueue_fp32(c);
}

// Query count of a graph class: Q rounded up to one of eight steps per
// octave (at most 1/8 of padding rows), 8 and 16 below that.
int64_t graph_class(int64_t Q) {
    if (Q <= 8) return 8;
    if (Q <= 16) return 16;
    int k = 0;
    while ((int64_t(1) << (k + 1)) < Q) ++k;  // 2^k < Q <= 2^(k+1)
    const int64_t step = (int64_t(1) << k) / 8;
    return (Q + step - 1) / step * step;
}

// The arena of stream s, grown to hold Qc query rows and `bytes` of scratch.
// Growing it frees the old buffers (after the stream has drained) and drops
// the stream's graphs, which point into them.
int graph_arena(os_ann_index* ix, hipStream_t s, int64_t Qc, size_t bytes, GraphArena** out) {
    GraphArena* a = nullptr;
    for (auto& e : ix->arenas)
        if (e.s == s) a = &e;
    if (!a) {
        ix->arenas.push_back(GraphArena{s});
        a = &ix->arenas.back();
    }
    if (a->cap_q >= Qc && a->ws_bytes >= bytes) {
        *out = a;
        return OS_ANN_OK;
    }
    OSANN_HIP(hipStreamSynchronize(s), "graph arena resize");
    for (auto it = ix->graphs.begin(); it != ix->graphs.end();) {
        if (it->key[0] == (int64_t)(intptr_t)s) {
            destroy_graph(*it);
            it = ix->graphs.erase(it);
        } else {
            ++it;
        }
    }
    const int64_t cap = std::max(Qc, a->cap_q);
    const size_t ws = std::max(align_up(bytes + bytes / 4, 1 << 20), a->ws_bytes);
    free_arena(ix, *a);
    int rc = OS_ANN_OK;
    if ((rc = dev_alloc(nullptr, (void**)&a->ws, ws, "graph scratch")) ||
        (rc = dev_alloc(nullptr, &a->q, (size_t)cap * ix->D * 4, "graph queries")) ||
        (rc = dev_alloc(nullptr, (void**)&a->oidx, (size_t)cap * 8, "graph rows")) ||
        (rc = dev_alloc(nullptr, (void**)&a->odist, (size_t)cap * 4, "graph distances")) ||
        (rc = dev_alloc(nullptr, (void**)&a->oncand, (size_t)cap * 8, "graph counts")) ||
        (rc = dev_alloc(nullptr, (void**)&a->capped, 8, "graph capped count"))) {
        free_arena(ix, *a);  // nothing counted yet: the sizes are still zero
        return rc;
    }
    a->cap_q = cap;
    a->ws_bytes = ws;
    ix->device_bytes += a->ws_bytes + (size_t)cap * (ix->D * 4 + 20) + 8;
    // staged rows past a call's Q are searched and thrown away: start them
    // as zero vectors (a fill kernel; the stream is not being captured)
    OSANN_HIP(launch_fill_u32(static_cast<uint32_t*>(a->q), cap * ix->D, 0u, s), "graph queries");
    a->qtype = kF32;
    *out = a;
    return OS_ANN_OK;
}

// A search through the graph of its shape class (stream, Q class, query
// type, mode, R, cone budget, budget): the queries are staged into the
// stream's arena, the class's graph (captured on first use, with the tiling
// the tuner picks for the class) runs on the arena, and the first Q results
// are copied to the caller's buffers.  Rows past Q in the class are earlier
// calls' queries (or zero vectors); each query's result is independent of
// the others in its batch, so they change nothing.
int search_graph(Call& c, int mode, int R, bool cones) {
    os_ann_index* ix = c.ix;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    OSANN_HIP(hipStreamIsCapturing(c.s, &st), "graph search");
    if (st != hipStreamCaptureStatusNone)
        return fail(OS_ANN_EINVAL, "OS_ANN_FLAG_GRAPH on a stream that is being captured");
    const int64_t Qc = graph_class(c.Q);
    Call g = c;
    g.Q = Qc;
    g.timing = false;
    g.p = plan_search(ix, Qc, c.budget, mode, R, cones);
    if (!g.p.fits)
        return fail(OS_ANN_ENOTSUP, "tiled mode: too many non-empty cones for the LDS cone list at this D");
    SearchPlan plans[kMaxPlans];
    int n_plans = 0;
    size_t bytes = g.p.bytes;
    if (mode == OS_ANN_MODE_TILED) {
        n_plans = tiled_plans(ix, Qc, c.budget, R, cones, plans);
        for (int k = 0; k < n_plans; ++k) bytes = std::max(bytes, plans[k].bytes);
        int rc = ensure_lowp(ix, c.s);
        if (rc) return rc;
    }
    std::lock_guard<std::mutex> lk(ix->graph_mu);
    GraphArena* a = nullptr;
    int rc = graph_arena(ix, c.s, Qc, bytes, &a);
    if (rc) return rc;
    const size_t row_bytes = (size_t)ix->D * elem_bytes(c.qtype);
    if (a->qtype != c.qtype) {  // rows staged in another type may not be valid in this one
        OSANN_HIP(launch_fill_u32(static_cast<uint32_t*>(a->q), a->cap_q * ix->D, 0u, c.s), "graph queries");
        a->qtype = c.qtype;
    }
    OSANN_HIP(hipMemcpyAsync(a->q, c.queries, (size_t)c.Q * row_bytes, hipMemcpyDeviceToDevice, c.s),
              "graph queries");
    g.queries = a->q;
    g.out_idx = a->oidx;
    g.out_dist = a->odist;
    g.out_ncand = a->oncand;
    g.walks_capped = c.walks_capped ? a->capped : nullptr;
    g.base = a->ws;
    const std::vector<int64_t> key = {(int64_t)(intptr_t)c.s, Qc, c.qtype, mode, R, cones ? 1 : 0, c.budget,
                                      c.walks_capped ? 1 : 0};
    GraphEntry* hit = nullptr;
    for (auto& e : ix->graphs)
        if (e.key == key) hit = &e;
    if (!hit) {
        int S = 1;
        if (mode == OS_ANN_MODE_TILED) {
            hipError_t e = hipSuccess;
            S = choose_tiling(g, plans, n_plans, true, &e);  // may time candidates on the arena
            if (e != hipSuccess) return hip_fail(e, "tiling autotune");
        }
        GraphEntry ne;
        ne.key = key;
        OSANN_HIP(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal), "graph capture");
        hipError_t e = enqueue(g, S);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(c.s, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e != hipSuccess ? e : e2, "graph capture");
        }
        ne.graph = graph;
        e = hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "graph instantiate");
        }
        if (ix->graphs.size() >= max_graphs()) {
            auto lru = std::min_element(ix->graphs.begin(), ix->graphs.end(),
                                        [](const GraphEntry& x, const GraphEntry& y) { return x.used < y.used; });
            // its last replay may still run on a stream of its own (which the
            // caller may have destroyed since): wait for the whole device
            e = hipDeviceSynchronize();
            if (e != hipSuccess) {
                (void)hipGraphExecDestroy(ne.exec);
                (void)hipGraphDestroy(graph);
                return hip_fail(e, "graph eviction");
            }
            destroy_graph(*lru);
            ix->graphs.erase(lru);
        }
        ix->graphs.push_back(ne);
        hit = &ix->graphs.back();
        ++ix->graph_captures;
    }
    hit->used = ++ix->graph_tick;
    hipGraphExec_t exec = hit->exec;
    OSANN_HIP(timed_launch(ix, c.timing, OS_ANN_KERNEL_GRAPH, c.s, [&] { return hipGraphLaunch(exec, c.s); }),
              "graph launch");
    ++ix->graph_replays;
    OSANN_HIP(hipMemcpyAsync(c.out_idx, a->oidx, (size_t)c.Q * 8, hipMemcpyDeviceToDevice, c.s), "graph rows");
    OSANN_HIP(hipMemcpyAsync(c.out_dist, a->odist, (size_t)c.Q * 4, hipMemcpyDeviceToDevice, c.s), "graph distances");
    if (c.out_ncand)
        OSANN_HIP(hipMemcpyAsync(c.out_ncand, a->oncand, (size_t)c.Q * 8, hipMemcpyDeviceToDevice, c.s),
                  "graph counts");
    if (c.walks_capped)
        OSANN_HIP(hipMemcpyAsync(c.walks_capped, a->capped, 8, hipMemcpyDeviceToDevice, c.s), "graph capped count");
    return OS_ANN_OK;
}

}  // namespace

extern "C" {

int os_ann_last_error(void) { return g_err; }
const char* os_ann_last_error_message(void) { return g_msg.c_str(); }
const char* os_ann_version(void) { return "osann 0.2 gfx950"; }

}  // extern "C"

namespace {
// Eigen-decomposition of the symmetric n x n matrix A (row-major, float64)
// by cyclic Jacobi rotations: on return A's diagonal holds the eigenvalues
// and column i of V the eigenvector of A[i][i].  Sweeps stop when the
// off-diagonal mass falls below 1e-30 of the total (or after 100 sweeps).
void jacobi_eigen(std::vector<double>& A, int n, std::vector<double>& V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double total = 0.0;
    for (double v : A) total += v * v;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += 2.0 * A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (off <= 1e-30 * total) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {  // V <- V J
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
}

// One table: the rows `keys` (type key_dtype) are hashed and bucketed; the
// table stores the rows `db` (type dtype) in that bucket order.  For one
// basis both are the database; for basis r of several, keys holds the
// database's coordinates in that basis.
//
// defer: the closing check (non-finite rows, non-empty count) is not taken
// here but by ensure_lowp's one synchronisation at its end, which the caller
// runs next; until then the index holds the flags and the sort scratch.
os_ann_index* build_table(const void* keys, int32_t key_dtype, int32_t Dk, const void* db, int32_t dtype, int64_t N,
                          int32_t D, int32_t L, int64_t nc, hipStream_t s, const uint32_t* group = nullptr,
                          int32_t n_groups = 1, bool defer = false) {

    auto* ix = new os_ann_index();
    ix->N = N;
    ix->D = D;
    ix->Dk = Dk;
    ix->L = L;
    ix->dtype = dtype;
    ix->n_cones = nc;
    ix->n_groups = n_groups;
    const int64_t nb = nc * n_groups;  // buckets
    ix->n_sub = binom_host(Dk, L);
    ix->epc = chunk_elems(dtype);
    ix->nch = (D + ix->epc - 1) / ix->epc;
    (void)hipGetDevice(&ix->device);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ix->device) == hipSuccess && ncu > 0)
        ix->num_cu = ncu;

    uint32_t* tmp = nullptr;
    uint32_t* small = nullptr;  // [0] non-finite flag, [1] non-empty count
    auto bail = [&](int) -> os_ann_index* {
        (void)hipDeviceSynchronize();
        dev_free(tmp);
        dev_free(small);
        release(ix);
        return nullptr;
    };
    const size_t n = (size_t)N;
    if (dev_alloc(ix, (void**)&ix->row_cone, n * 4, "row_cone") ||
        dev_alloc(ix, (void**)&ix->row_top, n * 8, "row_top") ||
        dev_alloc(ix, (void**)&ix->perm, n * 4, "perm") ||
        dev_alloc(ix, (void**)&ix->sorted_cone, n * 4, "sorted_cone") ||
        dev_alloc(ix, (void**)&ix->offsets, (size_t)(nb + 1) * 4, "offsets") ||
        dev_alloc(ix, &ix->planes, (size_t)ix->nch * n * 16, "planes") ||
        dev_alloc(ix, (void**)&ix->lexsub, (size_t)ix->n_sub * L, "lexsub") ||
        dev_alloc(ix, (void**)&ix->maskord, 128, "maskord") ||
        dev_alloc(ix, (void**)&ix->binom, 256 * 8 * 4, "binom") ||
        dev_alloc(nullptr, (void**)&tmp, (size_t)(4 * N + radix_hist_words(N)) * 4, "sort scratch") ||
        dev_alloc(nullptr, (void**)&small, 16, "flags"))
        return bail(0);

    auto step = [&](hipError_t e, const char* what) -> bool {
        if (e != hipSuccess) {
            hip_fail(e, what);
            return false;
        }
        return true;
    };
    if (!step(hipMemsetAsync(small, 0, 16, s), "memset") ||
        !step(launch_row_keys(keys, key_dtype, N, Dk, L, ix->row_cone, ix->row_top, small, s), "key kernel") ||
        !step(group ? launch_compose_cones(ix->row_cone, group, N, nc, s) : hipSuccess, "cluster buckets") ||
        !step(launch_sort_by_cone(ix->row_cone, N, nb, tmp, ix->perm, ix->sorted_cone, s), "radix sort") ||
        !step(launch_offsets(ix->sorted_cone, N, nb, ix->offsets, s), "offsets") ||
        !step(launch_gather_planes(db, dtype, N, D, ix->perm, ix->planes, s), "gather") ||
        !step(launch_probe_tables(Dk, L, ix->lexsub, ix->maskord, s), "probe tables") ||
        !step(launch_binom_table(ix->binom, s), "binomial table") ||
        !step(launch_count_nonempty(ix->offsets, nb, small + 1, s), "count"))
        return bail(0);
    if (defer) {
        ix->pending_small = small;
        ix->pending_tmp = tmp;
        return ix;
    }
    uint32_t host_small[2] = {0, 0};
    if (!step(hipMemcpyAsync(host_small, small, 8, hipMemcpyDeviceToHost, s), "copy flags") ||
        !step(hipStreamSynchronize(s), "build sync"))
        return bail(0);
    if (host_small[0]) {
        fail(OS_ANN_ENONFINITE, "database holds NaN or infinity");
        return bail(0);
    }
    ix->n_nonempty = host_small[1];
    dev_free(tmp);
    dev_free(small);
    tmp = small = nullptr;
    return ix;
}
// Sparse table (Section 4, second-level hash) for C(D,L) 2^L above 2^24:
// 64-bit cone ids of the rows, a stable sort by id, the distinct ids with
// their row offsets, and a hash table from id to bucket number.
os_ann_index* build_sparse(const void* db, int32_t dtype, int64_t N, int32_t D, int32_t L, int64_t nc,
                           hipStream_t s) {
    auto* ix = new os_ann_index();
    ix->N = N;
    ix->D = D;
    ix->Dk = D;
    ix->L = L;
    ix->dtype = dtype;
    ix->n_cones = nc;
    ix->n_sub = binom_host(D, L);
    ix->epc = chunk_elems(dtype);
    ix->nch = (D + ix->epc - 1) / ix->epc;
    ix->sparse = true;
    (void)hipGetDevice(&ix->device);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ix->device) == hipSuccess && ncu > 0)
        ix->num_cu = ncu;
    int end_bit = 1;
    while (end_bit < 64 && ((uint64_t)(nc - 1) >> end_bit) != 0) ++end_bit;
    const size_t n = (size_t)N;
    const size_t sort_bytes = sparse_sort_tmp_bytes(N, end_bit);
    uint64_t *key = nullptr, *sorted = nullptr;
    uint32_t *flag = nullptr, *pos = nullptr, *scan_tmp = nullptr, *small = nullptr;
    void* sort_tmp = nullptr;
    auto bail = [&]() -> os_ann_index* {
        (void)hipDeviceSynchronize();
        dev_free(key);
        dev_free(sorted);
        dev_free(flag);
        dev_free(pos);
        dev_free(scan_tmp);
        dev_free(small);
        dev_free(sort_tmp);
        release(ix);
        return nullptr;
    };
    auto step = [&](hipError_t e, const char* what) -> bool {
        if (e != hipSuccess) {
            hip_fail(e, what);
            return false;
        }
        return true;
    };
    if (dev_alloc(ix, (void**)&ix->row_cone, n * 4, "row_cone") ||
        dev_alloc(ix, (void**)&ix->row_top, n * 8, "row_top") ||
        dev_alloc(ix, (void**)&ix->perm, n * 4, "perm") ||
        dev_alloc(ix, &ix->planes, (size_t)ix->nch * n * 16, "planes") ||
        dev_alloc(ix, (void**)&ix->maskord, 128, "maskord") ||
        dev_alloc(ix, (void**)&ix->binom64, 257 * 8 * 8, "binomials") ||
        dev_alloc(nullptr, (void**)&key, n * 8, "sparse keys") ||
        dev_alloc(nullptr, (void**)&sorted, n * 8, "sorted keys") ||
        dev_alloc(nullptr, (void**)&flag, n * 4, "heads") ||
        dev_alloc(nullptr, (void**)&pos, (n + 1) * 4, "head positions") ||
        dev_alloc(nullptr, (void**)&scan_tmp, (size_t)exclusive_scan_tmp_words(N) * 4, "scan scratch") ||
        dev_alloc(nullptr, (void**)&small, 16, "flags") ||
        dev_alloc(nullptr, &sort_tmp, sort_bytes > 0 ? sort_bytes : 16, "sort scratch"))
        return bail();
    // C(n, k) for n <= 256, k <= 7, and the flip masks by popcount, then value
    std::vector<uint64_t> hb(257 * 8, 0);
    for (int nn = 0; nn <= 256; ++nn)
        for (int k = 0; k < 8; ++k) hb[nn * 8 + k] = (uint64_t)binom_host(nn, k);
    std::vector<uint8_t> hm(128, 0);
    int at = 0;
    for (int h = 0; h <= L; ++h)
        for (int m = 0; m < (1 << L); ++m)
            if (__builtin_popcount(m) == h) hm[at++] = (uint8_t)m;
    uint32_t host_small[1] = {0};
    uint32_t host_ne = 0;
    if (!step(hipMemcpyAsync(ix->binom64, hb.data(), hb.size() * 8, hipMemcpyHostToDevice, s), "binomials") ||
        !step(hipMemcpyAsync(ix->maskord, hm.data(), 128, hipMemcpyHostToDevice, s), "masks") ||
        !step(hipMemsetAsync(small, 0, 16, s), "memset") ||
        !step(launch_row_keys(db, dtype, N, D, L, ix->row_cone, ix->row_top, small, s), "key kernel") ||
        !step(launch_sparse_keys(ix->row_top, N, L, ix->binom64, key, s), "cone ids") ||
        !step(launch_sparse_sort(key, sorted, ix->perm, N, end_bit, sort_tmp, sort_bytes, s), "sort") ||
        !step(launch_sparse_heads(sorted, N, flag, s), "heads") ||
        !step(launch_exclusive_scan(flag, N, pos, scan_tmp, s), "head scan") ||
        !step(hipMemcpyAsync(host_small, small, 4, hipMemcpyDeviceToHost, s), "copy flags") ||
        !step(hipMemcpyAsync(&host_ne, pos + N, 4, hipMemcpyDeviceToHost, s), "copy count") ||
        !step(hipStreamSynchronize(s), "build sync"))
        return bail();
    if (host_small[0]) {
        fail(OS_ANN_ENONFINITE, "database holds NaN or infinity");
        return bail();
    }
    uint64_t cap = 64;
    while (cap < 2 * (uint64_t)host_ne) cap <<= 1;
    ix->sp_cap = cap;
    ix->sp_fbits = sparse_filter_bits(host_ne);
    ix->n_nonempty = host_ne;
    if (dev_alloc(ix, (void**)&ix->sp_keys, (size_t)host_ne * 8, "cone ids") ||
        dev_alloc(ix, (void**)&ix->offsets, ((size_t)host_ne + 1) * 4, "offsets") ||
        dev_alloc(ix, (void**)&ix->sp_hkeys, (size_t)cap * 8, "hash keys") ||
        dev_alloc(ix, (void**)&ix->sp_hval, (size_t)cap * 4, "hash values") ||
        dev_alloc(ix, (void**)&ix->sp_filt, (size_t)(ix->sp_fbits / 8), "hash filter"))
        return bail();
    if (!step(launch_sparse_compact(sorted, flag, pos, N, ix->sp_keys, ix->offsets, s), "compact") ||
        !step(launch_sparse_hash(ix->sp_keys, host_ne, ix->sp_hkeys, ix->sp_hval, cap, ix->sp_filt, ix->sp_fbits,
                                 s), "hash table") ||
        !step(launch_gather_planes(db, dtype, N, D, ix->perm, ix->planes, s), "gather") ||
        !step(hipStreamSynchronize(s), "build sync"))
        return bail();
    dev_free(key);
    dev_free(sorted);
    dev_free(flag);
    dev_free(pos);
    dev_free(scan_tmp);
    dev_free(small);
    dev_free(sort_tmp);
    return ix;
}

// Several bases: a table per basis from the rows' coordinates in it.  basis
// holds n_rot dense D x D matrices, or (wht) n_rot sign vectors of H diag(s).
os_ann_index* build_bases(const void* db, int64_t N, int32_t D, int32_t L, const float* basis, int32_t n_rot,
                          bool wht, const os_ann_build_opts* opts) {
    clear_error();
    const int32_t dtype = opts ? opts->dtype : kF32;
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    StreamScope ss(s);
    int64_t nc = 0;
    if (!db || !basis) {
        fail(OS_ANN_EINVAL, "null db or bases");
        return nullptr;
    }
    if (!dtype_ok(dtype)) {
        fail(OS_ANN_EINVAL, "bad db dtype");
        return nullptr;
    }
    if (n_rot < 1 || n_rot > kMaxRot) {
        fail(OS_ANN_EINVAL, "n_rot must be in [1, 16]");
        return nullptr;
    }
    if (opts && opts->want_lowp) {
        fail(OS_ANN_ENOTSUP, "several bases: FP32 mode only");
        return nullptr;
    }
    if (check_shape(N, D, L, &nc)) return nullptr;
    const size_t n = (size_t)N, R = (size_t)n_rot;
    const size_t basis_floats = wht ? R * D : R * D * D;
    if (wht) {
        if (D & (D - 1)) {
            fail(OS_ANN_EINVAL, "structured bases need D a power of two");
            return nullptr;
        }
        std::vector<float> hs(basis_floats);
        hipError_t e = hipMemcpy(hs.data(), basis, basis_floats * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            hip_fail(e, "reading the signs");
            return nullptr;
        }
        for (float v : hs)
            if (v != 1.0f && v != -1.0f) {
                fail(OS_ANN_EINVAL, "every sign must be +1 or -1");
                return nullptr;
            }
    }
    auto* ix = new os_ann_index();
    ix->N = N;
    ix->D = D;
    ix->Dk = D;
    ix->L = L;
    ix->dtype = dtype;
    ix->n_cones = nc;
    ix->n_sub = binom_host(D, L);
    ix->epc = chunk_elems(dtype);
    ix->nch = (D + ix->epc - 1) / ix->epc;
    ix->n_rot = n_rot;
    (void)hipGetDevice(&ix->device);
    float* coords = nullptr;
    auto bail = [&]() -> os_ann_index* {
        (void)hipDeviceSynchronize();
        dev_free(coords);
        release(ix);
        return nullptr;
    };
    float** keep = wht ? &ix->rot_signs : &ix->rot;
    if (dev_alloc(ix, (void**)keep, basis_floats * 4, "bases") ||
        dev_alloc(ix, (void**)&ix->rot_offsets, R * (size_t)(nc + 1) * 4, "basis offsets") ||
        dev_alloc(ix, (void**)&ix->rot_perm, R * n * 4, "basis perms") ||
        dev_alloc(ix, (void**)&ix->xtop, R * R * n * 8, "cross tops") ||
        dev_alloc(ix, (void**)&ix->planes_tab, R * sizeof(void*), "plane table") ||
        dev_alloc(nullptr, (void**)&coords, n * D * 4, "coordinates"))
        return bail();
    hipError_t e = hipMemcpyAsync(*keep, basis, basis_floats * 4, hipMemcpyDeviceToDevice, s);
    for (int r = 0; r < n_rot && e == hipSuccess; ++r) {
        e = wht ? launch_wht(db, dtype, N, D, ix->rot_signs + (size_t)r * D, coords, s)
                : launch_rotate(db, dtype, N, D, ix->rot + (size_t)r * D * D, coords, s);
        if (e != hipSuccess) break;
        os_ann_index* t = build_table(coords, kF32, D, db, dtype, N, D, L, nc, s);
        if (!t) return bail();
        ix->sub.push_back(t);
        ix->device_bytes += t->device_bytes;
        e = hipMemcpyAsync(ix->rot_offsets + (size_t)r * (nc + 1), t->offsets, (size_t)(nc + 1) * 4,
                           hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ix->rot_perm + (size_t)r * n, t->perm, n * 4, hipMemcpyDeviceToDevice, s);
    }
    for (int r = 0; r < n_rot && e == hipSuccess; ++r)
        for (int r2 = 0; r2 < n_rot && e == hipSuccess; ++r2)
            if (r2 != r)
                e = launch_gather_top(ix->sub[r]->perm, N, ix->sub[r2]->row_top,
                                      ix->xtop + ((size_t)r * R + r2) * n, s);
    std::vector<void*> tab_host;
    for (auto* t : ix->sub) tab_host.push_back(t->planes);
    if (e == hipSuccess && (int)tab_host.size() == n_rot)
        e = hipMemcpyAsync(ix->planes_tab, tab_host.data(), R * sizeof(void*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hip_fail(e, "several-bases build");
        return bail();
    }
    dev_free(coords);
    ix->n_nonempty = ix->sub[0]->n_nonempty;
    return ix;
}

}  // namespace

extern "C" {

os_ann_index* os_ann_build_ex(const void* db, int64_t N, int32_t D, int32_t L, const os_ann_build_opts* opts) {
    clear_error();
    const int32_t dtype = opts ? opts->dtype : kF32;
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    StreamScope ss(s);
    int64_t nc = 0;
    if (!db) {
        fail(OS_ANN_EINVAL, "null db");
        return nullptr;
    }
    if (!dtype_ok(dtype)) {
        fail(OS_ANN_EINVAL, "bad db dtype");
        return nullptr;
    }
    if (check_shape(N, D, L, &nc, true)) return nullptr;
    if (nc > kMaxCones) {  // sparse table
        if (opts && opts->want_lowp) {
            fail(OS_ANN_ENOTSUP, "sparse table: FP32 mode only");
            return nullptr;
        }
        return build_sparse(db, dtype, N, D, L, nc, s);
    }
    const bool lowp = opts && opts->want_lowp;
    os_ann_index* ix = build_table(db, dtype, D, db, dtype, N, D, L, nc, s, nullptr, 1, lowp);
    if (ix && lowp && ensure_lowp(ix, s)) {
        release(ix);
        return nullptr;
    }
    return ix;
}

os_ann_index* os_ann_build_rot(const void* db, int64_t N, int32_t D, int32_t L, const float* rot, int32_t n_rot,
                               const os_ann_build_opts* opts) {
    return build_bases(db, N, D, L, rot, n_rot, false, opts);
}

os_ann_index* os_ann_build_wht(const void* db, int64_t N, int32_t D, int32_t L, const float* signs, int32_t n_rot,
                               const os_ann_build_opts* opts) {
    return build_bases(db, N, D, L, signs, n_rot, true, opts);
}

int os_ann_pca(const void* db, int64_t N, int32_t D, int32_t k, const os_ann_build_opts* opts, float* mean_out,
               float* basis_out, double* var_out) {
    clear_error();
    const int32_t dtype = opts ? opts->dtype : kF32;
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    StreamScope ss(s);
    if (!db || !mean_out || !basis_out) return fail(OS_ANN_EINVAL, "null db or output");
    if (!dtype_ok(dtype)) return fail(OS_ANN_EINVAL, "bad db dtype");
    if (N < 1 || N >= (int64_t(1) << 31)) return fail(OS_ANN_EINVAL, "N must be in [1, 2^31)");
    if (D < 1 || D > kMaxD) return fail(OS_ANN_EINVAL, "D must be in [1, 256]");
    if (k < 1 || k > D) return fail(OS_ANN_EINVAL, "k must be in [1, D]");
    double *mean = nullptr, *cov = nullptr, *scratch = nullptr;
    auto done = [&](int code) {
        (void)hipDeviceSynchronize();
        dev_free(mean);
        dev_free(cov);
        dev_free(scratch);
        return code;
    };
    int rc = dev_alloc(nullptr, (void**)&mean, (size_t)D * 8, "pca mean");
    if (!rc) rc = dev_alloc(nullptr, (void**)&cov, (size_t)D * D * 8, "pca covariance");
    if (!rc) rc = dev_alloc(nullptr, (void**)&scratch, moments_scratch_doubles(N, D) * 8, "pca scratch");
    if (rc) return done(rc);
    std::vector<double> hmean(D), A((size_t)D * D);
    hipError_t e = launch_moments(db, dtype, N, D, mean, cov, scratch, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hmean.data(), mean, (size_t)D * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(A.data(), cov, (size_t)D * D * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(hip_fail(e, "pca moments"));
    done(OS_ANN_OK);
    for (double v : A)
        if (!std::isfinite(v)) return fail(OS_ANN_ENONFINITE, "database holds NaN or infinity");
    std::vector<double> V;
    jacobi_eigen(A, D, V);
    std::vector<int> pick(D);
    for (int i = 0; i < D; ++i) pick[i] = i;
    std::stable_sort(pick.begin(), pick.end(), [&](int a, int b) {
        return A[(size_t)a * D + a] > A[(size_t)b * D + b];
    });
    for (int r = 0; r < k; ++r) {
        const int col = pick[r];
        int jm = 0;
        for (int j = 1; j < D; ++j)
            if (std::fabs(V[(size_t)j * D + col]) > std::fabs(V[(size_t)jm * D + col])) jm = j;
        const double sg = V[(size_t)jm * D + col] < 0 ? -1.0 : 1.0;
        for (int j = 0; j < D; ++j) basis_out[(size_t)r * D + j] = (float)(sg * V[(size_t)j * D + col]);
        if (var_out) var_out[r] = A[(size_t)col * D + col];
    }
    for (int j = 0; j < D; ++j) mean_out[j] = (float)hmean[j];
    return OS_ANN_OK;
}

os_ann_index* os_ann_build_proj(const void* db, int64_t N, int32_t D, int32_t L, const float* mean,
                                const float* basis, int32_t k, const os_ann_build_opts* opts) {
    clear_error();
    const int32_t dtype = opts ? opts->dtype : kF32;
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    StreamScope ss(s);
    int64_t nc = 0, nc_rows = 0;
    if (!db || !basis) {
        fail(OS_ANN_EINVAL, "null db or basis");
        return nullptr;
    }
    if (!dtype_ok(dtype)) {
        fail(OS_ANN_EINVAL, "bad db dtype");
        return nullptr;
    }
    if (opts && opts->want_lowp) {
        fail(OS_ANN_ENOTSUP, "projected table: FP32 mode only");
        return nullptr;
    }
    if (check_shape(N, D, 1, &nc_rows)) return nullptr;
    if (k < 1 || k > D) {
        fail(OS_ANN_EINVAL, "k must be in [1, D]");
        return nullptr;
    }
    if (check_shape(N, k, L, &nc)) return nullptr;
    float *mu = nullptr, *P = nullptr, *keys = nullptr;
    auto bail = [&]() -> os_ann_index* {
        (void)hipDeviceSynchronize();
        dev_free(mu);
        dev_free(P);
        dev_free(keys);
        return nullptr;
    };
    if ((mean && dev_alloc(nullptr, (void**)&mu, (size_t)D * 4, "projection mean")) ||
        dev_alloc(nullptr, (void**)&P, (size_t)k * D * 4, "projection basis") ||
        dev_alloc(nullptr, (void**)&keys, (size_t)N * k * 4, "keys"))
        return bail();
    hipError_t e = hipSuccess;
    if (mean) e = hipMemcpyAsync(mu, mean, (size_t)D * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P, basis, (size_t)k * D * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_project(db, dtype, N, D, mu, P, k, keys, s);
    if (e != hipSuccess) {
        hip_fail(e, "projection");
        return bail();
    }
    os_ann_index* ix = build_table(keys, kF32, k, db, dtype, N, D, L, nc, s);  // synchronizes
    if (!ix) return bail();
    dev_free(keys);
    ix->proj = true;
    ix->proj_mu = mu;
    ix->proj_P = P;
    ix->device_bytes += (mu ? (size_t)D * 4 : 0) + (size_t)k * D * 4;
    return ix;
}

int os_ann_kmeans(const void* db, int64_t N, int32_t D, int32_t C, int32_t iters, const float* init,
                  const os_ann_build_opts* opts, float* out) {
    clear_error();
    const int32_t dtype = opts ? opts->dtype : kF32;
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    StreamScope ss(s);
    if (!db || !init || !out) return fail(OS_ANN_EINVAL, "null db, init or out");
    if (!dtype_ok(dtype)) return fail(OS_ANN_EINVAL, "bad db dtype");
    if (N < 1 || N >= (int64_t(1) << 31)) return fail(OS_ANN_EINVAL, "N must be in [1, 2^31)");
    if (D < 1 || D > kMaxD) return fail(OS_ANN_EINVAL, "D must be in [1, 256]");
    if (C < 1 || C > 4096) return fail(OS_ANN_EINVAL, "C must be in [1, 4096]");
    if (iters < 0) return fail(OS_ANN_EINVAL, "iters must be >= 0");
    float *ca = nullptr, *cb = nullptr;
    uint32_t *asg = nullptr, *tmp = nullptr, *members = nullptr, *sorted = nullptr, *off = nullptr;
    auto done = [&](int code) {
        (void)hipDeviceSynchronize();
        for (void* q : {(void*)ca, (void*)cb, (void*)asg, (void*)tmp, (void*)members, (void*)sorted, (void*)off})
            dev_free(q);
        return code;
    };
    const size_t cd = (size_t)C * D * 4;
    int rc = dev_alloc(nullptr, (void**)&ca, cd, "centroids");
    if (!rc) rc = dev_alloc(nullptr, (void**)&cb, cd, "centroids");
    if (!rc) rc = dev_alloc(nullptr, (void**)&asg, (size_t)N * 4, "assignment");
    if (!rc) rc = dev_alloc(nullptr, (void**)&tmp, (size_t)(4 * N + radix_hist_words(N)) * 4, "sort scratch");
    if (!rc) rc = dev_alloc(nullptr, (void**)&members, (size_t)N * 4, "members");
    if (!rc) rc = dev_alloc(nullptr, (void**)&sorted, (size_t)N * 4, "sorted clusters");
    if (!rc) rc = dev_alloc(nullptr, (void**)&off, (size_t)(C + 1) * 4, "cluster offsets");
    if (rc) return done(rc);
    hipError_t e = hipMemcpyAsync(ca, init, cd, hipMemcpyDeviceToDevice, s);
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
        e = launch_assign(db, dtype, N, D, ca, C, asg, s);
        if (e == hipSuccess) e = launch_sort_by_cone(asg, N, C, tmp, members, sorted, s);
        if (e == hipSuccess) e = launch_offsets(sorted, N, C, off, s);
        if (e == hipSuccess) e = launch_centroid_update(db, dtype, N, D, members, off, C, ca, cb, s);
        std::swap(ca, cb);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, ca, cd, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(hip_fail(e, "k-means"));
    return done(OS_ANN_OK);
}

os_ann_index* os_ann_build_ivf(const void* db, int64_t N, int32_t D, int32_t L, const float* centroids, int32_t C,
                               int32_t nprobe, const os_ann_build_opts* opts) {
    clear_error();
    const int32_t dtype = opts ? opts->dtype : kF32;
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    StreamScope ss(s);
    int64_t nc = 0;
    if (!db || !centroids) {
        fail(OS_ANN_EINVAL, "null db or centroids");
        return nullptr;
    }
    if (!dtype_ok(dtype)) {
        fail(OS_ANN_EINVAL, "bad db dtype");
        return nullptr;
    }
    if (opts && opts->want_lowp) {
        fail(OS_ANN_ENOTSUP, "clustered table: FP32 mode only");
        return nullptr;
    }
    if (check_shape(N, D, L, &nc)) return nullptr;
    if (C < 1 || C > kMaxClusters || nprobe < 1 || nprobe > C || nprobe > 64) {
        fail(OS_ANN_EINVAL, "need 1 <= nprobe <= min(C, 64) and C <= 1024");
        return nullptr;
    }
    if (nc * C > kMaxCones) {
        fail(OS_ANN_ENOTSUP, "clusters x cones exceeds 2^24 buckets");
        return nullptr;
    }
    float *cent = nullptr, *keys = nullptr;
    uint32_t* asg = nullptr;
    auto bail = [&]() -> os_ann_index* {
        (void)hipDeviceSynchronize();
        dev_free(cent);
        dev_free(keys);
        dev_free(asg);
        return nullptr;
    };
    if (dev_alloc(nullptr, (void**)&cent, (size_t)C * D * 4, "centroids") ||
        dev_alloc(nullptr, (void**)&keys, (size_t)N * D * 4, "residuals") ||
        dev_alloc(nullptr, (void**)&asg, (size_t)N * 4, "assignment"))
        return bail();
    hipError_t e = hipMemcpyAsync(cent, centroids, (size_t)C * D * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_assign(db, dtype, N, D, cent, C, asg, s);
    if (e == hipSuccess) e = launch_residual_rows(db, dtype, N, D, cent, asg, keys, s);
    if (e != hipSuccess) {
        hip_fail(e, "cluster assignment");
        return bail();
    }
    os_ann_index* ix = build_table(keys, kF32, D, db, dtype, N, D, L, nc, s, asg, C);  // synchronizes
    if (!ix) return bail();
    dev_free(keys);
    dev_free(asg);
    ix->ivf_cent = cent;
    ix->nprobe = nprobe;
    ix->device_bytes += (size_t)C * D * 4;
    return ix;
}

int os_ann_set_nprobe(os_ann_index* ix, int32_t nprobe) {
    clear_error();
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    if (!ix->ivf_cent) return fail(OS_ANN_EINVAL, "not a clustered table");
    if (nprobe < 1 || nprobe > ix->n_groups || nprobe > 64) return fail(OS_ANN_EINVAL, "nprobe out of range");
    std::lock_guard<std::mutex> g(ix->graph_mu);
    if (!ix->graphs.empty()) OSANN_HIP(hipDeviceSynchronize(), "set_nprobe");  // replays may still run
    drop_graphs(ix);  // captured searches used the old count
    ix->nprobe = nprobe;
    return OS_ANN_OK;
}

int os_ann_export_basis(const os_ann_index* ix, int32_t r, uint32_t* row_cone, uint64_t* row_top,
                        int64_t* offsets, int64_t* perm, void* stream) {
    clear_error();
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    if (ix->n_rot == 0) {
        if (r != 0) return fail(OS_ANN_EINVAL, "basis out of range");
        return os_ann_export(ix, row_cone, row_top, offsets, perm, stream);
    }
    if (r < 0 || r >= ix->n_rot) return fail(OS_ANN_EINVAL, "basis out of range");
    return os_ann_export(ix->sub[r], row_cone, row_top, offsets, perm, stream);
}



os_ann_index* os_ann_build(const float* db, int64_t N, int32_t D, int32_t L) {
    return os_ann_build_ex(db, N, D, L, nullptr);
}

void os_ann_free(os_ann_index* idx) { release(idx); }

int os_ann_graph_stats(const os_ann_index* cidx, int64_t* captured, int64_t* replayed, int64_t* cached) {
    clear_error();
    if (!cidx) return fail(OS_ANN_EINVAL, "null index");
    auto* ix = const_cast<os_ann_index*>(cidx);
    std::lock_guard<std::mutex> g(ix->graph_mu);
    if (captured) *captured = ix->graph_captures;
    if (replayed) *replayed = ix->graph_replays;
    if (cached) *cached = (int64_t)ix->graphs.size();
    return OS_ANN_OK;
}

int os_ann_last_tiling(const os_ann_index* idx, int32_t* kernel, int32_t* order, int32_t* groups,
                       int32_t* splits) {
    clear_error();
    if (!idx) return fail(OS_ANN_EINVAL, "null index");
    if (kernel) *kernel = idx->last_kern;
    if (order) *order = idx->last_order;
    if (groups) *groups = idx->last_groups;
    if (splits) *splits = idx->last_splits;
    return OS_ANN_OK;
}

int os_ann_trim(void) {
    clear_error();
    trim_blocks();
    return OS_ANN_OK;
}

int os_ann_set_allocator(os_ann_alloc_fn alloc, os_ann_free_fn free_fn, void* ctx) {
    clear_error();
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(OS_ANN_EINVAL, "set_allocator: give both functions or neither");
    {
        std::lock_guard<std::mutex> g(block_cache().mu);
        g_hook.alloc = alloc;
        g_hook.free = free_fn;
        g_hook.ctx = alloc ? ctx : nullptr;
    }
    if (alloc) trim_blocks();  // idle blocks of the library's own are not needed any more
    return OS_ANN_OK;
}

int64_t os_ann_workspace_bytes(const os_ann_index* idx, int64_t Q, int64_t max_candidates,
                               const os_ann_search_opts* opts) {
    clear_error();
    int rc = search_checks(idx, idx, Q, max_candidates, opts);
    if (rc) return rc;
    const int mode = opts ? opts->mode : OS_ANN_MODE_FP32;
    const int R = opts && opts->rerank_r ? opts->rerank_r : 8;
    const bool cones = opts && (opts->flags & OS_ANN_FLAG_BUDGET_CONES);
    if (mode == OS_ANN_MODE_TILED && !idx->sparse && idx->n_rot == 0 && !idx->proj && !idx->ivf_cent) {
        SearchPlan plans[kMaxPlans];
        const int np = tiled_plans(idx, Q, max_candidates, R, cones, plans);
        size_t bytes = 0;
        for (int k = 0; k < np; ++k) bytes = std::max(bytes, plans[k].bytes);
        return (int64_t)bytes;
    }
    return (int64_t)plan_search(idx, Q, max_candidates, mode, R, cones).bytes;
}

int os_ann_search_ex(const os_ann_index* cidx, const void* queries, int64_t Q, int64_t max_candidates,
                     const os_ann_search_opts* opts, int64_t* out_idx, float* out_dist,
                     int64_t* out_ncand) {
    clear_error();
    int rc = search_checks(cidx, queries, Q, max_candidates, opts);
    if (rc) return rc;
    if (Q == 0) return OS_ANN_OK;
    if (!out_idx || !out_dist) return fail(OS_ANN_EINVAL, "null output");
    auto* ix = const_cast<os_ann_index*>(cidx);
    Call c{};
    c.ix = ix;
    c.queries = queries;
    c.qtype = opts ? opts->query_dtype : kF32;
    c.Q = Q;
    c.budget = max_candidates;
    c.out_idx = out_idx;
    c.out_dist = out_dist;
    c.out_ncand = out_ncand;
    c.walks_capped = opts ? opts->walks_capped : nullptr;
    c.s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    StreamScope ss(c.s);
    c.timing = opts && (opts->flags & OS_ANN_FLAG_TIME_KERNELS);
    const int mode = opts ? opts->mode : OS_ANN_MODE_FP32;
    const int R = opts && opts->rerank_r ? opts->rerank_r : 8;
    const bool cones = opts && (opts->flags & OS_ANN_FLAG_BUDGET_CONES);
    if (opts && (opts->flags & OS_ANN_FLAG_GRAPH)) {
        if (!c.s) return fail(OS_ANN_EINVAL, "OS_ANN_FLAG_GRAPH needs a non-null stream");
        return search_graph(c, mode, R, cones);
    }
    c.p = plan_search(ix, Q, max_candidates, mode, R, cones);
    if (!c.p.fits)
        return fail(OS_ANN_ENOTSUP, "tiled mode: too many non-empty cones for the LDS cone list at this D");
    SearchPlan plans[kMaxPlans];
    int n_plans = 0;
    size_t bytes = c.p.bytes;
    if (mode == OS_ANN_MODE_TILED) {  // one scratch layout per tile width; room for the largest
        n_plans = tiled_plans(ix, Q, max_candidates, R, cones, plans);
        for (int k = 0; k < n_plans; ++k) bytes = std::max(bytes, plans[k].bytes);
    }
    if ((rc = get_scratch(ix, opts, bytes, &c.base))) return rc;
    int S = 1;
    if (mode == OS_ANN_MODE_TILED) {
        if ((rc = ensure_lowp(ix, c.s))) return rc;
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (c.s) (void)hipStreamIsCapturing(c.s, &st);
        hipError_t e = hipSuccess;
        S = choose_tiling(c, plans, n_plans, st == hipStreamCaptureStatusNone, &e);
        if (e != hipSuccess) return hip_fail(e, "tiling autotune");
    }
    OSANN_HIP(enqueue(c, S), mode == OS_ANN_MODE_TILED ? "tiled search" : "fp32 search");
    return OS_ANN_OK;
}

int os_ann_search_static(const os_ann_index* cidx, const void* queries, int64_t Q, int64_t max_candidates,
                         const os_ann_search_opts* opts, int64_t* out_idx, float* out_dist, int64_t* out_ncand) {
    clear_error();
    int rc = search_checks(cidx, queries, Q, max_candidates, opts);
    if (rc) return rc;
    if (opts && opts->mode != OS_ANN_MODE_FP32)
        return fail(OS_ANN_ENOTSUP, "search_static: FP32 mode only (tiled mode builds its low-precision copy on first use)");
    if (opts && opts->workspace) return fail(OS_ANN_EINVAL, "search_static: takes no workspace");
    if (opts && (opts->flags & ~OS_ANN_FLAG_BUDGET_CONES))
        return fail(OS_ANN_EINVAL, "search_static: only OS_ANN_FLAG_BUDGET_CONES applies");
    if (Q == 0) return OS_ANN_OK;
    if (!out_idx || !out_dist) return fail(OS_ANN_EINVAL, "null output");
    auto* ix = const_cast<os_ann_index*>(cidx);
    const bool cones = opts && (opts->flags & OS_ANN_FLAG_BUDGET_CONES);
    Call c{};
    c.ix = ix;
    c.queries = queries;
    c.qtype = opts ? opts->query_dtype : kF32;
    c.Q = Q;
    c.budget = max_candidates;
    c.out_idx = out_idx;
    c.out_dist = out_dist;
    c.out_ncand = out_ncand;
    c.walks_capped = opts ? opts->walks_capped : nullptr;
    c.s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    c.timing = false;
    c.p = plan_search(ix, Q, max_candidates, OS_ANN_MODE_FP32, 8, cones);
    if (c.p.bytes > kStaticScratchBytes) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "search_static: %lld queries need %zu bytes of scratch, the static scratch holds %zu "
                      "(split the batch)", (long long)Q, c.p.bytes, kStaticScratchBytes);
        return fail(OS_ANN_EINVAL, msg);
    }
    // the device address of this GPU's copy of the array, looked up once
    static std::mutex mu;
    static std::unordered_map<int, void*> addr;
    int dev = 0;
    OSANN_HIP(hipGetDevice(&dev), "search_static: current device");
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = addr.find(dev);
        if (it == addr.end()) {
            void* p = nullptr;
            OSANN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "search_static: scratch address");
            it = addr.emplace(dev, p).first;
        }
        c.base = static_cast<char*>(it->second);
    }
    OSANN_HIP(enqueue(c, 1), "search_static");
    return OS_ANN_OK;
}

int os_ann_search(const os_ann_index* idx, const float* queries, int64_t Q, int64_t max_candidates,
                  int64_t* out_idx, float* out_dist) {
    return os_ann_search_ex(idx, queries, Q, max_candidates, nullptr, out_idx, out_dist, nullptr);
}

int os_ann_classify(const os_ann_index* cidx, const void* queries, int32_t query_dtype, int64_t Q,
                    int64_t max_candidates, uint32_t* q_cone, uint64_t* q_top, int64_t* q_ncand,
                    void* stream) {
    clear_error();
    if (cidx && cidx->n_rot > 0) return fail(OS_ANN_ENOTSUP, "classify: one basis only");
    if (cidx && cidx->proj) return fail(OS_ANN_ENOTSUP, "classify: not for a projected table");
    if (cidx && cidx->ivf_cent) return fail(OS_ANN_ENOTSUP, "classify: not for a clustered table");
    if (cidx && cidx->sparse) return fail(OS_ANN_ENOTSUP, "classify: not for a sparse table");
    os_ann_search_opts o{};
    o.query_dtype = query_dtype;
    int rc = search_checks(cidx, queries, Q, max_candidates, &o);
    if (rc) return rc;
    if (Q == 0) return OS_ANN_OK;
    const os_ann_index* ix = cidx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    ProbeArgs pa{};
    pa.Y = queries;
    pa.qtype = query_dtype;
    pa.Q = Q;
    pa.D = ix->Dk;
    pa.L = ix->L;
    pa.offsets = ix->offsets;
    pa.n_cones = ix->n_cones;
    pa.n_sub = ix->n_sub;
    pa.N = ix->N;
    pa.budget = max_candidates;
    pa.lexsub = ix->lexsub;
    pa.maskord = ix->maskord;
    pa.binom = ix->binom;
    pa.q_cone = q_cone;
    pa.q_top = q_top;
    pa.ncand = q_ncand;
    OSANN_HIP(launch_probe(pa, s), "probe kernel");
    return OS_ANN_OK;
}

int os_ann_export(const os_ann_index* ix, uint32_t* row_cone, uint64_t* row_top, int64_t* offsets,
                  int64_t* perm, void* stream) {
    clear_error();
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    if (ix->n_rot > 0) ix = ix->sub[0];  // basis 0
    if (ix->sparse && (row_cone || offsets))
        return fail(OS_ANN_ENOTSUP, "sparse table: cone ids and offsets through os_ann_export_sparse");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (row_cone)
        OSANN_HIP(hipMemcpyAsync(row_cone, ix->row_cone, (size_t)ix->N * 4, hipMemcpyDeviceToDevice, s),
                  "export cone");
    if (row_top)
        OSANN_HIP(hipMemcpyAsync(row_top, ix->row_top, (size_t)ix->N * 8, hipMemcpyDeviceToDevice, s),
                  "export top");
    if (offsets)
        OSANN_HIP(launch_widen_u32(ix->offsets, ix->n_cones * ix->n_groups + 1, offsets, s), "export offsets");
    if (perm) OSANN_HIP(launch_widen_u32(ix->perm, ix->N, perm, s), "export perm");
    return OS_ANN_OK;
}

int os_ann_export_sparse(const os_ann_index* ix, uint64_t* cone_ids, int64_t* offsets, int64_t* perm,
                         void* stream) {
    clear_error();
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    if (!ix->sparse) return fail(OS_ANN_EINVAL, "not a sparse table");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (cone_ids)
        OSANN_HIP(hipMemcpyAsync(cone_ids, ix->sp_keys, (size_t)ix->n_nonempty * 8, hipMemcpyDeviceToDevice, s),
                  "export cone ids");
    if (offsets) OSANN_HIP(launch_widen_u32(ix->offsets, ix->n_nonempty + 1, offsets, s), "export offsets");
    if (perm) OSANN_HIP(launch_widen_u32(ix->perm, ix->N, perm, s), "export perm");
    return OS_ANN_OK;
}

int os_ann_export_rows(const os_ann_index* ix, float* rows, void* stream) {
    clear_error();
    if (!ix || !rows) return fail(OS_ANN_EINVAL, "null argument");
    if (ix->n_rot > 0) ix = ix->sub[0];  // basis 0's order
    OSANN_HIP(launch_planes_to_rows(ix->planes, ix->dtype, ix->N, ix->D, rows, static_cast<hipStream_t>(stream)),
              "export rows");
    return OS_ANN_OK;
}

int os_ann_kernel_time(const os_ann_index* cidx, int32_t kernel, int64_t* launches, double* total_ms) {
    clear_error();
    if (!cidx) return fail(OS_ANN_EINVAL, "null index");
    if (kernel < 0 || kernel >= OS_ANN_KERNEL_COUNT) return fail(OS_ANN_EINVAL, "bad kernel id");
    auto* ix = const_cast<os_ann_index*>(cidx);
    std::lock_guard<std::mutex> g(ix->time_mu);
    int64_t n = 0;
    double ms = 0.0;
    std::vector<os_ann_index::Timed> keep;
    for (auto& t : ix->timed) {
        if (t.kernel != kernel) {
            keep.push_back(t);
            continue;
        }
        float one = 0.0f;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&one, t.start, t.stop);
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
        if (e != hipSuccess) {
            ix->timed.clear();
            return hip_fail(e, "kernel timing");
        }
        ++n;
        ms += one;
    }
    ix->timed.swap(keep);
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    return OS_ANN_OK;
}

int os_ann_info(const os_ann_index* ix, int64_t* N, int32_t* D, int32_t* L, int64_t* n_cones,
                int64_t* n_nonempty, int64_t* device_bytes) {
    clear_error();
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    if (N) *N = ix->N;
    if (D) *D = ix->D;
    if (L) *L = ix->L;
    if (n_cones) *n_cones = ix->n_cones * ix->n_groups;  // buckets
    if (n_nonempty) *n_nonempty = ix->n_nonempty;
    if (device_bytes) *device_bytes = (int64_t)ix->device_bytes;
    return OS_ANN_OK;
}

}  // extern "C"
