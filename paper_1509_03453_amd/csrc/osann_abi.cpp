// Host side of the C ABI declared in include/osann.h: argument checks, device
// memory of an index, and the launch sequence of the gfx950 kernels.
#include "osann.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "osann_kernels.h"

using namespace osann;

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

#define OSANN_HIP(call, what)                      \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct os_ann_index {
    int64_t N = 0;
    int32_t D = 0, L = 0, dtype = 0;
    int64_t n_cones = 0, n_sub = 0, n_nonempty = 0;
    int nch = 0, epc = 0;
    int device = 0;
    size_t device_bytes = 0;
    uint32_t* row_cone = nullptr;
    uint64_t* row_top = nullptr;
    uint32_t* perm = nullptr;
    uint32_t* offsets = nullptr;
    void* planes = nullptr;
    uint8_t* lexsub = nullptr;
    uint8_t* maskord = nullptr;
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
};

namespace {

int dev_alloc(os_ann_index* ix, void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return hip_fail(e, what);
    }
    if (ix) ix->device_bytes += bytes;
    return OS_ANN_OK;
}

void release(os_ann_index* ix) {
    if (!ix) return;
    for (auto& t : ix->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    void* ptrs[] = {ix->row_cone, ix->row_top, ix->perm, ix->offsets, ix->planes,
                    ix->lexsub,   ix->maskord, ix->scratch};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete ix;
}

int check_shape(int64_t N, int32_t D, int32_t L, int64_t* n_cones) {
    if (N < 1 || N >= (int64_t(1) << 31)) return fail(OS_ANN_EINVAL, "N must be in [1, 2^31)");
    if (D < 1 || D > kMaxD) return fail(OS_ANN_EINVAL, "D must be in [1, 256]");
    if (L < 1 || L > kMaxL || L > D) return fail(OS_ANN_EINVAL, "L must be in [1, min(D, 7)]");
    const int64_t nc = binom_host(D, L) << L;
    if (nc > kMaxCones) return fail(OS_ANN_ENOTSUP, "C(D,L)*2^L exceeds 2^24 cones");
    *n_cones = nc;
    return OS_ANN_OK;
}

bool dtype_ok(int32_t t) { return t == kF32 || t == kF16 || t == kU8; }

// Scratch layout of one search: FP32 query copy, probe descriptors, probe
// counts, candidate counts.
struct SearchPlan {
    int64_t Q = 0, cap = 0;
    int dpad = 0;
    size_t off_yf = 0, off_desc = 0, off_np = 0, off_nc = 0, bytes = 0;
};

SearchPlan plan_search(const os_ann_index* ix, int64_t Q, int64_t budget) {
    SearchPlan p;
    p.Q = Q;
    p.dpad = ix->nch * ix->epc;
    p.cap = budget >= ix->N ? 1 : (budget < ix->n_nonempty ? budget : ix->n_nonempty);
    if (p.cap < 1) p.cap = 1;
    size_t at = 0;
    p.off_yf = at;
    at = align_up(at + (size_t)Q * p.dpad * sizeof(float), 256);
    p.off_desc = at;
    at = align_up(at + (size_t)Q * p.cap * sizeof(uint2), 256);
    p.off_np = at;
    at = align_up(at + (size_t)Q * sizeof(uint32_t), 256);
    p.off_nc = at;
    at = align_up(at + (size_t)Q * sizeof(int64_t), 256);
    p.bytes = at;
    return p;
}

int search_checks(const os_ann_index* ix, const void* queries, int64_t Q, int64_t budget,
                  const os_ann_search_opts* o) {
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    if (Q < 0) return fail(OS_ANN_EINVAL, "Q must be >= 0");
    if (budget < 1) return fail(OS_ANN_EINVAL, "max_candidates must be >= 1");
    if (Q > 0 && !queries) return fail(OS_ANN_EINVAL, "null queries");
    if (o) {
        if (!dtype_ok(o->query_dtype)) return fail(OS_ANN_EINVAL, "bad query dtype");
        if (o->mode != OS_ANN_MODE_FP32 && o->mode != OS_ANN_MODE_TILED)
            return fail(OS_ANN_EINVAL, "bad mode");
        if (o->mode == OS_ANN_MODE_TILED) return fail(OS_ANN_EINVAL, "tiled mode is not available");
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
            (void)hipFree(ix->scratch);
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

}  // namespace

extern "C" {

int os_ann_last_error(void) { return g_err; }
const char* os_ann_last_error_message(void) { return g_msg.c_str(); }
const char* os_ann_version(void) { return "osann 0.1 gfx950"; }

os_ann_index* os_ann_build_ex(const void* db, int64_t N, int32_t D, int32_t L,
                              const os_ann_build_opts* opts) {
    clear_error();
    const int32_t dtype = opts ? opts->dtype : kF32;
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    int64_t nc = 0;
    if (!db) {
        fail(OS_ANN_EINVAL, "null db");
        return nullptr;
    }
    if (!dtype_ok(dtype)) {
        fail(OS_ANN_EINVAL, "bad db dtype");
        return nullptr;
    }
    if (check_shape(N, D, L, &nc)) return nullptr;

    auto* ix = new os_ann_index();
    ix->N = N;
    ix->D = D;
    ix->L = L;
    ix->dtype = dtype;
    ix->n_cones = nc;
    ix->n_sub = binom_host(D, L);
    ix->epc = chunk_elems(dtype);
    ix->nch = (D + ix->epc - 1) / ix->epc;
    (void)hipGetDevice(&ix->device);

    uint32_t* tmp = nullptr;
    uint32_t* small = nullptr;  // [0] non-finite flag, [1] non-empty count
    auto bail = [&](int) -> os_ann_index* {
        if (tmp) (void)hipFree(tmp);
        if (small) (void)hipFree(small);
        release(ix);
        return nullptr;
    };
    const size_t n = (size_t)N;
    if (dev_alloc(ix, (void**)&ix->row_cone, n * 4, "row_cone") ||
        dev_alloc(ix, (void**)&ix->row_top, n * 8, "row_top") ||
        dev_alloc(ix, (void**)&ix->perm, n * 4, "perm") ||
        dev_alloc(ix, (void**)&ix->offsets, (size_t)(nc + 1) * 4, "offsets") ||
        dev_alloc(ix, &ix->planes, (size_t)ix->nch * n * 16, "planes") ||
        dev_alloc(ix, (void**)&ix->lexsub, (size_t)ix->n_sub * L, "lexsub") ||
        dev_alloc(ix, (void**)&ix->maskord, 128, "maskord") ||
        dev_alloc(nullptr, (void**)&tmp, (size_t)(5 * N + radix_hist_words(N)) * 4, "sort scratch") ||
        dev_alloc(nullptr, (void**)&small, 16, "flags"))
        return bail(0);

    auto step = [&](hipError_t e, const char* what) -> bool {
        if (e != hipSuccess) {
            hip_fail(e, what);
            return false;
        }
        return true;
    };
    uint32_t* sorted_cone = tmp + 4 * N + radix_hist_words(N);
    if (!step(hipMemsetAsync(small, 0, 16, s), "memset") ||
        !step(launch_row_keys(db, dtype, N, D, L, ix->row_cone, ix->row_top, small, s), "key kernel") ||
        !step(launch_sort_by_cone(ix->row_cone, N, nc, tmp, ix->perm, sorted_cone, s), "radix sort") ||
        !step(launch_offsets(sorted_cone, N, nc, ix->offsets, s), "offsets") ||
        !step(launch_gather_planes(db, dtype, N, D, ix->perm, ix->planes, s), "gather") ||
        !step(launch_probe_tables(D, L, ix->lexsub, ix->maskord, s), "probe tables") ||
        !step(launch_count_nonempty(ix->offsets, nc, small + 1, s), "count"))
        return bail(0);
    uint32_t host_small[2] = {0, 0};
    if (!step(hipMemcpyAsync(host_small, small, 8, hipMemcpyDeviceToHost, s), "copy flags") ||
        !step(hipStreamSynchronize(s), "build sync"))
        return bail(0);
    if (host_small[0]) {
        fail(OS_ANN_ENONFINITE, "database holds NaN or infinity");
        return bail(0);
    }
    ix->n_nonempty = host_small[1];
    (void)hipFree(tmp);
    (void)hipFree(small);
    return ix;
}

os_ann_index* os_ann_build(const float* db, int64_t N, int32_t D, int32_t L) {
    return os_ann_build_ex(db, N, D, L, nullptr);
}

void os_ann_free(os_ann_index* idx) { release(idx); }

int64_t os_ann_workspace_bytes(const os_ann_index* idx, int64_t Q, int64_t max_candidates,
                               const os_ann_search_opts* opts) {
    clear_error();
    if (!idx) return fail(OS_ANN_EINVAL, "null index");
    if (Q < 0 || max_candidates < 1) return fail(OS_ANN_EINVAL, "bad Q or max_candidates");
    if (opts && opts->mode == OS_ANN_MODE_TILED) return fail(OS_ANN_EINVAL, "tiled mode is not available");
    return (int64_t)plan_search(idx, Q, max_candidates).bytes;
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
    hipStream_t s = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
    const SearchPlan p = plan_search(ix, Q, max_candidates);
    char* base = nullptr;
    if ((rc = get_scratch(ix, opts, p.bytes, &base))) return rc;

    ProbeArgs pa{};
    pa.Y = queries;
    pa.qtype = opts ? opts->query_dtype : kF32;
    pa.Q = Q;
    pa.D = ix->D;
    pa.L = ix->L;
    pa.offsets = ix->offsets;
    pa.n_cones = ix->n_cones;
    pa.n_sub = ix->n_sub;
    pa.N = ix->N;
    pa.budget = max_candidates;
    pa.lexsub = ix->lexsub;
    pa.maskord = ix->maskord;
    pa.yf = reinterpret_cast<float*>(base + p.off_yf);
    pa.dpad = p.dpad;
    pa.desc = reinterpret_cast<uint2*>(base + p.off_desc);
    pa.cap = p.cap;
    pa.nprobe = reinterpret_cast<uint32_t*>(base + p.off_np);
    pa.ncand = out_ncand ? out_ncand : reinterpret_cast<int64_t*>(base + p.off_nc);
    const bool timing = opts && (opts->flags & OS_ANN_FLAG_TIME_KERNELS);
    OSANN_HIP(timed_launch(ix, timing, OS_ANN_KERNEL_PROBE, s, [&] { return launch_probe(pa, s); }),
              "probe kernel");

    ScanArgs sa{};
    sa.planes = ix->planes;
    sa.dtype = ix->dtype;
    sa.N = ix->N;
    sa.D = ix->D;
    sa.nch = ix->nch;
    sa.yf = pa.yf;
    sa.Q = Q;
    sa.desc = pa.desc;
    sa.cap = p.cap;
    sa.nprobe = pa.nprobe;
    sa.perm = ix->perm;
    sa.out_idx = out_idx;
    sa.out_dist = out_dist;
    const int64_t expect = max_candidates < ix->N ? max_candidates : ix->N;
    sa.waves_per_query = expect <= 8192 ? 1 : 4;
    OSANN_HIP(timed_launch(ix, timing, OS_ANN_KERNEL_SCAN, s, [&] { return launch_scan_fp32(sa, s); }),
              "scan kernel");
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
    os_ann_search_opts o{};
    o.query_dtype = query_dtype;
    int rc = search_checks(cidx, queries, Q, max_candidates, &o);
    if (rc) return rc;
    if (Q == 0) return OS_ANN_OK;
    auto* ix = const_cast<os_ann_index*>(cidx);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ProbeArgs pa{};
    pa.Y = queries;
    pa.qtype = query_dtype;
    pa.Q = Q;
    pa.D = ix->D;
    pa.L = ix->L;
    pa.offsets = ix->offsets;
    pa.n_cones = ix->n_cones;
    pa.n_sub = ix->n_sub;
    pa.N = ix->N;
    pa.budget = max_candidates;
    pa.lexsub = ix->lexsub;
    pa.maskord = ix->maskord;
    pa.q_cone = q_cone;
    pa.q_top = q_top;
    pa.ncand = q_ncand;
    pa.cap = 1;
    OSANN_HIP(launch_probe(pa, s), "probe kernel");
    return OS_ANN_OK;
}

int os_ann_export(const os_ann_index* ix, uint32_t* row_cone, uint64_t* row_top, int64_t* offsets,
                  int64_t* perm, void* stream) {
    clear_error();
    if (!ix) return fail(OS_ANN_EINVAL, "null index");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (row_cone)
        OSANN_HIP(hipMemcpyAsync(row_cone, ix->row_cone, (size_t)ix->N * 4, hipMemcpyDeviceToDevice, s),
                  "export cone");
    if (row_top)
        OSANN_HIP(hipMemcpyAsync(row_top, ix->row_top, (size_t)ix->N * 8, hipMemcpyDeviceToDevice, s),
                  "export top");
    if (offsets) OSANN_HIP(launch_widen_u32(ix->offsets, ix->n_cones + 1, offsets, s), "export offsets");
    if (perm) OSANN_HIP(launch_widen_u32(ix->perm, ix->N, perm, s), "export perm");
    return OS_ANN_OK;
}

int os_ann_export_rows(const os_ann_index* ix, float* rows, void* stream) {
    clear_error();
    if (!ix || !rows) return fail(OS_ANN_EINVAL, "null argument");
    OSANN_HIP(launch_planes_to_rows(ix->planes, ix->dtype, ix->N, ix->D, rows,
                                    static_cast<hipStream_t>(stream)),
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
    if (n_cones) *n_cones = ix->n_cones;
    if (n_nonempty) *n_nonempty = ix->n_nonempty;
    if (device_bytes) *device_bytes = (int64_t)ix->device_bytes;
    return OS_ANN_OK;
}

}  // extern "C"
