// libretina host side: context, device pool, argument validation, launch
// sequence and the C-ABI entry points declared in include/retina.h.
#include <math.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "proposer.h"
#include "rt_internal.h"
#include "validate.h"

using namespace rt;

namespace {

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

enum BufId {
    B_HITS, B_POFF, B_NHITS, B_SOFF, B_ORDER, B_ITEMS, B_STH, B_SR, B_SFL, B_SNR, B_MLEAD, B_MMEM,
    B_MKEYS, B_EVNT, B_EVFL, B_EVTOFF,
    // staging copies for host-memory calls
    B_INX, B_INY, B_INPL, B_INOFF, B_INSEEDS, B_INSOFF, B_INTH, B_INTHOFF, B_OUTTR, B_OUTTOFF,
    B_OUTEVF, B_OUTSTH, B_OUTSR, B_OUTSFL, B_OUTSNR, B_OUTR, B_OUTG, B_OUTH,
    // learned proposer workspace
    B_GRID, B_GRIDCNT, B_GRIDBASE, B_EVSORT,
    B_IMG, B_ACT1, B_ACT2, B_ACT3, B_LOGIT, B_HEADU, B_RESPPART, B_DZ4, B_DZ3, B_DZ2, B_DZ1, B_TGT, B_TGTIN, B_TGTOFF,
    B_DWPART, B_WT, B_LOSSPART, B_LOSS, B_BPART, B_PSCORE, B_PPIX, B_PCOUNT, B_PCONF, B_PFB,
    B_PSOFF, B_PSEEDS, B_OUTIMG, B_OUTLOGIT,
    B_COUNT
};

}  // namespace

struct retina_ctx {
    int device = 0;
    char arch[64] = {0};
    size_t lds_max = 65536;       // LDS bytes per work-group on this device
    hipStream_t own = nullptr;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    std::string err;
    int64_t max_bytes = 0;
    Buf buf[B_COUNT];
    Desc* d_desc = nullptr;
    Desc* h_desc = nullptr;       // pinned
    Counters* d_cnt = nullptr;
    Counters* h_cnt = nullptr;    // pinned
    HotConfig ascent_cfg[3];      // by meas_dim: dense seeding (>= kSparseSeeds per event)
    HotConfig sparse_cfg[3];      // by meas_dim: sparse seeding (fewer per event)
    HotConfig resp_cfg[3];
    bool prof = false;
    hipEvent_t ev[7] = {};        // 0..4: find_tracks / response stages, 5..6: proposer
    retina_profile prof_acc = {};
    // captured find_tracks launch sequences: every kernel reads its sizes from the
    // device descriptor and runs a fixed persistent grid, so one graph per
    // (meas_dim, launch shape, profiling) serves any batch
    bool use_graphs = true;
    struct GraphEntry {
        int D, cand, tile, grid, prof, update, prune, staged, split, small_merge;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    // the learned step (proposer, ascent, merge) captured as one graph, with
    // the by-value launch arguments it was captured with
    hipGraphExec_t learned_exec = nullptr;
    std::vector<unsigned char> learned_key;
    void* scratch = nullptr;      // this device's fixed workspace (retina_response_noalloc)
};

namespace {

const char* kNoCtx = "retina: NULL context";

int fail(retina_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(retina_ctx* c, int code, const char* fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof(msg), fmt, ap);
    va_end(ap);
    if (c) c->err = msg;
    return code;
}

#define HIP_TRY(c, expr)                                                                     \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail((c), RETINA_ERR_DEVICE, "HIP error %s at %s:%d", hipGetErrorString(_e), \
                        __FILE__, __LINE__);                                                 \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

size_t pool_bytes(const retina_ctx* c)
{
    size_t s = 0;
    for (int i = 0; i < B_COUNT; ++i) s += c->buf[i].cap;
    return s;
}

// grow-only buffer; contents are not preserved
int ensure(retina_ctx* c, int id, size_t bytes, void** out)
{
    Buf& b = c->buf[id];
    if (bytes == 0) bytes = 16;
    if (b.cap < bytes) {
        size_t want = std::max(bytes, b.cap + b.cap / 2);
        if (c->max_bytes > 0 && pool_bytes(c) - b.cap + want > (size_t)c->max_bytes) {
            want = bytes;
            if (pool_bytes(c) - b.cap + want > (size_t)c->max_bytes)
                return fail(c, RETINA_ERR_OUT_OF_MEMORY,
                            "device pool limit %lld bytes exceeded (need %zu more)",
                            (long long)c->max_bytes, want);
        }
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (hipMalloc(&b.p, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, RETINA_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", want);
        }
        b.cap = want;
    }
    *out = b.p;
    return RETINA_OK;
}

template <typename T>
int ensure_t(retina_ctx* c, int id, size_t count, T** out)
{
    void* p;
    int rc = ensure(c, id, count * sizeof(T), &p);
    *out = (T*)p;
    return rc;
}

// Fixed workspace for the allocation-free entry point: a bump allocator over
// the per-device scratch array (256-byte aligned pieces, no device work).
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};

// A pool buffer (ar == NULL) or the next piece of the arena.
template <typename T>
int take(retina_ctx* c, Arena* ar, int id, size_t count, T** out)
{
    if (!ar) return ensure_t(c, id, count, out);
    rtv::Check k;
    size_t off = 0;
    if (count > SIZE_MAX / sizeof(T)) return fail(c, RETINA_ERR_CAPACITY, "workspace request overflows");
    if (rtv::arena_take(k, ar->cap, ar->used, count * sizeof(T), &off)) return fail(c, k.code, "%s", k.msg);
    *out = reinterpret_cast<T*>(ar->base + off);
    return RETINA_OK;
}

int check_geometry(retina_ctx* c, const retina_geometry* g)
{
    rtv::Check k;
    return rtv::geometry(k, g) ? fail(c, k.code, "%s", k.msg) : RETINA_OK;
}

int check_hits(retina_ctx* c, const retina_geometry* g, const retina_hits* h)
{
    rtv::Check k;
    return rtv::hits(k, g, h) ? fail(c, k.code, "%s", k.msg) : RETINA_OK;
}

// read one int64 of a caller array in either memory space
int read_i64(retina_ctx* c, int mem, const int64_t* p, int64_t idx, int64_t* out)
{
    if (mem == RETINA_MEM_HOST) {
        *out = p[idx];
        return RETINA_OK;
    }
    HIP_TRY(c, hipMemcpyAsync(out, p + idx, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RETINA_OK;
}

int host_offsets_ok(const int64_t* off, int64_t n) { return rtv::offsets_ok(off, n); }

void fill_geometry(Desc& d, const retina_geometry* g)
{
    d.meas_dim = g->meas_dim;
    d.n_planes = g->n_planes;
    double s2 = 0.0, zmin = g->plane_z[0], zmax = g->plane_z[0];
    for (int p = 0; p < kMaxPlanes; ++p) d.plane_z[p] = p < g->n_planes ? g->plane_z[p] : 0.0f;
    for (int p = 0; p < g->n_planes; ++p) {
        const double z = g->plane_z[p];
        s2 += z * z;
        zmin = std::min(zmin, z);
        zmax = std::max(zmax, z);
    }
    d.z_first = (float)zmin;
    d.z_last = (float)zmax;
    d.z_ref = (float)sqrt(s2 / g->n_planes);
}

// clear the descriptor's fixed part (the lattice table is written by set_lattice)
void reset_desc(Desc& d)
{
    memset(&d, 0, offsetof(Desc, lat_coord));
}

// cell-centred lattice (seed lattice or search grid) into the descriptor: the
// FP32 rounding of lo + (i + 1/2)(hi - lo)/n, formed in FP64 on the host
int set_lattice(retina_ctx* c, Desc& d, const int32_t* n, const float* lo, const float* hi)
{
    rtv::Check chk;
    if (rtv::lattice_sides(chk, n)) return fail(c, chk.code, "%s", chk.msg);
    int o = 0;
    for (int k = 0; k < 2; ++k) {
        d.lattice_n[k] = n[k];
        d.lattice_lo[k] = lo[k];
        d.lattice_hi[k] = hi[k];
        for (int i = 0; i < n[k]; ++i)
            d.lat_coord[o++] = (float)((double)lo[k] + ((double)i + 0.5) * ((double)hi[k] - (double)lo[k]) / (double)n[k]);
    }
    return RETINA_OK;
}

// stage caller hits (copying host arrays into the pool when needed)
int stage_inputs(retina_ctx* c, Desc& d, const retina_geometry* g, const retina_hits* h, int64_t n_hits,
                 Arena* ar = nullptr)
{
    d.n_events = h->n_events;
    d.n_hits = n_hits;
    const int D = g->meas_dim;
    if (h->mem == RETINA_MEM_DEVICE) {
        d.in_off = h->event_offsets;
        d.in_x = h->x;
        d.in_y = D == 2 ? h->y : nullptr;
        d.in_plane = h->plane;
    } else {
        if (ar) return fail(c, RETINA_ERR_INVALID_ARG, "the fixed-workspace call takes device memory only");
        int64_t* off;
        float *x, *y = nullptr;
        int32_t* pl;
        int rc;
        if ((rc = ensure_t(c, B_INOFF, h->n_events + 1, &off))) return rc;
        if ((rc = ensure_t(c, B_INX, n_hits, &x))) return rc;
        if (D == 2 && (rc = ensure_t(c, B_INY, n_hits, &y))) return rc;
        if ((rc = ensure_t(c, B_INPL, n_hits, &pl))) return rc;
        HIP_TRY(c, hipMemcpyAsync(off, h->event_offsets, sizeof(int64_t) * (h->n_events + 1),
                                  hipMemcpyHostToDevice, c->stream));
        if (n_hits) {
            HIP_TRY(c, hipMemcpyAsync(x, h->x, sizeof(float) * n_hits, hipMemcpyHostToDevice, c->stream));
            if (D == 2)
                HIP_TRY(c, hipMemcpyAsync(y, h->y, sizeof(float) * n_hits, hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(pl, h->plane, sizeof(int32_t) * n_hits, hipMemcpyHostToDevice, c->stream));
        }
        d.in_off = off;
        d.in_x = x;
        d.in_y = y;
        d.in_plane = pl;
    }
    int rc;
    const int64_t E = h->n_events;
    if ((rc = take(c, ar, B_HITS, (size_t)std::max<int64_t>(n_hits, 1) * D, &d.hits))) return rc;
    if ((rc = take(c, ar, B_POFF, (size_t)E * (g->n_planes + 1) + 1, &d.plane_off))) return rc;
    if ((rc = take(c, ar, B_NHITS, (size_t)E + 1, &d.ev_nhits))) return rc;
    if ((rc = take(c, ar, B_SOFF, (size_t)E + 1, &d.seed_off))) return rc;
    if ((rc = take(c, ar, B_ORDER, (size_t)E + 1, &d.order))) return rc;
    return RETINA_OK;
}

int device_error(retina_ctx* c, uint32_t err)
{
    if (err & kErrOffsets) return fail(c, RETINA_ERR_INVALID_ARG, "event_offsets must start at 0 and be non-decreasing");
    if (err & kErrCoord) return fail(c, RETINA_ERR_INVALID_ARG, "a hit coordinate is NaN or infinite");
    if (err & kErrPlane) return fail(c, RETINA_ERR_INVALID_ARG, "a hit plane index is outside [0, n_planes)");
    if (err & kErrSeedOff) return fail(c, RETINA_ERR_INVALID_ARG, "seed_offsets must start at 0 and be non-decreasing");
    if (err & kErrSeedVal) return fail(c, RETINA_ERR_INVALID_ARG, "an explicit seed is NaN or infinite");
    if (err & kErrThetaOff) return fail(c, RETINA_ERR_INVALID_ARG, "theta_offsets must start at 0 and be non-decreasing");
    return fail(c, RETINA_ERR_INTERNAL, "device error bits 0x%x", err);
}

// find_tracks batches averaging fewer seeds per event than this run the
// ascent with the sparse-seeding launch shape (tuning kernel 2)
constexpr int64_t kSparseSeeds = 512;
// one candidate per lane with Newton steps runs several lanes per seed (each
// over a share of every plane's hits): an event's ~100-250 seeds then fill
// the work-groups' waves
constexpr bool kSplitSeeds = true;
// retina_response hit splitting: at most this many parts, each part at least
// this many hits of an average event
constexpr int kRespMaxParts = 32;
constexpr int64_t kRespMinPartHits = 128;

HotConfig& tuning_slot(retina_ctx* c, int D, int kernel)
{
    return kernel == 0 ? c->ascent_cfg[D] : kernel == 2 ? c->sparse_cfg[D] : c->resp_cfg[D];
}

HotConfig default_hot(const retina_ctx* c, int D, bool ascent)
{
    HotConfig h;
    h.cand = ascent ? 2 : 1;
    // ascent: 5632 hits (44 KB) + the line-search list (8.5 KB) keep three
    // work-groups per CU within 160 KB of LDS
    h.tile_hits = D == 2 ? (ascent ? 5632 : 6144) : 8192;
    h.grid = c->n_cu * hot_max_blocks_per_cu(D, h, ascent);
    return h;
}

// event i of the profiled launch sequence (no-op unless profiling)
void prof_mark(retina_ctx* c, int i)
{
    if (c->prof) (void)hipEventRecord(c->ev[i], c->stream);
}

// after the stream has drained: accumulate the kernel times
void prof_collect(retina_ctx* c)
{
    if (!c->prof) return;
    float t[4];
    for (int i = 0; i < 4; ++i)
        if (hipEventElapsedTime(&t[i], c->ev[i], c->ev[i + 1]) != hipSuccess) t[i] = 0.0f;
    float tot = 0.0f;
    if (hipEventElapsedTime(&tot, c->ev[0], c->ev[4]) != hipSuccess) tot = 0.0f;
    (void)hipGetLastError();  // a failed timing query must not linger as the thread's last error
    c->prof_acc.calls += 1;
    c->prof_acc.ms_stage += t[0];
    c->prof_acc.ms_plan += t[1];
    c->prof_acc.ms_hot += t[2];
    c->prof_acc.ms_merge += t[3];
    c->prof_acc.ms_total += tot;
    c->prof_acc.exec_pairs += (double)c->h_cnt->exec_pairs;
    c->prof_acc.exec_rpairs += (double)c->h_cnt->exec_rpairs;
}

// The find_tracks device sequence on stream st (profiling marks included when on).
void tracks_sequence(retina_ctx* c, int D, const HotConfig& hc, hipStream_t st)
{
    auto mark = [&](int i) {
        if (c->prof) (void)hipEventRecord(c->ev[i], st);
    };
    mark(0);
    launch_reset(c->d_desc, st);
    if (!hc.staged) launch_stage(c->d_desc, c->n_cu * 8, st);
    if (hc.prune) launch_sort_planes(c->d_desc, c->n_cu * 8, st);
    mark(1);
    launch_plan_tracks(c->d_desc, st);
    mark(2);
    launch_ascent(c->d_desc, D, hc, st);
    mark(3);
    launch_merge(c->d_desc, D, c->n_cu, hc.small_merge != 0, st);
    launch_finalize(c->d_desc, st);
    launch_emit(c->d_desc, D, c->n_cu * 4, st);
    mark(4);
}

// Run the sequence, through a captured graph when possible.  Capture happens
// on the library's own stream (the caller's may be the legacy null stream);
// the instantiated graph is then launched on the context's stream.
int run_tracks(retina_ctx* c, int D, const HotConfig& hc)
{
    // profiled calls launch eagerly: the per-kernel events are recorded on the
    // caller-visible stream, not inside a graph
    if (c->use_graphs && !c->prof) {
        hipGraphExec_t exec = nullptr;
        for (auto& g : c->graphs)
            if (g.D == D && g.cand == hc.cand && g.tile == hc.tile_hits && g.grid == hc.grid &&
                g.prof == (int)c->prof && g.update == hc.update && g.prune == hc.prune &&
                g.staged == hc.staged && g.split == hc.split && g.small_merge == hc.small_merge)
                exec = g.exec;
        if (!exec) {
            hipGraph_t graph = nullptr;
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            bool ok = hipStreamBeginCapture(c->own, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                tracks_sequence(c, D, hc, c->own);
                ok = hipStreamEndCapture(c->own, &graph) == hipSuccess && graph;
            }
            if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            if (!ok) {
                (void)hipGetLastError();
                c->use_graphs = false;  // capture unsupported here: launch eagerly from now on
            } else {
                c->graphs.push_back({D, hc.cand, hc.tile_hits, hc.grid, (int)c->prof, hc.update, hc.prune, hc.staged,
                                     hc.split, hc.small_merge, exec});
            }
        }
        if (exec) {
            HIP_TRY(c, hipGraphLaunch(exec, c->stream));
            return RETINA_OK;
        }
    }
    tracks_sequence(c, D, hc, c->stream);
    HIP_TRY(c, hipGetLastError());
    return RETINA_OK;
}

int upload_desc(retina_ctx* c)
{
    // the fixed part and the used entries of the lattice table
    const Desc& d = *c->h_desc;
    const size_t n_lat = (size_t)std::max(d.lattice_n[0], 0) + (size_t)std::max(d.lattice_n[1], 0);
    const size_t bytes = offsetof(Desc, lat_coord) + sizeof(float) * std::min<size_t>(n_lat, 2 * kMaxLatticeSide);
    HIP_TRY(c, hipMemcpyAsync(c->d_desc, c->h_desc, bytes, hipMemcpyHostToDevice, c->stream));
    return RETINA_OK;
}

int download_counters(retina_ctx* c)
{
    HIP_TRY(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RETINA_OK;
}

}  // namespace

// Per-device fixed workspace of retina_response_noalloc.  In host code the
// array's name is a stand-in, not a device address: every host-side use goes
// through the address hipGetSymbolAddress returns for the current device
// (kept per device in g_scratch_addr, taken once by retina_create).
constexpr size_t kScratchBytes = (size_t)RETINA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_addr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// once per device, with that device current
int scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return RETINA_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return RETINA_ERR_DEVICE;
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return RETINA_OK;
}
}  // namespace

extern "C" {

int retina_create(int device_ordinal, retina_ctx** out)
{
    if (!out) return RETINA_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return RETINA_ERR_DEVICE;
    }
    if (device_ordinal < 0 || device_ordinal >= n) return RETINA_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device_ordinal) != hipSuccess) return RETINA_ERR_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return RETINA_ERR_DEVICE;
    DeviceGuard guard(device_ordinal);
    retina_ctx* c = new retina_ctx();
    c->device = device_ordinal;
    c->n_cu = prop.multiProcessorCount;
    snprintf(c->arch, sizeof(c->arch), "%.20s", prop.gcnArchName);
    for (char* p = c->arch; *p; ++p)
        if (*p == ':' || *p == ' ') { *p = 0; break; }
    c->lds_max = prop.sharedMemPerBlock;
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&c->d_desc, sizeof(Desc)) != hipSuccess ||
        hipHostMalloc(&c->h_desc, sizeof(Desc), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&c->d_cnt, sizeof(Counters)) != hipSuccess ||
        hipHostMalloc(&c->h_cnt, sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
        retina_destroy(c);
        return RETINA_ERR_DEVICE;
    }
    c->stream = c->own;
    if (scratch_address(device_ordinal, &c->scratch) != RETINA_OK) {
        retina_destroy(c);
        return RETINA_ERR_DEVICE;
    }
    for (int D = 1; D <= 2; ++D) {
        c->ascent_cfg[D] = default_hot(c, D, true);
        c->resp_cfg[D] = default_hot(c, D, false);
        // few seeds per event (learned seeding): one candidate per lane with
        // several lanes per seed; a 5632-hit tile keeps all but the largest
        // events of an uneven batch resident (their line searches run
        // wave-local), at three work-groups per CU
        HotConfig h = c->ascent_cfg[D];
        h.cand = 1;
        h.tile_hits = D == 2 ? 5632 : 8192;
        h.grid = c->n_cu * hot_max_blocks_per_cu(D, h, true);
        c->sparse_cfg[D] = h;
    }
    *out = c;
    return RETINA_OK;
}

void retina_destroy(retina_ctx* c)
{
    if (!c) return;
    DeviceGuard guard(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < B_COUNT; ++i)
        if (c->buf[i].p) (void)hipFree(c->buf[i].p);
    if (c->d_desc) (void)hipFree(c->d_desc);
    if (c->h_desc) (void)hipHostFree(c->h_desc);
    if (c->d_cnt) (void)hipFree(c->d_cnt);
    if (c->h_cnt) (void)hipHostFree(c->h_cnt);
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    if (c->learned_exec) (void)hipGraphExecDestroy(c->learned_exec);
    for (int i = 0; i < 7; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->own) (void)hipStreamDestroy(c->own);
    (void)hipGetLastError();  // leave no error of ours behind for the caller's next check
    delete c;
}

const char* retina_last_error(const retina_ctx* c)
{
    if (!c) return kNoCtx;
    return c->err.c_str();
}

int retina_set_stream(retina_ctx* c, void* s)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->stream = s ? (hipStream_t)s : c->own;
    return RETINA_OK;
}

int retina_set_max_device_bytes(retina_ctx* c, int64_t max_bytes)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    if (max_bytes < 0) return fail(c, RETINA_ERR_INVALID_ARG, "max_bytes < 0");
    c->max_bytes = max_bytes;
    return RETINA_OK;
}

int retina_set_profiling(retina_ctx* c, int32_t enable)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    DeviceGuard guard(c->device);
    if (enable && !c->ev[0]) {
        for (int i = 0; i < 7; ++i)
            HIP_TRY(c, hipEventCreate(&c->ev[i]));
    }
    c->prof = enable != 0;
    return RETINA_OK;
}

int retina_get_profile(const retina_ctx* c, retina_profile* out)
{
    if (!c || !out) return RETINA_ERR_INVALID_ARG;
    *out = c->prof_acc;
    return RETINA_OK;
}

int retina_profile_reset(retina_ctx* c)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->prof_acc = retina_profile{};
    return RETINA_OK;
}

int retina_set_tuning(retina_ctx* c, int32_t meas_dim, int32_t kernel, int32_t cand, int32_t tile_hits)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    if (meas_dim != 1 && meas_dim != 2) return fail(c, RETINA_ERR_INVALID_ARG, "meas_dim must be 1 or 2");
    if (kernel < 0 || kernel > 2) return fail(c, RETINA_ERR_INVALID_ARG, "kernel must be 0, 1 or 2");
    if (cand != 1 && cand != 2) return fail(c, RETINA_ERR_INVALID_ARG, "cand must be 1 or 2");
    const int max_tile = meas_dim == 2 ? 16384 : 32768;
    if (tile_hits < 256 || tile_hits > max_tile)
        return fail(c, RETINA_ERR_INVALID_ARG, "tile_hits must be in [256, %d]", max_tile);
    if ((size_t)tile_hits * meas_dim * sizeof(float) + 4096 > c->lds_max)
        return fail(c, RETINA_ERR_INVALID_ARG, "tile_hits %d exceeds this device's %zu bytes of LDS per work-group",
                    tile_hits, c->lds_max);
    DeviceGuard guard(c->device);
    HotConfig h;
    h.cand = cand;
    h.tile_hits = tile_hits;
    const int per_cu = hot_max_blocks_per_cu(meas_dim, h, kernel != 1);
    h.grid = c->n_cu * per_cu;
    tuning_slot(c, meas_dim, kernel) = h;
    return RETINA_OK;
}

int retina_get_tuning(const retina_ctx* c, int32_t meas_dim, int32_t kernel, int32_t* cand,
                      int32_t* tile_hits, int32_t* grid)
{
    if (!c || (meas_dim != 1 && meas_dim != 2) || kernel < 0 || kernel > 2) return RETINA_ERR_INVALID_ARG;
    const HotConfig& h = tuning_slot(const_cast<retina_ctx*>(c), meas_dim, kernel);
    if (cand) *cand = h.cand;
    if (tile_hits) *tile_hits = h.tile_hits;
    if (grid) *grid = h.grid;
    return RETINA_OK;
}

}  // extern "C"

namespace {

// Eq. (1) and its derivatives at caller lines; workspace from the pool or,
// with ar != NULL, from the fixed arena (no allocation of any kind).
int response_impl(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const float* theta,
                  int64_t n_theta, const int64_t* theta_offsets, float sigma, uint32_t want, float* R,
                  float* grad, float* hess, Arena* ar)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_geometry(c, g)) || (rc = check_hits(c, g, h))) return rc;
    {
        rtv::Check k;
        if (rtv::response_args(k, h, theta, n_theta, theta_offsets, sigma, want, R, grad, hess))
            return fail(c, k.code, "%s", k.msg);
    }
    if (h->n_events == 0 || n_theta == 0) return RETINA_OK;
    DeviceGuard guard(c->device);
    const int D = g->meas_dim, NP = 2 * D, NH = NP * (NP + 1) / 2;
    const int64_t E = h->n_events;
    const bool host = h->mem == RETINA_MEM_HOST;
    if (host && !host_offsets_ok(h->event_offsets, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "event_offsets must start at 0 and be non-decreasing");
    if (host && theta_offsets && !host_offsets_ok(theta_offsets, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "theta_offsets must start at 0 and be non-decreasing");
    int64_t n_hits, th_last = n_theta;
    if ((rc = read_i64(c, h->mem, h->event_offsets, E, &n_hits))) return rc;
    if (theta_offsets && (rc = read_i64(c, h->mem, theta_offsets, E, &th_last))) return rc;
    if (th_last != n_theta) return fail(c, RETINA_ERR_INVALID_ARG, "theta_offsets[n_events] != n_theta");
    if (n_hits < 0 || n_hits > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "bad total hit count");

    Desc& d = *c->h_desc;
    reset_desc(d);
    fill_geometry(d, g);
    d.cnt = c->d_cnt;
    if ((rc = stage_inputs(c, d, g, h, n_hits, ar))) return rc;
    const HotConfig hc = c->resp_cfg[D];
    d.seeds_per_item = hot_seeds_per_item(hc);
    // few (event, theta block) items leave CUs idle: split each event's hits
    // into parts (each part at least kRespMinPartHits hits on average), reduced
    // in part order afterwards
    const int64_t blocks = n_theta / d.seeds_per_item + E;
    int parts = 1;
    while (parts < kRespMaxParts && blocks * parts < (int64_t)hc.grid &&
           n_hits / (E * parts * 2) >= kRespMinPartHits)
        parts *= 2;
    const size_t n_acc = D == 2 ? 16 : 8;
    if (ar) {
        // the fixed workspace: fewer parts when the partial sums would not fit
        // (results then differ only in FP32 summation order)
        const size_t left = ar->cap - ar->used;
        while (parts > 1 && ((size_t)(n_theta / d.seeds_per_item + E + 1) * parts * sizeof(int2) +
                             (size_t)parts * n_theta * n_acc * sizeof(float) + 2048) > left)
            parts /= 2;
    }
    d.resp_parts = parts;
    d.resp_ntheta = n_theta;
    d.items_cap = (n_theta / d.seeds_per_item + E + 1) * parts;
    if ((rc = take(c, ar, B_ITEMS, (size_t)d.items_cap, &d.items))) return rc;
    if (parts > 1 && (rc = take(c, ar, B_RESPPART, (size_t)parts * n_theta * n_acc, &d.resp_partial)))
        return rc;
    d.want = want | RETINA_WANT_R;
    d.resp_sigma = sigma;
    // inputs
    if (host) {
        float* th;
        int64_t* to;
        if ((rc = ensure_t(c, B_INTH, (size_t)n_theta * NP, &th))) return rc;
        if ((rc = ensure_t(c, B_INTHOFF, (size_t)E + 1, &to))) return rc;
        HIP_TRY(c, hipMemcpyAsync(th, theta, sizeof(float) * n_theta * NP, hipMemcpyHostToDevice, c->stream));
        if (theta_offsets) {
            HIP_TRY(c, hipMemcpyAsync(to, theta_offsets, sizeof(int64_t) * (E + 1), hipMemcpyHostToDevice, c->stream));
        } else {
            const int64_t tmp[2] = {0, n_theta};
            HIP_TRY(c, hipMemcpyAsync(to, tmp, sizeof(tmp), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
        d.in_theta = th;
        d.in_theta_off = to;
        if ((rc = ensure_t(c, B_OUTR, (size_t)n_theta, &d.out_R))) return rc;
        if ((want & RETINA_WANT_GRAD) && (rc = ensure_t(c, B_OUTG, (size_t)n_theta * NP, &d.out_grad))) return rc;
        if ((want & RETINA_WANT_HESS) && (rc = ensure_t(c, B_OUTH, (size_t)n_theta * NH, &d.out_hess))) return rc;
    } else {
        d.in_theta = theta;
        if (theta_offsets) {
            d.in_theta_off = theta_offsets;
        } else {
            d.single_off[0] = 0;
            d.single_off[1] = n_theta;
            d.in_theta_off = c->d_desc->single_off;  // travels with the descriptor upload
        }
        d.out_R = R;
        d.out_grad = grad;
        d.out_hess = hess;
    }
    if ((rc = upload_desc(c))) return rc;
    prof_mark(c, 0);
    launch_reset(c->d_desc, c->stream);
    launch_stage(c->d_desc, (int)std::min<int64_t>(E, (int64_t)c->n_cu * 8), c->stream);
    prof_mark(c, 1);
    launch_plan_response(c->d_desc, c->stream);
    prof_mark(c, 2);
    launch_response(c->d_desc, D, hc, (want & (RETINA_WANT_GRAD | RETINA_WANT_HESS)) != 0, c->stream);
    if (parts > 1)
        launch_response_reduce(c->d_desc, D, (want & (RETINA_WANT_GRAD | RETINA_WANT_HESS)) != 0, n_theta, c->stream);
    prof_mark(c, 3);
    prof_mark(c, 4);
    HIP_TRY(c, hipGetLastError());
    if ((rc = download_counters(c))) return rc;
    prof_collect(c);
    if (c->h_cnt->err) return device_error(c, c->h_cnt->err);
    if (host) {
        HIP_TRY(c, hipMemcpyAsync(R, d.out_R, sizeof(float) * n_theta, hipMemcpyDeviceToHost, c->stream));
        if (want & RETINA_WANT_GRAD)
            HIP_TRY(c, hipMemcpyAsync(grad, d.out_grad, sizeof(float) * n_theta * NP, hipMemcpyDeviceToHost, c->stream));
        if (want & RETINA_WANT_HESS)
            HIP_TRY(c, hipMemcpyAsync(hess, d.out_hess, sizeof(float) * n_theta * NH, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return RETINA_OK;
}

}  // namespace

extern "C" {

int retina_response(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const float* theta,
                    int64_t n_theta, const int64_t* theta_offsets, float sigma, uint32_t want, float* R,
                    float* grad, float* hess)
{
    return response_impl(c, g, h, theta, n_theta, theta_offsets, sigma, want, R, grad, hess, nullptr);
}

int retina_response_noalloc(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const float* theta,
                            int64_t n_theta, const int64_t* theta_offsets, float sigma, uint32_t want,
                            float* R, float* grad, float* hess)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    if (!c->scratch)
        return fail(c, RETINA_ERR_DEVICE, "the fixed device workspace has no address on device %d", c->device);
    if (h && h->mem != RETINA_MEM_DEVICE)
        return fail(c, RETINA_ERR_INVALID_ARG, "retina_response_noalloc takes device memory only (hits.mem = %d)",
                    h->mem);
    Arena ar;
    ar.base = static_cast<char*>(c->scratch);
    ar.cap = kScratchBytes;
    return response_impl(c, g, h, theta, n_theta, theta_offsets, sigma, want, R, grad, hess, &ar);
}

int retina_grid_search(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const retina_grid* grid,
                       float* R_grid, retina_track* tracks, int64_t capacity, int64_t* track_offsets)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_geometry(c, g)) || (rc = check_hits(c, g, h))) return rc;
    if (!grid) return fail(c, RETINA_ERR_INVALID_ARG, "grid is NULL");
    if (grid->n[0] < 1 || grid->n[1] < 1 || grid->n[0] > kMaxLatticeSide || grid->n[1] > kMaxLatticeSide)
        return fail(c, RETINA_ERR_INVALID_ARG, "grid n must be in [1, %d] per dimension", kMaxLatticeSide);
    for (int i = 0; i < 2; ++i)
        if (!isfinite(grid->lo[i]) || !isfinite(grid->hi[i]) || !(grid->lo[i] < grid->hi[i]))
            return fail(c, RETINA_ERR_INVALID_ARG, "grid box must be finite with lo < hi");
    if (!(grid->sigma > 0.0f) || !isfinite(grid->sigma))
        return fail(c, RETINA_ERR_INVALID_ARG, "grid sigma must be finite and > 0");
    if (!(grid->R0 > 0.0f) || !isfinite(grid->R0)) return fail(c, RETINA_ERR_INVALID_ARG, "grid R0 must be finite and > 0");
    if (capacity < 0) return fail(c, RETINA_ERR_INVALID_ARG, "capacity < 0");
    if (!track_offsets) return fail(c, RETINA_ERR_INVALID_ARG, "track_offsets is NULL");
    if (capacity > 0 && !tracks) return fail(c, RETINA_ERR_INVALID_ARG, "tracks is NULL");
    DeviceGuard guard(c->device);
    const int D = g->meas_dim;
    const int64_t E = h->n_events;
    const bool host = h->mem == RETINA_MEM_HOST;
    if (host && !host_offsets_ok(h->event_offsets, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "event_offsets must start at 0 and be non-decreasing");
    if (E == 0) {
        if (host) track_offsets[0] = 0;
        else HIP_TRY(c, hipMemsetAsync(track_offsets, 0, sizeof(int64_t), c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return RETINA_OK;
    }
    int64_t n_hits;
    if ((rc = read_i64(c, h->mem, h->event_offsets, E, &n_hits))) return rc;
    if (n_hits < 0 || n_hits > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "bad total hit count");
    const int64_t n_cells = (int64_t)grid->n[0] * grid->n[1], n_theta = E * n_cells;
    const int64_t nch = (n_cells + kGridChunk - 1) / kGridChunk;
    if (E * nch > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "batch too large for one grid search");

    Desc& d = *c->h_desc;
    reset_desc(d);
    fill_geometry(d, g);
    d.cnt = c->d_cnt;
    if ((rc = stage_inputs(c, d, g, h, n_hits))) return rc;
    const HotConfig hc = c->resp_cfg[D];
    d.seeds_per_item = hot_seeds_per_item(hc);
    const int64_t blocks = n_theta / d.seeds_per_item + E;
    int parts = 1;
    while (parts < kRespMaxParts && blocks * parts < (int64_t)hc.grid && n_hits / (E * parts * 2) >= kRespMinPartHits)
        parts *= 2;
    d.resp_parts = parts;
    d.resp_ntheta = n_theta;
    d.items_cap = (n_theta / d.seeds_per_item + E + 1) * parts;
    if ((rc = ensure_t(c, B_ITEMS, (size_t)d.items_cap, &d.items))) return rc;
    if (parts > 1 && (rc = ensure_t(c, B_RESPPART, (size_t)parts * n_theta * (D == 2 ? 16 : 8), &d.resp_partial)))
        return rc;
    d.want = RETINA_WANT_R;
    d.resp_sigma = grid->sigma;
    d.resp_grid = 1;
    if ((rc = set_lattice(c, d, grid->n, grid->lo, grid->hi))) return rc;
    d.grid_R0 = grid->R0;
    d.grid_chunks = (int32_t)nch;
    if (!host && R_grid) d.out_R = R_grid;
    else if ((rc = ensure_t(c, B_GRID, (size_t)n_theta, &d.out_R))) return rc;
    if ((rc = ensure_t(c, B_GRIDCNT, (size_t)(E * nch), &d.grid_cnt)) ||
        (rc = ensure_t(c, B_GRIDBASE, (size_t)(E * nch), &d.grid_base)))
        return rc;
    const int64_t host_cap = std::min<int64_t>(capacity, n_theta);
    if (host) {
        if ((rc = ensure_t(c, B_OUTTR, (size_t)std::max<int64_t>(host_cap, 1), &d.out_tracks)) ||
            (rc = ensure_t(c, B_OUTTOFF, (size_t)E + 1, &d.out_track_off)))
            return rc;
        d.out_capacity = host_cap;
    } else {
        d.out_tracks = tracks;
        d.out_capacity = capacity;
        d.out_track_off = track_offsets;
    }
    if ((rc = upload_desc(c))) return rc;
    prof_mark(c, 0);
    launch_reset(c->d_desc, c->stream);
    launch_stage(c->d_desc, (int)std::min<int64_t>(E, (int64_t)c->n_cu * 8), c->stream);
    prof_mark(c, 1);
    launch_plan_grid(c->d_desc, c->stream);
    prof_mark(c, 2);
    launch_response(c->d_desc, D, hc, false, c->stream);
    if (parts > 1) launch_response_reduce(c->d_desc, D, false, n_theta, c->stream);
    prof_mark(c, 3);
    launch_grid_peaks(c->d_desc, D, E * nch, c->stream);
    prof_mark(c, 4);
    HIP_TRY(c, hipGetLastError());
    if ((rc = download_counters(c))) return rc;
    prof_collect(c);
    const uint32_t err = c->h_cnt->err;
    const int64_t total = c->h_cnt->total_tracks;
    if (err & ~kErrCapacity) return device_error(c, err);
    if (err & kErrCapacity || total > capacity) {
        if (host) track_offsets[E] = total;
        return fail(c, RETINA_ERR_CAPACITY, "%lld peaks found, capacity %lld", (long long)total, (long long)capacity);
    }
    if (host) {
        if (total)
            HIP_TRY(c, hipMemcpyAsync(tracks, d.out_tracks, sizeof(retina_track) * total, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(track_offsets, d.out_track_off, sizeof(int64_t) * (E + 1), hipMemcpyDeviceToHost, c->stream));
    }
    if (R_grid && (host || R_grid != d.out_R))
        HIP_TRY(c, hipMemcpyAsync(R_grid, d.out_R, sizeof(float) * n_theta, host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RETINA_OK;
}

// seeds_dev: explicit seeds live in device memory (the learned path passes its
// own device-resident seeds together with host or device hits)
static int find_tracks_impl(retina_ctx* c, const retina_geometry* g, const retina_hits* h,
                            const retina_params* P, retina_track* tracks, int64_t capacity,
                            int64_t* track_offsets, int32_t* event_flags, const retina_seed_out* so,
                            bool seeds_dev, bool staged = false)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_geometry(c, g)) || (rc = check_hits(c, g, h))) return rc;
    {
        rtv::Check k;
        if (rtv::method_params(k, P, capacity, tracks, track_offsets)) return fail(c, k.code, "%s", k.msg);
    }
    DeviceGuard guard(c->device);
    const int D = g->meas_dim, NP = 2 * D;
    const int64_t E = h->n_events;
    const bool host = h->mem == RETINA_MEM_HOST;
    if (host && !host_offsets_ok(h->event_offsets, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "event_offsets must start at 0 and be non-decreasing");
    if (!seeds_dev && P->seed_mode == RETINA_SEED_EXPLICIT && !host_offsets_ok(P->seed_offsets, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "seed_offsets must start at 0 and be non-decreasing");
    if (E == 0) {
        if (host) track_offsets[0] = 0;
        else HIP_TRY(c, hipMemsetAsync(track_offsets, 0, sizeof(int64_t), c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return RETINA_OK;
    }
    int64_t n_hits, n_seeds;
    if ((rc = read_i64(c, h->mem, h->event_offsets, E, &n_hits))) return rc;
    if (n_hits < 0 || n_hits > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "bad total hit count");
    if (P->seed_mode == RETINA_SEED_EXPLICIT) {
        if ((rc = read_i64(c, seeds_dev ? RETINA_MEM_DEVICE : RETINA_MEM_HOST, P->seed_offsets, E, &n_seeds))) return rc;
        if (n_seeds < 0 || n_seeds > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "bad total seed count");
        rtv::Check k;
        if (!seeds_dev && rtv::host_seeds(k, P->seeds, n_seeds * NP)) return fail(c, k.code, "%s", k.msg);
    } else {
        n_seeds = E * (int64_t)P->lattice_n[0] * P->lattice_n[1];
        if (n_seeds > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "too many seeds in the batch");
    }
    if (so && so->capacity < n_seeds)
        return fail(c, RETINA_ERR_CAPACITY, "seeds_out holds %lld seeds, %lld needed",
                    (long long)so->capacity, (long long)n_seeds);

    Desc& d = *c->h_desc;
    reset_desc(d);
    fill_geometry(d, g);
    d.cnt = c->d_cnt;
    if ((rc = stage_inputs(c, d, g, h, n_hits))) return rc;
    HotConfig hc = n_seeds < kSparseSeeds * E ? c->sparse_cfg[D] : c->ascent_cfg[D];
    if (P->update != RETINA_UPDATE_NEWTON) {
        // the alternative rules run one candidate per lane (the sparse shape)
        hc = c->sparse_cfg[D];
        hc.cand = 1;
        hc.update = P->update;
    }
    hc.prune = P->prune_u > 0.0f;
    hc.staged = staged;
    if (kSplitSeeds && hc.cand == 1 && hc.update == RETINA_UPDATE_NEWTON) {
        hc.split = 1;
        hc.grid = c->n_cu * hot_max_blocks_per_cu(D, hc, true);
    }
    hc.small_merge = n_seeds <= (int64_t)kMergeSmallKeys * E;
    d.seeds_per_item = hot_seeds_per_item(hc);
    d.half_parts = hc.split;
    d.items_cap = n_seeds / d.seeds_per_item + 2 * E + 1;
    if ((rc = ensure_t(c, B_ITEMS, (size_t)d.items_cap, &d.items))) return rc;
    d.seed_mode = P->seed_mode;
    if (P->seed_mode == RETINA_SEED_LATTICE && (rc = set_lattice(c, d, P->lattice_n, P->lattice_lo, P->lattice_hi)))
        return rc;
    d.n_sigma = P->n_sigma;
    for (int i = 0; i < P->n_sigma; ++i) d.sigma[i] = P->sigma[i];
    d.sigma_final = P->sigma_final;
    d.n_final_steps = P->n_final_steps;
    d.n_polish = P->n_polish;
    d.ls_trials = P->ls_trials;
    d.n_slope_steps = P->n_slope_steps;
    d.armijo_c1 = P->armijo_c1;
    d.step_cap = P->step_cap_sigmas;
    d.small_step = P->small_step_sigmas;
    d.conv_tol = P->conv_tol;
    d.R0 = P->R0;
    d.d_merge = P->d_merge;
    d.prune_u = P->prune_u;
    if (P->prune_u > 0.0f && (rc = ensure_t(c, B_EVSORT, (size_t)E, &d.ev_sorted))) return rc;
    if (P->seed_mode == RETINA_SEED_EXPLICIT) {
        if (!seeds_dev) {
            double* s;
            int64_t* o;
            if ((rc = ensure_t(c, B_INSEEDS, (size_t)std::max<int64_t>(n_seeds, 1) * NP, &s))) return rc;
            if ((rc = ensure_t(c, B_INSOFF, (size_t)E + 1, &o))) return rc;
            if (n_seeds)
                HIP_TRY(c, hipMemcpyAsync(s, P->seeds, sizeof(double) * n_seeds * NP, hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(o, P->seed_offsets, sizeof(int64_t) * (E + 1), hipMemcpyHostToDevice, c->stream));
            d.in_seeds = s;
            d.in_seed_off = o;
        } else {
            d.in_seeds = P->seeds;
            d.in_seed_off = P->seed_offsets;
        }
    }
    const size_t ns1 = (size_t)std::max<int64_t>(n_seeds, 1);
    if ((rc = ensure_t(c, B_STH, ns1 * 4, &d.s_theta)) || (rc = ensure_t(c, B_SR, ns1, &d.s_R)) ||
        (rc = ensure_t(c, B_SFL, ns1, &d.s_flags)) || (rc = ensure_t(c, B_SNR, ns1, &d.s_nreval)) ||
        (rc = ensure_t(c, B_MLEAD, ns1, &d.m_leader)) || (rc = ensure_t(c, B_MMEM, ns1, &d.m_members)) ||
        (rc = ensure_t(c, B_MKEYS, ns1 * 2, &d.m_keys)) || (rc = ensure_t(c, B_EVNT, (size_t)E, &d.ev_ntracks)) ||
        (rc = ensure_t(c, B_EVFL, (size_t)E, &d.ev_flags)) || (rc = ensure_t(c, B_EVTOFF, (size_t)E + 1, &d.ev_toff)))
        return rc;
    // outputs
    const int64_t host_cap = std::min<int64_t>(capacity, n_seeds);
    if (host) {
        if ((rc = ensure_t(c, B_OUTTR, (size_t)std::max<int64_t>(host_cap, 1), &d.out_tracks)) ||
            (rc = ensure_t(c, B_OUTTOFF, (size_t)E + 1, &d.out_track_off)))
            return rc;
        d.out_capacity = host_cap;
        if (event_flags && (rc = ensure_t(c, B_OUTEVF, (size_t)E, &d.out_ev_flags))) return rc;
        if (so) {
            if (so->theta && (rc = ensure_t(c, B_OUTSTH, ns1 * NP, &d.out_s_theta))) return rc;
            if (so->R && (rc = ensure_t(c, B_OUTSR, ns1, &d.out_s_R))) return rc;
            if (so->flags && (rc = ensure_t(c, B_OUTSFL, ns1, &d.out_s_flags))) return rc;
            if (so->n_reval && (rc = ensure_t(c, B_OUTSNR, ns1, &d.out_s_nreval))) return rc;
        }
    } else {
        d.out_tracks = tracks;
        d.out_capacity = capacity;
        d.out_track_off = track_offsets;
        d.out_ev_flags = event_flags;
        if (so) {
            d.out_s_theta = so->theta;
            d.out_s_R = so->R;
            d.out_s_flags = so->flags;
            d.out_s_nreval = so->n_reval;
        }
    }
    if ((rc = upload_desc(c))) return rc;
    if ((rc = run_tracks(c, D, hc))) return rc;
    if ((rc = download_counters(c))) return rc;
    prof_collect(c);
    const uint32_t err = c->h_cnt->err;
    const int64_t total = c->h_cnt->total_tracks;
    if (err & ~kErrCapacity) return device_error(c, err);
    if (err & kErrCapacity || total > capacity) {
        if (host) track_offsets[E] = total;
        return fail(c, RETINA_ERR_CAPACITY, "%lld tracks found, capacity %lld", (long long)total,
                    (long long)capacity);
    }
    if (host) {
        if (total)
            HIP_TRY(c, hipMemcpyAsync(tracks, d.out_tracks, sizeof(retina_track) * total, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(track_offsets, d.out_track_off, sizeof(int64_t) * (E + 1), hipMemcpyDeviceToHost, c->stream));
        if (event_flags)
            HIP_TRY(c, hipMemcpyAsync(event_flags, d.out_ev_flags, sizeof(int32_t) * E, hipMemcpyDeviceToHost, c->stream));
        if (so && n_seeds) {
            if (so->theta) HIP_TRY(c, hipMemcpyAsync(so->theta, d.out_s_theta, sizeof(double) * n_seeds * NP, hipMemcpyDeviceToHost, c->stream));
            if (so->R) HIP_TRY(c, hipMemcpyAsync(so->R, d.out_s_R, sizeof(float) * n_seeds, hipMemcpyDeviceToHost, c->stream));
            if (so->flags) HIP_TRY(c, hipMemcpyAsync(so->flags, d.out_s_flags, sizeof(int32_t) * n_seeds, hipMemcpyDeviceToHost, c->stream));
            if (so->n_reval) HIP_TRY(c, hipMemcpyAsync(so->n_reval, d.out_s_nreval, sizeof(int32_t) * n_seeds, hipMemcpyDeviceToHost, c->stream));
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return RETINA_OK;
}

int retina_find_tracks(retina_ctx* c, const retina_geometry* g, const retina_hits* h,
                       const retina_params* P, retina_track* tracks, int64_t capacity,
                       int64_t* track_offsets, int32_t* event_flags, const retina_seed_out* so)
{
    return find_tracks_impl(c, g, h, P, tracks, capacity, track_offsets, event_flags, so,
                            h != nullptr && h->mem == RETINA_MEM_DEVICE);
}

int retina_set_graphs(retina_ctx* c, int32_t enable)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->use_graphs = enable != 0;
    return RETINA_OK;
}

int retina_autotune(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const retina_params* P,
                    const char* cache_path, int32_t* out_cand, int32_t* out_tile)
{
    if (!c) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_geometry(c, g)) || (rc = check_hits(c, g, h))) return rc;
    if (!P) return fail(c, RETINA_ERR_INVALID_ARG, "params is NULL");
    if (h->n_events < 1) return fail(c, RETINA_ERR_INVALID_ARG, "the sample needs at least one event");
    DeviceGuard guard(c->device);
    const int D = g->meas_dim;
    const int64_t E = h->n_events;
    int64_t n_hits, n_seeds;
    if ((rc = read_i64(c, h->mem, h->event_offsets, E, &n_hits))) return rc;
    if (P->seed_mode == RETINA_SEED_EXPLICIT) {
        if (!P->seed_offsets) return fail(c, RETINA_ERR_INVALID_ARG, "seed_offsets is NULL");
        if ((rc = read_i64(c, h->mem, P->seed_offsets, E, &n_seeds))) return rc;
    } else {
        n_seeds = E * (int64_t)P->lattice_n[0] * P->lattice_n[1];
    }
    const int kern = n_seeds < kSparseSeeds * E ? 2 : 0;  // the ascent slot this sample's seeding uses
    const int hit_class = (int)floor(log2(std::max<double>(1.0, (double)n_hits / (double)E)));
    const int seed_class = (int)floor(log2(std::max<double>(1.0, (double)n_seeds / (double)E)));
    char key[160];
    snprintf(key, sizeof(key), "%s meas_dim=%d hits=%d seeds=%d", c->arch, D, hit_class, seed_class);
    // cached choice?
    if (cache_path) {
        FILE* f = fopen(cache_path, "r");
        if (f) {
            char line[320];
            int best_c = 0, best_t = 0;
            while (fgets(line, sizeof(line), f)) {
                const size_t kl = strlen(key);
                int cc, tt;
                if (strncmp(line, key, kl) == 0 && line[kl] == ' ' &&
                    sscanf(line + kl, " cand=%d tile=%d", &cc, &tt) == 2) {
                    best_c = cc;
                    best_t = tt;
                }
            }
            fclose(f);
            if (best_c && retina_set_tuning(c, D, kern, best_c, best_t) == RETINA_OK) {
                if (out_cand) *out_cand = best_c;
                if (out_tile) *out_tile = best_t;
                return RETINA_OK;
            }
        }
    }
    // time every shape: outputs go nowhere (capacity 0: the pipeline still runs)
    int64_t* toff = nullptr;
    std::vector<int64_t> host_toff;
    if (h->mem == RETINA_MEM_DEVICE) {
        if ((rc = ensure_t(c, B_OUTTOFF, (size_t)E + 1, &toff))) return rc;
    } else {
        host_toff.resize(E + 1);
        toff = host_toff.data();
    }
    const HotConfig saved = tuning_slot(c, D, kern);
    const bool saved_prof = c->prof;
    const retina_profile saved_acc = c->prof_acc;
    if ((rc = retina_set_profiling(c, 1))) return rc;
    const int tiles[] = {2048, 4096, 5632, 6144, 8192, 12288};
    double best_ms = 1e300;
    int best_c = saved.cand, best_t = saved.tile_hits;
    for (int cand = 1; cand <= 2; ++cand) {
        for (int tile : tiles) {
            if ((size_t)tile * D * sizeof(float) + 4096 > c->lds_max) continue;
            if (retina_set_tuning(c, D, kern, cand, tile) != RETINA_OK) continue;
            double ms = 0.0;
            for (int rep = 0; rep < 2; ++rep) {  // first run warms up (graph capture, pool)
                c->prof_acc = retina_profile{};
                rc = retina_find_tracks(c, g, h, P, nullptr, 0, toff, nullptr, nullptr);
                if (rc != RETINA_OK && rc != RETINA_ERR_CAPACITY) {
                    tuning_slot(c, D, kern) = saved;
                    c->prof = saved_prof;
                    c->prof_acc = saved_acc;
                    return rc;
                }
                ms = c->prof_acc.ms_hot;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best_c = cand;
                best_t = tile;
            }
        }
    }
    c->prof = saved_prof;
    c->prof_acc = saved_acc;
    c->err.clear();
    if ((rc = retina_set_tuning(c, D, kern, best_c, best_t))) return rc;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s cand=%d tile=%d ms=%.3f\n", key, best_c, best_t, best_ms);
            fclose(f);
        }
    }
    if (out_cand) *out_cand = best_c;
    if (out_tile) *out_tile = best_t;
    return RETINA_OK;
}

}  // extern "C"

// ====================================================================== model
struct retina_model {
    retina_ctx* ctx = nullptr;
    NetLayout L;
    float* w32 = nullptr;     // FP32 master weights (padded layout)
    uint16_t* wbf = nullptr;  // BF16 copy used by the kernels
    float* m = nullptr;       // Adam moments
    float* v = nullptr;
    float* g = nullptr;       // gradient of the last step
    int64_t step = 0;
};

namespace {

constexpr int kPixPerChunk = 2048;  // pixels per weight-gradient partial (GEMM K of one work-group)
const char kModelMagic[8] = {'R', 'E', 'T', 'I', 'N', 'A', 'M', '1'};

int model_alloc(retina_ctx* c, retina_model* md)
{
    md->ctx = c;
    md->L = net_layout();
    const size_t n = (size_t)md->L.total;
    if (hipMalloc(&md->w32, n * 4) != hipSuccess || hipMalloc(&md->wbf, n * 2) != hipSuccess ||
        hipMalloc(&md->m, n * 4) != hipSuccess || hipMalloc(&md->v, n * 4) != hipSuccess ||
        hipMalloc(&md->g, n * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, RETINA_ERR_OUT_OF_MEMORY, "model allocation failed");
    }
    HIP_TRY(c, hipMemsetAsync(md->m, 0, n * 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(md->v, 0, n * 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(md->g, 0, n * 4, c->stream));
    return RETINA_OK;
}

// logical (W[co][tap][ci], b[co] per layer) <-> padded device layout
void logical_to_padded(const NetLayout& L, const float* in, std::vector<float>& out)
{
    out.assign((size_t)L.total, 0.0f);
    int64_t q = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int cin = kChan[l], cout = kChan[l + 1], K = conv_k(cin), Kp = conv_kp(cin);
        for (int co = 0; co < cout; ++co)
            for (int k = 0; k < K; ++k) out[L.w_off[l] + (int64_t)co * Kp + k] = in[q++];
        for (int co = 0; co < cout; ++co) out[L.b_off[l] + co] = in[q++];
    }
}

void padded_to_logical(const NetLayout& L, const float* in, float* out)
{
    int64_t q = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int cin = kChan[l], cout = kChan[l + 1], K = conv_k(cin), Kp = conv_kp(cin);
        for (int co = 0; co < cout; ++co)
            for (int k = 0; k < K; ++k) out[q++] = in[L.w_off[l] + (int64_t)co * Kp + k];
        for (int co = 0; co < cout; ++co) out[q++] = in[L.b_off[l] + co];
    }
}

uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}

// validate + stage hits (per-plane order, plane offsets) for the proposer;
// fills c->h_desc and leaves the staged arrays in the pool
int proposer_stage(retina_ctx* c, const retina_geometry* g, const retina_hits* h,
                   const retina_params* fallback = nullptr)
{
    int rc;
    if ((rc = check_geometry(c, g)) || (rc = check_hits(c, g, h))) return rc;
    if (g->meas_dim != 2) return fail(c, RETINA_ERR_INVALID_ARG, "the proposer needs meas_dim 2");
    const int64_t E = h->n_events;
    if (h->mem == RETINA_MEM_HOST && !host_offsets_ok(h->event_offsets, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "event_offsets must start at 0 and be non-decreasing");
    int64_t n_hits;
    if ((rc = read_i64(c, h->mem, h->event_offsets, E, &n_hits))) return rc;
    if (n_hits < 0 || n_hits > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "bad total hit count");
    Desc& d = *c->h_desc;
    reset_desc(d);
    fill_geometry(d, g);
    d.cnt = c->d_cnt;
    if ((rc = stage_inputs(c, d, g, h, n_hits))) return rc;
    if (fallback && (rc = set_lattice(c, d, fallback->lattice_n, fallback->lattice_lo, fallback->lattice_hi)))
        return rc;
    if ((rc = upload_desc(c))) return rc;
    launch_reset(c->d_desc, c->stream);
    launch_stage(c->d_desc, c->n_cu * 8, c->stream);
    HIP_TRY(c, hipGetLastError());
    if ((rc = download_counters(c))) return rc;
    if (c->h_cnt->err) return device_error(c, c->h_cnt->err);
    return RETINA_OK;
}

struct Acts {
    uint16_t* act[kLayers];  // act[0] = image, act[l] = output of layer l-1 (post-ReLU)
    float* u;                // inference: the head's band-edge terms
    float* logits;
};

int ensure_acts(retina_ctx* c, int64_t E, Acts& A, bool train)
{
    int rc;
    const size_t px = (size_t)E * kPix;
    A = Acts{};
    if ((rc = ensure_t(c, B_IMG, px * kChan[0], &A.act[0])) || (rc = ensure_t(c, B_ACT2, px * kChan[2], &A.act[2])) ||
        (rc = ensure_t(c, B_LOGIT, px, &A.logits)))
        return rc;
    if (train) {
        if ((rc = ensure_t(c, B_ACT1, px * kChan[1], &A.act[1])) || (rc = ensure_t(c, B_ACT3, px * kChan[3], &A.act[3])))
            return rc;
    } else if ((rc = ensure_t(c, B_HEADU, head_edge_floats(E), &A.u))) {
        return rc;
    }
    return RETINA_OK;
}

// image + 4 conv layers on the staged hits of c->h_desc
void forward_net(retina_ctx* c, const retina_model* md, int64_t E, const Acts& A, bool train)
{
    const Desc& d = *c->h_desc;
    launch_bin_image(d.hits, d.plane_off, d.n_planes, 2, c->d_desc->plane_z, E, A.act[0], &c->d_cnt->err, c->stream);
    launch_forward(A.act[0], md->wbf, md->w32, md->L, E, A.act[1], A.act[2], A.act[3], A.u, A.logits, train,
                   c->stream);
}

}  // namespace

extern "C" {

int retina_model_create(retina_ctx* c, uint64_t key, retina_model** out)
{
    if (!c || !out) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    *out = nullptr;
    DeviceGuard guard(c->device);
    retina_model* md = new retina_model();
    int rc = model_alloc(c, md);
    if (rc) { retina_model_free(md); return rc; }
    // He-normal weights from a counter-based generator keyed by `key`
    std::vector<float> logical(md->L.logical);
    uint64_t s = key;
    int64_t q = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int cin = kChan[l], cout = kChan[l + 1];
        const double sd = sqrt(2.0 / (9.0 * cin));
        for (int64_t i = 0; i < (int64_t)cout * conv_k(cin); ++i) {
            const double u1 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
            const double u2 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
            logical[q++] = (float)(sd * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
        }
        for (int co = 0; co < cout; ++co) logical[q++] = l == kLayers - 1 ? (float)log(0.01 / 0.99) : 0.0f;
    }
    if ((rc = retina_model_set_params(md, logical.data()))) { retina_model_free(md); return rc; }
    *out = md;
    return RETINA_OK;
}

void retina_model_free(retina_model* md)
{
    if (!md) return;
    DeviceGuard guard(md->ctx ? md->ctx->device : 0);
    if (md->ctx) (void)hipStreamSynchronize(md->ctx->stream);
    (void)hipFree(md->w32);
    (void)hipFree(md->wbf);
    (void)hipFree(md->m);
    (void)hipFree(md->v);
    (void)hipFree(md->g);
    (void)hipGetLastError();
    delete md;
}

int64_t retina_model_step(const retina_model* md) { return md ? md->step : -1; }

int retina_model_set_params(retina_model* md, const float* in)
{
    if (!md || !in) return RETINA_ERR_INVALID_ARG;
    retina_ctx* c = md->ctx;
    DeviceGuard guard(c->device);
    for (int64_t i = 0; i < md->L.logical; ++i)
        if (!isfinite(in[i])) return fail(c, RETINA_ERR_INVALID_ARG, "parameter %lld is not finite", (long long)i);
    std::vector<float> pad;
    logical_to_padded(md->L, in, pad);
    HIP_TRY(c, hipMemcpyAsync(md->w32, pad.data(), pad.size() * 4, hipMemcpyHostToDevice, c->stream));
    launch_to_bf16(md->w32, md->wbf, md->L.total, c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RETINA_OK;
}

int retina_model_get_params(const retina_model* md, float* out)
{
    if (!md || !out) return RETINA_ERR_INVALID_ARG;
    retina_ctx* c = md->ctx;
    DeviceGuard guard(c->device);
    std::vector<float> pad((size_t)md->L.total);
    HIP_TRY(c, hipMemcpyAsync(pad.data(), md->w32, pad.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    padded_to_logical(md->L, pad.data(), out);
    return RETINA_OK;
}

int retina_model_save(const retina_model* md, const char* path)
{
    if (!md || !path) return RETINA_ERR_INVALID_ARG;
    retina_ctx* c = md->ctx;
    DeviceGuard guard(c->device);
    const size_t n = (size_t)md->L.total;
    std::vector<float> buf(3 * n);
    HIP_TRY(c, hipMemcpyAsync(buf.data(), md->w32, n * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(buf.data() + n, md->m, n * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(buf.data() + 2 * n, md->v, n * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const uint64_t sum = fnv1a(buf.data(), buf.size() * 4);
    FILE* f = fopen(path, "wb");
    if (!f) return fail(c, RETINA_ERR_INVALID_ARG, "cannot open %s for writing", path);
    const uint32_t version = 1, layers = kLayers;
    const int64_t total = md->L.total, step = md->step;
    bool ok = fwrite(kModelMagic, 8, 1, f) == 1 && fwrite(&version, 4, 1, f) == 1 && fwrite(&layers, 4, 1, f) == 1 &&
              fwrite(&total, 8, 1, f) == 1 && fwrite(&step, 8, 1, f) == 1 && fwrite(&sum, 8, 1, f) == 1 &&
              fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(c, RETINA_ERR_INVALID_ARG, "writing %s failed", path);
    return RETINA_OK;
}

int retina_model_load(retina_ctx* c, const char* path, retina_model** out)
{
    if (!c || !path || !out) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    *out = nullptr;
    DeviceGuard guard(c->device);
    FILE* f = fopen(path, "rb");
    if (!f) return fail(c, RETINA_ERR_INVALID_ARG, "cannot open %s", path);
    char magic[8];
    uint32_t version = 0, layers = 0;
    int64_t total = 0, step = 0;
    uint64_t sum = 0;
    bool ok = fread(magic, 8, 1, f) == 1 && fread(&version, 4, 1, f) == 1 && fread(&layers, 4, 1, f) == 1 &&
              fread(&total, 8, 1, f) == 1 && fread(&step, 8, 1, f) == 1 && fread(&sum, 8, 1, f) == 1;
    const NetLayout L = net_layout();
    if (!ok || memcmp(magic, kModelMagic, 8) != 0 || version != 1 || layers != (uint32_t)kLayers || total != L.total) {
        fclose(f);
        return fail(c, RETINA_ERR_INVALID_ARG, "%s is not a libretina model file of this layout", path);
    }
    std::vector<float> buf(3 * (size_t)total);
    ok = fread(buf.data(), 4, buf.size(), f) == buf.size();
    fclose(f);
    if (!ok || fnv1a(buf.data(), buf.size() * 4) != sum)
        return fail(c, RETINA_ERR_INVALID_ARG, "%s is truncated or corrupted (checksum)", path);
    retina_model* md = new retina_model();
    int rc = model_alloc(c, md);
    if (rc) { retina_model_free(md); return rc; }
    const size_t n = (size_t)total;
    HIP_TRY(c, hipMemcpyAsync(md->w32, buf.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(md->m, buf.data() + n, n * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(md->v, buf.data() + 2 * n, n * 4, hipMemcpyHostToDevice, c->stream));
    launch_to_bf16(md->w32, md->wbf, md->L.total, c->stream);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    md->step = step;
    *out = md;
    return RETINA_OK;
}

int retina_model_forward(retina_ctx* c, const retina_model* md, const retina_geometry* g, const retina_hits* h,
                         uint16_t* image, float* logits)
{
    if (!c || !md) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    DeviceGuard guard(c->device);
    int rc;
    if ((rc = proposer_stage(c, g, h))) return rc;
    const int64_t E = h->n_events;
    if (E == 0) return RETINA_OK;
    Acts A;
    if ((rc = ensure_acts(c, E, A, false))) return rc;
    forward_net(c, md, E, A, false);
    HIP_TRY(c, hipGetLastError());
    const size_t px = (size_t)E * kPix;
    const hipMemcpyKind k = h->mem == RETINA_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (image) HIP_TRY(c, hipMemcpyAsync(image, A.act[0], px * 2 * 2, k, c->stream));
    if (logits) HIP_TRY(c, hipMemcpyAsync(logits, A.logits, px * 4, k, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RETINA_OK;
}

int retina_train_step(retina_ctx* c, retina_model* md, const retina_geometry* g, const retina_hits* h,
                      const double* targets, const int64_t* toff, float lr, float pos_weight, float* loss,
                      float* grad_out)
{
    if (!c || !md) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    if (!toff) return fail(c, RETINA_ERR_INVALID_ARG, "target_offsets is NULL");
    if (!(lr >= 0.0f) || !isfinite(lr) || !(pos_weight > 0.0f) || !isfinite(pos_weight))
        return fail(c, RETINA_ERR_INVALID_ARG, "lr must be >= 0 and pos_weight > 0");
    DeviceGuard guard(c->device);
    int rc;
    if ((rc = proposer_stage(c, g, h))) return rc;
    const int64_t E = h->n_events;
    if (E == 0) return fail(c, RETINA_ERR_INVALID_ARG, "empty batch");
    int64_t n_tg;
    const bool host = h->mem == RETINA_MEM_HOST;
    if (host && !host_offsets_ok(toff, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "target_offsets must start at 0 and be non-decreasing");
    if ((rc = read_i64(c, h->mem, toff, E, &n_tg))) return rc;
    if (n_tg > 0 && !targets) return fail(c, RETINA_ERR_INVALID_ARG, "targets is NULL");
    const double* tg = targets;
    const int64_t* to = toff;
    if (host) {
        double* dt;
        int64_t* dto;
        if ((rc = ensure_t(c, B_TGTIN, (size_t)std::max<int64_t>(n_tg, 1) * 2, &dt)) ||
            (rc = ensure_t(c, B_TGTOFF, (size_t)E + 1, &dto)))
            return rc;
        if (n_tg) HIP_TRY(c, hipMemcpyAsync(dt, targets, sizeof(double) * 2 * n_tg, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(dto, toff, sizeof(int64_t) * (E + 1), hipMemcpyHostToDevice, c->stream));
        tg = dt;
        to = dto;
    }
    Acts A;
    uint16_t* dz[kLayers];
    uint8_t* tgt;
    float *part, *lpart, *lsum, *bpart;
    uint16_t* wt;
    const size_t px = (size_t)E * kPix;
    const int n_chunks = (int)(px / kPixPerChunk);
    int64_t max_part = 0, max_wt = 0;
    for (int l = 0; l < kLayers; ++l) {
        max_part = std::max<int64_t>(max_part, (int64_t)kChan[l + 1] * conv_kp(kChan[l]));
        max_wt = std::max<int64_t>(max_wt, (int64_t)kChan[l] * conv_kp(kChan[l + 1]));
    }
    if ((rc = ensure_acts(c, E, A, true)) || (rc = ensure_t(c, B_DZ4, px * kChan[4], &dz[3])) ||
        (rc = ensure_t(c, B_DZ3, px * kChan[3], &dz[2])) || (rc = ensure_t(c, B_DZ2, px * kChan[2], &dz[1])) ||
        (rc = ensure_t(c, B_DZ1, px * kChan[1], &dz[0])) || (rc = ensure_t(c, B_TGT, px, &tgt)) ||
        (rc = ensure_t(c, B_DWPART, (size_t)n_chunks * max_part, &part)) || (rc = ensure_t(c, B_WT, (size_t)max_wt, &wt)) ||
        (rc = ensure_t(c, B_LOSSPART, 1024, &lpart)) || (rc = ensure_t(c, B_LOSS, 1, &lsum)) ||
        (rc = ensure_t(c, B_BPART, (size_t)n_chunks * 128, &bpart)))
        return rc;
    // forward
    forward_net(c, md, E, A, true);
    launch_target_image(tg, to, E, tgt, c->stream);
    launch_bce(A.logits, tgt, (int64_t)px, pos_weight, lpart, dz[3], c->stream);
    launch_sum(lpart, 1024, lsum, c->stream);
    // backward, last layer first; dz[l] = gradient wrt layer l's pre-activation
    for (int l = kLayers - 1; l >= 0; --l) {
        const int cin = kChan[l], cout = kChan[l + 1];
        GemmArgs a = {};
        a.mode = kBwdW;
        a.B = (int)E;
        a.cin = cin;
        a.cout = cout;
        a.x = A.act[l];
        a.dz = dz[l];
        a.partial = part;
        a.pix_per_chunk = kPixPerChunk;
        launch_gemm(a, c->stream);
        launch_reduce_dw(part, n_chunks, (int64_t)cout * conv_kp(cin), md->g + md->L.w_off[l], c->stream);
        launch_bias_grad(dz[l], (int64_t)px, cout, n_chunks, bpart, md->g + md->L.b_off[l], c->stream);
        if (l > 0) {
            launch_transpose_w(md->wbf + md->L.w_off[l], cin, cout, wt, c->stream);
            GemmArgs b = {};
            b.mode = kBwdData;
            b.B = (int)E;
            b.cin = cin;
            b.cout = cout;
            b.w = wt;
            b.dz = dz[l];
            b.xprev = A.act[l];
            b.y_bf16 = dz[l - 1];
            launch_gemm(b, c->stream);
        }
    }
    if (lr > 0.0f) {
        md->step += 1;
        launch_adam(md->w32, md->m, md->v, md->g, md->wbf, md->L.total, lr, 0.9f, 0.999f, 1e-8f, md->step, c->stream);
    }
    HIP_TRY(c, hipGetLastError());
    float l_host = 0.0f;
    HIP_TRY(c, hipMemcpyAsync(&l_host, lsum, 4, hipMemcpyDeviceToHost, c->stream));
    std::vector<float> gpad;
    if (grad_out) {
        gpad.resize((size_t)md->L.total);
        HIP_TRY(c, hipMemcpyAsync(gpad.data(), md->g, gpad.size() * 4, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (grad_out) padded_to_logical(md->L, gpad.data(), grad_out);
    if (loss) *loss = l_host;
    return RETINA_OK;
}

}  // extern "C"

namespace {

// proposer seeds into the pool (device): returns the total through *n_seeds
int propose_device(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const retina_model* md,
                   const retina_proposal* pr, const retina_params* P, ProposeArgs& pa, int64_t* n_seeds)
{
    int rc;
    if (!P || !pr) return fail(c, RETINA_ERR_INVALID_ARG, "params or proposal is NULL");
    const int32_t k_max = pr->k_max;
    const float tau = pr->tau, conf_min = pr->conf_min;
    if (k_max < 1 || k_max > 4096) return fail(c, RETINA_ERR_INVALID_ARG, "k_max must be in [1, 4096]");
    if (!(tau > 0.0f && tau < 1.0f) || !(conf_min >= 0.0f && conf_min <= 1.0f))
        return fail(c, RETINA_ERR_INVALID_ARG, "tau must be in (0, 1) and conf_min in [0, 1]");
    if (pr->nms != 0 && pr->nms != 1) return fail(c, RETINA_ERR_INVALID_ARG, "nms must be 0 or 1");
    if (P->lattice_n[0] < 1 || P->lattice_n[1] < 1 || P->lattice_n[0] > kMaxLatticeSide ||
        P->lattice_n[1] > kMaxLatticeSide || (int64_t)P->lattice_n[0] * P->lattice_n[1] > (1 << 24))
        return fail(c, RETINA_ERR_INVALID_ARG, "fallback lattice_n must be in [1, %d] with at most 2^24 seeds",
                    kMaxLatticeSide);
    if ((rc = proposer_stage(c, g, h, P))) return rc;
    const int64_t E = h->n_events;
    Acts A;
    if ((rc = ensure_acts(c, E, A, false))) return rc;
    prof_mark(c, 5);
    forward_net(c, md, E, A, false);
    const int64_t lat = (int64_t)P->lattice_n[0] * P->lattice_n[1];
    const int64_t cap = E * std::max<int64_t>(k_max, lat);
    pa = ProposeArgs{};
    pa.logits = A.logits;
    pa.n_events = E;
    pa.k_max = k_max;
    // thresholds as logits, computed in FP64 and rounded once to FP32
    pa.ltau = (float)log((double)tau / (1.0 - (double)tau));
    pa.lconf = conf_min <= 0.0f ? -INFINITY
             : conf_min >= 1.0f ? INFINITY : (float)log((double)conf_min / (1.0 - (double)conf_min));
    pa.nms = pr->nms;
    for (int i = 0; i < 2; ++i) pa.lattice_n[i] = P->lattice_n[i];
    pa.lat_coord = c->d_desc->lat_coord;  // device address: proposer_stage uploaded the table
    {
        const double w = ((double)kSlopeHi - (double)kSlopeLo) / kImg;
        for (int i = 0; i < kImg; ++i) pa.bin_centre[i] = (float)((double)kSlopeLo + ((double)i + 0.5) * w);
    }
    if ((rc = ensure_t(c, B_PSCORE, (size_t)E * k_max, &pa.cand_score)) ||
        (rc = ensure_t(c, B_PPIX, (size_t)E * k_max, &pa.cand_pix)) || (rc = ensure_t(c, B_PCOUNT, (size_t)E, &pa.count)) ||
        (rc = ensure_t(c, B_PCONF, (size_t)E, &pa.confidence)) || (rc = ensure_t(c, B_PFB, (size_t)E, &pa.fallback)) ||
        (rc = ensure_t(c, B_PSOFF, (size_t)E + 1, &pa.seed_off)))
        return rc;
    launch_propose_select(pa, c->stream);
    launch_propose_offsets(pa, c->stream);
    prof_mark(c, 6);
    HIP_TRY(c, hipGetLastError());
    if ((rc = read_i64(c, RETINA_MEM_DEVICE, pa.seed_off, E, n_seeds))) return rc;
    if (c->prof) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, c->ev[5], c->ev[6]) != hipSuccess) t = 0.0f;
        (void)hipGetLastError();
        c->prof_acc.ms_propose += t;
    }
    if (*n_seeds > cap) return fail(c, RETINA_ERR_INTERNAL, "seed count exceeds its bound");
    if ((rc = ensure_t(c, B_PSEEDS, (size_t)std::max<int64_t>(*n_seeds, 1) * 4, &pa.seeds))) return rc;
    launch_propose_write(pa, c->stream);
    HIP_TRY(c, hipGetLastError());
    return RETINA_OK;
}

// Algorithm 1 from the proposer's seeds in one device pass: staging, binning,
// network, seed selection (lattice fallback), work plan, ascent, merge and
// output, sized by the proposal bound E x max(k_max, lattice) so that no count
// returns to the host between the proposer and the ascent.  The sequence is
// replayed from one captured graph while its launch arguments stay the same.
// The launch shape follows the bound: the sparse-seeding ascent when k_max is
// below kSparseSeeds, the small-cache merge when k_max <= kMergeSmallKeys.
int learned_impl(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const retina_params* P,
                 const retina_model* md, const retina_proposal* pr, retina_track* tracks, int64_t capacity,
                 int64_t* track_offsets, int32_t* event_flags)
{
    int rc;
    if ((rc = check_geometry(c, g)) || (rc = check_hits(c, g, h))) return rc;
    if (g->meas_dim != 2) return fail(c, RETINA_ERR_INVALID_ARG, "the proposer needs meas_dim 2");
    if (!P || !pr) return fail(c, RETINA_ERR_INVALID_ARG, "params or proposal is NULL");
    {
        retina_params L = *P;
        L.seed_mode = RETINA_SEED_LATTICE;  // params carry the fallback lattice
        rtv::Check k;
        if (rtv::method_params(k, &L, capacity, tracks, track_offsets)) return fail(c, k.code, "%s", k.msg);
    }
    const int32_t k_max = pr->k_max;
    if (k_max < 1 || k_max > 4096) return fail(c, RETINA_ERR_INVALID_ARG, "k_max must be in [1, 4096]");
    if (!(pr->tau > 0.0f && pr->tau < 1.0f) || !(pr->conf_min >= 0.0f && pr->conf_min <= 1.0f))
        return fail(c, RETINA_ERR_INVALID_ARG, "tau must be in (0, 1) and conf_min in [0, 1]");
    if (pr->nms != 0 && pr->nms != 1) return fail(c, RETINA_ERR_INVALID_ARG, "nms must be 0 or 1");
    const int D = 2;
    const int64_t E = h->n_events;
    const bool host = h->mem == RETINA_MEM_HOST;
    if (host && !host_offsets_ok(h->event_offsets, E))
        return fail(c, RETINA_ERR_INVALID_ARG, "event_offsets must start at 0 and be non-decreasing");
    int64_t n_hits;
    if ((rc = read_i64(c, h->mem, h->event_offsets, E, &n_hits))) return rc;
    if (n_hits < 0 || n_hits > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "bad total hit count");
    const int64_t lat = (int64_t)P->lattice_n[0] * P->lattice_n[1];
    const int64_t cap = E * std::max<int64_t>(k_max, lat);  // seeds of the batch, at most
    if (cap > 0x7FFFFFFF) return fail(c, RETINA_ERR_INVALID_ARG, "too many seeds in the batch (proposal bound)");

    Desc& d = *c->h_desc;
    reset_desc(d);
    fill_geometry(d, g);
    d.cnt = c->d_cnt;
    if ((rc = stage_inputs(c, d, g, h, n_hits))) return rc;
    if ((rc = set_lattice(c, d, P->lattice_n, P->lattice_lo, P->lattice_hi))) return rc;
    // proposer
    Acts A;
    if ((rc = ensure_acts(c, E, A, false))) return rc;
    ProposeArgs pa = ProposeArgs{};
    pa.logits = A.logits;
    pa.n_events = E;
    pa.k_max = k_max;
    pa.ltau = (float)log((double)pr->tau / (1.0 - (double)pr->tau));
    pa.lconf = pr->conf_min <= 0.0f ? -INFINITY
             : pr->conf_min >= 1.0f ? INFINITY : (float)log((double)pr->conf_min / (1.0 - (double)pr->conf_min));
    pa.nms = pr->nms;
    for (int i = 0; i < 2; ++i) pa.lattice_n[i] = P->lattice_n[i];
    pa.lat_coord = c->d_desc->lat_coord;
    {
        const double w = ((double)kSlopeHi - (double)kSlopeLo) / kImg;
        for (int i = 0; i < kImg; ++i) pa.bin_centre[i] = (float)((double)kSlopeLo + ((double)i + 0.5) * w);
    }
    if ((rc = ensure_t(c, B_PSCORE, (size_t)E * k_max, &pa.cand_score)) ||
        (rc = ensure_t(c, B_PPIX, (size_t)E * k_max, &pa.cand_pix)) || (rc = ensure_t(c, B_PCOUNT, (size_t)E, &pa.count)) ||
        (rc = ensure_t(c, B_PCONF, (size_t)E, &pa.confidence)) || (rc = ensure_t(c, B_PFB, (size_t)E, &pa.fallback)) ||
        (rc = ensure_t(c, B_PSOFF, (size_t)E + 1, &pa.seed_off)) ||
        (rc = ensure_t(c, B_PSEEDS, (size_t)std::max<int64_t>(cap, 1) * 4, &pa.seeds)))
        return rc;
    // ascent and merge, sized by the bound
    HotConfig hc = k_max < kSparseSeeds ? c->sparse_cfg[D] : c->ascent_cfg[D];
    hc.prune = P->prune_u > 0.0f;
    hc.staged = 1;  // the sequence stages the hits before the proposer
    if (P->update != RETINA_UPDATE_NEWTON) {
        hc = c->sparse_cfg[D];
        hc.cand = 1;
        hc.update = P->update;
        hc.prune = 0;
        hc.staged = 1;
    }
    if (kSplitSeeds && hc.cand == 1 && hc.update == RETINA_UPDATE_NEWTON) {
        hc.split = 1;
        hc.grid = c->n_cu * hot_max_blocks_per_cu(D, hc, true);
    }
    hc.small_merge = k_max <= kMergeSmallKeys;
    d.seeds_per_item = hot_seeds_per_item(hc);
    d.half_parts = hc.split;
    d.items_cap = cap / d.seeds_per_item + 2 * E + 1;
    if ((rc = ensure_t(c, B_ITEMS, (size_t)d.items_cap, &d.items))) return rc;
    d.seed_mode = RETINA_SEED_EXPLICIT;
    d.in_seeds = pa.seeds;
    d.in_seed_off = pa.seed_off;
    d.n_sigma = P->n_sigma;
    for (int i = 0; i < P->n_sigma; ++i) d.sigma[i] = P->sigma[i];
    d.sigma_final = P->sigma_final;
    d.n_final_steps = P->n_final_steps;
    d.n_polish = P->n_polish;
    d.ls_trials = P->ls_trials;
    d.n_slope_steps = P->n_slope_steps;
    d.armijo_c1 = P->armijo_c1;
    d.step_cap = P->step_cap_sigmas;
    d.small_step = P->small_step_sigmas;
    d.conv_tol = P->conv_tol;
    d.R0 = P->R0;
    d.d_merge = P->d_merge;
    d.prune_u = hc.prune ? P->prune_u : 0.0f;
    if (hc.prune && (rc = ensure_t(c, B_EVSORT, (size_t)E, &d.ev_sorted))) return rc;
    const size_t ns1 = (size_t)std::max<int64_t>(cap, 1);
    if ((rc = ensure_t(c, B_STH, ns1 * 4, &d.s_theta)) || (rc = ensure_t(c, B_SR, ns1, &d.s_R)) ||
        (rc = ensure_t(c, B_SFL, ns1, &d.s_flags)) || (rc = ensure_t(c, B_SNR, ns1, &d.s_nreval)) ||
        (rc = ensure_t(c, B_MLEAD, ns1, &d.m_leader)) || (rc = ensure_t(c, B_MMEM, ns1, &d.m_members)) ||
        (rc = ensure_t(c, B_MKEYS, ns1 * 2, &d.m_keys)) || (rc = ensure_t(c, B_EVNT, (size_t)E, &d.ev_ntracks)) ||
        (rc = ensure_t(c, B_EVFL, (size_t)E, &d.ev_flags)) || (rc = ensure_t(c, B_EVTOFF, (size_t)E + 1, &d.ev_toff)))
        return rc;
    if (host) {
        const int64_t host_cap = std::min<int64_t>(capacity, cap);
        if ((rc = ensure_t(c, B_OUTTR, (size_t)std::max<int64_t>(host_cap, 1), &d.out_tracks)) ||
            (rc = ensure_t(c, B_OUTTOFF, (size_t)E + 1, &d.out_track_off)))
            return rc;
        d.out_capacity = host_cap;
        if (event_flags && (rc = ensure_t(c, B_OUTEVF, (size_t)E, &d.out_ev_flags))) return rc;
    } else {
        d.out_tracks = tracks;
        d.out_capacity = capacity;
        d.out_track_off = track_offsets;
        d.out_ev_flags = event_flags;
    }
    if ((rc = upload_desc(c))) return rc;
    prepare_forward();  // kernel attributes are set outside any capture

    const retina_model* mdl = md;
    auto sequence = [&](hipStream_t st) {
        auto mark = [&](int i) {
            if (c->prof) (void)hipEventRecord(c->ev[i], st);
        };
        mark(5);
        launch_reset(c->d_desc, st);
        launch_stage(c->d_desc, c->n_cu * 8, st);
        launch_bin_image(d.hits, d.plane_off, d.n_planes, 2, c->d_desc->plane_z, E, A.act[0], &c->d_cnt->err, st);
        launch_forward(A.act[0], mdl->wbf, mdl->w32, mdl->L, E, A.act[1], A.act[2], A.act[3], A.u, A.logits, false, st);
        launch_propose_select(pa, st);
        launch_propose_offsets(pa, st);
        launch_propose_write(pa, st);
        mark(6);
        mark(0);
        if (hc.prune) launch_sort_planes(c->d_desc, c->n_cu * 8, st);
        mark(1);
        launch_plan_tracks(c->d_desc, st);
        mark(2);
        launch_ascent(c->d_desc, D, hc, st);
        mark(3);
        launch_merge(c->d_desc, D, c->n_cu, hc.small_merge != 0, st);
        launch_finalize(c->d_desc, st);
        launch_emit(c->d_desc, D, c->n_cu * 4, st);
        launch_flag_fallback_desc(c->d_desc, pa.fallback, E, st);
        mark(4);
    };
    // every by-value launch argument of the sequence (pool and model addresses,
    // sizes, thresholds, launch shape) keys the captured graph
    struct Key {
        int64_t E;
        ProposeArgs pa;
        Acts A;
        const void* wbf;
        const void* w32;
        const void* hits;
        const void* plane_off;
        HotConfig hc;
        int n_planes, n_cu;
    } key;
    memset(&key, 0, sizeof(key));
    key.E = E;
    key.pa = pa;
    key.A = A;
    key.wbf = md->wbf;
    key.w32 = md->w32;
    key.hits = d.hits;
    key.plane_off = d.plane_off;
    key.hc = hc;
    key.n_planes = d.n_planes;
    key.n_cu = c->n_cu;
    bool launched = false;
    if (c->use_graphs && !c->prof) {
        const unsigned char* kb = reinterpret_cast<const unsigned char*>(&key);
        if (!c->learned_exec || c->learned_key.size() != sizeof(key) ||
            memcmp(c->learned_key.data(), kb, sizeof(key)) != 0) {
            if (c->learned_exec) (void)hipGraphExecDestroy(c->learned_exec);
            c->learned_exec = nullptr;
            c->learned_key.clear();
            hipGraph_t graph = nullptr;
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            bool ok = hipStreamBeginCapture(c->own, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                sequence(c->own);
                ok = hipStreamEndCapture(c->own, &graph) == hipSuccess && graph;
            }
            hipGraphExec_t exec = nullptr;
            if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            if (ok) {
                c->learned_exec = exec;
                c->learned_key.assign(kb, kb + sizeof(key));
            } else {
                (void)hipGetLastError();
                c->use_graphs = false;  // capture unsupported here: launch eagerly from now on
            }
        }
        if (c->learned_exec) {
            HIP_TRY(c, hipGraphLaunch(c->learned_exec, c->stream));
            launched = true;
        }
    }
    if (!launched) sequence(c->stream);
    HIP_TRY(c, hipGetLastError());
    if ((rc = download_counters(c))) return rc;
    if (c->prof) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, c->ev[5], c->ev[6]) != hipSuccess) t = 0.0f;
        (void)hipGetLastError();
        c->prof_acc.ms_propose += t;
    }
    prof_collect(c);
    const uint32_t err = c->h_cnt->err;
    const int64_t total = c->h_cnt->total_tracks;
    if (err & ~kErrCapacity) return device_error(c, err);
    if (err & kErrCapacity || total > capacity) {
        if (host) track_offsets[E] = total;
        return fail(c, RETINA_ERR_CAPACITY, "%lld tracks found, capacity %lld", (long long)total,
                    (long long)capacity);
    }
    if (host) {
        if (total)
            HIP_TRY(c, hipMemcpyAsync(tracks, d.out_tracks, sizeof(retina_track) * total, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(track_offsets, d.out_track_off, sizeof(int64_t) * (E + 1), hipMemcpyDeviceToHost, c->stream));
        if (event_flags)
            HIP_TRY(c, hipMemcpyAsync(event_flags, d.out_ev_flags, sizeof(int32_t) * E, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return RETINA_OK;
}

}  // namespace

extern "C" {

int retina_propose_seeds(retina_ctx* c, const retina_geometry* g, const retina_hits* h, const retina_model* md,
                         const retina_proposal* pr, const retina_params* P, double* seeds,
                         int64_t capacity, int64_t* seed_offsets, float* confidence, int32_t* fallback)
{
    if (!c || !md) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    if (!seed_offsets || capacity < 0 || (capacity > 0 && !seeds))
        return fail(c, RETINA_ERR_INVALID_ARG, "seeds / seed_offsets / capacity invalid");
    DeviceGuard guard(c->device);
    int rc;
    if (h && h->n_events == 0) {
        if (h->mem == RETINA_MEM_HOST) seed_offsets[0] = 0;
        else HIP_TRY(c, hipMemsetAsync(seed_offsets, 0, 8, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return RETINA_OK;
    }
    ProposeArgs pa;
    int64_t n;
    if ((rc = propose_device(c, g, h, md, pr, P, pa, &n))) return rc;
    const int64_t E = h->n_events;
    const hipMemcpyKind k = h->mem == RETINA_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (n > capacity) {
        HIP_TRY(c, hipMemcpyAsync(seed_offsets + E, pa.seed_off + E, 8, k, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return fail(c, RETINA_ERR_CAPACITY, "%lld seeds, capacity %lld", (long long)n, (long long)capacity);
    }
    if (n) HIP_TRY(c, hipMemcpyAsync(seeds, pa.seeds, sizeof(double) * 4 * n, k, c->stream));
    HIP_TRY(c, hipMemcpyAsync(seed_offsets, pa.seed_off, 8 * (E + 1), k, c->stream));
    if (confidence) HIP_TRY(c, hipMemcpyAsync(confidence, pa.confidence, 4 * E, k, c->stream));
    if (fallback) HIP_TRY(c, hipMemcpyAsync(fallback, pa.fallback, 4 * E, k, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return RETINA_OK;
}

int retina_find_tracks_learned(retina_ctx* c, const retina_geometry* g, const retina_hits* h,
                               const retina_params* P, const retina_model* md, const retina_proposal* pr,
                               retina_track* tracks, int64_t capacity, int64_t* track_offsets,
                               int32_t* event_flags)
{
    if (!c || !md) return RETINA_ERR_INVALID_ARG;
    c->err.clear();
    DeviceGuard guard(c->device);
    if (h && h->n_events == 0)
        return retina_find_tracks(c, g, h, P, tracks, capacity, track_offsets, event_flags, nullptr);
    return learned_impl(c, g, h, P, md, pr, tracks, capacity, track_offsets, event_flags);
}

}  // extern "C"
