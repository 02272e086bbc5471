// C-ABI of libens: argument validation, the trace store, the search schedule
// (plain per-sample evolution or ENS sweeps) and the objective entry points.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ens.h"
#include "device.h"
#include "launch.h"

namespace {

using ens::PAD;
using ens::TraceMeta;

// Grow-only device buffer owned by a context.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            bytes = 0;
            if (e != hipSuccess) return e;
        }
        if (n == 0) return hipSuccess;
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

}  // namespace

struct ens_ctx {
    hipStream_t stream = nullptr;
    std::string err;
    ens_tuning tuning{};
    // bound data (#data, #config)
    bool bound = false;
    int64_t n_tr = 0, ld = 0;
    int32_t nt = 0, n_cmp = 0, store_dtype = ENS_DTYPE_F32;
    float dt = 0.f, dx = 0.f;
    int32_t op = 0, window = 0, ap_lo = 0, ap_hi = 0;
    int32_t max_ap_traces = 0;   // the most traces any output CMP's widest aperture holds
    DevBuf store, master, scale, meta, cmp_ptr, ap_tab, qexp, wsc16;
    // binary16 window constants (StoreView h16_*)
    float h16_kq = 0.f;
    uint32_t h16_bbits = 0, h16_shift = 0;
    // search workspace
    DevBuf lo_tab, hi_tab, items, X, XS, Y, YS, counters, cmp_out, flag, progress, np_tab;
    // statistics of the last search, launch timing events
    ens_stats stats{};
    std::vector<hipEvent_t> events;
    // captured trace-step sequence of the last ENS search (replayed when the
    // next search issues exactly the same launches)
    struct Launch {
        ens::SearchArgs a;
        ens::InterpArgs ia;
        int32_t kind, n_blocks, dense;
        int32_t item_class;   // 0 first sweep, 1 backward sweeps, 2 later forward sweeps
        int32_t interp;       // 1: interpolation of the skipped samples (ia), not a search launch
    };
    std::vector<Launch> graph_seq;
    // measured launch shapes: key -> (slices, item order)
    struct Shape {
        int nsl, order, dense;
        int packed;           // waves of a packed workgroup, 0 when not packed, -1 not measured
    };
    std::map<std::string, Shape> tune_cache;
    std::string device_tag;   // "<arch>/<CUs>": prefix of the keys in the shape file
    void *scratch = nullptr;  // this device's copy of `scratch` (ens_stack_noalloc)
    hipError_t scratch_err = hipSuccess;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        graph_seq.clear();
    }
    ~ens_ctx()
    {
        drop_graph();
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (DevBuf *b : {&store, &master, &scale, &meta, &cmp_ptr, &ap_tab, &qexp, &wsc16, &lo_tab, &hi_tab, &items,
                          &X, &XS, &Y, &YS, &counters, &cmp_out, &flag, &progress, &np_tab})
            b->release();
    }
};

namespace {

ens_status fail(ens_ctx *ctx, ens_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
ens_status fail(ens_ctx *ctx, ens_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

#define HIP_OR_FAIL(ctx, expr)                                                                    \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, e_ == hipErrorOutOfMemory ? ENS_E_OOM : ENS_E_HIP, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                                   \
    } while (0)

// ---- memory for the entry point that allocates nothing (ens_stack_noalloc)

// the output-CMP list and the coherence RMS of ens_stack_noalloc
constexpr int32_t NOALLOC_MAX_CMPS = ENS_NOALLOC_MAX_CMPS;
constexpr size_t NOALLOC_RMS_BYTES = 256;   // the binary64 RMS, padded to the array's alignment
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_RMS_BYTES + sizeof(int32_t) * NOALLOC_MAX_CMPS;

}  // namespace

// One copy per device, held until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void *scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current); nullptr with the HIP error in *err.
void *scratch_address(hipError_t *err)
{
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        scratch_ptr[dev] = p;
    }
    return scratch_ptr[dev];
}

// generations per launch-shape trial (the search itself runs all of them)
constexpr int32_t TUNE_GENERATIONS = 8;

int32_t lerp_round(int32_t lo, int32_t hi, int32_t n0, int32_t nt)
{
    if (nt <= 1) return lo;
    const double v = lo + static_cast<double>(hi - lo) * static_cast<double>(n0) / static_cast<double>(nt - 1);
    return static_cast<int32_t>(std::floor(v + 0.5));
}

// Per-sample box: bounds whose mask bit is set are divided by max(n0 dt, dt)
// in binary32.
void sample_box(const ens_bounds &b, int32_t n0, float dt, float lo[3], float hi[3])
{
    const float t0 = static_cast<float>(n0) * dt;
    const float den = t0 > dt ? t0 : dt;
    for (int d = 0; d < 3; ++d) {
        lo[d] = b.lo[d];
        hi[d] = b.hi[d];
        if (b.inv_t0_mask >> d & 1u) {
            lo[d] = lo[d] / den;
            hi[d] = hi[d] / den;
        }
    }
}

ens::StoreView view_of(const ens_ctx *c, bool master)
{
    ens::StoreView v{};
    const bool use_master = master && c->store_dtype != ENS_DTYPE_F32;
    v.store = use_master ? c->master.p : c->store.p;
    const bool half = c->store_dtype != ENS_DTYPE_F32 && !use_master;
    v.ld = half ? 2 * c->ld : c->ld;
    v.copy1 = half ? static_cast<int32_t>(c->ld) : 0;
    v.scale = (c->store_dtype == ENS_DTYPE_F32 || use_master) ? nullptr : c->scale.as<float>();
    v.meta = c->meta.as<TraceMeta>();
    v.cmp_ptr = c->cmp_ptr.as<int64_t>();
    v.n_cmp = c->n_cmp;
    v.nt = c->nt;
    v.dt = c->dt;
    v.dx = c->dx;
    v.ap_tab = c->ap_tab.as<int32_t>();
    v.wsc16 = half ? c->wsc16.as<uint32_t>() : nullptr;
    v.h16_kq = c->h16_kq;
    v.h16_bbits = c->h16_bbits;
    v.h16_shift = c->h16_shift;
    v.tau_max = static_cast<float>(c->nt - 1);
    return v;
}

bool is_pow2(float x)
{
    if (!(x > 0.f) || !std::isfinite(x)) return false;
    int e = 0;
    return std::frexp(x, &e) == 0.5f;
}

bool finite(float x) { return std::isfinite(x); }

// Device-side range check of candidate indices (they live in device memory).
ens_status check_candidates(ens_ctx *ctx, const ens_candidates *cands);

// out[i] = i for i < n (the identity output-CMP list)
hipError_t launch_iota(int32_t *out, int32_t n, hipStream_t s);

// Measured launch shapes persist in a text file shared by the processes that
// load the library: one line "<device>/<key> <slices> <item order> <dense>
// <packed waves>" per shape.  The file is ENS_TUNE_CACHE if that is set
// ("off": none), else ens_tune_cache.txt beside the library.  Lines are appended as shapes are
// measured; a later line for the same key wins.  Unreadable or unwritable
// files are ignored: the shapes are then measured again.
std::mutex tune_file_mutex;

std::string tune_file_path()
{
    const char *env = std::getenv("ENS_TUNE_CACHE");
    if (env) return std::string(env) == "off" ? std::string() : std::string(env);
    Dl_info info{};
    if (!dladdr(reinterpret_cast<void *>(&ens_version), &info) || !info.dli_fname) return std::string();
    std::string lib(info.dli_fname);
    const size_t slash = lib.rfind('/');
    return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/ens_tune_cache.txt";
}

void load_tune_file(ens_ctx *ctx)
{
    const std::string path = tune_file_path();
    if (path.empty()) return;
    std::lock_guard<std::mutex> lock(tune_file_mutex);
    std::ifstream in(path);
    std::string line;
    const std::string prefix = ctx->device_tag + "/";
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string key;
        ens_ctx::Shape sh{};
        if (!(ls >> key >> sh.nsl >> sh.order >> sh.dense)) continue;
        // a line without the packed column predates packing: not measured (-1)
        if (!(ls >> sh.packed)) sh.packed = -1;
        if (!(sh.packed == -1 || sh.packed == 0 || sh.packed == 2 || sh.packed == 4 || sh.packed == 8)) continue;
        if (key.compare(0, prefix.size(), prefix) != 0) continue;
        if (!(sh.nsl == 1 || sh.nsl == 2 || sh.nsl == 4 || sh.nsl == 8) || sh.order < 1 || sh.order > 3 ||
            sh.dense < 0 || sh.dense > 1)
            continue;
        ctx->tune_cache[key.substr(prefix.size())] = sh;
    }
}

void save_tune_entry(const ens_ctx *ctx, const std::string &key, const ens_ctx::Shape &sh)
{
    const std::string path = tune_file_path();
    if (path.empty()) return;
    std::lock_guard<std::mutex> lock(tune_file_mutex);
    std::ofstream out(path, std::ios::app);
    if (out)
        out << ctx->device_tag << "/" << key << " " << sh.nsl << " " << sh.order << " " << sh.dense << " "
            << sh.packed << "\n";
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

const char *ens_version(void) { return "libens 0.1 (gfx950)"; }

ens_status ens_ctx_create(ens_ctx **out, void *stream)
{
    if (!out) return ENS_E_INVALID;
    *out = nullptr;
    ens_ctx *c = new (std::nothrow) ens_ctx();
    if (!c) return ENS_E_OOM;
    c->stream = static_cast<hipStream_t>(stream);
    c->tuning.struct_size = sizeof(ens_tuning);
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::string arch(prop.gcnArchName);
        arch = arch.substr(0, arch.find(':'));
        c->device_tag = arch + "/" + std::to_string(prop.multiProcessorCount);
        load_tune_file(c);
    }
    c->scratch = scratch_address(&c->scratch_err);
    *out = c;
    return ENS_OK;
}

void ens_ctx_destroy(ens_ctx *ctx) { delete ctx; }

const char *ens_last_error(const ens_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ens_status ens_set_tuning(ens_ctx *ctx, const ens_tuning *t)
{
    if (!ctx) return ENS_E_INVALID;
    if (!t || t->struct_size < sizeof(ens_tuning)) return fail(ctx, ENS_E_INVALID, "ens_tuning: bad struct_size");
    const int w = t->waves_per_sample_group;
    if (!(w == 0 || w == 1 || w == 2 || w == 4 || w == 8))
        return fail(ctx, ENS_E_RANGE, "waves_per_sample_group must be 0, 1, 2, 4 or 8 (got %d)", w);
    if (t->use_graph && t->collect_timing)
        return fail(ctx, ENS_E_INVALID, "use_graph and collect_timing exclude each other");
    if (t->item_order < 0 || t->item_order > 3)
        return fail(ctx, ENS_E_RANGE, "item_order must be 0, 1, 2 or 3 (got %d)", t->item_order);
    if (t->occupancy < 0 || t->occupancy > 2)
        return fail(ctx, ENS_E_RANGE, "occupancy must be 0, 1 or 2 (got %d)", t->occupancy);
    const int pk = t->packing;
    if (!(pk == 0 || pk == 1 || pk == 2 || pk == 4 || pk == 8))
        return fail(ctx, ENS_E_RANGE, "packing must be 0, 1, 2, 4 or 8 (got %d)", pk);
    if (t->gather < 0 || t->gather > 1) return fail(ctx, ENS_E_RANGE, "gather must be 0 or 1 (got %d)", t->gather);
    ctx->tuning = *t;
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_last_stats(const ens_ctx *ctx, ens_stats *out)
{
    if (!ctx || !out) return ENS_E_INVALID;
    if (out->struct_size < sizeof(ens_stats)) return ENS_E_INVALID;
    *out = ctx->stats;
    out->struct_size = sizeof(ens_stats);
    return ENS_OK;
}

ens_status ens_bind(ens_ctx *ctx, const ens_traces *tr, const ens_geometry *g, const ens_sem_cfg *sem)
{
    if (!ctx) return ENS_E_INVALID;
    if (!tr || !g || !sem) return fail(ctx, ENS_E_INVALID, "ens_bind: null argument");
    if (tr->struct_size < sizeof(ens_traces) || g->struct_size < sizeof(ens_geometry) ||
        sem->struct_size < sizeof(ens_sem_cfg))
        return fail(ctx, ENS_E_INVALID, "ens_bind: struct_size too small");
    if (!tr->data || !g->cmp_ptr || !g->offset) return fail(ctx, ENS_E_INVALID, "ens_bind: null array");
    if (tr->n_traces < 1 || tr->nt < 2 || tr->ld < tr->nt)
        return fail(ctx, ENS_E_INVALID, "ens_bind: need n_traces >= 1, nt >= 2, ld >= nt");
    if (tr->nt > (1 << 20)) return fail(ctx, ENS_E_RANGE, "ens_bind: nt too large");
    if (tr->n_traces >= (int64_t(1) << 31)) return fail(ctx, ENS_E_RANGE, "ens_bind: too many traces");
    if (!(tr->dt > 0.f) || !finite(tr->dt) || !(g->dx > 0.f) || !finite(g->dx))
        return fail(ctx, ENS_E_RANGE, "ens_bind: dt and dx must be positive");
    if (tr->store_dtype < ENS_DTYPE_F32 || tr->store_dtype > ENS_DTYPE_BF16)
        return fail(ctx, ENS_E_INVALID, "ens_bind: unknown store dtype %d", tr->store_dtype);
    if (tr->data_dtype < ENS_DTYPE_F32 || tr->data_dtype > ENS_DTYPE_BF16)
        return fail(ctx, ENS_E_INVALID, "ens_bind: unknown data dtype %d", tr->data_dtype);
    const bool data16 = tr->data_dtype != ENS_DTYPE_F32;
    if (data16 && tr->store_dtype != ENS_DTYPE_F32 && tr->store_dtype != tr->data_dtype)
        return fail(ctx, ENS_E_UNSUPPORTED, "ens_bind: 16-bit data are stored as they are or as binary32");
    if (data16 && !tr->scale) return fail(ctx, ENS_E_INVALID, "ens_bind: 16-bit data need per-trace scales");
    if (g->n_cmp < 1) return fail(ctx, ENS_E_INVALID, "ens_bind: n_cmp < 1");
    if (g->cmp_ptr[0] != 0 || g->cmp_ptr[g->n_cmp] != tr->n_traces)
        return fail(ctx, ENS_E_INVALID, "ens_bind: cmp_ptr must start at 0 and end at n_traces");
    for (int32_t c = 0; c < g->n_cmp; ++c)
        if (g->cmp_ptr[c + 1] < g->cmp_ptr[c]) return fail(ctx, ENS_E_INVALID, "ens_bind: cmp_ptr decreases at %d", c);
    for (int64_t i = 0; i < tr->n_traces; ++i)
        if (!finite(g->offset[i])) return fail(ctx, ENS_E_INVALID, "ens_bind: offset[%lld] not finite", (long long)i);
    if (sem->op != ENS_OP_CMP && sem->op != ENS_OP_CRS) return fail(ctx, ENS_E_INVALID, "ens_bind: unknown op %d", sem->op);
    if (sem->window < 1 || sem->window % 2 == 0 || !ens::window_supported(sem->window))
        return fail(ctx, ENS_E_RANGE, "ens_bind: window must be odd, 3..%d (got %d)", 2 * ENS_MAX_HALF_WINDOW + 1,
                    sem->window);
    if (sem->ap_lo < 0 || sem->ap_hi < 0) return fail(ctx, ENS_E_RANGE, "ens_bind: negative aperture");
    // binary16 windows: the traveltime grid 2^(lb-23) samples, 2^lb >= nt + PAD, stays at or
    // below 2^-9 samples
    static_assert(ENS_MAX_NT_F16 + PAD == (1 << 14), "binary16 record limit");
    if (tr->store_dtype == ENS_DTYPE_F16 && tr->nt > ENS_MAX_NT_F16)
        return fail(ctx, ENS_E_UNSUPPORTED,
                    "ens_bind: binary16 windows take records of at most %d samples (got %d); store longer "
                    "records as binary32 or bfloat16",
                    static_cast<int>(ENS_MAX_NT_F16), tr->nt);
    if (data16) {
        // the scales fold into binary16 interpolation weights exactly only as powers of two
        std::vector<float> sc(static_cast<size_t>(tr->n_traces));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(sc.data(), tr->scale, sc.size() * sizeof(float), hipMemcpyDeviceToHost,
                                        ctx->stream));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
        for (size_t i = 0; i < sc.size(); ++i)
            if (!is_pow2(sc[i]))
                return fail(ctx, ENS_E_RANGE, "ens_bind: scale[%zu] = %g is not a positive power of two", i,
                            static_cast<double>(sc[i]));
    }

    const int64_t n_tr = tr->n_traces;
    const int32_t nt = tr->nt;
    const int64_t ld = ((nt + 2 * PAD) + 63) / 64 * 64;
    ctx->bound = false;
    const bool store16 = tr->store_dtype != ENS_DTYPE_F32;
    // 16-bit rows hold two copies, the second shifted by one sample, so that
    // every window starts on a dword boundary in one of them
    const size_t row_bytes = store16 ? 2 * 2 * ld : 4 * ld;
    HIP_OR_FAIL(ctx, ctx->store.ensure(static_cast<size_t>(n_tr) * row_bytes));
    HIP_OR_FAIL(ctx, ctx->scale.ensure(static_cast<size_t>(n_tr) * sizeof(float)));
    HIP_OR_FAIL(ctx, ctx->qexp.ensure(static_cast<size_t>(n_tr) * sizeof(int32_t)));
    HIP_OR_FAIL(ctx, ctx->wsc16.ensure(static_cast<size_t>(n_tr) * sizeof(uint32_t)));
    if (!data16 && !store16) {
        HIP_OR_FAIL(ctx, ens::launch_store_f32(static_cast<const float *>(tr->data), tr->ld, n_tr, nt, ld,
                                               ctx->store.as<float>(), ctx->stream));
    } else if (!data16) {
        HIP_OR_FAIL(ctx, ctx->master.ensure(static_cast<size_t>(n_tr) * ld * 4));
        HIP_OR_FAIL(ctx, ens::launch_store_f32(static_cast<const float *>(tr->data), tr->ld, n_tr, nt, ld,
                                               ctx->master.as<float>(), ctx->stream));
        HIP_OR_FAIL(ctx, ens::launch_quantize(static_cast<const float *>(tr->data), tr->ld, n_tr, nt, tr->store_dtype,
                                              ctx->store.as<uint16_t>(), ld, PAD, ctx->scale.as<float>(), true,
                                              ctx->qexp.as<int32_t>(), ctx->stream));
    } else {
        // caller-quantised rows: the dual 16-bit layout when searched in 16 bits, the binary32
        // samples from master or dequantised
        float *f32_rows = nullptr;
        if (store16) {
            HIP_OR_FAIL(ctx, ctx->master.ensure(static_cast<size_t>(n_tr) * ld * 4));
            f32_rows = ctx->master.as<float>();
        } else {
            f32_rows = ctx->store.as<float>();
        }
        uint16_t *rows16 = store16 ? ctx->store.as<uint16_t>() : nullptr;
        HIP_OR_FAIL(ctx, ens::launch_store16(static_cast<const uint16_t *>(tr->data), tr->ld, n_tr, nt,
                                             tr->data_dtype, tr->scale, rows16, ld,
                                             tr->master ? nullptr : f32_rows, ctx->qexp.as<int32_t>(), ctx->stream));
        if (tr->master)
            HIP_OR_FAIL(ctx, ens::launch_store_f32(tr->master, tr->ld, n_tr, nt, ld, f32_rows, ctx->stream));
    }
    if (store16)
        HIP_OR_FAIL(ctx, ens::launch_relscale(ctx->qexp.as<int32_t>(), n_tr, ctx->scale.as<float>(),
                                              ctx->wsc16.as<uint32_t>(), ctx->stream));
    {
        // binary16 window grid: B = the smallest power of two >= max(4096, nt + PAD)
        int lb = 12;
        while ((int64_t(1) << lb) < static_cast<int64_t>(nt) + PAD) ++lb;
        const float B = std::ldexp(1.0f, lb);
        ctx->h16_kq = B + static_cast<float>(PAD - sem->window / 2);
        std::memcpy(&ctx->h16_bbits, &B, sizeof B);
        ctx->h16_shift = static_cast<uint32_t>(22 - lb);
    }
    std::vector<TraceMeta> meta(static_cast<size_t>(n_tr));
    for (int32_t c = 0; c < g->n_cmp; ++c)
        for (int64_t i = g->cmp_ptr[c]; i < g->cmp_ptr[c + 1]; ++i) {
            const float h = g->offset[i];
            meta[i].cx = static_cast<float>(c) * g->dx;
            meta[i].h2 = h * h;
            meta[i].cmp = c;
            meta[i].h = h;
        }
    std::vector<int32_t> ap(static_cast<size_t>(nt));
    for (int32_t n0 = 0; n0 < nt; ++n0) ap[n0] = lerp_round(sem->ap_lo, sem->ap_hi, n0, nt);
    HIP_OR_FAIL(ctx, ctx->meta.ensure(meta.size() * sizeof(TraceMeta)));
    HIP_OR_FAIL(ctx, ctx->cmp_ptr.ensure(sizeof(int64_t) * (g->n_cmp + 1)));
    HIP_OR_FAIL(ctx, ctx->ap_tab.ensure(sizeof(int32_t) * nt));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->meta.p, meta.data(), meta.size() * sizeof(TraceMeta),
                                    hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->cmp_ptr.p, g->cmp_ptr, sizeof(int64_t) * (g->n_cmp + 1),
                                    hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->ap_tab.p, ap.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice,
                                    ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    ctx->n_tr = n_tr;
    ctx->ld = ld;
    ctx->nt = nt;
    ctx->n_cmp = g->n_cmp;
    ctx->store_dtype = tr->store_dtype;
    ctx->dt = tr->dt;
    ctx->dx = g->dx;
    ctx->op = sem->op;
    ctx->window = sem->window;
    ctx->ap_lo = sem->ap_lo;
    ctx->ap_hi = sem->ap_hi;
    {
        const int32_t apm = std::max(sem->ap_lo, sem->ap_hi);
        int64_t most = 0;
        for (int32_t j = 0; j < g->n_cmp; ++j) {
            const int32_t lo = std::max(0, j - apm), hi = std::min(g->n_cmp - 1, j + apm);
            most = std::max<int64_t>(most, g->cmp_ptr[hi + 1] - g->cmp_ptr[lo]);
        }
        ctx->max_ap_traces = static_cast<int32_t>(most);
    }
    ctx->bound = true;
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_quantize(ens_ctx *ctx, const float *data, int64_t n_traces, int32_t nt, int64_t ld,
                        int32_t dtype, uint16_t *q, float *scale)
{
    if (!ctx) return ENS_E_INVALID;
    if (!data || !q || !scale) return fail(ctx, ENS_E_INVALID, "ens_quantize: null pointer");
    if (n_traces < 0 || nt < 1 || ld < nt) return fail(ctx, ENS_E_INVALID, "ens_quantize: bad sizes");
    if (dtype != ENS_DTYPE_F16 && dtype != ENS_DTYPE_BF16)
        return fail(ctx, ENS_E_INVALID, "ens_quantize: dtype must be F16 or BF16");
    HIP_OR_FAIL(ctx, ens::launch_quantize(data, ld, n_traces, nt, dtype, q, nt, 0, scale, false, nullptr,
                                          ctx->stream));
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_search(ens_ctx *ctx, const ens_traces *traces, const ens_geometry *geometry,
                      const ens_sem_cfg *sem, const ens_t0_grid *grid, const ens_bounds *bounds,
                      const ens_de_cfg *de, uint64_t seed, ens_result *out)
{
    if (!ctx) return ENS_E_INVALID;
    if (!grid || !bounds || !de || !out) return fail(ctx, ENS_E_INVALID, "ens_search: null argument");
    const ens_status st = ens_bind(ctx, traces, geometry, sem);
    if (st != ENS_OK) return st;
    return ens_search_bound(ctx, grid, bounds, de, seed, out);
}

ens_status ens_search_bound(ens_ctx *ctx, const ens_t0_grid *grid, const ens_bounds *bounds,
                            const ens_de_cfg *de, uint64_t seed, ens_result *out)
{
    if (!ctx) return ENS_E_INVALID;
    if (!ctx->bound) return fail(ctx, ENS_E_STATE, "ens_search_bound: call ens_bind first");
    if (!grid || !bounds || !de || !out) return fail(ctx, ENS_E_INVALID, "ens_search: null argument");
    if (grid->struct_size < sizeof(ens_t0_grid) || bounds->struct_size < sizeof(ens_bounds) ||
        de->struct_size < sizeof(ens_de_cfg) || out->struct_size < sizeof(ens_result))
        return fail(ctx, ENS_E_INVALID, "ens_search: struct_size too small");
    if (!out->params || !out->S) return fail(ctx, ENS_E_INVALID, "ens_search: null output");
    const int32_t P = ctx->op, nt = ctx->nt;
    const int32_t n_out = grid->cmp_out ? grid->n_cmp_out : ctx->n_cmp;
    if (n_out < 1) return fail(ctx, ENS_E_INVALID, "ens_search: no output CMPs");
    if (grid->cmp_out)
        for (int32_t o = 0; o < n_out; ++o)
            if (grid->cmp_out[o] < 0 || grid->cmp_out[o] >= ctx->n_cmp)
                return fail(ctx, ENS_E_RANGE, "ens_search: cmp_out[%d] = %d out of range", o, grid->cmp_out[o]);
    if (grid->t_begin < 0 || grid->t_end > nt || grid->t_begin >= grid->t_end)
        return fail(ctx, ENS_E_RANGE, "ens_search: need 0 <= t_begin < t_end <= nt");
    for (int d = 0; d < P; ++d)
        if (!finite(bounds->lo[d]) || !finite(bounds->hi[d]) || !(bounds->lo[d] < bounds->hi[d]))
            return fail(ctx, ENS_E_RANGE, "ens_search: bounds %d need lo < hi", d);
    if (de->n_skip < 0 || de->n_skip > 2) return fail(ctx, ENS_E_RANGE, "ens_search: n_skip must be 0, 1 or 2");
    if (de->n_skip > 0 && !de->ens_enabled)
        return fail(ctx, ENS_E_RANGE, "ens_search: n_skip needs ens_enabled");
    if (de->ng_f < 0 || de->ng_bf < 0 || de->n_cycle < 0)
        return fail(ctx, ENS_E_RANGE, "ens_search: negative generation or cycle count");
    if (de->np_lo < 4 || de->np_hi < 4 || de->np_lo > ENS_MAX_POP || de->np_hi > ENS_MAX_POP)
        return fail(ctx, ENS_E_RANGE, "ens_search: NP_f must lie in [4, %d]", ENS_MAX_POP);
    if (de->ens_enabled) {
        if (de->n_bucket < 1) return fail(ctx, ENS_E_RANGE, "ens_search: n_bucket < 1");
        if (de->n_cycle > 0 && (de->np_bf < 5 || de->np_bf > ENS_MAX_POP))
            return fail(ctx, ENS_E_RANGE, "ens_search: NP_bf must lie in [5, %d]", ENS_MAX_POP);
    }
    if (!finite(de->F) || !finite(de->CR) || de->CR < 0.f || de->CR > 1.f)
        return fail(ctx, ENS_E_RANGE, "ens_search: F must be finite and CR in [0, 1]");
    if (de->adapt != 0 && de->adapt != 1) return fail(ctx, ENS_E_RANGE, "ens_search: adapt must be 0 or 1");
    if (de->adapt && !(de->F > 0.f && de->F <= 1.f))
        return fail(ctx, ENS_E_RANGE, "ens_search: with adapt, F (the initial mean) must lie in (0, 1]");
    if (de->polish_steps < 0 || (de->polish_steps > 0 && !(de->polish_lr > 0.f)))
        return fail(ctx, ENS_E_RANGE, "ens_search: polish needs steps >= 0 and lr > 0");

    const int32_t t_begin = grid->t_begin, n_t = grid->t_end - grid->t_begin;
    const int64_t n_s = static_cast<int64_t>(n_out) * n_t;
    hipStream_t st = ctx->stream;

    // per-time tables
    std::vector<float> lo(static_cast<size_t>(nt) * 3), hi(static_cast<size_t>(nt) * 3);
    for (int32_t n0 = 0; n0 < nt; ++n0) sample_box(*bounds, n0, ctx->dt, &lo[n0 * 3], &hi[n0 * 3]);
    std::vector<int32_t> cmp_out(static_cast<size_t>(n_out));
    for (int32_t o = 0; o < n_out; ++o) cmp_out[o] = grid->cmp_out ? grid->cmp_out[o] : o;

    // work items: consecutive t with equal NP packed floor(64/NP) per wave, in
    // (group, t) order (order 1); the second copy puts the costliest items
    // first (order 2); the third keeps each XCD's contiguous share of the
    // (group, t) order and puts the costliest items of that share first
    // (order 3)
    const double traces_per_cmp = static_cast<double>(ctx->n_tr) / ctx->n_cmp;
    // item classes: 0 = first sweep (NP_f), 1 = backward sweeps, 2 = later
    // forward sweeps (NP_bf); each estimates t = t_begin + init + m stride
    const int32_t stride = de->n_skip + 1;
    const int32_t init_of[3] = {0, std::min(1, de->n_skip), de->n_skip};
    auto build_items = [&](int32_t n_groups, int cls, std::vector<int4> &items) {
        for (int32_t gidx = 0; gidx < n_groups; ++gidx) {
            int32_t t = t_begin + init_of[cls];
            while (t < grid->t_end) {
                const int32_t np = cls == 0 ? lerp_round(de->np_lo, de->np_hi, t, nt) : de->np_bf;
                const int32_t per = ens::WAVE / np;
                int32_t ns = 1;
                while (ns < per && t + ns * stride < grid->t_end &&
                       (cls == 0 ? lerp_round(de->np_lo, de->np_hi, t + ns * stride, nt) : de->np_bf) == np)
                    ++ns;
                items.push_back(make_int4(gidx, t, ns | (stride << 8), np));
                t += ns * stride;
            }
        }
    };
    // an item's cost: the lanes it evaluates (ns NP, or for a packed item the
    // lanes in .w) times the traces of its widest aperture
    auto costliest_first = [&](const std::vector<int4> &items, bool packed_items_) {
        std::vector<int4> v = items;
        auto cost = [&](const int4 &it) {
            const int32_t ns = it.z & 0xff, st = it.z >> 8;
            const int32_t tm = it.y + (ns - 1) * st;
            const int32_t ap = lerp_round(ctx->ap_lo, ctx->ap_hi, tm, nt);
            const double lanes = packed_items_ ? it.w : static_cast<double>(ns) * it.w;
            return lanes * (2 * ap + 1) * traces_per_cmp;
        };
        std::stable_sort(v.begin(), v.end(), [&](const int4 &x, const int4 &y) { return cost(x) > cost(y); });
        return v;
    };
    // the share of XCD x under the block remapping of the kernels (xcd_remap)
    auto xcd_costliest_first = [&](const std::vector<int4> &items, bool packed_items_) {
        std::vector<int4> v = items;
        const size_t n = v.size(), per = n / 8, rem = n % 8;
        for (size_t x = 0; x < 8; ++x) {
            const size_t b = x * per + std::min(x, rem), e = b + per + (x < rem ? 1 : 0);
            std::vector<int4> part(v.begin() + b, v.begin() + e);
            part = costliest_first(part, packed_items_);
            std::copy(part.begin(), part.end(), v.begin() + b);
        }
        return v;
    };
    const bool ens = de->ens_enabled != 0;
    const int32_t n_buckets = ens ? (n_out + de->n_bucket - 1) / de->n_bucket : 0;
    std::vector<int4> cls_items[3][4];  // [class][order 1, 2, 3 at index 1, 2, 3]
    build_items(ens ? n_buckets : n_out, 0, cls_items[0][1]);
    if (ens && de->n_cycle > 0) {
        build_items(n_buckets, 1, cls_items[1][1]);
        build_items(n_buckets, 2, cls_items[2][1]);
    }
    size_t item_off[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}, n_items_total = 0;
    for (int c = 0; c < 3; ++c) {
        cls_items[c][2] = costliest_first(cls_items[c][1], false);
        cls_items[c][3] = xcd_costliest_first(cls_items[c][1], false);
        for (int od = 1; od <= 3; ++od) {
            item_off[c][od] = n_items_total;
            n_items_total += cls_items[c][od].size();
        }
    }
    // packed exploration (fixed F and CR): consecutive estimated t of a group
    // laid end to end over the 64 G lanes of G waves
    // Packing is measured only where one population per lane group leaves
    // lanes idle: under 90% of the exploration items' lanes carrying a member
    // (populations of 33..63 members fill a wave only once).
    double lanes_busy = 0.0;
    for (const int4 &it : cls_items[0][1]) lanes_busy += static_cast<double>(it.z & 0xff) * it.w;
    const bool can_pack = !de->adapt;
    const bool measure_pack =
        can_pack && lanes_busy < 0.9 * static_cast<double>(ens::WAVE) * static_cast<double>(cls_items[0][1].size());
    constexpr int N_PACK = 3;
    const int32_t pack_waves[N_PACK] = {2, 4, 8};
    std::vector<int4> packed_items[N_PACK][4];   // [waves][order 1, 2, 3 at index 1, 2, 3]
    size_t packed_off[N_PACK][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    auto pack_index = [&](int waves) { return waves == 2 ? 0 : (waves == 4 ? 1 : 2); };
    if (can_pack) {
        for (int pi = 0; pi < N_PACK; ++pi) {
            const int32_t G = pack_waves[pi], lanes = ens::WAVE * G;
            const int32_t max_ns = std::min(255, ens::PACK_MAX_SAMPLES_PER_WAVE * G);
            for (int32_t gidx = 0; gidx < (ens ? n_buckets : n_out); ++gidx) {
                int32_t t = t_begin + init_of[0];
                while (t < grid->t_end) {
                    int32_t ns = 0, used = 0;
                    while (ns < max_ns && t + ns * stride < grid->t_end) {
                        const int32_t np = lerp_round(de->np_lo, de->np_hi, t + ns * stride, nt);
                        if (used + np > lanes) break;
                        used += np;
                        ++ns;
                    }
                    packed_items[pi][1].push_back(make_int4(gidx, t, ns | (stride << 8), used));
                    t += ns * stride;
                }
            }
            packed_items[pi][2] = costliest_first(packed_items[pi][1], true);
            packed_items[pi][3] = xcd_costliest_first(packed_items[pi][1], true);
            for (int od = 1; od <= 3; ++od) {
                packed_off[pi][od] = n_items_total;
                n_items_total += packed_items[pi][od].size();
            }
        }
    }
    std::vector<int32_t> np_tab(static_cast<size_t>(nt));
    for (int32_t n0 = 0; n0 < nt; ++n0) np_tab[n0] = lerp_round(de->np_lo, de->np_hi, n0, nt);
    const size_t pbytes = sizeof(float) * static_cast<size_t>(n_s) * P, sbytes = sizeof(float) * n_s;
    HIP_OR_FAIL(ctx, ctx->lo_tab.ensure(lo.size() * sizeof(float)));
    HIP_OR_FAIL(ctx, ctx->hi_tab.ensure(hi.size() * sizeof(float)));
    HIP_OR_FAIL(ctx, ctx->cmp_out.ensure(cmp_out.size() * sizeof(int32_t)));
    HIP_OR_FAIL(ctx, ctx->items.ensure(std::max<size_t>(n_items_total, 1) * sizeof(int4)));
    HIP_OR_FAIL(ctx, ctx->counters.ensure(8 * sizeof(unsigned long long)));
    HIP_OR_FAIL(ctx, ctx->np_tab.ensure(np_tab.size() * sizeof(int32_t)));
    if (ens) {
        HIP_OR_FAIL(ctx, ctx->X.ensure(pbytes));
        HIP_OR_FAIL(ctx, ctx->Y.ensure(pbytes));
        HIP_OR_FAIL(ctx, ctx->XS.ensure(sbytes));
        HIP_OR_FAIL(ctx, ctx->YS.ensure(sbytes));
    }
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->lo_tab.p, lo.data(), lo.size() * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->hi_tab.p, hi.data(), hi.size() * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->cmp_out.p, cmp_out.data(), cmp_out.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, st));
    int4 *dev_items = ctx->items.as<int4>();
    for (int c = 0; c < 3; ++c)
        for (int od = 1; od <= 3; ++od)
            if (!cls_items[c][od].empty())
                HIP_OR_FAIL(ctx, hipMemcpyAsync(dev_items + item_off[c][od], cls_items[c][od].data(),
                                                cls_items[c][od].size() * sizeof(int4), hipMemcpyHostToDevice, st));
    for (int pi = 0; pi < N_PACK; ++pi)
        for (int od = 1; od <= 3; ++od)
            if (!packed_items[pi][od].empty())
                HIP_OR_FAIL(ctx, hipMemcpyAsync(dev_items + packed_off[pi][od], packed_items[pi][od].data(),
                                                packed_items[pi][od].size() * sizeof(int4), hipMemcpyHostToDevice,
                                                st));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->np_tab.p, np_tab.data(), np_tab.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, st));

    float *final_params = nullptr, *final_S = nullptr;
    ens::SearchArgs a{};
    a.sv = view_of(ctx, false);
    a.cmp_out = ctx->cmp_out.as<int32_t>();
    a.n_out = n_out;
    a.t_begin = t_begin;
    a.n_t = n_t;
    a.lo_tab = ctx->lo_tab.as<float>();
    a.hi_tab = ctx->hi_tab.as<float>();
    a.n_bucket = de->n_bucket;
    a.inject = de->inject;
    a.seed = seed;
    a.F = de->F;
    a.CR = de->CR;
    a.adapt = de->adapt;
    a.cr_thr = static_cast<uint64_t>(std::ceil(static_cast<double>(de->CR) * 4294967296.0));
    a.counters = ctx->counters.as<unsigned long long>();
    a.np_tab = ctx->np_tab.as<int32_t>();
    a.packed = 0;
    // LDS-staged binary32 windows (ens_tuning.gather = 1; fixed F and CR, one
    // population per lane group), where the table fits
    a.tiles = ctx->tuning.gather == 1 && ctx->store_dtype == ENS_DTYPE_F32 && !de->adapt &&
              static_cast<size_t>(ctx->max_ap_traces) * 8 <= 64 * 1024;
    a.tile_cap = ctx->max_ap_traces;

    // launch sequence of the evolution (slices and item order filled in below)
    std::vector<ens_ctx::Launch> seq;
    auto search_launch = [&](const ens::SearchArgs &sa, int kind, int cls) {
        ens_ctx::Launch l{};
        l.a = sa;
        l.kind = kind;
        l.n_blocks = static_cast<int32_t>(cls_items[cls][1].size());
        l.item_class = cls;
        seq.push_back(l);
    };
    if (!ens) {
        a.plain = 1;
        a.stage = 0;
        a.k_begin = 0;
        a.k_end = 1;
        a.ng = de->ng_f;
        a.Yp = out->params;
        a.YS = out->S;
        search_launch(a, 0, 0);
    } else {
        float *X = ctx->X.as<float>(), *XS = ctx->XS.as<float>();
        float *Y = ctx->Y.as<float>(), *YS = ctx->YS.as<float>();
        a.plain = 0;
        const int32_t n_stage = 1 + 2 * de->n_cycle;
        // a stage's sweep is split into launches of at most STEPS trace steps
        constexpr int32_t STEPS = 32;
        const int32_t n_steps = std::min(de->n_bucket, n_out);
        for (int32_t s = 0; s < n_stage; ++s) {
            const int cls = s == 0 ? 0 : (s % 2 == 1 ? 1 : 2);
            a.stage = s;
            a.forward = (s % 2 == 0) ? 1 : 0;
            a.ng = s == 0 ? de->ng_f : de->ng_bf;
            a.n_items = static_cast<int32_t>(cls_items[cls][1].size());
            a.Xp = X;
            a.XS = XS;
            a.Yp = Y;
            a.YS = YS;
            for (int32_t k0 = 0; k0 < n_steps; k0 += STEPS) {
                a.k_begin = k0;
                a.k_end = std::min(n_steps, k0 + STEPS);
                search_launch(a, s == 0 ? 0 : 1, cls);
            }
            if (stride > 1) {
                ens_ctx::Launch l{};
                l.interp = 1;
                l.kind = s == 0 ? 0 : 1;
                l.item_class = cls;
                ens::InterpArgs &ia = l.ia;
                ia.sv = a.sv;
                ia.cmp_out = a.cmp_out;
                ia.n_out = n_out;
                ia.t_begin = t_begin;
                ia.n_t = n_t;
                ia.lo_tab = a.lo_tab;
                ia.hi_tab = a.hi_tab;
                ia.stride = stride;
                ia.init = init_of[cls];
                ia.stage = s;
                ia.kind = l.kind;
                ia.Xp = X;
                ia.XS = XS;
                ia.Yp = Y;
                ia.YS = YS;
                ia.counters = ctx->counters.as<unsigned long long>();
                seq.push_back(l);
            }
            std::swap(X, Y);
            std::swap(XS, YS);
        }
        final_params = X;
        final_S = XS;
    }
    // one step counter per ENS search launch (pacing), plus one for shape trials
    size_t n_paced = 0;
    for (const auto &l : seq)
        if (!l.interp && !l.a.plain) ++n_paced;
    HIP_OR_FAIL(ctx, ctx->progress.ensure((n_paced + 1) * sizeof(unsigned long long)));
    unsigned long long *const progress = ctx->progress.as<unsigned long long>();
    {
        size_t i = 0;
        for (auto &l : seq)
            if (!l.interp && !l.a.plain) l.a.progress = progress + i++;
    }
    ctx->stats = ens_stats{};
    ctx->stats.struct_size = sizeof(ens_stats);

    // launch shape per kernel kind: fixed by the caller, cached, or measured
    for (int kind = 0; kind < 2; ++kind) {
        const ens_ctx::Launch *first = nullptr;
        for (const auto &l : seq)
            if (l.kind == kind && !l.interp) {
                first = &l;
                break;
            }
        if (!first) continue;
        char key[256];
        // the generation count scales every shape's time alike, so it is not part of the key
        snprintf(key, sizeof key, "%d/%d/%d/%d/%d/%d/%d/%d/%d/%d/%d/%d", kind, P, ctx->store_dtype, ctx->window,
                 de->np_lo, de->np_hi, de->adapt, first->n_blocks, n_out, n_t, ctx->ap_hi, stride);
        int nsl = ctx->tuning.waves_per_sample_group, order = ctx->tuning.item_order;
        int dense = ctx->tuning.occupancy == 0 ? -1 : (ctx->tuning.occupancy == 2 ? 1 : 0);
        // packed waves: 0 not packed, -1 to be measured; packing is measured
        // only when the slice count and item order are too
        int packed = 0;
        if (kind == 0 && can_pack) {
            const int tp = ctx->tuning.packing;
            packed = tp >= 2 ? tp : (tp == 0 && measure_pack && nsl == 0 && order == 0 ? -1 : 0);
        }
        if (packed > 0) nsl = packed;
        if (nsl == 0 || order == 0 || dense < 0 || packed < 0) {
            auto hit = ctx->tune_cache.find(key);
            if (hit != ctx->tune_cache.end()) {
                if (packed < 0) {
                    packed = hit->second.packed;
                    if (packed > 0) nsl = packed;
                }
                if (nsl == 0) nsl = hit->second.nsl;
                if (order == 0) order = hit->second.order;
                if (dense < 0) dense = hit->second.dense;
            }
        }
        if (nsl == 0 || order == 0 || dense < 0 || packed < 0) {
            // time the first launch of this kind: every free slice count at the
            // first order and register budget, then the other orders and
            // budgets at the fastest count; then (where offered) each packed
            // width at the best order and budget so far, and the other orders
            // and budgets at the fastest width
            const int fixed_nsl = packed > 0 ? 0 : nsl, fixed_order = order, fixed_dense = dense,
                      fixed_packed = packed;
            const int od0 = fixed_order ? fixed_order : 1, dn0 = fixed_dense >= 0 ? fixed_dense : 0;
            const int max_dense = de->adapt ? 0 : 1;  // JADE: one register budget
            ens::SearchArgs ta = first->a;
            // every generation repeats the same trace loop, so the trials run at
            // most TUNE_GENERATIONS of them (all trace steps of the launch:
            // cutting those changed the ranking)
            ta.ng = std::min(ta.ng, TUNE_GENERATIONS);
            if (kind == 1) {
                HIP_OR_FAIL(ctx, hipMemsetAsync(ctx->X.p, 0, pbytes, st));
                HIP_OR_FAIL(ctx, hipMemsetAsync(ctx->XS.p, 0, sbytes, st));
                HIP_OR_FAIL(ctx, hipMemsetAsync(ctx->Y.p, 0, pbytes, st));
                HIP_OR_FAIL(ctx, hipMemsetAsync(ctx->YS.p, 0, sbytes, st));
            }
            while (ctx->events.size() < 2) {
                hipEvent_t e;
                HIP_OR_FAIL(ctx, hipEventCreate(&e));
                ctx->events.push_back(e);
            }
            if (ta.progress) ta.progress = progress + n_paced;
            for (int warm = 0; warm <= max_dense; ++warm) {  // load the kernel variants once
                if (ta.progress) HIP_OR_FAIL(ctx, hipMemsetAsync(ta.progress, 0, sizeof(unsigned long long), st));
                ta.nsl = fixed_nsl ? fixed_nsl : 1;
                ta.xcd_order = 1;
                ta.items = dev_items + item_off[first->item_class][1];
                HIP_OR_FAIL(ctx, ens::launch_search(P, ctx->store_dtype, ctx->window, kind, warm, ta,
                                                    first->n_blocks, st));
                if (fixed_packed != 0) {
                    const int pi = pack_index(fixed_packed > 0 ? fixed_packed : 2);
                    ens::SearchArgs pa = ta;
                    pa.packed = 1;
                    pa.nsl = pack_waves[pi];
                    pa.items = dev_items + packed_off[pi][1];
                    if (pa.progress)
                        HIP_OR_FAIL(ctx, hipMemsetAsync(pa.progress, 0, sizeof(unsigned long long), st));
                    HIP_OR_FAIL(ctx, ens::launch_search(P, ctx->store_dtype, ctx->window, kind, warm, pa,
                                                        static_cast<int32_t>(packed_items[pi][1].size()), st));
                }
            }
            float best = -1.f;
            // ns: slices (packed: waves), od: item order, dn: register budget,
            // pk: 1 for a packed workgroup of ns waves
            auto trial = [&](int ns, int od, int dn, int pk, float *ms_out) -> hipError_t {
                ta.nsl = ns;
                ta.xcd_order = od != 2;
                ta.packed = pk;
                ta.items = pk ? dev_items + packed_off[pack_index(ns)][od] : dev_items + item_off[first->item_class][od];
                const int32_t nb =
                    pk ? static_cast<int32_t>(packed_items[pack_index(ns)][od].size()) : first->n_blocks;
                hipError_t e = hipSuccess;
                float ms = -1.f;
                // launches under 5 ms are timed three times (the fastest counts):
                // one short timing is too noisy to rank shapes a few % apart
                for (int rep = 0; rep < 3; ++rep) {
                    if (ta.progress &&
                        (e = hipMemsetAsync(ta.progress, 0, sizeof(unsigned long long), st)) != hipSuccess)
                        return e;
                    if ((e = hipEventRecord(ctx->events[0], st)) != hipSuccess) return e;
                    if ((e = ens::launch_search(P, ctx->store_dtype, ctx->window, kind, dn, ta, nb, st)) !=
                        hipSuccess)
                        return e;
                    if ((e = hipEventRecord(ctx->events[1], st)) != hipSuccess) return e;
                    if ((e = hipEventSynchronize(ctx->events[1])) != hipSuccess) return e;
                    float t = 0.f;
                    if ((e = hipEventElapsedTime(&t, ctx->events[0], ctx->events[1])) != hipSuccess) return e;
                    ctx->stats.tune_ms += t;
                    ms = ms < 0.f ? t : std::min(ms, t);
                    if (t >= 5.f) break;
                }
                if (best < 0.f || ms < best) {
                    best = ms;
                    nsl = ns;
                    order = od;
                    dense = dn;
                    packed = pk ? ns : 0;
                }
                if (ms_out) *ms_out = ms;
                return hipSuccess;
            };
            if (fixed_packed <= 0) {
                const int nsl_opts[4] = {1, 2, 4, 8};
                for (int ns : nsl_opts)
                    if (fixed_nsl == 0 || ns == fixed_nsl) HIP_OR_FAIL(ctx, trial(ns, od0, dn0, 0, nullptr));
                const int ns_best = nsl;
                for (int od = 1; od <= 3; ++od)
                    for (int dn = 0; dn <= max_dense; ++dn)
                        if (!(od == od0 && dn == dn0) && (fixed_order == 0 || od == fixed_order) &&
                            (fixed_dense < 0 || dn == fixed_dense))
                            HIP_OR_FAIL(ctx, trial(ns_best, od, dn, 0, nullptr));
            }
            if (fixed_packed != 0) {
                const int od1 = best < 0.f ? od0 : order, dn1 = best < 0.f ? dn0 : dense;
                int g_best = fixed_packed;
                if (fixed_packed < 0) {
                    float t_best = -1.f;
                    for (int pi = 0; pi < N_PACK; ++pi) {
                        float t = -1.f;
                        HIP_OR_FAIL(ctx, trial(pack_waves[pi], od1, dn1, 1, &t));
                        if (t_best < 0.f || t < t_best) {
                            t_best = t;
                            g_best = pack_waves[pi];
                        }
                    }
                } else {
                    HIP_OR_FAIL(ctx, trial(g_best, od1, dn1, 1, nullptr));
                }
                for (int od = 1; od <= 3; ++od)
                    for (int dn = 0; dn <= max_dense; ++dn)
                        if (!(od == od1 && dn == dn1) && (fixed_order == 0 || od == fixed_order) &&
                            (fixed_dense < 0 || dn == fixed_dense))
                            HIP_OR_FAIL(ctx, trial(g_best, od, dn, 1, nullptr));
            }
            ctx->tune_cache[key] = {nsl, order, dense, packed};
            if (!ctx->device_tag.empty()) save_tune_entry(ctx, key, ctx->tune_cache[key]);
        }
        ctx->stats.waves_used[kind] = nsl;
        ctx->stats.order_used[kind] = order;
        ctx->stats.dense_used[kind] = dense;
        if (kind == 0) ctx->stats.packed_used = packed;
        for (auto &l : seq)
            if (l.kind == kind && !l.interp) {
                l.a.nsl = nsl;
                l.dense = dense;
                if (packed > 0) {
                    const int pi = pack_index(packed);
                    l.a.packed = 1;
                    l.a.xcd_order = order != 2;
                    l.a.items = dev_items + packed_off[pi][order];
                    l.n_blocks = static_cast<int32_t>(packed_items[pi][order].size());
                } else {
                    l.a.packed = 0;
                    l.a.xcd_order = order != 2;
                    l.a.items = dev_items + item_off[l.item_class][order];
                }
            }
    }
    HIP_OR_FAIL(ctx, hipMemsetAsync(ctx->counters.p, 0, 8 * sizeof(unsigned long long), st));
    HIP_OR_FAIL(ctx, hipMemsetAsync(progress, 0, (n_paced + 1) * sizeof(unsigned long long), st));
    for (const auto &l : seq) ctx->stats.launches[l.kind] += 1;
    const bool timing = ctx->tuning.collect_timing != 0;
    const bool graph = ctx->tuning.use_graph != 0 && !timing;
    if (timing) {
        while (ctx->events.size() < 2 * seq.size()) {
            hipEvent_t e;
            HIP_OR_FAIL(ctx, hipEventCreate(&e));
            ctx->events.push_back(e);
        }
    }
    if (graph) {
        bool same = ctx->graph_exec && ctx->graph_seq.size() == seq.size();
        for (size_t i = 0; same && i < seq.size(); ++i)
            same = std::memcmp(&seq[i], &ctx->graph_seq[i], sizeof(ens_ctx::Launch)) == 0;
        if (!same) {
            ctx->drop_graph();
            HIP_OR_FAIL(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            for (const auto &l : seq) {
                le = l.interp ? ens::launch_interp(P, ctx->store_dtype, ctx->window, l.ia, st)
                              : ens::launch_search(P, ctx->store_dtype, ctx->window, l.kind, l.dense, l.a, l.n_blocks, st);
                if (le != hipSuccess) break;
            }
            hipGraph_t gph = nullptr;
            hipError_t ce = hipStreamEndCapture(st, &gph);
            HIP_OR_FAIL(ctx, le);
            HIP_OR_FAIL(ctx, ce);
            ctx->graph = gph;
            HIP_OR_FAIL(ctx, hipGraphInstantiate(&ctx->graph_exec, gph, nullptr, nullptr, 0));
            ctx->graph_seq = seq;
        }
        HIP_OR_FAIL(ctx, hipGraphLaunch(ctx->graph_exec, st));
    } else {
        for (size_t i = 0; i < seq.size(); ++i) {
            const auto &l = seq[i];
            if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ctx->events[2 * i], st));
            if (l.interp)
                HIP_OR_FAIL(ctx, ens::launch_interp(P, ctx->store_dtype, ctx->window, l.ia, st));
            else
                HIP_OR_FAIL(ctx, ens::launch_search(P, ctx->store_dtype, ctx->window, l.kind, l.dense, l.a, l.n_blocks, st));
            if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ctx->events[2 * i + 1], st));
        }
    }
    if (ens) {
        HIP_OR_FAIL(ctx, hipMemcpyAsync(out->params, final_params, pbytes, hipMemcpyDeviceToDevice, st));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(out->S, final_S, sbytes, hipMemcpyDeviceToDevice, st));
    }
    hipEvent_t ev_p0 = nullptr, ev_p1 = nullptr, ev_r0 = nullptr, ev_r1 = nullptr;
    if (timing) {
        while (ctx->events.size() < 2 * seq.size() + 4) {
            hipEvent_t e;
            HIP_OR_FAIL(ctx, hipEventCreate(&e));
            ctx->events.push_back(e);
        }
        ev_p0 = ctx->events[2 * seq.size()];
        ev_p1 = ctx->events[2 * seq.size() + 1];
        ev_r0 = ctx->events[2 * seq.size() + 2];
        ev_r1 = ctx->events[2 * seq.size() + 3];
    }
    const bool polish = de->polish_steps > 0;
    const bool rescore = de->rescore_fp64 && out->S64;
    if (polish) {
        ens::PolishArgs pa{};
        pa.sv = view_of(ctx, false);
        pa.cmp_out = ctx->cmp_out.as<int32_t>();
        pa.n_out = n_out;
        pa.t_begin = t_begin;
        pa.n_t = n_t;
        pa.lo_tab = ctx->lo_tab.as<float>();
        pa.hi_tab = ctx->hi_tab.as<float>();
        pa.params = out->params;
        pa.S = out->S;
        pa.S_pre = out->S_pre_polish;
        pa.steps = de->polish_steps;
        pa.lr = de->polish_lr;
        pa.counters = ctx->counters.as<unsigned long long>();
        if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev_p0, st));
        HIP_OR_FAIL(ctx, ens::launch_polish(P, ctx->store_dtype, ctx->window, pa, st));
        if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev_p1, st));
        ctx->stats.launches[2] = 1;
    } else if (out->S_pre_polish) {
        HIP_OR_FAIL(ctx, hipMemcpyAsync(out->S_pre_polish, out->S, sbytes, hipMemcpyDeviceToDevice, st));
    }
    if (rescore) {
        if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev_r0, st));
        HIP_OR_FAIL(ctx, ens::launch_eval64_grid(P, ctx->window, view_of(ctx, true), ctx->cmp_out.as<int32_t>(),
                                                 n_out, t_begin, n_t, out->params, out->S64, st));
        if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ev_r1, st));
        ctx->stats.launches[3] = 1;
        ctx->stats.evals[3] = n_s;
    }
    unsigned long long cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    HIP_OR_FAIL(ctx, hipMemcpyAsync(cnt, ctx->counters.p, sizeof cnt, hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    for (int k = 0; k < 3; ++k) {
        ctx->stats.evals[k] = static_cast<int64_t>(cnt[2 * k]);
        ctx->stats.sum_m[k] = static_cast<int64_t>(cnt[2 * k + 1]);
    }
    if (timing) {
        for (size_t i = 0; i < seq.size(); ++i) {
            float ms = 0.f;
            HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ctx->events[2 * i], ctx->events[2 * i + 1]));
            ctx->stats.device_ms[seq[i].kind] += ms;
        }
        float ms = 0.f;
        if (polish) {
            HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ev_p0, ev_p1));
            ctx->stats.device_ms[2] = ms;
        }
        if (rescore) {
            HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ev_r0, ev_r1));
            ctx->stats.device_ms[3] = ms;
        }
    }
    out->n_evals = static_cast<int64_t>(cnt[0] + cnt[2]);
    out->sum_m = static_cast<int64_t>(cnt[1] + cnt[3]);
    ctx->err.clear();
    return ENS_OK;
}

ens_status semblance_eval(ens_ctx *ctx, const ens_candidates *cands, float *S_out, int32_t *M_out)
{
    if (!ctx) return ENS_E_INVALID;
    if (!ctx->bound) return fail(ctx, ENS_E_STATE, "semblance_eval: call ens_bind first");
    if (!cands || !S_out) return fail(ctx, ENS_E_INVALID, "semblance_eval: null argument");
    ens_status chk = check_candidates(ctx, cands);
    if (chk != ENS_OK) return chk;
    ens::CandView cv{cands->n, cands->cmp, cands->t, cands->params};
    HIP_OR_FAIL(ctx, ens::launch_eval(ctx->op, ctx->store_dtype, ctx->window, view_of(ctx, false), cv, S_out, M_out,
                                      ctx->stream));
    ctx->err.clear();
    return ENS_OK;
}

ens_status semblance_eval64(ens_ctx *ctx, const ens_candidates *cands, double *S_out)
{
    if (!ctx) return ENS_E_INVALID;
    if (!ctx->bound) return fail(ctx, ENS_E_STATE, "semblance_eval64: call ens_bind first");
    if (!cands || !S_out) return fail(ctx, ENS_E_INVALID, "semblance_eval64: null argument");
    ens_status chk = check_candidates(ctx, cands);
    if (chk != ENS_OK) return chk;
    ens::CandView cv{cands->n, cands->cmp, cands->t, cands->params};
    HIP_OR_FAIL(ctx, ens::launch_eval64(ctx->op, ctx->window, view_of(ctx, true), cv, S_out, ctx->stream));
    ctx->err.clear();
    return ENS_OK;
}

ens_status semblance_backward(ens_ctx *ctx, const ens_candidates *cands, const float *dS, float *dparams_out)
{
    if (!ctx) return ENS_E_INVALID;
    if (!ctx->bound) return fail(ctx, ENS_E_STATE, "semblance_backward: call ens_bind first");
    if (!cands || !dS || !dparams_out) return fail(ctx, ENS_E_INVALID, "semblance_backward: null argument");
    ens_status chk = check_candidates(ctx, cands);
    if (chk != ENS_OK) return chk;
    ens::CandView cv{cands->n, cands->cmp, cands->t, cands->params};
    HIP_OR_FAIL(ctx, ens::launch_backward(ctx->op, ctx->store_dtype, ctx->window, view_of(ctx, false), cv, dS,
                                          dparams_out, ctx->stream));
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_stack(ens_ctx *ctx, const ens_t0_grid *grid, const float *params, float *stack_out, const float *S,
                     double *coherence_rms)
{
    if (!ctx) return ENS_E_INVALID;
    if (!ctx->bound) return fail(ctx, ENS_E_STATE, "ens_stack: call ens_bind first");
    if (!grid || !params || !stack_out) return fail(ctx, ENS_E_INVALID, "ens_stack: null argument");
    if (grid->struct_size < sizeof(ens_t0_grid)) return fail(ctx, ENS_E_INVALID, "ens_stack: struct_size too small");
    if ((S == nullptr) != (coherence_rms == nullptr))
        return fail(ctx, ENS_E_INVALID, "ens_stack: S and coherence_rms go together");
    const int32_t n_out = grid->cmp_out ? grid->n_cmp_out : ctx->n_cmp;
    if (n_out < 1) return fail(ctx, ENS_E_INVALID, "ens_stack: no output CMPs");
    if (grid->cmp_out)
        for (int32_t o = 0; o < n_out; ++o)
            if (grid->cmp_out[o] < 0 || grid->cmp_out[o] >= ctx->n_cmp)
                return fail(ctx, ENS_E_RANGE, "ens_stack: cmp_out[%d] = %d out of range", o, grid->cmp_out[o]);
    if (grid->t_begin < 0 || grid->t_end > ctx->nt || grid->t_begin >= grid->t_end)
        return fail(ctx, ENS_E_RANGE, "ens_stack: need 0 <= t_begin < t_end <= nt");
    const int32_t n_t = grid->t_end - grid->t_begin;
    hipStream_t st = ctx->stream;
    std::vector<int32_t> cmp_out(static_cast<size_t>(n_out));
    for (int32_t o = 0; o < n_out; ++o) cmp_out[o] = grid->cmp_out ? grid->cmp_out[o] : o;
    HIP_OR_FAIL(ctx, ctx->cmp_out.ensure(cmp_out.size() * sizeof(int32_t)));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->cmp_out.p, cmp_out.data(), cmp_out.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(ctx, ens::launch_stack(ctx->op, view_of(ctx, true), ctx->cmp_out.as<int32_t>(), n_out,
                                       grid->t_begin, n_t, params, stack_out, st));
    if (S) {
        HIP_OR_FAIL(ctx, ctx->flag.ensure(sizeof(double)));
        double *dev = static_cast<double *>(ctx->flag.p);
        HIP_OR_FAIL(ctx, ens::launch_rms(S, static_cast<int64_t>(n_out) * n_t, dev, st));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(coherence_rms, dev, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    } else {
        // the host-side cmp_out copy must outlive the asynchronous upload
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    }
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_stack_noalloc(ens_ctx *ctx, const ens_t0_grid *grid, const float *params, float *stack_out,
                             const float *S, double *coherence_rms)
{
    if (!ctx) return ENS_E_INVALID;
    if (!ctx->bound) return fail(ctx, ENS_E_STATE, "ens_stack_noalloc: call ens_bind first");
    if (!grid || !params || !stack_out) return fail(ctx, ENS_E_INVALID, "ens_stack_noalloc: null argument");
    if (grid->struct_size < sizeof(ens_t0_grid))
        return fail(ctx, ENS_E_INVALID, "ens_stack_noalloc: struct_size too small");
    if ((S == nullptr) != (coherence_rms == nullptr))
        return fail(ctx, ENS_E_INVALID, "ens_stack_noalloc: S and coherence_rms go together");
    const int32_t n_out = grid->cmp_out ? grid->n_cmp_out : ctx->n_cmp;
    if (n_out < 1) return fail(ctx, ENS_E_INVALID, "ens_stack_noalloc: no output CMPs");
    if (n_out > NOALLOC_MAX_CMPS)
        return fail(ctx, ENS_E_RANGE, "ens_stack_noalloc: at most %d output CMPs (got %d); use ens_stack",
                    NOALLOC_MAX_CMPS, n_out);
    if (grid->cmp_out)
        for (int32_t o = 0; o < n_out; ++o)
            if (grid->cmp_out[o] < 0 || grid->cmp_out[o] >= ctx->n_cmp)
                return fail(ctx, ENS_E_RANGE, "ens_stack_noalloc: cmp_out[%d] = %d out of range", o,
                            grid->cmp_out[o]);
    if (grid->t_begin < 0 || grid->t_end > ctx->nt || grid->t_begin >= grid->t_end)
        return fail(ctx, ENS_E_RANGE, "ens_stack_noalloc: need 0 <= t_begin < t_end <= nt");
    if (!ctx->scratch)
        return fail(ctx, ENS_E_HIP, "ens_stack_noalloc: no device address for the scratch array: %s",
                    hipGetErrorString(ctx->scratch_err));
    const int32_t n_t = grid->t_end - grid->t_begin;
    hipStream_t st = ctx->stream;
    unsigned char *base = static_cast<unsigned char *>(ctx->scratch);
    double *rms_dev = reinterpret_cast<double *>(base);
    int32_t *cmp_dev = reinterpret_cast<int32_t *>(base + NOALLOC_RMS_BYTES);
    // the whole list is written before the stack reads it; nothing carries over between calls
    if (grid->cmp_out)
        HIP_OR_FAIL(ctx, hipMemcpyAsync(cmp_dev, grid->cmp_out, sizeof(int32_t) * n_out, hipMemcpyHostToDevice, st));
    else
        HIP_OR_FAIL(ctx, launch_iota(cmp_dev, n_out, st));
    HIP_OR_FAIL(ctx, ens::launch_stack(ctx->op, view_of(ctx, true), cmp_dev, n_out, grid->t_begin, n_t, params,
                                       stack_out, st));
    if (S) {
        HIP_OR_FAIL(ctx, ens::launch_rms(S, static_cast<int64_t>(n_out) * n_t, rms_dev, st));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(coherence_rms, rms_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    // the caller's host list and the returned RMS are settled before returning
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_philox(ens_ctx *ctx, int64_t n, const uint64_t *counters, const uint64_t *key, uint64_t *out)
{
    if (!ctx) return ENS_E_INVALID;
    if (n < 0 || (n > 0 && (!counters || !key || !out))) return fail(ctx, ENS_E_INVALID, "ens_philox: bad argument");
    HIP_OR_FAIL(ctx, ens::launch_philox(n, counters, key, out, ctx->stream));
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_de_trial(ens_ctx *ctx, int32_t n_pop, int32_t np, int32_t P, const float *pop, const float *S,
                        const uint64_t *words, float F, float CR, const float *lo, const float *hi, float *trial)
{
    if (!ctx) return ENS_E_INVALID;
    if (n_pop < 0 || (n_pop > 0 && (!pop || !S || !words || !lo || !hi || !trial)))
        return fail(ctx, ENS_E_INVALID, "ens_de_trial: bad argument");
    if (P != 1 && P != 3) return fail(ctx, ENS_E_INVALID, "ens_de_trial: P must be 1 or 3");
    if (np < 4 || np > ENS_MAX_POP) return fail(ctx, ENS_E_RANGE, "ens_de_trial: np must lie in [4, 64]");
    if (!finite(F) || !(CR >= 0.f && CR <= 1.f)) return fail(ctx, ENS_E_RANGE, "ens_de_trial: bad F or CR");
    const uint64_t thr = static_cast<uint64_t>(std::ceil(static_cast<double>(CR) * 4294967296.0));
    HIP_OR_FAIL(ctx, ens::launch_de_trial(n_pop, np, P, pop, S, words, F, thr, lo, hi, trial, ctx->stream));
    ctx->err.clear();
    return ENS_OK;
}

ens_status ens_jade_draws(ens_ctx *ctx, int64_t n, const uint64_t *words, double mu_cr, double mu_f, int32_t np,
                          int32_t *k_cr, int32_t *k_f, int32_t *a_idx)
{
    if (!ctx) return ENS_E_INVALID;
    if (n < 0 || (n > 0 && (!words || !k_cr || !k_f || !a_idx)))
        return fail(ctx, ENS_E_INVALID, "ens_jade_draws: bad argument");
    if (np < 4 || np > ENS_MAX_POP) return fail(ctx, ENS_E_RANGE, "ens_jade_draws: np must lie in [4, 64]");
    if (!finite(mu_cr) || !finite(mu_f)) return fail(ctx, ENS_E_RANGE, "ens_jade_draws: means must be finite");
    HIP_OR_FAIL(ctx, ens::launch_jade_draws(n, words, mu_cr, mu_f, np, k_cr, k_f, a_idx, ctx->stream));
    ctx->err.clear();
    return ENS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------

namespace {

__global__ void k_iota(int32_t *__restrict__ out, int32_t n)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) out[i] = i;
}

hipError_t launch_iota(int32_t *out, int32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, out, n);
    return hipGetLastError();
}

__global__ void k_check_candidates(int64_t n, const int32_t *__restrict__ cmp, const int32_t *__restrict__ t,
                                   int32_t n_cmp, int32_t nt, int32_t *__restrict__ flag)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cmp[i] < 0 || cmp[i] >= n_cmp || t[i] < 0 || t[i] >= nt) atomicOr(flag, 1);
}

ens_status check_candidates(ens_ctx *ctx, const ens_candidates *c)
{
    if (c->struct_size < sizeof(ens_candidates)) return fail(ctx, ENS_E_INVALID, "ens_candidates: struct_size too small");
    if (c->n < 0) return fail(ctx, ENS_E_INVALID, "ens_candidates: n < 0");
    if (c->n == 0) return ENS_OK;
    if (!c->cmp || !c->t || !c->params) return fail(ctx, ENS_E_INVALID, "ens_candidates: null array");
    HIP_OR_FAIL(ctx, ctx->flag.ensure(sizeof(int32_t)));
    HIP_OR_FAIL(ctx, hipMemsetAsync(ctx->flag.p, 0, sizeof(int32_t), ctx->stream));
    const unsigned blocks = static_cast<unsigned>((c->n + 255) / 256);
    hipLaunchKernelGGL(k_check_candidates, dim3(blocks), dim3(256), 0, ctx->stream, c->n, c->cmp, c->t, ctx->n_cmp,
                       ctx->nt, ctx->flag.as<int32_t>());
    HIP_OR_FAIL(ctx, hipGetLastError());
    int32_t flag = 0;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&flag, ctx->flag.p, sizeof flag, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    if (flag) return fail(ctx, ENS_E_RANGE, "ens_candidates: a CMP or time index is out of range");
    return ENS_OK;
}

}  // namespace
