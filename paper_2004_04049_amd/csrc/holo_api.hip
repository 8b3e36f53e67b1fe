// holo_api.hip -- host side of the C ABI declared in include/holo.h:
// argument validation, LUT tables, per-device twiddle tables, per-stream
// workspaces and the launch sequences of the OSPR, GS and reconstruction
// paths.  All arithmetic on image data runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <shared_mutex>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/holo.h"
#include "cnn.hpp"
#include "kernels.hpp"

struct holo_cnn {
    int device = 0;
    holo::CnnLayout lay;
    holo::CnnBuffers b{};
    size_t img_px = 0;          // capacity of the per-image buffers (pixels)
    int img_rows = 0;           // rows the gradient partials are sized for
    int step = 0;               // Adam steps taken
    float2* ph = nullptr;       // phasor scratch for training
};

struct holo_lut {
    int device;
    int kind;                    // holo::SRC_*
    uint64_t id;                 // unique per handle (graph keys), never reused
    uint64_t n_lut;              // as requested (0 = flat); PRNG: UINT64_MAX (unbounded); MSEQ: 2^31 - 1
    uint32_t n_dev;              // pool length of the cyclic kinds (>= 1)
    uint64_t seed;
    std::vector<double> phases;  // FP64 phases, host copy (TABLE)
    std::vector<uint8_t> host_codes;   // CODES8: the codes, host copy
    float2* dev = nullptr;       // TABLE: n_dev FP32 unit phasors; CODES8, MSEQ: the 256 code phasors
    uint8_t* codes = nullptr;    // CODES8: n_dev codes
    uint32_t* mseq = nullptr;    // MSEQ: x^(2^j) for j < 31, S_0, then [12][4][256] jump tables (strides 2^0..2^11)
};

namespace holo {
namespace {

thread_local std::string g_err;

holo_status fail(holo_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(HOLO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool pow2_in_range(int64_t n) { return n >= 16 && n <= 2048 && (n & (n - 1)) == 0; }

// Failure and debug hooks, read from the environment at each use so that a
// caller (or a test) can switch them between calls:
//   HOLO_WORKSPACE_CAP=<bytes>  a workspace request above it fails with
//                               HOLO_ENOMEM (as a failed allocation would);
//   HOLO_DEBUG_FAIL=device      every kernel or graph launch fails with
//                               HOLO_EDEVICE before anything is enqueued;
//   HOLO_DEBUG_POISON=1         each workspace handed to a call is first
//                               filled with 0xFF bytes (a NaN in FP32 and
//                               FP64), so a kernel that reads scratch it did
//                               not write shows up in the results.
size_t env_workspace_cap()
{
    const char* v = getenv("HOLO_WORKSPACE_CAP");
    if (!v || !*v) return SIZE_MAX;
    char* end = nullptr;
    const unsigned long long c = strtoull(v, &end, 10);
    return (end && *end == 0) ? (size_t)c : SIZE_MAX;
}
bool env_is(const char* name, const char* value)
{
    const char* v = getenv(name);
    return v && strcmp(v, value) == 0;
}
bool debug_fail_device() { return env_is("HOLO_DEBUG_FAIL", "device"); }
#define DEBUG_FAIL_CHECK(what) \
    do { \
        if (debug_fail_device()) return fail(HOLO_EDEVICE, "%s: launch failed (forced by HOLO_DEBUG_FAIL=device)", what); \
    } while (0)

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): golden-gamma increment and
// the variant-13 finaliser.
uint64_t splitmix64(uint64_t& s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Phase sources (phase_src.hpp): host side.
// ---------------------------------------------------------------------------
std::atomic<uint64_t> g_lut_ids{1};

// GF(2)[x] / (x^31 + x^3 + 1)
uint32_t gf_mul_host(uint32_t a, uint32_t b)
{
    uint64_t acc = 0;
    for (int i = 0; i < 31; ++i)
        if ((b >> i) & 1u) acc ^= (uint64_t)a << i;
    for (int r = 0; r < 2; ++r) {
        const uint64_t hi = acc >> 31;
        acc = (acc & kMseqM) ^ (hi << 3) ^ hi;
    }
    return (uint32_t)acc;
}
uint32_t gf_xpow_host(uint64_t e)   // x^e
{
    e %= kMseqM;
    uint32_t r = 1, b = 2;
    for (; e; e >>= 1) {
        if (e & 1) r = gf_mul_host(r, b);
        b = gf_mul_host(b, b);
    }
    return r;
}

// Pool position `v` as the kernels take it: mod the pool length for the
// cyclic kinds, unchanged (mod 2^64) for the counter-based PRNG.
uint64_t lut_wrap(const holo_lut* l, uint64_t v) { return l->kind == SRC_PRNG ? v : v % l->n_dev; }

PhaseSrc make_src(const holo_lut* l, const uint32_t* rows)
{
    PhaseSrc p{};
    p.kind = l->kind;
    p.tab = l->dev;
    p.codes = l->codes;
    p.jump = l->mseq ? l->mseq + 32 : nullptr;
    p.rows = rows;
    p.seed = l->seed;
    p.n = l->n_dev;
    return p;
}

struct Workspace {
    void* base = nullptr;
    size_t cap = 0;
};

struct DeviceState {
    std::map<int, float2*> twiddles;                   // length -> W_N^k table
    std::map<int, void*> dftops;                       // precision -> DFT-matrix operand table
    std::map<hipStream_t, Workspace> workspaces;       // per stream
};

std::mutex g_mu;
std::map<int, DeviceState> g_dev;

// Twiddle table W_N^k = exp(-2*pi*i*k/N) for the current device, generated in
// FP64 on the device at first use.
holo_status get_twiddles(int device, int n, hipStream_t s, const float2** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState& d = g_dev[device];
    auto it = d.twiddles.find(n);
    if (it != d.twiddles.end()) {
        *out = it->second;
        return HOLO_OK;
    }
    float2* tw = nullptr;
    if (hipMalloc(&tw, sizeof(float2) * (size_t)n) != hipSuccess) return fail(HOLO_ENOMEM, "twiddle table (%d)", n);
    HIP_TRY(launch_twiddle_gen(tw, n, s));
    HIP_TRY(hipStreamSynchronize(s));
    d.twiddles[n] = tw;
    *out = tw;
    return HOLO_OK;
}

// DFT-matrix operand table of the matrix-core stages for `prec`, generated
// in FP64 on the device at first use.
holo_status get_dftop(int device, int prec, hipStream_t s, const void** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState& d = g_dev[device];
    auto it = d.dftops.find(prec);
    if (it != d.dftops.end()) {
        *out = it->second;
        return HOLO_OK;
    }
    void* t = nullptr;
    if (hipMalloc(&t, kDftOpElems * sizeof(uint16_t)) != hipSuccess)
        return fail(HOLO_ENOMEM, "DFT operand table");
    HIP_TRY(launch_dft_operand_gen((uint16_t*)t, prec, s));
    HIP_TRY(hipStreamSynchronize(s));
    d.dftops[prec] = t;
    *out = t;
    return HOLO_OK;
}

// Scratch of at least `bytes` for (device, stream); grows by reallocation
// after the stream has drained (the only user of the old buffer).
holo_status get_workspace(int device, hipStream_t s, size_t bytes, void** out)
{
    const size_t ws_cap = env_workspace_cap();
    if (bytes > ws_cap)
        return fail(HOLO_ENOMEM, "workspace of %zu bytes exceeds HOLO_WORKSPACE_CAP=%zu", bytes, ws_cap);
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace& w = g_dev[device].workspaces[s];
    if (w.cap < bytes) {
        if (w.base) {
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipFree(w.base));
            w.base = nullptr;
            w.cap = 0;
        }
        size_t cap = bytes + (bytes >> 3);
        if (hipMalloc(&w.base, cap) != hipSuccess) {
            (void)hipGetLastError();
            w.base = nullptr;
            return fail(HOLO_ENOMEM, "workspace of %zu bytes", cap);
        }
        w.cap = cap;
    }
    if (env_is("HOLO_DEBUG_POISON", "1")) HIP_TRY(hipMemsetAsync(w.base, 0xFF, bytes, s));
    *out = w.base;
    return HOLO_OK;
}

// Carves aligned sub-buffers out of one workspace.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

// Kernel timing: when enabled, each launch is bracketed by a pair of HIP
// events recorded on the launch stream; durations are folded into per-kernel
// totals when read.  Off by default (no events are recorded).
struct ProfPending {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfPending> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
std::map<std::string, std::pair<double, int64_t>> g_prof_tot;

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Set while an entry point that must not create events runs on this thread.
thread_local bool t_prof_suppress = false;

struct ProfScope {
    const char* name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* n, hipStream_t st) : name(n), s(st)
    {
        if (t_prof_suppress) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on) return;
        a = prof_event();
        b = prof_event();
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~ProfScope()
    {
        if (!a || !b) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_pending.push_back({name, a, b});
    }
};

void prof_drain()
{
    for (auto& p : g_prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& t = g_prof_tot[p.name];
            t.first += ms;
            t.second += 1;
        }
        g_prof_pool.push_back(p.a);
        g_prof_pool.push_back(p.b);
    }
    g_prof_pending.clear();
}

#define LAUNCH(name, s, expr)           \
    do {                                \
        DEBUG_FAIL_CHECK(name);         \
        ProfScope ps_(name, s);         \
        HIP_TRY(expr);                  \
    } while (0)

holo_status check_lut(const holo_lut* lut, int device)
{
    if (!lut) return fail(HOLO_EINVAL, "lut is NULL");
    if (lut->device != device)
        return fail(HOLO_EINVAL, "lut lives on device %d, current device is %d", lut->device, device);
    return HOLO_OK;
}

holo_status copy_out(double* dst, const double* dev_src, size_t n, uint32_t flags, hipStream_t s)
{
    if (!dst) return HOLO_OK;
    if (flags & HOLO_F_NMSE_DEVICE) {
        HIP_TRY(hipMemcpyAsync(dst, dev_src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        HIP_TRY(hipMemcpyAsync(dst, dev_src, n * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return HOLO_OK;
}

LaunchCfg default_cfg() { return LaunchCfg{}; }

// ---------------------------------------------------------------------------
// Plans: launch shapes per (path, nx, ny, n_sf), defaulting to the kernels'
// built-in heuristics; filled by the autotuner or by holo_plan_set/load.
// ---------------------------------------------------------------------------
enum { PLAN_OSPR = 0, PLAN_GS = 1 };
struct PlanKey {
    int kind;
    int64_t nx, ny;
    int n_sf;
    bool operator<(const PlanKey& o) const
    {
        if (kind != o.kind) return kind < o.kind;
        if (nx != o.nx) return nx < o.nx;
        if (ny != o.ny) return ny < o.ny;
        return n_sf < o.n_sf;
    }
};
std::mutex g_plan_mu;
std::map<PlanKey, LaunchCfg> g_plans;

// The plan of (kind, nx, ny, n_sf); for OSPR without one of its own, the
// size's plan stored under n_sf = 0 (every sub-frame count); else defaults.
LaunchCfg plan_get(int kind, int64_t nx, int64_t ny, int n_sf)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(PlanKey{kind, nx, ny, kind == PLAN_GS ? 1 : n_sf});
    if (it == g_plans.end() && kind == PLAN_OSPR) it = g_plans.find(PlanKey{kind, nx, ny, 0});
    return it == g_plans.end() ? LaunchCfg{} : it->second;
}

void plan_put(int kind, int64_t nx, int64_t ny, int n_sf, const LaunchCfg& c)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[PlanKey{kind, nx, ny, kind == PLAN_GS ? 1 : n_sf}] = c;
}

// ---------------------------------------------------------------------------
// OSPR frame: K1 -> K2 -> K3 -> K4 on stream s with launch shapes `cfg`.
// ---------------------------------------------------------------------------
// Workspace of one OSPR frame: intermediate planes and reduction scratch.
struct OsprLayout {
    size_t o_x1, o_x2, o_part, o_nm, o_rs, bytes;
    int chunk;
};

// n_fields randomised fields per frame: n_sf, or n_sf/2 in pair mode
int ospr_fields(int n_sf, int mode) { return mode == OSPR_PAIRS ? n_sf / 2 : n_sf; }

OsprLayout ospr_layout(int64_t nx, int64_t ny, int n_sf, const LaunchCfg& cfg, int mode = OSPR_BINARY)
{
    OsprLayout l;
    const size_t pitch = (size_t)row_pitch((int)nx, cfg);
    const size_t plane = (size_t)ny * pitch;
    // half spectra of binary sub-frames (Hermitian), full spectra of 8-level ones
    const size_t nspec = (size_t)(mode == OSPR_LEVELS8 ? ny : ny / 2 + 1) * pitch;
    const int n_fields = ospr_fields(n_sf, mode);
    // Sub-frames are generated in chunks that reuse one set of intermediate
    // planes, so a chunk's planes can stay in the last-level cache between the
    // row pass that writes them and the column pass that reads them.  (Running
    // chunks concurrently on two streams was measured slower: the doubled
    // working set no longer fits that cache.)
    l.chunk = (cfg.chunk > 0 && cfg.chunk < n_fields) ? cfg.chunk : n_fields;
    Carver cv;
    l.o_x1 = cv.take(sizeof(float2) * plane * l.chunk);
    l.o_x2 = cv.take(sizeof(float2) * nspec * n_sf);
    l.o_part = cv.take(sizeof(double) * 5 * (size_t)ny);
    l.o_nm = cv.take(sizeof(double) * 2);
    l.o_rs = cv.take(sizeof(uint32_t) * (size_t)n_fields * (size_t)ny);   // M-sequence row states
    l.bytes = cv.off;
    return l;
}

// Device work of one OSPR frame on stream s, scratch at `b` (layout `l`),
// {NMSE, NMSE_sym} to device `nm_out`.  The frame starts in the pool at
// c0 + *c0_base (both reduced by lut_wrap; c0_base may be NULL).
holo_status ospr_enqueue(const float* target, int64_t nx, int64_t ny, int n_sf, const holo_lut* lut, uint64_t c0,
                         const uint64_t* c0_base, void* holo_out, float* recon, double* nm_out,
                         const float2* tw_x, const float2* tw_y, char* b, const OsprLayout& l, hipStream_t s,
                         const LaunchCfg& cfg, int mode = OSPR_BINARY)
{
    const size_t pitch = (size_t)row_pitch((int)nx, cfg);
    const bool half = mode != OSPR_LEVELS8;
    const size_t nspec = (size_t)(half ? ny / 2 + 1 : ny) * pitch;
    const int n_fields = ospr_fields(n_sf, mode);
    uint32_t* holo_bits = (uint32_t*)holo_out;
    float2* x1 = (float2*)(b + l.o_x1);
    float2* x2 = (float2*)(b + l.o_x2);
    double* part = (double*)(b + l.o_part);
    uint32_t* rs = (uint32_t*)(b + l.o_rs);
    const size_t words = (size_t)nx * (size_t)ny / 32;
    if (lut->kind == SRC_MSEQ)
        LAUNCH("mseq_rows", s, launch_mseq_rows(lut->mseq, c0, c0_base, (int)nx, (int)ny, n_fields, rs, s));
    for (int k0 = 0; k0 < n_fields; k0 += l.chunk) {
        const int ns = n_fields - k0 < l.chunk ? n_fields - k0 : l.chunk;
        const uint64_t ck = lut_wrap(lut, c0 + (uint64_t)k0 * (uint64_t)(nx * ny));
        const PhaseSrc src = make_src(lut, rs + (size_t)k0 * (size_t)ny);
        // binary frames transform only the Hermitian part of R
        if (mode == OSPR_BINARY)
            LAUNCH("ospr_rows", s, launch_ospr_rows_h(target, (int)nx, (int)ny, ns, src, ck, c0_base, x1, tw_x, cfg, s));
        else
            LAUNCH("ospr_rows", s, launch_ospr_rows(target, (int)nx, (int)ny, ns, src, ck, c0_base, x1, tw_x, cfg, s));
        if (mode == OSPR_BINARY)
            LAUNCH("ospr_cols", s, launch_ospr_cols(x1, (int)nx, (int)ny, ns, holo_bits + (size_t)k0 * words,
                                                    x2 + (size_t)k0 * nspec, tw_y, cfg, s));
        else if (mode == OSPR_PAIRS)
            LAUNCH("ospr_cols", s, launch_ospr_cols_mode(mode, x1, (int)nx, (int)ny, ns,
                                                         holo_bits + (size_t)(2 * k0) * words,
                                                         x2 + (size_t)(2 * k0) * nspec, tw_y, cfg, s));
        else
            LAUNCH("ospr_cols", s, launch_ospr_cols_mode(mode, x1, (int)nx, (int)ny, ns,
                                                         (uint8_t*)holo_out + (size_t)k0 * (size_t)(nx * ny),
                                                         x2 + (size_t)k0 * nspec, tw_y, cfg, s));
    }
    LAUNCH("recon_rows", s, launch_recon_rows(x2, (int)nx, (int)ny, n_sf, half, target, recon, part, tw_x, cfg, s));
    LAUNCH("nmse_finalize", s, launch_nmse_finalize(part, (int)(half ? ny / 2 + 1 : ny), nm_out, s));
    return HOLO_OK;
}

holo_status ospr_run(int device, const float* target, int64_t nx, int64_t ny, int n_sf, const holo_lut* lut,
                     uint64_t cursor, void* holo_out, float* recon, double* nmse2, uint32_t flags,
                     hipStream_t s, const LaunchCfg& cfg, int mode = OSPR_BINARY)
{
    holo_status st;
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)ny, s, &tw_y))) return st;
    const OsprLayout l = ospr_layout(nx, ny, n_sf, cfg, mode);
    void* ws;
    if ((st = get_workspace(device, s, l.bytes, &ws))) return st;
    char* b = (char*)ws;
    // a device destination takes the result straight from the kernel
    const bool direct = nmse2 && (flags & HOLO_F_NMSE_DEVICE);
    double* nm = direct ? nmse2 : (double*)(b + l.o_nm);
    if ((st = ospr_enqueue(target, nx, ny, n_sf, lut, lut_wrap(lut, cursor), nullptr, holo_out, recon, nm, tw_x,
                           tw_y, b, l, s, cfg, mode)))
        return st;
    return direct ? HOLO_OK : copy_out(nmse2, nm, 2, flags, s);
}

// ---------------------------------------------------------------------------
// GS: the device work of one call is a fixed sequence of 2*n_iter + 4..7
// launches.  Unless kernel timing is on, it is captured once into a HIP graph
// per (stream, arguments, workspace, plan) and replayed, which removes the
// per-launch host cost from the iteration loop.
// ---------------------------------------------------------------------------
struct GsArgs {
    const float* target;
    int64_t nx, ny;
    int n_iter;
    const holo_lut* lut;
    uint64_t cursor;
    const float* init;
    float* field;
    uint8_t* codes;
    double *nmse, *err, *final2;
    float* recon;
    uint32_t flags;
};

// Stream-ordered store of one 64-bit value (kernel argument, so no host
// buffer has to outlive the call).
__global__ void k_set_u64(uint64_t* p, uint64_t v) { *p = v; }

// Graph capture and the other threads' calls.  This HIP runtime can
// invalidate a stream capture when another host thread launches work or
// allocates meanwhile, whatever the capture mode, so the library's own calls
// exclude each other from captures: every call that enqueues GPU work holds
// g_call_mu shared (CallGuard, outermost call of a thread only), and a capture
// holds it exclusively (CaptureSection, which first gives up this thread's
// shared hold and takes it back afterwards).  Work that other code enqueues
// meanwhile is outside this protection.
std::shared_mutex g_call_mu;
thread_local int t_call_depth = 0;
thread_local bool t_capturing = false;

struct CallGuard {
    bool locked = false;
    CallGuard()
    {
        if (t_call_depth++ == 0 && !t_capturing) {
            g_call_mu.lock_shared();
            locked = true;
        }
    }
    ~CallGuard()
    {
        --t_call_depth;
        if (locked) g_call_mu.unlock_shared();
    }
    CallGuard(const CallGuard&) = delete;
    CallGuard& operator=(const CallGuard&) = delete;
};

struct CaptureSection {
    bool had_shared;
    CaptureSection() : had_shared(t_call_depth > 0 && !t_capturing)
    {
        if (had_shared) g_call_mu.unlock_shared();
        g_call_mu.lock();
        t_capturing = true;
    }
    ~CaptureSection()
    {
        t_capturing = false;
        g_call_mu.unlock();
        if (had_shared) g_call_mu.lock_shared();
    }
    CaptureSection(const CaptureSection&) = delete;
    CaptureSection& operator=(const CaptureSection&) = delete;
};

struct GraphKey {
    std::vector<uintptr_t> k;
    bool operator<(const GraphKey& o) const { return k < o.k; }
};
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;
std::map<GraphKey, void*> g_graph_bufs;   // device tables a graph's kernels read, freed with the graph
std::map<GraphKey, hipStream_t> g_graph_streams;   // the stream each graph is launched on (part of its key)
std::vector<GraphKey> g_graph_order;
bool g_use_graphs = true;

// Records a new graph for `key`, launched on stream s, and keeps at most 32:
// the oldest is destroyed, with its device table, once its own stream has
// drained (which may be another stream than s).  Called with g_graph_mu held.
void graph_insert_locked(const GraphKey& key, hipGraphExec_t exec, void* dtab, hipStream_t s)
{
    g_graphs[key] = exec;
    if (dtab) g_graph_bufs[key] = dtab;
    g_graph_streams[key] = s;
    g_graph_order.push_back(key);
    if (g_graph_order.size() <= 32) return;
    const GraphKey k0 = g_graph_order.front();
    g_graph_order.erase(g_graph_order.begin());
    auto os = g_graph_streams.find(k0);
    if (os != g_graph_streams.end()) {
        (void)hipStreamSynchronize(os->second);
        g_graph_streams.erase(os);
    }
    auto old = g_graphs.find(k0);
    if (old != g_graphs.end()) {
        (void)hipGraphExecDestroy(old->second);
        g_graphs.erase(old);
    }
    auto ob = g_graph_bufs.find(k0);
    if (ob != g_graph_bufs.end()) {
        (void)hipFree(ob->second);
        g_graph_bufs.erase(ob);
    }
}

// Launches the cached graph for `key` on s, if there is one (*launched), with
// the cache lock held so that no other thread's insertion evicts it between
// the lookup and the launch.
holo_status graph_launch_cached(const GraphKey& key, hipStream_t s, bool* launched)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    *launched = it != g_graphs.end();
    if (!*launched) return HOLO_OK;
    DEBUG_FAIL_CHECK("graph");
    HIP_TRY(hipGraphLaunch(it->second, s));
    return HOLO_OK;
}

// Caches a newly instantiated graph (with its device table) and launches it,
// under the cache lock.  If another thread cached the same key meanwhile, its
// graph is launched and the new one (never launched) is dropped.
holo_status graph_insert_launch(const GraphKey& key, hipGraphExec_t exec, void* dtab, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
        (void)hipGraphExecDestroy(exec);
        if (dtab) (void)hipFree(dtab);
        exec = it->second;
    } else {
        graph_insert_locked(key, exec, dtab, s);
    }
    DEBUG_FAIL_CHECK("graph");
    HIP_TRY(hipGraphLaunch(exec, s));
    return HOLO_OK;
}

// Scratch of one GS call, carved from one buffer.
struct GsLayout {
    size_t o_state, o_field, o_pinit, o_piter, o_consts, o_nm, o_er, o_x2, o_p5, o_f2, o_rs, o_cur, bytes;
};

GsLayout gs_layout(const GsArgs& a, const LaunchCfg& cfg)
{
    const size_t npix = (size_t)a.nx * (size_t)a.ny;
    const size_t pitched = (size_t)a.ny * (size_t)row_pitch((int)a.nx, cfg);
    const int ny = (int)a.ny;
    GsLayout L;
    Carver cv;
    L.o_state = cv.take(sizeof(float2) * pitched);
    L.o_field = cv.take(a.field ? 0 : sizeof(float2) * npix);
    L.o_pinit = cv.take(sizeof(double) * 2 * ny);
    L.o_piter = cv.take(sizeof(double) * 3 * ny * (size_t)a.n_iter);
    L.o_consts = cv.take(sizeof(GsConsts));
    L.o_nm = cv.take(sizeof(double) * a.n_iter);
    L.o_er = cv.take(sizeof(double) * a.n_iter);
    L.o_x2 = cv.take(a.codes ? sizeof(float2) * pitched : 0);
    L.o_p5 = cv.take(sizeof(double) * 5 * ny);
    L.o_f2 = cv.take(sizeof(double) * 2);
    L.o_rs = cv.take(sizeof(uint32_t) * ny);   // M-sequence row states
    L.o_cur = cv.take(sizeof(uint64_t));       // pool start of this call
    L.bytes = cv.off;
    return L;
}

holo_status gs_enqueue(const GsArgs& a, hipStream_t s, const LaunchCfg& cfg, const float2* tw_x, const float2* tw_y,
                       char* b, const GsLayout& L)
{
    const size_t o_state = L.o_state, o_field = L.o_field, o_pinit = L.o_pinit, o_piter = L.o_piter,
                 o_consts = L.o_consts, o_nm = L.o_nm, o_er = L.o_er, o_x2 = L.o_x2, o_p5 = L.o_p5,
                 o_f2 = L.o_f2, o_rs = L.o_rs, o_cur = L.o_cur;
    const int inx = (int)a.nx, iny = (int)a.ny;
    float2* state = (float2*)(b + o_state);
    float2* fout = a.field ? (float2*)a.field : (float2*)(b + o_field);
    double* pinit = (double*)(b + o_pinit);
    double* piter = (double*)(b + o_piter);
    GsConsts* consts = (GsConsts*)(b + o_consts);
    double* nm = (double*)(b + o_nm);
    double* er = (double*)(b + o_er);
    // the pool start comes from a device word written before the launches
    // (gs_run), so a captured graph serves every cursor
    const bool use_lut = a.init == nullptr;
    const uint64_t* dcur = (const uint64_t*)(b + o_cur);
    PhaseSrc src{};
    src.n = 1;
    if (use_lut) {
        uint32_t* rs = (uint32_t*)(b + o_rs);
        src = make_src(a.lut, rs);
        if (a.lut->kind == SRC_MSEQ)
            LAUNCH("mseq_rows", s, launch_mseq_rows(a.lut->mseq, 0, dcur, inx, iny, 1, rs, s));
    }
    LAUNCH("gs_rows", s, launch_gs_rows(GS_INIT, a.target, inx, iny, src, 0, use_lut ? dcur : nullptr,
                                        (const float2*)a.init, state, nullptr, pinit, consts, tw_x, cfg, s));
    LAUNCH("gs_consts", s, launch_gs_consts(pinit, iny, inx, consts, s));
    for (int it = 0; it < a.n_iter; ++it) {
        const bool last = it == a.n_iter - 1;
        LAUNCH("gs_cols", s, launch_gs_cols(state, inx, iny, last ? a.codes : nullptr, tw_y, cfg, s));
        LAUNCH("gs_rows", s, launch_gs_rows(last ? GS_FINAL : GS_ITER, a.target, inx, iny, src, 0, nullptr,
                                            nullptr, state, fout, piter + (size_t)it * 3 * iny, consts, tw_x, cfg,
                                            s));
    }
    LAUNCH("gs_finalize", s, launch_gs_finalize(piter, a.n_iter, iny, consts, nm, er, s));
    if (a.codes && (a.final2 || a.recon)) {
        float2* x2 = (float2*)(b + o_x2);
        double* p5 = (double*)(b + o_p5);
        double* f2 = (double*)(b + o_f2);
        LAUNCH("recon_cols", s, launch_recon_cols(a.codes, 8, inx, iny, 1, x2, tw_y, cfg, s));
        LAUNCH("recon_rows", s, launch_recon_rows(x2, inx, iny, 1, false, a.target, a.recon, p5, tw_x, cfg, s));
        LAUNCH("nmse_finalize", s, launch_nmse_finalize(p5, iny, f2, s));
    }
    return HOLO_OK;
}

holo_status gs_run(int device, const GsArgs& a, hipStream_t s, const LaunchCfg& cfg)
{
    holo_status st;
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)a.nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)a.ny, s, &tw_y))) return st;
    const int n_iter = a.n_iter;
    const GsLayout L = gs_layout(a, cfg);
    void* ws;
    if ((st = get_workspace(device, s, L.bytes, &ws))) return st;
    char* b = (char*)ws;
    if (!a.init) {
        hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, (uint64_t*)(b + L.o_cur), lut_wrap(a.lut, a.cursor));
        HIP_TRY(hipGetLastError());
    }

    bool prof_on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof_on = g_prof_on;
    }
    // the legacy default stream cannot be captured: launch directly there
    if (!g_use_graphs || prof_on || s == nullptr) {
        if ((st = gs_enqueue(a, s, cfg, tw_x, tw_y, b, L))) return st;
    } else {
        GraphKey key{{(uintptr_t)device, (uintptr_t)s, (uintptr_t)a.target, (uintptr_t)a.nx, (uintptr_t)a.ny,
                      (uintptr_t)a.n_iter, (uintptr_t)(a.init ? 0 : a.lut->id), (uintptr_t)a.init,
                      (uintptr_t)a.field,
                      (uintptr_t)a.codes, (uintptr_t)(a.final2 != nullptr), (uintptr_t)a.recon, (uintptr_t)ws,
                      (uintptr_t)cfg.cols_per_block, (uintptr_t)cfg.rows_per_block, (uintptr_t)cfg.ksplit,
                      (uintptr_t)cfg.recon_cols_per_block, (uintptr_t)(intptr_t)cfg.pad,
                      (uintptr_t)(intptr_t)cfg.chunk, (uintptr_t)cfg.pts}};
        hipGraphExec_t exec = nullptr;
        bool launched = false;
        if ((st = graph_launch_cached(key, s, &launched))) return st;
        if (!launched) {
            CaptureSection capture_section;   // no other library call runs while capturing
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            holo_status est = gs_enqueue(a, s, cfg, tw_x, tw_y, b, L);
            hipError_t ce = hipStreamEndCapture(s, &graph);
            if (est) {
                if (graph) (void)hipGraphDestroy(graph);
                return est;
            }
            if (ce != hipSuccess) return fail(HOLO_EDEVICE, "GS graph capture: %s", hipGetErrorString(ce));
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(HOLO_EDEVICE, "GS graph instantiate: %s", hipGetErrorString(ie));
            if ((st = graph_insert_launch(key, exec, nullptr, s))) return st;
        }
    }
    if (a.codes && a.final2) {
        if ((st = copy_out(a.final2, (double*)(b + L.o_f2), 2, a.flags, s))) return st;
    }
    if ((st = copy_out(a.nmse, (double*)(b + L.o_nm), n_iter, a.flags, s))) return st;
    if ((st = copy_out(a.err, (double*)(b + L.o_er), n_iter, a.flags, s))) return st;
    return HOLO_OK;
}


// ---------------------------------------------------------------------------
// Batched GS: frames of one size iterate together, every pass one launch over
// the frame table (device memory: owned by the captured graph, or by the call
// when launched directly).
// ---------------------------------------------------------------------------
holo_status gs_enqueue_group(const GsFrame* dtab, const std::vector<GsFrame>& tab,
                             const std::vector<GsArgs>& args, const std::vector<GsLayout>& L,
                             const std::vector<size_t>& o_frame, double* f2, int nx, int ny, int n_iter,
                             const PhaseSrc& src, const uint64_t* dcur, const float2* tw_x, const float2* tw_y,
                             char* b, const LaunchCfg& cfg, hipStream_t s)
{
    const int F = (int)tab.size();
    bool any_codes = false;
    for (const GsFrame& g : tab) any_codes = any_codes || g.codes;
    LAUNCH("gs_rows", s, launch_gs_rows(GS_INIT, nullptr, nx, ny, src, 0, dcur, nullptr, nullptr, nullptr, nullptr,
                                        nullptr, tw_x, cfg, s, dtab, F, 0));
    LAUNCH("gs_consts", s, launch_gs_consts(nullptr, ny, nx, nullptr, s, dtab, F));
    for (int it = 0; it < n_iter; ++it) {
        const bool last = it == n_iter - 1;
        // any non-null codes argument asks the grouped pass for every frame's
        // codes (frames without a codes buffer skip them)
        uint8_t* want = (last && any_codes) ? reinterpret_cast<uint8_t*>(b) : nullptr;
        LAUNCH("gs_cols", s, launch_gs_cols(nullptr, nx, ny, want, tw_y, cfg, s, dtab, F));
        LAUNCH("gs_rows", s, launch_gs_rows(last ? GS_FINAL : GS_ITER, nullptr, nx, ny, src, 0, nullptr, nullptr,
                                            nullptr, nullptr, nullptr, nullptr, tw_x, cfg, s, dtab, F,
                                            it * 3 * ny));
    }
    LAUNCH("gs_finalize", s, launch_gs_finalize(nullptr, n_iter, ny, nullptr, nullptr, nullptr, s, dtab, F));
    // the 8-level replay, frame by frame
    for (int f = 0; f < F; ++f) {
        const GsArgs& a = args[f];
        if (!a.codes || (!f2 && !a.recon)) continue;
        char* bf = b + o_frame[f];
        float2* x2 = (float2*)(bf + L[f].o_x2);
        double* p5 = (double*)(bf + L[f].o_p5);
        double* out2 = f2 ? f2 + 2 * f : (double*)(bf + L[f].o_f2);
        LAUNCH("recon_cols", s, launch_recon_cols(a.codes, 8, nx, ny, 1, x2, tw_y, cfg, s));
        LAUNCH("recon_rows", s, launch_recon_rows(x2, nx, ny, 1, false, a.target, a.recon, p5, tw_x, cfg, s));
        LAUNCH("nmse_finalize", s, launch_nmse_finalize(p5, ny, out2, s));
    }
    return HOLO_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free GS (holo_gs_iterate_noalloc): the call's scratch lives in a
// fixed device array of kNoAllocScratch bytes and its twiddle tables in a
// fixed device table, both static members of the library's code object (each
// GPU the library runs on holds its own copy until the process ends).  Host
// code never passes the arrays' names to a kernel: their device addresses are
// taken once per device with hipGetSymbolAddress and kept in g_noalloc.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratch = HOLO_GS_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocTwiddles = 4080;   // W_N^k for N = 16, 32, ..., 2048: table of N at offset N - 16
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];
static __device__ __align__(256) float2 noalloc_twiddles[kNoAllocTwiddles];

struct NoAllocDevice {
    char* scratch;    // device address of `scratch` on this device
    float2* tw;       // device address of `noalloc_twiddles`, tables generated
};
std::mutex g_noalloc_mu;
std::map<int, NoAllocDevice> g_noalloc;

// Device addresses of the fixed arrays on the current device; the first call
// on a device also generates the twiddle tables (FP64 on the device, as for
// the workspace path) and waits for them, so it must not run under capture.
holo_status noalloc_device(int device, hipStream_t s, NoAllocDevice* out)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc.find(device);
    if (it != g_noalloc.end()) {
        *out = it->second;
        return HOLO_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(HOLO_EUNSUPPORTED, "holo_gs_iterate_noalloc: the first call on a device sets up its tables "
                                       "and must not run under stream capture");
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    void* tw = nullptr;
    HIP_TRY(hipGetSymbolAddress(&tw, HIP_SYMBOL(noalloc_twiddles)));
    for (int n = 16; n <= 2048; n <<= 1) HIP_TRY(launch_twiddle_gen((float2*)tw + (n - 16), n, s));
    HIP_TRY(hipStreamSynchronize(s));
    NoAllocDevice d{(char*)ptr, (float2*)tw};
    g_noalloc[device] = d;
    *out = d;
    return HOLO_OK;
}

// Branch streams (default priority) for the batched graph's fork/join.
constexpr int kBranches = 4;
struct BatchSync {
    hipStream_t br[kBranches] = {};
    hipEvent_t fork = nullptr, join[kBranches] = {};
};
std::map<int, BatchSync> g_batch_sync;

holo_status get_batch_sync(int device, BatchSync** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    BatchSync& b = g_batch_sync[device];
    for (int i = 0; i < kBranches; ++i) {
        if (!b.br[i]) HIP_TRY(hipStreamCreateWithFlags(&b.br[i], hipStreamNonBlocking));
        if (!b.join[i]) HIP_TRY(hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming));
    }
    if (!b.fork) HIP_TRY(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
    *out = &b;
    return HOLO_OK;
}

// Median-free timing of `reps` back-to-back runs of f on stream s (ms per run).
template <typename F>
holo_status time_runs(hipStream_t s, int reps, F f, double* ms_out)
{
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    holo_status st = f();   // warm-up (and first-use allocations)
    if (!st) st = f();
    // the fastest of three batches: a single short batch is easily skewed by
    // clock ramps after the host-side checks between candidates
    float best = 0.0f;
    for (int b = 0; b < 3 && !st; ++b) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < reps && !st; ++r) st = f();
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (b == 0 || ms < best) best = ms;
    }
    if (!st) *ms_out = best / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace
}  // namespace holo

using namespace holo;

// A new handle on the current device (NULL after a failed device query).
static holo_lut* new_lut(int kind, uint64_t n_lut, uint32_t n_dev, uint64_t seed)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) {
        (void)hipGetLastError();
        fail(HOLO_EDEVICE, "no current device");
        return nullptr;
    }
    holo_lut* l = new holo_lut();
    l->device = device;
    l->kind = kind;
    l->id = g_lut_ids.fetch_add(1);
    l->n_lut = n_lut;
    l->n_dev = n_dev;
    l->seed = seed;
    return l;
}

// Copies `bytes` to a new device allocation *dst; on failure frees the whole handle.
static holo_status upload_lut(void** dst, const void* src, size_t bytes, holo_lut* l)
{
    if (hipMalloc(dst, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        holo_lut_free(l);
        return fail(HOLO_ENOMEM, "phase source of %zu bytes", bytes);
    }
    hipError_t e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        holo_lut_free(l);
        return fail(HOLO_EDEVICE, "phase source upload: %s", hipGetErrorString(e));
    }
    return HOLO_OK;
}

// The 256 code phasors exp(2*pi*i*q/256), FP64 then rounded.
static holo_status upload_code_phasors(holo_lut* l)
{
    std::vector<float2> ph(256);
    const double two_pi = 6.283185307179586476925286766559;
    for (int q = 0; q < 256; ++q)
        ph[q] = make_float2((float)std::cos(two_pi * (q / 256.0)), (float)std::sin(two_pi * (q / 256.0)));
    return upload_lut((void**)&l->dev, ph.data(), sizeof(float2) * 256, l);
}

extern "C" {

const char* holo_last_error(void) { return g_err.c_str(); }
int32_t holo_version(void) { return 1; }

holo_status holo_lut_from_phases(const double* phases, uint64_t n_lut, holo_lut** out)
{
    CallGuard call_guard;   // see g_call_mu
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_lut && !phases) return fail(HOLO_EINVAL, "phases is NULL");
    // the kernels address the table with 32-bit byte offsets
    if (n_lut >= (1ull << 29)) return fail(HOLO_EUNSUPPORTED, "n_lut %llu >= 2^29", (unsigned long long)n_lut);
    holo_lut* l = new_lut(SRC_TABLE, n_lut, n_lut ? (uint32_t)n_lut : 1u, 0);
    if (!l) return HOLO_EDEVICE;
    l->phases.assign(phases, phases + n_lut);
    std::vector<float2> ph(l->n_dev);
    if (n_lut == 0) ph[0] = make_float2(1.0f, 0.0f);
    for (uint64_t j = 0; j < n_lut; ++j) ph[j] = make_float2((float)std::cos(phases[j]), (float)std::sin(phases[j]));
    if (holo_status st = upload_lut((void**)&l->dev, ph.data(), sizeof(float2) * l->n_dev, l)) return st;
    *out = l;
    return HOLO_OK;
}

holo_status holo_lut_build(uint64_t n_lut, uint64_t seed, holo_lut** out)
{
    CallGuard call_guard;   // see g_call_mu
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    if (n_lut >= (1ull << 29)) return fail(HOLO_EUNSUPPORTED, "n_lut %llu >= 2^29", (unsigned long long)n_lut);
    std::vector<double> phi(n_lut);
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t s = seed;
    for (uint64_t j = 0; j < n_lut; ++j) {
        const uint64_t x = splitmix64(s);
        phi[j] = two_pi * ((double)(x >> 11) * 0x1.0p-53);
    }
    return holo_lut_from_phases(phi.data(), n_lut, out);
}

holo_status holo_lut_build_codes(uint64_t n_lut, uint64_t seed, holo_lut** out)
{
    CallGuard call_guard;   // see g_call_mu
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_lut == 0) return fail(HOLO_EINVAL, "n_lut must be >= 1");
    if (n_lut >= (1ull << 31)) return fail(HOLO_EUNSUPPORTED, "n_lut %llu >= 2^31", (unsigned long long)n_lut);
    holo_lut* l = new_lut(SRC_CODES8, n_lut, (uint32_t)n_lut, seed);
    if (!l) return HOLO_EDEVICE;
    // the host keeps the codes (1 byte each); holo_lut_phases derives phases from them
    l->host_codes.resize(n_lut);
    uint64_t s = seed;
    for (uint64_t j = 0; j < n_lut; ++j) l->host_codes[j] = (uint8_t)(splitmix64(s) >> 56);
    if (holo_status st = upload_lut((void**)&l->codes, l->host_codes.data(), n_lut, l)) return st;
    if (holo_status st = upload_code_phasors(l)) return st;
    *out = l;
    return HOLO_OK;
}

holo_status holo_lut_prng(uint64_t seed, holo_lut** out)
{
    CallGuard call_guard;   // see g_call_mu
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    *out = new_lut(SRC_PRNG, UINT64_MAX, 1u, seed);
    return *out ? HOLO_OK : HOLO_EDEVICE;
}

holo_status holo_lut_mseq(uint64_t seed, holo_lut** out)
{
    CallGuard call_guard;   // see g_call_mu
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    *out = nullptr;
    holo_lut* l = new_lut(SRC_MSEQ, kMseqM, kMseqM, seed);
    if (!l) return HOLO_EDEVICE;
    // first 31 bits s_0..s_30 = bits 30..0 of w; the Galois state with
    // coefficient-of-x^30 read-out that produces them is w ^ (w >> 28)
    uint64_t st = seed;
    uint32_t w = (uint32_t)(splitmix64(st) & kMseqM);
    if (w == 0) w = 1;
    std::vector<uint32_t> aux(32 + 12 * 1024);
    aux[0] = 2;   // x
    for (int j = 1; j < 31; ++j) aux[j] = gf_mul_host(aux[j - 1], aux[j - 1]);
    aux[31] = w ^ (w >> 28);
    uint32_t xb[4];   // x^(8b): the weight of byte b of a state
    for (int b = 0; b < 4; ++b) xb[b] = gf_xpow_host(8ull * b);
    for (int j = 0; j < 12; ++j) {   // stride 2^j: multiply by x^(8 * 2^j)
        const uint32_t c = gf_xpow_host(8ull << j);
        for (int b = 0; b < 4; ++b) {
            const uint32_t cb = gf_mul_host(c, xb[b]);
            for (uint32_t v = 0; v < 256; ++v) aux[32 + j * 1024 + b * 256 + v] = gf_mul_host(cb, v);
        }
    }
    if (holo_status e = upload_lut((void**)&l->mseq, aux.data(), aux.size() * sizeof(uint32_t), l)) return e;
    if (holo_status e = upload_code_phasors(l)) return e;
    *out = l;
    return HOLO_OK;
}

int32_t holo_lut_kind(const holo_lut* lut) { return lut ? lut->kind : -1; }

holo_status holo_lut_phases(const holo_lut* lut, double* out, uint64_t n)
{
    CallGuard call_guard;   // see g_call_mu
    if (!lut || (!out && n)) return fail(HOLO_EINVAL, "lut/out is NULL");
    if (lut->kind == SRC_PRNG || lut->kind == SRC_MSEQ)
        return fail(HOLO_EUNSUPPORTED, "this phase source keeps no table (holo_phase_mask gives its phasors)");
    uint64_t m = n < lut->n_lut ? n : lut->n_lut;
    if (lut->kind == SRC_CODES8) {
        const double two_pi = 6.283185307179586476925286766559;
        for (uint64_t j = 0; j < m; ++j) out[j] = two_pi * ((double)lut->host_codes[j] / 256.0);
    } else if (m) {
        std::memcpy(out, lut->phases.data(), m * sizeof(double));
    }
    return HOLO_OK;
}

uint64_t holo_lut_size(const holo_lut* lut) { return lut ? lut->n_lut : 0; }

void holo_lut_free(holo_lut* lut)
{
    CallGuard call_guard;   // see g_call_mu
    if (!lut) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(lut->device);
    if (lut->dev) (void)hipFree(lut->dev);
    if (lut->codes) (void)hipFree(lut->codes);
    if (lut->mseq) (void)hipFree(lut->mseq);
    (void)hipSetDevice(cur);
    delete lut;
}

uint32_t holo_lut_check(uint64_t n_lut, int64_t nx, int64_t ny, int32_t n_sf)
{
    uint32_t w = 0;
    if (n_lut == 0) return HOLO_LUT_FLAT | HOLO_LUT_LE_NSF | HOLO_LUT_LE_MAXDIM | HOLO_LUT_LT_FULL;
    bool prime = n_lut >= 2;
    for (uint64_t d = 2; prime && d * d <= n_lut; ++d)
        if (n_lut % d == 0) prime = false;
    if (!prime) w |= HOLO_LUT_NOT_PRIME;
    if (n_sf > 0 && n_lut <= (uint64_t)n_sf) w |= HOLO_LUT_LE_NSF;
    const int64_t md = nx > ny ? nx : ny;
    if (md > 0 && n_lut <= (uint64_t)md) w |= HOLO_LUT_LE_MAXDIM;
    if (nx > 0 && ny > 0 && ((uint64_t)(nx * ny)) % n_lut == 0) w |= HOLO_LUT_DIVIDES_FRAME;
    if (nx > 0 && ny > 0 && n_sf > 0 && n_lut < (uint64_t)nx * (uint64_t)ny * (uint64_t)n_sf) w |= HOLO_LUT_LT_FULL;
    return w;
}

namespace holo {
namespace {
// DFT-stage precision: FP32 everywhere; BF16/FP16 matrix-core stages for
// sides of 256 and more.
holo_status check_precision(int32_t precision, int64_t nx, int64_t ny)
{
    if (precision == HOLO_FP32) return HOLO_OK;
    if (precision != HOLO_BF16 && precision != HOLO_FP16)
        return fail(HOLO_EINVAL, "precision must be HOLO_FP32, HOLO_BF16 or HOLO_FP16 (got %d)", precision);
    if (nx < 256 || ny < 256)
        return fail(HOLO_EUNSUPPORTED, "BF16/FP16 DFT stages need nx, ny >= 256 (got %lld x %lld)", (long long)nx,
                    (long long)ny);
    return HOLO_OK;
}
}  // namespace
}  // namespace holo

// OSPR variant selected by the flags (HOLO_EINVAL for both, or an odd n_sf in pair mode).
holo_status ospr_mode_of(uint32_t flags, int n_sf, int* mode)
{
    const bool pairs = flags & HOLO_F_OSPR_PAIRS, l8 = flags & HOLO_F_OSPR_LEVELS8;
    if (pairs && l8) return fail(HOLO_EINVAL, "HOLO_F_OSPR_PAIRS and HOLO_F_OSPR_LEVELS8 exclude each other");
    if (pairs && (n_sf & 1)) return fail(HOLO_EINVAL, "pair mode needs an even n_sf (got %d)", n_sf);
    *mode = pairs ? OSPR_PAIRS : l8 ? OSPR_LEVELS8 : OSPR_BINARY;
    return HOLO_OK;
}

holo_status holo_ospr_generate(const float* target, int64_t nx, int64_t ny, int32_t n_sf, const holo_lut* lut,
                               uint64_t* cursor, void* holo_out, float* recon, double* nmse2,
                               int32_t precision, uint32_t flags, void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!target || !cursor || !holo_out) return fail(HOLO_EINVAL, "target, cursor and holo_out are required");
    if (n_sf < 1) return fail(HOLO_EINVAL, "n_sf must be >= 1 (got %d)", n_sf);
    int mode = OSPR_BINARY;
    if (holo_status e = ospr_mode_of(flags, n_sf, &mode)) return e;
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048] (got %lld x %lld)",
                    (long long)nx, (long long)ny);
    holo_status st = check_precision(precision, nx, ny);
    if (st) return st;
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if ((st = check_lut(lut, device))) return st;
    LaunchCfg cfg = plan_get(PLAN_OSPR, nx, ny, n_sf);
    cfg.prec = precision;
    if (precision && (st = get_dftop(device, precision, (hipStream_t)hip_stream, &cfg.dftop))) return st;
    if ((st = ospr_run(device, target, nx, ny, n_sf, lut, *cursor, holo_out, recon, nmse2, flags,
                       (hipStream_t)hip_stream, cfg, mode)))
        return st;
    *cursor += (uint64_t)ospr_fields(n_sf, mode) * (uint64_t)nx * (uint64_t)ny;
    return HOLO_OK;
}

holo_status holo_reconstruct_nmse(const void* holo, int32_t levels, int64_t nx, int64_t ny, int32_t n_sf,
                                  const float* target, float* recon, double* nmse2, uint32_t flags,
                                  void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!holo || !target) return fail(HOLO_EINVAL, "holo and target are required");
    if (levels != 2 && levels != 8) return fail(HOLO_EINVAL, "levels must be 2 or 8 (got %d)", levels);
    if (n_sf < 1) return fail(HOLO_EINVAL, "n_sf must be >= 1 (got %d)", n_sf);
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    hipStream_t s = (hipStream_t)hip_stream;
    holo_status st;
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)ny, s, &tw_y))) return st;
    const bool half = levels == 2;
    const int nrows = half ? (int)(ny / 2 + 1) : (int)ny;
    Carver cv;
    const LaunchCfg cfg = plan_get(PLAN_OSPR, nx, ny, n_sf);
    const size_t o_x2 = cv.take(sizeof(float2) * (size_t)nrows * (size_t)row_pitch((int)nx, cfg) * n_sf);
    const size_t o_part = cv.take(sizeof(double) * 5 * (size_t)nrows);
    const size_t o_nm = cv.take(sizeof(double) * 2);
    void* ws;
    if ((st = get_workspace(device, s, cv.off, &ws))) return st;
    char* b = (char*)ws;
    float2* x2 = (float2*)(b + o_x2);
    double* part = (double*)(b + o_part);
    double* nm = (double*)(b + o_nm);
    LAUNCH("recon_cols", s, launch_recon_cols(holo, levels, (int)nx, (int)ny, n_sf, x2, tw_y, cfg, s));
    LAUNCH("recon_rows", s, launch_recon_rows(x2, (int)nx, (int)ny, n_sf, half, target, recon, part, tw_x, cfg, s));
    LAUNCH("nmse_finalize", s, launch_nmse_finalize(part, nrows, nm, s));
    return copy_out(nmse2, nm, 2, flags, s);
}

holo_status holo_gs_iterate(const float* target, int64_t nx, int64_t ny, int32_t n_iter, const holo_lut* lut,
                            uint64_t* cursor, const float* init_phasor, float* field, uint8_t* codes,
                            double* nmse_per_iter, double* err_per_iter, double* nmse_final2, float* recon,
                            int32_t precision, uint32_t flags, void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!target || !cursor) return fail(HOLO_EINVAL, "target and cursor are required");
    if (n_iter < 1) return fail(HOLO_EINVAL, "n_iter must be >= 1 (got %d)", n_iter);
    if ((nmse_final2 || recon) && !codes) return fail(HOLO_EINVAL, "nmse_final2/recon need codes");
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    if (precision != HOLO_FP32) return fail(HOLO_EUNSUPPORTED, "holo_gs_iterate computes in FP32 only");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st;
    if (!init_phasor && (st = check_lut(lut, device))) return st;
    GsArgs a{target, nx, ny, n_iter, init_phasor ? nullptr : lut, init_phasor ? 0 : *cursor, init_phasor,
             field, codes, nmse_per_iter, err_per_iter, nmse_final2, recon, flags};
    const LaunchCfg cfg = plan_get(PLAN_GS, nx, ny, 1);
    if ((st = gs_run(device, a, (hipStream_t)hip_stream, cfg))) return st;
    if (!init_phasor) *cursor += (uint64_t)nx * (uint64_t)ny;
    return HOLO_OK;
}

holo_status holo_gs_iterate_batched(const holo_gs_frame* frames, int32_t n_frames, int64_t nx, int64_t ny,
                                    int32_t n_iter, const holo_lut* lut, uint64_t* cursor, double* nmse_per_iter,
                                    double* err_per_iter, double* nmse_final2, uint32_t flags, void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!frames || !cursor) return fail(HOLO_EINVAL, "frames and cursor are required");
    if (n_frames < 1 || n_frames > 256) return fail(HOLO_EINVAL, "n_frames must be in [1, 256] (got %d)", n_frames);
    if (n_iter < 1) return fail(HOLO_EINVAL, "n_iter must be >= 1 (got %d)", n_iter);
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    int n_pool = 0;
    for (int f = 0; f < n_frames; ++f) {
        const holo_gs_frame& fr = frames[f];
        if (!fr.target) return fail(HOLO_EINVAL, "frame %d: target is required", f);
        if (fr.recon && !fr.codes) return fail(HOLO_EINVAL, "frame %d: recon needs codes", f);
        if (nmse_final2 && !fr.codes) return fail(HOLO_EINVAL, "frame %d: nmse_final2 needs codes", f);
        if (!fr.init_phasor) ++n_pool;
    }
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st;
    if (n_pool) {
        if ((st = check_lut(lut, device))) return st;
        if (lut->kind == SRC_MSEQ)
            return fail(HOLO_EUNSUPPORTED, "holo_gs_iterate_batched: the M-sequence source is not supported");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const LaunchCfg cfg = plan_get(PLAN_GS, nx, ny, 1);
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)ny, s, &tw_y))) return st;
    // per-frame layouts (as holo_gs_iterate's), one after another
    std::vector<GsArgs> args(n_frames);
    std::vector<GsLayout> L(n_frames);
    std::vector<size_t> o_frame(n_frames);
    Carver cv;
    for (int f = 0; f < n_frames; ++f) {
        const holo_gs_frame& fr = frames[f];
        args[f] = GsArgs{fr.target, nx, ny, n_iter, fr.init_phasor ? nullptr : lut, 0, fr.init_phasor, fr.field,
                         fr.codes, nullptr, nullptr, nullptr, fr.recon, flags};
        L[f] = gs_layout(args[f], cfg);
        o_frame[f] = cv.take(L[f].bytes);
    }
    const size_t o_cur = cv.take(sizeof(uint64_t));
    const size_t o_nm = cv.take(sizeof(double) * (size_t)n_frames * n_iter);
    const size_t o_er = cv.take(sizeof(double) * (size_t)n_frames * n_iter);
    const size_t o_f2 = cv.take(sizeof(double) * 2 * (size_t)n_frames);
    void* ws;
    if ((st = get_workspace(device, s, cv.off, &ws))) return st;
    char* b = (char*)ws;
    uint64_t* dcur = (uint64_t*)(b + o_cur);
    double* nm = (double*)(b + o_nm);
    double* er = (double*)(b + o_er);
    double* f2 = nmse_final2 ? (double*)(b + o_f2) : nullptr;
    std::vector<GsFrame> tab(n_frames);
    uint64_t pool_off = 0;
    for (int f = 0; f < n_frames; ++f) {
        const holo_gs_frame& fr = frames[f];
        char* bf = b + o_frame[f];
        GsFrame& g = tab[f];
        g.target = fr.target;
        g.init = (const float2*)fr.init_phasor;
        g.state = (float2*)(bf + L[f].o_state);
        g.field = fr.field ? (float2*)fr.field : (float2*)(bf + L[f].o_field);
        g.codes = fr.codes;
        g.pinit = (double*)(bf + L[f].o_pinit);
        g.piter = (double*)(bf + L[f].o_piter);
        g.consts = (GsConsts*)(bf + L[f].o_consts);
        g.nmse = nm + (size_t)f * n_iter;
        g.err = er + (size_t)f * n_iter;
        g.c0 = fr.init_phasor ? 0 : lut_wrap(lut, pool_off);
        if (!fr.init_phasor) pool_off += (uint64_t)nx * (uint64_t)ny;
    }
    PhaseSrc src{};
    src.n = 1;
    if (n_pool) {
        src = make_src(lut, nullptr);
        hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, dcur, lut_wrap(lut, *cursor));
        HIP_TRY(hipGetLastError());
    }
    auto enqueue = [&](const GsFrame* dtab) {
        return gs_enqueue_group(dtab, tab, args, L, o_frame, f2, (int)nx, (int)ny, n_iter, src, dcur, tw_x, tw_y, b,
                                cfg, s);
    };
    auto new_table = [&](GsFrame** out) -> holo_status {
        if (hipMalloc((void**)out, sizeof(GsFrame) * tab.size()) != hipSuccess)
            return fail(HOLO_ENOMEM, "GS frame table (%zu frames)", tab.size());
        hipError_t me = hipMemcpy(*out, tab.data(), sizeof(GsFrame) * tab.size(), hipMemcpyHostToDevice);
        if (me != hipSuccess) {
            (void)hipFree(*out);
            return fail(HOLO_EDEVICE, "GS frame table: %s", hipGetErrorString(me));
        }
        return HOLO_OK;
    };
    bool prof_on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof_on = g_prof_on;
    }
    if (!g_use_graphs || prof_on || s == nullptr) {
        GsFrame* dtab = nullptr;
        if ((st = new_table(&dtab))) return st;
        st = enqueue(dtab);
        hipError_t se = hipStreamSynchronize(s);   // the table is read by the launches above
        (void)hipFree(dtab);
        if (st) return st;
        if (se != hipSuccess) return fail(HOLO_EDEVICE, "batched GS: %s", hipGetErrorString(se));
    } else {
        GraphKey key;
        key.k = {(uintptr_t)0x65B7, (uintptr_t)device, (uintptr_t)s, (uintptr_t)ws, (uintptr_t)nx, (uintptr_t)ny,
                 (uintptr_t)n_iter, (uintptr_t)(n_pool ? lut->id : 0), (uintptr_t)(f2 != nullptr),
                 (uintptr_t)cfg.cols_per_block, (uintptr_t)cfg.rows_per_block, (uintptr_t)(intptr_t)cfg.pad,
                 (uintptr_t)cfg.pts, (uintptr_t)n_frames};
        for (int f = 0; f < n_frames; ++f)
            key.k.insert(key.k.end(), {(uintptr_t)frames[f].target, (uintptr_t)frames[f].init_phasor,
                                       (uintptr_t)frames[f].field, (uintptr_t)frames[f].codes,
                                       (uintptr_t)frames[f].recon});
        hipGraphExec_t exec = nullptr;
        bool launched = false;
        if ((st = graph_launch_cached(key, s, &launched))) return st;
        if (!launched) {
            CaptureSection capture_section;   // no other library call runs while capturing
            GsFrame* dtab = nullptr;
            if ((st = new_table(&dtab))) return st;
            hipGraph_t graph = nullptr;
            hipError_t be = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (be != hipSuccess) {
                (void)hipFree(dtab);
                return fail(HOLO_EDEVICE, "batched GS graph capture: %s", hipGetErrorString(be));
            }
            holo_status est = enqueue(dtab);
            hipError_t ce = hipStreamEndCapture(s, &graph);
            if (est || ce != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipFree(dtab);
                if (est) return est;
                return fail(HOLO_EDEVICE, "batched GS graph capture: %s", hipGetErrorString(ce));
            }
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                (void)hipFree(dtab);
                return fail(HOLO_EDEVICE, "batched GS graph instantiate: %s", hipGetErrorString(ie));
            }
            if ((st = graph_insert_launch(key, exec, dtab, s))) return st;
        }
    }
    if (f2 && (st = copy_out(nmse_final2, f2, 2 * (size_t)n_frames, flags, s))) return st;
    if ((st = copy_out(nmse_per_iter, nm, (size_t)n_frames * n_iter, flags, s))) return st;
    if ((st = copy_out(err_per_iter, er, (size_t)n_frames * n_iter, flags, s))) return st;
    *cursor += (uint64_t)n_pool * (uint64_t)nx * (uint64_t)ny;
    return HOLO_OK;
}

holo_status holo_gs_iterate_noalloc(const float* target, int64_t nx, int64_t ny, int32_t n_iter,
                                    const holo_lut* lut, uint64_t* cursor, const float* init_phasor, float* field,
                                    uint8_t* codes, double* nmse_per_iter, double* err_per_iter,
                                    double* nmse_final2, float* recon, int32_t precision, uint32_t flags,
                                    void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!target || !cursor) return fail(HOLO_EINVAL, "target and cursor are required");
    if (n_iter < 1) return fail(HOLO_EINVAL, "n_iter must be >= 1 (got %d)", n_iter);
    if ((nmse_final2 || recon) && !codes) return fail(HOLO_EINVAL, "nmse_final2/recon need codes");
    if ((nmse_per_iter || err_per_iter || nmse_final2) && !(flags & HOLO_F_NMSE_DEVICE))
        return fail(HOLO_EINVAL, "holo_gs_iterate_noalloc writes NMSE values to device memory only "
                                 "(HOLO_F_NMSE_DEVICE)");
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    if (precision != HOLO_FP32) return fail(HOLO_EUNSUPPORTED, "holo_gs_iterate computes in FP32 only");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st;
    if (!init_phasor && (st = check_lut(lut, device))) return st;
    GsArgs a{target, nx, ny, n_iter, init_phasor ? nullptr : lut, init_phasor ? 0 : *cursor, init_phasor,
             field, codes, nmse_per_iter, err_per_iter, nmse_final2, recon, flags};
    const LaunchCfg cfg = plan_get(PLAN_GS, nx, ny, 1);
    const GsLayout L = gs_layout(a, cfg);
    if (L.bytes > kNoAllocScratch)
        return fail(HOLO_EUNSUPPORTED, "holo_gs_iterate_noalloc: %lldx%lld with %d iterations needs %zu bytes of "
                                       "scratch, more than the fixed %zu", (long long)nx, (long long)ny, n_iter,
                    L.bytes, kNoAllocScratch);
    hipStream_t s = (hipStream_t)hip_stream;
    NoAllocDevice d;
    if ((st = noalloc_device(device, s, &d))) return st;
    struct Suppress {
        Suppress() { t_prof_suppress = true; }
        ~Suppress() { t_prof_suppress = false; }
    } no_events;   // kernel timing would create events: not recorded here
    char* b = d.scratch;
    if (!a.init) {
        hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, (uint64_t*)(b + L.o_cur), lut_wrap(a.lut, a.cursor));
        HIP_TRY(hipGetLastError());
    }
    if ((st = gs_enqueue(a, s, cfg, d.tw + (nx - 16), d.tw + (ny - 16), b, L))) return st;
    if (codes && nmse_final2) {
        if ((st = copy_out(nmse_final2, (double*)(b + L.o_f2), 2, flags, s))) return st;
    }
    if ((st = copy_out(nmse_per_iter, (double*)(b + L.o_nm), n_iter, flags, s))) return st;
    if ((st = copy_out(err_per_iter, (double*)(b + L.o_er), n_iter, flags, s))) return st;
    if (!init_phasor) *cursor += (uint64_t)nx * (uint64_t)ny;
    return HOLO_OK;
}

holo_status holo_fft2(const float* in, float* out, int64_t nx, int64_t ny, int32_t sign, int32_t precision,
                      void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!in || !out) return fail(HOLO_EINVAL, "in and out are required");
    if (sign != 1 && sign != -1) return fail(HOLO_EINVAL, "sign must be +1 or -1");
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    holo_status st = check_precision(precision, nx, ny);
    if (st) return st;
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    hipStream_t s = (hipStream_t)hip_stream;
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)ny, s, &tw_y))) return st;
    void* ws;
    if ((st = get_workspace(device, s, sizeof(float2) * (size_t)nx * ny, &ws))) return st;
    LaunchCfg cfg = default_cfg();
    cfg.prec = precision;
    if (precision && (st = get_dftop(device, precision, s, &cfg.dftop))) return st;
    LAUNCH("fft2", s, launch_fft2((const float2*)in, (float2*)ws, (float2*)out, (int)nx, (int)ny, sign, tw_x, tw_y,
                                  cfg, s));
    return HOLO_OK;
}

holo_status holo_phase_mask(const holo_lut* lut, uint64_t cursor, int64_t nx, int64_t ny, int32_t n_sf, float* out,
                            void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!out) return fail(HOLO_EINVAL, "out is required");
    if (n_sf < 1) return fail(HOLO_EINVAL, "n_sf must be >= 1");
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st = check_lut(lut, device);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const uint64_t c0 = lut_wrap(lut, cursor);
    uint32_t* rs = nullptr;
    if (lut->kind == SRC_MSEQ) {
        void* ws;
        if ((st = get_workspace(device, s, sizeof(uint32_t) * (size_t)n_sf * (size_t)ny, &ws))) return st;
        rs = (uint32_t*)ws;
        LAUNCH("mseq_rows", s, launch_mseq_rows(lut->mseq, c0, nullptr, (int)nx, (int)ny, n_sf, rs, s));
    }
    LAUNCH("phase_mask", s, launch_phase_mask(make_src(lut, rs), c0, (int)nx, (int)ny, n_sf, (float2*)out, s));
    return HOLO_OK;
}

holo_status holo_ospr_generate_batched(const holo_frame* frames, int32_t n_frames, const holo_lut* lut,
                                       uint64_t* cursor, double* nmse_out, int32_t precision, uint32_t flags,
                                       void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!frames || !cursor) return fail(HOLO_EINVAL, "frames and cursor are required");
    if (n_frames < 1 || n_frames > 4096) return fail(HOLO_EINVAL, "n_frames must be in [1, 4096] (got %d)", n_frames);
    int mode = OSPR_BINARY;
    for (int f = 0; f < n_frames; ++f) {
        const holo_frame& fr = frames[f];
        if (!fr.target || !fr.holo_bits) return fail(HOLO_EINVAL, "frame %d: target and holo_bits are required", f);
        if (fr.n_sf < 1) return fail(HOLO_EINVAL, "frame %d: n_sf must be >= 1", f);
        if (holo_status e = ospr_mode_of(flags, fr.n_sf, &mode)) return e;
        if (!pow2_in_range(fr.nx) || !pow2_in_range(fr.ny))
            return fail(HOLO_EUNSUPPORTED, "frame %d: nx, ny must be powers of two in [16, 2048]", f);
        if (holo_status e = check_precision(precision, fr.nx, fr.ny)) return e;
    }
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st = check_lut(lut, device);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;

    // per-frame plans, layouts, pool offsets (exclusive prefix sum of n_sf*N)
    std::vector<LaunchCfg> cfg(n_frames);
    std::vector<OsprLayout> lay(n_frames);
    std::vector<uint64_t> off(n_frames);
    uint64_t total = 0;
    const void* dftop = nullptr;
    if (precision && (st = get_dftop(device, precision, s, &dftop))) return st;
    for (int f = 0; f < n_frames; ++f) {
        const holo_frame& fr = frames[f];
        cfg[f] = plan_get(PLAN_OSPR, fr.nx, fr.ny, fr.n_sf);
        cfg[f].prec = precision;
        cfg[f].dftop = dftop;
        lay[f] = ospr_layout(fr.nx, fr.ny, fr.n_sf, cfg[f], mode);
        off[f] = total;
        total += (uint64_t)ospr_fields(fr.n_sf, mode) * (uint64_t)fr.nx * (uint64_t)fr.ny;
    }
    bool prof_on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof_on = g_prof_on;
    }
    const bool use_graph = g_use_graphs && !prof_on && s != nullptr;
    // Graph replays of binary frames drawn from a pool without per-row states
    // run grouped: frames of one size and launch shape share one launch per
    // pass (K1..K4), each frame with its own planes (no chunking).  Otherwise
    // each frame runs its own launches (chunked, branch-local planes).
    const bool grouped = use_graph && mode == OSPR_BINARY && lut->kind != SRC_MSEQ;
    std::vector<std::vector<int>> units;   // frames launched together
    if (grouped) {
        std::map<std::vector<int>, int> gid;
        for (int f = 0; f < n_frames; ++f) {
            const holo_frame& fr = frames[f];
            const LaunchCfg& c = cfg[f];
            const std::vector<int> k = {(int)fr.nx, (int)fr.ny, c.cols_per_block, c.rows_per_block, c.ksplit,
                                        c.pad, c.pts, recon_rows_groups((int)fr.nx, fr.n_sf, c)};
            auto it = gid.find(k);
            if (it == gid.end()) {
                it = gid.emplace(k, (int)units.size()).first;
                units.emplace_back();
            }
            units[it->second].push_back(f);
        }
        // groups are split (frames in order) so that a unit's half planes
        // stay within 64 MiB -- the four branches' row-pass output then fits
        // the last-level cache until the column pass reads it -- and within
        // an eighth of the batch's work (balanced branches)
        double all = 0.0;
        for (int f = 0; f < n_frames; ++f) all += (double)frames[f].n_sf * frames[f].nx * frames[f].ny;
        const double cap = std::min(all / (2.0 * kBranches), (double)(64u << 20) / 4.0);
        std::vector<std::vector<int>> split;
        for (const auto& g : units) {
            split.emplace_back();
            double w = 0.0;
            for (int f : g) {
                const double wf = (double)frames[f].n_sf * frames[f].nx * frames[f].ny;
                if (!split.back().empty() && w + wf > cap) {
                    split.emplace_back();
                    w = 0.0;
                }
                split.back().push_back(f);
                w += wf;
            }
        }
        units.swap(split);
    } else {
        for (int f = 0; f < n_frames; ++f) units.push_back({f});
    }
    // units to branches: longest first onto the least-loaded branch
    const int nu = (int)units.size();
    const int nb = nu < kBranches ? nu : kBranches;
    std::vector<double> work(nu, 0.0);
    for (int u = 0; u < nu; ++u)
        for (int f : units[u]) work[u] += (double)frames[f].n_sf * frames[f].nx * frames[f].ny;
    std::vector<int> order(nu), branch(nu);
    for (int u = 0; u < nu; ++u) order[u] = u;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return work[x] != work[y] ? work[x] > work[y] : x < y; });
    std::vector<double> load(nb, 0.0);
    std::vector<size_t> bbytes(nb, 0);
    for (int u : order) {
        int bi = 0;
        for (int i = 1; i < nb; ++i)
            if (load[i] < load[bi]) bi = i;
        branch[u] = bi;
        load[bi] += work[u];
        if (!grouped && lay[units[u][0]].bytes > bbytes[bi]) bbytes[bi] = lay[units[u][0]].bytes;
    }
    Carver cv;
    std::vector<size_t> o_branch(nb), o_x1(n_frames), o_x2(n_frames), o_part(n_frames);
    if (grouped) {
        // a unit's frames get planes of their own, at offsets within the unit;
        // the units of one branch run one after another and reuse one region
        // (sized for the branch's largest unit), which also keeps a branch's
        // planes warm in the last-level cache from one unit to the next
        for (int u = 0; u < nu; ++u) {
            Carver cu;
            for (int f : units[u]) {
                const size_t plane = (size_t)(frames[f].ny / 2 + 1) * (size_t)row_pitch((int)frames[f].nx, cfg[f]);
                o_x1[f] = cu.take(sizeof(float2) * plane * (size_t)frames[f].n_sf);
                o_x2[f] = cu.take(sizeof(float2) * plane * (size_t)frames[f].n_sf);
                o_part[f] = cu.take(sizeof(double) * 5 * (size_t)(frames[f].ny / 2 + 1));
            }
            bbytes[branch[u]] = std::max(bbytes[branch[u]], cu.off);
        }
        for (int i = 0; i < nb; ++i) o_branch[i] = cv.take(bbytes[i]);
        for (int u = 0; u < nu; ++u)
            for (int f : units[u]) {
                o_x1[f] += o_branch[branch[u]];
                o_x2[f] += o_branch[branch[u]];
                o_part[f] += o_branch[branch[u]];
            }
    } else {
        for (int i = 0; i < nb; ++i) o_branch[i] = cv.take(bbytes[i]);
    }
    const size_t o_base = cv.take(sizeof(uint64_t));
    const size_t o_nm = cv.take(sizeof(double) * 2 * n_frames);
    // twiddle tables first: they synchronise, which capture forbids
    std::map<int, const float2*> tw;
    for (int f = 0; f < n_frames; ++f)
        for (int n : {(int)frames[f].nx, (int)frames[f].ny})
            if (!tw.count(n)) {
                const float2* t = nullptr;
                if ((st = get_twiddles(device, n, s, &t))) return st;
                tw[n] = t;
            }
    void* ws;
    if ((st = get_workspace(device, s, cv.off, &ws))) return st;
    char* b = (char*)ws;
    uint64_t* dbase = (uint64_t*)(b + o_base);
    double* nm = (double*)(b + o_nm);

    // grouped: the frame table, unit by unit (each unit's entries contiguous)
    std::vector<GroupFrame> table;
    std::vector<int> ustart(nu, 0);
    if (grouped) {
        for (int u = 0; u < nu; ++u) {
            ustart[u] = (int)table.size();
            for (int f : units[u]) {
                const holo_frame& fr = frames[f];
                GroupFrame g{};
                g.target = fr.target;
                g.x1 = (float2*)(b + o_x1[f]);
                g.bits = (uint32_t*)fr.holo_bits;
                g.x2 = (float2*)(b + o_x2[f]);
                g.recon = fr.recon;
                g.part = (double*)(b + o_part[f]);
                g.nm = nm + 2 * f;
                g.c0 = lut_wrap(lut, off[f]);
                g.inv_scale = (float)(1.0 / ((double)fr.n_sf * (double)fr.nx * (double)fr.ny));
                g.n_sf = fr.n_sf;
                ospr_rows_h_shape((int)fr.nx, (int)fr.ny, fr.n_sf, cfg[f], &g.k1_blocks, &g.spb);
                g.k2_tiles = ospr_cols_tiles((int)fr.nx, (int)fr.ny, fr.n_sf, cfg[f]);
                table.push_back(g);
            }
        }
    }

    // the only per-call value inside the graph: the pool start, in device memory
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, dbase, lut_wrap(lut, *cursor));
    HIP_TRY(hipGetLastError());

    auto enqueue_all = [&](bool branches, BatchSync* bs, const GroupFrame* dtab) -> holo_status {
        for (int u = 0; u < nu; ++u) {
            hipStream_t fs = branches ? bs->br[branch[u]] : s;
            if (grouped) {
                const int f0 = units[u][0];
                const PhaseSrc src = make_src(lut, nullptr);
                LAUNCH("ospr_group", fs,
                       launch_ospr_group(dtab + ustart[u], &table[ustart[u]], (int)units[u].size(), (int)frames[f0].nx,
                                         (int)frames[f0].ny, src, dbase, tw[(int)frames[f0].nx],
                                         tw[(int)frames[f0].ny], cfg[f0], fs));
                continue;
            }
            const int f = units[u][0];
            const holo_frame& fr = frames[f];
            holo_status e = ospr_enqueue(fr.target, fr.nx, fr.ny, fr.n_sf, lut, lut_wrap(lut, off[f]), dbase,
                                         fr.holo_bits, fr.recon, nm + 2 * f, tw[(int)fr.nx], tw[(int)fr.ny],
                                         b + o_branch[branch[u]], lay[f], fs, cfg[f], mode);
            if (e) return e;
        }
        return HOLO_OK;
    };
    if (!use_graph) {
        if ((st = enqueue_all(false, nullptr, nullptr))) return st;
    } else {
        BatchSync* bs = nullptr;
        if ((st = get_batch_sync(device, &bs))) return st;
        GraphKey key;
        key.k = {(uintptr_t)0xBA7C, (uintptr_t)device, (uintptr_t)s, (uintptr_t)ws, (uintptr_t)lut->id,
                 (uintptr_t)n_frames, (uintptr_t)mode, (uintptr_t)grouped};
        for (int f = 0; f < n_frames; ++f) {
            const holo_frame& fr = frames[f];
            const LaunchCfg& c = cfg[f];
            key.k.insert(key.k.end(), {(uintptr_t)fr.nx, (uintptr_t)fr.ny, (uintptr_t)fr.n_sf, (uintptr_t)fr.target,
                                       (uintptr_t)fr.holo_bits, (uintptr_t)fr.recon, (uintptr_t)lut_wrap(lut, off[f]),
                                       (uintptr_t)c.cols_per_block, (uintptr_t)c.rows_per_block,
                                       (uintptr_t)c.ksplit, (uintptr_t)c.recon_cols_per_block,
                                       (uintptr_t)(intptr_t)c.pad, (uintptr_t)(intptr_t)c.chunk,
                                       (uintptr_t)c.pts, (uintptr_t)c.prec});
        }
        hipGraphExec_t exec = nullptr;
        bool launched = false;
        if ((st = graph_launch_cached(key, s, &launched))) return st;
        if (!launched) {
            CaptureSection capture_section;   // no other library call runs while capturing
            // the frame table lives with the graph (device memory written once)
            GroupFrame* dtab = nullptr;
            if (grouped) {
                if (hipMalloc((void**)&dtab, sizeof(GroupFrame) * table.size()) != hipSuccess)
                    return fail(HOLO_ENOMEM, "batch frame table (%zu frames)", table.size());
                hipError_t me = hipMemcpy(dtab, table.data(), sizeof(GroupFrame) * table.size(), hipMemcpyHostToDevice);
                if (me != hipSuccess) {
                    (void)hipFree(dtab);
                    return fail(HOLO_EDEVICE, "batch frame table: %s", hipGetErrorString(me));
                }
            }
            hipGraph_t graph = nullptr;
            hipError_t be = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (be != hipSuccess) {
                if (dtab) (void)hipFree(dtab);
                return fail(HOLO_EDEVICE, "batch graph capture: %s", hipGetErrorString(be));
            }
            holo_status est = HOLO_OK;
            hipError_t he = hipEventRecord(bs->fork, s);
            for (int i = 0; i < nb && he == hipSuccess; ++i) he = hipStreamWaitEvent(bs->br[i], bs->fork, 0);
            if (he == hipSuccess) est = enqueue_all(true, bs, dtab);
            for (int i = 0; i < nb && he == hipSuccess; ++i) {
                he = hipEventRecord(bs->join[i], bs->br[i]);
                if (he == hipSuccess) he = hipStreamWaitEvent(s, bs->join[i], 0);
            }
            hipError_t ce = hipStreamEndCapture(s, &graph);
            if (est || he != hipSuccess || ce != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                if (dtab) (void)hipFree(dtab);
                if (est) return est;
                return fail(HOLO_EDEVICE, "batch graph capture: %s",
                            hipGetErrorString(he != hipSuccess ? he : ce));
            }
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                if (dtab) (void)hipFree(dtab);
                return fail(HOLO_EDEVICE, "batch graph instantiate: %s", hipGetErrorString(ie));
            }
            if ((st = graph_insert_launch(key, exec, dtab, s))) return st;
        }
    }
    if ((st = copy_out(nmse_out, nm, 2 * (size_t)n_frames, flags, s))) return st;
    *cursor += total;
    return HOLO_OK;
}

holo_status holo_autotune_ospr(const float* target, int64_t nx, int64_t ny, int32_t n_sf, const holo_lut* lut,
                               uint32_t* scratch_bits, int32_t reps, int32_t* chosen, void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!target || !scratch_bits) return fail(HOLO_EINVAL, "target and scratch_bits are required");
    if (n_sf < 1 || reps < 1) return fail(HOLO_EINVAL, "n_sf and reps must be >= 1");
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st = check_lut(lut, device);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t nwords = (size_t)n_sf * (size_t)nx * (size_t)ny / 32;
    std::vector<uint32_t> ref_bits(nwords), bits(nwords);
    double ref_nm[2], nm[2];
    // reference: built-in heuristic shapes
    LaunchCfg best{};
    if ((st = ospr_run(device, target, nx, ny, n_sf, lut, 0, scratch_bits, nullptr, ref_nm, 0, s, best))) return st;
    HIP_TRY(hipMemcpy(ref_bits.data(), scratch_bits, nwords * 4, hipMemcpyDeviceToHost));
    double best_ms = 0.0;
    auto run = [&](const LaunchCfg& c) {
        return ospr_run(device, target, nx, ny, n_sf, lut, 0, scratch_bits, nullptr, nullptr, 0, s, c);
    };
    // bring the clocks up before anything is timed: candidates are timed in a
    // fixed order, and a ramp during the search favours the later ones
    for (int i = 0; i < 200; ++i)
        if ((st = run(best))) return st;
    if ((st = time_runs(s, reps, [&] { return run(best); }, &best_ms))) return st;
    // coordinate descent over each kernel's shape; a candidate with the
    // reference's points per thread counts only if it reproduces the reference
    // holograms bit for bit; one with other points per thread (another radix
    // factorisation) rounds differently, and may flip pixels whose Re h is
    // within that rounding of 0: at most 1e-5 of the bits; either way the NMSE
    // must agree to 1e-6 relative (FP32 summation order)
    const int ref_pts = best.pts;
    auto try_plan = [&](const LaunchCfg& c) {
        double ms = 0.0;
        if (run(c) != HOLO_OK) {
            g_err.clear();
            return;
        }
        if (ospr_run(device, target, nx, ny, n_sf, lut, 0, scratch_bits, nullptr, nm, 0, s, c)) return;
        if (hipMemcpy(bits.data(), scratch_bits, nwords * 4, hipMemcpyDeviceToHost) != hipSuccess) return;
        size_t flips = 0;
        for (size_t w = 0; w < nwords; ++w) flips += (size_t)__builtin_popcount(bits[w] ^ ref_bits[w]);
        const size_t allowed = c.pts == ref_pts ? 0 : (size_t)(1e-5 * 32.0 * (double)nwords);
        if (flips > allowed || std::fabs(nm[0] - ref_nm[0]) > 1e-6 * std::fabs(ref_nm[0]) ||
            std::fabs(nm[1] - ref_nm[1]) > 1e-6 * std::fabs(ref_nm[1]))
            return;
        if (time_runs(s, reps, [&] { return run(c); }, &ms)) return;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    };
    // radix factorisation (points per thread of the row, column and
    // reconstruction passes: the per-pass default, all 16 -- 1024 = 16*16*4 --
    // or all 8 -- 8*8*8*2), column-tile width and chunking interact
    // (registers and waves, tile lines, cache residency): search them jointly,
    // then the remaining shapes one at a time
    const int pts_opts[] = {0, 16, 8};
    const int cols_opts[] = {8, 16};
    const int chunk_opts[] = {0, 4, 6, 8, 12};
    const LaunchCfg base = best;
    for (int pt : pts_opts)
        for (int ci : cols_opts)
            for (int ch : chunk_opts) {
                LaunchCfg c = base;
                c.pts = pt;
                c.cols_per_block = ci;
                c.chunk = ch;
                try_plan(c);
            }
    const int rows_opts[] = {1, 2, 4, 8};
    const int ks_opts[] = {1, 2, 4, 8};
    const int pad_opts[] = {0, 16, 64};
    for (int r : rows_opts) {
        LaunchCfg c = best;
        c.rows_per_block = r;
        try_plan(c);
    }
    for (int k : ks_opts) {
        LaunchCfg c = best;
        c.ksplit = k;
        try_plan(c);
    }
    for (int p : pad_opts) {
        LaunchCfg c = best;
        c.pad = p;
        try_plan(c);
    }
    plan_put(PLAN_OSPR, nx, ny, n_sf, best);
    if (chosen) {
        chosen[0] = best.cols_per_block;
        chosen[1] = best.rows_per_block;
        chosen[2] = best.ksplit;
        chosen[3] = best.recon_cols_per_block;
        chosen[4] = best.pad;
        chosen[5] = best.chunk;
        chosen[6] = best.pts;
    }
    g_err.clear();
    return HOLO_OK;
}

holo_status holo_autotune_gs(const float* target, int64_t nx, int64_t ny, const holo_lut* lut, int32_t reps,
                             int32_t* chosen, void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    if (!target) return fail(HOLO_EINVAL, "target is required");
    if (reps < 1) return fail(HOLO_EINVAL, "reps must be >= 1");
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st = check_lut(lut, device);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const int n_iter = 4;
    const size_t npix = (size_t)nx * (size_t)ny;
    uint8_t* codes = nullptr;
    if (hipMalloc(&codes, npix) != hipSuccess) return fail(HOLO_ENOMEM, "autotune scratch");
    std::vector<uint8_t> ref_codes(npix), cd(npix);
    double ref_nm[n_iter], nm[n_iter];
    GsArgs a{target, nx, ny, n_iter, lut, 0, nullptr, nullptr, codes, ref_nm, nullptr, nullptr, nullptr, 0};
    LaunchCfg best{};
    double best_ms = 0.0;
    st = gs_run(device, a, s, best);
    if (!st) {
        (void)hipMemcpy(ref_codes.data(), codes, npix, hipMemcpyDeviceToHost);
        GsArgs q = a;
        q.nmse = nullptr;
        auto run = [&](const LaunchCfg& c) { return gs_run(device, q, s, c); };
        for (int i = 0; i < 20 && !st; ++i) st = run(best);   // clocks up before timing
        if (!st) st = time_runs(s, reps, [&] { return run(best); }, &best_ms);
        // points per thread first (changes the FP32 factorisation, so its
        // guard is a tolerance: per-iteration NMSE within 1e-5 relative and
        // codes within 1e-3 of the pixels), then the shapes (exact guard)
        const int pts_opts[] = {16, 8, 8, 8};
        const int cols_opts[] = {2, 4, 8, 16};
        const int rows_opts[] = {1, 2, 4, 8};
        const int pad_opts[] = {0, 16, 64, 64};
        for (int dim = 0; dim < 4 && !st; ++dim) {
            const int* opts = dim == 0 ? pts_opts : dim == 1 ? cols_opts : dim == 2 ? rows_opts : pad_opts;
            if (dim == 1) {   // later dimensions compare against the chosen pts
                GsArgs v = a;
                v.nmse = ref_nm;
                if ((st = gs_run(device, v, s, best))) break;
                (void)hipMemcpy(ref_codes.data(), codes, npix, hipMemcpyDeviceToHost);
            }
            for (int i = 0; i < 4; ++i) {
                LaunchCfg c = best;
                (dim == 0 ? c.pts : dim == 1 ? c.cols_per_block : dim == 2 ? c.rows_per_block : c.pad) = opts[i];
                GsArgs v = a;
                v.nmse = nm;
                if (gs_run(device, v, s, c) != HOLO_OK) {
                    (void)hipGetLastError();
                    continue;
                }
                (void)hipMemcpy(cd.data(), codes, npix, hipMemcpyDeviceToHost);
                bool same = true;
                if (dim == 0) {
                    size_t diff = 0;
                    for (size_t p = 0; p < npix; ++p) diff += cd[p] != ref_codes[p];
                    same = diff <= npix / 1000;
                    for (int k = 0; k < n_iter; ++k) same = same && std::fabs(nm[k] - ref_nm[k]) <= 1e-5 * ref_nm[k];
                } else {
                    same = cd == ref_codes;
                    for (int k = 0; k < n_iter; ++k) same = same && nm[k] == ref_nm[k];
                }
                if (!same) continue;
                double ms = 0.0;
                if (time_runs(s, reps, [&] { return run(c); }, &ms)) continue;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(codes);
    if (st) return st;
    plan_put(PLAN_GS, nx, ny, 1, best);
    if (chosen) {
        chosen[0] = best.cols_per_block;
        chosen[1] = best.rows_per_block;
        chosen[2] = best.ksplit;
        chosen[3] = best.recon_cols_per_block;
        chosen[4] = best.pad;
        chosen[5] = best.chunk;
        chosen[6] = best.pts;
    }
    g_err.clear();
    return HOLO_OK;
}

// Points per thread of a plan: GS 0, 4, 8 or 16; OSPR 0, 8 or 16.
holo_status plan_check_pts(int kind, int pts)
{
    if (kind == PLAN_GS ? (pts != 0 && pts != 4 && pts != 8 && pts != 16) : (pts != 0 && pts != 8 && pts != 16))
        return fail(HOLO_EINVAL, "points per thread must be 0, %s8 or 16 (got %d)", kind == PLAN_GS ? "4, " : "", pts);
    return HOLO_OK;
}

holo_status holo_plan_set(int32_t kind, int64_t nx, int64_t ny, int32_t n_sf, const int32_t* cfg)
{
    if ((kind != 0 && kind != 1) || !cfg) return fail(HOLO_EINVAL, "kind must be 0 (OSPR) or 1 (GS), cfg set");
    if (n_sf < 0) return fail(HOLO_EINVAL, "n_sf must be >= 0 (0: every sub-frame count)");
    if (holo_status st = plan_check_pts(kind, cfg[6])) return st;
    LaunchCfg c;
    c.cols_per_block = cfg[0];
    c.rows_per_block = cfg[1];
    c.ksplit = cfg[2];
    c.recon_cols_per_block = cfg[3];
    c.pad = cfg[4];
    c.chunk = cfg[5];
    c.pts = cfg[6];
    plan_put(kind, nx, ny, n_sf, c);
    return HOLO_OK;
}

holo_status holo_plan_get(int32_t kind, int64_t nx, int64_t ny, int32_t n_sf, int32_t* cfg)
{
    if ((kind != 0 && kind != 1) || !cfg) return fail(HOLO_EINVAL, "kind must be 0 (OSPR) or 1 (GS), cfg set");
    const LaunchCfg c = plan_get(kind, nx, ny, n_sf);
    cfg[0] = c.cols_per_block;
    cfg[1] = c.rows_per_block;
    cfg[2] = c.ksplit;
    cfg[3] = c.recon_cols_per_block;
    cfg[4] = c.pad;
    cfg[5] = c.chunk;
    cfg[6] = c.pts;
    return HOLO_OK;
}

holo_status holo_plan_save(const char* path)
{
    if (!path) return fail(HOLO_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(HOLO_EINVAL, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    std::fprintf(f, "{\"plans\": [");
    bool first = true;
    for (auto& kv : g_plans) {
        std::fprintf(f,
                     "%s\n  {\"kind\": %d, \"nx\": %lld, \"ny\": %lld, \"n_sf\": %d, \"cfg\": [%d, %d, %d, %d, %d, %d, %d]}",
                     first ? "" : ",", kv.first.kind, (long long)kv.first.nx, (long long)kv.first.ny, kv.first.n_sf,
                     kv.second.cols_per_block, kv.second.rows_per_block, kv.second.ksplit,
                     kv.second.recon_cols_per_block, kv.second.pad, kv.second.chunk, kv.second.pts);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    std::fclose(f);
    return HOLO_OK;
}

holo_status holo_plan_load(const char* path)
{
    if (!path) return fail(HOLO_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(HOLO_EINVAL, "cannot read %s", path);
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    std::fclose(f);
    // entries written by holo_plan_save: {"kind": K, "nx": X, "ny": Y, "n_sf": S, "cfg": [7 ints]}
    size_t pos = 0;
    while ((pos = txt.find("{\"kind\"", pos)) != std::string::npos) {
        int kind, sf, c0, c1, c2, c3, c4, c5, c6;
        long long nx, ny;
        if (std::sscanf(txt.c_str() + pos,
                        "{\"kind\": %d, \"nx\": %lld, \"ny\": %lld, \"n_sf\": %d, \"cfg\": [%d, %d, %d, %d, %d, %d, %d]}",
                        &kind, &nx, &ny, &sf, &c0, &c1, &c2, &c3, &c4, &c5, &c6) == 11) {
            if (kind != PLAN_OSPR && kind != PLAN_GS) return fail(HOLO_EINVAL, "plan kind %d in %s", kind, path);
            if (sf < 0) return fail(HOLO_EINVAL, "plan n_sf %d in %s (must be >= 0)", sf, path);
            if (holo_status st = plan_check_pts(kind, c6)) return st;
            LaunchCfg c;
            c.cols_per_block = c0;
            c.rows_per_block = c1;
            c.ksplit = c2;
            c.recon_cols_per_block = c3;
            c.pad = c4;
            c.chunk = c5;
            c.pts = c6;
            plan_put(kind, nx, ny, sf, c);
        } else {
            return fail(HOLO_EINVAL, "malformed plan entry in %s", path);
        }
        ++pos;
    }
    return HOLO_OK;
}

holo_status holo_set_graphs(int32_t on)
{
    g_use_graphs = on != 0;
    return HOLO_OK;
}

// ---------------------------------------------------------------------------
// Learned GS seed network
// ---------------------------------------------------------------------------
namespace holo {
namespace {
bool cnn_size_ok(int64_t n) { return n >= 64 && n <= 2048 && (n & (n - 1)) == 0; }

void cnn_free_images(holo_cnn* c)
{
    for (int i = 0; i < 4; ++i) (void)hipFree(c->b.act[i]), c->b.act[i] = nullptr;
    for (int i = 0; i < 2; ++i) (void)hipFree(c->b.dact[i]), c->b.dact[i] = nullptr;
    (void)hipFree(c->b.o5), (void)hipFree(c->b.d5), (void)hipFree(c->b.part), (void)hipFree(c->ph);
    c->b.o5 = c->b.d5 = nullptr;
    c->b.part = nullptr;
    c->ph = nullptr;
    c->img_px = 0;
}

holo_status cnn_images(holo_cnn* c, int64_t nx, int64_t ny)
{
    const size_t npx = (size_t)nx * (size_t)ny;
    const int rpb = 1;   // one image row per weight-gradient block: ny blocks
    const int nblk = (int)((ny + rpb - 1) / rpb);
    if (npx <= c->img_px && nblk <= c->img_rows) {
        c->b.rows_per_block = rpb;
        return HOLO_OK;
    }
    HIP_TRY(hipDeviceSynchronize());
    cnn_free_images(c);
    bool ok = true;
    for (int i = 0; i < 4; ++i) ok = ok && hipMalloc(&c->b.act[i], npx * 32 * 2) == hipSuccess;
    for (int i = 0; i < 2; ++i) ok = ok && hipMalloc(&c->b.dact[i], npx * 32 * 2) == hipSuccess;
    ok = ok && hipMalloc(&c->b.o5, npx * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc(&c->b.d5, npx * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc(&c->ph, npx * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc(&c->b.part, (size_t)nblk * (32 * 32 * 9 + 32) * sizeof(float)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        cnn_free_images(c);
        return fail(HOLO_ENOMEM, "network buffers for %lld x %lld", (long long)nx, (long long)ny);
    }
    c->img_px = npx;
    c->img_rows = nblk;
    c->b.rows_per_block = rpb;
    return HOLO_OK;
}

holo_status cnn_check(const holo_cnn* c, int64_t nx, int64_t ny)
{
    if (!c) return fail(HOLO_EINVAL, "network is NULL");
    if (!cnn_size_ok(nx) || !cnn_size_ok(ny))
        return fail(HOLO_EUNSUPPORTED, "network images must be powers of two in [64, 2048]");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if (device != c->device) return fail(HOLO_EINVAL, "network lives on device %d", c->device);
    return HOLO_OK;
}
}  // namespace
}  // namespace holo

int32_t holo_cnn_nparams(void) { return CnnLayout().n; }

holo_status holo_cnn_create(uint64_t seed, holo_cnn** out)
{
    CallGuard call_guard;   // see g_call_mu
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    *out = nullptr;
    holo_cnn* c = new holo_cnn();
    HIP_TRY(hipGetDevice(&c->device));
    const int n = c->lay.n;
    for (int l = 0; l < 5; ++l) c->b.off[l] = c->lay.off[l];
    // He-uniform initialisation from SplitMix64: w ~ U(-a, a), a = sqrt(6 / fan_in); biases 0
    std::vector<float> p(n, 0.0f);
    uint64_t st = seed;
    for (int l = 0; l < 5; ++l) {
        const int ci = l == 0 ? 1 : kCnnC, co = l == 4 ? 2 : kCnnC;
        const double a = std::sqrt(6.0 / (9.0 * ci));
        for (int j = 0; j < co * ci * 9; ++j) {
            const double u = (double)(splitmix64(st) >> 11) * 0x1.0p-53;
            p[c->lay.off[l] + j] = (float)((2.0 * u - 1.0) * a);
        }
    }
    bool ok = hipMalloc(&c->b.params, n * 4) == hipSuccess && hipMalloc(&c->b.m, n * 4) == hipSuccess &&
              hipMalloc(&c->b.v, n * 4) == hipSuccess && hipMalloc(&c->b.grad, n * 4) == hipSuccess &&
              hipMalloc(&c->b.loss_part, 256 * 3 * 8) == hipSuccess && hipMalloc(&c->b.zsum, 5 * 8) == hipSuccess &&
              hipMalloc(&c->b.w5, 9 * 16 * 2 * 4) == hipSuccess;
    for (int i = 0; i < 3 && ok; ++i)
        ok = hipMalloc(&c->b.wf[i], 32 * 32 * 9 * 2) == hipSuccess && hipMalloc(&c->b.wt[i], 32 * 32 * 9 * 2) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        holo_cnn_free(c);
        return fail(HOLO_ENOMEM, "network parameters");
    }
    HIP_TRY(hipMemcpy(c->b.params, p.data(), n * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(c->b.m, 0, n * 4));
    HIP_TRY(hipMemset(c->b.v, 0, n * 4));
    HIP_TRY(cnn_launch_pack(c->b, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    *out = c;
    return HOLO_OK;
}

holo_status holo_cnn_get_params(const holo_cnn* c, float* host_out, int32_t n)
{
    CallGuard call_guard;   // see g_call_mu
    if (!c || !host_out) return fail(HOLO_EINVAL, "network and out are required");
    if (n != c->lay.n) return fail(HOLO_EINVAL, "network has %d parameters, not %d", c->lay.n, n);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(host_out, c->b.params, (size_t)n * 4, hipMemcpyDeviceToHost));
    return HOLO_OK;
}

holo_status holo_cnn_set_params(holo_cnn* c, const float* host_in, int32_t n)
{
    CallGuard call_guard;   // see g_call_mu
    if (!c || !host_in) return fail(HOLO_EINVAL, "network and parameters are required");
    if (n != c->lay.n) return fail(HOLO_EINVAL, "network has %d parameters, not %d", c->lay.n, n);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(c->b.params, host_in, (size_t)n * 4, hipMemcpyHostToDevice));
    HIP_TRY(cnn_launch_pack(c->b, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return HOLO_OK;
}

holo_status holo_cnn_infer(holo_cnn* c, const float* target, int64_t nx, int64_t ny, float* phasor_out,
                           void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    holo_status st = cnn_check(c, nx, ny);
    if (st) return st;
    if (!target || !phasor_out) return fail(HOLO_EINVAL, "target and phasor_out are required");
    if ((st = cnn_images(c, nx, ny))) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    LAUNCH("cnn_forward", s, cnn_launch_forward(c->b, target, (int)ny, (int)nx, (float2*)phasor_out, s));
    return HOLO_OK;
}

holo_status holo_cnn_loss_grad(holo_cnn* c, const float* target, const float* label, int64_t nx, int64_t ny,
                               double* loss_out, float* grad_out, void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    holo_status st = cnn_check(c, nx, ny);
    if (st) return st;
    if (!target || !label) return fail(HOLO_EINVAL, "target and label are required");
    if ((st = cnn_images(c, nx, ny))) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = (int)(nx * ny);
    LAUNCH("cnn_forward", s, cnn_launch_forward(c->b, target, (int)ny, (int)nx, c->ph, s));
    LAUNCH("cnn_loss", s, cnn_launch_loss(c->b, target, (const float2*)label, c->ph, n, 0, 1.0, s));
    LAUNCH("cnn_backward", s, cnn_launch_backward(c->b, target, (const float2*)label, (int)ny, (int)nx, 1.0f, 0, s));
    if (loss_out) {
        HIP_TRY(hipMemcpyAsync(loss_out, c->b.zsum + 3, 8, hipMemcpyDeviceToHost, s));
    }
    if (grad_out) {
        HIP_TRY(hipMemcpyAsync(grad_out, c->b.grad, (size_t)c->lay.n * 4, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return HOLO_OK;
}

holo_status holo_cnn_train_step(holo_cnn* c, const float* targets, const float* labels, int32_t batch, int64_t nx,
                                int64_t ny, float lr, double* loss_out, void* hip_stream)
{
    CallGuard call_guard;   // see g_call_mu
    holo_status st = cnn_check(c, nx, ny);
    if (st) return st;
    if (!targets || !labels) return fail(HOLO_EINVAL, "targets and labels are required");
    if (batch < 1) return fail(HOLO_EINVAL, "batch must be >= 1 (got %d)", batch);
    if (!(lr > 0.0f)) return fail(HOLO_EINVAL, "lr must be > 0");
    if ((st = cnn_images(c, nx, ny))) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = (int)(nx * ny);
    const double inv_b = 1.0 / batch;
    for (int i = 0; i < batch; ++i) {
        const float* t = targets + (size_t)i * n;
        const float2* q = reinterpret_cast<const float2*>(labels) + (size_t)i * n;
        LAUNCH("cnn_forward", s, cnn_launch_forward(c->b, t, (int)ny, (int)nx, c->ph, s));
        LAUNCH("cnn_loss", s, cnn_launch_loss(c->b, t, q, c->ph, n, i > 0, inv_b, s));
        LAUNCH("cnn_backward", s, cnn_launch_backward(c->b, t, q, (int)ny, (int)nx, (float)inv_b, i > 0, s));
    }
    c->step += 1;
    LAUNCH("cnn_adam", s, cnn_launch_adam(c->b, c->lay.n, lr, c->step, s));
    if (loss_out) {
        HIP_TRY(hipMemcpyAsync(loss_out, c->b.zsum + 4, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return HOLO_OK;
}

holo_status holo_cnn_save(const holo_cnn* c, const char* path)
{
    CallGuard call_guard;   // see g_call_mu
    if (!c || !path) return fail(HOLO_EINVAL, "network and path are required");
    const int n = c->lay.n;
    std::vector<float> buf((size_t)3 * n);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(buf.data(), c->b.params, n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(buf.data() + n, c->b.m, n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(buf.data() + 2 * n, c->b.v, n * 4, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(HOLO_EINVAL, "cannot write %s", path);
    const char magic[8] = {'H', 'O', 'L', 'O', 'C', 'N', 'N', '1'};
    int32_t hdr[2] = {n, c->step};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    return ok ? HOLO_OK : fail(HOLO_EINVAL, "short write to %s", path);
}

holo_status holo_cnn_load(const char* path, holo_cnn** out)
{
    CallGuard call_guard;   // see g_call_mu
    if (!path || !out) return fail(HOLO_EINVAL, "path and out are required");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(HOLO_EINVAL, "cannot read %s", path);
    char magic[8];
    int32_t hdr[2];
    const int n = CnnLayout().n;
    std::vector<float> buf((size_t)3 * n);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "HOLOCNN1", 8) == 0 &&
              std::fread(hdr, 4, 2, f) == 2 && hdr[0] == n && std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(HOLO_EINVAL, "%s is not a saved network", path);
    holo_cnn* c = nullptr;
    holo_status st = holo_cnn_create(0, &c);
    if (st) return st;
    HIP_TRY(hipMemcpy(c->b.params, buf.data(), n * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->b.m, buf.data() + n, n * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->b.v, buf.data() + 2 * n, n * 4, hipMemcpyHostToDevice));
    HIP_TRY(cnn_launch_pack(c->b, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    c->step = hdr[1];
    *out = c;
    return HOLO_OK;
}

void holo_cnn_free(holo_cnn* c)
{
    CallGuard call_guard;   // see g_call_mu
    if (!c) return;
    (void)hipDeviceSynchronize();
    cnn_free_images(c);
    (void)hipFree(c->b.params), (void)hipFree(c->b.m), (void)hipFree(c->b.v), (void)hipFree(c->b.grad);
    (void)hipFree(c->b.loss_part), (void)hipFree(c->b.zsum), (void)hipFree(c->b.w5);
    for (int i = 0; i < 3; ++i) (void)hipFree(c->b.wf[i]), (void)hipFree(c->b.wt[i]);
    delete c;
}

holo_status holo_prof_enable(int32_t on)
{
    CallGuard call_guard;   // see g_call_mu
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return HOLO_OK;
}

holo_status holo_prof_read(const char* kernel, double* total_ms, int64_t* count)
{
    CallGuard call_guard;   // see g_call_mu
    if (!kernel || !total_ms || !count) return fail(HOLO_EINVAL, "kernel, total_ms and count are required");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    auto it = g_prof_tot.find(kernel);
    *total_ms = it == g_prof_tot.end() ? 0.0 : it->second.first;
    *count = it == g_prof_tot.end() ? 0 : it->second.second;
    return HOLO_OK;
}

void holo_prof_reset(void)
{
    CallGuard call_guard;   // see g_call_mu
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    g_prof_tot.clear();
}

void holo_shutdown(void)
{
    std::unique_lock<std::shared_mutex> calls(g_call_mu);   // no call in flight
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_dev) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        for (auto& t : kv.second.twiddles) (void)hipFree(t.second);
        for (auto& t : kv.second.dftops) (void)hipFree(t.second);
        for (auto& w : kv.second.workspaces)
            if (w.second.base) (void)hipFree(w.second.base);
    }
    g_dev.clear();
    for (auto& kv : g_batch_sync) {
        for (int i = 0; i < kBranches; ++i) {
            if (kv.second.br[i]) (void)hipStreamDestroy(kv.second.br[i]);
            if (kv.second.join[i]) (void)hipEventDestroy(kv.second.join[i]);
        }
        if (kv.second.fork) (void)hipEventDestroy(kv.second.fork);
    }
    g_batch_sync.clear();
    {
        std::lock_guard<std::mutex> gl(g_graph_mu);
        for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
        g_graphs.clear();
        for (auto& kv : g_graph_bufs) (void)hipFree(kv.second);
        g_graph_bufs.clear();
        g_graph_streams.clear();
        g_graph_order.clear();
    }
    (void)hipSetDevice(cur);
}

}  // extern "C"
