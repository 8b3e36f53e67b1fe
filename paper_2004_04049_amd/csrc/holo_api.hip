// holo_api.hip -- host side of the C ABI declared in include/holo.h:
// argument validation, LUT tables, per-device twiddle tables, per-stream
// workspaces and the launch sequences of the OSPR, GS and reconstruction
// paths.  All arithmetic on image data runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/holo.h"
#include "kernels.hpp"

struct holo_lut {
    int device;
    uint64_t n_lut;              // as requested (0 = flat)
    uint32_t n_dev;              // entries on the device (>= 1)
    std::vector<double> phases;  // FP64 phases, host copy
    float2* dev;                 // FP32 unit phasors on `device`
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

struct Workspace {
    void* base = nullptr;
    size_t cap = 0;
};

struct DeviceState {
    std::map<int, float2*> twiddles;                   // length -> W_N^k table
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

// Scratch of at least `bytes` for (device, stream); grows by reallocation
// after the stream has drained (the only user of the old buffer).
holo_status get_workspace(int device, hipStream_t s, size_t bytes, void** out)
{
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

struct ProfScope {
    const char* name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* n, hipStream_t st) : name(n), s(st)
    {
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

}  // namespace
}  // namespace holo

using namespace holo;

extern "C" {

const char* holo_last_error(void) { return g_err.c_str(); }
int32_t holo_version(void) { return 1; }

holo_status holo_lut_from_phases(const double* phases, uint64_t n_lut, holo_lut** out)
{
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_lut && !phases) return fail(HOLO_EINVAL, "phases is NULL");
    if (n_lut >= (1ull << 31)) return fail(HOLO_EUNSUPPORTED, "n_lut %llu >= 2^31", (unsigned long long)n_lut);
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_lut* l = new holo_lut();
    l->device = device;
    l->n_lut = n_lut;
    l->n_dev = n_lut ? (uint32_t)n_lut : 1u;
    l->phases.assign(phases, phases + n_lut);
    std::vector<float2> ph(l->n_dev);
    if (n_lut == 0) ph[0] = make_float2(1.0f, 0.0f);
    for (uint64_t j = 0; j < n_lut; ++j) ph[j] = make_float2((float)std::cos(phases[j]), (float)std::sin(phases[j]));
    if (hipMalloc(&l->dev, sizeof(float2) * l->n_dev) != hipSuccess) {
        (void)hipGetLastError();
        delete l;
        return fail(HOLO_ENOMEM, "LUT of %u entries", l->n_dev);
    }
    hipError_t e = hipMemcpy(l->dev, ph.data(), sizeof(float2) * l->n_dev, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(l->dev);
        delete l;
        return fail(HOLO_EDEVICE, "LUT upload: %s", hipGetErrorString(e));
    }
    *out = l;
    return HOLO_OK;
}

holo_status holo_lut_build(uint64_t n_lut, uint64_t seed, holo_lut** out)
{
    if (!out) return fail(HOLO_EINVAL, "out is NULL");
    if (n_lut >= (1ull << 31)) return fail(HOLO_EUNSUPPORTED, "n_lut %llu >= 2^31", (unsigned long long)n_lut);
    std::vector<double> phi(n_lut);
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t s = seed;
    for (uint64_t j = 0; j < n_lut; ++j) {
        const uint64_t x = splitmix64(s);
        phi[j] = two_pi * ((double)(x >> 11) * 0x1.0p-53);
    }
    return holo_lut_from_phases(phi.data(), n_lut, out);
}

holo_status holo_lut_phases(const holo_lut* lut, double* out, uint64_t n)
{
    if (!lut || (!out && n)) return fail(HOLO_EINVAL, "lut/out is NULL");
    uint64_t m = n < lut->n_lut ? n : lut->n_lut;
    if (m) std::memcpy(out, lut->phases.data(), m * sizeof(double));
    return HOLO_OK;
}

uint64_t holo_lut_size(const holo_lut* lut) { return lut ? lut->n_lut : 0; }

void holo_lut_free(holo_lut* lut)
{
    if (!lut) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(lut->device);
    (void)hipFree(lut->dev);
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

holo_status holo_ospr_generate(const float* target, int64_t nx, int64_t ny, int32_t n_sf, const holo_lut* lut,
                               uint64_t* cursor, uint32_t* holo_bits, float* recon, double* nmse2,
                               int32_t precision, uint32_t flags, void* hip_stream)
{
    if (!target || !cursor || !holo_bits) return fail(HOLO_EINVAL, "target, cursor and holo_bits are required");
    if (n_sf < 1) return fail(HOLO_EINVAL, "n_sf must be >= 1 (got %d)", n_sf);
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048] (got %lld x %lld)",
                    (long long)nx, (long long)ny);
    if (precision != HOLO_FP32) return fail(HOLO_EUNSUPPORTED, "holo_ospr_generate computes in FP32 only");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    holo_status st = check_lut(lut, device);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)ny, s, &tw_y))) return st;

    const size_t npix = (size_t)nx * (size_t)ny;
    const size_t nspec = (size_t)(ny / 2 + 1) * (size_t)nx;
    Carver cv;
    const size_t o_x1 = cv.take(sizeof(float2) * npix * n_sf);
    const size_t o_x2 = cv.take(sizeof(float2) * nspec * n_sf);
    const size_t o_part = cv.take(sizeof(double) * 5 * (size_t)(ny / 2 + 1));
    const size_t o_nm = cv.take(sizeof(double) * 2);
    void* ws;
    if ((st = get_workspace(device, s, cv.off, &ws))) return st;
    char* b = (char*)ws;
    float2* x1 = (float2*)(b + o_x1);
    float2* x2 = (float2*)(b + o_x2);
    double* part = (double*)(b + o_part);
    double* nm = (double*)(b + o_nm);

    const uint32_t L = lut->n_dev;
    const uint64_t c0 = *cursor % L;
    const LaunchCfg cfg = default_cfg();
    LAUNCH("ospr_rows", s, launch_ospr_rows(target, (int)nx, (int)ny, n_sf, lut->dev, L, c0, x1, tw_x, cfg, s));
    LAUNCH("ospr_cols", s, launch_ospr_cols(x1, (int)nx, (int)ny, n_sf, holo_bits, x2, tw_y, cfg, s));
    LAUNCH("recon_rows", s, launch_recon_rows(x2, (int)nx, (int)ny, n_sf, true, target, recon, part, tw_x, cfg, s));
    LAUNCH("nmse_finalize", s, launch_nmse_finalize(part, (int)(ny / 2 + 1), nm, s));
    if ((st = copy_out(nmse2, nm, 2, flags, s))) return st;
    *cursor += (uint64_t)n_sf * (uint64_t)npix;
    return HOLO_OK;
}

holo_status holo_reconstruct_nmse(const void* holo, int32_t levels, int64_t nx, int64_t ny, int32_t n_sf,
                                  const float* target, float* recon, double* nmse2, uint32_t flags,
                                  void* hip_stream)
{
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
    const size_t o_x2 = cv.take(sizeof(float2) * (size_t)nrows * nx * n_sf);
    const size_t o_part = cv.take(sizeof(double) * 5 * (size_t)nrows);
    const size_t o_nm = cv.take(sizeof(double) * 2);
    void* ws;
    if ((st = get_workspace(device, s, cv.off, &ws))) return st;
    char* b = (char*)ws;
    float2* x2 = (float2*)(b + o_x2);
    double* part = (double*)(b + o_part);
    double* nm = (double*)(b + o_nm);
    const LaunchCfg cfg = default_cfg();
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
    hipStream_t s = (hipStream_t)hip_stream;
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)ny, s, &tw_y))) return st;

    const size_t npix = (size_t)nx * (size_t)ny;
    Carver cv;
    const size_t o_state = cv.take(sizeof(float2) * npix);
    const size_t o_field = cv.take(field ? 0 : sizeof(float2) * npix);
    const size_t o_pinit = cv.take(sizeof(double) * 2 * ny);
    const size_t o_piter = cv.take(sizeof(double) * 3 * ny * (size_t)n_iter);
    const size_t o_consts = cv.take(sizeof(GsConsts));
    const size_t o_nm = cv.take(sizeof(double) * n_iter);
    const size_t o_er = cv.take(sizeof(double) * n_iter);
    const size_t o_x2 = cv.take(codes ? sizeof(float2) * npix : 0);
    const size_t o_p5 = cv.take(sizeof(double) * 5 * ny);
    const size_t o_f2 = cv.take(sizeof(double) * 2);
    void* ws;
    if ((st = get_workspace(device, s, cv.off, &ws))) return st;
    char* b = (char*)ws;
    float2* state = (float2*)(b + o_state);
    float2* fout = field ? (float2*)field : (float2*)(b + o_field);
    double* pinit = (double*)(b + o_pinit);
    double* piter = (double*)(b + o_piter);
    GsConsts* consts = (GsConsts*)(b + o_consts);
    double* nm = (double*)(b + o_nm);
    double* er = (double*)(b + o_er);

    const bool use_lut = init_phasor == nullptr;
    const uint32_t L = use_lut ? lut->n_dev : 1u;
    const uint64_t c0 = use_lut ? *cursor % L : 0;
    const float2* lutp = use_lut ? lut->dev : nullptr;
    const LaunchCfg cfg = default_cfg();
    const int inx = (int)nx, iny = (int)ny;
    LAUNCH("gs_rows", s, launch_gs_rows(GS_INIT, target, inx, iny, lutp, L, c0, (const float2*)init_phasor, state, nullptr,
                           pinit, consts, tw_x, cfg, s));
    LAUNCH("gs_consts", s, launch_gs_consts(pinit, iny, inx, consts, s));
    for (int it = 0; it < n_iter; ++it) {
        const bool last = it == n_iter - 1;
        LAUNCH("gs_cols", s, launch_gs_cols(state, inx, iny, last ? codes : nullptr, tw_y, cfg, s));
        LAUNCH("gs_rows", s, launch_gs_rows(last ? GS_FINAL : GS_ITER, target, inx, iny, lutp, L, c0, nullptr, state, fout,
                               piter + (size_t)it * 3 * ny, consts, tw_x, cfg, s));
    }
    LAUNCH("gs_finalize", s, launch_gs_finalize(piter, n_iter, iny, consts, nm, er, s));
    if (codes && (nmse_final2 || recon)) {
        float2* x2 = (float2*)(b + o_x2);
        double* p5 = (double*)(b + o_p5);
        double* f2 = (double*)(b + o_f2);
        LAUNCH("recon_cols", s, launch_recon_cols(codes, 8, inx, iny, 1, x2, tw_y, cfg, s));
        LAUNCH("recon_rows", s, launch_recon_rows(x2, inx, iny, 1, false, target, recon, p5, tw_x, cfg, s));
        LAUNCH("nmse_finalize", s, launch_nmse_finalize(p5, iny, f2, s));
        if ((st = copy_out(nmse_final2, f2, 2, flags, s))) return st;
    }
    if ((st = copy_out(nmse_per_iter, nm, n_iter, flags, s))) return st;
    if ((st = copy_out(err_per_iter, er, n_iter, flags, s))) return st;
    if (use_lut) *cursor += npix;
    return HOLO_OK;
}

holo_status holo_fft2(const float* in, float* out, int64_t nx, int64_t ny, int32_t sign, void* hip_stream)
{
    if (!in || !out) return fail(HOLO_EINVAL, "in and out are required");
    if (sign != 1 && sign != -1) return fail(HOLO_EINVAL, "sign must be +1 or -1");
    if (!pow2_in_range(nx) || !pow2_in_range(ny))
        return fail(HOLO_EUNSUPPORTED, "nx, ny must be powers of two in [16, 2048]");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    hipStream_t s = (hipStream_t)hip_stream;
    holo_status st;
    const float2 *tw_x, *tw_y;
    if ((st = get_twiddles(device, (int)nx, s, &tw_x))) return st;
    if ((st = get_twiddles(device, (int)ny, s, &tw_y))) return st;
    void* ws;
    if ((st = get_workspace(device, s, sizeof(float2) * (size_t)nx * ny, &ws))) return st;
    LAUNCH("fft2", s, launch_fft2((const float2*)in, (float2*)ws, (float2*)out, (int)nx, (int)ny, sign, tw_x, tw_y,
                        default_cfg(), s));
    return HOLO_OK;
}

holo_status holo_prof_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return HOLO_OK;
}

holo_status holo_prof_read(const char* kernel, double* total_ms, int64_t* count)
{
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
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    g_prof_tot.clear();
}

void holo_shutdown(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_dev) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        for (auto& t : kv.second.twiddles) (void)hipFree(t.second);
        for (auto& w : kv.second.workspaces)
            if (w.second.base) (void)hipFree(w.second.base);
    }
    g_dev.clear();
    (void)hipSetDevice(cur);
}

}  // extern "C"
