// C ABI of libnbody.so (declared in include/nbody.h): argument checks,
// device checks, workspace cache, variant choice and tuning table.
#include "common.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

namespace nbody {

// ---------------------------------------------------------------- errors

namespace {
thread_local std::string t_last_error;
}

void clear_error() { t_last_error.clear(); }
const char *last_error_cstr() { return t_last_error.c_str(); }

nbody_status fail(nbody_status status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return status;
}

nbody_status hip_fail(hipError_t err, const char *what)
{
    const nbody_status st = (err == hipErrorOutOfMemory) ? NBODY_ERROR_OUT_OF_MEMORY
                            : (err == hipErrorInvalidDeviceFunction || err == hipErrorLaunchFailure ||
                               err == hipErrorInvalidConfiguration)
                                ? NBODY_ERROR_LAUNCH_FAILED
                                : NBODY_ERROR_INTERNAL;
    return fail(st, "%s: %s (%d)", what, hipGetErrorString(err), (int)err);
}

nbody_status check_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return NBODY_OK;
    nbody_status st = hip_fail(e, what);
    if (st == NBODY_ERROR_INTERNAL) st = NBODY_ERROR_LAUNCH_FAILED;
    return st;
}

bool fault_injected(const char *what)
{
    const char *env = std::getenv("NBODY_FAULT");
    return env && std::strcmp(env, what) == 0;
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// ---------------------------------------------------------------- devices

namespace {
struct DeviceState {
    bool probed = false;
    bool supported = false;
    int num_cu = 0;
    std::string arch;
};
std::mutex g_dev_mu;
std::map<int, DeviceState> g_devices;
}  // namespace

nbody_status current_device(Device *dev)
{
    int id = -1;
    hipError_t e = hipGetDevice(&id);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_dev_mu);
    DeviceState &d = g_devices[id];
    if (!d.probed) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, id);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        d.arch = prop.gcnArchName;
        d.supported = d.arch.compare(0, 6, "gfx950") == 0;
        d.num_cu = prop.multiProcessorCount;
        d.probed = true;
    }
    if (!d.supported)
        return fail(NBODY_ERROR_UNSUPPORTED_DEVICE, "device %d is %s; libnbody is built for gfx950",
                    id, d.arch.c_str());
    dev->id = id;
    dev->num_cu = d.num_cu;
    return NBODY_OK;
}

// ---------------------------------------------------------------- workspace

namespace {
struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
// (device, stream, 0 for workspace() or 1 for workspace_aux())
std::map<std::tuple<int, hipStream_t, int>, Buffer> g_ws;

nbody_status grow_buffer(const Device &dev, hipStream_t stream, int slot, size_t bytes, void **ptr)
{
    if (fault_injected("alloc")) return fail(NBODY_ERROR_OUT_OF_MEMORY, "injected allocation fault");
    std::lock_guard<std::mutex> lock(g_ws_mu);
    Buffer &b = g_ws[{dev.id, stream, slot}];
    if (b.bytes < bytes) {
        if (b.ptr) {
            // hipFree waits for the device, so kernels still reading the old
            // buffer on this stream finish first.
            hipError_t e = hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
        }
        const size_t grow = std::max(bytes, (size_t)1 << 20);
        hipError_t e = hipMalloc(&b.ptr, grow);
        if (e != hipSuccess) {
            b.ptr = nullptr;
            return hip_fail(e, "hipMalloc(workspace)");
        }
        b.bytes = grow;
    }
    *ptr = b.ptr;
    return NBODY_OK;
}
}  // namespace

nbody_status workspace(const Device &dev, hipStream_t stream, size_t bytes, void **ptr)
{
    return grow_buffer(dev, stream, 0, bytes, ptr);
}

nbody_status workspace_aux(const Device &dev, hipStream_t stream, size_t bytes, void **ptr)
{
    return grow_buffer(dev, stream, 1, bytes, ptr);
}

size_t workspace_size(const Device &dev, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto it = g_ws.find({dev.id, stream, 0});
    return it == g_ws.end() ? 0 : it->second.bytes;
}

nbody_status workspace_trim(const Device &dev, hipStream_t stream, size_t bytes)
{
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto it = g_ws.find({dev.id, stream, 0});
    if (it == g_ws.end() || it->second.bytes <= bytes) return NBODY_OK;
    Buffer &b = it->second;
    hipError_t e = hipFree(b.ptr);  // waits for the device
    b.ptr = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
    if (bytes == 0) return NBODY_OK;
    e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return hip_fail(e, "hipMalloc(workspace)");
    }
    b.bytes = bytes;
    return NBODY_OK;
}

size_t tune_workspace_cap(size_t free_bytes)
{
    size_t cap = (size_t)2 << 30;
    if (const char *env = std::getenv("NBODY_TUNE_WORKSPACE_CAP")) {
        const unsigned long long v = std::strtoull(env, nullptr, 10);
        if (v > 0) cap = (size_t)v;
    }
    return std::min(cap, free_bytes / 4);
}

namespace {
struct CounterBuf {
    int *ptr = nullptr;
    size_t count = 0;
};
std::mutex g_cnt_mu;
std::map<std::pair<int, hipStream_t>, CounterBuf> g_cnt;
}  // namespace

nbody_status counters(const Device &dev, hipStream_t stream, size_t count, int **ptr)
{
    if (fault_injected("alloc")) return fail(NBODY_ERROR_OUT_OF_MEMORY, "injected allocation fault");
    std::lock_guard<std::mutex> lock(g_cnt_mu);
    CounterBuf &b = g_cnt[{dev.id, stream}];
    if (b.count < count) {
        if (b.ptr) {
            hipError_t e = hipFree(b.ptr);  // waits for the device
            b.ptr = nullptr;
            b.count = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFree(counters)");
        }
        const size_t grow = std::max(count, (size_t)256);
        hipError_t e = hipMalloc(&b.ptr, grow * sizeof(int));
        if (e != hipSuccess) {
            b.ptr = nullptr;
            return hip_fail(e, "hipMalloc(counters)");
        }
        nbody_status st = fill_zero_int(b.ptr, grow, stream);
        if (st != NBODY_OK) {
            (void)hipFree(b.ptr);
            b.ptr = nullptr;
            return st;
        }
        b.count = grow;
    }
    *ptr = b.ptr;
    return NBODY_OK;
}

nbody_status Arena::get(const Device &dev, hipStream_t stream, size_t bytes, void **ptr) const
{
    if (!base) return workspace(dev, stream, bytes, ptr);
    if (bytes > cap)
        return fail(NBODY_ERROR_INVALID_ARGUMENT,
                    "the call needs %zu bytes of workspace; the fixed region holds %zu", bytes, cap);
    *ptr = base;
    return NBODY_OK;
}

nbody_status Arena::get_counters(const Device &dev, hipStream_t stream, size_t count, int **ptr) const
{
    if (!base) return nbody::counters(dev, stream, count, ptr);
    if (count > counter_count)
        return fail(NBODY_ERROR_INVALID_ARGUMENT,
                    "the call needs %zu counters; the fixed region holds %zu", count, counter_count);
    *ptr = counters;
    return NBODY_OK;
}

// ---------------------------------------------------------------- profiling

namespace {
constexpr size_t kProfCalls = 256;
std::atomic<bool> g_prof_on{false};
// One recorded call: an event before and after each of its pair kernels
// (a call may launch several), and one after its last kernel.
struct ProfCall {
    std::vector<hipEvent_t> pair;  // begin, end, begin, end, ...
    hipEvent_t end = nullptr;
};
struct ProfState {
    int device = -1;
    std::vector<hipEvent_t> pool;  // free events of `device`
    std::deque<ProfCall> calls;    // finished calls, oldest first
    ProfCall cur;                  // the call being recorded
    bool pending = false;          // cur holds a pair kernel's events
    void give(ProfCall &c)
    {
        for (hipEvent_t e : c.pair) pool.push_back(e);
        if (c.end) pool.push_back(c.end);
        c.pair.clear();
        c.end = nullptr;
    }
    void clear()
    {
        for (auto &c : calls) give(c);
        calls.clear();
        give(cur);
        pending = false;
    }
    void destroy()
    {
        clear();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
    hipEvent_t take()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        return hipEventCreate(&e) == hipSuccess ? e : nullptr;
    }
    ~ProfState() { destroy(); }
};
thread_local ProfState t_prof;
}  // namespace

void prof_mark(hipStream_t stream, int which)
{
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return;
    if (t_prof.device != dev) {
        t_prof.destroy();
        t_prof.device = dev;
    }
    if (which < 0) {  // a new call begins: drop what a failed call left
        t_prof.give(t_prof.cur);
        t_prof.pending = false;
        return;
    }
    if (which == 1 && !t_prof.pending) return;
    if (which == 2) {
        if (!t_prof.pending) return;  // a call that launched no pair kernel is not recorded
        hipEvent_t e = t_prof.take();
        if (!e) return;
        (void)hipEventRecord(e, stream);
        t_prof.cur.end = e;
        t_prof.calls.push_back(std::move(t_prof.cur));
        t_prof.cur = ProfCall{};
        t_prof.pending = false;
        if (t_prof.calls.size() > kProfCalls) {
            t_prof.give(t_prof.calls.front());
            t_prof.calls.pop_front();
        }
        return;
    }
    hipEvent_t e = t_prof.take();
    if (!e) return;
    (void)hipEventRecord(e, stream);
    t_prof.cur.pair.push_back(e);
    if (which == 0) t_prof.pending = true;
}

// ---------------------------------------------------------------- variants

namespace {
std::mutex g_var_mu;
int g_forced[3] = {-1, -1, -1};
bool g_env_read = false;
std::map<std::pair<int, int>, std::string> g_tuned;  // (kind, log2 bucket) -> variant name
bool g_cache_read = false;

int variant_count(int kind)
{
    switch (kind) {
    case NBODY_KIND_FORWARD: return forward_variant_count();
    case NBODY_KIND_BACKWARD: return backward_variant_count();
    case NBODY_KIND_BATCHED: return batched_variant_count();
    default: return 0;
    }
}

const char *variant_name(int kind, int index)
{
    switch (kind) {
    case NBODY_KIND_FORWARD: return forward_variant_name(index);
    case NBODY_KIND_BACKWARD: return backward_variant_name(index);
    case NBODY_KIND_BATCHED: return batched_variant_name(index);
    default: return nullptr;
    }
}

int bucket_of(int64_t n)
{
    int b = 0;
    while (n > 1) {
        n >>= 1;
        ++b;
    }
    return b;
}

// NBODY_VARIANT=<kind>:<index>[,<kind>:<index>...]
void read_env_locked()
{
    if (g_env_read) return;
    g_env_read = true;
    const char *env = std::getenv("NBODY_VARIANT");
    if (!env) return;
    std::string s(env);
    size_t pos = 0;
    while (pos < s.size()) {
        size_t end = s.find(',', pos);
        if (end == std::string::npos) end = s.size();
        int kind = -1, index = -1;
        if (std::sscanf(s.substr(pos, end - pos).c_str(), "%d:%d", &kind, &index) == 2 &&
            kind >= 0 && kind < 3 && index >= 0 && index < variant_count(kind))
            g_forced[kind] = index;
        pos = end + 1;
    }
}

// Tuning cache file: one entry per line,
//   {"kind": K, "bucket": B, "variant": "name"}
void read_cache_locked()
{
    if (g_cache_read) return;
    g_cache_read = true;
    const char *path = std::getenv("NBODY_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        int kind = -1, bucket = -1;
        char name[128] = {0};
        const char *p = std::strstr(line, "\"kind\"");
        if (!p) continue;
        if (std::sscanf(p, "\"kind\": %d, \"bucket\": %d, \"variant\": \"%127[^\"]\"", &kind,
                        &bucket, name) == 3)
            g_tuned[{kind, bucket}] = name;
    }
    std::fclose(f);
}

void write_cache_locked()
{
    const char *path = std::getenv("NBODY_TUNE_CACHE");
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\"entries\": [\n");
    size_t k = 0;
    for (const auto &kv : g_tuned) {
        std::fprintf(f, "  {\"kind\": %d, \"bucket\": %d, \"variant\": \"%s\"}%s\n", kv.first.first,
                     kv.first.second, kv.second.c_str(), (++k < g_tuned.size()) ? "," : "");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

int index_of(int kind, const std::string &name)
{
    for (int k = 0; k < variant_count(kind); ++k)
        if (name == variant_name(kind, k)) return k;
    return -1;
}
}  // namespace

int forced_variant(int kind)
{
    std::lock_guard<std::mutex> lock(g_var_mu);
    read_env_locked();
    return (kind >= 0 && kind < 3) ? g_forced[kind] : -1;
}

int tuned_variant(int kind, int64_t n)
{
    std::lock_guard<std::mutex> lock(g_var_mu);
    read_cache_locked();
    auto it = g_tuned.find({kind, bucket_of(n)});
    if (it == g_tuned.end()) return -1;
    return index_of(kind, it->second);
}

void record_tuned_variant(int kind, int64_t n, int index)
{
    std::lock_guard<std::mutex> lock(g_var_mu);
    read_cache_locked();
    g_tuned[{kind, bucket_of(n)}] = variant_name(kind, index);
    write_cache_locked();
}

int select_variant(int kind, int64_t n)
{
    int v = forced_variant(kind);
    if (v >= 0) return v;
    v = tuned_variant(kind, n);
    if (v >= 0) return v;
    switch (kind) {
    case NBODY_KIND_FORWARD: return forward_default_variant(n);
    case NBODY_KIND_BACKWARD: return backward_default_variant(n);
    default: return batched_default_variant(n);
    }
}

}  // namespace nbody

using namespace nbody;

// ====================================================================== ABI

bool nbody::bad_eps2(float eps2) { return !(eps2 >= 0.0f) || std::isinf(eps2); }

extern "C" {

int nbody_abi_version(void) { return NBODY_ABI_VERSION; }

const char *nbody_status_string(nbody_status status)
{
    // A C caller may pass any int; read it as one (an out-of-range value of
    // the enum type would be undefined behaviour in C++).
    int code;
    std::memcpy(&code, &status, sizeof code);
    switch (code) {
    case NBODY_OK: return "NBODY_OK";
    case NBODY_ERROR_INVALID_ARGUMENT: return "NBODY_ERROR_INVALID_ARGUMENT";
    case NBODY_ERROR_UNSUPPORTED_DEVICE: return "NBODY_ERROR_UNSUPPORTED_DEVICE";
    case NBODY_ERROR_OUT_OF_MEMORY: return "NBODY_ERROR_OUT_OF_MEMORY";
    case NBODY_ERROR_LAUNCH_FAILED: return "NBODY_ERROR_LAUNCH_FAILED";
    case NBODY_ERROR_INTERNAL: return "NBODY_ERROR_INTERNAL";
    }
    return "NBODY_ERROR_UNKNOWN";
}

const char *nbody_last_error(void) { return nbody::last_error_cstr(); }

nbody_status nbody_forces(const float *x, const float *m, int64_t n, float eps2, float *a,
                          float *p, void *stream)
{
    return nbody_forces_ex(x, m, n, eps2, a, p, 0u, stream);
}

nbody_status nbody_forces_ex(const float *x, const float *m, int64_t n, float eps2, float *a,
                             float *p, uint32_t flags, void *stream)
{
    clear_error();
    if (flags & ~(uint32_t)NBODY_FORCES_F64_SUM)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "unknown flag bits 0x%x",
                    (unsigned)(flags & ~(uint32_t)NBODY_FORCES_F64_SUM));
    if (n < 0 || n > NBODY_MAX_N)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "n = %lld outside [0, %lld]", (long long)n,
                    (long long)NBODY_MAX_N);
    if (bad_eps2(eps2)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "eps2 = %g is negative or not finite", eps2);
    if (n == 0) return NBODY_OK;
    if (!x || !m || !a) return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL x, m or a with n = %lld", (long long)n);
    const size_t v3 = 12 * (size_t)n, v1 = 4 * (size_t)n;
    if (overlaps(a, v3, x, v3) || overlaps(a, v3, m, v1) || overlaps(p, v1, x, v3) ||
        overlaps(p, v1, m, v1) || overlaps(a, v3, p, v1))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "output arrays overlap each other or the inputs");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    int variant = select_variant(NBODY_KIND_FORWARD, n);
    if ((flags & NBODY_FORCES_F64_SUM) && !forward_variant_f64sum(variant)) {
        const int forced = forced_variant(NBODY_KIND_FORWARD);
        variant = forward_variant_f64sum(forced) ? forced : forward_default_f64sum_variant(n);
    }
    prof_mark((hipStream_t)stream, -1);
    st = forward_run(variant, dev, x, m, (int)n, eps2, a, p, (hipStream_t)stream);
    if (st == NBODY_OK) prof_mark((hipStream_t)stream, 2);
    return st;
}

nbody_status nbody_forces_backward(const float *x, const float *m, int64_t n, float eps2,
                                   const float *grad_a, const float *grad_p, float *grad_x,
                                   float *grad_m, void *stream)
{
    clear_error();
    if (n < 0 || n > NBODY_MAX_N)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "n = %lld outside [0, %lld]", (long long)n,
                    (long long)NBODY_MAX_N);
    if (bad_eps2(eps2)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "eps2 = %g is negative or not finite", eps2);
    if (n == 0) return NBODY_OK;
    if (!x || !m || !grad_x)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL x, m or grad_x with n = %lld", (long long)n);
    const size_t v3 = 12 * (size_t)n, v1 = 4 * (size_t)n;
    const void *ins[4] = {x, m, grad_a, grad_p};
    const size_t inb[4] = {v3, v1, v3, v1};
    for (int k = 0; k < 4; ++k)
        if (overlaps(grad_x, v3, ins[k], inb[k]) || overlaps(grad_m, v1, ins[k], inb[k]))
            return fail(NBODY_ERROR_INVALID_ARGUMENT, "output arrays overlap the inputs");
    if (overlaps(grad_x, v3, grad_m, v1))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "grad_x and grad_m overlap");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    prof_mark((hipStream_t)stream, -1);
    st = backward_run(select_variant(NBODY_KIND_BACKWARD, n), dev, x, m, (int)n, eps2, grad_a,
                      grad_p, grad_x, grad_m, (hipStream_t)stream);
    if (st == NBODY_OK) prof_mark((hipStream_t)stream, 2);
    return st;
}

static nbody_status check_offsets(const int64_t *offsets, int64_t num_systems)
{
    if (num_systems < 0) return fail(NBODY_ERROR_INVALID_ARGUMENT, "num_systems = %lld < 0", (long long)num_systems);
    if (!offsets) return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL offsets");
    if (offsets[0] != 0) return fail(NBODY_ERROR_INVALID_ARGUMENT, "offsets[0] = %lld, must be 0", (long long)offsets[0]);
    for (int64_t s = 0; s < num_systems; ++s) {
        const int64_t ns = offsets[s + 1] - offsets[s];
        if (ns < 0)
            return fail(NBODY_ERROR_INVALID_ARGUMENT, "offsets decrease at system %lld", (long long)s);
        if (ns > NBODY_MAX_N || offsets[s + 1] > NBODY_MAX_N)
            return fail(NBODY_ERROR_INVALID_ARGUMENT, "system %lld exceeds NBODY_MAX_N", (long long)s);
    }
    return NBODY_OK;
}

nbody_status nbody_forces_batched(const int64_t *offsets, int64_t num_systems, const float *x,
                                  const float *m, float eps2, float *a, float *p, void *stream)
{
    clear_error();
    nbody_status ost = check_offsets(offsets, num_systems);
    if (ost != NBODY_OK) return ost;
    if (bad_eps2(eps2)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "eps2 = %g is negative or not finite", eps2);
    const int64_t n = offsets[num_systems];
    if (n == 0) return NBODY_OK;
    if (!x || !m || !a) return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL x, m or a with %lld particles", (long long)n);
    const size_t v3 = 12 * (size_t)n, v1 = 4 * (size_t)n;
    if (overlaps(a, v3, x, v3) || overlaps(a, v3, m, v1) || overlaps(p, v1, x, v3) ||
        overlaps(p, v1, m, v1) || overlaps(a, v3, p, v1))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "output arrays overlap each other or the inputs");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    const int64_t mean_n = num_systems > 0 ? n / num_systems : 0;
    prof_mark((hipStream_t)stream, -1);
    st = batched_run(select_variant(NBODY_KIND_BATCHED, mean_n), dev, offsets, num_systems, x,
                     m, eps2, a, p, (hipStream_t)stream);
    if (st == NBODY_OK) prof_mark((hipStream_t)stream, 2);
    return st;
}

nbody_status nbody_axpy(float *y, const float *xv, int64_t len, float alpha, void *stream)
{
    clear_error();
    if (len < 0) return fail(NBODY_ERROR_INVALID_ARGUMENT, "len = %lld < 0", (long long)len);
    if (!std::isfinite(alpha)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "alpha is not finite");
    if (len == 0) return NBODY_OK;
    if (!y || !xv) return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL y or x with len = %lld", (long long)len);
    if (overlaps(y, 4 * (size_t)len, xv, 4 * (size_t)len))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "y and x overlap");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    return axpy_run(y, xv, len, alpha, (hipStream_t)stream);
}

nbody_status nbody_kick_drift(float *x, float *v, const float *a, int64_t n, float kick, float dt,
                              void *stream)
{
    clear_error();
    if (n < 0 || n > NBODY_MAX_N) return fail(NBODY_ERROR_INVALID_ARGUMENT, "n = %lld out of range", (long long)n);
    if (!std::isfinite(kick) || !std::isfinite(dt))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "kick and dt must be finite");
    if (n == 0) return NBODY_OK;
    if (!x || !v || !a) return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL x, v or a with n = %lld", (long long)n);
    const size_t b = 12 * (size_t)n;
    if (overlaps(x, b, v, b) || overlaps(x, b, a, b) || overlaps(v, b, a, b))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "x, v and a overlap");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    return kick_drift_run(x, v, a, 3 * n, kick, dt, (hipStream_t)stream);
}

nbody_status nbody_leapfrog(float *x, float *v, float *a, const float *m, int64_t n, float eps2,
                            float dt, int64_t steps, float *x_hist, void *stream)
{
    clear_error();
    if (n < 0 || n > NBODY_MAX_N)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "n = %lld outside [0, %lld]", (long long)n,
                    (long long)NBODY_MAX_N);
    if (bad_eps2(eps2)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "eps2 = %g is negative or not finite", eps2);
    if (!std::isfinite(dt)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "dt is not finite");
    if (steps < 0 || steps > NBODY_MAX_STEPS)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "steps = %lld outside [0, %lld]", (long long)steps,
                    (long long)NBODY_MAX_STEPS);
    if (n == 0 || steps == 0) return NBODY_OK;
    if (!x || !v || !a || !m)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL x, v, a or m with n = %lld", (long long)n);
    const size_t v3 = 12 * (size_t)n, v1 = 4 * (size_t)n;
    const void *arr[5] = {x, v, a, m, x_hist};
    const size_t len[5] = {v3, v3, v3, v1, v3 * (size_t)steps};
    for (int i = 0; i < 5; ++i)
        for (int k = i + 1; k < 5; ++k)
            if (overlaps(arr[i], len[i], arr[k], len[k]))
                return fail(NBODY_ERROR_INVALID_ARGUMENT, "x, v, a, m and x_hist must not overlap");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    const int variant = select_variant(NBODY_KIND_FORWARD, n);
    const float kick = -0.5f * dt;  // half kick with the physical acceleration -a
    // start kick and drift of the first step
    LfEpi e;
    e.mode = kLfKick;
    e.kicks = 1;
    e.drift = 1;
    e.k1 = kick;
    e.k2 = kick;
    e.dt = dt;
    e.v = v;
    e.x = x;
    e.xh = x_hist;
    st = lf_epilogue_run(a, nullptr, n, e, s);
    for (int64_t t = 0; t < steps && st == NBODY_OK; ++t) {
        // a(x) of this step, its end kick and, unless it is the last step,
        // the next step's start kick and drift
        const bool last = t == steps - 1;
        e.kicks = last ? 1 : 2;
        e.drift = last ? 0 : 1;
        e.xh = (!last && x_hist) ? x_hist + 3 * (size_t)n * (size_t)(t + 1) : nullptr;
        bool fused = false;
        prof_mark(s, -1);
        st = forward_run(variant, dev, x, m, (int)n, eps2, a, nullptr, s, &e, &fused);
        if (st == NBODY_OK && !fused) st = lf_epilogue_run(a, nullptr, n, e, s);
        if (st == NBODY_OK) prof_mark(s, 2);
    }
    return st;
}

nbody_status nbody_leapfrog_adjoint(const float *pos, const float *m, int64_t n, float eps2,
                                    float dt, int64_t steps, uint32_t flags, float *lx, float *lv,
                                    float *lm, void *stream)
{
    clear_error();
    const uint32_t known = NBODY_LEAPFROG_FINAL | NBODY_LEAPFROG_INITIAL;
    if (flags & ~known)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "unknown flag bits 0x%x", (unsigned)(flags & ~known));
    if (n < 0 || n > NBODY_MAX_N)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "n = %lld outside [0, %lld]", (long long)n,
                    (long long)NBODY_MAX_N);
    if (bad_eps2(eps2)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "eps2 = %g is negative or not finite", eps2);
    if (!std::isfinite(dt)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "dt is not finite");
    if (steps < 0 || steps > NBODY_MAX_STEPS)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "steps = %lld outside [0, %lld]", (long long)steps,
                    (long long)NBODY_MAX_STEPS);
    if (n == 0 || steps == 0) return NBODY_OK;
    if (!pos || !m || !lx || !lv || !lm)
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL pos, m, lx, lv or lm with n = %lld", (long long)n);
    const size_t v3 = 12 * (size_t)n, v1 = 4 * (size_t)n;
    const void *arr[5] = {pos, m, lx, lv, lm};
    const size_t len[5] = {v3 * (size_t)(steps + 1), v1, v3, v3, v1};
    for (int i = 0; i < 5; ++i)
        for (int k = i + 1; k < 5; ++k)
            if (overlaps(arr[i], len[i], arr[k], len[k]))
                return fail(NBODY_ERROR_INVALID_ARGUMENT, "pos, m, lx, lv and lm must not overlap");
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    const int variant = select_variant(NBODY_KIND_BACKWARD, n);
    // VJP results of variants that cannot take the update in their final
    // reduction
    void *aux = nullptr;
    st = workspace_aux(dev, s, 16 * (size_t)n, &aux);
    if (st != NBODY_OK) return st;
    float *gx = static_cast<float *>(aux);
    float *gm = gx + 3 * (size_t)n;
    LfEpi e;
    e.mode = kLfAdjoint;
    e.dt = dt;
    e.lx = lx;
    e.lm = lm;
    e.lv = lv;
    // lx, lm += c VJP(positions)[lv]; then lv += dt lx if `chain`
    auto vjp = [&](const float *xp, float c, bool chain) {
        e.c = c;
        e.chain = chain ? 1 : 0;
        bool fused = false;
        prof_mark(s, -1);
        nbody_status r = backward_run(variant, dev, xp, m, (int)n, eps2, lv, nullptr, gx, gm, s,
                                      &e, &fused);
        if (r == NBODY_OK && !fused) r = lf_epilogue_run(gx, gm, n, e, s);
        if (r == NBODY_OK) prof_mark(s, 2);
        return r;
    };
    const float half = 0.5f * dt;
    const size_t stride = 3 * (size_t)n;
    if (flags & NBODY_LEAPFROG_FINAL)
        st = vjp(pos + stride * (size_t)steps, -half, true);  // end kick of the last step
    else
        st = axpy_run(lv, lx, 3 * n, dt, s);  // drift of the segment's last step
    for (int64_t t = steps; t >= 1 && st == NBODY_OK; --t) {
        // positions before step t of the segment: its start kick, plus the
        // end kick of the step before at the same positions (none at step 0)
        const bool first = (flags & NBODY_LEAPFROG_INITIAL) && t == 1;
        st = vjp(pos + stride * (size_t)(t - 1), first ? -half : -dt, t > 1);
    }
    return st;
}

int64_t nbody_variant_plan(int kind, int index, int64_t n, int num_cu, int blocks_per_cu,
                           int64_t free_bytes, int *timed)
{
    clear_error();
    if (timed) *timed = 0;
    int64_t bytes = -1, max_n = -1;
    if (kind == NBODY_KIND_FORWARD) {
        bytes = forward_plan_bytes(index, n, num_cu, blocks_per_cu);
        max_n = forward_variant_max_n(index);
    } else if (kind == NBODY_KIND_BACKWARD) {
        bytes = backward_plan_bytes(index, n, num_cu, blocks_per_cu);
        max_n = backward_variant_max_n(index);
    }
    if (bytes < 0 || free_bytes < 0) {
        fail(NBODY_ERROR_INVALID_ARGUMENT, "no plan for kind %d variant %d at n = %lld", kind, index,
             (long long)n);
        return -1;
    }
    if (timed) *timed = tune_admissible(n, max_n, bytes, tune_workspace_cap((size_t)free_bytes));
    return bytes;
}

int nbody_variant_count(int kind) { return variant_count(kind); }

const char *nbody_variant_name(int kind, int index) { return variant_name(kind, index); }

nbody_status nbody_set_variant(int kind, int index)
{
    clear_error();
    if (kind < 0 || kind > 2) return fail(NBODY_ERROR_INVALID_ARGUMENT, "unknown kind %d", kind);
    if (index < -1 || index >= variant_count(kind))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "variant %d out of range for kind %d", index, kind);
    std::lock_guard<std::mutex> lock(g_var_mu);
    read_env_locked();
    g_forced[kind] = index;
    return NBODY_OK;
}

int nbody_selected_variant(int kind, int64_t n)
{
    if (kind < 0 || kind > 2 || n < 0) return -1;
    return select_variant(kind, n);
}

nbody_status nbody_release_workspace(void)
{
    clear_error();
    release_batched_plans();
    std::lock_guard<std::mutex> lock(g_ws_mu);
    nbody_status st = NBODY_OK;
    for (auto &kv : g_ws) {
        if (kv.second.ptr) {
            int cur = -1;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(std::get<0>(kv.first));
            hipError_t e = hipFree(kv.second.ptr);
            (void)hipSetDevice(cur);
            if (e != hipSuccess && st == NBODY_OK) st = hip_fail(e, "hipFree(workspace)");
        }
    }
    g_ws.clear();
    std::lock_guard<std::mutex> lock2(g_cnt_mu);
    for (auto &kv : g_cnt) {
        if (kv.second.ptr) {
            int cur = -1;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(kv.first.first);
            hipError_t e = hipFree(kv.second.ptr);
            (void)hipSetDevice(cur);
            if (e != hipSuccess && st == NBODY_OK) st = hip_fail(e, "hipFree(counters)");
        }
    }
    g_cnt.clear();
    return st;
}

nbody_status nbody_profile_enable(int on)
{
    clear_error();
    g_prof_on.store(on != 0);
    t_prof.clear();
    return NBODY_OK;
}

nbody_status nbody_profile_read(double *main_ms, double *total_ms, int *calls, double *launches)
{
    clear_error();
    double sm = 0.0, st = 0.0, nl = 0.0;
    const size_t cnt = t_prof.calls.size();
    for (ProfCall &c : t_prof.calls) {
        nl += (double)(c.pair.size() / 2);
        hipError_t err = hipEventSynchronize(c.end);
        if (err != hipSuccess) return hip_fail(err, "hipEventSynchronize(profile)");
        for (size_t k = 0; k + 1 < c.pair.size(); k += 2) {
            float a = 0.f;
            err = hipEventElapsedTime(&a, c.pair[k], c.pair[k + 1]);
            if (err != hipSuccess) return hip_fail(err, "hipEventElapsedTime(profile)");
            sm += a;
        }
        float b = 0.f;
        err = hipEventElapsedTime(&b, c.pair[0], c.end);
        if (err != hipSuccess) return hip_fail(err, "hipEventElapsedTime(profile)");
        st += b;
    }
    if (main_ms) *main_ms = cnt ? sm / cnt : 0.0;
    if (total_ms) *total_ms = cnt ? st / cnt : 0.0;
    if (calls) *calls = (int)cnt;
    if (launches) *launches = cnt ? nl / cnt : 0.0;
    t_prof.clear();
    return NBODY_OK;
}

nbody_status nbody_autotune(int kind, const int64_t *sizes, int64_t count, void *stream)
{
    clear_error();
    if (kind < 0 || kind > 2) return fail(NBODY_ERROR_INVALID_ARGUMENT, "unknown kind %d", kind);
    if (count < 0 || (count > 0 && !sizes)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "bad size list");
    for (int64_t k = 0; k < count; ++k)
        if (sizes[k] < 2 || sizes[k] > (1 << 22))
            return fail(NBODY_ERROR_INVALID_ARGUMENT, "tuning size %lld outside [2, 2^22]", (long long)sizes[k]);
    if (count == 0) return NBODY_OK;
    Device dev;
    nbody_status st = current_device(&dev);
    if (st != NBODY_OK) return st;
    return autotune_run(kind, dev, sizes, count, (hipStream_t)stream);
}

nbody_status nbody_autotune_batched(const int64_t *offsets, int64_t num_systems, const float *x,
                                    const float *m, float eps2, void *stream)
{
    clear_error();
    nbody_status st = check_offsets(offsets, num_systems);
    if (st != NBODY_OK) return st;
    if (bad_eps2(eps2)) return fail(NBODY_ERROR_INVALID_ARGUMENT, "eps2 = %g is negative or not finite", eps2);
    const int64_t n = offsets[num_systems];
    if (n == 0) return NBODY_OK;
    if (!x || !m) return fail(NBODY_ERROR_INVALID_ARGUMENT, "NULL x or m with %lld particles", (long long)n);
    if (overlaps(x, 12 * (size_t)n, m, 4 * (size_t)n))
        return fail(NBODY_ERROR_INVALID_ARGUMENT, "x and m overlap");
    Device dev;
    st = current_device(&dev);
    if (st != NBODY_OK) return st;
    return autotune_batched_run(dev, offsets, num_systems, x, m, eps2, (hipStream_t)stream);
}

}  // extern "C"
