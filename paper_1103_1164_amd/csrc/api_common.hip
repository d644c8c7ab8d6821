// api_common.hip -- host side of libfspb shared by the entry points: error
// reporting, argument checks of tables and the device checks.
#include "api_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>

namespace fspb {

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace {
// -1: not yet read from the environment
std::atomic<int> g_log_level{-1};

int clamp_level(long v) { return v < 0 ? 0 : v > 3 ? 3 : (int)v; }
}  // namespace

int log_level() {
    int v = g_log_level.load(std::memory_order_relaxed);
    if (v >= 0) return v;
    const char* e = getenv("FSPB_LOG_LEVEL");
    char* end = nullptr;
    const long x = e ? strtol(e, &end, 10) : 0;
    int fresh = (e && end != e && *end == '\0') ? clamp_level(x) : 0;
    int expected = -1;
    // another thread (or fspb_set_log_level) may have set it meanwhile
    if (!g_log_level.compare_exchange_strong(expected, fresh)) fresh = expected;
    return fresh;
}

void log_msg(int level, const char* fmt, ...) {
    if (log_level() < level) return;
    char buf[640];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[fspb] %s\n", buf);
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    log_msg(1, "error %d (%s): %s", code, fspb_error_string(code), buf);
    return code;
}

bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }

int check_table(const fspb_table1d& t, const char* name) {
    if (t.n < 1 || !t.v) return fail(FSPB_E_ARG, "table %s: needs n >= 1 and values", name);
    if (!isfinite(t.start) || (t.n > 1 && !finite_pos(t.step)))
        return fail(FSPB_E_ARG, "table %s: start must be finite and step > 0", name);
    return FSPB_OK;
}

namespace {
// Per device, looked up once (the property query is slow compared with
// creating a plan): whether it is a gfx950 (0 unknown, 1 yes, -1 no) and its
// compute units.
constexpr int kMaxDevices = 64;
std::atomic<int> g_arch_ok[kMaxDevices];
std::atomic<int> g_cu_count[kMaxDevices];
}  // namespace

int check_device(int* dev) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return fail(FSPB_E_UNSUPPORTED, "no HIP device available");
    }
    HIP_TRY(hipGetDevice(dev));
    if (*dev < 0 || *dev >= kMaxDevices)
        return fail(FSPB_E_UNSUPPORTED, "device %d: at most %d devices", *dev, kMaxDevices);
    const int v = g_arch_ok[*dev].load();
    if (v == 1) return FSPB_OK;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, *dev));
    const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    g_cu_count[*dev].store(prop.multiProcessorCount);
    g_arch_ok[*dev].store(ok ? 1 : -1);
    if (!ok)
        return fail(FSPB_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", *dev,
                    prop.gcnArchName);
    return FSPB_OK;
}

int device_cu_count(int dev) {
    return dev >= 0 && dev < kMaxDevices ? g_cu_count[dev].load() : 0;
}

int check_same_device(int dev, const char* what) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) return fail(FSPB_E_STATE, "%s: handle lives on device %d, current is %d", what, dev, cur);
    return FSPB_OK;
}

const char* last_error_text() { return g_last_error.c_str(); }
void clear_last_error() { g_last_error.clear(); }

}  // namespace fspb

extern "C" {

const char* fspb_error_string(int code) {
    switch (code) {
        case FSPB_OK: return "success";
        case FSPB_E_ARG: return "invalid argument";
        case FSPB_E_HIP: return "HIP runtime error";
        case FSPB_E_NOMEM: return "out of memory";
        case FSPB_E_STATE: return "invalid state for this handle";
        case FSPB_E_UNSUPPORTED: return "unsupported device";
        default: return "unknown error";
    }
}

const char* fspb_last_error(void) { return fspb::last_error_text(); }

int fspb_set_log_level(int level) {
    const int prev = fspb::log_level();
    fspb::g_log_level.store(level < 0 ? 0 : level > 3 ? 3 : level);
    return prev;
}

}  // extern "C"
