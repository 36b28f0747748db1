// Opt-in per-kernel timing: HIP event pairs recorded around the library's
// own kernel launches, on the launch stream.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.h"

namespace genie {
namespace {

struct Pending {
    hipEvent_t start, stop;
    int kind;  // 0 scan, 1 merge, 2 fallback scan
};

std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_free;
std::vector<Pending> g_pending;
genie_kernel_times g_totals{};

hipEvent_t take_event() {
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

}  // namespace

bool timing_enabled() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on;
}

void *timing_begin(hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on)
        return nullptr;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, st) != hipSuccess) {
        g_free.push_back(e);
        return nullptr;
    }
    return e;
}

void timing_end(void *start, hipStream_t st, int kind) {
    if (!start)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e = take_event();
    if (!e || hipEventRecord(e, st) != hipSuccess) {
        g_free.push_back((hipEvent_t)start);
        if (e)
            g_free.push_back(e);
        return;
    }
    g_pending.push_back({(hipEvent_t)start, e, kind});
}

}  // namespace genie

using namespace genie;

extern "C" int genie_kernel_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return GENIE_OK;
}

extern "C" int genie_kernel_timing_read(genie_kernel_times *out, int reset) {
    clear_error();
    if (!out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = GENIE_OK;
    for (const Pending &p : g_pending) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(p.stop);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, p.start, p.stop);
        if (e != hipSuccess && rc == GENIE_OK)
            rc = hip_fail(e, "kernel timing event");
        if (p.kind == 0) {
            g_totals.scan_launches++;
            g_totals.scan_ms += ms;
        } else if (p.kind == 1) {
            g_totals.merge_launches++;
            g_totals.merge_ms += ms;
        } else {
            g_totals.fallback_launches++;
            g_totals.fallback_ms += ms;
        }
        g_free.push_back(p.start);
        g_free.push_back(p.stop);
    }
    g_pending.clear();
    *out = g_totals;
    if (reset)
        g_totals = genie_kernel_times{};
    return rc;
}
