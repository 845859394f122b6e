// Kernel timing: HIP events around CPI step-kernel launches, grouped by
// kernel variant (see tpa_profile_enable in tpa.h).

#include <mutex>
#include <vector>

#include "profile.h"

namespace tpa {
namespace {

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> begin, end;   // event pool (pairs)
    std::vector<int> code;                // variant of each recorded pair
    size_t used = 0;
    int period = 1;
    int64_t seen[128] = {};               // launches seen per code (for sampling)
    int64_t launches[128] = {};
    double ms[128] = {};
};

Profiler &prof() {
    static Profiler p;
    return p;
}

tpa_status drain(Profiler &p) {
    for (size_t i = 0; i < p.used; ++i) {
        TPA_TRY_HIP(hipEventSynchronize(p.end[i]));
        float t = 0.f;
        TPA_TRY_HIP(hipEventElapsedTime(&t, p.begin[i], p.end[i]));
        p.launches[p.code[i]] += 1;
        p.ms[p.code[i]] += t;
    }
    p.used = 0;
    return TPA_OK;
}

}  // namespace

int profile_begin(int code, hipStream_t st) {
    Profiler &p = prof();
    if (!p.on) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return -1;
    std::lock_guard<std::mutex> lk(p.mu);
    if (p.seen[code]++ % p.period != 0) return -1;
    if (p.used == p.begin.size() && drain(p) != TPA_OK) return -1;
    const int slot = (int)p.used++;
    p.code[slot] = code;
    if (hipEventRecord(p.begin[slot], st) != hipSuccess) return -1;
    return slot;
}

void profile_end(int slot, hipStream_t st) {
    if (slot < 0) return;
    (void)hipEventRecord(prof().end[slot], st);
}

}  // namespace tpa

using namespace tpa;

extern "C" tpa_status tpa_profile_enable(int enable, int capacity, int sample_period) {
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (!enable) {
        TPA_TRY(drain(p));
        p.on = false;
        return TPA_OK;
    }
    if (capacity < 1 || capacity > (1 << 20)) return fail(TPA_ERR_INVALID_ARG, "capacity must be in 1..2^20");
    if (sample_period < 1) return fail(TPA_ERR_INVALID_ARG, "sample_period must be >= 1");
    p.period = sample_period;
    while ((int)p.begin.size() < capacity) {
        hipEvent_t a, b;
        TPA_TRY_HIP(hipEventCreate(&a));
        TPA_TRY_HIP(hipEventCreate(&b));
        p.begin.push_back(a);
        p.end.push_back(b);
        p.code.push_back(0);
    }
    p.on = true;
    return TPA_OK;
}

extern "C" tpa_status tpa_profile_read(int code, int64_t *launches, double *total_ms) {
    if (code < 0 || code > 127) return fail(TPA_ERR_INVALID_ARG, "code must be in 0..127");
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    TPA_TRY(drain(p));
    if (launches) *launches = p.launches[code];
    if (total_ms) *total_ms = p.ms[code];
    return TPA_OK;
}

extern "C" tpa_status tpa_profile_reset(void) {
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    TPA_TRY(drain(p));
    for (int i = 0; i < 128; ++i) {
        p.seen[i] = 0;
        p.launches[i] = 0;
        p.ms[i] = 0.0;
    }
    return TPA_OK;
}
