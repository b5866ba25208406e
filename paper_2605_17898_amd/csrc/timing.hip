// Optional per-launch timing of the entry sweeps (thread-local; see
// mfgp_timing_enable in include/mfgp.h).
#include <vector>

#include "internal.hpp"

namespace mfgp {

namespace {
struct Rec {
    hipEvent_t a, b;
    int kind;
    double entries, flops;
};
struct TimingState {
    bool on = false;
    bool suspended = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double phase[3] = {0.0, 0.0, 0.0};
};
thread_local TimingState g_timing;

hipEvent_t take_event() {
    if (!g_timing.pool.empty()) {
        hipEvent_t e = g_timing.pool.back();
        g_timing.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

double sweep_flops_per_entry(int family, int d, int t, bool adjoint) {
    if (adjoint) return 5.0 * d + 4.0 + 2.0 * t;
    switch (family) {
        case MFGP_RBF: return 3.0 * d + 1.0 + 2.0 * t;
        case MFGP_MATERN12: return 3.0 * d + 2.0 + 2.0 * t;
        case MFGP_MATERN32: return 3.0 * d + 5.0 + 2.0 * t;
        default: return 3.0 * d + 7.0 + 2.0 * t;
    }
}

void timing_suspend(bool on) { g_timing.suspended = on; }

void* timing_begin(hipStream_t s) {
    if (!g_timing.on || g_timing.suspended) return nullptr;
    hipEvent_t a = take_event();
    if (!a) return nullptr;
    (void)hipEventRecord(a, s);
    return reinterpret_cast<void*>(a);
}

void timing_end(void* tok, hipStream_t s, int kind, double entries, double flops) {
    if (!tok) return;
    hipEvent_t b = take_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    g_timing.recs.push_back(Rec{reinterpret_cast<hipEvent_t>(tok), b, kind, entries, flops});
}

bool timing_on() { return g_timing.on && !g_timing.suspended; }

void timing_phase(int which, double ms) {
    if (g_timing.on && which >= 0 && which < 3) g_timing.phase[which] += ms;
}

static void release_all() {
    for (auto& r : g_timing.recs) {
        g_timing.pool.push_back(r.a);
        g_timing.pool.push_back(r.b);
    }
    g_timing.recs.clear();
    for (double& p : g_timing.phase) p = 0.0;
}

}  // namespace mfgp

using namespace mfgp;

extern "C" int mfgp_timing_enable(int32_t on) {
    release_all();
    if (!on) {
        for (hipEvent_t e : g_timing.pool) (void)hipEventDestroy(e);
        g_timing.pool.clear();
    }
    g_timing.on = on != 0;
    return MFGP_OK;
}

extern "C" int mfgp_timing_phases(double* cg_ms, double* slq_ms, double* adjoint_ms) {
    if (cg_ms) *cg_ms = g_timing.phase[0];
    if (slq_ms) *slq_ms = g_timing.phase[1];
    if (adjoint_ms) *adjoint_ms = g_timing.phase[2];
    return MFGP_OK;
}

extern "C" int mfgp_timing_read(int32_t kind, double* sweep_ms, int64_t* launches, double* entries,
                                double* flops) {
    double ms = 0.0, en = 0.0, fl = 0.0;
    int64_t cnt = 0;
    for (auto& r : g_timing.recs) {
        if (kind >= 0 && r.kind != kind) continue;
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) {
            set_last_hip_error(e);
            return MFGP_ERR_HIP;
        }
        float x = 0.0f;
        e = hipEventElapsedTime(&x, r.a, r.b);
        if (e != hipSuccess) {
            set_last_hip_error(e);
            return MFGP_ERR_HIP;
        }
        ms += x;
        cnt += 1;
        en += r.entries;
        fl += r.flops;
    }
    if (sweep_ms) *sweep_ms = ms;
    if (launches) *launches = cnt;
    if (entries) *entries = en;
    if (flops) *flops = fl;
    return MFGP_OK;
}
