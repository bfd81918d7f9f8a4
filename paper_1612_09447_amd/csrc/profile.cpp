// Per-kernel-class timing with HIP events. Classes of one kernel take the
// start/stop events of the launch itself (hipExtLaunchKernelGGL: the
// kernel's own execution, as a kernel trace reports it); the V-cycle class
// brackets its launches with events recorded on the stream.
#include "eqs_internal.h"

namespace eqs {

void prof_begin(eqs_ctx* c, int cls, hipStream_t s) {
    if (!(c->prof_mask & (1u << cls))) return;
    std::vector<hipEvent_t>& ev = c->prof_ev[cls];
    const size_t need = 2 * (size_t)(c->prof_used[cls] + 1);
    while (ev.size() < need) {
        hipEvent_t e;
        EQS_HIP(hipEventCreate(&e));
        ev.push_back(e);
    }
    EQS_HIP(hipEventRecord(ev[2 * c->prof_used[cls]], s));
}

bool prof_pair(eqs_ctx* c, int cls, hipEvent_t* e0, hipEvent_t* e1) {
    if (cls < 0 || !(c->prof_mask & (1u << cls))) return false;  // cls < 0: a launch that is never timed
    std::vector<hipEvent_t>& ev = c->prof_ev[cls];
    const size_t need = 2 * (size_t)(c->prof_used[cls] + 1);
    while (ev.size() < need) {
        hipEvent_t e;
        EQS_HIP(hipEventCreate(&e));
        ev.push_back(e);
    }
    *e0 = ev[2 * c->prof_used[cls]];
    *e1 = ev[2 * c->prof_used[cls] + 1];
    c->prof_used[cls]++;
    return true;
}

void prof_end(eqs_ctx* c, int cls, hipStream_t s) {
    if (!(c->prof_mask & (1u << cls))) return;
    EQS_HIP(hipEventRecord(c->prof_ev[cls][2 * c->prof_used[cls] + 1], s));
    c->prof_used[cls]++;
}

void prof_release(eqs_ctx* c) {
    for (auto& v : c->prof_ev) {
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
        v.clear();
    }
    for (auto& u : c->prof_used) u = 0;
    c->prof_mask = 0;
}

}  // namespace eqs

extern "C" int eqs_profile_enable_impl(eqs_ctx* c, uint32_t mask) {
    for (auto& u : c->prof_used) u = 0;
    c->prof_mask = mask & ((1u << EQS_KCLASS_COUNT) - 1);
    return EQS_OK;
}

extern "C" int eqs_profile_read_impl(eqs_ctx* c, int32_t cls, int64_t* launches, double* total_ms) {
    EQS_HIP(hipStreamSynchronize(c->stream));
    double ms = 0.0;
    for (int64_t i = 0; i < c->prof_used[cls]; ++i) {
        float t = 0.0f;
        EQS_HIP(hipEventElapsedTime(&t, c->prof_ev[cls][2 * i], c->prof_ev[cls][2 * i + 1]));
        ms += t;
    }
    *launches = c->prof_used[cls];
    *total_ms = ms;
    return EQS_OK;
}
