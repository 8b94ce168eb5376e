// Opt-in launch timing: when enabled, hot launches are bracketed by a pair
// of HIP events on their own stream; vmps_trace_collect() waits for the
// events and returns the summed time and launch count per kernel kind.
// Off by default; costs nothing when off.
#include <mutex>
#include <vector>

#include "vmps_internal.hpp"

namespace vmps {

namespace {
struct Rec {
    int kind;
    hipEvent_t a, b;
};
struct TraceState {
    std::mutex mu;
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
TraceState& state()
{
    static TraceState s;
    return s;
}
}  // namespace

bool trace_suspend()
{
    TraceState& S = state();
    std::lock_guard<std::mutex> g(S.mu);
    const bool was = S.on;
    S.on = false;
    return was;
}

void trace_resume(bool was_on)
{
    TraceState& S = state();
    std::lock_guard<std::mutex> g(S.mu);
    S.on = was_on;
}

TraceScope::TraceScope(int kind, hipStream_t s) : kind_(kind), stream_(s), a_(nullptr)
{
    TraceState& st = state();
    std::lock_guard<std::mutex> g(st.mu);
    if (!st.on) return;
    a_ = st.get();
    if (a_) hipEventRecord((hipEvent_t)a_, s);
}

TraceScope::~TraceScope()
{
    if (!a_) return;
    TraceState& st = state();
    std::lock_guard<std::mutex> g(st.mu);
    hipEvent_t b = st.get();
    if (!b) return;
    hipEventRecord(b, stream_);
    st.recs.push_back(Rec{kind_, (hipEvent_t)a_, b});
}

}  // namespace vmps

extern "C" {

vmps_status vmps_trace_enable(int on)
{
    vmps::TraceState& st = vmps::state();
    std::lock_guard<std::mutex> g(st.mu);
    st.on = on != 0;
    return VMPS_OK;
}

vmps_status vmps_trace_collect(double* ms, int64_t* launches, int32_t nkinds)
{
    if (!ms || !launches || nkinds < 0) return VMPS_ERR_INVALID_ARG;
    vmps::TraceState& st = vmps::state();
    std::lock_guard<std::mutex> g(st.mu);
    for (int i = 0; i < nkinds; ++i) { ms[i] = 0.0; launches[i] = 0; }
    vmps_status rc = VMPS_OK;
    for (auto& r : st.recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            rc = VMPS_ERR_DEVICE;
        if (r.kind >= 0 && r.kind < nkinds) {
            ms[r.kind] += t;
            launches[r.kind] += 1;
        }
        st.pool.push_back(r.a);
        st.pool.push_back(r.b);
    }
    st.recs.clear();
    return rc;
}

}  // extern "C"
