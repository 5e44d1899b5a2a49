// Kernel-class event timers: a pool of HIP events and one record per launch.
#include <vector>

#include "prof.hpp"

namespace harp {
namespace prof {
namespace {

struct Rec {
    int cls;
    hipEvent_t start, stop;
    double flops, bytes;
};

// Heap objects that are never destroyed: the library has no static object
// whose destructor runs at process exit (the HIP runtime may already be
// finalised by then); pooled events are destroyed by harp_prof_release.
bool g_on = false;
std::vector<Rec>& g_recs = *new std::vector<Rec>();
std::vector<hipEvent_t>& g_pool = *new std::vector<hipEvent_t>();
size_t g_used = 0;

hipEvent_t next_event() {
    if (g_used == g_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_pool.push_back(e);
    }
    return g_pool[g_used++];
}

}  // namespace

bool enabled() { return g_on; }

int begin(int cls, hipStream_t stream) {
    if (!g_on) return -1;
    Rec r{cls, next_event(), next_event(), 0.0, 0.0};
    if (!r.start || !r.stop) return -1;
    if (hipEventRecord(r.start, stream) != hipSuccess) return -1;
    g_recs.push_back(r);
    return int(g_recs.size()) - 1;
}

void end(int token, hipStream_t stream, double flops, double bytes) {
    if (token < 0 || size_t(token) >= g_recs.size()) return;
    Rec& r = g_recs[size_t(token)];
    hipEventRecord(r.stop, stream);
    r.flops = flops;
    r.bytes = bytes;
}

int begin_ext(int cls, hipEvent_t* start, hipEvent_t* stop) {
    *start = *stop = nullptr;
    if (!g_on) return -1;
    Rec r{cls, next_event(), next_event(), 0.0, 0.0};
    if (!r.start || !r.stop) return -1;
    *start = r.start;
    *stop = r.stop;
    g_recs.push_back(r);
    return int(g_recs.size()) - 1;
}

void end_ext(int token, double flops, double bytes) {
    if (token < 0 || size_t(token) >= g_recs.size()) return;
    g_recs[size_t(token)].flops = flops;
    g_recs[size_t(token)].bytes = bytes;
}

}  // namespace prof
}  // namespace harp

using namespace harp;

extern "C" harp_status harp_prof_enable(int32_t on) {
    prof::g_on = on != 0;
    if (on) {
        prof::g_recs.clear();
        prof::g_used = 0;
    }
    return HARP_OK;
}

extern "C" harp_status harp_prof_release(void) {
    prof::g_on = false;
    prof::g_recs.clear();
    harp_status st = HARP_OK;
    for (hipEvent_t e : prof::g_pool)
        if (hipEventDestroy(e) != hipSuccess) st = HARP_E_HIP;
    prof::g_pool.clear();
    prof::g_used = 0;
    return st;
}

namespace {
harp_status prof_sum(int32_t cls, int32_t site, int64_t* launches, double* ms, double* flops, double* bytes) {
    if (cls < 0 || cls >= HARP_K_COUNT || !launches || !ms || !flops || !bytes) return HARP_E_ARG;
    int64_t n = 0;
    double t = 0.0, f = 0.0, b = 0.0;
    for (const auto& r : prof::g_recs) {
        if ((r.cls & 0xff) != cls) continue;
        if (site >= 0 && (r.cls >> 8) != site) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return HARP_E_HIP;
        float e = 0.0f;
        if (hipEventElapsedTime(&e, r.start, r.stop) != hipSuccess) return HARP_E_HIP;
        ++n;
        t += e;
        f += r.flops;
        b += r.bytes;
    }
    *launches = n;
    *ms = t;
    *flops = f;
    *bytes = b;
    return HARP_OK;
}
}  // namespace

extern "C" harp_status harp_prof_read(int32_t cls, int64_t* launches, double* ms, double* flops, double* bytes) {
    return prof_sum(cls, -1, launches, ms, flops, bytes);
}

extern "C" harp_status harp_prof_read_site(int32_t cls, int32_t site, int64_t* launches, double* ms, double* flops,
                                           double* bytes) {
    if (site < 0 || site >= HARP_SITE_COUNT) return HARP_E_ARG;
    return prof_sum(cls, site, launches, ms, flops, bytes);
}
