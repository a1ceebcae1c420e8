// Per-kernel timing: while enabled, each launch made by the library is
// bracketed by two hipEvents recorded on the launch stream.  Events come from
// a pool that is created on first use and reused afterwards.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace nsm {
namespace {

struct Record {
    char name[64];
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Record> g_open;        // recorded, not yet read
std::vector<hipEvent_t> g_pool;
Record g_cur;
bool g_cur_valid = false;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

bool trace_on() { return g_on; }

namespace {
thread_local bool t_debug = false;
thread_local hipError_t t_debug_err = hipSuccess;
}  // namespace

bool debug_sync_begin() {
    const char* e = std::getenv("NSM_DEBUG_SYNC");
    t_debug = e && e[0] == '1' && e[1] == '\0';
    t_debug_err = hipSuccess;
    return t_debug;
}

void debug_check(hipStream_t s) {
    if (!t_debug) return;
    const hipError_t e = hipStreamSynchronize(s);
    const hipError_t l = hipGetLastError();
    if (t_debug_err == hipSuccess) t_debug_err = e != hipSuccess ? e : l;
}

hipError_t debug_sync_end(hipStream_t s) {
    if (!t_debug) return hipSuccess;
    debug_check(s);
    t_debug = false;
    return t_debug_err;
}

void trace_begin(const char* name, const char* suffix, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    g_cur.start = take_event();
    g_cur.stop = take_event();
    if (!g_cur.start || !g_cur.stop) { g_cur_valid = false; return; }
    std::snprintf(g_cur.name, sizeof(g_cur.name), "%s%s", name, suffix ? suffix : "");
    g_cur_valid = hipEventRecord(g_cur.start, s) == hipSuccess;
}

void trace_end(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || !g_cur_valid) return;
    if (hipEventRecord(g_cur.stop, s) == hipSuccess) g_open.push_back(g_cur);
    g_cur_valid = false;
}

}  // namespace nsm

extern "C" {

nsm_status nsm_trace_enable(int on) {
    std::lock_guard<std::mutex> lk(nsm::g_mu);
    nsm::g_on = on != 0;
    return NSM_OK;
}

nsm_status nsm_trace_read(int max_records, char* names, float* ms, int* n_out) {
    if (!n_out || max_records < 0 || (max_records > 0 && (!names || !ms))) return NSM_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(nsm::g_mu);
    int n = 0;
    nsm_status st = NSM_OK;
    for (auto& r : nsm::g_open) {
        if (n < max_records) {
            float t = 0.0f;
            if (hipEventSynchronize(r.stop) != hipSuccess ||
                hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess)
                st = NSM_E_DEVICE;
            std::memcpy(names + 64 * n, r.name, 64);
            ms[n] = t;
        }
        ++n;
        nsm::g_pool.push_back(r.start);
        nsm::g_pool.push_back(r.stop);
    }
    nsm::g_open.clear();
    *n_out = n;
    return st;
}

}  // extern "C"
