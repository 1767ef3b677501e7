// Optional HIP-event timing of the library's kernels (rose_profile_*).
#include <mutex>
#include <vector>

#include "common.h"

namespace rose {

namespace {
struct Pending {
    hipEvent_t a, b;
    int kind;
    double evals;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
rose_profile g_tot = {};
std::vector<float> g_fit_ms;  // duration of every resolved fitness launch, in launch order

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

bool prof_on() {
    std::lock_guard<std::mutex> l(g_mu);
    return g_on;
}

int prof_begin(int kind, hipStream_t s) {
    std::lock_guard<std::mutex> l(g_mu);
    if (!g_on) return -1;
    Pending p{take_event(), take_event(), kind, 0.0};
    if (!p.a || !p.b) return -1;
    (void)hipEventRecord(p.a, s);
    g_pending.push_back(p);
    return (int)g_pending.size() - 1;
}

void prof_end(int tok, hipStream_t s, double evals) {
    std::lock_guard<std::mutex> l(g_mu);
    if (tok < 0 || tok >= (int)g_pending.size()) return;
    g_pending[tok].evals = evals;
    (void)hipEventRecord(g_pending[tok].b, s);
}

void prof_set_evals(int tok, double evals) {
    std::lock_guard<std::mutex> l(g_mu);
    if (tok < 0 || tok >= (int)g_pending.size()) return;
    g_pending[tok].evals = evals;
}

static void resolve_locked() {
    for (Pending& p : g_pending) {
        float ms = 0.0f;
        (void)hipEventSynchronize(p.b);
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            if (p.kind == PROF_FITNESS) {
                g_fit_ms.push_back(ms);
                g_tot.fitness_ms += ms;
                g_tot.fitness_launches += 1;
                g_tot.fitness_evals += p.evals;
            } else if (p.kind == PROF_UPDATE) {
                g_tot.update_ms += ms;
                g_tot.update_launches += 1;
            } else {
                g_tot.integrate_ms += ms;
                g_tot.integrate_launches += 1;
            }
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}

}  // namespace rose

using namespace rose;

extern "C" {

rose_status rose_profile_enable(int32_t on) {
    clear_error();
    std::lock_guard<std::mutex> l(g_mu);
    g_on = on != 0;
    return ROSE_OK;
}

rose_status rose_profile_reset(void) {
    clear_error();
    std::lock_guard<std::mutex> l(g_mu);
    resolve_locked();
    g_tot = rose_profile{};
    g_fit_ms.clear();
    return ROSE_OK;
}

rose_status rose_profile_fitness_launches(float* ms_out, int64_t cap, int64_t* count_out) {
    clear_error();
    ROSE_REQUIRE(count_out != nullptr && (ms_out != nullptr || cap == 0) && cap >= 0, ROSE_E_ARG,
                 "rose_profile_fitness_launches: bad arguments");
    std::lock_guard<std::mutex> l(g_mu);
    resolve_locked();
    const int64_t n = (int64_t)g_fit_ms.size();
    for (int64_t i = 0; i < n && i < cap; ++i) ms_out[i] = g_fit_ms[(size_t)i];
    *count_out = n;
    return ROSE_OK;
}

rose_status rose_profile_read(rose_profile* out) {
    clear_error();
    ROSE_REQUIRE(out != nullptr, ROSE_E_ARG, "rose_profile_read: NULL output");
    std::lock_guard<std::mutex> l(g_mu);
    resolve_locked();
    *out = g_tot;
    return ROSE_OK;
}

}  // extern "C"
