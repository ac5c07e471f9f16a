// Event-based timing of the per-voxel kernels (ecc_profile_* in ecc.h).
#include <mutex>
#include <vector>

#include "ecc_internal.h"

namespace ecc {

namespace {
struct Pair {
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pair> g_pending;  // recorded, not yet read
std::vector<Pair> g_free;
double g_ms = 0.0;
int64_t g_n = 0;
}  // namespace

bool profile_on() { return g_on; }

int profile_begin(hipStream_t s, void **token) {
    *token = nullptr;
    if (!g_on) return ECC_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    Pair p;
    if (!g_free.empty()) {
        p = g_free.back();
        g_free.pop_back();
    } else {
        ECC_HIP(hipEventCreate(&p.a));
        ECC_HIP(hipEventCreate(&p.b));
    }
    ECC_HIP(hipEventRecord(p.a, s));
    g_pending.push_back(p);
    *token = (void *)(intptr_t)(g_pending.size());
    return ECC_OK;
}

int profile_end(hipStream_t s, void *token) {
    if (!token) return ECC_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    const size_t i = (size_t)(intptr_t)token - 1;
    if (i >= g_pending.size()) return ECC_OK;
    ECC_HIP(hipEventRecord(g_pending[i].b, s));
    return ECC_OK;
}

static int drain() {
    for (Pair &p : g_pending) {
        ECC_HIP(hipEventSynchronize(p.b));
        float ms = 0.f;
        ECC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        g_ms += ms;
        g_n += 1;
        g_free.push_back(p);
    }
    g_pending.clear();
    return ECC_OK;
}

}  // namespace ecc

using namespace ecc;

extern "C" {

int ecc_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return ECC_OK;
}

int ecc_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = drain();
    g_ms = 0.0;
    g_n = 0;
    return rc;
}

int ecc_profile_read(double *kernel_ms, int64_t *launches) {
    if (!kernel_ms || !launches) {
        set_error("ecc_profile_read: NULL output");
        return ECC_E_ARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = drain();
    *kernel_ms = g_ms;
    *launches = g_n;
    return rc;
}

}
