// Live per-kernel timing with HIP events on the launching stream.
#include "common.h"

namespace gsc {

const char *kernel_name(int id) {
    static const char *names[KP_COUNT] = {"spmm_seed", "spmm_S",  "shift_update", "cg_update",
                                          "cg_dir",    "update_r", "rho_dot",     "p_update",
                                          "ctrl",      "post",     "proj_update", "cheb_step",
                                          "ring_transpose", "lz_hprod", "lz_update", "lz_scale",
                                          "cheb_mx",   "mx_resid"};
    return (id >= 0 && id < KP_COUNT) ? names[id] : "";
}

hipEvent_t Profiler::get_event() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    GSC_HIP(hipEventCreate(&e));
    return e;
}

void Profiler::begin_group(hipStream_t st, int id) {
    open_id_ = id;
    if (!on || (only >= 0 && id != only)) return;
    Pending p{id, get_event(), get_event(), 0.0, 0};
    GSC_HIP(hipEventRecord(p.a, st));
    pending.push_back(p);
    open_ = true;
}

void Profiler::end_group(hipStream_t st, long long launches, double bytes) {
    if (!on) return;
    if (!open_) {
        // kernel not timed: count its launches and bytes only
        if (open_id_ >= 0) {
            acc[open_id_].launches += launches;
            acc[open_id_].bytes += bytes;
        }
        return;
    }
    GSC_HIP(hipEventRecord(pending.back().b, st));
    pending.back().launches = launches;
    pending.back().bytes = bytes;
    open_ = false;
}

void Profiler::resolve() {
    for (auto &p : pending) {
        float ms = 0.f;
        GSC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        acc[p.id].ms += ms;
        acc[p.id].launches += p.launches;
        acc[p.id].bytes += p.bytes;
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}

void Profiler::reset() {
    for (auto &a : acc) a = Acc{};
    for (auto &p : pending) { pool.push_back(p.a); pool.push_back(p.b); }
    pending.clear();
}

Profiler::~Profiler() {
    for (auto &p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace gsc
