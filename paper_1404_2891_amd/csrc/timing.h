// Optional per-phase device timing with HIP events recorded on the launching stream.
#pragma once

#include <vector>

#include "common.h"
#include "record.h"

namespace fm {

enum Phase {
    PH_LU_UPDATE = 0, PH_LU_PANEL = 1, PH_LU_OTHER = 2, PH_SOLVE = 3, PH_REFINE = 4, PH_RR = 5,
    PH_HOST_REDUCED = 6,   // host wall time: reduced eigenproblems
    PH_HOST_ORTHO = 7,     // host wall time: Cholesky factorisations of the orthonormalisation
    PH_HOST_DRIVER = 8,    // host wall time: enqueueing the device phases, convergence bookkeeping
    PH_HOST_WAIT = 9,      // host wall time: waiting at the iteration's synchronisation points
    PH_COUNT = 10
};
inline bool is_host_phase(int p) { return p >= PH_HOST_REDUCED; }

struct Timer {
    bool on = false;
    struct Span { hipEvent_t a, b; };
    std::vector<Span> open[PH_COUNT];
    std::vector<hipEvent_t> pool;
    double flops[PH_COUNT] = {0};
    long launches[PH_COUNT] = {0};
    hipEvent_t cur_a[PH_COUNT] = {nullptr};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // while device work is recorded (record.h) the marks are recorded with it
    void mark(Phase p, bool is_start, double fl) {
        RecOp r;
        r.kind = REC_MARK;
        r.phase = p;
        r.start = is_start;
        r.flops = fl;
        op_log()->ops.push_back(std::move(r));
    }
    void start(Phase p, hipStream_t st) {
        if (!on) return;
        if (op_log()) return mark(p, true, 0.0);
        cur_a[p] = get();
        if (cur_a[p]) (void)hipEventRecord(cur_a[p], st);
    }
    void stop(Phase p, hipStream_t st, double fl) {
        if (!on) return;
        if (op_log()) return mark(p, false, fl);
        if (!cur_a[p]) return;
        hipEvent_t b = get();
        if (!b) return;
        (void)hipEventRecord(b, st);
        open[p].push_back({cur_a[p], b});
        cur_a[p] = nullptr;
        flops[p] += fl;
        launches[p] += 1;
    }
    // Total milliseconds of phase p (synchronises on its last event).
    double host_ms[PH_COUNT] = {0};
    void add_host(Phase p, double ms_) {
        if (!on) return;
        host_ms[p] += ms_;
        launches[p] += 1;
    }
    double ms(Phase p) {
        if (is_host_phase(p)) return host_ms[p];
        double tot = 0.0;
        if (open[p].empty()) return 0.0;
        (void)hipEventSynchronize(open[p].back().b);
        for (auto& s : open[p]) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, s.a, s.b) == hipSuccess) tot += t;
        }
        return tot;
    }
    void reset() {
        for (int p = 0; p < PH_COUNT; ++p) {
            for (auto& s : open[p]) {
                pool.push_back(s.a);
                pool.push_back(s.b);
            }
            open[p].clear();
            flops[p] = 0;
            launches[p] = 0;
            host_ms[p] = 0;
        }
    }
    ~Timer() {
        reset();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace fm
