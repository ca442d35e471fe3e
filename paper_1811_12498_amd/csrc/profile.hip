// Phase timing: while enabled, the library records a HIP event on a stream at the start
// of each entry point (or of work it moves to another stream) and after each phase; a
// phase's time is measured from the previous mark on the same stream.
#include <mutex>

#include "stk_internal.hpp"

namespace stk {
namespace {

struct Mark {
    int phase;  // -1 = start of an entry point
    hipEvent_t ev;
    hipStream_t s;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Mark> g_marks;

}  // namespace

void prof_mark(int phase, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipEvent_t e;
    STK_HIP(hipEventCreate(&e));
    STK_HIP(hipEventRecord(e, s));
    g_marks.push_back({phase, e, s});
}

void prof_enable(bool on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on;
}

void prof_read(double *ms, int64_t *count) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (int i = 0; i < STK_NPHASES; ++i) {
        if (ms) ms[i] = 0.0;
        if (count) count[i] = 0;
    }
    for (size_t i = 0; i < g_marks.size(); ++i) {
        STK_HIP(hipEventSynchronize(g_marks[i].ev));
        if (g_marks[i].phase < 0) continue;
        size_t j = i;  // the previous mark on the same stream
        while (j > 0 && g_marks[j - 1].s != g_marks[i].s) --j;
        if (j == 0) continue;
        float t = 0.f;
        STK_HIP(hipEventElapsedTime(&t, g_marks[j - 1].ev, g_marks[i].ev));
        const int p = g_marks[i].phase;
        if (p < STK_NPHASES) {
            if (ms) ms[p] += t;
            if (count) count[p] += 1;
        }
    }
    for (auto &m : g_marks) (void)hipEventDestroy(m.ev);
    g_marks.clear();
}

}  // namespace stk
