// Autotuner for the fused sweep (sv_tune).
//
// The best tile shape depends on the circuit: more always-resident low bits
// make longer contiguous runs per access but leave fewer free slots, which can
// cost whole extra passes; a larger tile fits more qubits per pass but holds
// fewer workgroups per CU.  The tuner plans the circuit for each candidate
// shape, drops candidates whose pass count is not within one of the best,
// times the rest on the device (same launch path as sv_apply_fused, on the
// caller's scratch state) and remembers the fastest per circuit content.
// sv_apply_fused / sv_simulate called with opts == NULL use the remembered
// shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "qsv_internal.h"

namespace qsv {
namespace {

struct TuneKey {
    int n, lb, le;
    std::string gates;
    bool operator<(const TuneKey &o) const {
        if (n != o.n) return n < o.n;
        if (lb != o.lb) return lb < o.lb;
        if (le != o.le) return le < o.le;
        return gates < o.gates;
    }
};

std::mutex g_tmu;
std::map<TuneKey, qsv_fuse_opts> g_tuned;

TuneKey key_of(const qsv_circuit *c, int lb, int le) {
    TuneKey k;
    k.n = c->n;
    k.lb = lb;
    k.le = le;
    k.gates.assign(reinterpret_cast<const char *>(c->gates.data()), c->gates.size() * sizeof(qsv_gate));
    return k;
}

}  // namespace

bool tuned_opts(const qsv_circuit *c, int lb, int le, qsv_fuse_opts *out) {
    std::lock_guard<std::mutex> g(g_tmu);
    if (g_tuned.empty()) return false;
    auto it = g_tuned.find(key_of(c, lb, le));
    if (it == g_tuned.end()) return false;
    *out = it->second;
    return true;
}

}  // namespace qsv

using namespace qsv;

extern "C" qsv_status sv_tune(void *amps_scratch, const qsv_circuit *c, int layer_begin,
                              int layer_end, qsv_fuse_opts *out, double *best_ms, void *stream) {
    if (!c || !out || !amps_scratch) return fail(QSV_EINVAL, "sv_tune: null argument");
    struct Cand { int R, T, c; };
    static const Cand cands[] = {{5, 8, 4}, {5, 8, 5}, {4, 8, 4}, {4, 8, 5}, {5, 9, 4}, {5, 9, 5},
                                 {6, 8, 4}, {5, 7, 4}, {4, 7, 4}};
    std::vector<std::pair<int, qsv_fuse_opts>> plans;
    int best_passes = 1 << 30;
    for (const Cand &k : cands) {
        if (k.R + k.T > c->n) continue;
        qsv_fuse_opts o{k.R, k.T, k.c, 0, 0};
        int np = 0;
        qsv_status st = sv_plan_info(c, layer_begin, layer_end, &o, &np, nullptr, nullptr, 0,
                                     nullptr, 0);
        if (st != QSV_OK) continue;
        plans.push_back({np, o});
        best_passes = std::min(best_passes, np);
    }
    if (plans.empty()) return fail(QSV_EUNSUPPORTED, "sv_tune: no tile shape fits this circuit");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(QSV_EHIP, "sv_tune: event create");
    double best = 1e30;
    qsv_fuse_opts pick = plans[0].second;
    for (auto &pp : plans) {
        if (pp.first > best_passes + 1) continue;
        qsv_fuse_opts o = pp.second;
        // warm-up (plans and compiles), then the median of three timed runs
        qsv_status st = sv_apply_fused(amps_scratch, c, 0, layer_begin, layer_end, &o, stream);
        if (st != QSV_OK) continue;
        float t[3];
        bool ok = true;
        for (int r = 0; r < 3 && ok; ++r) {
            ok = hipEventRecord(e0, s) == hipSuccess &&
                 sv_apply_fused(amps_scratch, c, 0, layer_begin, layer_end, &o, stream) == QSV_OK &&
                 hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
        }
        if (!ok) continue;
        std::sort(t, t + 3);
        if (t[1] < best) {
            best = t[1];
            pick = o;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best >= 1e30) return fail(QSV_EHIP, "sv_tune: no candidate ran");
    {
        std::lock_guard<std::mutex> g(g_tmu);
        g_tuned[key_of(c, layer_begin, layer_end)] = pick;
    }
    *out = pick;
    if (best_ms) *best_ms = best;
    return QSV_OK;
}
