// Autotuner for the fused sweep (sv_tune).
//
// The best tile shape depends on the circuit: more always-resident low bits
// make longer contiguous runs per access but leave fewer free slots, which can
// cost whole extra passes; a larger tile fits more qubits per pass but holds
// fewer workgroups per CU.  The tuner plans the circuit for each candidate
// shape, drops candidates whose pass count is not within one of the best,
// times the rest on the device (the sweep as sv_simulate runs it, on the
// caller's scratch state and workspace; above 2^30 amplitudes on a sample of
// the tiles), then the persistent kernel form of the fastest three, and
// remembers the fastest options per circuit content.  Calls with opts == NULL
// use them.  With QSV_TUNE_CACHE=<file> the choices are also kept on disk and
// a later process takes them from there instead of timing again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "jit.h"
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

// Persistent tuning results (QSV_TUNE_CACHE=<file>): one line per tuned
// circuit and layer range, "<key> R T c jit out_of_place pass_forms ms",
// the key a 64-bit FNV-1a hash (Fowler, Noll, Vo) of the qubit count, the
// layer range, the gate list and the device (architecture, compute units).
uint64_t fnv1a(const void *p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

uint64_t disk_key(const qsv_circuit *c, int lb, int le) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof(prop));
    if (hipGetDevice(&dev) == hipSuccess) (void)hipGetDeviceProperties(&prop, dev);
    const int head[4] = {c->n, lb, le, prop.multiProcessorCount};
    uint64_t h = fnv1a(head, sizeof(head));
    h = fnv1a(prop.gcnArchName, std::strlen(prop.gcnArchName), h);
    return fnv1a(c->gates.data(), c->gates.size() * sizeof(qsv_gate), h);
}

bool disk_lookup(uint64_t key, qsv_fuse_opts *out, double *ms) {
    const char *path = std::getenv("QSV_TUNE_CACHE");
    if (!path || !path[0]) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    unsigned long long k;
    int R, T, cl, jit, oop;
    unsigned forms;
    double t;
    while (std::fscanf(f, "%llx %d %d %d %d %d %u %lf", &k, &R, &T, &cl, &jit, &oop, &forms, &t) == 8) {
        if (k != key) continue;
        *out = qsv_fuse_opts{R, T, cl, 0, jit, oop, forms};
        *ms = t;
        found = true;  // the last line for a key wins
    }
    std::fclose(f);
    return found;
}

void disk_store(uint64_t key, const qsv_fuse_opts &o, double ms) {
    const char *path = std::getenv("QSV_TUNE_CACHE");
    if (!path || !path[0]) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    if (FILE *f = std::fopen(path, "a")) {
        std::fprintf(f, "%016llx %d %d %d %d %d %u %.6f\n", (unsigned long long)key, o.reg_qubits, o.thread_qubits,
                     o.low_qubits, o.jit, o.out_of_place, o.pass_forms, ms);
        std::fclose(f);
    }
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

extern "C" qsv_status sv_tune(void *amps_scratch, const qsv_circuit *c, int layer_begin, int layer_end,
                              void *workspace, size_t ws_bytes, qsv_fuse_opts *out, double *best_ms,
                              void *stream) {
    if (!c || !out || !amps_scratch) return fail(QSV_EINVAL, "sv_tune: null argument");
    // a result tuned in an earlier process (QSV_TUNE_CACHE)
    const uint64_t dkey = disk_key(c, layer_begin, layer_end);
    {
        qsv_fuse_opts o;
        double ms = 0;
        if (disk_lookup(dkey, &o, &ms)) {
            std::lock_guard<std::mutex> g(g_tmu);
            g_tuned[key_of(c, layer_begin, layer_end)] = o;
            *out = o;
            if (best_ms) *best_ms = ms;
            return QSV_OK;
        }
    }
    struct Cand { int R, T, c; };
    // (tiles of 2^15 amplitudes, R = 6, T = 9, are not candidates: at 34
    // qubits they save a pass but each pass runs 30 % longer)
    static const Cand cands[] = {{5, 8, 4}, {5, 8, 5}, {4, 8, 4}, {4, 8, 5}, {5, 9, 4}, {5, 9, 5},
                                 {6, 8, 4}, {5, 7, 4}, {4, 7, 4}};
    std::vector<std::pair<int, qsv_fuse_opts>> plans;
    int best_passes = 1 << 30;
    for (const Cand &k : cands) {
        if (k.R + k.T > c->n) continue;
        qsv_fuse_opts o{k.R, k.T, k.c, 0, 0, 0, 0u};
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
    // States above 2^31 amplitudes are timed on a sample: every pass runs
    // its first 2^(31 - R - T) tiles only (tens of thousands of workgroups,
    // still many per CU), which ranks the candidates as the full sweep does
    // at an eighth of the cost at 34 qubits.
    constexpr int kSampleQubits = 31;
    constexpr int kReps = 5;  // timings per candidate (median): forms differ by a few percent
    auto sample_tiles = [&](const qsv_fuse_opts &o) -> uint64_t {
        const int L = o.reg_qubits + o.thread_qubits;
        return (c->n > kSampleQubits && L > 0) ? (1ull << (kSampleQubits - L)) : 0;
    };
    // warm-up (plans and compiles), then the median of kReps timed runs of
    // the whole sweep as sv_simulate runs it (state generated by the first
    // pass); compiled sweeps are timed pass by pass (summed)
    auto time_one = [&](const qsv_fuse_opts &o, float *ms) {
        std::vector<float> pm;
        if (time_sweep_passes(c, layer_begin, layer_end, &o, amps_scratch, workspace, ws_bytes, s,
                              sample_tiles(o), pm) == QSV_OK) {
            float t[kReps];
            for (int r = 0; r < kReps; ++r) {
                if (time_sweep_passes(c, layer_begin, layer_end, &o, amps_scratch, workspace, ws_bytes, s,
                                      sample_tiles(o), pm) != QSV_OK)
                    return false;
                t[r] = 0.f;
                for (float x : pm) t[r] += x;
            }
            std::sort(t, t + kReps);
            *ms = t[kReps / 2];
            return true;
        }
        if (sv_simulate(amps_scratch, c, 0, QSV_INIT_PLUS, 0, layer_begin, layer_end, &o, nullptr,
                        nullptr, 0, nullptr, 0, workspace, ws_bytes, stream) != QSV_OK)
            return false;
        float t[kReps];
        for (int r = 0; r < kReps; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess ||
                sv_simulate(amps_scratch, c, 0, QSV_INIT_PLUS, 0, layer_begin, layer_end, &o, nullptr,
                            nullptr, 0, nullptr, 0, workspace, ws_bytes, stream) != QSV_OK ||
                hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
                return false;
        }
        std::sort(t, t + kReps);
        *ms = t[kReps / 2];
        return true;
    };
    // shapes first with the default kernel form, then, for the fastest three,
    // the persistent form and the form that stages exchanges whole
    std::vector<std::pair<float, qsv_fuse_opts>> timed;
    for (auto &pp : plans) {
        if (pp.first > best_passes + 1) continue;
        float ms;
        if (time_one(pp.second, &ms)) timed.push_back({ms, pp.second});
    }
    std::sort(timed.begin(), timed.end(),
              [](const std::pair<float, qsv_fuse_opts> &a, const std::pair<float, qsv_fuse_opts> &b) {
                  return a.first < b.first;
              });
    const size_t shapes = timed.size();
    for (size_t i = 0; i < std::min<size_t>(3, shapes); ++i) {
        for (int form : {2, 4}) {  // persistent; one tile per workgroup with exchanges staged whole
            qsv_fuse_opts o = timed[i].second;
            o.jit = form;
            float ms;
            if (time_one(o, &ms)) timed.push_back({ms, o});
        }
    }
    if (shapes > 0) {
        // per-pass kernel form for the fastest shape: each pass in the faster
        // of the two forms (median of kReps timings per pass)
        qsv_fuse_opts o1 = timed[0].second, o2 = timed[0].second;
        o1.jit = 1;
        o2.jit = 2;
        std::vector<std::vector<float>> t1(kReps), t2(kReps);
        bool ok = true;
        for (int r = 0; r < kReps && ok; ++r)
            ok = time_sweep_passes(c, layer_begin, layer_end, &o1, amps_scratch, workspace, ws_bytes, s,
                                   sample_tiles(o1), t1[r]) == QSV_OK &&
                 time_sweep_passes(c, layer_begin, layer_end, &o2, amps_scratch, workspace, ws_bytes, s,
                                   sample_tiles(o2), t2[r]) == QSV_OK;
        if (ok && t1[0].size() == t2[0].size()) {
            uint32_t mask = 0;
            const size_t np = std::min<size_t>(t1[0].size(), kJitPassBits);
            for (size_t p = 0; p < np; ++p) {
                float a[kReps], b[kReps];
                for (int r = 0; r < kReps; ++r) {
                    a[r] = t1[size_t(r)][p];
                    b[r] = t2[size_t(r)][p];
                }
                std::sort(a, a + kReps);
                std::sort(b, b + kReps);
                if (b[kReps / 2] < a[kReps / 2]) mask |= 1u << p;
            }
            const uint32_t all = np >= 32 ? ~0u : ((1u << np) - 1);
            if (mask != 0 && mask != all) {
                qsv_fuse_opts o3 = timed[0].second;
                o3.jit = 3;
                o3.pass_forms = mask;
                float ms;
                if (time_one(o3, &ms)) timed.push_back({ms, o3});
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (timed.empty()) return fail(QSV_EHIP, "sv_tune: no candidate ran");
    auto best = std::min_element(
        timed.begin(), timed.end(),
        [](const std::pair<float, qsv_fuse_opts> &a, const std::pair<float, qsv_fuse_opts> &b) {
            return a.first < b.first;
        });
    {
        std::lock_guard<std::mutex> g(g_tmu);
        g_tuned[key_of(c, layer_begin, layer_end)] = best->second;
    }
    *out = best->second;
    if (best_ms) *best_ms = best->first;
    disk_store(dkey, best->second, best->first);
    return QSV_OK;
}

// Options chosen for another circuit of the same size class (batches tune
// one representative per class and hand its choice to the others).
extern "C" qsv_status sv_tune_set(const qsv_circuit *c, int layer_begin, int layer_end,
                                  const qsv_fuse_opts *opts) {
    if (!c || !opts) return fail(QSV_EINVAL, "sv_tune_set: null argument");
    if (opts->reg_qubits < 0 || opts->thread_qubits < 0 || opts->low_qubits < 0)
        return fail(QSV_EINVAL, "sv_tune_set: negative tile shape");
    std::lock_guard<std::mutex> g(g_tmu);
    g_tuned[key_of(c, layer_begin, layer_end)] = *opts;
    return QSV_OK;
}

