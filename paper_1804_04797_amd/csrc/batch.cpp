// Batched execution of many states (sv_batch_*).
//
// Many states - the branches of the halves of a cut circuit (Fig. 2, eq. (1))
// or independent circuits of uneven size - are swept together.  Every entry
// has its own state, branch index and pass plan; the pass programs of all
// plans live in one device array.  Pass round r (the r-th pass of every
// entry that has one) is a single launch of the generic tile kernel whose
// blocks cover the tiles of all those entries, located through a segment
// table.  The launches of all rounds and the closing gather of every entry's
// sampled amplitudes are captured once into a hipGraph and replayed: one
// graph launch per batch run.  A kernel boundary between rounds orders the
// passes of each entry; no block waits on another block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <thread>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "jit.h"
#include "kernels.h"
#include "qsv_internal.h"

struct qsv_batch {
    int R = 0, T = 0, c = 0;
    int jit_mode = 0;  // opts->jit: 1 always, -1 never, 0 for plans shared by >= 8 entries
    std::vector<std::vector<uint32_t>> group;       // entries of each plan
    std::vector<char> plan_jit;                     // plan runs as compiled kernels
    std::vector<qsv::BatchEntry *> d_group_ents;    // per compiled plan: its entries' table
    std::vector<const qsv_circuit *> circs;
    std::vector<uint64_t> branches;
    // built for the layer range of the current run
    int built_lb = -1;
    std::vector<std::shared_ptr<qsv::Plan>> plans;
    std::vector<uint32_t> entry_plan;
    std::vector<int> round_seg_off, round_nseg;
    std::vector<uint64_t> round_blocks;
    qsv::PassProg *d_progs = nullptr;
    qsv::BatchEntry *d_ents = nullptr;
    qsv::BatchSeg *d_segs = nullptr;
    std::vector<qsv::BatchEntry> h_ents;
    // captured graph and the arguments it was captured for
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    std::vector<void *> g_ptrs;
    int g_init = -1;
    const void *g_bits = nullptr;
    size_t g_m = 0;
    void *g_table = nullptr;
};

namespace qsv {
namespace {

qsv_status hipfail(hipError_t e, const char *where) {
    return fail(QSV_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

void free_tables(qsv_batch *b) {
    for (auto *p : b->d_group_ents)
        if (p) hipFree(p);
    b->d_group_ents.clear();
    if (b->d_progs) hipFree(b->d_progs);
    if (b->d_ents) hipFree(b->d_ents);
    if (b->d_segs) hipFree(b->d_segs);
    b->d_progs = nullptr;
    b->d_ents = nullptr;
    b->d_segs = nullptr;
}

void drop_graph(qsv_batch *b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

// Size classes: states of 2^21 amplitudes or more stream from HBM (or the
// last-level cache) and are
// swept by compiled kernels of their own plan (unless jit = -1); smaller ones
// share the batch's tile shape and the generic kernel (or compiled kernels per
// plan shared by >= 8 entries).
constexpr int kBigState = 21;
bool big_state(const qsv_batch *b, int n) { return b->jit_mode >= 0 && n >= kBigState; }

// Plans and device tables for layers [lb, end) of every entry.
qsv_status build_tables(qsv_batch *b, int lb) {
    drop_graph(b);
    free_tables(b);
    b->plans.clear();
    b->entry_plan.assign(b->circs.size(), 0);
    std::map<const qsv_circuit *, uint32_t> idx;
    for (size_t i = 0; i < b->circs.size(); ++i) {
        auto it = idx.find(b->circs[i]);
        if (it == idx.end()) {
            qsv_circuit *c = const_cast<qsv_circuit *>(b->circs[i]);
            // states of the HBM-streaming class get their own compiled
            // kernels with the single-state default tile shape
            TileShape sh{b->R, b->T, b->c};
            if (big_state(b, c->n)) {
                sh = default_shape(c->n);
                // the autotuned shape of this circuit (sv_tune / sv_tune_set), if any
                qsv_fuse_opts t;
                if (tuned_opts(c, lb, -1, &t) && t.reg_qubits > 0 && t.thread_qubits > 0 &&
                    fused_shape_supported(t.reg_qubits, t.thread_qubits) &&
                    t.reg_qubits + t.thread_qubits <= c->n) {
                    sh.R = t.reg_qubits;
                    sh.T = t.thread_qubits;
                    sh.c = t.low_qubits > 0 ? t.low_qubits : std::min(5, sh.T + 1);
                }
            }
            PlanKey key{lb, -1, sh.R, sh.T, sh.c, false};
            std::shared_ptr<Plan> p;
            {
                std::lock_guard<std::mutex> g(c->mu);
                auto pit = c->plans.find(key);
                if (pit != c->plans.end()) {
                    p = pit->second;
                } else {
                    p = std::make_shared<Plan>();
                    qsv_status st = build_plan(*c, lb, -1, sh, *p);
                    if (st != QSV_OK) return st;
                    c->plans[key] = p;
                }
            }
            it = idx.emplace(b->circs[i], uint32_t(b->plans.size())).first;
            b->plans.push_back(p);
        }
        b->entry_plan[i] = it->second;
    }
    b->group.assign(b->plans.size(), {});
    for (size_t i = 0; i < b->circs.size(); ++i) b->group[b->entry_plan[i]].push_back(uint32_t(i));
    b->plan_jit.assign(b->plans.size(), 0);
    b->d_group_ents.assign(b->plans.size(), nullptr);
    for (size_t p = 0; p < b->plans.size(); ++p) {
        const bool shared = b->group[p].size() >= 8;
        const bool big = big_state(b, b->plans[p]->n);
        b->plan_jit[p] = !b->plans[p]->passes.empty() &&
                         (b->jit_mode > 0 || (b->jit_mode == 0 && (shared || big))) &&
                         b->group[p].size() < 65536;
        if (b->plan_jit[p]) {
            hipError_t e = hipMalloc(reinterpret_cast<void **>(&b->d_group_ents[p]),
                                     b->group[p].size() * sizeof(BatchEntry));
            if (e != hipSuccess) return fail(QSV_ENOMEM, "sv_batch: group entry table");
        }
    }
    // program array
    std::vector<PassProg> progs;
    std::vector<uint32_t> prog0(b->plans.size());
    size_t max_passes = 0;
    for (size_t p = 0; p < b->plans.size(); ++p) {
        prog0[p] = uint32_t(progs.size());
        for (const Pass &ps : b->plans[p]->passes) progs.push_back(ps.prog);
        max_passes = std::max(max_passes, b->plans[p]->passes.size());
    }
    // entries
    b->h_ents.assign(b->circs.size(), BatchEntry{});
    for (size_t i = 0; i < b->circs.size(); ++i) {
        BatchEntry &e = b->h_ents[i];
        e.amps = nullptr;
        e.branch = b->branches[i];
        e.prog0 = prog0[b->entry_plan[i]];
        e.n = uint32_t(b->circs[i]->n);
        e.init_val = float(std::pow(2.0, -0.5 * e.n));
    }
    // segments per round
    std::vector<BatchSeg> segs;
    b->round_seg_off.clear();
    b->round_nseg.clear();
    b->round_blocks.clear();
    const int L = b->R + b->T;
    for (size_t r = 0; r < max_passes; ++r) {
        b->round_seg_off.push_back(int(segs.size()));
        uint64_t blocks = 0;
        for (size_t i = 0; i < b->circs.size(); ++i) {
            if (b->plan_jit[b->entry_plan[i]]) continue;  // swept by compiled kernels
            if (b->plans[b->entry_plan[i]]->passes.size() <= r) continue;
            BatchSeg s{};
            s.start = blocks;
            s.entry = uint32_t(i);
            segs.push_back(s);
            blocks += 1ull << (b->circs[i]->n - L);
        }
        b->round_nseg.push_back(int(segs.size()) - b->round_seg_off.back());
        b->round_blocks.push_back(blocks);
        if (blocks > (1ull << 31)) return fail(QSV_ERANGE, "sv_batch: too many tiles in one round");
    }
    hipError_t e;
    if (!progs.empty()) {
        e = hipMalloc(reinterpret_cast<void **>(&b->d_progs), progs.size() * sizeof(PassProg));
        if (e != hipSuccess) return fail(QSV_ENOMEM, "sv_batch: program table");
        e = hipMemcpy(b->d_progs, progs.data(), progs.size() * sizeof(PassProg), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(e, "sv_batch: program upload");
    }
    e = hipMalloc(reinterpret_cast<void **>(&b->d_ents), b->h_ents.size() * sizeof(BatchEntry));
    if (e != hipSuccess) return fail(QSV_ENOMEM, "sv_batch: entry table");
    if (!segs.empty()) {
        e = hipMalloc(reinterpret_cast<void **>(&b->d_segs), segs.size() * sizeof(BatchSeg));
        if (e != hipSuccess) return fail(QSV_ENOMEM, "sv_batch: segment table");
        e = hipMemcpy(b->d_segs, segs.data(), segs.size() * sizeof(BatchSeg), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(e, "sv_batch: segment upload");
    }
    b->built_lb = lb;
    b->g_ptrs.clear();
    return QSV_OK;
}

}  // namespace
}  // namespace qsv

using namespace qsv;

extern "C" {

qsv_status sv_batch_create(const qsv_circuit *const *circs, const uint64_t *branch_ids,
                           size_t count, const qsv_fuse_opts *opts, qsv_batch **out) {
    if (!out) return fail(QSV_EINVAL, "sv_batch_create: out is null");
    *out = nullptr;
    if (!circs || count == 0) return fail(QSV_EINVAL, "sv_batch_create: no entries");
    if (count > (1u << 24)) return fail(QSV_ERANGE, "sv_batch_create: too many entries");
    int nmin = 64;
    for (size_t i = 0; i < count; ++i) {
        if (!circs[i]) return fail(QSV_EINVAL, "sv_batch_create: null circuit");
        if (circs[i]->n > kMaxQubits) return fail(QSV_ERANGE, "sv_batch_create: n > 34");
        nmin = std::min(nmin, circs[i]->n);
    }
    auto b = std::unique_ptr<qsv_batch>(new qsv_batch);
    // one tile shape for the whole batch (the generic kernel is instantiated
    // for a few shapes); the largest that fits the smallest state
    static const int shapes[][2] = {{5, 8}, {5, 7}, {4, 7}};
    b->R = 0;
    for (auto &s : shapes)
        if (s[0] + s[1] <= nmin) { b->R = s[0]; b->T = s[1]; break; }
    if (opts && opts->reg_qubits && opts->thread_qubits) {
        b->R = opts->reg_qubits;
        b->T = opts->thread_qubits;
    }
    if (b->R == 0 || nmin < kBatchMinQubits)
        return fail(QSV_EUNSUPPORTED, "sv_batch_create: states need >= 11 qubits");
    const bool ok = (b->R == 5 && (b->T == 8 || b->T == 7)) || (b->R == 4 && (b->T == 8 || b->T == 7));
    if (!ok) return fail(QSV_EUNSUPPORTED, "sv_batch_create: no batch kernel for this tile shape");
    if (b->R + b->T > nmin) return fail(QSV_EUNSUPPORTED, "sv_batch_create: tile larger than a state");
    b->c = (opts && opts->low_qubits) ? opts->low_qubits : std::min(5, b->T + 1);
    b->jit_mode = opts ? opts->jit : 0;
    b->circs.assign(circs, circs + count);
    b->branches.assign(count, 0);
    if (branch_ids) b->branches.assign(branch_ids, branch_ids + count);
    // set kernel attributes outside any capture
    hipError_t e = launch_fused_batch(b->R, b->T, nullptr, 0, nullptr, nullptr, 0, 0, 0, nullptr);
    if (e != hipSuccess) return fail(QSV_EHIP, std::string("sv_batch_create: ") + hipGetErrorString(e));
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(QSV_EHIP, "sv_batch_create: capture stream");
    *out = b.release();
    return QSV_OK;
}

qsv_status sv_batch_run(qsv_batch *b, void *const *amps_dev, int init_plus,
                        const uint64_t *bitstrings_dev, size_t m, void *amp_table_dev,
                        void *stream) {
    if (!b || !amps_dev) return fail(QSV_EINVAL, "sv_batch_run: null argument");
    if (m && (!bitstrings_dev || !amp_table_dev))
        return fail(QSV_EINVAL, "sv_batch_run: null gather buffer");
    const size_t count = b->circs.size();
    for (size_t i = 0; i < count; ++i) {
        if (!amps_dev[i]) return fail(QSV_EINVAL, "sv_batch_run: null state pointer");
        if (reinterpret_cast<uintptr_t>(amps_dev[i]) % 16)
            return fail(QSV_EINVAL, "sv_batch_run: state pointer not 16-byte aligned");
    }
    const int lb = init_plus ? 1 : 0;
    qsv_status st;
    if (b->built_lb != lb && (st = build_tables(b, lb)) != QSV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool same = b->exec && b->g_init == (init_plus ? 1 : 0) && b->g_bits == bitstrings_dev &&
                      b->g_m == m && b->g_table == amp_table_dev && b->g_ptrs.size() == count &&
                      std::equal(b->g_ptrs.begin(), b->g_ptrs.end(), amps_dev);
    if (!same) {
        drop_graph(b);
        for (size_t i = 0; i < count; ++i) b->h_ents[i].amps = amps_dev[i];
        // the previous graph may still read the entry table
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hipfail(e, "sv_batch_run");
        e = hipMemcpy(b->d_ents, b->h_ents.data(), count * sizeof(BatchEntry), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(e, "sv_batch_run: entry upload");
        const int variant = kJitBatched | (init_plus ? (kJitInit | QSV_INIT_PLUS) : 0);
        std::vector<size_t> jp;
        for (size_t p = 0; p < b->plans.size(); ++p) {
            if (!b->plan_jit[p]) continue;
            std::vector<BatchEntry> ge;
            for (uint32_t i : b->group[p]) ge.push_back(b->h_ents[i]);
            e = hipMemcpy(b->d_group_ents[p], ge.data(), ge.size() * sizeof(BatchEntry),
                          hipMemcpyHostToDevice);
            if (e != hipSuccess) return hipfail(e, "sv_batch_run: group entry upload");
            jp.push_back(p);
        }
        // compile the plans' kernels concurrently
        {
            int dev = 0;
            if ((e = hipGetDevice(&dev)) != hipSuccess) return hipfail(e, "sv_batch_run");
            const unsigned nth = std::max(1u, std::min<unsigned>(16, std::thread::hardware_concurrency()));
            std::atomic<size_t> next{0};
            std::vector<qsv_status> res(jp.size(), QSV_OK);
            std::vector<std::thread> pool;
            for (unsigned w = 0; w < std::min<size_t>(nth, jp.size()); ++w)
                pool.emplace_back([&, dev] {
                    (void)hipSetDevice(dev);
                    for (size_t k; (k = next++) < jp.size();) {
                        std::lock_guard<std::mutex> g(b->plans[jp[k]]->jit_mu);
                        res[k] = jit_prepare(*b->plans[jp[k]], variant);
                    }
                });
            for (auto &th : pool) th.join();
            for (qsv_status r : res)
                if (r != QSV_OK) return fail(r, "sv_batch_run: compiling pass kernels failed");
        }
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hipfail(e, "sv_batch_run: begin capture");
        hipError_t le = hipSuccess;
        for (size_t p = 0; p < b->plans.size() && le == hipSuccess; ++p) {
            if (!b->plan_jit[p]) continue;
            if (jit_launch_batched(*b->plans[p], variant, b->d_group_ents[p],
                                   unsigned(b->group[p].size()), b->cap) != QSV_OK)
                le = hipErrorLaunchFailure;
        }
        for (size_t r = 0; r < b->round_blocks.size() && le == hipSuccess; ++r)
            le = launch_fused_batch(b->R, b->T, b->d_segs + b->round_seg_off[r], b->round_nseg[r],
                                    b->d_ents, b->d_progs, int(r), b->round_blocks[r],
                                    init_plus ? 1 : 0, b->cap);
        if (le == hipSuccess && m)
            le = launch_gather_batch(b->d_ents, count, bitstrings_dev, m,
                                     static_cast<float2 *>(amp_table_dev), b->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hipfail(le, "sv_batch_run: launch during capture");
        }
        if (e != hipSuccess) return hipfail(e, "sv_batch_run: end capture");
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return hipfail(e, "sv_batch_run: instantiate");
        b->g_ptrs.assign(amps_dev, amps_dev + count);
        b->g_init = init_plus ? 1 : 0;
        b->g_bits = bitstrings_dev;
        b->g_m = m;
        b->g_table = amp_table_dev;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hipfail(e, "sv_batch_run: graph launch");
    return QSV_OK;
}

void sv_batch_destroy(qsv_batch *b) {
    if (!b) return;
    drop_graph(b);
    free_tables(b);
    if (b->cap) hipStreamDestroy(b->cap);
    delete b;
}

}  // extern "C"
