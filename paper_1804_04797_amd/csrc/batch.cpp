// Batched execution of many states (sv_batch_*).
//
// Many states - the branches of the halves of a cut circuit (Fig. 2, eq. (1))
// or independent circuits of uneven size - are swept together.  Every entry
// has its own state, branch index and pass plan; the pass programs of all
// plans live in one device array.  Entries fall into size classes:
//  - states of 2^14 amplitudes or fewer: one tile holds the whole state (the
//    whole circuit in one workgroup, registers and LDS: one read and one
//    write of the state per pass, usually one pass);
//  - larger states below 2^21 amplitudes: the batch's tile shape;
//  - states of 2^21 amplitudes or more: compiled kernels of their own plan
//    on the tile shape autotuned for their class (one launch per plan and
//    pass, all entries of the plan in its grid).
// The generic-kernel classes run as one launch per tile shape and pass
// round, ordered by kernel boundaries.  A persistent form (one launch per
// tile shape over work items (pass round, entry, tile) taken in order from a
// device counter, per-entry counters of completed tiles ordering each
// entry's passes, BatchRound) is built but switched off: its first runs on
// the device did not finish and the cause is not yet found.  The launches
// and the closing gather of every entry's sampled amplitudes are captured
// once into a hipGraph and replayed: one graph launch per run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <thread>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "jit.h"
#include "kernels.h"
#include "qsv_internal.h"

// Entries of the generic kernel that share one tile shape.
struct BatchShape {
    int R = 0, T = 0, c = 0;
    std::vector<uint32_t> entries;
    std::vector<int> round_seg_off, round_nseg;  // per-round launches: their segments
    std::vector<uint64_t> round_blocks;
    std::vector<qsv::BatchRound> rounds;         // persistent launch
    uint64_t items = 0;
    unsigned grid = 0;
    qsv::BatchRound *d_rounds = nullptr;         // into the batch's table block
    qsv::BatchSeg *d_segs = nullptr;
    unsigned long long *d_next = nullptr;
};

struct qsv_batch {
    int R = 0, T = 0, c = 0;
    bool forced_shape = false;  // opts gave a tile shape: every generic entry uses it
    bool persistent = false;    // one persistent launch per tile shape (switched off, see sv_batch_create)
    uint32_t wait_us = 200000;  // longest wait of one persistent work item
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
    std::vector<BatchShape> shapes;
    qsv::PassProg *d_progs = nullptr;
    qsv::BatchEntry *d_ents = nullptr;
    void *d_tabs = nullptr;           // rounds, segments and counters of every shape
    uint32_t *d_done = nullptr;       // per entry: completed tiles (persistent launches)
    uint32_t *d_err = nullptr;        // a bounded wait gave up
    size_t n_counters = 0;            // 32-bit words cleared before every run
    uint32_t *h_abort = nullptr;      // pinned host flag polled by the waits
    uint32_t *d_abort = nullptr;      // its device address
    std::vector<qsv::BatchEntry> h_ents;
    // captured graph and the arguments it was captured for
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    // side streams of the capture: the compiled plans' launches become
    // parallel branches of the graph (fork and join events)
    std::vector<hipStream_t> lanes;
    std::vector<hipEvent_t> lane_done;
    hipEvent_t fork = nullptr;
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
    if (b->d_tabs) hipFree(b->d_tabs);
    b->d_progs = nullptr;
    b->d_ents = nullptr;
    b->d_tabs = nullptr;
    b->d_done = nullptr;
    b->d_err = nullptr;
    b->shapes.clear();
}

void drop_graph(qsv_batch *b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

// Size classes: states of 2^21 amplitudes or more stream from HBM (or the
// last-level cache) and are swept by compiled kernels of their own plan
// (unless jit = -1); smaller ones run the generic kernel (or compiled kernels
// per plan shared by >= 8 entries): states of at most 2^14 amplitudes on a
// tile that holds the whole state, the others on the batch's tile shape.
constexpr int kBigState = 21;
// side streams of a batch's capture (512 uneven circuits: 53.2 ms with
// none, 47.2 with 2, 45.6 with 4, 45.8 with 8, 46.1 with 16)
constexpr int kLanes = 4;
constexpr int kLdsState = 14;
bool big_state(const qsv_batch *b, int n) { return b->jit_mode >= 0 && n >= kBigState; }

// Tile shape (R, T) with R + T = n for a state held by one tile.
bool lds_shape(int n, int *R, int *T) {
    switch (n) {
    case 14: *R = 5; *T = 9; return true;
    case 13: *R = 5; *T = 8; return true;
    case 12: *R = 5; *T = 7; return true;
    case 11: *R = 4; *T = 7; return true;
    default: return false;
    }
}

// Schedule of one tile shape's entries (qubits n[i], pass count np[i],
// entry id ids[i]): per round, a segment per entry that has the pass, block
// offsets within the round, and the round's first work item.
void make_schedule(const std::vector<int> &n, const std::vector<size_t> &np, const std::vector<uint32_t> &ids, int L,
                   std::vector<BatchRound> &rounds, std::vector<BatchSeg> &segs, std::vector<uint64_t> &round_blocks,
                   uint64_t &items) {
    size_t max_passes = 0;
    for (size_t x : np) max_passes = std::max(max_passes, x);
    items = 0;
    for (size_t r = 0; r < max_passes; ++r) {
        BatchRound rd{items, uint32_t(segs.size()), 0};
        uint64_t blocks = 0;
        for (size_t i = 0; i < n.size(); ++i) {
            if (np[i] <= r) continue;
            BatchSeg sg{};
            sg.start = blocks;
            sg.entry = ids[i];
            segs.push_back(sg);
            blocks += 1ull << (n[i] - L);
        }
        rd.nseg = uint32_t(segs.size()) - rd.seg_off;
        rounds.push_back(rd);
        round_blocks.push_back(blocks);
        items += blocks;
    }
}

// Plans and device tables for layers [lb, end) of every entry.
qsv_status build_tables(qsv_batch *b, int lb) {
    drop_graph(b);
    free_tables(b);
    b->plans.clear();
    b->entry_plan.assign(b->circs.size(), 0);
    std::map<const qsv_circuit *, uint32_t> idx;
    std::vector<TileShape> plan_shape;
    for (size_t i = 0; i < b->circs.size(); ++i) {
        auto it = idx.find(b->circs[i]);
        if (it == idx.end()) {
            qsv_circuit *c = const_cast<qsv_circuit *>(b->circs[i]);
            TileShape sh{b->R, b->T, b->c};
            int lr = 0, lt = 0;
            if (big_state(b, c->n)) {
                // states of the HBM-streaming class get their own compiled
                // kernels with the single-state default tile shape
                sh = default_shape(c->n);
                // the autotuned shape of this circuit (sv_tune / sv_tune_set), if any
                qsv_fuse_opts t;
                if (tuned_opts(c, lb, -1, &t) && t.reg_qubits > 0 && t.thread_qubits > 0 &&
                    compiled_shape_supported(t.reg_qubits, t.thread_qubits) &&
                    t.reg_qubits + t.thread_qubits <= c->n) {
                    sh.R = t.reg_qubits;
                    sh.T = t.thread_qubits;
                    sh.c = t.low_qubits > 0 ? t.low_qubits : std::min(5, sh.T + 1);
                }
            } else if (!b->forced_shape && c->n <= kLdsState && lds_shape(c->n, &lr, &lt)) {
                sh = TileShape{lr, lt, std::min(5, lt + 1)};
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
            plan_shape.push_back(sh);
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
    for (size_t p = 0; p < b->plans.size(); ++p) {
        prog0[p] = uint32_t(progs.size());
        for (const Pass &ps : b->plans[p]->passes) progs.push_back(ps.prog);
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
    // generic-kernel entries by tile shape: segments of every pass round
    // (block / item offsets within the round) and the persistent schedule
    std::map<std::pair<int, int>, size_t> shape_of;
    for (size_t i = 0; i < b->circs.size(); ++i) {
        const uint32_t p = b->entry_plan[i];
        if (b->plan_jit[p] || b->plans[p]->passes.empty()) continue;
        const auto key = std::make_pair(plan_shape[p].R, plan_shape[p].T);
        auto it = shape_of.find(key);
        if (it == shape_of.end()) {
            it = shape_of.emplace(key, b->shapes.size()).first;
            BatchShape bs;
            bs.R = plan_shape[p].R;
            bs.T = plan_shape[p].T;
            bs.c = plan_shape[p].c;
            b->shapes.push_back(bs);
        }
        b->shapes[it->second].entries.push_back(uint32_t(i));
    }
    std::vector<std::vector<BatchSeg>> shape_segs(b->shapes.size());
    for (size_t k = 0; k < b->shapes.size(); ++k) {
        BatchShape &bs = b->shapes[k];
        std::vector<int> nq;
        std::vector<size_t> np;
        for (uint32_t i : bs.entries) {
            nq.push_back(b->circs[i]->n);
            np.push_back(b->plans[b->entry_plan[i]]->passes.size());
        }
        make_schedule(nq, np, bs.entries, bs.R + bs.T, bs.rounds, shape_segs[k], bs.round_blocks, bs.items);
        for (const BatchRound &rd : bs.rounds) {
            bs.round_seg_off.push_back(int(rd.seg_off));
            bs.round_nseg.push_back(int(rd.nseg));
        }
        for (uint64_t blocks : bs.round_blocks)
            if (blocks > (1ull << 31)) return fail(QSV_ERANGE, "sv_batch: too many tiles in one round");
        const uint64_t items = bs.items;
        unsigned resident = 0;
        hipError_t e = launch_fused_persistent(bs.R, bs.T, nullptr, 0, nullptr, 0, nullptr, nullptr, 0, nullptr,
                                               nullptr, nullptr, nullptr, 0, 0, nullptr, &resident);
        if (e != hipSuccess) return hipfail(e, "sv_batch: occupancy of the persistent kernel");
        bs.grid = unsigned(std::min<uint64_t>(items, resident));
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
    // one block for the schedule tables and the counters: per shape its
    // rounds and segments, then (cleared before every run) the per-entry
    // done counters, the error word and each shape's item counter
    size_t bytes = 0;
    std::vector<size_t> off_r(b->shapes.size()), off_s(b->shapes.size()), off_n(b->shapes.size());
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    for (size_t k = 0; k < b->shapes.size(); ++k) {
        off_r[k] = bytes;
        bytes = align(bytes + b->shapes[k].rounds.size() * sizeof(BatchRound));
        off_s[k] = bytes;
        bytes = align(bytes + shape_segs[k].size() * sizeof(BatchSeg));
    }
    const size_t off_c = bytes;
    const size_t off_err = off_c + b->circs.size() * sizeof(uint32_t);
    size_t off_next = align(off_err + sizeof(uint32_t));
    for (size_t k = 0; k < b->shapes.size(); ++k) off_n[k] = off_next + k * sizeof(unsigned long long);
    bytes = off_next + b->shapes.size() * sizeof(unsigned long long);
    b->n_counters = (bytes - off_c) / sizeof(uint32_t);
    e = hipMalloc(&b->d_tabs, bytes);
    if (e != hipSuccess) return fail(QSV_ENOMEM, "sv_batch: schedule tables");
    char *base = static_cast<char *>(b->d_tabs);
    std::vector<char> h(off_c, 0);
    for (size_t k = 0; k < b->shapes.size(); ++k) {
        BatchShape &bs = b->shapes[k];
        if (!bs.rounds.empty()) std::memcpy(h.data() + off_r[k], bs.rounds.data(), bs.rounds.size() * sizeof(BatchRound));
        if (!shape_segs[k].empty())
            std::memcpy(h.data() + off_s[k], shape_segs[k].data(), shape_segs[k].size() * sizeof(BatchSeg));
        bs.d_rounds = reinterpret_cast<BatchRound *>(base + off_r[k]);
        bs.d_segs = reinterpret_cast<BatchSeg *>(base + off_s[k]);
        bs.d_next = reinterpret_cast<unsigned long long *>(base + off_n[k]);
    }
    b->d_done = reinterpret_cast<uint32_t *>(base + off_c);
    b->d_err = reinterpret_cast<uint32_t *>(base + off_err);
    if (off_c) {
        e = hipMemcpy(b->d_tabs, h.data(), off_c, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(e, "sv_batch: schedule upload");
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
    if (nmin < kBatchMinQubits) return fail(QSV_EUNSUPPORTED, "sv_batch_create: states need >= 11 qubits");
    // generic-kernel tile shape of the states that one tile cannot hold
    // (the LDS class has a shape per qubit count); opts may force one shape
    // for every generic entry
    b->R = 5;
    b->T = 8;
    if (opts && opts->reg_qubits && opts->thread_qubits) {
        b->R = opts->reg_qubits;
        b->T = opts->thread_qubits;
        b->forced_shape = true;
        const bool ok = (b->R == 5 && (b->T == 9 || b->T == 8 || b->T == 7)) || (b->R == 4 && (b->T == 8 || b->T == 7));
        if (!ok) return fail(QSV_EUNSUPPORTED, "sv_batch_create: no batch kernel for this tile shape");
        if (b->R + b->T > nmin) return fail(QSV_EUNSUPPORTED, "sv_batch_create: tile larger than a state");
    }
    b->c = (opts && opts->low_qubits) ? opts->low_qubits : std::min(5, b->T + 1);
    b->jit_mode = opts ? opts->jit : 0;
    // The persistent launch is switched off: its first runs on the device did
    // not finish (the cause is not yet found), so asking for it is refused
    // and every batch runs one launch per pass round.
    if (const char *v = std::getenv("QSV_BATCH_PERSISTENT"))
        if (v[0] != '0')
            return fail(QSV_EUNSUPPORTED, "sv_batch_create: the persistent batch launch is switched off");
    if (const char *v = std::getenv("QSV_BATCH_WAIT_US")) b->wait_us = uint32_t(std::strtoul(v, nullptr, 10));
    b->circs.assign(circs, circs + count);
    b->branches.assign(count, 0);
    if (branch_ids) b->branches.assign(branch_ids, branch_ids + count);
    // set kernel attributes outside any capture
    hipError_t e = hipSuccess;
    static const int kShapes[][2] = {{5, 9}, {5, 8}, {4, 8}, {5, 7}, {4, 7}};
    for (auto &sh : kShapes)
        if (e == hipSuccess) e = launch_fused_batch(sh[0], sh[1], nullptr, 0, nullptr, nullptr, 0, 0, 0, nullptr);
    if (e != hipSuccess) return fail(QSV_EHIP, std::string("sv_batch_create: ") + hipGetErrorString(e));
    e = hipHostMalloc(reinterpret_cast<void **>(&b->h_abort), sizeof(uint32_t), hipHostMallocCoherent);
    if (e != hipSuccess) return fail(QSV_ENOMEM, "sv_batch_create: abort flag");
    *b->h_abort = 0;
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&b->d_abort), b->h_abort, 0);
    if (e != hipSuccess) return fail(QSV_EHIP, "sv_batch_create: abort flag device address");
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
        // the side streams and their events (below), made before the first
        // capture that has two compiled chains to run side by side
        if (std::count_if(b->plan_jit.begin(), b->plan_jit.end(), [](char j) { return j != 0; }) > 1 &&
            b->lanes.empty()) {
            e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
            for (int k = 0; k < kLanes && e == hipSuccess; ++k) {
                hipStream_t ls = nullptr;
                hipEvent_t je = nullptr;
                if ((e = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking)) != hipSuccess) break;
                if ((e = hipEventCreateWithFlags(&je, hipEventDisableTiming)) != hipSuccess) {
                    hipStreamDestroy(ls);
                    break;
                }
                b->lanes.push_back(ls);
                b->lane_done.push_back(je);
            }
            if (e != hipSuccess) return hipfail(e, "sv_batch_run: side streams");
        }
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hipfail(e, "sv_batch_run: begin capture");
        // counters of the persistent launches start at zero in every replay
        hipError_t le = b->persistent ? launch_zero_u32(b->d_done, b->n_counters, b->cap) : hipSuccess;
        // Each compiled plan's passes form a chain of their own: the chains
        // go to the side streams (largest work first, each to the least
        // loaded stream), so the graph holds them as parallel branches and
        // small states do not leave the device idle one after another; the
        // generic-kernel rounds stay on the capture stream, alongside.
        std::vector<size_t> jplans;
        for (size_t p = 0; p < b->plans.size(); ++p)
            if (b->plan_jit[p]) jplans.push_back(p);
        auto work = [&](size_t p) {
            return double(b->group[p].size()) * std::ldexp(double(b->plans[p]->passes.size()), b->plans[p]->n);
        };
        std::stable_sort(jplans.begin(), jplans.end(), [&](size_t x, size_t y) { return work(x) > work(y); });
        size_t joined = 0;  // side streams that joined the capture
        if (le == hipSuccess && jplans.size() > 1 && !b->lanes.empty()) {
            le = hipEventRecord(b->fork, b->cap);
            while (le == hipSuccess && joined < b->lanes.size()) {
                le = hipStreamWaitEvent(b->lanes[joined], b->fork, 0);
                if (le == hipSuccess) ++joined;
            }
        }
        std::vector<double> load(std::max<size_t>(joined, 1), 0.0);
        for (size_t p : jplans) {
            if (le != hipSuccess) break;
            const size_t k = size_t(std::min_element(load.begin(), load.end()) - load.begin());
            load[k] += work(p);
            if (jit_launch_batched(*b->plans[p], variant, b->d_group_ents[p], unsigned(b->group[p].size()),
                                   joined ? b->lanes[k] : b->cap) != QSV_OK)
                le = hipErrorLaunchFailure;
        }
        for (const BatchShape &bs : b->shapes) {
            if (le != hipSuccess) break;
            if (b->persistent) {
                le = launch_fused_persistent(bs.R, bs.T, bs.d_rounds, int(bs.rounds.size()), bs.d_segs, bs.items,
                                             b->d_ents, b->d_progs, init_plus ? 1 : 0, b->d_done, bs.d_next,
                                             b->d_err, b->d_abort, b->wait_us, bs.grid, b->cap, nullptr);
            } else {
                for (size_t r = 0; r < bs.round_blocks.size() && le == hipSuccess; ++r)
                    le = launch_fused_batch(bs.R, bs.T, bs.d_segs + bs.round_seg_off[r], bs.round_nseg[r],
                                            b->d_ents, b->d_progs, int(r), bs.round_blocks[r],
                                            init_plus ? 1 : 0, b->cap);
            }
        }
        // join every side stream back (also after an error: the capture
        // must end with all of them joined)
        for (size_t k = 0; k < joined; ++k) {
            hipError_t je = hipEventRecord(b->lane_done[k], b->lanes[k]);
            if (je == hipSuccess) je = hipStreamWaitEvent(b->cap, b->lane_done[k], 0);
            if (le == hipSuccess) le = je;
        }
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

qsv_status sv_batch_status(qsv_batch *b, void *stream) {
    if (!b) return fail(QSV_EINVAL, "sv_batch_status: null batch");
    if (!b->d_err) return QSV_OK;  // never run
    uint32_t err = 0;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipMemcpy(&err, b->d_err, sizeof(err), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hipfail(e, "sv_batch_status");
    __atomic_store_n(b->h_abort, 0u, __ATOMIC_SEQ_CST);  // the queued work is done: later runs wait again
    if (err) return fail(QSV_EINTERNAL, "sv_batch_status: a bounded wait of the persistent launch gave up");
    return QSV_OK;
}

qsv_status sv_batch_abort(qsv_batch *b) {
    if (!b || !b->h_abort) return fail(QSV_EINVAL, "sv_batch_abort: null batch");
    __atomic_store_n(b->h_abort, 1u, __ATOMIC_SEQ_CST);
    return QSV_OK;
}

// Host emulation of a persistent launch's schedule (CPU check of the
// ordering rule; no product entry point calls it): `workers` virtual
// workgroups take the work items in order, an item of round r > 0 waits
// until its entry has completed r * tiles items, and a random running item
// completes at each step (planted_early_start != 0: a deliberately wrong
// rule that lets an item start one tile early, for the test that the check
// catches it).  Fails if the emulation stalls, if an item starts
// before every tile of its entry's earlier passes completed, or if some
// (entry, pass, tile) is not run exactly once.
qsv_status sv_debug_batch_schedule(const int *n_qubits, const int *passes, size_t count, int tile_qubits,
                                   int workers, uint64_t seed, int planted_early_start, uint64_t *items_out) {
    if (!n_qubits || !passes || count == 0 || workers <= 0 || tile_qubits <= 0)
        return fail(QSV_EINVAL, "sv_debug_batch_schedule: bad argument");
    std::vector<int> nq(n_qubits, n_qubits + count);
    std::vector<size_t> np(passes, passes + count);
    std::vector<uint32_t> ids(count);
    for (size_t i = 0; i < count; ++i) {
        if (nq[i] < tile_qubits || nq[i] > 30 || passes[i] < 0)
            return fail(QSV_EINVAL, "sv_debug_batch_schedule: state size out of range");
        ids[i] = uint32_t(i);
    }
    std::vector<BatchRound> rounds;
    std::vector<BatchSeg> segs;
    std::vector<uint64_t> blocks;
    uint64_t items = 0;
    make_schedule(nq, np, ids, tile_qubits, rounds, segs, blocks, items);
    if (items_out) *items_out = items;
    std::vector<uint64_t> done(count, 0);
    std::vector<std::vector<uint64_t>> runs(count);  // per entry: times each (pass, tile) ran
    for (size_t i = 0; i < count; ++i) runs[i].assign(np[i] << (nq[i] - tile_qubits), 0);
    struct W { bool busy = false, running = false; int r = 0; uint32_t e = 0; uint64_t t = 0; };
    std::vector<W> w(static_cast<size_t>(workers));
    uint64_t next = 0, rng = seed | 1;
    auto rnd = [&rng]() { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return rng; };
    uint64_t finished = 0;
    while (finished < items) {
        bool progress = false;
        for (W &x : w) {  // take items, start those whose dependency holds
            if (!x.busy && next < items) {
                batch_decode(rounds.data(), int(rounds.size()), segs.data(), next++, &x.r, &x.e, &x.t);
                x.busy = true;
                x.running = false;
                progress = true;
            }
            const uint64_t need = uint64_t(x.r) << (nq[x.e] - tile_qubits);
            if (x.busy && !x.running && done[x.e] + (planted_early_start && need ? 1 : 0) >= need) {
                // every tile of the earlier passes has completed, none of this one yet started early
                for (int r2 = 0; r2 < x.r; ++r2)
                    for (uint64_t t2 = 0; t2 < (1ull << (nq[x.e] - tile_qubits)); ++t2)
                        if (runs[x.e][(uint64_t(r2) << (nq[x.e] - tile_qubits)) + t2] != 1)
                            return fail(QSV_EINTERNAL, "schedule: an item started before its dependency");
                x.running = true;
                progress = true;
            }
        }
        std::vector<size_t> run_idx;
        for (size_t k = 0; k < w.size(); ++k)
            if (w[k].running) run_idx.push_back(k);
        if (run_idx.empty()) {
            if (!progress) return fail(QSV_EINTERNAL, "schedule: the emulated launch stalls");
            continue;
        }
        W &x = w[run_idx[rnd() % run_idx.size()]];
        if (x.r >= int(np[x.e]) || x.t >= (1ull << (nq[x.e] - tile_qubits)))
            return fail(QSV_EINTERNAL, "schedule: decoded item out of range");
        ++runs[x.e][(uint64_t(x.r) << (nq[x.e] - tile_qubits)) + x.t];
        ++done[x.e];
        ++finished;
        x.busy = x.running = false;
    }
    for (size_t i = 0; i < count; ++i)
        for (uint64_t v : runs[i])
            if (v != 1) return fail(QSV_EINTERNAL, "schedule: an item ran other than once");
    return QSV_OK;
}

void sv_batch_destroy(qsv_batch *b) {
    if (!b) return;
    drop_graph(b);
    free_tables(b);
    if (b->cap) hipStreamDestroy(b->cap);
    for (hipStream_t ls : b->lanes) hipStreamDestroy(ls);
    for (hipEvent_t ev : b->lane_done) hipEventDestroy(ev);
    if (b->fork) hipEventDestroy(b->fork);
    if (b->h_abort) hipHostFree(b->h_abort);
    delete b;
}

}  // extern "C"
