// Internal declarations of the qsv library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/qsv.h"

namespace qsv {

constexpr int kMaxQubits = 34;   // 2^34 complex64 = 128 GiB per state
constexpr int kBatchMinQubits = 11;  // smallest state of a batch (tile 2^(4+7))
constexpr int kMaxSlots = 16;    // register + thread slots of one tile
constexpr int kMaxOps = 384;     // op words per pass program (kernel argument)

// Opcodes of a pass program.  Each op is one 64-bit word; XCHG is followed by
// one extra word holding the slot permutation.
enum Opcode : uint32_t {
    OP_END = 0,
    OP_H = 1,      // a = register slot: (x, y) -> (x + y, x - y)
    OP_SX = 2,     // (x, y) -> (x - i y, y - i x)
    OP_SY = 3,     // (x, y) -> (x - y, x + y)
    OP_SXDG = 4,   // (x, y) -> (x + i y, y + i x)
    OP_SYDG = 5,   // (x, y) -> (x + y, y - x)
    OP_PHASE = 8,  // a = locator, b = k: multiply amplitudes with bit = 1 by w^k, w = e^{i pi/4}
    OP_CZ = 9,     // a, b = locators: negate amplitudes with both bits = 1
    OP_PROJ = 10,  // a = locator, b = value l, c = 1 -> l is branch bit b: zero amplitudes with bit != l
    OP_ZB = 11,    // a = locator, b = branch bit j: negate amplitudes with bit = 1 if branch bit j is 1
    OP_XCHG = 12,  // next word: new slot s takes the data of old slot perm[s] (4 bits each)
    OP_SCALE = 13, // multiply every amplitude by the pass scale
};

// Locator byte: < 0x80 -> slot index (register slots 0..R-1, thread slots
// R..R+T-1); 0x80 | p -> non-resident physical index bit p.
constexpr uint8_t kLocGlobal = 0x80;

inline uint64_t make_op(uint32_t code, uint32_t a = 0, uint32_t b = 0, uint32_t c = 0) {
    return uint64_t(code) | (uint64_t(a & 0xff) << 8) | (uint64_t(b & 0xff) << 16) |
           (uint64_t(c & 0xff) << 24);
}

// Kernel argument block of one fused pass.  Plain old data, copied by value
// into the kernel argument segment at launch.
struct PassProg {
    uint64_t ops[kMaxOps];
    uint8_t ld_phys[kMaxSlots];   // physical bit of each slot when loading
    uint8_t st_phys[kMaxSlots];   // physical bit of each slot when storing
    uint8_t glob_bits[48];        // tile index bit i -> physical bit when loading
    uint8_t glob_st[48];          // tile index bit i -> physical bit when storing
    float scale_re, scale_im;
    int32_t n_ops;
    int32_t n_glob;
};
// no padding: the compiled-kernel cache keys on the raw bytes
static_assert(sizeof(PassProg) == 8 * kMaxOps + 2 * kMaxSlots + 96 + 16, "PassProg has padding");

// Device-side tables of a batch (batch.cpp).
struct BatchEntry {
    void *amps;         // state of the entry (complex64[2^n])
    uint64_t branch;    // branch index of PB/ZB gates
    uint32_t prog0;     // index of the entry's first pass program
    uint32_t n;         // qubits
    float init_val;     // 2^{-n/2}
    uint32_t pad;
};
struct BatchSeg {
    uint64_t start;     // first block (work item) of the segment within its round
    uint32_t entry;
    uint32_t pad;
};

// Persistent batch launch (one per tile shape of the generic kernel): work
// items are ordered by pass round, then by entry, then by tile; a workgroup
// takes the next item from a device counter.  Item i of round r is tile
// (i - item_start - seg.start) of entry seg.entry, for the round's last
// segment with start <= i - item_start.  An item of round r > 0 waits until
// its entry has completed r * tiles(entry) items (every tile of its earlier
// passes); it only ever waits on items taken before it, which are held by
// running workgroups, so the launch cannot deadlock.
struct BatchRound {
    uint64_t item_start;  // first item of the round
    uint32_t seg_off;     // its segments in the segment table
    uint32_t nseg;
};

#if defined(__HIP__)
#define QSV_HD __host__ __device__
#else
#define QSV_HD
#endif
// Work item -> (round, entry, tile); items < total items of the launch.
QSV_HD inline void batch_decode(const BatchRound *rounds, int nrounds, const BatchSeg *segs, uint64_t item,
                                int *round, uint32_t *entry, uint64_t *tile) {
    int lo = 0, hi = nrounds - 1;
    while (lo < hi) {  // last round with item_start <= item
        const int mid = (lo + hi + 1) >> 1;
        if (rounds[mid].item_start <= item) lo = mid; else hi = mid - 1;
    }
    const uint64_t local = item - rounds[lo].item_start;
    const BatchSeg *sg = segs + rounds[lo].seg_off;
    int a = 0, b = int(rounds[lo].nseg) - 1;
    while (a < b) {  // last segment with start <= local
        const int mid = (a + b + 1) >> 1;
        if (sg[mid].start <= local) a = mid; else b = mid - 1;
    }
    *round = lo;
    *entry = sg[a].entry;
    *tile = local - sg[a].start;
}

struct Pass {
    PassProg prog;
    std::vector<int> gates;       // circuit gate indices, in program order
    uint64_t resident_logical;    // logical qubits resident in this pass
};

struct PlanKey {
    int lb, le, R, T, c;
    bool oop;
    bool operator<(const PlanKey &o) const {
        return std::tie(lb, le, R, T, c, oop) < std::tie(o.lb, o.le, o.R, o.T, o.c, o.oop);
    }
};

// Dense-block plan (dense.cpp): every block is a 2^k x 2^k complex matrix
// on k qubits (local bit i = qubits[i]).
struct DenseBlock {
    std::vector<int> qubits;
    std::vector<float> re, im;      // row-major M
    std::vector<float> re_t, im_t;  // row-major M^T (device layout)
    std::vector<int> gates;
};
struct DensePlan {
    int n = 0, k = 0;
    std::vector<DenseBlock> blocks;
    float *d_mats = nullptr;        // device copy, kept for the life of the process
    std::mutex mu;
};
struct DenseKey {
    int lb, le, k;
    uint64_t branch;
    bool operator<(const DenseKey &o) const {
        return std::tie(lb, le, k, branch) < std::tie(o.lb, o.le, o.k, o.branch);
    }
};

struct Plan {
    int n = 0, R = 0, T = 0, c = 0;
    bool oop = false;  // passes write a second buffer (free qubit-to-bit maps)
    std::vector<Pass> passes;
    std::vector<int> gate_range;  // indices of the gates in the layer range
    std::map<int, std::shared_ptr<void>> jit_variants;  // compiled kernels (jit.cpp)
    std::mutex jit_mu;
};

}  // namespace qsv

struct qsv_circuit {
    int n = 0;
    int depth = 0;
    std::vector<qsv_gate> gates;
    std::mutex mu;
    std::map<qsv::PlanKey, std::shared_ptr<qsv::Plan>> plans;
    std::map<qsv::DenseKey, std::shared_ptr<qsv::DensePlan>> dense;
};

namespace qsv {

// error reporting and the device check (capi.cpp)
qsv_status fail(qsv_status s, const std::string &msg);
qsv_status check_gfx950();  // QSV_EUNSUPPORTED unless the current device is gfx950

// circuit.cpp
bool gate_is_diagonal(uint8_t kind);
bool gate_is_single(uint8_t kind);
qsv_status generate_lattice_circuit(int rows, int cols, const uint8_t *present, int depth,
                                    uint64_t seed, qsv_circuit *out);

// planner.cpp
// oop: every pass but the first reads one buffer and writes the other, so a
// pass may write the state under any qubit-to-bit map; otherwise every pass
// works in place in the natural map.
struct TileShape { int R, T, c; bool oop = false; };
qsv_status build_plan(const qsv_circuit &c, int lb, int le, TileShape shape, Plan &out);
TileShape default_shape(int n);
void gates_in_range(const qsv_circuit &c, int lb, int le, std::vector<int> &idx);

// partition.cpp: the parts of a three-part partition and the combine's
// branch layout (for sv_partition_simulate)
struct PartitionLayout {
    int n = 0, na = 0, nb = 0, eb = 0, ka = 0, kb = 0;
    std::vector<int> qa, qb;              // local -> global qubit (selectors on top)
    std::vector<int32_t> fold_a, fold_b;  // folded pairs (global)
    size_t c_gates = 0;
};
const qsv_circuit *partition_part(const qsv_partition *p, int which);  // 0 A, 1 B, 2 C
void partition_layout(const qsv_partition *p, PartitionLayout &L);
qsv_batch **partition_batch(qsv_partition *p, void ***ws);

// tune.cpp: the shape sv_tune picked for this circuit and layer range, if any
bool tuned_opts(const qsv_circuit *c, int lb, int le, qsv_fuse_opts *out);
// capi.cpp: per-pass times of the compiled sweep from |+>^n (for the tuner)
// max_tiles > 0: every pass runs only its first max_tiles tiles (timing
// on a sample of a large state; the result is not the sweep's)
qsv_status time_sweep_passes(const qsv_circuit *c, int lb, int le, const qsv_fuse_opts *opts,
                             void *amps, void *workspace, size_t ws_bytes, hipStream_t s,
                             uint64_t max_tiles, std::vector<float> &ms);

// dense.cpp
qsv_status build_dense_plan(const qsv_circuit &c, int lb, int le, int k, uint64_t branch,
                            DensePlan &out);

// emulate.cpp
// src == dst for in-place passes
void emulate_pass(const PassProg &p, int n, int R, int T, uint64_t branch, const float *src, float *dst);

}  // namespace qsv
