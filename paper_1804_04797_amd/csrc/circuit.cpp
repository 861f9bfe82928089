// Random lattice circuits and their Schmidt split (host side).
//
// The circuit family is the universal random circuit of Section 2: a 2D grid
// of qubits, an opening layer of Hadamards (layer 0, not counted in the
// depth), CZ gates between lattice neighbours at positions fixed per layer,
// and single-qubit gates drawn from {T, X^1/2, Y^1/2}.  The concrete pattern
// classes, their cycle order and the placement rule are the reading that
// reproduces the gate counts of Table "28qubit" and the cut counts quoted in
// Section 2.1.2; they are spelled out in qsv.h next to circuit_create.
#include <algorithm>
#include <memory>
#include <cstring>

#include "qsv_internal.h"

namespace qsv {

bool gate_is_diagonal(uint8_t k) {
    switch (k) {
    case QSV_T: case QSV_TDG: case QSV_Z: case QSV_CZ: case QSV_P0: case QSV_P1:
    case QSV_PB: case QSV_ZB:
        return true;
    default:
        return false;
    }
}

bool gate_is_single(uint8_t k) { return k != QSV_CZ; }

namespace {

// SplitMix64 (Steele, Lea, Flood: "Fast splittable pseudorandom number
// generators", OOPSLA 2014): a Weyl sequence with golden-ratio increment
// passed through a 64-bit finaliser.
struct SplitMix64 {
    uint64_t s;
    explicit SplitMix64(uint64_t seed) : s(seed) {}
    uint64_t next() {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

struct PatternClass { bool horizontal; int a, b; };

// Cycle of the eight CZ pattern classes; layer t >= 1 uses entry (t-1) mod 8.
const PatternClass kCycle[8] = {
    {true, 0, 0}, {true, 0, 1}, {false, 1, 0}, {false, 1, 1},
    {true, 1, 0}, {false, 0, 1}, {false, 0, 0}, {true, 1, 1},
};

}  // namespace

qsv_status generate_lattice_circuit(int rows, int cols, const uint8_t *present, int depth,
                                    uint64_t seed, qsv_circuit *out) {
    if (rows <= 0 || cols <= 0 || rows * cols > 64)
        return fail(QSV_EINVAL, "lattice must have 1..64 sites");
    if (depth < 0 || depth > 60000)
        return fail(QSV_EINVAL, "depth out of range");
    std::vector<int> qid(rows * cols, -1);
    int n = 0;
    for (int i = 0; i < rows * cols; ++i)
        if (!present || present[i])
            qid[i] = n++;
    if (n == 0)
        return fail(QSV_EINVAL, "lattice has no present site");
    if (n > 63)
        return fail(QSV_ERANGE, "at most 63 qubits per circuit");

    auto site = [&](int r, int c) { return qid[r * cols + c]; };
    // bonds of each class, as sorted (min, max) qubit pairs
    std::vector<std::vector<std::pair<int, int>>> cls(8);
    for (int k = 0; k < 8; ++k) {
        const PatternClass &pc = kCycle[k];
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) {
                int q0, q1;
                if (pc.horizontal) {
                    if (c % 2 != pc.a || r % 2 != pc.b || c + 1 >= cols) continue;
                    q0 = site(r, c); q1 = site(r, c + 1);
                } else {
                    if (r % 2 != pc.a || c % 2 != pc.b || r + 1 >= rows) continue;
                    q0 = site(r, c); q1 = site(r + 1, c);
                }
                if (q0 < 0 || q1 < 0) continue;
                cls[k].push_back({std::min(q0, q1), std::max(q0, q1)});
            }
        std::sort(cls[k].begin(), cls[k].end());
    }

    SplitMix64 rng(seed);
    std::vector<qsv_gate> g;
    auto push = [&](uint8_t kind, int q0, int q1, int layer) {
        qsv_gate x{};
        x.kind = kind; x.q0 = uint8_t(q0); x.q1 = uint8_t(q1 < 0 ? 0 : q1);
        x.layer = uint16_t(layer);
        g.push_back(x);
    };
    for (int q = 0; q < n; ++q) push(QSV_H, q, -1, 0);
    std::vector<char> prev(n, 0), cur(n, 0);
    static const uint8_t kDraw[3] = {QSV_T, QSV_SX, QSV_SY};
    for (int t = 1; t <= depth; ++t) {
        std::fill(cur.begin(), cur.end(), 0);
        for (auto &pr : cls[(t - 1) % 8]) {
            push(QSV_CZ, pr.first, pr.second, t);
            cur[pr.first] = cur[pr.second] = 1;
        }
        for (int q = 0; q < n; ++q) {
            if (prev[q] && !cur[q]) {
                uint64_t r = rng.next();
                int k = int(((r >> 32) * 3ull) >> 32);
                push(kDraw[k], q, -1, t);
            }
        }
        std::swap(prev, cur);
    }
    out->n = n;
    out->depth = depth;
    out->gates.swap(g);
    return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" qsv_status circuit_split(const qsv_circuit *c, uint64_t side_a_mask,
                                    qsv_circuit **half_a, qsv_circuit **half_b, int *c_eff,
                                    int32_t *folded_a, int32_t *folded_b, size_t cap,
                                    size_t *n_folded) {
    if (!c || !half_a || !half_b || !c_eff || !n_folded)
        return fail(QSV_EINVAL, "circuit_split: null argument");
    if (cap && (!folded_a || !folded_b))
        return fail(QSV_EINVAL, "circuit_split: folded arrays are null but cap > 0");
    const int n = c->n;
    const uint64_t all = (n == 64) ? ~0ull : ((1ull << n) - 1);
    if (side_a_mask & ~all)
        return fail(QSV_ERANGE, "circuit_split: mask names qubits beyond n");
    if ((side_a_mask & all) == 0 || (side_a_mask & all) == all)
        return fail(QSV_EINVAL, "circuit_split: both sides must hold qubits");

    std::vector<int> local(n), side(n);
    int na = 0, nb = 0;
    for (int q = 0; q < n; ++q) {
        side[q] = (side_a_mask >> q) & 1;
        local[q] = side[q] ? na++ : nb++;
    }
    // last non-diagonal gate on each qubit
    std::vector<long> last_nd(n, -1);
    for (size_t i = 0; i < c->gates.size(); ++i) {
        const qsv_gate &g = c->gates[i];
        if (!gate_is_diagonal(g.kind)) last_nd[g.q0] = long(i);
    }
    auto A = std::unique_ptr<qsv_circuit>(new qsv_circuit);
    auto B = std::unique_ptr<qsv_circuit>(new qsv_circuit);
    A->n = na; B->n = nb; A->depth = B->depth = c->depth;
    int cuts = 0;
    size_t folds = 0;
    for (size_t i = 0; i < c->gates.size(); ++i) {
        const qsv_gate &g = c->gates[i];
        if (g.kind == QSV_CZ && side[g.q0] != side[g.q1]) {
            int a = side[g.q0] ? g.q0 : g.q1;
            int b = side[g.q0] ? g.q1 : g.q0;
            if (last_nd[a] < long(i) && last_nd[b] < long(i)) {
                if (folds < cap) { folded_a[folds] = a; folded_b[folds] = b; }
                ++folds;
                continue;
            }
            if (cuts >= 63)
                return fail(QSV_ERANGE, "circuit_split: more than 63 cut CZ gates");
            qsv_gate pa{}; pa.kind = QSV_PB; pa.q0 = uint8_t(local[a]); pa.arg = uint8_t(cuts);
            pa.layer = g.layer;
            qsv_gate zb{}; zb.kind = QSV_ZB; zb.q0 = uint8_t(local[b]); zb.arg = uint8_t(cuts);
            zb.layer = g.layer;
            A->gates.push_back(pa);
            B->gates.push_back(zb);
            ++cuts;
            continue;
        }
        if (g.kind == QSV_CZ && side[g.q0] == side[g.q1]) {
            qsv_gate x = g;
            x.q0 = uint8_t(local[g.q0]); x.q1 = uint8_t(local[g.q1]);
            (side[g.q0] ? A : B)->gates.push_back(x);
            continue;
        }
        qsv_gate x = g;
        x.q0 = uint8_t(local[g.q0]);
        (side[g.q0] ? A : B)->gates.push_back(x);
    }
    *half_a = A.release();
    *half_b = B.release();
    *c_eff = cuts;
    *n_folded = folds;
    return QSV_OK;
}

// Branch levels of a circuit with PB / ZB gates (a circuit_split half).  The
// layers holding PB / ZB gates, ascending, define levels 1..L; every gate gets
// the deepest level among the branch bits it depends on through a chain of
// gates that share a qubit and do not commute, 0 if none (two diagonal gates
// commute, so only a non-diagonal gate on either side of a shared qubit links
// them).  hot[q]: level that every later gate on q inherits (the deepest
// non-diagonal gate on q so far); diag[q]: level that a later non-diagonal
// gate on q inherits (the deepest diagonal gate on q so far).
static void branch_levels(const qsv_circuit &c, std::vector<int> &lev, std::vector<int> &cut_layers,
                          std::vector<uint64_t> &bits) {
    cut_layers.clear();
    for (const qsv_gate &g : c.gates)
        if (g.kind == QSV_PB || g.kind == QSV_ZB) cut_layers.push_back(g.layer);
    std::sort(cut_layers.begin(), cut_layers.end());
    cut_layers.erase(std::unique(cut_layers.begin(), cut_layers.end()), cut_layers.end());
    bits.assign(cut_layers.size(), 0);
    std::vector<int> hot(size_t(c.n), 0), diag(size_t(c.n), 0);
    lev.resize(c.gates.size());
    for (size_t i = 0; i < c.gates.size(); ++i) {
        const qsv_gate &g = c.gates[i];
        const bool nd = !gate_is_diagonal(g.kind), two = g.kind == QSV_CZ;
        int l = 0;
        if (g.kind == QSV_PB || g.kind == QSV_ZB) {
            l = 1 + int(std::lower_bound(cut_layers.begin(), cut_layers.end(), int(g.layer)) - cut_layers.begin());
            bits[size_t(l - 1)] |= 1ull << g.arg;
        }
        l = std::max(l, hot[g.q0]);
        if (two) l = std::max(l, hot[g.q1]);
        if (nd) l = std::max(l, diag[g.q0]);
        lev[i] = l;
        if (nd) {
            hot[g.q0] = l;
        } else {
            diag[g.q0] = std::max(diag[g.q0], l);
            if (two) diag[g.q1] = std::max(diag[g.q1], l);
        }
    }
}

extern "C" qsv_status circuit_branch_levels(const qsv_circuit *c, int *n_levels, uint64_t *level_bits,
                                            size_t cap) {
    if (!c || !n_levels) return fail(QSV_EINVAL, "circuit_branch_levels: null argument");
    if (cap && !level_bits) return fail(QSV_EINVAL, "circuit_branch_levels: level_bits is null but cap > 0");
    std::vector<int> lev, layers;
    std::vector<uint64_t> bits;
    branch_levels(*c, lev, layers, bits);
    *n_levels = int(layers.size());
    for (size_t k = 0; k < bits.size() && k < cap; ++k) level_bits[k] = bits[k];
    return QSV_OK;
}

// The gates of levels [level_begin, level_end) in their original order.  For
// every branch, the stages [0, l1), [l1, l2), ..., [lk, L + 1) run one after
// the other give the circuit's state: a gate moves ahead of another only if
// its level is lower, and then the two commute (otherwise the later one
// would have inherited the level).
extern "C" qsv_status circuit_branch_stage(const qsv_circuit *c, int level_begin, int level_end,
                                           qsv_circuit **out) {
    if (!c || !out) return fail(QSV_EINVAL, "circuit_branch_stage: null argument");
    std::vector<int> lev, layers;
    std::vector<uint64_t> bits;
    branch_levels(*c, lev, layers, bits);
    const int top = int(layers.size()) + 1;
    if (level_end < 0) level_end = top;
    if (level_begin < 0 || level_end > top || level_begin >= level_end)
        return fail(QSV_EINVAL, "circuit_branch_stage: level range outside [0, levels + 1)");
    auto r = std::unique_ptr<qsv_circuit>(new qsv_circuit);
    r->n = c->n;
    r->depth = c->depth;
    for (size_t i = 0; i < c->gates.size(); ++i)
        if (lev[i] >= level_begin && lev[i] < level_end) r->gates.push_back(c->gates[i]);
    *out = r.release();
    return QSV_OK;
}

// Adjoint circuit: reversed order, each gate replaced by its adjoint (T <-> T^dagger,
// X^1/2 <-> (X^1/2)^dagger, Y^1/2 <-> (Y^1/2)^dagger; H, CZ, Z, ZB self-adjoint; the
// projectors P0, P1, PB are self-adjoint).  Layer numbers are mirrored so that
// layer ranges keep their meaning.  Used for the Task-2 amplitude <x|U|psi> =
// <U^dagger x|psi> with the circuit split in time (Section 2.2).
extern "C" qsv_status circuit_inverse(const qsv_circuit *c, qsv_circuit **out) {
    if (!c || !out) return fail(QSV_EINVAL, "circuit_inverse: null argument");
    auto r = std::unique_ptr<qsv_circuit>(new qsv_circuit);
    r->n = c->n;
    r->depth = c->depth;
    int top = 0;
    for (const qsv_gate &g : c->gates) top = std::max(top, int(g.layer));
    r->gates.reserve(c->gates.size());
    for (size_t i = c->gates.size(); i-- > 0;) {
        qsv_gate g = c->gates[i];
        switch (g.kind) {
        case QSV_T: g.kind = QSV_TDG; break;
        case QSV_TDG: g.kind = QSV_T; break;
        case QSV_SX: g.kind = QSV_SXDG; break;
        case QSV_SXDG: g.kind = QSV_SX; break;
        case QSV_SY: g.kind = QSV_SYDG; break;
        case QSV_SYDG: g.kind = QSV_SY; break;
        default: break;  // H, CZ, Z, ZB, P0, P1, PB
        }
        g.layer = uint16_t(top - int(g.layer));
        r->gates.push_back(g);
    }
    *out = r.release();
    return QSV_OK;
}
