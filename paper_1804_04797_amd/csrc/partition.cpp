// Three-part partition of a lattice circuit (host side): Section 2.1.1
// (implicit decomposition, eqs. (2)-(3)) and Section 2.1.2 (the dynamic
// programme of Algorithm 1).
//
// Two splitting lines run between lattice rows.  Initially both lie between
// rows r0-1 and r0 (part A = sites above, part B = sites below).  From the
// separation layer t_s on they move apart, the upper one up by i_k rows and
// the lower one down by j_k rows in column k (offsets never decrease); the
// sites between them form part C.  While the lines coincide every CZ joining
// the two sides is cut, CZ = sum_l Z^l (x) P_l; afterwards no CZ may join two
// different parts.  All gates of A and B commute with the later gates of C
// (disjoint qubits), so psi_out = U_C sum_l phi_l (x) xi_l, and U_C acts on
// the block of each fixed value of the qubits outside C (eq. (3)).
//
// A cut is free on side B when its B qubit sees no non-diagonal gate of part
// B after the cut: the projector then commutes to the end of part B and
// xi_l[x] = [x_b = l] xi'[x], so B needs no branch bit for it and the sum over
// l picks phi_{l = x_b}.  Free on side A alike; free on both sides it is the
// output sign (-1)^{x_a x_b}.  Space exponents: f = n_A + (cuts not free on
// A), g = n_B + (cuts not free on B), c = |C| after the last layer; the plan
// minimises 2^f + 2^g + 2^c.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "qsv_internal.h"

namespace qsv {
namespace {

constexpr int kNoLayer = 1 << 30;
constexpr size_t kMaxStates = size_t(1) << 22;  // positions of one line

struct Geometry {
    int rows = 0, cols = 0, r0 = 0, n = 0, depth = 0;
    std::vector<int> row, col;  // per qubit
    std::vector<int> at;        // site -> qubit or -1
    int qubit_at(int r, int c) const {
        return (r < 0 || r >= rows || c < 0 || c >= cols) ? -1 : at[r * cols + c];
    }
};

struct Cut {
    size_t gate;
    int a, b, layer;
    int nd_a, nd_b;  // layer of the first non-diagonal gate on a / b after the cut
};

struct Scheme {
    int t_s = 1;
    std::vector<uint8_t> ups, dns;  // (depth + 1 - t_s) x cols
};

qsv_status make_geometry(const qsv_circuit &c, int rows, int cols, const uint8_t *present, int r0,
                         Geometry &G) {
    if (rows <= 0 || cols <= 0 || rows * cols > 64)
        return fail(QSV_EINVAL, "partition: lattice must have 1..64 sites");
    if (r0 < 1 || r0 >= rows) return fail(QSV_EINVAL, "partition: r0 must lie in 1..rows-1");
    G.rows = rows; G.cols = cols; G.r0 = r0;
    G.at.assign(rows * cols, -1);
    int q = 0;
    for (int r = 0; r < rows; ++r)
        for (int k = 0; k < cols; ++k)
            if (!present || present[r * cols + k]) {
                G.at[r * cols + k] = q++;
                G.row.push_back(r);
                G.col.push_back(k);
            }
    if (q != c.n) return fail(QSV_EINVAL, "partition: lattice size does not match the circuit");
    G.n = q;
    G.depth = 0;
    for (const qsv_gate &g : c.gates) {
        if (g.kind == QSV_PB || g.kind == QSV_ZB)
            return fail(QSV_EINVAL, "partition: circuit already holds branch gates");
        G.depth = std::max(G.depth, int(g.layer));
    }
    int na = 0;
    for (int x = 0; x < G.n; ++x) na += G.row[x] < r0;
    if (na == 0 || na == G.n) return fail(QSV_EINVAL, "partition: both sides must hold qubits");
    return QSV_OK;
}

// CZs of layers 1..t_s-1 joining the two sides, with the layer of the first
// later non-diagonal gate on each of their qubits.
std::vector<Cut> cuts_before(const qsv_circuit &c, const Geometry &G, int t_s) {
    std::vector<Cut> out;
    for (size_t i = 0; i < c.gates.size(); ++i) {
        const qsv_gate &g = c.gates[i];
        if (g.kind != QSV_CZ || g.layer < 1 || int(g.layer) >= t_s) continue;
        const bool s0 = G.row[g.q0] < G.r0, s1 = G.row[g.q1] < G.r0;
        if (s0 == s1) continue;
        Cut x;
        x.gate = i;
        x.a = s0 ? g.q0 : g.q1;
        x.b = s0 ? g.q1 : g.q0;
        x.layer = g.layer;
        x.nd_a = x.nd_b = kNoLayer;
        for (size_t j = i + 1; j < c.gates.size(); ++j) {
            const qsv_gate &h = c.gates[j];
            if (gate_is_diagonal(h.kind)) continue;
            if (h.q0 == x.a && x.nd_a == kNoLayer) x.nd_a = h.layer;
            if (h.q0 == x.b && x.nd_b == kNoLayer) x.nd_b = h.layer;
        }
        out.push_back(x);
    }
    return out;
}

// part of a site under offsets u (upper) and d (lower): 0 = A, 1 = B, 2 = C
int part_of(const Geometry &G, int q, const uint8_t *u, const uint8_t *d) {
    const int r = G.row[q], k = G.col[q];
    if (r < G.r0 - u[k]) return 0;
    if (r >= G.r0 + d[k]) return 1;
    return 2;
}

// ---------------------------------------------------------------------------
// Algorithm 1 for one line.  Positions are mixed-radix numbers (digit k =
// offset of column k).  h[s] = the largest number of this side's cuts made
// free so far (f = n + K - h); a move from j to i at layer t puts the sites
// between the two positions into part C from layer t on.  The maximum over
// all earlier positions j <= i is taken one column at a time (the gain of a
// move is a sum of per-column terms), tracking the predecessor of each state.
struct LineDP {
    int cols = 0;
    std::vector<int> radix, stride;
    size_t states = 0;
    std::vector<std::vector<char>> legal;  // [layer][state]
    int digit(size_t s, int k) const { return int(s / stride[k]) % radix[k]; }
};

qsv_status line_setup(const qsv_circuit &c, const Geometry &G, int max_move, bool upper, LineDP &L) {
    L.cols = G.cols;
    L.radix.resize(G.cols);
    L.stride.resize(G.cols);
    size_t s = 1;
    for (int k = 0; k < G.cols; ++k) {
        L.radix[k] = 1 + std::min(max_move, upper ? G.r0 : G.rows - G.r0);
        L.stride[k] = int(s);
        s *= size_t(L.radix[k]);
        if (s > kMaxStates) return fail(QSV_EUNSUPPORTED, "partition: too many line positions");
    }
    L.states = s;
    // legality per layer: no CZ with exactly one qubit on the far side of the line
    std::vector<std::vector<std::pair<int, int>>> cz(G.depth + 1);
    for (const qsv_gate &g : c.gates)
        if (g.kind == QSV_CZ) cz[g.layer].push_back({g.q0, g.q1});
    L.legal.assign(G.depth + 1, std::vector<char>());
    for (int t = 1; t <= G.depth; ++t) {
        std::vector<char> &lg = L.legal[t];
        lg.assign(L.states, 1);
        for (size_t st = 0; st < L.states; ++st) {
            for (auto &pq : cz[t]) {
                const int p = pq.first, q = pq.second;
                const int op = L.digit(st, G.col[p]), oq = L.digit(st, G.col[q]);
                const bool fp = upper ? G.row[p] < G.r0 - op : G.row[p] >= G.r0 + op;
                const bool fq = upper ? G.row[q] < G.r0 - oq : G.row[q] >= G.r0 + oq;
                if (fp != fq) { lg[st] = 0; break; }
            }
        }
    }
    return QSV_OK;
}

// Runs the DP for separation layer t_s.  best[s] = gain of final position s
// (or -1 if unreachable); path reconstructs the positions of layers t_s..depth.
void line_run(const Geometry &G, const LineDP &L, const std::vector<Cut> &cuts, bool upper, int t_s,
              std::vector<int> &best, std::vector<std::vector<uint32_t>> &pred) {
    const int NEG = std::numeric_limits<int>::min() / 4;
    std::vector<int> h(L.states, NEG), nh(L.states);
    std::vector<uint32_t> org(L.states), norg(L.states);
    pred.assign(G.depth + 1 >= t_s ? G.depth + 1 - t_s : 0, std::vector<uint32_t>());
    // cuts of this side per qubit (layer of the first later non-diagonal
    // gate); a cut with none is free whatever the lines do and is counted
    // in the initial value
    std::vector<std::vector<int>> nd_of(G.n);
    int base = 0;
    for (const Cut &x : cuts) {
        const int nd = upper ? x.nd_a : x.nd_b;
        if (nd == kNoLayer) ++base;
        else nd_of[upper ? x.a : x.b].push_back(nd);
    }
    h[0] = base;
    for (int t = t_s; t <= G.depth; ++t) {
        for (size_t s = 0; s < L.states; ++s) org[s] = uint32_t(s);
        for (int k = 0; k < L.cols; ++k) {
            const int R = L.radix[k];
            // gain of moving column k from offset j to offset i at layer t
            std::vector<int> gain_to(R + 1, 0);  // prefix: sites at steps < s
            for (int step = 0; step < R - 1; ++step) {
                const int r = upper ? G.r0 - 1 - step : G.r0 + step;
                const int q = G.qubit_at(r, k);
                int g = 0;
                if (q >= 0)
                    for (int nd : nd_of[q]) g += nd >= t;
                gain_to[step + 1] = gain_to[step] + g;
            }
            for (size_t s = 0; s < L.states; ++s) {
                const int i = L.digit(s, k);
                const size_t base = s - size_t(i) * L.stride[k];
                int bv = NEG;
                uint32_t bo = 0;
                for (int j = 0; j <= i; ++j) {
                    const size_t sj = base + size_t(j) * L.stride[k];
                    if (h[sj] == NEG) continue;
                    const int v = h[sj] + gain_to[i] - gain_to[j];
                    if (v > bv) { bv = v; bo = org[sj]; }
                }
                nh[s] = bv;
                norg[s] = bo;
            }
            std::swap(h, nh);
            std::swap(org, norg);
        }
        const std::vector<char> &lg = L.legal[t];
        for (size_t s = 0; s < L.states; ++s)
            if (!lg[s]) h[s] = NEG;
        pred[t - t_s] = org;
    }
    best.assign(L.states, -1);
    for (size_t s = 0; s < L.states; ++s)
        if (h[s] != NEG) best[s] = h[s];
}

void unpack(const LineDP &L, size_t s, uint8_t *out) {
    for (int k = 0; k < L.cols; ++k) out[k] = uint8_t(L.digit(s, k));
}

int sites_between(const Geometry &G, const LineDP &L, size_t s, bool upper) {
    int c = 0;
    for (int k = 0; k < L.cols; ++k)
        for (int step = 0; step < L.digit(s, k); ++step)
            c += G.qubit_at(upper ? G.r0 - 1 - step : G.r0 + step, k) >= 0;
    return c;
}

}  // namespace
}  // namespace qsv

using namespace qsv;

struct qsv_partition {
    Geometry G;
    Scheme S;
    std::vector<Cut> cuts;
    std::vector<char> free_a, free_b;
    std::vector<int> qa, qb, qc;            // global qubits (A and B: local order)
    int eb = 0;                             // branch bits shared by both sides
    std::vector<int> sel_a, sel_b;          // A / B qubits selecting the other side's branch
    std::vector<int32_t> fold_a, fold_b;    // folded pairs (global)
    int f = 0, g = 0;
    std::unique_ptr<qsv_circuit> A, B, C;
    // device run state
    qsv_batch *batch = nullptr;
    void *batch_ws = nullptr;
    ~qsv_partition() {
        if (batch) sv_batch_destroy(batch);
    }
};

namespace qsv {
namespace {

// Offsets of the scheme at layer t (all zero before t_s).
const uint8_t *offsets(const qsv_partition &p, const std::vector<uint8_t> &v, int t,
                       const std::vector<uint8_t> &zero) {
    if (t < p.S.t_s) return zero.data();
    return v.data() + size_t(t - p.S.t_s) * p.G.cols;
}

qsv_status check_scheme(const qsv_circuit &c, const qsv_partition &p) {
    const Geometry &G = p.G;
    const Scheme &S = p.S;
    if (S.t_s < 1 || S.t_s > G.depth + 1) return fail(QSV_EINVAL, "partition: t_s outside 1..depth+1");
    const size_t nl = size_t(G.depth + 1 - S.t_s);
    if (S.ups.size() != nl * G.cols || S.dns.size() != nl * G.cols)
        return fail(QSV_EINVAL, "partition: offsets must cover layers t_s..depth");
    for (size_t l = 0; l < nl; ++l)
        for (int k = 0; k < G.cols; ++k) {
            const int u = S.ups[l * G.cols + k], d = S.dns[l * G.cols + k];
            const int pu = l ? S.ups[(l - 1) * G.cols + k] : 0, pd = l ? S.dns[(l - 1) * G.cols + k] : 0;
            if (u < pu || d < pd || u > G.r0 || d > G.rows - G.r0)
                return fail(QSV_EINVAL, "partition: offsets decrease or leave the lattice");
        }
    std::vector<uint8_t> zero(G.cols, 0);
    for (const qsv_gate &g : c.gates) {
        if (g.kind != QSV_CZ || int(g.layer) < S.t_s) continue;
        const uint8_t *u = offsets(p, S.ups, g.layer, zero), *d = offsets(p, S.dns, g.layer, zero);
        if (part_of(G, g.q0, u, d) != part_of(G, g.q1, u, d))
            return fail(QSV_EINVAL, "partition: a CZ after the separation joins two parts");
    }
    return QSV_OK;
}

// Cut bookkeeping, the three part circuits and the combine's branch layout.
qsv_status build_parts(const qsv_circuit &c, qsv_partition &p) {
    const Geometry &G = p.G;
    const Scheme &S = p.S;
    std::vector<uint8_t> zero(G.cols, 0);
    // layer at which each qubit enters part C
    std::vector<int> enter(G.n, kNoLayer);
    for (int t = S.t_s; t <= G.depth; ++t) {
        const uint8_t *u = offsets(p, S.ups, t, zero), *d = offsets(p, S.dns, t, zero);
        for (int q = 0; q < G.n; ++q)
            if (enter[q] == kNoLayer && part_of(G, q, u, d) == 2) enter[q] = t;
    }
    p.cuts = cuts_before(c, G, S.t_s);
    const size_t K = p.cuts.size();
    p.free_a.assign(K, 0);
    p.free_b.assign(K, 0);
    p.sel_a.clear(); p.sel_b.clear(); p.fold_a.clear(); p.fold_b.clear();
    int n_exp = 0, n_not_a = 0, n_not_b = 0;
    for (size_t i = 0; i < K; ++i) {
        const Cut &x = p.cuts[i];
        p.free_a[i] = x.nd_a >= enter[x.a];
        p.free_b[i] = x.nd_b >= enter[x.b];
        n_not_a += !p.free_a[i];
        n_not_b += !p.free_b[i];
        if (p.free_a[i] && p.free_b[i]) {
            p.fold_a.push_back(x.a);
            p.fold_b.push_back(x.b);
        } else if (p.free_a[i]) {
            if (std::find(p.sel_a.begin(), p.sel_a.end(), x.a) == p.sel_a.end()) p.sel_a.push_back(x.a);
        } else if (p.free_b[i]) {
            if (std::find(p.sel_b.begin(), p.sel_b.end(), x.b) == p.sel_b.end()) p.sel_b.push_back(x.b);
        } else {
            ++n_exp;
        }
    }
    p.eb = n_exp;
    int na = 0;
    for (int q = 0; q < G.n; ++q) na += G.row[q] < G.r0;
    p.f = na + n_not_a;
    p.g = (G.n - na) + n_not_b;
    const int bits_a = p.eb + int(p.sel_b.size()), bits_b = p.eb + int(p.sel_a.size());
    if (bits_a > 40 || bits_b > 40) return fail(QSV_ERANGE, "partition: more than 40 branch bits");
    // local order: qubits that select nothing (ascending), then the selectors
    p.qa.clear(); p.qb.clear();
    for (int q = 0; q < G.n; ++q) {
        const bool in_a = G.row[q] < G.r0;
        std::vector<int> &sel = in_a ? p.sel_a : p.sel_b;
        if (std::find(sel.begin(), sel.end(), q) != sel.end()) continue;
        (in_a ? p.qa : p.qb).push_back(q);
    }
    p.qa.insert(p.qa.end(), p.sel_a.begin(), p.sel_a.end());
    p.qb.insert(p.qb.end(), p.sel_b.begin(), p.sel_b.end());
    std::vector<int> loc(G.n);
    for (size_t i = 0; i < p.qa.size(); ++i) loc[p.qa[i]] = int(i);
    for (size_t i = 0; i < p.qb.size(); ++i) loc[p.qb[i]] = int(i);
    // final part C
    p.qc.clear();
    {
        const uint8_t *u = offsets(p, S.ups, G.depth, zero), *d = offsets(p, S.dns, G.depth, zero);
        if (S.t_s <= G.depth)
            for (int q = 0; q < G.n; ++q)
                if (part_of(G, q, u, d) == 2) p.qc.push_back(q);
    }
    // the three circuits
    p.A.reset(new qsv_circuit);
    p.B.reset(new qsv_circuit);
    p.C.reset(new qsv_circuit);
    p.A->n = int(p.qa.size());
    p.B->n = int(p.qb.size());
    p.C->n = G.n;
    p.A->depth = p.B->depth = p.C->depth = G.depth;
    std::vector<long> cut_of(c.gates.size(), -1);
    for (size_t i = 0; i < K; ++i) cut_of[p.cuts[i].gate] = long(i);
    int next_exp = 0;
    for (size_t i = 0; i < c.gates.size(); ++i) {
        const qsv_gate &g = c.gates[i];
        if (cut_of[i] >= 0) {
            const size_t j = size_t(cut_of[i]);
            const Cut &x = p.cuts[j];
            qsv_gate za{}, pb{};
            za.layer = pb.layer = g.layer;
            if (p.free_a[j] && p.free_b[j]) continue;  // output sign
            if (p.free_b[j]) {
                // P absorbed on side B; A's Z^l takes l from the B qubit's selector bit
                const int sb = int(std::find(p.sel_b.begin(), p.sel_b.end(), x.b) - p.sel_b.begin());
                za.kind = QSV_ZB; za.q0 = uint8_t(loc[x.a]); za.arg = uint8_t(p.eb + sb);
                p.A->gates.push_back(za);
            } else if (p.free_a[j]) {
                // P absorbed on side A; B's Z^l takes l from the A qubit's selector bit
                const int sa = int(std::find(p.sel_a.begin(), p.sel_a.end(), x.a) - p.sel_a.begin());
                za.kind = QSV_ZB; za.q0 = uint8_t(loc[x.b]); za.arg = uint8_t(p.eb + sa);
                p.B->gates.push_back(za);
            } else {
                za.kind = QSV_ZB; za.q0 = uint8_t(loc[x.a]); za.arg = uint8_t(next_exp);
                pb.kind = QSV_PB; pb.q0 = uint8_t(loc[x.b]); pb.arg = uint8_t(next_exp);
                p.A->gates.push_back(za);
                p.B->gates.push_back(pb);
                ++next_exp;
            }
            continue;
        }
        int part;
        if (int(g.layer) < S.t_s) {
            part = G.row[g.q0] < G.r0 ? 0 : 1;
        } else {
            const uint8_t *u = offsets(p, S.ups, g.layer, zero), *d = offsets(p, S.dns, g.layer, zero);
            part = part_of(G, g.q0, u, d);
        }
        qsv_gate y = g;
        if (part == 2) {
            p.C->gates.push_back(y);
            continue;
        }
        y.q0 = uint8_t(loc[g.q0]);
        if (g.kind == QSV_CZ) y.q1 = uint8_t(loc[g.q1]);
        (part == 0 ? p.A : p.B)->gates.push_back(y);
    }
    return QSV_OK;
}

qsv_status plan_scheme(const qsv_circuit &c, const Geometry &G, int max_move, Scheme &out) {
    LineDP U, D;
    qsv_status st;
    if ((st = line_setup(c, G, max_move, true, U)) != QSV_OK) return st;
    if ((st = line_setup(c, G, max_move, false, D)) != QSV_OK) return st;
    int na = 0;
    for (int q = 0; q < G.n; ++q) na += G.row[q] < G.r0;
    const int nb = G.n - na;
    double best_obj = std::numeric_limits<double>::infinity();
    for (int t_s = 1; t_s <= G.depth + 1; ++t_s) {
        const std::vector<Cut> cuts = cuts_before(c, G, t_s);
        const int K = int(cuts.size());
        std::vector<int> bu, bd;
        std::vector<std::vector<uint32_t>> pu, pd;
        line_run(G, U, cuts, true, t_s, bu, pu);
        line_run(G, D, cuts, false, t_s, bd, pd);
        // best gain per number of C sites, for each line
        std::vector<std::pair<int, size_t>> cu(G.n + 1, {-1, 0}), cd(G.n + 1, {-1, 0});
        for (size_t s = 0; s < U.states; ++s)
            if (bu[s] >= 0) {
                const int k = sites_between(G, U, s, true);
                if (bu[s] > cu[k].first) cu[k] = {bu[s], s};
            }
        for (size_t s = 0; s < D.states; ++s)
            if (bd[s] >= 0) {
                const int k = sites_between(G, D, s, false);
                if (bd[s] > cd[k].first) cd[k] = {bd[s], s};
            }
        for (int a = 0; a <= G.n; ++a) {
            if (cu[a].first < 0) continue;
            for (int b = 0; a + b <= G.n; ++b) {
                if (cd[b].first < 0) continue;
                const int f = na + K - cu[a].first, g = nb + K - cd[b].first;
                const double obj = std::ldexp(1.0, f) + std::ldexp(1.0, g) + std::ldexp(1.0, a + b);
                if (obj < best_obj) {
                    best_obj = obj;
                    out.t_s = t_s;
                    const size_t nl = size_t(G.depth + 1 - t_s);
                    out.ups.assign(nl * G.cols, 0);
                    out.dns.assign(nl * G.cols, 0);
                    size_t su = cu[a].second, sd = cd[b].second;
                    for (size_t l = nl; l-- > 0;) {
                        unpack(U, su, &out.ups[l * G.cols]);
                        unpack(D, sd, &out.dns[l * G.cols]);
                        su = pu[l][su];
                        sd = pd[l][sd];
                    }
                }
            }
        }
    }
    if (!std::isfinite(best_obj)) return fail(QSV_EINTERNAL, "partition: no legal scheme");
    return QSV_OK;
}

}  // namespace
}  // namespace qsv

extern "C" {

qsv_status circuit_partition_plan(const qsv_circuit *c, int rows, int cols, const uint8_t *present,
                                  int r0, int max_move, qsv_partition **out) {
    if (!c || !out) return fail(QSV_EINVAL, "circuit_partition_plan: null argument");
    if (max_move < 0) return fail(QSV_EINVAL, "circuit_partition_plan: max_move < 0");
    auto p = std::unique_ptr<qsv_partition>(new qsv_partition);
    qsv_status st = make_geometry(*c, rows, cols, present, r0, p->G);
    if (st != QSV_OK) return st;
    if ((st = plan_scheme(*c, p->G, max_move, p->S)) != QSV_OK) return st;
    if ((st = check_scheme(*c, *p)) != QSV_OK) return st;
    if ((st = build_parts(*c, *p)) != QSV_OK) return st;
    *out = p.release();
    return QSV_OK;
}

qsv_status circuit_partition_create(const qsv_circuit *c, int rows, int cols, const uint8_t *present,
                                    int r0, int t_s, const uint8_t *ups, const uint8_t *dns,
                                    qsv_partition **out) {
    if (!c || !out) return fail(QSV_EINVAL, "circuit_partition_create: null argument");
    auto p = std::unique_ptr<qsv_partition>(new qsv_partition);
    qsv_status st = make_geometry(*c, rows, cols, present, r0, p->G);
    if (st != QSV_OK) return st;
    if (t_s < 1 || t_s > p->G.depth + 1)
        return fail(QSV_EINVAL, "circuit_partition_create: t_s outside 1..depth+1");
    const size_t cnt = size_t(p->G.depth + 1 - t_s) * size_t(cols);
    if (cnt && (!ups || !dns)) return fail(QSV_EINVAL, "circuit_partition_create: null offsets");
    p->S.t_s = t_s;
    p->S.ups.assign(ups, ups + cnt);
    p->S.dns.assign(dns, dns + cnt);
    if ((st = check_scheme(*c, *p)) != QSV_OK) return st;
    if ((st = build_parts(*c, *p)) != QSV_OK) return st;
    *out = p.release();
    return QSV_OK;
}

qsv_status circuit_partition_info(const qsv_partition *p, qsv_partition_info *out) {
    if (!p || !out) return fail(QSV_EINVAL, "circuit_partition_info: null argument");
    std::memset(out, 0, sizeof(*out));
    out->r0 = p->G.r0;
    out->t_s = p->S.t_s;
    out->depth = p->G.depth;
    out->cols = p->G.cols;
    out->n_a = int(p->qa.size());
    out->n_b = int(p->qb.size());
    out->n_c = int(p->qc.size());
    out->cuts = int(p->cuts.size());
    out->explicit_bits = p->eb;
    out->sel_a = int(p->sel_a.size());
    out->sel_b = int(p->sel_b.size());
    out->folded = int(p->fold_a.size());
    out->f = p->f;
    out->g = p->g;
    out->objective = std::ldexp(1.0, p->f) + std::ldexp(1.0, p->g) + std::ldexp(1.0, out->n_c);
    out->branches_a = uint64_t(1) << (p->eb + int(p->sel_b.size()));
    out->branches_b = uint64_t(1) << (p->eb + int(p->sel_a.size()));
    return QSV_OK;
}

qsv_status circuit_partition_offsets(const qsv_partition *p, uint8_t *ups, uint8_t *dns, size_t cap) {
    if (!p) return fail(QSV_EINVAL, "circuit_partition_offsets: null partition");
    const size_t cnt = p->S.ups.size();
    if (cnt > cap) return fail(QSV_ERANGE, "circuit_partition_offsets: buffers too small");
    if (cnt && (!ups || !dns)) return fail(QSV_EINVAL, "circuit_partition_offsets: null buffer");
    std::copy(p->S.ups.begin(), p->S.ups.end(), ups);
    std::copy(p->S.dns.begin(), p->S.dns.end(), dns);
    return QSV_OK;
}

qsv_status circuit_partition_parts(const qsv_partition *p, qsv_circuit **a, qsv_circuit **b,
                                   qsv_circuit **c, int32_t *qubits_a, int32_t *qubits_b) {
    if (!p || !a || !b || !c) return fail(QSV_EINVAL, "circuit_partition_parts: null argument");
    auto copy = [](const qsv_circuit &x) {
        qsv_circuit *y = new qsv_circuit;
        y->n = x.n;
        y->depth = x.depth;
        y->gates = x.gates;
        return y;
    };
    *a = copy(*p->A);
    *b = copy(*p->B);
    *c = copy(*p->C);
    if (qubits_a) std::copy(p->qa.begin(), p->qa.end(), qubits_a);
    if (qubits_b) std::copy(p->qb.begin(), p->qb.end(), qubits_b);
    return QSV_OK;
}

void circuit_partition_destroy(qsv_partition *p) { delete p; }

}  // extern "C"

namespace qsv {

// Device side (capi.cpp): the block combines and the part-C sweep.
const qsv_circuit *partition_part(const qsv_partition *p, int which) {
    return which == 0 ? p->A.get() : which == 1 ? p->B.get() : p->C.get();
}
void partition_layout(const qsv_partition *p, PartitionLayout &L) {
    L.n = p->G.n;
    L.na = int(p->qa.size());
    L.nb = int(p->qb.size());
    L.eb = p->eb;
    L.ka = int(p->sel_a.size());
    L.kb = int(p->sel_b.size());
    L.qa = p->qa;
    L.qb = p->qb;
    L.fold_a = p->fold_a;
    L.fold_b = p->fold_b;
    L.c_gates = p->C->gates.size();
}
qsv_batch **partition_batch(qsv_partition *p, void ***ws) {
    *ws = &p->batch_ws;
    return &p->batch;
}

}  // namespace qsv
