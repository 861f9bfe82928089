// Pass planner: groups the gates of a layer range into full-state passes.
//
// Section 2.4 observes that a chunk of the state held in fast local memory
// can absorb every gate on the chunk's "local" qubits before it is written
// back, that diagonal gates (T, CZ) can be applied on any qubit, and that
// qubit reordering makes this repeatable.  Here a pass streams the whole
// state once in tiles of 2^(R+T) amplitudes: R qubits live in each thread's
// registers, T qubits across the threads of a workgroup, and the remaining
// index bits select the tile.  A non-diagonal gate needs its qubit in a
// register slot; slot contents are permuted through LDS by XCHG ops (the
// analogue of the paper's rank swaps, done per tile instead of as a separate
// transpose of the whole state).  Diagonal gates read the bit of a thread
// slot from the thread index and the bit of a non-resident qubit from the
// tile index.
//
// Scalar factors are pulled out of the non-diagonal gates: H, SX, SY (and
// adjoints) are applied as sum/difference butterflies and each pass ends by
// multiplying the state with the product of the removed factors, so the
// state is exact (up to rounding) after every pass.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

void gates_in_range(const qsv_circuit &c, int lb, int le, std::vector<int> &idx) {
    idx.clear();
    for (size_t i = 0; i < c.gates.size(); ++i) {
        int l = c.gates[i].layer;
        if (l >= lb && (le < 0 || l < le)) idx.push_back(int(i));
    }
}

TileShape default_shape(int n) {
    // (R, T) of the compiled kernels, largest tile first; the tuner may pick
    // another one.  c low bits stay resident so every access is a run of
    // 2^c amplitudes (2^c * 8 bytes).
    static const int shapes[][2] = {{5, 8}, {5, 7}, {4, 7}, {4, 6}, {3, 6}, {3, 4}, {2, 3}};
    for (auto &s : shapes) {
        if (s[0] + s[1] <= n) {
            int c = std::min(5, s[1] + 1);
            return {s[0], s[1], c};
        }
    }
    return {0, 0, 0};
}

namespace {

// Thread slots hold the lowest resident index bits at load and store.
constexpr bool kLanesLow = true;
// Exchanges prefer thread slots 4 and 5 (cross-lane swaps, see build_plan).
constexpr bool kLanePorts = true;

struct G {
    uint8_t kind;
    int q0, q1;   // q1 = -1 for single-qubit gates
    int arg;
    bool nd;      // non-diagonal
};

struct DepGraph {
    std::vector<G> g;
    std::vector<double> w;  // selection weight of each gate
    std::vector<std::vector<int>> succ;
    std::vector<int> npred;
};

DepGraph build_deps(const qsv_circuit &c, const std::vector<int> &idx) {
    DepGraph d;
    const int n = c.n;
    d.g.resize(idx.size());
    d.succ.resize(idx.size());
    d.npred.assign(idx.size(), 0);
    std::vector<int> last_nd(n, -1);
    std::vector<std::vector<int>> since(n);
    for (size_t i = 0; i < idx.size(); ++i) {
        const qsv_gate &x = c.gates[idx[i]];
        G &y = d.g[i];
        y.kind = x.kind;
        y.q0 = x.q0;
        y.q1 = (x.kind == QSV_CZ) ? x.q1 : -1;
        y.arg = x.arg;
        y.nd = !gate_is_diagonal(x.kind);
        std::vector<int> pre;
        int qs[2] = {y.q0, y.q1};
        for (int k = 0; k < 2; ++k) {
            int q = qs[k];
            if (q < 0) continue;
            if (y.nd) {
                for (int p : since[q]) pre.push_back(p);
                if (last_nd[q] >= 0) pre.push_back(last_nd[q]);
            } else if (last_nd[q] >= 0) {
                pre.push_back(last_nd[q]);
            }
        }
        std::sort(pre.begin(), pre.end());
        pre.erase(std::unique(pre.begin(), pre.end()), pre.end());
        for (int p : pre) d.succ[p].push_back(int(i));
        d.npred[i] = int(pre.size());
        for (int k = 0; k < 2; ++k) {
            int q = qs[k];
            if (q < 0) continue;
            if (y.nd) {
                last_nd[q] = int(i);
                since[q].clear();
            } else {
                since[q].push_back(int(i));
            }
        }
    }
    return d;
}

// Gates (in a valid order) that one pass with resident set `res` can apply,
// given the current done flags and pending-predecessor counts.
double simulate_pass(const DepGraph &d, const std::vector<char> &done, const std::vector<int> &pend,
                  uint64_t res, std::vector<int> *order) {
    std::vector<int> p = pend;
    std::vector<char> dn = done;
    // process in index order with a min-heap of ready gates
    std::vector<int> ready;
    for (size_t i = 0; i < d.g.size(); ++i)
        if (!dn[i] && p[i] == 0) ready.push_back(int(i));
    std::make_heap(ready.begin(), ready.end(), std::greater<int>());
    double count = 0;
    while (!ready.empty()) {
        std::pop_heap(ready.begin(), ready.end(), std::greater<int>());
        int i = ready.back();
        ready.pop_back();
        const G &x = d.g[i];
        if (x.nd && !((res >> x.q0) & 1)) continue;  // blocked for this pass
        dn[i] = 1;
        count += d.w[i];
        if (order) order->push_back(i);
        for (int s : d.succ[i]) {
            if (--p[s] == 0) {
                ready.push_back(s);
                std::push_heap(ready.begin(), ready.end(), std::greater<int>());
            }
        }
    }
    return count;
}

int first_pending_nd(const DepGraph &d, const std::vector<char> &done, int q) {
    for (size_t i = 0; i < d.g.size(); ++i)
        if (!done[i] && d.g[i].nd && d.g[i].q0 == q) return int(i);
    return 1 << 30;
}

uint64_t choose_resident(const DepGraph &d, const std::vector<char> &done,
                         const std::vector<int> &pend, int n, int L, uint64_t forced) {
    uint64_t S = forced;
    int size = __builtin_popcountll(S);
    std::vector<int> first(n);
    for (int q = 0; q < n; ++q) first[q] = first_pending_nd(d, done, q);
    while (size < L) {
        int best_q = -1, best_first = 0;
        double best_gain = -1;
        for (int q = 0; q < n; ++q) {
            if ((S >> q) & 1) continue;
            double gain = simulate_pass(d, done, pend, S | (1ull << q), nullptr);
            if (gain > best_gain || (gain == best_gain && first[q] < best_first)) {
                best_gain = gain;
                best_q = q;
                best_first = first[q];
            }
        }
        S |= 1ull << best_q;
        ++size;
    }
    // hill climbing: swap one non-forced member for one outsider
    double cur = simulate_pass(d, done, pend, S, nullptr);
    for (int iter = 0; iter < 4; ++iter) {
        bool improved = false;
        for (int a = 0; a < n && !improved; ++a) {
            if (!((S >> a) & 1) || ((forced >> a) & 1)) continue;
            for (int b = 0; b < n; ++b) {
                if ((S >> b) & 1) continue;
                uint64_t S2 = (S & ~(1ull << a)) | (1ull << b);
                double v = simulate_pass(d, done, pend, S2, nullptr);
                if (v > cur) {
                    S = S2;
                    cur = v;
                    improved = true;
                    break;
                }
            }
        }
        if (!improved) break;
    }
    return S;
}

// Slot bookkeeping of one tile during a pass.
struct Slots {
    int R, T, L;
    int occ[kMaxSlots];   // qubit held by slot
    int where[64];        // slot of a resident qubit, -1 otherwise
    void set(int s, int q) { occ[s] = q; where[q] = s; }
};

struct ProgBuilder {
    std::vector<uint64_t> ops;
    void op(uint64_t w) { ops.push_back(w); }
    // permutation: new slot s takes old slot perm[s]
    void xchg(const int *perm, int L) {
        uint64_t w = 0;
        for (int s = 0; s < L; ++s) w |= uint64_t(perm[s] & 0xf) << (4 * s);
        ops.push_back(make_op(OP_XCHG));
        ops.push_back(w);
    }
};

// slot of a resident qubit, else its physical bit (tile-index bit) at load
uint8_t locator(const Slots &sl, const int *phys, int q) {
    int s = sl.where[q];
    return s >= 0 ? uint8_t(s) : uint8_t(kLocGlobal | phys[q]);
}

}  // namespace

namespace {

// One plan.  The resident set of each pass maximises the summed weight of
// the gates the pass can apply; gate i of the range weighs
// 1 + lambda * (1 - i / count), so lambda > 0 favours finishing old gates.
// nd_cap > 0: a pass applies at most nd_cap non-diagonal gates (the rest
// wait for a later pass), which spreads the butterfly work over the passes.
//
// follow (out-of-place plans): each pass writes the map its final slot
// layout gives, so the store needs no restoring exchange; the qubits in
// register slot 0 and thread slots 0..cl-2 at the end of the pass are then
// forced into the next pass.  Otherwise the map puts the next pass's best
// qubits at the low bits and the pass restores that layout before its store.
qsv_status build_plan_weighted(const qsv_circuit &c, int lb, int le, TileShape shape, double lambda,
                               bool follow, int nd_cap, Plan &out) {
    const int n = c.n;
    const int R = shape.R, T = shape.T, L = R + T, cl = shape.c;
    if (R < 1 || T < 1 || L > n || L > kMaxSlots || cl < 1 || cl - 1 > T || cl > L)
        return fail(QSV_EUNSUPPORTED, "tile shape does not fit the circuit");
    out.passes.clear();
    out.gate_range.clear();
    out.jit_variants.clear();
    out.n = n; out.R = R; out.T = T; out.c = cl; out.oop = shape.oop;
    gates_in_range(c, lb, le, out.gate_range);
    const std::vector<int> &idx = out.gate_range;
    DepGraph d = build_deps(c, idx);
    d.w.resize(d.g.size());
    for (size_t i = 0; i < d.g.size(); ++i)
        d.w[i] = 1.0 + lambda * (1.0 - double(i) / double(d.g.size()));
    const size_t NG = idx.size();
    std::vector<char> done(NG, 0);
    std::vector<int> pend = d.npred;
    size_t n_done = 0;
    // Qubit-to-bit map.  Every pass reads the state under the current map
    // and may write it under another one: the next pass's resident qubits
    // are placed at the lowest physical bits, so that its tiles are compact
    // blocks of memory.  The call starts and ends in the natural map.  The
    // qubits at physical bits 0..cl-1 are resident in the pass that writes
    // that map and in the pass that reads it, so every access is a run of
    // 2^cl contiguous amplitudes (bit 0 pairs two amplitudes per 16-byte
    // access).
    int phys[64], qat[64];
    for (int q = 0; q < n; ++q) phys[q] = qat[q] = q;
    const uint64_t natural = (cl >= 64) ? ~0ull : ((1ull << cl) - 1);
    auto completes = [&](uint64_t Sx) {  // one pass over Sx applies every remaining gate
        std::vector<int> ord;
        simulate_pass(d, done, pend, Sx, &ord);
        return ord.size() == NG - n_done;
    };
    int total_phase = 0;  // exponent of w = e^{i pi/4} removed so far
    int carry_half = 0;   // removed factors of 2^{-1/2} not yet applied
    bool final_scaled = false;

    if (NG == 0) return QSV_OK;
    uint64_t S = choose_resident(d, done, pend, n, L, natural);
    for (;;) {
        const bool natural_now = [&] {
            for (int q = 0; q < n; ++q)
                if (phys[q] != q) return false;
            return true;
        }();
        if (n_done == NG && natural_now && final_scaled) break;
        // --- slot assignment at load time -----------------------------------
        // slot 0 <- the qubit at bit 0; thread slots 0..cl-2 <- the qubits at
        // bits 1..cl-1; with kLanesLow the other thread slots take the lowest
        // remaining bits and the registers the highest, in order of first
        // non-diagonal use in the pass.
        std::vector<int> porder;
        simulate_pass(d, done, pend, S, &porder);
        std::vector<int> first_use(n, 1 << 30);
        for (size_t k = 0; k < porder.size(); ++k) {
            const G &x = d.g[porder[k]];
            if (x.nd && first_use[x.q0] == (1 << 30)) first_use[x.q0] = int(k);
        }
        Slots sl;
        sl.R = R; sl.T = T; sl.L = L;
        std::fill(sl.where, sl.where + 64, -1);
        std::fill(sl.occ, sl.occ + kMaxSlots, -1);
        sl.set(0, qat[0]);
        for (int u = 0; u < cl - 1; ++u) sl.set(R + u, qat[u + 1]);
        std::vector<int> rest;
        for (int b = cl; b < n; ++b)
            if ((S >> qat[b]) & 1) rest.push_back(qat[b]);  // ascending physical bit
        if (kLanesLow) {
            size_t k = 0;
            for (int u = cl - 1; u < T && k < rest.size(); ++u) sl.set(R + u, rest[k++]);
            std::vector<int> hi(rest.begin() + k, rest.end());
            std::stable_sort(hi.begin(), hi.end(),
                             [&](int a, int b) { return first_use[a] < first_use[b]; });
            for (int s2 = 1; s2 < R && size_t(s2 - 1) < hi.size(); ++s2) sl.set(s2, hi[s2 - 1]);
        } else {
            std::stable_sort(rest.begin(), rest.end(),
                             [&](int a, int b) { return first_use[a] < first_use[b]; });
            size_t k = 0;
            for (int s2 = 1; s2 < R && k < rest.size(); ++s2) sl.set(s2, rest[k++]);
            std::sort(rest.begin() + k, rest.end(), [&](int a, int b) { return phys[a] < phys[b]; });
            for (int u = cl - 1; u < T && k < rest.size(); ++u) sl.set(R + u, rest[k++]);
        }
        Pass pass;
        PassProg &P = pass.prog;
        std::memset(&P, 0, sizeof(P));
        pass.resident_logical = S;
        for (int s2 = 0; s2 < L; ++s2) P.ld_phys[s2] = uint8_t(phys[sl.occ[s2]]);
        // tile-index bit i <- the i-th non-resident qubit in physical order
        std::vector<int> tq;
        for (int b = 0; b < n; ++b)
            if (!((S >> qat[b]) & 1)) tq.push_back(qat[b]);
        P.n_glob = int(tq.size());
        for (size_t i = 0; i < tq.size(); ++i) P.glob_bits[i] = uint8_t(phys[tq[i]]);

        // --- list scheduling with register-slot exchanges -------------------
        std::vector<char> dn = done;
        std::vector<int> pd = pend;
        std::vector<char> in_pass(NG, 0);
        for (int i : porder) in_pass[i] = 1;
        ProgBuilder pb;
        const int budget = kMaxOps - 3 - 2;  // keep room for a final XCHG and SCALE
        int m_nd = 0, phase = 0;
        std::vector<int> sched;
        size_t remaining = porder.size();
        while (remaining > 0) {
            bool progress = true;
            while (progress) {
                progress = false;
                for (size_t k = 0; k < porder.size(); ++k) {
                    int i = porder[k];
                    if (dn[i] || pd[i] != 0) continue;
                    const G &x = d.g[i];
                    if (x.nd && !(sl.where[x.q0] >= 0 && sl.where[x.q0] < R)) continue;
                    if (x.nd && nd_cap > 0 && m_nd >= nd_cap) continue;
                    if (int(pb.ops.size()) + 1 > budget) break;
                    // emit
                    switch (x.kind) {
                    case QSV_H: pb.op(make_op(OP_H, sl.where[x.q0])); ++m_nd; break;
                    case QSV_SX: pb.op(make_op(OP_SX, sl.where[x.q0])); ++m_nd; phase += 1; break;
                    case QSV_SY: pb.op(make_op(OP_SY, sl.where[x.q0])); ++m_nd; phase += 1; break;
                    case QSV_SXDG: pb.op(make_op(OP_SXDG, sl.where[x.q0])); ++m_nd; phase += 7; break;
                    case QSV_SYDG: pb.op(make_op(OP_SYDG, sl.where[x.q0])); ++m_nd; phase += 7; break;
                    case QSV_T: pb.op(make_op(OP_PHASE, locator(sl, phys, x.q0), 1)); break;
                    case QSV_TDG: pb.op(make_op(OP_PHASE, locator(sl, phys, x.q0), 7)); break;
                    case QSV_Z: pb.op(make_op(OP_PHASE, locator(sl, phys, x.q0), 4)); break;
                    case QSV_CZ: pb.op(make_op(OP_CZ, locator(sl, phys, x.q0), locator(sl, phys, x.q1))); break;
                    case QSV_P0: pb.op(make_op(OP_PROJ, locator(sl, phys, x.q0), 0, 0)); break;
                    case QSV_P1: pb.op(make_op(OP_PROJ, locator(sl, phys, x.q0), 1, 0)); break;
                    case QSV_PB: pb.op(make_op(OP_PROJ, locator(sl, phys, x.q0), x.arg, 1)); break;
                    case QSV_ZB: pb.op(make_op(OP_ZB, locator(sl, phys, x.q0), x.arg)); break;
                    default: return fail(QSV_EINTERNAL, "planner: unknown gate kind");
                    }
                    dn[i] = 1;
                    --remaining;
                    sched.push_back(i);
                    for (int s : d.succ[i]) --pd[s];
                    progress = true;
                }
                if (int(pb.ops.size()) + 1 > budget) break;
            }
            if (remaining == 0 || int(pb.ops.size()) + 3 > budget) break;
            if (nd_cap > 0 && m_nd >= nd_cap) break;  // the other gates wait for a later pass
            // Stuck: bring the qubits of ready non-diagonal gates into registers.
            std::vector<int> want;
            std::vector<int> next_use(n, 1 << 30);
            for (size_t k = 0; k < porder.size(); ++k) {
                int i = porder[k];
                if (dn[i]) continue;
                const G &x = d.g[i];
                if (!x.nd) continue;
                if (next_use[x.q0] == (1 << 30)) next_use[x.q0] = int(k);
                if (pd[i] == 0 && sl.where[x.q0] >= R &&
                    std::find(want.begin(), want.end(), x.q0) == want.end())
                    want.push_back(x.q0);
            }
            if (want.empty()) break;  // should not happen: some gate is ready
            // victims: register slots ordered by furthest next use
            std::vector<int> regs(R);
            std::iota(regs.begin(), regs.end(), 0);
            std::sort(regs.begin(), regs.end(), [&](int a, int b) {
                return next_use[sl.occ[a]] > next_use[sl.occ[b]];
            });
            int perm[kMaxSlots];
            for (int s2 = 0; s2 < L; ++s2) perm[s2] = s2;
            // Thread slots 4 and 5 are lane bits 4 and 5 of a wave: a register
            // slot swapped with one of them is a cross-lane swap inside each
            // wave (no LDS, no barrier).  Use it when every wanted qubit sits there.
            bool ports = kLanePorts && T >= 6 && want.size() <= 2;
            for (int q : want) ports = ports && (sl.where[q] == R + 4 || sl.where[q] == R + 5);
            if (ports) {
                int k = 0;
                for (int q : want) {
                    const int vs = regs[k++], ts = sl.where[q];
                    perm[vs] = ts;
                    perm[ts] = vs;
                }
                pb.xchg(perm, L);
                int occ_old[kMaxSlots];
                std::copy(sl.occ, sl.occ + L, occ_old);
                for (int s2 = 0; s2 < L; ++s2) sl.set(s2, occ_old[perm[s2]]);
                continue;
            }
            // fill the remaining register capacity with the next-needed thread qubits
            std::vector<int> cand;
            for (int q = 0; q < n; ++q)
                if (sl.where[q] >= R && next_use[q] < (1 << 30) &&
                    std::find(want.begin(), want.end(), q) == want.end())
                    cand.push_back(q);
            std::sort(cand.begin(), cand.end(),
                      [&](int a, int b) { return next_use[a] < next_use[b]; });
            int k = 0;
            std::vector<int> incoming = want;
            for (int q : cand) incoming.push_back(q);
            for (int q : incoming) {
                if (k >= R) break;
                int vs = regs[k];
                // only evict a register qubit that is needed later than q
                if (k >= int(want.size()) && next_use[sl.occ[vs]] <= next_use[q]) break;
                int ts = sl.where[q];
                perm[vs] = ts;
                perm[ts] = vs;
                ++k;
            }
            if (kLanePorts && T >= 6) {
                // a general exchange also parks the next-needed thread qubits
                // at the lane ports for a later cross-lane swap
                std::vector<int> nxt;
                for (int s2 = R; s2 < L; ++s2) {
                    const int q = sl.occ[perm[s2]];
                    if (next_use[q] < (1 << 30)) nxt.push_back(q);
                }
                std::sort(nxt.begin(), nxt.end(), [&](int a, int b) { return next_use[a] < next_use[b]; });
                for (int pi = 0; pi < 2 && pi < int(nxt.size()); ++pi) {
                    const int port = R + 4 + pi;
                    int t2 = -1;
                    for (int s2 = R; s2 < L; ++s2)
                        if (sl.occ[perm[s2]] == nxt[pi]) t2 = s2;
                    if (t2 >= 0 && t2 != port && !(pi == 1 && t2 == R + 4)) std::swap(perm[port], perm[t2]);
                }
            }
            pb.xchg(perm, L);
            int occ_old[kMaxSlots];
            std::copy(sl.occ, sl.occ + L, occ_old);
            for (int s = 0; s < L; ++s) sl.set(s, occ_old[perm[s]]);
        }
        if (sched.empty() && n_done < NG)
            return fail(QSV_EINTERNAL, "planner made no progress");
        // commit the scheduled gates
        for (int i : sched) {
            done[i] = 1;
            ++n_done;
            for (int s2 : d.succ[i]) --pend[s2];
        }

        // --- resident set of the next pass and the map this pass writes -----
        int nphys[64];
        uint64_t S_next = 0;
        if (!shape.oop) {
            // in place: the tile a pass writes is the tile it read
            for (int q = 0; q < n; ++q) nphys[q] = q;
            if (n_done < NG) S_next = choose_resident(d, done, pend, n, L, natural);
        } else if (n_done == NG && (S & natural) == natural) {
            for (int q = 0; q < n; ++q) nphys[q] = q;  // final store in natural order
        } else if (follow && n_done < NG) {
            // The written map follows the slots at the end of the pass, so the
            // store needs no exchange: register slot 0 -> bit 0, thread slots
            // in order -> bits 1..T, the other registers next, then the next
            // pass's new qubits, then the rest.  The qubits at bits 0..cl-1 are
            // forced into the next pass (every access stays a contiguous run).
            std::vector<int> anchor;
            anchor.push_back(sl.occ[0]);
            for (int u = 0; u < cl - 1; ++u) anchor.push_back(sl.occ[R + u]);
            uint64_t A = 0;
            for (int q : anchor) A |= 1ull << q;
            S_next = choose_resident(d, done, pend, n, L, A);
            if (completes(S_next) && (S_next & natural) != natural) {
                const uint64_t S2 = choose_resident(d, done, pend, n, L, A | natural);
                if (completes(S2)) S_next = S2;
            }
            std::vector<int> order;
            order.push_back(sl.occ[0]);
            for (int u = 0; u < T; ++u) order.push_back(sl.occ[R + u]);
            for (int s2 = 1; s2 < R; ++s2) order.push_back(sl.occ[s2]);
            for (int pass2 = 0; pass2 < 2; ++pass2)
                for (int bb = 0; bb < n; ++bb) {
                    const int q = qat[bb];
                    if ((S >> q) & 1) continue;
                    if (((S_next >> q) & 1) == (pass2 == 0)) order.push_back(q);
                }
            for (int b = 0; b < n; ++b) nphys[order[b]] = b;
        } else {
            // anchors: cl qubits resident now and in the next pass
            uint64_t Sf = (n_done < NG) ? choose_resident(d, done, pend, n, L, 0) : natural;
            std::vector<int> anchor;
            for (int b = 0; b < n && int(anchor.size()) < cl; ++b)
                if (((S & Sf) >> qat[b]) & 1) anchor.push_back(qat[b]);
            for (int b = 0; b < n && int(anchor.size()) < cl; ++b)  // top up from S
                if (((S & ~Sf) >> qat[b]) & 1) anchor.push_back(qat[b]);
            uint64_t A = 0;
            for (int q : anchor) A |= 1ull << q;
            S_next = ((Sf & A) == A) ? Sf : choose_resident(d, done, pend, n, L, A);
            if (n_done < NG && completes(S_next) && (S_next & natural) != natural) {
                // a last pass must also hold the natural low bits for its store
                const uint64_t S2 = choose_resident(d, done, pend, n, L, A | natural);
                if (completes(S2)) S_next = S2;
            }
            if (n_done == NG) S_next = choose_resident(d, done, pend, n, L, A | natural);
            // new map from bit 0 up: the anchors, the other qubits resident in
            // both passes, then alternately one resident only in the next pass
            // (its load) and one resident only now (this store), then the rest
            std::vector<int> both, next_only, now_only, other;
            std::vector<char> is_anchor(n, 0);
            for (int q : anchor) is_anchor[q] = 1;
            for (int bb = 0; bb < n; ++bb) {
                const int q = qat[bb];
                if (is_anchor[q]) continue;
                const bool nx = (S_next >> q) & 1, now = (S >> q) & 1;
                (nx && now ? both : nx ? next_only : now ? now_only : other).push_back(q);
            }
            std::vector<int> order(anchor);
            order.insert(order.end(), both.begin(), both.end());
            for (size_t i = 0; i < std::max(next_only.size(), now_only.size()); ++i) {
                if (i < next_only.size()) order.push_back(next_only[i]);
                if (i < now_only.size()) order.push_back(now_only[i]);
            }
            order.insert(order.end(), other.begin(), other.end());
            for (int b = 0; b < n; ++b) nphys[order[b]] = b;
        }
        int nqat[64];
        for (int q = 0; q < n; ++q) nqat[nphys[q]] = q;

        // --- layout for the store ----------------------------------------------
        // slot 0 <- the qubit written to bit 0, thread slots 0..cl-2 <- those
        // written to bits 1..cl-1; with kLanesLow the other thread slots take
        // the resident qubits with the lowest written bits.
        {
            int target[kMaxSlots];  // new slot -> qubit
            for (int s2 = 0; s2 < L; ++s2) target[s2] = -1;
            std::vector<char> used(L, 0), placed(n, 0);
            target[0] = nqat[0];
            used[0] = 1;
            placed[nqat[0]] = 1;
            std::vector<int> res;  // resident qubits by written bit
            for (int b = 1; b < n; ++b)
                if ((S >> nqat[b]) & 1) res.push_back(nqat[b]);
            const int fixed_thr = kLanesLow ? T : cl - 1;
            for (int u = 0; u < fixed_thr && u < int(res.size()); ++u) {
                target[R + u] = res[u];
                used[R + u] = 1;
                placed[res[u]] = 1;
            }
            // everything else stays in its slot where possible
            std::vector<int> homeless;
            for (int q : res) {
                if (placed[q]) continue;
                int s2 = sl.where[q];
                if (!used[s2]) { target[s2] = q; used[s2] = 1; }
                else homeless.push_back(q);
            }
            size_t h = 0;
            for (int s2 = 0; s2 < L; ++s2)
                if (!used[s2]) { target[s2] = homeless[h++]; used[s2] = 1; }
            bool same = true;
            for (int s2 = 0; s2 < L; ++s2) same = same && sl.occ[s2] == target[s2];
            if (!same) {
                int perm[kMaxSlots];
                for (int s2 = 0; s2 < L; ++s2) perm[s2] = sl.where[target[s2]];
                pb.xchg(perm, L);
                int occ_old[kMaxSlots];
                std::copy(sl.occ, sl.occ + L, occ_old);
                for (int s2 = 0; s2 < L; ++s2) sl.set(s2, occ_old[perm[s2]]);
            }
        }
        for (int s2 = 0; s2 < L; ++s2) P.st_phys[s2] = uint8_t(nphys[sl.occ[s2]]);
        for (size_t i = 0; i < tq.size(); ++i) P.glob_st[i] = uint8_t(nphys[tq[i]]);

        total_phase = (total_phase + phase) & 7;
        // The removed factors 2^{-1/2} are applied by the pass that applies
        // the last gates, together with the accumulated phase, so at most one
        // inexact factor is rounded per call.  Until then the state between
        // passes is the true state times 2^{carry_half/2} (true amplitudes
        // have modulus <= 1): powers of two scale FP32 values exactly, so
        // deferring them changes no rounding and saves each intermediate
        // pass a multiply of every amplitude.  Only when the deferred growth
        // would pass 2^60 does an intermediate pass apply its even part.
        carry_half += m_nd;
        const bool last_gates = (n_done == NG) && !final_scaled;
        double mag = 1.0;
        if (last_gates) {
            mag = std::pow(2.0, -0.5 * carry_half);
            carry_half = 0;
        } else if (carry_half > 120) {
            mag = std::ldexp(1.0, -(carry_half / 2));
            carry_half &= 1;
        }
        double sr = mag, si = 0.0;
        if (last_gates) {
            double ang = M_PI / 4.0 * total_phase;
            sr = mag * std::cos(ang);
            si = mag * std::sin(ang);
            if (total_phase % 2 == 0) {  // exact multiples of i
                const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
                sr = mag * re[total_phase / 2];
                si = mag * im[total_phase / 2];
            }
            final_scaled = true;
        }
        P.scale_re = float(sr);
        P.scale_im = float(si);
        // every program closes with SCALE: it also applies the phases that
        // the generic kernel accumulated on thread and tile-index bits
        pb.op(make_op(OP_SCALE));
        if (pb.ops.size() > size_t(kMaxOps))
            return fail(QSV_EINTERNAL, "planner: program too long");
        std::copy(pb.ops.begin(), pb.ops.end(), P.ops);
        P.n_ops = int(pb.ops.size());
        for (int i : sched) pass.gates.push_back(idx[i]);
        out.passes.push_back(std::move(pass));
        std::copy(nphys, nphys + n, phys);
        std::copy(nqat, nqat + n, qat);
        S = S_next;
        if (out.passes.size() > 4 * NG + 8) return fail(QSV_EINTERNAL, "planner does not terminate");
    }
    return QSV_OK;
}

// Exchanges staged through LDS (a swap of register slots with thread slots
// 4/5 only is a cross-lane swap and is not counted).
int exchanges(const Plan &p) {
    int k = 0;
    for (const Pass &x : p.passes)
        for (int pc = 0; pc < x.prog.n_ops; ++pc) {
            if ((x.prog.ops[pc] & 0xff) != OP_XCHG) continue;
            const uint64_t w = x.prog.ops[++pc];
            const int L = p.R + p.T;
            bool lane = p.T >= 6, any = false;
            for (int s = 0; s < L && lane; ++s) {
                const int o = int((w >> (4 * s)) & 0xf);
                if (o == s) continue;
                any = true;
                const int back = int((w >> (4 * o)) & 0xf);
                lane = back == s && ((s < p.R && (o == p.R + 4 || o == p.R + 5)) ||
                                     (o < p.R && (s == p.R + 4 || s == p.R + 5)));
            }
            if (!(lane && any)) ++k;
        }
    return k;
}

// Non-diagonal (butterfly) ops of a pass program.
int butterflies(const Pass &x) {
    int k = 0;
    for (int pc = 0; pc < x.prog.n_ops; ++pc) {
        const int code = int(x.prog.ops[pc] & 0xff);
        if (code == OP_XCHG) ++pc;
        else if (code >= OP_H && code <= OP_SYDG) ++k;
    }
    return k;
}

// Estimated time of a plan in units of one full-state read and write.  A
// pass streams the state once (its first pass, which usually generates the
// state, only writes it); its butterflies cost 2 vector instructions per
// amplitude each, and about kBalance of them take as long as the pass's
// memory traffic at the copy rate (8 B per amplitude each way at ~6 TB/s
// against ~39e12 vector instructions per second, less the pass's other
// instructions).  A pass takes the longer of the two.
constexpr double kBalance = 43.0;
double plan_cost(const Plan &p) {
    double t = 0;
    for (size_t i = 0; i < p.passes.size(); ++i)
        t += std::max(i == 0 ? 0.5 : 1.0, butterflies(p.passes[i]) / kBalance);
    return t;
}

}  // namespace

// The greedy selection is tried with a few gate weightings (and, out of
// place, both map policies); the plan with the fewest passes, then the
// fewest LDS exchanges, is kept.  Then the same greedy runs with a cap on
// the butterflies per pass, from the even share upwards: a capped plan
// with no more passes replaces it when its estimated time (plan_cost) is
// lower, so that no pass is bound by vector-instruction issue while
// another has room.
qsv_status build_plan(const qsv_circuit &c, int lb, int le, TileShape shape, Plan &out) {
    static const double kLambda[] = {0.0, 0.5, 1.0};
    static const int kCapSlack[] = {0, 3, 6, 10, 15};
    const int nl = int(sizeof(kLambda) / sizeof(kLambda[0]));
    const int variants = nl * (shape.oop ? 2 : 1);
    // the variants are independent: plan them concurrently
    std::vector<std::unique_ptr<Plan>> alt(size_t(variants - 1));
    std::vector<qsv_status> ast(size_t(variants - 1), QSV_EINTERNAL);
    std::vector<std::thread> pool;
    for (int v = 1; v < variants; ++v) {
        alt[size_t(v - 1)].reset(new Plan);
        pool.emplace_back([&, v] {
            ast[size_t(v - 1)] = build_plan_weighted(c, lb, le, shape, kLambda[v % nl], v >= nl, 0,
                                                     *alt[size_t(v - 1)]);
        });
    }
    qsv_status st = build_plan_weighted(c, lb, le, shape, kLambda[0], false, 0, out);
    for (auto &th : pool) th.join();
    if (st != QSV_OK) return st;
    for (int v = 1; v < variants; ++v) {
        Plan &a = *alt[size_t(v - 1)];
        if (ast[size_t(v - 1)] != QSV_OK) continue;
        const size_t pa = a.passes.size(), po = out.passes.size();
        if (pa < po || (pa == po && exchanges(a) < exchanges(out))) out.passes = std::move(a.passes);
    }
    // balanced variants
    const size_t P0 = out.passes.size();
    int nd_total = 0;
    for (const Pass &x : out.passes) nd_total += butterflies(x);
    if (P0 < 2 || nd_total == 0) return QSV_OK;
    const int share = int((size_t(nd_total) + P0 - 1) / P0);
    const int ncap = int(sizeof(kCapSlack) / sizeof(kCapSlack[0]));
    const int cvariants = ncap * variants;
    std::vector<std::unique_ptr<Plan>> cap(static_cast<size_t>(cvariants));
    std::vector<qsv_status> cst(static_cast<size_t>(cvariants), QSV_EINTERNAL);
    pool.clear();
    for (int v = 0; v < cvariants; ++v) {
        cap[size_t(v)].reset(new Plan);
        pool.emplace_back([&, v] {
            const int w = v % variants;
            cst[size_t(v)] = build_plan_weighted(c, lb, le, shape, kLambda[w % nl], w >= nl,
                                                 share + kCapSlack[v / variants], *cap[size_t(v)]);
        });
    }
    for (auto &th : pool) th.join();
    double best = plan_cost(out);
    for (int v = 0; v < cvariants; ++v) {
        Plan &a = *cap[size_t(v)];
        if (cst[size_t(v)] != QSV_OK || a.passes.size() > P0) continue;
        const double ca = plan_cost(a);
        if (ca < best - 1e-9) {
            best = ca;
            out.passes = std::move(a.passes);
        }
    }
    return QSV_OK;
}

}  // namespace qsv
