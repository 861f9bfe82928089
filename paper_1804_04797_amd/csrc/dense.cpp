// Dense-block fusion on matrix cores (sv_apply_dense).
//
// The gates of a layer range are grouped into blocks that act on at most k
// qubits; each block becomes one 2^k x 2^k complex matrix M (products of the
// gate matrices formed in FP64 on the host, rounded to complex64) and one
// full-state pass computes Y = M X, where the columns of X are the 2^k
// amplitudes that share all other index bits.  This is the "gate fusion"
// that Section 2.4 contrasts with its local-qubit batching: its cost is
// 8 * 2^k real flops per amplitude whatever the number of gates in the block,
// so it is a matrix-core (FP32 MFMA) workload rather than an HBM one.
//
// Blocks are chosen like passes: repeatedly pick the k-qubit set that admits
// the most gates whose predecessors are applied (every gate of a block acts
// only on the block's qubits, diagonal or not), absorb those gates in
// dependency order, repeat.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "kernels.h"
#include "qsv_internal.h"

namespace qsv {
namespace {

using cd = std::complex<double>;

// 2x2 matrix of a single-qubit gate (row = output bit, column = input bit).
bool gate2(uint8_t kind, int branch_bit, cd m[2][2]) {
    const double s = std::sqrt(0.5);
    const cd i(0, 1);
    m[0][0] = m[1][1] = 1;
    m[0][1] = m[1][0] = 0;
    switch (kind) {
    case QSV_H: m[0][0] = s; m[0][1] = s; m[1][0] = s; m[1][1] = -s; return true;
    case QSV_T: m[1][1] = std::polar(1.0, M_PI / 4); return true;
    case QSV_TDG: m[1][1] = std::polar(1.0, -M_PI / 4); return true;
    case QSV_Z: m[1][1] = -1; return true;
    case QSV_SX: m[0][0] = m[1][1] = 0.5 * (1.0 + i); m[0][1] = m[1][0] = 0.5 * (1.0 - i); return true;
    case QSV_SY: m[0][0] = m[1][0] = m[1][1] = 0.5 * (1.0 + i); m[0][1] = -0.5 * (1.0 + i); return true;
    case QSV_SXDG: m[0][0] = m[1][1] = 0.5 * (1.0 - i); m[0][1] = m[1][0] = 0.5 * (1.0 + i); return true;
    case QSV_SYDG:  // adjoint of SY
        m[0][0] = m[1][1] = 0.5 * (1.0 - i); m[0][1] = 0.5 * (1.0 - i); m[1][0] = -0.5 * (1.0 - i);
        return true;
    case QSV_P0: m[1][1] = 0; return true;
    case QSV_P1: m[0][0] = 0; return true;
    case QSV_PB: if (branch_bit) m[0][0] = 0; else m[1][1] = 0; return true;
    case QSV_ZB: if (branch_bit) m[1][1] = -1; return true;
    default: return false;
    }
}

struct DG { uint8_t kind; int q0, q1, arg; bool nd; };

}  // namespace

qsv_status build_dense_plan(const qsv_circuit &c, int lb, int le, int k, uint64_t branch,
                            DensePlan &out) {
    const int n = c.n;
    if (k < 1 || k > n) return fail(QSV_EINVAL, "dense: k out of range");
    std::vector<int> idx;
    gates_in_range(c, lb, le, idx);
    const size_t G = idx.size();
    std::vector<DG> g(G);
    // predecessors: every earlier gate on a shared qubit (diagonal gates are
    // not reordered across each other here: blocks keep circuit order per qubit)
    std::vector<std::vector<int>> succ(G);
    std::vector<int> last(n, -1);
    for (size_t i = 0; i < G; ++i) {
        const qsv_gate &x = c.gates[idx[i]];
        g[i] = DG{x.kind, x.q0, x.kind == QSV_CZ ? x.q1 : -1, x.arg, !gate_is_diagonal(x.kind)};
        int qs[2] = {g[i].q0, g[i].q1};
        for (int q : qs) {
            if (q < 0) continue;
            if (last[q] >= 0) succ[last[q]].push_back(int(i));
            last[q] = int(i);
        }
    }
    std::vector<char> done(G, 0);
    size_t n_done = 0;
    out.k = k;
    out.n = n;
    out.blocks.clear();
    auto qubits_of = [&](size_t i) {
        uint64_t m = 1ull << g[i].q0;
        if (g[i].q1 >= 0) m |= 1ull << g[i].q1;
        return m;
    };
    while (n_done < G) {
        // gates that can join a block on qubit set S (closure in dependency order)
        auto absorb = [&](uint64_t S, std::vector<int> *order) {
            std::vector<char> dn = done;
            // pending predecessors of every gate not yet applied
            std::vector<int> ready, cnt(G, 0);
            for (size_t i = 0; i < G; ++i)
                for (int s : succ[i])
                    if (!dn[i]) ++cnt[s];
            for (size_t i = 0; i < G; ++i)
                if (!dn[i] && cnt[i] == 0) ready.push_back(int(i));
            int count = 0;
            std::make_heap(ready.begin(), ready.end(), std::greater<int>());
            while (!ready.empty()) {
                std::pop_heap(ready.begin(), ready.end(), std::greater<int>());
                int i = ready.back();
                ready.pop_back();
                if ((qubits_of(i) & ~S) != 0) continue;  // leaves the block
                dn[i] = 1;
                ++count;
                if (order) order->push_back(i);
                for (int s : succ[i])
                    if (--cnt[s] == 0) {
                        ready.push_back(s);
                        std::push_heap(ready.begin(), ready.end(), std::greater<int>());
                    }
            }
            return count;
        };
        // grow S greedily by the gain of one more qubit
        uint64_t S = 0;
        int size = 0;
        {
            // seed with the qubits of the earliest pending gate
            for (size_t i = 0; i < G; ++i)
                if (!done[i]) { S = qubits_of(i); break; }
            size = __builtin_popcountll(S);
        }
        while (size < k) {
            int best_q = -1, best = -1;
            for (int q = 0; q < n; ++q) {
                if ((S >> q) & 1) continue;
                int v = absorb(S | (1ull << q), nullptr);
                if (v > best) { best = v; best_q = q; }
            }
            S |= 1ull << best_q;
            ++size;
        }
        std::vector<int> order;
        absorb(S, &order);
        if (order.empty()) return fail(QSV_EINTERNAL, "dense planner made no progress");
        DenseBlock blk;
        for (int q = 0; q < n; ++q)
            if ((S >> q) & 1) blk.qubits.push_back(q);
        const int dim = 1 << k;
        std::vector<cd> M(size_t(dim) * dim, 0.0);
        for (int r = 0; r < dim; ++r) M[size_t(r) * dim + r] = 1.0;
        auto local = [&](int q) {
            return int(std::find(blk.qubits.begin(), blk.qubits.end(), q) - blk.qubits.begin());
        };
        for (int i : order) {
            const DG &x = g[i];
            if (x.kind == QSV_CZ) {
                const int a = local(x.q0), b = local(x.q1);
                for (int r = 0; r < dim; ++r)
                    if (((r >> a) & 1) && ((r >> b) & 1))
                        for (int col = 0; col < dim; ++col) M[size_t(r) * dim + col] = -M[size_t(r) * dim + col];
                continue;
            }
            cd u[2][2];
            if (!gate2(x.kind, int((branch >> x.arg) & 1), u))
                return fail(QSV_EINTERNAL, "dense: unknown gate");
            const int a = local(x.q0);
            // rows r (bit a = 0) and r | 2^a of M become u applied to them
            for (int r = 0; r < dim; ++r) {
                if ((r >> a) & 1) continue;
                const int r1 = r | (1 << a);
                for (int col = 0; col < dim; ++col) {
                    const cd x0 = M[size_t(r) * dim + col], x1 = M[size_t(r1) * dim + col];
                    M[size_t(r) * dim + col] = u[0][0] * x0 + u[0][1] * x1;
                    M[size_t(r1) * dim + col] = u[1][0] * x0 + u[1][1] * x1;
                }
            }
        }
        blk.re.resize(size_t(dim) * dim);
        blk.im.resize(size_t(dim) * dim);
        for (size_t e = 0; e < M.size(); ++e) {
            blk.re[e] = float(M[e].real());
            blk.im[e] = float(M[e].imag());
        }
        // transposed copy for the device (matrix-core A operands read rows of M^T)
        blk.re_t.resize(blk.re.size());
        blk.im_t.resize(blk.im.size());
        for (int r = 0; r < dim; ++r)
            for (int col = 0; col < dim; ++col) {
                blk.re_t[size_t(col) * dim + r] = blk.re[size_t(r) * dim + col];
                blk.im_t[size_t(col) * dim + r] = blk.im[size_t(r) * dim + col];
            }
        for (int i : order) {
            done[i] = 1;
            ++n_done;
            blk.gates.push_back(idx[i]);
        }
        out.blocks.push_back(std::move(blk));
    }
    return QSV_OK;
}

// Host emulation of one dense block on a complex64 array (CPU checks).
void emulate_dense_block(const DenseBlock &b, int n, float *amps) {
    const int k = int(b.qubits.size());
    const int dim = 1 << k;
    uint64_t qmask = 0;
    for (int q : b.qubits) qmask |= 1ull << q;
    std::vector<float> xr(dim), xi(dim);
    for (uint64_t base = 0; base < (1ull << n); ++base) {
        if (base & qmask) continue;
        auto addr = [&](int r) {
            uint64_t a = base;
            for (int i = 0; i < k; ++i)
                if ((r >> i) & 1) a |= 1ull << b.qubits[i];
            return a;
        };
        for (int r = 0; r < dim; ++r) {
            const uint64_t a = addr(r);
            xr[r] = amps[2 * a];
            xi[r] = amps[2 * a + 1];
        }
        for (int r = 0; r < dim; ++r) {
            double yr = 0, yi = 0;
            for (int col = 0; col < dim; ++col) {
                const double mr = b.re[size_t(r) * dim + col], mi = b.im[size_t(r) * dim + col];
                yr += mr * xr[col] - mi * xi[col];
                yi += mr * xi[col] + mi * xr[col];
            }
            const uint64_t a = addr(r);
            amps[2 * a] = float(yr);
            amps[2 * a + 1] = float(yi);
        }
    }
}

}  // namespace qsv

using namespace qsv;

namespace {

qsv_status dense_prepare(const qsv_circuit *c, int lb, int le, int k, uint64_t branch,
                         std::shared_ptr<DensePlan> &out) {
    if (!c) return fail(QSV_EINVAL, "dense: null circuit");
    if (k < 4 || k > 7) return fail(QSV_EUNSUPPORTED, "dense: k must be 4..7");
    if (c->n < k + 6) return fail(QSV_EUNSUPPORTED, "dense: needs n >= k + 6");
    qsv_circuit *cc = const_cast<qsv_circuit *>(c);
    std::lock_guard<std::mutex> g(cc->mu);
    DenseKey key{lb, le, k, branch};
    auto it = cc->dense.find(key);
    if (it != cc->dense.end()) { out = it->second; return QSV_OK; }
    auto p = std::make_shared<DensePlan>();
    qsv_status st = build_dense_plan(*c, lb, le, k, branch, *p);
    if (st != QSV_OK) return st;
    cc->dense[key] = p;
    out = p;
    return QSV_OK;
}

}  // namespace

extern "C" {

qsv_status sv_apply_dense(void *amps, const qsv_circuit *c, uint64_t branch, int layer_begin,
                          int layer_end, int k, int *n_blocks, void *stream) {
    if (!amps || !c) return fail(QSV_EINVAL, "sv_apply_dense: null argument");
    if (reinterpret_cast<uintptr_t>(amps) % 16) return fail(QSV_EINVAL, "sv_apply_dense: misaligned state");
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_apply_dense: layer_begin < 0");
    std::shared_ptr<DensePlan> plan;
    qsv_status st = dense_prepare(c, layer_begin, layer_end, k, branch, plan);
    if (st != QSV_OK) return st;
    if (n_blocks) *n_blocks = int(plan->blocks.size());
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        std::lock_guard<std::mutex> g(plan->mu);
        if (!plan->d_mats && !plan->blocks.empty()) {
            const size_t per = size_t(2) << (2 * k);  // re + im floats per block
            std::vector<float> host(per * plan->blocks.size());
            for (size_t b = 0; b < plan->blocks.size(); ++b) {
                std::copy(plan->blocks[b].re_t.begin(), plan->blocks[b].re_t.end(), host.begin() + b * per);
                std::copy(plan->blocks[b].im_t.begin(), plan->blocks[b].im_t.end(),
                          host.begin() + b * per + (per / 2));
            }
            hipError_t e = hipMalloc(reinterpret_cast<void **>(&plan->d_mats), host.size() * sizeof(float));
            if (e != hipSuccess) return fail(QSV_ENOMEM, "sv_apply_dense: matrix table");
            e = hipMemcpy(plan->d_mats, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(QSV_EHIP, "sv_apply_dense: matrix upload");
        }
    }
    const size_t per = size_t(2) << (2 * k);
    for (size_t b = 0; b < plan->blocks.size(); ++b) {
        hipError_t e = launch_dense(static_cast<float2 *>(amps), c->n, k, plan->blocks[b].qubits.data(),
                                    plan->d_mats + b * per, s);
        if (e != hipSuccess) return fail(QSV_EHIP, std::string("sv_apply_dense: ") + hipGetErrorString(e));
    }
    return QSV_OK;
}

qsv_status sv_debug_emulate_dense(void *amps_host, const qsv_circuit *c, uint64_t branch,
                                  int layer_begin, int layer_end, int k, int *n_blocks) {
    if (!amps_host || !c) return fail(QSV_EINVAL, "sv_debug_emulate_dense: null argument");
    if (c->n > 24) return fail(QSV_ERANGE, "sv_debug_emulate_dense: n must be <= 24");
    std::shared_ptr<DensePlan> plan;
    qsv_status st = dense_prepare(c, layer_begin, layer_end, k, branch, plan);
    if (st != QSV_OK) return st;
    if (n_blocks) *n_blocks = int(plan->blocks.size());
    for (const DenseBlock &b : plan->blocks) emulate_dense_block(b, c->n, static_cast<float *>(amps_host));
    return QSV_OK;
}

}  // extern "C"
