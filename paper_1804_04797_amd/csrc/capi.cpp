// C-ABI entry points of the qsv library (declared in include/qsv.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "jit.h"
#include "kernels.h"
#include "qsv_internal.h"

namespace {
thread_local std::string g_err;
}

namespace qsv {

qsv_status fail(qsv_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

namespace {

qsv_status hip_fail(hipError_t e, const char *where) {
    return fail(QSV_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

// gfx950 check, cached per device ordinal.
qsv_status check_gfx950() {
    static std::mutex mu;
    static int state[64] = {0};  // 0 unknown, 1 ok, 2 unsupported
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(QSV_EUNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> g(mu);
    if (state[dev] == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        state[dev] = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : 2;
    }
    if (state[dev] != 1) return fail(QSV_EUNSUPPORTED, "device is not gfx950");
    return QSV_OK;
}

namespace {

qsv_status check_device() { return check_gfx950(); }

// FP64 partial sums of the standalone reductions (sv_norm_fp64,
// sv_inner_product): one fixed buffer of 2 * 65536 doubles per device and
// stream, allocated by the first such call on that stream and never regrown,
// so calls on different streams never share one and nothing is freed while
// queued work may read it.  qsv_release_device_buffers frees them.
constexpr size_t kStreamPartials = 2 * 65536;
std::mutex g_part_mu;
std::map<std::pair<int, hipStream_t>, double *> g_part;

qsv_status stream_partials(hipStream_t s, double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_part_mu);
    double *&buf = g_part[{dev, s}];
    if (!buf) {
        e = hipMalloc(reinterpret_cast<void **>(&buf), kStreamPartials * sizeof(double));
        if (e != hipSuccess) {
            buf = nullptr;
            (void)hipGetLastError();
            return fail(QSV_ENOMEM, "partial sums: hipMalloc failed");
        }
    }
    *out = buf;
    return QSV_OK;
}

qsv_status check_state(const void *amps, int n) {
    if (!amps) return fail(QSV_EINVAL, "null state pointer");
    if (n < 0 || n > kMaxQubits) return fail(QSV_ERANGE, "n_qubits must be in 0..34");
    if (reinterpret_cast<uintptr_t>(amps) % 16 != 0)
        return fail(QSV_EINVAL, "state pointer must be 16-byte aligned");
    return QSV_OK;
}

// Range check of m device bitstrings against 2^n, before a call enqueues
// anything: a small kernel raises a flag in mapped host memory (one word per
// thread and device, allocated on first use and kept), and the host waits
// for the stream, so the call returns QSV_ERANGE with nothing enqueued.  On
// a stream under graph capture the wait is impossible: the check is skipped
// and the gather writes NaN for such entries.
qsv_status check_bitstrings(const uint64_t *xs, size_t m, int n, hipStream_t s, const char *who) {
    if (m == 0 || n >= 64) return QSV_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return hip_fail(e, who);
    if (cs != hipStreamCaptureStatusNone) return QSV_OK;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, who);
    thread_local std::map<int, std::pair<unsigned int *, unsigned int *>> flags;  // host, device address
    auto &f = flags[dev];
    if (!f.first) {
        unsigned int *h = nullptr, *d = nullptr;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(unsigned int),
                               hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess)
            return fail(QSV_ENOMEM, std::string(who) + ": range-check flag");
        if ((e = hipHostGetDevicePointer(reinterpret_cast<void **>(&d), h, 0)) != hipSuccess) {
            (void)hipHostFree(h);
            return hip_fail(e, who);
        }
        f = {h, d};
    }
    __atomic_store_n(f.first, 0u, __ATOMIC_SEQ_CST);
    if ((e = launch_check_range(xs, m, n, f.second, s)) != hipSuccess) return hip_fail(e, who);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, who);
    if (__atomic_load_n(f.first, __ATOMIC_SEQ_CST))
        return fail(QSV_ERANGE, std::string(who) + ": bitstring >= 2^n");
    return QSV_OK;
}

// Caller-owned workspace of a sweep call (sv_workspace_bytes): when the
// plan runs out of place, the second state buffer (8 * 2^n bytes) at offset
// 0 and the FP64 partial sums of the norm or inner-product epilogue after
// it; otherwise the partial sums at offset 0.
struct Workspace {
    char *p = nullptr;
    size_t bytes = 0;
};

size_t state_bytes(int n) { return sizeof(float) * 2 * (size_t(1) << n); }

// Partial-sum region: two doubles per tile of the smallest tile the tuner
// considers (2^11 amplitudes), at least 2 * 65536 for the generic kernels'
// reductions, so that a workspace sized before tuning still fits.
size_t partial_bytes(int n, int L) {
    const int l = std::min(L > 0 ? L : 11, 11);
    const size_t tiles = n > l ? size_t(1) << (n - l) : 1;
    return 2 * sizeof(double) * std::max<size_t>(tiles, 65536);
}

// opts as given, else the autotuned options of this circuit and layer range
// (sv_tune), else NULL (defaults)
const qsv_fuse_opts *effective_opts(const qsv_circuit *c, const qsv_fuse_opts *opts, int lb, int le,
                                    qsv_fuse_opts *store) {
    if (opts) return opts;
    if (tuned_opts(c, lb, le, store)) return store;
    return nullptr;
}

qsv_status resolve_shape(const qsv_circuit *c, const qsv_fuse_opts *opts, TileShape &sh,
                         int lb = 0, int le = -1) {
    (void)lb; (void)le;
    sh = default_shape(c->n);
    if (opts) {
        if (opts->reg_qubits) sh.R = opts->reg_qubits;
        if (opts->thread_qubits) sh.T = opts->thread_qubits;
        if (opts->low_qubits) sh.c = opts->low_qubits;
        else if (opts->reg_qubits || opts->thread_qubits) sh.c = std::min(5, sh.T + 1);
    }
    if (sh.R == 0) return QSV_OK;  // too small for a tile: plain path
    if (!compiled_shape_supported(sh.R, sh.T))
        return fail(QSV_EUNSUPPORTED, "no fused kernel compiled for this (reg, thread) shape");
    if (sh.R + sh.T > c->n) return fail(QSV_EUNSUPPORTED, "tile larger than the state");
    if (sh.c < 1 || sh.c - 1 > sh.T || sh.c > sh.R + sh.T)
        return fail(QSV_EINVAL, "low_qubits out of range for the tile shape");
    return QSV_OK;
}

// Out-of-place sweeps (compiled pass kernels only): opts->out_of_place
// 1 = required, -1 = never, 0 = for states of 2^24 amplitudes or more.
int oop_mode(const qsv_circuit *c, const qsv_fuse_opts *opts, int jm) {
    const int o = opts ? opts->out_of_place : 0;
    if (!jm || o < 0) return 0;
    if (o > 0) return 2;
    return c->n >= 24 ? 1 : 0;
}

qsv_status get_plan(const qsv_circuit *cc, int lb, int le, TileShape sh,
                    std::shared_ptr<Plan> &out);

// Plan and second buffer of a fused call.  `reads_state`: the first pass
// loads the caller's state (sv_apply_fused); an out-of-place plan then needs
// an even number of passes to end in the caller's buffer, else the in-place
// plan is used.  An automatic out-of-place choice falls back to in place when
// the second buffer does not fit.
qsv_status select_plan(const qsv_circuit *c, int lb, int le, TileShape sh, int oop, bool reads_state,
                       std::shared_ptr<Plan> &plan) {
    qsv_status st;
    if (oop) {
        sh.oop = true;
        if ((st = get_plan(c, lb, le, sh, plan)) != QSV_OK) return st;
        if (!(reads_state && plan->passes.size() % 2)) return QSV_OK;
    }
    sh.oop = false;
    return get_plan(c, lb, le, sh, plan);
}

// Plan, second buffer and partial sums of a fused call.  part_need: bytes
// of FP64 partial sums the call writes (0 = none).  An out-of-place plan
// runs only when the workspace holds the second buffer and the partials;
// otherwise a forced one (oop > 1) fails and an automatic one runs in place.
qsv_status get_fused_plan(const qsv_circuit *c, int lb, int le, TileShape sh, int oop,
                          bool reads_state, const Workspace &ws, size_t part_need,
                          std::shared_ptr<Plan> &plan, void **scratch, double **part) {
    *scratch = nullptr;
    if (part) *part = nullptr;
    qsv_status st = select_plan(c, lb, le, sh, oop, reads_state, plan);
    if (st != QSV_OK) return st;
    if (plan->oop) {
        const size_t sb = state_bytes(c->n);
        if (ws.p && ws.bytes >= sb + part_need) {
            *scratch = ws.p;
            if (part && part_need) *part = reinterpret_cast<double *>(ws.p + sb);
            return QSV_OK;
        }
        if (oop > 1)
            return fail(QSV_EINVAL, "out-of-place sweep: the workspace is smaller than sv_workspace_bytes");
        sh.oop = false;
        if ((st = get_plan(c, lb, le, sh, plan)) != QSV_OK) return st;
    }
    if (part_need) {
        if (!ws.p || ws.bytes < part_need)
            return fail(QSV_EINVAL, "the FP64 reduction needs a workspace of sv_workspace_bytes bytes");
        if (part) *part = reinterpret_cast<double *>(ws.p);
    }
    return QSV_OK;
}

qsv_status get_plan(const qsv_circuit *cc, int lb, int le, TileShape sh,
                    std::shared_ptr<Plan> &out) {
    qsv_circuit *c = const_cast<qsv_circuit *>(cc);
    PlanKey key{lb, le, sh.R, sh.T, sh.c, sh.oop};
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        out = it->second;
        return QSV_OK;
    }
    auto p = std::make_shared<Plan>();
    qsv_status st = build_plan(*c, lb, le, sh, *p);
    if (st != QSV_OK) return st;
    c->plans[key] = p;
    out = p;
    return QSV_OK;
}

// 0 = generic pass kernel; otherwise the kJit* flags the compiled kernels add
int jit_mode(const qsv_circuit *c, const qsv_fuse_opts *opts) {
    int j = opts ? opts->jit : 0;
    if (j == 0) {
        const char *env = std::getenv("QSV_JIT");
        if (env && env[0] == '0') return 0;
        if (c->n < 24) return 0;
        j = 1;
    }
    if (j < 0) return 0;
    if (j == 3) return 1 | kJitPerPass | int((opts->pass_forms & ((1u << kJitPassBits) - 1u)) << 8);
    if (j == 4) return 1 | kJitWhole;
    return j >= 2 ? (1 | kJitLoop) : 1;
}

void gate_matrix_f32(uint8_t kind, float m[8]) {
    const double s = std::sqrt(0.5);
    double r[8] = {0};
    switch (kind) {
    case QSV_H: { double t[8] = {s, 0, s, 0, s, 0, -s, 0}; std::memcpy(r, t, sizeof r); } break;
    case QSV_SX: { double t[8] = {.5, .5, .5, -.5, .5, -.5, .5, .5}; std::memcpy(r, t, sizeof r); } break;
    case QSV_SY: { double t[8] = {.5, .5, -.5, -.5, .5, .5, .5, .5}; std::memcpy(r, t, sizeof r); } break;
    case QSV_SXDG: { double t[8] = {.5, -.5, .5, .5, .5, .5, .5, -.5}; std::memcpy(r, t, sizeof r); } break;
    case QSV_SYDG: { double t[8] = {.5, -.5, .5, -.5, -.5, .5, .5, -.5}; std::memcpy(r, t, sizeof r); } break;
    default: break;
    }
    for (int i = 0; i < 8; ++i) m[i] = float(r[i]);
}

}  // namespace

// Per-pass times of the sweep as sv_simulate runs it from |+>^n (the
// autotuner's choice of kernel form per pass).
qsv_status time_sweep_passes(const qsv_circuit *c, int lb, int le, const qsv_fuse_opts *opts,
                             void *amps, void *workspace, size_t ws_bytes, hipStream_t s,
                             uint64_t max_tiles, std::vector<float> &ms) {
    TileShape sh;
    qsv_status st = resolve_shape(c, opts, sh, lb, le);
    if (st != QSV_OK) return st;
    const int jm = jit_mode(c, opts);
    if (sh.R == 0 || !jm) return fail(QSV_EUNSUPPORTED, "pass timing needs compiled pass kernels");
    std::shared_ptr<Plan> plan;
    void *scratch = nullptr;
    const Workspace ws{static_cast<char *>(workspace), ws_bytes};
    if ((st = get_fused_plan(c, lb, le, sh, oop_mode(c, opts, jm), false, ws, 0, plan, &scratch, nullptr)) !=
        QSV_OK)
        return st;
    if (plan->passes.empty()) return fail(QSV_EUNSUPPORTED, "empty layer range");
    const int variant = kJitInit | QSV_INIT_PLUS | (jm & ~3);
    {
        std::lock_guard<std::mutex> g(plan->jit_mu);
        if ((st = jit_prepare(*plan, variant)) != QSV_OK) return st;
    }
    return jit_launch(*plan, variant, amps, scratch, 0, 0, nullptr, s, &ms, nullptr, nullptr, nullptr, 0,
                      nullptr, 1, 0, max_tiles);
}

}  // namespace qsv

using namespace qsv;

extern "C" {

const char *qsv_last_error(void) { return g_err.c_str(); }
qsv_status qsv_release_device_buffers(void) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(QSV_EUNSUPPORTED, "device ordinal out of range");
    e = hipDeviceSynchronize();  // queued sweeps may still use them
    if (e != hipSuccess) return hip_fail(e, "qsv_release_device_buffers");
    {
        std::lock_guard<std::mutex> g(g_part_mu);
        for (auto it = g_part.begin(); it != g_part.end();) {
            if (it->first.first == dev) {
                if (it->second) hipFree(it->second);
                it = g_part.erase(it);
            } else {
                ++it;
            }
        }
    }
    return QSV_OK;
}

const char *qsv_version(void) { return "qsv 0.9 gfx950"; }

qsv_status circuit_create(int rows, int cols, const uint8_t *present, int depth, uint64_t seed,
                          const qsv_gate *gates, size_t n_gates, qsv_circuit **out) {
    if (!out) return fail(QSV_EINVAL, "circuit_create: out is null");
    *out = nullptr;
    auto c = std::unique_ptr<qsv_circuit>(new (std::nothrow) qsv_circuit);
    if (!c) return fail(QSV_ENOMEM, "circuit_create: out of host memory");
    if (!gates) {
        qsv_status st = generate_lattice_circuit(rows, cols, present, depth, seed, c.get());
        if (st != QSV_OK) return st;
    } else {
        if (rows <= 0 || cols <= 0 || rows * cols > 64)
            return fail(QSV_EINVAL, "lattice must have 1..64 sites");
        int n = 0;
        for (int i = 0; i < rows * cols; ++i) n += (!present || present[i]) ? 1 : 0;
        if (n == 0) return fail(QSV_EINVAL, "lattice has no present site");
        int maxl = 0;
        for (size_t i = 0; i < n_gates; ++i) {
            const qsv_gate &g = gates[i];
            if (g.kind > QSV_ZB) return fail(QSV_EINVAL, "unknown gate kind");
            if (g.q0 >= n || (g.kind == QSV_CZ && (g.q1 >= n || g.q1 == g.q0)))
                return fail(QSV_ERANGE, "gate qubit out of range");
            if ((g.kind == QSV_PB || g.kind == QSV_ZB) && g.arg >= 64)
                return fail(QSV_ERANGE, "branch bit out of range");
            maxl = std::max(maxl, int(g.layer));
        }
        c->n = n;
        c->depth = maxl;
        c->gates.assign(gates, gates + n_gates);
    }
    *out = c.release();
    return QSV_OK;
}

void circuit_destroy(qsv_circuit *c) { delete c; }

qsv_status circuit_info(const qsv_circuit *c, int *n_qubits, int *depth, size_t *n_gates) {
    if (!c) return fail(QSV_EINVAL, "circuit_info: null circuit");
    if (n_qubits) *n_qubits = c->n;
    if (depth) *depth = c->depth;
    if (n_gates) *n_gates = c->gates.size();
    return QSV_OK;
}

qsv_status circuit_gates(const qsv_circuit *c, qsv_gate *out, size_t cap, size_t *n_written) {
    if (!c || (!out && cap) || !n_written) return fail(QSV_EINVAL, "circuit_gates: null argument");
    size_t k = std::min(cap, c->gates.size());
    if (k) std::memcpy(out, c->gates.data(), k * sizeof(qsv_gate));
    *n_written = k;
    return QSV_OK;
}

qsv_status sv_init(void *amps, int n_qubits, int kind, uint64_t basis, void *stream) {
    qsv_status st = check_state(amps, n_qubits);
    if (st != QSV_OK) return st;
    if (kind < 0 || kind > 2) return fail(QSV_EINVAL, "sv_init: unknown kind");
    if (kind == QSV_INIT_BASIS && n_qubits < 64 && basis >= (1ull << n_qubits))
        return fail(QSV_ERANGE, "sv_init: basis index >= 2^n");
    if ((st = check_device()) != QSV_OK) return st;
    hipError_t e = launch_init(static_cast<float2 *>(amps), n_qubits, kind, basis,
                               static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_init");
}

qsv_status sv_apply_plain(void *amps, const qsv_circuit *c, uint64_t branch, int layer_begin,
                          int layer_end, void *stream) {
    if (!c) return fail(QSV_EINVAL, "sv_apply_plain: null circuit");
    qsv_status st = check_state(amps, c->n);
    if (st != QSV_OK) return st;
    if (c->n < 2) return fail(QSV_EUNSUPPORTED, "sv_apply_plain: needs n >= 2");
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_apply_plain: layer_begin < 0");
    if ((st = check_device()) != QSV_OK) return st;
    std::vector<int> idx;
    gates_in_range(*c, layer_begin, layer_end, idx);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float2 *a = static_cast<float2 *>(amps);
    const float h = float(std::sqrt(0.5));
    for (int i : idx) {
        const qsv_gate &g = c->gates[i];
        hipError_t e = hipSuccess;
        switch (g.kind) {
        case QSV_H: case QSV_SX: case QSV_SY: case QSV_SXDG: case QSV_SYDG: {
            float m[8];
            gate_matrix_f32(g.kind, m);
            e = launch_plain_1q(a, c->n, g.q0, m, s);
            break;
        }
        case QSV_T: e = launch_plain_phase(a, c->n, g.q0, h, h, s); break;
        case QSV_TDG: e = launch_plain_phase(a, c->n, g.q0, h, -h, s); break;
        case QSV_Z: e = launch_plain_phase(a, c->n, g.q0, -1.f, 0.f, s); break;
        case QSV_CZ: e = launch_plain_cz(a, c->n, g.q0, g.q1, s); break;
        case QSV_P0: e = launch_plain_zero(a, c->n, g.q0, 0, s); break;
        case QSV_P1: e = launch_plain_zero(a, c->n, g.q0, 1, s); break;
        case QSV_PB: e = launch_plain_zero(a, c->n, g.q0, int((branch >> g.arg) & 1), s); break;
        case QSV_ZB:
            if ((branch >> g.arg) & 1) e = launch_plain_phase(a, c->n, g.q0, -1.f, 0.f, s);
            break;
        default: return fail(QSV_EINTERNAL, "unknown gate kind");
        }
        if (e != hipSuccess) return hip_fail(e, "sv_apply_plain");
    }
    return QSV_OK;
}

qsv_status sv_apply_fused(void *amps, const qsv_circuit *c, uint64_t branch, int layer_begin,
                          int layer_end, const qsv_fuse_opts *opts, void *workspace, size_t ws_bytes,
                          void *stream) {
    if (!c) return fail(QSV_EINVAL, "sv_apply_fused: null circuit");
    qsv_status st = check_state(amps, c->n);
    if (st != QSV_OK) return st;
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_apply_fused: layer_begin < 0");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    if (opts && opts->plain) return sv_apply_plain(amps, c, branch, layer_begin, layer_end, stream);
    TileShape sh;
    if ((st = resolve_shape(c, opts, sh, layer_begin, layer_end)) != QSV_OK) return st;
    if (sh.R == 0) return sv_apply_plain(amps, c, branch, layer_begin, layer_end, stream);
    if ((st = check_device()) != QSV_OK) return st;
    std::shared_ptr<Plan> plan;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (const int jm = jit_mode(c, opts)) {
        void *scratch = nullptr;
        const Workspace ws{static_cast<char *>(workspace), ws_bytes};
        if ((st = get_fused_plan(c, layer_begin, layer_end, sh, oop_mode(c, opts, jm), true, ws, 0, plan,
                                 &scratch, nullptr)) != QSV_OK)
            return st;
        if (plan->passes.empty()) return QSV_OK;  // no gates in the range
        const int variant = kJitPlain | (jm & ~3);
        {
            std::lock_guard<std::mutex> g(plan->jit_mu);
            if ((st = jit_prepare(*plan, variant)) != QSV_OK) return st;
        }
        return jit_launch(*plan, variant, amps, scratch, branch, 0, nullptr, s);
    }
    if (!fused_shape_supported(sh.R, sh.T))
        return fail(QSV_EUNSUPPORTED, "sv_apply_fused: this tile shape runs compiled passes only (jit >= 1)");
    if ((st = get_plan(c, layer_begin, layer_end, sh, plan)) != QSV_OK) return st;
    for (const Pass &p : plan->passes) {
        hipError_t e = launch_fused(static_cast<float2 *>(amps), c->n, sh.R, sh.T, p.prog, branch, s);
        if (e != hipSuccess) return hip_fail(e, "sv_apply_fused");
    }
    return QSV_OK;
}

qsv_status sv_apply_fused_from(const void *src, void *dst, const qsv_circuit *c, uint64_t branch,
                               int layer_begin, int layer_end, const qsv_fuse_opts *opts, void *workspace,
                               size_t ws_bytes, void *stream) {
    if (!c) return fail(QSV_EINVAL, "sv_apply_fused_from: null circuit");
    qsv_status st = check_state(src, c->n);
    if (st != QSV_OK) return st;
    if ((st = check_state(dst, c->n)) != QSV_OK) return st;
    if (src == dst)
        return sv_apply_fused(dst, c, branch, layer_begin, layer_end, opts, workspace, ws_bytes, stream);
    const size_t bytes = sizeof(float) * 2 * (size_t(1) << c->n);
    const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(dst);
    if (a < b + bytes && b < a + bytes) return fail(QSV_EINVAL, "sv_apply_fused_from: src and dst overlap");
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_apply_fused_from: layer_begin < 0");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    if ((st = check_device()) != QSV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileShape sh;
    bool fused = !(opts && opts->plain);
    if (fused) {
        if ((st = resolve_shape(c, opts, sh, layer_begin, layer_end)) != QSV_OK) return st;
        fused = sh.R != 0;
    }
    const int jm = fused ? jit_mode(c, opts) : 0;
    if (jm) {
        // the first pass reads src and writes dst or the second buffer, so
        // any pass count ends in dst and src is never written
        std::shared_ptr<Plan> plan;
        void *scratch = nullptr;
        const Workspace ws{static_cast<char *>(workspace), ws_bytes};
        if ((st = get_fused_plan(c, layer_begin, layer_end, sh, oop_mode(c, opts, jm), false, ws, 0, plan,
                                 &scratch, nullptr)) != QSV_OK)
            return st;
        if (plan->passes.empty()) {  // no gates in the range: dst = src
            hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
            return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_apply_fused_from: copy");
        }
        const int variant = kJitPlain | (jm & ~3);
        {
            std::lock_guard<std::mutex> g(plan->jit_mu);
            if ((st = jit_prepare(*plan, variant)) != QSV_OK) return st;
        }
        return jit_launch(*plan, variant, dst, scratch, branch, 0, nullptr, s, nullptr, src);
    }
    // generic kernel or per-gate path: copy, then sweep dst in place
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "sv_apply_fused_from: copy");
    return sv_apply_fused(dst, c, branch, layer_begin, layer_end, opts, workspace, ws_bytes, stream);
}

}  // extern "C"

struct qsv_sampler {
    const qsv_circuit *c = nullptr;
    int lb = 0, le = -1;
    bool has_opts = false;
    qsv_fuse_opts opts{};
    uint64_t m = 0, ntiles = 0;
    bool compiled = false;     // sampling pass kernels; else sweep + gather
    bool tiles = false;        // the listed tiles are stored whole into a state
    std::vector<uint64_t> h_tiles;  // tile indices of the last pass, host copy
    TileShape sh{};
    int jm = 0;
    std::shared_ptr<Plan> plan;
    void *d_mem = nullptr;     // SampleTab + its arrays
    uint64_t *d_xs = nullptr;  // bitstrings for the gather form
    ~qsv_sampler() {
        if (d_mem) hipFree(d_mem);
        if (d_xs) hipFree(d_xs);
    }
};

extern "C" {

static qsv_status sampler_create(const qsv_circuit *c, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                                 const uint64_t *bitstrings, size_t m, bool tiles, qsv_sampler **out) {
    if (!c || !out || (m && !bitstrings)) return fail(QSV_EINVAL, "sv_sampler_create: null argument");
    if (m == 0 || m > (size_t(1) << 32)) return fail(QSV_ERANGE, "sv_sampler_create: m out of range");
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_sampler_create: layer_begin < 0");
    for (size_t k = 0; k < m; ++k)
        if (bitstrings[k] >> c->n) return fail(QSV_ERANGE, "sv_sampler_create: bitstring >= 2^n");
    qsv_status st = check_device();
    if (st != QSV_OK) return st;
    auto S = std::unique_ptr<qsv_sampler>(new qsv_sampler);
    S->c = c; S->lb = layer_begin; S->le = layer_end; S->m = m;
    if (opts) { S->opts = *opts; S->has_opts = true; }
    qsv_fuse_opts tuned;
    const qsv_fuse_opts *eo = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    bool fused = !(eo && eo->plain);
    if (fused) {
        if ((st = resolve_shape(c, eo, S->sh, layer_begin, layer_end)) != QSV_OK) return st;
        fused = S->sh.R != 0;
    }
    S->jm = fused ? jit_mode(c, eo) : 0;
    hipError_t e;
    if (S->jm) {
        // the plan the runs use when their workspace holds a second state
        // buffer; runs without one plan in place and need their own sampler
        if ((st = select_plan(c, layer_begin, layer_end, S->sh, oop_mode(c, eo, S->jm), false, S->plan)) != QSV_OK)
            return st;
        S->compiled = !S->plan->passes.empty();
    }
    if (tiles && !S->compiled)
        return fail(QSV_EUNSUPPORTED, "sv_sampler_create_tiles: needs compiled pass kernels (opts jit >= 1)");
    S->tiles = tiles;
    if (S->compiled) {
        // entries sorted by the tile of the last pass that holds them
        const PassProg &L = S->plan->passes.back().prog;
        std::vector<std::pair<uint64_t, uint32_t>> ent(m);
        for (size_t k = 0; k < m; ++k) {
            uint64_t tile = 0;
            for (int i = 0; i < L.n_glob; ++i) tile |= ((bitstrings[k] >> L.glob_st[i]) & 1ull) << i;
            ent[k] = {tile, uint32_t(k)};
        }
        std::sort(ent.begin(), ent.end());
        std::vector<uint64_t> tiles, xs(m);
        std::vector<uint32_t> start, slot(m);
        for (size_t k = 0; k < m; ++k) {
            if (tiles.empty() || tiles.back() != ent[k].first) {
                tiles.push_back(ent[k].first);
                start.push_back(uint32_t(k));
            }
            xs[k] = bitstrings[ent[k].second];
            slot[k] = ent[k].second;
        }
        start.push_back(uint32_t(m));
        S->ntiles = tiles.size();
        S->h_tiles = tiles;
        const size_t off_t = 64, off_s = off_t + 8 * tiles.size(), off_x = (off_s + 4 * start.size() + 7) / 8 * 8,
                     off_l = off_x + 8 * m, bytes = off_l + 4 * m;
        if ((e = hipMalloc(&S->d_mem, bytes)) != hipSuccess) return hip_fail(e, "sv_sampler_create");
        char *d = static_cast<char *>(S->d_mem);
        SampleTab head{reinterpret_cast<const uint64_t *>(d + off_t), reinterpret_cast<const uint32_t *>(d + off_s),
                       reinterpret_cast<const uint64_t *>(d + off_x), reinterpret_cast<const uint32_t *>(d + off_l)};
        std::vector<char> h(bytes, 0);
        std::memcpy(h.data(), &head, sizeof(head));
        std::memcpy(h.data() + off_t, tiles.data(), 8 * tiles.size());
        std::memcpy(h.data() + off_s, start.data(), 4 * start.size());
        std::memcpy(h.data() + off_x, xs.data(), 8 * m);
        std::memcpy(h.data() + off_l, slot.data(), 4 * m);
        if ((e = hipMemcpy(S->d_mem, h.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "sv_sampler_create");
        std::lock_guard<std::mutex> g(S->plan->jit_mu);
        if ((st = jit_prepare(*S->plan, kJitPlain | kJitSample | (S->tiles ? kJitTiles : 0) | (S->jm & ~3))) != QSV_OK)
            return st;
    } else {
        if ((e = hipMalloc(&S->d_xs, 8 * m)) != hipSuccess) return hip_fail(e, "sv_sampler_create");
        if ((e = hipMemcpy(S->d_xs, bitstrings, 8 * m, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "sv_sampler_create");
    }
    *out = S.release();
    return QSV_OK;
}

qsv_status sv_sampler_create(const qsv_circuit *c, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                             const uint64_t *bitstrings, size_t m, qsv_sampler **out) {
    return sampler_create(c, layer_begin, layer_end, opts, bitstrings, m, false, out);
}

qsv_status sv_sampler_create_tiles(const qsv_circuit *c, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                                   const uint64_t *indices, size_t m, qsv_sampler **out) {
    return sampler_create(c, layer_begin, layer_end, opts, indices, m, true, out);
}

qsv_status sv_sampler_inputs(const qsv_sampler *S, uint64_t *out, size_t cap, size_t *count) {
    if (!S || !count || (cap && !out)) return fail(QSV_EINVAL, "sv_sampler_inputs: null argument");
    if (!S->compiled || S->plan->passes.size() != 1)
        return fail(QSV_EUNSUPPORTED, "sv_sampler_inputs: the sweep has more than one pass (it reads the whole state)");
    const PassProg &P = S->plan->passes[0].prog;
    const int L = S->plan->R + S->plan->T;
    const size_t per = size_t(1) << L;
    *count = S->h_tiles.size() * per;
    size_t k = 0;
    for (uint64_t tile : S->h_tiles) {
        uint64_t base = 0;
        for (int i = 0; i < P.n_glob; ++i) base |= ((tile >> i) & 1ull) << P.glob_bits[i];
        for (size_t l = 0; l < per && k < cap; ++l, ++k) {
            uint64_t x = base;
            for (int sl = 0; sl < L; ++sl)
                if ((l >> sl) & 1) x |= 1ull << P.ld_phys[sl];
            out[k] = x;
        }
    }
    return QSV_OK;
}

// The second state buffer of a sampler run: the sampler's plan is fixed at
// creation, so an out-of-place plan needs it in every run's workspace.
static qsv_status sampler_scratch(const qsv_sampler *S, void *workspace, size_t ws_bytes, void **scratch) {
    *scratch = nullptr;
    if (!S->plan || !S->plan->oop) return QSV_OK;
    if (!workspace || ws_bytes < state_bytes(S->c->n))
        return fail(QSV_EINVAL, "sampler run: the out-of-place plan needs a workspace of sv_workspace_bytes bytes");
    *scratch = workspace;
    return QSV_OK;
}

qsv_status sv_sampler_run(qsv_sampler *S, const void *src, void *work, uint64_t branch, void *out_dev,
                          void *workspace, size_t ws_bytes, void *stream) {
    if (!S || !out_dev) return fail(QSV_EINVAL, "sv_sampler_run: null argument");
    const qsv_circuit *c = S->c;
    qsv_status st = check_state(src, c->n);
    if (st != QSV_OK) return st;
    if ((st = check_state(work, c->n)) != QSV_OK) return st;
    if (src == work) return fail(QSV_EINVAL, "sv_sampler_run: work must not be src");
    if ((st = check_device()) != QSV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const qsv_fuse_opts *opts = S->has_opts ? &S->opts : nullptr;
    if (!S->compiled) {
        if ((st = sv_apply_fused_from(src, work, c, branch, S->lb, S->le, opts, workspace, ws_bytes, stream)) !=
            QSV_OK)
            return st;
        hipError_t e = launch_gather(static_cast<const float2 *>(work), c->n, S->d_xs, S->m, out_dev, 0, s);
        return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_sampler_run");
    }
    const std::shared_ptr<Plan> &plan = S->plan;
    void *scratch = nullptr;
    if ((st = sampler_scratch(S, workspace, ws_bytes, &scratch)) != QSV_OK) return st;
    if (S->tiles && (out_dev == src || (plan->passes.size() > 1 && out_dev == work)))
        return fail(QSV_EINVAL, "sv_sampler_run: the tile state must be neither src nor work");
    const int variant = kJitPlain | kJitSample | (S->tiles ? kJitTiles : 0) | (S->jm & ~3);
    return jit_launch(*plan, variant, work, scratch, branch, 0, nullptr, s, nullptr, src, nullptr,
                      static_cast<const SampleTab *>(S->d_mem), S->ntiles, out_dev);
}

qsv_status sv_sampler_run_subtree(qsv_sampler *S, const void *src, void *work, uint64_t prefix, uint64_t mask,
                                  void *out_dev, void *workspace, size_t ws_bytes, void *stream) {
    if (!S || !out_dev) return fail(QSV_EINVAL, "sv_sampler_run_subtree: null argument");
    if (S->tiles) return fail(QSV_EINVAL, "sv_sampler_run_subtree: a tile sampler writes one state per run");
    if (prefix & mask) return fail(QSV_EINVAL, "sv_sampler_run_subtree: prefix and mask share bits");
    const int k = __builtin_popcountll(mask);
    if (k > 15) return fail(QSV_ERANGE, "sv_sampler_run_subtree: more than 15 branch bits");
    const qsv_circuit *c = S->c;
    qsv_status st = check_state(src, c->n);
    if (st != QSV_OK) return st;
    if ((st = check_state(work, c->n)) != QSV_OK) return st;
    if (src == work) return fail(QSV_EINVAL, "sv_sampler_run_subtree: work must not be src");
    if ((st = check_device()) != QSV_OK) return st;
    const size_t rows = size_t(1) << k;
    const std::shared_ptr<Plan> &plan = S->plan;
    void *scratch = nullptr;
    if (S->compiled && (st = sampler_scratch(S, workspace, ws_bytes, &scratch)) != QSV_OK) return st;
    if (!S->compiled || plan->passes.size() != 1) {
        // earlier passes are per branch: one run per row
        for (size_t y = 0; y < rows; ++y) {
            uint64_t br = prefix, msk = mask, yy = y;
            while (msk) {
                const uint64_t low = msk & (~msk + 1);
                if (yy & 1) br |= low;
                yy >>= 1;
                msk ^= low;
            }
            void *out = static_cast<char *>(out_dev) + y * S->m * sizeof(float2);
            if ((st = sv_sampler_run(S, src, work, br, out, workspace, ws_bytes, stream)) != QSV_OK) return st;
        }
        return QSV_OK;
    }
    const int variant = kJitPlain | kJitSample | (S->jm & ~3);
    return jit_launch(*plan, variant, work, scratch, prefix, mask, nullptr, static_cast<hipStream_t>(stream), nullptr,
                      src, nullptr, static_cast<const SampleTab *>(S->d_mem), S->ntiles, out_dev, rows, S->m);
}

qsv_status sv_sampler_run_branches(qsv_sampler *S, const void *src, void *work, const uint64_t *branches,
                                   size_t count, void *out_dev, void *workspace, size_t ws_bytes, void *stream) {
    if (!S || !out_dev || (count && !branches)) return fail(QSV_EINVAL, "sv_sampler_run_branches: null argument");
    if (S->tiles) return fail(QSV_EINVAL, "sv_sampler_run_branches: a tile sampler writes one state per run");
    // every call below validates the same arguments; the first one reports
    for (size_t i = 0; i < count; ++i) {
        void *out = static_cast<char *>(out_dev) + i * S->m * sizeof(float2);
        qsv_status st = sv_sampler_run(S, src, work, branches[i], out, workspace, ws_bytes, stream);
        if (st != QSV_OK) return st;
    }
    return QSV_OK;
}

void sv_sampler_destroy(qsv_sampler *S) { delete S; }

qsv_status sv_amplitudes(const void *amps, int n_qubits, const uint64_t *bitstrings_dev, size_t m,
                         void *out_dev, int out_c128, void *stream) {
    qsv_status st = check_state(amps, n_qubits);
    if (st != QSV_OK) return st;
    if (m && (!bitstrings_dev || !out_dev)) return fail(QSV_EINVAL, "sv_amplitudes: null buffer");
    if ((st = check_device()) != QSV_OK) return st;
    if ((st = check_bitstrings(bitstrings_dev, m, n_qubits, static_cast<hipStream_t>(stream), "sv_amplitudes")) !=
        QSV_OK)
        return st;
    hipError_t e = launch_gather(static_cast<const float2 *>(amps), n_qubits, bitstrings_dev, m,
                                 out_dev, out_c128 ? 1 : 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_amplitudes");
}

qsv_status sv_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst) return fail(QSV_EINVAL, "sv_stream_copy: null buffer");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(QSV_EINVAL, "sv_stream_copy: buffers and size must be multiples of 16 bytes");
    const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(dst);
    if (a < b + bytes && b < a + bytes) return fail(QSV_EINVAL, "sv_stream_copy: buffers overlap");
    qsv_status st = check_device();
    if (st != QSV_OK) return st;
    hipError_t e = launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_stream_copy");
}

qsv_status sv_norm_fp64(const void *amps, int n_qubits, double *out_dev, void *stream) {
    qsv_status st = check_state(amps, n_qubits);
    if (st != QSV_OK) return st;
    if (!out_dev) return fail(QSV_EINVAL, "sv_norm_fp64: null output");
    if ((st = check_device()) != QSV_OK) return st;
    double *part = nullptr;
    if ((st = stream_partials(static_cast<hipStream_t>(stream), &part)) != QSV_OK) return st;
    hipError_t e = launch_norm(static_cast<const float2 *>(amps), n_qubits, out_dev, part,
                               static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_norm_fp64");
}

qsv_status sv_inner_product(const void *a, const void *b, int n_qubits, double *out_dev, void *stream) {
    qsv_status st = check_state(a, n_qubits);
    if (st != QSV_OK) return st;
    if ((st = check_state(b, n_qubits)) != QSV_OK) return st;
    if (!out_dev) return fail(QSV_EINVAL, "sv_inner_product: null output");
    if ((st = check_device()) != QSV_OK) return st;
    double *part = nullptr;
    if ((st = stream_partials(static_cast<hipStream_t>(stream), &part)) != QSV_OK) return st;
    hipError_t e = launch_dot(static_cast<const float2 *>(a), static_cast<const float2 *>(b), n_qubits,
                              out_dev, part, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_inner_product");
}

qsv_status sv_branch_combine_full(const void *a_states, const void *b_states, size_t n_branches,
                                  int n_a, int n_b, uint64_t side_a_mask, const int32_t *folded_a,
                                  const int32_t *folded_b, size_t n_folded, void *out_state, int flags,
                                  void *stream) {
    if (flags & ~(QSV_COMBINE_OUT_C128 | QSV_COMBINE_FP32))
        return fail(QSV_EINVAL, "sv_branch_combine_full: unknown flag");
    if (!a_states || !b_states || !out_state) return fail(QSV_EINVAL, "sv_branch_combine_full: null buffer");
    if (n_folded && (!folded_a || !folded_b))
        return fail(QSV_EINVAL, "sv_branch_combine_full: null folded pairs");
    const int n = n_a + n_b;
    if (n_a < 7 || n_b < 7 || n_b > 22 || n > kMaxQubits)
        return fail(QSV_EUNSUPPORTED, "sv_branch_combine_full: needs 7 <= n_a, 7 <= n_b <= 22, n_a + n_b <= 34");
    if (n_branches == 0 || n_branches > (size_t(1) << 30))
        return fail(QSV_ERANGE, "sv_branch_combine_full: branch count out of range");
    if (n_folded > 64) return fail(QSV_ERANGE, "sv_branch_combine_full: more than 64 folded pairs");
    const uint64_t all = (1ull << n) - 1;
    if ((side_a_mask & ~all) || __builtin_popcountll(side_a_mask) != n_a)
        return fail(QSV_EINVAL, "sv_branch_combine_full: side mask does not match n_a");
    for (const void *p : {a_states, b_states, static_cast<const void *>(out_state)})
        if (reinterpret_cast<uintptr_t>(p) % 8) return fail(QSV_EINVAL, "sv_branch_combine_full: misaligned buffer");
    CombineArgs P;
    std::memset(&P, 0, sizeof(P));
    P.na = P.na_blk = n_a;
    P.nb = P.nb_blk = n_b;
    P.a_stride = 1ull << n_a;
    P.b_stride = 1ull << n_b;
    int local[64];
    {
        int ka = 0, kb = 0;
        for (int q = 0; q < n; ++q) {
            if ((side_a_mask >> q) & 1) { P.pos_a[ka] = uint8_t(q); local[q] = ka++; }
            else { P.pos_b[kb] = uint8_t(q); local[q] = kb++; }
        }
    }
    for (size_t f = 0; f < n_folded; ++f) {
        const int a = folded_a[f], b = folded_b[f];
        if (a < 0 || a >= n || b < 0 || b >= n || !((side_a_mask >> a) & 1) || ((side_a_mask >> b) & 1))
            return fail(QSV_EINVAL, "sv_branch_combine_full: folded pair is not (side A, side B)");
        P.fold_a[f] = uint8_t(local[a]);
        P.fold_b[f] = uint8_t(local[b]);
    }
    P.n_fold = int32_t(n_folded);
    qsv_status st = check_device();
    if (st != QSV_OK) return st;
    hipError_t e = launch_combine_gemm(static_cast<const float2 *>(a_states), static_cast<const float2 *>(b_states),
                                       n_branches, P, out_state, !(flags & QSV_COMBINE_FP32),
                                       (flags & QSV_COMBINE_OUT_C128) != 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_branch_combine_full");
}

qsv_status sv_partition_workspace_bytes(const qsv_partition *p, size_t *bytes) {
    if (!p || !bytes) return fail(QSV_EINVAL, "sv_partition_workspace_bytes: null argument");
    PartitionLayout L;
    partition_layout(p, L);
    const int ea = L.na + L.eb + L.kb, eb = L.nb + L.eb + L.ka;
    if (ea > 40 || eb > 40) return fail(QSV_ERANGE, "sv_partition_workspace_bytes: parts too large");
    // branch states of A and B, then the workspace of part C's sweep
    size_t c_ws = 0;
    if (L.c_gates) {
        qsv_status st = sv_workspace_bytes(partition_part(p, 2), 0, -1, nullptr, &c_ws);
        if (st != QSV_OK) return st;
    }
    *bytes = sizeof(float) * 2 * ((size_t(1) << ea) + (size_t(1) << eb)) + c_ws;
    return QSV_OK;
}

qsv_status sv_partition_simulate(qsv_partition *p, void *workspace, size_t ws_bytes, void *out_state,
                                 void *stream) {
    if (!p || !workspace || !out_state) return fail(QSV_EINVAL, "sv_partition_simulate: null argument");
    PartitionLayout L;
    partition_layout(p, L);
    qsv_status st = check_state(out_state, L.n);
    if (st != QSV_OK) return st;
    size_t need = 0;
    if ((st = sv_partition_workspace_bytes(p, &need)) != QSV_OK) return st;
    if (ws_bytes < need) return fail(QSV_EINVAL, "sv_partition_simulate: workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(QSV_EINVAL, "sv_partition_simulate: misaligned workspace");
    const int rows_blk = L.na - L.ka, cols_blk = L.nb - L.kb;
    if (rows_blk < 7 || cols_blk < 7 || cols_blk > 22)
        return fail(QSV_EUNSUPPORTED, "sv_partition_simulate: needs n_a - sel_a >= 7 and 7 <= n_b - sel_b <= 22");
    if (L.fold_a.size() > 64) return fail(QSV_ERANGE, "sv_partition_simulate: more than 64 folded pairs");
    if ((st = check_device()) != QSV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nbr_a = size_t(1) << (L.eb + L.kb), nbr_b = size_t(1) << (L.eb + L.ka);
    float2 *wa = static_cast<float2 *>(workspace);
    float2 *wb = wa + (nbr_a << L.na);
    // 1. branch states of both parts from |+> (layer 0 folded): one batch
    // (built once per workspace) for the parts of kBatchMinQubits or more,
    // one sv_simulate call per branch for a smaller part
    void **bws = nullptr;
    qsv_batch **batch = partition_batch(p, &bws);
    if (*batch && *bws != workspace) {
        sv_batch_destroy(*batch);
        *batch = nullptr;
    }
    const bool bat_a = L.na >= kBatchMinQubits, bat_b = L.nb >= kBatchMinQubits;
    std::vector<void *> ptrs;
    std::vector<const qsv_circuit *> circs;
    std::vector<uint64_t> ids;
    for (int side = 0; side < 2; ++side) {
        const bool bat = side ? bat_b : bat_a;
        const size_t nbr = side ? nbr_b : nbr_a;
        const int nq = side ? L.nb : L.na;
        float2 *w = side ? wb : wa;
        for (size_t i = 0; i < nbr; ++i) {
            if (bat) {
                ptrs.push_back(w + (i << nq));
                circs.push_back(partition_part(p, side));
                ids.push_back(i);
            } else if ((st = sv_simulate(w + (i << nq), partition_part(p, side), i, QSV_INIT_PLUS, 0, 1, -1,
                                         nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr, 0, stream)) != QSV_OK) {
                return st;
            }
        }
    }
    if (!ptrs.empty()) {
        if (!*batch) {
            if ((st = sv_batch_create(circs.data(), ids.data(), circs.size(), nullptr, batch)) != QSV_OK)
                return st;
            *bws = workspace;
        }
        if ((st = sv_batch_run(*batch, ptrs.data(), 1, nullptr, 0, nullptr, stream)) != QSV_OK) return st;
    }
    // 2. psi_in, one GEMM per value (v_a, v_b) of the selector qubits
    CombineArgs P;
    std::memset(&P, 0, sizeof(P));
    P.na = L.na;
    P.nb = L.nb;
    P.na_blk = rows_blk;
    P.nb_blk = cols_blk;
    P.a_stride = 1ull << L.na;
    P.b_stride = 1ull << L.nb;
    std::vector<int> loc(L.n, -1);
    for (int i = 0; i < L.na; ++i) { P.pos_a[i] = uint8_t(L.qa[i]); loc[L.qa[i]] = i; }
    for (int i = 0; i < L.nb; ++i) { P.pos_b[i] = uint8_t(L.qb[i]); loc[L.qb[i]] = i; }
    for (size_t f = 0; f < L.fold_a.size(); ++f) {
        P.fold_a[f] = uint8_t(loc[L.fold_a[f]]);
        P.fold_b[f] = uint8_t(loc[L.fold_b[f]]);
    }
    P.n_fold = int32_t(L.fold_a.size());
    const uint64_t ne = 1ull << L.eb;
    for (uint64_t va = 0; va < (1ull << L.ka); ++va)
        for (uint64_t vb = 0; vb < (1ull << L.kb); ++vb) {
            P.row_base = va << rows_blk;
            P.col_base = vb << cols_blk;
            // A's branch (e, u = vb), B's branch (e, w = va)
            P.a_off = ((vb << L.eb) << L.na) + P.row_base;
            P.b_off = ((va << L.eb) << L.nb) + P.col_base;
            hipError_t e = launch_combine_gemm(wa, wb, ne, P, out_state, true, false, s);
            if (e != hipSuccess) return hip_fail(e, "sv_partition_simulate: combine");
        }
    // 3. part C on the complete state (its sweep workspace follows the
    // branch states)
    if (L.c_gates == 0) return QSV_OK;
    const size_t used = sizeof(float) * 2 * ((nbr_a << L.na) + (nbr_b << L.nb));
    return sv_apply_fused(out_state, partition_part(p, 2), 0, 0, -1, nullptr, static_cast<char *>(workspace) + used,
                          ws_bytes - used, stream);
}

qsv_status sv_branch_combine(const void *a_tab, const void *b_tab, size_t n_branches, size_t m,
                             const int8_t *sign_dev, void *out_dev, void *stream) {
    if (m && (!a_tab || !b_tab || !out_dev)) return fail(QSV_EINVAL, "sv_branch_combine: null buffer");
    if (m > (size_t(1) << 36) || n_branches > (size_t(1) << 40))
        return fail(QSV_ERANGE, "sv_branch_combine: size out of range");
    qsv_status st = check_device();
    if (st != QSV_OK) return st;
    hipError_t e = launch_branch_combine(static_cast<const float2 *>(a_tab),
                                         static_cast<const float2 *>(b_tab), n_branches, m, sign_dev,
                                         static_cast<double2 *>(out_dev),
                                         static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_branch_combine");
}

qsv_status sv_simulate(void *amps, const qsv_circuit *c, uint64_t branch, int init_kind,
                       uint64_t basis, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                       double *norm_out_dev, const uint64_t *bitstrings_dev, size_t m,
                       void *amps_out_dev, int out_c128, void *workspace, size_t ws_bytes, void *stream) {
    if (!c) return fail(QSV_EINVAL, "sv_simulate: null circuit");
    qsv_status st = check_state(amps, c->n);
    if (st != QSV_OK) return st;
    if (init_kind < 0 || init_kind > 2) return fail(QSV_EINVAL, "sv_simulate: unknown init kind");
    if (init_kind == QSV_INIT_BASIS && basis >= (1ull << c->n))
        return fail(QSV_ERANGE, "sv_simulate: basis index >= 2^n");
    if (init_kind == QSV_INIT_ZERO) basis = 0;
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_simulate: layer_begin < 0");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    if (m && (!bitstrings_dev || !amps_out_dev)) return fail(QSV_EINVAL, "sv_simulate: null gather buffer");
    if ((st = check_device()) != QSV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Workspace ws{static_cast<char *>(workspace), ws_bytes};
    TileShape sh;
    bool fused = !(opts && opts->plain);
    if (fused) {
        if ((st = resolve_shape(c, opts, sh, layer_begin, layer_end)) != QSV_OK) return st;
        fused = sh.R != 0;
    }
    std::shared_ptr<Plan> plan;
    const int jm = fused ? jit_mode(c, opts) : 0;
    void *scratch = nullptr;
    double *part = nullptr;
    if (jm) {
        const uint64_t tiles = 1ull << (c->n - sh.R - sh.T);
        const size_t need = norm_out_dev ? tiles * sizeof(double) : 0;
        if ((st = get_fused_plan(c, layer_begin, layer_end, sh, oop_mode(c, opts, jm), false, ws, need, plan,
                                 &scratch, &part)) != QSV_OK)
            return st;
    } else if (fused && (st = get_plan(c, layer_begin, layer_end, sh, plan)) != QSV_OK) {
        return st;
    }
    if ((st = check_bitstrings(bitstrings_dev, m, c->n, s, "sv_simulate")) != QSV_OK) return st;
    if (jm && !plan->passes.empty()) {
        // initial state generated by the first pass, norm by the last
        const int variant = kJitInit | init_kind | (norm_out_dev ? kJitNorm : 0) | (jm & ~3);
        {
            std::lock_guard<std::mutex> g(plan->jit_mu);
            if ((st = jit_prepare(*plan, variant)) != QSV_OK) return st;
        }
        const uint64_t tiles = 1ull << (c->n - sh.R - sh.T);
        if ((st = jit_launch(*plan, variant, amps, scratch, branch, basis, part, s)) != QSV_OK) return st;
        if (norm_out_dev) {
            hipError_t e = launch_sum_partials(part, tiles, norm_out_dev, s);
            if (e != hipSuccess) return hip_fail(e, "sv_simulate");
        }
    } else {
        // generic kernel or per-gate path: init, sweep in place, then the
        // norm's own reduction with its partial sums in the workspace
        const size_t need = norm_out_dev ? norm_partial_count(c->n) * sizeof(double) : 0;
        if (need && (!ws.p || ws.bytes < need))
            return fail(QSV_EINVAL, "sv_simulate: the FP64 norm needs a workspace of sv_workspace_bytes bytes");
        hipError_t e = launch_init(static_cast<float2 *>(amps), c->n, init_kind, basis, s);
        if (e != hipSuccess) return hip_fail(e, "sv_simulate");
        st = fused ? sv_apply_fused(amps, c, branch, layer_begin, layer_end, opts, workspace, ws_bytes, stream)
                   : sv_apply_plain(amps, c, branch, layer_begin, layer_end, stream);
        if (st != QSV_OK) return st;
        if (norm_out_dev) {
            e = launch_norm(static_cast<const float2 *>(amps), c->n, norm_out_dev, reinterpret_cast<double *>(ws.p),
                            s);
            if (e != hipSuccess) return hip_fail(e, "sv_simulate: norm");
        }
    }
    if (m) {
        hipError_t e = launch_gather(static_cast<const float2 *>(amps), c->n, bitstrings_dev, m,
                                     amps_out_dev, out_c128 ? 1 : 0, s);
        if (e != hipSuccess) return hip_fail(e, "sv_simulate");
    }
    return QSV_OK;
}

qsv_status sv_simulate_dot(void *amps, const qsv_circuit *c, uint64_t branch, int init_kind,
                           uint64_t basis, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                           const void *other, double *out_dev, void *workspace, size_t ws_bytes, void *stream) {
    if (!c) return fail(QSV_EINVAL, "sv_simulate_dot: null circuit");
    qsv_status st = check_state(amps, c->n);
    if (st != QSV_OK) return st;
    if ((st = check_state(other, c->n)) != QSV_OK) return st;
    if (!out_dev) return fail(QSV_EINVAL, "sv_simulate_dot: null output");
    if (other == amps) return fail(QSV_EINVAL, "sv_simulate_dot: other must not be the work buffer");
    if (init_kind < 0 || init_kind > 2) return fail(QSV_EINVAL, "sv_simulate_dot: unknown init kind");
    if (init_kind == QSV_INIT_BASIS && basis >= (1ull << c->n))
        return fail(QSV_ERANGE, "sv_simulate_dot: basis index >= 2^n");
    if (init_kind == QSV_INIT_ZERO) basis = 0;
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_simulate_dot: layer_begin < 0");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    if ((st = check_device()) != QSV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Workspace ws{static_cast<char *>(workspace), ws_bytes};
    TileShape sh;
    bool fused = !(opts && opts->plain);
    if (fused) {
        if ((st = resolve_shape(c, opts, sh, layer_begin, layer_end)) != QSV_OK) return st;
        fused = sh.R != 0;
    }
    const int jm = fused ? jit_mode(c, opts) : 0;
    std::shared_ptr<Plan> plan;
    void *scratch = nullptr;
    double *part = nullptr;
    const uint64_t tiles = fused ? 1ull << (c->n - sh.R - sh.T) : 0;
    if (jm && (st = get_fused_plan(c, layer_begin, layer_end, sh, oop_mode(c, opts, jm), false, ws,
                                   2 * tiles * sizeof(double), plan, &scratch, &part)) != QSV_OK)
        return st;
    if (!jm || plan->passes.empty()) {
        // the sweep into amps, then the inner product (two kernels, the
        // reduction's partial sums in the workspace)
        const size_t need = 2 * 65536 * sizeof(double);
        if (!ws.p || ws.bytes < need)
            return fail(QSV_EINVAL, "sv_simulate_dot: needs a workspace of sv_workspace_bytes bytes");
        if ((st = sv_simulate(amps, c, branch, init_kind, basis, layer_begin, layer_end, opts, nullptr, nullptr,
                              0, nullptr, 0, workspace, ws_bytes, stream)) != QSV_OK)
            return st;
        hipError_t e = launch_dot(static_cast<const float2 *>(amps), static_cast<const float2 *>(other), c->n,
                                  out_dev, reinterpret_cast<double *>(ws.p), s);
        return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_simulate_dot");
    }
    // initial state from the first pass; the last pass stores nothing and
    // writes the FP64 partials of <result|other>
    const int variant = kJitInit | init_kind | kJitDot | (jm & ~3);
    {
        std::lock_guard<std::mutex> g(plan->jit_mu);
        if ((st = jit_prepare(*plan, variant)) != QSV_OK) return st;
    }
    if ((st = jit_launch(*plan, variant, amps, scratch, branch, basis, part, s, nullptr, nullptr, other)) != QSV_OK)
        return st;
    hipError_t e = launch_sum_partials(part, tiles, out_dev, s);
    if (e == hipSuccess) e = launch_sum_partials(part + tiles, tiles, out_dev + 1, s);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "sv_simulate_dot");
}

qsv_status sv_simulate_c128(void *amps, const qsv_circuit *c, uint64_t branch, int init_kind,
                            uint64_t basis, int layer_begin, int layer_end, double *norm_out_dev,
                            const uint64_t *bitstrings_dev, size_t m, void *amps_out_dev,
                            void *workspace, size_t ws_bytes, void *stream) {
    if (!c || !amps) return fail(QSV_EINVAL, "sv_simulate_c128: null argument");
    if (reinterpret_cast<uintptr_t>(amps) % 16) return fail(QSV_EINVAL, "sv_simulate_c128: misaligned state");
    if (c->n < 12 || c->n > kMaxQubits) return fail(QSV_EUNSUPPORTED, "sv_simulate_c128: needs 12 <= n <= 34");
    if (init_kind < 0 || init_kind > 2) return fail(QSV_EINVAL, "sv_simulate_c128: unknown init kind");
    if (init_kind == QSV_INIT_BASIS && basis >= (1ull << c->n))
        return fail(QSV_ERANGE, "sv_simulate_c128: basis index >= 2^n");
    if (init_kind == QSV_INIT_ZERO) basis = 0;
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_simulate_c128: layer_begin < 0");
    if (m && (!bitstrings_dev || !amps_out_dev)) return fail(QSV_EINVAL, "sv_simulate_c128: null gather buffer");
    const TileShape sh{4, 8, 4};
    const uint64_t tiles = 1ull << (c->n - sh.R - sh.T);
    if (norm_out_dev && (!workspace || ws_bytes < tiles * sizeof(double)))
        return fail(QSV_EINVAL, "sv_simulate_c128: the FP64 norm needs a workspace of sv_workspace_bytes bytes");
    qsv_status st = check_device();
    if (st != QSV_OK) return st;
    std::shared_ptr<Plan> plan;
    if ((st = get_plan(c, layer_begin, layer_end, sh, plan)) != QSV_OK) return st;
    if (plan->passes.empty()) return fail(QSV_EUNSUPPORTED, "sv_simulate_c128: empty layer range");
    const int variant = kJitDouble | kJitInit | init_kind | (norm_out_dev ? kJitNorm : 0);
    {
        std::lock_guard<std::mutex> g(plan->jit_mu);
        if ((st = jit_prepare(*plan, variant)) != QSV_OK) return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = check_bitstrings(bitstrings_dev, m, c->n, s, "sv_simulate_c128")) != QSV_OK) return st;
    double *part = norm_out_dev ? static_cast<double *>(workspace) : nullptr;
    if ((st = jit_launch(*plan, variant, amps, nullptr, branch, basis, part, s)) != QSV_OK) return st;
    if (norm_out_dev) {
        hipError_t e = launch_sum_partials(part, tiles, norm_out_dev, s);
        if (e != hipSuccess) return hip_fail(e, "sv_simulate_c128");
    }
    if (m) {
        hipError_t e = launch_gather_c128(amps, c->n, bitstrings_dev, m, amps_out_dev, s);
        if (e != hipSuccess) return hip_fail(e, "sv_simulate_c128");
    }
    return QSV_OK;
}

qsv_status sv_workspace_bytes(const qsv_circuit *c, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                              size_t *bytes) {
    if (!c || !bytes) return fail(QSV_EINVAL, "sv_workspace_bytes: null argument");
    if (layer_begin < 0) return fail(QSV_EINVAL, "sv_workspace_bytes: layer_begin < 0");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    TileShape sh{0, 0, 0};
    const bool fused = !(opts && opts->plain);
    if (fused) {
        qsv_status st = resolve_shape(c, opts, sh, layer_begin, layer_end);
        if (st != QSV_OK) return st;
    }
    const int jm = (fused && sh.R) ? jit_mode(c, opts) : 0;
    *bytes = partial_bytes(c->n, sh.R + sh.T);
    if (jm && oop_mode(c, opts, jm)) *bytes += state_bytes(c->n);
    return QSV_OK;
}

qsv_status sv_plan_info(const qsv_circuit *c, int layer_begin, int layer_end,
                        const qsv_fuse_opts *opts, int *n_passes, int32_t *pass_of_gate,
                        int32_t *order_in_pass, size_t n_gate_cap, uint64_t *resident_mask,
                        size_t pass_cap) {
    if (!c || !n_passes) return fail(QSV_EINVAL, "sv_plan_info: null argument");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    TileShape sh;
    qsv_status st = resolve_shape(c, opts, sh, layer_begin, layer_end);
    if (st != QSV_OK) return st;
    if (sh.R == 0) return fail(QSV_EUNSUPPORTED, "sv_plan_info: state too small for a tile");
    std::shared_ptr<Plan> plan;
    if ((st = select_plan(c, layer_begin, layer_end, sh, oop_mode(c, opts, jit_mode(c, opts)), false,
                          plan)) != QSV_OK)
        return st;
    *n_passes = int(plan->passes.size());
    if (pass_of_gate || order_in_pass) {
        size_t ng = std::min(n_gate_cap, c->gates.size());
        for (size_t i = 0; i < ng; ++i) {
            if (pass_of_gate) pass_of_gate[i] = -1;
            if (order_in_pass) order_in_pass[i] = -1;
        }
        for (size_t p = 0; p < plan->passes.size(); ++p) {
            const auto &gs = plan->passes[p].gates;
            for (size_t k = 0; k < gs.size(); ++k) {
                if (size_t(gs[k]) >= ng) continue;
                if (pass_of_gate) pass_of_gate[gs[k]] = int32_t(p);
                if (order_in_pass) order_in_pass[gs[k]] = int32_t(k);
            }
        }
    }
    if (resident_mask)
        for (size_t p = 0; p < std::min(pass_cap, plan->passes.size()); ++p)
            resident_mask[p] = plan->passes[p].resident_logical;
    return QSV_OK;
}

qsv_status sv_debug_emulate(void *amps_host, const qsv_circuit *c, uint64_t branch,
                            int layer_begin, int layer_end, const qsv_fuse_opts *opts) {
    if (!c || !amps_host) return fail(QSV_EINVAL, "sv_debug_emulate: null argument");
    if (c->n > 26) return fail(QSV_ERANGE, "sv_debug_emulate: n must be <= 26");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    TileShape sh;
    qsv_status st = resolve_shape(c, opts, sh);
    if (st != QSV_OK) return st;
    if (sh.R == 0) return fail(QSV_EUNSUPPORTED, "sv_debug_emulate: state too small for a tile");
    std::shared_ptr<Plan> plan;
    if ((st = select_plan(c, layer_begin, layer_end, sh, oop_mode(c, opts, jit_mode(c, opts)), true,
                          plan)) != QSV_OK)
        return st;
    // the same buffer schedule as the device sweep
    float *amps = static_cast<float *>(amps_host);
    std::vector<float> second(plan->oop ? size_t(2) << c->n : 0);
    const size_t np = plan->passes.size();
    const float *in = amps;
    for (size_t p = 0; p < np; ++p) {
        float *out = (!plan->oop || (np - p) % 2 == 1) ? amps : second.data();
        emulate_pass(plan->passes[p].prog, c->n, sh.R, sh.T, branch, in, out);
        in = out;
    }
    return QSV_OK;
}

qsv_status sv_debug_jit_compile(const qsv_circuit *c, int layer_begin, int layer_end,
                                const qsv_fuse_opts *opts, size_t *code_bytes, double *seconds) {
    if (!c) return fail(QSV_EINVAL, "sv_debug_jit_compile: null circuit");
    qsv_fuse_opts tuned;
    opts = effective_opts(c, opts, layer_begin, layer_end, &tuned);
    TileShape sh;
    qsv_status st = resolve_shape(c, opts, sh);
    if (st != QSV_OK) return st;
    if (sh.R == 0) return fail(QSV_EUNSUPPORTED, "sv_debug_jit_compile: state too small for a tile");
    std::shared_ptr<Plan> plan;
    if ((st = select_plan(c, layer_begin, layer_end, sh, oop_mode(c, opts, jit_mode(c, opts)), false,
                          plan)) != QSV_OK)
        return st;
    return jit_compile_only(*plan, code_bytes, seconds);
}

}  // extern "C"
