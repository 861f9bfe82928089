// Runtime specialisation of fused passes (hipRTC).
//
// The generic tile kernel interprets a pass program op by op.  For large
// states the program of every pass is instead turned into straight-line HIP
// source (register slots, physical bit positions, LDS permutations and gate
// constants all become literals), compiled once for gfx950 with hipRTC and
// cached by its source text for the life of the process.  The generated
// kernels perform exactly the ops of the program, in order.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "jit.h"
#include "qsv_internal.h"

namespace qsv {

namespace {

const char *kPrelude = R"(
typedef float v4f __attribute__((ext_vector_type(4)));
#define F2(x, y) make_float2((x), (y))
__device__ __forceinline__ float2 cm(float2 a, float cr, float ci) {
    return make_float2(a.x * cr - a.y * ci, a.x * ci + a.y * cr);
}
__constant__ float QW[16] = {1.f, 0.70710678118654752f, 0.f, -0.70710678118654752f,
                            -1.f, -0.70710678118654752f, 0.f, 0.70710678118654752f,
                            0.f, 0.70710678118654752f, 1.f, 0.70710678118654752f,
                            0.f, -0.70710678118654752f, -1.f, -0.70710678118654752f};
__device__ __forceinline__ float2 xsign(float2 a, unsigned m) {
    return make_float2(__uint_as_float(__float_as_uint(a.x) ^ m),
                       __uint_as_float(__float_as_uint(a.y) ^ m));
}
struct SampleTabJ {  // layout of the library's sampling table
    const unsigned long long *tiles;
    const unsigned *start;
    const unsigned long long *xs;
    const unsigned *slot;
};
struct BatchEntryJ {  // layout of the library's batch entry table
    void *amps;
    unsigned long long branch;
    unsigned prog0, n;
    float init_val;
    unsigned pad;
};
typedef double v2d __attribute__((ext_vector_type(2)));
#define D2(x, y) make_double2((x), (y))
__device__ __forceinline__ double2 cmd(double2 a, double cr, double ci) {
    return make_double2(a.x * cr - a.y * ci, a.x * ci + a.y * cr);
}
__constant__ double QWD[16] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440,
                               -1.0, -0.70710678118654752440, 0.0, 0.70710678118654752440,
                               0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440,
                               0.0, -0.70710678118654752440, -1.0, -0.70710678118654752440};
__device__ __forceinline__ double2 xsignd(double2 a, unsigned m) {
    return m ? make_double2(-a.x, -a.y) : a;
}
)";

std::string hex64(uint64_t v) {
    char b[32];
    std::snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
    return b;
}

std::string flt(double v) {
    char b[48];
    std::snprintf(b, sizeof b, "%.9ef", v);
    return b;
}

std::string dbl(double v) {
    char b[48];
    std::snprintf(b, sizeof b, "%.17e", v);
    return b;
}

// OR of ((src >> i0) & mask) << p0 over maximal runs where consecutive source
// bits map to consecutive target bits.
std::string scatter_expr(const std::string &src, const std::vector<int> &target, bool wide) {
    std::ostringstream o;
    const char *one = wide ? "1ull" : "1u";
    bool first = true;
    size_t i = 0;
    while (i < target.size()) {
        size_t j = i;
        while (j + 1 < target.size() && target[j + 1] == target[j] + 1) ++j;
        const int len = int(j - i + 1);
        if (!first) o << " | ";
        first = false;
        o << "((((unsigned long long)(" << src << ") >> " << i << ") & ((" << one << " << " << len
          << ") - 1)) << " << target[i] << ")";
        i = j + 1;
    }
    if (first) o << "0ull";
    return o.str();
}

// Code generator for one pass.
//
// Besides turning every op into literal code, the generator keeps factors
// that multiply whole registers out of the per-amplitude arithmetic:
//  - per register, at compile time, a rotation i^m and a power 2^{-h/2}:
//    even phases (Z, S, CZ between register qubits) only change m; T on a
//    register qubit multiplies by (1 + i) and adds one to h; butterflies
//    absorb both by choosing signs, components and an FMA coefficient;
//  - per register slot s, at run time, a sign sg<s> = +-1 of the registers
//    whose bit s is set: CZ between a register qubit and a thread or
//    tile-index qubit only flips sg<s>, and the next butterfly on slot s uses
//    it as its FMA coefficient;
//  - per thread, at run time, an exponent e of w = e^{i pi/4} and a zero
//    flag: diagonal gates on thread or tile-index qubits only update e.
// All of them are applied (at most one complex multiply per amplitude) before
// an LDS exchange and, together with the pass scale, before the store.
// Exchanges whose chosen layout failed its injectivity check and fell back
// to the plain weights (a generator defect; sv_debug_jit_compile reports it).
std::atomic<unsigned> g_layout_fallbacks{0};

struct Gen {
    const PassProg &P;
    int R, T, N, L;
    std::ostringstream o;
    int m[64];            // pending rotation i^m of each register
    int h[64];            // pending factor 2^{-h/2} of each register
    int w[64];            // pending factor e^{i pi/4} (1) or none (0) of each register
    bool sdirty[8];       // slot s carries the run-time sign sg<s>
    bool e_dirty = false; // e or the zero flag may differ from (0, alive)
    bool dp;              // complex128 state (validation instantiation)
    int uid = 0;          // unique temporaries
    std::string CT, RT, MK, CM, XS, QT, ZERO;
    Gen(const PassProg &p, int r, int t, bool double_precision = false)
        : P(p), R(r), T(t), N(1 << r), L(r + t), dp(double_precision) {
        for (int j = 0; j < 64; ++j) m[j] = h[j] = w[j] = 0;
        for (int s = 0; s < 8; ++s) sdirty[s] = false;
        CT = dp ? "double2" : "float2";
        RT = dp ? "double" : "float";
        MK = dp ? "D2" : "F2";
        CM = dp ? "cmd" : "cm";
        XS = dp ? "xsignd" : "xsign";
        QT = dp ? "QWD" : "QW";
        ZERO = dp ? "0.0" : "0.f";
    }
    std::string lit(double v) const { return dp ? dbl(v) : flt(v); }
    std::string tmpname(const char *p) { return std::string(p) + std::to_string(uid++); }

    bool is_reg(uint32_t loc) const { return loc < uint32_t(R); }
    bool is_glob(uint32_t loc) const { return loc & 0x80u; }
    std::string pred(uint32_t loc) const {
        std::ostringstream s;
        if (is_glob(loc)) s << "unsigned((base >> " << (loc & 0x7f) << ") & 1ull)";
        else s << "((t >> " << (loc - R) << ") & 1u)";
        return s.str();
    }
    static std::string sgn(int s) { return "sg" + std::to_string(s); }

    // component c (0 = re, 1 = im) of i^r * Z as a signed term
    static std::string term(const char *z, int r, int c) {
        r &= 3;
        static const char *comp[4][2] = {{"+%s.x", "+%s.y"}, {"-%s.y", "+%s.x"},
                                         {"-%s.x", "-%s.y"}, {"+%s.y", "-%s.x"}};
        char b[32];
        std::snprintf(b, sizeof b, comp[r][c], z);
        return b;
    }
    // i^a * X + coef * i^b * Y ; coef == "" means 1
    std::string sum(int a, int b, const std::string &coef) const {
        std::string re, im;
        if (coef.empty()) {
            re = term("x", a, 0) + term("y", b, 0);
            im = term("x", a, 1) + term("y", b, 1);
        } else {
            re = term("x", a, 0) + "+" + coef + "*(" + term("y", b, 0) + ")";
            im = term("x", a, 1) + "+" + coef + "*(" + term("y", b, 1) + ")";
        }
        return MK + "(" + re + "," + im + ")";
    }

    // sign flip of slot s by a 0/1 predicate expression
    void flip_slot(int s, const std::string &p) {
        if (sdirty[s]) {
            o << sgn(s) << " = (" << p << ") ? -" << sgn(s) << " : " << sgn(s) << ";\n";
        } else {
            if (!declared_sg[s]) o << RT << " ";
            o << sgn(s) << " = (" << p << ") ? " << lit(-1.0) << " : " << lit(1.0) << ";\n";
        }
        declared_sg[s] = true;
        sdirty[s] = true;
    }
    bool declared_sg[8] = {false, false, false, false, false, false, false, false};

    void butterfly(uint32_t code, int S) {
        // a pending e^{i pi/4} common to both inputs of a pair stays pending
        // on both outputs; on one input only it is applied first
        for (int j = 0; j < N; ++j) {
            if (j & (1 << S)) continue;
            const int k = j | (1 << S);
            if (w[j] != w[k]) omega_reg(w[j] ? j : k);
        }
        // coefficient of Y relative to X per distinct h difference
        std::map<int, std::string> coef;
        for (int j = 0; j < N; ++j) {
            if (j & (1 << S)) continue;
            const int k = j | (1 << S);
            const int dh = h[k] - h[j];
            if (coef.count(dh)) continue;
            const double mag = std::pow(2.0, -0.5 * dh);
            if (!sdirty[S]) {
                coef[dh] = (dh == 0) ? "" : lit(mag);
            } else if (dh == 0) {
                coef[dh] = sgn(S);
            } else {
                const std::string nm = tmpname("c");
                o << "const " << RT << " " << nm << " = " << sgn(S) << " * " << lit(mag) << ";\n";
                coef[dh] = nm;
            }
        }
        for (int j = 0; j < N; ++j) {
            if (j & (1 << S)) continue;
            const int k = j | (1 << S);
            const int d = (m[k] - m[j]) & 3;
            // outputs relative to the common factor i^{m[j]} 2^{-h[j]/2}
            int a0 = 0, b0 = d, a1 = 0, b1 = d;  // x' = i^a0 X + c i^b0 Y ; y' = i^a1 X + c i^b1 Y
            switch (code) {
            case OP_H: b1 = d + 2; break;                       // x+y, x-y
            case OP_SX: b0 = d + 3; a1 = 3; break;              // x-iy, -ix+y
            case OP_SY: b0 = d + 2; break;                      // x-y, x+y
            case OP_SXDG: b0 = d + 1; a1 = 1; break;            // x+iy, ix+y
            case OP_SYDG: a1 = 2; break;                        // x+y, -x+y
            }
            const std::string &cf = coef[h[k] - h[j]];
            o << "{const " << CT << " x=v[" << j << "],y=v[" << k << "];v[" << j << "]=" << sum(a0, b0, cf)
              << ";v[" << k << "]=" << sum(a1, b1, cf) << ";}\n";
            m[k] = m[j];
            h[k] = h[j];
            w[k] = w[j];
        }
        sdirty[S] = false;  // absorbed
    }
    void rot_reg(int j, int k) { m[j] = (m[j] + k / 2) & 3; }
    // apply the pending e^{i pi/4} = (1 + i)/sqrt2 of register j: the stored
    // value times (1 + i), the 1/sqrt2 joins its power of two
    void omega_reg(int j) {
        o << "v[" << j << "]=" << MK << "(v[" << j << "].x-v[" << j << "].y,v[" << j << "].x+v[" << j
          << "].y);\n";
        h[j] += 1;
        w[j] = 0;
    }
    // e^{i pi k/4}: the multiple of i/2 rotates, an odd k toggles the pending
    // e^{i pi/4} (two of them are i), so T gates cost nothing until a
    // butterfly pairs the register with one that lacks the factor
    void phase_reg(int j, int k) {
        k &= 7;
        rot_reg(j, k & 6);
        if (k & 1) {
            if (w[j]) {
                w[j] = 0;
                m[j] = (m[j] + 1) & 3;
            } else {
                w[j] = 1;
            }
        }
    }
    void zero_reg(int j) {
        o << "v[" << j << "]=" << MK << "(" << ZERO << "," << ZERO << ");\n";
        m[j] = h[j] = w[j] = 0;
    }

    void op_phase(uint32_t loc, int k) {
        if (is_reg(loc)) {
            for (int j = 0; j < N; ++j)
                if (j & (1 << loc)) phase_reg(j, k);
            return;
        }
        o << "e += " << pred(loc) << " * " << (k & 7) << "u;\n";
        e_dirty = true;
    }

    void op_cz(uint32_t a, uint32_t b) {
        if (!is_reg(a) && is_reg(b)) std::swap(a, b);
        if (is_reg(a) && is_reg(b)) {
            for (int j = 0; j < N; ++j)
                if ((j & (1 << a)) && (j & (1 << b))) rot_reg(j, 4);
            return;
        }
        if (is_reg(a)) {
            flip_slot(int(a), pred(b));
            return;
        }
        o << "e += (" << pred(a) << " & " << pred(b) << ") * 4u;\n";
        e_dirty = true;
    }

    void op_proj(uint32_t loc, uint32_t b, uint32_t c) {
        std::string l = c ? "unsigned((branch >> " + std::to_string(b) + ") & 1ull)"
                          : std::to_string(b) + "u";
        if (is_reg(loc)) {
            if (!c) {
                for (int j = 0; j < N; ++j)
                    if (((j >> loc) & 1) != int(b)) zero_reg(j);
                return;
            }
            // branch-dependent: both arms leave the surviving registers' state unchanged
            o << "if (" << l << ") {\n";
            for (int j = 0; j < N; ++j)
                if (!(j & (1 << loc))) o << "v[" << j << "]=" << MK << "(" << ZERO << "," << ZERO << ");\n";
            o << "} else {\n";
            for (int j = 0; j < N; ++j)
                if (j & (1 << loc)) o << "v[" << j << "]=" << MK << "(" << ZERO << "," << ZERO << ");\n";
            o << "}\n";
            return;
        }
        o << "alive &= unsigned((" << pred(loc) << ") == " << l << ");\n";
        e_dirty = true;
    }

    void op_zb(uint32_t loc, uint32_t b) {
        const std::string bit = "unsigned((branch >> " + std::to_string(b) + ") & 1ull)";
        if (is_reg(loc)) {
            flip_slot(int(loc), bit);
            return;
        }
        o << "e += (" << bit << " & " << pred(loc) << ") * 4u;\n";
        e_dirty = true;
    }

    // Multiply every register by its pending factors and by (sr + i si), then
    // reset them: i^{m_j} 2^{-h_j/2} (compile time), prod of sg<s> over the
    // register's set bits of dirty slots, w^e * alive (run time).
    // move_mask < 0: apply every pending factor.  Otherwise (an exchange that
    // moves the register slots in move_mask to thread slots, no pending
    // per-thread phase) apply the run-time signs and only the part of each
    // register's compile-time factor that depends on those slots: register j
    // gets K_j / K_{j with them cleared}; the remaining compile-time factors
    // depend on staying register bits only, which op_xchg then renames to
    // their new slots.  (The signs are functions of the thread that computed
    // them; an exchange hands the data to other threads, so they are applied.)
    void materialize(double sr, double si, int move_mask = -1) {
        const bool partial = move_mask >= 0;
        if (partial && e_dirty) return materialize(sr, si);
        int dmask = 0;
        for (int s = 0; s < R; ++s)
            if (sdirty[s]) dmask |= 1 << s;
        std::map<int, std::string> sig;  // sign products by slot mask
        auto sign_of = [&](int mask) -> std::string {
            if (mask == 0) return "";
            std::string prev;
            int acc = 0;
            for (int s = 0; s < R; ++s) {  // build the product bit by bit, reusing prefixes
                if (!(mask & (1 << s))) continue;
                acc |= 1 << s;
                auto it = sig.find(acc);
                if (it == sig.end()) {
                    const std::string nm = tmpname("s");
                    o << "const " << RT << " " << nm << " = " << (prev.empty() ? "" : prev + " * ") << sgn(s)
                      << ";\n";
                    it = sig.emplace(acc, nm).first;
                }
                prev = it->second;
            }
            return prev;
        };
        if (e_dirty) {
            o << "const " << RT << " wr" << uid << " = alive ? " << QT << "[e & 7u] : " << ZERO << ", wi" << uid
              << " = alive ? " << QT << "[8u + (e & 7u)] : " << ZERO << ";\n";
        }
        const int wid = uid++;
        for (int j = 0; j < N; ++j) {
            // compile-time factor K = i^m 2^{-h/2} (sr + i si), relative to
            // register j0 in the partial form
            const int j0 = partial ? (j & ~move_mask) : -1;
            const int dm = partial ? m[j] - m[j0] : m[j], dh = partial ? h[j] - h[j0] : h[j];
            const int dw = partial ? w[j] - w[j0] : w[j];
            const double mag = std::pow(2.0, -0.5 * dh);
            double kr = sr * mag, ki = si * mag;
            for (int q = 0; q < (dm & 3); ++q) { double t2 = -ki; ki = kr; kr = t2; }
            if (dw != 0) {  // times e^{+-i pi/4}
                const double c = std::sqrt(0.5), r2 = kr, i2 = ki;
                kr = c * (dw > 0 ? r2 - i2 : r2 + i2);
                ki = c * (dw > 0 ? r2 + i2 : i2 - r2);
            }
            const std::string sj = sign_of(j & dmask);
            if (!e_dirty) {
                const bool real = (ki == 0.0), imag = (kr == 0.0);
                if (sj.empty() && kr == 1.0 && ki == 0.0) continue;
                if (real || imag) {
                    // K = k * i^r with real k: components swap/negate, one scale each
                    const int r = real ? (kr > 0 ? 0 : 2) : (ki > 0 ? 1 : 3);
                    const double k = real ? std::fabs(kr) : std::fabs(ki);
                    std::string f;
                    if (sj.empty()) f = (k == 1.0) ? "" : lit(k);
                    else f = (k == 1.0) ? sj : ("(" + sj + "*" + lit(k) + ")");
                    o << "{const " << CT << " x=v[" << j << "];v[" << j << "]=" << MK << "(";
                    if (f.empty()) o << term("x", r, 0) << "," << term("x", r, 1);
                    else o << "(" << term("x", r, 0) << ")*" << f << ",(" << term("x", r, 1) << ")*" << f;
                    o << ");}\n";
                } else if (sj.empty()) {
                    o << "v[" << j << "]=" << CM << "(v[" << j << "]," << lit(kr) << "," << lit(ki) << ");\n";
                } else {
                    o << "v[" << j << "]=" << CM << "(v[" << j << "]," << sj << "*" << lit(kr) << "," << sj << "*"
                      << lit(ki) << ");\n";
                }
            } else {
                // (wr + i wi) * K * sign
                std::string fr = "(wr" + std::to_string(wid) + "*" + lit(kr) + "-wi" + std::to_string(wid) + "*" +
                                 lit(ki) + ")";
                std::string fi = "(wr" + std::to_string(wid) + "*" + lit(ki) + "+wi" + std::to_string(wid) + "*" +
                                 lit(kr) + ")";
                if (!sj.empty()) { fr = sj + "*" + fr; fi = sj + "*" + fi; }
                o << "v[" << j << "]=" << CM << "(v[" << j << "]," << fr << "," << fi << ");\n";
            }
        }
        if (partial) {
            for (int j = 0; j < N; ++j) { m[j] = m[j & ~move_mask]; h[j] = h[j & ~move_mask]; w[j] = w[j & ~move_mask]; }
            for (int s = 0; s < R; ++s) sdirty[s] = false;
            return;
        }
        for (int j = 0; j < N; ++j) m[j] = h[j] = w[j] = 0;
        for (int s = 0; s < R; ++s) sdirty[s] = false;
        if (e_dirty) o << "e = 0u; alive = 1u;\n";
        e_dirty = false;
    }

    // After an exchange: the compile-time factors left by a partial
    // materialize depend on staying register slots only; move them with
    // their slots.
    void rename_factors(const int *perm) {
        int mo[64], ho[64], wo[64];
        std::copy(m, m + N, mo);
        std::copy(h, h + N, ho);
        std::copy(w, w + N, wo);
        for (int jn = 0; jn < N; ++jn) {
            int jo = 0;  // old register index of the staying bits of jn
            for (int sn = 0; sn < R; ++sn)
                if (((jn >> sn) & 1) && perm[sn] < R) jo |= 1 << perm[sn];
            m[jn] = mo[jo];
            h[jn] = ho[jo];
            w[jn] = wo[jo];
        }
    }

    // LDS staging of one exchange.  When some register slot s of the new
    // layout takes an old register slot (perm[s] < R), the data splits into
    // two independent halves by that bit, which go through LDS one after the
    // other: half the buffer, so twice the workgroups per CU.  A tile whose
    // whole buffer exceeds the LDS (2^15 amplitudes) may also split on a
    // qubit that is a thread slot in both layouts: in each half the threads
    // whose old bit has that value store and those whose new bit has it load.
    //
    // The buffer is indexed in the slot coordinates of either the old layout
    // (the store is a plain register store, the load gathers) or the new one
    // (the other way round), leaving out the split slot.  Coordinate q has the
    // element weight 2^tau[q] (register slots) or (M + 1) * 2^k + d[k] with
    // k = sigma[q - R] (thread slots), M = registers per half (or all): tau
    // and sigma are bit permutations, and d[k] >= d[0] + ... + d[k-1] - 1
    // keeps the weights super-increasing (each exceeds the sum of all smaller
    // ones), so the address is injective and stays below
    // (M + 1) * 2^T + d[0] + ... + d[T-1]; each register's offset is a
    // literal.  They are chosen so that the lanes the LDS serves together hit
    // distinct banks on the store and on the load.  With d = 0 the weights of
    // the thread coordinates from k = 4 on are multiples of 16 elements, i.e.
    // all in one bank pair; a nonzero d[k] moves such a coordinate to another
    // bank pair, which an exchange needs when more than four thread
    // coordinates sit at the low lane bits of the store or of the load.
    struct XLayout {
        bool by_new = false;
        int split = -1;      // new register slot s of the split, or -1
        int tsplit = -1;     // new thread slot s of a thread split (perm[s] >= R), or -1
        int skip = -1;       // coordinate left out (perm[s] or s), or -1
        int M = 0;           // registers per staged part
        int tau[kMaxSlots] = {};
        int sigma[kMaxSlots] = {};
        uint32_t d[kMaxSlots] = {};  // extra weight of the thread coordinate of rank k
        uint32_t dsum = 0;           // sum of d
    };
    int lds_elems = 0;       // largest staging buffer of the pass (elements)
    bool persistent = false; // generating the persistent (prefetching) form
    bool stage_whole = false; // one tile per workgroup, exchanges staged whole when they fit
    bool sample_rows = false; // sampling pass with one grid row per sibling branch

    uint32_t xweight(const XLayout &x, int q) const {
        if (q == x.skip) return 0;
        return q < R ? (1u << x.tau[q]) : (uint32_t(x.M + 1) << x.sigma[q - R]) + x.d[x.sigma[q - R]];
    }
    // worst number of lanes sharing a bank pair among the lanes whose low
    // `lanes_log2` bits vary (lane bit u carries weight w[u]), for 8-byte
    // elements on `banks` 4-byte banks.  A lane bit of weight 0 is the thread
    // split of a part: the lanes with the other value of that bit sit the
    // part out, so it does not vary among the lanes served together.
    static int conflict(const uint32_t *w, int nb, int lanes_log2, int banks) {
        const int bits = std::min(nb, lanes_log2);
        const uint32_t mod = uint32_t(banks / 2);
        uint32_t wv[kMaxSlots];
        int nv = 0;
        for (int u = 0; u < bits; ++u)
            if (w[u]) wv[nv++] = w[u];
        int cnt[64] = {};
        int worst = 0;
        for (int l = 0; l < (1 << nv); ++l) {
            uint32_t a = 0;
            for (int u = 0; u < nv; ++u)
                if ((l >> u) & 1) a += wv[u];
            worst = std::max(worst, ++cnt[a % mod]);
        }
        return worst;
    }
    // lane weights of the store (old thread slots) and the load (new thread slots)
    void lane_weights(const XLayout &x, const int *perm, const int *inv, uint32_t *ww, uint32_t *wr) const {
        for (int u = 0; u < T; ++u) {
            ww[u] = xweight(x, x.by_new ? inv[R + u] : R + u);
            wr[u] = xweight(x, x.by_new ? R + u : perm[R + u]);
        }
    }
    int xcost(const XLayout &x, const int *perm, const int *inv) const {
        uint32_t ww[kMaxSlots], wr[kMaxSlots];
        lane_weights(x, perm, inv, ww, wr);
        // gfx950 serves an 8-byte LDS access 16 lanes at a time from 32
        // 4-byte banks (measured: lane stride 2^k elements costs min(2^k, 16)
        // times the conflict-free rate, odd strides are conflict-free)
        return conflict(ww, T, 4, 32) + conflict(wr, T, 4, 32);
    }
    void base_layout(XLayout &x, bool by_new, int split, const int *perm, int tsplit = -1) const {
        x.by_new = by_new;
        x.split = split;
        x.tsplit = split < 0 ? tsplit : -1;
        x.skip = split >= 0 ? (by_new ? split : perm[split]) : x.tsplit >= 0 ? (by_new ? x.tsplit : perm[x.tsplit]) : -1;
        x.M = split < 0 ? N : N / 2;
        int k = 0;
        for (int q = 0; q < R; ++q) x.tau[q] = (q == x.skip) ? 0 : k++;
        k = 0;
        for (int u = 0; u < T; ++u) x.sigma[u] = (R + u == x.skip) ? 0 : k++;
    }
    // thread slots of the buffer: all, or all but a thread split's
    int buf_threads_log2(const XLayout &x) const { return x.tsplit >= 0 ? T - 1 : T; }
    // elements of the staging buffer (one past the largest address)
    int buf_elems(const XLayout &x) const { return ((x.M + 1) << buf_threads_log2(x)) + int(x.dsum); }
    // new thread slot of a qubit that is a thread slot in both layouts, or
    // -1: preferably one that keeps its slot (a thread then stores and loads
    // in the same half, straight back into its registers) and is a wave
    // index bit (whole waves sit out a half)
    int tsplit_slot(const int *perm) const {
        int best = -1, best_score = -1;
        for (int u = 0; u < T; ++u) {
            if (perm[R + u] < R) continue;
            const int score = (perm[R + u] == R + u ? 2 : 0) + (u >= 6 && perm[R + u] - R >= 6 ? 1 : 0);
            if (score > best_score) { best_score = score; best = R + u; }
        }
        return best;
    }
    int split_slot(const int *perm) const {  // prefer a register slot that stays in place
        for (int q = 0; q < R; ++q)
            if (perm[q] == q) return q;
        for (int q = 0; q < R; ++q)
            if (perm[q] < R) return q;
        return -1;
    }
    // Every element of every part has one address, the same for its store
    // (old thread, old register) and its load (new thread, new register),
    // below buf_elems, and no two elements of a part share one.
    bool layout_valid(const XLayout &x, const int *perm, const int *inv) const {
        uint32_t ww[kMaxSlots], wr[kMaxSlots];
        lane_weights(x, perm, inv, ww, wr);
        const int parts = (x.split < 0 && x.tsplit < 0) ? 1 : 2;
        const int tso = x.tsplit >= 0 ? perm[x.tsplit] - R : -1;
        const uint32_t lim = uint32_t(buf_elems(x));
        std::vector<char> used(lim);
        for (int h = 0; h < parts; ++h) {
            std::fill(used.begin(), used.end(), 0);
            for (uint32_t t = 0; t < (1u << T); ++t) {
                if (tso >= 0 && ((t >> tso) & 1u) != uint32_t(h)) continue;
                for (int j = 0; j < N; ++j) {
                    if (x.split >= 0 && ((j >> perm[x.split]) & 1) != h) continue;
                    int val[kMaxSlots];
                    for (int s2 = 0; s2 < L; ++s2) val[s2] = s2 < R ? (j >> s2) & 1 : int((t >> (s2 - R)) & 1u);
                    uint32_t st = 0, ld = 0, tn = 0;
                    int jn = 0;
                    for (int u = 0; u < T; ++u) {
                        if ((t >> u) & 1u) st += ww[u];
                        if (val[perm[R + u]]) { ld += wr[u]; tn |= 1u << u; }
                    }
                    for (int s2 = 0; s2 < R; ++s2) {
                        if ((j >> s2) & 1) st += xweight(x, x.by_new ? inv[s2] : s2);
                        if (val[perm[s2]]) { ld += xweight(x, x.by_new ? s2 : perm[s2]); jn |= 1 << s2; }
                    }
                    (void)tn; (void)jn;
                    if (st != ld || st >= lim || used[st]) return false;
                    used[st] = 1;
                }
            }
        }
        return true;
    }
    XLayout choose_layout(const int *perm, const int *inv) const {
        // Staging in two halves (on a register slot that stays a register
        // slot, else on a qubit that is a thread slot in both layouts) halves
        // the buffer but doubles the barriers.  For one tile per workgroup it
        // pays from 2^13-amplitude tiles up: twice the workgroups fit a CU
        // (the 34-qubit sweep on (5, 8, 4): 286 against 312 ms).  The
        // persistent form holds two register sets, which limits it to two
        // workgroups per CU anyway: it stages whole (measured 6 % faster)
        // unless the whole buffer exceeds the LDS (2^15-amplitude tiles).
        const size_t whole = (size_t(N + 1) << T) * (dp ? 16 : 8);
        const bool big = whole > size_t(32) << 10;
        const bool huge = whole > size_t(160) << 10;  // more than a workgroup's LDS
        const bool halves = big && ((!persistent && !stage_whole) || huge);
        const int split = halves ? split_slot(perm) : -1;
        const int tsplit = (halves && split < 0) ? tsplit_slot(perm) : -1;
        XLayout best;
        base_layout(best, false, split, perm, tsplit);
        int best_cost = xcost(best, perm, inv);
        const int floor_cost = 2;  // store and load conflict-free
        uint64_t rng = 0x9E3779B97F4A7C15ull ^ uint64_t(uid);
        auto next = [&rng]() {
            rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
            return rng;
        };
        // extra weights (complex64 staging only): at most kMaxPad elements in all
        constexpr uint32_t kMaxPad = 256;
        for (int trial = 0; trial < 8000 && best_cost > floor_cost; ++trial) {
            XLayout x;
            base_layout(x, (trial & 1) != 0, split, perm, tsplit);
            if (trial >= 2) {
                int regs[kMaxSlots], nr = 0;
                for (int q = 0; q < R; ++q)
                    if (q != x.skip) regs[nr++] = q;
                for (int i = nr - 1; i > 0; --i)
                    std::swap(x.tau[regs[i]], x.tau[regs[next() % uint64_t(i + 1)]]);
                int thr[kMaxSlots], nt = 0;
                for (int u = 0; u < T; ++u)
                    if (R + u != x.skip) thr[nt++] = u;
                for (int i = nt - 1; i > 0; --i)
                    std::swap(x.sigma[thr[i]], x.sigma[thr[next() % uint64_t(i + 1)]]);
            }
            if (!dp && trial >= 4000) {
                // move some of the thread coordinates of rank 4 and up off
                // the bank pair of multiples of 16 (their weight mod 16 is d)
                uint32_t D = 0;
                const int tb = buf_threads_log2(x);
                for (int k = 4; k < tb; ++k) {
                    const uint32_t lo = D > 0 ? D - 1 : 0;
                    uint32_t dk = lo;
                    if (next() & 1) {
                        const uint32_t r = uint32_t(next() % 16);
                        dk = lo + ((r + 16 - lo % 16) % 16);
                    }
                    x.d[k] = dk;
                    D += dk;
                }
                x.dsum = D;
                if (D > kMaxPad) continue;
            }
            const int c = xcost(x, perm, inv);
            if (c < best_cost || (c == best_cost && x.dsum < best.dsum)) { best_cost = c; best = x; }
        }
        if (best.dsum && !layout_valid(best, perm, inv)) {  // keep to the plain weights
            base_layout(best, false, split, perm, tsplit);
            g_layout_fallbacks.fetch_add(1, std::memory_order_relaxed);
        }
        return best;
    }
    std::string lane_base(const uint32_t *w, int M) const {
        bool plain = true;
        for (int u = 0; u < T; ++u) plain = plain && w[u] == (uint32_t(M + 1) << u);
        if (plain) return "t * " + std::to_string(M + 1) + "u";
        std::ostringstream e;
        e << "0u";
        for (int u = 0; u < T; ++u)
            if (w[u]) e << " + ((t >> " << u << ") & 1u) * " << w[u] << "u";
        return e.str();
    }

    // An exchange that only swaps register slots with thread slots 4 and 5
    // (lane bits 4 and 5 of a wave) is a 2x2 transpose between a register
    // bit and a lane bit: v_permlane16_swap (lane bit 4) and
    // v_permlane32_swap (lane bit 5) on every register pair, no LDS.
    bool lane_swaps(const int *perm) {
        if (dp || T < 6) return false;
        std::vector<std::pair<int, int>> pairs;  // (register slot, lane bit)
        for (int s = 0; s < L; ++s) {
            if (perm[s] == s) continue;
            const int o = perm[s];
            if (perm[o] != s) return false;
            if (s < R && (o == R + 4 || o == R + 5)) pairs.push_back({s, o - R});
            else if (!(o < R && (s == R + 4 || s == R + 5))) return false;
        }
        if (pairs.empty()) return false;
        for (auto &pr : pairs) {
            const char *fn = pr.second == 4 ? "__builtin_amdgcn_permlane16_swap" : "__builtin_amdgcn_permlane32_swap";
            for (int j = 0; j < N; ++j) {
                if (j & (1 << pr.first)) continue;
                const int k = j | (1 << pr.first);
                o << "{const auto rx = " << fn << "(__float_as_uint(v[" << j << "].x), __float_as_uint(v[" << k
                  << "].x), false, false);const auto ry = " << fn << "(__float_as_uint(v[" << j
                  << "].y), __float_as_uint(v[" << k << "].y), false, false);v[" << j
                  << "]=F2(__uint_as_float(rx[0]),__uint_as_float(ry[0]));v[" << k
                  << "]=F2(__uint_as_float(rx[1]),__uint_as_float(ry[1]));}\n";
            }
        }
        return true;
    }

    void op_xchg(uint64_t pw) {
        int perm[kMaxSlots], inv[kMaxSlots];
        for (int s = 0; s < L; ++s) perm[s] = int((pw >> (4 * s)) & 0xf);
        for (int s = 0; s < L; ++s) inv[perm[s]] = s;
        int move_mask = 0;  // old register slots that become thread slots
        for (int s = 0; s < R; ++s)
            if (inv[s] >= R) move_mask |= 1 << s;
        const bool carry = !e_dirty;
        materialize(1.0, 0.0, carry ? move_mask : -1);
        if (lane_swaps(perm)) {
            if (carry) rename_factors(perm);
            return;
        }
        const XLayout x = choose_layout(perm, inv);
        lds_elems = std::max(lds_elems, buf_elems(x));
        uint32_t ww[kMaxSlots], wr[kMaxSlots];
        lane_weights(x, perm, inv, ww, wr);
        const int id = uid++;
        const int parts = (x.split < 0 && x.tsplit < 0) ? 1 : 2;
        // thread split: the old and the new thread bit of the split qubit
        const int tso = x.tsplit >= 0 ? perm[x.tsplit] - R : -1, tsn = x.tsplit >= 0 ? x.tsplit - R : -1;
        // register j of the old layout is stored at wb + offset, register j
        // of the new layout is loaded from rb + offset (into nv: the old
        // values of the second part are still to be stored)
        o << "{const unsigned wb" << id << " = " << lane_base(ww, x.M) << ";\n";
        o << "const unsigned rb" << id << " = " << lane_base(wr, x.M) << ";\n";
        // a thread split on a qubit that keeps its thread slot: each thread
        // stores and loads in the same half, so it loads into v directly
        const bool direct = tso >= 0 && tso == tsn;
        const std::string dst = direct ? std::string("v") : "nv" + std::to_string(id);
        if (!direct) o << CT << " nv" << id << "[" << N << "];\n";
        for (int h = 0; h < parts; ++h) {
            o << "__syncthreads();\n";
            if (tso >= 0) o << "if (((t >> " << tso << ") & 1u) == " << h << "u) {\n";
            for (int j = 0; j < N; ++j) {
                if (x.split >= 0 && ((j >> perm[x.split]) & 1) != h) continue;
                uint32_t off = 0;
                for (int s = 0; s < R; ++s)
                    if ((j >> s) & 1) off += xweight(x, x.by_new ? inv[s] : s);
                o << "lds[wb" << id << "+" << off << "u]=v[" << j << "];\n";
            }
            if (tso >= 0) o << "}\n";
            o << "__syncthreads();\n";
            if (tsn >= 0) o << "if (((t >> " << tsn << ") & 1u) == " << h << "u) {\n";
            for (int j = 0; j < N; ++j) {
                if (x.split >= 0 && ((j >> x.split) & 1) != h) continue;
                uint32_t off = 0;
                for (int s = 0; s < R; ++s)
                    if ((j >> s) & 1) off += xweight(x, x.by_new ? s : perm[s]);
                o << dst << "[" << j << "]=lds[rb" << id << "+" << off << "u];\n";
            }
            if (tsn >= 0) o << "}\n";
        }
        if (!direct)
            for (int j = 0; j < N; ++j) o << "v[" << j << "]=nv" << id << "[" << j << "];\n";
        o << "}\n";
        if (carry) rename_factors(perm);
    }

    // Offset (in elements) of register j under the physical bits of the slots.
    uint64_t reg_offset(int j, const uint8_t *phys, int s0) const {
        uint64_t r = 0;
        for (int s = s0; s < R; ++s)
            if ((j >> s) & 1) r |= 1ull << phys[s];
        return r;
    }
    // Load this thread's 2^R amplitudes of the tile at `basev` into `dst`.
    // Projections (OP_PROJ) that the program applies before its first
    // exchange and, on a register slot, before any non-diagonal op on that
    // slot: until then nothing mixes the amplitudes they zero with the
    // others, so those amplitudes need not be loaded (zeros give the same
    // result).  Each entry: locator, surviving bit value (expression).
    std::vector<std::pair<uint32_t, std::string>> early_projections() const {
        std::vector<std::pair<uint32_t, std::string>> out;
        bool nd[kMaxSlots] = {};
        for (int pc = 0; pc < P.n_ops; ++pc) {
            const uint64_t op = P.ops[pc];
            const uint32_t code = uint32_t(op & 0xff), a = uint32_t((op >> 8) & 0xff);
            const uint32_t b = uint32_t((op >> 16) & 0xff), c = uint32_t((op >> 24) & 0xff);
            if (code == OP_XCHG) break;
            if (code == OP_H || code == OP_SX || code == OP_SY || code == OP_SXDG || code == OP_SYDG) {
                if (a < uint32_t(kMaxSlots)) nd[a] = true;
                continue;
            }
            if (code != OP_PROJ || (is_reg(a) && nd[a])) continue;
            out.push_back({a, c ? "unsigned((branch >> " + std::to_string(b) + ") & 1ull)" : std::to_string(b) + "u"});
        }
        return out;
    }
    void emit_load(const std::string &dst, const std::string &basev, const std::vector<int> &tld) {
        // loads of amplitudes that an early projection zeroes are skipped:
        // a per-thread condition (thread and tile-index bits) and, per load,
        // the register bits
        const auto proj = early_projections();
        std::string ok;
        std::vector<std::pair<int, std::string>> regp;  // (register slot, surviving value)
        for (const auto &pr : proj) {
            const uint32_t loc = pr.first;
            if (is_reg(loc)) {
                regp.push_back({int(loc), pr.second});
            } else {
                const std::string bit = is_glob(loc)
                    ? "unsigned(((" + basev + ") >> " + std::to_string(loc & 0x7f) + ") & 1ull)"
                    : "((t >> " + std::to_string(loc - R) + ") & 1u)";
                ok += " && (" + bit + " == " + pr.second + ")";
            }
        }
        const int lid = ok.empty() ? -1 : uid++;  // no new names otherwise
        if (!ok.empty()) o << "const bool ldok" << lid << " = true" << ok << ";\n";
        // condition of a load covering the registers of `mask` bits equal to those of j
        auto cond = [&](int j, int s0) -> std::string {
            std::string c = ok.empty() ? "" : "ldok" + std::to_string(lid);
            for (const auto &rp : regp) {
                if (rp.first < s0) continue;
                c += std::string(c.empty() ? "" : " && ") + "(" + (((j >> rp.first) & 1) ? "1u" : "0u") + " == " +
                     rp.second + ")";
            }
            return c;
        };
        if (dp) {
            o << "{const v2d* src = (const v2d*)(srcp + (" << basev << " | " << scatter_expr("t", tld, true)
              << "));\n";
            for (int j = 0; j < N; ++j) {
                const std::string c = cond(j, 0);
                if (!c.empty()) o << "if (" << c << ") ";
                o << "{const v2d w = __builtin_nontemporal_load(src + " << hex64(reg_offset(j, P.ld_phys, 0))
                  << ");" << dst << "[" << j << "]=D2(w.x,w.y);}\n";
                if (!c.empty()) o << "else {" << dst << "[" << j << "]=D2(0.0,0.0);}\n";
            }
        } else {
            o << "{const v4f* src = (const v4f*)(srcp + (" << basev << " | " << scatter_expr("t", tld, true)
              << "));\n";
            for (int j = 0; j < N; j += 2) {
                const std::string c = cond(j, 1);  // a load covers both values of slot 0
                if (!c.empty()) o << "if (" << c << ") ";
                o << "{const v4f w = __builtin_nontemporal_load(src + " << hex64(reg_offset(j, P.ld_phys, 1) / 2)
                  << ");" << dst << "[" << j << "]=F2(w.x,w.y);" << dst << "[" << j + 1 << "]=F2(w.z,w.w);}\n";
                if (!c.empty())
                    o << "else {" << dst << "[" << j << "]=F2(0.f,0.f);" << dst << "[" << j + 1 << "]=F2(0.f,0.f);}\n";
            }
        }
        o << "}\n";
    }
    void emit_store(const std::vector<int> &tst) {
        if (dp) {
            o << "{v2d* dst = (v2d*)(a + (bst | " << scatter_expr("t", tst, true) << "));\n";
            for (int j = 0; j < N; ++j)
                o << "{const v2d w = {v[" << j << "].x,v[" << j << "].y};__builtin_nontemporal_store(w, dst + "
                  << hex64(reg_offset(j, P.st_phys, 0)) << ");}\n";
        } else {
            o << "{v4f* dst = (v4f*)(a + (bst | " << scatter_expr("t", tst, true) << "));\n";
            for (int j = 0; j < N; j += 2)
                o << "{const v4f w = {v[" << j << "].x,v[" << j << "].y,v[" << j + 1 << "].x,v[" << j + 1
                  << "].y};__builtin_nontemporal_store(w, dst + " << hex64(reg_offset(j, P.st_phys, 1) / 2)
                  << ");}\n";
        }
        o << "}\n";
    }
    // FP64 |amp|^2 of the tile into part[tile]: products of FP32 values are
    // exact in FP64; fixed order: registers, then an xor butterfly over the
    // wave, then the waves of the workgroup in index order.  In a loop the
    // reduction buffer alternates between two halves so that a wave of the
    // next tile cannot overwrite a value thread 0 has not read yet.
    void emit_norm(bool loop) {
        o << "{double acc = 0.0;\n";
        for (int j = 0; j < N; ++j)
            o << "acc += (double)v[" << j << "].x*(double)v[" << j << "].x + (double)v[" << j << "].y*(double)v["
              << j << "].y;\n";
        const int waves = (1 << T) >= 64 ? (1 << T) / 64 : 1;
        const int width = (1 << T) >= 64 ? 64 : (1 << T);
        for (int off = width / 2; off >= 1; off /= 2)
            o << "acc += __shfl_xor(acc, " << off << ", " << width << ");\n";
        o << "__shared__ double red[" << 2 * waves << "];\n";
        const std::string half = loop ? "(unsigned(it & 1u) * " + std::to_string(waves) + "u)" : "0u";
        o << "if ((t & " << (width - 1) << "u) == 0u) red[" << half << " + t / " << width << "u] = acc;\n";
        o << "__syncthreads();\nif (t == 0u) {double s = 0.0;\n";
        for (int w = 0; w < waves; ++w) o << "s += red[" << half << " + " << w << "u];\n";
        o << "part[tile] = s;}\n}\n";
    }
    // Sampling pass: for each listed output index x of this tile, the thread
    // whose slots hold x writes its amplitude to part (complex64) at the
    // entry's slot; x's thread and register coordinates are its bits at the
    // store positions of the thread and register slots.
    void emit_sample() {
        o << "{" << CT << "* outp = (" << CT << "*)part;\n";
        o << "const unsigned e1 = tab->start[blockIdx.x + 1u];\n";
        o << "for (unsigned e = tab->start[blockIdx.x]; e < e1; ++e) {\n";
        o << "const unsigned long long x = tab->xs[e];\nunsigned tt = 0u, jj = 0u;\n";
        for (int u = 0; u < T; ++u)
            o << "tt |= unsigned((x >> " << int(P.st_phys[R + u]) << ") & 1ull) << " << u << ";\n";
        for (int q = 0; q < R; ++q)
            o << "jj |= unsigned((x >> " << int(P.st_phys[q]) << ") & 1ull) << " << q << ";\n";
        o << "if (tt == t) {" << CT << " val = v[0];\nswitch (jj) {\n";
        for (int j = 1; j < N; ++j) o << "case " << j << "u: val = v[" << j << "]; break;\n";
        o << "default: break;\n}\noutp[" << (sample_rows ? "tile0 * blockIdx.y + " : "")
          << "tab->slot[e]] = val;}\n}\n}\n";
    }
    // FP64 <result|other> of the tile: the other state (the kernel's `a`) is
    // read at the addresses the store would write; conj(v) * w with exact
    // FP64 products of the FP32 values, summed in the fixed order of
    // emit_norm into part[tile] (re) and part[ntile + tile] (im).
    void emit_dot(bool loop, const std::vector<int> &tst) {
        o << "{double dre = 0.0, dim = 0.0;\n";
        if (dp) {
            o << "const v2d* oth = (const v2d*)(a + (bst | " << scatter_expr("t", tst, true) << "));\n";
            for (int j = 0; j < N; ++j)
                o << "{const v2d w = __builtin_nontemporal_load(oth + " << hex64(reg_offset(j, P.st_phys, 0))
                  << ");dre += v[" << j << "].x*w.x + v[" << j << "].y*w.y;dim += v[" << j << "].x*w.y - v["
                  << j << "].y*w.x;}\n";
        } else {
            o << "const v4f* oth = (const v4f*)(a + (bst | " << scatter_expr("t", tst, true) << "));\n";
            for (int j = 0; j < N; j += 2) {
                o << "{const v4f w = __builtin_nontemporal_load(oth + " << hex64(reg_offset(j, P.st_phys, 1) / 2)
                  << ");\n";
                for (int h2 = 0; h2 < 2; ++h2) {
                    const std::string vx = "(double)v[" + std::to_string(j + h2) + "].x";
                    const std::string vy = "(double)v[" + std::to_string(j + h2) + "].y";
                    const std::string wx = h2 ? "(double)w.z" : "(double)w.x";
                    const std::string wy = h2 ? "(double)w.w" : "(double)w.y";
                    o << "dre += " << vx << "*" << wx << " + " << vy << "*" << wy << ";dim += " << vx << "*" << wy
                      << " - " << vy << "*" << wx << ";\n";
                }
                o << "}\n";
            }
        }
        const int waves = (1 << T) >= 64 ? (1 << T) / 64 : 1;
        const int width = (1 << T) >= 64 ? 64 : (1 << T);
        for (int off = width / 2; off >= 1; off /= 2)
            o << "dre += __shfl_xor(dre, " << off << ", " << width << ");dim += __shfl_xor(dim, " << off << ", "
              << width << ");\n";
        o << "__shared__ double rdot[" << 4 * waves << "];\n";
        const std::string half = loop ? "(unsigned(it & 1u) * " + std::to_string(2 * waves) + "u)" : "0u";
        o << "if ((t & " << (width - 1) << "u) == 0u) {rdot[" << half << " + t / " << width << "u] = dre;rdot["
          << half << " + " << waves << "u + t / " << width << "u] = dim;}\n";
        o << "__syncthreads();\nif (t == 0u) {double sr = 0.0, si = 0.0;\n";
        for (int w = 0; w < waves; ++w)
            o << "sr += rdot[" << half << " + " << w << "u];si += rdot[" << half << " + " << waves + w << "u];\n";
        o << "part[tile - tile0] = sr;part[ntile + (tile - tile0)] = si;}\n}\n";
    }
    void emit_ops() {
        bool scaled = false;
        for (int pc = 0; pc < P.n_ops; ++pc) {
            const uint64_t op = P.ops[pc];
            const uint32_t code = op & 0xff, a = (op >> 8) & 0xff, b = (op >> 16) & 0xff,
                           c = (op >> 24) & 0xff;
            switch (code) {
            case OP_H: case OP_SX: case OP_SY: case OP_SXDG: case OP_SYDG: butterfly(code, int(a)); break;
            case OP_PHASE: op_phase(a, int(b)); break;
            case OP_CZ: op_cz(a, b); break;
            case OP_PROJ: op_proj(a, b, c); break;
            case OP_ZB: op_zb(a, b); break;
            case OP_XCHG: op_xchg(P.ops[++pc]); break;
            case OP_SCALE: materialize(P.scale_re, P.scale_im); scaled = true; break;
            default: break;
            }
        }
        if (!scaled) materialize(1.0, 0.0);
    }
    void emit_init(int init_kind, int n, const std::vector<int> &tld) {
        if (init_kind == 1) {
            const std::string val = lit(std::pow(2.0, -0.5 * n));
            for (int j = 0; j < N; ++j) o << "v[" << j << "]=" << MK << "(" << val << "," << ZERO << ");\n";
        } else {
            o << "{const unsigned long long me = base | " << scatter_expr("t", tld, true) << ";\n";
            for (int j = 0; j < N; ++j)
                o << "v[" << j << "]=" << MK << "((me | " << hex64(reg_offset(j, P.ld_phys, 0)) << ") == basis ? "
                  << lit(1.0) << " : " << ZERO << ", " << ZERO << ");\n";
            o << "}\n";
        }
    }

    // init_kind: -1 = load the state; 0/1/2 = generate |0>, |+>^n or |basis>
    // in registers (first pass of sv_simulate).  norm: accumulate the FP64
    // sum of |amp|^2 of the tile into part[tile] after the store.
    // batched: the state pointer and branch come from an entry table indexed
    // by blockIdx.y (all entries share this plan).
    // loop: each workgroup walks the tiles tile0 + blockIdx.x, + gridDim.x,
    // ... below tile0 + ntile, loading the next tile into a second register
    // set while it computes the current one.
    std::string emit(const std::string &name, bool &uses_lds, int init_kind = -1, bool norm = false,
                     int n = 0, bool batched = false, bool loop = false, bool dot = false,
                     bool sample = false, bool tiles = false) {
        if (sample) loop = false;  // one workgroup per listed tile
        tiles = tiles && sample;
        sample_rows = sample && !tiles && init_kind < 0;
        uses_lds = false;
        persistent = loop;
        for (int pc = 0; pc < P.n_ops; ++pc) {
            if ((P.ops[pc] & 0xff) == OP_XCHG) { uses_lds = true; ++pc; }
        }
        std::vector<int> glob(P.glob_bits, P.glob_bits + P.n_glob);
        std::vector<int> globst(P.glob_st, P.glob_st + P.n_glob);
        std::vector<int> tld, tst;
        for (int u = 0; u < T; ++u) { tld.push_back(P.ld_phys[R + u]); tst.push_back(P.st_phys[R + u]); }
        o << "extern \"C\" __global__ void __launch_bounds__(" << (1 << T) << ") " << name;
        if (batched) {
            o << "(const BatchEntryJ* __restrict__ ents, unsigned long long tile0) {\n";
            o << "const BatchEntryJ en = ents[blockIdx.y];\n";
            o << CT << "* a = (" << CT << "*)en.amps;\n";
            o << "const " << CT << "* srcp = a;\n";
            o << "const unsigned long long branch = en.branch, basis = 0ull;\n";
            o << "double* part = nullptr;\n";
        } else if (sample_rows) {
            // Sampling several sibling branches in one launch: row y = blockIdx.y
            // samples branch branch0 | (the bits of y deposited on the set bits
            // of `basis`) and writes its amplitudes at outp + y * tile0.
            o << "(const " << CT << "* srcp, " << CT << "* a, unsigned long long branch0, unsigned long long tile0, "
                 "unsigned long long basis, double* __restrict__ part, unsigned long long ntile) {\n";
            o << "unsigned long long branch = branch0;\n"
                 "{unsigned long long msk = basis, y = blockIdx.y;\n"
                 "while (msk) {const unsigned long long low = msk & (~msk + 1ull);\n"
                 "if (y & 1ull) branch |= low;\ny >>= 1;\nmsk ^= low;}}\n";
        } else {
            // srcp == a for passes that work in place
            o << "(const " << CT << "* srcp, " << CT << "* a, unsigned long long branch, unsigned long long tile0, "
                 "unsigned long long basis, double* __restrict__ part, unsigned long long ntile) {\n";
        }
        if (uses_lds) o << "extern __shared__ " << CT << " lds[];\n";
        o << "const unsigned t = threadIdx.x;\n(void)basis; (void)part; (void)branch; (void)srcp;\n";
        if (sample) {
            o << "const SampleTabJ* tab = (const SampleTabJ*)a;\n";
            o << "const unsigned long long tile = tab->tiles[blockIdx.x];\n";
            o << "const unsigned long long base = " << scatter_expr("tile", glob, true) << ";\n";
            if (tiles) {  // the listed tiles go whole into the state at `part`
                o << "a = (" << CT << "*)part;\n";
                o << "const unsigned long long bst = " << scatter_expr("tile", globst, true) << ";\n";
            }
            o << CT << " v[" << N << "];\n";
            if (init_kind >= 0) emit_init(init_kind, n, tld);
            else emit_load("v", "base", tld);
        } else if (!loop) {
            o << "const unsigned long long tile = tile0 + blockIdx.x;\n";
            o << "const unsigned long long base = " << scatter_expr("tile", glob, true) << ";\n";
            o << "const unsigned long long bst = " << scatter_expr("tile", globst, true) << ";\n";
            o << CT << " v[" << N << "];\n";
            if (init_kind >= 0) emit_init(init_kind, n, tld);
            else emit_load("v", "base", tld);
        } else {
            const bool pre = init_kind < 0;
            o << "const unsigned long long tend = tile0 + ntile;\n";
            o << "unsigned long long tile = tile0 + blockIdx.x;\n";
            if (pre) {
                o << CT << " nx[" << N << "];\n";
                o << "if (tile < tend) {const unsigned long long nb = " << scatter_expr("tile", glob, true) << ";\n";
                emit_load("nx", "nb", tld);
                o << "}\n";
            }
            o << "for (unsigned it = 0u; tile < tend; tile += gridDim.x, ++it) {\n";
            o << "const unsigned long long base = " << scatter_expr("tile", glob, true) << ";\n";
            o << "const unsigned long long bst = " << scatter_expr("tile", globst, true) << ";\n";
            o << CT << " v[" << N << "];\n";
            if (pre) {
                for (int j = 0; j < N; ++j) o << "v[" << j << "]=nx[" << j << "];\n";
                o << "{const unsigned long long nt = tile + gridDim.x;\nif (nt < tend) {"
                  << "const unsigned long long nb = " << scatter_expr("nt", glob, true) << ";\n";
                emit_load("nx", "nb", tld);
                o << "}}\n";
            } else {
                emit_init(init_kind, n, tld);
            }
        }
        o << "unsigned e = 0u, alive = 1u;\n(void)e; (void)alive;\n";
        emit_ops();
        if (sample && !tiles) {
            emit_sample();
        } else if (dot) {
            emit_dot(loop, tst);
        } else {
            emit_store(tst);
            if (norm) emit_norm(loop);
        }
        if (loop) o << "}\n";
        o << "}\n";
        return o.str();
    }
};

struct CacheEntry {
    hipModule_t mod = nullptr;
    std::vector<hipFunction_t> fns;
    std::vector<size_t> lds;
    std::vector<unsigned> resident;  // workgroups of each pass kernel the device holds at once
    double compile_s = 0;
};

std::mutex g_mu;
std::map<std::pair<int, std::string>, std::shared_ptr<CacheEntry>> g_cache;   // by source text
std::map<std::pair<int, std::string>, std::shared_ptr<CacheEntry>> g_pcache;  // by pass programs

// The generated source is a function of the pass programs, the tile shape, n
// and the variant: a plan whose programs were compiled before (e.g. the same
// circuit created again) reuses the kernels without generating the source.
std::string program_key(const Plan &plan, int variant) {
    std::string k;
    const int head[4] = {variant, plan.n, plan.R, plan.T};
    k.append(reinterpret_cast<const char *>(head), sizeof(head));
    for (const Pass &p : plan.passes)
        k.append(reinterpret_cast<const char *>(&p.prog), sizeof(PassProg));
    return k;
}
double g_total_compile_s = 0;

// 64-bit FNV-1a hash (Fowler, Noll, Vo) of a byte string.
uint64_t fnv1a(const void *p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

// On-disk cache of compiled code objects (QSV_JIT_CACHE=<directory>): a
// code object is stored under the hash of its source text and the compiler
// options, so a later process loads it instead of compiling it again.
std::string cache_path(const std::string &src, const char *const *opts, size_t nopt) {
    const char *dir = std::getenv("QSV_JIT_CACHE");
    if (!dir || !dir[0]) return std::string();
    uint64_t h = fnv1a(src.data(), src.size());
    for (size_t i = 0; i < nopt; ++i) h = fnv1a(opts[i], std::strlen(opts[i]), h);
    char name[64];
    std::snprintf(name, sizeof name, "/qsv_%016llx.co", (unsigned long long)h);
    return std::string(dir) + name;
}

bool read_file(const std::string &path, std::vector<char> &out) {
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    bool ok = n > 0;
    if (ok) {
        out.resize(size_t(n));
        ok = std::fread(out.data(), 1, size_t(n), f) == size_t(n);
    }
    std::fclose(f);
    return ok;
}

void write_file_atomically(const std::string &path, const std::vector<char> &data) {
    char suffix[32];
    std::snprintf(suffix, sizeof suffix, ".tmp%llx",
                  (unsigned long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    const std::string tmp = path + suffix;
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    std::fclose(f);
    if (ok) std::rename(tmp.c_str(), path.c_str());
    else std::remove(tmp.c_str());
}

qsv_status compile_source(const std::string &src, std::vector<char> &code, std::string &log) {
    if (const char *dump = std::getenv("QSV_JIT_DUMP")) {  // debugging aid: keep the source
        if (FILE *f = std::fopen(dump, "w")) {
            std::fwrite(src.data(), 1, src.size(), f);
            std::fclose(f);
        }
    }
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-mllvm", "-simplifycfg-sink-common=false"};
    const size_t nopt = sizeof(opts) / sizeof(opts[0]);
    const std::string cached = cache_path(src, opts, nopt);
    if (!cached.empty() && read_file(cached, code)) return QSV_OK;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "qsv_pass.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return fail(QSV_EINTERNAL, "hiprtcCreateProgram failed");
    hiprtcResult r = hiprtcCompileProgram(prog, int(nopt), opts);
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    log.assign(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    if (r != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return fail(QSV_EINTERNAL, "hipRTC compile failed: " + log.substr(0, 2000));
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    if (!cached.empty()) write_file_atomically(cached, code);
    return QSV_OK;
}

}  // namespace

// Kernel name of pass p: the last pass of an inner-product or sampling
// variant is named for what it does, so traces tell the kinds apart.
std::string pass_name(const Plan &plan, int variant, size_t p) {
    const bool last = p + 1 == plan.passes.size() && !(variant & kJitBatched);
    const char *kind = (last && (variant & kJitDot))      ? "qsv_dot_"
                       : (last && (variant & kJitTiles))  ? "qsv_tiles_"
                       : (last && (variant & kJitSample)) ? "qsv_sample_"
                                                          : "qsv_pass_";
    return kind + std::to_string(p);
}

std::string jit_source(const Plan &plan, std::vector<size_t> *lds_bytes, int variant) {
    const int init_kind = (variant & 4) ? (variant & 3) : -1;
    const bool norm = (variant & 8) != 0;
    const bool dot = (variant & kJitDot) != 0;
    const bool sample = (variant & kJitSample) != 0;
    const bool tiles = (variant & kJitTiles) != 0;
    const bool dp = (variant & kJitDouble) != 0;
    const bool batched = (variant & kJitBatched) != 0;
    std::string src = kPrelude;
    for (size_t p = 0; p < plan.passes.size(); ++p) {
        Gen g(plan.passes[p].prog, plan.R, plan.T, dp);
        g.stage_whole = (variant & kJitWhole) != 0;
        bool uses_lds = false;
        const bool loop = jit_pass_loop(variant, p) && !batched;
        const bool last = p + 1 == plan.passes.size();
        src += g.emit(pass_name(plan, variant, p), uses_lds, p == 0 ? init_kind : -1,
                      norm && !batched && last, plan.n, batched, loop, dot && !batched && last,
                      sample && !batched && last, tiles);
        if (lds_bytes) lds_bytes->push_back(uses_lds ? size_t(g.lds_elems) * (dp ? 16 : 8) : 0);
    }
    return src;
}

qsv_status jit_compile_only(const Plan &plan, size_t *code_bytes, double *seconds) {
    std::vector<size_t> lds;
    std::vector<char> code;
    std::string log;
    {
        // every form's exchange layouts pass their check (generation only)
        const unsigned before = g_layout_fallbacks.load();
        for (int v : {kJitInit | 1 | kJitNorm, kJitInit | 1 | kJitNorm | kJitLoop,
                      kJitInit | 1 | kJitNorm | kJitWhole, kJitSample, kJitBatched | kJitInit | 1})
            (void)jit_source(plan, &lds, v);
        if (g_layout_fallbacks.load() != before)
            return fail(QSV_EINTERNAL, "an exchange layout failed its injectivity check");
    }
    auto t0 = std::chrono::steady_clock::now();
    // the complex128 instantiation must compile too
    qsv_status st = compile_source(jit_source(plan, &lds, kJitDouble | kJitInit | 1 | kJitNorm), code, log);
    if (st != QSV_OK) return st;
    st = compile_source(jit_source(plan, &lds, kJitInit | 1 | kJitNorm | kJitLoop), code, log);
    if (st != QSV_OK) return st;
    // the inner-product epilogue, both forms
    st = compile_source(jit_source(plan, &lds, kJitInit | 2 | kJitDot), code, log);
    if (st != QSV_OK) return st;
    st = compile_source(jit_source(plan, &lds, kJitInit | 2 | kJitDot | kJitLoop), code, log);
    if (st != QSV_OK) return st;
    st = compile_source(jit_source(plan, &lds, kJitSample), code, log);  // sampling last pass
    if (st != QSV_OK) return st;
    // the batched form (entry table per grid row), from |+> as batches run it
    st = compile_source(jit_source(plan, &lds, kJitBatched | kJitInit | 1), code, log);
    if (st != QSV_OK) return st;
    std::string src = jit_source(plan, &lds, kJitInit | 1 | kJitNorm);
    st = compile_source(src, code, log);
    if (st != QSV_OK) return st;
    if (seconds)
        *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (code_bytes) *code_bytes = code.size();
    return QSV_OK;
}

// Compiles outside the cache lock, so that several plans can be prepared
// from concurrent threads (the batch does); a source compiled twice by racing
// threads keeps the first module.
qsv_status jit_prepare(Plan &plan, int variant) {
    if (plan.jit_variants.count(variant)) return QSV_OK;
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return fail(QSV_EHIP, "hipGetDevice failed");
    const auto pkey = std::make_pair(dev, program_key(plan, variant));
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto pit = g_pcache.find(pkey);
        if (pit != g_pcache.end()) {
            plan.jit_variants[variant] = pit->second;
            return QSV_OK;
        }
    }
    std::vector<size_t> lds;
    std::string src = jit_source(plan, &lds, variant);
    for (size_t b : lds)  // a workgroup holds at most 160 KiB of LDS on gfx950
        if (b > (size_t(160) << 10))
            return fail(QSV_EUNSUPPORTED, "compiled pass needs more LDS than a workgroup holds "
                                          "(tiles of 2^15 amplitudes run one tile per workgroup)");
    auto key = std::make_pair(dev, src);
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            g_pcache[pkey] = it->second;
            plan.jit_variants[variant] = it->second;
            return QSV_OK;
        }
    }
    auto e = std::make_shared<CacheEntry>();
    std::vector<char> code;
    std::string log;
    auto t0 = std::chrono::steady_clock::now();
    qsv_status st = compile_source(src, code, log);
    if (st != QSV_OK) return st;
    he = hipModuleLoadData(&e->mod, code.data());
    if (he != hipSuccess) return fail(QSV_EHIP, std::string("hipModuleLoadData: ") + hipGetErrorString(he));
    int cus = 0;
    he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (he != hipSuccess) return fail(QSV_EHIP, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(he));
    for (size_t p = 0; p < plan.passes.size(); ++p) {
        hipFunction_t f;
        he = hipModuleGetFunction(&f, e->mod, pass_name(plan, variant, p).c_str());
        if (he != hipSuccess)
            return fail(QSV_EHIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(he));
        e->fns.push_back(f);
        int per_cu = 0;
        he = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 1 << plan.T, lds[p]);
        if (he != hipSuccess) return fail(QSV_EHIP, std::string("occupancy query: ") + hipGetErrorString(he));
        e->resident.push_back(unsigned(std::max(1, per_cu) * std::max(1, cus)));
    }
    e->lds = lds;
    e->compile_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::lock_guard<std::mutex> g(g_mu);
    auto ins = g_cache.emplace(key, e);
    if (ins.second) g_total_compile_s += e->compile_s;
    else hipModuleUnload(e->mod);  // another thread compiled the same source first
    g_pcache[pkey] = ins.first->second;
    plan.jit_variants[variant] = ins.first->second;
    return QSV_OK;
}

qsv_status jit_launch(const Plan &plan, int variant, void *amps, void *scratch, uint64_t branch,
                      uint64_t basis, double *part, hipStream_t s, std::vector<float> *pass_ms,
                      const void *src0, const void *dot_other, const SampleTab *sample_tab,
                      uint64_t sample_tiles, void *sample_out, uint64_t sample_rows, uint64_t sample_stride,
                      uint64_t max_tiles) {
    auto vit = plan.jit_variants.find(variant);
    if (vit == plan.jit_variants.end()) return fail(QSV_EINTERNAL, "jit variant not prepared");
    const CacheEntry &e = *static_cast<const CacheEntry *>(vit->second.get());
    const int L = plan.R + plan.T;
    const uint64_t all_tiles = 1ull << (plan.n - L);
    const uint64_t tiles = (max_tiles && max_tiles < all_tiles) ? max_tiles : all_tiles;
    const uint64_t chunk = 1ull << 30;
    const size_t np = plan.passes.size();
    if (plan.oop && (!scratch || (!(variant & kJitInit) && !src0 && np % 2)))
        return fail(QSV_EINTERNAL, "out-of-place plan without a usable buffer schedule");
    // Out-of-place plans alternate between the two buffers so that the last
    // pass writes the caller's: pass p writes amps when np - p is odd.
    std::vector<hipEvent_t> ev;
    if (pass_ms) {  // timing of each pass (autotuner)
        ev.resize(np + 1);
        for (auto &x : ev)
            if (hipEventCreate(&x) != hipSuccess) return fail(QSV_EHIP, "jit_launch: event create");
    }
    void *in = src0 ? const_cast<void *>(src0) : amps;  // never written: pass 0 writes amps or scratch
    for (size_t p = 0; p < np; ++p) {
        if (pass_ms && hipEventRecord(ev[p], s) != hipSuccess) return fail(QSV_EHIP, "jit_launch: event");
        void *outb = (!plan.oop || (np - p) % 2 == 1) ? amps : scratch;
        if ((variant & kJitSample) && p + 1 == np) {
            // the listed tiles only; writes the listed amplitudes
            if (sample_tiles) {
                // basis: bit mask of the sibling branches' own bits (0 for one
                // branch); tt: the output row stride in amplitudes
                unsigned long long br = branch, tt = sample_stride, bs = basis, nt = sample_tiles;
                void *src = in, *dst = const_cast<SampleTab *>(sample_tab);
                double *pt = static_cast<double *>(sample_out);
                void *args[] = {&src, &dst, &br, &tt, &bs, &pt, &nt};
                hipError_t he = hipModuleLaunchKernel(e.fns[p], unsigned(sample_tiles), unsigned(sample_rows), 1,
                                                      1u << plan.T, 1, 1, unsigned(e.lds[p]), s, args, nullptr);
                if (he != hipSuccess)
                    return fail(QSV_EHIP, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(he));
            }
            break;
        }
        for (uint64_t t0 = 0; t0 < tiles; t0 += chunk) {
            const uint64_t cnt = (tiles - t0 < chunk) ? tiles - t0 : chunk;
            unsigned long long br = branch, tt = t0, bs = basis, nt = cnt;
            void *src = in, *dst = outb;
            double *pt = part;
            if ((variant & kJitDot) && p + 1 == np) {
                // the dot pass reads the other state; its partials are indexed
                // from t0 (re at [0, cnt), im at [cnt, 2 cnt) of this chunk's block)
                dst = const_cast<void *>(dot_other);
                pt = part + 2 * t0;
            }
            void *args[] = {&src, &dst, &br, &tt, &bs, &pt, &nt};
            // a looping kernel gets as many workgroups as the device holds at once
            const uint64_t grid = jit_pass_loop(variant, p) ? std::min<uint64_t>(cnt, e.resident[p]) : cnt;
            hipError_t he = hipModuleLaunchKernel(e.fns[p], unsigned(grid), 1, 1, 1u << plan.T, 1, 1,
                                                  unsigned(e.lds[p]), s, args, nullptr);
            if (he != hipSuccess)
                return fail(QSV_EHIP, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(he));
        }
        in = outb;
    }
    if (pass_ms) {
        bool ok = hipEventRecord(ev[np], s) == hipSuccess && hipEventSynchronize(ev[np]) == hipSuccess;
        pass_ms->assign(np, 0.f);
        for (size_t p = 0; p < np && ok; ++p) ok = hipEventElapsedTime(&(*pass_ms)[p], ev[p], ev[p + 1]) == hipSuccess;
        for (auto &x : ev) hipEventDestroy(x);
        if (!ok) return fail(QSV_EHIP, "jit_launch: pass timing");
    }
    return QSV_OK;
}

qsv_status jit_launch_batched(const Plan &plan, int variant, const void *ents, unsigned count,
                              hipStream_t s) {
    auto vit = plan.jit_variants.find(variant);
    if (vit == plan.jit_variants.end()) return fail(QSV_EINTERNAL, "jit variant not prepared");
    const CacheEntry &e = *static_cast<const CacheEntry *>(vit->second.get());
    const int L = plan.R + plan.T;
    const uint64_t tiles = 1ull << (plan.n - L);
    const uint64_t chunk = 1ull << 30;
    for (size_t p = 0; p < plan.passes.size(); ++p) {
        for (uint64_t t0 = 0; t0 < tiles; t0 += chunk) {
            const uint64_t cnt = (tiles - t0 < chunk) ? tiles - t0 : chunk;
            const void *en = ents;
            unsigned long long tt = t0;
            void *args[] = {&en, &tt};
            hipError_t he = hipModuleLaunchKernel(e.fns[p], unsigned(cnt), count, 1, 1u << plan.T, 1, 1,
                                                  unsigned(e.lds[p]), s, args, nullptr);
            if (he != hipSuccess)
                return fail(QSV_EHIP, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(he));
        }
    }
    return QSV_OK;
}

double jit_total_compile_seconds() {
    std::lock_guard<std::mutex> g(g_mu);
    return g_total_compile_s;
}

}  // namespace qsv
