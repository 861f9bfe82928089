// Host emulation of one fused pass program (planner/encoding check only).
//
// Executes exactly the op semantics of the GPU tile kernel on a host
// complex64 array: tile index -> non-resident bits, slots -> resident bits,
// XCHG = permutation of slot bits, butterflies with factored-out scalars.
// Used by sv_debug_emulate for CPU-only test runs; no product entry point
// calls it.
#include <cmath>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

void emulate_pass(const PassProg &P, int n, int R, int T, uint64_t branch, const float *src, float *dst) {
    const int L = R + T;
    const int N = 1 << R, NT = 1 << T;
    const uint64_t tiles = 1ull << (n - L);
    const double s2 = std::sqrt(0.5);
    const float wr[8] = {1.f, float(s2), 0.f, float(-s2), -1.f, float(-s2), 0.f, float(s2)};
    const float wi[8] = {0.f, float(s2), 1.f, float(s2), 0.f, float(-s2), -1.f, float(-s2)};
    std::vector<float> v(size_t(2) << L), w(size_t(2) << L);
    for (uint64_t tile = 0; tile < tiles; ++tile) {
        uint64_t base = 0, bst = 0;  // tile origin in the read and the written map
        for (int i = 0; i < P.n_glob; ++i) base |= ((tile >> i) & 1ull) << P.glob_bits[i];
        for (int i = 0; i < P.n_glob; ++i) bst |= ((tile >> i) & 1ull) << P.glob_st[i];
        auto addr = [&](const uint8_t *phys, uint32_t x, uint64_t origin) {
            uint64_t a = origin;
            for (int s = 0; s < L; ++s)
                if ((x >> s) & 1) a |= 1ull << phys[s];
            return a;
        };
        // slot coordinate x = j | t << R
        for (uint32_t x = 0; x < (1u << L); ++x) {
            uint64_t a = addr(P.ld_phys, x, base);
            v[2 * x] = src[2 * a];
            v[2 * x + 1] = src[2 * a + 1];
        }
        auto bit = [&](uint32_t x, uint32_t loc) -> int {
            if (loc & kLocGlobal) return int((base >> (loc & 0x7f)) & 1);
            return int((x >> loc) & 1);
        };
        for (int pc = 0; pc < P.n_ops; ++pc) {
            const uint64_t op = P.ops[pc];
            const uint32_t code = op & 0xff, a = (op >> 8) & 0xff, b = (op >> 16) & 0xff,
                           c = (op >> 24) & 0xff;
            switch (code) {
            case OP_H: case OP_SX: case OP_SY: case OP_SXDG: case OP_SYDG:
                for (uint32_t x = 0; x < (1u << L); ++x) {
                    if ((x >> a) & 1) continue;
                    uint32_t y = x | (1u << a);
                    float xr = v[2 * x], xi = v[2 * x + 1], yr = v[2 * y], yi = v[2 * y + 1];
                    float ar, ai, br, bi;
                    if (code == OP_H) { ar = xr + yr; ai = xi + yi; br = xr - yr; bi = xi - yi; }
                    else if (code == OP_SX) { ar = xr + yi; ai = xi - yr; br = yr + xi; bi = yi - xr; }
                    else if (code == OP_SY) { ar = xr - yr; ai = xi - yi; br = xr + yr; bi = xi + yi; }
                    else if (code == OP_SXDG) { ar = xr - yi; ai = xi + yr; br = yr - xi; bi = yi + xr; }
                    else { ar = xr + yr; ai = xi + yi; br = yr - xr; bi = yi - xi; }
                    v[2 * x] = ar; v[2 * x + 1] = ai; v[2 * y] = br; v[2 * y + 1] = bi;
                }
                break;
            case OP_PHASE:
                for (uint32_t x = 0; x < (1u << L); ++x) {
                    if (!bit(x, a)) continue;
                    float xr = v[2 * x], xi = v[2 * x + 1];
                    v[2 * x] = xr * wr[b] - xi * wi[b];
                    v[2 * x + 1] = xr * wi[b] + xi * wr[b];
                }
                break;
            case OP_CZ:
                for (uint32_t x = 0; x < (1u << L); ++x)
                    if (bit(x, a) && bit(x, b)) { v[2 * x] = -v[2 * x]; v[2 * x + 1] = -v[2 * x + 1]; }
                break;
            case OP_PROJ: {
                int l = c ? int((branch >> b) & 1) : int(b);
                for (uint32_t x = 0; x < (1u << L); ++x)
                    if (bit(x, a) != l) { v[2 * x] = 0.f; v[2 * x + 1] = 0.f; }
                break;
            }
            case OP_ZB:
                if ((branch >> b) & 1)
                    for (uint32_t x = 0; x < (1u << L); ++x)
                        if (bit(x, a)) { v[2 * x] = -v[2 * x]; v[2 * x + 1] = -v[2 * x + 1]; }
                break;
            case OP_XCHG: {
                const uint64_t pw = P.ops[++pc];
                int perm[kMaxSlots];
                for (int s = 0; s < L; ++s) perm[s] = int((pw >> (4 * s)) & 0xf);
                for (uint32_t x = 0; x < (1u << L); ++x) {
                    uint32_t y = 0;  // old coordinate of the element that lands at x
                    for (int s = 0; s < L; ++s)
                        if ((x >> s) & 1) y |= 1u << perm[s];
                    w[2 * x] = v[2 * y];
                    w[2 * x + 1] = v[2 * y + 1];
                }
                v.swap(w);
                break;
            }
            case OP_SCALE:
                for (uint32_t x = 0; x < (1u << L); ++x) {
                    float xr = v[2 * x], xi = v[2 * x + 1];
                    v[2 * x] = xr * P.scale_re - xi * P.scale_im;
                    v[2 * x + 1] = xr * P.scale_im + xi * P.scale_re;
                }
                break;
            default:
                break;
            }
        }
        for (uint32_t x = 0; x < (1u << L); ++x) {
            uint64_t ad = addr(P.st_phys, x, bst);
            dst[2 * ad] = v[2 * x];
            dst[2 * ad + 1] = v[2 * x + 1];
        }
    }
    (void)N; (void)NT;
}

}  // namespace qsv
