// HIP kernels of the state-vector sweep for gfx950 (MI355X), and their
// host-side launchers.
//
// State: 2^n complex64 amplitudes, interleaved (re, im) float32, qubit k =
// index bit k (Section 2, preliminaries).  All kernels use 64-bit indices
// (2^34 amplitudes exceed 32 bits).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "kernels.h"

namespace qsv {
namespace {

__device__ __forceinline__ float2 f2(float x, float y) { return make_float2(x, y); }

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

// e^{i pi k / 4}, k = 0..7
__constant__ float c_wr[8] = {1.f, 0.70710678118654752f, 0.f, -0.70710678118654752f,
                              -1.f, -0.70710678118654752f, 0.f, 0.70710678118654752f};
__constant__ float c_wi[8] = {0.f, 0.70710678118654752f, 1.f, 0.70710678118654752f,
                              0.f, -0.70710678118654752f, -1.f, -0.70710678118654752f};

// ---------------------------------------------------------------------------
// Register-slot primitives.  v[j] holds the amplitude whose register-slot
// bits are j; slot S pairs v[j] with v[j | 2^S].
// ---------------------------------------------------------------------------

template <int S, int N> __device__ __forceinline__ void bf_h(float2 (&v)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j & (1 << S)) continue;
        const float2 x = v[j], y = v[j | (1 << S)];
        v[j] = f2(x.x + y.x, x.y + y.y);
        v[j | (1 << S)] = f2(x.x - y.x, x.y - y.y);
    }
}
template <int S, int N> __device__ __forceinline__ void bf_sx(float2 (&v)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j & (1 << S)) continue;
        const float2 x = v[j], y = v[j | (1 << S)];
        v[j] = f2(x.x + y.y, x.y - y.x);            // x - i y
        v[j | (1 << S)] = f2(y.x + x.y, y.y - x.x); // y - i x
    }
}
template <int S, int N> __device__ __forceinline__ void bf_sy(float2 (&v)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j & (1 << S)) continue;
        const float2 x = v[j], y = v[j | (1 << S)];
        v[j] = f2(x.x - y.x, x.y - y.y);
        v[j | (1 << S)] = f2(x.x + y.x, x.y + y.y);
    }
}
template <int S, int N> __device__ __forceinline__ void bf_sxdg(float2 (&v)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j & (1 << S)) continue;
        const float2 x = v[j], y = v[j | (1 << S)];
        v[j] = f2(x.x - y.y, x.y + y.x);            // x + i y
        v[j | (1 << S)] = f2(y.x - x.y, y.y + x.x); // y + i x
    }
}
template <int S, int N> __device__ __forceinline__ void bf_sydg(float2 (&v)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j & (1 << S)) continue;
        const float2 x = v[j], y = v[j | (1 << S)];
        v[j] = f2(x.x + y.x, x.y + y.y);
        v[j | (1 << S)] = f2(y.x - x.x, y.y - x.y);
    }
}
__device__ __forceinline__ float2 cmul(float2 a, float cr, float ci) {
    return f2(a.x * cr - a.y * ci, a.x * ci + a.y * cr);
}
// multiply amplitudes with slot bit S = 1 by (cr, ci)
template <int S, int N> __device__ __forceinline__ void ph_slot(float2 (&v)[N], float cr, float ci) {
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (j & (1 << S)) v[j] = cmul(v[j], cr, ci);
}
template <int S, int N> __device__ __forceinline__ void neg_slot(float2 (&v)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (j & (1 << S)) v[j] = f2(-v[j].x, -v[j].y);
}
template <int S1, int S2, int N> __device__ __forceinline__ void neg_slot2(float2 (&v)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j)
        if ((j & (1 << S1)) && (j & (1 << S2))) v[j] = f2(-v[j].x, -v[j].y);
}
// zero amplitudes whose slot bit S differs from l
template <int S, int N> __device__ __forceinline__ void proj_slot(float2 (&v)[N], int l) {
    if (l) {
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (!(j & (1 << S))) v[j] = f2(0.f, 0.f);
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (j & (1 << S)) v[j] = f2(0.f, 0.f);
    }
}

// Dispatch a runtime register-slot index to a compile-time template.  The
// last slot is the default so that every path of the switch computes: an
// empty path would make the register allocator copy the whole amplitude
// array at the merge.
#define QSV_SLOT_DISPATCH(s, CALL)                                                  \
    switch (s) {                                                                    \
    case 0: if constexpr (R - 1 > 0) { constexpr int S_ = 0; CALL; break; } [[fallthrough]]; \
    case 1: if constexpr (R - 1 > 1) { constexpr int S_ = 1; CALL; break; } [[fallthrough]]; \
    case 2: if constexpr (R - 1 > 2) { constexpr int S_ = 2; CALL; break; } [[fallthrough]]; \
    case 3: if constexpr (R - 1 > 3) { constexpr int S_ = 3; CALL; break; } [[fallthrough]]; \
    case 4: if constexpr (R - 1 > 4) { constexpr int S_ = 4; CALL; break; } [[fallthrough]]; \
    default: { constexpr int S_ = R - 1; CALL; } break;                             \
    }

// negate amplitudes with slot bit S = 1 when m has the sign bit set
template <int S, int N> __device__ __forceinline__ void xneg_slot(float2 (&v)[N], uint32_t m) {
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (j & (1 << S))
            v[j] = f2(__uint_as_float(__float_as_uint(v[j].x) ^ m),
                      __uint_as_float(__float_as_uint(v[j].y) ^ m));
}
// zero amplitudes whose slot bit S differs from l (branch-free)
template <int S, int N> __device__ __forceinline__ void proj_sel(float2 (&v)[N], uint32_t l) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const bool z = (uint32_t((j >> S) & 1) != l);
        v[j] = z ? f2(0.f, 0.f) : v[j];
    }
}
template <int R, int S1, int N>
__device__ __forceinline__ void cz_reg_reg(float2 (&v)[N], uint32_t s2) {
    // the slot pair is distinct by construction; S1 == S2 cannot occur
    QSV_SLOT_DISPATCH(s2, (neg_slot2<S1, S_, N>(v)));
}

// ---------------------------------------------------------------------------
// Fused tile pass (generic: interprets a pass program).
//
// One workgroup of 2^T threads owns one tile of 2^(R+T) amplitudes: slot
// coordinate x = j | t << R (j = register index, t = thread index) sits at
// physical index base | sum_{s: x_s = 1} 2^{phys[s]}.  Loads and stores are
// 16-byte (two amplitudes: register slot 0 is physical bit 0) and the thread
// slots 0..c-2 hold physical bits 1..c-1, so each wave access is made of
// contiguous runs of 2^c amplitudes.  XCHG permutes slot bits through LDS
// (write at padded old coordinate, read at padded new coordinate; one pad
// element per 2^R keeps the 64 lanes of a wave on distinct banks).
// Diagonal gates whose qubit is a thread or tile-index bit multiply every
// amplitude of a thread by the same power of w = e^{i pi/4}: they only add to
// the per-thread exponent e, applied before an XCHG (when the op says so) and
// by the closing SCALE.
// init: 0 = load the tile, 1 = every amplitude = init_val (|+>^n).
// ---------------------------------------------------------------------------
template <int R, int T>
__device__ __forceinline__ void fused_tile(float2 *__restrict__ amps, const PassProg &P,
                                           uint64_t branch, uint64_t tile, int init,
                                           float init_val, float2 *lds) {
    constexpr int N = 1 << R;
    const uint32_t t = threadIdx.x;

    uint64_t base = 0;  // tile origin in the map the pass reads
    for (int i = 0; i < P.n_glob; ++i) base |= ((tile >> i) & 1ull) << P.glob_bits[i];

    float2 v[N];
    if (init) {
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = f2(init_val, 0.f);
    } else {
        uint64_t toff = 0;
#pragma unroll
        for (int u = 0; u < T; ++u)
            if ((t >> u) & 1u) toff |= 1ull << P.ld_phys[R + u];
        const float2 *src = amps + (base | toff);
#pragma unroll
        for (int j = 0; j < N; j += 2) {
            uint64_t roff = 0;
#pragma unroll
            for (int s = 1; s < R; ++s)
                if ((j >> s) & 1) roff |= 1ull << P.ld_phys[s];
            const v4f w = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(src + roff));
            v[j] = f2(w.x, w.y);
            v[j + 1] = f2(w.z, w.w);
        }
    }

    auto pred = [&](uint32_t loc) -> uint32_t {
        if (loc & 0x80u) return uint32_t((base >> (loc & 0x7fu)) & 1ull);
        return (t >> (loc - R)) & 1u;
    };
    uint32_t e = 0, alive = 1;

    int pc = 0;
    do {
        const uint64_t op = P.ops[pc];
        const uint32_t code = uint32_t(op) & 0xffu;
        const uint32_t a = uint32_t(op >> 8) & 0xffu;
        const uint32_t b = uint32_t(op >> 16) & 0xffu;
        const uint32_t c = uint32_t(op >> 24) & 0xffu;
        switch (code) {
        case 1: QSV_SLOT_DISPATCH(a, (bf_h<S_, N>(v))); break;
        case 2: QSV_SLOT_DISPATCH(a, (bf_sx<S_, N>(v))); break;
        case 3: QSV_SLOT_DISPATCH(a, (bf_sy<S_, N>(v))); break;
        case 4: QSV_SLOT_DISPATCH(a, (bf_sxdg<S_, N>(v))); break;
        case 5: QSV_SLOT_DISPATCH(a, (bf_sydg<S_, N>(v))); break;
        case 8: {  // PHASE
            if (a < uint32_t(R)) {
                const float cr = c_wr[b], ci = c_wi[b];
                QSV_SLOT_DISPATCH(a, (ph_slot<S_, N>(v, cr, ci)));
            } else {
                e += pred(a) * b;
            }
            break;
        }
        case 9: {  // CZ
            uint32_t x = a, y = b;
            if (x >= uint32_t(R) && y < uint32_t(R)) { uint32_t tmp = x; x = y; y = tmp; }
            if (x < uint32_t(R) && y < uint32_t(R)) {
                QSV_SLOT_DISPATCH(x, (cz_reg_reg<R, S_, N>(v, y)));
            } else if (x < uint32_t(R)) {
                const uint32_t m = pred(y) << 31;
                QSV_SLOT_DISPATCH(x, (xneg_slot<S_, N>(v, m)));
            } else {
                e += (pred(x) & pred(y)) * 4u;
            }
            break;
        }
        case 10: {  // PROJ
            const uint32_t l = c ? uint32_t((branch >> b) & 1ull) : b;
            if (a < uint32_t(R)) {
                QSV_SLOT_DISPATCH(a, (proj_sel<S_, N>(v, l)));
            } else {
                alive &= uint32_t(pred(a) == l);
            }
            break;
        }
        case 11: {  // ZB
            const uint32_t bit = uint32_t((branch >> b) & 1ull);
            if (a < uint32_t(R)) {
                QSV_SLOT_DISPATCH(a, (xneg_slot<S_, N>(v, bit << 31)));
            } else {
                e += (bit & pred(a)) * 4u;
            }
            break;
        }
        case 12: {  // XCHG: new slot s takes old slot perm[s]
            const uint64_t pw = P.ops[++pc];
            {   // phases accumulated on thread/tile bits are applied first
                // (unconditionally: a skipped path would cost a full copy of v)
                const float fr = alive ? c_wr[e & 7u] : 0.f, fi = alive ? c_wi[e & 7u] : 0.f;
#pragma unroll
                for (int j = 0; j < N; ++j) v[j] = cmul(v[j], fr, fi);
                e = 0;
                alive = 1;
                (void)c;
            }
            __syncthreads();  // earlier reads of LDS are complete
            const uint32_t wt = (t << R) + t;  // padded old coordinate of (t, 0)
#pragma unroll
            for (int j = 0; j < N; ++j) lds[wt + j] = v[j];
            uint32_t yt = 0;
#pragma unroll
            for (int u = 0; u < T; ++u)
                if ((t >> u) & 1u) yt |= 1u << ((pw >> (4 * (R + u))) & 0xf);
            const uint32_t rt = yt + (yt >> R);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < N; ++j) {
                uint32_t yj = 0;
#pragma unroll
                for (int s = 0; s < R; ++s)
                    if ((j >> s) & 1) yj |= 1u << ((pw >> (4 * s)) & 0xf);
                v[j] = lds[rt + yj + (yj >> R)];
            }
            break;
        }
        default: {  // SCALE (closes every program): pass scale x w^e x alive
            const float wr = alive ? c_wr[e & 7u] : 0.f, wi = alive ? c_wi[e & 7u] : 0.f;
            const float cr = P.scale_re * wr - P.scale_im * wi;
            const float ci = P.scale_re * wi + P.scale_im * wr;
#pragma unroll
            for (int j = 0; j < N; ++j) v[j] = cmul(v[j], cr, ci);
            e = 0;
            alive = 1;
            break;
        }
        }
    } while (++pc < P.n_ops);

    {
        uint64_t bst = 0;  // tile origin in the map the pass writes
        for (int i = 0; i < P.n_glob; ++i) bst |= ((tile >> i) & 1ull) << P.glob_st[i];
        uint64_t toff = 0;
#pragma unroll
        for (int u = 0; u < T; ++u)
            if ((t >> u) & 1u) toff |= 1ull << P.st_phys[R + u];
        float2 *dst = amps + (bst | toff);
#pragma unroll
        for (int j = 0; j < N; j += 2) {
            uint64_t roff = 0;
#pragma unroll
            for (int s = 1; s < R; ++s)
                if ((j >> s) & 1) roff |= 1ull << P.st_phys[s];
            const v4f w = {v[j].x, v[j].y, v[j + 1].x, v[j + 1].y};
            __builtin_nontemporal_store(w, reinterpret_cast<v4f *>(dst + roff));
        }
    }
}

template <int R, int T>
__global__ void __launch_bounds__(1 << T)
k_fused(float2 *__restrict__ amps, const PassProg P, uint64_t branch, uint64_t tile0) {
    extern __shared__ float2 lds[];
    fused_tile<R, T>(amps, P, branch, tile0 + blockIdx.x, 0, 0.f, lds);
}

// One pass round of a batch: block b belongs to the segment with the largest
// start <= b; the segment names the entry (state, branch, program) and the
// first tile.  Entries whose round is their first pass may generate |+>^n.
template <int R, int T>
__global__ void __launch_bounds__(1 << T)
k_fused_batch(const BatchSeg *__restrict__ segs, int nseg, const BatchEntry *__restrict__ ents,
              const PassProg *__restrict__ progs, int round, int init_plus) {
    extern __shared__ float2 lds[];
    const uint64_t blk = blockIdx.x;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {  // last segment with start <= blk
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].start <= blk) lo = mid; else hi = mid - 1;
    }
    const BatchSeg sg = segs[lo];
    const BatchEntry en = ents[sg.entry];
    const PassProg &P = progs[en.prog0 + round];
    const int init = (init_plus && round == 0) ? 1 : 0;
    fused_tile<R, T>(reinterpret_cast<float2 *>(en.amps), P, en.branch, blk - sg.start, init,
                     en.init_val, lds);
}

// Persistent form of a batch's generic tile passes: one launch for every
// pass round of every entry of one tile shape.  Workgroups take work items
// (round, entry, tile) in order from *next (batch_decode); an item of round
// r > 0 first waits until done[entry] reaches r * tiles(entry), i.e. until
// every tile of the entry's earlier passes is stored.  The device has one L2
// per XCD, so the counters are updated and polled with system-scope atomics
// (performed past the XCD caches), a tile's stores are written back
// (system-scope release fence of every wave) before its entry's counter is
// raised, and the waiting workgroup invalidates its caches (acquire fence)
// once the counter has reached its target, before any wave loads.  Every
// wait is bounded in time: after wait_ticks ticks of the constant-rate
// device clock, or when the host sets *abort (pinned host memory, polled
// every 256 tries), the workgroup records the failure in *err and goes on,
// so the launch always drains within a bounded time.
template <int R, int T>
__global__ void __launch_bounds__(1 << T)
k_fused_persistent(const BatchRound *__restrict__ rounds, int nrounds, const BatchSeg *__restrict__ segs,
                   uint64_t total, const BatchEntry *__restrict__ ents, const PassProg *__restrict__ progs,
                   int init_plus, uint32_t *done, unsigned long long *next, uint32_t *err,
                   const volatile uint32_t *abort, uint64_t wait_ticks) {
    extern __shared__ float2 lds[];
    __shared__ unsigned long long item_s;
    constexpr int L = R + T;
    for (;;) {
        if (threadIdx.x == 0)
            item_s = __hip_atomic_fetch_add(next, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __syncthreads();
        const uint64_t item = item_s;
        __syncthreads();  // every wave has the item before it is overwritten
        if (item >= total) break;
        int r = 0;
        uint32_t e = 0;
        uint64_t tile = 0;
        batch_decode(rounds, nrounds, segs, item, &r, &e, &tile);
        const BatchEntry en = ents[e];
        if (r > 0) {
            if (threadIdx.x == 0) {
                const uint32_t need = uint32_t(r) << (en.n - L);
                const uint64_t t0 = wall_clock64();
                for (uint32_t k = 1;
                     __hip_atomic_load(done + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) < need; ++k) {
                    if (wall_clock64() - t0 > wait_ticks || ((k & 255u) == 0 && *abort)) {
                        __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __syncthreads();
            __atomic_thread_fence(__ATOMIC_ACQUIRE);  // system scope: drop stale cached lines
        }
        fused_tile<R, T>(reinterpret_cast<float2 *>(en.amps), progs[en.prog0 + r], en.branch, tile,
                         (init_plus && r == 0) ? 1 : 0, en.init_val, lds);
        __threadfence_system();  // this wave's stores are written back
        __syncthreads();         // ... for every wave of the tile
        if (threadIdx.x == 0) __hip_atomic_fetch_add(done + e, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Clears the counters of a persistent batch launch (a kernel, not a memset:
// it is replayed inside the batch's graph).
__global__ void __launch_bounds__(256) k_zero_u32(uint32_t *__restrict__ p, uint64_t count) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0u;
}

// Gather for every entry of a batch: out[e*m + k] = amps_e[xs[e*m + k]].
__global__ void __launch_bounds__(256)
k_gather_batch(const BatchEntry *__restrict__ ents, uint64_t count, const uint64_t *__restrict__ xs,
               uint64_t m, float2 *__restrict__ out) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count * m) return;
    const BatchEntry en = ents[i / m];
    const uint64_t x = xs[i];
    const float2 *a = reinterpret_cast<const float2 *>(en.amps);
    out[i] = (x < (1ull << en.n)) ? a[x] : f2(__builtin_nanf(""), __builtin_nanf(""));
}


// ---------------------------------------------------------------------------
// Dense block on matrix cores: Y = M X for a 2^K x 2^K complex matrix M on K
// qubits.  A tile is 2^K rows (the block's qubits) x 64 columns (the six
// lowest other index bits); the remaining bits select the tile.  Persistent
// workgroups keep M^T (re, im) in LDS and loop over tiles: load the tile into
// LDS as separate re/im planes, form Yr = Mr Xr - Mi Xi and Yi = Mr Xi + Mi Xr
// with v_mfma_f32_16x16x4_f32 (four real products; wave w owns 16-row output
// blocks), write Y back through LDS and store it in place.
// ---------------------------------------------------------------------------
struct DenseArgs {
    uint64_t tiles;
    uint8_t glob_bits[48];     // tile index bit i -> physical bit
    uint8_t phys[16];          // tile local bit i -> physical bit
    uint8_t sub[16];           // position of local bit i within the row or column index
    uint8_t sub_row[8];        // row index bit b -> tile local bit
    uint8_t sub_col[8];        // column index bit b -> tile local bit
    uint16_t rowmask;          // local bits that belong to the row index
    int32_t n_glob;
};

template <int K>
__global__ void __launch_bounds__(256)
k_dense(float2 *__restrict__ amps, const float *__restrict__ mat_t, const DenseArgs A) {
    constexpr int DIM = 1 << K;
    constexpr int COLS = 64;
    constexpr int XS = COLS + 4;             // padded row stride of the X planes
    constexpr int PER = (DIM * COLS) / 256;  // elements per thread
    constexpr int NB = DIM / 16;             // 16x16 output blocks per wave
    __shared__ float mtr[DIM * DIM], mti[DIM * DIM];
    __shared__ float xr[DIM * XS], xi[DIM * XS];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    for (uint32_t i = t; i < uint32_t(DIM * DIM); i += 256) {
        mtr[i] = mat_t[i];
        mti[i] = mat_t[DIM * DIM + i];
    }
    // thread part of the tile-local index: bits 0..7
    uint64_t poff_t = 0;
    uint32_t row_t = 0, col_t = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (!((t >> b) & 1u)) continue;
        poff_t |= 1ull << A.phys[b];
        if ((A.rowmask >> b) & 1u) row_t |= 1u << A.sub[b];
        else col_t |= 1u << A.sub[b];
    }
    const uint32_t rb0 = (w * NB) / 4;       // row block of this wave
    const uint32_t cb0 = (w * NB) % 4;       // first column block
    for (uint64_t tile = blockIdx.x; tile < A.tiles; tile += gridDim.x) {
        uint64_t base = 0;
        for (int i = 0; i < A.n_glob; ++i) base |= ((tile >> i) & 1ull) << A.glob_bits[i];
        __syncthreads();  // previous tile's LDS reads are complete
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            uint64_t poff = poff_t;
            uint32_t row = row_t, col = col_t;
#pragma unroll
            for (int b = 8; b < K + 6; ++b) {
                if (!((it >> (b - 8)) & 1)) continue;
                poff |= 1ull << A.phys[b];
                if ((A.rowmask >> b) & 1u) row |= 1u << A.sub[b];
                else col |= 1u << A.sub[b];
            }
            const float2 v = amps[base | poff];
            xr[row * XS + col] = v.x;
            xi[row * XS + col] = v.y;
        }
        __syncthreads();
        v4f ar[NB], ai[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) { ar[b] = v4f{0, 0, 0, 0}; ai[b] = v4f{0, 0, 0, 0}; }
        const uint32_t lr = lane & 15u, lk = lane >> 4;
#pragma unroll 4
        for (int kk = 0; kk < DIM; kk += 4) {
            const float a_r = mtr[(kk + lk) * DIM + rb0 * 16 + lr];
            const float a_i = mti[(kk + lk) * DIM + rb0 * 16 + lr];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const uint32_t cb = cb0 + b;
                const float b_r = xr[(kk + lk) * XS + cb * 16 + lr];
                const float b_i = xi[(kk + lk) * XS + cb * 16 + lr];
                ar[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_r, b_r, ar[b], 0, 0, 0);
                ar[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a_i, b_i, ar[b], 0, 0, 0);
                ai[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_r, b_i, ai[b], 0, 0, 0);
                ai[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_i, b_r, ai[b], 0, 0, 0);
            }
        }
        __syncthreads();  // all waves are done reading X
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint32_t cb = cb0 + b;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t row = rb0 * 16 + 4 * lk + r, col = cb * 16 + lr;
                xr[row * XS + col] = ar[b][r];
                xi[row * XS + col] = ai[b][r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            uint64_t poff = poff_t;
            uint32_t row = row_t, col = col_t;
#pragma unroll
            for (int b = 8; b < K + 6; ++b) {
                if (!((it >> (b - 8)) & 1)) continue;
                poff |= 1ull << A.phys[b];
                if ((A.rowmask >> b) & 1u) row |= 1u << A.sub[b];
                else col |= 1u << A.sub[b];
            }
            amps[base | poff] = f2(xr[row * XS + col], xi[row * XS + col]);
        }
    }
}

// Dense block for k = 6, 7: Y = M X with the 2^k x 2^k matrix M held in
// registers.  Wave w of a workgroup owns output rows [16 w, 16 w + 16) (its
// strip of Mr and Mi, 2^k / 2 registers per lane, loaded once) and computes
// them for a tile of 64 columns: Yr = Mr Xr - Mi Xi and Yi = Mr Xi + Mi Xr on
// v_mfma_f32_16x16x4f32 (FP32 accumulation; the two products of Yi of a
// block are issued four instructions apart).  A tile is 2^(k+6) amplitudes whose
// local index bits are its physical bits from the lowest up (the block's k
// qubits and the 6 lowest other qubits; physical bit 0 is always among
// them), so thread t's 16-byte accesses at local indices 2 (i NT + t) are
// contiguous across a wave whatever the block's qubits.  Loads go to
// registers, then to LDS planes (re, im) at each element's (row, column):
// element (r, c) at 80 r + r / 4 + c (a stride of 80 puts the 4 rows one
// MFMA operand read covers on distinct bank groups; the extra r / 4 spreads
// rows that differ in their higher bits, as when the block holds the lowest
// qubits and a wave's lanes walk its rows, over distinct banks, and is a
// constant per operand read).  The results go back through the same planes
// and leave in the same physical order (16-byte stores from every lane:
// faster than storing the accumulators' 8-byte elements directly, even
// where 16 lanes would write 16 consecutive amplitudes).  Persistent workgroups walk the tiles;
// the next tile's loads are issued before the current tile's matrix-core work.
template <int K>
__global__ void __launch_bounds__(64 * (1 << K) / 16, K == 6 ? 2 : 1)
k_dense_strip(float2 *__restrict__ amps, const float *__restrict__ mat_t, const DenseArgs A) {
    constexpr int DIM = 1 << K;
    constexpr int WAVES = DIM / 16;
    constexpr int NT = 64 * WAVES;          // threads
    constexpr int COLS = 64;
    constexpr int XS = 80;                   // row stride of the X planes (floats)
    constexpr int KS = DIM / 4;              // k-steps of 4
    constexpr int PAIRS = DIM * COLS / 2;    // amplitude pairs of a tile
    constexpr int PER = PAIRS / NT;          // pairs per thread (8)
    static_assert(PER * NT == PAIRS, "tile split");
    constexpr int PLANE = DIM * XS + DIM / 4;
    __shared__ float xr[PLANE], xi[PLANE];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint32_t lr = lane & 15u, lk = lane >> 4;
    auto at = [](uint32_t row, uint32_t col) { return row * XS + (row >> 2) + col; };
    // this wave's strip of M: A operand of k-step ks, lane (k % 4) * 16 + i
    float mr[KS], mi[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const uint32_t k = uint32_t(ks) * 4u + lk, row = w * 16u + lr;
        mr[ks] = mat_t[k * DIM + row];
        mi[ks] = mat_t[DIM * DIM + k * DIM + row];
    }
    // pair it of this thread: local index l = 2 (it NT + t).  Bits 1..TB of
    // l come from t and the higher ones from it, so its physical offset and
    // its (row, column) are the OR of a per-thread part and a part common to
    // the workgroup; l + 1 is the next amplitude in memory and differs in
    // local bit 0 (a row or a column bit).
    constexpr int TB = K + 2;  // log2(NT)
    static_assert((1 << TB) == NT && (PER << TB) == PAIRS, "pair index split");
    uint64_t off_t = 0;
    uint32_t row_t = 0, col_t = 0;
#pragma unroll
    for (int b = 1; b <= TB; ++b) {
        if (!((t >> (b - 1)) & 1u)) continue;
        off_t |= 1ull << A.phys[b];
        if ((A.rowmask >> b) & 1u) row_t |= 1u << A.sub[b];
        else col_t |= 1u << A.sub[b];
    }
    auto off_it = [&](int it) {
        uint64_t o = 0;
#pragma unroll
        for (int b = TB + 1; b < K + 6; ++b)
            if ((it >> (b - TB - 1)) & 1) o |= 1ull << A.phys[b];
        return o;
    };
    auto rc_it = [&](int it, uint32_t &row, uint32_t &col) {
        row = row_t;
        col = col_t;
#pragma unroll
        for (int b = TB + 1; b < K + 6; ++b) {
            if (!((it >> (b - TB - 1)) & 1)) continue;
            if ((A.rowmask >> b) & 1u) row |= 1u << A.sub[b];
            else col |= 1u << A.sub[b];
        }
    };
    const bool b0row = (A.rowmask & 1u) != 0;
    const uint32_t b0 = 1u << A.sub[0];
    v4f nx[PER];
    auto tile_base = [&](uint64_t tile) {
        uint64_t base = 0;
        for (int i = 0; i < A.n_glob; ++i) base |= ((tile >> i) & 1ull) << A.glob_bits[i];
        return base;
    };
    auto fetch = [&](uint64_t tile) {
        const uint64_t base = tile_base(tile);
#pragma unroll
        for (int it = 0; it < PER; ++it)
            nx[it] = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(amps + (base | off_t | off_it(it))));
    };
    uint64_t tile = blockIdx.x;
    if (tile < A.tiles) fetch(tile);
    for (; tile < A.tiles; tile += gridDim.x) {
        const uint64_t base = tile_base(tile);
        __syncthreads();  // the previous tile's LDS reads are complete
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            uint32_t row, col;
            rc_it(it, row, col);
            const uint32_t p0 = at(row, col), p1 = b0row ? at(row | b0, col) : at(row, col | b0);
            xr[p0] = nx[it].x;
            xi[p0] = nx[it].y;
            xr[p1] = nx[it].z;
            xi[p1] = nx[it].w;
        }
        __syncthreads();
        if (tile + gridDim.x < A.tiles) fetch(tile + gridDim.x);  // in flight during the MFMA work
        v4f arr[4], aii[4], ai[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            arr[c] = v4f{0, 0, 0, 0};
            aii[c] = arr[c];
            ai[c] = arr[c];
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const uint32_t krow = uint32_t(ks) * 4u + lk;
            float br[4], bi[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                br[c] = xr[at(krow, uint32_t(c) * 16u + lr)];
                bi[c] = xi[at(krow, uint32_t(c) * 16u + lr)];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) ai[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(mr[ks], bi[c], ai[c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                arr[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(mr[ks], br[c], arr[c], 0, 0, 0);
                aii[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(mi[ks], bi[c], aii[c], 0, 0, 0);
                ai[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(mi[ks], br[c], ai[c], 0, 0, 0);
            }
        }
        // element r of block c: row 16 w + 4 lk + r, column 16 c + lr
        __syncthreads();  // every wave's operand reads of X are complete
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t p = at(w * 16u + 4u * lk + uint32_t(r), uint32_t(c) * 16u + lr);
                xr[p] = arr[c][r] - aii[c][r];
                xi[p] = ai[c][r];
            }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            uint32_t row, col;
            rc_it(it, row, col);
            const uint32_t p0 = at(row, col), p1 = b0row ? at(row | b0, col) : at(row, col | b0);
            const v4f y = {xr[p0], xi[p0], xr[p1], xi[p1]};
            __builtin_nontemporal_store(y, reinterpret_cast<v4f *>(amps + (base | off_t | off_it(it))));
        }
    }
}

template <int K>
hipError_t launch_dense_strip_t(float2 *amps, const float *mat_t, const DenseArgs &A, hipStream_t s) {
    constexpr int NT = 64 * (1 << K) / 16;
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(&k_dense_strip<K>), NT, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const uint64_t resident = uint64_t(std::max(1, per_cu)) * uint64_t(std::max(1, cus));
    const uint64_t grid = A.tiles < resident ? A.tiles : resident;
    hipLaunchKernelGGL((k_dense_strip<K>), dim3(unsigned(grid)), dim3(NT), 0, s, amps, mat_t, A);
    return hipGetLastError();
}

template <int K>
hipError_t launch_dense_t(float2 *amps, int n, const int *qubits, const float *mat_t,
                          hipStream_t s) {
    DenseArgs A;
    std::memset(&A, 0, sizeof(A));
    uint64_t qmask = 0;
    for (int i = 0; i < K; ++i) qmask |= 1ull << qubits[i];
    // column bits: the six lowest bits outside the block
    uint64_t cmask = 0;
    for (int q = 0, c = 0; q < n && c < 6; ++q)
        if (!((qmask >> q) & 1)) { cmask |= 1ull << q; ++c; }
    const uint64_t res = qmask | cmask;
    int li = 0, ri = 0, ci = 0;
    for (int q = 0; q < n; ++q) {
        if (!((res >> q) & 1)) continue;
        A.phys[li] = uint8_t(q);
        if ((qmask >> q) & 1) {
            A.rowmask |= uint16_t(1u << li);
            // row index bit = position of q in the block's qubit list
            int pos = 0;
            while (qubits[pos] != q) ++pos;
            A.sub[li] = uint8_t(pos);
            ++ri;
        } else {
            A.sub[li] = uint8_t(ci++);
        }
        ++li;
    }
    int g = 0;
    for (int q = 0; q < n; ++q)
        if (!((res >> q) & 1)) A.glob_bits[g++] = uint8_t(q);
    A.n_glob = g;
    A.tiles = 1ull << (n - K - 6);
    (void)ri;
    for (int l = 0; l < K + 6; ++l) {
        if ((A.rowmask >> l) & 1u) A.sub_row[A.sub[l]] = uint8_t(l);
        else A.sub_col[A.sub[l]] = uint8_t(l);
    }
    if constexpr (K >= 6) {
        return launch_dense_strip_t<K>(amps, mat_t, A, s);
    } else {
        const uint64_t grid = A.tiles < 1024 ? A.tiles : 1024;
        hipLaunchKernelGGL((k_dense<K>), dim3(unsigned(grid)), dim3(256), 0, s, amps, mat_t, A);
        return hipGetLastError();
    }
}

// ---------------------------------------------------------------------------
// Plain (unfused) gate kernels: one launch per gate.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t insert_zero(uint64_t i, int q) {
    const uint64_t lo = i & ((1ull << q) - 1);
    return ((i >> q) << (q + 1)) | lo;
}

// General single-qubit gate, pair rule of Section 2 (preliminaries).
__global__ void __launch_bounds__(256)
k_plain_1q(float2 *__restrict__ a, uint64_t pairs, int q, float m0r, float m0i, float m1r,
           float m1i, float m2r, float m2i, float m3r, float m3i) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < pairs; i += stride) {
        const uint64_t lo = insert_zero(i, q), hi = lo | (1ull << q);
        const float2 x = a[lo], y = a[hi];
        a[lo] = f2(m0r * x.x - m0i * x.y + m1r * y.x - m1i * y.y,
                   m0r * x.y + m0i * x.x + m1r * y.y + m1i * y.x);
        a[hi] = f2(m2r * x.x - m2i * x.y + m3r * y.x - m3i * y.y,
                   m2r * x.y + m2i * x.x + m3r * y.y + m3i * y.x);
    }
}

// Multiply amplitudes with bit q = 1 by (cr, ci): touches half the state.
__global__ void __launch_bounds__(256)
k_plain_phase(float2 *__restrict__ a, uint64_t count, int q, float cr, float ci) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t k = insert_zero(i, q) | (1ull << q);
        a[k] = cmul(a[k], cr, ci);
    }
}

// Negate amplitudes with bits q0 and q1 set (q0 < q1): a quarter of the state.
__global__ void __launch_bounds__(256)
k_plain_cz(float2 *__restrict__ a, uint64_t count, int q0, int q1) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t k = insert_zero(insert_zero(i, q0), q1) | (1ull << q0) | (1ull << q1);
        const float2 x = a[k];
        a[k] = f2(-x.x, -x.y);
    }
}

// Zero amplitudes whose bit q is != l (projector P_l): write-only, half the state.
__global__ void __launch_bounds__(256)
k_plain_zero(float2 *__restrict__ a, uint64_t count, int q, int l) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t k = insert_zero(i, q) | (uint64_t(1 - l) << q);
        a[k] = f2(0.f, 0.f);
    }
}

// ---------------------------------------------------------------------------
// Initialisation, gather, norm, branch combine.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_init(v4f *__restrict__ a, uint64_t quads, float val, int kind, uint64_t basis) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < quads; i += stride) {
        v4f w;
        if (kind == 1) {
            w = v4f{val, 0.f, val, 0.f};
        } else {
            w = v4f{0.f, 0.f, 0.f, 0.f};
            if ((basis >> 1) == i) {
                if (basis & 1) w.z = 1.f; else w.x = 1.f;
            }
        }
        __builtin_nontemporal_store(w, a + i);
    }
}

__global__ void __launch_bounds__(256)
k_init_small(float2 *__restrict__ a, uint64_t dim, float val, int kind, uint64_t basis) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= dim) return;
    if (kind == 1) a[i] = f2(val, 0.f);
    else a[i] = f2(i == basis ? 1.f : 0.f, 0.f);
}

__global__ void __launch_bounds__(256)
k_gather(const float2 *__restrict__ a, uint64_t dim, const uint64_t *__restrict__ xs, uint64_t m,
         void *__restrict__ out, int c128) {
    const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint64_t x = xs[k];
    float2 v;
    if (x < dim) v = a[x];
    else v = f2(__builtin_nanf(""), __builtin_nanf(""));
    if (c128) reinterpret_cast<double2 *>(out)[k] = make_double2(double(v.x), double(v.y));
    else reinterpret_cast<float2 *>(out)[k] = v;
}

// Range check of device bitstrings: raises *flag (mapped host memory) when
// some xs[k] >= dim.  Grid-stride; the flag is only ever set, never read here.
__global__ void __launch_bounds__(256)
k_check_range(const uint64_t *__restrict__ xs, uint64_t m, uint64_t dim, unsigned int *flag) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    bool bad = false;
    for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < m; k += stride) bad = bad || xs[k] >= dim;
    if (bad) __hip_atomic_fetch_or(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(256)
k_gather_c128(const double2 *__restrict__ a, uint64_t dim, const uint64_t *__restrict__ xs,
              uint64_t m, double2 *__restrict__ out) {
    const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint64_t x = xs[k];
    out[k] = (x < dim) ? a[x] : make_double2(__builtin_nan(""), __builtin_nan(""));
}

// Block b sums |a_i|^2 over its contiguous chunk in FP64 (products of FP32
// values are exact in FP64); fixed thread-then-tree order.
__global__ void __launch_bounds__(256)
k_norm_partial(const float4 *__restrict__ a, uint64_t quads_per_block, double *__restrict__ part) {
    __shared__ double s[256];
    const uint64_t start = uint64_t(blockIdx.x) * quads_per_block;
    double acc = 0.0;
    for (uint64_t i = threadIdx.x; i < quads_per_block; i += 256) {
        const float4 w = a[start + i];
        const double x0 = w.x, y0 = w.y, x1 = w.z, y1 = w.w;
        acc += (x0 * x0 + y0 * y0) + (x1 * x1 + y1 * y1);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Sum of count partials by one block of 1024 threads: each thread keeps
// eight independent accumulators over a fixed strided subset, then a fixed
// tree over the threads.
__global__ void __launch_bounds__(1024)
k_sum_partials(const double *__restrict__ part, uint64_t count, double *__restrict__ out) {
    __shared__ double s[1024];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t i = threadIdx.x;
    for (; i + 7 * 1024 < count; i += 8 * 1024) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += part[i + k * 1024];
    }
    for (int k = 0; i < count; i += 1024, ++k) acc[k & 7] += part[i];
    s[threadIdx.x] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// <a|b> = sum conj(a_i) b_i with FP64 products of the FP32 inputs (exact),
// same fixed-order tree as the norm: per-block partials (re at part[blk],
// im at part[nblk + blk]), then k_sum_partials on each half.
__global__ void __launch_bounds__(256)
k_dot_partial(const float4 *__restrict__ a, const float4 *__restrict__ b, uint64_t quads_per_block,
              double *__restrict__ part) {
    __shared__ double sr[256], si[256];
    const uint64_t start = uint64_t(blockIdx.x) * quads_per_block;
    double ar = 0.0, ai = 0.0;
    for (uint64_t i = threadIdx.x; i < quads_per_block; i += 256) {
        const float4 x = a[start + i], y = b[start + i];
        const double x0 = x.x, x1 = x.y, x2 = x.z, x3 = x.w;
        const double y0 = y.x, y1 = y.y, y2 = y.z, y3 = y.w;
        ar += (x0 * y0 + x1 * y1) + (x2 * y2 + x3 * y3);
        ai += (x0 * y1 - x1 * y0) + (x2 * y3 - x3 * y2);
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            sr[threadIdx.x] += sr[threadIdx.x + h];
            si[threadIdx.x] += si[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sr[0];
        part[gridDim.x + blockIdx.x] = si[0];
    }
}

__global__ void __launch_bounds__(256)
k_dot_small(const float2 *__restrict__ a, const float2 *__restrict__ b, uint64_t dim,
            double *__restrict__ out) {
    __shared__ double sr[256], si[256];
    double ar = 0.0, ai = 0.0;
    for (uint64_t i = threadIdx.x; i < dim; i += 256) {
        const double x0 = a[i].x, x1 = a[i].y, y0 = b[i].x, y1 = b[i].y;
        ar += x0 * y0 + x1 * y1;
        ai += x0 * y1 - x1 * y0;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            sr[threadIdx.x] += sr[threadIdx.x + h];
            si[threadIdx.x] += si[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sr[0];
        out[1] = si[0];
    }
}

__global__ void __launch_bounds__(256)
k_norm_small(const float2 *__restrict__ a, uint64_t dim, double *__restrict__ out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (uint64_t i = threadIdx.x; i < dim; i += 256) {
        const double x = a[i].x, y = a[i].y;
        acc += x * x + y * y;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// out[x] = sign[x] * sum_b A[b][x] * B[b][x]: 64 outputs per block, four
// branch groups of 64 lanes each; FP64 products and sums, fixed order.
__global__ void __launch_bounds__(256)
k_branch_combine(const float2 *__restrict__ A, const float2 *__restrict__ B, uint64_t nb,
                 uint64_t m, const int8_t *__restrict__ sign, double2 *__restrict__ out) {
    __shared__ double sr[4][64], si[4][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const uint64_t x = uint64_t(blockIdx.x) * 64 + lane;
    double ar = 0.0, ai = 0.0;
    if (x < m) {
        for (uint64_t b = grp; b < nb; b += 4) {
            const float2 p = A[b * m + x], q = B[b * m + x];
            const double pr = p.x, pi = p.y, qr = q.x, qi = q.y;
            ar += pr * qr - pi * qi;
            ai += pr * qi + pi * qr;
        }
    }
    sr[grp][lane] = ar;
    si[grp][lane] = ai;
    __syncthreads();
    if (grp == 0 && x < m) {
        double r = (sr[0][lane] + sr[1][lane]) + (sr[2][lane] + sr[3][lane]);
        double i = (si[0][lane] + si[1][lane]) + (si[2][lane] + si[3][lane]);
        if (sign && sign[x] < 0) { r = -r; i = -i; }
        out[x] = make_double2(r, i);
    }
}

// Streaming copy with the sweep's access pattern (16-byte nontemporal loads
// and stores, 8 in flight per thread): the HBM rate a pass that does no
// arithmetic would reach, the ceiling the fused passes are compared with.
__global__ void __launch_bounds__(256)
k_stream_copy(const v4f *__restrict__ src, v4f *__restrict__ dst, uint64_t count) {
    constexpr int U = 8;
    const uint64_t stride = uint64_t(gridDim.x) * 256u * U;
    for (uint64_t base = uint64_t(blockIdx.x) * 256u * U + threadIdx.x; base < count; base += stride) {
        v4f w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + uint64_t(u) * 256u;
            if (i < count) w[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + uint64_t(u) * 256u;
            if (i < count) __builtin_nontemporal_store(w[u], dst + i);
        }
    }
}

unsigned grid_for(uint64_t work, unsigned per_block = 256, unsigned cap = 1u << 20) {
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

template <int R, int T>
hipError_t launch_fused_t(float2 *amps, int n, const PassProg &p, uint64_t branch, hipStream_t s) {
    constexpr int L = R + T;
    const size_t lds = (size_t(1) << L) * sizeof(float2) + (size_t(1) << T) * sizeof(float2);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused<R, T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const uint64_t tiles = 1ull << (n - L);
    const uint64_t chunk = 1ull << 30;  // blocks per launch
    for (uint64_t t0 = 0; t0 < tiles; t0 += chunk) {
        const uint64_t cnt = (tiles - t0 < chunk) ? tiles - t0 : chunk;
        hipLaunchKernelGGL((k_fused<R, T>), dim3(unsigned(cnt)), dim3(1 << T), lds, s, amps, p,
                           branch, t0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int R, int T>
hipError_t launch_fused_batch_t(const BatchSeg *segs, int nseg, const BatchEntry *ents,
                                const PassProg *progs, int round, uint64_t blocks, int init_plus,
                                hipStream_t s) {
    constexpr int L = R + T;
    const size_t lds = (size_t(1) << L) * sizeof(float2) + (size_t(1) << T) * sizeof(float2);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused_batch<R, T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (blocks == 0) return hipSuccess;
    if (blocks > (1ull << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_fused_batch<R, T>), dim3(unsigned(blocks)), dim3(1 << T), lds, s, segs,
                       nseg, ents, progs, round, init_plus);
    return hipGetLastError();
}

template <int R, int T>
hipError_t launch_fused_persistent_t(const BatchRound *rounds, int nrounds, const BatchSeg *segs, uint64_t total,
                                     const BatchEntry *ents, const PassProg *progs, int init_plus, uint32_t *done,
                                     unsigned long long *next, uint32_t *err, const uint32_t *abort,
                                     uint32_t wait_us, unsigned grid, hipStream_t s, unsigned *resident) {
    constexpr int L = R + T;
    const size_t lds = (size_t(1) << L) * sizeof(float2) + (size_t(1) << T) * sizeof(float2);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused_persistent<R, T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (resident) {  // workgroups the device holds at once
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_fused_persistent<R, T>), 1 << T, lds);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        *resident = unsigned(std::max(1, per_cu) * std::max(1, cus));
        return hipSuccess;
    }
    if (total == 0 || grid == 0) return hipSuccess;
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    const uint64_t wait_ticks = uint64_t(wait_us) * uint64_t(khz > 0 ? khz : 100000) / 1000u;
    hipLaunchKernelGGL((k_fused_persistent<R, T>), dim3(grid), dim3(1 << T), lds, s, rounds, nrounds, segs, total,
                       ents, progs, init_plus, done, next, err, reinterpret_cast<const volatile uint32_t *>(abort),
                       wait_ticks);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_persistent(int R, int T, const BatchRound *rounds, int nrounds, const BatchSeg *segs,
                                   uint64_t total, const BatchEntry *ents, const PassProg *progs, int init_plus,
                                   uint32_t *done, unsigned long long *next, uint32_t *err, const uint32_t *abort,
                                   uint32_t wait_us, unsigned grid, hipStream_t s, unsigned *resident) {
#define QSV_PERSIST(RR, TT)                                                                                     \
    case RR * 16 + TT:                                                                                          \
        return launch_fused_persistent_t<RR, TT>(rounds, nrounds, segs, total, ents, progs, init_plus, done, next, \
                                                 err, abort, wait_us, grid, s, resident);
    switch (R * 16 + T) {
        QSV_PERSIST(5, 9)
        QSV_PERSIST(5, 8)
        QSV_PERSIST(4, 8)
        QSV_PERSIST(5, 7)
        QSV_PERSIST(4, 7)
    default: return hipErrorInvalidValue;
    }
#undef QSV_PERSIST
}

hipError_t launch_zero_u32(uint32_t *p, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(count, 256, 1024)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_fused_batch(int R, int T, const BatchSeg *segs, int nseg, const BatchEntry *ents,
                              const PassProg *progs, int round, uint64_t blocks, int init_plus,
                              hipStream_t s) {
    switch (R * 16 + T) {
    case 5 * 16 + 8: return launch_fused_batch_t<5, 8>(segs, nseg, ents, progs, round, blocks, init_plus, s);
    case 4 * 16 + 8: return launch_fused_batch_t<4, 8>(segs, nseg, ents, progs, round, blocks, init_plus, s);
    case 5 * 16 + 7: return launch_fused_batch_t<5, 7>(segs, nseg, ents, progs, round, blocks, init_plus, s);
    case 4 * 16 + 7: return launch_fused_batch_t<4, 7>(segs, nseg, ents, progs, round, blocks, init_plus, s);
    case 5 * 16 + 9: return launch_fused_batch_t<5, 9>(segs, nseg, ents, progs, round, blocks, init_plus, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather_batch(const BatchEntry *ents, uint64_t count, const uint64_t *xs,
                               uint64_t m, float2 *out, hipStream_t s) {
    if (count * m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_batch, dim3(unsigned((count * m + 255) / 256)), dim3(256), 0, s,
                       ents, count, xs, m, out);
    return hipGetLastError();
}

hipError_t launch_dense(float2 *amps, int n, int k, const int *qubits, const float *mat_t,
                        hipStream_t s) {
    switch (k) {
    case 4: return launch_dense_t<4>(amps, n, qubits, mat_t, s);
    case 5: return launch_dense_t<5>(amps, n, qubits, mat_t, s);
    case 6: return launch_dense_t<6>(amps, n, qubits, mat_t, s);
    case 7: return launch_dense_t<7>(amps, n, qubits, mat_t, s);
    default: return hipErrorInvalidValue;
    }
}

bool fused_shape_supported(int R, int T) {
    switch (R * 16 + T) {
    case 5 * 16 + 8: case 5 * 16 + 7: case 4 * 16 + 7: case 4 * 16 + 6: case 3 * 16 + 6:
    case 3 * 16 + 4: case 2 * 16 + 3: case 4 * 16 + 8: case 6 * 16 + 8: case 5 * 16 + 9:
    case 4 * 16 + 9: case 6 * 16 + 7:
        return true;
    default:
        return false;
    }
}

bool compiled_shape_supported(int R, int T) { return fused_shape_supported(R, T) || (R == 6 && T == 9); }

hipError_t launch_fused(float2 *amps, int n, int R, int T, const PassProg &p, uint64_t branch,
                        hipStream_t s) {
    switch (R * 16 + T) {
    case 5 * 16 + 8: return launch_fused_t<5, 8>(amps, n, p, branch, s);
    case 5 * 16 + 7: return launch_fused_t<5, 7>(amps, n, p, branch, s);
    case 4 * 16 + 7: return launch_fused_t<4, 7>(amps, n, p, branch, s);
    case 4 * 16 + 6: return launch_fused_t<4, 6>(amps, n, p, branch, s);
    case 3 * 16 + 6: return launch_fused_t<3, 6>(amps, n, p, branch, s);
    case 3 * 16 + 4: return launch_fused_t<3, 4>(amps, n, p, branch, s);
    case 2 * 16 + 3: return launch_fused_t<2, 3>(amps, n, p, branch, s);
    case 4 * 16 + 8: return launch_fused_t<4, 8>(amps, n, p, branch, s);
    case 6 * 16 + 8: return launch_fused_t<6, 8>(amps, n, p, branch, s);
    case 5 * 16 + 9: return launch_fused_t<5, 9>(amps, n, p, branch, s);
    case 4 * 16 + 9: return launch_fused_t<4, 9>(amps, n, p, branch, s);
    case 6 * 16 + 7: return launch_fused_t<6, 7>(amps, n, p, branch, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_plain_1q(float2 *amps, int n, int q, const float m[8], hipStream_t s) {
    const uint64_t pairs = 1ull << (n - 1);
    hipLaunchKernelGGL(k_plain_1q, dim3(grid_for(pairs)), dim3(256), 0, s, amps, pairs, q, m[0],
                       m[1], m[2], m[3], m[4], m[5], m[6], m[7]);
    return hipGetLastError();
}

hipError_t launch_plain_phase(float2 *amps, int n, int q, float cr, float ci, hipStream_t s) {
    const uint64_t cnt = 1ull << (n - 1);
    hipLaunchKernelGGL(k_plain_phase, dim3(grid_for(cnt)), dim3(256), 0, s, amps, cnt, q, cr, ci);
    return hipGetLastError();
}

hipError_t launch_plain_cz(float2 *amps, int n, int q0, int q1, hipStream_t s) {
    if (q0 > q1) { int t = q0; q0 = q1; q1 = t; }
    const uint64_t cnt = 1ull << (n - 2);
    hipLaunchKernelGGL(k_plain_cz, dim3(grid_for(cnt)), dim3(256), 0, s, amps, cnt, q0, q1);
    return hipGetLastError();
}

hipError_t launch_plain_zero(float2 *amps, int n, int q, int l, hipStream_t s) {
    const uint64_t cnt = 1ull << (n - 1);
    hipLaunchKernelGGL(k_plain_zero, dim3(grid_for(cnt)), dim3(256), 0, s, amps, cnt, q, l);
    return hipGetLastError();
}

hipError_t launch_init(float2 *amps, int n, int kind, uint64_t basis, hipStream_t s) {
    const uint64_t dim = 1ull << n;
    const float val = float(1.0 / __builtin_sqrt(double(dim)));
    if (n >= 1) {
        const uint64_t quads = dim / 2;
        hipLaunchKernelGGL(k_init, dim3(grid_for(quads)), dim3(256), 0, s,
                           reinterpret_cast<v4f *>(amps), quads, val, kind, basis);
    } else {
        hipLaunchKernelGGL(k_init_small, dim3(1), dim3(256), 0, s, amps, dim, val, kind, basis);
    }
    return hipGetLastError();
}

hipError_t launch_gather(const float2 *amps, int n, const uint64_t *xs, uint64_t m, void *out,
                         int c128, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(m, 256, 1u << 30)), dim3(256), 0, s, amps,
                       1ull << n, xs, m, out, c128);
    return hipGetLastError();
}

hipError_t launch_check_range(const uint64_t *xs, uint64_t m, int n, unsigned int *flag, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_range, dim3(grid_for(m, 256, 1024)), dim3(256), 0, s, xs, m, 1ull << n, flag);
    return hipGetLastError();
}

hipError_t launch_gather_c128(const void *amps, int n, const uint64_t *xs, uint64_t m, void *out,
                              hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_c128, dim3(grid_for(m, 256, 1u << 30)), dim3(256), 0, s,
                       static_cast<const double2 *>(amps), 1ull << n, xs, m, static_cast<double2 *>(out));
    return hipGetLastError();
}

size_t norm_partial_count(int n) {
    if (n < 14) return 0;
    // log2(blocks) so that each block has 1024 quads, at most 65536 blocks
    const int lb = n - 1 - 10 > 16 ? 16 : n - 1 - 10;
    return size_t(1) << lb;
}

hipError_t launch_norm(const float2 *amps, int n, double *out, double *partials, hipStream_t s) {
    const uint64_t dim = 1ull << n;
    if (n < 14) {
        hipLaunchKernelGGL(k_norm_small, dim3(1), dim3(256), 0, s, amps, dim, out);
        return hipGetLastError();
    }
    // at most 65536 blocks; each block a contiguous chunk of >= 1024 quads
    const unsigned blocks = unsigned(norm_partial_count(n));
    const int lb = __builtin_ctz(blocks);
    const uint64_t qpb = (dim / 2) >> lb;
    hipLaunchKernelGGL(k_norm_partial, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(amps), qpb, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, partials, uint64_t(blocks), out);
    return hipGetLastError();
}

hipError_t launch_dot(const float2 *a, const float2 *b, int n, double *out, double *partials,
                      hipStream_t s) {
    const uint64_t dim = 1ull << n;
    if (n < 14) {
        hipLaunchKernelGGL(k_dot_small, dim3(1), dim3(256), 0, s, a, b, dim, out);
        return hipGetLastError();
    }
    int lb = n - 1 - 10;  // blocks of 1024 quads, at most 65536 blocks
    if (lb > 16) lb = 16;
    const unsigned blocks = 1u << lb;
    const uint64_t qpb = (dim / 2) >> lb;
    hipLaunchKernelGGL(k_dot_partial, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const float4 *>(a),
                       reinterpret_cast<const float4 *>(b), qpb, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, partials, uint64_t(blocks), out);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, partials + blocks, uint64_t(blocks),
                       out + 1);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s) {
    const uint64_t count = bytes / 16;
    if (count == 0) return hipSuccess;
    // 8 workgroups of 256 threads per CU on 256 CUs, each thread 8 x 16 B in flight
    const uint64_t per_block = 256u * 8u;
    uint64_t grid = (count + per_block - 1) / per_block;
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(k_stream_copy, dim3(unsigned(grid)), dim3(256), 0, s, static_cast<const v4f *>(src),
                       static_cast<v4f *>(dst), count);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, uint64_t count, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, part, count, out);
    return hipGetLastError();
}

hipError_t launch_branch_combine(const float2 *A, const float2 *B, uint64_t nb, uint64_t m,
                                 const int8_t *sign, double2 *out, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_branch_combine, dim3(unsigned((m + 63) / 64)), dim3(256), 0, s, A, B, nb,
                       m, sign, out);
    return hipGetLastError();
}

}  // namespace qsv
