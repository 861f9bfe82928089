// Full-state branch combine on matrix cores (Fig. 2, eq. (1); eqs. (6)-(7)):
//
//   Psi[x] = s(x) * sum_b A_b[x_A] B_b[x_B]
//
// for a circuit cut into sides A and B (circuit_split): x_A / x_B are the
// bits of x on the two sides, A_b / B_b the branch states of the halves and
// s(x) = (-1)^{sum over folded pairs x_a x_b}.  As matrices, Psi = Ahat Bhat^T
// with Ahat[x_A][b] = A_b[x_A], a complex GEMM of shape 2^nA x 2^nB x nb.  It
// runs as two real GEMMs over an interleaved K index k = 2b + part:
//   Mr = sum_k A1[k] B1[k],  A1 = (Ar, -Ai),  B1 = (Br, Bi)
//   Mi = sum_k A2[k] B1[k],  A2 = (Ai,  Ar)
// The default form sums the branch products in FP64: the FP32 inputs are
// widened and multiplied on v_mfma_f64_16x16x4f64, so every product is exact
// and every partial sum is an FP64 sum; the result is rounded once, to the
// complex64 state or not at all for a complex128 output.  The FP32 form
// (v_mfma_f32_16x16x4f32, FP32 accumulation) runs at twice the matrix-core
// rate and is selected explicitly.  A workgroup owns a 128 x 128 output tile:
// the FP32 form's four waves a 64 x 64 quadrant each (4 x 4 MFMA blocks for
// each of Mr, Mi), the FP64 form's eight waves a 64 x 32 part each (4 x 2
// blocks).  Branch chunks of 16 are staged in LDS as
// k-major planes; the next chunk's global loads are issued before the current
// chunk's MFMA work so that they overlap it.  The epilogue applies s(x) and
// scatters the tile to the state's natural index order through per-tile
// tables of the rows' and columns' output bits.  A launch covers one
// block of rows and columns (CombineArgs): the whole matrix for a two-part
// split, one value of the selector qubits for a three-part partition.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <type_traits>

#include "kernels.h"

namespace qsv {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;  // output rows (x_A) and columns (x_B) per workgroup
constexpr int kBr = 16;     // branches per LDS chunk
constexpr int kK = 2 * kBr; // interleaved K per chunk

// F64: FP64 products and sums on eight waves (each a 64 x 32 part of the
// tile: 128 accumulator registers per lane, so two waves share a SIMD and
// one's staging hides behind the other's matrix work); otherwise FP32
// accumulation on four waves (each a 64 x 64 quadrant; two workgroups per
// CU).  out_c128: the output state is complex128.
template <bool F64>
__global__ void __launch_bounds__(F64 ? 512 : 256, F64 ? 1 : 2)
k_combine_gemm(const float2 *__restrict__ A, const float2 *__restrict__ B, uint64_t nbr,
               const CombineArgs P, void *__restrict__ out, int out_c128) {
    using Acc = typename std::conditional<F64, v4d, v4f>::type;
    constexpr int NTH = F64 ? 512 : 256;  // threads
    constexpr int NC = F64 ? 2 : 4;       // 16-column blocks per wave
    __shared__ __attribute__((aligned(16))) float a1[kK][kTile];  // also the epilogue's 64-bit tables
    __shared__ float a2[kK][kTile], b1[kK][kTile];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint64_t i0 = uint64_t(blockIdx.x) * kTile, j0 = uint64_t(blockIdx.y) * kTile;
    // this wave's part: rows wr * 64 + [0, 64), columns wc * 16 NC + [0, 16 NC)
    const uint32_t wr = w & 1u, wc = w >> 1;
    const uint32_t lr = lane & 15u, lk = lane >> 4;
    Acc accr[4][NC], acci[4][NC];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            accr[m][c] = Acc{0, 0, 0, 0};
            acci[m][c] = Acc{0, 0, 0, 0};
        }
    // staging: thread t always loads in-tile row tr of branches tb, tb + BS,
    // ... of a chunk, so one pointer per side and a uniform stride address them
    constexpr int BS = NTH / kTile;          // branches staged at once
    constexpr int kPer = kBr * kTile / NTH;  // staged elements per thread and side
    static_assert(kTile == 128 && kPer * BS == kBr, "staging covers a chunk");
    const uint32_t tb = t >> 7, tr = t & 127u;
    const float2 *pa = A + P.a_off + tb * P.a_stride + i0 + tr;
    const float2 *pb = B + P.b_off + tb * P.b_stride + j0 + tr;
    const uint64_t sa = BS * P.a_stride, sb = BS * P.b_stride;
    float2 na_[kPer], nb_[kPer];
    auto fetch = [&](uint64_t b0) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            na_[q] = make_float2(0.f, 0.f);
            nb_[q] = make_float2(0.f, 0.f);
            if (b0 + tb + BS * q < nbr) {
                na_[q] = pa[q * sa];
                nb_[q] = pb[q * sb];
            }
        }
        pa += kBr * P.a_stride;
        pb += kBr * P.b_stride;
    };
    fetch(0);
    for (uint64_t b0 = 0; b0 < nbr; b0 += kBr) {
        __syncthreads();  // previous chunk's fragments are read
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const uint32_t b = tb + BS * q;
            a1[2 * b][tr] = na_[q].x;
            a1[2 * b + 1][tr] = -na_[q].y;
            a2[2 * b][tr] = na_[q].y;
            a2[2 * b + 1][tr] = na_[q].x;
            b1[2 * b][tr] = nb_[q].x;
            b1[2 * b + 1][tr] = nb_[q].y;
        }
        __syncthreads();
        if (b0 + kBr < nbr) fetch(b0 + kBr);  // in flight during the MFMA work
#pragma unroll
        for (int ks = 0; ks < kK; ks += 4) {
            float fa1[4], fa2[4], fb[NC];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                fa1[m] = a1[ks + lk][wr * 64 + m * 16 + lr];
                fa2[m] = a2[ks + lk][wr * 64 + m * 16 + lr];
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) fb[c] = b1[ks + lk][wc * 16 * NC + c * 16 + lr];
            if constexpr (F64) {
                double da1[4], da2[4], db[NC];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    da1[m] = double(fa1[m]);
                    da2[m] = double(fa2[m]);
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) db[c] = double(fb[c]);
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        accr[m][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(da1[m], db[c], accr[m][c], 0, 0, 0);
                        acci[m][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(da2[m], db[c], acci[m][c], 0, 0, 0);
                    }
            } else {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        accr[m][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa1[m], fb[c], accr[m][c], 0, 0, 0);
                        acci[m][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa2[m], fb[c], acci[m][c], 0, 0, 0);
                    }
            }
        }
    }
    // epilogue: block (m, c) element r of this lane is row 4*lk + r (FP32
    // accumulators) or row 4*r + lk (FP64 accumulators), column lr.
    // The output bits of the tile's 128 rows and 128 columns and the sign mask
    // of each row are tabulated once in the (now free) LDS staging area.
    __syncthreads();  // last chunk's fragments are read
    uint64_t *rowx = reinterpret_cast<uint64_t *>(&a1[0][0]);
    uint64_t *rowf = rowx + kTile;
    uint64_t *colx = rowf + kTile;
    if (t < 256) {
        const uint32_t k = t & 127u;
        if (t < 128) {
            const uint64_t i = P.row_base + i0 + k;
            uint64_t x = 0, f = 0;
            for (int q = 0; q < P.na; ++q)
                if ((i >> q) & 1ull) x |= 1ull << P.pos_a[q];
            for (int g = 0; g < P.n_fold; ++g)
                if ((i >> P.fold_a[g]) & 1ull) f ^= 1ull << P.fold_b[g];
            rowx[k] = x;
            rowf[k] = f;
        } else {
            const uint64_t j = P.col_base + j0 + k;
            uint64_t x = 0;
            for (int q = 0; q < P.nb; ++q)
                if ((j >> q) & 1ull) x |= 1ull << P.pos_b[q];
            colx[k] = x;
        }
    }
    __syncthreads();
    const uint64_t j0b = P.col_base + j0;
    uint64_t xb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xb[c] = colx[wc * 16 * NC + c * 16 + lr];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t il = wr * 64 + m * 16 + (F64 ? 4 * r + lk : 4 * lk + r);
            const uint64_t xa = rowx[il], fm = rowf[il] & j0b;
            const uint32_t fl = uint32_t(rowf[il]) & 127u;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const uint32_t jl = wc * 16 * NC + c * 16 + lr;
                const bool neg = ((__popcll(fm) + __popc(fl & jl)) & 1) != 0;
                double vr = double(accr[m][c][r]), vi = double(acci[m][c][r]);
                if (neg) { vr = -vr; vi = -vi; }
                if (out_c128) static_cast<double2 *>(out)[xa | xb[c]] = make_double2(vr, vi);
                else static_cast<float2 *>(out)[xa | xb[c]] = make_float2(float(vr), float(vi));
            }
        }
    }
}

// Leading local bits of a side that land on output bits 0, 1, 2, ... in order.
static int low_run(const uint8_t *pos, int n) {
    int k = 0;
    while (k < n && pos[k] == k) ++k;
    return k;
}

}  // namespace

// The 16 lanes of an accumulator row hold 16 consecutive columns, so the
// epilogue's stores are contiguous when the column side carries the lowest
// output bits: the product is symmetric in the two sides (A_b B_b = B_b A_b,
// the sign is symmetric), so the sides are exchanged when side A holds the
// longer run of low output bits.
hipError_t launch_combine_gemm(const float2 *A, const float2 *B, uint64_t nbr, const CombineArgs &P,
                               void *out, bool fp64, bool out_c128, hipStream_t s) {
    CombineArgs Q = P;
    const float2 *X = A, *Y = B;
    if (low_run(P.pos_a, P.na) > low_run(P.pos_b, P.nb) && P.na_blk <= 22) {
        X = B;
        Y = A;
        Q.na = P.nb; Q.nb = P.na;
        Q.na_blk = P.nb_blk; Q.nb_blk = P.na_blk;
        Q.a_off = P.b_off; Q.b_off = P.a_off;
        Q.a_stride = P.b_stride; Q.b_stride = P.a_stride;
        Q.row_base = P.col_base; Q.col_base = P.row_base;
        std::memcpy(Q.pos_a, P.pos_b, sizeof(Q.pos_a));
        std::memcpy(Q.pos_b, P.pos_a, sizeof(Q.pos_b));
        std::memcpy(Q.fold_a, P.fold_b, sizeof(Q.fold_a));
        std::memcpy(Q.fold_b, P.fold_a, sizeof(Q.fold_b));
    }
    const dim3 grid(unsigned(1ull << (Q.na_blk - 7)), unsigned(1ull << (Q.nb_blk - 7)));
    if (fp64) hipLaunchKernelGGL(k_combine_gemm<true>, grid, dim3(512), 0, s, X, Y, nbr, Q, out, out_c128 ? 1 : 0);
    else hipLaunchKernelGGL(k_combine_gemm<false>, grid, dim3(256), 0, s, X, Y, nbr, Q, out, out_c128 ? 1 : 0);
    return hipGetLastError();
}

}  // namespace qsv
