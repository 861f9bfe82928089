// Host-side launchers of the HIP kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "qsv_internal.h"

namespace qsv {

// (R, T) of the generic tile kernel (every fused path)
bool fused_shape_supported(int R, int T);
// (R, T) of the compiled passes: the generic shapes plus tiles of 2^15
// amplitudes, whose exchanges only fit LDS staged in halves (one tile per
// workgroup; compiled passes only)
bool compiled_shape_supported(int R, int T);
hipError_t launch_fused(float2 *amps, int n, int R, int T, const PassProg &p, uint64_t branch,
                        hipStream_t s);
hipError_t launch_fused_batch(int R, int T, const BatchSeg *segs, int nseg, const BatchEntry *ents,
                              const PassProg *progs, int round, uint64_t blocks, int init_plus,
                              hipStream_t s);
// One persistent launch over every work item of a tile shape's rounds (see
// BatchRound).  resident != NULL: only report the workgroups the device holds
// at once (no launch).  abort: pinned host flag the waits poll; wait_us:
// longest wait of one work item before it gives up.
hipError_t launch_fused_persistent(int R, int T, const BatchRound *rounds, int nrounds, const BatchSeg *segs,
                                   uint64_t total, const BatchEntry *ents, const PassProg *progs, int init_plus,
                                   uint32_t *done, unsigned long long *next, uint32_t *err, const uint32_t *abort,
                                   uint32_t wait_us, unsigned grid, hipStream_t s, unsigned *resident);
hipError_t launch_zero_u32(uint32_t *p, uint64_t count, hipStream_t s);
hipError_t launch_gather_batch(const BatchEntry *ents, uint64_t count, const uint64_t *xs,
                               uint64_t m, float2 *out, hipStream_t s);
hipError_t launch_dense(float2 *amps, int n, int k, const int *qubits, const float *mat_t,
                        hipStream_t s);
hipError_t launch_plain_1q(float2 *amps, int n, int q, const float m[8], hipStream_t s);
hipError_t launch_plain_phase(float2 *amps, int n, int q, float cr, float ci, hipStream_t s);
hipError_t launch_plain_cz(float2 *amps, int n, int q0, int q1, hipStream_t s);
hipError_t launch_plain_zero(float2 *amps, int n, int q, int l, hipStream_t s);
hipError_t launch_init(float2 *amps, int n, int kind, uint64_t basis, hipStream_t s);
hipError_t launch_gather(const float2 *amps, int n, const uint64_t *xs, uint64_t m, void *out,
                         int c128, hipStream_t s);
hipError_t launch_gather_c128(const void *amps, int n, const uint64_t *xs, uint64_t m, void *out,
                              hipStream_t s);
// sets *flag (mapped host memory) when some xs[k] >= 2^n
hipError_t launch_check_range(const uint64_t *xs, uint64_t m, int n, unsigned int *flag, hipStream_t s);
hipError_t launch_norm(const float2 *amps, int n, double *out, double *partials, hipStream_t s);
// partial sums launch_norm writes for a state of 2^n amplitudes (at most 65536)
size_t norm_partial_count(int n);
// <a|b> in FP64 into out[0] (re), out[1] (im); partials: 2 * 65536 doubles
hipError_t launch_dot(const float2 *a, const float2 *b, int n, double *out, double *partials,
                      hipStream_t s);
// Full-state branch combine (combine.hip).  Local bit q of side A / B sits at
// global bit pos_a[q] / pos_b[q]; folded pair f couples local A bit fold_a[f]
// with local B bit fold_b[f].
// One block of the full-state combine: rows row_base + [0, 2^na_blk) of side
// A's local index and columns col_base + [0, 2^nb_blk) of side B's.  Branch
// b's rows start at A + a_off + b * a_stride (likewise for B); pos_a / pos_b
// map local bits (of the full local index) to output bits.
struct CombineArgs {
    int32_t na, nb, n_fold, pad;
    int32_t na_blk, nb_blk, pad2[2];
    uint64_t a_off, a_stride, b_off, b_stride, row_base, col_base;
    uint8_t pos_a[64], pos_b[64];
    uint8_t fold_a[64], fold_b[64];
};
// fp64: FP64 products and sums (else FP32 accumulation); out_c128: out is
// complex128 (else complex64)
hipError_t launch_combine_gemm(const float2 *A, const float2 *B, uint64_t nbr, const CombineArgs &P,
                               void *out, bool fp64, bool out_c128, hipStream_t s);
hipError_t launch_sum_partials(const double *part, uint64_t count, double *out, hipStream_t s);
// dst = src, bytes a multiple of 16, both 16-byte aligned
hipError_t launch_stream_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s);
hipError_t launch_branch_combine(const float2 *A, const float2 *B, uint64_t nb, uint64_t m,
                                 const int8_t *sign, double2 *out, hipStream_t s);

}  // namespace qsv
