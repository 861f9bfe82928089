// Runtime specialisation of fused passes (hipRTC); see jit.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

// Kernel variants: bit 2 set -> the first pass generates the initial state
// of kind (variant & 3) instead of loading it; bit 3 set -> the last pass
// writes the FP64 norm partial of every tile.
constexpr int kJitPlain = 0;
constexpr int kJitInit = 4;
constexpr int kJitNorm = 8;
constexpr int kJitDouble = 16;  // complex128 state (validation instantiation)
constexpr int kJitBatched = 32; // state and branch per blockIdx.y from a batch entry table
constexpr int kJitLoop = 64;    // persistent workgroups, next tile prefetched into registers
constexpr int kJitPerPass = 128; // pass p persistent iff bit (8 + p) of the variant (p < 19)
constexpr int kJitPassBits = 19;
constexpr int kJitWhole = 1 << 27; // one tile per workgroup, exchanges staged whole (not in halves)
constexpr int kJitTiles = 1 << 28;  // with kJitSample: the listed tiles are stored whole instead
constexpr int kJitSample = 1 << 29; // the last pass runs only listed tiles and writes listed amplitudes
constexpr int kJitDot = 1 << 30; // the last pass stores nothing: FP64 <result|other> partials per tile
inline bool jit_pass_loop(int variant, size_t p) {
    if (variant & kJitLoop) return true;
    return (variant & kJitPerPass) && p < size_t(kJitPassBits) && ((variant >> (8 + p)) & 1);
}

// HIP source of every pass of the plan as kernels qsv_pass_<p>.
std::string jit_source(const Plan &plan, std::vector<size_t> *lds_bytes, int variant);
// Compile (cached by source text and device) and attach the kernels to plan.
qsv_status jit_prepare(Plan &plan, int variant);
// Launch all passes of a prepared plan on stream s.  src0 (optional): the
// first pass reads this state instead of amps, which it leaves unchanged.
// kJitDot variants: the last pass reads dot_other at its store addresses and
// writes the FP64 partials of <result|other> to part (re of every tile, then
// im of every tile) instead of storing the result.
// kJitSample | kJitTiles: the last pass runs the listed tiles and stores each
// of them whole into sample_out (a state) instead of writing amplitudes.
// kJitSample variants: the last pass runs sample_tiles workgroups over the
// tile list of the device table sample_tab and writes the listed amplitudes
// to sample_out (complex64) instead of storing the state.  With sample_rows
// > 1 its grid has that many rows of sibling branches: row y samples branch
// `branch` with the bits of y deposited on the set bits of `basis`, and
// writes at sample_out + y * sample_stride (the earlier passes, if any, run
// for `branch` only, so callers use rows with one-pass plans).
// max_tiles > 0: each pass runs only its first max_tiles tiles (timing).
struct SampleTab {  // device layout read by the sampling pass
    const uint64_t *tiles;   // tile index of workgroup b
    const uint32_t *start;   // entries of workgroup b: [start[b], start[b + 1])
    const uint64_t *xs;      // output index of each entry
    const uint32_t *slot;    // position of each entry in the output array
};
qsv_status jit_launch(const Plan &plan, int variant, void *amps, void *scratch, uint64_t branch,
                      uint64_t basis, double *part, hipStream_t s,
                      std::vector<float> *pass_ms = nullptr, const void *src0 = nullptr,
                      const void *dot_other = nullptr, const SampleTab *sample_tab = nullptr,
                      uint64_t sample_tiles = 0, void *sample_out = nullptr, uint64_t sample_rows = 1,
                      uint64_t sample_stride = 0, uint64_t max_tiles = 0);
// Launch all passes over `count` batch entries (BatchEntry table on the device).
qsv_status jit_launch_batched(const Plan &plan, int variant, const void *ents, unsigned count,
                              hipStream_t s);
// Compile without loading (no device needed).
qsv_status jit_compile_only(const Plan &plan, size_t *code_bytes, double *seconds);
double jit_total_compile_seconds();

}  // namespace qsv
