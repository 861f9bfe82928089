// Runtime specialisation of fused passes (hipRTC); see jit.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

// HIP source of every pass of the plan as kernels qsv_pass_<p>.
std::string jit_source(const Plan &plan, std::vector<size_t> *lds_bytes);
// Compile (cached by source text and device) and attach the kernels to plan.
qsv_status jit_prepare(Plan &plan);
// Launch all passes of a prepared plan on stream s.
qsv_status jit_launch(const Plan &plan, void *amps, uint64_t branch, hipStream_t s);
// Compile without loading (no device needed).
qsv_status jit_compile_only(const Plan &plan, size_t *code_bytes, double *seconds);
double jit_total_compile_seconds();

}  // namespace qsv
