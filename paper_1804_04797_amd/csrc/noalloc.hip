// The FP64 norm without any allocation: sv_norm_fp64_noalloc.
//
// sv_norm_fp64 reduces into a partial-sum buffer that the library allocates
// per device and stream on first use.  Callers that cannot allocate (code
// under graph capture, loops that forbid hipMalloc) use this variant instead:
// its partial sums live in a fixed file-scope device array, one copy per GPU,
// held for the life of the process.  Its address on each device is looked up
// once (hipGetSymbolAddress, with that device current) and only that address
// is passed to the kernels; the array's name in host code is not a device
// address.  Calls on one device share the array, so calls that overlap on
// one device race; every call writes all the partials it reads, so nothing
// needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kernels.h"
#include "qsv_internal.h"

namespace qsv {
namespace {

// The norm of a state of 2^n amplitudes uses min(2^(n - 11), 65536)
// partials (one per block of 1024 quads); states below 2^14 amplitudes use
// none.
constexpr size_t kNoallocPartials = 65536;

static __device__ __align__(256) double scratch[kNoallocPartials];

std::mutex g_mu;
double *g_addr[64] = {nullptr};

qsv_status scratch_address(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(QSV_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(QSV_EUNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QSV_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_addr[dev] = static_cast<double *>(p);
    }
    *out = g_addr[dev];
    return QSV_OK;
}

}  // namespace
}  // namespace qsv

using namespace qsv;

extern "C" qsv_status sv_norm_fp64_noalloc(const void *amps, int n_qubits, double *out_dev, void *stream) {
    if (!amps || !out_dev) return fail(QSV_EINVAL, "sv_norm_fp64_noalloc: null argument");
    if (n_qubits < 0 || n_qubits > kMaxQubits) return fail(QSV_ERANGE, "sv_norm_fp64_noalloc: n_qubits must be in 0..34");
    if (reinterpret_cast<uintptr_t>(amps) % 16 != 0)
        return fail(QSV_EINVAL, "sv_norm_fp64_noalloc: state pointer must be 16-byte aligned");
    if (norm_partial_count(n_qubits) > kNoallocPartials)
        return fail(QSV_ERANGE, "sv_norm_fp64_noalloc: the state needs more partial sums than the fixed array holds");
    qsv_status st = check_gfx950();
    if (st != QSV_OK) return st;
    double *part = nullptr;
    if ((st = scratch_address(&part)) != QSV_OK) return st;
    hipError_t e = launch_norm(static_cast<const float2 *>(amps), n_qubits, out_dev, part,
                               static_cast<hipStream_t>(stream));
    return e == hipSuccess ? QSV_OK : fail(QSV_EHIP, std::string("sv_norm_fp64_noalloc: ") + hipGetErrorString(e));
}
