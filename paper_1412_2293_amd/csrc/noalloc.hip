// Allocation-free fidelity: the overlap reductions of qs_fidelity with their partial sums in a
// fixed device array of this library instead of a handle's scratch, so that a caller which
// cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc) can form <a|b>, <a|a> and <b|b> of two state vectors it owns.
//
// The array is a file-scope device variable: every GPU the library runs on holds one copy until
// the process ends.  Its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is passed to kernels and copies; the variable's
// name in host code is a host-side stand-in, not a device address.  Every call on one GPU uses
// the same array, so calls that overlap on one GPU (on different streams, or from different
// host threads) race; calls on one stream are ordered.  The reduction kernels write every
// partial they read, so nothing needs clearing between calls.
#include <mutex>

#include "internal.h"

namespace qs {

// Partial sums of two overlap reductions of one slot each (red_log_blocks caps the blocks per
// slot at 2^9, three doubles each, and the density-matrix form at four), then the two 5-double
// outputs of the final sums.
constexpr size_t kNoAllocPartials = 2048;
constexpr size_t kNoAllocDoubles = kNoAllocPartials + 16;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static double *g_noalloc_ptr[kNoAllocMaxDevices] = {};

// The device address of this device's copy of `scratch` (looked up on first use per device).
static hipError_t noalloc_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_noalloc_ptr[dev] = (double *)p;
    }
    *out = g_noalloc_ptr[dev];
    return hipSuccess;
}

// out[0..1] = <a|b>, out[2] = <a|a>, out[3] = <b|b>, from the two reductions' outputs (each
// 5 doubles: Re, Im of the overlap with the reference, the state's squared norm, and the
// marked amplitude, unused here).
__global__ void k_noalloc_pack(const double *red, double *out)
{
    if (threadIdx.x == 0) {
        out[0] = red[0];
        out[1] = red[1];
        out[2] = red[5 + 2];
        out[3] = red[2];
    }
}

}  // namespace qs

using namespace qs;

extern "C" qs_status qs_fidelity_noalloc(const void *a_dev, const void *b_dev, int n_qubits, qs_dtype dt,
                                         void *hip_stream, double *out_dev)
{
    clear_error();
    if (!a_dev || !b_dev || !out_dev) return fail(QS_EINVAL, "fidelity_noalloc: NULL pointer");
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_EINVAL, "fidelity_noalloc: unknown dtype");
    if (n_qubits < 1 || n_qubits > 34)
        return fail(QS_EINVAL, "fidelity_noalloc: n_qubits must be in 1..34 (the fixed scratch holds the "
                               "partials of states up to 34 qubits)");
    if (reduce_partials_doubles(n_qubits, 1) > kNoAllocPartials)
        return fail(QS_EINVAL, "fidelity_noalloc: the reduction needs more than the " +
                                   std::to_string(kNoAllocPartials) + " doubles of the fixed scratch");
    double *sc = nullptr;
    hipError_t e = noalloc_scratch(&sc);
    if (e != hipSuccess) return hip_fail(e, "fidelity_noalloc: scratch address");
    hipStream_t st = (hipStream_t)hip_stream;
    double *red = sc + kNoAllocPartials;
    // the same reductions, in the same order, as qs_fidelity: <a|b> with b's norm, then <a|a>
    QS_HIP(launch_overlaps(a_dev, 0, b_dev, dt, n_qubits, 1, -1, sc, red, st));
    QS_HIP(launch_overlaps(a_dev, 0, a_dev, dt, n_qubits, 1, -1, sc, red + 5, st));
    hipLaunchKernelGGL(k_noalloc_pack, dim3(1), dim3(64), 0, st, red, out_dev);
    QS_HIP(hipGetLastError());
    return QS_OK;
}
