// sdpc_potrf_static: the dense FP64 Cholesky of sdpc_potrf (type (i) of
// Section 3.1) for callers that cannot allocate device memory.  It needs no
// handle: its workspace (the parked diagonal factors of the column steps and the
// failure flag) lives in one fixed device array per GPU, `scratch`, which the
// code object holds until the process ends.
//
// In host code `scratch` names a host-side stand-in, not the device copy: its
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and only that address is handed to kernels.  Every call
// on one GPU shares that GPU's array, so calls that overlap on one GPU (two
// streams, two host threads) race and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/sdpc.h"
#include "kernels.h"

namespace sdpc {

namespace {

constexpr int kStaticMaxM = 65535;           // largest order accepted
constexpr size_t kWorkDoubles = 2 * 64 * 64; // parked diagonal factors (potrf_work_doubles)
constexpr size_t kScratchDoubles = kWorkDoubles + 32;   // + the failure flag, on its own 256 bytes
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

__global__ void k_flag_clear(int *flag) {
    if (threadIdx.x == 0) flag[0] = 0;
}

__global__ void k_flag_out(const int *flag, int32_t *info) {
    if (threadIdx.x == 0) info[0] = flag[0];
}

// Device address of this device's scratch array (looked up on the first call
// on each device, with that device current).
sdpc_status scratch_ptr(hipStream_t st, double **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SDPC_E_HIP;
    if (st) {
        int sdev = dev;
        if (hipStreamGetDevice(st, &sdev) != hipSuccess) return SDPC_E_HIP;
        dev = sdev;
    }
    if (dev < 0 || dev >= kMaxDevices) return SDPC_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return SDPC_E_HIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return SDPC_E_HIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return SDPC_E_HIP;
        }
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return SDPC_OK;
}

}  // namespace

}  // namespace sdpc

extern "C" sdpc_status sdpc_potrf_static(double *d_B, int64_t ldb, int32_t m, int32_t *d_info, hipStream_t stream) {
    using namespace sdpc;
    if (m < 0 || (m > 0 && !d_B) || ldb < (m > 0 ? m : 1)) {
        set_unbound_error("sdpc_potrf_static: bad arguments (need d_B != NULL, m >= 0, ldb >= max(1, m))");
        return SDPC_E_ARG;
    }
    if (m > kStaticMaxM) {
        set_unbound_error("sdpc_potrf_static: m = " + std::to_string(m) + " exceeds the limit of " +
                          std::to_string(kStaticMaxM));
        return SDPC_E_ARG;
    }
    double *ptr = nullptr;
    const sdpc_status s = scratch_ptr(stream, &ptr);
    if (s != SDPC_OK) {
        set_unbound_error("sdpc_potrf_static: device address of the scratch array not available");
        return s;
    }
    int *flag = reinterpret_cast<int *>(ptr + kWorkDoubles);
    hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(64), 0, stream, flag);
    launch_potrf(m, d_B, ldb, ptr, flag, stream);
    if (d_info) hipLaunchKernelGGL(k_flag_out, dim3(1), dim3(64), 0, stream, (const int *)flag, d_info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_unbound_error(std::string("sdpc_potrf_static: launch failed: ") + hipGetErrorString(e));
        return SDPC_E_HIP;
    }
    if (d_info) return SDPC_OK;   // asynchronous: the outcome arrives in *d_info
    int f = 0;
    e = hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        set_unbound_error(std::string("sdpc_potrf_static: ") + hipGetErrorString(e));
        return SDPC_E_HIP;
    }
    if (f < 0) {
        set_unbound_error("sdpc_potrf_static: internal hand-over wait ran out");
        return SDPC_E_HIP;
    }
    if (f > 0) {
        set_unbound_error("sdpc_potrf_static: matrix not positive definite at pivot " + std::to_string(f - 1));
        return SDPC_E_NOT_PD;
    }
    return SDPC_OK;
}
