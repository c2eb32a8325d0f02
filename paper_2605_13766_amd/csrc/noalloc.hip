// noalloc.hip -- the statically allocated device buffer of rod_energy_noalloc.
//
// rod_energy stages its per-rod energies in a device buffer that the library
// allocates with the batch.  Callers that may not allocate device memory at
// all get the same computation with that staging in `scratch`, a file-scope
// device array of fixed size that every call on a GPU shares.  Host code never
// passes the array's name to a kernel (in host code it is a host-side
// stand-in): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and that address is what the
// kernels receive.
#include "rod.h"
#include "rod_internal.h"

#include <hip/hip_runtime.h>
#include <mutex>
#include <string>

namespace rodk {

namespace {

// [0, 5 * NOALLOC_MAX_RODS): energies, 5 per rod; then one int32 (the first
// non-finite rod) in the next double's bytes; padded to a multiple of 256 B.
constexpr int64_t SCRATCH_DOUBLES = 5 * NOALLOC_MAX_RODS + 32;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_ptr[MAX_DEVICES] = {};

// out[0] = the smallest r < n whose flags have the non-finite bit, or n when there is none.
// One workgroup; every lane's slot of the LDS reduction is written before it
// is read, so nothing needs clearing beforehand.
__global__ __launch_bounds__(256) void first_flagged_kernel(const int32_t *flags, int n, int32_t *out)
{
    __shared__ int32_t red[256];
    int m = n;
    for (int r = threadIdx.x; r < n; r += 256)
        if (flags[r] & ROD_FLAG_NONFINITE) {   // other flag bits do not fail the call
            m = r;
            break;
        }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

int noalloc_scratch(double **energies, int32_t **first_flagged)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(ROD_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES)
        return set_error(ROD_EUNSUPPORTED, "device " + std::to_string(dev) + " is beyond the "
                                               + std::to_string(MAX_DEVICES) + " devices the static buffer serves");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(ROD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = static_cast<double *>(p);
    }
    *energies = g_ptr[dev];
    *first_flagged = reinterpret_cast<int32_t *>(g_ptr[dev] + 5 * NOALLOC_MAX_RODS);
    return ROD_OK;
}

hipError_t launch_first_flagged(const int32_t *flags, int n, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(first_flagged_kernel, dim3(1), dim3(256), 0, s, flags, n, out);
    return hipGetLastError();
}

}  // namespace rodk
