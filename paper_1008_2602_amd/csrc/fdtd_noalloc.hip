// Fixed device scratch of the allocation-free probe spectrum
// (fdtd_probe_fft_noalloc): the FFT's two ping-pong buffers live in a
// file-scope device array, so that call allocates nothing.
//
// The array's name is a host-side stand-in in host code, not a device address:
// its address on a device is looked up once per device, with that device
// current, and only that address is handed to kernels and copies.  Each device
// holds its own copy of the array until the process ends; every call on a device
// shares it, so calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fdtd_internal.h"

namespace fdtd {

static __device__ __align__(256) double2 scratch[2 * kNoAllocFftMax];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this process's scratch array on `device`; the first call for
// a device makes that device current for the lookup and restores the caller's.
hipError_t noalloc_scratch(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return e;
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return hipSuccess;
}

// Split bins 0..nbins-1 of a complex spectrum into re[0..nbins) and
// im[0..nbins) of one double array (out = re, out + nbins = im).
__global__ void fft_split(const double2* __restrict__ x, int nbins, double* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nbins) return;
    const double2 v = x[k];
    out[k] = v.x;
    out[nbins + k] = v.y;
}

hipError_t launch_fft_split(const double2* x, int nbins, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(fft_split, dim3((nbins + 255) / 256), dim3(256), 0, st, x, nbins, out);
    return hipGetLastError();
}

}  // namespace fdtd
