// Device-side helpers shared by the field kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace fdtd {

// Global-address-space views of the board's buffers: loads and stores through
// them are global_* instructions (counted in vmcnt only), so LDS barriers never
// wait on outstanding HBM traffic.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) const float cgfloat;
typedef __attribute__((address_space(4))) const float kfloat;  // uniform, scalar loads

// Hardware dispatches block b to XCD b % 8.  Map blocks so that each XCD walks
// a contiguous run of the tile list (neighbouring tiles share halos in its L2).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int x = b & 7, slot = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + slot;
}

}  // namespace fdtd
