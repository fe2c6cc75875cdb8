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

// Access at a 32-bit byte offset from a uniform base.  Base (scalar registers)
// plus a zero-extended 32-bit offset is the global instructions' scalar-base
// form, so no 64-bit address arithmetic runs per lane and one offset serves every
// array of the same layout.  The library keeps padded arrays below 2^30 nodes,
// so every byte offset fits in 32 bits.
typedef __attribute__((address_space(1))) char gbyte;
__device__ __forceinline__ float ld_at(const float* base, uint32_t off)
{
    return *(const __attribute__((address_space(1))) float*)((const gbyte*)base + off);
}
// NT: a non-temporal (streaming) store, which the caches do not keep: for
// launches whose fields are far larger than the caches, so that the lines a
// launch reads, not the ones it has written, stay in L2 and the Infinity Cache
template <bool NT = false>
__device__ __forceinline__ void st_at(float* base, uint32_t off, float v)
{
    gfloat* p = (gfloat*)((gbyte*)base + off);
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
template <typename T>
__device__ __forceinline__ T ld_at_t(const void* base, uint32_t off)
{
    return *(const __attribute__((address_space(1))) T*)((const gbyte*)base + off);
}

// E^{n+1} of an interior edge that carries a conduction current (a resistive
// voltage source's lumped conductance, Results section, the Table 1 run; or a
// lossy dielectric).  Outside every PML (kappa 1, sigma 0, D never enters) and
// in the scaled units the current is beta (E^n + E^{n+1}) plus any Norton part,
// already subtracted in ch; with b = beta / eps_r the update
// (E' - E) / inv_eps_r = ch - beta (E + E') solved for E' is
// ((1 - b) E + inv_eps_r ch) / (1 + b).  beta = c0 dt eta0 dz / (2 R dx dy) for
// a resistor, sigma_c dt / (2 eps0) for a conductivity.
__device__ __forceinline__ float conductive_e(float e_old, float ch, float inv_eps, float beta)
{
    const float b = inv_eps * beta;
    return (fmaf(-b, e_old, e_old) + inv_eps * ch) / (1.0f + b);
}

// Hardware dispatches block b to XCD b % 8.  Map blocks so that each XCD walks
// a contiguous run of the tile list (neighbouring tiles share halos in its L2).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int x = b & 7, slot = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + slot;
}

}  // namespace fdtd
