// Leapfrog step for boards the tiled kernels do not cover: Eq. 2's eps_rw with a
// dielectric reaching into a PML slab (every sigma_w in s_w = kappa_w + sigma_w /
// (j w eps0 eps_rw) divided by the relative permittivity at the field location,
// so the update coefficients of a PML node depend on its material as well as
// its position), and lossy dielectrics (a conduction current sigma_c Ebar on
// interior edges, solved for E^{n+1} like a resistive source's).
// Two plain passes (B then H, D then E; one thread per (i, j) column marching
// up in z) recompute each axis's five coefficients from kappa and q / eps_rw;
// they share the fused kernels' layout, buffers, class flags, sources, probes
// and plane ring, and run only for those boards (all other boards take the
// fused field kernels).
#include <algorithm>

#include "fdtd_device.h"
#include "fdtd_internal.h"

namespace fdtd {

namespace {

struct Sc {
    float cam1, ca, rp, ph, q;
};

// q and kappa of one axis at one table index (node or half node)
struct Qk {
    float q, kap;
};
__device__ __forceinline__ Qk qk_at(cgfloat* tab, int n1, int half, int idx)
{
    return Qk{tab[(kQ * 2 + half) * n1 + idx], tab[(kKappa * 2 + half) * n1 + idx]};
}

// Coefficients of one axis from its q and kappa for a field location of inverse
// relative permittivity inv_eps (q scaled by 1/eps_rw).
__device__ __forceinline__ Sc sc_of(Qk t, float inv_eps)
{
    const float q = t.q * inv_eps;
    const float kap = t.kap;
    Sc s;
    s.q = q;
    s.ph = fmaf(0.5f, q, kap);
    s.rp = 1.0f / s.ph;
    s.ca = fmaf(-0.5f, q, kap) * s.rp;
    s.cam1 = -q * s.rp;
    return s;
}

struct ColCtx {
    int i, j, nx, ny, nz, sy, sz, k0, k1;   // planes k0 .. k1-1
    uint32_t nb0;        // byte offset of node (i, j, 0)
    bool px, py;         // column inside the x / y PML slab
    int par;
};

// One thread per (i, j) column and z chunk of zl planes, marching up in z.  Only
// nodes with i < nx, j < ny, k < nz are stepped: a node on the far wall holds
// only E tangential to the wall, H normal to it (which touches only such E) or
// components that do not exist, all zero.  Every neighbour a stepped node reads
// at +1 is then inside the arrays; the E pass clamps those at -1 to the node
// itself on the low walls (the components that read them are tangential there,
// held at zero), so its loads need no branch.
__device__ __forceinline__ bool col_ctx(const BoardDev& B, int flip, ColCtx& c)
{
    c.i = blockIdx.x * blockDim.x + threadIdx.x;
    c.j = blockIdx.y * blockDim.y + threadIdx.y;
    c.nx = B.nx;
    c.ny = B.ny;
    c.nz = B.nz;
    if (c.i >= c.nx || c.j >= c.ny) return false;
    c.sy = B.pitch;
    c.sz = B.pitch * (c.ny + 1);
    c.nb0 = (uint32_t)(c.i + c.j * c.sy) * 4u;
    c.px = (c.i < B.pml[0]) || (B.pml[1] > 0 && c.i >= c.nx - B.pml[1]);
    c.py = (c.j < B.pml[2]) || (B.pml[3] > 0 && c.j >= c.ny - B.pml[3]);
    c.par = (int)((B.step[1] + flip) & 1);
    return true;
}

__device__ __forceinline__ void col_chunk(int zl, ColCtx& c)
{
    c.k0 = blockIdx.z * zl;
    c.k1 = min(c.k0 + zl, c.nz);
}

template <typename CT>
__device__ __forceinline__ int class_of(const BoardDev& B, uint32_t nb)
{
    return (int)ld_at_t<CT>(B.cls, sizeof(CT) == 1 ? nb >> 2 : nb >> 1);
}

}  // namespace

// B then H of every node from E at step n (buffer par) into buffer par ^ 1.
// E_x, E_y of plane k+1 carry over as plane k of the next iteration.
template <typename CT>
__global__ __launch_bounds__(256) void eps_h_pass(const BoardDev* __restrict__ board, int flip, int zl)
{
    const BoardDev& B = *board;
    ColCtx c;
    if (!col_ctx(B, flip, c)) return;
    col_chunk(zl, c);
    const uint32_t cs = B.cstride, cs2 = 2u * B.cstride;
    const uint32_t dyb = (uint32_t)c.sy * 4u, dzb = (uint32_t)c.sz * 4u;
    const float* gE = B.f[c.par][0];
    const float* gH = B.f[c.par][3];
    const float* gB = B.f[c.par][6];
    float* dH = B.f[c.par ^ 1][3];
    float* dB = B.f[c.par ^ 1][6];
    cgfloat* cx = (cgfloat*)B.coef[0];
    cgfloat* cy = (cgfloat*)B.coef[1];
    cgfloat* cz = (cgfloat*)B.coef[2];
    const int nx1 = c.nx + 1, ny1 = c.ny + 1, nz1 = c.nz + 1;
    const float crdx = B.crd_x, crdy = B.crd_y, crdz = B.crd_z;
    const int i = c.i, j = c.j;
    // the x and y tables at the column, read once (the stores below may alias
    // them as far as the compiler knows, so it would reload them every plane)
    const Qk x0 = qk_at(cx, nx1, 0, i), x1 = qk_at(cx, nx1, 1, i);
    const Qk y0 = qk_at(cy, ny1, 0, j), y1 = qk_at(cy, ny1, 1, j);
    float exo = ld_at(gE, c.nb0 + (uint32_t)c.k0 * dzb), eyo = ld_at(gE, c.nb0 + (uint32_t)c.k0 * dzb + cs);
    for (int k = c.k0; k < c.k1; ++k) {
        const uint32_t nb = c.nb0 + (uint32_t)k * dzb;
        const bool pz = (k < B.pml[4]) || (B.pml[5] > 0 && k >= c.nz - B.pml[5]);
        const Qk z0 = qk_at(cz, nz1, 0, k), z1 = qk_at(cz, nz1, 1, k);
        const float ezo = ld_at(gE, nb + cs2);
        const float exu = ld_at(gE, nb + dzb), eyu = ld_at(gE, nb + dzb + cs);
        const int id = class_of<CT>(B, nb);
        cgfloat* hf = (cgfloat*)B.node_aux + 6 * id;   // inverse eps_r at the Hx, Hy, Hz faces
        // Hx(i, j+1/2, k+1/2): Bx with y at j+1/2; Hx with z at k+1/2, x at i.  B is
        // read only where a PML keeps it: the branch also keeps each component's
        // loads next to their use, which holds the register count (and so the
        // occupancy) of this streaming pass up
        float hx;
        {
            const float cxe = (ld_at(gE, nb + dyb + cs2) - ezo) * crdy - (eyu - eyo) * crdz;
            const float inv = hf[0];
            const Sc Y = sc_of(y1, inv), Z = sc_of(z1, inv), X = sc_of(x0, inv);
            const bool keep = c.px || c.py;
            const float bo = keep ? ld_at(gB, nb) : 0.f;
            const float db = fmaf(Y.cam1, bo, -Y.rp * cxe);
            hx = fmaf(Z.ca, ld_at(gH, nb), Z.rp * fmaf(X.ph, db, X.q * bo));
            if (keep) st_at(dB, nb, bo + db);
        }
        st_at(dH, nb, hx);
        // Hy(i+1/2, j, k+1/2): By with z at k+1/2; Hy with x at i+1/2, y at j
        float hy;
        {
            const float cye = (exu - exo) * crdz - (ld_at(gE, nb + 4u + cs2) - ezo) * crdx;
            const float inv = hf[1];
            const Sc Z = sc_of(z1, inv), X = sc_of(x1, inv), Y = sc_of(y0, inv);
            const bool keep = c.py || pz;
            const float bo = keep ? ld_at(gB, nb + cs) : 0.f;
            const float db = fmaf(Z.cam1, bo, -Z.rp * cye);
            hy = fmaf(X.ca, ld_at(gH, nb + cs), X.rp * fmaf(Y.ph, db, Y.q * bo));
            if (keep) st_at(dB, nb + cs, bo + db);
        }
        st_at(dH, nb + cs, hy);
        // Hz(i+1/2, j+1/2, k): Bz with x at i+1/2; Hz with y at j+1/2, z at k
        float hz;
        {
            const float cze = (ld_at(gE, nb + 4u + cs) - eyo) * crdx - (ld_at(gE, nb + dyb) - exo) * crdy;
            const float inv = hf[2];
            const Sc X = sc_of(x1, inv), Y = sc_of(y1, inv), Z = sc_of(z0, inv);
            const bool keep = pz || c.px;
            const float bo = keep ? ld_at(gB, nb + cs2) : 0.f;
            const float db = fmaf(X.cam1, bo, -X.rp * cze);
            hz = fmaf(Y.ca, ld_at(gH, nb + cs2), Y.rp * fmaf(Z.ph, db, Z.q * bo));
            if (keep) st_at(dB, nb + cs2, bo + db);
        }
        st_at(dH, nb + cs2, hz);
        exo = exu;
        eyo = eyu;
    }
}

// D then E of every node from H at n+1/2 (buffer par ^ 1, written by the H
// pass) and E, D at n (buffer par) into buffer par ^ 1, with the sources,
// probes, plane ring and watchdog of the fused kernels.  H_x, H_y of plane k
// carry over as plane k-1 of the next iteration.
template <typename CT>
__global__ __launch_bounds__(256) void eps_e_pass(const BoardDev* __restrict__ board, int rel, int flip,
                                                  int zl)
{
    const BoardDev& B = *board;
    ColCtx c;
    if (!col_ctx(B, flip, c)) return;
    col_chunk(zl, c);
    const uint32_t cs = B.cstride, cs2 = 2u * B.cstride;
    const uint32_t dyb = (uint32_t)c.sy * 4u, dzb = (uint32_t)c.sz * 4u;
    const float* gE = B.f[c.par][0];
    const float* gD = B.d[c.par][0];
    const float* nH = B.f[c.par ^ 1][3];
    float* dE = B.f[c.par ^ 1][0];
    float* dD = B.d[c.par ^ 1][0];
    cgfloat* cx = (cgfloat*)B.coef[0];
    cgfloat* cy = (cgfloat*)B.coef[1];
    cgfloat* cz = (cgfloat*)B.coef[2];
    const int nx1 = c.nx + 1, ny1 = c.ny + 1, nz1 = c.nz + 1;
    const __attribute__((address_space(1))) ClassEntry* ctab =
        (const __attribute__((address_space(1))) ClassEntry*)B.ctab;
    const float crdx = B.crd_x, crdy = B.crd_y, crdz = B.crd_z;
    const int i = c.i, j = c.j;
    const int64_t step = B.step[0] + rel;
    const int64_t ms = B.max_steps;
    bool bad = false;
    // H_x, H_y of plane k-1
    float hxm = c.k0 > 0 ? ld_at(nH, c.nb0 + (uint32_t)(c.k0 - 1) * dzb) : 0.f;
    float hym = c.k0 > 0 ? ld_at(nH, c.nb0 + (uint32_t)(c.k0 - 1) * dzb + cs) : 0.f;
    // byte steps to the -x and -y neighbours, 0 on the low walls (see col_ctx)
    const uint32_t mxb = i > 0 ? 4u : 0u, myb = j > 0 ? dyb : 0u;
    const uint32_t guardb = dzb * (uint32_t)(c.nz + 1);   // first guard word of each array
    // the x and y tables at the column, read once (as in the H pass)
    const Qk x0 = qk_at(cx, nx1, 0, i), x1 = qk_at(cx, nx1, 1, i);
    const Qk y0 = qk_at(cy, ny1, 0, j), y1 = qk_at(cy, ny1, 1, j);
    for (int k = c.k0; k < c.k1; ++k) {
        const uint32_t nb = c.nb0 + (uint32_t)k * dzb;
        const bool pz = (k < B.pml[4]) || (B.pml[5] > 0 && k >= c.nz - B.pml[5]);
        const Qk z0 = qk_at(cz, nz1, 0, k), z1 = qk_at(cz, nz1, 1, k);
        const int id = class_of<CT>(B, nb);
        const float inv_x = ctab[id].inv_x, inv_y = ctab[id].inv_y, inv_z = ctab[id].inv_z;
        const uint32_t flags = ctab[id].flags;
        cgfloat* loss = (cgfloat*)B.node_aux + 6 * id + 3;   // conduction of the Ex, Ey, Ez edges
        // the PML sigma seen by each edge: / eps_r with Eq. 2's eps_rw, else as is
        const float wx = B.eps_rw ? inv_x : 1.0f, wy = B.eps_rw ? inv_y : 1.0f,
                    wz = B.eps_rw ? inv_z : 1.0f;
        const float hx = ld_at(nH, nb), hy = ld_at(nH, nb + cs), hz = ld_at(nH, nb + cs2);
        const float hzj = ld_at(nH, nb - myb + cs2), hzi = ld_at(nH, nb - mxb + cs2);
        const float hyi = ld_at(nH, nb - mxb + cs), hxj = ld_at(nH, nb - myb);
        const float exo = ld_at(gE, nb), eyo = ld_at(gE, nb + cs), ezo = ld_at(gE, nb + cs2);
        // D where a PML keeps it; elsewhere the load reads the zero guard words
        // after the array (one cache line for the whole wave, no HBM traffic)
        const bool kx = c.px || c.py, ky = c.py || pz, kz = pz || c.px;
        const float dxo = ld_at(gD, kx ? nb : guardb), dyo = ld_at(gD, (ky ? nb : guardb) + cs),
                    dzo = ld_at(gD, (kz ? nb : guardb) + cs2);
        const float lx = loss[0], ly = loss[1], lz = loss[2];
        // Ex(i+1/2, j, k): Dx with y at j; Ex with z at k, x at i+1/2
        const float chx = (hz - hzj) * crdy - (hy - hym) * crdz;
        float ddx, exn;
        {
            const Sc Y = sc_of(y0, wx), Z = sc_of(z0, wx), X = sc_of(x1, wx);
            ddx = fmaf(Y.cam1, dxo, Y.rp * chx);
            exn = fmaf(Z.ca, exo, Z.rp * (inv_x * fmaf(X.ph, ddx, X.q * dxo)));
        }
        if (lx != 0.0f) {   // lossy interior edge; D (kept on a PML interface) gains eps_r (E' - E)
            exn = conductive_e(exo, chx, inv_x, lx);
            ddx = chx - lx * (exn + exo);
        }
        // Ey(i, j+1/2, k): Dy with z at k; Ey with x at i, y at j+1/2
        const float chy = (hx - hxm) * crdz - (hz - hzi) * crdx;
        float ddy, eyn;
        {
            const Sc Z = sc_of(z0, wy), X = sc_of(x0, wy), Y = sc_of(y1, wy);
            ddy = fmaf(Z.cam1, dyo, Z.rp * chy);
            eyn = fmaf(X.ca, eyo, X.rp * (inv_y * fmaf(Y.ph, ddy, Y.q * dyo)));
        }
        if (ly != 0.0f) {
            eyn = conductive_e(eyo, chy, inv_y, ly);
            ddy = chy - ly * (eyn + eyo);
        }
        // Ez(i, j, k+1/2): Dz with x at i; Ez with y at j, z at k+1/2
        float chz = (hy - hyi) * crdx - (hx - hxj) * crdy;
        float bs = 0.f;
        if (flags & kSrcEz) {
            const int node = (int)(nb >> 2);
            const __attribute__((address_space(1))) int32_t* sn =
                (const __attribute__((address_space(1))) int32_t*)B.src_node;
            cgfloat* sj = (cgfloat*)B.src_j;
            cgfloat* sb = (cgfloat*)B.src_beta;
            float js = 0.f;
            for (int q = 0; q < B.nsrc; ++q)
                if (sn[q] == node) {
                    js += sj[q * ms + step];
                    bs += sb[q];
                }
            chz -= js;
        }
        float ddz, ezn;
        {
            const Sc X = sc_of(x0, wz), Y = sc_of(y0, wz), Z = sc_of(z1, wz);
            ddz = fmaf(X.cam1, dzo, X.rp * chz);
            ezn = fmaf(Y.ca, ezo, Y.rp * (inv_z * fmaf(Z.ph, ddz, Z.q * dzo)));
        }
        bs += lz;   // a resistive source's lumped conductance adds to the medium's
        if (bs != 0.0f) {
            ezn = conductive_e(ezo, chz, inv_z, bs);
            ddz = chz - bs * (ezn + ezo);
        }
        // components on the outer wall or on PEC stay zero and keep their D
        const bool ux = flags & kUpdEx, uy = flags & kUpdEy, uz = flags & kUpdEz;
        exn = ux ? exn : 0.f;
        eyn = uy ? eyn : 0.f;
        ezn = uz ? ezn : 0.f;
        st_at(dE, nb, exn);
        st_at(dE, nb + cs, eyn);
        st_at(dE, nb + cs2, ezn);
        if (kx) st_at(dD, nb, ux ? dxo + ddx : dxo);
        if (ky) st_at(dD, nb + cs, uy ? dyo + ddy : dyo);
        if (kz) st_at(dD, nb + cs2, uz ? dzo + ddz : dzo);
        if (flags & kPrbEz) {
            const int node = (int)(nb >> 2);
            const __attribute__((address_space(1))) int32_t* pn =
                (const __attribute__((address_space(1))) int32_t*)B.prb_node;
            gfloat* ps = (gfloat*)B.prb_series;
            for (int q = 0; q < B.nprb; ++q)
                if (pn[q] == node) ps[q * ms + step] = ezn;
        }
        if (flags & kPlnEz)
            st_at(B.plane_ring, (uint32_t)(step & (kPlaneRing - 1)) * dzb + c.nb0, ezn);
        bad |= !isfinite(exn + eyn + ezn);
        hxm = hx;
        hym = hy;
    }
    if (bad) *(__attribute__((address_space(1))) int32_t*)B.bad = 1;
}

hipError_t launch_eps_step(const BoardDev* board, int nx, int ny, int nz, int rel, int flip,
                           bool wide, hipStream_t st)
{
    // z chunks of up to 12 planes (a plane carried in registers saves a z
    // neighbour load; 12 timed 1 % faster than 8 or 16 and 3 % faster than 4 on
    // a 1048x792x88 board), shorter when the columns alone leave the GPU idle
    const dim3 block(64, 4);
    const int64_t bxy = (int64_t)((nx + 63) / 64) * ((ny + 3) / 4);
    const int zl = (int)std::max<int64_t>(1, std::min<int64_t>(12, (int64_t)nz * bxy / 2048));
    const dim3 grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4), (unsigned)((nz + zl - 1) / zl));
    if (wide) {
        hipLaunchKernelGGL(eps_h_pass<uint16_t>, grid, block, 0, st, board, flip, zl);
        hipLaunchKernelGGL(eps_e_pass<uint16_t>, grid, block, 0, st, board, rel, flip, zl);
    } else {
        hipLaunchKernelGGL(eps_h_pass<uint8_t>, grid, block, 0, st, board, flip, zl);
        hipLaunchKernelGGL(eps_e_pass<uint8_t>, grid, block, 0, st, board, rel, flip, zl);
    }
    return hipGetLastError();
}

}  // namespace fdtd
