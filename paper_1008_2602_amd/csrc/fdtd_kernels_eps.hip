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

// Addressing.  Boards within the 4 GiB window: one base per field (its x, y, z
// arrays cstride bytes apart), byte offsets from node (0, 0, 0).  Larger boards
// (BIG): one base per component, moved once per thread to the chunk's base plane
// kb = max(k0 - 1, 0), byte offsets from that plane (a chunk spans at most a
// few planes, so they stay within 32 bits); absent D reads zero directly, and
// source and probe nodes are compared as 64-bit indices.
template <bool BIG>
struct View;
template <>
struct View<false> {
    const float* p;
    uint32_t cs;
    __device__ __forceinline__ View(const float* base, const BoardDev& B, uint64_t)
        : p(base), cs(B.cstride) {}
    __device__ __forceinline__ float ld(int c, uint32_t off) const { return ld_at(p, off + (uint32_t)c * cs); }
    __device__ __forceinline__ void st(int c, uint32_t off, float v) const
    {
        st_at<true>((float*)p, off + (uint32_t)c * cs, v);
    }
};
template <>
struct View<true> {
    const float* p[3];
    __device__ __forceinline__ View(const float* base, const BoardDev& B, uint64_t shift)
    {
        for (int c = 0; c < 3; ++c)
            p[c] = (const float*)((const char*)base + (uint64_t)c * B.cstride64 + shift);
    }
    __device__ __forceinline__ float ld(int c, uint32_t off) const { return ld_at(p[c], off); }
    __device__ __forceinline__ void st(int c, uint32_t off, float v) const
    {
        st_at<true>((float*)p[c], off, v);
    }
};

// plane the chunk's offsets are measured from, and its byte shift
template <bool BIG>
__device__ __forceinline__ int base_plane(const ColCtx& c)
{
    return BIG ? max(c.k0 - 1, 0) : 0;
}

template <typename CT, bool BIG>
__device__ __forceinline__ int class_of(const BoardDev& B, uint64_t cls_shift, uint32_t nb)
{
    const void* cls = BIG ? (const void*)((const char*)B.cls + cls_shift) : B.cls;
    return (int)ld_at_t<CT>(cls, sizeof(CT) == 1 ? nb >> 2 : nb >> 1);
}

// node index of the node at offset nb (for the source and probe lists)
template <bool BIG>
__device__ __forceinline__ int64_t node_of(int kb, int sz, uint32_t nb)
{
    return BIG ? (int64_t)kb * sz + (int64_t)(nb >> 2) : (int64_t)(nb >> 2);
}

}  // namespace

// B then H of every node from E at step n (buffer par) into buffer par ^ 1.
// E_x, E_y of plane k+1 carry over as plane k of the next iteration.
template <typename CT, bool BIG>
__global__ __launch_bounds__(256) void eps_h_pass(const BoardDev* __restrict__ board, int flip, int zl)
{
    const BoardDev& B = *board;
    ColCtx c;
    if (!col_ctx(B, flip, c)) return;
    col_chunk(zl, c);
    const uint32_t dyb = (uint32_t)c.sy * 4u, dzb = (uint32_t)c.sz * 4u;
    const int kb = base_plane<BIG>(c);
    const uint64_t shift = (uint64_t)kb * dzb;
    const uint64_t cls_shift = (uint64_t)kb * (uint64_t)c.sz * sizeof(CT);
    const View<BIG> gE(B.f[c.par][0], B, shift);
    const View<BIG> gH(B.f[c.par][3], B, shift);
    const View<BIG> gB(B.f[c.par][6], B, shift);
    const View<BIG> dH(B.f[c.par ^ 1][3], B, shift);
    const View<BIG> dB(B.f[c.par ^ 1][6], B, shift);
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
    const uint32_t nbk0 = c.nb0 + (uint32_t)(c.k0 - kb) * dzb;
    float exo = gE.ld(0, nbk0), eyo = gE.ld(1, nbk0);
    for (int k = c.k0; k < c.k1; ++k) {
        const uint32_t nb = c.nb0 + (uint32_t)(k - kb) * dzb;
        const bool pz = (k < B.pml[4]) || (B.pml[5] > 0 && k >= c.nz - B.pml[5]);
        const Qk z0 = qk_at(cz, nz1, 0, k), z1 = qk_at(cz, nz1, 1, k);
        const float ezo = gE.ld(2, nb);
        const float exu = gE.ld(0, nb + dzb), eyu = gE.ld(1, nb + dzb);
        const int id = class_of<CT, BIG>(B, cls_shift, nb);
        cgfloat* hf = (cgfloat*)B.node_aux + 6 * id;   // inverse eps_r at the Hx, Hy, Hz faces
        // Hx(i, j+1/2, k+1/2): Bx with y at j+1/2; Hx with z at k+1/2, x at i.  B is
        // read only where a PML keeps it: the branch also keeps each component's
        // loads next to their use, which holds the register count (and so the
        // occupancy) of this streaming pass up
        float hx;
        {
            const float cxe = (gE.ld(2, nb + dyb) - ezo) * crdy - (eyu - eyo) * crdz;
            const float inv = hf[0];
            const Sc Y = sc_of(y1, inv), Z = sc_of(z1, inv), X = sc_of(x0, inv);
            const bool keep = c.px || c.py;
            const float bo = keep ? gB.ld(0, nb) : 0.f;
            const float db = fmaf(Y.cam1, bo, -Y.rp * cxe);
            hx = fmaf(Z.ca, gH.ld(0, nb), Z.rp * fmaf(X.ph, db, X.q * bo));
            if (keep) dB.st(0, nb, bo + db);
        }
        dH.st(0, nb, hx);
        // Hy(i+1/2, j, k+1/2): By with z at k+1/2; Hy with x at i+1/2, y at j
        float hy;
        {
            const float cye = (exu - exo) * crdz - (gE.ld(2, nb + 4u) - ezo) * crdx;
            const float inv = hf[1];
            const Sc Z = sc_of(z1, inv), X = sc_of(x1, inv), Y = sc_of(y0, inv);
            const bool keep = c.py || pz;
            const float bo = keep ? gB.ld(1, nb) : 0.f;
            const float db = fmaf(Z.cam1, bo, -Z.rp * cye);
            hy = fmaf(X.ca, gH.ld(1, nb), X.rp * fmaf(Y.ph, db, Y.q * bo));
            if (keep) dB.st(1, nb, bo + db);
        }
        dH.st(1, nb, hy);
        // Hz(i+1/2, j+1/2, k): Bz with x at i+1/2; Hz with y at j+1/2, z at k
        float hz;
        {
            const float cze = (gE.ld(1, nb + 4u) - eyo) * crdx - (gE.ld(0, nb + dyb) - exo) * crdy;
            const float inv = hf[2];
            const Sc X = sc_of(x1, inv), Y = sc_of(y1, inv), Z = sc_of(z0, inv);
            const bool keep = pz || c.px;
            const float bo = keep ? gB.ld(2, nb) : 0.f;
            const float db = fmaf(X.cam1, bo, -X.rp * cze);
            hz = fmaf(Y.ca, gH.ld(2, nb), Y.rp * fmaf(Z.ph, db, Z.q * bo));
            if (keep) dB.st(2, nb, bo + db);
        }
        dH.st(2, nb, hz);
        exo = exu;
        eyo = eyu;
    }
}

// D then E of every node from H at n+1/2 (buffer par ^ 1, written by the H
// pass) and E, D at n (buffer par) into buffer par ^ 1, with the sources,
// probes, plane ring and watchdog of the fused kernels.  H_x, H_y of plane k
// carry over as plane k-1 of the next iteration.
template <typename CT, bool BIG>
__global__ __launch_bounds__(256) void eps_e_pass(const BoardDev* __restrict__ board, int rel, int flip,
                                                  int zl)
{
    const BoardDev& B = *board;
    ColCtx c;
    if (!col_ctx(B, flip, c)) return;
    col_chunk(zl, c);
    const uint32_t dyb = (uint32_t)c.sy * 4u, dzb = (uint32_t)c.sz * 4u;
    const int kb = base_plane<BIG>(c);
    const uint64_t shift = (uint64_t)kb * dzb;
    const uint64_t cls_shift = (uint64_t)kb * (uint64_t)c.sz * sizeof(CT);
    const View<BIG> gE(B.f[c.par][0], B, shift);
    const View<BIG> gD(B.d[c.par][0], B, shift);
    const View<BIG> nH(B.f[c.par ^ 1][3], B, shift);
    const View<BIG> dE(B.f[c.par ^ 1][0], B, shift);
    const View<BIG> dD(B.d[c.par ^ 1][0], B, shift);
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
    float hxm = c.k0 > 0 ? nH.ld(0, c.nb0 + (uint32_t)(c.k0 - 1 - kb) * dzb) : 0.f;
    float hym = c.k0 > 0 ? nH.ld(1, c.nb0 + (uint32_t)(c.k0 - 1 - kb) * dzb) : 0.f;
    // byte steps to the -x and -y neighbours, 0 on the low walls (see col_ctx)
    const uint32_t mxb = i > 0 ? 4u : 0u, myb = j > 0 ? dyb : 0u;
    const uint32_t guardb = dzb * (uint32_t)(c.nz + 1);   // first guard word of each array
    // the x and y tables at the column, read once (as in the H pass)
    const Qk x0 = qk_at(cx, nx1, 0, i), x1 = qk_at(cx, nx1, 1, i);
    const Qk y0 = qk_at(cy, ny1, 0, j), y1 = qk_at(cy, ny1, 1, j);
    for (int k = c.k0; k < c.k1; ++k) {
        const uint32_t nb = c.nb0 + (uint32_t)(k - kb) * dzb;
        const bool pz = (k < B.pml[4]) || (B.pml[5] > 0 && k >= c.nz - B.pml[5]);
        const Qk z0 = qk_at(cz, nz1, 0, k), z1 = qk_at(cz, nz1, 1, k);
        const int id = class_of<CT, BIG>(B, cls_shift, nb);
        const float inv_x = ctab[id].inv_x, inv_y = ctab[id].inv_y, inv_z = ctab[id].inv_z;
        const uint32_t flags = ctab[id].flags;
        cgfloat* loss = (cgfloat*)B.node_aux + 6 * id + 3;   // conduction of the Ex, Ey, Ez edges
        // the PML sigma seen by each edge: / eps_r with Eq. 2's eps_rw, else as is
        const float wx = B.eps_rw ? inv_x : 1.0f, wy = B.eps_rw ? inv_y : 1.0f,
                    wz = B.eps_rw ? inv_z : 1.0f;
        const float hx = nH.ld(0, nb), hy = nH.ld(1, nb), hz = nH.ld(2, nb);
        const float hzj = nH.ld(2, nb - myb), hzi = nH.ld(2, nb - mxb);
        const float hyi = nH.ld(1, nb - mxb), hxj = nH.ld(0, nb - myb);
        const float exo = gE.ld(0, nb), eyo = gE.ld(1, nb), ezo = gE.ld(2, nb);
        // D where a PML keeps it; elsewhere the load reads the zero guard words
        // after the array (one cache line for the whole wave, no HBM traffic)
        const bool kx = c.px || c.py, ky = c.py || pz, kz = pz || c.px;
        float dxo, dyo, dzo;
        if (BIG) {
            dxo = kx ? gD.ld(0, nb) : 0.f;
            dyo = ky ? gD.ld(1, nb) : 0.f;
            dzo = kz ? gD.ld(2, nb) : 0.f;
        } else {
            dxo = gD.ld(0, kx ? nb : guardb);
            dyo = gD.ld(1, ky ? nb : guardb);
            dzo = gD.ld(2, kz ? nb : guardb);
        }
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
            const int64_t node = node_of<BIG>(kb, c.sz, nb);
            const __attribute__((address_space(1))) int64_t* sn =
                (const __attribute__((address_space(1))) int64_t*)B.src_node64;
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
        dE.st(0, nb, exn);
        dE.st(1, nb, eyn);
        dE.st(2, nb, ezn);
        if (kx) dD.st(0, nb, ux ? dxo + ddx : dxo);
        if (ky) dD.st(1, nb, uy ? dyo + ddy : dyo);
        if (kz) dD.st(2, nb, uz ? dzo + ddz : dzo);
        if (flags & kPrbEz) {
            const int64_t node = node_of<BIG>(kb, c.sz, nb);
            const __attribute__((address_space(1))) int64_t* pn =
                (const __attribute__((address_space(1))) int64_t*)B.prb_node64;
            gfloat* ps = (gfloat*)B.prb_series;
            for (int q = 0; q < B.nprb; ++q)
                if (pn[q] == node) ps[q * ms + step] = ezn;
        }
        if (flags & kPlnEz)
            st_at<true>(B.plane_ring, (uint32_t)(step & (kPlaneRing - 1)) * dzb + c.nb0, ezn);
        bad |= !isfinite(exn + eyn + ezn);
        hxm = hx;
        hym = hy;
    }
    if (bad) *(__attribute__((address_space(1))) int32_t*)B.bad = 1;
}

template <typename CT, bool BIG>
static void launch_eps2(dim3 grid, dim3 block, const BoardDev* board, int rel, int flip, int zl,
                        hipStream_t st)
{
    hipLaunchKernelGGL((eps_h_pass<CT, BIG>), grid, block, 0, st, board, flip, zl);
    hipLaunchKernelGGL((eps_e_pass<CT, BIG>), grid, block, 0, st, board, rel, flip, zl);
}

hipError_t launch_eps_step(const BoardDev* board, int nx, int ny, int nz, int64_t plane_bytes,
                           bool big, int rel, int flip, bool wide, hipStream_t st)
{
    // z chunks of up to 12 planes (a plane carried in registers saves a z
    // neighbour load; 12 timed 1 % faster than 8 or 16 and 3 % faster than 4 on
    // a 1048x792x88 board), shorter when the columns alone leave the GPU idle;
    // on BIG boards the chunk and its neighbour planes (zl + 2 planes from the
    // chunk's base plane) stay within the 32-bit offsets
    const dim3 block(64, 4);
    const int64_t bxy = (int64_t)((nx + 63) / 64) * ((ny + 3) / 4);
    int64_t zl = std::max<int64_t>(1, std::min<int64_t>(12, (int64_t)nz * bxy / 2048));
    if (big) zl = std::max<int64_t>(1, std::min<int64_t>(zl, (int64_t(1) << 32) / plane_bytes - 3));
    const dim3 grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4), (unsigned)((nz + zl - 1) / zl));
    if (wide) {
        if (big)
            launch_eps2<uint16_t, true>(grid, block, board, rel, flip, (int)zl, st);
        else
            launch_eps2<uint16_t, false>(grid, block, board, rel, flip, (int)zl, st);
    } else {
        if (big)
            launch_eps2<uint8_t, true>(grid, block, board, rel, flip, (int)zl, st);
        else
            launch_eps2<uint8_t, false>(grid, block, board, rel, flip, (int)zl, st);
    }
    return hipGetLastError();
}

}  // namespace fdtd
