// gfx950 two-step field kernel of libfdtd.
//
// field_step2 advances a tile by two full leapfrog steps (Model section: B->H
// then D->E, Eqs. 1-4, twice) in one pass over HBM.  Step n+1's fields never
// leave the compute unit: they live in LDS and registers while the block
// marches along z, one plane behind for the second step.  Each step widens the
// dependence cone by one cell, so the block recomputes the first step on a
// two-cell halo:
//
//   H^{n+1/2}   on rows j0-2 .. j0+Hh,   columns i0-2 .. i0+W   (H1)
//   E^{n+1}     on rows j0-1 .. j0+Hh,   columns i0-1 .. i0+W   (E1)
//   H^{n+3/2}   on rows j0-1 .. j0+Hh-1, columns i0-1 .. i0+W-1 (H2)
//   E^{n+2}     on rows j0   .. j0+Hh-1, columns i0   .. i0+W-1 (E2, owned)
//
// with W = 64 aligned columns and Hh = TY-3 owned rows.  TY row waves cover
// columns i0..i0+63 of the H1 rows; helper wave A takes the three halo columns
// (i0-2, i0-1, i0+W) and stages column i0+W+1, helper wave B stages the row
// above.  Per front plane k the block, with a barrier after each of 1-3,
//   1. computes H1 of plane k from E^n of planes k and k+1 (staged in LDS),
//   2. computes E1 of plane k (from H1 of planes k and k-1),
//   3. computes H2 of plane k-1 (from E1 of planes k-1 and k, both in LDS) and
//      stages E^n for the next front plane (Ex, Ey of plane k+2 into plane k's
//      slot, Ez of plane k+1),
//   4. computes E2 of plane k-1 on the owned patch and stores E2, H2 and the
//      kept D/B of step n+2.
// Every per-node update is written with exactly the expressions of the one-step
// kernel, so the two kernels give bitwise equal fields.  Fields are read from
// one buffer and written to the other, as in the one-step kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdtd_device.h"
#include "fdtd_internal.h"

namespace fdtd {

// coefficient set of one axis at one node position (node "n" and half-node "h");
// kappa only in the material variant
struct AxisCoef {
    float cam1_n, ca_n, rp_n, ph_n, q_n;
    float cam1_h, ca_h, rp_h, ph_h, q_h;
    float k_n, k_h;
};

// The material variant (MT): a PML node's coefficients rebuilt from q scaled by
// the field location's 1/eps_rw (Eq. 2) and kappa, in exactly the node passes'
// arithmetic, so that the two give the same bits (the node passes take the odd
// step of a material board).  A material board's table holds these values
// rebuilt at 1/eps_rw = 1, so nodes whose class flags no scaled location read
// the table instead (most of the PML, where the board holds air).
__device__ __forceinline__ AxisCoef scale_coef(const AxisCoef& a, float w)
{
    AxisCoef o;
    o.q_n = a.q_n * w;
    o.ph_n = fmaf(0.5f, o.q_n, a.k_n);
    o.rp_n = 1.0f / o.ph_n;
    o.ca_n = fmaf(-0.5f, o.q_n, a.k_n) * o.rp_n;
    o.cam1_n = -o.q_n * o.rp_n;
    o.q_h = a.q_h * w;
    o.ph_h = fmaf(0.5f, o.q_h, a.k_h);
    o.rp_h = 1.0f / o.ph_h;
    o.ca_h = fmaf(-0.5f, o.q_h, a.k_h) * o.rp_h;
    o.cam1_h = -o.q_h * o.rp_h;
    o.k_n = a.k_n;
    o.k_h = a.k_h;
    return o;
}

// MM: 0 the plain kernel; 1 the material variant (PML coefficients rebuilt,
// conducting edges solved); 2 its conduction-only flavour (conducting edges
// solved, no rebuild: tile planes whose nodes need no rebuilt coefficient).
// SS: the fields are stored with non-temporal (streaming) stores, for launches
// whose fields outgrow the caches
template <int TY, typename CT, bool PL, int MM, bool SS>
__global__ __launch_bounds__(64 * TY + 128)
__attribute__((amdgpu_waves_per_eu(TY <= 6 ? 4 : 1))) void field_step2(const BoardDev* __restrict__ boards,
                                                             const TileRef* __restrict__ tiles,
                                                             int rel, int flip)
{
    constexpr bool MT = MM != 0;     // the material arithmetic (class aux data, conduction)
    constexpr bool RB = MM == 1;     // and PML coefficients rebuilt for 1/eps_rw
    constexpr int W = 64;            // owned columns
    constexpr int SC = W + 4;        // LDS columns: c = i - (i0 - 2), i0-2 .. i0+W+1
    constexpr int NT = 64 * TY + 128;
    static_assert(TY >= 5 && 4 * TY + 4 <= 64 && NT <= 1024, "tile shape");
    __shared__ float sE0x[2][TY + 1][SC];
    __shared__ float sE0y[2][TY + 1][SC];
    __shared__ float sE0z[TY + 1][SC];
    __shared__ float sH1x[TY][SC];
    __shared__ float sH1y[TY][SC];
    __shared__ float sH1z[TY][SC];
    __shared__ float sE1x[2][TY][SC];
    __shared__ float sE1y[2][TY][SC];
    __shared__ float sE1z[2][TY][SC];
    __shared__ float sH2x[TY][SC];
    __shared__ float sH2y[TY][SC];
    __shared__ float sH2z[TY][SC];
    constexpr int kLdsClasses = sizeof(CT) == 1 ? 256 : 1;
    __shared__ ClassEntry sTab[kLdsClasses];
    // material variant: each class's 1/eps_r at the H faces and the conduction
    // of its E edges (six floats), in LDS for one-byte class indices
    constexpr int kLdsAux = MT && sizeof(CT) == 1 ? 256 : 1;
    __shared__ float sAux[kLdsAux][6];
    // z coefficients of plane p in slot p & 3 (planes k-1, k and k+1 are live at
    // once), staged by the last wave; the material variant also keeps kappa
    constexpr int NZE = RB ? 12 : 10;
    __shared__ float sZ[4][NZE];

    const TileRef t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (t.board < 0) return;   // idle entry padding an XCD's list
    const BoardDev& B = boards[t.board];
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int sy = B.pitch, sz = B.pitch * (ny + 1), guard = sz * (nz + 1);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int i0 = t.tx * W, j0 = t.ty * (TY - 3);
    // the row waves that run the second step's H (rows 1 .. TY-2; from row 2 on
    // also its E) set each phase's length: they issue first (the outer halo rows
    // and the helper waves have less to do)
    if (wave >= 1 && wave <= TY - 2) __builtin_amdgcn_s_setprio(1);

    // ---- lane roles: LDS position (r, c) and which stages it computes
    int r, c;
    bool comp = true;   // computes H1 (else it only stages E)
    if (wave < TY) {
        r = wave;
        c = lane + 2;
    } else if (wave == TY) {
        if (lane < 3 * TY) {
            const int g = lane / TY;
            r = lane - g * TY;
            c = g == 0 ? 0 : (g == 1 ? 1 : W + 2);
        } else if (lane < 4 * TY) {
            r = lane - 3 * TY;
            c = W + 3;
            comp = false;
        } else {
            // the four corners of the row above; lanes past them repeat the last
            // corner (same value to the same place)
            const int q = lane - 4 * TY;
            r = TY;
            c = q == 0 ? 0 : (q == 1 ? 1 : (q == 2 ? W + 2 : W + 3));
            comp = false;
        }
    } else {
        r = TY;
        c = lane + 2;
        comp = false;
    }
    const int i = i0 - 2 + c, j = j0 - 2 + r;
    const bool rH1 = comp;
    const bool rE1 = rH1 && r >= 1 && c >= 1;
    const bool rH2 = rE1 && r <= TY - 2 && c <= W + 1;
    const bool rE2 = rH2 && r >= 2 && c >= 2;
    const bool ib = ((unsigned)i <= (unsigned)nx) & ((unsigned)j <= (unsigned)ny);
    const bool own = rE2 && ib;

    const int kb = t.kb, ke = t.ke, k0 = kb > 2 ? kb - 2 : 0;
    const int64_t step = B.step[0] + rel;
    // uniform by construction; readfirstlane lets the compiler keep the array
    // bases it selects in scalar registers
    const int par = __builtin_amdgcn_readfirstlane((int)((B.step[1] + flip) & 1));
    // one base per field and copy; y and z sit cs and 2 cs bytes after x
    const float* gE = B.f[par][0];
    const float* gH = B.f[par][3];
    const float* gB = B.f[par][6];
    const float* gD = B.d[par][0];
    float* dE = B.f[par ^ 1][0];
    float* dH = B.f[par ^ 1][3];
    float* dB = B.f[par ^ 1][6];
    float* dD = B.d[par ^ 1][0];
    const uint32_t cs = B.cstride, cs2 = 2u * B.cstride;
    // byte offsets (4 bytes per node) into the field arrays
    const uint32_t szb = (uint32_t)sz * 4u, guardb = (uint32_t)guard * 4u;
    const void* cls = B.cls;
    const __attribute__((address_space(1))) ClassEntry* __restrict__ ctab =
        (const __attribute__((address_space(1))) ClassEntry*)B.ctab;
    const float crdx = B.crd_x, crdy = B.crd_y, crdz = B.crd_z;
    const int pml_zlo = B.pml[4], pml_zhi = B.pml[5];
    auto in_px = [&](int ii) { return (ii < B.pml[0]) || (B.pml[1] > 0 && ii >= nx - B.pml[1]); };
    auto in_py = [&](int jj) { return (jj < B.pml[2]) || (B.pml[3] > 0 && jj >= ny - B.pml[3]); };
    auto in_pz = [&](int k) { return (k < pml_zlo) || (pml_zhi > 0 && k >= nz - pml_zhi); };
    cgfloat* __restrict__ cxp = (cgfloat*)B.coef[0];
    cgfloat* __restrict__ cyp = (cgfloat*)B.coef[1];
    kfloat* __restrict__ czp = (kfloat*)B.coef[2];
    const int nx1 = nx + 1, ny1 = ny + 1, nz1 = nz + 1;
    auto axis_coef = [&](cgfloat* tab, int n1, int idx) {
        const int q = min(max(idx, 0), n1 - 1);
        AxisCoef a;
        a.cam1_n = tab[(kCam1 * 2 + 0) * n1 + q];
        a.ca_n = tab[(kCa * 2 + 0) * n1 + q];
        a.rp_n = tab[(kRp * 2 + 0) * n1 + q];
        a.ph_n = tab[(kPh * 2 + 0) * n1 + q];
        a.q_n = tab[(kQ * 2 + 0) * n1 + q];
        a.cam1_h = tab[(kCam1 * 2 + 1) * n1 + q];
        a.ca_h = tab[(kCa * 2 + 1) * n1 + q];
        a.rp_h = tab[(kRp * 2 + 1) * n1 + q];
        a.ph_h = tab[(kPh * 2 + 1) * n1 + q];
        a.q_h = tab[(kQ * 2 + 1) * n1 + q];
        a.k_n = RB ? tab[(kKappa * 2 + 0) * n1 + q] : 1.0f;
        a.k_h = RB ? tab[(kKappa * 2 + 1) * n1 + q] : 1.0f;
        return a;
    };
    // z coefficients from the LDS ring (entry kind*2 + half of the table)
    auto z_coef = [&](int k) {
        const float* z = sZ[k & 3];
        AxisCoef a;
        a.cam1_n = z[kCam1 * 2 + 0];
        a.ca_n = z[kCa * 2 + 0];
        a.rp_n = z[kRp * 2 + 0];
        a.ph_n = z[kPh * 2 + 0];
        a.q_n = z[kQ * 2 + 0];
        a.cam1_h = z[kCam1 * 2 + 1];
        a.ca_h = z[kCa * 2 + 1];
        a.rp_h = z[kRp * 2 + 1];
        a.ph_h = z[kPh * 2 + 1];
        a.q_h = z[kQ * 2 + 1];
        a.k_n = RB ? z[(kKappa * 2 + 0) % NZE] : 1.0f;
        a.k_h = RB ? z[(kKappa * 2 + 1) % NZE] : 1.0f;
        return a;
    };
    const bool z_lane = wave == TY + 1 && lane < NZE;   // writes entry `lane` of the ring
    const int zent = lane % NZE;

    if (sizeof(CT) == 1) {
        for (int e = tid; e < kLdsClasses; e += NT) {
            const int q = min(e, B.nclass - 1);
            sTab[e].inv_x = ctab[q].inv_x;
            sTab[e].inv_y = ctab[q].inv_y;
            sTab[e].inv_z = ctab[q].inv_z;
            sTab[e].flags = ctab[q].flags;
            if (MT)
                for (int v = 0; v < 6; ++v) sAux[e % kLdsAux][v] = ((cgfloat*)B.node_aux)[6 * q + v];
        }
    }
    // a class's material data: 1/eps_r at the Hx, Hy, Hz faces, then the
    // conduction of the Ex, Ey, Ez edges
    auto aux_of = [&](CT id, int v) {
        if (sizeof(CT) == 1) return sAux[(int)id % kLdsAux][v];
        return ((cgfloat*)B.node_aux)[6 * (int)id + v];
    };
    auto class_entry = [&](CT id) {
        ClassEntry ce;
        if (sizeof(CT) == 1) {
            ce = sTab[id];
        } else {
            ce.inv_x = ctab[id].inv_x;
            ce.inv_y = ctab[id].inv_y;
            ce.inv_z = ctab[id].inv_z;
            ce.flags = ctab[id].flags;
        }
        return ce;
    };


    const bool px = in_px(i), py = in_py(j);
    const AxisCoef X = axis_coef(cxp, nx1, i), Y = axis_coef(cyp, ny1, j);
    // byte offset of this lane's node in plane 0 (meaningful only where ib holds)
    const uint32_t node0b = (uint32_t)(i + j * sy) * 4u;
    // byte offset of this lane's node in plane p, or of the guard words
    auto at_plane = [&](int p) { return ib && (unsigned)p <= (unsigned)nz ? node0b + (uint32_t)p * szb : guardb; };
    const int64_t ms = B.max_steps;

    struct Stage { float ex, ey, ez, z; };
    struct Col { float hx, hy, hz, bx, by, bz, dx, dy, dz; CT c; };
    auto load_stage = [&](int p) {
        Stage s;
        const uint32_t up = at_plane(p + 1);
        s.ex = ld_at(gE, up);
        s.ey = ld_at(gE, up + cs);
        s.ez = ld_at(gE, at_plane(p) + cs2);
        s.z = czp[zent * nz1 + min(p, nz)];       // every lane loads one (exact wait counts)
        return s;
    };
    // Every load is issued on every path (absent operands read the zero guard
    // words), so the wait counts stay exact.  The next plane's column operands are issued in two groups so that the
    // vector memory pipe is not flooded at one point of the plane: H_x and H_y
    // (read by H1) at the top of the plane; H_z, B (H1), the class and D (E1) once
    // H1 is done; the staging loads follow the H2 phase.
    auto load_col_h = [&](int p, Col& o) {
        const uint32_t n = node0b + (uint32_t)p * szb;
        const bool okh = rH1 && ib && p <= nz;
        const uint32_t nh = okh ? n : guardb;
        o.hx = ld_at(gH, nh);
        o.hy = ld_at(gH, nh + cs);
    };
    auto load_col_hz = [&](int p, Col& o) {
        const uint32_t n = node0b + (uint32_t)p * szb;
        const bool okh = rH1 && ib && p <= nz;
        o.hz = ld_at(gH, (okh ? n : guardb) + cs2);
    };
    auto load_col_b = [&](int p, Col& o) {
        const uint32_t n = node0b + (uint32_t)p * szb;
        const bool pz = in_pz(p);
        const bool okh = rH1 && ib && p <= nz;
        o.bx = ld_at(gB, okh && (px || py) ? n : guardb);
        o.by = ld_at(gB, (okh && (py || pz) ? n : guardb) + cs);
        o.bz = ld_at(gB, (okh && (pz || px) ? n : guardb) + cs2);
    };
    auto load_col_cd = [&](int p, Col& o) {
        const uint32_t n = node0b + (uint32_t)p * szb;
        const bool pz = in_pz(p);
        const bool oke = rE1 && ib && p <= nz;
        // the material variant's H1 needs the class on every H1 lane
        const uint32_t ne = (RB ? rH1 && ib && p <= nz : oke) ? n : guardb;
        o.c = ld_at_t<CT>(cls, sizeof(CT) == 1 ? ne >> 2 : ne >> 1);
        o.dx = ld_at(gD, oke && (px || py) ? n : guardb);
        o.dy = ld_at(gD, (oke && (py || pz) ? n : guardb) + cs);
        o.dz = ld_at(gD, (oke && (pz || px) ? n : guardb) + cs2);
    };
    // Ez of a source edge: the sources' Js of step s enters the D_z curl, and a
    // resistive source's update is solved for Ez^{n+1}.  Recomputes ddz and ezn
    // from the plain curl, so edges without a source never carry the extra terms.
    auto source_ez = [&](int node, int64_t s, float chz, float e_old, float d_old,
                         float inv_z, const AxisCoef& Zc, float& ddz, float& ezn) {
        const __attribute__((address_space(1))) int32_t* sn =
            (const __attribute__((address_space(1))) int32_t*)B.src_node;
        cgfloat* sj = (cgfloat*)B.src_j;
        cgfloat* sb = (cgfloat*)B.src_beta;
        float js = 0.0f, bs = 0.0f;
        for (int q = 0; q < B.nsrc; ++q)
            if (sn[q] == node) {
                js += sj[q * ms + s];
                bs += sb[q];
            }
        const float chs = chz - js;
        ddz = fmaf(X.cam1_n, d_old, X.rp_n * chs);
        ezn = fmaf(Y.ca_n, e_old, Y.rp_n * (inv_z * fmaf(Zc.ph_h, ddz, Zc.q_h * d_old)));
        if (bs != 0.0f) ezn = conductive_e(e_old, chs, inv_z, bs);
    };
    // B then H of one node from the curls of E (the material variant's non-PML
    // nodes; the plain kernel writes the same expressions in place)
    auto h_plain = [&](const AxisCoef& Z, float cxe, float cye, float cze, float hxo, float hyo,
                       float hzo, float bxo, float byo, float bzo, float& dbx, float& dby, float& dbz,
                       float& hx, float& hy, float& hz) {
        dbx = fmaf(Y.cam1_h, bxo, -Y.rp_h * cxe);
        hx = fmaf(Z.ca_h, hxo, Z.rp_h * fmaf(X.ph_n, dbx, X.q_n * bxo));
        dby = fmaf(Z.cam1_h, byo, -Z.rp_h * cye);
        hy = fmaf(X.ca_h, hyo, X.rp_h * fmaf(Y.ph_n, dby, Y.q_n * byo));
        dbz = fmaf(X.cam1_h, bzo, -X.rp_h * cze);
        hz = fmaf(Y.ca_h, hzo, Y.rp_h * fmaf(Z.ph_n, dbz, Z.q_n * bzo));
    };
    // D then E of one node without sources or conduction from the table's
    // coefficients (the material variant's nodes whose 1/eps_rw leaves them
    // unscaled; the plain kernel writes the same expressions in place)
    auto e_plain = [&](const ClassEntry& ce, const AxisCoef& Z, float chx, float chy, float chz,
                       float exo, float eyo, float ezo, float dxo, float dyo, float dzo, float& ddx,
                       float& ddy, float& ddz, float& exn, float& eyn, float& ezn) {
        ddx = fmaf(Y.cam1_n, dxo, Y.rp_n * chx);
        exn = fmaf(Z.ca_n, exo, Z.rp_n * (ce.inv_x * fmaf(X.ph_h, ddx, X.q_h * dxo)));
        ddy = fmaf(Z.cam1_n, dyo, Z.rp_n * chy);
        eyn = fmaf(X.ca_n, eyo, X.rp_n * (ce.inv_y * fmaf(Y.ph_h, ddy, Y.q_h * dyo)));
        ddz = fmaf(X.cam1_n, dzo, X.rp_n * chz);
        ezn = fmaf(Y.ca_n, ezo, Y.rp_n * (ce.inv_z * fmaf(Z.ph_h, ddz, Z.q_h * dzo)));
    };
    // the same in a PML node of a material board: every axis's coefficients
    // rebuilt for the face's 1/eps_rw (one at each of the Hx, Hy, Hz faces)
    auto h_material = [&](CT id, const AxisCoef& Z, float cxe, float cye, float cze, float hxo,
                          float hyo, float hzo, float bxo, float byo, float bzo, float& dbx,
                          float& dby, float& dbz, float& hx, float& hy, float& hz) {
        {
            const float w = aux_of(id, 0);
            const AxisCoef Ys = scale_coef(Y, w), Zs = scale_coef(Z, w), Xs = scale_coef(X, w);
            dbx = fmaf(Ys.cam1_h, bxo, -Ys.rp_h * cxe);
            hx = fmaf(Zs.ca_h, hxo, Zs.rp_h * fmaf(Xs.ph_n, dbx, Xs.q_n * bxo));
        }
        {
            const float w = aux_of(id, 1);
            const AxisCoef Zs = scale_coef(Z, w), Xs = scale_coef(X, w), Ys = scale_coef(Y, w);
            dby = fmaf(Zs.cam1_h, byo, -Zs.rp_h * cye);
            hy = fmaf(Xs.ca_h, hyo, Xs.rp_h * fmaf(Ys.ph_n, dby, Ys.q_n * byo));
        }
        {
            const float w = aux_of(id, 2);
            const AxisCoef Xs = scale_coef(X, w), Ys = scale_coef(Y, w), Zs = scale_coef(Z, w);
            dbz = fmaf(Xs.cam1_h, bzo, -Xs.rp_h * cze);
            hz = fmaf(Ys.ca_h, hzo, Ys.rp_h * fmaf(Zs.ph_n, dbz, Zs.q_n * bzo));
        }
    };
    // D then E of one node on a material board, in the node passes' arithmetic:
    // with `rebuild` (a PML node with some edge's 1/eps_rw != 1) every axis's
    // coefficients rebuilt for each edge's 1/eps_rw, else the table's (the same
    // bits as rebuilt at 1); an edge that conducts (lossy dielectric, resistive
    // sheet, resistive source) solved for E^{n+1} with its conduction
    auto e_material = [&](const ClassEntry& ce, CT id, bool rebuild, int node, int64_t s,
                          const AxisCoef& Z, float chx, float chy, float chz, float exo, float eyo,
                          float ezo, float dxo, float dyo, float dzo, float& ddx, float& ddy,
                          float& ddz, float& exn, float& eyn, float& ezn) {
        const float wx = B.eps_rw ? ce.inv_x : 1.0f, wy = B.eps_rw ? ce.inv_y : 1.0f,
                    wz = B.eps_rw ? ce.inv_z : 1.0f;
        {
            AxisCoef Ys = Y, Zs = Z, Xs = X;
            if (rebuild) {
                Ys = scale_coef(Y, wx);
                Zs = scale_coef(Z, wx);
                Xs = scale_coef(X, wx);
            }
            ddx = fmaf(Ys.cam1_n, dxo, Ys.rp_n * chx);
            exn = fmaf(Zs.ca_n, exo, Zs.rp_n * (ce.inv_x * fmaf(Xs.ph_h, ddx, Xs.q_h * dxo)));
        }
        const float lx = aux_of(id, 3);
        if (lx != 0.0f) {
            exn = conductive_e(exo, chx, ce.inv_x, lx);
            ddx = chx - lx * (exn + exo);
        }
        {
            AxisCoef Zs = Z, Xs = X, Ys = Y;
            if (rebuild) {
                Zs = scale_coef(Z, wy);
                Xs = scale_coef(X, wy);
                Ys = scale_coef(Y, wy);
            }
            ddy = fmaf(Zs.cam1_n, dyo, Zs.rp_n * chy);
            eyn = fmaf(Xs.ca_n, eyo, Xs.rp_n * (ce.inv_y * fmaf(Ys.ph_h, ddy, Ys.q_h * dyo)));
        }
        const float ly = aux_of(id, 4);
        if (ly != 0.0f) {
            eyn = conductive_e(eyo, chy, ce.inv_y, ly);
            ddy = chy - ly * (eyn + eyo);
        }
        float chs = chz, bs = 0.0f;
        if (ce.flags & kSrcEz) {
            const __attribute__((address_space(1))) int32_t* sn =
                (const __attribute__((address_space(1))) int32_t*)B.src_node;
            cgfloat* sj = (cgfloat*)B.src_j;
            cgfloat* sb = (cgfloat*)B.src_beta;
            float js = 0.0f;
            for (int q = 0; q < B.nsrc; ++q)
                if (sn[q] == node) {
                    js += sj[q * ms + s];
                    bs += sb[q];
                }
            chs -= js;
        }
        {
            AxisCoef Xs = X, Ys = Y, Zs = Z;
            if (rebuild) {
                Xs = scale_coef(X, wz);
                Ys = scale_coef(Y, wz);
                Zs = scale_coef(Z, wz);
            }
            ddz = fmaf(Xs.cam1_n, dzo, Xs.rp_n * chs);
            ezn = fmaf(Ys.ca_n, ezo, Ys.rp_n * (ce.inv_z * fmaf(Zs.ph_h, ddz, Zs.q_h * dzo)));
        }
        bs += aux_of(id, 5);   // a resistive source's lumped conductance adds to the medium's
        if (bs != 0.0f) {
            ezn = conductive_e(ezo, chs, ce.inv_z, bs);
            ddz = chs - bs * (ezn + ezo);
        }
    };
    auto record_probe = [&](int node, int64_t s, float ez) {
        const __attribute__((address_space(1))) int32_t* pn =
            (const __attribute__((address_space(1))) int32_t*)B.prb_node;
        gfloat* ps = (gfloat*)B.prb_series;
        for (int q = 0; q < B.nprb; ++q)
            if (pn[q] == node) ps[q * ms + s] = ez;
    };
    // Ez of the plane-DFT plane at step (launch step + extra) into ring slot
    // step mod kPlaneRing (slots are node planes of the field layout).  The step
    // is read afresh here (volatile): a loop-invariant slot offset would be
    // hoisted out of the plane loop and held in registers the hot path needs.
    auto plane_sample = [&](int extra, float ez) {
        const int64_t now = *(const volatile int64_t*)B.step + rel + extra;
        st_at<SS>(B.plane_ring, (uint32_t)(now & (kPlaneRing - 1)) * szb + node0b, ez);
    };

    // staging of the first front plane: E_x, E_y of planes k0 (slot 0) and k0+1
    // (slot 1), E_z of plane k0.  Stage p (E_x, E_y of plane p+1, E_z of plane p)
    // is loaded two front planes before it is written.
    sE0x[0][r][c] = ld_at(gE, at_plane(k0));
    sE0y[0][r][c] = ld_at(gE, at_plane(k0) + cs);
    {
        const Stage t = load_stage(k0);
        sE0x[1][r][c] = t.ex;
        sE0y[1][r][c] = t.ey;
        sE0z[r][c] = t.ez;
        if (z_lane) sZ[k0 & 3][lane] = t.z;
    }
    Stage s0 = load_stage(k0 + 1), s1 = load_stage(k0 + 2);
    Col cA, cB;
    load_col_h(k0, cA);
    load_col_hz(k0, cA);
    load_col_b(k0, cA);
    load_col_cd(k0, cA);
    __syncthreads();

    // carried from the previous front plane (k-1): H1, B1, own E1, D1 and class;
    // H2 of plane k-2
    float p_h1x = 0.f, p_h1y = 0.f, p_h1z = 0.f, p_b1x = 0.f, p_b1y = 0.f, p_b1z = 0.f;
    float p_e1x = 0.f, p_e1y = 0.f, p_e1z = 0.f, p_d1x = 0.f, p_d1y = 0.f, p_d1z = 0.f;
    CT p_c = 0;
    float p_h2x = 0.f, p_h2y = 0.f;
    bool bad = false;

    // st holds stage k+1 on entry: it is written once E1 of plane k has read plane
    // k's E^n, so the staging needs no barrier of its own (three per plane)
    auto plane_step = [&](int k, Stage& st, const Col& o, Col& nxt_col) {
        const int cur = (k - k0) & 1, nxt = cur ^ 1;
        const int m = k - 1;   // plane of the second step
        load_col_h(k + 1, nxt_col);
        const AxisCoef Zk = z_coef(k);

        // ---- H1 of plane k: B then H, step n -> n+1/2
        const bool okk = ib && k <= nz;
        const bool pz = in_pz(k);
        float h1x = 0.f, h1y = 0.f, h1z = 0.f, b1x = 0.f, b1y = 0.f, b1z = 0.f;
        if (rH1 && okk) {
            const float exo = sE0x[cur][r][c], eyo = sE0y[cur][r][c], ezo = sE0z[r][c];
            float dbx, dby, dbz;
            if constexpr (MT) {
                const float cxe = (sE0z[r + 1][c] - ezo) * crdy - (sE0y[nxt][r][c] - eyo) * crdz;
                const float cye = (sE0x[nxt][r][c] - exo) * crdz - (sE0z[r][c + 1] - ezo) * crdx;
                const float cze = (sE0y[cur][r][c + 1] - eyo) * crdx - (sE0x[cur][r + 1][c] - exo) * crdy;
                if (RB && (px || py || pz) && (class_entry(o.c).flags & kMatH))
                    h_material(o.c, Zk, cxe, cye, cze, o.hx, o.hy, o.hz, o.bx, o.by, o.bz, dbx, dby,
                               dbz, h1x, h1y, h1z);
                else
                    h_plain(Zk, cxe, cye, cze, o.hx, o.hy, o.hz, o.bx, o.by, o.bz, dbx, dby, dbz, h1x,
                            h1y, h1z);
            } else {
                const float cxe = (sE0z[r + 1][c] - ezo) * crdy - (sE0y[nxt][r][c] - eyo) * crdz;
                dbx = fmaf(Y.cam1_h, o.bx, -Y.rp_h * cxe);
                h1x = fmaf(Zk.ca_h, o.hx, Zk.rp_h * fmaf(X.ph_n, dbx, X.q_n * o.bx));
                const float cye = (sE0x[nxt][r][c] - exo) * crdz - (sE0z[r][c + 1] - ezo) * crdx;
                dby = fmaf(Zk.cam1_h, o.by, -Zk.rp_h * cye);
                h1y = fmaf(X.ca_h, o.hy, X.rp_h * fmaf(Y.ph_n, dby, Y.q_n * o.by));
                const float cze = (sE0y[cur][r][c + 1] - eyo) * crdx - (sE0x[cur][r + 1][c] - exo) * crdy;
                dbz = fmaf(X.cam1_h, o.bz, -X.rp_h * cze);
                h1z = fmaf(Y.ca_h, o.hz, Y.rp_h * fmaf(Zk.ph_n, dbz, Zk.q_n * o.bz));
            }
            b1x = (px || py) ? o.bx + dbx : 0.f;
            b1y = (py || pz) ? o.by + dby : 0.f;
            b1z = (pz || px) ? o.bz + dbz : 0.f;
        }
        if (rH1) {
            sH1x[r][c] = h1x;
            sH1y[r][c] = h1y;
            sH1z[r][c] = h1z;
        }
        __syncthreads();

        load_col_hz(k + 1, nxt_col);
        load_col_b(k + 1, nxt_col);
        load_col_cd(k + 1, nxt_col);
        // ---- E1 of plane k: D then E, step n -> n+1
        float e1x = 0.f, e1y = 0.f, e1z = 0.f, d1x = 0.f, d1y = 0.f, d1z = 0.f;
        const int e = cur;   // E1 plane slot of plane k (plane k-1 is in e ^ 1)
        if (rE1 && okk) {
            const ClassEntry ce = class_entry(o.c);
            const int node = (int)(node0b >> 2) + k * sz;   // node index (source/probe match)
            const float exo = sE0x[cur][r][c], eyo = sE0y[cur][r][c], ezo = sE0z[r][c];
            float ddx, ddy, ddz, exn, eyn, ezn;
            if constexpr (MT) {
                const float chx = (h1z - sH1z[r - 1][c]) * crdy - (h1y - p_h1y) * crdz;
                const float chy = (h1x - p_h1x) * crdz - (h1z - sH1z[r][c - 1]) * crdx;
                const float chz = (h1y - sH1y[r][c - 1]) * crdx - (h1x - sH1x[r - 1][c]) * crdy;
                const bool rebuild = RB && (px || py || pz) && (ce.flags & kMatE);
                if (rebuild || (ce.flags & (kCondE | kSrcEz)))
                    e_material(ce, o.c, rebuild, node, step, Zk, chx, chy, chz, exo, eyo, ezo, o.dx,
                               o.dy, o.dz, ddx, ddy, ddz, exn, eyn, ezn);
                else
                    e_plain(ce, Zk, chx, chy, chz, exo, eyo, ezo, o.dx, o.dy, o.dz, ddx, ddy, ddz, exn,
                            eyn, ezn);
            } else {
                const float chx = (h1z - sH1z[r - 1][c]) * crdy - (h1y - p_h1y) * crdz;
                ddx = fmaf(Y.cam1_n, o.dx, Y.rp_n * chx);
                exn = fmaf(Zk.ca_n, exo, Zk.rp_n * (ce.inv_x * fmaf(X.ph_h, ddx, X.q_h * o.dx)));
                const float chy = (h1x - p_h1x) * crdz - (h1z - sH1z[r][c - 1]) * crdx;
                ddy = fmaf(Zk.cam1_n, o.dy, Zk.rp_n * chy);
                eyn = fmaf(X.ca_n, eyo, X.rp_n * (ce.inv_y * fmaf(Y.ph_h, ddy, Y.q_h * o.dy)));
                const float chz = (h1y - sH1y[r][c - 1]) * crdx - (h1x - sH1x[r - 1][c]) * crdy;
                ddz = fmaf(X.cam1_n, o.dz, X.rp_n * chz);
                ezn = fmaf(Y.ca_n, ezo, Y.rp_n * (ce.inv_z * fmaf(Zk.ph_h, ddz, Zk.q_h * o.dz)));
                if (ce.flags & kSrcEz) source_ez(node, step, chz, ezo, o.dz, ce.inv_z, Zk, ddz, ezn);
            }
            e1x = (ce.flags & kUpdEx) ? exn : 0.0f;
            e1y = (ce.flags & kUpdEy) ? eyn : 0.0f;
            e1z = (ce.flags & kUpdEz) ? ezn : 0.0f;
            d1x = ((px || py) && (ce.flags & kUpdEx)) ? o.dx + ddx : o.dx;
            d1y = ((py || pz) && (ce.flags & kUpdEy)) ? o.dy + ddy : o.dy;
            d1z = ((pz || px) && (ce.flags & kUpdEz)) ? o.dz + ddz : o.dz;
            if (own && k >= kb && k < ke && (ce.flags & kPrbEz)) record_probe(node, step, e1z);
            if (PL && own && k >= kb && k < ke && (ce.flags & kPlnEz)) plane_sample(0, e1z);
        }
        if (rE1) {
            sE1x[e][r][c] = e1x;
            sE1y[e][r][c] = e1y;
            sE1z[e][r][c] = e1z;
        }
        __syncthreads();

        // ---- H2 of plane m = k-1: B then H, step n+1/2 -> n+3/2
        const bool okm = ib && m >= 0 && m <= nz;
        const bool livem = m >= kb && m < ke;
        const AxisCoef Zm = z_coef(m);
        const bool pzm = in_pz(m);
        float h2x = 0.f, h2y = 0.f, h2z = 0.f;
        if (rH2 && okm) {
            const int pe = e ^ 1;
            const float exo = sE1x[pe][r][c], eyo = sE1y[pe][r][c], ezo = sE1z[pe][r][c];
            float dbx, dby, dbz;
            if constexpr (MT) {
                const float cxe = (sE1z[pe][r + 1][c] - ezo) * crdy - (sE1y[e][r][c] - eyo) * crdz;
                const float cye = (sE1x[e][r][c] - exo) * crdz - (sE1z[pe][r][c + 1] - ezo) * crdx;
                const float cze = (sE1y[pe][r][c + 1] - eyo) * crdx - (sE1x[pe][r + 1][c] - exo) * crdy;
                if (RB && (px || py || pzm) && (class_entry(p_c).flags & kMatH))
                    h_material(p_c, Zm, cxe, cye, cze, p_h1x, p_h1y, p_h1z, p_b1x, p_b1y, p_b1z, dbx,
                               dby, dbz, h2x, h2y, h2z);
                else
                    h_plain(Zm, cxe, cye, cze, p_h1x, p_h1y, p_h1z, p_b1x, p_b1y, p_b1z, dbx, dby, dbz,
                            h2x, h2y, h2z);
            } else {
                const float cxe = (sE1z[pe][r + 1][c] - ezo) * crdy - (sE1y[e][r][c] - eyo) * crdz;
                dbx = fmaf(Y.cam1_h, p_b1x, -Y.rp_h * cxe);
                h2x = fmaf(Zm.ca_h, p_h1x, Zm.rp_h * fmaf(X.ph_n, dbx, X.q_n * p_b1x));
                const float cye = (sE1x[e][r][c] - exo) * crdz - (sE1z[pe][r][c + 1] - ezo) * crdx;
                dby = fmaf(Zm.cam1_h, p_b1y, -Zm.rp_h * cye);
                h2y = fmaf(X.ca_h, p_h1y, X.rp_h * fmaf(Y.ph_n, dby, Y.q_n * p_b1y));
                const float cze = (sE1y[pe][r][c + 1] - eyo) * crdx - (sE1x[pe][r + 1][c] - exo) * crdy;
                dbz = fmaf(X.cam1_h, p_b1z, -X.rp_h * cze);
                h2z = fmaf(Y.ca_h, p_h1z, Y.rp_h * fmaf(Zm.ph_n, dbz, Zm.q_n * p_b1z));
            }
            if (own && livem) {
                const uint32_t nb = node0b + (uint32_t)m * szb;
                st_at<SS>(dH, nb, h2x);
                st_at<SS>(dH, nb + cs, h2y);
                st_at<SS>(dH, nb + cs2, h2z);
                if (px || py) st_at<SS>(dB, nb, p_b1x + dbx);
                if (py || pzm) st_at<SS>(dB, nb + cs, p_b1y + dby);
                if (pzm || px) st_at<SS>(dB, nb + cs2, p_b1z + dbz);
            }
        }
        if (rH2) {
            sH2x[r][c] = h2x;
            sH2y[r][c] = h2y;
            sH2z[r][c] = h2z;
        }
        // ---- stage k+1: E_x, E_y of plane k+2 into plane k's slot, E_z of plane k+1
        sE0x[cur][r][c] = st.ex;
        sE0y[cur][r][c] = st.ey;
        sE0z[r][c] = st.ez;
        if (z_lane) sZ[(k + 1) & 3][lane] = st.z;
        __syncthreads();
        st = load_stage(k + 3);

        // ---- E2 of plane m on the owned patch: D then E, step n+1 -> n+2
        if (own && livem) {
            const ClassEntry ce = class_entry(p_c);
            const int node = (int)(node0b >> 2) + m * sz;
            float ddx, ddy, ddz, exn, eyn, ezn;
            if constexpr (MT) {
                const float chx = (h2z - sH2z[r - 1][c]) * crdy - (h2y - p_h2y) * crdz;
                const float chy = (h2x - p_h2x) * crdz - (h2z - sH2z[r][c - 1]) * crdx;
                const float chz = (h2y - sH2y[r][c - 1]) * crdx - (h2x - sH2x[r - 1][c]) * crdy;
                const bool rebuild = RB && (px || py || pzm) && (ce.flags & kMatE);
                if (rebuild || (ce.flags & (kCondE | kSrcEz)))
                    e_material(ce, p_c, rebuild, node, step + 1, Zm, chx, chy, chz, p_e1x, p_e1y,
                               p_e1z, p_d1x, p_d1y, p_d1z, ddx, ddy, ddz, exn, eyn, ezn);
                else
                    e_plain(ce, Zm, chx, chy, chz, p_e1x, p_e1y, p_e1z, p_d1x, p_d1y, p_d1z, ddx, ddy,
                            ddz, exn, eyn, ezn);
            } else {
                const float chx = (h2z - sH2z[r - 1][c]) * crdy - (h2y - p_h2y) * crdz;
                ddx = fmaf(Y.cam1_n, p_d1x, Y.rp_n * chx);
                exn = fmaf(Zm.ca_n, p_e1x, Zm.rp_n * (ce.inv_x * fmaf(X.ph_h, ddx, X.q_h * p_d1x)));
                const float chy = (h2x - p_h2x) * crdz - (h2z - sH2z[r][c - 1]) * crdx;
                ddy = fmaf(Zm.cam1_n, p_d1y, Zm.rp_n * chy);
                eyn = fmaf(X.ca_n, p_e1y, X.rp_n * (ce.inv_y * fmaf(Y.ph_h, ddy, Y.q_h * p_d1y)));
                const float chz = (h2y - sH2y[r][c - 1]) * crdx - (h2x - sH2x[r - 1][c]) * crdy;
                ddz = fmaf(X.cam1_n, p_d1z, X.rp_n * chz);
                ezn = fmaf(Y.ca_n, p_e1z, Y.rp_n * (ce.inv_z * fmaf(Zm.ph_h, ddz, Zm.q_h * p_d1z)));
                if (ce.flags & kSrcEz) source_ez(node, step + 1, chz, p_e1z, p_d1z, ce.inv_z, Zm, ddz, ezn);
            }
            exn = (ce.flags & kUpdEx) ? exn : 0.0f;
            eyn = (ce.flags & kUpdEy) ? eyn : 0.0f;
            ezn = (ce.flags & kUpdEz) ? ezn : 0.0f;
            const uint32_t nb = node0b + (uint32_t)m * szb;
            st_at<SS>(dE, nb, exn);
            st_at<SS>(dE, nb + cs, eyn);
            st_at<SS>(dE, nb + cs2, ezn);
            if (px || py) st_at<SS>(dD, nb, (ce.flags & kUpdEx) ? p_d1x + ddx : p_d1x);
            if (py || pzm) st_at<SS>(dD, nb + cs, (ce.flags & kUpdEy) ? p_d1y + ddy : p_d1y);
            if (pzm || px) st_at<SS>(dD, nb + cs2, (ce.flags & kUpdEz) ? p_d1z + ddz : p_d1z);
            if (ce.flags & kPrbEz) record_probe(node, step + 1, ezn);
            if (PL && (ce.flags & kPlnEz)) plane_sample(1, ezn);
            bad |= !isfinite(exn + eyn + ezn);
        }
        // plane k's step-one values become the carried ones
        p_h1x = h1x; p_h1y = h1y; p_h1z = h1z;
        p_b1x = b1x; p_b1y = b1y; p_b1z = b1z;
        p_e1x = e1x; p_e1y = e1y; p_e1z = e1z;
        p_d1x = d1x; p_d1y = d1y; p_d1z = d1z;
        p_c = o.c;
        p_h2x = h2x; p_h2y = h2y;
    };
    for (int k = k0; k <= ke; k += 2) {
        plane_step(k, s0, cA, cB);
        if (k + 1 <= ke) plane_step(k + 1, s1, cB, cA);
    }
    if (bad) *(__attribute__((address_space(1))) int32_t*)B.bad = 1;
}

// ---------------------------------------------------------------------------
struct Shape2 {
    int tx, ty;
};
// 64*TY + 128 threads.  TY = 14 and 12 run four waves per SIMD (128 VGPRs, two
// values spilled, four in the plane-DFT variant); 10, 9 and 8 run three (the
// kernel's 129-131 VGPRs fit); TY = 6 is held to 128 VGPRs so that two of its
// 512-thread blocks share a compute unit.  Taller tiles recompute fewer halo rows
// per owned row.
static const Shape2 kShapes2[] = {{64, 14}, {64, 12}, {64, 10}, {64, 9}, {64, 8}, {64, 6}};
static const int kNumShapes2 = sizeof(kShapes2) / sizeof(kShapes2[0]);

int num_shapes2() { return kNumShapes2; }
void shape2_at(int s, int* tx, int* ty)
{
    *tx = kShapes2[s].tx;
    *ty = kShapes2[s].ty;
}

template <int TY, bool PL, int MM, bool SS>
static void launch2_tpn(const BoardDev* boards, const TileRef* tiles, int ntiles, int rel, int flip,
                        bool wide, hipStream_t st)
{
    if (wide)
        hipLaunchKernelGGL((field_step2<TY, uint16_t, PL, MM, SS>), dim3(ntiles), dim3(64 * TY + 128),
                           0, st, boards, tiles, rel, flip);
    else
        hipLaunchKernelGGL((field_step2<TY, uint8_t, PL, MM, SS>), dim3(ntiles), dim3(64 * TY + 128),
                           0, st, boards, tiles, rel, flip);
}

template <int TY, bool PL, int MM>
static void launch2_tp(const BoardDev* boards, const TileRef* tiles, int ntiles, int rel, int flip,
                       bool wide, bool nt, hipStream_t st)
{
    if (nt)
        launch2_tpn<TY, PL, MM, true>(boards, tiles, ntiles, rel, flip, wide, st);
    else
        launch2_tpn<TY, PL, MM, false>(boards, tiles, ntiles, rel, flip, wide, st);
}

// plane: some board of the launch keeps a plane DFT (the variant with the ring
// store; the other never spends registers on it)
template <int TY>
static hipError_t launch2_t(const BoardDev* boards, const TileRef* tiles, int ntiles, int rel,
                            int flip, bool wide, bool plane, bool nt, hipStream_t st)
{
    if (plane)
        launch2_tp<TY, true, 0>(boards, tiles, ntiles, rel, flip, wide, nt, st);
    else
        launch2_tp<TY, false, 0>(boards, tiles, ntiles, rel, flip, wide, nt, st);
    return hipGetLastError();
}

template <int TY>
static int occupancy2_t(bool wide)
{
    int n = 0;
    hipError_t e = wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &n, field_step2<TY, uint16_t, false, 0, true>, 64 * TY + 128, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &n, field_step2<TY, uint8_t, false, 0, true>, 64 * TY + 128, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

int field_step2_occupancy(int tile_y, bool wide)
{
    switch (tile_y) {
        case 14: return occupancy2_t<14>(wide);
        case 12: return occupancy2_t<12>(wide);
        case 10: return occupancy2_t<10>(wide);
        case 9: return occupancy2_t<9>(wide);
        case 8: return occupancy2_t<8>(wide);
        case 6: return occupancy2_t<6>(wide);
        default: return 1;
    }
}

hipError_t launch_field_step2(int tile_y, const BoardDev* boards, const TileRef* tiles, int ntiles,
                              int rel, int flip, bool wide, bool plane, bool nt, hipStream_t st)
{
    switch (tile_y) {
        case 14: return launch2_t<14>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
        case 12: return launch2_t<12>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
        case 10: return launch2_t<10>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
        case 9: return launch2_t<9>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
        case 8: return launch2_t<8>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
        case 6: return launch2_t<6>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
        default: return hipErrorInvalidValue;
    }
}

// The material variant (Eq. 2's eps_rw in a dielectric PML, conduction), in two
// shapes.  64 x kHybridTY x 2 shares the plain kernel's tiles on a material
// board (which runs each tile's planes near material nodes on it and the rest
// on the plain kernel); at 128 VGPRs it spills about 15 values.  64 x kMatTY x 2,
// whose three waves per SIMD leave it the registers it needs, takes planes where
// such nodes fill the board.  The conduction-only flavour (no rebuilt coefficients)
// fits 64 x kHybridTY x 2 in 128 VGPRs without spilling.
template <int TY, int MM>
static int mat_occupancy(bool wide)
{
    int n = 0;
    hipError_t e = wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &n, field_step2<TY, uint16_t, false, MM, true>, 64 * TY + 128, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &n, field_step2<TY, uint8_t, false, MM, true>, 64 * TY + 128, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

// mode 1: the material variant (tile_y kHybridTY or kMatTY); mode 2: its
// conduction-only flavour (kHybridTY)
int field_step2_material_occupancy(int tile_y, int mode, bool wide)
{
    if (mode == 2) return mat_occupancy<kHybridTY, 2>(wide);
    return tile_y == kHybridTY ? mat_occupancy<kHybridTY, 1>(wide) : mat_occupancy<kMatTY, 1>(wide);
}

template <int TY, int MM>
static void mat_launch(const BoardDev* boards, const TileRef* tiles, int ntiles, int rel, int flip,
                       bool wide, bool plane, bool nt, hipStream_t st)
{
    if (plane)
        launch2_tp<TY, true, MM>(boards, tiles, ntiles, rel, flip, wide, nt, st);
    else
        launch2_tp<TY, false, MM>(boards, tiles, ntiles, rel, flip, wide, nt, st);
}

hipError_t launch_field_step2_material(int tile_y, int mode, const BoardDev* boards,
                                       const TileRef* tiles, int ntiles, int rel, int flip,
                                       bool wide, bool plane, bool nt, hipStream_t st)
{
    if (mode == 2 && tile_y == kHybridTY)
        mat_launch<kHybridTY, 2>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
    else if (mode == 1 && tile_y == kHybridTY)
        mat_launch<kHybridTY, 1>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
    else if (mode == 1 && tile_y == kMatTY)
        mat_launch<kMatTY, 1>(boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fdtd
