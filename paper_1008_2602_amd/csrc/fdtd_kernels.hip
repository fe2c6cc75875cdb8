// gfx950 kernels of libfdtd.
//
// field_step: one full leapfrog step (Model section: B->H then D->E, Eqs. 1-4)
// for one tile of columns of one board, fused in a single pass.  A block owns a
// TX x (TY-1) patch of (i, j) columns, starting on a 128-byte boundary of the
// padded rows, and marches along z.  Its TY*TX/64 row waves cover the patch plus
// the row below it (a halo owned by the neighbouring tile); one more wave
// stages the extra row and columns and recomputes the halo column left of the
// patch.  Per z plane the block
//   1. stages E^n of planes k+1 (Ex, Ey) and k (Ez) for (TX+2) x (TY+1) columns
//      in LDS (Ex, Ey of plane k are kept from the previous plane),
//   2. computes B/H^{n+1/2} of plane k for the patch, the halo row and the halo
//      column, so that no second pass over H is needed,
//   3. computes D/E^{n+1} of plane k for the owned columns from the new H of
//      planes k (LDS) and k-1 (registers).
// Staging loads run two planes ahead and column operands one plane ahead; the
// plane loop is unrolled by two so no register in flight is ever moved.
// State is ping-ponged (E, H, B and D read from one copy, written to the other)
// so halo recomputation never sees a neighbour's already-updated values.  D and
// B are stored and moved only where a PML loss acts on them (elsewhere the
// update reduces to plain Yee with those terms exactly zero).  Sources and
// probes are folded into the same pass through per-node material classes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdtd_device.h"
#include "fdtd_internal.h"

namespace fdtd {


template <int TX, int TY, typename CT>
__global__ __launch_bounds__(TX* TY + 64) void field_step(const BoardDev* __restrict__ boards,
                                                          const TileRef* __restrict__ tiles,
                                                          int rel, int flip)
{
    static_assert(TX % 64 == 0 && TY + 1 <= 32 && TX * TY + 64 <= 1024, "tile shape");
    // LDS staging: columns i0-1 .. i0+TX (index c = i - i0 + 1), rows j0-1 .. j0-1+TY
    __shared__ float sEx[2][TY + 1][TX + 2];
    __shared__ float sEy[2][TY + 1][TX + 2];
    __shared__ float sEz[TY + 1][TX + 2];
    // new H of the plane: column 0 is the halo column i0-1 (Hy, Hz only)
    __shared__ float sHx[TY][TX + 1];
    __shared__ float sHy[TY][TX + 1];
    __shared__ float sHz[TY][TX + 1];
    // class table in LDS when the class index is one byte (<= 256 classes)
    constexpr int kLdsClasses = sizeof(CT) == 1 ? 256 : 1;
    __shared__ ClassEntry sTab[kLdsClasses];

    const TileRef t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (t.board < 0) return;   // idle entry padding an XCD's list
    const BoardDev& B = boards[t.board];
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int sy = B.pitch, sz = B.pitch * (ny + 1), guard = sz * (nz + 1);
    const int tid = threadIdx.x;
    // waves 0 .. TY*TX/64-1 own whole rows; the last wave handles the halo column
    // and the staging of the extra row and columns
    const bool main_wave = __builtin_amdgcn_readfirstlane(tid) < TX * TY;
    const int tx = tid % TX;
    const int ty = __builtin_amdgcn_readfirstlane(tid / TX);   // == TY in the extra wave
    const int lane = tid & 63;
    const int i0 = t.tx * TX, j0 = t.ty * (TY - 1);
    const int i = i0 + tx, j = j0 - 1 + ty;
    // planes kb .. ke-1 are stepped; a piece that starts above the bottom first
    // recomputes H of plane kb-1 (not stored) for the z-differences of plane kb
    const int kb = t.kb, ke = t.ke, k0 = kb > 0 ? kb - 1 : 0;
    const bool col_ok = main_wave && (i <= nx) && (j >= 0) && (j <= ny);
    const bool own = col_ok && ty > 0;
    const int64_t step = B.step[0] + B.rel0 + rel;
    // uniform by construction; readfirstlane lets the compiler keep the array
    // bases it selects in scalar registers (scalar-base 32-bit addressing)
    const int par = __builtin_amdgcn_readfirstlane((int)((B.step[1] + B.flip0 + flip) & 1));
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
    const uint32_t szb = (uint32_t)sz * 4u, guardb = (uint32_t)guard * 4u;
    const void* cls = B.cls;
    const __attribute__((address_space(1))) ClassEntry* __restrict__ ctab =
        (const __attribute__((address_space(1))) ClassEntry*)B.ctab;
    const float crdx = B.crd_x, crdy = B.crd_y, crdz = B.crd_z;
    const int pml_zlo = B.pml[4], pml_zhi = B.pml[5];
    auto in_px = [&](int ii) { return (ii < B.pml[0]) || (B.pml[1] > 0 && ii >= nx - B.pml[1]); };
    auto in_py = [&](int jj) { return (jj < B.pml[2]) || (B.pml[3] > 0 && jj >= ny - B.pml[3]); };
    auto in_pz = [&](int k) { return (k < pml_zlo) || (pml_zhi > 0 && k >= nz - pml_zhi); };
    cgfloat* __restrict__ cx = (cgfloat*)B.coef[0];
    cgfloat* __restrict__ cy = (cgfloat*)B.coef[1];
    kfloat* __restrict__ cz = (kfloat*)B.coef[2];
    const int nx1 = nx + 1, ny1 = ny + 1, nz1 = nz + 1;
    auto CXf = [&](int kind, int half, int ii) { return cx[(kind * 2 + half) * nx1 + min(max(ii, 0), nx)]; };
    auto CYf = [&](int kind, int half, int jj) { return cy[(kind * 2 + half) * ny1 + min(max(jj, 0), ny)]; };

    if (sizeof(CT) == 1) {
        for (int e = tid; e < kLdsClasses; e += TX * TY + 64) {
            const int c = min(e, B.nclass - 1);
            sTab[e].inv_x = ctab[c].inv_x;
            sTab[e].inv_y = ctab[c].inv_y;
            sTab[e].inv_z = ctab[c].inv_z;
            sTab[e].flags = ctab[c].flags;
        }
    }
    // byte offset of node (ii, jj, k), or of the guard words when it is off the grid
    auto node_at = [&](int ii, int jj, int k) {
        const bool ok = ((unsigned)ii <= (unsigned)nx) & ((unsigned)jj <= (unsigned)ny) &
                        ((unsigned)k <= (unsigned)nz);
        return ok ? (uint32_t)(ii + jj * sy + k * sz) * 4u : guardb;
    };

    if (main_wave) {
        // ------------------------------------------------------------ owned rows
        const bool px = in_px(i), py = in_py(j);
        const float x_cam1_n = CXf(kCam1, 0, i), x_ca_n = CXf(kCa, 0, i), x_rp_n = CXf(kRp, 0, i),
                    x_ph_n = CXf(kPh, 0, i), x_q_n = CXf(kQ, 0, i);
        const float x_cam1_h = CXf(kCam1, 1, i), x_ca_h = CXf(kCa, 1, i), x_rp_h = CXf(kRp, 1, i),
                    x_ph_h = CXf(kPh, 1, i), x_q_h = CXf(kQ, 1, i);
        const float y_cam1_n = CYf(kCam1, 0, j), y_ca_n = CYf(kCa, 0, j), y_rp_n = CYf(kRp, 0, j),
                    y_ph_n = CYf(kPh, 0, j), y_q_n = CYf(kQ, 0, j);
        const float y_cam1_h = CYf(kCam1, 1, j), y_ca_h = CYf(kCa, 1, j), y_rp_h = CYf(kRp, 1, j),
                    y_ph_h = CYf(kPh, 1, j), y_q_h = CYf(kQ, 1, j);
        const int c = tx + 1;
        const int node0 = i + j * sy;               // used only where col_ok holds
        const uint32_t node0b = (uint32_t)node0 * 4u;
        struct Stage { float ex, ey, ez; };
        struct Col { float hx, hy, hz, bx, by, bz, dx, dy, dz; CT c; };
        auto load_stage = [&](int p) {
            Stage s;
            const uint32_t up = node_at(i, j, p + 1);
            s.ex = ld_at(gE, up);
            s.ey = ld_at(gE, up + cs);
            s.ez = ld_at(gE, node_at(i, j, p) + cs2);
            return s;
        };
        // every load is issued on every path (absent operands read the zero
        // guard words), so the wait counts stay exact and the prefetch overlaps
        auto load_col = [&](int p, Col& o) {
            const uint32_t n = node0b + (uint32_t)p * szb;
            const bool pz = in_pz(p);
            const bool okp = col_ok && p <= nz, ownp = own && p <= nz;
            const bool live = ownp && p >= kb;   // E of this plane is stepped here
            const uint32_t nh = okp ? n : guardb;
            // the halo row only feeds Hx and Hz to the row above it
            o.hx = ld_at(gH, nh);
            o.hy = ld_at(gH, (ownp ? n : guardb) + cs);
            o.hz = ld_at(gH, nh + cs2);
            o.bx = ld_at(gB, okp && (px || py) ? n : guardb);
            o.by = ld_at(gB, (ownp && (py || pz) ? n : guardb) + cs);
            o.bz = ld_at(gB, (okp && (pz || px) ? n : guardb) + cs2);
            const uint32_t ne = live ? n : guardb;
            o.c = ld_at_t<CT>(cls, sizeof(CT) == 1 ? ne >> 2 : ne >> 1);
            o.dx = ld_at(gD, live && (px || py) ? n : guardb);
            o.dy = ld_at(gD, (live && (py || pz) ? n : guardb) + cs);
            o.dz = ld_at(gD, (live && (pz || px) ? n : guardb) + cs2);
        };
        sEx[0][ty][c] = ld_at(gE, node_at(i, j, k0));
        sEy[0][ty][c] = ld_at(gE, node_at(i, j, k0) + cs);
        Stage s0 = load_stage(k0), s1 = load_stage(k0 + 1);
        Col cA, cB;
        load_col(k0, cA);
        float hx_prev = 0.0f, hy_prev = 0.0f;
        bool bad = false;
        const int64_t ms = B.max_steps;

        auto plane_step = [&](int k, Stage& st, const Col& o, Col& nxt_col) {
            const int cur = (k - k0) & 1, nxt = cur ^ 1;
            const bool live = k >= kb;
            const bool pz = in_pz(k);
            const bool nbx = px || py, nby = py || pz, nbz = pz || px;
            const int node = node0 + k * sz;
            const uint32_t nb = node0b + (uint32_t)k * szb;
            sEx[nxt][ty][c] = st.ex;
            sEy[nxt][ty][c] = st.ey;
            sEz[ty][c] = st.ez;
            st = load_stage(k + 2);
            load_col(k + 1, nxt_col);
            kfloat* czk = cz + k;
            const float z_cam1_n = czk[(kCam1 * 2 + 0) * nz1], z_ca_n = czk[(kCa * 2 + 0) * nz1],
                        z_rp_n = czk[(kRp * 2 + 0) * nz1], z_ph_n = czk[(kPh * 2 + 0) * nz1],
                        z_q_n = czk[(kQ * 2 + 0) * nz1];
            const float z_cam1_h = czk[(kCam1 * 2 + 1) * nz1], z_ca_h = czk[(kCa * 2 + 1) * nz1],
                        z_rp_h = czk[(kRp * 2 + 1) * nz1], z_ph_h = czk[(kPh * 2 + 1) * nz1],
                        z_q_h = czk[(kQ * 2 + 1) * nz1];
            __syncthreads();

            // ---- B then H of plane k (own columns; row 0 is the y halo) ----
            float hxn = 0.f, hyn = 0.f, hzn = 0.f;
            const float exo = sEx[cur][ty][c], eyo = sEy[cur][ty][c], ezo = sEz[ty][c];
            if (col_ok) {
                // Hx(i, j+1/2, k+1/2): Bx uses y at j+1/2; Hx uses z at k+1/2, x at i
                const float cxe = (sEz[ty + 1][c] - ezo) * crdy - (sEy[nxt][ty][c] - eyo) * crdz;
                const float dbx = fmaf(y_cam1_h, o.bx, -y_rp_h * cxe);
                hxn = fmaf(z_ca_h, o.hx, z_rp_h * fmaf(x_ph_n, dbx, x_q_n * o.bx));
                // Hy(i+1/2, j, k+1/2): By uses z at k+1/2; Hy uses x at i+1/2, y at j
                const float cye = (sEx[nxt][ty][c] - exo) * crdz - (sEz[ty][c + 1] - ezo) * crdx;
                const float dby = fmaf(z_cam1_h, o.by, -z_rp_h * cye);
                hyn = fmaf(x_ca_h, o.hy, x_rp_h * fmaf(y_ph_n, dby, y_q_n * o.by));
                // Hz(i+1/2, j+1/2, k): Bz uses x at i+1/2; Hz uses y at j+1/2, z at k
                const float cze = (sEy[cur][ty][c + 1] - eyo) * crdx - (sEx[cur][ty + 1][c] - exo) * crdy;
                const float dbz = fmaf(x_cam1_h, o.bz, -x_rp_h * cze);
                hzn = fmaf(y_ca_h, o.hz, y_rp_h * fmaf(z_ph_n, dbz, z_q_n * o.bz));
                if (own && live) {
                    st_at(dH, nb, hxn);
                    st_at(dH, nb + cs, hyn);
                    st_at(dH, nb + cs2, hzn);
                    if (nbx) st_at(dB, nb, o.bx + dbx);
                    if (nby) st_at(dB, nb + cs, o.by + dby);
                    if (nbz) st_at(dB, nb + cs2, o.bz + dbz);
                }
            }
            sHx[ty][c] = hxn;
            sHy[ty][c] = hyn;
            sHz[ty][c] = hzn;
            __syncthreads();

            // ---- D then E of plane k (own columns) ----
            if (own && live) {
                ClassEntry ce;
                if (sizeof(CT) == 1) {
                    ce = sTab[o.c];
                } else {
                    ce.inv_x = ctab[o.c].inv_x;
                    ce.inv_y = ctab[o.c].inv_y;
                    ce.inv_z = ctab[o.c].inv_z;
                    ce.flags = ctab[o.c].flags;
                }
                // Ex(i+1/2, j, k): Dx uses y at j; Ex uses z at k, x at i+1/2
                const float chx = (hzn - sHz[ty - 1][c]) * crdy - (hyn - hy_prev) * crdz;
                const float ddx = fmaf(y_cam1_n, o.dx, y_rp_n * chx);
                float exn = fmaf(z_ca_n, exo, z_rp_n * (ce.inv_x * fmaf(x_ph_h, ddx, x_q_h * o.dx)));
                // Ey(i, j+1/2, k): Dy uses z at k; Ey uses x at i, y at j+1/2
                const float chy = (hxn - hx_prev) * crdz - (hzn - sHz[ty][c - 1]) * crdx;
                const float ddy = fmaf(z_cam1_n, o.dy, z_rp_n * chy);
                float eyn = fmaf(x_ca_n, eyo, x_rp_n * (ce.inv_y * fmaf(y_ph_h, ddy, y_q_h * o.dy)));
                // Ez(i, j, k+1/2): Dz uses x at i; Ez uses y at j, z at k+1/2
                const float chz = (hyn - sHy[ty][c - 1]) * crdx - (hxn - sHx[ty - 1][c]) * crdy;
                float ddz = fmaf(x_cam1_n, o.dz, x_rp_n * chz);
                float ezn = fmaf(y_ca_n, ezo, y_rp_n * (ce.inv_z * fmaf(z_ph_h, ddz, z_q_h * o.dz)));
                if (ce.flags & kSrcEz) {
                    // source edge: the sources' Js enters the D_z curl, and a
                    // resistive source's update is solved for Ez^{n+1}
                    const __attribute__((address_space(1))) int32_t* sn =
                        (const __attribute__((address_space(1))) int32_t*)B.src_node;
                    cgfloat* sj = (cgfloat*)B.src_j;
                    cgfloat* sb = (cgfloat*)B.src_beta;
                    float js = 0.0f, bs = 0.0f;
                    for (int s = 0; s < B.nsrc; ++s)
                        if (sn[s] == node) {
                            js += sj[s * ms + step];
                            bs += sb[s];
                        }
                    const float chs = chz - js;
                    ddz = fmaf(x_cam1_n, o.dz, x_rp_n * chs);
                    ezn = fmaf(y_ca_n, ezo, y_rp_n * (ce.inv_z * fmaf(z_ph_h, ddz, z_q_h * o.dz)));
                    if (bs != 0.0f) ezn = conductive_e(ezo, chs, ce.inv_z, bs);
                }
                exn = (ce.flags & kUpdEx) ? exn : 0.0f;
                eyn = (ce.flags & kUpdEy) ? eyn : 0.0f;
                ezn = (ce.flags & kUpdEz) ? ezn : 0.0f;
                st_at(dE, nb, exn);
                st_at(dE, nb + cs, eyn);
                st_at(dE, nb + cs2, ezn);
                if (nbx) st_at(dD, nb, (ce.flags & kUpdEx) ? o.dx + ddx : o.dx);
                if (nby) st_at(dD, nb + cs, (ce.flags & kUpdEy) ? o.dy + ddy : o.dy);
                if (nbz) st_at(dD, nb + cs2, (ce.flags & kUpdEz) ? o.dz + ddz : o.dz);
                if (ce.flags & kPrbEz) {
                    const __attribute__((address_space(1))) int32_t* pn =
                        (const __attribute__((address_space(1))) int32_t*)B.prb_node;
                    gfloat* ps = (gfloat*)B.prb_series;
                    for (int p = 0; p < B.nprb; ++p)
                        if (pn[p] == node) ps[p * ms + step] = ezn;
                }
                if (ce.flags & kPlnEz)   // plane-DFT sample into ring slot step mod kPlaneRing
                    st_at(B.plane_ring, (uint32_t)(step & (kPlaneRing - 1)) * szb + node0b, ezn);
                bad |= !isfinite(exn + eyn + ezn);
            }
            hx_prev = hxn;
            hy_prev = hyn;
        };
        for (int k = k0; k < ke; k += 2) {
            plane_step(k, s0, cA, cB);
            if (k + 1 < ke) plane_step(k + 1, s1, cB, cA);
        }
        if (bad) *(__attribute__((address_space(1))) int32_t*)B.bad = 1;
    } else {
        // ------------------------------------------------------------ extra wave
        // staging of row TY (columns i0 .. i0+TX-1, TX/64 per lane) and of the
        // columns i0-1 (lanes 0..TY) and i0+TX (lanes 32..32+TY); the new Hy, Hz
        // of the halo column i0-1 for rows 1..TY-1 (lanes 1..TY-1).  Only what
        // the stencil reads is loaded: row TY feeds Hx (Ez) and Hz (Ex) of row
        // TY-1, column i0+TX feeds Hy (Ez) and Hz (Ey) of column i0+TX-1.
        constexpr int R = TX / 64;
        const int jr = j0 - 1 + TY;
        const int cc = lane < 32 ? 0 : TX + 1;          // staging column of this lane
        const int cr = lane & 31;                       // its row
        const bool col_lane = cr <= TY;
        const int ic_ = i0 - 1 + cc, jc_ = j0 - 1 + cr;
        // halo column
        const bool halo = lane >= 1 && lane < TY;
        const int ih = i0 - 1, jh = j0 - 1 + lane;
        const bool h_ok = halo && ih >= 0 && jh >= 0 && jh <= ny;
        const bool hpx = in_px(ih), hpy = in_py(jh);
        const float hx_rp_h = CXf(kRp, 1, ih), hx_ca_h = CXf(kCa, 1, ih), hx_cam1_h = CXf(kCam1, 1, ih);
        const float hy_ph_n = CYf(kPh, 0, jh), hy_q_n = CYf(kQ, 0, jh), hy_ca_h = CYf(kCa, 1, jh),
                    hy_rp_h = CYf(kRp, 1, jh);
        const uint32_t hnode0b = (uint32_t)(ih + jh * sy) * 4u;   // used only where h_ok holds
        struct XStage { float rx[R], rz[R], cx_, cy_, cz_; };
        struct XCol { float hy, hz, by, bz; };
        auto load_xstage = [&](int p) {
            XStage s;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ii = i0 + lane + 64 * r;
                s.rx[r] = ld_at(gE, node_at(ii, jr, p + 1));
                s.rz[r] = ld_at(gE, node_at(ii, jr, p) + cs2);
            }
            const int ii = col_lane ? ic_ : -1;
            s.cx_ = ld_at(gE, node_at(cc == 0 ? ii : -1, jc_, p + 1));
            s.cy_ = ld_at(gE, node_at(ii, jc_, p + 1) + cs);
            s.cz_ = ld_at(gE, node_at(ii, jc_, p) + cs2);
            return s;
        };
        auto load_xcol = [&](int p, XCol& o) {
            const uint32_t n = hnode0b + (uint32_t)p * szb;
            const bool pz = in_pz(p);
            const bool okp = h_ok && p <= nz;
            o.hy = ld_at(gH, (okp ? n : guardb) + cs);
            o.hz = ld_at(gH, (okp ? n : guardb) + cs2);
            o.by = ld_at(gB, (okp && (hpy || pz) ? n : guardb) + cs);
            o.bz = ld_at(gB, (okp && (pz || hpx) ? n : guardb) + cs2);
        };
        {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ii = i0 + lane + 64 * r;
                sEx[0][TY][1 + lane + 64 * r] = ld_at(gE, node_at(ii, jr, k0));
            }
            if (col_lane) {
                sEx[0][cr][cc] = ld_at(gE, node_at(cc == 0 ? ic_ : -1, jc_, k0));
                sEy[0][cr][cc] = ld_at(gE, node_at(ic_, jc_, k0) + cs);
            }
        }
        XStage s0 = load_xstage(k0), s1 = load_xstage(k0 + 1);
        XCol hA, hB;
        load_xcol(k0, hA);
        auto plane_step = [&](int k, XStage& st, const XCol& o, XCol& nxt_col) {
            const int cur = (k - k0) & 1, nxt = cur ^ 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sEx[nxt][TY][1 + lane + 64 * r] = st.rx[r];
                sEz[TY][1 + lane + 64 * r] = st.rz[r];
            }
            if (col_lane) {
                sEx[nxt][cr][cc] = st.cx_;
                sEy[nxt][cr][cc] = st.cy_;
                sEz[cr][cc] = st.cz_;
            }
            st = load_xstage(k + 2);
            load_xcol(k + 1, nxt_col);
            kfloat* czk = cz + k;
            const float z_cam1_h = czk[(kCam1 * 2 + 1) * nz1], z_rp_h = czk[(kRp * 2 + 1) * nz1];
            const float z_ph_n = czk[(kPh * 2 + 0) * nz1], z_q_n = czk[(kQ * 2 + 0) * nz1];
            __syncthreads();
            // Hy, Hz of the halo column i0-1 (needed by Ey, Ez of column i0)
            float hyn = 0.f, hzn = 0.f;
            if (h_ok) {
                const float exo = sEx[cur][lane][0], eyo = sEy[cur][lane][0], ezo = sEz[lane][0];
                const float cye = (sEx[nxt][lane][0] - exo) * crdz - (sEz[lane][1] - ezo) * crdx;
                const float dby = fmaf(z_cam1_h, o.by, -z_rp_h * cye);
                hyn = fmaf(hx_ca_h, o.hy, hx_rp_h * fmaf(hy_ph_n, dby, hy_q_n * o.by));
                const float cze = (sEy[cur][lane][1] - eyo) * crdx - (sEx[cur][lane + 1][0] - exo) * crdy;
                const float dbz = fmaf(hx_cam1_h, o.bz, -hx_rp_h * cze);
                hzn = fmaf(hy_ca_h, o.hz, hy_rp_h * fmaf(z_ph_n, dbz, z_q_n * o.bz));
            }
            if (halo) {
                sHy[lane][0] = hyn;
                sHz[lane][0] = hzn;
            }
            __syncthreads();
        };
        for (int k = k0; k < ke; k += 2) {
            plane_step(k, s0, hA, hB);
            if (k + 1 < ke) plane_step(k + 1, s1, hB, hA);
        }
    }
}

// Advance each board's device step counter by n after a batch of launches.
// Advance each board's device counters after a batch of launches: n[2b] steps
// done in n[2b+1] launches (each launch swaps the field buffers).
__global__ void advance_steps(BoardDev* boards, int nb, const int64_t* n)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) {
        boards[b].step[0] += n[2 * b];
        boards[b].step[1] = (boards[b].step[1] + n[2 * b + 1]) & 1;
    }
}

__global__ void advance_one(int64_t* step, int64_t n, int64_t launches)
{
    if (threadIdx.x == 0) {
        step[0] += n;
        step[1] = (step[1] + launches) & 1;
    }
}

// Running DFT (FP64): for probe p and frequency q add the samples s in [s0, s1):
// A += e[s] * exp(-i 2 pi f_q (s+1) dt) * dt.  The phase is reduced to [0, 1)
// turns in FP64 before sincospi.
// With `step` set, the range is the last `back` steps before the device step
// counter, [step[0] - back, step[0]) (a replayed graph's call advances it).
__global__ void dft_accumulate(const float* __restrict__ series, int64_t max_steps,
                               const double* __restrict__ freqs, int nf, int np,
                               double dt, int64_t s0, int64_t s1, const int64_t* __restrict__ step,
                               int64_t back, double* __restrict__ re, double* __restrict__ im)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (q >= nf || p >= np) return;
    if (step) {
        s1 = step[0];
        s0 = s1 - back;
    }
    const double fdt = freqs[q] * dt;
    double ar = 0.0, ai = 0.0;
    const float* e = series + (int64_t)p * max_steps;
    for (int64_t s = s0; s < s1; ++s) {
        double turns = fdt * (double)(s + 1);
        turns -= floor(turns);
        double sn, cs;
        sincospi(2.0 * turns, &sn, &cs);
        const double v = (double)e[s];
        ar = fma(v, cs, ar);
        ai = fma(-v, sn, ai);
    }
    re[p * nf + q] += ar * dt;
    im[p * nf + q] += ai * dt;
}

// Twiddles of one fold: tw[f][q] = (cos, -sin)(2 pi f (s0 + q + 1) dt) * dt for
// the steps s0 + q of the fold (s0 = device step counter + rel_from), computed
// once per fold so that the fold reads them as wave-uniform scalar loads.
__global__ __launch_bounds__(256) void plane_twiddle(const double* __restrict__ freqs, int nf,
                                                     double dt, const int64_t* __restrict__ step,
                                                     int64_t rel_from, int n, double* __restrict__ tw)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nf * kPlaneRing) return;
    const int f = t / kPlaneRing, q = t % kPlaneRing;
    double cs = 0.0, sn = 0.0;
    if (q < n) {
        double turns = freqs[f] * dt * (double)(step[0] + rel_from + q + 1);
        turns -= floor(turns);
        sincospi(2.0 * turns, &sn, &cs);
    }
    tw[2 * t] = cs * dt;
    tw[2 * t + 1] = -sn * dt;
}

// Fold the ring samples of steps [s0, s1) (s1 - s0 = n <= kPlaneRing; s0, s1 are
// the device step counter plus rel_from, rel_to) into the plane accumulators:
// A_f(node) += e_s(node) exp(-i 2 pi f (s+1) dt) dt for each s in order, the
// probe DFT's definition applied to every node of the plane.  Every sample is
// added to the accumulator on its own, so the result does not depend on how the
// steps were grouped into folds.  One thread per node (padded row layout); the
// twiddles come from plane_twiddle's table through the scalar cache.
__global__ __launch_bounds__(256) void plane_fold(const float* __restrict__ ring, int64_t plane_nodes,
                                                  int nf, const int64_t* __restrict__ step,
                                                  int64_t rel_from, int n,
                                                  const double* __restrict__ tw,
                                                  double* __restrict__ re, double* __restrict__ im)
{
    const int64_t s0 = step[0] + rel_from;
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= plane_nodes) return;
    float e[kPlaneRing];
#pragma unroll
    for (int q = 0; q < kPlaneRing; ++q)
        e[q] = q < n ? ring[(int64_t)((s0 + q) & (kPlaneRing - 1)) * plane_nodes + node] : 0.0f;
    // the next frequency's accumulators are loaded while this one's are summed
    double ar = re[node], ai = im[node];
    for (int f = 0; f < nf; ++f) {
        const int64_t a = (int64_t)f * plane_nodes + node;
        double nr = 0.0, ni = 0.0;
        if (f + 1 < nf) {
            nr = re[a + plane_nodes];
            ni = im[a + plane_nodes];
        }
        const double* w = tw + 2 * kPlaneRing * f;
        // slots q >= n hold e = 0 and zero twiddles: those terms add exact zeros
#pragma unroll
        for (int q = 0; q < kPlaneRing; ++q) {
            const double v = (double)e[q];
            ar = fma(v, w[2 * q], ar);
            ai = fma(v, w[2 * q + 1], ai);
        }
        re[a] = ar;
        im[a] = ai;
        ar = nr;
        ai = ni;
    }
}

// Zero-padded complex FP64 input for the probe FFT.
__global__ void fft_load(const float* __restrict__ series, int64_t n_samples, int n_fft,
                         double2* __restrict__ out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_fft) return;
    out[s] = make_double2(s < n_samples ? (double)series[s] : 0.0, 0.0);
}

// One radix-2 Stockham pass (natural-order output after log2(n) passes):
// for j < n/2 with span ns: v0 = x[j], v1 = x[j + n/2] * exp(-2 pi i (j mod ns) / (2 ns)),
// y[(j/ns)*2ns + j%ns] = v0 + v1, y[... + ns] = v0 - v1.
__global__ void fft_pass(const double2* __restrict__ x, double2* __restrict__ y, int n, int ns)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n / 2) return;
    const int r = j % ns;
    double sn, cs;
    sincospi(-(double)r / (double)ns, &sn, &cs);
    const double2 a = x[j];
    const double2 b0 = x[j + n / 2];
    const double2 b = make_double2(b0.x * cs - b0.y * sn, b0.x * sn + b0.y * cs);
    const int o = (j / ns) * 2 * ns + r;
    y[o] = make_double2(a.x + b.x, a.y + b.y);
    y[o + ns] = make_double2(a.x - b.x, a.y - b.y);
}

// Plain fill, used instead of memset so the stream's work stays capturable.
__global__ void fill_zero(float* __restrict__ p, int64_t n)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0.0f;
}

// ---------------------------------------------------------------------------
// launchers (host side)

struct Shape {
    int tx, ty;
};
static const Shape kShapes[] = {{64, 15}, {64, 12}, {64, 8},  {64, 4},  {64, 10},
                                {64, 14}, {128, 7}, {128, 4}, {128, 6}, {128, 5}};
static const int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int num_shapes() { return kNumShapes; }
void shape_at(int s, int* tx, int* ty)
{
    *tx = kShapes[s].tx;
    *ty = kShapes[s].ty;
}

template <int TX, int TY>
static hipError_t launch_tt(const BoardDev* boards, const TileRef* tiles, int ntiles, int rel,
                            int flip, bool wide, hipStream_t st)
{
    if (wide)
        hipLaunchKernelGGL((field_step<TX, TY, uint16_t>), dim3(ntiles), dim3(TX * TY + 64), 0, st,
                           boards, tiles, rel, flip);
    else
        hipLaunchKernelGGL((field_step<TX, TY, uint8_t>), dim3(ntiles), dim3(TX * TY + 64), 0, st,
                           boards, tiles, rel, flip);
    return hipGetLastError();
}

template <int TX, int TY>
static int occupancy_tt(bool wide)
{
    int n = 0;
    hipError_t e = wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &n, field_step<TX, TY, uint16_t>, TX * TY + 64, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &n, field_step<TX, TY, uint8_t>, TX * TY + 64, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

// Blocks of the field kernel that one compute unit holds at once.
int field_step_occupancy(int tile_x, int tile_y, bool wide)
{
#define SHAPE(X, Y) \
    if (tile_x == X && tile_y == Y) return occupancy_tt<X, Y>(wide);
    SHAPE(64, 15) SHAPE(64, 12) SHAPE(64, 8) SHAPE(64, 4) SHAPE(64, 10) SHAPE(64, 14)
    SHAPE(128, 7) SHAPE(128, 4) SHAPE(128, 6) SHAPE(128, 5)
#undef SHAPE
    return 1;
}

hipError_t launch_field_step(int tile_x, int tile_y, const BoardDev* boards,
                             const TileRef* tiles, int ntiles, int rel, int flip, bool wide,
                             hipStream_t st)
{
#define SHAPE(X, Y) \
    if (tile_x == X && tile_y == Y) return launch_tt<X, Y>(boards, tiles, ntiles, rel, flip, wide, st);
    SHAPE(64, 15) SHAPE(64, 12) SHAPE(64, 8) SHAPE(64, 4) SHAPE(64, 10) SHAPE(64, 14)
    SHAPE(128, 7) SHAPE(128, 4) SHAPE(128, 6) SHAPE(128, 5)
#undef SHAPE
    return hipErrorInvalidValue;
}

hipError_t launch_advance(BoardDev* boards, int nb, const int64_t* n, hipStream_t st)
{
    hipLaunchKernelGGL(advance_steps, dim3((nb + 63) / 64), dim3(64), 0, st, boards, nb, n);
    return hipGetLastError();
}

hipError_t launch_advance_one(int64_t* step, int64_t n, int64_t launches, hipStream_t st)
{
    hipLaunchKernelGGL(advance_one, dim3(1), dim3(64), 0, st, step, n, launches);
    return hipGetLastError();
}

hipError_t launch_dft(const float* series, int64_t max_steps, const double* freqs, int nf,
                      int np, double dt, int64_t s0, int64_t s1, double* re, double* im,
                      hipStream_t st)
{
    if (np <= 0 || nf <= 0 || s1 <= s0) return hipSuccess;
    dim3 grid((nf + 63) / 64, np);
    hipLaunchKernelGGL(dft_accumulate, grid, dim3(64), 0, st, series, max_steps, freqs, nf, np,
                       dt, s0, s1, (const int64_t*)nullptr, (int64_t)0, re, im);
    return hipGetLastError();
}

hipError_t launch_dft_back(const float* series, int64_t max_steps, const double* freqs, int nf,
                           int np, double dt, const int64_t* step, int64_t back, double* re,
                           double* im, hipStream_t st)
{
    if (np <= 0 || nf <= 0 || back <= 0) return hipSuccess;
    dim3 grid((nf + 63) / 64, np);
    hipLaunchKernelGGL(dft_accumulate, grid, dim3(64), 0, st, series, max_steps, freqs, nf, np,
                       dt, (int64_t)0, (int64_t)0, step, back, re, im);
    return hipGetLastError();
}

hipError_t launch_plane_fold(const float* ring, int64_t plane_nodes, const double* freqs, int nf,
                             double dt, const int64_t* step, int64_t rel_from, int64_t rel_to,
                             double* tw, double* re, double* im, hipStream_t st)
{
    if (nf <= 0 || rel_to <= rel_from) return hipSuccess;
    if (rel_to - rel_from > kPlaneRing) return hipErrorInvalidValue;
    const int n = (int)(rel_to - rel_from);
    hipLaunchKernelGGL(plane_twiddle, dim3((unsigned)((nf * kPlaneRing + 255) / 256)), dim3(256), 0,
                       st, freqs, nf, dt, step, rel_from, n, tw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(plane_fold, dim3((unsigned)((plane_nodes + 255) / 256)), dim3(256), 0, st,
                       ring, plane_nodes, nf, step, rel_from, n, (const double*)tw, re, im);
    return hipGetLastError();
}

hipError_t launch_fft(const float* series, int64_t n_samples, int n_fft, double2* a, double2* b,
                      double2** result, hipStream_t st)
{
    hipLaunchKernelGGL(fft_load, dim3((n_fft + 255) / 256), dim3(256), 0, st, series, n_samples,
                       n_fft, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double2* x = a;
    double2* y = b;
    for (int ns = 1; ns < n_fft; ns *= 2) {
        hipLaunchKernelGGL(fft_pass, dim3((n_fft / 2 + 255) / 256), dim3(256), 0, st, x, y, n_fft,
                           ns);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        double2* tmp = x;
        x = y;
        y = tmp;
    }
    *result = x;
    return hipSuccess;
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace fdtd
