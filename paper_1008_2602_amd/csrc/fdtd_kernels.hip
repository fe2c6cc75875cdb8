// gfx950 kernels of libfdtd.
//
// field_step: one full leapfrog step (Model section: B->H then D->E, Eqs. 1-4)
// for one tile of columns of one board, fused in a single pass.  A block owns a
// (TX-1) x (TY-1) patch of (i, j) columns and marches along z.  Per z plane it
//   1. stages E^n of planes k+1 (Ex, Ey) and k (Ez) for (TX+1) x (TY+1) columns
//      in LDS (Ex, Ey of plane k are kept from the previous plane),
//   2. computes B/H^{n+1/2} of plane k for all TX x TY columns (the first column
//      and row are a halo owned by the neighbouring tiles, recomputed here so
//      that no second pass over H is needed),
//   3. computes D/E^{n+1} of plane k for the owned columns from the new H of
//      planes k (LDS) and k-1 (registers).
// State is ping-ponged (E, H, B read from one copy, written to the other) so
// halo recomputation never sees a neighbour's already-updated values; D is only
// read by its owner and is updated in place.  D and B are stored and moved only
// where a PML loss acts on them (elsewhere the update reduces to plain Yee with
// those terms exactly zero).  Sources and probes are folded into the same pass
// through per-node material classes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdtd_internal.h"

namespace fdtd {

// Global-address-space views of the board's buffers: loads and stores through
// them are global_* instructions (counted in vmcnt only), so LDS barriers never
// wait on outstanding HBM traffic.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) const float cgfloat;
typedef __attribute__((address_space(4))) const float kfloat;  // uniform, scalar loads

// Branch-free staging load: out-of-range nodes read the guard word (index
// `guard`, one past the last node, kept at zero) instead of selecting after
// the load, so the load's latency is not exposed where it is issued.
__device__ __forceinline__ float ld_or0(cgfloat* __restrict__ p, int i, int j, int k, int nx,
                                        int ny, int nz, int sy, int sz, int guard)
{
    const bool ok = ((unsigned)i <= (unsigned)nx) & ((unsigned)j <= (unsigned)ny) &
                    ((unsigned)k <= (unsigned)nz);
    return p[ok ? i + j * sy + k * sz : guard];
}

// Hardware dispatches block b to XCD b % 8.  Map blocks so that each XCD walks
// a contiguous run of the tile list (neighbouring tiles share halos in its L2).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int x = b & 7, slot = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + slot;
}

template <int TX, int TY, typename CT>
__global__ __launch_bounds__(TX* TY) void field_step(const BoardDev* __restrict__ boards,
                                                     const TileRef* __restrict__ tiles,
                                                     int rel)
{
    __shared__ float sEx[2][TY + 1][TX + 1];
    __shared__ float sEy[2][TY + 1][TX + 1];
    __shared__ float sEz[TY + 1][TX + 1];
    __shared__ float sHx[TY][TX];
    __shared__ float sHy[TY][TX];
    __shared__ float sHz[TY][TX];
    // class table in LDS when the class index is one byte (<= 256 classes)
    constexpr int kLdsClasses = sizeof(CT) == 1 ? 256 : 1;
    __shared__ ClassEntry sTab[kLdsClasses];

    const TileRef t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BoardDev& B = boards[t.board];
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int sy = nx + 1, sz = (nx + 1) * (ny + 1), guard = sz * (nz + 1);
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int ox = t.tx * (TX - 1) - 1, oy = t.ty * (TY - 1) - 1;
    const int i = ox + tx, j = oy + ty;
    const bool col_ok = (i >= 0) && (i <= nx) && (j >= 0) && (j <= ny);
    const bool own = col_ok && tx > 0 && ty > 0;
    const int64_t step = *B.step + rel;
    const int par = (int)(step & 1);
    cgfloat* __restrict__ gEx = (cgfloat*)B.f[par][0];
    cgfloat* __restrict__ gEy = (cgfloat*)B.f[par][1];
    cgfloat* __restrict__ gEz = (cgfloat*)B.f[par][2];
    cgfloat* __restrict__ gHx = (cgfloat*)B.f[par][3];
    cgfloat* __restrict__ gHy = (cgfloat*)B.f[par][4];
    cgfloat* __restrict__ gHz = (cgfloat*)B.f[par][5];
    cgfloat* __restrict__ gBx = (cgfloat*)B.f[par][6];
    cgfloat* __restrict__ gBy = (cgfloat*)B.f[par][7];
    cgfloat* __restrict__ gBz = (cgfloat*)B.f[par][8];
    gfloat* __restrict__ dEx = (gfloat*)B.f[par ^ 1][0];
    gfloat* __restrict__ dEy = (gfloat*)B.f[par ^ 1][1];
    gfloat* __restrict__ dEz = (gfloat*)B.f[par ^ 1][2];
    gfloat* __restrict__ dHx = (gfloat*)B.f[par ^ 1][3];
    gfloat* __restrict__ dHy = (gfloat*)B.f[par ^ 1][4];
    gfloat* __restrict__ dHz = (gfloat*)B.f[par ^ 1][5];
    gfloat* __restrict__ dBx = (gfloat*)B.f[par ^ 1][6];
    gfloat* __restrict__ dBy = (gfloat*)B.f[par ^ 1][7];
    gfloat* __restrict__ dBz = (gfloat*)B.f[par ^ 1][8];
    gfloat* __restrict__ Dx = (gfloat*)B.d[0];
    gfloat* __restrict__ Dy = (gfloat*)B.d[1];
    gfloat* __restrict__ Dz = (gfloat*)B.d[2];
    const __attribute__((address_space(1))) CT* __restrict__ cls =
        (const __attribute__((address_space(1))) CT*)B.cls;
    const __attribute__((address_space(1))) ClassEntry* __restrict__ ctab =
        (const __attribute__((address_space(1))) ClassEntry*)B.ctab;
    const float crdx = B.crd_x, crdy = B.crd_y, crdz = B.crd_z;
    const int pml_zlo = B.pml[4], pml_zhi = B.pml[5];

    // PML membership of this column (x, y); per plane for z: where D/B are kept
    const bool px = (i < B.pml[0]) || (B.pml[1] > 0 && i >= nx - B.pml[1]);
    const bool py = (j < B.pml[2]) || (B.pml[3] > 0 && j >= ny - B.pml[3]);
    auto in_pz = [&](int k) { return (k < pml_zlo) || (pml_zhi > 0 && k >= nz - pml_zhi); };

    // per-axis coefficients of this column (node n / half node h)
    const int ic = min(max(i, 0), nx), jc = min(max(j, 0), ny);
    cgfloat* __restrict__ cx = (cgfloat*)B.coef[0];
    cgfloat* __restrict__ cy = (cgfloat*)B.coef[1];
    kfloat* __restrict__ cz = (kfloat*)B.coef[2];
    const int nx1 = nx + 1, ny1 = ny + 1, nz1 = nz + 1;
#define CX(kind, half) cx[((kind) * 2 + (half)) * nx1 + ic]
#define CY(kind, half) cy[((kind) * 2 + (half)) * ny1 + jc]
    const float x_cam1_n = CX(kCam1, 0), x_ca_n = CX(kCa, 0), x_rp_n = CX(kRp, 0),
                x_ph_n = CX(kPh, 0), x_q_n = CX(kQ, 0);
    const float x_cam1_h = CX(kCam1, 1), x_ca_h = CX(kCa, 1), x_rp_h = CX(kRp, 1),
                x_ph_h = CX(kPh, 1), x_q_h = CX(kQ, 1);
    const float y_cam1_n = CY(kCam1, 0), y_ca_n = CY(kCa, 0), y_rp_n = CY(kRp, 0),
                y_ph_n = CY(kPh, 0), y_q_n = CY(kQ, 0);
    const float y_cam1_h = CY(kCam1, 1), y_ca_h = CY(kCa, 1), y_rp_h = CY(kRp, 1),
                y_ph_h = CY(kPh, 1), y_q_h = CY(kQ, 1);
#undef CX
#undef CY

    // extra staging element of this thread: column a = TX (rows 0..TY) or row
    // b = TY (columns 0..TX-1); the rest of the block stages nothing extra
    const bool has_extra = tid < TY + 1 + TX;
    const int ea = tid < TY + 1 ? TX : tid - (TY + 1);
    const int eb = tid < TY + 1 ? tid : TY;
    const int ei = ox + ea, ej = oy + eb;

    // prologue: Ex, Ey of plane 0 into LDS slot 0; prefetch plane 0's operands
    sEx[0][ty][tx] = ld_or0(gEx, i, j, 0, nx, ny, nz, sy, sz, guard);
    sEy[0][ty][tx] = ld_or0(gEy, i, j, 0, nx, ny, nz, sy, sz, guard);
    if (has_extra) {
        sEx[0][eb][ea] = ld_or0(gEx, ei, ej, 0, nx, ny, nz, sy, sz, guard);
        sEy[0][eb][ea] = ld_or0(gEy, ei, ej, 0, nx, ny, nz, sy, sz, guard);
    }
    // prefetched operands of the plane about to be computed
    float pEx = ld_or0(gEx, i, j, 1, nx, ny, nz, sy, sz, guard);
    float pEy = ld_or0(gEy, i, j, 1, nx, ny, nz, sy, sz, guard);
    float pEz = ld_or0(gEz, i, j, 0, nx, ny, nz, sy, sz, guard);
    float qEx = 0.f, qEy = 0.f, qEz = 0.f;
    if (has_extra) {
        qEx = ld_or0(gEx, ei, ej, 1, nx, ny, nz, sy, sz, guard);
        qEy = ld_or0(gEy, ei, ej, 1, nx, ny, nz, sy, sz, guard);
        qEz = ld_or0(gEz, ei, ej, 0, nx, ny, nz, sy, sz, guard);
    }
    const int node0 = i + j * sy;
    float pHx = 0.f, pHy = 0.f, pHz = 0.f, pBx = 0.f, pBy = 0.f, pBz = 0.f;
    float pDx = 0.f, pDy = 0.f, pDz = 0.f;
    CT pC = 0;
    if (sizeof(CT) == 1) {
        for (int e = tid; e < kLdsClasses; e += TX * TY) {
            const int c = min(e, B.nclass - 1);
            sTab[e].inv_x = ctab[c].inv_x;
            sTab[e].inv_y = ctab[c].inv_y;
            sTab[e].inv_z = ctab[c].inv_z;
            sTab[e].flags = ctab[c].flags;
        }
    }
    {
        const bool pz0 = in_pz(0);
        if (col_ok) {
            pHx = gHx[node0];
            pHy = gHy[node0];
            pHz = gHz[node0];
            if (px || py) pBx = gBx[node0];
            if (py || pz0) pBy = gBy[node0];
            if (pz0 || px) pBz = gBz[node0];
        }
        if (own) {
            pC = cls[node0];
            if (px || py) pDx = Dx[node0];
            if (py || pz0) pDy = Dy[node0];
            if (pz0 || px) pDz = Dz[node0];
        }
    }
    float hx_prev = 0.0f, hy_prev = 0.0f;
    const int64_t ms = B.max_steps;

    for (int k = 0; k <= nz; ++k) {
        const int cur = k & 1, nxt = cur ^ 1;
        const bool pz = in_pz(k);
        const bool nbx = px || py, nby = py || pz, nbz = pz || px;
        const int node = node0 + k * sz;

        // ---- stage this plane's prefetched E into LDS, take own operands ----
        sEx[nxt][ty][tx] = pEx;
        sEy[nxt][ty][tx] = pEy;
        sEz[ty][tx] = pEz;
        if (has_extra) {
            sEx[nxt][eb][ea] = qEx;
            sEy[nxt][eb][ea] = qEy;
            sEz[eb][ea] = qEz;
        }
        const float hxo = pHx, hyo = pHy, hzo = pHz, bxo = pBx, byo = pBy, bzo = pBz;
        const float dxo = pDx, dyo = pDy, dzo = pDz;
        const CT c = pC;

        // ---- prefetch the next plane's operands (in flight during this plane) ----
        if (k < nz) {
            const int k1 = k + 1;
            const bool pz1 = in_pz(k1);
            pEx = ld_or0(gEx, i, j, k1 + 1, nx, ny, nz, sy, sz, guard);
            pEy = ld_or0(gEy, i, j, k1 + 1, nx, ny, nz, sy, sz, guard);
            pEz = ld_or0(gEz, i, j, k1, nx, ny, nz, sy, sz, guard);
            if (has_extra) {
                qEx = ld_or0(gEx, ei, ej, k1 + 1, nx, ny, nz, sy, sz, guard);
                qEy = ld_or0(gEy, ei, ej, k1 + 1, nx, ny, nz, sy, sz, guard);
                qEz = ld_or0(gEz, ei, ej, k1, nx, ny, nz, sy, sz, guard);
            }
            const int n1 = node + sz;
            if (col_ok) {
                pHx = gHx[n1];
                pHy = gHy[n1];
                pHz = gHz[n1];
                pBx = (px || py) ? gBx[n1] : 0.f;
                pBy = (py || pz1) ? gBy[n1] : 0.f;
                pBz = (pz1 || px) ? gBz[n1] : 0.f;
            }
            if (own) {
                pC = cls[n1];
                pDx = (px || py) ? Dx[n1] : 0.f;
                pDy = (py || pz1) ? Dy[n1] : 0.f;
                pDz = (pz1 || px) ? Dz[n1] : 0.f;
            }
        }
        // z coefficients of this plane (uniform over the block)
        kfloat* czk = cz + k;
        const float z_cam1_n = czk[(kCam1 * 2 + 0) * nz1], z_ca_n = czk[(kCa * 2 + 0) * nz1],
                    z_rp_n = czk[(kRp * 2 + 0) * nz1], z_ph_n = czk[(kPh * 2 + 0) * nz1],
                    z_q_n = czk[(kQ * 2 + 0) * nz1];
        const float z_cam1_h = czk[(kCam1 * 2 + 1) * nz1], z_ca_h = czk[(kCa * 2 + 1) * nz1],
                    z_rp_h = czk[(kRp * 2 + 1) * nz1], z_ph_h = czk[(kPh * 2 + 1) * nz1],
                    z_q_h = czk[(kQ * 2 + 1) * nz1];
        __syncthreads();

        // ---- B then H of plane k (own + halo columns) ----
        float hxn = 0.f, hyn = 0.f, hzn = 0.f;
        const float exo = sEx[cur][ty][tx], eyo = sEy[cur][ty][tx], ezo = sEz[ty][tx];
        if (col_ok) {
            // Hx(i, j+1/2, k+1/2): Bx uses y at j+1/2; Hx uses z at k+1/2, x at i
            const float cxe = (sEz[ty + 1][tx] - ezo) * crdy - (sEy[nxt][ty][tx] - eyo) * crdz;
            const float dbx = fmaf(y_cam1_h, bxo, -y_rp_h * cxe);
            hxn = fmaf(z_ca_h, hxo, z_rp_h * fmaf(x_ph_n, dbx, x_q_n * bxo));
            // Hy(i+1/2, j, k+1/2): By uses z at k+1/2; Hy uses x at i+1/2, y at j
            const float cye = (sEx[nxt][ty][tx] - exo) * crdz - (sEz[ty][tx + 1] - ezo) * crdx;
            const float dby = fmaf(z_cam1_h, byo, -z_rp_h * cye);
            hyn = fmaf(x_ca_h, hyo, x_rp_h * fmaf(y_ph_n, dby, y_q_n * byo));
            // Hz(i+1/2, j+1/2, k): Bz uses x at i+1/2; Hz uses y at j+1/2, z at k
            const float cze =
                (sEy[cur][ty][tx + 1] - eyo) * crdx - (sEx[cur][ty + 1][tx] - exo) * crdy;
            const float dbz = fmaf(x_cam1_h, bzo, -x_rp_h * cze);
            hzn = fmaf(y_ca_h, hzo, y_rp_h * fmaf(z_ph_n, dbz, z_q_n * bzo));
            if (own) {
                dHx[node] = hxn;
                dHy[node] = hyn;
                dHz[node] = hzn;
                if (nbx) dBx[node] = bxo + dbx;
                if (nby) dBy[node] = byo + dby;
                if (nbz) dBz[node] = bzo + dbz;
            }
        }
        sHx[ty][tx] = hxn;
        sHy[ty][tx] = hyn;
        sHz[ty][tx] = hzn;
        __syncthreads();

        // ---- D then E of plane k (own columns) ----
        if (own) {
            ClassEntry ce;
            if (sizeof(CT) == 1) {
                ce = sTab[c];
            } else {
                ce.inv_x = ctab[c].inv_x;
                ce.inv_y = ctab[c].inv_y;
                ce.inv_z = ctab[c].inv_z;
                ce.flags = ctab[c].flags;
            }
            // Ex(i+1/2, j, k): Dx uses y at j; Ex uses z at k, x at i+1/2
            const float chx = (hzn - sHz[ty - 1][tx]) * crdy - (hyn - hy_prev) * crdz;
            const float ddx = fmaf(y_cam1_n, dxo, y_rp_n * chx);
            float exn = fmaf(z_ca_n, exo, z_rp_n * (ce.inv_x * fmaf(x_ph_h, ddx, x_q_h * dxo)));
            // Ey(i, j+1/2, k): Dy uses z at k; Ey uses x at i, y at j+1/2
            const float chy = (hxn - hx_prev) * crdz - (hzn - sHz[ty][tx - 1]) * crdx;
            const float ddy = fmaf(z_cam1_n, dyo, z_rp_n * chy);
            float eyn = fmaf(x_ca_n, eyo, x_rp_n * (ce.inv_y * fmaf(y_ph_h, ddy, y_q_h * dyo)));
            // Ez(i, j, k+1/2): Dz uses x at i; Ez uses y at j, z at k+1/2
            float js = 0.0f;
            if (ce.flags & kSrcEz) {
                const __attribute__((address_space(1))) int32_t* sn =
                    (const __attribute__((address_space(1))) int32_t*)B.src_node;
                cgfloat* sj = (cgfloat*)B.src_j;
                for (int s = 0; s < B.nsrc; ++s)
                    if (sn[s] == node) js += sj[s * ms + step];
            }
            const float chz =
                ((hyn - sHy[ty][tx - 1]) * crdx - (hxn - sHx[ty - 1][tx]) * crdy) - js;
            const float ddz = fmaf(x_cam1_n, dzo, x_rp_n * chz);
            float ezn = fmaf(y_ca_n, ezo, y_rp_n * (ce.inv_z * fmaf(z_ph_h, ddz, z_q_h * dzo)));
            exn = (ce.flags & kUpdEx) ? exn : 0.0f;
            eyn = (ce.flags & kUpdEy) ? eyn : 0.0f;
            ezn = (ce.flags & kUpdEz) ? ezn : 0.0f;
            dEx[node] = exn;
            dEy[node] = eyn;
            dEz[node] = ezn;
            if (nbx && (ce.flags & kUpdEx)) Dx[node] = dxo + ddx;
            if (nby && (ce.flags & kUpdEy)) Dy[node] = dyo + ddy;
            if (nbz && (ce.flags & kUpdEz)) Dz[node] = dzo + ddz;
            if (ce.flags & kPrbEz) {
                const __attribute__((address_space(1))) int32_t* pn =
                    (const __attribute__((address_space(1))) int32_t*)B.prb_node;
                gfloat* ps = (gfloat*)B.prb_series;
                for (int p = 0; p < B.nprb; ++p)
                    if (pn[p] == node) ps[p * ms + step] = ezn;
            }
            if (!isfinite(exn + eyn + ezn)) *(__attribute__((address_space(1))) int32_t*)B.bad = 1;
        }
        hx_prev = hxn;
        hy_prev = hyn;
    }
}

// Advance each board's device step counter by n after a batch of launches.
__global__ void advance_steps(BoardDev* boards, int nb, const int64_t* n)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) *boards[b].step += n[b];
}

__global__ void advance_one(int64_t* step, int64_t n)
{
    if (threadIdx.x == 0) *step += n;
}

// Running DFT (FP64): for probe p and frequency q add the samples s in [s0, s1):
// A += e[s] * exp(-i 2 pi f_q (s+1) dt) * dt.  The phase is reduced to [0, 1)
// turns in FP64 before sincospi.
__global__ void dft_accumulate(const float* __restrict__ series, int64_t max_steps,
                               const double* __restrict__ freqs, int nf, int np,
                               double dt, int64_t s0, int64_t s1,
                               double* __restrict__ re, double* __restrict__ im)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (q >= nf || p >= np) return;
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
static const Shape kShapes[] = {{64, 8}, {64, 4}, {64, 16}, {128, 4}, {32, 8}, {32, 16}};
static const int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int num_shapes() { return kNumShapes; }
void shape_at(int s, int* tx, int* ty)
{
    *tx = kShapes[s].tx;
    *ty = kShapes[s].ty;
}

template <int TX, int TY>
static hipError_t launch_tt(const BoardDev* boards, const TileRef* tiles, int ntiles, int rel,
                            bool wide, hipStream_t st)
{
    if (wide)
        hipLaunchKernelGGL((field_step<TX, TY, uint16_t>), dim3(ntiles), dim3(TX * TY), 0, st,
                           boards, tiles, rel);
    else
        hipLaunchKernelGGL((field_step<TX, TY, uint8_t>), dim3(ntiles), dim3(TX * TY), 0, st,
                           boards, tiles, rel);
    return hipGetLastError();
}

hipError_t launch_field_step(int tile_x, int tile_y, const BoardDev* boards,
                             const TileRef* tiles, int ntiles, int rel, bool wide,
                             hipStream_t st)
{
    if (tile_x == 64 && tile_y == 8) return launch_tt<64, 8>(boards, tiles, ntiles, rel, wide, st);
    if (tile_x == 64 && tile_y == 4) return launch_tt<64, 4>(boards, tiles, ntiles, rel, wide, st);
    if (tile_x == 64 && tile_y == 16) return launch_tt<64, 16>(boards, tiles, ntiles, rel, wide, st);
    if (tile_x == 128 && tile_y == 4) return launch_tt<128, 4>(boards, tiles, ntiles, rel, wide, st);
    if (tile_x == 32 && tile_y == 8) return launch_tt<32, 8>(boards, tiles, ntiles, rel, wide, st);
    if (tile_x == 32 && tile_y == 16) return launch_tt<32, 16>(boards, tiles, ntiles, rel, wide, st);
    return hipErrorInvalidValue;
}

hipError_t launch_advance(BoardDev* boards, int nb, const int64_t* n, hipStream_t st)
{
    hipLaunchKernelGGL(advance_steps, dim3((nb + 63) / 64), dim3(64), 0, st, boards, nb, n);
    return hipGetLastError();
}

hipError_t launch_advance_one(int64_t* step, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(advance_one, dim3(1), dim3(64), 0, st, step, n);
    return hipGetLastError();
}

hipError_t launch_dft(const float* series, int64_t max_steps, const double* freqs, int nf,
                      int np, double dt, int64_t s0, int64_t s1, double* re, double* im,
                      hipStream_t st)
{
    if (np <= 0 || nf <= 0 || s1 <= s0) return hipSuccess;
    dim3 grid((nf + 63) / 64, np);
    hipLaunchKernelGGL(dft_accumulate, grid, dim3(64), 0, st, series, max_steps, freqs, nf, np,
                       dt, s0, s1, re, im);
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
