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

__device__ __forceinline__ float ld_or0(const float* __restrict__ p, int i, int j, int k,
                                        int nx, int ny, int nz, int sy, int sz)
{
    return (i >= 0 && i <= nx && j >= 0 && j <= ny && k >= 0 && k <= nz)
               ? p[i + j * sy + k * sz]
               : 0.0f;
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

    const TileRef t = tiles[blockIdx.x];
    const BoardDev& B = boards[t.board];
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int sy = nx + 1, sz = (nx + 1) * (ny + 1);
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int ox = t.tx * (TX - 1) - 1, oy = t.ty * (TY - 1) - 1;
    const int i = ox + tx, j = oy + ty;
    const bool col_ok = (i >= 0) && (i <= nx) && (j >= 0) && (j <= ny);
    const bool own = col_ok && tx > 0 && ty > 0;
    const int64_t step = *B.step + rel;
    const int par = (int)(step & 1);
    const float* __restrict__ sEx_g = B.f[par][0];
    const float* __restrict__ sEy_g = B.f[par][1];
    const float* __restrict__ sEz_g = B.f[par][2];
    const float* __restrict__ hxo_g = B.f[par][3];
    const float* __restrict__ hyo_g = B.f[par][4];
    const float* __restrict__ hzo_g = B.f[par][5];
    const float* __restrict__ bxo_g = B.f[par][6];
    const float* __restrict__ byo_g = B.f[par][7];
    const float* __restrict__ bzo_g = B.f[par][8];
    float* __restrict__ dEx = B.f[par ^ 1][0];
    float* __restrict__ dEy = B.f[par ^ 1][1];
    float* __restrict__ dEz = B.f[par ^ 1][2];
    float* __restrict__ dHx = B.f[par ^ 1][3];
    float* __restrict__ dHy = B.f[par ^ 1][4];
    float* __restrict__ dHz = B.f[par ^ 1][5];
    float* __restrict__ dBx = B.f[par ^ 1][6];
    float* __restrict__ dBy = B.f[par ^ 1][7];
    float* __restrict__ dBz = B.f[par ^ 1][8];
    float* __restrict__ Dx = B.d[0];
    float* __restrict__ Dy = B.d[1];
    float* __restrict__ Dz = B.d[2];
    const CT* __restrict__ cls = static_cast<const CT*>(B.cls);
    const float crdx = B.crd_x, crdy = B.crd_y, crdz = B.crd_z;

    // PML membership of this column (x, y) and per plane (z): where D/B are kept
    const bool px = (i < B.pml[0]) || (B.pml[1] > 0 && i >= nx - B.pml[1]);
    const bool py = (j < B.pml[2]) || (B.pml[3] > 0 && j >= ny - B.pml[3]);

    // per-axis coefficients of this column (node n / half node h)
    const int ic = min(max(i, 0), nx), jc = min(max(j, 0), ny);
    const float* __restrict__ cx = B.coef[0];
    const float* __restrict__ cy = B.coef[1];
    const float* __restrict__ cz = B.coef[2];
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

    // prologue: Ex, Ey of plane 0 into LDS slot 0
    {
        sEx[0][ty][tx] = ld_or0(sEx_g, i, j, 0, nx, ny, nz, sy, sz);
        sEy[0][ty][tx] = ld_or0(sEy_g, i, j, 0, nx, ny, nz, sy, sz);
        if (tid < TY + 1) {  // extra column a = TX
            sEx[0][tid][TX] = ld_or0(sEx_g, ox + TX, oy + tid, 0, nx, ny, nz, sy, sz);
            sEy[0][tid][TX] = ld_or0(sEy_g, ox + TX, oy + tid, 0, nx, ny, nz, sy, sz);
        } else if (tid < TY + 1 + TX) {  // extra row b = TY
            const int a = tid - (TY + 1);
            sEx[0][TY][a] = ld_or0(sEx_g, ox + a, oy + TY, 0, nx, ny, nz, sy, sz);
            sEy[0][TY][a] = ld_or0(sEy_g, ox + a, oy + TY, 0, nx, ny, nz, sy, sz);
        }
    }
    float hx_prev = 0.0f, hy_prev = 0.0f;
    const int64_t ms = B.max_steps;

    for (int k = 0; k <= nz; ++k) {
        const int cur = k & 1, nxt = cur ^ 1;
        const bool pz = (k < B.pml[4]) || (B.pml[5] > 0 && k >= nz - B.pml[5]);
        const bool nbx = px || py, nby = py || pz, nbz = pz || px;
        const int node = i + j * sy + k * sz;

        // ---- phase A: stage E^n, load own old H/B/D ----
        sEx[nxt][ty][tx] = ld_or0(sEx_g, i, j, k + 1, nx, ny, nz, sy, sz);
        sEy[nxt][ty][tx] = ld_or0(sEy_g, i, j, k + 1, nx, ny, nz, sy, sz);
        sEz[ty][tx] = ld_or0(sEz_g, i, j, k, nx, ny, nz, sy, sz);
        if (tid < TY + 1) {
            const int ii = ox + TX, jj = oy + tid;
            sEx[nxt][tid][TX] = ld_or0(sEx_g, ii, jj, k + 1, nx, ny, nz, sy, sz);
            sEy[nxt][tid][TX] = ld_or0(sEy_g, ii, jj, k + 1, nx, ny, nz, sy, sz);
            sEz[tid][TX] = ld_or0(sEz_g, ii, jj, k, nx, ny, nz, sy, sz);
        } else if (tid < TY + 1 + TX) {
            const int a = tid - (TY + 1);
            const int ii = ox + a, jj = oy + TY;
            sEx[nxt][TY][a] = ld_or0(sEx_g, ii, jj, k + 1, nx, ny, nz, sy, sz);
            sEy[nxt][TY][a] = ld_or0(sEy_g, ii, jj, k + 1, nx, ny, nz, sy, sz);
            sEz[TY][a] = ld_or0(sEz_g, ii, jj, k, nx, ny, nz, sy, sz);
        }
        float hxo = 0.f, hyo = 0.f, hzo = 0.f, bxo = 0.f, byo = 0.f, bzo = 0.f;
        float dxo = 0.f, dyo = 0.f, dzo = 0.f;
        uint32_t c = 0;
        if (col_ok) {
            hxo = hxo_g[node];
            hyo = hyo_g[node];
            hzo = hzo_g[node];
            if (nbx) bxo = bxo_g[node];
            if (nby) byo = byo_g[node];
            if (nbz) bzo = bzo_g[node];
            if (own) {
                c = cls[node];
                if (nbx) dxo = Dx[node];
                if (nby) dyo = Dy[node];
                if (nbz) dzo = Dz[node];
            }
        }
        // z coefficients of this plane (uniform over the block)
        const float* czk = cz + k;
        const float z_cam1_n = czk[(kCam1 * 2 + 0) * nz1], z_ca_n = czk[(kCa * 2 + 0) * nz1],
                    z_rp_n = czk[(kRp * 2 + 0) * nz1], z_ph_n = czk[(kPh * 2 + 0) * nz1],
                    z_q_n = czk[(kQ * 2 + 0) * nz1];
        const float z_cam1_h = czk[(kCam1 * 2 + 1) * nz1], z_ca_h = czk[(kCa * 2 + 1) * nz1],
                    z_rp_h = czk[(kRp * 2 + 1) * nz1], z_ph_h = czk[(kPh * 2 + 1) * nz1],
                    z_q_h = czk[(kQ * 2 + 1) * nz1];
        __syncthreads();

        // ---- phase C: B then H of plane k (own + halo columns) ----
        float hxn = 0.f, hyn = 0.f, hzn = 0.f;
        const float exo = sEx[cur][ty][tx], eyo = sEy[cur][ty][tx], ezo = sEz[ty][tx];
        if (col_ok) {
            // Hx(i, j+1/2, k+1/2): Bx uses y at j+1/2; Hx uses z at k+1/2, x at i
            const float cxe = (sEz[ty + 1][tx] - ezo) * crdy - (sEy[nxt][ty][tx] - eyo) * crdz;
            const float dbx = fmaf(y_cam1_h, bxo, -y_rp_h * cxe);
            const float bxn = bxo + dbx;
            hxn = fmaf(z_ca_h, hxo, z_rp_h * fmaf(x_ph_n, dbx, x_q_n * bxo));
            // Hy(i+1/2, j, k+1/2): By uses z at k+1/2; Hy uses x at i+1/2, y at j
            const float cye = (sEx[nxt][ty][tx] - exo) * crdz - (sEz[ty][tx + 1] - ezo) * crdx;
            const float dby = fmaf(z_cam1_h, byo, -z_rp_h * cye);
            const float byn = byo + dby;
            hyn = fmaf(x_ca_h, hyo, x_rp_h * fmaf(y_ph_n, dby, y_q_n * byo));
            // Hz(i+1/2, j+1/2, k): Bz uses x at i+1/2; Hz uses y at j+1/2, z at k
            const float cze = (sEy[cur][ty][tx + 1] - eyo) * crdx - (sEx[cur][ty + 1][tx] - exo) * crdy;
            const float dbz = fmaf(x_cam1_h, bzo, -x_rp_h * cze);
            const float bzn = bzo + dbz;
            hzn = fmaf(y_ca_h, hzo, y_rp_h * fmaf(z_ph_n, dbz, z_q_n * bzo));
            if (own) {
                dHx[node] = hxn;
                dHy[node] = hyn;
                dHz[node] = hzn;
                if (nbx) dBx[node] = bxn;
                if (nby) dBy[node] = byn;
                if (nbz) dBz[node] = bzn;
            }
        }
        sHx[ty][tx] = hxn;
        sHy[ty][tx] = hyn;
        sHz[ty][tx] = hzn;
        __syncthreads();

        // ---- phase F: D then E of plane k (own columns) ----
        if (own) {
            const ClassEntry ce = B.ctab[c];
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
                for (int s = 0; s < B.nsrc; ++s)
                    if (B.src_node[s] == node) js += B.src_j[s * ms + step];
            }
            const float chz = ((hyn - sHy[ty][tx - 1]) * crdx - (hxn - sHx[ty - 1][tx]) * crdy) - js;
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
                for (int p = 0; p < B.nprb; ++p)
                    if (B.prb_node[p] == node) B.prb_series[p * ms + step] = ezn;
            }
            if (!isfinite(exn + eyn + ezn)) *B.bad = 1;
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
