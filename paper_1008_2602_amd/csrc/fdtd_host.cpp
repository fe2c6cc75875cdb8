// Host side of libfdtd: argument checking, set-up arithmetic in FP64 (time step,
// UPML profiles, per-node material classes, source samples), device memory,
// launch sequencing, probe spectra and state I/O.  See include/fdtd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "fdtd.h"
#include "fdtd_internal.h"

namespace fdtd {
// kernels (fdtd_kernels.hip)
int num_shapes();
void shape_at(int s, int* tx, int* ty);
hipError_t launch_field_step(int tile_x, int tile_y, const BoardDev* boards, const TileRef* tiles,
                             int ntiles, int rel, int flip, bool wide, hipStream_t st);
int field_step_occupancy(int tile_x, int tile_y, bool wide);
int num_shapes2();
void shape2_at(int s, int* tx, int* ty);
hipError_t launch_field_step2(int tile_y, const BoardDev* boards, const TileRef* tiles, int ntiles,
                              int rel, int flip, bool wide, bool plane, bool nt, hipStream_t st);
int field_step2_occupancy(int tile_y, bool wide);
hipError_t launch_field_step2_material(int tile_y, int mode, const BoardDev* boards,
                                       const TileRef* tiles, int ntiles, int rel, int flip,
                                       bool wide, bool plane, bool nt, hipStream_t st);
int field_step2_material_occupancy(int tile_y, int mode, bool wide);
hipError_t launch_advance(BoardDev* boards, int nb, const int64_t* n, hipStream_t st);
hipError_t launch_advance_one(int64_t* step, int64_t n, int64_t launches, hipStream_t st);
hipError_t launch_eps_step(const BoardDev* board, int nx, int ny, int nz, int64_t plane_bytes,
                           bool big, int rel, int flip, bool wide, hipStream_t st);
hipError_t launch_plane_fold(const float* ring, int64_t plane_nodes, const double* freqs, int nf,
                             double dt, const int64_t* step, int64_t rel_from, int64_t rel_to,
                             double* tw, double* re, double* im, hipStream_t st);
hipError_t launch_dft(const float* series, int64_t max_steps, const double* freqs, int nf, int np,
                      double dt, int64_t s0, int64_t s1, double* re, double* im, hipStream_t st);
hipError_t launch_dft_back(const float* series, int64_t max_steps, const double* freqs, int nf,
                           int np, double dt, const int64_t* step, int64_t back, double* re,
                           double* im, hipStream_t st);
hipError_t launch_fft(const float* series, int64_t n_samples, int n_fft, double2* a, double2* b,
                      double2** result, hipStream_t st);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t st);
// fdtd_noalloc.hip
hipError_t noalloc_scratch(int device, void** out);
hipError_t launch_fft_split(const double2* x, int nbins, double* out, hipStream_t st);
}  // namespace fdtd

using namespace fdtd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OR_FAIL(expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(FDTD_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                        __FILE__, __LINE__);                                                \
    } while (0)

struct SourceH {
    int i, j, k, wave;
    double J0, t0, sigma;
    double R;   // 0: current source (J0 in A/m^2); > 0: resistive voltage source (J0 = V0)
};

struct VoltageProbeH {
    int first, count;   // Ez probes first .. first+count-1, one per z cell
};

// a class: the E edges' 1/eps_r, the flags and (node passes only) the H faces'
// 1/eps_r and the E edges' conduction coefficients
struct ClassKey {
    uint32_t a, b, c, f, hx, hy, hz, lx, ly, lz;
    bool operator==(const ClassKey& o) const
    {
        return a == o.a && b == o.b && c == o.c && f == o.f && hx == o.hx && hy == o.hy &&
               hz == o.hz && lx == o.lx && ly == o.ly && lz == o.lz;
    }
};
struct ClassKeyHash {
    size_t operator()(const ClassKey& k) const
    {
        uint64_t h = 1469598103934665603ull;
        for (uint32_t v : {k.a, k.b, k.c, k.f, k.hx, k.hy, k.hz, k.lx, k.ly, k.lz}) {
            h ^= v;
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};

uint32_t fbits(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    return u;
}

}  // namespace

struct fdtd_grid {
    fdtd_grid_desc d{};
    double dt = 0.0;
    int64_t nodes = 0;      // (nx+1)(ny+1)(nz+1) grid nodes
    int64_t pitch = 0;      // device row pitch in nodes: nx+1 rounded up to 32
    int64_t dnodes = 0;     // device nodes per field array: pitch (ny+1)(nz+1)
    int64_t cstride = 0;    // bytes between the x, y, z arrays of one field
    bool big = false;       // 3 cstride beyond 32-bit offsets: the node passes with per-component bases
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    std::vector<void*> allocs;
    int64_t device_bytes = 0;

    // device state
    float* f[2][9] = {};
    float* dd[2][3] = {};
    float* coef[3] = {};
    void* cls = nullptr;
    ClassEntry* ctab = nullptr;
    float* node_aux = nullptr;
    int32_t* src_node = nullptr;
    int64_t* src_node64 = nullptr;
    int64_t* prb_node64 = nullptr;
    float* src_j = nullptr;
    float* src_beta = nullptr;
    int32_t* prb_node = nullptr;
    float* prb_series = nullptr;
    double* dft_f = nullptr;
    double* dft_re = nullptr;
    double* dft_im = nullptr;
    float* plane_ring = nullptr;    // kPlaneRing slots of one padded plane
    double* plane_f = nullptr;
    double* plane_tw = nullptr;     // [nf][kPlaneRing] (cos, -sin) * dt of one fold
    double* plane_re = nullptr;     // [nf][ny+1][pitch]
    double* plane_im = nullptr;
    int64_t* step_dev = nullptr;
    int32_t* bad_dev = nullptr;
    BoardDev* board_dev = nullptr;
    TileRef* tiles_dev = nullptr;   // work list of the current tile shape
    int ntiles = 0;
    TileRef* tiles1_dev = nullptr;  // one-step list for the odd step of a two-step shape
    int ntiles1 = 0;
    int tiles1_cap = 0;
    // material boards: planes whose nodes need the material arithmetic (a
    // conducting edge, or a PML node with a scaled 1/eps_rw), the tiles of the
    // plain kernel's grid that hold such nodes per plane, and the list of plain
    // two-step pieces (64 x kHybridTY x 2) clear of them, which the plain kernel
    // steps with the same bits
    std::vector<uint8_t> mat_plane;
    std::vector<uint8_t> tile_need;  // per tile of the hybrid grid and node plane
    TileRef* tilesP_dev = nullptr;
    int ntilesP = 0;
    int tilesP_cap = 0;
    // the same pieces on the host (board index 0), for batched calls
    std::vector<TileRef> pc_plain, pc_cd, pc_rb;
    TileRef* tilesC_dev = nullptr;  // pieces of the conduction-only flavour (64 x kHybridTY x 2)
    int ntilesC = 0;
    int tilesC_cap = 0;
    int cond_permille = 0;          // share of tile planes on the conduction-only flavour
    int mat_permille = 0;           // share of tile planes on the material variant
    int mat_ty = kHybridTY;         // the material variant's tile rows (kHybridTY or kMatTY)
    int mat_split = 0;              // 1: per tile, 2: per plane
    // the material variant's launch runs beside the plain one on a second stream
    // (forked from and joined to the handle's stream by events), so that each
    // fills the other's last partial round
    hipStream_t aux_stream = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    int buf = 0;                    // field buffer (0/1) holding the current step
    int tiles_cap = 0;
    BoardDev board_host{};

    // host-side set-up
    std::vector<float> eps;
    std::vector<float> sigma;       // conductivity per cell (S/m), empty: lossless
    std::vector<uint8_t> pec;
    bool have_materials = false;
    std::vector<SourceH> sources;
    std::vector<std::array<int, 3>> probes;
    std::vector<VoltageProbeH> vprobes;
    std::vector<double> freqs;
    int plane_k = -1;               // plane-DFT node plane, -1: none
    bool pml_eps_rw = false;        // Eq. 2's eps_rw requested
    double sheet_R = 0.0;           // > 0: PEC Ex/Ey edges are resistive sheets (ohm per square)
    bool node_pass = false;         // steps run the node passes' arithmetic (eps_rw in a dielectric PML, or loss)
    bool mat = false;               // of which pairs of steps on the material two-step kernel
    std::vector<double> plane_freqs;
    int n_classes = 0;
    bool wide = false;
    bool finalized = false;
    int64_t step = 0;
    int tile_x = 64, tile_y = 14, tile_steps = 2;
    int cus = 0;            // compute units of the device
    int64_t step_bytes = 0;

    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    int64_t timed_launches = 0;

    // graph of kGraphChunk steps (field launches + counter advance), replayed by step_n
    hipGraphExec_t graph_exec = nullptr;
    bool graph_failed = false;
    hipEvent_t sync_ev = nullptr;

    // batched calls led by this handle: their plans (tables in device memory and
    // a captured graph), most recently used kept
    uint64_t serial = 0;            // unique per handle created in this process
    std::vector<struct BatchPlan*> plans;
    std::vector<struct BatchPlan*> retired;   // evicted, freed once their last launch is done
    uint64_t plan_clock = 0;
};

namespace {

void* dev_alloc(fdtd_grid* g, size_t bytes)
{
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (g->d.dev_alloc) {
        p = g->d.dev_alloc(bytes, g->d.alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        g->allocs.push_back(p);
        g->device_bytes += (int64_t)bytes;
    }
    return p;
}

void* temp_alloc(fdtd_grid* g, size_t bytes)
{
    bytes = (bytes + 255) & ~size_t(255);
    if (g->d.dev_alloc) return g->d.dev_alloc(bytes, g->d.alloc_ctx);
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void temp_free(fdtd_grid* g, void* p)
{
    if (!p) return;
    if (g->d.dev_free)
        g->d.dev_free(p, g->d.alloc_ctx);
    else
        (void)hipFree(p);
}

// Stream-ordered copy that has completed when it returns (the handle's stream
// may be a non-blocking one, which the legacy null stream does not order with).
hipError_t copy_sync(fdtd_grid* g, void* dst, const void* src, size_t bytes, hipMemcpyKind kind)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, g->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(g->stream);
}

// Copy one field array between the packed host layout ((nx+1) nodes per row)
// and the padded device layout (pitch nodes per row): one contiguous copy of
// the padded array through a host staging buffer (the padding columns hold
// zeros), repacked row by row on the host, with every value multiplied by
// `scale` on the way.
hipError_t copy_field_sync(fdtd_grid* g, void* dst, const void* src, hipMemcpyKind kind,
                           float scale = 1.0f)
{
    const size_t nrow = (size_t)g->d.nx + 1, pitch = (size_t)g->pitch;
    const size_t rows = (size_t)(g->d.ny + 1) * (g->d.nz + 1);
    std::vector<float> stage(rows * pitch, 0.0f);
    if (kind == hipMemcpyHostToDevice) {
        const float* in = (const float*)src;
        for (size_t r = 0; r < rows; ++r) {
            float* o = stage.data() + r * pitch;
            const float* x = in + r * nrow;
            if (scale == 1.0f)
                memcpy(o, x, nrow * 4);
            else
                for (size_t i = 0; i < nrow; ++i) o[i] = x[i] * scale;
        }
        hipError_t e = hipMemcpyAsync(dst, stage.data(), stage.size() * 4, kind, g->stream);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(g->stream);
    }
    hipError_t e = hipMemcpyAsync(stage.data(), src, stage.size() * 4, kind, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return e;
    float* out = (float*)dst;
    for (size_t r = 0; r < rows; ++r) {
        const float* x = stage.data() + r * pitch;
        float* o = out + r * nrow;
        if (scale == 1.0f)
            memcpy(o, x, nrow * 4);
        else
            for (size_t i = 0; i < nrow; ++i) o[i] = x[i] * scale;
    }
    return hipSuccess;
}

int64_t row_pitch(int nx) { return ((int64_t)nx + 1 + 31) / 32 * 32; }

// Bytes between the x, y and z arrays of one field (padded nodes + guard words,
// rounded up to 256 bytes).
int64_t component_stride(int64_t dnodes) { return ((dnodes + kGuard) * 4 + 255) / 256 * 256; }

// Owned rows of a tile: the one-step kernel spends one row of its TY on the halo,
// the two-step kernel three.
int owned_rows(int ty, int steps) { return steps == 2 ? ty - 3 : ty - 1; }

// The one-step shape that takes the odd step of a two-step shape.
constexpr int kOddX = 64, kOddY = 15;

// Tiles of a shape: tx aligned columns and `rows` owned rows each.  The tiles
// cover node columns 0..nx-1 and rows 0..ny-1 (and the kernels step planes
// 0..nz-1): a node on the far wall (i = nx, j = ny or k = nz) carries only
// components that are tangential E on the wall (held at zero), H normal to the
// wall (which touches nothing but such E, so it stays zero) or components that
// do not exist, so nothing there is ever stepped.
void tile_counts(int nx, int ny, int tx, int rows, int* cx, int* cy)
{
    *cx = (nx + tx - 1) / tx;
    *cy = (ny + rows - 1) / rows;
}

// One launch of the field kernel of a shape (one or two steps per pass); plane:
// some board of the launch keeps a plane DFT; nt: the two-step kernel stores the
// fields with non-temporal stores (stream_stores).
hipError_t launch_pass(int tx, int ty, int steps, const BoardDev* boards, const TileRef* tiles,
                       int ntiles, int rel, int flip, bool wide, bool plane, bool nt, hipStream_t st)
{
    if (steps == 2)
        return launch_field_step2(ty, boards, tiles, ntiles, rel, flip, wide, plane, nt, st);
    return launch_field_step(tx, ty, boards, tiles, ntiles, rel, flip, wide, st);
}

// Whether the two-step kernels of a launch over these boards store their fields
// with non-temporal stores.  A launch reads every field once and writes the
// other copy once, so when the fields far outgrow the caches (32 MB of L2, the
// 256 MB Infinity Cache) ordinary stores only push out lines that the launch
// is still reading, which non-temporal stores keep (the large board: 0.618 ->
// 0.597 ms per step); boards whose fields fit in the Infinity Cache find
// them there at the next launch with ordinary stores (the z-convergence batch,
// about 100 MB: 7 % slower with non-temporal stores).  The measure is the
// library's fused step count (one read and one write of every kept array).
constexpr int64_t kStreamStoreBytes = 192ll << 20;
bool stream_stores(const fdtd_grid* const* gs, int ng)
{
    int64_t b = 0;
    for (int h = 0; h < ng; ++h) b += gs[h]->step_bytes;
    return b > kStreamStoreBytes;
}

constexpr int kXcds = 8;   // the kernel deals block b to XCD b % 8 (xcd_tile)

// Work list of one field launch.  Tiles arrive in board order, row-major within
// a board.  They are cut into kXcds contiguous runs of about equal plane count,
// one per XCD, so that neighbouring tiles share halos in that XCD's L2.  On each
// XCD the tiles left over after its last full round of concurrent blocks would
// leave most of the XCD idle in that round; they are split in z into S pieces
// (S chosen to shorten the estimated tail, each piece after the first pays one
// recomputed plane).  Pieces go piece-major so that concurrent pieces are
// spatial neighbours at the same depth.  Every run is padded with idle entries
// to the common length, so the launch has kXcds * length blocks.
void build_work(const std::vector<TileRef>& tiles, int slots_per_xcd, std::vector<TileRef>& out)
{
    out.clear();
    const size_t T = tiles.size();
    if (T == 0) return;
    double W = 0.0;
    for (const TileRef& t : tiles) W += t.ke - t.kb;
    std::vector<std::vector<TileRef>> runs(kXcds);
    size_t idx = 0;
    double acc = 0.0;
    for (int x = 0; x < kXcds; ++x) {
        const double target = W * (x + 1) / kXcds;
        std::vector<TileRef> whole;
        while (idx < T && (x == kXcds - 1 || acc + 0.5 * (tiles[idx].ke - tiles[idx].kb) <= target)) {
            whole.push_back(tiles[idx]);
            acc += tiles[idx].ke - tiles[idx].kb;
            ++idx;
        }
        const size_t n = whole.size(), C = (size_t)std::max(1, slots_per_xcd);
        const size_t m = n % C;  // tiles of the partial last round
        int S = 1;
        if (m > 0) {
            double pbar = 0.0;
            for (size_t q = n - m; q < n; ++q) pbar += whole[q].ke - whole[q].kb;
            pbar /= (double)m;
            double best = pbar;
            // up to 16 pieces of at least two planes: small boards (a few tiles,
            // 30-plane columns) are latency bound, and shorter pieces cut the
            // planes each block walks in sequence
            for (int cand = 2; cand <= 16 && pbar / cand >= 2.0; ++cand) {
                const double rounds = std::ceil((double)(m * cand) / (double)C);
                const double cost = rounds * (pbar / cand + 1.0);
                if (cost < 0.97 * best) {
                    best = cost;
                    S = cand;
                }
            }
        }
        std::vector<TileRef>& r = runs[x];
        r.assign(whole.begin(), whole.end() - (S > 1 ? (std::ptrdiff_t)m : 0));
        if (S > 1)
            for (int piece = 0; piece < S; ++piece)
                for (size_t q = n - m; q < n; ++q) {
                    TileRef t = whole[q];
                    const int planes = t.ke - t.kb;
                    t.ke = t.kb + (int)((int64_t)planes * (piece + 1) / S);
                    t.kb = t.kb + (int)((int64_t)planes * piece / S);
                    if (t.kb < t.ke) r.push_back(t);   // a shallow tile may give fewer pieces
                }
    }
    size_t L = 0;
    for (const auto& r : runs) L = std::max(L, r.size());
    out.reserve(L * kXcds);
    for (const auto& r : runs) {
        out.insert(out.end(), r.begin(), r.end());
        out.insert(out.end(), L - r.size(), TileRef{-1, 0, 0, 0, 0});
    }
}

// Whole tiles of board b (row-major), planes 0..nz-1.
void board_tiles(int b, int nx, int ny, int nz, int tx, int rows, std::vector<TileRef>& out)
{
    int cx, cy;
    tile_counts(nx, ny, tx, rows, &cx, &cy);
    for (int y = 0; y < cy; ++y)
        for (int x = 0; x < cx; ++x) out.push_back(TileRef{b, x, y, 0, nz});
}

// mode: 0 the plain kernels, 1 the material variant, 2 its conduction-only flavour
int slots_per_xcd(const fdtd_grid* g, int tx, int ty, int steps, bool wide, int mode)
{
    const int occ = steps == 2 ? (mode ? field_step2_material_occupancy(ty, mode, wide)
                                      : field_step2_occupancy(ty, wide))
                               : field_step_occupancy(tx, ty, wide);
    return std::max(1, g->cus / kXcds) * occ;
}

void dev_free_all(fdtd_grid* g)
{
    for (void* p : g->allocs) {
        if (g->d.dev_free)
            g->d.dev_free(p, g->d.alloc_ctx);
        else
            (void)hipFree(p);
    }
    g->allocs.clear();
}

// Eq. 5 grading at coordinate pos (cell units) on an axis of n cells with PML
// depths nlo/nhi: depth from the PML interface towards the outer wall.
void profile(const fdtd_grid_desc& d, double pos, int n, int nlo, int nhi, double delta,
             double* sigma, double* kappa)
{
    double depth = 0.0, N = 0.0;
    if (nlo > 0 && pos < nlo) {
        depth = nlo - pos;
        N = nlo;
    } else if (nhi > 0 && pos > n - nhi) {
        depth = pos - (n - nhi);
        N = nhi;
    }
    if (depth <= 0.0) {
        *sigma = 0.0;
        *kappa = 1.0;
        return;
    }
    depth = std::min(depth, N);  // half nodes past the wall only feed components that stay 0
    const double fr = std::pow(depth / N, d.pml_m);
    const double smax = -(d.pml_m + 1.0) * std::log(d.pml_R) / (2.0 * kEta0 * N * delta);
    *sigma = fr * smax;
    *kappa = 1.0 + (d.pml_kappa_max - 1.0) * fr;
}

std::vector<float> coef_table(const fdtd_grid_desc& d, int axis, double dt)
{
    const int n = axis == 0 ? d.nx : axis == 1 ? d.ny : d.nz;
    const double delta = axis == 0 ? d.dx : axis == 1 ? d.dy : d.dz;
    const int nlo = d.npml[2 * axis], nhi = d.npml[2 * axis + 1];
    std::vector<float> t((size_t)kNumCoef * 2 * (n + 1));
    for (int half = 0; half < 2; ++half)
        for (int i = 0; i <= n; ++i) {
            double s, k;
            profile(d, i + 0.5 * half, n, nlo, nhi, delta, &s, &k);
            const double q = s * dt / kEps0;
            const double ph = k + 0.5 * q;
            const double v[kNumCoef] = {-q / ph, (k - 0.5 * q) / ph, 1.0 / ph, ph, q, k};
            for (int c = 0; c < kNumCoef; ++c)
                t[((size_t)c * 2 + half) * (n + 1) + i] = (float)v[c];
        }
    return t;
}

// A material board's table: the coefficients as the material kernels rebuild
// them from the FP32 q and kappa at 1/eps_rw = 1, in the same FP32 operations
// (one rounding each: fmaf, a correctly rounded division, products), so that a
// node whose material leaves its coefficients unscaled can read them instead.
void material_coefs(std::vector<float>& t, int n1)
{
    for (int half = 0; half < 2; ++half)
        for (int i = 0; i < n1; ++i) {
            auto at = [&](int c) -> float& { return t[((size_t)c * 2 + half) * n1 + i]; };
            const float q = at(kQ), k = at(kKappa);
            const float ph = std::fmaf(0.5f, q, k);
            const float rp = 1.0f / ph;
            at(kPh) = ph;
            at(kRp) = rp;
            at(kCa) = std::fmaf(-0.5f, q, k) * rp;
            at(kCam1) = -q * rp;
        }
}

double waveform(const SourceH& s, double t)
{
    const double u = (t - s.t0) / s.sigma;
    if (s.wave == FDTD_WAVE_DGAUSS) return s.J0 * u * std::exp(-u * u);
    return s.J0 * std::exp(-0.5 * u * u);
}

int check_grid(fdtd_grid* g)
{
    if (!g) return fail(FDTD_EINVAL, "null grid handle");
    return FDTD_OK;
}

// index into the packed host arrays (PEC mask, field images)
int64_t node_index(const fdtd_grid* g, int i, int j, int k)
{
    return (int64_t)i + (int64_t)(g->d.nx + 1) * ((int64_t)j + (int64_t)(g->d.ny + 1) * k);
}

// index into the padded device arrays
int64_t dev_index(const fdtd_grid* g, int i, int j, int k)
{
    return (int64_t)i + g->pitch * ((int64_t)j + (int64_t)(g->d.ny + 1) * k);
}

// Count the bytes one field step must move with this layout: E and H read and
// written once per stepped node (i < nx, j < ny, k < nz: one per cell), the
// class byte(s) once, and each stored D/B component read and written once where
// its PML predicate holds.
// Marks, for one node plane, every tile of the 64 x kHybridTY x 2 grid whose
// footprint holds a node with need bit `bit` (need: one byte per node of the
// plane, x fastest): out[tile * stride] |= bit, tiles row-major.  A tile's
// footprint is the nodes its block computes or reads: columns i0-2 .. i0+65,
// rows j0-2 .. j0+kHybridTY-1.  2-D prefix sums of the plane's marks (pre is
// scratch) make each tile one lookup.
void mark_tile_need(const uint8_t* need, int nx, int ny, uint8_t bit, std::vector<int32_t>& pre,
                    uint8_t* out, size_t stride)
{
    int hcx = 0, hcy = 0;
    tile_counts(nx, ny, 64, owned_rows(kHybridTY, 2), &hcx, &hcy);
    const int px = nx + 2;
    // row 0 and column 0 stay zero; every other entry is written below
    if (pre.size() != (size_t)(nx + 2) * (ny + 2)) pre.assign((size_t)(nx + 2) * (ny + 2), 0);
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i)
            pre[(size_t)(j + 1) * px + i + 1] = ((need[(size_t)j * (nx + 1) + i] & bit) ? 1 : 0) +
                                                pre[(size_t)j * px + i + 1] + pre[(size_t)(j + 1) * px + i] -
                                                pre[(size_t)j * px + i];
    for (int y = 0; y < hcy; ++y)
        for (int x = 0; x < hcx; ++x) {
            const int j0 = y * owned_rows(kHybridTY, 2), i0 = 64 * x;
            const int ja = std::max(0, j0 - 2), jb = std::min(ny, j0 + kHybridTY - 1);
            const int ia = std::max(0, i0 - 2), ib = std::min(nx, i0 + 65);
            const int64_t sum = (int64_t)pre[(size_t)(jb + 1) * px + ib + 1] - pre[(size_t)ja * px + ib + 1] -
                                pre[(size_t)(jb + 1) * px + ia] + pre[(size_t)ja * px + ia];
            if (sum > 0) out[((size_t)y * hcx + x) * stride] |= bit;
        }
}

// How a material board's pairs of steps are split between the plain two-step
// kernel and the material variants.
struct MaterialSplit {
    std::vector<TileRef> rb, cd, plain;   // material variant, conduction-only flavour, plain kernel
    int mat_ty = kHybridTY;               // the material variant's tile rows
    int split = 0;                        // 0 none, 1 per tile, 2 per plane
    int mat_permille = 0, cond_permille = 0;
};

// The split of a board of nx x ny x nz cells from tile_need (per tile of the
// 64 x kHybridTY x 2 grid and node plane, bits 1 rebuilt coefficients, 2
// conduction; empty: none).  A piece [kb, ke) of a tile computes first-step H
// and E on planes kb-2 .. ke, so its plane k needs the kind of node found in
// the footprint on planes k-2 .. k+1.  Planes near PML nodes whose
// coefficients are rebuilt run the material variant; the others near
// conducting edges its conduction-only flavour (which fits the hybrid shape
// without spilling); the rest the plain kernel.  Runs of one kind in a tile
// are one piece.  The material variant's planes are split one of two ways, the
// cheaper by the measured cost of a tile plane on each kernel (large board, per
// step: plain 64 x 14 0.615 ms, material 64 x 14 1.00 ms, material 64 x 10
// 0.82 ms):
//  * per tile: each tile's planes near such nodes on the variant in the plain
//    kernel's tiles (where it spills), best when few tiles hold them (a board
//    running into the PML with eps_rw);
//  * per plane: planes near such nodes in any tile on the 64 x kMatTY variant
//    for every tile, best when such nodes fill those planes.
void split_material(int nx, int ny, int nz, const std::vector<uint8_t>& tile_need, MaterialSplit& out)
{
    out = MaterialSplit();
    int cx, cy;
    tile_counts(nx, ny, 64, owned_rows(kHybridTY, 2), &cx, &cy);
    std::vector<uint8_t> kind((size_t)cx * cy * nz, 0), anyR((size_t)nz, 0);
    int64_t rb_tp = 0;
    for (size_t t = 0; t < (size_t)cx * cy; ++t) {
        const uint8_t* tn = tile_need.empty() ? nullptr : &tile_need[t * (nz + 1)];
        for (int k = 0; k < nz && tn; ++k) {
            uint8_t m = 0;
            for (int q = std::max(0, k - 2); q <= std::min(nz, k + 1); ++q) m |= tn[q];
            const uint8_t kd = (m & 1) ? 1 : (m & 2) ? 2 : 0;   // 1 material, 2 conduction
            kind[t * nz + k] = kd;
            rb_tp += kd == 1;
            anyR[k] |= kd == 1;
        }
    }
    const double all = std::max<double>(1.0, (double)cx * cy * nz);
    int64_t any_planes = 0;
    for (int k = 0; k < nz; ++k) any_planes += anyR[k];
    const double f_tile = rb_tp / all, f_plane = any_planes / (double)nz;
    const double cost_tile = (1.0 - f_tile) * 0.615 + f_tile * 1.00;
    const double cost_plane = (1.0 - f_plane) * 0.615 + f_plane * 0.82;
    const bool per_plane = any_planes > 0 && cost_plane < cost_tile;
    out.mat_ty = per_plane ? kMatTY : kHybridTY;
    out.split = any_planes == 0 ? 0 : per_plane ? 2 : 1;
    // pieces: runs of one kind in each tile (per plane: the material planes
    // leave the tiles and go to 64 x kMatTY tiles over the whole board)
    int64_t cd_tp = 0, rb_planes = 0;
    for (int y = 0; y < cy; ++y)
        for (int x = 0; x < cx; ++x) {
            const uint8_t* kd = &kind[((size_t)y * cx + x) * nz];
            auto k_of = [&](int k) -> int { return per_plane && anyR[k] ? 3 : kd[k]; };
            for (int k = 0; k < nz;) {
                const int c = k_of(k);
                int e = k;
                while (e < nz && k_of(e) == c) ++e;
                if (c == 1) {
                    out.rb.push_back(TileRef{0, x, y, k, e});
                    rb_planes += e - k;
                } else if (c == 2) {
                    out.cd.push_back(TileRef{0, x, y, k, e});
                    cd_tp += e - k;
                } else if (c == 0) {
                    out.plain.push_back(TileRef{0, x, y, k, e});
                }
                k = e;
            }
        }
    if (per_plane) {
        std::vector<TileRef> mt;
        board_tiles(0, nx, ny, nz, 64, owned_rows(kMatTY, 2), mt);
        for (int k = 0; k < nz;) {
            int e = k;
            while (e < nz && anyR[e] == anyR[k]) ++e;
            if (anyR[k])
                for (TileRef t : mt) {
                    t.kb = k;
                    t.ke = e;
                    out.rb.push_back(t);
                }
            k = e;
        }
        rb_planes = (int64_t)(f_plane * all + 0.5);
    }
    out.mat_permille = (int)(1000.0 * rb_planes / all);
    out.cond_permille = (int)(1000.0 * cd_tp / all);
}

int64_t count_step_bytes(const fdtd_grid* g)
{
    const fdtd_grid_desc& d = g->d;
    auto in_pml = [](int idx, int n, int lo, int hi) {
        return idx < lo || (hi > 0 && idx >= n - hi);
    };
    int64_t px = 0, py = 0, pz = 0;
    for (int i = 0; i < d.nx; ++i) px += in_pml(i, d.nx, d.npml[0], d.npml[1]);
    for (int j = 0; j < d.ny; ++j) py += in_pml(j, d.ny, d.npml[2], d.npml[3]);
    for (int k = 0; k < d.nz; ++k) pz += in_pml(k, d.nz, d.npml[4], d.npml[5]);
    const int64_t X = d.nx, Y = d.ny, Z = d.nz;
    // nodes where (a or b) holds, a/b independent predicates on two axes
    auto either = [](int64_t pa, int64_t na, int64_t pb, int64_t nb, int64_t other) {
        return (pa * nb + na * pb - pa * pb) * other;
    };
    const int64_t aux_x = either(px, X, py, Y, Z);  // Dx, Bx: x or y PML
    const int64_t aux_y = either(py, Y, pz, Z, X);  // Dy, By: y or z PML
    const int64_t aux_z = either(pz, Z, px, X, Y);  // Dz, Bz: z or x PML
    const int64_t cls_bytes = g->wide ? 2 : 1;
    return X * Y * Z * (24 + 24 + cls_bytes) + (aux_x + aux_y + aux_z) * 2 * 8;
}

}  // namespace
static int upload_tiles(fdtd_grid* g);
namespace {

int finalize(fdtd_grid* g)
{
    if (g->finalized) return FDTD_OK;
    const fdtd_grid_desc& d = g->d;
    if (!g->have_materials) return fail(FDTD_ESTATE, "fdtd_set_materials was never called");
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int64_t N = g->nodes, ND = g->dnodes;
    // sources and probes
    for (const SourceH& s : g->sources) {
        if (g->pec[node_index(g, s.i, s.j, s.k)] & 4)
            return fail(FDTD_EINVAL, "source at (%d,%d,%d) sits on a PEC edge", s.i, s.j, s.k);
    }
    std::vector<int32_t> src_node, prb_node;
    std::vector<int64_t> src_node64, prb_node64;
    for (const SourceH& s : g->sources) {
        src_node64.push_back(dev_index(g, s.i, s.j, s.k));
        src_node.push_back((int32_t)src_node64.back());   // tiled kernels: boards within 2^31 nodes
    }
    for (const auto& p : g->probes) {
        prb_node64.push_back(dev_index(g, p[0], p[1], p[2]));
        prb_node.push_back((int32_t)prb_node64.back());
    }
    std::vector<uint8_t> is_src(0), is_prb(0);

    // per-node classes: edge permittivity (mean of the touching cells), stepped
    // components (not on the outer wall, not PEC), source/probe marks
    std::unordered_map<ClassKey, uint32_t, ClassKeyHash> map;
    std::vector<ClassEntry> table;
    // padding columns keep class 0 and are never read; kGuard class-0 entries past
    // the last node serve the kernel's reads for absent nodes
    const int64_t NC = ND + kGuard;
    std::vector<uint16_t> ids((size_t)NC, 0);
    std::vector<uint8_t> mark((size_t)N, 0);
    for (const SourceH& s : g->sources) mark[node_index(g, s.i, s.j, s.k)] |= 1;
    for (const auto& p : g->probes) mark[node_index(g, p[0], p[1], p[2])] |= 2;
    const float* er = g->eps.data();
    auto cell = [&](int i, int j, int k) -> double {
        return (double)er[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)];
    };
    ClassKey last{~0u, ~0u, ~0u, ~0u, ~0u, ~0u, ~0u, ~0u, ~0u, ~0u};
    uint32_t last_id = 0;
    // node passes: 1/eps_r at the H faces of each class (two cells share a face;
    // one on the outer wall) and the edges' conduction, and whether any PML
    // location has eps_r != 1 (with eps_rw) or any edge conducts
    std::vector<float> node_aux;
    const bool lossy = !g->sigma.empty();
    auto sig = [&](int i, int j, int k) -> double {
        return (double)g->sigma[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)];
    };
    const double lscale = g->dt / (2.0 * kEps0);   // sigma_c -> sigma_c dt / (2 eps0)
    auto in_slab = [](int idx, int n, int lo, int hi) { return idx < lo || (hi > 0 && idx >= n - hi); };
    // resistive sheets: a PEC-marked Ex/Ey edge carries the sheet current
    // Ebar / R_s within its dual cell of height dz, a conductivity 1 / (R_s dz)
    const bool sheets = g->sheet_R > 0.0;
    const double g_sheet = sheets ? 1.0 / (g->sheet_R * d.dz) : 0.0;
    auto pml_cell = [&](int i, int j, int k) {
        return in_slab(i, nx, d.npml[0], d.npml[1]) || in_slab(j, ny, d.npml[2], d.npml[3]) ||
               in_slab(k, nz, d.npml[4], d.npml[5]);
    };
    g->node_pass = g->big;
    // material boards: the nodes that need the material arithmetic, one node
    // plane at a time; every tile of the hybrid grid (64 x kHybridTY x 2) whose
    // footprint holds one is marked for that plane
    std::vector<uint8_t> mat_plane((size_t)nz + 1, 0), need((size_t)(nx + 1) * (ny + 1), 0);
    int hcx = 0, hcy = 0;
    tile_counts(nx, ny, 64, owned_rows(kHybridTY, 2), &hcx, &hcy);
    std::vector<uint8_t> tile_need;
    std::vector<int32_t> pre;
    for (int k = 0; k <= nz; ++k) {
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                const int64_t n = node_index(g, i, j, k);
                const uint8_t pm = g->pec[n];
                const bool shx = sheets && (pm & 1), shy = sheets && (pm & 2);
                uint32_t fl = 0;
                float ix = 0.f, iy = 0.f, iz = 0.f;
                if (i < nx && j >= 1 && j < ny && k >= 1 && k < nz && (!(pm & 1) || shx)) {
                    if (shx && (pml_cell(i, j - 1, k - 1) || pml_cell(i, j, k - 1) ||
                                pml_cell(i, j - 1, k) || pml_cell(i, j, k)))
                        return fail(FDTD_EINVAL,
                                    "resistive sheet edge Ex(%d,%d,%d) touches a PML cell", i, j, k);
                    fl |= kUpdEx;
                    ix = (float)(4.0 / (cell(i, j - 1, k - 1) + cell(i, j, k - 1) +
                                        cell(i, j - 1, k) + cell(i, j, k)));
                }
                if (i >= 1 && i < nx && j < ny && k >= 1 && k < nz && (!(pm & 2) || shy)) {
                    if (shy && (pml_cell(i - 1, j, k - 1) || pml_cell(i, j, k - 1) ||
                                pml_cell(i - 1, j, k) || pml_cell(i, j, k)))
                        return fail(FDTD_EINVAL,
                                    "resistive sheet edge Ey(%d,%d,%d) touches a PML cell", i, j, k);
                    fl |= kUpdEy;
                    iy = (float)(4.0 / (cell(i - 1, j, k - 1) + cell(i, j, k - 1) +
                                        cell(i - 1, j, k) + cell(i, j, k)));
                }
                if (i >= 1 && i < nx && j >= 1 && j < ny && k < nz && !(pm & 4)) {
                    fl |= kUpdEz;
                    iz = (float)(4.0 / (cell(i - 1, j - 1, k) + cell(i, j - 1, k) +
                                        cell(i - 1, j, k) + cell(i, j, k)));
                }
                if (mark[n] & 1) fl |= kSrcEz;
                if (mark[n] & 2) fl |= kPrbEz;
                if (k == g->plane_k) fl |= kPlnEz;
                float fx = 1.f, fy = 1.f, fz = 1.f;
                if (g->pml_eps_rw) {
                    if (j < ny && k < nz)
                        fx = (float)(2.0 / (cell(i > 0 ? i - 1 : 0, j, k) + cell(i < nx ? i : nx - 1, j, k)));
                    if (i < nx && k < nz)
                        fy = (float)(2.0 / (cell(i, j > 0 ? j - 1 : 0, k) + cell(i, j < ny ? j : ny - 1, k)));
                    if (i < nx && j < ny)
                        fz = (float)(2.0 / (cell(i, j, k > 0 ? k - 1 : 0) + cell(i, j, k < nz ? k : nz - 1)));
                    const bool slab = in_slab(i, nx, d.npml[0], d.npml[1]) ||
                                      in_slab(j, ny, d.npml[2], d.npml[3]) ||
                                      in_slab(k, nz, d.npml[4], d.npml[5]);
                    if (slab && (((fl & kUpdEx) && ix != 1.f) || ((fl & kUpdEy) && iy != 1.f) ||
                                 ((fl & kUpdEz) && iz != 1.f) || fx != 1.f || fy != 1.f || fz != 1.f))
                        g->node_pass = true;
                }
                float lx = 0.f, ly = 0.f, lz = 0.f;
                if (lossy || sheets) {
                    if (fl & kUpdEx)
                        lx = (float)(lscale * ((lossy ? 0.25 * (sig(i, j - 1, k - 1) + sig(i, j, k - 1) +
                                                                sig(i, j - 1, k) + sig(i, j, k))
                                                      : 0.0) +
                                               (shx ? g_sheet : 0.0)));
                    if (fl & kUpdEy)
                        ly = (float)(lscale * ((lossy ? 0.25 * (sig(i - 1, j, k - 1) + sig(i, j, k - 1) +
                                                                sig(i - 1, j, k) + sig(i, j, k))
                                                      : 0.0) +
                                               (shy ? g_sheet : 0.0)));
                    if ((fl & kUpdEz) && lossy)
                        lz = (float)(lscale * 0.25 * (sig(i - 1, j - 1, k) + sig(i, j - 1, k) +
                                                      sig(i - 1, j, k) + sig(i, j, k)));
                    if (lx != 0.f || ly != 0.f || lz != 0.f) {
                        g->node_pass = true;
                        fl |= kCondE;
                    }
                }
                if (fx != 1.f || fy != 1.f || fz != 1.f) fl |= kMatH;
                if (g->pml_eps_rw && (((fl & kUpdEx) && ix != 1.f) || ((fl & kUpdEy) && iy != 1.f) ||
                                      ((fl & kUpdEz) && iz != 1.f)))
                    fl |= kMatE;
                // the material variant rebuilds only PML nodes' coefficients and
                // solves conducting edges; every other node is the plain kernel's
                const bool node_pml = in_slab(i, nx, d.npml[0], d.npml[1]) ||
                                      in_slab(j, ny, d.npml[2], d.npml[3]) ||
                                      in_slab(k, nz, d.npml[4], d.npml[5]);
                // bit 1: coefficients rebuilt (the material variant); bit 2: a
                // conducting edge (its conduction-only flavour will do)
                const uint8_t needs = (uint8_t)((((fl & (kMatH | kMatE)) && node_pml) ? 1 : 0) |
                                                ((fl & kCondE) ? 2 : 0));
                need[(size_t)j * (nx + 1) + i] = needs;
                mat_plane[k] |= needs;
                const ClassKey key{fbits(ix), fbits(iy), fbits(iz), fl, fbits(fx), fbits(fy), fbits(fz),
                                   fbits(lx), fbits(ly), fbits(lz)};
                uint32_t id;
                if (key == last) {
                    id = last_id;
                } else {
                    auto it = map.find(key);
                    if (it == map.end()) {
                        if (table.size() >= 65535)
                            return fail(FDTD_EINVAL,
                                        "more than 65535 distinct (edge permittivity, PEC, "
                                        "source, probe) node classes");
                        id = (uint32_t)table.size();
                        map.emplace(key, id);
                        table.push_back(ClassEntry{ix, iy, iz, fl});
                        node_aux.insert(node_aux.end(), {fx, fy, fz, lx, ly, lz});
                    } else {
                        id = it->second;
                    }
                    last = key;
                    last_id = id;
                }
                ids[(size_t)dev_index(g, i, j, k)] = (uint16_t)id;
            }
        if (!mat_plane[k]) continue;
        if (tile_need.empty()) tile_need.assign((size_t)hcx * hcy * (nz + 1), 0);
        for (uint8_t bit = 1; bit <= 2; bit <<= 1)
            if (mat_plane[k] & bit) mark_tile_need(need.data(), nx, ny, bit, pre, &tile_need[k], nz + 1);
    }
    g->n_classes = (int)table.size();
    g->wide = table.size() > 256;
    g->mat_plane.swap(mat_plane);
    g->tile_need.swap(tile_need);
    hipStream_t st = g->stream;
    if (g->wide) {
        g->cls = dev_alloc(g, (size_t)NC * 2);
        if (!g->cls) return fail(FDTD_ENOMEM, "class map allocation failed");
        HIP_OR_FAIL(hipMemcpyAsync(g->cls, ids.data(), (size_t)NC * 2, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(hipStreamSynchronize(st));
    } else {
        std::vector<uint8_t> ids8((size_t)NC);
        for (size_t t = 0; t < (size_t)NC; ++t) ids8[t] = (uint8_t)ids[t];
        g->cls = dev_alloc(g, (size_t)NC);
        if (!g->cls) return fail(FDTD_ENOMEM, "class map allocation failed");
        HIP_OR_FAIL(hipMemcpyAsync(g->cls, ids8.data(), (size_t)NC, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(hipStreamSynchronize(st));
    }
    g->ctab = (ClassEntry*)dev_alloc(g, table.size() * sizeof(ClassEntry));
    if (!g->ctab) return fail(FDTD_ENOMEM, "class table allocation failed");
    HIP_OR_FAIL(hipMemcpyAsync(g->ctab, table.data(), table.size() * sizeof(ClassEntry),
                               hipMemcpyHostToDevice, st));
    std::vector<float> tabs[3];
    if (g->node_pass) {
        g->node_aux = (float*)dev_alloc(g, node_aux.size() * 4);
        if (!g->node_aux) return fail(FDTD_ENOMEM, "node table allocation failed");
        HIP_OR_FAIL(hipMemcpyAsync(g->node_aux, node_aux.data(), node_aux.size() * 4, hipMemcpyHostToDevice, st));
        for (int a = 0; a < 3; ++a) {
            const int n1 = (a == 0 ? nx : a == 1 ? ny : nz) + 1;
            tabs[a] = coef_table(d, a, g->dt);
            material_coefs(tabs[a], n1);
            HIP_OR_FAIL(hipMemcpyAsync(g->coef[a], tabs[a].data(), tabs[a].size() * 4,
                                       hipMemcpyHostToDevice, st));
        }
    }
    HIP_OR_FAIL(hipStreamSynchronize(st));   // table, node_aux and tabs are locals

    // sources: Js = c0 dt eta0 J at the half steps (s + 1/2) dt.  A resistive
    // voltage source (R > 0) carries its Norton current c0 dt eta0 V_s / (R dx dy)
    // there and beta = c0 dt eta0 dz / (2 R dx dy), half its lumped conductance.
    const int ns = (int)g->sources.size(), np = (int)g->probes.size();
    const int64_t ms = d.max_steps;
    if (ns) {
        std::vector<float> js((size_t)ns * ms), beta((size_t)ns, 0.f);
        const double sc = kC0 * g->dt * kEta0;
        for (int s = 0; s < ns; ++s) {
            const SourceH& q = g->sources[s];
            const double scale = q.R > 0.0 ? sc / (q.R * d.dx * d.dy) : sc;
            if (q.R > 0.0) beta[s] = (float)(0.5 * sc * d.dz / (q.R * d.dx * d.dy));
            for (int64_t t = 0; t < ms; ++t)
                js[(size_t)s * ms + t] = (float)(scale * waveform(q, (t + 0.5) * g->dt));
        }
        g->src_node = (int32_t*)dev_alloc(g, ns * 4);
        g->src_node64 = (int64_t*)dev_alloc(g, ns * 8);
        g->src_j = (float*)dev_alloc(g, js.size() * 4);
        g->src_beta = (float*)dev_alloc(g, ns * 4);
        if (!g->src_node || !g->src_node64 || !g->src_j || !g->src_beta)
            return fail(FDTD_ENOMEM, "source table allocation failed");
        HIP_OR_FAIL(hipMemcpyAsync(g->src_node, src_node.data(), ns * 4, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(hipMemcpyAsync(g->src_node64, src_node64.data(), ns * 8, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(hipMemcpyAsync(g->src_j, js.data(), js.size() * 4, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(hipMemcpyAsync(g->src_beta, beta.data(), ns * 4, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(hipStreamSynchronize(st));
    }
    if (np) {
        g->prb_node = (int32_t*)dev_alloc(g, np * 4);
        g->prb_node64 = (int64_t*)dev_alloc(g, np * 8);
        g->prb_series = (float*)dev_alloc(g, (size_t)np * ms * 4);
        if (!g->prb_node || !g->prb_node64 || !g->prb_series)
            return fail(FDTD_ENOMEM, "probe buffer allocation failed");
        HIP_OR_FAIL(hipMemcpyAsync(g->prb_node, prb_node.data(), np * 4, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(hipMemcpyAsync(g->prb_node64, prb_node64.data(), np * 8, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(launch_fill_zero(g->prb_series, (int64_t)np * ms, st));
    }
    const int nf = (int)g->freqs.size();
    if (np && nf) {
        g->dft_f = (double*)dev_alloc(g, nf * 8);
        g->dft_re = (double*)dev_alloc(g, (size_t)np * nf * 8);
        g->dft_im = (double*)dev_alloc(g, (size_t)np * nf * 8);
        if (!g->dft_f || !g->dft_re || !g->dft_im) return fail(FDTD_ENOMEM, "DFT buffer allocation failed");
        HIP_OR_FAIL(hipMemcpyAsync(g->dft_f, g->freqs.data(), nf * 8, hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(launch_fill_zero((float*)g->dft_re, (int64_t)np * nf * 2, st));
        HIP_OR_FAIL(launch_fill_zero((float*)g->dft_im, (int64_t)np * nf * 2, st));
    }

    // plane DFT: sample ring (zeroed, so padding columns hold zeros) and FP64
    // accumulators in the padded row layout
    if (g->plane_k >= 0) {
        const int64_t pn = g->pitch * (d.ny + 1);
        const int pf = (int)g->plane_freqs.size();
        g->plane_ring = (float*)dev_alloc(g, (size_t)kPlaneRing * pn * 4);
        g->plane_f = (double*)dev_alloc(g, (size_t)pf * 8);
        g->plane_tw = (double*)dev_alloc(g, (size_t)pf * kPlaneRing * 16);
        g->plane_re = (double*)dev_alloc(g, (size_t)pf * pn * 8);
        g->plane_im = (double*)dev_alloc(g, (size_t)pf * pn * 8);
        if (!g->plane_ring || !g->plane_f || !g->plane_tw || !g->plane_re || !g->plane_im)
            return fail(FDTD_ENOMEM, "plane DFT allocation failed");
        HIP_OR_FAIL(hipMemcpyAsync(g->plane_f, g->plane_freqs.data(), (size_t)pf * 8,
                                   hipMemcpyHostToDevice, st));
        HIP_OR_FAIL(launch_fill_zero(g->plane_ring, (int64_t)kPlaneRing * pn, st));
        HIP_OR_FAIL(launch_fill_zero((float*)g->plane_re, (int64_t)pf * pn * 2, st));
        HIP_OR_FAIL(launch_fill_zero((float*)g->plane_im, (int64_t)pf * pn * 2, st));
    }

    // board descriptor and tile list
    BoardDev& b = g->board_host;
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < 9; ++c) b.f[p][c] = g->f[p][c];
    for (int c = 0; c < 3; ++c) {
        b.d[0][c] = g->dd[0][c];
        b.d[1][c] = g->dd[1][c];
        b.coef[c] = g->coef[c];
    }
    b.cls = g->cls;
    b.ctab = g->ctab;
    b.node_aux = g->node_aux;
    b.src_node = g->src_node;
    b.src_node64 = g->src_node64;
    b.prb_node64 = g->prb_node64;
    b.cstride64 = (uint64_t)g->cstride;
    b.src_j = g->src_j;
    b.src_beta = g->src_beta;
    b.prb_node = g->prb_node;
    b.prb_series = g->prb_series;
    b.step = g->step_dev;
    b.bad = g->bad_dev;
    b.nx = nx;
    b.ny = ny;
    b.nz = nz;
    b.pitch = (int32_t)g->pitch;
    b.cstride = g->big ? 0u : (uint32_t)g->cstride;   // the tiled kernels never run a big board
    b.nsrc = ns;
    b.nprb = np;
    b.nclass = (int32_t)table.size();
    for (int c = 0; c < 6; ++c) b.pml[c] = d.npml[c];
    b.max_steps = ms;
    b.crd_x = (float)(kC0 * g->dt / d.dx);
    b.crd_y = (float)(kC0 * g->dt / d.dy);
    b.crd_z = (float)(kC0 * g->dt / d.dz);
    b.plane_ring = g->plane_ring;
    b.eps_rw = g->pml_eps_rw ? 1 : 0;
    g->board_dev = (BoardDev*)dev_alloc(g, sizeof(BoardDev));
    if (!g->board_dev) return fail(FDTD_ENOMEM, "descriptor allocation failed");
    if (int e = upload_tiles(g)) return e;
    g->step_bytes = count_step_bytes(g);
    g->finalized = true;
    return FDTD_OK;
}

int record_event(fdtd_grid* g)
{
    if (g->ev_used == g->ev_pool.size()) {
        hipEvent_t e;
        HIP_OR_FAIL(hipEventCreate(&e));
        g->ev_pool.push_back(e);
    }
    HIP_OR_FAIL(hipEventRecord(g->ev_pool[g->ev_used++], g->stream));
    return FDTD_OK;
}

int check_bad(fdtd_grid* g)
{
    if (!g->finalized) return FDTD_OK;
    int32_t bad = 0;
    HIP_OR_FAIL(copy_sync(g, &bad, g->bad_dev, 4, hipMemcpyDeviceToHost));
    if (bad) return fail(FDTD_EUNSTABLE, "non-finite field value (unstable run or bad input)");
    return FDTD_OK;
}

}  // namespace

extern "C" {

const char* fdtd_last_error(void) { return g_err.c_str(); }

int fdtd_tile_shapes(int* xys, int cap)
{
    const int n1 = num_shapes(), n2 = num_shapes2();
    for (int q = 0; q < n1 + n2 && q < cap; ++q) {
        if (q < n1)
            shape_at(q, &xys[3 * q], &xys[3 * q + 1]);
        else
            shape2_at(q - n1, &xys[3 * q], &xys[3 * q + 1]);
        xys[3 * q + 2] = q < n1 ? 1 : 2;
    }
    return n1 + n2;
}

int fdtd_create_grid(const fdtd_grid_desc* desc, fdtd_grid** out)
{
    if (!desc || !out) return fail(FDTD_EINVAL, "null argument");
    *out = nullptr;
    fdtd_grid_desc d = *desc;
    if (d.nx < 2 || d.ny < 2 || d.nz < 2) return fail(FDTD_EINVAL, "nx, ny, nz must be >= 2");
    const int64_t nodes = (int64_t)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    const int64_t pitch = row_pitch(d.nx);
    const int64_t dnodes = pitch * (d.ny + 1) * (d.nz + 1);
    const int64_t cstride = component_stride(dnodes);
    // past the 4 GiB window of the tiled kernels' offsets the node passes step
    // the board from per-component bases; they need three planes in 32 bits
    const int64_t plane_bytes = pitch * (d.ny + 1) * 4;
    if (3 * plane_bytes >= (int64_t(1) << 32))
        return fail(FDTD_EINVAL, "grid too large: three node planes (%lld bytes each) must fit 4 GiB",
                    (long long)plane_bytes);
    if (!(d.dx > 0) || !(d.dy > 0) || !(d.dz > 0) || !std::isfinite(d.dx) ||
        !std::isfinite(d.dy) || !std::isfinite(d.dz))
        return fail(FDTD_EINVAL, "cell sizes must be positive and finite");
    if (d.courant == 0.0) d.courant = 0.99;
    if (!(d.courant > 0.0 && d.courant < 1.0)) return fail(FDTD_EINVAL, "courant must be in (0, 1)");
    if (d.pml_m == 0.0) d.pml_m = 3.0;
    if (d.pml_R == 0.0) d.pml_R = 1e-6;
    if (d.pml_kappa_max == 0.0) d.pml_kappa_max = 1.0;
    if (!(d.pml_m > 0.0) || !(d.pml_R > 0.0 && d.pml_R <= 1.0) || !(d.pml_kappa_max >= 1.0))
        return fail(FDTD_EINVAL, "PML parameters out of range");
    const int ncell[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        if (d.npml[2 * a] < 0 || d.npml[2 * a + 1] < 0)
            return fail(FDTD_EINVAL, "PML depths must be >= 0");
        if (d.npml[2 * a] + d.npml[2 * a + 1] > ncell[a])
            return fail(FDTD_EINVAL, "opposite PML layers overlap on axis %d", a);
    }
    if (d.max_steps < 1) return fail(FDTD_EINVAL, "max_steps must be >= 1");
    if ((d.dev_alloc == nullptr) != (d.dev_free == nullptr))
        return fail(FDTD_EINVAL, "dev_alloc and dev_free must be given together");
    // Eq. 7 with the free-space speed (the fastest medium on the grid)
    const double cfl = 1.0 / (kC0 * std::sqrt(1.0 / (d.dx * d.dx) + 1.0 / (d.dy * d.dy) +
                                              1.0 / (d.dz * d.dz)));
    double dt = d.dt;
    if (dt == 0.0) dt = d.courant * cfl;
    if (!(dt > 0.0) || !(dt < cfl)) return fail(FDTD_EINVAL, "dt %.6g is not below the CFL limit %.6g", dt, cfl);

    fdtd_grid* g = new (std::nothrow) fdtd_grid();
    if (!g) return fail(FDTD_ENOMEM, "host allocation failed");
    static std::atomic<uint64_t> next_serial{1};
    g->serial = next_serial.fetch_add(1);
    g->d = d;
    g->dt = dt;
    g->nodes = nodes;
    g->pitch = pitch;
    g->dnodes = dnodes;
    if (hipGetDevice(&g->device) != hipSuccess ||
        hipDeviceGetAttribute(&g->cus, hipDeviceAttributeMultiprocessorCount, g->device) !=
            hipSuccess) {
        delete g;
        return fail(FDTD_EDEVICE, "no HIP device");
    }
    // the allocation-free probe spectrum's fixed scratch: its address on this
    // device is looked up once per device, here, with the device current
    {
        void* s = nullptr;
        if (noalloc_scratch(g->device, &s) != hipSuccess) {
            delete g;
            return fail(FDTD_EDEVICE, "device scratch lookup failed");
        }
    }
    if (d.hip_stream) {
        g->stream = (hipStream_t)d.hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
            delete g;
            return fail(FDTD_EDEVICE, "hipStreamCreate failed");
        }
        g->own_stream = true;
    }
    auto bail = [&](int code, const char* msg) {
        std::string m = msg;
        fdtd_destroy_grid(g);
        return fail(code, "%s", m.c_str());
    };
    // every field array carries kGuard zero words past its last node: the kernels
    // read out-of-range neighbours from there and never write them.  E, H, B and
    // D are one allocation per copy each, holding the x, y and z arrays at a
    // fixed stride, so one base address and a 32-bit offset reach all three.
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 4; ++q) {
            char* blk = (char*)dev_alloc(g, (size_t)(3 * cstride));
            if (!blk) return bail(FDTD_ENOMEM, "field allocation failed");
            if (launch_fill_zero((float*)blk, 3 * cstride / 4, g->stream) != hipSuccess)
                return bail(FDTD_EDEVICE, "zero fill failed");
            for (int c = 0; c < 3; ++c) {
                float* a = (float*)(blk + c * cstride);
                if (q < 3)
                    g->f[p][3 * q + c] = a;
                else
                    g->dd[p][c] = a;
            }
        }
    g->cstride = cstride;
    g->big = 3 * cstride >= (int64_t(1) << 32);
    for (int a = 0; a < 3; ++a) {
        std::vector<float> t = coef_table(d, a, dt);
        if (!(g->coef[a] = (float*)dev_alloc(g, t.size() * 4)))
            return bail(FDTD_ENOMEM, "coefficient allocation failed");
        if (hipMemcpyAsync(g->coef[a], t.data(), t.size() * 4, hipMemcpyHostToDevice, g->stream) !=
                hipSuccess ||
            hipStreamSynchronize(g->stream) != hipSuccess)
            return bail(FDTD_EDEVICE, "coefficient upload failed");
    }
    g->step_dev = (int64_t*)dev_alloc(g, 16);   // step count, field buffer index
    g->bad_dev = (int32_t*)dev_alloc(g, 4);
    if (!g->step_dev || !g->bad_dev) return bail(FDTD_ENOMEM, "counter allocation failed");
    if (launch_fill_zero((float*)g->step_dev, 4, g->stream) != hipSuccess ||
        launch_fill_zero((float*)g->bad_dev, 1, g->stream) != hipSuccess ||
        hipStreamSynchronize(g->stream) != hipSuccess)
        return bail(FDTD_EDEVICE, "counter init failed");
    *out = g;
    return FDTD_OK;
}

int fdtd_set_materials(fdtd_grid* g, const float* eps_r_cell, const uint8_t* pec_edge_mask)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "materials are fixed after the first step");
    if (!eps_r_cell) return fail(FDTD_EINVAL, "eps_r_cell is null");
    const size_t ncell = (size_t)g->d.nx * g->d.ny * g->d.nz;
    for (size_t t = 0; t < ncell; ++t)
        if (!(eps_r_cell[t] >= 1.0f) || !std::isfinite(eps_r_cell[t]))
            return fail(FDTD_EINVAL, "eps_r_cell[%zu] = %g is not finite and >= 1", t,
                        (double)eps_r_cell[t]);
    g->eps.assign(eps_r_cell, eps_r_cell + ncell);
    if (pec_edge_mask)
        g->pec.assign(pec_edge_mask, pec_edge_mask + g->nodes);
    else
        g->pec.assign((size_t)g->nodes, 0);
    g->have_materials = true;
    return FDTD_OK;
}

namespace {

// shared checks of fdtd_add_source and fdtd_add_voltage_source
int check_source(fdtd_grid* g, int i, int j, int k, int waveform, double J0, double t0,
                 double sigma)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "sources are fixed after the first step");
    if (i < 1 || i >= g->d.nx || j < 1 || j >= g->d.ny || k < 0 || k >= g->d.nz)
        return fail(FDTD_EINVAL, "source (%d,%d,%d) is not an interior Ez edge", i, j, k);
    if (waveform != FDTD_WAVE_GAUSS && waveform != FDTD_WAVE_DGAUSS)
        return fail(FDTD_EINVAL, "unknown waveform %d", waveform);
    if (!(sigma > 0) || !std::isfinite(J0) || !std::isfinite(t0) || !std::isfinite(sigma))
        return fail(FDTD_EINVAL, "source parameters must be finite with sigma > 0");
    if (g->have_materials && (g->pec[node_index(g, i, j, k)] & 4))
        return fail(FDTD_EINVAL, "source at (%d,%d,%d) sits on a PEC edge", i, j, k);
    return FDTD_OK;
}

// a resistive source owns its edge: no second source of either kind may share it
bool edge_has_resistor(const fdtd_grid* g, int i, int j, int k, bool any)
{
    for (const SourceH& s : g->sources)
        if (s.i == i && s.j == j && s.k == k && (any || s.R > 0.0)) return true;
    return false;
}

}  // namespace

int fdtd_add_source(fdtd_grid* g, int i, int j, int k, int waveform, double J0, double t0,
                    double sigma, int* id)
{
    if (int e = check_source(g, i, j, k, waveform, J0, t0, sigma)) return e;
    if (edge_has_resistor(g, i, j, k, false))
        return fail(FDTD_EINVAL, "edge (%d,%d,%d) already holds a resistive source", i, j, k);
    g->sources.push_back(SourceH{i, j, k, waveform, J0, t0, sigma, 0.0});
    if (id) *id = (int)g->sources.size() - 1;
    return FDTD_OK;
}

int fdtd_add_voltage_source(fdtd_grid* g, int i, int j, int k, int waveform, double V0,
                            double t0, double sigma, double R, int* id)
{
    if (int e = check_source(g, i, j, k, waveform, V0, t0, sigma)) return e;
    if (!(R > 0.0) || !std::isfinite(R))
        return fail(FDTD_EINVAL, "source resistance must be finite and > 0");
    const int* p = g->d.npml;
    if (i < p[0] || i >= g->d.nx - p[1] || j < p[2] || j >= g->d.ny - p[3] || k < p[4] ||
        k >= g->d.nz - p[5])
        return fail(FDTD_EINVAL, "resistive source (%d,%d,%d) lies in a PML slab", i, j, k);
    if (edge_has_resistor(g, i, j, k, true))
        return fail(FDTD_EINVAL, "edge (%d,%d,%d) already holds a source", i, j, k);
    g->sources.push_back(SourceH{i, j, k, waveform, V0, t0, sigma, R});
    if (id) *id = (int)g->sources.size() - 1;
    return FDTD_OK;
}

int fdtd_add_probe(fdtd_grid* g, int i, int j, int k, int* id)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "probes are fixed after the first step");
    if (i < 0 || i > g->d.nx || j < 0 || j > g->d.ny || k < 0 || k >= g->d.nz)
        return fail(FDTD_EINVAL, "probe (%d,%d,%d) is outside the grid", i, j, k);
    g->probes.push_back({i, j, k});
    if (id) *id = (int)g->probes.size() - 1;
    return FDTD_OK;
}

int fdtd_add_voltage_probe(fdtd_grid* g, int i, int j, int k0, int k1, int* id)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "probes are fixed after the first step");
    if (i < 0 || i > g->d.nx || j < 0 || j > g->d.ny || k0 < 0 || k1 <= k0 || k1 > g->d.nz)
        return fail(FDTD_EINVAL, "voltage probe (%d,%d,%d..%d) is outside the grid", i, j, k0, k1);
    const int first = (int)g->probes.size();
    for (int k = k0; k < k1; ++k) g->probes.push_back({i, j, k});
    g->vprobes.push_back(VoltageProbeH{first, k1 - k0});
    if (id) *id = (int)g->vprobes.size() - 1;
    return FDTD_OK;
}

int fdtd_set_conductivity(fdtd_grid* g, const float* sigma_cell)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "the conductivity is fixed after the first step");
    const fdtd_grid_desc& d = g->d;
    if (!sigma_cell) {
        g->sigma.clear();
        return FDTD_OK;
    }
    const int* p = d.npml;
    bool any = false;
    for (int k = 0; k < d.nz; ++k)
        for (int j = 0; j < d.ny; ++j)
            for (int i = 0; i < d.nx; ++i) {
                const float v = sigma_cell[(size_t)i + (size_t)d.nx * ((size_t)j + (size_t)d.ny * k)];
                if (!(v >= 0.f) || !std::isfinite(v))
                    return fail(FDTD_EINVAL, "conductivity of cell (%d,%d,%d) is negative or not finite", i, j, k);
                const bool slab = i < p[0] || i >= d.nx - p[1] || j < p[2] || j >= d.ny - p[3] ||
                                  k < p[4] || k >= d.nz - p[5];
                if (v != 0.f && slab)
                    return fail(FDTD_EINVAL, "conductive cell (%d,%d,%d) lies in a PML slab", i, j, k);
                any |= v != 0.f;
            }
    if (any)
        g->sigma.assign(sigma_cell, sigma_cell + (size_t)d.nx * d.ny * d.nz);
    else
        g->sigma.clear();
    return FDTD_OK;
}

int fdtd_set_sheet_resistance(fdtd_grid* g, double ohms_per_square)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "the sheet resistance is fixed after the first step");
    if (!(ohms_per_square >= 0.0) || !std::isfinite(ohms_per_square))
        return fail(FDTD_EINVAL, "sheet resistance must be finite and >= 0");
    g->sheet_R = ohms_per_square;
    return FDTD_OK;
}

int fdtd_set_pml_eps_rw(fdtd_grid* g, int on)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "eps_rw is fixed after the first step");
    g->pml_eps_rw = on != 0;
    return FDTD_OK;
}

int fdtd_set_plane_dft(fdtd_grid* g, int k, const double* f_hz, int nf)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "the plane DFT is fixed after the first step");
    if (k < 0 || k >= g->d.nz) return fail(FDTD_EINVAL, "plane %d is not an Ez plane (0 <= k < nz)", k);
    if (!f_hz || nf < 1 || nf > 256) return fail(FDTD_EINVAL, "need 1 <= nf <= 256 frequencies");
    for (int q = 0; q < nf; ++q)
        if (!(f_hz[q] >= 0.0) || !std::isfinite(f_hz[q]))
            return fail(FDTD_EINVAL, "frequency %d is negative or not finite", q);
    // ring slots are addressed with 32-bit byte offsets
    if ((int64_t)kPlaneRing * g->pitch * (g->d.ny + 1) * 4 >= (int64_t(1) << 32))
        return fail(FDTD_EINVAL, "plane too large for the plane DFT (more than 2^25 padded nodes)");
    g->plane_k = k;
    g->plane_freqs.assign(f_hz, f_hz + nf);
    return FDTD_OK;
}

int fdtd_set_dft_freqs(fdtd_grid* g, const double* f_hz, int nf)
{
    if (int e = check_grid(g)) return e;
    if (g->finalized) return fail(FDTD_ESTATE, "DFT frequencies are fixed after the first step");
    if (!f_hz || nf < 1 || nf > 4096) return fail(FDTD_EINVAL, "need 1 <= nf <= 4096 frequencies");
    for (int q = 0; q < nf; ++q)
        if (!(f_hz[q] >= 0.0) || !std::isfinite(f_hz[q]))
            return fail(FDTD_EINVAL, "frequency %d is negative or not finite", q);
    g->freqs.assign(f_hz, f_hz + nf);
    return FDTD_OK;
}

// Work list of the handle's board for a shape, in device memory (reallocated when
// it grows).
static int upload_work(fdtd_grid* g, const std::vector<TileRef>& tl, TileRef** dev, int* n, int* cap)
{
    if (tl.empty()) {
        *n = 0;
        return FDTD_OK;
    }
    const int nt = (int)tl.size();
    if (nt > *cap) {
        *dev = (TileRef*)dev_alloc(g, tl.size() * sizeof(TileRef));
        if (!*dev) return fail(FDTD_ENOMEM, "tile list allocation failed");
        *cap = nt;
    }
    HIP_OR_FAIL(copy_sync(g, *dev, tl.data(), tl.size() * sizeof(TileRef), hipMemcpyHostToDevice));
    *n = nt;
    return FDTD_OK;
}

// Work list of given two-step pieces of the handle's board (64 x ty tiles) for
// the kernel of `mode` (as slots_per_xcd).
static int upload_pieces(fdtd_grid* g, int ty, int mode, const std::vector<TileRef>& pieces,
                         TileRef** dev, int* n, int* cap)
{
    std::vector<TileRef> tl;
    build_work(pieces, slots_per_xcd(g, 64, ty, 2, g->wide, mode), tl);
    return upload_work(g, tl, dev, n, cap);
}

static int upload_list(fdtd_grid* g, int tx, int ty, int steps, TileRef** dev, int* n, int* cap)
{
    std::vector<TileRef> whole, tl;
    board_tiles(0, g->d.nx, g->d.ny, g->d.nz, tx, owned_rows(ty, steps), whole);
    build_work(whole, slots_per_xcd(g, tx, ty, steps, g->wide, 0), tl);
    if (tl.empty()) {
        *n = 0;
        return FDTD_OK;
    }
    const int nt = (int)tl.size();
    if (nt > *cap) {
        *dev = (TileRef*)dev_alloc(g, tl.size() * sizeof(TileRef));
        if (!*dev) return fail(FDTD_ENOMEM, "tile list allocation failed");
        *cap = nt;
    }
    HIP_OR_FAIL(copy_sync(g, *dev, tl.data(), tl.size() * sizeof(TileRef), hipMemcpyHostToDevice));
    *n = nt;
    return FDTD_OK;
}

static int upload_tiles(fdtd_grid* g)
{
    BoardDev& b = g->board_host;
    if (g->node_pass) {
        // a material board takes pairs of steps on two-step kernels of one shape,
        // 64 x kHybridTY x 2 (the plain kernel and its material variant), when a
        // two-step shape is set, the default; with a one-step shape, and on
        // boards past the tiled kernels' offset window, every step runs the
        // node passes
        g->mat = !g->big && g->tile_steps == 2;
        if (g->mat) {
            g->tile_x = 64;
            g->tile_y = kHybridTY;
        }
    }
    tile_counts(g->d.nx, g->d.ny, g->tile_x, owned_rows(g->tile_y, g->tile_steps), &b.tiles_x,
                &b.tiles_y);
    g->ntilesP = 0;
    g->ntilesC = 0;
    g->mat_permille = 0;
    g->cond_permille = 0;
    g->mat_split = 0;
    if (g->mat) {
        // Tile planes near nodes that need the material arithmetic run a variant
        // of the plain kernel, the rest the plain kernel (split_material).  The
        // kernels read one field copy and write the other, each its own pieces'
        // nodes, and give the node passes' bits.
        MaterialSplit ms;
        split_material(g->d.nx, g->d.ny, g->d.nz, g->tile_need, ms);
        g->mat_ty = ms.mat_ty;
        g->mat_split = ms.split;
        g->mat_permille = ms.mat_permille;
        g->cond_permille = ms.cond_permille;
        g->pc_plain = ms.plain;
        g->pc_cd = ms.cd;
        g->pc_rb = ms.rb;
        if (int e = upload_pieces(g, g->mat_ty, 1, ms.rb, &g->tiles_dev, &g->ntiles, &g->tiles_cap))
            return e;
        if (int e = upload_pieces(g, kHybridTY, 2, ms.cd, &g->tilesC_dev, &g->ntilesC, &g->tilesC_cap))
            return e;
        if (int e = upload_pieces(g, kHybridTY, 0, ms.plain, &g->tilesP_dev, &g->ntilesP, &g->tilesP_cap))
            return e;
        if (g->ntilesP > 0 && g->ntiles + g->ntilesC > 0 && !g->aux_stream) {
            HIP_OR_FAIL(hipStreamCreateWithFlags(&g->aux_stream, hipStreamNonBlocking));
            HIP_OR_FAIL(hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming));
            HIP_OR_FAIL(hipEventCreateWithFlags(&g->join_ev, hipEventDisableTiming));
        }
    } else if (int e = upload_list(g, g->tile_x, g->tile_y, g->tile_steps, &g->tiles_dev, &g->ntiles,
                                   &g->tiles_cap)) {
        return e;
    }
    if (g->tile_steps == 2 && !g->node_pass)
        if (int e = upload_list(g, kOddX, kOddY, 1, &g->tiles1_dev, &g->ntiles1, &g->tiles1_cap))
            return e;
    HIP_OR_FAIL(copy_sync(g, g->board_dev, &b, sizeof(BoardDev), hipMemcpyHostToDevice));
    if (g->graph_exec) {
        (void)hipGraphExecDestroy(g->graph_exec);
        g->graph_exec = nullptr;
    }
    g->graph_failed = false;
    return FDTD_OK;
}

int fdtd_set_tile(fdtd_grid* g, int tile_x, int tile_y, int steps)
{
    if (int e = check_grid(g)) return e;
    bool found = false;
    if (steps == 1) {
        for (int q = 0; q < num_shapes() && !found; ++q) {
            int tx, ty;
            shape_at(q, &tx, &ty);
            found = tx == tile_x && ty == tile_y;
        }
    } else if (steps == 2) {
        for (int q = 0; q < num_shapes2() && !found; ++q) {
            int tx, ty;
            shape2_at(q, &tx, &ty);
            found = tx == tile_x && ty == tile_y;
        }
    }
    if (!found)
        return fail(FDTD_EINVAL, "unsupported tile shape %dx%d with %d steps per pass", tile_x,
                    tile_y, steps);
    g->tile_x = tile_x;
    g->tile_y = tile_y;
    g->tile_steps = steps;
    return g->finalized ? upload_tiles(g) : FDTD_OK;
}

// Fold the plane-DFT samples of steps [step + rel_from, step + rel_to) into the
// accumulators (step: the device counter when the fold runs).
static int fold_plane(fdtd_grid* g, int64_t rel_from, int64_t rel_to, hipStream_t st)
{
    if (g->plane_k < 0) return FDTD_OK;
    HIP_OR_FAIL(launch_plane_fold(g->plane_ring, g->pitch * (g->d.ny + 1), g->plane_f,
                                  (int)g->plane_freqs.size(), g->dt, g->step_dev, rel_from, rel_to,
                                  g->plane_tw, g->plane_re, g->plane_im, st));
    return FDTD_OK;
}

// One step of a material board on the node passes (an H pass, then an E pass).
static hipError_t node_step(fdtd_grid* g, int rel, int flip, hipStream_t st)
{
    return launch_eps_step(g->board_dev, g->d.nx, g->d.ny, g->d.nz, g->pitch * (g->d.ny + 1) * 4,
                           g->big, rel, flip, g->wide, st);
}

// A pair of steps of a material board: the plain two-step kernel over the z runs
// clear of material nodes, the material variant over the rest.
static hipError_t material_pair(fdtd_grid* g, int rel, int flip, hipStream_t st)
{
    const bool plane = g->plane_k >= 0;
    // the variants' pieces on the second stream beside the plain kernel's
    const bool fork = g->ntilesP > 0 && g->ntiles + g->ntilesC > 0 && g->aux_stream;
    hipStream_t vs = fork ? g->aux_stream : st;
    hipError_t e = hipSuccess;
    if (fork) {
        e = hipEventRecord(g->fork_ev, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(vs, g->fork_ev, 0);
    }
    const bool nt = stream_stores(&g, 1);
    if (e == hipSuccess && g->ntiles > 0)
        e = launch_field_step2_material(g->mat_ty, 1, g->board_dev, g->tiles_dev, g->ntiles, rel, flip,
                                        g->wide, plane, nt, vs);
    if (e == hipSuccess && g->ntilesC > 0)
        e = launch_field_step2_material(kHybridTY, 2, g->board_dev, g->tilesC_dev, g->ntilesC, rel,
                                        flip, g->wide, plane, nt, vs);
    if (e == hipSuccess && g->ntilesP > 0)
        e = launch_field_step2(kHybridTY, g->board_dev, g->tilesP_dev, g->ntilesP, rel, flip, g->wide,
                               plane, nt, st);
    if (fork) {
        if (e == hipSuccess) e = hipEventRecord(g->join_ev, vs);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, g->join_ev, 0);
    }
    return e;
}

// One field launch of the handle's shape (two steps, or one with the odd-step
// shape when `single`; a material board's odd step runs the node passes),
// optionally bracketed by timing events.
static int enqueue_launch(fdtd_grid* g, bool single, int rel, int flip)
{
    if (g->timing)
        if (int e = record_event(g)) return e;
    if (g->mat)
        HIP_OR_FAIL(single ? node_step(g, rel, flip, g->stream) : material_pair(g, rel, flip, g->stream));
    else if (single && g->tile_steps == 2)
        HIP_OR_FAIL(launch_pass(kOddX, kOddY, 1, g->board_dev, g->tiles1_dev, g->ntiles1, rel, flip,
                                g->wide, g->plane_k >= 0, false, g->stream));
    else
        HIP_OR_FAIL(launch_pass(g->tile_x, g->tile_y, g->tile_steps, g->board_dev, g->tiles_dev,
                                g->ntiles, rel, flip, g->wide, g->plane_k >= 0, stream_stores(&g, 1),
                                g->stream));
    if (g->timing) {
        if (int e = record_event(g)) return e;
        ++g->timed_launches;
    }
    return FDTD_OK;
}

// Enqueue n steps as launches of the handle's shape (two-step shapes end with
// one single step when n is odd); returns the launch count through *launches.
static int enqueue_steps(fdtd_grid* g, int64_t n, int64_t* launches)
{
    if (g->node_pass && !g->mat) {
        // one H pass and one E pass per step (one buffer flip)
        for (int64_t s = 0; s < n; ++s) {
            if (g->timing)
                if (int e = record_event(g)) return e;
            HIP_OR_FAIL(node_step(g, (int)s, (int)(s & 1), g->stream));
            if (g->timing) {
                if (int e = record_event(g)) return e;
                ++g->timed_launches;
            }
        }
        *launches = n;
        return FDTD_OK;
    }
    const int per = g->tile_steps;
    int64_t l = 0, s = 0;
    for (; s + per <= n; s += per, ++l)
        if (int e = enqueue_launch(g, false, (int)s, (int)(l & 1))) return e;
    for (; s < n; ++s, ++l)
        if (int e = enqueue_launch(g, true, (int)s, (int)(l & 1))) return e;
    *launches = l;
    return FDTD_OK;
}

// Capture the launches of kGraphChunk steps and the counter advance into one
// graph.  The kernels take the step and the field buffer from the device
// counters, and a chunk has an even number of launches, so the same graph serves
// every chunk.  Any failure leaves plain launches in use.
static void build_graph(fdtd_grid* g)
{
    if (g->graph_exec || g->graph_failed) return;
    g->graph_failed = true;
    if (!g->own_stream && g->stream == nullptr) return;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return;
    bool ok = true;
    const int per = g->node_pass && !g->mat ? 1 : g->tile_steps, nl = kGraphChunk / per;
    for (int l = 0; l < nl && ok; ++l)
        ok = (g->mat         ? material_pair(g, l * per, l & 1, g->stream)
              : g->node_pass ? node_step(g, l, l & 1, g->stream)
                             : launch_pass(g->tile_x, g->tile_y, per, g->board_dev, g->tiles_dev,
                                           g->ntiles, l * per, l & 1, g->wide, g->plane_k >= 0,
                                           stream_stores(&g, 1), g->stream)) == hipSuccess;
    if (ok) ok = launch_advance_one(g->step_dev, kGraphChunk, nl, g->stream) == hipSuccess;
    if (ok) ok = fold_plane(g, -kGraphChunk, 0, g->stream) == FDTD_OK;
    const bool ended = hipStreamEndCapture(g->stream, &graph) == hipSuccess;
    if (ok && ended && graph &&
        hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0) == hipSuccess)
        g->graph_failed = false;
    else
        g->graph_exec = nullptr;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
}

int fdtd_step_n(fdtd_grid* g, int64_t n)
{
    if (int e = check_grid(g)) return e;
    if (n < 0) return fail(FDTD_EINVAL, "negative step count");
    if (g->step + n > g->d.max_steps)
        return fail(FDTD_ESTATE, "%lld steps would exceed max_steps %lld",
                    (long long)(g->step + n), (long long)g->d.max_steps);
    if (int e = finalize(g)) return e;
    if (n == 0) return FDTD_OK;
    int64_t done = 0, launches = 0;
    if (!g->timing && n >= kGraphChunk) {
        build_graph(g);
        if (g->graph_exec) {
            for (; done + kGraphChunk <= n; done += kGraphChunk) {
                HIP_OR_FAIL(hipGraphLaunch(g->graph_exec, g->stream));
                launches += kGraphChunk / (g->node_pass && !g->mat ? 1 : g->tile_steps);
            }
        }
    }
    while (done < n) {
        // kernels add the launch-relative step and buffer to the device counters,
        // which the graphs above have already advanced; with a plane DFT the ring
        // is folded at least every kPlaneRing steps
        const int64_t m = g->plane_k >= 0 ? std::min<int64_t>(n - done, kPlaneRing) : n - done;
        int64_t l = 0;
        if (int e = enqueue_steps(g, m, &l)) return e;
        HIP_OR_FAIL(launch_advance_one(g->step_dev, m, l, g->stream));
        if (int e = fold_plane(g, -m, 0, g->stream)) return e;
        launches += l;
        done += m;
    }
    if (g->dft_f)
        HIP_OR_FAIL(launch_dft(g->prb_series, g->d.max_steps, g->dft_f, (int)g->freqs.size(),
                               (int)g->probes.size(), g->dt, g->step, g->step + n, g->dft_re,
                               g->dft_im, g->stream));
    g->step += n;
    g->buf = (int)((g->buf + launches) & 1);
    return FDTD_OK;
}

static int ensure_event(fdtd_grid* g)
{
    if (!g->sync_ev) HIP_OR_FAIL(hipEventCreateWithFlags(&g->sync_ev, hipEventDisableTiming));
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// Batched stepping.  A call is planned once per (handles, step counts, lead
// shape): the per-board descriptors, the balanced work lists and the counter
// advances of every round go to one device buffer, and the call's launches are
// captured into a graph that later calls with the same plan replay (one graph
// launch per call).  Plans live with the lead handle.

namespace {

// launches of one work list: passes s0 .. s1-1 of `steps` steps each, or the
// single-step tail launch (which reads the boards' tail copies)
// Passes s0 .. s1-1 of a set of boards: each pass is one launch per list, in
// list order (the lists of one board's pieces depend on each other pass by pass).
struct Span {
    int w, steps;
    int64_t s0, s1;
    int nl = 0;       // lists
    int kind[4];      // 0 the plain group's whole tiles (the lead's shape); a material board's
                      // pieces: 1 plain, 2 conduction-only, 3 material 64 x kHybridTY, 4 material
                      // 64 x kMatTY
    int off[4], count[4];   // into the round's tile list
    bool tail;
};

// A material board's odd last step of a round, on the node passes.
struct NodeTail {
    int h;            // handle (call order)
    int rel, flip;    // after the board's pairs of the round
};

// One round: every handle advances by n[h] steps (at most kPlaneRing when some
// handle keeps a plane DFT, whose ring is folded after every round).
struct RoundHost {
    std::vector<int64_t> n;         // per handle, call order
    std::vector<int> order;         // boards in launch order
    std::vector<BoardDev> boards;   // [0, ng): passes; [ng, 2 ng): the single-step tail
    std::vector<int64_t> adv;       // per board: steps, launches (field-buffer flips)
    std::vector<Span> spans;
    std::vector<TileRef> items;
    std::vector<NodeTail> node_tails;
};

}  // namespace

struct BatchPlan {
    std::vector<uint64_t> key;
    std::vector<int64_t> n;          // per handle, the call's steps
    std::vector<int64_t> flips;      // per handle, field-buffer flips of the call
    std::vector<RoundHost> rounds;
    char* dev = nullptr;             // device tables of every round
    size_t dev_bytes = 0;
    std::vector<size_t> off_boards, off_adv, off_tiles;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;       // recorded after every launch of the plan
    uint64_t used = 0;
};

namespace {

// Host side of one round (board order, descriptors, work lists).
void plan_round(fdtd_grid* const* gs, int ng, const int64_t* n, RoundHost& r)
{
    fdtd_grid* lead = gs[0];
    const int tx = lead->tile_x, ty = lead->tile_y, per = lead->tile_steps;
    r.n.assign(n, n + ng);
    // order boards by step count (descending): at pass s the boards still running
    // form a prefix, and so do their tiles; narrow and wide class maps, and
    // material boards, go to separate launches (the kernel is specialised on
    // the class index width and on the material arithmetic)
    r.order.resize(ng);
    for (int h = 0; h < ng; ++h) r.order[h] = h;
    auto group = [&](int h) { return 2 * (int)gs[h]->mat + (int)gs[h]->wide; };
    std::stable_sort(r.order.begin(), r.order.end(), [&](int a, int b) {
        if (group(a) != group(b)) return group(a) < group(b);
        return n[a] > n[b];
    });
    // board b runs np[b] passes of `per` steps, then (two-step shapes) one single
    // step when its count is odd.  boards[ng + b] is the copy the single-step
    // launch reads: its step and buffer offsets skip the board's own passes.
    r.boards.assign(2 * (size_t)ng, BoardDev{});
    r.adv.assign(2 * (size_t)ng, 0);
    std::vector<int64_t> np(ng), odd(ng);
    int64_t max_np = 0;
    for (int b = 0; b < ng; ++b) {
        const int64_t nb = n[r.order[b]];
        const int pb = gs[r.order[b]]->mat ? 2 : per;
        np[b] = nb / pb;
        odd[b] = nb - np[b] * pb;
        max_np = std::max(max_np, np[b]);
        r.boards[b] = gs[r.order[b]]->board_host;
        r.boards[ng + b] = r.boards[b];
        r.boards[ng + b].rel0 = (int32_t)(np[b] * pb);
        r.boards[ng + b].flip0 = (int32_t)(np[b] & 1);
        r.adv[2 * b] = nb;
        r.adv[2 * b + 1] = np[b] + odd[b];
    }
    // Each group (class width, material or not) is a range [b0, b1) of the
    // order; at pass s the boards still running are a prefix [b0, active) of it.
    // One balanced work list per distinct prefix, plus one for the single-step
    // tail, all in one buffer; a material board's single step runs the node
    // passes on its own.
    r.spans.clear();
    r.items.clear();
    r.node_tails.clear();
    std::vector<TileRef> whole, list;
    for (int grp = 0; grp < 4; ++grp) {
        const int w = grp & 1;
        const bool mat = grp >= 2;
        int b0 = 0;
        while (b0 < ng && group(r.order[b0]) != grp) ++b0;
        if (b0 == ng) continue;
        int b1 = b0;
        while (b1 < ng && group(r.order[b1]) == grp) ++b1;
        int64_t s = 0;
        for (int active = b1; active > b0 && s < max_np;) {
            const int64_t s_end = np[active - 1];  // boards [b0, active) all run through s_end
            if (s_end > s) {
                // plain boards: whole tiles of the lead's shape; material boards:
                // their own pieces (plain, conduction-only, material), each kind a
                // list (and a launch per pass) of its own
                Span sp{w, mat ? 2 : per, s, s_end};
                sp.tail = false;
                for (int kind = mat ? 1 : 0; kind <= (mat ? 4 : 0); ++kind) {
                    const int kty = kind == 0 ? ty : kind == 4 ? kMatTY : kHybridTY;
                    const int ktx = kind == 0 ? tx : 64, kper = kind == 0 ? per : 2;
                    const int mode = kind >= 3 ? 1 : kind == 2 ? 2 : 0;
                    whole.clear();
                    for (int b = b0; b < active; ++b) {
                        const fdtd_grid* g = gs[r.order[b]];
                        if (kind == 0) {
                            board_tiles(b, g->d.nx, g->d.ny, g->d.nz, tx, owned_rows(ty, per), whole);
                            continue;
                        }
                        const std::vector<TileRef>* pc =
                            kind == 1 ? &g->pc_plain
                                      : kind == 2 ? &g->pc_cd
                                                  : (g->mat_ty == (kind == 3 ? kHybridTY : kMatTY)
                                                         ? &g->pc_rb
                                                         : nullptr);
                        if (pc)
                            for (TileRef t : *pc) {
                                t.board = b;
                                whole.push_back(t);
                            }
                    }
                    if (whole.empty()) continue;
                    build_work(whole, slots_per_xcd(lead, ktx, kty, kper, w == 1, mode), list);
                    sp.kind[sp.nl] = kind;
                    sp.off[sp.nl] = (int)r.items.size();
                    sp.count[sp.nl] = (int)list.size();
                    ++sp.nl;
                    r.items.insert(r.items.end(), list.begin(), list.end());
                }
                if (sp.nl > 0) r.spans.push_back(sp);
                s = s_end;
            }
            --active;
        }
        if (mat) {
            for (int b = b0; b < b1; ++b)
                if (odd[b])
                    r.node_tails.push_back(NodeTail{r.order[b], (int)(np[b] * 2), (int)(np[b] & 1)});
            continue;
        }
        whole.clear();
        for (int b = b0; b < b1; ++b)
            if (odd[b]) {
                const fdtd_grid* g = gs[r.order[b]];
                board_tiles(b, g->d.nx, g->d.ny, g->d.nz, kOddX, owned_rows(kOddY, 1), whole);
            }
        if (!whole.empty()) {
            build_work(whole, slots_per_xcd(lead, kOddX, kOddY, 1, w == 1, 0), list);
            Span sp{w, 1, 0, 1};
            sp.nl = 1;
            sp.kind[0] = 0;
            sp.off[0] = (int)r.items.size();
            sp.count[0] = (int)list.size();
            sp.tail = true;
            r.spans.push_back(sp);
            r.items.insert(r.items.end(), list.begin(), list.end());
        }
    }
}

bool any_plane(fdtd_grid* const* gs, int ng)
{
    for (int h = 0; h < ng; ++h)
        if (gs[h]->plane_k >= 0) return true;
    return false;
}

void free_plan(fdtd_grid* lead, BatchPlan* p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->dev) {
        temp_free(lead, p->dev);
        lead->device_bytes -= (int64_t)p->dev_bytes;
    }
    delete p;
}

// Enqueue a plan's launches on st (also used inside graph capture): every
// round's field launches and counter advance, the plane folds after each
// round, then each handle's probe DFT over the whole call.
int enqueue_plan(fdtd_grid* const* gs, int ng, const BatchPlan& P, hipStream_t st)
{
    const fdtd_grid* lead = gs[0];
    const int tx = lead->tile_x, ty = lead->tile_y;
    const bool planes = any_plane(gs, ng), nt = stream_stores(gs, ng);
    for (size_t q = 0; q < P.rounds.size(); ++q) {
        const RoundHost& R = P.rounds[q];
        const BoardDev* db = (const BoardDev*)(P.dev + P.off_boards[q]);
        const int64_t* dn = (const int64_t*)(P.dev + P.off_adv[q]);
        const TileRef* dt = (const TileRef*)(P.dev + P.off_tiles[q]);
        for (const Span& sp : R.spans) {
            if (sp.tail) {
                HIP_OR_FAIL(launch_pass(kOddX, kOddY, 1, db + ng, dt + sp.off[0], sp.count[0], 0, 0,
                                        sp.w == 1, planes, false, st));
                continue;
            }
            const bool wide = sp.w == 1;
            for (int64_t k = sp.s0; k < sp.s1; ++k) {
                const int rel = (int)(k * sp.steps), flip = (int)(k & 1);
                for (int l = 0; l < sp.nl; ++l) {
                    const TileRef* tl = dt + sp.off[l];
                    const int n = sp.count[l];
                    hipError_t e;
                    switch (sp.kind[l]) {
                        case 0:
                            e = launch_pass(tx, ty, sp.steps, db, tl, n, rel, flip, wide, planes, nt,
                                            st);
                            break;
                        case 1:
                            e = launch_field_step2(kHybridTY, db, tl, n, rel, flip, wide, planes, nt,
                                                   st);
                            break;
                        case 2:
                            e = launch_field_step2_material(kHybridTY, 2, db, tl, n, rel, flip, wide,
                                                            planes, nt, st);
                            break;
                        case 3:
                            e = launch_field_step2_material(kHybridTY, 1, db, tl, n, rel, flip, wide,
                                                            planes, nt, st);
                            break;
                        default:
                            e = launch_field_step2_material(kMatTY, 1, db, tl, n, rel, flip, wide,
                                                            planes, nt, st);
                            break;
                    }
                    HIP_OR_FAIL(e);
                }
            }
        }
        for (const NodeTail& t : R.node_tails)
            HIP_OR_FAIL(node_step(gs[t.h], t.rel, t.flip, st));
        HIP_OR_FAIL(launch_advance((BoardDev*)db, ng, dn, st));
        for (int h = 0; h < ng; ++h)
            if (R.n[h] > 0)
                if (int e = fold_plane(gs[h], -R.n[h], 0, st)) return e;
    }
    for (int h = 0; h < ng; ++h) {
        const fdtd_grid* g = gs[h];
        if (g->dft_f && P.n[h] > 0)
            HIP_OR_FAIL(launch_dft_back(g->prb_series, g->d.max_steps, g->dft_f,
                                        (int)g->freqs.size(), (int)g->probes.size(), g->dt,
                                        g->step_dev, P.n[h], g->dft_re, g->dft_im, st));
    }
    return FDTD_OK;
}

// Plan a batched call: rounds, device tables (copied with a synchronous copy
// that does not wait for the handles' streams) and, where the lead's stream can
// be captured, the graph of its launches.
int build_plan(fdtd_grid* const* gs, int ng, const int64_t* n, BatchPlan* P)
{
    fdtd_grid* lead = gs[0];
    P->n.assign(n, n + ng);
    P->flips.assign(ng, 0);
    std::vector<int64_t> left(n, n + ng), r(ng);
    const bool planes = any_plane(gs, ng);
    for (bool more = true; more;) {
        more = false;
        for (int h = 0; h < ng; ++h) {
            r[h] = planes ? std::min<int64_t>(left[h], kPlaneRing) : left[h];
            left[h] -= r[h];
            more |= left[h] > 0;
        }
        P->rounds.emplace_back();
        plan_round(gs, ng, r.data(), P->rounds.back());
        const RoundHost& R = P->rounds.back();
        for (int b = 0; b < ng; ++b) P->flips[R.order[b]] += R.adv[2 * b + 1];
    }
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t total = 0;
    for (const RoundHost& R : P->rounds) {
        P->off_boards.push_back(total);
        total += up(R.boards.size() * sizeof(BoardDev));
        P->off_adv.push_back(total);
        total += up(R.adv.size() * sizeof(int64_t));
        P->off_tiles.push_back(total);
        total += up(std::max<size_t>(1, R.items.size()) * sizeof(TileRef));
    }
    std::vector<char> host(total, 0);
    for (size_t q = 0; q < P->rounds.size(); ++q) {
        const RoundHost& R = P->rounds[q];
        memcpy(host.data() + P->off_boards[q], R.boards.data(), R.boards.size() * sizeof(BoardDev));
        memcpy(host.data() + P->off_adv[q], R.adv.data(), R.adv.size() * sizeof(int64_t));
        if (!R.items.empty())
            memcpy(host.data() + P->off_tiles[q], R.items.data(), R.items.size() * sizeof(TileRef));
    }
    HIP_OR_FAIL(hipEventCreateWithFlags(&P->done, hipEventDisableTiming));
    P->dev = (char*)temp_alloc(lead, total);
    if (!P->dev) return fail(FDTD_ENOMEM, "batch plan allocation failed");
    P->dev_bytes = up(total);
    lead->device_bytes += (int64_t)P->dev_bytes;
    HIP_OR_FAIL(hipMemcpy(P->dev, host.data(), total, hipMemcpyHostToDevice));
    // capture the launches (a stream that cannot be captured keeps plain launches)
    if (!lead->own_stream && lead->stream == nullptr) return FDTD_OK;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(lead->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const int e = enqueue_plan(gs, ng, *P, lead->stream);
        const bool ended = hipStreamEndCapture(lead->stream, &graph) == hipSuccess;
        if (e != FDTD_OK || !ended || !graph ||
            hipGraphInstantiate(&P->exec, graph, nullptr, nullptr, 0) != hipSuccess)
            P->exec = nullptr;
        if (graph) (void)hipGraphDestroy(graph);
    }
    (void)hipGetLastError();
    return FDTD_OK;
}

constexpr size_t kPlansKept = 4;

// The plan of this call from the lead's cache, built if missing.
int find_plan(fdtd_grid* const* gs, int ng, const int64_t* n, BatchPlan** out)
{
    fdtd_grid* lead = gs[0];
    std::vector<uint64_t> key;
    key.reserve(2 * (size_t)ng + 3);
    key.push_back((uint64_t)lead->tile_x);
    key.push_back((uint64_t)lead->tile_y);
    key.push_back((uint64_t)lead->tile_steps);
    for (int h = 0; h < ng; ++h) {
        key.push_back(gs[h]->serial);
        key.push_back((uint64_t)n[h]);
    }
    ++lead->plan_clock;
    // free the retired plans whose last launch has finished
    for (size_t q = 0; q < lead->retired.size();) {
        if (hipEventQuery(lead->retired[q]->done) == hipSuccess) {
            free_plan(lead, lead->retired[q]);
            lead->retired.erase(lead->retired.begin() + (std::ptrdiff_t)q);
        } else {
            ++q;
        }
    }
    (void)hipGetLastError();   // hipErrorNotReady from the queries
    for (BatchPlan* p : lead->plans)
        if (p->key == key) {
            p->used = lead->plan_clock;
            *out = p;
            return FDTD_OK;
        }
    if (lead->plans.size() >= kPlansKept) {
        auto lru = std::min_element(lead->plans.begin(), lead->plans.end(),
                                    [](const BatchPlan* a, const BatchPlan* b) { return a->used < b->used; });
        // the evicted plan's last launch may still run: it is freed later
        lead->retired.push_back(*lru);
        lead->plans.erase(lru);
    }
    BatchPlan* p = new (std::nothrow) BatchPlan();
    if (!p) return fail(FDTD_ENOMEM, "host allocation failed");
    p->key = std::move(key);
    p->used = lead->plan_clock;
    if (int e = build_plan(gs, ng, n, p)) {
        free_plan(lead, p);
        return e;
    }
    lead->plans.push_back(p);
    *out = p;
    return FDTD_OK;
}

}  // namespace

int fdtd_step_many(fdtd_grid* const* gs, int ng, const int64_t* n)
{
    if (!gs || !n || ng < 1) return fail(FDTD_EINVAL, "need at least one handle and step counts");
    for (int h = 0; h < ng; ++h) {
        if (!gs[h]) return fail(FDTD_EINVAL, "null handle %d", h);
        if (n[h] < 0) return fail(FDTD_EINVAL, "negative step count for handle %d", h);
        for (int o = 0; o < h; ++o)
            if (gs[o] == gs[h]) return fail(FDTD_EINVAL, "handle %d appears twice", h);
        if (gs[h]->device != gs[0]->device) return fail(FDTD_EINVAL, "handles on different devices");
        if (gs[h]->step + n[h] > gs[h]->d.max_steps)
            return fail(FDTD_ESTATE, "handle %d: steps would exceed max_steps", h);
    }
    for (int h = 0; h < ng; ++h)
        if (int e = finalize(gs[h])) return e;
    // boards whose every step runs the node passes (past the tiled kernels'
    // offset window, or a one-step shape set) step alone on their own streams;
    // the rest, material boards included, share the batched launches
    std::vector<fdtd_grid*> fused;
    std::vector<int64_t> nfused;
    for (int h = 0; h < ng; ++h) {
        if (gs[h]->node_pass && !gs[h]->mat) {
            if (int e = fdtd_step_n(gs[h], n[h])) return e;
        } else {
            fused.push_back(gs[h]);
            nfused.push_back(n[h]);
        }
    }
    if (fused.size() < (size_t)ng) {
        if (fused.empty()) return FDTD_OK;
        return fdtd_step_many(fused.data(), (int)fused.size(), nfused.data());
    }
    bool any = false;
    for (int h = 0; h < ng; ++h) any |= n[h] > 0;
    if (!any) return FDTD_OK;
    fdtd_grid* lead = gs[0];
    hipStream_t st = lead->stream;
    BatchPlan* P = nullptr;
    if (int e = find_plan(gs, ng, n, &P)) return e;
    // order after the work already queued on every handle's stream
    for (int h = 1; h < ng; ++h) {
        if (gs[h]->stream == st) continue;
        if (int e = ensure_event(gs[h])) return e;
        HIP_OR_FAIL(hipEventRecord(gs[h]->sync_ev, gs[h]->stream));
        HIP_OR_FAIL(hipStreamWaitEvent(st, gs[h]->sync_ev, 0));
    }
    if (P->exec)
        HIP_OR_FAIL(hipGraphLaunch(P->exec, st));
    else if (int e = enqueue_plan(gs, ng, *P, st))
        return e;
    HIP_OR_FAIL(hipEventRecord(P->done, st));
    for (int h = 0; h < ng; ++h) {
        fdtd_grid* g = gs[h];
        g->step += n[h];
        g->buf = (int)((g->buf + P->flips[h]) & 1);
    }
    // later work on every handle's own stream orders after the batch
    if (int e = ensure_event(lead)) return e;
    HIP_OR_FAIL(hipEventRecord(lead->sync_ev, st));
    for (int h = 1; h < ng; ++h)
        if (gs[h]->stream != st) HIP_OR_FAIL(hipStreamWaitEvent(gs[h]->stream, lead->sync_ev, 0));
    return FDTD_OK;
}

int64_t fdtd_estimate_bytes(const fdtd_grid_desc* d, int n_sources, int n_probes, int n_freqs)
{
    if (!d || d->nx < 2 || d->ny < 2 || d->nz < 2 || d->max_steps < 1 || n_sources < 0 ||
        n_probes < 0 || n_freqs < 0)
        return fail(FDTD_EINVAL, "bad descriptor or counts");
    auto r = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int64_t nodes = row_pitch(d->nx) * (d->ny + 1) * (d->nz + 1);      // padded rows
    int64_t t = 8 * r(3 * component_stride(nodes));                             // fields
    t += r(2 * (nodes + kGuard));                                               // class map (upper bound)
    t += r(65535 * (int64_t)sizeof(ClassEntry));                                // class table (upper bound)
    t += r(65535 * 6 * 4);                                                      // node-pass class data (upper bound)
    t += r((int64_t)kNumCoef * 2 * (d->nx + 1) * 4) + r((int64_t)kNumCoef * 2 * (d->ny + 1) * 4) +
         r((int64_t)kNumCoef * 2 * (d->nz + 1) * 4);                            // coefficients
    t += 2 * r(4 * (int64_t)n_sources) + r(4 * (int64_t)n_sources * d->max_steps);   // sources
    t += r(4 * (int64_t)n_probes) + r(4 * (int64_t)n_probes * d->max_steps);     // probes
    t += r(8 * (int64_t)n_freqs) + 2 * r(8 * (int64_t)n_probes * n_freqs);       // DFT
    const int64_t max_tiles = ((d->nx + 64) / 64) * ((d->ny + 3) / 3);         // 64 x 4, the most tiles
    const int64_t max_items = 2 * kXcds * (max_tiles + 7 * 256);                // two lists, pieces, padding
    t += 8 * 256 + r(sizeof(BoardDev)) + r(sizeof(TileRef) * max_items);        // small buffers
    return t;
}

int fdtd_synchronize(fdtd_grid* g)
{
    if (int e = check_grid(g)) return e;
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    return check_bad(g);
}

int fdtd_get_stream(fdtd_grid* g, void** out)
{
    if (int e = check_grid(g)) return e;
    if (!out) return fail(FDTD_EINVAL, "null output");
    *out = (void*)g->stream;
    return FDTD_OK;
}

int fdtd_get_probe(fdtd_grid* g, int id, float* out, int64_t n)
{
    if (int e = check_grid(g)) return e;
    if (id < 0 || id >= (int)g->probes.size()) return fail(FDTD_EINVAL, "no probe %d", id);
    if (n < 0 || n > g->step || (!out && n > 0)) return fail(FDTD_EINVAL, "bad sample count %lld", (long long)n);
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    if (n > 0)
        HIP_OR_FAIL(copy_sync(g, out, g->prb_series + (size_t)id * g->d.max_steps, (size_t)n * 4,
                              hipMemcpyDeviceToHost));
    return check_bad(g);
}

int fdtd_get_voltage(fdtd_grid* g, int id, double* out, int64_t n)
{
    if (int e = check_grid(g)) return e;
    if (id < 0 || id >= (int)g->vprobes.size()) return fail(FDTD_EINVAL, "no voltage probe %d", id);
    if (n < 0 || n > g->step || (!out && n > 0)) return fail(FDTD_EINVAL, "bad sample count %lld", (long long)n);
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    if (n == 0) return check_bad(g);
    const VoltageProbeH& v = g->vprobes[id];
    std::vector<float> ez((size_t)v.count * n);
    for (int q = 0; q < v.count; ++q)
        HIP_OR_FAIL(copy_sync(g, ez.data() + (size_t)q * n,
                              g->prb_series + (size_t)(v.first + q) * g->d.max_steps,
                              (size_t)n * 4, hipMemcpyDeviceToHost));
    // V = -sum_k Ez(k+1/2) dz, summed upwards in z
    for (int64_t s = 0; s < n; ++s) {
        double acc = 0.0;
        for (int q = 0; q < v.count; ++q) acc += (double)ez[(size_t)q * n + s];
        out[s] = -g->d.dz * acc;
    }
    return check_bad(g);
}

int fdtd_get_dft(fdtd_grid* g, int id, double* re, double* im)
{
    if (int e = check_grid(g)) return e;
    if (id < 0 || id >= (int)g->probes.size()) return fail(FDTD_EINVAL, "no probe %d", id);
    if (g->freqs.empty()) return fail(FDTD_ESTATE, "no DFT frequencies were set");
    if (!re || !im) return fail(FDTD_EINVAL, "null output");
    const int nf = (int)g->freqs.size();
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    if (!g->finalized) {
        std::fill(re, re + nf, 0.0);
        std::fill(im, im + nf, 0.0);
        return FDTD_OK;
    }
    HIP_OR_FAIL(copy_sync(g, re, g->dft_re + (size_t)id * nf, nf * 8, hipMemcpyDeviceToHost));
    HIP_OR_FAIL(copy_sync(g, im, g->dft_im + (size_t)id * nf, nf * 8, hipMemcpyDeviceToHost));
    return check_bad(g);
}

int fdtd_get_plane_dft(fdtd_grid* g, double* re, double* im)
{
    if (int e = check_grid(g)) return e;
    if (g->plane_k < 0) return fail(FDTD_ESTATE, "no plane DFT was set");
    if (!re || !im) return fail(FDTD_EINVAL, "null output");
    const int nf = (int)g->plane_freqs.size();
    const size_t row = (size_t)(g->d.nx + 1) * 8, prow = (size_t)g->pitch * 8;
    const size_t rows = (size_t)nf * (g->d.ny + 1);
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    if (!g->finalized) {
        std::fill(re, re + rows * (g->d.nx + 1), 0.0);
        std::fill(im, im + rows * (g->d.nx + 1), 0.0);
        return FDTD_OK;
    }
    HIP_OR_FAIL(hipMemcpy2DAsync(re, row, g->plane_re, prow, row, rows, hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(hipMemcpy2DAsync(im, row, g->plane_im, prow, row, rows, hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    return check_bad(g);
}

int fdtd_probe_fft(fdtd_grid* g, int id, int n_fft, double* re, double* im)
{
    if (int e = check_grid(g)) return e;
    if (id < 0 || id >= (int)g->probes.size()) return fail(FDTD_EINVAL, "no probe %d", id);
    if (n_fft < 2 || (n_fft & (n_fft - 1)) || n_fft > (1 << 26) || n_fft < g->step)
        return fail(FDTD_EINVAL, "n_fft %d must be a power of two >= the step count %lld", n_fft,
                    (long long)g->step);
    if (!re || !im) return fail(FDTD_EINVAL, "null output");
    if (int e = finalize(g)) return e;
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    double2* a = (double2*)temp_alloc(g, (size_t)n_fft * sizeof(double2));
    double2* b = (double2*)temp_alloc(g, (size_t)n_fft * sizeof(double2));
    if (!a || !b) {
        temp_free(g, a);
        temp_free(g, b);
        return fail(FDTD_ENOMEM, "FFT scratch allocation failed");
    }
    double2* res = nullptr;
    hipError_t e = launch_fft(g->prb_series + (size_t)id * g->d.max_steps, g->step, n_fft, a, b,
                              &res, g->stream);
    std::vector<double2> h((size_t)n_fft / 2 + 1);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess)
        e = copy_sync(g, h.data(), res, h.size() * sizeof(double2), hipMemcpyDeviceToHost);
    temp_free(g, a);
    temp_free(g, b);
    if (e != hipSuccess) return fail(FDTD_EDEVICE, "probe FFT failed: %s", hipGetErrorString(e));
    for (size_t k = 0; k < h.size(); ++k) {
        re[k] = h[k].x;
        im[k] = h[k].y;
    }
    return check_bad(g);
}

int fdtd_probe_fft_noalloc(fdtd_grid* g, int id, int n_fft, double* re, double* im)
{
    if (int e = check_grid(g)) return e;
    if (id < 0 || id >= (int)g->probes.size()) return fail(FDTD_EINVAL, "no probe %d", id);
    if (n_fft < 2 || (n_fft & (n_fft - 1)) || n_fft < g->step)
        return fail(FDTD_EINVAL, "n_fft %d must be a power of two >= the step count %lld", n_fft,
                    (long long)g->step);
    if (n_fft > kNoAllocFftMax)
        return fail(FDTD_EINVAL,
                    "n_fft %d exceeds the allocation-free maximum %d (use fdtd_probe_fft)", n_fft,
                    kNoAllocFftMax);
    if (!re || !im) return fail(FDTD_EINVAL, "null output");
    const int nbins = n_fft / 2 + 1;
    if (!g->finalized) {
        // nothing stepped yet (set-up, which allocates, has not run): no samples
        std::fill(re, re + nbins, 0.0);
        std::fill(im, im + nbins, 0.0);
        return FDTD_OK;
    }
    void* s = nullptr;
    HIP_OR_FAIL(noalloc_scratch(g->device, &s));
    double2* a = (double2*)s;
    double2* b = a + kNoAllocFftMax;
    double2* res = nullptr;
    HIP_OR_FAIL(launch_fft(g->prb_series + (size_t)id * g->d.max_steps, g->step, n_fft, a, b,
                           &res, g->stream));
    // the buffer the last pass did not write holds the split bins
    double* split = (double*)(res == a ? b : a);
    HIP_OR_FAIL(launch_fft_split(res, nbins, split, g->stream));
    HIP_OR_FAIL(hipMemcpyAsync(re, split, (size_t)nbins * 8, hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(hipMemcpyAsync(im, split + nbins, (size_t)nbins * 8, hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    return check_bad(g);
}

static double field_scale(int comp)
{
    switch (comp) {
        case FDTD_HX: case FDTD_HY: case FDTD_HZ: return 1.0 / kEta0;  // Hs = eta0 H
        case FDTD_DX: case FDTD_DY: case FDTD_DZ: return kEps0;        // Ds = D / eps0
        case FDTD_BX: case FDTD_BY: case FDTD_BZ: return 1.0 / kC0;    // Bs = c0 B
        default: return 1.0;
    }
}

static float* comp_ptr(fdtd_grid* g, int comp)
{
    const int par = g->buf;
    if (comp <= FDTD_HZ) return g->f[par][comp];
    if (comp <= FDTD_DZ) return g->dd[g->buf][comp - FDTD_DX];
    return g->f[par][6 + comp - FDTD_BX];
}

int fdtd_get_field(fdtd_grid* g, int comp, float* out)
{
    if (int e = check_grid(g)) return e;
    if (comp < 0 || comp > FDTD_BZ || !out) return fail(FDTD_EINVAL, "bad component or output");
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    const double s = field_scale(comp);
    if (s == 1.0) {
        HIP_OR_FAIL(copy_field_sync(g, out, comp_ptr(g, comp), hipMemcpyDeviceToHost));
        return FDTD_OK;
    }
    std::vector<float> h((size_t)g->nodes);
    HIP_OR_FAIL(copy_field_sync(g, h.data(), comp_ptr(g, comp), hipMemcpyDeviceToHost));
    for (size_t t = 0; t < h.size(); ++t) out[t] = (float)((double)h[t] * s);
    return FDTD_OK;
}

int fdtd_get_plane(fdtd_grid* g, int comp, int k, float* out)
{
    if (int e = check_grid(g)) return e;
    if (comp < 0 || comp > FDTD_BZ || !out) return fail(FDTD_EINVAL, "bad component or output");
    if (k < 0 || k > g->d.nz) return fail(FDTD_EINVAL, "plane %d is outside 0..nz", k);
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    const size_t row = (size_t)(g->d.nx + 1) * 4, prow = (size_t)g->pitch * 4;
    const float* src = comp_ptr(g, comp) + (size_t)k * g->pitch * (g->d.ny + 1);
    HIP_OR_FAIL(hipMemcpy2DAsync(out, row, src, prow, row, (size_t)g->d.ny + 1,
                                 hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    const double sc = field_scale(comp);
    const size_t nn = (size_t)(g->d.nx + 1) * (g->d.ny + 1);
    if (sc != 1.0)
        for (size_t t = 0; t < nn; ++t) out[t] = (float)((double)out[t] * sc);
    return check_bad(g);
}

int fdtd_set_field(fdtd_grid* g, int comp, const float* in)
{
    if (int e = check_grid(g)) return e;
    if (comp < 0 || comp > FDTD_BZ || !in) return fail(FDTD_EINVAL, "bad component or input");
    const fdtd_grid_desc& d = g->d;
    const double s = 1.0 / field_scale(comp);
    std::vector<float> h((size_t)g->nodes);
    // State entries only: an E edge exists for index < n along its own axis and
    // is tangential to the wall (held at zero) at 0 or n along the others; an H
    // face exists for index < n along the other two axes and, on the wall normal
    // to it (0 or n along its own axis), touches only such E edges, so it
    // carries nothing either.  Auxiliaries exist only where their PML predicate
    // holds (the component's own or cyclic-next axis in a PML slab).
    const int axis = comp >= FDTD_DX ? (comp - FDTD_DX) % 3 : -1;
    const bool e_like = comp <= FDTD_EZ || (comp >= FDTD_DX && comp <= FDTD_DZ);
    const int u = comp % 3;
    const int n3[3] = {d.nx, d.ny, d.nz};
    std::vector<uint8_t> ok[3], pml[3];
    for (int a = 0; a < 3; ++a) {
        const int n = n3[a], lo = d.npml[2 * a], hi = d.npml[2 * a + 1];
        const bool own = a == u;
        ok[a].resize((size_t)n + 1);
        pml[a].resize((size_t)n + 1);
        for (int q = 0; q <= n; ++q) {
            ok[a][q] = (e_like ? own : !own) ? q < n : (q > 0 && q < n);
            pml[a][q] = q < lo || (hi > 0 && q >= n - hi);
        }
    }
    // the aux predicate: axis 0 (x or y PML), 1 (y or z), 2 (z or x)
    const int pa = axis < 0 ? 0 : axis, pb = axis < 0 ? 0 : (axis + 1) % 3;
    const size_t row = (size_t)d.nx + 1;
    for (int k = 0; k <= d.nz; ++k)
        for (int j = 0; j <= d.ny; ++j) {
            const int64_t base = node_index(g, 0, j, k);
            const bool rok = ok[1][j] && ok[2][k];
            const int qj[3] = {0, j, k};
            for (size_t i = 0; i < row; ++i) {
                bool keep = rok && ok[0][i];
                if (keep && axis >= 0) {
                    const bool ia = pa == 0 ? pml[0][i] : pml[pa][qj[pa]];
                    const bool ib = pb == 0 ? pml[0][i] : pml[pb][qj[pb]];
                    keep = ia || ib;
                }
                h[(size_t)base + i] = keep ? (float)((double)in[base + i] * s) : 0.0f;
            }
        }
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    HIP_OR_FAIL(copy_field_sync(g, comp_ptr(g, comp), h.data(), hipMemcpyHostToDevice));
    return FDTD_OK;
}

// checkpoint header: magic, nx, ny, nz, step, probes, probe frequencies,
// max_steps, plane-DFT plane, plane frequencies
constexpr int kStateHeader = 80;

int64_t fdtd_state_bytes(fdtd_grid* g)
{
    if (!g) return fail(FDTD_EINVAL, "null grid handle");
    const int64_t np = (int64_t)g->probes.size(), nf = (int64_t)g->freqs.size();
    const int64_t pf = g->plane_k >= 0 ? (int64_t)g->plane_freqs.size() : 0;
    return kStateHeader + 12 * g->nodes * 4 + np * g->d.max_steps * 4 + (np && nf ? np * nf * 16 : 0) +
           pf * (g->d.nx + 1) * (g->d.ny + 1) * 16;
}

int fdtd_save_state(fdtd_grid* g, void* host_buf, int64_t bytes)
{
    if (int e = check_grid(g)) return e;
    if (!host_buf || bytes < fdtd_state_bytes(g)) return fail(FDTD_EINVAL, "buffer too small");
    if (int e = finalize(g)) return e;
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    char* p = (char*)host_buf;
    int64_t hdr[kStateHeader / 8] = {0x4644544453544154ll, g->d.nx, g->d.ny, g->d.nz, g->step,
                                     (int64_t)g->probes.size(), (int64_t)g->freqs.size(),
                                     g->d.max_steps, g->plane_k, (int64_t)g->plane_freqs.size()};
    memcpy(p, hdr, kStateHeader);
    p += kStateHeader;
    for (int c = 0; c < 12; ++c) {
        HIP_OR_FAIL(copy_field_sync(g, p, comp_ptr(g, c), hipMemcpyDeviceToHost));
        p += g->nodes * 4;
    }
    const int64_t np = (int64_t)g->probes.size(), nf = (int64_t)g->freqs.size();
    if (np) {
        HIP_OR_FAIL(copy_sync(g, p, g->prb_series, np * g->d.max_steps * 4, hipMemcpyDeviceToHost));
        p += np * g->d.max_steps * 4;
    }
    if (np && nf) {
        HIP_OR_FAIL(copy_sync(g, p, g->dft_re, np * nf * 8, hipMemcpyDeviceToHost));
        p += np * nf * 8;
        HIP_OR_FAIL(copy_sync(g, p, g->dft_im, np * nf * 8, hipMemcpyDeviceToHost));
        p += np * nf * 8;
    }
    if (g->plane_k >= 0) {
        // the ring is always folded when a call returns: the accumulators are the state
        const int64_t pn = (int64_t)g->plane_freqs.size() * (g->d.nx + 1) * (g->d.ny + 1);
        if (int e = fdtd_get_plane_dft(g, (double*)p, (double*)p + pn)) return e;
    }
    return FDTD_OK;
}

int fdtd_load_state(fdtd_grid* g, const void* host_buf, int64_t bytes)
{
    if (int e = check_grid(g)) return e;
    if (!host_buf || bytes < fdtd_state_bytes(g)) return fail(FDTD_EINVAL, "buffer too small");
    if (int e = finalize(g)) return e;
    const char* p = (const char*)host_buf;
    int64_t hdr[kStateHeader / 8];
    memcpy(hdr, p, kStateHeader);
    p += kStateHeader;
    if (hdr[0] != 0x4644544453544154ll || hdr[1] != g->d.nx || hdr[2] != g->d.ny ||
        hdr[3] != g->d.nz || hdr[5] != (int64_t)g->probes.size() ||
        hdr[6] != (int64_t)g->freqs.size() || hdr[7] != g->d.max_steps ||
        hdr[8] != g->plane_k || hdr[9] != (int64_t)g->plane_freqs.size())
        return fail(FDTD_EINVAL, "state image does not match this grid");
    if (hdr[4] < 0 || hdr[4] > g->d.max_steps) return fail(FDTD_EINVAL, "bad step in state image");
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    g->step = hdr[4];
    for (int c = 0; c < 12; ++c) {
        HIP_OR_FAIL(copy_field_sync(g, comp_ptr(g, c), p, hipMemcpyHostToDevice));
        p += g->nodes * 4;
    }
    const int64_t np = (int64_t)g->probes.size(), nf = (int64_t)g->freqs.size();
    if (np) {
        HIP_OR_FAIL(copy_sync(g, g->prb_series, p, np * g->d.max_steps * 4, hipMemcpyHostToDevice));
        p += np * g->d.max_steps * 4;
    }
    if (np && nf) {
        HIP_OR_FAIL(copy_sync(g, g->dft_re, p, np * nf * 8, hipMemcpyHostToDevice));
        p += np * nf * 8;
        HIP_OR_FAIL(copy_sync(g, g->dft_im, p, np * nf * 8, hipMemcpyHostToDevice));
        p += np * nf * 8;
    }
    if (g->plane_k >= 0) {
        const size_t row = (size_t)(g->d.nx + 1) * 8, prow = (size_t)g->pitch * 8;
        const size_t rows = g->plane_freqs.size() * (size_t)(g->d.ny + 1);
        HIP_OR_FAIL(hipMemcpy2DAsync(g->plane_re, prow, p, row, row, rows, hipMemcpyHostToDevice, g->stream));
        p += rows * row;
        HIP_OR_FAIL(hipMemcpy2DAsync(g->plane_im, prow, p, row, row, rows, hipMemcpyHostToDevice, g->stream));
        HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    }
    HIP_OR_FAIL(copy_sync(g, g->step_dev, &g->step, 8, hipMemcpyHostToDevice));
    const int32_t zero = 0;
    HIP_OR_FAIL(copy_sync(g, g->bad_dev, &zero, 4, hipMemcpyHostToDevice));
    return FDTD_OK;
}

int fdtd_get_info(fdtd_grid* g, fdtd_info* out)
{
    if (int e = check_grid(g)) return e;
    if (!out) return fail(FDTD_EINVAL, "null output");
    out->dt = g->dt;
    out->step = g->step;
    out->max_steps = g->d.max_steps;
    out->cells = (int64_t)g->d.nx * g->d.ny * g->d.nz;
    out->nodes = g->nodes;
    out->step_bytes = g->finalized ? g->step_bytes : count_step_bytes(g);
    out->device_bytes = g->device_bytes;
    out->n_sources = (int32_t)g->sources.size();
    out->n_probes = (int32_t)g->probes.size();
    out->n_freqs = (int32_t)g->freqs.size();
    out->n_classes = g->n_classes;
    out->tile_x = g->tile_x;
    out->tile_y = g->tile_y;
    out->tile_steps = g->tile_steps;
    out->plane_k = g->plane_k;
    out->plane_nf = (int32_t)g->plane_freqs.size();
    out->node_passes = g->node_pass ? 1 : 0;
    out->material_two_step = g->mat ? 1 : 0;
    out->material_permille = g->mat ? g->mat_permille : 0;
    out->material_split = g->mat ? g->mat_split : 0;
    out->conduct_permille = g->mat ? g->cond_permille : 0;
    out->batch_plans = (int32_t)g->plans.size();
    out->batch_graphs = 0;
    for (const BatchPlan* p : g->plans) out->batch_graphs += p->exec != nullptr;
    return FDTD_OK;
}

int fdtd_set_timing(fdtd_grid* g, int on)
{
    if (int e = check_grid(g)) return e;
    g->timing = on != 0;
    return FDTD_OK;
}

int fdtd_get_timing(fdtd_grid* g, double* ms, int64_t* launches)
{
    if (int e = check_grid(g)) return e;
    if (!ms || !launches) return fail(FDTD_EINVAL, "null output");
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    double total = 0.0;
    for (size_t t = 0; t + 1 < g->ev_used; t += 2) {
        float v = 0.f;
        HIP_OR_FAIL(hipEventElapsedTime(&v, g->ev_pool[t], g->ev_pool[t + 1]));
        total += v;
    }
    *ms = total;
    *launches = g->timed_launches;
    g->ev_used = 0;
    g->timed_launches = 0;
    return FDTD_OK;
}

int fdtd_destroy_grid(fdtd_grid* g)
{
    if (!g) return FDTD_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (hipEvent_t e : g->ev_pool) (void)hipEventDestroy(e);
    if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
    if (g->sync_ev) (void)hipEventDestroy(g->sync_ev);
    for (BatchPlan* p : g->plans) free_plan(g, p);
    for (BatchPlan* p : g->retired) free_plan(g, p);
    g->plans.clear();
    g->retired.clear();
    if (g->aux_stream) (void)hipStreamSynchronize(g->aux_stream);
    dev_free_all(g);
    if (g->fork_ev) (void)hipEventDestroy(g->fork_ev);
    if (g->join_ev) (void)hipEventDestroy(g->join_ev);
    if (g->aux_stream) (void)hipStreamDestroy(g->aux_stream);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
    return FDTD_OK;
}

}  // extern "C"
