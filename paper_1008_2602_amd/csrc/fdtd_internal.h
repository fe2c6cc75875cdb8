// Internal layout shared by the libfdtd host code and its gfx950 kernels.
//
// Units inside the library.  E keeps SI units (V/m).  The other state is scaled
// to V/m so that every update coefficient is O(1) in FP32:
//   Hs = eta0 H,  Bs = c0 B,  Ds = D / eps0.
// With crd_w = c0 dt / delta_w, the Eq. 4 two-step update (D then E; B then H
// with the same stretch factors, Eq. 1) becomes, for a component u with cyclic
// partners (v, w) and q = sigma dt / eps0, ph = kappa + q/2, rp = 1/ph,
// ca = (kappa - q/2)/(kappa + q/2), cam1 = ca - 1 = -q/(kappa + q/2):
//   dDs   = cam1_v Ds + rp_v (curl_u(Hs) - Js)          Ds += dDs
//   E_u'  = ca_w E_u + rp_w inv_eps_r (ph_u dDs + q_u Ds)
//   dBs   = cam1_v Bs - rp_v curl_u(E)                  Bs += dBs
//   Hs_u' = ca_w Hs_u + rp_w (ph_u dBs + q_u Bs)
// where curl terms are differences times crd and Js = c0 dt eta0 J.  The form
// p+ dD + (p+ - p-) D^n replaces p+ D^{n+1} - p- D^n: algebraically equal, and
// outside the u-axis PML (q_u = 0) it never subtracts two large numbers.
#pragma once
#include <stdint.h>

namespace fdtd {

constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kEps0 = 1.0 / (kMu0 * kC0 * kC0);
constexpr double kEta0 = kMu0 * kC0;

// steps per replayable graph in fdtd_step_n
constexpr int kGraphChunk = 32;

// slots of the plane-DFT sample ring (one plane of Ez per step); folded into the
// accumulators at least every kPlaneRing steps
constexpr int kPlaneRing = 32;
static_assert(kGraphChunk == kPlaneRing, "a graph chunk fills the ring exactly once");

// largest transform of the allocation-free probe spectrum: its two FP64 complex
// ping-pong buffers (32 B per point, 32 MiB) sit in a fixed device array
constexpr int kNoAllocFftMax = 1 << 20;

// tile rows of the two-step kernel's material variant (64 x kMatTY x 2), and of
// the plain two-step pieces that step a material board's planes clear of
// material nodes (64 x kHybridTY x 2)
constexpr int kMatTY = 10;
constexpr int kHybridTY = 14;

// zero words allocated past the last node of every field array
constexpr int64_t kGuard = 64;

// per-axis coefficient table: 6 quantities x {node, half node} x (n+1) entries
// (kappa is read only by the material kernels, which rebuild the others from
// it; on a material board the table's others are those rebuilt values at
// 1/eps_rw = 1, in FP32, so that reading them gives the same bits)
enum CoefKind { kCam1 = 0, kCa = 1, kRp = 2, kPh = 3, kQ = 4, kKappa = 5, kNumCoef = 6 };

// class flags (per node): which E components are stepped, and source/probe marks
// (kPlnEz: the node lies on the plane-DFT plane, its Ez goes to the sample ring).
// On a material board: kMatH, some H face has 1/eps_rw != 1 (its PML
// coefficients are rebuilt); kMatE, the same for a stepped E edge (eps_rw on);
// kCondE, some E edge conducts (lossy cell, resistive sheet).
enum : uint32_t {
    kUpdEx = 1u, kUpdEy = 2u, kUpdEz = 4u, kSrcEz = 8u, kPrbEz = 16u, kPlnEz = 32u,
    kMatH = 64u, kMatE = 128u, kCondE = 256u
};

struct ClassEntry {
    float inv_x, inv_y, inv_z;  // 1/eps_r of the Ex, Ey, Ez edges owned by the node
    uint32_t flags;
};

// Everything one field launch needs about one board.  Lives in device memory
// (an array of these for batched launches).
struct BoardDev {
    // state: [buffer][0..8] = Ex Ey Ez Hx Hy Hz Bx By Bz and [buffer][0..2] =
    // Dx Dy Dz.  Every launch reads one buffer and writes the other (one or two
    // steps per launch), so a block may read any neighbour's fields as they were
    float* f[2][9];
    float* d[2][3];
    const void* cls;             // uint8_t or uint16_t per node
    const ClassEntry* ctab;
    // node passes (eps_rw, lossy dielectric), 6 floats per class: 1/eps_r at the
    // Hx, Hy, Hz faces, then the conduction coefficient sigma_c dt / (2 eps0) of
    // the Ex, Ey, Ez edges
    const float* node_aux;
    const float* coef[3];        // per axis: [kind][node/half][n+1]
    const int32_t* src_node;     // node index of each source's Ez edge
    const float* src_j;          // [nsrc][max_steps] Js samples
    const float* src_beta;       // [nsrc] 0, or a resistive source's beta (lumped conductance)
    const int32_t* prb_node;
    float* prb_series;           // [nprb][max_steps]
    int64_t* step;               // [0] completed steps, [1] buffer (0/1) holding the fields
    int32_t* bad;                // watchdog flag
    int32_t nx, ny, nz;
    int32_t pitch;               // row pitch in nodes: nx+1 rounded up to 32 (128 bytes)
    uint32_t cstride;            // bytes from a field's x array to its y array (y to z alike)
    int32_t nsrc, nprb;
    int32_t nclass;
    int32_t pml[6];
    int64_t max_steps;
    float crd_x, crd_y, crd_z;
    int32_t tiles_x, tiles_y;
    // added to a launch's step and buffer offsets (nonzero only in the one-step
    // tail launch of a batch, whose boards have done different numbers of pairs)
    int32_t rel0, flip0;
    // plane DFT: Ez of the nodes flagged kPlnEz goes to slot (step mod kPlaneRing)
    // of the ring, each slot one node plane of the field layout
    float* plane_ring;
    // node passes: 1 when Eq. 2's eps_rw scales the PML sigma (else eps_rw = 1)
    int32_t eps_rw;
    // node passes: the bytes between a field's x, y and z arrays in 64 bits (the
    // 32-bit cstride does not hold them on boards past the 4 GiB window), and
    // the source and probe nodes as 64-bit indices
    uint64_t cstride64;
    const int64_t* src_node64;
    const int64_t* prb_node64;
};

// One work item of the field kernel: tile (tx, ty) of a board, planes kb..ke-1.
// board < 0 marks an idle entry that pads an XCD's share of the launch.
struct TileRef {
    int32_t board;
    int32_t tx, ty;
    int32_t kb, ke;
};

}  // namespace fdtd
