/*
 * libfdtd: MI355X (gfx950) Yee/UPML leapfrog for PCB power/ground-plane stacks.
 *
 * The method is the one of "A Time Domain Approach to Power Integrity for Printed
 * Circuit Boards" (Mattey, Edwards, Hood): Maxwell's curl equations on a Yee
 * grid (Model section, Fig. 2), terminated by a uniaxial PML whose auxiliary D
 * and B fields are stepped in a two-step D->E / B->H process (Eqs. 1-4) with a
 * polynomially graded loss (Eq. 5) and an outer PEC wall, a time step bounded by
 * the CFL limit (Eq. 7), PEC power/ground planes that zero tangential Ex/Ey
 * (Model section), a current source (Results section, Eq. 8) and the FFT of a
 * probe's Ez (Results section, Fig. 5 / Table 1).
 *
 * Conventions for every call:
 *   - Grid: nx, ny, nz cells including air and PML; nodes run 0..n on each axis.
 *     Field arrays exchanged with the caller have (nz+1)*(ny+1)*(nx+1) entries,
 *     x fastest: index = i + (nx+1)*(j + (ny+1)*k).  Ex(i,j,k) is Ex at
 *     (i+1/2, j, k); Ey at (i, j+1/2, k); Ez at (i, j, k+1/2); Hx at
 *     (i, j+1/2, k+1/2); Hy at (i+1/2, j, k+1/2); Hz at (i+1/2, j+1/2, k).
 *   - Pointers marked "host" are host memory, read (or written) during the call
 *     only; the caller keeps ownership.  Device memory is owned by the handle.
 *   - Return value: 0 (FDTD_OK) or a negative FDTD_E* code; the message of the
 *     last failure on the calling thread is in fdtd_last_error().  No call
 *     throws.  A handle is not thread safe; distinct handles are independent.
 *   - Stepping is asynchronous on the handle's HIP stream; every call that
 *     returns data to the host synchronises that stream first.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDTD_OK 0
#define FDTD_EINVAL (-1)    /* null / out-of-range argument, dt above the CFL limit, ... */
#define FDTD_ESTATE (-2)    /* call not allowed in the handle's current state */
#define FDTD_ENOMEM (-3)    /* device or host allocation failed (nothing leaked) */
#define FDTD_EDEVICE (-4)   /* a HIP runtime call failed */
#define FDTD_EUNSTABLE (-5) /* non-finite field value found by the watchdog */

#define FDTD_WAVE_GAUSS 0   /* J0 exp(-(t-t0)^2 / (2 sigma^2)) */
#define FDTD_WAVE_DGAUSS 1  /* J0 ((t-t0)/tau) exp(-((t-t0)/tau)^2): Eq. 8 read as a pulse */

/* field component ids for fdtd_get_field / fdtd_set_field */
enum {
    FDTD_EX = 0, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ,
    FDTD_DX, FDTD_DY, FDTD_DZ, FDTD_BX, FDTD_BY, FDTD_BZ
};

typedef struct fdtd_grid fdtd_grid;

/* Optional device allocator (e.g. PyTorch's caching allocator).  alloc returns a
 * device pointer of at least `bytes` bytes aligned to 256 B, or NULL; free
 * releases it.  Both are called only from fdtd_create_grid/fdtd_set_dft_freqs
 * and fdtd_destroy_grid. */
typedef void* (*fdtd_alloc_fn)(size_t bytes, void* ctx);
typedef void (*fdtd_free_fn)(void* ptr, void* ctx);

typedef struct {
    int32_t nx, ny, nz;          /* cells incl. air and PML; each >= 2 */
    double dx, dy, dz;           /* cell size in metres (anisotropic allowed, Model section) */
    double dt;                   /* seconds; 0 => courant * Eq. 7 limit with c0 */
    double courant;              /* used when dt == 0; in (0, 1) (0 => 0.99) */
    int32_t npml[6];             /* PML depth in cells on -x,+x,-y,+y,-z,+z (0 = bare PEC wall) */
    double pml_m;                /* Eq. 5 grading order (0 => 3) */
    double pml_R;                /* target normal-incidence reflection in (0, 1] (0 => 1e-6) */
    double pml_kappa_max;        /* Eq. 5 kappa_max >= 1 (0 => 1) */
    int64_t max_steps;           /* capacity of the probe series and source tables, >= 1 */
    void* hip_stream;            /* hipStream_t to run on; NULL => the handle creates one */
    fdtd_alloc_fn dev_alloc;     /* NULL => hipMalloc */
    fdtd_free_fn dev_free;       /* NULL => hipFree; must be set iff dev_alloc is */
    void* alloc_ctx;
} fdtd_grid_desc;

typedef struct {
    double dt;                   /* time step in use */
    int64_t step;                /* completed steps */
    int64_t max_steps;
    int64_t cells;               /* nx*ny*nz (the unit of "cell-updates") */
    int64_t nodes;               /* (nx+1)(ny+1)(nz+1) */
    int64_t step_bytes;          /* algorithmic HBM bytes one step of the field kernel must move:
                                    E, H read and written and the class read per cell,
                                    each kept D/B component read and written */
    int64_t device_bytes;        /* device memory held by the handle */
    int32_t n_sources, n_probes, n_freqs;
    int32_t n_classes;           /* distinct per-node material classes after finalisation */
    int32_t tile_x, tile_y;      /* tile shape the field kernel runs with */
    int32_t tile_steps;          /* leapfrog steps per pass of that shape (1 or 2) */
    int32_t plane_k;             /* plane of the plane DFT, -1 if none */
    int32_t plane_nf;            /* its number of frequencies */
    int32_t node_passes;         /* 1: steps run the node passes' arithmetic (fdtd_set_pml_eps_rw,
                                    fdtd_set_conductivity, fdtd_set_sheet_resistance) */
    int32_t material_two_step;   /* 1: of which pairs of steps run on the material two-step kernel */
    int32_t material_permille;   /* of its tiles' node planes, the share (per mille) on the material
                                    variant; the others run the plain two-step kernel */
    int32_t material_split;      /* how: 1 per tile (the variant in the plain kernel's 64 x 14 tiles),
                                    2 per plane (planes near material nodes in any tile run the
                                    64 x 10 variant for every tile), 0 no such planes */
    int32_t conduct_permille;    /* the share (per mille) on the conduction-only flavour of the
                                    variant (planes near conducting edges only, 64 x 14 tiles) */
    int32_t batch_plans;         /* plans of fdtd_step_many calls this handle led, kept for reuse */
    int32_t batch_graphs;        /* of which captured as a graph (one graph launch per call) */
} fdtd_info;

/* Create a grid (Model section: Yee grid with anisotropic spacing, UPML of
 * Eqs. 1-5 with sigma_max = -(m+1) ln R / (2 eta0 N delta) on each face, outer PEC
 * wall; Eq. 7 time step).  All fields start at zero.  EINVAL: sizes < 2, more
 * than about 3.5e8 nodes once rows are padded to 32 nodes (the x, y and z arrays
 * of a field share one 4 GiB window), non-positive spacing, dt at or above the
 * Eq. 7 limit (c0),
 * courant outside (0, 1), npml < 0 or two opposite layers overlapping,
 * max_steps < 1.  ENOMEM: device allocation failed (no handle is returned). */
int fdtd_create_grid(const fdtd_grid_desc* desc, fdtd_grid** out);

/* Materials (Model section, Fig. 1): eps_r_cell (host, nx*ny*nz floats, x fastest,
 * each finite and >= 1) is the relative permittivity of every cell; each E edge
 * takes the mean of the cells that touch it.  pec_edge_mask (host,
 * (nx+1)(ny+1)(nz+1) bytes, NULL = none) marks PEC edges: bit 0 Ex(i+1/2,j,k),
 * bit 1 Ey(i,j+1/2,k), bit 2 Ez(i,j,k+1/2); marked edges stay exactly 0 (the
 * power and ground planes).  ESTATE after the first step.  EINVAL if the
 * material classes exceed 65535. */
int fdtd_set_materials(fdtd_grid* g, const float* eps_r_cell, const uint8_t* pec_edge_mask);

/* Current source Jz (A/m^2) on the edge Ez(i, j, k+1/2), 1 <= i < nx,
 * 1 <= j < ny, 0 <= k < nz, not PEC (Results section: current source through the
 * D update).  waveform FDTD_WAVE_GAUSS or FDTD_WAVE_DGAUSS with width sigma > 0;
 * sampled at the half step (s+1/2) dt.  *id receives the source index.  EINVAL
 * if the edge holds a resistive voltage source; ESTATE after the first step. */
int fdtd_add_source(fdtd_grid* g, int i, int j, int k, int waveform, double J0,
                    double t0, double sigma, int* id);

/* Resistive voltage source on the edge Ez(i, j, k+1/2) (Results section, the
 * Table 1 run: amplitude V0 in volts, source resistance R in ohms, semi-explicit
 * update coefficients): an EMF V_s(t) = V0 * waveform that raises node k+1 over
 * node k, in series with R.  Its branch current density (dz Ebar + V_s)/(R dx dy),
 * with Ebar the mean of Ez at steps n and n+1, enters the Ez update like a
 * current source and the update is solved for Ez^{n+1}; open-circuited the edge
 * holds dz Ez = -V_s, and as R grows it tends to a current source of
 * V0 / (R dx dy).  V_s is sampled at the half step (s+1/2) dt.  Index ranges,
 * waveform and width as fdtd_add_source; *id receives the index in the same
 * source list.  EINVAL if R is not finite and > 0, the edge is PEC, lies in a PML
 * slab (i < npml[0], i >= nx - npml[1], likewise in y, k < npml[4] or
 * k >= nz - npml[5]) or holds another source; ESTATE after the first step. */
int fdtd_add_voltage_source(fdtd_grid* g, int i, int j, int k, int waveform, double V0,
                            double t0, double sigma, double R, int* id);

/* Probe of Ez(i, j, k+1/2), 0 <= i <= nx, 0 <= j <= ny, 0 <= k < nz (Results
 * section: ground-plane Ez recorded every step).  Sample s of the series is Ez at
 * time (s+1) dt, stored in FP32.  *id receives the probe index.  ESTATE after the
 * first step. */
int fdtd_add_probe(fdtd_grid* g, int i, int j, int k, int* id);

/* Plane-voltage probe: V = -sum_{k=k0}^{k1-1} Ez(i, j, k+1/2) dz, the potential of
 * node (i, j, k1) over node (i, j, k0) along the column (Results section: the
 * voltage between the power and ground planes), 0 <= i <= nx, 0 <= j <= ny,
 * 0 <= k0 < k1 <= nz.  Built from k1-k0 Ez probes (added to the probe list with
 * consecutive indices, so they count in fdtd_info.n_probes and carry DFT
 * accumulators if frequencies are set).  *id receives the voltage-probe index.
 * ESTATE after the first step. */
int fdtd_add_voltage_probe(fdtd_grid* g, int i, int j, int k0, int k1, int* id);

/* Optional running DFT of every probe (FP64 accumulators, FP32 samples):
 * A[p][q] = sum_s e_p[s] exp(-i 2 pi f_q (s+1) dt) dt.  f_hz (host, nf values,
 * each >= 0 and finite), 1 <= nf <= 4096.  ESTATE after the first step. */
int fdtd_set_dft_freqs(fdtd_grid* g, const double* f_hz, int nf);

/* Eq. 2's eps_rw (Model section): with on != 0 every PML sigma_w in
 * s_w = kappa_w + sigma_w / (j w eps0 eps_rw) is divided by the relative
 * permittivity at the field location: the edge mean of the touching cells for
 * E and D, the mean of the two cells sharing the face (one on the outer wall)
 * for H and B, since Eq. 1 puts the same s-bar on mu.  Off (the default),
 * eps_rw = 1, which is the same wherever the PML holds air (eps_r = 1).  When it
 * is on and some PML location has eps_r != 1 (a board running into the PML),
 * steps run in the node passes' arithmetic (each PML node's coefficients rebuilt
 * from kappa and sigma / eps_rw; fdtd_info.node_passes = 1).  With a two-step
 * tile shape (the default) pairs of steps run two-step kernels of the shape
 * 64 x 14 x 2 and their variants (fdtd_info.material_two_step = 1): a tile's
 * planes whose footprint holds, within two planes below or one above, a PML
 * node with eps_r != 1 at a field location run the material variant, in that
 * tile (few tiles hold such nodes) or, for every tile, in 64 x 10 x 2 tiles (such
 * nodes fill those planes), whichever is estimated cheaper; planes near
 * conducting edges only run its conduction-only flavour in that tile; the
 * other planes run the plain kernel (fdtd_info.material_permille,
 * material_split, conduct_permille).  The odd last step of a call runs the node
 * passes (two per-node passes, H then E).  With a one-step shape set, and on
 * boards past the tiled kernels' 4 GiB offset window, every step runs the node
 * passes.  All give the same bits.  ESTATE after the first step. */
int fdtd_set_pml_eps_rw(fdtd_grid* g, int on);

/* Lossy dielectric (the Results section notes the lossless model overstates how
 * long the resonances last): sigma_cell (host, nx*ny*nz floats, x fastest, S/m,
 * each finite and >= 0, NULL = lossless) is the conductivity of every cell; each
 * E edge takes the mean of the touching cells and carries the conduction
 * current sigma_c Ebar (Ebar the mean of E^n and E^{n+1}), solved for E^{n+1}
 * as for a resistive source, whose lumped conductance it adds to.  Cells in a
 * PML slab must be lossless (EINVAL otherwise).  A board with any conductive
 * edge steps in the node passes' arithmetic (see fdtd_set_pml_eps_rw).  ESTATE
 * after the first step. */
int fdtd_set_conductivity(fdtd_grid* g, const float* sigma_cell);

/* Conductor loss (the Results section names the perfect conductors, beside the
 * lossless dielectric, as why the modelled resonances ring too long): with
 * ohms_per_square > 0 every PEC-marked Ex/Ey edge (the power and ground planes)
 * is a thin resistive sheet of that surface resistance R_s instead of a
 * perfect conductor.  Its sheet current Ebar / R_s (A/m; Ebar the mean of E^n
 * and E^{n+1}) flows within the edge's dual cell of height dz, so the edge
 * carries the conductivity 1 / (R_s dz), is solved for E^{n+1} like a lossy
 * dielectric and adds to any conductivity set by fdtd_set_conductivity; PEC Ez
 * edges stay perfect.  0 (the default) keeps perfect conductors.  A board with
 * sheets steps in the node passes' arithmetic (see fdtd_set_pml_eps_rw).  EINVAL if the
 * value is negative or not finite, and at the first step if a stepped sheet
 * edge touches a cell of a PML slab; ESTATE after the first step. */
int fdtd_set_sheet_resistance(fdtd_grid* g, double ohms_per_square);

/* Plane DFT: the running DFT of Ez(i, j, k+1/2) over every node of the node plane
 * k (0 <= k < nz; the ground-plane field of the Results section, Figs. 3-5, in the
 * frequency domain): A_f(i, j) = sum_s Ez_s(i, j) exp(-i 2 pi f (s+1) dt) dt, FP32
 * samples and FP64 accumulators, the probe DFT's definition on every node.  f_hz
 * (host, nf values, each >= 0 and finite), 1 <= nf <= 256.  The field kernels
 * store the plane's Ez of every step into a 32-step ring; a separate kernel folds
 * it into the accumulators every 32 steps and at the end of every stepping call,
 * so results do not depend on how steps are split into calls.  Device memory:
 * 128 + 16 nf bytes per plane node (rows padded to 32 nodes).  One plane per
 * handle; EINVAL if the padded plane exceeds 2^25 nodes; ESTATE after the first
 * step. */
int fdtd_set_plane_dft(fdtd_grid* g, int k, const double* f_hz, int nf);

/* Enqueue n >= 0 leapfrog steps (per step: B then H at n+1/2 from E at n, D then E
 * at n+1 with the source, PEC planes and probes; Model section, Eqs. 3-4).  The
 * first call finalises the set-up.  Whole chunks of 32 steps replay one captured
 * HIP graph; the rest are plain launches (results are identical either way).
 * ESTATE if steps would exceed max_steps or materials were never set.  The field
 * kernel flags any non-finite E value; every synchronising call after that
 * (getters, fdtd_synchronize, fdtd_probe_fft) returns FDTD_EUNSTABLE. */
int fdtd_step_n(fdtd_grid* g, int64_t n);

/* Batched stepping: advance ng handles by n[h] steps each in shared launches
 * (one field launch per pass covers every handle still running; handles whose
 * class index widths differ go to launches of their own, and material boards
 * (fdtd_info.material_two_step) to one launch per kind of their pieces per pass
 * (plain, conduction-only, material), the split each has alone, with their odd
 * last steps on the node passes).  Handles must be distinct and share one
 * device; results are bitwise those of stepping each alone (the probe
 * DFT to rounding: it sums each call's samples in one pass).  Runs on the first
 * handle's stream, ordered after (and before) work on the other handles'
 * streams by events; uses the first handle's tile shape.  The first call with a
 * given (handles in order, step counts, lead tile shape) builds a plan: the
 * per-board tables and work lists in device memory, and the call's launches
 * captured as a HIP graph when the lead's stream can be captured; later calls
 * with the same plan replay it as one graph launch and return without waiting
 * for the device.  The lead keeps its last 4 plans.  Boards whose every step
 * runs the node passes step on their own streams.  Same errors as fdtd_step_n. */
int fdtd_step_many(fdtd_grid* const* g, int ng, const int64_t* n);

/* Upper bound of the device memory (bytes) fdtd_create_grid with this
 * descriptor, plus the given numbers of sources, probes and DFT frequencies, can
 * allocate over the handle's life (for admission by HBM footprint).  A plane DFT
 * (fdtd_set_plane_dft) comes on top: 128 B + 16 B per frequency for each padded
 * node of one plane, plus 520 B per frequency.  Negative FDTD_EINVAL on a bad
 * descriptor. */
int64_t fdtd_estimate_bytes(const fdtd_grid_desc* desc, int n_sources, int n_probes, int n_freqs);

/* Spectrum of probe `id` over the steps run so far (Results section, Fig. 5):
 * X[k] = sum_{s<N} e[s] exp(-2 pi i k s / n_fft) for k = 0..n_fft/2 with a
 * rectangular window, zero padding, FP64; bin k is at k / (n_fft dt).  n_fft a
 * power of two >= N (N = completed steps), <= 2^26.  re, im: host, n_fft/2+1
 * doubles each.  Synchronises. */
int fdtd_probe_fft(fdtd_grid* g, int id, int n_fft, double* re, double* im);

/* fdtd_probe_fft without any allocation, for callers that cannot allocate
 * device memory (code running under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same spectrum, bit for bit, with the
 * same arguments and errors, computed in a fixed device scratch array of the
 * library (32 MiB, held on every device the library runs on until the process
 * ends) instead of temporary buffers.  n_fft <= 2^20 (EINVAL beyond, with a
 * message naming fdtd_probe_fft).  Every call on a device shares that device's
 * scratch: calls that overlap on one device (from several threads, or on
 * several streams) race; calls that follow one another do not, since each
 * synchronises its handle's stream before returning.  Before the first step
 * (nothing finalised) the spectrum is all zeros.  Synchronises. */
int fdtd_probe_fft_noalloc(fdtd_grid* g, int id, int n_fft, double* re, double* im);

/* Copy the first n samples (n <= completed steps) of probe `id` into out (host,
 * n floats).  Synchronises. */
int fdtd_get_probe(fdtd_grid* g, int id, float* out, int64_t n);

/* Copy the first n samples (n <= completed steps) of voltage probe `id` into out
 * (host, n doubles): sample s is V at time (s+1) dt in volts, the FP32 Ez samples
 * summed in FP64 upwards in k.  Synchronises. */
int fdtd_get_voltage(fdtd_grid* g, int id, double* out, int64_t n);

/* Copy probe `id`'s DFT accumulators into re, im (host, nf doubles each).
 * Synchronises. */
int fdtd_get_dft(fdtd_grid* g, int id, double* re, double* im);

/* Copy the plane-DFT accumulators into re, im (host, nf*(ny+1)*(nx+1) doubles
 * each, frequency-major then y then x).  ESTATE if no plane DFT was set.
 * Synchronises. */
int fdtd_get_plane_dft(fdtd_grid* g, double* re, double* im);

/* Field access in SI units (host buffers of (nx+1)(ny+1)(nz+1) floats).  D and B
 * are the UPML auxiliaries of Eq. 4 (zero where the layout keeps none: the
 * library stores D/B only where a PML loss acts on them).  set is allowed before
 * the first step or between steps; it replaces the state at the current step.
 * set stores zero for entries outside the state: a component that does not
 * exist at the node (Ex at i = nx, ...), E tangential to the outer PEC wall, and
 * H (and B) on the outer wall normal to itself (Hx at i = 0 or nx, ...), which
 * touches only such E and so never changes.  Synchronises. */
int fdtd_get_field(fdtd_grid* g, int comp, float* out);
int fdtd_set_field(fdtd_grid* g, int comp, const float* in);

/* Snapshot of one component on node plane k (0 <= k <= nz) in SI units: out (host,
 * (ny+1)(nx+1) floats, x fastest), e.g. Ez on the ground plane at the current
 * step for the animations of the Results section (Figs. 3, 4).  Synchronises. */
int fdtd_get_plane(fdtd_grid* g, int comp, int k, float* out);

/* Checkpoint: the whole stepping state (fields, auxiliaries, step counter, probe
 * samples, DFT and plane-DFT accumulators) as an opaque byte image of fdtd_state_bytes(g)
 * bytes.  Loading an image saved from a handle with identical set-up and
 * continuing gives bitwise the same results as never stopping.  Synchronises. */
int64_t fdtd_state_bytes(fdtd_grid* g);
int fdtd_save_state(fdtd_grid* g, void* host_buf, int64_t bytes);
int fdtd_load_state(fdtd_grid* g, const void* host_buf, int64_t bytes);

/* Information about the handle (valid at any time). */
int fdtd_get_info(fdtd_grid* g, fdtd_info* out);

/* Tile shape of the field kernel, (tile_x, tile_y, steps) from
 * fdtd_tile_shapes() (Model section: the leapfrog of Eqs. 1-4, fused per pass).
 *   steps = 1: a block of tile_x*tile_y + 64 threads advances tile_x columns
 *     (aligned to 128 bytes of the padded device rows) by tile_y-1 rows through
 *     one full step, recomputing H on one halo row and one halo column.
 *   steps = 2: a block of 64*tile_y + 128 threads advances 64 columns by
 *     tile_y-3 rows through two full steps in one pass over memory; the first
 *     step is recomputed on a two-cell halo and never stored.  An odd step count
 *     ends with one step of the 64x15 one-step shape.
 * Results do not depend on the shape (bitwise).  May be changed between steps;
 * EINVAL for an unsupported shape.  The default is the two-step 64x14. */
int fdtd_set_tile(fdtd_grid* g, int tile_x, int tile_y, int steps);

/* Supported tile shapes: writes up to `cap` triples (tile_x, tile_y, steps) into
 * xys (host, 3*cap ints) and returns the number of shapes. */
int fdtd_tile_shapes(int* xys, int cap);

/* Kernel timing for measurement: while on, every launch of the field kernel is
 * bracketed by HIP events on the stream it runs on.  fdtd_get_timing synchronises
 * and returns the summed duration (ms) and the launch count since it was
 * switched on, then clears them. */
int fdtd_set_timing(fdtd_grid* g, int on);
int fdtd_get_timing(fdtd_grid* g, double* ms, int64_t* launches);

/* Block until all work enqueued on the handle's stream has finished. */
int fdtd_synchronize(fdtd_grid* g);

/* The hipStream_t the handle runs on (the caller's from fdtd_grid_desc.hip_stream,
 * else the one the handle created), written to *out: for callers that order
 * their own work or events with the handle's (a batched call runs on its first
 * handle's stream).  The handle keeps ownership. */
int fdtd_get_stream(fdtd_grid* g, void** out);

/* Release everything the handle holds.  NULL is accepted. */
int fdtd_destroy_grid(fdtd_grid* g);

/* Message of the last failed call on this thread ("" if none). */
const char* fdtd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_H */
