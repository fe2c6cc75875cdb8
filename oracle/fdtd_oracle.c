/*
 * FP64 CPU oracle for the Yee / UPML leapfrog of "A Time Domain Approach to
 * Power Integrity for Printed Circuit Boards" (Mattey, Edwards, Hood).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * constant generator with the HIP library; the two meet only at the seeded
 * board inputs.
 *
 * What it computes, in the paper's order (Model section):
 *   - the domain is discretised on a Yee grid, E and H staggered by half a cell
 *     and half a step, every field starting at zero (Model, Fig. 2);
 *   - the uniaxial PML is the anisotropic medium eps1*s, mu1*s with
 *     s = diag(sy sz/sx, sx sz/sy, sx sy/sz) (Eq. 1) and per-axis stretch
 *     factors s_w = kappa_w + sigma_w/(j w eps0) (Eq. 2, PML in air so eps_rw=1);
 *     sigma = 0, kappa = 1 outside it, so one update runs everywhere;
 *   - D is introduced by Dx = eps sz/sx Ex, Dy = eps sx/sy Ey, Dz = eps sy/sz Ez;
 *     curl H = d/dt(kappa D) + sigma D/eps0 row by row (Eq. 4, last row read as
 *     the z component); D is stepped first and E follows from D, and
 *     likewise B then H using the same s (mu2 = mu1 s in Eq. 1);
 *   - sigma and kappa are graded polynomially from the PML interface to the
 *     outer PEC wall (Eq. 5, read as (depth/d)^m);
 *   - with pml_eps_rw set, Eq. 2's s_w = kappa_w + sigma_w / (j w eps0 eps_rw)
 *     takes eps_rw as the relative permittivity at each field location: the
 *     edge mean for E and D, the mean of the two cells sharing the face for H
 *     and B (Eq. 1 puts the same s-bar on mu); otherwise eps_rw = 1;
 *   - the power and ground planes zero the tangential Ex, Ey on their edges;
 *   - a current source enters the D_z update as -J_z at the half step;
 *   - a lossy dielectric (the Results section notes the lossless model overstates
 *     how long the ringing lasts): conductivity sigma_c per cell, the edge mean of
 *     the touching cells, with eps dE/dt + sigma_c Ebar = curl H - J and Ebar the
 *     mean of E^n and E^{n+1}, solved for E^{n+1} (interior edges only);
 *   - conductor loss (the Results section names the perfect conductors, with the
 *     lossless dielectric, as why the ringing lasts too long): with sheet_R > 0
 *     every PEC-marked Ex/Ey edge is a thin resistive sheet of surface
 *     resistance sheet_R (ohms per square) instead of a perfect conductor.  Its
 *     sheet current density K = Ebar / sheet_R (A/m) flows within the edge's
 *     dual cell, of height dz, so the edge carries the volume conductivity
 *     1 / (sheet_R dz), added to any dielectric loss and stepped like it;
 *   - a resistive voltage source (Results section, the Table 1 run, built with
 *     semi-explicit update coefficients) is a lumped element on one E_z edge of
 *     the interior: an EMF V_s that raises node k+1 over node k, in series with
 *     R.  Its branch current density (dz Ebar + V_s)/(R dx dy) enters like J_z,
 *     with Ebar the mean of E_z^n and E_z^{n+1}, and the update is solved for
 *     E_z^{n+1}; open-circuited it holds dz E_z = -V_s.
 * Every array is stored for every node (the paper's unified storage of D and B
 * beside E and H).  Loops are plain triple loops in FP64, with no tiling.
 *
 * Time discretisation (centred at the half step, trapezoidal loss term):
 *   D^{n+1} = a_v D^n + b_v (curl H^{n+1/2} - J^{n+1/2})
 *   E^{n+1} = a_w E^n + (p+_u D^{n+1} - p-_u D^n) / (eps p+_w)
 * with a = (2 eps0 kappa - sigma dt)/(2 eps0 kappa + sigma dt),
 * b = 2 eps0 dt/(2 eps0 kappa + sigma dt), p+- = 2 eps0 kappa +- sigma dt, and
 * (u, v, w) = (x, y, z) for Ex, (y, z, x) for Ey, (z, x, y) for Ez.  The H side
 * is the same with B, mu0 and a minus sign on curl E.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_C0 299792458.0
#define OR_MU0 (4.0e-7 * 3.14159265358979323846)
#define OR_EPS0 (1.0 / (OR_MU0 * OR_C0 * OR_C0))
#define OR_ETA0 (OR_MU0 * OR_C0)
#define OR_PI 3.14159265358979323846

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double dt;                 /* > 0: used as is; 0: courant * CFL (Eq. 7, c0) */
    double courant;
    int32_t npml[6];           /* -x +x -y +y -z +z */
    double pml_m, pml_R, pml_kappa_max;
    const float* eps_r_cell;   /* nz*ny*nx, x fastest */
    const float* sigma_cell;   /* NULL or nz*ny*nx conductivity in S/m, zero in PML slabs */
    const uint8_t* pec_mask;   /* (nz+1)(ny+1)(nx+1), bit0 Ex bit1 Ey bit2 Ez */
    int32_t nsrc;
    const int32_t* src_ijk;    /* 3*nsrc */
    const int32_t* src_wave;   /* 0 Gaussian, 1 differentiated Gaussian */
    const double* src_J0;
    const double* src_t0;
    const double* src_sigma;
    const double* src_R;       /* NULL or per source: 0 current source (J0 in A/m^2),
                                  > 0 resistive voltage source (J0 = V0 in volts) */
    int32_t nprobe;
    const int32_t* probe_ijk;  /* 3*nprobe, Ez(i,j,k+1/2) */
    int32_t nfreq;
    const double* freqs;       /* Hz */
    int32_t pml_eps_rw;        /* 1: Eq. 2's sigma_w / eps_rw with the local eps_r at each
                                  field location; 0: eps_rw = 1 */
    int32_t plane_k;           /* >= 0: running DFT of Ez(i, j, plane_k+1/2) over the plane */
    int32_t nplane_freq;
    const double* plane_freqs; /* Hz */
    double sheet_R;            /* > 0: PEC-marked Ex/Ey edges are resistive sheets of this
                                  surface resistance (ohm per square); 0: perfect conductors */
} or_problem;

typedef struct {
    /* each (nz+1)(ny+1)(nx+1), x fastest, caller owned */
    double *ex, *ey, *ez, *hx, *hy, *hz;
    double *ddx, *ddy, *ddz, *bbx, *bby, *bbz;
    int64_t step;              /* completed steps */
} or_state;

/* Eq. 7 with the free-space phase velocity (the fastest medium in the grid). */
double or_cfl_dt(double dx, double dy, double dz)
{
    return 1.0 / (OR_C0 * sqrt(1.0 / (dx * dx) + 1.0 / (dy * dy) + 1.0 / (dz * dz)));
}

double or_time_step(const or_problem* p)
{
    if (p->dt > 0.0) return p->dt;
    return p->courant * or_cfl_dt(p->dx, p->dy, p->dz);
}

/* Eq. 5: sigma(depth) = (depth/d)^m sigma_max, kappa = 1 + (kappa_max-1)(depth/d)^m,
 * depth measured from the PML interface towards the outer PEC wall, in cells.
 * sigma_max = -(m+1) ln R / (2 eta0 N delta) (polynomial-grading design rule for a
 * target normal-incidence reflection R; the paper does not print a value). */
static void or_profile(double pos, int n, int nlo, int nhi, double delta,
                       const or_problem* p, double* sigma, double* kappa)
{
    double depth = 0.0, npml = 0.0;
    if (nlo > 0 && pos < (double)nlo) {
        depth = (double)nlo - pos;
        npml = (double)nlo;
    } else if (nhi > 0 && pos > (double)(n - nhi)) {
        depth = pos - (double)(n - nhi);
        npml = (double)nhi;
    }
    if (depth <= 0.0) {
        *sigma = 0.0;
        *kappa = 1.0;
        return;
    }
    double frac = pow(depth / npml, p->pml_m);
    double smax = -(p->pml_m + 1.0) * log(p->pml_R) / (2.0 * OR_ETA0 * npml * delta);
    *sigma = frac * smax;
    *kappa = 1.0 + (p->pml_kappa_max - 1.0) * frac;
}

/* Per-axis 1-D coefficients at nodes (pos = i) and half nodes (pos = i + 1/2),
 * with the raw sigma and kappa they come from. */
typedef struct {
    double *a_n, *b_n, *pp_n, *pm_n;   /* n+1 entries, node i */
    double *a_h, *b_h, *pp_h, *pm_h;   /* n+1 entries, half node i+1/2 (last unused) */
    double *sig_n, *kap_n, *sig_h, *kap_h;
} or_axis;

/* The four update coefficients of one axis at one field location. */
typedef struct {
    double a, b, pp, pm;
} or_coef;

static void or_axis_fill(or_axis* ax, int n, int nlo, int nhi, double delta, double dt,
                         const or_problem* p)
{
    size_t sz = (size_t)(n + 1) * sizeof(double);
    ax->a_n = malloc(sz); ax->b_n = malloc(sz); ax->pp_n = malloc(sz); ax->pm_n = malloc(sz);
    ax->a_h = malloc(sz); ax->b_h = malloc(sz); ax->pp_h = malloc(sz); ax->pm_h = malloc(sz);
    ax->sig_n = malloc(sz); ax->kap_n = malloc(sz); ax->sig_h = malloc(sz); ax->kap_h = malloc(sz);
    for (int i = 0; i <= n; ++i) {
        for (int half = 0; half < 2; ++half) {
            double s, k;
            or_profile((double)i + 0.5 * half, n, nlo, nhi, delta, p, &s, &k);
            if (half) { ax->sig_h[i] = s; ax->kap_h[i] = k; }
            else      { ax->sig_n[i] = s; ax->kap_n[i] = k; }
            double pp = 2.0 * OR_EPS0 * k + s * dt;
            double pm = 2.0 * OR_EPS0 * k - s * dt;
            double a = pm / pp;
            double b = 2.0 * OR_EPS0 * dt / pp;
            if (half) { ax->a_h[i] = a; ax->b_h[i] = b; ax->pp_h[i] = pp; ax->pm_h[i] = pm; }
            else      { ax->a_n[i] = a; ax->b_n[i] = b; ax->pp_n[i] = pp; ax->pm_n[i] = pm; }
        }
    }
}

static void or_axis_free(or_axis* ax)
{
    free(ax->a_n); free(ax->b_n); free(ax->pp_n); free(ax->pm_n);
    free(ax->a_h); free(ax->b_h); free(ax->pp_h); free(ax->pm_h);
    free(ax->sig_n); free(ax->kap_n); free(ax->sig_h); free(ax->kap_h);
}

/* Coefficients of axis ax at index i (half: at i + 1/2) seen from a field
 * location whose relative permittivity is eps_rw: Eq. 2 divides sigma by eps_rw
 * (the same s-bar enters mu, so H and B use it too).  eps_rw == 1 is the table. */
static inline __attribute__((always_inline)) or_coef or_at(const or_axis* ax, int i, int half,
                                                         double eps_rw, double dt)
{
    or_coef c;
    if (eps_rw == 1.0) {
        if (half) { c.a = ax->a_h[i]; c.b = ax->b_h[i]; c.pp = ax->pp_h[i]; c.pm = ax->pm_h[i]; }
        else      { c.a = ax->a_n[i]; c.b = ax->b_n[i]; c.pp = ax->pp_n[i]; c.pm = ax->pm_n[i]; }
        return c;
    }
    const double s = (half ? ax->sig_h[i] : ax->sig_n[i]) / eps_rw;
    const double k = half ? ax->kap_h[i] : ax->kap_n[i];
    c.pp = 2.0 * OR_EPS0 * k + s * dt;
    c.pm = 2.0 * OR_EPS0 * k - s * dt;
    c.a = c.pm / c.pp;
    c.b = 2.0 * OR_EPS0 * dt / c.pp;
    return c;
}

/* An interior edge (kappa 1, PML sigma 0, so D = eps E and the D update is
 * D += dt (curl - J)) carrying a conduction current g Ebar, Ebar the mean of E^n
 * and E^{n+1}: eps (E' - E)/dt = curl - g (E' + E)/2, solved for E'. */
static void or_lossy(double* e, double* d, double curl, double g, double eps, double dt)
{
    const double beta = 0.5 * dt * g / eps;
    const double e_n = ((1.0 - beta) * *e + dt / eps * curl) / (1.0 + beta);
    *d += eps * (e_n - *e);
    *e = e_n;
}

/* Source waveform (Results section, Eq. 8 and the workload's plain Gaussian). */
double or_waveform(int wave, double J0, double t0, double sigma, double t)
{
    double u = (t - t0) / sigma;
    if (wave == 1) return J0 * u * exp(-u * u);
    return J0 * exp(-0.5 * u * u);
}

#define IX(i, j, k) (((size_t)(k) * (size_t)(ny + 1) + (size_t)(j)) * (size_t)(nx + 1) + (size_t)(i))
#define CELL(i, j, k) (((size_t)(k) * (size_t)ny + (size_t)(j)) * (size_t)nx + (size_t)(i))

/*
 * Advance the state by nsteps full steps.  probe_series receives nprobe rows of
 * nsteps samples (row p, column s = Ez at the probe at time (step+s+1) dt);
 * dft_re/dft_im (nprobe x nfreq) are accumulated, not cleared:
 *   A_pq += e_p[s] exp(-i 2 pi f_q (s+1) dt) dt.
 * plane_re/plane_im (nplane_freq x (ny+1) x (nx+1)) accumulate the same sum for
 * every node (i, j) of Ez on plane plane_k (the field at the ground plane over
 * the whole board, Results section, Figs. 3-5).
 * Any output pointer may be NULL.  Returns 0.
 */
int or_run(const or_problem* p, or_state* st, int64_t nsteps,
           double* probe_series, double* dft_re, double* dft_im,
           double* plane_re, double* plane_im)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const double dt = or_time_step(p);
    const double rdx = 1.0 / p->dx, rdy = 1.0 / p->dy, rdz = 1.0 / p->dz;
    or_axis X, Y, Z;
    or_axis_fill(&X, nx, p->npml[0], p->npml[1], p->dx, dt, p);
    or_axis_fill(&Y, ny, p->npml[2], p->npml[3], p->dy, dt, p);
    or_axis_fill(&Z, nz, p->npml[4], p->npml[5], p->dz, dt, p);
    const float* er = p->eps_r_cell;
    const uint8_t* pec = p->pec_mask;
    double *ex = st->ex, *ey = st->ey, *ez = st->ez;
    double *hx = st->hx, *hy = st->hy, *hz = st->hz;
    double *Dx = st->ddx, *Dy = st->ddy, *Dz = st->ddz;
    double *Bx = st->bbx, *By = st->bby, *Bz = st->bbz;

    for (int64_t s = 0; s < nsteps; ++s) {
        const int64_t n = st->step;

        /* ---- B then H at n+1/2 from E at n ---- */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    /* Hx(i, j+1/2, k+1/2); eps_rw: the two cells sharing its x face */
                    size_t c = IX(i, j, k);
                    const double ew = p->pml_eps_rw ?
                        0.5 * ((double)er[CELL(i > 0 ? i - 1 : 0, j, k)] +
                               (double)er[CELL(i < nx ? i : nx - 1, j, k)]) : 1.0;
                    const or_coef cx = or_at(&X, i, 0, ew, dt), cy = or_at(&Y, j, 1, ew, dt),
                                  cz = or_at(&Z, k, 1, ew, dt);
                    double curl = (ez[IX(i, j + 1, k)] - ez[c]) * rdy
                                - (ey[IX(i, j, k + 1)] - ey[c]) * rdz;
                    double bo = Bx[c];
                    double bn = cy.a * bo - cy.b * curl;
                    Bx[c] = bn;
                    hx[c] = cz.a * hx[c] + (cx.pp * bn - cx.pm * bo) / (OR_MU0 * cz.pp);
                }
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    /* Hy(i+1/2, j, k+1/2); eps_rw: the two cells sharing its y face */
                    size_t c = IX(i, j, k);
                    const double ew = p->pml_eps_rw ?
                        0.5 * ((double)er[CELL(i, j > 0 ? j - 1 : 0, k)] +
                               (double)er[CELL(i, j < ny ? j : ny - 1, k)]) : 1.0;
                    const or_coef cx = or_at(&X, i, 1, ew, dt), cy = or_at(&Y, j, 0, ew, dt),
                                  cz = or_at(&Z, k, 1, ew, dt);
                    double curl = (ex[IX(i, j, k + 1)] - ex[c]) * rdz
                                - (ez[IX(i + 1, j, k)] - ez[c]) * rdx;
                    double bo = By[c];
                    double bn = cz.a * bo - cz.b * curl;
                    By[c] = bn;
                    hy[c] = cx.a * hy[c] + (cy.pp * bn - cy.pm * bo) / (OR_MU0 * cx.pp);
                }
#pragma omp parallel for schedule(static)
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    /* Hz(i+1/2, j+1/2, k); eps_rw: the two cells sharing its z face */
                    size_t c = IX(i, j, k);
                    const double ew = p->pml_eps_rw ?
                        0.5 * ((double)er[CELL(i, j, k > 0 ? k - 1 : 0)] +
                               (double)er[CELL(i, j, k < nz ? k : nz - 1)]) : 1.0;
                    const or_coef cx = or_at(&X, i, 1, ew, dt), cy = or_at(&Y, j, 1, ew, dt),
                                  cz = or_at(&Z, k, 0, ew, dt);
                    double curl = (ey[IX(i + 1, j, k)] - ey[c]) * rdx
                                - (ex[IX(i, j + 1, k)] - ex[c]) * rdy;
                    double bo = Bz[c];
                    double bn = cx.a * bo - cx.b * curl;
                    Bz[c] = bn;
                    hz[c] = cy.a * hz[c] + (cz.pp * bn - cz.pm * bo) / (OR_MU0 * cy.pp);
                }

        /* ---- D then E at n+1 from H at n+1/2 ---- */
        const double tJ = ((double)n + 0.5) * dt;
#pragma omp parallel for schedule(static)
        for (int k = 1; k < nz; ++k)
            for (int j = 1; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    /* Ex(i+1/2, j, k) */
                    size_t c = IX(i, j, k);
                    if ((pec[c] & 1) && !(p->sheet_R > 0.0)) { ex[c] = 0.0; continue; }
                    /* a resistive sheet's edge: sheet conductance over the dual cell height */
                    const double g_sh = (pec[c] & 1) ? 1.0 / (p->sheet_R * p->dz) : 0.0;
                    const double er_e = 0.25 *
                        ((double)er[CELL(i, j - 1, k - 1)] + (double)er[CELL(i, j, k - 1)] +
                         (double)er[CELL(i, j - 1, k)] + (double)er[CELL(i, j, k)]);
                    const double eps = OR_EPS0 * er_e;
                    const double ew = p->pml_eps_rw ? er_e : 1.0;
                    const or_coef cx = or_at(&X, i, 1, ew, dt), cy = or_at(&Y, j, 0, ew, dt),
                                  cz = or_at(&Z, k, 0, ew, dt);
                    double curl = (hz[c] - hz[IX(i, j - 1, k)]) * rdy
                                - (hy[c] - hy[IX(i, j, k - 1)]) * rdz;
                    const double sg = g_sh + (!p->sigma_cell ? 0.0 : 0.25 *
                        ((double)p->sigma_cell[CELL(i, j - 1, k - 1)] + (double)p->sigma_cell[CELL(i, j, k - 1)] +
                         (double)p->sigma_cell[CELL(i, j - 1, k)] + (double)p->sigma_cell[CELL(i, j, k)]));
                    if (sg != 0.0) {
                        or_lossy(&ex[c], &Dx[c], curl, sg, eps, dt);
                        continue;
                    }
                    double d_o = Dx[c];
                    double d_n = cy.a * d_o + cy.b * curl;
                    Dx[c] = d_n;
                    ex[c] = cz.a * ex[c] + (cx.pp * d_n - cx.pm * d_o) / (eps * cz.pp);
                }
#pragma omp parallel for schedule(static)
        for (int k = 1; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 1; i < nx; ++i) {
                    /* Ey(i, j+1/2, k) */
                    size_t c = IX(i, j, k);
                    if ((pec[c] & 2) && !(p->sheet_R > 0.0)) { ey[c] = 0.0; continue; }
                    const double g_sh = (pec[c] & 2) ? 1.0 / (p->sheet_R * p->dz) : 0.0;
                    const double er_e = 0.25 *
                        ((double)er[CELL(i - 1, j, k - 1)] + (double)er[CELL(i, j, k - 1)] +
                         (double)er[CELL(i - 1, j, k)] + (double)er[CELL(i, j, k)]);
                    const double eps = OR_EPS0 * er_e;
                    const double ew = p->pml_eps_rw ? er_e : 1.0;
                    const or_coef cx = or_at(&X, i, 0, ew, dt), cy = or_at(&Y, j, 1, ew, dt),
                                  cz = or_at(&Z, k, 0, ew, dt);
                    double curl = (hx[c] - hx[IX(i, j, k - 1)]) * rdz
                                - (hz[c] - hz[IX(i - 1, j, k)]) * rdx;
                    const double sg = g_sh + (!p->sigma_cell ? 0.0 : 0.25 *
                        ((double)p->sigma_cell[CELL(i - 1, j, k - 1)] + (double)p->sigma_cell[CELL(i, j, k - 1)] +
                         (double)p->sigma_cell[CELL(i - 1, j, k)] + (double)p->sigma_cell[CELL(i, j, k)]));
                    if (sg != 0.0) {
                        or_lossy(&ey[c], &Dy[c], curl, sg, eps, dt);
                        continue;
                    }
                    double d_o = Dy[c];
                    double d_n = cz.a * d_o + cz.b * curl;
                    Dy[c] = d_n;
                    ey[c] = cx.a * ey[c] + (cy.pp * d_n - cy.pm * d_o) / (eps * cx.pp);
                }
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 1; j < ny; ++j)
                for (int i = 1; i < nx; ++i) {
                    /* Ez(i, j, k+1/2) */
                    size_t c = IX(i, j, k);
                    if (pec[c] & 4) { ez[c] = 0.0; continue; }
                    const double er_e = 0.25 *
                        ((double)er[CELL(i - 1, j - 1, k)] + (double)er[CELL(i, j - 1, k)] +
                         (double)er[CELL(i - 1, j, k)] + (double)er[CELL(i, j, k)]);
                    const double eps = OR_EPS0 * er_e;
                    const double ew = p->pml_eps_rw ? er_e : 1.0;
                    double J = 0.0, g_l = 0.0;
                    for (int q = 0; q < p->nsrc; ++q)
                        if (p->src_ijk[3 * q] == i && p->src_ijk[3 * q + 1] == j &&
                            p->src_ijk[3 * q + 2] == k) {
                            const double w = or_waveform(p->src_wave[q], p->src_J0[q],
                                                         p->src_t0[q], p->src_sigma[q], tJ);
                            if (p->src_R && p->src_R[q] > 0.0) {
                                /* branch current density = g_l Ebar + V_s/(R dx dy) */
                                g_l += p->dz / (p->src_R[q] * p->dx * p->dy);
                                J += w / (p->src_R[q] * p->dx * p->dy);
                            } else {
                                J += w;
                            }
                        }
                    double curl = (hy[c] - hy[IX(i - 1, j, k)]) * rdx
                                - (hx[c] - hx[IX(i, j - 1, k)]) * rdy - J;
                    const double sg = !p->sigma_cell ? 0.0 : 0.25 *
                        ((double)p->sigma_cell[CELL(i - 1, j - 1, k)] + (double)p->sigma_cell[CELL(i, j - 1, k)] +
                         (double)p->sigma_cell[CELL(i - 1, j, k)] + (double)p->sigma_cell[CELL(i, j, k)]);
                    if (g_l + sg != 0.0) {
                        /* resistive source and/or lossy dielectric on an interior edge:
                         * the lumped conductance g_l (curl already holds -V_s/(R dx dy))
                         * adds to the medium's sigma_c */
                        or_lossy(&ez[c], &Dz[c], curl, g_l + sg, eps, dt);
                        continue;
                    }
                    const or_coef cx = or_at(&X, i, 0, ew, dt), cy = or_at(&Y, j, 0, ew, dt),
                                  cz = or_at(&Z, k, 1, ew, dt);
                    double d_o = Dz[c];
                    double d_n = cx.a * d_o + cx.b * curl;
                    Dz[c] = d_n;
                    ez[c] = cy.a * ez[c] + (cz.pp * d_n - cz.pm * d_o) / (eps * cy.pp);
                }

        /* ---- probes and the running DFT at t = (n+1) dt ---- */
        for (int q = 0; q < p->nprobe; ++q) {
            const int32_t* pq = p->probe_ijk + 3 * q;
            double e = ez[IX(pq[0], pq[1], pq[2])];
            if (probe_series) probe_series[(size_t)q * (size_t)nsteps + (size_t)s] = e;
            if (dft_re && dft_im)
                for (int f = 0; f < p->nfreq; ++f) {
                    double ph = 2.0 * OR_PI * p->freqs[f] * (double)(n + 1) * dt;
                    dft_re[(size_t)q * p->nfreq + f] += e * cos(ph) * dt;
                    dft_im[(size_t)q * p->nfreq + f] -= e * sin(ph) * dt;
                }
        }
        if (p->plane_k >= 0 && plane_re && plane_im) {
            const size_t np = (size_t)(nx + 1) * (size_t)(ny + 1);
            for (int f = 0; f < p->nplane_freq; ++f) {
                const double ph = 2.0 * OR_PI * p->plane_freqs[f] * (double)(n + 1) * dt;
                const double cph = cos(ph), sph = sin(ph);
                double* re = plane_re + (size_t)f * np;
                double* im = plane_im + (size_t)f * np;
                for (int j = 0; j <= ny; ++j)
                    for (int i = 0; i <= nx; ++i) {
                        const double e = ez[IX(i, j, p->plane_k)];
                        re[(size_t)j * (nx + 1) + i] += e * cph * dt;
                        im[(size_t)j * (nx + 1) + i] -= e * sph * dt;
                    }
            }
        }
        st->step = n + 1;
    }
    or_axis_free(&X);
    or_axis_free(&Y);
    or_axis_free(&Z);
    return 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Physical constants used by the oracle, for tests that need the same values. */
void or_constants(double* c0, double* mu0, double* eps0, double* eta0)
{
    *c0 = OR_C0; *mu0 = OR_MU0; *eps0 = OR_EPS0; *eta0 = OR_ETA0;
}

/* sigma and kappa at coordinate pos (cell units) along axis 0/1/2, for tests. */
void or_sigma_kappa(const or_problem* p, int axis, double pos, double* sigma, double* kappa)
{
    const int n[3] = {p->nx, p->ny, p->nz};
    const double d[3] = {p->dx, p->dy, p->dz};
    or_profile(pos, n[axis], p->npml[2 * axis], p->npml[2 * axis + 1], d[axis], p, sigma, kappa);
}
