"""Pins of the FP64 oracle against things other than itself.

* P1  brute-force sparse-matrix leapfrog (Kronecker curls, diagonal coefficients)
* P2  PML off: a plain Yee loop written with array slices, and E == D / eps
* P3  discrete energy of a lossless PEC box is invariant
* P4  eigen-angles of the one-step map == closed-form discrete dispersion
* P8  linearity, reciprocity and mirror symmetry
* P10 the probe FFT against a direct DFT
* P11 resistive voltage source: discrete energy balance, R -> infinity limits
* P12 plane-wide DFT: closed form on a cavity eigenmode, agreement with the probe DFT
* P13 Eq. 2's eps_rw: uniform-medium equivalence, no-op in air, absorption in dielectric
* P15 lossy dielectric: closed-form recurrence of a lossy cavity eigenmode
* P17 conductor loss (resistive sheets): discrete energy balance, the closed-form
      decay of a parallel-plate resonator, the R_s -> 0 and R_s -> infinity limits
* Eq. 5 / Eq. 7 hand values (sigma_max, CFL step of the paper's grid)
"""
import numpy as np
import pytest

import boardgen
import bruteforce
from _util import live_masks, rel_max

C0 = 299792458.0
MU0 = 4e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 ** 2)


def _random_state(oracle, board, seed, aux=True):
    st = oracle.new_state(board)
    m = live_masks(board)
    rng = np.random.default_rng(seed)
    for n in oracle.FIELD_NAMES:
        if n.startswith(("dd", "bb")) and not aux:
            continue
        st[n][...] = np.where(m[n], rng.standard_normal(st[n].shape), 0.0)
    # give H a physical scale relative to E so both curls matter
    for n in ("hx", "hy", "hz"):
        st[n] /= 376.73
    for n in ("ddx", "ddy", "ddz"):
        st[n] *= EPS0
    for n in ("bbx", "bby", "bbz"):
        st[n] *= MU0 / 376.73
    return st


BF_NAME = {"ddx": "dx", "ddy": "dy", "ddz": "dz", "bbx": "bx", "bby": "by", "bbz": "bz"}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p1_bruteforce_sources_from_zero(oracle_mod, seed):
    b = boardgen.random_tiny(seed, steps=40)
    # make the pulses fire inside the short window
    for s in b.sources:
        s.t0 = 15 * oracle_mod.time_step(b)
        s.sigma = 4 * oracle_mod.time_step(b)
    r = oracle_mod.run(b)
    bf, probes = bruteforce.run(b, r.dt, b.steps)
    for n in oracle_mod.FIELD_NAMES:
        ref = bf[BF_NAME.get(n, n)]
        assert np.abs(ref).max() > 0, n
        assert rel_max(r.state[n], ref) < 1e-12, n
    assert rel_max(r.probes, probes) < 1e-12


@pytest.mark.parametrize("seed", [3, 4])
def test_p1_bruteforce_random_state(oracle_mod, seed):
    b = boardgen.random_tiny(seed, nx=9, ny=11, nz=7, npml=3, steps=6)
    b.sources = []
    st = _random_state(oracle_mod, b, seed)
    init = {BF_NAME.get(n, n): st[n].copy() for n in oracle_mod.FIELD_NAMES}
    r = oracle_mod.run(b, state=st)
    bf, _ = bruteforce.run(b, r.dt, b.steps, init=init)
    for n in oracle_mod.FIELD_NAMES:
        assert rel_max(r.state[n], bf[BF_NAME.get(n, n)]) < 1e-12, n


def _plain_yee(board, dt, st, nsteps):
    """Textbook Yee in a PEC box (no PML), E and H only, array slices."""
    ex, ey, ez, hx, hy, hz = (st[n].copy() for n in ("ex", "ey", "ez", "hx", "hy", "hz"))
    nx, ny, nz = board.nx, board.ny, board.nz
    er = board.eps_r_cell.astype(np.float64)
    ex_eps = EPS0 * 0.25 * (er[:-1, :-1, :] + er[1:, :-1, :] + er[:-1, 1:, :] + er[1:, 1:, :])
    ey_eps = EPS0 * 0.25 * (er[:-1, :, :-1] + er[1:, :, :-1] + er[:-1, :, 1:] + er[1:, :, 1:])
    ez_eps = EPS0 * 0.25 * (er[:, :-1, :-1] + er[:, 1:, :-1] + er[:, :-1, 1:] + er[:, 1:, 1:])
    pec = board.pec_edge_mask
    dx, dy, dz = board.dx, board.dy, board.dz
    for _ in range(nsteps):
        hx[:nz, :ny, :] -= dt / MU0 * ((ez[:nz, 1:, :] - ez[:nz, :-1, :]) / dy
                                       - (ey[1:, :ny, :] - ey[:-1, :ny, :]) / dz)
        hy[:nz, :, :nx] -= dt / MU0 * ((ex[1:, :, :nx] - ex[:-1, :, :nx]) / dz
                                       - (ez[:nz, :, 1:] - ez[:nz, :, :-1]) / dx)
        hz[:, :ny, :nx] -= dt / MU0 * ((ey[:, :ny, 1:] - ey[:, :ny, :-1]) / dx
                                       - (ex[:, 1:, :nx] - ex[:, :-1, :nx]) / dy)
        ex[1:nz, 1:ny, :nx] += dt / ex_eps * ((hz[1:nz, 1:ny, :nx] - hz[1:nz, :ny - 1, :nx]) / dy
                                              - (hy[1:nz, 1:ny, :nx] - hy[:nz - 1, 1:ny, :nx]) / dz)
        ey[1:nz, :ny, 1:nx] += dt / ey_eps * ((hx[1:nz, :ny, 1:nx] - hx[:nz - 1, :ny, 1:nx]) / dz
                                              - (hz[1:nz, :ny, 1:nx] - hz[1:nz, :ny, :nx - 1]) / dx)
        ez[:nz, 1:ny, 1:nx] += dt / ez_eps * ((hy[:nz, 1:ny, 1:nx] - hy[:nz, 1:ny, :nx - 1]) / dx
                                              - (hx[:nz, 1:ny, 1:nx] - hx[:nz, :ny - 1, 1:nx]) / dy)
        ex[(pec & 1) != 0] = 0.0
        ey[(pec & 2) != 0] = 0.0
        ez[(pec & 4) != 0] = 0.0
    return dict(ex=ex, ey=ey, ez=ez, hx=hx, hy=hy, hz=hz)


def _inhomogeneous_box(seed, nx=12, ny=10, nz=8):
    rng = np.random.default_rng(seed)
    b = boardgen.cavity_box(nx, ny, nz, 1e-3, 0.8e-3, 0.3e-3, 1.0, steps=60)
    b.eps_r_cell[:] = rng.choice([1.0, 2.5, 4.4], size=b.eps_r_cell.shape).astype(np.float32)
    boardgen.pec_sheet(b.pec_edge_mask, nz // 2, 2, nx - 3, 3, ny - 2)
    return b


def test_p2_pml_off_is_plain_yee(oracle_mod):
    b = _inhomogeneous_box(7)
    st = _random_state(oracle_mod, b, 7, aux=False)
    r0 = {n: st[n].copy() for n in oracle_mod.FIELD_NAMES}
    r = oracle_mod.run(b, state=st)
    ref = _plain_yee(b, r.dt, r0, b.steps)
    for n in ("ex", "ey", "ez", "hx", "hy", "hz"):
        assert rel_max(r.state[n], ref[n]) < 1e-12, n


def test_p2_e_equals_d_over_eps_without_pml(oracle_mod):
    b = _inhomogeneous_box(8)
    b.sources = [boardgen.Source(5, 5, 2, boardgen.GAUSS, 1e6, 20e-12, 5e-12)]
    r = oracle_mod.run(b, nsteps=80)
    s = bruteforce.Stepper(b, r.dt)
    for e, d in (("ex", "ddx"), ("ey", "ddy"), ("ez", "ddz")):
        m = live_masks(b)[e]
        ratio_ref = r.state[d][m] / s.eps[e][m]
        assert rel_max(r.state[e][m], ratio_ref) < 1e-12, e


def _energy(b, e_now, h_a, h_b, eps):
    """Discrete Yee energy W^n = 1/2 sum eps (E^n)^2 V + 1/2 sum mu0 H^{n-1/2} H^{n+1/2} V
    (uniform dual volumes V = dx dy dz); invariant for a lossless source-free PEC box."""
    V = b.dx * b.dy * b.dz
    m = live_masks(b)
    w = 0.0
    for e in ("ex", "ey", "ez"):
        w += 0.5 * np.sum(eps[e][m[e]] * e_now[e][m[e]] ** 2) * V
    for h in ("hx", "hy", "hz"):
        w += 0.5 * MU0 * np.sum(h_a[h][m[h]] * h_b[h][m[h]]) * V
    return w


def _energy_series(b, states, eps):
    """states[n] = (E^{n+1}, H^{n+1/2}) after step n; W^{n+1} pairs E^{n+1} with
    H^{n+1/2} H^{n+3/2}."""
    return np.array([_energy(b, states[n][0], states[n][1], states[n + 1][1], eps)
                     for n in range(len(states) - 1)])


def _snap(st):
    return ({e: st[e].copy() for e in ("ex", "ey", "ez")},
            {h: st[h].copy() for h in ("hx", "hy", "hz")})


def test_p3_energy_invariant_lossless_box(oracle_mod):
    b = _inhomogeneous_box(9)
    st = _random_state(oracle_mod, b, 9, aux=False)
    eps = bruteforce.Stepper(b, oracle_mod.time_step(b)).eps
    states = []
    for _ in range(150):
        oracle_mod.run(b, nsteps=1, state=st)
        states.append(_snap(st))
    W = _energy_series(b, states, eps)
    assert np.all(np.isfinite(W)) and W[0] > 0
    assert np.abs(W - W[0]).max() / W[0] < 1e-12


def test_p3_energy_breaks_with_a_flipped_curl_sign(oracle_mod):
    """Sanity of the pin itself: a mistake in one curl sign breaks invariance."""
    b = _inhomogeneous_box(10)
    st = _random_state(oracle_mod, b, 10, aux=False)
    s = bruteforce.Stepper(b, oracle_mod.time_step(b))
    flat = {bruteforce_name(n): st[n].ravel().copy() for n in oracle_mod.FIELD_NAMES}
    shape = st["ex"].shape

    def run(stepper):
        f = {k: v.copy() for k, v in flat.items()}
        states = []
        for n in range(120):
            stepper.step(f, n)
            states.append(_snap({k: f[k].reshape(shape) for k in
                                 ("ex", "ey", "ez", "hx", "hy", "hz")}))
        W = _energy_series(b, states, stepper.eps)
        return np.abs(W - W[0]).max() / abs(W[0])

    assert run(s) < 1e-12                   # the matrix form conserves it too
    h1, D1, h2, D2 = s.curlH["ex"]          # flip d(Hy)/dz inside curl_x H
    s.curlH["ex"] = (h1, D1, h2, -D2)
    assert run(s) > 1e-6


def bruteforce_name(n):
    return BF_NAME.get(n, n)


def _discrete_modes(nx, ny, nz, dx, dy, dz, v, dt):
    """Closed-form eigen-angles omega*dt of the Yee grid in a PEC box."""
    out = []
    for p in range(nx):
        for q in range(ny):
            for r in range(nz):
                zeros = (p == 0) + (q == 0) + (r == 0)
                mult = {0: 2, 1: 1}.get(zeros, 0)
                if mult == 0:
                    continue
                s2 = (v * dt) ** 2 * (np.sin(p * np.pi / (2 * nx)) ** 2 / dx ** 2
                                      + np.sin(q * np.pi / (2 * ny)) ** 2 / dy ** 2
                                      + np.sin(r * np.pi / (2 * nz)) ** 2 / dz ** 2)
                w = 2 * np.arcsin(np.sqrt(s2))
                out += [w] * mult
    return np.sort(np.array(out))


def test_p4_one_step_map_eigenangles(oracle_mod):
    nx, ny, nz = 4, 3, 3
    eps_r = 2.0
    b = boardgen.cavity_box(nx, ny, nz, 1.0e-3, 1.3e-3, 0.7e-3, eps_r, steps=1)
    dt = oracle_mod.time_step(b)
    m = live_masks(b)
    unknowns = [(n, idx) for n in ("ex", "ey", "ez", "hx", "hy", "hz")
                for idx in zip(*np.nonzero(m[n]))]
    N = len(unknowns)
    # scale E and H so the map is orthogonal-like (eigenvalues are scale-free anyway)
    M = np.zeros((N, N))
    for col, (n, idx) in enumerate(unknowns):
        st = oracle_mod.new_state(b)
        st[n][idx] = 1.0
        oracle_mod.run(b, nsteps=1, state=st)
        M[:, col] = [st[nn][ii] for (nn, ii) in unknowns]
    lam = np.linalg.eigvals(M)
    assert np.abs(np.abs(lam) - 1).max() < 1e-9
    ang = np.sort(np.abs(np.angle(lam)))
    nonzero = ang[ang > 1e-6]
    # each oscillating mode contributes the pair exp(+-i w dt)
    got = np.sort(nonzero)[::2]
    want = _discrete_modes(nx, ny, nz, b.dx, b.dy, b.dz, C0 / np.sqrt(eps_r), dt)
    assert len(nonzero) == 2 * len(want)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)


def test_p8_linearity(oracle_mod):
    b = boardgen.random_tiny(11, steps=60)
    for s in b.sources:
        s.t0 = 20 * oracle_mod.time_step(b)
        s.sigma = 5 * oracle_mod.time_step(b)
    both = oracle_mod.run(b).probes
    parts = []
    for s in b.sources:
        bi = boardgen.random_tiny(11, steps=60)
        bi.sources = [s]
        parts.append(oracle_mod.run(bi).probes)
    assert rel_max(both, parts[0] + parts[1]) < 1e-12
    # scaling
    b2 = boardgen.random_tiny(11, steps=60)
    b2.sources = [boardgen.Source(s.i, s.j, s.k, s.waveform, -3.5 * s.J0, s.t0, s.sigma)
                  for s in b.sources]
    assert rel_max(oracle_mod.run(b2).probes, -3.5 * both) < 1e-12


def test_p8_reciprocity_lossless(oracle_mod):
    b = _inhomogeneous_box(12, nx=14, ny=12, nz=6)
    a_pt, b_pt = (3, 4, 2), (10, 8, 3)
    outs = []
    for src, prb in ((a_pt, b_pt), (b_pt, a_pt)):
        bb = _inhomogeneous_box(12, nx=14, ny=12, nz=6)
        bb.pec_edge_mask[:] = b.pec_edge_mask
        bb.sources = [boardgen.Source(*src, boardgen.DGAUSS, 1e6, 10e-12, 3e-12)]
        bb.probes = [prb]
        outs.append(oracle_mod.run(bb, nsteps=300).probes[0])
    assert np.abs(outs[0]).max() > 0
    assert rel_max(outs[0], outs[1]) < 1e-10


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_p8_mirror_symmetry_with_pml(oracle_mod, axis):
    """A board symmetric about a mid plane (PML on both sides) gives mirror-equal
    probes: catches a misplaced node/half-node coefficient on that axis."""
    nx, ny, nz = 16, 14, 12
    ci, cj, ck = nx // 2, ny // 2, nz // 2
    eps, mask = boardgen.air(nx, ny, nz)
    # cell blocks symmetric about x = ci, y = cj and z = ck
    eps[4:8, 5:9, 3:13] = 3.0
    eps[4:8, 3:11, 6:10] = 2.0
    b = boardgen.Board("mirror", nx, ny, nz, 1e-3, 0.9e-3, 0.5e-3, eps, mask,
                       npml=(3, 3, 4, 4, 2, 2), steps=120)
    w = (boardgen.DGAUSS, 1e6, 30e-12, 8e-12)
    if axis == "x":       # Ez on the plane x = ci is even under x -> -x
        b.sources = [boardgen.Source(ci, 5, 4, *w)]
        b.probes = [(ci - 5, 9, 3), (ci + 5, 9, 3)]
    elif axis == "y":
        b.sources = [boardgen.Source(5, cj, 4, *w)]
        b.probes = [(9, cj - 4, 3), (9, cj + 4, 3)]
    else:
        # Ez(k+1/2) maps to -Ez(2 ck - 1 - k + 1/2) under z -> -z; two equal sources
        # at k = ck-1 and k = ck make the configuration odd, so Ez is even
        b.sources = [boardgen.Source(5, 4, ck - 1, *w), boardgen.Source(5, 4, ck, *w)]
        b.probes = [(9, 4, ck - 4), (9, 4, ck + 3)]
    r = oracle_mod.run(b)
    assert np.abs(r.probes[0]).max() > 0
    assert rel_max(r.probes[0], r.probes[1]) < 1e-11


def test_p10_probe_fft_against_direct_dft(oracle_mod):
    rng = np.random.default_rng(5)
    e = rng.standard_normal(300)
    n_fft = 512
    X = oracle_mod.probe_fft(e, n_fft)
    s = np.arange(300)
    k = np.arange(n_fft // 2 + 1)
    direct = (e[None, :] * np.exp(-2j * np.pi * np.outer(k, s) / n_fft)).sum(1)
    assert np.abs(X - direct).max() / np.abs(direct).max() < 1e-12


def test_eq7_time_step_values(oracle_mod):
    # the paper's grid: dx = dy = 2 mm, dz = 0.4 mm -> Eq. 7 with c0
    dtc = oracle_mod._load().or_cfl_dt(2e-3, 2e-3, 0.4e-3)
    want = 1.0 / (C0 * np.sqrt(2 / 2e-3 ** 2 + 1 / 0.4e-3 ** 2))
    assert abs(dtc - want) / want < 1e-15
    assert abs(dtc - 1.28389e-12) < 1e-17
    # config 1 at courant 0.99 -> 0.6355 ps
    assert abs(oracle_mod.time_step(boardgen.small_board()) - 0.6355e-12) < 1e-16
    # the paper's 1 ps step is below the limit; 1.33 ps equals dz / c0
    assert 1e-12 < dtc and abs(0.4e-3 / C0 - 1.334e-12) < 1e-15


def test_dt_override_is_used(oracle_mod):
    b = boardgen.table1_board(steps=10)
    assert oracle_mod.time_step(b) == 1e-12


def test_waveforms(oracle_mod):
    # Gaussian: peak J0 at t0, J0 e^{-1/2} one sigma away
    assert oracle_mod.waveform(0, 2.0, 1e-10, 3e-11, 1e-10) == 2.0
    assert abs(oracle_mod.waveform(0, 2.0, 1e-10, 3e-11, 1.3e-10) - 2 * np.exp(-0.5)) < 1e-15
    # differentiated Gaussian (Eq. 8 read with the square): odd about t0, extremum at tau/sqrt2
    t0, tau = 1e-10, 5e-11
    assert oracle_mod.waveform(1, 1.0, t0, tau, t0) == 0.0
    a = oracle_mod.waveform(1, 1.0, t0, tau, t0 + 2e-11)
    assert abs(a + oracle_mod.waveform(1, 1.0, t0, tau, t0 - 2e-11)) < 1e-15
    tt = t0 + tau / np.sqrt(2)
    g = [oracle_mod.waveform(1, 1.0, t0, tau, tt + d) for d in (-1e-14, 0, 1e-14)]
    assert g[1] > g[0] and g[1] > g[2]


def test_eq5_grading_hand_values(oracle_mod):
    """sigma_max = -(m+1) ln R / (2 eta0 N delta): 9.168 S/m in x and 45.84 S/m in z
    for the 48 x 40 mm board (N = 8, 1 mm / 0.2 mm cells, m = 3, R = 1e-6); zero at
    the PML interface, sigma_max (depth/N)^3 inside, kappa = 1."""
    b = boardgen.small_board()
    sx_wall, kx = oracle_mod.sigma_kappa(b, 0, 0.0)
    sz_wall, _ = oracle_mod.sigma_kappa(b, 2, float(b.nz))
    assert abs(sx_wall - 9.1676) < 1e-3 and abs(sz_wall - 45.838) < 1e-2 and kx == 1.0
    assert oracle_mod.sigma_kappa(b, 0, 8.0) == (0.0, 1.0)           # interface node
    assert oracle_mod.sigma_kappa(b, 1, 30.5) == (0.0, 1.0)          # interior
    s_half, _ = oracle_mod.sigma_kappa(b, 0, 4.0)                    # half depth
    assert abs(s_half - sx_wall / 8) < 1e-12
    s_hi, _ = oracle_mod.sigma_kappa(b, 0, b.nx - 0.5)               # 7.5 cells deep, +x side
    assert abs(s_hi - sx_wall * (7.5 / 8) ** 3) < 1e-12
    b2 = boardgen.small_board()
    b2.pml_kappa_max = 5.0
    assert abs(oracle_mod.sigma_kappa(b2, 2, 2.0)[1] - (1 + 4 * (6 / 8) ** 3)) < 1e-12


# ---------------------------------------------------------------------------
# P11  resistive voltage source (Results section, the Table 1 run): a lumped
# element on one E_z edge, an EMF V_s raising node k+1 over node k in series
# with R, branch current density (dz Ebar + V_s)/(R dx dy)
# ---------------------------------------------------------------------------

def _resistive_run(oracle_mod, b, st, nsteps, ijk):
    dt = oracle_mod.time_step(b)
    eps = bruteforce.Stepper(b, dt).eps
    states = [_snap(st)]
    for _ in range(nsteps):
        oracle_mod.run(b, nsteps=1, state=st)
        states.append(_snap(st))
    i, j, k = ijk
    ez = np.array([s[0]["ez"][k, j, i] for s in states])
    return dt, eps, states, ez


def _lumped_balance(oracle_mod, b, src, dt, eps, states, ez):
    """Residual and scale of the discrete Poynting balance
    W^{n+1} - W^n = -dt (Vbar + V_s) Vbar / R,  Vbar = dz (E^{n+1} + E^n) / 2,
    with V_s taken at the half step.  states[0] is the initial (E^0, H^{-1/2});
    the energy W^n pairs E^n with H^{n-1/2} H^{n+1/2}."""
    W = np.array([_energy(b, states[n][0], states[n][1], states[n + 1][1], eps)
                  for n in range(len(states) - 1)])
    n = np.arange(len(W) - 1)
    vbar = b.dz * 0.5 * (ez[n + 1] + ez[n])
    vs = np.array([oracle_mod.waveform(src.waveform, src.J0, src.t0, src.sigma,
                                       (m + 0.5) * dt) for m in n])
    dW = W[1:] - W[:-1]
    loss = -dt * (vbar + vs) * vbar / src.R
    return dict(res=dW - loss, dW=dW, vbar=vbar, vs=vs,
                diss=dt * vbar * vbar / src.R, gain=-dt * vs * vbar / src.R)


def test_p11_resistor_energy_balance_no_drive(oracle_mod):
    """V_s = 0: the resistor only dissipates, exactly dt Vbar^2 / R per step."""
    b = _inhomogeneous_box(21)
    src = boardgen.Source(5, 4, 2, boardgen.GAUSS, 0.0, 20e-12, 5e-12, R=10.0)
    b.sources = [src]
    st = _random_state(oracle_mod, b, 21, aux=False)
    st["ez"][2, 4, 5] *= 30.0     # a large start value at the resistor
    dt, eps, states, ez = _resistive_run(oracle_mod, b, st, 160, (5, 4, 2))
    r = _lumped_balance(oracle_mod, b, src, dt, eps, states, ez)
    W0 = _energy(b, states[0][0], states[0][1], states[1][1], eps)
    assert np.all(r["dW"] <= 1e-13 * W0)                 # never gains energy
    assert r["diss"].sum() > 1e-3 * W0                   # the loss is far above the residual
    assert np.abs(r["res"]).max() < 1e-11 * W0


def test_p11_resistor_energy_balance_driven(oracle_mod):
    """V_s != 0 from rest: source power -dt V_s Vbar / R in, dt Vbar^2 / R lost."""
    b = _inhomogeneous_box(22)
    src = boardgen.Source(6, 5, 3, boardgen.GAUSS, 5.0, 40e-12, 10e-12, R=10.0)
    b.sources = [src]
    st = oracle_mod.new_state(b)
    dt, eps, states, ez = _resistive_run(oracle_mod, b, st, 220, (6, 5, 3))
    r = _lumped_balance(oracle_mod, b, src, dt, eps, states, ez)
    scale = np.abs(r["gain"]).sum()
    assert scale > 0 and r["diss"].sum() > 1e-3 * scale
    assert np.abs(r["res"]).max() < 1e-11 * scale
    # the balance tells the oracle's update from plausible mistakes: a flipped
    # source sign, or a resistor taken explicitly at E^n instead of at Ebar
    flipped = r["dW"] + dt * (r["vbar"] - r["vs"]) * r["vbar"] / src.R
    assert np.abs(flipped).max() > 1e-3 * scale
    e_n = b.dz * ez[:len(r["dW"])]
    explicit = r["dW"] + dt * (e_n + r["vs"]) * r["vbar"] / src.R
    assert np.abs(explicit).max() > 1e3 * np.abs(r["res"]).max()


def test_p11_resistor_tends_to_a_current_source(oracle_mod):
    """R -> infinity with V_s = J R dx dy held fixed: the branch current density
    (dz Ebar + V_s)/(R dx dy) tends to the plain current density J (Eq. 4 with
    -J in the D_z update); the difference shrinks like 1/R."""
    b = _inhomogeneous_box(23)
    b.probes = [(4, 6, 2), (8, 3, 5)]
    J = 1e6
    ref_b = _inhomogeneous_box(23)
    ref_b.probes = b.probes
    ref_b.sources = [boardgen.Source(6, 5, 3, boardgen.GAUSS, J, 40e-12, 10e-12)]
    ref = oracle_mod.run(ref_b, nsteps=200).probes
    errs = []
    for R in (1e6, 1e8):
        b.sources = [boardgen.Source(6, 5, 3, boardgen.GAUSS, J * R * b.dx * b.dy,
                                     40e-12, 10e-12, R=R)]
        got = oracle_mod.run(b, nsteps=200).probes
        errs.append(rel_max(got, ref))
    assert errs[0] < 1e-3 and errs[1] < 1e-5
    assert 50 < errs[0] / errs[1] < 200


def test_p11_resistor_zero_drive_infinite_r_is_no_source(oracle_mod):
    b = _inhomogeneous_box(24)
    st0 = _random_state(oracle_mod, b, 24, aux=False)
    st1 = {n: (v.copy() if isinstance(v, np.ndarray) else v) for n, v in st0.items()}
    oracle_mod.run(b, nsteps=50, state=st0)
    b.sources = [boardgen.Source(6, 5, 3, boardgen.GAUSS, 0.0, 40e-12, 10e-12, R=1e30)]
    oracle_mod.run(b, nsteps=50, state=st1)
    for n in ("ex", "ey", "ez", "hx", "hy", "hz"):
        assert rel_max(st1[n], st0[n]) < 1e-14, n


# ---------------------------------------------------------------------------
# P12  running DFT of Ez over a whole plane (the ground-plane field of the
# Results section, Figs. 3-5, taken in the frequency domain)
# ---------------------------------------------------------------------------

def test_p12_plane_dft_of_a_cavity_eigenmode_closed_form(oracle_mod):
    """A TM_pq0 eigenmode of the Yee grid in a PEC box, started consistently
    (E^0 = A S, H^{-1/2} = (dt / 2 mu0) curl E^0), evolves as E^n = A cos(n theta) S
    with sin(theta/2) = c dt sqrt(lambda)/2, lambda the discrete Laplacian
    eigenvalue.  Its plane DFT is then the closed form
    A S(i, j) sum_s cos((s+1) theta) exp(-i 2 pi f (s+1) dt) dt on every node."""
    nx, ny, nz, er = 12, 9, 3, 2.2
    dx, dy, dz = 1e-3, 1.3e-3, 0.5e-3
    b = boardgen.cavity_box(nx, ny, nz, dx, dy, dz, er, steps=400)
    dt = oracle_mod.time_step(b)
    p, q, A = 2, 1, 3.0
    ii = np.arange(nx + 1)
    jj = np.arange(ny + 1)
    S = np.outer(np.sin(q * np.pi * jj / ny), np.sin(p * np.pi * ii / nx))   # [j, i]
    st = oracle_mod.new_state(b)
    st["ez"][:nz] = A * S[None]
    # H^{-1/2} = (dt / (2 mu0)) curl E^0: Hx(i, j+1/2) from dEz/dy, Hy(i+1/2, j) from -dEz/dx
    ez0 = A * S
    st["hx"][:nz, :ny, :] = dt / (2 * MU0) * ((ez0[1:, :] - ez0[:-1, :]) / dy)[None]
    st["hy"][:nz, :, :nx] = dt / (2 * MU0) * (-(ez0[:, 1:] - ez0[:, :-1]) / dx)[None]
    c = C0 / np.sqrt(float(np.float32(er)))     # the board stores eps_r in FP32
    lam = 4 * np.sin(p * np.pi / (2 * nx)) ** 2 / dx ** 2 + 4 * np.sin(q * np.pi / (2 * ny)) ** 2 / dy ** 2
    theta = 2 * np.arcsin(c * dt * np.sqrt(lam) / 2)
    f_mode = theta / (2 * np.pi * dt)
    freqs = np.array([0.0, 0.5 * f_mode, f_mode, 1.3 * f_mode])
    b.plane_dft = (1, freqs)
    r = oracle_mod.run(b, state=st)
    n = np.arange(1, b.steps + 1)
    for fi, f in enumerate(freqs):
        amp = np.sum(np.cos(n * theta) * np.exp(-2j * np.pi * f * n * dt)) * dt
        ref = A * amp * S
        got = r.plane_dft[fi]
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(A * dt * b.steps), (fi, np.abs(got - ref).max())
    # the pin sees a transposed plane, a dropped dt or a flipped imaginary sign
    good = r.plane_dft[3]
    ref2 = A * np.sum(np.cos(n * theta) * np.exp(-2j * np.pi * freqs[3] * n * dt)) * dt * S
    assert np.abs(np.conj(good) - ref2).max() > 1e-3 * np.abs(ref2).max()
    assert np.abs(good / dt - ref2).max() > 1e-3 * np.abs(ref2).max()
    assert np.abs(good.T[:ny + 1, :ny + 1] - ref2[:, :ny + 1]).max() > 1e-3 * np.abs(ref2).max()


def test_p12_plane_dft_equals_probe_dft_on_its_nodes(oracle_mod):
    """The plane accumulators and the probe accumulators are separate code paths
    with the same definition: on a board with sources and PML they agree exactly
    at every probed node of the plane, and the plane is zero on PEC edges."""
    b = boardgen.random_tiny(31, nx=13, ny=11, nz=9, npml=2, steps=70)
    k = 3
    rng = np.random.default_rng(5)
    b.probes = [(int(rng.integers(0, b.nx + 1)), int(rng.integers(0, b.ny + 1)), k)
                for _ in range(12)]
    b.plane_dft = (k, b.dft_freqs)
    r = oracle_mod.run(b)
    for q, (i, j, _k) in enumerate(b.probes):
        assert np.array_equal(r.plane_dft[:, j, i], r.dft[q]), (i, j)
    assert np.abs(r.plane_dft).max() > 0
    pec = (b.pec_edge_mask[k] & 4) != 0
    assert np.all(r.plane_dft[:, pec] == 0)
    # carried accumulators: two halves equal one run
    h1 = oracle_mod.run(b, nsteps=30)
    h2 = oracle_mod.run(b, nsteps=40, state=h1.state, plane_dft=h1.plane_dft)
    assert np.allclose(h2.plane_dft, r.plane_dft, rtol=0, atol=1e-12 * np.abs(r.plane_dft).max())


# ---------------------------------------------------------------------------
# P13  Eq. 2's eps_rw: each PML sigma divided by the relative permittivity at
# the field location (E, D: the edge; H, B: the face)
# ---------------------------------------------------------------------------

def _pml_box(eps_r, seed, n=(14, 12, 10), npml=3):
    nx, ny, nz = n
    eps, mask = boardgen.air(nx, ny, nz)
    eps[:] = np.float32(eps_r)
    return boardgen.Board(f"pmlbox{seed}", nx, ny, nz, 1e-3, 0.8e-3, 0.5e-3, eps, mask,
                          npml=(npml, npml + 1, npml, npml - 1, npml, npml), steps=40)


def test_p13_eps_rw_in_a_uniform_medium_is_sigma_over_eps_r(oracle_mod):
    """In a medium of uniform eps_r every location sees eps_rw = eps_r, so Eq. 2
    equals eps_rw = 1 with every sigma divided by eps_r, i.e. sigma_max / eps_r,
    i.e. a design reflection R^(1/eps_r).  A dropped, squared or inverted eps_rw,
    or one applied to E but not to H, fails this."""
    er = 4.0
    a = _pml_box(er, 1)
    a.pml_eps_rw = True
    b = _pml_box(er, 1)
    b.pml_R = a.pml_R ** (1.0 / er)
    st_a = _random_state(oracle_mod, a, 3)
    st_b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st_a.items()}
    oracle_mod.run(a, state=st_a)
    oracle_mod.run(b, state=st_b)
    for n in oracle_mod.FIELD_NAMES:
        assert rel_max(st_a[n], st_b[n]) < 1e-12, n
    # and the scaling is not a no-op here
    c = _pml_box(er, 1)
    st_c = _random_state(oracle_mod, c, 3)
    oracle_mod.run(c, state=st_c)
    assert rel_max(st_c["ddx"], st_a["ddx"]) > 1e-3


def test_p13_eps_rw_is_a_no_op_where_the_pml_is_air(oracle_mod):
    b = boardgen.random_tiny(40, nx=16, ny=14, nz=12, npml=2, steps=30)
    p = b.npml
    b.eps_r_cell[:] = 1.0
    b.eps_r_cell[p[4] + 1:b.nz - p[5] - 1, p[2] + 1:b.ny - p[3] - 1, p[0] + 1:b.nx - p[1] - 1] = 4.4
    r0 = oracle_mod.run(b)
    b.pml_eps_rw = True
    r1 = oracle_mod.run(b)
    for n in oracle_mod.FIELD_NAMES:
        assert np.array_equal(r0.state[n], r1.state[n]), n
    assert np.array_equal(r0.probes, r1.probes)


@pytest.mark.slow
def test_p13_eps_rw_pml_absorbs_in_dielectric(oracle_mod):
    """A dielectric (eps_r 4.4) filling the whole domain, PML included: with Eq. 2's
    eps_rw the reflection seen two cells in front of the PML, against the same
    geometry in a box large enough to show none, stays below -40 dB (-42.5 dB);
    with eps_rw = 1 the effective grading is eps_r times steeper and the same
    layer reflects far more (-31 dB)."""
    d, er, npml, half_small, half_big = 1e-3, 4.4, 10, 12, 40
    wave = (boardgen.DGAUSS, 1e6, 40e-12, 10e-12)

    def box(half, rw):
        n = 2 * half + 2 * npml
        eps, mask = boardgen.air(n, n, n)
        eps[:] = np.float32(er)
        c = n // 2
        b = boardgen.Board(f"pmldiel{half}", n, n, n, d, d, d, eps, mask, npml=(npml,) * 6,
                           steps=300, pml_eps_rw=rw)
        b.sources = [boardgen.Source(c, c, c, *wave)]
        b.probes = [(c - half_small + 2, c, c)]
        return b

    def reflection(rw):
        e = oracle_mod.run(box(half_small, rw), threads=8).probes[0]
        e_ref = oracle_mod.run(box(half_big, rw), threads=8).probes[0]
        return 20 * np.log10(np.abs(e - e_ref).max() / np.abs(e_ref).max())

    assert reflection(True) < -40.0
    assert reflection(False) > -35.0


# ---------------------------------------------------------------------------
# P15  lossy dielectric: conduction current sigma_c Ebar, solved for E^{n+1}
# ---------------------------------------------------------------------------

def test_p15_lossy_cavity_eigenmode_recurrence(oracle_mod):
    """A TM_pq0 eigenmode of a PEC box filled with a uniformly lossy dielectric
    keeps its shape S(i, j); its amplitude obeys, in closed form,
    (1 + beta) u_{n+1} - (2 - s2) u_n + (1 - beta) u_{n-1} = 0 with
    beta = sigma dt / (2 eps) and s2 = (c dt)^2 lambda, so it decays by
    sqrt((1 - beta) / (1 + beta)) per step.  An explicit loss term (sigma E^n) or
    a dropped factor 1/2 gives another recurrence and fails."""
    nx, ny, nz, er = 12, 9, 3, 2.2
    dx, dy, dz = 1e-3, 1.3e-3, 0.5e-3
    b = boardgen.cavity_box(nx, ny, nz, dx, dy, dz, er, steps=1)
    sigma = 0.05
    b.sigma_cell = np.full(b.eps_r_cell.shape, sigma, np.float32)
    dt = oracle_mod.time_step(b)
    p, q, A = 2, 1, 3.0
    ii, jj = np.arange(nx + 1), np.arange(ny + 1)
    S = np.outer(np.sin(q * np.pi * jj / ny), np.sin(p * np.pi * ii / nx))
    st = oracle_mod.new_state(b)
    st["ez"][:nz] = A * S[None]
    ez0 = A * S
    st["hx"][:nz, :ny, :] = dt / (2 * MU0) * ((ez0[1:, :] - ez0[:-1, :]) / dy)[None]
    st["hy"][:nz, :, :nx] = dt / (2 * MU0) * (-(ez0[:, 1:] - ez0[:, :-1]) / dx)[None]
    u = [A]
    for _ in range(300):
        oracle_mod.run(b, nsteps=1, state=st)
        plane = st["ez"][1]
        un = float(np.sum(plane * S) / np.sum(S * S))
        assert np.abs(plane - un * S).max() <= 1e-12 * A       # the shape is kept
        u.append(un)
    u = np.array(u)
    eps = EPS0 * float(np.float32(er))
    beta = float(np.float32(sigma)) * dt / (2 * eps)
    lam = 4 * np.sin(p * np.pi / (2 * nx)) ** 2 / dx ** 2 + 4 * np.sin(q * np.pi / (2 * ny)) ** 2 / dy ** 2
    s2 = dt ** 2 * lam / (MU0 * eps)
    res = (1 + beta) * u[2:] - (2 - s2) * u[1:-1] + (1 - beta) * u[:-2]
    assert np.abs(res).max() <= 1e-11 * A
    assert abs(u[1] - ((1 - beta) - s2 / 2) / (1 + beta) * u[0]) <= 1e-12 * A
    assert beta > 1e-3 and abs(u[-1]) < 0.7 * A                  # the loss is visible
    explicit = u[2:] - (2 - s2 - 2 * beta) * u[1:-1] + (1 - 2 * beta) * u[:-2]
    half = (1 + beta / 2) * u[2:] - (2 - s2) * u[1:-1] + (1 - beta / 2) * u[:-2]
    assert np.abs(explicit).max() > 1e3 * np.abs(res).max()
    assert np.abs(half).max() > 1e3 * np.abs(res).max()


# ---------------------------------------------------------------------------
# P17  conductor loss: the PEC sheets as thin resistive sheets of surface
# resistance R_s (sheet current Ebar / R_s within the edge's dual cell)
# ---------------------------------------------------------------------------

def _sheet_masks(b):
    """Live masks with the sheet edges counted as ordinary (stepped) edges."""
    import dataclasses
    open_b = dataclasses.replace(b, pec_edge_mask=(b.pec_edge_mask & 4).astype(np.uint8))
    return live_masks(open_b)


def _sheet_energy(b, e_now, h_a, h_b, eps, m):
    V = b.dx * b.dy * b.dz
    w = 0.0
    for e in ("ex", "ey", "ez"):
        w += 0.5 * np.sum(eps[e][m[e]] * e_now[e][m[e]] ** 2) * V
    for h in ("hx", "hy", "hz"):
        w += 0.5 * MU0 * np.sum(h_a[h][m[h]] * h_b[h][m[h]]) * V
    return w


def test_p17_sheet_energy_balance(oracle_mod):
    """Undriven, from an arbitrary state: the discrete energy falls each step by
    exactly the power the sheets dissipate, dt * sum over sheet edges of
    Ebar^2 / R_s * dx dy (the sheet area one edge carries; Ebar the mean of E^n
    and E^{n+1}).  A loss taken at E^n (explicit) or spread over dx instead of dz
    breaks the balance."""
    b = _inhomogeneous_box(31, nx=14, ny=11, nz=9)
    b.sheet_R = 0.7
    dt = oracle_mod.time_step(b)
    eps = bruteforce.Stepper(b, dt).eps
    m = _sheet_masks(b)
    st = _random_state(oracle_mod, b, 31, aux=False)
    sheet = {"ex": (b.pec_edge_mask & 1) != 0, "ey": (b.pec_edge_mask & 2) != 0}
    for e in ("ex", "ey"):
        st[e] = np.where(m[e], st[e] + 0.0, 0.0)
        st[e][sheet[e] & m[e]] *= 20.0          # large start values on the sheet
    states = [_snap(st)]
    for _ in range(120):
        oracle_mod.run(b, nsteps=1, state=st)
        states.append(_snap(st))
    W = np.array([_sheet_energy(b, states[n][0], states[n][1], states[n + 1][1], eps, m)
                  for n in range(len(states) - 1)])
    dW = W[1:] - W[:-1]

    def loss(ebar_of, area):
        out = np.zeros(len(dW))
        for n in range(len(dW)):
            for e in ("ex", "ey"):
                sel = sheet[e] & m[e]
                out[n] += dt * np.sum(ebar_of(n, e)[sel] ** 2) / b.sheet_R * area
        return out

    ebar = lambda n, e: 0.5 * (states[n][0][e] + states[n + 1][0][e])
    res = dW + loss(ebar, b.dx * b.dy)
    assert np.all(dW <= 1e-13 * W[0]) and -dW.sum() > 1e-2 * W[0]
    assert np.abs(res).max() < 1e-11 * W[0]
    explicit = dW + loss(lambda n, e: states[n][0][e], b.dx * b.dy)
    wrong_h = dW + loss(ebar, b.dy * b.dz)
    assert np.abs(explicit).max() > 1e3 * np.abs(res).max()
    assert np.abs(wrong_h).max() > 1e3 * np.abs(res).max()


def _plate_cavity(sheet_R, nx=20, ny=16, k0=2, k1=6, nz=8, dx=1e-3, dz=0.25e-3, eps_r=1.0,
                  backing_sigma=20.0):
    """PEC box with two full resistive sheets at planes k0 < k1: a parallel-plate
    resonator between them.  The layers outside the sheets are a strongly lossy
    dielectric (backing_sigma S/m), so that what leaks through a sheet is absorbed
    there: an air layer would be a resonator with the same TM_mn0 frequencies as
    the inner one and would trade energy with it."""
    b = boardgen.cavity_box(nx, ny, nz, dx, dx, dz, eps_r, steps=1)
    boardgen.pec_sheet(b.pec_edge_mask, k0, 0, nx, 0, ny)
    boardgen.pec_sheet(b.pec_edge_mask, k1, 0, nx, 0, ny)
    b.sheet_R = sheet_R
    sig = np.zeros(b.eps_r_cell.shape, np.float32)
    sig[:k0] = backing_sigma
    sig[k1:] = backing_sigma
    b.sigma_cell = sig
    return b


def _plate_mode_energy(oracle_mod, b, k0, k1, nsteps, p=1, q=1):
    """Start the TM_pq0 mode of the plate pair consistently (Ez = S between the
    plates, H at -1/2 from one half step of Faraday's law) and return the
    discrete energy of the whole box at every step, and dt."""
    nx, ny = b.nx, b.ny
    dt = oracle_mod.time_step(b)
    ii, jj = np.arange(nx + 1), np.arange(ny + 1)
    S = np.outer(np.sin(q * np.pi * jj / ny), np.sin(p * np.pi * ii / nx))
    st = oracle_mod.new_state(b)
    st["ez"][k0:k1] = S[None]
    st["hx"][k0:k1, :ny, :] = dt / (2 * MU0) * ((S[1:, :] - S[:-1, :]) / b.dy)[None]
    st["hy"][k0:k1, :, :nx] = dt / (2 * MU0) * (-(S[:, 1:] - S[:, :-1]) / b.dx)[None]
    eps = bruteforce.Stepper(b, dt).eps
    m = _sheet_masks(b)
    prev = _snap(st)
    W = []
    for _ in range(nsteps):
        oracle_mod.run(b, nsteps=1, state=st)
        cur = _snap(st)
        W.append(_sheet_energy(b, prev[0], prev[1], cur[1], eps, m))
        prev = cur
    return np.array(W), dt


def test_p17_plate_pair_decay_closed_form(oracle_mod):
    """A TM_110 mode between two plates of surface resistance R_s, h apart,
    loses energy at the rate of the textbook surface-resistance loss of a
    parallel-plate resonator: P = R_s |H_t|^2 per plate area against the stored
    mu0 |H|^2 h / 2, so the energy decays as exp(-2 R_s t / (mu0 h)) for every
    TM_mn0 mode.  Fitted over 3000 steps (about 28 periods) for two R_s, within
    1.5 % (measured 0.1-0.7 %: the sheet leaks a fraction of order R_s / eta0 into
    the backing, and the grid's dispersion shifts the mode)."""
    k0, k1, dz = 2, 6, 0.25e-3
    h = (k1 - k0) * dz
    for R_s in (0.5, 1.5):
        b = _plate_cavity(R_s, k0=k0, k1=k1, dz=dz)
        W, dt = _plate_mode_energy(oracle_mod, b, k0, k1, 3000)
        t = (np.arange(len(W)) + 1) * dt
        slope = np.polyfit(t, np.log(W), 1)[0]
        alpha = R_s / (MU0 * h)
        print(f"R_s {R_s}: fitted {-slope / 2:.4e} /s, closed form {alpha:.4e} /s")
        assert abs(-slope / 2 / alpha - 1.0) < 0.015, (R_s, -slope / 2, alpha)
        assert W[-1] < 0.5 * W[0]


def test_p17_sheet_limits(oracle_mod):
    """R_s -> 0 is the perfect conductor and R_s -> infinity no sheet at all, on
    a board with a source, from zero, to 1e-10 of the field."""
    base = _inhomogeneous_box(33, nx=14, ny=11, nz=9)
    base.sources = [boardgen.Source(6, 5, 2, boardgen.GAUSS, 1e6, 20e-12, 6e-12)]
    base.steps = 150
    import dataclasses
    pec = oracle_mod.run(base).state
    tiny = oracle_mod.run(dataclasses.replace(base, sheet_R=1e-12)).state
    none = oracle_mod.run(dataclasses.replace(
        base, pec_edge_mask=(base.pec_edge_mask & 4).astype(np.uint8))).state
    huge = oracle_mod.run(dataclasses.replace(base, sheet_R=1e30)).state
    for n in ("ex", "ey", "ez", "hx", "hy", "hz"):
        scale = np.abs(pec[n]).max()
        assert np.abs(tiny[n] - pec[n]).max() <= 1e-10 * scale, n
        assert np.abs(huge[n] - none[n]).max() <= 1e-10 * np.abs(none[n]).max(), n
    assert np.abs(none["ez"] - pec["ez"]).max() > 1e-3 * np.abs(pec["ez"]).max()
