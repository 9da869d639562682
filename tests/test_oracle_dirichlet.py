"""Pins of the oracle's fixed-temperature (Dirichlet, T = 0) walls and
source term Q, the setting of the smooth test of section 3.2, checked
against closed forms, textbook reductions, a dense brute-force assembly and
a balance invariant; and the second-order convergence of the perpendicular
numerical diffusivity that the section reports."""
import itertools

import numpy as np
import pytest

import synth
from tests.test_oracle_pins import LIMITERS, _random_unit_field, const_field


def _sine_mode(shape, ks):
    """prod_d sin(pi k_d (i_d + 1/2) / n_d): an eigenvector of the cell-centred
    second difference with odd ghosts (zero on the wall face)."""
    nxyz = tuple(reversed(shape))
    grids = np.meshgrid(*[np.arange(n) for n in reversed(nxyz)], indexing="ij")  # (.., y, x)
    m = np.ones(shape)
    for d, k in enumerate(ks):
        i = grids[len(shape) - 1 - d]
        m = m * np.sin(np.pi * k * (i + 0.5) / nxyz[d])
    return m


def _lam(k, n):
    """Eigenvalue of -delta^2 (times h^2) on that mode: 4 sin^2(pi k / 2n)."""
    return 4.0 * np.sin(np.pi * k / (2 * n)) ** 2


@pytest.mark.parametrize("limiter", LIMITERS)
@pytest.mark.parametrize("chi_perp", [0.0, 0.2])
@pytest.mark.parametrize("ncfl", [0.5, 50.0, 1e4])
def test_dirichlet_field_along_x_sine_mode(orc, limiter, chi_perp, ncfl):
    """b = x_hat: no transverse terms, D_xx = chi, D_yy = chi_perp; each
    sweep is the textbook backward-Euler step with the cell-centred
    Dirichlet second difference, whose eigenvectors are the sine modes: one
    step multiplies the mode by 1/(1 + a_x lam_x) 1/(1 + a_y lam_y)."""
    shape = (11, 16)
    h = (1 / 16, 1.3 / 11)
    chi = 0.8
    g = orc.OracleGrid(const_field(shape, (1.0, 0.0)), h, bc="dirichlet", limiter=limiter, chi_par=chi,
                       chi_perp=chi_perp)
    dt = g.dt_from_ncfl(ncfl)
    for ks in [(1, 1), (3, 2), (15, 10), (8, 5)]:
        T0 = _sine_mode(shape, ks)
        ax, ay = dt * chi / h[0] ** 2, dt * chi_perp / h[1] ** 2
        r = 1.0 / (1.0 + ax * _lam(ks[0], 16)) / (1.0 + ay * _lam(ks[1], 11))
        np.testing.assert_allclose(g.step_si(T0, dt, 1), r * T0, rtol=0, atol=1e-13)
        # four-step: two half-step solves per direction
        r4 = (1.0 + 0.5 * ax * _lam(ks[0], 16)) ** -2 * (1.0 + 0.5 * ay * _lam(ks[1], 11)) ** -2
        np.testing.assert_allclose(g.step_si(T0, dt, 1, four_step=True), r4 * T0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("ks", [(1, 1, 1), (2, 3, 1), (5, 1, 4)])
def test_dirichlet_3d_isotropic_sine_mode(orc, ks):
    """chi_perp = chi_par: D = chi I for any b; the step is the LOD implicit
    split with Dirichlet walls: factor prod_d 1/(1 + a_d lam_d), and the
    explicit step 1 - sum_d a_d lam_d."""
    shape = (6, 7, 9)
    nxyz = (9, 7, 6)
    h = (1 / 9, 1.2 / 7, 0.9 / 6)
    rng = np.random.default_rng(sum(ks))
    b = _random_unit_field(shape, rng)
    g = orc.OracleGrid(b, h, bc="dirichlet", chi_par=0.6, chi_perp=0.6)
    T0 = _sine_mode(shape, ks)
    dt = 0.37
    a = [dt * 0.6 / h[d] ** 2 for d in range(3)]
    r = np.prod([1.0 / (1.0 + a[d] * _lam(ks[d], nxyz[d])) for d in range(3)])
    np.testing.assert_allclose(g.step_si(T0, dt, 1), r * T0, rtol=0, atol=1e-13)
    dte = 0.1 * min(h) ** 2 / 0.6
    ae = [dte * 0.6 / h[d] ** 2 for d in range(3)]
    re = 1.0 - sum(ae[d] * _lam(ks[d], nxyz[d]) for d in range(3))
    np.testing.assert_allclose(g.step_explicit(T0, dte, 1), re * T0, rtol=0, atol=1e-14)


def _dirichlet_laplacian_1d(n):
    """Cell-centred second difference with odd ghosts: tridiag(1, -2, 1) with
    -3 in the two corner diagonal entries."""
    L = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    L[0, 0] = L[-1, -1] = -3.0
    return L


def test_dirichlet_isotropic_2d_is_lod_with_dense_matrices(orc):
    """chi_perp = chi_par, random b and T: the 2-D step equals
    (I - dt chi L_y)^-1 (I - dt chi L_x)^-1 (T + dt Q), L the dense Dirichlet
    second differences (the source enters the first, x, sweep)."""
    rng = np.random.default_rng(12)
    ny, nx = 9, 13
    h = (0.07, 0.05)
    b = _random_unit_field((ny, nx), rng)
    T0 = rng.standard_normal((ny, nx))
    Q = rng.standard_normal((ny, nx))
    chi, dt = 1.3, 0.004
    g = orc.OracleGrid(b, h, bc="dirichlet", chi_par=chi, chi_perp=chi, src=Q)
    Mx = np.eye(nx) - dt * chi / h[0] ** 2 * _dirichlet_laplacian_1d(nx)
    My = np.eye(ny) - dt * chi / h[1] ** 2 * _dirichlet_laplacian_1d(ny)
    Ts = np.linalg.solve(Mx, (T0 + dt * Q).T).T
    ref = np.linalg.solve(My, Ts)
    np.testing.assert_allclose(g.step_si(T0, dt, 1), ref, rtol=1e-12, atol=1e-12)
    # explicit: forward Euler with the 5-point Dirichlet stencil plus dt Q
    Lx = _dirichlet_laplacian_1d(nx) / h[0] ** 2
    Ly = _dirichlet_laplacian_1d(ny) / h[1] ** 2
    dte = 0.2 * min(h) ** 2 / chi
    ref_e = T0 + dte * chi * (T0 @ Lx.T + Ly @ T0) + dte * Q
    np.testing.assert_allclose(g.step_explicit(T0, dte, 1), ref_e, rtol=1e-12, atol=1e-13)


def test_source_one_step_and_steady_state(orc):
    """b = x_hat, chi_perp = 0, T0 = 0, Q a sine mode along x: one step gives
    dt Q / (1 + a lam) (the source is solved implicitly with the first sweep;
    the y sweep is the identity), and the step map converges to the discrete
    steady state Q h^2 / (chi lam)."""
    shape = (5, 24)
    h = (1 / 24, 0.2)
    chi = 2.0
    Q = 3.0 * _sine_mode(shape, (3, 1)) / np.sin(np.pi * (np.arange(5)[:, None] + 0.5) / 5)
    g = orc.OracleGrid(const_field(shape, (1.0, 0.0)), h, bc="dirichlet", chi_par=chi, src=Q)
    dt = g.dt_from_ncfl(100.0)
    a = dt * chi / h[0] ** 2
    lam = _lam(3, 24)
    np.testing.assert_allclose(g.step_si(np.zeros(shape), dt, 1), dt * Q / (1 + a * lam), rtol=1e-13, atol=1e-15)
    T = g.step_si(np.zeros(shape), dt, 400)
    np.testing.assert_allclose(T, Q * h[0] ** 2 / (chi * lam), rtol=1e-11, atol=1e-13)
    # explicit: one forward-Euler step from 0 is exactly dt Q
    np.testing.assert_array_equal(g.step_explicit(np.zeros(shape), 0.1 * h[0] ** 2, 1), 0.1 * h[0] ** 2 * Q)


def _brute_force_dirichlet_step(b, h, limiter, T, dt, chi_par, chi, Q, four_step=False):
    """Dense assembly of each sweep on a grid with T = 0 walls: interior
    faces as in section 2; a wall face adds 2 alpha_w (b and chi of its
    cell) to its cell's diagonal and carries no transverse flux; transverse
    differences read odd ghosts; dt Q joins the first sweep's right-hand
    side.  Coordinates from an explicit neighbour table."""
    shape = T.shape
    nd = len(shape)
    nxyz = tuple(reversed(shape))
    N = T.size
    coords = list(itertools.product(*[range(n) for n in reversed(nxyz)]))
    index = {c: k for k, c in enumerate(coords)}
    chic = np.full(N, chi_par) if chi is None else chi.ravel()

    def lim2(a, c):
        if limiter == "linear":
            return 0.5 * (a + c)
        if a * c <= 0:
            return 0.0
        if limiter == "vanleer":
            return 2 * a * c / (a + c)
        if limiter == "minmod":
            return np.sign(a) * min(abs(a), abs(c))
        return np.sign(a) * min(2 * abs(a), 2 * abs(c), abs(a + c) / 2)

    def shift(c, axis, s):
        pos = list(c)
        k = nd - 1 - axis
        m = pos[k] + s
        if m < 0 or m >= nxyz[axis]:
            return None
        pos[k] = m
        return tuple(pos)

    def val(U, c, axis, s):
        c2 = shift(c, axis, s)
        return -U[index[c]] if c2 is None else U[index[c2]]

    x = T.ravel().copy()
    bf = [bb.ravel() for bb in b]
    for i, d in enumerate(range(nd)):
        U = x.copy()
        dt_n = 0.5 * dt if four_step else dt
        A = np.eye(N)
        S = np.zeros(N)
        if i == 0:
            S += dt * Q.ravel()
        for c in coords:
            k0 = index[c]
            for s in (-1, +1):
                if shift(c, d, s) is None:  # a wall face of this cell
                    A[k0, k0] += 2 * dt_n * chic[k0] * bf[d][k0] ** 2 / h[d] ** 2
            c1 = shift(c, d, +1)
            if c1 is None:
                continue
            k1 = index[c1]
            chif = 2 * chic[k0] * chic[k1] / (chic[k0] + chic[k1])
            bface = [0.5 * (bf[q][k0] + bf[q][k1]) for q in range(nd)]
            e = np.zeros(N)
            e[k0], e[k1] = 1.0, -1.0
            A += dt_n * chif * bface[d] ** 2 / h[d] ** 2 * np.outer(e, e)
            F = 0.0
            for t in range(nd):
                if t == d:
                    continue
                p1 = lim2(val(U, c1, t, +1) - U[k1], U[k1] - val(U, c1, t, -1))
                p0 = lim2(val(U, c, t, +1) - U[k0], U[k0] - val(U, c, t, -1))
                F += dt * chif * bface[d] * bface[t] / (h[d] * h[t]) * lim2(p1, p0)
            S += F * e
        x = np.linalg.solve(A, U + S)
        if four_step:
            A2 = np.eye(N)
            for c in coords:
                k0 = index[c]
                for s in (-1, +1):
                    if shift(c, d, s) is None:
                        A2[k0, k0] += 2 * dt_n * chic[k0] * bf[d][k0] ** 2 / h[d] ** 2
                c1 = shift(c, d, +1)
                if c1 is None:
                    continue
                k1 = index[c1]
                chif = 2 * chic[k0] * chic[k1] / (chic[k0] + chic[k1])
                bd = 0.5 * (bf[d][k0] + bf[d][k1])
                e = np.zeros(N)
                e[k0], e[k1] = 1.0, -1.0
                A2 += dt_n * chif * bd ** 2 / h[d] ** 2 * np.outer(e, e)
            x = np.linalg.solve(A2, x)
    return x.reshape(shape)


@pytest.mark.parametrize("shape", [(4, 4), (3, 5), (3, 3, 3), (4, 3, 3)])
@pytest.mark.parametrize("limiter", LIMITERS)
def test_dirichlet_brute_force_dense_step(orc, shape, limiter):
    rng = np.random.default_rng(7 * len(shape) + shape[0])
    h = tuple(0.1 + 0.04 * q for q in range(len(shape)))
    b = _random_unit_field(shape, rng)
    chi = np.exp(rng.standard_normal(shape))
    T0 = rng.standard_normal(shape)
    Q = rng.standard_normal(shape)
    dt = 0.02
    g = orc.OracleGrid(b, h, bc="dirichlet", limiter=limiter, chi_par=1.0, chi=chi, src=Q)
    ref = T0
    for _ in range(2):
        ref = _brute_force_dirichlet_step(b, h, limiter, ref, dt, 1.0, chi, Q)
    np.testing.assert_allclose(g.step_si(T0, dt, 2), ref, rtol=1e-12, atol=1e-13)
    ref4 = _brute_force_dirichlet_step(b, h, limiter, T0, dt, 1.0, chi, Q, four_step=True)
    np.testing.assert_allclose(g.step_si(T0, dt, 1, four_step=True), ref4, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("ndim", [2, 3])
def test_dirichlet_sweep_balance(orc, ndim):
    """Interior fluxes telescope: over one sweep along d,
    sum(out - U) = dt_q sum Q - sum over wall cells of 2 alpha_w out_c,
    alpha_w from the wall cell's own b_d and chi."""
    rng = np.random.default_rng(3 + ndim)
    shape = (9, 12) if ndim == 2 else (5, 6, 7)
    nxyz = tuple(reversed(shape))
    h = tuple(1.0 / n for n in nxyz)
    b = _random_unit_field(shape, rng)
    chi = np.exp(0.5 * rng.standard_normal(shape))
    U = 1.0 + rng.random(shape)
    Q = rng.standard_normal(shape)
    cp = 0.05
    g = orc.OracleGrid(b, h, bc="dirichlet", chi_par=1.0, chi_perp=cp, chi=chi, src=Q)
    dt, dtq = 3e-3, 1.7e-3
    for d in range(ndim):
        out = g.sweep3(d, dt, dt, dtq, U)
        ax = ndim - 1 - d
        aw = dt * (cp + (chi - cp) * b[d] ** 2) / h[d] ** 2
        lo = [slice(None)] * ndim
        hi = [slice(None)] * ndim
        lo[ax], hi[ax] = 0, -1
        wall = (2 * aw[tuple(lo)] * out[tuple(lo)]).sum() + (2 * aw[tuple(hi)] * out[tuple(hi)]).sum()
        lhs = (out - U).sum()
        assert abs(lhs - (dtq * Q.sum() - wall)) <= 1e-12 * (abs(wall) + abs(dtq * Q).sum())


def test_perpendicular_numerical_diffusion_converges_second_order(orc):
    """Section 3.2 (smooth test, T = 0 walls, Q = 2 pi^2 cos(pi x) cos(pi y),
    b along the contours of Q, no explicit chi_perp, ncfl = 1000): the
    steady maximum gives chi_perp,num = cos cos / T at that cell; it falls
    close to second order with the grid (ratio near 4 per doubling at the
    finer grids) and does not depend much on ncfl."""
    vals = {}
    for n in (16, 32, 64):
        p = synth.sovinec_problem(n)
        g = orc.OracleGrid(p.b, p.h, bc="dirichlet", chi_par=p.chi_par, src=p.src)
        dt = g.dt_from_ncfl(1000.0)
        T, prev = np.zeros(p.shape), 0.0
        for _ in range(400):
            T = g.step_si(T, dt, 100)
            if abs(T.max() - prev) < 1e-8 * T.max():
                break
            prev = T.max()
        assert abs(T.max() - prev) < 1e-8 * T.max(), n
        i = np.unravel_index(np.argmax(T), T.shape)
        vals[n] = p.meta["psi"][i] / T[i]  # steady state psi / chi_perp,num
    assert 2.0 < vals[16] / vals[32] < 4.5, vals
    assert 3.3 < vals[32] / vals[64] < 4.5, vals
    assert 5e-4 < vals[64] < 3e-3, vals


def test_harmonic_face_chi_is_series_conduction(orc):
    """Harmonic face diffusivity (section 2: a variable chi is averaged
    harmonically at faces) is exact series conduction.  b = x_hat, a per-cell
    chi that jumps by up to 100x from cell to cell, T = 0 walls and a source
    in one column only: in the steady state every source-free stretch of a
    row carries one constant heat flux F, and for a conductivity that is
    constant inside each cell the exact solution drops by F times the two
    half-cell resistances h/(2 chi_i) + h/(2 chi_i+1) between neighbouring
    centres, and by F h/(2 chi) between a wall and its cell.  The fluxes
    leaving the source column on both sides add up to Q h.  An arithmetic
    face mean, or a wall face at a full cell width, fails these."""
    nx, ny, k = 24, 3, 7
    shape = (ny, nx)
    h = (1.0 / nx, 0.25)
    rng = np.random.default_rng(29)
    chi_row = np.exp(rng.uniform(np.log(0.1), np.log(10.0), nx))
    chi = np.tile(chi_row, (ny, 1))
    q = 5.0
    Q = np.zeros(shape)
    Q[:, k] = q
    g = orc.OracleGrid(const_field(shape, (1.0, 0.0)), h, bc="dirichlet", chi_par=1.0, chi=chi, src=Q)
    dt = 1e3
    T = g.step_si(np.zeros(shape), dt, 40)
    T2 = g.step_si(T, dt, 1)
    np.testing.assert_allclose(T2, T, rtol=1e-14, atol=0)  # steady
    hx = h[0]
    for row in T:
        # right of the source: F_R leaves through the right wall
        F_R = row[-1] / (hx / (2 * chi_row[-1]))
        for i in range(k + 1, nx - 1):
            R = hx / (2 * chi_row[i]) + hx / (2 * chi_row[i + 1])
            assert abs((row[i] - row[i + 1]) / R - F_R) <= 1e-12 * abs(F_R)
        # left of the source: F_L leaves through the left wall
        F_L = row[0] / (hx / (2 * chi_row[0]))
        for i in range(0, k - 1):
            R = hx / (2 * chi_row[i]) + hx / (2 * chi_row[i + 1])
            assert abs((row[i + 1] - row[i]) / R - F_L) <= 1e-12 * abs(F_L)
        assert abs(F_L + F_R - q * hx) <= 1e-12 * q * hx
        # the two faces of the source cell carry the same fluxes
        R_k = hx / (2 * chi_row[k]) + hx / (2 * chi_row[k + 1])
        assert abs((row[k] - row[k + 1]) / R_k - F_R) <= 1e-12 * abs(F_R)
    # an arithmetic face mean would give different drops across the stretch
    row = T[0]
    arith = [(row[i] - row[i + 1]) * 0.5 * (chi_row[i] + chi_row[i + 1]) / hx for i in range(k + 1, nx - 1)]
    assert np.ptp(arith) > 1e-2 * abs(np.mean(arith))
