"""Pins of the oracle's 4-step scheme (section 2.1, Eq. 4step):

    T^{n+1} = (1 + dt D_yy/2)^-2 (1 - dt D_yx) (1 + dt D_xx/2)^-2 (1 - dt D_xy) T^n

(and its 3-D analogue), checked against closed forms, a textbook reduction,
an invariant and the paper's statement that it is unconditionally stable in
three dimensions."""
import itertools

import numpy as np
import pytest

from tests.test_oracle_pins import _angles, _coefs, _laplacian_1d, _mode, _random_unit_field, const_field, unit


def _r_sweep4(d, theta, a, beta):
    """Fourier factor of one direction of the 4-step scheme with linear
    averaging and constant b: the transverse numerator of the 2-step r_d
    (dt) over the square of the half-step normal operator,
    (1 + 2 alpha_d sin^2(theta_d/2))^2."""
    num = 1.0
    for (dd, t), bt in beta.items():
        if dd == d:
            num -= bt * np.sin(theta[d]) * np.sin(theta[t])
    return num / (1.0 + 2.0 * a[d] * np.sin(theta[d] / 2.0) ** 2) ** 2


@pytest.mark.parametrize("ncfl", [0.5, 10.0, 1e4])
@pytest.mark.parametrize("chi_perp", [0.0, 0.3])
def test_four_step_2d_one_step_fourier_factor(orc, ncfl, chi_perp):
    rng = np.random.default_rng(int(ncfl * 10) + int(chi_perp * 100) + 1)
    shape = (24, 40)
    h = (1.0 / 40, 1.3 / 24)
    for _ in range(6):
        b = unit(rng.standard_normal(2))
        k = (int(rng.integers(-19, 20)), int(rng.integers(-11, 12)))
        theta = _angles(shape, k)
        dt = ncfl * min(h) ** 2 / 4.0
        g = orc.OracleGrid(const_field(shape, b), h, bc="periodic", limiter="linear", chi_perp=chi_perp)
        T0 = _mode(shape, theta)
        T1 = g.step_si(T0, dt, 1, four_step=True)
        a, beta = _coefs(1.0, chi_perp, b, h, dt)
        r = _r_sweep4(0, theta, a, beta) * _r_sweep4(1, theta, a, beta)
        np.testing.assert_allclose(T1, r * T0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("alpha_max", [0.2, 2.5, 8.0, 50.0])
def test_four_step_3d_one_step_fourier_factor(orc, alpha_max):
    rng = np.random.default_rng(int(alpha_max * 10) + 3)
    shape = (6, 8, 10)
    h = (1 / 10, 1 / 8, 1 / 6)
    for _ in range(4):
        b = unit(rng.standard_normal(3))
        k = tuple(int(rng.integers(-(n // 2) + 1, n // 2)) for n in (10, 8, 6))
        theta = _angles(shape, k)
        dt = alpha_max * min(h) ** 2
        g = orc.OracleGrid(const_field(shape, b), h, bc="periodic", limiter="linear")
        T0 = _mode(shape, theta)
        T1 = g.step_si(T0, dt, 1, four_step=True)
        a, beta = _coefs(1.0, 0.0, b, h, dt)
        r = np.prod([_r_sweep4(d, theta, a, beta) for d in range(3)])
        np.testing.assert_allclose(T1, r * T0, rtol=0, atol=1e-12)


def _max_growth_3d_four_step(alpha, starts):
    from scipy.optimize import minimize

    def neg(p):
        b = unit([np.cos(p[0]) * np.sin(p[1]), np.sin(p[0]) * np.sin(p[1]), np.cos(p[1])])
        th = p[2:5]
        a = [alpha * b[d] ** 2 for d in range(3)]
        beta = {(d, t): alpha * b[d] * b[t] for d in range(3) for t in range(3) if d != t}
        return -abs(np.prod([_r_sweep4(d, th, a, beta) for d in range(3)]))

    best = 0.0
    for s in starts:
        res = minimize(neg, s, method="Nelder-Mead", options=dict(xatol=1e-10, fatol=1e-13, maxiter=20000))
        best = max(best, -res.fun)
    return best


@pytest.mark.parametrize("alpha", [8.25, 12.0, 100.0, 1e4])
def test_four_step_3d_unconditionally_stable(alpha):
    """Section 2.1: the 4-step scheme is unconditionally stable in 3-D (the
    2-step one is limited to chi dt/dx^2 <= 8.25): max |r1 r2 r3| <= 1 at
    chi dt/dx^2 well above that limit, from the 2-step scheme's worst mode
    and from random starts, and on a coarse grid of directions and modes."""
    rng = np.random.default_rng(int(alpha) % 1000 + 17)
    b = unit([-0.358, -0.358, -0.863])
    starts = [np.array([np.arctan2(b[1], b[0]), np.arccos(b[2]), 0.526, 0.526, -0.672])]
    starts += [np.concatenate([rng.uniform(0, 2 * np.pi, 1), rng.uniform(0, np.pi, 1),
                               rng.uniform(-np.pi, np.pi, 3)]) for _ in range(8)]
    assert _max_growth_3d_four_step(alpha, starts) <= 1.0 + 1e-12
    th = np.linspace(-np.pi, np.pi, 25)
    TX, TY, TZ = np.meshgrid(th, th, th, indexing="ij")
    for bb in [unit(rng.standard_normal(3)) for _ in range(40)] + [b]:
        a = [alpha * bb[d] ** 2 for d in range(3)]
        beta = {(d, t): alpha * bb[d] * bb[t] for d in range(3) for t in range(3) if d != t}
        r = np.prod([_r_sweep4(d, (TX, TY, TZ), a, beta) for d in range(3)], axis=0)
        assert np.max(np.abs(r)) <= 1.0 + 1e-12


def test_four_step_3d_oracle_does_not_grow_where_two_step_does(orc):
    """16^3 periodic, linear averaging, b along the 2-step scheme's worst
    direction, chi dt/dx^2 = 12: the mode the 2-step scheme amplifies is
    damped by the 4-step scheme, and a random field does not grow in L2."""
    n = 16
    shape = (n, n, n)
    h = (1.0 / n,) * 3
    b = unit([-0.358, -0.358, -0.863])
    g = orc.OracleGrid(const_field(shape, b), h, limiter="linear")
    dt = 12.0 * h[0] ** 2
    a, beta = _coefs(1.0, 0.0, b, h, dt)
    ks = range(-n // 2 + 1, n // 2)
    worst2, k2 = 0.0, None
    for k in itertools.product(ks, ks, ks):
        th = [2 * np.pi * k[q] / n for q in range(3)]
        from tests.test_oracle_pins import _r_sweep
        r = abs(np.prod([_r_sweep(d, th, a, beta) for d in range(3)]))
        if r > worst2:
            worst2, k2 = r, k
    assert worst2 > 1.0
    theta = _angles(shape, k2)
    T0 = _mode(shape, theta)
    T1 = g.step_si(T0, dt, 1, four_step=True)
    r4 = np.prod([_r_sweep4(d, theta, a, beta) for d in range(3)])
    assert abs(r4) < 1.0
    np.testing.assert_allclose(T1, r4 * T0, atol=1e-12)
    rng = np.random.default_rng(2)
    T = rng.standard_normal(shape)
    norms = [np.linalg.norm(T)]
    for _ in range(4):
        T = g.step_si(T, dt, 1, four_step=True)
        norms.append(np.linalg.norm(T))
    assert all(norms[i + 1] <= norms[i] * (1 + 1e-12) for i in range(4))


@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_four_step_field_along_x_is_two_half_backward_euler_steps(orc, bc):
    """b = x_hat: no transverse terms; each row takes two textbook
    backward-Euler heat steps of dt/2, (1 - chi dt/2 delta_x^2)^-2 T, and
    the y direction is the identity."""
    rng = np.random.default_rng(9)
    shape = (9, 23)
    h = (0.03, 0.05)
    g = orc.OracleGrid(const_field(shape, (1.0, 0.0)), h, bc=bc, chi_par=0.7)
    T0 = rng.standard_normal(shape)
    dt = 0.013
    T1 = g.step_si(T0, dt, 1, four_step=True)
    M = np.eye(23) - 0.7 * (dt / 2) / h[0] ** 2 * _laplacian_1d(23, bc == "periodic")
    ref = np.linalg.solve(M, np.linalg.solve(M, T0.T)).T
    np.testing.assert_allclose(T1, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("bc", ["periodic", "insulating"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_four_step_conserves_energy(orc, bc, ndim):
    rng = np.random.default_rng(21 + ndim)
    shape = (13, 17) if ndim == 2 else (5, 7, 6)
    nxyz = tuple(reversed(shape))
    h = tuple(1.0 / n for n in nxyz)
    b = _random_unit_field(shape, rng)
    chi = np.exp(rng.standard_normal(shape))
    T0 = 1.0 + rng.random(shape)
    g = orc.OracleGrid(b, h, bc=bc, limiter="vanleer", chi_perp=0.01, chi=chi)
    _, e = g.step_si(T0, g.dt_from_ncfl(200.0), 20, energy=True, four_step=True)
    assert np.max(np.abs(e - e[0])) <= 1e-13 * abs(e[0])


def test_four_step_sweep2_splits_as_stated(orc):
    """The 4-step direction update is the generalised sweep with the normal
    part at dt/2 and the transverse part at dt, followed by a pure solve at
    dt/2: composing the two sweeps by hand reproduces one step."""
    rng = np.random.default_rng(4)
    shape = (12, 14)
    h = (1 / 14, 1 / 12)
    b = _random_unit_field(shape, rng)
    g = orc.OracleGrid(b, h, bc="periodic")
    T0 = 1.0 + rng.random(shape)
    dt = g.dt_from_ncfl(30.0)
    x = T0
    for d in range(2):
        x = g.sweep2(d, dt / 2, 0.0, g.sweep2(d, dt / 2, dt, x))
    np.testing.assert_array_equal(x, g.step_si(T0, dt, 1, four_step=True))
    # dt_t = dt_n = dt is the 2-step sweep
    np.testing.assert_array_equal(g.sweep2(0, dt, dt, T0), g.sweep(0, dt, T0))
