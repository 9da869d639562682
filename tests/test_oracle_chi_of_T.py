"""Pins of the oracle's temperature-dependent diffusivity chi_par(T) =
chi_par (T / T_ref)^p (p = 5/2 in the paper's application, section 3.3),
taken per cell from the state each sweep reads and averaged harmonically at
faces (the per-cell rule of section 2)."""
import itertools

import numpy as np
import pytest

from tests.test_oracle_pins import _random_unit_field


def _brute_force_step_chi_T(b, h, bc, T, dt, chi0, p, tref):
    """Dense assembly of each sweep (section 2) with face chi the harmonic
    mean of chi0 (U/tref)^p of the two cells, U the sweep's input, van Leer
    transverse differences; coordinates from an explicit neighbour table."""
    shape = T.shape
    nd = len(shape)
    nxyz = tuple(reversed(shape))
    N = T.size
    coords = list(itertools.product(*[range(n) for n in reversed(nxyz)]))
    index = {c: k for k, c in enumerate(coords)}

    def vl(a, c):
        return 0.0 if a * c <= 0 else 2 * a * c / (a + c)

    def shift(c, axis, s):
        pos = list(c)
        k = nd - 1 - axis
        m = pos[k] + s
        if m < 0 or m >= nxyz[axis]:
            if bc == "periodic":
                m %= nxyz[axis]
            else:
                return None
        pos[k] = m
        return tuple(pos)

    def val(U, c, axis, s):
        c2 = shift(c, axis, s)
        return U[index[c]] if c2 is None else U[index[c2]]

    x = T.ravel().copy()
    bf = [bb.ravel() for bb in b]
    for d in range(nd):
        U = x.copy()
        chic = chi0 * (U / tref) ** p
        A = np.eye(N)
        S = np.zeros(N)
        for c in coords:
            c1 = shift(c, d, +1)
            if c1 is None:
                continue
            k0, k1 = index[c], index[c1]
            chif = 2 * chic[k0] * chic[k1] / (chic[k0] + chic[k1])
            bface = [0.5 * (bf[q][k0] + bf[q][k1]) for q in range(nd)]
            alpha = dt * chif * bface[d] ** 2 / h[d] ** 2
            e = np.zeros(N)
            e[k0], e[k1] = 1.0, -1.0
            A += alpha * np.outer(e, e)
            F = 0.0
            for t in range(nd):
                if t == d:
                    continue
                p1 = vl(val(U, c1, t, +1) - U[k1], U[k1] - val(U, c1, t, -1))
                p0 = vl(val(U, c, t, +1) - U[k0], U[k0] - val(U, c, t, -1))
                F += dt * chif * bface[d] * bface[t] / (h[d] * h[t]) * vl(p1, p0)
            S += F * e
        x = np.linalg.solve(A, U + S)
    return x.reshape(shape)


@pytest.mark.parametrize("shape", [(4, 5), (3, 3, 4)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_chi_of_T_brute_force_dense_step(orc, shape, bc):
    rng = np.random.default_rng(31 + len(shape))
    h = tuple(0.1 + 0.05 * q for q in range(len(shape)))
    b = _random_unit_field(shape, rng)
    T0 = 0.5 + rng.random(shape)
    dt = 0.03
    g = orc.OracleGrid(b, h, bc=bc, chi_par=0.7, chi_exp=2.5, chi_tref=0.8)
    ref = T0
    for _ in range(3):
        ref = _brute_force_step_chi_T(b, h, bc, ref, dt, 0.7, 2.5, 0.8)
    np.testing.assert_allclose(g.step_si(T0, dt, 3), ref, rtol=1e-12, atol=1e-13)


def test_chi_of_T_is_the_per_cell_rule_with_each_sweeps_input(orc):
    """A chi(T) step equals, sweep by sweep, the per-cell-chi sweep with the
    field chi_par (U / T_ref)^p of that sweep's input U (T^n for x, T* for
    y); likewise the explicit step with the field of T^n."""
    rng = np.random.default_rng(5)
    shape = (14, 18)
    h = (1 / 18, 1 / 14)
    b = _random_unit_field(shape, rng)
    T0 = 0.3 + rng.random(shape)
    chi0, p, tref = 0.9, 2.5, 0.7
    g = orc.OracleGrid(b, h, bc="periodic", chi_par=chi0, chi_exp=p, chi_tref=tref)
    dt = 4e-3
    field = lambda U: chi0 * (U / tref) ** p  # noqa: E731
    gx = orc.OracleGrid(b, h, bc="periodic", chi_par=1.0, chi=field(T0))
    Ts = gx.sweep(0, dt, T0)
    gy = orc.OracleGrid(b, h, bc="periodic", chi_par=1.0, chi=field(Ts))
    T1 = gy.sweep(1, dt, Ts)
    # (agreement to rounding: the C oracle and numpy evaluate the power differently)
    np.testing.assert_allclose(g.step_si(T0, dt, 1), T1, rtol=1e-14, atol=0)
    dte = 0.2 * min(h) ** 2 / float(field(T0).max())
    np.testing.assert_allclose(g.step_explicit(T0, dte, 1), gx.step_explicit(T0, dte, 1), rtol=1e-14, atol=0)


@pytest.mark.parametrize("bc", ["periodic", "insulating"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_chi_of_T_conserves_energy(orc, bc, ndim):
    rng = np.random.default_rng(41 + ndim)
    shape = (13, 17) if ndim == 2 else (5, 7, 6)
    nxyz = tuple(reversed(shape))
    h = tuple(1.0 / n for n in nxyz)
    b = _random_unit_field(shape, rng)
    T0 = 0.2 + rng.random(shape)
    g = orc.OracleGrid(b, h, bc=bc, chi_par=1.0, chi_perp=0.0, chi_exp=2.5, chi_tref=1.0)
    _, e = g.step_si(T0, 50 * min(h) ** 2, 15, energy=True)
    assert np.max(np.abs(e - e[0])) <= 1e-13 * abs(e[0])
    _, e = g.step_si(T0, 50 * min(h) ** 2, 15, energy=True, four_step=True)
    assert np.max(np.abs(e - e[0])) <= 1e-13 * abs(e[0])
    _, e = g.step_explicit(T0, 0.05 * min(h) ** 2, 15, energy=True)
    assert np.max(np.abs(e - e[0])) <= 1e-13 * abs(e[0])


def test_chi_of_T_hot_region_diffuses_faster(orc):
    """Along a uniform field, a small bump on a background of 1 and on a
    background of 2: with chi ~ T^(5/2) the second bump loses its excess
    about 2^(5/2) ~ 5.7 times as fast over a short time (near-linear regime,
    the conductivity set by the background)."""
    n = 128
    shape = (1 + 2, n)
    x = (np.arange(n) + 0.5) / n
    bump = np.exp(-((x - 0.5) / 0.05) ** 2)
    h = (1.0 / n, 1.0 / 3)
    b = (np.ones(shape), np.zeros(shape))
    drops = []
    for base in (1.0, 2.0):
        T0 = np.tile(base * (1.0 + 0.02 * bump), (3, 1))
        g = orc.OracleGrid(b, h, bc="periodic", chi_par=1e-3, chi_exp=2.5, chi_tref=1.0)
        T = g.step_si(T0, 0.01, 2)
        drops.append((T0.max() - T.max()) / (T0.max() - base))
    assert 4.0 < drops[1] / drops[0] < 7.0, drops
