"""Pins of the reverse-mode reference (oracle/torch_ref.py): its forward
equals the C oracle cell by cell, and its gradients equal central finite
differences of the C oracle, away from limiter kinks."""
import numpy as np
import pytest
import torch

import synth
from oracle import torch_ref

LIMITERS = ["vanleer", "minmod", "mc", "linear"]


def _problem(shape, seed, chi=True):
    ny, nx = shape
    rng = np.random.default_rng(seed)
    v = [synth.smoothed_normal(shape, seed + q, 2.0) + 0.3 * rng.standard_normal() for q in range(2)]
    m = np.sqrt(v[0] ** 2 + v[1] ** 2)
    b = [v[0] / m, v[1] / m]
    T0 = 1.0 + 0.3 * synth.smoothed_normal(shape, seed + 5, 1.5)
    chi_f = np.exp(0.4 * synth.smoothed_normal(shape, seed + 9, 2.0)) if chi else None
    h = (1.0 / nx, 1.2 / ny)
    return b, T0, chi_f, h


@pytest.mark.parametrize("bc", ["periodic", "insulating"])
@pytest.mark.parametrize("limiter", LIMITERS)
def test_torch_forward_matches_c_oracle(orc, bc, limiter):
    b, T0, chi, h = _problem((11, 14), 3)
    dt = 0.7 * min(h) ** 2 * 20
    g = orc.OracleGrid(b, h, bc=bc, limiter=limiter, chi_par=1.0, chi_perp=0.05, chi=chi)
    ref = g.step_si(T0, dt, 4)
    bt = [torch.from_numpy(c) for c in b]
    got = torch_ref.run(torch.from_numpy(T0), bt, torch.from_numpy(chi), h, dt, 4, periodic=bc == "periodic",
                        limiter=limiter, chi_perp=0.05).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def _fd(orc, b, T0, chi, h, dt, nsteps, w, bc, limiter, which, cell, eps):
    def loss(T0v, chiv):
        g = orc.OracleGrid(b, h, bc=bc, limiter=limiter, chi=chiv)
        return float(np.sum(w * g.step_si(T0v, dt, nsteps)))

    def bumped(s):
        T1, c1 = T0.copy(), chi.copy()
        (T1 if which == "T" else c1)[cell] += s
        return loss(T1, c1)

    return (bumped(eps) - bumped(-eps)) / (2 * eps)


@pytest.mark.parametrize("bc", ["periodic", "insulating"])
@pytest.mark.parametrize("limiter", LIMITERS)
def test_torch_gradients_match_central_differences(orc, bc, limiter):
    """L = sum w T_N: dL/dT0 and dL/dchi by autograd against central
    differences of the C oracle.  A cell whose difference quotient changes
    between eps and eps/2 straddles a limiter kink and is skipped."""
    b, T0, chi, h = _problem((10, 12), 7)
    dt = 20 * min(h) ** 2 / 4
    nsteps = 3
    rng = np.random.default_rng(1)
    w = rng.standard_normal(T0.shape)
    gT, gC, _ = torch_ref.reverse_gradients(T0, b, chi, h, dt, nsteps, w, periodic=bc == "periodic",
                                            limiter=limiter)
    checked = 0
    cells = [tuple(rng.integers(0, s) for s in T0.shape) for _ in range(8)]
    for which, grad in (("T", gT), ("chi", gC)):
        for cell in cells:
            e = 1e-5
            f1 = _fd(orc, b, T0, chi, h, dt, nsteps, w, bc, limiter, which, cell, e)
            f2 = _fd(orc, b, T0, chi, h, dt, nsteps, w, bc, limiter, which, cell, e / 2)
            scale = max(abs(f1), 1e-3)
            if abs(f1 - f2) > 1e-6 * scale + 1e-9:
                continue  # kink between the two step sizes
            assert grad[cell] == pytest.approx(f2, rel=1e-6, abs=1e-8), (which, cell)
            checked += 1
    assert checked >= 10


def test_linear_limiter_adjoint_identity():
    """With plain averaging the step is linear, T_N = M T0, so the autograd
    vector-Jacobian product must satisfy <M v, w> = <v, M^T w> exactly."""
    b, T0, chi, h = _problem((9, 13), 11)
    dt = 50 * min(h) ** 2
    rng = np.random.default_rng(2)
    v = rng.standard_normal(T0.shape)
    w = rng.standard_normal(T0.shape)
    bt = [torch.from_numpy(c) for c in b]
    Mv = torch_ref.run(torch.from_numpy(v), bt, torch.from_numpy(chi), h, dt, 3, limiter="linear").numpy()
    MTw, _, _ = torch_ref.reverse_gradients(v, b, chi, h, dt, 3, w, limiter="linear")
    assert np.sum(Mv * w) == pytest.approx(np.sum(v * MTw), rel=1e-12)
