"""T = 0 walls and the source term on the GPU (section 3.2) against the
oracle, and the perpendicular numerical diffusivity of the smooth test."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
from oracle import oracle
from paper_1008_0861_amd import binding as asd
from tests.gpu_util import TOL, GpuProblem, max_rel_err, mixed_rel_err, oracle_run
from tests.test_gpu_parity import _random_problem

pytestmark = pytest.mark.gpu


def _dirichlet(shape, seed, source=True, per_cell_chi=False, nsteps=4, ncfl=20.0, chi_perp=0.0, limiter="vanleer"):
    p = _random_problem(shape, "insulating", seed=seed, ncfl=ncfl, nsteps=nsteps, per_cell_chi=per_cell_chi,
                        chi_perp=chi_perp, limiter=limiter)
    src = None
    if source:
        src = 3.0 * synth.smoothed_normal(shape, seed + 50, 2.0)
    return dataclasses.replace(p, bc="dirichlet", src=src)


_mixed_err = mixed_rel_err


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 200), (64, 64), (130, 67), (12, 20, 33), (2, 9), (5, 2)])
@pytest.mark.parametrize("four_step", [False, True])
@pytest.mark.parametrize("source", [False, True])
def test_dirichlet_semi_implicit_matches_oracle(prec, shape, four_step, source):
    p = _dirichlet(shape, seed=sum(shape) + 3, source=source)
    ref = oracle_run(p, prec, four_step=four_step)
    got = GpuProblem(p, prec, four_step=four_step).run()
    assert _mixed_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("limiter", ["minmod", "mc", "linear"])
def test_dirichlet_limiters_chi_field_chi_perp(prec, limiter):
    p = _dirichlet((40, 56), seed=9, per_cell_chi=True, chi_perp=0.05, limiter=limiter)
    ref = oracle_run(p, prec)
    got = GpuProblem(p, prec).run()
    assert _mixed_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(40, 56), (9, 14, 22), (3, 70)])
@pytest.mark.parametrize("source", [False, True])
def test_dirichlet_explicit_matches_oracle(prec, shape, source):
    p = _dirichlet(shape, seed=sum(shape), source=source, nsteps=6)
    dt = 0.2 * min(p.h) ** 2 / p.chi_par
    ref = oracle_run(p, prec, scheme="ex", dt=dt)
    got = GpuProblem(p, prec).run(scheme="ex", dt=dt)
    assert _mixed_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("four_step", [False, True])
def test_dirichlet_with_chi_of_T(four_step):
    p = _dirichlet((48, 72), seed=3, ncfl=10.0, nsteps=6)
    p = dataclasses.replace(p, src=np.full(p.shape, 5.0))
    ref = oracle_run(p, "f64", four_step=four_step, chi_exp=2.5, chi_tref=1.5)
    assert np.all(np.isfinite(ref)) and ref.min() > 0
    got = GpuProblem(p, "f64", four_step=four_step, chi_exp=2.5, chi_tref=1.5).run()
    assert max_rel_err(got, ref) <= TOL["f64"]


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("scheme", ["si", "ex"])
def test_dirichlet_energy_series_and_no_drift_flag(graphs, scheme):
    """Per-step energy (not conserved: wall outflow and source) equals the
    oracle's; the status call raises no energy-drift flag."""
    p = _dirichlet((48, 40), seed=8, nsteps=37)
    dt = p.dt if scheme == "si" else 0.2 * min(p.h) ** 2 / p.chi_par
    ref, eref = oracle_run(p, "f64", scheme=scheme, dt=dt, energy=True)
    gp = GpuProblem(p, "f64")
    gp.g.set_graphs(graphs)
    got, e = gp.run(scheme=scheme, dt=dt, energy=True)
    assert _mixed_err(got, ref) <= TOL["f64"]
    np.testing.assert_allclose(e, eref, rtol=1e-12, atol=1e-14 * np.abs(eref).max())
    assert abs(e[-1] - e[0]) > 1e-3 * abs(e[0])
    with torch.cuda.stream(gp.stream):
        flags, _ = gp.g.status()
    assert not flags & asd.STATUS_ENERGY_DRIFT


def test_source_needs_forward_order():
    p = _dirichlet((16, 16), seed=1)
    gp = GpuProblem(p, "f64", reverse_order=True)
    with pytest.raises(asd.AsdError) as ei:
        gp.run()
    assert ei.value.name == "EUNSUPPORTED"


def _sovinec_gpu(n, nsteps_chunk, max_chunks, ncfl=1000.0, tol=1e-9):
    """Smooth test to steady state on the GPU (FP64): returns
    (chi_perp,num, steps, T)."""
    p = synth.sovinec_problem(n, ncfl=ncfl)
    gp = GpuProblem(p, "f64")
    prev, steps = 0.0, 0
    for _ in range(max_chunks):
        gp.run(nsteps=nsteps_chunk)
        steps += nsteps_chunk
        with torch.cuda.stream(gp.stream):
            _, (_, _, tmax) = gp.g.status()
        if abs(tmax - prev) < tol * tmax:
            break
        prev = tmax
    T = gp.T.double().cpu().numpy()
    i = np.unravel_index(np.argmax(T), T.shape)
    return p.meta["psi"][i] / T[i], steps, T


@pytest.mark.parametrize("n", [16, 32])
def test_sovinec_matches_oracle_at_equal_steps(n):
    p = synth.sovinec_problem(n)
    nsteps = 600
    ref = oracle.OracleGrid(p.b, p.h, bc="dirichlet", chi_par=p.chi_par, src=p.src).step_si(p.T0, p.dt, nsteps)
    got = GpuProblem(p, "f64").run(nsteps=nsteps)
    assert _mixed_err(got, ref) <= 1e-11


def test_sovinec_chi_perp_num_second_order():
    """Section 3.2: chi_perp,num / chi_par from the steady maximum falls
    close to second order with the grid at ncfl = 1000 (ratio ~4 per
    doubling at 64 -> 128)."""
    c64, _, _ = _sovinec_gpu(64, 1000, 60)
    c128, s128, _ = _sovinec_gpu(128, 5000, 120)
    assert 5e-4 < c64 < 3e-3, c64
    assert 3.3 < c64 / c128 < 4.5, (c64, c128, s128)
