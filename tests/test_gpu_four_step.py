"""The 4-step scheme (section 2.1, Eq. 4step) on the GPU against the
oracle's, cell by cell, on the same seeded inputs."""
import numpy as np
import pytest
import torch

import synth
from paper_1008_0861_amd import binding as asd
from tests.gpu_util import TOL, GpuProblem, max_rel_err, oracle_run
from tests.test_gpu_parity import _random_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 200), (64, 64), (130, 67), (9, 13, 21), (16, 16, 16)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_four_step_matches_oracle(prec, shape, bc):
    p = _random_problem(shape, bc, seed=sum(shape) + 1, nsteps=4, ncfl=60.0 if len(shape) == 2 else 20.0)
    ref = oracle_run(p, prec, four_step=True)
    got = GpuProblem(p, prec, four_step=True).run()
    assert max_rel_err(got, ref) <= TOL[prec]


def test_four_step_energy_series_fp64():
    p = _random_problem((48, 40), "periodic", seed=8, nsteps=40, ncfl=100.0)
    _, eref = oracle_run(p, "f64", four_step=True, energy=True)
    _, e = GpuProblem(p, "f64", four_step=True).run(energy=True)
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)


def test_four_step_3d_runs_beyond_the_two_step_limit():
    """chi dt/dx^2 = 12 in 3-D: the 2-step grid refuses the step
    (EUNSTABLE, section 2.1), the 4-step grid takes it and matches the
    oracle, with the FP64 energy conserved."""
    n = 24
    p = _random_problem((n, n, n), "periodic", seed=12, nsteps=6)
    p.dt = 12.0 * min(p.h) ** 2 / p.chi_par
    two = GpuProblem(p, "f64")
    with pytest.raises(asd.AsdError) as ei:
        two.run()
    assert ei.value.name == "EUNSTABLE"
    ref, eref = oracle_run(p, "f64", four_step=True, energy=True)
    got, e = GpuProblem(p, "f64", four_step=True).run(energy=True)
    assert max_rel_err(got, ref) <= TOL["f64"]
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)


def test_four_step_graph_and_eager_agree():
    p = synth.grf2d_problem(128, nsteps=9)
    g1 = GpuProblem(p, "f32", four_step=True)
    g2 = GpuProblem(p, "f32", four_step=True)
    g2.g.set_graphs(False)
    a = g1.run()
    b = g2.run()
    assert np.array_equal(a, b)
    ref = oracle_run(p, "f32", four_step=True)
    assert max_rel_err(a, ref) <= TOL["f32"]


def test_four_step_refused_by_adjoint_and_batch():
    p = synth.adjoint_problem(n=32, nsteps=2)
    gp = GpuProblem(p, "f64", four_step=True)
    T0 = gp.T.clone()
    lam = torch.ones_like(T0)
    with pytest.raises(asd.AsdError) as ei:
        gp.g.adjoint(p.dt, 2, 1, T0, lam)
    assert ei.value.name == "EUNSUPPORTED"
