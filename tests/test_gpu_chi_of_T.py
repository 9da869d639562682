"""Temperature-dependent diffusivity chi_par(T) = chi_par (T / T_ref)^p on
the GPU (chi ~ T^(5/2), section 3.3) against the oracle: per cell from the
state each sweep (or explicit step) reads, harmonic mean at faces."""
import numpy as np
import pytest

from tests.gpu_util import TOL, GpuProblem, max_rel_err, oracle_run
from tests.test_gpu_parity import _random_problem

pytestmark = pytest.mark.gpu

P_EXP, T_REF = 2.5, 1.5


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 200), (64, 64), (130, 67), (12, 20, 33)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
@pytest.mark.parametrize("four_step", [False, True])
def test_chi_of_T_semi_implicit_matches_oracle(prec, shape, bc, four_step):
    p = _random_problem(shape, bc, seed=sum(shape) + 11, ncfl=10.0, nsteps=4)
    ref = oracle_run(p, prec, four_step=four_step, chi_exp=P_EXP, chi_tref=T_REF)
    assert np.all(np.isfinite(ref)) and ref.min() > 0
    got = GpuProblem(p, prec, four_step=four_step, chi_exp=P_EXP, chi_tref=T_REF).run()
    assert max_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("four_step", [False, True])
def test_chi_of_T_reverse_order_matches_oracle(prec, four_step):
    p = _random_problem((48, 72), "insulating", seed=23, ncfl=10.0, nsteps=3)
    ref = oracle_run(p, prec, four_step=four_step, reverse=True, chi_exp=P_EXP, chi_tref=T_REF)
    got = GpuProblem(p, prec, four_step=four_step, reverse_order=True, chi_exp=P_EXP, chi_tref=T_REF).run()
    assert max_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(40, 56), (9, 14, 22)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_chi_of_T_explicit_matches_oracle(prec, shape, bc):
    p = _random_problem(shape, bc, seed=sum(shape) + 2, nsteps=6)
    chi_max = p.chi_par * (float(p.T0.max()) / T_REF) ** P_EXP
    dt = 0.2 * min(p.h) ** 2 / chi_max
    ref = oracle_run(p, prec, scheme="ex", dt=dt, chi_exp=P_EXP, chi_tref=T_REF)
    got = GpuProblem(p, prec, chi_exp=P_EXP, chi_tref=T_REF).run(scheme="ex", dt=dt)
    assert max_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("scheme", ["si", "ex"])
def test_chi_of_T_energy_and_paths(graphs, scheme):
    """Many steps through both launch paths (captured graph, eager): state
    and per-step energy equal the oracle's; the energy is conserved."""
    p = _random_problem((48, 40), "insulating", seed=8, ncfl=10.0, nsteps=37)
    dt = p.dt
    if scheme == "ex":
        dt = 0.2 * min(p.h) ** 2 / (p.chi_par * (float(p.T0.max()) / T_REF) ** P_EXP)
    ref, eref = oracle_run(p, "f64", scheme=scheme, dt=dt, energy=True, chi_exp=P_EXP, chi_tref=T_REF)
    gp = GpuProblem(p, "f64", chi_exp=P_EXP, chi_tref=T_REF)
    gp.g.set_graphs(graphs)
    got, e = gp.run(scheme=scheme, dt=dt, energy=True)
    assert max_rel_err(got, ref) <= TOL["f64"]
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)
    assert np.max(np.abs(e - e[0])) <= 1e-12 * abs(e[0])



def test_chi_of_T_refused_by_adjoint():
    import torch

    from paper_1008_0861_amd import binding as asd
    p = _random_problem((32, 32), "periodic", seed=1)
    gp = GpuProblem(p, "f64", chi_exp=P_EXP, chi_tref=T_REF)
    T0 = gp.T.clone()
    lam = torch.ones_like(T0)
    with pytest.raises(asd.AsdError) as ei:
        gp.g.adjoint(p.dt, 2, 1, T0, lam, grad_chi=False)
    assert ei.value.name == "EUNSUPPORTED"
