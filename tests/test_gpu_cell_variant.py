"""The cell-slot tile body of the sweep (sweep_cell.h) against the oracle:
the same cases as the face-slot body's parity tests, with every sweep
forced onto the cell-slot body (the autotuner chooses between the two per
sweep, so both must hold the parity bars on their own)."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import TOL, GpuProblem, max_rel_err, mixed_rel_err, oracle_run
from tests.test_gpu_parity import _random_problem

pytestmark = pytest.mark.gpu

CELL = 1


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 200), (130, 67), (64, 64), (5, 1000), (300, 7), (12, 20, 33)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_cell_body_ragged_shapes(prec, shape, bc):
    p = _random_problem(shape, bc, seed=sum(shape))
    ref = oracle_run(p, prec)
    got = GpuProblem(p, prec, variant=CELL).run()
    assert max_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("limiter", ["vanleer", "minmod", "mc", "linear"])
@pytest.mark.parametrize("form", ["plain", "chi_perp", "per_cell_chi"])
def test_cell_body_limiters_and_tensor_forms(limiter, form):
    p = _random_problem((72, 90), "periodic", limiter=limiter, chi_perp=1e-3 if form == "chi_perp" else 0.0,
                        per_cell_chi=form == "per_cell_chi", seed=3)
    for prec in ("f64", "f32"):
        ref = oracle_run(p, prec)
        got = GpuProblem(p, prec, variant=CELL).run()
        assert max_rel_err(got, ref) <= TOL[prec], (prec, max_rel_err(got, ref))


@pytest.mark.parametrize("n", [2, 3, 5, 63, 64, 65, 129, 1023, 1025, 4096])
def test_cell_body_line_lengths(n):
    bc = "insulating" if n == 2 else "periodic"
    for shape in ((6, n), (n, 6)):
        p = _random_problem(shape, bc, seed=n, nsteps=3)
        ref = oracle_run(p, "f64")
        got = GpuProblem(p, "f64", variant=CELL).run()
        assert max_rel_err(got, ref) <= TOL["f64"], (shape, max_rel_err(got, ref))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 200), (12, 20, 33), (5, 2)])
@pytest.mark.parametrize("four_step", [False, True])
@pytest.mark.parametrize("source", [False, True])
def test_cell_body_dirichlet_and_source(prec, shape, four_step, source):
    """T = 0 walls (the EXT instantiation), with and without a source, in
    both schemes (the 4-step scheme runs the solve-only and keep-layout
    modes)."""
    p = _random_problem(shape, "insulating", seed=sum(shape) + 3, nsteps=4)
    src = 3.0 * synth.smoothed_normal(shape, sum(shape) + 53, 2.0) if source else None
    p = dataclasses.replace(p, bc="dirichlet", src=src)
    ref = oracle_run(p, prec, four_step=four_step)
    got = GpuProblem(p, prec, four_step=four_step, variant=CELL).run()
    assert mixed_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("four_step", [False, True])
def test_cell_body_reverse_order_and_chi_of_T(prec, four_step):
    p = _random_problem((48, 72), "insulating", seed=23, ncfl=10.0, nsteps=3)
    ref = oracle_run(p, prec, four_step=four_step, reverse=True, chi_exp=2.5, chi_tref=1.5)
    got = GpuProblem(p, prec, four_step=four_step, reverse_order=True, chi_exp=2.5, chi_tref=1.5,
                     variant=CELL).run()
    assert max_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("graphs", [True, False])
def test_cell_body_energy_series(graphs):
    """The FP64 energy of every step, the first entry reduced from the first
    sweep's input by this body."""
    p = _random_problem((48, 40), "periodic", seed=6, nsteps=35)
    ref, eref = oracle_run(p, "f64", energy=True)
    gp = GpuProblem(p, "f64", variant=CELL)
    gp.g.set_graphs(graphs)
    got, e = gp.run(energy=True)
    assert max_rel_err(got, ref) <= TOL["f64"]
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)
    flags, _ = gp.g.status()
    assert flags == 0


@pytest.mark.parametrize("prec,shape", [("f32", (2, 4)), ("f64", (2, 2))])
def test_cell_body_grf_1024_full_size(prec, shape):
    """The 1024^2 workload as configured (100 steps at 20x the Courant step)
    on the cell-slot body in the shape the autotuner picks for it."""
    p = synth.grf2d_problem(1024, nsteps=100)
    ref = oracle_run(p, prec)
    gp = GpuProblem(p, prec)
    for axis in range(2):
        gp.g.set_sweep_config(axis, *shape, 1, CELL)
    got = gp.run()
    err = max_rel_err(got, ref)
    print(f"\ngrf 1024^2 {prec} cell-slot body {shape}: max rel err {err:.3e}")
    assert err <= TOL[prec], err


def test_both_bodies_on_one_problem():
    """Both bodies on one FP64 problem: each within the bar of the oracle
    (their rounding differs: the faces are formed in a different order)."""
    p = _random_problem((96, 160), "periodic", seed=41, nsteps=6)
    ref = oracle_run(p, "f64")
    a = GpuProblem(p, "f64", variant=0).run()
    b = GpuProblem(p, "f64", variant=CELL).run()
    assert max_rel_err(a, ref) <= TOL["f64"] and max_rel_err(b, ref) <= TOL["f64"]
    assert max_rel_err(a, b) <= 2 * TOL["f64"]


@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_cell_body_adjoint_fp64(bc):
    """The adjoint with every sweep on the cell-slot body (its recomputation
    stores T* in both layouts through that body's second store) against
    the reverse-mode reference."""
    from oracle import torch_ref
    from tests.test_gpu_adjoint import AdjGrid, _problem, _rel
    b, T0, chi, h, dt = _problem((40, 56), 3, bc)
    lam = np.random.default_rng(4).standard_normal(T0.shape)
    gT_ref, gC_ref, _ = torch_ref.reverse_gradients(T0, b, chi, h, dt, 7, lam, periodic=bc == "periodic",
                                                    chi_par=float(chi.max()))
    ag = AdjGrid(b, chi, h, "f64", bc=bc)
    for axis in range(2):
        c = ag.g.sweep_config(axis)
        ag.g.set_sweep_config(axis, c["wpl"], c["lpw"], 1, CELL)
    gT, gC = ag.adjoint(T0, lam, dt, 7, 3)
    assert _rel(gT, gT_ref) <= 1e-10
    assert _rel(gC, gC_ref) <= 1e-10
