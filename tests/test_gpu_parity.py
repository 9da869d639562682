"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
identical seeded inputs, cell by cell.  FP64 state: 1e-12 relative; FP32
state: 1e-5 relative against the oracle fed the FP32-rounded inputs."""
import numpy as np
import pytest
import torch

import synth
from synth.configs import Problem
from tests.gpu_util import TOL, GpuProblem, max_rel_err, oracle_run

pytestmark = pytest.mark.gpu


def _random_problem(shape, bc, limiter="vanleer", chi_perp=0.0, per_cell_chi=False, ncfl=20.0, nsteps=5,
                    seed=0):
    """Random smooth b field and blob temperature on an arbitrary grid."""
    nd = len(shape)
    if nd == 2:
        ny, nx = shape
        bx, by = synth.grf_unit_field_2d(nx, ny, seed, kmax2=16)
        T0 = synth.blobs_2d(nx, ny, seed + 1, nblobs=4, rmin=0.1, rmax=0.3, width=0.05)
        b = (bx, by)
        h = (1.0 / nx, 1.3 / ny)
    else:
        nz, ny, nx = shape
        rng = np.random.default_rng(seed)
        v = [synth.smoothed_normal(shape, seed + q, 2.0) + 0.3 * rng.standard_normal() for q in range(3)]
        m = np.sqrt(sum(c * c for c in v))
        b = tuple(c / m for c in v)
        T0 = np.exp(0.3 * synth.smoothed_normal(shape, seed + 7, 2.0))
        h = (1.0 / nx, 1.1 / ny, 0.9 / nz)
    chi = synth.chi_field_2d(shape[-1], shape[-2], seed + 3) if (per_cell_chi and nd == 2) else None
    if per_cell_chi and nd == 3:
        chi = np.exp(0.4 * synth.smoothed_normal(shape, seed + 3, 2.0))
    chi_max = 1.0 if chi is None else float(chi.max())
    dt = synth.ncfl_dt(ncfl, h, chi_max)
    if nd == 3:
        dt = min(dt, 6.0 * min(h) ** 2 / chi_max)
    return Problem("rand", b, T0, h, bc=bc, limiter=limiter, chi_par=1.0, chi_perp=chi_perp, chi=chi, dt=dt,
                   nsteps=nsteps)


def test_ring_64_fp64_200_steps():
    """The 64^2 ring (T = 12 in the patch, 10 elsewhere), insulating walls,
    200 steps at 10x the explicit step, FP64: every cell and the energy
    series within 1e-12 of the oracle."""
    p = synth.ring_problem(n=64)
    ref, eref = oracle_run(p, "f64", energy=True)
    got, e = GpuProblem(p, "f64").run(energy=True)
    assert max_rel_err(got, ref) <= TOL["f64"]
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 200), (130, 67), (64, 64), (5, 1000), (300, 7)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_si_2d_ragged_shapes(prec, shape, bc):
    p = _random_problem(shape, bc, seed=sum(shape))
    ref = oracle_run(p, prec)
    got = GpuProblem(p, prec).run()
    assert max_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("limiter", ["vanleer", "minmod", "mc", "linear"])
@pytest.mark.parametrize("variant", ["plain", "chi_perp", "per_cell_chi"])
def test_si_2d_limiters_and_tensor_forms(limiter, variant):
    p = _random_problem((72, 90), "periodic", limiter=limiter, chi_perp=1e-3 if variant == "chi_perp" else 0.0,
                        per_cell_chi=variant == "per_cell_chi", seed=3)
    for prec in ("f64", "f32"):
        ref = oracle_run(p, prec)
        got = GpuProblem(p, prec).run()
        assert max_rel_err(got, ref) <= TOL[prec], (prec, max_rel_err(got, ref))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 31, 63, 64, 65, 127, 129, 1000, 1023, 1025, 2048, 4096])
def test_si_line_lengths(n):
    """Line lengths around every segment/lane boundary of the line solver,
    on both axes (n x 6 and 6 x n), insulating for n = 2, else periodic."""
    bc = "insulating" if n == 2 else "periodic"
    for shape in ((6, n), (n, 6)):
        p = _random_problem(shape, bc, seed=n, nsteps=3)
        ref = oracle_run(p, "f64")
        got = GpuProblem(p, "f64").run()
        assert max_rel_err(got, ref) <= TOL["f64"], (shape, max_rel_err(got, ref))


@pytest.mark.parametrize("prec,shape", [("f32", (5, 16109)), ("f32", (16109, 5)), ("f32", (4, 16384)),
                                        ("f64", (5, 4096)), ("f64", (3, 4, 4096)), ("f64", (4096, 3, 4)),
                                        ("f32", (3, 16109, 4)), ("f32", (3, 4, 16109))])
def test_si_longest_lines(prec, shape):
    """The longest lines the LDS holds (16109 cells in FP32, and 16384;
    4096 in FP64), on each axis in turn."""
    p = _random_problem(shape, "periodic", ncfl=10.0, seed=sum(shape), nsteps=2)
    ref = oracle_run(p, prec)
    got = GpuProblem(p, prec).run()
    assert max_rel_err(got, ref) <= TOL[prec], (shape, max_rel_err(got, ref))


@pytest.mark.parametrize("case", ["b_x", "b_y", "b_diag", "isotropic", "b_z_3d"])
@pytest.mark.parametrize("scheme", ["si", "ex"])
def test_degenerate_fields(case, scheme):
    """Degenerate cases of the operator, FP64, against the oracle: b along a
    grid axis (the transverse terms vanish; with b = x every row diffuses on
    its own and the y sweep is the identity), b along a diagonal, isotropic
    diffusion (chi_perp = chi_par) and b = z in 3-D."""
    rng = np.random.default_rng(11)
    shape = (8, 12, 16) if case == "b_z_3d" else (36, 44)
    T0 = 1.0 + 0.5 * rng.random(shape)
    one, zero = np.ones(shape), np.zeros(shape)
    b = {"b_x": (one, zero), "b_y": (zero, one), "b_diag": (one / np.sqrt(2), one / np.sqrt(2)),
         "isotropic": (one / np.sqrt(2), one / np.sqrt(2)), "b_z_3d": (zero, zero, one)}[case]
    h = (1.0 / shape[-1],) * len(shape)
    chi_perp = 1.0 if case == "isotropic" else 0.0
    ncfl = 0.2 if scheme == "ex" else 8.0
    dt = synth.ncfl_dt(ncfl, h, 1.0)
    p = Problem(case, b, T0, h, bc="periodic", chi_par=1.0, chi_perp=chi_perp, dt=dt, nsteps=4)
    ref = oracle_run(p, "f64", scheme=scheme)
    got = GpuProblem(p, "f64").run(scheme=scheme)
    assert max_rel_err(got, ref) <= TOL["f64"], max_rel_err(got, ref)
    if case == "b_x":
        # no coupling between rows: each row's sum is conserved on its own
        np.testing.assert_allclose(got.sum(axis=1), T0.sum(axis=1), rtol=1e-13)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("scheme", ["si", "ex"])
def test_zero_steps(prec, scheme):
    """nsteps = 0 leaves T bit for bit and reports the initial energy (the
    oracle's FP64 sum of the same rounded state); the series call returns
    the one row (E0, min T, max T)."""
    p = _random_problem((40, 50), "periodic", seed=9)
    dt = p.dt if scheme == "si" else p.dt / 40
    ref, eref = oracle_run(p, prec, nsteps=0, scheme=scheme, dt=dt, energy=True)
    gp = GpuProblem(p, prec)
    got, e = gp.run(nsteps=0, scheme=scheme, dt=dt, energy=True)
    assert np.array_equal(got, ref)
    assert e.shape == (1,)
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)
    with torch.cuda.stream(gp.stream):
        ser = gp.g.step_series(scheme, dt, 0)
    gp.stream.synchronize()
    ser = ser.cpu().numpy()
    assert ser.shape == (1, 3)
    np.testing.assert_allclose(ser[0], [eref[0], ref.min(), ref.max()], rtol=1e-13, atol=0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(9, 13, 21), (20, 24, 17), (3, 40, 5)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_si_3d(prec, shape, bc):
    p = _random_problem(shape, bc, ncfl=10.0, seed=len(shape) + shape[0], nsteps=4)
    ref = oracle_run(p, prec)
    got = GpuProblem(p, prec).run()
    assert max_rel_err(got, ref) <= TOL[prec]


def test_si_3d_per_cell_chi_and_chi_perp():
    p = _random_problem((12, 14, 16), "periodic", chi_perp=1e-2, per_cell_chi=True, ncfl=8.0, seed=5)
    ref = oracle_run(p, "f64")
    got = GpuProblem(p, "f64").run()
    assert max_rel_err(got, ref) <= TOL["f64"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 200), (64, 64), (9, 13, 21), (16, 16, 16)])
@pytest.mark.parametrize("bc", ["periodic", "insulating"])
def test_explicit_parity(prec, shape, bc):
    p = _random_problem(shape, bc, seed=11, nsteps=7)
    dt = synth.ncfl_dt(1.0 if len(shape) == 2 else 0.8, p.h, 1.0)
    ref = oracle_run(p, prec, scheme="ex", dt=dt)
    got = GpuProblem(p, prec).run(scheme="ex", dt=dt)
    assert max_rel_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("scheme", ["si", "ex"])
@pytest.mark.parametrize("graphs", [True, False])
def test_energy_series_across_fold_batches(scheme, graphs):
    """75 steps: the per-step energies are folded in batches of up to 32
    steps (two full batches and a remainder); every entry matches the
    oracle's FP64 energy, on the captured-graph and on the eager path."""
    p = _random_problem((48, 40), "insulating", seed=5, nsteps=75)
    dt = p.dt if scheme == "si" else synth.ncfl_dt(1.0, p.h, 1.0)
    _, eref = oracle_run(p, "f64", scheme=scheme, dt=dt, energy=True)
    gp = GpuProblem(p, "f64")
    gp.g.set_graphs(graphs)
    _, e = gp.run(scheme=scheme, dt=dt, energy=True)
    assert e.shape == (76,)
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("nsteps", [1, 2, 30, 31, 32, 33, 70])
def test_energy_entry_zero_folded_with_the_steps(nsteps):
    """Square grid, both sweeps with the same block count: the initial
    state's partials (reduced by the first sweep from its input) share ring
    slot 0 with the steps' and are folded with them; every fold length
    around the ring's capacity (32 entries) gives the oracle's energies, no
    status flag, and the series (E, min, max) of every state."""
    p = _random_problem((64, 64), "periodic", seed=12, nsteps=nsteps)
    _, eref = oracle_run(p, "f64", energy=True)
    gp = GpuProblem(p, "f64")
    for axis in range(2):
        gp.g.set_sweep_config(axis, 1, 4)
    _, e = gp.run(energy=True)
    np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)
    with torch.cuda.stream(gp.stream):
        flags, stats = gp.g.status()
    assert flags == 0
    np.testing.assert_allclose(stats[0], eref[-1], rtol=1e-13)
    gs = GpuProblem(p, "f64")
    with torch.cuda.stream(gs.stream):
        series = gs.g.step_series("si", p.dt, nsteps)
    gs.stream.synchronize()
    np.testing.assert_allclose(series.cpu().numpy()[:, 0], eref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("limiter", ["vanleer", "minmod", "mc", "linear"])
def test_explicit_limiters_per_cell_chi(limiter):
    p = _random_problem((50, 70), "insulating", limiter=limiter, per_cell_chi=True, chi_perp=1e-3, seed=2)
    dt = synth.ncfl_dt(1.0, p.h, float(p.chi.max()))
    ref = oracle_run(p, "f64", scheme="ex", dt=dt, nsteps=6)
    got = GpuProblem(p, "f64").run(scheme="ex", dt=dt, nsteps=6)
    assert max_rel_err(got, ref) <= TOL["f64"]


@pytest.mark.parametrize("chi_perp", [0.0, 1e-3])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_grf_1024_full_size(prec, chi_perp):
    """The 1024^2 periodic random-field workload as configured (100 steps at
    20x the Courant step, chi_perp 0 and 1e-3, FP64 and FP32) against the
    oracle cell by cell, in the default launch shape and in the shapes the
    autotuner picks for the benchmark (2 waves per line, 4 lines per block in
    FP32; 2 and 2 in FP64)."""
    p = synth.grf2d_problem(1024, nsteps=100, chi_perp=chi_perp)
    ref = oracle_run(p, prec)
    shapes = [None, (2, 4) if prec == "f32" else (2, 2)]
    for shape in shapes:
        gp = GpuProblem(p, prec)
        if shape is not None:
            for axis in range(2):
                gp.g.set_sweep_config(axis, *shape)
            assert gp.g.sweep_config(0)["wpl"] == shape[0] and gp.g.sweep_config(0)["lpw"] == shape[1]
        got = gp.run()
        err = max_rel_err(got, ref)
        print(f"\ngrf 1024^2 {prec} chi_perp {chi_perp:g} 100 steps shape {shape}: max rel err {err:.3e}")
        assert err <= TOL[prec], (shape, err)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_explicit_1024_full_size(prec):
    """The explicit limited step on the 1024^2 workload at ncfl = 1, as the
    benchmark runs it, against the oracle for 20 steps."""
    p = synth.grf2d_problem(1024, nsteps=20)
    dt = synth.ncfl_dt(1.0, p.h, 1.0)
    ref = oracle_run(p, prec, scheme="ex", dt=dt)
    got = GpuProblem(p, prec).run(scheme="ex", dt=dt)
    assert max_rel_err(got, ref) <= TOL[prec], max_rel_err(got, ref)


def test_curl3d_256_full_size_tuned():
    """The 256^3 FP32 3-D workload at full size, 2 steps, in the launch shapes
    the autotuner picks (as the benchmark does), against the oracle."""
    p = synth.curl3d_problem(256, nsteps=2, ncfl=10.0)
    ref = oracle_run(p, "f32")
    gp = GpuProblem(p, "f32")
    with torch.cuda.stream(gp.stream):
        gp.g.tune(p.dt, reps=2)
        gp.T.copy_(torch.from_numpy(p.T0).float())
    gp.stream.synchronize()
    got = gp.run()
    assert max_rel_err(got, ref) <= TOL["f32"], max_rel_err(got, ref)


def test_energy_conserved_and_deterministic_100_steps():
    """FP32 state, 100 steps at 1024^2 in the benchmark's launch shape (2
    waves per line, 4 lines per block): the FP64 energy series stays at its
    initial value to FP32 rounding, and two runs are bitwise equal."""
    p = synth.grf2d_problem(1024, nsteps=100)
    runs = []
    for _ in range(2):
        gp = GpuProblem(p, "f32")
        for axis in range(2):
            gp.g.set_sweep_config(axis, 2, 4)
        runs.append(gp.run(energy=True))
    (a, ea), (b, eb) = runs
    assert np.array_equal(a, b) and np.array_equal(ea, eb)
    assert np.max(np.abs(ea - ea[0])) <= 2e-6 * abs(ea[0])


def test_graph_and_eager_paths_agree():
    p = synth.grf2d_problem(256, nsteps=12)
    g1 = GpuProblem(p, "f32")
    g1.g.set_graphs(True)  # capture the 12-step calls (the default launches them directly)
    g2 = GpuProblem(p, "f32")
    g2.g.set_graphs(False)
    a = g1.run()
    b = g2.run()
    assert np.array_equal(a, b)
    # replay the cached graph three more times, with eager work in between
    for _ in range(3):
        a = g1.run(nsteps=12)
        b = g2.run(nsteps=12)
        torch.cuda.synchronize()
        assert np.array_equal(a, b)


def test_default_graph_mode_captures_long_calls_only():
    """The default mode launches a short call directly and replays a captured
    graph for a call of 64 steps or more; both agree with the eager path bit
    for bit, the long call also on replays with eager work in between."""
    p = synth.grf2d_problem(256, nsteps=70)
    auto = GpuProblem(p, "f32")
    eager = GpuProblem(p, "f32")
    eager.g.set_graphs(False)
    for n in (12, 70, 70, 70):
        a = auto.run(nsteps=n)
        b = eager.run(nsteps=n)
        torch.cuda.synchronize()
        assert np.array_equal(a, b), n


def test_launch_shapes_agree():
    """Every admissible launch shape gives the oracle's result."""
    p = _random_problem((40, 256), "periodic", seed=9, nsteps=3)
    ref = oracle_run(p, "f64")
    for wpl in (1, 2, 4):
        for lpw in (1, 2, 4):
            gp = GpuProblem(p, "f64")
            try:
                gp.g.set_sweep_config(0, wpl, lpw)
            except Exception:
                continue
            got = gp.run()
            assert max_rel_err(got, ref) <= TOL["f64"], (wpl, lpw)


def test_tuner_keeps_results():
    p = synth.grf2d_problem(512, nsteps=5)
    ref = oracle_run(p, "f32")
    gp = GpuProblem(p, "f32")
    with torch.cuda.stream(gp.stream):
        cfgs = gp.g.tune(p.dt, reps=3)
    assert len(cfgs) == 2
    got = gp.run()
    assert max_rel_err(got, ref) <= TOL["f32"]


def test_status_flags():
    p = synth.ring_problem(n=64, nsteps=5)
    gp = GpuProblem(p, "f64")
    gp.run(energy=True)
    with torch.cuda.stream(gp.stream):
        flags, stats = gp.g.status()
    assert flags == 0
    assert stats[1] >= 10.0 - 1e-9 and stats[2] <= 12.0 + 1e-9
    # a negative temperature is reported
    with torch.cuda.stream(gp.stream):
        gp.T[3, 3] = -1.0
        flags, stats = gp.g.status()
    assert flags & 2 and stats[1] == -1.0
