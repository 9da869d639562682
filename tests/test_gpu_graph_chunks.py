"""Step calls longer than one captured graph (2048 steps): the chunked
replay gives bit for bit the state of direct launches, with and without
per-step outputs, for both schemes."""
import numpy as np
import pytest
import torch

from tests.gpu_util import GpuProblem
from tests.test_gpu_parity import _random_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scheme", ["si", "ex"])
@pytest.mark.parametrize("energy", [False, True])
def test_long_call_chunked_graph_equals_direct(scheme, energy):
    p = _random_problem((24, 40), "periodic", seed=4, ncfl=5.0, nsteps=2 * 2048 + 37)
    dt = p.dt if scheme == "si" else 0.2 * min(p.h) ** 2
    outs = []
    for graphs in (True, False):
        gp = GpuProblem(p, "f64")
        gp.g.set_graphs(graphs)
        r = gp.run(scheme=scheme, dt=dt, energy=energy)
        outs.append(r)
    if energy:
        np.testing.assert_array_equal(outs[0][0], outs[1][0])
        np.testing.assert_array_equal(outs[0][1], outs[1][1])
    else:
        np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("shape,bc", [((64, 96), "periodic"), ((40, 24), "insulating"), ((37, 50), "periodic")])
def test_one_call_equals_single_step_calls(prec, shape, bc):
    """A multi-step call keeps its intermediate states in the workspace
    between steps; single-step calls start from and end in T.  The
    arithmetic is the same, so the states agree bit for bit."""
    p = _random_problem(shape, bc, seed=sum(shape), ncfl=10.0, nsteps=9)
    a = GpuProblem(p, prec)
    a.g.set_graphs(False)
    one = a.run(nsteps=9)
    b = GpuProblem(p, prec)
    b.g.set_graphs(False)
    for _ in range(9):
        many = b.run(nsteps=1)
    np.testing.assert_array_equal(one, many)
