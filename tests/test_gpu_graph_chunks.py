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
