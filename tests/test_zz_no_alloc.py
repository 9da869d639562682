"""The no-allocation entry point (asd_step_semi_implicit_noalloc, static
device scratch) against the workspace entry point (asd_step_semi_implicit)
on the same inputs: two calls in a row, the second on a smaller grid, so
that the second call's kernels run on scratch that the first one filled."""
import numpy as np
import pytest
import torch

import synth
from paper_1008_0861_amd import binding as asd
from tests.gpu_util import TOL, GpuProblem, max_rel_err

pytestmark = pytest.mark.gpu


def _noalloc(p, prec, energy):
    dt = {"f32": torch.float32, "f64": torch.float64}[prec]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        T = torch.from_numpy(p.T0).to(dt).cuda()
        b = [torch.from_numpy(c).to(dt).cuda() for c in p.b]
        e = torch.empty(p.nsteps + 1, dtype=torch.float64, device="cuda") if energy else None
        asd.step_semi_implicit_noalloc(T, b, p.h, p.dt, p.nsteps, bc=p.bc, chi_par=p.chi_par,
                                       chi_perp=p.chi_perp, energy=e, stream=st)
    st.synchronize()
    return T.double().cpu().numpy(), (e.cpu().numpy() if energy else None)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_workspace_entry_point(prec):
    big = synth.grf2d_problem(1024, nsteps=12)
    small = synth.grf2d_problem(200, 136, nsteps=7, chi_perp=1e-3)
    for p in (big, small):
        got, e = _noalloc(p, prec, energy=True)
        ref, eref = GpuProblem(p, prec).run(energy=True)
        err = max_rel_err(got, ref)
        assert err <= TOL[prec], (p.shape, err)
        np.testing.assert_allclose(e, eref, rtol=1e-13, atol=0)


def test_noalloc_refuses_grids_beyond_the_scratch():
    T = torch.zeros((1800, 1800), dtype=torch.float32, device="cuda")
    b = [torch.ones_like(T), torch.zeros_like(T)]
    with pytest.raises(asd.AsdError) as ei:
        asd.step_semi_implicit_noalloc(T, b, (1 / 1800, 1 / 1800), 1e-6, 1)
    assert ei.value.name == "EUNSUPPORTED"
