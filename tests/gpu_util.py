"""Helpers for the GPU tests: run a synthetic problem through the C ABI and
through the oracle on identical inputs."""
import numpy as np
import torch

from oracle import oracle
from paper_1008_0861_amd import binding as asd

DT = {"f32": torch.float32, "f64": torch.float64}
NP = {"f32": np.float32, "f64": np.float64}

# parity bars (relative, per cell): FP64 state 1e-12; FP32 state 1e-5 against
# the FP64 oracle fed the FP32-rounded inputs
TOL = {"f64": 1e-12, "f32": 1e-5}


def rounded(p, prec):
    """Inputs as the GPU sees them, back in float64 for the oracle."""
    r = lambda a: None if a is None else a.astype(NP[prec]).astype(np.float64)  # noqa: E731
    return [r(c) for c in p.b], r(p.T0), r(p.chi)


def rounded_src(p, prec):
    src = getattr(p, "src", None)
    return None if src is None else src.astype(NP[prec]).astype(np.float64)


def oracle_run(p, prec, nsteps=None, scheme="si", dt=None, energy=False, four_step=False, reverse=False,
               chi_exp=0.0, chi_tref=1.0):
    b, T0, chi = rounded(p, prec)
    g = oracle.OracleGrid(b, p.h, bc=p.bc, limiter=p.limiter, chi_par=p.chi_par, chi_perp=p.chi_perp, chi=chi,
                          chi_exp=chi_exp, chi_tref=chi_tref, src=rounded_src(p, prec))
    nsteps = p.nsteps if nsteps is None else nsteps
    dt = p.dt if dt is None else dt
    if scheme == "si":
        return g.step_si(T0, dt, nsteps, energy=energy, four_step=four_step, reverse=reverse)
    return g.step_explicit(T0, dt, nsteps, energy=energy)


def stored_oracle_run(p, prec, nsteps=None, rounding_seed=None):
    """The oracle on the inputs the GPU sees, with its state rounded to the
    GPU's storage type after every sweep (oracle.OracleGrid.step_si_stored;
    rounding_seed: faithful rounding in seeded random directions)."""
    b, T0, chi = rounded(p, prec)
    g = oracle.OracleGrid(b, p.h, bc=p.bc, limiter=p.limiter, chi_par=p.chi_par, chi_perp=p.chi_perp, chi=chi)
    nsteps = p.nsteps if nsteps is None else nsteps
    return g.step_si_stored(T0, p.dt, nsteps, store=NP[prec], rounding_seed=rounding_seed)


class GpuProblem:
    """A problem resident on the GPU, advanced on a private stream."""

    def __init__(self, p, prec, stream=None, allow_unstable=False, four_step=False, reverse_order=False,
                 chi_exp=0.0, chi_tref=1.0, variant=None):
        self.p = p
        self.prec = prec
        self.stream = stream or torch.cuda.Stream()
        dt = DT[prec]
        chi_par = p.chi_par if p.chi is None else float(max(p.chi.max(), p.chi_par))
        with torch.cuda.stream(self.stream):
            self.g = asd.Grid(p.shape, p.h, bc=p.bc, dtype=dt, limiter=p.limiter, chi_par=chi_par,
                              chi_perp=p.chi_perp, per_cell_chi=p.chi is not None,
                              allow_unstable=allow_unstable, four_step=four_step, reverse_order=reverse_order,
                              chi_exp=chi_exp, chi_tref=chi_tref)
            self.b = [torch.from_numpy(c).to(dt).cuda() for c in p.b]
            self.T = torch.from_numpy(p.T0).to(dt).cuda()
            self.g.set_b(*self.b)
            self.g.set_field("T", self.T)
            if p.chi is not None:
                self.chi = torch.from_numpy(p.chi).to(dt).cuda()
                self.g.set_field("chi", self.chi)
            if getattr(p, "src", None) is not None:
                self.Q = torch.from_numpy(p.src).to(dt).cuda()
                self.g.set_field("Q", self.Q)
        if variant is not None:
            # every sweep on the given tile body, in its default shape with io = 1
            for axis in range(len(p.shape)):
                c = self.g.sweep_config(axis)
                self.g.set_sweep_config(axis, c["wpl"], c["lpw"], 1, variant)
                assert self.g.sweep_config(axis)["variant"] == variant

    def run(self, nsteps=None, scheme="si", dt=None, energy=False):
        nsteps = self.p.nsteps if nsteps is None else nsteps
        dt = self.p.dt if dt is None else dt
        with torch.cuda.stream(self.stream):
            f = self.g.step_semi_implicit if scheme == "si" else self.g.step_explicit
            e = f(dt, nsteps, energy=energy)
        self.stream.synchronize()
        out = self.T.double().cpu().numpy()
        return (out, e.cpu().numpy()) if energy else out


def max_rel_err(got, ref):
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))


def mixed_rel_err(got, ref):
    """Relative error per cell with the denominator floored at 0.1 max|T|.
    T = 0 walls pull cells towards zero; there the solve forms the cell as
    U + delta with U and delta of the field's size, so its rounding is
    absolute (a few eps max|T|), not relative to the small result.  The
    floor turns the bar into an absolute 0.1 TOL max|T| for those cells
    (1e-6 max|T| in FP32, about 16 eps; 1e-13 in FP64) and leaves it
    relative elsewhere."""
    scale = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 0.1 * scale)))
