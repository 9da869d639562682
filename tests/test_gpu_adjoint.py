"""GPU adjoint (asd_adjoint_step) against the FP64 reverse-mode reference
(oracle/torch_ref.py, pinned to the C oracle and to finite differences),
and against central differences of the GPU forward at full size."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle, torch_ref
from paper_1008_0861_amd import binding as asd
from paper_1008_0861_amd.autograd import semi_implicit_steps

pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f64": torch.float64}


def _problem(shape, seed, bc="periodic"):
    ny, nx = shape
    rng = np.random.default_rng(seed)
    v = [synth.smoothed_normal(shape, seed + q, 2.0) + 0.3 * rng.standard_normal() for q in range(2)]
    m = np.sqrt(v[0] ** 2 + v[1] ** 2)
    b = (v[0] / m, v[1] / m)
    T0 = 1.0 + 0.3 * synth.smoothed_normal(shape, seed + 5, 1.5)
    chi = np.exp(0.4 * synth.smoothed_normal(shape, seed + 9, 2.0))
    h = (1.0 / nx, 1.2 / ny)
    dt = 20 * min(h) ** 2 / (4 * chi.max())
    return b, T0, chi, h, dt


class AdjGrid:
    def __init__(self, b, chi, h, prec, bc="periodic", limiter="vanleer", chi_perp=0.0):
        self.stream = torch.cuda.Stream()
        self.dt = DT[prec]
        with torch.cuda.stream(self.stream):
            self.g = asd.Grid(b[0].shape, h, bc=bc, dtype=self.dt, limiter=limiter, chi_par=float(chi.max()),
                              chi_perp=chi_perp, per_cell_chi=True)
            self.b = [torch.from_numpy(c).to(self.dt).cuda() for c in b]
            self.chi = torch.from_numpy(chi).to(self.dt).cuda()
            self.g.set_b(*self.b)
            self.g.set_field("chi", self.chi)

    def adjoint(self, T0, lam, dt, nsteps, k):
        with torch.cuda.stream(self.stream):
            t0 = torch.from_numpy(T0).to(self.dt).cuda()
            la = torch.from_numpy(lam).to(self.dt).cuda()
            gT, gC = self.g.adjoint(dt, nsteps, k, t0, la)
        self.stream.synchronize()
        return gT.double().cpu().numpy(), gC.double().cpu().numpy()

    def forward(self, T0, dt, nsteps, chi=None):
        with torch.cuda.stream(self.stream):
            if chi is not None:
                self.chi = torch.from_numpy(chi).to(self.dt).cuda()
                self.g.set_field("chi", self.chi)
            T = torch.from_numpy(T0).to(self.dt).cuda()
            self.g.set_field("T", T)
            self.g.step_semi_implicit(dt, nsteps)
        self.stream.synchronize()
        return T.double().cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("bc", ["periodic", "insulating"])
@pytest.mark.parametrize("limiter", ["vanleer", "minmod", "mc", "linear"])
def test_adjoint_matches_reverse_reference_fp64(bc, limiter):
    b, T0, chi, h, dt = _problem((40, 56), 3, bc)
    rng = np.random.default_rng(4)
    lam = rng.standard_normal(T0.shape)
    gT_ref, gC_ref, _ = torch_ref.reverse_gradients(T0, b, chi, h, dt, 7, lam, periodic=bc == "periodic",
                                                    limiter=limiter, chi_par=float(chi.max()))
    gT, gC = AdjGrid(b, chi, h, "f64", bc=bc, limiter=limiter).adjoint(T0, lam, dt, 7, 3)
    assert _rel(gT, gT_ref) <= 1e-10
    assert _rel(gC, gC_ref) <= 1e-10


def _rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_adjoint_fp32_against_reference():
    """FP32 state: relative L2 error within the rounding bound
    steps x sweeps x condition x eps32 ~ 20 x 21 x 6e-8 ~ 2.5e-5 (x4 margin);
    in max norm a few cells may sit where FP32 and FP64 states take
    different sides of a limiter kink, hence 2e-3."""
    b, T0, chi, h, dt = _problem((96, 96), 5)
    r = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    rng = np.random.default_rng(6)
    lam = r(rng.standard_normal(T0.shape))
    gT_ref, gC_ref, _ = torch_ref.reverse_gradients(r(T0), [r(c) for c in b], r(chi), h, dt, 10, lam,
                                                    chi_par=float(chi.max()))
    gT, gC = AdjGrid(b, chi, h, "f32").adjoint(T0, lam, dt, 10, 4)
    assert _rel2(gT, gT_ref) <= 1e-4 and _rel(gT, gT_ref) <= 2e-3
    assert _rel2(gC, gC_ref) <= 1e-4 and _rel(gC, gC_ref) <= 2e-3


def test_checkpoint_interval_does_not_change_the_result():
    b, T0, chi, h, dt = _problem((48, 40), 8)
    lam = np.random.default_rng(9).standard_normal(T0.shape)
    ag = AdjGrid(b, chi, h, "f64")
    ref = ag.adjoint(T0, lam, dt, 12, 1)
    for k in (5, 7, 12, 50):
        got = ag.adjoint(T0, lam, dt, 12, k)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), k


def test_adjoint_128_fp64_target_loss():
    """The adjoint workload's FP64 check size: 128^2, per-cell chi =
    exp(0.5 g), 50 steps, checkpoints every 10, L = sum (T_N - T_target)^2
    with T_target from the perturbed diffusivity."""
    p = synth.adjoint_problem(n=128, nsteps=50)
    chi_t = p.meta["chi_target"]
    og = oracle.OracleGrid(p.b, p.h, bc=p.bc, chi=chi_t)
    T_target = og.step_si(p.T0, p.dt, p.nsteps)
    TN = oracle.OracleGrid(p.b, p.h, bc=p.bc, chi=p.chi).step_si(p.T0, p.dt, p.nsteps)
    lam = 2.0 * (TN - T_target)
    gT_ref, gC_ref, _ = torch_ref.reverse_gradients(p.T0, p.b, p.chi, p.h, p.dt, p.nsteps, lam)
    ag = AdjGrid(p.b, p.chi, p.h, "f64")
    gT, gC = ag.adjoint(p.T0, lam, p.dt, p.nsteps, 10)
    assert _rel(gT, gT_ref) <= 1e-10
    assert _rel(gC, gC_ref) <= 1e-10


def test_autograd_function_matches_reference():
    b, T0, chi, h, dt = _problem((32, 48), 12)
    target = np.random.default_rng(13).standard_normal(T0.shape) * 0.01 + 1.0
    ag = AdjGrid(b, chi, h, "f64")
    with torch.cuda.stream(ag.stream):
        t0 = torch.from_numpy(T0).cuda().requires_grad_(True)
        ch = torch.from_numpy(chi).cuda().requires_grad_(True)
        TN = semi_implicit_steps(t0, ch, ag.g, dt, 6, 4)
        loss = ((TN - torch.from_numpy(target).cuda()) ** 2).sum()
        loss.backward()
    torch.cuda.synchronize()
    TN_ref = torch_ref.run(torch.from_numpy(T0), [torch.from_numpy(c) for c in b], torch.from_numpy(chi), h, dt, 6,
                           chi_par=float(chi.max())).numpy()
    lam = 2.0 * (TN_ref - target)
    gT_ref, gC_ref, _ = torch_ref.reverse_gradients(T0, b, chi, h, dt, 6, lam, chi_par=float(chi.max()))
    assert _rel(TN.detach().cpu().numpy(), TN_ref) <= 1e-12
    assert _rel(t0.grad.cpu().numpy(), gT_ref) <= 1e-9
    assert _rel(ch.grad.cpu().numpy(), gC_ref) <= 1e-9


def test_adjoint_1024_fp32_against_central_differences():
    """The full adjoint workload: 1024^2 FP32, 50 steps, checkpoints every 10,
    L = sum (T_N - T_target)^2.  dL/dchi and dL/dT0 at the same 32 random
    cells each against central differences of the FP64 GPU forward (itself
    at oracle parity).  A cell whose quotient changes between eps and eps/2
    sits on a limiter kink and is skipped; at most a quarter of each
    gradient's cells may be.  Bar per cell: 1 % of the difference quotient,
    plus 1e-4 of the gradient's largest magnitude for gradients near zero
    (the FP32 adjoint's rounding is relative to the field, not to the cell)."""
    p = synth.adjoint_problem(n=1024, nsteps=50)
    chi_t = p.meta["chi_target"]
    f64 = AdjGrid(p.b, p.chi, p.h, "f64")
    T_target = f64.forward(p.T0, p.dt, p.nsteps, chi=chi_t)
    TN = f64.forward(p.T0, p.dt, p.nsteps, chi=p.chi)
    lam = 2.0 * (TN - T_target)
    gT, gC = AdjGrid(p.b, p.chi, p.h, "f32").adjoint(p.T0, lam, p.dt, p.nsteps, 10)

    def loss(T0v, chiv):
        return float(np.sum((f64.forward(T0v, p.dt, p.nsteps, chi=chiv) - T_target) ** 2))

    rng = np.random.default_rng(53)
    cells = [tuple(int(v) for v in rng.integers(0, 1024, 2)) for _ in range(32)]
    bad = []
    for which, grad, base in (("chi", gC, p.chi), ("T", gT, p.T0)):
        gscale = float(np.max(np.abs(grad)))
        skipped = 0
        for cell in cells:
            def fd(eps):
                up, dn = base.copy(), base.copy()
                up[cell] += eps
                dn[cell] -= eps
                if which == "chi":
                    return (loss(p.T0, up) - loss(p.T0, dn)) / (2 * eps)
                return (loss(up, p.chi) - loss(dn, p.chi)) / (2 * eps)
            e = 1e-4 * (base[cell] if which == "chi" else 1.0)
            f1, f2 = fd(e), fd(e / 2)
            kink = abs(f1 - f2) > 1e-3 * max(abs(f1), 1e-3 * gscale)
            tol = 1e-2 * abs(f2) + 1e-4 * gscale
            print(f"\n{which} {cell} grad {grad[cell]:.6e} fd {f2:.6e} fd(2eps) {f1:.6e} "
                  f"err/tol {abs(grad[cell] - f2) / tol:.3f}{' kink' if kink else ''}")
            if kink:
                skipped += 1
                continue
            if abs(grad[cell] - f2) > tol:
                bad.append((which, cell, float(grad[cell]), f2))
        print(f"\n{which}: {32 - skipped} of 32 cells checked, {skipped} on a limiter kink")
        assert skipped <= 8, (which, skipped)
    assert not bad, bad


def _stored_vs_recomputed(ag, T0, lams, dt, nsteps, k):
    """asd_adjoint_forward then asd_adjoint_step_stored (once per lambda, on
    one set of checkpoints) against asd_step_semi_implicit and
    asd_adjoint_step; returns the max differences."""
    with torch.cuda.stream(ag.stream):
        t0 = torch.from_numpy(T0).to(ag.dt).cuda()
        T_step = t0.clone()
        ag.g.set_field("T", T_step)
        ag.g.step_semi_implicit(dt, nsteps)
        T_fwd = t0.clone()
        ag.g.set_field("T", T_fwd)
        ws = ag.g.adjoint_forward(dt, nsteps, k)
        out = []
        for lam in lams:
            la = torch.from_numpy(lam).to(ag.dt).cuda()
            stored = ag.g.adjoint_stored(dt, nsteps, k, ws, la)
            recomputed = ag.g.adjoint(dt, nsteps, k, t0, la)
            out.append((stored, recomputed))
    ag.stream.synchronize()
    assert torch.equal(T_fwd, T_step)
    for (sT, sC), (rT, rC) in out:
        assert torch.equal(sT, rT) and torch.equal(sC, rC)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nsteps,k", [(12, 1), (12, 5), (12, 12), (12, 50), (13, 4), (0, 3)])
def test_stored_checkpoints_give_the_same_states_and_gradients(prec, nsteps, k):
    """The checkpointing forward leaves T exactly as the stepping entry point
    does, and the reverse pass from its checkpoints equals the reverse pass
    that takes its own (same kernels, same states: bit for bit), also for a
    second lambda on the same checkpoints."""
    b, T0, chi, h, dt = _problem((48, 40), 21)
    rng = np.random.default_rng(22)
    lams = [rng.standard_normal(T0.shape) for _ in range(2)]
    _stored_vs_recomputed(AdjGrid(b, chi, h, prec), T0, lams, dt, nsteps, k)


def test_stored_checkpoints_1024_fp32_workload():
    """The adjoint workload's shape (1024^2 FP32, 50 steps, checkpoints every
    10) with the sweeps autotuned, so the tuned launch shapes run."""
    p = synth.adjoint_problem(n=1024, nsteps=50)
    ag = AdjGrid(p.b, p.chi, p.h, "f32")
    with torch.cuda.stream(ag.stream):
        T = torch.from_numpy(p.T0).float().cuda()
        ag.g.set_field("T", T)
        ag.g.tune(p.dt, reps=3)
    lam = np.random.default_rng(23).standard_normal(p.T0.shape)
    _stored_vs_recomputed(ag, p.T0, [lam], p.dt, p.nsteps, 10)
    # five segments (the recomputation on the second stream beside the
    # reverse pass) against one segment (one stream), bit for bit
    five = ag.adjoint(p.T0, lam, p.dt, p.nsteps, 10)
    one = ag.adjoint(p.T0, lam, p.dt, p.nsteps, 50)
    assert np.array_equal(five[0], one[0]) and np.array_equal(five[1], one[1])


def test_autograd_two_forwards_before_backward():
    """Two forward calls on one grid with different chi, then both backward
    passes: each keeps its own checkpoints, and the backward sets its own chi
    again, so both gradients match the reverse-mode reference."""
    b, T0, chi, h, dt = _problem((32, 40), 31)
    chi2 = chi * np.exp(0.2 * synth.smoothed_normal(chi.shape, 32, 2.0))
    cmax = float(max(chi.max(), chi2.max()))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = asd.Grid(b[0].shape, h, bc="periodic", dtype=torch.float64, chi_par=cmax, per_cell_chi=True)
        g.set_b(*[torch.from_numpy(c).cuda() for c in b])
        t0s = [torch.from_numpy(T0).cuda().requires_grad_(True) for _ in range(2)]
        chs = [torch.from_numpy(c).cuda().requires_grad_(True) for c in (chi, chi2)]
        outs = [semi_implicit_steps(t0s[i], chs[i], g, dt, 7, 3) for i in range(2)]
        for o in outs:
            (o ** 2).sum().backward()
    torch.cuda.synchronize()
    for i, c in enumerate((chi, chi2)):
        TN = torch_ref.run(torch.from_numpy(T0), [torch.from_numpy(v) for v in b], torch.from_numpy(c), h, dt, 7,
                           chi_par=cmax).numpy()
        gT_ref, gC_ref, _ = torch_ref.reverse_gradients(T0, b, c, h, dt, 7, 2.0 * TN, chi_par=cmax)
        assert _rel(outs[i].detach().cpu().numpy(), TN) <= 1e-12
        assert _rel(t0s[i].grad.cpu().numpy(), gT_ref) <= 1e-9
        assert _rel(chs[i].grad.cpu().numpy(), gC_ref) <= 1e-9
