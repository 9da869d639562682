"""Benchmark of the semi-implicit anisotropic diffusion hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 1024 x 1024 periodic random-field problem (b from a random
vector potential A_z with |m|^2 <= 64, chi_par = 1, chi_perp = 0, blob
initial T), FP32 state, dt = 20x the explicit Courant step.  A "step" is one
full semi-implicit step: x sweep + y sweep (face coefficients, limited
transverse fluxes, one tridiagonal solve per line) with the FP64 energy /
min / max reduction fused into the second sweep.  Inputs are resident in
HBM before timing; K steps are timed as one graph-captured call.

Prints one JSON line with the throughput (Gcell-updates/s), the roofline
of the dominant kernel (HBM bound, algorithmic bytes over its event-timed
average duration), the FP64 oracle timed on the host, and secondary
figures (FP64 state, explicit limited step, copy-kernel bandwidth).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
EXPLICIT_MAX_NCFL = 1.99  # largest explicit 2-D step used (the library admits ncfl <= 2 on square cells)
NX = 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip secondary measurements")
    ap.add_argument("--extra", default="all",
                    help="comma-separated secondary measurements to run: copy, fp64, explicit, speedup, "
                         "batched, 3d, adjoint, ring, sovinec, slab, large (default all)")
    ap.add_argument("--tune", type=int, default=1, help="run the launch-shape autotuner first")
    ap.add_argument("--calib", action="store_true",
                    help="also run one plain copy of 64 MiB (calibrates rocprofv3 byte counters)")
    ap.add_argument("--n", type=int, default=NX,
                    help="side of the square grid of the timed step loop (default 1024; the secondary "
                         "measurements keep their own sizes)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of sweep launch shapes: loaded if present (no tuning), else written")
    return ap.parse_args()


def timed(fn, stream, torch):
    """Run fn() between two events on `stream`; returns milliseconds."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def make_grid(p, prec, stream, torch, asd, four_step=False):
    dt = torch.float32 if prec == "f32" else torch.float64
    with torch.cuda.stream(stream):
        g = asd.Grid(p.shape, p.h, bc=p.bc, dtype=dt, chi_par=p.chi_par, chi_perp=p.chi_perp, four_step=four_step)
        b = [torch.from_numpy(c).to(dt).cuda() for c in p.b]
        T = torch.from_numpy(p.T0).to(dt).cuda()
        g.set_b(*b)
        g.set_field("T", T)
    g._keep = b
    stream.synchronize()
    return g


def run_si(g, p, steps, warmup, stream, torch):
    """Warm up with `warmup` steps, then one untimed call of exactly `steps`
    steps (it captures the graph the timed call replays, whatever the warm-up
    length), then time exactly `steps` steps; returns ms per step."""
    ebuf = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        left = warmup
        while left > 0:
            n = steps if left >= steps else left
            g.step_semi_implicit(p.dt, n, out=ebuf)
            left -= n
        g.step_semi_implicit(p.dt, steps, out=ebuf)
        stream.synchronize()
        ms = timed(lambda: g.step_semi_implicit(p.dt, steps, out=ebuf), stream, torch)
    e = ebuf.cpu().numpy()
    return ms / steps, e


def sweep_duration_in_loop(g, p, stream, torch, steps=400):
    """Average duration of one sweep launch inside the step loop: steps whole
    steps (x sweep then y sweep, each reading what the previous one wrote,
    no energy) launched eagerly on the grid's stream between two events,
    divided by the 2 * steps launches."""
    g.set_graphs(False)
    with torch.cuda.stream(stream):
        g.step_semi_implicit(p.dt, 10)
        ms = timed(lambda: g.step_semi_implicit(p.dt, steps), stream, torch)
    g.set_graphs("auto")
    return ms / (2 * steps)


def kernel_durations_repeated(g, p, stream, torch, reps=200):
    """Average duration of each sweep kernel launched back to back on the
    same input (its data stays cache-resident: an optimistic figure, shown
    for comparison only; T is not modified)."""
    out = []
    with torch.cuda.stream(stream):
        g.bench_sweep(0, p.dt, 0)  # valid inputs for every sweep
        for axis in range(len(p.shape)):
            g.bench_sweep(axis, p.dt, 5)
            ms = timed(lambda: g.bench_sweep(axis, p.dt, reps), stream, torch)
            out.append(ms / reps)
    return out


def copy_bandwidth(stream, torch, asd, nbytes=1 << 30, wide=True):
    """Read + write bandwidth of a copy of nbytes (1 GiB: four times the
    Infinity Cache) with the 16-byte streaming copy (wide) or the plain one."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        for _ in range(3):
            asd.bench_copy(src, dst, stream, wide=wide)
        reps = 20
        ms = timed(lambda: [asd.bench_copy(src, dst, stream, wide=wide) for _ in range(reps)], stream, torch)
    return 2 * nbytes * reps / (ms * 1e-3) / 1e9


def traffic_file(n):
    return os.path.join(ROOT, "profiles", f"traffic_sweep_grf2d{n}_fp32.json")


def kernel_source_digest():
    """Digest of the sources and build flags that define the timed sweep kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_tile.h", "sweep_cell.h", "asd_device.h", "asd_launch.h"):
        h.update(open(os.path.join(ROOT, "paper_1008_0861_amd", "csrc", f), "rb").read())
    from paper_1008_0861_amd import build as _build
    h.update(repr((_build.FLAGS, _build.SOURCE_FLAGS.get("sweep.hip", []))).encode())
    return h.hexdigest()[:16]


def measured_traffic(cfg, n):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs
    on the n x n grid, or None if they were taken on other kernel sources or
    launch shapes."""
    if not os.path.exists(traffic_file(n)):
        return None
    t = json.load(open(traffic_file(n)))
    if t.get("kernel_digest") != kernel_source_digest() or t.get("sweep_config") != cfg:
        return None
    return t.get("bytes_per_launch")


def matched_l1_speedup(stream, torch, asd):
    """Wall-clock speed-up of the semi-implicit scheme over the explicit
    limited scheme at matched L1 error, on the 1024^2 FP32 workload run to
    t_end = 100 semi-implicit steps at ncfl = 20.  Reference: the explicit
    scheme in FP64 at ncfl = 0.25.  The explicit run counted is the fastest
    stable one of ncfl = 1, 1.25, 1.5, 1.75 and 1.99 (the largest admitted
    step); stable: finite, within the initial range, and an L1 error that
    grows with the step no faster than a first-order time error does (at
    most twice that of ncfl = 1 scaled by (ncfl - 0.25) / 0.75; a faster
    growth is a mode of the limited scheme taking off).  The semi-implicit
    run counted is the one at the largest ncfl whose L1 error is within
    max(L1 of that explicit run, tol), tol = 1e-3, 1e-2 and 3e-2 of
    ||T_end - T_0||_1."""
    import synth
    base = synth.grf2d_problem(NX, nsteps=1)
    h = base.h
    unit = min(h) ** 2 / 4.0  # dt at ncfl = 1
    t_end = 100 * 20 * unit

    def run(prec, scheme, ncfl, time_it=False):
        nsteps = int(round(t_end / (ncfl * unit)))
        g = make_grid(base, prec, stream, torch, asd)
        dt = t_end / nsteps
        f = g.step_semi_implicit if scheme == "si" else g.step_explicit
        with torch.cuda.stream(stream):
            if scheme == "si":
                g.tune(dt, reps=10)
            if time_it:  # same call twice: the first captures the step graph
                T0 = g.T.clone()
                f(dt, nsteps)
                g.T.copy_(T0)
                stream.synchronize()
                ms = timed(lambda: f(dt, nsteps), stream, torch)
            else:
                f(dt, nsteps)
                ms = None
        stream.synchronize()
        return g.T.double(), ms, nsteps

    ref, _, nref = run("f64", "ex", 0.25)
    T0 = torch.from_numpy(base.T0).cuda()
    change = float((ref - T0).abs().mean())
    eps = 1e-3 * change
    # the explicit scheme from ncfl 1 up to the largest step the library
    # admits in 2-D (chi dt (1/hx^2 + 1/hy^2) <= 1, i.e. ncfl 2 on square
    # cells; 1.99 keeps it off the marginal checkerboard mode).  The limited
    # scheme can still grow a mode below that bound: only runs that stay
    # finite, inside the initial range (the limited fluxes keep it there) and
    # close to the reference count.
    lo, hi = float(T0.min()), float(T0.max())
    explicit = []
    l1_first = None
    for ncfl_ex in (1.0, 1.25, 1.5, 1.75, EXPLICIT_MAX_NCFL):
        ex, ms_ex, n_ex = run("f32", "ex", ncfl_ex, time_it=True)
        l1 = float((ex - ref).abs().mean())
        ncfl_run = t_end / n_ex / unit
        bounded = bool(torch.isfinite(ex).all()) and float(ex.min()) >= lo - 1e-3 * (hi - lo) \
            and float(ex.max()) <= hi + 1e-3 * (hi - lo)
        if l1_first is None:
            l1_first = l1
        stable = bounded and l1 <= 2.0 * l1_first * (ncfl_run - 0.25) / 0.75
        explicit.append(dict(ncfl=round(ncfl_run, 4), steps=n_ex, l1=l1, ms=round(ms_ex, 3), stable=stable))
    ex_used = min((r for r in explicit if r["stable"]), key=lambda r: r["ms"])
    rows = []
    for ncfl in (2, 5, 10, 20, 50, 100):
        si, ms, n = run("f32", "si", float(ncfl), time_it=True)
        rows.append(dict(ncfl=ncfl, steps=n, l1=float((si - ref).abs().mean()), ms=round(ms, 3)))
    def pick(tol):
        ok = [r for r in rows if r["l1"] <= max(ex_used["l1"], tol)]
        best = max(ok, key=lambda r: r["ncfl"]) if ok else None
        return dict(tolerance=tol, ncfl=best["ncfl"] if best else None,
                    speedup=round(ex_used["ms"] / best["ms"], 2) if best else None)

    return {
        "reference": f"explicit FP64, ncfl 0.25, {nref} steps",
        "l1_change": change,
        "explicit": ex_used,
        "explicit_runs": explicit,
        "semi_implicit": rows,
        # L1 tolerance as a fraction of ||T_end - T_0||_1 (mean per cell)
        "at_1e-3_change": pick(eps),
        "at_1e-2_change": pick(10 * eps),
        "at_3e-2_change": pick(30 * eps),
    }


def batched(stream, torch, asd, nsteps=100):
    """256 independent problems (sides 64..512, FP32), nsteps steps: tuned
    batched schedule vs one launch per problem per sweep."""
    import synth
    probs = synth.batch_problems(nprob=256, master_seed=40, nsteps=nsteps)
    with torch.cuda.stream(stream):
        items = [dict(shape=p.shape, h=p.h, chi_par=p.chi_par, dt=p.dt, T=torch.from_numpy(p.T0).float().cuda(),
                      bx=torch.from_numpy(p.b[0]).float().cuda(), by=torch.from_numpy(p.b[1]).float().cuda())
                 for p in probs]
        b = asd.Batch(items, dtype=torch.float32)
        mode, nthreads = b.tune(probe_steps=5)
        b.step(2)
    stream.synchronize()
    cells = sum(p.ncells for p in probs)
    out = {"problems": 256, "cells": cells, "steps": nsteps, "tuned_mode": mode, "tuned_threads": nthreads,
           "tuned_tile_body": ["face slots", "cell slots"][b.variant()], "graph_per_call": True}
    for name, m, energy in (("tuned", -1, False), ("tuned_energy", -1, True), ("persistent", 0, False),
                            ("persistent_energy", 0, True), ("grouped", 2, False), ("sequential", 1, False)):
        with torch.cuda.stream(stream):
            b.step(nsteps, m, energy=energy)  # same call untimed first: it captures the call's graph
            ms = timed(lambda: b.step(nsteps, m, energy=energy), stream, torch)
        out[name + "_Gcells"] = round(cells * nsteps / (ms * 1e-3) / 1e9, 3)
    flags, _ = b.status()
    out["status_flags_raised"] = int((flags != 0).sum())
    out["tuned_vs_sequential"] = round(out["tuned_Gcells"] / out["sequential_Gcells"], 2)
    return out


def three_d(stream, torch, asd, nsteps=50, ncfl=10.0, four_step=False):
    """256^3 periodic curl-field problem, FP32 state, FP64 energy every step:
    Gcell-updates/s and energy drift.  Default: the 2-step scheme at ncfl =
    10 (chi dt/h^2 = 2.5); the 4-step scheme also runs beyond the 2-step
    scheme's 3-D limit of 8.25."""
    import synth
    p = synth.curl3d_problem(256, nsteps=nsteps, ncfl=ncfl)
    g = make_grid(p, "f32", stream, torch, asd, four_step=four_step)
    ebuf = torch.empty(nsteps + 1, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        g.tune(p.dt, reps=5)
        T0 = g.T.clone()
        g.step_semi_implicit(p.dt, nsteps, out=ebuf)
        g.T.copy_(T0)
        stream.synchronize()
        ms = timed(lambda: g.step_semi_implicit(p.dt, nsteps, out=ebuf), stream, torch)
    e = ebuf.cpu().numpy()
    return {"scheme": "4-step" if four_step else "2-step", "chi_dt_over_h2": round(ncfl / 4.0, 3),
            "cells": p.ncells, "steps": nsteps, "ms_per_step": round(ms / nsteps, 4),
            "Gcells": round(p.ncells * nsteps / (ms * 1e-3) / 1e9, 3),
            # per cell-update: 3 sweeps x (4 B in + 4 B out + 12 B coefficients); the
            # 4-step scheme adds per direction a solve (4 B in + 4 B alpha + 4 B out)
            "algorithmic_GBs": round(p.ncells * (96 if four_step else 60) * nsteps / (ms * 1e-3) / 1e9, 1),
            "energy_rel_drift": float(abs(e[-1] - e[0]) / abs(e[0]))}


def slab_shares(stream, torch, asd, nsteps=200):
    """One GPU's share of the 1024^2 FP32 workload sliced into G slabs along
    y: the semi-implicit step on 1024 x (1024 / G) cells, autotuned.  The y
    sweep runs on periodic lines of 1024 / G cells, standing in for the local
    part of the partitioned solve that would span the GPUs."""
    import synth
    out = []
    for G in (2, 4, 8):
        p = synth.grf2d_problem(NX, NX // G, nsteps=nsteps)
        g = make_grid(p, "f32", stream, torch, asd)
        with torch.cuda.stream(stream):
            g.tune(p.dt, reps=10)
        ms, _ = run_si(g, p, nsteps, nsteps, stream, torch)
        out.append({"gpus": G, "cells_per_gpu": p.ncells, "ms_per_step": round(ms, 6),
                    "Gcells_per_gpu": round(p.ncells / (ms * 1e-3) / 1e9, 3)})
    return out


def large_grids(stream, torch, asd, sizes=(2048, 4096, 8192), nsteps=20):
    """The same random-field workload on grids too large for the 256 MB
    Infinity Cache to hold the step's arrays (4096^2 moves 0.54 GB per
    step, 8192^2 2.1 GB): FP32 semi-implicit steps, autotuned, with the FP64
    energy of every step; ms per step, Gcell-updates/s and the step's
    fraction of the HBM peak at 32 B per cell-update."""
    import synth
    out = []
    for n in sizes:
        p = synth.grf2d_problem(n, nsteps=nsteps)
        g = make_grid(p, "f32", stream, torch, asd)
        with torch.cuda.stream(stream):
            g.tune(p.dt, reps=4)
        ms, e = run_si(g, p, nsteps, nsteps, stream, torch)
        gbs = p.ncells * 32 / (ms * 1e-3) / 1e9
        out.append({"n": n, "ms_per_step": round(ms, 5), "Gcells": round(p.ncells / (ms * 1e-3) / 1e9, 3),
                    "step_algorithmic_GBs": round(gbs, 1), "step_frac": round(gbs / HBM_PEAK_GBS, 4),
                    "sweep_configs": [g.sweep_config(a) for a in range(2)],
                    "energy_rel_drift": float(abs(e[-1] - e[0]) / abs(e[0]))})
        del g
        torch.cuda.empty_cache()
    return out


def explicit_3d(stream, torch, asd, nsteps=50):
    """The explicit limited step on the 256^3 FP32 problem at ncfl = 1
    (chi dt/h^2 = 0.25, inside the 3-D limit of 0.444)."""
    import synth
    p = synth.curl3d_problem(256, nsteps=nsteps)
    g = make_grid(p, "f32", stream, torch, asd)
    dt = synth.ncfl_dt(1.0, p.h, 1.0)
    ebuf = torch.empty(nsteps + 1, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        g.step_explicit(dt, nsteps, out=ebuf)
        ms = timed(lambda: g.step_explicit(dt, nsteps, out=ebuf), stream, torch)
    return {"cells": p.ncells, "steps": nsteps, "ms_per_step": round(ms / nsteps, 4),
            "Gcells": round(p.ncells * nsteps / (ms * 1e-3) / 1e9, 3),
            # 4 B in + 12 B b + 4 B out per cell
            "algorithmic_GBs": round(p.ncells * 20 * nsteps / (ms * 1e-3) / 1e9, 1)}


def adjoint_1024(stream, torch, asd, n=1024, nsteps=50, ckpt_every=10):
    """The adjoint workload: 1024^2 FP32, per-cell chi, 50 semi-implicit
    steps with checkpoints every 10, sweep launch shapes autotuned.  Times,
    medians of 3: the forward steps alone (captured loop); the forward that
    stores the checkpoints (asd_adjoint_forward); the backward from those
    checkpoints (recomputation plus the reverse sweeps, gradients with
    respect to T0 and chi; asd_adjoint_step_stored); and the backward that
    takes its own checkpoints from T0 (asd_adjoint_step)."""
    import numpy as np
    import synth

    p = synth.adjoint_problem(n=n, nsteps=nsteps)
    with torch.cuda.stream(stream):
        g = asd.Grid(p.shape, p.h, bc=p.bc, dtype=torch.float32, chi_par=float(p.chi.max()), per_cell_chi=True)
        b = [torch.from_numpy(c).float().cuda() for c in p.b]
        chi = torch.from_numpy(p.chi).float().cuda()
        g.set_b(*b)
        g.set_field("chi", chi)
        T0 = torch.from_numpy(p.T0).float().cuda()
        T = T0.clone()
        g.set_field("T", T)
        g.tune(p.dt, reps=10)  # launch shapes of the sweeps (forward and reverse share them)
        T.copy_(T0)
        lam = torch.from_numpy(np.random.default_rng(7).standard_normal(p.T0.shape)).float().cuda()
        ws = g.adjoint_workspace(nsteps, ckpt_every)

    def fwd():
        T.copy_(T0)
        g.step_semi_implicit(p.dt, nsteps)

    def fwd_ckpt():
        T.copy_(T0)
        g.adjoint_forward(p.dt, nsteps, ckpt_every, ws)

    def bwd_stored():
        g.adjoint_stored(p.dt, nsteps, ckpt_every, ws, lam)

    def bwd_from_T0():
        g.adjoint(p.dt, nsteps, ckpt_every, T0, lam)

    with torch.cuda.stream(stream):
        fwd()
        fwd_ckpt()
        bwd_stored()
        bwd_from_T0()
        tf = sorted(timed(fwd, stream, torch) for _ in range(3))[1]
        tfc = sorted(timed(fwd_ckpt, stream, torch) for _ in range(3))[1]
        tb = sorted(timed(bwd_stored, stream, torch) for _ in range(3))[1]
        tb0 = sorted(timed(bwd_from_T0, stream, torch) for _ in range(3))[1]
    N = n * n
    # the differentiable map runs fwd_ckpt then bwd_stored; the ratio is of
    # those two, and the backward that takes its own checkpoints (from T0)
    # is reported beside it
    return {"cells": N, "steps": nsteps, "ckpt_every": ckpt_every, "forward_ms": round(tf, 3),
            "forward_ckpt_ms": round(tfc, 3), "backward_ms": round(tb, 3),
            "backward_over_forward": round(tb / tfc, 2), "backward_over_plain_forward": round(tb / tf, 2),
            "backward_from_T0_ms": round(tb0, 3), "backward_Gcells": round(N * nsteps / (tb * 1e-3) / 1e9, 3)}


def ring512(stream, torch, asd):
    """Ring diffusion of section 3.1 on 512^2 (T = 10 in the patch, 0.1
    elsewhere, chi = 0.01, insulating) to t = 20, FP64: minimum temperature
    over all steps for the semi-implicit scheme at ncfl = 1 .. 10^4 and for
    the explicit scheme at ncfl = 1 with and without (linear averaging) the
    van Leer limiter.  The paper's printed values: semi-implicit ncfl = 1000
    about 0.08, positive up to ncfl = 10^4; unlimited explicit -0.41."""
    import numpy as np
    import synth

    def run(ncfl, scheme, limiter):
        p = synth.ring_problem(n=512, t_in=10.0, t_out=0.1, ncfl=ncfl, nsteps=0, limiter=limiter)
        nsteps = int(np.ceil(20.0 / p.dt))
        with torch.cuda.stream(stream):
            g = asd.Grid(p.shape, p.h, bc=p.bc, dtype=torch.float64, limiter=limiter, chi_par=p.chi_par)
            b = [torch.from_numpy(c).cuda() for c in p.b]
            T = torch.from_numpy(p.T0).cuda()
            g.set_b(*b)
            g.set_field("T", T)
            g.set_graphs(False)
            s = g.step_series(scheme, p.dt, nsteps)
        stream.synchronize()
        s = s.cpu().numpy()
        return round(float(s[:, 1].min()), 5), nsteps

    out = {"si_min_T": {}, "steps": {}}
    for ncfl in (1, 10, 100, 1000, 10000):
        m, n = run(float(ncfl), "si", "vanleer")
        out["si_min_T"][str(ncfl)] = m
        out["steps"][str(ncfl)] = n
    out["explicit_vanleer_min_T"], _ = run(1.0, "ex", "vanleer")
    out["explicit_unlimited_min_T"], _ = run(1.0, "ex", "linear")
    return out


def sovinec(stream, torch, asd):
    """Smooth test of section 3.2 (T = 0 walls on [-0.5, 0.5]^2, source
    2 pi^2 cos(pi x) cos(pi y), b along its contours, no explicit chi_perp),
    FP64, run to steady state: chi_perp,num / chi_par = psi / T at the hottest
    cell, psi = cos(pi x) cos(pi y).  The approach to steady state is
    dominated by the slowest mode, T_max(t) = T_inf - A exp(-lambda t), so
    T_inf is extrapolated from three equally spaced maxima (Aitken's delta^2)
    once successive estimates agree to 1e-7.  ncfl = 1000 at n = 16 .. 128
    (the paper reports close to second-order convergence at ncfl = 1000) and
    n = 256 at ncfl = 10^4 (the paper finds chi_perp,num nearly independent
    of ncfl there; n = 256 at ncfl = 1000 needs about 1.6 million steps, too
    many for this run)."""
    import math

    import numpy as np
    import synth

    def run(n, ncfl):
        p = synth.sovinec_problem(n, ncfl=ncfl)
        with torch.cuda.stream(stream):
            g = asd.Grid(p.shape, p.h, bc="dirichlet", dtype=torch.float64, chi_par=p.chi_par)
            b = [torch.from_numpy(c).cuda() for c in p.b]
            T = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
            Q = torch.from_numpy(p.src).cuda()
            g.set_b(*b)
            g.set_field("T", T)
            g.set_field("Q", Q)
        # chunk: about 1/20 of the slowest mode's decay time for a second-order
        # guess of chi_perp,num, at least 200 steps
        lam_dt = 2 * math.pi ** 2 * 0.25 / n ** 2 * p.dt
        chunk = max(200, int(0.05 / lam_dt))
        print(f"bench: sovinec n={n} ncfl={ncfl:g} chunk={chunk}", file=sys.stderr, flush=True)
        maxima, est, steps, t0 = [], [], 0, time.perf_counter()
        for _ in range(4000):
            with torch.cuda.stream(stream):
                g.step_semi_implicit(p.dt, chunk)
                _, (_, _, tmax) = g.status()
            steps += chunk
            maxima.append(tmax)
            if len(maxima) >= 3:
                d1, d2 = maxima[-2] - maxima[-3], maxima[-1] - maxima[-2]
                inf = maxima[-1] - d2 * d2 / (d2 - d1) if d2 != d1 else maxima[-1]
                est.append(inf)
                if abs(d2) < 1e-12 * tmax or (len(est) >= 2 and abs(est[-1] - est[-2]) < 1e-7 * abs(est[-1])):
                    break
        ms = (time.perf_counter() - t0) * 1e3
        Th = T.cpu().numpy()
        i = np.unravel_index(np.argmax(Th), Th.shape)
        t_inf = est[-1] if est else maxima[-1]
        return dict(n=n, ncfl=ncfl, steps=steps, chi_perp_num=float(p.meta["psi"][i] / t_inf),
                    ms=round(ms, 1))

    rows = [run(n, 1000.0) for n in (16, 32, 64, 128)]
    for lo, hi in zip(rows, rows[1:]):
        hi["order_vs_previous"] = round(math.log2(lo["chi_perp_num"] / hi["chi_perp_num"]), 3)
    r256 = run(256, 1e4)
    r256["order_vs_previous"] = round(math.log2(rows[-1]["chi_perp_num"] / r256["chi_perp_num"]), 3)
    return dict(ncfl1000=rows, n256_ncfl1e4=r256)


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0))}


def cpu_baseline(budget_serial_s=12.0, budget_omp_s=6.0):
    """The FP64 oracle on the same 1024^2 workload, as many whole steps as fit
    in about the budget (at least 2): the OpenMP build on all the host's
    cores (the reported value) and the serial build on one core."""
    import synth
    from oracle import oracle

    p = synth.grf2d_problem(NX, nsteps=1)

    def run(omp, budget_s):
        g = oracle.OracleGrid(p.b, p.h, bc=p.bc, chi_par=p.chi_par, chi_perp=p.chi_perp, omp=omp)
        T = p.T0
        t0 = time.perf_counter()
        T = g.step_si(T, p.dt, 1)
        one = time.perf_counter() - t0
        n = max(1, int(budget_s / max(one, 1e-3)) - 1)
        t0 = time.perf_counter()
        T = g.step_si(T, p.dt, n)
        total = time.perf_counter() - t0 + one
        return n + 1, total, oracle.num_threads(omp)

    steps_s, t_s, _ = run(False, budget_serial_s)
    steps_p, t_p, threads = run(True, budget_omp_s)
    return {
        "value": round(p.ncells * steps_p / t_p / 1e9, 6),
        "unit": "Gcell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps_p} semi-implicit steps of the 1024^2 periodic random-field problem, FP64, "
                  f"C oracle built with OpenMP over the lines of each sweep, {threads} threads, {t_p:.1f} s",
        "serial": {"value": round(p.ncells * steps_s / t_s / 1e9, 6), "cores": 1,
                   "sample": f"{steps_s} steps, serial C oracle, {t_s:.1f} s"},
        "host": host_cpu(),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the semi-implicit path runs on one GPU; multi-GPU sharding of the "
              f"line sweeps is not implemented (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_1008_0861_amd import binding as asd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    asd.lib()
    stream = torch.cuda.Stream()
    p = synth.grf2d_problem(args.n, nsteps=args.steps)
    g = make_grid(p, "f32", stream, torch, asd)
    if args.tune_cache and os.path.exists(args.tune_cache):
        for a, c in enumerate(json.load(open(args.tune_cache))):
            g.set_sweep_config(a, c["wpl"], c["lpw"], c.get("io", 1), c.get("variant", 0))
    elif args.tune:
        with torch.cuda.stream(stream):
            g.tune(p.dt, reps=20)
    cfgs = [g.sweep_config(a) for a in range(2)]
    if args.tune_cache and not os.path.exists(args.tune_cache):
        json.dump(cfgs, open(args.tune_cache, "w"))
    ms_step, e = run_si(g, p, args.steps, args.warmup, stream, torch)
    N = p.ncells
    value = N / (ms_step * 1e-3) / 1e9
    drift = float(abs(e[-1] - e[0]) / abs(e[0]))

    if args.calib:
        src = torch.ones(16 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            asd.bench_copy(src, dst, stream)
        stream.synchronize()

    d_loop = sweep_duration_in_loop(g, p, stream, torch)
    durs = kernel_durations_repeated(g, p, stream, torch)
    bytes_per_launch = N * (4 + 4 + 8)  # T in, T out, (b_n, b_t) per cell, FP32
    achieved = bytes_per_launch / (d_loop * 1e-3) / 1e9
    step_gbs = N * 32 / (ms_step * 1e-3) / 1e9

    result = {
        "metric": "Gcell-updates/s per semi-implicit step + %HBM peak; speedup vs explicit at equal L1 error",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"grf2d-{args.n}x{args.n}-periodic-fp32-ncfl20-vanleer", "nx": args.n, "ny": args.n,
                   "chi_par": 1.0, "chi_perp": 0.0, "fused_fp64_energy": True, "sweep_configs": cfgs},
        "roofline": {
            "bound": "hbm",
            "kernel": "sweep_kernel (x and y sweeps, average launch inside the step loop)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(cfgs, args.n),
            "kernel_ms": round(d_loop, 6),
            "kernel_ms_repeated_input": [round(d, 6) for d in durs],
            "step_algorithmic_GBs": round(step_gbs, 1),
            "step_frac": round(step_gbs / HBM_PEAK_GBS, 4),
            "kernel_digest": kernel_source_digest(),
        },
        "energy_rel_drift": drift,
    }
    names = set() if args.no_extra else (
        {"copy", "fp64", "explicit", "speedup", "batched", "3d", "adjoint", "ring", "sovinec", "slab", "large"}
        if args.extra == "all" else set(args.extra.split(",")))
    if names:
        extra = {}
        if "copy" in names:
            extra["copy_kernel_GBs"] = round(copy_bandwidth(stream, torch, asd), 1)
            extra["copy_kernel_plain_GBs"] = round(copy_bandwidth(stream, torch, asd, wide=False), 1)
        if "fp64" in names:
            p64 = synth.grf2d_problem(NX, nsteps=200)
            g64 = make_grid(p64, "f64", stream, torch, asd)
            with torch.cuda.stream(stream):
                g64.tune(p64.dt, reps=10)
            ms64, _ = run_si(g64, p64, 200, 200, stream, torch)
            extra["fp64_si_Gcells"] = round(p64.ncells / (ms64 * 1e-3) / 1e9, 3)
        if "explicit" in names:
            gx = make_grid(p, "f32", stream, torch, asd)
            dtx = synth.ncfl_dt(1.0, p.h, 1.0)
            ebx = torch.empty(2001, dtype=torch.float64, device="cuda")
            with torch.cuda.stream(stream):
                gx.step_explicit(dtx, 2000, out=ebx)
                msx = timed(lambda: gx.step_explicit(dtx, 2000, out=ebx), stream, torch) / 2000
            extra["explicit_fp32_Gcells"] = round(N / (msx * 1e-3) / 1e9, 3)
            extra["explicit_ms_per_step"] = round(msx, 6)
        if "speedup" in names:
            result["speedup_vs_explicit"] = matched_l1_speedup(stream, torch, asd)
        if "batched" in names:
            extra["batched"] = batched(stream, torch, asd)
        if "3d" in names:
            extra["curl3d_256"] = three_d(stream, torch, asd)
            extra["curl3d_256_four_step"] = three_d(stream, torch, asd, ncfl=40.0, four_step=True)
            extra["curl3d_256_explicit"] = explicit_3d(stream, torch, asd)
        if "adjoint" in names:
            extra["adjoint_1024"] = adjoint_1024(stream, torch, asd)
        if "ring" in names:
            extra["ring512"] = ring512(stream, torch, asd)
        if "sovinec" in names:
            extra["sovinec"] = sovinec(stream, torch, asd)
        if "slab" in names:
            extra["slab_shares"] = slab_shares(stream, torch, asd)
        if "large" in names:
            extra["large_grids"] = large_grids(stream, torch, asd)
        result["extra"] = extra
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
