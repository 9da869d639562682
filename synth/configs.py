"""The workload recipes, as seeded problem descriptions (inputs only)."""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

from . import fields


@dataclass
class Problem:
    """One grid problem.  Arrays are float64, shape (ny, nx) or (nz, ny, nx)."""
    name: str
    b: Tuple[np.ndarray, ...]
    T0: np.ndarray
    h: Tuple[float, ...]
    bc: str = "periodic"             # "periodic" | "insulating" | "dirichlet"
    limiter: str = "vanleer"         # "vanleer" | "minmod" | "mc" | "linear"
    chi_par: float = 1.0
    chi_perp: float = 0.0
    chi: Optional[np.ndarray] = None  # per-cell chi_par (None: constant)
    src: Optional[np.ndarray] = None  # per-cell source Q (None: none)
    dt: float = 0.0
    nsteps: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.b)

    @property
    def shape(self):
        return self.T0.shape

    @property
    def ncells(self):
        return int(np.prod(self.T0.shape))


def ncfl_dt(ncfl, h, chi_max):
    """Time step from the Courant factor of the paper: dt = ncfl * h^2 / (4 chi),
    h the smallest cell width, chi the largest diffusivity (Eq. ncfl)."""
    return float(ncfl) * min(h) ** 2 / (4.0 * float(chi_max))


def ring_problem(n=64, t_in=12.0, t_out=10.0, ncfl=10.0, nsteps=200, chi_par=0.01,
                 limiter="vanleer"):
    """Ring diffusion (section 3.1): insulating box [-1,1]^2, circular b.
    Defaults are the 64x64 case with T = 12 in the patch, 10 elsewhere,
    200 steps at 10x the explicit Courant step."""
    bx, by, T0, h = fields.ring(n, t_in, t_out)
    return Problem("ring", (bx, by), T0, (h, h), bc="insulating", limiter=limiter,
                   chi_par=chi_par, dt=ncfl_dt(ncfl, (h, h), chi_par), nsteps=nsteps,
                   meta=dict(n=n, t_in=t_in, t_out=t_out, ncfl=ncfl))


def sovinec_problem(n=64, ncfl=1000.0, nsteps=100, chi_par=1.0, limiter="vanleer"):
    """Smooth test of section 3.2: [-0.5, 0.5]^2, T = 0 on the walls and at
    t = 0, source Q = 2 pi^2 cos(pi x) cos(pi y), b along the contours of Q,
    no explicit chi_perp, 1000x the Courant step.  meta["psi"] holds
    cos(pi x) cos(pi y) at the cells (the shape of the steady state)."""
    bx, by, Q, psi, h = fields.sovinec(n)
    return Problem("sovinec", (bx, by), np.zeros((n, n)), (h, h), bc="dirichlet", limiter=limiter,
                   chi_par=chi_par, src=Q, dt=ncfl_dt(ncfl, (h, h), chi_par), nsteps=nsteps,
                   meta=dict(n=n, ncfl=ncfl, psi=psi))


def grf2d_problem(nx=1024, ny=None, chi_perp=0.0, ncfl=20.0, nsteps=100, seed_b=20, seed_t=21,
                  chi_par=1.0, kmax2=64, limiter="vanleer"):
    """Periodic unit square, b from a random potential A_z (|m|^2 <= 64),
    T = 1 + 0.5 * tanh-edged blobs, 100 steps at 20x the Courant step."""
    ny = nx if ny is None else ny
    bx, by = fields.grf_unit_field_2d(nx, ny, seed_b, kmax2=kmax2)
    T0 = fields.blobs_2d(nx, ny, seed_t)
    h = (1.0 / nx, 1.0 / ny)
    return Problem("grf2d", (bx, by), T0, h, bc="periodic", limiter=limiter, chi_par=chi_par,
                   chi_perp=chi_perp, dt=ncfl_dt(ncfl, h, chi_par), nsteps=nsteps,
                   meta=dict(nx=nx, ny=ny, ncfl=ncfl, seed_b=seed_b, seed_t=seed_t))


def curl3d_problem(n=256, ncfl=10.0, nsteps=50, seed_b=30, seed_t=31, kmax2=36,
                   limiter="vanleer"):
    """Periodic unit cube, b = curl A/|curl A| (|m|^2 <= 36), log-normal T
    (sigma 0.3, smoothed over 4 cells), 50 steps at 10x the Courant step."""
    bx, by, bz = fields.curl_unit_field_3d(n, seed_b, kmax2=kmax2)
    T0 = fields.lognormal_3d(n, seed_t)
    h = (1.0 / n,) * 3
    return Problem("curl3d", (bx, by, bz), T0, h, bc="periodic", limiter=limiter, chi_par=1.0,
                   dt=ncfl_dt(ncfl, h, 1.0), nsteps=nsteps,
                   meta=dict(n=n, ncfl=ncfl, seed_b=seed_b, seed_t=seed_t))


def batch_problems(nprob=256, master_seed=40, sides=None, ncfl=20.0, nsteps=100):
    """Independent 2-D problems with sides drawn from {64, 96, ..., 512}
    (nx and ny independently), chi_par ~ U[0.1, 1], each with its own random
    A_z field and blob initial T (seed 4000 + p), periodic, 20x Courant."""
    rng = np.random.default_rng(np.random.PCG64(master_seed))
    if sides is None:
        sides = np.arange(64, 513, 32)
    probs = []
    for p in range(nprob):
        nx = int(rng.choice(sides))
        ny = int(rng.choice(sides))
        chi = float(rng.uniform(0.1, 1.0))
        seed = 4000 + p
        bx, by = fields.grf_unit_field_2d(nx, ny, seed)
        T0 = fields.blobs_2d(nx, ny, seed + 100000)
        h = (1.0 / nx, 1.0 / ny)
        probs.append(Problem(f"batch{p}", (bx, by), T0, h, bc="periodic", chi_par=chi,
                             dt=ncfl_dt(ncfl, h, chi), nsteps=nsteps,
                             meta=dict(nx=nx, ny=ny, seed=seed)))
    return probs


def adjoint_problem(n=1024, nsteps=50, ncfl=20.0, seed_b=50, seed_chi=51, seed_pert=52):
    """Periodic unit square with per-cell chi = exp(0.5 g) (g smoothed, unit
    variance), b from a random A_z; meta["chi_target"] = chi * exp(0.1 g')
    is the perturbed diffusivity that defines the target temperature.
    T0 = exp(0.3 g'') with g'' smoothed over 4 cells: smooth everywhere, so
    the limiters are differentiable at almost every face (a two-level or
    flat field puts many faces on the a*b = 0 kink)."""
    bx, by = fields.grf_unit_field_2d(n, n, seed_b)
    chi = fields.chi_field_2d(n, n, seed_chi, amp=0.5)
    chi_t = chi * np.exp(0.1 * fields.smoothed_normal((n, n), seed_pert))
    T0 = np.exp(0.3 * fields.smoothed_normal((n, n), seed_b + 1000))
    h = (1.0 / n, 1.0 / n)
    dt = ncfl_dt(ncfl, h, max(chi.max(), chi_t.max()))
    return Problem("adjoint", (bx, by), T0, h, bc="periodic", chi_par=1.0, chi=chi, dt=dt,
                   nsteps=nsteps, meta=dict(n=n, chi_target=chi_t, ncfl=ncfl))
