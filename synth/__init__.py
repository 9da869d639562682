"""Seeded synthetic inputs for the anisotropic diffusion workloads.

This module builds input fields only (unit vectors b, initial temperatures,
diffusivity fields, grid descriptions).  It holds none of the scheme's
arithmetic, so both the GPU path and the CPU oracle may consume its output.

Every generator takes an explicit seed and uses numpy's PCG64 generator; the
same seed gives the same arrays on every machine.  Arrays are float64, C order,
shape (ny, nx) in 2-D or (nz, ny, nx) in 3-D (x fastest).

Workloads (the paper uses no dataset; these stand in for its test problems):
  ring      section 3.1 ring test: circular b on [-1,1]^2, hot patch
  sovinec   section 3.2 smooth test: T = 0 walls on [-0.5,0.5]^2, source
            Q = 2 pi^2 cos(pi x) cos(pi y), b along the contours of Q
  grf2d     periodic unit square, b from a Gaussian random vector potential
            A_z (flat spectrum over integer modes 1 <= |m|^2 <= kmax2),
            T = 1 + 0.5 * sum of 8 tanh-edged blobs
  curl3d    periodic unit cube, b = curl A / |curl A| with three independent
            random potentials, T log-normal, smoothed over 4 cells
  batch     many small grf2d problems of uneven sizes
  chi field per-cell diffusivity exp(a g) with g a smoothed unit-variance field
"""
from .fields import (  # noqa: F401
    ring,
    sovinec,
    grf_unit_field_2d,
    curl_unit_field_3d,
    blobs_2d,
    smoothed_normal,
    lognormal_3d,
    chi_field_2d,
    gaussian_pulse_x,
)
from .configs import (  # noqa: F401
    Problem,
    ring_problem,
    sovinec_problem,
    grf2d_problem,
    curl3d_problem,
    batch_problems,
    adjoint_problem,
    ncfl_dt,
)
