"""FP64 torch-CPU statement of the 2-D semi-implicit step, for reverse-mode
reference gradients (TEST INFRASTRUCTURE ONLY).

The forward pass restates section 2 (Eqs. xup / yup, face averaging of b,
harmonic face chi, limited transverse differences) with plain torch CPU
ops, so that torch autograd differentiates it.  It is pinned to the C
oracle's forward, cell by cell, and its gradients to central differences of
the C oracle (tests/test_oracle_adjoint.py).

Derivative conventions (the limiters are piecewise smooth):
  - every limiter has zero derivative where a*b <= 0 (the kink at ab = 0
    and the clipped region), including van Leer;
  - minmod picks its first argument when |a| == |b|;
  - MC picks 2|a|, then 2|b|, then |a+b|/2, the first that is not larger
    than the others.
Arrays are (ny, nx) float64 tensors, x fastest.  Tridiagonal systems are
solved by dense batched torch.linalg.solve (small grids only).
"""
import torch


def _shift(U, axis, s, periodic):
    """U at the neighbour displaced by s along axis (0 = x, 1 = y of (ny, nx)).
    Insulating boundaries repeat the wall cell (mirror ghost)."""
    dim = 1 if axis == 0 else 0
    if periodic:
        return torch.roll(U, shifts=-s, dims=dim)
    n = U.shape[dim]
    idx = torch.arange(n) + s
    idx = idx.clamp(0, n - 1)
    return U.index_select(dim, idx)


def lim2(a, b, limiter):
    if limiter == "linear":
        return 0.5 * (a + b)
    ab = a * b
    pos = ab > 0
    if limiter == "vanleer":
        den = torch.where(pos, a + b, torch.ones_like(a))
        return torch.where(pos, 2.0 * ab / den, torch.zeros_like(a))
    if limiter == "minmod":
        m = torch.where(a.abs() <= b.abs(), a, b)
        return torch.where(pos, m, torch.zeros_like(a))
    if limiter == "mc":
        two_a, two_b, mean = 2.0 * a, 2.0 * b, 0.5 * (a + b)
        m = torch.where(two_a.abs() <= two_b.abs(), two_a, two_b)
        m = torch.where(m.abs() <= mean.abs(), m, mean)
        return torch.where(pos, m, torch.zeros_like(a))
    raise ValueError(limiter)


def face_coefficients(b, chi, h, dt, d, periodic, chi_par, chi_perp):
    """alpha_f and beta_f of the face between each cell and its +e_d
    neighbour (zero for a wall face when not periodic)."""
    t = 1 - d
    bn = 0.5 * (b[d] + _shift(b[d], d, 1, periodic))
    bt = 0.5 * (b[t] + _shift(b[t], d, 1, periodic))
    if chi is None:
        chif = torch.full_like(bn, chi_par)
    else:
        c1 = _shift(chi, d, 1, periodic)
        s = chi + c1
        chif = torch.where(s != 0, 2.0 * chi * c1 / torch.where(s != 0, s, torch.ones_like(s)),
                           torch.zeros_like(s))
    dpar = chif - chi_perp
    alpha = dt * (chi_perp + dpar * bn * bn) / (h[d] * h[d])
    beta = dt * dpar * bn * bt / (h[d] * h[t])
    if not periodic:
        dim = 1 if d == 0 else 0
        n = bn.shape[dim]
        mask = torch.ones(n, dtype=bn.dtype)
        mask[n - 1] = 0.0
        mask = mask.view(1, n) if dim == 1 else mask.view(n, 1)
        alpha = alpha * mask
        beta = beta * mask
    return alpha, beta


def sweep(U, b, chi, h, dt, d, periodic, limiter, chi_par=1.0, chi_perp=0.0):
    """(1 + dt D_dd)^-1 (U + F_{+} - F_{-}) along axis d (Eq. xup / yup)."""
    t = 1 - d
    alpha, beta = face_coefficients(b, chi, h, dt, d, periodic, chi_par, chi_perp)
    slope = lim2(_shift(U, t, 1, periodic) - U, U - _shift(U, t, -1, periodic), limiter)
    G = lim2(_shift(slope, d, 1, periodic), slope, limiter)
    F = beta * G
    Fm = _shift(F, d, -1, True)  # face c-1/2 is stored at cell c-1
    am = _shift(alpha, d, -1, True)
    if not periodic:
        dim = 1 if d == 0 else 0
        n = U.shape[dim]
        first = torch.ones(n, dtype=U.dtype)
        first[0] = 0.0
        first = first.view(1, n) if dim == 1 else first.view(n, 1)
        Fm = Fm * first
        am = am * first
    r = U + F - Fm
    # lines as batches: rows for d = 0, columns for d = 1
    if d == 1:
        r, alpha_l, am_l = r.T, alpha.T, am.T
    else:
        alpha_l, am_l = alpha, am
    nl, n = r.shape
    A = torch.zeros(nl, n, n, dtype=U.dtype)
    i = torch.arange(n)
    A[:, i, i] = 1.0 + am_l + alpha_l
    A[:, i, (i + 1) % n] = A[:, i, (i + 1) % n] - alpha_l
    A[:, i, (i - 1) % n] = A[:, i, (i - 1) % n] - am_l
    x = torch.linalg.solve(A, r.unsqueeze(-1)).squeeze(-1)
    return x.T if d == 1 else x


def step(T, b, chi, h, dt, periodic, limiter, chi_par=1.0, chi_perp=0.0):
    Ts = sweep(T, b, chi, h, dt, 0, periodic, limiter, chi_par, chi_perp)
    return sweep(Ts, b, chi, h, dt, 1, periodic, limiter, chi_par, chi_perp)


def run(T0, b, chi, h, dt, nsteps, periodic=True, limiter="vanleer", chi_par=1.0, chi_perp=0.0):
    T = T0
    for _ in range(nsteps):
        T = step(T, b, chi, h, dt, periodic, limiter, chi_par, chi_perp)
    return T


def reverse_gradients(T0, b, chi, h, dt, nsteps, lam, periodic=True, limiter="vanleer", chi_par=1.0,
                      chi_perp=0.0):
    """dL/dT0 and dL/dchi for L with dL/dT_N = lam (numpy or torch arrays)."""
    T0 = torch.as_tensor(T0, dtype=torch.float64).clone().requires_grad_(True)
    bt = [torch.as_tensor(c, dtype=torch.float64) for c in b]
    ch = None
    if chi is not None:
        ch = torch.as_tensor(chi, dtype=torch.float64).clone().requires_grad_(True)
    TN = run(T0, bt, ch, h, dt, nsteps, periodic, limiter, chi_par, chi_perp)
    TN.backward(torch.as_tensor(lam, dtype=torch.float64))
    return T0.grad.numpy(), (ch.grad.numpy() if ch is not None else None), TN.detach().numpy()
