"""Discrete Navier-Stokes right-hand side N(q) and its linearisation (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Governing equations: Section "Governing equations", eq. (navier_stokes), in
the variables q = [p, u_i, s] (the shorthand N(q) is defined right after the
equations).  Readings taken where the printed system is incomplete:

* The pressure equation is read with the material derivative Dp/Dt (the
  printed left side lacks the advection term); substituting the entropy
  equation gives p/(c_v rho T) = gamma - 1 in front of the heat terms.
* The entropy equation is taken with the physical sign
  rho T Ds/Dt = +(div(lambda grad T) + Phi).
* Bulk viscosity mu_v = 0; Sutherland's law mu = mu_ref T^1.5 (1+S)/(T+S),
  S = 110.4 K / 288.15 K; ideal gas with gamma = 1.4; conductivity
  lambda = c_p mu / Pr.  Non-dimensional: rho_ref = T_ref = u_inf = delta = 1,
  R = 1/(gamma M^2) so that the reference pressure is 1/(gamma M^2) and
  c_ref = 1/M; mu_ref = 1/Re (0 for an inviscid case).
* First derivatives: explicit 6th-order central differences (reduced to 4th
  and 2nd order on the two rows next to each wall), or, with
  prob.scheme == 1, the 6th-order compact (tridiagonal) scheme of Lele that
  the paper uses for its wave terms (Section "Governing equations", last
  paragraph), on the collocated grid, with Lele's 4th-order compact row and
  3rd-order one-sided compact row at each wall.  Second derivatives are the
  explicit 6th-order central ones in both cases (the paper's 5th-order
  dissipation scheme is not specified).  Mixed derivatives are products of
  first differences; gradients of mu and lambda use the chain rule
  mu'(T) D T.
  The viscous terms are expanded:
      d_j tau_ij = mu L u_i + (mu/3) G_i
                   + mu'(T) [ D_j T (D_j u_i + D_i u_j) - 2/3 D_i T D_k u_k ]
      G_i = D2_i u_i + sum_{j != i} D_i (D_j u_j),   L = sum_j D2_j
      Q   = lambda L T + lambda'(T) D_j T D_j T       (= div(lambda grad T))
      Phi = mu [2 s_ij s_ij - 2/3 s_kk^2]             (= tau_ij s_ij)
* Wall rows (y = +-Ly/2) carry zero perturbation: the operator is P J P with
  P zeroing the wall rows.
* Grid stretching in y (Section "Model problem": points clustered where the
  velocity gradients are largest), prob.stretch = beta > 0: the rows sit at
  y(eta) = (Ly/2) sinh(beta eta)/sinh(beta) of a uniform eta grid on [-1, 1],
  the stencils above act along eta, and the chain rule with the analytic
  metric gives D_y f = D_eta f / y' and
  D_yy f = D_etaeta f / y'^2 - (y''/y'^2) D_y f
  (D_y the scheme's first derivative, explicit or compact).

Everything is written so that it is complex-analytic (no abs, no branches on
values), which lets ``jv_cstep`` obtain the exact derivative of the discrete
N by the complex-step method (Squire & Trefethen 1998).
"""
from __future__ import annotations

import math

import numpy as np

BC_PERIODIC = 0
BC_WALL = 1

EPS_MACHINE = 2.0 ** -52


class Constants:
    """Non-dimensional gas constants of one problem (plain definitions)."""

    def __init__(self, prob):
        self.gamma = float(prob.gamma)
        self.mach = float(prob.mach)
        self.pr = float(prob.pr)
        self.suth = float(prob.sutherland)
        self.p_ref = 1.0 / (self.gamma * self.mach ** 2)
        self.R = 1.0 / (self.gamma * self.mach ** 2)
        self.cv = self.R / (self.gamma - 1.0)
        self.cp = self.gamma * self.R / (self.gamma - 1.0)
        self.mu_ref = 1.0 / prob.re if prob.re > 0 else 0.0


def spacings(prob):
    """Grid spacings (dx, dy, dz): periodic axes x_i = i L / N, wall axis with
    N points including both walls; with y stretching, dy is the spacing of
    the computational coordinate eta in [-1, 1]."""
    out = []
    for a in range(3):
        n = prob.n[a]
        L = prob.length[a]
        if a >= prob.ndim:
            out.append(1.0)
        elif a == 1 and stretched(prob):
            out.append(2.0 / (n - 1))
        elif prob.bc[a] == BC_WALL:
            out.append(L / (n - 1))
        else:
            out.append(L / n)
    return tuple(out)


def stretched(prob):
    return float(getattr(prob, "stretch", 0.0)) > 0.0


def y_metrics(prob):
    """(1/y'(eta_j), -y''(eta_j)/y'(eta_j)^2) of the mapping
    y = (Ly/2) sinh(beta eta)/sinh(beta), as (Ny, 1) columns."""
    beta = float(prob.stretch)
    ny = prob.n[1]
    if prob.bc[1] != BC_WALL:
        raise ValueError("grid stretching needs walls in y")
    eta = -1.0 + np.arange(ny) * (2.0 / (ny - 1))
    half = 0.5 * prob.length[1] / math.sinh(beta)
    yp = half * beta * np.cosh(beta * eta)
    ypp = half * beta * beta * np.sinh(beta * eta)
    return (1.0 / yp)[:, None], (-ypp / (yp * yp))[:, None]


# ---------------------------------------------------------------------------
# Finite-difference stencils.  Arrays carry the grid in their trailing axes:
# x is axis -1, y is axis -2, z is axis -3.
# ---------------------------------------------------------------------------
_D1_6 = (3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0)            # coefficients of f(+m) - f(-m)
_D2_6 = (-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0)  # centre, then f(+m) + f(-m)
_D1_4 = (2.0 / 3.0, -1.0 / 12.0)
_D2_4 = (-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0)
_D1_2 = (1.0 / 2.0,)
_D2_2 = (-2.0, 1.0)


def _axis_of(a):
    return -1 - a          # a = 0 (x) -> -1, 1 (y) -> -2, 2 (z) -> -3


def d1(f, a, h, bc):
    """First derivative along grid axis a (0=x, 1=y, 2=z)."""
    ax = _axis_of(a)
    if bc == BC_PERIODIC:
        out = 0.0
        for m, c in enumerate(_D1_6, start=1):
            out = out + c * (np.roll(f, -m, axis=ax) - np.roll(f, m, axis=ax))
        return out / h
    g = np.moveaxis(f, ax, 0)
    n = g.shape[0]
    out = np.zeros_like(g)
    # 6th order from the fourth row inward
    acc = 0.0
    for m, c in enumerate(_D1_6, start=1):
        acc = acc + c * (g[3 + m:n - 3 + m] - g[3 - m:n - 3 - m])
    out[3:n - 3] = acc / h
    # 4th order on rows 2 and n-3
    for j in (2, n - 3):
        out[j] = (_D1_4[0] * (g[j + 1] - g[j - 1]) + _D1_4[1] * (g[j + 2] - g[j - 2])) / h
    # 2nd order on rows 1 and n-2
    for j in (1, n - 2):
        out[j] = _D1_2[0] * (g[j + 1] - g[j - 1]) / h
    return np.moveaxis(out, 0, ax)


# Lele's tridiagonal 6th-order first derivative (J. Comput. Phys. 103, 1992):
#   alpha f'_{i-1} + f'_i + alpha f'_{i+1}
#       = a (f_{i+1} - f_{i-1}) / (2h) + b (f_{i+2} - f_{i-2}) / (4h)
# with alpha = 1/3, a = 14/9, b = 1/9; at a wall the row next to it is the
# 4th-order Pade scheme (alpha = 1/4, a = 3/2, b = 0) and the wall row the
# 3rd-order one-sided scheme f'_0 + 2 f'_1 = (-5/2 f_0 + 2 f_1 + 1/2 f_2)/h.
_C6_ALPHA, _C6_A, _C6_B = 1.0 / 3.0, 14.0 / 9.0, 1.0 / 9.0


def compact_matrices(n, periodic):
    """(A, B) with A f' = B f / h for the compact first derivative on n points."""
    A = np.zeros((n, n))
    B = np.zeros((n, n))

    def interior(i, alpha, a, b):
        for m, c in ((1, a / 2.0), (2, b / 4.0)):
            if c == 0.0:
                continue
            B[i, (i + m) % n] += c
            B[i, (i - m) % n] -= c
        A[i, i] = 1.0
        A[i, (i + 1) % n] += alpha
        A[i, (i - 1) % n] += alpha

    if periodic:
        for i in range(n):
            interior(i, _C6_ALPHA, _C6_A, _C6_B)
        return A, B
    for i in range(2, n - 2):
        interior(i, _C6_ALPHA, _C6_A, _C6_B)
    for i in (1, n - 2):
        interior(i, 0.25, 1.5, 0.0)
    A[0, 0], A[0, 1] = 1.0, 2.0
    B[0, 0], B[0, 1], B[0, 2] = -2.5, 2.0, 0.5
    A[n - 1, n - 1], A[n - 1, n - 2] = 1.0, 2.0
    B[n - 1, n - 1], B[n - 1, n - 2], B[n - 1, n - 3] = 2.5, -2.0, -0.5
    return A, B


def d1_compact(f, a, h, bc):
    """Compact first derivative along grid axis a: f' = A^-1 B f / h."""
    ax = _axis_of(a)
    g = np.moveaxis(np.asarray(f), ax, 0)
    n = g.shape[0]
    A, B = compact_matrices(n, bc == BC_PERIODIC)
    rhs_ = (B @ g.reshape(n, -1)) / h
    out = np.linalg.solve(A, rhs_).reshape(g.shape)
    return np.moveaxis(out, 0, ax)


def d2(f, a, h, bc):
    """Second derivative along grid axis a."""
    ax = _axis_of(a)
    if bc == BC_PERIODIC:
        out = _D2_6[0] * f
        for m, c in enumerate(_D2_6[1:], start=1):
            out = out + c * (np.roll(f, -m, axis=ax) + np.roll(f, m, axis=ax))
        return out / (h * h)
    g = np.moveaxis(f, ax, 0)
    n = g.shape[0]
    out = np.zeros_like(g)
    acc = _D2_6[0] * g[3:n - 3]
    for m, c in enumerate(_D2_6[1:], start=1):
        acc = acc + c * (g[3 + m:n - 3 + m] + g[3 - m:n - 3 - m])
    out[3:n - 3] = acc / (h * h)
    for j in (2, n - 3):
        out[j] = (_D2_4[0] * g[j] + _D2_4[1] * (g[j + 1] + g[j - 1])
                  + _D2_4[2] * (g[j + 2] + g[j - 2])) / (h * h)
    for j in (1, n - 2):
        out[j] = (_D2_2[0] * g[j] + _D2_2[1] * (g[j + 1] + g[j - 1])) / (h * h)
    return np.moveaxis(out, 0, ax)


# ---------------------------------------------------------------------------
# Thermodynamics (ideal gas, entropy zero at the reference state).
# ---------------------------------------------------------------------------
def deriv(prob, f, a):
    """First derivative along physical axis a of the problem's discrete
    operator: the scheme's stencil along the grid index, over the spacing,
    and with y stretching divided by y'(eta)."""
    h = spacings(prob)[a]
    bc = prob.bc[a]
    first = d1_compact if getattr(prob, "scheme", 0) == 1 else d1
    d = first(f, a, h, bc)
    if a == 1 and stretched(prob):
        d = d * y_metrics(prob)[0]
    return d


def deriv2(prob, f, a):
    """Second derivative along physical axis a: the explicit stencil, and
    with y stretching D_etaeta f / y'^2 - (y''/y'^2) D_y f."""
    d = d2(f, a, spacings(prob)[a], prob.bc[a])
    if a == 1 and stretched(prob):
        iyp, mq = y_metrics(prob)
        d = d * (iyp * iyp) + mq * deriv(prob, f, 1)
    return d


def density(c, p, s):
    """rho(p, s) = (p/p_ref)^(1/gamma) exp(-s/c_p)."""
    return (p / c.p_ref) ** (1.0 / c.gamma) * np.exp(-s / c.cp)


def temperature(c, p, rho):
    """T = p / (rho R)."""
    return p / (rho * c.R)


def viscosity(c, T):
    """Sutherland: mu(T) = mu_ref T^1.5 (1 + S)/(T + S)."""
    return c.mu_ref * T ** 1.5 * (1.0 + c.suth) / (T + c.suth)


def dviscosity(c, T):
    """mu'(T) = mu(T) (3/(2T) - 1/(T+S))."""
    return viscosity(c, T) * (1.5 / T - 1.0 / (T + c.suth))


def interior_mask(prob):
    """1.0 on rows the operator updates, 0.0 on wall rows (grid shape)."""
    nx, ny, nz = prob.n
    m = np.ones((ny, nx))
    if prob.bc[1] == BC_WALL:
        m[0, :] = 0.0
        m[-1, :] = 0.0
    if prob.ndim == 3:
        m = np.broadcast_to(m, (nz, ny, nx)).copy()
    return m


def rhs(prob, q):
    """N(q): the discrete right-hand side dq/dt = N(q) of eq. (navier_stokes).

    q has shape (..., nv, [Nz,] Ny, Nx) with variables (p, u, v, [w,] s);
    leading axes are a batch.  Works for real and complex q."""
    c = Constants(prob)
    nd = prob.ndim
    vax = -(nd + 1)
    q = np.asarray(q)
    p = np.take(q, 0, axis=vax)
    u = [np.take(q, 1 + i, axis=vax) for i in range(nd)]
    s = np.take(q, nd + 1, axis=vax)

    rho = density(c, p, s)
    T = temperature(c, p, rho)
    mu = viscosity(c, T)
    dmu = dviscosity(c, T)
    lam = c.cp * mu / c.pr
    dlam = c.cp * dmu / c.pr

    D = lambda f, a: deriv(prob, f, a)      # noqa: E731
    D2 = lambda f, a: deriv2(prob, f, a)    # noqa: E731

    Dp = [D(p, a) for a in range(nd)]
    Ds = [D(s, a) for a in range(nd)]
    DT = [D(T, a) for a in range(nd)]
    A = [[D(u[i], j) for j in range(nd)] for i in range(nd)]   # A[i][j] = D_j u_i
    theta = sum(A[k][k] for k in range(nd))
    LT = sum(D2(T, a) for a in range(nd))

    # viscous stress divergence, expanded form
    V = []
    for i in range(nd):
        Lu = sum(D2(u[i], a) for a in range(nd))
        G = D2(u[i], i)
        for j in range(nd):
            if j != i:
                G = G + D(A[j][j], i)          # D_i (D_j u_j)
        cross = sum(DT[j] * (A[i][j] + A[j][i]) for j in range(nd))
        V.append(mu * Lu + (mu / 3.0) * G + dmu * (cross - (2.0 / 3.0) * DT[i] * theta))

    Q = lam * LT + dlam * sum(DT[j] * DT[j] for j in range(nd))
    sij2 = 0.0
    for i in range(nd):
        for j in range(nd):
            sij = 0.5 * (A[i][j] + A[j][i])
            sij2 = sij2 + sij * sij
    Phi = mu * (2.0 * sij2 - (2.0 / 3.0) * theta * theta)
    heat = Q + Phi

    adv = lambda g: sum(u[j] * g[j] for j in range(nd))
    Np = -adv(Dp) - c.gamma * p * theta + (c.gamma - 1.0) * heat
    Nu = [-sum(u[j] * A[i][j] for j in range(nd)) - Dp[i] / rho + V[i] / rho
          for i in range(nd)]
    Ns = -adv(Ds) + heat / (rho * T)

    out = np.stack([Np] + Nu + [Ns], axis=vax)
    return out * interior_mask(prob)


def project(prob, v):
    """P: zero the wall rows of every variable."""
    return np.asarray(v) * interior_mask(prob)


def jv_cstep(prob, q0, v, h=1e-30):
    """Exact J(q0) v = d/de N(q0 + e P v)|_{e=0}, projected, by complex step.

    This is the linearised operator N_lin of eq. (frechet) without the
    truncation error of the finite quotient."""
    v = project(prob, v)
    return np.imag(rhs(prob, q0 + 1j * h * v)) / h


def jv_frechet(prob, q0, v, n0=None):
    """The paper's Frechet quotient, eq. (frechet):
        J v ~ [N(q0 + eps v) - N(q0)] / eps.
    The printed eps = ||q|| sqrt(eps_m) is read as eps = sqrt(eps_m)/||v||_2,
    which coincides with it for the unit vectors Krylov methods apply the
    operator to and keeps ||eps v|| at sqrt(eps_m).  N(q0) may be passed in
    (cached), so that each product costs one evaluation of N."""
    v = project(prob, v)
    nv = np.linalg.norm(v.ravel())
    if nv == 0.0:
        return np.zeros_like(v)
    eps = math.sqrt(EPS_MACHINE) / nv
    if n0 is None:
        n0 = rhs(prob, q0)
    return (rhs(prob, q0 + eps * v) - n0) / eps


def interior_index(prob):
    """Flat indices (into the full SoA vector) of the interior DOFs."""
    m = interior_mask(prob).ravel().astype(bool)
    full = np.tile(m, prob.nv)
    return np.nonzero(full)[0]


def dense_jacobian(prob, q0, batch=128, interior_only=True):
    """Brute-force dense J: column k is J e_k by complex step.

    With interior_only the rows and columns of wall DOFs (identically zero)
    are dropped, leaving the operator on the interior subspace."""
    idx = interior_index(prob) if interior_only else np.arange(prob.ndof)
    n = prob.ndof
    m = len(idx)
    J = np.empty((m, m))
    hstep = 1e-30
    for start in range(0, m, batch):
        cols = idx[start:start + batch]
        E = np.zeros((len(cols), n))
        E[np.arange(len(cols)), cols] = 1.0
        E = project(prob, E.reshape((len(cols),) + prob.shape))
        Y = np.imag(rhs(prob, q0[None] + 1j * hstep * E)) / hstep
        J[:, start:start + len(cols)] = Y.reshape(len(cols), n)[:, idx].T
    return J


def _colour_count(n, periodic, reach=3):
    """Smallest colour count c > 2*reach usable along an axis of n points
    (for a periodic axis c must divide n, else every point is its own colour)."""
    need = 2 * reach + 1
    if not periodic:
        return min(need, n)
    for c in range(need, n + 1):
        if n % c == 0:
            return c
    return n


def sparse_jacobian(prob, q0, reach=3):
    """J (all DOFs) as a scipy CSR matrix, from coloured complex-step probes:
    points whose indices agree modulo c_a (c_a > 2*reach) on every axis share
    a probe, so each row sees at most one probed column per probe."""
    import scipy.sparse as sp
    nd = prob.ndim
    dims = [prob.n[a] for a in range(nd)]
    periodic = [prob.bc[a] == BC_PERIODIC for a in range(nd)]
    cols = [_colour_count(dims[a], periodic[a], reach) for a in range(nd)]
    npts = prob.npts
    grids = np.meshgrid(*[np.arange(d) for d in dims[::-1]], indexing="ij")
    coord = [g.ravel() for g in grids[::-1]]           # coord[a] = index along axis a
    hstep = 1e-30
    rows_all, cols_all, vals_all = [], [], []
    import itertools
    for colour in itertools.product(*[range(c) for c in cols]):
        sel = np.ones(npts, dtype=bool)
        for a in range(nd):
            sel &= (coord[a] % cols[a]) == colour[a]
        # for every point, the probed point within reach along every axis
        src = np.zeros(npts, dtype=np.int64)
        valid = np.ones(npts, dtype=bool)
        strides = [1, prob.n[0], prob.n[0] * prob.n[1]]
        for a in range(nd):
            c = cols[a]
            off = (colour[a] - coord[a]) % c
            off = np.where(off > reach, off - c, off)       # in [-reach, reach] if reachable
            ok = np.abs(off) <= reach
            tgt = coord[a] + off
            if periodic[a]:
                tgt = tgt % dims[a]
            else:
                ok &= (tgt >= 0) & (tgt < dims[a])
            valid &= ok
            src += np.where(ok, tgt, 0) * strides[a]
        for var in range(prob.nv):
            e = np.zeros(prob.ndof)
            e[var * npts + np.nonzero(sel)[0]] = 1.0
            y = np.imag(rhs(prob, q0 + 1j * hstep * project(prob, e.reshape(prob.shape)))) / hstep
            y = y.reshape(prob.nv, npts)
            for ov in range(prob.nv):
                nz = valid & (y[ov] != 0.0)
                r = ov * npts + np.nonzero(nz)[0]
                cidx = var * npts + src[nz]
                rows_all.append(r)
                cols_all.append(cidx)
                vals_all.append(y[ov][nz])
    rows_all = np.concatenate(rows_all)
    cols_all = np.concatenate(cols_all)
    vals_all = np.concatenate(vals_all)
    return sp.csr_matrix((vals_all, (rows_all, cols_all)), shape=(prob.ndof, prob.ndof))
