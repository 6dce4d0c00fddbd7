"""Shallow-water right-hand sides and the implicit solve, plain FP64.

Equations: Sec. 2, eqs. geopotential_equation, vorticity_equation,
divergence_equation, with the split of eq. linear_nonlinear_decomposition
into L_G (eq. linear_wave_motion_induced_by_gravitational_forces), L_F (eq.
linear_harmonic_oscillator_on_the_velocity_components) and N (eq.
nonlinear_operators).  IMEX split (Sec. 4.1, eqs. system_of_odes_implicit_part
and system_of_odes_explicit_part): F_I = L_G, F_E = L_F + N.

The paper defers the spectral form of the right-hand side to other work; the
reading used here (derived from the equations above, see the docstrings):

  L_n = n(n+1)/a^2;  psi = -zeta/L_n, chi = -delta/L_n (n >= 1; 0 for n = 0)
  cos-weighted wind U = u cos(phi), V = v cos(phi) (Sec. 2, eq. helmholtz_theorem):
    U^m_n = [(n-1) eps^m_n psi^m_{n-1} - (n+2) eps^m_{n+1} psi^m_{n+1} + i m chi^m_n] / a
    V^m_n = [i m psi^m_n - (n-1) eps^m_n chi^m_{n-1} + (n+2) eps^m_{n+1} chi^m_{n+1}] / a
    for n = m..N+1.
  grid products: eta = zeta + 2 Omega mu,  A = eta U, B = eta V, C = Phi' U,
    D = Phi' V, E = (U^2 + V^2) / (2 cos^2 phi).
  analyses: X^_n = sum_j w_j/(1-mu_j^2) X_m(mu_j) P^m_n(mu_j) for X in {A,B,C,D}
    (n <= N+1), E^_n with weights w_j (n <= N).
  divergence / curl of a cos-weighted vector (X east, Y north):
    div_n  = [i m X^_n + n eps_{n+1} Y^_{n+1} - (n+1) eps_n Y^_{n-1}] / a
    curl_n = [i m Y^_n - n eps_{n+1} X^_{n+1} + (n+1) eps_n X^_{n-1}] / a
  F_E = [-div(C, D), -div(A, B), curl(A, B) + L_n E^]
  F_I = [-Phibar delta - nu L Phi', -nu L zeta, L Phi' - nu L delta]

State ordering (Phi', zeta, delta), as U = [Phi, zeta, delta] in Sec. 2.
Part of the test infrastructure.
"""
from dataclasses import dataclass

import torch

from .sht import CT, DT, Grid, degrees, eps, split_m


@dataclass(frozen=True)
class SWEParams:
    a: float = 6.37122e6
    omega: float = 7.292e-5
    g: float = 9.80616
    phibar: float = 2.94e4
    nu: float = 1.0e5


def lap_eig(N, a, nmax=None):
    """L_n = n(n+1)/a^2 for every flat entry (so that nabla^2 -> -L_n)."""
    n = degrees(N, nmax).to(DT)
    return n * (n + 1.0) / (a * a)


def _eps_vec(m, n0, n1):
    """eps^m_n for n = n0..n1 as a float64 tensor."""
    return torch.tensor([eps(n, m) for n in range(n0, n1 + 1)], dtype=DT)


def velocity_coeffs(zeta, delta, N, a):
    """Spectral coefficients of U = u cos(phi), V = v cos(phi), degrees m..N+1.

    Follows the Helmholtz decomposition V = k x grad psi + grad chi
    (Sec. 2, eq. helmholtz_theorem) with zeta = lap psi, delta = lap chi,
    u cos(phi) = [-(1-mu^2) psi_mu + chi_lambda]/a,
    v cos(phi) = [psi_lambda + (1-mu^2) chi_mu]/a, and
    (1-mu^2) dP^m_n/dmu = -n eps^m_{n+1} P^m_{n+1} + (n+1) eps^m_n P^m_{n-1}.
    Returns two flat tensors in the degree-(N+1) layout.
    """
    L = lap_eig(N, a)
    inv = torch.where(L > 0, 1.0 / torch.where(L > 0, L, torch.ones_like(L)), torch.zeros_like(L))
    ps = split_m(-zeta * inv, N)
    ch = split_m(-delta * inv, N)
    U, V = [], []
    for m in range(N + 1):
        n = torch.arange(m, N + 2, dtype=DT)                 # output degrees m..N+1
        c_dn = (n - 1.0) * _eps_vec(m, m, N + 1)             # (n-1) eps_n
        c_up = (n + 2.0) * _eps_vec(m, m + 1, N + 2)         # (n+2) eps_{n+1}
        z = torch.zeros(ps[m].shape[:-1] + (1,), dtype=CT)
        # padded copies: index k+1 holds degree m+k; degrees m-1, N+1, N+2 are 0
        pp = torch.cat([z, ps[m], z, z], dim=-1)
        cp = torch.cat([z, ch[m], z, z], dim=-1)
        cnt = N + 2 - m
        p_dn, p_0, p_up = pp[..., 0:cnt], pp[..., 1:cnt + 1], pp[..., 2:cnt + 2]
        c_dn_, c_0, c_up_ = cp[..., 0:cnt], cp[..., 1:cnt + 1], cp[..., 2:cnt + 2]
        U.append((c_dn * p_dn - c_up * p_up + (1j * m) * c_0) / a)
        V.append(((1j * m) * p_0 - c_dn * c_dn_ + c_up * c_up_) / a)
    return torch.cat(U, dim=-1), torch.cat(V, dim=-1)


def div_curl(X, Y, N, a):
    """Divergence and curl (degrees n <= N) of the vector whose cos-weighted
    components have weighted analyses X^, Y^ (degrees m..N+1).

    Obtained from div = [d_lambda X + (1-mu^2) d_mu Y] / (a (1-mu^2)) and
    curl = [d_lambda Y - (1-mu^2) d_mu X] / (a (1-mu^2)) by projecting on
    P^m_n e^{i m lambda} and integrating by parts in mu (the cos-weighted
    components vanish at the poles).
    """
    Xs = split_m(X, N, N + 1)
    Ys = split_m(Y, N, N + 1)
    dv, cl = [], []
    for m in range(N + 1):
        n = torch.arange(m, N + 1, dtype=DT)                 # output degrees m..N
        c_up = n * _eps_vec(m, m + 1, N + 1)                 # n eps_{n+1}
        c_dn = (n + 1.0) * _eps_vec(m, m, N)                 # (n+1) eps_n
        cnt = N + 1 - m
        z = torch.zeros(Xs[m].shape[:-1] + (1,), dtype=CT)
        xp = torch.cat([z, Xs[m]], dim=-1)                   # index k+1 holds degree m+k
        yp = torch.cat([z, Ys[m]], dim=-1)
        x0, x_up, x_dn = xp[..., 1:cnt + 1], xp[..., 2:cnt + 2], xp[..., 0:cnt]
        y0, y_up, y_dn = yp[..., 1:cnt + 1], yp[..., 2:cnt + 2], yp[..., 0:cnt]
        dv.append(((1j * m) * x0 + c_up * y_up - c_dn * y_dn) / a)
        cl.append(((1j * m) * y0 - c_up * x_up + c_dn * x_dn) / a)
    return torch.cat(dv, dim=-1), torch.cat(cl, dim=-1)


def grid_fields(state, grid: Grid, p: SWEParams):
    """Synthesised grid fields (zeta, Phi', U, V) of a state [..., 3, nspec]."""
    N = grid.N
    phi, zeta, delta = state[..., 0, :], state[..., 1, :], state[..., 2, :]
    U, V = velocity_coeffs(zeta, delta, N, p.a)
    zg = grid.sh_inverse(zeta)
    pg = grid.sh_inverse(phi)
    ug = grid.sh_inverse(U, N + 1)
    vg = grid.sh_inverse(V, N + 1)
    return zg, pg, ug, vg


def f_explicit(state, grid: Grid, p: SWEParams):
    """F_E = L_F + N (Sec. 4.1, eq. system_of_odes_explicit_part), spectral."""
    N = grid.N
    zg, pg, ug, vg = grid_fields(state, grid, p)
    f = 2.0 * p.omega * grid.mu[:, None]
    eta = zg + f
    A = eta * ug
    B = eta * vg
    C = pg * ug
    D = pg * vg
    E = (ug * ug + vg * vg) / (2.0 * grid.cos2phi[:, None])
    wv = grid.w / grid.cos2phi
    Ah = grid.legendre_analysis(grid.fourier_analysis(A), wv, N + 1)
    Bh = grid.legendre_analysis(grid.fourier_analysis(B), wv, N + 1)
    Ch = grid.legendre_analysis(grid.fourier_analysis(C), wv, N + 1)
    Dh = grid.legendre_analysis(grid.fourier_analysis(D), wv, N + 1)
    Eh = grid.legendre_analysis(grid.fourier_analysis(E), grid.w, N)
    div_ab, curl_ab = div_curl(Ah, Bh, N, p.a)
    div_cd, _ = div_curl(Ch, Dh, N, p.a)
    L = lap_eig(N, p.a)
    return torch.stack([-div_cd, -div_ab, curl_ab + L * Eh], dim=-2)


def f_implicit(state, N, p: SWEParams):
    """F_I = L_G (Sec. 2, eq. linear_wave_motion_induced_by_gravitational_forces)
    with nabla^2 -> -L_n."""
    L = lap_eig(N, p.a)
    phi, zeta, delta = state[..., 0, :], state[..., 1, :], state[..., 2, :]
    return torch.stack([-p.phibar * delta - p.nu * L * phi,
                        -p.nu * L * zeta,
                        L * phi - p.nu * L * delta], dim=-2)


def imex_solve(b, h, N, p: SWEParams):
    """Solve Theta - h F_I(Theta) = b (Sec. 4.4, eq. implicit_systems).

    Per coefficient, with c = 1 + h nu L_n: the geopotential first,
      Phi' = (c b_Phi - h Phibar b_delta) / (c^2 + h^2 Phibar L_n),
    then delta = (b_delta + h L_n Phi') / c and zeta = b_zeta / c.
    """
    L = lap_eig(N, p.a)
    c = 1.0 + h * p.nu * L
    bphi, bzeta, bdelta = b[..., 0, :], b[..., 1, :], b[..., 2, :]
    phi = (c * bphi - h * p.phibar * bdelta) / (c * c + h * h * p.phibar * L)
    delta = (bdelta + h * L * phi) / c
    zeta = bzeta / c
    return torch.stack([phi, zeta, delta], dim=-2)


class SWEProblem:
    """The semi-discrete system dTheta/dt = F_I + F_E (Sec. 3, eq.
    semidiscrete_system) on one spectral level, as seen by the SDC sweep."""

    def __init__(self, N, J, I, params: SWEParams = SWEParams()):
        self.N = N
        self.grid = Grid(N, J, I)
        self.p = params
        self.n_eval = 0
        self.n_solve = 0

    def evaluate(self, theta):
        self.n_eval += 1
        return f_implicit(theta, self.N, self.p), f_explicit(theta, self.grid, self.p)

    def solve(self, b, h):
        self.n_solve += 1
        return imex_solve(b, h, self.N, self.p)
