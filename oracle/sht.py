"""Spherical-harmonic transform pair, plain FP64 (torch CPU).

Follows Sec. 3 of the paper:
  synthesis  xi(lambda, mu) = sum_{r=-R}^{R} sum_{s=|r|}^{R} xi^r_s P^r_s(mu) e^{i r lambda}
             (eq. spectral_to_physical_space)
  Fourier    xi^r(mu) = (1/I) sum_iota xi(lambda_iota, mu) e^{-i r lambda_iota}
             (eq. fourier_transform)
  Legendre   xi^r_s = sum_j xi^r(mu_j) P^r_s(mu_j) w_j   (eq. legendre_transform)

Readings (the paper leaves them open):
  * r is the zonal order m, s the degree n.
  * P^m_n is normalised so that int_{-1}^{1} (P^m_n)^2 dmu = 1, with no
    Condon-Shortley phase and P^{-m}_n = P^m_n; this is the normalisation for
    which the three formulas above are inverse to each other with the
    standard Gauss weights (sum w = 2).
  * Real fields store m >= 0 only, xi^{-m} = conj(xi^m), so the synthesis is
    Re xi_0 + 2 Re sum_{m>=1} xi_m e^{i m lambda}.
  * Longitudes lambda_i = 2 pi i / I, i = 0..I-1 (the same point set as the
    paper's iota = 1..I).
  * Latitudes ordered north to south.

Spectral storage: flat complex tensor, m-major: for m = 0..mmax the degrees
n = m..nmax follow each other.  Part of the test infrastructure.
"""
import math

import numpy as np
import torch

from .quadrature import gauss_legendre

DT = torch.float64
CT = torch.complex128


def nspec(N, nmax=None):
    """Number of stored coefficients for m = 0..N, n = m..nmax (nmax >= N)."""
    nmax = N if nmax is None else nmax
    return sum(nmax + 1 - m for m in range(N + 1))


def mstart(N, m, nmax=None):
    """Flat index of (m, n = m)."""
    nmax = N if nmax is None else nmax
    return sum(nmax + 1 - k for k in range(m))


def degrees(N, nmax=None):
    """Degree n of every flat entry (int64 tensor)."""
    nmax = N if nmax is None else nmax
    return torch.cat([torch.arange(m, nmax + 1) for m in range(N + 1)])


def orders(N, nmax=None):
    """Zonal order m of every flat entry (int64 tensor)."""
    nmax = N if nmax is None else nmax
    return torch.cat([torch.full((nmax + 1 - m,), m) for m in range(N + 1)])


def split_m(flat, N, nmax=None):
    """List over m of the views flat[..., m-block] (degrees m..nmax)."""
    nmax = N if nmax is None else nmax
    out, s = [], 0
    for m in range(N + 1):
        c = nmax + 1 - m
        out.append(flat[..., s:s + c])
        s += c
    return out


def eps(n, m):
    """epsilon^m_n = sqrt((n^2 - m^2) / (4 n^2 - 1)); zero for n <= m."""
    if n <= m:
        return 0.0
    return math.sqrt((n * n - m * m) / (4.0 * n * n - 1.0))


def legendre_m(m, nmax, mu, sin_theta):
    """Normalised associated Legendre functions P^m_n(mu_j), n = m..nmax.

    Returns a float64 numpy array of shape (nmax + 1 - m, J).
    Recurrences (standard for the orthonormal functions):
      P^0_0 = 1/sqrt(2),
      P^m_m = sqrt((2m+1)/(2m)) sin(theta) P^{m-1}_{m-1},
      P^m_{m+1} = sqrt(2m+3) mu P^m_m,
      P^m_n = (mu P^m_{n-1} - eps^m_{n-1} P^m_{n-2}) / eps^m_n.
    The recurrence runs in extended precision (x87 long double, 64-bit
    significand) from the FP64 values of mu and sin(theta), and the result is
    rounded to FP64: run in FP64 it accumulates relative errors of several
    1e-13 by degree 1000, which the factor n(n+1) of the Laplacian turns into
    errors near 1e-10 in the divergence tendency at T1023.
    """
    LD = np.longdouble
    mu = np.asarray(mu, dtype=np.float64).astype(LD)
    st = np.asarray(sin_theta, dtype=np.float64).astype(LD)
    out = np.zeros((max(nmax + 1 - m, 0), mu.size), dtype=LD)
    if nmax < m:
        return out.astype(np.float64)

    def e(n):
        if n <= m:
            return LD(0)
        return np.sqrt(LD(n * n - m * m) / LD(4 * n * n - 1))

    pmm = np.full_like(mu, np.sqrt(LD(1) / LD(2)))
    for k in range(1, m + 1):
        pmm = pmm * (np.sqrt(LD(2 * k + 1) / LD(2 * k)) * st)
    out[0] = pmm
    if nmax >= m + 1:
        out[1] = np.sqrt(LD(2 * m + 3)) * mu * pmm
    for n in range(m + 2, nmax + 1):
        out[n - m] = (mu * out[n - m - 1] - e(n - 1) * out[n - m - 2]) / e(n)
    return out.astype(np.float64)


class Grid:
    """Triangular truncation T_N on a Gaussian grid with I longitudes and J latitudes.

    Holds mu_j, sin(theta_j), 1 - mu_j^2, w_j (from oracle.quadrature) and the
    table P[m] of shape (nmax + 1 - m, J) with nmax = N + 1 (the vector
    fields of the tendency reach degree N + 1).
    """

    def __init__(self, N, J, I):
        self.N, self.J, self.I = N, J, I
        mu, st, c2, w = gauss_legendre(J)
        self.mu = torch.tensor(mu, dtype=DT)
        self.sin_theta = torch.tensor(st, dtype=DT)
        self.cos2phi = torch.tensor(c2, dtype=DT)
        self.w = torch.tensor(w, dtype=DT)
        self.P = [torch.tensor(legendre_m(m, N + 1, mu, st), dtype=DT) for m in range(N + 1)]
        self.lam = 2.0 * math.pi * torch.arange(I, dtype=DT) / I

    # -- Legendre step -------------------------------------------------
    def legendre_synthesis(self, spec, nmax=None):
        """xi_m(mu_j) = sum_{n=m}^{nmax} xi^m_n P^m_n(mu_j).

        spec: [..., nspec(N, nmax)] complex -> [..., J, N+1] complex.
        """
        N = self.N
        nmax = N if nmax is None else nmax
        blocks = split_m(spec, N, nmax)
        cols = []
        for m in range(N + 1):
            Pm = self.P[m][: nmax + 1 - m].to(CT)          # (deg, J)
            cols.append(blocks[m] @ Pm)                      # [..., J]
        return torch.stack(cols, dim=-1)

    def legendre_analysis(self, four, weights, nmax=None):
        """xi^m_n = sum_j weights_j xi_m(mu_j) P^m_n(mu_j), n = m..nmax.

        four: [..., J, N+1] complex, weights: [J] -> [..., nspec(N, nmax)].
        """
        N = self.N
        nmax = N if nmax is None else nmax
        out = []
        for m in range(N + 1):
            Pm = self.P[m][: nmax + 1 - m].to(CT)          # (deg, J)
            g = four[..., :, m] * weights.to(CT)             # [..., J]
            out.append(g @ Pm.transpose(0, 1))               # [..., deg]
        return torch.cat(out, dim=-1)

    # -- Fourier step --------------------------------------------------
    def fourier_synthesis(self, four):
        """grid = Re xi_0 + 2 Re sum_{m=1}^{N} xi_m e^{i m lambda_i}.

        four: [..., J, N+1] -> grid [..., J, I].  Uses the inverse real FFT
        (x_i = (1/I) sum over the Hermitian spectrum), scaled by I.
        """
        I = self.I
        assert 2 * self.N < I
        pad = torch.zeros(four.shape[:-1] + (I // 2 + 1,), dtype=CT)
        pad[..., : self.N + 1] = four
        pad[..., 0] = pad[..., 0].real.to(CT)
        return torch.fft.irfft(pad, n=I, dim=-1) * I

    def fourier_analysis(self, grid):
        """xi_m(mu_j) = (1/I) sum_i grid(lambda_i, mu_j) e^{-i m lambda_i}, m = 0..N."""
        return torch.fft.rfft(grid, dim=-1)[..., : self.N + 1] / self.I

    # -- the pair ------------------------------------------------------
    def sh_inverse(self, spec, nmax=None):
        """Spectral [..., nspec] -> grid [..., J, I] (eq. spectral_to_physical_space)."""
        return self.fourier_synthesis(self.legendre_synthesis(spec, nmax))

    def sh_forward(self, grid, nmax=None):
        """Grid [..., J, I] -> spectral [..., nspec] (eqs. fourier_transform, legendre_transform)."""
        return self.legendre_analysis(self.fourier_analysis(grid), self.w, nmax)


def truncate(spec, N_from, N_to):
    """Spectral truncation D (Sec. 4.3.3, eq. space_restriction): keep m, n <= N_to."""
    blocks = split_m(spec, N_from)
    return torch.cat([blocks[m][..., : N_to + 1 - m] for m in range(N_to + 1)], dim=-1)


def zero_pad(spec, N_from, N_to):
    """Spectral zero-padding P^s = D^T (Sec. 4.3.3)."""
    blocks = split_m(spec, N_from)
    out = []
    for m in range(N_to + 1):
        z = torch.zeros(spec.shape[:-1] + (N_to + 1 - m,), dtype=spec.dtype)
        if m <= N_from:
            z[..., : N_from + 1 - m] = blocks[m]
        out.append(z)
    return torch.cat(out, dim=-1)
