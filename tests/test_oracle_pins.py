"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one oracle function against something other than itself:
closed forms, library routines, invariants, brute force, or numbers printed
in the paper (tests/golden/paper_numbers.json).  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps
import torch

from oracle import quadrature as Qd
from oracle import sdc, sht, swe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CT, DT = sht.CT, sht.DT


def rand_spec(N, gen, nmax=None, zero_n0=True):
    n = sht.nspec(N, nmax)
    x = torch.randn(n, dtype=DT, generator=gen) + 1j * torch.randn(n, dtype=DT, generator=gen)
    x = torch.where(sht.orders(N, nmax) == 0, x.real.to(CT), x)
    if zero_n0:
        x[0] = 0
    return x


def relerr(a, b):
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


# ---------------------------------------------------------------- Gauss latitudes
def test_gauss_closed_forms():
    mu, st, c2, w = Qd.gauss_legendre(2)
    assert np.allclose(mu, [1 / math.sqrt(3), -1 / math.sqrt(3)], atol=2.3e-16, rtol=0)
    assert np.allclose(w, [1, 1], atol=2e-16, rtol=0)
    mu, st, c2, w = Qd.gauss_legendre(3)
    assert np.allclose(mu, [math.sqrt(0.6), 0, -math.sqrt(0.6)], atol=2e-16, rtol=0)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=2e-16, rtol=0)


@pytest.mark.parametrize("J", [48, 96, 192])
def test_gauss_exactness_and_library(J):
    mu, st, c2, w = Qd.gauss_legendre(J)
    assert np.all(np.diff(mu) < 0)                         # north to south
    assert np.allclose(st ** 2, c2, rtol=1e-15, atol=0)
    assert np.allclose(st ** 2 + mu ** 2, 1.0, atol=3e-16, rtol=0)
    for k in range(0, 2 * J, 7):                           # exact up to degree 2J-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, mu ** k) - exact) < 1e-14
    x, ww = np.polynomial.legendre.leggauss(J)
    assert np.abs(np.sort(mu) - x).max() < 1e-15
    assert np.abs(np.sort(w) - np.sort(ww)).max() < 1e-12 * ww.max()


@pytest.mark.parametrize("J", [768, 1536])
def test_gauss_exactness_large(J, oracle_gauss):
    """The latitude counts of the T511 and T1023 grids: monomials up to degree
    2J-1 and the orthogonality of the Legendre polynomials P_0..P_{J-1} (Bonnet's
    recurrence in FP64; every product has degree <= 2J-2) hold to rounding."""
    mu, st, c2, w = oracle_gauss(J)
    assert np.all(np.diff(mu) < 0)
    assert np.allclose(st ** 2 + mu ** 2, 1.0, atol=3e-16, rtol=0)
    assert np.array_equal(mu, -mu[::-1]) and np.array_equal(w, w[::-1])
    for k in range(0, 2 * J, 7):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, mu ** k) - exact) < 1e-14
    P = np.zeros((J, J))
    P[0], P[1] = 1.0, mu
    for n in range(1, J - 1):
        P[n + 1] = ((2 * n + 1) * mu * P[n] - n * P[n - 1]) / (n + 1)
    G = (P * w) @ P.T
    assert np.abs(G - np.diag(2.0 / (2 * np.arange(J) + 1))).max() < 5e-15
    x, _ = np.polynomial.legendre.leggauss(J)
    assert np.abs(np.sort(mu) - x).max() < 1e-15


# ---------------------------------------------------------------- Legendre functions
def test_plm_closed_forms():
    mu, st, _, _ = Qd.gauss_legendre(11)
    P0 = sht.legendre_m(0, 2, mu, st)
    P1 = sht.legendre_m(1, 1, mu, st)
    assert np.allclose(P0[0], 1 / math.sqrt(2), atol=1e-16)
    assert np.allclose(P0[1], math.sqrt(1.5) * mu, atol=1e-15)
    assert np.allclose(P0[2], math.sqrt(2.5) * (3 * mu ** 2 - 1) / 2, atol=1e-15)
    assert np.allclose(P1[0], math.sqrt(3) / 2 * st, atol=1e-15)


def test_plm_vs_scipy():
    """scipy's lpmv carries the Condon-Shortley phase and no normalisation."""
    J = 40
    mu, st, _, _ = Qd.gauss_legendre(J)
    for m in range(0, 25):
        P = sht.legendre_m(m, 40, mu, st)
        for n in range(m, 41):
            norm = math.sqrt((2 * n + 1) / 2 * math.exp(math.lgamma(n - m + 1) - math.lgamma(n + m + 1)))
            ref = (-1) ** m * norm * sps.lpmv(m, n, mu)
            assert np.abs(P[n - m] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_plm_high_degree_accuracy():
    """At the degrees of T1023 the tabulated values match the same recurrence
    run in 50-digit arithmetic (mpmath) on the same FP64 inputs mu and
    sin(theta) to 3e-15 of the column's largest value (the recurrence itself
    is pinned by the closed forms and scipy above).  The forward recurrence
    amplifies rounding errors roughly like n^2 near the poles: run in FP64 it
    is off by about 1e-12 of the column maximum at degree 1023 next to the
    pole, in long double by about 1e-15."""
    from mpmath import mp
    mu = np.array([0.9999987751809604, 0.7071067811865476, 0.31415926535897931, 0.001])
    with mp.workdps(50):
        st = np.array([float(mp.sqrt(1 - mp.mpf(float(x)) ** 2)) for x in mu])
        for m in (0, 1, 300, 900):
            P = sht.legendre_m(m, 1024, mu, st)
            for j in range(mu.size):
                scale = np.abs(P[:, j]).max()
                x, s = mp.mpf(float(mu[j])), mp.mpf(float(st[j]))
                pmm = 1 / mp.sqrt(2)
                for k in range(1, m + 1):
                    pmm *= mp.sqrt(mp.mpf(2 * k + 1) / (2 * k)) * s
                ref = [pmm, mp.sqrt(2 * m + 3) * x * pmm]
                e = [mp.mpf(0)] * 1025
                for n in range(m + 1, 1025):
                    e[n] = mp.sqrt(mp.mpf(n * n - m * m) / (4 * n * n - 1))
                for n in range(m + 2, 1025):
                    ref.append((x * ref[-1] - e[n - 1] * ref[-2]) / e[n])
                err = max(abs(P[k, j] - float(ref[k])) for k in range(len(ref)))
                assert err <= 3e-15 * scale, (m, j, err, scale)


def test_plm_discrete_orthonormality():
    N, J = 63, 96
    mu, st, _, w = Qd.gauss_legendre(J)
    for m in (0, 1, 17, 40, 63):
        P = sht.legendre_m(m, N, mu, st)
        G = (P * w) @ P.T
        assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


def test_plm_parity():
    mu, st, _, _ = Qd.gauss_legendre(50)
    for m in (0, 3, 20):
        P = sht.legendre_m(m, 40, mu, st)
        sign = np.array([(-1) ** k for k in range(P.shape[0])])[:, None]
        assert np.abs(P[:, ::-1] - sign * P).max() < 1e-13


# ---------------------------------------------------------------- transforms
@pytest.mark.parametrize("N,J,I", [(31, 48, 96), (63, 96, 192)])
def test_sh_roundtrip_and_fft(N, J, I):
    gen = torch.Generator().manual_seed(N)
    g = sht.Grid(N, J, I)
    x = rand_spec(N, gen, zero_n0=False)
    grid = g.sh_inverse(x)
    assert relerr(g.sh_forward(grid), x) < 1e-14
    # Fourier step against numpy's real FFT
    X = g.fourier_analysis(grid).numpy()
    ref = np.fft.rfft(grid.numpy(), axis=-1)[..., : N + 1] / I
    assert np.abs(X - ref).max() < 1e-15 * np.abs(ref).max()


def test_sh_inverse_brute_force():
    """Synthesis against a direct sum over (m, n) at a few points."""
    N, J, I = 12, 20, 40
    gen = torch.Generator().manual_seed(3)
    g = sht.Grid(N, J, I)
    x = rand_spec(N, gen, zero_n0=False)
    grid = g.sh_inverse(x).numpy()
    mu, st, _, _ = Qd.gauss_legendre(J)
    xs = x.numpy()
    for j in (0, 7, 19):
        for i in (0, 5, 33):
            lam = 2 * math.pi * i / I
            val = 0.0
            for m in range(N + 1):
                n = np.arange(m, N + 1)
                norm = np.sqrt((2 * n + 1) / 2 * np.exp(sps.gammaln(n - m + 1) - sps.gammaln(n + m + 1)))
                Pnm = (-1) ** m * norm * sps.lpmv(m, n, mu[j])
                c = np.sum(xs[sht.mstart(N, m): sht.mstart(N, m) + N + 1 - m] * Pnm)
                val += (c.real if m == 0 else 2 * (c * np.exp(1j * m * lam)).real)
            assert abs(grid[j, i] - val) < 1e-13


# ---------------------------------------------------------------- vector calculus
@pytest.fixture(scope="module")
def t31():
    return sht.Grid(31, 48, 96)


def _vector_analyses(g, U, V):
    N = g.N
    wv = g.w / g.cos2phi
    ug, vg = g.sh_inverse(U, N + 1), g.sh_inverse(V, N + 1)
    return (g.legendre_analysis(g.fourier_analysis(ug), wv, N + 1),
            g.legendre_analysis(g.fourier_analysis(vg), wv, N + 1))


def test_laplacian_eigenvalues(t31):
    """div(grad chi) = -L chi, curl(grad chi) = 0, curl(k x grad psi) = -L psi,
    div(k x grad psi) = 0, with L = n(n+1)/a^2."""
    N, a = 31, swe.SWEParams().a
    gen = torch.Generator().manual_seed(11)
    L = swe.lap_eig(N, a)
    chi = rand_spec(N, gen)
    psi = rand_spec(N, gen)
    zero = torch.zeros_like(chi)
    U, V = swe.velocity_coeffs(zero, -L * chi, N, a)
    d, c = swe.div_curl(*_vector_analyses(t31, U, V), N, a)
    s = torch.linalg.vector_norm(L * chi)
    assert torch.linalg.vector_norm(d + L * chi) / s < 1e-13
    assert torch.linalg.vector_norm(c) / s < 1e-13
    U, V = swe.velocity_coeffs(-L * psi, zero, N, a)
    d, c = swe.div_curl(*_vector_analyses(t31, U, V), N, a)
    s = torch.linalg.vector_norm(L * psi)
    assert torch.linalg.vector_norm(c + L * psi) / s < 1e-13
    assert torch.linalg.vector_norm(d) / s < 1e-13


def test_velocity_from_stream_function_pointwise(t31):
    """u = -(1/a) dpsi/dphi for a zonal stream function psi = c P^0_1 (closed form)."""
    N, a = 31, swe.SWEParams().a
    psi = torch.zeros(sht.nspec(N), dtype=CT)
    psi[1] = 1e6
    L = swe.lap_eig(N, a)
    U, V = swe.velocity_coeffs(-L * psi, torch.zeros_like(psi), N, a)
    ug = t31.sh_inverse(U, N + 1)
    # psi = 1e6 sqrt(3/2) mu -> U = u cos(phi) = -(1-mu^2) psi_mu / a
    expect = -(t31.cos2phi * 1e6 * math.sqrt(1.5)) / a
    assert torch.abs(ug - expect[:, None]).max() < 1e-14 * expect.abs().max()
    assert torch.abs(t31.sh_inverse(V, N + 1)).max() < 1e-20


# ---------------------------------------------------------------- tendencies
def test_rigid_rotation_closed_form(t31):
    """zeta = Z mu, delta = Phi' = 0: F_E vanishes except the (n=2, m=0)
    divergence coefficient 2 (Z^2/4 + Omega Z) / sqrt(5/2)."""
    N, p = 31, swe.SWEParams()
    Z = 1.3e-5
    st = torch.zeros(3, sht.nspec(N), dtype=CT)
    st[1, 1] = Z / math.sqrt(1.5)
    fe = swe.f_explicit(st, t31, p)
    expect = 2 * (Z * Z / 4 + p.omega * Z) / math.sqrt(2.5)
    assert abs(fe[2, 2].item() - expect) < 1e-13 * abs(expect)
    fe[2, 2] = 0
    assert fe.abs().max().item() < 1e-13 * abs(expect)


# Closed forms of the two flux rows of F_E (Sec. 2, eqs. geopotential_equation
# and vorticity_equation; Sec. 4.1, eq. system_of_odes_explicit_part).  Each
# helper returns the relative deviation of `fexp` (an F_E implementation with
# the signature of swe.f_explicit) from the closed form, so that the same
# checks can be run against a deliberately broken copy below.
def _flux_pin_solid_body(fexp, g):
    """Solid-body wind zeta = 2 w mu (u = w a cos(phi), v = 0), delta = 0, any
    band-limited Phi': the flux divergence is pure advection in longitude,
    -div(Phi' V) = -w dPhi'/dlambda, so F_E,Phi = -i m w Phi'^m_n."""
    N, p = g.N, swe.SWEParams()
    w = 1.0e-5
    gen = torch.Generator().manual_seed(21)
    st = torch.zeros(3, sht.nspec(N), dtype=CT)
    st[0] = 100.0 * rand_spec(N, gen)
    st[1, 1] = 2.0 * w / math.sqrt(1.5)                  # zeta = 2 w mu
    expect = -1j * sht.orders(N).to(DT) * w * st[0]
    return relerr(fexp(st, g, p)[0], expect)


def _flux_pin_constant_geopotential(fexp, g):
    """Phi' = c P^0_0 = c/sqrt(2) (constant), any zeta and delta:
    -div(Phi' V) = -(c/sqrt(2)) div V, so F_E,Phi = -(c/sqrt(2)) delta."""
    N, p = g.N, swe.SWEParams()
    c = 300.0
    gen = torch.Generator().manual_seed(22)
    st = torch.zeros(3, sht.nspec(N), dtype=CT)
    st[0, 0] = c
    st[1] = 1e-5 * rand_spec(N, gen)
    st[2] = 1e-6 * rand_spec(N, gen)
    expect = -(c / math.sqrt(2.0)) * st[2]
    return relerr(fexp(st, g, p)[0], expect)


def _flux_pin_divergent_coriolis(fexp, g):
    """delta = D P^0_1, zeta = Phi' = 0: chi = -D a^2 sqrt(3/2) mu / 2, the
    cos-weighted northward wind is V = -D a sqrt(3/2) (1 - mu^2)/2, and with
    eta = 2 Omega mu, -div(eta V) = -Omega D sqrt(3/2) (3 mu^2 - 1): a single
    (n = 2, m = 0) coefficient -2 Omega D sqrt(3/5) of F_E,zeta; F_E,Phi = 0."""
    N, p = g.N, swe.SWEParams()
    D = 2.0e-6
    st = torch.zeros(3, sht.nspec(N), dtype=CT)
    st[2, 1] = D
    expect = torch.zeros(sht.nspec(N), dtype=CT)
    expect[2] = -2.0 * p.omega * D * math.sqrt(0.6)
    fe = fexp(st, g, p)
    return max(relerr(fe[1], expect), fe[0].abs().max().item() / abs(expect[2].item()))


FLUX_PINS = [_flux_pin_solid_body, _flux_pin_constant_geopotential, _flux_pin_divergent_coriolis]


@pytest.mark.parametrize("pin", FLUX_PINS, ids=lambda f: f.__name__[10:])
def test_flux_rows_closed_forms(pin, t31):
    assert pin(swe.f_explicit, t31) < 1e-13


@pytest.mark.parametrize("row", [0, 1])
def test_flux_pins_detect_a_sign_error(row, t31):
    """A planted mistake in the oracle (one flux row of F_E negated) fails at
    least one of the closed-form pins above."""
    def broken(st, g, p):
        fe = swe.f_explicit(st, g, p).clone()
        fe[..., row, :] = -fe[..., row, :]
        return fe
    assert max(pin(broken, t31) for pin in FLUX_PINS) > 1e-3


def _seeded_state(N, seed, wind=1e-5, phi=100.0):
    import workload
    raw = torch.tensor(workload.raw_spectrum(N, seed))
    raw[0] *= phi
    raw[1:] *= wind
    return raw


def test_grid_independence():
    """F_E on the alias-free grid equals F_E on a finer Gauss grid (exact quadrature)."""
    N = 31
    st = _seeded_state(N, 5)
    p = swe.SWEParams()
    fe1 = swe.f_explicit(st, sht.Grid(N, 48, 96), p)
    fe2 = swe.f_explicit(st, sht.Grid(N, 72, 144), p)
    for f in range(3):
        assert relerr(fe1[f], fe2[f]) < 1e-12


def test_zonal_shift_equivariance(t31):
    """Rotating the state by one grid spacing in longitude rotates F_E the same way."""
    N, p = 31, swe.SWEParams()
    st = _seeded_state(N, 6)
    ph = torch.exp(-1j * sht.orders(N).to(DT) * (2 * math.pi / 96))
    fe = swe.f_explicit(st, t31, p)
    fe_s = swe.f_explicit(st * ph, t31, p)
    for f in range(3):
        assert relerr(fe_s[f], fe[f] * ph) < 1e-13


def test_global_means_of_tendencies(t31):
    """n = 0 coefficients of F_E and F_I vanish (global integrals of div/curl/lap)."""
    N, p = 31, swe.SWEParams()
    st = _seeded_state(N, 7)
    fe = swe.f_explicit(st, t31, p)
    fi = swe.f_implicit(st, N, p)
    scale = fe.abs().max().item()
    assert fe[:, 0].abs().max().item() < 1e-13 * scale
    assert fi[:, 0].abs().max().item() == 0.0


def test_imex_solve_inverts_implicit_operator():
    N, p = 31, swe.SWEParams()
    gen = torch.Generator().manual_seed(2)
    b = torch.stack([rand_spec(N, gen) * 100, rand_spec(N, gen) * 1e-5, rand_spec(N, gen) * 1e-5])
    for h in (0.0, 37.5, 600.0):
        x = swe.imex_solve(b, h, N, p)
        r = x - h * swe.f_implicit(x, N, p) - b
        for f in range(3):
            assert relerr(r[f] + b[f], b[f]) < 1e-14


def test_linear_gravity_waves_reach_pade():
    """With F_E switched off each (n, m) evolves by d/dt (Phi', delta) = A_n
    (Phi', delta), A_n = [[-nu L, -Phibar], [L, -nu L]]; converged SDC on
    Gauss-Lobatto nodes gives the (M, M) Pade approximant of exp(dt A_n)."""
    N, p = 15, swe.SWEParams()

    class Linear:
        def evaluate(self, th):
            return swe.f_implicit(th, N, p), torch.zeros_like(th)

        def solve(self, b, h):
            return swe.imex_solve(b, h, N, p)

    gen = torch.Generator().manual_seed(4)
    th0 = torch.stack([rand_spec(N, gen) * 100, rand_spec(N, gen) * 1e-5, rand_spec(N, gen) * 1e-5])
    dt = 600.0
    lev = sdc.Level(Linear(), "lobatto", 3)
    th1 = sdc.mlsdc_step(lev, None, dt, th0, niter=30)
    L = swe.lap_eig(N, p.a).numpy()
    M = 2
    c = [math.factorial(2 * M - k) * math.factorial(M) / (math.factorial(2 * M) * math.factorial(k) * math.factorial(M - k)) for k in range(M + 1)]
    for i in range(1, sht.nspec(N)):
        A = dt * np.array([[-p.nu * L[i], -p.phibar], [L[i], -p.nu * L[i]]])
        num = sum(ck * np.linalg.matrix_power(A, k) for k, ck in enumerate(c))
        den = sum(ck * np.linalg.matrix_power(-A, k) for k, ck in enumerate(c))
        R = np.linalg.solve(den, num)
        v = np.array([th0[0, i].item(), th0[2, i].item()])
        w = R @ v
        got = np.array([th1[0, i].item(), th1[2, i].item()])
        assert np.abs(got - w).max() < 1e-12 * np.abs(w).max() + 1e-30
        zexp = th0[1, i].item() / (1 + 0)  # zeta: pure diffusion, Pade of -dt nu L
        z = -dt * p.nu * L[i]
        Rz = sum(ck * z ** k for k, ck in enumerate(c)) / sum(ck * (-z) ** k for k, ck in enumerate(c))
        assert abs(th1[1, i].item() - Rz * zexp) < 1e-12 * abs(zexp) + 1e-30


# ---------------------------------------------------------------- SDC matrices
def test_sdc_matrices_lobatto3():
    m = Qd.sdc_matrices("lobatto", 3)
    Q = np.array([[0, 0, 0], [5 / 24, 1 / 3, -1 / 24], [1 / 6, 2 / 3, 1 / 6]])
    assert np.abs(m.Q - Q).max() < 1e-16
    assert np.abs(m.QD[1:, 1:] - np.array([[1 / 3, 0], [2 / 3, 1 / 4]])).max() < 1e-16
    assert np.abs(m.QE - np.array([[0, 0, 0], [0.5, 0, 0], [0.5, 0.5, 0]])).max() == 0


def test_sdc_matrices_lobatto5_and_transfer():
    m5 = Qd.sdc_matrices("lobatto", 5)
    last = np.array([1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20])
    assert np.abs(m5.Q[-1] - last).max() < 1e-16
    assert np.allclose(m5.tau, [0, (1 - math.sqrt(3 / 7)) / 2, 0.5, (1 + math.sqrt(3 / 7)) / 2, 1], atol=1e-16)
    m3 = Qd.sdc_matrices("lobatto", 3)
    m2 = Qd.sdc_matrices("lobatto", 2)
    # time restriction is injection for 5 -> 3 and 3 -> 2 nodes (Sec. 4.3.3)
    assert np.abs(Qd.transfer_matrix(m5, m3) - np.eye(5)[[0, 2, 4]]).max() < 1e-15
    assert np.abs(Qd.transfer_matrix(m3, m2) - np.eye(3)[[0, 2]]).max() < 1e-15
    # interpolation 3 -> 5 is exact for quadratics
    P = Qd.transfer_matrix(m3, m5)
    for k in range(3):
        assert np.abs(P @ m3.tau ** k - m5.tau ** k).max() < 1e-15


@pytest.mark.parametrize("kind,nn", [("lobatto", 3), ("lobatto", 5), ("radau", 4), ("radau", 6)])
def test_lu_trick_nilpotent_and_quadrature(kind, nn):
    """I - QD^-1 Qhat is nilpotent (stiff limit converges in M sweeps), and Q
    integrates polynomials of degree < number of basis nodes exactly."""
    m = Qd.sdc_matrices(kind, nn)
    M = nn - 1
    Qh, QDh = m.Q[1:, 1:], m.QD[1:, 1:]
    E = np.eye(M) - np.linalg.solve(QDh, Qh)
    assert np.abs(np.linalg.matrix_power(E, M)).max() < 1e-12
    assert np.allclose(np.triu(QDh, 1), 0)
    nb = M + 1 if kind == "lobatto" else M
    for k in range(nb):
        assert np.abs(m.Q @ m.tau ** k - m.tau ** (k + 1) / (k + 1)).max() < 1e-15


# ---------------------------------------------------------------- sweeps
class Dahlquist:
    def __init__(self, li, le):
        self.li, self.le = li, le
        self.n_eval = self.n_solve = 0

    def evaluate(self, y):
        self.n_eval += 1
        return self.li * y, self.le * y

    def solve(self, b, h):
        self.n_solve += 1
        return b / (1 - h * self.li)


def _pade(p, q, z):
    num = sum(math.factorial(p + q - k) * math.factorial(p) / (math.factorial(p + q) * math.factorial(k) * math.factorial(p - k)) * z ** k for k in range(p + 1))
    den = sum(math.factorial(p + q - k) * math.factorial(q) / (math.factorial(p + q) * math.factorial(k) * math.factorial(q - k)) * (-z) ** k for k in range(q + 1))
    return num / den


@pytest.mark.parametrize("kind,nn", [("lobatto", 3), ("lobatto", 5), ("radau", 4)])
def test_sdc_converges_to_collocation_pade(kind, nn):
    li, le = -2.0 + 0j, 1.5j
    lev = sdc.Level(Dahlquist(li, le), kind, nn)
    y = sdc.mlsdc_step(lev, None, 0.7, torch.tensor(1 + 0j, dtype=CT), niter=80)
    M = nn - 1
    z = 0.7 * (li + le)
    R = _pade(M, M, z) if kind == "lobatto" else _pade(M - 1, M, z)
    assert abs(y.item() - R) < 1e-13


@pytest.mark.parametrize("nn,K", [(3, 1), (3, 2), (3, 3), (5, 3), (5, 4)])
def test_sdc_order_per_sweep(nn, K):
    """Each sweep raises the order by one up to the collocation order (Sec. 4.2)."""
    errs = []
    for nsteps in (8, 16):
        lev = sdc.Level(Dahlquist(-1.0 + 0j, 1j), "lobatto", nn)
        y = torch.tensor(1 + 0j, dtype=CT)
        for _ in range(nsteps):
            y = sdc.mlsdc_step(lev, None, 1.0 / nsteps, y, niter=K)
        errs.append(abs(y.item() - np.exp(-1 + 1j)))
    order = math.log2(errs[0] / errs[1])
    assert abs(order - min(K, 2 * (nn - 1))) < 0.25


def test_stiff_limit_reaches_collocation_in_M_sweeps():
    li = -1e8 + 0j
    lev = sdc.Level(Dahlquist(li, 0j), "lobatto", 5)
    y = sdc.mlsdc_step(lev, None, 1.0, torch.tensor(1 + 0j, dtype=CT), niter=4)
    assert abs(y.item() - _pade(4, 4, li)) < 1e-13


# ---------------------------------------------------------------- MLSDC
@pytest.fixture(scope="module")
def swe_levels():
    p = swe.SWEParams()
    fine = swe.SWEProblem(31, 48, 96, p)
    coarse = swe.SWEProblem(15, 24, 48, p)
    return fine, coarse


def test_mlsdc_identical_levels_equals_double_sdc(swe_levels):
    """With identical levels tau = 0 and step D copies the coarse sweep, so
    MLSDC with N_ML iterations equals SDC with 2 N_ML sweeps."""
    fine, _ = swe_levels
    st = _seeded_state(31, 8)
    R, P = (lambda x: x), (lambda x: x)
    lf = sdc.Level(fine, "lobatto", 3)
    lc = sdc.Level(fine, "lobatto", 3)
    a = sdc.mlsdc_step(lf, lc, 600.0, st, niter=2, restrict_space=R, interp_space=P)
    b = sdc.mlsdc_step(lf, None, 600.0, st, niter=4)
    for f in range(3):
        assert relerr(a[f], b[f]) < 1e-13


def test_fas_fixed_point(swe_levels):
    """The restriction of the converged fine collocation solution solves the
    coarse FAS problem (Sec. 4.3.1), so an MLSDC iteration leaves it fixed."""
    fine, coarse = swe_levels
    st = _seeded_state(31, 9)
    lf = sdc.Level(fine, "lobatto", 3)
    lc = sdc.Level(coarse, "lobatto", 2)
    R, P = sdc.spectral_transfer(31, 15)
    hist = []
    sdc.mlsdc_step(lf, None, 300.0, st, niter=25, history=hist)
    conv = hist[-1]
    assert sdc.collocation_residual(lf, 300.0, conv) < 1e-14
    # one more MLSDC iteration from the converged nodes
    th = list(conv)
    fi = [None] * 3
    fe = [None] * 3
    for m in range(3):
        fi[m], fe[m] = fine.evaluate(th[m])
    th2, fi2, fe2 = sdc.sweep(lf, 300.0, th, fi, fe)
    Pi_cf = Qd.transfer_matrix(lf.mat, lc.mat)
    thc = [R(sum(float(Pi_cf[i, j]) * th2[j] for j in range(3))) for i in range(2)]
    fic, fec = zip(*[coarse.evaluate(t) for t in thc])
    tau = sdc.fas_tau(lf, lc, 300.0, fi2, fe2, list(fic), list(fec), R, Pi_cf)
    thc2, _, _ = sdc.sweep(lc, 300.0, thc, list(fic), list(fec), tau)
    for f in range(3):
        assert relerr(thc2[1][f], thc[1][f]) < 1e-12


def test_mass_conservation(swe_levels):
    """Phi'^0_0 is constant: F_I and F_E have no n = 0 component."""
    fine, coarse = swe_levels
    st = _seeded_state(31, 10)
    st[0, 0] = 123.0
    lf = sdc.Level(fine, "lobatto", 3)
    lc = sdc.Level(coarse, "lobatto", 2)
    R, P = sdc.spectral_transfer(31, 15)
    out = sdc.mlsdc_step(lf, lc, 600.0, st, niter=2, restrict_space=R, interp_space=P)
    assert abs(out[0, 0].item() - 123.0) < 1e-13 * 123.0


def test_theoretical_speedup_from_evaluation_counts():
    """Count solves and evaluations of one MLSDC and one SDC step in the
    oracle, price them with the paper's cost model (C^s = C^fi = C^fe,
    cost proportional to K = 3 R (R+1)/2, step-start evaluations not counted,
    Sec. 4.5) and compare with the speedups the paper prints."""
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        nums = json.load(f)
    for key, d in nums.items():
        Rf = d["R_f"]
        Rc = d["alpha"] * Rf
        Kf, Kc = Rf * (Rf + 1), Rc * (Rc + 1)

        def counts(coarse_on):
            pf, pc = Dahlquist(-1.0 + 0j, 0.5j), Dahlquist(-1.0 + 0j, 0.5j)
            lf = sdc.Level(pf, "lobatto", d["Mf"] + 1)
            lc = sdc.Level(pc, "lobatto", d["Mc"] + 1) if coarse_on else None
            ident = (lambda x: x)
            sdc.mlsdc_step(lf, lc, 0.1, torch.tensor(1 + 0j, dtype=CT),
                           niter=d["N_ML"] if coarse_on else d["N_S"],
                           restrict_space=ident, interp_space=ident)
            # each evaluation gives F_I and F_E: two unit costs; a solve one
            ef = pf.n_eval - 1
            ec = pc.n_eval - (1 if coarse_on else 0)
            return Kf * (pf.n_solve + 2 * ef) + Kc * (pc.n_solve + 2 * ec)

        S = counts(False) / counts(True)
        a = d["alpha"]
        formula = d["N_S"] / d["N_ML"] / (1 + a * a * 5 * (Rf + 1 / a) * d["Mc"] / (3 * (Rf + 1) * d["Mf"]))
        assert abs(S - formula) < 1e-12
        # the paper prints the formula rounded to two decimals (1.654 -> "about 1.66")
        assert abs(S - d["value"]) <= d["rounding"], (key, S)


def test_dome_sdc_temporal_order():
    """The oracle's SDC(3,4) (three Gauss-Lobatto nodes, four sweeps) is
    fourth order in time (collocation order 2M - 2 = 4 reached after four
    sweeps, Sec. 4.2) on the Gaussian dome of Sec. 5.2 at T15: the errors at
    dt = 450, 225, 112.5 s after 30 minutes, against SDC(5,8) at 112.5 s,
    fall by 2^4 per halving (observed orders within 3.5 .. 4.5)."""
    import workload
    N, J, I = 15, 24, 48
    p = swe.SWEParams(phibar=workload.dome_phibar())
    g = sht.Grid(N, J, I)
    x0 = torch.zeros(3, workload.nspec(N), dtype=torch.complex128)
    x0[0] = g.sh_forward(torch.tensor(workload.dome_grid(g.mu.numpy(), I))[None])[0]

    def run(nodes, K, dt, T=1800.0):
        lev = sdc.Level(swe.SWEProblem(N, J, I, p), "lobatto", nodes)
        x = x0.clone()
        for _ in range(int(round(T / dt))):
            x = sdc.mlsdc_step(lev, None, dt, x, niter=K)
        return x

    ref = run(5, 8, 112.5)
    err = [(run(3, 4, dt)[0] - ref[0]).abs().max().item() for dt in (450.0, 225.0, 112.5)]
    orders = [math.log2(err[i] / err[i + 1]) for i in range(2)]
    assert all(3.5 < o < 4.5 for o in orders), (err, orders)


def _small_state(N, seed):
    import workload
    raw = torch.tensor(workload.raw_spectrum(N, seed, 3))
    return raw * torch.tensor([100.0, 1e-5, 1e-5], dtype=torch.float64)[:, None]


def test_mlsdc_multi_two_levels_is_algorithm1():
    """The multi-level V-cycle with two levels is Algorithm 1 operation for
    operation: identical results to mlsdc_step (T15 / T10, 3 / 2 nodes)."""
    lf = sdc.Level(swe.SWEProblem(15, 24, 48), "lobatto", 3)
    lc = sdc.Level(swe.SWEProblem(10, 16, 32), "lobatto", 2)
    R, P = sdc.spectral_transfer(15, 10)
    x = _small_state(15, 77)
    a = sdc.mlsdc_step(lf, lc, 300.0, x, niter=2, restrict_space=R, interp_space=P)
    b = sdc.mlsdc_step_multi([lf, lc], 300.0, x, 2, [1, 1], [(R, P)])
    assert torch.equal(a, b)


def test_mlsdc_three_levels_converge_to_collocation():
    """Three levels (T15 / T10 / T5 with 5 / 3 / 2 Gauss-Lobatto nodes,
    dt = 300 s): iterated to convergence the V-cycle reaches the fine
    collocation solution (Sec. 4.2), its residual falling below 1e-13 within
    12 iterations.  That fixed point needs the restricted middle-level FAS
    term in the coarsest level's tau (eq. tau_term_level_l+1 with
    tau_l != 0): without it the residual stalls near 4e-5."""
    L = [sdc.Level(swe.SWEProblem(15, 24, 48), "lobatto", 5), sdc.Level(swe.SWEProblem(10, 16, 32), "lobatto", 3),
         sdc.Level(swe.SWEProblem(5, 8, 16), "lobatto", 2)]
    tr = [sdc.spectral_transfer(15, 10), sdc.spectral_transfer(10, 5)]
    hist = []
    sdc.mlsdc_step_multi(L, 300.0, _small_state(15, 77), 12, [1, 1, 1], tr, history=hist)
    res = [sdc.collocation_residual(L[0], 300.0, h) for h in hist]
    assert res[-1] < 1e-13, res
    assert res[0] > 1e-5, res


def test_adjoint_jvp_golden_matches_oracle_reverse_mode():
    """The stored forward-mode directional derivatives (tests/golden/
    adjoint_jvp.json, T31/T15, 3 steps) equal the oracle's reverse-mode
    gradient dotted with the same seeded directions: the two modes of
    differentiation agree on the whole integration."""
    import json
    import os
    import workload
    from oracle import sdc as OS
    from oracle import sht as OH
    from oracle import swe as OW
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_jvp.json")) as f:
        c = json.load(f)["T31_T15_3steps"]
    lf = OS.Level(OW.SWEProblem(*c["fine"]), "lobatto", 5)
    lc = OS.Level(OW.SWEProblem(*c["coarse"]), "lobatto", 3)
    R, P = OS.spectral_transfer(c["fine"][0], c["coarse"][0])
    th0 = torch.tensor(workload.state(c["fine"][0], c["seed_state"]))
    x = th0.clone().requires_grad_(True)
    y = x
    for _ in range(c["nsteps"]):
        y = OS.mlsdc_step(lf, lc, c["dt"], y, niter=4, nsweep_fine=2, nsweep_coarse=2, restrict_space=R,
                          interp_space=P)
    w = torch.where(OH.orders(c["fine"][0]) == 0, 1.0, 2.0).to(torch.float64)
    (0.5 * (w * (y[0].real ** 2 + y[0].imag ** 2)).sum()).backward()
    dirs = torch.tensor(workload.directions(c["fine"][0], c["ndirs"], c["seed_dirs"],
                                            torch.linalg.vector_norm(th0[1]).item()))
    g = x.grad[1]
    got = torch.stack([(g.real * d.real + g.imag * d.imag).sum() for d in dirs]).numpy()
    ref = np.array(c["dL"])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------- reduced-precision emulation
def test_mixed_accumulation_is_recursive_fp32():
    """FP32 accumulation one term at a time: 1 + 2^-25 added 64 times stays 1
    (each addition rounds the increment away, to nearest even), while any
    summation that first adds the small terms together (pairwise or blocked)
    returns 1 + 2^-19 exactly."""
    from oracle import mixed as OM
    K = 65
    A = torch.ones(1, K, dtype=torch.float64)
    B = torch.full((K, 1), 2.0 ** -25, dtype=torch.float64)
    B[0, 0] = 1.0
    assert OM.mixed_matmul(A, B, "fp32").item() == 1.0
    assert (A @ B).item() == 1.0 + 64 * 2.0 ** -25
    # exact small-integer contractions come out exact in every mode
    gen = torch.Generator().manual_seed(3)
    Ai = torch.randint(-8, 9, (5, 7), generator=gen).to(torch.float64)
    Bi = torch.randint(-8, 9, (7, 4), generator=gen).to(torch.float64)
    for mode in ("fp32", "bf16x2", "bf16x3"):
        assert torch.equal(OM.mixed_matmul(Ai, Bi, mode), Ai @ Bi), mode


def test_mixed_split_pieces():
    """bf16 pieces: hi has 8 significant bits, two pieces hold a value to
    about 2^-16 relative and three to about 2^-24."""
    from oracle import mixed as OM
    gen = torch.Generator().manual_seed(4)
    x = torch.randn(4000, generator=gen, dtype=torch.float64) * torch.exp(torch.randn(4000, generator=gen, dtype=torch.float64) * 5)
    p = OM.split(x, 3)
    hi_bits = p[0].view(torch.int32) & 0xFFFF
    assert int(hi_bits.abs().max()) == 0                      # bf16: the low 16 bits of the FP32 pattern are zero
    r2 = ((p[0].double() + p[1].double() - x).abs() / x.abs()).max().item()
    r3 = ((p[0].double() + p[1].double() + p[2].double() - x).abs() / x.abs()).max().item()
    assert 2.0 ** -19 < r2 <= 2.0 ** -16 and r3 <= 2.0 ** -24


@pytest.mark.parametrize("mode,u", [("fp32", 2.0 ** -24), ("bf16x2", 2.0 ** -16), ("bf16x3", 2.0 ** -24)])
def test_mixed_error_within_recursive_summation_bound(mode, u):
    """Error of the emulated contraction against the exact one within the
    standard bound for rounded operands and recursive summation,
    |err| <= (2 u_in + gamma_K) sum_k |a_k b_k|, gamma_K = K u / (1 - K u),
    u = 2^-24 for the FP32 sums and u_in the operand precision; and not far
    below it on random data (the chain does round: above 1e-5 of the bound,
    where an FP64 contraction would sit near 1e-9)."""
    from oracle import mixed as OM
    gen = torch.Generator().manual_seed(5)
    K = 1536
    A = torch.randn(64, K, generator=gen, dtype=torch.float64)
    B = torch.randn(K, 3, generator=gen, dtype=torch.float64) + 0.3
    got = OM.mixed_matmul(A, B, mode)
    exact = A @ B
    s = A.abs() @ B.abs()
    uacc = 2.0 ** -24
    gam = K * uacc / (1 - K * uacc)
    ratio = ((got - exact).abs() / ((2 * u + gam) * s)).max().item()
    assert 1e-5 < ratio <= 1.0, ratio
