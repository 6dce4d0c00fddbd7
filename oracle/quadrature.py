"""Quadrature data of the method, computed in extended precision (mpmath).

* Gaussian latitudes and weights of the discrete Legendre transform
  (Sec. 3, eq. legendre_transform: mu_j are the roots of P_J, w_j the Gauss
  weights).
* SDC nodes (Sec. 4.2: Gauss-Lobatto nodes on [t^n, t^n + dt]) and the
  Gauss-Radau-right variant.
* The SDC matrices: collocation matrix Q (eq. weights), forward-Euler
  matrix Q_E (Sec. 4.2), the LU-trick matrix Q_Delta (Sec. 4.2, after Weiser),
  and the Lagrange time-transfer matrices Pi (Sec. 4.3.3).

All values are produced with >= 34 significant digits and rounded to FP64 at
the very end.  Part of the test infrastructure (see oracle/__init__.py).
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

_DPS = 40


def _legendre_pair(n, x):
    """P_n(x), P_{n-1}(x) by the three-term recurrence (mpmath)."""
    p0, p1 = mp.mpf(1), x
    if n == 0:
        return p0, mp.mpf(0)
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p1, p0


@lru_cache(maxsize=None)
def gauss_legendre(J):
    """Gaussian latitudes for the Legendre transform, ordered north to south.

    Returns float64 arrays (mu, sin_theta, cos2phi, w):
      mu_j      = cos(theta_j), the J roots of P_J (Sec. 3, eq. legendre_transform),
      sin_theta = sqrt(1 - mu_j^2), stored directly (never recomputed from mu),
      cos2phi   = 1 - mu_j^2 = sin^2(theta_j),
      w_j       = Gauss weights, sum w = 2.

    Newton iteration on theta from the classical asymptotic first guess
    theta_k = pi (k - 1/4) / (J + 1/2): float64 until converged, then three
    steps in 40-digit arithmetic.
    """
    # float64 Newton on theta, vectorised, to get within rounding of the root
    k = np.arange(1, (J + 1) // 2 + 1)
    th0 = np.pi * (k - 0.25) / (J + 0.5)
    for _ in range(20):
        x = np.cos(th0)
        p0, p1 = np.ones_like(x), x.copy()
        for n in range(2, J + 1):
            p0, p1 = p1, ((2 * n - 1) * x * p1 - (n - 1) * p0) / n
        th0 = th0 + p1 * np.sin(th0) / (J * (p0 - x * p1))
    with mp.workdps(_DPS):
        mu = np.empty(J)
        st = np.empty(J)
        c2 = np.empty(J)
        w = np.empty(J)
        for kk in k:
            th = mp.mpf(th0[kk - 1])
            # each extended-precision Newton step squares the relative error
            for _ in range(3):
                x = mp.cos(th)
                pj, pjm1 = _legendre_pair(J, x)
                s = mp.sin(th)
                # d/dtheta P_J(cos theta) = -J (P_{J-1} - x P_J) / sin(theta)
                dth = -J * (pjm1 - x * pj) / s
                th = th - pj / dth
            x = mp.cos(th)
            s = mp.sin(th)
            pj, pjm1 = _legendre_pair(J, x)
            wk = 2 * s * s / (J * pjm1) ** 2
            j = kk - 1
            mu[j], st[j], c2[j], w[j] = float(x), float(s), float(s * s), float(wk)
            jm = J - 1 - j
            if jm != j:
                mu[jm], st[jm], c2[jm], w[jm] = -float(x), float(s), float(s * s), float(wk)
            else:
                mu[j] = 0.0
    return mu, st, c2, w


# ---------------------------------------------------------------------------
# SDC nodes and matrices (Sec. 4.2, eqs. update_equation_sdcq_discrete_form,
# weights; Sec. 4.3.3 for Pi)
# ---------------------------------------------------------------------------

def _poly_mul(a, b):
    out = [mp.mpf(0)] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            out[i + j] += ai * bj
    return out


def _legendre_coeffs(n):
    """Monomial coefficients (ascending) of P_n."""
    p0, p1 = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    if n == 0:
        return p0
    for k in range(2, n + 1):
        xp1 = [mp.mpf(0)] + p1
        nxt = [mp.mpf(0)] * (k + 1)
        for i, c in enumerate(xp1):
            nxt[i] += (2 * k - 1) * c / k
        for i, c in enumerate(p0):
            nxt[i] -= (k - 1) * c / k
        p0, p1 = p1, nxt
    return p1


def _real_roots(coeffs):
    """Real roots (sorted) of a polynomial given by ascending coefficients."""
    desc = list(reversed(coeffs))
    while abs(desc[0]) == 0:
        desc = desc[1:]
    roots = mp.polyroots(desc, maxsteps=400, extraprec=400)
    return sorted(mp.re(r) for r in roots)


def _nodes_mp(kind, nnodes):
    """SDC nodes on [0, 1] as mpf, including tau_0 = 0.

    kind 'lobatto': nnodes Gauss-Lobatto points (Sec. 4.2), endpoints included.
    kind 'radau'  : tau_0 = 0 (the initial value) followed by the nnodes-1
                    Gauss-Radau-right (Radau IIA) points, which end at 1.
    """
    if kind == "lobatto":
        M = nnodes - 1
        if M == 1:
            xs = [mp.mpf(-1), mp.mpf(1)]
        else:
            pm = _legendre_coeffs(M)
            dp = [i * c for i, c in enumerate(pm)][1:]
            xs = [mp.mpf(-1)] + _real_roots(dp) + [mp.mpf(1)]
        return [(x + 1) / 2 for x in xs]
    if kind == "radau":
        s = nnodes - 1
        ps = _legendre_coeffs(s)
        psm = _legendre_coeffs(s - 1) + [mp.mpf(0)]
        diff = [a - b for a, b in zip(ps, psm)]
        xs = _real_roots(diff)
        xs[-1] = mp.mpf(1)
        return [mp.mpf(0)] + [(x + 1) / 2 for x in xs]
    raise ValueError(kind)


def _lagrange_coeffs(nodes, j):
    """Ascending coefficients of the Lagrange polynomial L^j on `nodes`."""
    c = [mp.mpf(1)]
    for k, tk in enumerate(nodes):
        if k == j:
            continue
        d = nodes[j] - tk
        c = _poly_mul(c, [-tk / d, 1 / d])
    return c


def _poly_eval(c, x):
    return sum(ci * x ** i for i, ci in enumerate(c))


def _poly_int0(c, x):
    """Integral from 0 to x of the polynomial c."""
    return sum(ci * x ** (i + 1) / (i + 1) for i, ci in enumerate(c))


class SDCMatrices:
    """Nodes and matrices of one SDC level (float64 numpy, from mpmath).

    tau   : (M+1,) nodes on [0, 1], tau[0] = 0, tau[M] = 1
    Q     : (M+1, M+1) q_{i,j} = int_0^{tau_i} L^j  (eq. weights, per unit dt)
    QE    : (M+1, M+1) forward-Euler weights, QE[i, j] = tau_{j+1} - tau_j for j < i
    QD    : (M+1, M+1) implicit weights of the LU trick: with Qhat = Q[1:, 1:],
            Qhat^T = L U (Doolittle), QD[1:, 1:] = U^T, row/column 0 zero
    For the Radau kind the Lagrange basis lives on the collocation points
    tau_1..tau_M only, so column 0 of Q is zero.
    """

    def __init__(self, kind, nnodes):
        with mp.workdps(_DPS):
            t = _nodes_mp(kind, nnodes)
            M = nnodes - 1
            self.kind, self.M = kind, M
            if kind == "lobatto":
                basis_nodes, col0 = t, 0
            else:
                basis_nodes, col0 = t[1:], 1
            Q = mp.zeros(M + 1, M + 1)
            for jj in range(len(basis_nodes)):
                c = _lagrange_coeffs(basis_nodes, jj)
                for i in range(M + 1):
                    Q[i, jj + col0] = _poly_int0(c, t[i])
            QE = mp.zeros(M + 1, M + 1)
            for i in range(M + 1):
                for j in range(i):
                    QE[i, j] = t[j + 1] - t[j]
            # Doolittle LU of Qhat^T without pivoting
            A = mp.matrix(M, M)
            for i in range(M):
                for j in range(M):
                    A[i, j] = Q[j + 1, i + 1]
            U = mp.zeros(M, M)
            Lm = mp.eye(M)
            for i in range(M):
                for j in range(i, M):
                    U[i, j] = A[i, j] - sum(Lm[i, k] * U[k, j] for k in range(i))
                for r in range(i + 1, M):
                    Lm[r, i] = (A[r, i] - sum(Lm[r, k] * U[k, i] for k in range(i))) / U[i, i]
            QD = mp.zeros(M + 1, M + 1)
            for i in range(M):
                for j in range(M):
                    QD[i + 1, j + 1] = U[j, i]
            self._t_mp = t
            self._basis_nodes = basis_nodes
            self._col0 = col0
            self.tau = np.array([float(x) for x in t])
            self.Q = np.array([[float(Q[i, j]) for j in range(M + 1)] for i in range(M + 1)])
            self.QE = np.array([[float(QE[i, j]) for j in range(M + 1)] for i in range(M + 1)])
            self.QD = np.array([[float(QD[i, j]) for j in range(M + 1)] for i in range(M + 1)])


def transfer_matrix(src: SDCMatrices, dst: SDCMatrices):
    """Pi with Pi[i, j] = L^j_src(tau^dst_i) (Sec. 4.3.3, time restriction and
    interpolation).  Node 0 holds the initial value on both levels; for the
    Radau kind it is not a collocation node and maps to itself."""
    assert src.kind == dst.kind
    with mp.workdps(_DPS):
        Ms, Md = src.M, dst.M
        P = np.zeros((Md + 1, Ms + 1))
        col0 = src._col0
        if col0:
            P[0, 0] = 1.0
        for jj in range(len(src._basis_nodes)):
            c = _lagrange_coeffs(src._basis_nodes, jj)
            for i in range(col0, Md + 1):
                P[i, jj + col0] = float(_poly_eval(c, dst._t_mp[i]))
    return P


@lru_cache(maxsize=None)
def sdc_matrices(kind, nnodes):
    return SDCMatrices(kind, nnodes)
