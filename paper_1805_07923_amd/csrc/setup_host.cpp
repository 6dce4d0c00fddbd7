// Host-side setup numerics in quad precision (__float128, libquadmath):
//   * Gaussian latitudes / weights of the Legendre transform (Sec. 3, eq.
//     legendre_transform: mu_j roots of P_J, w_j Gauss weights);
//   * SDC nodes and matrices (Sec. 4.2: Gauss-Lobatto nodes; collocation
//     matrix Q of eq. weights; forward-Euler weights; LU-trick weights) and the
//     Lagrange time-transfer matrices (Sec. 4.3.3);
//   * FFT twiddle factors for the longitude transform (eq. fourier_transform).
// Everything is rounded to FP64 only when stored.  Compiled by the host C++
// compiler (no device code here).
#include <quadmath.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "setup_host.h"

namespace {

typedef __float128 qd;

const qd QPI = M_PIq;

// P_n(x) and P_{n-1}(x) by the three-term recurrence.
template <class T>
void legendre_pair(int n, T x, T& pn, T& pnm1) {
    T p0 = 1, p1 = x;
    if (n == 0) { pn = 1; pnm1 = 0; return; }
    for (int k = 2; k <= n; ++k) {
        T p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    pn = p1;
    pnm1 = p0;
}

// Roots of a smooth function on (a, b): sign changes on a fine sampling,
// then bisection to quad precision.
template <class F>
std::vector<qd> roots_in(F f, qd a, qd b, int samples) {
    std::vector<qd> out;
    qd xprev = a, fprev = f(a);
    for (int i = 1; i <= samples; ++i) {
        qd x = a + (b - a) * i / samples;
        qd fx = f(x);
        if (fx == 0) {
            out.push_back(x);
        } else if ((fprev < 0 && fx > 0) || (fprev > 0 && fx < 0)) {
            qd lo = xprev, hi = x, flo = fprev;
            for (int it = 0; it < 200; ++it) {
                qd mid = (lo + hi) / 2;
                qd fm = f(mid);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            out.push_back((lo + hi) / 2);
        }
        xprev = x;
        fprev = fx;
    }
    return out;
}

// Lagrange basis polynomial j on `nodes`, evaluated at x.
qd lagrange(const std::vector<qd>& nodes, int j, qd x) {
    qd v = 1;
    for (size_t k = 0; k < nodes.size(); ++k)
        if ((int)k != j) v *= (x - nodes[k]) / (nodes[j] - nodes[k]);
    return v;
}

// 12-point Gauss-Legendre rule on [-1, 1] in quad precision (exact to degree 23).
void gauss12(qd* x, qd* w) {
    const int n = 12;
    for (int k = 1; k <= n; ++k) {
        qd t = cosq(QPI * (k - (qd)0.25) / (n + (qd)0.5));
        for (int it = 0; it < 100; ++it) {
            qd pn, pnm1;
            legendre_pair<qd>(n, t, pn, pnm1);
            qd dp = n * (t * pn - pnm1) / (t * t - 1);
            qd step = pn / dp;
            t -= step;
            if (fabsq(step) < 1e-33Q) break;
        }
        qd pn, pnm1;
        legendre_pair<qd>(n, t, pn, pnm1);
        qd dp = n * (t * pn - pnm1) / (t * t - 1);
        x[k - 1] = t;
        w[k - 1] = 2 / ((1 - t * t) * dp * dp);
    }
}

std::vector<qd> sdc_nodes_q(int kind, int nnodes) {
    std::vector<qd> t;
    const int M = nnodes - 1;
    if (kind == 0) {  // Gauss-Lobatto: endpoints and the roots of P_M'
        auto dP = [M](qd x) {
            qd pn, pnm1;
            legendre_pair<qd>(M, x, pn, pnm1);
            return M * (pnm1 - x * pn);   // (1 - x^2) P_M'(x): same interior roots
        };
        // the interior roots of P_M' (M <= 8) lie inside |x| < 0.97
        std::vector<qd> r = (M >= 2) ? roots_in(dP, (qd)-0.999Q, (qd)0.999Q, 3999)
                                     : std::vector<qd>();
        t.push_back(0);
        for (qd x : r) t.push_back((x + 1) / 2);
        t.push_back(1);
    } else {          // t^n, then Radau-IIA points: roots of P_s - P_{s-1}, s = M
        const int s = M;
        auto f = [s](qd x) {
            qd ps, psm1;
            legendre_pair<qd>(s, x, ps, psm1);
            return ps - psm1;
        };
        std::vector<qd> r = roots_in(f, (qd)-1 + 1e-30Q, (qd)1 - 1e-20Q, 4000);
        t.push_back(0);
        for (qd x : r) t.push_back((x + 1) / 2);
        t.push_back(1);
    }
    return t;
}

}  // namespace

extern "C" int shx_host_gauss(int J, double* mu, double* sin_theta, double* cos2phi, double* w) {
    if (J < 2) return -1;
    const int half = (J + 1) / 2;
    for (int k = 1; k <= half; ++k) {
        // FP64 Newton in theta from the asymptotic guess, then quad-precision steps
        double th = M_PI * (k - 0.25) / (J + 0.5);
        for (int it = 0; it < 50; ++it) {
            double x = std::cos(th), pn, pnm1;
            legendre_pair<double>(J, x, pn, pnm1);
            double d = -J * (pnm1 - x * pn) / std::sin(th);
            double step = pn / d;
            th -= step;
            if (std::fabs(step) < 1e-15 * th) break;
        }
        qd tq = th;
        for (int it = 0; it < 3; ++it) {
            qd x = cosq(tq), pn, pnm1;
            legendre_pair<qd>(J, x, pn, pnm1);
            qd d = -J * (pnm1 - x * pn) / sinq(tq);
            tq -= pn / d;
        }
        qd x = cosq(tq), s = sinq(tq), pn, pnm1;
        legendre_pair<qd>(J, x, pn, pnm1);
        qd wk = 2 * s * s / ((J * pnm1) * (J * pnm1));
        int j = k - 1, jm = J - 1 - j;
        mu[j] = (double)x;
        mu[jm] = -(double)x;
        sin_theta[j] = sin_theta[jm] = (double)s;
        cos2phi[j] = cos2phi[jm] = (double)(s * s);
        w[j] = w[jm] = (double)wk;
        if (j == jm) mu[j] = 0.0;
    }
    return 0;
}

extern "C" int shx_host_sdc(int kind, int nnodes, double* tau, double* Q, double* QE, double* QD) {
    if (nnodes < 2 || nnodes > 9 || (kind != 0 && kind != 1)) return -1;
    const int M = nnodes - 1, n1 = M + 1;
    std::vector<qd> t = sdc_nodes_q(kind, nnodes);
    if ((int)t.size() != n1) return -2;
    // collocation basis: all nodes (Lobatto) or the M Radau points (node 0 is
    // the initial value only, so column 0 of Q is zero)
    std::vector<qd> basis(t.begin() + (kind == 0 ? 0 : 1), t.end());
    const int c0 = (kind == 0) ? 0 : 1;
    qd gx[12], gw[12];
    gauss12(gx, gw);
    std::vector<qd> q(n1 * n1, 0), qe(n1 * n1, 0), qdm(n1 * n1, 0);
    for (int i = 0; i < n1; ++i) {
        for (size_t j = 0; j < basis.size(); ++j) {
            qd s = 0;
            for (int g = 0; g < 12; ++g) {
                qd x = t[i] * (gx[g] + 1) / 2;   // int_0^{t_i}
                s += gw[g] * lagrange(basis, (int)j, x);
            }
            q[i * n1 + j + c0] = s * t[i] / 2;
        }
        for (int j = 0; j < i; ++j) qe[i * n1 + j] = t[j + 1] - t[j];
    }
    // LU trick: Qhat = Q[1:,1:], Qhat^T = L U (Doolittle), QD[1:,1:] = U^T
    std::vector<qd> A(M * M), U(M * M, 0), L(M * M, 0);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) A[i * M + j] = q[(j + 1) * n1 + (i + 1)];
    for (int i = 0; i < M; ++i) {
        L[i * M + i] = 1;
        for (int j = i; j < M; ++j) {
            qd s = A[i * M + j];
            for (int k = 0; k < i; ++k) s -= L[i * M + k] * U[k * M + j];
            U[i * M + j] = s;
        }
        for (int r = i + 1; r < M; ++r) {
            qd s = A[r * M + i];
            for (int k = 0; k < i; ++k) s -= L[r * M + k] * U[k * M + i];
            L[r * M + i] = s / U[i * M + i];
        }
    }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) qdm[(i + 1) * n1 + (j + 1)] = U[j * M + i];
    for (int i = 0; i < n1; ++i) {
        if (tau) tau[i] = (double)t[i];
        for (int j = 0; j < n1; ++j) {
            if (Q) Q[i * n1 + j] = (double)q[i * n1 + j];
            if (QE) QE[i * n1 + j] = (double)qe[i * n1 + j];
            if (QD) QD[i * n1 + j] = (double)qdm[i * n1 + j];
        }
    }
    return 0;
}

extern "C" int shx_host_transfer(int kind, int n_src, int n_dst, double* Pi) {
    std::vector<qd> ts = sdc_nodes_q(kind, n_src), td = sdc_nodes_q(kind, n_dst);
    if ((int)ts.size() != n_src || (int)td.size() != n_dst) return -2;
    const int c0 = (kind == 0) ? 0 : 1;
    std::vector<qd> basis(ts.begin() + c0, ts.end());
    for (int i = 0; i < n_dst; ++i)
        for (int j = 0; j < n_src; ++j) Pi[i * n_src + j] = 0.0;
    if (c0) Pi[0] = 1.0;
    for (int i = c0; i < n_dst; ++i)
        for (size_t j = 0; j < basis.size(); ++j) {
            qd v = lagrange(basis, (int)j, td[i]);
            Pi[i * n_src + j + c0] = (fabsq(v) < 1e-30Q) ? 0.0 : (double)v;
        }
    return 0;
}

extern "C" void shx_host_twiddles(int L, double* re, double* im) {
    for (int t = 0; t < L; ++t) {
        qd a = 2 * QPI * t / L;
        re[t] = (double)cosq(a);
        im[t] = -(double)sinq(a);   // e^{-2 pi i t / L}
    }
}

// ------------------------------------------------------------------------
// Value that a Legendre contraction of working precision `prec` uses for the
// FP64 value x: x (FP64), x rounded to FP32 (SHX_FP32), or the sum of its
// bf16 pieces (SHX_SPLIT_BF16_2 / _3: each piece the round-to-nearest-even
// bf16 of the FP32-rounded remainder).
static unsigned short host_f2bf(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
static float host_bf2f(unsigned short h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
double shx_host_working_value(int prec, double x) {
    if (prec == 1) return (double)(float)x;
    if (prec == 2 || prec == 3) {
        double rem = x, sum = 0.0;
        for (int q = 0; q < prec; ++q) {
            const double v = host_bf2f(host_f2bf((float)rem));
            sum += v;
            rem -= v;
        }
        return sum;
    }
    return x;
}
