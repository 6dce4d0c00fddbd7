// Host setup routines (quad precision), see setup_host.cpp.
#pragma once
#ifdef __cplusplus
extern "C" {
#endif
// Gaussian latitudes north to south: mu_j, sin(theta_j), 1 - mu_j^2, w_j.
int shx_host_gauss(int J, double* mu, double* sin_theta, double* cos2phi, double* w);
// SDC nodes tau[n] and row-major n x n matrices Q, Q_E, Q_Delta (kind 0 =
// Gauss-Lobatto, 1 = Radau right).  Pointers may be NULL.
int shx_host_sdc(int kind, int nnodes, double* tau, double* Q, double* QE, double* QD);
// Lagrange transfer matrix Pi[n_dst][n_src], Pi_ij = L^j_src(tau^dst_i).
int shx_host_transfer(int kind, int n_src, int n_dst, double* Pi);
// e^{-2 pi i t / L}, t = 0..L-1.
void shx_host_twiddles(int L, double* re, double* im);

// The value a Legendre contraction of working precision prec uses for x
// (FP64: x; FP32: rounded; split bf16: the sum of the pieces).
double shx_host_working_value(int prec, double x);
#ifdef __cplusplus
}
#endif
