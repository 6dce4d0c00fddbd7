// Spectral-space kernels, FP64, one thread per coefficient (m, n):
//   * wind coefficients and combine of the shallow-water tendency (Sec. 2-3);
//   * the diagonal implicit solve (Sec. 4.4, eq. implicit_systems);
//   * the node update of the IMEX SDC sweep (Sec. 4.2, eq.
//     update_equation_sdcq_discrete_form; Sec. 4.3.1, eq.
//     modified_update_equation_sdcq_discrete_form);
//   * the FAS term (Sec. 4.3.1, eq. tau_term_level_l+1) and the space-time
//     transfer by truncation / zero padding and Lagrange interpolation in time
//     (Sec. 4.3.3);
//   * the collocation residual (Sec. 4.2, eq. collocation_problem).
// The spectral form of the right-hand side is derived from Sec. 2 (the paper
// defers it to other work); with L_n = n (n+1) / a^2, psi = -zeta / L_n and
// chi = -delta / L_n (zero at n = 0):
//   U_n = [(n-1) eps_n psi_{n-1} - (n+2) eps_{n+1} psi_{n+1} + i m chi_n] / a,
//   V_n = [i m psi_n - (n-1) eps_n chi_{n-1} + (n+2) eps_{n+1} chi_{n+1}] / a,
// for the cos-weighted wind (U, V) = (u, v) cos(phi), and for the weighted
// analyses X^, Y^ of a cos-weighted flux
//   div_n  = [i m X^_n + n eps_{n+1} Y^_{n+1} - (n+1) eps_n Y^_{n-1}] / a,
//   curl_n = [i m Y^_n - n eps_{n+1} X^_{n+1} + (n+1) eps_n X^_{n-1}] / a.
#include "internal.h"
#include "swe_node.h"

namespace {

using namespace swe_node;

constexpr int TB = 256;

__global__ void k_spec_to_ext(const int* __restrict__ ord_e, const int* __restrict__ deg_e,
                              const double2* __restrict__ spec, double2* __restrict__ cin, int N,
                              long long nspec, long long nspec_e, int F, int halve) {
    const long long e = (long long)blockIdx.x * TB + threadIdx.x;
    if (e >= nspec_e) return;
    const int m = ord_e[e], n = deg_e[e];
    const double sc = (halve && m > 0) ? 0.5 : 1.0;
    for (int f = 0; f < F; ++f)
        cin[e * F + f] = (n <= N) ? cscale(sc, spec[f * nspec + spec_idx(N, m, n)]) : make_double2(0.0, 0.0);
}

__global__ void k_ext_to_spec(const int* __restrict__ ord, const int* __restrict__ deg,
                              const double2* __restrict__ cout, double2* __restrict__ spec, int N,
                              long long nspec, int F) {
    const long long i = (long long)blockIdx.x * TB + threadIdx.x;
    if (i >= nspec) return;
    const long long e = ext_idx(N, ord[i], deg[i]);
    for (int f = 0; f < F; ++f) spec[f * nspec + i] = cout[e * F + f];
}


// Field c of combine_one (F_E, F_I of Phi', zeta or delta).
__device__ __forceinline__ void combine_field(const double2* __restrict__ cout, const double2* __restrict__ st,
                                              int N, long long nspec, const swe_params& p, long long i, int m, int n,
                                              int c, double2& fe, double2& fi) {
    const double L = n * (n + 1.0) / (p.a * p.a);
    const double2* x0 = cout + ext_idx(N, m, n) * 5;
    const double2* xu = cout + ext_idx(N, m, n + 1) * 5;
    const bool has_dn = (n - 1 >= m);
    const double2* xd = has_dn ? cout + ext_idx(N, m, n - 1) * 5 : nullptr;
    const double cu = n * eps_nm(n + 1, m), cd = (n + 1.0) * eps_nm(n, m);
    const double ia = 1.0 / p.a;
    const double2 zero = make_double2(0.0, 0.0);
    // c = 0: -div(C, D); c = 1: -div(A, B); c = 2: curl(A, B) + L E
    const int X = (c == 0) ? 2 : 0, Y = X + 1;
    if (c < 2) {
        double2 r = cim(m, x0[X]);
        r = caxpy(cu, xu[Y], r);
        r = caxpy(-cd, has_dn ? xd[Y] : zero, r);
        fe = cscale(-ia, r);
    } else {
        double2 r = cim(m, x0[Y]);
        r = caxpy(-cu, xu[X], r);
        r = caxpy(cd, has_dn ? xd[X] : zero, r);
        fe = caxpy(L, x0[4], cscale(ia, r));
    }
    if (c == 1) {
        const double2 ze = st[nspec + i];
        fi = make_double2(-p.nu * L * ze.x, -p.nu * L * ze.y);
    } else {
        const double2 ph = st[i], de = st[2 * nspec + i];
        fi = (c == 0) ? make_double2(-p.phibar * de.x - p.nu * L * ph.x, -p.phibar * de.y - p.nu * L * ph.y)
                      : make_double2(L * ph.x - p.nu * L * de.x, L * ph.y - p.nu * L * de.y);
    }
}

// F_E, F_I from the weighted analyses (A, B, C, D, E) and the state.
__global__ void k_swe_combine(const int* __restrict__ ord, const int* __restrict__ deg,
                              const double2* __restrict__ cout, const double2* __restrict__ state,
                              double2* __restrict__ fi, double2* __restrict__ fe, int N, long long nspec,
                              long long nspec_e, swe_params p, int S) {
    const long long i = (long long)blockIdx.x * TB + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= nspec || s >= S) return;
    const int m = ord[i], n = deg[i];
    const double2* st = state + (long long)s * 3 * nspec;
    if (fe) {
        double2 e[3], f[3];
        combine_one(cout + (long long)s * nspec_e * 5, st, N, nspec, p, i, m, n, e, f);
        double2* o = fe + (long long)s * 3 * nspec;
        o[i] = e[0];
        o[nspec + i] = e[1];
        o[2 * nspec + i] = e[2];
    }
    if (fi) {
        const double L = n * (n + 1.0) / (p.a * p.a);
        const double2 ph = st[i], ze = st[nspec + i], de = st[2 * nspec + i];
        double2* o = fi + (long long)s * 3 * nspec;
        o[i] = make_double2(-p.phibar * de.x - p.nu * L * ph.x, -p.phibar * de.y - p.nu * L * ph.y);
        o[nspec + i] = make_double2(-p.nu * L * ze.x, -p.nu * L * ze.y);
        o[2 * nspec + i] = make_double2(L * ph.x - p.nu * L * de.x, L * ph.y - p.nu * L * de.y);
    }
}


__global__ void k_imex_solve(const int* __restrict__ deg, const double2* rhs, double2* out, long long nspec,
                             swe_params p, double h, int S) {
    const long long i = (long long)blockIdx.x * TB + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= nspec || s >= S) return;
    const int n = deg[i];
    const double L = n * (n + 1.0) / (p.a * p.a);
    const double2* b = rhs + (long long)s * 3 * nspec;
    double2* x = out + (long long)s * 3 * nspec;
    double2 xp, xz, xd;
    solve_one(L, h, p, b[i], b[nspec + i], b[2 * nspec + i], xp, xz, xd);
    x[i] = xp;
    x[nspec + i] = xz;
    x[2 * nspec + i] = xd;
}

// Node updates of a sweep, nodes m+1 = 1..M (eq. update_equation_sdcq_discrete_form
// and eq. modified_update_equation_sdcq_discrete_form with the IMEX split):
//   b_m = Theta^0 + sum_j dtQ[m+1][j] (F_I + F_E)^{j,old}
//         + sum_{j=1}^{m} [dtQE[m+1][j] dF_E^j + dtQD[m+1][j] dF_I^j]
//         - h_m F_I^{m+1,old} + tau^{m+1},   Theta^{m+1} = solve(b_m, h_m),
// with dF^j = F^{j,new} - F^{j,old}.  The part of b_m that holds no new F,
//   S_m = Theta^0 + sum_j dtQ[m+1][j] (F_I + F_E)^{j,old}
//         - sum_{j=1}^{m} [dtQE[m+1][j] F_E^{j,old} + dtQD[m+1][j] F_I^{j,old}]
//         - h_m F_I^{m+1,old} + tau^{m+1},
// is formed for every m by the first update (k_sdc_node_first), which reads
// the old F once (when the previous sweep left the F of node M unformed,
// cout_M != null, it forms that F from node M's analyses and Theta^M): it solves with S_0 and stores S_m, m >= 1, in the slot of
// the new F_E of node m+1, which the sweep fills only later (node m+1's
// update, or the closing combine for node M).  k_sdc_node (m >= 1) reads
// S_m, forms the new F at node m from the analyses of node m's tendency
// (cout) and Theta^m, stores it to (fi, fe) node m, and adds
// sum_{j=1}^{m} [dtQE[m+1][j] F_E^{j,new} + dtQD[m+1][j] F_I^{j,new}].
// k_sdc_node: blocks of NODE_CO coefficients x 3 fields, thread group c
// accumulates field c; the 2 x 2 solve of (Phi', delta) meets the three
// right-hand sides in LDS.  32 coefficients per block (96 threads, a quarter
// of the second wave idle) measured faster than 64 (8.8 vs 10.1 us at T255):
// twice the blocks spread the memory-bound loop over more CUs.
constexpr int NODE_CO = 32;

__device__ __forceinline__ void node_solve(const int* __restrict__ deg, const swe_params& p, double h, int c,
                                           int loc, long long i, bool on, double2 acc, double2 (*bsh)[NODE_CO],
                                           double2* __restrict__ out, double2* __restrict__ rec, long long o) {
    bsh[c][loc] = acc;
    __syncthreads();
    if (!on) return;
    const int n = deg[i];
    const double L = n * (n + 1.0) / (p.a * p.a);
    double2 xp, xz, xd;
    solve_one(L, h, p, bsh[0][loc], bsh[1][loc], bsh[2][loc], xp, xz, xd);
    const double2 v = (c == 0) ? xp : ((c == 1) ? xz : xd);
    out[o] = v;
    if (rec) rec[o] = v;
}

// The first update: one thread per coefficient with its three fields in
// registers (the solve needs no exchange), M + 1 old F per field; 64-thread
// blocks, a quarter of the wavefronts of one thread per (coefficient, field).
constexpr int NODE_T1 = 64;
template <int M>
__global__ __launch_bounds__(NODE_T1) void k_sdc_node_first(const int* __restrict__ ord,
                                                          const int* __restrict__ deg, int N, long long nspec,
                                                          swe_params p, NodeRows R, double2* __restrict__ theta,
                                                          const double2* __restrict__ fi_old,
                                                          const double2* __restrict__ fe_old,
                                                          const double2* __restrict__ cout_M,
                                                          const double2* __restrict__ tau,
                                                          double2* __restrict__ sq, double2* __restrict__ rec) {
    const long long i = (long long)blockIdx.x * NODE_T1 + threadIdx.x;
    if (i >= nspec) return;
    const long long ns3 = 3 * nspec;
    double2 fi[M + 1][3], fe[M + 1][3];                 // the old F at nodes 0..M
    const int JL = cout_M ? M : M + 1;                  // nodes read from memory
#pragma unroll
    for (int j = 0; j <= M; ++j)
        if (j < JL) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                fi[j][c] = fi_old[j * ns3 + c * nspec + i];
                fe[j][c] = fe_old[j * ns3 + c * nspec + i];
            }
        }
    if (cout_M)                                         // node M's F from its analyses and Theta^M
        combine_one(cout_M, theta + M * ns3, N, nspec, p, i, ord[i], deg[i], fe[M], fi[M]);
    double2 t0[3], acc0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) t0[c] = theta[c * nspec + i];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double2 acc = t0[c];
#pragma unroll
            for (int j = 0; j <= M; ++j) acc = caxpy(R.q[m][j], cadd(fi[j][c], fe[j][c]), acc);
#pragma unroll
            for (int j = 1; j <= m; ++j) {
                acc = caxpy(-R.qe[m][j], fe[j][c], acc);
                acc = caxpy(-R.qd[m][j], fi[j][c], acc);
            }
            acc = caxpy(-R.h[m], fi[m + 1][c], acc);
            if (tau) acc = cadd(acc, tau[(m + 1) * ns3 + c * nspec + i]);
            if (m == 0)
                acc0[c] = acc;
            else
                sq[(m + 1) * ns3 + c * nspec + i] = acc;
        }
    const int n = deg[i];
    double2 x[3];
    solve_one(n * (n + 1.0) / (p.a * p.a), R.h[0], p, acc0[0], acc0[1], acc0[2], x[0], x[1], x[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        theta[ns3 + c * nspec + i] = x[c];
        if (rec) rec[c * nspec + i] = x[c];
    }
}

__global__ __launch_bounds__(3 * NODE_CO) void k_sdc_node(const int* __restrict__ ord, const int* __restrict__ deg,
                                                        int N, long long nspec, swe_params p, int m,
                                                        NodeWeights wt, double h, double2* __restrict__ theta,
                                                        double2* __restrict__ fi, double2* __restrict__ fe,
                                                        const double2* __restrict__ cout,
                                                        double2* __restrict__ rec) {
    __shared__ double2 bsh[3][NODE_CO];
    const int c = threadIdx.x / NODE_CO, loc = threadIdx.x - c * NODE_CO;
    const long long i = (long long)blockIdx.x * NODE_CO + loc;
    const bool on = i < nspec;
    const long long ns3 = 3 * nspec, o = c * nspec + i;
    double2 acc = make_double2(0.0, 0.0);
    if (on) {
        double2 fem, fim;
        combine_field(cout, theta + m * ns3, N, nspec, p, i, ord[i], deg[i], c, fem, fim);
        acc = fe[(m + 1) * ns3 + o];                    // S_m from the sweep's first update
        fe[m * ns3 + o] = fem;
        fi[m * ns3 + o] = fim;
        for (int j = 1; j < m; ++j) {
            acc = caxpy(wt.qe[j], fe[j * ns3 + o], acc);
            acc = caxpy(wt.qd[j], fi[j * ns3 + o], acc);
        }
        acc = caxpy(wt.qe[m], fem, acc);
        acc = caxpy(wt.qd[m], fim, acc);
    }
    node_solve(deg, p, h, c, loc, i, on, acc, bsh, theta + (m + 1) * ns3, rec, o);
}

// dst[i][c] = sum_j Pi[i][j] src[j][map(c)], i in [i0, i1); c runs over the
// coarse coefficients, map(c) is the fine index of the same (m, n).  One
// thread per (coefficient, field = blockIdx.y, node i0 + blockIdx.z).
__global__ void k_restrict(const int* __restrict__ ordc, const int* __restrict__ degc, int Nf, int Nc,
                           long long nsf, long long nsc, Mat9x9 Pi, int nsrc, int i0,
                           const double2* __restrict__ src, double2* __restrict__ dst,
                           double2* __restrict__ dst2) {
    const long long c = (long long)blockIdx.x * TB + threadIdx.x;
    if (c >= nsc) return;
    const int f = blockIdx.y, i = i0 + blockIdx.z;
    const long long fidx = spec_idx(Nf, ordc[c], degc[c]);
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < nsrc; ++j) {
        const double w = Pi.a[i * nsrc + j];
        if (w != 0.0) acc = caxpy(w, src[(j * 3 + f) * nsf + fidx], acc);
    }
    dst[(i * 3 + f) * nsc + c] = acc;
    if (dst2) dst2[(i * 3 + f) * nsc + c] = acc;
}

// dst_p[m] = src_p[0] for nodes m = first_p..last_p (element-wise over n3).
__global__ void k_node_copies(NodeCopies nc, long long n3) {
    const long long e = (long long)blockIdx.x * TB + threadIdx.x;
    if (e >= n3) return;
    for (int q = 0; q < nc.n; ++q) {
        const double2 v = nc.src[q][e];
        for (int m = nc.first[q]; m <= nc.last[q]; ++m) nc.dst[q][m * n3 + e] = v;
    }
}

// tau_c^i = dt [sum_j (Pi Q_f)_{ij} D(F_f^j) - sum_j (Q_c)_{ij} F_c^j], i = 0..nc-1.
// One thread per (coefficient, field = blockIdx.y, node i = blockIdx.z).
__global__ void k_fas_tau(const int* __restrict__ ordc, const int* __restrict__ degc, int Nf, int Nc,
                          long long nsf, long long nsc, Mat9x9 PQ, Mat9x9 Qc, int nf, int nc, double dt,
                          const double2* __restrict__ fi_f, const double2* __restrict__ fe_f,
                          const double2* __restrict__ fi_c, const double2* __restrict__ fe_c,
                          double2* __restrict__ tau) {
    const long long c = (long long)blockIdx.x * TB + threadIdx.x;
    if (c >= nsc) return;
    const int f = blockIdx.y, i = blockIdx.z;
    const long long fidx = spec_idx(Nf, ordc[c], degc[c]);
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < nf; ++j) {
        const long long o = (j * 3 + f) * nsf + fidx;
        acc = caxpy(PQ.a[i * nf + j], cadd(fi_f[o], fe_f[o]), acc);
    }
    for (int j = 0; j < nc; ++j) {
        const long long o = (j * 3 + f) * nsc + c;
        acc = caxpy(-Qc.a[i * nc + j], cadd(fi_c[o], fe_c[o]), acc);
    }
    tau[(i * 3 + f) * nsc + c] = cscale(dt, acc);
}

// For fine nodes m = 1..nf-1: X_f^m += Pad(sum_i Pfc[m][i] (X_c^i - X~_c^i)) for
// X in {Theta, F_I, F_E}; only the coefficients with n <= N_c change.  One
// thread per (coarse coefficient, field = blockIdx.y) reads the coarse
// differences once and updates every fine node (nf, nc <= 9).
__global__ __launch_bounds__(64) void k_interp(const int* __restrict__ ordc, const int* __restrict__ degc, int Nf,
                                               int Nc, long long nsf, long long nsc, Mat9x9 P, int nf, int nc,
                                               const double2* __restrict__ thc, const double2* __restrict__ thct,
                                               const double2* __restrict__ fic, const double2* __restrict__ fict,
                                               const double2* __restrict__ fec, const double2* __restrict__ fect,
                                               double2* __restrict__ thf, double2* __restrict__ fif,
                                               double2* __restrict__ fef) {
    const long long c = (long long)blockIdx.x * 64 + threadIdx.x;
    if (c >= nsc) return;
    const int f = blockIdx.y;
    const long long fidx = spec_idx(Nf, ordc[c], degc[c]);
    double2 a[8], b[8], d[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) a[m] = b[m] = d[m] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (i < nc) {
            const long long o = (i * 3 + f) * nsc + c;
            const double2 x = csub(thc[o], thct[o]), y = csub(fic[o], fict[o]), z = csub(fec[o], fect[o]);
#pragma unroll
            for (int m = 1; m < 9; ++m)
                if (m < nf) {
                    const double w = P.a[m * nc + i];
                    a[m - 1] = caxpy(w, x, a[m - 1]);
                    b[m - 1] = caxpy(w, y, b[m - 1]);
                    d[m - 1] = caxpy(w, z, d[m - 1]);
                }
        }
#pragma unroll
    for (int m = 1; m < 9; ++m)
        if (m < nf) {
            const long long o = (m * 3 + f) * nsf + fidx;
            thf[o] = cadd(thf[o], a[m - 1]);
            fif[o] = cadd(fif[o], b[m - 1]);
            fef[o] = cadd(fef[o], d[m - 1]);
        }
}

// Per-block partial sums for the residual: [blk][M+1] of ||r^m||^2 (m >= 1)
// and slot 0 holds ||Theta^0||^2.  r^m = Theta^0 + dt sum_j Q[m][j] F^j - Theta^m.
__global__ void k_residual(long long nspec, Mat9x9 Q, int M, double dt, const double2* __restrict__ th,
                           const double2* __restrict__ fi, const double2* __restrict__ fe,
                           double* __restrict__ partial) {
    __shared__ double red[TB];
    const long long ns3 = 3 * nspec;
    double loc[10];
    for (int m = 0; m <= M; ++m) loc[m] = 0.0;
    for (long long o = (long long)blockIdx.x * TB + threadIdx.x; o < ns3; o += (long long)gridDim.x * TB) {
        const double2 t0 = th[o];
        loc[0] += t0.x * t0.x + t0.y * t0.y;
        for (int m = 1; m <= M; ++m) {
            double2 r = t0;
            for (int j = 0; j <= M; ++j) r = caxpy(dt * Q.a[m * (M + 1) + j], cadd(fi[j * ns3 + o], fe[j * ns3 + o]), r);
            r = csub(r, th[m * ns3 + o]);
            loc[m] += r.x * r.x + r.y * r.y;
        }
    }
    for (int m = 0; m <= M; ++m) {
        red[threadIdx.x] = loc[m];
        __syncthreads();
        for (int w = TB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blockIdx.x * (M + 1) + m] = red[0];
        __syncthreads();
    }
}

// status[0] = max_m sqrt(sum r^m) / sqrt(sum Theta^0) (or 0); status[1] = any non-finite.
__global__ void k_status(const double* __restrict__ partial, int nblk, int M, const double2* __restrict__ th,
                         long long n3, double* __restrict__ status, int residual_on) {
    __shared__ int bad;
    __shared__ double red[TB];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int lbad = 0;
    for (long long o = threadIdx.x; o < n3; o += TB) {
        const double2 v = th[o];
        if (!isfinite(v.x) || !isfinite(v.y)) lbad = 1;
    }
    if (lbad) atomicOr(&bad, 1);
    double res = 0.0;
    if (residual_on) {
        double s0 = 0.0;
        for (int m = 0; m <= M; ++m) {
            double loc = 0.0;
            for (int b = threadIdx.x; b < nblk; b += TB) loc += partial[b * (M + 1) + m];
            red[threadIdx.x] = loc;
            __syncthreads();
            for (int w = TB / 2; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            const double tot = red[0];
            __syncthreads();
            if (m == 0) s0 = tot;
            else res = fmax(res, sqrt(tot));
        }
        res = (s0 > 0.0) ? res / sqrt(s0) : res;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        status[0] = res;
        status[1] = bad ? 1.0 : 0.0;
    }
}

inline unsigned nblocks(long long n) { return (unsigned)((n + TB - 1) / TB); }

}  // namespace

hipError_t launch_spec_to_ext(const shx_plan* pl, const double2* spec, double2* cin, int F, int halve,
                              hipStream_t st) {
    k_spec_to_ext<<<nblocks(pl->nspec_e), TB, 0, st>>>(pl->ord_e, pl->deg_e, spec, cin, pl->N, pl->nspec,
                                                        pl->nspec_e, F, halve);
    return hipGetLastError();
}

hipError_t launch_ext_to_spec(const shx_plan* pl, const double2* cout, double2* spec, int F, hipStream_t st) {
    k_ext_to_spec<<<nblocks(pl->nspec), TB, 0, st>>>(pl->ord, pl->deg, cout, spec, pl->N, pl->nspec, F);
    return hipGetLastError();
}

hipError_t launch_swe_combine(const shx_plan* pl, const swe_params& p, const double2* cout,
                              const double2* state, double2* fi, double2* fe, int S, hipStream_t st) {
    dim3 g(nblocks(pl->nspec), S);
    k_swe_combine<<<g, TB, 0, st>>>(pl->ord, pl->deg, cout, state, fi, fe, pl->N, pl->nspec, pl->nspec_e, p, S);
    return hipGetLastError();
}

hipError_t launch_imex_solve(const shx_plan* pl, const swe_params& p, double h, const double2* rhs,
                             double2* out, int S, hipStream_t st) {
    dim3 g(nblocks(pl->nspec), S);
    k_imex_solve<<<g, TB, 0, st>>>(pl->deg, rhs, out, pl->nspec, p, h, S);
    return hipGetLastError();
}

hipError_t launch_sdc_node_first(const shx_plan* pl, const swe_params& p, int M, const NodeRows& rows,
                                 double2* theta, const double2* fi_old, const double2* fe_old, const double2* cout_M,
                                 const double2* tau, double2* sq, double2* rec, hipStream_t st) {
    const unsigned nb = (unsigned)((pl->nspec + NODE_T1 - 1) / NODE_T1);
    switch (M) {
#define SHX_NODE_FIRST(MM)                                                                                        \
    case MM:                                                                                                      \
        k_sdc_node_first<MM><<<nb, NODE_T1, 0, st>>>(pl->ord, pl->deg, pl->N, pl->nspec, p, rows, theta, fi_old, \
                                                     fe_old, cout_M, tau, sq, rec);                              \
        break;
        SHX_NODE_FIRST(1) SHX_NODE_FIRST(2) SHX_NODE_FIRST(3) SHX_NODE_FIRST(4)
        SHX_NODE_FIRST(5) SHX_NODE_FIRST(6) SHX_NODE_FIRST(7) SHX_NODE_FIRST(8)
#undef SHX_NODE_FIRST
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sdc_node(const shx_plan* pl, const swe_params& p, int m, int M, const NodeWeights& wts,
                           double h, double2* theta, double2* fi, double2* fe, const double2* cout_m,
                           double2* rec, hipStream_t st) {
    if (!cout_m || m < 1 || m >= M) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((pl->nspec + NODE_CO - 1) / NODE_CO);
    k_sdc_node<<<nb, 3 * NODE_CO, 0, st>>>(pl->ord, pl->deg, pl->N, pl->nspec, p, m, wts, h, theta, fi, fe,
                                          cout_m, rec);
    return hipGetLastError();
}

hipError_t launch_restrict(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pi, int nsrc, int i0,
                           int i1, const double2* src, double2* dst, double2* dst2, hipStream_t st) {
    if (i1 <= i0) return hipSuccess;
    dim3 g(nblocks(coarse->nspec), 3, i1 - i0);
    k_restrict<<<g, TB, 0, st>>>(coarse->ord, coarse->deg, fine->N, coarse->N, fine->nspec, coarse->nspec, Pi,
                                 nsrc, i0, src, dst, dst2);
    return hipGetLastError();
}

hipError_t launch_node_copies(const NodeCopies& nc, long long n3, hipStream_t st) {
    k_node_copies<<<nblocks(n3), TB, 0, st>>>(nc, n3);
    return hipGetLastError();
}

hipError_t launch_fas_tau(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& PQ, const Mat9x9& Qc,
                          int nf, int nc, double dt, const double2* fi_f, const double2* fe_f,
                          const double2* fi_c, const double2* fe_c, double2* tau, hipStream_t st) {
    dim3 g(nblocks(coarse->nspec), 3, nc);
    k_fas_tau<<<g, TB, 0, st>>>(coarse->ord, coarse->deg, fine->N, coarse->N, fine->nspec, coarse->nspec, PQ, Qc,
                                nf, nc, dt, fi_f, fe_f, fi_c, fe_c, tau);
    return hipGetLastError();
}

hipError_t launch_interp(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pfc, int nf, int nc,
                         const double2* th_c, const double2* th_ct, const double2* fi_c, const double2* fi_ct,
                         const double2* fe_c, const double2* fe_ct, double2* th_f, double2* fi_f,
                         double2* fe_f, hipStream_t st) {
    if (nf < 2) return hipSuccess;
    if (nf > 9 || nc > 9) return hipErrorInvalidValue;
    dim3 g((unsigned)((coarse->nspec + 63) / 64), 3);
    k_interp<<<g, 64, 0, st>>>(coarse->ord, coarse->deg, fine->N, coarse->N, fine->nspec, coarse->nspec, Pfc, nf,
                               nc, th_c, th_ct, fi_c, fi_ct, fe_c, fe_ct, th_f, fi_f, fe_f);
    return hipGetLastError();
}

int residual_blocks(const shx_plan* pl) {
    long long n = 3 * pl->nspec;
    long long b = (n + TB - 1) / TB;
    return (int)(b < 512 ? b : 512);
}

hipError_t launch_residual(const shx_plan* pl, const Mat9x9& Q, int M, double dt, const double2* theta,
                           const double2* fi, const double2* fe, double* partial, int nblk, hipStream_t st) {
    k_residual<<<nblk, TB, 0, st>>>(pl->nspec, Q, M, dt, theta, fi, fe, partial);
    return hipGetLastError();
}

hipError_t launch_status(const shx_plan* pl, const double* partial, int nblk, int M, const double2* theta_new,
                         double* status, int residual_on, hipStream_t st) {
    k_status<<<1, TB, 0, st>>>(partial, nblk, M, theta_new, 3 * pl->nspec, status, residual_on);
    return hipGetLastError();
}
