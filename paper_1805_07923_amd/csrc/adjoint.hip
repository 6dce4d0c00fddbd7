// Adjoint (transposed-Jacobian) kernels of the MLSDC-SH step, FP64.
//
// Inner products: spectral arrays <x, y> = sum over the stored (m >= 0)
// coefficients of Re x Re y + Im x Im y; grids <g, h> = sum_ij g_ij h_ij.
// With these, for the transforms of Sec. 3 (eqs. spectral_to_physical_space,
// fourier_transform, legendre_transform):
//   synthesis S:  (S^T h)^m_n = c_m sum_j P^m_n(mu_j) sum_i h_ij e^{-i m lambda_i},
//                 c_0 = 1, c_m = 2 (m >= 1);
//   analysis A_W: (A_W^T s)_ij = (W_j / I) sum_{m >= 0} Re[(sum_n s^m_n P^m_n(mu_j)) e^{i m lambda_i}],
// i.e. the analysis adjoint is a synthesis of the coefficients with those of
// m >= 1 halved.  The tendency adjoint runs: combine^T (div/curl/Laplacian),
// halving, Legendre synthesis of the cotangents, per latitude row the inverse
// FFTs of state and cotangents, the linearised products^T, forward FFTs with
// the factor c_m, the Legendre analysis with unit weights, and the wind^T
// (Helmholtz) and F_I^T.  The step-level kernels transpose the linear parts of
// the sweep node update, the FAS term and the space-time transfers.
#include "internal.h"
#include "row_fft.h"

namespace {

constexpr int TB = 256;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 caxpy(double s, double2 a, double2 y) {
    return make_double2(fma(s, a.x, y.x), fma(s, a.y, y.y));
}
// i * m * a
__device__ __forceinline__ double2 cim(double m, double2 a) { return make_double2(-m * a.y, m * a.x); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
inline unsigned nblocks(long long n) { return (unsigned)((n + TB - 1) / TB); }

// Transpose of the wind coefficients and of F_I, accumulated into lam_state:
// lam4[s][e] holds the adjoints of the synthesised (zeta, Phi', U, V) coefficients.
__global__ void k_prep_adj(const int* __restrict__ ord, const int* __restrict__ deg,
                           const double2* __restrict__ lam4, const double2* __restrict__ lfi,
                           double2* __restrict__ lstate, int N, long long nspec, long long nspec_e, swe_params p,
                           int S, int has_fe) {
    const long long i = (long long)blockIdx.x * TB + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= nspec || s >= S) return;
    const int m = ord[i], n = deg[i];
    const double L = n * (n + 1.0) / (p.a * p.a);
    double2 lphi = make_double2(0.0, 0.0), lzeta = lphi, ldelta = lphi;
    if (has_fe) {
        const double2* l4 = lam4 + (long long)s * nspec_e * 4;
        // a value, not a reference, on both branches (no address select with a local)
        auto g4 = [&](int k, int f) -> double2 {
            if (k < m || k > N + 1) return make_double2(0.0, 0.0);
            return l4[ext_idx(N, m, k) * 4 + f];
        };
        const double ia = 1.0 / p.a;
        const double cu = n * eps_nm(n + 1, m), cd = (n + 1.0) * eps_nm(n, m);
        // psi_n appears in U_{n+1} (n eps_{n+1}), U_{n-1} (-(n+1) eps_n), V_n (i m)
        double2 lpsi = cim(-m, g4(n, 3));
        lpsi = caxpy(cu, g4(n + 1, 2), lpsi);
        lpsi = caxpy(-cd, g4(n - 1, 2), lpsi);
        // chi_n appears in U_n (i m), V_{n+1} (-n eps_{n+1}), V_{n-1} ((n+1) eps_n)
        double2 lchi = cim(-m, g4(n, 2));
        lchi = caxpy(-cu, g4(n + 1, 3), lchi);
        lchi = caxpy(cd, g4(n - 1, 3), lchi);
        lpsi = cscale(ia, lpsi);
        lchi = cscale(ia, lchi);
        lzeta = g4(n, 0);
        lphi = g4(n, 1);
        if (n >= 1) {
            lzeta = caxpy(-1.0 / L, lpsi, lzeta);          // psi = -zeta / L
            ldelta = caxpy(-1.0 / L, lchi, ldelta);        // chi = -delta / L
        }
    }
    if (lfi) {
        // F_I = [-Phibar delta - nu L Phi', -nu L zeta, L Phi' - nu L delta]
        const double2* l = lfi + (long long)s * 3 * nspec;
        const double2 a0 = l[i], a1 = l[nspec + i], a2 = l[2 * nspec + i];
        lphi = caxpy(-p.nu * L, a0, lphi);
        lphi = caxpy(L, a2, lphi);
        lzeta = caxpy(-p.nu * L, a1, lzeta);
        ldelta = caxpy(-p.phibar, a0, ldelta);
        ldelta = caxpy(-p.nu * L, a2, ldelta);
    }
    double2* o = lstate + (long long)s * 3 * nspec;
    o[i] = cadd(o[i], lphi);
    o[nspec + i] = cadd(o[nspec + i], lzeta);
    o[2 * nspec + i] = cadd(o[2 * nspec + i], ldelta);
}

using rowfft::Cfg;
using rowfft::padded;
using rowfft::pidx;

// Tendency adjoint, grid part: one workgroup per (latitude row j, state s).
// FIs[s]: [2][Jh][N+1][4] state (zeta, Phi', U, V); FIl[s]: [2][Jh][N+1][5]
// cotangents of (A, B, C, D, E)^ after combine^T and halving.  Output
// Ga[s][j][m][4] = c_m * DFT_m of the grid cotangents of (zeta, Phi', U, V).
template <int L>
__global__ __launch_bounds__(Cfg<L>::T) void k_swe_grid_adj(const double2* __restrict__ FIs,
                                                               const double2* __restrict__ FIl,
                                                               const double2* __restrict__ tw,
                                                               const double* __restrict__ mu,
                                                               const double* __restrict__ cos2,
                                                               const double* __restrict__ w,
                                                               double2* __restrict__ Ga, int N, int J,
                                                               double two_omega) {
    constexpr int L2 = L / 2, T = Cfg<L>::T, P = padded(L2);
    // two 9-row buffers while the footprint stays small (L <= 192), else in place
    constexpr bool PP = (18 * P + L2) * (int)sizeof(double2) <= rowfft::PP_LDS_MAX;
    __shared__ double2 lds[(PP ? 18 : 9) * P];
    __shared__ double2 tws[L2];
    const int j = blockIdx.x, s = blockIdx.y;
    const int Jh = J / 2;
    const int jp = (j < Jh) ? j : J - 1 - j;
    const double sgn = (j < Jh) ? 1.0 : -1.0;
    // rows 0..3: the state (zeta, Phi', U, V); rows 4..8: the cotangents
    const long long ps4 = (long long)Jh * (N + 1) * 4, ps5 = (long long)Jh * (N + 1) * 5;
    const double2* e4 = FIs + (long long)s * J * (N + 1) * 4 + (long long)jp * (N + 1) * 4;
    const double2* e5 = FIl + (long long)s * J * (N + 1) * 5 + (long long)jp * (N + 1) * 5;
    auto coef = [&](int f, int m) {
        double2 a, b;
        if (f < 4) {
            a = e4[(long long)m * 4 + f];
            b = e4[(long long)m * 4 + f + ps4];
        } else {
            a = e5[(long long)m * 5 + f - 4];
            b = e5[(long long)m * 5 + f - 4 + ps5];
        }
        return make_double2(a.x + sgn * b.x, a.y + sgn * b.y);
    };
    double2* other = lds + (PP ? 9 * P : 0);
    rowfft::pack_rows<L, 9>(lds, tws, tw, N, coef);
    __syncthreads();
    double2* x = rowfft::fft<L2, T, 9, PP>(lds, other, tws, 1.0);
    double2* y = (x == lds) ? other : lds;
    const double fc = two_omega * mu[j];
    const double ic2 = 1.0 / cos2[j];
    const double wv = w[j] / (L * cos2[j]), we = w[j] / L;
    for (int k = threadIdx.x; k < L2; k += T) {
        const int q = pidx(k);
        const double2 z = x[q], ph = x[P + q], U = x[2 * P + q], V = x[3 * P + q];
        const double2 lA = x[4 * P + q], lB = x[5 * P + q], lC = x[6 * P + q], lD = x[7 * P + q],
                      lE = x[8 * P + q];
        const double2 eta = make_double2(z.x + fc, z.y + fc);
        // A = eta U, B = eta V, C = Phi' U, D = Phi' V, E = (U^2 + V^2) / (2 cos^2 phi)
        double2 gz, gp, gu, gv;
        gz.x = wv * (lA.x * U.x + lB.x * V.x);
        gz.y = wv * (lA.y * U.y + lB.y * V.y);
        gp.x = wv * (lC.x * U.x + lD.x * V.x);
        gp.y = wv * (lC.y * U.y + lD.y * V.y);
        gu.x = wv * (lA.x * eta.x + lC.x * ph.x) + we * lE.x * U.x * ic2;
        gu.y = wv * (lA.y * eta.y + lC.y * ph.y) + we * lE.y * U.y * ic2;
        gv.x = wv * (lB.x * eta.x + lD.x * ph.x) + we * lE.x * V.x * ic2;
        gv.y = wv * (lB.y * eta.y + lD.y * ph.y) + we * lE.y * V.y * ic2;
        x[q] = gz;
        x[P + q] = gp;
        x[2 * P + q] = gu;
        x[3 * P + q] = gv;
    }
    __syncthreads();
    const double2* r = rowfft::fft<L2, T, 4, PP>(x, y, tws, -1.0);
    double2* out = Ga + ((long long)s * J + j) * (N + 1) * 4;
    for (int m = threadIdx.x; m <= N; m += T) {
        const double c = (m == 0) ? 1.0 : 2.0;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double2 X = rowfft::unpack<L>(r + f * P, tws, m);
            out[(long long)m * 4 + f] = cscale(c, X);
        }
    }
}

// Transposed implicit solve: lam_b = (I - h F_I)^{-T} lam_x per coefficient.
__device__ __forceinline__ void solve_adj_one(double L, double h, const swe_params& p, double2 lp, double2 lz,
                                              double2 ld, double2& yp, double2& yz, double2& yd) {
    const double c = 1.0 + h * p.nu * L;
    const double det = c * c + h * h * p.phibar * L;
    yp = make_double2((c * lp.x + h * L * ld.x) / det, (c * lp.y + h * L * ld.y) / det);
    yd = make_double2((c * ld.x - h * p.phibar * lp.x) / det, (c * ld.y - h * p.phibar * lp.y) / det);
    yz = make_double2(lz.x / c, lz.y / c);
}

__global__ void k_imex_solve_adj(const int* __restrict__ deg, const double2* lx, double2* lb, long long nspec,
                                 swe_params p, double h, int S) {
    const long long i = (long long)blockIdx.x * TB + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= nspec || s >= S) return;
    const int n = deg[i];
    const double L = n * (n + 1.0) / (p.a * p.a);
    const double2* x = lx + (long long)s * 3 * nspec;
    double2* b = lb + (long long)s * 3 * nspec;
    double2 yp, yz, yd;
    solve_adj_one(L, h, p, x[i], x[nspec + i], x[2 * nspec + i], yp, yz, yd);
    b[i] = yp;
    b[nspec + i] = yz;
    b[2 * nspec + i] = yd;
}

// Transpose of one sweep node update (node m+1) given lth[m+1] (already
// including the tendency adjoint at that node): lam_b = solve^T(lth[m+1]),
// lth[m+1] = 0, and lam_b is spread over the inputs of the quadrature.
// Blocks of NODE_ADJ_CO coefficients x 3 fields: every thread solves the
// transposed 2 x 2 system of its coefficient (the three cotangents of node
// m+1 are read before any is cleared) and applies field c of the result.
constexpr int NODE_ADJ_CO = 32;
__global__ __launch_bounds__(3 * NODE_ADJ_CO) void k_sdc_node_adj(const int* __restrict__ deg, long long nspec,
                                                                swe_params p, int m, int M, NodeWeights wt,
                                                                double h, double2* __restrict__ lth,
                                                                double2* __restrict__ lfi_new,
                                                                double2* __restrict__ lfe_new,
                                                                double2* __restrict__ lfi_in,
                                                                double2* __restrict__ lfe_in,
                                                                double2* __restrict__ ltau) {
    const int c = threadIdx.x / NODE_ADJ_CO, loc = threadIdx.x - c * NODE_ADJ_CO;
    const long long i = (long long)blockIdx.x * NODE_ADJ_CO + loc;
    const bool on = i < nspec;
    const long long ns3 = 3 * nspec;
    double2* t = lth + (m + 1) * ns3;
    double2 lb[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    if (on) {
        const int n = deg[i];
        const double L = n * (n + 1.0) / (p.a * p.a);
        solve_adj_one(L, h, p, t[i], t[nspec + i], t[2 * nspec + i], lb[0], lb[1], lb[2]);
    }
    __syncthreads();                                    // all three reads of node m+1 done
    if (!on) return;
    const long long o = c * nspec + i;
    const double2 b = (c == 0) ? lb[0] : ((c == 1) ? lb[1] : lb[2]);
    t[o] = make_double2(0.0, 0.0);
    lth[o] = cadd(lth[o], b);
    for (int j = 0; j <= M; ++j) {
        lfi_in[j * ns3 + o] = caxpy(wt.q[j], b, lfi_in[j * ns3 + o]);
        lfe_in[j * ns3 + o] = caxpy(wt.q[j], b, lfe_in[j * ns3 + o]);
    }
    for (int j = 1; j <= m; ++j) {
        lfe_new[j * ns3 + o] = caxpy(wt.qe[j], b, lfe_new[j * ns3 + o]);
        lfe_in[j * ns3 + o] = caxpy(-wt.qe[j], b, lfe_in[j * ns3 + o]);
        lfi_new[j * ns3 + o] = caxpy(wt.qd[j], b, lfi_new[j * ns3 + o]);
        lfi_in[j * ns3 + o] = caxpy(-wt.qd[j], b, lfi_in[j * ns3 + o]);
    }
    lfi_in[(m + 1) * ns3 + o] = caxpy(-h, b, lfi_in[(m + 1) * ns3 + o]);
    if (ltau) ltau[(m + 1) * ns3 + o] = cadd(ltau[(m + 1) * ns3 + o], b);
}

// lf[j][map(c)] += sum_{i0 <= i < i1} Pi[i][j] lc[i][c]   (restriction^T = zero padding)
__global__ void k_restrict_adj(const int* __restrict__ ordc, const int* __restrict__ degc, int Nf, long long nsf,
                               long long nsc, Mat9x9 Pi, int nsrc, int i0, int i1, const double2* __restrict__ lc,
                               double2* __restrict__ lf) {
    const long long c = (long long)blockIdx.x * TB + threadIdx.x;
    const int f = blockIdx.y, j = blockIdx.z;           // field, target node
    if (c >= nsc) return;
    const long long fidx = spec_idx(Nf, ordc[c], degc[c]);
    double2 acc = lf[(j * 3 + f) * nsf + fidx];
    for (int i = i0; i < i1; ++i) acc = caxpy(Pi.a[i * nsrc + j], lc[(i * 3 + f) * nsc + c], acc);
    lf[(j * 3 + f) * nsf + fidx] = acc;
}

// Transpose of step D for Theta, F_I, F_E: for coarse node i,
// q = sum_{m >= 1} Pfc[m][i] D(lf[m]); lc[i] += q; lct[i] -= q.
__global__ void k_interp_adj(const int* __restrict__ ordc, const int* __restrict__ degc, int Nf, long long nsf,
                             long long nsc, Mat9x9 P, int nf, int nc, const double2* __restrict__ lthf,
                             const double2* __restrict__ lfif, const double2* __restrict__ lfef,
                             double2* __restrict__ lthc, double2* __restrict__ lthct, double2* __restrict__ lfic,
                             double2* __restrict__ lfict, double2* __restrict__ lfec, double2* __restrict__ lfect) {
    const long long c = (long long)blockIdx.x * TB + threadIdx.x;
    const int f = blockIdx.y, i = blockIdx.z;           // field, coarse node
    if (c >= nsc) return;
    const long long fidx = spec_idx(Nf, ordc[c], degc[c]);
    double2 a = make_double2(0.0, 0.0), b = a, d = a;
    for (int m = 1; m < nf; ++m) {
        const double wgt = P.a[m * nc + i];
        const long long o = (m * 3 + f) * nsf + fidx;
        a = caxpy(wgt, lthf[o], a);
        b = caxpy(wgt, lfif[o], b);
        d = caxpy(wgt, lfef[o], d);
    }
    const long long o = (i * 3 + f) * nsc + c;
    lthc[o] = cadd(lthc[o], a);
    lthct[o] = csub(lthct[o], a);
    lfic[o] = cadd(lfic[o], b);
    lfict[o] = csub(lfict[o], b);
    lfec[o] = cadd(lfec[o], d);
    lfect[o] = csub(lfect[o], d);
}

// Transpose of the FAS term: lfi_f[j], lfe_f[j] += dt Pad(sum_i PQ[i][j] ltau[i]);
// lfi_c[j], lfe_c[j] -= dt sum_i Qc[i][j] ltau[i].
__global__ void k_fas_tau_adj(const int* __restrict__ ordc, const int* __restrict__ degc, int Nf, long long nsf,
                              long long nsc, Mat9x9 PQ, Mat9x9 Qc, int nf, int nc, double dt,
                              const double2* __restrict__ ltau, double2* __restrict__ lfif,
                              double2* __restrict__ lfef, double2* __restrict__ lfic, double2* __restrict__ lfec) {
    const long long c = (long long)blockIdx.x * TB + threadIdx.x;
    const int f = blockIdx.y, z = blockIdx.z;           // field; fine node z < nf, else coarse node z - nf
    if (c >= nsc) return;
    if (z < nf) {
        const long long fidx = spec_idx(Nf, ordc[c], degc[c]);
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < nc; ++i) acc = caxpy(PQ.a[i * nf + z], ltau[(i * 3 + f) * nsc + c], acc);
        const long long o = (z * 3 + f) * nsf + fidx;
        lfif[o] = caxpy(dt, acc, lfif[o]);
        lfef[o] = caxpy(dt, acc, lfef[o]);
    } else {
        const int j = z - nf;
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < nc; ++i) acc = caxpy(Qc.a[i * nc + j], ltau[(i * 3 + f) * nsc + c], acc);
        const long long o = (j * 3 + f) * nsc + c;
        lfic[o] = caxpy(-dt, acc, lfic[o]);
        lfec[o] = caxpy(-dt, acc, lfec[o]);
    }
}

// y[e] (+)= sum_{m = 0}^{nn-1} x[m][e]  (node sums), acc != 0 adds to y.
__global__ void k_node_sum(const double2* __restrict__ x, double2* __restrict__ y, long long n3, int nn, int acc) {
    const long long e = (long long)blockIdx.x * TB + threadIdx.x;
    if (e >= n3) return;
    double2 s = acc ? y[e] : make_double2(0.0, 0.0);
    for (int m = 0; m < nn; ++m) s = cadd(s, x[m * n3 + e]);
    y[e] = s;
}

// y += x (elementwise over n complex values).
__global__ void k_add(const double2* __restrict__ x, double2* __restrict__ y, long long n) {
    const long long e = (long long)blockIdx.x * TB + threadIdx.x;
    if (e < n) y[e] = cadd(y[e], x[e]);
}

// The same over the arrays of a list (blockIdx.y picks the array).
__global__ void k_zero_n(ArrayList a, long long n) {
    const long long e = (long long)blockIdx.x * TB + threadIdx.x;
    if (e < n) a.y[blockIdx.y][e] = make_double2(0.0, 0.0);
}
__global__ void k_add_n(ArrayList a, long long n) {
    const long long e = (long long)blockIdx.x * TB + threadIdx.x;
    double2* y = a.y[blockIdx.y];
    if (e < n) y[e] = cadd(y[e], a.x[blockIdx.y][e]);
}

template <int L>
hipError_t grid_adj_t(const shx_plan* pl, const double2* FIs, const double2* FIl, double2* Ga, int S, double omega,
                      hipStream_t st) {
    dim3 g(pl->J, S);
    k_swe_grid_adj<L><<<g, Cfg<L>::T, 0, st>>>(FIs, FIl, pl->tw, pl->mu, pl->cos2, pl->w, Ga, pl->N, pl->J,
                                                   2.0 * omega);
    return hipGetLastError();
}

#define SHX_ADJ_LENGTHS(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(48) X(96) X(192) X(384) X(768) X(1536)

// The same transposed products for rows too long for the nine rows of the
// kernel above to fit in LDS (2048, 3072 points), on grids in HBM:
// g[9][J][L] holds the inverse transforms of (zeta, Phi', U, V) and of the
// cotangents of (A, B, C, D, E); the grid cotangents of (zeta, Phi', U, V)
// are written over rows 4..7.  One thread per grid point.
__global__ void k_swe_adj_prod(double* __restrict__ g, const double* __restrict__ mu,
                               const double* __restrict__ cos2, const double* __restrict__ w, int J, int L,
                               double two_omega) {
    const long long n = (long long)J * L;
    const long long e = (long long)blockIdx.x * TB + threadIdx.x;
    if (e >= n) return;
    const int j = (int)(e / L);
    const double fc = two_omega * mu[j];
    const double ic2 = 1.0 / cos2[j];
    const double wv = w[j] / (L * cos2[j]), we = w[j] / L;
    const double z = g[e], ph = g[n + e], U = g[2 * n + e], V = g[3 * n + e];
    const double lA = g[4 * n + e], lB = g[5 * n + e], lC = g[6 * n + e], lD = g[7 * n + e], lE = g[8 * n + e];
    const double eta = z + fc;
    g[4 * n + e] = wv * (lA * U + lB * V);
    g[5 * n + e] = wv * (lC * U + lD * V);
    g[6 * n + e] = wv * (lA * eta + lC * ph) + we * lE * U * ic2;
    g[7 * n + e] = wv * (lB * eta + lD * ph) + we * lE * V * ic2;
}

bool lds_adj_length(int L) {
    switch (L) {
#define CASE(n) case n:
        SHX_ADJ_LENGTHS(CASE)
#undef CASE
        return true;
        default: return false;
    }
}

}  // namespace

bool adjoint_length_supported(int L) { return lds_adj_length(L) || fft_length_supported(L); }

size_t adj_grid_doubles(const shx_plan* pl, int S) {
    return lds_adj_length(pl->I) ? 0 : (size_t)S * 9 * pl->J * pl->I;
}

hipError_t launch_prep_adj(const shx_plan* pl, const swe_params& p, const double2* lam4, const double2* lfi,
                           double2* lstate, int S, int has_fe, hipStream_t st) {
    dim3 g(nblocks(pl->nspec), S);
    k_prep_adj<<<g, TB, 0, st>>>(pl->ord, pl->deg, lam4, lfi, lstate, pl->N, pl->nspec, pl->nspec_e, p, S, has_fe);
    return hipGetLastError();
}

hipError_t launch_swe_grid_adj(const shx_plan* pl, const double2* FIs, const double2* FIl, double2* Ga, int S,
                               double omega, double* grid, hipStream_t st) {
    switch (pl->I) {
#define CASE(n) case n: return grid_adj_t<n>(pl, FIs, FIl, Ga, S, omega, st);
        SHX_ADJ_LENGTHS(CASE)
#undef CASE
        default: break;
    }
    // longer rows: inverse transforms into HBM, pointwise products, forward
    // transforms with the factor c_m (1 for m = 0, else 2)
    if (!grid) return hipErrorInvalidValue;
    const long long fj = (long long)pl->J * (pl->N + 1), n = (long long)pl->J * pl->I;
    for (int s = 0; s < S; ++s) {
        double* g = grid + (long long)s * 9 * n;
        hipError_t e = launch_fft_inv(pl, FIs + s * fj * 4, g, 4, 0, st);
        if (e == hipSuccess) e = launch_fft_inv(pl, FIl + s * fj * 5, g + 4 * n, 5, 0, st);
        if (e != hipSuccess) return e;
        k_swe_adj_prod<<<(unsigned)((n + TB - 1) / TB), TB, 0, st>>>(g, pl->mu, pl->cos2, pl->w, pl->J, pl->I,
                                                                    2.0 * omega);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_fft_fwd(pl, g + 4 * n, Ga + s * fj * 4, 4, 1, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_imex_solve_adj(const shx_plan* pl, const swe_params& p, double h, const double2* lx,
                                 double2* lb, int S, hipStream_t st) {
    dim3 g(nblocks(pl->nspec), S);
    k_imex_solve_adj<<<g, TB, 0, st>>>(pl->deg, lx, lb, pl->nspec, p, h, S);
    return hipGetLastError();
}

hipError_t launch_sdc_node_adj(const shx_plan* pl, const swe_params& p, int m, int M, const NodeWeights& wt,
                               double h, double2* lth, double2* lfi_new, double2* lfe_new, double2* lfi_in,
                               double2* lfe_in, double2* ltau, hipStream_t st) {
    const unsigned nb = (unsigned)((pl->nspec + NODE_ADJ_CO - 1) / NODE_ADJ_CO);
    k_sdc_node_adj<<<nb, 3 * NODE_ADJ_CO, 0, st>>>(pl->deg, pl->nspec, p, m, M, wt, h, lth, lfi_new, lfe_new,
                                                  lfi_in, lfe_in, ltau);
    return hipGetLastError();
}

hipError_t launch_restrict_adj(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pi, int nsrc, int i0,
                               int i1, const double2* lc, double2* lf, hipStream_t st) {
    if (nsrc <= 0) return hipSuccess;
    const dim3 g((unsigned)nblocks(coarse->nspec), 3, (unsigned)nsrc);
    k_restrict_adj<<<g, TB, 0, st>>>(coarse->ord, coarse->deg, fine->N, fine->nspec,
                                                           coarse->nspec, Pi, nsrc, i0, i1, lc, lf);
    return hipGetLastError();
}

hipError_t launch_interp_adj(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pfc, int nf, int nc,
                             const double2* lthf, const double2* lfif, const double2* lfef, double2* lthc,
                             double2* lthct, double2* lfic, double2* lfict, double2* lfec, double2* lfect,
                             hipStream_t st) {
    if (nc <= 0) return hipSuccess;
    const dim3 g((unsigned)nblocks(coarse->nspec), 3, (unsigned)nc);
    k_interp_adj<<<g, TB, 0, st>>>(coarse->ord, coarse->deg, fine->N, fine->nspec,
                                                         coarse->nspec, Pfc, nf, nc, lthf, lfif, lfef, lthc, lthct,
                                                         lfic, lfict, lfec, lfect);
    return hipGetLastError();
}

hipError_t launch_fas_tau_adj(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& PQ, const Mat9x9& Qc,
                              int nf, int nc, double dt, const double2* ltau, double2* lfif, double2* lfef,
                              double2* lfic, double2* lfec, hipStream_t st) {
    const dim3 g((unsigned)nblocks(coarse->nspec), 3, (unsigned)(nf + nc));
    k_fas_tau_adj<<<g, TB, 0, st>>>(coarse->ord, coarse->deg, fine->N, fine->nspec,
                                                          coarse->nspec, PQ, Qc, nf, nc, dt, ltau, lfif, lfef, lfic,
                                                          lfec);
    return hipGetLastError();
}

hipError_t launch_node_sum(const double2* x, double2* y, long long n3, int nn, int acc, hipStream_t st) {
    k_node_sum<<<nblocks(n3), TB, 0, st>>>(x, y, n3, nn, acc);
    return hipGetLastError();
}

hipError_t launch_add(const double2* x, double2* y, long long n, hipStream_t st) {
    k_add<<<nblocks(n), TB, 0, st>>>(x, y, n);
    return hipGetLastError();
}

hipError_t launch_zero_n(const ArrayList& a, long long n, hipStream_t st) {
    if (n <= 0 || a.k < 1) return hipSuccess;
    if (a.k > 8) return hipErrorInvalidValue;
    k_zero_n<<<dim3(nblocks(n), a.k), TB, 0, st>>>(a, n);
    return hipGetLastError();
}

hipError_t launch_add_n(const ArrayList& a, long long n, hipStream_t st) {
    if (n <= 0 || a.k < 1) return hipSuccess;
    if (a.k > 8) return hipErrorInvalidValue;
    k_add_n<<<dim3(nblocks(n), a.k), TB, 0, st>>>(a, n);
    return hipGetLastError();
}

