// Internal types and device helpers of the MLSDC-SH library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "../../include/mlsdc_sh.h"

// ------------------------------------------------------------------ layouts
// Standard spectral layout (m = 0..N, n = m..N) and the extended layout used
// inside the tendency (m = 0..N, n = m..N+1; the cos-weighted wind and the
// flux analyses reach degree N+1).
__host__ __device__ inline long long spec_idx(int N, int m, int n) {
    return (long long)m * (2 * N + 3 - m) / 2 + (n - m);
}
__host__ __device__ inline long long ext_idx(int N, int m, int n) {
    return (long long)m * (2 * N + 5 - m) / 2 + (n - m);
}
__host__ __device__ inline long long nspec_of(int N) { return (long long)(N + 1) * (N + 2) / 2; }
__host__ __device__ inline long long nspec_ext_of(int N) { return (long long)(N + 1) * (N + 4) / 2; }

// latitude pairs up to which the FP64 analysis of up to 6 fields streams
// its table (beyond: the matrix-core kernel that generates P^m_n)
constexpr int AN_TAB_JH = 256;
// latitude pairs up to which FP32 plans with tables hold the tiled FP32
// analysis table (the first summed group of a tile is packed in a byte:
// at most 255 groups of 4 pairs)
constexpr int AN_TAB_JH_F32 = 1020;

// Polar truncation of the table analysis (the near-pole omission of the
// transform library of Sec. 3, Schaeffer 2013): a group of 4 latitude pairs
// is left out of the sum for a 16-degree tile when it and every group nearer
// the pole hold only |P^m_n| < AN_POLAR_TAU.  A coefficient then changes by
// at most AN_POLAR_TAU times the sum of |weighted Fourier data| over the
// omitted latitudes, 10^4 below the FP64 unit roundoff relative to the data.
constexpr double AN_POLAR_TAU = 1e-20;
// Table loads in flight per lane in the table analysis: batches of 8 groups
// of 4 latitude pairs from 160 pairs up, of 4 below (measured: T255 17.4
// against 17.7 us with 4; T127, where two wavefronts share each tile's
// latitude sum, 8.1 against 8.5 with 8).  The summed run of
// a tile starts where it holds whole batches (a ragged run would wait for
// its last loads one at a time): at max(0, ngrp - B ceil((ngrp - c0) / B))
// for the first group c0 with |P^m_n| >= AN_POLAR_TAU and ngrp groups.
constexpr int an_batch(int Jh) { return Jh >= 160 ? 8 : 4; }

// Rows of the parity block p (n - m = p mod 2) of order m for degrees <= nmax.
__host__ __device__ inline int kcount(int nmax, int m, int p) {
    return (nmax - m - p >= 0) ? (nmax - m - p) / 2 + 1 : 0;
}

// epsilon^m_n = sqrt((n^2 - m^2) / (4 n^2 - 1)), zero for n <= m.
__host__ __device__ inline double eps_nm(int n, int m) {
    if (n <= m) return 0.0;
    const double nn = (double)n, mm = (double)m;
    return sqrt((nn * nn - mm * mm) / (4.0 * nn * nn - 1.0));
}

// ------------------------------------------------ tendency input rows
// Degree factors of the rows below, tabulated per plan so that the rows are
// formed with loads and a few multiplications (no FP64 division or square
// root, which would wait behind the matrix-core products of the wavefronts
// sharing the SIMD): pf[ext(m, n)] = ((n-1) eps^m_n, (n+2) eps^m_{n+1}),
// ninv[n] = -1 / (n (n+1)) (0 at n = 0), nn1[n] = n (n+1), n <= N+2.
//
// The four grid fields of the shallow-water tendency at (m, n), n <= N+1,
// from a state (Phi', zeta, delta), each [nspec]: zeta, Phi' (zero above N)
// and the cos-weighted wind (U, V) = (u, v) cos(phi) from the stream
// function psi = -zeta / L_n and velocity potential chi = -delta / L_n
// (L_n = n (n+1) / a^2, zero at n = 0):
//   U_n = [(n-1) eps_n psi_{n-1} - (n+2) eps_{n+1} psi_{n+1} + i m chi_n] / a,
//   V_n = [i m psi_n - (n-1) eps_n chi_{n-1} + (n+2) eps_{n+1} chi_{n+1}] / a.
// pfm = pf + ext(m, m); a2 = a^2, ia = 1/a.
// ld(f, nn): state field f (0 Phi', 1 zeta, 2 delta) at degree nn of order m,
// called with m <= nn <= N only.
template <class Ld>
__device__ inline void swe_prep_row_t(Ld ld, int N, double a2, double ia, const double2* __restrict__ pfm,
                                      const double* __restrict__ ninv, int m, int n, double2 o[4]) {
    // every load is issued before the first is used: degrees outside m..N
    // are clamped to a stored entry of the order and their factor is zero
    auto cl = [&](int nn) { return nn < m ? m : (nn > N ? N : nn); };
    const int id = cl(n - 1), i0 = cl(n), iu = cl(n + 1);
    const double2 zd = ld(1, id), z0 = ld(1, i0), zu = ld(1, iu);
    const double2 dd = ld(2, id), d0 = ld(2, i0), du = ld(2, iu);
    const double2 p0 = ld(0, i0);
    const double2 cf = pfm[n - m];
    const double nd = ninv[n > 0 ? n - 1 : 0], n0 = ninv[n], nu = ninv[n + 1];
    // -1/L_nn (zero outside the stored degrees and at nn = 0)
    const double rd = (n - 1 < m || n - 1 > N) ? 0.0 : a2 * nd;
    const double r0 = (n > N) ? 0.0 : a2 * n0;
    const double ru = (n + 1 > N) ? 0.0 : a2 * nu;
    const double c_dn = cf.x, c_up = cf.y;
    auto sc = [](double r, double2 v) { return make_double2(r * v.x, r * v.y); };
    const double2 psd = sc(rd, zd), ps0 = sc(r0, z0), psu = sc(ru, zu);
    const double2 chd = sc(rd, dd), ch0 = sc(r0, d0), chu = sc(ru, du);
    const double2 U = make_double2(c_dn * psd.x - c_up * psu.x - m * ch0.y, c_dn * psd.y - c_up * psu.y + m * ch0.x);
    const double2 V = make_double2(-m * ps0.y - c_dn * chd.x + c_up * chu.x, m * ps0.x - c_dn * chd.y + c_up * chu.y);
    const bool in = n <= N;
    o[0] = in ? z0 : make_double2(0.0, 0.0);
    o[1] = in ? p0 : make_double2(0.0, 0.0);
    o[2] = make_double2(ia * U.x, ia * U.y);
    o[3] = make_double2(ia * V.x, ia * V.y);
}

__device__ inline void swe_prep_row(const double2* __restrict__ state, long long nspec, int N, double a2,
                                    double ia, const double2* __restrict__ pfm, const double* __restrict__ ninv,
                                    int m, int n, double2 o[4]) {
    swe_prep_row_t([&](int f, int nn) { return state[f * nspec + spec_idx(N, m, nn)]; }, N, a2, ia, pfm, ninv, m,
                   n, o);
}

// Transpose of the F_E combine (F_E = [-div(C, D), -div(A, B), curl(A, B)
// + L E^] of the weighted analyses A..E) at ext entry (m, n), followed by
// the halving of m >= 1 that turns the analysis adjoint into a synthesis.
// lfe: cotangents of F_E [3][nspec] (Phi', zeta, delta); o: cotangents of
// (A, B, C, D, E)^ at (m, n).  With the cotangent q of div(X, Y):
// X_n += -i m q_n / a, Y_n += [(n-1) eps_n q_{n-1} - (n+2) eps_{n+1} q_{n+1}] / a;
// with the cotangent r of curl(X, Y): Y_n += -i m r_n / a,
// X_n += [-(n-1) eps_n r_{n-1} + (n+2) eps_{n+1} r_{n+1}] / a.
// pfm, nn1 as for swe_prep_row; ia = 1/a, ia2 = 1/a^2.
__device__ inline void swe_combine_adj_row(const double2* __restrict__ lfe, long long nspec, int N, double ia,
                                           double ia2, const double2* __restrict__ pfm,
                                           const double* __restrict__ nn1, int m, int n, double2 o[5]) {
    const double2* lp = lfe;
    const double2* lz = lp + nspec;
    const double2* ld = lz + nspec;
    // every load is issued before the first is used: indices outside m..N
    // are clamped to a stored entry of the order and masked afterwards
    auto at = [&](int k) { return spec_idx(N, m, k < m ? m : (k > N ? N : k)); };
    const long long id = at(n - 1), i0 = at(n), iu = at(n + 1);
    const double2 vz0 = lz[i0], vzd = lz[id], vzu = lz[iu];
    const double2 vp0 = lp[i0], vpd = lp[id], vpu = lp[iu];
    const double2 vd0 = ld[i0], vdd = ld[id], vdu = ld[iu];
    const double2 cf = pfm[n - m];
    const double nn = nn1[n];
    const bool k0 = n >= m && n <= N, kd = n - 1 >= m && n - 1 <= N, ku = n + 1 >= m && n + 1 <= N;
    auto msk = [](bool b, double2 v) { return b ? v : make_double2(0.0, 0.0); };
    auto neg = [](double2 v) { return make_double2(-v.x, -v.y); };
    auto cim = [](double mu, double2 v) { return make_double2(-mu * v.y, mu * v.x); };   // i mu v
    auto axpy = [](double s, double2 x, double2 y) { return make_double2(fma(s, x.x, y.x), fma(s, x.y, y.y)); };
    const double cdn = cf.x, cup = cf.y;
    // q_AB = -lz, q_CD = -lp, r_AB = ld
    const double2 qab0 = neg(msk(k0, vz0)), qabd = neg(msk(kd, vzd)), qabu = neg(msk(ku, vzu));
    const double2 qcd0 = neg(msk(k0, vp0)), qcdd = neg(msk(kd, vpd)), qcdu = neg(msk(ku, vpu));
    const double2 r0 = msk(k0, vd0), rd = msk(kd, vdd), ru = msk(ku, vdu);
    double2 A = cim(-m, qab0);
    A = axpy(-cdn, rd, A);
    A = axpy(cup, ru, A);
    double2 B = cim(-m, r0);
    B = axpy(cdn, qabd, B);
    B = axpy(-cup, qabu, B);
    const double2 C = cim(-m, qcd0);
    double2 D = make_double2(0.0, 0.0);
    D = axpy(cdn, qcdd, D);
    D = axpy(-cup, qcdu, D);
    const double L = nn * ia2;
    const double2 E = (n <= N) ? make_double2(L * r0.x, L * r0.y) : make_double2(0.0, 0.0);
    const double hm = (m == 0) ? ia : 0.5 * ia;          // 1/a and the halving for m >= 1
    const double he = (m == 0) ? 1.0 : 0.5;
    o[0] = make_double2(hm * A.x, hm * A.y);
    o[1] = make_double2(hm * B.x, hm * B.y);
    o[2] = make_double2(hm * C.x, hm * C.y);
    o[3] = make_double2(hm * D.x, hm * D.y);
    o[4] = make_double2(he * E.x, he * E.y);
}

// ------------------------------------------------------ XCD-aware blocks
// Workgroups go to the 8 XCDs of the chip round robin by hardware id, and
// each XCD has its own L2.  A Legendre launch has gx blocks per (order m,
// parity p); they all stage the same operand of order m.  With the blocks
// numbered so that every block of an order runs on one XCD, the repeated
// staging reads hit that XCD's L2; orders are dealt to the XCDs round robin
// (m = xcd, xcd + 8, ...), which keeps the XCDs' shares of work even.
// np = 1 for launches that take both parities of an order in one block.
// Restart segmentation of the in-kernel Legendre recurrence: the K degrees
// of an order are cut into 4 R segments of L degrees (a multiple of 8),
// R = ceil(K / 256), so that no segment runs more than 64 plain FP64
// recurrence steps.
__host__ __device__ inline int seg_rounds(int K) { return (K + 255) / 256; }
__host__ __device__ inline int seg_len(int K) {
    const int R = seg_rounds(K);
    return 8 * ((K + 32 * R - 1) / (32 * R));
}

struct LegTile {
    int x, p, m;
};
__device__ inline LegTile leg_tile(int gx, int nm, int np = 2) {
    const int hw = blockIdx.x, per_m = np * gx;
    if (nm % 8 == 0) {
        const int xcd = hw % 8, slot = hw / 8;
        const int i = slot / per_m, r = slot - i * per_m;
        return {r % gx, r / gx, xcd + 8 * i};
    }
    const int r = hw % per_m;
    return {r % gx, r / gx, hw / per_m};
}

// -------------------------------------------------------------------- plans
struct shx_plan {
    int N = 0, J = 0, I = 0, prec = 0, dev = 0;
    int tmode = SHX_TABLE_HBM;      // P^m_n tables held in HBM, or regenerated on the fly (no tables)
    int nmax = 0;                   // N + 1: degree range of tables / ext layout
    int Jh = 0;                     // J / 2 latitude pairs
    long long nspec = 0, nspec_e = 0;
    double* mu = nullptr;           // device [J]
    double* sint = nullptr;         // device [J]
    double* cos2 = nullptr;         // device [J], 1 - mu^2
    double* w = nullptr;            // device [J]
    double2* tw = nullptr;          // device [I], e^{-2 pi i t / I}
    double* psyn = nullptr;         // FP64 table, [m][p][k][jp] (FP64 plans)
    double* pan = nullptr;          // FP64 table, [m][p][jp][k]: the source of pan4 and of the
                                    // reduced-precision analysis tables, freed once they are built
    float* psyn32 = nullptr;        // FP32 tables (SHX_FP32 plans), same layouts
    float* pan32 = nullptr;
    unsigned short* an16 = nullptr;   // bf16 split planes for the analysis, [q][m][p][k][jp pad 16]
    unsigned short* syn16 = nullptr;  // bf16 split planes for the synthesis, [q][m][p][jp][k pad 16]
    long long an16_plane = 0, syn16_plane = 0;
    long long* off_an16 = nullptr;    // device [(N+1)*2] offsets into a bf16 plane
    long long* off_syn16 = nullptr;
    long long* off = nullptr;       // device [(N+1)*2] table offsets (elements)
    // Analysis table laid out for the matrix-core table analyses (FP64
    // plans with tables and at most 256 latitude pairs; pan4f for FP32):
    // pan4[off4[2m+p] + kt * ngrp * 64 + (c * 4 + kq) * r + i] = P^m_{m+p+2k}(mu_jp),
    // k = 16 kt + i (i < r), jp = 4 c + kq, ngrp = ceil(Jh / 4), r = the rows
    // of tile kt (16, fewer in the block's last tile); zero past the latitude
    // pairs, so that one operand of r degrees x 4 latitude pairs is 4 r
    // consecutive values (64 for a whole tile) and no padding rows are stored.
    double* pan4 = nullptr;
    float* pan4f = nullptr;         // the same layout rounded to FP32 (SHX_FP32 plans, Jh <= AN_TAB_JH_F32)
    long long* off4 = nullptr;
    // an_c0[(2m+p) * an_kt + kt]: first latitude group c of tile kt of pan4
    // that holds a value of magnitude >= AN_POLAR_TAU (ngrp if none); an_kt =
    // tiles of the largest order-parity block.  Set-up only: h_an_c0 keeps
    // the first summed groups (moved back to whole load batches).
    int* an_c0 = nullptr;
    int an_kt = 0;
    // Recurrence data of the FP64 kernels that generate P^m_n in registers:
    // ck[ckoff[m] + g * Jh + jp] = (P^m_{m+g*L}, P^m_{m+g*L+1}) at mu_jp for the
    // 4 R segments g of the order (L = seg_len, R = seg_rounds of its
    // nmax - m + 1 degrees; zero past nmax), from the double-double recurrence;
    // rc[ext(m, n)] = (1/eps^m_n, eps^m_{n-1}/eps^m_n) for n >= m + 2.
    double2* ck = nullptr;
    long long* ckoff = nullptr;     // device [N+1]
    double2* rc = nullptr;          // device [nspec_e]
    double* rq = nullptr;           // device [nspec_e], (eps^m_{n-1})^2 for n >= m + 2, else 0
    double* cs = nullptr;           // device [nspec_e], C_n of the restart segments (P = C Q)
    double2* pf = nullptr;          // device [nspec_e], degree factors of swe_prep_row
    double* ninv = nullptr;         // device [N+3], -1/(n(n+1)), 0 at n = 0
    double* nn1 = nullptr;          // device [N+3], n(n+1)
    // Blocks of the FP64 analysis, (m, segment g) pairs [2 an_nblk]: all
    // blocks of an order on one XCD (block b runs on XCD b mod 8), (-1, -1)
    // for padding.
    int* anblk = nullptr;
    int an_nblk = 0;
    // Blocks of the table analysis [4 tb_nblk]: (2 m + p, tile of 64 degrees,
    // first summed latitude group of each of its four 16-degree tiles (byte
    // w for tile w; ngrp past the rows), the smallest of these) for the tiles
    // that hold rows (n <= N+1), listed XCD by XCD as anblk, -1 for padding.
    // Only plans with pan4 have it.
    int* tblk = nullptr;
    int tb_nblk = 0;
    int* ord = nullptr;             // device [nspec] zonal order of each entry
    int* deg = nullptr;             // device [nspec] degree of each entry
    int* ord_e = nullptr;           // device [nspec_e]
    int* deg_e = nullptr;           // device [nspec_e]
    long long table_elems = 0;
    std::vector<double> h_mu, h_sint, h_cos2, h_w;
    std::vector<long long> h_off;
    std::vector<int> h_an_c0;       // first summed group per tile, an_c0's layout (plans with pan4)
};

struct sdc_level {
    const shx_plan* plan = nullptr;
    swe_params p{};
    int kind = 0, nnodes = 0;
    double tau[9]{}, Q[81]{}, QE[81]{}, QD[81]{};
};

// Small matrices passed by value to kernels.
struct NodeWeights {
    double q[9];      // dt * Q[m+1][j]
    double qe[9];     // dt * QE[m+1][j]
    double qd[9];     // dt * QD[m+1][j]
};
struct Mat9x9 {
    double a[81];
};
// A node update m >= 1 of an FP64 sweep formed in the staging of the next
// tendency's synthesis (that of Theta^{m+1}): the data of the separate
// update (k_sdc_node).
struct NodeFuse {
    int m = 0;                        // node whose new F is formed; Theta^{m+1} is computed
    double h = 0.0;                   // dt * QD[m+1][m+1]
    NodeWeights wt{};                 // row m+1 of dt Q, dt QE, dt QD
    swe_params p{};
    const double2* cout = nullptr;    // analyses of node m's tendency, [ext][5]
    double2* theta = nullptr;         // the sweep's nodes, [M+1][3][nspec]
    double2* fi = nullptr;            // new F_I at the nodes
    double2* fe = nullptr;            // new F_E at the nodes; node m+1 holds the old-F part S_m
    double2* rec = nullptr;           // tape of Theta^{m+1}, or null
};
// The weights of every node update of a sweep (row m = node m+1, M <= 8).
struct NodeRows {
    double q[8][9];   // dt * Q[m+1][j]
    double qe[8][9];  // dt * QE[m+1][j]
    double qd[8][9];  // dt * QD[m+1][j]
    double h[8];      // dt * QD[m+1][m+1]
};

// ----------------------------------------------------- launch wrappers
// legendre.hip
hipError_t launch_plm_table(const shx_plan* pl, hipStream_t st);
hipError_t launch_an_tab4(const shx_plan* pl, long long max_block, hipStream_t st);
hipError_t launch_an_polar(const shx_plan* pl, hipStream_t st);
// P^m_n at the northern latitudes by the double-double recurrence, rounded to
// FP64, into out[Jh] (device): the table export of plans without tables.
hipError_t launch_plm_one(const shx_plan* pl, int m, int n, double* out, hipStream_t st);
hipError_t launch_leg_syn(const shx_plan* pl, const double2* cin, double2* out, int F, int S,
                          int nmax_use, hipStream_t st);
// Synthesis of the tendency's four grid fields straight from S states
// [S][3][nspec]: swe_prep_row feeds the staging (any working precision).
hipError_t launch_leg_syn_swe(const shx_plan* pl, double a, const double2* state, double2* out, int S,
                              hipStream_t st);
// Synthesis of the five cotangent fields of the tendency adjoint straight
// from the F_E cotangents [S][3][nspec]: swe_combine_adj_row feeds the
// staging (FP64 plans).
hipError_t launch_leg_syn_swe_adj(const shx_plan* pl, double a, const double2* lfe, double2* out, int S,
                                  hipStream_t st);
hipError_t launch_leg_an(const shx_plan* pl, const double2* G, double2* cout, int F, int S,
                         int nmax_use, hipStream_t st);
// legendre_mixed.hip (plans with a reduced working precision)
hipError_t launch_leg_an_mixed(const shx_plan* pl, const double2* G, double2* cout, int F, int S, int nmax_use,
                               hipStream_t st);
hipError_t launch_leg_syn_mixed(const shx_plan* pl, const double2* cin, double2* out, int F, int S, int nmax_use,
                                hipStream_t st);
hipError_t launch_leg_syn_mixed_swe(const shx_plan* pl, double a, const double2* state, double2* out, int S,
                                    hipStream_t st);
hipError_t launch_tables_to_f32(const shx_plan* pl, hipStream_t st);
hipError_t launch_tables_to_bf16(const shx_plan* pl, const int* d_rows_an, const int* d_cols_an,
                                 const int* d_colsp_an, const int* d_rows_syn, const int* d_cols_syn,
                                 const int* d_colsp_syn, hipStream_t st);
// fourier.hip
// mode 0: the transforms; mode 1: their transposes' Fourier parts (inverse:
// grid scaled by w_j / nlon; forward: coefficient m scaled by c_m = 1, 2, 2, ...)
hipError_t launch_fft_inv(const shx_plan* pl, const double2* FI, double* grid, int F, int mode, hipStream_t st);
hipError_t launch_fft_fwd(const shx_plan* pl, const double* grid, double2* G, int F, int mode, hipStream_t st);
hipError_t launch_swe_grid(const shx_plan* pl, const double2* FI, double2* G, int S, double omega,
                           hipStream_t st);
bool fft_length_supported(int L);
// spectral.hip
// halve != 0 multiplies the coefficients of m >= 1 by 1/2 (analysis transpose)
hipError_t launch_spec_to_ext(const shx_plan* pl, const double2* spec, double2* cin, int F, int halve,
                              hipStream_t st);
hipError_t launch_ext_to_spec(const shx_plan* pl, const double2* cout, double2* spec, int F, hipStream_t st);
hipError_t launch_swe_combine(const shx_plan* pl, const swe_params& p, const double2* cout,
                              const double2* state, double2* fi, double2* fe, int S, hipStream_t st);
hipError_t launch_imex_solve(const shx_plan* pl, const swe_params& p, double h, const double2* rhs,
                             double2* out, int S, hipStream_t st);
// cout_m != nullptr (m >= 1): the new F at node m is formed from these
// analyses of node m's tendency inside the node update (and stored).
// rec != nullptr: Theta^{m+1} is also stored there (the adjoint's tape).
// The tendency synthesis with a sweep's node update formed in its staging
// (FP64 plans, and reduced-precision plans whose tendency synthesis
// regenerates P^m_n).
bool leg_syn_swe_node_supported(const shx_plan* pl);
bool leg_syn_mixed_swe_node_supported(const shx_plan* pl);
hipError_t launch_leg_syn_swe_node(const shx_plan* pl, const NodeFuse& nf, double2* out, hipStream_t st);
hipError_t launch_leg_syn_mixed_swe_node(const shx_plan* pl, const NodeFuse& nf, double2* out, hipStream_t st);
hipError_t launch_sdc_node_first(const shx_plan* pl, const swe_params& p, int M, const NodeRows& rows,
                                 double2* theta, const double2* fi_old, const double2* fe_old, const double2* cout_M,
                                 const double2* tau, double2* sq, double2* rec, hipStream_t st);
hipError_t launch_sdc_node(const shx_plan* pl, const swe_params& p, int m, int M, const NodeWeights& wts,
                           double h, double2* theta, double2* fi, double2* fe, const double2* cout_m,
                           double2* rec, hipStream_t st);
hipError_t launch_restrict(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pi, int nsrc,
                           int i0, int i1, const double2* src, double2* dst, double2* dst2, hipStream_t st);
// Copies of node 0 of up to 6 node arrays to node ranges of (other) node arrays.
struct NodeCopies {
    const double2* src[6];
    double2* dst[6];
    int first[6], last[6];
    int n = 0;
    void add(const double2* s, double2* d, int f, int l) {
        src[n] = s;
        dst[n] = d;
        first[n] = f;
        last[n] = l;
        ++n;
    }
};
hipError_t launch_node_copies(const NodeCopies& nc, long long n3, hipStream_t st);
hipError_t launch_fas_tau(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& PQ,
                          const Mat9x9& Qc, int nf, int nc, double dt, const double2* fi_f,
                          const double2* fe_f, const double2* fi_c, const double2* fe_c,
                          double2* tau, hipStream_t st);
hipError_t launch_interp(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pfc, int nf,
                         int nc, const double2* th_c, const double2* th_ct, const double2* fi_c,
                         const double2* fi_ct, const double2* fe_c, const double2* fe_ct,
                         double2* th_f, double2* fi_f, double2* fe_f, hipStream_t st);
hipError_t launch_residual(const shx_plan* pl, const Mat9x9& Q, int M, double dt, const double2* theta,
                           const double2* fi, const double2* fe, double* partial, int nblk,
                           hipStream_t st);
hipError_t launch_status(const shx_plan* pl, const double* partial, int nblk, int M,
                         const double2* theta_new, double* status, int residual_on, hipStream_t st);
int residual_blocks(const shx_plan* pl);
// adjoint.hip
bool adjoint_length_supported(int L);
// doubles of HBM grid workspace the tendency adjoint needs for S states (0
// when its rows fit in LDS)
size_t adj_grid_doubles(const shx_plan* pl, int S);
hipError_t launch_prep_adj(const shx_plan* pl, const swe_params& p, const double2* lam4, const double2* lfi,
                           double2* lstate, int S, int has_fe, hipStream_t st);
hipError_t launch_swe_grid_adj(const shx_plan* pl, const double2* FIs, const double2* FIl, double2* Ga, int S,
                               double omega, double* grid, hipStream_t st);
hipError_t launch_imex_solve_adj(const shx_plan* pl, const swe_params& p, double h, const double2* lx,
                                 double2* lb, int S, hipStream_t st);
hipError_t launch_sdc_node_adj(const shx_plan* pl, const swe_params& p, int m, int M, const NodeWeights& wt,
                               double h, double2* lth, double2* lfi_new, double2* lfe_new, double2* lfi_in,
                               double2* lfe_in, double2* ltau, hipStream_t st);
hipError_t launch_restrict_adj(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pi, int nsrc, int i0,
                               int i1, const double2* lc, double2* lf, hipStream_t st);
hipError_t launch_interp_adj(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& Pfc, int nf, int nc,
                             const double2* lthf, const double2* lfif, const double2* lfef, double2* lthc,
                             double2* lthct, double2* lfic, double2* lfict, double2* lfec, double2* lfect,
                             hipStream_t st);
hipError_t launch_fas_tau_adj(const shx_plan* fine, const shx_plan* coarse, const Mat9x9& PQ, const Mat9x9& Qc,
                              int nf, int nc, double dt, const double2* ltau, double2* lfif, double2* lfef,
                              double2* lfic, double2* lfec, hipStream_t st);
hipError_t launch_node_sum(const double2* x, double2* y, long long n3, int nn, int acc, hipStream_t st);
hipError_t launch_add(const double2* x, double2* y, long long n, hipStream_t st);
// Up to 8 arrays of the same length in one launch: y[i] = 0, or y[i] += x[i].
struct ArrayList {
    double2* y[8];
    const double2* x[8];
    int k;
    void add(double2* yi, const double2* xi = nullptr) { y[k] = yi; x[k] = xi; ++k; }
};
hipError_t launch_zero_n(const ArrayList& a, long long n, hipStream_t st);
hipError_t launch_add_n(const ArrayList& a, long long n, hipStream_t st);
