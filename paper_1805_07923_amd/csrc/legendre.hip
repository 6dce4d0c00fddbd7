// Legendre step of the SH transform pair (Sec. 3): per zonal order m, the
// contraction between the normalised P^m_n(mu_j) and the Fourier
// coefficients, eq. spectral_to_physical_space (synthesis) and eq.
// legendre_transform (analysis), FP64.
//
// Hemisphere symmetry: P^m_n(-mu) = (-1)^{n-m} P^m_n(mu), so each order m
// splits into an even (p = 0) and an odd (p = 1) block of degrees n = m+2k+p
// and only the nlat/2 northern latitudes are tabulated:
//   synthesis  E_m(mu_j) = sum_{p=0 rows} xi P,  O_m(mu_j) = sum_{p=1 rows} xi P,
//              north = E + O, south = E - O;
//   analysis   xi^m_n = sum_{j < J/2} P^m_n(mu_j) (g_north +/- g_south).
// The tables are built once per plan by a double-double recurrence (FP64
// operations) on the device, rounded to FP64, in two layouts:
// pan[m][p][jp][k] (lanes = degrees), streamed by the FP64 analysis, and
// psyn[m][p][k][jp], the source of the reduced-precision tables and of the
// table export.  The FP64 synthesis reads no table: it generates P^m_n with
// the recurrence on the fly from exact restart values and contracts on the
// matrix cores (k_leg_syn_m).  The second operand of the analysis (the
// Fourier coefficients of one latitude) is the same for every lane and is
// staged in LDS.
#include "internal.h"
#include "swe_node.h"

namespace {

// matrix-core synthesis with LS sets of 16 latitudes per wavefront: 4
// wavefronts per block for one set, 3 for two (96 latitudes per block)
__host__ __device__ constexpr int syn_wb(int LS) { return LS == 1 ? 4 : 3; }
__host__ __device__ constexpr int syn_lat(int LS) { return 16 * LS * syn_wb(LS); }
typedef double v4d __attribute__((ext_vector_type(4)));

// Value of lane src (wave-uniform) of a per-lane double, for every lane.
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Double-double arithmetic (an unevaluated sum hi + lo of two FP64 numbers,
// about 106 significant bits) from FP64 operations: error-free sum (Knuth)
// and product (FMA), division and square root by one correction step each.
// The error-free transformations need every product and sum rounded on its
// own, so floating-point contraction is switched off in this part of the
// file (the backend would otherwise fuse a product into a later sum).
#pragma clang fp contract(off)
struct dd {
    double h, l;
};
__device__ __forceinline__ dd dd_norm(double a, double b) {    // |a| >= |b|
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_sub(dd a, dd b) {
    const double s = a.h - b.h;
    const double bb = s - a.h;
    const double e = (a.h - (s - bb)) + (-b.h - bb);
    return dd_norm(s, e + (a.l - b.l));
}
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    const double p = a.h * b.h;
    double e = fma(a.h, b.h, -p);
    e = fma(a.h, b.l, e);
    e = fma(a.l, b.h, e);
    return dd_norm(p, e);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
    const double p = a.h * b;
    double e = fma(a.h, b, -p);
    e = fma(a.l, b, e);
    return dd_norm(p, e);
}
__device__ __forceinline__ dd dd_div(dd a, dd b) {
    const double q1 = a.h / b.h;
    const dd r = dd_sub(a, dd_mul_d(b, q1));
    const double q2 = r.h / b.h;
    const dd r2 = dd_sub(r, dd_mul_d(b, q2));
    const double q3 = r2.h / b.h;
    const dd q = dd_norm(q1, q2);
    return dd_norm(q.h, q.l + q3);
}
__device__ __forceinline__ dd dd_sqrt(dd a) {                  // a > 0
    const double x = sqrt(a.h);
    const double p = x * x;
    const double e = fma(x, x, -p);
    const dd r = dd_sub(a, dd{p, e});
    return dd_norm(x, r.h / (2.0 * x));
}
// eps^m_n = sqrt((n^2 - m^2) / (4 n^2 - 1)) in double-double (n > m).
__device__ __forceinline__ dd dd_eps(int n, int m) {
    return dd_sqrt(dd_div(dd{(double)n * n - (double)m * m, 0.0}, dd{4.0 * n * n - 1.0, 0.0}));
}

// P^m_n(mu_j) for one (m, jp) by the standard recurrence of the orthonormal
// functions: P^0_0 = 1/sqrt(2); P^m_m = sqrt((2m+1)/(2m)) sin(theta) P^{m-1}_{m-1};
// P^m_{m+1} = sqrt(2m+3) mu P^m_m; eps^m_n P^m_n = mu P^m_{n-1} - eps^m_{n-1} P^m_{n-2}.
// The recurrence runs in double-double from the FP64 mu and sin(theta) and
// each value is rounded to FP64: in plain FP64 the forward recurrence
// amplifies rounding errors roughly like n^2 near the poles (about 1e-12 of
// the column maximum at degree 1000), which the Laplacian's n(n+1) turns
// into visible errors of the divergence tendency at T1023.  Besides the two
// tables the kernel stores the restart values of the FP64 kernels that
// generate P^m_n themselves (at the start of every seg_len segment, so that
// their plain FP64 recurrence never runs more than 64 steps from an exact
// value) and
// the recurrence coefficients 1/eps^m_n and eps^m_{n-1}/eps^m_n; and, for the
// analysis' form of the recurrence, Q_n = mu Q_{n-1} - (eps^m_{n-1})^2 Q_{n-2}
// with P^m_n = C_n Q_n, the coefficients (eps^m_{n-1})^2 and the factors C_n
// of each restart segment (C = 1 at its first degree, C_n = C_{n-1} / eps^m_n).
__global__ void k_plm_table(const double* __restrict__ mu, const double* __restrict__ sint,
                            const long long* __restrict__ off, double* __restrict__ psyn,
                            double* __restrict__ pan, double2* __restrict__ ck,
                            const long long* __restrict__ ckoff, double2* __restrict__ rc,
                            double* __restrict__ rq, double* __restrict__ cs, int N, int nmax,
                            int Jh) {
    const int jp = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (jp >= Jh) return;
    const double x = mu[jp], s = sint[jp];
    dd pmm = dd_sqrt(dd{0.5, 0.0});
    for (int k = 1; k <= m; ++k)
        pmm = dd_mul_d(dd_mul(pmm, dd_sqrt(dd_div(dd{2.0 * k + 1.0, 0.0}, dd{2.0 * k, 0.0}))), s);
    const int K0 = kcount(nmax, m, 0), K1 = kcount(nmax, m, 1);
    double* ps0 = psyn + off[2 * m];
    double* ps1 = psyn + off[2 * m + 1];
    double* pa0 = pan + off[2 * m];
    double* pa1 = pan + off[2 * m + 1];
    dd p2{0.0, 0.0}, p1 = pmm;   // P_{n-2}, P_{n-1}
    dd e_prev = (m + 1 <= nmax) ? dd_eps(m + 1, m) : dd{1.0, 0.0};
    double2* ckm = ck + ckoff[m] + jp;
    const int L = seg_len(nmax - m + 1);
    double2* rcm = rc + ext_idx(N, m, m);
    double* rqm = rq + ext_idx(N, m, m);
    double* csm = cs + ext_idx(N, m, m);
    dd cn{1.0, 0.0};                                    // C_n of the current segment
    for (int n = m; n <= nmax; ++n) {
        dd pn;
        double2 r = make_double2(0.0, 0.0);
        double b = 0.0;
        if (n == m) {
            pn = pmm;
        } else if (n == m + 1) {
            pn = dd_mul_d(dd_mul(dd_sqrt(dd{2.0 * m + 3.0, 0.0}), pmm), x);
        } else {
            const dd en = dd_eps(n, m);
            pn = dd_div(dd_sub(dd_mul_d(p1, x), dd_mul(e_prev, p2)), en);
            const dd ra = dd_div(dd{1.0, 0.0}, en), rb = dd_div(e_prev, en), e2 = dd_mul(e_prev, e_prev);
            r = make_double2(ra.h + ra.l, rb.h + rb.l);
            b = e2.h + e2.l;
            e_prev = en;
        }
        if ((n - m) % L == 0) cn = dd{1.0, 0.0};
        else cn = dd_div(cn, dd_eps(n, m));
        if (jp == 0) {
            rcm[n - m] = r;
            rqm[n - m] = b;
            csm[n - m] = cn.h + cn.l;
        }
        if (n > m) { p2 = p1; p1 = pn; }
        const double v = pn.h + pn.l;
        const int g = (n - m) / L, gr = (n - m) - g * L;
        if (gr == 0) ckm[(long long)g * Jh] = make_double2(v, 0.0);
        if (gr == 1) ckm[(long long)g * Jh].y = v;
        if (!psyn) continue;                            // plan without tables: restart data only
        const int p = (n - m) & 1, k = (n - m) >> 1;
        if (p == 0) {
            ps0[(long long)k * Jh + jp] = v;
            pa0[(long long)jp * K0 + k] = v;
        } else {
            ps1[(long long)k * Jh + jp] = v;
            pa1[(long long)jp * K1 + k] = v;
        }
    }
}

// One row P^m_n(mu_jp), jp < Jh, by the same double-double recurrence.
__global__ void k_plm_one(const double* __restrict__ mu, const double* __restrict__ sint, int m, int n, int Jh,
                          double* __restrict__ out) {
    const int jp = blockIdx.x * blockDim.x + threadIdx.x;
    if (jp >= Jh) return;
    const double x = mu[jp], s = sint[jp];
    dd pmm = dd_sqrt(dd{0.5, 0.0});
    for (int k = 1; k <= m; ++k)
        pmm = dd_mul_d(dd_mul(pmm, dd_sqrt(dd_div(dd{2.0 * k + 1.0, 0.0}, dd{2.0 * k, 0.0}))), s);
    dd p2{0.0, 0.0}, p1 = pmm, pn = pmm;
    if (n > m) {
        pn = dd_mul_d(dd_mul(dd_sqrt(dd{2.0 * m + 3.0, 0.0}), pmm), x);
        p2 = pmm;
        p1 = pn;
    }
    dd e_prev = dd_eps(m + 1, m);
    for (int k = m + 2; k <= n; ++k) {
        const dd en = dd_eps(k, m);
        pn = dd_div(dd_sub(dd_mul_d(p1, x), dd_mul(e_prev, p2)), en);
        e_prev = en;
        p2 = p1;
        p1 = pn;
    }
    out[jp] = pn.h + pn.l;
}
#pragma clang fp contract(fast)

// Synthesis on the matrix cores with P^m_n generated in registers instead of
// read from the table: out[s][p][jp][m][f0+f] = sum_{n = m+p mod 2} P^m_n(mu_jp) cin[s][ext(m, n)][f0+f].
// gx (N+1) blocks (gx = ceil(Jh/64), all blocks of an order on one XCD),
// 256 threads, one wavefront per 16 latitudes.  Per order the sum over n is
// a (16 latitudes) x (n) x (2 NF real columns) product, done by the
// four-block v_mfma_f64_4x4x4f64 (block b: latitudes 4b..4b+3, one group of
// four real columns; ceil(NF/2) instructions per degree, so that a product
// of fewer than 8 fields keeps no idle columns, as a 16-column tile would)
// with the 4-deep inner dimension taken by four
// degree segments: lane (i, q) = (lane % 16, lane / 16) owns latitude i and
// segment q of the current round, starts from the stored exact pair
// (P_{m+gL}, P_{m+gL+1}) and advances two degrees per step with the
// three-term recurrence of the orthonormal functions (Sec. 3),
// P_n = (mu P_{n-1} - eps_{n-1} P_{n-2}) / eps_n, in FP64.  Each step feeds
// one even-degree and one odd-degree product (E and O accumulators, the two
// hemisphere halves); the B operand is the lane's coefficient row of that
// degree, column 4 g + lane % 4 for column group g.  STAGE = 0: cin holds coefficients in the ext
// layout, F per entry; STAGE = 1: cin holds states [S][3][nspec] and the
// staged rows are the tendency's grid fields (swe_prep_row; NF = F = 4);
// STAGE = 2: cin holds F_E cotangents [S][3][nspec] and the staged rows are
// the cotangents of the five weighted analyses (swe_combine_adj_row;
// NF = F = 5); STAGE = 3: as STAGE 1 for the state that a sweep's node
// update produces, formed by each block for its order in LDS first (nfu).  The coefficient rows and the recurrence coefficients of the
// round's 4 L degrees are staged in LDS, segment by segment, each segment
// padded by 32 bytes so that the four segments' reads of one step fall on
// different banks; rows past nmax_use are staged as zeros and recurrence
// coefficients past the table as zeros (P then continues as 0), so every
// lane reads its next eight degrees at fixed offsets from one address, with
// no clamping and no per-degree selection.
template <int NF, int STAGE = 0, int SYN_LS = 1>
__global__ __launch_bounds__(64 * syn_wb(SYN_LS)) void k_leg_syn_m(const double2* __restrict__ ck,
                                                   const long long* __restrict__ ckoff,
                                                   const double* __restrict__ rq,
                                                   const double* __restrict__ cs,
                                                   const double* __restrict__ mu,
                                                   const double2* __restrict__ cin,
                                                   double2* __restrict__ out, int N, int nmax_tab,
                                                   int nmax_use, int Jh, int F, int f0, int S,
                                                   long long cin_stride, long long out_stride, int gx,
                                                   long long nspec, double a, int Lmax,
                                                   const double2* __restrict__ pf,
                                                   const double* __restrict__ ninv,
                                                   const double* __restrict__ nn1, NodeFuse nfu) {
    static_assert(NF >= 1 && NF <= 8, "16 real columns per product");
    constexpr int U = 8;                                // degrees per batch of LDS reads
    constexpr int NG = (2 * NF + 3) / 4;                // groups of 4 real columns
    extern __shared__ double2 csh[];                    // [4][L NF + 2] rows, then [4][L + 2] coefficients
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, q = lane >> 4;
    const LegTile tile = leg_tile(gx, N + 1, 1);
    const int m = tile.m;
    const int jw = tile.x * syn_lat(SYN_LS) + wv * 16 * SYN_LS;  // first latitude of this wavefront
    const int Kt = nmax_tab - m + 1, Ku = nmax_use - m + 1;
    const int R = seg_rounds(Kt), L = seg_len(Kt);
    const int SC = L * NF + 2, SR = L + 2;              // padded segment strides (double2)
    double x[SYN_LS];                                   // latitude set ls: jw + 16 ls + i
    const double2* ckm[SYN_LS];
#pragma unroll
    for (int ls = 0; ls < SYN_LS; ++ls) {
        const int jp = jw + 16 * ls + i;
        const bool active = jp < Jh;
        x[ls] = mu[active ? jp : 0];
        ckm[ls] = ck + ckoff[m] + (active ? jp : 0);
    }
    double* rsh = reinterpret_cast<double*>(csh + 4 * (Lmax * NF + 2));
    const double* cq = reinterpret_cast<const double*>(csh + q * SC);        // segment q
    int cg[NG];                                         // B columns 4 g + lane % 4 (clamped; >= 2 NF unused)
#pragma unroll
    for (int g = 0; g < NG; ++g) cg[g] = min(4 * g + (lane & 3), 2 * NF - 1);
    const double* rqs = rsh + q * SR;
    const double* rqm = rq + ext_idx(N, m, m);
    const double* csm = cs + ext_idx(N, m, m);
    const double2* pfm = pf + ext_idx(N, m, m);
    const double ia = 1.0 / a, a2 = a * a, ia2 = ia * ia;
    // STAGE 3: the sweep's node update of order m (S = 1), Theta^{k+1} =
    // solve(S_k + sum_{j<=k} [dtQE F_E^j + dtQD F_I^j], h) with F at node k =
    // nfu.m formed from its analyses, into LDS thn [3][N+1] (degrees m..N);
    // the block of the first latitude group also stores Theta^{k+1} and the
    // F of node k (the sweep's outputs) and the tape
    double2* thn = csh + 4 * (Lmax * (NF + 1) + 4);
    double2 c0first[SYN_LS];                            // round 0's restart pairs, loaded before the update
    if constexpr (STAGE == 3) {
#pragma unroll
        for (int ls = 0; ls < SYN_LS; ++ls) c0first[ls] = ckm[ls][(long long)q * Jh];
    }
    if constexpr (STAGE == 3) {
        static_assert(STAGE != 3 || NF == 4, "the tendency synthesis has four fields");
        // the staging below reads thn after its first barrier
        swe_node::node_update_order(nfu, N, nspec, m, tile.x == 0, thn, threadIdx.x, 64 * syn_wb(SYN_LS));
    }
    for (int s = 0; s < S; ++s) {
        double accE[SYN_LS][NG], accO[SYN_LS][NG];
#pragma unroll
        for (int ls = 0; ls < SYN_LS; ++ls)
#pragma unroll
            for (int g = 0; g < NG; ++g) accE[ls][g] = accO[ls][g] = 0.0;
        for (int r = 0; r < R; ++r) {
            const int kr0 = 4 * r * L;
            if (kr0 >= Ku) break;                       // uniform
            const int g = 4 * r + q;
            double2 c0[SYN_LS];                         // in flight during the staging
#pragma unroll
            for (int ls = 0; ls < SYN_LS; ++ls)
                c0[ls] = (STAGE == 3 && r == 0) ? c0first[ls] : ckm[ls][(long long)g * Jh];
            const double qinv = (g * L + 1 < Kt) ? 1.0 / csm[g * L + 1] : 0.0;   // Q_{gL+1} = P_{gL+1} / C
            __syncthreads();                            // previous readers of the rows are done
            for (int kl = threadIdx.x; kl < 4 * L; kl += 64 * syn_wb(SYN_LS)) {
                const int qs = kl / L, ts = kl - qs * L, kk = kr0 + kl;
                double2* row = csh + qs * SC + ts * NF;
                if (kk < Ku) {
                    if constexpr (STAGE == 3) {
                        double2 o[4];
                        swe_prep_row_t([&](int f, int nn) { return thn[f * (N + 1) + (nn - m)]; }, N, a2, ia, pfm,
                                       ninv, m, m + kk, o);
                        const double c = csm[kk];
#pragma unroll
                        for (int f = 0; f < 4; ++f) row[f] = make_double2(c * o[f].x, c * o[f].y);
                    } else if constexpr (STAGE == 1) {
                        static_assert(STAGE != 1 || NF == 4, "the tendency synthesis has four fields");
                        double2 o[4];
                        swe_prep_row(cin + s * cin_stride, nspec, N, a2, ia, pfm, ninv, m, m + kk, o);
                        const double c = csm[kk];
#pragma unroll
                        for (int f = 0; f < 4; ++f) row[f] = make_double2(c * o[f].x, c * o[f].y);
                    } else if constexpr (STAGE == 2) {
                        static_assert(STAGE != 2 || NF == 5, "the tendency adjoint synthesises five fields");
                        double2 o[5];
                        swe_combine_adj_row(cin + s * cin_stride, nspec, N, ia, ia2, pfm, nn1, m, m + kk, o);
                        const double c = csm[kk];
#pragma unroll
                        for (int f = 0; f < 5; ++f) row[f] = make_double2(c * o[f].x, c * o[f].y);
                    } else {
                        const double2* cg = cin + s * cin_stride + (ext_idx(N, m, m) + kk) * F + f0;
                        const double c = csm[kk];
#pragma unroll
                        for (int f = 0; f < NF; ++f) row[f] = make_double2(c * cg[f].x, c * cg[f].y);
                    }
                } else {
#pragma unroll
                    for (int f = 0; f < NF; ++f) row[f] = make_double2(0.0, 0.0);
                }
                rsh[qs * SR + ts] = (kk < Kt) ? rqm[kk] : 0.0;
            }
            __syncthreads();
            if (jw >= Jh) continue;                     // uniform: no latitudes for this wavefront
            double pe[SYN_LS], po[SYN_LS];              // P_{m+gL}, P_{m+gL+1}
#pragma unroll
            for (int ls = 0; ls < SYN_LS; ++ls) {
                pe[ls] = c0[ls].x;
                po[ls] = c0[ls].y * qinv;
            }
            for (int t = 0; t < L; t += U) {
                double rr[U];
                double bb[U][NG];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    rr[u] = rqs[t + u];
#pragma unroll
                    for (int g = 0; g < NG; ++g) bb[u][g] = cq[(t + u) * 2 * NF + cg[g]];
                }
#pragma unroll
                for (int u = 0; u < U; u += 2) {
#pragma unroll
                    for (int ls = 0; ls < SYN_LS; ++ls) {
                        if (u > 0 || t > 0) {
                            const double ne = fma(x[ls], po[ls], -(rr[u] * pe[ls]));
                            po[ls] = fma(x[ls], ne, -(rr[u + 1] * po[ls]));
                            pe[ls] = ne;
                        }
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            accE[ls][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(pe[ls], bb[u][g], accE[ls][g], 0, 0, 0);
                            accO[ls][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(po[ls], bb[u + 1][g], accO[ls][g], 0, 0, 0);
                        }
                    }
                }
            }
        }
        // D layout (f64 4x4x4, 4 blocks): lane 4 b + j + 16 r holds row r of
        // block b (latitude 4 b + r) and column j of the group
#pragma unroll
        for (int ls = 0; ls < SYN_LS; ++ls) {
            const int jr = jw + 16 * ls + 4 * (i >> 2) + q;
            if (jw < Jh && jr < Jh) {
                double* o0 = reinterpret_cast<double*>(out + s * out_stride + ((long long)jr * (N + 1) + m) * F + f0);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const int c = 4 * g + (lane & 3);
                    if (c < 2 * NF) {
                        o0[c] = accE[ls][g];
                        o0[c + (long long)Jh * (N + 1) * F * 2] = accO[ls][g];
                    }
                }
            }
        }
    }
}

// Analysis on the matrix cores with P^m_n generated in registers instead of
// read from the table:
// cout[s][ext(m, n)][f0+f] = sum_jp P^m_n(mu_jp) (G[s][jp][m][f0+f] + (-1)^{n-m} G[s][J-1-jp][m][f0+f]).
// One block of nw = min(4, ceil(Jh/64)) wavefronts (64 nw threads) per (order m, restart
// segment g) of the synthesis segmentation (degrees m + gL .. m + gL + L - 1,
// L <= 64), listed XCD by XCD in blist so that all blocks of an order share
// one L2.  Wavefront w takes the latitude groups w, w + nw, ... of 64
// latitudes; for each, lane = latitude runs the three-term recurrence of the
// orthonormal functions (Sec. 3) from the stored exact pair (P_{m+gL},
// P_{m+gL+1}) in FP64 and stores the P of 32 degrees in a wave-private LDS
// tile, split by parity ([latitude][16] for even and for odd degrees,
// rows padded to 17 so that both the stores and the operand reads are
// free of bank conflicts).  v_mfma_f64_16x16x4f64 then contracts 16 degrees
// of one parity x 4 latitudes x 16 real columns; the B operand, the
// north +/- south combination of the Fourier coefficients, is read by each
// lane straight from G (column lane % 16 of latitude 4 c + lane / 16).  The
// recurrence coefficients of the segment's degrees are loaded one per lane
// and broadcast with readlane (a scalar load per degree would make every
// step wait on the counter it shares with the LDS stores).  The partial sums
// of the latitude groups are added through LDS in wavefront order.
template <int NF>
__global__ __launch_bounds__(256) void k_leg_an_m(const int* __restrict__ blist,
                                                  const double2* __restrict__ ck,
                                                  const long long* __restrict__ ckoff,
                                                  const double* __restrict__ rq,
                                                  const double* __restrict__ cs,
                                                  const double* __restrict__ mu,
                                                  const double2* __restrict__ G,
                                                  double2* __restrict__ cout, int N, int nmax_tab,
                                                  int nmax_use, int J, int F, int f0, int S,
                                                  long long G_stride, long long cout_stride, int nw) {
    static_assert(NF >= 1 && NF <= 8, "16 real columns per product");
    constexpr int TP = 17;                              // padded tile row
    extern __shared__ double lsh[];                     // [nw][2][64][TP]; then the partial sums
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, q = lane >> 4;
    const int m = blist[2 * blockIdx.x], g = blist[2 * blockIdx.x + 1];
    if (m < 0) return;                                  // padding block (uniform)
    const int Jh = J / 2;
    const int Kt = nmax_tab - m + 1, Ku = nmax_use - m + 1;
    const int L = seg_len(Kt);
    const int k0 = g * L;
    if (k0 >= Ku) return;                               // uniform
    const int kend = min(k0 + L, Ku);                   // degrees k0 .. kend-1 are this block's
    const int ntp = (kend - k0 + 31) / 32;              // 32-degree tile pairs (1 or 2)
    const int ngrp = (Jh + 63) / 64;
    double* PE = lsh + wv * (2 * 64 * TP);
    double* PO = PE + 64 * TP;
    double* red = lsh;                                  // [nw][2 tile pairs][2 parities][4][64] afterwards
    const double* rqm = rq + ext_idx(N, m, m);
    const double* csm = cs + ext_idx(N, m, m);
    const long long rs = (long long)(N + 1) * F * 2;    // latitude row stride of G in doubles
    // Q_{k0+1} = P_{k0+1} / C_{k0+1} (the segment's second restart value)
    const double qs = (k0 + 1 < Kt) ? 1.0 / csm[k0 + 1] : 0.0;
    const int jc = i < 2 * NF ? i : 2 * NF - 1;         // B column (clamped; columns >= 2 NF unused)
    for (int s = 0; s < S; ++s) {
        v4d acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = v4d{0.0, 0.0, 0.0, 0.0};
        const double* gs = reinterpret_cast<const double*>(G + s * G_stride + (long long)m * F + f0) + jc;
        for (int lg = wv; lg < ngrp; lg += nw) {
            const int jp = lg * 64 + lane;
            const bool act = jp < Jh;
            const double x = mu[act ? jp : 0];
            const double2 c0 = act ? ck[ckoff[m] + (long long)g * Jh + jp] : make_double2(0.0, 0.0);
            double be[16], bo[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int jb = lg * 64 + 4 * c + q;
                const bool ab = jb < Jh;
                const int jr = ab ? jb : 0;
                const double vn = gs[jr * rs], vs = gs[(J - 1 - jr) * rs];
                be[c] = ab ? vn + vs : 0.0;
                bo[c] = ab ? vn - vs : 0.0;
            }
            double pe = c0.x, po = c0.y * qs;           // Q_{m+k0} = P_{m+k0}, Q_{m+k0+1}
            // recurrence coefficients of the 64 degrees: lane t holds degree k0 + t
            const double rbv = rqm[min(k0 + lane, Kt - 1)];
            for (int tp = 0; tp < ntp; ++tp) {
#pragma unroll
                for (int i2 = 0; i2 < 16; ++i2) {
                    if (tp > 0 || i2 > 0) {
                        const int t = 32 * tp + 2 * i2;     // wave-uniform lane of the degree
                        const double b0 = lane_bcast(rbv, t), b1 = lane_bcast(rbv, t + 1);
                        const double ne = fma(x, po, -(b0 * pe));
                        po = fma(x, ne, -(b1 * po));
                        pe = ne;
                    }
                    PE[lane * TP + i2] = pe;
                    PO[lane * TP + i2] = po;
                }
                // same-wavefront LDS accesses complete in order: the tile is
                // complete for the reads below
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    const double ae = PE[(4 * c + q) * TP + i];
                    const double ao = PO[(4 * c + q) * TP + i];
                    if (tp == 0) {
                        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, be[c], acc[0][0], 0, 0, 0);
                        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao, bo[c], acc[0][1], 0, 0, 0);
                    } else {
                        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, be[c], acc[1][0], 0, 0, 0);
                        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao, bo[c], acc[1][1], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();                                // all tile reads done
        {
            for (int tp = 0; tp < ntp; ++tp)
#pragma unroll
                for (int eo = 0; eo < 2; ++eo)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
                        red[(((wv * 2 + tp) * 2 + eo) * 4 + rr) * 64 + lane] = acc[tp][eo][rr];
        }
        __syncthreads();
        // wavefront w writes the tiles (tp, eo) = (u / 2, u % 2), u = w, w + nw, ...;
        // D layout (f64 16x16x4): the lane holds rows q + 4 rr (degree pairs) of column i
        for (int u = wv; u < 2 * ntp && i < 2 * NF; u += nw) {
            const int tp = u >> 1, eo = u & 1;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int k = k0 + 32 * tp + 2 * (q + 4 * rr) + eo;
                if (k < kend) {
                    double v = 0.0;
                    for (int w = 0; w < nw; ++w) v += red[(((w * 2 + tp) * 2 + eo) * 4 + rr) * 64 + lane];
                    reinterpret_cast<double*>(cout + s * cout_stride + ext_idx(N, m, m + k) * F + f0)[i] =
                        csm[k] * v;
                }
            }
        }
        __syncthreads();                                // before the next state's tiles
    }
}

// pan4 (FP64) or pan4f (FP32, rounded) from pan (layout in shx_plan): one
// thread per element of the block's tiles counted as whole (order-parity
// block blockIdx.y = 2 m + p); the rows past the last degree are not stored.
template <class T>
__global__ void k_an_tab4(const double* __restrict__ pan, const long long* __restrict__ off,
                          const long long* __restrict__ off4, T* __restrict__ pan4, int nmax, int Jh) {
    const int mp = blockIdx.y, m = mp >> 1, p = mp & 1;
    const int K = kcount(nmax, m, p);
    const int ngrp = (Jh + 3) / 4;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (K <= 0 || e >= (long long)((K + 15) / 16) * ngrp * 64) return;
    const long long blk = e / 64;
    const int l = (int)(e - blk * 64);
    const int kt = (int)(blk / ngrp), c = (int)(blk - (long long)kt * ngrp);
    const int i = l & 15, kq = l >> 4;
    const int r = K - 16 * kt < 16 ? K - 16 * kt : 16;  // rows of tile kt
    if (i >= r) return;
    const int k = 16 * kt + i, jp = 4 * c + kq;
    pan4[off4[mp] + (long long)kt * ngrp * 64 + (long long)(4 * c + kq) * r + i] =
        (T)(jp < Jh ? pan[off[mp] + (long long)jp * K + k] : 0.0);
}

// First summed latitude group of each 16-degree tile of pan4 (an_c0 in
// shx_plan): one wavefront per (tile kt, order-parity block blockIdx.y)
// scans the groups from the pole and stops at the first with a value of
// magnitude >= tau.
template <class T>
__global__ __launch_bounds__(64) void k_an_polar(const T* __restrict__ pan4,
                                                 const long long* __restrict__ off4, int* __restrict__ c0,
                                                 int nmax, int Jh, int kt_all, double tau) {
    const int mp = blockIdx.y, kt = blockIdx.x, lane = threadIdx.x;
    const int ngrp = (Jh + 3) / 4;
    const int K = kcount(nmax, mp >> 1, mp & 1);
    int c = ngrp;
    if (16 * kt < K) {
        const int r = K - 16 * kt < 16 ? K - 16 * kt : 16, i = lane & 15;
        const bool on = i < r;                          // lanes of stored rows
        const T* t = pan4 + off4[mp] + (long long)kt * ngrp * 64 + (lane >> 4) * r + (on ? i : 0);
        for (c = 0; c < ngrp; ++c)
            if (__ballot(on && fabs((double)t[(long long)c * 4 * r]) >= tau) != 0) break;
    }
    if (lane == 0) c0[mp * kt_all + kt] = c;
}

// Analysis from the table on the matrix cores (plans with up to AN_TAB_JH
// latitude pairs, 1-16 fields per launch; beyond, k_leg_an_m generates P^m_n
// instead):
// cout[s][ext(m, m+2k+p)][f0+f] = sum_jp P[m][p][jp][k] (G[s][jp][m] + (-1)^p G[s][J-1-jp][m]).
// One block per (m, p, 64-degree tile holding rows) from the plan's list
// (the blocks of an order on one XCD), one wavefront per 16 degrees summing
// over all latitude pairs, so no partial sums cross wavefronts.  Per group
// of 4 latitude pairs the four-block v_mfma_f64_4x4x4f64 takes A = 16
// degrees x 4 latitude pairs of the table, 64 consecutive values of pan4 (one
// 8-byte load per lane; 4 x the rows of the block's last tile there), and B = the north +/- south Fourier data of the
// same latitude pairs staged in LDS (column 4 g + lane % 4): one instruction
// per pair of fields; D lane 4 b + j + 16 i holds degree row 4 b + i,
// column 4 g + j.  With an odd field count the last field's two columns are
// summed on the VALU by each lane over its latitude slot (lane / 16) and the
// four slots added by lane exchange, instead of a third, half-empty matrix
// product per group.  Each wavefront starts at its tile's first summed group
// (polar truncation, AN_POLAR_TAU; the run is whole batches of UNR =
// an_batch(Jh) loads), and the block stages the Fourier data from the
// smallest first group of its tiles on.  SPLIT = 2 (below 160 latitude
// pairs, where one wavefront per tile leaves about one wavefront per SIMD)
// gives each tile two wavefronts of 512-thread blocks, each summing half of
// the tile's batches; the second hands its partial sums to the first through
// LDS (measured at T127: 8.1-8.4 against 9.3 us; at T255 19.7 against 17.3).
template <int NF, int UNR, int SPLIT>
__global__ __launch_bounds__(256 * SPLIT) void k_leg_an(const int4* __restrict__ tblk, const double* __restrict__ pan4,
                                                          const long long* __restrict__ off4,
                                                          const double2* __restrict__ G,
                                                          double2* __restrict__ cout, int N, int nmax_tab,
                                                          int nmax_use, int J, int F, int f0, int S,
                                                          long long G_stride, long long cout_stride) {
    static_assert(SPLIT == 1 || SPLIT == 2, "one or two wavefronts per tile");
    constexpr int NG = NF / 2;                          // groups of 4 real columns (two fields) on MFMA
    constexpr bool ODD = NF % 2 == 1;                   // last field: its two columns on the VALU
    constexpr int NR = NG + (ODD ? 2 : 0);              // partial sums per lane handed between halves
    extern __shared__ double2 gsh[];                    // [4 ngrp][NF], then (SPLIT 2) [4][NR][64] doubles
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tw = wv & 3, half = wv >> 2;              // tile of the block, latitude half (SPLIT 2)
    const int4 tb = tblk[blockIdx.x];                   // (2m+p, tile, first groups, their minimum)
    const int mp = tb.x, tx = tb.y;
    if (mp < 0) return;                                 // padding block (uniform)
    const int m = mp >> 1, p = mp & 1;
    const int K = kcount(nmax_use, m, p);
    if (tx * 64 >= K) return;                           // whole block idle (uniform)
    const int Jh = J / 2;
    const int k0 = tx * 64 + 16 * tw;                   // this wavefront's first degree row
    const bool rows = k0 < K;                           // wave-uniform
    const int kq = lane >> 4;                           // latitude slot of the operands
    const int ngrp = (Jh + 3) / 4;                      // groups of 4 latitude pairs
    // A operands of this wavefront's degrees: 4 r consecutive values per
    // group, r = the tile's stored rows (16 but in the block's last tile);
    // lanes of the missing rows read row 0 again, and their output rows are
    // not stored
    const int Kt = kcount(nmax_tab, m, p);
    const int r = __builtin_amdgcn_readfirstlane(Kt - k0 < 16 ? (Kt - k0 > 0 ? Kt - k0 : 1) : 16);
    const int os = 4 * r;                               // operand stride
    const double* P = pan4 + off4[2 * m + p] + (long long)(k0 >> 4) * ngrp * 64 + kq * r +
                      ((lane & 15) < r ? (lane & 15) : 0);
    const int cb0 = tb.w;                               // first staged latitude group
    // the tile's first summed group (wave-uniform: kept in a scalar register
    // so that the group loop and its addresses stay scalar)
    const int cw0 = __builtin_amdgcn_readfirstlane(rows ? (tb.z >> (8 * tw)) & 255 : ngrp);
    const double sg = p ? -1.0 : 1.0;
    const long long rowstride = (long long)(N + 1) * F;
    const double* gs = reinterpret_cast<const double*>(gsh);
    const int cb = lane & 3;                            // B column within a group
    // the tile sums groups cw0 .. ngrp-1 (a multiple of UNR where ngrp
    // allows); with SPLIT 2 the first half of its batches goes to the
    // wavefront of half 0, the rest to half 1
    const int nrun = ngrp - cw0;
    int cbeg = 0, cend = nrun;
    if constexpr (SPLIT == 2) {
        const int b0 = (nrun / UNR + 1) / 2;
        if (half == 0) cend = b0 * UNR; else cbeg = b0 * UNR;
    }
    const double* Pw = P + (long long)(cw0 + cbeg) * os;
    const int nmine = cend - cbeg, jw = 4 * (cw0 + cbeg) + kq;
    // the first batch of table values is loaded before the Fourier data are
    // staged, so that the two memory round trips overlap; the table is the
    // same for every state
    const bool pre = rows && nmine >= UNR;              // wave-uniform
    double pv0[UNR];
    if (pre) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) pv0[u] = Pw[u * os];
    }
    double* red = reinterpret_cast<double*>(gsh + (size_t)4 * ngrp * NF) + (size_t)tw * NR * 64 + lane;
    for (int s = 0; s < S; ++s) {
        const double2* g = G + s * G_stride + (long long)m * F + f0;
        __syncthreads();                                // previous state's readers are done
        // rows of whole latitude groups: zeros past the last pair, so that
        // the products read their operands without a bounds test
        for (int i = 4 * cb0 * NF + threadIdx.x; i < 4 * ngrp * NF; i += 256 * SPLIT) {
            const int jp = i / NF, f = i - jp * NF;
            double2 v = make_double2(0.0, 0.0);
            if (jp < Jh) {
                const double2 a = g[jp * rowstride + f], b = g[(J - 1 - jp) * rowstride + f];
                v = make_double2(a.x + sg * b.x, a.y + sg * b.y);
            }
            gsh[i] = v;
        }
        __syncthreads();
        double acc[NG > 0 ? NG : 1];
#pragma unroll
        for (int g2 = 0; g2 < NG; ++g2) acc[g2] = 0.0;
        double vr = 0.0, vi = 0.0;                      // odd field: this lane's latitude slot
        auto step = [&](double a, int jp) {
#pragma unroll
            for (int g2 = 0; g2 < NG; ++g2) {
                const double b = gs[jp * 2 * NF + 4 * g2 + cb];
                acc[g2] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[g2], 0, 0, 0);
            }
            if constexpr (ODD) {
                const double2 z = gsh[jp * NF + NF - 1];
                vr = fma(a, z.x, vr);
                vi = fma(a, z.y, vi);
            }
        };
        if (rows) {
            int c = 0;
            if (pre) {
#pragma unroll
                for (int u = 0; u < UNR; ++u) step(pv0[u], jw + 4 * u);
                c = UNR;
            }
            for (; c + UNR <= nmine; c += UNR) {
                double pv[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) pv[u] = Pw[(c + u) * os];
#pragma unroll
                for (int u = 0; u < UNR; ++u) step(pv[u], jw + 4 * (c + u));
            }
            for (; c < nmine; ++c) step(Pw[c * os], jw + 4 * c);
        }
        if constexpr (SPLIT == 2) {
            // half 1 hands its partial sums to half 0 (same lane, same tile),
            // which adds them after its own
            if (half == 1 && rows) {
#pragma unroll
                for (int g2 = 0; g2 < NG; ++g2) red[g2 * 64] = acc[g2];
                if constexpr (ODD) {
                    red[NG * 64] = vr;
                    red[(NG + 1) * 64] = vi;
                }
            }
            __syncthreads();
            if (half == 0 && rows) {
#pragma unroll
                for (int g2 = 0; g2 < NG; ++g2) acc[g2] += red[g2 * 64];
                if constexpr (ODD) {
                    vr += red[NG * 64];
                    vi += red[(NG + 1) * 64];
                }
            }
        }
        if (half != 0 || !rows) continue;               // uniform
        // MFMA D: lane 4 b + j + 16 i holds degree row 4 b + i, column 4 g + j
        const int k = k0 + 4 * ((lane & 15) >> 2) + (lane >> 4);
        if (k < K) {
            double* o = reinterpret_cast<double*>(cout + s * cout_stride + ext_idx(N, m, m + p + 2 * k) * F + f0);
#pragma unroll
            for (int g2 = 0; g2 < NG; ++g2) o[4 * g2 + cb] = acc[g2];
        }
        if constexpr (ODD) {
            // sum of the four latitude slots (lanes l, l ^ 16, l ^ 32, l ^ 48), fixed order
            vr += __shfl_xor(vr, 16);
            vi += __shfl_xor(vi, 16);
            vr += __shfl_xor(vr, 32);
            vi += __shfl_xor(vi, 32);
            const int kv = k0 + (lane & 15);
            if (kq == 0 && kv < K)
                cout[s * cout_stride + ext_idx(N, m, m + p + 2 * kv) * F + f0 + NF - 1] = make_double2(vr, vi);
        }
    }
}


template <int NF, int STAGE = 0>
void syn_r(const shx_plan* pl, const double2* cin, double2* out, int F, int f0, int S, int nmax_use,
           long long cin_stride, double a, hipStream_t st, const NodeFuse& nfu = NodeFuse{}) {
    int Lmax = 0;                                       // longest segment over the orders
    for (int m = 0; m <= pl->N; ++m) Lmax = seg_len(pl->nmax - m + 1) > Lmax ? seg_len(pl->nmax - m + 1) : Lmax;
    const size_t lds = (size_t)4 * (Lmax * (NF + 1) + 4) * sizeof(double2) +
                       (STAGE == 3 ? (size_t)3 * (pl->N + 1) * sizeof(double2) : 0);
    const long long os = (long long)pl->J * (pl->N + 1) * F;
    // two latitude sets per wavefront from 384 latitude pairs up (fewer
    // wavefronts; measured faster at T1023, slower at T255 and below)
    if (pl->Jh >= 384) {
        const int gx = (pl->Jh + syn_lat(2) - 1) / syn_lat(2);
        k_leg_syn_m<NF, STAGE, 2><<<gx * (pl->N + 1), 64 * syn_wb(2), lds, st>>>(
            pl->ck, pl->ckoff, pl->rq, pl->cs, pl->mu, cin, out, pl->N, pl->nmax, nmax_use, pl->Jh, F, f0, S,
            cin_stride, os,
            gx, pl->nspec, a, Lmax, pl->pf, pl->ninv, pl->nn1, nfu);
    } else {
        const int gx = (pl->Jh + syn_lat(1) - 1) / syn_lat(1);
        k_leg_syn_m<NF, STAGE, 1><<<gx * (pl->N + 1), 64 * syn_wb(1), lds, st>>>(
            pl->ck, pl->ckoff, pl->rq, pl->cs, pl->mu, cin, out, pl->N, pl->nmax, nmax_use, pl->Jh, F, f0, S,
            cin_stride, os,
            gx, pl->nspec, a, Lmax, pl->pf, pl->ninv, pl->nn1, nfu);
    }
}

template <int NF>
void syn_chunk(const shx_plan* pl, const double2* cin, double2* out, int F, int f0, int S,
               int nmax_use, hipStream_t st) {
    syn_r<NF>(pl, cin, out, F, f0, S, nmax_use, pl->nspec_e * F, 0.0, st);
}

template <int NF>
void an_tab(const shx_plan* pl, const double2* G, double2* cout, int F, int f0, int S, int nmax_use,
            hipStream_t st) {
    {                                                   // FP64 plans with tables, Jh <= AN_TAB_JH
        const size_t lds = (size_t)4 * ((pl->Jh + 3) / 4) * NF * sizeof(double2);
        const int4* tb = reinterpret_cast<const int4*>(pl->tblk);
        const long long gst = (long long)pl->J * (pl->N + 1) * F, cst = pl->nspec_e * F;
        constexpr int NR = NF / 2 + (NF % 2 ? 2 : 0);
        const size_t lds2 = lds + (size_t)4 * NR * 64 * sizeof(double);
        if (an_batch(pl->Jh) == 8)
            k_leg_an<NF, 8, 1><<<pl->tb_nblk, 256, lds, st>>>(tb, pl->pan4, pl->off4, G, cout, pl->N, pl->nmax,
                                                             nmax_use, pl->J, F, f0, S, gst, cst);
        else
            k_leg_an<NF, 4, 2><<<pl->tb_nblk, 512, lds2, st>>>(tb, pl->pan4, pl->off4, G, cout, pl->N, pl->nmax,
                                                              nmax_use, pl->J, F, f0, S, gst, cst);
    }
}

template <int NF>
void an_chunk(const shx_plan* pl, const double2* G, double2* cout, int F, int f0, int S, int nmax_use,
              hipStream_t st) {
    const int ngrp = (pl->Jh + 63) / 64;
    const int nw = ngrp < 4 ? ngrp : 4;
    const size_t lds = (size_t)nw * 2 * 64 * 17 * sizeof(double);
    k_leg_an_m<NF><<<pl->an_nblk, 64 * nw, lds, st>>>(pl->anblk, pl->ck, pl->ckoff, pl->rq, pl->cs, pl->mu, G, cout,
                                                     pl->N,
                                                     pl->nmax, nmax_use, pl->J, F, f0, S,
                                                     (long long)pl->J * (pl->N + 1) * F, pl->nspec_e * F, nw);
}

}  // namespace

hipError_t launch_plm_table(const shx_plan* pl, hipStream_t st) {
    dim3 grid((pl->Jh + 63) / 64, pl->N + 1);
    k_plm_table<<<grid, 64, 0, st>>>(pl->mu, pl->sint, pl->off, pl->psyn, pl->pan, pl->ck, pl->ckoff, pl->rc,
                                     pl->rq, pl->cs,
                                     pl->N, pl->nmax, pl->Jh);
    return hipGetLastError();
}

hipError_t launch_an_tab4(const shx_plan* pl, long long max_block, hipStream_t st) {
    dim3 grid((unsigned)((max_block + 255) / 256), 2 * (pl->N + 1));
    if (pl->pan4f)
        k_an_tab4<float><<<grid, 256, 0, st>>>(pl->pan, pl->off, pl->off4, pl->pan4f, pl->nmax, pl->Jh);
    else
        k_an_tab4<double><<<grid, 256, 0, st>>>(pl->pan, pl->off, pl->off4, pl->pan4, pl->nmax, pl->Jh);
    return hipGetLastError();
}

hipError_t launch_an_polar(const shx_plan* pl, hipStream_t st) {
    dim3 grid(pl->an_kt, 2 * (pl->N + 1));
    if (pl->pan4f)
        k_an_polar<float><<<grid, 64, 0, st>>>(pl->pan4f, pl->off4, pl->an_c0, pl->nmax, pl->Jh, pl->an_kt,
                                               AN_POLAR_TAU);
    else
        k_an_polar<double><<<grid, 64, 0, st>>>(pl->pan4, pl->off4, pl->an_c0, pl->nmax, pl->Jh, pl->an_kt,
                                                AN_POLAR_TAU);
    return hipGetLastError();
}

hipError_t launch_plm_one(const shx_plan* pl, int m, int n, double* out, hipStream_t st) {
    k_plm_one<<<(pl->Jh + 63) / 64, 64, 0, st>>>(pl->mu, pl->sint, m, n, pl->Jh, out);
    return hipGetLastError();
}

// Fields are processed in chunks of at most 8 (16 accumulators per lane).
hipError_t launch_leg_syn(const shx_plan* pl, const double2* cin, double2* out, int F, int S,
                          int nmax_use, hipStream_t st) {
    if (pl->prec != SHX_FP64) return launch_leg_syn_mixed(pl, cin, out, F, S, nmax_use, st);
    for (int f0 = 0; f0 < F; f0 += 8) {
        const int nf = (F - f0 < 8) ? F - f0 : 8;
        switch (nf) {
            case 1: syn_chunk<1>(pl, cin, out, F, f0, S, nmax_use, st); break;
            case 2: syn_chunk<2>(pl, cin, out, F, f0, S, nmax_use, st); break;
            case 3: syn_chunk<3>(pl, cin, out, F, f0, S, nmax_use, st); break;
            case 4: syn_chunk<4>(pl, cin, out, F, f0, S, nmax_use, st); break;
            case 5: syn_chunk<5>(pl, cin, out, F, f0, S, nmax_use, st); break;
            case 6: syn_chunk<6>(pl, cin, out, F, f0, S, nmax_use, st); break;
            case 7: syn_chunk<7>(pl, cin, out, F, f0, S, nmax_use, st); break;
            default: syn_chunk<8>(pl, cin, out, F, f0, S, nmax_use, st); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_leg_syn_swe(const shx_plan* pl, double a, const double2* state, double2* out, int S,
                              hipStream_t st) {
    if (pl->prec != SHX_FP64) return launch_leg_syn_mixed_swe(pl, a, state, out, S, st);
    syn_r<4, 1>(pl, state, out, 4, 0, S, pl->nmax, 3 * pl->nspec, a, st);
    return hipGetLastError();
}

bool leg_syn_swe_node_supported(const shx_plan* pl) {
    return pl->prec == SHX_FP64 || leg_syn_mixed_swe_node_supported(pl);
}

hipError_t launch_leg_syn_swe_node(const shx_plan* pl, const NodeFuse& nf, double2* out, hipStream_t st) {
    if (nf.m < 1 || !nf.cout || !nf.theta || !nf.fi || !nf.fe) return hipErrorInvalidValue;
    if (pl->prec != SHX_FP64) return launch_leg_syn_mixed_swe_node(pl, nf, out, st);
    syn_r<4, 3>(pl, nullptr, out, 4, 0, 1, pl->nmax, 0, nf.p.a, st, nf);
    return hipGetLastError();
}

hipError_t launch_leg_syn_swe_adj(const shx_plan* pl, double a, const double2* lfe, double2* out, int S,
                                  hipStream_t st) {
    if (pl->prec != SHX_FP64) return hipErrorInvalidValue;
    syn_r<5, 2>(pl, lfe, out, 5, 0, S, pl->nmax, 3 * pl->nspec, a, st);
    return hipGetLastError();
}

hipError_t launch_leg_an(const shx_plan* pl, const double2* G, double2* cout, int F, int S,
                         int nmax_use, hipStream_t st) {
    if (pl->prec != SHX_FP64) return launch_leg_an_mixed(pl, G, cout, F, S, nmax_use, st);
    if (pl->pan4) {                                     // the table streamed once per 16 fields
        for (int f0 = 0; f0 < F; f0 += 16) {
            switch (F - f0 < 16 ? F - f0 : 16) {
                case 1: an_tab<1>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 2: an_tab<2>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 3: an_tab<3>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 4: an_tab<4>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 5: an_tab<5>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 6: an_tab<6>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 7: an_tab<7>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 8: an_tab<8>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 9: an_tab<9>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 10: an_tab<10>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 11: an_tab<11>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 12: an_tab<12>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 13: an_tab<13>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 14: an_tab<14>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 15: an_tab<15>(pl, G, cout, F, f0, S, nmax_use, st); break;
                default: an_tab<16>(pl, G, cout, F, f0, S, nmax_use, st); break;
            }
        }
        return hipGetLastError();
    }
    for (int f0 = 0; f0 < F; f0 += 8) {
        const int nf = (F - f0 < 8) ? F - f0 : 8;
        switch (nf) {
            case 1: an_chunk<1>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 2: an_chunk<2>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 3: an_chunk<3>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 4: an_chunk<4>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 5: an_chunk<5>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 6: an_chunk<6>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 7: an_chunk<7>(pl, G, cout, F, f0, S, nmax_use, st); break;
            default: an_chunk<8>(pl, G, cout, F, f0, S, nmax_use, st); break;
        }
    }
    return hipGetLastError();
}
