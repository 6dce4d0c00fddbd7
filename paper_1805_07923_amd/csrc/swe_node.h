// Per-coefficient pieces of the shallow-water right-hand side and of the
// sweep's implicit solve (Sec. 2 and Sec. 4.1: F_E from the weighted
// analyses of the grid products, F_I = L_G, and the diagonal implicit
// systems of eq. implicit_systems), shared by the node-update kernels and the
// synthesis that forms a node update in its staging.
#pragma once
#include "internal.h"

namespace swe_node {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 caxpy(double s, double2 a, double2 y) {
    return make_double2(fma(s, a.x, y.x), fma(s, a.y, y.y));
}
// i * m * a
__device__ __forceinline__ double2 cim(double m, double2 a) { return make_double2(-m * a.y, m * a.x); }

// F_E (from the weighted analyses A, B, C, D, E in the extended layout,
// cout = [ext][5]) and F_I (from the state st = [3][nspec]) at the
// coefficient i = (m, n).
__device__ __forceinline__ void combine_one(const double2* __restrict__ cout, const double2* __restrict__ st,
                                            int N, long long nspec, const swe_params& p, long long i, int m, int n,
                                            double2 fe[3], double2 fi[3]) {
    const double L = n * (n + 1.0) / (p.a * p.a);
    const double2* x0 = cout + ext_idx(N, m, n) * 5;
    const double2* xu = cout + ext_idx(N, m, n + 1) * 5;
    const double2 zero = make_double2(0.0, 0.0);
    const bool has_dn = (n - 1 >= m);
    const double2* xd = has_dn ? cout + ext_idx(N, m, n - 1) * 5 : nullptr;
    const double cu = n * eps_nm(n + 1, m), cd = (n + 1.0) * eps_nm(n, m);
    const double ia = 1.0 / p.a;
    auto div = [&](int X, int Y) {
        double2 r = cim(m, x0[X]);
        r = caxpy(cu, xu[Y], r);
        r = caxpy(-cd, has_dn ? xd[Y] : zero, r);
        return cscale(ia, r);
    };
    auto curl = [&](int X, int Y) {
        double2 r = cim(m, x0[Y]);
        r = caxpy(-cu, xu[X], r);
        r = caxpy(cd, has_dn ? xd[X] : zero, r);
        return cscale(ia, r);
    };
    const double2 dcd = div(2, 3), dab = div(0, 1), cab = curl(0, 1);
    fe[0] = make_double2(-dcd.x, -dcd.y);
    fe[1] = make_double2(-dab.x, -dab.y);
    fe[2] = caxpy(L, x0[4], cab);
    const double2 ph = st[i], ze = st[nspec + i], de = st[2 * nspec + i];
    fi[0] = make_double2(-p.phibar * de.x - p.nu * L * ph.x, -p.phibar * de.y - p.nu * L * ph.y);
    fi[1] = make_double2(-p.nu * L * ze.x, -p.nu * L * ze.y);
    fi[2] = make_double2(L * ph.x - p.nu * L * de.x, L * ph.y - p.nu * L * de.y);
}

__device__ __forceinline__ void solve_one(double L, double h, const swe_params& p, double2 bp, double2 bz,
                                          double2 bd, double2& xp, double2& xz, double2& xd) {
    // (1 + h nu L) Phi' + h Phibar delta = b_Phi ; (1 + h nu L) delta - h L Phi' = b_delta
    const double c = 1.0 + h * p.nu * L;
    const double den = c * c + h * h * p.phibar * L;
    xp = make_double2((c * bp.x - h * p.phibar * bd.x) / den, (c * bp.y - h * p.phibar * bd.y) / den);
    xd = make_double2((bd.x + h * L * xp.x) / c, (bd.y + h * L * xp.y) / c);
    xz = make_double2(bz.x / c, bz.y / c);
}

// The sweep's node update k = nf.m >= 1 for the coefficients of order m
// (degrees m..N), done by threads tid, tid + nthreads, ... of a block:
//   Theta^{k+1} = solve(S_k + sum_{j<=k} [dtQE F_E^j + dtQD F_I^j], h),
// S_k from the new-F_E slot of node k+1, the F of node k formed from its
// analyses (nf.cout) and Theta^k.  Theta^{k+1} goes to thn [3][N+1] (LDS,
// degree n at n - m); with store, also Theta^{k+1} and the F of node k to
// memory and Theta^{k+1} to the tape.
__device__ inline void node_update_order(const NodeFuse& nf, int N, long long nspec, int m, bool store,
                                         double2* thn, int tid, int nthreads) {
    const long long ns3 = 3 * nspec;
    const int k = nf.m;
    for (int t = tid; t <= N - m; t += nthreads) {
        const int n = m + t;
        const long long i = spec_idx(N, m, n);
        double2 fem[3], fim[3], acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = nf.fe[(k + 1) * ns3 + c * nspec + i];   // S_k
        combine_one(nf.cout, nf.theta + k * ns3, N, nspec, nf.p, i, m, n, fem, fim);
        for (int j = 1; j < k; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[c] = caxpy(nf.wt.qe[j], nf.fe[j * ns3 + c * nspec + i], acc[c]);
                acc[c] = caxpy(nf.wt.qd[j], nf.fi[j * ns3 + c * nspec + i], acc[c]);
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c] = caxpy(nf.wt.qe[k], fem[c], acc[c]);
            acc[c] = caxpy(nf.wt.qd[k], fim[c], acc[c]);
        }
        const double L = n * (n + 1.0) / (nf.p.a * nf.p.a);
        double2 x[3];
        solve_one(L, nf.h, nf.p, acc[0], acc[1], acc[2], x[0], x[1], x[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) thn[c * (N + 1) + t] = x[c];
        if (store) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long long o = c * nspec + i;
                nf.theta[(k + 1) * ns3 + o] = x[c];
                nf.fe[k * ns3 + o] = fem[c];
                nf.fi[k * ns3 + o] = fim[c];
                if (nf.rec) nf.rec[o] = x[c];
            }
        }
    }
}

}  // namespace swe_node
