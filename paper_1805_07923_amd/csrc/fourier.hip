// Fourier step of the SH transform pair (Sec. 3, eq. fourier_transform and
// the longitude sum of eq. spectral_to_physical_space) and the grid-space
// products of the shallow-water tendency, FP64.  Every real latitude row is
// transformed on its own (row_fft.h), so the round-off of a row scales with
// that row alone.
//
// The tendency kernel fuses, per latitude row: the syntheses of zeta, Phi',
// U, V, the pointwise products A = eta U, B = eta V, C = Phi' U, D = Phi' V,
// E = (U^2 + V^2) / (2 cos^2 phi) with eta = zeta + 2 Omega mu, and the five
// analyses; the grid never leaves LDS.
#include "internal.h"
#include "row_fft.h"

namespace {

using rowfft::Cfg;
using rowfft::padded;
using rowfft::pidx;

// Inverse: one workgroup per (latitude row j, field f).  FI: [2][Jh][N+1][F]
// (even / odd Legendre sums); X = E + sgn O with sgn = +1 north, -1 south.
template <int L>
__global__ __launch_bounds__(Cfg<L>::T) void k_fft_inv(const double2* __restrict__ FI,
                                                       const double2* __restrict__ tw,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ grid, int N, int J, int F,
                                                       int mode) {
    constexpr int L2 = L / 2, T = Cfg<L>::T, P = padded(L2);
    __shared__ double2 row[2 * P];
    __shared__ double2 tws[L2];
    const int j = blockIdx.x, f = blockIdx.y;
    const int Jh = J / 2;
    const int jp = (j < Jh) ? j : J - 1 - j;
    const double sgn = (j < Jh) ? 1.0 : -1.0;
    const long long pstride = (long long)Jh * (N + 1) * F;
    const double2* e = FI + (long long)jp * (N + 1) * F + f;
    auto coef = [&](int, int m) {
        const double2 a = e[(long long)m * F], b = e[(long long)m * F + pstride];
        return make_double2(a.x + sgn * b.x, a.y + sgn * b.y);
    };
    rowfft::pack_rows<L, 1>(row, tws, tw, N, coef);
    __syncthreads();
    const double2* z = rowfft::fft<L2, T, 1, true>(row, row + P, tws, 1.0);
    double2* g = reinterpret_cast<double2*>(grid + ((long long)f * J + j) * L);
    const double gs = mode ? w[j] / L : 1.0;
    for (int k = threadIdx.x; k < L2; k += T) {
        const double2 v = z[pidx(k)];
        g[k] = make_double2(gs * v.x, gs * v.y);
    }
}

// Forward: one workgroup per (latitude row j, field f); G[j][m][f] = w_j X_m / L.
template <int L>
__global__ __launch_bounds__(Cfg<L>::T) void k_fft_fwd(const double* __restrict__ grid,
                                                       const double2* __restrict__ tw,
                                                       const double* __restrict__ w,
                                                       double2* __restrict__ G, int N, int J, int F,
                                                       int mode) {
    constexpr int L2 = L / 2, T = Cfg<L>::T, IT = (L2 + T - 1) / T, P = padded(L2);
    __shared__ double2 row[2 * P];
    __shared__ double2 tws[L2];
    const int j = blockIdx.x, f = blockIdx.y;
    const double2* g = reinterpret_cast<const double2*>(grid + ((long long)f * J + j) * L);
    double2 tv[IT], rv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int k = threadIdx.x + it * T;
        if (k < L2) {
            tv[it] = tw[k];
            rv[it] = g[k];
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int k = threadIdx.x + it * T;
        if (k < L2) {
            tws[k] = tv[it];
            row[pidx(k)] = rv[it];
        }
    }
    __syncthreads();
    const double2* z = rowfft::fft<L2, T, 1, true>(row, row + P, tws, -1.0);
    double2* out = G + (long long)j * (N + 1) * F + f;
    for (int m = threadIdx.x; m <= N; m += T) {
        const double sc = mode ? (m == 0 ? 1.0 : 2.0) : w[j] / L;
        const double2 X = rowfft::unpack<L>(z, tws, m);
        out[(long long)m * F] = make_double2(sc * X.x, sc * X.y);
    }
}

// Tendency grid kernel: one workgroup of five wavefronts per (latitude row
// j, state s).  FI[s]: [2][Jh][N+1][4] (zeta, Phi', U, V); G[s]: [J][N+1][5]
// (A, B, C, D, E), weighted for the analysis: w_j / (L cos^2 phi_j) for A..D,
// w_j / L for E.  Wavefront f < 4 synthesises field f along the row on its
// own (pack and inverse FFT, no workgroup barrier) while wavefront 4 copies
// the twiddles; after a barrier the whole workgroup forms the five products
// in place; after another, wavefront f analyses product row f on its own
// (forward FFT, unpack, weights) and stores it.  Blocks are numbered so
// that the two rows of a latitude pair (which read the same even / odd
// Legendre sums) run one after the other on one XCD (workgroups go to the
// XCDs round robin), where the second reads the sums from that XCD's L2.
constexpr int GRID_T = 320;
__device__ inline int grid_row(int b, int J) {
    const int Jh = J / 2;
    if (Jh % 8 != 0) return b;
    const int x = b % 8, t = b / 8;                     // XCD, slot on it
    const int k = 8 * (t / 2) + x;                      // latitude pair
    return (t % 2 == 0) ? k : J - 1 - k;
}
template <int L>
__global__ __launch_bounds__(GRID_T) void k_swe_grid(const double2* __restrict__ FI,
                                                     const double2* __restrict__ tw,
                                                     const double* __restrict__ mu,
                                                     const double* __restrict__ cos2,
                                                     const double* __restrict__ w,
                                                     double2* __restrict__ G, int N, int J,
                                                     double two_omega) {
    constexpr int L2 = L / 2, P = padded(L2);
    __shared__ double2 lds[5 * P];
    __shared__ double2 tws[L2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = grid_row(blockIdx.x, J), s = blockIdx.y;
    const int Jh = J / 2;
    const int jp = (j < Jh) ? j : J - 1 - j;
    const double sgn = (j < Jh) ? 1.0 : -1.0;
    if (wv < 4) {
        const long long pstride = (long long)Jh * (N + 1) * 4;
        const double2* e = FI + (long long)s * J * (N + 1) * 4 + (long long)jp * (N + 1) * 4 + wv;
        rowfft::wpack<L>(lds + wv * P, tw, N, lane, [&](int m) {
            const double2 a = e[(long long)m * 4], b = e[(long long)m * 4 + pstride];
            return make_double2(a.x + sgn * b.x, a.y + sgn * b.y);
        });
    } else {
        for (int t = lane; t < L2; t += 64) tws[t] = tw[t];
    }
    __syncthreads();
    if (wv < 4) rowfft::wfft<L2>(lds + wv * P, tws, 1.0, lane);
    __syncthreads();
    const double fc = two_omega * mu[j];
    const double hk = 0.5 / cos2[j];
    for (int k = threadIdx.x; k < L2; k += GRID_T) {
        // (x_{2k}, x_{2k+1}) of zeta, Phi', U, V; the five products in place
        const int q = pidx(k);
        const double2 z = lds[q], ph = lds[P + q], U = lds[2 * P + q], V = lds[3 * P + q];
        const double2 eta = make_double2(z.x + fc, z.y + fc);
        lds[q] = make_double2(eta.x * U.x, eta.y * U.y);
        lds[P + q] = make_double2(eta.x * V.x, eta.y * V.y);
        lds[2 * P + q] = make_double2(ph.x * U.x, ph.y * U.y);
        lds[3 * P + q] = make_double2(ph.x * V.x, ph.y * V.y);
        lds[4 * P + q] = make_double2((U.x * U.x + V.x * V.x) * hk, (U.y * U.y + V.y * V.y) * hk);
    }
    __syncthreads();
    double2* row = lds + wv * P;
    rowfft::wfft<L2>(row, tws, -1.0, lane);
    const double sc = (wv < 4) ? w[j] / (L * cos2[j]) : w[j] / L;
    double2* out = G + ((long long)s * J + j) * (N + 1) * 5 + wv;
    for (int m = lane; m <= N; m += 64) {
        const double2 X = rowfft::unpack<L>(row, tws, m);
        out[(long long)m * 5] = make_double2(sc * X.x, sc * X.y);
    }
}

template <int L>
hipError_t inv_t(const shx_plan* pl, const double2* FI, double* grid, int F, int mode, hipStream_t st) {
    dim3 g(pl->J, F);
    k_fft_inv<L><<<g, Cfg<L>::T, 0, st>>>(FI, pl->tw, pl->w, grid, pl->N, pl->J, F, mode);
    return hipGetLastError();
}
template <int L>
hipError_t fwd_t(const shx_plan* pl, const double* grid, double2* G, int F, int mode, hipStream_t st) {
    dim3 g(pl->J, F);
    k_fft_fwd<L><<<g, Cfg<L>::T, 0, st>>>(grid, pl->tw, pl->w, G, pl->N, pl->J, F, mode);
    return hipGetLastError();
}
template <int L>
hipError_t swe_t(const shx_plan* pl, const double2* FI, double2* G, int S, double omega, hipStream_t st) {
    dim3 g(pl->J, S);
    k_swe_grid<L><<<g, GRID_T, 0, st>>>(FI, pl->tw, pl->mu, pl->cos2, pl->w, G, pl->N, pl->J,
                                               2.0 * omega);
    return hipGetLastError();
}

#define SHX_FFT_LENGTHS(X) \
    X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) \
    X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)

}  // namespace

bool fft_length_supported(int L) {
    switch (L) {
#define CASE(n) case n:
        SHX_FFT_LENGTHS(CASE)
#undef CASE
        return true;
        default: return false;
    }
}

hipError_t launch_fft_inv(const shx_plan* pl, const double2* FI, double* grid, int F, int mode, hipStream_t st) {
    switch (pl->I) {
#define CASE(n) case n: return inv_t<n>(pl, FI, grid, F, mode, st);
        SHX_FFT_LENGTHS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fft_fwd(const shx_plan* pl, const double* grid, double2* G, int F, int mode, hipStream_t st) {
    switch (pl->I) {
#define CASE(n) case n: return fwd_t<n>(pl, grid, G, F, mode, st);
        SHX_FFT_LENGTHS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_swe_grid(const shx_plan* pl, const double2* FI, double2* G, int S, double omega,
                           hipStream_t st) {
    switch (pl->I) {
#define CASE(n) case n: return swe_t<n>(pl, FI, G, S, omega, st);
        SHX_FFT_LENGTHS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}
