// Fourier step of the SH transform pair (Sec. 3, eq. fourier_transform and
// the longitude sum of eq. spectral_to_physical_space) and the grid-space
// products of the shallow-water tendency, FP64.
//
// Every real latitude row of length L = nlon (2^k or 3 * 2^k) is transformed
// on its own through a complex FFT of length L/2 of z_k = x_{2k} + i x_{2k+1}
// (the standard half-length real transform), so the round-off of a row scales
// with that row alone and a row needs L * 8 bytes of LDS.  The complex FFT is
// an in-LDS Stockham transform (radix-4 stages, at most one radix-2 stage,
// then the radix-3 stage); each stage loads its butterflies into registers,
// meets a barrier and writes back in place.  Twiddles e^{-2 pi i t / L} come
// from a table computed on the host in quad precision.
//
//   synthesis:  Z_m = (X_m + conj X_{L/2-m}) + i e^{2 pi i m / L} (X_m - conj X_{L/2-m}),
//               z = sum_m Z_m e^{2 pi i m k / (L/2)}  ->  x_{2k} = Re z_k, x_{2k+1} = Im z_k;
//   analysis:   Z = FFT_{L/2}(z),  E_m = (Z_m + conj Z_{-m}) / 2,  O_m = (Z_m - conj Z_{-m}) / (2 i),
//               X_m = E_m + e^{-2 pi i m / L} O_m.
//
// The tendency kernel fuses, per latitude row: the syntheses of zeta, Phi',
// U, V, the pointwise products A = eta U, B = eta V, C = Phi' U, D = Phi' V,
// E = (U^2 + V^2) / (2 cos^2 phi) with eta = zeta + 2 Omega mu, and the five
// analyses; the grid never leaves LDS.
#include "internal.h"

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-register DFT of size R with exponent sign sg (-1 forward, +1 inverse).
template <int R>
__device__ __forceinline__ void dft(double2* v, double sg);

template <>
__device__ __forceinline__ void dft<2>(double2* v, double) {
    const double2 a = v[0], b = v[1];
    v[0] = make_double2(a.x + b.x, a.y + b.y);
    v[1] = make_double2(a.x - b.x, a.y - b.y);
}

template <>
__device__ __forceinline__ void dft<4>(double2* v, double sg) {
    const double2 s0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
    const double2 s1 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
    const double2 s2 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
    const double2 s3 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
    // sg * i * s3
    const double2 r3 = make_double2(-sg * s3.y, sg * s3.x);
    v[0] = make_double2(s0.x + s2.x, s0.y + s2.y);
    v[2] = make_double2(s0.x - s2.x, s0.y - s2.y);
    v[1] = make_double2(s1.x + r3.x, s1.y + r3.y);
    v[3] = make_double2(s1.x - r3.x, s1.y - r3.y);
}

template <>
__device__ __forceinline__ void dft<3>(double2* v, double sg) {
    const double c = 0.86602540378443864676;   // sin(2 pi / 3)
    const double2 t = make_double2(v[1].x + v[2].x, v[1].y + v[2].y);
    const double2 d = make_double2(v[1].x - v[2].x, v[1].y - v[2].y);
    const double2 a = v[0];
    const double2 mm = make_double2(a.x - 0.5 * t.x, a.y - 0.5 * t.y);
    const double2 r = make_double2(-sg * c * d.y, sg * c * d.x);   // sg * i * c * d
    v[0] = make_double2(a.x + t.x, a.y + t.y);
    v[1] = make_double2(mm.x + r.x, mm.y + r.y);
    v[2] = make_double2(mm.x - r.x, mm.y - r.y);
}

// Stockham stages for NR complex rows of length L held in LDS (row stride L),
// T threads; Ns is the length of the sub-transforms already done.
// Twiddles come from an LDS half table tws[t] = e^{-2 pi i t / (L TWM)},
// t < L TWM / 2 (the other half is its negative), shared with the real-row
// packing; the factor e^{-2 pi i t / L} sits at index t * TWM.
__device__ __forceinline__ double2 tw_half(const double2* tws, int idx, int half) {
    const double2 w = tws[idx < half ? idx : idx - half];
    return idx < half ? w : make_double2(-w.x, -w.y);
}

template <int L, int T, int NR, int Ns, int TWM>
__device__ __forceinline__ void fft_stages(double2* buf, const double2* tw, double sg) {
    constexpr int rem = L / Ns;
    if constexpr (rem > 1) {
        constexpr int R = (rem % 4 == 0) ? 4 : ((rem % 2 == 0) ? 2 : 3);
        constexpr int NB = L / R;
        constexpr int ITEMS = NR * NB;
        constexpr int IPT = (ITEMS + T - 1) / T;
        constexpr int TWS = L / (Ns * R) * TWM;
        double2 v[IPT][R];
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const int item = threadIdx.x + it * T;
            if (ITEMS % T == 0 || item < ITEMS) {
                const int row = item / NB, j = item - row * NB, k = j % Ns;
                const double2* b = buf + row * L;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double2 x = b[j + r * NB];
                    if (Ns > 1 && r > 0) {
                        double2 w = tw_half(tw, r * k * TWS, L * TWM / 2);
                        w.y *= -sg;
                        x = cmul(x, w);
                    }
                    v[it][r] = x;
                }
                dft<R>(v[it], sg);
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const int item = threadIdx.x + it * T;
            if (ITEMS % T == 0 || item < ITEMS) {
                const int row = item / NB, j = item - row * NB, k = j % Ns;
                const int base = (j / Ns) * Ns * R + k;
                double2* b = buf + row * L;
#pragma unroll
                for (int q = 0; q < R; ++q) b[base + q * Ns] = v[it][q];
            }
        }
        __syncthreads();
        fft_stages<L, T, NR, Ns * R, TWM>(buf, tw, sg);
    }
}

// Launch shape for real rows of length L (complex FFT length L/2).
template <int L>
struct FftCfg {
    static constexpr int L2 = L / 2;
    static constexpr int T0 = L2 / 2 < 64 ? 64 : (L2 / 2 > 1024 ? 1024 : L2 / 2);
    static constexpr int T = (T0 + 63) / 64 * 64;
};

// Build Z (length L/2) for the synthesis of one real row from its Fourier
// coefficients X_m, m = 0..N (X_m = 0 above N; Im X_0 ignored).  `coef(m)`
// returns X_m.  Caller syncs before the FFT.
// LDS copy of tw[0..L/2) (e^{-2 pi i t / L}); caller syncs.
template <int L>
__device__ __forceinline__ void load_twiddles(double2* tws, const double2* __restrict__ tw) {
    for (int t = threadIdx.x; t < L / 2; t += FftCfg<L>::T) tws[t] = tw[t];
}

template <int L, class Coef>
__device__ __forceinline__ void pack_synthesis(double2* row, const double2* tw, int N, Coef coef) {
    constexpr int L2 = L / 2, T = FftCfg<L>::T;
    for (int m = threadIdx.x; m < L2; m += T) {
        double2 A = make_double2(0.0, 0.0), B = A;
        if (m <= N) A = coef(m);
        if (m == 0) A.y = 0.0;
        const int j = L2 - m;
        if (m > 0 && j <= N) {
            const double2 x = coef(j);
            B = make_double2(x.x, -x.y);
        }
        const double2 s = make_double2(A.x + B.x, A.y + B.y);
        const double2 d = make_double2(A.x - B.x, A.y - B.y);
        // i e^{+2 pi i m / L} d, with tw[m] = e^{-2 pi i m / L}
        const double2 e = make_double2(tw[m].x, -tw[m].y);
        const double2 ed = cmul(e, d);
        row[m] = make_double2(s.x - ed.y, s.y + ed.x);
    }
}

// X_m (m <= N) of the real row whose half-length FFT is in `row`.
template <int L>
__device__ __forceinline__ double2 unpack_analysis(const double2* row, const double2* tw, int m) {
    constexpr int L2 = L / 2;
    const double2 z = row[m];
    const double2 zc = row[(L2 - m) % L2];
    const double2 E = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
    const double2 O = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    const double2 wo = cmul(tw[m], O);
    return make_double2(E.x + wo.x, E.y + wo.y);
}

// Inverse: one workgroup per (latitude row j, field f).  FI: [2][Jh][N+1][F]
// (even / odd Legendre sums); X = E + sgn O with sgn = +1 north, -1 south.
template <int L>
__global__ __launch_bounds__(FftCfg<L>::T) void k_fft_inv(const double2* __restrict__ FI,
                                                          const double2* __restrict__ tw,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ grid, int N, int J,
                                                          int F, int mode) {
    constexpr int L2 = L / 2, T = FftCfg<L>::T;
    __shared__ double2 row[L2];
    __shared__ double2 tws[L2];
    load_twiddles<L>(tws, tw);
    __syncthreads();
    const int j = blockIdx.x, f = blockIdx.y;
    const int Jh = J / 2;
    const int jp = (j < Jh) ? j : J - 1 - j;
    const double sgn = (j < Jh) ? 1.0 : -1.0;
    const long long pstride = (long long)Jh * (N + 1) * F;
    const double2* e = FI + (long long)jp * (N + 1) * F + f;
    auto coef = [&](int m) {
        const double2 a = e[(long long)m * F], b = e[(long long)m * F + pstride];
        return make_double2(a.x + sgn * b.x, a.y + sgn * b.y);
    };
    pack_synthesis<L>(row, tws, N, coef);
    __syncthreads();
    fft_stages<L2, T, 1, 1, 2>(row, tws, 1.0);
    double2* g = reinterpret_cast<double2*>(grid + ((long long)f * J + j) * L);
    const double gs = mode ? w[j] / L : 1.0;
    for (int k = threadIdx.x; k < L2; k += T) g[k] = make_double2(gs * row[k].x, gs * row[k].y);
}

// Forward: one workgroup per (latitude row j, field f); G[j][m][f] = w_j X_m / L.
template <int L>
__global__ __launch_bounds__(FftCfg<L>::T) void k_fft_fwd(const double* __restrict__ grid,
                                                          const double2* __restrict__ tw,
                                                          const double* __restrict__ w,
                                                          double2* __restrict__ G, int N, int J,
                                                          int F, int mode) {
    constexpr int L2 = L / 2, T = FftCfg<L>::T;
    __shared__ double2 row[L2];
    __shared__ double2 tws[L2];
    load_twiddles<L>(tws, tw);
    const int j = blockIdx.x, f = blockIdx.y;
    const double2* g = reinterpret_cast<const double2*>(grid + ((long long)f * J + j) * L);
    for (int k = threadIdx.x; k < L2; k += T) row[k] = g[k];
    __syncthreads();
    fft_stages<L2, T, 1, 1, 2>(row, tws, -1.0);
    double2* out = G + (long long)j * (N + 1) * F + f;
    for (int m = threadIdx.x; m <= N; m += T) {
        const double sc = mode ? (m == 0 ? 1.0 : 2.0) : w[j] / L;
        const double2 X = unpack_analysis<L>(row, tws, m);
        out[(long long)m * F] = make_double2(sc * X.x, sc * X.y);
    }
}

// Tendency grid kernel: one workgroup per (latitude row j, state s).
// FI[s]: [2][Jh][N+1][4] (zeta, Phi', U, V); G[s]: [J][N+1][5] (A, B, C, D, E),
// weighted for the analysis: w_j / (L cos^2 phi_j) for A..D, w_j / L for E.
template <int L>
__global__ __launch_bounds__(FftCfg<L>::T) void k_swe_grid(const double2* __restrict__ FI,
                                                           const double2* __restrict__ tw,
                                                           const double* __restrict__ mu,
                                                           const double* __restrict__ cos2,
                                                           const double* __restrict__ w,
                                                           double2* __restrict__ G, int N, int J,
                                                           double two_omega) {
    constexpr int L2 = L / 2, T = FftCfg<L>::T;
    __shared__ double2 lds[5 * L2];
    __shared__ double2 tws[L2];
    load_twiddles<L>(tws, tw);
    __syncthreads();
    const int j = blockIdx.x, s = blockIdx.y;
    const int Jh = J / 2;
    const int jp = (j < Jh) ? j : J - 1 - j;
    const double sgn = (j < Jh) ? 1.0 : -1.0;
    const long long pstride = (long long)Jh * (N + 1) * 4;
    const double2* e = FI + (long long)s * J * (N + 1) * 4 + (long long)jp * (N + 1) * 4;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        auto coef = [&](int m) {
            const double2 a = e[(long long)m * 4 + f], b = e[(long long)m * 4 + f + pstride];
            return make_double2(a.x + sgn * b.x, a.y + sgn * b.y);
        };
        pack_synthesis<L>(lds + f * L2, tws, N, coef);
    }
    __syncthreads();
    fft_stages<L2, T, 4, 1, 2>(lds, tws, 1.0);
    const double fc = two_omega * mu[j];
    const double hk = 0.5 / cos2[j];
    for (int k = threadIdx.x; k < L2; k += T) {
        // (x_{2k}, x_{2k+1}) of zeta, Phi', U, V
        const double2 z = lds[k], ph = lds[L2 + k], U = lds[2 * L2 + k], V = lds[3 * L2 + k];
        const double2 eta = make_double2(z.x + fc, z.y + fc);
        lds[k] = make_double2(eta.x * U.x, eta.y * U.y);
        lds[L2 + k] = make_double2(eta.x * V.x, eta.y * V.y);
        lds[2 * L2 + k] = make_double2(ph.x * U.x, ph.y * U.y);
        lds[3 * L2 + k] = make_double2(ph.x * V.x, ph.y * V.y);
        lds[4 * L2 + k] = make_double2((U.x * U.x + V.x * V.x) * hk, (U.y * U.y + V.y * V.y) * hk);
    }
    __syncthreads();
    fft_stages<L2, T, 5, 1, 2>(lds, tws, -1.0);
    const double sv = w[j] / (L * cos2[j]);
    const double se = w[j] / L;
    double2* out = G + ((long long)s * J + j) * (N + 1) * 5;
    for (int m = threadIdx.x; m <= N; m += T) {
        double2* o = out + (long long)m * 5;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const double2 X = unpack_analysis<L>(lds + f * L2, tws, m);
            const double sc = (f < 4) ? sv : se;
            o[f] = make_double2(sc * X.x, sc * X.y);
        }
    }
}

template <int L>
hipError_t inv_t(const shx_plan* pl, const double2* FI, double* grid, int F, int mode, hipStream_t st) {
    dim3 g(pl->J, F);
    k_fft_inv<L><<<g, FftCfg<L>::T, 0, st>>>(FI, pl->tw, pl->w, grid, pl->N, pl->J, F, mode);
    return hipGetLastError();
}
template <int L>
hipError_t fwd_t(const shx_plan* pl, const double* grid, double2* G, int F, int mode, hipStream_t st) {
    dim3 g(pl->J, F);
    k_fft_fwd<L><<<g, FftCfg<L>::T, 0, st>>>(grid, pl->tw, pl->w, G, pl->N, pl->J, F, mode);
    return hipGetLastError();
}
template <int L>
hipError_t swe_t(const shx_plan* pl, const double2* FI, double2* G, int S, double omega, hipStream_t st) {
    dim3 g(pl->J, S);
    k_swe_grid<L><<<g, FftCfg<L>::T, 0, st>>>(FI, pl->tw, pl->mu, pl->cos2, pl->w, G, pl->N, pl->J,
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
