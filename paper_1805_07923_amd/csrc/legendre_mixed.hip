// Reduced-precision Legendre contractions on MFMA (the same sums as
// legendre.hip: eq. spectral_to_physical_space over n, eq.
// legendre_transform over the Gaussian latitudes), FP32 accumulation.
//
//   SHX_FP32         tables in FP32; v_mfma_f32_16x16x4_f32 with the
//                    Fourier / spectral operand rounded to FP32.
//   SHX_SPLIT_BF16_2 x = x_hi + x_lo (bf16 each) for the table and the
//                    operand; products hi*hi + hi*lo + lo*hi on
//                    v_mfma_f32_16x16x16_bf16.
//   SHX_SPLIT_BF16_3 x = x_hi + x_mid + x_lo; the six products whose split
//                    orders sum to <= 2.
// The tables are built by the FP64 recurrence and then rounded / split.  The
// leading product (hi*hi) and the corrections accumulate in separate FP32
// registers and are added in FP64 at the end.
//
// MFMA operand layouts (64 lanes, lane l): A (16 x kk): row l % 16; B (kk x 16):
// column l % 16; D (16 x 16): D[4 (l / 16) + r][l % 16], r = 0..3.
//   16x16x4 f32:   A[l%16][l/16],          B[l/16][l%16]
//   16x16x16 bf16: A[l%16][4(l/16) + r],   B[4(l/16) + r][l%16]
// The bf16 tables keep the reduction dimension contiguous (analysis:
// [m][p][k][jp], synthesis: [m][p][jp][k]) padded with zeros to a multiple of
// 16, so each lane reads its four reduction elements as one 8-byte load.
#include "internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int U4 = 8;     // FP32 MFMA: chunks of 4 reduction elements per batch of loads
constexpr int U16 = 2;    // bf16 MFMA: chunks of 16 reduction elements per batch of loads
constexpr int AN_JC = 256;   // latitudes staged per chunk in the analysis (a multiple of 16)
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);          // round to nearest even (finite values)
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Split x into NP bf16 planes: x ~ sum_q planes[q], each the rounded remainder.
template <int NP>
__device__ __forceinline__ void split_bf16(double x, unsigned short* planes) {
    double rem = x;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const unsigned short h = f2bf((float)rem);
        planes[q] = h;
        rem -= (double)bf2f(h);
    }
}

// FP64 table -> FP32 copy (same layout), or -> NP bf16 planes with the
// other layout and padded reduction rows.
__global__ void k_tab_to_f32(const double* __restrict__ src, float* __restrict__ dst, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// dst planes [q][off16 + r * cols_pad + c] = split(src[off + r * cols + c]) for
// one (m, p) block per blockIdx.y; padding columns are zero.
template <int NP>
__global__ void k_tab_to_bf16(const double* __restrict__ src, const long long* __restrict__ off,
                              const long long* __restrict__ off16, const int* __restrict__ rows,
                              const int* __restrict__ cols, const int* __restrict__ cols_pad,
                              unsigned short* __restrict__ dst, long long plane) {
    const int b = blockIdx.y;
    const int R = rows[b], C = cols[b], Cp = cols_pad[b];
    const long long total = (long long)R * Cp;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
        const int r = (int)(i / Cp), c = (int)(i - (long long)r * Cp);
        unsigned short h[NP];
        if (c < C) {
            split_bf16<NP>(src[off[b] + (long long)r * C + c], h);
        } else {
#pragma unroll
            for (int q = 0; q < NP; ++q) h[q] = 0;
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) dst[q * plane + off16[b] + i] = h[q];
    }
}

// Products of split operands: MODE 2 -> (hi, lo), MODE 3 -> (hi, mid, lo).
// acc0 += hi*hi; acc1 += the correction products.
template <int MODE>
__device__ __forceinline__ void mfma_split(const shortx4* a, const shortx4* b, floatx4& acc0, floatx4& acc1) {
    acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[0], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[1], acc1, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[0], acc1, 0, 0, 0);
    if constexpr (MODE == 3) {
        acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[2], acc1, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[0], acc1, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[1], acc1, 0, 0, 0);
    }
}

// ------------------------------------------------------------------ analysis
// D[k][c] = sum_jp P[jp][k] g[jp][c], g = (G_north +/- G_south) of order m,
// columns c = 2 (f - f0) + {re, im}.  grid (ceil(K/64), N+1, 2), 4 waves:
// wave w owns rows k0 + 16 w .. + 15 and NCT column tiles.
template <int MODE, int NCT>
__global__ __launch_bounds__(256) void k_leg_an_mx(const void* __restrict__ tab, long long plane,
                                                   const long long* __restrict__ off,
                                                   const double2* __restrict__ G, double2* __restrict__ cout,
                                                   int N, int nmax_tab, int nmax_use, int J, int F, int f0, int NF,
                                                   int S, long long G_stride, long long cout_stride, int gx) {
    constexpr int NP = (MODE == 1) ? 1 : MODE;
    constexpr int CW = 16 * NCT;                        // columns
    extern __shared__ unsigned char smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const LegTile tile = leg_tile(gx, N + 1);
    const int m = tile.m, p = tile.p;
    const int K = kcount(nmax_use, m, p);
    const int kb = tile.x * 64;
    if (kb >= K) return;
    const int Ktab = kcount(nmax_tab, m, p);
    const int Jh = J / 2;
    const int Jhp = (Jh + 15) / 16 * 16;
    const double sg = p ? -1.0 : 1.0;
    const long long rowstride = (long long)(N + 1) * F;
    const int k0 = kb + 16 * wv;                        // this wave's row tile
    const bool wave_on = k0 < K;
    const int row = k0 + (lane & 15);
    const bool row_ok = row < K;
    for (int s = 0; s < S; ++s) {
        const double2* g = G + s * G_stride + (long long)m * F + f0;
        floatx4 acc0[NCT], acc1[NCT];
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            acc0[t] = floatx4{0.f, 0.f, 0.f, 0.f};
            acc1[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        // latitudes in chunks of at most AN_JC (a multiple of 16; one chunk
        // up to T255), so that the staged operand stays small at T511 / T1023
        for (int c0 = 0; c0 < Jh; c0 += AN_JC) {
            const int cj = min(AN_JC, Jh - c0);
            const int cjp = (cj + 15) / 16 * 16;        // bf16 reduction rows of this chunk
            __syncthreads();                            // previous chunk's / state's readers are done
            // stage g: FP32 as [jp][CW]; bf16 planes as [q][c][cjp].  One thread
            // per complex value (both columns of a field), in rounds of 4 per
            // thread whose loads (indices clamped to the range) are all issued
            // before any is used.
            constexpr int CH = CW / 2;
            const int tot = cjp * CH;
            for (int i0 = threadIdx.x; i0 < tot; i0 += 4 * 256) {
                double2 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = min(i0 + u * 256, tot - 1);
                    const int jl = i / CH, f = i - jl * CH;
                    const bool in = jl < cj && f < NF;
                    const int jc = in ? c0 + jl : 0, fc = in ? f : 0;
                    const double2 a = g[jc * rowstride + fc], b = g[(J - 1 - jc) * rowstride + fc];
                    v[u] = in ? make_double2(a.x + sg * b.x, a.y + sg * b.y) : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * 256;
                    if (i >= tot) break;
                    const int jl = i / CH, f = i - jl * CH;
                    if constexpr (MODE == 1) {
                        float* d = reinterpret_cast<float*>(smem) + jl * CW + 2 * f;
                        d[0] = (float)v[u].x;
                        d[1] = (float)v[u].y;
                    } else {
                        unsigned short hr[NP], hi[NP];
                        split_bf16<NP>(v[u].x, hr);
                        split_bf16<NP>(v[u].y, hi);
                        unsigned short* d = reinterpret_cast<unsigned short*>(smem);
#pragma unroll
                        for (int q = 0; q < NP; ++q) {
                            d[q * cjp * CW + (2 * f) * cjp + jl] = hr[q];
                            d[q * cjp * CW + (2 * f + 1) * cjp + jl] = hi[q];
                        }
                    }
                }
            }
            __syncthreads();
            if (!wave_on) continue;                     // no rows: staging and barriers only
            if constexpr (MODE == 1) {
                const float* P = static_cast<const float*>(tab) + off[2 * m + p] + (long long)c0 * Ktab +
                                 (row_ok ? row : 0);
                const float* gs = reinterpret_cast<const float*>(smem);
                // U4 chunks of 4 latitudes: their table loads are issued before the MFMAs
                for (int jc = 0; jc < cj; jc += 4 * U4) {
                    float a[U4];
#pragma unroll
                    for (int u = 0; u < U4; ++u) {
                        const int jp = jc + 4 * u + (lane >> 4);
                        a[u] = (row_ok && jp < cj) ? P[(long long)jp * Ktab] : 0.f;
                    }
#pragma unroll
                    for (int u = 0; u < U4; ++u) {
                        const int jp = jc + 4 * u + (lane >> 4);
#pragma unroll
                        for (int t = 0; t < NCT; ++t) {
                            const float b = (jp < cj) ? gs[jp * CW + 16 * t + (lane & 15)] : 0.f;
                            acc0[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b, acc0[t], 0, 0, 0);
                        }
                    }
                }
            } else {
                const unsigned short* P = static_cast<const unsigned short*>(tab);
                const long long base = off[2 * m + p] + (long long)(row_ok ? row : 0) * Jhp + c0;
                const unsigned short* gs = reinterpret_cast<const unsigned short*>(smem);
                for (int jc = 0; jc < cjp; jc += 16 * U16) {
                    shortx4 a[U16][NP];
#pragma unroll
                    for (int u = 0; u < U16; ++u) {
                        const int q4 = jc + 16 * u + 4 * (lane >> 4);
#pragma unroll
                        for (int q = 0; q < NP; ++q) {
                            const shortx4 v = (q4 < cjp) ? *reinterpret_cast<const shortx4*>(P + q * plane + base + q4)
                                                         : shortx4{0, 0, 0, 0};
                            a[u][q] = row_ok ? v : shortx4{0, 0, 0, 0};
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U16; ++u) {
                        const int q4 = jc + 16 * u + 4 * (lane >> 4);
                        if (jc + 16 * u >= cjp) break;
#pragma unroll
                        for (int t = 0; t < NCT; ++t) {
                            shortx4 b[NP];
                            const int c = 16 * t + (lane & 15);
#pragma unroll
                            for (int q = 0; q < NP; ++q)
                                b[q] = *reinterpret_cast<const shortx4*>(gs + q * cjp * CW + c * cjp + q4);
                            mfma_split<MODE>(a[u], b, acc0[t], acc1[t]);
                        }
                    }
                }
            }
        }
        if (!wave_on) continue;
        // D[4 (l/16) + r][l % 16]: row k0 + 4 (l/16) + r, column 16 t + l % 16
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = 16 * t + (lane & 15);
            if (c >= 2 * NF) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = k0 + 4 * (lane >> 4) + r;
                if (k >= K) continue;
                double* o = reinterpret_cast<double*>(cout + s * cout_stride + ext_idx(N, m, m + p + 2 * k) * F +
                                                      f0 + c / 2);
                o[c & 1] = (double)acc0[t][r] + (double)acc1[t][r];
            }
        }
    }
}

// ----------------------------------------------------------------- synthesis
// D[jp][c] = sum_k P[k][jp] C[k][c], C = coefficients of order m, parity p.
// grid (ceil(Jh/64), N+1, 2), 4 waves: wave w owns latitudes jb + 16 w .. + 15.
template <int MODE, int NCT, bool PREP = false>
__global__ __launch_bounds__(256) void k_leg_syn_mx(const void* __restrict__ tab, long long plane,
                                                    const long long* __restrict__ off,
                                                    const double2* __restrict__ cin, double2* __restrict__ out,
                                                    int N, int nmax_tab, int nmax_use, int Jh, int F, int f0,
                                                    int NF, int S, long long cin_stride, long long out_stride,
                                                    int gx, long long nspec, double a,
                                                    const double2* __restrict__ pf,
                                                    const double* __restrict__ ninv) {
    constexpr int NP = (MODE == 1) ? 1 : MODE;
    constexpr int CW = 16 * NCT;
    extern __shared__ unsigned char smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const LegTile tile = leg_tile(gx, N + 1);
    const int m = tile.m, p = tile.p;
    const int K = kcount(nmax_use, m, p);
    const int Ktab = kcount(nmax_tab, m, p);
    const int Kp = (Ktab + 15) / 16 * 16;
    const int j0 = tile.x * 64 + 16 * wv;               // this wave's latitude tile
    const bool wave_on = j0 < Jh;
    const long long e0 = ext_idx(N, m, m + p);
    const int KL = (MODE == 1) ? K : Kp;                // staged rows
    for (int s = 0; s < S; ++s) {
        const double2* c = cin + s * cin_stride + e0 * F + f0;
        __syncthreads();
        // stage C: FP32 as [k][CW]; bf16 planes as [q][c][Kp]
        auto put = [&](int k, int cc, double v) {
            if constexpr (MODE == 1) {
                reinterpret_cast<float*>(smem)[k * CW + cc] = (float)v;
            } else {
                unsigned short h[NP];
                split_bf16<NP>(v, h);
#pragma unroll
                for (int q = 0; q < NP; ++q)
                    reinterpret_cast<unsigned short*>(smem)[q * Kp * CW + cc * Kp + k] = h[q];
            }
        };
        if constexpr (PREP) {
            // one thread per row: the tendency's four fields from the state
            for (int k = threadIdx.x; k < KL; k += 256) {
                double2 o[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                                make_double2(0.0, 0.0)};
                if (k < K)
                    swe_prep_row(cin + s * cin_stride, nspec, N, a * a, 1.0 / a, pf + ext_idx(N, m, m), ninv, m,
                                 m + p + 2 * k, o);
#pragma unroll
                for (int cc = 0; cc < CW; ++cc) {
                    const double2 x = o[(cc / 2) & 3];
                    put(k, cc, (cc < 8) ? ((cc & 1) ? x.y : x.x) : 0.0);
                }
            }
        } else {
            // one thread per complex value (both columns of a field), in
            // rounds of 4 per thread whose loads (indices clamped to the
            // range) are all issued before any is used
            constexpr int CH = CW / 2;
            const int tot = KL * CH;
            for (int i0 = threadIdx.x; i0 < tot; i0 += 4 * 256) {
                double2 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = min(i0 + u * 256, tot - 1);
                    const int k = i / CH, f = i - k * CH;
                    const bool in = k < K && f < NF;
                    const double2 x = c[(long long)(2 * (in ? k : 0)) * F + (in ? f : 0)];
                    v[u] = in ? x : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * 256;
                    if (i >= tot) break;
                    const int k = i / CH, f = i - k * CH;
                    put(k, 2 * f, v[u].x);
                    put(k, 2 * f + 1, v[u].y);
                }
            }
        }
        __syncthreads();
        if (!wave_on) continue;
        floatx4 acc0[NCT], acc1[NCT];
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            acc0[t] = floatx4{0.f, 0.f, 0.f, 0.f};
            acc1[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        const int jr = j0 + (lane & 15);
        const bool j_ok = jr < Jh;
        if constexpr (MODE == 1) {
            const float* P = static_cast<const float*>(tab) + off[2 * m + p] + (j_ok ? jr : 0);
            const float* cs = reinterpret_cast<const float*>(smem);
            for (int kc = 0; kc < K; kc += 4 * U4) {
                float a[U4];
#pragma unroll
                for (int u = 0; u < U4; ++u) {
                    const int k = kc + 4 * u + (lane >> 4);
                    a[u] = (j_ok && k < K) ? P[(long long)k * Jh] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < U4; ++u) {
                    const int k = kc + 4 * u + (lane >> 4);
#pragma unroll
                    for (int t = 0; t < NCT; ++t) {
                        const float b = (k < K) ? cs[k * CW + 16 * t + (lane & 15)] : 0.f;
                        acc0[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b, acc0[t], 0, 0, 0);
                    }
                }
            }
        } else {
            const unsigned short* P = static_cast<const unsigned short*>(tab);
            const long long base = off[2 * m + p] + (long long)(j_ok ? jr : 0) * Kp;
            const unsigned short* cs = reinterpret_cast<const unsigned short*>(smem);
            for (int kc = 0; kc < K; kc += 16 * U16) {
                shortx4 a[U16][NP];
#pragma unroll
                for (int u = 0; u < U16; ++u) {
                    const int q4 = kc + 16 * u + 4 * (lane >> 4);
#pragma unroll
                    for (int q = 0; q < NP; ++q) {
                        const shortx4 v = (q4 < Kp) ? *reinterpret_cast<const shortx4*>(P + q * plane + base + q4)
                                                    : shortx4{0, 0, 0, 0};
                        a[u][q] = j_ok ? v : shortx4{0, 0, 0, 0};
                    }
                }
#pragma unroll
                for (int u = 0; u < U16; ++u) {
                    const int q4 = kc + 16 * u + 4 * (lane >> 4);
                    if (kc + 16 * u >= K) break;
#pragma unroll
                    for (int t = 0; t < NCT; ++t) {
                        shortx4 b[NP];
                        const int cc = 16 * t + (lane & 15);
#pragma unroll
                        for (int q = 0; q < NP; ++q)
                            b[q] = *reinterpret_cast<const shortx4*>(cs + q * Kp * CW + cc * Kp + q4);
                        mfma_split<MODE>(a[u], b, acc0[t], acc1[t]);
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int cc = 16 * t + (lane & 15);
            if (cc >= 2 * NF) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jp = j0 + 4 * (lane >> 4) + r;
                if (jp >= Jh) continue;
                double* o = reinterpret_cast<double*>(out + s * out_stride +
                                                      (((long long)p * Jh + jp) * (N + 1) + m) * F + f0 + cc / 2);
                o[cc & 1] = (double)acc0[t][r] + (double)acc1[t][r];
            }
        }
    }
}

template <int MODE, int NCT>
void an_mx(const shx_plan* pl, const double2* G, double2* cout, int F, int f0, int NF, int S, int nmax_use,
           hipStream_t st) {
    const int gx = (kcount(nmax_use, 0, 0) + 63) / 64;
    const unsigned grid = gx * (pl->N + 1) * 2;
    const int Jhp = (pl->Jh + 15) / 16 * 16;
    const int NP = MODE == 1 ? 1 : MODE;
    const int JC = Jhp < AN_JC ? Jhp : AN_JC;
    const size_t lds = (MODE == 1) ? (size_t)JC * 16 * NCT * 4 : (size_t)NP * JC * 16 * NCT * 2;
    const void* tab = (MODE == 1) ? (const void*)pl->pan32 : (const void*)pl->an16;
    k_leg_an_mx<MODE, NCT><<<grid, 256, lds, st>>>(tab, pl->an16_plane, MODE == 1 ? pl->off : pl->off_an16, G, cout,
                                                    pl->N, pl->nmax, nmax_use, pl->J, F, f0, NF, S,
                                                    (long long)pl->J * (pl->N + 1) * F, pl->nspec_e * F, gx);
}

// PREP: cin holds states [S][3][nspec] and the staged rows are the
// tendency's four grid fields (F = NF = 4, NCT = 1).
template <int MODE, int NCT, bool PREP = false>
void syn_mx(const shx_plan* pl, const double2* cin, double2* out, int F, int f0, int NF, int S, int nmax_use,
            hipStream_t st, double a = 0.0) {
    const int gx = (pl->Jh + 63) / 64;
    const unsigned grid = gx * (pl->N + 1) * 2;
    const int Kp = (kcount(pl->nmax, 0, 0) + 15) / 16 * 16;
    const int NP = MODE == 1 ? 1 : MODE;
    const size_t lds = (MODE == 1) ? (size_t)Kp * 16 * NCT * 4 : (size_t)NP * Kp * 16 * NCT * 2;
    const void* tab = (MODE == 1) ? (const void*)pl->psyn32 : (const void*)pl->syn16;
    k_leg_syn_mx<MODE, NCT, PREP><<<grid, 256, lds, st>>>(
        tab, pl->syn16_plane, MODE == 1 ? pl->off : pl->off_syn16, cin, out, pl->N, pl->nmax, nmax_use, pl->Jh, F,
        f0, NF, S, PREP ? 3 * pl->nspec : pl->nspec_e * F, (long long)pl->J * (pl->N + 1) * F, gx, pl->nspec, a,
        pl->pf, pl->ninv);
}

template <int MODE>
void an_mode(const shx_plan* pl, const double2* G, double2* cout, int F, int S, int nmax_use, hipStream_t st) {
    for (int f0 = 0; f0 < F; f0 += 16) {
        const int nf = F - f0 < 16 ? F - f0 : 16;
        if (nf <= 8) an_mx<MODE, 1>(pl, G, cout, F, f0, nf, S, nmax_use, st);
        else an_mx<MODE, 2>(pl, G, cout, F, f0, nf, S, nmax_use, st);
    }
}

template <int MODE>
void syn_mode(const shx_plan* pl, const double2* cin, double2* out, int F, int S, int nmax_use, hipStream_t st) {
    for (int f0 = 0; f0 < F; f0 += 16) {
        const int nf = F - f0 < 16 ? F - f0 : 16;
        if (nf <= 8) syn_mx<MODE, 1>(pl, cin, out, F, f0, nf, S, nmax_use, st);
        else syn_mx<MODE, 2>(pl, cin, out, F, f0, nf, S, nmax_use, st);
    }
}

}  // namespace

hipError_t launch_leg_an_mixed(const shx_plan* pl, const double2* G, double2* cout, int F, int S, int nmax_use,
                               hipStream_t st) {
    switch (pl->prec) {
        case SHX_FP32: an_mode<1>(pl, G, cout, F, S, nmax_use, st); break;
        case SHX_SPLIT_BF16_2: an_mode<2>(pl, G, cout, F, S, nmax_use, st); break;
        case SHX_SPLIT_BF16_3: an_mode<3>(pl, G, cout, F, S, nmax_use, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_leg_syn_mixed_swe(const shx_plan* pl, double a, const double2* state, double2* out, int S,
                                    hipStream_t st) {
    switch (pl->prec) {
        case SHX_FP32: syn_mx<1, 1, true>(pl, state, out, 4, 0, 4, S, pl->nmax, st, a); break;
        case SHX_SPLIT_BF16_2: syn_mx<2, 1, true>(pl, state, out, 4, 0, 4, S, pl->nmax, st, a); break;
        case SHX_SPLIT_BF16_3: syn_mx<3, 1, true>(pl, state, out, 4, 0, 4, S, pl->nmax, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_leg_syn_mixed(const shx_plan* pl, const double2* cin, double2* out, int F, int S, int nmax_use,
                                hipStream_t st) {
    switch (pl->prec) {
        case SHX_FP32: syn_mode<1>(pl, cin, out, F, S, nmax_use, st); break;
        case SHX_SPLIT_BF16_2: syn_mode<2>(pl, cin, out, F, S, nmax_use, st); break;
        case SHX_SPLIT_BF16_3: syn_mode<3>(pl, cin, out, F, S, nmax_use, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tables_to_f32(const shx_plan* pl, hipStream_t st) {
    const unsigned nb = (unsigned)((pl->table_elems + 255) / 256);
    k_tab_to_f32<<<nb, 256, 0, st>>>(pl->psyn, pl->psyn32, pl->table_elems);
    k_tab_to_f32<<<nb, 256, 0, st>>>(pl->pan, pl->pan32, pl->table_elems);
    return hipGetLastError();
}

// Analysis planes from psyn ([k][jp] per (m, p)), synthesis planes from pan
// ([jp][k]); per-(m, p) block descriptors are device arrays prepared by the host.
hipError_t launch_tables_to_bf16(const shx_plan* pl, const int* d_rows_an, const int* d_cols_an,
                                 const int* d_colsp_an, const int* d_rows_syn, const int* d_cols_syn,
                                 const int* d_colsp_syn, hipStream_t st) {
    dim3 g(64, 2 * (pl->N + 1));
    if (pl->prec == SHX_SPLIT_BF16_2) {
        k_tab_to_bf16<2><<<g, 256, 0, st>>>(pl->psyn, pl->off, pl->off_an16, d_rows_an, d_cols_an, d_colsp_an,
                                            pl->an16, pl->an16_plane);
        k_tab_to_bf16<2><<<g, 256, 0, st>>>(pl->pan, pl->off, pl->off_syn16, d_rows_syn, d_cols_syn, d_colsp_syn,
                                            pl->syn16, pl->syn16_plane);
    } else {
        k_tab_to_bf16<3><<<g, 256, 0, st>>>(pl->psyn, pl->off, pl->off_an16, d_rows_an, d_cols_an, d_colsp_an,
                                            pl->an16, pl->an16_plane);
        k_tab_to_bf16<3><<<g, 256, 0, st>>>(pl->pan, pl->off, pl->off_syn16, d_rows_syn, d_cols_syn, d_colsp_syn,
                                            pl->syn16, pl->syn16_plane);
    }
    return hipGetLastError();
}
