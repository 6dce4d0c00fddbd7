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
#include "swe_node.h"

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

// FP32 analysis from the tiled FP32 table pan4f (SHX_FP32 plans with tables
// and at most AN_TAB_JH_F32 latitude pairs), the counterpart of the FP64 table
// analysis: one block per (m, parity, 64 degrees) from the plan's block list,
// one wavefront per 16 degrees summing the latitude groups of 4 pairs from
// its tile's first summed group on (polar truncation, AN_POLAR_TAU; runs of
// whole batches of UNR loads, the first issued before the Fourier staging).
// Per group v_mfma_f32_16x16x4f32 takes A = 16 degrees x 4 latitude pairs,
// 64 consecutive FP32 table values (one 4-byte load per lane; 4 x the rows
// of the block's last tile there), and B = the
// north +/- south Fourier data of the same pairs rounded to FP32 and staged
// in LDS as [jp][16 NCT] (columns 2f, 2f+1 = Re, Im of field f, zero past
// 2 NF; NCT = 1 or 2 products of 16 columns per group for up to 8 or 16
// fields); FP32 accumulation over the latitudes in order, as the untiled
// kernel.
template <int NF, int UNR>
__global__ __launch_bounds__(256) void k_leg_an_f32(const int4* __restrict__ tblk, const float* __restrict__ pan4f,
                                                    const long long* __restrict__ off4,
                                                    const double2* __restrict__ G, double2* __restrict__ cout,
                                                    int N, int nmax_tab, int nmax_use, int J, int F, int f0,
                                                    int S, long long G_stride, long long cout_stride) {
    static_assert(NF >= 1 && NF <= 16, "two 16-column products at most");
    constexpr int NCT = (NF + 7) / 8;                   // 16-column products per latitude group
    constexpr int CW = 16 * NCT;                        // staged columns
    extern __shared__ float gsf[];                      // [4 ngrp][CW]
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int4 tb = tblk[blockIdx.x];                   // (2m+p, tile, first groups, their minimum)
    const int mp = tb.x, tx = tb.y;
    if (mp < 0) return;                                 // padding block (uniform)
    const int m = mp >> 1, p = mp & 1;
    const int K = kcount(nmax_use, m, p);
    if (tx * 64 >= K) return;                           // whole block idle (uniform)
    const int Jh = J / 2;
    const int k0 = tx * 64 + 16 * wv;                   // this wavefront's first degree row
    const bool rows = k0 < K;                           // wave-uniform
    const int kq = lane >> 4, col = lane & 15;
    const int ngrp = (Jh + 3) / 4;
    // 4 r consecutive values per group, r = the tile's stored rows; lanes of
    // missing rows read row 0 again and their output rows are not stored
    const int Kt = kcount(nmax_tab, m, p);
    const int r = __builtin_amdgcn_readfirstlane(Kt - k0 < 16 ? (Kt - k0 > 0 ? Kt - k0 : 1) : 16);
    const int os = 4 * r;                               // operand stride
    const float* P = pan4f + off4[mp] + (long long)(k0 >> 4) * ngrp * 64 + kq * r + (col < r ? col : 0);
    const int cb0 = tb.w;                               // first staged latitude group
    const int cw0 = __builtin_amdgcn_readfirstlane(rows ? (tb.z >> (8 * wv)) & 255 : ngrp);
    const float* Pw = P + (long long)cw0 * os;
    const int nrun = ngrp - cw0, jw = 4 * cw0 + kq;
    const bool pre = rows && nrun >= UNR;               // wave-uniform
    float pv0[UNR];
    if (pre) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) pv0[u] = Pw[u * os];
    }
    const double sg = p ? -1.0 : 1.0;
    const long long rowstride = (long long)(N + 1) * F;
    for (int s = 0; s < S; ++s) {
        const double2* g = G + s * G_stride + (long long)m * F + f0;
        __syncthreads();                                // previous state's readers are done
        // rows of whole latitude groups (zeros past the last pair), so that
        // the products read their operands without a bounds test
        for (int i = 4 * cb0 * (CW / 2) + threadIdx.x; i < 4 * ngrp * (CW / 2); i += 256) {
            const int jp = i / (CW / 2), f = i - jp * (CW / 2);
            float re = 0.f, im = 0.f;
            if (f < NF && jp < Jh) {
                const double2 a = g[jp * rowstride + f], b = g[(J - 1 - jp) * rowstride + f];
                re = (float)(a.x + sg * b.x);
                im = (float)(a.y + sg * b.y);
            }
            gsf[jp * CW + 2 * f] = re;
            gsf[jp * CW + 2 * f + 1] = im;
        }
        __syncthreads();
        if (!rows) continue;                            // uniform
        floatx4 acc[NCT];
#pragma unroll
        for (int t = 0; t < NCT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        auto step = [&](float a, int jp) {
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const float b = gsf[jp * CW + 16 * t + col];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
            }
        };
        int c = 0;
        if (pre) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) step(pv0[u], jw + 4 * u);
            c = UNR;
        }
        for (; c + UNR <= nrun; c += UNR) {
            float pv[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) pv[u] = Pw[(c + u) * os];
#pragma unroll
            for (int u = 0; u < UNR; ++u) step(pv[u], jw + 4 * (c + u));
        }
        for (; c < nrun; ++c) step(Pw[c * os], jw + 4 * c);
        // D[4 (l/16) + r][l % 16]: row k0 + 4 (l/16) + r, column 16 t + l % 16
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = 16 * t + col;
            if (c >= 2 * NF) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = k0 + 4 * kq + r;
                if (k < K) {
                    double* o = reinterpret_cast<double*>(cout + s * cout_stride + ext_idx(N, m, m + p + 2 * k) * F +
                                                          f0 + c / 2);
                    o[c & 1] = (double)acc[t][r];
                }
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

// ------------------------------------------- without tables (on the fly)
// Plans created with SHX_TABLE_ONTHEFLY hold no table: P^m_n comes from the
// FP64 three-term recurrence of the orthonormal functions (Sec. 3), run from
// the plan's exact restart values as in the FP64 matrix-core kernels of
// legendre.hip, and is rounded to FP32 (MODE 1) or split into bf16 pieces
// (MODE 2, 3) in registers right before the product; the other operand is
// rounded / split the same way; FP32 accumulation.

// Value of lane src (wave-uniform) of a per-lane double, for every lane.
__device__ __forceinline__ double bcast_lane(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// NP bf16 pieces of four values, packed as the 4-element MFMA operands.
template <int NP>
__device__ __forceinline__ void split4(const double* v, shortx4* out) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        unsigned short h[NP];
        split_bf16<NP>(v[r], h);
#pragma unroll
        for (int q = 0; q < NP; ++q) out[q][r] = (short)h[q];
    }
}

// Synthesis: the organisation of k_leg_syn_m (one wavefront per 16
// latitudes, lane (i, q) = latitude i and restart segment q of the round,
// two degrees per recurrence step, even / odd accumulators).  MODE 1:
// v_mfma_f32_16x16x4_f32 per degree pair, A = P (lane's latitude, segment)
// and B = the lane's coefficient, both rounded to FP32.  MODE 2, 3:
// v_mfma_f32_16x16x16_bf16 per four degrees of one parity: the lane's four
// P values (k slots 4q..4q+3) and its four coefficients are split into bf16
// pieces (the lane supplies exactly the k slots of its own segment).  D:
// D[4 (l/16) + r][l % 16] = latitude 4 (l/16) + r, column l % 16.
template <int NF, int MODE, int STAGE>
__global__ __launch_bounds__(256) void k_leg_syn_mo(const double2* __restrict__ ck,
                                                    const long long* __restrict__ ckoff,
                                                    const double2* __restrict__ rc,
                                                    const double* __restrict__ mu,
                                                    const double2* __restrict__ cin, double2* __restrict__ out,
                                                    int N, int nmax_tab, int nmax_use, int Jh, int F, int f0, int S,
                                                    long long cin_stride, long long out_stride, int gx,
                                                    long long nspec, double a, int Lmax,
                                                    const double2* __restrict__ pf,
                                                    const double* __restrict__ ninv, NodeFuse nfu) {
    static_assert(NF >= 1 && NF <= 8, "16 real columns per product");
    constexpr int NP = (MODE == 1) ? 1 : MODE;
    constexpr int U = 8;                                // degrees per batch of LDS reads
    extern __shared__ double2 csh[];                    // [4][L NF + 2] rows, then [4][L + 2] rc, then (STAGE 3) [3][N+1]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = lane & 15, q = lane >> 4;
    const int ic = i < 2 * NF ? i : 2 * NF - 1;
    const LegTile tile = leg_tile(gx, N + 1, 1);
    const int m = tile.m;
    const int jw = tile.x * 64 + wv * 16;
    const int jp = jw + i;
    const bool active = jp < Jh;
    const int Kt = nmax_tab - m + 1, Ku = nmax_use - m + 1;
    const int R = seg_rounds(Kt), L = seg_len(Kt);
    const int SC = L * NF + 2, SR = L + 2;
    const double x = mu[active ? jp : 0];
    const double2* ckm = ck + ckoff[m] + (active ? jp : 0);
    double2* rsh = csh + 4 * (Lmax * NF + 2);
    const double* cq = reinterpret_cast<const double*>(csh + q * SC) + ic;
    const double2* rq = rsh + q * SR;
    const double2* rcm = rc + ext_idx(N, m, m);
    const double2* pfm = pf + ext_idx(N, m, m);
    const double ia = 1.0 / a, a2 = a * a;
    // STAGE 3: the sweep's node update of order m (FP64) into LDS first, the
    // tendency rows (as STAGE 1) then staged from there; the block of the
    // first latitude group stores the sweep's outputs (S = 1)
    double2* thn = csh + 4 * (Lmax * (NF + 1) + 4);
    if constexpr (STAGE == 3) {
        static_assert(STAGE != 3 || NF == 4, "the tendency synthesis has four fields");
        swe_node::node_update_order(nfu, N, nspec, m, tile.x == 0, thn, threadIdx.x, 256);
    }
    for (int s = 0; s < S; ++s) {
        floatx4 e0 = {0.f, 0.f, 0.f, 0.f}, e1 = e0, o0 = e0, o1 = e0;
        for (int r = 0; r < R; ++r) {
            const int kr0 = 4 * r * L;
            if (kr0 >= Ku) break;                       // uniform
            const int g = 4 * r + q;
            const double2 c0 = ckm[(long long)g * Jh];
            __syncthreads();
            for (int kl = threadIdx.x; kl < 4 * L; kl += 256) {
                const int qs = kl / L, ts = kl - qs * L, kk = kr0 + kl;
                double2* row = csh + qs * SC + ts * NF;
                if (kk < Ku) {
                    if constexpr (STAGE == 1) {
                        static_assert(STAGE != 1 || NF == 4, "the tendency synthesis has four fields");
                        double2 o[4];
                        swe_prep_row(cin + s * cin_stride, nspec, N, a2, ia, pfm, ninv, m, m + kk, o);
#pragma unroll
                        for (int f = 0; f < 4; ++f) row[f] = o[f];
                    } else if constexpr (STAGE == 3) {
                        double2 o[4];
                        swe_prep_row_t([&](int f, int nn) { return thn[f * (N + 1) + (nn - m)]; }, N, a2, ia, pfm,
                                       ninv, m, m + kk, o);
#pragma unroll
                        for (int f = 0; f < 4; ++f) row[f] = o[f];
                    } else {
                        const double2* cg = cin + s * cin_stride + (ext_idx(N, m, m) + kk) * F + f0;
#pragma unroll
                        for (int f = 0; f < NF; ++f) row[f] = cg[f];
                    }
                } else {
#pragma unroll
                    for (int f = 0; f < NF; ++f) row[f] = make_double2(0.0, 0.0);
                }
                rsh[qs * SR + ts] = (kk < Kt) ? rcm[kk] : make_double2(0.0, 0.0);
            }
            __syncthreads();
            if (jw >= Jh) continue;
            double pe = c0.x, po = c0.y;
            for (int t = 0; t < L; t += U) {
                double2 rr[U];
                double bb[U], pv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    rr[u] = rq[t + u];
                    bb[u] = cq[(t + u) * 2 * NF];
                }
#pragma unroll
                for (int u = 0; u < U; u += 2) {
                    if (u > 0 || t > 0) {
                        const double ne = fma(rr[u].x * x, po, -(rr[u].y * pe));
                        po = fma(rr[u + 1].x * x, ne, -(rr[u + 1].y * po));
                        pe = ne;
                    }
                    pv[u] = pe;
                    pv[u + 1] = po;
                    if constexpr (MODE == 1) {
                        e0 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)pe, (float)bb[u], e0, 0, 0, 0);
                        o0 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)po, (float)bb[u + 1], o0, 0, 0, 0);
                    }
                }
                if constexpr (MODE != 1) {
                    const double ve[4] = {pv[0], pv[2], pv[4], pv[6]}, vo[4] = {pv[1], pv[3], pv[5], pv[7]};
                    const double we[4] = {bb[0], bb[2], bb[4], bb[6]}, wo[4] = {bb[1], bb[3], bb[5], bb[7]};
                    shortx4 aE[NP], aO[NP], bE[NP], bO[NP];
                    split4<NP>(ve, aE);
                    split4<NP>(vo, aO);
                    split4<NP>(we, bE);
                    split4<NP>(wo, bO);
                    mfma_split<MODE>(aE, bE, e0, e1);
                    mfma_split<MODE>(aO, bO, o0, o1);
                }
            }
        }
        if (jw < Jh && i < 2 * NF) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int jr = jw + 4 * q + rr;
                if (jr < Jh) {
                    double* d = reinterpret_cast<double*>(out + s * out_stride +
                                                          ((long long)jr * (N + 1) + m) * F + f0) + i;
                    d[0] = (double)e0[rr] + (double)e1[rr];
                    d[(long long)Jh * (N + 1) * F * 2] = (double)o0[rr] + (double)o1[rr];
                }
            }
        }
    }
}

// Analysis: the organisation of k_leg_an_m (one block per (order m,
// restart segment g), wavefronts over groups of 64 latitudes, lane =
// latitude running the recurrence into a wave-private LDS tile of 32
// degrees per parity; partial sums of the latitude groups added through LDS
// in wavefront order, in FP64).  MODE 1: v_mfma_f32_16x16x4_f32, A = P of 16
// degrees x 4 latitudes from the tile, B = the north +/- south Fourier
// coefficients, both rounded to FP32.  MODE 2, 3: v_mfma_f32_16x16x16_bf16
// over 16 latitudes, lane (i, q) = degree i and latitudes 4q..4q+3 of the
// chunk, operands split into bf16 pieces.
template <int NF, int MODE>
__global__ __launch_bounds__(256) void k_leg_an_mo(const int* __restrict__ blist,
                                                   const double2* __restrict__ ck,
                                                   const long long* __restrict__ ckoff,
                                                   const double2* __restrict__ rc,
                                                   const double* __restrict__ mu,
                                                   const double2* __restrict__ G,
                                                   double2* __restrict__ cout, int N, int nmax_tab,
                                                   int nmax_use, int J, int F, int f0, int S,
                                                   long long G_stride, long long cout_stride, int nw) {
    static_assert(NF >= 1 && NF <= 8, "16 real columns per product");
    constexpr int NP = (MODE == 1) ? 1 : MODE;
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
    const int kend = min(k0 + L, Ku);
    const int ntp = (kend - k0 + 31) / 32;
    const int ngrp = (Jh + 63) / 64;
    double* PE = lsh + wv * (2 * 64 * TP);
    double* PO = PE + 64 * TP;
    double* red = lsh;
    const double2* rcm = rc + ext_idx(N, m, m);
    const long long rs = (long long)(N + 1) * F * 2;
    const int jc = i < 2 * NF ? i : 2 * NF - 1;
    for (int s = 0; s < S; ++s) {
        floatx4 acc[2][2][2];                           // [tile pair][parity][leading, corrections]
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b][0] = acc[a][b][1] = floatx4{0.f, 0.f, 0.f, 0.f};
        const double* gs = reinterpret_cast<const double*>(G + s * G_stride + (long long)m * F + f0) + jc;
        for (int lg = wv; lg < ngrp; lg += nw) {
            const int jp = lg * 64 + lane;
            const bool act = jp < Jh;
            const double x = mu[act ? jp : 0];
            const double2 c0 = act ? ck[ckoff[m] + (long long)g * Jh + jp] : make_double2(0.0, 0.0);
            // B operands: the Fourier data of latitude lg 64 + jl for the lane's column
            // (MODE 1: jl = 4c + q; MODE 2, 3: jl = 16 c4 + 4q + r)
            double be[16], bo[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int jl = (MODE == 1) ? 4 * c + q : 16 * (c >> 2) + 4 * q + (c & 3);
                const int jb = lg * 64 + jl;
                const bool ab = jb < Jh;
                const int jr = ab ? jb : 0;
                const double vn = gs[jr * rs], vs = gs[(J - 1 - jr) * rs];
                be[c] = ab ? vn + vs : 0.0;
                bo[c] = ab ? vn - vs : 0.0;
            }
            double pe = c0.x, po = c0.y;
            const double2 rcv = rcm[min(k0 + lane, Kt - 1)];
            for (int tp = 0; tp < ntp; ++tp) {
#pragma unroll
                for (int i2 = 0; i2 < 16; ++i2) {
                    if (tp > 0 || i2 > 0) {
                        const int t = 32 * tp + 2 * i2;
                        const double r0x = bcast_lane(rcv.x, t), r0y = bcast_lane(rcv.y, t);
                        const double r1x = bcast_lane(rcv.x, t + 1), r1y = bcast_lane(rcv.y, t + 1);
                        const double ne = fma(r0x * x, po, -(r0y * pe));
                        po = fma(r1x * x, ne, -(r1y * po));
                        pe = ne;
                    }
                    PE[lane * TP + i2] = pe;
                    PO[lane * TP + i2] = po;
                }
                if constexpr (MODE == 1) {
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const float ae = (float)PE[(4 * c + q) * TP + i];
                        const float ao = (float)PO[(4 * c + q) * TP + i];
                        acc[tp][0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ae, (float)be[c], acc[tp][0][0], 0, 0, 0);
                        acc[tp][1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ao, (float)bo[c], acc[tp][1][0], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4) {
                        double ve[4], vo[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            ve[r] = PE[(16 * c4 + 4 * q + r) * TP + i];
                            vo[r] = PO[(16 * c4 + 4 * q + r) * TP + i];
                        }
                        shortx4 aE[NP], aO[NP], bE[NP], bO[NP];
                        split4<NP>(ve, aE);
                        split4<NP>(vo, aO);
                        split4<NP>(be + 4 * c4, bE);
                        split4<NP>(bo + 4 * c4, bO);
                        mfma_split<MODE>(aE, bE, acc[tp][0][0], acc[tp][0][1]);
                        mfma_split<MODE>(aO, bO, acc[tp][1][0], acc[tp][1][1]);
                    }
                }
            }
        }
        __syncthreads();                                // all tile reads done
        for (int tp = 0; tp < ntp; ++tp)
#pragma unroll
            for (int eo = 0; eo < 2; ++eo)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    red[(((wv * 2 + tp) * 2 + eo) * 4 + rr) * 64 + lane] =
                        (double)acc[tp][eo][0][rr] + (double)acc[tp][eo][1][rr];
        __syncthreads();
        // D layout (16x16, f32): the lane holds rows 4q + rr (degree pairs) of column i
        for (int u = wv; u < 2 * ntp && i < 2 * NF; u += nw) {
            const int tp = u >> 1, eo = u & 1;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int k = k0 + 32 * tp + 2 * (4 * q + rr) + eo;
                if (k < kend) {
                    double v = 0.0;
                    for (int w = 0; w < nw; ++w) v += red[(((w * 2 + tp) * 2 + eo) * 4 + rr) * 64 + lane];
                    reinterpret_cast<double*>(cout + s * cout_stride + ext_idx(N, m, m + k) * F + f0)[i] = v;
                }
            }
        }
        __syncthreads();
    }
}

template <int NF, int MODE, int STAGE>
void syn_mo(const shx_plan* pl, const double2* cin, double2* out, int F, int f0, int S, int nmax_use,
            long long cin_stride, double a, hipStream_t st, const NodeFuse& nfu = NodeFuse{}) {
    const int gx = (pl->Jh + 63) / 64;
    int Lmax = 0;
    for (int m = 0; m <= pl->N; ++m) Lmax = seg_len(pl->nmax - m + 1) > Lmax ? seg_len(pl->nmax - m + 1) : Lmax;
    const size_t lds = (size_t)4 * (Lmax * (NF + 1) + 4) * sizeof(double2) +
                       (STAGE == 3 ? (size_t)3 * (pl->N + 1) * sizeof(double2) : 0);
    k_leg_syn_mo<NF, MODE, STAGE><<<gx * (pl->N + 1), 256, lds, st>>>(
        pl->ck, pl->ckoff, pl->rc, pl->mu, cin, out, pl->N, pl->nmax, nmax_use, pl->Jh, F, f0, S, cin_stride,
        (long long)pl->J * (pl->N + 1) * F, gx, pl->nspec, a, Lmax, pl->pf, pl->ninv, nfu);
}

template <int NF, int MODE>
void an_mo(const shx_plan* pl, const double2* G, double2* cout, int F, int f0, int S, int nmax_use,
           hipStream_t st) {
    const int ngrp = (pl->Jh + 63) / 64;
    const int nw = ngrp < 4 ? ngrp : 4;
    const size_t lds = (size_t)nw * 2 * 64 * 17 * sizeof(double);
    k_leg_an_mo<NF, MODE><<<pl->an_nblk, 64 * nw, lds, st>>>(pl->anblk, pl->ck, pl->ckoff, pl->rc, pl->mu, G, cout,
                                                            pl->N, pl->nmax, nmax_use, pl->J, F, f0, S,
                                                            (long long)pl->J * (pl->N + 1) * F, pl->nspec_e * F,
                                                            nw);
}

template <int MODE>
void syn_mo_fields(const shx_plan* pl, const double2* cin, double2* out, int F, int S, int nmax_use,
                   hipStream_t st) {
    const long long cs = pl->nspec_e * F;
    for (int f0 = 0; f0 < F; f0 += 8) {
        switch (F - f0 < 8 ? F - f0 : 8) {
            case 1: syn_mo<1, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
            case 2: syn_mo<2, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
            case 3: syn_mo<3, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
            case 4: syn_mo<4, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
            case 5: syn_mo<5, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
            case 6: syn_mo<6, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
            case 7: syn_mo<7, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
            default: syn_mo<8, MODE, 0>(pl, cin, out, F, f0, S, nmax_use, cs, 0.0, st); break;
        }
    }
}

template <int MODE>
void an_mo_fields(const shx_plan* pl, const double2* G, double2* cout, int F, int S, int nmax_use,
                  hipStream_t st) {
    for (int f0 = 0; f0 < F; f0 += 8) {
        switch (F - f0 < 8 ? F - f0 : 8) {
            case 1: an_mo<1, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 2: an_mo<2, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 3: an_mo<3, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 4: an_mo<4, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 5: an_mo<5, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 6: an_mo<6, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
            case 7: an_mo<7, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
            default: an_mo<8, MODE>(pl, G, cout, F, f0, S, nmax_use, st); break;
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

template <int NF>
void an_f32(const shx_plan* pl, const double2* G, double2* cout, int F, int f0, int S, int nmax_use,
            hipStream_t st) {
    const size_t lds = (size_t)4 * ((pl->Jh + 3) / 4) * 16 * ((NF + 7) / 8) * sizeof(float);
    const int4* tb = reinterpret_cast<const int4*>(pl->tblk);
    const long long gst = (long long)pl->J * (pl->N + 1) * F, cst = pl->nspec_e * F;
    if (an_batch(pl->Jh) == 8)
        k_leg_an_f32<NF, 8><<<pl->tb_nblk, 256, lds, st>>>(tb, pl->pan4f, pl->off4, G, cout, pl->N, pl->nmax, nmax_use,
                                                          pl->J, F, f0, S, gst, cst);
    else
        k_leg_an_f32<NF, 4><<<pl->tb_nblk, 256, lds, st>>>(tb, pl->pan4f, pl->off4, G, cout, pl->N, pl->nmax, nmax_use,
                                                          pl->J, F, f0, S, gst, cst);
}

template <int MODE>
void an_mode(const shx_plan* pl, const double2* G, double2* cout, int F, int S, int nmax_use, hipStream_t st) {
    if (MODE == 1 && pl->pan4f) {                       // tiled FP32 table, chunks of 16 fields
        // (of 8 where 16 fields would stage more than 64 KB of LDS)
        const int chunk = (size_t)4 * ((pl->Jh + 3) / 4) * 32 * sizeof(float) <= 65536 ? 16 : 8;
        for (int f0 = 0; f0 < F; f0 += chunk) {
            switch (F - f0 < chunk ? F - f0 : chunk) {
                case 1: an_f32<1>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 2: an_f32<2>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 3: an_f32<3>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 4: an_f32<4>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 5: an_f32<5>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 6: an_f32<6>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 7: an_f32<7>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 8: an_f32<8>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 9: an_f32<9>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 10: an_f32<10>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 11: an_f32<11>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 12: an_f32<12>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 13: an_f32<13>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 14: an_f32<14>(pl, G, cout, F, f0, S, nmax_use, st); break;
                case 15: an_f32<15>(pl, G, cout, F, f0, S, nmax_use, st); break;
                default: an_f32<16>(pl, G, cout, F, f0, S, nmax_use, st); break;
            }
        }
        return;
    }
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
    if (pl->tmode == SHX_TABLE_ONTHEFLY) {
        switch (pl->prec) {
            case SHX_FP32: an_mo_fields<1>(pl, G, cout, F, S, nmax_use, st); break;
            case SHX_SPLIT_BF16_2: an_mo_fields<2>(pl, G, cout, F, S, nmax_use, st); break;
            case SHX_SPLIT_BF16_3: an_mo_fields<3>(pl, G, cout, F, S, nmax_use, st); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
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
    // the tendency's 4-field FP32 synthesis regenerates P^m_n from 160
    // latitude pairs up also where the plan holds tables: there the FP32
    // table stream costs more than the recurrence (T255: 14.1 against 12.5
    // us), below it less (T127: 7.5 against 7.8)
    if (pl->tmode == SHX_TABLE_ONTHEFLY || (pl->prec == SHX_FP32 && pl->Jh >= 160)) {
        const long long cs = 3 * pl->nspec;
        switch (pl->prec) {
            case SHX_FP32: syn_mo<4, 1, 1>(pl, state, out, 4, 0, S, pl->nmax, cs, a, st); break;
            case SHX_SPLIT_BF16_2: syn_mo<4, 2, 1>(pl, state, out, 4, 0, S, pl->nmax, cs, a, st); break;
            case SHX_SPLIT_BF16_3: syn_mo<4, 3, 1>(pl, state, out, 4, 0, S, pl->nmax, cs, a, st); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (pl->prec) {
        case SHX_FP32: syn_mx<1, 1, true>(pl, state, out, 4, 0, 4, S, pl->nmax, st, a); break;
        case SHX_SPLIT_BF16_2: syn_mx<2, 1, true>(pl, state, out, 4, 0, 4, S, pl->nmax, st, a); break;
        case SHX_SPLIT_BF16_3: syn_mx<3, 1, true>(pl, state, out, 4, 0, 4, S, pl->nmax, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// the fused update uses the synthesis that regenerates P^m_n: every FP32
// plan (below 160 latitude pairs its table synthesis is a little faster
// alone, 7.5 against 7.8 us at T127, but not against the node-update launch
// that the fusion saves) and the plans without tables
bool leg_syn_mixed_swe_node_supported(const shx_plan* pl) {
    return pl->tmode == SHX_TABLE_ONTHEFLY || pl->prec == SHX_FP32;
}

hipError_t launch_leg_syn_mixed_swe_node(const shx_plan* pl, const NodeFuse& nf, double2* out, hipStream_t st) {
    if (!leg_syn_mixed_swe_node_supported(pl)) return hipErrorInvalidValue;
    switch (pl->prec) {
        case SHX_FP32: syn_mo<4, 1, 3>(pl, nullptr, out, 4, 0, 1, pl->nmax, 0, nf.p.a, st, nf); break;
        case SHX_SPLIT_BF16_2: syn_mo<4, 2, 3>(pl, nullptr, out, 4, 0, 1, pl->nmax, 0, nf.p.a, st, nf); break;
        case SHX_SPLIT_BF16_3: syn_mo<4, 3, 3>(pl, nullptr, out, 4, 0, 1, pl->nmax, 0, nf.p.a, st, nf); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_leg_syn_mixed(const shx_plan* pl, const double2* cin, double2* out, int F, int S, int nmax_use,
                                hipStream_t st) {
    if (pl->tmode == SHX_TABLE_ONTHEFLY) {
        switch (pl->prec) {
            case SHX_FP32: syn_mo_fields<1>(pl, cin, out, F, S, nmax_use, st); break;
            case SHX_SPLIT_BF16_2: syn_mo_fields<2>(pl, cin, out, F, S, nmax_use, st); break;
            case SHX_SPLIT_BF16_3: syn_mo_fields<3>(pl, cin, out, F, S, nmax_use, st); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
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
    if (pl->pan32) k_tab_to_f32<<<nb, 256, 0, st>>>(pl->pan, pl->pan32, pl->table_elems);
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
