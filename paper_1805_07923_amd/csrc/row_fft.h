// Real latitude-row FFTs in LDS, shared by the transform, tendency and
// adjoint kernels (the longitude sums of eq. fourier_transform and eq.
// spectral_to_physical_space).
//
// A real row of length L (2^k or 3 * 2^k) goes through a complex FFT of
// length L2 = L/2 of z_k = x_{2k} + i x_{2k+1}:
//   synthesis:  Z_m = (X_m + conj X_{L2-m}) + i e^{2 pi i m / L} (X_m - conj X_{L2-m}),
//               z = sum_m Z_m e^{2 pi i m k / L2}  ->  x_{2k} = Re z_k, x_{2k+1} = Im z_k;
//   analysis:   Z = FFT_{L2}(z),  E_m = (Z_m + conj Z_{-m}) / 2,  O_m = (Z_m - conj Z_{-m}) / (2 i),
//               X_m = E_m + e^{-2 pi i m / L} O_m.
// The complex FFT is a Stockham transform in LDS with radix-8 stages first,
// then one stage of radix 6, 4, 3 or 2 as the remaining length requires (384 =
// 8 8 6, 1536 = 8 8 8 3).  Each stage loads its butterflies into registers
// and writes them to a second LDS buffer (one barrier per stage) while the
// workgroup's LDS stays under PP_LDS_MAX, or back in place after a barrier.
// Twiddles e^{-2 pi i t / L},
// t < L2, come from a table computed on the host in quad precision and copied
// to LDS; e^{-2 pi i t / L2} is entry 2t, and the upper half of the circle is
// the negated lower half.
#pragma once
#include <hip/hip_runtime.h>

namespace rowfft {

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
    const double2 r3 = make_double2(-sg * s3.y, sg * s3.x);   // sg * i * s3
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

// Radix 6 and 8 by one radix-2 split (decimation in frequency) into two
// DFTs of size 3 or 4: X_{2k} = DFT(x_j + x_{j+R/2}), X_{2k+1} =
// DFT((x_j - x_{j+R/2}) w_R^j), w_R = e^{sg 2 pi i / R}.
template <>
__device__ __forceinline__ void dft<6>(double2* v, double sg) {
    const double c = 0.86602540378443864676;   // sin(2 pi / 3)
    double2 a[3], b[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        a[j] = make_double2(v[j].x + v[j + 3].x, v[j].y + v[j + 3].y);
        b[j] = make_double2(v[j].x - v[j + 3].x, v[j].y - v[j + 3].y);
    }
    b[1] = cmul(b[1], make_double2(0.5, sg * c));
    b[2] = cmul(b[2], make_double2(-0.5, sg * c));
    dft<3>(a, sg);
    dft<3>(b, sg);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[2 * k] = a[k];
        v[2 * k + 1] = b[k];
    }
}

template <>
__device__ __forceinline__ void dft<8>(double2* v, double sg) {
    const double h = 0.70710678118654752440;   // sqrt(1/2)
    double2 a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j] = make_double2(v[j].x + v[j + 4].x, v[j].y + v[j + 4].y);
        b[j] = make_double2(v[j].x - v[j + 4].x, v[j].y - v[j + 4].y);
    }
    b[1] = make_double2(h * (b[1].x - sg * b[1].y), h * (b[1].y + sg * b[1].x));
    b[2] = make_double2(-sg * b[2].y, sg * b[2].x);
    b[3] = make_double2(h * (-b[3].x - sg * b[3].y), h * (-b[3].y + sg * b[3].x));
    dft<4>(a, sg);
    dft<4>(b, sg);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = a[k];
        v[2 * k + 1] = b[k];
    }
}

// Radix of the next stage for a remaining length rem.
__host__ __device__ constexpr int next_radix(int rem) {
    return rem % 8 == 0 ? 8 : (rem == 6 ? 6 : (rem % 4 == 0 ? 4 : (rem % 2 == 0 ? 2 : 3)));
}
// Number of stages of a length-C transform.
__host__ __device__ constexpr int stage_count(int C) {
    int n = 0;
    for (int rem = C; rem > 1; rem /= next_radix(rem)) ++n;
    return n;
}

// e^{-2 pi i idx / (2 half)} from the half table tws[0..half).
__device__ __forceinline__ double2 tw_half(const double2* tws, int idx, int half) {
    const double2 w = tws[idx < half ? idx : idx - half];
    return idx < half ? w : make_double2(-w.x, -w.y);
}

// Padded LDS row layout: one spare element after every 16, so that the
// strided butterfly writes of a stage (stride R elements for the first
// stage) spread over the LDS banks instead of piling onto a few of them.
// A row of C complex values takes padded(C) slots; element i sits at pidx(i).
__host__ __device__ constexpr int padded(int C) { return C + C / 16; }
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// Largest LDS footprint (bytes per workgroup) for which a row kernel keeps a
// second set of row buffers for ping-pong stages.  Measured on the 768-point
// tendency rows (384 workgroups): 71 KB with ping-pong ran 18.1 us, the same
// kernel in place with 38.8 KB 14.0 us, and the in-place kernel padded with
// unused LDS to 57 KB or 71 KB again 18.8 us: fewer resident workgroups per
// CU cost more than the barriers that the second buffer saves.
constexpr int PP_LDS_MAX = 40 * 1024;

// Launch shape for real rows of length L: T threads per workgroup, one per
// complex point of the half-length FFT (at least 64, at most 1024).
template <int L>
struct Cfg {
    static constexpr int L2 = L / 2;
    static constexpr int T0 = L2 < 64 ? 64 : (L2 > 1024 ? 1024 : L2);
    static constexpr int T = (T0 + 63) / 64 * 64;
};

// One Stockham stage for NR complex rows of length C (padded rows), T
// threads; Ns is the length of the sub-transforms already done.  tws is the
// LDS twiddle table of the real length 2C (C entries).  Reads src; writes dst
// (dst == src: in place, with a barrier between the reads and the writes).
template <int C, int T, int NR, int Ns>
__device__ __forceinline__ void stage(const double2* src, double2* dst, const double2* tws, double sg) {
    constexpr int R = next_radix(C / Ns);
    constexpr int NB = C / R;
    constexpr int ITEMS = NR * NB;
    constexpr int IPT = (ITEMS + T - 1) / T;
    constexpr int TWS = C / (Ns * R) * 2;
    double2 v[IPT][R];
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int item = threadIdx.x + it * T;
        if (ITEMS % T == 0 || item < ITEMS) {
            const int row = item / NB, j = item - row * NB, k = j % Ns;
            const double2* b = src + row * padded(C);
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = b[pidx(j + r * NB)];
            if constexpr (Ns > 1) {
                // twiddles as powers of one table value (as in wstage)
                double2 w[R];
                w[1] = tw_half(tws, k * TWS, C);
                w[1].y *= -sg;
#pragma unroll
                for (int r = 2; r < R; ++r) w[r] = (r % 2 == 0) ? cmul(w[r / 2], w[r / 2]) : cmul(w[r - 1], w[1]);
#pragma unroll
                for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], w[r]);
            }
            dft<R>(v[it], sg);
        }
    }
    if (src == dst) __syncthreads();
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int item = threadIdx.x + it * T;
        if (ITEMS % T == 0 || item < ITEMS) {
            const int row = item / NB, j = item - row * NB, k = j % Ns;
            const int base = (j / Ns) * Ns * R + k;
            double2* b = dst + row * padded(C);
#pragma unroll
            for (int q = 0; q < R; ++q) b[pidx(base + q * Ns)] = v[it][q];
        }
    }
    __syncthreads();
}

// All stages in place in buf.
template <int C, int T, int NR, int Ns>
__device__ __forceinline__ void stages(double2* buf, const double2* tws, double sg) {
    if constexpr (C / Ns > 1) {
        stage<C, T, NR, Ns>(buf, buf, tws, sg);
        stages<C, T, NR, Ns * next_radix(C / Ns)>(buf, tws, sg);
    }
}

// All stages between two buffers (a holds the input); the result ends in a
// when the stage count is even, else in b.
template <int C, int T, int NR, int Ns>
__device__ __forceinline__ void stages_pp(double2* a, double2* b, const double2* tws, double sg) {
    if constexpr (C / Ns > 1) {
        stage<C, T, NR, Ns>(a, b, tws, sg);
        stages_pp<C, T, NR, Ns * next_radix(C / Ns)>(b, a, tws, sg);
    }
}

// FFT of NR rows held in a; with PP the second buffer b is used and the
// returned pointer says where the result is.
template <int C, int T, int NR, bool PP>
__device__ __forceinline__ double2* fft(double2* a, double2* b, const double2* tws, double sg) {
    if constexpr (PP) {
        stages_pp<C, T, NR, 1>(a, b, tws, sg);
        return (stage_count(C) % 2 == 0) ? a : b;
    } else {
        stages<C, T, NR, 1>(a, tws, sg);
        return a;
    }
}

// Synthesis input of NR real rows of length L: Z_m of row f at
// rows[f * padded(L2) + pidx(m)], and the LDS twiddle table tws[0..L2) from the global table twg.  The
// coefficients X_m (m <= N < L2; zero above N, Im X_0 ignored) come from
// coef(f, m).  Thread t owns the index pairs (m, L2 - m), m = t, t + T, ...
// < L2/2; the pair of m = 0 is the middle index L2/2 (e^{2 pi i (L2/2) / L} = i,
// so Z_{L2/2} = 2 conj X_{L2/2}).  Every coefficient is read once, and all
// global loads of a thread are issued before any of them is used.  Caller
// syncs.
template <int L, int NR, class Coef>
__device__ __forceinline__ void pack_rows(double2* rows, double2* tws, const double2* __restrict__ twg, int N,
                                          Coef coef) {
    constexpr int L2 = L / 2, H = L2 / 2, T = Cfg<L>::T, P = padded(L2);
    constexpr int IP = (H + T - 1) / T;
    constexpr int ITW = (L2 + T - 1) / T;
    double2 twv[ITW];
#pragma unroll
    for (int it = 0; it < ITW; ++it) {
        const int t = threadIdx.x + it * T;
        if (t < L2) twv[it] = twg[t];
    }
    double2 xa[IP][NR], xb[IP][NR];
#pragma unroll
    for (int ip = 0; ip < IP; ++ip) {
        const int m = threadIdx.x + ip * T;
        const int j = (m == 0) ? H : L2 - m;
        const bool on = m < H;
        const bool ina = on && m <= N, inb = on && j <= N;
        // unconditional loads from a valid index, then select: every load of
        // the thread is issued before the first one is waited for
        const int ma = ina ? m : 0, jb = inb ? j : 0;
#pragma unroll
        for (int f = 0; f < NR; ++f) {
            const double2 va = coef(f, ma), vb = coef(f, jb);
            xa[ip][f] = ina ? va : make_double2(0.0, 0.0);
            xb[ip][f] = inb ? vb : make_double2(0.0, 0.0);
        }
    }
#pragma unroll
    for (int it = 0; it < ITW; ++it) {
        const int t = threadIdx.x + it * T;
        if (t < L2) tws[t] = twv[it];
    }
#pragma unroll
    for (int ip = 0; ip < IP; ++ip) {
        const int m = threadIdx.x + ip * T, j = L2 - m;
        if (m >= H) continue;
        if (m == 0) {
#pragma unroll
            for (int f = 0; f < NR; ++f) {
                const double a = xa[ip][f].x;                  // Z_0 = X_0 + i X_0, X_0 real
                rows[f * P] = make_double2(a, a);
                rows[f * P + pidx(H)] = make_double2(2.0 * xb[ip][f].x, -2.0 * xb[ip][f].y);
            }
            continue;
        }
        // twv[ip] = tw[m] (same index as the twiddle copy); e^{+2 pi i m / L} =
        // conj(tw[m]), e^{+2 pi i j / L} = -tw[m]
        const double2 tm = twv[ip];
        const double2 em = make_double2(tm.x, -tm.y);
        const double2 ej = make_double2(-tm.x, -tm.y);
#pragma unroll
        for (int f = 0; f < NR; ++f) {
            const double2 A = xa[ip][f], B = xb[ip][f];
            {   // Z_m, partner conj X_j
                const double2 s = make_double2(A.x + B.x, A.y - B.y);
                const double2 d = make_double2(A.x - B.x, A.y + B.y);
                const double2 ed = cmul(em, d);
                rows[f * P + pidx(m)] = make_double2(s.x - ed.y, s.y + ed.x);
            }
            {   // Z_j, partner conj X_m
                const double2 s = make_double2(B.x + A.x, B.y - A.y);
                const double2 d = make_double2(B.x - A.x, B.y + A.y);
                const double2 ed = cmul(ej, d);
                rows[f * P + pidx(j)] = make_double2(s.x - ed.y, s.y + ed.x);
            }
        }
    }
}

// X_m (m <= N) of the real row whose half-length FFT is in `row` (padded).
template <int L>
__device__ __forceinline__ double2 unpack(const double2* row, const double2* tws, int m) {
    constexpr int L2 = L / 2;
    const double2 z = row[pidx(m)];
    const double2 zc = row[pidx((L2 - m) % L2)];
    const double2 E = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
    const double2 O = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    const double2 wo = cmul(tws[m], O);
    return make_double2(E.x + wo.x, E.y + wo.y);
}

// ------------------------------------------------ one row per wavefront
// The same transforms with one wavefront owning one row: the stages of a row
// then need no workgroup barrier, only the wavefront's own LDS accesses in
// program order (a wavefront's LDS instructions are executed in the order
// issued; the fence keeps the compiler from moving a store of one lane's
// butterfly above a load of another lane's, which it could otherwise do
// where it proves that one lane's own addresses do not overlap).
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// One Stockham stage of a row of C complex values (padded), in place, by the
// 64 lanes of one wavefront; Ns as in stage().
template <int C, int Ns>
__device__ __forceinline__ void wstage(double2* row, const double2* tws, double sg, int lane) {
    constexpr int R = next_radix(C / Ns);
    constexpr int NB = C / R;
    constexpr int IPT = (NB + 63) / 64;
    constexpr int TWS = C / (Ns * R) * 2;
    double2 v[IPT][R];
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int j = lane + it * 64, k = j % Ns;
        if (NB % 64 == 0 || j < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = row[pidx(j + r * NB)];
            if constexpr (Ns > 1) {
                // twiddles w^r, r = 1..R-1, as powers of the one table value
                // w = e^{-+2 pi i k TWS / (2 C)} (squares and one product per
                // step), so that a stage reads one twiddle from LDS, not R - 1
                double2 w[R];
                w[1] = tw_half(tws, k * TWS, C);
                w[1].y *= -sg;
#pragma unroll
                for (int r = 2; r < R; ++r) w[r] = (r % 2 == 0) ? cmul(w[r / 2], w[r / 2]) : cmul(w[r - 1], w[1]);
#pragma unroll
                for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], w[r]);
            }
            dft<R>(v[it], sg);
        }
    }
    wave_fence();
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int j = lane + it * 64, k = j % Ns;
        if (NB % 64 == 0 || j < NB) {
            const int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) row[pidx(base + q * Ns)] = v[it][q];
        }
    }
    wave_fence();
}

// All stages of one row, in place, by one wavefront.
template <int C, int Ns = 1>
__device__ __forceinline__ void wfft(double2* row, const double2* tws, double sg, int lane) {
    if constexpr (C / Ns > 1) {
        wstage<C, Ns>(row, tws, sg, lane);
        wfft<C, Ns * next_radix(C / Ns)>(row, tws, sg, lane);
    }
}

// Synthesis input of one real row by one wavefront (pack_rows for a single
// row): lane l owns the index pairs (m, L2 - m), m = l, l + 64, ... < L2/2.
// coef(m) gives X_m (called for m <= N only); twg is the global twiddle table.
// Every load of the lane is issued before the first is used.
template <int L, class Coef>
__device__ __forceinline__ void wpack(double2* row, const double2* __restrict__ twg, int N, int lane, Coef coef) {
    constexpr int L2 = L / 2, H = L2 / 2;
    constexpr int IP = (H + 63) / 64;
    double2 xa[IP], xb[IP], tm[IP];
#pragma unroll
    for (int ip = 0; ip < IP; ++ip) {
        const int m = lane + ip * 64;
        const int j = (m == 0) ? H : L2 - m;
        const bool on = m < H;
        const bool ina = on && m <= N, inb = on && j <= N;
        const double2 va = coef(ina ? m : 0), vb = coef(inb ? j : 0);
        tm[ip] = twg[on ? m : 0];
        xa[ip] = ina ? va : make_double2(0.0, 0.0);
        xb[ip] = inb ? vb : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int ip = 0; ip < IP; ++ip) {
        const int m = lane + ip * 64, j = L2 - m;
        if (m >= H) continue;
        const double2 A = xa[ip], B = xb[ip];
        if (m == 0) {
            row[0] = make_double2(A.x, A.x);                    // Z_0 = X_0 + i X_0, X_0 real
            row[pidx(H)] = make_double2(2.0 * B.x, -2.0 * B.y);
            continue;
        }
        const double2 em = make_double2(tm[ip].x, -tm[ip].y);  // e^{+2 pi i m / L}
        const double2 ej = make_double2(-tm[ip].x, -tm[ip].y); // e^{+2 pi i j / L}
        {
            const double2 s = make_double2(A.x + B.x, A.y - B.y);
            const double2 d = make_double2(A.x - B.x, A.y + B.y);
            const double2 ed = cmul(em, d);
            row[pidx(m)] = make_double2(s.x - ed.y, s.y + ed.x);
        }
        {
            const double2 s = make_double2(B.x + A.x, B.y - A.y);
            const double2 d = make_double2(B.x - A.x, B.y + A.y);
            const double2 ed = cmul(ej, d);
            row[pidx(j)] = make_double2(s.x - ed.y, s.y + ed.x);
        }
    }
    wave_fence();
}

}  // namespace rowfft
