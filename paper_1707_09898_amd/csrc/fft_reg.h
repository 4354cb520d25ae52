// Register-resident Stockham FFT for power-of-two lengths fixed at compile
// time.
//
// A line of length L is held by P = L / E threads; thread p holds the E
// elements x[p + P m], m = 0..E-1.  Every stage has a radix R dividing E and
// thread p computes the E / R butterflies j = p + P b, b = 0..E/R-1.  With
// this assignment the inputs of butterfly b are the thread's own elements
// m = b + r E/R, so the first stage needs no exchange, and the last stage's
// outputs land in the same register slots (x[p + P m] again, now in natural
// frequency order).  Between stages the outputs go through LDS.  Every twiddle
// depends only on (p, b, stage), so a thread loads its twiddles once, from the
// extended-precision table, and keeps them in registers.
#pragma once

#include "fft.h"

namespace regfft {

constexpr int ilog2c(int v)
{
    int n = 0;
    while (v > 1) v /= 2, ++n;
    return n;
}

// LDS slot of line position i: one pad slot per 32 complex keeps strided
// accesses from piling onto one bank.  A line occupies padded_len(L) slots,
// enough for every layout below; the pitch is 16 slots past a multiple of
// 32, so that kernels reading the same position of neighbouring lines spread
// over the banks.
__device__ __forceinline__ int swz(int i) { return i + (i >> 5); }
constexpr int padded_len(int L) { return (L + L / 8 + 31) / 32 * 32 + 16; }

// Layout of the exchange after stage S.  With E = 8 and a line of at least
// 16 lanes (16 lanes' 8-byte accesses fill the 32 four-byte banks), the
// exchange after the first stage writes 8 consecutive positions per lane
// (lanes 8 positions apart): one pad slot per 16 positions puts 16 lanes on
// 16 different bank pairs.  After the second stage it writes runs of 8
// lanes x 8 consecutive positions 64 positions apart: 8 pad slots per 64
// positions put consecutive runs half a bank row apart.  The reads
// (consecutive positions across lanes) stay conflict free, and a lane's 8
// outputs stay contiguous, so the paired LDS writes keep their immediate
// offsets.  Measured: 4x fewer bank-conflict cycles in the fused kernels.
template <int L, int E, int S>
__device__ __forceinline__ int swz_x(int i)
{
    constexpr int P = L / E;
    if constexpr (E == 8 && P >= 16 && S == 0) return i + (i >> 4);
    else if constexpr (E == 8 && P >= 16 && S == 1) return i + 8 * (i >> 6);
    else return swz(i);
}

// number of full radix-E stages, and the total stage count
constexpr int full_stages(int L, int E) { return ilog2c(L) / ilog2c(E); }
constexpr int last_radix(int L, int E) { return L >> (full_stages(L, E) * ilog2c(E)); }
constexpr int num_stages(int L, int E) { return full_stages(L, E) + (last_radix(L, E) > 1 ? 1 : 0); }
constexpr int stage_radix(int L, int E, int s) { return s < full_stages(L, E) ? E : last_radix(L, E); }
constexpr int stage_ns(int L, int E, int s)
{
    int n = 1;   // a loop, not recursion: always inlined where it is not folded
    for (int q = 0; q < s; ++q) n *= stage_radix(L, E, q);
    return n;
}
// twiddle slots (complex) a thread keeps: stages 1.. need (E/R)(R-1) each
constexpr int twiddle_count(int L, int E)
{
    int n = 0;
    for (int s = 1; s < num_stages(L, E); ++s) n += (E / stage_radix(L, E, s)) * (stage_radix(L, E, s) - 1);
    return n;
}

// Ordering of the exchange through LDS.  A line whose P threads lie in one
// wave (threads l P .. l P + P - 1 with P dividing 64) needs no block
// barrier: a wave's LDS accesses are performed in issue order, so a fence
// that keeps the compiler from reordering them is enough, and the waves of a
// block then run their lines independently.  Lines spread over several waves
// use the block barrier.
template <bool WAVE>
__device__ __forceinline__ void exchange_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <typename R>
__device__ __forceinline__ void dft16(cplx<R> *v, bool inv)
{
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle w16^(n2 k1), DFT4 over n2
    const R c1 = (R)0.92387953251128675612818318939678828682;   // cos(pi/8)
    const R s1 = (R)0.38268343236508977172845998403039886676;   // sin(pi/8)
    const R h = (R)0.70710678118654752440084436210484903928;
    cplx<R> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cplx<R> x0 = v[n2], x1 = v[n2 + 4], x2 = v[n2 + 8], x3 = v[n2 + 12];
        dft4(x0, x1, x2, x3, inv);
        a[n2][0] = x0; a[n2][1] = x1; a[n2][2] = x2; a[n2][3] = x3;
    }
    // w16^e for e = n2 k1 in {0..9}; forward exp(-i pi e / 8), inverse conj
    const R sg = inv ? (R)1 : (R)-1;
    auto tw = [&](cplx<R> x, int e) -> cplx<R> {
        R c, s;
        switch (e) {
        case 0: return x;
        case 1: c = c1; s = s1; break;
        case 2: c = h; s = h; break;
        case 3: c = s1; s = c1; break;
        case 4: c = 0; s = 1; break;
        case 6: c = -h; s = h; break;
        default: c = -c1; s = -s1; break;   // e = 9: cos(9pi/8), sin(9pi/8)
        }
        s *= sg;
        return cplx<R>{x.x * c - x.y * s, x.x * s + x.y * c};
    };
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) a[n2][k1] = tw(a[n2][k1], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<R> y0 = a[0][k1], y1 = a[1][k1], y2 = a[2][k1], y3 = a[3][k1];
        dft4(y0, y1, y2, y3, inv);
        v[k1] = y0; v[k1 + 4] = y1; v[k1 + 8] = y2; v[k1 + 12] = y3;
    }
}

// ZIN: the upper half u[RAD/2 ..] is zero (its contents are ignored).
template <typename R, int RAD, bool ZIN = false>
__device__ __forceinline__ void dft_pow2(cplx<R> *u, bool inv)
{
    if constexpr (ZIN && RAD != 8) {
#pragma unroll
        for (int r = RAD / 2; r < RAD; ++r) u[r] = cplx<R>{0, 0};
    }
    if constexpr (RAD == 2) dft2(u);
    else if constexpr (RAD == 4) dft4(u[0], u[1], u[2], u[3], inv);
    else if constexpr (RAD == 8) dft8<R, ZIN>(u, inv);
    else dft16(u, inv);
}

// Per-thread twiddles of line position p: for each stage s >= 1 and
// butterfly b, w_{Ns R}^{r ((p + P b) mod Ns)} for r = 1..R-1.
template <typename R, int L, int E>
__device__ __forceinline__ void load_twiddles(const cplx<R> *table, int p, cplx<R> *tw)
{
    constexpr int P = L / E;
    constexpr int NS = num_stages(L, E);
    int at = 0;
#pragma unroll
    for (int s = 1; s < NS; ++s) {
        const int Rr = stage_radix(L, E, s);
        const int Ns = stage_ns(L, E, s);
        const int step = L / (Ns * Rr);
#pragma unroll
        for (int b = 0; b < E / Rr; ++b) {
            const int k = (p + P * b) & (Ns - 1);
#pragma unroll
            for (int r = 1; r < Rr; ++r) tw[at++] = table[(k * r * step) & (L - 1)];
        }
    }
}

// One stage S of the transform (S = 0 .. num_stages - 1), then the rest.
// ZIN: the line's upper half (positions L/2 .., slots m >= E/2) is zero on
// entry; the first stage, whose butterflies take slots m and m + E/2 of the
// thread, then skips that half.
template <typename R, int L, int E, int S, bool WAVE, bool ZIN = false>
__device__ __forceinline__ void fft_stages(cplx<R> *v, const cplx<R> *tw, cplx<R> *lds, int p, bool inv)
{
    constexpr int P = L / E;
    constexpr int NS = num_stages(L, E);
    if constexpr (S < NS) {
        constexpr int Rr = stage_radix(L, E, S);
        constexpr int Ns = stage_ns(L, E, S);
        constexpr bool last = (S == NS - 1);
        // twiddle slots used by the stages before S
        constexpr int at = [] {
            int n = 0;
            for (int q = 1; q < S; ++q) n += (E / stage_radix(L, E, q)) * (stage_radix(L, E, q) - 1);
            return n;
        }();
#pragma unroll
        for (int b = 0; b < E / Rr; ++b) {
            cplx<R> u[Rr];
#pragma unroll
            for (int r = 0; r < Rr; ++r) u[r] = v[b + r * (E / Rr)];
            if constexpr (S > 0) {
#pragma unroll
                for (int r = 1; r < Rr; ++r) {
                    cplx<R> w = tw[at + b * (Rr - 1) + (r - 1)];
                    if (inv) w.y = -w.y;
                    u[r] = cmul(u[r], w);
                }
            }
            dft_pow2<R, Rr, ZIN && S == 0>(u, inv);
            if constexpr (last) {
#pragma unroll
                for (int r = 0; r < Rr; ++r) v[b + r * (E / Rr)] = u[r];
            } else {
                const int j = p + P * b;
                const int base = (j / Ns) * (Ns * Rr) + (j & (Ns - 1));
#pragma unroll
                for (int r = 0; r < Rr; ++r) lds[swz_x<L, E, S>(base + r * Ns)] = u[r];
            }
        }
        if constexpr (!last) {
            exchange_sync<WAVE>();
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds[swz_x<L, E, S>(p + P * m)];
            exchange_sync<WAVE>();
            fft_stages<R, L, E, S + 1, WAVE, ZIN>(v, tw, lds, p, inv);
        }
    }
}

// NV independent lines at once (line j: v[j][m], exchange area lds + j
// area): each stage runs for all lines between the same two syncs, which
// halves the syncs per line and gives the scheduler independent work.
template <typename R, int L, int E, int S, int NV, bool WAVE, bool ZIN = false>
__device__ __forceinline__ void fft_stages_n(cplx<R> (*v)[E], const cplx<R> *tw, cplx<R> *lds, int area, int p,
                                             bool inv)
{
    constexpr int P = L / E;
    constexpr int NS = num_stages(L, E);
    if constexpr (S < NS) {
        constexpr int Rr = stage_radix(L, E, S);
        constexpr int Ns = stage_ns(L, E, S);
        constexpr bool last = (S == NS - 1);
        constexpr int at = [] {
            int n = 0;
            for (int q = 1; q < S; ++q) n += (E / stage_radix(L, E, q)) * (stage_radix(L, E, q) - 1);
            return n;
        }();
#pragma unroll
        for (int j = 0; j < NV; ++j) {
#pragma unroll
            for (int b = 0; b < E / Rr; ++b) {
                cplx<R> u[Rr];
#pragma unroll
                for (int r = 0; r < Rr; ++r) u[r] = v[j][b + r * (E / Rr)];
                if constexpr (S > 0) {
#pragma unroll
                    for (int r = 1; r < Rr; ++r) {
                        cplx<R> w = tw[at + b * (Rr - 1) + (r - 1)];
                        if (inv) w.y = -w.y;
                        u[r] = cmul(u[r], w);
                    }
                }
                dft_pow2<R, Rr, ZIN && S == 0>(u, inv);
                if constexpr (last) {
#pragma unroll
                    for (int r = 0; r < Rr; ++r) v[j][b + r * (E / Rr)] = u[r];
                } else {
                    const int jj = p + P * b;
                    const int base = (jj / Ns) * (Ns * Rr) + (jj & (Ns - 1));
#pragma unroll
                    for (int r = 0; r < Rr; ++r) lds[j * area + swz_x<L, E, S>(base + r * Ns)] = u[r];
                }
            }
        }
        if constexpr (!last) {
            exchange_sync<WAVE>();
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int m = 0; m < E; ++m) v[j][m] = lds[j * area + swz_x<L, E, S>(p + P * m)];
            exchange_sync<WAVE>();
            fft_stages_n<R, L, E, S + 1, NV, WAVE, ZIN>(v, tw, lds, area, p, inv);
        }
    }
}

template <typename R, int L, int E, int NV, bool WAVE = false, bool ZIN = false>
__device__ __forceinline__ void fft_lines(cplx<R> (*v)[E], const cplx<R> *tw, cplx<R> *lds, int area, int p, bool inv)
{
    static_assert(!WAVE || 64 % (L / E) == 0, "a wave-synchronized line must lie inside one wave");
    static_assert(!ZIN || stage_radix(L, E, 0) == E, "the zero half is skipped in a first stage of radix E");
    fft_stages_n<R, L, E, 0, NV, WAVE, ZIN>(v, tw, lds, area, p, inv);
}

// Transform one line held as v[m] = x[p + P m] by thread p.  `lds` is this
// line's exchange area (padded_len(L) complex; position i at swz(i)).  With
// WAVE false all threads of the block call it together (it contains block
// barriers); with WAVE true the line's threads must be P consecutive threads
// of one wave (see exchange_sync).  On return v[m] holds X[p + P m].
// Forward: exp(-2 pi i jk/L); inverse: exp(+2 pi i jk/L), unscaled.
// With ZIN the caller asserts that v[m] = 0 for m >= E/2 (the line's upper
// half); those slots are then not read.
template <typename R, int L, int E, bool WAVE = false, bool ZIN = false>
__device__ __forceinline__ void fft_line(cplx<R> *v, const cplx<R> *tw, cplx<R> *lds, int p, bool inv)
{
    static_assert(!WAVE || 64 % (L / E) == 0, "a wave-synchronized line must lie inside one wave");
    static_assert(!ZIN || stage_radix(L, E, 0) == E, "the zero half is skipped in a first stage of radix E");
    fft_stages<R, L, E, 0, WAVE, ZIN>(v, tw, lds, p, inv);
}

}  // namespace regfft
