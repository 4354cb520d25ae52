// Device FFT building blocks for the padded convolution: complex type, small
// DFT butterflies and a mixed-radix Stockham autosort FFT over lines staged in
// LDS.  Radices 2, 3, 4, 5, 7, 8 cover every 7-smooth padded length.
//
// Stockham stage with radix R after a product Ns of earlier radices (Ns = 1
// for the first stage): butterfly j in [0, L/R) reads the R inputs
// x[j + r L/R], multiplies input r by w_{Ns R}^{r (j mod Ns)}, applies an
// R-point DFT and writes output r to y[(j / Ns) Ns R + (j mod Ns) + r Ns].
// After the last stage the line holds the DFT in natural order.  Twiddles come
// from a table of w_L^k = exp(-2 pi i k / L), computed in extended precision on
// the host and rounded once (no recurrences).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename R>
__device__ __forceinline__ cplx<R> mul_mi(cplx<R> a, bool inv)
{
    return inv ? cplx<R>{-a.y, a.x} : cplx<R>{a.y, -a.x};
}

#define TOF_MAX_STAGES 16

// One FFT length: radix sequence and twiddle table (device, cplx<R>[L]).
struct FftPlanDev {
    int L;
    int nst;
    int radix[TOF_MAX_STAGES];
    const void *tw;
};

template <typename R>
__device__ __forceinline__ void dft2(cplx<R> *v)
{
    cplx<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename R>
__device__ __forceinline__ void dft4(cplx<R> &a0, cplx<R> &a1, cplx<R> &a2, cplx<R> &a3, bool inv)
{
    cplx<R> t0 = cadd(a0, a2), t1 = csub(a0, a2);
    cplx<R> t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3), inv);
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// ZIN: v[4..7] are zero (not read), so the first layer reduces to copies.
template <typename R, bool ZIN = false>
__device__ __forceinline__ void dft8(cplx<R> *v, bool inv)
{
    // X[2k] = DFT4(v_n + v_{n+4}), X[2k+1] = DFT4(w8^n (v_n - v_{n+4}))
    const R h = (R)0.70710678118654752440084436210484903928;
    cplx<R> a[4], b[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        if constexpr (ZIN) {
            a[n] = v[n];
            b[n] = v[n];
        } else {
            a[n] = cadd(v[n], v[n + 4]);
            b[n] = csub(v[n], v[n + 4]);
        }
    }
    // w8 = (1 - i)/sqrt2 forward, (1 + i)/sqrt2 inverse
    b[1] = inv ? cplx<R>{(b[1].x - b[1].y) * h, (b[1].x + b[1].y) * h}
               : cplx<R>{(b[1].x + b[1].y) * h, (b[1].y - b[1].x) * h};
    b[2] = mul_mi(b[2], inv);
    b[3] = inv ? cplx<R>{-(b[3].x + b[3].y) * h, (b[3].x - b[3].y) * h}
               : cplx<R>{(b[3].y - b[3].x) * h, -(b[3].x + b[3].y) * h};
    dft4(a[0], a[1], a[2], a[3], inv);
    dft4(b[0], b[1], b[2], b[3], inv);
    v[0] = a[0]; v[2] = a[1]; v[4] = a[2]; v[6] = a[3];
    v[1] = b[0]; v[3] = b[1]; v[5] = b[2]; v[7] = b[3];
}

// cos and sin of 2 pi m / P for the odd-prime butterflies
struct PrimeTable {
    double c[7], s[7];
};
__device__ __constant__ static const PrimeTable kPrime3 = {
    {1.0, -0.5, -0.5, 0, 0, 0, 0},
    {0.0, 0.866025403784438646763723170752936183, -0.866025403784438646763723170752936183, 0, 0, 0, 0}};
__device__ __constant__ static const PrimeTable kPrime5 = {
    {1.0, 0.309016994374947424102293417182819059, -0.809016994374947424102293417182819059,
     -0.809016994374947424102293417182819059, 0.309016994374947424102293417182819059, 0, 0},
    {0.0, 0.951056516295153572116439333379382143, 0.587785252292473129168705954639072769,
     -0.587785252292473129168705954639072769, -0.951056516295153572116439333379382143, 0, 0}};
__device__ __constant__ static const PrimeTable kPrime7 = {
    {1.0, 0.623489801858733530525004884004239811, -0.222520933956314404288902564496794759,
     -0.900968867902419126236102319507445051, -0.900968867902419126236102319507445051,
     -0.222520933956314404288902564496794759, 0.623489801858733530525004884004239811},
    {0.0, 0.78183148246802980870844452667405775, 0.974927912181823607018131682993931217,
     0.433883739117558120475768332848358755, -0.433883739117558120475768332848358755,
     -0.974927912181823607018131682993931217, -0.78183148246802980870844452667405775}};

// Direct odd-prime DFT, X[k] = sum_n v[n] exp(-+ 2 pi i n k / P).
template <typename R, int P>
__device__ __forceinline__ void dft_prime(cplx<R> *v, bool inv, const PrimeTable &t)
{
    cplx<R> in[P];
#pragma unroll
    for (int n = 0; n < P; ++n) in[n] = v[n];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        cplx<R> acc = in[0];
#pragma unroll
        for (int n = 1; n < P; ++n) {
            const int m = (n * k) % P;
            const R c = (R)t.c[m];
            const R s = inv ? (R)t.s[m] : (R)-t.s[m];
            acc.x += in[n].x * c - in[n].y * s;
            acc.y += in[n].x * s + in[n].y * c;
        }
        v[k] = acc;
    }
}

template <typename R>
__device__ __forceinline__ void dft_any(cplx<R> *v, int r, bool inv)
{
    switch (r) {
    case 2: dft2(v); break;
    case 3: dft_prime<R, 3>(v, inv, kPrime3); break;
    case 4: dft4(v[0], v[1], v[2], v[3], inv); break;
    case 5: dft_prime<R, 5>(v, inv, kPrime5); break;
    case 7: dft_prime<R, 7>(v, inv, kPrime7); break;
    default: dft8(v, inv); break;
    }
}

// Transform `nlines` lines of length plan.L held in LDS at a[line * pitch + i].
// b is scratch of the same shape.  Returns the buffer holding the result (a or
// b).  All threads of the block must call it; it ends with a barrier.
template <typename R>
__device__ cplx<R> *fft_lines_lds(cplx<R> *a, cplx<R> *b, int nlines, int pitch,
                                  const FftPlanDev &plan, bool inv)
{
    const int L = plan.L;
    const cplx<R> *tw = (const cplx<R> *)plan.tw;
    const int nthr = blockDim.x;
    int Ns = 1;
    for (int s = 0; s < plan.nst; ++s) {
        const int Rr = plan.radix[s];
        const int nb = L / Rr;
        const int twstep = L / (Ns * Rr);
        const int total = nlines * nb;
        for (int idx = threadIdx.x; idx < total; idx += nthr) {
            const int line = idx / nb;
            const int j = idx - line * nb;
            const int k = j % Ns;
            const cplx<R> *src = a + line * pitch;
            cplx<R> v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if (r < Rr) v[r] = src[j + r * nb];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < 8; ++r)
                    if (r < Rr) {
                        cplx<R> w = tw[k * r * twstep];
                        if (inv) w.y = -w.y;
                        v[r] = cmul(v[r], w);
                    }
            }
            dft_any(v, Rr, inv);
            cplx<R> *dst = b + line * pitch + (j / Ns) * Ns * Rr + k;
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if (r < Rr) dst[r * Ns] = v[r];
        }
        __syncthreads();
        cplx<R> *t = a;
        a = b;
        b = t;
        Ns *= Rr;
    }
    return a;
}
