// Device helpers shared by the pass kernels (kernels.hip) and the fused
// y-transform / z-sum kernels (yzsum.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "engine.h"
#include "fft.h"

namespace tofdev {

// v with its sign bit flipped where the mask's top bit is set (exact
// multiplication by -1 without a branch on the value)
__device__ __forceinline__ float flip_sign(float v, unsigned m) { return __uint_as_float(__float_as_uint(v) ^ m); }
__device__ __forceinline__ double flip_sign(double v, unsigned m)
{
    return __hiloint2double(__double2hiint(v) ^ (int)m, __double2loint(v));
}
constexpr unsigned kSignBit = 0x80000000u;

// Line index of the calling thread when P threads share a line.  With P a
// multiple of the wave size every wave lies inside one line, so the index is
// made wave-uniform (scalar registers: row pointers need no per-lane math).
template <int P>
__device__ __forceinline__ int line_of_thread()
{
    const int l = threadIdx.x / P;
    if constexpr (P % 64 == 0) return __builtin_amdgcn_readfirstlane(l);
    return l;
}

// Parity class of the product's tensor components.  With kParRuntime each
// component's parity is read from prod.comp (or is q itself when all six are
// used); kParEven fixes at compile time that the single component is a
// diagonal one (xx, yy or zz: even in x, y and z), so its Kt values are real
// and need no sign flips.
constexpr int kParRuntime = -1;
constexpr int kParEven = 0;

template <int NC, int PAR>
__device__ __forceinline__ int comp_of(const ProductDev &prod, int q)
{
    return NC == 6 ? q : prod.comp[q];
}
// odd in z: xz, yz.  These are also the components odd in exactly one of x
// and y, whose Kt (transformed along x and y) is imaginary.
template <int NC, int PAR>
__device__ __forceinline__ bool odd_z(const ProductDev &prod, int q)
{
    if constexpr (PAR == kParEven) return false;
    const int c = comp_of<NC, PAR>(prod, q);
    return c == 4 || c == 5;
}
// odd in y: xy, yz
template <int NC, int PAR>
__device__ __forceinline__ bool odd_y(const ProductDev &prod, int q)
{
    if constexpr (PAR == kParEven) return false;
    const int c = comp_of<NC, PAR>(prod, q);
    return c == 3 || c == 5;
}

// Kt_q(kx, ky, d) for the product's NC components, with the parity sign of
// the z offset (xz and yz are odd in z); `d` must satisfy |d| < nzk.
template <typename R, int NC, int PAR = kParRuntime>
__device__ __forceinline__ void kt_at(const KtDev<R> &kt, const ProductDev &prod, int kx, int ky, int d, R *K)
{
    const int dq = d < 0 ? -d : d;
    const unsigned dsg = d < 0 ? kSignBit : 0u;
    const long long at = ((long long)kx * kt.nzk + dq) * kt.ky_pitch + ky;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int c = comp_of<NC, PAR>(prod, q);
        const R v = (NC < 6 || (prod.need >> c & 1)) ? kt.k[c * kt.comp_stride + at] : (R)0;
        K[q] = flip_sign(v, (odd_z<NC, PAR>(prod, q) ? ~0u : 0u) & dsg);
    }
}

// out_o += sum_i (sum_q W[o][i][q] K_q) x_i; K_q is real, or imaginary
// (the stored value times i) for the xz and yz components.  A coefficient
// known to be purely real (or imaginary) scales x without a full complex
// product.
template <typename R, int CI, int CO, int NC, int PAR = kParRuntime>
__device__ __forceinline__ void zsum_mac(const ProductDev &prod, const R *K, const cplx<R> *x, cplx<R> *out)
{
#pragma unroll
    for (int o = 0; o < CO; ++o)
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            if constexpr (PAR == kParEven) {
                static_assert(NC == 1, "a fixed parity class describes a single component");
                const R w = (R)prod.Wq[o][i][0] * K[0];
                out[o].x = fma(w, x[i].x, out[o].x);
                out[o].y = fma(w, x[i].y, out[o].y);
            } else {
                R cre = 0, cim = 0;
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    const R w = (R)(NC == 6 ? prod.W[o][i][q] : prod.Wq[o][i][q]) * K[q];
                    const bool im = odd_z<NC, PAR>(prod, q);
                    cre += im ? (R)0 : w;
                    cim += im ? w : (R)0;
                }
                out[o] = cadd(out[o], cmul(cplx<R>{cre, cim}, x[i]));
            }
        }
}

// J from the objective's block sums (see JFinal); called by all 64 lanes of
// one wave.  Lane i holds sum b0 + i; the adds run in block order, the same
// order as a single thread summing them.
__device__ __forceinline__ void finalize_j(const JFinal &jf)
{
    const int lane = threadIdx.x & 63;
    double total = 0.0;
    for (int b0 = 0; b0 < jf.nb; b0 += 64) {
        const double v = b0 + lane < jf.nb ? jf.partials[b0 + lane] : 0.0;
        const int n = min(64, jf.nb - b0);
        for (int i = 0; i < n; ++i) total += __shfl(v, i);
    }
    if (lane == 0) *jf.J = jf.div ? total / jf.c : jf.c * total;
}

// In a batched launch (a one-dimensional grid over the blocks of n designs,
// design d owning blocks starts[d] .. starts[d+1] - 1): the calling block's
// design d (a uniform binary search), its arguments and its place in that
// design's own grid.
template <typename A>
__device__ __forceinline__ A batch_args(const A *__restrict__ tab, const int *__restrict__ starts, int n, BlockPos &bp)
{
    const int b = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const A a = tab[lo];
    const int local = b - starts[lo];
    bp.gx_ = a.bg.gx;
    bp.gy_ = a.bg.gy;
    bp.gz_ = a.bg.gz;
    bp.x_ = local % bp.gx_;
    bp.y_ = (local / bp.gx_) % bp.gy_;
    bp.z_ = local / (bp.gx_ * bp.gy_);
    return a;
}

}  // namespace tofdev
