// Passes 2-4 fused for a convolution whose source or target spans only a few
// z rows (the objective's plane).  With Kt, the tensor transformed along x
// and y only, the z part of the convolution is a direct sum per (kx, ky)
// column, out(zt) = sum_zs Kt(zt - zs) x(zs), and needs no z transform; the
// y transforms of the many-row side can then run in the same kernel, so the
// y spectra of those rows never go through HBM.
//
//   gather  (few target rows): per kx, the y FFT of every source row times
//           Kt, summed over the source rows of a group and transformed back
//           along y; each group writes its partial target rows in y space,
//           and the next kernel (the inverse x pass, or the fused objective,
//           for which the rows are stored with kx fastest) adds the partials
//           in group order while staging.  (Adding them in the last block of
//           each kx instead needs a device-scope release per block, an L2
//           write-back on this chip, which costs far more.)
//   scatter (few source rows): per kx, the y FFT of the source rows (kept in
//           LDS), then for every target row the sum against Kt and the
//           inverse y FFT, written straight into the layout of the inverse x
//           pass.  Its first wave can also form J from the objective's
//           block sums (JFinal).
//
// A y line is held by P = L / E threads (thread p: positions p + P m, see
// fft_reg.h); a 256-thread block runs NL = 256 / P lines side by side.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "engine.h"
#include "fft_reg.h"

namespace {

using namespace tofdev;

// Minimum waves per SIMD the compiler must allow (register budget) for the
// gather and the scatter, FP32 and FP64; 1 leaves the register count to the
// compiler.
#ifndef TOF_YZ_GATHER_WAVES
#define TOF_YZ_GATHER_WAVES 1
#endif
#ifndef TOF_YZ_SCATTER_WAVES
#define TOF_YZ_SCATTER_WAVES 1
#endif
#ifndef TOF_YZ_GATHER_WAVES_F64
#define TOF_YZ_GATHER_WAVES_F64 1
#endif
#ifndef TOF_YZ_SCATTER_WAVES_F64
#define TOF_YZ_SCATTER_WAVES_F64 1
#endif
#ifndef TOF_YZ_ROWS
#define TOF_YZ_ROWS 1
#endif

constexpr int kE = 8;           // elements per thread of a y line
constexpr int kBlock = 256;     // threads per block

// Source line of length L with data at positions [y0, y0 + ny): row[y - y0];
// zero elsewhere and when !ok.  Addresses are clamped into the row, so the
// loads need no branch.
template <typename R, int L, int E>
__device__ __forceinline__ void load_line(const cplx<R> *row, int y0, int ny, int p, bool ok, cplx<R> *v)
{
    constexpr int P = L / E;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int n = p + P * m;
        const cplx<R> a = row[min(max(n - y0, 0), ny - 1)];
        v[m] = (ok && n >= y0 && n < y0 + ny) ? a : cplx<R>{0, 0};
    }
}

// Kt_q(kx, ky, d) at a line thread's frequencies ky = p + P m, m < E.  Only
// the half ky <= L/2 is read (L/2 + 1 values a line): the other half follows
// from the parity in y of each component (Kt(L - ky) = Kt(ky), negated for
// xy and yz, which are odd in y), taken from lane P - p of the same line,
// slot E - 1 - m (lane 0 keeps its own slot E - m).
//
// kt_half loads the half (slots 0 .. E/2 - 1 and ky = L/2); kt_full completes
// the line, so the loads of a later row can be issued before the lane
// exchange of the current one.
template <typename R, int L, int E, int NC, int PAR>
__device__ __forceinline__ void kt_half(const KtDev<R> &kt, const ProductDev &prod, int kx, int p, int d,
                                        R (*lo)[NC])
{
    constexpr int P = L / E;
    constexpr int H = E / 2;
#pragma unroll
    for (int m = 0; m < H; ++m) kt_at<R, NC, PAR>(kt, prod, kx, p + P * m, d, lo[m]);
    kt_at<R, NC, PAR>(kt, prod, kx, L / 2, d, lo[H]);   // ky = L/2: lane 0's slot H
}

template <typename R, int L, int E, int NC, int PAR>
__device__ __forceinline__ void kt_full(const ProductDev &prod, int p, const R (*lo)[NC], R (*K)[NC])
{
    constexpr int P = L / E;
    constexpr int H = E / 2;
    static_assert(E % 2 == 0 && 64 % P == 0, "a line spans a power-of-two lane group");
    const int lane = threadIdx.x & 63;
    const int src = lane - p + ((P - p) & (P - 1));
#pragma unroll
    for (int m = 0; m < H; ++m)
#pragma unroll
        for (int q = 0; q < NC; ++q) K[m][q] = lo[m][q];
#pragma unroll
    for (int m = H; m < E; ++m)
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const unsigned oy = odd_y<NC, PAR>(prod, q) ? kSignBit : 0u;
            const R mirrored = flip_sign(__shfl(lo[E - 1 - m][q], src), oy);
            // lane 0: ky = P m mirrors to P (E - m), its own slot (m = H is ky = L/2 itself,
            // where the odd components vanish, so no sign is needed)
            K[m][q] = p == 0 ? (m == H ? lo[H][q] : flip_sign(lo[E - m][q], oy)) : mirrored;
        }
}

// Arguments of the fused kernels (one design).
template <typename R>
struct YzKArgs {
    BatchGrid bg;
    const cplx<R> *A;
    int hx, ys0, nys, zs0, nzs, zt0, nzt, rpg, yt0, nyt;
    KtDev<R> kt;
    ProductDev prod;
    cplx<R> *out;          // gather: the partial rows; scatter: C
    const cplx<R> *table;
    int kxf;               // gather: partial rows with kx fastest
    JFinal jf;             // scatter: J to form first, or none
};

// Few target rows.  Block (kx, g) takes source rows [g rpg, (g+1) rpg) of
// the source box; line slot l transforms rows l, l + NL, ... of that range.
// A is [CI][hx][nzs][nys] (the x pass output); part is [G][CO][hx][nzt][nyt]
// with y from yt0: G copies of the inverse x pass's input, to be added; with
// kxf [G][CO][nzt][nyt][hx] (rows with kx fastest, for the fused objective).
// HALF: 1: the source rows lie in the lower half of the line (ys0 + nys <=
// L/2, which the 2n padding always gives), so only that half is loaded and
// the first stage skips the zero half; 2: they fill it exactly (ys0 = 0,
// nys = L/2), so the loads need no bounds either.
template <typename R, int L, int E, int CI, int CO, int NC, int NR, int PAR, int HALF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? TOF_YZ_GATHER_WAVES_F64 : TOF_YZ_GATHER_WAVES))) void k_yzsum_gather(
    const cplx<R> *A, int hx, int ys0, int nys, int zs0, int nzs, int zt0, int nzt, int rpg, int yt0, int nyt,
    KtDev<R> kt, ProductDev prod, cplx<R> *part, const cplx<R> *table, int kxf)
{
#define TOF_BX ((int)blockIdx.x)
#define TOF_BY ((int)blockIdx.y)
#define TOF_BZ ((int)blockIdx.z)
#define TOF_BGX ((int)gridDim.x)
#define TOF_BGY ((int)gridDim.y)
#define TOF_BGZ ((int)gridDim.z)
#include "body_yzsum_gather.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

template <typename R, int L, int E, int CI, int CO, int NC, int NR, int PAR, int HALF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? TOF_YZ_GATHER_WAVES_F64 : TOF_YZ_GATHER_WAVES))) void k_yzsum_gather_batch(const YzKArgs<R> *__restrict__ tab, const int *__restrict__ starts, int n)
{
    BlockPos bp;
    const YzKArgs<R> a = batch_args(tab, starts, n, bp);
    const auto &A = a.A;
    const auto &hx = a.hx;
    const auto &ys0 = a.ys0;
    const auto &nys = a.nys;
    const auto &zs0 = a.zs0;
    const auto &nzs = a.nzs;
    const auto &zt0 = a.zt0;
    const auto &nzt = a.nzt;
    const auto &rpg = a.rpg;
    const auto &yt0 = a.yt0;
    const auto &nyt = a.nyt;
    const auto &kt = a.kt;
    const auto &prod = a.prod;
    const auto &part = a.out;
    const auto &table = a.table;
    const auto &kxf = a.kxf;
#define TOF_BX (bp.x_)
#define TOF_BY (bp.y_)
#define TOF_BZ (bp.z_)
#define TOF_BGX (bp.gx_)
#define TOF_BGY (bp.gy_)
#define TOF_BGZ (bp.gz_)
#include "body_yzsum_gather.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

// Few source rows.  Block (kx, g) takes target rows [g rpg, (g+1) rpg) of
// the target box; line slot l handles rows l, l + NL, ... of that range.
// A is [CI][hx][nzs][nys]; C is [CO][hx][nzt][nyt] with y from yt0 (the
// input layout of the inverse x pass).
// HALF: the target rows fill exactly the lower half of the line (yt0 = 0,
// nyt = L/2): the upper half of the inverse transform is never formed.
// jf: J formed first by the first wave of block (0, 0) (see JFinal).
template <typename R, int L, int E, int CI, int CO, int NC, int NR, int PAR, bool HALF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? TOF_YZ_SCATTER_WAVES_F64 : TOF_YZ_SCATTER_WAVES))) void k_yzsum_scatter(
    const cplx<R> *A, int hx, int ys0, int nys, int zs0, int nzs, int zt0, int nzt, int rpg, int yt0, int nyt,
    KtDev<R> kt, ProductDev prod, cplx<R> *C, const cplx<R> *table, JFinal jf)
{
#define TOF_BX ((int)blockIdx.x)
#define TOF_BY ((int)blockIdx.y)
#define TOF_BZ ((int)blockIdx.z)
#define TOF_BGX ((int)gridDim.x)
#define TOF_BGY ((int)gridDim.y)
#define TOF_BGZ ((int)gridDim.z)
#include "body_yzsum_scatter.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

template <typename R, int L, int E, int CI, int CO, int NC, int NR, int PAR, bool HALF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? TOF_YZ_SCATTER_WAVES_F64 : TOF_YZ_SCATTER_WAVES))) void k_yzsum_scatter_batch(const YzKArgs<R> *__restrict__ tab, const int *__restrict__ starts, int n)
{
    BlockPos bp;
    const YzKArgs<R> a = batch_args(tab, starts, n, bp);
    const auto &A = a.A;
    const auto &hx = a.hx;
    const auto &ys0 = a.ys0;
    const auto &nys = a.nys;
    const auto &zs0 = a.zs0;
    const auto &nzs = a.nzs;
    const auto &zt0 = a.zt0;
    const auto &nzt = a.nzt;
    const auto &rpg = a.rpg;
    const auto &yt0 = a.yt0;
    const auto &nyt = a.nyt;
    const auto &kt = a.kt;
    const auto &prod = a.prod;
    const auto &C = a.out;
    const auto &table = a.table;
    const auto &jf = a.jf;
#define TOF_BX (bp.x_)
#define TOF_BY (bp.y_)
#define TOF_BZ (bp.z_)
#define TOF_BGX (bp.gx_)
#define TOF_BGY (bp.gy_)
#define TOF_BGZ (bp.gz_)
#include "body_yzsum_scatter.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

// Register and LDS limits of the fused kernels: the gather keeps NR x CO
// accumulators per element, both keep NR x NC tensor values per element, the
// scatter keeps NR x CI source spectra in LDS.
constexpr bool gather_fits(int CO, int NC, int NR) { return NR * CO <= 4 && NR * NC <= 6; }
constexpr size_t scatter_lds(int L, int CI, int NR, size_t csz)
{
    return ((size_t)TOF_YZ_ROWS * (kBlock / (L / kE)) * regfft::padded_len(L) + (size_t)NR * CI * L) * csz;
}
constexpr bool scatter_fits(int L, int CI, int NC, int NR, size_t csz)
{
    return NR * NC <= 6 && scatter_lds(L, CI, NR, csz) <= 96 * 1024;
}

template <typename R>
YzKArgs<R> gather_args(const YzSumArgs<R> &a, const KtDev<R> &kt, const ProductDev &prod, const cplx<R> *table)
{
    return YzKArgs<R>{{}, a.A, a.hx, a.ys0, a.nys, a.zs0, a.nzs, a.zt0, a.nzt, a.rpg, a.yt0, a.nyt, kt, prod, a.part,
                      table, a.part_kx_fast, JFinal{}};
}

template <typename R>
YzKArgs<R> scatter_args(const YzSumArgs<R> &a, const KtDev<R> &kt, const ProductDev &prod, const cplx<R> *table)
{
    return YzKArgs<R>{{}, a.A, a.hx, a.ys0, a.nys, a.zs0, a.nzs, a.zt0, a.nzt, a.rpg, a.yt0, a.nyt, kt, prod, a.C,
                      table, 0, a.jf};
}

template <typename R, int L, int CI, int CO, int NC, int PAR, int HALF>
hipError_t launch_yzsum_h(hipStream_t st, const YzSumArgs<R> &a, int rows, const KtDev<R> &kt,
                          const ProductDev &prod, const cplx<R> *table, bool check_only)
{
    constexpr int NRM = kZsumMaxRows;
    constexpr size_t csz = sizeof(cplx<R>);
    const int G = (rows + a.rpg - 1) / a.rpg;
    const dim3 grid(a.hx, G);
    if (a.nzt <= NRM) {
        if (a.nzt == 1) {
            if constexpr (gather_fits(CO, NC, 1)) {
                if (check_only) return hipSuccess;
                TOF_LAUNCH_B((k_yzsum_gather<R, L, kE, CI, CO, NC, 1, PAR, HALF>),
                             (k_yzsum_gather_batch<R, L, kE, CI, CO, NC, 1, PAR, HALF>), grid, dim3(kBlock), st,
                             gather_args(a, kt, prod, table), a.A, a.hx, a.ys0, a.nys, a.zs0, a.nzs, a.zt0, a.nzt,
                             a.rpg, a.yt0, a.nyt, kt, prod, a.part, table, a.part_kx_fast);
                return hipGetLastError();
            }
        } else {
            if constexpr (gather_fits(CO, NC, NRM)) {
                if (check_only) return hipSuccess;
                TOF_LAUNCH_B((k_yzsum_gather<R, L, kE, CI, CO, NC, NRM, PAR, HALF>),
                             (k_yzsum_gather_batch<R, L, kE, CI, CO, NC, NRM, PAR, HALF>), grid, dim3(kBlock), st,
                             gather_args(a, kt, prod, table), a.A, a.hx, a.ys0, a.nys, a.zs0, a.nzs, a.zt0, a.nzt,
                             a.rpg, a.yt0, a.nyt, kt, prod, a.part, table, a.part_kx_fast);
                return hipGetLastError();
            }
        }
        return hipErrorInvalidValue;
    }
    if (a.nzs == 1) {
        if constexpr (scatter_fits(L, CI, NC, 1, csz)) {
            if (check_only) return hipSuccess;
            TOF_LAUNCH_B((k_yzsum_scatter<R, L, kE, CI, CO, NC, 1, PAR, HALF == 2>),
                         (k_yzsum_scatter_batch<R, L, kE, CI, CO, NC, 1, PAR, HALF == 2>), grid, dim3(kBlock), st,
                         scatter_args(a, kt, prod, table), a.A, a.hx, a.ys0, a.nys, a.zs0, a.nzs, a.zt0, a.nzt,
                         a.rpg, a.yt0, a.nyt, kt, prod, a.C, table, a.jf);
            return hipGetLastError();
        }
    } else if (a.nzs <= NRM) {
        if constexpr (scatter_fits(L, CI, NC, NRM, csz)) {
            if (check_only) return hipSuccess;
            TOF_LAUNCH_B((k_yzsum_scatter<R, L, kE, CI, CO, NC, NRM, PAR, HALF == 2>),
                         (k_yzsum_scatter_batch<R, L, kE, CI, CO, NC, NRM, PAR, HALF == 2>), grid, dim3(kBlock), st,
                         scatter_args(a, kt, prod, table), a.A, a.hx, a.ys0, a.nys, a.zs0, a.nzs, a.zt0, a.nzt,
                         a.rpg, a.yt0, a.nyt, kt, prod, a.C, table, a.jf);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

// Where the many-row side lies in the y line: 2 when it fills exactly the
// lower half (the source rows for the gather, the target rows for the
// scatter), 1 when the gather's source rows lie in the lower half, else 0
// (the scatter has forms 2 and 0 only).
template <typename R, int L, int CI, int CO, int NC, int PAR>
hipError_t launch_yzsum_l(hipStream_t st, const YzSumArgs<R> &a, int rows, const KtDev<R> &kt,
                          const ProductDev &prod, const cplx<R> *table, bool check_only)
{
    const bool gather = a.nzt <= kZsumMaxRows;
    const int half = gather ? (a.ys0 == 0 && a.nys == L / 2 ? 2 : (a.ys0 + a.nys <= L / 2 ? 1 : 0))
                            : (a.yt0 == 0 && a.nyt == L / 2 ? 2 : 0);
    if (half == 2) return launch_yzsum_h<R, L, CI, CO, NC, PAR, 2>(st, a, rows, kt, prod, table, check_only);
    if (half == 1) return launch_yzsum_h<R, L, CI, CO, NC, PAR, 1>(st, a, rows, kt, prod, table, check_only);
    return launch_yzsum_h<R, L, CI, CO, NC, PAR, 0>(st, a, rows, kt, prod, table, check_only);
}

template <typename R, int L>
hipError_t launch_yzsum_c(hipStream_t st, const YzSumArgs<R> &a, int rows, const KtDev<R> &kt,
                          const ProductDev &prod, const cplx<R> *table, bool check_only)
{
    const int key = prod.c_in * 4 + prod.c_out;
    if (key == 5 && prod.nc == 1) {
        if (prod.comp[0] <= 2)   // a diagonal component: real, even in x, y and z
            return launch_yzsum_l<R, L, 1, 1, 1, kParEven>(st, a, rows, kt, prod, table, check_only);
        return launch_yzsum_l<R, L, 1, 1, 1, kParRuntime>(st, a, rows, kt, prod, table, check_only);
    }
    switch (key) {
    case 5: return launch_yzsum_l<R, L, 1, 1, 6, kParRuntime>(st, a, rows, kt, prod, table, check_only);
    case 7: return launch_yzsum_l<R, L, 1, 3, 6, kParRuntime>(st, a, rows, kt, prod, table, check_only);
    case 13: return launch_yzsum_l<R, L, 3, 1, 6, kParRuntime>(st, a, rows, kt, prod, table, check_only);
    case 15: return launch_yzsum_l<R, L, 3, 3, 6, kParRuntime>(st, a, rows, kt, prod, table, check_only);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename R>
hipError_t launch_yz_sum(hipStream_t st, const YzSumArgs<R> &a, const KtDev<R> &kt, const ProductDev &prod,
                         const FftPlanDev &plan, bool check_only)
{
    if (a.rpg < 1 || a.nzs < 1 || a.nzt < 1 || a.nys < 1 || a.nyt < 1) return hipErrorInvalidValue;
    const int rows = a.nzt <= kZsumMaxRows ? a.nzs : a.nzt;
    const cplx<R> *table = (const cplx<R> *)plan.tw;
    switch (plan.L) {
    case 32: return launch_yzsum_c<R, 32>(st, a, rows, kt, prod, table, check_only);
    case 64: return launch_yzsum_c<R, 64>(st, a, rows, kt, prod, table, check_only);
    case 128: return launch_yzsum_c<R, 128>(st, a, rows, kt, prod, table, check_only);
    case 256: return launch_yzsum_c<R, 256>(st, a, rows, kt, prod, table, check_only);
    case 512: return launch_yzsum_c<R, 512>(st, a, rows, kt, prod, table, check_only);
    default: return hipErrorInvalidValue;
    }
}

#ifndef TOF_NO_F32
template hipError_t launch_yz_sum<float>(hipStream_t, const YzSumArgs<float> &, const KtDev<float> &,
                                         const ProductDev &, const FftPlanDev &, bool);
#endif
#ifndef TOF_NO_F64
template hipError_t launch_yz_sum<double>(hipStream_t, const YzSumArgs<double> &, const KtDev<double> &,
                                          const ProductDev &, const FftPlanDev &, bool);
#endif
