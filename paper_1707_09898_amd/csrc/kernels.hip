// HIP kernels of the gradient engine (gfx950).
//
// One convolution H = -N (*) M (eq. (convolution)) runs as five passes over
// the zero-padded box (L = padded lengths, hx = Lx/2 + 1):
//   x_forward   source rows -> real-to-complex FFT along x       A[c][kx][z][y]
//   line_fft    complex FFT along y (source rows only)           B[c][kx][z][ky]
//   z_pass      FFT along z, spectral tensor product, inverse z  B (in place)
//   line_fft    inverse FFT along y, target rows only            C[c][kx][z][y]
//   x_inverse   complex-to-real inverse FFT along x + epilogue   H or dJ/drho
// The zero padding is never stored: each pass fills it in LDS.  Source and
// target index boxes restrict every pass to the rows that carry data or are
// read afterwards (the convolution's result at a target cell does not depend
// on which other targets are computed).  The tensor spectra are real (each
// component is even or odd along each axis) and stored for one octant of
// frequencies with -1/(Lx Ly Lz) folded in, so no pass normalizes.
#include <hip/hip_runtime.h>

#include "dd.h"
#include "device_common.h"
#include "engine.h"
#include "fft_reg.h"

// Minimum waves per SIMD the compiler must allow (register budget) for the
// register x passes, forward and inverse (the inverse one with one
// component and no partial copies, FP32 and FP64; its other forms need more
// registers); 1 leaves it to the compiler.
#ifndef TOF_XF_WAVES
#define TOF_XF_WAVES 1
#endif
#ifndef TOF_XI_WAVES
#define TOF_XI_WAVES 8
#endif
#ifndef TOF_XI_WAVES_F64
#define TOF_XI_WAVES_F64 4
#endif
#ifndef TOF_ZSUM_U
#define TOF_ZSUM_U 4
#endif
#ifndef TOF_ZSUM_THREADS
#define TOF_ZSUM_THREADS 256
#endif

namespace {

using namespace tofdev;

constexpr int kThreads = 256;


// x[m] <- x[m]^p, m < N, by repeated multiplication from the left (the same
// rounding as ipow_dev); p is uniform, so one branch serves all N values.
template <typename R, int N>
__device__ __forceinline__ void ipow_n(R *x, int p)
{
    switch (p) {
    case 0:
#pragma unroll
        for (int m = 0; m < N; ++m) x[m] = (R)1;
        break;
    case 1: break;
    case 2:
#pragma unroll
        for (int m = 0; m < N; ++m) x[m] = x[m] * x[m];
        break;
    case 3:
#pragma unroll
        for (int m = 0; m < N; ++m) x[m] = x[m] * x[m] * x[m];
        break;
    case 4:
#pragma unroll
        for (int m = 0; m < N; ++m) x[m] = x[m] * x[m] * x[m] * x[m];
        break;
    default:
#pragma unroll
        for (int m = 0; m < N; ++m) {
            R v = x[m];
            for (int i = 1; i < p; ++i) v *= x[m];
            x[m] = v;
        }
    }
}

template <typename R>
__device__ __forceinline__ R ipow_dev(R x, int p)
{
    R v = (R)1;
    for (int i = 0; i < p; ++i) v *= x;
    return v;
}

template <typename R>
__device__ __forceinline__ R source_value(int mode, const DesignDev<R> &d, const View4<const R> &s,
                                          int c, int x, int y, int z)
{
    if (mode == SRC_ARRAY)
        return s.ptr[c * s.cs + (long long)(z - s.oz) * s.zs + (long long)(y - s.oy) * s.ys + (x - s.ox)];
    if (!d.design.has(x, y, z)) return (R)0;
    const long long idx = ((long long)z * d.ny + y) * d.nx + x;
    if (d.mask && !d.mask[idx]) return (R)0;
    R v = ipow_dev(d.rho[idx], d.p);
    if (mode == SRC_RHO_VECTOR) v *= d.m0f[(long long)c * d.nx * d.ny * d.nz + idx];
    return v;
}

// Arguments of the register x passes (one design).
template <typename R>
struct XfArgs {
    BatchGrid bg;
    int mode;
    DesignDev<R> dsg;
    View4<const R> src;
    Box S;
    cplx<R> *out;
    int hx;
    const cplx<R> *table;
};

template <typename R>
struct XiArgs {
    BatchGrid bg;
    const cplx<R> *C;
    int hx;
    Box T;
    int grad_epi;
    View4<R> out;
    DesignDev<R> dsg;
    R m0u0, m0u1, m0u2;
    R *grad;
    const cplx<R> *table;
    int zrows;
    int nsum;
    long long sum_stride;
};

template <typename R>
struct ObjXfArgs {
    BatchGrid bg;
    ObjectiveDev<R> o;
    cplx<R> *out;
    int hx;
    const cplx<R> *table;
    const cplx<R> *spec;
    int nsum;
    long long sum_stride;
    int kxf;
};

// ---------------------------------------------------------------------------
// Pass 1: real-to-complex FFT along x of TY source rows (one z, one component).
// Two real rows share one complex line (a + i b); the two half spectra are
// separated with A[k] = (Z[k] + conj Z[-k]) / 2, B[k] = (Z[k] - conj Z[-k]) / 2i.
// Output A[c][kx][z - S.z0][y - S.y0].
template <typename R>
__global__ __launch_bounds__(kThreads) void k_x_forward(int mode, DesignDev<R> dsg, View4<const R> src,
                                                      Box S, FftPlanDev plan, cplx<R> *out, int hx,
                                                      int TY, int pitch)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<R> *buf0 = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf1 = buf0 + (TY / 2) * pitch;
    const int L = plan.L;
    const int c = blockIdx.z;
    const int zrel = blockIdx.y;
    const int z = S.z0 + zrel;
    const int ybase = S.y0 + blockIdx.x * TY;
    const int nrow = min(TY, S.y1 - ybase);
    const int nline = (nrow + 1) / 2;
    for (int e = threadIdx.x; e < nline * L; e += blockDim.x) {
        const int l = e / L;
        const int pos = e - l * L;
        R re = 0, im = 0;
        if (pos >= S.x0 && pos < S.x1) {
            const int r0 = 2 * l;
            if (r0 < nrow) re = source_value(mode, dsg, src, c, pos, ybase + r0, z);
            if (r0 + 1 < nrow) im = source_value(mode, dsg, src, c, pos, ybase + r0 + 1, z);
        }
        buf0[l * pitch + pos] = cplx<R>{re, im};
    }
    __syncthreads();
    const cplx<R> *res = fft_lines_lds(buf0, buf1, nline, pitch, plan, false);
    const int nys = S.ny(), nzs = S.nz();
    const long long kxs = (long long)nzs * nys;
    cplx<R> *o = out + (long long)c * hx * kxs + (long long)zrel * nys + (ybase - S.y0);
    const R half = (R)0.5;
    for (int e = threadIdx.x; e < hx * nrow; e += blockDim.x) {
        const int k = e / nrow;
        const int r = e - k * nrow;
        const cplx<R> *line = res + (r >> 1) * pitch;
        const cplx<R> Zk = line[k];
        const cplx<R> Zm = line[k == 0 ? 0 : L - k];
        cplx<R> v;
        if ((r & 1) == 0) v = cplx<R>{(Zk.x + Zm.x) * half, (Zk.y - Zm.y) * half};
        else v = cplx<R>{(Zk.y + Zm.y) * half, (Zm.x - Zk.x) * half};
        o[k * kxs + r] = v;
    }
}

// ---------------------------------------------------------------------------
// Passes 2 and 4: complex FFT of contiguous lines.  Line l reads n_in values
// at in[(l / inner) in_outer + (l % inner) in_inner] into positions
// [p_in, p_in + n_in) (zero elsewhere) and writes positions [p_out, p_out + n_out).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_line_fft(const cplx<R> *in, cplx<R> *out, int nlines,
                                                     int inner, long long in_outer, long long in_inner,
                                                     long long out_outer, long long out_inner, int p_in,
                                                     int n_in, int p_out, int n_out, FftPlanDev plan,
                                                     int inv, int NL, int pitch, BlockMap bin, BlockMap bout)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<R> *buf0 = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf1 = buf0 + NL * pitch;
    const int L = plan.L;
    const int l0 = blockIdx.x * NL;
    const int nl = min(NL, nlines - l0);
    for (int e = threadIdx.x; e < nl * L; e += blockDim.x) {
        const int l = e / L;
        const int pos = e - l * L;
        const int line = l0 + l;
        cplx<R> v{0, 0};
        if (pos >= p_in && pos < p_in + n_in)
            v = in[(long long)(line / inner) * in_outer + (long long)(line % inner) * in_inner + bin.at(pos - p_in)];
        buf0[l * pitch + pos] = v;
    }
    __syncthreads();
    const cplx<R> *res = fft_lines_lds(buf0, buf1, nl, pitch, plan, inv != 0);
    for (int e = threadIdx.x; e < nl * n_out; e += blockDim.x) {
        const int l = e / n_out;
        const int q = e - l * n_out;
        const int line = l0 + l;
        out[(long long)(line / inner) * out_outer + (long long)(line % inner) * out_inner + bout.at(q)] =
            res[l * pitch + p_out + q];
    }
}

// Tensor spectrum at one frequency as a full symmetric 3x3 matrix.  The
// octant holds |ky|, |kz| (kx is never negative in the half spectrum); odd
// components change sign with the frequency along their odd axes.
template <typename R>
__device__ __forceinline__ void spectrum_at(const SpectrumDev<R> &sp, int need, int kx, int kyq,
                                            int kzq, R sy, R sz, R K[3][3])
{
    R v[6];
    const long long at = ((long long)kx * sp.hkz + kzq) * sp.ky_pitch + kyq;
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = (need >> c & 1) ? sp.k[c * sp.comp_stride + at] : (R)0;
    v[3] *= sy;        // xy: odd in y
    v[4] *= sz;        // xz: odd in z
    v[5] *= sy * sz;   // yz: odd in y and z
    K[0][0] = v[0]; K[1][1] = v[1]; K[2][2] = v[2];
    K[0][1] = K[1][0] = v[3];
    K[0][2] = K[2][0] = v[4];
    K[1][2] = K[2][1] = v[5];
}

// ---------------------------------------------------------------------------
// Pass 3: for TK consecutive ky columns of one kx: forward FFT along z of the
// source rows, per-frequency product out_o = sum_i (U K V)_oi in_i, inverse
// FFT along z, store the target rows.  In place in B; a block owns its
// columns, and reads all of them before it writes.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_z_pass(cplx<R> *B, int hx, int Ly, int Zrows, int zs0,
                                                   int nzs, int zt0, int nzt, SpectrumDev<R> spec,
                                                   ProductDev prod, int forward_only, FftPlanDev plan,
                                                   int TK, int pitch, BlockMap bm)
{
    extern __shared__ unsigned char smem_raw[];
    const int cmax = max(prod.c_in, prod.c_out);
    cplx<R> *buf0 = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf1 = buf0 + cmax * TK * pitch;
    const int L = plan.L;
    const int kx = blockIdx.y;
    const int k0 = blockIdx.x * TK;
    const int ncol = min(TK, Ly - k0);
    const long long cstride = (long long)hx * Zrows * Ly;
    cplx<R> *base = B + (long long)kx * Zrows * Ly;
    const int c_in = prod.c_in, c_out = prod.c_out;
    for (int e = threadIdx.x; e < c_in * L * TK; e += blockDim.x) {
        const int col = e % TK;
        const int rest = e / TK;
        const int pos = rest % L;
        const int i = rest / L;
        cplx<R> v{0, 0};
        if (col < ncol && pos >= zs0 && pos < zs0 + nzs) v = base[i * cstride + bm.col(k0 + col, pos - zs0)];
        buf0[(i * TK + col) * pitch + pos] = v;
    }
    __syncthreads();
    cplx<R> *res = fft_lines_lds(buf0, buf1, c_in * TK, pitch, plan, false);
    if (forward_only) {
        for (int e = threadIdx.x; e < c_in * L * TK; e += blockDim.x) {
            const int col = e % TK;
            const int rest = e / TK;
            const int pos = rest % L;
            const int i = rest / L;
            if (col < ncol) base[i * cstride + bm.col(k0 + col, pos)] = res[(i * TK + col) * pitch + pos];
        }
        return;
    }
    cplx<R> *other = (res == buf0) ? buf1 : buf0;
    R U[3][3], V[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            U[a][b] = (R)prod.U[a][b];
            V[a][b] = (R)prod.V[a][b];
        }
    const int hLy = Ly / 2, hLz = L / 2;
    for (int e = threadIdx.x; e < TK * L; e += blockDim.x) {
        const int col = e % TK;
        const int kz = e / TK;
        const int ky = min(k0 + col, Ly - 1);
        const int kyq = ky <= hLy ? ky : Ly - ky;
        const int kzq = kz <= hLz ? kz : L - kz;
        const R sy = ky > hLy ? (R)-1 : (R)1;
        const R sz = kz > hLz ? (R)-1 : (R)1;
        R K[3][3];
        spectrum_at(spec, prod.need, kx, kyq, kzq, sy, sz, K);
        // KV[a][i] = sum_b K[a][b] V[b][i]
        R KV[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) KV[a][i] = K[a][0] * V[0][i] + K[a][1] * V[1][i] + K[a][2] * V[2][i];
        cplx<R> in[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) in[i] = i < c_in ? res[(i * TK + col) * pitch + kz] : cplx<R>{0, 0};
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            if (o >= c_out) break;
            cplx<R> acc{0, 0};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const R coef = U[o][0] * KV[0][i] + U[o][1] * KV[1][i] + U[o][2] * KV[2][i];
                acc.x += coef * in[i].x;
                acc.y += coef * in[i].y;
            }
            other[(o * TK + col) * pitch + kz] = acc;
        }
    }
    __syncthreads();
    const cplx<R> *res2 = fft_lines_lds(other, res, c_out * TK, pitch, plan, true);
    for (int e = threadIdx.x; e < c_out * nzt * TK; e += blockDim.x) {
        const int col = e % TK;
        const int rest = e / TK;
        const int zq = rest % nzt;
        const int o = rest / nzt;
        if (col < ncol) base[o * cstride + bm.col(k0 + col, zq)] = res2[(o * TK + col) * pitch + zt0 + zq];
    }
}

// ---------------------------------------------------------------------------
// Pass 5: complex-to-real inverse FFT along x of TY target rows (one z, all
// components).  Two Hermitian half spectra A, B become one complex line
// Z = A + iB (extended by Z[L-k] = conj A[k] + i conj B[k]); the real and
// imaginary parts of its inverse transform are the two rows.  Epilogue:
// the field (strided store) or dJ/drho = chi p rho^(p-1) sum_c coef_c A_c over
// whole x rows (zero outside the design region).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_x_inverse(const cplx<R> *C, int hx, int nc, Box T,
                                                      FftPlanDev plan, int grad_epi, View4<R> out,
                                                      DesignDev<R> dsg, R m0u0, R m0u1, R m0u2,
                                                      R *grad, int TY, int pitch)
{
    extern __shared__ unsigned char smem_raw[];
    const int nlmax = TY / 2;
    cplx<R> *buf0 = reinterpret_cast<cplx<R> *>(smem_raw);
    cplx<R> *buf1 = buf0 + nc * nlmax * pitch;
    const int L = plan.L;
    const int zrel = blockIdx.y;
    const int z = T.z0 + zrel;
    const int ybase = T.y0 + blockIdx.x * TY;
    const int nrow = min(TY, T.y1 - ybase);
    const int nline = (nrow + 1) / 2;
    const int nyt = T.ny(), nzt = T.nz();
    // stage the half spectra as [c][r][k] in buf1 (pitch >= L + 2 makes it fit)
    cplx<R> *stage = buf1;
    for (int e = threadIdx.x; e < nc * hx * nrow; e += blockDim.x) {
        const int r = e % nrow;
        const int rest = e / nrow;
        const int k = rest % hx;
        const int cc = rest / hx;
        stage[(cc * TY + r) * hx + k] =
            C[((long long)(cc * hx + k) * nzt + zrel) * nyt + (ybase - T.y0 + r)];
    }
    __syncthreads();
    const int hL = L / 2;
    for (int e = threadIdx.x; e < nc * nline * L; e += blockDim.x) {
        const int pos = e % L;
        const int rest = e / L;
        const int l = rest % nline;
        const int cc = rest / nline;
        const int rA = 2 * l, rB = 2 * l + 1;
        cplx<R> a, b;
        if (pos <= hL) {
            a = stage[(cc * TY + rA) * hx + pos];
            b = rB < nrow ? stage[(cc * TY + rB) * hx + pos] : cplx<R>{0, 0};
            if (pos == 0 || pos == hL) {
                a.y = 0;
                b.y = 0;
            }
        } else {
            const int q = L - pos;
            a = cconj(stage[(cc * TY + rA) * hx + q]);
            b = rB < nrow ? cconj(stage[(cc * TY + rB) * hx + q]) : cplx<R>{0, 0};
        }
        buf0[(cc * nline + l) * pitch + pos] = cplx<R>{a.x - b.y, a.y + b.x};
    }
    __syncthreads();
    const cplx<R> *res = fft_lines_lds(buf0, buf1, nc * nline, pitch, plan, true);
    if (!grad_epi) {
        const int nxt = T.nx();
        for (int e = threadIdx.x; e < nc * nrow * nxt; e += blockDim.x) {
            const int xq = e % nxt;
            const int rest = e / nxt;
            const int r = rest % nrow;
            const int cc = rest / nrow;
            const cplx<R> v = res[(cc * nline + (r >> 1)) * pitch + T.x0 + xq];
            const int y = ybase + r;
            out.ptr[cc * out.cs + (long long)(z - out.oz) * out.zs + (long long)(y - out.oy) * out.ys +
                    (T.x0 + xq - out.ox)] = (r & 1) ? v.y : v.x;
        }
    } else {
        const int nx = dsg.nx;
        const long long ncell = (long long)dsg.nx * dsg.ny * dsg.nz;
        const R m0u[3] = {m0u0, m0u1, m0u2};
        for (int e = threadIdx.x; e < nrow * nx; e += blockDim.x) {
            const int x = e % nx;
            const int r = e / nx;
            const int y = ybase + r;
            const long long idx = ((long long)z * dsg.ny + y) * nx + x;
            R gval = 0;
            if (x >= T.x0 && x < T.x1 && dsg.design.has(x, y, z) && (!dsg.mask || dsg.mask[idx])) {
                R s = 0;
                for (int cc = 0; cc < nc; ++cc) {
                    const cplx<R> v = res[(cc * nline + (r >> 1)) * pitch + x];
                    const R a = (r & 1) ? v.y : v.x;
                    const R coef = dsg.m0f ? dsg.m0f[cc * ncell + idx] : m0u[cc];
                    s += coef * a;
                }
                gval = (R)dsg.p * ipow_dev(dsg.rho[idx], dsg.p - 1) * s;
            }
            grad[idx] = gval;
        }
    }
}

// Zero the x rows (y, z) outside keep.y x keep.z: first the whole layers with
// z outside keep.z, then the rows of the kept layers with y outside keep.y.
// Block b writes one row.
// Row q of the (z, y) rows outside `keep` (x spans the grid): first the
// layers outside keep's z range, then the rows of keep's layers outside its
// y range.  There are (nz - keep.nz) ny + keep.nz (ny - keep.ny) of them.
__device__ __forceinline__ void outside_row(int q, int ny, const Box &keep, int &y, int &z)
{
    const int dz = keep.z1 - keep.z0, dy = keep.y1 - keep.y0;
    const int below = keep.z0 * ny;
    if (q < below) {
        z = q / ny;
        y = q % ny;
        return;
    }
    q -= below;
    const int oy = ny - dy;
    if (q < dz * oy) {
        z = keep.z0 + q / oy;
        const int yy = q % oy;
        y = yy < keep.y0 ? yy : keep.y1 + (yy - keep.y0);
        return;
    }
    q -= dz * oy;
    z = keep.z1 + q / ny;
    y = q % ny;
}

__host__ __device__ constexpr long long outside_rows(int ny, int nz, const Box &keep)
{
    return (long long)(nz - keep.nz()) * ny + (long long)keep.nz() * (ny - keep.ny());
}

constexpr int kZeroRowsPerBlock = 8;

template <typename R>
__global__ __launch_bounds__(kThreads) void k_zero_outside(R *a, int nx, int ny, int nz, Box keep)
{
    int y, z;
    outside_row(blockIdx.x, ny, keep, y, z);
    R *row = a + ((long long)z * ny + y) * nx;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) row[x] = (R)0;
}

// dJ/dH_cc at the objective-box cell (x, y, z), and in jterm the cell's term
// of J's sum (zero off the sensor); the same discrete J as k_objective.  H(x, y)
// returns component cc of the field at (x, y, z) for any (x, y) of ob.
template <typename R, typename HF>
__device__ __forceinline__ double objective_cell(const ObjectiveDev<R> &o, int cc, int x, int y, int z, HF H,
                                                 double &jterm)
{
    const Box &sb = o.sb;
    const bool in = sb.has(x, y, z);
    const double invS = o.inv_s;
    const double h = H(x, y);
    if (o.kind == 3) {
        const int s = in ? ((z - sb.z0) * sb.ny() + (y - sb.y0)) * sb.nx() + (x - sb.x0) : 0;
        const double d = h - o.ht[(long long)cc * o.S + s];
        jterm = in ? d * d : 0.0;
        return in ? 2.0 * d * invS : 0.0;
    }
    if (o.kind == 4) {
        jterm = in ? h * h : 0.0;
        return in ? -o.vcell * h : 0.0;
    }
    if (o.kind == 5) {
        // field region (the sensor): Hz^2; strip cells q outside it on the -x, +x
        // and -y sides with outward normal n: lam D^2, D = (Hz(q + n) - Hz(q)) / h_n.
        // dJ/dHz collects -V Hz on the field and the derivative of -1/2 V lam D^2
        // at q (+V lam D / h_n) and at q + n (-V lam D / h_n).
        const double V = o.vcell, beta = o.lam;
        double v = in ? -V * h : 0.0;
        jterm = in ? h * h : 0.0;
        const bool zin = z >= sb.z0 && z < sb.z1;
        const bool yin = zin && y >= sb.y0 && y < sb.y1;
        const bool xin = zin && x >= sb.x0 && x < sb.x1;
        const double rdx = o.rdx, rdy = o.rdy;
        if (yin && x == sb.x0 - 1) {
            const double D = (H(x - 1, y) - h) * rdx;
            jterm += beta * D * D;
            v += V * beta * D * rdx;
        }
        if (yin && x == sb.x0 - 2) v -= V * beta * ((h - H(x + 1, y)) * rdx) * rdx;
        if (yin && x == sb.x1) {
            const double D = (H(x + 1, y) - h) * rdx;
            jterm += beta * D * D;
            v += V * beta * D * rdx;
        }
        if (yin && x == sb.x1 + 1) v -= V * beta * ((h - H(x - 1, y)) * rdx) * rdx;
        if (xin && y == sb.y0 - 1) {
            const double D = (H(x, y - 1) - h) * rdy;
            jterm += beta * D * D;
            v += V * beta * D * rdy;
        }
        if (xin && y == sb.y0 - 2) v -= V * beta * ((h - H(x, y + 1)) * rdy) * rdy;
        return v;
    }
    const double d = h - o.t;
    double v = in ? 2.0 * d * invS : 0.0;
    jterm = in ? d * d : 0.0;
    if (o.kind == 2) {
        // central differences at this cell (its J term) and at the four sensor
        // neighbours whose differences read this cell (the transpose); the
        // divisions by 2 dx, 2 dy as products with their reciprocals
        const double rx = o.rx, ry = o.ry;
        const double gx = (H(x + 1, y) - H(x - 1, y)) * rx;
        const double gy = (H(x, y + 1) - H(x, y - 1)) * ry;
        if (in) jterm += o.lam * (gx * gx + gy * gy);
        const double cxs = o.cxs, cys = o.cys;
        if (sb.has(x - 1, y, z)) v += cxs * ((h - H(x - 2, y)) * rx);
        if (sb.has(x + 1, y, z)) v -= cxs * ((H(x + 2, y) - h) * rx);
        if (sb.has(x, y - 1, z)) v += cys * ((h - H(x, y - 2)) * ry);
        if (sb.has(x, y + 1, z)) v -= cys * ((H(x, y + 2) - h) * ry);
    }
    return v;
}

// ---------------------------------------------------------------------------
// Objective J(H) in FP64 with a fixed-order reduction (deterministic), and
// g = dJ/dH (exact derivative of the discrete J) on the whole objective box.
// Hs: [c_j][ob] dense (c_j = 1: Hz only; 3: Hx, Hy, Hz).
constexpr int kObjThreads = 256;

template <typename R>
__device__ __forceinline__ double hval(const R *Hs, const Box &ob, int cc, int x, int y, int z)
{
    const long long n = (long long)ob.nx() * ob.ny() * ob.nz();
    return (double)Hs[cc * n + ((long long)(z - ob.z0) * ob.ny() + (y - ob.y0)) * ob.nx() + (x - ob.x0)];
}

template <typename R>
__device__ __forceinline__ double dx_at(const R *Hs, const Box &ob, int x, int y, int z, double dx)
{
    return (hval(Hs, ob, 0, x + 1, y, z) - hval(Hs, ob, 0, x - 1, y, z)) / (2.0 * dx);
}

template <typename R>
__device__ __forceinline__ double dy_at(const R *Hs, const Box &ob, int x, int y, int z, double dy)
{
    return (hval(Hs, ob, 0, x, y + 1, z) - hval(Hs, ob, 0, x, y - 1, z)) / (2.0 * dy);
}

// Block b: g on its slice of the objective box, and a partial J over its
// slice of the sensor cells (fixed-order tree in LDS).  The last block to
// finish (ticket counter) adds the partials in block order, writes J and
// re-arms the counter, so J is the same on every run.
template <typename R>
__global__ __launch_bounds__(kObjThreads) void k_objective(int kind, const R *Hs, Box ob, Box sb, int c_j,
                                                         double t, double lam, double dx, double dy,
                                                         double vcell, const double *ht, double *J, R *g,
                                                         double *partials, unsigned int *ticket)
{
    __shared__ double red[kObjThreads];
    __shared__ bool last;
    const int S = sb.nx() * sb.ny() * sb.nz();
    const int nb = gridDim.x;
    double acc = 0.0;
    const long long nob = (long long)ob.nx() * ob.ny() * ob.nz();
    if (kind == 5) {
        // field and strip terms and dJ/dHz per objective-box cell
        ObjectiveDev<R> o{kind, Hs, ob, sb, c_j, nob, S, t, lam, dx, dy, vcell, ht, J, partials, ticket};
        objective_consts(o);
        for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nob;
             q += (long long)nb * blockDim.x) {
            const int x = ob.x0 + (int)(q % ob.nx());
            const int y = ob.y0 + (int)((q / ob.nx()) % ob.ny());
            const int z = ob.z0 + (int)(q / ((long long)ob.nx() * ob.ny()));
            auto H = [&](int xx, int yy) -> double {
                xx = min(max(xx, ob.x0), ob.x1 - 1);
                yy = min(max(yy, ob.y0), ob.y1 - 1);
                return hval(Hs, ob, 0, xx, yy, z);
            };
            double jt;
            g[q] = (R)objective_cell(o, 0, x, y, z, H, jt);
            acc += jt;
        }
    }
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; kind != 5 && s < S; s += nb * blockDim.x) {
        const int x = sb.x0 + s % sb.nx();
        const int y = sb.y0 + (s / sb.nx()) % sb.ny();
        const int z = sb.z0 + s / (sb.nx() * sb.ny());
        if (kind == 3) {
            for (int cc = 0; cc < 3; ++cc) {
                const double d = hval(Hs, ob, cc, x, y, z) - ht[(long long)cc * S + s];
                acc += d * d;
            }
        } else if (kind == 4) {
            const double h = hval(Hs, ob, 0, x, y, z);
            acc += h * h;
        } else {
            const double d = hval(Hs, ob, 0, x, y, z) - t;
            acc += d * d;
            if (kind == 2) {
                const double gx = dx_at(Hs, ob, x, y, z, dx);
                const double gy = dy_at(Hs, ob, x, y, z, dy);
                acc += lam * (gx * gx + gy * gy);
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }

    const double invS = 1.0 / (double)S;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; kind != 5 && q < c_j * nob;
         q += (long long)nb * blockDim.x) {
        const int cc = (int)(q / nob);
        const long long w = q % nob;
        const int x = ob.x0 + (int)(w % ob.nx());
        const int y = ob.y0 + (int)((w / ob.nx()) % ob.ny());
        const int z = ob.z0 + (int)(w / ((long long)ob.nx() * ob.ny()));
        const bool in = sb.has(x, y, z);
        double v = 0.0;
        if (kind == 3) {
            if (in) {
                const int s = ((z - sb.z0) * sb.ny() + (y - sb.y0)) * sb.nx() + (x - sb.x0);
                v = 2.0 * (hval(Hs, ob, cc, x, y, z) - ht[(long long)cc * S + s]) * invS;
            }
        } else if (kind == 4) {
            if (in) v = -vcell * hval(Hs, ob, 0, x, y, z);
        } else {
            if (in) v = 2.0 * (hval(Hs, ob, 0, x, y, z) - t) * invS;
            if (kind == 2) {
                // transpose of the central differences: the sensor cells s = (x -+ 1, y)
                // and (x, y -+ 1) whose difference reads this cell
                const double cxs = lam * invS / dx, cys = lam * invS / dy;
                if (sb.has(x - 1, y, z)) v += cxs * dx_at(Hs, ob, x - 1, y, z, dx);
                if (sb.has(x + 1, y, z)) v -= cxs * dx_at(Hs, ob, x + 1, y, z, dx);
                if (sb.has(x, y - 1, z)) v += cys * dy_at(Hs, ob, x, y - 1, z, dy);
                if (sb.has(x, y + 1, z)) v -= cys * dy_at(Hs, ob, x, y + 1, z, dy);
            }
        }
        g[q] = (R)v;
    }

    if (threadIdx.x == 0) {
        partials[blockIdx.x] = red[0];
        __threadfence();
        last = atomicAdd(ticket, 1u) == (unsigned int)(nb - 1);
    }
    __syncthreads();
    if (last) {
        // the block sums into LDS by all threads at once, then added in block order
        __shared__ double sums[kObjMaxBlocks];
        __threadfence();
        for (int b = threadIdx.x; b < nb; b += blockDim.x) sums[b] = partials[b];
        __syncthreads();
        if (threadIdx.x == 0) {
            double total = 0.0;
            for (int b = 0; b < nb; ++b) total += sums[b];
            if (J) *J = (kind == 4 || kind == 5) ? -0.5 * vcell * total : total / (double)S;
            *ticket = 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// The objective fused with the adjoint's x pass (see launch_objective_xf).

// Block: one row pair (y, y + 1) of ob at one z, one component; NLN = 3
// lines of P threads.  The field rows the pair needs (with the stencil's
// reach) come straight from the forward convolution: line slot l transforms
// rows ty0 + 2l, ty0 + 2l + 1 back along x from their kx spectra (nsum
// copies sum_stride apart, added in order; [cc][kx][zrel][y], or with kxf
// [cc][zrel][y][kx]), so the field is never stored.
template <typename R, int L, int E>
__global__ __launch_bounds__(3 * (L / E)) void k_objective_xf(ObjectiveDev<R> o, cplx<R> *out, int hx,
                                                            const cplx<R> *table, const cplx<R> *spec, int nsum,
                                                            long long sum_stride, int kxf)
{
#define TOF_BX ((int)blockIdx.x)
#define TOF_BY ((int)blockIdx.y)
#define TOF_BZ ((int)blockIdx.z)
#define TOF_BGX ((int)gridDim.x)
#define TOF_BGY ((int)gridDim.y)
#define TOF_BGZ ((int)gridDim.z)
#include "body_objective_xf.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

template <typename R, int L, int E>
__global__ __launch_bounds__(3 * (L / E)) void k_objective_xf_batch(const ObjXfArgs<R> *__restrict__ tab,
                                                                   const int *__restrict__ starts, int n)
{
    BlockPos bp;
    const ObjXfArgs<R> a = batch_args(tab, starts, n, bp);
    const auto &o = a.o;
    const auto &out = a.out;
    const auto &hx = a.hx;
    const auto &table = a.table;
    const auto &spec = a.spec;
    const auto &nsum = a.nsum;
    const auto &sum_stride = a.sum_stride;
    const auto &kxf = a.kxf;
#define TOF_BX (bp.x_)
#define TOF_BY (bp.y_)
#define TOF_BZ (bp.z_)
#define TOF_BGX (bp.gx_)
#define TOF_BGY (bp.gy_)
#define TOF_BGZ (bp.gz_)
#include "body_objective_xf.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

// One wave: J from the objective's block sums.
__global__ __launch_bounds__(64) void k_finalize_j(JFinal jf) { finalize_j(jf); }

// ---------------------------------------------------------------------------
// Projected gradient step on the design cells chi (box and mask):
// rho <- clamp(rho - alpha grad / G, 0, 1), G = max over chi of |grad|.
// Two launches and no atomics: every block of the first writes the largest
// |grad| of its cells to part[blockIdx.x] (all nb entries are written, so
// nothing needs clearing between calls), and every block of the second
// reduces the nb partial maxima itself (at most kStepMaxBlocks values) before
// moving its cells.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_absmax_part(const R *grad, const uint8_t *mask, int nx, int ny, Box d,
                                                        double *part)
{
    const long long n = (long long)d.nx() * d.ny() * d.nz();
    double m = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = d.x0 + (int)(i % d.nx());
        const int y = d.y0 + (int)((i / d.nx()) % d.ny());
        const int z = d.z0 + (int)(i / ((long long)d.nx() * d.ny()));
        const long long idx = ((long long)z * ny + y) * nx + x;
        if (!mask || mask[idx]) m = fmax(m, fabs((double)grad[idx]));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    __shared__ double wmax[kThreads / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wmax[0];
        for (int w = 1; w < kThreads / 64; ++w) b = fmax(b, wmax[w]);
        part[blockIdx.x] = b;
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_project(R *rho, const R *grad, const uint8_t *mask, int nx, int ny,
                                                    Box d, double alpha, const double *part, int nb)
{
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, part[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    __shared__ double wmax[kThreads / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    double gmax = wmax[0];
    for (int w = 1; w < kThreads / 64; ++w) gmax = fmax(gmax, wmax[w]);
    if (!(gmax > 0.0)) return;
    const double step = alpha / gmax;
    const long long n = (long long)d.nx() * d.ny() * d.nz();
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = d.x0 + (int)(i % d.nx());
        const int y = d.y0 + (int)((i / d.nx()) % d.ny());
        const int z = d.z0 + (int)(i / ((long long)d.nx() * d.ny()));
        const long long idx = ((long long)z * ny + y) * nx + x;
        if (mask && !mask[idx]) continue;
        const R v = rho[idx] - (R)(step * (double)grad[idx]);
        rho[idx] = v < (R)0 ? (R)0 : (v > (R)1 ? (R)1 : v);
    }
}

__global__ void k_clear_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Sets *flag to 1 when any of the n values is NaN or infinite.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_nonfinite(const R *a, long long n, unsigned long long *flag)
{
    bool bad = false;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        bad |= !isfinite((double)a[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1ull);
}

// ---------------------------------------------------------------------------
// Tensor setup (FP64, double-double).
__global__ __launch_bounds__(128) void k_newell_lattice(int c, int lx, int ly, int lz, double dx,
                                                      double dy, double dz, double *lat)
{
    const long long n = (long long)lx * ly * lz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % lx);
        const int j = (int)((q / lx) % ly);
        const int k = (int)(q / ((long long)lx * ly));
        // lattice coordinates i*dx exactly (a double-double product is exact)
        const dd X = two_prod((double)i, dx), Y = two_prod((double)j, dy), Z = two_prod((double)k, dz);
        const dd v = newell_component_dd(c, X, Y, Z);
        lat[2 * q] = v.hi;
        lat[2 * q + 1] = v.lo;
    }
}

// N_c(k) for 0 <= k < m: separable (-1, 2, -1) second difference of the
// lattice values, times 1/(4 pi V), summed in double-double and rounded once.
// Writes the octant (if `octant`) and/or the wrapped periodic array (if
// `wrapped`): offset -k sits at L - k, with the component's parity sign.
__global__ __launch_bounds__(128) void k_newell_stencil(int c, int mx, int my, int mz, int lx, int ly,
                                                      dd scale, const double *lat, double *wrapped,
                                                      int Lx, int Ly, int Lz, double *octant)
{
    const long long n = (long long)mx * my * mz;
    const bool ox = comp_odd_x(c), oy = comp_odd_y(c), oz = comp_odd_z(c);
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % mx);
        const int j = (int)((q / mx) % my);
        const int k = (int)(q / ((long long)mx * my));
        dd acc = dd_make(0.0);
        for (int sz = -1; sz <= 1; ++sz)
            for (int sy = -1; sy <= 1; ++sy)
                for (int sx = -1; sx <= 1; ++sx) {
                    int a = i + sx, b = j + sy, e = k + sz;
                    int sign = 1;
                    if (a < 0) { a = -a; if (ox) sign = -sign; }
                    if (b < 0) { b = -b; if (oy) sign = -sign; }
                    if (e < 0) { e = -e; if (oz) sign = -sign; }
                    const int w = (sx ? -1 : 2) * (sy ? -1 : 2) * (sz ? -1 : 2) * sign;
                    const long long at = ((long long)e * ly + b) * lx + a;
                    const dd v{lat[2 * at], lat[2 * at + 1]};
                    acc = dd_add(acc, dd_mul_d(v, (double)w));
                }
        const double val = dd_mul(acc, scale).hi;
        if (octant) octant[q] = val;
        if (wrapped) {
            for (int fz = 0; fz < 2; ++fz) {
                if (fz && k == 0) continue;
                for (int fy = 0; fy < 2; ++fy) {
                    if (fy && j == 0) continue;
                    for (int fx = 0; fx < 2; ++fx) {
                        if (fx && i == 0) continue;
                        const int px = fx ? Lx - i : i, py = fy ? Ly - j : j, pz = fz ? Lz - k : k;
                        double s = 1.0;
                        if (fx && ox) s = -s;
                        if (fy && oy) s = -s;
                        if (fz && oz) s = -s;
                        wrapped[((long long)pz * Ly + py) * Lx + px] = s * val;
                    }
                }
            }
        }
    }
}

// Setup self-check of the trace: T[q] += N_c(k) for the octant offsets
// 0 <= k < n (q in C order), read from the wrapped array; after the three
// diagonal components T holds tr N(k), which is 1 at k = 0 (the self term of
// any cuboid) and 0 elsewhere (the Laplacian of 1/r vanishes off the origin).
__global__ __launch_bounds__(kThreads) void k_trace_accumulate(const double *wrapped, int Lx, int Ly, int nx, int ny,
                                                             int nz, double *T)
{
    const long long n = (long long)nx * ny * nz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % nx);
        const int j = (int)((q / nx) % ny);
        const int k = (int)(q / ((long long)nx * ny));
        T[q] += wrapped[((long long)k * Ly + j) * Lx + i];
    }
}

// Largest |T[q] - delta_q0| as bits of a non-negative double (atomic max).
__global__ __launch_bounds__(kThreads) void k_trace_error(const double *T, long long n, unsigned long long *maxbits)
{
    double m = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        m = fmax(m, fabs(T[q] - (q == 0 ? 1.0 : 0.0)));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
}

// The tensor at every signed offset from its octant: out[c][kz + nz - 1]
// [ky + ny - 1][kx + nx - 1] = N_c(|kx|, |ky|, |kz|) times the component's
// parity signs (xy odd in x and y, xz in x and z, yz in y and z).
__global__ __launch_bounds__(kThreads) void k_tensor_full(const double *oct, int nx, int ny, int nz, double *out)
{
    const int fx = 2 * nx - 1, fy = 2 * ny - 1, fz = 2 * nz - 1;
    const long long per = (long long)fx * fy * fz, octn = (long long)nx * ny * nz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < 6 * per;
         q += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(q / per);
        const long long r = q - c * per;
        const int kx = (int)(r % fx) - (nx - 1);
        const int ky = (int)((r / fx) % fy) - (ny - 1);
        const int kz = (int)(r / ((long long)fx * fy)) - (nz - 1);
        double v = oct[c * octn + ((long long)abs(kz) * ny + abs(ky)) * nx + abs(kx)];
        if ((comp_odd_x(c) && kx < 0) != (comp_odd_y(c) && ky < 0) != (comp_odd_z(c) && kz < 0)) v = -v;
        out[q] = v;
    }
}

// One value added to one element (the test hook that perturbs the tensor).
__global__ void k_add_at(double *a, long long idx, double v)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) a[idx] += v;
}

// Real part of the forward transform on the frequency octant, times `scale`,
// rounded to the working precision; also the largest |imag| and |real| (bits).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_extract_spectrum(const cplx<double> *B, int hx, int Ly,
                                                             int Lz, double scale, R *spec, int hkz,
                                                             int ky_pitch, unsigned long long *mx_imag,
                                                             unsigned long long *mx_real)
{
    const int hky = Ly / 2 + 1;
    const long long n = (long long)hx * hkz * hky;
    double mi = 0.0, mr = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int ky = (int)(q % hky);
        const int kz = (int)((q / hky) % hkz);
        const int kx = (int)(q / ((long long)hky * hkz));
        const cplx<double> v = B[((long long)kx * Lz + kz) * Ly + ky];
        spec[((long long)kx * hkz + kz) * ky_pitch + ky] = (R)(scale * v.x);
        mi = fmax(mi, fabs(v.y));
        mr = fmax(mr, fabs(v.x));
    }
    atomicMax(mx_imag, (unsigned long long)__double_as_longlong(mi));
    atomicMax(mx_real, (unsigned long long)__double_as_longlong(mr));
}


// ===========================================================================
// Register-resident variants for power-of-two lengths fixed at compile time.
// Same passes, layouts and epilogues as above; thread p of a line holds
// x[p + P m] (see fft_reg.h).

// -- passes 2 and 4: contiguous lines --------------------------------------
template <typename R, int L, int E, int NL>
__global__ __launch_bounds__(NL *(L / E)) void k_line_reg(const cplx<R> *in, cplx<R> *out, int nlines, int inner,
                                                        long long in_outer, long long in_inner, long long out_outer,
                                                        long long out_inner, int p_in, int n_in, int p_out,
                                                        int n_out, const cplx<R> *table, int inv, BlockMap bin,
                                                        BlockMap bout)
{
    constexpr int P = L / E;
    constexpr int PITCH = regfft::padded_len(L);
    constexpr int NT = regfft::twiddle_count(L, E);
    __shared__ cplx<R> lds[NL * PITCH];
    const int l = line_of_thread<P>();
    const int p = threadIdx.x % P;
    const int line = blockIdx.x * NL + l;
    const bool live = line < nlines;
    cplx<R> tw[NT > 0 ? NT : 1];
    regfft::load_twiddles<R, L, E>(table, p, tw);
    cplx<R> v[E];
    const int lc = live ? line : 0;   // a dead slot reads line 0 and stores nothing
    const long long ib = (long long)(lc / inner) * in_outer + (long long)(lc % inner) * in_inner;
    // addresses clamped into the line: every load issued before the first use
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = in[ib + bin.at(min(max(p + P * m - p_in, 0), n_in - 1))];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int n = p + P * m;
        if (!(live && n >= p_in && n < p_in + n_in)) v[m] = cplx<R>{0, 0};
    }
    regfft::fft_line<R, L, E, true>(v, tw, lds + l * PITCH, p, inv != 0);
    if (live) {
        const long long ob = (long long)(line / inner) * out_outer + (long long)(line % inner) * out_inner;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int n = p + P * m;
            if (n >= p_out && n < p_out + n_out) out[ob + bout.at(n - p_out)] = v[m];
        }
    }
}

// -- pass 3: z FFT, tensor product, inverse z --------------------------------
// Block: TKC consecutive ky columns of one kx; lanes run over the columns so
// every row access is TKC contiguous complex values.  NC = number of tensor
// components the product reads (1: a single projected component; 6: all,
// with zero weights where unused).  A single source row skips the forward
// FFT (its transform is a phase ramp); a single target row replaces the
// inverse FFT by one inverse DFT sum per column.
#ifndef TOF_Z_WAVES_PER_EU
#define TOF_Z_WAVES_PER_EU 1
#endif

template <typename R, int L, int E, int TKC, int CI, int CO, int NC>
__global__ __launch_bounds__(TKC *(L / E)) __attribute__((amdgpu_waves_per_eu(TOF_Z_WAVES_PER_EU))) void k_z_reg(cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs,
                                                      int zt0, int nzt, SpectrumDev<R> spec, ProductDev prod,
                                                      const cplx<R> *table, BlockMap bm)
{
    constexpr int P = L / E;
    constexpr int PITCH = regfft::padded_len(L) + 1;   // odd: columns start on different banks
    constexpr int NT = regfft::twiddle_count(L, E);
    static_assert(CO * P <= PITCH, "reduction area must fit");
    __shared__ cplx<R> lds[TKC * PITCH];
    const int col = threadIdx.x % TKC;
    const int p = threadIdx.x / TKC;
    const int kx = blockIdx.y;
    const int ky = blockIdx.x * TKC + col;
    const bool live = ky < Ly;
    const long long cstride = (long long)hx * Zrows * Ly;
    // this column's element of row z is colp[bm.row * z]
    cplx<R> *colp = B + (long long)kx * Zrows * Ly + bm.col(live ? ky : 0, 0);
    cplx<R> tw[NT > 0 ? NT : 1];
    regfft::load_twiddles<R, L, E>(table, p, tw);
    cplx<R> *my = lds + col * PITCH;

    // tensor spectrum at this thread's frequencies, fetched before the data
    const int hLy = Ly / 2;
    const int kyq = live ? (ky <= hLy ? ky : Ly - ky) : 0;
    const unsigned ysg = ky > hLy ? kSignBit : 0u;
    R K[NC][E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int kz = p + P * m;
        const int kzq = kz <= L / 2 ? kz : L - kz;
        const unsigned zsg = kz > L / 2 ? kSignBit : 0u;
        const long long at = ((long long)kx * spec.hkz + kzq) * spec.ky_pitch + kyq;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int c = NC == 6 ? q : prod.comp[q];
            // parity signs as bit masks, so no branch waits on the load:
            // xy odd in y, xz odd in z, yz odd in y and z
            const unsigned oy = (c == 3 || c == 5) ? ~0u : 0u, oz = (c == 4 || c == 5) ? ~0u : 0u;
            const R v = (NC < 6 || (prod.need >> c & 1)) ? spec.k[c * spec.comp_stride + at] : (R)0;
            K[q][m] = flip_sign(v, (oy & ysg) ^ (oz & zsg));
        }
    }

    cplx<R> X[CI][E];
    if (nzs == 1) {
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const cplx<R> x = live ? colp[i * cstride] : cplx<R>{0, 0};
#pragma unroll
            for (int m = 0; m < E; ++m) X[i][m] = cmul(x, table[((p + P * m) * zs0) & (L - 1)]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < CI; ++i) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int n = p + P * m;
                const int rc = min(max(n - zs0, 0), nzs - 1);
                const cplx<R> xv = colp[i * cstride + (long long)rc * bm.row];
                X[i][m] = (live && n >= zs0 && n < zs0 + nzs) ? xv : cplx<R>{0, 0};
            }
            regfft::fft_line<R, L, E>(X[i], tw, my, p, false);
        }
    }
    // per-frequency product: C_oi = sum_q Wq[o][i][q] K_q
    cplx<R> Y[CO][E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
#pragma unroll
        for (int o = 0; o < CO; ++o) {
            cplx<R> acc{0, 0};
#pragma unroll
            for (int i = 0; i < CI; ++i) {
                R coef = 0;
#pragma unroll
                for (int q = 0; q < NC; ++q) coef += (R)(NC == 6 ? prod.W[o][i][q] : prod.Wq[o][i][q]) * K[q][m];
                acc.x += coef * X[i][m].x;
                acc.y += coef * X[i][m].y;
            }
            Y[o][m] = acc;
        }
    }
    if (nzt == 1) {
        // one target row: inverse DFT at z = zt0, summed over the column's P threads
#pragma unroll
        for (int o = 0; o < CO; ++o) {
            cplx<R> part{0, 0};
#pragma unroll
            for (int m = 0; m < E; ++m) part = cadd(part, cmul(Y[o][m], cconj(table[((p + P * m) * zt0) & (L - 1)])));
            my[o * P + p] = part;
        }
        __syncthreads();
        if (p == 0 && live) {
#pragma unroll
            for (int o = 0; o < CO; ++o) {
                cplx<R> sum{0, 0};
                for (int q = 0; q < P; ++q) sum = cadd(sum, my[o * P + q]);
                colp[o * cstride] = sum;
            }
        }
    } else {
#pragma unroll
        for (int o = 0; o < CO; ++o) {
            regfft::fft_line<R, L, E>(Y[o], tw, my, p, true);
            if (live) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int n = p + P * m;
                    if (n >= zt0 && n < zt0 + nzt) colp[o * cstride + (long long)(n - zt0) * bm.row] = Y[o][m];
                }
            }
        }
    }
}

// -- pass 3 as a direct sum against Kt (few source or few target rows) ------
// Column (kx, ky), rows in B relative to the source / target box.  Kt_q at
// offset d = zt - zs, with the parity signs of its component; imaginary
// components (xz, yz) multiply by i.


// Few target rows: TH threads per column split the source rows; partial
// sums are added in thread order through LDS.
template <typename R, int TKC, int TH, int CI, int CO, int NC, int NR>
__global__ __launch_bounds__(TKC *TH) void k_zsum_gather(cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs,
                                                       int zt0, int nzt, KtDev<R> kt, ProductDev prod, BlockMap bm)
{
    __shared__ cplx<R> red[TH * CO * NR * TKC];
    const int col = threadIdx.x % TKC;
    const int t = threadIdx.x / TKC;
    const int kx = blockIdx.y;
    const int ky = blockIdx.x * TKC + col;
    const bool live = ky < Ly;
    const long long cstride = (long long)hx * Zrows * Ly;
    cplx<R> *colp = B + (long long)kx * Zrows * Ly + bm.col(live ? ky : 0, 0);
    const int kyl = live ? ky : 0;
    cplx<R> acc[NR][CO];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int o = 0; o < CO; ++o) acc[r][o] = cplx<R>{0, 0};
    if (live) {
        // U source rows per round, their loads issued before the arithmetic
        constexpr int U = TOF_ZSUM_U;
        for (int zr0 = t; zr0 < nzs; zr0 += TH * U) {
            cplx<R> x[U][CI];
            R K[U][NR][NC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // clamped rows keep every load in bounds and branch-free
                const int zr = zr0 + u * TH;
                const bool ok = zr < nzs;
                const int zrc = min(zr, nzs - 1);
#pragma unroll
                for (int i = 0; i < CI; ++i) {
                    const cplx<R> xv = colp[i * cstride + (long long)zrc * bm.row];
                    x[u][i] = ok ? xv : cplx<R>{0, 0};
                }
                // rows past nzs carry x = 0; rows r >= nzt are never added
#pragma unroll
                for (int r = 0; r < NR; ++r) kt_at<R, NC>(kt, prod, kx, kyl, zt0 + min(r, nzt - 1) - (zs0 + zrc), K[u][r]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (r < nzt) zsum_mac<R, CI, CO, NC>(prod, K[u][r], x[u], acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int o = 0; o < CO; ++o) red[((t * CO + o) * NR + r) * TKC + col] = acc[r][o];
    __syncthreads();
    if (t == 0 && live) {
        for (int r = 0; r < nzt; ++r)
#pragma unroll
            for (int o = 0; o < CO; ++o) {
                cplx<R> sum{0, 0};
                for (int u = 0; u < TH; ++u) sum = cadd(sum, red[((u * CO + o) * NR + r) * TKC + col]);
                colp[o * cstride + (long long)r * bm.row] = sum;
            }
    }
}

// Few source rows: every thread reads them, then TH threads per column split
// the target rows.  The barrier keeps the in-place writes after all reads.
template <typename R, int TKC, int TH, int CI, int CO, int NC, int NR>
__global__ __launch_bounds__(TKC *TH) void k_zsum_scatter(cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs,
                                                        int zt0, int nzt, KtDev<R> kt, ProductDev prod, BlockMap bm)
{
    const int col = threadIdx.x % TKC;
    const int t = threadIdx.x / TKC;
    const int kx = blockIdx.y;
    const int ky = blockIdx.x * TKC + col;
    const bool live = ky < Ly;
    const long long cstride = (long long)hx * Zrows * Ly;
    cplx<R> *colp = B + (long long)kx * Zrows * Ly + bm.col(live ? ky : 0, 0);
    const int kyl = live ? ky : 0;
    cplx<R> x[NR][CI];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            const cplx<R> xv = colp[i * cstride + (long long)min(r, nzs - 1) * bm.row];
            x[r][i] = (live && r < nzs) ? xv : cplx<R>{0, 0};
        }
    __syncthreads();
    if (!live) return;
    constexpr int U = CI * NC <= 2 ? 16 : 4;
    for (int zr0 = t; zr0 < nzt; zr0 += TH * U) {
        // tensor values of U target rows first, then the sums and stores
        R K[U][NR][NC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // clamped rows: every load in bounds; rows past nzt are never stored
            const int zt = zt0 + min(zr0 + u * TH, nzt - 1);
#pragma unroll
            for (int r = 0; r < NR; ++r) kt_at<R, NC>(kt, prod, kx, kyl, zt - (zs0 + min(r, nzs - 1)), K[u][r]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int zr = zr0 + u * TH;
            if (zr >= nzt) break;
            cplx<R> out[CO];
#pragma unroll
            for (int o = 0; o < CO; ++o) out[o] = cplx<R>{0, 0};
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nzs) zsum_mac<R, CI, CO, NC>(prod, K[u][r], x[r], out);
#pragma unroll
            for (int o = 0; o < CO; ++o) colp[o * cstride + (long long)zr * bm.row] = out[o];
        }
    }
}

// Kt from the x-y transform of the wrapped tensor (B = [kx][Zb rows][ky], plain):
// the real or imaginary part times `scale` for z offsets 0..nz-1, and the
// largest |other part| and |part| (bits) for the setup self-check.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_extract_kt(const cplx<double> *B, int hx, int Ly, int Zb, int nz,
                                                       double scale, int imaginary, R *kt, int ky_pitch,
                                                       unsigned long long *mx_other, unsigned long long *mx_part)
{
    const long long n = (long long)hx * nz * Ly;
    double mo = 0.0, mp = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int ky = (int)(q % Ly);
        const int d = (int)((q / Ly) % nz);
        const int kx = (int)(q / ((long long)Ly * nz));
        const cplx<double> v = B[((long long)kx * Zb + d) * Ly + ky];
        const double part = imaginary ? v.y : v.x, other = imaginary ? v.x : v.y;
        kt[((long long)kx * nz + d) * ky_pitch + ky] = (R)(scale * part);
        mo = fmax(mo, fabs(other));
        mp = fmax(mp, fabs(part));
    }
    atomicMax(mx_other, (unsigned long long)__double_as_longlong(mo));
    atomicMax(mx_part, (unsigned long long)__double_as_longlong(mp));
}

// -- pass 1: real-to-complex FFT along x, transposed store ------------------
// Block: NLC complex lines = 2 NLC source rows of one z (and one component);
// each thread transforms LPT of them in turn.  HALF (design sources only):
// 1: the design rows lie in the lower half of the line (x < L/2, which the
// 2n padding always gives), 2: they fill it exactly; either way the upper
// half is neither loaded nor transformed in the first stage, and with 2 the
// loads need no clamp and no range select.
template <typename R, int L, int E, int NLC, int LPT, int HALF>
__global__ __launch_bounds__((NLC / LPT) * (L / E)) __attribute__((amdgpu_waves_per_eu(TOF_XF_WAVES))) void k_xf_reg(int mode, DesignDev<R> dsg, View4<const R> src,
                                                                Box S, cplx<R> *out, int hx, const cplx<R> *table)
{
#define TOF_BX ((int)blockIdx.x)
#define TOF_BY ((int)blockIdx.y)
#define TOF_BZ ((int)blockIdx.z)
#define TOF_BGX ((int)gridDim.x)
#define TOF_BGY ((int)gridDim.y)
#define TOF_BGZ ((int)gridDim.z)
#include "body_xf_reg.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

template <typename R, int L, int E, int NLC, int LPT, int HALF>
__global__ __launch_bounds__((NLC / LPT) * (L / E)) __attribute__((amdgpu_waves_per_eu(TOF_XF_WAVES))) void k_xf_reg_batch(
    const XfArgs<R> *__restrict__ tab, const int *__restrict__ starts, int n)
{
    BlockPos bp;
    const XfArgs<R> a = batch_args(tab, starts, n, bp);
    const auto &mode = a.mode;
    const auto &dsg = a.dsg;
    const auto &src = a.src;
    const auto &S = a.S;
    const auto &out = a.out;
    const auto &hx = a.hx;
    const auto &table = a.table;
#define TOF_BX (bp.x_)
#define TOF_BY (bp.y_)
#define TOF_BZ (bp.z_)
#define TOF_BGX (bp.gx_)
#define TOF_BGY (bp.gy_)
#define TOF_BGZ (bp.gz_)
#include "body_xf_reg.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

// -- pass 5: complex-to-real inverse FFT along x + epilogue -----------------
// Block: NLC complex lines = 2 NLC target rows of one z, all CO components;
// each thread transforms LPT lines in turn.  HALF: every column the pass
// stores lies in the lower half of the line (x < L/2).
template <typename R, int L, int E, int NLC, int LPT, int CO, bool PS, bool HALF>
__global__ __launch_bounds__((NLC / LPT) * (L / E)) __attribute__((amdgpu_waves_per_eu(CO == 1 && !PS ? (sizeof(R) == 8 ? TOF_XI_WAVES_F64 : TOF_XI_WAVES) : 1))) void k_xi_reg(const cplx<R> *C, int hx, Box T, int grad_epi,
                                                                View4<R> out, DesignDev<R> dsg, R m0u0, R m0u1,
                                                                R m0u2, R *grad, const cplx<R> *table, int zrows,
                                                                int nsum, long long sum_stride)
{
#define TOF_BX ((int)blockIdx.x)
#define TOF_BY ((int)blockIdx.y)
#define TOF_BZ ((int)blockIdx.z)
#define TOF_BGX ((int)gridDim.x)
#define TOF_BGY ((int)gridDim.y)
#define TOF_BGZ ((int)gridDim.z)
#include "body_xi_reg.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

template <typename R, int L, int E, int NLC, int LPT, int CO, bool PS, bool HALF>
__global__ __launch_bounds__((NLC / LPT) * (L / E)) __attribute__((amdgpu_waves_per_eu(CO == 1 && !PS ? (sizeof(R) == 8 ? TOF_XI_WAVES_F64 : TOF_XI_WAVES) : 1))) void k_xi_reg_batch(const XiArgs<R> *__restrict__ tab, const int *__restrict__ starts,
                                                         int n)
{
    BlockPos bp;
    const XiArgs<R> a = batch_args(tab, starts, n, bp);
    const auto &C = a.C;
    const auto &hx = a.hx;
    const auto &T = a.T;
    const auto &grad_epi = a.grad_epi;
    const auto &out = a.out;
    const auto &dsg = a.dsg;
    const auto &m0u0 = a.m0u0;
    const auto &m0u1 = a.m0u1;
    const auto &m0u2 = a.m0u2;
    const auto &grad = a.grad;
    const auto &table = a.table;
    const auto &zrows = a.zrows;
    const auto &nsum = a.nsum;
    const auto &sum_stride = a.sum_stride;
#define TOF_BX (bp.x_)
#define TOF_BY (bp.y_)
#define TOF_BZ (bp.z_)
#define TOF_BGX (bp.gx_)
#define TOF_BGY (bp.gy_)
#define TOF_BGZ (bp.gz_)
#include "body_xi_reg.inc"
#undef TOF_BX
#undef TOF_BY
#undef TOF_BZ
#undef TOF_BGX
#undef TOF_BGY
#undef TOF_BGZ
}

// ---- launch configuration helpers ----

constexpr size_t kLdsBudget = 64 * 1024;

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers

// Complex lines per block (NLC) and lines per thread (LPT) of the register
// x passes, forward (XF) and inverse (XI), for lengths 256 and 512.  At
// 256x256x128 the forward pass runs best with two lines a thread, the
// inverse one (which holds the gradient's accumulators) with one.
#ifndef TOF_XF_NLC512
#define TOF_XF_NLC512 8
#endif
#ifndef TOF_XF_LPT512
#define TOF_XF_LPT512 2
#endif
#ifndef TOF_XI_NLC512
#define TOF_XI_NLC512 8
#endif
#ifndef TOF_XI_LPT512
#define TOF_XI_LPT512 1
#endif
#ifndef TOF_XF_NLC256
#define TOF_XF_NLC256 8
#endif
#ifndef TOF_XF_LPT256
#define TOF_XF_LPT256 1
#endif
#ifndef TOF_XI_NLC256
#define TOF_XI_NLC256 8
#endif
#ifndef TOF_XI_LPT256
#define TOF_XI_LPT256 1
#endif
// FP64 at length 512 (twice the LDS and registers per line)
#ifndef TOF_XF_NLC512_F64
#define TOF_XF_NLC512_F64 TOF_XF_NLC512
#endif
#ifndef TOF_XF_LPT512_F64
#define TOF_XF_LPT512_F64 TOF_XF_LPT512
#endif
#ifndef TOF_XI_NLC512_F64
#define TOF_XI_NLC512_F64 4
#endif
#ifndef TOF_XI_LPT512_F64
#define TOF_XI_LPT512_F64 TOF_XI_LPT512
#endif

template <typename R, int L, int NLC, int LPT, int HALF>
hipError_t launch_xf_reg_h(hipStream_t st, int mode, const DesignDev<R> &dsg, View4<const R> src, Box S, int c_in,
                           const FftPlanDev &plan, cplx<R> *out, int hx, int xtile)
{
    constexpr int E = 8;
    const bool few = (long long)((S.ny() + 2 * NLC - 1) / (2 * NLC)) * S.nz() * c_in < 512;
    if (xtile == kXTilePair || (xtile == kXTileAuto && few)) {
        // few rows: one row pair per block
        dim3 grid((S.ny() + 1) / 2, S.nz(), c_in);
        const XfArgs<R> a{{}, mode, dsg, src, S, out, hx, (const cplx<R> *)plan.tw};
        TOF_LAUNCH_B((k_xf_reg<R, L, E, 1, 1, HALF>), (k_xf_reg_batch<R, L, E, 1, 1, HALF>), grid, dim3(L / E), st, a,
                     mode, dsg, src, S, out, hx, (const cplx<R> *)plan.tw);
        return hipGetLastError();
    }
    dim3 grid((S.ny() + 2 * NLC - 1) / (2 * NLC), S.nz(), c_in);
    const XfArgs<R> a{{}, mode, dsg, src, S, out, hx, (const cplx<R> *)plan.tw};
    TOF_LAUNCH_B((k_xf_reg<R, L, E, NLC, LPT, HALF>), (k_xf_reg_batch<R, L, E, NLC, LPT, HALF>), grid,
                 dim3((NLC / LPT) * (L / E)), st, a, mode, dsg, src, S, out, hx, (const cplx<R> *)plan.tw);
    return hipGetLastError();
}

// Design sources take the HALF forms: 2 when their rows fill exactly x in
// [0, L/2), else 1 when the grid's rows lie in the lower half (always, with
// L >= 2 nx).
template <typename R, int L, int NLC, int LPT>
hipError_t launch_xf_reg(hipStream_t st, int mode, const DesignDev<R> &dsg, View4<const R> src, Box S, int c_in,
                         const FftPlanDev &plan, cplx<R> *out, int hx, int xtile)
{
    const int xl = S.x0 > dsg.design.x0 ? S.x0 : dsg.design.x0;
    const int xh = S.x1 < dsg.design.x1 ? S.x1 : dsg.design.x1;
    if (mode != SRC_ARRAY && xl == 0 && xh == L / 2 && dsg.nx == L / 2)
        return launch_xf_reg_h<R, L, NLC, LPT, 2>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
    if (mode != SRC_ARRAY && dsg.nx <= L / 2)
        return launch_xf_reg_h<R, L, NLC, LPT, 1>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
    return launch_xf_reg_h<R, L, NLC, LPT, 0>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
}

template <typename R>
hipError_t launch_x_forward(hipStream_t st, int mode, const DesignDev<R> &dsg, View4<const R> src,
                            Box S, int c_in, const FftPlanDev &plan, cplx<R> *out, int hx, int xtile)
{
    switch (plan.L) {
    case 32: return launch_xf_reg<R, 32, 16, 1>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
    case 64: return launch_xf_reg<R, 64, 16, 1>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
    case 128: return launch_xf_reg<R, 128, 16, 1>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
    case 256: return launch_xf_reg<R, 256, TOF_XF_NLC256, TOF_XF_LPT256>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
    case 512:
        if constexpr (sizeof(R) == 8)
            return launch_xf_reg<R, 512, TOF_XF_NLC512_F64, TOF_XF_LPT512_F64>(st, mode, dsg, src, S, c_in, plan, out,
                                                                             hx, xtile);
        else
            return launch_xf_reg<R, 512, TOF_XF_NLC512, TOF_XF_LPT512>(st, mode, dsg, src, S, c_in, plan, out, hx, xtile);
    default: break;
    }
    const int L = plan.L;
    const int pitch = L + 1;
    const size_t per_line = 2 * (size_t)pitch * sizeof(cplx<R>);
    int TY = 2 * (int)(kLdsBudget / per_line);
    TY = TY > 32 ? 32 : (TY < 2 ? 2 : TY);
    const size_t lds = (size_t)(TY / 2) * per_line;
    hipError_t e = allow_lds(k_x_forward<R>, lds);
    if (e != hipSuccess) return e;
    dim3 grid((S.ny() + TY - 1) / TY, S.nz(), c_in);
    TOF_LAUNCH(k_x_forward<R>, grid, dim3(kThreads), lds, st, mode, dsg, src, S, plan, out, hx,
                       TY, pitch);
    return hipGetLastError();
}

template <typename R, int L>
hipError_t launch_line_reg(hipStream_t st, const cplx<R> *in, cplx<R> *out, int nlines, int inner,
                           long long in_outer, long long in_inner, long long out_outer, long long out_inner,
                           int p_in, int n_in, int p_out, int n_out, const FftPlanDev &plan, bool inv, BlockMap bin,
                           BlockMap bout)
{
    constexpr int E = 8;
    constexpr int NL = 256 / (L / E);
    if (nlines < 2048) {
        // few lines (the sensor plane): one line per block spreads them over more CUs
        TOF_LAUNCH((k_line_reg<R, L, E, 1>), dim3(nlines), dim3(L / E), 0, st, in, out, nlines, inner,
                           in_outer, in_inner, out_outer, out_inner, p_in, n_in, p_out, n_out,
                           (const cplx<R> *)plan.tw, inv ? 1 : 0, bin, bout);
        return hipGetLastError();
    }
    dim3 grid((nlines + NL - 1) / NL);
    TOF_LAUNCH((k_line_reg<R, L, E, NL>), grid, dim3(256), 0, st, in, out, nlines, inner, in_outer,
                       in_inner, out_outer, out_inner, p_in, n_in, p_out, n_out, (const cplx<R> *)plan.tw,
                       inv ? 1 : 0, bin, bout);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_line_fft(hipStream_t st, const cplx<R> *in, cplx<R> *out, int nlines, int inner,
                           long long in_outer, long long in_inner, long long out_outer,
                           long long out_inner, int p_in, int n_in, int p_out, int n_out,
                           const FftPlanDev &plan, bool inv, BlockMap bin, BlockMap bout)
{
    if (nlines <= 0) return hipSuccess;
#define TOF_LINE_CASE(LL)                                                                                    \
    case LL:                                                                                                 \
        return launch_line_reg<R, LL>(st, in, out, nlines, inner, in_outer, in_inner, out_outer, out_inner, \
                                      p_in, n_in, p_out, n_out, plan, inv, bin, bout);
    switch (plan.L) {
        TOF_LINE_CASE(32)
        TOF_LINE_CASE(64)
        TOF_LINE_CASE(128)
        TOF_LINE_CASE(256)
        TOF_LINE_CASE(512)
    default: break;
    }
#undef TOF_LINE_CASE
    const int pitch = plan.L + 1;
    const size_t per_line = 2 * (size_t)pitch * sizeof(cplx<R>);
    int NL = (int)(kLdsBudget / per_line);
    NL = NL > 16 ? 16 : (NL < 1 ? 1 : NL);
    const size_t lds = (size_t)NL * per_line;
    hipError_t e = allow_lds(k_line_fft<R>, lds);
    if (e != hipSuccess) return e;
    dim3 grid((nlines + NL - 1) / NL);
    TOF_LAUNCH(k_line_fft<R>, grid, dim3(kThreads), lds, st, in, out, nlines, inner, in_outer,
                       in_inner, out_outer, out_inner, p_in, n_in, p_out, n_out, plan, inv ? 1 : 0, NL,
                       pitch, bin, bout);
    return hipGetLastError();
}

#ifndef TOF_Z_TKC32
#define TOF_Z_TKC32 TOF_KB32
#endif
#ifndef TOF_Z_TKC64
#define TOF_Z_TKC64 16
#endif

template <typename R, int L, int E, int CI, int CO, int NC>
hipError_t launch_z_reg(hipStream_t st, cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs, int zt0, int nzt,
                        const SpectrumDev<R> &spec, const ProductDev &prod, const FftPlanDev &plan, BlockMap bm)
{
    constexpr int P = L / E;
    constexpr int TKC0 = sizeof(R) == 4 ? TOF_Z_TKC32 : TOF_Z_TKC64;
    constexpr int TKC = TKC0 * P > 1024 ? 1024 / P : TKC0;
    if (bm.s < 30 && (1 << bm.s) != TKC) return hipErrorInvalidValue;   // a block must own one KB-block
    dim3 grid((Ly + TKC - 1) / TKC, hx);
    TOF_LAUNCH((k_z_reg<R, L, E, TKC, CI, CO, NC>), grid, dim3(TKC * P), 0, st, B, hx, Ly, Zrows, zs0, nzs,
                       zt0, nzt, spec, prod, (const cplx<R> *)plan.tw, bm);
    return hipGetLastError();
}

template <typename R, int L, int E>
hipError_t launch_z_reg_c(hipStream_t st, cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs, int zt0, int nzt,
                          const SpectrumDev<R> &spec, const ProductDev &prod, const FftPlanDev &plan, BlockMap bm)
{
    const int key = prod.c_in * 4 + prod.c_out;
    if (key == 5 && prod.nc == 1)
        return launch_z_reg<R, L, E, 1, 1, 1>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
    switch (key) {
    case 5: return launch_z_reg<R, L, E, 1, 1, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
    case 7: return launch_z_reg<R, L, E, 1, 3, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
    case 13: return launch_z_reg<R, L, E, 3, 1, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
    case 15: return launch_z_reg<R, L, E, 3, 3, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_z_pass(hipStream_t st, cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs,
                         int zt0, int nzt, const SpectrumDev<R> &spec, const ProductDev &prod,
                         bool forward_only, const FftPlanDev &plan, BlockMap bm)
{
    const bool regular = (prod.c_in == 1 || prod.c_in == 3) && (prod.c_out == 1 || prod.c_out == 3);
    if (!forward_only && regular) {
        switch (plan.L) {
        case 32: return launch_z_reg_c<R, 32, 8>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
        case 64: return launch_z_reg_c<R, 64, 8>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
        case 128: return launch_z_reg_c<R, 128, 16>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
        case 256: return launch_z_reg_c<R, 256, 16>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
        case 512: return launch_z_reg_c<R, 512, 16>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, spec, prod, plan, bm);
        default: break;
        }
    }
    const int pitch = plan.L + 1;
    const int cmax = prod.c_in > prod.c_out ? prod.c_in : prod.c_out;
    const size_t per_col = 2 * (size_t)cmax * pitch * sizeof(cplx<R>);
    int TK = (int)(kLdsBudget / per_col);
    TK = TK > 16 ? 16 : (TK < 1 ? 1 : TK);
    const size_t lds = (size_t)TK * per_col;
    hipError_t e = allow_lds(k_z_pass<R>, lds);
    if (e != hipSuccess) return e;
    dim3 grid((Ly + TK - 1) / TK, hx);
    TOF_LAUNCH(k_z_pass<R>, grid, dim3(kThreads), lds, st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt,
                       spec, prod, forward_only ? 1 : 0, plan, TK, pitch, bm);
    return hipGetLastError();
}

template <typename R, int L, int NLC, int LPT>
hipError_t launch_xi_reg(hipStream_t st, const cplx<R> *C, int hx, int c, Box T, const FftPlanDev &plan,
                         bool grad_epilogue, View4<R> out, const DesignDev<R> &dsg, const R *m0u, R *grad, int zrows,
                         int nsum, long long sum_stride, int xtile)
{
    constexpr int E = 8;
    const bool few = (long long)((T.ny() + 2 * NLC - 1) / (2 * NLC)) * T.nz() < 512;
    if (NLC > 1 && (xtile == kXTilePair || (xtile == kXTileAuto && few)))
        return launch_xi_reg<R, L, 1, 1>(st, C, hx, c, T, plan, grad_epilogue, out, dsg, m0u, grad, zrows, nsum,
                                         sum_stride, xtile);
    const int gx = (T.ny() + 2 * NLC - 1) / (2 * NLC);
    // extra block rows for the zero fill, kZeroRowsPerBlock rows each
    const int gz = (int)((zrows + (long long)gx * kZeroRowsPerBlock - 1) / ((long long)gx * kZeroRowsPerBlock));
    dim3 grid(gx, T.nz() + gz);
    dim3 block((NLC / LPT) * (L / E));
    // every stored column in the lower half of the line: the upper half of
    // the last stage and of the epilogue is never formed
    const bool half = T.x1 <= L / 2 && (!grad_epilogue || dsg.nx <= L / 2);
    const XiArgs<R> xa{{}, C, hx, T, grad_epilogue ? 1 : 0, out, dsg, m0u[0], m0u[1], m0u[2], grad,
                       (const cplx<R> *)plan.tw, zrows, nsum, sum_stride};
#define TOF_XI_LAUNCH(CC, PSV, HV)                                                                    \
    TOF_LAUNCH_B((k_xi_reg<R, L, E, NLC, LPT, CC, PSV, HV>), (k_xi_reg_batch<R, L, E, NLC, LPT, CC, PSV, HV>), \
                 grid, block, st, xa, C, hx, T, grad_epilogue ? 1 : 0, out, dsg, m0u[0], m0u[1], m0u[2], grad,      \
                 (const cplx<R> *)plan.tw, zrows, nsum, sum_stride)
#define TOF_XI_LAUNCH_H(CC, PSV)                  \
    do {                                          \
        if (half) TOF_XI_LAUNCH(CC, PSV, true);   \
        else TOF_XI_LAUNCH(CC, PSV, false);       \
    } while (0)
    if (c == 1 && nsum == 1) TOF_XI_LAUNCH_H(1, false);
    else if (c == 1) TOF_XI_LAUNCH_H(1, true);
    else if (c == 3 && nsum == 1) TOF_XI_LAUNCH_H(3, false);
    else if (c == 3) TOF_XI_LAUNCH_H(3, true);
    else return hipErrorInvalidValue;
#undef TOF_XI_LAUNCH_H
#undef TOF_XI_LAUNCH
    return hipGetLastError();
}

template <typename R>
hipError_t launch_x_inverse(hipStream_t st, const cplx<R> *C, int hx, int c, Box T,
                            const FftPlanDev &plan, bool grad_epilogue, View4<R> out,
                            const DesignDev<R> &dsg, const R *m0u, R *grad, bool zero_outside, int nsum,
                            long long sum_stride, int xtile)
{
    if (nsum < 1) return hipErrorInvalidValue;
    const long long zr = grad_epilogue && zero_outside ? outside_rows(dsg.ny, dsg.nz, dsg.design) : 0;
    if (zr > (1LL << 30)) return hipErrorInvalidValue;
    const int zrows = (int)zr;
    if (c == 1 || c == 3) {
        switch (plan.L) {
        case 32: return launch_xi_reg<R, 32, 16, 1>(st, C, hx, c, T, plan, grad_epilogue, out, dsg, m0u, grad, zrows, nsum, sum_stride, xtile);
        case 64: return launch_xi_reg<R, 64, 16, 1>(st, C, hx, c, T, plan, grad_epilogue, out, dsg, m0u, grad, zrows, nsum, sum_stride, xtile);
        case 128:
            return launch_xi_reg<R, 128, 16, 1>(st, C, hx, c, T, plan, grad_epilogue, out, dsg, m0u, grad, zrows, nsum, sum_stride, xtile);
        case 256:
            return launch_xi_reg<R, 256, TOF_XI_NLC256, TOF_XI_LPT256>(st, C, hx, c, T, plan, grad_epilogue, out, dsg, m0u,
                                                                    grad, zrows, nsum, sum_stride, xtile);
        case 512:
            if constexpr (sizeof(R) == 8)
                return launch_xi_reg<R, 512, TOF_XI_NLC512_F64, TOF_XI_LPT512_F64>(st, C, hx, c, T, plan, grad_epilogue,
                                                                                 out, dsg, m0u, grad, zrows, nsum,
                                                                                 sum_stride, xtile);
            else
                return launch_xi_reg<R, 512, TOF_XI_NLC512, TOF_XI_LPT512>(st, C, hx, c, T, plan, grad_epilogue, out, dsg, m0u,
                                                                    grad, zrows, nsum, sum_stride, xtile);
        default: break;
        }
    }
    if (nsum != 1) return hipErrorInvalidValue;   // partial copies: register lengths only
    const int pitch = plan.L + 2;
    const size_t per_line = 2 * (size_t)c * pitch * sizeof(cplx<R>);
    int TY = 2 * (int)(kLdsBudget / per_line);
    TY = TY > 32 ? 32 : (TY < 2 ? 2 : TY);
    const size_t lds = (size_t)(TY / 2) * per_line;
    hipError_t e = allow_lds(k_x_inverse<R>, lds);
    if (e != hipSuccess) return e;
    dim3 grid((T.ny() + TY - 1) / TY, T.nz());
    TOF_LAUNCH(k_x_inverse<R>, grid, dim3(kThreads), lds, st, C, hx, c, T, plan,
                       grad_epilogue ? 1 : 0, out, dsg, m0u[0], m0u[1], m0u[2], grad, TY, pitch);
    e = hipGetLastError();
    if (e != hipSuccess || zrows == 0) return e;
    TOF_LAUNCH(k_zero_outside<R>, dim3(zrows), dim3(kThreads), 0, st, grad, dsg.nx, dsg.ny, dsg.nz, dsg.design);
    return hipGetLastError();
}

#ifndef TOF_NO_COMMON
hipError_t launch_finalize_j(hipStream_t st, const JFinal &jf)
{
    if (!jf.partials || !jf.J || jf.nb < 1) return hipErrorInvalidValue;
    TOF_LAUNCH(k_finalize_j, dim3(1), dim3(64), 0, st, jf);
    return hipGetLastError();
}
#endif

template <typename R>
hipError_t launch_objective_xf(hipStream_t st, const ObjectiveDev<R> &o, const FftPlanDev &plan, cplx<R> *A, int hx,
                              bool check_only, const cplx<R> *spec, int nsum, long long sum_stride, bool kx_fast)
{
    const long long nb = (long long)((o.ob.ny() + 1) / 2) * o.ob.nz() * o.c_j;
    if (nb < 1 || nb > kObjMaxBlocks || o.ob.nz() > 65535 || nsum < 1) return hipErrorInvalidValue;
    if (!check_only && !spec) return hipErrorInvalidValue;
    constexpr int E = 8;
    const dim3 grid((o.ob.ny() + 1) / 2, o.ob.nz(), o.c_j);
    const cplx<R> *tw = (const cplx<R> *)plan.tw;
#define TOF_OBJ_CASE(LL)                                                                                     \
    case LL:                                                                                                 \
        if (check_only) return hipSuccess;                                                                   \
        TOF_LAUNCH_B((k_objective_xf<R, LL, E>), (k_objective_xf_batch<R, LL, E>), grid, dim3(3 * (LL / E)), st, \
                     (ObjXfArgs<R>{{}, o, A, hx, tw, spec, nsum, sum_stride, kx_fast ? 1 : 0}), o, A, hx, tw,   \
                     spec, nsum, sum_stride, kx_fast ? 1 : 0);                                                  \
        return hipGetLastError();
    switch (plan.L) {
        TOF_OBJ_CASE(32)
        TOF_OBJ_CASE(64)
        TOF_OBJ_CASE(128)
        TOF_OBJ_CASE(256)
        TOF_OBJ_CASE(512)
    default: return hipErrorInvalidValue;
    }
#undef TOF_OBJ_CASE
}

template <typename R>
hipError_t launch_objective(hipStream_t st, int kind, const R *Hs, Box ob, Box sensor, int c_j,
                            double target, double lam, double dx, double dy, double vcell,
                            const double *h_target, double *J, R *g, double *partials, unsigned int *ticket)
{
    const long long work = (long long)c_j * ob.nx() * ob.ny() * ob.nz();
    int nb = (int)((work + kObjThreads - 1) / kObjThreads);
    nb = nb < 1 ? 1 : (nb > kObjMaxBlocks ? kObjMaxBlocks : nb);
    TOF_LAUNCH(k_objective<R>, dim3(nb), dim3(kObjThreads), 0, st, kind, Hs, ob, sensor, c_j, target, lam,
                       dx, dy, vcell, h_target, J, g, partials, ticket);
    return hipGetLastError();
}

static int step_blocks(Box design)
{
    const long long n = (long long)design.nx() * design.ny() * design.nz();
    long long blocks = (n + kThreads - 1) / kThreads;
    return (int)(blocks > kStepMaxBlocks ? kStepMaxBlocks : (blocks < 1 ? 1 : blocks));
}

template <typename R>
hipError_t launch_project_step(hipStream_t st, R *rho, const R *grad, const uint8_t *mask, int nx, int ny, int nz,
                               Box design, double alpha, double *part)
{
    (void)nz;
    const int blocks = step_blocks(design);
    TOF_LAUNCH(k_absmax_part<R>, dim3(blocks), dim3(kThreads), 0, st, grad, mask, nx, ny, design, part);
    TOF_LAUNCH(k_project<R>, dim3(blocks), dim3(kThreads), 0, st, rho, grad, mask, nx, ny, design, alpha, part,
               blocks);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_nonfinite(hipStream_t st, const R *a, long long n, unsigned long long *flag)
{
    TOF_LAUNCH(k_clear_u64, dim3(1), dim3(64), 0, st, flag, 1);
    long long blocks = (n + kThreads - 1) / kThreads;
    blocks = blocks > 4096 ? 4096 : (blocks < 1 ? 1 : blocks);
    TOF_LAUNCH(k_nonfinite<R>, dim3((int)blocks), dim3(kThreads), 0, st, a, n, flag);
    return hipGetLastError();
}

#ifndef TOF_NO_COMMON
hipError_t launch_trace_accumulate(hipStream_t st, const double *wrapped, int Lx, int Ly, int nx, int ny, int nz,
                                   double *T)
{
    long long blocks = ((long long)nx * ny * nz + kThreads - 1) / kThreads;
    blocks = blocks > 65536 ? 65536 : blocks;
    TOF_LAUNCH(k_trace_accumulate, dim3((int)blocks), dim3(kThreads), 0, st, wrapped, Lx, Ly, nx, ny, nz, T);
    return hipGetLastError();
}
#endif

#ifndef TOF_NO_COMMON
hipError_t launch_trace_error(hipStream_t st, const double *T, long long n, unsigned long long *maxbits)
{
    TOF_LAUNCH(k_clear_u64, dim3(1), dim3(64), 0, st, maxbits, 1);
    long long blocks = (n + kThreads - 1) / kThreads;
    blocks = blocks > 4096 ? 4096 : (blocks < 1 ? 1 : blocks);
    TOF_LAUNCH(k_trace_error, dim3((int)blocks), dim3(kThreads), 0, st, T, n, maxbits);
    return hipGetLastError();
}
#endif

#ifndef TOF_NO_COMMON
hipError_t launch_tensor_full(hipStream_t st, const double *oct, int nx, int ny, int nz, double *out)
{
    const long long n = 6LL * (2 * nx - 1) * (2 * ny - 1) * (2 * nz - 1);
    long long blocks = (n + kThreads - 1) / kThreads;
    blocks = blocks > 65536 ? 65536 : blocks;
    TOF_LAUNCH(k_tensor_full, dim3((int)blocks), dim3(kThreads), 0, st, oct, nx, ny, nz, out);
    return hipGetLastError();
}
#endif

#ifndef TOF_NO_COMMON
hipError_t launch_add_at(hipStream_t st, double *a, long long idx, double v)
{
    TOF_LAUNCH(k_add_at, dim3(1), dim3(64), 0, st, a, idx, v);
    return hipGetLastError();
}
#endif

#ifndef TOF_NO_COMMON
hipError_t launch_newell_lattice(hipStream_t st, int c, int lx, int ly, int lz, double dx, double dy,
                                 double dz, double *lat)
{
    const long long n = (long long)lx * ly * lz;
    int blocks = (int)((n + 127) / 128);
    blocks = blocks > 65536 ? 65536 : blocks;
    TOF_LAUNCH(k_newell_lattice, dim3(blocks), dim3(128), 0, st, c, lx, ly, lz, dx, dy, dz, lat);
    return hipGetLastError();
}
#endif

#ifndef TOF_NO_COMMON
hipError_t launch_newell_stencil(hipStream_t st, int c, int mx, int my, int mz, int lx, int ly, double dx,
                                 double dy, double dz, const double *lat, double *wrapped, int Lx, int Ly,
                                 int Lz, double *octant)
{
    const long long n = (long long)mx * my * mz;
    int blocks = (int)((n + 127) / 128);
    blocks = blocks > 65536 ? 65536 : blocks;
    const dd scale = inv_4pi_volume(dx, dy, dz);
    TOF_LAUNCH(k_newell_stencil, dim3(blocks), dim3(128), 0, st, c, mx, my, mz, lx, ly, scale, lat,
                       wrapped, Lx, Ly, Lz, octant);
    return hipGetLastError();
}
#endif

template <typename R>
hipError_t launch_extract_spectrum(hipStream_t st, const cplx<double> *B, int hx, int Ly, int Lz,
                                   double scale, R *spec, int hkz, int ky_pitch, unsigned long long *mi,
                                   unsigned long long *mr)
{
    TOF_LAUNCH(k_clear_u64, dim3(1), dim3(64), 0, st, mi, 1);
    TOF_LAUNCH(k_clear_u64, dim3(1), dim3(64), 0, st, mr, 1);
    const long long n = (long long)hx * hkz * (Ly / 2 + 1);
    int blocks = (int)((n + kThreads - 1) / kThreads);
    blocks = blocks > 8192 ? 8192 : blocks;
    TOF_LAUNCH(k_extract_spectrum<R>, dim3(blocks), dim3(kThreads), 0, st, B, hx, Ly, Lz, scale,
                       spec, hkz, ky_pitch, mi, mr);
    return hipGetLastError();
}

template <typename R, int CI, int CO, int NC>
hipError_t launch_zsum_t(hipStream_t st, cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs, int zt0, int nzt,
                         const KtDev<R> &kt, const ProductDev &prod, BlockMap bm)
{
    constexpr int TKC = sizeof(R) == 4 ? TOF_KB32 : 16;
    constexpr int TH = TOF_ZSUM_THREADS / TKC;
    if (bm.s < 30 && (1 << bm.s) != TKC) return hipErrorInvalidValue;   // a block must own one KB-block
    dim3 grid((Ly + TKC - 1) / TKC, hx);
    constexpr int NRM = kZsumMaxRows;
    if (nzt == 1)
        TOF_LAUNCH((k_zsum_gather<R, TKC, TH, CI, CO, NC, 1>), grid, dim3(TKC * TH), 0, st, B, hx, Ly, Zrows,
                           zs0, nzs, zt0, nzt, kt, prod, bm);
    else if (nzt <= NRM)
        TOF_LAUNCH((k_zsum_gather<R, TKC, TH, CI, CO, NC, NRM>), grid, dim3(TKC * TH), 0, st, B, hx, Ly,
                           Zrows, zs0, nzs, zt0, nzt, kt, prod, bm);
    else if (nzs == 1)
        TOF_LAUNCH((k_zsum_scatter<R, TKC, TH, CI, CO, NC, 1>), grid, dim3(TKC * TH), 0, st, B, hx, Ly, Zrows,
                           zs0, nzs, zt0, nzt, kt, prod, bm);
    else if (nzs <= NRM)
        TOF_LAUNCH((k_zsum_scatter<R, TKC, TH, CI, CO, NC, NRM>), grid, dim3(TKC * TH), 0, st, B, hx, Ly,
                           Zrows, zs0, nzs, zt0, nzt, kt, prod, bm);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R>
hipError_t launch_z_sum(hipStream_t st, cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs, int zt0, int nzt,
                        const KtDev<R> &kt, const ProductDev &prod, BlockMap bm)
{
    const int key = prod.c_in * 4 + prod.c_out;
    if (key == 5 && prod.nc == 1)
        return launch_zsum_t<R, 1, 1, 1>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, kt, prod, bm);
    switch (key) {
    case 5: return launch_zsum_t<R, 1, 1, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, kt, prod, bm);
    case 7: return launch_zsum_t<R, 1, 3, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, kt, prod, bm);
    case 13: return launch_zsum_t<R, 3, 1, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, kt, prod, bm);
    case 15: return launch_zsum_t<R, 3, 3, 6>(st, B, hx, Ly, Zrows, zs0, nzs, zt0, nzt, kt, prod, bm);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_extract_kt(hipStream_t st, const cplx<double> *B, int hx, int Ly, int Zb, int nz, double scale,
                             bool imaginary, R *kt, int ky_pitch, unsigned long long *mo, unsigned long long *mp)
{
    TOF_LAUNCH(k_clear_u64, dim3(1), dim3(64), 0, st, mo, 1);
    TOF_LAUNCH(k_clear_u64, dim3(1), dim3(64), 0, st, mp, 1);
    const long long n = (long long)hx * nz * Ly;
    int blocks = (int)((n + kThreads - 1) / kThreads);
    blocks = blocks > 8192 ? 8192 : blocks;
    TOF_LAUNCH(k_extract_kt<R>, dim3(blocks), dim3(kThreads), 0, st, B, hx, Ly, Zb, nz, scale,
                       imaginary ? 1 : 0, kt, ky_pitch, mo, mp);
    return hipGetLastError();
}

#define TOF_INSTANTIATE(R)                                                                              \
    template hipError_t launch_x_forward<R>(hipStream_t, int, const DesignDev<R> &, View4<const R>, Box, \
                                            int, const FftPlanDev &, cplx<R> *, int, int);               \
    template hipError_t launch_line_fft<R>(hipStream_t, const cplx<R> *, cplx<R> *, int, int, long long, \
                                           long long, long long, long long, int, int, int, int,          \
                                           const FftPlanDev &, bool, BlockMap, BlockMap);                \
    template hipError_t launch_z_pass<R>(hipStream_t, cplx<R> *, int, int, int, int, int, int, int,     \
                                         const SpectrumDev<R> &, const ProductDev &, bool,               \
                                         const FftPlanDev &, BlockMap);                                  \
    template hipError_t launch_x_inverse<R>(hipStream_t, const cplx<R> *, int, int, Box,                 \
                                            const FftPlanDev &, bool, View4<R>, const DesignDev<R> &,    \
                                            const R *, R *, bool, int, long long, int);                  \
    template hipError_t launch_objective_xf<R>(hipStream_t, const ObjectiveDev<R> &, const FftPlanDev &,  \
                                               cplx<R> *, int, bool, const cplx<R> *, int, long long,     \
                                               bool);                                                     \
    template hipError_t launch_objective<R>(hipStream_t, int, const R *, Box, Box, int, double, double,  \
                                            double, double, double, const double *, double *, R *,       \
                                            double *, unsigned int *);                                   \
    template hipError_t launch_project_step<R>(hipStream_t, R *, const R *, const uint8_t *, int, int, int, \
                                               Box, double, double *);                                   \
    template hipError_t launch_nonfinite<R>(hipStream_t, const R *, long long, unsigned long long *);      \
    template hipError_t launch_z_sum<R>(hipStream_t, cplx<R> *, int, int, int, int, int, int, int,       \
                                        const KtDev<R> &, const ProductDev &, BlockMap);                 \
    template hipError_t launch_extract_kt<R>(hipStream_t, const cplx<double> *, int, int, int, int, double, \
                                             bool, R *, int, unsigned long long *,                      \
                                             unsigned long long *);                                     \
    template hipError_t launch_extract_spectrum<R>(hipStream_t, const cplx<double> *, int, int, int,     \
                                                   double, R *, int, int, unsigned long long *,          \
                                                   unsigned long long *);

#ifndef TOF_NO_F32
TOF_INSTANTIATE(float)
#endif
#ifndef TOF_NO_F64
TOF_INSTANTIATE(double)
#endif
