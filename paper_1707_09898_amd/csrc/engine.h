// Internal interface between the C-ABI host code (api.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <vector>

#include "fft.h"

struct Box {
    int x0, x1, y0, y1, z0, z1;
    __host__ __device__ int nx() const { return x1 - x0; }
    __host__ __device__ int ny() const { return y1 - y0; }
    __host__ __device__ int nz() const { return z1 - z0; }
    __host__ __device__ bool has(int x, int y, int z) const
    {
        return x >= x0 && x < x1 && y >= y0 && y < y1 && z >= z0 && z < z1;
    }
};

// ky-block width of the y-spectrum buffer in FP32 (FP64 uses 16): 256-byte rows
#ifndef TOF_KB32
#define TOF_KB32 32
#endif

// Element addressing of a ky line in the y-spectrum buffer B, which is
// [c][kx][ky / KB][z][ky % KB] (KB = 2^s; KB = Ly, i.e. s large, is the plain
// [c][kx][z][ky] layout).  Element q of a line is at blk * (q >> s) + (q & mask);
// the element of column ky in row z is at col(ky, z).
struct BlockMap {
    int s;           // log2 KB
    long long blk;   // elements between consecutive KB-blocks (Zrows * KB)
    long long row;   // elements between consecutive z rows (KB)
    __host__ __device__ long long at(int q) const { return blk * (q >> s) + (q & ((1 << s) - 1)); }
    __host__ __device__ long long col(int ky, int z) const { return at(ky) + row * z; }
};

// Where the first (x) pass takes its source values from.
enum SrcMode {
    SRC_RHO_SCALAR = 0,   // chi rho^p          (uniform M0 folded into the spectrum coefficients)
    SRC_RHO_VECTOR = 1,   // chi rho^p M0_c(x)  (spatially varying M0)
    SRC_ARRAY = 2         // src[c][z][y][x] of a strided array
};

// Density / magnetization description shared by the first and last passes.
template <typename R>
struct DesignDev {
    const R *rho;          // [nz][ny][nx]
    const uint8_t *mask;   // optional [nz][ny][nx]
    const R *m0f;          // optional [3][nz][ny][nx]
    Box design;
    int p;
    int nx, ny, nz;
};

// Strided 4-D array view: a[c*cs + (z-oz)*zs + (y-oy)*ys + (x-ox)].
template <typename T>
struct View4 {
    T *ptr;
    long long cs, zs, ys;
    int ox, oy, oz;
};

// Spectrum product coefficients: out_o = sum_i C_oi in_i with
// C = U K V, K the 3x3 symmetric tensor spectrum at the frequency.
struct ProductDev {
    int c_in, c_out;
    double U[3][3];     // [o][a]
    double V[3][3];     // [b][i]
    double W[3][3][6];  // [o][i][c]: C_oi = sum_c W[o][i][c] K_c (U and V folded per component)
    int need;           // bit mask of tensor components (xx, yy, zz, xy, xz, yz) to load
    int nc;             // number of components in `need`
    int comp[6];        // the needed components, in order
    double Wq[3][3][6]; // [o][i][q] = W[o][i][comp[q]]
};

// Octant-compressed real tensor spectra, [6][hx][Lz/2+1][ky_pitch].
template <typename R>
struct SpectrumDev {
    const R *k;
    long long comp_stride;
    int hkz, ky_pitch;
};

// Tensor transformed along x and y only, per z offset d >= 0:
// Kt_c(kx, ky, d) = -FFT2_xy(N_c)(kx, ky, d) / (Lx Ly), stored as
// [6][hx][nz][kt_pitch] over all ky in [0, Ly) (rows aligned to 128 bytes).
// Components even in x (xx, yy, zz, xy) are real; xz and yz (odd in x) are
// imaginary and stored as their imaginary part.  Negative offsets follow by
// parity in z (xz, yz are odd).  With it a z pass whose source or target is
// a few rows becomes out(zt) = sum_zs Kt(zt - zs) x(zs) per (kx, ky) column.
template <typename R>
struct KtDev {
    const R *k;
    long long comp_stride;
    int nzk, ky_pitch;
};

// rows below which the z pass sums against Kt instead of transforming
constexpr int kZsumMaxRows = 4;

// Arguments of the fused y-transform / z-sum kernels (yzsum.hip).
// J from the objective's per-block sums, formed by a later kernel of the
// same evaluation: total = the sums partials[0 .. nb) added in block order,
// J = c total (div 0) or total / c (div 1).  partials null: nothing to form.
struct JFinal {
    const double *partials;
    int nb;
    int div;
    double c;
    double *J;
};

template <typename R>
struct YzSumArgs {
    const cplx<R> *A;        // x-pass output [c_in][hx][nzs][nys]
    cplx<R> *part;           // gather: partial rows [G][c_out][hx][nzt][nyt] (y space),
                             // or [G][c_out][nzt][nyt][hx] with part_kx_fast
    cplx<R> *C;              // scatter: inverse-x input [c_out][hx][nzt][nyt]
    int hx;
    int ys0, nys, zs0, nzs;  // source box rows
    int yt0, nyt, zt0, nzt;  // target box rows
    int rpg;                 // rows per block group: source rows (gather) or target rows (scatter)
    int part_kx_fast;        // gather: partial rows with kx fastest (for the fused objective)
    JFinal jf;               // scatter: J to form first (block (0, 0), one wave), or none
};

// In a batched launch, the block's place in the grid of its design.
struct BlockPos {
    int x_, y_, z_;
    int gx_, gy_, gz_;
};

// Grid of one design's launch; the first member of every argument struct of
// a kernel that can run batched (the batched launch reads it per design).
// The kernels' bodies are in body_*.inc, included in the kernel that runs
// one design and in the batched kernel, so each is compiled in its own
// kernel's context.
struct BatchGrid {
    int gx, gy, gz;
};

// A launch recorded for the batched form: the batched kernel of the same
// instantiation (parameters: const Args *table, const int *starts, int n),
// the launch's own grid and block, and its argument struct.
struct BatchLaunch {
    const void *kernel;
    dim3 grid, block;
    std::vector<unsigned char> args;
};

// While set, the launchers of the batchable kernels append their launch here
// instead of launching, and any other launch sets g_batch_unbatchable to its
// kernel's text and is skipped.
extern thread_local std::vector<BatchLaunch> *g_batch_record;
extern thread_local const char *g_batch_unbatchable;

template <typename A>
inline void batch_record(const void *kernel, dim3 grid, dim3 block, A a)
{
    a.bg = BatchGrid{(int)grid.x, (int)grid.y, (int)grid.z};
    BatchLaunch bl;
    bl.kernel = kernel;
    bl.grid = grid;
    bl.block = block;
    bl.args.resize(sizeof(A));
    std::memcpy(bl.args.data(), &a, sizeof(A));
    g_batch_record->push_back(std::move(bl));
}

// Text of the kernel expression last launched by this thread and its work
// items (grid times block), for the per-launch timing record; set by TOF_LAUNCH.
extern thread_local const char *g_last_kernel;
extern thread_local long long g_last_items;
// While set, the next TOF_LAUNCH takes this event as its kernel's own
// completion timestamp (hipExtLaunchKernelGGL: no packet is added to the
// stream) and clears it; g_prof_launches counts the launches meanwhile and
// g_launch_seq all launches.
extern thread_local hipEvent_t g_prof_stop;
extern thread_local int g_prof_launches;
extern thread_local unsigned long long g_launch_seq;
#define TOF_LAUNCH(K, G, B, SHM, ST, ...)                                                         \
    do {                                                                                          \
        g_last_kernel = #K;                                                                       \
        const dim3 g_ = dim3(G), b_ = dim3(B);                                                    \
        g_last_items = (long long)g_.x * g_.y * g_.z * b_.x * b_.y * b_.z;                        \
        if (g_batch_record) {                                                                     \
            g_batch_unbatchable = #K;                                                             \
            break;                                                                                \
        }                                                                                         \
        ++g_prof_launches;                                                                        \
        ++g_launch_seq;                                                                           \
        if (g_prof_stop) {                                                                        \
            hipExtLaunchKernelGGL(K, g_, b_, SHM, ST, nullptr, g_prof_stop, 0, __VA_ARGS__);      \
            g_prof_stop = nullptr;                                                                \
        } else {                                                                                  \
            hipLaunchKernelGGL(K, g_, b_, SHM, ST, __VA_ARGS__);                                  \
        }                                                                                         \
    } while (0)

// Launch of a batchable kernel K with the kernel arguments that follow A
// (no dynamic LDS), or, while recording, the record of argument struct A
// with the batched kernel KB.
#define TOF_LAUNCH_B(K, KB, G, B, st, A, ...)                                                     \
    do {                                                                                          \
        if (g_batch_record) {                                                                     \
            batch_record(reinterpret_cast<const void *>(KB), dim3(G), dim3(B), A);                \
            break;                                                                                \
        }                                                                                         \
        TOF_LAUNCH(K, G, B, 0, st, __VA_ARGS__);                                                  \
    } while (0)

// ---- host launchers (kernels.hip); all enqueue on `st` and return hipError_t ----

// Tiles of the register x passes (power-of-two lengths): the full tile of
// the length's knobs (several row pairs a block), one row pair a block, or
// (auto) one row pair a block when the full tiles would give fewer than 512
// blocks.
constexpr int kXTileAuto = 0, kXTileFull = 1, kXTilePair = 2;

template <typename R>
hipError_t launch_x_forward(hipStream_t st, int mode, const DesignDev<R> &dsg, View4<const R> src,
                            Box S, int c_in, const FftPlanDev &plan, cplx<R> *out, int hx, int xtile = kXTileAuto);

template <typename R>
hipError_t launch_line_fft(hipStream_t st, const cplx<R> *in, cplx<R> *out, int nlines, int inner,
                           long long in_outer, long long in_inner, long long out_outer,
                           long long out_inner, int p_in, int n_in, int p_out, int n_out,
                           const FftPlanDev &plan, bool inv, BlockMap bin, BlockMap bout);

template <typename R>
hipError_t launch_z_pass(hipStream_t st, cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs,
                         int zt0, int nzt, const SpectrumDev<R> &spec, const ProductDev &prod,
                         bool forward_only, const FftPlanDev &plan, BlockMap bm);

// z pass as a direct sum against Kt; requires nzt <= kZsumMaxRows or nzs <= kZsumMaxRows
template <typename R>
hipError_t launch_z_sum(hipStream_t st, cplx<R> *B, int hx, int Ly, int Zrows, int zs0, int nzs, int zt0, int nzt,
                        const KtDev<R> &kt, const ProductDev &prod, BlockMap bm);

// Passes 2-4 fused (yzsum.hip): the gather (nzt <= kZsumMaxRows) writes
// G = ceil(nzs / rpg) partial copies of the inverse x input into `part`
// (added by launch_x_inverse with nsum = G); the scatter (nzs <=
// kZsumMaxRows) writes C.  Requires a power-of-two Ly in
// [32, 512].  check_only: report whether the case is supported, launch nothing.
template <typename R>
hipError_t launch_yz_sum(hipStream_t st, const YzSumArgs<R> &a, const KtDev<R> &kt, const ProductDev &prod,
                         const FftPlanDev &plan, bool check_only);

template <typename R>
hipError_t launch_extract_kt(hipStream_t st, const cplx<double> *B, int hx, int Ly, int Zb, int nz, double scale,
                             bool imaginary, R *kt, int ky_pitch, unsigned long long *other_max_bits,
                             unsigned long long *part_max_bits);

// zero_outside (with the gradient epilogue, T the design box): also zero the
// gradient rows outside the design box, in the same launch where possible.
// nsum > 1 (power-of-two Lx only): the input is the sum, in order, of nsum
// copies sum_stride elements apart.
template <typename R>
hipError_t launch_x_inverse(hipStream_t st, const cplx<R> *C, int hx, int c, Box T,
                            const FftPlanDev &plan, bool grad_epilogue, View4<R> out,
                            const DesignDev<R> &dsg, const R *m0u, R *grad, bool zero_outside, int nsum = 1,
                            long long sum_stride = 0, int xtile = kXTileAuto);

// blocks the objective kernel may use (partials buffer length)
constexpr int kObjMaxBlocks = 1024;

// The objective's inputs and outputs on the device.
template <typename R>
struct ObjectiveDev {
    int kind;
    const R *Hs;          // [c_j][ob] field on the objective box
    Box ob, sb;           // objective box (sensor grown by the stencil), sensor box
    int c_j;              // field components J reads (1: Hz; 3: Hx, Hy, Hz)
    long long nob;        // cells of ob
    int S;                // sensor cells
    double t, lam, dx, dy, vcell;
    const double *ht;     // [3][sb] target field (kind 3)
    double *J;            // J (one double)
    double *partials;     // kObjMaxBlocks block sums
    unsigned int *ticket; // completion counter, 0 between launches
    // uniform quotients, formed once per launch (objective_consts)
    double inv_s;         // 1 / S
    double rx, ry;        // 1 / (2 dx), 1 / (2 dy)
    double cxs, cys;      // lam / S / dx, lam / S / dy
    double rdx, rdy;      // 1 / dx, 1 / dy
};

template <typename R>
__host__ __device__ inline void objective_consts(ObjectiveDev<R> &o)
{
    o.inv_s = 1.0 / (double)o.S;
    o.rx = 0.5 / o.dx;
    o.ry = 0.5 / o.dy;
    o.cxs = o.lam * o.inv_s / o.dx;
    o.cys = o.lam * o.inv_s / o.dy;
    o.rdx = 1.0 / o.dx;
    o.rdy = 1.0 / o.dy;
}

// The objective fused with the first pass of the adjoint: per row pair of ob,
// dJ/dH from the field, the J terms of its sensor cells (one sum per block
// into o.partials; the caller forms J from them with a JFinal in a later
// kernel), and the real-to-complex FFT along x of
// dJ/dH into A ([c_j][hx][ob.nz][ob.ny], the x-pass layout with source box
// ob).  The field comes straight from the forward convolution's inverse x
// input `spec` [c_j][hx][ob.nz][ob.ny], or the same with kx fastest
// ([c_j][ob.nz][ob.ny][hx], kx_fast), nsum copies sum_stride apart, added in
// order, transformed back along x here.  Needs a power-of-two Lx in
// [32, 512], at most kObjMaxBlocks row pairs and (unless check_only) spec,
// else hipErrorInvalidValue; check_only: report, launch nothing.
template <typename R>
hipError_t launch_objective_xf(hipStream_t st, const ObjectiveDev<R> &o, const FftPlanDev &plan, cplx<R> *A, int hx,
                              bool check_only, const cplx<R> *spec = nullptr, int nsum = 1,
                              long long sum_stride = 0, bool kx_fast = false);

// One wave forms J from the objective's block sums (when no later kernel of
// the evaluation does it).
hipError_t launch_finalize_j(hipStream_t st, const JFinal &jf);

template <typename R>
hipError_t launch_objective(hipStream_t st, int kind, const R *Hs, Box ob, Box sensor, int c_j,
                            double target, double lam, double dx, double dy, double vcell,
                            const double *h_target, double *J, R *g, double *partials, unsigned int *ticket);

// Largest block count of the projected step (size of its partial-maxima buffer).
constexpr int kStepMaxBlocks = 2048;

// rho <- clamp(rho - alpha grad / G, 0, 1) on chi (design box and mask, if
// not null), G = max over chi of |grad|; `part` holds kStepMaxBlocks doubles
// of partial maxima (written by the first launch, read by the second).
template <typename R>
hipError_t launch_project_step(hipStream_t st, R *rho, const R *grad, const uint8_t *mask, int nx, int ny, int nz,
                               Box design, double alpha, double *part);

// *flag (one word) becomes 1 when any of the n values is NaN or infinite, else 0.
template <typename R>
hipError_t launch_nonfinite(hipStream_t st, const R *a, long long n, unsigned long long *flag);

// Setup self-check of the tensor trace (FP64): T += the octant of a wrapped
// component; then the largest |T - delta_0| as double bits.
hipError_t launch_trace_accumulate(hipStream_t st, const double *wrapped, int Lx, int Ly, int nx, int ny, int nz,
                                   double *T);
hipError_t launch_trace_error(hipStream_t st, const double *T, long long n, unsigned long long *maxbits);
hipError_t launch_add_at(hipStream_t st, double *a, long long idx, double v);
// out [6][2nz-1][2ny-1][2nx-1]: the tensor at every signed offset from the octant [6][nz][ny][nx]
hipError_t launch_tensor_full(hipStream_t st, const double *oct, int nx, int ny, int nz, double *out);

hipError_t launch_newell_lattice(hipStream_t st, int c, int lx, int ly, int lz, double dx,
                                 double dy, double dz, double *lat /* [lz][ly][lx][2] */);

hipError_t launch_newell_stencil(hipStream_t st, int c, int mx, int my, int mz, int lx, int ly,
                                 double dx, double dy, double dz, const double *lat,
                                 double *wrapped, int Lx, int Ly, int Lz, double *octant);

template <typename R>
hipError_t launch_extract_spectrum(hipStream_t st, const cplx<double> *B, int hx, int Ly, int Lz,
                                   double scale, R *spec, int hkz, int ky_pitch,
                                   unsigned long long *imag_max_bits, unsigned long long *real_max_bits);
