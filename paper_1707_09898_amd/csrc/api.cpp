// C-ABI host side of the gradient engine: argument validation, FFT plans,
// workspace ownership, the GPU tensor setup and the order of the passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tof.h"
#include "dd.h"
#include "engine.h"

thread_local const char *g_last_kernel = "";
thread_local long long g_last_items = 0;
thread_local std::vector<BatchLaunch> *g_batch_record = nullptr;
thread_local hipEvent_t g_prof_stop = nullptr;
thread_local int g_prof_launches = 0;
thread_local unsigned long long g_launch_seq = 0;
thread_local const char *g_batch_unbatchable = nullptr;

namespace {

thread_local std::string g_thread_error;

constexpr int kMaxL = 1024;

struct Plan1D {
    int L = 0;
    std::vector<int> radix;
    void *tw_f = nullptr;   // cplx<float>[L]
    void *tw_d = nullptr;   // cplx<double>[L]
    FftPlanDev dev(bool f64) const
    {
        FftPlanDev p{};
        p.L = L;
        p.nst = (int)radix.size();
        for (size_t i = 0; i < radix.size(); ++i) p.radix[i] = radix[i];
        p.tw = f64 ? tw_d : tw_f;
        return p;
    }
};

struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct tof_ctx {
    int nx = 0, ny = 0, nz = 0;
    double dx = 1, dy = 1, dz = 1;
    int Lx = 0, Ly = 0, Lz = 0, hx = 0;
    bool f64 = false;
    size_t wsize = 4;   // bytes per real
    Plan1D px, py, pz;
    // spectra [6][hx][hkz][ky_pitch] and x-y transforms [6][hx][nz][ky_pitch], working precision
    DeviceBuf spec, kt;
    int hkz = 0, ky_pitch = 0, kt_pitch = 0;
    long long comp_stride = 0, comp_stride_kt = 0;
    // pass workspaces
    DeviceBuf A, B, C;
    int Zrows = 0;
    BlockMap bmap{};   // layout of B: [c][kx][ky / KB][z][ky % KB]
    // objective buffers
    DeviceBuf Hs, G, Ht;
    DeviceBuf scratch64;          // [0] validation flag
    DeviceBuf steppart;           // projected step: per-block partial maxima (kStepMaxBlocks doubles)
    DeviceBuf partials, ticket;   // objective: per-block partial sums, completion counter (kept at 0)
    bool validate = false;        // hot calls reject non-finite inputs (and synchronize)
    int flags = 0;                // tof_grid.flags
    // design
    bool has_design = false;
    Box design{};
    const uint8_t *mask = nullptr;
    double m0[3] = {0, 0, 1};
    const void *m0f = nullptr;
    int p = 3;
    // objective
    bool has_obj = false;
    int kind = 0;
    Box sensor{}, ob{};
    double target = 0, lam = 0;
    // per-launch timing
    bool prof_on = false;
    int prof_calls[TOF_PROFILE_SLOTS] = {};
    std::vector<hipEvent_t> prof_ev;     // [slot][call]: the launch's stop event
    std::vector<hipEvent_t> prof_refs;   // chain anchors, recorded where a chain of launches starts
    std::vector<int> prof_rec_ref;       // [slot][call]: the anchor of the launch's chain
    std::vector<hipEvent_t> prof_rec_prev;   // [slot][call]: stop event of the launch before it, or null
    int prof_nref = 0, prof_cur_ref = -1;
    hipEvent_t prof_last = nullptr;      // stop event of the last timed launch
    hipStream_t prof_last_st = nullptr;
    unsigned long long prof_last_seq = 0;
    // bursts: the pass of a slot launched again back to back, between two events
    uint32_t prof_burst_mask = 0;
    int prof_burst_reps = 0;
    hipEvent_t prof_burst_ev[TOF_PROFILE_SLOTS][2] = {};
    int prof_burst_done[TOF_PROFILE_SLOTS] = {};
    double prof_bytes[TOF_PROFILE_SLOTS] = {};
    std::string prof_kernel[TOF_PROFILE_SLOTS];
    long long prof_items[TOF_PROFILE_SLOTS] = {};
    // pass choices (tof_set_option)
    bool opt_zsum = true;    // direct z sum against Kt for few source / target rows
    bool opt_fuse = true;    // that sum fused with the y transforms
    bool opt_fuse_obj = true;   // the objective fused with the adjoint's x pass
    int opt_xtile = kXTileAuto;    // tile of the register x passes
    int opt_gather_groups = 0;     // row groups of the fused gather (0: the default rule)
    int opt_scatter_groups = 0;    // row groups of the fused scatter (0: the default rule)
    std::string err;
};

// The batched form: the launches of one gradient evaluation of every design,
// grouped per pass into one launch per kernel instantiation over a device
// table of the designs' arguments.
struct tof_batch {
    struct Group {
        const void *kernel;   // batched kernel: (const Args *table, const int *starts, int n)
        dim3 block;
        int n = 0;             // designs in the group
        long long blocks = 0;  // total blocks of the launch
        void *tab = nullptr;   // device: n argument structs
        int *starts = nullptr; // device: n + 1 first-block indices
    };
    std::vector<std::vector<Group>> passes;
    void *buf = nullptr;   // one device allocation holding every table
    std::string err;
};

// The groups of a pass run one after another on the caller's stream:
// forking them onto side streams and joining back with events measured
// slower (each join left 30-40 us with no kernel running).
void batch_release(tof_batch *b)
{
    if (b->buf) (void)hipFree(b->buf);
    b->buf = nullptr;
}

namespace {

constexpr int kProfCalls = 1024;
constexpr int kProfAnchors = 256;
// largest |tr N(k) - delta_k0| the setup accepts (the FP64 tensor entries are
// each within half an ulp of |N| <= 1 after the double-double evaluation)
constexpr double kTraceTol = 1e-12;
// Row groups of the fused y / z-sum kernels (blocks = groups x (Lx/2+1)).
// At 256x256x128 the evaluation runs best with 3 gather groups among 2 to 6
// (6 makes the gather no faster and the objective kernel, which adds the
// groups' copies, 0.9 us slower), the scatter with 8 among 4, 6, 8 and 16.
#ifndef TOF_YZ_GATHER_GROUPS
#define TOF_YZ_GATHER_GROUPS 3
#endif
#ifndef TOF_YZ_SCATTER_GROUPS
#define TOF_YZ_SCATTER_GROUPS 8
#endif

tof_status fail(tof_ctx *ctx, tof_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    g_thread_error = msg;
    return st;
}

tof_status hip_fail(tof_ctx *ctx, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? TOF_ERR_OOM : TOF_ERR_HIP, m);
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

// Launch through `fn` and, when timing is on, time it.  The stop event of
// the slot goes with the kernel launch (its completion timestamp,
// hipExtLaunchKernelGGL), or is recorded after the last launch when `fn`
// launches several.  A launch whose stream ran a timed launch just before it
// (nothing launched in between) is timed from that launch's end to its own:
// the two ends are read against the anchor of their chain, so no packet is
// added between the kernels.  Where no such launch precedes, an anchor event
// is recorded first and the launch is timed from it (that time also holds
// the anchor's latency).  `bytes` is the pass's algorithmic traffic.
template <typename F>
hipError_t timed_once(tof_ctx *ctx, hipStream_t st, int slot, double bytes, F fn)
{
    if (!ctx->prof_on || ctx->prof_calls[slot] >= kProfCalls) return fn();
    const size_t idx = (size_t)slot * kProfCalls + ctx->prof_calls[slot];
    const bool chained = ctx->prof_last && ctx->prof_last_st == st && ctx->prof_last_seq == g_launch_seq;
    if (!chained) {
        if (ctx->prof_nref >= (int)ctx->prof_refs.size()) return fn();   // out of anchors: not timed
        hipError_t e = hipEventRecord(ctx->prof_refs[ctx->prof_nref], st);
        if (e != hipSuccess) return e;
        ctx->prof_cur_ref = ctx->prof_nref++;
    }
    hipEvent_t stop = ctx->prof_ev[idx];
    g_prof_stop = stop;
    g_prof_launches = 0;
    hipError_t e = fn();
    const bool consumed = g_prof_stop == nullptr;
    g_prof_stop = nullptr;
    if (e != hipSuccess) return e;
    if (!consumed) return hipSuccess;   // nothing was launched: nothing to time
    if (g_prof_launches > 1) {
        e = hipEventRecord(stop, st);
        if (e != hipSuccess) return e;
    }
    ctx->prof_rec_ref[idx] = ctx->prof_cur_ref;
    ctx->prof_rec_prev[idx] = chained ? ctx->prof_last : nullptr;
    ctx->prof_last = stop;
    ctx->prof_last_st = st;
    ctx->prof_last_seq = g_launch_seq;
    ctx->prof_calls[slot]++;
    ctx->prof_bytes[slot] = bytes;
    // the launch expression, e.g. "(k_xi_reg<R, L, ...>)", reduced to the kernel's name
    std::string k = g_last_kernel;
    if (!k.empty() && k[0] == '(') k = k.substr(1);
    ctx->prof_kernel[slot] = k.substr(0, k.find_first_of("<(), "));
    ctx->prof_items[slot] = g_last_items;
    return hipSuccess;
}

// timed_once, then, when a burst is armed for the slot, the same pass again
// prof_burst_reps times back to back between two events.  A repeatable pass
// writes only its outputs, from inputs it does not change, so the repeats
// leave the results as they are; a pass that works in place is not repeated.
template <typename F>
hipError_t timed(tof_ctx *ctx, hipStream_t st, int slot, double bytes, F fn, bool repeatable = true)
{
    hipError_t e = timed_once(ctx, st, slot, bytes, fn);
    if (e != hipSuccess || !ctx->prof_on || !((ctx->prof_burst_mask >> slot) & 1u)) return e;
    if (!repeatable) return hipSuccess;
    ctx->prof_burst_mask &= ~(1u << slot);
    hipEvent_t *bev = ctx->prof_burst_ev[slot];
    if ((e = hipEventRecord(bev[0], st)) != hipSuccess) return e;
    for (int r = 0; r < ctx->prof_burst_reps; ++r)
        if ((e = fn()) != hipSuccess) return e;
    if ((e = hipEventRecord(bev[1], st)) != hipSuccess) return e;
    ctx->prof_burst_done[slot] = ctx->prof_burst_reps;
    return hipSuccess;
}

bool smooth7(int L)
{
    if (L < 1) return false;
    for (int f : {2, 3, 5, 7})
        while (L % f == 0) L /= f;
    return L == 1;
}

// 2n when it is 7-smooth, else the smallest even 7-smooth length >= 2n - 1
// (the real-to-complex pass along x needs an even length; the other axes
// use the same rule for simplicity).
int choose_length(int n)
{
    int L = 2 * n;
    while (!smooth7(L)) L += 2;
    return L;
}

std::vector<int> factor_radices(int L)
{
    std::vector<int> r;
    while (L % 8 == 0) { r.push_back(8); L /= 8; }
    while (L % 4 == 0) { r.push_back(4); L /= 4; }
    while (L % 2 == 0) { r.push_back(2); L /= 2; }
    for (int f : {3, 5, 7})
        while (L % f == 0) { r.push_back(f); L /= f; }
    return r;
}

// Everything tof_create derives from a grid: padded lengths, the layout of
// the spectra and the bytes of every buffer it allocates.
struct GridLayout {
    int L[3] = {0, 0, 0};
    int hx = 0, hkz = 0, ky_pitch = 0, kt_pitch = 0;
    long long comp_stride = 0, comp_stride_kt = 0;
    size_t wsize = 4;
    size_t spec = 0, kt = 0, A = 0, B = 0, C = 0, small = 0;
    size_t total() const { return spec + kt + A + B + C + small; }
};

tof_status grid_layout(const tof_grid &g, GridLayout &out, std::string &err)
{
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > kMaxL / 2 || g.ny > kMaxL / 2 || g.nz > kMaxL / 2) {
        err = "grid sizes must be in [1, 512]";
        return TOF_ERR_INVALID;
    }
    if (!(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0) || !std::isfinite(g.dx) || !std::isfinite(g.dy) ||
        !std::isfinite(g.dz)) {
        err = "cell sizes must be positive and finite";
        return TOF_ERR_INVALID;
    }
    if (g.dtype != TOF_F32 && g.dtype != TOF_F64) {
        err = "dtype must be TOF_F32 or TOF_F64";
        return TOF_ERR_INVALID;
    }
    if (g.validate != 0 && g.validate != 1) {
        err = "validate must be 0 or 1";
        return TOF_ERR_INVALID;
    }
    if (g.flags & ~TOF_GRID_SELFTEST_PERTURB) {
        err = "unknown grid flags";
        return TOF_ERR_INVALID;
    }
    int L[3] = {g.Lx, g.Ly, g.Lz};
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        if (L[a] == 0) L[a] = choose_length(n[a]);
        if (L[a] < 2 * n[a] - 1 || L[a] > kMaxL || !smooth7(L[a]) || (L[a] & 1)) {
            err = "padded length must be even, 7-smooth, >= 2n-1 and <= 1024 (axis " + std::to_string(a) + ")";
            return TOF_ERR_UNSUPPORTED;
        }
        out.L[a] = L[a];
    }
    out.wsize = g.dtype == TOF_F64 ? 8 : 4;
    out.hx = L[0] / 2 + 1;
    out.hkz = L[2] / 2 + 1;
    out.ky_pitch = ((L[1] / 2 + 1) + 15) / 16 * 16;
    out.comp_stride = (long long)out.hx * out.hkz * out.ky_pitch;
    out.kt_pitch = (L[1] + 31) / 32 * 32;
    out.comp_stride_kt = (long long)out.hx * g.nz * out.kt_pitch;
    const size_t cw = 2 * out.wsize;
    out.spec = out.wsize * 6 * (size_t)out.comp_stride;
    out.kt = out.wsize * 6 * (size_t)out.comp_stride_kt;
    out.A = cw * 3 * (size_t)out.hx * g.nz * g.ny;
    out.B = cw * 3 * (size_t)out.hx * g.nz * L[1];
    out.C = cw * 3 * (size_t)out.hx * g.nz * g.ny;
    // twiddle tables (FP32 and FP64 per axis), scratch words, step partials,
    // objective block sums and counter
    size_t tw = 0;
    for (int a = 0; a < 3; ++a) tw += (sizeof(float) + sizeof(double)) * 2 * (size_t)L[a];
    out.small = tw + 64 + sizeof(double) * kStepMaxBlocks + sizeof(double) * kObjMaxBlocks + 64;
    return TOF_OK;
}

tof_status dev_alloc(tof_ctx *ctx, DeviceBuf &b, size_t bytes)
{
    if (b.p && b.bytes >= bytes) return TOF_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) return TOF_OK;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(ctx, TOF_ERR_OOM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
    return TOF_OK;
}

tof_status make_plan(tof_ctx *ctx, Plan1D &pl, int L)
{
    pl.L = L;
    pl.radix = factor_radices(L);
    if ((int)pl.radix.size() > TOF_MAX_STAGES)
        return fail(ctx, TOF_ERR_UNSUPPORTED, "too many FFT stages");
    std::vector<float> tf(2 * L);
    std::vector<double> td(2 * L);
    for (int k = 0; k < L; ++k) {
        // w_L^k = exp(-2 pi i k / L) in extended precision, rounded once
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)L;
        const long double c = cosl(a), s = -sinl(a);
        td[2 * k] = (double)c;
        td[2 * k + 1] = (double)s;
        tf[2 * k] = (float)c;
        tf[2 * k + 1] = (float)s;
    }
    HIP_TRY(ctx, hipMalloc(&pl.tw_f, sizeof(float) * 2 * L));
    HIP_TRY(ctx, hipMalloc(&pl.tw_d, sizeof(double) * 2 * L));
    HIP_TRY(ctx, hipMemcpy(pl.tw_f, tf.data(), sizeof(float) * 2 * L, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(pl.tw_d, td.data(), sizeof(double) * 2 * L, hipMemcpyHostToDevice));
    return TOF_OK;
}

bool box_ok(const Box &b, int nx, int ny, int nz)
{
    return b.x0 >= 0 && b.x1 <= nx && b.y0 >= 0 && b.y1 <= ny && b.z0 >= 0 && b.z1 <= nz && b.x0 < b.x1 &&
           b.y0 < b.y1 && b.z0 < b.z1;
}

Box to_box(const tof_box &b) { return Box{b.x0, b.x1, b.y0, b.y1, b.z0, b.z1}; }

int comp_of(int a, int b)
{
    if (a == b) return a;
    if (a > b) std::swap(a, b);
    if (a == 0) return b == 1 ? 3 : 4;
    return 5;
}

void finish_product(ProductDev &pr)
{
    pr.need = 0;
    std::memset(pr.W, 0, sizeof(pr.W));
    for (int o = 0; o < pr.c_out; ++o)
        for (int i = 0; i < pr.c_in; ++i)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    if (pr.U[o][a] != 0.0 && pr.V[b][i] != 0.0) {
                        const int c = comp_of(a, b);
                        pr.need |= 1 << c;
                        pr.W[o][i][c] += pr.U[o][a] * pr.V[b][i];
                    }
    pr.nc = 0;
    std::memset(pr.Wq, 0, sizeof(pr.Wq));
    for (int c = 0; c < 6; ++c)
        if (pr.need >> c & 1) {
            for (int o = 0; o < 3; ++o)
                for (int i = 0; i < 3; ++i) pr.Wq[o][i][pr.nc] = pr.W[o][i][c];
            pr.comp[pr.nc++] = c;
        }
    for (int q = pr.nc; q < 6; ++q) pr.comp[q] = 0;
}

// ---- one convolution: five passes ----
// slot0 = 0 for the forward convolution, 6 for the adjoint one.
// Where a convolution stopped when its caller takes over the last pass: the
// inverse x pass's input [c][kx][T.z][T.y] (nsum copies sum_stride apart).
struct XTail {
    const void *spec = nullptr;
    int nsum = 1;
    long long stride = 0;
    bool kx_fast = false;   // rows with kx fastest (the fused gather's partials)
};

template <typename R>
// jf (if not null and not yet formed): J from the objective's block sums;
// the fused scatter forms it in its first wave and clears jf->partials.
tof_status convolve(tof_ctx *ctx, hipStream_t st, int slot0, int mode, const DesignDev<R> &dsg,
                    View4<const R> src, Box S, Box T, const ProductDev &prod, bool grad_epi, View4<R> out,
                    const R *m0u, R *grad, bool a_ready = false, XTail *tail = nullptr, JFinal *jf = nullptr)
{
    // the gradient epilogue (T = design box) also zeroes the gradient outside the design box
    const bool zero_rest = grad_epi;
    const bool f64 = sizeof(R) == 8;
    const FftPlanDev plx = ctx->px.dev(f64), ply = ctx->py.dev(f64), plz = ctx->pz.dev(f64);
    cplx<R> *A = (cplx<R> *)ctx->A.p, *B = (cplx<R> *)ctx->B.p, *C = (cplx<R> *)ctx->C.p;
    const int hx = ctx->hx, Ly = ctx->Ly, Zr = ctx->Zrows;
    SpectrumDev<R> sp{(const R *)ctx->spec.p, ctx->comp_stride, ctx->hkz, ctx->ky_pitch};
    // algorithmic bytes of each pass
    const double w = sizeof(R), cw = 2.0 * sizeof(R);
    const double nS = (double)S.nx() * S.ny() * S.nz();
    const double src_bytes = mode == SRC_ARRAY ? prod.c_in * nS * w
                                               : nS * w * (mode == SRC_RHO_VECTOR ? 4.0 : 1.0);
    const double a_elems = (double)prod.c_in * hx * S.nz() * S.ny();
    const double b_in = (double)prod.c_in * hx * S.nz() * Ly;
    const double b_out = (double)prod.c_out * hx * T.nz() * Ly;
    const double c_elems = (double)prod.c_out * hx * T.nz() * T.ny();
    int ncomp = 0;
    for (int c = 0; c < 6; ++c) ncomp += prod.need >> c & 1;
    const double spec_bytes = ncomp * (double)hx * ctx->hkz * (Ly / 2 + 1) * w;
    const double nTrow = (double)T.ny() * T.nz();
    const Box &d = dsg.design;
    const double zero_bytes = zero_rest ? ((double)ctx->nx * ctx->ny * ctx->nz - (double)ctx->nx * d.ny() * d.nz()) * w : 0.0;
    const double x_out = grad_epi ? nTrow * ctx->nx * w * (2.0 + (dsg.m0f ? 3.0 : 0.0)) + zero_bytes
                                  : prod.c_out * nTrow * T.nx() * w;
    if (!a_ready) {   // else the caller's kernel has written the x pass output into A
        HIP_TRY(ctx, timed(ctx, st, slot0 + 0, src_bytes + a_elems * cw, [&] {
            return launch_x_forward<R>(st, mode, dsg, src, S, prod.c_in, plx, A, hx, ctx->opt_xtile);
        }));
    }
    const bool zsum_counts = (prod.c_in == 1 || prod.c_in == 3) && (prod.c_out == 1 || prod.c_out == 3);
    const bool few = ctx->opt_zsum && zsum_counts && (S.nz() <= kZsumMaxRows || T.nz() <= kZsumMaxRows);
    KtDev<R> kt{(const R *)ctx->kt.p, ctx->comp_stride_kt, ctx->nz, ctx->kt_pitch};
    const int drows = std::min(ctx->nz, S.nz() + T.nz() - 1);
    const double kt_bytes = ncomp * (double)hx * drows * Ly * w;
    if (few && ctx->opt_fuse) {
        // y transforms fused with the direct z sum: no y spectra in HBM
        YzSumArgs<R> ya{A, B, C, hx, S.y0, S.ny(), S.z0, S.nz(), T.y0, T.ny(), T.z0, T.nz(), 1, tail ? 1 : 0};
        const bool gather = T.nz() <= kZsumMaxRows;
        const int rows = gather ? S.nz() : T.nz();
        // the gather's partial rows must fit in B
        const int Gopt = gather ? ctx->opt_gather_groups : ctx->opt_scatter_groups;
        int G = std::max(1, std::min(rows, Gopt > 0 ? Gopt : (gather ? TOF_YZ_GATHER_GROUPS : TOF_YZ_SCATTER_GROUPS)));
        // the gather's partial copies of the inverse x input (y space), added by that pass
        const long long part_rows = (long long)prod.c_out * hx * T.nz() * T.ny();
        if (gather) G = (int)std::max(1LL, std::min<long long>(G, (long long)(ctx->B.bytes / sizeof(cplx<R>)) / part_rows));
        ya.rpg = (rows + G - 1) / G;
        G = (rows + ya.rpg - 1) / ya.rpg;
        // the gather leaves G partial copies for the inverse x pass to add: register x lengths only
        const bool x_reg = (ctx->Lx & (ctx->Lx - 1)) == 0 && ctx->Lx >= 32 && ctx->Lx <= 512;
        if ((!gather || x_reg) && launch_yz_sum<R>(st, ya, kt, prod, ply, true) == hipSuccess) {
            const double part_bytes = (double)G * part_rows * cw;
            // the fused kernels read Kt for ky <= Ly/2 only (parity in y gives the rest)
            const double kt_half = ncomp * (double)hx * drows * (Ly / 2 + 1) * w;
            if (gather) {
                HIP_TRY(ctx, timed(ctx, st, slot0 + 2, a_elems * cw + kt_half + part_bytes, [&] {
                    return launch_yz_sum<R>(st, ya, kt, prod, ply, false);
                }));
                if (tail) {
                    *tail = XTail{B, G, part_rows, true};
                    return TOF_OK;
                }
                HIP_TRY(ctx, timed(ctx, st, slot0 + 4, part_bytes + x_out, [&] {
                    return launch_x_inverse<R>(st, B, hx, prod.c_out, T, plx, grad_epi, out, dsg, m0u, grad, zero_rest,
                                               G, part_rows, ctx->opt_xtile);
                }));
                return TOF_OK;
            }
            if (jf && jf->partials) ya.jf = *jf;
            HIP_TRY(ctx, timed(ctx, st, slot0 + 2, a_elems * cw + kt_half + c_elems * cw, [&] {
                return launch_yz_sum<R>(st, ya, kt, prod, ply, false);
            }));
            if (jf) jf->partials = nullptr;
            if (tail) {
                *tail = XTail{C, 1, 0};
                return TOF_OK;
            }
            HIP_TRY(ctx, timed(ctx, st, slot0 + 4, c_elems * cw + x_out, [&] {
                return launch_x_inverse<R>(st, C, hx, prod.c_out, T, plx, grad_epi, out, dsg, m0u, grad, zero_rest, 1,
                                           0, ctx->opt_xtile);
            }));
            return TOF_OK;
        }
    }
    const BlockMap plain{30, 0, 0};
    const BlockMap bm = ctx->bmap;
    HIP_TRY(ctx, timed(ctx, st, slot0 + 1, (a_elems + b_in) * cw, [&] {
        return launch_line_fft<R>(st, A, B, prod.c_in * hx * S.nz(), S.nz(), (long long)S.nz() * S.ny(), S.ny(),
                                  (long long)Zr * Ly, bm.row, S.y0, S.ny(), 0, Ly, ply, false, plain, bm);
    }));
    if (few) {
        // few source or target rows: direct sum against the x-y transformed tensor
        HIP_TRY(ctx, timed(ctx, st, slot0 + 2, (b_in + b_out) * cw + kt_bytes, [&] {
            return launch_z_sum<R>(st, B, hx, Ly, Zr, S.z0, S.nz(), T.z0, T.nz(), kt, prod, bm);
        }, false));
    } else {
        HIP_TRY(ctx, timed(ctx, st, slot0 + 2, (b_in + b_out) * cw + spec_bytes, [&] {
            return launch_z_pass<R>(st, B, hx, Ly, Zr, S.z0, S.nz(), T.z0, T.nz(), sp, prod, false, plz, bm);
        }, false));
    }
    HIP_TRY(ctx, timed(ctx, st, slot0 + 3, (b_out + c_elems) * cw, [&] {
        return launch_line_fft<R>(st, B, C, prod.c_out * hx * T.nz(), T.nz(), (long long)Zr * Ly, bm.row,
                                  (long long)T.nz() * T.ny(), T.ny(), 0, Ly, T.y0, T.ny(), ply, true, bm, plain);
    }));
    if (tail) {
        *tail = XTail{C, 1, 0};
        return TOF_OK;
    }
    HIP_TRY(ctx, timed(ctx, st, slot0 + 4, c_elems * cw + x_out, [&] {
        return launch_x_inverse<R>(st, C, hx, prod.c_out, T, plx, grad_epi, out, dsg, m0u, grad, zero_rest, 1, 0,
                                   ctx->opt_xtile);
    }));
    return TOF_OK;
}

template <typename R>
DesignDev<R> design_dev(const tof_ctx *ctx, const void *rho)
{
    DesignDev<R> d{};
    d.rho = (const R *)rho;
    d.mask = ctx->mask;
    d.m0f = (const R *)ctx->m0f;
    d.design = ctx->design;
    d.p = ctx->p;
    d.nx = ctx->nx;
    d.ny = ctx->ny;
    d.nz = ctx->nz;
    return d;
}

// Forward product: source chi rho^p (uniform M0 folded in via V) or
// chi rho^p M0_c (three components); outputs the components in comps_mask.
ProductDev forward_product(const tof_ctx *ctx, int comps_mask)
{
    ProductDev pr{};
    std::memset(&pr, 0, sizeof(pr));
    if (ctx->m0f) {
        pr.c_in = 3;
        for (int b = 0; b < 3; ++b) pr.V[b][b] = 1.0;
    } else {
        pr.c_in = 1;
        for (int b = 0; b < 3; ++b) pr.V[b][0] = ctx->m0[b];
    }
    int o = 0;
    for (int a = 0; a < 3; ++a)
        if (comps_mask >> a & 1) pr.U[o++][a] = 1.0;
    pr.c_out = o;
    finish_product(pr);
    return pr;
}

// Adjoint product: source = dJ/dH components in comps_mask; output M0 . A
// (one component, uniform M0) or A (three components, varying M0).
ProductDev adjoint_product(const tof_ctx *ctx, int comps_mask)
{
    ProductDev pr{};
    std::memset(&pr, 0, sizeof(pr));
    int i = 0;
    for (int b = 0; b < 3; ++b)
        if (comps_mask >> b & 1) pr.V[b][i++] = 1.0;
    pr.c_in = i;
    if (ctx->m0f) {
        pr.c_out = 3;
        for (int a = 0; a < 3; ++a) pr.U[a][a] = 1.0;
    } else {
        pr.c_out = 1;
        for (int a = 0; a < 3; ++a) pr.U[0][a] = ctx->m0[a];
    }
    finish_product(pr);
    return pr;
}

int popcount3(int m) { return (m & 1) + (m >> 1 & 1) + (m >> 2 & 1); }

template <typename R>
tof_status adjoint_to_grad(tof_ctx *ctx, hipStream_t st, const void *rho, View4<const R> src, Box S,
                           int comps_mask, void *grad, bool a_ready = false, JFinal *jf = nullptr)
{
    DesignDev<R> dsg = design_dev<R>(ctx, rho);
    ProductDev pr = adjoint_product(ctx, comps_mask);
    const R one[3] = {(R)1, (R)0, (R)0};
    View4<R> none{};
    // the last pass also zeroes the gradient outside the design box
    tof_status s = convolve<R>(ctx, st, 6, SRC_ARRAY, dsg, src, S, ctx->design, pr, true, none, one, (R *)grad,
                               a_ready, nullptr, jf);
    if (s != TOF_OK || !jf || !jf->partials) return s;
    // no kernel of the adjoint formed J: a wave of its own does
    HIP_TRY(ctx, timed(ctx, st, 11, 8.0 * jf->nb + 8.0, [&] { return launch_finalize_j(st, *jf); }));
    return TOF_OK;
}

template <typename R>
tof_status run_field(tof_ctx *ctx, hipStream_t st, const void *rho, void *H, int comps_mask)
{
    DesignDev<R> dsg = design_dev<R>(ctx, rho);
    ProductDev pr = forward_product(ctx, comps_mask);
    const long long n = (long long)ctx->nx * ctx->ny * ctx->nz;
    View4<R> out{(R *)H, n, (long long)ctx->ny * ctx->nx, ctx->nx, 0, 0, 0};
    View4<const R> nosrc{};
    const Box all{0, ctx->nx, 0, ctx->ny, 0, ctx->nz};
    const R zero3[3] = {0, 0, 0};
    return convolve<R>(ctx, st, 0, ctx->m0f ? SRC_RHO_VECTOR : SRC_RHO_SCALAR, dsg, nosrc, ctx->design, all, pr,
                       false, out, zero3, nullptr);
}

template <typename R>
tof_status run_objective_and_grad(tof_ctx *ctx, hipStream_t st, const void *rho, double *J, void *grad)
{
    DesignDev<R> dsg = design_dev<R>(ctx, rho);
    const int jmask = ctx->kind == TOF_J_MEAN_SQ_H_TARGET ? 7 : 4;
    const int cj = popcount3(jmask);
    const Box ob = ctx->ob;
    const long long nob = (long long)ob.nx() * ob.ny() * ob.nz();
    ProductDev pf = forward_product(ctx, jmask);
    View4<R> hs{(R *)ctx->Hs.p, nob, (long long)ob.ny() * ob.nx(), ob.nx(), ob.x0, ob.y0, ob.z0};
    View4<const R> nosrc{};
    const R zero3[3] = {0, 0, 0};
    const int mode = ctx->m0f ? SRC_RHO_VECTOR : SRC_RHO_SCALAR;
    if (ctx->opt_fuse_obj) {
        // the forward stops before its inverse x pass; the objective kernel
        // transforms the field rows it needs back along x itself, evaluates J
        // and dJ/dH and transforms dJ/dH along x into A for the adjoint
        ObjectiveDev<R> o{ctx->kind, (const R *)ctx->Hs.p, ob, ctx->sensor, cj, nob,
                          ctx->sensor.nx() * ctx->sensor.ny() * ctx->sensor.nz(), ctx->target, ctx->lam, ctx->dx,
                          ctx->dy, ctx->dx * ctx->dy * ctx->dz, (const double *)ctx->Ht.p, J,
                          (double *)ctx->partials.p, (unsigned int *)ctx->ticket.p};
        objective_consts(o);
        const FftPlanDev plx = ctx->px.dev(sizeof(R) == 8);
        cplx<R> *A = (cplx<R> *)ctx->A.p;
        if (launch_objective_xf<R>(st, o, plx, A, ctx->hx, true) == hipSuccess) {
            XTail tail;
            tof_status s = convolve<R>(ctx, st, 0, mode, dsg, nosrc, ctx->design, ob, pf, false, hs, zero3, nullptr,
                                       false, &tail);
            if (s != TOF_OK) return s;
            const double ht_bytes = ctx->kind == TOF_J_MEAN_SQ_H_TARGET ? 3.0 * o.S * 8.0 : 0.0;
            // the spectra of the pair and its stencil rows (up to 3x the pairs' rows), all copies; dJ/dH spectra out
            const double rows_read = std::min(3.0 * ob.ny(), ob.ny() + 4.0 * ((ob.ny() + 1) / 2));
            const double fbytes = tail.nsum * cj * ctx->hx * ob.nz() * rows_read * 2.0 * sizeof(R) + ht_bytes +
                                  2.0 * sizeof(R) * cj * ctx->hx * ob.nz() * ob.ny();
            HIP_TRY(ctx, timed(ctx, st, 5, fbytes, [&] {
                return launch_objective_xf<R>(st, o, plx, A, ctx->hx, false, (const cplx<R> *)tail.spec, tail.nsum,
                                              tail.stride, tail.kx_fast);
            }));
            View4<const R> nosrc2{};
            // J from the objective's block sums, formed by the adjoint's fused
            // scatter (its first kernel) or a kernel of its own; nothing when
            // the caller passes no J
            const bool half_vsum = ctx->kind == TOF_J_NEG_HALF_HZ2 || ctx->kind == TOF_J_FIELD_GRADIENT;
            JFinal jf{(const double *)ctx->partials.p, (int)(((ob.ny() + 1) / 2) * ob.nz() * cj), half_vsum ? 0 : 1,
                      half_vsum ? -0.5 * o.vcell : (double)o.S, J};
            return adjoint_to_grad<R>(ctx, st, rho, nosrc2, ob, jmask, grad, true, J ? &jf : nullptr);
        }
    }
    tof_status s = convolve<R>(ctx, st, 0, mode, dsg, nosrc, ctx->design, ob, pf, false, hs, zero3, nullptr);
    if (s != TOF_OK) return s;
    const double obytes = 2.0 * cj * nob * sizeof(R);
    HIP_TRY(ctx, timed(ctx, st, 5, obytes, [&] {
        return launch_objective<R>(st, ctx->kind, (const R *)ctx->Hs.p, ob, ctx->sensor, cj, ctx->target, ctx->lam,
                                   ctx->dx, ctx->dy, ctx->dx * ctx->dy * ctx->dz, (const double *)ctx->Ht.p, J,
                                   (R *)ctx->G.p, (double *)ctx->partials.p, (unsigned int *)ctx->ticket.p);
    }));
    View4<const R> gsrc{(const R *)ctx->G.p, nob, (long long)ob.ny() * ob.nx(), ob.nx(), ob.x0, ob.y0, ob.z0};
    return adjoint_to_grad<R>(ctx, st, rho, gsrc, ob, jmask, grad);
}

// ---- tensor setup ----
tof_status compute_spectra(tof_ctx *ctx, hipStream_t st)
{
    const int nx = ctx->nx, ny = ctx->ny, nz = ctx->nz;
    const int Lx = ctx->Lx, Ly = ctx->Ly, Lz = ctx->Lz, hx = ctx->hx;
    const int lx = nx + 1, ly = ny + 1, lz = nz + 1;
    DeviceBuf lat, W, A64, B64, bits, T;
    struct Guard {
        DeviceBuf *b[6];
        ~Guard()
        {
            for (DeviceBuf *x : b)
                if (x->p) (void)hipFree(x->p);
        }
    } guard{{&lat, &W, &A64, &B64, &bits, &T}};
    tof_status s;
    const long long noct = (long long)nx * ny * nz;
    if ((s = dev_alloc(ctx, T, sizeof(double) * (size_t)noct)) != TOF_OK) return s;
    HIP_TRY(ctx, hipMemsetAsync(T.p, 0, T.bytes, st));
    if ((s = dev_alloc(ctx, lat, sizeof(double) * 2 * (size_t)lx * ly * lz)) != TOF_OK) return s;
    if ((s = dev_alloc(ctx, W, sizeof(double) * (size_t)Lx * Ly * Lz)) != TOF_OK) return s;
    if ((s = dev_alloc(ctx, A64, sizeof(cplx<double>) * (size_t)hx * Lz * Ly)) != TOF_OK) return s;
    if ((s = dev_alloc(ctx, B64, sizeof(cplx<double>) * (size_t)hx * Lz * Ly)) != TOF_OK) return s;
    if ((s = dev_alloc(ctx, bits, 2 * sizeof(unsigned long long))) != TOF_OK) return s;
    const FftPlanDev plx = ctx->px.dev(true), ply = ctx->py.dev(true), plz = ctx->pz.dev(true);
    const double scale = -1.0 / ((double)Lx * Ly * Lz);
    SpectrumDev<double> nospec{};
    ProductDev fwd{};
    std::memset(&fwd, 0, sizeof(fwd));
    fwd.c_in = fwd.c_out = 1;
    DesignDev<double> nodsg{};
    const Box whole{0, Lx, 0, Ly, 0, Lz};
    View4<const double> wsrc{(const double *)W.p, 0, (long long)Ly * Lx, Lx, 0, 0, 0};
    unsigned long long *mi = (unsigned long long *)bits.p, *mr = mi + 1;
    for (int c = 0; c < 6; ++c) {
        HIP_TRY(ctx, launch_newell_lattice(st, c, lx, ly, lz, ctx->dx, ctx->dy, ctx->dz, (double *)lat.p));
        HIP_TRY(ctx, hipMemsetAsync(W.p, 0, W.bytes, st));
        HIP_TRY(ctx, launch_newell_stencil(st, c, nx, ny, nz, lx, ly, ctx->dx, ctx->dy, ctx->dz,
                                           (const double *)lat.p, (double *)W.p, Lx, Ly, Lz, nullptr));
        if (c == 0 && (ctx->flags & TOF_GRID_SELFTEST_PERTURB))
            HIP_TRY(ctx, launch_add_at(st, (double *)W.p, 0, 1e-9));   // the self term of xx
        if (c < 3) {
            // the trace of the real-space tensor: tr N(k) = delta_k0
            HIP_TRY(ctx, launch_trace_accumulate(st, (const double *)W.p, Lx, Ly, nx, ny, nz, (double *)T.p));
            if (c == 2) {
                HIP_TRY(ctx, launch_trace_error(st, (const double *)T.p, noct, (unsigned long long *)bits.p));
                unsigned long long hb;
                HIP_TRY(ctx, hipMemcpyAsync(&hb, bits.p, sizeof(hb), hipMemcpyDeviceToHost, st));
                HIP_TRY(ctx, hipStreamSynchronize(st));
                double terr;
                std::memcpy(&terr, &hb, 8);
                if (!(terr < kTraceTol))
                    return fail(ctx, TOF_ERR_NUMERIC, "tensor trace self-check failed: max |tr N(k) - delta_k0| = " +
                                                          std::to_string(terr));
            }
        }
        HIP_TRY(ctx, launch_x_forward<double>(st, SRC_ARRAY, nodsg, wsrc, whole, 1, plx, (cplx<double> *)A64.p, hx));
        const BlockMap plain{30, 0, Ly};
        HIP_TRY(ctx, launch_line_fft<double>(st, (const cplx<double> *)A64.p, (cplx<double> *)B64.p, hx * Lz, Lz,
                                             (long long)Lz * Ly, Ly, (long long)Lz * Ly, Ly, 0, Ly, 0, Ly, ply,
                                             false, plain, plain));
        // x-y transform at z offsets 0..nz-1: real for components even in x, imaginary for xz, yz
        const bool imag = (c == 4 || c == 5);
        const double scale2 = -1.0 / ((double)Lx * Ly);
        if (ctx->f64)
            HIP_TRY(ctx, launch_extract_kt<double>(st, (const cplx<double> *)B64.p, hx, Ly, Lz, nz, scale2, imag,
                                                   (double *)ctx->kt.p + c * ctx->comp_stride_kt, ctx->kt_pitch, mi, mr));
        else
            HIP_TRY(ctx, launch_extract_kt<float>(st, (const cplx<double> *)B64.p, hx, Ly, Lz, nz, scale2, imag,
                                                  (float *)ctx->kt.p + c * ctx->comp_stride_kt, ctx->kt_pitch, mi, mr));
        {
            unsigned long long hb[2];
            HIP_TRY(ctx, hipMemcpyAsync(hb, bits.p, sizeof(hb), hipMemcpyDeviceToHost, st));
            HIP_TRY(ctx, hipStreamSynchronize(st));
            double other, part;
            std::memcpy(&other, &hb[0], 8);
            std::memcpy(&part, &hb[1], 8);
            if (!(other <= 1e-9 * part) && part > 0)
                return fail(ctx, TOF_ERR_NUMERIC, "x-y tensor transform of component " + std::to_string(c) +
                                                      " has the wrong phase (ratio " + std::to_string(other / part) + ")");
        }
        HIP_TRY(ctx, launch_z_pass<double>(st, (cplx<double> *)B64.p, hx, Ly, Lz, 0, Lz, 0, Lz, nospec, fwd, true,
                                           plz, plain));
        if (ctx->f64)
            HIP_TRY(ctx, launch_extract_spectrum<double>(st, (const cplx<double> *)B64.p, hx, Ly, Lz, scale,
                                                         (double *)ctx->spec.p + c * ctx->comp_stride, ctx->hkz,
                                                         ctx->ky_pitch, mi, mr));
        else
            HIP_TRY(ctx, launch_extract_spectrum<float>(st, (const cplx<double> *)B64.p, hx, Ly, Lz, scale,
                                                        (float *)ctx->spec.p + c * ctx->comp_stride, ctx->hkz,
                                                        ctx->ky_pitch, mi, mr));
        unsigned long long hb[2];
        HIP_TRY(ctx, hipMemcpyAsync(hb, bits.p, sizeof(hb), hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        double im, re;
        std::memcpy(&im, &hb[0], 8);
        std::memcpy(&re, &hb[1], 8);
        if (!(im <= 1e-9 * re) && re > 0)
            return fail(ctx, TOF_ERR_NUMERIC, "tensor spectrum of component " + std::to_string(c) +
                                                  " is not real (max|imag|/max|real| = " +
                                                  std::to_string(im / re) + ")");
    }
    return TOF_OK;
}

void release(tof_ctx *ctx)
{
    for (hipEvent_t ev : ctx->prof_ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : ctx->prof_refs) (void)hipEventDestroy(ev);
    for (auto &pair : ctx->prof_burst_ev)
        for (hipEvent_t &ev : pair)
            if (ev) {
                (void)hipEventDestroy(ev);
                ev = nullptr;
            }
    ctx->prof_ev.clear();
    ctx->prof_refs.clear();
    DeviceBuf *bufs[] = {&ctx->spec, &ctx->kt, &ctx->A, &ctx->B, &ctx->C, &ctx->Hs, &ctx->G, &ctx->Ht,
                         &ctx->scratch64, &ctx->steppart, &ctx->partials, &ctx->ticket};
    for (DeviceBuf *b : bufs)
        if (b->p) {
            (void)hipFree(b->p);
            b->p = nullptr;
        }
    for (Plan1D *pl : {&ctx->px, &ctx->py, &ctx->pz}) {
        if (pl->tw_f) (void)hipFree(pl->tw_f);
        if (pl->tw_d) (void)hipFree(pl->tw_d);
        pl->tw_f = pl->tw_d = nullptr;
    }
}

tof_status check_ready(tof_ctx *ctx, bool need_obj)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    if (!ctx->has_design) return fail(ctx, TOF_ERR_STATE, "tof_set_design has not been called");
    if (need_obj && !ctx->has_obj) return fail(ctx, TOF_ERR_STATE, "tof_set_objective has not been called");
    return TOF_OK;
}

// With validation on: TOF_ERR_INVALID when any of the n values of `a` is NaN
// or infinite (a device check, then a wait for its one-word result).
template <typename R>
tof_status check_finite(tof_ctx *ctx, hipStream_t st, const void *a, long long n, const char *what)
{
    if (!ctx->validate) return TOF_OK;
    unsigned long long *flag = (unsigned long long *)ctx->scratch64.p;
    HIP_TRY(ctx, launch_nonfinite<R>(st, (const R *)a, n, flag));
    unsigned long long h = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (h) return fail(ctx, TOF_ERR_INVALID, std::string(what) + " holds NaN or infinite values");
    return TOF_OK;
}

tof_status check_finite_any(tof_ctx *ctx, hipStream_t st, const void *a, long long n, const char *what)
{
    return ctx->f64 ? check_finite<double>(ctx, st, a, n, what) : check_finite<float>(ctx, st, a, n, what);
}

// Scratch of tof_project_step_static: the partial maxima of its first
// launch.  Every GPU the library runs on holds its own copy of this array
// until the process ends; host code never uses its name as an address, only
// the per-device pointer from hipGetSymbolAddress (static_scratch_ptr).
static __device__ __align__(256) double scratch[kStepMaxBlocks];

constexpr int kMaxDevices = 64;

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept; nullptr on failure (msg says why).
double *static_scratch_ptr(std::string &msg)
{
    static std::mutex mu;
    static void *ptrs[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        msg = std::string("hipGetDevice: ") + (e != hipSuccess ? hipGetErrorString(e) : "device index out of range");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        ptrs[dev] = p;
    }
    return (double *)ptrs[dev];
}

}  // namespace

extern "C" {

tof_status tof_create(const tof_grid *grid, void *stream, tof_ctx **out)
{
    if (!out) return fail(nullptr, TOF_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!grid) return fail(nullptr, TOF_ERR_INVALID, "grid is null");
    const tof_grid g = *grid;
    GridLayout lay;
    std::string lerr;
    tof_status s = grid_layout(g, lay, lerr);
    if (s != TOF_OK) return fail(nullptr, s, lerr);
    const int *L = lay.L;
    tof_ctx *ctx = new (std::nothrow) tof_ctx();
    if (!ctx) return fail(nullptr, TOF_ERR_OOM, "host allocation failed");
    ctx->nx = g.nx; ctx->ny = g.ny; ctx->nz = g.nz;
    ctx->dx = g.dx; ctx->dy = g.dy; ctx->dz = g.dz;
    ctx->Lx = L[0]; ctx->Ly = L[1]; ctx->Lz = L[2];
    ctx->hx = lay.hx;
    ctx->f64 = g.dtype == TOF_F64;
    ctx->wsize = lay.wsize;
    ctx->validate = g.validate != 0;
    ctx->flags = g.flags;
    ctx->design = Box{0, g.nx, 0, g.ny, 0, g.nz};
    hipStream_t st = (hipStream_t)stream;
    auto bail = [&](tof_status code) {
        release(ctx);
        g_thread_error = ctx->err;
        delete ctx;
        return code;
    };
    if ((s = make_plan(ctx, ctx->px, L[0])) != TOF_OK) return bail(s);
    if ((s = make_plan(ctx, ctx->py, L[1])) != TOF_OK) return bail(s);
    if ((s = make_plan(ctx, ctx->pz, L[2])) != TOF_OK) return bail(s);
    ctx->hkz = lay.hkz;
    ctx->ky_pitch = lay.ky_pitch;
    ctx->comp_stride = lay.comp_stride;
    ctx->kt_pitch = lay.kt_pitch;
    ctx->comp_stride_kt = lay.comp_stride_kt;
    if ((s = dev_alloc(ctx, ctx->spec, lay.spec)) != TOF_OK) return bail(s);
    if ((s = dev_alloc(ctx, ctx->kt, lay.kt)) != TOF_OK) return bail(s);
    ctx->Zrows = g.nz;
    {
        // ky-blocked B (KB columns of 256 bytes) when both the y and the z
        // passes take the register path; plain [c][kx][z][ky] otherwise
        auto pow2_fast = [](int v) { return v >= 32 && v <= 512 && (v & (v - 1)) == 0; };
        const int KB = ctx->f64 ? 16 : TOF_KB32;
        int kbs = 0;
        while ((1 << kbs) < KB) ++kbs;
        if (pow2_fast(L[1]) && pow2_fast(L[2]))
            ctx->bmap = BlockMap{kbs, (long long)g.nz * KB, KB};
        else
            ctx->bmap = BlockMap{30, 0, L[1]};
    }
    if ((s = dev_alloc(ctx, ctx->A, lay.A)) != TOF_OK) return bail(s);
    if ((s = dev_alloc(ctx, ctx->B, lay.B)) != TOF_OK) return bail(s);
    if ((s = dev_alloc(ctx, ctx->C, lay.C)) != TOF_OK) return bail(s);
    if ((s = dev_alloc(ctx, ctx->scratch64, 64)) != TOF_OK) return bail(s);
    if ((s = dev_alloc(ctx, ctx->steppart, sizeof(double) * kStepMaxBlocks)) != TOF_OK) return bail(s);
    if ((s = dev_alloc(ctx, ctx->partials, sizeof(double) * kObjMaxBlocks)) != TOF_OK) return bail(s);
    if ((s = dev_alloc(ctx, ctx->ticket, 64)) != TOF_OK) return bail(s);
    {
        hipError_t e0 = hipMemsetAsync(ctx->ticket.p, 0, 64, st);
        if (e0 != hipSuccess) return bail(hip_fail(ctx, e0, "hipMemsetAsync(counters)"));
    }
    if ((s = compute_spectra(ctx, st)) != TOF_OK) return bail(s);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "tensor setup"));
    *out = ctx;
    return TOF_OK;
}

void tof_destroy(tof_ctx *ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    release(ctx);
    delete ctx;
}

tof_status tof_set_design(tof_ctx *ctx, const tof_box *design, const uint8_t *mask, const double m0_host[3],
                          const void *m0_field, int32_t p)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    Box d = design ? to_box(*design) : Box{0, ctx->nx, 0, ctx->ny, 0, ctx->nz};
    if (!box_ok(d, ctx->nx, ctx->ny, ctx->nz)) return fail(ctx, TOF_ERR_INVALID, "design box outside the grid or empty");
    if (p < 1 || p > 16) return fail(ctx, TOF_ERR_INVALID, "p must be in [1, 16]");
    if (!m0_field) {
        if (!m0_host) return fail(ctx, TOF_ERR_INVALID, "give m0_host or m0_field");
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(m0_host[a])) return fail(ctx, TOF_ERR_INVALID, "M0 must be finite");
        if (m0_host[0] == 0 && m0_host[1] == 0 && m0_host[2] == 0)
            return fail(ctx, TOF_ERR_INVALID, "M0 must not be zero");
        for (int a = 0; a < 3; ++a) ctx->m0[a] = m0_host[a];
    }
    ctx->design = d;
    ctx->mask = mask;
    ctx->m0f = m0_field;
    ctx->p = p;
    ctx->has_design = true;
    return TOF_OK;
}

tof_status tof_set_objective(tof_ctx *ctx, const tof_objective *obj)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    if (!obj) return fail(ctx, TOF_ERR_INVALID, "objective is null");
    if (obj->kind < 1 || obj->kind > 5) return fail(ctx, TOF_ERR_INVALID, "unknown objective kind");
    Box sb = to_box(obj->sensor);
    if (!box_ok(sb, ctx->nx, ctx->ny, ctx->nz)) return fail(ctx, TOF_ERR_INVALID, "sensor box outside the grid or empty");
    Box ob = sb;
    if (obj->kind == TOF_J_MEAN_SQ_HZ_GRADXY) {
        if (sb.x0 < 1 || sb.y0 < 1 || sb.x1 > ctx->nx - 1 || sb.y1 > ctx->ny - 1)
            return fail(ctx, TOF_ERR_INVALID, "the gradient term needs in-grid x and y neighbours of the sensor");
        ob = Box{sb.x0 - 1, sb.x1 + 1, sb.y0 - 1, sb.y1 + 1, sb.z0, sb.z1};
    }
    if (obj->kind == TOF_J_FIELD_GRADIENT) {
        if (sb.x0 < 2 || sb.y0 < 2 || sb.x1 > ctx->nx - 2)
            return fail(ctx, TOF_ERR_INVALID, "the gradient strip and its outer neighbours must be in the grid");
        ob = Box{sb.x0 - 2, sb.x1 + 2, sb.y0 - 2, sb.y1, sb.z0, sb.z1};
    }
    if (obj->kind == TOF_J_MEAN_SQ_H_TARGET && !obj->h_target_host == !obj->h_target_dev)
        return fail(ctx, TOF_ERR_INVALID, "kind 3 needs exactly one of h_target_host and h_target_dev");
    if (!std::isfinite(obj->target) || !std::isfinite(obj->lambda_grad))
        return fail(ctx, TOF_ERR_INVALID, "target and lambda must be finite");
    // from here on a failure leaves the context without an objective
    ctx->has_obj = false;
    const int cj = obj->kind == TOF_J_MEAN_SQ_H_TARGET ? 3 : 1;
    const size_t nob = (size_t)ob.nx() * ob.ny() * ob.nz();
    const size_t S = (size_t)sb.nx() * sb.ny() * sb.nz();
    tof_status s;
    if ((s = dev_alloc(ctx, ctx->Hs, ctx->wsize * cj * nob)) != TOF_OK) return s;
    if ((s = dev_alloc(ctx, ctx->G, ctx->wsize * cj * nob)) != TOF_OK) return s;
    if (obj->kind == TOF_J_MEAN_SQ_H_TARGET) {
        if ((s = dev_alloc(ctx, ctx->Ht, sizeof(double) * 3 * S)) != TOF_OK) return s;
        if (obj->h_target_host)
            HIP_TRY(ctx, hipMemcpy(ctx->Ht.p, obj->h_target_host, sizeof(double) * 3 * S, hipMemcpyHostToDevice));
        else
            HIP_TRY(ctx, hipMemcpy(ctx->Ht.p, obj->h_target_dev, sizeof(double) * 3 * S, hipMemcpyDeviceToDevice));
    }
    ctx->kind = obj->kind;
    ctx->sensor = sb;
    ctx->ob = ob;
    ctx->target = obj->target;
    ctx->lam = obj->lambda_grad;
    ctx->has_obj = true;
    return TOF_OK;
}

tof_status tof_field(tof_ctx *ctx, const void *rho, void *H, int32_t comps_mask, void *stream)
{
    tof_status s = check_ready(ctx, false);
    if (s != TOF_OK) return s;
    if (!rho || !H) return fail(ctx, TOF_ERR_INVALID, "rho and H must be non-null");
    if (comps_mask < 1 || comps_mask > 7) return fail(ctx, TOF_ERR_INVALID, "comps_mask must be in [1, 7]");
    hipStream_t st = (hipStream_t)stream;
    const long long n = (long long)ctx->nx * ctx->ny * ctx->nz;
    if ((s = check_finite_any(ctx, st, rho, n, "rho")) != TOF_OK) return s;
    return ctx->f64 ? run_field<double>(ctx, st, rho, H, comps_mask) : run_field<float>(ctx, st, rho, H, comps_mask);
}

tof_status tof_objective_and_grad(tof_ctx *ctx, const void *rho, double *J, void *grad, void *stream)
{
    tof_status s = check_ready(ctx, true);
    if (s != TOF_OK) return s;
    if (!rho || !grad) return fail(ctx, TOF_ERR_INVALID, "rho and grad must be non-null");
    hipStream_t st = (hipStream_t)stream;
    const long long n = (long long)ctx->nx * ctx->ny * ctx->nz;
    if ((s = check_finite_any(ctx, st, rho, n, "rho")) != TOF_OK) return s;
    return ctx->f64 ? run_objective_and_grad<double>(ctx, st, rho, J, grad)
                    : run_objective_and_grad<float>(ctx, st, rho, J, grad);
}

tof_status tof_adjoint(tof_ctx *ctx, const void *rho, const void *gH, void *grad, void *stream)
{
    tof_status s = check_ready(ctx, false);
    if (s != TOF_OK) return s;
    if (!rho || !gH || !grad) return fail(ctx, TOF_ERR_INVALID, "rho, gH and grad must be non-null");
    hipStream_t st = (hipStream_t)stream;
    const long long n = (long long)ctx->nx * ctx->ny * ctx->nz;
    if ((s = check_finite_any(ctx, st, rho, n, "rho")) != TOF_OK) return s;
    if ((s = check_finite_any(ctx, st, gH, 3 * n, "gH")) != TOF_OK) return s;
    const Box all{0, ctx->nx, 0, ctx->ny, 0, ctx->nz};
    if (ctx->f64) {
        View4<const double> src{(const double *)gH, n, (long long)ctx->ny * ctx->nx, ctx->nx, 0, 0, 0};
        return adjoint_to_grad<double>(ctx, st, rho, src, all, 7, grad);
    }
    View4<const float> src{(const float *)gH, n, (long long)ctx->ny * ctx->nx, ctx->nx, 0, 0, 0};
    return adjoint_to_grad<float>(ctx, st, rho, src, all, 7, grad);
}

tof_status tof_project_step(tof_ctx *ctx, void *rho, const void *grad, double alpha, void *stream)
{
    tof_status s = check_ready(ctx, false);
    if (s != TOF_OK) return s;
    if (!rho || !grad) return fail(ctx, TOF_ERR_INVALID, "rho and grad must be non-null");
    if (!std::isfinite(alpha) || alpha < 0) return fail(ctx, TOF_ERR_INVALID, "alpha must be finite and >= 0");
    hipStream_t st = (hipStream_t)stream;
    const long long n = (long long)ctx->nx * ctx->ny * ctx->nz;
    if ((s = check_finite_any(ctx, st, rho, n, "rho")) != TOF_OK) return s;
    if ((s = check_finite_any(ctx, st, grad, n, "grad")) != TOF_OK) return s;
    double *part = (double *)ctx->steppart.p;
    if (ctx->f64)
        HIP_TRY(ctx, launch_project_step<double>(st, (double *)rho, (const double *)grad, ctx->mask, ctx->nx, ctx->ny,
                                                 ctx->nz, ctx->design, alpha, part));
    else
        HIP_TRY(ctx, launch_project_step<float>(st, (float *)rho, (const float *)grad, ctx->mask, ctx->nx, ctx->ny,
                                                ctx->nz, ctx->design, alpha, part));
    return TOF_OK;
}

tof_status tof_project_step_static(const tof_grid *grid, const tof_box *design, const uint8_t *mask, void *rho,
                                   const void *grad, double alpha, void *stream)
{
    if (!grid) return fail(nullptr, TOF_ERR_INVALID, "grid is null");
    const tof_grid &g = *grid;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > kMaxL / 2 || g.ny > kMaxL / 2 || g.nz > kMaxL / 2)
        return fail(nullptr, TOF_ERR_INVALID, "grid sizes must be in [1, 512] (the largest grid the static scratch serves)");
    if (g.dtype != TOF_F32 && g.dtype != TOF_F64) return fail(nullptr, TOF_ERR_INVALID, "dtype must be TOF_F32 or TOF_F64");
    if (!rho || !grad) return fail(nullptr, TOF_ERR_INVALID, "rho and grad must be non-null");
    if (!std::isfinite(alpha) || alpha < 0) return fail(nullptr, TOF_ERR_INVALID, "alpha must be finite and >= 0");
    const Box d = design ? to_box(*design) : Box{0, g.nx, 0, g.ny, 0, g.nz};
    if (!box_ok(d, g.nx, g.ny, g.nz)) return fail(nullptr, TOF_ERR_INVALID, "design box outside the grid or empty");
    std::string msg;
    double *part = static_scratch_ptr(msg);
    if (!part) return fail(nullptr, TOF_ERR_HIP, msg);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = g.dtype == TOF_F64
                       ? launch_project_step<double>(st, (double *)rho, (const double *)grad, mask, g.nx, g.ny, g.nz, d,
                                                     alpha, part)
                       : launch_project_step<float>(st, (float *)rho, (const float *)grad, mask, g.nx, g.ny, g.nz, d,
                                                    alpha, part);
    if (e != hipSuccess) return hip_fail(nullptr, e, "tof_project_step_static");
    return TOF_OK;
}

tof_status tof_tensor(tof_ctx *ctx, double *N, void *stream)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    if (!N) return fail(ctx, TOF_ERR_INVALID, "N is null");
    hipStream_t st = (hipStream_t)stream;
    const int lx = ctx->nx + 1, ly = ctx->ny + 1, lz = ctx->nz + 1;
    DeviceBuf lat;
    tof_status s = dev_alloc(ctx, lat, sizeof(double) * 2 * (size_t)lx * ly * lz);
    if (s != TOF_OK) return s;
    const size_t plane = (size_t)ctx->nx * ctx->ny * ctx->nz;
    hipError_t e = hipSuccess;
    for (int c = 0; c < 6 && e == hipSuccess; ++c) {
        e = launch_newell_lattice(st, c, lx, ly, lz, ctx->dx, ctx->dy, ctx->dz, (double *)lat.p);
        if (e == hipSuccess)
            e = launch_newell_stencil(st, c, ctx->nx, ctx->ny, ctx->nz, lx, ly, ctx->dx, ctx->dy, ctx->dz,
                                      (const double *)lat.p, nullptr, ctx->Lx, ctx->Ly, ctx->Lz, N + c * plane);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(lat.p);
    if (e != hipSuccess) return hip_fail(ctx, e, "tof_tensor");
    return TOF_OK;
}

tof_status tof_tensor_full(tof_ctx *ctx, double *N, void *stream)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    if (!N) return fail(ctx, TOF_ERR_INVALID, "N is null");
    hipStream_t st = (hipStream_t)stream;
    DeviceBuf oct;
    tof_status s = dev_alloc(ctx, oct, sizeof(double) * 6 * (size_t)ctx->nx * ctx->ny * ctx->nz);
    if (s != TOF_OK) return s;
    s = tof_tensor(ctx, (double *)oct.p, stream);
    hipError_t e = hipSuccess;
    if (s == TOF_OK) {
        e = launch_tensor_full(st, (const double *)oct.p, ctx->nx, ctx->ny, ctx->nz, N);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    (void)hipFree(oct.p);
    if (s != TOF_OK) return s;
    if (e != hipSuccess) return hip_fail(ctx, e, "tof_tensor_full");
    return TOF_OK;
}

tof_status tof_profile_enable(tof_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    if (enable && ctx->prof_ev.empty()) {
        const size_t n = (size_t)TOF_PROFILE_SLOTS * kProfCalls;
        ctx->prof_ev.resize(n, nullptr);
        ctx->prof_refs.resize(kProfAnchors, nullptr);
        ctx->prof_rec_ref.assign(n, -1);
        ctx->prof_rec_prev.assign(n, nullptr);
        // timing events without the system-scope fence: the default event
        // writes back the L2 at each record, which lengthens the timed launch
        for (hipEvent_t &ev : ctx->prof_ev) HIP_TRY(ctx, hipEventCreateWithFlags(&ev, hipEventDisableSystemFence));
        for (hipEvent_t &ev : ctx->prof_refs) HIP_TRY(ctx, hipEventCreateWithFlags(&ev, hipEventDisableSystemFence));
        for (auto &pair : ctx->prof_burst_ev)
            for (hipEvent_t &ev : pair) HIP_TRY(ctx, hipEventCreate(&ev));
    }
    ctx->prof_on = enable != 0;
    ctx->prof_last = nullptr;   // a chain of timed launches starts afresh
    return TOF_OK;
}

tof_status tof_profile_read(tof_ctx *ctx, double ms_host[], int64_t count_host[], double bytes_host[])
{
    if (!ctx || !ms_host || !count_host || !bytes_host) return fail(ctx, TOF_ERR_INVALID, "null argument");
    for (int slot = 0; slot < TOF_PROFILE_SLOTS; ++slot) {
        // launches timed from the end of the one before them, and the first
        // launches of chains (from their anchor) apart: a slot reports the
        // former when it has any
        double sum_c = 0.0, sum_a = 0.0;
        int64_t n_c = 0, n_a = 0;
        for (int i = 0; i < ctx->prof_calls[slot]; ++i) {
            const size_t idx = (size_t)slot * kProfCalls + i;
            hipEvent_t stop = ctx->prof_ev[idx], ref = ctx->prof_refs[(size_t)ctx->prof_rec_ref[idx]];
            HIP_TRY(ctx, hipEventSynchronize(stop));
            float a = 0.f;
            HIP_TRY(ctx, hipEventElapsedTime(&a, ref, stop));
            if (hipEvent_t prev = ctx->prof_rec_prev[idx]) {
                float b = 0.f;
                HIP_TRY(ctx, hipEventElapsedTime(&b, ref, prev));
                sum_c += (double)a - (double)b;
                ++n_c;
            } else {
                sum_a += a;
                ++n_a;
            }
        }
        ms_host[slot] = n_c ? sum_c : sum_a;
        count_host[slot] = n_c ? n_c : n_a;
        bytes_host[slot] = ctx->prof_bytes[slot];
        ctx->prof_calls[slot] = 0;
    }
    ctx->prof_nref = 0;
    ctx->prof_last = nullptr;
    return TOF_OK;
}

tof_status tof_profile_burst(tof_ctx *ctx, uint32_t slot_mask, int32_t repeats)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    if (!ctx->prof_on) return fail(ctx, TOF_ERR_INVALID, "timing is off (tof_profile_enable first)");
    if (repeats < 1 || repeats > TOF_PROFILE_MAX_BURST)
        return fail(ctx, TOF_ERR_INVALID, "repeats outside [1, " + std::to_string(TOF_PROFILE_MAX_BURST) + "]");
    if (slot_mask >> TOF_PROFILE_SLOTS) return fail(ctx, TOF_ERR_INVALID, "slot_mask names no slot");
    ctx->prof_burst_mask = slot_mask;
    ctx->prof_burst_reps = repeats;
    for (int slot = 0; slot < TOF_PROFILE_SLOTS; ++slot)
        if ((slot_mask >> slot) & 1u) ctx->prof_burst_done[slot] = 0;
    return TOF_OK;
}

tof_status tof_profile_burst_read(tof_ctx *ctx, double ms_host[])
{
    if (!ctx || !ms_host) return fail(ctx, TOF_ERR_INVALID, "null argument");
    for (int slot = 0; slot < TOF_PROFILE_SLOTS; ++slot) {
        ms_host[slot] = 0.0;
        if (!ctx->prof_burst_done[slot]) continue;
        HIP_TRY(ctx, hipEventSynchronize(ctx->prof_burst_ev[slot][1]));
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->prof_burst_ev[slot][0], ctx->prof_burst_ev[slot][1]));
        ms_host[slot] = (double)ms / ctx->prof_burst_done[slot];
        ctx->prof_burst_done[slot] = 0;
    }
    return TOF_OK;
}

const char *tof_profile_kernel(const tof_ctx *ctx, int32_t slot, int64_t *work_items)
{
    if (work_items) *work_items = 0;
    if (!ctx || slot < 0 || slot >= TOF_PROFILE_SLOTS) return "";
    if (work_items) *work_items = ctx->prof_items[slot];
    return ctx->prof_kernel[slot].c_str();
}

tof_status tof_set_option(tof_ctx *ctx, int32_t option, int32_t value)
{
    if (!ctx) return fail(nullptr, TOF_ERR_INVALID, "null context");
    const bool flag = option >= TOF_OPT_ZSUM && option <= TOF_OPT_FUSE_OBJECTIVE;
    if (flag && value != 0 && value != 1) return fail(ctx, TOF_ERR_INVALID, "option values are 0 or 1");
    switch (option) {
    case TOF_OPT_ZSUM: ctx->opt_zsum = value != 0; return TOF_OK;
    case TOF_OPT_FUSE_YZ: ctx->opt_fuse = value != 0; return TOF_OK;
    case TOF_OPT_FUSE_OBJECTIVE: ctx->opt_fuse_obj = value != 0; return TOF_OK;
    case TOF_OPT_X_TILE:
        if (value < kXTileAuto || value > kXTilePair) return fail(ctx, TOF_ERR_INVALID, "x tile is 0, 1 or 2");
        ctx->opt_xtile = value;
        return TOF_OK;
    case TOF_OPT_GATHER_GROUPS:
    case TOF_OPT_SCATTER_GROUPS:
        if (value < 0 || value > 64) return fail(ctx, TOF_ERR_INVALID, "row groups are 0 (default) to 64");
        (option == TOF_OPT_GATHER_GROUPS ? ctx->opt_gather_groups : ctx->opt_scatter_groups) = value;
        return TOF_OK;
    default: return fail(ctx, TOF_ERR_INVALID, "unknown option");
    }
}

tof_status tof_padded_lengths(const tof_ctx *ctx, int32_t out[3])
{
    if (!ctx || !out) return fail(nullptr, TOF_ERR_INVALID, "null argument");
    out[0] = ctx->Lx;
    out[1] = ctx->Ly;
    out[2] = ctx->Lz;
    return TOF_OK;
}

size_t tof_workspace_bytes(const tof_grid *grid)
{
    if (!grid) return 0;
    GridLayout lay;
    std::string err;
    if (grid_layout(*grid, lay, err) != TOF_OK) {
        g_thread_error = err;
        return 0;
    }
    return lay.total();
}

size_t tof_ctx_bytes(const tof_ctx *ctx)
{
    if (!ctx) return 0;
    size_t tw = 0;
    for (const Plan1D *pl : {&ctx->px, &ctx->py, &ctx->pz}) tw += (sizeof(float) + sizeof(double)) * 2 * (size_t)pl->L;
    return ctx->spec.bytes + ctx->kt.bytes + ctx->A.bytes + ctx->B.bytes + ctx->C.bytes + ctx->Hs.bytes + ctx->G.bytes +
           ctx->Ht.bytes + ctx->scratch64.bytes + ctx->steppart.bytes + ctx->partials.bytes + ctx->ticket.bytes + tw;
}

const char *tof_last_error(const tof_ctx *ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_thread_error.c_str();
}

tof_status tof_batch_create(tof_ctx *const *ctxs, const void *const *rho, double *const *J, void *const *grad,
                            int32_t n, tof_batch **out)
{
    if (!out) return fail(nullptr, TOF_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!ctxs || !rho || !J || !grad || n < 1) return fail(nullptr, TOF_ERR_INVALID, "null arrays or n < 1");
    // record every design's launches (nothing runs)
    std::vector<std::vector<BatchLaunch>> recs((size_t)n);
    for (int i = 0; i < n; ++i) {
        tof_ctx *ctx = ctxs[i];
        tof_status s = check_ready(ctx, true);
        if (s != TOF_OK) return fail(nullptr, s, "design " + std::to_string(i) + ": " + g_thread_error);
        if (!rho[i] || !J[i] || !grad[i]) return fail(nullptr, TOF_ERR_INVALID, "null buffer of design " + std::to_string(i));
        if (ctx->validate || ctx->prof_on)
            return fail(nullptr, TOF_ERR_INVALID, "design " + std::to_string(i) + ": no validation or timing in a batch");
        g_batch_record = &recs[i];
        g_batch_unbatchable = nullptr;
        s = ctx->f64 ? run_objective_and_grad<double>(ctx, nullptr, rho[i], J[i], grad[i])
                     : run_objective_and_grad<float>(ctx, nullptr, rho[i], J[i], grad[i]);
        const char *bad = g_batch_unbatchable;
        g_batch_record = nullptr;
        g_batch_unbatchable = nullptr;
        if (s != TOF_OK) return fail(nullptr, s, "design " + std::to_string(i) + ": " + ctx->err);
        if (bad)
            return fail(nullptr, TOF_ERR_UNSUPPORTED, "design " + std::to_string(i) + " launches " + bad +
                                                         ", which has no batched form (the batch needs the fused passes)");
        if (recs[i].size() != recs[0].size())
            return fail(nullptr, TOF_ERR_UNSUPPORTED, "design " + std::to_string(i) + " has a different number of passes");
    }
    tof_batch *b = new (std::nothrow) tof_batch();
    if (!b) return fail(nullptr, TOF_ERR_OOM, "host allocation failed");
    // group per pass by (kernel, block); lay the tables out in one host image
    std::vector<unsigned char> image;
    struct Pending { size_t tab_off, starts_off; };
    std::vector<std::vector<Pending>> pend;
    const size_t npass = recs[0].size();
    b->passes.resize(npass);
    pend.resize(npass);
    auto align = [&](size_t a) { image.resize((image.size() + a - 1) / a * a); };
    for (size_t k = 0; k < npass; ++k) {
        std::vector<int> done((size_t)n, 0);
        for (int i = 0; i < n; ++i) {
            if (done[i]) continue;
            const BatchLaunch &r0 = recs[i][k];
            tof_batch::Group g;
            g.kernel = r0.kernel;
            g.block = r0.block;
            std::vector<int> members;
            for (int j = i; j < n; ++j) {
                const BatchLaunch &r = recs[j][k];
                if (!done[j] && r.kernel == r0.kernel && r.block.x == r0.block.x && r.block.y == r0.block.y &&
                    r.block.z == r0.block.z && r.args.size() == r0.args.size()) {
                    members.push_back(j);
                    done[j] = 1;
                }
            }
            g.n = (int)members.size();
            align(256);
            const size_t tab_off = image.size();
            for (int j : members) image.insert(image.end(), recs[j][k].args.begin(), recs[j][k].args.end());
            align(256);
            const size_t starts_off = image.size();
            std::vector<int> starts;
            long long tot = 0;
            for (int j : members) {
                starts.push_back((int)tot);
                const dim3 &gr = recs[j][k].grid;
                tot += (long long)gr.x * gr.y * gr.z;
            }
            starts.push_back((int)tot);
            if (tot > (1LL << 30)) {
                delete b;
                return fail(nullptr, TOF_ERR_UNSUPPORTED, "batch too large for one launch");
            }
            g.blocks = tot;
            const unsigned char *sp = reinterpret_cast<const unsigned char *>(starts.data());
            image.insert(image.end(), sp, sp + sizeof(int) * starts.size());
            b->passes[k].push_back(g);
            pend[k].push_back(Pending{tab_off, starts_off});
        }
    }
    hipError_t e = hipMalloc(&b->buf, image.size());
    if (e == hipSuccess) e = hipMemcpy(b->buf, image.data(), image.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (b->buf) (void)hipFree(b->buf);
        delete b;
        return hip_fail(nullptr, e, "tof_batch_create");
    }
    for (size_t k = 0; k < npass; ++k)
        for (size_t q = 0; q < b->passes[k].size(); ++q) {
            b->passes[k][q].tab = (unsigned char *)b->buf + pend[k][q].tab_off;
            b->passes[k][q].starts = (int *)((unsigned char *)b->buf + pend[k][q].starts_off);
        }
    *out = b;
    return TOF_OK;
}

tof_status tof_batch_run(tof_batch *b, void *stream)
{
    if (!b) return fail(nullptr, TOF_ERR_INVALID, "null batch");
    hipStream_t st = (hipStream_t)stream;
    for (const auto &pass : b->passes) {
        for (const tof_batch::Group &g : pass) {
            const void *tab = g.tab;
            const int *starts = g.starts;
            int n = g.n;
            void *args[] = {(void *)&tab, (void *)&starts, (void *)&n};
            const hipError_t e = hipLaunchKernel(g.kernel, dim3((unsigned)g.blocks), g.block, args, 0, st);
            if (e != hipSuccess) {
                b->err = std::string("hipLaunchKernel: ") + hipGetErrorString(e);
                return fail(nullptr, TOF_ERR_HIP, b->err);
            }
        }
    }
    return TOF_OK;
}

int32_t tof_batch_launches(const tof_batch *b)
{
    if (!b) return 0;
    int32_t c = 0;
    for (const auto &pass : b->passes) c += (int32_t)pass.size();
    return c;
}

void tof_batch_destroy(tof_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    batch_release(b);
    delete b;
}

double tof_dd_newell_host(int32_t c, int32_t kx, int32_t ky, int32_t kz, double dx, double dy, double dz)
{
    if (c < 0 || c > 5 || kx < 0 || ky < 0 || kz < 0 || !(dx > 0) || !(dy > 0) || !(dz > 0)) return NAN;
    const bool ox = comp_odd_x(c), oy = comp_odd_y(c), oz = comp_odd_z(c);
    dd acc = dd_make(0.0);
    for (int sz = -1; sz <= 1; ++sz)
        for (int sy = -1; sy <= 1; ++sy)
            for (int sx = -1; sx <= 1; ++sx) {
                int a = kx + sx, b = ky + sy, e = kz + sz;
                int sign = 1;
                if (a < 0) { a = -a; if (ox) sign = -sign; }
                if (b < 0) { b = -b; if (oy) sign = -sign; }
                if (e < 0) { e = -e; if (oz) sign = -sign; }
                const int w = (sx ? -1 : 2) * (sy ? -1 : 2) * (sz ? -1 : 2) * sign;
                const dd v = newell_component_dd(c, two_prod((double)a, dx), two_prod((double)b, dy),
                                                 two_prod((double)e, dz));
                acc = dd_add(acc, dd_mul_d(v, (double)w));
            }
    return dd_mul(acc, inv_4pi_volume(dx, dy, dz)).hi;
}

}  // extern "C"
