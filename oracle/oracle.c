/*
 * CPU oracle for the FD topology-optimization gradient (Abert et al. 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links, calls or includes it, and it includes nothing
 * of the product.
 *
 * Two functions carry the arithmetic:
 *
 *  oracle_newell_table  the discrete demagnetization tensor of Sec.
 *      "Discretization", eq. (demag_tensor): the cell-averaged field of a
 *      uniformly magnetized cuboid cell, which depends only on the index
 *      difference of the two cells.  It is evaluated with the closed form of
 *      Newell, Williams and Dunlop (J. Geophys. Res. 98, 9551, 1993), to which
 *      that section defers: the auxiliary functions f and g at lattice points,
 *      then the separable (-1, 2, -1) second difference along each axis.  The
 *      second difference cancels O(r^6) relative at offset r, so the lattice
 *      and the difference are evaluated in IEEE binary128 (__float128) and
 *      only the finished entry is rounded to double.
 *
 *      Sign: the stored tensor is the positive (Newell) one, trace 1 at zero
 *      offset, a cube's self term 1/3 on the diagonal.  The paper's tensor in
 *      eq. (demag_tensor) is its negative; the field is then H = -N (*) M.
 *
 *  oracle_field  the discrete convolution of eq. (convolution) as a plain
 *      direct sum over source cells, H_a(t) = -sum_s sum_b N_ab(t - s) M_b(s),
 *      for target cells t of an index box.  No FFT, no padding: this is the
 *      definition the FFT method reaches exactly (up to rounding).
 *
 * Component order of all six-component arrays: xx, yy, zz, xy, xz, yz.
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 quad;

enum { C_XX = 0, C_YY = 1, C_ZZ = 2, C_XY = 3, C_XZ = 4, C_YZ = 5 };

/* Newell's f, even in each argument.  A term whose polynomial prefactor is
 * zero is zero (this covers the 0*asinh(./0) and 0*atan(./0) limits). */
static quad newell_f(quad x, quad y, quad z)
{
    x = fabsq(x);
    y = fabsq(y);
    z = fabsq(z);
    const quad x2 = x * x, y2 = y * y, z2 = z * z;
    const quad R = sqrtq(x2 + y2 + z2);
    quad r = 0;
    quad c;
    c = y / 2 * (z2 - x2);
    if (c != 0) r += c * asinhq(y / sqrtq(x2 + z2));
    c = z / 2 * (y2 - x2);
    if (c != 0) r += c * asinhq(z / sqrtq(x2 + y2));
    c = x * y * z;
    if (c != 0) r -= c * atanq(y * z / (x * R));
    r += (2 * x2 - y2 - z2) * R / 6;
    return r;
}

/* Newell's g, odd in its first two arguments and even in the third. */
static quad newell_g(quad x, quad y, quad z)
{
    int sgn = 1;
    if (x < 0) { x = -x; sgn = -sgn; }
    if (y < 0) { y = -y; sgn = -sgn; }
    z = fabsq(z);
    const quad x2 = x * x, y2 = y * y, z2 = z * z;
    const quad R = sqrtq(x2 + y2 + z2);
    quad r = 0;
    quad c;
    c = x * y * z;
    if (c != 0) r += c * asinhq(z / sqrtq(x2 + y2));
    c = y / 6 * (3 * z2 - y2);
    if (c != 0) r += c * asinhq(x / sqrtq(y2 + z2));
    c = x / 6 * (3 * z2 - x2);
    if (c != 0) r += c * asinhq(y / sqrtq(x2 + z2));
    c = z * z2 / 6;
    if (c != 0) r -= c * atanq(x * y / (z * R));
    c = z * y2 / 2;
    if (c != 0) r -= c * atanq(x * z / (y * R));
    c = z * x2 / 2;
    if (c != 0) r -= c * atanq(y * z / (x * R));
    r -= x * y * R / 3;
    return sgn > 0 ? r : -r;
}

/* The auxiliary function of tensor component c at lattice coordinates
 * (X, Y, Z): the diagonal components permute f's arguments, the off-diagonal
 * ones g's. */
static quad component_fn(int c, quad X, quad Y, quad Z)
{
    switch (c) {
    case C_XX: return newell_f(X, Y, Z);
    case C_YY: return newell_f(Y, X, Z);
    case C_ZZ: return newell_f(Z, Y, X);
    case C_XY: return newell_g(X, Y, Z);
    case C_XZ: return newell_g(X, Z, Y);
    default:   return newell_g(Y, Z, X);
    }
}

/*
 * Discrete demagnetization tensor for index offsets 0 <= k_a < m_a.
 * out: [6][mz][my][mx] doubles; components not in comp_mask are untouched.
 * Offsets of either sign follow by parity: the diagonal components are even
 * in every axis, xy is odd in x and y, xz odd in x and z, yz odd in y and z.
 * Returns 0, or -1 on bad arguments / out of memory.
 */
int oracle_newell_table(int mx, int my, int mz, double dx, double dy, double dz,
                        int comp_mask, double *out)
{
    if (mx <= 0 || my <= 0 || mz <= 0 || !(dx > 0) || !(dy > 0) || !(dz > 0) || !out)
        return -1;
    /* lattice coordinates i*dx for i in [-1, m]; stored for i in [0, m+1) */
    const long lx = mx + 1, ly = my + 1, lz = mz + 1;
    quad *lat = (quad *)malloc(sizeof(quad) * (size_t)(lx * ly * lz));
    if (!lat) return -1;
    const quad hx = dx, hy = dy, hz = dz;
    const quad inv4piV = 1 / (4 * M_PIq * hx * hy * hz);
    const size_t plane = (size_t)mx * my * mz;
    for (int c = 0; c < 6; ++c) {
        if (!(comp_mask & (1 << c))) continue;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
        for (long k = 0; k < lz; ++k)
            for (long j = 0; j < ly; ++j)
                for (long i = 0; i < lx; ++i)
                    lat[(k * ly + j) * lx + i] = component_fn(c, i * hx, j * hy, k * hz);
        /* odd axes of this component: lattice value at a negative coordinate
         * is minus the value at the mirrored one */
        const int oddx = (c == C_XY || c == C_XZ);
        const int oddy = (c == C_XY || c == C_YZ);
        const int oddz = (c == C_XZ || c == C_YZ);
#pragma omp parallel for collapse(2) schedule(static)
        for (long k = 0; k < mz; ++k)
            for (long j = 0; j < my; ++j)
                for (long i = 0; i < mx; ++i) {
                    quad acc = 0;
                    for (int sz = -1; sz <= 1; ++sz)
                        for (int sy = -1; sy <= 1; ++sy)
                            for (int sx = -1; sx <= 1; ++sx) {
                                long a = i + sx, b = j + sy, e = k + sz;
                                int sign = 1;
                                if (a < 0) { a = -a; if (oddx) sign = -sign; }
                                if (b < 0) { b = -b; if (oddy) sign = -sign; }
                                if (e < 0) { e = -e; if (oddz) sign = -sign; }
                                const int w = (sx ? -1 : 2) * (sy ? -1 : 2) * (sz ? -1 : 2);
                                const quad v = lat[(e * ly + b) * lx + a];
                                acc += (sign * w) * v;
                            }
                    out[c * plane + (size_t)(k * my + j) * mx + i] = (double)(acc * inv4piV);
                }
    }
    free(lat);
    return 0;
}

static int comp_index(int a, int b)
{
    if (a == b) return a;
    if (a > b) { int t = a; a = b; b = t; }
    if (a == 0) return b == 1 ? C_XY : C_XZ;
    return C_YZ;
}

/*
 * Direct-sum field H_a(t) = -sum_{s in sbox} sum_{b in src_mask} N_ab(t - s) M_b(s)
 * for t in tbox and a in tgt_mask (bit a = component a).  M and H are
 * [3][nz][ny][nx]; H entries outside tbox or components outside tgt_mask are
 * untouched.  Boxes are {x0, x1, y0, y1, z0, z1}, half-open.  The table holds
 * offsets [0, m) per axis and must cover every |t - s|.  The sum runs over
 * source cells in C order (z, y, x) and over source components in order.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_field(int nx, int ny, int nz, const double *table, int mx, int my, int mz,
                 const double *M, int src_mask, const int *sbox,
                 int tgt_mask, const int *tbox, double *H)
{
    if (!table || !M || !H || !sbox || !tbox) return -1;
    const int *S = sbox, *T = tbox;
    if (S[0] < 0 || S[1] > nx || S[2] < 0 || S[3] > ny || S[4] < 0 || S[5] > nz) return -1;
    if (T[0] < 0 || T[1] > nx || T[2] < 0 || T[3] > ny || T[4] < 0 || T[5] > nz) return -1;
    if (S[0] >= S[1] || S[2] >= S[3] || S[4] >= S[5]) return 0;
    if (T[0] >= T[1] || T[2] >= T[3] || T[4] >= T[5]) return 0;
    /* every offset must be in the table */
    if (T[1] - 1 - S[0] >= mx || S[1] - 1 - T[0] >= mx) return -1;
    if (T[3] - 1 - S[2] >= my || S[3] - 1 - T[2] >= my) return -1;
    if (T[5] - 1 - S[4] >= mz || S[5] - 1 - T[4] >= mz) return -1;
    const size_t n = (size_t)nx * ny * nz;
    const size_t plane = (size_t)mx * my * mz;
    const long tnx = T[1] - T[0], tny = T[3] - T[2], tnz = T[5] - T[4];
    const long ntgt = tnx * tny * tnz;

    /* the (target component, source component, tensor component) triples */
    int np = 0, pa[9], pb[9], pc[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if ((tgt_mask & (1 << a)) && (src_mask & (1 << b))) {
                pa[np] = a; pb[np] = b; pc[np] = comp_index(a, b); ++np;
            }

#pragma omp parallel for schedule(dynamic, 1)
    for (long q = 0; q < ntgt; ++q) {
        const int tx = T[0] + (int)(q % tnx);
        const int ty = T[2] + (int)((q / tnx) % tny);
        const int tz = T[4] + (int)(q / (tnx * tny));
        double acc[3] = {0, 0, 0};
        for (int sz = S[4]; sz < S[5]; ++sz)
            for (int sy = S[2]; sy < S[3]; ++sy)
                for (int sx = S[0]; sx < S[1]; ++sx) {
                    const int kx = tx - sx, ky = ty - sy, kz = tz - sz;
                    const size_t at = ((size_t)abs(kz) * my + abs(ky)) * mx + abs(kx);
                    const size_t src = ((size_t)sz * ny + sy) * nx + sx;
                    for (int u = 0; u < np; ++u) {
                        const int c = pc[u];
                        double sign = 1.0;
                        if (c == C_XY && (kx < 0) != (ky < 0)) sign = -1.0;
                        if (c == C_XZ && (kx < 0) != (kz < 0)) sign = -1.0;
                        if (c == C_YZ && (ky < 0) != (kz < 0)) sign = -1.0;
                        acc[pa[u]] += sign * table[c * plane + at] * M[pb[u] * n + src];
                    }
                }
        const size_t dst = ((size_t)tz * ny + ty) * nx + tx;
        for (int a = 0; a < 3; ++a)
            if (tgt_mask & (1 << a)) H[a * n + dst] = -acc[a];
    }
    return 0;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }
