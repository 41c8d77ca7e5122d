/*
 * Plain CPU oracle for the midplane self-gravitational force of an
 * infinitesimally thin disk (Tseng, Shang & Yen, "Direct Calculation of
 * Self-Gravitational Force for Infinitesimally Thin Gaseous Disks Using
 * Adaptive Mesh Refinement", Section 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU baseline
 * of the benchmark do.  It shares no code, header or table with the GPU
 * library.
 *
 * What it computes (Section 2, decomposition of the force integral over
 * disjoint zones D_i with a first-order Taylor density in each zone): for
 * every target point t,
 *
 *   F_x(t) = G * sum_i [ s_i K^{x,0}_i(t) + dx_i K^{x,x}_i(t) + dy_i K^{x,y}_i(t) ]
 *   F_y(t) = G * sum_i [ s_i K^{y,0}_i(t) + dx_i K^{y,x}_i(t) + dy_i K^{y,y}_i(t) ]
 *
 * with the exact cell integrals of Section 2 at z = 0, written with the
 * corner offsets u = xbar - x_t in [u1, u2], v = ybar - y_t in [v1, v2],
 * R = sqrt(u^2 + v^2) and the double difference
 *   DD[f] = (f(u2,v2) - f(u1,v2)) - (f(u2,v1) - f(u1,v1)):
 *
 *   K^{x,0} = -DD[ ln(v + R) ]            (= integral of u / r^3)
 *   I_uu    =  DD[ v ln(u + R) ]          (= integral of u^2 / r^3)
 *   I_uv    = -DD[ R ]                    (= integral of u v / r^3)
 *   K^{x,x} = (x_t - x_c) K^{x,0} + I_uu
 *   K^{x,y} = (y_t - y_c) K^{x,0} + I_uv
 *
 * and the y family by exchanging the roles of x and y.  The sign is the
 * physical (attractive) one: mass at xbar > x_t pulls the target towards +x.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - ln(a + sqrt(a^2+b^2)) is evaluated as ln(b^2 / (R - a)) when a < 0,
 *    an algebraic identity that avoids the cancellation of a + R.
 *  - When the target lies on the line through a cell edge (b == 0) the
 *    modified kernel of Section 2 is used: ln(a + R) -> sgn(a) ln|a|, applied
 *    to both families by symmetry; v ln(u + R) -> 0 when v == 0.
 *  - Each closed form is evaluated in x87 extended precision (long double)
 *    and rounded to double.  The double difference of a far cell cancels
 *    about 2 log10(d) digits (d its offset in cells), and the first-moment
 *    kernels then subtract (x_t - x_c) K^{x,0} from I_uu, two terms of the
 *    monopole's size, so extended precision does not remove the far-field
 *    error, it bounds it: with S = |K^{x,0}| + |K^{y,0}|, each centre kernel
 *    is within 1e-18 d^2 S and each first-moment kernel within
 *    1e-14 d^2 S h of its exact value (checked against 40-digit quadrature
 *    up to d = 6000: at d = 4096, 1.7e-11 S and 1.7e-7 S h).  Far entries
 *    are small beside the near-field ones, so sums over a grid keep the
 *    parity bar; single far entries are not a reference to that accuracy.
 *    All sums are double precision with Neumaier compensation per target.
 *  - On a uniform grid the kernel of a source cell depends only on its
 *    offset from the target in cells (the convolution structure the paper
 *    relies on for uniform grids); oracle_uniform evaluates each offset's
 *    closed form once and then performs the same O(N^4) double sum.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math:
 * the compensated summation depends on IEEE rounding).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;

/* ln(a + sqrt(a^2 + b^2)) with the x-bar = x convention of Section 2. */
static ld lam(ld a, ld b)
{
    if (b == 0.0L) {
        /* a == 0 here would be a target on a cell corner: callers reject it */
        return a > 0.0L ? logl(a) : -logl(-a);
    }
    ld R = sqrtl(a * a + b * b);
    if (a >= 0.0L) return logl(a + R);
    return logl((b * b) / (R - a));
}

/* v ln(u + R), with the v == 0 limit 0 */
static ld vlam(ld v, ld u)
{
    if (v == 0.0L) return 0.0L;
    return v * lam(u, v);
}

static ld rad(ld u, ld v) { return sqrtl(u * u + v * v); }

/* Returns 1 if the target touches the closed source rectangle anywhere other
 * than strictly inside it (edge or corner): the kernels diverge there. */
static int singular(ld u1, ld u2, ld v1, ld v2)
{
    int in_u = (u1 <= 0.0L && 0.0L <= u2);
    int in_v = (v1 <= 0.0L && 0.0L <= v2);
    if (in_u && (v1 == 0.0L || v2 == 0.0L)) return 1;
    if (in_v && (u1 == 0.0L || u2 == 0.0L)) return 1;
    return 0;
}

/*
 * Exact kernels of one source rectangle [xl,xr] x [yd,yu] at target (xt,yt),
 * Section 2 at z = 0.  out = {K^{x,0}, K^{x,x}, K^{x,y}, K^{y,0}, K^{y,x}, K^{y,y}}.
 * Returns 0, or -1 (and NaNs) if the target lies on the rectangle's boundary.
 */
int oracle_cell_kernels(double xt, double yt, double xl, double xr,
                        double yd, double yu, double *out)
{
    ld u1 = (ld)xl - (ld)xt, u2 = (ld)xr - (ld)xt;
    ld v1 = (ld)yd - (ld)yt, v2 = (ld)yu - (ld)yt;
    if (singular(u1, u2, v1, v2)) {
        for (int k = 0; k < 6; ++k) out[k] = NAN;
        return -1;
    }
    ld dxc = (ld)xt - 0.5L * ((ld)xl + (ld)xr); /* x_t - x_c */
    ld dyc = (ld)yt - 0.5L * ((ld)yd + (ld)yu); /* y_t - y_c */

    /* x family: inner differences taken along u */
    ld kx0 = -((lam(v2, u2) - lam(v2, u1)) - (lam(v1, u2) - lam(v1, u1)));
    ld iuu = (vlam(v2, u2) - vlam(v2, u1)) - (vlam(v1, u2) - vlam(v1, u1));
    ld iuv = -((rad(u2, v2) - rad(u1, v2)) - (rad(u2, v1) - rad(u1, v1)));
    /* y family: the same with x and y exchanged, inner differences along v */
    ld ky0 = -((lam(u2, v2) - lam(u2, v1)) - (lam(u1, v2) - lam(u1, v1)));
    ld ivv = (vlam(u2, v2) - vlam(u2, v1)) - (vlam(u1, v2) - vlam(u1, v1));
    ld ivu = -((rad(v2, u2) - rad(v1, u2)) - (rad(v2, u1) - rad(v1, u1)));

    out[0] = (double)kx0;
    out[1] = (double)(dxc * kx0 + iuu);
    out[2] = (double)(dyc * kx0 + iuv);
    out[3] = (double)ky0;
    out[4] = (double)(dxc * ky0 + ivu);
    out[5] = (double)(dyc * ky0 + ivv);
    return 0;
}

/* Neumaier's compensated summation (improved Kahan). */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

/* The compensated sum of n doubles in the given order, through the same
 * nadd / nval that every force sum below uses (exported so that the
 * summation itself can be checked against an exactly rounded sum). */
double oracle_nsum(int64_t n, const double *x)
{
    nsum a = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&a, x[i]);
    return nval(&a);
}

static int pick_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/*
 * Direct sum over arbitrary disjoint source rectangles (the leaf-by-leaf sum
 * of Section 2; the paper's AMR computation, O(targets x sources)).
 *   rect: nsrc x 4 doubles {xl, xr, yd, yu}
 *   sig, dsx, dsy: nsrc values (dsx/dsy may be NULL: zero slopes)
 *   txy: ntgt x 2 target coordinates
 * Returns 0, or -1 if some target touches a source boundary.
 */
int oracle_direct(int64_t nsrc, const double *rect, const double *sig,
                  const double *dsx, const double *dsy, int64_t ntgt,
                  const double *txy, double G, double *fx, double *fy,
                  int nthreads)
{
    int bad = 0;
    int nt = pick_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt) reduction(| : bad)
    for (int64_t t = 0; t < ntgt; ++t) {
        nsum ax = {0, 0}, ay = {0, 0};
        double xt = txy[2 * t], yt = txy[2 * t + 1];
        for (int64_t s = 0; s < nsrc; ++s) {
            double k[6];
            const double *r = rect + 4 * s;
            if (oracle_cell_kernels(xt, yt, r[0], r[1], r[2], r[3], k)) {
                bad = 1;
                continue;
            }
            double ex = 0.0, dx = dsx ? dsx[s] : 0.0, dy = dsy ? dsy[s] : 0.0;
            double ey;
            ex = sig[s] * k[0] + dx * k[1] + dy * k[2];
            ey = sig[s] * k[3] + dx * k[4] + dy * k[5];
            nadd(&ax, ex);
            nadd(&ay, ey);
        }
        fx[t] = G * nval(&ax);
        fy[t] = G * nval(&ay);
    }
    return bad ? -1 : 0;
}

/*
 * Uniform n x n grid of cells of size h with lower-left corner (x0, y0);
 * arrays are row-major, row j = y index, x fastest.  Targets are all cell
 * centres (or the subset listed in tgt, if ntgt > 0: flat cell indices).
 * The six kernels are evaluated once per offset (dx, dy) in cells and the
 * double sum is taken over every source cell, in row-major source order.
 */
int oracle_uniform(int n, double x0, double y0, double h, const double *sig,
                   const double *dsx, const double *dsy, double G,
                   int64_t ntgt, const int64_t *tgt, double *fx, double *fy,
                   int nthreads)
{
    (void)x0; (void)y0;
    if (n <= 0) return 0;
    int64_t w = 2 * (int64_t)n - 1;
    double *tab = (double *)malloc(sizeof(double) * 6 * (size_t)(w * w));
    if (!tab) return -2;
    int nt = pick_threads(nthreads);
    int bad = 0;
    /* offsets d = source - target in cells; target at the origin */
#pragma omp parallel for schedule(static) num_threads(nt) reduction(| : bad)
    for (int64_t q = 0; q < w * w; ++q) {
        int64_t dy = q / w - (n - 1), dx = q % w - (n - 1);
        double k[6];
        bad |= oracle_cell_kernels(0.0, 0.0, ((double)dx - 0.5) * h,
                                   ((double)dx + 0.5) * h, ((double)dy - 0.5) * h,
                                   ((double)dy + 0.5) * h, k) != 0;
        for (int c = 0; c < 6; ++c) tab[(size_t)c * w * w + q] = k[c];
    }
    int64_t ncell = (int64_t)n * n;
    int64_t nout = ntgt > 0 ? ntgt : ncell;
#pragma omp parallel for schedule(dynamic, 8) num_threads(nt)
    for (int64_t o = 0; o < nout; ++o) {
        int64_t cell = ntgt > 0 ? tgt[o] : o;
        int64_t ti = cell % n, tj = cell / n;
        nsum ax = {0, 0}, ay = {0, 0};
        for (int64_t sj = 0; sj < n; ++sj) {
            const double *rowt = tab + (sj - tj + n - 1) * w + (n - 1 - ti);
            const double *srow = sig + sj * n;
            const double *xrow = dsx ? dsx + sj * n : NULL;
            const double *yrow = dsy ? dsy + sj * n : NULL;
            for (int64_t si = 0; si < n; ++si) {
                const double *kk = rowt + si;
                size_t st = (size_t)w * w;
                double dx = xrow ? xrow[si] : 0.0, dy = yrow ? yrow[si] : 0.0;
                double ex = srow[si] * kk[0] + dx * kk[st] + dy * kk[2 * st];
                double ey = srow[si] * kk[3 * st] + dx * kk[4 * st] + dy * kk[5 * st];
                nadd(&ax, ex);
                nadd(&ay, ey);
            }
        }
        fx[o] = G * nval(&ax);
        fy[o] = G * nval(&ay);
    }
    free(tab);
    return bad ? -1 : 0;
}

/*
 * Off-plane targets (Section 2 at z != 0): the target sits at height z above
 * the disk plane z = 0.  Written from the defining integrals with
 * R = sqrt(u^2 + v^2 + z^2) and a = |z| > 0:
 *
 *   K^{x,0} = integral of u / R^3          = -DD[ ln(v + R) ]
 *   I_uu    = integral of u^2 / R^3        =  DD[ v ln(u + R) - a atan(u v / (a R)) ]
 *   I_uv    = integral of u v / R^3        = -DD[ R ]
 *   J       = integral of 1 / R^3          =  DD[ atan(u v / (a R)) ] / a
 *   K^{z,0} = integral of (0 - z) / R^3    = -z J
 *   K^{x,x} = (x_t - x_c) K^{x,0} + I_uu,     K^{x,y} = (y_t - y_c) K^{x,0} + I_uv
 *   K^{z,x} = (x_t - x_c) K^{z,0} - z K^{x,0}, K^{z,y} = (y_t - y_c) K^{z,0} - z K^{y,0}
 *
 * (the y family by exchanging x and y), and F = G sum_i [s_i K^{.,0} +
 * dx_i K^{.,x} + dy_i K^{.,y}] for each of the three components.  The paper
 * prints the arctangent arguments with the target coordinates; the
 * integrals fix them to the corner offsets u v, as used here.  With z != 0
 * nothing is singular.  ln(b + R) for b < 0 is evaluated as
 * ln((R^2 - b^2) / (R - b)), the identity that avoids cancellation.
 */
static ld lnz(ld b, ld c, ld a2) /* ln(b + sqrt(b^2 + c^2 + a2)) */
{
    ld R = sqrtl(b * b + c * c + a2);
    if (b >= 0.0L) return logl(b + R);
    return logl((c * c + a2) / (R - b));
}
static ld atz(ld u, ld v, ld a) /* atan(u v / (a R)) */
{
    ld R = sqrtl(u * u + v * v + a * a);
    return atanl(u * v / (a * R));
}

/*
 * Exact kernels of one source rectangle at target (xt, yt, z), z != 0.
 * out = {K^{x,0}, K^{x,x}, K^{x,y}, K^{y,0}, K^{y,x}, K^{y,y},
 *        K^{z,0}, K^{z,x}, K^{z,y}}.  Returns 0, or -1 (NaNs) for z == 0.
 */
int oracle_cell_kernels_z(double xt, double yt, double z, double xl, double xr,
                          double yd, double yu, double *out)
{
    if (z == 0.0 || !isfinite(z)) {
        for (int k = 0; k < 9; ++k) out[k] = NAN;
        return -1;
    }
    ld u[2] = {(ld)xl - (ld)xt, (ld)xr - (ld)xt};
    ld v[2] = {(ld)yd - (ld)yt, (ld)yu - (ld)yt};
    ld zz = (ld)z, a = fabsl(zz), a2 = a * a;
    ld dxc = (ld)xt - 0.5L * ((ld)xl + (ld)xr);
    ld dyc = (ld)yt - 0.5L * ((ld)yd + (ld)yu);
    ld kx0 = 0, iuu = 0, iuv = 0, ky0 = 0, ivv = 0, jj = 0;
    /* DD[f] = f(u2,v2) - f(u1,v2) - f(u2,v1) + f(u1,v1) */
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            ld sgn = ((i + j) % 2 == 0) ? 1.0L : -1.0L; /* (1,1) and (0,0): +, mixed: - */
            ld R = sqrtl(u[i] * u[i] + v[j] * v[j] + a2);
            ld at = atz(u[i], v[j], a);
            kx0 += sgn * -lnz(v[j], u[i], a2);
            ky0 += sgn * -lnz(u[i], v[j], a2);
            iuu += sgn * (v[j] * lnz(u[i], v[j], a2) - a * at);
            ivv += sgn * (u[i] * lnz(v[j], u[i], a2) - a * at);
            iuv += sgn * -R;
            jj += sgn * at;
        }
    jj /= a;
    ld kz0 = -zz * jj;
    out[0] = (double)kx0;
    out[1] = (double)(dxc * kx0 + iuu);
    out[2] = (double)(dyc * kx0 + iuv);
    out[3] = (double)ky0;
    out[4] = (double)(dxc * ky0 + iuv);
    out[5] = (double)(dyc * ky0 + ivv);
    out[6] = (double)kz0;
    out[7] = (double)(dxc * kz0 - zz * kx0);
    out[8] = (double)(dyc * kz0 - zz * ky0);
    return 0;
}

/*
 * Direct sum for targets at height z != 0 above the disk (same arguments as
 * oracle_direct, plus z and the third component fz).
 */
int oracle_direct_z(int64_t nsrc, const double *rect, const double *sig,
                    const double *dsx, const double *dsy, int64_t ntgt,
                    const double *txy, double z, double G, double *fx, double *fy,
                    double *fz, int nthreads)
{
    if (z == 0.0 || !isfinite(z)) return -1;
    int nt = pick_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t t = 0; t < ntgt; ++t) {
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        double xt = txy[2 * t], yt = txy[2 * t + 1];
        for (int64_t s = 0; s < nsrc; ++s) {
            double k[9];
            const double *r = rect + 4 * s;
            oracle_cell_kernels_z(xt, yt, z, r[0], r[1], r[2], r[3], k);
            double dx = dsx ? dsx[s] : 0.0, dy = dsy ? dsy[s] : 0.0;
            nadd(&ax, sig[s] * k[0] + dx * k[1] + dy * k[2]);
            nadd(&ay, sig[s] * k[3] + dx * k[4] + dy * k[5]);
            nadd(&az, sig[s] * k[6] + dx * k[7] + dy * k[8]);
        }
        fx[t] = G * nval(&ax);
        fy[t] = G * nval(&ay);
        fz[t] = G * nval(&az);
    }
    return 0;
}

/* Number of threads OpenMP would use by default (for reporting). */
int oracle_max_threads(void) { return pick_threads(0); }
