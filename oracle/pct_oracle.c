/*
 * pct_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for the proton-CT
 * data simulator of Witt et al., "A Proton Simulator for Testing Implementations of
 * Proton CT Reconstruction Algorithms on GPGPU Clusters" (arXiv 2108.12369).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The product path never does; it shares no
 * code, header, table or constant with this file.
 *
 * What it computes (paper passages in brackets):
 *   - the true solution vector x of Ax=b: voxelised RSP of a phantom made of ellipse /
 *     ellipsoid regions ("non-homogeneous ellipse object") with the center-point or the
 *     corner-point-averaging rule [Sec. II-A];
 *   - per proton: a parallel-beam entry offset drawn uniformly along t (and v in 3D)
 *     [Sec. II-B], the projection angle of its beam [Sec. II-B], entry and exit points
 *     against the outer boundary [Sec. II-B], a straight or cubic-spline path with
 *     Gaussian multiple-scattering deflections drawn with the Marsaglia polar method and
 *     turned into a correlated pair through the covariance matrix [Sec. II-B, bivariate
 *     normal density], and straight continuation outside the phantom [Sec. II-B];
 *   - the path mapped from the beam frame (t,v,u) to the fixed frame (x,y,z) by a
 *     Givens rotation and intersected with the voxels by a digital-difference traversal,
 *     giving one CSR row of A whose entries are the chord lengths of the path in each
 *     voxel [Sec. II-C];
 *   - the WEPL b_i as the inner product of row i with x, optionally with noise
 *     [Sec. II-C];
 *   - optionally, exit-pair widths per proton from Highland's formula [Sec. II-B];
 *   - the string-averaging projection (SAP) reconstruction that consumes A and b
 *     [Sec. II-D].
 * Where the paper is silent the readings are those listed in the design notes of the
 * repository (Gaussian relative WEPL noise instead of the PSTAR/Tschalar model, a
 * counter-based Philox4x32-10 generator instead of C rand(), a cubic Hermite curve for
 * the "cubic-spline" path, exact chord lengths instead of the constant pixel length).
 *
 * Every value is computed in IEEE binary64, built with -ffp-contract=off so that no
 * multiply-add is fused behind the reader's back.  No blocking, fusion or reordering
 * beyond the definitions below.
 *
 * Per row the oracle also reports a "margin" (mm): how close any integer decision of
 * the traversal came to flipping (a sample or clipped end point near an interior voxel
 * face, two face crossings at nearly the same point, a path grazing the grid box, a
 * near-tangent boundary solve, a Hermite sample count at a rounding edge).  Rows with a
 * margin below 1e-6 mm are the ones whose column sequence may legitimately differ in
 * another correct implementation that rounds differently.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ public structs */

enum { OR_ELLIPSE = 0, OR_ELLIPSOID = 1 };          /* ellipse ignores z (cylinder in 3D) */
enum { OR_CORNER_AVG = 0, OR_CENTER = 1, OR_AREA_AVG = 2 };
enum { OR_STRAIGHT = 0, OR_HERMITE = 1 };
enum { OR_KIND_MISS_GRID = 0, OR_KIND_STRAIGHT = 1, OR_KIND_CURVED = 2,
       OR_KIND_STRAIGHT_FALLBACK = 3 };

typedef struct {
    int32_t shape;
    double center[3];
    double semi[3];
    float rsp;
    double angle_deg;       /* semi-axes turned counterclockwise in the x-y plane */
} or_region;

typedef struct {
    int32_t dim;            /* 2 or 3 */
    int32_t n[3];           /* voxels per axis; n[2] ignored in 2D */
    double h[3];            /* voxel size (mm) */
    double origin[3];       /* lower corner of the grid box (mm) */
    int32_t n_regions;
    const or_region *regions;  /* painter's order, region 0 is the outer boundary */
    int32_t voxelize;
    int32_t area_samples;      /* weighted-area rule: midpoints per axis */
} or_phantom;

typedef struct {
    uint64_t seed;
    int32_t n_angles;
    double angle0_deg, dangle_deg;
    int64_t n_protons;
    double t_range[2], v_range[2];
    int32_t path;
    double sigma_in, sigma_out, sigma_lat, rho, step;
    double noise_rel;
    int32_t scatter;        /* 0: widths as given; 1: Highland per proton */
    double energy_mev;      /* Highland: constant kinetic energy */
    double x0_mm;           /* Highland: radiation length of the medium */
} or_beam;

/* ------------------------------------------------------------ Philox4x32-10 (RNG) */
/* Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11:
 * a round multiplies counter words 0 and 2 by two odd constants, keeps the high and
 * low halves of both 64-bit products, xors the high halves with the other two counter
 * words and the key, and permutes; the key is bumped by two Weyl increments between
 * rounds; ten rounds. */

static void or_philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    const uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        or_philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* Draw `draw` of stream `stream` for proton g: counter (draw, stream, g_lo, g_hi),
 * key (seed_lo, seed_hi); returned as two 64-bit words (out0|out1<<32, out2|out3<<32). */
void or_draw64(uint64_t seed, uint32_t stream, uint64_t g, uint32_t draw, uint64_t w[2])
{
    const uint32_t ctr[4] = {draw, stream, (uint32_t)g, (uint32_t)(g >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    w[0] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    w[1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
}

/* Uniform double in [0,1) from the top 53 bits of a 64-bit word. */
double or_uniform53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

/* Marsaglia polar method [Sec. II-B]: two independent standard normals from uniform
 * pairs; attempt a uses draw a of the stream; after 64 rejections both are 0. */
int or_normal_pair(uint64_t seed, uint32_t stream, uint64_t g, double *z1, double *z2)
{
    for (uint32_t a = 0; a < 64; ++a) {
        uint64_t w[2];
        or_draw64(seed, stream, g, a, w);
        const double v1 = 2.0 * or_uniform53(w[0]) - 1.0;
        const double v2 = 2.0 * or_uniform53(w[1]) - 1.0;
        const double s = v1 * v1 + v2 * v2;
        if (s > 0.0 && s < 1.0) {
            const double f = sqrt(-2.0 * log(s) / s);
            *z1 = v1 * f;
            *z2 = v2 * f;
            return (int)a + 1;
        }
    }
    *z1 = 0.0;
    *z2 = 0.0;
    return 0;
}

/* ------------------------------------------------------------------- beam geometry */

/* Projection angle k in degrees; cosine and sine exact at multiples of 90 degrees. */
void or_angle(double angle0_deg, double dangle_deg, int32_t k, double *c, double *s)
{
    const double phi = angle0_deg + (double)k * dangle_deg;
    const double q = phi / 90.0;
    if (floor(q) == q) {
        long m = (long)fmod(q, 4.0);
        if (m < 0) m += 4;
        static const double C[4] = {1.0, 0.0, -1.0, 0.0};
        static const double S[4] = {0.0, 1.0, 0.0, -1.0};
        *c = C[m];
        *s = S[m];
        return;
    }
    const double rad = phi * (3.14159265358979323846 / 180.0);
    *c = cos(rad);
    *s = sin(rad);
}

/* Angle-major proton order: angle k holds protons [floor(kP/K), floor((k+1)P/K)). */
int32_t or_angle_of(int64_t g, int64_t P, int32_t K)
{
    return (int32_t)((((g + 1) * (int64_t)K) - 1) / P);
}

static double dot3(const double a[3], const double b[3]) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }

static void normalize3(double v[3])
{
    const double n = sqrt(dot3(v, v));
    v[0] /= n; v[1] /= n; v[2] /= n;
}

/* Line Q + l d against the outer boundary (region 0) [Sec. II-B entry and exit points].
 * Returns 1 on a hit with l1 < l2.  *half_chord (mm) is sqrt(|disc|)/a * |d|: how far
 * the line is from being tangent (imaginary for a miss). */
/* A vector expressed in the frame of a region's turned semi-axes: rotation by minus the
 * region's angle in the x-y plane (z unchanged). */
static void to_region_frame(const or_region *r, const double v[3], double u[3])
{
    u[0] = v[0];
    u[1] = v[1];
    u[2] = v[2];
    if (r->angle_deg != 0.0) {
        const double ang = r->angle_deg * (3.14159265358979323846 / 180.0);
        const double c = cos(ang), s = sin(ang);
        u[0] = c * v[0] + s * v[1];
        u[1] = c * v[1] - s * v[0];
    }
}

int or_boundary_hit(const or_phantom *ph, const double Q[3], const double d[3],
                    double *l1, double *l2, double *half_chord)
{
    const or_region *r = &ph->regions[0];
    const int naxes = (r->shape == OR_ELLIPSOID && ph->dim == 3) ? 3 : 2;
    double a = 0.0, b = 0.0, c = -1.0;
    const double qc[3] = {Q[0] - r->center[0], Q[1] - r->center[1], Q[2] - r->center[2]};
    double qr[3], dr[3];
    to_region_frame(r, qc, qr);
    to_region_frame(r, d, dr);
    for (int i = 0; i < naxes; ++i) {
        const double q = qr[i];
        const double s2 = r->semi[i] * r->semi[i];
        a += dr[i] * dr[i] / s2;
        b += q * dr[i] / s2;
        c += q * q / s2;
    }
    const double disc = b * b - a * c;
    *half_chord = (a > 0.0) ? sqrt(fabs(disc)) / a * sqrt(dot3(d, d)) : 0.0;
    if (!(a > 0.0) || !(disc > 0.0)) return 0;
    const double sq = sqrt(disc);
    /* numerically stable pair of roots */
    const double t = (b >= 0.0) ? -(b + sq) : (-b + sq);
    double r1 = t / a, r2 = c / t;
    if (r1 > r2) { const double tmp = r1; r1 = r2; r2 = tmp; }
    *l1 = r1;
    *l2 = r2;
    return 1;
}

/* Cubic Hermite curve between P0 and P1 with tangents L d0 and L d1 [Sec. II-B spline]. */
void or_hermite(const double P0[3], const double d0[3], const double P1[3], const double d1[3],
                double L, double s, double out[3])
{
    const double s2 = s * s, s3 = s2 * s;
    const double h00 = 2.0 * s3 - 3.0 * s2 + 1.0;
    const double h10 = s3 - 2.0 * s2 + s;
    const double h01 = -2.0 * s3 + 3.0 * s2;
    const double h11 = s3 - s2;
    for (int i = 0; i < 3; ++i)
        out[i] = h00 * P0[i] + h10 * L * d0[i] + h01 * P1[i] + h11 * L * d1[i];
}

/* ------------------------------------------------------------------------- phantom */

static int region_contains(const or_region *r, int dim, const double p[3])
{
    const int naxes = (r->shape == OR_ELLIPSOID && dim == 3) ? 3 : 2;
    const double v[3] = {p[0] - r->center[0], p[1] - r->center[1], p[2] - r->center[2]};
    double w[3];
    to_region_frame(r, v, w);
    double q = 0.0;
    for (int i = 0; i < naxes; ++i) {
        const double u = w[i] / r->semi[i];
        q += u * u;
    }
    return q <= 1.0;
}

/* RSP at a point: the last region (painter's order) containing it, else air (0). */
double or_rsp_at(const or_phantom *ph, const double p[3])
{
    double v = 0.0;
    for (int k = 0; k < ph->n_regions; ++k)
        if (region_contains(&ph->regions[k], ph->dim, p)) v = (double)ph->regions[k].rsp;
    return v;
}

/* True solution vector x, x fastest then y then z [Sec. II-A pixel value rules]. */
void or_phantom_build(const or_phantom *ph, float *x)
{
    const int nz = (ph->dim == 3) ? ph->n[2] : 1;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ph->n[1]; ++iy)
            for (int ix = 0; ix < ph->n[0]; ++ix) {
                const int idx[3] = {ix, iy, iz};
                double val = 0.0;
                if (ph->voxelize == OR_AREA_AVG) {
                    /* weighted-area average: each region's RSP times the fraction of the
                     * voxel it covers (painter's order), the fractions taken over S^dim
                     * midpoints (i + 1/2) / S per axis */
                    const int S = ph->area_samples;
                    const int sz = (ph->dim == 3) ? S : 1;
                    double sum = 0.0;
                    for (int kz = 0; kz < sz; ++kz)
                        for (int ky = 0; ky < S; ++ky)
                            for (int kx = 0; kx < S; ++kx) {
                                const int k[3] = {kx, ky, kz};
                                double p[3] = {0, 0, 0};
                                for (int d = 0; d < ph->dim; ++d)
                                    p[d] = ph->origin[d] + ((double)idx[d] + ((double)k[d] + 0.5) / (double)S) * ph->h[d];
                                sum += or_rsp_at(ph, p);
                            }
                    val = sum / ((double)S * (double)S * (double)sz);
                } else if (ph->voxelize == OR_CENTER) {
                    double p[3] = {0, 0, 0};
                    for (int d = 0; d < ph->dim; ++d)
                        p[d] = ph->origin[d] + ((double)idx[d] + 0.5) * ph->h[d];
                    val = or_rsp_at(ph, p);
                } else {
                    const int ncorner = 1 << ph->dim;
                    double sum = 0.0;
                    for (int c = 0; c < ncorner; ++c) {
                        double p[3] = {0, 0, 0};
                        for (int d = 0; d < ph->dim; ++d)
                            p[d] = ph->origin[d] + (double)(idx[d] + ((c >> d) & 1)) * ph->h[d];
                        sum += or_rsp_at(ph, p);
                    }
                    val = sum / (double)ncorner;
                }
                x[(int64_t)ix + (int64_t)ph->n[0] * ((int64_t)iy + (int64_t)ph->n[1] * iz)] = (float)val;
            }
}

/* ---------------------------------------------------------------- row accumulation */

typedef struct {
    int32_t *cols;
    double *vals;
    int64_t n, cap;
} or_vec;

static void vec_push(or_vec *v, int32_t col, double len)
{
    if (v->n == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 1024;
        v->cols = (int32_t *)realloc(v->cols, (size_t)v->cap * sizeof(int32_t));
        v->vals = (double *)realloc(v->vals, (size_t)v->cap * sizeof(double));
    }
    v->cols[v->n] = col;
    v->vals[v->n] = len;
    v->n++;
}

typedef struct {
    const or_phantom *ph;
    or_vec *out;
    int64_t row_start;     /* index in out of this row's first entry */
    double margin;         /* mm */
    int fragile;
} or_row;

static void margin_min(or_row *row, double m)
{
    if (m < row->margin) row->margin = m;
}

static int grid_n(const or_phantom *ph, int d) { return (d < ph->dim) ? ph->n[d] : 1; }

static int32_t voxel_index(const or_phantom *ph, int d, double p)
{
    const double f = floor((p - ph->origin[d]) / ph->h[d]);
    const int n = grid_n(ph, d);
    if (f < 0.0) return 0;
    if (f > (double)(n - 1)) return n - 1;
    return (int32_t)f;
}

/* distance of a point to the nearest interior face (faces 1..n-1) along every axis */
static void point_margin(or_row *row, const double p[3])
{
    const or_phantom *ph = row->ph;
    for (int d = 0; d < ph->dim; ++d) {
        const int n = ph->n[d];
        if (n < 2) continue;
        const double f = (p[d] - ph->origin[d]) / ph->h[d];
        double j = floor(f + 0.5);
        if (j < 1.0) j = 1.0;
        if (j > (double)(n - 1)) j = (double)(n - 1);
        margin_min(row, fabs(f - j) * ph->h[d]);
    }
}

static void emit(or_row *row, int first_of_segment, int32_t col, double len)
{
    or_vec *v = row->out;
    if (first_of_segment && v->n > row->row_start && v->cols[v->n - 1] == col) {
        v->vals[v->n - 1] += len;   /* same voxel across a joint of the path */
        return;
    }
    vec_push(v, col, len);
}

/* Traverse the part of the segment A + l D, l in [lo, hi], that lies in the grid box.
 * If B is given it is the exact point at l = hi (a Hermite sample) and replaces A+hi*D
 * when the upper end is not clipped.  Chord length in voxel = (l_out - l_in) |D|. */
static void trace_segment(or_row *row, const double A[3], const double D[3], double lo, double hi,
                          const double *B)
{
    const or_phantom *ph = row->ph;
    const int dim = ph->dim;
    const double hi0 = hi;
    for (int d = 0; d < dim; ++d) {
        const double box_lo = ph->origin[d];
        const double box_hi = ph->origin[d] + (double)ph->n[d] * ph->h[d];
        if (D[d] != 0.0) {
            const double t1 = (box_lo - A[d]) / D[d];
            const double t2 = (box_hi - A[d]) / D[d];
            lo = fmax(lo, fmin(t1, t2));
            hi = fmin(hi, fmax(t1, t2));
        } else {
            margin_min(row, fmin(fabs(A[d] - box_lo), fabs(A[d] - box_hi)));
            if (A[d] < box_lo || A[d] > box_hi) return;
        }
    }
    double Dn2 = 0.0;
    for (int d = 0; d < dim; ++d) Dn2 += D[d] * D[d];
    const double Dn = sqrt(Dn2);
    if (isfinite(lo) && isfinite(hi)) margin_min(row, fabs(hi - lo) * Dn);
    if (!(lo < hi)) return;

    double P[3] = {0, 0, 0}, E[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        P[d] = A[d] + lo * D[d];
        E[d] = (hi == hi0 && B) ? B[d] : A[d] + hi * D[d];
    }
    point_margin(row, P);
    point_margin(row, E);

    int32_t i[3] = {0, 0, 0}, e[3] = {0, 0, 0}, s[3] = {0, 0, 0}, budget[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        i[d] = voxel_index(ph, d, P[d]);
        e[d] = voxel_index(ph, d, E[d]);
        budget[d] = abs(e[d] - i[d]);
        s[d] = (e[d] > i[d]) ? 1 : -1;
    }
    const int64_t nx = ph->n[0], ny = ph->n[1];
    double lp = lo;
    int first = 1;
    for (;;) {
        int a = -1;
        double la = 0.0, second = INFINITY;
        for (int d = 0; d < dim; ++d) {
            if (budget[d] == 0) continue;
            const double plane = ph->origin[d] + (double)(i[d] + (s[d] > 0 ? 1 : 0)) * ph->h[d];
            const double ld = (D[d] != 0.0) ? (plane - A[d]) / D[d] : INFINITY;
            if (a < 0 || ld < la) {
                if (a >= 0) second = fmin(second, la);
                a = d;
                la = ld;
            } else {
                second = fmin(second, ld);
            }
        }
        if (a < 0) break;
        if (isfinite(second)) margin_min(row, (second - la) * Dn);
        const double lc = fmin(fmax(la, lp), hi);
        emit(row, first, (int32_t)(i[0] + nx * (i[1] + ny * i[2])), (lc - lp) * Dn);
        first = 0;
        lp = lc;
        i[a] += s[a];
        budget[a] -= 1;
    }
    emit(row, first, (int32_t)(i[0] + nx * (i[1] + ny * i[2])), (hi - lp) * Dn);
}

/* ---------------------------------------------------------------------- proton rows */

typedef struct {
    int32_t kind;
    int32_t n_samples;     /* Hermite N */
    double t, v;
    double P0[3], P1[3], d0[3], d1[3];
    double L;
    double thickness;      /* straight entry line inside the outer boundary (mm) */
    double sigma_out, sigma_lat, rho;   /* exit-pair widths and correlation used */
} or_path;

/* Highland's projected width of the multiple-scattering angle with the Particle Data
 * Group constants [Sec. II-B]: for a particle of unit charge, momentum p and speed
 * beta c after a thickness x of a medium of radiation length X0,
 *     theta0 = 13.6 MeV / (beta c p) sqrt(x / X0) (1 + 0.038 ln(x / (X0 beta^2))).
 * The proton keeps the kinetic energy T over the whole path: with the rest energy m,
 * p c = sqrt(T^2 + 2 T m) and beta = p c / (T + m).  Where the bracket would be
 * negative (thicknesses far below the formula's range) the width is 0. */
double or_highland(double T_mev, double x0_mm, double x_mm)
{
    const double m = 938.27208816;      /* proton rest energy, MeV */
    const double pc = sqrt(T_mev * T_mev + 2.0 * T_mev * m);
    const double beta = pc / (T_mev + m);
    if (!(x_mm > 0.0)) return 0.0;
    const double bracket = 1.0 + 0.038 * log(x_mm / (x0_mm * beta * beta));
    if (bracket < 0.0) return 0.0;
    return 13.6 / (beta * pc) * sqrt(x_mm / x0_mm) * bracket;
}

static void tangency(or_row *row, double half_chord)
{
    if (half_chord < 1e-4) row->fragile = 1;
}

/* Build and traverse the path of proton g [Sec. II-B, II-C]. */
static void trace_proton(or_row *row, const or_beam *bm, int64_t g, or_path *path)
{
    const or_phantom *ph = row->ph;
    const int dim = ph->dim;
    const int32_t k = or_angle_of(g, bm->n_protons, bm->n_angles);
    double c, s;
    or_angle(bm->angle0_deg, bm->dangle_deg, k, &c, &s);
    const double u_hat[3] = {c, s, 0.0};
    const double t_hat[3] = {-s, c, 0.0};
    const double v_hat[3] = {0.0, 0.0, 1.0};

    uint64_t w[2];
    or_draw64(bm->seed, 0, (uint64_t)g, 0, w);
    const double t = bm->t_range[0] + (bm->t_range[1] - bm->t_range[0]) * or_uniform53(w[0]);
    const double v = (dim == 3) ? bm->v_range[0] + (bm->v_range[1] - bm->v_range[0]) * or_uniform53(w[1]) : 0.0;
    double Q[3];
    for (int i = 0; i < 3; ++i) Q[i] = t * t_hat[i] + v * v_hat[i];

    memset(path, 0, sizeof *path);
    path->t = t;
    path->v = v;

    if (bm->path == OR_STRAIGHT) {
        path->kind = OR_KIND_STRAIGHT;
        memcpy(path->d0, u_hat, sizeof u_hat);
        trace_segment(row, Q, u_hat, -INFINITY, INFINITY, NULL);
        return;
    }

    /* entry direction: projected angular deflections in the ut and uv planes */
    double zt, zv;
    or_normal_pair(bm->seed, 1, (uint64_t)g, &zt, &zv);
    const double tan_t_in = tan(bm->sigma_in * zt);
    const double tan_v_in = (dim == 3) ? tan(bm->sigma_in * zv) : 0.0;
    double d0[3];
    for (int i = 0; i < 3; ++i) d0[i] = u_hat[i] + tan_t_in * t_hat[i] + tan_v_in * v_hat[i];
    normalize3(d0);
    memcpy(path->d0, d0, sizeof d0);

    double l1, l2, hc;
    const int hit = or_boundary_hit(ph, Q, d0, &l1, &l2, &hc);
    tangency(row, hc);
    if (!hit) {
        path->kind = OR_KIND_STRAIGHT_FALLBACK;
        trace_segment(row, Q, d0, -INFINITY, INFINITY, NULL);
        return;
    }
    double P0[3], P1s[3];
    for (int i = 0; i < 3; ++i) { P0[i] = Q[i] + l1 * d0[i]; P1s[i] = Q[i] + l2 * d0[i]; }

    /* exit pair per plane: lateral displacement and exit angle, correlation rho; with
     * Highland's model the widths follow from the thickness x of the phantom along the
     * entry line, as for a uniform slab: sigma_out = theta0, sigma_lat = theta0 x / sqrt 3,
     * correlation sqrt(3) / 2 */
    double sig_out = bm->sigma_out, sig_lat = bm->sigma_lat, rho = bm->rho;
    path->thickness = l2 - l1;
    if (bm->scatter == 1) {
        const double x = l2 - l1;
        sig_out = or_highland(bm->energy_mev, bm->x0_mm, x);
        sig_lat = sig_out * x / sqrt(3.0);
        rho = sqrt(3.0) / 2.0;
    }
    path->sigma_out = sig_out;
    path->sigma_lat = sig_lat;
    path->rho = rho;
    const double cr = sqrt(1.0 - rho * rho);
    double z1, z2;
    or_normal_pair(bm->seed, 2, (uint64_t)g, &z1, &z2);
    const double lat_t = sig_lat * z1;
    const double ang_t = sig_out * (rho * z1 + cr * z2);
    double lat_v = 0.0, ang_v = 0.0;
    if (dim == 3) {
        or_normal_pair(bm->seed, 3, (uint64_t)g, &z1, &z2);
        lat_v = sig_lat * z1;
        ang_v = sig_out * (rho * z1 + cr * z2);
    }
    double nt[3], nv[3];
    const double tdot = dot3(t_hat, d0), vdot = dot3(v_hat, d0);
    for (int i = 0; i < 3; ++i) { nt[i] = t_hat[i] - tdot * d0[i]; nv[i] = v_hat[i] - vdot * d0[i]; }
    normalize3(nt);
    if (dim == 3) normalize3(nv); else { nv[0] = nv[1] = nv[2] = 0.0; }

    double Qd[3];
    for (int i = 0; i < 3; ++i) Qd[i] = Q[i] + lat_t * nt[i] + lat_v * nv[i];
    double P1[3];
    double m1, m2, hc2;
    if (or_boundary_hit(ph, Qd, d0, &m1, &m2, &hc2)) {
        for (int i = 0; i < 3; ++i) P1[i] = Qd[i] + m2 * d0[i];
    } else {
        memcpy(P1, P1s, sizeof P1);
    }
    tangency(row, hc2);

    double d1[3];
    const double tan_t_out = tan(ang_t), tan_v_out = tan(ang_v);
    for (int i = 0; i < 3; ++i) d1[i] = d0[i] + tan_t_out * nt[i] + tan_v_out * nv[i];
    normalize3(d1);

    double dP[3];
    for (int i = 0; i < 3; ++i) dP[i] = P1[i] - P0[i];
    const double L = sqrt(dot3(dP, dP));
    const double steps = L / bm->step;
    int64_t N = (int64_t)ceil(steps);
    if (N < 1) N = 1;
    if (fabs(steps - floor(steps + 0.5)) * bm->step < 1e-9) row->fragile = 1;

    path->kind = OR_KIND_CURVED;
    path->n_samples = (int32_t)N;
    path->L = L;
    memcpy(path->P0, P0, sizeof P0);
    memcpy(path->P1, P1, sizeof P1);
    memcpy(path->d1, d1, sizeof d1);

    /* straight line before the entry point */
    trace_segment(row, P0, d0, -INFINITY, 0.0, NULL);
    /* the spline, as chords between N+1 uniform parameter samples */
    double A[3];
    memcpy(A, P0, sizeof A);
    for (int64_t j = 1; j <= N; ++j) {
        double B[3];
        if (j == N) memcpy(B, P1, sizeof B);
        else or_hermite(P0, d0, P1, d1, L, (double)j / (double)N, B);
        const double D[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        trace_segment(row, A, D, 0.0, 1.0, B);
        memcpy(A, B, sizeof A);
    }
    /* straight line after the exit point */
    trace_segment(row, P1, d1, 0.0, INFINITY, NULL);
}

/* ----------------------------------------------------------------------- run rows */

typedef struct {
    int64_t nrows;
    int64_t *row_ptr;     /* nrows + 1 */
    or_vec entries;
    double *b;            /* with noise if noise_rel > 0 */
    double *b_clean;
    double *margin;
    or_path *paths;
} or_result;

/* Rows are global proton ids.  x must be the phantom's stored (binary32) solution. */
or_result *or_run(const or_phantom *ph, const or_beam *bm, const float *x,
                  const int64_t *rows, int64_t nrows)
{
    or_result *res = (or_result *)calloc(1, sizeof *res);
    res->nrows = nrows;
    res->row_ptr = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    res->b = (double *)calloc((size_t)nrows + 1, sizeof(double));
    res->b_clean = (double *)calloc((size_t)nrows + 1, sizeof(double));
    res->margin = (double *)calloc((size_t)nrows + 1, sizeof(double));
    res->paths = (or_path *)calloc((size_t)nrows + 1, sizeof(or_path));
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t g = rows[r];
        or_row row = {ph, &res->entries, res->entries.n, INFINITY, 0};
        trace_proton(&row, bm, g, &res->paths[r]);
        const int64_t n0 = row.row_start, n1 = res->entries.n;
        if (n1 == n0 && res->paths[r].kind != OR_KIND_CURVED) res->paths[r].kind = OR_KIND_MISS_GRID;
        /* WEPL: inner product of the row with the stored solution vector */
        double b = 0.0;
        for (int64_t e = n0; e < n1; ++e) b += res->entries.vals[e] * (double)x[res->entries.cols[e]];
        res->b_clean[r] = b;
        if (bm->noise_rel > 0.0) {
            double z1, z2;
            or_normal_pair(bm->seed, 4, (uint64_t)g, &z1, &z2);
            b = b * (1.0 + bm->noise_rel * z1);
        }
        res->b[r] = b;
        res->margin[r] = row.fragile ? 0.0 : row.margin;
        res->row_ptr[r + 1] = n1;
    }
    return res;
}

/* Traverse an arbitrary list of segments as one row (used by the pins). */
or_result *or_trace_segments(const or_phantom *ph, int32_t nseg, const double *A, const double *D,
                             const double *lo, const double *hi)
{
    or_result *res = (or_result *)calloc(1, sizeof *res);
    res->nrows = 1;
    res->row_ptr = (int64_t *)calloc(2, sizeof(int64_t));
    res->margin = (double *)calloc(1, sizeof(double));
    or_row row = {ph, &res->entries, 0, INFINITY, 0};
    for (int32_t k = 0; k < nseg; ++k) trace_segment(&row, A + 3 * k, D + 3 * k, lo[k], hi[k], NULL);
    res->row_ptr[1] = res->entries.n;
    res->margin[0] = row.margin;
    return res;
}

int64_t or_result_nnz(const or_result *r) { return r->entries.n; }

void or_result_copy(const or_result *r, int64_t *row_ptr, int32_t *cols, double *vals, double *b,
                    double *b_clean, double *margin, or_path *paths)
{
    if (row_ptr) memcpy(row_ptr, r->row_ptr, (size_t)(r->nrows + 1) * sizeof(int64_t));
    if (cols && r->entries.n) memcpy(cols, r->entries.cols, (size_t)r->entries.n * sizeof(int32_t));
    if (vals && r->entries.n) memcpy(vals, r->entries.vals, (size_t)r->entries.n * sizeof(double));
    if (b && r->b) memcpy(b, r->b, (size_t)r->nrows * sizeof(double));
    if (b_clean && r->b_clean) memcpy(b_clean, r->b_clean, (size_t)r->nrows * sizeof(double));
    if (margin) memcpy(margin, r->margin, (size_t)r->nrows * sizeof(double));
    if (paths && r->paths) memcpy(paths, r->paths, (size_t)r->nrows * sizeof(or_path));
}

void or_result_free(or_result *r)
{
    if (!r) return;
    free(r->row_ptr);
    free(r->entries.cols);
    free(r->entries.vals);
    free(r->b);
    free(r->b_clean);
    free(r->margin);
    free(r->paths);
    free(r);
}

int32_t or_sizeof_path(void) { return (int32_t)sizeof(or_path); }
int32_t or_sizeof_region(void) { return (int32_t)sizeof(or_region); }
int32_t or_sizeof_phantom(void) { return (int32_t)sizeof(or_phantom); }
int32_t or_sizeof_beam(void) { return (int32_t)sizeof(or_beam); }

/* ------------------------------------------------------- SAP reconstruction [Sec. II-D] */
/* String-averaging projections on A x = b (A in CSR: m rows, n columns).  One iteration
 * from the iterate x_k: for every string t (rows order[s_t] .. order[s_{t+1} - 1], with
 * s_t = floor(t m / M)), y starts at x_k and takes, row by row in string order, the
 * relaxed projection onto the row's hyperplane
 *     y <- y + lambda (b_i - <a_i, y>) / ||a_i||^2 a_i     (rows with ||a_i|| = 0 skipped);
 * the next iterate is the weighted sum x_{k+1} = sum_t w_t y_t.  The update uses the
 * current y, with the residual b_i - <a_i, y> (the standard Kaczmarz sign; the printed
 * update has the other sign and x_k in place of y).  Everything in binary64.
 * weights == NULL: w_t = 1/M.  order == NULL: rows in their natural order.  ||a_i|| is
 * the norm of the row as a vector of R^n: entries of a row that share a column (a curved
 * path re-entering a voxel) add into that one component, so the squared norm is the sum
 * over the row's distinct columns of (sum of their values)^2; the dot product and the
 * update, taken entry by entry, act on that same vector.  With lambda = 1 a row update
 * then lands exactly on the row's hyperplane. */
void or_sap(int64_t m, int32_t n, const int64_t *row_ptr, const int32_t *cols, const double *vals,
            const double *b, int32_t M, double lambda, const double *weights, const int64_t *order,
            double *x, int32_t n_iter)
{
    const size_t nn = (size_t)(n > 0 ? n : 1);
    double *y = (double *)malloc(nn * sizeof(double));
    double *acc = (double *)malloc(nn * sizeof(double));
    double *comp = (double *)malloc(nn * sizeof(double));    /* a_i as a vector of R^n */
    int64_t *mark = (int64_t *)malloc(nn * sizeof(int64_t)); /* row whose component comp[j] holds */
    for (size_t j = 0; j < nn; ++j) mark[j] = -1;
    int64_t stamp = 0;
    for (int32_t it = 0; it < n_iter; ++it) {
        for (int32_t j = 0; j < n; ++j) acc[j] = 0.0;
        for (int32_t t = 0; t < M; ++t) {
            const int64_t s0 = (int64_t)t * m / M, s1 = (int64_t)(t + 1) * m / M;
            for (int32_t j = 0; j < n; ++j) y[j] = x[j];
            for (int64_t s = s0; s < s1; ++s) {
                const int64_t i = order ? order[s] : s;
                double dot = 0.0, nrm = 0.0;
                /* the components of a_i: the values of every column, summed */
                const int64_t tag = 2 * (stamp++);
                for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                    if (mark[cols[e]] != tag) {
                        mark[cols[e]] = tag;
                        comp[cols[e]] = 0.0;
                    }
                    comp[cols[e]] += vals[e];
                    dot += vals[e] * y[cols[e]];
                }
                /* ||a_i||^2: each distinct column once */
                for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                    if (mark[cols[e]] == tag) {
                        nrm += comp[cols[e]] * comp[cols[e]];
                        mark[cols[e]] = tag + 1;
                    }
                }
                if (nrm == 0.0) continue;
                const double alpha = lambda * (b[i] - dot) / nrm;
                for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) y[cols[e]] += alpha * vals[e];
            }
            const double w = weights ? weights[t] : 1.0 / (double)M;
            for (int32_t j = 0; j < n; ++j) acc[j] += w * y[j];
        }
        for (int32_t j = 0; j < n; ++j) x[j] = acc[j];
    }
    free(comp);
    free(mark);
    free(y);
    free(acc);
}
