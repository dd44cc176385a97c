/* Drives every entry point of the oracle on small inputs, so that a build with the
 * address and undefined-behaviour sanitizers (tests/test_oracle_sanitize.py) checks its
 * memory accesses, arithmetic and frees.  Exit status 0 when everything ran; the
 * sanitizers abort the run on the first error they find.
 *
 * The oracle is one translation unit of plain C; it is included here so that its
 * structs and functions need no separate header. */
#include "pct_oracle.c"

#include <stdio.h>

static or_region region(int32_t shape, double cx, double cy, double cz, double a, double b, double c, float rsp,
                        double angle)
{
    or_region r;
    memset(&r, 0, sizeof r);
    r.shape = shape;
    r.center[0] = cx;
    r.center[1] = cy;
    r.center[2] = cz;
    r.semi[0] = a;
    r.semi[1] = b;
    r.semi[2] = c;
    r.rsp = rsp;
    r.angle_deg = angle;
    return r;
}

static or_phantom phantom(int dim, int nx, int ny, int nz, double h, const or_region *regs, int nreg, int vox)
{
    or_phantom ph;
    memset(&ph, 0, sizeof ph);
    ph.dim = dim;
    ph.n[0] = nx;
    ph.n[1] = ny;
    ph.n[2] = nz;
    for (int d = 0; d < 3; ++d) ph.h[d] = h;
    ph.origin[0] = -nx * h / 2;
    ph.origin[1] = -ny * h / 2;
    ph.origin[2] = -nz * h / 2;
    ph.n_regions = nreg;
    ph.regions = regs;
    ph.voxelize = vox;
    ph.area_samples = 3;
    return ph;
}

static or_beam beam(int path, int64_t P, int K, double span, int highland, double noise)
{
    or_beam bm;
    memset(&bm, 0, sizeof bm);
    bm.seed = 12369u + (uint64_t)P;
    bm.n_angles = K;
    bm.angle0_deg = 3.0;
    bm.dangle_deg = 360.0 / K;
    bm.n_protons = P;
    bm.t_range[0] = -span;
    bm.t_range[1] = span;
    bm.v_range[0] = -span / 2;
    bm.v_range[1] = span / 2;
    bm.path = path;
    bm.sigma_in = 0.02;
    bm.sigma_out = 0.02;
    bm.sigma_lat = 1.0;
    bm.rho = 0.3;
    bm.step = 0.7;
    bm.noise_rel = noise;
    bm.scatter = highland;
    bm.energy_mev = 200.0;
    bm.x0_mm = 360.8;
    return bm;
}

/* One workload: phantom build, every row traced, the result copied and freed; then
 * SAP on the system.  Returns the number of entries. */
static int64_t run(const or_phantom *ph, const or_beam *bm)
{
    const int64_t nvox = (int64_t)ph->n[0] * ph->n[1] * (ph->dim == 3 ? ph->n[2] : 1);
    float *x = (float *)malloc((size_t)nvox * sizeof(float));
    or_phantom_build(ph, x);
    int64_t *rows = (int64_t *)malloc((size_t)bm->n_protons * sizeof(int64_t));
    for (int64_t r = 0; r < bm->n_protons; ++r) rows[r] = r;
    or_result *res = or_run(ph, bm, x, rows, bm->n_protons);
    const int64_t nnz = or_result_nnz(res);
    int64_t *row_ptr = (int64_t *)malloc((size_t)(bm->n_protons + 1) * sizeof(int64_t));
    int32_t *cols = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    double *vals = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    double *b = (double *)malloc((size_t)bm->n_protons * sizeof(double));
    double *bc = (double *)malloc((size_t)bm->n_protons * sizeof(double));
    double *mg = (double *)malloc((size_t)bm->n_protons * sizeof(double));
    or_path *paths = (or_path *)malloc((size_t)bm->n_protons * sizeof(or_path));
    or_result_copy(res, row_ptr, cols, vals, b, bc, mg, paths);
    or_result_free(res);

    /* SAP: natural order and uniform weights; a permuted order, weights and more
     * strings than rows */
    double *xs = (double *)calloc((size_t)nvox, sizeof(double));
    or_sap(bm->n_protons, (int32_t)nvox, row_ptr, cols, vals, b, 3, 0.5, NULL, NULL, xs, 2);
    const int32_t M = (int32_t)bm->n_protons + 5;
    double *w = (double *)malloc((size_t)M * sizeof(double));
    for (int32_t t = 0; t < M; ++t) w[t] = 1.0 / M;
    for (int64_t r = 0; r < bm->n_protons; ++r) rows[r] = bm->n_protons - 1 - r;
    or_sap(bm->n_protons, (int32_t)nvox, row_ptr, cols, vals, b, M, 1.2, w, rows, xs, 1);

    free(w);
    free(xs);
    free(paths);
    free(mg);
    free(bc);
    free(b);
    free(vals);
    free(cols);
    free(row_ptr);
    free(rows);
    free(x);
    return nnz;
}

int main(void)
{
    int64_t total = 0;
    /* 2D: outer ellipse, a turned inner one and an air pocket; three pixel rules */
    or_region r2[3] = {region(OR_ELLIPSE, 0, 0, 0, 18, 14, 0, 1.6f, 0.0),
                       region(OR_ELLIPSE, 2, 1, 0, 9, 5, 0, 1.04f, 30.0),
                       region(OR_ELLIPSE, -4, 3, 0, 2, 1.5, 0, 0.0f, -20.0)};
    for (int vox = 0; vox < 3; ++vox) {
        or_phantom ph = phantom(2, 24, 20, 1, 1.7, r2, 3, vox);
        or_beam s = beam(OR_STRAIGHT, 360, 36, 25.0, 0, 0.0);
        or_beam c = beam(OR_HERMITE, 300, 30, 25.0, 0, 0.01);
        or_beam h = beam(OR_HERMITE, 300, 30, 25.0, 1, 0.01);
        total += run(&ph, &s) + run(&ph, &c) + run(&ph, &h);
    }
    /* 3D: an ellipsoid with an elliptic cylinder inside; straight and curved */
    or_region r3[2] = {region(OR_ELLIPSOID, 0, 0, 0, 14, 11, 9, 1.0f, 0.0),
                       region(OR_ELLIPSE, 1, -1, 0, 5, 3, 0, 1.6f, 45.0)};
    for (int vox = 0; vox < 3; ++vox) {
        or_phantom ph = phantom(3, 14, 12, 10, 2.1, r3, 2, vox);
        or_beam s = beam(OR_STRAIGHT, 120, 12, 16.0, 0, 0.0);
        or_beam c = beam(OR_HERMITE, 120, 12, 16.0, 1, 0.02);
        total += run(&ph, &s) + run(&ph, &c);
    }
    /* a 1 x 1 grid, and protons that miss the grid */
    or_region r1[1] = {region(OR_ELLIPSE, 0, 0, 0, 0.4, 0.3, 0, 1.0f, 0.0)};
    or_phantom tiny = phantom(2, 1, 1, 1, 1.0, r1, 1, OR_CORNER_AVG);
    or_beam far = beam(OR_STRAIGHT, 40, 4, 5.0, 0, 0.0);
    or_beam cur = beam(OR_HERMITE, 40, 4, 0.4, 0, 0.0);
    total += run(&tiny, &far) + run(&tiny, &cur);
    /* arbitrary segments through the 2D grid, and Highland's formula */
    or_phantom ph = phantom(2, 24, 20, 1, 1.7, r2, 3, OR_CENTER);
    const double A[6] = {-30, -1, 0, 3, -30, 0}, D[6] = {1, 0.1, 0, -0.05, 1, 0};
    const double lo[2] = {0, 0}, hi[2] = {60, 60};
    or_result *seg = or_trace_segments(&ph, 2, A, D, lo, hi);
    total += or_result_nnz(seg);
    or_result_free(seg);
    const double th = or_highland(200.0, 360.8, 150.0) + or_highland(100.0, 360.8, 0.0);
    printf("entries %lld, highland %.6f\n", (long long)total, th);
    return total > 0 && th > 0 ? 0 : 1;
}
