/*
 * pct.h -- C ABI of the MI355X proton-CT data simulator hot path.
 *
 * The library produces the three parts of the linear system A x = b that the
 * simulator of Witt et al. (arXiv 2108.12369, Sec. II) writes for reconstruction:
 *   x  the true relative stopping power (RSP) of every voxel of a phantom (Sec. II-A),
 *   A  one sparse row per proton holding the length of its path in every voxel it
 *      crosses, in CSR form (Sec. II-C),
 *   b  the water-equivalent path length of every proton, the inner product of its row
 *      with x, optionally with noise (Sec. II-C).
 *
 * Conventions for every entry point:
 *   - units are mm, projection angles in degrees, scattering widths in radians;
 *   - pointers named *_dev are device memory owned by the caller; every other pointer is
 *     host memory owned by the caller and only read during the call;
 *   - `stream` is a hipStream_t (NULL: the default stream); every call only enqueues
 *     work on it, never synchronises it (except pct_device_status) and never allocates
 *     device memory;
 *   - descriptors are validated on the host before anything is enqueued; on failure
 *     nothing is written and the status says why;
 *   - calls on different streams with disjoint workspaces and outputs may overlap.
 */
#ifndef PCT_H
#define PCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
typedef int32_t pct_status;
#define PCT_OK          0
#define PCT_EINVAL     (-1)  /* a descriptor field is out of its documented range      */
#define PCT_ERANGE     (-2)  /* a size overflows the index types (>= 2^31 voxels)       */
#define PCT_ECAPACITY  (-3)  /* (device) a row did not fit in nnz_capacity: not stored  */
#define PCT_EWORKSPACE (-4)  /* workspace missing or smaller than pct_workspace_bytes   */
#define PCT_EHIP       (-5)  /* a HIP runtime call failed                               */
#define PCT_EINTERNAL  (-6)  /* (device) emitted entries differ from the counted ones   */
#define PCT_EIO        (-7)  /* a file could not be opened or written                   */
#define PCT_ESCRATCH   (-8)  /* more jobs or rows than pct_wepl_static's static scratch */

/* ------------------------------------------------------------------ enumerations */
#define PCT_ELLIPSE    0   /* ellipse in the x-y plane; in 3D an elliptic cylinder along z */
#define PCT_ELLIPSOID  1   /* ellipsoid (3D); in 2D the same as PCT_ELLIPSE                 */

#define PCT_CORNER_AVG 0   /* pixel value = mean RSP at its 4 (8) corners (Sec. II-A)       */
#define PCT_CENTER     1   /* pixel value = RSP at its center point (Sec. II-A)             */
#define PCT_AREA_AVG   2   /* pixel value = sum of region RSP x area (volume) fraction      */
                           /* (Sec. II-A), the fractions from area_samples^dim midpoints    */

#define PCT_STRAIGHT   0   /* straight-line proton paths (Sec. II-B)                        */
#define PCT_HERMITE    1   /* cubic spline between entry and exit, straight outside (II-B)  */

#define PCT_F32        0   /* stored lengths: binary32                                      */
#define PCT_F16        1   /* stored lengths: binary16, round to nearest even               */

#define PCT_MIXED      0   /* FP64 geometry and traversal order, FP32 lengths, FP64 WEPL sum */
#define PCT_PLAIN_F32  1   /* FP32 everywhere (comparison form)                              */

#define PCT_SCATTER_FIXED    0  /* exit pair widths and correlation as given in the beam     */
#define PCT_SCATTER_HIGHLAND 1  /* per proton from Highland's formula (Sec. II-B), see below */

#define PCT_MAX_REGIONS 16

/* One region of a non-homogeneous ellipse object (Sec. II-A).  A point p belongs to
 * the region when sum((u / semi)^2) <= 1, u = p - center turned by -angle_deg about z
 * (u_x = c d_x + s d_y, u_y = -s d_x + c d_y with c, s the cosine and sine of the angle,
 * d = p - center), over x, y (and z for an ellipsoid in 3D).  Regions are painted in
 * array order: a later region replaces the RSP of an earlier one.  Region 0 is the outer
 * boundary used for the proton entry and exit. */
typedef struct {
    int32_t shape;      /* PCT_ELLIPSE | PCT_ELLIPSOID */
    float rsp;          /* relative stopping power, >= 0 */
    double center[3];   /* mm */
    double semi[3];     /* semi-axes, mm, > 0 (z ignored unless ellipsoid in 3D) */
    double angle_deg;   /* rotation of the semi-axes in the x-y plane, counterclockwise */
} pct_region;

/* Voxel grid and phantom (Sec. II-A).  Voxel (ix, iy, iz) covers
 * [origin + i*h, origin + (i+1)*h) per axis and is column ix + n[0]*(iy + n[1]*iz) of A
 * and element of x.  In 2D n[2] and h[2] are ignored. */
typedef struct {
    int32_t dim;                 /* 2 or 3 */
    int32_t n[3];                /* voxels per axis, >= 1; product < 2^31 */
    double h[3];                 /* voxel size, mm, > 0 */
    double origin[3];            /* lower corner of the grid box, mm */
    int32_t n_regions;           /* 1..PCT_MAX_REGIONS */
    int32_t voxelize;            /* PCT_CORNER_AVG | PCT_CENTER | PCT_AREA_AVG */
    const pct_region *regions;   /* host array of n_regions */
    int32_t area_samples;        /* PCT_AREA_AVG: midpoints per axis, 1..64 (0: 8) */
} pct_phantom;

/* Parallel beam and proton source (Sec. II-B).  Proton g (0 <= g < n_protons) belongs
 * to projection angle k with floor(k P/K) <= g < floor((k+1) P/K), i.e. angle-major
 * order, angle k at angle0_deg + k*dangle_deg.  Its entry offset is uniform on
 * [t_range) along t (and [v_range) along v in 3D).  Every random number of proton g is
 * drawn from Philox4x32-10 keyed by `seed` with a counter built from g, so any row can
 * be produced alone.  A call covers the rows [row_begin, row_begin + row_count). */
typedef struct {
    uint64_t seed;
    int32_t n_angles;            /* K >= 1 */
    int32_t path;                /* PCT_STRAIGHT | PCT_HERMITE */
    double angle0_deg;
    double dangle_deg;
    int64_t n_protons;           /* P >= 0 */
    int64_t row_begin;           /* 0 <= row_begin, row_begin + row_count <= P */
    int64_t row_count;
    double t_range[2];           /* mm, t_range[0] <= t_range[1] */
    double v_range[2];           /* mm (3D) */
    double sigma_in_rad;         /* entry angular spread per plane, 0..0.1 */
    double sigma_out_rad;        /* exit angular spread per plane, 0..0.1 */
    double sigma_lat_mm;         /* exit lateral displacement per plane, >= 0 */
    double rho;                  /* correlation of (lateral, angle) at exit, |rho| <= 1 */
    double step_mm;              /* spline sample spacing, > 0 (Hermite only); at most
                                    2^22 samples per outer-boundary diameter x 6, else
                                    PCT_ERANGE */
    double noise_rel;            /* relative WEPL noise sigma, >= 0 (0: noiseless) */
    /* Multiple-scattering model of the exit pair (Hermite paths; Sec. II-B).
     * PCT_SCATTER_FIXED: sigma_out_rad, sigma_lat_mm and rho as given above.
     * PCT_SCATTER_HIGHLAND: with x the length of the straight entry line inside the outer
     * boundary (mm), Highland's width with the Particle Data Group constants
     *   theta0 = 13.6 MeV / (beta c p) * sqrt(x / X0) * (1 + 0.038 ln(x / (X0 beta^2)))
     * (taken as 0 where the bracket is negative), for a proton of the constant kinetic
     * energy energy_mev, and the exit pair of a uniform slab of thickness x:
     *   sigma_out = theta0, sigma_lat = theta0 x / sqrt(3), rho = sqrt(3) / 2;
     * sigma_out_rad, sigma_lat_mm and rho are then ignored (but must still be valid). */
    int32_t scatter;             /* PCT_SCATTER_FIXED | PCT_SCATTER_HIGHLAND */
    double energy_mev;           /* Highland: kinetic energy, 1..10000 MeV */
    double x0_mm;                /* Highland: radiation length of the medium, > 0 (water 360.8) */
} pct_beam;

/* One simulation job: one phantom, one beam, one range of rows. */
typedef struct {
    const pct_phantom *phantom;  /* host */
    const pct_beam *beam;        /* host */
    const float *x_dev;          /* true RSP vector from pct_phantom_build (for b) */
    int64_t *row_ptr_dev;        /* row_count + 1 entries, row_ptr[0] = 0 (job-relative) */
    int32_t *cols_dev;           /* nnz_capacity entries */
    void *vals_dev;              /* nnz_capacity entries of val_dtype */
    int64_t nnz_capacity;        /* >= 0 */
    float *b_dev;                /* row_count entries; may be NULL in pct_emit_csr */
    int32_t val_dtype;           /* PCT_F32 | PCT_F16 */
    int32_t precision;           /* PCT_MIXED | PCT_PLAIN_F32; equal for all jobs of a call */
    double chord_mm;             /* 0: every stored value is the path length in its voxel;
                                    > 0: every stored value is chord_mm, the constant chord
                                    length of the paper's examples (Sec. II-C), while b stays
                                    the WEPL of the true path lengths */
} pct_job;

/* Human-readable name of a status code (static string). */
const char *pct_status_string(pct_status status);

/* Library version, major*10000 + minor*100 + patch. */
int32_t pct_version(void);

/* Voxelise the phantom into x_dev (n[0]*n[1]*(dim==3 ? n[2] : 1) floats) with a
 * pixel-value rule of Sec. II-A: the RSP at the voxel center; the mean of the RSP at its
 * 4 (2D) or 8 (3D) corners; or the weighted-area average, the mean RSP over the
 * S^dim points ((i + 1/2) / S of the voxel per axis, S = area_samples), which is
 * sum_r RSP_r x (fraction of the points in region r) and tends to the exact area
 * fractions as S grows.  The point tests are done in binary64 and the value is rounded
 * once to binary32. */
pct_status pct_phantom_build(const pct_phantom *phantom, float *x_dev, void *stream);

/* Bytes of device workspace that pct_count_rows / pct_emit_csr / pct_wepl need for
 * these jobs (0 if a descriptor is invalid).  The workspace holds the job table, the
 * per-row counts, the scan partials, a description of every row's path, a status word
 * and, for each 3D job, and each 2D job with PCT_STRAIGHT paths, with n[0] <= 1024 and
 * n[1], n[2] <= 2048, a copy of x in bricks of 8 x 8 x 1 voxels that pct_emit_csr and
 * pct_wepl refill from x_dev on every call
 * (the gathers of b read it: a cache line then covers a patch of a plane instead of a
 * stretch of one grid row).  pct_emit_csr reads the path descriptions that
 * pct_count_rows wrote: pass it the same workspace and the same jobs (output pointers
 * may differ). */
size_t pct_workspace_bytes(int32_t n_jobs, const pct_job *jobs);

/* Count pass: for every row of every job the number of CSR entries the path produces
 * (Sec. II-C), then an exclusive scan into row_ptr_dev of each job, and
 * nnz_total_dev[j] = row_ptr_j[row_count_j] (device int64 array of n_jobs).  Clears the
 * device status word.  The caller reads nnz_total to size cols / vals. */
pct_status pct_count_rows(int32_t n_jobs, const pct_job *jobs, void *ws_dev, size_t ws_bytes,
                          int64_t *nnz_total_dev, void *stream);

/* Emit pass (after pct_count_rows on the same jobs and workspace): walk every path and
 * write its entries at
 * [row_ptr[r], row_ptr[r+1]) of cols_dev (voxel column) and vals_dev (path length in
 * that voxel, mm), in path order from entry to exit, and, if b_dev is not NULL, its
 * WEPL b[r] = sum of length * x[col] (with noise when noise_rel > 0).  row_ptr_dev must
 * hold the result of pct_count_rows for the same jobs.  A row that would end beyond
 * nnz_capacity is not written and sets PCT_ECAPACITY in the device status word. */
pct_status pct_emit_csr(int32_t n_jobs, const pct_job *jobs, void *ws_dev, size_t ws_bytes,
                        void *stream);

/* WEPL only: b_dev[r] for every row, bit-identical to the b that pct_emit_csr writes,
 * without storing A (row_ptr, cols, vals are not read or written).  It runs its own
 * count pass and, like pct_count_rows, clears the device status word first. */
pct_status pct_wepl(int32_t n_jobs, const pct_job *jobs, void *ws_dev, size_t ws_bytes,
                    void *stream);

/* pct_wepl without a caller workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same kernels and the same b, bit for bit, with the workspace taken from a static
 * device array of 64 MiB per GPU (resolved on the first call on each device and held
 * until the process ends).  The call allocates nothing, on the device or on the host.
 * Its gathers of b read x_dev itself (no bricked copy of x).  Limits: at most 64 jobs,
 * and no more rows than the workspace of the jobs without the bricked copies
 * (pct_workspace_bytes less those) fits in 64 MiB (about 180,000 rows); beyond either
 * nothing is enqueued and PCT_ESCRATCH is returned.  status_dev (device int32, nullable) receives the device status word after
 * the call (PCT_OK, or PCT_EINTERNAL).  Every call on one GPU uses that GPU's one array:
 * calls that overlap on one GPU (other streams, other host threads) race and must be
 * ordered by the caller. */
pct_status pct_wepl_static(int32_t n_jobs, const pct_job *jobs, int32_t *status_dev, void *stream);

/* Synchronise the stream and return the device status word of the workspace:
 * PCT_OK, PCT_ECAPACITY or PCT_EINTERNAL (first error since the last count pass). */
pct_status pct_device_status(const void *ws_dev, void *stream);

/* ------------------------------------------------------------- batched launches
 * Many jobs (phantoms, grids, beams of uneven size) share one launch of every kernel
 * of a pass.  How the emit pass spreads them over the GPU is set by a process-wide
 * launch configuration (read when a call is enqueued; set it between calls, not
 * during them).  It does not change any output: every row is computed the same way
 * whatever the order or grouping of the rows. */
#define PCT_ORDER_GIVEN 0   /* emit tiles in the order of the job array                 */
#define PCT_ORDER_LPT   1   /* jobs with the costliest rows first (longest processing   */
                            /* time first), so that cheap tiles fill the tail           */

typedef struct {
    int32_t rows_per_wave;  /* 16, 32 or 64: consecutive rows walked by one wavefront    */
    int32_t order;          /* PCT_ORDER_GIVEN | PCT_ORDER_LPT (within each grid          */
                            /* dimension: the emit takes the 2D jobs, then the 3D jobs)  */
    int32_t blocks_per_cu;  /* 0: one block of 4 wavefronts per emit tile, a grid over   */
                            /* every tile; 1-8: a persistent grid of this many blocks    */
                            /* per compute unit, each block taking the next tile of its  */
                            /* grid dimension from a counter in the workspace until none */
                            /* is left (the counters are reset by a kernel of the call,  */
                            /* so a graph replay needs no memset)                         */
} pct_launch_config;

/* Set (NULL: reset to the default {64, PCT_ORDER_LPT, 0}) or read the configuration. */
pct_status pct_set_launch_config(const pct_launch_config *cfg);
pct_status pct_get_launch_config(pct_launch_config *cfg);

/* Autotuner: runs pct_count_rows once and then pct_emit_csr with every candidate
 * configuration (rows_per_wave 16/32/64 x both orders x blocks_per_cu 0/4), timing each
 * emit with HIP events on `stream` (this call synchronises it), keeps the fastest as the
 * process-wide configuration and returns it in *best.  The jobs must be ready for
 * pct_emit_csr (outputs sized from an earlier count); their outputs hold a complete,
 * valid result afterwards.
 * Results are cached per process, keyed by the GPU architecture, the HIP runtime version
 * and the shape of the batch (per job: grid dimension and sizes, path, precision, value
 * type and the row count to within a factor of two).  A call whose key is cached takes
 * that configuration without timing (it still runs the count and the final emit).  With
 * the environment variable PCT_TUNE_CACHE naming a file, the cache is read from it at the
 * first call and every new result is appended to it (one line per key). */
pct_status pct_autotune(int32_t n_jobs, const pct_job *jobs, void *ws_dev, size_t ws_bytes,
                        int64_t *nnz_total_dev, void *stream, pct_launch_config *best);
/* The cached configuration for these jobs on the current device, if any: *found = 1 and
 * *cfg set, else *found = 0.  Only host work. */
pct_status pct_autotune_cached(int32_t n_jobs, const pct_job *jobs, pct_launch_config *cfg, int32_t *found);
/* Forget every cached configuration of this process (the file is not touched). */
pct_status pct_autotune_cache_clear(void);

/* A whole batch recorded once into a HIP graph and replayed with one call: optionally
 * the voxelisation of every job's phantom into its x_dev (build_x != 0; jobs that share
 * an x_dev build it once), then pct_count_rows and pct_emit_csr for all jobs.  The
 * descriptors and the launch configuration are captured at creation: a replay writes
 * the same outputs as the eager calls would.  The graph owns no device memory; the
 * caller's buffers and workspace must outlive it.  Creation runs the host validation of
 * the calls and returns its status; nothing is enqueued on any caller stream. */
typedef struct pct_graph_s *pct_graph;
pct_status pct_graph_create(int32_t n_jobs, const pct_job *jobs, int32_t build_x, void *ws_dev,
                            size_t ws_bytes, int64_t *nnz_total_dev, pct_graph *graph);
/* The same for n_sets job sets run one after another, for instance the row chunks of one
 * workload that reuse one set of output buffers: jobs holds the sets back to back
 * (set_sizes[k] jobs each), and set k counts (into nnz_total_dev[off_k ...], off_k = the
 * jobs of the sets before it) and emits after set k-1 has emitted, with one workspace
 * large enough for every set.  The phantom builds (build_x) run once, beside the first
 * set's count.  A set whose rows need more entries than a job's nnz_capacity sets
 * PCT_ECAPACITY in the device status word (pct_device_status after the replay), so the
 * capacities may come from a bound rather than from a count of every set. */
pct_status pct_graph_create_sets(int32_t n_sets, const int32_t *set_sizes, const pct_job *jobs, int32_t build_x,
                                 void *ws_dev, size_t ws_bytes, int64_t *nnz_total_dev, pct_graph *graph);
pct_status pct_graph_launch(pct_graph graph, void *stream);
pct_status pct_graph_destroy(pct_graph graph);

/* ------------------------------------------------------- reconstruction (Sec. II-D)
 * String-averaging projections (SAP) on A x = b, the reconstruction the paper runs on
 * the system the simulator writes.  One iteration from the iterate x_k: the rows, taken
 * in the order `order_dev` (NULL: 0 .. m-1), are split into M strings of consecutive
 * positions, string t covering positions [floor(t m / M), floor((t+1) m / M)); every
 * string starts from y = x_k and applies, row after row,
 *     y <- y + lambda (b_i - <a_i, y>) / ||a_i||^2 a_i     (rows with ||a_i|| = 0 skipped),
 * and x_{k+1} = sum_t w_t y_t.  This is the usual Kaczmarz sign with the current y in
 * the residual; the printed update uses x_k and the opposite sign.  a_i is the row as a
 * vector of R^n: entries of a row that share a column add into that one component (in
 * ||a_i||^2 as in <a_i, y> and the update), so the result does not depend on whether the
 * caller stores a column once or as several entries.
 * Arithmetic: y in binary32, <a_i, y> and ||a_i||^2 accumulated in binary64, the
 * weighted sum over strings in binary64 in string order (deterministic). */
typedef struct {
    int64_t n_rows;               /* m >= 0 */
    int32_t n_cols;               /* 1 <= n < 2^29, the length of x */
    int32_t val_dtype;            /* PCT_F32 | PCT_F16 */
    int64_t nnz;                  /* length of cols_dev and vals_dev */
    const int64_t *row_ptr_dev;   /* m + 1 entries, non-decreasing, within [0, nnz] */
    const int32_t *cols_dev;      /* each in [0, n) */
    const void *vals_dev;         /* val_dtype */
    const float *b_dev;           /* m entries */
} pct_csr;

typedef struct {
    int32_t n_strings;            /* M >= 1 */
    float relax;                  /* lambda, 0 < lambda < 2 */
    const double *weights;        /* host, M entries >= 0 summing to 1 within 1e-9, copied
                                     by pct_sap_prepare; NULL: 1/M */
    const int64_t *order_dev;     /* device, m row indices in [0, m); NULL: natural order */
} pct_sap;

/* Bytes of device workspace for pct_sap_prepare / pct_sap_iterate (0 if a descriptor is
 * invalid): a status word, one coefficient per row and M x n binary32 string iterates. */
size_t pct_sap_workspace_bytes(const pct_csr *A, const pct_sap *p);

/* Per-row coefficients lambda / ||a_i||^2 and the weights into the workspace.  Checks
 * row_ptr, the columns and the order on the device: a row with an out-of-range column or
 * bounds, or an out-of-range order entry, is skipped by pct_sap_iterate and sets
 * PCT_EINVAL in the device status word (read it with pct_device_status on this
 * workspace).  Clears the status word first. */
pct_status pct_sap_prepare(const pct_csr *A, const pct_sap *p, void *ws_dev, size_t ws_bytes, void *stream);

/* n_iter >= 0 iterations from x_dev (n floats, read and overwritten with the result),
 * after pct_sap_prepare on the same A, parameters and workspace.  Each string is one
 * workgroup.  Its iterate lives in LDS when n binary32 fit a workgroup's LDS (one
 * wavefront), else in the workspace (one wavefront loads the rows, one projects them).
 * A row's entries are all applied, also where a column repeats in the row; ||a_i|| is
 * then the norm of their sum per column. */
pct_status pct_sap_iterate(const pct_csr *A, const pct_sap *p, float *x_dev, int32_t n_iter, void *ws_dev,
                           size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------- file output
 * The system written to disk in a form that reads straight into CSR (Sec. II-C): one
 * binary file, little-endian, a 128-byte header then 64-byte-aligned sections.
 *   offset  0  char    magic[8]      "PCTCSR01"
 *           8  int64   n_rows        m
 *          16  int64   n_cols        n
 *          24  int64   nnz           row_ptr[m]
 *          32  int32   val_dtype     PCT_F32 | PCT_F16
 *          36  int32   version       1
 *          40  int64   off_row_ptr   m + 1 int64
 *          48  int64   off_cols      nnz int32
 *          56  int64   off_vals      nnz values of val_dtype
 *          64  int64   off_b         m float32 (0: not written)
 *          72  int64   off_x         n float32, the true solution (0: not written)
 *          80  zero up to 128
 * Gaps between sections are zero. */
#define PCT_CSR_MAGIC "PCTCSR01"

/* Write A (row_ptr, cols, vals), b if A->b_dev is not NULL and x if x_dev is not NULL to
 * `path` (created or truncated).  Waits for the work already enqueued on `stream`, then
 * streams the device arrays through two pinned host buffers of 64 MiB (allocated and
 * freed by the call), copying the next chunk while the current one is written.  Returns
 * when the file is complete (this call synchronises `stream`).  nnz is read from
 * row_ptr[m] and must not exceed A->nnz. */
pct_status pct_csr_write(const char *path, const pct_csr *A, const float *x_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PCT_H */
