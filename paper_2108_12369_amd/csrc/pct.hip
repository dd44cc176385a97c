// pct.hip -- kernels and C ABI of the proton-CT hot path (see include/pct.h).
//
// Pipeline of one batch of jobs (one stream, no host synchronisation):
//   pct_phantom_build : k_phantom          one thread per voxel -> x (FP32)
//   pct_count_rows    : k_put_jobs          job table into the workspace (kernel args)
//                       k_count             one lane per row -> per-row entry counts,
//                                           per-tile sums
//                       k_scan_tiles        exclusive scan of the tile sums, job totals
//                       k_row_ptr           per-tile scan of the counts -> row_ptr
//   pct_emit_csr      : k_put_jobs, k_emit  one lane per row -> cols, vals, b
//   pct_wepl          : k_put_jobs, k_emit  (no A stores) -> b
#include "../../include/pct.h"
#include "pct_device.h"
#include "pct_wave.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <unordered_map>
#include <vector>

namespace pct {

constexpr int TILE = 256;            // rows per tile (= threads per block of k_count/k_emit)
constexpr int SCAN_THREADS = 1024, SCAN_ITEMS = 4;

// Workspace layout (bytes): [0,256) header | job table | tile sums | tile offsets | counts |
// per-row path descriptions
struct WsHeader {
    int32_t status;
    int32_t pad[31];
    unsigned long long qnext[2];   // next emit tile of the persistent grid (2D, 3D): own cache line
    unsigned long long pad2[14];
};
static_assert(sizeof(WsHeader) == 256, "the header is 256 bytes");

static inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t jobs_off, order_off, sums_off, offs_off, flags_off, counts_off, rows_off, bricks_off, total;
    int64_t total_tiles, total_rows;
};

// per-row path descriptions (the larger of the two precisions)
constexpr size_t ROWW_BYTES = rv_bytes<double>() > rv_bytes<float>() ? rv_bytes<double>() : rv_bytes<float>();
static_assert(TILE == RV_TILE, "descriptions are stored per count tile");

// Bricked copy of x (8 x 8 x 1 voxels per brick) for a 3D job, or a 2D job with straight
// paths, whose voxel coordinates pack into 32 bits (x < 1024, y < 2048, z < 2048) and
// whose padded grid stays below 2^31 voxels: its element count, else 0.
static int64_t brick_elems(const pct_phantom &ph, const pct_beam &bm) {
    // 2D: only for straight paths (their walk is cheap, so the fewer cache lines per
    // gather pay for the unpacking; curved 2D rows were 1-6% slower with it)
    if (ph.dim == 2 ? bm.path != PCT_STRAIGHT : ph.dim != 3) return 0;
    if (ph.n[0] > 1024 || ph.n[1] > 2048 || (ph.dim == 3 && ph.n[2] > 2048)) return 0;
    const int64_t nz = ph.dim == 3 ? ph.n[2] : 1;
    const int64_t e = (int64_t)((ph.n[0] + 7) / 8) * 8 * (int64_t)((ph.n[1] + 7) / 8) * 8 * nz;
    return e < ((int64_t)1 << 31) ? e : 0;
}

// Workspace layout; brick_bytes: per job, the bytes of its bricked copy of x (null: none).
static Layout layout_of(int32_t n_jobs, const int64_t *row_counts, const size_t *brick_bytes = nullptr) {
    Layout L{};
    int64_t tiles = 0, rows = 0;
    for (int j = 0; j < n_jobs; ++j) {
        tiles += (row_counts[j] + TILE - 1) / TILE;
        rows += row_counts[j];
    }
    L.total_tiles = tiles;
    L.total_rows = rows;
    L.jobs_off = align256(sizeof(WsHeader));
    L.order_off = align256(L.jobs_off + (size_t)n_jobs * sizeof(JobDev));
    L.sums_off = align256(L.order_off + 2 * (size_t)n_jobs * sizeof(int32_t));   // emit order, count order
    L.offs_off = align256(L.sums_off + (size_t)(tiles + 1) * sizeof(int64_t));
    L.flags_off = align256(L.offs_off + (size_t)(tiles + 1) * sizeof(int64_t));
    L.counts_off = align256(L.flags_off + (size_t)(tiles + 1) * sizeof(int32_t));
    L.rows_off = align256(L.counts_off + (size_t)rows * sizeof(int32_t));
    L.bricks_off = align256(L.rows_off + (size_t)tiles * RV_TILE * ROWW_BYTES);   // whole tiles of descriptions
    size_t bricks = 0;
    if (brick_bytes)
        for (int j = 0; j < n_jobs; ++j) bricks += align256(brick_bytes[j]);
    L.total = L.bricks_off + bricks;
    return L;
}

// ------------------------------------------------------------------------ kernels

constexpr int JOBS_PER_PACK = 3800 / (int)sizeof(JobDev);
struct JobPack {
    int32_t count;
    int32_t first;
    JobDev jobs[JOBS_PER_PACK];
};

// Kernel arguments are copied at launch (and into a graph node at capture), so the
// job table reaches the device without a host buffer that has to outlive the call.
// Bricked copy of x for the b gathers of a job (blockIdx.y: the job; jobs without one
// return at once).  Brick (bx, by, z) holds the voxels x in [8 bx, 8 bx + 8) and y in
// [8 by, 8 by + 8) of plane z, x fastest; the bricks follow x, then y, then z, so that a
// 128-byte line covers an 8 x 4 patch of a plane.  Voxels past the grid are 0; no gather
// index reaches them.  The copy has fewer than 2^31 elements (brick_elems).
constexpr int BRICK_BLOCKS = 512;
__global__ void __launch_bounds__(256) k_brick(const JobDev *__restrict__ jobs, int32_t job0) {
    const JobDev &J = jobs[job0 + (int32_t)blockIdx.y];
    float *xb = J.xb;
    if (!xb) return;
    const uint32_t nbx = (uint32_t)J.nbx, nby = (uint32_t)J.nby, n0 = (uint32_t)J.n[0], n1 = (uint32_t)J.n[1];
    const uint32_t total = nbx * nby * (uint32_t)J.n[2] * 64u;
    const float *x = J.x;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const uint32_t brick = e >> 6, r = brick / nbx;
        const uint32_t ix = (brick - r * nbx) * 8u + (e & 7u);
        const uint32_t iz = r / nby;
        const uint32_t iy = (r - iz * nby) * 8u + ((e >> 3) & 7u);
        xb[e] = (ix < n0 && iy < n1) ? x[(size_t)ix + (size_t)n0 * ((size_t)iy + (size_t)n1 * iz)] : 0.0f;
    }
}

__global__ void k_put_jobs(JobDev *dst, JobPack pack) {
    const int words = (int)(sizeof(JobDev) / sizeof(uint64_t)) * pack.count;
    const uint64_t *src = reinterpret_cast<const uint64_t *>(pack.jobs);
    uint64_t *out = reinterpret_cast<uint64_t *>(dst + pack.first);
    for (int w = threadIdx.x; w < words; w += blockDim.x) out[w] = src[w];
}

constexpr int ORDER_PER_PACK = 900;
struct OrderPack {
    int32_t count;
    int32_t first;
    int32_t idx[ORDER_PER_PACK];
};

__global__ void k_put_order(int32_t *dst, OrderPack pack) {
    for (int i = threadIdx.x; i < pack.count; i += blockDim.x) dst[pack.first + i] = pack.idx[i];
}

__global__ void k_clear_status(WsHeader *h) {
    if (threadIdx.x == 0) h->status = PCT_OK;
}

// The tile counters of the persistent emit, reset by the call that uses them (a kernel,
// so that a captured graph holds no memset node).
__global__ void k_reset_queue(WsHeader *h) {
    if (threadIdx.x < 2) h->qnext[threadIdx.x] = 0ull;
}

__device__ __forceinline__ void set_status(int32_t *status, int32_t code) { set_status_dev(status, code); }

// Count tile -> job: the jobs' count tiles follow the count order (corder: the 2D jobs,
// then the 3D jobs, each in the caller's order); binary search on their tile_base.
__device__ __forceinline__ int job_of_tile(const JobDev *jobs, const int32_t *corder, int n_jobs, int64_t tile) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[corder[mid]].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return corder[lo];
}

// Emit tile -> job: the jobs are laid out in launch order (eorder); binary search on
// their etile_base.
__device__ __forceinline__ int job_of_etile(const JobDev *jobs, const int32_t *eorder, int n_jobs, int64_t tile) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[eorder[mid]].etile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return eorder[lo];
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *lds) {
    // wave reduce, then across the 4 waves of a 256-thread block
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    int64_t s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w];
    return s;
}

// Count pass (one lane per row): describe the row's path in the workspace and count its
// CSR entries.  With COUNT false the counts are not stored (WEPL-only calls).  One
// instance per grid dimension: a block whose job has the other dimension leaves at once
// and writes nothing (the other instance's launch covers its tile).
template <typename R, bool COUNT, int DIM>
__global__ void __launch_bounds__(TILE) k_count(const JobDev *__restrict__ jobs, const int32_t *__restrict__ corder,
                                                int n_jobs, int32_t *__restrict__ counts,
                                                int64_t *__restrict__ tile_sums, int32_t *__restrict__ tile_flags,
                                                char *__restrict__ rowbuf, int64_t tile_base) {
    __shared__ int64_t red[TILE / 64];
    const int64_t tile = tile_base + blockIdx.x;   // the tiles of DIM's jobs are one range
    const int jid = job_of_tile(jobs, corder, n_jobs, tile);
    const JobDev &J = jobs[jid];
    if (J.dim != DIM) return;   // block-uniform (never, with the range right)
    const int64_t r = (tile - J.tile_base) * TILE + threadIdx.x;
    int64_t cnt = 0;
    int lane_walk = 0;
    if (r < J.row_count) {
        const int64_t g = J.row_begin + r;
        // counted in both forms: the count decides which rows the per-lane walk takes
        const RowRefD<R, DIM> w = row_ref<R, DIM>(rowbuf, J, r);
        const RowSetup su = setup_row<R, DIM>(J, g, w);
        cnt = count_row<R, DIM>(J, w, g, su, lane_walk);
        if (COUNT) counts[J.count_off + r] = (int32_t)cnt;
    }
    // whether the per-lane emit kernel has a row in this tile
    const int any_lane = __syncthreads_or(lane_walk);
    if (threadIdx.x == 0) tile_flags[tile] = any_lane;
    if (COUNT) {
        const int64_t tot = block_sum_i64(cnt, red);
        if (threadIdx.x == 0) tile_sums[tile] = tot;
    }
}

// The count kernel's launches for a batch: one per grid dimension present.
// One instance per grid dimension, over that dimension's count tiles only (cbase,
// ctiles: the first tile and the tile count of the 2D jobs, then of the 3D jobs).
template <typename R, bool COUNT>
void launch_count(const int64_t cbase[2], const int64_t ctiles[2], hipStream_t s, const JobDev *J,
                  const int32_t *corder, int n_jobs, int32_t *counts, int64_t *sums, int32_t *flags, char *rows) {
    if (ctiles[0] > 0)
        hipLaunchKernelGGL((k_count<R, COUNT, 2>), dim3((unsigned)ctiles[0]), dim3(TILE), 0, s, J, corder, n_jobs,
                           counts, sums, flags, rows, cbase[0]);
    if (ctiles[1] > 0)
        hipLaunchKernelGGL((k_count<R, COUNT, 3>), dim3((unsigned)ctiles[1]), dim3(TILE), 0, s, J, corder, n_jobs,
                           counts, sums, flags, rows, cbase[1]);
}

// Grid dimensions present among the jobs that have rows.
void dims_present(int32_t n_jobs, const pct_job *jobs, bool &has2, bool &has3) {
    has2 = has3 = false;
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].beam->row_count == 0) continue;
        (jobs[j].phantom->dim == 3 ? has3 : has2) = true;
    }
}

// Exclusive scan of all tile sums (one block): offs[t] = sum of sums[0..t), offs[T] = total.
// Each job's row_ptr is relative to offs[tile_base]; its total goes to nnz_total and
// row_ptr[row_count].
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tiles(const JobDev *__restrict__ jobs, int n_jobs,
                                                             int64_t T, const int64_t *__restrict__ sums,
                                                             int64_t *__restrict__ offs,
                                                             int64_t *__restrict__ nnz_total) {
    // chunks of SCAN_THREADS * SCAN_ITEMS sums, loaded and stored coalesced through LDS;
    // thread t scans items [SCAN_ITEMS t, SCAN_ITEMS (t + 1)) of a chunk, the threads'
    // totals are scanned across the block (Hillis-Steele), and a carry runs over the chunks
    __shared__ int64_t buf[SCAN_THREADS * SCAN_ITEMS];
    __shared__ int64_t part[SCAN_THREADS];
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int64_t base = 0; base < T; base += SCAN_THREADS * SCAN_ITEMS) {
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            const int64_t e = base + i * SCAN_THREADS + t;
            buf[i * SCAN_THREADS + t] = e < T ? sums[e] : 0;
        }
        __syncthreads();
        int64_t acc = 0;
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; ++i) acc += buf[t * SCAN_ITEMS + i];
        part[t] = acc;
        __syncthreads();
        for (int off = 1; off < SCAN_THREADS; off <<= 1) {
            const int64_t v = (t >= off) ? part[t - off] : 0;
            __syncthreads();
            part[t] += v;
            __syncthreads();
        }
        int64_t run = carry + part[t] - acc;
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            const int64_t v = buf[t * SCAN_ITEMS + i];
            buf[t * SCAN_ITEMS + i] = run;
            run += v;
        }
        carry += part[SCAN_THREADS - 1];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            const int64_t e = base + i * SCAN_THREADS + t;
            if (e < T) offs[e] = buf[i * SCAN_THREADS + t];
        }
        __syncthreads();
    }
    if (t == 0) offs[T] = carry;
    __threadfence_block();
    __syncthreads();
    for (int j = threadIdx.x; j < n_jobs; j += SCAN_THREADS) {
        const JobDev &J = jobs[j];
        const int64_t tot = offs[J.tile_base + J.n_tiles] - offs[J.tile_base];
        nnz_total[j] = tot;
        J.row_ptr[J.row_count] = tot;
    }
}

// row_ptr[r] = (offset of the tile within its job) + exclusive scan of the tile's counts.
__global__ void __launch_bounds__(TILE) k_row_ptr(const JobDev *__restrict__ jobs, const int32_t *__restrict__ corder,
                                                  int n_jobs, const int32_t *__restrict__ counts,
                                                  const int64_t *__restrict__ offs) {
    __shared__ int64_t sc[TILE];
    __shared__ int wsum[TILE / WAVE];
    const int64_t tile = blockIdx.x;
    const int jid = job_of_tile(jobs, corder, n_jobs, tile);
    const JobDev &J = jobs[jid];
    const int64_t r = (tile - J.tile_base) * TILE + threadIdx.x;
    const int64_t c = (r < J.row_count) ? counts[J.count_off + r] : 0;
    const int64_t base = offs[tile] - offs[J.tile_base];
    if (offs[tile + 1] - offs[tile] <= INT32_MAX) {
        // the tile's entries fit in 32 bits: scans per wave (DPP) and over the 4 waves
        const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
        const int incl = wave_incl_scan((int)c);
        if (lane == WAVE - 1) wsum[w] = incl;
        __syncthreads();
        int before = 0;
        for (int i = 0; i < w; ++i) before += wsum[i];
        if (r < J.row_count) J.row_ptr[r] = base + (int64_t)(before + incl - (int)c);
        return;
    }
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < TILE; off <<= 1) {
        const int64_t v = (threadIdx.x >= (unsigned)off) ? sc[threadIdx.x - off] : 0;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    if (r < J.row_count) J.row_ptr[r] = base + sc[threadIdx.x] - c;
}

// Wave-cooperative emit: each wavefront of the block takes 64 rows of the tile.

// One instance per grid dimension (the register needs differ), launched over that
// dimension's emit tiles only: they are one range, [tile_base, tile_base + gridDim.x),
// of the launch order.  A block is one emit tile: 4 waves of rpw rows.
template <typename R, bool STORE, int DIM>
__global__ void __launch_bounds__(TILE) k_emit_wave(const JobDev *__restrict__ jobs, const int32_t *__restrict__ eorder,
                                                    int n_jobs, char *__restrict__ rowbuf,
                                                    int32_t *__restrict__ status, int64_t tile_base) {
    __shared__ __attribute__((aligned(16))) uint2 stage[TILE / WAVE][STAGE_CAP + 1];   // 1024 slots per wave
    const int64_t tile = tile_base + blockIdx.x;
    const int jid = job_of_etile(jobs, eorder, n_jobs, tile);
    const JobDev &J = jobs[jid];
    if (J.dim != DIM) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x % WAVE;
    const int64_t r0 = ((tile - J.etile_base) * (TILE / WAVE) + wave) * J.rpw;
    emit_rows_wave<R, DIM, STORE>(J, rowbuf, r0, J.rpw, lane, stage[wave], status);
}

// The same work from a persistent grid: each block takes the next emit tile of its grid
// dimension (tiles [tile_base, tile_base + n_tiles), jobs of DIM only) from the counter
// *qnext until none is left.  Every block leaves once the counter has passed n_tiles.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename R, bool STORE, int DIM>
__global__ void __launch_bounds__(TILE) k_emit_queue(const JobDev *__restrict__ jobs, const int32_t *__restrict__ eorder,
                                                     int n_jobs, char *__restrict__ rowbuf, int32_t *__restrict__ status,
                                                     unsigned long long *__restrict__ qnext, int64_t tile_base,
                                                     int64_t n_tiles) {
    __shared__ __attribute__((aligned(16))) uint2 stage[TILE / WAVE][STAGE_CAP + 1];   // 1024 slots per wave
    __shared__ int64_t taken;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x % WAVE;
    for (;;) {
        if (threadIdx.x == 0) taken = (int64_t)atomicAdd(qnext, 1ull);
        __syncthreads();
        const int64_t k = uniform_i64(taken);
        __syncthreads();   // every wave has read it before the next tile is taken
        if (k >= n_tiles) break;
        const int64_t tile = tile_base + k;
        const int jid = job_of_etile(jobs, eorder, n_jobs, tile);
        const JobDev &J = jobs[jid];
        if (J.dim != DIM) {   // the tile ranges of the dimensions were laid out wrongly
            if (threadIdx.x == 0) set_status(status, PCT_EINTERNAL);
            continue;
        }
        const int64_t r0 = ((tile - J.etile_base) * (TILE / WAVE) + wave) * J.rpw;
        emit_rows_wave<R, DIM, STORE>(J, rowbuf, r0, J.rpw, lane, stage[wave], status);
    }
}

// Rows whose spline may leave the grid box: one lane per row.
template <typename R, bool STORE>
__global__ void __launch_bounds__(TILE) k_emit_lane(const JobDev *__restrict__ jobs, const int32_t *__restrict__ corder,
                                                    int n_jobs, char *__restrict__ rowbuf,
                                                    const int32_t *__restrict__ tile_flags,
                                                    int32_t *__restrict__ status) {
    const int64_t tile = blockIdx.x;
    if (tile_flags[tile] == 0) return;   // no row of this tile needs the per-lane walk
    const int jid = job_of_tile(jobs, corder, n_jobs, tile);
    const JobDev &J = jobs[jid];
    const int64_t r = (tile - J.tile_base) * TILE + threadIdx.x;
    if (r >= J.row_count) return;
    if (J.dim == 3) {
        const RowRefD<R, 3> w = row_ref<R, 3>(rowbuf, J, r);
        if (RV(w, kind) == 3) emit_row_lane<R, 3, STORE>(J, w, r, status);
    } else {
        const RowRefD<R, 2> w = row_ref<R, 2>(rowbuf, J, r);
        if (RV(w, kind) == 3) emit_row_lane<R, 2, STORE>(J, w, r, status);
    }
}

// ---------------------------------------------------------------- phantom build
struct RegionDev {
    int32_t axes;   // 2: ellipse / cylinder, 3: ellipsoid
    float rsp;
    int32_t rot, pad;
    double c[3], s[3];
    double cr, sr;   // cosine and sine of the region's angle
    double hw[2];    // half-widths of its bounding box in x and y
};
struct PhantomArgs {
    int32_t dim, voxelize, n_regions, samples;
    int32_t n[3];
    double h[3], o[3];
    RegionDev reg[PCT_MAX_REGIONS];
};

// sum over the region's axes of (u_i / s_i)^2, u = p - c turned by minus the angle
__device__ __forceinline__ double region_q(const RegionDev &g, const double p[3]) {
    double d[3] = {p[0] - g.c[0], p[1] - g.c[1], p[2] - g.c[2]};
    if (g.rot) {
        const double u0 = g.cr * d[0] + g.sr * d[1];
        const double u1 = g.cr * d[1] - g.sr * d[0];
        d[0] = u0;
        d[1] = u1;
    }
    double q = 0.0;
    for (int i = 0; i < g.axes; ++i) {
        const double u = d[i] / g.s[i];
        q += u * u;
    }
    return q;
}

__device__ __forceinline__ double rsp_at(const PhantomArgs &A, const double p[3]) {
    double v = 0.0;
    for (int k = 0; k < A.n_regions; ++k)
        if (region_q(A.reg[k], p) <= 1.0) v = (double)A.reg[k].rsp;
    return v;
}

// Whether region g certainly contains (+1) or certainly misses (-1) every point of the
// box [lo, hi], with a margin of 1e-9 in q; 0 if the box may meet its boundary.
__device__ __forceinline__ int region_box(const RegionDev &g, const double lo[3], const double hi[3]) {
    constexpr double EPS = 1e-9;
    if (!g.rot) {
        double qmin = 0.0, qmax = 0.0;
        for (int i = 0; i < g.axes; ++i) {
            const double a = (lo[i] - g.c[i]) / g.s[i], b = (hi[i] - g.c[i]) / g.s[i];
            const double near = (a > 0.0) ? a : ((b < 0.0) ? b : 0.0);
            qmin += near * near;
            qmax += fmax(a * a, b * b);
        }
        if (qmax < 1.0 - EPS) return 1;
        if (qmin > 1.0 + EPS) return -1;
        return 0;
    }
    // turned ellipse: convex, so inside if every corner is; outside if the box misses
    // its bounding box (by a margin)
    bool all_in = true;
    const int nc = 1 << g.axes;
    for (int c = 0; c < nc; ++c) {
        double p[3];
        for (int i = 0; i < 3; ++i) p[i] = ((c >> i) & 1) ? hi[i] : lo[i];
        all_in = all_in && region_q(g, p) < 1.0 - EPS;
    }
    if (all_in) return 1;
    const double m = EPS * (g.s[0] + g.s[1]);
    bool out = false;
    for (int i = 0; i < 2; ++i) out = out || lo[i] > g.c[i] + g.hw[i] + m || hi[i] < g.c[i] - g.hw[i] - m;
    if (g.axes == 3) out = out || lo[2] > g.c[2] + g.s[2] * (1.0 + EPS) || hi[2] < g.c[2] - g.s[2] * (1.0 + EPS);
    return out ? -1 : 0;
}

// Voxel j (< 2^31: a grid has fewer voxels, see check_phantom) of the phantom A.
__device__ __forceinline__ void phantom_voxel(const PhantomArgs &A, float *__restrict__ x, uint32_t j) {
    const uint32_t n0 = (uint32_t)A.n[0], n1 = (uint32_t)A.n[1];
    int idx[3];
    idx[0] = (int)(j % n0);
    idx[1] = (int)((j / n0) % n1);
    idx[2] = (int)(j / (n0 * n1));
    double val;
    if (A.voxelize == PCT_AREA_AVG) {
        // weighted-area average: the mean RSP over S^dim midpoints of the voxel; a voxel
        // that no region boundary meets takes the one RSP all of them would give
        double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < A.dim; ++d) {
            lo[d] = A.o[d] + (double)idx[d] * A.h[d];
            hi[d] = A.o[d] + (double)(idx[d] + 1) * A.h[d];
        }
        bool uniform = true;
        double v = 0.0;
        for (int k = 0; k < A.n_regions; ++k) {
            const int st = region_box(A.reg[k], lo, hi);
            uniform = uniform && st != 0;
            if (st > 0) v = (double)A.reg[k].rsp;
        }
        if (uniform) {
            val = v;
        } else {
            const int S = A.samples;
            const int nz = A.dim == 3 ? S : 1;
            double sum = 0.0;
            for (int iz = 0; iz < nz; ++iz)
                for (int iy = 0; iy < S; ++iy)
                    for (int ix = 0; ix < S; ++ix) {
                        const int ii[3] = {ix, iy, iz};
                        double p[3] = {0.0, 0.0, 0.0};
                        for (int d = 0; d < A.dim; ++d) {
                            const double t = ((double)ii[d] + 0.5) / (double)S;
                            p[d] = A.o[d] + ((double)idx[d] + t) * A.h[d];
                        }
                        sum += rsp_at(A, p);
                    }
            val = sum / ((double)S * (double)S * (double)nz);
        }
    } else if (A.voxelize == PCT_CENTER) {
        double p[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < A.dim; ++d) p[d] = A.o[d] + ((double)idx[d] + 0.5) * A.h[d];
        val = rsp_at(A, p);
    } else {
        // corner average.  The corners share their coordinates per axis, so for a region
        // whose axes are not turned the scaled coordinates (p - c) / s are divided once per
        // axis and corner side and reused: the same values, summed in the same order, as
        // testing every corner on its own
        const int nc = 1 << A.dim;
        double pc[3][2];
        for (int d = 0; d < 3; ++d)
            for (int b = 0; b < 2; ++b) pc[d][b] = d < A.dim ? A.o[d] + (double)(idx[d] + b) * A.h[d] : 0.0;
        double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < A.n_regions; ++k) {
            const RegionDev &g = A.reg[k];
            const double rsp = (double)g.rsp;
            if (!g.rot) {
                double u[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    if (d < g.axes)
#pragma unroll
                        for (int b = 0; b < 2; ++b) u[d][b] = (pc[d][b] - g.c[d]) / g.s[d];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (c < nc) {
                        double q = 0.0;
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            if (i < g.axes) {
                                const double w = u[i][(c >> i) & 1];
                                q += w * w;
                            }
                        }
                        if (q <= 1.0) v[c] = rsp;
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (c < nc) {
                        const double p[3] = {pc[0][c & 1], pc[1][(c >> 1) & 1], pc[2][(c >> 2) & 1]};
                        if (region_q(g, p) <= 1.0) v[c] = rsp;
                    }
                }
            }
        }
        double sum = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < nc) sum += v[c];
        val = sum / (double)nc;
    }
    x[j] = (float)val;
}

// Corner average of PV voxels that follow one another along the last axis L (y in 2D, z
// in 3D), from voxel (i0, i1, i2) on; only cnt <= PV of them are written.  The corners
// of these voxels lie on 2 grid lines across each other axis and on cnt + 1 along L, so
// for a region whose axes are not turned each scaled coordinate (p - c) / s and its
// square are taken once per line and shared by the corners on it.  A corner's sum of
// squares is formed in the same order as in phantom_voxel ((s0 + s1) + s2, the leading
// 0 + s0 being exact), so every voxel gets the value phantom_voxel gives it.
constexpr int PV = 4;
template <int DIM>
__device__ __forceinline__ void phantom_corner_run(const PhantomArgs &A, float *__restrict__ x, int i0, int i1,
                                                   int i2, int cnt) {
    constexpr int L = DIM - 1, nc = 1 << DIM;
    const int idx[3] = {i0, i1, i2};
    // grid-line coordinates: pc[d][b], b < 2 across L, b <= PV along it
    double pc[3][PV + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int b = 0; b <= PV; ++b) pc[d][b] = d < DIM ? A.o[d] + (double)(idx[d] + b) * A.h[d] : 0.0;
    float v[PV][nc];   // RSP at each corner (binary32 values, exact in binary64)
#pragma unroll
    for (int t = 0; t < PV; ++t)
#pragma unroll
        for (int c = 0; c < nc; ++c) v[t][c] = 0.f;
    for (int k = 0; k < A.n_regions; ++k) {
        const RegionDev &g = A.reg[k];
        if (!g.rot) {
            // squares of the scaled coordinates per line (unused on an axis the region lacks)
            double sq[3][PV + 1];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int b = 0; b <= PV; ++b) {
                    sq[d][b] = 0.0;
                    if (d < DIM && (b < 2 || d == L) && d < g.axes) {
                        const double u = (pc[d][b] - g.c[d]) / g.s[d];
                        sq[d][b] = u * u;
                    }
                }
#pragma unroll
            for (int t = 0; t < PV; ++t)
#pragma unroll
                for (int c = 0; c < nc; ++c) {
                    double q = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        if (i < g.axes) {
                            const double si = sq[i][((c >> i) & 1) + (i == L ? t : 0)];
                            q = i == 0 ? si : q + si;
                        }
                    }
                    if (q <= 1.0) v[t][c] = g.rsp;
                }
        } else {
#pragma unroll
            for (int t = 0; t < PV; ++t)
#pragma unroll
                for (int c = 0; c < nc; ++c) {
                    double p[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) p[i] = pc[i][((c >> i) & 1) + (i == L ? t : 0)];
                    if (region_q(g, p) <= 1.0) v[t][c] = g.rsp;
                }
        }
    }
    const int64_t n0 = A.n[0], n01 = (int64_t)A.n[0] * A.n[1];
#pragma unroll
    for (int t = 0; t < PV; ++t) {
        if (t < cnt) {
            double sum = 0.0;
#pragma unroll
            for (int c = 0; c < nc; ++c) sum += (double)v[t][c];
            const int j1 = i1 + (L == 1 ? t : 0), j2 = i2 + (L == 2 ? t : 0);
            x[i0 + n0 * j1 + n01 * j2] = (float)(sum / (double)nc);
        }
    }
}

// The corner rule: one thread per run of PV voxels along the last axis (x fastest, then
// the other axis across it, then the run); the other rules: one thread per voxel.
__global__ void __launch_bounds__(256) k_phantom(PhantomArgs A, float *__restrict__ x, int64_t nvox) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (A.voxelize != PCT_CORNER_AVG) {
        if (j < nvox) phantom_voxel(A, x, (uint32_t)j);
        return;
    }
    const uint32_t n0 = (uint32_t)A.n[0];
    const uint32_t nacr = A.dim == 3 ? (uint32_t)A.n[1] : 1u;
    const uint32_t nL = (uint32_t)A.n[A.dim - 1];
    const uint32_t runs = (nL + PV - 1) / PV;
    if (j >= (int64_t)n0 * nacr * runs) return;
    const uint32_t jj = (uint32_t)j;
    const int i0 = (int)(jj % n0);
    const int ia = (int)((jj / n0) % nacr);
    const int lo = (int)(jj / (n0 * nacr)) * PV, cnt = min(PV, (int)nL - lo);
    if (A.dim == 3) phantom_corner_run<3>(A, x, i0, ia, lo, cnt);
    else phantom_corner_run<2>(A, x, i0, lo, 0, cnt);
}

// ------------------------------------------------------------------ host helpers

static bool finite_d(double v) { return isfinite(v) != 0; }

static pct_status check_phantom(const pct_phantom *ph) {
    if (!ph) return PCT_EINVAL;
    if (ph->dim != 2 && ph->dim != 3) return PCT_EINVAL;
    if (ph->n_regions < 1 || ph->n_regions > PCT_MAX_REGIONS || !ph->regions) return PCT_EINVAL;
    if (ph->voxelize != PCT_CORNER_AVG && ph->voxelize != PCT_CENTER && ph->voxelize != PCT_AREA_AVG)
        return PCT_EINVAL;
    if (ph->voxelize == PCT_AREA_AVG && (ph->area_samples < 0 || ph->area_samples > 64)) return PCT_EINVAL;
    int64_t nv = 1;
    for (int d = 0; d < ph->dim; ++d) {
        if (ph->n[d] < 1) return PCT_EINVAL;
        if (!(ph->h[d] > 0.0) || !finite_d(ph->h[d]) || !finite_d(ph->origin[d])) return PCT_EINVAL;
        nv *= ph->n[d];
        if (nv >= ((int64_t)1 << 31)) return PCT_ERANGE;
    }
    for (int k = 0; k < ph->n_regions; ++k) {
        const pct_region &r = ph->regions[k];
        if (r.shape != PCT_ELLIPSE && r.shape != PCT_ELLIPSOID) return PCT_EINVAL;
        if (!(r.rsp >= 0.0f) || !isfinite(r.rsp)) return PCT_EINVAL;
        const int na = (r.shape == PCT_ELLIPSOID && ph->dim == 3) ? 3 : 2;
        for (int i = 0; i < na; ++i) {
            if (!(r.semi[i] > 0.0) || !finite_d(r.semi[i]) || !finite_d(r.center[i])) return PCT_EINVAL;
        }
        if (!finite_d(r.angle_deg) || fabs(r.angle_deg) > 360.0) return PCT_EINVAL;
    }
    return PCT_OK;
}

static int64_t n_voxels(const pct_phantom *ph) {
    int64_t nv = 1;
    for (int d = 0; d < ph->dim; ++d) nv *= ph->n[d];
    return nv;
}

static pct_status check_beam(const pct_beam *b) {
    if (!b) return PCT_EINVAL;
    if (b->n_angles < 1 || b->n_protons < 0) return PCT_EINVAL;
    if (b->row_begin < 0 || b->row_count < 0 || b->row_begin + b->row_count > b->n_protons) return PCT_EINVAL;
    if (b->path != PCT_STRAIGHT && b->path != PCT_HERMITE) return PCT_EINVAL;
    const double f[] = {b->angle0_deg, b->dangle_deg, b->t_range[0], b->t_range[1], b->v_range[0],
                        b->v_range[1], b->sigma_in_rad, b->sigma_out_rad, b->sigma_lat_mm, b->rho,
                        b->step_mm, b->noise_rel};
    for (double v : f)
        if (!finite_d(v)) return PCT_EINVAL;
    if (b->t_range[0] > b->t_range[1] || b->v_range[0] > b->v_range[1]) return PCT_EINVAL;
    if (b->sigma_in_rad < 0 || b->sigma_out_rad < 0 || b->sigma_lat_mm < 0 || b->noise_rel < 0) return PCT_EINVAL;
    if (b->rho < -1.0 || b->rho > 1.0) return PCT_EINVAL;
    if (b->sigma_in_rad > 0.1 || b->sigma_out_rad > 0.1) return PCT_EINVAL;
    if (b->path == PCT_HERMITE && !(b->step_mm > 0.0)) return PCT_EINVAL;
    if (b->scatter != PCT_SCATTER_FIXED && b->scatter != PCT_SCATTER_HIGHLAND) return PCT_EINVAL;
    if (b->scatter == PCT_SCATTER_HIGHLAND) {
        if (!(b->energy_mev >= 1.0 && b->energy_mev <= 10000.0)) return PCT_EINVAL;
        if (!(b->x0_mm > 0.0) || !finite_d(b->x0_mm)) return PCT_EINVAL;
    }
    // (g + 1) * K must not overflow int64 in the row decode
    if (b->n_protons > 0 && (double)b->n_protons * (double)b->n_angles > 9.0e18) return PCT_ERANGE;
    return PCT_OK;
}

static pct_status check_jobs(int32_t n_jobs, const pct_job *jobs, bool need_csr, bool need_b) {
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return PCT_EINVAL;
    for (int j = 0; j < n_jobs; ++j) {
        const pct_job &jb = jobs[j];
        pct_status st = check_phantom(jb.phantom);
        if (st != PCT_OK) return st;
        st = check_beam(jb.beam);
        if (st != PCT_OK) return st;
        if (jb.val_dtype != PCT_F32 && jb.val_dtype != PCT_F16) return PCT_EINVAL;
        if (jb.precision != PCT_MIXED && jb.precision != PCT_PLAIN_F32) return PCT_EINVAL;
        if (jb.precision != jobs[0].precision) return PCT_EINVAL;
        if (jb.nnz_capacity < 0) return PCT_EINVAL;
        if (!(jb.chord_mm >= 0.0) || !(jb.chord_mm < 1.0e30)) return PCT_EINVAL;
        if (!jb.x_dev && (need_b || jb.b_dev)) return PCT_EINVAL;
        if (need_csr && !jb.row_ptr_dev) return PCT_EINVAL;
        if (need_csr && jb.nnz_capacity > 0 && (!jb.cols_dev || !jb.vals_dev)) return PCT_EINVAL;
        if (need_b && !jb.b_dev) return PCT_EINVAL;
        if (jb.beam->path == PCT_HERMITE) {
            // bound on the spline sample count: entry and exit lie on the outer boundary and
            // the entry direction is within atan(tan(1.2)) of the beam axis (|sigma z| <= 1.2),
            // so the chord is at most 3 outer diameters (cylinder) -- keep per-row work finite
            const pct_region &o = jb.phantom->regions[0];
            double smax = 0.0;
            for (int i = 0; i < 3; ++i)
                if (i < 2 || (o.shape == PCT_ELLIPSOID && jb.phantom->dim == 3)) smax = fmax(smax, o.semi[i]);
            if (6.0 * smax / jb.beam->step_mm > (double)(1 << 22)) return PCT_ERANGE;
        }
    }
    return PCT_OK;
}

static JobDev make_job(const pct_job &jb, int64_t count_off, int64_t tile_base) {
    const pct_phantom &ph = *jb.phantom;
    const pct_beam &bm = *jb.beam;
    JobDev J;
    memset(&J, 0, sizeof J);
    J.dim = ph.dim;
    J.path = bm.path;
    J.val_dtype = jb.val_dtype;
    const pct_region &o = ph.regions[0];
    J.outer_axes = (o.shape == PCT_ELLIPSOID && ph.dim == 3) ? 3 : 2;
    for (int d = 0; d < 3; ++d) {
        const bool on = d < ph.dim;
        J.n[d] = on ? ph.n[d] : 1;
        J.h[d] = on ? ph.h[d] : 1.0;
        J.invh[d] = 1.0 / J.h[d];
        J.o[d] = on ? ph.origin[d] : 0.0;
        J.top[d] = J.o[d] + (double)J.n[d] * J.h[d];
        J.oc[d] = o.center[d];
        J.inv_s2[d] = (d < J.outer_axes) ? 1.0 / (o.semi[d] * o.semi[d]) : 0.0;
    }
    J.orot_on = o.angle_deg != 0.0 ? 1 : 0;
    const double oang = o.angle_deg * (3.14159265358979323846 / 180.0);
    J.orot[0] = J.orot_on ? cos(oang) : 1.0;
    J.orot[1] = J.orot_on ? sin(oang) : 0.0;
    J.K = bm.n_angles;
    J.seed = bm.seed;
    J.angle0 = bm.angle0_deg;
    J.dangle = bm.dangle_deg;
    J.P = bm.n_protons;
    J.row_begin = bm.row_begin;
    J.row_count = bm.row_count;
    J.t_lo = bm.t_range[0];
    J.t_span = bm.t_range[1] - bm.t_range[0];
    J.v_lo = bm.v_range[0];
    J.v_span = bm.v_range[1] - bm.v_range[0];
    J.sig_in = bm.sigma_in_rad;
    J.sig_out = bm.sigma_out_rad;
    J.sig_lat = bm.sigma_lat_mm;
    J.rho = bm.rho;
    J.crho = sqrt(1.0 - bm.rho * bm.rho);
    J.step = bm.step_mm;
    J.noise = bm.noise_rel;
    J.highland = bm.scatter == PCT_SCATTER_HIGHLAND ? 1 : 0;
    if (J.highland) {
        // proton of kinetic energy T: p c = sqrt(T (T + 2 m)), beta = p c / (T + m)
        const double mp = 938.27208816;   // proton mass, MeV
        const double T = bm.energy_mev, E = T + mp, pc = sqrt(T * (T + 2.0 * mp));
        const double beta = pc / E;
        J.hl_k = 13.6 / (beta * pc);
        J.hl_x0inv = 1.0 / bm.x0_mm;
        J.hl_lnb2 = log(beta * beta);
    }
    J.chord = (float)jb.chord_mm;
    J.x = jb.x_dev;
    J.row_ptr = jb.row_ptr_dev;
    J.cols = jb.cols_dev;
    J.vals = jb.vals_dev;
    J.b = jb.b_dev;
    J.cap = jb.nnz_capacity;
    J.count_off = count_off;
    J.tile_base = tile_base;
    J.n_tiles = (bm.row_count + TILE - 1) / TILE;
    J.nmax = J.n[0] > J.n[1] ? J.n[0] : J.n[1];
    J.nmax = J.n[2] > J.nmax ? J.n[2] : J.nmax;
    return J;
}

// Process-wide launch configuration of the emit pass (read-mostly).
static constexpr pct_launch_config DEFAULT_CFG = {64, PCT_ORDER_LPT, 0};
static pct_launch_config g_cfg = DEFAULT_CFG;

static bool config_ok(const pct_launch_config &c) {
    return (c.rows_per_wave == 16 || c.rows_per_wave == 32 || c.rows_per_wave == 64) &&
           (c.order == PCT_ORDER_GIVEN || c.order == PCT_ORDER_LPT) && c.blocks_per_cu >= 0 &&
           c.blocks_per_cu <= 8;
}

// Compute units of the current device (queried once per device).
static int cu_count() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    if (dev < 64) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    if (dev < 64) cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

// ---------------------------------------------------------------- autotuner cache
// Key: FNV-1a over the device's architecture name, the HIP runtime version and the shape
// of the batch (per job: dimension, grid sizes, path, precision, value type, whether b is
// written, and floor(log2(row count))).
struct TuneCache {
    std::mutex mu;
    std::unordered_map<uint64_t, pct_launch_config> map;
    bool loaded = false;
};
static TuneCache g_tune;

static void fnv1a(uint64_t &h, const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
}

static bool tune_key(int32_t n_jobs, const pct_job *jobs, uint64_t &key) {
    static std::atomic<uint64_t> arch_hash[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return false;
    uint64_t ah = dev < 64 ? arch_hash[dev].load(std::memory_order_relaxed) : 0;
    if (ah == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
        int rt = 0;
        if (hipRuntimeGetVersion(&rt) != hipSuccess) return false;
        ah = 1469598103934665603ull;
        fnv1a(ah, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
        fnv1a(ah, &rt, sizeof rt);
        if (ah == 0) ah = 1;
        if (dev < 64) arch_hash[dev].store(ah, std::memory_order_relaxed);
    }
    uint64_t h = ah;
    fnv1a(h, &n_jobs, sizeof n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        const pct_job &jb = jobs[j];
        int64_t rc = jb.beam->row_count;
        int32_t lg = 0;
        while (rc > 1) {
            rc >>= 1;
            ++lg;
        }
        const int32_t f[9] = {jb.phantom->dim, jb.phantom->n[0], jb.phantom->n[1], jb.phantom->n[2], jb.beam->path,
                              jb.precision, jb.val_dtype, jb.b_dev != nullptr ? 1 : 0, lg};
        fnv1a(h, f, sizeof f);
    }
    key = h;
    return true;
}

// The file named by PCT_TUNE_CACHE, read once: lines "<key in hex> rows_per_wave order blocks_per_cu".
static void tune_load_locked() {
    if (g_tune.loaded) return;
    g_tune.loaded = true;
    const char *path = getenv("PCT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    unsigned long long k = 0;
    int r = 0, o = 0, q = 0;
    while (fscanf(f, "%llx %d %d %d", &k, &r, &o, &q) == 4) {
        const pct_launch_config c{r, o, q};
        if (config_ok(c)) g_tune.map[(uint64_t)k] = c;
    }
    fclose(f);
}

static bool tune_lookup(uint64_t key, pct_launch_config &cfg) {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    tune_load_locked();
    const auto it = g_tune.map.find(key);
    if (it == g_tune.map.end()) return false;
    cfg = it->second;
    return true;
}

static void tune_store(uint64_t key, const pct_launch_config &cfg) {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    tune_load_locked();
    g_tune.map[key] = cfg;
    const char *path = getenv("PCT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%016llx %d %d %d\n", (unsigned long long)key, cfg.rows_per_wave, cfg.order, cfg.blocks_per_cu);
    fclose(f);
}

// Relative cost of one row of a job: voxels a path crosses (about the sum of the grid
// sizes) plus, for spline paths, the samples over an outer-boundary diameter.
static double row_cost(const pct_job &jb) {
    const pct_phantom &ph = *jb.phantom;
    double c = 0.0;
    for (int d = 0; d < ph.dim; ++d) c += ph.n[d];
    if (jb.beam->path == PCT_HERMITE) {
        double smax = 0.0;
        for (int i = 0; i < 3; ++i) smax = fmax(smax, ph.regions[0].semi[i]);
        c += 2.0 * smax / jb.beam->step_mm;
    }
    return c;
}

// Host-side arrays of one call: on the stack for up to FIXED jobs (so that a call with
// few jobs allocates no host memory either), on the heap beyond.
struct HostJobs {
    static constexpr int FIXED = 64;
    int64_t rc_fixed[FIXED];
    JobDev jobs_fixed[FIXED];
    int32_t order_fixed[FIXED * 2];   // emit order, then count order
    double cost_fixed[FIXED];
    size_t bb_fixed[FIXED];
    std::vector<int64_t> rc_heap;
    std::vector<JobDev> jobs_heap;
    std::vector<int32_t> order_heap;
    std::vector<double> cost_heap;
    std::vector<size_t> bb_heap;
    int64_t *rc = rc_fixed;
    JobDev *jobs = jobs_fixed;
    int32_t *order = order_fixed;
    double *cost = cost_fixed;
    size_t *bb = bb_fixed;   // bytes of each job's bricked copy of x
    explicit HostJobs(int32_t n) {
        if (n > FIXED) {
            rc_heap.resize(n);
            jobs_heap.resize(n);
            order_heap.resize(2 * (size_t)n);
            cost_heap.resize(n);
            bb_heap.resize(n);
            rc = rc_heap.data();
            jobs = jobs_heap.data();
            order = order_heap.data();
            cost = cost_heap.data();
            bb = bb_heap.data();
        }
    }
    HostJobs(const HostJobs &) = delete;
    HostJobs &operator=(const HostJobs &) = delete;
};

struct Prepared {
    Layout L;
    HostJobs H;
    pct_launch_config cfg = DEFAULT_CFG;
    int64_t total_etiles = 0;
    int64_t dim_base[2] = {0, 0}, dim_tiles[2] = {0, 0};   // emit tiles of the 2D jobs, then the 3D jobs
    int64_t cdim_base[2] = {0, 0}, cdim_tiles[2] = {0, 0}; // count tiles likewise
    bool any_bricks = false;                                 // some job has a bricked copy of x to fill
    explicit Prepared(int32_t n) : H(n) {}
};

// Job table (caller's order; the count pass uses it as is) and the emit launch order,
// both uploaded through kernel arguments.  bricks: jobs that allow it get a bricked
// copy of x in the workspace (every call on a workspace sized by pct_workspace_bytes).
static pct_status prepare(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes, Prepared &P,
                          hipStream_t st, bool bricks = true) {
    int64_t *rc = P.H.rc;
    JobDev *jd = P.H.jobs;
    size_t *bb = P.H.bb;
    for (int j = 0; j < n_jobs; ++j) {
        rc[j] = jobs[j].beam->row_count;
        bb[j] = bricks ? (size_t)brick_elems(*jobs[j].phantom, *jobs[j].beam) * sizeof(float) : 0;
    }
    P.L = layout_of(n_jobs, rc, bb);
    if (!ws || ws_bytes < P.L.total) return PCT_EWORKSPACE;
    int64_t count_off = 0;
    size_t boff = P.L.bricks_off;
    for (int j = 0; j < n_jobs; ++j) {
        jd[j] = make_job(jobs[j], count_off, 0);
        count_off += rc[j];
        if (bb[j] > 0 && jobs[j].x_dev) {
            jd[j].xb = reinterpret_cast<float *>((char *)ws + boff);
            jd[j].nbx = (jd[j].n[0] + 7) / 8;
            jd[j].nby = (jd[j].n[1] + 7) / 8;
            P.any_bricks = true;
        }
        boff += align256(bb[j]);
    }
    // count tiles (and the row descriptions stored per tile): the 2D jobs, then the 3D
    // jobs, each in the caller's order, so that each dimension's count kernel takes one
    // range of tiles; independent of the launch configuration, so that a count and an
    // emit under different configurations agree
    int32_t *corder = P.H.order + n_jobs;
    {
        int k = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < n_jobs; ++j)
                if ((jd[j].dim == 3) == (pass == 1)) corder[k++] = j;
        int64_t tile = 0;
        for (int k2 = 0; k2 < n_jobs; ++k2) {
            JobDev &J = jd[corder[k2]];
            J.tile_base = tile;
            const int di = J.dim == 3 ? 1 : 0;
            if (P.cdim_tiles[di] == 0) P.cdim_base[di] = tile;
            P.cdim_tiles[di] += J.n_tiles;
            tile += J.n_tiles;
        }
    }
    const pct_launch_config cfg = g_cfg;
    P.cfg = cfg;
    int32_t *order = P.H.order;
    for (int j = 0; j < n_jobs; ++j) order[j] = j;
    // launch order: the 2D jobs, then the 3D jobs (so that each dimension's emit tiles are
    // one range), each in the caller's order or costliest rows first
    const bool lpt = cfg.order == PCT_ORDER_LPT;
    double *cost = P.H.cost;
    for (int j = 0; j < n_jobs; ++j) cost[j] = lpt ? row_cost(jobs[j]) : 0.0;
    auto before = [&](int a, int b) {
        const int da = jd[a].dim, db = jd[b].dim;
        return da != db ? da < db : cost[a] > cost[b];
    };
    if (n_jobs <= HostJobs::FIXED) {
        // stable insertion sort: no temporary buffer
        for (int i = 1; i < n_jobs; ++i) {
            const int32_t v = order[i];
            int k = i;
            for (; k > 0 && before(v, order[k - 1]); --k) order[k] = order[k - 1];
            order[k] = v;
        }
    } else {
        std::stable_sort(order, order + n_jobs, before);
    }
    const int64_t rows_per_etile = (int64_t)(TILE / WAVE) * cfg.rows_per_wave;
    int64_t etile = 0;
    for (int k = 0; k < n_jobs; ++k) {
        JobDev &J = jd[order[k]];
        J.rpw = cfg.rows_per_wave;
        J.etile_base = etile;
        J.n_etiles = (J.row_count + rows_per_etile - 1) / rows_per_etile;
        const int di = J.dim == 3 ? 1 : 0;
        if (P.dim_tiles[di] == 0) P.dim_base[di] = etile;
        P.dim_tiles[di] += J.n_etiles;
        etile += J.n_etiles;
    }
    P.total_etiles = etile;
    char *w = (char *)ws;
    JobDev *dst = reinterpret_cast<JobDev *>(w + P.L.jobs_off);
    for (int first = 0; first < n_jobs; first += JOBS_PER_PACK) {
        JobPack pack;
        memset(&pack, 0, sizeof pack);
        pack.first = first;
        pack.count = (n_jobs - first < JOBS_PER_PACK) ? n_jobs - first : JOBS_PER_PACK;
        for (int k = 0; k < pack.count; ++k) pack.jobs[k] = jd[first + k];
        hipLaunchKernelGGL(k_put_jobs, dim3(1), dim3(256), 0, st, dst, pack);
    }
    // the emit order, then the count order
    int32_t *odst = reinterpret_cast<int32_t *>(w + P.L.order_off);
    for (int first = 0; first < 2 * n_jobs; first += ORDER_PER_PACK) {
        OrderPack pack;
        memset(&pack, 0, sizeof pack);
        pack.first = first;
        pack.count = (2 * n_jobs - first < ORDER_PER_PACK) ? 2 * n_jobs - first : ORDER_PER_PACK;
        for (int k = 0; k < pack.count; ++k) pack.idx[k] = order[first + k];
        hipLaunchKernelGGL(k_put_order, dim3(1), dim3(256), 0, st, odst, pack);
    }
    return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
}

// The emit kernels of one call: per grid dimension either a grid over its tiles or a
// persistent grid that takes them from a queue; then the per-lane kernel.
template <typename R, bool STORE>
static void launch_emit(const Prepared &P, bool has2, bool has3, hipStream_t s, const JobDev *J,
                        const int32_t *eorder, int n_jobs, char *rb, int32_t *flags, int32_t *status, WsHeader *hdr,
                        dim3 grid) {
    const dim3 block(TILE);
    if (P.cfg.blocks_per_cu > 0) {
        hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, hdr);
        const int64_t cap = (int64_t)cu_count() * P.cfg.blocks_per_cu;
        const int64_t n2 = has2 ? P.dim_tiles[0] : 0, n3 = has3 ? P.dim_tiles[1] : 0;
        if (n2 > 0)
            hipLaunchKernelGGL((k_emit_queue<R, STORE, 2>), dim3((unsigned)(n2 < cap ? n2 : cap)), block, 0, s, J,
                               eorder, n_jobs, rb, status, &hdr->qnext[0], P.dim_base[0], n2);
        if (n3 > 0)
            hipLaunchKernelGGL((k_emit_queue<R, STORE, 3>), dim3((unsigned)(n3 < cap ? n3 : cap)), block, 0, s, J,
                               eorder, n_jobs, rb, status, &hdr->qnext[1], P.dim_base[1], n3);
    } else {
        if (has2 && P.dim_tiles[0] > 0)
            hipLaunchKernelGGL((k_emit_wave<R, STORE, 2>), dim3((unsigned)P.dim_tiles[0]), block, 0, s, J, eorder,
                               n_jobs, rb, status, P.dim_base[0]);
        if (has3 && P.dim_tiles[1] > 0)
            hipLaunchKernelGGL((k_emit_wave<R, STORE, 3>), dim3((unsigned)P.dim_tiles[1]), block, 0, s, J, eorder,
                               n_jobs, rb, status, P.dim_base[1]);
    }
    hipLaunchKernelGGL((k_emit_lane<R, STORE>), grid, block, 0, s, J, eorder + n_jobs, n_jobs, rb, flags, status);
}

}  // namespace pct

using namespace pct;

extern "C" {

const char *pct_status_string(pct_status s) {
    switch (s) {
        case PCT_OK: return "PCT_OK";
        case PCT_EINVAL: return "PCT_EINVAL: invalid descriptor";
        case PCT_ERANGE: return "PCT_ERANGE: size overflows the index types";
        case PCT_ECAPACITY: return "PCT_ECAPACITY: row did not fit in nnz_capacity";
        case PCT_EWORKSPACE: return "PCT_EWORKSPACE: workspace missing or too small";
        case PCT_EHIP: return "PCT_EHIP: HIP runtime error";
        case PCT_EINTERNAL: return "PCT_EINTERNAL: emitted entries differ from the count";
        case PCT_EIO: return "PCT_EIO: a file could not be opened or written";
        case PCT_ESCRATCH: return "PCT_ESCRATCH: more jobs or rows than the static scratch of pct_wepl_static holds";
        default: return "unknown pct status";
    }
}

int32_t pct_version(void) { return 100; }

pct_status pct_phantom_build(const pct_phantom *ph, float *x_dev, void *stream) {
    pct_status st = check_phantom(ph);
    if (st != PCT_OK) return st;
    if (!x_dev) return PCT_EINVAL;
    PhantomArgs A;
    memset(&A, 0, sizeof A);
    A.dim = ph->dim;
    A.voxelize = ph->voxelize;
    A.n_regions = ph->n_regions;
    A.samples = ph->area_samples > 0 ? ph->area_samples : 8;
    for (int d = 0; d < 3; ++d) {
        A.n[d] = d < ph->dim ? ph->n[d] : 1;
        A.h[d] = d < ph->dim ? ph->h[d] : 1.0;
        A.o[d] = d < ph->dim ? ph->origin[d] : 0.0;
    }
    for (int k = 0; k < ph->n_regions; ++k) {
        const pct_region &r = ph->regions[k];
        A.reg[k].axes = (r.shape == PCT_ELLIPSOID && ph->dim == 3) ? 3 : 2;
        A.reg[k].rsp = r.rsp;
        for (int i = 0; i < 3; ++i) {
            A.reg[k].c[i] = r.center[i];
            A.reg[k].s[i] = r.semi[i];
        }
        A.reg[k].rot = r.angle_deg != 0.0 ? 1 : 0;
        const double ang = r.angle_deg * (3.14159265358979323846 / 180.0);
        A.reg[k].cr = A.reg[k].rot ? cos(ang) : 1.0;
        A.reg[k].sr = A.reg[k].rot ? sin(ang) : 0.0;
        const double cr = A.reg[k].cr, sr = A.reg[k].sr;
        A.reg[k].hw[0] = sqrt(r.semi[0] * r.semi[0] * cr * cr + r.semi[1] * r.semi[1] * sr * sr);
        A.reg[k].hw[1] = sqrt(r.semi[0] * r.semi[0] * sr * sr + r.semi[1] * r.semi[1] * cr * cr);
    }
    const int64_t nv = n_voxels(ph);
    const int64_t nL = A.n[A.dim - 1];
    const int64_t threads = A.voxelize == PCT_CORNER_AVG ? nv / nL * ((nL + PV - 1) / PV) : nv;
    const int64_t blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(k_phantom, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, A, x_dev, nv);
    return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
}

size_t pct_workspace_bytes(int32_t n_jobs, const pct_job *jobs) {
    if (check_jobs(n_jobs, jobs, false, false) != PCT_OK) return 0;
    std::vector<int64_t> rc(n_jobs > 0 ? n_jobs : 1);
    std::vector<size_t> bb(n_jobs > 0 ? n_jobs : 1);
    for (int j = 0; j < n_jobs; ++j) {
        rc[j] = jobs[j].beam->row_count;
        bb[j] = (size_t)brick_elems(*jobs[j].phantom, *jobs[j].beam) * sizeof(float);
    }
    return layout_of(n_jobs, rc.data(), bb.data()).total;
}

}  // extern "C"
static pct_status count_common(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes,
                               int64_t *nnz_total_dev, void *stream, bool clear_status);
extern "C" {

pct_status pct_count_rows(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes,
                          int64_t *nnz_total_dev, void *stream) {
    return count_common(n_jobs, jobs, ws, ws_bytes, nnz_total_dev, stream, true);
}

}  // extern "C"

// The count pass; clear_status: start the device status word afresh (every public count
// call; a later set of a graph of sets keeps the earlier sets' errors).
static pct_status count_common(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes,
                               int64_t *nnz_total_dev, void *stream, bool clear_status) {
    pct_status st = check_jobs(n_jobs, jobs, true, false);
    if (st != PCT_OK) return st;
    if (n_jobs > 0 && !nnz_total_dev) return PCT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!ws) return PCT_EWORKSPACE;
    Prepared P(n_jobs);
    st = prepare(n_jobs, jobs, ws, ws_bytes, P, s);
    if (st != PCT_OK) return st;
    char *w = (char *)ws;
    if (clear_status) hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, (WsHeader *)w);
    if (n_jobs == 0) return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
    const JobDev *J = (const JobDev *)(w + P.L.jobs_off);
    const int32_t *corder = (const int32_t *)(w + P.L.order_off) + n_jobs;
    int64_t *sums = (int64_t *)(w + P.L.sums_off);
    int64_t *offs = (int64_t *)(w + P.L.offs_off);
    int32_t *counts = (int32_t *)(w + P.L.counts_off);
    const int64_t T = P.L.total_tiles;
    if (T > 0) {
        if (jobs[0].precision == PCT_MIXED)
            launch_count<double, true>(P.cdim_base, P.cdim_tiles, s, J, corder, n_jobs, counts, sums,
                                       (int32_t *)(w + P.L.flags_off), w + P.L.rows_off);
        else
            launch_count<float, true>(P.cdim_base, P.cdim_tiles, s, J, corder, n_jobs, counts, sums,
                                      (int32_t *)(w + P.L.flags_off), w + P.L.rows_off);
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(SCAN_THREADS), 0, s, J, n_jobs, T, sums, offs, nnz_total_dev);
    if (T > 0) hipLaunchKernelGGL(k_row_ptr, dim3((unsigned)T), dim3(TILE), 0, s, J, corder, n_jobs, counts, offs);
    return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
}

extern "C" {

static pct_status emit_common(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes, void *stream,
                              bool store, bool bricks = true) {
    pct_status st = check_jobs(n_jobs, jobs, store, !store);
    if (st != PCT_OK) return st;
    if (n_jobs == 0) return PCT_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!ws) return PCT_EWORKSPACE;
    Prepared P(n_jobs);
    st = prepare(n_jobs, jobs, ws, ws_bytes, P, s, bricks);
    if (st != PCT_OK) return st;
    char *w = (char *)ws;
    const JobDev *J = (const JobDev *)(w + P.L.jobs_off);
    if (P.any_bricks && P.L.total_tiles > 0)
        for (int32_t j0 = 0; j0 < n_jobs; j0 += 65535) {
            const int32_t nj = n_jobs - j0 < 65535 ? n_jobs - j0 : 65535;
            hipLaunchKernelGGL(k_brick, dim3(BRICK_BLOCKS, (unsigned)nj), dim3(256), 0, s, J, j0);
        }
    int32_t *status = &((WsHeader *)w)->status;
    // WEPL only runs its own count pass: the status word starts afresh, as in a count call
    if (!store) hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, (WsHeader *)w);
    const int64_t T = P.L.total_tiles;
    if (T == 0) return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
    const bool mixed = jobs[0].precision == PCT_MIXED;
    bool has2, has3;
    dims_present(n_jobs, jobs, has2, has3);
    const int32_t *eorder = (const int32_t *)(w + P.L.order_off);
    int32_t *flags = (int32_t *)(w + P.L.flags_off);
    void *rows = w + P.L.rows_off;
    const dim3 grid((unsigned)T);
    char *rb = (char *)rows;
    WsHeader *hdr = (WsHeader *)w;
    if (mixed) {
        if (!store)
            launch_count<double, false>(P.cdim_base, P.cdim_tiles, s, J, eorder + n_jobs, n_jobs, nullptr, nullptr,
                                        flags, rb);
        if (store) launch_emit<double, true>(P, has2, has3, s, J, eorder, n_jobs, rb, flags, status, hdr, grid);
        else launch_emit<double, false>(P, has2, has3, s, J, eorder, n_jobs, rb, flags, status, hdr, grid);
    } else {
        if (!store)
            launch_count<float, false>(P.cdim_base, P.cdim_tiles, s, J, eorder + n_jobs, n_jobs, nullptr, nullptr,
                                       flags, rb);
        if (store) launch_emit<float, true>(P, has2, has3, s, J, eorder, n_jobs, rb, flags, status, hdr, grid);
        else launch_emit<float, false>(P, has2, has3, s, J, eorder, n_jobs, rb, flags, status, hdr, grid);
    }
    return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
}

pct_status pct_emit_csr(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes, void *stream) {
    return emit_common(n_jobs, jobs, ws, ws_bytes, stream, true);
}

pct_status pct_wepl(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes, void *stream) {
    return emit_common(n_jobs, jobs, ws, ws_bytes, stream, false);
}

}  // extern "C"

namespace pct {
// Device memory of pct_wepl_static: one array per GPU the library runs on, held until the
// process ends.  Its address on a device comes from hipGetSymbolAddress with that device
// current; host code uses only that address (the array's name is a host-side stand-in).
constexpr size_t STATIC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int STATIC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[STATIC_MAX_DEVICES];

// The scratch address on the device of `stream` (NULL: the current device), looked up
// once per device.
static pct_status static_scratch(hipStream_t stream, void **out) {
    int cur = 0, dev = 0;
    if (hipGetDevice(&cur) != hipSuccess) return PCT_EHIP;
    dev = cur;
    if (stream) {
        hipDevice_t d = 0;
        if (hipStreamGetDevice(stream, &d) != hipSuccess) return PCT_EHIP;
        dev = (int)d;
    }
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return PCT_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur && hipSetDevice(dev) != hipSuccess) return PCT_EHIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return PCT_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PCT_OK;
}

// The status word of a workspace into the caller's int32 (PCT_OK when h is NULL).
__global__ void k_copy_status(const WsHeader *h, int32_t *dst) {
    if (threadIdx.x == 0) *dst = h ? h->status : PCT_OK;
}
}  // namespace pct

extern "C" {

pct_status pct_wepl_static(int32_t n_jobs, const pct_job *jobs, int32_t *status_dev, void *stream) {
    pct_status st = check_jobs(n_jobs, jobs, false, true);
    if (st != PCT_OK) return st;
    if (n_jobs > HostJobs::FIXED) return PCT_ESCRATCH;
    int64_t rc[HostJobs::FIXED];
    for (int j = 0; j < n_jobs; ++j) rc[j] = jobs[j].beam->row_count;
    if (layout_of(n_jobs, rc).total > STATIC_SCRATCH_BYTES) return PCT_ESCRATCH;
    void *ws = nullptr;
    st = static_scratch((hipStream_t)stream, &ws);
    if (st != PCT_OK) return st;
    st = emit_common(n_jobs, jobs, ws, STATIC_SCRATCH_BYTES, stream, false, false);
    if (st != PCT_OK) return st;
    if (status_dev) {
        // (with no job the status word was not cleared: report OK without reading it)
        if (n_jobs == 0) hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, (hipStream_t)stream,
                                            (const WsHeader *)nullptr, status_dev);
        else hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, (hipStream_t)stream, (const WsHeader *)ws,
                                status_dev);
    }
    return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
}

pct_status pct_set_launch_config(const pct_launch_config *cfg) {
    if (!cfg) {
        g_cfg = DEFAULT_CFG;
        return PCT_OK;
    }
    if (!config_ok(*cfg)) return PCT_EINVAL;
    g_cfg = *cfg;
    return PCT_OK;
}

pct_status pct_get_launch_config(pct_launch_config *cfg) {
    if (!cfg) return PCT_EINVAL;
    *cfg = g_cfg;
    return PCT_OK;
}

pct_status pct_autotune(int32_t n_jobs, const pct_job *jobs, void *ws, size_t ws_bytes, int64_t *nnz_total_dev,
                        void *stream, pct_launch_config *best) {
    if (!best) return PCT_EINVAL;
    pct_status st = check_jobs(n_jobs, jobs, true, false);
    if (st != PCT_OK) return st;
    const pct_launch_config saved = g_cfg;
    hipStream_t s = (hipStream_t)stream;
    uint64_t key = 0;
    const bool keyed = tune_key(n_jobs, jobs, key);
    pct_launch_config cached;
    if (keyed && tune_lookup(key, cached)) {
        g_cfg = cached;
        st = pct_count_rows(n_jobs, jobs, ws, ws_bytes, nnz_total_dev, stream);
        if (st == PCT_OK) st = pct_emit_csr(n_jobs, jobs, ws, ws_bytes, stream);   // final outputs
        if (st != PCT_OK) g_cfg = saved;
        *best = g_cfg;
        return st;
    }
    st = pct_count_rows(n_jobs, jobs, ws, ws_bytes, nnz_total_dev, stream);
    if (st != PCT_OK) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PCT_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PCT_EHIP;
    }
    const int rpws[3] = {16, 32, 64};
    const int orders[2] = {PCT_ORDER_GIVEN, PCT_ORDER_LPT};
    const int bpcs[2] = {0, 4};
    float best_ms = -1.f;
    pct_launch_config pick = saved;
    for (int q = 0; q < 2 && st == PCT_OK; ++q) {
        for (int o = 0; o < 2 && st == PCT_OK; ++o) {
            for (int r = 0; r < 3 && st == PCT_OK; ++r) {
                g_cfg = pct_launch_config{rpws[r], orders[o], bpcs[q]};
                float ms = 0.f;
                for (int rep = 0; rep < 2 && st == PCT_OK; ++rep) {
                    if (hipEventRecord(e0, s) != hipSuccess) st = PCT_EHIP;
                    if (st == PCT_OK) st = pct_emit_csr(n_jobs, jobs, ws, ws_bytes, stream);
                    if (st == PCT_OK && hipEventRecord(e1, s) != hipSuccess) st = PCT_EHIP;
                    if (st == PCT_OK && hipEventSynchronize(e1) != hipSuccess) st = PCT_EHIP;
                    if (st == PCT_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = PCT_EHIP;
                }
                if (st == PCT_OK && (best_ms < 0.f || ms < best_ms)) {
                    best_ms = ms;
                    pick = g_cfg;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_cfg = (st == PCT_OK) ? pick : saved;
    if (st == PCT_OK) st = pct_emit_csr(n_jobs, jobs, ws, ws_bytes, stream);   // final outputs
    if (st == PCT_OK && keyed) tune_store(key, g_cfg);
    *best = g_cfg;
    return st;
}

pct_status pct_autotune_cached(int32_t n_jobs, const pct_job *jobs, pct_launch_config *cfg, int32_t *found) {
    if (!cfg || !found) return PCT_EINVAL;
    *found = 0;
    const pct_status st = check_jobs(n_jobs, jobs, false, false);
    if (st != PCT_OK) return st;
    uint64_t key = 0;
    if (!tune_key(n_jobs, jobs, key)) return PCT_EHIP;
    pct_launch_config c;
    if (tune_lookup(key, c)) {
        *cfg = c;
        *found = 1;
    }
    return PCT_OK;
}

pct_status pct_autotune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    g_tune.map.clear();
    g_tune.loaded = true;   // the file, if any, is not read again
    return PCT_OK;
}

}  // extern "C"

struct pct_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

pct_status pct_graph_create_sets(int32_t n_sets, const int32_t *set_sizes, const pct_job *jobs, int32_t build_x,
                                 void *ws, size_t ws_bytes, int64_t *nnz_total_dev, pct_graph *graph) {
    if (!graph) return PCT_EINVAL;
    *graph = nullptr;
    if (n_sets < 1 || !set_sizes) return PCT_EINVAL;
    int64_t total = 0;
    for (int k = 0; k < n_sets; ++k) {
        if (set_sizes[k] < 0) return PCT_EINVAL;
        total += set_sizes[k];
    }
    if (total > INT32_MAX) return PCT_ERANGE;
    if (total > 0 && (!jobs || !nnz_total_dev)) return PCT_EINVAL;
    for (int64_t k = 0, off = 0; k < n_sets; off += set_sizes[k], ++k) {
        const pct_status st = check_jobs(set_sizes[k], jobs + off, true, false);
        if (st != PCT_OK) return st;
    }
    if (build_x) {
        for (int64_t j = 0; j < total; ++j)
            if (!jobs[j].x_dev) return PCT_EINVAL;
    }
    // The count pass does not read x, so the phantom builds form branches of their own
    // (streams b[0 .. NB-1], forked from and joined back into the capture stream s) that
    // run beside the first set's count pass; its emit, which gathers x, waits for all of
    // them.  The builds are dealt round-robin over the branches: one chain of small
    // launches would outlast the count pass.  The sets follow one another on s: count,
    // then emit, each into its own slice of nnz_total_dev.
    constexpr int NB = 4;
    pct_status st = PCT_OK;
    hipStream_t s = nullptr, b[NB] = {};
    hipEvent_t fork = nullptr, join[NB] = {};
    bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < NB && ok; ++i)
        ok = hipStreamCreateWithFlags(&b[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&join[i], hipEventDisableTiming) == hipSuccess;
    bool capturing = ok && hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (!capturing) st = PCT_EHIP;
    int nb = 0;   // branches in use
    if (st == PCT_OK && build_x) {
        if (hipEventRecord(fork, s) != hipSuccess) st = PCT_EHIP;
        std::vector<const float *> done;
        for (int64_t j = 0; j < total && st == PCT_OK; ++j) {
            const float *x = jobs[j].x_dev;
            if (std::find(done.begin(), done.end(), x) != done.end()) continue;
            const int i = (int)(done.size() % NB);
            done.push_back(x);
            if (i >= nb) {
                if (hipStreamWaitEvent(b[i], fork, 0) != hipSuccess) st = PCT_EHIP;
                nb = i + 1;
            }
            if (st == PCT_OK) st = pct_phantom_build(jobs[j].phantom, const_cast<float *>(x), b[i]);
        }
    }
    for (int64_t k = 0, off = 0; k < n_sets && st == PCT_OK; off += set_sizes[k], ++k) {
        st = count_common(set_sizes[k], jobs + off, ws, ws_bytes, nnz_total_dev + off, s, k == 0);
        for (int i = 0; i < nb && k == 0 && st == PCT_OK; ++i)
            if (hipEventRecord(join[i], b[i]) != hipSuccess || hipStreamWaitEvent(s, join[i], 0) != hipSuccess)
                st = PCT_EHIP;
        if (st == PCT_OK) st = pct_emit_csr(set_sizes[k], jobs + off, ws, ws_bytes, s);
    }
    // a failed capture still has to be ended; branches forked from it must be joined
    // for the end to succeed, which a failure above may have left undone (the graph is
    // then discarded)
    for (int i = 0; i < nb && st != PCT_OK && capturing; ++i)
        if (hipEventRecord(join[i], b[i]) == hipSuccess) (void)hipStreamWaitEvent(s, join[i], 0);
    hipGraph_t g = nullptr;
    const hipError_t ec = capturing ? hipStreamEndCapture(s, &g) : hipSuccess;
    for (int i = 0; i < NB; ++i) {
        if (join[i]) (void)hipEventDestroy(join[i]);
        if (b[i]) (void)hipStreamDestroy(b[i]);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (s) (void)hipStreamDestroy(s);
    if (st == PCT_OK && ec != hipSuccess) st = PCT_EHIP;
    if (st != PCT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return PCT_EHIP;
    }
    pct_graph h = new pct_graph_s;
    h->graph = g;
    h->exec = e;
    *graph = h;
    return PCT_OK;
}

pct_status pct_graph_create(int32_t n_jobs, const pct_job *jobs, int32_t build_x, void *ws, size_t ws_bytes,
                            int64_t *nnz_total_dev, pct_graph *graph) {
    if (n_jobs < 0) return PCT_EINVAL;
    return pct_graph_create_sets(1, &n_jobs, jobs, build_x, ws, ws_bytes, nnz_total_dev, graph);
}

pct_status pct_graph_launch(pct_graph graph, void *stream) {
    if (!graph || !graph->exec) return PCT_EINVAL;
    return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? PCT_OK : PCT_EHIP;
}

pct_status pct_graph_destroy(pct_graph graph) {
    if (!graph) return PCT_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return PCT_OK;
}

pct_status pct_device_status(const void *ws, void *stream) {
    if (!ws) return PCT_EWORKSPACE;
    int32_t v = PCT_OK;
    if (hipMemcpyAsync(&v, ws, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess) return PCT_EHIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PCT_EHIP;
    return v;
}

}  // extern "C"
