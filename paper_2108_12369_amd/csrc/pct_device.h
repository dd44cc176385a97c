// pct_device.h -- device-side building blocks of the proton-CT hot path (gfx950).
//
// Per proton (one lane per row): decode the row into (angle, proton id), draw its
// random numbers from a counter-based Philox4x32-10 stream, rotate the beam frame
// (t, v, u) into the fixed frame (x, y, z) [Sec. II-C, Givens rotation], solve entry and
// exit against the outer boundary [Sec. II-B], build a straight or cubic-spline path
// with Gaussian scattering [Sec. II-B], and walk the voxels it crosses with a
// digital-difference traversal [Sec. II-C].  The walker feeds a "sink" that either
// counts CSR entries or emits them (column, length) and accumulates the WEPL.
//
// Geometry type R is double for the mixed-precision form (FP64 positions and face
// ordering, lengths rounded once to FP32) and float for the plain FP32 form.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/pct.h"

namespace pct {

// First error wins: the status word keeps the first non-OK code written to it.
__device__ __forceinline__ void set_status_dev(int32_t *status, int32_t code) {
    atomicCAS(status, PCT_OK, code);
}

// --------------------------------------------------------------- job descriptor
// Flattened, device-resident form of one pct_job (host fills it, a kernel stores it
// in the workspace).  Everything a lane needs for any row of the job.
struct JobDev {
    int32_t dim, path, val_dtype, outer_axes;
    int32_t n[3];
    int32_t K;
    double h[3], invh[3], o[3], top[3];
    double oc[3], inv_s2[3];          // outer boundary: center, 1/semi^2
    uint64_t seed;
    double angle0, dangle;
    int64_t P, row_begin, row_count;
    double t_lo, t_span, v_lo, v_span;
    double sig_in, sig_out, sig_lat, rho, crho, step, noise;
    const float *x;
    int64_t *row_ptr;
    int32_t *cols;
    void *vals;
    float *b;
    int64_t cap;
    int64_t count_off;   // first element of this job in the workspace count array
    int64_t tile_base;   // first tile of this job (count pass: TILE rows per tile)
    int64_t n_tiles;
    int64_t etile_base;  // first emit tile of this job (emit tiles are laid out in the
    int64_t n_etiles;    // launch order of the jobs, 4 * rpw rows each)
    int32_t rpw;         // rows per wavefront in the emit pass
    int32_t nmax;        // largest n[d]
    int32_t highland;    // exit pair widths per proton from Highland's formula
    float chord;         // > 0: the stored value of every entry (constant chord length)
    double hl_k;         // Highland: 13.6 MeV / (beta c p)
    double hl_x0inv;     // Highland: 1 / X0 (1/mm)
    double hl_lnb2;      // Highland: ln(beta^2)
    double orot[2];      // outer boundary turned by its angle: cosine, sine
    int32_t orot_on;     // the outer boundary is turned
    int32_t pad2_;
    // 3D jobs: a copy of x in bricks of 8 x 8 x 1 voxels (in the workspace) that the b
    // gathers of the wave emit read; null when the job has none.  nbx, nby: bricks per
    // grid row and per plane.
    float *xb;
    int32_t nbx, nby;
};

// ------------------------------------------------------------------ math helpers
template <typename R> __device__ __forceinline__ R r_floor(R v) {
    if constexpr (std::is_same<R, float>::value) return floorf(v); else return floor(v);
}
template <typename R> __device__ __forceinline__ R r_ceil(R v) {
    if constexpr (std::is_same<R, float>::value) return ceilf(v); else return ceil(v);
}
template <typename R> __device__ __forceinline__ R r_sqrt(R v) {
    if constexpr (std::is_same<R, float>::value) return sqrtf(v); else return sqrt(v);
}
template <typename R> __device__ __forceinline__ R r_log(R v) {
    if constexpr (std::is_same<R, float>::value) return logf(v); else return log(v);
}
template <typename R> __device__ __forceinline__ R r_tan(R v) {
    if constexpr (std::is_same<R, float>::value) return tanf(v); else return tan(v);
}
template <typename R> __device__ __forceinline__ R r_fma(R a, R b, R c) {
    if constexpr (std::is_same<R, float>::value) return fmaf(a, b, c); else return fma(a, b, c);
}
template <typename R> __device__ __forceinline__ void r_sincos(R v, R *s, R *c) {
    if constexpr (std::is_same<R, float>::value) sincosf(v, s, c); else sincos(v, s, c);
}
template <typename R> __device__ __forceinline__ R r_inf() {
    if constexpr (std::is_same<R, float>::value) return __builtin_huge_valf(); else return __builtin_huge_val();
}

// --------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32x32->64-bit
// products on counter words 0 and 2 with the published multipliers, high halves mixed
// into the other two words with the round key, the key advanced by the published Weyl
// increments after each round.
__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a_lo = 0xD2511F53u * c0, a_hi = __umulhi(0xD2511F53u, c0);
        const uint32_t b_lo = 0xCD9E8D57u * c2, b_hi = __umulhi(0xCD9E8D57u, c2);
        const uint32_t x0 = b_hi ^ c1 ^ k0;
        const uint32_t x2 = a_hi ^ c3 ^ k1;
        c0 = x0;
        c1 = b_lo;
        c2 = x2;
        c3 = a_lo;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Draw `draw` of `stream` for proton g as two 64-bit words.
__device__ __forceinline__ void draw2(uint64_t seed, uint32_t stream, uint64_t g, uint32_t draw,
                                      uint64_t &w0, uint64_t &w1) {
    uint32_t c0 = draw, c1 = stream, c2 = (uint32_t)g, c3 = (uint32_t)(g >> 32);
    philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    w0 = (uint64_t)c0 | ((uint64_t)c1 << 32);
    w1 = (uint64_t)c2 | ((uint64_t)c3 << 32);
}

// Uniform in [0, 1): top 53 bits (FP64) or top 24 bits (FP32) of a word.
template <typename R> __device__ __forceinline__ R unit_uniform(uint64_t w) {
    if constexpr (std::is_same<R, float>::value) return (float)(uint32_t)(w >> 40) * 0x1.0p-24f;
    else return (double)(w >> 11) * 0x1.0p-53;
}

// Marsaglia polar method: attempt a uses draw a; 64 rejections in a row give (0, 0).
template <typename R>
__device__ __forceinline__ void normal_pair(uint64_t seed, uint32_t stream, uint64_t g, R &z1, R &z2) {
    for (uint32_t a = 0; a < 64; ++a) {
        uint64_t w0, w1;
        draw2(seed, stream, g, a, w0, w1);
        const R v1 = R(2) * unit_uniform<R>(w0) - R(1);
        const R v2 = R(2) * unit_uniform<R>(w1) - R(1);
        const R s = v1 * v1 + v2 * v2;
        if (s > R(0) && s < R(1)) {
            const R f = r_sqrt<R>(R(-2) * r_log<R>(s) / s);
            z1 = v1 * f;
            z2 = v2 * f;
            return;
        }
    }
    z1 = R(0);
    z2 = R(0);
}

// ---------------------------------------------------------------------- geometry
// Projection angle k: exact cosine/sine at multiples of 90 degrees.
template <typename R>
__device__ __forceinline__ void beam_angle(const JobDev &J, int32_t k, R &c, R &s) {
    const R phi = R(J.angle0) + R(k) * R(J.dangle);
    const R q = phi / R(90);
    if (r_floor<R>(q) == q) {
        int m = (int)(q - R(4) * r_floor<R>(q / R(4)));
        c = (m == 0) ? R(1) : (m == 2) ? R(-1) : R(0);
        s = (m == 1) ? R(1) : (m == 3) ? R(-1) : R(0);
        return;
    }
    r_sincos<R>(phi * (R(3.14159265358979323846) / R(180)), &s, &c);
}

// Line Q + l d against the outer boundary; stable roots, l1 < l2; false if no chord.
template <typename R, int DIM>
__device__ __forceinline__ bool boundary_hit(const JobDev &J, const R Q[3], const R d[3], R &l1, R &l2) {
    R a = R(0), b = R(0), c = R(-1);
    const int na = (DIM == 3 && J.outer_axes == 3) ? 3 : 2;
    R qv[3], dv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        qv[i] = Q[i] - R(J.oc[i]);
        dv[i] = d[i];
    }
    if (J.orot_on) {
        // into the frame of the turned ellipse (x-y rotation by minus its angle)
        const R cr = R(J.orot[0]), sr = R(J.orot[1]);
        const R q0 = cr * qv[0] + sr * qv[1], q1 = cr * qv[1] - sr * qv[0];
        const R d0 = cr * dv[0] + sr * dv[1], d1 = cr * dv[1] - sr * dv[0];
        qv[0] = q0;
        qv[1] = q1;
        dv[0] = d0;
        dv[1] = d1;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i < na) {
            const R q = qv[i];
            const R w = R(J.inv_s2[i]);
            a += dv[i] * dv[i] * w;
            b += q * dv[i] * w;
            c += q * q * w;
        }
    }
    const R disc = b * b - a * c;
    if (!(a > R(0)) || !(disc > R(0))) return false;
    const R sq = r_sqrt<R>(disc);
    const R t = (b >= R(0)) ? -(b + sq) : (sq - b);
    R r1 = t / a, r2 = c / t;
    l1 = r1 < r2 ? r1 : r2;
    l2 = r1 < r2 ? r2 : r1;
    return true;
}

template <typename R> __device__ __forceinline__ void normalize3(R v[3]) {
    const R n = r_sqrt<R>(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n;
    v[1] /= n;
    v[2] /= n;
}

template <typename R>
__device__ __forceinline__ int vox_index(R p, double o, double invh, int n) {
    R f = r_floor<R>((p - R(o)) * R(invh));
    f = f < R(0) ? R(0) : f;
    f = f > R(n - 1) ? R(n - 1) : f;
    return (int)f;
}

// Unclamped floor index (inside-the-box test of sample points).
template <typename R>
__device__ __forceinline__ R vox_floor(R p, double o, double invh) {
    return r_floor<R>((p - R(o)) * R(invh));
}

template <int DIM>
__device__ __forceinline__ int32_t col_of(const JobDev &J, const int i[3]) {
    return DIM == 3 ? i[0] + J.n[0] * (i[1] + J.n[1] * i[2]) : i[0] + J.n[0] * i[1];
}

// ------------------------------------------------------------------------- sinks
// Count sink: number of CSR entries; the first voxel of a segment that equals the
// previous entry is merged with it (same voxel across a joint of the path).
struct CountSink {
    int64_t n = 0;
    int32_t last = -1;
};

// Emit sink: the pending entry is held until the next distinct voxel so that joints
// merge; its x value is fetched when the entry opens and consumed when it closes, so
// the gather latency overlaps the walk.  Lengths are FP32, stored as FP32 or FP16 at
// [pos, end); the WEPL is accumulated in TW.
template <typename R, typename TW>
struct EmitSink {
    int32_t *cols;
    void *vals;
    const float *x;
    int64_t pos, end;
    int32_t pcol = -1;
    float plen = 0.0f;
    float px = 0.0f;
    TW wepl = TW(0);
    float chord = 0.0f;   // > 0: stored instead of the length (b keeps the length)
    bool store, half, want_b;

    __device__ __forceinline__ void flush() {
        if (pcol >= 0) {
            if (want_b) wepl += (TW)plen * (TW)px;
            if (store && pos < end) {
                const float sv = chord > 0.0f ? chord : plen;
                cols[pos] = pcol;
                if (half) ((__half *)vals)[pos] = __float2half_rn(sv);
                else ((float *)vals)[pos] = sv;
            }
            ++pos;
        }
    }
    __device__ __forceinline__ void put(bool first, int32_t col, float len) {
        if (first && col == pcol) {
            plen += len;
            return;
        }
        flush();
        pcol = col;
        plen = len;
        if (want_b) px = x[col];
    }
};

template <class S> struct is_count : std::false_type {};
template <> struct is_count<CountSink> : std::true_type {};

// ------------------------------------------------------------------ the traversal
// Clip A + l D, l in [lo, hi], to the grid box (slab test).  False if it misses.
template <typename R, int DIM>
__device__ __forceinline__ bool clip_box(const JobDev &J, const R A[3], const R D[3], R &lo, R &hi) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        if (D[d] != R(0)) {
            const R t1 = (R(J.o[d]) - A[d]) / D[d];
            const R t2 = (R(J.top[d]) - A[d]) / D[d];
            lo = fmax(lo, fmin(t1, t2));
            hi = fmin(hi, fmax(t1, t2));
        } else if (A[d] < R(J.o[d]) || A[d] > R(J.top[d])) {
            return false;
        }
    }
    return lo < hi;
}

// Walk from P (parameter lo) to E (parameter hi) along A + l D.  The step count per
// axis is fixed by the voxel indices of P and E; the order of the face crossings is
// decided by their parameters l = (face - A_d) / D_d (one reciprocal per axis).
template <typename R, int DIM, class S>
__device__ __forceinline__ void walk(const JobDev &J, const R A[3], const R D[3], R lo, R hi,
                                     const R P[3], const R E[3], S &s) {
    int i[3] = {0, 0, 0}, e[3] = {0, 0, 0}, st[3] = {0, 0, 0}, bud[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        i[d] = vox_index<R>(P[d], J.o[d], J.invh[d], J.n[d]);
        e[d] = vox_index<R>(E[d], J.o[d], J.invh[d], J.n[d]);
        bud[d] = abs(e[d] - i[d]);
        st[d] = e[d] > i[d] ? 1 : -1;
    }
    if constexpr (is_count<S>::value) {
        int64_t c = 1;
#pragma unroll
        for (int d = 0; d < DIM; ++d) c += bud[d];
        if (col_of<DIM>(J, i) == s.last) c -= 1;
        s.n += c;
        s.last = col_of<DIM>(J, e);
    } else {
        R dn2 = R(0);
        R inv[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            dn2 += D[d] * D[d];
            inv[d] = (bud[d] > 0 && D[d] != R(0)) ? R(1) / D[d] : R(0);
        }
        const R Dn = r_sqrt<R>(dn2);
        R lp = lo;
        bool first = true;
        for (;;) {
            int a = -1;
            R la = R(0);
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (bud[d] > 0) {
                    const R plane = R(J.o[d]) + R(i[d] + (st[d] > 0 ? 1 : 0)) * R(J.h[d]);
                    const R ld = (D[d] != R(0)) ? (plane - A[d]) * inv[d] : r_inf<R>();
                    if (a < 0 || ld < la) {
                        a = d;
                        la = ld;
                    }
                }
            }
            if (a < 0) break;
            R lc = la > lp ? la : lp;
            lc = lc < hi ? lc : hi;
            s.put(first, col_of<DIM>(J, i), (float)((lc - lp) * Dn));
            first = false;
            lp = lc;
            if (a == 0) { i[0] += st[0]; bud[0] -= 1; }
            else if (a == 1) { i[1] += st[1]; bud[1] -= 1; }
            else { i[2] += st[2]; bud[2] -= 1; }
        }
        s.put(first, col_of<DIM>(J, i), (float)((hi - lp) * Dn));
    }
}

// General segment: clip to the box, then walk.  B (optional) is the exact end point
// used when the upper end is not clipped.
template <typename R, int DIM, class S>
__device__ __forceinline__ void segment(const JobDev &J, const R A[3], const R D[3], R lo, R hi,
                                        const R *B, S &s) {
    const R hi0 = hi;
    if (!clip_box<R, DIM>(J, A, D, lo, hi)) return;
    R P[3] = {R(0), R(0), R(0)}, E[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        P[d] = A[d] + lo * D[d];
        E[d] = (hi == hi0 && B) ? B[d] : A[d] + hi * D[d];
    }
    walk<R, DIM>(J, A, D, lo, hi, P, E, s);
}

// Position of the previous spline sample and its voxel, carried from chord to chord.
template <typename R>
struct ChordState {
    R A[3];
    R fa[3];       // unclamped floor((A - o) / h) per axis
    bool a_in;     // A lies in the grid box
    int32_t ca;    // column of A's voxel (when a_in)
};

template <typename R, int DIM>
__device__ __forceinline__ void chord_start(const JobDev &J, const R P0[3], ChordState<R> &c) {
    c.a_in = true;
    int i[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c.A[d] = P0[d];
        c.fa[d] = R(0);
        if (d < DIM) {
            c.fa[d] = vox_floor<R>(P0[d], J.o[d], J.invh[d]);
            c.a_in = c.a_in && (c.fa[d] >= R(0)) && (c.fa[d] <= R(J.n[d] - 1));
            i[d] = (int)c.fa[d];
        }
    }
    c.ca = c.a_in ? col_of<DIM>(J, i) : -1;
}

// Chord from the carried sample A to the new sample B.  When both lie in the box no
// clipping can move them: the walk starts at A's voxel and takes |i_d(B) - i_d(A)|
// steps per axis, ordered by comparing the crossing parameters cross-multiplied in R
// (no division); the lengths of the pieces are formed in FP32.
template <typename R, int DIM, class S>
__device__ __forceinline__ void chord_to(const JobDev &J, ChordState<R> &c, const R B[3], S &s) {
    R fb[3] = {R(0), R(0), R(0)};
    bool b_in = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        fb[d] = vox_floor<R>(B[d], J.o[d], J.invh[d]);
        b_in = b_in && (fb[d] >= R(0)) && (fb[d] <= R(J.n[d] - 1));
    }
    int ib[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) ib[d] = (int)fb[d];
    const int32_t cb = b_in ? col_of<DIM>(J, ib) : -1;
    if (c.a_in && b_in) {
        int ia[3] = {0, 0, 0}, bud[3] = {0, 0, 0}, st[3] = {0, 0, 0};
        int tot = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            ia[d] = (int)c.fa[d];
            bud[d] = abs(ib[d] - ia[d]);
            st[d] = ib[d] > ia[d] ? 1 : -1;
            tot += bud[d];
        }
        if constexpr (is_count<S>::value) {
            s.n += tot + (c.ca != s.last ? 1 : 0);
            s.last = cb;
        } else {
            R D[3] = {R(0), R(0), R(0)};
            float Df[3] = {0.f, 0.f, 0.f};
            float dn2 = 0.f;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                D[d] = B[d] - c.A[d];
                Df[d] = (float)D[d];
                dn2 = fmaf(Df[d], Df[d], dn2);
            }
            const float len = __builtin_amdgcn_sqrtf(dn2);
            if (tot == 0) {
                s.put(true, c.ca, len);
            } else {
                float lp = 0.f;
                bool first = true;
                int32_t ci = c.ca;
                while (tot > 0) {
                    // axis of the nearest crossing: l_d = |face_d - A_d| / |D_d|
                    int a = -1;
                    R na = R(0), da = R(1);
#pragma unroll
                    for (int d = 0; d < DIM; ++d) {
                        if (bud[d] > 0) {
                            const R plane = R(J.o[d]) + R(ia[d] + (st[d] > 0 ? 1 : 0)) * R(J.h[d]);
                            const R nd = plane - c.A[d];
                            const R ad = D[d] < R(0) ? -D[d] : D[d];
                            const R an = nd < R(0) ? -nd : nd;
                            if (a < 0 || an * da < na * ad) {
                                a = d;
                                na = an;
                                da = ad;
                            }
                        }
                    }
                    float lc = (float)na * __builtin_amdgcn_rcpf((float)da);
                    lc = lc > lp ? lc : lp;
                    lc = lc < 1.f ? lc : 1.f;
                    s.put(first, ci, (lc - lp) * len);
                    first = false;
                    lp = lc;
                    if (a == 0) { ia[0] += st[0]; bud[0] -= 1; }
                    else if (a == 1) { ia[1] += st[1]; bud[1] -= 1; }
                    else { ia[2] += st[2]; bud[2] -= 1; }
                    --tot;
                    ci = col_of<DIM>(J, ia);
                }
                s.put(first, ci, (1.f - lp) * len);
            }
        }
    } else {
        R D[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int d = 0; d < DIM; ++d) D[d] = B[d] - c.A[d];
        segment<R, DIM>(J, c.A, D, R(0), R(1), B, s);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c.A[d] = B[d];
        c.fa[d] = fb[d];
    }
    c.a_in = b_in;
    c.ca = cb;
}

// ------------------------------------------------------------------------ one row
// Geometry of proton g's path [Sec. II-B]: a straight line (Q, u) or, for a spline path
// that meets the outer boundary, entry P0 with direction d0, exit P1 with direction d1
// and the power basis c1..c3 of the cubic Hermite curve (origin P0), N chords.
template <typename R>
struct PathGeom {
    bool curved;
    R Q[3], u[3];
    R P0[3], d0[3], P1[3], d1[3];
    R c1[3], c2[3], c3[3];
    R L, invN;
    int32_t N;
};

template <typename R, int DIM, bool CURVED>
__device__ __forceinline__ void make_path(const JobDev &J, int64_t g, PathGeom<R> &p) {
    const int32_t k = (int32_t)(((g + 1) * (int64_t)J.K - 1) / J.P);
    R c, sn;
    beam_angle<R>(J, k, c, sn);
    const R u[3] = {c, sn, R(0)};
    const R th[3] = {-sn, c, R(0)};
    uint64_t w0, w1;
    draw2(J.seed, 0, (uint64_t)g, 0, w0, w1);
    const R t = R(J.t_lo) + R(J.t_span) * unit_uniform<R>(w0);
    const R v = (DIM == 3) ? R(J.v_lo) + R(J.v_span) * unit_uniform<R>(w1) : R(0);
    p.Q[0] = t * th[0];
    p.Q[1] = t * th[1];
    p.Q[2] = v;
    p.u[0] = u[0];
    p.u[1] = u[1];
    p.u[2] = u[2];
    p.curved = false;
    if constexpr (CURVED) {
        R zt, zv;
        normal_pair<R>(J.seed, 1, (uint64_t)g, zt, zv);
        const R tti = r_tan<R>(R(J.sig_in) * zt);
        const R tvi = (DIM == 3) ? r_tan<R>(R(J.sig_in) * zv) : R(0);
        R d0[3] = {u[0] + tti * th[0], u[1] + tti * th[1], tvi};
        normalize3<R>(d0);
        R l1, l2;
        if (!boundary_hit<R, DIM>(J, p.Q, d0, l1, l2)) {
            // misses the phantom: straight along the entry direction
            p.u[0] = d0[0];
            p.u[1] = d0[1];
            p.u[2] = d0[2];
            return;
        }
        p.curved = true;
        R P0[3], P1[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            P0[i] = p.Q[i] + l1 * d0[i];
            P1[i] = p.Q[i] + l2 * d0[i];
        }
        R z1, z2;
        normal_pair<R>(J.seed, 2, (uint64_t)g, z1, z2);
        R crho = R(J.crho), rho = R(J.rho), sig_lat = R(J.sig_lat), sig_out = R(J.sig_out);
        if (J.highland) {
            // Highland's width for the straight entry line's length inside the outer
            // boundary, and the exit pair of a uniform slab of that thickness [Sec. II-B]
            const R x = l2 - l1;
            const R u = x * R(J.hl_x0inv);
            R th0 = R(0);
            if (u > R(0)) {
                const R br = R(1) + R(0.038) * (r_log<R>(u) - R(J.hl_lnb2));
                th0 = br > R(0) ? R(J.hl_k) * r_sqrt<R>(u) * br : R(0);
            }
            sig_out = th0;
            sig_lat = th0 * x * R(0.57735026918962576451);   // 1/sqrt(3)
            rho = R(0.86602540378443864676);                  // sqrt(3)/2
            crho = R(0.5);
        }
        const R lat_t = sig_lat * z1;
        const R ang_t = sig_out * (rho * z1 + crho * z2);
        R lat_v = R(0), ang_v = R(0);
        if (DIM == 3) {
            normal_pair<R>(J.seed, 3, (uint64_t)g, z1, z2);
            lat_v = sig_lat * z1;
            ang_v = sig_out * (rho * z1 + crho * z2);
        }
        const R tdot = th[0] * d0[0] + th[1] * d0[1];
        R nt[3] = {th[0] - tdot * d0[0], th[1] - tdot * d0[1], -tdot * d0[2]};
        normalize3<R>(nt);
        R nv[3] = {R(0), R(0), R(0)};
        if (DIM == 3) {
            const R vdot = d0[2];
            nv[0] = -vdot * d0[0];
            nv[1] = -vdot * d0[1];
            nv[2] = R(1) - vdot * d0[2];
            normalize3<R>(nv);
        }
        R Qd[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) Qd[i] = p.Q[i] + lat_t * nt[i] + lat_v * nv[i];
        R m1, m2;
        if (boundary_hit<R, DIM>(J, Qd, d0, m1, m2)) {
#pragma unroll
            for (int i = 0; i < 3; ++i) P1[i] = Qd[i] + m2 * d0[i];
        }
        const R tto = r_tan<R>(ang_t), tvo = r_tan<R>(ang_v);
        R d1[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) d1[i] = d0[i] + tto * nt[i] + tvo * nv[i];
        normalize3<R>(d1);

        R dP[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) dP[i] = P1[i] - P0[i];
        const R L = r_sqrt<R>(dP[0] * dP[0] + dP[1] * dP[1] + dP[2] * dP[2]);
        const R steps = L / R(J.step);
        int32_t N = (int32_t)r_ceil<R>(steps);
        p.N = N < 1 ? 1 : N;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            p.P0[i] = P0[i];
            p.P1[i] = P1[i];
            p.d0[i] = d0[i];
            p.d1[i] = d1[i];
            p.c1[i] = L * d0[i];
            p.c2[i] = R(3) * dP[i] - R(2) * L * d0[i] - L * d1[i];
            p.c3[i] = R(-2) * dP[i] + L * d0[i] + L * d1[i];
        }
        p.L = L;
        p.invN = R(1) / R(p.N);
    }
}

template <typename R, int DIM>
__device__ __forceinline__ void spline_point(const PathGeom<R> &p, int32_t j, R B[3]) {
    const R sj = R(j) * p.invN;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        B[i] = (i < DIM) ? r_fma<R>(r_fma<R>(r_fma<R>(p.c3[i], sj, p.c2[i]), sj, p.c1[i]), sj, p.P0[i]) : R(0);
}

template <typename R, int DIM, bool CURVED, class S>
__device__ __forceinline__ void trace_row(const JobDev &J, int64_t g, S &s) {
    PathGeom<R> p;
    make_path<R, DIM, CURVED>(J, g, p);
    const R ninf = -r_inf<R>(), pinf = r_inf<R>();
    if (!p.curved) {
        segment<R, DIM>(J, p.Q, p.u, ninf, pinf, (const R *)nullptr, s);
        return;
    }
    segment<R, DIM>(J, p.P0, p.d0, ninf, R(0), (const R *)nullptr, s);
    ChordState<R> cs;
    chord_start<R, DIM>(J, p.P0, cs);
    for (int32_t j = 1; j < p.N; ++j) {
        R B[3];
        spline_point<R, DIM>(p, j, B);
        chord_to<R, DIM>(J, cs, B, s);
    }
    chord_to<R, DIM>(J, cs, p.P1, s);
    segment<R, DIM>(J, p.P1, p.d1, R(0), pinf, (const R *)nullptr, s);
}

template <typename R, class S>
__device__ __forceinline__ void trace_any(const JobDev &J, int64_t g, S &s) {
    if (J.dim == 3) {
        if (J.path == 1) trace_row<R, 3, true>(J, g, s);
        else trace_row<R, 3, false>(J, g, s);
    } else {
        if (J.path == 1) trace_row<R, 2, true>(J, g, s);
        else trace_row<R, 2, false>(J, g, s);
    }
}

}  // namespace pct
