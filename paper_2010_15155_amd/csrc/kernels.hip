// HIP kernels (gfx950) of the kernel aggregated FMM evaluation pass.
//
// Layouts (all leaf-sorted, normalised coordinates in [0,1)^3):
//   source record  float[R]: xh yh zh xl yl zl v...   (hi/lo split of FP64)
//   target record  float[8]: xh yh zh 0 xl yl zl 0
//   box geometry   double4 : cx cy cz h
//   densities      float  [box][ncomp][Mp]   (Mp = M rounded up to 32, padding 0)
//   check values   double [box][ncomp][M]
//   target values  double [n_trg][NACC]       (near and far parts separately)
// A target chunk is up to 256 targets of one leaf; its block holds one target
// per lane.  No floating-point atomics anywhere: every output element has one
// writer, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernel_math.hpp"
#include "kernels.hpp"

namespace kafmm {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void two_sum_shift(float &hi, float &lo, float s) {
    // (hi + lo) - s with the rounding error of hi - s moved into lo
    float sum = hi - s;
    float bp = sum - hi;
    float err = (hi - (sum - bp)) + (-s - bp);
    hi = sum;
    lo += err;
}

__device__ __forceinline__ int shift_comp(int code, int k) { return ((code >> (2 * k)) & 3) - 1; }

__global__ void fill_f64(double *p, int64_t n, double v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

__global__ void fill_f32(float *p, int64_t n, float v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------------ packing
// Leaf-sorted source positions (hi/lo FP32 of the normalised FP64 value);
// value slots are zeroed here and written by each run's value packing.
__global__ void pack_sources(int64_t n, const double *__restrict__ xyz, const int32_t *__restrict__ perm,
                             double3 origin, double inv_len, int rec, float *__restrict__ out) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    float *o = out + i * rec;
    double u[3] = {(xyz[3 * j] - origin.x) * inv_len, (xyz[3 * j + 1] - origin.y) * inv_len,
                   (xyz[3 * j + 2] - origin.z) * inv_len};
    for (int k = 0; k < 3; ++k) {
        double w = u[k] - floor(u[k]);      // wrap (a no-op for validated open-BC input)
        if (w >= 1.0) w = 0.0;
        float h = float(w);
        o[k] = h;
        o[3 + k] = float(w - double(h));
    }
    for (int k = 6; k < rec; ++k) o[k] = 0.0f;
}

__global__ void pack_targets(int64_t n, const double *__restrict__ xyz, const int32_t *__restrict__ perm,
                             double3 origin, double inv_len, float *__restrict__ out) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    double u[3] = {(xyz[3 * j] - origin.x) * inv_len, (xyz[3 * j + 1] - origin.y) * inv_len,
                   (xyz[3 * j + 2] - origin.z) * inv_len};
    float4 hi, lo;
    float *h = &hi.x, *l = &lo.x;
    for (int k = 0; k < 3; ++k) {
        double w = u[k] - floor(u[k]);
        if (w >= 1.0) w = 0.0;
        h[k] = float(w);
        l[k] = float(w - double(h[k]));
    }
    hi.w = 0.0f;
    lo.w = 0.0f;
    reinterpret_cast<float4 *>(out)[2 * i] = hi;
    reinterpret_cast<float4 *>(out)[2 * i + 1] = lo;
}

// ------------------------------------------------------------------ P2P (S->T over direct lists)
// One block per task: up to 256 targets of one leaf (one per lane) against a
// slice of the leaf's direct list (U list plus W/X pairs evaluated directly;
// every entry is a leaf).  Source records are wave-uniform, so they arrive
// through scalar loads.  FP32 pair arithmetic; each run of 64 sources is
// summed in FP32 and added to FP64 accumulators; the task writes its partial
// sums, which the combine step adds in task order.
//
// r = x - y is formed in one of two ways:
//   hi/lo  r = (x_hi - y_hi) + (x_lo - y_lo): nearly exact for any pair;
//   REL    per entry the target is moved, in FP64, into the frame of the
//          source leaf's centre and rounded once; r = x_rel - y_rel with y_rel
//          the FP32 source position relative to its leaf centre.  The error
//          of r is a few ulp of the leaf side, a relative error of order
//          1e-7 h / |r| per pair, and it saves 6 of about 26 operations per
//          pair.  Used where the kernel's singularity is mild enough (the
//          Stokeslet, 1/r) for that to stay far below the FMM error.
//
// Coincident points (r = 0) contribute nothing.  Only the target leaf's own
// entry can hold them (equal positions fall in the same leaf), so the REL
// loop guards 1/r against r = 0 there and nowhere else; distinct points of
// different leaves closer than about 2^-22 of the root box, which FP32
// leaf-relative positions cannot separate, give a non-finite result.
template <class K, bool GUARD>
__device__ __forceinline__ void p2p_rel_run(const float *__restrict__ src, int j0, int j1, float xr, float yr,
                                            float zr, double *acc) {
    for (int r0 = j0; r0 < j1; r0 += 64) {
        const int r1 = min(r0 + 64, j1);
        float part[K::NACC];
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) part[k] = 0.0f;
#pragma unroll 4
        for (int j = r0; j < r1; ++j) {
            const float *s = src + int64_t(j) * K::RS;
            const float dx = xr - s[9], dy = yr - s[10], dz = zr - s[11];
            const float r2 = dot3(dx, dy, dz, dx, dy, dz);
            const float ri = GUARD ? rsq_or_zero(r2) : __builtin_amdgcn_rsqf(r2);
            K::sl(dx, dy, dz, ri, s + 6, part);
        }
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) acc[k] += double(part[k]);
    }
}

template <class K>
__device__ __forceinline__ void p2p_run(const float *__restrict__ src, int j0, int j1, float xh, float yh,
                                        float zh, float xl, float yl, float zl, double *acc, bool dl) {
    for (int r0 = j0; r0 < j1; r0 += 64) {
        const int r1 = min(r0 + 64, j1);
        float part[K::NACC];
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) part[k] = 0.0f;
        const int rs = dl ? (K::RD > 0 ? K::RD : 1) : K::RS;
#pragma unroll 4
        for (int j = r0; j < r1; ++j) {
            const float *s = src + int64_t(j) * rs;
            const float dx = (xh - s[0]) + (xl - s[3]);
            const float dy = (yh - s[1]) + (yl - s[4]);
            const float dz = (zh - s[2]) + (zl - s[5]);
            const float ri = rsq_or_zero(dot3(dx, dy, dz, dx, dy, dz));
            if (dl) K::dl(dx, dy, dz, ri, s + 6, part);
            else K::sl(dx, dy, dz, ri, s + 6, part);
        }
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) acc[k] += double(part[k]);
    }
}

// A wave whose chunk leaves it m <= 32 targets spreads each target over
// g = floor(64/m) lanes: lane l serves target l mod m and the sources
// j0 + l/m, j0 + l/m + g, ... of every list entry (per-lane loads instead of
// wave-uniform ones), and the g partial sums of a target are added in lane
// order through cross-lane reads, so the result is deterministic.  Lanes
// past g m take no sources.
template <class K, bool GUARD>
__device__ __forceinline__ void p2p_rel_split(const float *__restrict__ src, int j0, int j1, int g, float xr,
                                              float yr, float zr, double *acc) {
    for (int r0 = j0; r0 < j1; r0 += 64 * g) {
        const int r1 = min(r0 + 64 * g, j1);
        float part[K::NACC];
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) part[k] = 0.0f;
        for (int j = r0; j < r1; j += g) {
            const float *s = src + int64_t(j) * K::RS;
            const float dx = xr - s[9], dy = yr - s[10], dz = zr - s[11];
            const float r2 = dot3(dx, dy, dz, dx, dy, dz);
            const float ri = GUARD ? rsq_or_zero(r2) : __builtin_amdgcn_rsqf(r2);
            K::sl(dx, dy, dz, ri, s + 6, part);
        }
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) acc[k] += double(part[k]);
    }
}

template <class K>
__device__ __forceinline__ void p2p_run_split(const float *__restrict__ src, int j0, int j1, int g, float xh,
                                              float yh, float zh, float xl, float yl, float zl, double *acc,
                                              bool dl) {
    const int rs = dl ? (K::RD > 0 ? K::RD : 1) : K::RS;
    for (int r0 = j0; r0 < j1; r0 += 64 * g) {
        const int r1 = min(r0 + 64 * g, j1);
        float part[K::NACC];
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) part[k] = 0.0f;
        for (int j = r0; j < r1; j += g) {
            const float *s = src + int64_t(j) * rs;
            const float dx = (xh - s[0]) + (xl - s[3]);
            const float dy = (yh - s[1]) + (yl - s[4]);
            const float dz = (zh - s[2]) + (zl - s[5]);
            const float ri = rsq_or_zero(dot3(dx, dy, dz, dx, dy, dz));
            if (dl) K::dl(dx, dy, dz, ri, s + 6, part);
            else K::sl(dx, dy, dz, ri, s + 6, part);
        }
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) acc[k] += double(part[k]);
    }
}

template <class K>
__device__ __forceinline__ void p2p_wave_split(const P2PArgs &a, int4 task, int4 ch, int first, int m, int wbase) {
    const int lane = int(threadIdx.x) & 63;
    const int g = 64 / m;
    const int tl = lane % m, sg = lane / m;       // target slot and source group of this lane
    const bool works = sg < g;
    const int ti = first + tl;
    const float4 p0 = reinterpret_cast<const float4 *>(a.trg)[2 * ti];
    const float4 p1 = reinterpret_cast<const float4 *>(a.trg)[2 * ti + 1];
    double acc[K::NACC];
#pragma unroll
    for (int k = 0; k < K::NACC; ++k) acc[k] = 0.0;
    for (int e = task.y; e < task.z; ++e) {
        const int2 en = a.ent[e];
        const int sx = shift_comp(en.y, 0), sy = shift_comp(en.y, 1), sz = shift_comp(en.y, 2);
        const int2 rs = a.box_sl[en.x];
        const int j0 = works ? rs.x + sg : rs.y;
        if (K::REL) {
            const double4 gm = a.geom[en.x];
            const float xr = float((double(p0.x) - (gm.x + sx)) + double(p1.x));
            const float yr = float((double(p0.y) - (gm.y + sy)) + double(p1.y));
            const float zr = float((double(p0.z) - (gm.z + sz)) + double(p1.z));
            if (en.x == ch.x && en.y == kZeroShift) p2p_rel_split<K, true>(a.sl, j0, rs.y, g, xr, yr, zr, acc);
            else p2p_rel_split<K, false>(a.sl, j0, rs.y, g, xr, yr, zr, acc);
        } else {
            float xh = p0.x, yh = p0.y, zh = p0.z, xl = p1.x, yl = p1.y, zl = p1.z;
            if (sx) two_sum_shift(xh, xl, float(sx));
            if (sy) two_sum_shift(yh, yl, float(sy));
            if (sz) two_sum_shift(zh, zl, float(sz));
            p2p_run_split<K>(a.sl, j0, rs.y, g, xh, yh, zh, xl, yl, zl, acc, false);
            if (K::RD > 0) {
                const int2 rd = a.box_dl[en.x];
                p2p_run_split<K>(a.dl, works ? rd.x + sg : rd.y, rd.y, g, xh, yh, zh, xl, yl, zl, acc, true);
            }
        }
    }
    // lane tl (< m) adds the partial sums of lanes tl + q m, q = 1 .. g-1, in order
#pragma unroll
    for (int k = 0; k < K::NACC; ++k) {
        double v = acc[k];
        for (int q = 1; q < g; ++q) {
            const double w = __shfl(acc[k], tl + q * m, 64);
            v += w;
        }
        acc[k] = v;
    }
    if (lane < m) {
        double *o = a.part + (int64_t(blockIdx.x) * 256 + wbase + lane) * K::NACC;
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) o[k] = acc[k];
    }
}

template <class K>
__global__ __launch_bounds__(256) void p2p_kernel(P2PArgs a) {
    static_assert(!K::REL || K::RD == 0, "REL positions exist for single-layer records only");
    const int4 task = a.tasks[blockIdx.x];
    const int4 ch = a.chunks[task.x];
    const int wbase = int(threadIdx.x & ~63u);
    const int first = ch.y + wbase;
    if (first >= ch.z) return;                       // whole wave idle
    const int m = min(64, ch.z - first);             // targets of this wave
    if (m <= 32) {                                   // partly filled wave: sources split over lanes
        p2p_wave_split<K>(a, task, ch, first, m, wbase);
        return;
    }
    const int t = ch.y + int(threadIdx.x);
    const bool active = t < ch.z;
    const int ti = active ? t : ch.z - 1;
    const float4 p0 = reinterpret_cast<const float4 *>(a.trg)[2 * ti];
    const float4 p1 = reinterpret_cast<const float4 *>(a.trg)[2 * ti + 1];
    double acc[K::NACC];
#pragma unroll
    for (int k = 0; k < K::NACC; ++k) acc[k] = 0.0;
    for (int e = task.y; e < task.z; ++e) {
        const int2 en = a.ent[e];
        const int sx = shift_comp(en.y, 0), sy = shift_comp(en.y, 1), sz = shift_comp(en.y, 2);
        const int2 rs = a.box_sl[en.x];
        if (K::REL) {
            // target relative to the (image of the) source leaf's centre
            const double4 g = a.geom[en.x];
            const float xr = float((double(p0.x) - (g.x + sx)) + double(p1.x));
            const float yr = float((double(p0.y) - (g.y + sy)) + double(p1.y));
            const float zr = float((double(p0.z) - (g.z + sz)) + double(p1.z));
            if (en.x == ch.x && en.y == kZeroShift) p2p_rel_run<K, true>(a.sl, rs.x, rs.y, xr, yr, zr, acc);
            else p2p_rel_run<K, false>(a.sl, rs.x, rs.y, xr, yr, zr, acc);
        } else {
            float xh = p0.x, yh = p0.y, zh = p0.z, xl = p1.x, yl = p1.y, zl = p1.z;
            if (sx) two_sum_shift(xh, xl, float(sx));
            if (sy) two_sum_shift(yh, yl, float(sy));
            if (sz) two_sum_shift(zh, zl, float(sz));
            p2p_run<K>(a.sl, rs.x, rs.y, xh, yh, zh, xl, yl, zl, acc, false);
            if (K::RD > 0) {
                const int2 rd = a.box_dl[en.x];
                p2p_run<K>(a.dl, rd.x, rd.y, xh, yh, zh, xl, yl, zl, acc, true);
            }
        }
    }
    if (active) {
        double *o = a.part + (int64_t(blockIdx.x) * 256 + threadIdx.x) * K::NACC;
#pragma unroll
        for (int k = 0; k < K::NACC; ++k) o[k] = acc[k];
    }
}

// Plan-time check of the leaf-relative P2P form (one block per P2P task, a
// target per thread, as p2p_kernel): for every entry other than the
// target's own leaf, a target within delta = 2^-12 of the source leaf's side
// from that (image-shifted) leaf's box is compared with each of its
// sources in FP64; a pair closer than delta sets *flag.  Such a pair's
// leaf-relative r would carry a relative error above about 2^-11 (or be 0).
__global__ __launch_bounds__(256) void rel_check_kernel(P2PArgs a, int rec, unsigned *flag) {
    const int4 task = a.tasks[blockIdx.x];
    const int4 ch = a.chunks[task.x];
    const int t = ch.y + int(threadIdx.x);
    if (t >= ch.z) return;
    const float4 p0 = reinterpret_cast<const float4 *>(a.trg)[2 * t];
    const float4 p1 = reinterpret_cast<const float4 *>(a.trg)[2 * t + 1];
    const double x[3] = {double(p0.x) + double(p1.x), double(p0.y) + double(p1.y), double(p0.z) + double(p1.z)};
    for (int e = task.y; e < task.z; ++e) {
        const int2 en = a.ent[e];
        if (en.x == ch.x && en.y == kZeroShift) continue;
        const double sh[3] = {double(shift_comp(en.y, 0)), double(shift_comp(en.y, 1)), double(shift_comp(en.y, 2))};
        const double4 g = a.geom[en.x];
        const double delta = g.w * (1.0 / 4096.0);
        const double c[3] = {g.x + sh[0], g.y + sh[1], g.z + sh[2]};
        double db = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double o = fmax(fabs(x[k] - c[k]) - 0.5 * g.w, 0.0);
            db += o * o;
        }
        if (db >= delta * delta) continue;
        const int2 rs = a.box_sl[en.x];
        for (int j = rs.x; j < rs.y; ++j) {
            const float *s = a.sl + int64_t(j) * rec;
            double d2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double d = x[k] - (double(s[k]) + double(s[3 + k]) + sh[k]);
                d2 += d * d;
            }
            if (d2 < delta * delta) atomicOr(flag, 1u);
        }
    }
}

// Leaf-relative FP32 source positions (record slots 9..11) for kernels whose
// P2P forms r in the REL way: y_rel = (y_hi - c) + y_lo, rounded once.
__global__ __launch_bounds__(256) void rel_positions_kernel(const int *__restrict__ leaves,
                                                            const int2 *__restrict__ box_sl,
                                                            const double4 *__restrict__ geom, int rec,
                                                            float *__restrict__ sl) {
    const int b = leaves[blockIdx.x];
    const int2 r = box_sl[b];
    const double4 g = geom[b];
    for (int j = r.x + int(threadIdx.x); j < r.y; j += blockDim.x) {
        float *s = sl + int64_t(j) * rec;
        const float x = float((double(s[0]) - g.x) + double(s[3]));
        const float y = float((double(s[1]) - g.y) + double(s[4]));
        const float z = float((double(s[2]) - g.z) + double(s[5]));
        s[9] = x;
        s[10] = y;
        s[11] = z;
    }
}

// ------------------------------------------------------------------ S2M / S2L surface tiles
// Check potentials of the 4-Laplace (or 1-Laplace) densities of a source
// leaf's points at the M check points of a destination box (radius alpha).
//
// Sources are first staged once per run (stage_sources_kernel): position
// relative to the centre of their own leaf and the Laplace charges/dipoles
// carried relative to that centre.  A task {dst, shift | src << 6, j0, j1}
// evaluates sources [j0, j1) of leaf src (image shift) at dst's check
// points: 256 staged records at a time are copied to LDS and every thread
// evaluates them at 2-4 check points (reusing each LDS read).  The Psi
// potential is then moved from the source leaf's origin to dst's:
// Psi_dst = Psi_src + (c_src - c_dst).Phi.
//
// Staged records (RS floats per source), by source kind:
//   0 Stokeslet f     [yr, f, yr.f, 0]           Phi_j charge f_j, Psi charge yr.f
//   1 RPY f, b^2      [yr, f, yr.f, 0, m, 0]     + Psi dipole m = (b^2/3) f
//   2 Laplace q       [yr, q]                    charge
//   3 Laplace d       [yr, d, 0, 0]              dipole
//   4 Stokes f, q     [yr, f, yr.f + q, 0]       Phi_j charge f_j, Psi charge
//   5 Stokes D^s      [yr, D^s (6), 0, 0, 0]     Phi_j dipole -D^s_j., Psi dipole -D^s yr
//   8 Laplace Q^s     [yr, Q^s (6), 0, 0, 0]     quadrupole (second derivative of a charge)
//   7 regularized     [yr, f, yr.f, 0, t, 0,     Phi_j charge f_j, Psi charge yr.f; the torque
//     force, torque    m, 0]                      (rotlet) as Phi_i dipoles (e_i x t)/2 and, with
//                                                 the eps^2 term, Psi dipole m = (eps^2/2) f + (yr x t)/2
constexpr int kS2CTile = 256;   // staged records per LDS tile

template <int SRC> struct S2CKind;
template <> struct S2CKind<0> { static constexpr int NC = 4, RS = 8; };
template <> struct S2CKind<1> { static constexpr int NC = 4, RS = 12; };
template <> struct S2CKind<2> { static constexpr int NC = 1, RS = 4; };
template <> struct S2CKind<3> { static constexpr int NC = 1, RS = 8; };
template <> struct S2CKind<4> { static constexpr int NC = 4, RS = 8; };
template <> struct S2CKind<5> { static constexpr int NC = 4, RS = 12; };
template <> struct S2CKind<7> { static constexpr int NC = 4, RS = 16; };
template <> struct S2CKind<8> { static constexpr int NC = 1, RS = 12; };

int s2c_stage_stride(int src_kind) {
    switch (src_kind) {
        case 0: return S2CKind<0>::RS;
        case 1: return S2CKind<1>::RS;
        case 2: return S2CKind<2>::RS;
        case 3: return S2CKind<3>::RS;
        case 4: return S2CKind<4>::RS;
        case 5: return S2CKind<5>::RS;
        case 7: return S2CKind<7>::RS;
        case 8: return S2CKind<8>::RS;
        default: return 0;
    }
}

// One block per leaf holding sources of this kind; rec = packed record stride.
template <int SRC>
__global__ __launch_bounds__(256) void stage_sources_kernel(const int *__restrict__ leaves,
                                                            const int2 *__restrict__ box_range,
                                                            const double4 *__restrict__ geom,
                                                            const float *__restrict__ src, int rec,
                                                            float *__restrict__ out) {
    constexpr int RS = S2CKind<SRC>::RS;
    const int b = leaves[blockIdx.x];
    const int2 r = box_range[b];
    const double4 g = geom[b];
    for (int j = r.x + int(threadIdx.x); j < r.y; j += blockDim.x) {
        const float *s = src + int64_t(j) * rec;
        const float yx = float((double(s[0]) - g.x) + double(s[3]));
        const float yy = float((double(s[1]) - g.y) + double(s[4]));
        const float yz = float((double(s[2]) - g.z) + double(s[5]));
        float o[RS];
#pragma unroll
        for (int k = 0; k < RS; ++k) o[k] = 0.0f;
        o[0] = yx; o[1] = yy; o[2] = yz;
        if constexpr (SRC == 0 || SRC == 1 || SRC == 4) {
            o[3] = s[6]; o[4] = s[7]; o[5] = s[8];
            o[6] = dot3(yx, yy, yz, s[6], s[7], s[8]) + (SRC == 4 ? s[9] : 0.0f);
            if constexpr (SRC == 1) {
                const float c = s[9] * (1.0f / 3.0f);
                o[8] = c * s[6]; o[9] = c * s[7]; o[10] = c * s[8];
            }
        } else if constexpr (SRC == 2) {
            o[3] = s[6];
        } else if constexpr (SRC == 3) {
            o[3] = s[6]; o[4] = s[7]; o[5] = s[8];
        } else if constexpr (SRC == 7) {
            // record: f at 6..8, t at 9..11, (3/2) eps^2 at 12
            const float f0 = s[6], f1 = s[7], f2 = s[8], t0 = s[9], t1 = s[10], t2 = s[11];
            const float ce = s[12] * (1.0f / 3.0f);     // eps^2 / 2
            o[3] = f0; o[4] = f1; o[5] = f2;
            o[6] = dot3(yx, yy, yz, f0, f1, f2);
            o[8] = t0; o[9] = t1; o[10] = t2;
            o[12] = fmaf(ce, f0, 0.5f * (yy * t2 - yz * t1));
            o[13] = fmaf(ce, f1, 0.5f * (yz * t0 - yx * t2));
            o[14] = fmaf(ce, f2, 0.5f * (yx * t1 - yy * t0));
        } else {   // 5 and 8: the symmetric tensor as packed
#pragma unroll
            for (int k = 0; k < 6; ++k) o[3 + k] = s[6 + k];
        }
        float4 *d = reinterpret_cast<float4 *>(out + int64_t(j) * RS);
#pragma unroll
        for (int k = 0; k < RS / 4; ++k) d[k] = make_float4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
    }
}

template <int SRC, int PTS>
__global__ __launch_bounds__(1024) void s2c_kernel(S2CArgs a) {
    constexpr int NC = S2CKind<SRC>::NC, RS = S2CKind<SRC>::RS, R4 = RS / 4;
    __shared__ float4 tile[kS2CTile * R4];
    const int4 task = a.tasks[blockIdx.x];         // {dst, shift | src << 6, j0, j1}
    const int code = task.y & 63, srcbox = task.y >> 6;
    const double4 cb = a.geom[task.x], ca = a.geom[srcbox];
    // destination centre relative to the (image of the) source leaf centre
    const double ox = cb.x - (ca.x + shift_comp(code, 0)), oy = cb.y - (ca.y + shift_comp(code, 1)),
                 oz = cb.z - (ca.z + shift_comp(code, 2));
    const double rad = a.alpha * 0.5 * cb.w;
    const int nthr = int(blockDim.x);
    float zx[PTS], zy[PTS], zz[PTS], pot[PTS][NC];
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
        const int m = int(threadIdx.x) + nthr * i;
        const int mm = m < a.M ? m : 0;
        zx[i] = float(ox + rad * a.grid[3 * mm]);
        zy[i] = float(oy + rad * a.grid[3 * mm + 1]);
        zz[i] = float(oz + rad * a.grid[3 * mm + 2]);
#pragma unroll
        for (int c = 0; c < NC; ++c) pot[i][c] = 0.0f;
    }
    for (int j0 = task.z; j0 < task.w; j0 += kS2CTile) {
        const int n = min(kS2CTile, task.w - j0);
        __syncthreads();
        const float4 *src = reinterpret_cast<const float4 *>(a.staged + int64_t(j0) * RS);
        for (int q = int(threadIdx.x); q < n * R4; q += nthr) tile[q] = src[q];
        __syncthreads();
#pragma unroll 2
        for (int j = 0; j < n; ++j) {
            float y[RS];
#pragma unroll
            for (int k = 0; k < R4; ++k) {
                const float4 v = tile[j * R4 + k];
                y[4 * k] = v.x; y[4 * k + 1] = v.y; y[4 * k + 2] = v.z; y[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int i = 0; i < PTS; ++i) {
                // check points lie outside every source box: r > 0
                const float dx = zx[i] - y[0], dy = zy[i] - y[1], dz = zz[i] - y[2];
                const float ri = __builtin_amdgcn_rsqf(dot3(dx, dy, dz, dx, dy, dz));
                if constexpr (SRC == 0 || SRC == 4) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) pot[i][c] = fmaf(y[3 + c], ri, pot[i][c]);
                } else if constexpr (SRC == 1) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) pot[i][c] = fmaf(y[3 + c], ri, pot[i][c]);
                    pot[i][3] = fmaf(dot3(y[8], y[9], y[10], dx, dy, dz), ri * ri * ri, pot[i][3]);
                } else if constexpr (SRC == 2) {
                    pot[i][0] = fmaf(y[3], ri, pot[i][0]);
                } else if constexpr (SRC == 3) {
                    pot[i][0] = fmaf(dot3(y[3], y[4], y[5], dx, dy, dz), ri * ri * ri, pot[i][0]);
                } else if constexpr (SRC == 7) {
                    // charges; Phi_i dipoles (e_i x t)/2: (e_i x t).d / 2 = (t x d)_i / 2; Psi dipole
                    const float ri3 = ri * ri * ri, hr3 = 0.5f * ri3;
#pragma unroll
                    for (int c = 0; c < 4; ++c) pot[i][c] = fmaf(y[3 + c], ri, pot[i][c]);
                    pot[i][0] = fmaf(hr3, y[9] * dz - y[10] * dy, pot[i][0]);
                    pot[i][1] = fmaf(hr3, y[10] * dx - y[8] * dz, pot[i][1]);
                    pot[i][2] = fmaf(hr3, y[8] * dy - y[9] * dx, pot[i][2]);
                    pot[i][3] = fmaf(dot3(y[12], y[13], y[14], dx, dy, dz), ri3, pot[i][3]);
                } else if constexpr (SRC == 8) {
                    // Q_jk d_j d_k (1/r) = 3 (d.Q.d)/r^5 - tr Q/r^3
                    float wx, wy, wz;
                    sym_apply(y + 3, dx, dy, dz, wx, wy, wz);
                    const float ri2 = ri * ri, ri3 = ri2 * ri;
                    const float B = dot3(dx, dy, dz, wx, wy, wz), tr = y[3] + y[6] + y[8];
                    pot[i][0] = fmaf(fmaf(3.0f * B, ri2, -tr), ri3, pot[i][0]);
                } else {
                    // w = D^s (z - y): Phi_j += -w_j / r^3, Psi += -(yr . w) / r^3
                    float wx, wy, wz;
                    sym_apply(y + 3, dx, dy, dz, wx, wy, wz);
                    const float mri3 = -(ri * ri * ri);
                    pot[i][0] = fmaf(wx, mri3, pot[i][0]);
                    pot[i][1] = fmaf(wy, mri3, pot[i][1]);
                    pot[i][2] = fmaf(wz, mri3, pot[i][2]);
                    pot[i][3] = fmaf(dot3(y[0], y[1], y[2], wx, wy, wz), mri3, pot[i][3]);
                }
            }
        }
    }
    float *o = a.part + int64_t(blockIdx.x) * NC * a.M;
    const float dx = float(-ox), dy = float(-oy), dz = float(-oz);   // c_src - c_dst
#pragma unroll
    for (int i = 0; i < PTS; ++i) {
        const int m = int(threadIdx.x) + nthr * i;
        if (m >= a.M) continue;
        if constexpr (NC == 4) pot[i][3] = fmaf(dx, pot[i][0], fmaf(dy, pot[i][1], fmaf(dz, pot[i][2], pot[i][3])));
#pragma unroll
        for (int c = 0; c < NC; ++c) o[c * a.M + m] = pot[i][c];
    }
}

// chk[dst][c][m] (+)= (1/4 pi) sum over the dst's tasks of part[task][c][m], in task order
__global__ __launch_bounds__(256) void s2c_reduce(S2CReduceArgs a) {
    const int dst = a.dst[blockIdx.x];
    const int t0 = a.off[blockIdx.x], t1 = a.off[blockIdx.x + 1];
    const int n = a.ncomp * a.M;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double acc = 0.0;
        for (int t = t0; t < t1; ++t) acc += double(a.part[int64_t(a.task[t]) * n + i]);
        double *o = a.chk + int64_t(dst) * n + i;
        acc *= kInv4Pi;
        *o = a.accumulate ? *o + acc : acc;
    }
}

// ------------------------------------------------------------------ grouped FP32 MFMA GEMM
// Y[:, col] = A_op * X[:, col] for tiles of 128 columns sharing one operator.
// A_op: [R][K] row-major (operators opsz floats apart); columns of X (K
// floats) and Y (R floats) are contiguous, at bcol * xs and ycol * ys.
// Block 256 threads = 4 waves in a 2x2 arrangement, each wave 64x64 as 2x2
// v_mfma_f32_32x32x2f32 tiles; K staged through LDS in steps of 32.
constexpr int kGT = 128;
constexpr int kGK = 32;
constexpr int kGLd = kGK + 1;

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Workgroups are dealt to the 8 XCDs in turn (workgroup i to XCD i mod 8).
// Tiles sharing an operator are consecutive, so tile t of n is given to
// workgroup i such that each XCD runs one contiguous range of tiles and
// keeps their operator in its own L2: XCD k = i mod 8 takes tiles
// [k q + min(k, r), ...) in order, q = n / 8, r = n mod 8 (a bijection of
// [0, n)).
__device__ __forceinline__ int xcd_tile(int i, int n) {
    const int k = i & 7, j = i >> 3, q = n >> 3, r = n & 7;
    return k * q + min(k, r) + j;
}

// WR row waves x 2 column waves: block tile (64 WR) rows x 128 columns.
template <int WR>
__global__ __launch_bounds__(128 * WR) void gemm_f32_mfma(GemmArgs a) {
    constexpr int TR = 64 * WR, NT = 128 * WR;
    constexpr int NA = TR * 8 / NT, NB = (kGT * 8 + NT - 1) / NT;   // float4 slots per thread
    __shared__ float As[TR * kGLd];
    __shared__ float Bs[kGT * kGLd];
    const int4 tile = a.tiles[xcd_tile(int(blockIdx.x), int(gridDim.x))];            // op, col0, ncol, -
    const int row0 = blockIdx.y * TR;
    const float *A = a.ops + int64_t(tile.x) * a.opsz;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    // rows at or past Mr are zero padding: their MFMAs are skipped (the
    // accumulators stay 0, which is what the padding rows would give)
    const bool live0 = row0 + wr < a.Mr, live1 = row0 + wr + 32 < a.Mr;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    // per-thread load slots: float4s of A (row, k) and of B (column, k) per K step
    int ar[NA], ak[NA], br[NB], bk[NB];
    bool arow_ok[NA], bcol_ok[NB];
    const float *bptr[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int idx = tid + NT * i;
        ar[i] = idx >> 3;
        ak[i] = (idx & 7) * 4;
        arow_ok[i] = row0 + ar[i] < a.R;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int idx = tid + NT * i;
        br[i] = idx >> 3;
        bk[i] = (idx & 7) * 4;
        bcol_ok[i] = idx < kGT * 8 && br[i] < tile.z;
        const int c = bcol_ok[i] ? a.bcol[tile.y + br[i]] : 0;
        bptr[i] = a.X + int64_t(c) * a.xs;
    }
    // the next K step's tiles are fetched into registers while the MFMAs
    // run on the current one (one LDS buffer, two barriers per step)
    float4 ra[NA], rb[NB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
            ra[i] = arow_ok[i] ? *reinterpret_cast<const float4 *>(A + int64_t(row0 + ar[i]) * a.K + k0 + ak[i])
                               : make_float4(0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < NB; ++i)
            rb[i] = bcol_ok[i] ? *reinterpret_cast<const float4 *>(bptr[i] + k0 + bk[i]) : make_float4(0, 0, 0, 0);
    };
    fetch(0);
    for (int k0 = 0; k0 < a.Mk; k0 += kGK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            float *da = As + ar[i] * kGLd + ak[i];
            da[0] = ra[i].x; da[1] = ra[i].y; da[2] = ra[i].z; da[3] = ra[i].w;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (tid + NT * i >= kGT * 8) continue;
            float *db = Bs + br[i] * kGLd + bk[i];
            db[0] = rb[i].x; db[1] = rb[i].y; db[2] = rb[i].z; db[3] = rb[i].w;
        }
        __syncthreads();
        if (k0 + kGK < a.Mk) fetch(k0 + kGK);
        const int kend = min(kGK, a.Mk - k0);
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 2) {
            if (kk < kend) {
                const int k = kk + (lane >> 5);
                float av[2], bv[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) av[i] = As[(wr + 32 * i + (lane & 31)) * kGLd + k];
#pragma unroll
                for (int j = 0; j < 2; ++j) bv[j] = Bs[(wc + 32 * j + (lane & 31)) * kGLd + k];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (live0) acc[0][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[0], bv[j], acc[0][j], 0, 0, 0);
                    if (live1) acc[1][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[1], bv[j], acc[1][j], 0, 0, 0);
                }
            }
        }
    }
    // epilogue: lane holds column (lane & 31) and rows 8*(v/4) + 4*(lane/32) + v%4
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = wc + 32 * j + (lane & 31);
        if (col >= tile.z) continue;
        float *Y = a.Y + int64_t(a.ycol[tile.y + col]) * a.ys;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int row = row0 + wr + 32 * i + 8 * g + 4 * (lane >> 5);
                if (row < a.R) {
                    float4 v = make_float4(acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2],
                                           acc[i][j][4 * g + 3]);
                    *reinterpret_cast<float4 *>(Y + row) = v;
                }
            }
    }
}

// Row-strip variant for operator sides that 64-row tiles would pad (R = 32 NR
// rows): two waves per 32-row strip of all NR strips, each owning 32 rows x
// 64 of the tile's 128 columns (two 32 x 32 accumulators), so no wave
// computes padding rows and the 2 NR equal waves spread evenly over a CU's
// 4 SIMDs (with one wave per strip and 128 columns each, a block's 5 waves
// could not, and the launch ran 37 % slower).  Same staging, K steps
// and per-output MFMA order as gemm_f32_mfma, hence the same results.
template <int NR>
__global__ __launch_bounds__(128 * NR) void gemm_f32_strip(GemmArgs a) {
    constexpr int TR = 32 * NR, NT = 128 * NR;
    constexpr int NA = TR * 8 / NT, NB = (kGT * 8 + NT - 1) / NT;   // float4 slots per thread
    __shared__ float As[TR * kGLd];
    __shared__ float Bs[kGT * kGLd];
    const int4 tile = a.tiles[xcd_tile(int(blockIdx.x), int(gridDim.x))];            // op, col0, ncol, -
    const float *A = a.ops + int64_t(tile.x) * a.opsz;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 64;   // two waves per strip, 64 columns each
    const bool live = wr < a.Mr;                     // rows at or past Mr are zero padding
    floatx16 acc[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[j][v] = 0.0f;
    int ar[NA], ak[NA], br[NB], bk[NB];
    bool arow_ok[NA], bcol_ok[NB], bslot[NB];
    const float *bptr[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int idx = tid + NT * i;
        ar[i] = idx >> 3;
        ak[i] = (idx & 7) * 4;
        arow_ok[i] = ar[i] < a.R;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int idx = tid + NT * i;
        br[i] = idx >> 3;
        bk[i] = (idx & 7) * 4;
        bslot[i] = idx < kGT * 8;
        bcol_ok[i] = bslot[i] && br[i] < tile.z;
        const int c = bcol_ok[i] ? a.bcol[tile.y + br[i]] : 0;
        bptr[i] = a.X + int64_t(c) * a.xs;
    }
    float4 ra[NA], rb[NB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
            ra[i] = arow_ok[i] ? *reinterpret_cast<const float4 *>(A + int64_t(ar[i]) * a.K + k0 + ak[i])
                               : make_float4(0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < NB; ++i)
            rb[i] = bcol_ok[i] ? *reinterpret_cast<const float4 *>(bptr[i] + k0 + bk[i]) : make_float4(0, 0, 0, 0);
    };
    fetch(0);
    for (int k0 = 0; k0 < a.Mk; k0 += kGK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            float *da = As + ar[i] * kGLd + ak[i];
            da[0] = ra[i].x; da[1] = ra[i].y; da[2] = ra[i].z; da[3] = ra[i].w;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (!bslot[i]) continue;
            float *db = Bs + br[i] * kGLd + bk[i];
            db[0] = rb[i].x; db[1] = rb[i].y; db[2] = rb[i].z; db[3] = rb[i].w;
        }
        __syncthreads();
        if (k0 + kGK < a.Mk) fetch(k0 + kGK);
        const int kend = min(kGK, a.Mk - k0);
        if (live) {
#pragma unroll
            for (int kk = 0; kk < kGK; kk += 2) {
                if (kk < kend) {
                    const int k = kk + (lane >> 5);
                    const float av = As[(wr + (lane & 31)) * kGLd + k];
                    float bv[2];
#pragma unroll
                    for (int j = 0; j < 2; ++j) bv[j] = Bs[(wc + 32 * j + (lane & 31)) * kGLd + k];
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[j], acc[j], 0, 0, 0);
                }
            }
        }
    }
    // epilogue: lane holds column (lane & 31) and rows 8*(v/4) + 4*(lane/32) + v%4
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = wc + 32 * j + (lane & 31);
        if (col >= tile.z) continue;
        float *Y = a.Y + int64_t(a.ycol[tile.y + col]) * a.ys;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int row = wr + 8 * g + 4 * (lane >> 5);
            if (row < a.R) {
                float4 v = make_float4(acc[j][4 * g], acc[j][4 * g + 1], acc[j][4 * g + 2], acc[j][4 * g + 3]);
                *reinterpret_cast<float4 *>(Y + row) = v;
            }
        }
    }
}

// ------------------------------------------------------------------ split-BF16 grouped GEMM
// Same tiling as gemm_f32_mfma, arithmetic in three BF16 passes:
// A = Ah + Al, X = Xh + Xl (hi = RN_bf16(v), lo = RN_bf16(v - hi)), and
// Y = Ah Xh + Ah Xl + Al Xh with FP32 accumulation (the Al Xl term, of
// relative size 2^-16, is dropped).  The split is done while staging tiles
// to LDS; v_mfma_f32_32x32x16_bf16 takes 8 consecutive k per lane.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kBLd = 40;   // LDS row stride in bf16 (32 + 8): conflict-free 16-byte reads

__global__ __launch_bounds__(256) void gemm_bf16x3_mfma(GemmArgs a) {
    __shared__ __bf16 Ah[kGT * kBLd], Al[kGT * kBLd], Bh[kGT * kBLd], Bl[kGT * kBLd];
    const int4 tile = a.tiles[xcd_tile(int(blockIdx.x), int(gridDim.x))];
    const int row0 = blockIdx.y * kGT;
    const float *A = a.ops + int64_t(tile.x) * a.opsz;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const bool live0 = row0 + wr < a.Mr, live1 = row0 + wr + 32 < a.Mr;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    const float *bptr[4];
    int lr[4], lk[4];
    bool arow_ok[4], bcol_ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int idx = tid + 256 * i;
        lr[i] = idx >> 3;
        lk[i] = (idx & 7) * 4;
        arow_ok[i] = row0 + lr[i] < a.R;
        bcol_ok[i] = lr[i] < tile.z;
        int c = bcol_ok[i] ? a.bcol[tile.y + lr[i]] : 0;
        bptr[i] = a.X + int64_t(c) * a.xs;
    }
    float4 ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ra[i] = arow_ok[i] ? *reinterpret_cast<const float4 *>(A + int64_t(row0 + lr[i]) * a.K + k0 + lk[i])
                               : make_float4(0, 0, 0, 0);
            rb[i] = bcol_ok[i] ? *reinterpret_cast<const float4 *>(bptr[i] + k0 + lk[i])
                               : make_float4(0, 0, 0, 0);
        }
    };
    for (int k0 = 0; k0 < a.Mk; k0 += kGK) {
        load(k0);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float va[4] = {ra[i].x, ra[i].y, ra[i].z, ra[i].w};
            const float vb[4] = {rb[i].x, rb[i].y, rb[i].z, rb[i].w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                __bf16 h = __bf16(va[q]);
                Ah[lr[i] * kBLd + lk[i] + q] = h;
                Al[lr[i] * kBLd + lk[i] + q] = __bf16(va[q] - float(h));
                h = __bf16(vb[q]);
                Bh[lr[i] * kBLd + lk[i] + q] = h;
                Bl[lr[i] * kBLd + lk[i] + q] = __bf16(vb[q] - float(h));
            }
        }
        __syncthreads();
        const int kend = min(kGK, a.Mk - k0);
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 16) {
            if (kk >= kend) continue;
            const int ko = kk + 8 * (lane >> 5);
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = (wr + 32 * i + (lane & 31)) * kBLd + ko;
                ah[i] = *reinterpret_cast<const bf16x8 *>(Ah + r);
                al[i] = *reinterpret_cast<const bf16x8 *>(Al + r);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int r = (wc + 32 * j + (lane & 31)) * kBLd + ko;
                bh[j] = *reinterpret_cast<const bf16x8 *>(Bh + r);
                bl[j] = *reinterpret_cast<const bf16x8 *>(Bl + r);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if (!(i == 0 ? live0 : live1)) continue;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = wc + 32 * j + (lane & 31);
        if (col >= tile.z) continue;
        float *Y = a.Y + int64_t(a.ycol[tile.y + col]) * a.ys;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int row = row0 + wr + 32 * i + 8 * g + 4 * (lane >> 5);
                if (row < a.R) {
                    float4 v = make_float4(acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2],
                                           acc[i][j][4 * g + 3]);
                    *reinterpret_cast<float4 *>(Y + row) = v;
                }
            }
    }
}

// Row-strip form of gemm_bf16x3_mfma for 160-row operators (rank 160): one
// block covers all rows, two waves per 32-row strip with 64 columns each
// (10 equal waves), so each column tile's source coefficients are gathered
// once and no wave computes padding rows; hi/lo values are staged with one
// 8-byte LDS write per four.  Same arithmetic per output as
// gemm_bf16x3_mfma.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <int NR>
__global__ __launch_bounds__(128 * NR) void gemm_bf16x3_strip(GemmArgs a) {
    constexpr int TR = 32 * NR, NT = 128 * NR;
    constexpr int NA = TR * 8 / NT, NB = (kGT * 8 + NT - 1) / NT;   // float4 slots per thread
    __shared__ __align__(16) __bf16 Ah[TR * kBLd], Al[TR * kBLd], Bh[kGT * kBLd], Bl[kGT * kBLd];
    const int4 tile = a.tiles[xcd_tile(int(blockIdx.x), int(gridDim.x))];
    const float *A = a.ops + int64_t(tile.x) * a.opsz;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 64;
    const bool live = wr < a.Mr;
    floatx16 acc[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[j][v] = 0.0f;
    int ar[NA], ak[NA], br[NB], bk[NB];
    bool arow_ok[NA], bcol_ok[NB], bslot[NB];
    const float *bptr[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int idx = tid + NT * i;
        ar[i] = idx >> 3;
        ak[i] = (idx & 7) * 4;
        arow_ok[i] = ar[i] < a.R;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int idx = tid + NT * i;
        br[i] = idx >> 3;
        bk[i] = (idx & 7) * 4;
        bslot[i] = idx < kGT * 8;
        bcol_ok[i] = bslot[i] && br[i] < tile.z;
        const int c = bcol_ok[i] ? a.bcol[tile.y + br[i]] : 0;
        bptr[i] = a.X + int64_t(c) * a.xs;
    }
    float4 ra[NA], rb[NB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
            ra[i] = arow_ok[i] ? *reinterpret_cast<const float4 *>(A + int64_t(ar[i]) * a.K + k0 + ak[i])
                               : make_float4(0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < NB; ++i)
            rb[i] = bcol_ok[i] ? *reinterpret_cast<const float4 *>(bptr[i] + k0 + bk[i]) : make_float4(0, 0, 0, 0);
    };
    auto split4 = [](float4 v, __bf16 *hi, __bf16 *lo) {
        bf16x4 h, l;
        h[0] = __bf16(v.x); l[0] = __bf16(v.x - float(h[0]));
        h[1] = __bf16(v.y); l[1] = __bf16(v.y - float(h[1]));
        h[2] = __bf16(v.z); l[2] = __bf16(v.z - float(h[2]));
        h[3] = __bf16(v.w); l[3] = __bf16(v.w - float(h[3]));
        *reinterpret_cast<bf16x4 *>(hi) = h;
        *reinterpret_cast<bf16x4 *>(lo) = l;
    };
    fetch(0);
    for (int k0 = 0; k0 < a.Mk; k0 += kGK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int o = ar[i] * kBLd + ak[i];
            split4(ra[i], Ah + o, Al + o);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (!bslot[i]) continue;
            const int o = br[i] * kBLd + bk[i];
            split4(rb[i], Bh + o, Bl + o);
        }
        __syncthreads();
        if (k0 + kGK < a.Mk) fetch(k0 + kGK);
        const int kend = min(kGK, a.Mk - k0);
        if (live) {
#pragma unroll
            for (int kk = 0; kk < kGK; kk += 16) {
                if (kk >= kend) continue;
                const int ko = kk + 8 * (lane >> 5);
                const int ra0 = (wr + (lane & 31)) * kBLd + ko;
                const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(Ah + ra0);
                const bf16x8 al = *reinterpret_cast<const bf16x8 *>(Al + ra0);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int rb0 = (wc + 32 * j + (lane & 31)) * kBLd + ko;
                    const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(Bh + rb0);
                    const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(Bl + rb0);
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = wc + 32 * j + (lane & 31);
        if (col >= tile.z) continue;
        float *Y = a.Y + int64_t(a.ycol[tile.y + col]) * a.ys;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int row = wr + 8 * g + 4 * (lane >> 5);
            if (row < a.R) {
                float4 v = make_float4(acc[j][4 * g], acc[j][4 * g + 1], acc[j][4 * g + 2], acc[j][4 * g + 3]);
                *reinterpret_cast<float4 *>(Y + row) = v;
            }
        }
    }
}

// ------------------------------------------------------------------ FP64 GEMM (pseudo-inverse)
// C[col][i] = scale(col) * sum_k A[i][k] * B[col][k],  i < R, k < K.
// B columns are FP64 (check values or scratch); C is FP64 scratch or FP32
// densities.  Block tile 64 rows x 64 columns, 4 waves in 2x2 each owning
// 32x32 as 2x2 v_mfma_f64_16x16x4f64 tiles, K staged through LDS by 16.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename TC>
__global__ __launch_bounds__(256) void gemm_f64(Gemm64Args a, TC *C) {
    __shared__ double As[64 * 17];
    __shared__ double Bs[64 * 17];
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    doublex4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    // each thread stages 4 elements of A and of B per K step
    const double *bcol[4];
    int lr[4], lk[4];
    bool rok[4], cok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int idx = tid + 256 * i;
        lr[i] = idx >> 4;
        lk[i] = idx & 15;
        rok[i] = row0 + lr[i] < a.R;
        cok[i] = col0 + lr[i] < a.ncol;
        bcol[i] = a.B + int64_t(cok[i] ? a.bidx[col0 + lr[i]] : 0) * a.ldb;
    }
    // the next K step's elements are fetched into registers while the MFMAs
    // run on the current one
    double ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + lk[i];
            ra[i] = (rok[i] && k < a.K) ? a.A[int64_t(row0 + lr[i]) * a.lda + k] : 0.0;
            rb[i] = (cok[i] && k < a.K) ? bcol[i][k] : 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < a.K; k0 += 16) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            As[lr[i] * 17 + lk[i]] = ra[i];
            Bs[lr[i] * 17 + lk[i]] = rb[i];
        }
        __syncthreads();
        if (k0 + 16 < a.K) fetch(k0 + 16);
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const int k = kk + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[(wr + 16 * i + (lane & 15)) * 17 + k];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[(wc + 16 * j + (lane & 15)) * 17 + k];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    // lane holds column (lane & 15) and rows (lane/16) + 4 v of each 16x16 tile
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int c = col0 + wc + 16 * j + (lane & 15);
        if (c >= a.ncol) continue;
        const double s = a.cscale ? a.cscale[c] : 1.0;
        TC *o = C + int64_t(a.cidx[c]) * a.ldc;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = row0 + wr + 16 * i + (lane >> 4) + 4 * v;
                if (r < a.R) o[r] = TC(s * acc[i][j][v]);
            }
    }
}

// ------------------------------------------------------------------ downward check-to-check translation
// chk[child][c][i] += sum_k L[op][i][k] * x[k], x = chk[parent][c] (for c = 3
// of the 4-Laplace tree the Psi origin shift x = Psi - delta.Phi is applied
// to the parent's values first: the translation is linear and the same for
// every component).  FP64 throughout: these potentials feed the leaf
// pseudo-inverses, which amplify rounding noise into the high-frequency
// density modes that target derivatives see.  Block tile 64 rows x 64
// columns (16 pairs x 4 components or 64 pairs x 1) as in gemm_f64.
template <int NC>
__global__ __launch_bounds__(256) void l2l_check_kernel(L2LArgs a) {
    __shared__ double As[64 * 17];
    __shared__ double Bs[64 * 17];
    const int4 blk = a.blocks[blockIdx.y];
    const int M = a.M, row0 = blockIdx.x * 64, ncol = blk.z * NC;
    const double *A = a.ops + int64_t(blk.x) * M * M;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    doublex4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    const double *pc[4];
    int lr[4], lk[4], comp[4];
    bool rok[4], cok[4];
    double dx[4], dy[4], dz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = tid + 256 * i;
        lr[i] = idx >> 4;
        lk[i] = idx & 15;
        rok[i] = row0 + lr[i] < M;
        cok[i] = lr[i] < ncol;
        const int pr = blk.y + (cok[i] ? lr[i] / NC : 0);
        comp[i] = lr[i] % NC;
        pc[i] = a.chk + int64_t(a.pairs[pr].x) * NC * M;
        dx[i] = NC == 4 ? a.delta[3 * pr] : 0.0;
        dy[i] = NC == 4 ? a.delta[3 * pr + 1] : 0.0;
        dz[i] = NC == 4 ? a.delta[3 * pr + 2] : 0.0;
    }
    // (prefetching the next K step into registers, as gemm_f64 does,
    // measured slower here: 0.70 against 0.57 ms for the 1M downward pass)
    for (int k0 = 0; k0 < M; k0 += 16) {
        double ra[4], rb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + lk[i];
            const bool kok = k < M;
            ra[i] = (rok[i] && kok) ? A[int64_t(row0 + lr[i]) * M + k] : 0.0;
            double b = 0.0;
            if (cok[i] && kok) {
                b = pc[i][comp[i] * M + k];
                if (NC == 4 && comp[i] == 3) b -= dx[i] * pc[i][k] + dy[i] * pc[i][M + k] + dz[i] * pc[i][2 * M + k];
            }
            rb[i] = b;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            As[lr[i] * 17 + lk[i]] = ra[i];
            Bs[lr[i] * 17 + lk[i]] = rb[i];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const int k = kk + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[(wr + 16 * i + (lane & 15)) * 17 + k];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[(wc + 16 * j + (lane & 15)) * 17 + k];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = wc + 16 * j + (lane & 15);
        if (col >= ncol) continue;
        const int pr = blk.y + col / NC, c = col % NC;
        double *o = a.chk + (int64_t(a.pairs[pr].y) * NC + c) * M;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = row0 + wr + 16 * i + (lane >> 4) + 4 * v;
                if (r < M) o[r] += acc[i][j][v];
            }
    }
}

// ------------------------------------------------------------------ translation reduce
// chk[dst][c][m] (+)= sum over pairs p of scale_p * (Y_p[c][m] - [c == 3] delta_p . Y_p[0..2][m])
// (the Psi origin shift; Laplace problems have one component and no shift).
template <int NC>
__global__ __launch_bounds__(1024) void reduce_kernel(ReduceArgs a) {
    const int task = blockIdx.x;
    const int dst = a.dst[task];
    const int p0 = a.off[task], p1 = a.off[task + 1];
    constexpr int nc = NC;
    constexpr int U = 4;                     // pairs whose loads are issued together
    for (int m = threadIdx.x; m < a.M; m += blockDim.x) {
        double acc[4] = {0, 0, 0, 0};
        for (int q0 = p0; q0 < p1; q0 += U) {
            float y[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q0 + u >= p1) break;
                const float *Y = a.Y + int64_t(a.pair[q0 + u]) * nc * a.ys + m;
#pragma unroll
                for (int c = 0; c < nc; ++c) y[u][c] = Y[c * a.ys];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = q0 + u;
                if (p >= p1) break;
                const double s = a.scale[p];
                if (nc == 4) {
                    const double y0 = y[u][0], y1 = y[u][1], y2 = y[u][2], y3 = y[u][3];
                    const float *dl = a.delta + 3 * int64_t(p);
                    acc[0] += s * y0;
                    acc[1] += s * y1;
                    acc[2] += s * y2;
                    acc[3] += s * (y3 - (double(dl[0]) * y0 + double(dl[1]) * y1 + double(dl[2]) * y2));
                } else {
                    acc[0] += s * double(y[u][0]);
                }
            }
        }
        for (int c = 0; c < nc; ++c) {
            double *o = a.chk + (int64_t(dst) * nc + c) * a.M + m;
            *o = a.accumulate ? *o + acc[c] : acc[c];
        }
    }
}

// Compressed translations: the pairs' Y columns hold kc coefficients in the
// basis U_k.  The block sums them per destination (as reduce_kernel) into
// LDS, then expands y = U_k * coefficients at the M check points.
template <int NC>
__global__ __launch_bounds__(1024) void reduce_expand_kernel(ReduceArgs a) {
    __shared__ double cf[kMaxCompressed * NC];        // [k][c]
    const int task = blockIdx.x;
    const int dst = a.dst[task];
    const int p0 = a.off[task], p1 = a.off[task + 1];
    constexpr int U = 4;
    for (int k = threadIdx.x; k < a.kc; k += blockDim.x) {
        double acc[4] = {0, 0, 0, 0};
        for (int q0 = p0; q0 < p1; q0 += U) {
            float y[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q0 + u >= p1) break;
                const float *Y = a.Y + int64_t(a.pair[q0 + u]) * NC * a.ys + k;
#pragma unroll
                for (int c = 0; c < NC; ++c) y[u][c] = Y[c * a.ys];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = q0 + u;
                if (p >= p1) break;
                const double s = a.scale[p];
                if (NC == 4) {
                    const double y0 = y[u][0], y1 = y[u][1], y2 = y[u][2], y3 = y[u][3];
                    const float *dl = a.delta + 3 * int64_t(p);
                    acc[0] += s * y0;
                    acc[1] += s * y1;
                    acc[2] += s * y2;
                    acc[3] += s * (y3 - (double(dl[0]) * y0 + double(dl[1]) * y1 + double(dl[2]) * y2));
                } else {
                    acc[0] += s * double(y[u][0]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) cf[k * NC + c] = acc[c];
    }
    __syncthreads();
    for (int m = threadIdx.x; m < a.M; m += blockDim.x) {
        double v[4] = {0, 0, 0, 0};
        const float *ut = a.basis_t + m;                 // U_k^T [kc][Mp], column m
        for (int k = 0; k < a.kc; ++k) {
            const double u = ut[int64_t(k) * a.Mp];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] += u * cf[k * NC + c];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double *o = a.chk + (int64_t(dst) * NC + c) * a.M + m;
            *o = a.accumulate ? *o + v[c] : v[c];
        }
    }
}

// periodic far images: chk[root][c][i] += sum_j T[i][j] dens[root][c][j]
__global__ __launch_bounds__(256) void periodic_kernel(const double *__restrict__ T, const float *__restrict__ dens,
                                                       double *__restrict__ chk, int M, int Mp, int nc, int root) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < M * nc; i += blockDim.x * gridDim.x) {
        int c = i / M, r = i % M;
        const float *d = dens + (int64_t(root) * nc + c) * Mp;
        double s = 0.0;
        for (int j = 0; j < M; ++j) s += T[int64_t(r) * M + j] * double(d[j]);
        chk[(int64_t(root) * nc + c) * M + r] += s;
    }
}

// ------------------------------------------------------------------ L2T / M2T
// Target values from equivalent densities.  A task is up to 256 targets of a
// leaf against a slice of its equivalent-point sets: the leaf's own downward
// set (radius a_out, entry code kLocalSet) and upward sets of W-list boxes
// (radius a_in, image shift in the code), staged through LDS 256 points at a
// time.  Partial sums per task, added by the combine step.
template <class E>
__global__ __launch_bounds__(256) void l2t_kernel(L2TArgs a) {
    constexpr int NC = E::NC;
    constexpr int NV = 3 + NC;
    __shared__ float tile[256 * NV];
    const int4 task = a.tasks[blockIdx.x];
    const int4 ch = a.chunks[task.x];
    const int leaf = ch.x;
    const int t = ch.y + int(threadIdx.x);
    const bool active = t < ch.z;
    const int ti = active ? t : ch.z - 1;
    const double4 cb = a.geom[leaf];
    const float4 p0 = reinterpret_cast<const float4 *>(a.trg)[2 * ti];
    const float4 p1 = reinterpret_cast<const float4 *>(a.trg)[2 * ti + 1];
    // target relative to the leaf centre
    const float xr = float((double(p0.x) - cb.x) + double(p1.x));
    const float yr = float((double(p0.y) - cb.y) + double(p1.y));
    const float zr = float((double(p0.z) - cb.z) + double(p1.z));
    double acc[E::NACC];
#pragma unroll
    for (int k = 0; k < E::NACC; ++k) acc[k] = 0.0;
    for (int e = task.y; e < task.z; ++e) {
        const int2 en = a.ent[e];
        const int box = en.x;
        const bool local = en.y == kLocalSet;
        const double4 g = a.geom[box];
        double ox = 0, oy = 0, oz = 0;      // set's box centre (image) relative to the leaf centre
        if (!local) {
            ox = (g.x + shift_comp(en.y, 0)) - cb.x;
            oy = (g.y + shift_comp(en.y, 1)) - cb.y;
            oz = (g.z + shift_comp(en.y, 2)) - cb.z;
        }
        const double rad = (local ? a.alpha_out : a.alpha_in) * 0.5 * g.w;
        const float *dens = local ? a.dn_dens : a.up_dens;
        // s = psi - (x - c_origin).phi with the origin at the set's box centre
        const float cx = xr - float(ox), cy = yr - float(oy), cz = zr - float(oz);
        float part[E::NACC];
#pragma unroll
        for (int k = 0; k < E::NACC; ++k) part[k] = 0.0f;
        for (int j0 = 0; j0 < a.M; j0 += 256) {
            const int n = min(256, a.M - j0);
            __syncthreads();
            if (int(threadIdx.x) < n) {
                const int m = j0 + threadIdx.x;
                float *o = tile + threadIdx.x * NV;
                o[0] = float(ox + rad * a.grid[3 * m]);
                o[1] = float(oy + rad * a.grid[3 * m + 1]);
                o[2] = float(oz + rad * a.grid[3 * m + 2]);
                for (int c = 0; c < NC; ++c) o[3 + c] = dens[(int64_t(box) * NC + c) * a.Mp + m];
            }
            __syncthreads();
            if (!active) continue;
#pragma unroll 2
            for (int j = 0; j < n; ++j) {
                const float *y = tile + j * NV;
                // equivalent points lie outside the target leaf: r > 0
                float dx = xr - y[0], dy = yr - y[1], dz = zr - y[2];
                float ri = __builtin_amdgcn_rsqf(dot3(dx, dy, dz, dx, dy, dz));
                float s = NC == 4 ? y[6] - dot3(cx, cy, cz, y[3], y[4], y[5]) : 0.0f;
                E::eq(dx, dy, dz, ri, y + 3, s, part);
            }
        }
#pragma unroll
        for (int k = 0; k < E::NACC; ++k) acc[k] += double(part[k]);
    }
    if (active) {
        double *o = a.part + (int64_t(blockIdx.x) * 256 + threadIdx.x) * E::NACC;
#pragma unroll
        for (int k = 0; k < E::NACC; ++k) o[k] = acc[k];
    }
}

// ------------------------------------------------------------------ combine + un-permute
// One block per target chunk.  user[perm[t]][k] = scale_k * (sum of the
// chunk's P2P task partials + sum of its L2T task partials) at component
// src_k (a negative src_k gives 0); symmetric tensors are expanded by the map.
__global__ __launch_bounds__(256) void combine_kernel(CombineArgs a) {
    const int4 ch = a.chunks[blockIdx.x];
    const int4 tr = a.chunk_tasks[blockIdx.x];     // {p2p t0, t1, l2t t0, t1}
    const int t = ch.y + int(threadIdx.x);
    if (t >= ch.z) return;
    double v[kMaxAcc];
    for (int k = 0; k < a.nacc; ++k) v[k] = 0.0;
    for (int q = tr.x; q < tr.y; ++q) {
        const double *p = a.near + (int64_t(q) * 256 + threadIdx.x) * a.nacc;
        for (int k = 0; k < a.nacc; ++k) v[k] += p[k];
    }
    for (int q = tr.z; q < tr.w; ++q) {
        const double *p = a.far + (int64_t(q) * 256 + threadIdx.x) * a.nacc;
        for (int k = 0; k < a.nacc; ++k) v[k] += p[k];
    }
    double *o = a.out + int64_t(a.perm[t]) * a.kt;
    for (int k = 0; k < a.kt; ++k) {
        const int s = a.map.src[k];
        o[k] = s >= 0 ? a.map.scale[k] * v[s] : 0.0;
    }
}

// ------------------------------------------------------------------ FP64 direct sum (error judge)
template <class K>
__global__ __launch_bounds__(256) void direct_f64_kernel(DirectArgs a) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool active = t < a.n_trg;
    const int64_t ti = active ? t : 0;
    const int slice = blockIdx.y;
    const double x0 = a.trg[3 * ti], x1 = a.trg[3 * ti + 1], x2 = a.trg[3 * ti + 2];
    double acc[kMaxAcc] = {};
    __shared__ double ys[256 * 13];
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t ns = pass == 0 ? a.n_sl : a.n_dl;
        const double *xyz = pass == 0 ? a.sl : a.dl;
        const double *val = pass == 0 ? a.sl_val : a.dl_val;
        const int kv = pass == 0 ? a.k_sl : a.k_dl;
        const int64_t s0 = ns * slice / a.slices, s1 = ns * (slice + 1) / a.slices;
        for (int64_t j0 = s0; j0 < s1; j0 += 256) {
            const int n = int(min(int64_t(256), s1 - j0));
            __syncthreads();
            if (int(threadIdx.x) < n) {
                double *o = ys + threadIdx.x * 13;
                const int64_t j = j0 + threadIdx.x;
                o[0] = xyz[3 * j]; o[1] = xyz[3 * j + 1]; o[2] = xyz[3 * j + 2];
                for (int k = 0; k < kv; ++k) o[3 + k] = val[j * kv + k];
            }
            __syncthreads();
            if (!active) continue;
            for (int j = 0; j < n; ++j) {
                const double *y = ys + j * 13;
                double r[3] = {x0 - y[0], x1 - y[1], x2 - y[2]};
                K::pair(pass, r, y + 3, acc);
            }
        }
    }
    if (!active) return;
    double *o = a.slices > 1 ? a.work + (int64_t(slice) * a.n_trg + t) * a.k_trg : a.out + t * a.k_trg;
    for (int k = 0; k < a.k_trg; ++k) o[k] = acc[k];
}

// out[i] = sum over slices, in slice order, of work[slice][i]
__global__ void direct_slices_reduce(int64_t n, int slices, const double *__restrict__ work,
                                     double *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int q = 0; q < slices; ++q) s += work[int64_t(q) * n + i];
    out[i] = s;
}

// FP64 pair functions in user layouts (outputs already scaled).
struct F64Stokeslet {
    __device__ static void pair(int, const double *r, const double *v, double *a) {
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        double ri = 1.0 / sqrt(rr), ri3 = ri / rr;
        double rf = r[0] * v[0] + r[1] * v[1] + r[2] * v[2];
        for (int i = 0; i < 3; ++i) a[i] += kInv8Pi * (v[i] * ri + r[i] * rf * ri3);
    }
};
struct F64StokesReg {     // v = f, eps
    __device__ static void pair(int, const double *r, const double *v, double *a) {
        const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double e2 = v[3] * v[3], s = rr + e2;
        if (s == 0.0) return;
        const double h2 = 1.0 / (s * sqrt(s)), h1 = (rr + 2.0 * e2) * h2;
        const double rf = r[0] * v[0] + r[1] * v[1] + r[2] * v[2];
        for (int i = 0; i < 3; ++i) a[i] += kInv8Pi * (h1 * v[i] + h2 * rf * r[i]);
    }
};
struct F64StokesRegFT {   // v = f, t, eps -> u, omega
    __device__ static void pair(int, const double *r, const double *v, double *a) {
        const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double e2 = v[6] * v[6], s = rr + e2;
        if (s == 0.0) return;
        const double sq = sqrt(s), s3 = s * sq, s5 = s3 * s, s7 = s5 * s;
        const double h1 = (rr + 2.0 * e2) / s3, h2 = 1.0 / s3, q = (2.0 * rr + 5.0 * e2) / s5;
        const double d1 = (10.0 * e2 * e2 - 7.0 * e2 * rr - 2.0 * rr * rr) / s7, d2 = (21.0 * e2 + 6.0 * rr) / s7;
        const double *f = v, *t = v + 3;
        const double rf = r[0] * f[0] + r[1] * f[1] + r[2] * f[2], rt = r[0] * t[0] + r[1] * t[1] + r[2] * t[2];
        const double txr[3] = {t[1] * r[2] - t[2] * r[1], t[2] * r[0] - t[0] * r[2], t[0] * r[1] - t[1] * r[0]};
        const double fxr[3] = {f[1] * r[2] - f[2] * r[1], f[2] * r[0] - f[0] * r[2], f[0] * r[1] - f[1] * r[0]};
        for (int i = 0; i < 3; ++i) {
            a[i] += kInv8Pi * (h1 * f[i] + h2 * rf * r[i] + 0.5 * q * txr[i]);
            a[3 + i] += kInv8Pi * (0.5 * q * fxr[i] + 0.25 * (d1 * t[i] + d2 * rt * r[i]));
        }
    }
};
struct F64LapHess {       // SL q, DL d -> phi, grad phi, Hessian (xx, xy, xz, yy, yz, zz)
    __device__ static void pair(int pass, const double *r, const double *v, double *a) {
        const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        const double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr, i7 = i5 / rr;
        int k = 4;
        if (pass == 0) {
            const double q = v[0];
            a[0] += kInv4Pi * q * i1;
            for (int i = 0; i < 3; ++i) a[1 + i] -= kInv4Pi * q * r[i] * i3;
            for (int i = 0; i < 3; ++i)
                for (int j = i; j < 3; ++j) a[k++] += kInv4Pi * q * (3.0 * r[i] * r[j] * i5 - (i == j ? i3 : 0.0));
        } else {
            const double dr = v[0] * r[0] + v[1] * r[1] + v[2] * r[2];
            a[0] += kInv4Pi * dr * i3;
            for (int i = 0; i < 3; ++i) a[1 + i] += kInv4Pi * (v[i] * i3 - 3.0 * dr * r[i] * i5);
            for (int i = 0; i < 3; ++i)
                for (int j = i; j < 3; ++j)
                    a[k++] += kInv4Pi * (-3.0 * (v[j] * r[i] + v[i] * r[j] + (i == j ? dr : 0.0)) * i5 +
                                         15.0 * dr * r[i] * r[j] * i7);
        }
    }
};
// quadrupole Q (9, row-major): phi, grad phi, Hessian from w = Q^s r, B = r.w
struct F64LapQuad {
    __device__ static void pair(int, const double *r, const double *v, double *a) {
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        double ri = 1.0 / sqrt(rr), ri3 = ri / rr, ri5 = ri3 / rr, ri7 = ri5 / rr, ri9 = ri7 / rr;
        double Qs[3][3], w[3], tr = v[0] + v[4] + v[8];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) Qs[j][k] = 0.5 * (v[3 * j + k] + v[3 * k + j]);
        for (int j = 0; j < 3; ++j) w[j] = Qs[j][0] * r[0] + Qs[j][1] * r[1] + Qs[j][2] * r[2];
        const double B = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
        a[0] += kInv4Pi * (3.0 * B * ri5 - tr * ri3);
        for (int i = 0; i < 3; ++i) a[1 + i] += kInv4Pi * (6.0 * w[i] * ri5 + (3.0 * tr * ri5 - 15.0 * B * ri7) * r[i]);
        int k = 4;
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j)
                a[k++] += kInv4Pi * (6.0 * Qs[i][j] * ri5 - 30.0 * (w[i] * r[j] + r[i] * w[j]) * ri7 +
                                     (105.0 * B * ri9 - 15.0 * tr * ri7) * r[i] * r[j] +
                                     (i == j ? 3.0 * tr * ri5 - 15.0 * B * ri7 : 0.0));
    }
};
struct F64RPY {
    __device__ static void pair(int, const double *r, const double *v, double *a) {
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        double ri = 1.0 / sqrt(rr), ri3 = ri / rr, ri5 = ri3 / rr;
        double rf = r[0] * v[0] + r[1] * v[1] + r[2] * v[2], b2 = v[3] * v[3];
        for (int i = 0; i < 3; ++i) {
            a[i] += kInv8Pi * ((ri + b2 / 3.0 * ri3) * v[i] + (ri3 - b2 * ri5) * rf * r[i]);
            a[3 + i] += kInv8Pi * (2.0 * ri3 * v[i] - 6.0 * rf * ri5 * r[i]);
        }
    }
};
struct F64Lap {
    __device__ static void pair(int pass, const double *r, const double *v, double *a) {
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        double ri = 1.0 / sqrt(rr), ri3 = ri / rr, ri5 = ri3 / rr;
        if (pass == 0) {
            a[0] += kInv4Pi * v[0] * ri;
            for (int i = 0; i < 3; ++i) a[1 + i] -= kInv4Pi * v[0] * r[i] * ri3;
        } else {
            double dr = v[0] * r[0] + v[1] * r[1] + v[2] * r[2];
            a[0] += kInv4Pi * dr * ri3;
            for (int i = 0; i < 3; ++i) a[1 + i] += kInv4Pi * (v[i] * ri3 - 3.0 * dr * r[i] * ri5);
        }
    }
};
struct F64PVel {
    __device__ static void pair(int pass, const double *r, const double *v, double *a) {
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        double ri = 1.0 / sqrt(rr), ri3 = ri / rr, ri5 = ri3 / rr;
        if (pass == 0) {
            double rf = r[0] * v[0] + r[1] * v[1] + r[2] * v[2];
            a[0] += kInv4Pi * rf * ri3;
            for (int i = 0; i < 3; ++i) a[1 + i] += kInv8Pi * (v[i] * ri + r[i] * (rf - v[3]) * ri3);
        } else {
            double A = 0, tr = v[0] + v[4] + v[8];
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) A += r[j] * v[3 * j + k] * r[k];
            a[0] += kInv4Pi * (-3.0 * A * ri5 + tr * ri3);
            for (int i = 0; i < 3; ++i) a[1 + i] += -3.0 * kInv8Pi * r[i] * A * ri5;
        }
    }
};
// (p, u, grad p, grad u) (16), or with LAP (p, u, lap u) (7)
template <bool LAP>
struct F64PVelDeriv {
    __device__ static void pair(int pass, const double *r, const double *v, double *a) {
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        double ri = 1.0 / sqrt(rr), ri3 = ri / rr, ri5 = ri3 / rr, ri7 = ri5 / rr;
        if (pass == 0) {
            const double rf = r[0] * v[0] + r[1] * v[1] + r[2] * v[2], g = rf - v[3];
            a[0] += kInv4Pi * rf * ri3;
            for (int i = 0; i < 3; ++i) {
                a[1 + i] += kInv8Pi * (v[i] * ri + r[i] * g * ri3);
                a[4 + i] += kInv8Pi * (2.0 * v[i] * ri3 - 6.0 * rf * r[i] * ri5);
                if (!LAP)
                    for (int j = 0; j < 3; ++j)
                        a[7 + 3 * i + j] += kInv8Pi * ((r[i] * v[j] - v[i] * r[j] + (i == j ? g : 0.0)) * ri3 -
                                                       3.0 * g * r[i] * r[j] * ri5);
            }
        } else {
            double w[3], tr = v[0] + v[4] + v[8];
            for (int j = 0; j < 3; ++j) {
                w[j] = 0;
                for (int k = 0; k < 3; ++k) w[j] += 0.5 * (v[3 * j + k] + v[3 * k + j]) * r[k];
            }
            const double A = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
            a[0] += kInv4Pi * (-3.0 * A * ri5 + tr * ri3);
            for (int i = 0; i < 3; ++i) {
                a[1 + i] += -3.0 * kInv8Pi * r[i] * A * ri5;
                a[4 + i] += kInv8Pi * (-12.0 * w[i] * ri5 + (30.0 * A * ri7 - 6.0 * tr * ri5) * r[i]);
                if (!LAP)
                    for (int j = 0; j < 3; ++j)
                        a[7 + 3 * i + j] += -3.0 * kInv8Pi * ((i == j ? A * ri5 : 0.0) + 2.0 * r[i] * w[j] * ri5 -
                                                              5.0 * r[i] * r[j] * A * ri7);
            }
        }
    }
};
struct F64Traction {
    __device__ static void pair(int pass, const double *r, const double *v, double *a) {
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (rr == 0.0) return;
        double ri = 1.0 / sqrt(rr), ri3 = ri / rr, ri5 = ri3 / rr, ri7 = ri5 / rr;
        if (pass == 0) {
            double rf = r[0] * v[0] + r[1] * v[1] + r[2] * v[2], q = v[3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    a[3 * i + j] += kInv4Pi * (3.0 * (q - rf) * r[i] * r[j] * ri5 - (i == j ? q * ri3 : 0.0));
        } else {
            double w[3], tr = v[0] + v[4] + v[8];
            for (int j = 0; j < 3; ++j) {
                w[j] = 0;
                for (int k = 0; k < 3; ++k) w[j] += 0.5 * (v[3 * j + k] + v[3 * k + j]) * r[k];
            }
            double A = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    a[3 * i + j] += kInv4Pi * (-(i == j ? tr * ri3 : 0.0) - 3.0 * (r[i] * w[j] + w[i] * r[j]) * ri5 +
                                               15.0 * A * r[i] * r[j] * ri7);
        }
    }
};

// ------------------------------------------------------------------ launchers
static inline int blocks_for(int64_t n, int b) { return int((n + b - 1) / b); }

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int nb = std::min<int64_t>(blocks_for(n, 256), 4096);
    hipLaunchKernelGGL(fill_f64, dim3(nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int nb = std::min<int64_t>(blocks_for(n, 256), 4096);
    hipLaunchKernelGGL(fill_f32, dim3(nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_pack_sources(int64_t n, const double *xyz, const int32_t *perm, double3 origin, double inv_len,
                               int rec, float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_sources, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, xyz, perm, origin, inv_len, rec,
                       out);
    return hipGetLastError();
}

hipError_t launch_pack_targets(int64_t n, const double *xyz, const int32_t *perm, double3 origin,
                               double inv_len, float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_targets, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, xyz, perm, origin, inv_len,
                       out);
    return hipGetLastError();
}

hipError_t launch_rel_check(int ntasks, const P2PArgs &a, int rec, unsigned *flag, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(rel_check_kernel, dim3(ntasks), dim3(256), 0, s, a, rec, flag);
    return hipGetLastError();
}

hipError_t launch_p2p(int kernel, int ntasks, const P2PArgs &a, bool exact_r, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    if (exact_r && kernel == kStokeslet) {
        hipLaunchKernelGGL(p2p_kernel<DStokesletExact>, dim3(ntasks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    switch (kernel) {
        case kStokeslet: hipLaunchKernelGGL(p2p_kernel<DStokeslet>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kRPY: hipLaunchKernelGGL(p2p_kernel<DRPY>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kLapPGrad: hipLaunchKernelGGL(p2p_kernel<DLapPGrad>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kPVel: hipLaunchKernelGGL(p2p_kernel<DPVel>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kTraction: hipLaunchKernelGGL(p2p_kernel<DTraction>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kStokesRegVel: hipLaunchKernelGGL(p2p_kernel<DStokesReg>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kLapPGradGrad: hipLaunchKernelGGL(p2p_kernel<DLapPGradGrad>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kStokesRegVelOmega:
            hipLaunchKernelGGL(p2p_kernel<DStokesRegFT>, dim3(ntasks), dim3(256), 0, s, a);
            break;
        case kPVelGrad: hipLaunchKernelGGL(p2p_kernel<DPVelDeriv<true>>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kLapQPGradGrad:
            hipLaunchKernelGGL(p2p_kernel<DLapQPGradGrad>, dim3(ntasks), dim3(256), 0, s, a);
            break;
        case kPVelLaplacian:
            hipLaunchKernelGGL(p2p_kernel<DPVelDeriv<false>>, dim3(ntasks), dim3(256), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Check points per thread: the count in {2, 3, 4} that pads the fewest
// lanes (ties to the larger count, which reads the LDS tile less often).
static int s2c_points_per_thread(int M) {
    int best = 2, best_slots = 1 << 30;
    for (int pts = 2; pts <= 4; ++pts) {
        const int slots = pts * (((M + pts - 1) / pts + 63) / 64 * 64);
        if (slots <= best_slots) best = pts, best_slots = slots;
    }
    return best;
}

template <int SRC>
static void launch_s2c_kind(int ntasks, const S2CArgs &a, hipStream_t s) {
    const int pts = a.M > 4096 ? 0 : s2c_points_per_thread(a.M);
    const int nthr = ((a.M + pts - 1) / pts + 63) / 64 * 64;
    switch (pts) {
        case 2: hipLaunchKernelGGL((s2c_kernel<SRC, 2>), dim3(ntasks), dim3(nthr), 0, s, a); break;
        case 3: hipLaunchKernelGGL((s2c_kernel<SRC, 3>), dim3(ntasks), dim3(nthr), 0, s, a); break;
        default: hipLaunchKernelGGL((s2c_kernel<SRC, 4>), dim3(ntasks), dim3(nthr), 0, s, a); break;
    }
}

hipError_t launch_s2c(int src_kind, int ntasks, const S2CArgs &a, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    if (a.M < 1 || a.M > 4096) return hipErrorInvalidValue;
    switch (src_kind) {
        case 0: launch_s2c_kind<0>(ntasks, a, s); break;
        case 1: launch_s2c_kind<1>(ntasks, a, s); break;
        case 2: launch_s2c_kind<2>(ntasks, a, s); break;
        case 3: launch_s2c_kind<3>(ntasks, a, s); break;
        case 4: launch_s2c_kind<4>(ntasks, a, s); break;
        case 5: launch_s2c_kind<5>(ntasks, a, s); break;
        case 7: launch_s2c_kind<7>(ntasks, a, s); break;
        case 8: launch_s2c_kind<8>(ntasks, a, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stage_sources(int src_kind, int nleaves, const int *leaves, const int2 *box_range,
                                const double4 *geom, const float *src, int rec, float *out, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
    const int need = src_kind == 2 ? 7 : src_kind == 1 || src_kind == 4 ? 10 : src_kind == 5 || src_kind == 8 ? 12
                   : src_kind == 7 ? 13 : 9;
    if (rec < need) return hipErrorInvalidValue;
    dim3 g(nleaves), b(256);
    switch (src_kind) {
        case 0: hipLaunchKernelGGL(stage_sources_kernel<0>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        case 1: hipLaunchKernelGGL(stage_sources_kernel<1>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        case 2: hipLaunchKernelGGL(stage_sources_kernel<2>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        case 3: hipLaunchKernelGGL(stage_sources_kernel<3>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        case 4: hipLaunchKernelGGL(stage_sources_kernel<4>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        case 5: hipLaunchKernelGGL(stage_sources_kernel<5>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        case 7: hipLaunchKernelGGL(stage_sources_kernel<7>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        case 8: hipLaunchKernelGGL(stage_sources_kernel<8>, g, b, 0, s, leaves, box_range, geom, src, rec, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// shapes the grouped GEMMs assume: R, K multiples of 32; live extents within
// them (Mk a multiple of 16); columns at least as long as the operator sides
static bool gemm_args_ok(const GemmArgs &a) {
    return a.R > 0 && a.K > 0 && a.R % 32 == 0 && a.K % 32 == 0 && a.Mr >= 1 && a.Mr <= a.R && a.Mk >= 1 &&
           a.Mk <= a.K && a.Mk % 16 == 0 && a.xs >= a.K && a.ys >= a.R && a.opsz >= int64_t(a.R) * a.K;
}

hipError_t launch_gemm_f32(int ntiles, const GemmArgs &a, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (!gemm_args_ok(a)) return hipErrorInvalidValue;
    // 160-row operators (rank 160, the learned plans' translations): the
    // row-strip kernel, which computes no padding rows (measured 1.64 against
    // 1.72 ms for the 1M V-list launch); at 224 rows the 256-row tile of
    // gemm_f32_mfma<4> measured faster (0.67 against 0.76 ms), and 192 rows
    // need no padding
    if (a.R == 160) {
        hipLaunchKernelGGL(gemm_f32_strip<5>, dim3(ntiles), dim3(640), 0, s, a);
        return hipGetLastError();
    }
    // row tiles of 64 WR rows (WR = 2..4): the fewest padded rows, then the
    // fewest row blocks (each row block reads the column tile again)
    int wr = 2;
    for (int w = 3; w <= 4; ++w) {
        const int pad_w = (a.R + 64 * w - 1) / (64 * w) * 64 * w, pad_r = (a.R + 64 * wr - 1) / (64 * wr) * 64 * wr;
        if (pad_w < pad_r || (pad_w == pad_r && pad_w / (64 * w) < pad_r / (64 * wr))) wr = w;
    }
    const int rblocks = (a.R + 64 * wr - 1) / (64 * wr);
    if (wr == 4) hipLaunchKernelGGL(gemm_f32_mfma<4>, dim3(ntiles, rblocks), dim3(512), 0, s, a);
    else if (wr == 3) hipLaunchKernelGGL(gemm_f32_mfma<3>, dim3(ntiles, rblocks), dim3(384), 0, s, a);
    else hipLaunchKernelGGL(gemm_f32_mfma<2>, dim3(ntiles, rblocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16x3(int ntiles, const GemmArgs &a, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (!gemm_args_ok(a)) return hipErrorInvalidValue;
    if (a.R == 160) {
        hipLaunchKernelGGL(gemm_bf16x3_strip<5>, dim3(ntiles), dim3(640), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(gemm_bf16x3_mfma, dim3(ntiles, (a.R + kGT - 1) / kGT), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm_f64(const Gemm64Args &a, double *C, hipStream_t s) {
    if (a.ncol <= 0 || a.R <= 0) return hipSuccess;
    hipLaunchKernelGGL(gemm_f64<double>, dim3((a.R + 63) / 64, (a.ncol + 63) / 64), dim3(256), 0, s, a, C);
    return hipGetLastError();
}

hipError_t launch_gemm_f64_to_f32(const Gemm64Args &a, float *C, hipStream_t s) {
    if (a.ncol <= 0 || a.R <= 0) return hipSuccess;
    hipLaunchKernelGGL(gemm_f64<float>, dim3((a.R + 63) / 64, (a.ncol + 63) / 64), dim3(256), 0, s, a, C);
    return hipGetLastError();
}

hipError_t launch_reduce(int ntasks, const ReduceArgs &a, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    if (a.ncomp != 1 && a.ncomp != 4) return hipErrorInvalidValue;
    if (a.kc > 0) {
        if (a.kc > kMaxCompressed || a.basis_t == nullptr || a.ys < a.kc) return hipErrorInvalidValue;
        const int nthr = std::min(1024, (std::max(a.M, a.kc) + 63) / 64 * 64);
        if (a.ncomp == 4) hipLaunchKernelGGL(reduce_expand_kernel<4>, dim3(ntasks), dim3(nthr), 0, s, a);
        else hipLaunchKernelGGL(reduce_expand_kernel<1>, dim3(ntasks), dim3(nthr), 0, s, a);
    } else {
        if (a.ys < a.M) return hipErrorInvalidValue;
        const int nthr = std::min(1024, (a.M + 63) / 64 * 64);
        if (a.ncomp == 4) hipLaunchKernelGGL(reduce_kernel<4>, dim3(ntasks), dim3(nthr), 0, s, a);
        else hipLaunchKernelGGL(reduce_kernel<1>, dim3(ntasks), dim3(nthr), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_l2l_check(int nblocks, int ncomp, const L2LArgs &a, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (a.M < 1 || (ncomp != 1 && ncomp != 4)) return hipErrorInvalidValue;
    dim3 g((a.M + 63) / 64, nblocks);
    if (ncomp == 4) hipLaunchKernelGGL(l2l_check_kernel<4>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(l2l_check_kernel<1>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_periodic(const double *T, const float *dens, double *chk, int M, int Mp, int nc, int root,
                           hipStream_t s) {
    hipLaunchKernelGGL(periodic_kernel, dim3(blocks_for(int64_t(M) * nc, 256)), dim3(256), 0, s, T, dens, chk,
                       M, Mp, nc, root);
    return hipGetLastError();
}

hipError_t launch_l2t(int kernel, int ntasks, const L2TArgs &a, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    switch (kernel) {
        case kStokeslet: hipLaunchKernelGGL(l2t_kernel<EStokeslet>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kRPY: hipLaunchKernelGGL(l2t_kernel<ERPY>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kLapPGrad: hipLaunchKernelGGL(l2t_kernel<ELapPGrad>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kPVel: hipLaunchKernelGGL(l2t_kernel<EPVel>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kTraction: hipLaunchKernelGGL(l2t_kernel<ETraction>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kStokesRegVel: hipLaunchKernelGGL(l2t_kernel<EStokeslet>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kLapPGradGrad: hipLaunchKernelGGL(l2t_kernel<ELapPGradGrad>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kStokesRegVelOmega: hipLaunchKernelGGL(l2t_kernel<EStokesFT>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kPVelGrad: hipLaunchKernelGGL(l2t_kernel<EPVelDeriv<true>>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kLapQPGradGrad: hipLaunchKernelGGL(l2t_kernel<ELapPGradGrad>, dim3(ntasks), dim3(256), 0, s, a); break;
        case kPVelLaplacian:
            hipLaunchKernelGGL(l2t_kernel<EPVelDeriv<false>>, dim3(ntasks), dim3(256), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_combine(int nchunks, const CombineArgs &a, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(combine_kernel, dim3(nchunks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_s2c_reduce(int ndst, const S2CReduceArgs &a, hipStream_t s) {
    if (ndst <= 0) return hipSuccess;
    hipLaunchKernelGGL(s2c_reduce, dim3(ndst), dim3(256), 0, s, a);
    return hipGetLastError();
}

int direct_f64_slices(int64_t n_trg, int64_t n_src) {
    const int64_t bt = std::max<int64_t>(1, blocks_for(n_trg, 256));
    int64_t q = (2048 + bt - 1) / bt;
    q = std::min<int64_t>(q, std::max<int64_t>(1, n_src / 1024));
    return int(std::max<int64_t>(1, std::min<int64_t>(q, 256)));
}

hipError_t launch_direct_f64(int kernel, const DirectArgs &a, hipStream_t s) {
    if (a.n_trg <= 0) return hipSuccess;
    if (a.slices < 1 || a.slices > 256 || (a.slices > 1 && a.work == nullptr)) return hipErrorInvalidValue;
    dim3 g(blocks_for(a.n_trg, 256), a.slices);
    switch (kernel) {
        case kStokeslet: hipLaunchKernelGGL(direct_f64_kernel<F64Stokeslet>, g, dim3(256), 0, s, a); break;
        case kRPY: hipLaunchKernelGGL(direct_f64_kernel<F64RPY>, g, dim3(256), 0, s, a); break;
        case kLapPGrad: hipLaunchKernelGGL(direct_f64_kernel<F64Lap>, g, dim3(256), 0, s, a); break;
        case kPVel: hipLaunchKernelGGL(direct_f64_kernel<F64PVel>, g, dim3(256), 0, s, a); break;
        case kTraction: hipLaunchKernelGGL(direct_f64_kernel<F64Traction>, g, dim3(256), 0, s, a); break;
        case kStokesRegVel: hipLaunchKernelGGL(direct_f64_kernel<F64StokesReg>, g, dim3(256), 0, s, a); break;
        case kLapPGradGrad: hipLaunchKernelGGL(direct_f64_kernel<F64LapHess>, g, dim3(256), 0, s, a); break;
        case kStokesRegVelOmega:
            hipLaunchKernelGGL(direct_f64_kernel<F64StokesRegFT>, g, dim3(256), 0, s, a);
            break;
        case kPVelGrad: hipLaunchKernelGGL(direct_f64_kernel<F64PVelDeriv<false>>, g, dim3(256), 0, s, a); break;
        case kLapQPGradGrad: hipLaunchKernelGGL(direct_f64_kernel<F64LapQuad>, g, dim3(256), 0, s, a); break;
        case kPVelLaplacian:
            hipLaunchKernelGGL(direct_f64_kernel<F64PVelDeriv<true>>, g, dim3(256), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    if (a.slices > 1) {
        const int64_t n = a.n_trg * a.k_trg;
        hipLaunchKernelGGL(direct_slices_reduce, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, a.slices, a.work, a.out);
    }
    return hipGetLastError();
}

bool p2p_uses_rel(int kernel) {
    switch (kernel) {
        case kStokeslet: return DStokeslet::REL;
        case kRPY: return DRPY::REL;
        case kLapPGrad: return DLapPGrad::REL;
        case kPVel: return DPVel::REL;
        case kTraction: return DTraction::REL;
        case kStokesRegVel: return DStokesReg::REL;
        case kLapPGradGrad: return DLapPGradGrad::REL;
        case kStokesRegVelOmega: return DStokesRegFT::REL;
        case kPVelGrad: return DPVelDeriv<true>::REL;
        case kLapQPGradGrad: return DLapQPGradGrad::REL;
        case kPVelLaplacian: return DPVelDeriv<false>::REL;
        default: return false;
    }
}

hipError_t launch_rel_positions(int nleaves, const int *leaves, const int2 *box_sl, const double4 *geom, int rec,
                                float *sl, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
    if (rec < 12) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rel_positions_kernel, dim3(nleaves), dim3(256), 0, s, leaves, box_sl, geom, rec, sl);
    return hipGetLastError();
}

}  // namespace kafmm
