// Per-pair arithmetic of every kernel, shared by the HIP kernels.
//
// r = x - y (target minus source), ri = 1/|r| (0 for r = 0), mu = 1.  The
// 1/(4 pi) and 1/(8 pi) prefactors are applied once per target by the
// callers (see the scale tables), not per pair.
//
// Direct (S->T) kernels, with their definitions:
//   Stokeslet   u  = (f/r + r (r.f)/r^3)                            [x 1/8pi] Sec. II.B
//   RegStokeslet u = H1 f + H2 r (r.f), s = r^2 + eps^2, H1 = (r^2 + 2 eps^2)/s^(3/2),
//               H2 = 1/s^(3/2)                                      [x 1/8pi] Sec. II.B
//   RegStokes FT u += (Q/2) t x r, omega = (Q/2) f x r + (D1 t + D2 (r.t) r)/4
//               (Q, D1, D2 of Sec. II.B's force-torque extension)     [x 1/8pi]
//   RPY         u  = (1/r + b^2/(3 r^3)) f + (1/r^3 - b^2/r^5) r (r.f)
//               lap u = 2 f/r^3 - 6 r (r.f)/r^5                     [x 1/8pi] Eq. RPYkernel
//   Laplace     phi = q/r + d.r/r^3, grad phi = -q r/r^3 + d/r^3 - 3 (d.r) r/r^5
//                                                                   [x 1/4pi] Sec. II.A
//   PVel SL     p = 2 (r.f)/r^3, u = (r^2 f + r (r.f) - q r)/r^3    [x 1/8pi] Eqs. stkslp, stkslvel
//   PVel DL     p = 2 (-3 A/r^5 + tr D/r^3), u = -3 r A/r^5, A = r.D.r
//                                                                   [x 1/8pi] Eqs. stkdlp, stkdlvel
//   PVel grad   SL d_j p = 2 (f_j/r^3 - 3 rf r_j/r^5), rf = r.f,
//               d_j u_i = r_i f_j/r^3 - f_i r_j/r^3 + delta_ij g/r^3 - 3 g r_i r_j/r^5, g = rf - q
//               DL d_j p = -12 w_j/r^5 + (30 A/r^7 - 6 tr D/r^5) r_j,
//               d_j u_i = -3 delta_ij A/r^5 - 6 r_i w_j/r^5 + 15 A r_i r_j/r^7
//               lap u = grad p for both (Stokes equations; the q r/r^3 part is harmonic)
//                                                                   [x 1/8pi] tab:implement
//   Laplace Q   phi = Q_jk d_j d_k (1/r) = 3 r.Q.r/r^5 - tr Q/r^3, with its
//               gradient and Hessian                                [x 1/4pi] Sec. II.A
//   Traction SL sigma = 3 (q - r.f) r r^T/r^5 - q I/r^3             [x 1/4pi] Eq. stressdef
//   Traction DL sigma = -tr D I/r^3 - 3 (r w^T + w r^T)/r^5 + 15 A r r^T/r^7, w = D^s r
//                                                                   [x 1/4pi] Eq. stressdef
// Symmetric 3x3 results are accumulated as (xx, xy, xz, yy, yz, zz).
//
// ML-tree (4-Laplace) representation of the Stokes kernels.  With Laplace
// fields Phi_j and Psi of charges (and dipoles) carried relative to a box
// origin c:
//   u_i = 1/2 [Phi_i - (x - c)_j d_i Phi_j + d_i Psi]
//   p   = -d_j Phi_j,        lap u_i = -d_i d_j Phi_j,
//   sigma_ij = -p delta_ij + d_i d_j [Psi - (x - c)_l Phi_l]   ((x - c) held fixed)
// Source densities at y (relative to c):
//   force f:        Phi_j charge f_j, Psi charge (y - c).f
//   source q:       Psi charge q
//   RPY radius b:   Psi dipole (b^2/3) f
//   double layer D: Phi_j dipole -D^s_j., Psi dipole -(y - c)^T D^s
// Moving the origin from c_A to c_B: Psi_B = Psi_A - (c_B - c_A).Phi.
#pragma once

#include <hip/hip_runtime.h>

namespace kafmm {

constexpr double kInv4Pi = 0.079577471545947667884;   // 1/(4 pi)
constexpr double kInv8Pi = 0.039788735772973833942;   // 1/(8 pi)

__device__ __forceinline__ float rsq_or_zero(float r2) {
    return r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
}

// Accumulations are written as explicit fused multiply-add chains: the
// compiler may not reassociate a += x*y + z*w into two FMAs by itself.
__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
    return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

// ------------------------------------------------------------------ direct kernels
// Source records: [xh, yh, zh, xl, yl, zl, values...]; value layouts below.
// REL: the record also holds the source's position relative to its leaf
// centre in FP32 at [9, 10, 11], and the P2P kernel forms r from it (see the
// kernel); otherwise r is formed from the hi/lo coordinates.

struct DStokeslet {       // SL f0 f1 f2 ; leaf-relative position at 9..11
    static constexpr int RS = 12, RD = 0, NACC = 3;
    static constexpr bool REL = true;
    // u = (1/r) (f + r (r.f)/r^2)
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float q = dot3(dx, dy, dz, v[0], v[1], v[2]) * (ri * ri);
        a[0] = fmaf(ri, fmaf(dx, q, v[0]), a[0]);
        a[1] = fmaf(ri, fmaf(dy, q, v[1]), a[1]);
        a[2] = fmaf(ri, fmaf(dz, q, v[2]), a[2]);
    }
    __device__ static void dl(float, float, float, float, const float *, float *) {}
};

// The Stokeslet with r from the hi/lo coordinates (slots 0..5) instead of
// the leaf-relative positions: the form of plans in which two distinct
// points of different leaves are too close for the leaf-relative one.
struct DStokesletExact : DStokeslet {
    static constexpr bool REL = false;
};

struct DStokesReg {       // SL f0 f1 f2, (3/2) eps^2, eps^2
    static constexpr int RS = 12, RD = 0, NACC = 3;
    static constexpr bool REL = false;
    // u = H1 f + H2 (r.f) r with s = r^2 + eps^2: H1 = (s + eps^2)/s^(3/2),
    // H2 = 1/s^(3/2)  (the ri argument is unused: s replaces r^2)
    __device__ static void sl(float dx, float dy, float dz, float, const float *v, float *a) {
        const float e2 = v[4];
        const float s = dot3(dx, dy, dz, dx, dy, dz) + e2;
        const float ri = rsq_or_zero(s);
        const float h2 = ri * ri * ri;
        const float h1 = (s + e2) * h2;
        const float t = dot3(dx, dy, dz, v[0], v[1], v[2]) * h2;
        a[0] = fmaf(dx, t, fmaf(h1, v[0], a[0]));
        a[1] = fmaf(dy, t, fmaf(h1, v[1], a[1]));
        a[2] = fmaf(dz, t, fmaf(h1, v[2], a[2]));
    }
    __device__ static void dl(float, float, float, float, const float *, float *) {}
};

struct DStokesRegFT {     // SL f0 f1 f2 t0 t1 t2, (3/2) eps^2, eps^2     out u, omega
    static constexpr int RS = 16, RD = 0, NACC = 6;
    static constexpr bool REL = false;
    // with s = r^2 + eps^2 (so r^2 + 2 eps^2 = s + eps^2, 2 r^2 + 5 eps^2 = 2 s + 3 eps^2,
    // 10 eps^4 - 7 eps^2 r^2 - 2 r^4 = 15 eps^4 - 3 eps^2 s - 2 s^2, 21 eps^2 + 6 r^2 = 15 eps^2 + 6 s):
    //   u     += H1 f + H2 (r.f) r + (Q/2) t x r
    //   omega += (Q/2) f x r + (D1 t + D2 (r.t) r) / 4
    __device__ static void sl(float dx, float dy, float dz, float, const float *v, float *a) {
        const float e2 = v[7];
        const float s = dot3(dx, dy, dz, dx, dy, dz) + e2;
        const float ri = rsq_or_zero(s);
        const float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
        const float h1 = (s + e2) * ri3;
        const float hq = 0.5f * fmaf(2.0f, s, 3.0f * e2) * ri5;
        const float d1 = 0.25f * fmaf(15.0f * e2, e2, -s * fmaf(3.0f, e2, 2.0f * s)) * ri7;
        const float d2 = 0.25f * fmaf(6.0f, s, 15.0f * e2) * ri7;
        const float f0 = v[0], f1 = v[1], f2 = v[2], t0 = v[3], t1 = v[4], t2 = v[5];
        const float tu = dot3(dx, dy, dz, f0, f1, f2) * ri3;
        const float tw = dot3(dx, dy, dz, t0, t1, t2) * d2;
        a[0] = fmaf(hq, t1 * dz - t2 * dy, fmaf(dx, tu, fmaf(h1, f0, a[0])));
        a[1] = fmaf(hq, t2 * dx - t0 * dz, fmaf(dy, tu, fmaf(h1, f1, a[1])));
        a[2] = fmaf(hq, t0 * dy - t1 * dx, fmaf(dz, tu, fmaf(h1, f2, a[2])));
        a[3] = fmaf(hq, f1 * dz - f2 * dy, fmaf(dx, tw, fmaf(d1, t0, a[3])));
        a[4] = fmaf(hq, f2 * dx - f0 * dz, fmaf(dy, tw, fmaf(d1, t1, a[4])));
        a[5] = fmaf(hq, f0 * dy - f1 * dx, fmaf(dz, tw, fmaf(d1, t2, a[5])));
    }
    __device__ static void dl(float, float, float, float, const float *, float *) {}
};

struct DRPY {             // SL f0 f1 f2 b^2
    static constexpr int RS = 12, RD = 0, NACC = 6;
    static constexpr bool REL = false;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float rf = dot3(dx, dy, dz, v[0], v[1], v[2]);
        float b2 = v[3];
        float cf = fmaf(b2 * (1.0f / 3.0f), ri3, ri);
        float cr = fmaf(-b2, ri5, ri3) * rf;
        a[0] = fmaf(cr, dx, fmaf(cf, v[0], a[0]));
        a[1] = fmaf(cr, dy, fmaf(cf, v[1], a[1]));
        a[2] = fmaf(cr, dz, fmaf(cf, v[2], a[2]));
        float lf = 2.0f * ri3, lr = -6.0f * rf * ri5;
        a[3] = fmaf(lr, dx, fmaf(lf, v[0], a[3]));
        a[4] = fmaf(lr, dy, fmaf(lf, v[1], a[4]));
        a[5] = fmaf(lr, dz, fmaf(lf, v[2], a[5]));
    }
    __device__ static void dl(float, float, float, float, const float *, float *) {}
};

struct DLapPGrad {        // SL q ; DL d0 d1 d2
    static constexpr int RS = 8, RD = 12, NACC = 4;
    static constexpr bool REL = false;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float q = v[0];
        float t = -q * (ri * ri * ri);
        a[0] = fmaf(q, ri, a[0]);
        a[1] = fmaf(t, dx, a[1]);
        a[2] = fmaf(t, dy, a[2]);
        a[3] = fmaf(t, dz, a[3]);
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri;
        float dr = dot3(dx, dy, dz, v[0], v[1], v[2]);
        float t = -3.0f * dr * (ri3 * ri2);
        a[0] = fmaf(dr, ri3, a[0]);
        a[1] = fmaf(t, dx, fmaf(v[0], ri3, a[1]));
        a[2] = fmaf(t, dy, fmaf(v[1], ri3, a[2]));
        a[3] = fmaf(t, dz, fmaf(v[2], ri3, a[3]));
    }
};

// Laplace with the Hessian (xx, xy, xz, yy, yz, zz) after phi and grad phi:
//   charge q:  d_i d_j (q/r) = q (3 r_i r_j/r^5 - delta_ij/r^3)
//   dipole d:  d_i d_j (d.r/r^3) = -3 (d_i r_j + d_j r_i + (d.r) delta_ij)/r^5 + 15 (d.r) r_i r_j/r^7
__device__ __forceinline__ void lap_hess_charge(float dx, float dy, float dz, float q, float ri, float *a) {
    const float ri3 = ri * ri * ri, c = 3.0f * q * ri3 * ri * ri, d = q * ri3;
    a[0] = fmaf(q, ri, a[0]);
    a[1] = fmaf(-d, dx, a[1]);
    a[2] = fmaf(-d, dy, a[2]);
    a[3] = fmaf(-d, dz, a[3]);
    const float cx = c * dx, cy = c * dy;
    a[4] = fmaf(cx, dx, a[4] - d);
    a[5] = fmaf(cx, dy, a[5]);
    a[6] = fmaf(cx, dz, a[6]);
    a[7] = fmaf(cy, dy, a[7] - d);
    a[8] = fmaf(cy, dz, a[8]);
    a[9] = fmaf(c * dz, dz, a[9] - d);
}

struct DLapPGradGrad {    // SL q ; DL d0 d1 d2      out phi, grad phi, Hessian (10)
    static constexpr int RS = 8, RD = 12, NACC = 10;
    static constexpr bool REL = false;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        lap_hess_charge(dx, dy, dz, v[0], ri, a);
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        const float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
        const float d0 = v[0], d1 = v[1], d2 = v[2];
        const float dr = dot3(dx, dy, dz, d0, d1, d2);
        const float t = -3.0f * dr * ri5, g = -3.0f * ri5, e = 15.0f * dr * ri7;
        a[0] = fmaf(dr, ri3, a[0]);
        a[1] = fmaf(t, dx, fmaf(d0, ri3, a[1]));
        a[2] = fmaf(t, dy, fmaf(d1, ri3, a[2]));
        a[3] = fmaf(t, dz, fmaf(d2, ri3, a[3]));
        const float ex = e * dx, ey = e * dy;
        a[4] = fmaf(ex, dx, fmaf(g, 2.0f * d0 * dx, a[4] + t));
        a[5] = fmaf(ex, dy, fmaf(g, fmaf(d0, dy, d1 * dx), a[5]));
        a[6] = fmaf(ex, dz, fmaf(g, fmaf(d0, dz, d2 * dx), a[6]));
        a[7] = fmaf(ey, dy, fmaf(g, 2.0f * d1 * dy, a[7] + t));
        a[8] = fmaf(ey, dz, fmaf(g, fmaf(d1, dz, d2 * dy), a[8]));
        a[9] = fmaf(e * dz, dz, fmaf(g, 2.0f * d2 * dz, a[9] + t));
    }
};

// Laplace quadrupole Q^s (xx, xy, xz, yy, yz, zz): phi = Q_jk d_j d_k (1/r) and
// its gradient and Hessian, written with the unit vector n = r/r so that no
// power of 1/r above 5 is formed (1/r^9 would overflow FP32 for close pairs):
//   phi   = (3 B - tr)/r^3,                B = n.Q.n, w = Q n
//   d_i   = (6 w_i + (3 tr - 15 B) n_i)/r^4
//   d_ij  = (6 Q_ij - 30 (w_i n_j + n_i w_j) + (105 B - 15 tr) n_i n_j
//            + (3 tr - 15 B) delta_ij)/r^5                        [x 1/4pi]
struct DLapQPGradGrad {   // SL Q^s (6)                            out phi, grad phi, Hessian (10)
    static constexpr int RS = 12, RD = 12, NACC = 10;
    static constexpr bool REL = false;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        const float nx = dx * ri, ny = dy * ri, nz = dz * ri;
        const float wx = dot3(v[0], v[1], v[2], nx, ny, nz);
        const float wy = dot3(v[1], v[3], v[4], nx, ny, nz);
        const float wz = dot3(v[2], v[4], v[5], nx, ny, nz);
        const float B = dot3(nx, ny, nz, wx, wy, wz), tr = v[0] + v[3] + v[5];
        const float ri2 = ri * ri, ri3 = ri2 * ri, ri4 = ri2 * ri2, ri5 = ri4 * ri;
        a[0] = fmaf(fmaf(3.0f, B, -tr), ri3, a[0]);
        const float c = fmaf(3.0f, tr, -15.0f * B) * ri4, w6 = 6.0f * ri4;
        a[1] = fmaf(c, nx, fmaf(w6, wx, a[1]));
        a[2] = fmaf(c, ny, fmaf(w6, wy, a[2]));
        a[3] = fmaf(c, nz, fmaf(w6, wz, a[3]));
        const float e = fmaf(105.0f, B, -15.0f * tr) * ri5, g = -30.0f * ri5, q6 = 6.0f * ri5;
        const float d = fmaf(3.0f, tr, -15.0f * B) * ri5;
        const float ex = e * nx, ey = e * ny, gx = g * nx, gy = g * ny, gz = g * nz;
        a[4] = fmaf(ex, nx, fmaf(2.0f * gx, wx, fmaf(q6, v[0], a[4] + d)));
        a[5] = fmaf(ex, ny, fmaf(gx, wy, fmaf(gy, wx, fmaf(q6, v[1], a[5]))));
        a[6] = fmaf(ex, nz, fmaf(gx, wz, fmaf(gz, wx, fmaf(q6, v[2], a[6]))));
        a[7] = fmaf(ey, ny, fmaf(2.0f * gy, wy, fmaf(q6, v[3], a[7] + d)));
        a[8] = fmaf(ey, nz, fmaf(gy, wz, fmaf(gz, wy, fmaf(q6, v[4], a[8]))));
        a[9] = fmaf(e * nz, nz, fmaf(2.0f * gz, wz, fmaf(q6, v[5], a[9] + d)));
    }
    __device__ static void dl(float, float, float, float, const float *, float *) {}
};

// symmetric D^s stored (xx, xy, xz, yy, yz, zz)
__device__ __forceinline__ void sym_apply(const float *s, float dx, float dy, float dz,
                                          float &wx, float &wy, float &wz) {
    wx = dot3(s[0], s[1], s[2], dx, dy, dz);
    wy = dot3(s[1], s[3], s[4], dx, dy, dz);
    wz = dot3(s[2], s[4], s[5], dx, dy, dz);
}

struct DPVel {            // SL f0 f1 f2 q ; DL D^s (6)      out p, u   [x 1/8pi]
    static constexpr int RS = 12, RD = 12, NACC = 4;
    static constexpr bool REL = false;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri;
        float rf = dot3(dx, dy, dz, v[0], v[1], v[2]);
        a[0] = fmaf(2.0f * rf, ri3, a[0]);
        float t = (rf - v[3]) * ri3;
        a[1] = fmaf(dx, t, fmaf(v[0], ri, a[1]));
        a[2] = fmaf(dy, t, fmaf(v[1], ri, a[2]));
        a[3] = fmaf(dz, t, fmaf(v[2], ri, a[3]));
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float wx, wy, wz;
        sym_apply(v, dx, dy, dz, wx, wy, wz);
        float A = dot3(dx, dy, dz, wx, wy, wz);
        float tr = v[0] + v[3] + v[5];
        float t = -3.0f * A * ri5;
        a[0] = fmaf(2.0f, fmaf(tr, ri3, t), a[0]);
        a[1] = fmaf(t, dx, a[1]);
        a[2] = fmaf(t, dy, a[2]);
        a[3] = fmaf(t, dz, a[3]);
    }
};

struct DTraction {        // SL f0 f1 f2 q ; DL D^s (6)     out sigma sym (6)  [x 1/4pi]
    static constexpr int RS = 12, RD = 12, NACC = 6;
    static constexpr bool REL = false;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float rf = dot3(dx, dy, dz, v[0], v[1], v[2]);
        float q = v[3];
        float c = 3.0f * (q - rf) * ri5, d = q * ri3;
        float cx = c * dx, cy = c * dy;
        a[0] = fmaf(cx, dx, a[0] - d);
        a[1] = fmaf(cx, dy, a[1]);
        a[2] = fmaf(cx, dz, a[2]);
        a[3] = fmaf(cy, dy, a[3] - d);
        a[4] = fmaf(cy, dz, a[4]);
        a[5] = fmaf(c * dz, dz, a[5] - d);
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
        float wx, wy, wz;
        sym_apply(v, dx, dy, dz, wx, wy, wz);
        float A = dot3(dx, dy, dz, wx, wy, wz);
        float tr = v[0] + v[3] + v[5];
        float e = 15.0f * A * ri7, g = -3.0f * ri5, d = tr * ri3;
        float ex = e * dx, ey = e * dy;
        float gx = g * dx, gy = g * dy, gz = g * dz;
        a[0] = fmaf(ex, dx, fmaf(2.0f * gx, wx, a[0] - d));
        a[1] = fmaf(ex, dy, fmaf(gx, wy, fmaf(gy, wx, a[1])));
        a[2] = fmaf(ex, dz, fmaf(gx, wz, fmaf(gz, wx, a[2])));
        a[3] = fmaf(ey, dy, fmaf(2.0f * gy, wy, a[3] - d));
        a[4] = fmaf(ey, dz, fmaf(gy, wz, fmaf(gz, wy, a[4])));
        a[5] = fmaf(e * dz, dz, fmaf(2.0f * gz, wz, a[5] - d));
    }
};

// PVel with its derivatives: out p, u, grad p (7), and with GRADU grad u
// row-major (d_j u_i at 7 + 3 i + j, 16).  grad p doubles as lap u.
template <bool GRADU>
struct DPVelDeriv {       // SL f0 f1 f2 q ; DL D^s (6)                  [x 1/8pi]
    static constexpr int RS = 12, RD = 12, NACC = GRADU ? 16 : 7;
    static constexpr bool REL = false;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        const float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        const float rf = dot3(dx, dy, dz, v[0], v[1], v[2]);
        const float g = rf - v[3], t = g * ri3;
        a[0] = fmaf(2.0f * rf, ri3, a[0]);
        a[1] = fmaf(dx, t, fmaf(v[0], ri, a[1]));
        a[2] = fmaf(dy, t, fmaf(v[1], ri, a[2]));
        a[3] = fmaf(dz, t, fmaf(v[2], ri, a[3]));
        const float c = -6.0f * rf * ri5, d = 2.0f * ri3;
        a[4] = fmaf(c, dx, fmaf(d, v[0], a[4]));
        a[5] = fmaf(c, dy, fmaf(d, v[1], a[5]));
        a[6] = fmaf(c, dz, fmaf(d, v[2], a[6]));
        if constexpr (GRADU) {
            const float r[3] = {dx, dy, dz};
            const float F[3] = {v[0] * ri3, v[1] * ri3, v[2] * ri3};
            const float e = -3.0f * g * ri5;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float er = e * r[i];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    float &o = a[7 + 3 * i + j];
                    o = fmaf(er, r[j], fmaf(r[i], F[j], fmaf(-F[i], r[j], i == j ? o + t : o)));
                }
            }
        }
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        const float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
        float wx, wy, wz;
        sym_apply(v, dx, dy, dz, wx, wy, wz);
        const float A = dot3(dx, dy, dz, wx, wy, wz);
        const float tr = v[0] + v[3] + v[5];
        const float t = -3.0f * A * ri5;
        a[0] = fmaf(2.0f, fmaf(tr, ri3, t), a[0]);
        a[1] = fmaf(t, dx, a[1]);
        a[2] = fmaf(t, dy, a[2]);
        a[3] = fmaf(t, dz, a[3]);
        const float c = fmaf(30.0f * A, ri7, -6.0f * tr * ri5), d = -12.0f * ri5;
        a[4] = fmaf(c, dx, fmaf(d, wx, a[4]));
        a[5] = fmaf(c, dy, fmaf(d, wy, a[5]));
        a[6] = fmaf(c, dz, fmaf(d, wz, a[6]));
        if constexpr (GRADU) {
            const float r[3] = {dx, dy, dz}, w[3] = {wx, wy, wz};
            const float h = 15.0f * A * ri7, g = -6.0f * ri5;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float hr = h * r[i], gr = g * r[i];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    float &o = a[7 + 3 * i + j];
                    o = fmaf(hr, r[j], fmaf(gr, w[j], i == j ? o + t : o));
                }
            }
        }
    }
};

// ------------------------------------------------------------------ 4-Laplace target side
// Equivalent point with charges phi[0..2], psi (Stokes) or q (Laplace);
// s = psi - (x - c).phi is formed per target by the caller.

struct EStokeslet {       // u_i += phi_i/r - r_i s/r^3      [x 1/(8 pi)]
    static constexpr int NC = 4, NACC = 3;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float t = -s * (ri * ri);
        a[0] = fmaf(ri, fmaf(dx, t, ph[0]), a[0]);
        a[1] = fmaf(ri, fmaf(dy, t, ph[1]), a[1]);
        a[2] = fmaf(ri, fmaf(dz, t, ph[2]), a[2]);
    }
};

struct EStokesFT {        // u as EStokeslet; omega = (1/2) curl Phi: += phi x r / r^3   [x 1/(8 pi)]
    static constexpr int NC = 4, NACC = 6;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        const float ri2 = ri * ri, t = -s * ri2, ri3 = ri2 * ri;
        a[0] = fmaf(ri, fmaf(dx, t, ph[0]), a[0]);
        a[1] = fmaf(ri, fmaf(dy, t, ph[1]), a[1]);
        a[2] = fmaf(ri, fmaf(dz, t, ph[2]), a[2]);
        a[3] = fmaf(ri3, ph[1] * dz - ph[2] * dy, a[3]);
        a[4] = fmaf(ri3, ph[2] * dx - ph[0] * dz, a[4]);
        a[5] = fmaf(ri3, ph[0] * dy - ph[1] * dx, a[5]);
    }
};

struct ERPY {             // + lap u_i = -(3 r_i (r.phi)/r^5 - phi_i/r^3)   [x 1/(4 pi), stored x2 for 1/(8 pi)]
    static constexpr int NC = 4, NACC = 6;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri;
        float t = -s * ri2;
        a[0] = fmaf(ri, fmaf(dx, t, ph[0]), a[0]);
        a[1] = fmaf(ri, fmaf(dy, t, ph[1]), a[1]);
        a[2] = fmaf(ri, fmaf(dz, t, ph[2]), a[2]);
        float rp = dot3(dx, dy, dz, ph[0], ph[1], ph[2]);
        float c = -6.0f * rp * (ri3 * ri2);
        float d = 2.0f * ri3;
        a[3] = fmaf(c, dx, fmaf(d, ph[0], a[3]));
        a[4] = fmaf(c, dy, fmaf(d, ph[1], a[4]));
        a[5] = fmaf(c, dz, fmaf(d, ph[2], a[5]));
    }
};

struct ELapPGrad {        // phi += q/r, grad phi += -q r/r^3   [x 1/(4 pi)]
    static constexpr int NC = 1, NACC = 4;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float, float *a) {
        float q = ph[0];
        float t = -q * (ri * ri * ri);
        a[0] = fmaf(q, ri, a[0]);
        a[1] = fmaf(t, dx, a[1]);
        a[2] = fmaf(t, dy, a[2]);
        a[3] = fmaf(t, dz, a[3]);
    }
};

struct ELapPGradGrad {    // phi, grad phi, Hessian of q/r   [x 1/(4 pi)]
    static constexpr int NC = 1, NACC = 10;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float, float *a) {
        lap_hess_charge(dx, dy, dz, ph[0], ri, a);
    }
};

struct EPVel {            // p = (r.phi)/r^3 [x 1/(4 pi) -> x2 for 1/(8 pi)], u as Stokeslet
    static constexpr int NC = 4, NACC = 4;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri;
        float rp = dot3(dx, dy, dz, ph[0], ph[1], ph[2]);
        a[0] = fmaf(2.0f * rp, ri3, a[0]);
        float t = -s * ri2;
        a[1] = fmaf(ri, fmaf(dx, t, ph[0]), a[1]);
        a[2] = fmaf(ri, fmaf(dy, t, ph[1]), a[2]);
        a[3] = fmaf(ri, fmaf(dz, t, ph[2]), a[3]);
    }
};

// p, u, grad p (= lap u) and with GRADU grad u of one equivalent point, with
// s = psi - (x - c).phi (so d_k s = -phi_k):
//   d_k u_i = (phi_k r_i - phi_i r_k)/r^3 + s (3 r_i r_k/r^5 - delta_ik/r^3)   [x 1/(8 pi)]
template <bool GRADU>
struct EPVelDeriv {
    static constexpr int NC = 4, NACC = GRADU ? 16 : 7;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        const float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        const float rp = dot3(dx, dy, dz, ph[0], ph[1], ph[2]);
        a[0] = fmaf(2.0f * rp, ri3, a[0]);
        const float t = -s * ri2;
        a[1] = fmaf(ri, fmaf(dx, t, ph[0]), a[1]);
        a[2] = fmaf(ri, fmaf(dy, t, ph[1]), a[2]);
        a[3] = fmaf(ri, fmaf(dz, t, ph[2]), a[3]);
        const float c = -6.0f * rp * ri5, d = 2.0f * ri3;
        a[4] = fmaf(c, dx, fmaf(d, ph[0], a[4]));
        a[5] = fmaf(c, dy, fmaf(d, ph[1], a[5]));
        a[6] = fmaf(c, dz, fmaf(d, ph[2], a[6]));
        if constexpr (GRADU) {
            const float r[3] = {dx, dy, dz};
            const float P[3] = {ph[0] * ri3, ph[1] * ri3, ph[2] * ri3};
            const float e = 3.0f * s * ri5, sd = s * ri3;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float er = e * r[i];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float &o = a[7 + 3 * i + k];
                    o = fmaf(er, r[k], fmaf(P[k], r[i], fmaf(-P[i], r[k], i == k ? o - sd : o)));
                }
            }
        }
    }
};

struct ETraction {        // sigma_ij += (3 r_i r_j/r^5 - delta_ij/r^3) s - delta_ij (r.phi)/r^3  [x 1/(4 pi)]
    static constexpr int NC = 4, NACC = 6;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float rp = dot3(dx, dy, dz, ph[0], ph[1], ph[2]);
        float c = 3.0f * s * ri5;
        float d = (s + rp) * ri3;
        float cx = c * dx, cy = c * dy;
        a[0] = fmaf(cx, dx, a[0] - d);
        a[1] = fmaf(cx, dy, a[1]);
        a[2] = fmaf(cx, dz, a[2]);
        a[3] = fmaf(cy, dy, a[3] - d);
        a[4] = fmaf(cy, dz, a[4]);
        a[5] = fmaf(c * dz, dz, a[5] - d);
    }
};

}  // namespace kafmm
