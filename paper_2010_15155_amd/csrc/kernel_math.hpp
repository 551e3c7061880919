// Per-pair arithmetic of every kernel, shared by the HIP kernels.
//
// r = x - y (target minus source), ri = 1/|r| (0 for r = 0), mu = 1.  The
// 1/(4 pi) and 1/(8 pi) prefactors are applied once per target by the
// callers (see the scale tables), not per pair.
//
// Direct (S->T) kernels, with their definitions:
//   Stokeslet   u  = (f/r + r (r.f)/r^3)                            [x 1/8pi] Sec. II.B
//   RPY         u  = (1/r + b^2/(3 r^3)) f + (1/r^3 - b^2/r^5) r (r.f)
//               lap u = 2 f/r^3 - 6 r (r.f)/r^5                     [x 1/8pi] Eq. RPYkernel
//   Laplace     phi = q/r + d.r/r^3, grad phi = -q r/r^3 + d/r^3 - 3 (d.r) r/r^5
//                                                                   [x 1/4pi] Sec. II.A
//   PVel SL     p = 2 (r.f)/r^3, u = (r^2 f + r (r.f) - q r)/r^3    [x 1/8pi] Eqs. stkslp, stkslvel
//   PVel DL     p = 2 (-3 A/r^5 + tr D/r^3), u = -3 r A/r^5, A = r.D.r
//                                                                   [x 1/8pi] Eqs. stkdlp, stkdlvel
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

// ------------------------------------------------------------------ direct kernels
// Source records: [xh, yh, zh, xl, yl, zl, values...]; value layouts below.

struct DStokeslet {       // SL f0 f1 f2
    static constexpr int RS = 12, RD = 0, NACC = 3;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri3 = ri * ri * ri;
        float t = (dx * v[0] + dy * v[1] + dz * v[2]) * ri3;
        a[0] += v[0] * ri + dx * t;
        a[1] += v[1] * ri + dy * t;
        a[2] += v[2] * ri + dz * t;
    }
    __device__ static void dl(float, float, float, float, const float *, float *) {}
};

struct DRPY {             // SL f0 f1 f2 b^2
    static constexpr int RS = 12, RD = 0, NACC = 6;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float rf = dx * v[0] + dy * v[1] + dz * v[2];
        float b2 = v[3];
        float cf = ri + (b2 * (1.0f / 3.0f)) * ri3;
        float cr = (ri3 - b2 * ri5) * rf;
        a[0] += cf * v[0] + cr * dx;
        a[1] += cf * v[1] + cr * dy;
        a[2] += cf * v[2] + cr * dz;
        float lf = 2.0f * ri3, lr = -6.0f * rf * ri5;
        a[3] += lf * v[0] + lr * dx;
        a[4] += lf * v[1] + lr * dy;
        a[5] += lf * v[2] + lr * dz;
    }
    __device__ static void dl(float, float, float, float, const float *, float *) {}
};

struct DLapPGrad {        // SL q ; DL d0 d1 d2
    static constexpr int RS = 8, RD = 12, NACC = 4;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float q = v[0];
        float t = q * ri * ri * ri;
        a[0] += q * ri;
        a[1] -= t * dx;
        a[2] -= t * dy;
        a[3] -= t * dz;
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri;
        float dr = dx * v[0] + dy * v[1] + dz * v[2];
        float t = -3.0f * dr * ri3 * ri2;
        a[0] += dr * ri3;
        a[1] += v[0] * ri3 + t * dx;
        a[2] += v[1] * ri3 + t * dy;
        a[3] += v[2] * ri3 + t * dz;
    }
};

// symmetric D^s stored (xx, xy, xz, yy, yz, zz)
__device__ __forceinline__ void sym_apply(const float *s, float dx, float dy, float dz,
                                          float &wx, float &wy, float &wz) {
    wx = s[0] * dx + s[1] * dy + s[2] * dz;
    wy = s[1] * dx + s[3] * dy + s[4] * dz;
    wz = s[2] * dx + s[4] * dy + s[5] * dz;
}

struct DPVel {            // SL f0 f1 f2 q ; DL D^s (6)      out p, u   [x 1/8pi]
    static constexpr int RS = 12, RD = 12, NACC = 4;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri;
        float rf = dx * v[0] + dy * v[1] + dz * v[2];
        a[0] += 2.0f * rf * ri3;
        float t = (rf - v[3]) * ri3;
        a[1] += v[0] * ri + dx * t;
        a[2] += v[1] * ri + dy * t;
        a[3] += v[2] * ri + dz * t;
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float wx, wy, wz;
        sym_apply(v, dx, dy, dz, wx, wy, wz);
        float A = dx * wx + dy * wy + dz * wz;
        float tr = v[0] + v[3] + v[5];
        a[0] += 2.0f * (tr * ri3 - 3.0f * A * ri5);
        float t = -3.0f * A * ri5;
        a[1] += t * dx;
        a[2] += t * dy;
        a[3] += t * dz;
    }
};

struct DTraction {        // SL f0 f1 f2 q ; DL D^s (6)     out sigma sym (6)  [x 1/4pi]
    static constexpr int RS = 12, RD = 12, NACC = 6;
    __device__ static void sl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float rf = dx * v[0] + dy * v[1] + dz * v[2];
        float q = v[3];
        float c = 3.0f * (q - rf) * ri5, d = q * ri3;
        a[0] += c * dx * dx - d;
        a[1] += c * dx * dy;
        a[2] += c * dx * dz;
        a[3] += c * dy * dy - d;
        a[4] += c * dy * dz;
        a[5] += c * dz * dz - d;
    }
    __device__ static void dl(float dx, float dy, float dz, float ri, const float *v, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
        float wx, wy, wz;
        sym_apply(v, dx, dy, dz, wx, wy, wz);
        float A = dx * wx + dy * wy + dz * wz;
        float tr = v[0] + v[3] + v[5];
        float e = 15.0f * A * ri7, g = -3.0f * ri5, d = tr * ri3;
        a[0] += e * dx * dx + 2.0f * g * dx * wx - d;
        a[1] += e * dx * dy + g * (dx * wy + wx * dy);
        a[2] += e * dx * dz + g * (dx * wz + wx * dz);
        a[3] += e * dy * dy + 2.0f * g * dy * wy - d;
        a[4] += e * dy * dz + g * (dy * wz + wy * dz);
        a[5] += e * dz * dz + 2.0f * g * dz * wz - d;
    }
};

// ------------------------------------------------------------------ 4-Laplace target side
// Equivalent point with charges phi[0..2], psi (Stokes) or q (Laplace);
// s = psi - (x - c).phi is formed per target by the caller.

struct EStokeslet {       // u_i += phi_i/r - r_i s/r^3      [x 1/(8 pi)]
    static constexpr int NC = 4, NACC = 3;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float t = s * ri * ri * ri;
        a[0] += ph[0] * ri - dx * t;
        a[1] += ph[1] * ri - dy * t;
        a[2] += ph[2] * ri - dz * t;
    }
};

struct ERPY {             // + lap u_i = -(3 r_i (r.phi)/r^5 - phi_i/r^3)   [x 1/(4 pi), stored x2 for 1/(8 pi)]
    static constexpr int NC = 4, NACC = 6;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri;
        float t = s * ri3;
        a[0] += ph[0] * ri - dx * t;
        a[1] += ph[1] * ri - dy * t;
        a[2] += ph[2] * ri - dz * t;
        float rp = dx * ph[0] + dy * ph[1] + dz * ph[2];
        float c = -6.0f * rp * ri3 * ri2;
        float d = 2.0f * ri3;
        a[3] += c * dx + d * ph[0];
        a[4] += c * dy + d * ph[1];
        a[5] += c * dz + d * ph[2];
    }
};

struct ELapPGrad {        // phi += q/r, grad phi += -q r/r^3   [x 1/(4 pi)]
    static constexpr int NC = 1, NACC = 4;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float, float *a) {
        float q = ph[0];
        float t = q * ri * ri * ri;
        a[0] += q * ri;
        a[1] -= t * dx;
        a[2] -= t * dy;
        a[3] -= t * dz;
    }
};

struct EPVel {            // p = (r.phi)/r^3 [x 1/(4 pi) -> x2 for 1/(8 pi)], u as Stokeslet
    static constexpr int NC = 4, NACC = 4;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float ri3 = ri * ri * ri;
        float rp = dx * ph[0] + dy * ph[1] + dz * ph[2];
        a[0] += 2.0f * rp * ri3;
        float t = s * ri3;
        a[1] += ph[0] * ri - dx * t;
        a[2] += ph[1] * ri - dy * t;
        a[3] += ph[2] * ri - dz * t;
    }
};

struct ETraction {        // sigma_ij += (3 r_i r_j/r^5 - delta_ij/r^3) s - delta_ij (r.phi)/r^3  [x 1/(4 pi)]
    static constexpr int NC = 4, NACC = 6;
    __device__ static void eq(float dx, float dy, float dz, float ri, const float *ph, float s, float *a) {
        float ri2 = ri * ri, ri3 = ri2 * ri, ri5 = ri3 * ri2;
        float rp = dx * ph[0] + dy * ph[1] + dz * ph[2];
        float c = 3.0f * s * ri5;
        float d = (s + rp) * ri3;
        a[0] += c * dx * dx - d;
        a[1] += c * dx * dy;
        a[2] += c * dx * dz;
        a[3] += c * dy * dy - d;
        a[4] += c * dy * dz;
        a[5] += c * dz * dz - d;
    }
};

}  // namespace kafmm
