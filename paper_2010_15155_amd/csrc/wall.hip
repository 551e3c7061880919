// Stokeslet and RPY above a no-slip wall (Sec. III, the no-slip wall
// section, tab:rpywall): the image sources of the free-space summations and
// the assembly of their results at the targets.
//
// The wall is the plane z = zw.  With heights h = y_3 - zw of the sources
// and x_3 = x_3 - zw of the targets, images y^I = (y_1, y_2, 2 zw - y_3),
// the image system is
//
//   S    RPY               (f_1, f_2, 0, b) at y, (-f_1, -f_2, 0, b) at y^I
//   SD   Laplace q + d     q = -f_3/2 at y, +f_3/2 at y^I; d = h (-f_1, -f_2, f_3) at y^I
//   SDZ  Laplace q + d     q = +-h f_3/2 at y, y^I; d = (b^2/6)(0, 0, f_3) at y and y^I
//   Q    Laplace Q         (b^2/3) [[f_3,0,0],[0,f_3,0],[f_1,f_2,0]] at y^I
//
//   u     = u^S + grad phi^SDZ + x_3 grad(phi^SD + phi^Q) - e_3 (phi^SD + phi^Q)
//   lap u = lap u^S + 2 d_3 grad(phi^SD + phi^Q)
//
// (b = 0 for the Stokeslet, whose Q and SDZ dipoles vanish).  The SD charges
// (-f_3/2, +f_3/2) and the quadrupole's place (the image) are derived from
// the free-space Stokeslet of a normal force and from the source-side RPY
// operator (1 + b^2/6 lap_y) acting on the image dipole; the table prints
// f_3, -f_3 and the source column.
//
// What runs here is the same sum regrouped so that no two large terms cancel
// in FP32 (each regrouping is an identity, checked against the table's form
// in FP64 to 2e-15):
// * the three terms at y (SD charge -f_3/2, SDZ charge h f_3/2, SDZ dipole
//   (b^2/6) f_3 e_3) assemble to exactly the free-space RPY flow of f_3 e_3
//   at y ((x_3 - h) grad(1/r) = r_3 grad(1/r));
// * the image charges (SD f_3/2, SDZ -h f_3/2) assemble to minus the RPY
//   flow of f_3 e_3 at y^I plus grad of a charge -h f_3 at y^I, and the SDZ
//   image dipole (b^2/6) f_3 e_3 becomes (b^2/3) f_3 e_3 (lap_y of that
//   charge term).
// Assembled from Laplace sums the first two cancel: near a source x_3 and h
// agree to the distance while each term is x_3/r^2 (measured in FP32: the two
// gradient sums 20x the flow, relative L2 1.5e-5).  As run:
//
//   S    RPY               (f_1, f_2, f_3, b) at y, (-f_1, -f_2, -f_3, b) at y^I
//   SD   Laplace d         h (-f_1, -f_2, f_3) at y^I
//   SDZ  Laplace q + d     q = -h f_3, d = (b^2/3)(0, 0, f_3), at y^I
//   Q    as above.
//
// The Stokeslet's S summation also runs as RPY with b = 0 (the RPY P2P forms
// r from hi/lo coordinates; near the wall the source and image flows cancel
// to the no-slip value).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"

namespace kafmm {

namespace {

__global__ void wall_positions_kernel(int64_t n, const double *__restrict__ y, double zw, double *__restrict__ y2,
                                      double *__restrict__ yi) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = y[3 * i], b = y[3 * i + 1], c = y[3 * i + 2], ci = 2.0 * zw - c;
    y2[3 * i] = a; y2[3 * i + 1] = b; y2[3 * i + 2] = c;
    y2[3 * (n + i)] = a; y2[3 * (n + i) + 1] = b; y2[3 * (n + i) + 2] = ci;
    yi[3 * i] = a; yi[3 * i + 1] = b; yi[3 * i + 2] = ci;
}

__global__ void wall_values_kernel(WallValueArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = a.n;
    if (i >= n) return;
    const double *v = a.val + (a.rpy ? 4 : 3) * i;
    const double f1 = v[0], f2 = v[1], f3 = v[2], b = a.rpy ? v[3] : 0.0;
    const double h = a.y[3 * i + 2] - a.zw;
    double *s0 = a.vs + 4 * i, *s1 = a.vs + 4 * (n + i);
    s0[0] = f1; s0[1] = f2; s0[2] = f3; s0[3] = b;
    s1[0] = -f1; s1[1] = -f2; s1[2] = -f3; s1[3] = b;
    a.sd_dl[3 * i] = -h * f1; a.sd_dl[3 * i + 1] = -h * f2; a.sd_dl[3 * i + 2] = h * f3;
    a.sdz_sl[i] = -h * f3;
    if (a.rpy) {
        double *d = a.sdz_dl + 3 * i;
        d[0] = d[1] = 0.0;
        d[2] = b * b / 3.0 * f3;
        const double s = b * b / 3.0;
        double *q = a.q + 9 * i;
        q[0] = s * f3; q[1] = 0.0; q[2] = 0.0;
        q[3] = 0.0; q[4] = s * f3; q[5] = 0.0;
        q[6] = s * f1; q[7] = s * f2; q[8] = 0.0;
    }
}

// Laplace outputs: (phi, grad phi[, xx, xy, xz, yy, yz, zz]); d_3 grad = (xz, yz, zz) at 6, 8, 9
__global__ void wall_assemble_kernel(WallAssembleArgs a) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= a.nt) return;
    const double x3 = a.x[3 * t + 2] - a.zw;
    const double *us = a.us + 6 * t;
    const double *sd = a.sd + a.ksd * t;
    const double *sz = a.sdz + 4 * t;
    double phi = sd[0], g0 = sd[1], g1 = sd[2], g2 = sd[3];
    double h0 = 0.0, h1 = 0.0, h2 = 0.0;
    if (a.rpy) {
        const double *q = a.qp + 10 * t;
        phi += q[0]; g0 += q[1]; g1 += q[2]; g2 += q[3];
        h0 = sd[6] + q[6]; h1 = sd[8] + q[8]; h2 = sd[9] + q[9];
    }
    double *o = a.out + (a.rpy ? 6 : 3) * t;
    o[0] = us[0] + sz[1] + x3 * g0;
    o[1] = us[1] + sz[2] + x3 * g1;
    o[2] = us[2] + sz[3] + x3 * g2 - phi;
    if (a.rpy) {
        o[3] = us[3] + 2.0 * h0;
        o[4] = us[4] + 2.0 * h1;
        o[5] = us[5] + 2.0 * h2;
    }
}

inline int nblocks(int64_t n) { return int((n + 255) / 256); }

}  // namespace

hipError_t launch_wall_positions(int64_t n, const double *y, double zw, double *y2, double *yi, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(wall_positions_kernel, dim3(nblocks(n)), dim3(256), 0, s, n, y, zw, y2, yi);
    return hipGetLastError();
}

hipError_t launch_wall_values(const WallValueArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(wall_values_kernel, dim3(nblocks(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_wall_assemble(const WallAssembleArgs &a, hipStream_t s) {
    if (a.nt <= 0) return hipSuccess;
    if (a.ksd != 4 && a.ksd != 10) return hipErrorInvalidValue;
    if (a.rpy && (a.ksd != 10 || a.qp == nullptr)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wall_assemble_kernel, dim3(nblocks(a.nt)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace kafmm
