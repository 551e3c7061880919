/*
 * FP64 direct kernel sums -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is part of the oracle: a plain, slow, obviously correct CPU
 * evaluation of the kernel summation problem g_i(x) = sum_b K_ij(x, y_b) s_j
 * (Sec. I, Eq. kernelsumlinear; the nonlinear-in-source form Eq. kernelsum
 * for RPY).  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code with the HIP library.
 *
 * Conventions (all kernels):
 *   r = x - y (target minus source), mu = 1, pairs with r == 0 add nothing.
 *   Points are AoS [n][3]; values are AoS [n][k].
 *   OpenMP over targets, each target sums all sources in index order.
 *
 * Kernels and where they are defined:
 *   Laplace L = 1/(4 pi r), dipole L^D_j = -dL/dx_j           Sec. II.A
 *   Stokeslet G_ij = (delta_ij/r + r_i r_j/r^3)/(8 pi)        Sec. II.B
 *   RPY G^RPY = (1 + b^2 lap/6) G, target [u, lap u]          Sec. II.B, Eq. RPYkernel
 *   regularized Stokeslet G^eps = H1(r) delta + H2(r) r r^T,
 *     H1 = (r^2 + 2 eps^2)/(8 pi (r^2+eps^2)^(3/2)), H2 = 1/(8 pi (r^2+eps^2)^(3/2))
 *                                                             Sec. II.B, tab:ktab_reg
 *   regularized force + torque -> [u, omega]                  Sec. II.B, tab:ktab_regftvw
 *   StokesPVel [f,q] -> [p,u]                                 Sec. II.C, Eqs. stkslp, stkslvel
 *   Stokes double layer D -> [p,u], T_ijk = -3 r_i r_j r_k/(8 pi r^5)
 *                                                             Sec. II.C, Eqs. stkdlp, stkdlvel
 *   Traction sigma = -p I + grad u + grad u^T                 Sec. II.C, Eq. stressdef
 *   PVelGrad / PVelLaplacian: (p, u) and their derivatives   tab:implement
 *   LapQPGradGrad phi = Q_jk d_j d_k L                       Sec. II.A, tab:implement
 * Output component orders (the paper prints none; see the oracle README
 * strings in direct.py): Hessian (xx,xy,xz,yy,yz,zz), D and sigma row-major.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

#define PI 3.14159265358979323846

/* Threads the parallel loops below use, and a way to change that (the
 * benchmark's CPU baseline times the oracle on all host threads and on one). */
int oracle_max_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* Stokeslet: f (3) -> u (3). */
void oracle_stokeslet(int64_t ns, const double *ys, const double *f,
                      int64_t nt, const double *xs, double *out)
{
    const double c = 1.0 / (8.0 * PI);
#pragma omp parallel for schedule(dynamic, 16) if (nt * ns > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double u0 = 0, u1 = 0, u2 = 0;
        for (int64_t s = 0; s < ns; ++s) {
            double r0 = xs[3*t] - ys[3*s], r1 = xs[3*t+1] - ys[3*s+1], r2 = xs[3*t+2] - ys[3*s+2];
            double rr = r0*r0 + r1*r1 + r2*r2;
            if (rr == 0.0) continue;
            double r = sqrt(rr);
            double f0 = f[3*s], f1 = f[3*s+1], f2 = f[3*s+2];
            double rf = r0*f0 + r1*f1 + r2*f2;
            double a = 1.0 / r, b = rf / (rr * r);
            u0 += a*f0 + b*r0;
            u1 += a*f1 + b*r1;
            u2 += a*f2 + b*r2;
        }
        out[3*t] = c*u0; out[3*t+1] = c*u1; out[3*t+2] = c*u2;
    }
}

/* Regularized Stokeslet: (f1,f2,f3,eps) (4) -> u (3).  The kernel is bounded,
 * so only a coincident pair with eps == 0 is skipped. */
void oracle_stokes_reg(int64_t ns, const double *ys, const double *fe,
                       int64_t nt, const double *xs, double *out)
{
    const double c = 1.0 / (8.0 * PI);
#pragma omp parallel for schedule(dynamic, 16) if (nt * ns > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double u0 = 0, u1 = 0, u2 = 0;
        for (int64_t s = 0; s < ns; ++s) {
            double r0 = xs[3*t] - ys[3*s], r1 = xs[3*t+1] - ys[3*s+1], r2 = xs[3*t+2] - ys[3*s+2];
            double rr = r0*r0 + r1*r1 + r2*r2;
            const double *fs = fe + 4*s;
            double e2 = fs[3] * fs[3];
            double d = rr + e2;
            if (d == 0.0) continue;
            double d32 = d * sqrt(d);
            double h1 = (rr + 2.0 * e2) / d32, h2 = 1.0 / d32;
            double rf = r0*fs[0] + r1*fs[1] + r2*fs[2];
            u0 += h1*fs[0] + h2*rf*r0;
            u1 += h1*fs[1] + h2*rf*r1;
            u2 += h1*fs[2] + h2*rf*r2;
        }
        out[3*t] = c*u0; out[3*t+1] = c*u1; out[3*t+2] = c*u2;
    }
}

/* Regularized force and torque: (f1,f2,f3,t1,t2,t3,eps) (7) -> (u, omega) (6),
 * u = G^eps f + T^eps t, omega = Omega^eps f + W^eps t with
 *   G^eps_ij = H1 delta_ij + H2 r_i r_j,   Omega^eps_ij = T^eps_ij = Q eps_ijk r_k / 2,
 *   W^eps_ij = (D1 delta_ij + D2 r_i r_j) / 4, s = r^2 + eps^2 and
 *   H1 = (r^2 + 2 eps^2)/(8 pi s^(3/2)), H2 = 1/(8 pi s^(3/2)),
 *   Q = (2 r^2 + 5 eps^2)/(8 pi s^(5/2)),
 *   D1 = (10 eps^4 - 7 eps^2 r^2 - 2 r^4)/(8 pi s^(7/2)), D2 = (21 eps^2 + 6 r^2)/(8 pi s^(7/2))
 * (Sec. II.B, the force-torque extension).  eps_ijk r_k a_j = (a x r)_i. */
void oracle_stokes_reg_ft(int64_t ns, const double *ys, const double *fte,
                          int64_t nt, const double *xs, double *out)
{
    const double c = 1.0 / (8.0 * PI);
#pragma omp parallel for schedule(dynamic, 16) if (nt * ns > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double u[3] = {0, 0, 0}, w[3] = {0, 0, 0};
        for (int64_t s = 0; s < ns; ++s) {
            double r[3] = {xs[3*t] - ys[3*s], xs[3*t+1] - ys[3*s+1], xs[3*t+2] - ys[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            const double *v = fte + 7*s;
            const double *f = v, *tq = v + 3;
            double e2 = v[6] * v[6];
            double d = rr + e2;
            if (d == 0.0) continue;
            double sq = sqrt(d), d3 = d * sq, d5 = d3 * d, d7 = d5 * d;
            double h1 = (rr + 2.0 * e2) / d3, h2 = 1.0 / d3;
            double q = (2.0 * rr + 5.0 * e2) / d5;
            double D1 = (10.0 * e2 * e2 - 7.0 * e2 * rr - 2.0 * rr * rr) / d7;
            double D2 = (21.0 * e2 + 6.0 * rr) / d7;
            double rf = r[0]*f[0] + r[1]*f[1] + r[2]*f[2];
            double rt = r[0]*tq[0] + r[1]*tq[1] + r[2]*tq[2];
            double txr[3] = {tq[1]*r[2] - tq[2]*r[1], tq[2]*r[0] - tq[0]*r[2], tq[0]*r[1] - tq[1]*r[0]};
            double fxr[3] = {f[1]*r[2] - f[2]*r[1], f[2]*r[0] - f[0]*r[2], f[0]*r[1] - f[1]*r[0]};
            for (int i = 0; i < 3; ++i) {
                u[i] += h1 * f[i] + h2 * rf * r[i] + 0.5 * q * txr[i];
                w[i] += 0.5 * q * fxr[i] + 0.25 * (D1 * tq[i] + D2 * rt * r[i]);
            }
        }
        for (int i = 0; i < 3; ++i) {
            out[6*t + i] = c * u[i];
            out[6*t + 3 + i] = c * w[i];
        }
    }
}

/* RPY: (f1,f2,f3,b) (4) -> (u, lap u) (6).
 * u = G f + (b^2/6) lap G f,  lap G_ij = (2 delta_ij/r^3 - 6 r_i r_j/r^5)/(8 pi),
 * lap u = lap G f (the b^2 term drops because lap lap G = 0). */
void oracle_rpy(int64_t ns, const double *ys, const double *fb,
                int64_t nt, const double *xs, double *out)
{
    const double c = 1.0 / (8.0 * PI);
#pragma omp parallel for schedule(dynamic, 16) if (nt * ns > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double u[3] = {0, 0, 0}, l[3] = {0, 0, 0};
        for (int64_t s = 0; s < ns; ++s) {
            double r[3] = {xs[3*t] - ys[3*s], xs[3*t+1] - ys[3*s+1], xs[3*t+2] - ys[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double rn = sqrt(rr);
            const double *fs = fb + 4*s;
            double b2 = fs[3] * fs[3];
            double rf = r[0]*fs[0] + r[1]*fs[1] + r[2]*fs[2];
            double i1 = 1.0 / rn, i3 = i1 / rr, i5 = i3 / rr;
            /* Stokeslet part */
            double gd = i1, gr = rf * i3;
            /* lap G f = 2 f/r^3 - 6 r (r.f)/r^5 */
            double ld = 2.0 * i3, lr = -6.0 * rf * i5;
            for (int i = 0; i < 3; ++i) {
                double g = gd * fs[i] + gr * r[i];
                double lg = ld * fs[i] + lr * r[i];
                u[i] += g + (b2 / 6.0) * lg;
                l[i] += lg;
            }
        }
        for (int i = 0; i < 3; ++i) { out[6*t+i] = c*u[i]; out[6*t+3+i] = c*l[i]; }
    }
}

/* Laplace charges q (SL, 1) and dipoles d (DL, 3) -> phi, grad phi and,
 * when hess != 0, the Hessian (xx,xy,xz,yy,yz,zz).  kt = 4 or 10. */
void oracle_laplace(int64_t nsl, const double *ysl, const double *q,
                    int64_t ndl, const double *ydl, const double *d,
                    int64_t nt, const double *xs, double *out, int hess)
{
    const double c = 1.0 / (4.0 * PI);
    const int kt = hess ? 10 : 4;
#pragma omp parallel for schedule(dynamic, 16) if (nt * (nsl + ndl) > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double acc[10] = {0};
        for (int64_t s = 0; s < nsl; ++s) {
            double r[3] = {xs[3*t] - ysl[3*s], xs[3*t+1] - ysl[3*s+1], xs[3*t+2] - ysl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr;
            double qs = q[s];
            acc[0] += qs * i1;
            for (int i = 0; i < 3; ++i) acc[1+i] += -qs * r[i] * i3;
            if (hess) {
                int k = 4;
                for (int i = 0; i < 3; ++i)
                    for (int j = i; j < 3; ++j)
                        acc[k++] += qs * (3.0 * r[i] * r[j] * i5 - (i == j ? i3 : 0.0));
            }
        }
        for (int64_t s = 0; s < ndl; ++s) {
            double r[3] = {xs[3*t] - ydl[3*s], xs[3*t+1] - ydl[3*s+1], xs[3*t+2] - ydl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr, i7 = i5 / rr;
            const double *ds = d + 3*s;
            double dr = ds[0]*r[0] + ds[1]*r[1] + ds[2]*r[2];
            acc[0] += dr * i3;
            for (int i = 0; i < 3; ++i) acc[1+i] += ds[i] * i3 - 3.0 * dr * r[i] * i5;
            if (hess) {
                int k = 4;
                for (int i = 0; i < 3; ++i)
                    for (int j = i; j < 3; ++j)
                        acc[k++] += -3.0 * (ds[j] * r[i] + ds[i] * r[j] + (i == j ? dr : 0.0)) * i5
                                    + 15.0 * dr * r[i] * r[j] * i7;
            }
        }
        for (int k = 0; k < kt; ++k) out[kt*t+k] = c * acc[k];
    }
}

/* Laplace quadrupoles Q (9, row-major Q[3j+k] = Q_jk) -> phi, grad phi,
 * Hessian (xx,xy,xz,yy,yz,zz) (10).  phi = Q_jk d_j d_k L with L = 1/(4 pi r)
 * (Sec. II.A, the quadrupole kernel), so the outputs contract Q with the
 * second, third and fourth derivatives of 1/r:
 *   T2_jk   = 3 r_j r_k/r^5 - delta_jk/r^3
 *   T3_ijk  = -15 r_i r_j r_k/r^7 + 3 (delta_ij r_k + delta_ik r_j + delta_jk r_i)/r^5
 *   T4_lijk = 105 r_l r_i r_j r_k/r^9 - 15 (six delta_ab r_c r_d terms)/r^7
 *             + 3 (delta_li delta_jk + delta_lj delta_ik + delta_lk delta_ij)/r^5 */
static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

void oracle_laplace_quad(int64_t nq, const double *y, const double *Q,
                         int64_t nt, const double *xs, double *out)
{
    const double c = 1.0 / (4.0 * PI);
#pragma omp parallel for schedule(dynamic, 16) if (nt * nq > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double acc[10] = {0};
        for (int64_t s = 0; s < nq; ++s) {
            double r[3] = {xs[3*t] - y[3*s], xs[3*t+1] - y[3*s+1], xs[3*t+2] - y[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr, i7 = i5 / rr, i9 = i7 / rr;
            const double *Qs = Q + 9*s;
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) {
                    const double q = Qs[3*j+k];
                    acc[0] += q * (3.0 * r[j] * r[k] * i5 - kd(j, k) * i3);
                    for (int i = 0; i < 3; ++i)
                        acc[1+i] += q * (-15.0 * r[i] * r[j] * r[k] * i7
                                         + 3.0 * (kd(i, j) * r[k] + kd(i, k) * r[j] + kd(j, k) * r[i]) * i5);
                    int h = 4;
                    for (int l = 0; l < 3; ++l)
                        for (int i = l; i < 3; ++i) {
                            double t4 = 105.0 * r[l] * r[i] * r[j] * r[k] * i9
                                      - 15.0 * (kd(l, i) * r[j] * r[k] + kd(l, j) * r[i] * r[k] + kd(l, k) * r[i] * r[j]
                                                + kd(i, j) * r[l] * r[k] + kd(i, k) * r[l] * r[j] + kd(j, k) * r[l] * r[i]) * i7
                                      + 3.0 * (kd(l, i) * kd(j, k) + kd(l, j) * kd(i, k) + kd(l, k) * kd(i, j)) * i5;
                            acc[h++] += q * t4;
                        }
                }
        }
        for (int k = 0; k < 10; ++k) out[10*t+k] = c * acc[k];
    }
}

/* StokesPVel: SL (f,q) (4) and DL D (9, row-major D[3j+k] = D_jk) -> (p, u) (4). */
void oracle_pvel(int64_t nsl, const double *ysl, const double *fq,
                 int64_t ndl, const double *ydl, const double *D,
                 int64_t nt, const double *xs, double *out)
{
    const double c4 = 1.0 / (4.0 * PI), c8 = 1.0 / (8.0 * PI);
#pragma omp parallel for schedule(dynamic, 16) if (nt * (nsl + ndl) > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double p = 0, u[3] = {0, 0, 0};
        for (int64_t s = 0; s < nsl; ++s) {
            double r[3] = {xs[3*t] - ysl[3*s], xs[3*t+1] - ysl[3*s+1], xs[3*t+2] - ysl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr;
            const double *v = fq + 4*s;
            double rf = r[0]*v[0] + r[1]*v[1] + r[2]*v[2];
            p += c4 * rf * i3;
            for (int i = 0; i < 3; ++i)
                u[i] += c8 * ((rr * v[i] + r[i] * rf) * i3 - r[i] * v[3] * i3);
        }
        for (int64_t s = 0; s < ndl; ++s) {
            double r[3] = {xs[3*t] - ydl[3*s], xs[3*t+1] - ydl[3*s+1], xs[3*t+2] - ydl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr;
            const double *Ds = D + 9*s;
            double rDr = 0, tr = Ds[0] + Ds[4] + Ds[8];
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) rDr += r[j] * Ds[3*j+k] * r[k];
            p += c4 * (-3.0 * rDr * i5 + tr * i3);
            for (int i = 0; i < 3; ++i) u[i] += -3.0 * c8 * r[i] * rDr * i5;
        }
        out[4*t] = p; out[4*t+1] = u[0]; out[4*t+2] = u[1]; out[4*t+3] = u[2];
    }
}

/* PVel with derivatives: SL (f,q) and DL D -> when lap == 0 (PVelGrad)
 * (p, u, grad p, grad u) with grad u[3i+j] = du_i/dx_j (16 values); when
 * lap != 0 (PVelLaplacian) (p, u, lap u) (7 values).  Per source, with
 * rf = r.f, A = r.D.r, w = D^s r:
 *   SL  u_i = (f_i/r + r_i (rf - q)/r^3)/(8 pi),  p = rf/(4 pi r^3)
 *       du_i/dx_j = (-f_i r_j/r^3 + delta_ij (rf - q)/r^3 + r_i f_j/r^3
 *                    - 3 r_i r_j (rf - q)/r^5)/(8 pi)
 *       dp/dx_j = (f_j/r^3 - 3 rf r_j/r^5)/(4 pi)
 *       lap u_i = (2 f_i/r^3 - 6 r_i rf/r^5)/(8 pi)  (the q r/r^3 part is harmonic)
 *   DL  u_i = -3 r_i A/(8 pi r^5),  p = (-3 A/r^5 + tr D/r^3)/(4 pi)
 *       du_i/dx_j = -3 (delta_ij A/r^5 + 2 r_i w_j/r^5 - 5 r_i r_j A/r^7)/(8 pi)
 *       dp/dx_j = (-6 w_j/r^5 + 15 A r_j/r^7 - 3 tr D r_j/r^5)/(4 pi)
 *       lap u_i = -3 lap(r_i A/r^5)/(8 pi), lap(r_i g) = r_i lap g + 2 d_i g with
 *       g = A/r^5, lap g = 2 tr D/r^5:  lap u_i = (-6 tr D r_i/r^5 - 12 w_i/r^5
 *       + 30 A r_i/r^7)/(8 pi). */
void oracle_pvel_deriv(int64_t nsl, const double *ysl, const double *fq,
                       int64_t ndl, const double *ydl, const double *D,
                       int64_t nt, const double *xs, double *out, int lap)
{
    const double c4 = 1.0 / (4.0 * PI), c8 = 1.0 / (8.0 * PI);
    const int kt = lap ? 7 : 16;
#pragma omp parallel for schedule(dynamic, 16) if (nt * (nsl + ndl) > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double p = 0, u[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, gu[9] = {0}, lu[3] = {0, 0, 0};
        for (int64_t s = 0; s < nsl; ++s) {
            double r[3] = {xs[3*t] - ysl[3*s], xs[3*t+1] - ysl[3*s+1], xs[3*t+2] - ysl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr;
            const double *f = fq + 4*s;
            double rf = r[0]*f[0] + r[1]*f[1] + r[2]*f[2], g = rf - f[3];
            p += c4 * rf * i3;
            for (int i = 0; i < 3; ++i) {
                u[i] += c8 * (f[i] * i1 + r[i] * g * i3);
                gp[i] += c4 * (f[i] * i3 - 3.0 * rf * r[i] * i5);
                lu[i] += c8 * (2.0 * f[i] * i3 - 6.0 * r[i] * rf * i5);
                for (int j = 0; j < 3; ++j)
                    gu[3*i+j] += c8 * (-f[i] * r[j] * i3 + (i == j ? g * i3 : 0.0) + r[i] * f[j] * i3
                                       - 3.0 * r[i] * r[j] * g * i5);
            }
        }
        for (int64_t s = 0; s < ndl; ++s) {
            double r[3] = {xs[3*t] - ydl[3*s], xs[3*t+1] - ydl[3*s+1], xs[3*t+2] - ydl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr, i7 = i5 / rr;
            const double *Ds = D + 9*s;
            double A = 0, tr = Ds[0] + Ds[4] + Ds[8], w[3];
            for (int j = 0; j < 3; ++j) {
                w[j] = 0;
                for (int k = 0; k < 3; ++k) {
                    A += r[j] * Ds[3*j+k] * r[k];
                    w[j] += 0.5 * (Ds[3*j+k] + Ds[3*k+j]) * r[k];
                }
            }
            p += c4 * (-3.0 * A * i5 + tr * i3);
            for (int i = 0; i < 3; ++i) {
                u[i] += -3.0 * c8 * r[i] * A * i5;
                gp[i] += c4 * (-6.0 * w[i] * i5 + 15.0 * A * r[i] * i7 - 3.0 * tr * r[i] * i5);
                lu[i] += c8 * (-6.0 * tr * r[i] * i5 - 12.0 * w[i] * i5 + 30.0 * A * r[i] * i7);
                for (int j = 0; j < 3; ++j)
                    gu[3*i+j] += -3.0 * c8 * ((i == j ? A * i5 : 0.0) + 2.0 * r[i] * w[j] * i5
                                              - 5.0 * r[i] * r[j] * A * i7);
            }
        }
        double *o = out + kt * t;
        o[0] = p;
        for (int i = 0; i < 3; ++i) o[1+i] = u[i];
        if (lap) {
            for (int i = 0; i < 3; ++i) o[4+i] = lu[i];
        } else {
            for (int i = 0; i < 3; ++i) o[4+i] = gp[i];
            for (int k = 0; k < 9; ++k) o[7+k] = gu[k];
        }
    }
}

/* Traction sigma (9, row-major sigma[3i+j]) from SL (f,q) and DL D:
 * sigma = -p I + grad u + grad u^T applied to the PVel flow fields. */
void oracle_traction(int64_t nsl, const double *ysl, const double *fq,
                     int64_t ndl, const double *ydl, const double *D,
                     int64_t nt, const double *xs, double *out)
{
    const double c4 = 1.0 / (4.0 * PI);
#pragma omp parallel for schedule(dynamic, 16) if (nt * (nsl + ndl) > 200000)
    for (int64_t t = 0; t < nt; ++t) {
        double sg[9] = {0};
        for (int64_t s = 0; s < nsl; ++s) {
            double r[3] = {xs[3*t] - ysl[3*s], xs[3*t+1] - ysl[3*s+1], xs[3*t+2] - ysl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr;
            const double *v = fq + 4*s;
            double rf = r[0]*v[0] + r[1]*v[1] + r[2]*v[2];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    sg[3*i+j] += -3.0 * c4 * r[i] * r[j] * rf * i5
                                 - c4 * v[3] * ((i == j ? i3 : 0.0) - 3.0 * r[i] * r[j] * i5);
        }
        for (int64_t s = 0; s < ndl; ++s) {
            double r[3] = {xs[3*t] - ydl[3*s], xs[3*t+1] - ydl[3*s+1], xs[3*t+2] - ydl[3*s+2]};
            double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
            if (rr == 0.0) continue;
            double i1 = 1.0 / sqrt(rr), i3 = i1 / rr, i5 = i3 / rr, i7 = i5 / rr;
            const double *Ds = D + 9*s;
            double tr = Ds[0] + Ds[4] + Ds[8];
            double w[3];     /* sym(D) r */
            for (int j = 0; j < 3; ++j) {
                w[j] = 0;
                for (int k = 0; k < 3; ++k) w[j] += 0.5 * (Ds[3*j+k] + Ds[3*k+j]) * r[k];
            }
            double A = r[0]*w[0] + r[1]*w[1] + r[2]*w[2];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    sg[3*i+j] += c4 * (-(i == j ? tr * i3 : 0.0)
                                       - 3.0 * (r[i] * w[j] + w[i] * r[j]) * i5
                                       + 15.0 * A * r[i] * r[j] * i7);
        }
        for (int k = 0; k < 9; ++k) out[9*t+k] = sg[k];
    }
}
