/*
 * Doubly periodic Stokeslet and its Laplacian by Ewald summation --
 * TEST INFRASTRUCTURE ONLY (oracle; loaded by the tests, the smoke check and
 * the benchmark's CPU leg, never by the HIP library).
 *
 * Periodic boundary conditions in x and y with period L, open in z (Sec. III
 * and its appendix on periodicity; the doubly periodic case of Sec. III.C):
 *
 *     u(x) = sum_j sum_{n in Z^2} G(x - y_j - n L) f_j,
 *     G(r) = (I/r + r r^T/r^3)/(8 pi)                       (Sec. II.B, mu = 1).
 *
 * The lattice sum does not converge absolutely.  Its definition here is the
 * Fourier series in the periodic directions (area A = L^2):
 *   k_par != 0:  the transform of G in z, (1/2pi) int dk_z (I - k k^T/k^2)/k^2 e^{i k_z z};
 *   k_par  = 0:  the sheet flow u_par(z) = -(1/2A) sum_j f_j,par |z - z_j|, u_z = 0,
 * with zero net force (the constant that a net force would leave is
 * dropped).  Far above and below the sources u_par tends to
 * +-(1/2A) sum_j f_j,par z_j.
 *
 * Ewald split with Hasimoto's factor phi(k) = (1 + k^2/4xi^2) e^{-k^2/4xi^2}:
 *   real     sum over the in-plane images of the screened kernel
 *            8 pi G_R(r) = (erfc(xi r)/r - c e) I + (erfc(xi r)/r + c e) r r^T/r^2,
 *            c = 2 xi/sqrt(pi), e = exp(-xi^2 r^2);
 *   spectral (1/A) sum_{k_par} e^{i k_par.rho} (1/2pi) int dk_z phi(k) (I - k k^T/k^2)/k^2 e^{i k_z z}.
 *            With kappa = |k_par| the k_z integrals are, in closed form,
 *              E0 = (1/2pi) int e^{-k^2/4xi^2} e^{i k_z z} = (xi/sqrt(pi)) g,  g = e^{-kappa^2/4xi^2 - xi^2 z^2},
 *              E2 = (1/2pi) int e^{-k^2/4xi^2}/k^2 e^{i k_z z} = S/(4 kappa),
 *              S  = e^{kappa z} erfc(kappa/2xi + xi z) + e^{-kappa z} erfc(kappa/2xi - xi z),
 *              D  = e^{kappa z} erfc(kappa/2xi + xi z) - e^{-kappa z} erfc(kappa/2xi - xi z),
 *              I2 = (1/2pi) int phi/k^2 e^{i k_z z} = E2 + E0/(4 xi^2),
 *              I4 = (1/2pi) int phi/k^4 e^{i k_z z} = -(1/2 kappa) dE2/dkappa
 *                 = E2/(2 kappa^2) - (z D - 2 g/(xi sqrt(pi)))/(8 kappa^2),
 *              dI4/dz = -z E2/2,
 *            so that per mode (a, b in {x, y})
 *              G_ab: cos(k.rho) [delta_ab I2 - k_a k_b I4],
 *              G_az = G_za: sin(k.rho) k_a z E2/2,   G_zz: cos(k.rho) kappa^2 I4;
 *            and the mode k_par = 0 (its 1/(2 kappa) divergence is the
 *            dropped constant) G_ab: delta_ab [-z erf(xi z)/2 - e^{-xi^2 z^2}/(4 xi sqrt(pi))];
 *   self     a target on a source drops the smooth part of its own term,
 *            u -= xi/(2 pi^{3/2}) f (the split is local: as in three dimensions).
 *
 * The Laplacian lap G = (2 I/r^3 - 6 r r^T/r^5)/(8 pi) (the RPY correction
 * (b^2/6) lap G f and the RPY target Laplacian, Sec. II.B) is split the
 * same way: the real part of the triply periodic oracle's lap G_R over the
 * in-plane images, the spectral amplitude -phi(k) (I - k k^T/k^2), i.e.
 *   J0 = (1/2pi) int phi e^{i k_z z} = E0 (3/2 + kappa^2/4xi^2 - xi^2 z^2),
 *   dI2/dz = D/4 - z E0/2,
 *   lap G_ab: cos(k.rho) [-delta_ab J0 + k_a k_b I2],
 *   lap G_az = lap G_za: sin(k.rho) k_a dI2/dz,   lap G_zz: -cos(k.rho) kappa^2 I2,
 *   k_par = 0: lap G_ab = -delta_ab (xi/sqrt(pi)) e^{-xi^2 z^2} (3/2 - xi^2 z^2),
 * and the self term +(5/3) xi^3/pi^{3/2} f.
 *
 * Plain FP64 loops over targets, sources, images and modes (the z
 * integrals couple z_i - z_j, so nothing factorises).
 */
#include <math.h>
#include <stdint.h>

#define PI 3.14159265358979323846

/* exp(a^2) erfc(a) for a >= 0: directly below 26, where neither factor
 * over- or underflows, else its asymptotic series (summed while the terms
 * decrease and exceed 1e-17). */
static double erfcx_pos(double a)
{
    if (a < 26.0) return exp(a * a) * erfc(a);
    const double ia2 = 1.0 / (2.0 * a * a);
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 60; ++n) {
        const double next = -term * (2 * n - 1) * ia2;
        if (fabs(next) >= fabs(term) || fabs(next) < 1e-17) break;
        term = next;
        sum += term;
    }
    return sum / (a * sqrt(PI));
}

/* e^{s kappa Z} erfc(kappa/2xi + s xi Z) for Z >= 0, s = +1 or -1, written
 * as g erfcx(.) (g = e^{-kappa^2/4xi^2 - xi^2 Z^2}) where the argument is
 * non-negative, so that no factor overflows at large kappa Z. */
static double exp_erfc(double kap, double Z, double xi, double g, double s)
{
    const double a = kap / (2.0 * xi) + s * xi * Z;
    if (a >= 0.0) return g * erfcx_pos(a);
    return exp(s * kap * Z) * erfc(a);
}

/*
 * Doubly periodic Stokeslet velocity (and, with lap != NULL, the Laplacian
 * sum lap G f) of forces f [ns][3] at ys [ns][3], at xs [nt][3].  w [ns]
 * (may be NULL) weights a Laplacian term added to the velocity: u += w_j
 * lap G f_j (RPY: w = b^2/6).  xi: split parameter; rc: real-space cutoff;
 * nk: spectral modes |m_x|, |m_y| <= nk.  out [nt][3], lap [nt][3]
 * overwritten.
 */
void oracle_stokes_dp(int64_t ns, const double *ys, const double *f, const double *w, int64_t nt,
                      const double *xs, double L, double xi, double rc, int nk, double *out, double *lap)
{
    const double c = 2.0 * xi / sqrt(PI), x2 = xi * xi, x4 = x2 * x2, A = L * L;
    const int nr = (int)ceil(rc / L) + 1;
    const double self_u = xi / (2.0 * PI * sqrt(PI)), self_l = 5.0 / 3.0 * xi * x2 / (PI * sqrt(PI));
    const int want_lap = lap != 0 || w != 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; ++t) {
        double u[3] = {0.0, 0.0, 0.0}, l[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < ns; ++j) {
            const double *fj = f + 3 * j;
            double d[3];
            int same = 1;
            for (int k = 0; k < 3; ++k) {
                d[k] = xs[3 * t + k] - ys[3 * j + k];
                same = same && d[k] == 0.0;
            }
            d[0] -= L * nearbyint(d[0] / L);
            d[1] -= L * nearbyint(d[1] / L);
            double gu[3] = {0.0, 0.0, 0.0}, gl[3] = {0.0, 0.0, 0.0};   /* G f and lap G f of this source */
            if (same)
                for (int k = 0; k < 3; ++k) {
                    gu[k] -= self_u * fj[k];
                    gl[k] += self_l * fj[k];
                }
            /* real space: in-plane images within rc */
            for (int a = -nr; a <= nr; ++a)
                for (int b = -nr; b <= nr; ++b) {
                    const double r[3] = {d[0] - L * a, d[1] - L * b, d[2]};
                    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                    if (rr >= rc * rc || rr == 0.0) continue;
                    const double rho = sqrt(rr), e = exp(-x2 * rr), ec = erfc(xi * rho) / rho;
                    const double rf = r[0] * fj[0] + r[1] * fj[1] + r[2] * fj[2];
                    const double Au = (ec - c * e) / (8.0 * PI), Bu = (ec + c * e) / rr / (8.0 * PI);
                    for (int k = 0; k < 3; ++k) gu[k] += Au * fj[k] + Bu * rf * r[k];
                    if (want_lap) {
                        const double ec3 = ec / rr;
                        const double Al = (c * e * (8.0 * x2 - 4.0 * x4 * rr + 2.0 / rr) + 2.0 * ec3) / (8.0 * PI);
                        const double Bl = (c * e * (-4.0 * x2 + 4.0 * x4 * rr - 6.0 / rr) - 6.0 * ec3) / rr / (8.0 * PI);
                        for (int k = 0; k < 3; ++k) gl[k] += Al * fj[k] + Bl * rf * r[k];
                    }
                }
            /* spectral, k_par != 0 */
            const double z = d[2], Z = fabs(z), sg = z < 0.0 ? -1.0 : 1.0;
            for (int mx = -nk; mx <= nk; ++mx)
                for (int my = -nk; my <= nk; ++my) {
                    if (mx == 0 && my == 0) continue;
                    const double kx = 2.0 * PI * mx / L, ky = 2.0 * PI * my / L;
                    const double kap2 = kx * kx + ky * ky, kap = sqrt(kap2);
                    const double ph = kx * d[0] + ky * d[1], cs = cos(ph), sn = sin(ph);
                    const double g = exp(-kap2 / (4.0 * x2) - x2 * z * z);
                    const double P = exp_erfc(kap, Z, xi, g, 1.0), Q = exp_erfc(kap, Z, xi, g, -1.0);
                    const double E2 = (P + Q) / (4.0 * kap), Dz = sg * (P - Q), E0 = g * xi / sqrt(PI);
                    const double I2 = E2 + E0 / (4.0 * x2);
                    const double I4 = E2 / (2.0 * kap2) - (z * Dz - 2.0 * g / (xi * sqrt(PI))) / (8.0 * kap2);
                    const double kf = kx * fj[0] + ky * fj[1], kv[2] = {kx, ky};
                    for (int q = 0; q < 2; ++q)
                        gu[q] += (cs * (fj[q] * I2 - kv[q] * kf * I4) + sn * kv[q] * z * E2 / 2.0 * fj[2]) / A;
                    gu[2] += (sn * z * E2 / 2.0 * kf + cs * kap2 * I4 * fj[2]) / A;
                    if (want_lap) {
                        const double J0 = E0 * (1.5 + kap2 / (4.0 * x2) - x2 * z * z);
                        const double dI2 = Dz / 4.0 - z * E0 / 2.0;
                        for (int q = 0; q < 2; ++q)
                            gl[q] += (cs * (-fj[q] * J0 + kv[q] * kf * I2) + sn * kv[q] * dI2 * fj[2]) / A;
                        gl[2] += (sn * dI2 * kf - cs * kap2 * I2 * fj[2]) / A;
                    }
                }
            /* spectral, k_par = 0: horizontal components only */
            const double ez = exp(-x2 * z * z);
            const double s0 = (-z * erf(xi * z) / 2.0 - ez / (4.0 * xi * sqrt(PI))) / A;
            gu[0] += s0 * fj[0];
            gu[1] += s0 * fj[1];
            if (want_lap) {
                const double l0 = -(xi / sqrt(PI)) * ez * (1.5 - x2 * z * z) / A;
                gl[0] += l0 * fj[0];
                gl[1] += l0 * fj[1];
            }
            const double wj = w ? w[j] : 0.0;
            for (int k = 0; k < 3; ++k) {
                u[k] += gu[k] + wj * gl[k];
                l[k] += gl[k];
            }
        }
        for (int k = 0; k < 3; ++k) {
            out[3 * t + k] = u[k];
            if (lap) lap[3 * t + k] = l[k];
        }
    }
}
