/*
 * FP64 Ewald summation for triply periodic Laplace charges and dipoles --
 * TEST INFRASTRUCTURE ONLY (part of the oracle; no code shared with the HIP
 * library).
 *
 * Problem: phi(x) = sum_j sum_n [q_j L(x - y_j + nL) + d_j . r/(4 pi |r|^3)
 *                                + Q_j : grad grad L(x - y_j + nL)]
 * over the periodic lattice, with L(r) = 1/(4 pi r) (Sec. II.A), the
 * periodic boundary condition of Sec. III and its appendix on periodicity.
 * The lattice sum is only conditionally convergent, so the oracle fixes
 * the textbook Ewald definition: zero net charge is required, the k = 0 term
 * is dropped and no surface (dipole) term is added ("tin-foil" boundary).
 *
 * Split with parameter xi:
 *   real part   q B0(rho) + (d . r) B(rho)                   (rho = |r|)
 *               B0 = erfc(xi rho)/(4 pi rho)
 *               B  = [erfc(xi rho) + 2 xi rho/sqrt(pi) e^{-xi^2 rho^2}]/(4 pi rho^3)
 *               C  = [3 erfc(xi rho) + 2 xi rho/sqrt(pi) (3 + 2 xi^2 rho^2) e^{-xi^2 rho^2}]/(4 pi rho^5)
 *               D  = [15 erfc(xi rho) + 2 xi rho/sqrt(pi) (15 + 10 xi^2 rho^2 + 4 xi^4 rho^4)
 *                     e^{-xi^2 rho^2}]/(4 pi rho^7)
 *               grad: -q B r + d B - (d . r) C r
 *               Hessian: q (C r r^T - B I)
 *                        - C (d r^T + r d^T) - (d . r) C I + (d . r) D r r^T
 *   reciprocal  (1/V) sum_{k != 0} e^{-k^2/(4 xi^2)}/k^2 Re[S(k) e^{i k.x}],
 *               S(k) = sum_j (q_j - i k.d_j) e^{-i k.y_j},  k = 2 pi n / L
 *   reciprocal Hessian: -k k^T g Re[S(k) e^{i k.x}]
 *   self        a target that coincides with source j drops the smooth
 *               self part: phi -= q_j xi / (2 pi^{3/2}),
 *               grad phi -= d_j xi^3 / (3 pi^{3/2}),
 *               Hessian += q_j xi^3 / (3 pi^{3/2}) I (the dipole's smooth
 *               part is odd, its second derivatives vanish at the source).
 * Quadrupoles Q (9, row-major; the symmetric part acts), with
 * E = [105 erfc + 2 xi rho/sqrt(pi) (105 + 70 x^2 + 28 x^4 + 8 x^6) e^{-x^2}]/(4 pi rho^9),
 * x = xi rho, A = r.Q.r, w = Q r, T = tr Q:
 *   real      phi  C A - B T
 *             grad -D A r + 2 C w + C T r
 *             Hess E A r r^T - D A I - 2 D (r w^T + w r^T) + 2 C Q - D T r r^T + C T I
 *   reciprocal amplitude -k.Q.k in S(k)
 *   self      phi += T xi^3/(3 pi^{3/2}),
 *             Hess -= 2 xi^5/(5 pi^{3/2}) (T I + 2 Q)  (fourth derivatives of the
 *             smooth part erf(xi r)/(4 pi r) at r = 0).
 * Hessian order (xx, xy, xz, yy, yz, zz).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* Linear index of lattice vector n in the cube [-nmax, nmax]^3. */
static inline int64_t kidx(int nx, int ny, int nz, int nmax)
{
    int w = 2 * nmax + 1;
    return ((int64_t)(nz + nmax) * w + (ny + nmax)) * w + (nx + nmax);
}

/* Half-space predicate: exactly one of n and -n is kept, n = 0 excluded. */
static inline int khalf(int nx, int ny, int nz)
{
    return nz > 0 || (nz == 0 && (ny > 0 || (ny == 0 && nx > 0)));
}

/* Structure factor S(k) on the half space of the cube [-nmax,nmax]^3. */
void oracle_ewald_structure(int64_t ns, const double *ys, const double *q,
                            const double *d, const double *Q, double L, int nmax,
                            double *S_re, double *S_im)
{
    int w = 2 * nmax + 1;
    int64_t nk = (int64_t)w * w * w;
    memset(S_re, 0, sizeof(double) * nk);
    memset(S_im, 0, sizeof(double) * nk);
#pragma omp parallel
    {
        double *sr = calloc(nk, sizeof(double));
        double *si = calloc(nk, sizeof(double));
        double *cx = malloc(sizeof(double) * 6 * w);
        double *sx = cx + 3 * w;
#pragma omp for schedule(static)
        for (int64_t j = 0; j < ns; ++j) {
            /* e^{-i 2 pi n y_a / L} = cos - i sin, per axis a and n */
            for (int a = 0; a < 3; ++a)
                for (int n = -nmax; n <= nmax; ++n) {
                    double ang = 2.0 * PI * n * ys[3*j+a] / L;
                    cx[a*w + n + nmax] = cos(ang);
                    sx[a*w + n + nmax] = -sin(ang);
                }
            double qj = q ? q[j] : 0.0;
            double dx = d ? d[3*j] : 0.0, dy = d ? d[3*j+1] : 0.0, dz = d ? d[3*j+2] : 0.0;
            for (int nz = 0; nz <= nmax; ++nz)
                for (int ny = -nmax; ny <= nmax; ++ny)
                    for (int nx = -nmax; nx <= nmax; ++nx) {
                        if (!khalf(nx, ny, nz)) continue;
                        /* phase e^{-i k.y} */
                        double ar = cx[nx + nmax], ai = sx[nx + nmax];
                        double br = cx[w + ny + nmax], bi = sx[w + ny + nmax];
                        double cr = cx[2*w + nz + nmax], ci = sx[2*w + nz + nmax];
                        double tr = ar*br - ai*bi, ti = ar*bi + ai*br;
                        double er = tr*cr - ti*ci, ei = tr*ci + ti*cr;
                        /* amplitude q - i k.d - k.Q.k */
                        double kd = 2.0 * PI / L * (nx*dx + ny*dy + nz*dz);
                        double mr = qj, mi = -kd;
                        if (Q) {
                            const double kv[3] = {2.0 * PI / L * nx, 2.0 * PI / L * ny, 2.0 * PI / L * nz};
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b) mr -= kv[a] * Q[9*j + 3*a + b] * kv[b];
                        }
                        int64_t id = kidx(nx, ny, nz, nmax);
                        sr[id] += mr*er - mi*ei;
                        si[id] += mr*ei + mi*er;
                    }
        }
#pragma omp critical
        for (int64_t i = 0; i < nk; ++i) { S_re[i] += sr[i]; S_im[i] += si[i]; }
        free(sr); free(si); free(cx);
    }
}

/* phi and grad phi (4 values per target), and with hess != 0 the Hessian
 * (10 values), from the real, reciprocal and self parts. */
void oracle_ewald_eval(int64_t ns, const double *ys, const double *q, const double *d,
                       const double *Q, int64_t nt, const double *xs, double L, double xi, double rc,
                       int nmax, const double *S_re, const double *S_im, double *out, int hess)
{
    const int kt = hess ? 10 : 4;
    const double V = L * L * L;
    const int nimg = (int)ceil(rc / L);
    const double sqpi = sqrt(PI);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; ++t) {
        double acc[10] = {0};
        const double *x = xs + 3*t;
        /* real space */
        for (int64_t j = 0; j < ns; ++j) {
            double qj = q ? q[j] : 0.0;
            double dj[3] = {d ? d[3*j] : 0.0, d ? d[3*j+1] : 0.0, d ? d[3*j+2] : 0.0};
            double Qs[3][3] = {{0}}, Tq = 0.0;
            if (Q) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Qs[a][b] = 0.5 * (Q[9*j + 3*a + b] + Q[9*j + 3*b + a]);
                Tq = Qs[0][0] + Qs[1][1] + Qs[2][2];
            }
            int self = 0;
            for (int a = -nimg; a <= nimg; ++a)
                for (int b = -nimg; b <= nimg; ++b)
                    for (int c = -nimg; c <= nimg; ++c) {
                        double r[3] = {x[0] - ys[3*j] + a*L, x[1] - ys[3*j+1] + b*L, x[2] - ys[3*j+2] + c*L};
                        double rr = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
                        if (rr == 0.0) { self = 1; continue; }
                        if (rr >= rc*rc) continue;
                        double rho = sqrt(rr), xr = xi * rho;
                        double ec = erfc(xr), ex = exp(-xr*xr);
                        double B0 = ec / (4.0*PI*rho);
                        double B = (ec + 2.0*xr/sqpi*ex) / (4.0*PI*rho*rr);
                        double C = (3.0*ec + 2.0*xr/sqpi*(3.0 + 2.0*xr*xr)*ex) / (4.0*PI*rho*rr*rr);
                        double dr = dj[0]*r[0] + dj[1]*r[1] + dj[2]*r[2];
                        acc[0] += qj * B0 + dr * B;
                        for (int i = 0; i < 3; ++i)
                            acc[1+i] += -qj * B * r[i] + dj[i] * B - dr * C * r[i];
                        double x2 = xr*xr;
                        double D = (15.0*ec + 2.0*xr/sqpi*(15.0 + 10.0*x2 + 4.0*x2*x2)*ex) / (4.0*PI*rho*rr*rr*rr);
                        double w[3] = {0, 0, 0}, A = 0.0;
                        if (Q) {
                            for (int a = 0; a < 3; ++a) {
                                for (int b = 0; b < 3; ++b) w[a] += Qs[a][b] * r[b];
                                A += r[a] * w[a];
                            }
                            acc[0] += C * A - B * Tq;
                            for (int i = 0; i < 3; ++i) acc[1+i] += -D * A * r[i] + 2.0 * C * w[i] + C * Tq * r[i];
                        }
                        if (hess) {
                            int h = 4;
                            for (int i = 0; i < 3; ++i)
                                for (int k = i; k < 3; ++k) {
                                    double dik = (i == k) ? 1.0 : 0.0;
                                    acc[h] += qj * (C * r[i] * r[k] - B * dik)
                                              - C * (dj[i] * r[k] + r[i] * dj[k]) - dr * C * dik + dr * D * r[i] * r[k];
                                    if (Q) {
                                        double E = (105.0*ec + 2.0*xr/sqpi*(105.0 + 70.0*x2 + 28.0*x2*x2 + 8.0*x2*x2*x2)*ex)
                                                   / (4.0*PI*rho*rr*rr*rr*rr);
                                        acc[h] += E * A * r[i] * r[k] - D * A * dik - 2.0 * D * (r[i] * w[k] + w[i] * r[k])
                                                + 2.0 * C * Qs[i][k] - D * Tq * r[i] * r[k] + C * Tq * dik;
                                    }
                                    ++h;
                                }
                        }
                    }
            if (self) {
                acc[0] -= qj * xi / (2.0 * PI * sqpi);
                for (int i = 0; i < 3; ++i) acc[1+i] -= dj[i] * xi*xi*xi / (3.0 * PI * sqpi);
                if (hess) {
                    acc[4] += qj * xi*xi*xi / (3.0 * PI * sqpi);
                    acc[7] += qj * xi*xi*xi / (3.0 * PI * sqpi);
                    acc[9] += qj * xi*xi*xi / (3.0 * PI * sqpi);
                }
                if (Q) {
                    acc[0] += Tq * xi*xi*xi / (3.0 * PI * sqpi);
                    if (hess) {
                        const double c5 = 2.0 * xi*xi*xi*xi*xi / (5.0 * PI * sqpi);
                        int h = 4;
                        for (int i = 0; i < 3; ++i)
                            for (int k = i; k < 3; ++k) acc[h++] -= c5 * ((i == k ? Tq : 0.0) + 2.0 * Qs[i][k]);
                    }
                }
            }
        }
        /* reciprocal space: the half space counted twice */
        for (int nz = 0; nz <= nmax; ++nz)
            for (int ny = -nmax; ny <= nmax; ++ny)
                for (int nx = -nmax; nx <= nmax; ++nx) {
                    if (!khalf(nx, ny, nz)) continue;
                    double k[3] = {2.0*PI*nx/L, 2.0*PI*ny/L, 2.0*PI*nz/L};
                    double k2 = k[0]*k[0] + k[1]*k[1] + k[2]*k[2];
                    double g = 2.0 * exp(-k2 / (4.0*xi*xi)) / (k2 * V);
                    double ph = k[0]*x[0] + k[1]*x[1] + k[2]*x[2];
                    double cr = cos(ph), ci = sin(ph);
                    int64_t id = kidx(nx, ny, nz, nmax);
                    double zr = S_re[id]*cr - S_im[id]*ci;   /* Re[S e^{ikx}] */
                    double zi = S_re[id]*ci + S_im[id]*cr;   /* Im[S e^{ikx}] */
                    acc[0] += g * zr;
                    for (int i = 0; i < 3; ++i) acc[1+i] += -g * k[i] * zi;  /* Re[i k S e^{ikx}] */
                    if (hess) {
                        int h = 4;
                        for (int i = 0; i < 3; ++i)
                            for (int m = i; m < 3; ++m) acc[h++] += -g * k[i] * k[m] * zr;
                    }
                }
        for (int i = 0; i < kt; ++i) out[kt*t+i] = acc[i];
    }
}

/*
 * Real-space part of the triply periodic Stokeslet (Hasimoto split; the
 * reciprocal part is summed in stokes_periodic.py, which states the
 * definition): for each target, every image of every source within rc,
 *   8 pi G_R(r) = (erfc(xi r)/r - c e) I + (erfc(xi r)/r + c e) r r^T/r^2,
 *   c = 2 xi/sqrt(pi), e = exp(-xi^2 r^2),
 * and for a target on a source the self term -xi/(2 pi^{3/2}) f.
 * out [nt][3] is overwritten.
 */
void oracle_stokes_ewald_real(int64_t ns, const double *ys, const double *f, int64_t nt, const double *xs,
                              double L, double xi, double rc, double *out)
{
    const double c = 2.0 * xi / sqrt(PI);
    const int nimg = (int)floor(rc / L + 0.5);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        double u[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < ns; ++j) {
            double d[3];
            int same = 1;
            for (int k = 0; k < 3; ++k) {
                d[k] = xs[3 * t + k] - ys[3 * j + k];
                same = same && d[k] == 0.0;
                d[k] -= L * nearbyint(d[k] / L);
            }
            if (same)
                for (int k = 0; k < 3; ++k) u[k] -= xi / (2.0 * PI * sqrt(PI)) * 8.0 * PI * f[3 * j + k];
            for (int a = -nimg; a <= nimg; ++a)
                for (int b = -nimg; b <= nimg; ++b)
                    for (int e3 = -nimg; e3 <= nimg; ++e3) {
                        const double r[3] = {d[0] - L * a, d[1] - L * b, d[2] - L * e3};
                        const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                        if (rr >= rc * rc || rr == 0.0) continue;
                        const double rho = sqrt(rr), e = exp(-xi * xi * rr), ec = erfc(xi * rho) / rho;
                        const double A = ec - c * e, B = (ec + c * e) / rr;
                        const double rf = r[0] * f[3 * j] + r[1] * f[3 * j + 1] + r[2] * f[3 * j + 2];
                        for (int k = 0; k < 3; ++k) u[k] += A * f[3 * j + k] + B * rf * r[k];
                    }
        }
        for (int k = 0; k < 3; ++k) out[3 * t + k] = u[k] / (8.0 * PI);
    }
}

/*
 * Real-space part of the triply periodic Laplacian of the Stokeslet,
 * lap G = (2 I/r^3 - 6 r r^T/r^5)/(8 pi) (Hasimoto split as above): with
 * H = lap B_R = 2 erfc(xi r)/r - c e,
 *   8 pi lap G_R = [c e (8 xi^2 - 4 xi^4 r^2 + 2/r^2) + 2 erfc(xi r)/r^3] I
 *                + [c e (-4 xi^2 + 4 xi^4 r^2 - 6/r^2) - 6 erfc(xi r)/r^3] r r^T/r^2,
 * and for a target on a source the self term +(5/3) xi^3/pi^{3/2} f (minus
 * the smooth part at r = 0, -(5/3) xi^3/pi^{3/2} I).  w [ns] weights each
 * source (b^2/6 for the RPY velocity, 1 for its Laplacian).  out [nt][3] is
 * overwritten.
 */
void oracle_stokes_lap_ewald_real(int64_t ns, const double *ys, const double *f, const double *w, int64_t nt,
                                  const double *xs, double L, double xi, double rc, double *out)
{
    const double c = 2.0 * xi / sqrt(PI);
    const int nimg = (int)floor(rc / L + 0.5);
    const double x2 = xi * xi, x4 = x2 * x2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        double u[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < ns; ++j) {
            double d[3], fw[3];
            int same = 1;
            for (int k = 0; k < 3; ++k) {
                d[k] = xs[3 * t + k] - ys[3 * j + k];
                same = same && d[k] == 0.0;
                d[k] -= L * nearbyint(d[k] / L);
                fw[k] = w[j] * f[3 * j + k];
            }
            if (same)
                for (int k = 0; k < 3; ++k) u[k] += 5.0 / 3.0 * xi * x2 / (PI * sqrt(PI)) * 8.0 * PI * fw[k];
            for (int a = -nimg; a <= nimg; ++a)
                for (int b = -nimg; b <= nimg; ++b)
                    for (int e3 = -nimg; e3 <= nimg; ++e3) {
                        const double r[3] = {d[0] - L * a, d[1] - L * b, d[2] - L * e3};
                        const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                        if (rr >= rc * rc || rr == 0.0) continue;
                        const double rho = sqrt(rr), e = exp(-x2 * rr), ec = erfc(xi * rho) / (rho * rr);
                        const double A = c * e * (8.0 * x2 - 4.0 * x4 * rr + 2.0 / rr) + 2.0 * ec;
                        const double B = (c * e * (-4.0 * x2 + 4.0 * x4 * rr - 6.0 / rr) - 6.0 * ec) / rr;
                        const double rf = r[0] * fw[0] + r[1] * fw[1] + r[2] * fw[2];
                        for (int k = 0; k < 3; ++k) u[k] += A * fw[k] + B * rf * r[k];
                    }
        }
        for (int k = 0; k < 3; ++k) out[3 * t + k] = u[k] / (8.0 * PI);
    }
}

/*
 * Real-space part of the triply periodic double layer grad G : D^s (the
 * Stokeslet's gradient contracted with the symmetric part of D, Hasimoto
 * split as above): with A = erfc(xi r)/r - c e, B = (erfc(xi r)/r + c e)/r^2
 * (8 pi G_R = A I + B r r^T),
 *   8 pi (grad G_R : D)_i = (A'/r + B) (D r)_i + (B'/r (r.D.r) + B tr D) r_i,
 *   A'/r + B = 2 c xi^2 e,  B'/r = -3 erfc(xi r)/r^5 - 3 c e/r^4 - 2 c xi^2 e/r^2.
 * The smooth part is odd: no self term.  D [ns][9] row-major; out [nt][3]
 * overwritten.
 */
void oracle_stokes_dl_ewald_real(int64_t ns, const double *ys, const double *D, int64_t nt, const double *xs,
                                 double L, double xi, double rc, double *out)
{
    const double c = 2.0 * xi / sqrt(PI);
    const int nimg = (int)floor(rc / L + 0.5);
    const double x2 = xi * xi;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        double u[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < ns; ++j) {
            double d[3], S[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) S[3 * a + b] = 0.5 * (D[9 * j + 3 * a + b] + D[9 * j + 3 * b + a]);
            const double tr = S[0] + S[4] + S[8];
            for (int k = 0; k < 3; ++k) {
                d[k] = xs[3 * t + k] - ys[3 * j + k];
                d[k] -= L * nearbyint(d[k] / L);
            }
            for (int a = -nimg; a <= nimg; ++a)
                for (int b = -nimg; b <= nimg; ++b)
                    for (int e3 = -nimg; e3 <= nimg; ++e3) {
                        const double r[3] = {d[0] - L * a, d[1] - L * b, d[2] - L * e3};
                        const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                        if (rr >= rc * rc || rr == 0.0) continue;
                        const double rho = sqrt(rr), e = exp(-x2 * rr), ec = erfc(xi * rho);
                        const double c1 = 2.0 * c * x2 * e;
                        const double bpr = -3.0 * ec / (rr * rr * rho) - 3.0 * c * e / (rr * rr) - 2.0 * c * x2 * e / rr;
                        const double B = (ec / rho + c * e) / rr;
                        double Dr[3], rDr = 0.0;
                        for (int k = 0; k < 3; ++k) {
                            Dr[k] = S[3 * k] * r[0] + S[3 * k + 1] * r[1] + S[3 * k + 2] * r[2];
                            rDr += r[k] * Dr[k];
                        }
                        const double c2 = bpr * rDr + B * tr;
                        for (int k = 0; k < 3; ++k) u[k] += c1 * Dr[k] + c2 * r[k];
                    }
        }
        for (int k = 0; k < 3; ++k) out[3 * t + k] = u[k] / (8.0 * PI);
    }
}

