// Precomputed translation operators of the Laplace ML tree (host, FP64).
//
// Every problem uses the scalar Laplace kernel L = 1/(4 pi r) on its ML tree
// (Sec. II, kernel aggregation), so one operator set per order p serves all
// kernels.  Operators are built for a box of side 1 centred at the origin;
// L is homogeneous of degree -1, so a box of side h uses them scaled by 1/h
// (check potentials) or h (pseudo-inverse).
//
//   surfaces      cube-surface lattice with p points per edge, M = 6(p-1)^2+2
//                 points (Sec. III); radii a_in (upward equivalent, downward
//                 check) and a_out (upward check, downward equivalent).
//   UC2UE         pseudo-inverse of L(uc, ue) by a truncated SVD (Sec. II:
//                 backward-stable SVD instead of Tikhonov), kept as two FP64
//                 factors.  Because L is symmetric and dc = ue, de = uc
//                 (same radii), L(dc, de) = L(uc, ue)^T and DC2DE is the
//                 transpose of UC2UE.
//   M2M[o], L2L[o]  parent/child operators for the 8 octants.
//   M2L[o]        for the 316 relative offsets of the V list.
//   M2L basis     optional compression of the V-list translations: with U_k
//                 the leading left singular vectors of [M2L[o] for all o]
//                 (eigenvectors of S = sum_o M2L[o] M2L[o]^T; since
//                 M2L[-o] = M2L[o]^T, U_k also spans the leading right
//                 singular space), M2L[o] ~ U_k C[o] U_k^T with
//                 C[o] = U_k^T M2L[o] U_k.  k is the number of singular values
//                 above m2l_tol times the largest, rounded up to 32.
//   T_M2L         periodic images beyond the 3x3x3 near block, by Ewald
//                 summation (triply periodic, Sec. III and its appendix).
//   periodic Stokes  the far images of the root for the triply periodic
//                 Stokeslet (Hasimoto's Ewald split), applied through
//                 Stokeslet fits at the root: see build_periodic_stokes.
//
// The SVD is a one-sided Jacobi (Hestenes) iteration with a round-robin
// pair schedule whose rounds run on a pool of host threads.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.hpp"
#include "pool.hpp"

namespace kafmm {

namespace {

constexpr double kPi = 3.14159265358979323846;

void surface_lattice(int p, std::vector<double> &g) {
    g.clear();
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int k = 0; k < p; ++k) {
                if (!(i == 0 || i == p - 1 || j == 0 || j == p - 1 || k == 0 || k == p - 1)) continue;
                g.push_back(-1.0 + 2.0 * i / (p - 1));
                g.push_back(-1.0 + 2.0 * j / (p - 1));
                g.push_back(-1.0 + 2.0 * k / (p - 1));
            }
}

// Laplace matrix K[i][j] = L(x_i - y_j), x_i = cx + ax * g_i, y_j = cy + ay * g_j.
void laplace_block(const std::vector<double> &g, int M, const double cx[3], double ax,
                   const double cy[3], double ay, double *K, int ld) {
    for (int i = 0; i < M; ++i) {
        double x[3] = {cx[0] + ax * g[3 * i], cx[1] + ax * g[3 * i + 1], cx[2] + ax * g[3 * i + 2]};
        for (int j = 0; j < M; ++j) {
            double r0 = x[0] - (cy[0] + ay * g[3 * j]);
            double r1 = x[1] - (cy[1] + ay * g[3 * j + 1]);
            double r2 = x[2] - (cy[2] + ay * g[3 * j + 2]);
            K[i * ld + j] = 1.0 / (4.0 * kPi * std::sqrt(r0 * r0 + r1 * r1 + r2 * r2));
        }
    }
}

// One-sided Jacobi SVD of the square matrix A (row-major, n x n):
// A = U diag(s) V^T.  U, V returned row-major n x n; s descending.  Each
// round of the round-robin schedule rotates disjoint column pairs, split
// over the pool's threads.
void jacobi_svd(Pool &pool, const std::vector<double> &A, int n, std::vector<double> &U,
                std::vector<double> &s, std::vector<double> &V) {
    const int m = n + (n & 1);                // even number of columns for the schedule
    std::vector<double> a(size_t(m) * n, 0.0), v(size_t(m) * m, 0.0);   // column-major
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) a[size_t(j) * n + i] = A[size_t(i) * n + j];
    for (int j = 0; j < m; ++j) v[size_t(j) * m + j] = 1.0;
    // round r pairs slot k with slot m-1-k; slot 0 holds column 0 and slot
    // i >= 1 holds column 1 + ((i - 1 - r) mod (m - 1))
    auto col = [m](int round, int i) { return i == 0 ? 0 : 1 + ((i - 1 - round) % (m - 1) + (m - 1)) % (m - 1); };
    const double eps = 1e-15;
    const int nt = pool.size();
    std::vector<double> offt(nt, 0.0);
    pool.each([&](int t) {
        for (int sweep = 0; sweep < 60; ++sweep) {
            double off_local = 0.0;
            for (int round = 0; round < m - 1; ++round) {
                for (int k = t; k < m / 2; k += nt) {
                    int p = col(round, k), q = col(round, m - 1 - k);
                    if (p > q) std::swap(p, q);
                    double *ap = &a[size_t(p) * n], *aq = &a[size_t(q) * n];
                    double al = 0, be = 0, ga = 0;
                    for (int i = 0; i < n; ++i) {
                        al += ap[i] * ap[i];
                        be += aq[i] * aq[i];
                        ga += ap[i] * aq[i];
                    }
                    if (ga == 0.0 || std::fabs(ga) <= eps * std::sqrt(al * be)) continue;
                    off_local = std::max(off_local, std::fabs(ga) / std::sqrt(al * be));
                    double zeta = (be - al) / (2.0 * ga);
                    double tt = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                    double c = 1.0 / std::sqrt(1.0 + tt * tt), sn = c * tt;
                    for (int i = 0; i < n; ++i) {
                        double x = ap[i], y = aq[i];
                        ap[i] = c * x - sn * y;
                        aq[i] = sn * x + c * y;
                    }
                    double *vp = &v[size_t(p) * m], *vq = &v[size_t(q) * m];
                    for (int i = 0; i < m; ++i) {
                        double x = vp[i], y = vq[i];
                        vp[i] = c * x - sn * y;
                        vq[i] = sn * x + c * y;
                    }
                }
                pool.barrier();
            }
            offt[t] = off_local;
            pool.barrier();
            const double off = *std::max_element(offt.begin(), offt.end());
            pool.barrier();
            if (off < 1e-14) break;
        }
    });
    std::vector<double> nrm(m);
    for (int j = 0; j < m; ++j) {
        double x = 0;
        for (int i = 0; i < n; ++i) x += a[size_t(j) * n + i] * a[size_t(j) * n + i];
        nrm[j] = std::sqrt(x);
    }
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    U.assign(size_t(n) * n, 0.0);
    V.assign(size_t(n) * n, 0.0);
    s.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        int j = ord[k];
        s[k] = nrm[j];
        for (int i = 0; i < n; ++i) {
            U[size_t(i) * n + k] = nrm[j] > 0 ? a[size_t(j) * n + i] / nrm[j] : 0.0;
            V[size_t(i) * n + k] = v[size_t(j) * m + i];
        }
    }
}

// Periodic Laplace potential of a unit charge at separation r, summed over
// all images n with max|n_k| >= 2 of the unit lattice: the Ewald sum (k = 0
// term dropped, zero-mean convention) minus the 27 near images, written so
// that no singular term is formed.
struct FarImages {
    double xi, rc;
    int nmax, nimg;
    std::vector<double> kx, ky, kz, kw;   // half-space reciprocal vectors and weights

    FarImages() {
        xi = 4.0;
        double s = std::sqrt(-std::log(1e-16)) + 0.5;
        rc = s / xi;
        nimg = int(std::ceil(rc + 2.0));
        double kc = 2.0 * xi * s;
        nmax = int(std::ceil(kc / (2.0 * kPi)));
        for (int a = -nmax; a <= nmax; ++a)
            for (int b = -nmax; b <= nmax; ++b)
                for (int c = 0; c <= nmax; ++c) {
                    bool half = c > 0 || (c == 0 && (b > 0 || (b == 0 && a > 0)));
                    if (!half) continue;
                    double k[3] = {2 * kPi * a, 2 * kPi * b, 2 * kPi * c};
                    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                    kx.push_back(k[0]);
                    ky.push_back(k[1]);
                    kz.push_back(k[2]);
                    kw.push_back(2.0 * std::exp(-k2 / (4 * xi * xi)) / k2);
                }
    }

    // real-space part: far images erfc-screened, near images minus their
    // smooth part, plus the zero-mean constant
    double real_part(double r0, double r1, double r2) const {
        double sum = 0.0;
        for (int a = -nimg; a <= nimg; ++a)
            for (int b = -nimg; b <= nimg; ++b)
                for (int c = -nimg; c <= nimg; ++c) {
                    double x = r0 + a, y = r1 + b, z = r2 + c;
                    double rr = x * x + y * y + z * z;
                    bool near = std::abs(a) <= 1 && std::abs(b) <= 1 && std::abs(c) <= 1;
                    if (near) {
                        // remove the smooth part of a near image: erf(xi rho)/(4 pi rho)
                        double rho = std::sqrt(rr);
                        sum -= rho > 0 ? std::erf(xi * rho) / (4 * kPi * rho) : xi / (2 * kPi * std::sqrt(kPi));
                    } else if (rr < rc * rc) {
                        double rho = std::sqrt(rr);
                        sum += std::erfc(xi * rho) / (4 * kPi * rho);
                    }
                }
        return sum - 1.0 / (4.0 * xi * xi);   // zero-mean convention (unit cell volume 1)
    }
};

// Far images of the triply periodic Stokeslet G(r) = (I/r + r r^T/r^3)/(8 pi)
// of a unit force at separation r: all images n with max|n_k| >= 2 of the
// unit lattice, i.e. the Ewald sum minus the 27 near images.  The Ewald sum
// uses Hasimoto's split phi(k) = (1 + k^2/(4 xi^2)) exp(-k^2/(4 xi^2)) of the
// Fourier series (I - k k^T/k^2)/k^2 (net force zero, k = 0 dropped):
//   real part     8 pi G_R = (erfc(xi r)/r - c e) I + (erfc(xi r)/r + c e) r r^T/r^2,
//                 c = 2 xi/sqrt(pi), e = exp(-xi^2 r^2)  (G_R = (I lap - grad grad) B/(8 pi),
//                 B' = erfc(xi r));
//   near images   minus their smooth part G - G_R, which at r = 0 is 2c I/(8 pi);
//   reciprocal    sum_{k != 0} phi(k)/k^2 (I - k k^T/k^2) cos(k.r).
struct StokesFarImages {
    double xi, rc, c;
    std::vector<double> kx, ky, kz, kw;   // half-space reciprocal vectors, weight 2 phi/k^2

    StokesFarImages() {
        xi = 4.0;
        const double s = std::sqrt(-std::log(1e-16)) + 0.5;
        rc = s / xi;
        c = 2.0 * xi / std::sqrt(kPi);
        const int nmax = int(std::ceil(2.0 * xi * s / (2.0 * kPi)));
        for (int a = -nmax; a <= nmax; ++a)
            for (int b = -nmax; b <= nmax; ++b)
                for (int q = 0; q <= nmax; ++q) {
                    const bool half = q > 0 || (q == 0 && (b > 0 || (b == 0 && a > 0)));
                    if (!half) continue;
                    const double k0 = 2 * kPi * a, k1 = 2 * kPi * b, k2 = 2 * kPi * q;
                    const double kk = k0 * k0 + k1 * k1 + k2 * k2, t = kk / (4 * xi * xi);
                    kx.push_back(k0);
                    ky.push_back(k1);
                    kz.push_back(k2);
                    kw.push_back(2.0 * (1.0 + t) * std::exp(-t) / kk);
                }
    }

    // real-space part of the far-image block at separation r, added to B (3x3)
    void real_part(const double r[3], double B[9]) const {
        auto add = [&](const double x[3], double A, double Bc) {
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) B[3 * i + j] += (i == j ? A : 0.0) + Bc * x[i] * x[j];
        };
        const double inv8pi = 1.0 / (8.0 * kPi);
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b)
                for (int q = -1; q <= 1; ++q) {
                    const double x[3] = {r[0] + a, r[1] + b, r[2] + q};
                    const double rho = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                    if (rho == 0.0) {
                        add(x, -2.0 * c * inv8pi, 0.0);
                        continue;
                    }
                    const double e = std::exp(-xi * xi * rho * rho), ef = std::erf(xi * rho) / rho;
                    add(x, -(ef + c * e) * inv8pi, -(ef - c * e) / (rho * rho) * inv8pi);
                }
        int lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = int(std::floor(-r[k] - rc));
            hi[k] = int(std::ceil(-r[k] + rc));
        }
        for (int a = lo[0]; a <= hi[0]; ++a)
            for (int b = lo[1]; b <= hi[1]; ++b)
                for (int q = lo[2]; q <= hi[2]; ++q) {
                    if (std::abs(a) <= 1 && std::abs(b) <= 1 && std::abs(q) <= 1) continue;
                    const double x[3] = {r[0] + a, r[1] + b, r[2] + q};
                    const double rr = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
                    if (rr >= rc * rc) continue;
                    const double rho = std::sqrt(rr);
                    const double e = std::exp(-xi * xi * rr), ec = std::erfc(xi * rho) / rho;
                    add(x, (ec - c * e) * inv8pi, (ec + c * e) / rr * inv8pi);
                }
    }
};

// Far images of the doubly periodic Stokeslet (periods 1 in x and y, open in
// z) of a unit force at separation r: the in-plane images n = (n_x, n_y, 0)
// with max(|n_x|, |n_y|) >= 2, i.e. the doubly periodic Ewald sum minus the 9
// near images.  The sum is the Fourier series in x and y; its k_par = 0 mode
// is the sheet flow -|z|/2 (zero net force, no added constant).  With
// Hasimoto's split and kappa = |k_par|:
//   real part     the screened kernel G_R (as above) over the far images;
//   near images   minus their smooth part G - G_R (2c I/(8 pi) at r = 0);
//   spectral      per mode k_par != 0 the k_z integral of phi (I - k k^T/k^2)/k^2:
//                 G_ab = cos(k.r) (delta_ab I2 - k_a k_b I4),
//                 G_az = G_za = sin(k.r) k_a z E2/2,  G_zz = cos(k.r) kappa^2 I4,
//                 E2 = (e^{kappa z} erfc(kappa/2xi + xi z) + e^{-kappa z} erfc(kappa/2xi - xi z))/(4 kappa),
//                 E0 = (xi/sqrt(pi)) g, g = e^{-kappa^2/4xi^2 - xi^2 z^2},  I2 = E2 + E0/(4 xi^2),
//                 I4 = -(1/2 kappa) dE2/dkappa
//                    = E2/(2 kappa^2) - (z D - 2 g/(xi sqrt(pi)))/(8 kappa^2),
//                 D = e^{kappa z} erfc(kappa/2xi + xi z) - e^{-kappa z} erfc(kappa/2xi - xi z);
//                 the mode k_par = 0: G_ab = delta_ab (-z erf(xi z)/2 - e^{-xi^2 z^2}/(4 xi sqrt(pi))).
struct StokesFarImages2P {
    double xi, rc, c;
    int nk;

    StokesFarImages2P() {
        xi = 4.0;
        const double s = std::sqrt(-std::log(1e-16)) + 0.5;
        rc = s / xi;
        c = 2.0 * xi / std::sqrt(kPi);
        nk = int(std::ceil(2.0 * xi * s / (2.0 * kPi)));
    }

    // e^{sg kappa Z} erfc(kappa/2xi + sg xi Z), Z >= 0, without overflow:
    // g * exp(a^2) erfc(a) when a >= 0 (asymptotic series for large a)
    double exp_erfc(double kap, double Z, double g, double sg) const {
        const double a = kap / (2.0 * xi) + sg * xi * Z;
        if (a < 0.0) return std::exp(sg * kap * Z) * std::erfc(a);
        double sx;
        if (a < 26.0) {
            sx = std::exp(a * a) * std::erfc(a);
        } else {
            double term = 1.0, sum = 1.0;
            const double h = 1.0 / (2.0 * a * a);
            for (int n = 1; n < 40; ++n) {
                const double nx = -term * (2 * n - 1) * h;
                if (std::fabs(nx) >= std::fabs(term) || std::fabs(nx) < 1e-17) break;
                term = nx;
                sum += nx;
            }
            sx = sum / (a * std::sqrt(kPi));
        }
        return g * sx;
    }

    // far-image block at separation r, added to B (3x3)
    void block(const double r[3], double B[9]) const {
        const double inv8pi = 1.0 / (8.0 * kPi);
        auto add = [&](const double x[3], double A, double Bc) {
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) B[3 * i + j] += (i == j ? A : 0.0) + Bc * x[i] * x[j];
        };
        const int nr = int(std::ceil(rc)) + 2;
        for (int a = -nr; a <= nr; ++a)
            for (int b = -nr; b <= nr; ++b) {
                const double x[3] = {r[0] + a, r[1] + b, r[2]};
                const double rr = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
                if (std::abs(a) <= 1 && std::abs(b) <= 1) {
                    if (rr == 0.0) {
                        add(x, -2.0 * c * inv8pi, 0.0);
                        continue;
                    }
                    const double rho = std::sqrt(rr), e = std::exp(-xi * xi * rr), ef = std::erf(xi * rho) / rho;
                    add(x, -(ef + c * e) * inv8pi, -(ef - c * e) / rr * inv8pi);
                    continue;
                }
                if (rr >= rc * rc) continue;
                const double rho = std::sqrt(rr), e = std::exp(-xi * xi * rr), ec = std::erfc(xi * rho) / rho;
                add(x, (ec - c * e) * inv8pi, (ec + c * e) / rr * inv8pi);
            }
        const double z = r[2], Z = std::fabs(z), sg = z < 0.0 ? -1.0 : 1.0, x2 = xi * xi;
        for (int mx = -nk; mx <= nk; ++mx)
            for (int my = -nk; my <= nk; ++my) {
                if (mx == 0 && my == 0) continue;
                const double kx = 2.0 * kPi * mx, ky = 2.0 * kPi * my, k2 = kx * kx + ky * ky, kap = std::sqrt(k2);
                const double ph = kx * r[0] + ky * r[1], cs = std::cos(ph), sn = std::sin(ph);
                const double g = std::exp(-k2 / (4.0 * x2) - x2 * z * z);
                const double P = exp_erfc(kap, Z, g, 1.0), Q = exp_erfc(kap, Z, g, -1.0);
                const double E2 = (P + Q) / (4.0 * kap), D = sg * (P - Q), E0 = g * xi / std::sqrt(kPi);
                const double I2 = E2 + E0 / (4.0 * x2);
                const double I4 = E2 / (2.0 * k2) - (z * D - 2.0 * g / (xi * std::sqrt(kPi))) / (8.0 * k2);
                const double kv[2] = {kx, ky};
                for (int a = 0; a < 2; ++a) {
                    for (int b = 0; b < 2; ++b) B[3 * a + b] += cs * ((a == b ? I2 : 0.0) - kv[a] * kv[b] * I4);
                    B[3 * a + 2] += sn * kv[a] * z * E2 / 2.0;
                    B[6 + a] += sn * kv[a] * z * E2 / 2.0;
                }
                B[8] += cs * k2 * I4;
            }
        const double s0 = -z * std::erf(xi * z) / 2.0 - std::exp(-x2 * z * z) / (4.0 * xi * std::sqrt(kPi));
        B[0] += s0;
        B[4] += s0;
    }
};

// Stokeslet block G(x - y) (row-major 3x3)
void stokeslet_block(const double x[3], const double y[3], double G[9]) {
    const double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2], ri = 1.0 / std::sqrt(r2);
    const double s = ri / (8.0 * kPi), s3 = s / r2;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[3 * i + j] = (i == j ? s : 0.0) + s3 * r[i] * r[j];
}

// X <- pinv(G) X for a square n x n G (truncated SVD, relative tol), X n x m
void apply_pinv(Pool &pool, const std::vector<double> &G, int n, double tol, std::vector<double> &X, int m) {
    std::vector<double> U, sv, V;
    jacobi_svd(pool, G, n, U, sv, V);
    int r = 0;
    while (r < n && sv[r] > tol * sv[0]) ++r;
    std::vector<double> Y(size_t(r) * m, 0.0);   // diag(1/s) U^T X
    pool.parallel_for(r, [&](int k) {
        double *y = &Y[size_t(k) * m];
        for (int i = 0; i < n; ++i) {
            const double u = U[size_t(i) * n + k];
            const double *x = &X[size_t(i) * m];
            for (int j = 0; j < m; ++j) y[j] += u * x[j];
        }
        for (int j = 0; j < m; ++j) y[j] /= sv[k];
    });
    pool.parallel_for(n, [&](int i) {
        double *x = &X[size_t(i) * m];
        std::fill(x, x + m, 0.0);
        for (int k = 0; k < r; ++k) {
            const double v = V[size_t(i) * n + k];
            const double *y = &Y[size_t(k) * m];
            for (int j = 0; j < m; ++j) x[j] += v * y[j];
        }
    });
}

}  // namespace

std::string build_periodic_stokes(int p, double svd_tol, bool doubly, std::vector<double> &Q,
                                  std::vector<double> &X, std::vector<double> &Z) {
    if (p < 2 || p > 16) return "p must lie in [2, 16]";
    Pool pool(pool_threads());
    std::vector<double> g;
    surface_lattice(p, g);
    const int M = int(g.size() / 3), n3 = 3 * M;
    const double aIn = 0.5 * kAlphaIn, aOut = 0.5 * kAlphaOut;
    auto pt = [&](int m, double a, double x[3]) {
        for (int k = 0; k < 3; ++k) x[k] = a * g[3 * m + k];
    };
    std::vector<double> G(size_t(n3) * n3);
    auto fill_stokeslet = [&](double ax, double ay) {
        pool.parallel_for(M, [&](int i) {
            double x[3], y[3], B[9];
            pt(i, ax, x);
            for (int m = 0; m < M; ++m) {
                pt(m, ay, y);
                stokeslet_block(x, y, B);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) G[size_t(3 * i + a) * n3 + 3 * m + b] = B[3 * a + b];
            }
        });
    };
    // Stokeslet forces on the upward equivalent points (radius a_in) with the
    // root's flow on its upward check surface (radius a_out): W = pinv(G_up).
    // The downward fit (check points at a_in, equivalent points at a_out)
    // has the transposed matrix (G is even and symmetric), so its
    // pseudo-inverse is W^T.
    std::vector<double> W(size_t(n3) * n3, 0.0);
    for (int i = 0; i < n3; ++i) W[size_t(i) * n3 + i] = 1.0;
    fill_stokeslet(aOut, aIn);
    apply_pinv(pool, G, n3, svd_tol, W, n3);
    // their far images at the downward check points (radius a_in, as the
    // upward equivalent points)
    std::vector<double> T(size_t(n3) * n3);
    if (doubly) {
        // separations are a_in * 2 d/(p - 1) for integer d in [-(p-1), p-1]^3:
        // one block per d
        const int w = 2 * p - 1;
        StokesFarImages2P far2;
        std::vector<double> blocks(size_t(w) * w * w * 9);
        pool.parallel_for(w * w * w, [&](int q) {
            const int d[3] = {q % w - (p - 1), (q / w) % w - (p - 1), q / (w * w) - (p - 1)};
            const double r[3] = {aIn * 2.0 * d[0] / (p - 1), aIn * 2.0 * d[1] / (p - 1), aIn * 2.0 * d[2] / (p - 1)};
            double *B = &blocks[size_t(q) * 9];
            for (int k = 0; k < 9; ++k) B[k] = 0.0;
            far2.block(r, B);
        });
        auto lattice = [&](double v) { return int(std::lround((v + 1.0) * (p - 1) / 2.0)); };
        pool.parallel_for(M, [&](int i) {
            for (int m = 0; m < M; ++m) {
                const int q = (lattice(g[3 * i]) - lattice(g[3 * m]) + p - 1) +
                              w * (lattice(g[3 * i + 1]) - lattice(g[3 * m + 1]) + p - 1) +
                              w * w * (lattice(g[3 * i + 2]) - lattice(g[3 * m + 2]) + p - 1);
                const double *B = &blocks[size_t(q) * 9];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) T[size_t(3 * i + a) * n3 + 3 * m + b] = B[3 * a + b];
            }
        });
    } else {
        StokesFarImages far;
        const int nk = int(far.kw.size());
        std::vector<double> C(size_t(M) * nk), S(size_t(M) * nk), KK(size_t(6) * nk);
        for (int k = 0; k < nk; ++k) {
            const double kk = far.kx[k] * far.kx[k] + far.ky[k] * far.ky[k] + far.kz[k] * far.kz[k];
            const double kv[3] = {far.kx[k], far.ky[k], far.kz[k]};
            int q = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = a; b < 3; ++b) KK[size_t(q++) * nk + k] = kv[a] * kv[b] / kk;
        }
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < nk; ++k) {
                const double ph = aIn * (far.kx[k] * g[3 * i] + far.ky[k] * g[3 * i + 1] + far.kz[k] * g[3 * i + 2]);
                C[size_t(i) * nk + k] = std::cos(ph);
                S[size_t(i) * nk + k] = std::sin(ph);
            }
        pool.parallel_for(M, [&](int i) {
            for (int m = 0; m < M; ++m) {
                const double r[3] = {aIn * (g[3 * i] - g[3 * m]), aIn * (g[3 * i + 1] - g[3 * m + 1]),
                                     aIn * (g[3 * i + 2] - g[3 * m + 2])};
                double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                far.real_part(r, B);
                double s0 = 0.0, sq[6] = {0, 0, 0, 0, 0, 0};
                const double *ci = &C[size_t(i) * nk], *cm = &C[size_t(m) * nk];
                const double *si = &S[size_t(i) * nk], *sm = &S[size_t(m) * nk];
                for (int k = 0; k < nk; ++k) {
                    const double w = far.kw[k] * (ci[k] * cm[k] + si[k] * sm[k]);
                    s0 += w;
                    for (int q = 0; q < 6; ++q) sq[q] += w * KK[size_t(q) * nk + k];
                }
                const int qi[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        T[size_t(3 * i + a) * n3 + 3 * m + b] = B[3 * a + b] + (a == b ? s0 : 0.0) - sq[qi[a][b]];
            }
        });
    }
    std::vector<double> TW(size_t(n3) * n3, 0.0);   // T W
    pool.parallel_for(n3, [&](int i) {
        double *y = &TW[size_t(i) * n3];
        for (int k = 0; k < n3; ++k) {
            const double t = T[size_t(i) * n3 + k];
            const double *w = &W[size_t(k) * n3];
            for (int j = 0; j < n3; ++j) y[j] += t * w[j];
        }
    });
    // Stokeslet forces on the downward equivalent points (radius a_out) with
    // that field on the downward check surface (inside it they give the far
    // images' flow): Q = W^T T W
    Q.assign(size_t(n3) * n3, 0.0);
    pool.parallel_for(n3, [&](int i) {
        double *y = &Q[size_t(i) * n3];
        for (int k = 0; k < n3; ++k) {
            const double w = W[size_t(k) * n3 + i];
            const double *t = &TW[size_t(k) * n3];
            for (int j = 0; j < n3; ++j) y[j] += w * t[j];
        }
    });
    X.resize(size_t(n3));
    Z.resize(size_t(n3));
    for (int m = 0; m < M; ++m) {
        pt(m, aOut, &X[3 * size_t(m)]);
        pt(m, aOut, &Z[3 * size_t(m)]);
    }
    return "";
}

std::string build_operators(int p, double svd_tol, bool periodic, Operators &ops, double m2l_tol) {
    if (p < 2 || p > 16) return "p must lie in [2, 16]";
    ops = Operators();
    ops.p = p;
    ops.svd_tol = svd_tol;
    ops.m2l_tol = m2l_tol;
    Pool pool(pool_threads());
    surface_lattice(p, ops.grid);
    const int M = int(ops.grid.size() / 3);
    const int Mp = (M + 31) / 32 * 32;
    ops.M = M;
    ops.Mp = Mp;
    const double zero[3] = {0, 0, 0};
    const double aIn = 0.5 * kAlphaIn, aOut = 0.5 * kAlphaOut;   // half-side radii, side 1

    // UC2UE = pinv(L(uc, ue)) = V S^+ U^T
    std::vector<double> K(size_t(M) * M), U, s, V;
    laplace_block(ops.grid, M, zero, aOut, zero, aIn, K.data(), M);
    jacobi_svd(pool, K, M, U, s, V);
    int r = 0;
    while (r < M && s[r] > svd_tol * s[0]) ++r;
    ops.rank = r;
    ops.up1.assign(size_t(M) * r, 0.0);   // V S^+  [M][r]
    ops.up2.assign(size_t(r) * M, 0.0);   // U^T    [r][M]
    for (int i = 0; i < M; ++i)
        for (int k = 0; k < r; ++k) ops.up1[size_t(i) * r + k] = V[size_t(i) * M + k] / s[k];
    for (int k = 0; k < r; ++k)
        for (int j = 0; j < M; ++j) ops.up2[size_t(k) * M + j] = U[size_t(j) * M + k];

    // octant operators (parent side 1, child side 1/2, child centre +-1/4).
    // The downward translation maps the parent's check potentials straight to
    // the child's: L2L[o] * DC2DE (child dc <- parent de <- parent dc), formed
    // here in FP64; it is scale free (the two factors scale as 1/h and h).
    ops.m2m.assign(size_t(8) * Mp * Mp, 0.0f);
    ops.l2l_cc.assign(size_t(8) * M * M, 0.0);
    std::vector<double> dc2de(size_t(M) * M, 0.0);   // DC2DE = P2^T P1^T (side 1)
    pool.parallel_for(M, [&](int i) {
        for (int j = 0; j < M; ++j) {
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc += ops.up2[size_t(k) * M + i] * ops.up1[size_t(j) * r + k];
            dc2de[size_t(i) * M + j] = acc;
        }
    });
    pool.parallel_for(8, [&](int o) {
        std::vector<double> B(size_t(M) * M);
        double c[3] = {((o >> 2) & 1) ? 0.25 : -0.25, ((o >> 1) & 1) ? 0.25 : -0.25, (o & 1) ? 0.25 : -0.25};
        laplace_block(ops.grid, M, zero, aOut, c, 0.5 * aIn, B.data(), M);   // parent uc <- child ue
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) ops.m2m[(size_t(o) * Mp + i) * Mp + j] = float(B[size_t(i) * M + j]);
        laplace_block(ops.grid, M, c, 0.5 * aIn, zero, aOut, B.data(), M);   // child dc <- parent de
        double *L = &ops.l2l_cc[size_t(o) * M * M];
        for (int i = 0; i < M; ++i) {
            const double *bi = &B[size_t(i) * M];
            for (int k = 0; k < M; ++k) {
                const double b = bi[k];
                const double *dk = &dc2de[size_t(k) * M];
                for (int j = 0; j < M; ++j) L[size_t(i) * M + j] += b * dk[j];
            }
        }
    });
    // V-list offsets: dense operators, or the compressed basis and cores
    auto is_v_offset = [](int idx) {
        const int ox = idx % 7 - 3, oy = (idx / 7) % 7 - 3, oz = idx / 49 - 3;
        return std::max({std::abs(ox), std::abs(oy), std::abs(oz)}) >= 2;
    };
    auto m2l_block = [&](int idx, std::vector<double> &Bl) {
        const double c[3] = {double(idx % 7 - 3), double((idx / 7) % 7 - 3), double(idx / 49 - 3)};
        Bl.resize(size_t(M) * M);
        laplace_block(ops.grid, M, zero, aIn, c, aIn, Bl.data(), M);   // target dc <- source ue
    };
    int kc = 0;
    std::vector<double> Ub;   // [M][kc] basis (row-major)
    if (m2l_tol > 0) {
        // S = sum_o B_o B_o^T, each thread summing its own offsets (upper triangle)
        const int nt = pool.size();
        std::vector<std::vector<double>> Sp(nt, std::vector<double>(size_t(M) * M, 0.0));
        pool.each([&](int t) {
            std::vector<double> Bl;
            double *S = Sp[t].data();
            for (int idx = t; idx < 343; idx += nt) {
                if (!is_v_offset(idx)) continue;
                m2l_block(idx, Bl);
                for (int i = 0; i < M; ++i) {
                    const double *bi = &Bl[size_t(i) * M];
                    for (int j = i; j < M; ++j) {
                        const double *bj = &Bl[size_t(j) * M];
                        double d0 = 0, d1 = 0, d2 = 0, d3 = 0;
                        int l = 0;
                        for (; l + 4 <= M; l += 4) {
                            d0 += bi[l] * bj[l];
                            d1 += bi[l + 1] * bj[l + 1];
                            d2 += bi[l + 2] * bj[l + 2];
                            d3 += bi[l + 3] * bj[l + 3];
                        }
                        for (; l < M; ++l) d0 += bi[l] * bj[l];
                        S[size_t(i) * M + j] += (d0 + d1) + (d2 + d3);
                    }
                }
            }
        });
        std::vector<double> S(size_t(M) * M, 0.0);
        for (int t = 0; t < nt; ++t)
            for (size_t e = 0; e < S.size(); ++e) S[e] += Sp[t][e];
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < i; ++j) S[size_t(i) * M + j] = S[size_t(j) * M + i];
        std::vector<double> Us, ss, Vs;
        jacobi_svd(pool, S, M, Us, ss, Vs);          // S = Us diag(ss) Us^T, ss = singular values^2
        int k = 0;
        while (k < M && ss[k] > m2l_tol * m2l_tol * ss[0]) ++k;
        kc = (k + 31) / 32 * 32;
        if (kc > M || 4 * kc > 3 * Mp) kc = 0;      // not worth compressing
        if (kc > 0) {
            Ub.assign(size_t(M) * kc, 0.0);
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < kc; ++j) Ub[size_t(i) * kc + j] = Us[size_t(i) * M + j];
        }
    }
    ops.kc = kc;
    if (kc == 0) {
        ops.m2l.assign(size_t(343) * Mp * Mp, 0.0f);
        pool.parallel_for(343, [&](int idx) {
            if (!is_v_offset(idx)) return;
            std::vector<double> Bl;
            m2l_block(idx, Bl);
            float *dst = &ops.m2l[size_t(idx) * Mp * Mp];
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j) dst[size_t(i) * Mp + j] = float(Bl[size_t(i) * M + j]);
        });
    } else {
        ops.cbasis.assign(size_t(Mp) * kc, 0.0f);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < kc; ++j) ops.cbasis[size_t(i) * kc + j] = float(Ub[size_t(i) * kc + j]);
        ops.m2l_c.assign(size_t(343) * kc * kc, 0.0f);
        pool.parallel_for(343, [&](int idx) {
            if (!is_v_offset(idx)) return;
            std::vector<double> Bl, T(size_t(M) * kc, 0.0), C(size_t(kc) * kc, 0.0);
            m2l_block(idx, Bl);
            for (int i = 0; i < M; ++i) {             // T = B U
                double *ti = &T[size_t(i) * kc];
                for (int l = 0; l < M; ++l) {
                    const double b = Bl[size_t(i) * M + l];
                    const double *ul = &Ub[size_t(l) * kc];
                    for (int j = 0; j < kc; ++j) ti[j] += b * ul[j];
                }
            }
            for (int l = 0; l < M; ++l) {             // C = U^T T
                const double *ul = &Ub[size_t(l) * kc], *tl = &T[size_t(l) * kc];
                for (int i = 0; i < kc; ++i) {
                    const double u = ul[i];
                    double *ci = &C[size_t(i) * kc];
                    for (int j = 0; j < kc; ++j) ci[j] += u * tl[j];
                }
            }
            float *dst = &ops.m2l_c[size_t(idx) * kc * kc];
            for (size_t e = 0; e < C.size(); ++e) dst[e] = float(C[e]);
        });
    }
    if (periodic) {
        // T[i][j] = sum over far images of L(dc_i - ue_j - n); dc and ue are
        // the same point set (radius a_in).  Reciprocal part factorised:
        // cos(k.(x_i - x_j)) = cos k.x_i cos k.x_j + sin k.x_i sin k.x_j.
        FarImages far;
        const int nk = int(far.kw.size());
        std::vector<double> C(size_t(M) * nk), S(size_t(M) * nk);
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < nk; ++k) {
                double ph = aIn * (far.kx[k] * ops.grid[3 * i] + far.ky[k] * ops.grid[3 * i + 1] +
                                   far.kz[k] * ops.grid[3 * i + 2]);
                C[size_t(i) * nk + k] = std::cos(ph);
                S[size_t(i) * nk + k] = std::sin(ph);
            }
        ops.t_m2l.assign(size_t(M) * M, 0.0);
        pool.parallel_for(M, [&](int i) {
            for (int j = 0; j < M; ++j) {
                double r0 = aIn * (ops.grid[3 * i] - ops.grid[3 * j]);
                double r1 = aIn * (ops.grid[3 * i + 1] - ops.grid[3 * j + 1]);
                double r2 = aIn * (ops.grid[3 * i + 2] - ops.grid[3 * j + 2]);
                double rec = 0.0;
                const double *ci = &C[size_t(i) * nk], *cj = &C[size_t(j) * nk];
                const double *si = &S[size_t(i) * nk], *sj = &S[size_t(j) * nk];
                for (int k = 0; k < nk; ++k) rec += far.kw[k] * (ci[k] * cj[k] + si[k] * sj[k]);
                ops.t_m2l[size_t(i) * M + j] = far.real_part(r0, r1, r2) + rec;
            }
        });
    }
    return "";
}

}  // namespace kafmm
