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

}  // namespace

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
