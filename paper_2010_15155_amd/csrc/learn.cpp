// Host side of the learned order / leaf-capacity predictor: per-leaf
// features and the per-leaf cost model behind the capacity labels.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace kafmm {

namespace {

// number of keys of a sorted array inside the box (level, anchor)
int64_t count_in(const std::vector<uint64_t> &keys, int level, const int32_t a[3]) {
    const int n = 1 << level;
    for (int k = 0; k < 3; ++k)
        if (a[k] < 0 || a[k] >= n) return 0;
    const int sh = 3 * (kKeyBits - level);
    const uint64_t lo = morton_prefix(level, a) << sh, hi = (morton_prefix(level, a) + 1) << sh;
    return int64_t(std::lower_bound(keys.begin(), keys.end(), hi) - std::lower_bound(keys.begin(), keys.end(), lo));
}

struct Counter {
    const Tree &t;
    int64_t src(int level, const int32_t a[3]) const {
        return count_in(t.keys_sl, level, a) + count_in(t.keys_dl, level, a);
    }
    int64_t trg(int level, const int32_t a[3]) const { return count_in(t.keys_trg, level, a); }
    int64_t most(int level, const int32_t a[3]) const {
        return std::max({count_in(t.keys_sl, level, a), count_in(t.keys_dl, level, a), trg(level, a)});
    }
    // sources in the 3x3x3 block of same-level boxes around (level, a)
    int64_t near(int level, const int32_t a[3]) const {
        int64_t s = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int32_t b[3] = {a[0] + dx, a[1] + dy, a[2] + dz};
                    s += src(level, b);
                }
        return s;
    }
    // non-empty (sources) children of the parent's neighbours not adjacent to the box
    int64_t vcount(int level, const int32_t a[3]) const {
        if (level < 2) return 0;
        int32_t p[3] = {a[0] >> 1, a[1] >> 1, a[2] >> 1};
        int64_t v = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    for (int o = 0; o < 8; ++o) {
                        int32_t c[3] = {2 * (p[0] + dx) + ((o >> 2) & 1), 2 * (p[1] + dy) + ((o >> 1) & 1),
                                        2 * (p[2] + dz) + (o & 1)};
                        if (std::abs(c[0] - a[0]) <= 1 && std::abs(c[1] - a[1]) <= 1 && std::abs(c[2] - a[2]) <= 1)
                            continue;
                        if (src(level, c) > 0) ++v;
                    }
        return v;
    }
};

}  // namespace

void leaf_features(const Tree &t, const double *sl, const double *dl, const double *trg, double tol,
                   std::vector<float> &out) {
    (void)dl;
    const size_t nl = t.leaves.size();
    out.assign(nl * kNumFeatures, 0.0f);
    for (size_t i = 0; i < nl; ++i) {
        const int b = t.leaves[i];
        const Box &B = t.boxes[b];
        const double h = 1.0 / double(1 << B.level);
        const double c[3] = {(B.anchor[0] + 0.5) * h, (B.anchor[1] + 0.5) * h, (B.anchor[2] + 0.5) * h};
        const int64_t nt = B.trg[1] - B.trg[0], ns = B.nsrc_sub;
        // moments of the leaf's targets (or its SL sources) in box units u in [-1,1]^3
        const bool use_t = nt > 0;
        const int64_t r0 = use_t ? B.trg[0] : B.sl[0], r1 = use_t ? B.trg[1] : B.sl[1];
        const std::vector<int32_t> &perm = use_t ? t.perm_trg : t.perm_sl;
        const double *xs = use_t ? trg : sl;
        double s2[3] = {0, 0, 0}, face = 0;
        for (int64_t j = r0; j < r1; ++j) {
            const double *x = xs + 3 * int64_t(perm[j]);
            double m = 0;
            for (int k = 0; k < 3; ++k) {
                double u = (x[k] - c[k]) / (0.5 * h);
                s2[k] += u * u;
                m = std::max(m, std::fabs(u));
            }
            face += m;
        }
        const double n = double(std::max<int64_t>(r1 - r0, 1));
        for (double &v : s2) v /= n;
        const double mean2 = (s2[0] + s2[1] + s2[2]) / 3.0;
        const double aniso = (std::max({s2[0], s2[1], s2[2]}) - std::min({s2[0], s2[1], s2[2]})) / (mean2 + 1e-12);
        int64_t near = 0;
        for (int e = t.u_off[b]; e < t.u_off[b + 1]; ++e) near += t.boxes[t.u[e].box].nsrc_sub;
        float *f = &out[i * kNumFeatures];
        f[0] = float(std::log2(1.0 + nt));
        f[1] = float(std::log2(1.0 + ns));
        f[2] = float(B.level);
        f[3] = float(mean2);
        f[4] = float(face / n);
        f[5] = float(aniso);
        f[6] = float(std::log2(1.0 + (t.u_off[b + 1] - t.u_off[b])));
        f[7] = float(std::log2(1.0 + (t.v_off[b + 1] - t.v_off[b])));
        f[8] = float(std::log2(1.0 + (t.w_off[b + 1] - t.w_off[b])));
        f[9] = float(std::log2(1.0 + (t.x_off[b + 1] - t.x_off[b])));
        f[10] = float(std::log2(1.0 + near));
        f[11] = float(std::log10(tol));
    }
}

void leaf_costs(const Tree &t, const double rates[4], int M, int Mp, int ncomp, std::vector<double> &out) {
    const size_t nl = t.leaves.size();
    out.assign(nl * 4, 0.0);
    Counter cnt{t};
    const double m2l_flops = 2.0 * double(Mp) * double(Mp) * ncomp;
    struct B3 {
        int level;
        int32_t a[3];
    };
    std::vector<B3> stack;
    for (size_t i = 0; i < nl; ++i) {
        const Box &L = t.boxes[t.leaves[i]];
        for (int ci = 0; ci < 4; ++ci) {
            const int cap = kCapClasses[ci];
            double pairs = 0, evals = 0, flops = 0, boxes = 0;
            stack.assign(1, B3{L.level, {L.anchor[0], L.anchor[1], L.anchor[2]}});
            while (!stack.empty()) {
                B3 b = stack.back();
                stack.pop_back();
                const int64_t nt = cnt.trg(b.level, b.a), ns = cnt.src(b.level, b.a);
                if (nt + ns == 0) continue;
                boxes += 1;
                flops += double(cnt.vcount(b.level, b.a)) * m2l_flops;
                if (cnt.most(b.level, b.a) > cap && b.level < kMaxLevel) {
                    for (int o = 0; o < 8; ++o)
                        stack.push_back(B3{b.level + 1, {2 * b.a[0] + ((o >> 2) & 1), 2 * b.a[1] + ((o >> 1) & 1),
                                                         2 * b.a[2] + (o & 1)}});
                } else {
                    pairs += double(nt) * double(cnt.near(b.level, b.a));
                    evals += double(nt + ns) * M;
                }
            }
            out[i * 4 + ci] = pairs / rates[0] + flops / rates[1] + evals / rates[2] + boxes * rates[3];
        }
    }
}

}  // namespace kafmm
