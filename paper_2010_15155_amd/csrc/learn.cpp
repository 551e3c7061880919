// Host side of the learned order / leaf-capacity predictor: per-leaf
// features of a tree.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace kafmm {

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

}  // namespace kafmm
