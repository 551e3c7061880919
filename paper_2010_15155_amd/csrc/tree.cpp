// Adaptive octree and U/V/W/X interaction lists (host).
//
// The paper uses the standard KIFMM lists and defers their definitions to
// the KIFMM literature (Sec. II, "we omit those technical details"); the
// definitions implemented here:
//   colleagues(B)  same-level boxes adjacent to B (B included); with periodic
//                  boundaries these are images (box, shift) of boxes;
//   U(B), B leaf   leaves adjacent to B (B included), at any level;
//   V(B)           children of colleagues of parent(B) not adjacent to B;
//   W(B), B leaf   descendants of B's colleagues not adjacent to B whose
//                  parent is adjacent to B;
//   X(B)           boxes A with B in W(A).
// A box is split while it holds more than leaf_cap targets, SL sources or DL
// sources (Sec. III splits on targets with leaf_cap = 2000); empty boxes are
// not created.  Boxes are ordered breadth-first (level-sorted), points within
// a set by Morton key then input index, so the tree is deterministic.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "internal.hpp"
#include "pool.hpp"

namespace kafmm {

namespace {

inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

inline uint32_t grid_coord(double u) {
    const double scale = double(1u << kKeyBits);
    double g = std::floor(u * scale);
    if (g < 0) g = 0;
    if (g > scale - 1) g = scale - 1;
    return uint32_t(g);
}

// Octant digit order: (x bit << 2) | (y bit << 1) | z bit.
inline uint64_t morton(const double *p) {
    return (spread3(grid_coord(p[0])) << 2) | (spread3(grid_coord(p[1])) << 1) |
           spread3(grid_coord(p[2]));
}

struct Sorted {
    std::vector<uint64_t> key;
    std::vector<int32_t> perm;
};

// Stable LSD radix sort of the 63-bit Morton keys (six 11-bit digits) with
// the input index as payload: ties keep input order, as the tree requires.
Sorted sort_points(Pool &pool, const double *x, int64_t n) {
    Sorted s;
    s.key.resize(n);
    s.perm.resize(n);
    if (n == 0) return s;
    std::vector<uint64_t> k2(n);
    std::vector<int32_t> p2(n);
    const int nt = pool.size();
    pool.each([&](int t) {
        for (int64_t i = n * t / nt; i < n * (t + 1) / nt; ++i) {
            s.key[i] = morton(x + 3 * i);
            s.perm[i] = int32_t(i);
        }
    });
    // each pass: per-thread histograms of contiguous chunks, offsets in
    // (digit, thread) order, then each thread scatters its chunk in order
    constexpr int kDigit = 11, kBins = 1 << kDigit;
    std::vector<int64_t> count(size_t(nt) * kBins);
    uint64_t *ka = s.key.data(), *kb = k2.data();
    int32_t *pa = s.perm.data(), *pb = p2.data();
    for (int shift = 0; shift < 3 * kKeyBits; shift += kDigit) {
        pool.each([&](int t) {
            int64_t *c = &count[size_t(t) * kBins];
            std::fill(c, c + kBins, 0);
            for (int64_t i = n * t / nt; i < n * (t + 1) / nt; ++i) ++c[(ka[i] >> shift) & (kBins - 1)];
        });
        int64_t sum = 0;
        bool trivial = false;
        for (int b = 0; b < kBins; ++b) {
            int64_t tot = 0;
            for (int t = 0; t < nt; ++t) tot += count[size_t(t) * kBins + b];
            if (tot == n) trivial = true;      // one digit value: the pass is a no-op
            for (int t = 0; t < nt; ++t) {
                const int64_t c = count[size_t(t) * kBins + b];
                count[size_t(t) * kBins + b] = sum;
                sum += c;
            }
        }
        if (trivial) continue;
        pool.each([&](int t) {
            int64_t *c = &count[size_t(t) * kBins];
            for (int64_t i = n * t / nt; i < n * (t + 1) / nt; ++i) {
                const int64_t d = c[(ka[i] >> shift) & (kBins - 1)]++;
                kb[d] = ka[i];
                pb[d] = pa[i];
            }
        });
        std::swap(ka, kb);
        std::swap(pa, pb);
    }
    if (ka != s.key.data()) {
        std::memcpy(s.key.data(), ka, size_t(n) * sizeof(uint64_t));
        std::memcpy(s.perm.data(), pa, size_t(n) * sizeof(int32_t));
    }
    return s;
}

struct Img {
    int box;
    std::array<int8_t, 3> s;
};

class Lister {
  public:
    explicit Lister(Tree &t) : t_(t) {
        for (size_t i = 0; i < t.boxes.size(); ++i) {
            const Box &b = t.boxes[i];
            map_[box_hash(b.level, b.anchor[0], b.anchor[1], b.anchor[2])] = int(i);
        }
    }

    // Same-level adjacent boxes (images), including the box itself.
    void colleagues(int b, std::vector<Img> &out) const {
        out.clear();
        const Box &B = t_.boxes[b];
        const int32_t n = 1 << B.level;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int d[3] = {dx, dy, dz};
                    int32_t c[3];
                    std::array<int8_t, 3> s{0, 0, 0};
                    bool ok = true;
                    for (int k = 0; k < 3; ++k) {
                        int32_t v = B.anchor[k] + d[k];
                        if ((t_.pmask >> k) & 1) {
                            int32_t q = (v >= 0) ? v / n : -((-v + n - 1) / n);
                            v -= q * n;
                            s[k] = int8_t(q);
                        } else if (v < 0 || v >= n) {
                            ok = false;
                        }
                        c[k] = v;
                    }
                    if (!ok) continue;
                    auto it = map_.find(box_hash(B.level, c[0], c[1], c[2]));
                    if (it != map_.end()) out.push_back({it->second, s});
                }
    }

    // Closed cubes of image (a, sa) and box b (unshifted) intersect.
    bool adjacent(int a, const std::array<int8_t, 3> &sa, int b) const {
        const Box &A = t_.boxes[a], &B = t_.boxes[b];
        const int D = std::max(A.level, B.level);
        for (int k = 0; k < 3; ++k) {
            int64_t loA = (int64_t(A.anchor[k]) + int64_t(sa[k]) * (int64_t(1) << A.level)) << (D - A.level);
            int64_t hiA = loA + (int64_t(1) << (D - A.level));
            int64_t loB = int64_t(B.anchor[k]) << (D - B.level);
            int64_t hiB = loB + (int64_t(1) << (D - B.level));
            if (loA > hiB || loB > hiA) return false;
        }
        return true;
    }

  private:
    Tree &t_;
    std::unordered_map<uint64_t, int> map_;
};

inline int64_t nsrc(const Box &b) { return (b.sl[1] - b.sl[0]) + (b.dl[1] - b.dl[0]); }
inline int64_t ntrg(const Box &b) { return b.trg[1] - b.trg[0]; }

}  // namespace

std::string build_tree(const double *sl, int64_t n_sl, const double *dl, int64_t n_dl,
                       const double *trg, int64_t n_trg, int leaf_cap, int pmask, Tree &t,
                       const std::unordered_map<uint64_t, int> *leaf_caps) {
    t = Tree();
    t.pmask = pmask;
    // sets given by the same array are sorted once
    Pool pool(pool_threads());
    Sorted S[3];
    S[0] = sort_points(pool, sl, n_sl);
    S[1] = (dl == sl && n_dl == n_sl) ? S[0] : sort_points(pool, dl, n_dl);
    S[2] = (trg == sl && n_trg == n_sl) ? S[0] : (trg == dl && n_trg == n_dl) ? S[1] : sort_points(pool, trg, n_trg);
    t.perm_sl = S[0].perm;
    t.perm_dl = S[1].perm;
    t.perm_trg = S[2].perm;
    t.keys_sl = std::move(S[0].key);
    t.keys_dl = std::move(S[1].key);
    t.keys_trg = std::move(S[2].key);
    const std::vector<uint64_t> *keys[3] = {&t.keys_sl, &t.keys_dl, &t.keys_trg};
    // a box's capacity: its own entry in leaf_caps, else its parent's
    auto cap_of = [&](const Box &b, int parent_cap) {
        if (leaf_caps) {
            auto it = leaf_caps->find(box_hash(b.level, b.anchor[0], b.anchor[1], b.anchor[2]));
            if (it != leaf_caps->end()) return it->second;
        }
        return parent_cap;
    };

    Box root;
    root.sl[1] = n_sl;
    root.dl[1] = n_dl;
    root.trg[1] = n_trg;
    root.cap = cap_of(root, leaf_cap);
    t.boxes.push_back(root);
    for (size_t i = 0; i < t.boxes.size(); ++i) {
        Box b = t.boxes[i];
        int64_t cnt = std::max({b.sl[1] - b.sl[0], b.dl[1] - b.dl[0], b.trg[1] - b.trg[0]});
        if (cnt <= b.cap || b.level >= kMaxLevel) continue;
        const int shift = 3 * (kKeyBits - (b.level + 1));
        int64_t bound[3][9];
        int64_t *rng[3] = {b.sl, b.dl, b.trg};
        for (int s = 0; s < 3; ++s) {
            const auto &key = *keys[s];
            for (int o = 0; o <= 8; ++o) {
                auto first = key.begin() + rng[s][0], last = key.begin() + rng[s][1];
                bound[s][o] = std::partition_point(first, last, [&](uint64_t k) {
                                  return int((k >> shift) & 7) < o;
                              }) - key.begin();
            }
        }
        for (int o = 0; o < 8; ++o) {
            Box c;
            c.level = b.level + 1;
            c.anchor[0] = 2 * b.anchor[0] + ((o >> 2) & 1);
            c.anchor[1] = 2 * b.anchor[1] + ((o >> 1) & 1);
            c.anchor[2] = 2 * b.anchor[2] + (o & 1);
            c.parent = int(i);
            c.sl[0] = bound[0][o];  c.sl[1] = bound[0][o + 1];
            c.dl[0] = bound[1][o];  c.dl[1] = bound[1][o + 1];
            c.trg[0] = bound[2][o]; c.trg[1] = bound[2][o + 1];
            if (nsrc(c) + ntrg(c) == 0) continue;
            c.cap = cap_of(c, b.cap);
            t.boxes[i].child[o] = int(t.boxes.size());
            t.boxes[i].leaf = false;
            t.boxes.push_back(c);
        }
    }
    const int nb = int(t.boxes.size());
    for (int i = 0; i < nb; ++i) {
        Box &b = t.boxes[i];
        b.nsrc_sub = nsrc(b);
        b.ntrg_sub = ntrg(b);
        if (b.leaf) t.leaves.push_back(i);
        t.depth = std::max(t.depth, b.level);
    }
    t.level_start.assign(t.depth + 2, nb);
    for (int i = nb - 1; i >= 0; --i) t.level_start[t.boxes[i].level] = i;
    for (int l = t.depth; l >= 0; --l) t.level_start[l] = std::min(t.level_start[l], t.level_start[l + 1]);

    // ------------------------------------------------------------ lists
    Lister L(t);
    std::vector<std::vector<Img>> U(nb), W(nb), X(nb), V(nb);
    std::vector<Img> col;
    // U and W by descending from the colleagues of each leaf
    for (int b : t.leaves) {
        L.colleagues(b, col);
        std::vector<Img> stack;
        for (const Img &c : col) {
            const bool self = (c.box == b && c.s[0] == 0 && c.s[1] == 0 && c.s[2] == 0);
            if (self || t.boxes[c.box].leaf) {
                U[b].push_back(c);
                continue;
            }
            stack.push_back(c);
            while (!stack.empty()) {
                Img d = stack.back();
                stack.pop_back();
                for (int o = 0; o < 8; ++o) {
                    int ch = t.boxes[d.box].child[o];
                    if (ch < 0) continue;
                    Img e{ch, d.s};
                    if (L.adjacent(ch, d.s, b)) {
                        if (t.boxes[ch].leaf) {
                            U[b].push_back(e);
                            // the finer leaf sees this coarser leaf through the
                            // reverse relation
                            U[ch].push_back({b, {int8_t(-d.s[0]), int8_t(-d.s[1]), int8_t(-d.s[2])}});
                        } else {
                            stack.push_back(e);
                        }
                    } else {
                        W[b].push_back(e);
                    }
                }
            }
        }
    }
    // X is the dual of W
    for (int b : t.leaves)
        for (const Img &e : W[b])
            X[e.box].push_back({b, {int8_t(-e.s[0]), int8_t(-e.s[1]), int8_t(-e.s[2])}});
    // V: children of the parent's colleagues that are not adjacent
    pool.each([&](int th) {
        std::vector<Img> pc;
        for (int b = 1 + th; b < nb; b += pool.size()) {
            L.colleagues(t.boxes[b].parent, pc);
            for (const Img &c : pc)
                for (int o = 0; o < 8; ++o) {
                    int ch = t.boxes[c.box].child[o];
                    if (ch < 0 || L.adjacent(ch, c.s, b)) continue;
                    V[b].push_back({ch, c.s});
                }
        }
    });

    // ------------------------------------------------------------ prune and flatten
    auto flatten = [&](std::vector<std::vector<Img>> &lists, std::vector<int> &off,
                       std::vector<Entry> &ent, bool need_src, bool need_trg) {
        off.assign(nb + 1, 0);
        ent.clear();
        // deterministic order: by box id then shift
        pool.parallel_for(nb, [&](int b) {
            std::sort(lists[b].begin(), lists[b].end(), [](const Img &p, const Img &q) {
                if (p.box != q.box) return p.box < q.box;
                return p.s < q.s;
            });
        });
        for (int b = 0; b < nb; ++b) {
            off[b] = int(ent.size());
            const Box &B = t.boxes[b];
            if (need_trg && (B.leaf ? ntrg(B) : B.ntrg_sub) == 0) continue;
            for (const Img &e : lists[b]) {
                if (need_src && t.boxes[e.box].nsrc_sub == 0) continue;
                Entry en;
                en.box = e.box;
                std::memcpy(en.shift, e.s.data(), 3);
                ent.push_back(en);
            }
        }
        off[nb] = int(ent.size());
    };
    flatten(U, t.u_off, t.u, true, true);
    flatten(W, t.w_off, t.w, true, true);
    flatten(X, t.x_off, t.x, true, true);
    flatten(V, t.v_off, t.v, true, true);
    finish_tree(t);
    return "";
}

void finish_tree(Tree &t) {
    const int nb = int(t.boxes.size());
    t.v_rel.resize(3 * t.v.size());
    for (int b = 0; b < nb; ++b) {
        const Box &B = t.boxes[b];
        for (int i = t.v_off[b]; i < t.v_off[b + 1]; ++i) {
            const Box &A = t.boxes[t.v[i].box];
            for (int k = 0; k < 3; ++k)
                t.v_rel[3 * i + k] = int8_t(A.anchor[k] + int32_t(t.v[i].shift[k]) * (1 << A.level) - B.anchor[k]);
        }
    }
    t.has_local.assign(nb, 0);
    for (int b = 0; b < nb; ++b) {
        const Box &B = t.boxes[b];
        if (B.ntrg_sub == 0) continue;
        bool loc = (t.v_off[b + 1] > t.v_off[b]) || (t.x_off[b + 1] > t.x_off[b]);
        if (B.parent >= 0 && t.has_local[B.parent]) loc = true;
        if (b == 0 && t.pmask) loc = true;
        t.has_local[b] = loc;
    }
    t.p2p_pairs = 0;
    for (int b : t.leaves) {
        int64_t s = 0;
        for (int i = t.u_off[b]; i < t.u_off[b + 1]; ++i) s += t.boxes[t.u[i].box].nsrc_sub;
        t.p2p_pairs += s * ntrg(t.boxes[b]);
    }
}

}  // namespace kafmm
