// Internal types of the MI355X kernel aggregated FMM library.
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

namespace kafmm {

// Maximum octree depth; Morton keys carry 21 bits per dimension.
constexpr int kMaxLevel = 20;
constexpr int kKeyBits = 21;

// Surface radii (in units of half the box side): the upward equivalent and
// downward check surfaces sit just outside the box, the upward check and
// downward equivalent surfaces well outside it.  1 < a_in < a_out and
// a_in + a_out <= 4 keep every M2L check point outside the source box's
// upward check surface.
constexpr double kAlphaIn = 1.05;
constexpr double kAlphaOut = 2.95;

enum Kernel { kLapPGrad = 0, kStokeslet = 1, kRPY = 2, kPVel = 3, kTraction = 4, kStokesRegVel = 5,
              kStokesRegVelOmega = 6, kLapPGradGrad = 7, kPVelGrad = 8, kPVelLaplacian = 9,
              kLapQPGradGrad = 10, kNumKernels = 11 };

struct KernelInfo {
    int k_sl, k_dl, k_trg;   // user value widths
    int ncomp;               // Laplace components on the ML tree (1 or 4)
    int rec_sl, rec_dl;      // floats per packed source record (positions + values)
    int kt_acc;              // accumulated target values (symmetric tensors compressed)
};
const KernelInfo &kernel_info(int k);

// Box of the adaptive octree (normalised coordinates: root = [0,1)^3).
struct Box {
    int level = 0;
    int32_t anchor[3] = {0, 0, 0};
    int parent = -1;
    int child[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    bool leaf = true;
    int64_t sl[2] = {0, 0}, dl[2] = {0, 0}, trg[2] = {0, 0};   // ranges in sorted arrays
    int64_t nsrc_sub = 0, ntrg_sub = 0;                        // subtree totals
    int cap = 0;                                               // split threshold of this box
};

inline uint64_t box_hash(int level, int32_t ax, int32_t ay, int32_t az) {
    return (uint64_t(level) << 60) | (uint64_t(ax) << 40) | (uint64_t(ay) << 20) | uint64_t(az);
}

// A list entry: another box (or one of its periodic images) and the image
// shift in root-box units.
struct Entry {
    int box;
    int8_t shift[3];
};

struct Tree {
    std::vector<Box> boxes;          // breadth-first, so level-sorted
    std::vector<int> leaves;         // box ids of leaves
    std::vector<int> level_start;    // boxes of level l: [level_start[l], level_start[l+1])
    std::vector<int32_t> perm_sl, perm_dl, perm_trg;  // sorted position -> user index
    std::vector<uint64_t> keys_sl, keys_dl, keys_trg; // sorted Morton keys
    int depth = 0;
    int pmask = 0;                   // periodic axes: bit k set = periodic in axis k
    // Interaction lists (CSR by box id).
    std::vector<int> u_off, w_off, x_off, v_off;
    std::vector<Entry> u, w, x;      // U, W per leaf; X per box
    std::vector<Entry> v;            // V per box (shift unused, offset below)
    std::vector<int8_t> v_rel;       // 3 per V entry: anchor offset (source - target) at the level
    std::vector<uint8_t> has_local;  // box receives a downward expansion
    int64_t p2p_pairs = 0;
};

// Build the octree and interaction lists.  Coordinates are normalised to
// [0,1) (already wrapped in the periodic axes, bits of pmask).  Returns an empty string or an
// error message.
// leaf_caps (optional): capacity of the boxes named by box_hash and of their
// descendants; other boxes use leaf_cap.
std::string build_tree(const double *sl, int64_t n_sl, const double *dl, int64_t n_dl,
                       const double *trg, int64_t n_trg, int leaf_cap, int pmask, Tree &t,
                       const std::unordered_map<uint64_t, int> *leaf_caps = nullptr);

// The same tree built on the GPU from the caller's device coordinates
// (sl, dl, trg: [n][3] FP64, normalised with origin and box_len, wrapped if
// in the periodic axes of pmask), on the HIP stream `stream`.  Leaves keys_* empty.
std::string build_tree_gpu(const double *const xyz[3], const int64_t n[3], const double origin[3], double box_len,
                           int leaf_cap, int pmask, Tree &t,
                           const std::unordered_map<uint64_t, int> *leaf_caps, void *stream);

// Checks the caller's device coordinates [n][3] on the GPU: any not finite,
// and any coordinate of an open (non-periodic) axis outside [origin, origin + box_len).
std::string check_points_gpu(const double *xyz, int64_t n, const double origin[3], double box_len, int pmask,
                             bool *nonfinite, bool *outside, void *stream);

// V-list anchor offsets, local-expansion flags and the P2P pair count of a
// tree whose boxes and lists are set.
void finish_tree(Tree &t);


// ---- learned order / capacity predictor (host side)
constexpr int kNumFeatures = 12;
constexpr int kOrderClasses[4] = {6, 8, 10, 12};
constexpr int kCapClasses[4] = {250, 500, 1000, 2000};
constexpr int kReferenceCap = 2000;

// Per-leaf features of a tree: coordinates are the normalised user-order
// arrays the tree was built from.  out: [n_leaf][kNumFeatures].
void leaf_features(const Tree &t, const double *sl, const double *dl, const double *trg, double tol,
                   std::vector<float> &out);


// Host-side FP64 operators for order p (unit box: side 1, centre 0).
struct Operators {
    int p = 0, M = 0, Mp = 0, rank = 0;
    std::vector<double> grid;        // [M][3] unit surface lattice in [-1,1]^3
    // pseudo-inverse factors: UC2UE = P1 * P2 (P1 [M][rank], P2 [rank][M]),
    // DC2DE = P2^T * P1^T (kernel symmetry), all FP64
    std::vector<double> up1, up2;
    std::vector<float> m2m;          // [8][Mp][Mp]  parent check <- child equivalent (parent side 1)
    std::vector<double> l2l_cc;      // [8][M][M]    child check <- parent check (L2L * DC2DE, scale free)
    std::vector<float> m2l;          // [343][Mp][Mp] check <- equivalent at offset (side 1); |o|<=1 unused;
                                     // empty when the translations are compressed (kc > 0)
    int kc = 0;                      // rank of the compressed V-list translations (multiple of 32), 0 = dense
    std::vector<float> cbasis;       // [Mp][kc] basis U_k (rows >= M zero)
    std::vector<float> m2l_c;        // [343][kc][kc] cores C[o] = U_k^T M2L[o] U_k
    std::vector<double> t_m2l;       // [M][M] periodic far-image operator (side 1), empty if unused
    double svd_tol = 0, m2l_tol = 0;
};

// m2l_tol > 0 compresses the V-list translations (singular values of the
// stacked operators below m2l_tol times the largest are dropped); 0 keeps
// them dense.
std::string build_operators(int p, double svd_tol, bool periodic, Operators &ops, double m2l_tol = 0.0);

// Far images of the periodic Stokeslet at the root (unit box centred at the
// origin): Q [3M][3M] maps the root's flow at its M upward check points
// X [M][3] (the Stokeslet sum of the sources inside the root) to Stokeslet
// forces on the M downward equivalent points Z [M][3] whose flow inside the
// root is that of the far images (Hasimoto's Ewald sums, zero net force):
// triply periodic, every n with max|n_k| >= 2; doubly periodic (x, y), the
// in-plane n = (n_x, n_y, 0) with max(|n_x|, |n_y|) >= 2.
std::string build_periodic_stokes(int p, double svd_tol, bool doubly, std::vector<double> &Q,
                                  std::vector<double> &X, std::vector<double> &Z);

// On-disk operator cache (opcache.cpp, best effort).  cached_operators and
// cached_periodic_stokes load the set from a file of directory dir whose
// parameters and source hash match (*loaded = true), else build it and store
// it there; dir "" builds only.  They return the builders' error strings.
std::string cached_operators(const std::string &dir, int p, double svd_tol, bool periodic, double m2l_tol,
                             Operators &ops, bool *loaded);
std::string cached_periodic_stokes(const std::string &dir, int p, double svd_tol, bool doubly, std::vector<double> &Q,
                                   std::vector<double> &X, std::vector<double> &Z, bool *loaded);
// The cache directory by default: $STKFMM_OPERATOR_CACHE ("" disables),
// else $XDG_CACHE_HOME/stkfmm_operators, else $HOME/.cache/stkfmm_operators.
std::string default_operator_cache_dir();
// 64-bit hashes of a set as the cache file stores it (equal for a built and a loaded set).
uint64_t operators_digest(const Operators &ops, bool periodic);
uint64_t stokes_far_digest(int p, double svd_tol, bool doubly, const std::vector<double> &Q,
                           const std::vector<double> &X, const std::vector<double> &Z);

// Index of a relative offset o in [-3,3]^3.
inline int offset_index(int ox, int oy, int oz) { return ((oz + 3) * 7 + (oy + 3)) * 7 + (ox + 3); }

}  // namespace kafmm
