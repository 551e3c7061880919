// C ABI and evaluation engine of the MI355X kernel aggregated FMM.
//
// set_points: host octree + lists (t_tree), operators for p (cached), plan
//             arrays uploaded in one arena, points packed into leaf order.
// run:        the evaluation pass (t_run) on two streams:
//   stream A  pack values -> S2M -> [M2M -> UC2UE] per level (upward) ->
//             S2L (X) -> M2L (offset-grouped MFMA GEMM + reduce) ->
//             [periodic] -> [L2L -> DC2DE] per level (downward) -> L2T + M2T
//   stream B  P2P over U lists (independent of the far field)
//   join      combine near + far, un-permute into the caller's order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <array>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/stkfmm.h"
#include "internal.hpp"
#include "kernels.hpp"

namespace kafmm {

static const KernelInfo kInfo[kNumKernels] = {
    // k_sl k_dl k_trg ncomp rec_sl rec_dl kt_acc
    {1, 3, 4, 1, 8, 12, 4},    // LapPGrad
    {3, 0, 3, 4, 12, 0, 3},    // Stokeslet
    {4, 0, 6, 4, 12, 0, 6},    // RPY
    {4, 9, 4, 4, 12, 12, 4},   // PVel
    {4, 9, 9, 4, 12, 12, 6},   // Traction
    {4, 0, 3, 4, 12, 0, 3},    // StokesRegVel
    {7, 0, 6, 4, 16, 0, 6},    // StokesRegVelOmega
    {1, 3, 10, 1, 8, 12, 10},  // LapPGradGrad
    {4, 9, 16, 4, 12, 12, 16}, // PVelGrad
    {4, 9, 7, 4, 12, 12, 7},   // PVelLaplacian
    {9, 0, 10, 1, 12, 0, 10},  // LapQPGradGrad
};
const KernelInfo &kernel_info(int k) { return kInfo[k]; }

namespace {

constexpr double kPi = 3.14159265358979323846;

struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n) {
        if (n <= bytes) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, std::max<size_t>(n, 256));
        if (e == hipSuccess) bytes = std::max<size_t>(n, 256);
        else p = nullptr;
        return e;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Host staging area for plan arrays: one device allocation, one copy.  The
// context keeps it between plans (clear() keeps the memory), so a re-plan
// of a similar problem writes into pages it already holds.
struct Arena {
    std::vector<char> host;
    size_t used = 0;
    void clear() { used = 0; }
    // room for n values of T (uninitialised); ptr<T>(off) is valid until
    // the next reserve or add
    template <class T> size_t reserve(size_t n) {
        const size_t off = (used + 255) / 256 * 256;
        const size_t bytes = std::max<size_t>(n * sizeof(T), 1);
        if (off + bytes > host.size()) host.resize(std::max(off + bytes, host.size() + host.size() / 2));
        used = off + bytes;
        return off;
    }
    template <class T> T *ptr(size_t off) { return reinterpret_cast<T *>(host.data() + off); }
    template <class T> size_t add(const std::vector<T> &v) {
        const size_t off = reserve<T>(v.size());
        if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

struct DeviceOps {
    int p = 0, M = 0, Mp = 0, rank = 0;
    int kc = 0;                 // compressed V-list rank (0: dense m2l)
    bool periodic = false;
    DevMem grid, m2m, m2l, uc2ue, dc2de, tm2l;   // pseudo-inverses [M][M] FP64
    DevMem l2l_cc;              // [8][M][M] FP64 child check <- parent check
    DevMem uc2ue_m1, uc2ue_m2;  // UC2UE without the monopole / monopole and dipole
    DevMem basis_t, m2l_c;      // U_k^T [kc][Mp], cores [343][kc][kc]
};

// Far images of the triply periodic Stokeslet: Q [3M][3M], the upward check
// points X and the downward equivalent points Z [M][3] of the root, at a
// fixed order (p = 10, whatever the tree's order) so that they stay well
// below the tree's error.
constexpr int kStokesFarOrder = 10;
struct StokesFarOps {
    int M = 0;
    DevMem Q, X, Z;
};

// A batch of translations that share the grouped GEMM and one reduce launch.
struct Batch {
    int ntiles = 0, ntasks = 0;
    size_t tiles = 0, bcol = 0, ycol = 0, rdst = 0, roff = 0, rpair = 0, rscale = 0, rdelta = 0;
    int npairs = 0;
    int accumulate = 0;
};

// Downward check-to-check translations of one level, grouped by octant.
struct L2LLevel {
    int nblocks = 0;
    size_t blocks = 0, pairs = 0, delta = 0;
};

struct PinvLevel {
    int ncol = 0;
    size_t bidx = 0, cidx = 0, cscale = 0;
};

// Surface-tile tasks of one phase (S2M or S2L): SL tasks then DL tasks, and
// the per-destination reduction of their partial check potentials.
struct S2CPhase {
    int n_sl = 0, n_dl = 0, n_dst = 0;
    size_t tasks = 0, rdst = 0, roff = 0, rtask = 0;
};

struct Pair {
    int src, dst, op;
    float delta[3];
    double scale;
};

}  // namespace
}  // namespace kafmm

using namespace kafmm;

// No-slip wall plan: the free-space summations of the image system (S, SD,
// SDZ and, for RPY, Q), each its own context on the cube of side 2 box_len
// below which the images lie, and the buffers of their sources and results.
struct WallPlan {
    stkfmm_ctx *sub[4] = {nullptr, nullptr, nullptr, nullptr};
    int nsub = 0;
    int rpy = 0;
    int64_t n_src = 0, n_trg = 0;
    DevMem src, trg, y2, yi, vs, sd_dl, sdz_sl, sdz_dl, q, out[4];
    ~WallPlan() {
        for (stkfmm_ctx *c : sub) stkfmm_destroy(c);
    }
};

struct stkfmm_ctx {
    int device = 0;
    double origin[3] = {0, 0, 0};
    double box_len = 1.0;
    std::string err;
    double svd_tol = 1e-7;
    std::string op_cache = default_operator_cache_dir();   // operator cache directory ("" = none)
    double m2l_tol = 5e-8;      // compression of the V-list translations (0: dense)
    bool m2l_tol_set = false;   // set by the caller (else learned plans use tol / 50)
    bool rel_exact = false;     // P2P forms r from hi/lo coordinates (close pairs across leaves)
    int precision = 0;          // 0 fp32, 1 split_bf16
    hipStream_t side = nullptr; // P2P stream
    hipEvent_t ev[24] = {};
    // plan
    bool planned = false;
    int kernel = 0, bc = 0, p = 0, leaf_cap = 0;
    int64_t n_sl = 0, n_dl = 0, n_trg = 0;
    Tree tree;
    DeviceOps *ops = nullptr;
    Arena staging;              // host image of `arena`, reused between plans
    StokesFarOps *stk = nullptr; // periodic Stokeslet: far-image operator
    DevMem stk_F, stk_part;     // root check flow and far-image forces, partial sums
    DevMem arena, sl_rec, dl_rec, trg_rec, up_dens, dn_dens, up_chk, dn_chk, Ybuf, near_part, far_part,
        s2c_part, partial, direct_work, sl_stage, dl_stage, up_cmp;
    size_t a_perm_sl = 0, a_perm_dl = 0, a_perm_trg = 0, a_geom = 0, a_box_sl = 0, a_box_dl = 0, a_chunks = 0,
           a_chunk_tasks = 0, a_p2p_tasks = 0, a_p2p_ent = 0, a_l2t_tasks = 0, a_l2t_ent = 0, a_leaves_sl = 0,
           a_leaves_dl = 0, a_cmp_tiles = 0, a_cmp_cols = 0;
    int n_leaves_sl = 0, n_leaves_dl = 0, n_cmp_tiles = 0;
    int nchunks = 0, n_p2p_tasks = 0, n_l2t_tasks = 0, nbox = 0;
    S2CPhase s2m, s2l;
    int64_t w_direct = 0, x_direct = 0, direct_pairs = 0, p2p_lane_pairs = 0;
    // work of the plan by box: P2P lane pairs, P2P wave entries, M2L flops,
    // surface evaluations (S2M, S2L, L2T/M2T), 1 per box
    std::vector<std::array<double, 5>> box_work;
    int overlap = 1;
    int tree_gpu = 1;           // build the octree and lists on the GPU (0: host)
    // sources' vanishing moments: 0 none, 1 charge (dipoles only), 2 charge
    // and dipole (quadrupoles only); picks the moment-free UC2UE
    int moments = 0;
    std::unique_ptr<WallPlan> wall;   // no-slip wall plans (bc WALL)
    // learned order / capacity mode
    DevMem predictor, mlp_in, mlp_out, mlp_ws, coords[3], vbuf[4];
    bool has_predictor = false, learned = false, validated = false, fell_back = false;
    float order_table[16] = {};
    double tol = 1e-5, sampled_err = -1.0;
    int p_hist[4] = {0, 0, 0, 0}, cap_hist[4] = {0, 0, 0, 0};
    std::vector<double> hcoords[3];      // normalised user-order coordinates of the last plan
    bool hcoords_valid = false;          // (else copied from coords[] when asked for)
    double w_direct_frac = 0.73, x_direct_frac = 0.5;
    int64_t p2p_task_sources = 1024;  // measured on the 1M learned plan: 8.46 ms per pass against 8.60 at 2048
    Batch m2l;
    std::vector<Batch> m2m;                 // by parent level
    std::vector<L2LLevel> l2l;              // by child level
    std::vector<PinvLevel> upinv, dnpinv;   // by level
    int lmin_up = 0, lmin_dn = 0;
    size_t ybuf_floats = 0;
    double t_tree_ms = 0, t_run_ms = 0, stage_ms[16] = {};
};

namespace {

stkfmm_status fail(stkfmm_ctx *c, stkfmm_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return fail(ctx, e_ == hipErrorOutOfMemory ? STKFMM_E_NOMEM : STKFMM_E_DEVICE,              \
                        std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_));           \
    } while (0)

bool kernel_ok(int k) { return k >= 0 && k < kNumKernels; }

// source kinds of the packing kernel; stage_kind: of the surface tiles
// PVel and its derivative outputs: single layer (f, q), double layer D
bool pvel_family(int k) { return k == kPVel || k == kPVelGrad || k == kPVelLaplacian || k == kTraction; }
// Stokes kernels with a triply periodic plan (far images through the root)
bool periodic_stokes(int k) {
    return k == kStokeslet || k == kRPY || k == kStokesRegVel || k == kStokesRegVelOmega || pvel_family(k);
}

// Stokes kernels with a doubly periodic plan: point forces, with or without
// the RPY correction
bool doubly_periodic_stokes(int k) { return k == kStokeslet || k == kRPY; }

// periodic axes of a boundary condition: bit k set = periodic in axis k
int bc_axes(int bc) { return bc == STKFMM_BC_PXYZ ? 7 : bc == STKFMM_BC_PXY ? 3 : 0; }

int sl_kind(int k) {
    switch (k) {
        case kStokeslet: return 0;
        case kRPY: return 1;
        case kLapPGrad:
        case kLapPGradGrad: return 2;
        case kStokesRegVel: return 6;
        case kStokesRegVelOmega: return 7;
        case kLapQPGradGrad: return 8;
        default: return 4;
    }
}
// The regularized Stokeslet's far field is the RPY one with b^2 = 3 eps^2 / 2
// (to O(eps^4 / r^5)): its packed records carry that b^2 where RPY's do.
int stage_kind(int k) { return k == kStokesRegVel ? 1 : sl_kind(k); }   // kinds 7, 8 pack and stage alike
int dl_kind(int k) { return k == kLapPGrad || k == kLapPGradGrad ? 3 : 5; }

// Device operators are shared by every context of the process (the summations
// of a wall plan, repeated contexts): one set per (device, p, periodic,
// svd_tol, m2l_tol), built on first use and kept until the process ends (the
// map is never destroyed, so no device memory is freed after the runtime has
// shut down).
using OpsKey = std::tuple<int, int, bool, double, double>;
std::mutex g_ops_mutex;
std::map<OpsKey, std::unique_ptr<DeviceOps>> *g_ops = new std::map<OpsKey, std::unique_ptr<DeviceOps>>();

stkfmm_status get_ops(stkfmm_ctx *c, int p, bool periodic, double m2l_tol, DeviceOps **out) {
    std::lock_guard<std::mutex> lock(g_ops_mutex);
    const OpsKey key(c->device, p, periodic, c->svd_tol, m2l_tol);
    auto it = g_ops->find(key);
    if (it != g_ops->end()) {
        *out = it->second.get();
        return STKFMM_OK;
    }
    Operators h;
    std::string e = cached_operators(c->op_cache, p, c->svd_tol, periodic, m2l_tol, h, nullptr);
    if (!e.empty()) return fail(c, STKFMM_E_ARG, e);
    auto d = std::make_unique<DeviceOps>();
    d->p = p;
    d->M = h.M;
    d->Mp = h.Mp;
    d->rank = h.rank;
    d->kc = h.kc;
    d->periodic = periodic;
    std::vector<float> g(h.grid.begin(), h.grid.end());
    auto up = [&](DevMem &m, const void *src, size_t bytes) -> hipError_t {
        hipError_t er = m.ensure(bytes);
        if (er != hipSuccess) return er;
        return hipMemcpy(m.p, src, bytes, hipMemcpyHostToDevice);
    };
    HIP_TRY(c, up(d->grid, g.data(), g.size() * sizeof(float)));
    HIP_TRY(c, up(d->m2m, h.m2m.data(), h.m2m.size() * sizeof(float)));
    HIP_TRY(c, up(d->l2l_cc, h.l2l_cc.data(), h.l2l_cc.size() * sizeof(double)));
    if (h.kc > 0) {
        std::vector<float> bt(size_t(h.kc) * h.Mp);     // U_k^T
        for (int i = 0; i < h.Mp; ++i)
            for (int k = 0; k < h.kc; ++k) bt[size_t(k) * h.Mp + i] = h.cbasis[size_t(i) * h.kc + k];
        HIP_TRY(c, up(d->basis_t, bt.data(), bt.size() * sizeof(float)));
        HIP_TRY(c, up(d->m2l_c, h.m2l_c.data(), h.m2l_c.size() * sizeof(float)));
    } else {
        HIP_TRY(c, up(d->m2l, h.m2l.data(), h.m2l.size() * sizeof(float)));
    }
    // UC2UE = P1 P2 and DC2DE = UC2UE^T, formed once in FP64: one GEMM per
    // level applies them
    const int M = h.M, r = h.rank;
    std::vector<double> uc(size_t(M) * M, 0.0), dc(size_t(M) * M);
    for (int i = 0; i < M; ++i)
        for (int k = 0; k < r; ++k) {
            const double a = h.up1[size_t(i) * r + k];
            const double *b = &h.up2[size_t(k) * M];
            double *o = &uc[size_t(i) * M];
            for (int j = 0; j < M; ++j) o[j] += a * b[j];
        }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) dc[size_t(j) * M + i] = uc[size_t(i) * M + j];
    HIP_TRY(c, up(d->uc2ue, uc.data(), uc.size() * sizeof(double)));
    HIP_TRY(c, up(d->dc2de, dc.data(), dc.size() * sizeof(double)));
    // Moment-free variants for boxes whose sources carry no charge (dipoles
    // only) or no charge and no dipole moment (quadrupoles only): the fitted
    // density's monopole sum_i s_i (and dipole sum_i s_i y_i, y relative to
    // the box centre) are projected out, (I - W W^T) UC2UE with W the
    // orthonormal basis of {1} or {1, y_x, y_y, y_z} on the equivalent
    // surface.  The truncated fit and FP32 rounding leave small moments
    // there whose fields decay more slowly than the true field's and would
    // dominate it far away.  On the symmetric lattice the four vectors are
    // orthogonal, so W is them normalised.
    {
        std::vector<double> w[4];
        for (int k = 0; k < 4; ++k) {
            w[k].resize(M);
            double nn = 0.0;
            for (int i = 0; i < M; ++i) {
                w[k][i] = k == 0 ? 1.0 : h.grid[3 * size_t(i) + (k - 1)];
                nn += w[k][i] * w[k][i];
            }
            for (double &v : w[k]) v /= std::sqrt(nn);
        }
        std::vector<double> pm(uc);
        for (int nk = 1; nk <= 4; nk += 3) {
            for (int k = (nk == 1 ? 0 : 1); k < nk; ++k)
                for (int j = 0; j < M; ++j) {
                    double t = 0.0;
                    for (int i = 0; i < M; ++i) t += w[k][i] * pm[size_t(i) * M + j];
                    for (int i = 0; i < M; ++i) pm[size_t(i) * M + j] -= w[k][i] * t;
                }
            HIP_TRY(c, up(nk == 1 ? d->uc2ue_m1 : d->uc2ue_m2, pm.data(), pm.size() * sizeof(double)));
        }
    }
    if (periodic) HIP_TRY(c, up(d->tm2l, h.t_m2l.data(), h.t_m2l.size() * sizeof(double)));
    *out = d.get();
    (*g_ops)[key] = std::move(d);
    return STKFMM_OK;
}

// The periodic Stokeslet's far-image operator, one per (device, periodic
// axes, svd_tol), built on first use and kept like the operator sets.
std::map<std::tuple<int, int, double>, std::unique_ptr<StokesFarOps>> *g_stk =
    new std::map<std::tuple<int, int, double>, std::unique_ptr<StokesFarOps>>();

stkfmm_status get_periodic_stokes(stkfmm_ctx *c, int pmask, StokesFarOps **out) {
    std::lock_guard<std::mutex> lock(g_ops_mutex);
    const auto key = std::make_tuple(c->device, pmask, c->svd_tol);
    auto it = g_stk->find(key);
    if (it != g_stk->end()) {
        *out = it->second.get();
        return STKFMM_OK;
    }
    std::vector<double> Q, X, Z;
    std::string e = cached_periodic_stokes(c->op_cache, kStokesFarOrder, c->svd_tol, pmask == 3, Q, X, Z, nullptr);
    if (!e.empty()) return fail(c, STKFMM_E_ARG, e);
    auto d = std::make_unique<StokesFarOps>();
    d->M = int(X.size() / 3);
    HIP_TRY(c, d->Q.ensure(Q.size() * sizeof(double)));
    HIP_TRY(c, hipMemcpy(d->Q.p, Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, d->X.ensure(X.size() * sizeof(double)));
    HIP_TRY(c, hipMemcpy(d->X.p, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, d->Z.ensure(Z.size() * sizeof(double)));
    HIP_TRY(c, hipMemcpy(d->Z.p, Z.data(), Z.size() * sizeof(double), hipMemcpyHostToDevice));
    *out = d.get();
    (*g_stk)[key] = std::move(d);
    return STKFMM_OK;
}

// Group translation pairs by operator for the GEMM and by destination for the reduce.
Batch make_batch(Arena &ar, std::vector<Pair> &pairs, int nc, int accumulate, size_t &ybuf_floats, int Mp) {
    Batch b;
    b.accumulate = accumulate;
    const size_t np = pairs.size();
    // stable counting sorts: by operator for the GEMM tiles, by destination for the reduce
    auto stable_order = [&](auto key, int nkey) {
        std::vector<int> start(nkey + 1, 0), order(np);
        for (const Pair &pr : pairs) ++start[key(pr) + 1];
        for (int k = 0; k < nkey; ++k) start[k + 1] += start[k];
        for (size_t i = 0; i < np; ++i) order[start[key(pairs[i])]++] = int(i);
        return order;
    };
    {
        int nop = 0;
        for (const Pair &pr : pairs) nop = std::max(nop, pr.op + 1);
        const std::vector<int> byop = stable_order([](const Pair &pr) { return pr.op; }, nop);
        std::vector<Pair> sorted(np);
        for (size_t i = 0; i < np; ++i) sorted[i] = pairs[byop[i]];
        pairs.swap(sorted);
    }
    b.npairs = int(np);
    std::vector<int> bcol(np * nc), ycol(np * nc);
    std::vector<int4> tiles;
    for (size_t k = 0; k < np; ++k)
        for (int c = 0; c < nc; ++c) {
            bcol[k * nc + c] = pairs[k].src * nc + c;
            ycol[k * nc + c] = int(k) * nc + c;
        }
    for (size_t i = 0; i < np;) {
        size_t j = i;
        while (j < np && pairs[j].op == pairs[i].op) ++j;
        const int c0 = int(i) * nc, ncols = int(j - i) * nc;
        for (int t = 0; t < ncols; t += 128) tiles.push_back(make_int4(pairs[i].op, c0 + t, std::min(128, ncols - t), 0));
        i = j;
    }
    b.ntiles = int(tiles.size());
    // reduce by destination, pairs in index order
    int ndst = 0;
    for (const Pair &pr : pairs) ndst = std::max(ndst, pr.dst + 1);
    const std::vector<int> order = stable_order([](const Pair &pr) { return pr.dst; }, ndst);
    std::vector<int> rdst, roff, rpair(np);
    std::vector<double> rscale(np);
    std::vector<float> rdelta(3 * np);
    for (size_t i = 0; i < np;) {
        size_t j = i;
        while (j < np && pairs[order[j]].dst == pairs[order[i]].dst) ++j;
        rdst.push_back(pairs[order[i]].dst);
        roff.push_back(int(i));
        for (size_t k = i; k < j; ++k) {
            const Pair &pr = pairs[order[k]];
            rpair[k] = order[k];
            rscale[k] = pr.scale;
            for (int q = 0; q < 3; ++q) rdelta[3 * k + q] = pr.delta[q];
        }
        i = j;
    }
    roff.push_back(int(np));
    b.ntasks = int(rdst.size());
    b.tiles = ar.add(tiles);
    b.bcol = ar.add(bcol);
    b.ycol = ar.add(ycol);
    b.rdst = ar.add(rdst);
    b.roff = ar.add(roff);
    b.rpair = ar.add(rpair);
    b.rscale = ar.add(rscale);
    b.rdelta = ar.add(rdelta);
    ybuf_floats = std::max(ybuf_floats, np * nc * Mp);
    return b;
}

// The V-list batch (M2L), straight from the lists: pairs grouped by
// relative offset (stable in box order) for the GEMM tiles, and per
// destination box its pairs in that order for the reduce; the same arrays
// as make_batch gives for the pairs listed box by box.
Batch make_v_batch(Arena &ar, const Tree &t, const std::vector<double4> &geom, int nc, size_t &ybuf_floats, int Mp) {
    Batch b;
    b.accumulate = 1;
    const int nb = int(t.boxes.size());
    const int64_t ne = int64_t(t.v.size());
    std::vector<int16_t> op(ne, -1);
    std::vector<int> start(344, 0);
    for (int d = 0; d < nb; ++d) {
        if (!t.has_local[d]) continue;
        for (int i = t.v_off[d]; i < t.v_off[d + 1]; ++i) {
            const int8_t *o = &t.v_rel[3 * size_t(i)];
            op[i] = int16_t(offset_index(o[0], o[1], o[2]));
            ++start[op[i] + 1];
        }
    }
    for (int k = 0; k < 343; ++k) start[k + 1] += start[k];
    const int np = start[343];
    b.npairs = np;
    std::vector<int4> tiles;
    for (int k = 0; k < 343; ++k)
        for (int c0 = start[k] * nc, c1 = start[k + 1] * nc, c = c0; c < c1; c += 128)
            tiles.push_back(make_int4(k, c, std::min(128, c1 - c), 0));
    b.ntiles = int(tiles.size());
    int ndst = 0;
    for (int d = 0; d < nb; ++d) ndst += t.has_local[d] && t.v_off[d + 1] > t.v_off[d];
    // the large arrays are written in place in the staging area
    b.tiles = ar.add(tiles);
    b.bcol = ar.reserve<int>(size_t(np) * nc);
    b.ycol = ar.reserve<int>(size_t(np) * nc);
    b.rdst = ar.reserve<int>(ndst);
    b.roff = ar.reserve<int>(size_t(ndst) + 1);
    b.rpair = ar.reserve<int>(np);
    b.rscale = ar.reserve<double>(np);
    b.rdelta = ar.reserve<float>(3 * size_t(np));
    int *bcol = ar.ptr<int>(b.bcol), *ycol = ar.ptr<int>(b.ycol), *rdst = ar.ptr<int>(b.rdst);
    int *roff = ar.ptr<int>(b.roff), *rpair = ar.ptr<int>(b.rpair);
    double *rscale = ar.ptr<double>(b.rscale);
    float *rdelta = ar.ptr<float>(b.rdelta);
    // a destination's pairs have distinct offsets, and positions grow with
    // the offset, so visiting its entries by offset gives them in position
    // order (the reduce order)
    std::vector<int> next(start.begin(), start.end() - 1), slot(343, -1);
    int q = 0, r = 0;
    for (int d = 0; d < nb; ++d) {
        if (!t.has_local[d] || t.v_off[d + 1] == t.v_off[d]) continue;
        rdst[q] = d;
        roff[q] = r;
        ++q;
        for (int i = t.v_off[d]; i < t.v_off[d + 1]; ++i) slot[op[i]] = i;
        const double hb = geom[d].w;
        for (int o3 = 0; o3 < 343; ++o3) {
            const int i = slot[o3];
            if (i < 0) continue;
            slot[o3] = -1;
            const int k = next[o3]++;
            for (int c = 0; c < nc; ++c) {
                bcol[size_t(k) * nc + c] = t.v[i].box * nc + c;
                ycol[size_t(k) * nc + c] = k * nc + c;
            }
            const int8_t *o = &t.v_rel[3 * size_t(i)];
            rpair[r] = k;
            rscale[r] = 1.0 / hb;
            // Psi_B = Psi_A - (c_B - c_A).Phi,  c_A - c_B = o h
            for (int k3 = 0; k3 < 3; ++k3) rdelta[3 * size_t(r) + k3] = float(-o[k3] * hb);
            ++r;
        }
    }
    roff[q] = r;
    b.ntasks = ndst;
    ybuf_floats = std::max(ybuf_floats, size_t(np) * nc * Mp);
    return b;
}

template <class T> T *at(stkfmm_ctx *c, size_t off) { return reinterpret_cast<T *>(c->arena.as<char>() + off); }

// Translations of a batch: the grouped GEMM (dense M x M operators on
// densities, or, compressed, kc x kc cores on basis coefficients X) and the
// reduce into the destination check values.
stkfmm_status run_batch(stkfmm_ctx *c, const Batch &b, const float *ops, const float *X, double *chk,
                        hipStream_t s, bool split_bf16 = false, bool compressed = false,
                        hipEvent_t gemm_begin = nullptr, hipEvent_t gemm_end = nullptr) {
    if (b.npairs == 0) return STKFMM_OK;
    const DeviceOps &o = *c->ops;
    const int nc = kernel_info(c->kernel).ncomp;
    const int side = compressed ? o.kc : o.Mp;
    GemmArgs g;
    g.tiles = at<int4>(c, b.tiles);
    g.ops = ops;
    g.opsz = int64_t(side) * side;
    g.X = X;
    g.Y = c->Ybuf.as<float>();
    g.bcol = at<int>(c, b.bcol);
    g.ycol = at<int>(c, b.ycol);
    g.R = g.K = g.xs = g.ys = side;
    g.Mr = compressed ? o.kc : o.M;
    g.Mk = compressed ? o.kc : std::min(o.Mp, (o.M + 15) / 16 * 16);
    if (gemm_begin) HIP_TRY(c, hipEventRecord(gemm_begin, s));
    if (split_bf16) HIP_TRY(c, launch_gemm_bf16x3(b.ntiles, g, s));
    else HIP_TRY(c, launch_gemm_f32(b.ntiles, g, s));
    if (gemm_end) HIP_TRY(c, hipEventRecord(gemm_end, s));
    ReduceArgs r;
    r.dst = at<int>(c, b.rdst);
    r.off = at<int>(c, b.roff);
    r.pair = at<int>(c, b.rpair);
    r.scale = at<double>(c, b.rscale);
    r.delta = at<float>(c, b.rdelta);
    r.Y = c->Ybuf.as<float>();
    r.ys = side;
    r.chk = chk;
    r.M = o.M;
    r.Mp = o.Mp;
    r.ncomp = nc;
    r.accumulate = b.accumulate;
    r.kc = compressed ? o.kc : 0;
    r.basis_t = compressed ? o.basis_t.as<float>() : nullptr;
    HIP_TRY(c, launch_reduce(b.ntasks, r, s));
    return STKFMM_OK;
}

// Basis coefficients U_k^T x of every box's upward densities (one operator,
// all columns).
stkfmm_status run_compress(stkfmm_ctx *c, const float *dens, float *coef, hipStream_t s) {
    const DeviceOps &o = *c->ops;
    if (c->n_cmp_tiles == 0) return STKFMM_OK;
    GemmArgs g;
    g.tiles = at<int4>(c, c->a_cmp_tiles);
    g.ops = o.basis_t.as<float>();
    g.opsz = int64_t(o.kc) * o.Mp;
    g.X = dens;
    g.Y = coef;
    g.bcol = at<int>(c, c->a_cmp_cols);
    g.ycol = at<int>(c, c->a_cmp_cols);
    g.R = o.kc;
    g.K = o.Mp;
    g.xs = o.Mp;
    g.ys = o.kc;
    g.Mr = o.kc;
    g.Mk = std::min(o.Mp, (o.M + 15) / 16 * 16);
    HIP_TRY(c, launch_gemm_f32(c->n_cmp_tiles, g, s));
    return STKFMM_OK;
}

// dens(cols) = scale * F1 (F2 chk(cols)) in FP64 (the check-to-equivalent pseudo-inverse)
// dens(cols) = scale * P chk(cols) in FP64, P the check-to-equivalent
// pseudo-inverse (M x M), written as FP32 densities
stkfmm_status run_pinv(stkfmm_ctx *c, const PinvLevel &pl, const double *P, const double *chk, float *dens,
                       hipStream_t s) {
    if (pl.ncol == 0) return STKFMM_OK;
    const DeviceOps &o = *c->ops;
    Gemm64Args b;
    b.A = P; b.R = o.M; b.K = o.M; b.lda = o.M;
    b.B = chk; b.bidx = at<int>(c, pl.bidx); b.ldb = o.M;
    b.cidx = at<int>(c, pl.cidx); b.cscale = at<double>(c, pl.cscale); b.ldc = o.Mp;
    b.ncol = pl.ncol;
    HIP_TRY(c, launch_gemm_f64_to_f32(b, dens, s));
    return STKFMM_OK;
}

stkfmm_status validate_points(stkfmm_ctx *c, const std::vector<double> &h, int64_t n, int pmask,
                              const char *what) {
    for (int64_t i = 0; i < 3 * n; ++i) {
        if (!std::isfinite(h[i])) return fail(c, STKFMM_E_ARG, std::string(what) + ": non-finite coordinate");
        if (!((pmask >> (i % 3)) & 1)) {
            double u = (h[i] - c->origin[i % 3]) / c->box_len;
            if (!(u >= 0.0 && u < 1.0))
                return fail(c, STKFMM_E_DOMAIN, std::string(what) + ": point outside [origin, origin+box_len)");
        }
    }
    return STKFMM_OK;
}

// Host copies of point sets (device [n][3]) normalised to the unit box,
// wrapped in the periodic axes (bits of pmask); optionally validated first.
stkfmm_status copy_coords(stkfmm_ctx *c, const double *const src[3], const int64_t cnt[3], int pmask,
                          bool validate, std::vector<double> h[3], hipStream_t s) {
    for (int k = 0; k < 3; ++k) {
        h[k].resize(3 * cnt[k]);
        if (cnt[k] > 0)
            HIP_TRY(c, hipMemcpyAsync(h[k].data(), src[k], 3 * cnt[k] * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    const char *names[3] = {"sl_xyz", "dl_xyz", "trg_xyz"};
    for (int k = 0; k < 3; ++k) {
        if (validate) {
            stkfmm_status st = validate_points(c, h[k], cnt[k], pmask, names[k]);
            if (st != STKFMM_OK) return st;
        }
        for (int64_t i = 0; i < 3 * cnt[k]; ++i) {
            double u = (h[k][i] - c->origin[i % 3]) / c->box_len;
            if ((pmask >> (i % 3)) & 1) {
                u -= std::floor(u);
                if (u >= 1.0) u = 0.0;
            }
            h[k][i] = u;
        }
    }
    return STKFMM_OK;
}

// ---------------------------------------------------------------- no-slip wall
// Plan of the wall boundary: validate the points in the caller's box, mirror
// the sources, plan each summation of the image system on its own context.
stkfmm_status wall_set_points(stkfmm_ctx *c, int kernel, int64_t n_src, const double *src, int64_t n_trg,
                              const double *trg, int p, int leaf_cap, void *stream) {
    if (kernel != kStokeslet && kernel != kRPY)
        return fail(c, STKFMM_E_UNSUPPORTED, "the wall boundary is implemented for STOKESLET and RPY");
    if (p == 0 || leaf_cap == 0) return fail(c, STKFMM_E_UNSUPPORTED, "learned mode is open-boundary only");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(c, hipSetDevice(c->device));
    auto t0 = std::chrono::steady_clock::now();
    {
        std::vector<double> h;
        const double *pts[2] = {src, trg};
        const int64_t cnt[2] = {n_src, n_trg};
        const char *names[2] = {"sl_xyz", "trg_xyz"};
        for (int k = 0; k < 2; ++k) {
            h.resize(3 * cnt[k]);
            if (cnt[k] > 0)
                HIP_TRY(c, hipMemcpyAsync(h.data(), pts[k], 3 * cnt[k] * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            stkfmm_status st = validate_points(c, h, cnt[k], false, names[k]);
            if (st != STKFMM_OK) return st;
        }
    }
    if (!c->wall) c->wall = std::make_unique<WallPlan>();
    WallPlan &w = *c->wall;
    w.rpy = kernel == kRPY;
    w.nsub = w.rpy ? 4 : 3;
    w.n_src = n_src;
    w.n_trg = n_trg;
    // the summations run on the cube of side 2L whose lower half holds the images
    const double org[3] = {c->origin[0], c->origin[1], c->origin[2] - c->box_len};
    for (int k = 0; k < w.nsub; ++k) {
        if (w.sub[k]) continue;
        stkfmm_status st = stkfmm_setup(&w.sub[k], org, 2.0 * c->box_len, c->device, 0);
        if (st != STKFMM_OK) return fail(c, st, "wall summation context");
        stkfmm_ctx *sc = w.sub[k];
        sc->svd_tol = c->svd_tol;
        sc->op_cache = c->op_cache;
        sc->m2l_tol = c->m2l_tol;
        sc->precision = c->precision;
        sc->overlap = c->overlap;
        sc->p2p_task_sources = c->p2p_task_sources;
        sc->w_direct_frac = c->w_direct_frac;
        sc->x_direct_frac = c->x_direct_frac;
    }
    const int64_t n = n_src, ns = std::max<int64_t>(n, 1), nt = std::max<int64_t>(n_trg, 1);
    HIP_TRY(c, w.src.ensure(size_t(ns) * 3 * sizeof(double)));
    HIP_TRY(c, w.trg.ensure(size_t(nt) * 3 * sizeof(double)));
    HIP_TRY(c, w.y2.ensure(size_t(ns) * 6 * sizeof(double)));
    HIP_TRY(c, w.yi.ensure(size_t(ns) * 3 * sizeof(double)));
    HIP_TRY(c, w.vs.ensure(size_t(ns) * 2 * 4 * sizeof(double)));
    HIP_TRY(c, w.sd_dl.ensure(size_t(ns) * 3 * sizeof(double)));
    HIP_TRY(c, w.sdz_sl.ensure(size_t(ns) * sizeof(double)));
    HIP_TRY(c, w.sdz_dl.ensure(size_t(ns) * 3 * sizeof(double)));
    HIP_TRY(c, w.q.ensure(size_t(ns) * 9 * sizeof(double)));
    HIP_TRY(c, w.out[0].ensure(size_t(nt) * 6 * sizeof(double)));
    HIP_TRY(c, w.out[1].ensure(size_t(nt) * 10 * sizeof(double)));
    HIP_TRY(c, w.out[2].ensure(size_t(nt) * 4 * sizeof(double)));
    HIP_TRY(c, w.out[3].ensure(size_t(nt) * 10 * sizeof(double)));
    if (n > 0) HIP_TRY(c, hipMemcpyAsync(w.src.p, src, size_t(n) * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (n_trg > 0)
        HIP_TRY(c, hipMemcpyAsync(w.trg.p, trg, size_t(n_trg) * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, launch_wall_positions(n, w.src.as<double>(), c->origin[2], w.y2.as<double>(), w.yi.as<double>(), s));
    if (n > 0 && n_trg > 0) {
        const double *y2 = w.y2.as<double>(), *yi = w.yi.as<double>(), *xt = w.trg.as<double>();
        struct Sum {
            stkfmm_kernel k;
            int64_t nsl;
            const double *sl;
            int64_t ndl;
            const double *dl;
        };
        const Sum sums[4] = {
            {STKFMM_RPY, 2 * n, y2, 0, nullptr},   // b = 0 for the Stokeslet: hi/lo P2P
            {w.rpy ? STKFMM_LAP_PGRADGRAD : STKFMM_LAP_PGRAD, 0, nullptr, n, yi},
            {STKFMM_LAP_PGRAD, n, yi, w.rpy ? n : 0, w.rpy ? yi : nullptr},
            {STKFMM_LAP_QPGRADGRAD, n, yi, 0, nullptr},
        };
        for (int k = 0; k < w.nsub; ++k) {
            stkfmm_status st = stkfmm_set_points(w.sub[k], sums[k].k, STKFMM_BC_OPEN, sums[k].nsl, sums[k].sl,
                                                 sums[k].ndl, sums[k].dl, n_trg, xt, p, leaf_cap, stream);
            if (st != STKFMM_OK) return fail(c, st, std::string("wall summation: ") + w.sub[k]->err);
        }
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    c->kernel = kernel;
    c->bc = STKFMM_BC_WALL;
    c->p = p;
    c->leaf_cap = leaf_cap;
    c->n_sl = n_src;
    c->n_dl = 0;
    c->n_trg = n_trg;
    c->learned = false;
    c->validated = false;
    c->ops = nullptr;
    c->t_tree_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->planned = true;
    return STKFMM_OK;
}

// The evaluation pass of a wall plan: image strengths, the summations on the
// caller's stream, the assembly at the targets.
stkfmm_status wall_run(stkfmm_ctx *c, const double *sl_val, const double *dl_val, double *trg_val, void *stream) {
    WallPlan &w = *c->wall;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dl_val) return fail(c, STKFMM_E_ARG, "the wall kernels have no double-layer sources");
    if (w.n_trg == 0) return STKFMM_OK;
    if (!trg_val || (w.n_src > 0 && !sl_val)) return fail(c, STKFMM_E_ARG, "NULL value array");
    HIP_TRY(c, hipSetDevice(c->device));
    const int kt = w.rpy ? 6 : 3;
    std::memset(c->stage_ms, 0, sizeof(c->stage_ms));
    c->t_run_ms = 0.0;
    if (w.n_src == 0) {
        HIP_TRY(c, launch_fill_f64(trg_val, w.n_trg * kt, 0.0, s));
        return STKFMM_OK;
    }
    WallValueArgs va;
    va.n = w.n_src;
    va.y = w.src.as<double>();
    va.val = sl_val;
    va.rpy = w.rpy;
    va.zw = c->origin[2];
    va.vs = w.vs.as<double>();
    va.sd_dl = w.sd_dl.as<double>();
    va.sdz_sl = w.sdz_sl.as<double>();
    va.sdz_dl = w.sdz_dl.as<double>();
    va.q = w.q.as<double>();
    HIP_TRY(c, launch_wall_values(va, s));
    const double *sl[4] = {va.vs, nullptr, va.sdz_sl, va.q};
    const double *dl[4] = {nullptr, va.sd_dl, w.rpy ? va.sdz_dl : nullptr, nullptr};
    for (int k = 0; k < w.nsub; ++k) {
        stkfmm_status st = stkfmm_run(w.sub[k], sl[k], dl[k], w.out[k].as<double>(), stream);
        if (st != STKFMM_OK) return fail(c, st, std::string("wall summation: ") + w.sub[k]->err);
        c->t_run_ms += w.sub[k]->t_run_ms;
        for (int i = 0; i < 16; ++i) c->stage_ms[i] += w.sub[k]->stage_ms[i];
    }
    WallAssembleArgs aa;
    aa.nt = w.n_trg;
    aa.x = w.trg.as<double>();
    aa.zw = c->origin[2];
    aa.rpy = w.rpy;
    aa.us = w.out[0].as<double>();
    aa.sd = w.out[1].as<double>();
    aa.ksd = w.rpy ? 10 : 4;
    aa.sdz = w.out[2].as<double>();
    aa.qp = w.rpy ? w.out[3].as<double>() : nullptr;
    aa.out = trg_val;
    HIP_TRY(c, launch_wall_assemble(aa, s));
    return STKFMM_OK;
}

// Partial sums of stkfmm_direct_noalloc, one [slices][n_trg][k_trg] block
// per call, in a static device array instead of a hipMalloc'd buffer (for
// callers that cannot allocate).  Every GPU the library runs on holds its own
// copy, at its own address, until the process ends; host code reaches it
// only through that address, resolved once per device in stkfmm_setup.
constexpr int64_t kDirectScratchDoubles = int64_t(1) << 23;   // 64 MiB
static __device__ __align__(256) double scratch[kDirectScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;   // device -> device address of its scratch

// With `device` current: the address of this device's scratch (resolved on
// the first call for the device).
hipError_t resolve_scratch(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double *>(ptr);
    return hipSuccess;
}

double *scratch_ptr(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// Checks and fills the arguments shared by stkfmm_direct and
// stkfmm_direct_noalloc; the caller supplies a.work when a.slices > 1.
stkfmm_status direct_args(stkfmm_ctx *c, stkfmm_kernel kernel, int64_t n_sl, const double *sl_xyz,
                          const double *sl_val, int64_t n_dl, const double *dl_xyz, const double *dl_val,
                          int64_t n_trg, const double *trg_xyz, double *trg_val, DirectArgs &a) {
    if (!kernel_ok(int(kernel))) return fail(c, STKFMM_E_ARG, "unknown kernel");
    const KernelInfo &ki = kInfo[kernel];
    if (n_sl < 0 || n_dl < 0 || n_trg < 0) return fail(c, STKFMM_E_ARG, "negative size");
    if ((n_sl > 0 && (!sl_xyz || !sl_val)) || (n_dl > 0 && (!dl_xyz || !dl_val)) ||
        (n_trg > 0 && (!trg_xyz || !trg_val)))
        return fail(c, STKFMM_E_ARG, "NULL array");
    if (n_dl > 0 && ki.k_dl == 0) return fail(c, STKFMM_E_ARG, "kernel has no double-layer sources");
    a.n_sl = n_sl;
    a.n_dl = n_dl;
    a.n_trg = n_trg;
    a.sl = sl_xyz;
    a.sl_val = sl_val;
    a.dl = dl_xyz;
    a.dl_val = dl_val;
    a.trg = trg_xyz;
    a.k_sl = ki.k_sl;
    a.k_dl = ki.k_dl;
    a.k_trg = ki.k_trg;
    a.out = trg_val;
    a.slices = direct_f64_slices(n_trg, std::max(n_sl, n_dl));
    a.work = nullptr;
    return STKFMM_OK;
}

}  // namespace

namespace {
P2PArgs p2p_args(stkfmm_ctx *c);
}

extern "C" {

stkfmm_status stkfmm_kernel_dims(stkfmm_kernel k, int *k_sl, int *k_dl, int *k_trg) {
    if (!kernel_ok(int(k)) || !k_sl || !k_dl || !k_trg) return STKFMM_E_ARG;
    *k_sl = kInfo[k].k_sl;
    *k_dl = kInfo[k].k_dl;
    *k_trg = kInfo[k].k_trg;
    return STKFMM_OK;
}

stkfmm_status stkfmm_setup(stkfmm_ctx **out, const double origin[3], double box_len, int device, unsigned flags) {
    if (!out) return STKFMM_E_ARG;
    *out = nullptr;
    if (!origin || !(box_len > 0) || !std::isfinite(box_len) || flags != 0) return STKFMM_E_ARG;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(origin[k])) return STKFMM_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return STKFMM_E_DEVICE;
    auto *c = new (std::nothrow) stkfmm_ctx();
    if (!c) return STKFMM_E_NOMEM;
    c->device = device;
    std::memcpy(c->origin, origin, sizeof(c->origin));
    c->box_len = box_len;
    if (hipSetDevice(device) != hipSuccess || resolve_scratch(device) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return STKFMM_E_DEVICE;
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete c;
            return STKFMM_E_DEVICE;
        }
    *out = c;
    return STKFMM_OK;
}

void stkfmm_destroy(stkfmm_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->side) (void)hipStreamDestroy(c->side);
    delete c;
}

const char *stkfmm_last_error(const stkfmm_ctx *c) { return c ? c->err.c_str() : "null context"; }

stkfmm_status stkfmm_set_option(stkfmm_ctx *c, const char *key, const char *value) {
    if (!c || !key || !value) return STKFMM_E_ARG;
    if (c->wall)   // the wall plan's summations follow the context's options
        for (stkfmm_ctx *sc : c->wall->sub)
            if (sc) {
                stkfmm_status st = stkfmm_set_option(sc, key, value);
                if (st != STKFMM_OK) return fail(c, st, sc->err);
            }
    std::string k(key), v(value);
    if (k == "precision") {
        if (v == "fp32") c->precision = 0;
        else if (v == "split_bf16") c->precision = 1;
        else return fail(c, STKFMM_E_ARG, "precision must be fp32 or split_bf16");
        return STKFMM_OK;
    }
    if (k == "p2p_task_sources") {
        long n = std::atol(value);
        if (n < 64 || n > (1L << 24) || std::to_string(n) != v) return fail(c, STKFMM_E_ARG, "p2p_task_sources must lie in [64, 2^24]");
        c->p2p_task_sources = n;
        c->planned = false;
        return STKFMM_OK;
    }
    if (k == "tol") {
        char *end = nullptr;
        double t = std::strtod(value, &end);
        if (!end || *end || !(t > 0) || !(t < 1)) return fail(c, STKFMM_E_ARG, "tol must lie in (0, 1)");
        c->tol = t;
        c->planned = false;
        return STKFMM_OK;
    }
    if (k == "tree") {
        if (v == "gpu") c->tree_gpu = 1;
        else if (v == "host") c->tree_gpu = 0;
        else return fail(c, STKFMM_E_ARG, "tree must be gpu or host");
        c->planned = false;
        return STKFMM_OK;
    }
    if (k == "overlap") {
        if (v == "1") c->overlap = 1;
        else if (v == "0") c->overlap = 0;
        else return fail(c, STKFMM_E_ARG, "overlap must be 0 or 1");
        return STKFMM_OK;
    }
    if (k == "w_direct_frac" || k == "x_direct_frac") {
        char *end = nullptr;
        double t = std::strtod(value, &end);
        if (!end || *end || !(t >= 0) || !(t <= 16)) return fail(c, STKFMM_E_ARG, k + " must lie in [0, 16]");
        (k == "w_direct_frac" ? c->w_direct_frac : c->x_direct_frac) = t;
        c->planned = false;
        return STKFMM_OK;
    }
    if (k == "m2l_tol") {
        char *end = nullptr;
        double t = std::strtod(value, &end);
        if (!end || *end || !(t >= 0) || !(t < 1)) return fail(c, STKFMM_E_ARG, "m2l_tol must lie in [0, 1)");
        c->m2l_tol = t;
        c->m2l_tol_set = true;
        c->planned = false;
        return STKFMM_OK;
    }
    if (k == "svd_tol") {
        char *end = nullptr;
        double t = std::strtod(value, &end);
        if (!end || *end || !(t > 0) || !(t < 1)) return fail(c, STKFMM_E_ARG, "svd_tol must lie in (0, 1)");
        c->svd_tol = t;
        c->planned = false;
        return STKFMM_OK;
    }
    if (k == "operator_cache") {
        c->op_cache = v;
        return STKFMM_OK;
    }
    return fail(c, STKFMM_E_ARG, "unknown option " + k);
}

stkfmm_status stkfmm_prepare_operators(int p, stkfmm_bc bc, double svd_tol, double m2l_tol, const char *cache_dir,
                                       int *loaded, uint64_t *digest) {
    if (p < 2 || p > 16 || !(svd_tol > 0) || !(svd_tol < 1) || !(m2l_tol >= 0) || !(m2l_tol < 1))
        return STKFMM_E_ARG;
    if (bc != STKFMM_BC_OPEN && bc != STKFMM_BC_PXYZ && bc != STKFMM_BC_PXY && bc != STKFMM_BC_WALL)
        return STKFMM_E_ARG;
    const std::string dir = cache_dir ? cache_dir : "";
    const bool periodic = bc == STKFMM_BC_PXYZ;
    try {
        Operators h;
        bool ld = false;
        if (!cached_operators(dir, p, svd_tol, periodic, m2l_tol, h, &ld).empty()) return STKFMM_E_ARG;
        uint64_t dg = operators_digest(h, periodic);
        if (bc == STKFMM_BC_PXYZ || bc == STKFMM_BC_PXY) {
            std::vector<double> Q, X, Z;
            bool ls = false;
            if (!cached_periodic_stokes(dir, kStokesFarOrder, svd_tol, bc == STKFMM_BC_PXY, Q, X, Z, &ls).empty())
                return STKFMM_E_ARG;
            dg ^= stokes_far_digest(kStokesFarOrder, svd_tol, bc == STKFMM_BC_PXY, Q, X, Z) * 0x9e3779b97f4a7c15ull;
            ld = ld && ls;
        }
        if (loaded) *loaded = ld ? 1 : 0;
        if (digest) *digest = dg;
    } catch (const std::bad_alloc &) {
        return STKFMM_E_NOMEM;
    }
    return STKFMM_OK;
}

stkfmm_status stkfmm_get_timings(const stkfmm_ctx *c, double *t_tree, double *t_run, double stage_ms[16]) {
    if (!c) return STKFMM_E_ARG;
    if (t_tree) *t_tree = c->t_tree_ms;
    if (t_run) *t_run = c->t_run_ms;
    if (stage_ms) std::memcpy(stage_ms, c->stage_ms, sizeof(c->stage_ms));
    return STKFMM_OK;
}

stkfmm_status stkfmm_get_stats(const stkfmm_ctx *c, int64_t st[21]) {
    if (!c || !st) return STKFMM_E_ARG;
    if (!c->planned) return STKFMM_E_STATE;
    if (c->bc == STKFMM_BC_WALL) {
        if (c->wall && c->wall->sub[0] && c->wall->sub[0]->planned) return stkfmm_get_stats(c->wall->sub[0], st);
        std::memset(st, 0, 21 * sizeof(int64_t));
        st[8] = c->n_trg;
        st[9] = c->n_sl;
        return STKFMM_OK;
    }
    std::memset(st, 0, 21 * sizeof(int64_t));
    const Tree &t = c->tree;
    st[0] = int64_t(t.boxes.size());
    st[1] = int64_t(t.leaves.size());
    st[2] = t.depth;
    st[3] = t.p2p_pairs;
    st[4] = int64_t(t.v.size());
    st[5] = int64_t(t.w.size());
    st[6] = int64_t(t.x.size());
    st[7] = c->ops ? c->ops->M : 0;
    st[8] = c->n_trg;
    st[9] = c->n_sl;
    st[10] = c->n_dl;
    st[11] = int64_t(t.u.size());
    st[12] = c->direct_pairs;
    st[13] = c->w_direct;
    st[14] = c->x_direct;
    st[15] = c->n_p2p_tasks;
    st[16] = c->ops ? c->ops->kc : 0;
    st[17] = c->ops ? c->ops->Mp : 0;
    st[18] = c->ops ? c->ops->rank : 0;
    st[19] = c->p2p_lane_pairs;
    st[20] = c->rel_exact ? 1 : 0;
    return STKFMM_OK;
}

stkfmm_status stkfmm_get_tree(const stkfmm_ctx *c, int64_t sizes[8], int32_t *box, int32_t *perm, int32_t *off,
                              int32_t *ent) {
    if (!c || !sizes) return STKFMM_E_ARG;
    if (c->wall) return STKFMM_E_UNSUPPORTED;
    if (!c->planned) return STKFMM_E_STATE;
    const Tree &t = c->tree;
    const int64_t nb = int64_t(t.boxes.size());
    const std::vector<Entry> *L[4] = {&t.u, &t.v, &t.w, &t.x};
    const std::vector<int> *O[4] = {&t.u_off, &t.v_off, &t.w_off, &t.x_off};
    sizes[0] = nb;
    for (int q = 0; q < 4; ++q) sizes[1 + q] = int64_t(L[q]->size());
    sizes[5] = int64_t(t.perm_sl.size());
    sizes[6] = int64_t(t.perm_dl.size());
    sizes[7] = int64_t(t.perm_trg.size());
    if (!box) return STKFMM_OK;
    if (!perm || !off || !ent) return STKFMM_E_ARG;
    for (int64_t b = 0; b < nb; ++b) {
        const Box &B = t.boxes[b];
        int32_t *o = box + 12 * b;
        o[0] = B.level;
        for (int k = 0; k < 3; ++k) o[1 + k] = B.anchor[k];
        o[4] = B.parent;
        o[5] = B.leaf ? 1 : 0;
        o[6] = int32_t(B.sl[0]);  o[7] = int32_t(B.sl[1]);
        o[8] = int32_t(B.dl[0]);  o[9] = int32_t(B.dl[1]);
        o[10] = int32_t(B.trg[0]); o[11] = int32_t(B.trg[1]);
    }
    std::copy(t.perm_sl.begin(), t.perm_sl.end(), perm);
    std::copy(t.perm_dl.begin(), t.perm_dl.end(), perm + sizes[5]);
    std::copy(t.perm_trg.begin(), t.perm_trg.end(), perm + sizes[5] + sizes[6]);
    int64_t e0 = 0;
    for (int q = 0; q < 4; ++q) {
        std::copy(O[q]->begin(), O[q]->end(), off + q * (nb + 1));
        for (const Entry &en : *L[q]) {
            int32_t *o = ent + 4 * e0++;
            o[0] = en.box;
            for (int k = 0; k < 3; ++k) o[1 + k] = en.shift[k];
        }
    }
    return STKFMM_OK;
}

stkfmm_status stkfmm_set_points(stkfmm_ctx *c, stkfmm_kernel kernel, stkfmm_bc bc, int64_t n_sl,
                                const double *sl_xyz, int64_t n_dl, const double *dl_xyz, int64_t n_trg,
                                const double *trg_xyz, int p, int leaf_cap, void *stream) {
    if (!c) return STKFMM_E_ARG;
    c->planned = false;
    if (!kernel_ok(int(kernel))) return fail(c, STKFMM_E_ARG, "unknown kernel");
    const KernelInfo &ki = kInfo[kernel];
    if (n_sl < 0 || n_dl < 0 || n_trg < 0) return fail(c, STKFMM_E_ARG, "negative size");
    if ((n_sl > 0 && !sl_xyz) || (n_dl > 0 && !dl_xyz) || (n_trg > 0 && !trg_xyz))
        return fail(c, STKFMM_E_ARG, "NULL point array");
    if (n_dl > 0 && ki.k_dl == 0) return fail(c, STKFMM_E_ARG, "kernel has no double-layer sources");
    if (n_sl > INT32_MAX / 2 || n_dl > INT32_MAX / 2 || n_trg > INT32_MAX / 2)
        return fail(c, STKFMM_E_ARG, "too many points");
    if (p != 0 && (p < 2 || p > 16)) return fail(c, STKFMM_E_ARG, "p must be 0 (learned) or lie in [2, 16]");
    if (leaf_cap < 0) return fail(c, STKFMM_E_ARG, "leaf_cap must be 0 (learned) or >= 1");
    const bool learned = p == 0 || leaf_cap == 0;
    if (learned && !c->has_predictor) return fail(c, STKFMM_E_STATE, "learned mode needs stkfmm_set_predictor");
    if (learned && bc != STKFMM_BC_OPEN) return fail(c, STKFMM_E_UNSUPPORTED, "learned mode is open-boundary only");
    if (bc == STKFMM_BC_WALL)
        return wall_set_points(c, int(kernel), n_sl, sl_xyz, n_trg, trg_xyz, p, leaf_cap, stream);
    if (bc != STKFMM_BC_OPEN && bc != STKFMM_BC_PXYZ && bc != STKFMM_BC_PXY)
        return fail(c, STKFMM_E_UNSUPPORTED,
                    "only open, doubly and triply periodic and wall boundaries are implemented");
    if (bc == STKFMM_BC_PXYZ && kernel != STKFMM_LAP_PGRAD && kernel != STKFMM_LAP_PGRADGRAD &&
        kernel != STKFMM_LAP_QPGRADGRAD && !periodic_stokes(kernel))
        return fail(c, STKFMM_E_UNSUPPORTED,
                    "triply periodic boundary is implemented for the Laplace kernels and the Stokes kernels");
    if (bc == STKFMM_BC_PXY && !doubly_periodic_stokes(kernel))
        return fail(c, STKFMM_E_UNSUPPORTED,
                    "doubly periodic boundary is implemented for the Stokeslet and RPY");
    const int pmask = bc_axes(bc);
    const bool periodic = pmask != 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(c, hipSetDevice(c->device));
    auto t0 = std::chrono::steady_clock::now();
    const double *src[3] = {sl_xyz, dl_xyz, trg_xyz};
    const int64_t cnt[3] = {n_sl, n_dl, n_trg};
    const char *names[3] = {"sl_xyz", "dl_xyz", "trg_xyz"};
    // host copies of the coordinates (normalised, wrapped if periodic) where
    // the host needs them: the host tree builder and the learned mode's leaf
    // features; else the points are only checked, on the GPU
    std::vector<double> h[3];
    const bool host_coords = learned || !c->tree_gpu;
    if (host_coords) {
        stkfmm_status st = copy_coords(c, src, cnt, pmask, true, h, s);
        if (st != STKFMM_OK) return st;
    } else {
        for (int k = 0; k < 3; ++k) {
            bool nonfinite = false, outside = false;
            std::string e = check_points_gpu(src[k], cnt[k], c->origin, c->box_len, pmask, &nonfinite, &outside, stream);
            if (!e.empty()) return fail(c, STKFMM_E_DEVICE, e);
            if (nonfinite) return fail(c, STKFMM_E_ARG, std::string(names[k]) + ": non-finite coordinate");
            if (outside)
                return fail(c, STKFMM_E_DOMAIN, std::string(names[k]) + ": point outside [origin, origin+box_len)");
        }
    }
    // the caller's coordinates, kept for the accuracy check and fallback of
    // learned plans and for leaf features asked for later
    for (int k = 0; k < 3; ++k) {
        HIP_TRY(c, c->coords[k].ensure(std::max<int64_t>(cnt[k], 1) * 3 * sizeof(double)));
        if (cnt[k] > 0)
            HIP_TRY(c, hipMemcpyAsync(c->coords[k].p, src[k], cnt[k] * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    Tree &t = c->tree;
    c->learned = learned;
    c->validated = false;
    c->fell_back = false;
    c->sampled_err = -1.0;
    for (int k = 0; k < 4; ++k) c->p_hist[k] = c->cap_hist[k] = 0;
    std::string e;
    // the octree on the GPU from the caller's coordinates, or on the host
    // from the normalised copies (the same tree)
    auto build = [&](int cap, int pm, const std::unordered_map<uint64_t, int> *caps) {
        if (c->tree_gpu) return build_tree_gpu(src, cnt, c->origin, c->box_len, cap, pm, t, caps, stream);
        return build_tree(h[0].data(), n_sl, h[1].data(), n_dl, h[2].data(), n_trg, cap, pm, t, caps);
    };
    if (!learned) {
        e = build(leaf_cap, pmask, nullptr);
        if (!e.empty()) return fail(c, STKFMM_E_ARG, e);
    } else {
        // reference tree, per-leaf features, network on the GPU
        const int ref_cap = leaf_cap ? leaf_cap : kReferenceCap;
        e = build(ref_cap, 0, nullptr);
        if (!e.empty()) return fail(c, STKFMM_E_ARG, e);
        std::vector<float> feat;
        leaf_features(t, h[0].data(), h[1].data(), h[2].data(), c->tol, feat);
        const int64_t nl = int64_t(t.leaves.size());
        HIP_TRY(c, c->mlp_in.ensure(std::max<int64_t>(nl, 1) * kNumFeatures * sizeof(float)));
        HIP_TRY(c, c->mlp_out.ensure(std::max<int64_t>(nl, 1) * 8 * sizeof(float)));
        HIP_TRY(c, c->mlp_ws.ensure(std::max<int64_t>(stkfmm_mlp_workspace(nl), 1) * sizeof(float)));
        HIP_TRY(c, hipMemcpyAsync(c->mlp_in.p, feat.data(), feat.size() * sizeof(float), hipMemcpyHostToDevice, s));
        stkfmm_status sm = stkfmm_mlp_forward(c->predictor.as<float>(), nl, c->mlp_in.as<float>(), c->mlp_out.as<float>(),
                                              c->mlp_ws.as<float>(), stream);
        if (sm != STKFMM_OK) return fail(c, sm, "predictor inference failed");
        std::vector<float> logits(size_t(nl) * 8);
        HIP_TRY(c, hipMemcpy(logits.data(), c->mlp_out.p, logits.size() * sizeof(float), hipMemcpyDeviceToHost));
        // order: the smallest class whose estimated error over all targets,
        // from the calibration table (RMS error at each order of training
        // leaves of each predicted class), is within 0.8 tol
        const float *table = c->order_table;
        double est[4] = {0, 0, 0, 0}, ntot = 0;
        std::unordered_map<uint64_t, int> caps;
        for (int64_t i = 0; i < nl; ++i) {
            const float *l = &logits[size_t(i) * 8];
            const int pc = int(std::max_element(l, l + 4) - l), cc = int(std::max_element(l + 4, l + 8) - (l + 4));
            const Box &B = t.boxes[t.leaves[i]];
            const double nt = double(B.trg[1] - B.trg[0]);
            if (nt > 0) {
                c->p_hist[pc]++;
                c->cap_hist[cc]++;
                for (int q = 0; q < 4; ++q) est[q] += nt * double(table[pc * 4 + q]) * double(table[pc * 4 + q]);
                ntot += nt;
            }
            if (leaf_cap == 0 && kCapClasses[cc] < ref_cap)
                caps[box_hash(B.level, B.anchor[0], B.anchor[1], B.anchor[2])] = kCapClasses[cc];
        }
        int pq = 3;
        for (int q = 0; q < 4; ++q)
            if (ntot > 0 && std::sqrt(est[q] / ntot) <= 0.8 * c->tol) {
                pq = q;
                break;
            }
        if (p == 0) p = kOrderClasses[pq];
        if (leaf_cap == 0) {
            leaf_cap = ref_cap;
            if (!caps.empty()) {
                e = build(ref_cap, false, &caps);
                if (!e.empty()) return fail(c, STKFMM_E_ARG, e);
            }
        }
    }
    for (int k = 0; k < 3; ++k) c->hcoords[k].swap(h[k]);
    c->hcoords_valid = host_coords;
    DeviceOps *ops = nullptr;
    // learned plans size the translation compression to the error budget
    // (rank 160 at p = 8 for tol 1e-5) unless the caller set m2l_tol
    const double m2l_tol = learned && !c->m2l_tol_set && c->m2l_tol > 0 ? c->tol / 50.0 : c->m2l_tol;
    // the Laplace far-image operator is for triply periodic Laplace plans
    stkfmm_status st = get_ops(c, p, bc == STKFMM_BC_PXYZ, m2l_tol, &ops);
    if (st != STKFMM_OK) return st;
    c->stk = nullptr;
    if (periodic && periodic_stokes(kernel)) {
        st = get_periodic_stokes(c, pmask, &c->stk);
        if (st != STKFMM_OK) return st;
        const int Mf = c->stk->M;
        const int nch = stokes_root_chunks(n_sl) + stokes_root_chunks(n_dl);
        HIP_TRY(c, c->stk_F.ensure((size_t(6) * Mf + 3) * sizeof(double)));
        HIP_TRY(c, c->stk_part.ensure(size_t(std::max(nch, 1)) * (3 * Mf + 3) * sizeof(double)));
    }
    c->ops = ops;
    c->kernel = kernel;
    c->bc = bc;
    c->moments = kernel == STKFMM_LAP_QPGRADGRAD ? 2 : (n_sl == 0 && n_dl > 0) ? 1 : 0;
    c->p = p;
    c->leaf_cap = leaf_cap;
    c->n_sl = n_sl;
    c->n_dl = n_dl;
    c->n_trg = n_trg;
    if (t.boxes.size() >= (size_t(1) << 25)) return fail(c, STKFMM_E_UNSUPPORTED, "more than 2^25 boxes");
    const int nb = int(t.boxes.size());
    c->nbox = nb;
    const int nc = ki.ncomp, M = ops->M, Mp = ops->Mp;

    // ---------------------------------------------------------------- plan arrays
    Arena &ar = c->staging;
    ar.clear();
    c->a_perm_sl = ar.add(t.perm_sl);
    c->a_perm_dl = ar.add(t.perm_dl);
    c->a_perm_trg = ar.add(t.perm_trg);
    std::vector<double4> geom(nb);
    std::vector<int2> bsl(nb), bdl(nb);
    for (int b = 0; b < nb; ++b) {
        const Box &B = t.boxes[b];
        double hh = 1.0 / double(1 << B.level);
        geom[b] = make_double4((B.anchor[0] + 0.5) * hh, (B.anchor[1] + 0.5) * hh, (B.anchor[2] + 0.5) * hh, hh);
        bsl[b] = make_int2(int(B.sl[0]), int(B.sl[1]));
        bdl[b] = make_int2(int(B.dl[0]), int(B.dl[1]));
    }
    c->a_geom = ar.add(geom);
    c->a_box_sl = ar.add(bsl);
    c->a_box_dl = ar.add(bdl);
    std::vector<int> leaves_sl, leaves_dl;
    for (int b : t.leaves) {
        if (t.boxes[b].sl[1] > t.boxes[b].sl[0]) leaves_sl.push_back(b);
        if (t.boxes[b].dl[1] > t.boxes[b].dl[0]) leaves_dl.push_back(b);
    }
    c->n_leaves_sl = int(leaves_sl.size());
    c->a_leaves_sl = ar.add(leaves_sl);
    c->n_leaves_dl = int(leaves_dl.size());
    c->a_leaves_dl = ar.add(leaves_dl);
    // ---- direct (P2P) lists per leaf: U, plus W and X pairs cheaper to sum directly.
    // Per pair of points, a direct Stokes-kernel sum costs about 30 FP32
    // operations, an M2T evaluation 22 and a surface-tile (S2L) evaluation 15,
    // so a W pair with fewer than 0.73 M sources and an X pair whose target
    // box holds fewer than 0.5 M targets go to P2P.  Both routes are exact or
    // within the far-field error, so this only moves work.
    std::vector<std::vector<int2>> dlist(nb), wkeep(nb), xkeep(nb);
    c->w_direct = c->x_direct = 0;
    std::vector<int> stack;
    // a direct entry always names a leaf: a W box that is not a leaf enters as
    // the leaves below it that hold sources (same image shift)
    auto push_leaves = [&](std::vector<int2> &dst, int2 e) {
        stack.assign(1, e.x);
        while (!stack.empty()) {
            const int q = stack.back();
            stack.pop_back();
            const Box &Q = t.boxes[q];
            if (Q.nsrc_sub == 0) continue;
            if (Q.leaf) {
                dst.push_back(make_int2(q, e.y));
                continue;
            }
            for (int o = 7; o >= 0; --o)
                if (Q.child[o] >= 0) stack.push_back(Q.child[o]);
        }
    };
    for (int b : t.leaves) {
        if (t.boxes[b].ntrg_sub == 0) continue;
        for (int i = t.u_off[b]; i < t.u_off[b + 1]; ++i) dlist[b].push_back(make_int2(t.u[i].box, pack_shift(t.u[i].shift)));
        for (int i = t.w_off[b]; i < t.w_off[b + 1]; ++i) {
            int2 e = make_int2(t.w[i].box, pack_shift(t.w[i].shift));
            if (double(t.boxes[e.x].nsrc_sub) < c->w_direct_frac * M) {
                push_leaves(dlist[b], e);
                ++c->w_direct;
            } else {
                wkeep[b].push_back(e);
            }
        }
    }
    for (int b = 0; b < nb; ++b) {
        if (!t.has_local[b]) continue;
        for (int i = t.x_off[b]; i < t.x_off[b + 1]; ++i) {
            int2 e = make_int2(t.x[i].box, pack_shift(t.x[i].shift));
            if (double(t.boxes[b].ntrg_sub) < c->x_direct_frac * M) {
                ++c->x_direct;
                stack.assign(1, b);
                while (!stack.empty()) {
                    int q = stack.back();
                    stack.pop_back();
                    const Box &Q = t.boxes[q];
                    if (Q.ntrg_sub == 0) continue;
                    if (Q.leaf) dlist[q].push_back(e);
                    for (int o = 0; o < 8; ++o)
                        if (Q.child[o] >= 0) stack.push_back(Q.child[o]);
                }
            } else {
                xkeep[b].push_back(e);
            }
        }
    }
    // ---- target chunks and their P2P / L2T tasks
    const int64_t kP2PTaskSources = c->p2p_task_sources;   // sources per P2P task (balance)
    constexpr int kL2TTaskSets = 4;              // equivalent-point sets per L2T task
    std::vector<int4> chunks, chunk_tasks, p2p_tasks, l2t_tasks;
    std::vector<int2> p2p_ent, l2t_ent;
    c->direct_pairs = 0;
    c->p2p_lane_pairs = 0;
    // lane pairs of the P2P waves of a chunk of nt targets of leaf b: a full
    // wave takes one source per step; a wave left with m <= 32 targets splits
    // each entry's sources over floor(64/m) lane groups (p2p_kernel)
    auto chunk_lane_pairs = [&](int b, int64_t nt) {
        int64_t nsrc_all = 0;
        for (const int2 &e : dlist[b]) nsrc_all += t.boxes[e.x].nsrc_sub;
        int64_t lp = nsrc_all * (nt / 64 * 64);
        const int64_t m = nt % 64;
        if (m > 32) {
            lp += nsrc_all * 64;
        } else if (m > 0) {
            const int64_t g = 64 / m;
            for (const int2 &e : dlist[b]) lp += 64 * ((t.boxes[e.x].nsrc_sub + g - 1) / g);
        }
        return lp;
    };
    for (int b : t.leaves) {
        const Box &B = t.boxes[b];
        if (B.trg[1] == B.trg[0]) continue;
        const int e0 = int(p2p_ent.size());
        p2p_ent.insert(p2p_ent.end(), dlist[b].begin(), dlist[b].end());
        const int e1 = int(p2p_ent.size());
        const int q0 = int(l2t_ent.size());
        if (t.has_local[b]) l2t_ent.push_back(make_int2(b, kLocalSet));
        l2t_ent.insert(l2t_ent.end(), wkeep[b].begin(), wkeep[b].end());
        const int q1 = int(l2t_ent.size());
        int64_t nsrc_all = 0;
        for (int e = e0; e < e1; ++e) nsrc_all += t.boxes[p2p_ent[e].x].nsrc_sub;
        c->direct_pairs += nsrc_all * (B.trg[1] - B.trg[0]);
        for (int64_t t0i = B.trg[0]; t0i < B.trg[1]; t0i += 256)
            c->p2p_lane_pairs += chunk_lane_pairs(b, std::min<int64_t>(t0i + 256, B.trg[1]) - t0i);
        for (int64_t t0i = B.trg[0]; t0i < B.trg[1]; t0i += 256) {
            const int ci = int(chunks.size());
            chunks.push_back(make_int4(b, int(t0i), int(std::min<int64_t>(t0i + 256, B.trg[1])), 0));
            int4 ct;
            ct.x = int(p2p_tasks.size());
            int64_t acc = 0;
            int es = e0;
            for (int e = e0; e < e1; ++e) {
                int64_t n = t.boxes[p2p_ent[e].x].nsrc_sub;
                if (acc > 0 && acc + n > kP2PTaskSources) {
                    p2p_tasks.push_back(make_int4(ci, es, e, 0));
                    es = e;
                    acc = 0;
                }
                acc += n;
            }
            if (e1 > es) p2p_tasks.push_back(make_int4(ci, es, e1, 0));
            ct.y = int(p2p_tasks.size());
            ct.z = int(l2t_tasks.size());
            for (int q = q0; q < q1; q += kL2TTaskSets) l2t_tasks.push_back(make_int4(ci, q, std::min(q1, q + kL2TTaskSets), 0));
            ct.w = int(l2t_tasks.size());
            chunk_tasks.push_back(ct);
        }
    }
    c->nchunks = int(chunks.size());
    c->n_p2p_tasks = int(p2p_tasks.size());
    c->n_l2t_tasks = int(l2t_tasks.size());
    c->a_chunks = ar.add(chunks);
    c->a_chunk_tasks = ar.add(chunk_tasks);
    c->a_p2p_tasks = ar.add(p2p_tasks);
    c->a_p2p_ent = ar.add(p2p_ent);
    c->a_l2t_tasks = ar.add(l2t_tasks);
    c->a_l2t_ent = ar.add(l2t_ent);
    // ---- work by box (what the learned capacity labels are priced from)
    {
        const int side = ops->kc > 0 ? ops->kc : Mp;
        c->box_work.assign(nb, std::array<double, 5>{0, 0, 0, 0, 1});
        for (const int4 &ch : chunks) {
            const int b = ch.x;
            int64_t nsrc_all = 0;
            int ne = 0;
            for (const int2 &e : dlist[b]) nsrc_all += t.boxes[e.x].nsrc_sub, ++ne;
            const double waves = double((ch.z - ch.y + 63) / 64);
            c->box_work[b][0] += double(chunk_lane_pairs(b, ch.z - ch.y));
            c->box_work[b][1] += waves * ne;
        }
        for (int b = 0; b < nb; ++b) {
            const Box &B = t.boxes[b];
            if (t.has_local[b]) c->box_work[b][2] += double(t.v_off[b + 1] - t.v_off[b]) * 2.0 * side * side * nc;
            for (const int2 &e : xkeep[b]) c->box_work[b][3] += double(t.boxes[e.x].nsrc_sub) * M;
            if (!B.leaf) continue;
            c->box_work[b][3] += double(B.sl[1] - B.sl[0] + B.dl[1] - B.dl[0]) * M;
            c->box_work[b][3] += double(B.trg[1] - B.trg[0]) * M * ((t.has_local[b] ? 1 : 0) + wkeep[b].size());
        }
    }
    // ---- surface-tile tasks: S2M (each leaf's own sources) and S2L (kept X pairs)
    constexpr int kS2CTaskSources = 1024;
    size_t s2c_tasks_max = 0;
    auto make_phase = [&](const std::vector<std::pair<int, std::vector<int2>>> &dst_src) {
        S2CPhase ph;
        std::vector<int4> tsl, tdl;
        std::vector<std::vector<int>> own_sl(dst_src.size()), own_dl(dst_src.size());
        for (size_t d = 0; d < dst_src.size(); ++d) {
            const int dst = dst_src[d].first;
            for (const int2 &e : dst_src[d].second) {
                const Box &A = t.boxes[e.x];
                const int code = e.y | (e.x << 6);      // source leaf and image shift
                for (int64_t j = A.sl[0]; j < A.sl[1]; j += kS2CTaskSources) {
                    own_sl[d].push_back(int(tsl.size()));
                    tsl.push_back(make_int4(dst, code, int(j), int(std::min<int64_t>(j + kS2CTaskSources, A.sl[1]))));
                }
                for (int64_t j = A.dl[0]; j < A.dl[1]; j += kS2CTaskSources) {
                    own_dl[d].push_back(int(tdl.size()));
                    tdl.push_back(make_int4(dst, code, int(j), int(std::min<int64_t>(j + kS2CTaskSources, A.dl[1]))));
                }
            }
        }
        ph.n_sl = int(tsl.size());
        ph.n_dl = int(tdl.size());
        std::vector<int4> all(tsl);
        all.insert(all.end(), tdl.begin(), tdl.end());
        std::vector<int> rdst, roff, rtask;
        for (size_t d = 0; d < dst_src.size(); ++d) {
            if (own_sl[d].empty() && own_dl[d].empty()) continue;
            rdst.push_back(dst_src[d].first);
            roff.push_back(int(rtask.size()));
            rtask.insert(rtask.end(), own_sl[d].begin(), own_sl[d].end());
            for (int q : own_dl[d]) rtask.push_back(ph.n_sl + q);
        }
        roff.push_back(int(rtask.size()));
        ph.n_dst = int(rdst.size());
        ph.tasks = ar.add(all);
        ph.rdst = ar.add(rdst);
        ph.roff = ar.add(roff);
        ph.rtask = ar.add(rtask);
        s2c_tasks_max = std::max(s2c_tasks_max, all.size());
        return ph;
    };
    {
        std::vector<std::pair<int, std::vector<int2>>> up, dn;
        for (int b : t.leaves)
            if (t.boxes[b].nsrc_sub > 0) up.push_back({b, {make_int2(b, kZeroShift)}});
        for (int b = 0; b < nb; ++b)
            if (t.has_local[b] && !xkeep[b].empty()) dn.push_back({b, xkeep[b]});
        c->s2m = make_phase(up);
        c->s2l = make_phase(dn);
    }

    // levels carrying equivalent densities
    c->lmin_up = periodic ? 0 : 2;
    c->lmin_dn = periodic ? 0 : 2;
    c->ybuf_floats = 0;
    // M2L: V-list pairs grouped by offset
    c->m2l = make_v_batch(ar, t, geom, nc, c->ybuf_floats, Mp);
    // compression of every box's upward densities (compressed translations)
    c->n_cmp_tiles = 0;
    if (ops->kc > 0) {
        std::vector<int4> tiles;
        std::vector<int> cols(size_t(nb) * nc);
        std::iota(cols.begin(), cols.end(), 0);
        for (int t0 = 0; t0 < nb * nc; t0 += 128) tiles.push_back(make_int4(0, t0, std::min(128, nb * nc - t0), 0));
        c->n_cmp_tiles = int(tiles.size());
        c->a_cmp_tiles = ar.add(tiles);
        c->a_cmp_cols = ar.add(cols);
    }
    // M2M (by parent level) and L2L (by child level), grouped by octant
    c->m2m.assign(t.depth + 1, Batch());
    c->l2l.assign(t.depth + 1, L2LLevel());
    c->upinv.assign(t.depth + 1, PinvLevel());
    c->dnpinv.assign(t.depth + 1, PinvLevel());
    for (int l = 0; l <= t.depth; ++l) {
        std::vector<Pair> up, dn;
        std::vector<int> ub, uc, db, dcx;
        std::vector<double> us, ds;
        for (int b = t.level_start[l]; b < t.level_start[l + 1]; ++b) {
            const Box &B = t.boxes[b];
            const double hb = geom[b].w;
            if (l >= c->lmin_up && B.nsrc_sub > 0) {
                for (int o = 0; o < 8 && !B.leaf; ++o) {
                    int ch = B.child[o];
                    if (ch < 0 || t.boxes[ch].nsrc_sub == 0) continue;
                    Pair pr;
                    pr.src = ch;
                    pr.dst = b;
                    pr.op = o;
                    // Psi_P = Psi_C - (c_P - c_C).Phi
                    for (int k = 0; k < 3; ++k) pr.delta[k] = float(geom[b].x * 0 + ((&geom[b].x)[k] - (&geom[ch].x)[k]));
                    pr.scale = 1.0 / hb;
                    up.push_back(pr);
                }
                for (int k = 0; k < nc; ++k) {
                    ub.push_back(b * nc + k);
                    uc.push_back(b * nc + k);
                    us.push_back(hb);
                }
            }
            if (l >= c->lmin_dn && t.has_local[b]) {
                if (B.parent >= 0 && t.has_local[B.parent]) {
                    int o = -1;
                    for (int k = 0; k < 8; ++k)
                        if (t.boxes[B.parent].child[k] == b) o = k;
                    Pair pr;
                    pr.src = B.parent;
                    pr.dst = b;
                    pr.op = o;
                    // Psi_C = Psi_P - (c_C - c_P).Phi
                    for (int k = 0; k < 3; ++k) pr.delta[k] = float((&geom[b].x)[k] - (&geom[B.parent].x)[k]);
                    pr.scale = 1.0 / geom[B.parent].w;
                    dn.push_back(pr);
                }
                // densities only where targets read them: L2T at leaves
                for (int k = 0; k < nc && B.leaf; ++k) {
                    db.push_back(b * nc + k);
                    dcx.push_back(b * nc + k);
                    ds.push_back(hb);
                }
            }
        }
        c->m2m[l] = make_batch(ar, up, nc, 0, c->ybuf_floats, Mp);
        {
            // child check <- parent check, blocks of 64 / nc pairs sharing an octant
            std::stable_sort(dn.begin(), dn.end(), [](const Pair &x, const Pair &y) { return x.op < y.op; });
            const int per = 64 / nc;
            std::vector<int4> blocks;
            std::vector<int2> prs;
            std::vector<double> dl;
            for (size_t i = 0; i < dn.size();) {
                size_t j = i;
                while (j < dn.size() && dn[j].op == dn[i].op && int(j - i) < per) ++j;
                blocks.push_back(make_int4(dn[i].op, int(i), int(j - i), 0));
                i = j;
            }
            for (const Pair &pr : dn) {
                prs.push_back(make_int2(pr.src, pr.dst));
                for (int k = 0; k < 3; ++k) dl.push_back((&geom[pr.dst].x)[k] - (&geom[pr.src].x)[k]);
            }
            L2LLevel &ll = c->l2l[l];
            ll.nblocks = int(blocks.size());
            ll.blocks = ar.add(blocks);
            ll.pairs = ar.add(prs);
            ll.delta = ar.add(dl);
        }
        PinvLevel &pu = c->upinv[l];
        pu.ncol = int(ub.size());
        pu.bidx = ar.add(ub);
        pu.cidx = ar.add(uc);
        pu.cscale = ar.add(us);
        PinvLevel &pd = c->dnpinv[l];
        pd.ncol = int(db.size());
        pd.bidx = ar.add(db);
        pd.cidx = ar.add(dcx);
        pd.cscale = ar.add(ds);
    }
    HIP_TRY(c, c->arena.ensure(ar.used));
    HIP_TRY(c, hipMemcpyAsync(c->arena.p, ar.host.data(), ar.used, hipMemcpyHostToDevice, s));

    // ---------------------------------------------------------------- work buffers
    HIP_TRY(c, c->sl_rec.ensure(size_t(std::max<int64_t>(n_sl, 1)) * ki.rec_sl * sizeof(float)));
    HIP_TRY(c, c->dl_rec.ensure(size_t(std::max<int64_t>(n_dl, 1)) * std::max(ki.rec_dl, 1) * sizeof(float)));
    HIP_TRY(c, c->trg_rec.ensure(size_t(std::max<int64_t>(n_trg, 1)) * 8 * sizeof(float)));
    HIP_TRY(c, c->up_dens.ensure(size_t(nb) * nc * Mp * sizeof(float)));
    HIP_TRY(c, c->dn_dens.ensure(size_t(nb) * nc * Mp * sizeof(float)));
    HIP_TRY(c, c->up_chk.ensure(size_t(nb) * nc * M * sizeof(double)));
    HIP_TRY(c, c->dn_chk.ensure(size_t(nb) * nc * M * sizeof(double)));
    HIP_TRY(c, c->Ybuf.ensure(std::max<size_t>(c->ybuf_floats, 1) * sizeof(float)));
    if (ops->kc > 0) HIP_TRY(c, c->up_cmp.ensure(size_t(nb) * nc * ops->kc * sizeof(float)));
    HIP_TRY(c, c->near_part.ensure(size_t(std::max(c->n_p2p_tasks, 1)) * 256 * ki.kt_acc * sizeof(double)));
    HIP_TRY(c, c->far_part.ensure(size_t(std::max(c->n_l2t_tasks, 1)) * 256 * ki.kt_acc * sizeof(double)));
    HIP_TRY(c, c->s2c_part.ensure(std::max<size_t>(s2c_tasks_max, 1) * nc * M * sizeof(float)));
    HIP_TRY(c, c->sl_stage.ensure(size_t(std::max<int64_t>(n_sl, 1)) * s2c_stage_stride(stage_kind(kernel)) *
                                  sizeof(float)));
    HIP_TRY(c, c->dl_stage.ensure(size_t(std::max<int64_t>(n_dl, 1)) * s2c_stage_stride(dl_kind(kernel)) *
                                  sizeof(float)));
    HIP_TRY(c, c->partial.ensure(4096 * sizeof(double)));
    // densities: padding rows stay zero (the GEMM reads Mp rows)
    HIP_TRY(c, launch_fill_f32(c->up_dens.as<float>(), int64_t(nb) * nc * Mp, 0.0f, s));
    HIP_TRY(c, launch_fill_f32(c->dn_dens.as<float>(), int64_t(nb) * nc * Mp, 0.0f, s));
    // source/target positions in leaf order
    const double3 org = make_double3(c->origin[0], c->origin[1], c->origin[2]);
    const double inv = 1.0 / c->box_len;
    HIP_TRY(c, launch_pack_sources(n_sl, sl_xyz, at<int32_t>(c, c->a_perm_sl), org, inv, ki.rec_sl,
                                   c->sl_rec.as<float>(), s));
    HIP_TRY(c, launch_pack_sources(n_dl, dl_xyz, at<int32_t>(c, c->a_perm_dl), org, inv, std::max(ki.rec_dl, 8),
                                   c->dl_rec.as<float>(), s));
    HIP_TRY(c, launch_pack_targets(n_trg, trg_xyz, at<int32_t>(c, c->a_perm_trg), org, inv, c->trg_rec.as<float>(), s));
    c->rel_exact = false;
    if (p2p_uses_rel(c->kernel)) {
        HIP_TRY(c, launch_rel_positions(c->n_leaves_sl, at<int>(c, c->a_leaves_sl), at<int2>(c, c->a_box_sl),
                                        at<double4>(c, c->a_geom), ki.rec_sl, c->sl_rec.as<float>(), s));
        // distinct points of different leaves closer than the leaf-relative
        // positions resolve: this plan forms r from hi/lo coordinates instead
        unsigned *flag = reinterpret_cast<unsigned *>(c->partial.as<double>());
        HIP_TRY(c, launch_fill_f32(reinterpret_cast<float *>(flag), 1, 0.0f, s));
        HIP_TRY(c, launch_rel_check(c->n_p2p_tasks, p2p_args(c), ki.rec_sl, flag, s));
        unsigned h = 0;
        HIP_TRY(c, hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        c->rel_exact = h != 0;
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    c->t_tree_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->planned = true;
    return STKFMM_OK;
}

}  // extern "C"

namespace {


P2PArgs p2p_args(stkfmm_ctx *c) {
    P2PArgs a;
    a.tasks = at<int4>(c, c->a_p2p_tasks);
    a.chunks = at<int4>(c, c->a_chunks);
    a.trg = c->trg_rec.as<float>();
    a.ent = at<int2>(c, c->a_p2p_ent);
    a.box_sl = at<int2>(c, c->a_box_sl);
    a.box_dl = at<int2>(c, c->a_box_dl);
    a.sl = c->sl_rec.as<float>();
    a.dl = c->dl_rec.as<float>();
    a.geom = at<double4>(c, c->a_geom);
    a.part = c->near_part.as<double>();
    return a;
}

CombineMap combine_map(int k, double L) {
    CombineMap m;
    for (int i = 0; i < kMaxAcc; ++i) {
        m.src[i] = -1;
        m.scale[i] = 0;
    }
    const double c4 = 1.0 / (4.0 * kPi), c8 = 1.0 / (8.0 * kPi);
    switch (k) {
        case kStokeslet:
        case kStokesRegVel:
            for (int i = 0; i < 3; ++i) m.src[i] = i, m.scale[i] = c8 / L;
            break;
        case kStokesRegVelOmega:
            for (int i = 0; i < 3; ++i) m.src[i] = i, m.scale[i] = c8 / L;
            for (int i = 3; i < 6; ++i) m.src[i] = i, m.scale[i] = c8 / (L * L);
            break;
        case kRPY:
            for (int i = 0; i < 3; ++i) m.src[i] = i, m.scale[i] = c8 / L;
            for (int i = 3; i < 6; ++i) m.src[i] = i, m.scale[i] = c8 / (L * L * L);
            break;
        case kLapPGrad:
        case kLapPGradGrad:
        case kLapQPGradGrad:
            m.src[0] = 0, m.scale[0] = c4 / L;
            for (int i = 1; i < 4; ++i) m.src[i] = i, m.scale[i] = c4 / (L * L);
            if (k != kLapPGrad)
                for (int i = 4; i < 10; ++i) m.src[i] = i, m.scale[i] = c4 / (L * L * L);
            break;
        case kPVel:
        case kPVelGrad:
        case kPVelLaplacian:
            m.src[0] = 0, m.scale[0] = c8 / (L * L);
            for (int i = 1; i < 4; ++i) m.src[i] = i, m.scale[i] = c8 / L;
            if (k == kPVel) break;
            for (int i = 4; i < 7; ++i) m.src[i] = i, m.scale[i] = c8 / (L * L * L);
            if (k == kPVelGrad)
                for (int i = 7; i < 16; ++i) m.src[i] = i, m.scale[i] = c8 / (L * L);
            break;
        case kTraction: {
            const int sym[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
            for (int i = 0; i < 9; ++i) m.src[i] = sym[i], m.scale[i] = c4 / (L * L);
            break;
        }
    }
    return m;
}

__global__ void pack_values_kernel(int64_t n, const double *__restrict__ val, const int32_t *__restrict__ perm,
                                   double inv_len, int kind, int rec, float *__restrict__ out) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    float *o = out + i * rec;
    switch (kind) {
        case 0: {
            const double *v = val + 3 * j;
            o[6] = float(v[0]); o[7] = float(v[1]); o[8] = float(v[2]);
            break;
        }
        case 1: {
            const double *v = val + 4 * j;
            double b = v[3] * inv_len;
            o[6] = float(v[0]); o[7] = float(v[1]); o[8] = float(v[2]); o[9] = float(b * b);
            break;
        }
        case 2: o[6] = float(val[j]); break;
        case 3: {
            const double *v = val + 3 * j;
            o[6] = float(v[0] * inv_len); o[7] = float(v[1] * inv_len); o[8] = float(v[2] * inv_len);
            break;
        }
        case 4: {   // force f and flux q / L (its flow q r/r^3 falls one power faster than f/r)
            const double *v = val + 4 * j;
            o[6] = float(v[0]); o[7] = float(v[1]); o[8] = float(v[2]); o[9] = float(v[3] * inv_len);
            break;
        }
        case 5: {
            const double *D = val + 9 * j;
            o[6] = float(D[0] * inv_len);
            o[7] = float(0.5 * (D[1] + D[3]) * inv_len);
            o[8] = float(0.5 * (D[2] + D[6]) * inv_len);
            o[9] = float(D[4] * inv_len);
            o[10] = float(0.5 * (D[5] + D[7]) * inv_len);
            o[11] = float(D[8] * inv_len);
            break;
        }
        case 7: {   // regularized force and torque: f, t / L, (3/2) eps^2, eps^2
            const double *v = val + 7 * j;
            const double e = v[6] * inv_len;
            o[6] = float(v[0]); o[7] = float(v[1]); o[8] = float(v[2]);
            o[9] = float(v[3] * inv_len); o[10] = float(v[4] * inv_len); o[11] = float(v[5] * inv_len);
            o[12] = float(1.5 * e * e);
            o[13] = float(e * e);
            break;
        }
        case 8: {   // Laplace quadrupole: Q^s / L^2 (xx, xy, xz, yy, yz, zz)
            const double *Q = val + 9 * j;
            const double s2 = inv_len * inv_len;
            o[6] = float(Q[0] * s2);
            o[7] = float(0.5 * (Q[1] + Q[3]) * s2);
            o[8] = float(0.5 * (Q[2] + Q[6]) * s2);
            o[9] = float(Q[4] * s2);
            o[10] = float(0.5 * (Q[5] + Q[7]) * s2);
            o[11] = float(Q[8] * s2);
            break;
        }
        case 6: {   // regularized Stokeslet: f, then (3/2) eps^2 (far field) and eps^2 (P2P)
            const double *v = val + 4 * j;
            const double e = v[3] * inv_len;
            o[6] = float(v[0]); o[7] = float(v[1]); o[8] = float(v[2]);
            o[9] = float(1.5 * e * e);
            o[10] = float(e * e);
            break;
        }
    }
}

// per-block partial sums of q and |q| (net-charge check of periodic problems)
__global__ void charge_partials(int64_t n, const double *__restrict__ q, double *__restrict__ part) {
    __shared__ double s0[256], s1[256];
    double a = 0, b = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        a += q[i];
        b += fabs(q[i]);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

stkfmm_status run_pass(stkfmm_ctx *c, const double *sl_val, const double *dl_val, double *trg_val, void *stream) {
    if (!c) return STKFMM_E_ARG;
    if (!c->planned) return fail(c, STKFMM_E_STATE, "stkfmm_run before stkfmm_set_points");
    if ((c->n_sl > 0 && !sl_val) || (c->n_dl > 0 && !dl_val) || (c->n_trg > 0 && !trg_val))
        return fail(c, STKFMM_E_ARG, "NULL value array");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(c, hipSetDevice(c->device));
    const KernelInfo &ki = kInfo[c->kernel];
    const Tree &t = c->tree;
    const DeviceOps &o = *c->ops;
    const int nc = ki.ncomp;
    const bool periodic = bc_axes(c->bc) != 0;
    if (c->n_trg == 0) return STKFMM_OK;
    const bool pstokes = periodic && periodic_stokes(c->kernel);
    // sums of the first ncomp values of each source and of their absolute
    // values (one reduction on the device, a fixed order on the host)
    auto value_sums = [&](int64_t n, const double *v, int stride, int ncomp, double *sum,
                          double *abs_sum) -> stkfmm_status {
        const int nbk = 256;
        HIP_TRY(c, launch_value_partials(n, v, stride, ncomp, nbk, c->partial.as<double>(), s));
        std::vector<double> hp(size_t(ncomp + 1) * nbk);
        HIP_TRY(c, hipMemcpyAsync(hp.data(), c->partial.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        for (int k = 0; k <= ncomp; ++k) (k < ncomp ? sum[k] : *abs_sum) = 0.0;
        for (int i = 0; i < nbk; ++i) {
            for (int k = 0; k < ncomp; ++k) sum[k] += hp[size_t(ncomp + 1) * i + k];
            *abs_sum += hp[size_t(ncomp + 1) * i + ncomp];
        }
        return STKFMM_OK;
    };
    if (pstokes && c->n_sl > 0) {
        // zero net force (the Ewald convention drops the k = 0 mode) and,
        // for PVel, zero net flux q
        const int ncomp = pvel_family(c->kernel) ? 4 : 3;
        double f[4], fa;
        stkfmm_status st = value_sums(c->n_sl, sl_val, ki.k_sl, ncomp, f, &fa);
        if (st != STKFMM_OK) return st;
        for (int k = 0; k < 3; ++k)
            if (std::fabs(f[k]) > 1e-9 * std::max(1.0, fa))
                return fail(c, STKFMM_E_DOMAIN, "periodic Stokes needs zero net force");
        if (ncomp == 4 && std::fabs(f[3]) > 1e-9 * std::max(1.0, fa))
            return fail(c, STKFMM_E_DOMAIN, "periodic PVel needs zero net flux (sum of q)");
    }
    if (pstokes && c->n_dl > 0) {
        // the trace of D carries a flux (tr D r/r^3): its sum must vanish
        double d[9], da;
        stkfmm_status st = value_sums(c->n_dl, dl_val, ki.k_dl, 9, d, &da);
        if (st != STKFMM_OK) return st;
        if (std::fabs(d[0] + d[4] + d[8]) > 1e-9 * std::max(1.0, da))
            return fail(c, STKFMM_E_DOMAIN, "periodic PVel needs a zero sum of tr D over the double layer");
    }
    if (!pstokes && periodic && c->n_sl > 0 && c->kernel != kLapQPGradGrad) {
        // zero net charge (tin-foil Ewald convention needs a neutral cell;
        // quadrupoles carry none)
        const int nbk = 256;
        hipLaunchKernelGGL(charge_partials, dim3(nbk), dim3(256), 0, s, c->n_sl, sl_val, c->partial.as<double>());
        HIP_TRY(c, hipGetLastError());
        std::vector<double> hp(2 * nbk);
        HIP_TRY(c, hipMemcpyAsync(hp.data(), c->partial.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        double q = 0, qa = 0;
        for (int i = 0; i < nbk; ++i) q += hp[2 * i], qa += hp[2 * i + 1];
        if (std::fabs(q) > 1e-9 * std::max(1.0, qa))
            return fail(c, STKFMM_E_DOMAIN, "periodic Laplace needs zero net charge");
    }
    hipEvent_t *ev = c->ev;
    int ne = 0;
    bool m2l_timed = false;                                    // ev[22], ev[23]: the V-list GEMM
    HIP_TRY(c, hipEventRecord(ev[ne++], s));                  // 0 start
    const double inv = 1.0 / c->box_len;
    if (c->n_sl > 0) {
        hipLaunchKernelGGL(pack_values_kernel, dim3((c->n_sl + 255) / 256), dim3(256), 0, s, c->n_sl, sl_val,
                           at<int32_t>(c, c->a_perm_sl), inv, sl_kind(c->kernel), ki.rec_sl, c->sl_rec.as<float>());
        HIP_TRY(c, hipGetLastError());
    }
    if (c->n_dl > 0) {
        hipLaunchKernelGGL(pack_values_kernel, dim3((c->n_dl + 255) / 256), dim3(256), 0, s, c->n_dl, dl_val,
                           at<int32_t>(c, c->a_perm_dl), inv, dl_kind(c->kernel), ki.rec_dl, c->dl_rec.as<float>());
        HIP_TRY(c, hipGetLastError());
    }
    HIP_TRY(c, hipEventRecord(ev[ne++], s));                  // 1 packed
    // ---- near field: on the side stream (overlapping the far field) or first on s
    hipStream_t ps = c->overlap ? c->side : s;
    if (c->overlap) HIP_TRY(c, hipStreamWaitEvent(c->side, ev[1], 0));
    HIP_TRY(c, hipEventRecord(ev[20], ps));
    HIP_TRY(c, launch_p2p(c->kernel, c->n_p2p_tasks, p2p_args(c), c->rel_exact, ps));
    HIP_TRY(c, hipEventRecord(ev[21], ps));
    if (!c->overlap) HIP_TRY(c, hipEventRecord(ev[1], s));   // far-field stages start after P2P
    // ---- far field
    const bool far = t.depth >= 2 || periodic;
    double *upchk = c->up_chk.as<double>(), *dnchk = c->dn_chk.as<double>();
    float *updens = c->up_dens.as<float>(), *dndens = c->dn_dens.as<float>();
    auto s2c = [&](const S2CPhase &ph, double alpha, double *chk, int accumulate) -> hipError_t {
        S2CArgs a;
        a.tasks = at<int4>(c, ph.tasks);
        a.geom = at<double4>(c, c->a_geom);
        a.grid = o.grid.as<float>();
        a.M = o.M;
        a.alpha = alpha;
        a.part = c->s2c_part.as<float>();
        a.staged = c->sl_stage.as<float>();
        hipError_t e = launch_s2c(stage_kind(c->kernel), ph.n_sl, a, s);
        if (e != hipSuccess) return e;
        if (ph.n_dl > 0) {
            a.tasks = at<int4>(c, ph.tasks) + ph.n_sl;
            a.part = c->s2c_part.as<float>() + int64_t(ph.n_sl) * nc * o.M;
            a.staged = c->dl_stage.as<float>();
            e = launch_s2c(dl_kind(c->kernel), ph.n_dl, a, s);
            if (e != hipSuccess) return e;
        }
        S2CReduceArgs r;
        r.dst = at<int>(c, ph.rdst);
        r.off = at<int>(c, ph.roff);
        r.task = at<int>(c, ph.rtask);
        r.part = c->s2c_part.as<float>();
        r.chk = chk;
        r.M = o.M;
        r.ncomp = nc;
        r.accumulate = accumulate;
        return launch_s2c_reduce(ph.n_dst, r, s);
    };
    if (far) {
        // sources staged relative to their leaf centres (read by S2M and S2L)
        HIP_TRY(c, launch_stage_sources(stage_kind(c->kernel), c->n_leaves_sl, at<int>(c, c->a_leaves_sl),
                                        at<int2>(c, c->a_box_sl), at<double4>(c, c->a_geom), c->sl_rec.as<float>(),
                                        ki.rec_sl, c->sl_stage.as<float>(), s));
        if (c->n_dl > 0)
            HIP_TRY(c, launch_stage_sources(dl_kind(c->kernel), c->n_leaves_dl, at<int>(c, c->a_leaves_dl),
                                            at<int2>(c, c->a_box_dl), at<double4>(c, c->a_geom),
                                            c->dl_rec.as<float>(), ki.rec_dl, c->dl_stage.as<float>(), s));
        // upward pass
        HIP_TRY(c, s2c(c->s2m, kAlphaOut, upchk, 0));
        HIP_TRY(c, hipEventRecord(ev[ne++], s));              // 2 S2M
        for (int l = t.depth; l >= c->lmin_up; --l) {
            if (l < t.depth) {
                stkfmm_status st = run_batch(c, c->m2m[l], o.m2m.as<float>(), updens, upchk, s);
                if (st != STKFMM_OK) return st;
            }
            const DevMem &P = c->moments == 2 ? o.uc2ue_m2 : c->moments == 1 ? o.uc2ue_m1 : o.uc2ue;
            stkfmm_status st = run_pinv(c, c->upinv[l], P.as<double>(), upchk, updens, s);
            if (st != STKFMM_OK) return st;
        }
        HIP_TRY(c, hipEventRecord(ev[ne++], s));              // 3 upward
        HIP_TRY(c, launch_fill_f64(dnchk, int64_t(c->nbox) * nc * o.M, 0.0, s));
        stkfmm_status st = STKFMM_OK;
        if (o.kc > 0) {
            st = run_compress(c, updens, c->up_cmp.as<float>(), s);
            if (st != STKFMM_OK) return st;
            st = run_batch(c, c->m2l, o.m2l_c.as<float>(), c->up_cmp.as<float>(), dnchk, s, c->precision == 1, true,
                           ev[22], ev[23]);
        } else {
            st = run_batch(c, c->m2l, o.m2l.as<float>(), updens, dnchk, s, c->precision == 1, false, ev[22],
                           ev[23]);
        }
        m2l_timed = c->m2l.npairs > 0;
        if (st != STKFMM_OK) return st;
        HIP_TRY(c, hipEventRecord(ev[ne++], s));              // 4 M2L
        HIP_TRY(c, s2c(c->s2l, kAlphaIn, dnchk, 1));
        if (c->bc == STKFMM_BC_PXYZ && nc == 1) HIP_TRY(c, launch_periodic(o.tm2l.as<double>(), updens, dnchk, o.M, o.Mp, nc, 0, s));
        if (pstokes) {
            // the root's flow at its check points: single layer, then double
            // layer chunks, summed in that order
            const int M = c->stk->M;
            const int nch_sl = stokes_root_chunks(c->n_sl), nch_dl = stokes_root_chunks(c->n_dl);
            double *part = c->stk_part.as<double>();
            // the regularized Stokeslet's records carry b^2 = 3 eps^2 / 2: its far
            // field is RPY's
            const int kind = c->kernel == kRPY || c->kernel == kStokesRegVel ? 1
                           : pvel_family(c->kernel)         ? 2
                           : c->kernel == kStokesRegVelOmega ? 4
                                                             : 0;
            HIP_TRY(c, launch_stokes_root_check(kind, c->n_sl, c->sl_rec.as<float>(), ki.rec_sl,
                                                c->stk->X.as<double>(), M, part, s));
            HIP_TRY(c, launch_stokes_root_check(3, c->n_dl, c->dl_rec.as<float>(), ki.rec_dl,
                                                c->stk->X.as<double>(), M, part + size_t(nch_sl) * (3 * M + 3), s));
            HIP_TRY(c, launch_stokes_far_forces(nch_sl + nch_dl, c->stk->Q.as<double>(), M, part,
                                                c->stk_F.as<double>(), c->stk_F.as<double>() + 3 * M + 3, s));
        }
        HIP_TRY(c, hipEventRecord(ev[ne++], s));              // 5 S2L + periodic
        for (int l = c->lmin_dn; l <= t.depth; ++l) {
            const L2LLevel &ll = c->l2l[l];
            L2LArgs la;
            la.ops = o.l2l_cc.as<double>();
            la.M = o.M;
            la.blocks = at<int4>(c, ll.blocks);
            la.pairs = at<int2>(c, ll.pairs);
            la.delta = at<double>(c, ll.delta);
            la.chk = dnchk;
            HIP_TRY(c, launch_l2l_check(ll.nblocks, nc, la, s));
            st = run_pinv(c, c->dnpinv[l], o.dc2de.as<double>(), dnchk, dndens, s);
            if (st != STKFMM_OK) return st;
        }
        HIP_TRY(c, hipEventRecord(ev[ne++], s));              // 6 downward
        L2TArgs a;
        a.tasks = at<int4>(c, c->a_l2t_tasks);
        a.chunks = at<int4>(c, c->a_chunks);
        a.trg = c->trg_rec.as<float>();
        a.geom = at<double4>(c, c->a_geom);
        a.ent = at<int2>(c, c->a_l2t_ent);
        a.grid = o.grid.as<float>();
        a.up_dens = updens;
        a.dn_dens = dndens;
        a.M = o.M;
        a.Mp = o.Mp;
        a.alpha_in = kAlphaIn;
        a.alpha_out = kAlphaOut;
        a.part = c->far_part.as<double>();
        HIP_TRY(c, launch_l2t(c->kernel, c->n_l2t_tasks, a, s));
        HIP_TRY(c, hipEventRecord(ev[ne++], s));              // 7 L2T
    }
    if (c->overlap) HIP_TRY(c, hipStreamWaitEvent(s, ev[21], 0));
    HIP_TRY(c, hipEventRecord(ev[ne++], s));
    {
        CombineArgs a;
        a.chunks = at<int4>(c, c->a_chunks);
        a.chunk_tasks = at<int4>(c, c->a_chunk_tasks);
        a.near = c->near_part.as<double>();
        a.far = c->far_part.as<double>();
        a.perm = at<int32_t>(c, c->a_perm_trg);
        a.nacc = ki.kt_acc;
        a.kt = ki.k_trg;
        a.map = combine_map(c->kernel, c->box_len);
        a.out = trg_val;
        HIP_TRY(c, launch_combine(c->nchunks, a, s));
        if (pstokes) {
            // far images (each output with its power of 1/L)
            const double L = c->box_len;
            const int mode = c->kernel == kRPY ? 1 : c->kernel == kPVel ? 2 : c->kernel == kPVelGrad ? 3
                           : c->kernel == kPVelLaplacian ? 4 : c->kernel == kTraction ? 5
                           : c->kernel == kStokesRegVelOmega ? 6 : 0;
            const int M = c->stk->M;
            const double *V = c->stk_F.as<double>();    // check flow [3M], flux moment [3], forces [3M]
            HIP_TRY(c, launch_stokes_far_targets(c->n_trg, c->trg_rec.as<float>(), at<int32_t>(c, c->a_perm_trg),
                                                 mode, V + 3 * M + 3, c->stk->Z.as<double>(), M, 1.0 / L, V + 3 * M,
                                                 trg_val, s));
        }
    }
    HIP_TRY(c, hipEventRecord(ev[ne++], s));                  // end
    HIP_TRY(c, hipStreamSynchronize(s));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], ev[ne - 1]));
    c->t_run_ms = ms;
    std::memset(c->stage_ms, 0, sizeof(c->stage_ms));
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], c->overlap ? ev[1] : ev[20]));
    c->stage_ms[0] = ms;
    if (far) {
        for (int i = 0; i < 6; ++i) {   // S2M, upward, M2L, S2L(+periodic), downward, L2T
            HIP_TRY(c, hipEventElapsedTime(&ms, ev[1 + i], ev[2 + i]));
            c->stage_ms[1 + i] = ms;
        }
    }
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[20], ev[21]));
    c->stage_ms[7] = ms;
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[ne - 2], ev[ne - 1]));
    c->stage_ms[8] = ms;
    if (m2l_timed) {
        HIP_TRY(c, hipEventElapsedTime(&ms, ev[22], ev[23]));
        c->stage_ms[9] = ms;
    }
    return STKFMM_OK;
}

__global__ void gather_rows(const double *__restrict__ src, const int32_t *__restrict__ idx, int n, int w,
                            double *__restrict__ dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * w) return;
    dst[i] = src[int64_t(idx[i / w]) * w + i % w];
}

// Relative L2 error, per output field (the largest is returned), of the
// last run's result at up to 256 evenly spaced targets against the FP64
// direct sum on the GPU.
stkfmm_status sampled_error(stkfmm_ctx *c, const double *sl_val, const double *dl_val, const double *trg_val,
                            void *stream, double *err) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const KernelInfo &ki = kInfo[c->kernel];
    const int S = int(std::min<int64_t>(256, c->n_trg)), kt = ki.k_trg;
    std::vector<int32_t> idx(S);
    for (int k = 0; k < S; ++k) idx[k] = c->tree.perm_trg[size_t((int64_t(k) * c->n_trg) / S)];
    HIP_TRY(c, c->vbuf[0].ensure(S * sizeof(int32_t)));
    HIP_TRY(c, c->vbuf[1].ensure(size_t(S) * kt * sizeof(double)));
    HIP_TRY(c, c->vbuf[2].ensure(size_t(S) * 3 * sizeof(double)));
    HIP_TRY(c, c->vbuf[3].ensure(size_t(S) * kt * sizeof(double)));
    HIP_TRY(c, hipMemcpyAsync(c->vbuf[0].p, idx.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_rows, dim3((S * kt + 255) / 256), dim3(256), 0, s, trg_val, c->vbuf[0].as<int32_t>(), S,
                       kt, c->vbuf[1].as<double>());
    hipLaunchKernelGGL(gather_rows, dim3((S * 3 + 255) / 256), dim3(256), 0, s, c->coords[2].as<double>(),
                       c->vbuf[0].as<int32_t>(), S, 3, c->vbuf[2].as<double>());
    HIP_TRY(c, hipGetLastError());
    DirectArgs a;
    a.n_sl = c->n_sl;
    a.n_dl = c->n_dl;
    a.n_trg = S;
    a.sl = c->coords[0].as<double>();
    a.sl_val = sl_val;
    a.dl = c->coords[1].as<double>();
    a.dl_val = dl_val;
    a.trg = c->vbuf[2].as<double>();
    a.k_sl = ki.k_sl;
    a.k_dl = ki.k_dl;
    a.k_trg = kt;
    a.out = c->vbuf[3].as<double>();
    a.slices = direct_f64_slices(S, std::max(c->n_sl, c->n_dl));
    HIP_TRY(c, c->direct_work.ensure(std::max<size_t>(1, size_t(a.slices) * S * kt) * sizeof(double)));
    a.work = c->direct_work.as<double>();
    HIP_TRY(c, launch_direct_f64(c->kernel, a, s));
    std::vector<double> got(size_t(S) * kt), ref(size_t(S) * kt);
    HIP_TRY(c, hipMemcpyAsync(got.data(), c->vbuf[1].p, got.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(ref.data(), c->vbuf[3].p, ref.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    // output fields: (u), (u, lap u), (phi, grad phi), (p, u), (sigma), (u, omega),
    // (phi, grad phi, Hessian), (p, u, grad p, grad u), (p, u, lap u), (phi, grad phi, Hessian)
    static const int fields[kNumKernels][5] = {{0, 1, 4, 4, 4},  {0, 3, 3, 3, 3},  {0, 3, 6, 6, 6},
                                               {0, 1, 4, 4, 4},  {0, 9, 9, 9, 9},  {0, 3, 3, 3, 3},
                                               {0, 3, 6, 6, 6},  {0, 1, 4, 10, 10}, {0, 1, 4, 7, 16},
                                               {0, 1, 4, 7, 7},  {0, 1, 4, 10, 10}};
    const int *fb = fields[c->kernel];
    double worst = 0.0;
    for (int f = 0; f < 4; ++f) {
        const int a0 = fb[f], a1 = fb[f + 1];
        if (a1 <= a0) continue;
        double num = 0, den = 0;
        for (int k = 0; k < S; ++k)
            for (int j = a0; j < a1; ++j) {
                double d = got[size_t(k) * kt + j] - ref[size_t(k) * kt + j];
                num += d * d;
                den += ref[size_t(k) * kt + j] * ref[size_t(k) * kt + j];
            }
        worst = std::max(worst, den > 0 ? std::sqrt(num / den) : std::sqrt(num));
    }
    *err = worst;
    return STKFMM_OK;
}

}  // namespace

extern "C" {

stkfmm_status stkfmm_run(stkfmm_ctx *c, const double *sl_val, const double *dl_val, double *trg_val, void *stream) {
    if (c && c->planned && c->bc == STKFMM_BC_WALL) return wall_run(c, sl_val, dl_val, trg_val, stream);
    stkfmm_status st = run_pass(c, sl_val, dl_val, trg_val, stream);
    if (st != STKFMM_OK || !c->learned || c->validated || c->n_trg == 0) return st;
    // learned plan: one accuracy check against the FP64 direct sum on sampled
    // targets; above the tolerance, fall back to the fixed p = 10, leaf_cap = 2000 plan
    double err = 0.0;
    st = sampled_error(c, sl_val, dl_val, trg_val, stream, &err);
    if (st != STKFMM_OK) return st;
    c->validated = true;
    c->sampled_err = err;
    if (err <= c->tol) return STKFMM_OK;
    int hp[4], hc[4];
    std::memcpy(hp, c->p_hist, sizeof hp);
    std::memcpy(hc, c->cap_hist, sizeof hc);
    st = stkfmm_set_points(c, stkfmm_kernel(c->kernel), stkfmm_bc(c->bc), c->n_sl, c->coords[0].as<double>(), c->n_dl,
                           c->coords[1].as<double>(), c->n_trg, c->coords[2].as<double>(), 10, kReferenceCap, stream);
    if (st != STKFMM_OK) return st;
    st = run_pass(c, sl_val, dl_val, trg_val, stream);
    if (st != STKFMM_OK) return st;
    // c->coords still hold the caller's points: the fixed plan does not touch them
    st = sampled_error(c, sl_val, dl_val, trg_val, stream, &err);
    if (st != STKFMM_OK) return st;
    c->learned = true;
    c->validated = true;
    c->fell_back = true;
    c->sampled_err = err;
    std::memcpy(c->p_hist, hp, sizeof hp);
    std::memcpy(c->cap_hist, hc, sizeof hc);
    if (err > c->tol) return fail(c, STKFMM_E_ACCURACY, "sampled error above tol after the fixed-order fallback");
    return STKFMM_OK;
}

stkfmm_status stkfmm_set_predictor(stkfmm_ctx *c, const float *params, int n) {
    if (!c) return STKFMM_E_ARG;
    const int np = stkfmm_mlp_nparam();
    if (!params || n != np + 16) return fail(c, STKFMM_E_ARG, "predictor needs stkfmm_mlp_nparam() + 16 floats");
    for (int k = 0; k < 16; ++k)
        if (!(params[np + k] >= 0) || !std::isfinite(params[np + k]))
            return fail(c, STKFMM_E_ARG, "order table entries must be finite and >= 0");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, c->predictor.ensure(size_t(np) * sizeof(float)));
    HIP_TRY(c, hipMemcpy(c->predictor.p, params, size_t(np) * sizeof(float), hipMemcpyHostToDevice));
    std::memcpy(c->order_table, params + np, sizeof(c->order_table));
    c->has_predictor = true;
    return STKFMM_OK;
}

stkfmm_status stkfmm_get_learned(const stkfmm_ctx *c, int64_t info[12], double *sampled_err) {
    if (!c || !info) return STKFMM_E_ARG;
    info[0] = c->learned;
    info[1] = c->p;
    info[2] = c->fell_back;
    info[3] = c->validated;
    for (int k = 0; k < 4; ++k) {
        info[4 + k] = c->p_hist[k];
        info[8 + k] = c->cap_hist[k];
    }
    if (sampled_err) *sampled_err = c->sampled_err;
    return STKFMM_OK;
}

stkfmm_status stkfmm_get_leaf_features(stkfmm_ctx *c, float *features, int32_t *leaf_of_target, int64_t *n_leaf) {
    if (!c || !n_leaf) return STKFMM_E_ARG;
    if (!c->planned) return fail(c, STKFMM_E_STATE, "no plan");
    if (c->bc == STKFMM_BC_WALL) return fail(c, STKFMM_E_UNSUPPORTED, "wall plans have no single tree");
    const Tree &t = c->tree;
    *n_leaf = int64_t(t.leaves.size());
    if (features) {
        if (!c->hcoords_valid) {
            const double *src[3] = {c->coords[0].as<double>(), c->coords[1].as<double>(), c->coords[2].as<double>()};
            const int64_t cnt[3] = {c->n_sl, c->n_dl, c->n_trg};
            stkfmm_status st = copy_coords(c, src, cnt, bc_axes(c->bc), false, c->hcoords, nullptr);
            if (st != STKFMM_OK) return st;
            c->hcoords_valid = true;
        }
        std::vector<float> f;
        leaf_features(t, c->hcoords[0].data(), c->hcoords[1].data(), c->hcoords[2].data(), c->tol, f);
        std::memcpy(features, f.data(), f.size() * sizeof(float));
    }
    if (leaf_of_target)
        for (size_t i = 0; i < t.leaves.size(); ++i) {
            const Box &B = t.boxes[t.leaves[i]];
            for (int64_t j = B.trg[0]; j < B.trg[1]; ++j) leaf_of_target[t.perm_trg[j]] = int32_t(i);
        }
    return STKFMM_OK;
}

stkfmm_status stkfmm_get_plan_work(stkfmm_ctx *c, double *work) {
    if (!c || !work) return STKFMM_E_ARG;
    if (!c->planned) return fail(c, STKFMM_E_STATE, "no plan");
    if (c->bc == STKFMM_BC_WALL) return fail(c, STKFMM_E_UNSUPPORTED, "wall plans have no single tree");
    const Tree &t = c->tree;
    std::vector<double> w(size_t(c->n_trg) * 5, 0.0);      // sorted target order
    for (size_t b = 0; b < t.boxes.size(); ++b) {
        const Box &B = t.boxes[b];
        const int64_t n = B.trg[1] - B.trg[0];
        if (n <= 0) continue;
        for (int k = 0; k < 5; ++k) {
            const double share = c->box_work[b][k] / double(n);
            if (share == 0.0) continue;
            for (int64_t i = B.trg[0]; i < B.trg[1]; ++i) w[size_t(i) * 5 + k] += share;
        }
    }
    for (int64_t i = 0; i < c->n_trg; ++i)
        std::memcpy(work + size_t(t.perm_trg[i]) * 5, &w[size_t(i) * 5], 5 * sizeof(double));
    return STKFMM_OK;
}

stkfmm_status stkfmm_evaluate(stkfmm_ctx *c, stkfmm_kernel kernel, stkfmm_bc bc, int64_t n_sl, const double *sl_xyz,
                              const double *sl_val, int64_t n_dl, const double *dl_xyz, const double *dl_val,
                              int64_t n_trg, const double *trg_xyz, double *trg_val, int p, int leaf_cap,
                              void *stream) {
    stkfmm_status st = stkfmm_set_points(c, kernel, bc, n_sl, sl_xyz, n_dl, dl_xyz, n_trg, trg_xyz, p, leaf_cap,
                                         stream);
    if (st != STKFMM_OK) return st;
    return stkfmm_run(c, sl_val, dl_val, trg_val, stream);
}

stkfmm_status stkfmm_direct(stkfmm_ctx *c, stkfmm_kernel kernel, int64_t n_sl, const double *sl_xyz,
                            const double *sl_val, int64_t n_dl, const double *dl_xyz, const double *dl_val,
                            int64_t n_trg, const double *trg_xyz, double *trg_val, void *stream) {
    if (!c) return STKFMM_E_ARG;
    DirectArgs a;
    const stkfmm_status st =
        direct_args(c, kernel, n_sl, sl_xyz, sl_val, n_dl, dl_xyz, dl_val, n_trg, trg_xyz, trg_val, a);
    if (st != STKFMM_OK) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    if (a.slices > 1) {
        HIP_TRY(c, c->direct_work.ensure(size_t(a.slices) * size_t(n_trg) * a.k_trg * sizeof(double)));
        a.work = c->direct_work.as<double>();
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(c, launch_direct_f64(kernel, a, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return STKFMM_OK;
}

stkfmm_status stkfmm_direct_noalloc(stkfmm_ctx *c, stkfmm_kernel kernel, int64_t n_sl, const double *sl_xyz,
                                    const double *sl_val, int64_t n_dl, const double *dl_xyz,
                                    const double *dl_val, int64_t n_trg, const double *trg_xyz, double *trg_val,
                                    void *stream) {
    if (!c) return STKFMM_E_ARG;
    DirectArgs a;
    const stkfmm_status st =
        direct_args(c, kernel, n_sl, sl_xyz, sl_val, n_dl, dl_xyz, dl_val, n_trg, trg_xyz, trg_val, a);
    if (st != STKFMM_OK) return st;
    if (a.slices > 1) {
        // the same source slices as stkfmm_direct (identical sums); their
        // partial sums must fit the static scratch
        const int64_t need = int64_t(a.slices) * n_trg * a.k_trg;
        if (need > kDirectScratchDoubles)
            return fail(c, STKFMM_E_ARG,
                        "stkfmm_direct_noalloc: " + std::to_string(a.slices) + " source slices x " +
                            std::to_string(n_trg) + " targets x " + std::to_string(a.k_trg) +
                            " values need " + std::to_string(need) + " doubles of workspace, above its " +
                            std::to_string(kDirectScratchDoubles) + "-double static scratch");
        a.work = scratch_ptr(c->device);
        if (!a.work) return fail(c, STKFMM_E_DEVICE, "stkfmm_direct_noalloc: device scratch not resolved");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(c, launch_direct_f64(kernel, a, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return STKFMM_OK;
}

}  // extern "C"
