// Adaptive octree and U/V/W/X interaction lists built on the GPU.
//
// The tree and lists are those of the host builder (same splitting rule,
// box order, list definitions, pruning and entry order; Sec. II defers the
// lists to the KIFMM literature):
//   * Morton keys of the normalised coordinates (21 bits per dimension,
//     octant digit (x << 2) | (y << 1) | z), sorted stably with the input
//     index as payload by an 8-bit LSD radix sort;
//   * refinement level by level: a box splits while it holds more than its
//     capacity of targets, SL or DL sources (and is above the deepest
//     level); its non-empty children follow in octant order, so every level
//     lists its boxes in Morton order of their anchors (which the list
//     kernels use to find a box by binary search);
//   * U, W (per leaf), V (per box) and X (the dual of W) per box, entries
//     ordered by (box, periodic shift), entries without sources and lists of
//     boxes without targets dropped.
// The host finishes the tree from the copied box table and lists (leaf
// list, level starts, V offsets, local-expansion flags, pair counts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace kafmm {

namespace {

// ------------------------------------------------------------------ device scratch
struct DevArr {
    void *p = nullptr;
    size_t bytes = 0;
    DevArr() = default;
    DevArr(const DevArr &) = delete;
    DevArr &operator=(const DevArr &) = delete;
    ~DevArr() {
        if (p) (void)hipFree(p);
    }
    hipError_t ensure(size_t n) {
        if (n <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, std::max<size_t>(n, 256));
        if (e == hipSuccess) bytes = std::max<size_t>(n, 256);
        return e;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

#define TRY(expr)                                                                      \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return std::string("GPU tree build: ") + #expr + ": " + \
                                     hipGetErrorString(e_);                            \
    } while (0)

inline int nblk(int64_t n, int b) { return int((n + b - 1) / b); }

// ------------------------------------------------------------------ Morton keys
__device__ __forceinline__ uint64_t spread_bits(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

__device__ __forceinline__ uint32_t cell_of(double u) {
    const double scale = double(1u << kKeyBits);
    double g = floor(u * scale);
    if (g < 0) g = 0;
    if (g > scale - 1) g = scale - 1;
    return uint32_t(g);
}

struct KeyArgs {
    int64_t n;
    const double *xyz;       // user coordinates [n][3]
    double origin[3], len;
    int pmask;               // bit k: axis k periodic (coordinates wrapped)
    uint64_t *key;
    int32_t *idx;
};

__global__ void keys_kernel(KeyArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    uint32_t g[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double u = (a.xyz[3 * i + k] - a.origin[k]) / a.len;
        if ((a.pmask >> k) & 1) {
            u -= floor(u);
            if (u >= 1.0) u = 0.0;
        }
        g[k] = cell_of(u);
    }
    a.key[i] = (spread_bits(g[0]) << 2) | (spread_bits(g[1]) << 1) | spread_bits(g[2]);
    a.idx[i] = int32_t(i);
}

// ------------------------------------------------------------------ exclusive scan (uint32)
constexpr int kScanThreads = 256, kScanPer = 8, kScanItems = kScanThreads * kScanPer;

// In place over [n]; block totals to sums[nblk].
__global__ __launch_bounds__(kScanThreads) void scan_block_kernel(uint32_t *d, int64_t n, uint32_t *sums) {
    __shared__ uint32_t s[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * kScanItems + int64_t(tid) * kScanPer;
    uint32_t v[kScanPer], tot = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = base + j < n ? d[base + j] : 0u;
        tot += v[j];
    }
    s[tid] = tot;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t add = tid >= off ? s[tid - off] : 0u;
        __syncthreads();
        s[tid] += add;
        __syncthreads();
    }
    uint32_t run = s[tid] - tot;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < n) d[base + j] = run;
        run += v[j];
    }
    if (tid == kScanThreads - 1) sums[blockIdx.x] = s[tid];
}

__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(uint32_t *d, int64_t n, const uint32_t *sums) {
    const int64_t i = int64_t(blockIdx.x) * kScanItems + threadIdx.x;
    const uint32_t add = sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t k = i + int64_t(j) * kScanThreads;
        if (k < n) d[k] += add;
    }
}

// Scratch of a scan of n items: the block sums of every recursion level.
size_t scan_scratch(int64_t n) {
    size_t tot = 0;
    while (n > 1) {
        n = (n + kScanItems - 1) / kScanItems;
        tot += size_t(n);
    }
    return tot + 1;
}

hipError_t scan_exclusive(uint32_t *d, int64_t n, uint32_t *scratch, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nb = nblk(n, kScanItems);
    hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(kScanThreads), 0, s, d, n, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    e = scan_exclusive(scratch, nb, scratch + nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(kScanThreads), 0, s, d, n, scratch);
    return hipGetLastError();
}

// ------------------------------------------------------------------ stable LSD radix sort
constexpr int kSortThreads = 256, kSortTiles = 16, kSortItems = kSortThreads * kSortTiles;
constexpr int kRadix = 256;

// digit counts of each block: hist[digit * nb + block]
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(int64_t n, const uint64_t *key, int shift,
                                                                  int nb, uint32_t *hist) {
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortItems;
    for (int t = 0; t < kSortTiles; ++t) {
        const int64_t i = base + int64_t(t) * kSortThreads + tid;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[int64_t(tid) * nb + blockIdx.x] = h[tid];
}

// Each item goes to ofs[digit, block] + (items of its digit before it in the
// block): lanes of a wave find their equal-digit peers with eight ballots,
// waves are ordered through per-wave digit counts in LDS, tiles in order.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(int64_t n, const uint64_t *kin,
                                                                     const int32_t *vin, uint64_t *kout,
                                                                     int32_t *vout, int shift, int nb,
                                                                     const uint32_t *ofs) {
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t wh[kSortThreads / 64][kRadix];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    run[tid] = ofs[int64_t(tid) * nb + blockIdx.x];
    const int64_t base = int64_t(blockIdx.x) * kSortItems;
    for (int t = 0; t < kSortTiles; ++t) {
        const int64_t i = base + int64_t(t) * kSortThreads + tid;
        const bool valid = i < n;
        const uint64_t k = valid ? kin[i] : 0ull;
        const int32_t v = valid ? vin[i] : 0;
        const int d = int((k >> shift) & (kRadix - 1));
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; ++w) wh[w][tid] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int lower = __popcll(peers & below);
        if (valid && lower == 0) wh[wave][d] = uint32_t(__popcll(peers));
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + uint32_t(lower);
            for (int w = 0; w < wave; ++w) pos += wh[w][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; ++w) add += wh[w][tid];
        run[tid] += add;
    }
}

struct SortBufs {
    DevArr k2, v2, hist, scan;
};

// Sorts (key, val) of n items stably by the low `bits` bits of key, in place.
hipError_t radix_sort(uint64_t *key, int32_t *val, int64_t n, int bits, SortBufs &b, hipStream_t s) {
    if (n <= 1) return hipSuccess;
    const int nb = nblk(n, kSortItems);
    hipError_t e;
    if ((e = b.k2.ensure(size_t(n) * 8)) != hipSuccess) return e;
    if ((e = b.v2.ensure(size_t(n) * 4)) != hipSuccess) return e;
    if ((e = b.hist.ensure(size_t(kRadix) * nb * 4)) != hipSuccess) return e;
    if ((e = b.scan.ensure(scan_scratch(int64_t(kRadix) * nb) * 4)) != hipSuccess) return e;
    uint64_t *ka = key, *kb = b.k2.as<uint64_t>();
    int32_t *va = val, *vb = b.v2.as<int32_t>();
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nb), dim3(kSortThreads), 0, s, n, ka, shift, nb,
                           b.hist.as<uint32_t>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan_exclusive(b.hist.as<uint32_t>(), int64_t(kRadix) * nb, b.scan.as<uint32_t>(), s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nb), dim3(kSortThreads), 0, s, n, ka, va, kb, vb, shift, nb,
                           b.hist.as<uint32_t>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != key) {
        if ((e = hipMemcpyAsync(key, ka, size_t(n) * 8, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(val, va, size_t(n) * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ refinement
struct GBox {
    int32_t level, anchor[3], parent, cap, leaf;
    int32_t r[6];            // sl, dl, trg ranges in the sorted orders
    int32_t child[8];
};

__device__ __forceinline__ int32_t gb_nsrc(const GBox &b) { return (b.r[1] - b.r[0]) + (b.r[3] - b.r[2]); }
__device__ __forceinline__ int32_t gb_ntrg(const GBox &b) { return b.r[5] - b.r[4]; }

__device__ __forceinline__ uint64_t hash_of(int level, int32_t ax, int32_t ay, int32_t az) {
    return (uint64_t(level) << 60) | (uint64_t(ax) << 40) | (uint64_t(ay) << 20) | uint64_t(az);
}

struct SplitArgs {
    int b0, nbl;
    const GBox *box;
    const uint64_t *key[3];
    int32_t *cand;           // [nbl][8][6] child ranges
    uint32_t *cnt;           // [nbl + 1] non-empty children of split boxes (last: 0)
};

__global__ void split_kernel(SplitArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > a.nbl) return;
    if (j == a.nbl) {
        a.cnt[j] = 0;
        return;
    }
    const GBox B = a.box[a.b0 + j];
    const int32_t c = max(max(B.r[1] - B.r[0], B.r[3] - B.r[2]), B.r[5] - B.r[4]);
    if (c <= B.cap || B.level >= kMaxLevel) {
        a.cnt[j] = 0;
        return;
    }
    const int shift = 3 * (kKeyBits - (B.level + 1));
    int32_t bound[3][9];
    for (int s = 0; s < 3; ++s) {
        const uint64_t *k = a.key[s];
        const int32_t lo = B.r[2 * s], hi = B.r[2 * s + 1];
        bound[s][0] = lo;
        bound[s][8] = hi;
        for (int o = 1; o < 8; ++o) {
            // first position in [lo, hi) whose octant digit is >= o
            int32_t l = bound[s][o - 1], h = hi;
            while (l < h) {
                const int32_t m = l + (h - l) / 2;
                if (int((k[m] >> shift) & 7) < o) l = m + 1;
                else h = m;
            }
            bound[s][o] = l;
        }
    }
    uint32_t n = 0;
    int32_t *cd = a.cand + int64_t(j) * 48;
    for (int o = 0; o < 8; ++o) {
        int32_t tot = 0;
        for (int s = 0; s < 3; ++s) {
            cd[6 * o + 2 * s] = bound[s][o];
            cd[6 * o + 2 * s + 1] = bound[s][o + 1];
            tot += bound[s][o + 1] - bound[s][o];
        }
        n += tot > 0;
    }
    a.cnt[j] = n;
}

struct EmitArgs {
    int b0, nbl, nstart;
    GBox *box;
    const int32_t *cand;
    const uint32_t *cnt_ofs;  // exclusive offsets of the children
    const uint32_t *cnt;      // non-empty children (0: not split)
    const uint64_t *cap_key;  // sorted box hashes with their own capacities
    const int32_t *cap_val;
    int ncap;
};

__global__ void emit_kernel(EmitArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.nbl || a.cnt[j] == 0) return;
    GBox &B = a.box[a.b0 + j];
    int pos = a.nstart + int(a.cnt_ofs[j]);
    const int32_t *cd = a.cand + int64_t(j) * 48;
    for (int o = 0; o < 8; ++o) {
        const int32_t *r = cd + 6 * o;
        if ((r[1] - r[0]) + (r[3] - r[2]) + (r[5] - r[4]) == 0) continue;
        GBox C;
        C.level = B.level + 1;
        C.anchor[0] = 2 * B.anchor[0] + ((o >> 2) & 1);
        C.anchor[1] = 2 * B.anchor[1] + ((o >> 1) & 1);
        C.anchor[2] = 2 * B.anchor[2] + (o & 1);
        C.parent = a.b0 + j;
        C.leaf = 1;
        for (int q = 0; q < 6; ++q) C.r[q] = r[q];
        for (int q = 0; q < 8; ++q) C.child[q] = -1;
        C.cap = B.cap;
        if (a.ncap > 0) {
            const uint64_t h = hash_of(C.level, C.anchor[0], C.anchor[1], C.anchor[2]);
            int l = 0, u = a.ncap;
            while (l < u) {
                const int m = (l + u) / 2;
                if (a.cap_key[m] < h) l = m + 1;
                else u = m;
            }
            if (l < a.ncap && a.cap_key[l] == h) C.cap = a.cap_val[l];
        }
        a.box[pos] = C;
        B.child[o] = pos;
        ++pos;
    }
    B.leaf = 0;
}

// ------------------------------------------------------------------ lists
constexpr int kLevels = kMaxLevel + 2;
constexpr int kStack = 192;

struct ListView {
    const GBox *box;
    const uint64_t *bkey;         // Morton key of each box's anchor at its level
    int level_start[kLevels + 1]; // boxes of level l: [level_start[l], level_start[l + 1])
    int depth;
    int pmask;               // bit k: axis k periodic
};

// an entry: (box << 5) | shift code, code = 9 (s0 + 1) + 3 (s1 + 1) + (s2 + 1);
// ordering the codes orders (box, shift) lexicographically
__device__ __forceinline__ uint64_t ent_of(int box, int s0, int s1, int s2) {
    return (uint64_t(box) << 5) | uint64_t(9 * (s0 + 1) + 3 * (s1 + 1) + (s2 + 1));
}
__device__ __forceinline__ int ent_box(uint64_t e) { return int(e >> 5); }
__device__ __forceinline__ void ent_shift(uint64_t e, int s[3]) {
    const int c = int(e & 31);
    s[0] = c / 9 - 1;
    s[1] = (c / 3) % 3 - 1;
    s[2] = c % 3 - 1;
}

__global__ void box_keys_kernel(int nb, const GBox *box, uint64_t *bkey) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const GBox B = box[b];
    bkey[b] = (spread_bits(uint32_t(B.anchor[0])) << 2) | (spread_bits(uint32_t(B.anchor[1])) << 1) |
              spread_bits(uint32_t(B.anchor[2]));
}

__device__ int find_box(const ListView &v, int level, const int32_t c[3]) {
    if (level > v.depth) return -1;
    const uint64_t k = (spread_bits(uint32_t(c[0])) << 2) | (spread_bits(uint32_t(c[1])) << 1) |
                       spread_bits(uint32_t(c[2]));
    int l = v.level_start[level], h = v.level_start[level + 1];
    while (l < h) {
        const int m = l + (h - l) / 2;
        if (v.bkey[m] < k) l = m + 1;
        else h = m;
    }
    return (l < v.level_start[level + 1] && v.bkey[l] == k) ? l : -1;
}

// same-level adjacent boxes (periodic images), the box itself included
__device__ int colleagues(const ListView &v, int b, uint64_t out[27]) {
    const GBox B = v.box[b];
    const int32_t n = 1 << B.level;
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int d[3] = {dx, dy, dz};
                int32_t c[3];
                int s[3] = {0, 0, 0};
                bool ok = true;
                for (int k = 0; k < 3; ++k) {
                    int32_t w = B.anchor[k] + d[k];
                    if ((v.pmask >> k) & 1) {
                        const int32_t q = w >= 0 ? w / n : -((-w + n - 1) / n);
                        w -= q * n;
                        s[k] = q;
                    } else if (w < 0 || w >= n) {
                        ok = false;
                    }
                    c[k] = w;
                }
                if (!ok) continue;
                const int f = find_box(v, B.level, c);
                if (f >= 0) out[cnt++] = ent_of(f, s[0], s[1], s[2]);
            }
    return cnt;
}

// closed cubes of the image (a, shift) and of box b intersect
__device__ bool adjacent(const ListView &v, int a, const int s[3], int b) {
    const GBox &A = v.box[a], &B = v.box[b];
    const int D = max(A.level, B.level);
    for (int k = 0; k < 3; ++k) {
        const int64_t loA = (int64_t(A.anchor[k]) + int64_t(s[k]) * (int64_t(1) << A.level)) << (D - A.level);
        const int64_t hiA = loA + (int64_t(1) << (D - A.level));
        const int64_t loB = int64_t(B.anchor[k]) << (D - B.level);
        const int64_t hiB = loB + (int64_t(1) << (D - B.level));
        if (loA > hiB || loB > hiA) return false;
    }
    return true;
}

__device__ void sort_entries(uint64_t *e, int n) {
    for (int i = 1; i < n; ++i) {
        const uint64_t x = e[i];
        int j = i - 1;
        while (j >= 0 && e[j] > x) {
            e[j + 1] = e[j];
            --j;
        }
        e[j + 1] = x;
    }
}

struct VArgs {
    ListView v;
    int nb;
    uint32_t *cnt;            // [nb + 1]
    const uint32_t *ofs;      // fill pass: offsets (else null)
    uint64_t *ent;
};

// V(b): children of the colleagues of b's parent that are not adjacent to b
__global__ void v_list_kernel(VArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > a.nb) return;
    if (b == a.nb || b == 0 || gb_ntrg(a.v.box[b]) == 0) {
        if (!a.ofs) a.cnt[b] = 0;
        return;
    }
    uint64_t pc[27];
    const int np = colleagues(a.v, a.v.box[b].parent, pc);
    sort_entries(pc, np);
    uint64_t *out = a.ofs ? a.ent + a.ofs[b] : nullptr;
    uint32_t n = 0;
    for (int i = 0; i < np; ++i) {
        int s[3];
        ent_shift(pc[i], s);
        const GBox &C = a.v.box[ent_box(pc[i])];
        for (int o = 0; o < 8; ++o) {
            const int ch = C.child[o];
            if (ch < 0 || adjacent(a.v, ch, s, b) || gb_nsrc(a.v.box[ch]) == 0) continue;
            if (out) out[n] = ent_of(ch, s[0], s[1], s[2]);
            ++n;
        }
    }
    if (out) sort_entries(out, int(n));
    else a.cnt[b] = n;
}

struct UWArgs {
    ListView v;
    int nleaf;
    const int32_t *leaves;
    uint32_t *total;          // count pass: U, W, X entries
    uint32_t *cursor;         // fill pass: next free position of U, W, X
    uint64_t *ukey, *wkey, *xkey;
    int *overflow;
};

// One thread per (leaf B, slot): slots 0..26 take B's colleague of that
// index, slot 27 the coarser levels.
//   U(B): leaves adjacent to B at any level -- coarser ones are the leaf
//   colleagues of B's ancestors adjacent to B, the others are reached by
//   descending from B's colleagues through adjacent boxes;
//   W(B): descendants of B's colleagues not adjacent to B whose parent is;
//   X: each W entry A of B with sources in B and targets in A gives A the
//   entry B.
// Entries are keyed (owner << 30) | (box << 5) | shift code and written at
// positions claimed atomically; sorting the keys afterwards gives every list
// in (box, shift) order, independent of the claim order.
template <bool FILL>
__global__ void uw_list_kernel(UWArgs a) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= int64_t(a.nleaf) * 28) return;
    const int slot = int(g % 28);
    const int b = a.leaves[g / 28];
    const ListView &v = a.v;
    const GBox B = v.box[b];
    const bool keep = gb_ntrg(B) > 0, src_b = gb_nsrc(B) > 0;
    uint32_t n[3] = {0, 0, 0};
    auto emit_u = [&](uint64_t e) {
        if (FILL) a.ukey[atomicAdd(&a.cursor[0], 1u)] = (uint64_t(b) << 30) | e;
        else ++n[0];
    };
    auto emit_w = [&](uint64_t e) {
        if (FILL) a.wkey[atomicAdd(&a.cursor[1], 1u)] = (uint64_t(b) << 30) | e;
        else ++n[1];
    };
    auto emit_x = [&](int A, const int s[3]) {
        if (FILL)
            a.xkey[atomicAdd(&a.cursor[2], 1u)] = (uint64_t(A) << 30) | (uint64_t(b) << 5) |
                                                  uint64_t(9 * (1 - s[0]) + 3 * (1 - s[1]) + (1 - s[2]));
        else ++n[2];
    };
    uint64_t col[27];
    int s[3];
    if (slot == 27) {
        for (int p = B.parent; p >= 0; p = v.box[p].parent) {
            const int nc = colleagues(v, p, col);
            for (int k = 0; k < nc; ++k) {
                const int A = ent_box(col[k]);
                if (!v.box[A].leaf) continue;
                ent_shift(col[k], s);
                if (adjacent(v, A, s, b) && keep && gb_nsrc(v.box[A]) > 0) emit_u(col[k]);
            }
        }
    } else {
        const int nc = colleagues(v, b, col);
        if (slot < nc) {
            const int C = ent_box(col[slot]);
            ent_shift(col[slot], s);
            const bool self = C == b && s[0] == 0 && s[1] == 0 && s[2] == 0;
            if (self || v.box[C].leaf) {
                if (keep && gb_nsrc(v.box[C]) > 0) emit_u(col[slot]);
            } else {
                uint64_t stack[kStack];
                int top = 0;
                stack[top++] = col[slot];
                while (top > 0) {
                    const GBox &Dx = v.box[ent_box(stack[--top])];
                    for (int o = 0; o < 8; ++o) {
                        const int ch = Dx.child[o];
                        if (ch < 0) continue;
                        const uint64_t e = ent_of(ch, s[0], s[1], s[2]);
                        const GBox &Ch = v.box[ch];
                        if (adjacent(v, ch, s, b)) {
                            if (Ch.leaf) {
                                if (keep && gb_nsrc(Ch) > 0) emit_u(e);
                            } else if (top < kStack) {
                                stack[top++] = e;
                            } else {
                                atomicExch(a.overflow, 1);
                            }
                        } else {
                            if (keep && gb_nsrc(Ch) > 0) emit_w(e);
                            if (src_b && gb_ntrg(Ch) > 0) emit_x(ch, s);
                        }
                    }
                }
            }
        }
    }
    if (!FILL)
        for (int q = 0; q < 3; ++q)
            if (n[q]) atomicAdd(&a.total[q], n[q]);
}

// list lengths per owning box from the sorted keys, and the entries (box, shift)
__global__ void key_count_kernel(int64_t n, const uint64_t *key, uint32_t *cnt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    atomicAdd(&cnt[key[i] >> 30], 1u);
}

__global__ void key_entries_kernel(int64_t n, const uint64_t *key, uint64_t *ent) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ent[i] = key[i] & ((uint64_t(1) << 30) - 1);
}

// flags[0]: some coordinate is not finite; flags[1]: some coordinate of an
// open (non-periodic) axis lies outside [origin, origin + len), with the
// host's expression
__global__ void check_points_kernel(int64_t n3, const double *xyz, double ox, double oy, double oz, double len,
                                    int pmask, uint32_t *flags) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const double v = xyz[i];
    if (!isfinite(v)) {
        atomicOr(&flags[0], 1u);
        return;
    }
    const int k = int(i % 3);
    if ((pmask >> k) & 1) return;
    const double u = (v - (k == 0 ? ox : k == 1 ? oy : oz)) / len;
    if (!(u >= 0.0 && u < 1.0)) atomicOr(&flags[1], 1u);
}

__global__ void fill_u32(uint32_t *d, int64_t n, uint32_t v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

}  // namespace

std::string check_points_gpu(const double *xyz, int64_t n, const double origin[3], double box_len, int pmask,
                             bool *nonfinite, bool *outside, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    *nonfinite = *outside = false;
    if (n <= 0) return "";
    DevArr flags;
    TRY(flags.ensure(8));
    hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, s, flags.as<uint32_t>(), int64_t(2), 0u);
    TRY(hipGetLastError());
    hipLaunchKernelGGL(check_points_kernel, dim3(nblk(3 * n, 256)), dim3(256), 0, s, 3 * n, xyz, origin[0], origin[1],
                       origin[2], box_len, pmask, flags.as<uint32_t>());
    TRY(hipGetLastError());
    uint32_t h[2] = {0, 0};
    TRY(hipMemcpyAsync(h, flags.p, 8, hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    *nonfinite = h[0] != 0;
    *outside = h[1] != 0;
    return "";
}

std::string build_tree_gpu(const double *const xyz[3], const int64_t n[3], const double origin[3], double box_len,
                           int leaf_cap, int pmask, Tree &t,
                           const std::unordered_map<uint64_t, int> *leaf_caps, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    t = Tree();
    t.pmask = pmask;
    for (int k = 0; k < 3; ++k)
        if (n[k] > INT32_MAX / 2) return "GPU tree build: too many points";
    // ---------------------------------------------------------------- keys and sort
    DevArr key[3], perm[3];
    SortBufs sb;
    int same[3] = {0, 1, 2};   // sets given by the same array are sorted once
    if (xyz[1] == xyz[0] && n[1] == n[0]) same[1] = 0;
    if (xyz[2] == xyz[0] && n[2] == n[0]) same[2] = 0;
    else if (xyz[2] == xyz[1] && n[2] == n[1]) same[2] = same[1];
    for (int k = 0; k < 3; ++k) {
        if (same[k] != k) continue;
        TRY(key[k].ensure(std::max<int64_t>(n[k], 1) * 8));
        TRY(perm[k].ensure(std::max<int64_t>(n[k], 1) * 4));
        if (n[k] == 0) continue;
        KeyArgs ka{n[k], xyz[k], {origin[0], origin[1], origin[2]}, box_len, pmask,
                   key[k].as<uint64_t>(), perm[k].as<int32_t>()};
        hipLaunchKernelGGL(keys_kernel, dim3(nblk(n[k], 256)), dim3(256), 0, s, ka);
        TRY(hipGetLastError());
        TRY(radix_sort(key[k].as<uint64_t>(), perm[k].as<int32_t>(), n[k], 3 * kKeyBits, sb, s));
    }
    const uint64_t *kd[3];
    for (int k = 0; k < 3; ++k) kd[k] = key[same[k]].as<uint64_t>();
    std::vector<int32_t> *hp[3] = {&t.perm_sl, &t.perm_dl, &t.perm_trg};
    for (int k = 0; k < 3; ++k) {
        hp[k]->resize(n[k]);
        if (n[k] > 0)
            TRY(hipMemcpyAsync(hp[k]->data(), perm[same[k]].p, size_t(n[k]) * 4, hipMemcpyDeviceToHost, s));
    }
    // ---------------------------------------------------------------- refinement
    std::vector<uint64_t> ck;
    std::vector<int32_t> cv;
    if (leaf_caps) {
        std::vector<std::pair<uint64_t, int>> kv(leaf_caps->begin(), leaf_caps->end());
        std::sort(kv.begin(), kv.end());
        for (auto &q : kv) {
            ck.push_back(q.first);
            cv.push_back(q.second);
        }
    }
    DevArr capk, capv;
    TRY(capk.ensure(std::max<size_t>(ck.size(), 1) * 8));
    TRY(capv.ensure(std::max<size_t>(cv.size(), 1) * 4));
    if (!ck.empty()) {
        TRY(hipMemcpyAsync(capk.p, ck.data(), ck.size() * 8, hipMemcpyHostToDevice, s));
        TRY(hipMemcpyAsync(capv.p, cv.data(), cv.size() * 4, hipMemcpyHostToDevice, s));
    }
    auto root_cap = [&]() {
        if (leaf_caps) {
            auto it = leaf_caps->find(box_hash(0, 0, 0, 0));
            if (it != leaf_caps->end()) return it->second;
        }
        return leaf_cap;
    };
    GBox root{};
    root.cap = root_cap();
    root.parent = -1;
    root.leaf = 1;
    root.r[1] = int32_t(n[0]);
    root.r[3] = int32_t(n[1]);
    root.r[5] = int32_t(n[2]);
    for (int q = 0; q < 8; ++q) root.child[q] = -1;
    size_t cap_boxes = 4096;
    DevArr boxes, boxes2, cand, cnt, cnt_raw, scr;
    TRY(boxes.ensure(cap_boxes * sizeof(GBox)));
    TRY(hipMemcpyAsync(boxes.p, &root, sizeof(GBox), hipMemcpyHostToDevice, s));
    std::vector<int> level_start = {0};
    int nb = 1;
    for (int l = 0;; ++l) {
        const int b0 = level_start[l], nbl = nb - b0;
        if (nbl == 0 || l >= kMaxLevel) break;
        TRY(cand.ensure(size_t(nbl) * 48 * 4));
        TRY(cnt.ensure(size_t(nbl + 1) * 4));
        TRY(cnt_raw.ensure(size_t(nbl + 1) * 4));
        TRY(scr.ensure(scan_scratch(nbl + 1) * 4));
        SplitArgs sa{b0, nbl, boxes.as<GBox>(), {kd[0], kd[1], kd[2]}, cand.as<int32_t>(), cnt_raw.as<uint32_t>()};
        hipLaunchKernelGGL(split_kernel, dim3(nblk(nbl + 1, 128)), dim3(128), 0, s, sa);
        TRY(hipGetLastError());
        TRY(hipMemcpyAsync(cnt.p, cnt_raw.p, size_t(nbl + 1) * 4, hipMemcpyDeviceToDevice, s));
        TRY(scan_exclusive(cnt.as<uint32_t>(), nbl + 1, scr.as<uint32_t>(), s));
        uint32_t total = 0;
        TRY(hipMemcpyAsync(&total, cnt.as<uint32_t>() + nbl, 4, hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        if (total == 0) break;
        if (size_t(nb) + total >= (size_t(1) << 25)) return "more than 2^25 boxes";
        if (size_t(nb) + total > cap_boxes) {
            size_t nc = cap_boxes;
            while (nc < size_t(nb) + total) nc *= 2;
            TRY(boxes2.ensure(nc * sizeof(GBox)));
            TRY(hipMemcpyAsync(boxes2.p, boxes.p, size_t(nb) * sizeof(GBox), hipMemcpyDeviceToDevice, s));
            std::swap(boxes.p, boxes2.p);
            std::swap(boxes.bytes, boxes2.bytes);
            cap_boxes = nc;
        }
        EmitArgs ea{b0, nbl, nb, boxes.as<GBox>(), cand.as<int32_t>(), cnt.as<uint32_t>(), cnt_raw.as<uint32_t>(),
                    capk.as<uint64_t>(), capv.as<int32_t>(), int(ck.size())};
        hipLaunchKernelGGL(emit_kernel, dim3(nblk(nbl, 128)), dim3(128), 0, s, ea);
        TRY(hipGetLastError());
        level_start.push_back(nb);
        nb += int(total);
    }
    level_start.push_back(nb);
    const int depth = int(level_start.size()) - 2;
    // ---------------------------------------------------------------- lists
    DevArr bkey;
    TRY(bkey.ensure(size_t(nb) * 8));
    hipLaunchKernelGGL(box_keys_kernel, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, boxes.as<GBox>(), bkey.as<uint64_t>());
    TRY(hipGetLastError());
    std::vector<GBox> hb(nb);
    TRY(hipMemcpyAsync(hb.data(), boxes.p, size_t(nb) * sizeof(GBox), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    std::vector<int32_t> leaves;
    for (int b = 0; b < nb; ++b)
        if (hb[b].leaf) leaves.push_back(b);
    const int nleaf = int(leaves.size());
    ListView lv{};
    lv.box = boxes.as<GBox>();
    lv.bkey = bkey.as<uint64_t>();
    for (int l = 0; l <= kLevels; ++l) lv.level_start[l] = l <= depth + 1 ? level_start[l] : nb;
    lv.depth = depth;
    lv.pmask = pmask;
    DevArr dleaves, vcnt, vent, cnt3, oflow;
    DevArr lkey[3], lval[3], lent[3], lcnt[3];   // U, W, X: keys, sort payload, entries, counts by box
    TRY(dleaves.ensure(size_t(std::max(nleaf, 1)) * 4));
    TRY(hipMemcpyAsync(dleaves.p, leaves.data(), size_t(nleaf) * 4, hipMemcpyHostToDevice, s));
    TRY(vcnt.ensure(size_t(nb + 1) * 4));
    TRY(scr.ensure(scan_scratch(nb + 1) * 4));
    TRY(cnt3.ensure(6 * 4));
    TRY(oflow.ensure(4));
    hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, s, cnt3.as<uint32_t>(), int64_t(6), 0u);
    TRY(hipGetLastError());
    hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, s, oflow.as<uint32_t>(), int64_t(1), 0u);
    TRY(hipGetLastError());
    // count passes
    VArgs va{lv, nb, vcnt.as<uint32_t>(), nullptr, nullptr};
    hipLaunchKernelGGL(v_list_kernel, dim3(nblk(nb + 1, 128)), dim3(128), 0, s, va);
    TRY(hipGetLastError());
    UWArgs ua{lv, nleaf, dleaves.as<int32_t>(), cnt3.as<uint32_t>(), cnt3.as<uint32_t>() + 3, nullptr, nullptr,
              nullptr, oflow.as<int>()};
    const int64_t nthr = int64_t(nleaf) * 28;
    hipLaunchKernelGGL(uw_list_kernel<false>, dim3(nblk(nthr, 64)), dim3(64), 0, s, ua);
    TRY(hipGetLastError());
    TRY(scan_exclusive(vcnt.as<uint32_t>(), nb + 1, scr.as<uint32_t>(), s));
    uint32_t tot[4] = {0, 0, 0, 0}, uwx[3] = {0, 0, 0};   // tot: U, V, W, X
    TRY(hipMemcpyAsync(&tot[1], vcnt.as<uint32_t>() + nb, 4, hipMemcpyDeviceToHost, s));
    TRY(hipMemcpyAsync(uwx, cnt3.p, 12, hipMemcpyDeviceToHost, s));
    int of = 0;
    TRY(hipMemcpyAsync(&of, oflow.p, 4, hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    if (of) return "GPU tree build: descent stack overflow";
    tot[0] = uwx[0];
    tot[2] = uwx[1];
    tot[3] = uwx[2];
    TRY(vent.ensure(size_t(std::max<uint32_t>(tot[1], 1)) * 8));
    for (int q = 0; q < 3; ++q) {
        const size_t m = std::max<uint32_t>(uwx[q], 1);
        TRY(lkey[q].ensure(m * 8));
        TRY(lval[q].ensure(m * 4));
        TRY(lent[q].ensure(m * 8));
        TRY(lcnt[q].ensure(size_t(nb + 1) * 4));
    }
    // fill passes
    va.ofs = vcnt.as<uint32_t>();
    va.ent = vent.as<uint64_t>();
    hipLaunchKernelGGL(v_list_kernel, dim3(nblk(nb + 1, 128)), dim3(128), 0, s, va);
    TRY(hipGetLastError());
    ua.ukey = lkey[0].as<uint64_t>();
    ua.wkey = lkey[1].as<uint64_t>();
    ua.xkey = lkey[2].as<uint64_t>();
    hipLaunchKernelGGL(uw_list_kernel<true>, dim3(nblk(nthr, 64)), dim3(64), 0, s, ua);
    TRY(hipGetLastError());
    // U, W by (leaf, box, shift); X by (target box, source leaf, shift); then
    // the list lengths by owning box
    for (int q = 0; q < 3; ++q) {
        hipLaunchKernelGGL(fill_u32, dim3(nblk(nb + 1, 256)), dim3(256), 0, s, lcnt[q].as<uint32_t>(), int64_t(nb + 1), 0u);
        TRY(hipGetLastError());
        if (uwx[q] == 0) continue;
        hipLaunchKernelGGL(fill_u32, dim3(nblk(uwx[q], 256)), dim3(256), 0, s, lval[q].as<uint32_t>(), int64_t(uwx[q]), 0u);
        TRY(hipGetLastError());
        TRY(radix_sort(lkey[q].as<uint64_t>(), lval[q].as<int32_t>(), uwx[q], 55, sb, s));
        hipLaunchKernelGGL(key_count_kernel, dim3(nblk(uwx[q], 256)), dim3(256), 0, s, int64_t(uwx[q]),
                           lkey[q].as<uint64_t>(), lcnt[q].as<uint32_t>());
        TRY(hipGetLastError());
        hipLaunchKernelGGL(key_entries_kernel, dim3(nblk(uwx[q], 256)), dim3(256), 0, s, int64_t(uwx[q]),
                           lkey[q].as<uint64_t>(), lent[q].as<uint64_t>());
        TRY(hipGetLastError());
    }
    for (int q = 0; q < 3; ++q) TRY(scan_exclusive(lcnt[q].as<uint32_t>(), nb + 1, scr.as<uint32_t>(), s));
    // ---------------------------------------------------------------- to the host
    std::vector<uint32_t> off[4];
    std::vector<uint64_t> ent[4];
    DevArr *os[4] = {&lcnt[0], &vcnt, &lcnt[1], &lcnt[2]};
    DevArr *es[4] = {&lent[0], &vent, &lent[1], &lent[2]};
    for (int q = 0; q < 4; ++q) {
        off[q].resize(nb + 1);
        ent[q].resize(tot[q]);
        TRY(hipMemcpyAsync(off[q].data(), os[q]->p, size_t(nb + 1) * 4, hipMemcpyDeviceToHost, s));
        if (tot[q] > 0) TRY(hipMemcpyAsync(ent[q].data(), es[q]->p, size_t(tot[q]) * 8, hipMemcpyDeviceToHost, s));
    }
    TRY(hipStreamSynchronize(s));
    t.boxes.resize(nb);
    for (int b = 0; b < nb; ++b) {
        const GBox &g = hb[b];
        Box &B = t.boxes[b];
        B.level = g.level;
        for (int k = 0; k < 3; ++k) B.anchor[k] = g.anchor[k];
        B.parent = g.parent;
        for (int o = 0; o < 8; ++o) B.child[o] = g.child[o];
        B.leaf = g.leaf != 0;
        B.sl[0] = g.r[0]; B.sl[1] = g.r[1];
        B.dl[0] = g.r[2]; B.dl[1] = g.r[3];
        B.trg[0] = g.r[4]; B.trg[1] = g.r[5];
        B.nsrc_sub = (g.r[1] - g.r[0]) + (g.r[3] - g.r[2]);
        B.ntrg_sub = g.r[5] - g.r[4];
        B.cap = g.cap;
    }
    t.leaves.assign(leaves.begin(), leaves.end());
    t.depth = depth;
    t.level_start.assign(level_start.begin(), level_start.end());
    std::vector<int> *to[4] = {&t.u_off, &t.v_off, &t.w_off, &t.x_off};
    std::vector<Entry> *te[4] = {&t.u, &t.v, &t.w, &t.x};
    for (int q = 0; q < 4; ++q) {
        to[q]->assign(off[q].begin(), off[q].end());
        te[q]->resize(ent[q].size());
        for (size_t i = 0; i < ent[q].size(); ++i) {
            const uint64_t e = ent[q][i];
            const int c = int(e & 31);
            Entry &en = (*te[q])[i];
            en.box = int(e >> 5);
            en.shift[0] = int8_t(c / 9 - 1);
            en.shift[1] = int8_t((c / 3) % 3 - 1);
            en.shift[2] = int8_t(c % 3 - 1);
        }
    }
    finish_tree(t);
    return "";
}

}  // namespace kafmm
