// Argument blocks and launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace kafmm {

// Packed periodic image shift: bits (2k, 2k+1) hold shift_k + 1.
constexpr int kZeroShift = 1 | (1 << 2) | (1 << 4);
// Entry code of an L2T task entry that names the leaf's own downward set.
constexpr int kLocalSet = 64;
inline int pack_shift(const int8_t s[3]) { return (s[0] + 1) | ((s[1] + 1) << 2) | ((s[2] + 1) << 4); }

struct P2PArgs {
    const int4 *tasks;         // {chunk, e0, e1, -}: slice of the leaf's direct list
    const int4 *chunks;        // {leaf, t0, t1, -}
    const float *trg;          // [n_trg][8]
    const int2 *ent;           // direct entries {source box, packed shift}
    const int2 *box_sl, *box_dl;
    const float *sl, *dl;      // source records
    const double4 *geom;       // box geometry (REL kernels: source leaf centres)
    double *part;              // [task][256][NACC]
};

struct S2CArgs {
    const int4 *tasks;         // {dst box, packed shift | src leaf << 6, j0, j1}: sources [j0, j1) of src
    const float *staged;       // staged source records (stage_sources_kernel)
    const double4 *geom;
    const float *grid;         // [M][3] unit lattice
    int M;
    double alpha;              // surface radius in half box sides
    float *part;               // [task][ncomp][M]
};

struct S2CReduceArgs {
    const int *dst;            // destination box per block
    const int *off;            // per block: range of task indices
    const int *task;
    const float *part;
    double *chk;               // [box][ncomp][M]
    int M, ncomp, accumulate;
};

struct GemmArgs {
    const int4 *tiles;         // {op, col0, ncol, -}
    const float *ops;          // operators [R][K] row-major, opsz floats apart
    int64_t opsz;
    const float *X;            // input columns (K floats each, xs apart)
    float *Y;                  // output columns (R floats each, ys apart)
    const int *bcol, *ycol;    // column indices (units of xs / ys floats)
    int R, K;                  // operator shape, multiples of 32
    int xs, ys;
    int Mr;                    // rows >= Mr of the operators are zero (skipped)
    int Mk;                    // columns >= Mk of the operators are zero; multiple of 16, <= K
};

struct Gemm64Args {
    const double *A;           // [R][K] row-major, leading dimension lda
    int R, K, lda;
    const double *B;           // columns: B + bidx[c] * ldb
    const int *bidx;
    int ldb;
    const int *cidx;           // output columns: C + cidx[c] * ldc
    const double *cscale;      // per-column scale or null
    int ldc;
    int ncol;
};

// Downward translation of check potentials, child (+)= L2L_cc[op] * parent,
// FP64.  Pairs are grouped by octant into blocks of 64 / ncomp pairs.
struct L2LArgs {
    const double *ops;         // [8][M][M]
    int M;
    const int4 *blocks;        // {op, first pair, pair count, 0}
    const int2 *pairs;         // {parent box, child box}
    const double *delta;       // [pair][3] c_child - c_parent (Psi origin shift, ncomp 4)
    double *chk;               // [box][ncomp][M]
};

// Largest rank of compressed V-list translations.
constexpr int kMaxCompressed = 512;

struct ReduceArgs {
    const int *dst;            // destination box per task
    const int *off;            // per task: pair range
    const int *pair;           // Y pair index per entry
    const double *scale;       // per entry
    const float *delta;        // per entry: Psi origin shift (3)
    const float *Y;            // pair columns, ys floats apart per component
    int ys;
    double *chk;
    int M, Mp, ncomp, accumulate;
    int kc;                    // > 0: Y holds kc coefficients in the basis below
    const float *basis_t;      // U_k^T [kc][Mp]
};

struct L2TArgs {
    const int4 *tasks;         // {chunk, e0, e1, -}
    const int4 *chunks;
    const float *trg;
    const double4 *geom;
    const int2 *ent;           // {box, packed shift | kLocalSet}
    const float *grid;
    const float *up_dens, *dn_dens;
    int M, Mp;
    double alpha_in, alpha_out;
    double *part;              // [task][256][NACC]
};

constexpr int kMaxAcc = 16;    // most accumulated / output components of any kernel

struct CombineMap {
    int src[kMaxAcc];
    double scale[kMaxAcc];
};

struct CombineArgs {
    const int4 *chunks;
    const int4 *chunk_tasks;   // {p2p t0, t1, l2t t0, t1}
    const double *near, *far;  // task partials
    const int32_t *perm;
    int nacc, kt;
    CombineMap map;
    double *out;
};

struct DirectArgs {
    int64_t n_sl, n_dl, n_trg;
    const double *sl, *sl_val, *dl, *dl_val, *trg;
    int k_sl, k_dl, k_trg;
    double *out;
    int slices;                // source slices (grid.y); > 1 needs work
    double *work;              // [slices][n_trg][k_trg] partial sums, summed in slice order
};

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_pack_sources(int64_t n, const double *xyz, const int32_t *perm, double3 origin, double inv_len,
                               int rec, float *out, hipStream_t s);
hipError_t launch_pack_targets(int64_t n, const double *xyz, const int32_t *perm, double3 origin,
                               double inv_len, float *out, hipStream_t s);
// exact_r: the Stokeslet with r from hi/lo coordinates (plans that
// launch_rel_check flagged)
hipError_t launch_p2p(int kernel, int ntasks, const P2PArgs &a, bool exact_r, hipStream_t s);
// Plan-time check of the leaf-relative P2P form: *flag != 0 if two distinct
// points of different direct-list entries lie closer than 2^-12 of the
// source leaf's side (the flag is ORed, the caller clears it).
hipError_t launch_rel_check(int ntasks, const P2PArgs &a, int rec, unsigned *flag, hipStream_t s);
hipError_t launch_s2c(int src_kind, int ntasks, const S2CArgs &a, hipStream_t s);
// Floats per staged source record of a source kind (0 for an unknown kind).
int s2c_stage_stride(int src_kind);
// Stage the sources of every listed leaf (box_range: the leaves' SL or DL ranges).
hipError_t launch_stage_sources(int src_kind, int nleaves, const int *leaves, const int2 *box_range,
                                const double4 *geom, const float *src, int rec, float *out, hipStream_t s);
hipError_t launch_gemm_f32(int ntiles, const GemmArgs &a, hipStream_t s);
hipError_t launch_gemm_bf16x3(int ntiles, const GemmArgs &a, hipStream_t s);
hipError_t launch_gemm_f64(const Gemm64Args &a, double *C, hipStream_t s);
hipError_t launch_gemm_f64_to_f32(const Gemm64Args &a, float *C, hipStream_t s);
hipError_t launch_reduce(int ntasks, const ReduceArgs &a, hipStream_t s);
hipError_t launch_l2l_check(int nblocks, int ncomp, const L2LArgs &a, hipStream_t s);

// No-slip wall image summations (wall.hip).  Sources in the caller's order.
struct WallValueArgs {
    int64_t n;                 // sources
    const double *y;           // [n][3]
    const double *val;         // [n][3] f, or [n][4] (f, b) when rpy
    int rpy;
    double zw;                 // wall plane z
    double *vs;                // [2n][4] S summation, RPY (sources, then images)
    double *sd_dl;             // [n][3]      SD image dipoles
    double *sdz_sl, *sdz_dl;   // [n], [n][3] SDZ image charges, dipoles (rpy)
    double *q;                 // [n][9]      image quadrupoles (rpy)
};
struct WallAssembleArgs {
    int64_t nt;
    const double *x;           // [nt][3] targets
    double zw;
    int rpy;
    const double *us;          // [nt][6] (u, lap u) of the S summation
    const double *sd;          // [nt][ksd] phi, grad phi[, Hessian]
    int ksd;                   // 4, or 10 (rpy)
    const double *sdz;         // [nt][4]
    const double *qp;          // [nt][10] (rpy)
    double *out;               // [nt][3] or [nt][6]
};
hipError_t launch_wall_positions(int64_t n, const double *y, double zw, double *y2, double *yi, hipStream_t s);
hipError_t launch_wall_values(const WallValueArgs &a, hipStream_t s);
hipError_t launch_wall_assemble(const WallAssembleArgs &a, hipStream_t s);
// Triply periodic Stokes kernels (periodic.hip): the root's flow at its
// upward check points X from sorted source records of a kind (0 Stokeslet,
// 1 RPY, 2 PVel single layer, 3 PVel double layer, 4 regularized force and
// torque; chunks of 4096 sources,
// partial sums part [chunks][3M + 3], the last 3 the flux moment); then
// V [3M + 3] = the chunks' sum and the far images' forces F = Q V / (8 pi)
// [3M]; targets (sorted, unit-box records) add their far-image values in
// user order (mode 0 Stokeslet u; 1 RPY u, lap u; 2 PVel p, u; 3 PVelGrad
// p, u, grad p, grad u; 4 PVelLaplacian p, u, lap u; 5 Traction sigma;
// 6 force-torque u, omega;
// modes 2-4 less the flux moment's uniform flow, mom = V + 3M; inv_len =
// 1/L sets each output's power of the box size);
// per-block sums of the first ncomp values of each source and of their
// absolute values.
int stokes_root_chunks(int64_t n);
hipError_t launch_stokes_root_check(int kind, int64_t n_src, const float *src, int rec, const double *X, int M,
                                    double *part, hipStream_t s);
hipError_t launch_stokes_far_forces(int nchunks, const double *Q, int M, const double *part, double *V, double *F,
                                    hipStream_t s);
hipError_t launch_stokes_far_targets(int64_t n, const float *trg, const int32_t *perm, int mode, const double *F,
                                     const double *Z, int M, double inv_len, const double *mom, double *out,
                                     hipStream_t s);
hipError_t launch_value_partials(int64_t n, const double *f, int stride, int ncomp, int nblocks, double *part,
                                 hipStream_t s);
hipError_t launch_periodic(const double *T, const float *dens, double *chk, int M, int Mp, int nc, int root,
                           hipStream_t s);
hipError_t launch_l2t(int kernel, int ntasks, const L2TArgs &a, hipStream_t s);
hipError_t launch_s2c_reduce(int ndst, const S2CReduceArgs &a, hipStream_t s);
hipError_t launch_combine(int nchunks, const CombineArgs &a, hipStream_t s);
// Source slices of the FP64 direct sum for n_trg targets and n_src sources
// (enough blocks to fill the chip when there are few targets).
int direct_f64_slices(int64_t n_trg, int64_t n_src);
hipError_t launch_direct_f64(int kernel, const DirectArgs &a, hipStream_t s);
// True if the kernel's P2P forms r from leaf-relative positions (records
// then need launch_rel_positions after packing).
bool p2p_uses_rel(int kernel);
hipError_t launch_rel_positions(int nleaves, const int *leaves, const int2 *box_sl, const double4 *geom, int rec,
                                float *sl, hipStream_t s);

}  // namespace kafmm
