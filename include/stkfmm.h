/*
 * stkfmm.h -- C ABI of the MI355X kernel aggregated FMM evaluation pass.
 *
 * The library evaluates the kernel summation problem
 *     g_i(x^a) = sum_b K_ij(x^a, y^b) s_j^b            (Sec. I, Eq. kernelsumlinear)
 * (and its nonlinear-in-source form, Sec. II, Eq. kernelsum, for RPY) with a
 * kernel independent FMM whose tree-traversal (ML-tree) kernel is the scalar
 * Laplace kernel for every problem: Laplace problems carry 1 component,
 * Stokes problems (Stokeslet, RPY, StokesPVel double layer, traction) carry 4
 * Laplace components (3 Phi_j and one Psi).  The choice of ML-tree kernel is
 * the paper's kernel aggregation principle (Sec. II, kernel tables): it must
 * be linear and of low dimension.
 *
 * Memory and ownership
 *   - All point and value arrays are caller-owned DEVICE pointers (HIP global
 *     memory on the context's device), FP64, contiguous AoS: points [n][3],
 *     values [n][k].  The library never frees or retains them after a call
 *     returns, except that stkfmm_set_points keeps its own sorted copies.
 *   - The library allocates its own device workspace (hipMalloc) in
 *     stkfmm_set_points and stkfmm_run; it is released by stkfmm_destroy.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     ordered after prior work on that stream; calls return after the result
 *     is complete (they synchronise the stream).
 *
 * Errors
 *   - No function throws across the ABI.  Every failing call returns a
 *     status code and records a message readable by stkfmm_last_error.
 *   - On error, output arrays hold unspecified contents.
 *
 * Thread safety: one context per host thread; contexts are independent.
 */
#ifndef STKFMM_H
#define STKFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stkfmm_ctx stkfmm_ctx;

typedef enum {
    STKFMM_OK = 0,
    STKFMM_E_ARG = 1,          /* bad argument: NULL, negative size, bad p / leaf_cap, NaN */
    STKFMM_E_DOMAIN = 2,       /* point outside the box (open BC) or non-zero net charge / force / flux (periodic) */
    STKFMM_E_UNSUPPORTED = 3,  /* kernel / boundary combination not implemented */
    STKFMM_E_NOMEM = 4,        /* device or host allocation failed */
    STKFMM_E_DEVICE = 5,       /* HIP runtime error */
    STKFMM_E_ACCURACY = 6,     /* learned mode: sampled error above tolerance after fallback */
    STKFMM_E_STATE = 7         /* call out of order (run before set_points) */
} stkfmm_status;

/* Kernel names and value widths follow the appendix table of supported
 * kernels (tab:implement):                     SL        DL       target
 *   LAP_PGRAD      q -> phi, grad phi          q (1)     d (3)    (phi, dphi/dx, dphi/dy, dphi/dz) (4)
 *   LAP_PGRADGRAD  q -> phi, grad, Hessian     q (1)     d (3)    (phi, grad phi, xx xy xz yy yz zz) (10)
 *   LAP_QPGRADGRAD Q -> phi, grad, Hessian     Q (9)     --       (phi, grad phi, xx xy xz yy yz zz) (10)
 *   STOKESLET      f -> u                      f (3)     --       u (3)
 *   RPY            [f, b] -> [u, lap u]        f,b (4)   --       (u, lap u) (6)
 *   PVEL           [f, q], D -> [p, u]         f,q (4)   D (9)    (p, u) (4)
 *   PVEL_GRAD      [f, q], D -> [p, u, grad p, grad u]
 *                                              f,q (4)   D (9)    (p, u, grad p, grad u) (16)
 *   PVEL_LAPLACIAN [f, q], D -> [p, u, lap u]  f,q (4)   D (9)    (p, u, lap u) (7)
 *   TRACTION       [f, q], D -> sigma          f,q (4)   D (9)    sigma (9)
 *   STOKES_REG_VEL [f, eps] -> u               f,eps (4) --       u (3)
 *   STOKES_REG_VEL_OMEGA [f, t, eps] -> [u, w] f,t,eps (7) --     (u, angular velocity) (6)
 * STOKES_REG_VEL is the regularized Stokeslet of the blob psi^eps (Sec. II.B,
 * tab:ktab_reg), eps >= 0 per source; its far field is represented to
 * O((eps/r)^4), so eps must be far smaller than the smallest leaf box.
 * STOKES_REG_VEL_OMEGA adds point torques t and the angular velocity
 * w = curl(u)/2 (the force-torque extension of Sec. II.B, tab:ktab_regftvw).
 * LAP_QPGRADGRAD's quadrupole gives phi = Q_jk d_j d_k L, L = 1/(4 pi r) (Sec. II.A).
 * Q, D, sigma and grad u are row-major 3x3 (D[3j+k] = D_jk, sigma[3i+j],
 * grad u[3i+j] = du_i/dx_j); q in the PVEL kernels and TRACTION is twice the
 * physical source (Sec. II.C); viscosity mu = 1.  Away from the sources
 * lap u = grad p (the Stokes equations), and PVEL_LAPLACIAN returns it as such. */
typedef enum {
    STKFMM_LAP_PGRAD = 0,
    STKFMM_STOKESLET = 1,
    STKFMM_RPY = 2,
    STKFMM_PVEL = 3,
    STKFMM_TRACTION = 4,
    STKFMM_STOKES_REG_VEL = 5,
    STKFMM_STOKES_REG_VEL_OMEGA = 6,
    STKFMM_LAP_PGRADGRAD = 7,
    STKFMM_PVEL_GRAD = 8,
    STKFMM_PVEL_LAPLACIAN = 9,
    STKFMM_LAP_QPGRADGRAD = 10
} stkfmm_kernel;

/* Boundary conditions (Sec. III and its appendix on periodicity).  PXYZ is
 * implemented for LAP_PGRAD, LAP_PGRADGRAD and LAP_QPGRADGRAD (zero net
 * charge; Ewald's convention: no k = 0 term, no surface term) and for
 * every Stokes kernel: zero net force (a net torque is allowed), and for
 * the PVEL family also zero net flux q and a zero sum of tr D; the Fourier
 * series of the periodic Stokes equations without its k = 0 term, i.e. zero
 * mean velocity, summed with Hasimoto's Ewald split; the pressure, and so
 * TRACTION's isotropic part, is defined up to an additive constant.  PXY
 * (periodic in x and y with period box_len, open in z) is implemented for
 * STOKESLET and RPY: zero net force; the Fourier series in x and y whose
 * k = 0 mode is the sheet flow u_xy(z) = -(1/2A) sum_j f_j,xy |z - z_j|
 * (A = box_len^2, no added constant: far above and below the sources the
 * flow tends to +-(1/2A) sum_j f_j,xy z_j), summed with Hasimoto's Ewald
 * split; points are wrapped in x and y and must lie in
 * [origin_z, origin_z + box_len) in z.  WALL (Sec. III, the no-slip wall section,
 * tab:rpywall) is an open domain bounded below by a no-slip wall on the
 * plane z = origin[2], for STOKESLET and RPY only, fixed p and leaf_cap only:
 * the flow is assembled from three (Stokeslet) or four (RPY) free-space
 * summations over the sources and their mirror images, on a cube of side
 * 2 box_len holding both; all points must lie in [origin, origin + box_len)^3.
 * The others return STKFMM_E_UNSUPPORTED. */
typedef enum {
    STKFMM_BC_OPEN = 0,
    STKFMM_BC_PX = 1,
    STKFMM_BC_PXY = 2,
    STKFMM_BC_PXYZ = 3,
    STKFMM_BC_WALL = 4
} stkfmm_bc;

/* Create a context for the cube [origin, origin + box_len)^3 on HIP device
 * `device` (Sec. III: the points live in a cubic computational box, [0, L)^3
 * in the paper's benchmarks).  flags: reserved, pass 0.  Operators (surface pseudo-inverses,
 * M2M/L2L/M2L matrices, periodic operator) are built lazily per order p on
 * first use and shared by all contexts of the process on that device (one
 * set per p, periodicity, "svd_tol" and "m2l_tol"), kept until it exits.
 * Errors: E_ARG (out NULL, box_len <= 0 or not finite), E_DEVICE. */
stkfmm_status stkfmm_setup(stkfmm_ctx **out, const double origin[3], double box_len,
                           int device, unsigned flags);

/* Build the adaptive octree, the U/V/W/X interaction lists (Sec. II) and
 * the sorted device copies of the points (t_tree).  Points are device
 * pointers [n][3] FP64; n_sl or n_dl may be 0 with a NULL pointer.  A kernel
 * without DL sources requires n_dl == 0.  SL, DL and target sets are
 * independent and may alias.  p: equivalent-surface order (points per
 * surface M = 6(p-1)^2 + 2, Sec. III), 2 <= p <= 16, or 0 for the learned
 * order.  leaf_cap: a box is split while it holds more than leaf_cap
 * targets, SL or DL sources (Sec. III uses 2000); >= 1, or 0 for learned
 * per-leaf capacities (see the learned mode below).
 * Open BC: every point must lie in [origin, origin+box_len)^3, else E_DOMAIN.
 * PXYZ: points are wrapped into the box; PXY: wrapped in x and y.
 * Errors: E_ARG, E_DOMAIN, E_UNSUPPORTED, E_NOMEM, E_DEVICE. */
stkfmm_status stkfmm_set_points(stkfmm_ctx *ctx, stkfmm_kernel kernel, stkfmm_bc bc,
                                int64_t n_sl, const double *sl_xyz,
                                int64_t n_dl, const double *dl_xyz,
                                int64_t n_trg, const double *trg_xyz,
                                int p, int leaf_cap, void *hip_stream);

/* The evaluation pass (t_run) on the points of the last stkfmm_set_points:
 * sl_val [n_sl][k_sl], dl_val [n_dl][k_dl] in, trg_val [n_trg][k_trg] out
 * (overwritten, user order).  Periodic LAP_PGRAD requires sum q = 0
 * (relative to sum |q|, 1e-9), else E_DOMAIN; its potential is defined up to
 * an additive constant (the Ewald convention with the k = 0 term dropped).
 * Periodic Stokes kernels (PXYZ and PXY) require each component of sum f to vanish
 * (relative to sum |f_k|, 1e-9), else E_DOMAIN; the periodic PVEL family
 * (PVEL, PVEL_GRAD, PVEL_LAPLACIAN, TRACTION) also requires sum q = 0
 * (relative to the sum of |f_k| and |q|) and sum tr D = 0 over the double
 * layer (relative to the sum of |D_jk|), else E_DOMAIN, and its pressure
 * (TRACTION: sigma's isotropic part) is determined up to an additive
 * constant.
 * Errors: E_STATE (no points set), E_ARG, E_DOMAIN, E_NOMEM, E_DEVICE. */
stkfmm_status stkfmm_run(stkfmm_ctx *ctx, const double *sl_val, const double *dl_val,
                         double *trg_val, void *hip_stream);

/* The kernel summation problem of Sec. I (Eq. kernelsumlinear) for two sets
 * of sources, single layer and double layer, and one set of targets, all
 * three independent (Sec. III, implementation): stkfmm_set_points followed
 * by stkfmm_run. */
stkfmm_status stkfmm_evaluate(stkfmm_ctx *ctx, stkfmm_kernel kernel, stkfmm_bc bc,
                              int64_t n_sl, const double *sl_xyz, const double *sl_val,
                              int64_t n_dl, const double *dl_xyz, const double *dl_val,
                              int64_t n_trg, const double *trg_xyz, double *trg_val,
                              int p, int leaf_cap, void *hip_stream);

/* FP64 direct sum on the GPU of the same kernel summation problem (the
 * plain O(N_S N_T) definition, Sec. I) at the given targets: the error judge
 * of the learned mode and a measurement tool.  Open BC only; same layouts
 * and conventions as stkfmm_evaluate; pairs with r = 0 contribute nothing.
 * Errors: E_ARG, E_UNSUPPORTED, E_DEVICE. */
stkfmm_status stkfmm_direct(stkfmm_ctx *ctx, stkfmm_kernel kernel,
                            int64_t n_sl, const double *sl_xyz, const double *sl_val,
                            int64_t n_dl, const double *dl_xyz, const double *dl_val,
                            int64_t n_trg, const double *trg_xyz, double *trg_val,
                            void *hip_stream);

/* stkfmm_direct for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, the same source slices and so the same results as
 * stkfmm_direct, bit for bit, but its partial sums live in a static device
 * array of 2^23 doubles (64 MiB) that every GPU the library runs on holds
 * from its first stkfmm_setup until the process ends; the call itself
 * allocates nothing.  The caller still provides every input and output
 * array.  Sizes whose partial sums exceed the array (slices * n_trg * k_trg
 * doubles, only when the sources are split into slices, i.e. below about
 * 5e5 targets: never for k_trg <= 7) return E_ARG with the sizes in the
 * message.  Every call on one GPU shares that GPU's array and each call
 * overwrites the part it uses, so calls that overlap on one GPU (other
 * streams, other host threads, other contexts) race.
 * Errors: E_ARG, E_UNSUPPORTED, E_DEVICE. */
stkfmm_status stkfmm_direct_noalloc(stkfmm_ctx *ctx, stkfmm_kernel kernel,
                                    int64_t n_sl, const double *sl_xyz, const double *sl_val,
                                    int64_t n_dl, const double *dl_xyz, const double *dl_val,
                                    int64_t n_trg, const double *trg_xyz, double *trg_val,
                                    void *hip_stream);

/* Value widths of a kernel (tab:implement).  k_dl is 0 for kernels without
 * DL sources.  Pure host function.  Errors: E_ARG (NULL output, bad kernel). */
stkfmm_status stkfmm_kernel_dims(stkfmm_kernel kernel, int *k_sl, int *k_dl, int *k_trg);

/* Options (strings) of the method's knobs: the equivalent-surface order and
 * leaf size are arguments of stkfmm_set_points (Sec. III); these set the
 * arithmetic and the other parameters.
 * "precision" = "fp32" | "split_bf16"  (M2L arithmetic),
 * "svd_tol" = relative truncation of the check-to-equivalent pseudo-inverse
 * (default 1e-7), "overlap" = "1" (P2P concurrent with the far field, the
 * default) | "0" (serial, for per-stage timing), "tol" = accuracy target of
 * the learned mode (default 1e-5), "p2p_task_sources" = sources per P2P task
 * (default 1024), "w_direct_frac" / "x_direct_frac" = W / X pairs whose source
 * count / target count is below this fraction of M are summed directly
 * (defaults 0.73 / 0.5), "m2l_tol" = relative singular-value cut of the
 * shared basis that compresses the V-list translations (default 5e-8: rank
 * 192 at p = 8; learned plans use tol / 50 unless it was set, rank 160 at
 * p = 8 for tol 1e-5; "0" keeps them dense), "tree" = "gpu" (the default:
 * Morton keys, the sort, the refinement and the U/V/W/X lists are built by
 * the library's HIP kernels from the device coordinates) | "host" (the same
 * tree built on host threads), "operator_cache" = directory of the on-disk
 * operator cache ("" = none; default $STKFMM_OPERATOR_CACHE, else
 * $XDG_CACHE_HOME/stkfmm_operators, else $HOME/.cache/stkfmm_operators; see
 * stkfmm_prepare_operators).  Errors: E_ARG. */
stkfmm_status stkfmm_set_option(stkfmm_ctx *ctx, const char *key, const char *value);

/* The FP64 operator precomputation of Sec. II for order p and boundary bc
 * (check-to-equivalent pseudo-inverses, M2M/L2L, the V-list translations
 * and, with m2l_tol > 0, their compressed basis; the far images for PXYZ,
 * and for PXY and PXYZ the periodic Stokeslet's far-image fit), built or
 * loaded from cache_dir and stored there when built.  Host only: it touches
 * no device, so the cache can be filled before a run (the contexts read the
 * same files).  svd_tol and m2l_tol as the options of those names (0 keeps
 * the translations dense); cache_dir NULL or "" builds without the cache.
 * One file per set, named by its parameters and by a hash of the library's
 * operator sources (a changed library ignores older files); a file whose
 * size, parameters or trailing checksum do not match is rebuilt and
 * replaced; files are written to a temporary name and renamed, so
 * concurrent processes are safe.  *loaded (may be NULL) receives 1 when
 * every part came from the cache; *digest (may be NULL) a 64-bit hash of
 * the set (equal for a built and a loaded set).  Errors: E_ARG (p outside
 * [2, 16], tolerances outside (0, 1) / [0, 1), bad bc), E_NOMEM. */
stkfmm_status stkfmm_prepare_operators(int p, stkfmm_bc bc, double svd_tol, double m2l_tol, const char *cache_dir,
                                       int *loaded, uint64_t *digest);

/* Timings of the last set_points (t_tree_ms) and run (t_run_ms, device event
 * time): the tree-construction and tree-traversal times the paper reports
 * separately (Sec. III, t_tree and t_run).  stage_ms[16] (may be NULL) receives per-stage device times of the
 * last run in the order: 0 pack, 1 S2M, 2 M2M+UC2UE, 3 M2L, 4 S2L (X list)
 * and the periodic operator, 5 L2L+DC2DE, 6 L2T+M2T, 7 P2P, 8 combine,
 * 9 the V-list GEMM launch alone (part of stage 3: the translations before
 * their per-destination sum); others 0.  P2P runs on an internal stream concurrently with stages 1-6
 * unless the option "overlap" is "0".  For a WALL plan the times and stages
 * are summed over its summations. */
stkfmm_status stkfmm_get_timings(const stkfmm_ctx *ctx, double *t_tree_ms, double *t_run_ms,
                                 double stage_ms[16]);

/* Plan statistics of the last set_points; stats[21] receives:
 * 0 boxes, 1 leaves, 2 depth, 3 U-list pairs (sum over target leaves of
 * n_trg * sum of U-list source counts), 4 V-list pairs, 5 W-list pairs,
 * 6 X-list pairs, 7 M (points per surface), 8 n_trg, 9 n_sl, 10 n_dl,
 * 11 U-list entries, 12 P2P pairs evaluated (U pairs plus the W and X
 * pairs summed directly because that is cheaper), 13 W pairs summed
 * directly, 14 X pairs summed directly, 15 P2P tasks, 16 rank of the
 * compressed V-list translations (0: dense), 17 Mp (M padded to 32),
 * 18 rank of the check-to-equivalent pseudo-inverse, 19 P2P lane pairs
 * (pairs including the idle lanes of partly filled 64-target waves; a wave
 * left with at most 32 targets splits the sources over its lanes),
 * 20 1 if the Stokeslet P2P of this plan forms r from the hi/lo coordinates
 * rather than from leaf-relative FP32 positions, because two distinct points
 * of different leaves lie closer than 1/4096 of a leaf side (else 0).
 * For a WALL plan: the statistics of its Stokes summation (sources and
 * their images).  Errors: E_ARG, E_STATE. */
stkfmm_status stkfmm_get_stats(const stkfmm_ctx *ctx, int64_t stats[21]);

/* The adaptive octree and interaction lists of the last set_points (Sec. II:
 * the tree and the U, V, W, X lists of KIFMM), copied to caller-owned host
 * memory.  sizes[8] (out): n_box, n_u, n_v, n_w, n_x (list entries), n_sl,
 * n_dl, n_trg.  With box == NULL only sizes are written; else all of:
 *   box  [n_box][12] int32: level, anchor x, y, z (in cells of the level),
 *        parent (-1 for the root), is_leaf, then the [begin, end) ranges of
 *        the box's SL, DL and target points in the sorted orders;
 *   perm [n_sl + n_dl + n_trg] int32: sorted position -> input index, SL
 *        then DL then targets (points sorted by Morton key, ties by index);
 *   off  [4][n_box + 1] int32: CSR offsets of the U, V, W, X lists by box;
 *   ent  [n_u + n_v + n_w + n_x][4] int32: U, then V, W, X entries: source
 *        box and periodic image shift (x, y, z, in root-box lengths).
 * Boxes are breadth-first (level by level, each level in Morton order);
 * entries within a list are ordered by (box, shift); entries whose box holds
 * no sources and the lists of boxes without targets are dropped.
 * Errors: E_ARG, E_STATE (no plan), E_UNSUPPORTED (WALL plans hold one tree
 * per summation). */
stkfmm_status stkfmm_get_tree(const stkfmm_ctx *ctx, int64_t sizes[8], int32_t *box, int32_t *perm,
                              int32_t *off, int32_t *ent);

/* ---------------------------------------------------------------------
 * Learned order / leaf-capacity mode.  stkfmm_set_points with p = 0 and/or
 * leaf_cap = 0 builds the reference tree (leaf_cap 2000, Sec. III), computes
 * 12 features per leaf, runs the predictor network on the GPU and uses, for
 * each 0 argument, the predicted order (classes 6/8/10/12) and the
 * predicted per-leaf capacities (classes 250/500/1000/2000, applied by
 * refining each reference leaf).  The
 * order is the smallest class whose error over all targets, estimated from a
 * calibration table (RMS error at each order of training leaves of each
 * predicted class, weighted by the leaves' target counts), is within 0.8 tol.
 * The first stkfmm_run of such a plan checks the result on 256 sampled targets
 * against the FP64 direct sum; above the option "tol" (default 1e-5, relative
 * L2 per output field) it re-plans with the fixed p = 10, leaf_cap = 2000
 * and reruns; E_ACCURACY if that too misses tol.  Open BC only.  This mode is
 * not in the paper, which uses one global order and leaf size (Sec. III). */

/* Number of FP32 parameters of the predictor network.  Layout: mean[12],
 * std[12] (input scaling), W1[12][64], b1[64], W2[64][64], b2[64], W3[64][8],
 * b3[8]; logits 0-3 order classes, 4-7 capacity classes.  Pure host. */
int stkfmm_mlp_nparam(void);

/* Floats of device workspace the network kernels need for a batch. */
int64_t stkfmm_mlp_workspace(int64_t batch);

/* Install the predictor (host pointer, n = stkfmm_mlp_nparam() + 16): the
 * network parameters followed by the 4x4 order calibration table
 * table[class][order class] (relative RMS error, >= 0). */
stkfmm_status stkfmm_set_predictor(stkfmm_ctx *ctx, const float *params, int n);

/* After set_points: info[12] = {learned, order used, fell back, validated,
 * order-class histogram (4), capacity-class histogram (4)}; *sampled_err the
 * checked error (or -1).  Errors: E_ARG. */
stkfmm_status stkfmm_get_learned(const stkfmm_ctx *ctx, int64_t info[12], double *sampled_err);

/* Features [n_leaf][12] (host, may be NULL) of the current tree's leaves and
 * the leaf index of every target (host [n_trg], user order, may be NULL);
 * *n_leaf receives the leaf count.  Errors: E_ARG, E_STATE. */
stkfmm_status stkfmm_get_leaf_features(stkfmm_ctx *ctx, float *features, int32_t *leaf_of_target,
                                       int64_t *n_leaf);

/* Work of the current plan attributed to its targets (host [n_trg][5],
 * user order): 0 P2P lane pairs (as stats[19]: the leaf's targets in
 * 64-lane waves times the sources of its direct list, partly filled waves
 * with their sources split over the lanes), 1 P2P wave entries, 2 M2L
 * flops, 3 surface evaluations (S2M, S2L, L2T, M2T), 4 boxes.  Each box's
 * work is shared equally by the targets in it.  Used to price capacity
 * labels for the learned mode.  Errors: E_ARG, E_STATE, E_UNSUPPORTED
 * (WALL plans). */
stkfmm_status stkfmm_get_plan_work(stkfmm_ctx *ctx, double *work);

/* Predictor network kernels on device buffers (stream-ordered, synchronous).
 * x [batch][12], logits [batch][8], labels [batch][2] (order class, capacity
 * class), work >= stkfmm_mlp_workspace(batch) floats; grad, m, v [nparam].
 * loss_grad writes the mean cross-entropy (two heads, averaged) to *loss
 * (device) and its gradient; it copies the labels to the host first and
 * returns E_ARG unless every label lies in 0..3.  adam applies one
 * bias-corrected Adam step (beta 0.9, 0.999, eps 1e-8; the input scaling is
 * not updated), step >= 1.  Errors: E_ARG, E_DEVICE. */
stkfmm_status stkfmm_mlp_forward(const float *params, int64_t batch, const float *x, float *logits,
                                 float *work, void *hip_stream);
stkfmm_status stkfmm_mlp_loss_grad(const float *params, int64_t batch, const float *x, const int32_t *labels,
                                   float *grad, float *loss, float *work, void *hip_stream);
stkfmm_status stkfmm_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr,
                              void *hip_stream);

/* Last error message of the context (never NULL; "" if none). */
const char *stkfmm_last_error(const stkfmm_ctx *ctx);

/* Release the context and its device memory.  NULL is ignored. */
void stkfmm_destroy(stkfmm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* STKFMM_H */
