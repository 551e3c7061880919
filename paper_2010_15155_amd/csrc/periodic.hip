// Triply periodic Stokeslet: the root's far images (Sec. III and its
// appendix on periodicity).  The near images (max|n_k| <= 1) are part of the
// tree's shifted lists; the others reach the targets through Stokeslet forces
// F on the root's downward equivalent points: the root's flow is summed
// directly at its upward check points (V), and F = Q V with Q from the host
// (Stokeslet fits and Hasimoto's Ewald split, zero net force).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace kafmm {

namespace {

constexpr double kInv8Pi = 0.039788735772973836;   // 1/(8 pi)

constexpr int kRootChunk = 4096;   // sources per block of the check-surface sum
constexpr int kRootPer = 6;        // check points per thread (M <= 1536)

// part[chunk][3m + a] = 8 pi x the flow at check point X_m (relative to the
// root centre) of the chunk's sources (sorted records: hi, lo position in the
// unit box, f at slots 6..8); FP32 pair sums per LDS tile, FP64 across tiles
// Source kinds of the check-surface sum (sorted records, unit-box units):
//   0 Stokeslet  f at slots 6..8:           G f
//   1 RPY        f, b^2 at 9:              G f + (b^2/6) lap G f
//   2 PVel SL    f, q at 9:                G f - q r/r^3
//   3 PVel DL    D^s (xx xy xz yy yz zz) at 6..11:  -3 r (r.D.r)/r^5
//   4 regularized force and torque: f, t at 9..11, b^2 = 3 eps^2/2 at 12:
//                G f + (b^2/6) lap G f + (t x r)/r^3 (the blobs' far field)
// (all times 8 pi).  Row stride 3M + 3: the last three entries hold the
// chunk's flux moment sum_j w_j y_j (w = q for kind 2, tr D for kind 3, 0
// otherwise; y relative to the root centre), which sets the uniform flow
// that the Stokeslet fit cannot carry (see stokes_far_targets_kernel).
template <int KIND>
__global__ __launch_bounds__(256) void stokes_root_check_kernel(int64_t n, const float *__restrict__ src, int rec,
                                                                const double *__restrict__ X, int M,
                                                                double *__restrict__ part) {
    constexpr int NV = KIND == 3 ? 9 : KIND == 4 ? 10 : 7;
    constexpr bool kFlux = KIND == 2 || KIND == 3;
    __shared__ float tile[256 * NV];
    __shared__ double mred[kFlux ? 3 * 256 : 1];
    double mw[3] = {0.0, 0.0, 0.0};
    const int64_t j0 = int64_t(blockIdx.x) * kRootChunk, j1 = min(n, j0 + kRootChunk);
    float x[kRootPer][3];
    double acc[kRootPer][3];
#pragma unroll
    for (int q = 0; q < kRootPer; ++q) {
        const int m = int(threadIdx.x) + 256 * q;
        for (int k = 0; k < 3; ++k) {
            x[q][k] = m < M ? float(X[3 * m + k]) : 0.0f;
            acc[q][k] = 0.0;
        }
    }
    for (int64_t t0 = j0; t0 < j1; t0 += 256) {
        const int cnt = int(min<int64_t>(256, j1 - t0));
        __syncthreads();
        if (int(threadIdx.x) < cnt) {
            const float *r = src + (t0 + threadIdx.x) * rec;
            float *o = tile + NV * threadIdx.x;
            for (int k = 0; k < 3; ++k) o[k] = float((double(r[k]) - 0.5) + double(r[3 + k]));
            if (kFlux) {
                const double w = KIND == 2 ? double(r[9]) : double(r[6]) + double(r[9]) + double(r[11]);
                for (int k = 0; k < 3; ++k) mw[k] += w * double(o[k]);
            }
            if (KIND == 3) {
                for (int k = 0; k < 6; ++k) o[3 + k] = r[6 + k];
            } else {
                for (int k = 0; k < 3; ++k) o[3 + k] = r[6 + k];
                o[6] = KIND == 1 ? r[9] * (1.0f / 6.0f) : KIND == 2 ? r[9] : KIND == 4 ? r[12] * (1.0f / 6.0f) : 0.0f;
                if (KIND == 4)
                    for (int k = 0; k < 3; ++k) o[7 + k] = r[9 + k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kRootPer; ++q) {
            if (int(threadIdx.x) + 256 * q >= M) continue;
            float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;
            for (int j = 0; j < cnt; ++j) {
                const float *y = tile + NV * j;
                const float r0 = x[q][0] - y[0], r1 = x[q][1] - y[1], r2 = x[q][2] - y[2];
                const float ri = __builtin_amdgcn_rsqf(r0 * r0 + r1 * r1 + r2 * r2);
                const float ri2 = ri * ri, ri3 = ri2 * ri;
                if (KIND == 3) {
                    const float w0 = y[3] * r0 + y[4] * r1 + y[5] * r2;
                    const float w1 = y[4] * r0 + y[6] * r1 + y[7] * r2;
                    const float w2 = y[5] * r0 + y[7] * r1 + y[8] * r2;
                    const float c = -3.0f * (r0 * w0 + r1 * w1 + r2 * w2) * ri3 * ri2;
                    u0 += r0 * c;
                    u1 += r1 * c;
                    u2 += r2 * c;
                } else {
                    const float rdf = r0 * y[3] + r1 * y[4] + r2 * y[5];
                    // G f = f/r + r (r.f)/r^3;  RPY: + (b^2/6)(2 f/r^3 - 6 r (r.f)/r^5);  PVel: - q r/r^3
                    const float cf = KIND == 1 || KIND == 4 ? ri + 2.0f * y[6] * ri3 : ri;
                    const float cr = KIND == 1 || KIND == 4 ? (rdf * ri3) * (1.0f - 6.0f * y[6] * ri2)
                                     : KIND == 2 ? (rdf - y[6]) * ri3
                                                 : rdf * ri3;
                    u0 += y[3] * cf + r0 * cr;
                    u1 += y[4] * cf + r1 * cr;
                    u2 += y[5] * cf + r2 * cr;
                    if (KIND == 4) {    // rotlet (t x r)/r^3
                        u0 += (y[8] * r2 - y[9] * r1) * ri3;
                        u1 += (y[9] * r0 - y[7] * r2) * ri3;
                        u2 += (y[7] * r1 - y[8] * r0) * ri3;
                    }
                }
            }
            acc[q][0] += double(u0);
            acc[q][1] += double(u1);
            acc[q][2] += double(u2);
        }
    }
    double *o = part + int64_t(blockIdx.x) * (3 * M + 3);
#pragma unroll
    for (int q = 0; q < kRootPer; ++q) {
        const int m = int(threadIdx.x) + 256 * q;
        if (m < M)
            for (int k = 0; k < 3; ++k) o[3 * m + k] = acc[q][k];
    }
    if constexpr (kFlux) {
        for (int k = 0; k < 3; ++k) mred[256 * k + threadIdx.x] = mw[k];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w)
                for (int k = 0; k < 3; ++k) mred[256 * k + threadIdx.x] += mred[256 * k + threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x < 3) o[3 * M + threadIdx.x] = mred[256 * threadIdx.x];
    } else {
        if (threadIdx.x < 3) o[3 * M + threadIdx.x] = 0.0;
    }
}

// V[r] = sum over chunks of part[chunk][r], in chunk order (r < 3M + 3)
__global__ __launch_bounds__(256) void stokes_root_reduce_kernel(const double *__restrict__ part, int nchunks, int n3,
                                                                 double *__restrict__ V) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n3) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[int64_t(c) * n3 + r];
    V[r] = s;
}

// F[r] = sum_k Q[r][k] V[k] / (8 pi): one block per row, strided partial
// sums reduced in LDS (a fixed order)
__global__ __launch_bounds__(256) void stokes_far_forces_kernel(const double *__restrict__ Q,
                                                                const double *__restrict__ V, int n3,
                                                                double *__restrict__ F) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    const double *q = Q + int64_t(r) * n3;
    double s = 0.0;
    for (int k = threadIdx.x; k < n3; k += 256) s += q[k] * V[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) F[r] = red[0] * kInv8Pi;
}

// out[perm[i]][a] += scale sum_m G(x_i - z_m) F_m, x_i the sorted target
// (hi + lo, unit box) relative to the root centre; F and z staged in LDS.
// The far images' flow is smooth in the box (z_m lie outside it): FP32 pair
// terms, summed per tile in FP32 and across tiles in FP64.
// Output modes (values of the Stokeslets F at z_m, times 1/(8 pi)):
//   0 Stokeslet      u                                   stride 3
//   1 RPY            u, lap u = 2 F/r^3 - 6 r (r.F)/r^5    stride 6
//   2 PVel           p = 2 (r.F)/r^3, u                   stride 4
//   3 PVelGrad       p, u, grad p, grad u (d_j u_i row-major)  stride 16
//   4 PVelLaplacian  p, u, lap u (= grad p)               stride 7
//   5 Traction       sigma = -p I + grad u + grad u^T
//                          = -6 r r^T (r.F)/r^5          stride 9
//   6 force-torque   u, omega = curl(u)/2 = (F x r)/r^3    stride 6
// with grad p = 2 F/r^3 - 6 r (r.F)/r^5 and
// d_j u_i = (r_i F_j - F_i r_j + delta_ij (r.F))/r^3 - 3 (r.F) r_i r_j/r^5.
// Scales: u by s1 = 1/L, p, sigma, grad u and omega by 1/L^2, lap u and grad p
// by 1/L^3 (unit-box records).
// PVel's flux sources (q, tr D) are potential dipoles in total (zero net
// flux).  Their Ewald sum (the k = 0 mode dropped) has zero mean velocity;
// the Stokeslet fit carries them in divergence-free form, whose transform
// differs from theirs by the constant P/2 at k -> 0 (P = sum_j w_j y_j, the
// flux moment): modes 2-4 remove the resulting uniform flow P/(2 L^3) from u
// (mom = P in unit-box records (w/L), scaled by 1/L like u); derivatives do
// not see it.
template <int OUT>
__global__ __launch_bounds__(256) void stokes_far_targets_kernel(int64_t n, const float *__restrict__ trg,
                                                                 const int32_t *__restrict__ perm,
                                                                 const double *__restrict__ F,
                                                                 const double *__restrict__ Z, int M, double s1,
                                                                 const double *__restrict__ mom,
                                                                 double *__restrict__ out) {
    constexpr bool kP = OUT >= 2;                   // pressure
    constexpr bool kGP = OUT == 1 || OUT == 3 || OUT == 4;   // grad p (= lap u)
    constexpr bool kGU = OUT == 3 || OUT == 5;      // grad u
    constexpr bool kW = OUT == 6;                   // omega
    __shared__ float tile[256 * 6];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool active = i < n;
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
    if (active) {
        const float4 h = reinterpret_cast<const float4 *>(trg)[2 * i];
        const float4 l = reinterpret_cast<const float4 *>(trg)[2 * i + 1];
        x0 = float((double(h.x) - 0.5) + double(l.x));
        x1 = float((double(h.y) - 0.5) + double(l.y));
        x2 = float((double(h.z) - 0.5) + double(l.z));
    }
    double u[3] = {0, 0, 0}, pp = 0.0, gp[3] = {0, 0, 0}, gu[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int j0 = 0; j0 < M; j0 += 256) {
        const int cnt = min(256, M - j0);
        __syncthreads();
        if (int(threadIdx.x) < cnt) {
            const int m = j0 + threadIdx.x;
            float *o = tile + 6 * threadIdx.x;
            for (int k = 0; k < 3; ++k) {
                o[k] = float(Z[3 * m + k]);
                o[3 + k] = float(F[3 * m + k]);
            }
        }
        __syncthreads();
        if (!active) continue;
        float v[3] = {0.0f, 0.0f, 0.0f}, pv = 0.0f, g[3] = {0.0f, 0.0f, 0.0f};
        float h[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int j = 0; j < cnt; ++j) {
            const float *t = tile + 6 * j;
            const float r[3] = {x0 - t[0], x1 - t[1], x2 - t[2]};
            const float ri = __builtin_amdgcn_rsqf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            const float ri2 = ri * ri, ri3 = ri2 * ri;
            const float rdf = r[0] * t[3] + r[1] * t[4] + r[2] * t[5];
            const float rf = rdf * ri3;
#pragma unroll
            for (int a = 0; a < 3; ++a) v[a] += t[3 + a] * ri + r[a] * rf;
            if (kP) pv += rf;
            if (kW) {
                g[0] += (t[4] * r[2] - t[5] * r[1]) * ri3;
                g[1] += (t[5] * r[0] - t[3] * r[2]) * ri3;
                g[2] += (t[3] * r[1] - t[4] * r[0]) * ri3;
            }
            if (kGP) {
                const float c6 = -6.0f * rf * ri2;
#pragma unroll
                for (int a = 0; a < 3; ++a) g[a] += 2.0f * t[3 + a] * ri3 + r[a] * c6;
            }
            if (kGU) {
                const float c3 = -3.0f * rf * ri2;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        h[3 * a + b] += (r[a] * t[3 + b] - t[3 + a] * r[b]) * ri3 + r[a] * r[b] * c3 +
                                        (a == b ? rf : 0.0f);
            }
        }
        for (int a = 0; a < 3; ++a) u[a] += double(v[a]);
        pp += 2.0 * double(pv);
        for (int a = 0; a < 3; ++a) gp[a] += double(g[a]);
        for (int a = 0; a < 9; ++a) gu[a] += double(h[a]);
    }
    if (!active) return;
    constexpr int kStride[7] = {3, 6, 4, 16, 7, 9, 6};
    double *o = out + kStride[OUT] * int64_t(perm[i]);
    const double s2 = s1 * s1, s3 = s2 * s1;
    if (OUT == 0 || OUT == 1 || OUT == 6) {
        for (int k = 0; k < 3; ++k) o[k] += s1 * kInv8Pi * u[k];
        if (OUT == 1)
            for (int k = 0; k < 3; ++k) o[3 + k] += s3 * kInv8Pi * gp[k];
        if (OUT == 6)
            for (int k = 0; k < 3; ++k) o[3 + k] += s2 * kInv8Pi * gp[k];
        return;
    }
    if (OUT == 5) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                o[3 * a + b] += s2 * kInv8Pi * ((a == b ? -pp : 0.0) + gu[3 * a + b] + gu[3 * b + a]);
        return;
    }
    o[0] += s2 * kInv8Pi * pp;
    for (int k = 0; k < 3; ++k) o[1 + k] += s1 * (kInv8Pi * u[k] - 0.5 * mom[k]);
    if (OUT == 3 || OUT == 4)
        for (int k = 0; k < 3; ++k) o[4 + k] += s3 * kInv8Pi * gp[k];
    if (OUT == 3)
        for (int k = 0; k < 9; ++k) o[7 + k] += s2 * kInv8Pi * gu[k];
}

// per-block partial sums of the first ncomp (<= 9) values of each source
// (stride apart) and of their absolute values: part[block][ncomp + 1]
__global__ __launch_bounds__(256) void value_partials_kernel(int64_t n, const double *__restrict__ f, int stride,
                                                             int ncomp, double *__restrict__ part) {
    __shared__ double s[10][256];
    double a[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        for (int k = 0; k < ncomp; ++k) {
            const double v = f[stride * i + k];
            a[k] += v;
            a[9] += fabs(v);
        }
    for (int k = 0; k < 10; ++k) s[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w)
            for (int k = 0; k < 10; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < ncomp; ++k) part[(ncomp + 1) * blockIdx.x + k] = s[k][0];
        part[(ncomp + 1) * blockIdx.x + ncomp] = s[9][0];
    }
}

}  // namespace

int stokes_root_chunks(int64_t n) { return int((n + kRootChunk - 1) / kRootChunk); }

hipError_t launch_stokes_root_check(int kind, int64_t n_src, const float *src, int rec, const double *X, int M,
                                    double *part, hipStream_t s) {
    const int nch = stokes_root_chunks(n_src);
    if (nch == 0) return hipSuccess;
    if (M > 256 * kRootPer) return hipErrorInvalidValue;
    if (rec < (kind == 0 ? 9 : kind == 3 ? 12 : kind == 4 ? 13 : 10)) return hipErrorInvalidValue;
    const dim3 g(nch), b(256);
    switch (kind) {
        case 0: hipLaunchKernelGGL(stokes_root_check_kernel<0>, g, b, 0, s, n_src, src, rec, X, M, part); break;
        case 1: hipLaunchKernelGGL(stokes_root_check_kernel<1>, g, b, 0, s, n_src, src, rec, X, M, part); break;
        case 2: hipLaunchKernelGGL(stokes_root_check_kernel<2>, g, b, 0, s, n_src, src, rec, X, M, part); break;
        case 3: hipLaunchKernelGGL(stokes_root_check_kernel<3>, g, b, 0, s, n_src, src, rec, X, M, part); break;
        case 4: hipLaunchKernelGGL(stokes_root_check_kernel<4>, g, b, 0, s, n_src, src, rec, X, M, part); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stokes_far_forces(int nchunks, const double *Q, int M, const double *part, double *V, double *F,
                                    hipStream_t s) {
    const int n3 = 3 * M, n3p = 3 * M + 3;
    hipLaunchKernelGGL(stokes_root_reduce_kernel, dim3((n3p + 255) / 256), dim3(256), 0, s, part, nchunks, n3p, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stokes_far_forces_kernel, dim3(n3), dim3(256), 0, s, Q, V, n3, F);
    return hipGetLastError();
}

hipError_t launch_stokes_far_targets(int64_t n, const float *trg, const int32_t *perm, int mode, const double *F,
                                     const double *Z, int M, double inv_len, const double *mom, double *out,
                                     hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 g(int((n + 255) / 256)), b(256);
    switch (mode) {
#define KAFMM_FAR_TARGETS(K)                                                                                     \
    case K: hipLaunchKernelGGL(stokes_far_targets_kernel<K>, g, b, 0, s, n, trg, perm, F, Z, M, inv_len, mom, out); \
        break;
        KAFMM_FAR_TARGETS(0)
        KAFMM_FAR_TARGETS(1)
        KAFMM_FAR_TARGETS(2)
        KAFMM_FAR_TARGETS(3)
        KAFMM_FAR_TARGETS(4)
        KAFMM_FAR_TARGETS(5)
        KAFMM_FAR_TARGETS(6)
#undef KAFMM_FAR_TARGETS
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_value_partials(int64_t n, const double *f, int stride, int ncomp, int nblocks, double *part,
                                 hipStream_t s) {
    if (ncomp < 1 || ncomp > 9) return hipErrorInvalidValue;
    hipLaunchKernelGGL(value_partials_kernel, dim3(nblocks), dim3(256), 0, s, n, f, stride, ncomp, part);
    return hipGetLastError();
}

}  // namespace kafmm
