// Flexible GMRES, the outer Krylov solver of the paper's experiments
// (Section 5, with restarts; right preconditioning by the V-cycle).  The
// Arnoldi basis V (restart + 1 vectors) and the preconditioned directions Z
// (restart vectors) are stored as consecutive vectors of n entries.  Each
// Arnoldi step orthogonalises w = A z_j by classical Gram-Schmidt applied
// twice: h = V^T w and w -= V h, each one streaming pass over the basis.
// The (restart+1) x restart Hessenberg problem lives in device memory and
// is reduced by Givens rotations in a one-thread kernel, so the host reads
// back only the convergence flag.
#include "common.hpp"

namespace specmg {

constexpr int kDotChunk = 16;      // basis vectors per pass of the multi-dot
constexpr int kKryThreads = 256;
constexpr int kKryBlocks = 1024;   // grid of the streaming kernels (4 x 256 CUs)

// part[b][i] = sum over the rows of block b of V_i . w, i < cnt <= kDotChunk
__global__ __launch_bounds__(kKryThreads) void k_mdot_part(const double* __restrict__ V, int64_t pitch, int cnt,
                                                           const double* __restrict__ w, int64_t n,
                                                           double* __restrict__ part) {
    __shared__ double red[kKryThreads / 64][kDotChunk];
    double acc[kDotChunk];
#pragma unroll
    for (int i = 0; i < kDotChunk; ++i) acc[i] = 0.0;
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * blockDim.x) {
        const double wv = w[row];
#pragma unroll
        for (int i = 0; i < kDotChunk; ++i)
            if (i < cnt) acc[i] += V[i * pitch + row] * wv;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kDotChunk; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0) red[wid][i] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        double s = 0.0;
        for (int k = 0; k < kKryThreads / 64; ++k) s += red[k][threadIdx.x];
        part[(size_t)blockIdx.x * kDotChunk + threadIdx.x] = s;
    }
}

// out[i] = sum_b part[b][i] (block i; fixed summation order)
__global__ __launch_bounds__(kKryThreads) void k_mdot_final(const double* __restrict__ part, int nb,
                                                            double* __restrict__ out) {
    __shared__ double red[kKryThreads / 64];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(size_t)b * kDotChunk + i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kKryThreads / 64; ++k) t += red[k];
        out[i] = t;
    }
}

// w += sign * sum_{i < cnt} coef[i] V_i (coefficients in device memory)
__global__ __launch_bounds__(kKryThreads) void k_maxpy(const double* __restrict__ V, int64_t pitch, int cnt,
                                                       const double* __restrict__ coef, double sign,
                                                       double* __restrict__ w, int64_t n) {
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < cnt; ++i) s += coef[i] * V[i * pitch + row];
        w[row] += sign * s;
    }
}

// dst = src * (*factor)
__global__ __launch_bounds__(kKryThreads) void k_scale_dev(double* __restrict__ dst, const double* __restrict__ src,
                                                           const double* __restrict__ factor, int64_t n) {
    const double f = *factor;
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * blockDim.x)
        dst[row] = src[row] * f;
}

// (re)start: beta = ||r|| from nrm2, g = beta e_1, inv = 1 / beta
__global__ void k_gmres_begin(GmresState* st, double thr) {
    const double beta = sqrt(st->nrm2);
    st->beta = beta;
    for (int i = 0; i <= kMaxRestart; ++i) st->g[i] = 0.0;
    st->g[0] = beta;
    st->inv = beta > 0.0 ? 1.0 / beta : 0.0;
    st->res = beta;
    st->done = beta <= thr ? 1 : 0;
}

// Arnoldi step j: column j of H from the two Gram-Schmidt passes and
// ||w||; earlier rotations, the new rotation, g; done when |g_{j+1}| <= thr
// or w vanished (the Krylov space is invariant: the iterate is exact).
__global__ void k_gmres_step(GmresState* st, int j, double thr) {
    constexpr int ld = kMaxRestart + 1;
    double* Hj = st->H + (size_t)j * ld;
    for (int i = 0; i <= j; ++i) Hj[i] = st->h[i] + st->h2[i];
    const double hn = sqrt(st->nrm2);
    Hj[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = st->cs[i] * Hj[i] + st->sn[i] * Hj[i + 1];
        Hj[i + 1] = -st->sn[i] * Hj[i] + st->cs[i] * Hj[i + 1];
        Hj[i] = t;
    }
    const double d = hypot(Hj[j], Hj[j + 1]);
    const double c = d > 0.0 ? Hj[j] / d : 1.0, s = d > 0.0 ? Hj[j + 1] / d : 0.0;
    st->cs[j] = c;
    st->sn[j] = s;
    Hj[j] = d;
    Hj[j + 1] = 0.0;
    st->g[j + 1] = -s * st->g[j];
    st->g[j] = c * st->g[j];
    st->res = fabs(st->g[j + 1]);
    st->inv = hn > 0.0 ? 1.0 / hn : 0.0;
    st->done = (st->res <= thr || !(hn > 0.0)) ? 1 : 0;
    if (!(d > 0.0)) st->done = 2;   // singular Hessenberg column: breakdown
}

// y = R_k^{-1} g_k (R: the rotated, upper triangular H)
__global__ void k_gmres_lsq(GmresState* st, int k) {
    constexpr int ld = kMaxRestart + 1;
    for (int i = k - 1; i >= 0; --i) {
        double v = st->g[i];
        for (int l = i + 1; l < k; ++l) v -= st->H[(size_t)l * ld + i] * st->y[l];
        st->y[i] = v / st->H[(size_t)i * ld + i];
    }
}

// ---------------------------------------------------------------------------
// launchers

static int kry_blocks(int64_t n) {
    const int64_t b = (n + kKryThreads - 1) / kKryThreads;
    return (int)(b < kKryBlocks ? (b < 1 ? 1 : b) : kKryBlocks);
}

size_t mdot_part_doubles() { return (size_t)kKryBlocks * kDotChunk; }

void launch_mdot(const double* V, int64_t pitch, int cnt, const double* w, int64_t n, double* part, double* out,
                 hipStream_t s) {
    const int nb = kry_blocks(n);
    for (int i0 = 0; i0 < cnt; i0 += kDotChunk) {
        const int c = cnt - i0 < kDotChunk ? cnt - i0 : kDotChunk;
        hipLaunchKernelGGL(k_mdot_part, dim3(nb), dim3(kKryThreads), 0, s, V + (size_t)i0 * pitch, pitch, c, w, n,
                           part);
        hipLaunchKernelGGL(k_mdot_final, dim3(c), dim3(kKryThreads), 0, s, part, nb, out + i0);
    }
}

void launch_maxpy(const double* V, int64_t pitch, int cnt, const double* coef, double sign, double* w, int64_t n,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_maxpy, dim3(kry_blocks(n)), dim3(kKryThreads), 0, s, V, pitch, cnt, coef, sign, w, n);
}

void launch_scale_dev(double* dst, const double* src, const double* factor, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_dev, dim3(kry_blocks(n)), dim3(kKryThreads), 0, s, dst, src, factor, n);
}

void launch_gmres_begin(GmresState* st, double thr, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_begin, dim3(1), dim3(1), 0, s, st, thr);
}

void launch_gmres_step(GmresState* st, int j, double thr, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_step, dim3(1), dim3(1), 0, s, st, j, thr);
}

void launch_gmres_lsq(GmresState* st, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_lsq, dim3(1), dim3(1), 0, s, st, k);
}

}  // namespace specmg
