// Coarsest level: the pseudo-inverse A_L^+ of Algorithm 1 (step 5).
//
// A_L is symmetric positive semidefinite with the constants (coefficient
// vector z) as its kernel.  With z normalised and alpha > 0,
//   A_L^+ = (A_L + alpha z z^T)^{-1} - z z^T / alpha,
// so the set-up factors the SPD matrix A_L + alpha z z^T by Cholesky in
// float64 and forms its inverse explicitly; each V-cycle then applies A_L^+
// as one dense matrix-vector product.
//
// Matrices are row-major np x np with np a multiple of 32 (padding rows and
// columns carry an identity).  Blocked right-looking Cholesky with 32 x 32
// tiles: diagonal tile in LDS, panel solve, symmetric rank-32 update of the
// trailing lower triangle.  The inverse is W^T W with W = L^{-1}, W computed
// one 32-column strip per workgroup.
#include "common.hpp"

namespace specmg {

constexpr int NB = 32;

__global__ __launch_bounds__(256) void k_potrf_diag(double* A, int np, int k0, int* bad) {
    __shared__ double T[NB][NB + 1];
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t / NB, j = t % NB;
        T[i][j] = A[(size_t)(k0 + i) * np + k0 + j];
    }
    __syncthreads();
    for (int j = 0; j < NB; ++j) {
        if (threadIdx.x == 0) {
            double d = T[j][j];
            if (!(d > 0.0)) {
                atomicOr(bad, 4);
                d = 1.0;
            }
            T[j][j] = sqrt(d);
        }
        __syncthreads();
        const double ljj = T[j][j];
        for (int i = j + 1 + threadIdx.x; i < NB; i += blockDim.x) T[i][j] /= ljj;
        __syncthreads();
        for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
            const int i = t / NB, c = t % NB;
            if (c > j && i >= c) T[i][c] -= T[i][j] * T[c][j];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t / NB, j = t % NB;
        A[(size_t)(k0 + i) * np + k0 + j] = (j <= i) ? T[i][j] : 0.0;
    }
}

// rows i >= k0+NB: A[i, k0:k0+NB] <- A[i, k0:k0+NB] L_kk^{-T}
__global__ __launch_bounds__(64) void k_trsm_panel(double* A, int np, int k0) {
    __shared__ double Lk[NB][NB + 1];
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t / NB, j = t % NB;
        Lk[i][j] = A[(size_t)(k0 + i) * np + k0 + j];
    }
    __syncthreads();
    const int i = k0 + NB + blockIdx.x * 64 + threadIdx.x;
    if (i >= np) return;
    double x[NB];
    double* row = A + (size_t)i * np + k0;
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = row[j];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double v = x[j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= x[k] * Lk[j][k];
        x[j] = v / Lk[j][j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) row[j] = x[j];
}

// trailing update A[i][j] -= sum_k A[i][k0+k] A[j][k0+k] on lower tiles
__global__ __launch_bounds__(256) void k_syrk_update(double* A, int np, int k0) {
    __shared__ double Pi[NB][NB + 1], Pj[NB][NB + 1];
    // blockIdx.x enumerates lower tiles (ti >= tj) of the trailing matrix
    int b = blockIdx.x, ti = 0;
    while (b > ti) {
        b -= ti + 1;
        ++ti;
    }
    const int tj = b;
    const int base = k0 + NB;
    const int r0 = base + ti * NB, c0 = base + tj * NB;
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t / NB, k = t % NB;
        Pi[i][k] = A[(size_t)(r0 + i) * np + k0 + k];
        Pj[i][k] = A[(size_t)(c0 + i) * np + k0 + k];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t / NB, j = t % NB;
        if (ti == tj && j > i) continue;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < NB; ++k) s += Pi[i][k] * Pj[j][k];
        A[(size_t)(r0 + i) * np + c0 + j] -= s;
    }
}

// W = L^{-1}, one 32-column strip per workgroup, rows marched downwards
__global__ __launch_bounds__(256) void k_trtri_strip(const double* __restrict__ Lm, double* W, int np) {
    __shared__ double Lii[NB][NB + 1];
    __shared__ double R[NB][NB + 1];
    const int J = blockIdx.x;
    const int j0 = J * NB;
    const int nbk = np / NB;
    for (int I = J; I < nbk; ++I) {
        const int i0 = I * NB;
        for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
            const int i = t / NB, j = t % NB;
            Lii[i][j] = Lm[(size_t)(i0 + i) * np + i0 + j];
            double s = (I == J && i == j) ? 1.0 : 0.0;
            // s -= sum_{k in [j0, i0)} L[i0+i][k] W[k][j0+j]
            for (int k = j0; k < i0; ++k) s -= Lm[(size_t)(i0 + i) * np + k] * W[(size_t)k * np + j0 + j];
            R[i][j] = s;
        }
        __syncthreads();
        // forward substitution with Lii, one thread per column of the strip
        if (threadIdx.x < NB) {
            const int j = threadIdx.x;
            for (int i = 0; i < NB; ++i) {
                double v = R[i][j];
                for (int k = 0; k < i; ++k) v -= Lii[i][k] * R[k][j];
                R[i][j] = v / Lii[i][i];
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
            const int i = t / NB, j = t % NB;
            W[(size_t)(i0 + i) * np + j0 + j] = R[i][j];
        }
        __threadfence_block();
        __syncthreads();
    }
    // zero the strip above the diagonal block
    for (size_t t = threadIdx.x; t < (size_t)j0 * NB; t += blockDim.x) {
        const size_t i = t / NB, j = t % NB;
        W[i * np + j0 + j] = 0.0;
    }
}

// A = W^T W (lower tiles computed, then mirrored)
__global__ __launch_bounds__(256) void k_wtw(const double* __restrict__ W, double* A, int np) {
    __shared__ double Ti[NB][NB + 1], Tj[NB][NB + 1];
    int b = blockIdx.x, ti = 0;
    while (b > ti) {
        b -= ti + 1;
        ++ti;
    }
    const int tj = b;
    const int r0 = ti * NB, c0 = tj * NB;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // rows k >= r0 contribute (W lower triangular)
    for (int k0 = r0; k0 < np; k0 += NB) {
        for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
            const int k = t / NB, c = t % NB;
            Ti[k][c] = W[(size_t)(k0 + k) * np + r0 + c];
            Tj[k][c] = W[(size_t)(k0 + k) * np + c0 + c];
        }
        __syncthreads();
        for (int u = 0; u < 4; ++u) {
            const int t = threadIdx.x + 256 * u;
            const int i = t / NB, j = t % NB;
            double s = 0.0;
#pragma unroll 8
            for (int k = 0; k < NB; ++k) s += Ti[k][i] * Tj[k][j];
            acc[u] += s;
        }
        __syncthreads();
    }
    for (int u = 0; u < 4; ++u) {
        const int t = threadIdx.x + 256 * u;
        const int i = t / NB, j = t % NB;
        A[(size_t)(r0 + i) * np + c0 + j] = acc[u];
        A[(size_t)(c0 + j) * np + r0 + i] = acc[u];
    }
}

__global__ void k_rank1(double* A, int np, int n, const double* __restrict__ z, double alpha) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / n), j = (int)(t % n);
        A[(size_t)i * np + j] += alpha * z[i] * z[j];
    }
}

__global__ void k_pad_identity(double* A, int np, int n) {
    const int i = n + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) A[(size_t)i * np + i] = 1.0;
}

void launch_pad_identity(double* a, int np, int n, hipStream_t s) {
    if (np > n) hipLaunchKernelGGL(k_pad_identity, dim3((np - n + 63) / 64), dim3(64), 0, s, a, np, n);
}

int dense_spd_inverse(double* a, int np, double* work, int* bad, hipStream_t s) {
    const int nbk = np / NB;
    for (int kb = 0; kb < nbk; ++kb) {
        const int k0 = kb * NB;
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, a, np, k0, bad);
        const int rest = np - k0 - NB;
        if (rest > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3((rest + 63) / 64), dim3(64), 0, s, a, np, k0);
            const int T = rest / NB;
            hipLaunchKernelGGL(k_syrk_update, dim3(T * (T + 1) / 2), dim3(256), 0, s, a, np, k0);
        }
    }
    hipLaunchKernelGGL(k_trtri_strip, dim3(nbk), dim3(256), 0, s, a, work, np);
    hipLaunchKernelGGL(k_wtw, dim3(nbk * (nbk + 1) / 2), dim3(256), 0, s, work, a, np);
    return (int)hipGetLastError();
}

void launch_add_rank1(double* a, int np, int n, const double* z, double alpha, hipStream_t s) {
    hipLaunchKernelGGL(k_rank1, dim3(1024), dim3(256), 0, s, a, np, n, z, alpha);
}


}  // namespace specmg
