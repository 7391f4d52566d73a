// Coarsest level (Algorithm 1, step 5): the dense inverse of the regularised
// coarsest matrix A_L + alpha z z^T, which the V-cycle applies as one dense
// matrix-vector product.
//
// Matrices are row-major np x np with np a multiple of 32 (padding rows and
// columns carry an identity).  Cholesky A = L L^T is right-looking in panels
// of KB = 256 columns: inside a panel, 32 x 32 diagonal tiles in LDS, a panel
// solve and rank-32 updates restricted to the panel; after the panel, one
// rank-KB update of the trailing lower triangle.  W = L^{-1} is built from the
// bottom-right panel upwards: W_JJ = L_JJ^{-1}, then
// W[J+1:, J] = -(W[J+1:, J+1:] L[J+1:, J]) W_JJ.  Finally A^{-1} = W^T W.
// The rank-KB updates and the three products share one register-tiled
// FP64 tile product (64 x 64 outputs per 256-thread workgroup, 4 x 4 per
// thread, 16-deep k chunks staged in LDS).
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

// inside a panel: A[i][j] -= sum_{k < 32} A[i][kk+k] A[j][kk+k] for the lower
// 32 x 32 tiles (ti >= tj) of rows >= kk+32 whose column tile tj < ntc
__global__ __launch_bounds__(256) void k_syrk_panel(double* A, int np, int kk, int T) {
    __shared__ double Pi[NB][NB + 1], Pj[NB][NB + 1];
    int b = blockIdx.x, tj = 0;
    while (b >= T - tj) {
        b -= T - tj;
        ++tj;
    }
    const int ti = tj + b;
    const int base = kk + NB;
    const int r0 = base + ti * NB, c0 = base + tj * NB;
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t / NB, k = t % NB;
        Pi[i][k] = A[(size_t)(r0 + i) * np + kk + k];
        Pj[i][k] = A[(size_t)(c0 + i) * np + kk + k];
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

// ---------------------------------------------------------------------------
// register-tiled FP64 tile product
constexpr int KB = 256;   // outer panel width
constexpr int TG = 64;    // output tile edge
constexpr int TK = 16;    // k chunk
enum { OPN = 0, OPT = 1 };

// acc[r][c] += sum_{k in [kbeg, kend)} a(i, k) b(k, j) for the rows
// i = i0 + ty + 16 r and columns j = j0 + tx + 16 c of a 64 x 64 tile, with
//   a(i, k) = A[i lda + k] (AOP = OPN) or A[k lda + i] (OPT),
//   b(k, j) = B[k ldb + j] (BOP = OPN) or B[j ldb + k] (OPT);
// rows >= M and columns >= N read zero.  Called by all 256 threads.
template <int AOP, int BOP>
__device__ __forceinline__ void tile_product(const double* __restrict__ A, int lda, const double* __restrict__ B,
                                             int ldb, int M, int N, int i0, int j0, int kbeg, int kend,
                                             double (&acc)[4][4], double (*As)[TG + 1], double (*Bs)[TG + 1]) {
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = t + 256 * u;
            const int ia = AOP == OPN ? e / TK : e % TG, ka = AOP == OPN ? e % TK : e / TG;
            const int gi = i0 + ia, gka = k0 + ka;
            double v = 0.0;
            if (gi < M && gka < kend) v = AOP == OPN ? A[(size_t)gi * lda + gka] : A[(size_t)gka * lda + gi];
            As[ka][ia] = v;
            const int jb = BOP == OPN ? e % TG : e / TK, kb = BOP == OPN ? e / TG : e % TK;
            const int gj = j0 + jb, gkb = k0 + kb;
            double w = 0.0;
            if (gj < N && gkb < kend) w = BOP == OPN ? B[(size_t)gkb * ldb + gj] : B[(size_t)gj * ldb + gkb];
            Bs[kb][jb] = w;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TK; ++k) {
            double av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = As[k][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = Bs[k][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_fma(av[r], bv[c], acc[r][c]);
        }
        __syncthreads();
    }
}

// lower tile (ti >= tj) of a T x T tile grid from a linear block index
__device__ __forceinline__ void lower_tile(int b, int& ti, int& tj) {
    int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    ti = i;
    tj = b - i * (i + 1) / 2;
}

// after a panel [k0, k0+kw): A[i][j] -= sum_k A[i][k] A[j][k] for i >= j >= j0
__global__ __launch_bounds__(256) void k_chol_update(double* A, int np, int k0, int kw, int j0) {
    __shared__ double As[TK][TG + 1], Bs[TK][TG + 1];
    int ti, tj;
    lower_tile(blockIdx.x, ti, tj);
    const int i0 = j0 + ti * TG, c0 = j0 + tj * TG;
    double acc[4][4] = {};
    tile_product<OPN, OPT>(A, np, A, np, np, np, i0, c0, k0, k0 + kw, acc, As, Bs);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty + 16 * r, j = c0 + tx + 16 * c;
            if (i < np && j < np && i >= j) A[(size_t)i * np + j] -= acc[r][c];
        }
}

// W_JJ = L_JJ^{-1} for the kb x kb diagonal block at o: one workgroup per
// 32-column strip of the block, rows marched downwards
__global__ __launch_bounds__(256) void k_trtri_diag(const double* __restrict__ Lm, double* W, int np, int o,
                                                    int nbk) {
    __shared__ double Lii[NB][NB + 1];
    __shared__ double R[NB][NB + 1];
    const int J = blockIdx.x;
    const int j0 = o + J * NB;
    for (int I = J; I < nbk; ++I) {
        const int i0 = o + I * NB;
        for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
            const int i = t / NB, j = t % NB;
            Lii[i][j] = Lm[(size_t)(i0 + i) * np + i0 + j];
            double s = (I == J && i == j) ? 1.0 : 0.0;
            for (int k = j0; k < i0; ++k) s -= Lm[(size_t)(i0 + i) * np + k] * W[(size_t)k * np + j0 + j];
            R[i][j] = s;
        }
        __syncthreads();
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
}

// T[i][c] = sum_{k in [r0, i]} W[i][k] L[k][j0 + c] for rows i >= r0 = j0 + kb
// (W lower triangular, zero above the diagonal), columns c < kb
__global__ __launch_bounds__(256) void k_trmm_panel(const double* __restrict__ W, const double* __restrict__ Lm,
                                                    double* __restrict__ T, int np, int j0, int kb) {
    __shared__ double As[TK][TG + 1], Bs[TK][TG + 1];
    const int r0 = j0 + kb;
    const int i0 = r0 + blockIdx.x * TG, c0 = blockIdx.y * TG;
    double acc[4][4] = {};
    const int kend = min(i0 + TG, np);
    tile_product<OPN, OPN>(W, np, Lm + j0, np, np, kb, i0, c0, r0, kend, acc, As, Bs);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty + 16 * r, j = c0 + tx + 16 * c;
            if (i < np && j < kb) T[(size_t)i * KB + j] = acc[r][c];
        }
}

// W[i][j0 + c] = -sum_k T[i][k] W[j0 + k][j0 + c] for rows i >= j0 + kb
__global__ __launch_bounds__(256) void k_panel_times_diag(const double* __restrict__ T, double* W, int np, int j0,
                                                          int kb) {
    __shared__ double As[TK][TG + 1], Bs[TK][TG + 1];
    const int r0 = j0 + kb;
    const int i0 = r0 + blockIdx.x * TG, c0 = blockIdx.y * TG;
    double acc[4][4] = {};
    tile_product<OPN, OPN>(T, KB, W + (size_t)j0 * np + j0, np, np, kb, i0, c0, c0, kb, acc, As, Bs);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty + 16 * r, j = c0 + tx + 16 * c;
            if (i < np && j < kb) W[(size_t)i * np + j0 + j] = -acc[r][c];
        }
}

// A = W^T W on lower tiles (ti >= tj), mirrored: W[k][i] = 0 for k < i
__global__ __launch_bounds__(256) void k_wtw(const double* __restrict__ W, double* A, int np) {
    __shared__ double As[TK][TG + 1], Bs[TK][TG + 1];
    int ti, tj;
    lower_tile(blockIdx.x, ti, tj);
    const int i0 = ti * TG, c0 = tj * TG;
    double acc[4][4] = {};
    tile_product<OPT, OPN>(W, np, W, np, np, np, i0, c0, i0, np, acc, As, Bs);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty + 16 * r, j = c0 + tx + 16 * c;
            if (i < np && j < np && i >= j) {
                A[(size_t)i * np + j] = acc[r][c];
                A[(size_t)j * np + i] = acc[r][c];
            }
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

size_t dense_spd_inverse_tbuf_doubles(int np) { return (size_t)np * KB; }

int dense_spd_inverse(double* a, int np, double* work, double* tbuf, int* bad, hipStream_t s) {
    if (np % NB) return (int)hipErrorInvalidValue;
    // ---- Cholesky, panels of KB columns
    for (int k0 = 0; k0 < np; k0 += KB) {
        const int kw = std::min(KB, np - k0);
        for (int kk = k0; kk < k0 + kw; kk += NB) {
            hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, a, np, kk, bad);
            const int rest = np - kk - NB;
            if (rest > 0) {
                hipLaunchKernelGGL(k_trsm_panel, dim3((rest + 63) / 64), dim3(64), 0, s, a, np, kk);
                const int T = rest / NB, ntc = (k0 + kw - kk - NB) / NB;
                const int blocks = ntc * T - ntc * (ntc - 1) / 2;
                if (blocks > 0) hipLaunchKernelGGL(k_syrk_panel, dim3(blocks), dim3(256), 0, s, a, np, kk, T);
            }
        }
        const int j0 = k0 + kw;
        if (j0 < np) {
            const int T = (np - j0 + TG - 1) / TG;
            hipLaunchKernelGGL(k_chol_update, dim3(T * (T + 1) / 2), dim3(256), 0, s, a, np, k0, kw, j0);
        }
    }
    // ---- W = L^{-1}, panels from the bottom-right
    hipError_t e = hipMemsetAsync(work, 0, (size_t)np * np * sizeof(double), s);
    if (e != hipSuccess) return (int)e;
    const int last = ((np - 1) / KB) * KB;
    for (int j0 = last; j0 >= 0; j0 -= KB) {
        const int kb = std::min(KB, np - j0);
        hipLaunchKernelGGL(k_trtri_diag, dim3(kb / NB), dim3(256), 0, s, a, work, np, j0, kb / NB);
        const int m = np - j0 - kb;
        if (m > 0) {
            const dim3 grid((m + TG - 1) / TG, (kb + TG - 1) / TG);
            hipLaunchKernelGGL(k_trmm_panel, grid, dim3(256), 0, s, work, a, tbuf, np, j0, kb);
            hipLaunchKernelGGL(k_panel_times_diag, grid, dim3(256), 0, s, tbuf, work, np, j0, kb);
        }
    }
    // ---- A^{-1} = W^T W
    {
        const int T = (np + TG - 1) / TG;
        hipLaunchKernelGGL(k_wtw, dim3(T * (T + 1) / 2), dim3(256), 0, s, work, a, np);
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return (int)e;
    return (int)hipGetLastError();
}

void launch_add_rank1(double* a, int np, int n, const double* z, double alpha, hipStream_t s) {
    hipLaunchKernelGGL(k_rank1, dim3(1024), dim3(256), 0, s, a, np, n, z, alpha);
}


}  // namespace specmg
