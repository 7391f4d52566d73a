// Coarsest level (Algorithm 1, step 5): the dense inverse of the regularised
// coarsest matrix A_L + alpha z z^T, which the V-cycle applies as one dense
// matrix-vector product.
//
// Matrices are row-major np x np with np a multiple of 32 (padding rows and
// columns carry an identity).  Cholesky A = L L^T is right-looking in panels
// of KB = 256 columns: inside a panel, 32 x 32 diagonal tiles in LDS, a panel
// solve and rank-32 updates restricted to the panel; after the panel, one
// rank-KB update of the trailing lower triangle.  W = L^{-1}: every KB x KB
// diagonal block inverted at once, then halves joined bottom-up,
// W21 = -W22 (L21 W11).  Finally A^{-1} = W^T W.  The rank-KB updates and
// the products run on the FP64 matrix cores (k_gemm).
#include "common.hpp"

namespace specmg {

constexpr int NB = 32;
constexpr int KB = 256;   // panel width of the Cholesky factorisation, leaf of the triangular inverse

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

enum { OPN = 0, OPT = 1 };
typedef double dbl4 __attribute__((ext_vector_type(4)));

// lower tile (ti >= tj) of a T x T tile grid from a linear block index
__device__ __forceinline__ void lower_tile(int b, int& ti, int& tj) {
    int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    ti = i;
    tj = b - i * (i + 1) / 2;
}

// W_JJ = L_JJ^{-1} for every KB x KB diagonal block (blockIdx.y; the last
// one may be narrower): one workgroup per 32-column strip of the block, rows
// marched downwards
__global__ __launch_bounds__(256) void k_trtri_diag(const double* __restrict__ Lm, double* W, int np) {
    __shared__ double Lii[NB][NB + 1];
    __shared__ double R[NB][NB + 1];
    const int o = blockIdx.y * KB;
    const int nbk = min(KB, np - o) / NB;
    const int J = blockIdx.x;
    if (J >= nbk) return;   // whole workgroup
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

// ---------------------------------------------------------------------------
// FP64 matrix-core GEMM: C (M x N) = alpha op(A) op(B) over k in [kbeg, kend),
// a 128 x 128 tile per 256-thread workgroup, wave w owning the 64 x 64
// quarter (rows 64 (w >> 1), columns 64 (w & 1)) as 4 x 4 blocks of
// v_mfma_f64_16x16x4f64.  Operand lanes: A(i, k) with i = lane % 16,
// k = lane / 16; B(k, j) with j = lane % 16, k = lane / 16; result element r
// of a block in lane l is (l / 16 + 4 r, l % 16) of the block.  k chunks of
// 16 are staged through LDS; the next chunk's loads are issued before the
// current chunk's products.
//   kb_mode: 0 kbeg = 0; 1 kbeg = j0 (B lower triangular); 2 kbeg = i0 (A^T
//            of a lower triangular matrix)
//   ke_mode: 0 kend = K; 1 kend = min(i0 + 128, K) (A lower triangular)
//   lower:   the grid enumerates the lower tiles (ti >= tj) of a square C
//   EPI 0: C = alpha acc;  1: C -= acc on i >= j;  2: C = acc on i >= j, mirrored
constexpr int GT = 128;
constexpr int GK = 16;

struct GemmArgs {
    const double* A;
    const double* B;
    double* C;
    int lda, ldb, ldc;
    int M, N, K;
    double alpha;
    int kb_mode, ke_mode, lower;
};

template <int AOP, int BOP, int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm(GemmArgs g) {
    __shared__ double As[GK][GT + 1], Bs[GK][GT + 1];
    int ti, tj;
    if (g.lower) {
        lower_tile(blockIdx.x, ti, tj);
    } else {
        ti = blockIdx.x;
        tj = blockIdx.y;
    }
    const int i0 = ti * GT, j0 = tj * GT;
    const int kbeg = g.kb_mode == 1 ? j0 : (g.kb_mode == 2 ? i0 : 0);
    const int kend = g.ke_mode == 1 ? min(i0 + GT, g.K) : g.K;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
    const int li = l & 15, lk = l >> 4;
    dbl4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = dbl4{0.0, 0.0, 0.0, 0.0};
    // staging: 4 pairs of A and 4 of B per thread and chunk, each pair two
    // elements adjacent in memory (along k for OPN A / OPT B, along i or j
    // otherwise); K bounds are multiples of 16, so a pair never straddles kend
    double2 ra[4], rb[4];
    auto a_slot = [&](int u, int& ia, int& ka) {
        const int e = t + 256 * u;
        if (AOP == OPN) { ia = e >> 3; ka = 2 * (e & 7); }
        else { ia = 2 * (e & 63); ka = e >> 6; }
    };
    auto b_slot = [&](int u, int& jb, int& kb) {
        const int e = t + 256 * u;
        if (BOP == OPN) { jb = 2 * (e & 63); kb = e >> 6; }
        else { jb = e >> 3; kb = 2 * (e & 7); }
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int ia, ka, jb, kb;
            a_slot(u, ia, ka);
            b_slot(u, jb, kb);
            const int gi = i0 + ia, gka = k0 + ka;
            const bool va = gi < g.M && gka < kend;
            ra[u] = va ? *reinterpret_cast<const double2*>(AOP == OPN ? g.A + (size_t)gi * g.lda + gka
                                                                      : g.A + (size_t)gka * g.lda + gi)
                       : double2{0.0, 0.0};
            const int gj = j0 + jb, gkb = k0 + kb;
            const bool vb = gj < g.N && gkb < kend;
            rb[u] = vb ? *reinterpret_cast<const double2*>(BOP == OPN ? g.B + (size_t)gkb * g.ldb + gj
                                                                      : g.B + (size_t)gj * g.ldb + gkb)
                       : double2{0.0, 0.0};
        }
    };
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int ia, ka, jb, kb;
            a_slot(u, ia, ka);
            b_slot(u, jb, kb);
            if (AOP == OPN) {
                As[ka][ia] = ra[u].x;
                As[ka + 1][ia] = ra[u].y;
            } else {
                As[ka][ia] = ra[u].x;
                As[ka][ia + 1] = ra[u].y;
            }
            if (BOP == OPN) {
                Bs[kb][jb] = rb[u].x;
                Bs[kb][jb + 1] = rb[u].y;
            } else {
                Bs[kb][jb] = rb[u].x;
                Bs[kb + 1][jb] = rb[u].y;
            }
        }
        __syncthreads();
        if (k0 + GK < kend) load(k0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK / 4; ++kk) {
            const int k = 4 * kk + lk;
            double a[4], b[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) a[m] = As[k][wr + 16 * m + li];
#pragma unroll
            for (int n = 0; n < 4; ++n) b[n] = Bs[k][wc + 16 * n + li];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[n], acc[m][n], 0, 0, 0);
        }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr + 16 * m + lk + 4 * r, j = j0 + wc + 16 * n + li;
                if (i >= g.M || j >= g.N) continue;
                const double v = acc[m][n][r];
                if (EPI == 0) {
                    g.C[(size_t)i * g.ldc + j] = g.alpha * v;
                } else if (EPI == 1) {
                    if (i >= j) g.C[(size_t)i * g.ldc + j] -= v;
                } else {
                    if (i >= j) {
                        g.C[(size_t)i * g.ldc + j] = v;
                        g.C[(size_t)j * g.ldc + i] = v;
                    }
                }
            }
}

template <int AOP, int BOP, int EPI>
static void launch_gemm(const GemmArgs& g, hipStream_t s) {
    const int tm = (g.M + GT - 1) / GT, tn = (g.N + GT - 1) / GT;
    const dim3 grid = g.lower ? dim3(tm * (tm + 1) / 2) : dim3(tm, tn);
    if (tm > 0 && tn > 0) hipLaunchKernelGGL((k_gemm<AOP, BOP, EPI>), grid, dim3(256), 0, s, g);
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

// W[o:e, o:e] = L[o:e, o:e]^{-1} for the KB-blocks [b0, b1) (o = KB b0,
// e = min(KB b1, np)), leaves already inverted: inv([L11 0; L21 L22]) =
// [W11 0; -W22 L21 W11  W22], the two halves first (post-order), then
// P = L21 W11 (W11 lower triangular: k >= j) and W21 = -W22 P (W22 lower
// triangular: k <= i) as matrix-core GEMMs; P lives in tbuf.
static void trtri_node(const double* Lm, double* W, double* P, int np, int b0, int b1, hipStream_t s) {
    if (b1 - b0 < 2) return;
    const int bm = (b0 + b1) / 2;
    trtri_node(Lm, W, P, np, b0, bm, s);
    trtri_node(Lm, W, P, np, bm, b1, s);
    const int o = KB * b0, h = KB * (bm - b0), n = std::min(KB * b1, np) - o;
    GemmArgs g{};
    g.A = Lm + (size_t)(o + h) * np + o;
    g.lda = np;
    g.B = W + (size_t)o * np + o;
    g.ldb = np;
    g.C = P;
    g.ldc = h;
    g.M = n - h;
    g.N = h;
    g.K = h;
    g.alpha = 1.0;
    g.kb_mode = 1;
    launch_gemm<OPN, OPN, 0>(g, s);
    GemmArgs q{};
    q.A = W + (size_t)(o + h) * np + o + h;
    q.lda = np;
    q.B = P;
    q.ldb = h;
    q.C = W + (size_t)(o + h) * np + o;
    q.ldc = np;
    q.M = n - h;
    q.N = h;
    q.K = n - h;
    q.alpha = -1.0;
    q.ke_mode = 1;
    launch_gemm<OPN, OPN, 0>(q, s);
}

size_t dense_spd_inverse_tbuf_doubles(int np) {
    // P of the root node of trtri_node, the largest
    const int nb = (np + KB - 1) / KB;
    const size_t h = (size_t)KB * (nb / 2);
    return nb < 2 ? 1 : (size_t)(np - h) * h;
}

int dense_spd_inverse(double* a, int np, double* work, double* tbuf, int* bad, hipStream_t s) {
    if (np % NB) return (int)hipErrorInvalidValue;
    // ---- Cholesky, panels of KB columns; the trailing update on the matrix cores
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
            // A[i][j] -= sum_{k in panel} A[i][k] A[j][k], i >= j >= j0
            GemmArgs g{};
            g.A = a + (size_t)j0 * np + k0;
            g.lda = np;
            g.B = g.A;
            g.ldb = np;
            g.C = a + (size_t)j0 * np + j0;
            g.ldc = np;
            g.M = g.N = np - j0;
            g.K = kw;
            g.alpha = 1.0;
            g.lower = 1;
            launch_gemm<OPN, OPT, 1>(g, s);
        }
    }
    // ---- W = L^{-1}: the KB x KB diagonal blocks, then the recursive halves
    hipError_t e = hipMemsetAsync(work, 0, (size_t)np * np * sizeof(double), s);
    if (e != hipSuccess) return (int)e;
    const int nb = (np + KB - 1) / KB;
    hipLaunchKernelGGL(k_trtri_diag, dim3(KB / NB, nb), dim3(256), 0, s, a, work, np);
    trtri_node(a, work, tbuf, np, 0, nb, s);
    // ---- A^{-1} = W^T W (lower tiles, mirrored; W[k][i] = 0 for k < i)
    {
        GemmArgs g{};
        g.A = work;
        g.lda = np;
        g.B = work;
        g.ldb = np;
        g.C = a;
        g.ldc = np;
        g.M = g.N = g.K = np;
        g.alpha = 1.0;
        g.kb_mode = 2;
        g.lower = 1;
        launch_gemm<OPT, OPN, 2>(g, s);
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return (int)e;
    return (int)hipGetLastError();
}

void launch_add_rank1(double* a, int np, int n, const double* z, double alpha, hipStream_t s) {
    hipLaunchKernelGGL(k_rank1, dim3(1024), dim3(256), 0, s, a, np, n, z, alpha);
}


}  // namespace specmg
