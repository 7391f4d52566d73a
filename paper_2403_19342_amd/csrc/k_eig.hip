// Batched local eigensolves of the set-up phase (Section 3).
//
// Level 2 (eq. spepb): on every 8^3 element K, the smallest eigenpairs of
//   A_K phi = lambda S_K phi,  S_K = diag(tr kappa~),
// solved in the symmetric form A~ x = lambda x with A~ = S^-1/2 A_K S^-1/2,
// phi = S^-1/2 x (so phi^T S phi = 1, the normalisation of Section 3).
// Levels >= 3 (eq. spectral cc): on every parent element E the restricted
// problem H_E v = lambda v with H_E = B_E^T A_E B_E assembled from the level
// below (its Gram is the identity for S-normalised bases).
//
// Method: Chebyshev-filtered subspace iteration.  One workgroup per element
// holds a block of M vectors; each cycle applies a degree-DEG Chebyshev
// polynomial that damps the unwanted interval [a, b] (b: Gershgorin bound,
// a: largest Ritz value of the block), re-orthonormalises by Cholesky-QR
// (twice) and performs Rayleigh-Ritz with a one-wavefront parallel cyclic
// Jacobi eigensolver.  Only operator applications and M x M reductions are
// needed, so the whole solve stays in registers and LDS.
#include "common.hpp"

namespace specmg {

constexpr int kDeg = 20;          // Chebyshev degree per cycle of a relaxed, warm-started solve
constexpr int kDegExact = 40;     // ... of an exact solve (fewer cycles, so fewer orthonormalisations
                                  //     and Rayleigh-Ritz steps per filtered vector)
constexpr int kMaxCycles = 300;
constexpr int kMaxEigWaves = 12;   // workgroups of at most 768 threads
constexpr int kWarmCycles = 4;     // cycles a learned start gets to reach the relaxed residual


__device__ __forceinline__ double hash_noise(unsigned a, unsigned b, unsigned c) {
    unsigned h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u ^ (c + 0x165667B1u) * 0xC2B2AE3Du;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return (double)(h & 0xFFFFFF) / 8388608.0 - 1.0;   // [-1, 1)
}

// low-frequency cosine modes (p, q, r) by increasing p^2+q^2+r^2
__constant__ unsigned char kModes[16][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1},
    {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {2, 1, 0}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}};

template <typename T>
__device__ __forceinline__ T harm_e(T a, T b) {
    const T s = a + b;
    return s > T(0) ? (T(2) * a * b) / s : T(0);
}

// ---------------------------------------------------------------------------
// small dense helpers on LDS, run by one thread or one wavefront

// Circle-method round robin on M players (M even): in round r player M-1
// meets player r and every other pair (i, j) has i + j = 2r modulo M-1.
template <int M>
__device__ __forceinline__ int jac_partner(int i, int r) {
    constexpr int K = M - 1;
    if (i == K) return r;
    if (i == r) return K;
    int j = 2 * r - i;
    j = j < 0 ? j + K : (j >= K ? j - K : j);
    return j;
}

// Rotation (c, s) that annihilates H[p][q] (p < q): the rotated rows are
// p' = c p - s q and q' = s p + c q.
__device__ __forceinline__ void jac_rot(const double* H, int M, int p, int q, double& c, double& s) {
    const double hpp = H[p * M + p], hqq = H[q * M + q], hpq = H[p * M + q];
    c = 1.0;
    s = 0.0;
    if (hpq != 0.0) {
        const double tt = (hqq - hpp) / (2.0 * hpq);
        const double t = (tt >= 0.0 ? 1.0 : -1.0) / (fabs(tt) + sqrt(tt * tt + 1.0));
        c = 1.0 / sqrt(t * t + 1.0);
        s = t * c;
    }
}

// Symmetric eigendecomposition H = Q diag(th) Q^T, eigenvalues ascending,
// by parallel cyclic Jacobi in wavefront 0: each round applies M/2 disjoint
// rotations at once; lanes 0..M-1 derive the round's rotations (scr holds
// the cosines and sines), then every lane applies them to its own elements:
// a round is one rotation phase, one read phase and one write phase.  Stops
// when the largest off-diagonal entry is below 1e-15 times the largest
// diagonal entry.  H (M*M) is destroyed; Q (M*M)
// receives the eigenvectors as columns.  Must be called by all threads.
template <int M>
__device__ __forceinline__ void jacobi_eig(double* H, double* Q, double* th, double* scr, int* iscr) {
    static_assert(M % 2 == 0 && M <= 26, "Jacobi block size");
    constexpr int MM = M * M;
    constexpr int PER = (MM + 63) / 64;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int ei[PER], ej[PER];
        bool ev[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = lane + 64 * u;
            ev[u] = t < MM;
            ei[u] = ev[u] ? t / M : 0;
            ej[u] = ev[u] ? t % M : 0;
            if (ev[u]) Q[t] = (ei[u] == ej[u]) ? 1.0 : 0.0;
        }
        wave_sync();
#pragma unroll 1
        for (int sweep = 0; sweep < 30; ++sweep) {
            double off = 0.0, dg = 0.0;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const double h = ev[u] ? fabs(H[ei[u] * M + ej[u]]) : 0.0;
                if (ei[u] != ej[u]) off = fmax(off, h);
                else dg = fmax(dg, h);
            }
            off = wave_max(off);
            dg = wave_max(dg);
            if (off <= 1e-15 * dg || off == 0.0) break;
#pragma unroll 1
            for (int r = 0; r < M - 1; ++r) {
                // the round's M/2 rotations, once each: lane i < M stores the
                // rotation of its pair (both members hold the same one)
                if (lane < M) {
                    const int pl = jac_partner<M>(lane, r);
                    double cl, sl;
                    jac_rot(H, M, lane < pl ? lane : pl, lane < pl ? pl : lane, cl, sl);
                    scr[lane] = cl;
                    scr[M + lane] = sl;
                }
                wave_sync();
                double nh[PER], nq[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int i = ei[u], j = ej[u];
                    const int pi = jac_partner<M>(i, r), pj = jac_partner<M>(j, r);
                    const int ai = i < pi ? i : pi, bi = i < pi ? pi : i;
                    const int aj = j < pj ? j : pj, bj = j < pj ? pj : j;
                    const double ci = scr[i], si = scr[M + i], cj = scr[j], sj = scr[M + j];
                    const double wra = (i == ai) ? ci : si, wrb = (i == ai) ? -si : ci;
                    const double wca = (j == aj) ? cj : sj, wcb = (j == aj) ? -sj : cj;
                    nh[u] = wra * (wca * H[ai * M + aj] + wcb * H[ai * M + bj]) +
                            wrb * (wca * H[bi * M + aj] + wcb * H[bi * M + bj]);
                    // the annihilated entry of a rotated pair is zero exactly
                    if (ai == aj && bi == bj && i != j) nh[u] = 0.0;
                    nq[u] = wca * Q[i * M + aj] + wcb * Q[i * M + bj];
                }
                wave_sync();
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    if (ev[u]) {
                        H[ei[u] * M + ej[u]] = nh[u];
                        Q[ei[u] * M + ej[u]] = nq[u];
                    }
                }
                wave_sync();
            }
        }
        // ascending order: lane k < M finds the rank of H[k][k]
        if (lane < M) {
            const double hk = H[lane * M + lane];
            int rank = 0;
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const double hl = H[l * M + l];
                rank += (hl < hk || (hl == hk && l < lane)) ? 1 : 0;
            }
            iscr[rank] = lane;
            th[rank] = hk;
        }
        wave_sync();
        double nq[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) nq[u] = ev[u] ? Q[ei[u] * M + iscr[ej[u]]] : 0.0;
        wave_sync();
#pragma unroll
        for (int u = 0; u < PER; ++u)
            if (ev[u]) Q[ei[u] * M + ej[u]] = nq[u];
    }
    __syncthreads();
}

// Cholesky G = R^T R of the SPD M x M matrix G (R upper triangular, stored
// in Rm; dinv[j] = 1 / R[j][j]) by wavefront 0, one column per step with a
// lane-parallel trailing update.  G is left intact.  Returns false (in every
// thread) when G is not numerically positive definite.
template <int M>
__device__ __forceinline__ bool chol_wave(const double* G, double* Rm, double* dinv, int* flag) {
    constexpr int MM = M * M;
    constexpr int PER = (MM + 63) / 64;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int ei[PER], ej[PER];
        bool ev[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = lane + 64 * u;
            ev[u] = t < MM;
            ei[u] = ev[u] ? t / M : 0;
            ej[u] = ev[u] ? t % M : 0;
            if (ev[u]) Rm[t] = ei[u] <= ej[u] ? G[t] : 0.0;
        }
        wave_sync();
        int ok = 1;
#pragma unroll 1
        for (int j = 0; j < M; ++j) {
            double d = Rm[j * M + j];
            if (!(d > 0.0)) {
                ok = 0;
                d = 1.0;
            }
            const double inv_d = 1.0 / d;
            // trailing update of the upper triangle with the unscaled row j
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int i = ei[u], l = ej[u];
                if (ev[u] && i > j && l >= i) Rm[i * M + l] -= Rm[j * M + i] * Rm[j * M + l] * inv_d;
            }
            wave_sync();
            const double rjj = sqrt(d), ir = 1.0 / rjj;
            if (lane > j && lane < M) Rm[j * M + lane] *= ir;
            if (lane == j) {
                Rm[j * M + j] = rjj;
                dinv[j] = ir;
            }
            wave_sync();
        }
        if (lane == 0) *flag = ok;
    }
    __syncthreads();
    const bool ok = *flag != 0;
    __syncthreads();
    return ok;
}

// Cluster rule on ascending values th[0..n-1] (n >= target+4 or all values):
// keep `target`, grow to the end of a cluster of equal values up to
// target+3, or shrink before the cluster when it runs past that cap.
__device__ int cluster_cut_dev(const double* th, int n, int target, double rtol, double thr) {
    if (thr > 0.0) {
        // threshold rule (strategy 2 of Section 5): the eigenvalues below
        // thr, at least one and at most target, then the cluster rule
        int below = 0;
        for (int j = 0; j < n; ++j) below += th[j] < thr ? 1 : 0;
        target = below < 1 ? 1 : (below < target ? below : target);
    }
    if (target >= n) return n;
    auto same = [&](int k) { return th[k] - th[k - 1] <= rtol * fmax(fabs(th[k]), 1e-12); };
    int k = target;
    const int cap = target + 3 < n ? target + 3 : n;
    while (k < cap && same(k)) ++k;
    if (k == cap && k < n && same(k)) {
        k = target;
        while (k > 1 && same(k)) --k;
    }
    return k;
}

// Empty asm statements that take v as an operand: the arithmetic producing v
// runs before them, and no memory access moves across pin().  Used after
// every few columns of an operator apply, so that the compiler cannot hoist
// all of its LDS loads ahead of the arithmetic (a register per loaded value,
// which halves the waves per SIMD).
__device__ __forceinline__ void pin(double& v) { asm volatile("" : "+v"(v)::"memory"); }
__device__ __forceinline__ void pin_value(double& v) { asm volatile("" : "+v"(v)); }

// ---------------------------------------------------------------------------
// Block storage: the current block lives in LDS as Y[j * ld + row] (ld odd,
// so column-strided reads spread over the banks); each thread owns rows
// threadIdx.x + r * blockDim.x, r < R, and keeps at most three M-vectors of
// them in registers.

template <int M>
struct EigShared {
    double red[kMaxEigWaves * M * M];
    double G[M * M];
    double Q[M * M];
    double Rm[M * M];
    double scr[M * M];
    double dinv[M];
    double th[M];
    double nrm[M];
    double misc[kMaxEigWaves];
    int iscr[2 * M];
    int flag;
};

// G = sym(Y^T B) over all block rows: Y in LDS, B this thread's rows in
// registers.  With B = the thread's own rows of Y this is the Gram matrix.
// One wave reduction per entry; the M reductions of a row of G overlap.
template <int M, int R>
__device__ void gram_lds_reg(const double* Y, int ld, int n, const double (&B)[R][M], double* G,
                             double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll 1
    for (int i = 0; i < M; ++i) {
        double yi[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = threadIdx.x + r * blockDim.x;
            yi[r] = row < n ? Y[i * ld + row] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double v = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) v += yi[r] * B[r][j];
            v = wave_sum(v);
            if (lane == 0) red[w * M * M + i * M + j] = v;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < M * M; t += blockDim.x) {
        const int i = t / M, j = t % M;
        if (i <= j) {
            double x = 0.0, y = 0.0;
            for (int ww = 0; ww < nw; ++ww) {
                x += red[ww * M * M + i * M + j];
                y += red[ww * M * M + j * M + i];
            }
            const double v = 0.5 * (x + y);
            G[i * M + j] = v;
            G[j * M + i] = v;
        }
    }
    __syncthreads();
}

// column sums of squares of registers A into out[M]
template <int M, int R>
__device__ void colnorm2(const double (&A)[R][M], double* out, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) v += A[r][j] * A[r][j];
        v = wave_sum(v);
        if (lane == 0) red[w * M + j] = v;
    }
    __syncthreads();
    if (threadIdx.x < M) {
        double s = 0.0;
        for (int ww = 0; ww < nw; ++ww) s += red[ww * M + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// registers A <- A C (C: M*M in LDS, read by every lane at the same address);
// the row loop stays rolled and picks A[r][i] by selects, so no register
// array is indexed dynamically
template <int M, int R>
__device__ __forceinline__ void rmul(double (&A)[R][M], const double* C) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double t[M];
#pragma unroll
        for (int j = 0; j < M; ++j) t[j] = 0.0;
#pragma unroll 1
        for (int i = 0; i < M; ++i) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) a = (k == i) ? A[r][k] : a;
#pragma unroll
            for (int j = 0; j < M; ++j) t[j] += a * C[i * M + j];
        }
#pragma unroll
        for (int j = 0; j < M; ++j) A[r][j] = t[j];
    }
}

template <int M, int R>
__device__ __forceinline__ void store_block(double* Y, int ld, int n, const double (&A)[R][M]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = threadIdx.x + r * blockDim.x;
        if (row < n) {
#pragma unroll
            for (int j = 0; j < M; ++j) Y[j * ld + row] = A[r][j];
        }
    }
}

template <int M, int R>
__device__ __forceinline__ void load_block(const double* Y, int ld, int n, double (&A)[R][M]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = threadIdx.x + r * blockDim.x;
#pragma unroll
        for (int j = 0; j < M; ++j) A[r][j] = row < n ? Y[j * ld + row] : 0.0;
    }
}

// Inverse of the upper triangular factor (Rm, dinv from chol_wave) into
// Ri, by wavefront 0: rows from the bottom up, lane l owning column l.
template <int M>
__device__ __forceinline__ void trtri_wave(const double* Rm, const double* dinv, double* Ri) {
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
#pragma unroll 1
        for (int i = M - 1; i >= 0; --i) {
            if (l < M) {
                double v = (l == i) ? 1.0 : 0.0;
                for (int k = i + 1; k <= l; ++k) v -= Rm[i * M + k] * Ri[k * M + l];
                Ri[i * M + l] = l >= i ? v * dinv[i] : 0.0;
            }
            wave_sync();
        }
    }
    __syncthreads();
}

// Orthonormalise the LDS block (Cholesky-QR, twice): Y <- Y R^-1 with
// Y^T Y = R^T R.
template <int M, int R>
__device__ __forceinline__ void orthonormalise(double* Y, int ld, int n, EigShared<M>& sh) {
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        double A[R][M];
        load_block<M, R>(Y, ld, n, A);
        gram_lds_reg<M, R>(Y, ld, n, A, sh.G, sh.red);
        if (!chol_wave<M>(sh.G, sh.Rm, sh.dinv, &sh.flag)) {
            // rank-deficient block: a tiny diagonal shift keeps the factor
            // finite; the next Chebyshev cycle restores the lost directions
            if (threadIdx.x == 0) {
                double mx = 0.0;
                for (int i = 0; i < M; ++i) mx = fmax(mx, sh.G[i * M + i]);
                for (int i = 0; i < M; ++i) sh.G[i * M + i] += 1e-12 * mx + 1e-300;
            }
            __syncthreads();
            chol_wave<M>(sh.G, sh.Rm, sh.dinv, &sh.flag);
        }
        trtri_wave<M>(sh.Rm, sh.dinv, sh.scr);
        rmul<M, R>(A, sh.scr);
        store_block<M, R>(Y, ld, n, A);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// operators: out = A * (block in LDS), rows of this thread

// Level 2: A~ = S^-1/2 A_K S^-1/2 on one 8^3 element, thread = cell.
struct Op2 {
    double diag;
    double off[6];
    int nb[6];
    template <int M>
    __device__ __forceinline__ void apply(const double* Y, int ld, double (&out)[1][M]) const {
        const int c = threadIdx.x;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double s = diag * Y[j * ld + c];
#pragma unroll
            for (int d = 0; d < 6; ++d) s -= off[d] * Y[j * ld + nb[d]];
            out[0][j] = s;
            if (j % 3 == 2) {
                pin_value(out[0][j - 2]);
                pin_value(out[0][j - 1]);
                pin(out[0][j]);
            }
        }
    }
};

// Levels >= 3: block 7-point H_E on the agg^3 children of E, lp slots per
// child (the padded width of the lower level, at most kMaxLP); row =
// p * lp + a (child position p, slot a), one row per thread.  The row's own
// diagonal block stays in registers; the coupling rows of the six directions
// are re-read (from L2) on every apply, the loads of a direction issued
// together; a missing neighbour reads its own child with weight zero.
constexpr int kMaxLP = 23;   // lower-level widths up to target 20 + 3

// LPT > 0: the width is a compile-time constant; LPT = 0: run-time width lp
// (arrays sized for kMaxLP, slots beyond lp masked)
template <int LPT>
struct OpUp {
    static constexpr int kW = LPT > 0 ? LPT : kMaxLP;
    const double* Aoff;   // [m_lo][3][lp][lp]
    double hd[kW];        // H_d[c][a][0..lp-1], zero beyond lp
    int lp_rt;
    int c, a, p;          // child element, slot, child position in E
    int qx, qy, qz;       // child coordinates inside E (scalars: an indexed
    int sy, sz;           // array would live in scratch); element-index steps
                          // of the lower grid in y and z (1 in x)
    int agg;
    bool valid;           // kept slot of an existing child row
    __device__ __forceinline__ int lp() const { return LPT > 0 ? LPT : lp_rt; }
    template <int M>
    __device__ __forceinline__ void apply(const double* Y, int ld, double (&out)[1][M]) const {
        const int w = lp();
#pragma unroll
        for (int j = 0; j < M; ++j) out[0][j] = 0.0;
        if (!valid) return;
        // row base recomputed on every apply: hoisted out of the solver's loops,
        // one address per (column, slot) would stay live and spill
        int pw = p * w;
        asm volatile("" : "+v"(pw));
        const double* ys = Y + pw;
#pragma unroll
        for (int b = 0; b < kW; ++b) {
            if (b < w) {
#pragma unroll
                for (int j = 0; j < M; ++j) out[0][j] += hd[b] * ys[j * ld + b];
            }
        }
#pragma unroll 1
        for (int d = 0; d < 6; ++d) {
            const int ax = d >> 1;
            const int qa = ax == 0 ? qx : (ax == 1 ? qy : qz);
            const int cs = ax == 0 ? 1 : (ax == 1 ? sy : sz);
            const int ps = ax == 0 ? 1 : (ax == 1 ? agg : agg * agg);
            const bool in = (d & 1) ? (qa < agg - 1) : (qa > 0);
            const int cn = in ? ((d & 1) ? c + cs : c - cs) : c;
            const int pn = in ? ((d & 1) ? p + ps : p - ps) : p;
            const double msk = in ? 1.0 : 0.0;
            // + direction: A(c, cn)[a][b] = Aoff[c][ax][a][b]; - direction: Aoff[cn][ax][b][a]
            const size_t base = (d & 1) ? (((size_t)c * 3 + ax) * w + a) * w : (((size_t)cn * 3 + ax) * w) * w + a;
            const int st = (d & 1) ? 1 : w;
            double h[kW];
#pragma unroll
            for (int b = 0; b < kW; ++b) h[b] = b < w ? Aoff[base + (size_t)b * st] * msk : 0.0;
#pragma unroll
            for (int b = 0; b < kW; ++b) {
                if (b < w) {
#pragma unroll
                    for (int j = 0; j < M; ++j) out[0][j] += h[b] * Y[j * ld + pn * w + b];
                }
            }
        }
    }
};

// Chebyshev filter of degree deg applied to X (registers); the filtered
// block is left in LDS.  Wanted spectrum below a, damped interval [a, b],
// a0 below the whole spectrum.
template <int M, int R, class OP>
__device__ void cheb_filter(const OP& op, double (&X)[R][M], double* Y, int ld, int n, double a, double b,
                            double a0, int deg) {
    const double e = 0.5 * (b - a), cc = 0.5 * (b + a);
    double sigma = e / (a0 - cc);
    const double tau = 2.0 / sigma;
    double T[R][M];
    store_block<M, R>(Y, ld, n, X);
    __syncthreads();
    op.template apply<M>(Y, ld, T);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < M; ++j) T[r][j] = (T[r][j] - cc * X[r][j]) * (sigma / e);
    __syncthreads();
    store_block<M, R>(Y, ld, n, T);
    __syncthreads();
#pragma unroll 1
    for (int it = 2; it <= deg; ++it) {
        const double sn = 1.0 / (tau - sigma);
        op.template apply<M>(Y, ld, T);
        // own rows' base recomputed every step (hoisted, one address per
        // column would stay live across the loop)
        int tb = threadIdx.x;
        asm volatile("" : "+v"(tb));
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = tb + r * blockDim.x;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double yc = row < n ? Y[j * ld + row] : 0.0;
                T[r][j] = (T[r][j] - cc * yc) * (2.0 * sn / e) - (sigma * sn) * X[r][j];
                X[r][j] = yc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = tb + r * blockDim.x;
            if (row < n) {
#pragma unroll
                for (int j = 0; j < M; ++j) Y[j * ld + row] = T[r][j];
            }
        }
        __syncthreads();
        sigma = sn;
    }
}

// Rayleigh-Ritz on the orthonormal LDS block Y: X = Y Q (also left in
// LDS), AX = A X, sh.th ascending.  A Y is dead while the small
// eigenproblem runs; A X is formed afresh from X.
// With nval < M the columns nval.. of Y are zero: their diagonal entries of
// the projected matrix are set to pad (above the spectrum), so that they
// sort last and their Ritz vectors stay zero.
template <int M, int R, class OP>
__device__ void rayleigh_ritz(const OP& op, double* Y, int ld, int n, double (&X)[R][M],
                              double (&AX)[R][M], EigShared<M>& sh, int nval = M, double pad = 0.0) {
    {
        double AY[R][M];
        op.template apply<M>(Y, ld, AY);
        gram_lds_reg<M, R>(Y, ld, n, AY, sh.G, sh.red);
    }
    if (nval < M) {
        if ((int)threadIdx.x < M && (int)threadIdx.x >= nval) sh.G[threadIdx.x * M + threadIdx.x] = pad;
        __syncthreads();
    }
    jacobi_eig<M>(sh.G, sh.Q, sh.th, sh.scr, sh.iscr);
    load_block<M, R>(Y, ld, n, X);
    rmul<M, R>(X, sh.Q);
    __syncthreads();
    store_block<M, R>(Y, ld, n, X);
    __syncthreads();
    op.template apply<M>(Y, ld, AX);
}

// Full CheFSI loop.  X holds the start block on entry and the Ritz vectors
// on exit, AX = A X.  Returns the number of cycles, or -1 when the residual
// tolerance (relative to bnd) was not met within max_cycles.
// Convergence: vectors that the cluster rule keeps need residual <= tol*bnd;
// the remaining ones up to index need-1 only feed the cluster decision
// through their eigenvalues (error <= residual^2 / gap), so sqrt(tol)*bnd,
// unless their Ritz value already lies 5 % above the last kept one: then the
// decision cannot change (a partner of a kept eigenvalue would have been
// amplified like the kept vectors, which have converged; under the threshold
// rule this needs at least one filter cycle).  Without that
// exception a degenerate cluster straddling the block's end (the Laplace
// ladder of a homogeneous element) is never resolved: the filter's cut sits
// on the cluster.
template <int M, int R, class OP>
__device__ int chefsi(const OP& op, double* Y, int ld, int n, double (&X)[R][M], double (&AX)[R][M],
                      double bnd, int need, double tol, int target, double crtol, double thr, EigShared<M>& sh,
                      int max_cycles = kMaxCycles, int deg = kDegExact) {
    store_block<M, R>(Y, ld, n, X);
    __syncthreads();
    orthonormalise<M, R>(Y, ld, n, sh);
    for (int cyc = 0;; ++cyc) {
        rayleigh_ritz<M, R>(op, Y, ld, n, X, AX, sh);
        {
            double Rs[R][M];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < M; ++j) Rs[r][j] = AX[r][j] - sh.th[j] * X[r][j];
            colnorm2<M, R>(Rs, sh.nrm, sh.red);
        }
        const int nk = cluster_cut_dev(sh.th, M, target, crtol, thr);
        bool ok = true;
        for (int j = 0; j < need; ++j) {
            const double rj = sqrt(sh.nrm[j]);
            // under the threshold rule the 5 % separation counts only after
            // a filter cycle: an eigenvalue below the threshold that the start
            // block misses has not been amplified yet and would change the count
            const bool sep = (thr <= 0.0 || cyc > 0) && j >= nk && nk > 0 &&
                             sh.th[j] - sh.th[nk - 1] > 0.05 * fabs(sh.th[j]);
            ok = ok && (rj <= (j < nk ? tol : sqrt(tol)) * bnd || sep);
        }
        if (ok) return cyc;
        if (cyc >= max_cycles) return -1;
        const double a = fmin(sh.th[M - 1], 0.5 * bnd);
        const double a0 = fmin(sh.th[0], 0.0) - 1e-3 * bnd;
        __syncthreads();
        cheb_filter<M, R>(op, X, Y, ld, n, a, bnd, a0, deg);
        orthonormalise<M, R>(Y, ld, n, sh);
    }
}

__device__ __forceinline__ double block_max(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t = fmax(t, sh[i]);
    __syncthreads();
    return t;
}

// Per-column sums over all rows of registers A, written (by threads < cnt) to
// dst[j] (j < nk) and zero for nk <= j < cnt.
template <int M, int R>
__device__ void column_sums(const double (&A)[R][M], double* dst, int cnt, int nk, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) v += A[r][j];
        v = wave_sum(v);
        if (lane == 0) red[w * M + j] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        double s = 0.0;
        for (int ww = 0; ww < nw; ++ww) s += red[ww * M + threadIdx.x];
        dst[threadIdx.x] = ((int)threadIdx.x < nk) ? s : 0.0;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// level 2 kernel: one 512-thread workgroup per 8^3 element
// Learned start (warm != null): the first kw columns of the start block are
// the predicted cell vectors warm[blockIdx.x][0..kw-1][512] (row pitch kp),
// the rest the next cosine modes.  From that block the eigensolve runs to
// the relaxed residual ws_tol (times the spectral bound) within
// kWarmCycles cycles; an element that does not get there falls back to the
// exact solve (tolerance tol) from the cold start, and ws_fb[e] = 1.
// status[e] counts the cycles of both attempts.
// At most 128 VGPRs (four waves per SIMD): with about 68 KB of LDS per
// workgroup, two elements then share a CU, and one element's serial phases
// (Jacobi, Cholesky) overlap the other's filter.
template <int M>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_eig2(
    FineGeom g, const double* __restrict__ kt, int target, int L, double tol, double crtol,
    double* __restrict__ phi, double* __restrict__ lam, int* __restrict__ nkeep, double* __restrict__ Aint,
    double* __restrict__ zc, int* __restrict__ status, int e0, const float* __restrict__ warm, int kp, int kw,
    double ws_tol, int* __restrict__ ws_fb, double thr) {
    constexpr int LD = 513;
    __shared__ double sY[M * LD];
    __shared__ EigShared<M> sh;
    const int e = e0 + blockIdx.x;
    const int ex = e % g.mx, ey = (e / g.mx) % g.my, ez = e / (g.mx * g.my);
    const int c = threadIdx.x;
    const int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    auto gid = [&](int x, int y, int z) { return eidx(g, x, y, z); };
    // kappa~ per face direction: one array (isotropic) or three (orthotropic)
    const size_t N = g.ortho ? g.ncell() : 0;
    const size_t gc = gid(ex * 8 + i, ey * 8 + j, ez * 8 + k);
    const double kc[3] = {kt[gc], kt[N + gc], kt[2 * N + gc]};
    // weight tr K~: kappa~ (1 + cy + cz) with the y and z faces carrying cy
    // and cz, or the sum of the three components
    const double wsum = 1.0 + g.cy + g.cz;
    auto weight = [&](size_t q) { return g.ortho ? kt[q] + kt[N + q] + kt[2 * N + q] : wsum * kt[q]; };
    const double S = weight(gc);
    const double sq = sqrt(S);
    Op2 op;
    double diag = 0.0, rowsum = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int ii = i + (d == 0 ? -1 : (d == 1 ? 1 : 0));
        const int jj = j + (d == 2 ? -1 : (d == 3 ? 1 : 0));
        const int kk = k + (d == 4 ? -1 : (d == 5 ? 1 : 0));
        op.off[d] = 0.0;
        op.nb[d] = c;
        if (ii >= 0 && ii < 8 && jj >= 0 && jj < 8 && kk >= 0 && kk < 8) {
            const int ax = d >> 1;
            const size_t gn = gid(ex * 8 + ii, ey * 8 + jj, ez * 8 + kk);
            const double T = harm_e(kc[ax], kt[ax * N + gn]) * (ax == 0 ? 1.0 : (ax == 1 ? g.cy : g.cz));
            diag += T;
            op.off[d] = T / (sq * sqrt(weight(gn)));
            op.nb[d] = ii + 8 * (jj + 8 * kk);
            rowsum += op.off[d];
        }
    }
    op.diag = diag / S;
    const double bnd = block_max(op.diag + rowsum, sh.misc);

    double X[1][M], AX[1][M];
    const double pi8 = 3.14159265358979323846 / 8.0;
    const int nw = warm ? kw : 0;
#pragma unroll
    for (int jj = 0; jj < M; ++jj) {
        const double md = cos(pi8 * kModes[jj][0] * (i + 0.5)) * cos(pi8 * kModes[jj][1] * (j + 0.5)) *
                          cos(pi8 * kModes[jj][2] * (k + 0.5));
        const double cold = sq * (md + 0.05 * hash_noise((unsigned)e, (unsigned)jj, (unsigned)c));
        X[0][jj] = jj < nw ? sq * (double)warm[((size_t)blockIdx.x * kp + jj) * 512 + c] : cold;
    }
    const int need = (target + 4 < M - 2) ? target + 4 : M - 2;
    int cyc = -1, spent = 0;
    if (warm) {
        cyc = chefsi<M, 1>(op, sY, LD, 512, X, AX, bnd, need, ws_tol, target, crtol, thr, sh, kWarmCycles, kDeg);
        const bool fb = cyc < 0;
        if (fb) {
            spent = kWarmCycles + 1;
#pragma unroll
            for (int jj = 0; jj < M; ++jj) {
                const double md = cos(pi8 * kModes[jj][0] * (i + 0.5)) * cos(pi8 * kModes[jj][1] * (j + 0.5)) *
                                  cos(pi8 * kModes[jj][2] * (k + 0.5));
                X[0][jj] = sq * (md + 0.05 * hash_noise((unsigned)e, (unsigned)jj, (unsigned)c));
            }
        }
        if (c == 0) ws_fb[e] = fb ? 1 : 0;
        __syncthreads();
    }
    if (cyc < 0) {
        cyc = chefsi<M, 1>(op, sY, LD, 512, X, AX, bnd, need, tol, target, crtol, thr, sh);
        if (cyc >= 0) cyc += spent;
    }

    if (threadIdx.x == 0) {
        const int nk = cluster_cut_dev(sh.th, M, target, crtol, thr);
        sh.flag = nk;
        nkeep[e] = nk;
        status[e] = cyc;
        for (int a = 0; a < L; ++a) lam[(size_t)e * L + a] = sh.th[a];
    }
    __syncthreads();
    const int nk = sh.flag;
    __syncthreads();
    // interior block X^T A~ X on the kept vectors (= Phi^T A_K Phi)
    store_block<M, 1>(sY, LD, 512, X);
    __syncthreads();
    gram_lds_reg<M, 1>(sY, LD, 512, AX, sh.G, sh.red);
    for (int t = threadIdx.x; t < L * L; t += blockDim.x) {
        const int a = t / L, b = t % L;
        Aint[(size_t)e * L * L + t] = (a < nk && b < nk) ? sh.G[a * M + b] : 0.0;
    }
    // coefficients of the constant function: Phi^T S 1 = X^T S^1/2 1
    double zv[1][M];
#pragma unroll
    for (int jj = 0; jj < M; ++jj) zv[0][jj] = X[0][jj] * sq;
    column_sums<M, 1>(zv, zc + (size_t)e * L, L, nk, sh.red);
#pragma unroll
    for (int jj = 0; jj < M; ++jj) {
        if (jj < L) phi[((size_t)e * L + jj) * 512 + phi_pos(c)] = (jj < nk) ? X[0][jj] / sq : 0.0;
    }
}

// Hd[c] = Aint[c] + sum of D[c][d] over the faces of c interior to its parent
__global__ void k_build_hd(CoarseGeom lo, const double* __restrict__ Aint, const double* __restrict__ D,
                           double* __restrict__ Hd) {
    const int c = blockIdx.x;
    const int L = lo.L;
    const int cx = c % lo.mx, cy = (c / lo.mx) % lo.my, cz = c / (lo.mx * lo.my);
    const int q0 = cx % lo.agg, q1 = cy % lo.agg, q2 = cz % lo.agg;
    for (int t = threadIdx.x; t < L * L; t += blockDim.x) {
        double v = Aint[(size_t)c * L * L + t];
        for (int d = 0; d < 6; ++d) {
            const int ax = d >> 1;
            const int q = ax == 0 ? q0 : (ax == 1 ? q1 : q2);
            const bool interior = (d & 1) ? (q < lo.agg - 1) : (q > 0);
            if (interior) v += D[((size_t)c * 6 + d) * L * L + t];
        }
        Hd[(size_t)c * L * L + t] = v;
    }
}

// level >= 3 kernel: one workgroup per parent element E, one thread per row
// of H_E (blockDim = agg^3 * lo.L rounded up to whole wavefronts, <= 768).
// thr > 0 selects the kept count by the threshold rule (see cluster_cut_dev).
template <int M, int LPT>
__global__ __launch_bounds__(768) void k_eig_up(CoarseGeom lo, CoarseGeom up, const double* __restrict__ Hd,
                                                const double* __restrict__ Aoff,
                                                const int* __restrict__ nkeep_lo,
                                                const double* __restrict__ zlo, int target, double tol,
                                                double crtol, double thr, double* __restrict__ V,
                                                double* __restrict__ lam, int* __restrict__ nkeep,
                                                double* __restrict__ Aint, double* __restrict__ zup,
                                                int* __restrict__ status) {
    extern __shared__ double dyn[];
    __shared__ EigShared<M> sh;
    const int E = blockIdx.x;
    const int agg = lo.agg, Lu = up.L, LP = LPT > 0 ? LPT : lo.L;
    const int n = agg * agg * agg * LP;
    const int ld = n | 1;
    const int Ex = E % up.mx, Ey = (E / up.mx) % up.my, Ez = E / (up.mx * up.my);
    const int row = threadIdx.x;
    OpUp<LPT> op;
    op.Aoff = Aoff;
    op.lp_rt = LP;
    const int rr = row < n ? row : n - 1;
    const int p = rr / LP, a = rr % LP;
    const int qx = p % agg, qy = (p / agg) % agg, qz = p / (agg * agg);
    const int c = (Ex * agg + qx) + lo.mx * ((Ey * agg + qy) + lo.my * (Ez * agg + qz));
    op.c = c;
    op.a = a;
    op.p = p;
    op.qx = qx;
    op.qy = qy;
    op.qz = qz;
    op.sy = lo.mx;
    op.sz = lo.mx * lo.my;
    op.agg = agg;
    op.valid = row < n && a < nkeep_lo[c];
#pragma unroll
    for (int b = 0; b < OpUp<LPT>::kW; ++b) op.hd[b] = b < LP ? Hd[((size_t)c * LP + a) * LP + b] : 0.0;
    // Gershgorin bound: absolute row sum of H_E
    double rs = 0.0;
    if (op.valid) {
#pragma unroll
        for (int b = 0; b < OpUp<LPT>::kW; ++b) rs += fabs(op.hd[b]);
        for (int d = 0; d < 6; ++d) {
            const int ax = d >> 1;
            const int qa = ax == 0 ? qx : (ax == 1 ? qy : qz);
            const int cs = ax == 0 ? 1 : (ax == 1 ? lo.mx : lo.mx * lo.my);
            const bool in = (d & 1) ? (qa < agg - 1) : (qa > 0);
            if (!in) continue;
            const int cn = (d & 1) ? c + cs : c - cs;
            for (int b = 0; b < LP; ++b)
                rs += fabs((d & 1) ? Aoff[(((size_t)c * 3 + ax) * LP + a) * LP + b]
                                   : Aoff[(((size_t)cn * 3 + ax) * LP + b) * LP + a]);
        }
    }
    const double bnd = block_max(rs, sh.misc);
    // dimension of H_E (the kept slots of the children) and the compact
    // index of this row among them
    int nval = 0, ci = a;
    for (int pp = 0; pp < agg * agg * agg; ++pp) {
        const int c2 = (Ex * agg + pp % agg) + lo.mx * ((Ey * agg + (pp / agg) % agg) + lo.my * (Ez * agg + pp / (agg * agg)));
        const int k2 = nkeep_lo[c2];
        nval += k2;
        if (pp < p) ci += k2;
    }
    const double zr = op.valid ? zlo[(size_t)c * LP + a] : 0.0;
    double X[1][M], AX[1][M];
    int cyc = 0;
    if (nval <= M) {
        // the block can hold the whole space: unit vectors and one
        // Rayleigh-Ritz step give the exact eigenpairs
#pragma unroll
        for (int j = 0; j < M; ++j) X[0][j] = (op.valid && ci == j) ? 1.0 : 0.0;
        store_block<M, 1>(dyn, ld, n, X);
        __syncthreads();
        rayleigh_ritz<M, 1>(op, dyn, ld, n, X, AX, sh, nval, 2.0 * bnd + 1.0);
    } else {
        // start block: the constant function, smooth weights of the
        // children's constant modes, and noise on every kept slot.  The
        // noise has one amplitude for the whole element: the constant
        // function's coefficient zr vanishes on the children's non-constant
        // slots, and noise scaled by it would leave the block without those
        // directions, which a polynomial filter cannot restore
        const double pa = 3.14159265358979323846 / agg;
        const double az = block_max(op.valid ? fabs(zr) : 0.0, sh.misc) + 1e-300;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double v = 0.05 * az * hash_noise((unsigned)E + 77u, (unsigned)j, (unsigned)row);
            if (j == 0) v = zr;
            else if (a == 0)
                v += zr * cos(pa * kModes[j & 15][0] * (qx + 0.5)) * cos(pa * kModes[j & 15][1] * (qy + 0.5)) *
                     cos(pa * kModes[j & 15][2] * (qz + 0.5));
            X[0][j] = op.valid ? v : 0.0;
        }
        const int need = (target + 4 < M - 2) ? target + 4 : M - 2;
        cyc = chefsi<M, 1>(op, dyn, ld, n, X, AX, bnd, need, tol, target, crtol, thr, sh);
    }
    if (threadIdx.x == 0) {
        const int nk = cluster_cut_dev(sh.th, nval < M ? nval : M, target, crtol, thr);
        sh.flag = nk;
        nkeep[E] = nk;
        status[E] = cyc;
        for (int b = 0; b < Lu; ++b) lam[(size_t)E * Lu + b] = b < nval ? sh.th[b] : 0.0;
    }
    __syncthreads();
    const int nk = sh.flag;
    __syncthreads();
    store_block<M, 1>(dyn, ld, n, X);
    __syncthreads();
    gram_lds_reg<M, 1>(dyn, ld, n, AX, sh.G, sh.red);
    for (int t = threadIdx.x; t < Lu * Lu; t += blockDim.x) {
        const int i = t / Lu, j = t % Lu;
        Aint[(size_t)E * Lu * Lu + t] = (i < nk && j < nk) ? sh.G[i * M + j] : 0.0;
    }
    double zv[1][M];
#pragma unroll
    for (int jj = 0; jj < M; ++jj) zv[0][jj] = X[0][jj] * zr;
    column_sums<M, 1>(zv, zup + (size_t)E * Lu, Lu, nk, sh.red);
    if (row < n) {
#pragma unroll
        for (int jj = 0; jj < M; ++jj)
            if (jj < Lu) V[((size_t)E * Lu + jj) * n + row] = (jj < nk) ? X[0][jj] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// launchers

#define SPECMG_M_DISPATCH(MV, ...)                   \
    switch (MV) {                                    \
        case 10: {                                   \
            constexpr int M = 10;                    \
            __VA_ARGS__;                             \
        } break;                                     \
        case 12: {                                   \
            constexpr int M = 12;                    \
            __VA_ARGS__;                             \
        } break;                                     \
        default: {                                   \
            constexpr int M = 14;                    \
            __VA_ARGS__;                             \
        } break;                                     \
    }

void launch_eig2(const FineGeom& g, const double* kt, int target, int nvec, double tol, double crtol,
                 double* phi, double* lam, int* nkeep, double* Aint, int* status, double* zc, int e0, int count,
                 const float* warm, int kp, int kw, double ws_tol, int* ws_fb, double thr, hipStream_t s) {
    const int L = target + 3;
    SPECMG_M_DISPATCH(nvec, hipLaunchKernelGGL((k_eig2<M>), dim3(count), dim3(512), 0, s, g, kt, target, L, tol,
                                               crtol, phi, lam, nkeep, Aint, zc, status, e0, warm, kp, kw, ws_tol,
                                               ws_fb, thr));
}

void launch_eig_up(const CoarseGeom& lo, const CoarseGeom& up, const double* Aint_lo, const double* Dlo,
                   const double* Aofflo, const int* nkeep_lo, const double* zlo, double* Hd_work,
                   int target, int nvec, double tol, double crtol, double thr, double* V, double* lam, int* nkeep,
                   double* Aint, double* zup, int* status, hipStream_t s) {
    hipLaunchKernelGGL(k_build_hd, dim3(lo.m), dim3(128), 0, s, lo, Aint_lo, Dlo, Hd_work);
    const int n = lo.agg * lo.agg * lo.agg * lo.L;
    const int threads = (n + 63) / 64 * 64;
    if (up.L != target + 3 || lo.L > kMaxLP || threads > 768 || target < 1 || target > 20 || nvec < target + 6)
        throw HipError{hipErrorInvalidValue, "eig_up shape"};
    const size_t shmem = (size_t)nvec * (n | 1) * sizeof(double);
    // compile-time widths for the pairs (block size, lower width) that occur
    // when both levels have the same target; the run-time width otherwise
#define SPECMG_EIG_UP(MV, LV)                                                                                    \
    {                                                                                                            \
        hipFuncSetAttribute((const void*)k_eig_up<MV, LV>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem); \
        hipLaunchKernelGGL((k_eig_up<MV, LV>), dim3(up.m), dim3(threads), shmem, s, lo, up, Hd_work, Aofflo,       \
                           nkeep_lo, zlo, target, tol, crtol, thr, V, lam, nkeep, Aint, zup, status);               \
        return;                                                                                                  \
    }
    const int key = nvec * 100 + lo.L;
    switch (key) {
        case 1004: SPECMG_EIG_UP(10, 4)
        case 1005: SPECMG_EIG_UP(10, 5)
        case 1006: SPECMG_EIG_UP(10, 6)
        case 1007: SPECMG_EIG_UP(10, 7)
        case 1208: SPECMG_EIG_UP(12, 8)
        case 1209: SPECMG_EIG_UP(12, 9)
        case 1409: SPECMG_EIG_UP(14, 9)
        case 1410: SPECMG_EIG_UP(14, 10)
        case 1411: SPECMG_EIG_UP(14, 11)
        case 1609: SPECMG_EIG_UP(16, 9)
        case 1612: SPECMG_EIG_UP(16, 12)
        case 1613: SPECMG_EIG_UP(16, 13)
        default: break;
    }
    switch (nvec) {
        case 10: SPECMG_EIG_UP(10, 0)
        case 12: SPECMG_EIG_UP(12, 0)
        case 14: SPECMG_EIG_UP(14, 0)
        case 16: SPECMG_EIG_UP(16, 0)
        case 20: SPECMG_EIG_UP(20, 0)
        case 26: SPECMG_EIG_UP(26, 0)
        default: break;
    }
#undef SPECMG_EIG_UP
    throw HipError{hipErrorInvalidValue, "eig_up block size"};
}

}  // namespace specmg
