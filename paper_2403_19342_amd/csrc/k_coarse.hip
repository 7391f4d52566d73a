// Coarse levels of the V-cycle (Algorithm 1 steps 3-7, applied recursively)
// and their set-up.
//
// A coarse level l >= 2 has one block of L (padded) unknowns per element;
// its Galerkin operator A_l = R_l A_{l-1} R_l^T (text above Algorithm 1) is
// a block 7-point stencil stored as
//   Ad[e]        diagonal block  (L x L)
//   Aoff[e][d]   coupling A_l(e, e + unit vector d), d = x, y, z (L x L)
// The level-l smoother is one block-Jacobi sweep whose blocks are the
// level-(l+1) parent elements, each factored by block IC(0) over its agg^3
// children in lexicographic order (Section 5): pivots
//   D_c = Ad_c - sum_{lower neighbour c'} A(c, c') D_c'^{-1} A(c', c),
// stored inverted in Dinv.  Padded slots carry an identity pivot and zero
// couplings, so they stay zero.  For the substitutions the set-up also forms
//   G[c][2 ax]     = D_c^{-1} A(c, c - e_ax)   (lower neighbour, same parent)
//   G[c][2 ax + 1] = D_c^{-1} A(c, c + e_ax)   (upper neighbour, same parent)
// so that every hyperplane step is a single product:
//   forward   y_c = D_c^{-1} r_c - sum_lower G y_c'
//   backward  z_c = y_c - sum_upper G z_c''.
#include <vector>

#include "common.hpp"

namespace specmg {

__device__ __forceinline__ int log2_agg(int agg) { return agg == 4 ? 2 : 1; }

// level-l index of the child at position p (lexicographic in the parent) of
// parent E; agg is 2 or 4, so positions decode with shifts
__device__ __forceinline__ int child_of(const CoarseGeom& g, int E, int p) {
    const int a = g.agg, sh = log2_agg(a);
    const int Ex = E % g.px, Ey = (E / g.px) % g.py, Ez = E / (g.px * g.py);
    const int qx = p & (a - 1), qy = (p >> sh) & (a - 1), qz = p >> (2 * sh);
    return (Ex * a + qx) + g.mx * ((Ey * a + qy) + g.my * (Ez * a + qz));
}

// children positions sorted by qx+qy+qz for agg = 2 and agg = 4
struct ChildPlanes {
    unsigned char pos2[8], off2[5], rank2[8];
    unsigned char pos4[64], off4[11], rank4[64];
};

constexpr ChildPlanes make_child_planes() {
    ChildPlanes t{};
    int k = 0;
    for (int s = 0; s <= 3; ++s) {
        t.off2[s] = (unsigned char)k;
        for (int p = 0; p < 8; ++p)
            if ((p & 1) + ((p >> 1) & 1) + (p >> 2) == s) t.pos2[k++] = (unsigned char)p;
    }
    t.off2[4] = (unsigned char)k;
    k = 0;
    for (int s = 0; s <= 9; ++s) {
        t.off4[s] = (unsigned char)k;
        for (int p = 0; p < 64; ++p)
            if ((p & 3) + ((p >> 2) & 3) + (p >> 4) == s) t.pos4[k++] = (unsigned char)p;
    }
    t.off4[10] = (unsigned char)k;
    for (int i = 0; i < 8; ++i) t.rank2[t.pos2[i]] = (unsigned char)i;
    for (int i = 0; i < 64; ++i) t.rank4[t.pos4[i]] = (unsigned char)i;
    return t;
}

__constant__ ChildPlanes kCP = make_child_planes();

// positions of the agg^3 children sorted by qx+qy+qz, copied into LDS
__device__ void build_planes(int agg, int* pos, int* off) {
    const int nc = agg * agg * agg, np = 3 * (agg - 1) + 2;
    for (int t = threadIdx.x; t < nc; t += blockDim.x) pos[t] = agg == 4 ? kCP.pos4[t] : kCP.pos2[t];
    for (int t = threadIdx.x; t < np; t += blockDim.x) off[t] = agg == 4 ? kCP.off4[t] : kCP.off2[t];
    __syncthreads();
}

constexpr int kMaxLc = 23;   // padded widths up to target 20 + 3 (levels >= 3)
constexpr int kNarrow = 13;  // widths up to target 10 + 3 get their own instantiations

// y_c = (A_l u)_c for row a of child element c.  Blocks up to 9 wide: the
// diagonal block, then one axis at a time both coupling blocks, every load
// of an axis issued before its products (at the domain boundary from valid
// stand-in rows of the element itself, whose sums a select then drops), so
// a row waits for memory four times.  Wider blocks (register budget): the
// diagonal block, then each coupling block inside the domain in turn.
template <typename T, int LP = kMaxLc>
__device__ __forceinline__ T block_row_apply(const CoarseGeom& g, const T* __restrict__ Ad,
                                             const T* __restrict__ Aoff, const T* __restrict__ u, int c,
                                             int a) {
    const int L = g.L;
    const int cx = c % g.mx, cy = (c / g.mx) % g.my, cz = c / (g.mx * g.my);
    const int cc[3] = {cx, cy, cz};
    const int ext[3] = {g.mx, g.my, g.mz};
    const int stride[3] = {1, g.mx, g.mx * g.my};
    T acc = T(0);
    {
        const T* ad = Ad + ((size_t)c * L + a) * L;
        const T* uc = u + (size_t)c * L;
#pragma unroll
        for (int b = 0; b < LP; ++b) {
            const int bb = b < L ? b : L - 1;
            acc += (b < L ? ad[bb] : T(0)) * uc[bb];
        }
    }
    if constexpr (LP <= 9) {
#pragma unroll 1
        for (int ax = 0; ax < 3; ++ax) {
            const int cca = ax == 0 ? cx : (ax == 1 ? cy : cz);
            const int exa = ax == 0 ? g.mx : (ax == 1 ? g.my : g.mz);
            const int sta = ax == 0 ? 1 : (ax == 1 ? g.mx : g.mx * g.my);
            const bool hp = cca + 1 < exa, hm = cca > 0;
            const int cp = hp ? c + sta : c, cm = hm ? c - sta : c;
            // A(c, c+e) = Aoff[c][ax]; A(c, c-e) = Aoff[c-e][ax]^T
            const T* op = Aoff + (((size_t)c * 3 + ax) * L + a) * L;
            const T* om = Aoff + ((size_t)cm * 3 + ax) * L * L + a;
            const T* up = u + (size_t)cp * L;
            const T* um = u + (size_t)cm * L;
            T sp = T(0), sm = T(0);
#pragma unroll
            for (int b = 0; b < LP; ++b) {
                const int bb = b < L ? b : L - 1;
                sp += (b < L ? op[bb] : T(0)) * up[bb];
                sm += (b < L ? om[(size_t)bb * L] : T(0)) * um[bb];
            }
            acc += hp ? sp : T(0);
            acc += hm ? sm : T(0);
        }
    } else {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (cc[ax] + 1 < ext[ax]) {
                const int cn = c + stride[ax];
                const T* o = Aoff + (((size_t)c * 3 + ax) * L + a) * L;
                const T* un = u + (size_t)cn * L;
#pragma unroll
                for (int b = 0; b < LP; ++b) {
                    const int bb = b < L ? b : L - 1;
                    acc += (b < L ? o[bb] : T(0)) * un[bb];
                }
            }
            if (cc[ax] > 0) {
                const int cn = c - stride[ax];
                const T* o = Aoff + ((size_t)cn * 3 + ax) * L * L;
                const T* un = u + (size_t)cn * L;
#pragma unroll
                for (int b = 0; b < LP; ++b) {
                    const int bb = b < L ? b : L - 1;
                    acc += (b < L ? o[bb * L + a] : T(0)) * un[bb];
                }
            }
        }
    }
    return acc;
}

constexpr int kCoarseThreads = 1024;   // upper bound; launches use agg^3 L rounded to waves
constexpr int kMaxChildren = 64;   // agg <= 4
constexpr int kMaxL = kMaxLc;      // set-up arrays of the levels >= 3
constexpr int kMaxL2 = 16;         // level 2 (target <= 10)

// Level-l smoother on parent E, both substitutions in one kernel:
//   t = r (mode 0) or t = r - A_l u (mode 1)
//   w = D^-1 t per child; y = forward substitution, z = backward substitution
//   out = z (mode 0) or out = u + z (mode 1)
// One thread per row (child, slot) with the children in hyperplane order, so
// the rows of plane s are threads [off[s] LP, off[s+1] LP).  Each thread keeps
// the rows of its lower and upper couplings G in registers; only y lives in
// LDS.  A plane step is one LDS read per coupling entry, the products, a store
// and a barrier.  Missing neighbours read the thread's own child with weight 0.
template <typename T, int LP, bool A2>
__global__ __launch_bounds__(768) void k_coarse_sweep(CoarseGeom g, int mode, const T* __restrict__ Ad,
                                                      const T* __restrict__ Aoff, const T* __restrict__ Dinv,
                                                      const T* __restrict__ G, const T* __restrict__ r,
                                                      const T* u, T* out, const Scalars* sc, int check_done,
                                                      int npar) {
    if (check_done && sc->done) return;
    __shared__ T sY[kMaxChildren * LP];
    const int agg = g.agg, nc = agg * agg * agg, sh = log2_agg(agg);
    const int nplanes = 3 * (agg - 1) + 1;
    // npar parents per workgroup (several when a parent has few rows, so
    // that the wavefronts are full), each with its own nc * LP rows of sY
    const int per = nc * LP;
    const int t = threadIdx.x, qp = t / per, tt = t - qp * per;
    const int E = blockIdx.x * npar + qp;
    const bool row_ok = qp < npar && E < g.M;
    const int base = row_ok ? qp * per : 0;
    const int k = row_ok ? tt / LP : 0, a = tt % LP;
    const int p = agg == 4 ? kCP.pos4[k] : kCP.pos2[k];
    const int q[3] = {p & (agg - 1), (p >> sh) & (agg - 1), p >> (2 * sh)};
    const int plane = q[0] + q[1] + q[2];
    const int c = child_of(g, E, p);
    // neighbour rows in LDS and weights per direction (lower: 2 ax, upper: 2 ax + 1)
    int nb[6];
    T wgt[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int ax = d >> 1;
        const bool in = (d & 1) ? (q[ax] < agg - 1) : (q[ax] > 0);
        const int step = 1 << (sh * ax);
        const int pn = in ? ((d & 1) ? p + step : p - step) : p;
        nb[d] = base + (agg == 4 ? kCP.rank4[pn] : kCP.rank2[pn]) * LP;
        wgt[d] = in ? T(1) : T(0);
    }
    // slots beyond the child's kept count are zero rows of every block: their
    // threads load nothing and carry zeros
    const bool live = row_ok && (g.nkeep == nullptr || a < g.nkeep[c]);
    // right-hand side t = r (- A_l u): all loads of the row first
    const size_t row = (size_t)c * LP + a;
    T tv = live ? r[row] : T(0);
    if (mode && live) {
        const int cx = c % g.mx, cy = (c / g.mx) % g.my, cz = c / (g.mx * g.my);
        T acc = T(0);
#pragma unroll
        for (int b = 0; b < LP; ++b) acc += Ad[row * LP + b] * u[(size_t)c * LP + b];
        // one direction at a time keeps the loads in flight to 4 LP values
#pragma unroll 1
        for (int ax = 0; ax < 3; ++ax) {
            const int cca = ax == 0 ? cx : (ax == 1 ? cy : cz);
            const int exa = ax == 0 ? g.mx : (ax == 1 ? g.my : g.mz);
            const int sta = ax == 0 ? 1 : (ax == 1 ? g.mx : g.mx * g.my);
            const bool hp = cca + 1 < exa, hm = cca > 0;
            const int cp = hp ? c + sta : c, cm = hm ? c - sta : c;
            const T wp = hp ? T(1) : T(0), wm = hm ? T(1) : T(0);
            T sp = T(0), sm = T(0);
#pragma unroll
            for (int b = 0; b < LP; ++b) {
                // A(c, c+e) = Aoff[c][ax]; A(c, c-e) = Aoff[c-e][ax]^T
                sp += Aoff[(((size_t)c * 3 + ax) * LP + a) * LP + b] * u[(size_t)cp * LP + b];
                sm += Aoff[(((size_t)cm * 3 + ax) * LP + b) * LP + a] * u[(size_t)cm * LP + b];
            }
            acc += wp * sp + wm * sm;
        }
        tv -= acc;
    }
    if (row_ok) sY[t] = tv;
    // lower coupling rows G[c][2 ax][a][0..LP-1] and the pivot row, loaded
    // while the block synchronises; at widths up to 8 the upper rows too
    // (one memory round less), wider ones follow the forward sweep so that
    // the two sets are never live together
    // A2 (agg = 2): along each axis a child couples to exactly one sibling,
    // below or above it, so gl[ax] holds that one coupling row, all loaded
    // here, and the sweeps weight it by direction (gu unused)
    constexpr bool kUpperEarly = LP <= 8 && !A2;
    // couplings to children outside the parent are never loaded (with
    // agg = 2 half of them)
    T gl[3][LP], gu[3][LP], dv[LP];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const bool lo = wgt[2 * ax] != T(0);
        const bool in = live && (A2 || lo);
        const int d = (A2 && !lo) ? 2 * ax + 1 : 2 * ax;
#pragma unroll
        for (int b = 0; b < LP; ++b) gl[ax][b] = in ? G[(((size_t)c * 6 + d) * LP + a) * LP + b] : T(0);
    }
#pragma unroll
    for (int b = 0; b < LP; ++b) dv[b] = live ? Dinv[row * LP + b] : T(0);
    if (kUpperEarly) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const bool in = live && wgt[2 * ax + 1] != T(0);
#pragma unroll
            for (int b = 0; b < LP; ++b)
                gu[ax][b] = in ? G[(((size_t)c * 6 + 2 * ax + 1) * LP + a) * LP + b] : T(0);
        }
    }
    __syncthreads();
    T w = T(0);
    {
        const T* ty = sY + base + k * LP;
#pragma unroll
        for (int b = 0; b < LP; ++b) w += dv[b] * ty[b];
    }
    __syncthreads();
    // forward: y = w - sum_lower G y
    T y = T(0);
    for (int s = 0; s < nplanes; ++s) {
        if (row_ok && plane == s) {
            T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
            for (int b = 0; b < LP; ++b) {
                s0 += gl[0][b] * sY[nb[0] + b];
                s1 += gl[1][b] * sY[nb[2] + b];
                s2 += gl[2][b] * sY[nb[4] + b];
            }
            if (A2) {
                s0 *= wgt[0];
                s1 *= wgt[2];
                s2 *= wgt[4];
            }
            y = w - (s0 + s1 + s2);
            sY[t] = y;
        }
        __syncthreads();
    }
    // backward: z = y - sum_upper G z
    if (!kUpperEarly && !A2) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const bool in = live && wgt[2 * ax + 1] != T(0);
#pragma unroll
            for (int b = 0; b < LP; ++b)
                gu[ax][b] = in ? G[(((size_t)c * 6 + 2 * ax + 1) * LP + a) * LP + b] : T(0);
        }
    }
    T z = T(0);
    for (int s = nplanes - 1; s >= 0; --s) {
        if (row_ok && plane == s) {
            T s0 = T(0), s1 = T(0), s2 = T(0);
            if constexpr (A2) {
#pragma unroll
                for (int b = 0; b < LP; ++b) {
                    s0 += gl[0][b] * sY[nb[1] + b];
                    s1 += gl[1][b] * sY[nb[3] + b];
                    s2 += gl[2][b] * sY[nb[5] + b];
                }
                s0 *= wgt[1];
                s1 *= wgt[3];
                s2 *= wgt[5];
            } else {
#pragma unroll
                for (int b = 0; b < LP; ++b) {
                    s0 += gu[0][b] * sY[nb[1] + b];
                    s1 += gu[1][b] * sY[nb[3] + b];
                    s2 += gu[2][b] * sY[nb[5] + b];
                }
            }
            z = y - (s0 + s1 + s2);
            sY[t] = z;
        }
        __syncthreads();
    }
    if (row_ok) out[row] = mode ? u[row] + z : z;
}

// s = r - A_l u on the children of E, then r_up[E] = V_E^T s
template <typename T, int LP, int LU>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_resid_restrict(
    CoarseGeom g, const T* __restrict__ Ad, const T* __restrict__ Aoff, const T* __restrict__ r,
    const T* __restrict__ u, const T* __restrict__ V, const int* __restrict__ nkeep_up, int Lup,
    T* __restrict__ rup, const Scalars* sc, int check_done) {
    if (check_done && sc->done) return;
    __shared__ T sS[kMaxChildren * kMaxL];
    __shared__ double sred[kCoarseThreads / 64];
    const int E = blockIdx.x;
    const int L = g.L, nc = g.agg * g.agg * g.agg, n = nc * L;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int p = t / L, a = t % L;
        const int c = child_of(g, E, p);
        const bool live = g.nkeep == nullptr || a < g.nkeep[c];   // zero rows beyond the kept slots
        sS[t] = live ? r[(size_t)c * L + a] - block_row_apply<T, LP>(g, Ad, Aoff, u, c, a) : T(0);
    }
    __syncthreads();
    const int nk = nkeep_up[E];
    double acc[LU];
#pragma unroll
    for (int j = 0; j < LU; ++j) acc[j] = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double sv = (double)sS[t];
#pragma unroll
        for (int j = 0; j < LU; ++j) {
            const int jj = j < nk ? j : nk - 1;
            acc[j] += (j < nk ? (double)V[((size_t)E * Lup + jj) * n + t] : 0.0) * sv;
        }
    }
    __shared__ double sacc[kCoarseThreads / 64][LU];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < LU; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) sacc[w][j] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < Lup) {
        double t = 0.0;
        for (int ww = 0; ww < (int)(blockDim.x >> 6); ++ww) t += sacc[ww][threadIdx.x];
        rup[(size_t)E * Lup + threadIdx.x] = (int)threadIdx.x < nk ? (T)t : T(0);
    }
    (void)sred;
}

// u += V_E e_up[E] on the children of E
template <typename T, int LU>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_prolong(CoarseGeom g, T* __restrict__ u,
                                                                  const T* __restrict__ V,
                                                                  const int* __restrict__ nkeep_up, int Lup,
                                                                  const T* __restrict__ eup, const Scalars* sc,
                                                                  int check_done) {
    if (check_done && sc->done) return;
    const int E = blockIdx.x;
    const int L = g.L, nc = g.agg * g.agg * g.agg, n = nc * L;
    const int nk = nkeep_up[E];
    const T* ee = eup + (size_t)E * Lup;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int p = t / L, a = t % L;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < LU; ++j) {
            const int jj = j < nk ? j : nk - 1;
            acc += (j < nk ? V[((size_t)E * Lup + jj) * n + t] : T(0)) * ee[jj];
        }
        u[(size_t)child_of(g, E, p) * L + a] += acc;
    }
}

// e = B r at the coarsest level, B the dense inverse of the regularised
// coarsest matrix, over the compact unknowns (cmap: compact index -> padded
// index).  r is first gathered into a compact FP64 vector rc, staged through
// LDS in chunks of kCoarsestChunk values (any size fits the 160 KB of LDS).
// Spaces within one chunk give each wavefront one row; larger ones give each
// block kCoarsestRows consecutive rows that the whole block streams one row
// at a time (64 KB contiguous per row and chunk: concurrent streams of many
// rows a full row apart share few HBM channels and ran at 2.2 TB/s).
constexpr int kCoarsestRows = 16;

template <typename T>
__global__ void k_gather_compact(int n, const int* __restrict__ cmap, const T* __restrict__ r,
                                 double* __restrict__ rc, const Scalars* sc, int check_done) {
    if (check_done && sc->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) rc[i] = (double)r[cmap[i]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarsest_rows(int n, int np, const double* __restrict__ Pinv,
                                                        const int* __restrict__ cmap,
                                                        const double* __restrict__ rc, T* __restrict__ e,
                                                        const Scalars* sc, int check_done) {
    if (check_done && sc->done) return;
    extern __shared__ double srz[];
    __shared__ double red[4][kCoarsestRows];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int i0 = blockIdx.x * kCoarsestRows;
    double acc[kCoarsestRows];
#pragma unroll
    for (int r = 0; r < kCoarsestRows; ++r) acc[r] = 0.0;
    for (int c0 = 0; c0 < n; c0 += kCoarsestChunk) {
        const int cn = min(kCoarsestChunk, n - c0);
        if (c0) __syncthreads();
        for (int j = t; j < cn; j += 256) srz[j] = rc[c0 + j];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kCoarsestRows; ++r) {
            if (i0 + r < n) {
                const double* row = Pinv + (size_t)(i0 + r) * np + c0;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
                for (int j = t; j < cn; j += 512) {
                    a0 += row[j] * srz[j];
                    if (j + 256 < cn) a1 += row[j + 256] * srz[j + 256];
                }
                acc[r] += a0 + a1;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kCoarsestRows; ++r) {
        const double s = wave_sum(acc[r]);
        if (lane == 0) red[w][r] = s;
    }
    __syncthreads();
    if (t < kCoarsestRows && i0 + t < n) e[cmap[i0 + t]] = (T)((red[0][t] + red[1][t]) + (red[2][t] + red[3][t]));
}

// (spaces of one LDS chunk: each block gathers the compact right-hand side
// itself from the level vector r through cmap, so no separate gather launch)
template <typename T, int RW>
__global__ __launch_bounds__(256) void k_coarsest(int n, int np, const double* __restrict__ Pinv,
                                                   const int* __restrict__ cmap, const T* __restrict__ r,
                                                   T* __restrict__ e, const Scalars* sc, int check_done) {
    if (check_done && sc->done) return;
    extern __shared__ double srz[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i0 = blockIdx.x * 4 * RW + w * RW;
    double acc[RW];
#pragma unroll
    for (int qq = 0; qq < RW; ++qq) acc[qq] = 0.0;
    for (int c0 = 0; c0 < n; c0 += kCoarsestChunk) {
        const int cn = min(kCoarsestChunk, n - c0);
        if (c0) __syncthreads();
        for (int j = threadIdx.x; j < cn; j += blockDim.x) srz[j] = (double)r[cmap[c0 + j]];
        __syncthreads();
        for (int j = lane; j < cn; j += 64) {
            const double v = srz[j];
#pragma unroll
            for (int q = 0; q < RW; ++q)
                if (i0 + q < n) acc[q] += Pinv[(size_t)(i0 + q) * np + c0 + j] * v;
        }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0 && i0 + q < n) e[cmap[i0 + q]] = (T)s;
    }
}

// Coarsest product for spaces wider than one LDS chunk, reading the
// symmetric inverse once: only its tiles (I, J) with I >= J are stored,
// packed tile after tile (tile (I, J) at index I (I + 1) / 2 + J, each tile
// kSymT x kSymT row-major and contiguous), half the bytes of the full
// matrix.  Tile (I, J) contributes B_IJ r_J to e_I and, below the diagonal,
// B_IJ^T r_I to e_J.  A workgroup streams a chunk of up to kSymChunk tiles of
// one tile row I: lane l of wave w holds columns 2l, 2l + 1 and rows
// w, w + 4, ... of every tile, so each row of a tile is one coalesced 1 KB
// load per wave.  The row contributions accumulate in registers over the
// chunk and are written once per chunk to Q[I][chunk]; the column
// contributions of each off-diagonal tile are combined over the four waves
// and written to P[J][I].  k_coarsest_sym_reduce then sums, for every
// output tile I, its chunks' Q and the P written by the tiles below it, in a
// fixed order (no atomics: results are reproducible).
constexpr int kSymT = 128;
constexpr int kSymChunk = 8;
constexpr int kSymWaves = 8;                  // 512 threads per workgroup
constexpr int kSymRows = kSymT / kSymWaves;   // rows per wave and tile

__global__ void k_pack_lower_tiles(const double* __restrict__ dense, int np, double* __restrict__ packed) {
    const int t = blockIdx.x;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    double* dst = packed + (size_t)t * kSymT * kSymT;
    for (int k = threadIdx.x; k < kSymT * kSymT; k += blockDim.x) {
        const int i = k / kSymT, j = k % kSymT;
        dst[k] = dense[(size_t)(I * kSymT + i) * np + (size_t)J * kSymT + j];
    }
}

__global__ __launch_bounds__(64 * kSymWaves) void k_coarsest_sym(int nT, const int2* __restrict__ chunks,
                                                                 const double* __restrict__ packed,
                                                                 const double* __restrict__ rc,
                                                                 double* __restrict__ P, double* __restrict__ Q,
                                                                 int maxc, const Scalars* sc, int check_done) {
    if (check_done && sc->done) return;
    __shared__ double sri[kSymT];
    __shared__ double scol[kSymWaves][kSymT];
    const int2 ch = chunks[blockIdx.x];   // (tile row I, first tile J0)
    const int I = ch.x, J0 = ch.y, J1 = min(I + 1, J0 + kSymChunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < kSymT) sri[threadIdx.x] = rc[(size_t)I * kSymT + threadIdx.x];
    __syncthreads();
    double racc[kSymRows];
#pragma unroll
    for (int k = 0; k < kSymRows; ++k) racc[k] = 0.0;
    for (int J = J0; J < J1; ++J) {
        const double* tile = packed + ((size_t)I * (I + 1) / 2 + J) * kSymT * kSymT + (size_t)w * kSymT + 2 * lane;
        const double2 rj = *reinterpret_cast<const double2*>(rc + (size_t)J * kSymT + 2 * lane);
        double c0 = 0.0, c1 = 0.0;
        // all 16 rows of the wave in flight (16 KB per wave), then the sums
        double2 b[kSymRows];
#pragma unroll
        for (int k = 0; k < kSymRows; ++k)
            b[k] = *reinterpret_cast<const double2*>(tile + (size_t)(kSymWaves * k) * kSymT);
#pragma unroll
        for (int k = 0; k < kSymRows; ++k) {
            const double ri = sri[w + kSymWaves * k];
            racc[k] += b[k].x * rj.x + b[k].y * rj.y;
            c0 += b[k].x * ri;
            c1 += b[k].y * ri;
        }
        if (J < I) {
            scol[w][2 * lane] = c0;
            scol[w][2 * lane + 1] = c1;
            __syncthreads();
            if (threadIdx.x < kSymT) {
                const int j = threadIdx.x;
                double v = 0.0;
#pragma unroll
                for (int ww = 0; ww < kSymWaves; ++ww) v += scol[ww][j];
                P[((size_t)J * nT + I) * kSymT + j] = v;
            }
            __syncthreads();
        }
    }
    const int c = J0 / kSymChunk;
#pragma unroll
    for (int k = 0; k < kSymRows; ++k) {
        const double v = wave_sum(racc[k]);
        if (lane == 0) Q[((size_t)I * maxc + c) * kSymT + w + kSymWaves * k] = v;
    }
}

// One workgroup per output tile I: kSymRedGroups groups of kSymT threads
// split the tile's partial vectors (group q takes the chunks c = q mod G and
// the tiles K = I + 1 + q mod G, four loads in flight), then the group sums
// are added in group order, so the result does not depend on timing.
constexpr int kSymRedGroups = 8;

template <typename T>
__global__ __launch_bounds__(kSymT * kSymRedGroups) void k_coarsest_sym_reduce(
    int nT, int n, const double* __restrict__ P, const double* __restrict__ Q, int maxc,
    const int* __restrict__ cmap, T* __restrict__ e, const Scalars* sc, int check_done) {
    if (check_done && sc->done) return;
    __shared__ double part[kSymRedGroups][kSymT];
    constexpr int G = kSymRedGroups;
    const int I = blockIdx.x, i = threadIdx.x % kSymT, q = threadIdx.x / kSymT;
    const int nc = (I + kSymChunk) / kSymChunk;   // chunks of tile row I (I + 1 tiles)
    double v = 0.0;
    for (int c = q; c < nc; c += G) v += Q[((size_t)I * maxc + c) * kSymT + i];
    const double* pr = P + (size_t)I * nT * kSymT + i;
    int K = I + 1 + q;
    for (; K + 3 * G < nT; K += 4 * G) {
        const double a0 = pr[(size_t)K * kSymT], a1 = pr[(size_t)(K + G) * kSymT];
        const double a2 = pr[(size_t)(K + 2 * G) * kSymT], a3 = pr[(size_t)(K + 3 * G) * kSymT];
        v += (a0 + a1) + (a2 + a3);
    }
    for (; K < nT; K += G) v += pr[(size_t)K * kSymT];
    part[q][i] = v;
    __syncthreads();
    if (q != 0) return;
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) t += part[g][i];
    const int row = I * kSymT + i;
    if (row < n) e[cmap[row]] = (T)t;
}

// ---------------------------------------------------------------------------
// set-up kernels

// Level-2 face blocks from the fine faces on the element boundary:
//   D[e][d] = sum_{tau on face d} T_f phi(tau) phi(tau)^T       (d = -x,+x,-y,+y,-z,+z)
//   Aoff[e][ax] = -sum_{tau on face +ax} T_f phi_e(tau) phi_{e+ax}(tau')^T
// (the terms of eq. discrete varia for faces between elements)
__global__ __launch_bounds__(256) void k_galerkin2(FineGeom g, const double* __restrict__ kt,
                                                   const double* __restrict__ phi, const int* __restrict__ nkeep,
                                                   int L, double* __restrict__ D, double* __restrict__ Aoff) {
    __shared__ double sT[6][64];
    __shared__ double sP[6][kMaxL2][64];    // own face rows
    __shared__ double sN[3][kMaxL2][64];    // neighbour face rows (+ faces)
    const int e = blockIdx.x;
    const int ex = e % g.mx, ey = (e / g.mx) % g.my, ez = e / (g.mx * g.my);
    auto gid = [&](int x, int y, int z) { return eidx(g, x, y, z); };
    for (int t = threadIdx.x; t < 6 * 64; t += blockDim.x) {
        const int d = t / 64, f = t % 64;
        const int ax = d >> 1;
        const bool plus = d & 1;
        const int u = f & 7, v = f >> 3;     // in-face coordinates
        int i, j, k;
        if (ax == 0) { i = plus ? 7 : 0; j = u; k = v; }
        else if (ax == 1) { i = u; j = plus ? 7 : 0; k = v; }
        else { i = u; j = v; k = plus ? 7 : 0; }
        const int gx = ex * 8 + i, gy = ey * 8 + j, gz = ez * 8 + k;
        const int nx_ = gx + (ax == 0 ? (plus ? 1 : -1) : 0);
        const int ny_ = gy + (ax == 1 ? (plus ? 1 : -1) : 0);
        const int nz_ = gz + (ax == 2 ? (plus ? 1 : -1) : 0);
        const bool inside = nx_ >= 0 && nx_ < g.nx && ny_ >= 0 && ny_ < g.ny && nz_ >= 0 && nz_ < g.nz;
        double T = 0.0;
        if (inside) {
            // kappa~ of this face's direction (three arrays for orthotropic K)
            const size_t off = g.ortho ? (size_t)ax * g.ncell() : 0;
            const double a = kt[off + gid(gx, gy, gz)], b = kt[off + gid(nx_, ny_, nz_)];
            T = 2.0 * a * b / (a + b) * (ax == 0 ? 1.0 : (ax == 1 ? g.cy : g.cz));
        }
        sT[d][f] = T;
        const int c = i + 8 * (j + 8 * k);
        for (int jj = 0; jj < L; ++jj) sP[d][jj][f] = phi[((size_t)e * L + jj) * 512 + phi_pos(c)];
        if (plus) {
            const int en = e + (ax == 0 ? 1 : (ax == 1 ? g.mx : g.mx * g.my));
            const int ci = ax == 0 ? 0 : i, cj = ax == 1 ? 0 : j, ck = ax == 2 ? 0 : k;
            const int cn = ci + 8 * (cj + 8 * ck);
            for (int jj = 0; jj < L; ++jj)
                sN[ax][jj][f] = inside ? phi[((size_t)en * L + jj) * 512 + phi_pos(cn)] : 0.0;
        }
    }
    __syncthreads();
    const int LL = L * L;
    for (int t = threadIdx.x; t < 9 * LL; t += blockDim.x) {
        const int blk = t / LL, a = (t % LL) / L, b = t % L;
        double s = 0.0;
        if (blk < 6) {
            for (int f = 0; f < 64; ++f) s += sT[blk][f] * sP[blk][a][f] * sP[blk][b][f];
            D[((size_t)e * 6 + blk) * LL + a * L + b] = s;
        } else {
            const int ax = blk - 6;
            const int d = 2 * ax + 1;
            for (int f = 0; f < 64; ++f) s += sT[d][f] * sP[d][a][f] * sN[ax][b][f];
            Aoff[((size_t)e * 3 + ax) * LL + a * L + b] = -s;
        }
    }
}

// Face blocks of level l+1 from those of level l (Galerkin with V_E):
//   D_up[E][d] = sum_{c on face d of E} V_c^T D[c][d] V_c
//   Aoff_up[E][ax] = sum_{c on face +ax of E} V_c^T Aoff[c][ax] V'_{c+ax}
__global__ __launch_bounds__(256) void k_galerkin_up(CoarseGeom lo, CoarseGeom up, const double* __restrict__ Dlo,
                                                     const double* __restrict__ Aofflo,
                                                     const double* __restrict__ V,
                                                     const int* __restrict__ nkeep_up, double* __restrict__ Dup,
                                                     double* __restrict__ Aoffup) {
    __shared__ double sB[kMaxL * kMaxL];     // level-l block
    __shared__ double sV[kMaxL * kMaxL];     // V_c   (Lp x Lu)
    __shared__ double sW[kMaxL * kMaxL];     // V'_c' (Lp x Lu)
    __shared__ double sBW[kMaxL * kMaxL];    // B V'  (Lp x Lu)
    const int E = blockIdx.x;
    const int agg = lo.agg, Lp = lo.L, Lu = up.L;
    const int n = agg * agg * agg * Lp;
    const int Ex = E % up.mx, Ey = (E / up.mx) % up.my, Ez = E / (up.mx * up.my);
    const int Ec[3] = {Ex, Ey, Ez};
    const int ext[3] = {up.mx, up.my, up.mz};
    const int estride[3] = {1, up.mx, up.mx * up.my};
    const int cstride[3] = {1, lo.mx, lo.mx * lo.my};
    for (int blk = 0; blk < 9; ++blk) {
        const bool isD = blk < 6;
        const int d = isD ? blk : 2 * (blk - 6) + 1;
        const int ax = d >> 1;
        const bool plus = d & 1;
        const bool has_nb = isD || (Ec[ax] + 1 < ext[ax]);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (has_nb) {
            for (int f = 0; f < agg * agg; ++f) {
                const int u = f % agg, v = f / agg;
                int q[3];
                q[ax] = plus ? agg - 1 : 0;
                q[(ax + 1) % 3] = u;
                q[(ax + 2) % 3] = v;
                const int p = q[0] + agg * (q[1] + agg * q[2]);
                const int c = (Ex * agg + q[0]) + lo.mx * ((Ey * agg + q[1]) + lo.my * (Ez * agg + q[2]));
                // stage B, V_c and (for couplings) V'_{c'}
                for (int t = threadIdx.x; t < Lp * Lp; t += blockDim.x)
                    sB[t] = isD ? Dlo[((size_t)c * 6 + d) * Lp * Lp + t] : Aofflo[((size_t)c * 3 + ax) * Lp * Lp + t];
                for (int t = threadIdx.x; t < Lp * Lu; t += blockDim.x) {
                    const int b = t / Lu, j = t % Lu;
                    sV[t] = V[((size_t)E * Lu + j) * n + p * Lp + b];
                    if (isD) {
                        sW[t] = sV[t];
                    } else {
                        int qn[3] = {q[0], q[1], q[2]};
                        qn[ax] = 0;
                        const int pn = qn[0] + agg * (qn[1] + agg * qn[2]);
                        const int En = E + estride[ax];
                        sW[t] = V[((size_t)En * Lu + j) * n + pn * Lp + b];
                    }
                }
                __syncthreads();
                for (int t = threadIdx.x; t < Lp * Lu; t += blockDim.x) {
                    const int a = t / Lu, j = t % Lu;
                    double s = 0.0;
                    for (int b = 0; b < Lp; ++b) s += sB[a * Lp + b] * sW[b * Lu + j];
                    sBW[t] = s;
                }
                __syncthreads();
                for (int t = threadIdx.x, k = 0; t < Lu * Lu; t += blockDim.x, ++k) {
                    const int i = t / Lu, j = t % Lu;
                    double s = 0.0;
                    for (int a = 0; a < Lp; ++a) s += sV[a * Lu + i] * sBW[a * Lu + j];
                    acc[k] += s;
                }
                __syncthreads();
                (void)cstride;
            }
        }
        for (int t = threadIdx.x, k = 0; t < Lu * Lu; t += blockDim.x, ++k) {
            if (isD) Dup[((size_t)E * 6 + d) * Lu * Lu + t] = acc[k];
            else Aoffup[((size_t)E * 3 + ax) * Lu * Lu + t] = acc[k];
        }
    }
    (void)nkeep_up;
}

// Ad = Aint + sum_d D[e][d]
__global__ void k_assemble_diag(CoarseGeom g, const double* __restrict__ Aint, const double* __restrict__ D,
                                double* __restrict__ Ad) {
    const int e = blockIdx.x;
    const int LL = g.L * g.L;
    for (int t = threadIdx.x; t < LL; t += blockDim.x) {
        double v = Aint[(size_t)e * LL + t];
        for (int d = 0; d < 6; ++d) v += D[((size_t)e * 6 + d) * LL + t];
        Ad[(size_t)e * LL + t] = v;
    }
}

// In-place inverse of an SPD n x n matrix (n <= kMaxL) by one wavefront:
// lane 0 factors A = L L^T (Lw, lower), then lane k < n solves
// L L^T x = e_k for column k.  Padded slots (index >= nk) get identity.
// Returns false (in every lane) if A is not numerically SPD.
__device__ bool small_spd_inverse_wave(double* A, int n, int nk, double* Lw, int* flag) {
    const int lane = threadIdx.x & 63;
    for (int t = lane; t < n * n; t += 64) {
        const int i = t / n, j = t % n;
        if (i >= nk || j >= nk) A[t] = (i == j) ? 1.0 : 0.0;
    }
    wave_sync();
    if (lane == 0) {
        int ok = 1;
        for (int j = 0; j < n; ++j) {
            double d = A[j * n + j];
            for (int k = 0; k < j; ++k) d -= Lw[j * n + k] * Lw[j * n + k];
            if (!(d > 0.0)) {
                ok = 0;
                d = 1.0;
            }
            const double ljj = sqrt(d);
            Lw[j * n + j] = ljj;
            for (int i = j + 1; i < n; ++i) {
                double v = A[i * n + j];
                for (int k = 0; k < j; ++k) v -= Lw[i * n + k] * Lw[j * n + k];
                Lw[i * n + j] = v / ljj;
            }
            for (int i = 0; i < j; ++i) Lw[i * n + j] = 0.0;
        }
        *flag = ok;
    }
    wave_sync();
    if (lane < n) {
        const int kcol = lane;
        double y[kMaxL];
#pragma unroll
        for (int i = 0; i < kMaxL; ++i) {
            if (i < n) {
                double v = (i == kcol) ? 1.0 : 0.0;
#pragma unroll
                for (int k = 0; k < kMaxL; ++k)
                    if (k < i) v -= Lw[i * n + k] * y[k];
                y[i] = v / Lw[i * n + i];
            }
        }
#pragma unroll
        for (int i = kMaxL - 1; i >= 0; --i) {
            if (i < n) {
                double v = y[i];
#pragma unroll
                for (int k = 0; k < kMaxL; ++k)
                    if (k > i && k < n) v -= Lw[k * n + i] * y[k];
                y[i] = v / Lw[i * n + i];
            }
        }
#pragma unroll
        for (int i = 0; i < kMaxL; ++i)
            if (i < n) A[i * n + kcol] = y[i];
    }
    wave_sync();
    return *flag != 0;
}

// Block IC(0) pivots of the level-l smoother, one workgroup per parent:
// the children of one hyperplane (at most 12) are factored in parallel,
// one wavefront each, with the Schur updates of the lower neighbours'
// couplings lane-parallel over the L x L entries.
constexpr int kMaxPlane = 12;   // children per hyperplane of a 4^3 parent
__global__ __launch_bounds__(64 * kMaxPlane) void k_blockic_setup(CoarseGeom g, const double* __restrict__ Ad,
                                                                   const double* __restrict__ Aoff,
                                                                   const int* __restrict__ nkeep, double* Dinv,
                                                                   int* bad) {
    __shared__ int pos[kMaxChildren], off[12];
    extern __shared__ double work_lds[];   // [children of the widest plane][3][L * L]
    __shared__ int flags[kMaxPlane];
    const int E = blockIdx.x;
    const int L = g.L, agg = g.agg, LL = L * L;
    build_planes(agg, pos, off);
    const int nplanes = 3 * (agg - 1) + 1;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int s = 0; s < nplanes; ++s) {
        const int cnt = off[s + 1] - off[s];
        if (w < cnt) {
            const int p = pos[off[s] + w];
            const int c = child_of(g, E, p);
            double* P = work_lds + (size_t)(3 * w) * LL;
            double* T = P + LL;
            double* Lw = T + LL;
            for (int t = lane; t < LL; t += 64) P[t] = Ad[(size_t)c * LL + t];
            const int q[3] = {p % agg, (p / agg) % agg, p / (agg * agg)};
            const int cstep[3] = {1, g.mx, g.mx * g.my};
            wave_sync();
            for (int ax = 0; ax < 3; ++ax) {
                if (q[ax] == 0) continue;
                const int cn = c - cstep[ax];
                const double* O = Aoff + ((size_t)cn * 3 + ax) * LL;   // A(cn, c)
                const double* Di = Dinv + (size_t)cn * LL;
                // T = Dinv_cn O ; P -= O^T T
                for (int t = lane; t < LL; t += 64) {
                    const int i = t / L, j = t % L;
                    double v = 0.0;
                    for (int b = 0; b < L; ++b) v += Di[i * L + b] * O[b * L + j];
                    T[t] = v;
                }
                wave_sync();
                for (int t = lane; t < LL; t += 64) {
                    const int i = t / L, j = t % L;
                    double v = 0.0;
                    for (int b = 0; b < L; ++b) v += O[b * L + i] * T[b * L + j];
                    P[t] -= v;
                }
                wave_sync();
            }
            // symmetrise (all reads before the writes), invert
            double sym[(kMaxL * kMaxL + 63) / 64];
#pragma unroll
            for (int u = 0; u < (kMaxL * kMaxL + 63) / 64; ++u) {
                const int t = lane + 64 * u;
                sym[u] = t < LL ? 0.5 * (P[t] + P[(t % L) * L + t / L]) : 0.0;
            }
            wave_sync();
#pragma unroll
            for (int u = 0; u < (kMaxL * kMaxL + 63) / 64; ++u) {
                const int t = lane + 64 * u;
                if (t < LL) P[t] = sym[u];
            }
            wave_sync();
            if (!small_spd_inverse_wave(P, L, nkeep[c], Lw, &flags[w]) && lane == 0) atomicOr(bad, 2);
            for (int t = lane; t < LL; t += 64) Dinv[(size_t)c * LL + t] = P[t];
        }
        __threadfence();
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
}

// G[c][2ax] = Dinv_c A(c, c - e_ax), G[c][2ax+1] = Dinv_c A(c, c + e_ax) for
// neighbours inside the same parent (zero otherwise)
__global__ __launch_bounds__(256) void k_blockic_couple(CoarseGeom g, const double* __restrict__ Aoff,
                                                         const double* __restrict__ Dinv, double* __restrict__ G) {
    const int c = blockIdx.x;
    const int L = g.L, LL = L * L, agg = g.agg;
    const int cx = c % g.mx, cy = (c / g.mx) % g.my, cz = c / (g.mx * g.my);
    const int q[3] = {cx % agg, cy % agg, cz % agg};
    const int stride[3] = {1, g.mx, g.mx * g.my};
    const double* Di = Dinv + (size_t)c * LL;
    for (int t = threadIdx.x; t < 6 * LL; t += blockDim.x) {
        const int d = t / LL, a = (t % LL) / L, b = t % L;
        const int ax = d >> 1;
        const bool upper = d & 1;
        double v = 0.0;
        if (upper ? (q[ax] < agg - 1) : (q[ax] > 0)) {
            for (int k = 0; k < L; ++k) {
                // A(c, c - e) = Aoff[c - e][ax]^T ; A(c, c + e) = Aoff[c][ax]
                const double A = upper ? Aoff[(((size_t)c * 3 + ax) * L + k) * L + b]
                                       : Aoff[(((size_t)(c - stride[ax]) * 3 + ax) * L + b) * L + k];
                v += Di[a * L + k] * A;
            }
        }
        G[((size_t)c * 6 + d) * LL + a * L + b] = v;
    }
}

// coarsest dense matrix over the compact unknowns (cinv: padded -> compact
// or -1); the matrix must be zeroed beforehand
__global__ void k_build_coarsest(CoarseGeom g, const double* __restrict__ Ad, const double* __restrict__ Aoff,
                                 const int* __restrict__ cinv, int np, double* __restrict__ dense) {
    const int e = blockIdx.x;
    const int L = g.L, LL = L * L;
    const int cx = e % g.mx, cy = (e / g.mx) % g.my, cz = e / (g.mx * g.my);
    const int cc[3] = {cx, cy, cz};
    const int ext[3] = {g.mx, g.my, g.mz};
    const int stride[3] = {1, g.mx, g.mx * g.my};
    for (int t = threadIdx.x; t < LL; t += blockDim.x) {
        const int a = t / L, b = t % L;
        const int i = cinv[e * L + a];
        if (i < 0) continue;
        const int jd = cinv[e * L + b];
        if (jd >= 0) dense[(size_t)i * np + jd] = Ad[(size_t)e * LL + t];
        for (int ax = 0; ax < 3; ++ax) {
            if (cc[ax] + 1 >= ext[ax]) continue;
            const int en = e + stride[ax];
            const int j = cinv[en * L + b];
            if (j < 0) continue;
            const double v = Aoff[((size_t)e * 3 + ax) * LL + t];
            dense[(size_t)i * np + j] = v;
            dense[(size_t)j * np + i] = v;
        }
    }
}

template <typename S, typename T>
__global__ void k_convert(const S* __restrict__ src, T* __restrict__ dst, int64_t n, const Scalars* sc) {
    if (sc && sc->done) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (T)src[i];
}

// ---------------------------------------------------------------------------
// launchers

#define SPECMG_LP_DISPATCH(LV, ...)                           \
    switch (LV) {                                             \
        case 4: { constexpr int LP = 4; __VA_ARGS__; } break;     \
        case 5: { constexpr int LP = 5; __VA_ARGS__; } break;     \
        case 6: { constexpr int LP = 6; __VA_ARGS__; } break;     \
        case 7: { constexpr int LP = 7; __VA_ARGS__; } break;     \
        case 8: { constexpr int LP = 8; __VA_ARGS__; } break;     \
        case 9: { constexpr int LP = 9; __VA_ARGS__; } break;     \
        case 10: { constexpr int LP = 10; __VA_ARGS__; } break;   \
        case 11: { constexpr int LP = 11; __VA_ARGS__; } break;   \
        case 12: { constexpr int LP = 12; __VA_ARGS__; } break;   \
        case 13: { constexpr int LP = 13; __VA_ARGS__; } break;   \
        default: { constexpr int LP = kMaxLc; __VA_ARGS__; } break; \
    }

// The same for 2x aggregation and widths up to 9: one wavefront per parent.
// Its lanes take the kept rows of the 8 children in turn (row q of the
// parent is slot a of child position p, q = the kept rows of the positions
// before p, plus a), 64 rows per pass, so the dead padded slots take no
// lanes; the restriction sums are wavefront reductions, with no LDS and no
// block barrier.
template <typename T, int LP, int LU>
__global__ __launch_bounds__(256) void k_coarse_resid_restrict_w(
    CoarseGeom g, const T* __restrict__ Ad, const T* __restrict__ Aoff, const T* __restrict__ r,
    const T* __restrict__ u, const T* __restrict__ V, const int* __restrict__ nkeep_up, int Lup,
    T* __restrict__ rup, const Scalars* sc, int check_done) {
    if (check_done && sc->done) return;
    const int lane = threadIdx.x & 63;
    const int E = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (E >= g.M) return;   // whole wavefront; no block barriers below
    const int L = g.L, n = 8 * L;
    int pre[9];
    pre[0] = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) pre[q + 1] = pre[q] + (g.nkeep ? g.nkeep[child_of(g, E, q)] : L);
    const int rows = pre[8];
    const int nk = nkeep_up[E];
    double acc[LU];
#pragma unroll
    for (int j = 0; j < LU; ++j) acc[j] = 0.0;
    for (int q0 = 0; q0 < rows; q0 += 64) {
        const int qr = q0 + lane;
        if (qr < rows) {
            int p = 0;
#pragma unroll
            for (int q = 1; q < 8; ++q) p += qr >= pre[q] ? 1 : 0;
            const int a = qr - pre[p];
            const int c = child_of(g, E, p);
            const double sv = (double)(r[(size_t)c * L + a] - block_row_apply<T, LP>(g, Ad, Aoff, u, c, a));
            const T* vc = V + (size_t)E * Lup * n + (size_t)p * L + a;
#pragma unroll
            for (int j = 0; j < LU; ++j)
                if (j < nk) acc[j] += (double)vc[(size_t)j * n] * sv;
        }
    }
    double mine = 0.0;
#pragma unroll
    for (int j = 0; j < LU; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == j) mine = v;
    }
    if (lane < Lup) rup[(size_t)E * Lup + lane] = lane < nk ? (T)mine : T(0);
}

template <typename T>
void launch_coarse_resid_restrict(const CoarseGeom& g, const T* Ad, const T* Aoff, const T* r, const T* u,
                                  const T* V, const int* nkeep_up, int Lup, T* rup, const Scalars* sc,
                                  int check_done, hipStream_t s) {
    const int rows = g.agg * g.agg * g.agg * g.L;
    const int th = std::min(kCoarseThreads, (rows + 63) / 64 * 64);
    if (g.L < 4 || g.L > kMaxLc) throw HipError{hipErrorInvalidValue, "coarse residual width"};
    if (Lup > kMaxLc) throw HipError{hipErrorInvalidValue, "coarse residual upper width"};
    // wider blocks keep about 8 L > 64 rows per parent, two passes of the
    // wavefront: there the workgroup form is faster
    if (g.agg == 2 && g.L <= 9) {
        const int nb = (g.M + 3) / 4;
        if (Lup <= kNarrow) {
            SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_resid_restrict_w<T, LP, kNarrow>), dim3(nb),
                                                       dim3(256), 0, s, g, Ad, Aoff, r, u, V, nkeep_up, Lup, rup, sc,
                                                       check_done));
        } else {
            SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_resid_restrict_w<T, LP, kMaxLc>), dim3(nb),
                                                       dim3(256), 0, s, g, Ad, Aoff, r, u, V, nkeep_up, Lup, rup, sc,
                                                       check_done));
        }
    } else if (Lup <= kNarrow) {
        SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_resid_restrict<T, LP, kNarrow>), dim3(g.M), dim3(th), 0,
                                                   s, g, Ad, Aoff, r, u, V, nkeep_up, Lup, rup, sc, check_done));
    } else {
        SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_resid_restrict<T, LP, kMaxLc>), dim3(g.M), dim3(th), 0,
                                                   s, g, Ad, Aoff, r, u, V, nkeep_up, Lup, rup, sc, check_done));
    }
}

template <typename T>
void launch_coarse_prolong(const CoarseGeom& g, T* u, const T* V, const int* nkeep_up, int Lup, const T* eup,
                           const Scalars* sc, int check_done, hipStream_t s) {
    const int rows = g.agg * g.agg * g.agg * g.L;
    const int th = std::min(kCoarseThreads, (rows + 63) / 64 * 64);
    if (Lup > kMaxLc) throw HipError{hipErrorInvalidValue, "coarse prolongation upper width"};
    if (Lup <= kNarrow)
        hipLaunchKernelGGL((k_coarse_prolong<T, kNarrow>), dim3(g.M), dim3(th), 0, s, g, u, V, nkeep_up, Lup, eup, sc,
                           check_done);
    else
        hipLaunchKernelGGL((k_coarse_prolong<T, kMaxLc>), dim3(g.M), dim3(th), 0, s, g, u, V, nkeep_up, Lup, eup, sc,
                           check_done);
}

// dynamic LDS of the sweep kernels; couplings are staged when they fit
// parents per sweep workgroup: with 2x aggregation as many as fill about
// 512 threads (a parent has 8 L rows), otherwise one
static int sweep_parents(const CoarseGeom& g) {
    const int rows = g.agg * g.agg * g.agg * g.L;
    if (g.agg != 2) return 1;
    const int p = 512 / rows;
    return p < 1 ? 1 : (p > kMaxChildren / 8 ? kMaxChildren / 8 : p);
}
static int sweep_threads(const CoarseGeom& g) {
    const int rows = sweep_parents(g) * g.agg * g.agg * g.agg * g.L;
    return (rows + 63) / 64 * 64;
}
static int sweep_blocks(const CoarseGeom& g) {
    const int np = sweep_parents(g);
    return (g.M + np - 1) / np;
}

// u = M_l^{-1} r
template <typename T>
void launch_coarse_smooth(const CoarseGeom& g, const T* Dinv, const T* G, const T* r, T* u, const Scalars* sc,
                          int check_done, hipStream_t s) {
    if (g.L < 4 || g.L > kMaxLc || sweep_threads(g) > 768) throw HipError{hipErrorInvalidValue, "coarse sweep shape"};
    if (g.agg == 2) {
        SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_sweep<T, LP, true>), dim3(sweep_blocks(g)), dim3(sweep_threads(g)), 0,
                                                   s, g, 0, (const T*)nullptr, (const T*)nullptr, Dinv, G, r,
                                                   (const T*)nullptr, u, sc, check_done, sweep_parents(g)));
    } else {
        SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_sweep<T, LP, false>), dim3(sweep_blocks(g)), dim3(sweep_threads(g)), 0,
                                                   s, g, 0, (const T*)nullptr, (const T*)nullptr, Dinv, G, r,
                                                   (const T*)nullptr, u, sc, check_done, sweep_parents(g)));
    }
}

// e = u + M_l^{-1} (r - A_l u)
template <typename T>
void launch_coarse_resid_smooth(const CoarseGeom& g, const T* Ad, const T* Dinv, const T* Aoff, const T* G,
                                const T* r, const T* u, T* e, const Scalars* sc, int check_done, hipStream_t s) {
    if (g.L < 4 || g.L > kMaxLc || sweep_threads(g) > 768) throw HipError{hipErrorInvalidValue, "coarse sweep shape"};
    if (g.agg == 2) {
        SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_sweep<T, LP, true>), dim3(sweep_blocks(g)), dim3(sweep_threads(g)), 0,
                                                   s, g, 1, Ad, Aoff, Dinv, G, r, u, e, sc, check_done, sweep_parents(g)));
    } else {
        SPECMG_LP_DISPATCH(g.L, hipLaunchKernelGGL((k_coarse_sweep<T, LP, false>), dim3(sweep_blocks(g)), dim3(sweep_threads(g)), 0,
                                                   s, g, 1, Ad, Aoff, Dinv, G, r, u, e, sc, check_done, sweep_parents(g)));
    }
}

int coarsest_sym_tile() { return kSymT; }

size_t coarsest_sym_packed_doubles(int np) {
    const size_t nT = (size_t)np / kSymT;
    return nT * (nT + 1) / 2 * kSymT * kSymT;
}

// host-side chunk table of the symmetric product: (tile row, first tile)
std::vector<int2> coarsest_sym_chunks(int np, int* maxc) {
    const int nT = np / kSymT;
    std::vector<int2> ch;
    *maxc = (nT + kSymChunk - 1) / kSymChunk;
    for (int I = 0; I < nT; ++I)
        for (int J0 = 0; J0 <= I; J0 += kSymChunk) ch.push_back(make_int2(I, J0));
    return ch;
}

void launch_pack_lower_tiles(const double* dense, int np, double* packed, hipStream_t s) {
    const int nT = np / kSymT;
    hipLaunchKernelGGL(k_pack_lower_tiles, dim3(nT * (nT + 1) / 2), dim3(256), 0, s, dense, np, packed);
}

void launch_coarsest_sym(int n, int np, const double* packed, const int2* chunks, int nchunks, int maxc,
                         const int* cmap, const double* r, double* e, double* rc, double* P, double* Q,
                         const Scalars* sc, int check_done, hipStream_t s) {
    const int nT = np / kSymT;
    hipLaunchKernelGGL((k_gather_compact<double>), dim3(std::min((n + 255) / 256, 1024)), dim3(256), 0, s, n, cmap,
                       r, rc, sc, check_done);
    SPECMG_TIMED_LAUNCH(k_coarsest_sym, dim3(nchunks), dim3(64 * kSymWaves), 0, s, nT, chunks, packed, rc, P, Q,
                        maxc, sc, check_done);
    hipLaunchKernelGGL((k_coarsest_sym_reduce<double>), dim3(nT), dim3(kSymT * kSymRedGroups), 0, s, nT, n, P, Q, maxc, cmap, e, sc,
                       check_done);
}

template <typename T>
void launch_coarsest(int n, int np, const double* Pinv, const int* cmap, const T* r, T* e, double* rc,
                     const Scalars* sc, int check_done, hipStream_t s) {
    const size_t lds = (size_t)std::min(n, kCoarsestChunk) * sizeof(double);
    if (n <= kCoarsestChunk) {
        SPECMG_TIMED_LAUNCH((k_coarsest<T, 1>), dim3((n + 3) / 4), dim3(256), lds, s, n, np, Pinv, cmap, r, e, sc,
                            check_done);
    } else {
        hipLaunchKernelGGL((k_gather_compact<T>), dim3(std::min((n + 255) / 256, 1024)), dim3(256), 0, s, n, cmap, r,
                           rc, sc, check_done);
        SPECMG_TIMED_LAUNCH((k_coarsest_rows<T>), dim3((n + kCoarsestRows - 1) / kCoarsestRows), dim3(256), lds, s,
                            n, np, Pinv, cmap, rc, e, sc, check_done);
    }
}

void launch_galerkin2(const FineGeom& g, const double* kt, const double* phi, const int* nkeep, int L, double* D,
                      double* Aoff, hipStream_t s) {
    hipLaunchKernelGGL(k_galerkin2, dim3(g.mx * g.my * g.mz), dim3(256), 0, s, g, kt, phi, nkeep, L, D, Aoff);
}

void launch_galerkin_up(const CoarseGeom& lo, const CoarseGeom& up, const double* Dlo, const double* Aofflo,
                        const double* V, const int* nkeep_up, double* Dup, double* Aoffup, hipStream_t s) {
    hipLaunchKernelGGL(k_galerkin_up, dim3(up.m), dim3(256), 0, s, lo, up, Dlo, Aofflo, V, nkeep_up, Dup, Aoffup);
}

void launch_assemble_diag(const CoarseGeom& g, const double* Aint, const double* D, double* Ad, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble_diag, dim3(g.m), dim3(128), 0, s, g, Aint, D, Ad);
}

void launch_blockic_setup(const CoarseGeom& g, const double* Ad, const double* Aoff, const int* nkeep,
                          double* Dinv, double* G, int* bad, hipStream_t s) {
    // widest hyperplane of the parent's children: 3 (agg 2) or 12 (agg 4)
    const int wmax = g.agg == 2 ? 3 : kMaxPlane;
    const size_t shmem = (size_t)wmax * 3 * g.L * g.L * sizeof(double);
    if (g.L > kMaxL || shmem > 64 * 1024) throw HipError{hipErrorInvalidValue, "block-IC set-up shape"};
    hipLaunchKernelGGL(k_blockic_setup, dim3(g.M), dim3(64 * kMaxPlane), shmem, s, g, Ad, Aoff, nkeep, Dinv, bad);
    hipLaunchKernelGGL(k_blockic_couple, dim3(g.m), dim3(256), 0, s, g, Aoff, Dinv, G);
}

void launch_build_coarsest(const CoarseGeom& g, const double* Ad, const double* Aoff, const int* cinv, int np,
                           double* dense, hipStream_t s) {
    hipLaunchKernelGGL(k_build_coarsest, dim3(g.m), dim3(128), 0, s, g, Ad, Aoff, cinv, np, dense);
}

template <typename S, typename T>
void launch_convert(const S* src, T* dst, int64_t n, hipStream_t s, const Scalars* sc) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL((k_convert<S, T>), dim3((int)b), dim3(256), 0, s, src, dst, n, sc);
}

template void launch_coarse_smooth<double>(const CoarseGeom&, const double*, const double*, const double*, double*,
                                           const Scalars*, int, hipStream_t);
template void launch_coarse_smooth<float>(const CoarseGeom&, const float*, const float*, const float*, float*,
                                          const Scalars*, int, hipStream_t);
template void launch_coarse_resid_restrict<double>(const CoarseGeom&, const double*, const double*, const double*,
                                                   const double*, const double*, const int*, int, double*,
                                                   const Scalars*, int, hipStream_t);
template void launch_coarse_resid_restrict<float>(const CoarseGeom&, const float*, const float*, const float*,
                                                  const float*, const float*, const int*, int, float*,
                                                  const Scalars*, int, hipStream_t);
template void launch_coarse_prolong<double>(const CoarseGeom&, double*, const double*, const int*, int,
                                            const double*, const Scalars*, int, hipStream_t);
template void launch_coarse_prolong<float>(const CoarseGeom&, float*, const float*, const int*, int, const float*,
                                           const Scalars*, int, hipStream_t);
template void launch_coarse_resid_smooth<double>(const CoarseGeom&, const double*, const double*, const double*,
                                                 const double*, const double*, const double*, double*,
                                                 const Scalars*, int, hipStream_t);
template void launch_coarse_resid_smooth<float>(const CoarseGeom&, const float*, const float*, const float*,
                                                const float*, const float*, const float*, float*, const Scalars*,
                                                int, hipStream_t);
template void launch_coarsest<double>(int, int, const double*, const int*, const double*, double*, double*,
                                      const Scalars*, int, hipStream_t);
template void launch_coarsest<float>(int, int, const double*, const int*, const float*, float*, double*,
                                     const Scalars*, int, hipStream_t);
template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t, const Scalars*);
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t, const Scalars*);

}  // namespace specmg
