// Internal declarations shared by the specmg HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <vector>

namespace specmg {

// Event pair for the next timed kernel launch: hipExtLaunchKernelGGL stamps
// the dispatch's own start and end into them, so the interval is the
// kernel alone (no launch gaps, no neighbouring kernels).  Set by the
// context's profiling code on the calling thread, consumed by one launch.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelEvents g_kev;

#define SPECMG_TIMED_LAUNCH(K, GRID, BLOCK, SHM, S, ...)                                \
    do {                                                                                \
        if (::specmg::g_kev.start) {                                                    \
            const hipEvent_t ev0_ = ::specmg::g_kev.start, ev1_ = ::specmg::g_kev.stop;  \
            ::specmg::g_kev = ::specmg::KernelEvents{};                                 \
            hipExtLaunchKernelGGL(K, GRID, BLOCK, SHM, S, ev0_, ev1_, 0, __VA_ARGS__);   \
        } else {                                                                        \
            hipLaunchKernelGGL(K, GRID, BLOCK, SHM, S, __VA_ARGS__);                    \
        }                                                                               \
    } while (0)

// failure of a HIP call or of a launch precondition inside a launcher;
// caught at the C-ABI boundary and returned as SPECMG_EDEVICE
struct HipError {
    hipError_t e;
    const char* what;
};

// Device memory of a context: the caller's allocator callbacks when given
// (specmg_setup_alloc), hipMalloc / hipFree otherwise.  get() throws
// HipError when no memory is returned.
struct DevAlloc {
    void* (*alloc)(size_t, void*, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* user = nullptr;
    hipStream_t stream = nullptr;
    void* get(size_t bytes) const {
        if (bytes == 0) bytes = 1;
        void* p = nullptr;
        if (alloc) {
            p = alloc(bytes, (void*)stream, user);
            if (!p) throw HipError{hipErrorOutOfMemory, "allocator callback returned no memory"};
        } else {
            const hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess) throw HipError{e, "hipMalloc"};
        }
        return p;
    }
    void put(void* p) const {
        if (!p) return;
        if (release) release(p, user);
        else (void)hipFree(p);
    }
};

constexpr int kSub = 8;             // level-2 element edge in cells
constexpr int kSub3 = 512;          // cells per level-2 element

// Position of cell c = x + 8 l (l = y + 8 z, the pencil) of a level-2
// element inside a column of its spectral basis: pairs of x interleaved
// over the 64 pencils, pos = (x / 2) 128 + 2 l + x % 2, so that one 16-byte
// load per lane of pair i (lane = pencil) reads 1 KB contiguous.
__host__ __device__ constexpr int phi_pos(int c) { return ((c & 7) >> 1) * 128 + 2 * (c >> 3) + (c & 1); }
constexpr int kPlanes = 22;         // hyperplanes i+j+k = s in an 8^3 block
constexpr int kMaxRedBlocks = 262144;

// ---------------------------------------------------------------------------
// Device-resident CG scalars.  Kernels read and update them so that a whole
// CG iteration runs without a host round trip.
struct Scalars {
    double rz;        // r.z of the current iterate
    double rz_new;    // r.z after the latest preconditioner application
    double pq;        // p.A p
    double alpha;     // step length of the current iteration
    double alpha_x;   // step still to be added to x (x += alpha_x p_old)
    double beta;
    double rr;        // ||r||^2
    double thresh2;   // (tol ||b||)^2
    double zq;        // z_new . q (flexible beta)
    double sum;       // generic reduction result
    double sum2;
    int done;         // 0 running, 1 converged, 2 breakdown
    int iter;         // number of A p products so far
    int flexible;     // 1: Polak-Ribiere beta
    int pbuf;         // index of the p buffer written by the last spmv
};

// Scratch for grid-wide deterministic reductions: per-block partials plus
// one arrival counter per reduction site.
struct RedBuf {
    double* partial;      // [kMaxRedBlocks * 2]
    double* partial2;     // [kFinBlocks * 2]: block sums of the finalize's first stage
    unsigned* ticket;     // finalize blocks done so far; zero between launches
};
// the finalize: kFinThreads threads per block, kFinPer partials per thread
constexpr int kFinThreads = 256;
constexpr int kFinPer = 8;
constexpr int kFinSpan = kFinThreads * kFinPer;
constexpr int kFinBlocks = kMaxRedBlocks / kFinSpan;

void launch_finalize(int site, int nblocks, Scalars* sc, RedBuf rb, double* out, int check_done,
                     hipStream_t s);

// what the finalize kernel does with the totals
enum RedSite { RS_PQ = 0, RS_RR = 1, RS_RZ = 2, RS_GEN = 3, RS_GEN2 = 4 };

// ---------------------------------------------------------------------------
// wavefront / block reductions (wave64); fixed combination order, so results
// are reproducible run to run.
// Reductions over the 64 lanes of a wavefront (every lane active; every
// lane receives the result).  Exchanges inside each 16-lane row use DPP
// (quad permutations, half-row and row mirrors); the four row results are
// combined through readlane.  Every lane of a row forms the same sums in
// the same order, so the result is identical in all lanes.  The DPP and
// readlane builtins move 32-bit integers, so values travel as their bits.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double read_lane(double v, int lane) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | (unsigned long long)lo);
}
__device__ __forceinline__ float read_lane(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);   // row_half_mirror
    v += dpp_move<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }
__device__ __forceinline__ float wave_sum(float v) { return wave_sum_dpp(v); }

// orders this wave's LDS and memory accesses (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// every source lane of the four patterns lies in the same row, so no
// lane falls back to the identity
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_move<0xB1>(v));
    v = fmax(v, dpp_move<0x4E>(v));
    v = fmax(v, dpp_move<0x141>(v));
    v = fmax(v, dpp_move<0x140>(v));
    return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// Sum over the block; every thread receives the result.  `sh` holds at
// least blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += sh[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double atomic_load_relaxed(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide reductions: every block writes its NV block sums to
// partial[k * kMaxRedBlocks + block] (no floating-point atomics); the
// finalize kernel launched right after sums them in a fixed order (ranges
// of partials, then the range sums), so results are reproducible.
template <int NV>
__device__ __forceinline__ void write_partials(const double (&v)[NV], RedBuf rb) {
    if (threadIdx.x == 0) {
        const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        for (int k = 0; k < NV; ++k) rb.partial[(size_t)k * kMaxRedBlocks + b] = v[k];
    }
}

// ---------------------------------------------------------------------------
// Geometry of the fine grid and its tiling.  A tile is EX level-2 elements
// along x (8*EX x 8 x 8 cells); one wavefront per element.
struct FineGeom {
    int nx, ny, nz;
    int mx, my, mz;       // level-2 elements per axis
    int ex;               // elements per tile along x (1, 2 or 4)
    int ntx, nty, ntz;    // tiles per axis
    int ntiles;
    int xcd_remap;        // 1: blockIdx -> tile mapping keeps each XCD on a slab
    // y and z face factors (hx/hy)^2 and (hx/hz)^2: kappa~ is stored as
    // kappa / hx^2, so a y (z) face coefficient is cy (cz) times the
    // harmonic mean of kappa~; exactly 1 on equal spacings
    double cy = 1.0, cz = 1.0;
    // orthotropic K = diag(kappa_x, kappa_y, kappa_z): kappa~ holds three
    // arrays of n values, kappa_d / h_d^2, and faces of axis d take the
    // harmonic mean of array d (cy = cz = 1)
    int ortho = 0;
    __host__ __device__ size_t ncell() const { return (size_t)nx * ny * nz; }
};

// Element order of the fine-level arrays the library keeps (kappa~, the
// IC(0) pivots, every vector of the solve): the 512 cells of each 8^3
// level-2 element are one contiguous 4 KB block, and the elements follow
// each other x fastest.  Inside the block cell (x, j, k) sits at phi_pos(c),
// c = x + 8 (j + 8 k), the layout of the level-2 basis columns: the x-pencil
// of row (j, k) is four pairs 128 words apart, so when lane j + 8 k loads
// pair i of its pencil, the wavefront reads one contiguous 1 KB block.
// Arrays the caller passes (permeability, sources, solutions, fluxes) keep
// the natural order x + nx (y + ny z).
__host__ __device__ inline size_t eidx(const FineGeom& g, int x, int y, int z) {
    const size_t e = (size_t)(x >> 3) + (size_t)g.mx * ((size_t)(y >> 3) + (size_t)g.my * (size_t)(z >> 3));
    return e * 512 + (size_t)phi_pos((x & 7) + 8 * ((y & 7) + 8 * (z & 7)));
}

// Coarse level l >= 2: elements on an (mx,my,mz) grid, padded width L.
struct CoarseGeom {
    int mx, my, mz, m;
    int L;                 // padded per-element width (target + 3)
    int agg;               // children per axis of a parent (level l+1)
    int px, py, pz, M;     // parents per axis / total (0 if l is the coarsest)
    const int* nkeep = nullptr;   // kept slots per element (device); rows beyond are zero
};

// ---------------------------------------------------------------------------
// launchers (k_fine.hip).  The V-cycle's fine-level kernels take T, the
// stored word of kappa~, the IC(0) pivots and the V-cycle vectors u and t,
// TB that of the level-2 basis, and C, the word of the arithmetic and of the
// level-2 vectors: (double, double, double) float64, (float, float, float)
// the FP32 V-cycle, (double, float, double) the FP32-basis mode, (float,
// float, double) float32 storage with float64 arithmetic.
template <typename T, typename C>
void launch_pre_smooth(const FineGeom& g, const T* kt, const T* invd, double* r, const double* q,
                       T* u, Scalars* sc, RedBuf rb, int mode, hipStream_t s);
template <typename T, typename TB, typename C>
void launch_resid_restrict(const FineGeom& g, const T* kt, const T* u, const double* r, const TB* phi,
                           const int* nkeep, int L, C* r2, Scalars* sc, int check_done, hipStream_t s);
template <typename T, typename TB, typename C>
void launch_prolong(const FineGeom& g, T* u, const TB* phi, const int* nkeep, int L, const C* e2,
                    Scalars* sc, int check_done, hipStream_t s);
// z = u + M^{-1} (r - A u) in one pass (the residual is not stored)
template <typename T, typename C>
void launch_post_fused(const FineGeom& g, const T* kt, const T* invd, const T* u, const double* r,
                       const double* q, double* z, Scalars* sc, RedBuf rb, int mode, hipStream_t s);
// p = z + beta p_old (p = z when first), x += alpha_x p_old
void launch_p_update(const FineGeom& g, const double* z, const double* pold, double* pnew, double* x, Scalars* sc,
                     int first, hipStream_t s);
// q = A p, p.q; records pbuf (the p buffer index) for the final x update
void launch_spmv_pcg(const FineGeom& g, const double* kt, const double* p, double* q, Scalars* sc, RedBuf rb,
                     int pbuf, hipStream_t s);
void launch_apply_A(const FineGeom& g, const double* kt, const double* x, const double* b, double* y,
                    int resid, hipStream_t s);
void launch_ic_setup(const FineGeom& g, const double* kt, double* invd, float* invd32, int* bad,
                     hipStream_t s);
// kt (element order) = perm (natural order) * scale
void launch_perm_to_kt(const FineGeom& g, const double* perm, double* kt, float* kt32, double scale, int* bad,
                       hipStream_t s);
// three components: array d of kt (element order) = component d of perm * scale[d]
void launch_perm3_to_kt(const FineGeom& g, const double* perm, double* kt, double sx, double sy, double sz,
                        int* bad, hipStream_t s);
// natural order <-> element order of one cell array
void launch_to_elem(const FineGeom& g, const double* nat, double* el, hipStream_t s);
void launch_to_natural(const FineGeom& g, const double* el, double* nat, hipStream_t s);

// vector utilities (k_fine.hip)
void launch_dot(const double* a, const double* b, int64_t n, double* out, RedBuf rb, int site,
                hipStream_t s);
void launch_sum_abs(const double* a, int64_t n, double* out_sum, double* out_abs, RedBuf rb,
                    hipStream_t s);
void launch_axpy_x(double* x, const double* p0, const double* p1, Scalars* sc, int64_t n,
                   hipStream_t s);
void launch_sub_mean(double* x, int64_t n, const double* sum, hipStream_t s);

// flexible GMRES (k_krylov.hip): device state of one restart cycle
constexpr int kMaxRestart = 64;
struct GmresState {
    double H[(kMaxRestart + 1) * kMaxRestart];   // column j at H + j (kMaxRestart + 1)
    double cs[kMaxRestart], sn[kMaxRestart], y[kMaxRestart];
    double g[kMaxRestart + 1], h[kMaxRestart + 1], h2[kMaxRestart + 1];
    double nrm2, inv, res, beta;
    int done;   // 1: converged or invariant space, 2: singular Hessenberg column
};
size_t mdot_part_doubles();
void launch_mdot(const double* V, int64_t pitch, int cnt, const double* w, int64_t n, double* part, double* out,
                 hipStream_t s);
void launch_maxpy(const double* V, int64_t pitch, int cnt, const double* coef, double sign, double* w, int64_t n,
                  hipStream_t s);
void launch_scale_dev(double* dst, const double* src, const double* factor, int64_t n, hipStream_t s);
void launch_gmres_begin(GmresState* st, double thr, hipStream_t s);
void launch_gmres_step(GmresState* st, int j, double thr, hipStream_t s);
void launch_gmres_lsq(GmresState* st, int k, hipStream_t s);
// copy / convert a vector; with sc non-null nothing is done once the solve
// has converged (sc->done), as in the V-cycle kernels
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s, const Scalars* sc = nullptr);
void launch_fill(double* dst, double v, int64_t n, hipStream_t s);
void launch_pcg_init(Scalars* sc, double thresh2, int flexible, hipStream_t s);

// coarse levels (k_coarse.hip)
template <typename T>
void launch_coarse_smooth(const CoarseGeom& g, const T* Dinv, const T* G, const T* r, T* u,
                          const Scalars* sc, int check_done, hipStream_t s);
template <typename T>
void launch_coarse_resid_restrict(const CoarseGeom& g, const T* Ad, const T* Aoff, const T* r,
                                  const T* u, const T* V, const int* nkeep_up, int Lup, T* rup,
                                  const Scalars* sc, int check_done, hipStream_t s);
template <typename T>
void launch_coarse_prolong(const CoarseGeom& g, T* u, const T* V, const int* nkeep_up, int Lup,
                           const T* eup, const Scalars* sc, int check_done, hipStream_t s);
template <typename T>
void launch_coarse_resid_smooth(const CoarseGeom& g, const T* Ad, const T* Dinv, const T* Aoff,
                                const T* G, const T* r, const T* u, T* e, const Scalars* sc,
                                int check_done, hipStream_t s);
template <typename T>
void launch_coarsest(int n, int np, const double* Pinv, const int* cmap, const T* r, T* e, double* rc,
                     const Scalars* sc, int check_done, hipStream_t s);
// values of the coarsest right-hand side staged in LDS at a time; wider
// coarsest spaces use the symmetric product below
constexpr int kCoarsestChunk = 8192;
// coarsest product over the packed lower tiles of the symmetric inverse
// (spaces wider than one LDS chunk); np a multiple of coarsest_sym_tile()
int coarsest_sym_tile();
size_t coarsest_sym_packed_doubles(int np);
std::vector<int2> coarsest_sym_chunks(int np, int* maxc);
void launch_pack_lower_tiles(const double* dense, int np, double* packed, hipStream_t s);
void launch_coarsest_sym(int n, int np, const double* packed, const int2* chunks, int nchunks, int maxc,
                         const int* cmap, const double* r, double* e, double* rc, double* P, double* Q,
                         const Scalars* sc, int check_done, hipStream_t s);

// set-up (k_coarse.hip)
void launch_galerkin2(const FineGeom& g, const double* kt, const double* phi, const int* nkeep, int L,
                      double* D, double* Aoff, hipStream_t s);
void launch_galerkin_up(const CoarseGeom& lo, const CoarseGeom& up, const double* Dlo,
                        const double* Aofflo, const double* V, const int* nkeep_up, double* Dup,
                        double* Aoffup, hipStream_t s);
void launch_assemble_diag(const CoarseGeom& g, const double* Aint, const double* D, double* Ad,
                          hipStream_t s);
void launch_blockic_setup(const CoarseGeom& g, const double* Ad, const double* Aoff, const int* nkeep,
                          double* Dinv, double* G, int* bad, hipStream_t s);
void launch_build_coarsest(const CoarseGeom& g, const double* Ad, const double* Aoff,
                           const int* cmap_inv, int np, double* dense, hipStream_t s);
template <typename S, typename T>
void launch_convert(const S* src, T* dst, int64_t n, hipStream_t s, const Scalars* sc = nullptr);

// local eigensolves (k_eig.hip)
void launch_eig2(const FineGeom& g, const double* kt, int target, int nvec, double tol, double crtol,
                 double* phi, double* lam, int* nkeep, double* Aint, int* status, double* zc, int e0, int count,
                 const float* warm, int kp, int kw, double ws_tol, int* ws_fb, double thr, hipStream_t s);

// learned warm start (k_cnn.hip)
int64_t cnn_param_count(int k);
size_t cnn_pack_words(int kp);
void launch_cnn_patches(const FineGeom& g, const double* perm, int e0, int count, double s_scale, float* out,
                        double* s_out, hipStream_t s);
void launch_cnn_pack(const float* t32, const uint16_t* t16, int k, int kp, void* packs, hipStream_t s);
void launch_cnn_forward(const void* packs, int kp, const float* patches, int count, float* a1, float* a2, float* X,
                        hipStream_t s);
void launch_cnn_loss(const float* X, const double* phi, int ldphi, const double* sdiag, int k, int kp, int count,
                     double inv_m, double* loss_part, float* gX, hipStream_t s);
void launch_cnn_backward(const void* packs, int k, int kp, const float* patches, const float* a1, const float* a2,
                         const float* gX, int count, float* g2, float* g1, float* part, int nblk, float* grad,
                         hipStream_t s);
void launch_cnn_adam(float* theta, const float* grad, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                     float eps, float c1, float c2, uint16_t* theta16, hipStream_t s);
void launch_eig_up(const CoarseGeom& lo, const CoarseGeom& up, const double* Aint_lo, const double* Dlo,
                   const double* Aofflo, const int* nkeep_lo, const double* zlo, double* Hd_work,
                   int target, int nvec, double tol, double crtol, double thr, double* V, double* lam, int* nkeep,
                   double* Aint, double* zup, int* status, hipStream_t s);

// dense coarsest factorization (k_dense.hip); np is a multiple of 32
int dense_spd_inverse(double* a, int np, double* work, double* tbuf, int* bad, hipStream_t s);
size_t dense_spd_inverse_tbuf_doubles(int np);
void launch_add_rank1(double* a, int np, int n, const double* z, double alpha, hipStream_t s);
void launch_pad_identity(double* a, int np, int n, hipStream_t s);

}  // namespace specmg
