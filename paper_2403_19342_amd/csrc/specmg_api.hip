// C-ABI of the specmg library: context, set-up orchestration, the V-cycle
// recursion and the preconditioned CG driver.  Every numerical step runs in
// the kernels of k_fine / k_coarse / k_eig / k_dense; this file only sizes
// buffers, sequences launches and moves a few scalars.
#include <chrono>
#include <memory>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "../../include/specmg.h"

using namespace specmg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

}  // namespace

namespace specmg {
int fail_message(int code, const char* msg) { return fail(code, msg); }
}  // namespace specmg

namespace {

#define HIPCHK(x)                                                  \
    do {                                                           \
        hipError_t _e = (x);                                       \
        if (_e != hipSuccess) throw HipError{_e, #x};              \
    } while (0)

struct Level {
    int l = 0;             // level index (2 = first coarse level)
    CoarseGeom g{};        // element grid; parents filled unless coarsest
    int L = 0;             // padded width
    int rows = 0;          // basis rows per element: 512 (level 2) or agg^3 L_prev
    std::vector<int> nkeep_h;
    int dim = 0;
    int* nkeep = nullptr;
    int* status = nullptr;
    double* lam = nullptr;
    double* basis = nullptr;   // level 2: phi; level >= 3: V
    double* Aint = nullptr;
    double* D = nullptr;
    double* Aoff = nullptr;
    double* Ad = nullptr;
    double* Dinv = nullptr;
    double* G = nullptr;       // D_c^{-1} A(c, neighbour) for the smoother
    double* z = nullptr;
    float* basis32 = nullptr;  // level 2, the mixed modes: float32 copy of the basis
    double *r = nullptr, *u = nullptr, *e = nullptr;
    float *r32 = nullptr, *e32 = nullptr;  // level 2, FP32 V-cycle: the level's vectors as the fine kernels see them
};

}  // namespace

// device buffer released at scope exit (transient set-up workspaces), from
// the context's allocator
struct DevBuf {
    const DevAlloc& al;
    void* p = nullptr;
    DevBuf(const DevAlloc& a, size_t bytes) : al(a) { p = al.get(bytes); }
    ~DevBuf() { al.put(p); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
};

constexpr int kCnnSetupBatch = 8192;   // level-2 elements per network batch in set-up

struct specmg_ctx {
    specmg_grid grid{};
    specmg_opts opts{};
    int levels = 0, target = 0, L = 0, nvec = 0;          // level 2 (L: padded width)
    int target_cc = 0, Lcc = 0, nvec_cc = 0;               // levels >= 3
    double thr_cc = 0.0;                                   // threshold rule at levels >= 3 when > 0
    double thr_c = 0.0;                                    // threshold rule at level 2 when > 0
    int ncomp = 1;        // permeability components: 1 (kappa I) or 3 (diag(kappa_x, kappa_y, kappa_z))
    int fp32 = 0;
    int fp32_basis = 0;   // float64 fine level with a float32 copy of the level-2 basis
    int fp32_store = 0;   // fine level stored in float32 (kappa~, 1/d, basis, u, t), float64 arithmetic
    int flexible = 0;     // the V-cycle is not a fixed linear map: flexible (Polak-Ribiere) CG
    int nu = 1, nu_c = 1; // block-Jacobi sweeps before and after the correction: fine, coarse levels
    int64_t n = 0;
    FineGeom fg{};
    std::vector<void*> allocs;
    double* kt = nullptr;
    float* kt32 = nullptr;
    double* invd = nullptr;
    float* invd32 = nullptr;
    std::vector<Level> lev;    // lev[0] = level 2
    int nL = 0, npL = 0;
    double* Pinv = nullptr;     // dense inverse (coarsest spaces of one LDS chunk)
    double* Psym = nullptr;     // packed lower tiles of the inverse (wider spaces)
    int2* sym_chunks = nullptr;
    int sym_nchunks = 0, sym_maxc = 0;
    double *sym_P = nullptr, *sym_Q = nullptr;   // column and row partial sums of the tiles
    int* cmap = nullptr;
    double* rc = nullptr;       // coarsest right-hand side, compact
    // CG state (element order, see eidx)
    double *r = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr, *u1 = nullptr;
    // the caller's source and solution in element order (and the scratch of
    // apply_precond / apply_operator)
    double *b_e = nullptr, *x_e = nullptr;
    float* u1_32 = nullptr;
    double* dtmp = nullptr;     // scratch scalars
    int* dflag = nullptr;       // error flags
    Scalars* sc = nullptr;
    Scalars* sc_host = nullptr; // pinned
    int* ws_fb = nullptr;       // per level-2 element: 1 if the predicted start fell back
    // flexible GMRES workspace (allocated on first use, grown with the restart length)
    double* gm_buf = nullptr;
    int gm_restart = 0;
    GmresState* gm_state = nullptr;
    RedBuf rb{};
    specmg_solve_info setup_info{};
    // per-kernel-class event timing of pcg_solve (see specmg_set_profiling)
    int prof_on = 0;
    int cur_iter = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Rec { int cls, iter; size_t e0, e1; };
    std::vector<Rec> recs;
    double prof_ms[8] = {0};
    int prof_count[8] = {0};
    double coarse_bytes = 0.0;     // algorithmic bytes of one V-cycle's coarse part (levels >= 2)
    double coarsest_bytes = 0.0;   // of the coarsest product alone

    DevAlloc al;   // device memory of the context (caller's allocator or hipMalloc)

    template <typename T>
    T* alloc(size_t count) {
        void* ptr = al.get((count ? count : 1) * sizeof(T));
        allocs.push_back(ptr);
        return (T*)ptr;
    }
    ~specmg_ctx() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        if (!allocs.empty() || gm_buf || gm_state) (void)hipDeviceSynchronize();
        for (void* a : allocs) al.put(a);
        al.put(gm_buf);
        al.put(gm_state);
        if (sc_host) (void)hipHostFree(sc_host);
    }
};

namespace {

template <typename T>
struct VArgs;

// pointers of one precision variant of the V-cycle
struct VPtrs {
    const void* kt;
    const void* invd;
    void* u1;
};

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Kernel timing (no-op unless profiling is on).  prof_begin hands an event
// pair to the next timed launch (the fine-level kernels stamp their own
// dispatch); prof_begin_range / prof_end record plain events around a group
// of launches (the coarse levels).
enum ProfClass { PC_SPMV = 0, PC_PRE = 1, PC_RESTRICT = 2, PC_PROLONG = 3, PC_POST = 4, PC_COARSE = 5,
                 PC_COARSEST = 6, PC_PUPDATE = 7 };

static size_t prof_events(specmg_ctx* c) {
    if (c->ev_used + 2 > c->ev_pool.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            c->ev_pool.push_back(e);
        }
    }
    const size_t i = c->ev_used;
    c->ev_used += 2;
    return i;
}

size_t prof_begin(specmg_ctx* c, hipStream_t) {
    if (!c->prof_on) return (size_t)-1;
    const size_t i = prof_events(c);
    g_kev.start = c->ev_pool[i];
    g_kev.stop = c->ev_pool[i + 1];
    return i;
}

size_t prof_begin_range(specmg_ctx* c, hipStream_t s) {
    if (!c->prof_on) return (size_t)-1;
    const size_t i = prof_events(c);
    HIPCHK(hipEventRecord(c->ev_pool[i], s));
    return i | ((size_t)1 << 62);
}

void prof_end(specmg_ctx* c, size_t i, int cls, hipStream_t s) {
    if (i == (size_t)-1) return;
    if (i & ((size_t)1 << 62)) {
        i &= ~((size_t)1 << 62);
        HIPCHK(hipEventRecord(c->ev_pool[i + 1], s));
    } else if (g_kev.start) {
        g_kev = KernelEvents{};   // no timed launch consumed the pair
        return;
    }
    c->recs.push_back({cls, c->cur_iter, i, i + 1});
}

template <typename T>
T* pick(double* d, float* f);
template <>
double* pick<double>(double* d, float*) { return d; }
template <>
float* pick<float>(double*, float* f) { return f; }

// coarse levels from level index li (lev[li] holds r, receives e), float64
// in every precision mode: the kept coarse modes of high-contrast media have
// eigenvalues near float32 rounding of the operator's scale (inclusion and
// channel modes, about 1e-7), so float32 arithmetic at these levels, and even
// float32 copies of their blocks with float64 arithmetic, lose them
void coarse_cycle(specmg_ctx* c, size_t li, int check, hipStream_t s) {
    Level& lv = c->lev[li];
    double* r = lv.r;
    double* e = lv.e;
    if (li + 1 == c->lev.size()) {
        const size_t ev = prof_begin(c, s);
        if (c->Psym)
            launch_coarsest_sym(c->nL, c->npL, c->Psym, c->sym_chunks, c->sym_nchunks, c->sym_maxc, c->cmap, r, e,
                                c->rc, c->sym_P, c->sym_Q, c->sc, check, s);
        else
            launch_coarsest<double>(c->nL, c->npL, c->Pinv, c->cmap, r, e, c->rc, c->sc, check, s);
        prof_end(c, ev, PC_COARSEST, s);
        return;
    }
    Level& up = c->lev[li + 1];
    double* u = lv.u;
    // a repeated sweep u += M^-1 (r - A u) reads neighbouring blocks' u, so
    // it writes e (free until the last sweep) and copies back
    const int64_t nrow = (int64_t)lv.g.m * lv.g.L;
    launch_coarse_smooth<double>(lv.g, lv.Dinv, lv.G, r, u, c->sc, check, s);
    const Scalars* gate = check ? c->sc : nullptr;
    for (int it = 1; it < c->nu_c; ++it) {
        launch_coarse_resid_smooth<double>(lv.g, lv.Ad, lv.Dinv, lv.Aoff, lv.G, r, u, e, c->sc, check, s);
        launch_copy(u, e, nrow, s, gate);
    }
    launch_coarse_resid_restrict<double>(lv.g, lv.Ad, lv.Aoff, r, u, up.basis, up.nkeep, up.L, up.r, c->sc, check,
                                         s);
    coarse_cycle(c, li + 1, check, s);
    launch_coarse_prolong<double>(lv.g, u, up.basis, up.nkeep, up.L, up.e, c->sc, check, s);
    for (int it = 1; it < c->nu_c; ++it) {
        launch_coarse_resid_smooth<double>(lv.g, lv.Ad, lv.Dinv, lv.Aoff, lv.G, r, u, e, c->sc, check, s);
        launch_copy(u, e, nrow, s, gate);
    }
    launch_coarse_resid_smooth<double>(lv.g, lv.Ad, lv.Dinv, lv.Aoff, lv.G, r, u, e, c->sc, check, s);
}

// One repeated fine sweep u1 += M^-1 (r - A u1): the residual, the sweep
// written to z (the V-cycle's output, free until the last sweep), and z
// copied back into u1 (converted when u1 is stored in float32).
template <typename T, typename C>
void extra_fine_sweep(specmg_ctx* c, double* r, double* z, int check, hipStream_t s) {
    const T* kt = pick<T>(c->kt, c->kt32);
    const T* invd = pick<T>(c->invd, c->invd32);
    T* u1 = pick<T>(c->u1, c->u1_32);
    launch_post_fused<T, C>(c->fg, kt, invd, u1, r, nullptr, z, c->sc, c->rb, check ? 2 : 0, s);
    const Scalars* gate = check ? c->sc : nullptr;
    if constexpr (std::is_same<T, float>::value) launch_convert<double, float>(z, u1, c->n, s, gate);
    else launch_copy(u1, z, c->n, s, gate);
}

// z = P^{-1} r (fine level + recursion).  T: stored word of the fine
// level's coefficients and vectors, C: its arithmetic (see launch_pre_smooth).
// pre_mode / post_mode are the mode bits of the fine smoother kernels; check:
// return early when solve is done.
template <typename T, typename C, typename TB>
void vcycle_fine(specmg_ctx* c, double* r, double* z, const double* q, int pre_mode, int post_mode, int check,
                 hipStream_t s) {
    const T* kt = pick<T>(c->kt, c->kt32);
    const T* invd = pick<T>(c->invd, c->invd32);
    T* u1 = pick<T>(c->u1, c->u1_32);
    Level& l2 = c->lev[0];
    const TB* phi = pick<TB>(l2.basis, l2.basis32);
    C* r2 = pick<C>(l2.r, l2.r32);
    C* e2 = pick<C>(l2.e, l2.e32);
    size_t ev = prof_begin(c, s);
    launch_pre_smooth<T, C>(c->fg, kt, invd, r, q, u1, c->sc, c->rb, pre_mode, s);
    prof_end(c, ev, PC_PRE, s);
    for (int it = 1; it < c->nu; ++it) extra_fine_sweep<T, C>(c, r, z, check, s);
    ev = prof_begin(c, s);
    launch_resid_restrict<T, TB, C>(c->fg, kt, u1, r, phi, l2.nkeep, l2.L, r2, c->sc, check, s);
    prof_end(c, ev, PC_RESTRICT, s);
    ev = prof_begin_range(c, s);
    if constexpr (std::is_same<C, float>::value) {
        // the coarse levels run in float64 (see coarse_cycle)
        const int64_t n2 = (int64_t)l2.g.m * l2.L;
        const Scalars* gate = check ? c->sc : nullptr;
        launch_convert<float, double>(l2.r32, l2.r, n2, s, gate);
        coarse_cycle(c, 0, check, s);
        launch_convert<double, float>(l2.e, l2.e32, n2, s, gate);
    } else {
        coarse_cycle(c, 0, check, s);
    }
    prof_end(c, ev, PC_COARSE, s);
    ev = prof_begin(c, s);
    launch_prolong<T, TB, C>(c->fg, u1, phi, l2.nkeep, l2.L, e2, c->sc, check, s);
    prof_end(c, ev, PC_PROLONG, s);
    for (int it = 1; it < c->nu; ++it) extra_fine_sweep<T, C>(c, r, z, check, s);
    ev = prof_begin(c, s);
    launch_post_fused<T, C>(c->fg, kt, invd, u1, r, q, z, c->sc, c->rb, post_mode, s);
    prof_end(c, ev, PC_POST, s);
}

void run_vcycle(specmg_ctx* c, double* r, double* z, const double* q, int pre_mode, int post_mode, int check,
                hipStream_t s) {
    if (c->fp32) vcycle_fine<float, float, float>(c, r, z, q, pre_mode, post_mode, check, s);
    else if (c->fp32_store) vcycle_fine<float, double, float>(c, r, z, q, pre_mode, post_mode, check, s);
    else if (c->fp32_basis) vcycle_fine<double, double, float>(c, r, z, q, pre_mode, post_mode, check, s);
    else vcycle_fine<double, double, double>(c, r, z, q, pre_mode, post_mode, check, s);
}

int nvec_for(int target) {
    // block size: eigenvalues through index target+3 are needed by the
    // cluster rule, plus two guard vectors; even sizes 10 ... 16 are built,
    // and 20 and 26 for the wide coarse-coarse counts (targets 11 ... 20)
    int m = target + 6;
    if (m % 2) ++m;
    if (m < 10) m = 10;
    if (m > 16) m = m <= 20 ? 20 : 26;
    return m;
}

}  // namespace

// ---------------------------------------------------------------------------

// Algorithmic bytes of the coarse part of one V-cycle (kept widths, float64
// words): per non-coarsest level with kept counts k_e, diag = sum k_e^2,
// cpl = sum over neighbour pairs k_e k_f, dim = sum k_e, and the parents'
// bases Vsz = sum_E K_E sum_{c in E} k_c (dimup = sum K_E):
//   sweep (D^-1, the six couplings D^-1 A(c, n), r in; u out)   diag + 2 cpl + 2 dim
//   residual + restriction (A_l blocks, r, u, V in; r_up out)    diag + cpl + 2 dim + Vsz + dimup
//   prolongation (u in and out, V, e_up)                         2 dim + Vsz + dimup
//   residual + sweep (A_l, D^-1, couplings, r, u in; e out)      2 diag + 3 cpl + 3 dim
// and each further sweep pair (nu_c = 2) twice the last line plus a copy.
// The coarsest product reads the n_L x n_L inverse and three n_L vectors.
static void coarse_traffic(specmg_ctx* c) {
    double words = 0.0;
    for (size_t li = 0; li + 1 < c->lev.size(); ++li) {
        const Level& lv = c->lev[li];
        const Level& up = c->lev[li + 1];
        const CoarseGeom& g = lv.g;
        const int agg = g.agg;
        double diag = 0.0, cpl = 0.0, dim = 0.0, vsz = 0.0, dimup = 0.0;
        for (int e = 0; e < g.m; ++e) {
            const double k = lv.nkeep_h[e];
            const int ex = e % g.mx, ey = (e / g.mx) % g.my, ez = e / (g.mx * g.my);
            diag += k * k;
            dim += k;
            if (ex + 1 < g.mx) cpl += k * lv.nkeep_h[e + 1];
            if (ey + 1 < g.my) cpl += k * lv.nkeep_h[e + g.mx];
            if (ez + 1 < g.mz) cpl += k * lv.nkeep_h[e + g.mx * g.my];
        }
        for (int E = 0; E < up.g.m; ++E) {
            const int Ex = E % up.g.mx, Ey = (E / up.g.mx) % up.g.my, Ez = E / (up.g.mx * up.g.my);
            double rows = 0.0;
            for (int q = 0; q < agg * agg * agg; ++q) {
                const int cx = Ex * agg + q % agg, cy = Ey * agg + (q / agg) % agg, cz = Ez * agg + q / (agg * agg);
                rows += lv.nkeep_h[cx + g.mx * (cy + g.my * cz)];
            }
            vsz += up.nkeep_h[E] * rows;
            dimup += up.nkeep_h[E];
        }
        words += 4 * diag + 7 * cpl + 9 * dim + 2 * vsz + 2 * dimup;
        words += (c->nu_c - 1) * 2.0 * (2 * diag + 3 * cpl + 5 * dim);
    }
    double nl = 0.0;
    for (int k : c->lev.back().nkeep_h) nl += k;
    // the whole inverse, or its lower triangle beyond one LDS chunk
    c->coarsest_bytes = 8.0 * ((nl > kCoarsestChunk ? 0.5 * nl * (nl + 1.0) : nl * nl) + 3.0 * nl);
    c->coarse_bytes = 8.0 * words + c->coarsest_bytes;
    if (c->fp32) c->coarse_bytes += 2.0 * 12.0 * c->lev[0].dim;   // level-2 vectors widened and narrowed
}

extern "C" const char* specmg_last_error(void) { return g_last_error.c_str(); }

extern "C" void specmg_destroy(specmg_ctx* ctx) { delete ctx; }

static int do_setup(specmg_ctx* c, const double* perm, hipStream_t s) {
    const double t0 = now_ms();
    const specmg_grid& G = c->grid;
    const int levels = c->levels;
    c->n = (int64_t)G.nx * G.ny * G.nz;
    FineGeom& fg = c->fg;
    fg.nx = G.nx;
    fg.ny = G.ny;
    fg.nz = G.nz;
    fg.mx = G.nx / 8;
    fg.my = G.ny / 8;
    fg.mz = G.nz / 8;
    fg.ex = (fg.mx % 4 == 0) ? 4 : ((fg.mx % 2 == 0) ? 2 : 1);
    if (fg.ex == 4) fg.ex = 2;   // 2 elements per tile: 16x8x8 cells, 128-byte rows
    fg.ntx = fg.mx / fg.ex;
    fg.nty = fg.my;
    fg.ntz = fg.mz;
    fg.ntiles = fg.ntx * fg.nty * fg.ntz;
    fg.xcd_remap = (fg.ntiles % 8 == 0) ? 1 : 0;
    fg.ortho = c->ncomp == 3 ? 1 : 0;
    // isotropic: kappa~ = kappa / hx^2 and the y, z faces scaled by
    // (hx/hy)^2, (hx/hz)^2; orthotropic: kappa~_d = kappa_d / h_d^2 per axis
    fg.cy = fg.ortho ? 1.0 : (G.hx / G.hy) * (G.hx / G.hy);
    fg.cz = fg.ortho ? 1.0 : (G.hx / G.hz) * (G.hx / G.hz);
    if (fg.ntiles > kMaxRedBlocks) return fail(SPECMG_EINVAL, "grid too large for the reduction buffer");

    c->dflag = c->alloc<int>(8);
    HIPCHK(hipMemsetAsync(c->dflag, 0, 8 * sizeof(int), s));
    c->kt = c->alloc<double>((size_t)c->ncomp * c->n);
    c->invd = c->alloc<double>(c->n);
    if (c->fp32 || c->fp32_store) {
        c->kt32 = c->alloc<float>(c->n);
        c->invd32 = c->alloc<float>(c->n);
    }
    const double h = G.hx;
    if (fg.ortho)
        launch_perm3_to_kt(fg, perm, c->kt, 1.0 / (G.hx * G.hx), 1.0 / (G.hy * G.hy), 1.0 / (G.hz * G.hz),
                           c->dflag, s);
    else
        launch_perm_to_kt(fg, perm, c->kt, c->kt32, 1.0 / (h * h), c->dflag, s);
    int flags[8];
    HIPCHK(hipMemcpyAsync(flags, c->dflag, sizeof(flags), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flags[0]) return fail(SPECMG_EINVAL_PERM, "permeability must be positive and finite");
    launch_ic_setup(fg, c->kt, c->invd, c->invd32, c->dflag + 1, s);

    const int L = c->L;
    const double tol = c->opts.eig_tol > 0 ? c->opts.eig_tol : 1e-12;
    const double crtol = c->opts.cluster_rtol > 0 ? c->opts.cluster_rtol : 1e-6;
    c->lev.resize(levels - 1);
    // ---- level 2
    {
        Level& lv = c->lev[0];
        lv.l = 2;
        lv.L = L;
        lv.rows = 512;
        lv.g.mx = fg.mx;
        lv.g.my = fg.my;
        lv.g.mz = fg.mz;
        lv.g.m = fg.mx * fg.my * fg.mz;
        lv.g.L = L;
        const int m = lv.g.m;
        lv.nkeep = c->alloc<int>(m);
        lv.g.nkeep = lv.nkeep;
        lv.status = c->alloc<int>(m);
        lv.lam = c->alloc<double>((size_t)m * L);
        lv.basis = c->alloc<double>((size_t)m * L * 512);
        lv.Aint = c->alloc<double>((size_t)m * L * L);
        lv.D = c->alloc<double>((size_t)m * 6 * L * L);
        lv.Aoff = c->alloc<double>((size_t)m * 3 * L * L);
        lv.Ad = c->alloc<double>((size_t)m * L * L);
        lv.z = c->alloc<double>((size_t)m * L);
        if (c->opts.warm_start == SPECMG_WS_CNN) {
            // predicted start blocks, batch by batch, each batch's network
            // output consumed by the eigensolves of the same batch
            const int k = c->target, kp = k + (k & 1);
            const int batch = m < kCnnSetupBatch ? m : kCnnSetupBatch;
            DevBuf packs(c->al, cnn_pack_words(kp) * sizeof(uint32_t)),
                patches(c->al, (size_t)batch * 1000 * sizeof(float)),
                a1(c->al, (size_t)batch * 32 * 512 * sizeof(float)), a2(c->al, (size_t)batch * 32 * 512 * sizeof(float)),
                xw(c->al, (size_t)batch * kp * 512 * sizeof(float));
            c->ws_fb = c->alloc<int>(m);
            const double wtol = c->opts.ws_resid_tol > 0 ? c->opts.ws_resid_tol : 1e-3;
            launch_cnn_pack(nullptr, (const uint16_t*)c->opts.cnn_weights, k, kp, packs.p, s);
            for (int e0 = 0; e0 < m; e0 += batch) {
                const int cnt = m - e0 < batch ? m - e0 : batch;
                launch_cnn_patches(fg, perm, e0, cnt, 0.0, (float*)patches.p, nullptr, s);
                launch_cnn_forward(packs.p, kp, (const float*)patches.p, cnt, (float*)a1.p, (float*)a2.p,
                                   (float*)xw.p, s);
                launch_eig2(fg, c->kt, c->target, c->nvec, tol, crtol, lv.basis, lv.lam, lv.nkeep, lv.Aint,
                            lv.status, lv.z, e0, cnt, (const float*)xw.p, kp, k, wtol, c->ws_fb, c->thr_c, s);
            }
            HIPCHK(hipStreamSynchronize(s));
        } else {
            launch_eig2(fg, c->kt, c->target, c->nvec, tol, crtol, lv.basis, lv.lam, lv.nkeep, lv.Aint, lv.status,
                        lv.z, 0, m, nullptr, 0, 0, 0.0, nullptr, c->thr_c, s);
        }
        launch_galerkin2(fg, c->kt, lv.basis, lv.nkeep, L, lv.D, lv.Aoff, s);
        launch_assemble_diag(lv.g, lv.Aint, lv.D, lv.Ad, s);
    }
    // ---- levels 3..levels
    for (int li = 1; li < levels - 1; ++li) {
        Level& lo = c->lev[li - 1];
        Level& up = c->lev[li];
        const int agg = G.agg;
        up.l = li + 2;
        const int Lu = c->Lcc;
        up.L = Lu;
        up.g.mx = lo.g.mx / agg;
        up.g.my = lo.g.my / agg;
        up.g.mz = lo.g.mz / agg;
        up.g.m = up.g.mx * up.g.my * up.g.mz;
        up.g.L = Lu;
        up.rows = agg * agg * agg * lo.L;
        lo.g.agg = agg;
        lo.g.px = up.g.mx;
        lo.g.py = up.g.my;
        lo.g.pz = up.g.mz;
        lo.g.M = up.g.m;
        const int m = up.g.m;
        up.nkeep = c->alloc<int>(m);
        up.g.nkeep = up.nkeep;
        up.status = c->alloc<int>(m);
        up.lam = c->alloc<double>((size_t)m * Lu);
        up.basis = c->alloc<double>((size_t)m * Lu * up.rows);
        up.Aint = c->alloc<double>((size_t)m * Lu * Lu);
        up.D = c->alloc<double>((size_t)m * 6 * Lu * Lu);
        up.Aoff = c->alloc<double>((size_t)m * 3 * Lu * Lu);
        up.Ad = c->alloc<double>((size_t)m * Lu * Lu);
        up.z = c->alloc<double>((size_t)m * Lu);
        double* hd = c->alloc<double>((size_t)lo.g.m * lo.L * lo.L);
        launch_eig_up(lo.g, up.g, lo.Aint, lo.D, lo.Aoff, lo.nkeep, lo.z, hd, c->target_cc, c->nvec_cc, tol, crtol,
                      c->thr_cc, up.basis, up.lam, up.nkeep, up.Aint, up.z, up.status, s);
        launch_galerkin_up(lo.g, up.g, lo.D, lo.Aoff, up.basis, up.nkeep, up.D, up.Aoff, s);
        launch_assemble_diag(up.g, up.Aint, up.D, up.Ad, s);
    }
    // ---- smoothers of the non-coarsest coarse levels
    for (int li = 0; li < levels - 2; ++li) {
        Level& lv = c->lev[li];
        lv.Dinv = c->alloc<double>((size_t)lv.g.m * lv.L * lv.L);
        lv.G = c->alloc<double>((size_t)lv.g.m * 6 * lv.L * lv.L);
        launch_blockic_setup(lv.g, lv.Ad, lv.Aoff, lv.nkeep, lv.Dinv, lv.G, c->dflag + 2, s);
    }
    // ---- host copies of the kept counts, unconverged eigensolves
    int unconv = 0;
    for (auto& lv : c->lev) {
        lv.nkeep_h.resize(lv.g.m);
        std::vector<int> st(lv.g.m);
        HIPCHK(hipMemcpyAsync(lv.nkeep_h.data(), lv.nkeep, lv.g.m * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(st.data(), lv.status, lv.g.m * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        lv.dim = 0;
        for (int k : lv.nkeep_h) lv.dim += k;
        for (int v : st) unconv += (v < 0);
    }
    coarse_traffic(c);
    // ---- coarsest: A_L^+ = (A_L + alpha z z^T)^{-1} - z z^T / alpha
    {
        Level& top = c->lev.back();
        const int m = top.g.m;
        const int L = top.L;
        std::vector<int> cmap, cinv((size_t)m * L, -1);
        for (int e = 0; e < m; ++e)
            for (int a = 0; a < top.nkeep_h[e]; ++a) {
                cinv[(size_t)e * L + a] = (int)cmap.size();
                cmap.push_back(e * L + a);
            }
        const int nL = (int)cmap.size();
        // spaces wider than one LDS chunk keep only the lower tiles of the
        // symmetric inverse (the dense matrix is then a set-up workspace)
        const bool sym = nL > kCoarsestChunk;
        const int pad = sym ? coarsest_sym_tile() : 32;
        const int np = ((nL + pad - 1) / pad) * pad;
        c->nL = nL;
        c->npL = np;
        c->cmap = c->alloc<int>(nL);
        c->rc = c->alloc<double>(np);
        HIPCHK(hipMemsetAsync(c->rc, 0, (size_t)np * sizeof(double), s));
        int* dcinv = c->alloc<int>(cinv.size());
        HIPCHK(hipMemcpyAsync(c->cmap, cmap.data(), nL * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(dcinv, cinv.data(), cinv.size() * sizeof(int), hipMemcpyHostToDevice, s));
        std::unique_ptr<DevBuf> dense_ws;
        if (sym) {
            dense_ws.reset(new DevBuf(c->al, (size_t)np * np * sizeof(double)));
            c->Pinv = (double*)dense_ws->p;
        } else {
            c->Pinv = c->alloc<double>((size_t)np * np);
        }
        DevBuf work_buf(c->al, (size_t)np * np * sizeof(double));
        DevBuf tbuf(c->al, dense_spd_inverse_tbuf_doubles(np) * sizeof(double));
        double* work = (double*)work_buf.p;
        HIPCHK(hipMemsetAsync(c->Pinv, 0, (size_t)np * np * sizeof(double), s));
        launch_build_coarsest(top.g, top.Ad, top.Aoff, dcinv, np, c->Pinv, s);
        launch_pad_identity(c->Pinv, np, nL, s);
        // z (constant function) and alpha = trace / n on the host
        std::vector<double> zp((size_t)m * L), ad((size_t)m * L * L);
        HIPCHK(hipMemcpyAsync(zp.data(), top.z, zp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(ad.data(), top.Ad, ad.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<double> zc(nL);
        double zn = 0.0, tr = 0.0;
        for (int i = 0; i < nL; ++i) {
            zc[i] = zp[cmap[i]];
            zn += zc[i] * zc[i];
            const int e = cmap[i] / L, a = cmap[i] % L;
            tr += ad[((size_t)e * L + a) * L + a];
        }
        zn = std::sqrt(zn);
        if (!(zn > 0.0)) return fail(SPECMG_EFACT, "constant function not found in the coarsest space");
        for (double& v : zc) v /= zn;
        const double alpha = tr / nL;
        double* dz = c->alloc<double>(nL);
        HIPCHK(hipMemcpyAsync(dz, zc.data(), nL * sizeof(double), hipMemcpyHostToDevice, s));
        // B = (A_L + alpha z z^T)^-1 is applied as the coarsest solve.  It
        // differs from A_L^+ = B - z z^T / alpha only along z, which every
        // level prolongs to the constant function (the kernel of A), so the
        // mean-projected CG iterates are the same; unlike the difference, B
        // stays positive definite when rounding spoils the inverse of an
        // ill-conditioned A_L.
        launch_add_rank1(c->Pinv, np, nL, dz, alpha, s);
        const int de = dense_spd_inverse(c->Pinv, np, work, (double*)tbuf.p, c->dflag + 3, s);
        HIPCHK(hipStreamSynchronize(s));
        if (de != 0) return fail(SPECMG_EDEVICE, std::string("coarsest inverse: ") + hipGetErrorString((hipError_t)de));
        if (sym) {
            const int nT = np / coarsest_sym_tile();
            c->Psym = c->alloc<double>(coarsest_sym_packed_doubles(np));
            launch_pack_lower_tiles(c->Pinv, np, c->Psym, s);
            const std::vector<int2> ch = coarsest_sym_chunks(np, &c->sym_maxc);
            c->sym_nchunks = (int)ch.size();
            c->sym_chunks = c->alloc<int2>(ch.size());
            HIPCHK(hipMemcpyAsync(c->sym_chunks, ch.data(), ch.size() * sizeof(int2), hipMemcpyHostToDevice, s));
            c->sym_P = c->alloc<double>((size_t)nT * nT * coarsest_sym_tile());
            c->sym_Q = c->alloc<double>((size_t)nT * c->sym_maxc * coarsest_sym_tile());
            HIPCHK(hipStreamSynchronize(s));
            c->Pinv = nullptr;   // the dense workspace is released at scope exit
        }
    }
    // ---- float32 copy of the level-2 basis for the mixed-precision fine level
    if (c->fp32 || c->fp32_basis || c->fp32_store) {
        Level& lv = c->lev[0];
        const size_t nb = (size_t)lv.g.m * lv.L * lv.rows;
        lv.basis32 = c->alloc<float>(nb);
        launch_convert<double, float>(lv.basis, lv.basis32, (int64_t)nb, s);
    }
    // ---- vectors
    for (auto& lv : c->lev) {
        const size_t nv = (size_t)lv.g.m * lv.L;
        lv.r = c->alloc<double>(nv);
        lv.u = c->alloc<double>(nv);
        lv.e = c->alloc<double>(nv);
        HIPCHK(hipMemsetAsync(lv.r, 0, nv * sizeof(double), s));
        HIPCHK(hipMemsetAsync(lv.u, 0, nv * sizeof(double), s));
        HIPCHK(hipMemsetAsync(lv.e, 0, nv * sizeof(double), s));
        if (c->fp32 && &lv == &c->lev[0]) {
            lv.r32 = c->alloc<float>(nv);
            lv.e32 = c->alloc<float>(nv);
            HIPCHK(hipMemsetAsync(lv.r32, 0, nv * sizeof(float), s));
            HIPCHK(hipMemsetAsync(lv.e32, 0, nv * sizeof(float), s));
        }
    }
    c->r = c->alloc<double>(c->n);
    c->z = c->alloc<double>(c->n);
    c->p[0] = c->alloc<double>(c->n);
    c->p[1] = c->alloc<double>(c->n);
    c->q = c->alloc<double>(c->n);
    c->u1 = c->alloc<double>(c->n);
    if (c->fp32 || c->fp32_store) c->u1_32 = c->alloc<float>(c->n);
    c->b_e = c->alloc<double>(c->n);
    c->x_e = c->alloc<double>(c->n);
    c->dtmp = c->alloc<double>(8);
    c->sc = c->alloc<Scalars>(1);
    HIPCHK(hipHostMalloc((void**)&c->sc_host, sizeof(Scalars), hipHostMallocDefault));
    c->rb.partial = c->alloc<double>((size_t)2 * kMaxRedBlocks);
    c->rb.partial2 = c->alloc<double>((size_t)2 * kFinBlocks);
    c->rb.ticket = c->alloc<unsigned>(1);
    HIPCHK(hipMemsetAsync(c->rb.ticket, 0, sizeof(unsigned), s));
    launch_pcg_init(c->sc, 0.0, 0, s);
    HIPCHK(hipMemcpyAsync(flags, c->dflag, sizeof(flags), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());

    specmg_solve_info& si = c->setup_info;
    memset(&si, 0, sizeof(si));
    si.n_levels = levels;
    si.dims[0] = (int)c->n;
    for (size_t li = 0; li < c->lev.size() && li + 1 < 8; ++li) si.dims[li + 1] = c->lev[li].dim;
    si.eig_unconverged = unconv;
    if (c->ws_fb) {
        std::vector<int> fb(c->lev[0].g.m);
        HIPCHK(hipMemcpy(fb.data(), c->ws_fb, fb.size() * sizeof(int), hipMemcpyDeviceToHost));
        for (int v : fb) si.ws_fallbacks += v;
    }
    si.setup_ms = now_ms() - t0;
    if (flags[1]) return fail(SPECMG_EFACT, "fine IC(0) pivot not positive");
    if (flags[2]) return fail(SPECMG_EFACT, "coarse block IC(0) pivot not positive definite");
    if (flags[3]) return fail(SPECMG_EFACT, "coarsest factor not positive definite");
    if (unconv) return fail(SPECMG_EEIG, std::to_string(unconv) + " local eigensolves did not converge");
    return SPECMG_OK;
}

extern "C" int specmg_setup(const double* perm_dev, int32_t perm_components, const specmg_grid* grid,
                            const specmg_opts* opts, void* stream, specmg_ctx** out) {
    return specmg_setup_alloc(perm_dev, perm_components, grid, opts, nullptr, stream, out);
}

extern "C" int specmg_setup_alloc(const double* perm_dev, int32_t perm_components, const specmg_grid* grid,
                                  const specmg_opts* opts, const specmg_allocator* allocator, void* stream,
                                  specmg_ctx** out) {
    g_last_error.clear();
    if (!out || !grid || !opts || !perm_dev) return fail(SPECMG_EINVAL, "null argument");
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(SPECMG_EINVAL, "allocator needs both alloc and free");
    *out = nullptr;
    if (perm_components != 1 && perm_components != 3)
        return fail(SPECMG_EINVAL, "perm_components must be 1 (isotropic) or 3 (orthotropic)");
    if (perm_components == 3 && (opts->precision == SPECMG_FP32_VCYCLE || opts->precision == SPECMG_FP32_STORE))
        return fail(SPECMG_EINVAL, "orthotropic permeability needs a float64 fine level (FP64 or FP32_BASIS)");
    if (perm_components == 3 && opts->warm_start == SPECMG_WS_CNN)
        return fail(SPECMG_EINVAL, "the learned warm start needs isotropic permeability");
    const specmg_grid& G = *grid;
    if (G.sub != 8) return fail(SPECMG_EINVAL, "sub must be 8");
    if (G.agg != 2 && G.agg != 4) return fail(SPECMG_EINVAL, "agg must be 2 or 4");
    if (!(G.hx > 0) || !(G.hy > 0) || !(G.hz > 0) || !std::isfinite(G.hx) || !std::isfinite(G.hy) ||
        !std::isfinite(G.hz))
        return fail(SPECMG_EINVAL, "spacings must be positive and finite");
    if (opts->levels < 2 || opts->levels > 8) return fail(SPECMG_EINVAL, "levels must be in [2, 8]");
    if (opts->eigs_per_subdomain < 1 || opts->eigs_per_subdomain > 8)
        return fail(SPECMG_EINVAL, "eigs_per_subdomain must be in [1, 8]");
    if (opts->nu < 1 || opts->nu > 2) return fail(SPECMG_EINVAL, "nu must be 1 or 2");
    if (opts->nu_c < 0 || opts->nu_c > 2) return fail(SPECMG_EINVAL, "nu_c must be 0 (= nu), 1 or 2");
    if (opts->precision != SPECMG_FP64 && opts->precision != SPECMG_FP32_VCYCLE &&
        opts->precision != SPECMG_FP32_BASIS && opts->precision != SPECMG_FP32_STORE)
        return fail(SPECMG_EINVAL, "unknown precision");
    if (opts->warm_start != SPECMG_WS_NONE && opts->warm_start != SPECMG_WS_CNN)
        return fail(SPECMG_EINVAL, "unknown warm_start");
    if (opts->warm_start == SPECMG_WS_CNN && !opts->cnn_weights)
        return fail(SPECMG_EINVAL, "warm_start CNN needs cnn_weights");
    if (opts->warm_start == SPECMG_WS_CNN && (G.hx != G.hy || G.hx != G.hz))
        return fail(SPECMG_EINVAL, "warm_start CNN needs equal spacings (the network saw only those)");
    if (opts->warm_start == SPECMG_WS_CNN && (opts->eigs_per_subdomain & 1))
        return fail(SPECMG_EINVAL, "warm_start CNN needs an even eigs_per_subdomain");
    const int tcc = opts->eigs_coarse > 0 ? opts->eigs_coarse : opts->eigs_per_subdomain;
    if (opts->eigs_coarse < 0 || tcc > 20) return fail(SPECMG_EINVAL, "eigs_coarse must be in [0, 20]");
    if (G.agg == 4 && opts->levels >= 4 && tcc > 9)
        return fail(SPECMG_EINVAL, "agg 4 with four or more levels needs eigs_coarse <= 9");
    if (!(opts->eig_threshold_coarse >= 0.0) || !std::isfinite(opts->eig_threshold_coarse))
        return fail(SPECMG_EINVAL, "eig_threshold_coarse must be finite and >= 0");
    if (!(opts->eig_threshold >= 0.0) || !std::isfinite(opts->eig_threshold))
        return fail(SPECMG_EINVAL, "eig_threshold must be finite and >= 0");
    long div = 8;
    for (int l = 2; l < opts->levels; ++l) div *= G.agg;
    if (G.nx <= 0 || G.ny <= 0 || G.nz <= 0 || G.nx % div || G.ny % div || G.nz % div)
        return fail(SPECMG_EINVAL, "nx, ny, nz must be positive multiples of 8*agg^(levels-2)");
    if ((long)G.nx * G.ny * G.nz / 512 < 2) return fail(SPECMG_EINVAL, "need at least two 8^3 elements");
    specmg_ctx* c = new specmg_ctx();
    if (allocator) {
        c->al.alloc = allocator->alloc;
        c->al.release = allocator->free;
        c->al.user = allocator->user;
    }
    c->al.stream = (hipStream_t)stream;
    c->grid = G;
    c->opts = *opts;
    c->ncomp = perm_components;
    c->levels = opts->levels;
    c->target = opts->eigs_per_subdomain;
    c->L = c->target + 3;
    c->nvec = nvec_for(c->target);
    c->target_cc = tcc;
    c->Lcc = tcc + 3;
    c->nvec_cc = nvec_for(tcc);
    c->thr_cc = opts->eig_threshold_coarse;
    c->thr_c = opts->eig_threshold;
    c->fp32 = opts->precision == SPECMG_FP32_VCYCLE;
    c->fp32_basis = opts->precision == SPECMG_FP32_BASIS;
    c->fp32_store = opts->precision == SPECMG_FP32_STORE;
    c->flexible = c->fp32 || c->fp32_store;
    c->nu = opts->nu;
    c->nu_c = opts->nu_c > 0 ? opts->nu_c : opts->nu;
    int rc;
    try {
        rc = do_setup(c, perm_dev, (hipStream_t)stream);
    } catch (const HipError& e) {
        rc = fail(SPECMG_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    if (rc == SPECMG_OK || rc == SPECMG_EEIG) {
        *out = c;
    } else {
        delete c;
    }
    return rc;
}

extern "C" int specmg_apply_operator(specmg_ctx* c, const double* x, double* y, void* stream) {
    if (!c || !x || !y) return fail(SPECMG_EINVAL, "null argument");
    try {
        const hipStream_t s = (hipStream_t)stream;
        launch_to_elem(c->fg, x, c->b_e, s);
        launch_apply_A(c->fg, c->kt, c->b_e, nullptr, c->x_e, 0, s);
        launch_to_natural(c->fg, c->x_e, y, s);
        HIPCHK(hipGetLastError());
    } catch (const HipError& e) {
        return fail(SPECMG_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return SPECMG_OK;
}

extern "C" int specmg_apply_precond(specmg_ctx* c, const double* r, double* z, void* stream) {
    if (!c || !r || !z) return fail(SPECMG_EINVAL, "null argument");
    if (r == z) return fail(SPECMG_EINVAL, "r and z must not alias");
    try {
        const hipStream_t s = (hipStream_t)stream;
        launch_to_elem(c->fg, r, c->b_e, s);
        run_vcycle(c, c->b_e, c->x_e, nullptr, 0, 0, 0, s);
        launch_to_natural(c->fg, c->x_e, z, s);
        HIPCHK(hipGetLastError());
    } catch (const HipError& e) {
        return fail(SPECMG_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return SPECMG_OK;
}

static void read_scalars(specmg_ctx* c, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // a launch that failed since the last check (it did no work)
    HIPCHK(hipGetLastError());
}

static double dev_dot(specmg_ctx* c, const double* a, const double* b, hipStream_t s) {
    launch_dot(a, b, c->n, c->dtmp, c->rb, RS_GEN, s);
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, c->dtmp, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return v;
}

__global__ void k_reset_done(Scalars* sc) { sc->done = 0; }

static int do_solve(specmg_ctx* c, const double* b_nat, double* x_nat, int use_x0, double tol, int max_iter,
                    specmg_solve_info* info, hipStream_t s) {
    const double t0 = now_ms();
    const int64_t n = c->n;
    specmg_solve_info si = c->setup_info;
    c->ev_used = 0;
    c->recs.clear();
    c->cur_iter = 0;
    si.iters = 0;
    si.converged = 0;
    si.replacements = 0;
    // compatibility of the source: |sum f| <= 1e-12 sum |f|
    launch_sum_abs(b_nat, n, c->dtmp, c->dtmp + 1, c->rb, s);
    double sa[2];
    HIPCHK(hipMemcpyAsync(sa, c->dtmp, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (std::fabs(sa[0]) > 1e-12 * sa[1]) return fail(SPECMG_ERHS, "source does not sum to zero");
    const double nb = std::sqrt(dev_dot(c, b_nat, b_nat, s));
    if (nb == 0.0) {
        launch_fill(x_nat, 0.0, n, s);
        si.converged = 1;
        si.solve_ms = now_ms() - t0;
        if (info) *info = si;
        return SPECMG_OK;
    }
    // the solve runs in element order
    const double* b = c->b_e;
    double* x = c->x_e;
    launch_to_elem(c->fg, b_nat, c->b_e, s);
    if (use_x0) launch_to_elem(c->fg, x_nat, c->x_e, s);
    if (use_x0) launch_apply_A(c->fg, c->kt, x, b, c->r, 1, s);
    else {
        launch_fill(x, 0.0, n, s);
        launch_copy(c->r, b, n, s);
    }
    const double thresh2 = (tol * nb) * (tol * nb);
    const int flexible = c->flexible;
    launch_pcg_init(c->sc, thresh2, flexible, s);
    int rc = SPECMG_OK;
    double r0 = std::sqrt(dev_dot(c, c->r, c->r, s));
    bool converged = r0 <= tol * nb;
    int k = 0;   // CG iterations issued so far (= device iteration counter after a sync)
    bool restart = true;
    while (!converged) {
        if (restart) {
            // z = P^{-1} r, r.z and beta (first call: beta unused)
            run_vcycle(c, c->r, c->z, c->q, 0, 1, 0, s);
            restart = false;
        }
        const int chunk = 4;
        for (int i = 0; i < chunk && k < max_iter; ++i, ++k) {
            const int first = (k == 0) ? 1 : 0;
            const int pb = k & 1;
            c->cur_iter = k + 1;
            size_t ev = prof_begin(c, s);
            launch_p_update(c->fg, c->z, c->p[pb ^ 1], c->p[pb], x, c->sc, first, s);
            prof_end(c, ev, PC_PUPDATE, s);
            ev = prof_begin(c, s);
            launch_spmv_pcg(c->fg, c->kt, c->p[pb], c->q, c->sc, c->rb, pb, s);
            prof_end(c, ev, PC_SPMV, s);
            run_vcycle(c, c->r, c->z, c->q, 1 | 2, 1 | 2, 1, s);
        }
        read_scalars(c, s);
        const Scalars& h = *c->sc_host;
        k = h.iter;
        if (h.done == 2) {
            launch_axpy_x(x, c->p[0], c->p[1], c->sc, n, s);
            rc = fail(SPECMG_EBREAKDOWN, "breakdown: p^T A p not positive");
            break;
        }
        if (h.done == 1) {
            // confirm on the true residual; replace it when the check fails
            launch_axpy_x(x, c->p[0], c->p[1], c->sc, n, s);
            launch_apply_A(c->fg, c->kt, x, b, c->r, 1, s);
            const double rt = dev_dot(c, c->r, c->r, s);
            if (rt <= thresh2) {
                converged = true;
                break;
            }
            si.replacements += 1;
            hipLaunchKernelGGL(k_reset_done, dim3(1), dim3(1), 0, s, c->sc);
            restart = true;
            // the next spmv continues the direction update p = z + beta p
            if (k >= max_iter) break;
            continue;
        }
        if (k >= max_iter) {
            launch_axpy_x(x, c->p[0], c->p[1], c->sc, n, s);
            break;
        }
    }
    read_scalars(c, s);
    si.iters = c->sc_host->iter;
    si.rel_resid = std::sqrt(c->sc_host->rr) / nb;
    // zero-mean solution
    launch_sum_abs(x, n, c->dtmp, c->dtmp + 1, c->rb, s);
    launch_sub_mean(x, n, c->dtmp, s);
    launch_apply_A(c->fg, c->kt, x, b, c->q, 1, s);
    launch_to_natural(c->fg, x, x_nat, s);
    si.rel_resid_true = std::sqrt(dev_dot(c, c->q, c->q, s)) / nb;
    si.converged = converged ? 1 : 0;
    HIPCHK(hipStreamSynchronize(s));
    si.solve_ms = now_ms() - t0;
    if (c->prof_on) {
        // launches of iterations past the last executed one returned at once
        for (const auto& rcd : c->recs) {
            if (rcd.iter > si.iters) continue;
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[rcd.e0], c->ev_pool[rcd.e1]));
            c->prof_ms[rcd.cls] += ms;
            c->prof_count[rcd.cls] += 1;
        }
        c->recs.clear();
    }
    if (info) *info = si;
    if (rc != SPECMG_OK) return rc;
    if (!converged) return fail(SPECMG_ENOCONV, "maximum number of iterations reached");
    return SPECMG_OK;
}

extern "C" int specmg_pcg_solve(specmg_ctx* c, const double* rhs, double* x, int32_t use_x0, double tol,
                                int32_t max_iter, specmg_solve_info* info, void* stream) {
    g_last_error.clear();
    if (!c || !rhs || !x) return fail(SPECMG_EINVAL, "null argument");
    if (!(tol > 0) || max_iter < 1) return fail(SPECMG_EINVAL, "tol must be > 0 and max_iter >= 1");
    try {
        return do_solve(c, rhs, x, use_x0, tol, max_iter, info, (hipStream_t)stream);
    } catch (const HipError& e) {
        return fail(SPECMG_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
}

// Restarted flexible GMRES around the V-cycle (right preconditioning):
// x = x0 + Z_k y_k with z_j = P^{-1} v_j; classical Gram-Schmidt twice per
// Arnoldi step; the Arnoldi residual |g_{j+1}| decides the end of a cycle,
// the true residual b - A x the end of the solve (else a restart from it).
static int do_gmres(specmg_ctx* c, const double* b_nat, double* x_nat, int use_x0, int restart, double tol,
                    int max_iter, specmg_solve_info* info, hipStream_t s) {
    const double t0 = now_ms();
    const int64_t n = c->n;
    specmg_solve_info si = c->setup_info;
    si.iters = 0;
    si.converged = 0;
    si.replacements = 0;
    const int prof_saved = c->prof_on;   // the per-kernel timing covers pcg_solve only
    c->prof_on = 0;
    struct Restore {
        specmg_ctx* c;
        int v;
        ~Restore() { c->prof_on = v; }
    } restore{c, prof_saved};
    launch_sum_abs(b_nat, n, c->dtmp, c->dtmp + 1, c->rb, s);
    double sa[2];
    HIPCHK(hipMemcpyAsync(sa, c->dtmp, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (std::fabs(sa[0]) > 1e-12 * sa[1]) return fail(SPECMG_ERHS, "source does not sum to zero");
    const double nb = std::sqrt(dev_dot(c, b_nat, b_nat, s));
    if (nb == 0.0) {
        launch_fill(x_nat, 0.0, n, s);
        si.converged = 1;
        si.solve_ms = now_ms() - t0;
        if (info) *info = si;
        return SPECMG_OK;
    }
    if (restart > c->gm_restart) {
        if (c->gm_buf) {
            HIPCHK(hipStreamSynchronize(s));
            c->al.put(c->gm_buf);
        }
        c->gm_buf = nullptr;
        c->gm_restart = 0;
        const size_t doubles = (size_t)(2 * restart + 2) * (size_t)n + mdot_part_doubles();
        c->gm_buf = (double*)c->al.get(doubles * sizeof(double));
        c->gm_restart = restart;
    }
    if (!c->gm_state) c->gm_state = (GmresState*)c->al.get(sizeof(GmresState));
    double* V = c->gm_buf;                          // restart + 1 vectors
    double* Z = V + (size_t)(restart + 1) * n;      // restart vectors
    double* w = Z + (size_t)restart * n;
    double* part = w + n;
    GmresState* st = c->gm_state;
    const double thr = tol * nb;
    struct Host {
        double res, beta;
        int done;
    } hs{};
    auto read_state = [&]() {
        HIPCHK(hipMemcpyAsync(&hs.res, &st->res, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hs.beta, &st->beta, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hs.done, &st->done, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipGetLastError());
    };
    // the solve runs in element order
    const double* b = c->b_e;
    double* x = c->x_e;
    launch_to_elem(c->fg, b_nat, c->b_e, s);
    if (use_x0) launch_to_elem(c->fg, x_nat, c->x_e, s);
    // r0 into V_0
    if (use_x0) launch_apply_A(c->fg, c->kt, x, b, V, 1, s);
    else {
        launch_fill(x, 0.0, n, s);
        launch_copy(V, b, n, s);
    }
    launch_mdot(V, n, 1, V, n, part, &st->nrm2, s);
    launch_gmres_begin(st, thr, s);
    read_state();
    bool converged = hs.done != 0;
    int rc = SPECMG_OK;
    int it = 0;
    while (!converged && it < max_iter) {
        launch_scale_dev(V, V, &st->inv, n, s);
        int k = 0;
        for (int j = 0; j < restart && it < max_iter; ++j) {
            double* vj = V + (size_t)j * n;
            double* zj = Z + (size_t)j * n;
            run_vcycle(c, vj, zj, nullptr, 0, 0, 0, s);
            launch_apply_A(c->fg, c->kt, zj, nullptr, w, 0, s);
            launch_mdot(V, n, j + 1, w, n, part, st->h, s);
            launch_maxpy(V, n, j + 1, st->h, -1.0, w, n, s);
            launch_mdot(V, n, j + 1, w, n, part, st->h2, s);
            launch_maxpy(V, n, j + 1, st->h2, -1.0, w, n, s);
            launch_mdot(w, n, 1, w, n, part, &st->nrm2, s);
            launch_gmres_step(st, j, thr, s);
            launch_scale_dev(V + (size_t)(j + 1) * n, w, &st->inv, n, s);
            ++it;
            k = j + 1;
            read_state();
            if (hs.done) break;
        }
        if (hs.done == 2) {
            rc = fail(SPECMG_EBREAKDOWN, "GMRES breakdown: singular Hessenberg column");
            break;
        }
        launch_gmres_lsq(st, k, s);
        launch_maxpy(Z, n, k, st->y, 1.0, x, n, s);
        launch_apply_A(c->fg, c->kt, x, b, V, 1, s);
        launch_mdot(V, n, 1, V, n, part, &st->nrm2, s);
        launch_gmres_begin(st, thr, s);
        read_state();
        converged = hs.done != 0;
        if (!converged && it < max_iter) si.replacements += 1;
    }
    si.iters = it;
    si.rel_resid = hs.beta / nb;
    launch_sum_abs(x, n, c->dtmp, c->dtmp + 1, c->rb, s);
    launch_sub_mean(x, n, c->dtmp, s);
    launch_apply_A(c->fg, c->kt, x, b, w, 1, s);
    launch_to_natural(c->fg, x, x_nat, s);
    si.rel_resid_true = std::sqrt(dev_dot(c, w, w, s)) / nb;
    si.converged = converged ? 1 : 0;
    HIPCHK(hipStreamSynchronize(s));
    si.solve_ms = now_ms() - t0;
    if (info) *info = si;
    if (rc != SPECMG_OK) return rc;
    if (!converged) return fail(SPECMG_ENOCONV, "maximum number of iterations reached");
    return SPECMG_OK;
}

extern "C" int specmg_gmres_solve(specmg_ctx* c, const double* rhs, double* x, int32_t use_x0, int32_t restart,
                                  double tol, int32_t max_iter, specmg_solve_info* info, void* stream) {
    g_last_error.clear();
    if (!c || !rhs || !x) return fail(SPECMG_EINVAL, "null argument");
    if (!(tol > 0) || max_iter < 1) return fail(SPECMG_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (restart < 1 || restart > kMaxRestart) return fail(SPECMG_EINVAL, "restart must be in [1, 64]");
    if (rhs == x) return fail(SPECMG_EINVAL, "rhs and x must not alias");
    try {
        return do_gmres(c, rhs, x, use_x0, restart, tol, max_iter, info, (hipStream_t)stream);
    } catch (const HipError& e) {
        return fail(SPECMG_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
}

namespace specmg {
void launch_flux(const FineGeom& g, double hx, double hy, double hz, const double* kt, const double* p, double* vx,
                 double* vy, double* vz, hipStream_t s);
void launch_mass_balance(int nx, int ny, int nz, double hx, double hy, double hz, const double* vx, const double* vy,
                         const double* vz, const double* f, double* res, hipStream_t s);
}  // namespace specmg

extern "C" int specmg_recover_flux(specmg_ctx* c, const double* p, double* vx, double* vy, double* vz,
                                   void* stream) {
    g_last_error.clear();
    if (!c || !p || !vx || !vy || !vz) return fail(SPECMG_EINVAL, "null argument");
    try {
        launch_flux(c->fg, c->grid.hx, c->grid.hy, c->grid.hz, c->kt, p, vx, vy, vz, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    } catch (const HipError& e) {
        return fail(SPECMG_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return SPECMG_OK;
}

extern "C" int specmg_mass_balance(specmg_ctx* c, const double* vx, const double* vy, const double* vz,
                                   const double* f, double* res, void* stream) {
    g_last_error.clear();
    if (!c || !vx || !vy || !vz || !f || !res) return fail(SPECMG_EINVAL, "null argument");
    try {
        launch_mass_balance(c->fg.nx, c->fg.ny, c->fg.nz, c->grid.hx, c->grid.hy, c->grid.hz, vx, vy, vz, f, res,
                            (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    } catch (const HipError& e) {
        return fail(SPECMG_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return SPECMG_OK;
}

extern "C" int specmg_get_info(specmg_ctx* c, int32_t* levels, int32_t* dims, int32_t* elems, int32_t* widths,
                               specmg_solve_info* setup_info) {
    if (!c) return fail(SPECMG_EINVAL, "null context");
    if (levels) *levels = c->levels;
    if (widths) {
        for (int i = 0; i < 8; ++i) widths[i] = 0;
        widths[0] = 1;
        for (size_t li = 0; li < c->lev.size() && li + 1 < 8; ++li) widths[li + 1] = c->lev[li].L;
    }
    if (dims) {
        for (int i = 0; i < 8; ++i) dims[i] = 0;
        dims[0] = (int)c->n;
        for (size_t li = 0; li < c->lev.size() && li + 1 < 8; ++li) dims[li + 1] = c->lev[li].dim;
    }
    if (elems) {
        for (int i = 0; i < 8; ++i) elems[i] = 0;
        elems[0] = (int)c->n;
        for (size_t li = 0; li < c->lev.size() && li + 1 < 8; ++li) elems[li + 1] = c->lev[li].g.m;
    }
    if (setup_info) *setup_info = c->setup_info;
    return SPECMG_OK;
}

extern "C" int specmg_copy_level(specmg_ctx* c, int32_t level, int32_t which, void* dst, size_t bytes) {
    if (!c || !dst) return fail(SPECMG_EINVAL, "null argument");
    if (level < 2 || level > c->levels) return fail(SPECMG_EINVAL, "level out of range");
    Level& lv = c->lev[level - 2];
    const size_t m = lv.g.m, L = lv.L;
    const void* src = nullptr;
    size_t need = 0;
    switch (which) {
        case 0: src = lv.nkeep; need = m * sizeof(int); break;
        case 1: src = lv.lam; need = m * L * sizeof(double); break;
        case 2: src = lv.basis; need = m * L * lv.rows * sizeof(double); break;
        case 3: src = lv.Ad; need = m * L * L * sizeof(double); break;
        case 4: src = lv.Aoff; need = m * 3 * L * L * sizeof(double); break;
        case 5: src = lv.status; need = m * sizeof(int); break;
        default: return fail(SPECMG_EINVAL, "unknown array");
    }
    if (bytes != need) return fail(SPECMG_EINVAL, "size mismatch: expected " + std::to_string(need));
    if (which == 2 && level == 2) {
        // the level-2 basis is stored in the phi_pos order; exported with the
        // cells of each column in natural order x + 8 (y + 8 z)
        std::vector<double> tmp(m * L * 512);
        if (hipMemcpy(tmp.data(), src, need, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(SPECMG_EDEVICE, "copy failed");
        double* out = static_cast<double*>(dst);
        for (size_t col = 0; col < m * L; ++col)
            for (int cc = 0; cc < 512; ++cc) out[col * 512 + cc] = tmp[col * 512 + phi_pos(cc)];
        return SPECMG_OK;
    }
    if (hipMemcpy(dst, src, need, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(SPECMG_EDEVICE, "copy failed");
    return SPECMG_OK;
}

extern "C" int specmg_set_profiling(specmg_ctx* c, int32_t on) {
    if (!c) return fail(SPECMG_EINVAL, "null context");
    c->prof_on = on ? 1 : 0;
    for (int i = 0; i < 8; ++i) {
        c->prof_ms[i] = 0.0;
        c->prof_count[i] = 0;
    }
    return SPECMG_OK;
}

extern "C" int specmg_get_profile(specmg_ctx* c, double* ms, int32_t* launches, double* bytes) {
    if (!c) return fail(SPECMG_EINVAL, "null context");
    const double n = (double)c->n;
    const double w = (c->fp32 || c->fp32_store) ? 4.0 : 8.0;   // stored word of the fine V-cycle
    const double phi_cells = 512.0 * c->lev[0].dim; // sum over elements of 512 * nkeep
    double b[8] = {0};
    b[PC_SPMV] = n * 8.0 * 3.0;                      // p, kappa~ in; q out
    b[PC_PUPDATE] = n * 8.0 * 5.0;                   // z, p_old, x in; p, x out
    b[PC_PRE] = n * (8.0 * 3.0 + 2.0 * w + w);       // r, q in, r out; kappa~, 1/d in; u out
    const double wb = (c->fp32_basis || c->fp32_store) ? 4.0 : w;   // basis word size
    b[PC_RESTRICT] = n * (2.0 * w + 8.0) + phi_cells * wb;  // u, kappa~, r; phi
    b[PC_PROLONG] = n * 2.0 * w + phi_cells * wb;            // u in/out; phi
    b[PC_POST] = n * (3.0 * w + 8.0 * 2.0 + (c->flexible ? 8.0 : 0.0));  // kappa~, 1/d, u, r in; z out (q)
    b[PC_COARSE] = c->coarse_bytes;
    b[PC_COARSEST] = c->coarsest_bytes;
    for (int i = 0; i < 8; ++i) {
        if (ms) ms[i] = c->prof_ms[i];
        if (launches) launches[i] = c->prof_count[i];
        if (bytes) bytes[i] = b[i];
    }
    return SPECMG_OK;
}
