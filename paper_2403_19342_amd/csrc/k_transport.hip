// Two-phase flow of Section 6: the total-mobility scaling of the pressure
// permeability (eq. v) and the explicit saturation sub-steps of the improved
// IMPES scheme (eq. ES), plus their C-ABI entry points.
//
// Fluid model: S* = clamp((S - 0.2) / 0.6, 0, 1), k_w = S*^2,
// k_o = (1 - S*)^2, mu_w = 0.3, mu_o = 3.0; lambda = k_w/mu_w + k_o/mu_o
// and f_w = (k_w/mu_w) / lambda.  Wells are rate controlled: q > 0 injects
// water, q < 0 produces the cell's mixture (q_w = f_w(S) q).
//
// One sub-step is two grid-stride passes over the cells:
//   k_sat_rate    r_i = (q_w - sum_d (F_+ - F_-) / h_d) / phi_i with the
//                 face water flux F = f_w(S_upstream) v; each block writes
//                 the largest |r| of its cells to its own slot;
//   k_sat_update  every block first reduces those slots to the grid's
//                 largest rate (a max is exact in any order), then
//                 dt = DS_max / max|r| (0 when every rate is zero),
//                 S_i += dt r_i, and block 0 adds dt to the elapsed time.
// f_w of every cell is evaluated once per sub-step, by the pass that writes
// S (k_transport_begin for the initial S), and stored: the rate pass reads
// it for the cell and its upstream neighbours instead of re-evaluating the
// four divisions of the fluid law up to seven times per cell.
// A single atomic max per block onto one word serialises thousands of
// blocks at one L2 address; the slot array keeps the reduction in plain
// loads and stores.  Nothing is copied to the host between sub-steps.
#include <cstdint>
#include <mutex>
#include <string>

#include "common.hpp"
#include "../../include/specmg.h"

namespace specmg {
int fail_message(int code, const char* msg);   // sets the thread's last error, returns code
}

// Kernels live in the named namespace so that profiles show their names.
namespace specmg {

constexpr double kSwc = 0.2;
constexpr double kSpan = 0.6;
constexpr double kMuW = 0.3;
constexpr double kMuO = 3.0;

__device__ __forceinline__ void phase_mobilities(double s, double& lw, double& lo) {
    double sn = (s - kSwc) / kSpan;
    sn = fmin(fmax(sn, 0.0), 1.0);
    lw = sn * sn / kMuW;
    lo = (1.0 - sn) * (1.0 - sn) / kMuO;
}

__device__ __forceinline__ double water_fraction(double s) {
    double lw, lo;
    phase_mobilities(s, lw, lo);
    return lw / (lw + lo);
}

__global__ __launch_bounds__(256) void k_total_mobility(int64_t n, const double* __restrict__ perm,
                                                        const double* __restrict__ s, double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double lw, lo;
        phase_mobilities(s[i], lw, lo);
        out[i] = perm[i] * (lw + lo);
    }
}

constexpr int kMaxRateBlocks = 2048;   // slots of the per-block maxima in the workspace
constexpr int kMaxUpdateBlocks = 512;  // each update block re-reads every slot: keep that L2 traffic small

__global__ __launch_bounds__(256) void k_transport_begin(int64_t n, const double* __restrict__ s,
                                                         double* __restrict__ fw, double* t) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        fw[i] = water_fraction(s[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) *t = 0.0;
}

// cell coordinates of a flat index; 32-bit division when the grid allows it
__device__ __forceinline__ void cell_xyz(int64_t i, int nx, int ny, int64_t n, int& x, int& y, int& z) {
    if (n <= 0xffffffffll) {
        const uint32_t u = (uint32_t)i, row = u / (uint32_t)nx;
        x = (int)(u - row * (uint32_t)nx);
        z = (int)(row / (uint32_t)ny);
        y = (int)(row - (uint32_t)z * (uint32_t)ny);
    } else {
        const int64_t row = i / nx;
        x = (int)(i - row * nx);
        z = (int)(row / ny);
        y = (int)(row - (int64_t)z * ny);
    }
}

__global__ __launch_bounds__(256) void k_sat_rate(int nx, int ny, int nz, double hx, double hy, double hz,
                                                  const double* __restrict__ phi,
                                                  const double* __restrict__ q, const double* __restrict__ vx,
                                                  const double* __restrict__ vy, const double* __restrict__ vz,
                                                  const double* __restrict__ fw, double* __restrict__ rate,
                                                  double* __restrict__ block_max) {
    __shared__ double red[4];
    const int64_t sy = nx, sz = (int64_t)nx * ny, n = sz * nz;
    double m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        cell_xyz(i, nx, ny, n, x, y, z);
        const double fi = fw[i];
        // water flux through the + and - faces of one axis, upstream weighted;
        // the boundary faces carry nothing
        auto axis_div = [&](bool has_plus, bool has_minus, const double* __restrict__ v, int64_t st, double h) {
            double fp = 0.0, fm = 0.0;
            if (has_plus) {
                const double vp = v[i];
                fp = (vp >= 0.0 ? fi : fw[i + st]) * vp;
            }
            if (has_minus) {
                const double vm = v[i - st];
                fm = (vm >= 0.0 ? fw[i - st] : fi) * vm;
            }
            return (fp - fm) / h;
        };
        double div = axis_div(x + 1 < nx, x > 0, vx, 1, hx);
        div += axis_div(y + 1 < ny, y > 0, vy, sy, hy);
        div += axis_div(z + 1 < nz, z > 0, vz, sz, hz);
        const double qi = q[i];
        const double qw = qi > 0.0 ? qi : fi * qi;
        const double r = (qw - div) / phi[i];
        rate[i] = r;
        m = fmax(m, fabs(r));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) block_max[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_sat_update(int64_t n, const double* __restrict__ rate,
                                                    double* __restrict__ s, double* __restrict__ fw,
                                                    const double* __restrict__ block_max, int nmax, double ds_max,
                                                    double* t) {
    __shared__ double red[4];
    double m = 0.0;
    for (int k = threadIdx.x; k < nmax; k += blockDim.x) m = fmax(m, block_max[k]);
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double dt = m > 0.0 ? ds_max / m : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double si = s[i] + dt * rate[i];
        s[i] = si;
        fw[i] = water_fraction(si);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *t += dt;
}

static int blocks_for(int64_t n, int cap) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < cap ? (b < 1 ? 1 : b) : cap);
}

static int device_error(hipError_t e, const char* what) {
    return fail_message(SPECMG_EDEVICE, (std::string(what) + ": " + hipGetErrorString(e)).c_str());
}

}  // namespace specmg

using namespace specmg;

extern "C" int specmg_total_mobility(const double* perm_dev, const double* s_dev, double* perm_eff_dev, int64_t n,
                                     void* stream) {
    if (!perm_dev || !s_dev || !perm_eff_dev || n < 0) return fail_message(SPECMG_EINVAL, "bad arguments");
    if (n == 0) return SPECMG_OK;
    hipLaunchKernelGGL(k_total_mobility, dim3(blocks_for(n, 8192)), dim3(256), 0, (hipStream_t)stream, n, perm_dev,
                       s_dev, perm_eff_dev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECMG_OK : device_error(e, "k_total_mobility");
}

// Checks and launches shared by specmg_transport and its allocation-free
// variant; work holds 2 n + kMaxRateBlocks doubles (rates, f_w, block maxima).
static int run_transport(const specmg_grid* grid, const double* phi_dev, const double* q_dev, const double* vx_dev,
                         const double* vy_dev, const double* vz_dev, double* s_dev, int32_t substeps, double ds_max,
                         double* work_dev, double* t_dev, hipStream_t s) {
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    double* rate = work_dev;
    double* fw = work_dev + n;
    double* block_max = work_dev + 2 * n;
    const int nb = blocks_for(n, kMaxRateBlocks), nu = blocks_for(n, kMaxUpdateBlocks);
    hipLaunchKernelGGL(k_transport_begin, dim3(nu), dim3(256), 0, s, n, s_dev, fw, t_dev);
    for (int m = 0; m < substeps; ++m) {
        hipLaunchKernelGGL(k_sat_rate, dim3(nb), dim3(256), 0, s, grid->nx, grid->ny, grid->nz, grid->hx, grid->hy,
                           grid->hz, phi_dev,
                           q_dev, vx_dev, vy_dev, vz_dev, fw, rate, block_max);
        hipLaunchKernelGGL(k_sat_update, dim3(nu), dim3(256), 0, s, n, rate, s_dev, fw, block_max, nb, ds_max,
                           t_dev);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECMG_OK : device_error(e, "saturation sub-steps");
}

static int check_transport_args(const specmg_grid* grid, const double* phi_dev, const double* q_dev,
                                const double* vx_dev, const double* vy_dev, const double* vz_dev, const double* s_dev,
                                int32_t substeps, double ds_max, const double* t_dev) {
    if (!grid || !phi_dev || !q_dev || !vx_dev || !vy_dev || !vz_dev || !s_dev || !t_dev)
        return fail_message(SPECMG_EINVAL, "null argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail_message(SPECMG_EINVAL, "grid sizes must be >= 1");
    if (!(grid->hx > 0) || !(grid->hy > 0) || !(grid->hz > 0))
        return fail_message(SPECMG_EINVAL, "spacings must be positive");
    if (substeps < 0) return fail_message(SPECMG_EINVAL, "substeps must be >= 0");
    if (!(ds_max > 0) || ds_max > 1.0) return fail_message(SPECMG_EINVAL, "ds_max must be in (0, 1]");
    return SPECMG_OK;
}

extern "C" int specmg_transport(const specmg_grid* grid, const double* phi_dev, const double* q_dev,
                                const double* vx_dev, const double* vy_dev, const double* vz_dev, double* s_dev,
                                int32_t substeps, double ds_max, double* work_dev, double* t_dev, void* stream) {
    if (!work_dev) return fail_message(SPECMG_EINVAL, "null argument");
    const int rc = check_transport_args(grid, phi_dev, q_dev, vx_dev, vy_dev, vz_dev, s_dev, substeps, ds_max, t_dev);
    if (rc != SPECMG_OK) return rc;
    return run_transport(grid, phi_dev, q_dev, vx_dev, vy_dev, vz_dev, s_dev, substeps, ds_max, work_dev, t_dev,
                         (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the workspace is a file-scope device array,
// `scratch`, sized for SPECMG_TRANSPORT_NOALLOC_MAX_CELLS cells.  Each GPU
// holds its own copy (32 MiB + 16 KiB) from the library's load until the
// process ends.  Its device address is looked up once per device (with that
// device current) by hipGetSymbolAddress; host code never passes the
// array's name itself to a kernel.  Nothing in it needs clearing: every
// sub-step writes the rates and slots before reading them and the first
// kernel writes f_w.  Calls that overlap on one GPU share the array and race.
constexpr int64_t kNoAllocMaxCells = SPECMG_TRANSPORT_NOALLOC_MAX_CELLS;
constexpr int64_t kScratchDoubles = 2 * kNoAllocMaxCells + kMaxRateBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// device address of this device's scratch array (looked up on first use)
static int scratch_address(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail_message(SPECMG_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return device_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return SPECMG_OK;
}

extern "C" int specmg_transport_noalloc(const specmg_grid* grid, const double* phi_dev, const double* q_dev,
                                        const double* vx_dev, const double* vy_dev, const double* vz_dev,
                                        double* s_dev, int32_t substeps, double ds_max, double* t_dev, void* stream) {
    const int rc = check_transport_args(grid, phi_dev, q_dev, vx_dev, vy_dev, vz_dev, s_dev, substeps, ds_max, t_dev);
    if (rc != SPECMG_OK) return rc;
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    if (n > kNoAllocMaxCells)
        return fail_message(SPECMG_EINVAL, ("grid of " + std::to_string(n) + " cells exceeds the " +
                                            std::to_string(kNoAllocMaxCells) + " cells of the built-in workspace")
                                               .c_str());
    double* work = nullptr;
    const int ra = scratch_address(&work);
    if (ra != SPECMG_OK) return ra;
    return run_transport(grid, phi_dev, q_dev, vx_dev, vy_dev, vz_dev, s_dev, substeps, ds_max, work, t_dev,
                         (hipStream_t)stream);
}
