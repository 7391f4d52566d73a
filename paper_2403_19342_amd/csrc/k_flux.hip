// Velocity recovery and the cell mass balance (Section 2.2).  Once A p = f
// is solved, v = M_t^{-1} B^T p; with the trapezoidal quadrature this is
// the two-point flux of eq. (velocity) on every interior face of axis d,
//   v_{i+1/2} = -kappa_{i+1/2} (p_{i+1} - p_i) / h_d = -h_d c_d kappa~_{i+1/2} (p_{i+1} - p_i)
// (kappa~ = kappa / hx^2 as stored, c_d = (hx/h_d)^2, harmonic mean on the
// face; for orthotropic K the stored kappa~ of axis d is kappa_d / h_d^2
// and c_d = 1), and zero on the no-flow boundary.  The mass balance of a cell is
// the face areas times the flux jumps over the cell volume, minus f_i,
// which is (A p - f)_i up to rounding.  One thread per cell, grid-stride.
#include "common.hpp"

namespace specmg {

__device__ __forceinline__ double face_harm(double a, double b) {
    const double s = a + b;
    return s > 0.0 ? (2.0 * a * b) / s : 0.0;
}

// kt is in element order (eidx): kappa_d / h_d^2 for d = x, y, z in three
// arrays (g.ortho, cy = cz = 1), otherwise one array kappa / hx^2; p and the
// fluxes are in natural order
__global__ __launch_bounds__(256) void k_flux(FineGeom g, double hx, double hy, double hz,
                                              const double* __restrict__ kt, const double* __restrict__ p,
                                              double* __restrict__ vx, double* __restrict__ vy,
                                              double* __restrict__ vz) {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int64_t sy = nx, sz = (int64_t)nx * ny, n = sz * nz;
    const double* ky = g.ortho ? kt + n : kt;
    const double* kz = g.ortho ? kt + 2 * n : kt;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / sy) % ny), z = (int)(i / sz);
        const double pc = p[i];
        const size_t ei = eidx(g, x, y, z);
        vx[i] = x + 1 < nx ? -hx * face_harm(kt[ei], kt[eidx(g, x + 1, y, z)]) * (p[i + 1] - pc) : 0.0;
        vy[i] = y + 1 < ny ? -hy * (face_harm(ky[ei], ky[eidx(g, x, y + 1, z)]) * g.cy) * (p[i + sy] - pc) : 0.0;
        vz[i] = z + 1 < nz ? -hz * (face_harm(kz[ei], kz[eidx(g, x, y, z + 1)]) * g.cz) * (p[i + sz] - pc) : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_mass_balance(int nx, int ny, int nz, double hx, double hy, double hz,
                                                      const double* __restrict__ vx, const double* __restrict__ vy,
                                                      const double* __restrict__ vz, const double* __restrict__ f,
                                                      double* __restrict__ res) {
    const int64_t sy = nx, sz = (int64_t)nx * ny, n = sz * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / sy) % ny), z = (int)(i / sz);
        const double net = hy * hz * (vx[i] - (x > 0 ? vx[i - 1] : 0.0)) +
                           hx * hz * (vy[i] - (y > 0 ? vy[i - sy] : 0.0)) +
                           hx * hy * (vz[i] - (z > 0 ? vz[i - sz] : 0.0));
        res[i] = net / (hx * hy * hz) - f[i];
    }
}

static int flux_blocks(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

void launch_flux(const FineGeom& g, double hx, double hy, double hz, const double* kt, const double* p, double* vx,
                 double* vy, double* vz, hipStream_t s) {
    hipLaunchKernelGGL(k_flux, dim3(flux_blocks((int64_t)g.ncell())), dim3(256), 0, s, g, hx, hy, hz, kt, p, vx, vy,
                       vz);
}

void launch_mass_balance(int nx, int ny, int nz, double hx, double hy, double hz, const double* vx, const double* vy,
                         const double* vz, const double* f, double* res, hipStream_t s) {
    hipLaunchKernelGGL(k_mass_balance, dim3(flux_blocks((int64_t)nx * ny * nz)), dim3(256), 0, s, nx, ny, nz, hx, hy,
                       hz, vx, vy, vz, f, res);
}

}  // namespace specmg
