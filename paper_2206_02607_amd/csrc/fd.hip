// Full-order explicit finite-difference heat solver in FP64 (Sec.
// "Thermodynamics / Full-order Model": 3-point Laplacian; Sec. "Image
// Processing / Full-order Model": 5-point Laplacian; forward Euler; zero
// Dirichlet boundary).  It generates training snapshots, judges reduced-order
// rollouts and is the fallback when a latent step fails.
//
// HBM-bound stencil: each substep reads u once and writes it once (8 + 8
// bytes per node, plus nu when it varies per node).  Grids are batched:
// `n_grid` independent fields of the same shape, one after another.
#include "common.hpp"

// Evaluate exactly in the written order (no fused multiply-add), so that the
// solver reproduces a plain double-precision evaluation of the same formula.
#pragma clang fp contract(off)

namespace crom {

// One substep on a batch of 1D fields [n_grid][n]: u_out = u + dt nu Lap u,
// end nodes held at 0.
__global__ void fd1d_kernel(const double* __restrict__ u, double* __restrict__ v,
                            const double* __restrict__ nu, int nu_per_node, int64_t n, int64_t n_grid,
                            double dt, double dx2) {
  const int64_t total = n * n_grid;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gidx = k / n, i = k - gidx * n;
    double out = 0.0;
    if (i > 0 && i < n - 1) {
      // boundary nodes count as 0 whatever the input holds there
      const double c = u[k];
      const double l = i - 1 > 0 ? u[k - 1] : 0.0;
      const double r = i + 1 < n - 1 ? u[k + 1] : 0.0;
      const double lap = ((l + r) - 2.0 * c) / dx2;
      const double nv = nu_per_node ? nu[k] : nu[gidx];
      out = c + (dt * nv) * lap;
    }
    v[k] = out;
  }
}

// One substep on a batch of 2D fields [n_grid][nx][ny] (index [i_x][i_y]).
__global__ void fd2d_kernel(const double* __restrict__ u, double* __restrict__ v,
                            const double* __restrict__ nu, int nu_per_node, int64_t nx, int64_t ny,
                            int64_t n_grid, double dt, double dx2) {
  const int64_t plane = nx * ny, total = plane * n_grid;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gidx = k / plane, r = k - gidx * plane;
    const int64_t i = r / ny, j = r - i * ny;
    double out = 0.0;
    if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1) {
      const double c = u[k];
      const double xm = i - 1 > 0 ? u[k - ny] : 0.0, xp = i + 1 < nx - 1 ? u[k + ny] : 0.0;
      const double ym = j - 1 > 0 ? u[k - 1] : 0.0, yp = j + 1 < ny - 1 ? u[k + 1] : 0.0;
      const double lap = ((((xm + xp) + ym) + yp) - 4.0 * c) / dx2;
      const double nv = nu_per_node ? nu[k] : nu[gidx];
      out = c + (dt * nv) * lap;
    }
    v[k] = out;
  }
}

}  // namespace crom

using namespace crom;

extern "C" {

crom_status crom_fd_heat(int32_t dim, const int64_t* shape, int64_t n_grid, const double* nu,
                         int32_t nu_per_node, double dx, double dt, int64_t steps, double* u,
                         double* scratch, void* stream) {
  if (dim != 1 && dim != 2) return fail(CROM_ERR_INVALID_ARG, "dim must be 1 or 2");
  if (!shape) return fail(CROM_ERR_INVALID_ARG, "shape is NULL");
  const int64_t nx = shape[0], ny = dim == 2 ? shape[1] : 1;
  if (nx < 1 || ny < 1 || n_grid < 0 || steps < 0) return fail(CROM_ERR_INVALID_ARG, "negative size");
  if (!(dx > 0.0) || !(dt >= 0.0)) return fail(CROM_ERR_INVALID_ARG, "dx must be positive, dt non-negative");
  const int64_t total = nx * ny * n_grid;
  if (total == 0 || steps == 0) return CROM_OK;
  if (!u || !scratch || !nu) return fail(CROM_ERR_INVALID_ARG, "u, scratch and nu are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double dx2 = dx * dx;
  const int threads = 256;
  int64_t blocks = (total + threads - 1) / threads;
  if (blocks > 65536) blocks = 65536;
  double* a = u;
  double* b = scratch;
  for (int64_t s = 0; s < steps; ++s) {
    if (dim == 1)
      hipLaunchKernelGGL(fd1d_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, a, b, nu,
                         nu_per_node, nx, n_grid, dt, dx2);
    else
      hipLaunchKernelGGL(fd2d_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, a, b, nu,
                         nu_per_node, nx, ny, n_grid, dt, dx2);
    double* t = a;
    a = b;
    b = t;
  }
  crom_status s = hip_check(hipGetLastError(), "fd launch");
  if (s != CROM_OK) return s;
  if (a != u) s = hip_check(hipMemcpyAsync(u, a, total * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  return s;
}

}  // extern "C"
