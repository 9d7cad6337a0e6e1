// Full-order fallback for heat instances whose latent step failed (Sec.
// "Thermodynamics / Full-order Model", "Image Processing / Full-order
// Model": the finite-difference solver the reduced model stands in for).
// A failed step (singular normal equations, non-finite values, no
// acceptable line-search step) leaves q at the last good latent.  The
// fallback decodes that latent at every node of the full-order grid,
// advances the field with the FP64 solver over the time step, and projects
// the result back onto the decoder by the method's own inversion at every
// node (Sec. "Network Inversion"), so the rollout continues on the manifold
// from the full-order update.  The projection uses all nodes, not the
// instance's samples: a failed instance's samples may be what made its
// normal equations singular.
#include "common.hpp"

namespace crom {

// u[k][p] = g[k][p] (FP32 -> FP64), nu_g[k] = nu[inst[k]], q_g[k] = q_last[inst[k]].
__global__ __launch_bounds__(256) void fb_gather_kernel(const float* __restrict__ g, int64_t n, int64_t P, int r,
                                                        const int32_t* __restrict__ inst,
                                                        const double* __restrict__ nu,
                                                        const double* __restrict__ q_last, double* __restrict__ u,
                                                        double* __restrict__ nu_g, double* __restrict__ q_g) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = t0; e < n * P; e += stride) u[e] = (double)g[e];
  for (int64_t k = t0; k < n; k += stride) nu_g[k] = nu[inst[k]];
  for (int64_t e = t0; e < n * r; e += stride) q_g[e] = q_last[(int64_t)inst[e / r] * r + e % r];
}

// The projection's batch: every failed instance takes all P nodes.
__global__ __launch_bounds__(256) void fb_layout_kernel(const float* __restrict__ nodes, int64_t n, int64_t P,
                                                        float* __restrict__ y, int64_t* __restrict__ offsets) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = t0; e < n * P * 2; e += stride) y[e] = nodes[e % (P * 2)];
  for (int64_t k = t0; k <= n; k += stride) offsets[k] = k * P;
}

// q_next[inst[k]] = q_p[k], info[inst[k]] = info_p[k].
__global__ __launch_bounds__(64) void fb_scatter_kernel(const double* __restrict__ q_p,
                                                        const crom_step_info* __restrict__ info_p, int64_t n, int r,
                                                        const int32_t* __restrict__ inst, double* __restrict__ q_next,
                                                        crom_step_info* __restrict__ info) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * r; e += (int64_t)gridDim.x * blockDim.x) {
    q_next[(int64_t)inst[e / r] * r + e % r] = q_p[e];
    if (info && e % r == 0) info[inst[e / r]] = info_p[e / r];
  }
}

struct FallbackLayout {
  size_t inst, g, u, scratch, nu, q_g, q_p, info, y, offsets, step, step_bytes, total;
};

static inline size_t fb_al(size_t x) { return (x + 255) & ~size_t(255); }

static crom_status fb_layout(const crom_net* net, int32_t n, int64_t P, FallbackLayout* L) {
  size_t step_bytes = 0;
  crom_status s = crom_step_workspace(net, n, (int64_t)n * P, &step_bytes);
  if (s != CROM_OK) return s;
  size_t o = 0;
  L->inst = o;    o = fb_al(o + 4 * (size_t)n);
  L->g = o;       o = fb_al(o + 4 * (size_t)n * P);
  L->u = o;       o = fb_al(o + 8 * (size_t)n * P);
  L->scratch = o; o = fb_al(o + 8 * (size_t)n * P);
  L->nu = o;      o = fb_al(o + 8 * (size_t)n);
  L->q_g = o;     o = fb_al(o + 8 * (size_t)n * net->r);
  L->q_p = o;     o = fb_al(o + 8 * (size_t)n * net->r);
  L->info = o;    o = fb_al(o + sizeof(crom_step_info) * (size_t)n);
  L->y = o;       o = fb_al(o + 8 * (size_t)n * P);
  L->offsets = o; o = fb_al(o + 8 * ((size_t)n + 1));
  L->step = o;    o = fb_al(o + step_bytes);
  L->step_bytes = step_bytes;
  L->total = o + 256;  // room to align the caller's pointer
  return CROM_OK;
}

static crom_status fb_check(const crom_net* net, int32_t n_fail, int64_t nx, int64_t ny) {
  crom_status s = check_net(net, true);
  if (s != CROM_OK) return s;
  if (net->d != 1 || net->m != 2) return fail(CROM_ERR_UNSUPPORTED, "the heat fallback needs m == 2 and d == 1");
  if (n_fail < 1 || nx < 3 || ny < 3) return fail(CROM_ERR_INVALID_ARG, "n_fail >= 1 and a grid of at least 3 x 3");
  return CROM_OK;
}

static unsigned fb_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace crom

using namespace crom;

extern "C" {

crom_status crom_heat_fallback_workspace(const crom_net* net, int32_t n_fail, int64_t nx, int64_t ny, size_t* bytes) {
  if (!bytes) return fail(CROM_ERR_INVALID_ARG, "bytes is NULL");
  crom_status s = fb_check(net, n_fail, nx, ny);
  if (s != CROM_OK) return s;
  FallbackLayout L;
  if ((s = fb_layout(net, n_fail, nx * ny, &L)) != CROM_OK) return s;
  *bytes = L.total;
  return CROM_OK;
}

crom_status crom_heat_fallback(const crom_net* net, const float* nodes, int64_t nx, int64_t ny, double dx,
                               int32_t n_inst, int32_t n_fail, const int32_t* inst, const double* q_last,
                               const double* nu, double dt_fd, int64_t substeps, const crom_gn_opts* opts,
                               double* q_next, crom_step_info* info, void* ws, size_t ws_bytes, void* stream) {
  crom_status s = fb_check(net, n_fail, nx, ny);
  if (s != CROM_OK) return s;
  if (!nodes || !inst || !q_last || !nu || !q_next || !opts || !ws)
    return fail(CROM_ERR_INVALID_ARG, "nodes, inst, q_last, nu, q_next, opts and ws are required");
  if (!(dx > 0.0) || !(dt_fd > 0.0) || substeps < 0) return fail(CROM_ERR_INVALID_ARG, "dx, dt_fd > 0, substeps >= 0");
  for (int32_t k = 0; k < n_fail; ++k) {
    if (inst[k] < 0 || inst[k] >= n_inst) return fail(CROM_ERR_INVALID_ARG, "instance index out of range");
    for (int32_t j = 0; j < k; ++j)
      if (inst[j] == inst[k]) return fail(CROM_ERR_INVALID_ARG, "repeated instance index");
  }
  const int64_t P = nx * ny;
  FallbackLayout L;
  if ((s = fb_layout(net, n_fail, P, &L)) != CROM_OK) return s;
  if (ws_bytes < L.total) return fail(CROM_ERR_WORKSPACE, "workspace too small");
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  int32_t* d_inst = reinterpret_cast<int32_t*>(base + L.inst);
  float* g = reinterpret_cast<float*>(base + L.g);
  double* u = reinterpret_cast<double*>(base + L.u);
  double* scratch = reinterpret_cast<double*>(base + L.scratch);
  double* nu_g = reinterpret_cast<double*>(base + L.nu);
  double* q_g = reinterpret_cast<double*>(base + L.q_g);
  double* q_p = reinterpret_cast<double*>(base + L.q_p);
  crom_step_info* info_p = reinterpret_cast<crom_step_info*>(base + L.info);
  float* y = reinterpret_cast<float*>(base + L.y);
  int64_t* offsets = reinterpret_cast<int64_t*>(base + L.offsets);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the host list of instances travels with the stream's work
  if ((s = hip_check(hipMemcpyAsync(d_inst, inst, sizeof(int32_t) * n_fail, hipMemcpyHostToDevice, st),
                     "instance list copy")) != CROM_OK)
    return s;
  for (int32_t k = 0; k < n_fail; ++k) {
    s = crom_decode(net, nodes, P, q_last + (int64_t)inst[k] * net->r, g + (int64_t)k * P, stream);
    if (s != CROM_OK) return s;
  }
  hipLaunchKernelGGL(fb_gather_kernel, dim3(fb_grid((int64_t)n_fail * P)), dim3(256), 0, st, g, (int64_t)n_fail, P,
                     (int)net->r, d_inst, nu, q_last, u, nu_g, q_g);
  if ((s = hip_check(hipGetLastError(), "fallback gather launch")) != CROM_OK) return s;
  const int64_t shape[2] = {nx, ny};
  if ((s = crom_fd_heat(2, shape, n_fail, nu_g, 0, dx, dt_fd, substeps, u, scratch, stream)) != CROM_OK) return s;
  hipLaunchKernelGGL(fb_layout_kernel, dim3(fb_grid((int64_t)n_fail * P * 2)), dim3(256), 0, st, nodes,
                     (int64_t)n_fail, P, y, offsets);
  if ((s = hip_check(hipGetLastError(), "fallback layout launch")) != CROM_OK) return s;
  // the full-order fields are the targets of an inversion at every node
  crom_pde pde{};
  pde.kind = CROM_PDE_PROJECT;
  pde.coef = u;
  s = crom_step(net, &pde, n_fail, offsets, (int64_t)n_fail * P, y, nullptr, nullptr, q_g, q_p, opts, info_p,
                base + L.step, L.step_bytes, stream);
  if (s != CROM_OK) return s;
  hipLaunchKernelGGL(fb_scatter_kernel, dim3(1), dim3(64), 0, st, q_p, info_p, (int64_t)n_fail, (int)net->r, d_inst,
                     q_next, info);
  return hip_check(hipGetLastError(), "fallback scatter launch");
}

}  // extern "C"
