// Encoder-based initial guess for the heat step (Sec. "Initial Guess for the
// Nonlinear Solver"): the training encoder applied to the updated field at
// every node, f = g(x, q_n) + dt nu Laplacian g(x, q_n), which needs the
// decoder and its Laplacian over the whole node set, not only the samples.
#include "common.hpp"

namespace crom {

// f[i][p] = g[i][p] + dt nu_i lap[i][p] (FP64 arithmetic, FP32 result: the
// encoder's input type).
__global__ __launch_bounds__(256) void heat_field_kernel(const float* __restrict__ g, const float* __restrict__ lap,
                                                        const double* __restrict__ nu, double dt, int64_t P,
                                                        int64_t n, float* __restrict__ f) {
  const int64_t total = n * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    f[e] = (float)((double)g[e] + dt * nu[e / P] * (double)lap[e]);
}

__global__ __launch_bounds__(64) void widen_kernel(const float* __restrict__ x, int64_t n, double* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (double)x[e];
}

struct GuessLayout {
  size_t g, lap, f, q, enc, total;
};

static inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

static GuessLayout guess_layout(int32_t n_inst, int64_t P, int r, size_t enc_bytes) {
  GuessLayout L{};
  size_t o = 0;
  L.g = o;   o = al256(o + 4 * (size_t)n_inst * P);
  L.lap = o; o = al256(o + 4 * (size_t)n_inst * P);
  L.f = o;   o = al256(o + 4 * (size_t)n_inst * P);
  L.q = o;   o = al256(o + 4 * (size_t)n_inst * r);
  L.enc = o; o = al256(o + enc_bytes);
  L.total = o + 256;  // room to align the caller's pointer
  return L;
}

static crom_status guess_check(const crom_net* net, const crom_encoder* enc, int32_t n_inst, int64_t P,
                               size_t* enc_bytes) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (!enc) return fail(CROM_ERR_INVALID_ARG, "enc is NULL");
  if (net->d != 1) return fail(CROM_ERR_UNSUPPORTED, "the heat guess needs d == 1");
  if (net->m > 2) return fail(CROM_ERR_UNSUPPORTED, "the heat guess needs m <= 2");
  if (n_inst < 1 || P < 1) return fail(CROM_ERR_INVALID_ARG, "n_inst >= 1 and P >= 1 are required");
  if ((int64_t)enc->n_in != P * net->d || enc->r != net->r)
    return fail(CROM_ERR_INVALID_ARG, "the encoder must take P * d inputs and give r latents");
  return crom_encode_workspace(net, enc, n_inst, enc_bytes);
}

}  // namespace crom

using namespace crom;

extern "C" {

crom_status crom_heat_guess_workspace(const crom_net* net, const crom_encoder* enc, int32_t n_inst, int64_t P,
                                      size_t* bytes) {
  if (!bytes) return fail(CROM_ERR_INVALID_ARG, "bytes is NULL");
  size_t eb = 0;
  crom_status s = guess_check(net, enc, n_inst, P, &eb);
  if (s != CROM_OK) return s;
  *bytes = guess_layout(n_inst, P, net->r, eb).total;
  return CROM_OK;
}

crom_status crom_heat_guess(const crom_net* net, const crom_encoder* enc, const float* nodes, int64_t P,
                            int32_t n_inst, const double* q_n, const double* nu, double dt, double* q_guess,
                            void* ws, size_t ws_bytes, void* stream) {
  size_t eb = 0;
  crom_status s = guess_check(net, enc, n_inst, P, &eb);
  if (s != CROM_OK) return s;
  if (!nodes || !q_n || !nu || !q_guess || !ws) return fail(CROM_ERR_INVALID_ARG, "nodes, q_n, nu, q_guess and ws are required");
  const GuessLayout L = guess_layout(n_inst, P, net->r, eb);
  if (ws_bytes < L.total) return fail(CROM_ERR_WORKSPACE, "workspace too small");
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  float* g = reinterpret_cast<float*>(base + L.g);
  float* lap = reinterpret_cast<float*>(base + L.lap);
  float* f = reinterpret_cast<float*>(base + L.f);
  float* qf = reinterpret_cast<float*>(base + L.q);
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int32_t i = 0; i < n_inst; ++i) {
    s = crom_decode_jac_x(net, nodes, P, q_n + (int64_t)i * net->r, CROM_D2_LAPLACIAN, g + (int64_t)i * P, nullptr,
                          lap + (int64_t)i * P, stream);
    if (s != CROM_OK) return s;
  }
  int64_t blocks = (n_inst * P + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(heat_field_kernel, dim3((unsigned)blocks), dim3(256), 0, st, g, lap, nu, dt, P, (int64_t)n_inst, f);
  if ((s = hip_check(hipGetLastError(), "heat field launch")) != CROM_OK) return s;
  if ((s = crom_encode(net, enc, f, n_inst, qf, base + L.enc, eb, stream)) != CROM_OK) return s;
  hipLaunchKernelGGL(widen_kernel, dim3(1), dim3(64), 0, st, qf, (int64_t)n_inst * net->r, q_guess);
  return hip_check(hipGetLastError(), "widen launch");
}

}  // extern "C"
