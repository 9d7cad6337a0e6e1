// Standardization of the training data and its fold into the trained
// networks (Sec. "Training Details": the training fields are mapped to zero
// mean and unit variance, the coordinates of the ELU networks are
// standardized too).  The moments are population moments; after training
// the affine maps are folded into the decoder's first and output layers and
// the encoder's first layer, so the latent step runs in physical units:
//   g(x, q) = u_std g_s((x - x_mean) / x_std, q) + u_mean,  e(u) = e_s((u - u_mean) / u_std).
// Everything here runs once per training run: the moments are one
// workgroup's fixed-order FP64 sums (deterministic), the rest elementwise.
#include "common.hpp"

namespace crom {

constexpr int STD_THREADS = 1024;

// Fixed-order sum of one value per thread over the workgroup (LDS tree).
__device__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = STD_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Mean and population deviation of n values x[i * stride] (two passes: the
// mean, then the mean squared deviation from it).
template <class T>
__device__ void moments(const T* __restrict__ x, int64_t n, int stride, double* sh, double* mean, double* dev) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += STD_THREADS) s += (double)x[i * stride];
  const double mu = block_sum(s, sh) / (double)n;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += STD_THREADS) {
    const double e = (double)x[i * stride] - mu;
    v += e * e;
  }
  const double var = block_sum(v, sh) / (double)n;
  if (threadIdx.x == 0) {
    *mean = mu;
    *dev = sqrt(var);
  }
}

__global__ __launch_bounds__(STD_THREADS) void moments_kernel(const double* __restrict__ u, int64_t n_u,
                                                              const float* __restrict__ x, int64_t P, int m,
                                                              crom_standardization* __restrict__ s) {
  __shared__ double sh[STD_THREADS];
  double mean, dev;
  moments(u, n_u, 1, sh, &mean, &dev);
  if (threadIdx.x == 0) {
    s->u_mean = mean;
    s->u_std = dev;
  }
  for (int k = 0; k < 3; ++k) {
    if (k < m) moments(x + k, P, m, sh, &mean, &dev);
    if (threadIdx.x == 0) {
      s->x_mean[k] = k < m ? mean : 0.0;
      s->x_std[k] = k < m ? dev : 1.0;
    }
  }
}

// u_s = (u - u_mean) / u_std and x_s = (x - x_mean) / x_std in FP64, rounded
// once to FP32.
__global__ __launch_bounds__(256) void standardize_kernel(const crom_standardization* __restrict__ s,
                                                          const double* __restrict__ u, int64_t n_u,
                                                          float* __restrict__ u_s, const float* __restrict__ x,
                                                          int64_t nx, int m, float* __restrict__ x_s) {
  const double um = s->u_mean, us = s->u_std;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_u; i += stride)
    u_s[i] = (float)((u[i] - um) / us);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += stride) {
    const int k = (int)(i % m);
    x_s[i] = (float)(((double)x[i] - s->x_mean[k]) / s->x_std[k]);
  }
}

// Decoder: layer 1's coordinate columns divide by x_std and its bias loses
// W1x (x_mean / x_std) (one thread per unit, the sum over the m axes in
// axis order); the output layer scales by u_std and shifts its bias by
// u_mean.
__global__ __launch_bounds__(256) void fold_decoder_kernel(float* __restrict__ prm, ParamIndex pi, int m, int r,
                                                           int width, int depth, int d,
                                                           const crom_standardization* __restrict__ s) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < width) {
    float* W1 = prm + pi.w[0] + (int64_t)t * (m + r);
    double shift = 0.0;
    for (int k = 0; k < m; ++k) shift += (double)W1[k] * (s->x_mean[k] / s->x_std[k]);
    prm[pi.b[0] + t] = (float)((double)prm[pi.b[0] + t] - shift);
    for (int k = 0; k < m; ++k) W1[k] = (float)((double)W1[k] / s->x_std[k]);
  }
  const int n_out = d * width;
  if (t < n_out) {
    float* Wo = prm + pi.w[depth];
    Wo[t] = (float)((double)Wo[t] * s->u_std);
  }
  if (t < d) {
    float* bo = prm + pi.b[depth];
    bo[t] = (float)((double)bo[t] * s->u_std + s->u_mean);
  }
}

// Encoder's first layer (dense E1 [rows][cols], or the first convolution
// W [d][d][6] with rows = d, cols = 6 d): one workgroup per output row sums
// the row's weights in a fixed order (FP64), its bias loses
// (u_mean / u_std) times that sum, and the weights divide by u_std.
__global__ __launch_bounds__(STD_THREADS) void fold_encoder_kernel(float* __restrict__ W, float* __restrict__ c,
                                                                   int64_t cols,
                                                                   const crom_standardization* __restrict__ s) {
  __shared__ double sh[STD_THREADS];
  float* row = W + (int64_t)blockIdx.x * cols;
  double v = 0.0;
  for (int64_t j = threadIdx.x; j < cols; j += STD_THREADS) v += (double)row[j];
  const double sum = block_sum(v, sh);
  const double um = s->u_mean, us = s->u_std;
  for (int64_t j = threadIdx.x; j < cols; j += STD_THREADS) row[j] = (float)((double)row[j] / us);
  if (threadIdx.x == 0) c[blockIdx.x] = (float)((double)c[blockIdx.x] - (um / us) * sum);
}

static unsigned grid_of(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (unsigned)b;
}

}  // namespace crom

using namespace crom;

extern "C" {

crom_status crom_standardization_of(const double* u, int64_t n_u, const float* x, int64_t P, int32_t m,
                                    crom_standardization* s, void* stream) {
  if (!u || !x || !s) return fail(CROM_ERR_INVALID_ARG, "u, x and s are required");
  if (n_u < 1 || P < 1) return fail(CROM_ERR_INVALID_ARG, "n_u >= 1 and P >= 1 are required");
  if (m < 1 || m > 3) return fail(CROM_ERR_INVALID_ARG, "m must be 1, 2 or 3");
  hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(STD_THREADS), 0, static_cast<hipStream_t>(stream), u, n_u, x, P,
                     (int)m, s);
  return hip_check(hipGetLastError(), "moments launch");
}

crom_status crom_standardize(const crom_standardization* s, const double* u, int64_t n_u, float* u_s,
                             const float* x, int64_t P, int32_t m, float* x_s, void* stream) {
  if (!s) return fail(CROM_ERR_INVALID_ARG, "s is required");
  if (n_u < 0 || P < 0) return fail(CROM_ERR_INVALID_ARG, "n_u >= 0 and P >= 0 are required");
  if (n_u > 0 && (!u || !u_s)) return fail(CROM_ERR_INVALID_ARG, "u and u_s are required when n_u > 0");
  if (P > 0 && (!x || !x_s || m < 1 || m > 3))
    return fail(CROM_ERR_INVALID_ARG, "x, x_s and m in 1..3 are required when P > 0");
  if (n_u == 0 && P == 0) return CROM_OK;
  const int64_t nx = P * (m > 0 ? m : 1);
  hipLaunchKernelGGL(standardize_kernel, dim3(grid_of(n_u > nx ? n_u : nx)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), s, u, n_u, u_s, x, P > 0 ? nx : 0, m > 0 ? (int)m : 1, x_s);
  return hip_check(hipGetLastError(), "standardize launch");
}

crom_status crom_fold_standardization(const crom_net* net, const crom_encoder* enc, const crom_standardization* s,
                                      void* stream) {
  crom_status st = check_net(net, false);
  if (st != CROM_OK) return st;
  if (!s) return fail(CROM_ERR_INVALID_ARG, "s is required");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const ParamIndex pi = param_index(net->m, net->r, net->d, net->width, net->depth);
  float* prm = const_cast<float*>(net->params);
  const int n = net->width > net->d * net->width ? net->width : net->d * net->width;
  hipLaunchKernelGGL(fold_decoder_kernel, dim3((n + 255) / 256), dim3(256), 0, hs, prm, pi, net->m, net->r,
                     net->width, net->depth, net->d, s);
  if ((st = hip_check(hipGetLastError(), "fold decoder launch")) != CROM_OK) return st;
  if (!enc) return CROM_OK;
  if (!enc->params) return fail(CROM_ERR_INVALID_ARG, "enc->params is NULL");
  int64_t rows, cols;
  float* W = enc->params;
  if (enc->kind == CROM_ENC_CONV) {
    if (crom_conv_encoder_param_count(enc->n_in / net->d, net->d, enc->hidden, enc->r) == 0)
      return fail(CROM_ERR_INVALID_ARG, "invalid convolutional encoder sizes");
    rows = net->d;
    cols = 6 * (int64_t)net->d;
  } else if (enc->kind == CROM_ENC_DENSE) {
    if (crom_encoder_param_count(enc->n_in, enc->hidden, enc->r) == 0)
      return fail(CROM_ERR_INVALID_ARG, "invalid dense encoder sizes");
    rows = enc->hidden;
    cols = enc->n_in;
  } else {
    return fail(CROM_ERR_UNSUPPORTED, "unknown encoder kind");
  }
  hipLaunchKernelGGL(fold_encoder_kernel, dim3((unsigned)rows), dim3(STD_THREADS), 0, hs, W, W + rows * cols, cols,
                     s);
  return hip_check(hipGetLastError(), "fold encoder launch");
}

}  // extern "C"
