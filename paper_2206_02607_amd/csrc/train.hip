// Training of the manifold parameterisation (Sec. "Manifold Construction",
// eq. "loss"; Sec. "Training Details"): encoder q_b = E2 ELU(E1 u_b + c1) + c2,
// decoder g(x_p, q_b) at every point of every snapshot of the batch, loss =
// mean (g - u)^2, gradients by the reverse-mode chain rule written out layer
// by layer, and Adam with bias correction on FP32 master parameters.
//
// The decoder's rows are (snapshot, point) pairs, snapshot-major: row
// b * P + p.  Layer activations a_l = ELU(z_l) are kept for the backward
// pass (ELU'(z) is recovered from a: 1 where a > 0, a + 1 otherwise).  The
// matrix products run on the matrix cores through gemm.hpp, in bfloat16 with
// FP32 accumulation (FP32 when the net's precision is FP32); the first layer
// (K = m + r), the output layer and every reduction over rows are plain
// FP32 kernels with a fixed summation order.
#include "common.hpp"
#include "gemm.hpp"

namespace crom {

constexpr int MAX_SPLITS = 256;  // split-K partial tiles at most

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
template <class T>
__global__ void convert_kernel(const float* __restrict__ a, T* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (T)a[i];
}

// c[b][u] = b1[u] + sum_k W1[u][m + k] q[b][k]  (FP64 accumulation)
__global__ void fold_kernel(const float* __restrict__ W1, const float* __restrict__ b1, const float* __restrict__ q,
                            int B, int W, int m, int r, float* __restrict__ c) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B * W; i += gridDim.x * blockDim.x) {
    const int b = i / W, u = i % W;
    double s = b1[u];
    for (int k = 0; k < r; ++k) s += (double)W1[u * (m + r) + m + k] * q[b * r + k];
    c[i] = (float)s;
  }
}

// a1[row][u] = ELU(sum_i W1[u][i] x[p][i] + c[b][u]),  row = b * P + p.
// A thread takes 8 consecutive units of one row (W is a multiple of 8); the
// x-columns of W1 are staged in LDS, and every load of a thread is issued
// before its arithmetic (m is a compile-time constant).
constexpr int EW_MAX_W = 256;  // widest layer of the compiled shapes
constexpr int EW_MAX_MD = 3;   // largest m and d

// Sine networks (SINE): a1 = sin(z), and g1 = cos(z) for the backward.
template <class T, int M, bool SINE = false>
__global__ __launch_bounds__(256) void layer1_kernel(const float* __restrict__ W1, const float* __restrict__ c,
                                                     const float* __restrict__ x, int64_t P, int64_t rows, int W,
                                                     int r, T* __restrict__ a1, T* __restrict__ g1) {
  typedef T vec8 __attribute__((ext_vector_type(8)));
  __shared__ float wx[EW_MAX_W * M];
  for (int i = threadIdx.x; i < W * M; i += blockDim.x) wx[i] = W1[(i / M) * (M + r) + i % M];
  __syncthreads();
  const int G = W / 8;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows * G; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / G;
    const int u0 = (int)(i - row * G) * 8;
    const int64_t b = row / P, p = row - b * P;
    float xv[M];
#pragma unroll
    for (int k = 0; k < M; ++k) xv[k] = x[p * M + k];
    const float4 c0 = *reinterpret_cast<const float4*>(&c[b * W + u0]);
    const float4 c1 = *reinterpret_cast<const float4*>(&c[b * W + u0 + 4]);
    const float cz[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    vec8 o, oc;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float z = cz[e];
#pragma unroll
      for (int k = 0; k < M; ++k) z += wx[(u0 + e) * M + k] * xv[k];
      if constexpr (SINE) {
        const float rz = reduce_2pi(z);
        o[e] = (T)__sinf(rz);
        oc[e] = (T)__cosf(rz);
      } else {
        o[e] = (T)(z > 0.0f ? z : __expf(z) - 1.0f);
      }
    }
    *reinterpret_cast<vec8*>(&a1[row * W + u0]) = o;
    if constexpr (SINE) *reinterpret_cast<vec8*>(&g1[row * W + u0]) = oc;
  }
}

// g[row][o] = sum_u Wout[o][u] a[row][u] + bout[o]: one thread per row,
// 8 units per load, in unit order; Wout staged in LDS.
template <class T, int D>
__global__ __launch_bounds__(256) void output_kernel(const T* __restrict__ a, const float* __restrict__ Wout,
                                                     const float* __restrict__ bout, int64_t rows, int W,
                                                     float* __restrict__ g) {
  typedef T vec8 __attribute__((ext_vector_type(8)));
  __shared__ float wo[EW_MAX_W * D];
  for (int i = threadIdx.x; i < W * D; i += blockDim.x) wo[i] = Wout[i];
  __syncthreads();
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    float s[D];
#pragma unroll
    for (int o = 0; o < D; ++o) s[o] = 0.0f;
    for (int u0 = 0; u0 < W; u0 += 8) {
      const vec8 v = *reinterpret_cast<const vec8*>(&a[row * W + u0]);
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int o = 0; o < D; ++o) s[o] += wo[o * W + u0 + e] * (float)v[e];
    }
#pragma unroll
    for (int o = 0; o < D; ++o) g[row * D + o] = s[o] + bout[o];
  }
}

// dg = 2 (g - u) / n and per-block partial sums of (g - u)^2
__global__ void mse_kernel(const float* __restrict__ g, const float* __restrict__ u, int64_t n,
                           float* __restrict__ dg, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float e = g[i] - u[i];
    dg[i] = 2.0f * e / (float)n;
    s += (double)e * e;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// loss = sum of the block partials / n: each thread adds a strided quarter
// of them, then a fixed-order tree.
__global__ __launch_bounds__(256) void mse_final_kernel(const double* __restrict__ part, int nb, int64_t n,
                                                         float* loss) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(sh[0] / (double)n);
}

// dz[row][u] = (sum_o dg[row][o] Wout[o][u]) * ELU'(a[row][u]); 8 units
// of one row per thread, Wout staged in LDS.
// Sine networks (SINE): `a` holds the stored cos(z) and scales dz directly.
template <class T, int D, bool SINE = false>
__global__ __launch_bounds__(256) void dz_last_kernel(const float* __restrict__ dg, const float* __restrict__ Wout,
                                                      const T* __restrict__ a, int64_t rows, int W,
                                                      T* __restrict__ dz) {
  typedef T vec8 __attribute__((ext_vector_type(8)));
  __shared__ float wo[EW_MAX_W * D];
  for (int i = threadIdx.x; i < W * D; i += blockDim.x) wo[i] = Wout[i];
  __syncthreads();
  const int G = W / 8;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows * G; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / G;
    const int u0 = (int)(i - row * G) * 8;
    float d[D];
#pragma unroll
    for (int o = 0; o < D; ++o) d[o] = dg[row * D + o];
    const vec8 av = *reinterpret_cast<const vec8*>(&a[row * W + u0]);
    vec8 out;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float s = 0.0f;
#pragma unroll
      for (int o = 0; o < D; ++o) s += d[o] * wo[o * W + u0 + e];
      out[e] = (T)(SINE ? s * (float)av[e] : s * elu_d1_from_a((float)av[e]));
    }
    *reinterpret_cast<vec8*>(&dz[row * W + u0]) = out;
  }
}

// Weighted column sums over row segments, in two fixed-order passes.
//   out[seg][k][col] = sum over rows of the segment of w_k(row) X[row][col]
// with w_0 = 1 and w_k = wt[(row % wmod) * wstride + k - 1] (k = 1..nw-1).
// Pass 1: block (chunk, seg) sums `chunk_rows` rows of its segment.  Its
// threads split into row groups; a thread adds the rows of its group for
// VEC consecutive columns (VEC = 16 bytes of X when the rows are aligned,
// else 1), in FP32, then the groups are added in group order in FP64.
// Pass 2 adds the chunks in a fixed order.
template <class T, int VEC>
__global__ __launch_bounds__(256) void colsum_kernel(const T* __restrict__ X, int64_t ldx, int cols,
                                                     int64_t seg_rows, int chunk_rows,
                                                     const float* __restrict__ wt, int64_t wmod, int wstride,
                                                     int nw, double* __restrict__ part) {
  __shared__ double sh[4][256];
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  const int ch = blockIdx.x, seg = blockIdx.y, chunks = gridDim.x;
  const int64_t r0 = (int64_t)ch * chunk_rows;
  const int64_t r1 = min(seg_rows, r0 + chunk_rows);
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < cols; c0 += 256 * VEC) {
    const int cw = min(256 * VEC, cols - c0);       // columns of this pass
    const int tpr = (cw + VEC - 1) / VEC;           // threads per row
    const int G = 256 / tpr;                        // row groups
    const int cv = tid % tpr, rg = tid / tpr;
    const int col = c0 + cv * VEC;
    float s[4][VEC];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int e = 0; e < VEC; ++e) s[k][e] = 0.0f;
    if (rg < G) {
#pragma unroll 4
      for (int64_t r = r0 + rg; r < r1; r += G) {
        const int64_t row = seg * seg_rows + r;
        float v[VEC];
        if constexpr (VEC > 1) {
          const vec_t x = *reinterpret_cast<const vec_t*>(&X[row * ldx + col]);
#pragma unroll
          for (int e = 0; e < VEC; ++e) v[e] = (float)x[e];
        } else {
          v[0] = (float)X[row * ldx + col];
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) s[0][e] += v[e];
        for (int k = 1; k < nw; ++k) {
          const float w = wt[(row % wmod) * wstride + (k - 1)];
#pragma unroll
          for (int e = 0; e < VEC; ++e) s[k][e] += v[e] * w;
        }
      }
    }
    for (int e = 0; e < VEC; ++e) {
      for (int k = 0; k < nw; ++k) sh[k][tid] = rg < G ? (double)s[k][e] : 0.0;
      __syncthreads();
      if (tid < tpr && c0 + tid * VEC + e < cols) {
        for (int k = 0; k < nw; ++k) {
          double a = 0.0;
          for (int q = 0; q < G; ++q) a += sh[k][q * tpr + tid];
          part[(((int64_t)seg * chunks + ch) * nw + k) * cols + c0 + tid * VEC + e] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Pass 2: out[seg][k][col] = sum over chunks, in chunk order within each of
// 4 interleaved lanes, then the 4 lanes in order.
__global__ __launch_bounds__(256) void colsum_final_kernel(const double* __restrict__ part, int segs, int chunks,
                                                           int nw, int cols, double* __restrict__ out) {
  __shared__ double sh[4][64];
  const int n_out = nw * cols;
  const int o = blockIdx.x * 64 + (threadIdx.x & 63), lane4 = threadIdx.x >> 6, seg = blockIdx.y;
  double a = 0.0;
  if (o < n_out) {
#pragma unroll 8
    for (int c = lane4; c < chunks; c += 4) a += part[((int64_t)seg * chunks + c) * n_out + o];
  }
  sh[lane4][threadIdx.x & 63] = a;
  __syncthreads();
  if (threadIdx.x < 64 && o < n_out)
    out[(int64_t)seg * n_out + o] = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

// Column sums of X [segs * seg_rows][cols] (leading dimension ldx) per
// segment, weighted as in colsum_kernel, into out [segs][nw][cols] (FP64).
template <class T>
static void colsum(const T* X, int64_t ldx, int cols, int segs, int64_t seg_rows, const float* wt, int64_t wmod,
                   int wstride, int nw, double* part, int max_chunks, double* out, hipStream_t st) {
  int chunks = (int)((seg_rows + 255) / 256);
  const int cap = max(1, max_chunks / segs);
  if (chunks > cap) chunks = cap;
  if (chunks < 1) chunks = 1;
  const int chunk_rows = (int)((seg_rows + chunks - 1) / chunks);
  constexpr int VEC = 16 / (int)sizeof(T);
  if (cols % VEC == 0 && ldx % VEC == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0)
    hipLaunchKernelGGL((colsum_kernel<T, VEC>), dim3(chunks, segs), dim3(256), 0, st, X, ldx, cols, seg_rows,
                       chunk_rows, wt, wmod, wstride, nw, part);
  else
    hipLaunchKernelGGL((colsum_kernel<T, 1>), dim3(chunks, segs), dim3(256), 0, st, X, ldx, cols, seg_rows,
                       chunk_rows, wt, wmod, wstride, nw, part);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((nw * cols + 63) / 64, segs), dim3(256), 0, st, part, segs, chunks,
                     nw, cols, out);
}

// First-layer gradients from the per-snapshot sums S[b][0][u] = sum_p dz1,
// S[b][1 + i][u] = sum_p dz1 x_p[i] (i < m):
//   dW1[u][i] = sum_b S[b][1+i][u]; dW1[u][m+k] = sum_b S[b][0][u] q[b][k];
//   db1[u] = sum_b S[b][0][u];  dq[b][k] = sum_u S[b][0][u] W1[u][m+k]
__global__ void layer1_grad_kernel(const double* __restrict__ S, const float* __restrict__ q, const float* __restrict__ W1,
                                   int B, int W, int m, int r, float* __restrict__ dW1, float* __restrict__ db1,
                                   float* __restrict__ dq) {
  const int nw = 1 + m;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < W * (m + r) + W + B * r; i += gridDim.x * blockDim.x) {
    if (i < W * (m + r)) {
      const int u = i / (m + r), k = i % (m + r);
      double s = 0.0;
      for (int b = 0; b < B; ++b)
        s += k < m ? S[((int64_t)b * nw + 1 + k) * W + u] : S[((int64_t)b * nw) * W + u] * (double)q[b * r + (k - m)];
      dW1[i] = (float)s;
    } else if (i < W * (m + r) + W) {
      const int u = i - W * (m + r);
      double s = 0.0;
      for (int b = 0; b < B; ++b) s += S[((int64_t)b * nw) * W + u];
      db1[u] = (float)s;
    } else {
      const int j = i - W * (m + r) - W, b = j / r, k = j % r;
      double s = 0.0;
      for (int u = 0; u < W; ++u) s += S[((int64_t)b * nw) * W + u] * (double)W1[u * (m + r) + m + k];
      dq[j] = (float)s;
    }
  }
}

__global__ void d2f_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// Adam with bias correction (Kingma & Ba), FP32 state.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------------------
// host-side plumbing
// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t n, int threads = 256) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

// The square hidden-layer products in bfloat16 at widths whose weights fit
// a wave's registers go through rowgemm_kernel; returns false otherwise.
template <bool FWD>
static bool row_gemm(int W, const void* X, const void* Wt, const float* bias, const void* gate, void* C,
                     int64_t rows, hipStream_t st, crom_status* s, bool sine = false, void* G = nullptr) {
  RowGemmArgs g{static_cast<const __bf16*>(X), static_cast<const __bf16*>(Wt), bias,
                static_cast<const __bf16*>(gate), static_cast<__bf16*>(C), rows, static_cast<__bf16*>(G)};
  const int64_t tiles = (rows + 15) / 16;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks > 1024) blocks = 1024;  // four workgroups of four waves per CU, looping over row tiles
  if (blocks < 1) blocks = 1;
  if (W == 128 && sine) hipLaunchKernelGGL((rowgemm_kernel<128, FWD, true>), dim3((unsigned)blocks), dim3(256), 0, st, g);
  else if (W == 32 && sine) hipLaunchKernelGGL((rowgemm_kernel<32, FWD, true>), dim3((unsigned)blocks), dim3(256), 0, st, g);
  else if (W == 128) hipLaunchKernelGGL((rowgemm_kernel<128, FWD>), dim3((unsigned)blocks), dim3(256), 0, st, g);
  else if (W == 32) hipLaunchKernelGGL((rowgemm_kernel<32, FWD>), dim3((unsigned)blocks), dim3(256), 0, st, g);
  else return false;
  *s = hip_check(hipGetLastError(), "row gemm launch");
  return true;
}

// dW = X^T Y over `rows` rows for the 128-wide hidden layers in bfloat16:
// wgrad_kernel partials (at most MAX_SPLITS workgroups), then their sum in
// workgroup order.  Returns false for other widths.
static bool wgrad(int W, const void* X, const void* Y, int64_t rows, float* part, float* dW, hipStream_t st,
                  crom_status* s) {
  if (W != 128) return false;
  constexpr int KS = 32;
  int64_t nblk = (rows + KS - 1) / KS;
  if (nblk > MAX_SPLITS) nblk = MAX_SPLITS;
  if (nblk < 1) nblk = 1;
  int64_t per = (rows + nblk - 1) / nblk;
  per = (per + KS - 1) / KS * KS;
  nblk = per > 0 ? (rows + per - 1) / per : 1;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL((wgrad_kernel<128>), dim3((unsigned)nblk), dim3(256), 0, st, static_cast<const __bf16*>(X),
                     static_cast<const __bf16*>(Y), rows, per, part);
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((W * W + 63) / 64)), dim3(256), 0, st, part, (int)nblk,
                     W, W, dW, (int64_t)W, 0, (int)EPI_NONE, nullptr);
  *s = hip_check(hipGetLastError(), "weight gradient launch");
  return true;
}

template <class T, bool TA, bool TB, int EPI>
static crom_status gemm(GemmArgs g, hipStream_t st) {
  constexpr int BK = sizeof(T) == 2 ? 64 : 32;  // the kernel's K tile
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, 1);
  if (g.part) {
    // split K so that there are a few hundred blocks
    const int64_t tiles = (int64_t)grid.x * grid.y;
    int splits = (int)((1024 + tiles - 1) / tiles);
    const int maxs = (g.K + BK - 1) / BK;
    if (splits > maxs) splits = maxs;
    if (splits > MAX_SPLITS) splits = MAX_SPLITS;
    if (splits < 1) splits = 1;
    int kc = (g.K + splits - 1) / splits;
    kc = (kc + BK - 1) / BK * BK;
    splits = (g.K + kc - 1) / kc;
    g.kchunk = kc;
    grid.z = splits;
    if (EPI == EPI_DELU) return fail(CROM_ERR_INVALID_ARG, "split-K carries no gate");
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, EPI_NONE>), grid, dim3(256), 0, st, g);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)(((int64_t)g.M * g.N + 63) / 64)), dim3(256), 0, st,
                       g.part, splits, g.M, g.N, g.C, g.ldc, g.accumulate, EPI, g.bias);
  } else {
    g.kchunk = g.K;
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, EPI>), grid, dim3(256), 0, st, g);
  }
  return hip_check(hipGetLastError(), "gemm launch");
}

static GemmArgs gemm_args(int M, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  return g;
}

// Workspace carving (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t off;
  template <class U>
  U* take(size_t count) {
    U* p = reinterpret_cast<U*>(base ? base + off : nullptr);
    off = (off + count * sizeof(U) + 255) & ~size_t(255);
    return p;
  }
};

constexpr int COLSUM_CHUNKS = 2048;  // partial sums per column sum at most
constexpr int MSE_BLOCKS = 1024;

// The decoder's forward and backward over B snapshots x P points.  q: [B][r]
// FP32 latents.  dg_in: when not NULL the caller's dL/dg [B*P][D] (no loss);
// otherwise u [B][P] gives the MSE loss and dL/dg.  Writes grad_dec (natural
// parameter layout) and dq [B][r].
template <class T>
struct DecoderPass {
  T *a[16], *dz0, *dz1, *wt[16];
  T* gt[16];  // sine networks: cos(z_l) of each hidden layer
  float *c, *g, *dg, *part;
  double *cpart, *csum, *mpart;
  static size_t bytes(const crom_net* n, int B, int64_t P) {
    Carve cv{nullptr, 0};
    DecoderPass d;
    d.carve(cv, n, B, P);
    return cv.off;
  }
  void carve(Carve& cv, const crom_net* n, int B, int64_t P) {
    const int64_t rows = (int64_t)B * P;
    const int W = n->width, depth = n->depth, D = n->d;
    for (int l = 0; l < depth; ++l) a[l] = cv.take<T>((size_t)rows * W);
    for (int l = 0; l < depth; ++l) gt[l] = n->act == CROM_ACT_SINE ? cv.take<T>((size_t)rows * W) : nullptr;
    dz0 = cv.take<T>((size_t)rows * W);
    dz1 = cv.take<T>((size_t)rows * W);
    for (int l = 1; l < depth; ++l) wt[l] = cv.take<T>((size_t)W * W);
    c = cv.take<float>((size_t)B * W);
    g = cv.take<float>((size_t)rows * D);
    dg = cv.take<float>((size_t)rows * D);
    part = cv.take<float>((size_t)MAX_SPLITS * W * W);
    const int nw = 1 + n->m > D ? 1 + n->m : D;
    const int nmax = nw > 1 + D ? nw : 1 + D;
    cpart = cv.take<double>((size_t)(B > COLSUM_CHUNKS ? B : COLSUM_CHUNKS) * nmax * W);
    csum = cv.take<double>((size_t)B * nmax * W);
    mpart = cv.take<double>(MSE_BLOCKS);
  }
};

template <class T>
static crom_status decoder_fwd_bwd(const crom_net* n, const float* x, int B, int64_t P, const float* q,
                                   const float* u, const float* dg_in, float* grad, float* dq, float* loss,
                                   DecoderPass<T>& ws, hipStream_t st) {
  const int W = n->width, depth = n->depth, D = n->d, m = n->m, r = n->r;
  const int64_t rows = (int64_t)B * P;
  const ParamIndex pi = param_index(m, r, D, W, depth);
  const float* prm = n->params;
  const bool sine = n->act == CROM_ACT_SINE;  // bfloat16 row kernels only (checked at entry)
  crom_status s = CROM_OK;
  // weights in the GEMM precision
  for (int l = 1; l < depth; ++l)
    hipLaunchKernelGGL((convert_kernel<T>), dim3(grid_for((int64_t)W * W)), dim3(256), 0, st, prm + pi.w[l], ws.wt[l],
                       (int64_t)W * W);
  // ---- forward ----
  hipLaunchKernelGGL(fold_kernel, dim3(grid_for((int64_t)B * W)), dim3(256), 0, st, prm + pi.w[0], prm + pi.b[0], q,
                     B, W, m, r, ws.c);
  if (W > EW_MAX_W || W % 8 != 0 || m > EW_MAX_MD || D > EW_MAX_MD) return fail(CROM_ERR_UNSUPPORTED, "training shape");
  {
    const dim3 grid(grid_for(rows * W / 8));
    T* g1 = ws.gt[0];
    if (sine) {
      if (m == 1) hipLaunchKernelGGL((layer1_kernel<T, 1, true>), grid, dim3(256), 0, st, prm + pi.w[0], ws.c, x, P, rows, W, r, ws.a[0], g1);
      else if (m == 2) hipLaunchKernelGGL((layer1_kernel<T, 2, true>), grid, dim3(256), 0, st, prm + pi.w[0], ws.c, x, P, rows, W, r, ws.a[0], g1);
      else hipLaunchKernelGGL((layer1_kernel<T, 3, true>), grid, dim3(256), 0, st, prm + pi.w[0], ws.c, x, P, rows, W, r, ws.a[0], g1);
    } else {
      if (m == 1) hipLaunchKernelGGL((layer1_kernel<T, 1>), grid, dim3(256), 0, st, prm + pi.w[0], ws.c, x, P, rows, W, r, ws.a[0], g1);
      else if (m == 2) hipLaunchKernelGGL((layer1_kernel<T, 2>), grid, dim3(256), 0, st, prm + pi.w[0], ws.c, x, P, rows, W, r, ws.a[0], g1);
      else hipLaunchKernelGGL((layer1_kernel<T, 3>), grid, dim3(256), 0, st, prm + pi.w[0], ws.c, x, P, rows, W, r, ws.a[0], g1);
    }
  }
  for (int l = 1; l < depth; ++l) {
    if constexpr (sizeof(T) == 2) {
      if (row_gemm<true>(W, ws.a[l - 1], ws.wt[l], prm + pi.b[l], nullptr, ws.a[l], rows, st, &s, sine, ws.gt[l])) {
        if (s != CROM_OK) return s;
        continue;
      }
    }
    GemmArgs g = gemm_args((int)rows, W, W, ws.a[l - 1], W, ws.wt[l], W);
    g.bias = prm + pi.b[l];
    if constexpr (sizeof(T) == 2) {
      g.Cb = reinterpret_cast<__bf16*>(ws.a[l]);
      g.ldcb = W;
    } else {
      g.C = reinterpret_cast<float*>(ws.a[l]);
      g.ldc = W;
    }
    if ((s = gemm<T, false, true, EPI_BIAS_ELU>(g, st)) != CROM_OK) return s;
  }
  if (D == 1)
    hipLaunchKernelGGL((output_kernel<T, 1>), dim3(grid_for(rows)), dim3(256), 0, st, ws.a[depth - 1],
                       prm + pi.w[depth], prm + pi.b[depth], rows, W, ws.g);
  else
    hipLaunchKernelGGL((output_kernel<T, 3>), dim3(grid_for(rows)), dim3(256), 0, st, ws.a[depth - 1],
                       prm + pi.w[depth], prm + pi.b[depth], rows, W, ws.g);
  const float* dg = dg_in;
  if (!dg_in) {
    hipLaunchKernelGGL(mse_kernel, dim3(MSE_BLOCKS), dim3(256), 0, st, ws.g, u, rows * D, ws.dg, ws.mpart);
    hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, ws.mpart, MSE_BLOCKS, rows * D, loss);
    dg = ws.dg;
  }
  // ---- backward: output layer ----
  {
    // dWout[o][u] = sum_rows dg[row][o] a[row][u]; dbout[o] = sum dg[row][o]
    // (column sums of a weighted by dg, and of dg itself)
    colsum<T>(ws.a[depth - 1], W, W, 1, rows, dg, rows, D, 1 + D, ws.cpart, COLSUM_CHUNKS, ws.csum, st);
    // csum[1 + o][u] = dWout[o][u]
    hipLaunchKernelGGL(d2f_kernel, dim3(grid_for((int64_t)D * W)), dim3(256), 0, st, ws.csum + W, grad + pi.w[depth],
                       (int64_t)D * W);
    colsum<float>(dg, D, D, 1, rows, nullptr, 1, 0, 1, ws.cpart, COLSUM_CHUNKS, ws.csum, st);
    hipLaunchKernelGGL(d2f_kernel, dim3(1), dim3(64), 0, st, ws.csum, grad + pi.b[depth], (int64_t)D);
    if (sine && D == 1)
      hipLaunchKernelGGL((dz_last_kernel<T, 1, true>), dim3(grid_for(rows * W / 8)), dim3(256), 0, st, dg,
                         prm + pi.w[depth], ws.gt[depth - 1], rows, W, ws.dz0);
    else if (sine)
      hipLaunchKernelGGL((dz_last_kernel<T, 3, true>), dim3(grid_for(rows * W / 8)), dim3(256), 0, st, dg,
                         prm + pi.w[depth], ws.gt[depth - 1], rows, W, ws.dz0);
    else if (D == 1)
      hipLaunchKernelGGL((dz_last_kernel<T, 1>), dim3(grid_for(rows * W / 8)), dim3(256), 0, st, dg,
                         prm + pi.w[depth], ws.a[depth - 1], rows, W, ws.dz0);
    else
      hipLaunchKernelGGL((dz_last_kernel<T, 3>), dim3(grid_for(rows * W / 8)), dim3(256), 0, st, dg,
                         prm + pi.w[depth], ws.a[depth - 1], rows, W, ws.dz0);
  }
  // ---- hidden layers ----
  T* dz = ws.dz0;
  T* dzn = ws.dz1;
  for (int l = depth - 1; l >= 1; --l) {
    // dW_l = dz^T a_{l-1}  (split over rows)
    bool wg = false;
    if constexpr (sizeof(T) == 2) {
      wg = wgrad(W, dz, ws.a[l - 1], rows, ws.part, grad + pi.w[l], st, &s);
      if (s != CROM_OK) return s;
    }
    if (!wg) {
      GemmArgs gw = gemm_args(W, W, (int)rows, dz, W, ws.a[l - 1], W);
      gw.C = grad + pi.w[l];
      gw.ldc = W;
      gw.part = ws.part;
      if ((s = gemm<T, true, false, EPI_NONE>(gw, st)) != CROM_OK) return s;
    }
    // db_l = column sums of dz
    colsum<T>(dz, W, W, 1, rows, nullptr, 1, 0, 1, ws.cpart, COLSUM_CHUNKS, ws.csum, st);
    hipLaunchKernelGGL(d2f_kernel, dim3(grid_for(W)), dim3(256), 0, st, ws.csum, grad + pi.b[l], (int64_t)W);
    // dz_{l-1} = (dz W_l) * ELU'(a_{l-1})
    bool done = false;
    if constexpr (sizeof(T) == 2) {
      done = row_gemm<false>(W, dz, ws.wt[l], nullptr, sine ? ws.gt[l - 1] : ws.a[l - 1], dzn, rows, st, &s, sine);
      if (s != CROM_OK) return s;
    }
    if (done) {
      T* t = dz;
      dz = dzn;
      dzn = t;
      continue;
    }
    GemmArgs gd = gemm_args((int)rows, W, W, dz, W, ws.wt[l], W);
    gd.gate = ws.a[l - 1];
    gd.ldg = W;
    if constexpr (sizeof(T) == 2) {
      gd.Cb = reinterpret_cast<__bf16*>(dzn);
      gd.ldcb = W;
    } else {
      gd.C = reinterpret_cast<float*>(dzn);
      gd.ldc = W;
    }
    if ((s = gemm<T, false, false, EPI_DELU>(gd, st)) != CROM_OK) return s;
    T* t = dz;
    dz = dzn;
    dzn = t;
  }
  // ---- first layer: per-snapshot sums of dz1 and of dz1 * x_i ----
  {
    const int nw = 1 + m;
    colsum<T>(dz, W, W, B, P, x, P, m, nw, ws.cpart, COLSUM_CHUNKS, ws.csum, st);
    hipLaunchKernelGGL(layer1_grad_kernel, dim3(grid_for((int64_t)W * (m + r) + W + B * r)), dim3(256), 0, st,
                       ws.csum, q, prm + pi.w[0], B, W, m, r, grad + pi.w[0], grad + pi.b[0], dq);
  }
  return hip_check(hipGetLastError(), "decoder backward");
}

// Encoder: E1 [hidden][n_in], c1 [hidden], E2 [r][hidden], c2 [r] (FP32).
template <class T>
struct EncoderPass {
  T *e1, *ub, *h, *dh;
  float *q, *dq, *h32, *kpart;
  double *cpart, *csum;
  void carve(Carve& cv, const crom_encoder* e, int B) {
    e1 = cv.take<T>((size_t)e->hidden * e->n_in);
    ub = cv.take<T>((size_t)B * e->n_in);
    h = cv.take<T>((size_t)B * e->hidden);
    dh = cv.take<T>((size_t)B * e->hidden);
    q = cv.take<float>((size_t)B * e->r);
    dq = cv.take<float>((size_t)B * e->r);
    h32 = cv.take<float>((size_t)B * e->hidden);
    kpart = cv.take<float>((size_t)MAX_SPLITS * B * e->hidden);
    // column sums over the batch of dz1 [B][hidden] and of dq [B][r]
    const int cols = e->hidden > e->r ? e->hidden : e->r;
    cpart = cv.take<double>((size_t)COLSUM_CHUNKS * cols);
    csum = cv.take<double>((size_t)cols);
  }
};

static ParamIndex enc_index(const crom_encoder* e) {
  ParamIndex pi{};
  pi.w[0] = 0;
  pi.b[0] = (int64_t)e->hidden * e->n_in;
  pi.w[1] = pi.b[0] + e->hidden;
  pi.b[1] = pi.w[1] + (int64_t)e->r * e->hidden;
  return pi;
}

template <class T>
static crom_status encoder_fwd(const crom_encoder* e, const float* u, int B, EncoderPass<T>& ws, hipStream_t st) {
  const ParamIndex pi = enc_index(e);
  const float* prm = e->params;
  hipLaunchKernelGGL((convert_kernel<T>), dim3(grid_for((int64_t)e->hidden * e->n_in)), dim3(256), 0, st, prm,
                     ws.e1, (int64_t)e->hidden * e->n_in);
  hipLaunchKernelGGL((convert_kernel<T>), dim3(grid_for((int64_t)B * e->n_in)), dim3(256), 0, st, u, ws.ub,
                     (int64_t)B * e->n_in);
  // h = ELU(u E1^T + c1)  [B][hidden], kept in T (for the GEMM) and FP32
  GemmArgs g = gemm_args(B, e->hidden, e->n_in, ws.ub, e->n_in, ws.e1, e->n_in);
  g.bias = prm + pi.b[0];
  g.C = ws.h32;
  g.ldc = e->hidden;
  g.part = ws.kpart;  // few rows, long K: split K over blocks
  crom_status s = gemm<T, false, true, EPI_BIAS_ELU>(g, st);
  if (s != CROM_OK) return s;
  hipLaunchKernelGGL((convert_kernel<T>), dim3(grid_for((int64_t)B * e->hidden)), dim3(256), 0, st, ws.h32, ws.h,
                     (int64_t)B * e->hidden);
  // q = h E2^T + c2 (FP32 product of the FP32 activations)
  GemmArgs g2 = gemm_args(B, e->r, e->hidden, ws.h32, e->hidden, prm + pi.w[1], e->hidden);
  g2.bias = prm + pi.b[1];
  g2.C = ws.q;
  g2.ldc = e->r;
  return gemm<float, false, true, EPI_BIAS>(g2, st);
}

template <class T>
static crom_status encoder_bwd(const crom_encoder* e, int B, const float* dq, float* grad, EncoderPass<T>& ws,
                               float* split_part, hipStream_t st) {
  const ParamIndex pi = enc_index(e);
  const float* prm = e->params;
  crom_status s;
  // dE2 = dq^T h  [r][hidden], dc2 = sum_b dq
  {
    GemmArgs g = gemm_args(e->r, e->hidden, B, dq, e->r, ws.h32, e->hidden);
    g.C = grad + pi.w[1];
    g.ldc = e->hidden;
    if ((s = gemm<float, true, false, EPI_NONE>(g, st)) != CROM_OK) return s;
    colsum<float>(dq, e->r, e->r, 1, B, nullptr, 1, 0, 1, ws.cpart, COLSUM_CHUNKS, ws.csum, st);
    hipLaunchKernelGGL(d2f_kernel, dim3(1), dim3(64), 0, st, ws.csum, grad + pi.b[1], (int64_t)e->r);
  }
  // dz1 = (dq E2) * ELU'(h)  [B][hidden]
  {
    GemmArgs g = gemm_args(B, e->hidden, e->r, dq, e->r, prm + pi.w[1], e->hidden);
    g.gate = ws.h32;
    g.ldg = e->hidden;
    g.C = ws.h32;  // h is consumed by the gate in the same element: safe in place
    g.ldc = e->hidden;
    if ((s = gemm<float, false, false, EPI_DELU>(g, st)) != CROM_OK) return s;
  }
  hipLaunchKernelGGL((convert_kernel<T>), dim3(grid_for((int64_t)B * e->hidden)), dim3(256), 0, st, ws.h32, ws.dh,
                     (int64_t)B * e->hidden);
  // dE1 = dz1^T u  [hidden][n_in];  dc1 = sum_b dz1
  {
    GemmArgs g = gemm_args(e->hidden, e->n_in, B, ws.dh, e->hidden, ws.ub, e->n_in);
    g.C = grad + pi.w[0];
    g.ldc = e->n_in;
    if ((s = gemm<T, true, false, EPI_NONE>(g, st)) != CROM_OK) return s;
    colsum<float>(ws.h32, e->hidden, e->hidden, 1, B, nullptr, 1, 0, 1, ws.cpart, COLSUM_CHUNKS, ws.csum, st);
    hipLaunchKernelGGL(d2f_kernel, dim3(grid_for(e->hidden)), dim3(256), 0, st, ws.csum, grad + pi.b[0],
                       (int64_t)e->hidden);
  }
  (void)split_part;
  return hip_check(hipGetLastError(), "encoder backward");
}

// ---------------------------------------------------------------------------
// Convolutional encoder (Sec. "Network Details"): the snapshot as a 1D vector
// of its P points with d channels; 1D convolutions (kernel 6, stride 4, d
// output channels, no padding, ELU) until the length is the smallest one not
// below 32 / d; flattened channel-major; a dense layer of `hidden` values
// (ELU) and a linear dense layer to r.  FP32 storage, FP32 products inside a
// convolution window or a dense row, FP64 sums over the batch and over
// positions for the weight gradients (fixed order: deterministic).
// Parameters, FP32, in order: per convolution W [d][d][6], b [d]; then
// E1 [hidden][L d], c1 [hidden], E2 [r][hidden], c2 [r].
// ---------------------------------------------------------------------------
constexpr int CONV_K = 6, CONV_S = 4, CONV_MAXL = 16;

struct ConvShape {
  int d, nl, hidden, r;
  int64_t len[CONV_MAXL + 1];  // len[0] = P
  int64_t w[CONV_MAXL], b[CONV_MAXL], e1, c1, e2, c2, count;
};

static ConvShape conv_shape(int64_t P, int d, int hidden, int r) {
  ConvShape c{};
  c.d = d;
  c.hidden = hidden;
  c.r = r;
  c.len[0] = P;
  int64_t L = P;
  while (L >= CONV_K && c.nl < CONV_MAXL) {
    const int64_t nxt = (L - CONV_K) / CONV_S + 1;
    if (nxt * d < 32) break;
    c.len[++c.nl] = nxt;
    L = nxt;
  }
  int64_t o = 0;
  for (int l = 0; l < c.nl; ++l) {
    c.w[l] = o;
    o += (int64_t)d * d * CONV_K;
    c.b[l] = o;
    o += d;
  }
  c.e1 = o;
  o += (int64_t)hidden * L * d;
  c.c1 = o;
  o += hidden;
  c.e2 = o;
  o += (int64_t)r * hidden;
  c.c2 = o;
  o += r;
  c.count = o;
  return c;
}

__device__ __forceinline__ float elu_f(float z) { return z > 0.0f ? z : expm1f(z); }
__device__ __forceinline__ float delu_from_act(float a) { return a > 0.0f ? 1.0f : a + 1.0f; }

// y[b][o][j] = ELU(bias[o] + sum_{c,k} W[o][c][k] x(b, c, 4 j + k)), with
// x(b, c, i) = x[b * xb + c * xc + i * xi].
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float* __restrict__ x, int64_t xb, int64_t xc,
                                                      int64_t xi, const float* __restrict__ W,
                                                      const float* __restrict__ bias, int B, int d, int64_t Lo,
                                                      float* __restrict__ y) {
  const int64_t total = (int64_t)B * d * Lo;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e % Lo, bo = e / Lo;
    const int o = (int)(bo % d), b = (int)(bo / d);
    float s = bias[o];
    for (int c = 0; c < d; ++c) {
      const float* xp = x + b * xb + c * xc + (CONV_S * j) * xi;
      const float* wp = W + ((int64_t)o * d + c) * CONV_K;
#pragma unroll
      for (int k = 0; k < CONV_K; ++k) s += wp[k] * xp[k * xi];
    }
    y[e] = elu_f(s);
  }
}

// out[b][o] = act(bias[o] + sum_i W[o][i] in[b][i])  (act: ELU or none)
__global__ __launch_bounds__(256) void dense_fwd_kernel(const float* __restrict__ in, const float* __restrict__ W,
                                                       const float* __restrict__ bias, int B, int64_t n_in,
                                                       int n_out, int elu, float* __restrict__ out) {
  const int64_t total = (int64_t)B * n_out;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(e % n_out);
    const int64_t b = e / n_out;
    float s = bias[o];
    for (int64_t i = 0; i < n_in; ++i) s += W[o * n_in + i] * in[b * n_in + i];
    out[e] = elu ? elu_f(s) : s;
  }
}

// dW[o][i] = sum_b dy[b][o] x[b][i], db[o] = sum_b dy[b][o] (FP64 sums over b in order)
__global__ __launch_bounds__(256) void dense_wgrad_kernel(const float* __restrict__ dy, const float* __restrict__ x,
                                                         int B, int64_t n_in, int n_out, float* __restrict__ dW,
                                                         float* __restrict__ db) {
  const int64_t total = (int64_t)n_out * n_in + n_out;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    if (e < (int64_t)n_out * n_in) {
      const int64_t o = e / n_in, i = e % n_in;
      for (int b = 0; b < B; ++b) s += (double)dy[(int64_t)b * n_out + o] * (double)x[(int64_t)b * n_in + i];
      dW[e] = (float)s;
    } else {
      const int64_t o = e - (int64_t)n_out * n_in;
      for (int b = 0; b < B; ++b) s += (double)dy[(int64_t)b * n_out + o];
      db[o] = (float)s;
    }
  }
}

// dx[b][i] = (sum_o dy[b][o] W[o][i]) * ELU'(a[b][i])  (a NULL: no gate)
__global__ __launch_bounds__(256) void dense_dx_kernel(const float* __restrict__ dy, const float* __restrict__ W,
                                                      const float* __restrict__ a, int B, int64_t n_in, int n_out,
                                                      float* __restrict__ dx) {
  const int64_t total = (int64_t)B * n_in;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n_in, b = e / n_in;
    float s = 0.0f;
    for (int o = 0; o < n_out; ++o) s += dy[b * n_out + o] * W[(int64_t)o * n_in + i];
    dx[e] = a ? s * delu_from_act(a[e]) : s;
  }
}

// Weight and bias gradients of one convolution, in two fixed-order stages.
// Stage 1, block (e, chunk): e < d*d*6 takes W[o][c][k] =
// sum_{b,j} dz[b][o][j] x(b, c, 4 j + k), e = d*d*6 + o the bias
// sum_{b,j} dz[b][o][j], over the chunk's contiguous share of the (b, j)
// pairs (each thread a fixed stride in FP64, then a tree in LDS) into
// part[e][chunk].  Stage 2: each entry sums its chunks in order.
constexpr int CONV_RED = 256, CONV_CHUNKS = 64;
__global__ __launch_bounds__(CONV_RED) void conv_wgrad_kernel(const float* __restrict__ dz, const float* __restrict__ x,
                                                             int64_t xb, int64_t xc, int64_t xi, int B, int d,
                                                             int64_t Lo, double* __restrict__ part) {
  __shared__ double red[CONV_RED];
  const int e = blockIdx.x, chunk = blockIdx.y;
  const int nw = d * d * CONV_K;
  const int64_t n = (int64_t)B * Lo;
  const int64_t per = (n + CONV_CHUNKS - 1) / CONV_CHUNKS;
  const int64_t t0 = chunk * per, t1 = t0 + per < n ? t0 + per : n;
  double s = 0.0;
  if (e < nw) {
    const int o = e / (d * CONV_K), c = (e / CONV_K) % d, k = e % CONV_K;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += CONV_RED) {
      const int64_t b = t / Lo, j = t % Lo;
      s += (double)dz[(b * d + o) * Lo + j] * (double)x[b * xb + c * xc + (CONV_S * j + k) * xi];
    }
  } else {
    const int o = e - nw;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += CONV_RED) {
      const int64_t b = t / Lo, j = t % Lo;
      s += (double)dz[(b * d + o) * Lo + j];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = CONV_RED / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)e * CONV_CHUNKS + chunk] = red[0];
}

__global__ __launch_bounds__(64) void conv_wgrad_final_kernel(const double* __restrict__ part, int d,
                                                             float* __restrict__ dW, float* __restrict__ db) {
  const int nw = d * d * CONV_K;
  for (int e = threadIdx.x; e < nw + d; e += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < CONV_CHUNKS; ++c) s += part[(int64_t)e * CONV_CHUNKS + c];
    if (e < nw) dW[e] = (float)s;
    else db[e - nw] = (float)s;
  }
}

// Input gradient of one convolution, gated by the ELU of the layer below:
// dzp[b][c][i] = ELU'(a[b][c][i]) sum_o sum_{k: i = 4 j + k, 0 <= j < Lo} dz[b][o][j] W[o][c][k]
__global__ __launch_bounds__(256) void conv_dx_kernel(const float* __restrict__ dz, const float* __restrict__ W,
                                                     const float* __restrict__ a, int B, int d, int64_t Li,
                                                     int64_t Lo, float* __restrict__ dzp) {
  const int64_t total = (int64_t)B * d * Li;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % Li, bc = e / Li;
    const int c = (int)(bc % d);
    const int64_t b = bc / d;
    float s = 0.0f;
    for (int k = (int)(i % CONV_S); k < CONV_K; k += CONV_S) {
      const int64_t j = (i - k) / CONV_S;
      if (i < k || j >= Lo) continue;
      for (int o = 0; o < d; ++o) s += dz[(b * d + o) * Lo + j] * W[((int64_t)o * d + c) * CONV_K + k];
    }
    dzp[e] = s * delu_from_act(a[e]);
  }
}

struct ConvPass {
  float* a[CONV_MAXL + 1];  // a[l] = ELU(conv_l) [B][d][len[l]], l >= 1
  float *h, *q, *dq, *dh, *dz[2];
  double* wpart;  // [d*d*6 + d][CONV_CHUNKS] weight-gradient partials
  void carve(Carve& cv, const ConvShape& c, int B) {
    wpart = cv.take<double>((size_t)(c.d * c.d * CONV_K + c.d) * CONV_CHUNKS);
    for (int l = 1; l <= c.nl; ++l) a[l] = cv.take<float>((size_t)B * c.d * c.len[l]);
    const int64_t top = c.nl ? c.len[1] : c.len[0];
    h = cv.take<float>((size_t)B * c.hidden);
    dh = cv.take<float>((size_t)B * c.hidden);
    q = cv.take<float>((size_t)B * c.r);
    dq = cv.take<float>((size_t)B * c.r);
    dz[0] = cv.take<float>((size_t)B * c.d * top);
    dz[1] = cv.take<float>((size_t)B * c.d * top);
  }
};

// Strides of the activation entering convolution l (l = 0: the snapshot
// [B][P][d], point-major; else [B][d][len]).
static void conv_in(const ConvShape& c, const float* u, const ConvPass& w, int l, const float** x, int64_t* xb,
                    int64_t* xc, int64_t* xi) {
  if (l == 0) {
    *x = u;
    *xb = c.len[0] * c.d;
    *xc = 1;
    *xi = c.d;
  } else {
    *x = w.a[l];
    *xb = c.d * c.len[l];
    *xc = c.len[l];
    *xi = 1;
  }
}

static crom_status conv_encoder_fwd(const ConvShape& c, const float* prm, const float* u, int B, ConvPass& w,
                                    hipStream_t st) {
  for (int l = 0; l < c.nl; ++l) {
    const float* x;
    int64_t xb, xc, xi;
    conv_in(c, u, w, l, &x, &xb, &xc, &xi);
    hipLaunchKernelGGL(conv_fwd_kernel, dim3(grid_for((int64_t)B * c.d * c.len[l + 1])), dim3(256), 0, st, x, xb,
                       xc, xi, prm + c.w[l], prm + c.b[l], B, c.d, c.len[l + 1], w.a[l + 1]);
  }
  // the flattened top: [B][d][L] is [B][L d] channel-major; with no
  // convolution the snapshot itself ([B][P d], point-major)
  const float* flat = c.nl ? w.a[c.nl] : u;
  const int64_t n_flat = c.len[c.nl] * c.d;
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(grid_for((int64_t)B * c.hidden)), dim3(256), 0, st, flat, prm + c.e1,
                     prm + c.c1, B, n_flat, c.hidden, 1, w.h);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(grid_for((int64_t)B * c.r)), dim3(256), 0, st, w.h, prm + c.e2,
                     prm + c.c2, B, (int64_t)c.hidden, c.r, 0, w.q);
  return hip_check(hipGetLastError(), "convolutional encoder forward");
}

static crom_status conv_encoder_bwd(const ConvShape& c, const float* prm, const float* u, int B, const float* dq,
                                    float* grad, ConvPass& w, hipStream_t st) {
  const float* flat = c.nl ? w.a[c.nl] : u;
  const int64_t n_flat = c.len[c.nl] * c.d;
  // last layer: dE2, dc2; dh = (dq E2) ELU'(h)
  hipLaunchKernelGGL(dense_wgrad_kernel, dim3(grid_for((int64_t)c.r * c.hidden + c.r)), dim3(256), 0, st, dq, w.h, B,
                     (int64_t)c.hidden, c.r, grad + c.e2, grad + c.c2);
  hipLaunchKernelGGL(dense_dx_kernel, dim3(grid_for((int64_t)B * c.hidden)), dim3(256), 0, st, dq, prm + c.e2, w.h, B,
                     (int64_t)c.hidden, c.r, w.dh);
  // dense layer: dE1, dc1; the top convolution's output gradient
  hipLaunchKernelGGL(dense_wgrad_kernel, dim3(grid_for((int64_t)c.hidden * n_flat + c.hidden)), dim3(256), 0, st, w.dh,
                     flat, B, n_flat, c.hidden, grad + c.e1, grad + c.c1);
  if (c.nl == 0) return hip_check(hipGetLastError(), "convolutional encoder backward");
  hipLaunchKernelGGL(dense_dx_kernel, dim3(grid_for((int64_t)B * n_flat)), dim3(256), 0, st, w.dh, prm + c.e1,
                     w.a[c.nl], B, n_flat, c.hidden, w.dz[0]);
  int cur = 0;
  for (int l = c.nl - 1; l >= 0; --l) {  // convolution l: len[l] -> len[l + 1]
    const float* x;
    int64_t xb, xc, xi;
    conv_in(c, u, w, l, &x, &xb, &xc, &xi);
    hipLaunchKernelGGL(conv_wgrad_kernel, dim3(c.d * c.d * CONV_K + c.d, CONV_CHUNKS), dim3(CONV_RED), 0, st,
                       w.dz[cur], x, xb, xc, xi, B, c.d, c.len[l + 1], w.wpart);
    hipLaunchKernelGGL(conv_wgrad_final_kernel, dim3(1), dim3(64), 0, st, w.wpart, c.d, grad + c.w[l],
                       grad + c.b[l]);
    if (l > 0) {
      hipLaunchKernelGGL(conv_dx_kernel, dim3(grid_for((int64_t)B * c.d * c.len[l])), dim3(256), 0, st, w.dz[cur],
                         prm + c.w[l], w.a[l], B, c.d, c.len[l], c.len[l + 1], w.dz[1 - cur]);
      cur = 1 - cur;
    }
  }
  return hip_check(hipGetLastError(), "convolutional encoder backward");
}

static ConvShape conv_of(const crom_net* n, const crom_encoder* e) {
  return conv_shape(e->n_in / n->d, n->d, e->hidden, e->r);
}

static bool bf_mode(const crom_net* n) { return n->precision != CROM_PREC_FP32; }

template <class T>
static size_t train_bytes_t(const crom_net* n, const crom_encoder* e, int B) {
  Carve cv{nullptr, 0};
  DecoderPass<T> d;
  d.carve(cv, n, B, e->n_in / n->d);
  if (e->kind == CROM_ENC_CONV) {
    ConvPass cp;
    cp.carve(cv, conv_of(n, e), B);
  } else {
    EncoderPass<T> en;
    en.carve(cv, e, B);
  }
  return cv.off + 256;
}

static crom_status check_enc(const crom_net* n, const crom_encoder* e) {
  if (!e || !e->params) return fail(CROM_ERR_INVALID_ARG, "encoder and its params are required");
  if (e->n_in < 1 || e->hidden < 1 || e->r != n->r || e->n_in % n->d != 0)
    return fail(CROM_ERR_INVALID_ARG, "encoder shape: r must match the net and n_in = P * d");
  if (e->kind != CROM_ENC_DENSE && e->kind != CROM_ENC_CONV) return fail(CROM_ERR_INVALID_ARG, "encoder kind");
  if (e->kind == CROM_ENC_CONV && conv_of(n, e).nl < 1)
    return fail(CROM_ERR_INVALID_ARG, "the convolutional encoder needs room for one convolution (P d values)");
  return CROM_OK;
}

template <class T>
static crom_status train_grads_t(const crom_net* n, const crom_encoder* e, const float* u, const float* x, int B,
                                 float* grad_dec, float* grad_enc, float* loss, float* q_out, void* ws,
                                 hipStream_t st) {
  Carve cv{reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255)), 0};
  const int64_t P = e->n_in / n->d;
  DecoderPass<T> d;
  d.carve(cv, n, B, P);
  if (e->kind == CROM_ENC_CONV) {
    const ConvShape c = conv_of(n, e);
    ConvPass cp;
    cp.carve(cv, c, B);
    crom_status s = conv_encoder_fwd(c, e->params, u, B, cp, st);
    if (s != CROM_OK) return s;
    s = decoder_fwd_bwd<T>(n, x, B, P, cp.q, u, nullptr, grad_dec, cp.dq, loss, d, st);
    if (s != CROM_OK) return s;
    s = conv_encoder_bwd(c, e->params, u, B, cp.dq, grad_enc, cp, st);
    if (s != CROM_OK) return s;
    if (q_out) s = hip_check(hipMemcpyAsync(q_out, cp.q, sizeof(float) * B * e->r, hipMemcpyDeviceToDevice, st), "q copy");
    return s;
  }
  EncoderPass<T> en;
  en.carve(cv, e, B);
  crom_status s = encoder_fwd<T>(e, u, B, en, st);
  if (s != CROM_OK) return s;
  s = decoder_fwd_bwd<T>(n, x, B, P, en.q, u, nullptr, grad_dec, en.dq, loss, d, st);
  if (s != CROM_OK) return s;
  s = encoder_bwd<T>(e, B, en.dq, grad_enc, en, d.part, st);
  if (s != CROM_OK) return s;
  if (q_out) s = hip_check(hipMemcpyAsync(q_out, en.q, sizeof(float) * B * e->r, hipMemcpyDeviceToDevice, st), "q copy");
  return s;
}

}  // namespace crom

using namespace crom;

extern "C" {

size_t crom_encoder_param_count(int32_t n_in, int32_t hidden, int32_t r) {
  if (n_in < 1 || hidden < 1 || r < 1) return 0;
  return (size_t)hidden * n_in + hidden + (size_t)r * hidden + r;
}

size_t crom_conv_encoder_param_count(int64_t P, int32_t d, int32_t hidden, int32_t r) {
  if (P < 1 || d < 1 || hidden < 1 || r < 1) return 0;
  const ConvShape c = conv_shape(P, d, hidden, r);
  return c.nl < 1 ? 0 : (size_t)c.count;
}

crom_status crom_train_workspace(const crom_net* net, const crom_encoder* enc, int32_t B, size_t* bytes) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (net->act != CROM_ACT_ELU &&
      (net->act != CROM_ACT_SINE || net->precision == CROM_PREC_FP32 || (net->width != 32 && net->width != 128)))
    return fail(CROM_ERR_UNSUPPORTED, "training kernels: ELU networks, or sine networks of width 32 or 128 in bfloat16");
  if ((s = check_enc(net, enc)) != CROM_OK) return s;
  if (B < 1 || !bytes) return fail(CROM_ERR_INVALID_ARG, "B >= 1 and bytes are required");
  *bytes = bf_mode(net) ? train_bytes_t<__bf16>(net, enc, B) : train_bytes_t<float>(net, enc, B);
  return CROM_OK;
}

crom_status crom_train_grads(const crom_net* net, const crom_encoder* enc, const float* u, const float* x, int32_t B,
                             float* grad_dec, float* grad_enc, float* loss, float* q_out, void* ws, size_t ws_bytes,
                             void* stream) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (net->act != CROM_ACT_ELU &&
      (net->act != CROM_ACT_SINE || net->precision == CROM_PREC_FP32 || (net->width != 32 && net->width != 128)))
    return fail(CROM_ERR_UNSUPPORTED, "training kernels: ELU networks, or sine networks of width 32 or 128 in bfloat16");
  if ((s = check_enc(net, enc)) != CROM_OK) return s;
  if (B < 1 || !u || !x || !grad_dec || !grad_enc || !loss || !ws)
    return fail(CROM_ERR_INVALID_ARG, "u, x, gradients, loss and ws are required");
  size_t need = 0;
  crom_train_workspace(net, enc, B, &need);
  if (ws_bytes < need) return fail(CROM_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return bf_mode(net) ? train_grads_t<__bf16>(net, enc, u, x, B, grad_dec, grad_enc, loss, q_out, ws, st)
                      : train_grads_t<float>(net, enc, u, x, B, grad_dec, grad_enc, loss, q_out, ws, st);
}

crom_status crom_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, int64_t t, float lr,
                           float beta1, float beta2, float eps, void* stream) {
  if (n < 0 || t < 1) return fail(CROM_ERR_INVALID_ARG, "n >= 0 and t >= 1");
  if (n == 0) return CROM_OK;
  if (!params || !grad || !m || !v) return fail(CROM_ERR_INVALID_ARG, "params, grad, m and v are required");
  const float c1 = (float)(1.0 - pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)t));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), params, grad, m,
                     v, n, lr, beta1, beta2, eps, c1, c2);
  return hip_check(hipGetLastError(), "adam launch");
}

crom_status crom_train_step(const crom_net* net, void* packed, float* dec_grad, float* dec_m, float* dec_v,
                            const crom_encoder* enc, float* enc_grad, float* enc_m, float* enc_v, int64_t t,
                            const float* u, const float* x, int32_t B, float lr, float* loss, void* ws,
                            size_t ws_bytes, void* stream) {
  crom_status s = crom_train_grads(net, enc, u, x, B, dec_grad, enc_grad, loss, nullptr, ws, ws_bytes, stream);
  if (s != CROM_OK) return s;
  if (!dec_m || !dec_v || !enc_m || !enc_v) return fail(CROM_ERR_INVALID_ARG, "Adam moments are required");
  const int64_t nd = (int64_t)crom_net_param_count(net->m, net->r, net->d, net->width, net->depth);
  const int64_t ne = enc->kind == CROM_ENC_CONV ? conv_of(net, enc).count
                                                : (int64_t)crom_encoder_param_count(enc->n_in, enc->hidden, enc->r);
  s = crom_adam_step(const_cast<float*>(net->params), dec_grad, dec_m, dec_v, nd, t, lr, 0.9f, 0.999f, 1e-8f, stream);
  if (s != CROM_OK) return s;
  s = crom_adam_step(enc->params, enc_grad, enc_m, enc_v, ne, t, lr, 0.9f, 0.999f, 1e-8f, stream);
  if (s != CROM_OK) return s;
  if (packed) return crom_net_pack(net, packed, stream);
  return CROM_OK;
}

static int64_t enc_count(const crom_net* net, const crom_encoder* enc) {
  return enc->kind == CROM_ENC_CONV ? conv_of(net, enc).count
                                    : (int64_t)crom_encoder_param_count(enc->n_in, enc->hidden, enc->r);
}

crom_status crom_train_state_offsets(const crom_net* net, const crom_encoder* enc, crom_train_state_layout* out) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if ((s = check_enc(net, enc)) != CROM_OK) return s;
  if (!out) return fail(CROM_ERR_INVALID_ARG, "out is NULL");
  const size_t nd = 4 * crom_net_param_count(net->m, net->r, net->d, net->width, net->depth);
  const size_t ne = 4 * (size_t)enc_count(net, enc);
  size_t o = 0;
  auto take = [&o](size_t n) {
    const size_t at = o;
    o = (o + n + 255) & ~size_t(255);
    return at;
  };
  out->dec_params = take(nd);
  out->dec_grad = take(nd);
  out->dec_m = take(nd);
  out->dec_v = take(nd);
  out->enc_params = take(ne);
  out->enc_grad = take(ne);
  out->enc_m = take(ne);
  out->enc_v = take(ne);
  out->total = o;
  return CROM_OK;
}

size_t crom_train_state_bytes(const crom_net* net, const crom_encoder* enc) {
  crom_train_state_layout L;
  return crom_train_state_offsets(net, enc, &L) == CROM_OK ? L.total : 0;
}

crom_status crom_train_step_state(const crom_net* net, const crom_encoder* enc, void* state, void* packed, int64_t t,
                                  const float* u, const float* x, int32_t B, float lr, float* loss, void* ws,
                                  size_t ws_bytes, void* stream) {
  crom_train_state_layout L;
  crom_status s = crom_train_state_offsets(net, enc, &L);
  if (s != CROM_OK) return s;
  if (!state) return fail(CROM_ERR_INVALID_ARG, "state is NULL");
  if (reinterpret_cast<uintptr_t>(state) & 255) return fail(CROM_ERR_INVALID_ARG, "state must be 256-byte aligned");
  char* b = static_cast<char*>(state);
  crom_net n = *net;
  n.params = reinterpret_cast<const float*>(b + L.dec_params);
  crom_encoder e = *enc;
  e.params = reinterpret_cast<float*>(b + L.enc_params);
  return crom_train_step(&n, packed, reinterpret_cast<float*>(b + L.dec_grad), reinterpret_cast<float*>(b + L.dec_m),
                         reinterpret_cast<float*>(b + L.dec_v), &e, reinterpret_cast<float*>(b + L.enc_grad),
                         reinterpret_cast<float*>(b + L.enc_m), reinterpret_cast<float*>(b + L.enc_v), t, u, x, B, lr,
                         loss, ws, ws_bytes, stream);
}

crom_status crom_encode_workspace(const crom_net* net, const crom_encoder* enc, int32_t B, size_t* bytes) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (net->act != CROM_ACT_ELU &&
      (net->act != CROM_ACT_SINE || net->precision == CROM_PREC_FP32 || (net->width != 32 && net->width != 128)))
    return fail(CROM_ERR_UNSUPPORTED, "training kernels: ELU networks, or sine networks of width 32 or 128 in bfloat16");
  if ((s = check_enc(net, enc)) != CROM_OK) return s;
  if (B < 1 || !bytes) return fail(CROM_ERR_INVALID_ARG, "B >= 1 and bytes are required");
  Carve cv{nullptr, 0};
  if (enc->kind == CROM_ENC_CONV) {
    ConvPass cp;
    cp.carve(cv, conv_of(net, enc), B);
  } else if (bf_mode(net)) {
    EncoderPass<__bf16> en;
    en.carve(cv, enc, B);
  } else {
    EncoderPass<float> en;
    en.carve(cv, enc, B);
  }
  *bytes = cv.off + 256;
  return CROM_OK;
}

crom_status crom_encode(const crom_net* net, const crom_encoder* enc, const float* u, int32_t B, float* q, void* ws,
                        size_t ws_bytes, void* stream) {
  size_t need = 0;
  crom_status s = crom_encode_workspace(net, enc, B, &need);
  if (s != CROM_OK) return s;
  if (!u || !q || !ws) return fail(CROM_ERR_INVALID_ARG, "u, q and ws are required");
  if (ws_bytes < need) return fail(CROM_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carve cv{reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255)), 0};
  if (enc->kind == CROM_ENC_CONV) {
    const ConvShape c = conv_of(net, enc);
    ConvPass cp;
    cp.carve(cv, c, B);
    if ((s = conv_encoder_fwd(c, enc->params, u, B, cp, st)) != CROM_OK) return s;
    return hip_check(hipMemcpyAsync(q, cp.q, sizeof(float) * B * enc->r, hipMemcpyDeviceToDevice, st), "q copy");
  }
  if (bf_mode(net)) {
    EncoderPass<__bf16> en;
    en.carve(cv, enc, B);
    if ((s = encoder_fwd<__bf16>(enc, u, B, en, st)) != CROM_OK) return s;
    return hip_check(hipMemcpyAsync(q, en.q, sizeof(float) * B * enc->r, hipMemcpyDeviceToDevice, st), "q copy");
  }
  EncoderPass<float> en;
  en.carve(cv, enc, B);
  if ((s = encoder_fwd<float>(enc, u, B, en, st)) != CROM_OK) return s;
  return hip_check(hipMemcpyAsync(q, en.q, sizeof(float) * B * enc->r, hipMemcpyDeviceToDevice, st), "q copy");
}

crom_status crom_decode_vjp_workspace(const crom_net* net, int32_t B, int64_t P, size_t* bytes) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (net->act != CROM_ACT_ELU &&
      (net->act != CROM_ACT_SINE || net->precision == CROM_PREC_FP32 || (net->width != 32 && net->width != 128)))
    return fail(CROM_ERR_UNSUPPORTED, "training kernels: ELU networks, or sine networks of width 32 or 128 in bfloat16");
  if (B < 1 || P < 1 || !bytes) return fail(CROM_ERR_INVALID_ARG, "B >= 1, P >= 1 and bytes are required");
  *bytes = (bf_mode(net) ? DecoderPass<__bf16>::bytes(net, B, P) : DecoderPass<float>::bytes(net, B, P)) + 256;
  return CROM_OK;
}

crom_status crom_decode_vjp(const crom_net* net, const float* x, int64_t P, const float* q, int32_t B,
                            const float* dg, float* grad_params, float* grad_q, void* ws, size_t ws_bytes,
                            void* stream) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (net->act != CROM_ACT_ELU &&
      (net->act != CROM_ACT_SINE || net->precision == CROM_PREC_FP32 || (net->width != 32 && net->width != 128)))
    return fail(CROM_ERR_UNSUPPORTED, "training kernels: ELU networks, or sine networks of width 32 or 128 in bfloat16");
  if (B < 1 || P < 1) return fail(CROM_ERR_INVALID_ARG, "B >= 1 and P >= 1");
  if (!x || !q || !dg || !grad_params || !grad_q || !ws)
    return fail(CROM_ERR_INVALID_ARG, "x, q, dg, grad_params, grad_q and ws are required");
  size_t need = 0;
  crom_decode_vjp_workspace(net, B, P, &need);
  if (ws_bytes < need) return fail(CROM_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carve cv{reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255)), 0};
  if (bf_mode(net)) {
    DecoderPass<__bf16> d;
    d.carve(cv, net, B, P);
    return decoder_fwd_bwd<__bf16>(net, x, B, P, q, nullptr, dg, grad_params, grad_q, nullptr, d, st);
  }
  DecoderPass<float> d;
  d.carve(cv, net, B, P);
  return decoder_fwd_bwd<float>(net, x, B, P, q, nullptr, dg, grad_params, grad_q, nullptr, d, st);
}

}  // extern "C"
