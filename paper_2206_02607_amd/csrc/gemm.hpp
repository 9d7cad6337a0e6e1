// LDS-tiled matrix-core GEMM with fused epilogues, the building block of the
// training kernels:  C[M][N] = op(A)[M][K] * op(B)[K][N]  (+ epilogue)
//   op(A)(m, k) = TA ? A[k * lda + m] : A[m * lda + k]
//   op(B)(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n]
// T = __bf16 (v_mfma_f32_16x16x32_bf16) or float (v_mfma_f32_16x16x4_f32);
// accumulation is FP32.  Block tile 64 x 64 (K tile 64 in bfloat16, 32 in FP32), four waves of
// 32 x 32.  Split-K
// writes FP32 partial tiles that a second kernel sums in a fixed order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crom {

enum { EPI_NONE = 0, EPI_BIAS_ELU = 1, EPI_DELU = 2, EPI_BIAS = 3 };

struct GemmArgs {
  int M, N, K;
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  float* C;         // FP32 result (may be NULL)
  int64_t ldc;
  __bf16* Cb;       // bfloat16 copy of the result (may be NULL)
  int64_t ldcb;
  const float* bias;  // EPI_BIAS_ELU / EPI_BIAS: + bias[n]
  const void* gate;   // EPI_DELU: result *= ELU'(z) read from the stored a = ELU(z)
  int64_t ldg;
  int kchunk;         // split-K: K range of blockIdx.z (multiple of the K tile)
  float* part;        // split-K: partial tiles [gridDim.z][M][N]
  int accumulate;     // C += result (FP32 output only)
};

template <class T>
__device__ __forceinline__ float to_f(T v) { return (float)v; }

// ELU'(z) from a = ELU(z): 1 where a > 0, a + 1 = e^z otherwise.
__device__ __forceinline__ float elu_d1_from_a(float a) { return a > 0.0f ? 1.0f : a + 1.0f; }

template <class T, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  typedef __bf16 bf16x8_ __attribute__((ext_vector_type(8)));
  typedef float f32x4_ __attribute__((ext_vector_type(4)));
  constexpr bool BF = sizeof(T) == 2;
  constexpr int BK = BF ? 64 : 32;
  constexpr int LDK = BK + (BF ? 8 : 4);  // padded row (k contiguous) against bank conflicts
  __shared__ __align__(16) T As[64 * LDK];
  __shared__ __align__(16) T Bs[64 * LDK];
  const T* A = static_cast<const T*>(g.A);
  const T* B = static_cast<const T*>(g.B);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  f32x4_ acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_{0.0f, 0.0f, 0.0f, 0.0f};

  constexpr int VEC = 16 / (int)sizeof(T);  // elements per 16-byte load
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // Stage the A tile (rows m, k) and the B tile (columns n, k) into LDS,
    // k contiguous, with 16-byte loads along each operand's contiguous
    // direction; ragged edges (and unaligned rows) load element by element
    // and fill zeros outside the matrix.
    if constexpr (!TA) {
      for (int v = tid; v < 64 * BK / VEC; v += 256) {
        const int r = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        const int gm = m0 + r, gk = k0 + kk;
        const T* src = A + (int64_t)gm * g.lda + gk;
        if (gm < g.M && gk + VEC <= kend && ((uintptr_t)src & 15) == 0) {
          *reinterpret_cast<vec_t*>(&As[r * LDK + kk]) = *reinterpret_cast<const vec_t*>(src);
        } else {
#pragma unroll
          for (int i = 0; i < VEC; ++i)
            As[r * LDK + kk + i] = (gm < g.M && gk + i < kend) ? src[i] : T(0.0f);
        }
      }
    } else {
      for (int v = tid; v < BK * 64 / VEC; v += 256) {
        const int k = v / (64 / VEC), rr = (v % (64 / VEC)) * VEC;
        const int gk = k0 + k, gm = m0 + rr;
        const T* src = A + (int64_t)gk * g.lda + gm;
        if (gk < kend && gm + VEC <= g.M && ((uintptr_t)src & 15) == 0) {
          const vec_t e = *reinterpret_cast<const vec_t*>(src);
#pragma unroll
          for (int i = 0; i < VEC; ++i) As[(rr + i) * LDK + k] = e[i];
        } else {
#pragma unroll
          for (int i = 0; i < VEC; ++i)
            As[(rr + i) * LDK + k] = (gk < kend && gm + i < g.M) ? src[i] : T(0.0f);
        }
      }
    }
    if constexpr (TB) {
      for (int v = tid; v < 64 * BK / VEC; v += 256) {
        const int c = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        const int gn = n0 + c, gk = k0 + kk;
        const T* src = B + (int64_t)gn * g.ldb + gk;
        if (gn < g.N && gk + VEC <= kend && ((uintptr_t)src & 15) == 0) {
          *reinterpret_cast<vec_t*>(&Bs[c * LDK + kk]) = *reinterpret_cast<const vec_t*>(src);
        } else {
#pragma unroll
          for (int i = 0; i < VEC; ++i)
            Bs[c * LDK + kk + i] = (gn < g.N && gk + i < kend) ? src[i] : T(0.0f);
        }
      }
    } else {
      for (int v = tid; v < BK * 64 / VEC; v += 256) {
        const int k = v / (64 / VEC), cc = (v % (64 / VEC)) * VEC;
        const int gk = k0 + k, gn = n0 + cc;
        const T* src = B + (int64_t)gk * g.ldb + gn;
        if (gk < kend && gn + VEC <= g.N && ((uintptr_t)src & 15) == 0) {
          const vec_t e = *reinterpret_cast<const vec_t*>(src);
#pragma unroll
          for (int i = 0; i < VEC; ++i) Bs[(cc + i) * LDK + k] = e[i];
        } else {
#pragma unroll
          for (int i = 0; i < VEC; ++i)
            Bs[(cc + i) * LDK + k] = (gk < kend && gn + i < g.N) ? src[i] : T(0.0f);
        }
      }
    }
    __syncthreads();
    if constexpr (BF) {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 32) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const bf16x8_ af =
              *reinterpret_cast<const bf16x8_*>(&As[(wr + i * 16 + (lane & 15)) * LDK + ks + 8 * (lane >> 4)]);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const bf16x8_ bfr =
                *reinterpret_cast<const bf16x8_*>(&Bs[(wc + j * 16 + (lane & 15)) * LDK + ks + 8 * (lane >> 4)]);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[i][j], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float af = to_f(As[(wr + i * 16 + (lane & 15)) * LDK + ks + (lane >> 4)]);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const float bfr = to_f(Bs[(wc + j * 16 + (lane & 15)) * LDK + ks + (lane >> 4)]);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bfr, acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // epilogue: lane holds column (lane & 15), rows 4 * (lane >> 4) + v
  const T* gate = static_cast<const T*>(g.gate);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wr + i * 16 + 4 * (lane >> 4) + v;
        const int n = n0 + wc + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float x = acc[i][j][v];
        if (g.part) {
          g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = x;
          continue;
        }
        if constexpr (EPI == EPI_BIAS_ELU) {
          x += g.bias[n];
          x = x > 0.0f ? x : __expf(x) - 1.0f;
        } else if constexpr (EPI == EPI_BIAS) {
          x += g.bias[n];
        } else if constexpr (EPI == EPI_DELU) {
          x *= elu_d1_from_a(to_f(gate[(int64_t)m * g.ldg + n]));
        }
        if (g.C) {
          float* c = &g.C[(int64_t)m * g.ldc + n];
          *c = g.accumulate ? *c + x : x;
        }
        if (g.Cb) g.Cb[(int64_t)m * g.ldcb + n] = (__bf16)x;
      }
}

// Sum of split-K partials, then the epilogue (none, bias, or bias + ELU)
// and the FP32 store.  A block takes 64 outputs; each of its 4 lanes per
// output adds the splits z = lane, lane + 4, ... in order, and the 4 lane
// sums are added in lane order (a fixed order: the result is deterministic).
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* __restrict__ part, int splits, int M, int N,
                                                            float* C, int64_t ldc, int accumulate, int epi,
                                                            const float* __restrict__ bias) {
  __shared__ float sh[4][64];
  const int64_t MN = (int64_t)M * N;
  const int64_t e = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int l4 = threadIdx.x >> 6;
  float s = 0.0f;
  if (e < MN) {
#pragma unroll 8
    for (int z = l4; z < splits; z += 4) s += part[(int64_t)z * MN + e];
  }
  sh[l4][threadIdx.x & 63] = s;
  __syncthreads();
  if (threadIdx.x < 64 && e < MN) {
    float t = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
    const int m = (int)(e / N), n = (int)(e % N);
    if (epi == EPI_BIAS || epi == EPI_BIAS_ELU) t += bias[n];
    if (epi == EPI_BIAS_ELU) t = t > 0.0f ? t : __expf(t) - 1.0f;
    float* c = &C[(int64_t)m * ldc + n];
    *c = accumulate ? *c + t : t;
  }
}

}  // namespace crom
