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

// Row GEMM for the decoder's square hidden layers in bfloat16 (W <= 128):
//   forward   C[row][m] = ELU(sum_k Wt[m][k] X[row][k] + bias[m])
//   backward  C[row][m] = (sum_k X[row][k] Wt[k][m]) * ELU'(gate[row][m])
// The layer's output units are the MFMA M dimension and the rows its N
// dimension: the weight matrix is staged once per workgroup in LDS in
// A-operand fragment order (one contiguous 16-byte read per lane and
// fragment), 16-row tiles of X stream straight from memory as B-operand
// fragments (16 contiguous bytes per lane), and each lane ends with 4
// consecutive output units of one row, stored as one 8-byte write.  Waves
// loop over row tiles with the next tile's operands loaded ahead; few
// registers, so many waves per CU keep memory busy.  Same operands, K order
// and epilogue arithmetic as gemm_kernel.
// Sine (SIREN) networks: the forward writes a = sin(z) and the derivative
// cos(z) (G), and the backward's gate is that stored derivative.
struct RowGemmArgs {
  const __bf16* X;     // [rows][W]
  const __bf16* Wt;    // [W][W] bfloat16 copy of the layer weight (out, in)
  const float* bias;   // forward
  const __bf16* gate;  // backward: stored a = ELU(z) (ELU) or cos(z) (sine) of the layer below
  __bf16* C;           // [rows][W]
  int64_t rows;
  __bf16* G;           // forward, sine: cos(z) [rows][W]
};

template <int W, bool FWD, bool SINE = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void rowgemm_kernel(RowGemmArgs g) {
  typedef __bf16 bf16x8_ __attribute__((ext_vector_type(8)));
  typedef __bf16 bf16x4_ __attribute__((ext_vector_type(4)));
  typedef float f32x4_ __attribute__((ext_vector_type(4)));
  static_assert(W % 32 == 0 && W <= 128, "one weight matrix per workgroup in LDS");
  constexpr int MT = W / 16, KB = W / 32;
  __shared__ float sb[W];
  __shared__ __align__(16) bf16x8_ frag[MT * KB * 64];  // [i][kb][lane]
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  if constexpr (FWD) {
    for (int i = threadIdx.x; i < W; i += blockDim.x) sb[i] = g.bias[i];
  }
  // fragment (i, kb) of lane l: unit m = 16 i + (l & 15), inputs k = 32 kb + 8 (l >> 4) + e
  for (int f = threadIdx.x; f < MT * KB * 64; f += blockDim.x) {
    const int l = f & 63, ikb = f >> 6, i = ikb / KB, kb = ikb % KB;
    const int m = 16 * i + (l & 15), k = 32 * kb + 8 * (l >> 4);
    if constexpr (FWD) {
      frag[f] = *reinterpret_cast<const bf16x8_*>(&g.Wt[m * W + k]);
    } else {
      bf16x8_ v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = g.Wt[(k + e) * W + m];
      frag[f] = v;
    }
  }
  __syncthreads();
  const int64_t ntiles = (g.rows + 15) / 16;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  bf16x8_ bx[KB];
  const bf16x8_ zero8 = {};
  auto load_tile = [&](int64_t tt) {
    const int64_t row = tt * 16 + lr;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      bx[kb] = row < g.rows ? *reinterpret_cast<const bf16x8_*>(&g.X[row * W + 32 * kb + 8 * lg]) : zero8;
  };
  if (t < ntiles) load_tile(t);
  for (; t < ntiles; t += nw) {
    // keep the weight fragments in LDS (read per tile) rather than hoisted
    // into registers: the occupancy is what keeps memory busy
    asm volatile("" ::: "memory");
    bf16x8_ cur[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) cur[kb] = bx[kb];
    const int64_t row = t * 16 + lr;
    if (t + nw < ntiles) load_tile(t + nw);  // next tile in flight during this one
    f32x4_ acc[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) acc[i] = f32x4_{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int i = 0; i < MT; ++i)
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag[(i * KB + kb) * 64 + lane], cur[kb], acc[i], 0, 0, 0);
    bf16x4_ gv[MT];
    if constexpr (!FWD) {
      const bf16x4_ zero4 = {};
#pragma unroll
      for (int i = 0; i < MT; ++i)
        gv[i] = row < g.rows ? *reinterpret_cast<const bf16x4_*>(&g.gate[row * W + 16 * i + 4 * lg]) : zero4;
    }
    if (row < g.rows) {
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const int m0 = 16 * i + 4 * lg;  // this lane's 4 consecutive units
        bf16x4_ o, oc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float x = acc[i][v];
          if constexpr (FWD && SINE) {
            const float rz = reduce_2pi(x + sb[m0 + v]);
            x = __sinf(rz);
            oc[v] = (__bf16)__cosf(rz);
          } else if constexpr (FWD) {
            x += sb[m0 + v];
            x = x > 0.0f ? x : __expf(x) - 1.0f;
          } else if constexpr (SINE) {
            x *= (float)gv[i][v];
          } else {
            x *= elu_d1_from_a((float)gv[i][v]);
          }
          o[v] = (__bf16)x;
        }
        *reinterpret_cast<bf16x4_*>(&g.C[row * W + m0]) = o;
        if constexpr (FWD && SINE) *reinterpret_cast<bf16x4_*>(&g.G[row * W + m0]) = oc;
      }
    }
  }
}

// Weight gradient of a square hidden layer in bfloat16 (W = 128): partial
//   part[blk][m][n] = sum over the workgroup's rows r of X[r][m] Y[r][n]
// (X = dz of the layer, Y = the stored activations below it), K = rows.
// Each 32-row step of both operands is staged row-major in LDS with 16-byte
// writes, and the MFMA fragments (8 consecutive rows of one column per lane)
// come from LDS transpose reads (ds_read_b64_tr_b16: lane i of a 16-lane
// group receives column i of the 4 x 16 block its group addresses, 4 rows);
// the next step's rows load from memory while this step multiplies.  Four
// waves each own a 64 x 64 quadrant of the output; the partial tiles are
// summed in workgroup order by splitk_reduce_kernel.
template <int W>
__global__ __launch_bounds__(256) void wgrad_kernel(const __bf16* __restrict__ X, const __bf16* __restrict__ Y,
                                                    int64_t rows, int64_t rows_per_blk, float* __restrict__ part) {
  typedef __bf16 bf16x8_ __attribute__((ext_vector_type(8)));
  typedef short s16x4_ __attribute__((ext_vector_type(4)));
  typedef short s16x8_ __attribute__((ext_vector_type(8)));
  typedef float f32x4_ __attribute__((ext_vector_type(4)));
  static_assert(W == 128, "four 64 x 64 quadrants");
  constexpr int KS = 32;       // rows per step
  constexpr int LDR = W + 16;  // padded LDS row (elements)
  constexpr int CH = KS * W / 8;  // 16-byte chunks per operand and step
  __shared__ __align__(16) __bf16 xs[2][KS * LDR];
  __shared__ __align__(16) __bf16 ys[2][KS * LDR];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lg = lane >> 4, lj = lane & 15;
  const int mq = (wave >> 1) * 64, nq = (wave & 1) * 64;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < rows ? r0 + rows_per_blk : rows;
  f32x4_ acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_{0.0f, 0.0f, 0.0f, 0.0f};
  constexpr int PER = CH / 256;  // chunks per thread and operand
  bf16x8_ rx[PER], ry[PER];
  const bf16x8_ zero8 = {};
  auto load = [&](int64_t rb) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int c = threadIdx.x + 256 * u;
      const int rr = c / (W / 8), cc = (c % (W / 8)) * 8;
      const int64_t row = rb + rr;
      rx[u] = row < r1 ? *reinterpret_cast<const bf16x8_*>(&X[row * W + cc]) : zero8;
      ry[u] = row < r1 ? *reinterpret_cast<const bf16x8_*>(&Y[row * W + cc]) : zero8;
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int c = threadIdx.x + 256 * u;
      const int rr = c / (W / 8), cc = (c % (W / 8)) * 8;
      *reinterpret_cast<bf16x8_*>(&xs[b][rr * LDR + cc]) = rx[u];
      *reinterpret_cast<bf16x8_*>(&ys[b][rr * LDR + cc]) = ry[u];
    }
  };
  // fragment of 16 columns from c0: lane (lg, lj) receives rows 8 lg .. 8 lg + 7 of column c0 + lj
  auto frag = [&](const __bf16* T, int c0) {
    const __bf16* p = T + (8 * lg + (lj >> 2)) * LDR + c0 + 4 * (lj & 3);
    const s16x4_ lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
        (__attribute__((address_space(3))) s16x4_*)(p));
    const s16x4_ hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
        (__attribute__((address_space(3))) s16x4_*)(p + 4 * LDR));
    const s16x8_ v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(bf16x8_, v);
  };
  if (r0 < r1) {
    load(r0);
    store(0);
  }
  __syncthreads();
  int b = 0;
  for (int64_t rb = r0; rb < r1; rb += KS) {
    const bool more = rb + KS < r1;
    if (more) load(rb + KS);  // next step's rows in flight during this step's products
    bf16x8_ af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = frag(xs[b], mq + 16 * i);
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[j] = frag(ys[b], nq + 16 * j);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    if (more) store(b ^ 1);
    __syncthreads();  // this step's buffer is read and the next one written
    b ^= 1;
  }
  float* P = part + (size_t)blockIdx.x * W * W;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) P[(mq + 16 * i + 4 * lg + v) * W + nq + 16 * j + lj] = acc[i][j][v];
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
