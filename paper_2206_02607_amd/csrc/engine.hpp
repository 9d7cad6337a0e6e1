// Fused decoder engine for gfx950: the MLP g(x, q) evaluated together with
// forward-mode derivative columns, one workgroup per batch of points.
//
// What is computed (Sec. "Network Details"; Alg. "Network gradient" of
// Sec. "Network Gradients via Direct Differentiation", extended to second
// order in x and to the latent directions):
//   z_l = W_l a_{l-1} + b_l,  a_l = ELU(z_l)          value column
//   dz_l = W_l da_{l-1},      da_l = s1(z_l) dz_l      tangent columns (x_i, q_k)
//   D2z_l = W_l D2a_{l-1},    D2a_l = s2(z_l) dz_i dz_j + s1(z_l) D2z_l
// with s1 = ELU', s2 = ELU''; the Laplacian column carries sum_i of the
// diagonal second derivatives in one column (s2 * sum_i dz_i^2 + s1 * D2z).
// The first layer is folded: W_1 [x; q] + b_1 = W_1x x + c with the per-
// latent bias c = W_1q q + b_1 (FP64), so its tangents are columns of W_1
// and its second derivatives are zero.  The output layer is linear.
//
// Layout.  Points are the MFMA N dimension, 16 points per N-tile; every
// derivative column of a batch of 16 points is one more N-tile, so the
// epilogue coupling (s1, s2 of the value column scale the tangent columns of
// the same unit and point) stays inside one lane.  Output units are the M
// dimension, 16 per M-tile, split over the workgroup's waves.  The hidden
// activations of the batch live in LDS in the exact B-operand fragment
// order of v_mfma_f32_16x16x32_bf16 (or x4_f32), and the packed weights in
// the A-operand fragment order, so every operand load is one contiguous
// 16-byte read per lane.  The K order inside a fragment is permuted so that
// a lane writes back exactly the units it holds after the MFMA
// (unit = 16 * mtile + 4 * (lane / 16) + v for accumulator v).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crom {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int PT = 16;  // points per N-tile

enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };
enum { CK_VAL = 0, CK_XT = 1, CK_LAP = 2, CK_HESS = 3, CK_QT = 4 };
enum { D2_NONE = 0, D2_LAP = 1, D2_HESS = 2 };

template <int W_, int M_, int R_, int D_>
struct Shape {
  static constexpr int W = W_, M = M_, R = R_, D = D_;
  static constexpr int MTILES = W_ / 16;
  static constexpr int N0 = M_ + R_;
};

// Columns of one batch of 16 points: NV value columns (value 0 is the point
// the derivative columns belong to; values 1.. are extra latents, e.g. line-
// search trials), then the x tangents, the second-derivative columns and
// NQ latent tangents (latent indices qb .. qb+NQ-1, qb given at run time).
template <int M_, int R_, int NV_, bool XT_, int D2_, int NQ_>
struct Cols {
  static constexpr int M = M_, R = R_, NV = NV_, D2 = D2_;
  static constexpr int NX = (XT_ || D2_ != D2_NONE) ? M_ : 0;
  static constexpr int ND2 = D2_ == D2_LAP ? 1 : (D2_ == D2_HESS ? M_ * (M_ + 1) / 2 : 0);
  static constexpr int NQ = NQ_;
  static constexpr int C = NV + NX + ND2 + NQ;
  static constexpr int X0 = NV, D0 = NV + NX, Q0 = NV + NX + ND2;
  __host__ __device__ static constexpr int kind(int c) {
    return c < X0 ? CK_VAL : c < D0 ? CK_XT : c < Q0 ? (D2_ == D2_LAP ? CK_LAP : CK_HESS) : CK_QT;
  }
  // Hessian column k -> (i, j), upper triangle i <= j, row-major.
  __host__ __device__ static constexpr int hess_i(int k) {
    int i = 0, n = M_;
    while (k >= n) { k -= n; ++i; --n; }
    return i;
  }
  __host__ __device__ static constexpr int hess_j(int k) {
    int i = 0, n = M_;
    while (k >= n) { k -= n; ++i; --n; }
    return i + k;
  }
};

template <class S, int PREC>
struct Packing {
  // bf16: per hidden layer, [mtile][kb = W/32][lane][8] hi fragments, then
  // the same again for the lo part (W - hi rounded to bf16).
  // fp32: per hidden layer, [mtile][kq = W/16][lane][4].
  static constexpr int KQ = PREC == PREC_FP32 ? S::W / 16 : S::W / 32;
  static constexpr size_t FRAG_BYTES = 64 * 16;
  static constexpr size_t LAYER_BYTES =
      (size_t)S::MTILES * KQ * FRAG_BYTES * (PREC == PREC_FP32 ? 1 : 2);
};

// Offsets of each layer's W and b inside the natural FP32 parameter array.
struct ParamIndex {
  int64_t w[16], b[16];
};

__device__ __forceinline__ float elu_exp(float z) { return __expf(fminf(z, 0.0f)); }

// All per-batch tables live in one dynamic LDS block:
//   act    activations (fragment order), NT (+ lo tiles) tiles
//   xs     [NB*16][M] points (FP32)
//   fold   [NV][W] per-latent first-layer bias (FP32)
//   res    [D][NT][16] outputs (FP32)
// The cross-wave output reduction reuses `act`.
template <class S, class C, int NB, int NW, int PREC>
struct Engine {
  static constexpr int W = S::W, M = S::M, R = S::R, D = S::D;
  static constexpr int CC = C::C;
  static constexpr int NT = NB * CC;
  static constexpr int NVT = NB * C::NV;  // value tiles (split in BF16X3)
  static constexpr int MTILES = S::MTILES;
  static constexpr int MT = MTILES / NW;
  static_assert(MTILES % NW == 0, "waves must split the M-tiles evenly");
  static constexpr int NPTS = NB * PT;
  static constexpr bool SPLIT = PREC == PREC_BF16X3;
  static constexpr int KQ = Packing<S, PREC>::KQ;
  // activation tiles: every column, plus a lo tile per value column in split mode
  static constexpr int NACT = NT + (SPLIT ? NVT : 0);
  static constexpr int ACT_BYTES = NACT * KQ * 64 * 16;
  static constexpr int RED_BYTES = NW * D * NT * PT * 4;
  static constexpr int ACT_REGION = ACT_BYTES > RED_BYTES ? ACT_BYTES : RED_BYTES;
  static constexpr int XS_OFF = ACT_REGION;
  static constexpr int FOLD_OFF = XS_OFF + ((NPTS * M * 4 + 15) / 16) * 16;
  static constexpr int RES_OFF = FOLD_OFF + C::NV * W * 4;
  static constexpr int LDS_BYTES = RES_OFF + D * NT * PT * 4;
  static constexpr int THREADS = NW * 64;

  static __device__ __forceinline__ int tile_of(int b, int c) { return b * CC + c; }
  // lo tile of value tile (b, v) in split mode
  static __device__ __forceinline__ int lo_tile(int b, int v) { return NT + b * C::NV + v; }

  // ---- stage points and per-latent fold -------------------------------
  // Points first .. first+n_valid-1 of x (n_valid <= NPTS; the rest of the
  // batch is padded with x = 0); lat: NV latent vectors, vector v at
  // lat + v * lat_stride, FP64.
  static __device__ void stage(char* lds, const float* __restrict__ x, int64_t first, int n_valid,
                               const double* __restrict__ lat, int lat_stride,
                               const float* __restrict__ params, const ParamIndex& pi) {
    float* xs = reinterpret_cast<float*>(lds + XS_OFF);
    for (int i = threadIdx.x; i < NPTS * M; i += THREADS) {
      int p = i / M;
      xs[i] = p < n_valid ? x[(first + p) * M + (i - p * M)] : 0.0f;
    }
    float* fold = reinterpret_cast<float*>(lds + FOLD_OFF);
    const float* W1 = params + pi.w[0];
    const float* b1 = params + pi.b[0];
    for (int i = threadIdx.x; i < C::NV * W; i += THREADS) {
      int v = i / W, u = i - v * W;
      double s = (double)b1[u];
#pragma unroll
      for (int k = 0; k < R; ++k) s += (double)W1[u * (M + R) + M + k] * lat[v * lat_stride + k];
      fold[i] = (float)s;
    }
  }

  // ---- epilogue ---------------------------------------------------------
  // z[t] -> o[t] for one (unit, lane) across all tiles.
  static __device__ __forceinline__ void epilogue(const float (&z)[NT], float (&o)[NT]) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      float s1 = 1.0f, s2 = 0.0f;
#pragma unroll
      for (int c = 0; c < C::NV; ++c) {
        const float zz = z[b * CC + c];
        const float e = elu_exp(zz);
        const bool pos = zz > 0.0f;
        o[b * CC + c] = pos ? zz : e - 1.0f;
        if (c == 0) {
          s1 = pos ? 1.0f : e;
          s2 = pos ? 0.0f : e;
        }
      }
#pragma unroll
      for (int c = C::X0; c < C::D0; ++c) o[b * CC + c] = s1 * z[b * CC + c];
      if constexpr (C::D2 == D2_LAP) {
        float sq = 0.0f;
#pragma unroll
        for (int i = 0; i < C::NX; ++i) sq += z[b * CC + C::X0 + i] * z[b * CC + C::X0 + i];
        o[b * CC + C::D0] = s1 * z[b * CC + C::D0] + s2 * sq;
      } else if constexpr (C::D2 == D2_HESS) {
#pragma unroll
        for (int k = 0; k < C::ND2; ++k) {
          const float zi = z[b * CC + C::X0 + C::hess_i(k)];
          const float zj = z[b * CC + C::X0 + C::hess_j(k)];
          o[b * CC + C::D0 + k] = s1 * z[b * CC + C::D0 + k] + s2 * zi * zj;
        }
      }
#pragma unroll
      for (int c = C::Q0; c < CC; ++c) o[b * CC + c] = s1 * z[b * CC + c];
    }
  }

  // ---- write one M-tile of activations (all tiles, 4 units per lane) ----
  static __device__ __forceinline__ void write_act(char* lds, int mtg, int lane,
                                                   const float (&o)[NT][4]) {
    if constexpr (PREC == PREC_FP32) {
      f32x4* act = reinterpret_cast<f32x4*>(lds);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f32x4 v = {o[t][0], o[t][1], o[t][2], o[t][3]};
        act[(t * KQ + mtg) * 64 + lane] = v;
      }
    } else {
      // fragment (t, kb = mtg/2), element offset (mtg%2)*4
      bf16x4* act = reinterpret_cast<bf16x4*>(lds);
      const int half = mtg & 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        bf16x4 h;
        h[0] = (__bf16)o[t][0];
        h[1] = (__bf16)o[t][1];
        h[2] = (__bf16)o[t][2];
        h[3] = (__bf16)o[t][3];
        act[((t * KQ + (mtg >> 1)) * 64 + lane) * 2 + half] = h;
        if constexpr (SPLIT) {
          const int b = t / CC, c = t - (t / CC) * CC;
          if (c < C::NV) {
            bf16x4 l;
            l[0] = (__bf16)(o[t][0] - (float)h[0]);
            l[1] = (__bf16)(o[t][1] - (float)h[1]);
            l[2] = (__bf16)(o[t][2] - (float)h[2]);
            l[3] = (__bf16)(o[t][3] - (float)h[3]);
            act[((lo_tile(b, c) * KQ + (mtg >> 1)) * 64 + lane) * 2 + half] = l;
          }
        }
      }
    }
  }

  // ---- output layer partial sums for one M-tile --------------------------
  static __device__ __forceinline__ void out_accum(float (&part)[D][NT], const float (&o)[NT][4],
                                                   const float* __restrict__ Wout, int ubase) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int oo = 0; oo < D; ++oo) {
        const float w = Wout[oo * W + ubase + v];
#pragma unroll
        for (int t = 0; t < NT; ++t) part[oo][t] += w * o[t][v];
      }
    }
  }

  // ---- the whole network for one batch -----------------------------------
  // Leaves the outputs in res[D][NT][16]; all threads must call it.
  static __device__ void run(char* lds, const float* __restrict__ params, const ParamIndex& pi,
                             const char* __restrict__ packed, int depth, int qb) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    const float* xs = reinterpret_cast<const float*>(lds + XS_OFF);
    const float* fold = reinterpret_cast<const float*>(lds + FOLD_OFF);
    float part[D][NT];
#pragma unroll
    for (int oo = 0; oo < D; ++oo)
#pragma unroll
      for (int t = 0; t < NT; ++t) part[oo][t] = 0.0f;
    const float* Wout = params + pi.w[depth];

    // ---------------- layer 1 (VALU, folded) ----------------
    {
      const float* W1 = params + pi.w[0];
      float xr[NB][M];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < M; ++i) xr[b][i] = xs[(b * PT + j) * M + i];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int mtg = wave * MT + mt;
        float o4[NT][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int u = mtg * 16 + g * 4 + v;
          float wx[M];
#pragma unroll
          for (int i = 0; i < M; ++i) wx[i] = W1[u * (M + R) + i];
          float z[NT], o[NT];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            float lin = 0.0f;
#pragma unroll
            for (int i = 0; i < M; ++i) lin += wx[i] * xr[b][i];
#pragma unroll
            for (int c = 0; c < CC; ++c) {
              const int k = C::kind(c);
              float val;
              if (k == CK_VAL) val = lin + fold[c * W + u];
              else if (k == CK_XT) val = wx[c - C::X0];
              else if (k == CK_QT) val = W1[u * (M + R) + M + qb + (c - C::Q0)];
              else val = 0.0f;
              z[b * CC + c] = val;
            }
          }
          epilogue(z, o);
#pragma unroll
          for (int t = 0; t < NT; ++t) o4[t][v] = o[t];
        }
        if (depth > 1) write_act(lds, mtg, lane, o4);
        else out_accum(part, o4, Wout, mtg * 16 + g * 4);
      }
    }
    __syncthreads();

    // ---------------- hidden layers 2..depth (MFMA) ----------------
    for (int h = 0; h < depth - 1; ++h) {
      const char* wl = packed + (size_t)h * Packing<S, PREC>::LAYER_BYTES;
      const float* bias = params + pi.b[h + 1];
      f32x4 acc[MT][NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int mtg = wave * MT + mt;
        const float* bp = bias + mtg * 16 + g * 4;  // not 16-byte aligned in general
        const f32x4 bv = {bp[0], bp[1], bp[2], bp[3]};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bool isval = (t % CC) < C::NV;
          acc[mt][t] = isval ? bv : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
      }
      if constexpr (PREC == PREC_FP32) {
        const f32x4* act = reinterpret_cast<const f32x4*>(lds);
        const f32x4* wf = reinterpret_cast<const f32x4*>(wl);
#pragma unroll 2
        for (int kq = 0; kq < KQ; ++kq) {
          f32x4 a[MT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) a[mt] = wf[((wave * MT + mt) * KQ + kq) * 64 + lane];
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const f32x4 bfr = act[(t * KQ + kq) * 64 + lane];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
              acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt][0], bfr[0], acc[mt][t], 0, 0, 0);
              acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt][1], bfr[1], acc[mt][t], 0, 0, 0);
              acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt][2], bfr[2], acc[mt][t], 0, 0, 0);
              acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt][3], bfr[3], acc[mt][t], 0, 0, 0);
            }
          }
        }
      } else {
        const bf16x8* act = reinterpret_cast<const bf16x8*>(lds);
        const bf16x8* wf = reinterpret_cast<const bf16x8*>(wl);
        constexpr int LO = MTILES * KQ * 64;  // offset of the lo fragments
#pragma unroll 2
        for (int kb = 0; kb < KQ; ++kb) {
          bf16x8 a[MT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) a[mt] = wf[((wave * MT + mt) * KQ + kb) * 64 + lane];
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const bf16x8 bfr = act[(t * KQ + kb) * 64 + lane];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
              acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bfr, acc[mt][t], 0, 0, 0);
          }
          if constexpr (SPLIT) {
            bf16x8 al[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) al[mt] = wf[LO + ((wave * MT + mt) * KQ + kb) * 64 + lane];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
              for (int v = 0; v < C::NV; ++v) {
                const int t = b * CC + v;
                const bf16x8 bh = act[(t * KQ + kb) * 64 + lane];
                const bf16x8 bl = act[(lo_tile(b, v) * KQ + kb) * 64 + lane];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                  acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bl, acc[mt][t], 0, 0, 0);
                  acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bh, acc[mt][t], 0, 0, 0);
                }
              }
            }
          }
        }
      }
      __syncthreads();  // every wave has read this layer's activations
      const bool last = (h == depth - 2);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int mtg = wave * MT + mt;
        float o4[NT][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float z[NT], o[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) z[t] = acc[mt][t][v];
          epilogue(z, o);
#pragma unroll
          for (int t = 0; t < NT; ++t) o4[t][v] = o[t];
        }
        if (!last) write_act(lds, mtg, lane, o4);
        else out_accum(part, o4, Wout, mtg * 16 + g * 4);
      }
      __syncthreads();
    }

    // ---------------- output layer: reduce partial dot products ----------
#pragma unroll
    for (int oo = 0; oo < D; ++oo)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        float s = part[oo][t];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        part[oo][t] = s;
      }
    float* red = reinterpret_cast<float*>(lds);
    if (g == 0) {
#pragma unroll
      for (int oo = 0; oo < D; ++oo)
#pragma unroll
        for (int t = 0; t < NT; ++t) red[((wave * D + oo) * NT + t) * PT + j] = part[oo][t];
    }
    __syncthreads();
    float* res = reinterpret_cast<float*>(lds + RES_OFF);
    const float* bout = params + pi.b[depth];
    for (int i = threadIdx.x; i < D * NT * PT; i += THREADS) {
      const int oo = i / (NT * PT);
      const int t = (i / PT) % NT;
      float s = ((t % CC) < C::NV) ? bout[oo] : 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[w * D * NT * PT + i];
      res[i] = s;
    }
    __syncthreads();
  }
};

}  // namespace crom
