// Fused decoder engine for gfx950: the MLP g(x, q) evaluated together with
// forward-mode derivative columns, one workgroup per batch of points.
//
// What is computed (Sec. "Network Details"; Alg. "Network gradient" of
// Sec. "Network Gradients via Direct Differentiation", extended to second
// order in x and to the latent directions):
//   z_l = W_l a_{l-1} + b_l,  a_l = s(z_l)            value column
//   dz_l = W_l da_{l-1},      da_l = s1(z_l) dz_l      tangent columns (x_i, q_k)
//   D2z_l = W_l D2a_{l-1},    D2a_l = s2(z_l) dz_i dz_j + s1(z_l) D2z_l
// with s = ELU (s1 = ELU', s2 = ELU'') or, for SIREN networks (Sec.
// "Network Details"), s = sin (s1 = cos, s2 = -sin, the frequency omega_0
// folded into the weights); the Laplacian column carries sum_i of the
// diagonal second derivatives in one column (s2 * sum_i dz_i^2 + s1 * D2z).
// Difference columns carry g(x, q_t) - g(x, q_b) for latents q_t near the
// value column's latent q_b, layer by layer as
//   Dz_l = W_l Da_{l-1},      Da_l = s(z_l + Dz_l) - s(z_l),
// evaluated without cancellation (e^z expm1(Dz) on ELU's exponential
// branch; 2 cos(z + Dz/2) sin(Dz/2) for the sine), so their rounding error
// is relative to the difference itself.  The latent
// tangents then belong to the first difference column's latent
// (z_l + Dz_l); without difference columns, to the value column's.
// The first layer is folded: W_1 [x; q] + b_1 = W_1x x + c with the per-
// latent bias c = W_1q q + b_1 (FP64), so its tangents are columns of W_1
// and its second derivatives are zero; a difference column starts from
// W_1q (q_t - q_b).  The output layer is linear.
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

#include <type_traits>

namespace crom {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Rounds a and b to bfloat16 (nearest even, one packed conversion) and
// returns the pair (a in the low half); ra and rb receive the rounded values
// as floats, taken from the packed bits, for the hi/lo split.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b, float& ra, float& rb) {
  bf16x2 p;
  p[0] = (__bf16)a;
  p[1] = (__bf16)b;
  uint32_t u = __builtin_bit_cast(uint32_t, p);
  // the rounded values come from these bits: without the empty asm the
  // compiler converts a a second time, alone, for the low half
  asm volatile("" : "+v"(u));
  ra = __uint_as_float(u << 16);
  rb = __uint_as_float(u & 0xffff0000u);
  return u;
}
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int PT = 16;  // points per N-tile

// Arithmetic of the hidden-to-hidden layers (see crom.h):
//   FP32      FP32 MFMA
//   BF16      split hi+lo operands on value, difference and spatial-
//             derivative columns, plain bfloat16 on latent-tangent columns
//   BF16_PURE plain bfloat16 everywhere
//   BF16X3    split hi+lo operands on every column
enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_BF16_PURE = 2, PREC_BF16X3 = 3 };
enum { CK_VAL = 0, CK_DIFF = 1, CK_XT = 2, CK_LAP = 3, CK_HESS = 4, CK_QT = 5 };
enum { D2_NONE = 0, D2_LAP = 1, D2_HESS = 2 };
enum { ACT_ELU = 0, ACT_SINE = 1 };  // hidden-layer activation (CROM_ACT_*)

template <int W_, int M_, int R_, int D_, int ACT_ = ACT_ELU>
struct Shape {
  static constexpr int W = W_, M = M_, R = R_, D = D_, ACT = ACT_;
  static constexpr int MTILES = W_ / 16;
  static constexpr int N0 = M_ + R_;
};

// Columns of one batch of 16 points, in this order:
//   NV value columns (value 0 is the base latent of the derivative columns),
//   ND difference columns (latents q_t relative to value 0's latent),
//   the M x tangents (when XT or any second derivative is requested),
//   the second-derivative columns (Laplacian, or Hessian entries HB..HB+NH-1
//   of the upper triangle, row-major),
//   NQ latent tangents (latent indices qb .. qb+NQ-1, qb given at run time).
template <int M_, int R_, int NV_, int ND_, bool XT_, int D2_, int NQ_, int HB_ = 0,
          int NH_ = M_ * (M_ + 1) / 2>
struct Cols {
  static constexpr int M = M_, R = R_, NV = NV_, ND = ND_, D2 = D2_, HB = HB_;
  static constexpr int NX = (XT_ || D2_ != D2_NONE) ? M_ : 0;
  static constexpr int ND2 = D2_ == D2_LAP ? 1 : (D2_ == D2_HESS ? NH_ : 0);
  static constexpr int NQ = NQ_;
  static constexpr int C = NV + ND + NX + ND2 + NQ;
  static constexpr int F0 = NV, X0 = NV + ND, D0 = NV + ND + NX, Q0 = NV + ND + NX + ND2;
  __host__ __device__ static constexpr int kind(int c) {
    return c < F0 ? CK_VAL
         : c < X0 ? CK_DIFF
         : c < D0 ? CK_XT
         : c < Q0 ? (D2_ == D2_LAP ? CK_LAP : CK_HESS)
                  : CK_QT;
  }
  // Hessian column c -> (i, j) of the upper triangle i <= j (row-major),
  // in closed form for m <= 3 (rows start at 0, m, 2m - 1), so that an
  // unrolled loop index folds to a constant register index.
  static_assert(M_ <= 3, "Hessian entry map written for m <= 3");
  __host__ __device__ static constexpr int hess_i(int c) {
    return (c - D0 + HB_) < M_ ? 0 : ((c - D0 + HB_) < 2 * M_ - 1 ? 1 : 2);
  }
  __host__ __device__ static constexpr int hess_j(int c) {
    return hess_i(c) + (c - D0 + HB_) - (hess_i(c) == 0 ? 0 : (hess_i(c) == 1 ? M_ : 2 * M_ - 1));
  }
};

template <class C, int PREC>
__host__ __device__ constexpr bool is_split(int c) {
  return PREC == PREC_BF16X3 || (PREC == PREC_BF16 && C::kind(c) != CK_QT);
}

template <class C, int PREC>
__host__ __device__ constexpr int n_split_before(int c) {
  int n = 0;
  for (int i = 0; i < c; ++i) n += is_split<C, PREC>(i) ? 1 : 0;
  return n;
}

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

// e^z for the negative branch of the ELU.  Every caller selects the
// positive branch by z > 0 itself, so no clamp: for z > 0 the value (up to
// infinity) is never used, and a NaN z stays NaN.
__device__ __forceinline__ float elu_exp(float z) { return __expf(z); }

// e^x - 1 without cancellation: Taylor series (6 terms, relative error
// below 2e-12 for |x| < 1/32) near 0, e^x - 1 beyond.
__device__ __forceinline__ float expm1_acc(float x) {
  const float p = x * (1.0f + x * (0.5f + x * (1.0f / 6 + x * (1.0f / 24 + x * (1.0f / 120)))));
  return fabsf(x) < 0.03125f ? p : __expf(x) - 1.0f;
}

// Sine and cosine for the SIREN epilogue: a Cody-Waite reduction of x to
// [-pi, pi] (2 pi as a float plus its remainder, each product by one fused
// multiply-add), then the hardware approximations, which are accurate on
// that interval; the full-range library routines would more than double the
// registers of the engine's epilogue.
__device__ __forceinline__ float reduce_2pi(float x) {
  const float k = rintf(x * 0.159154943f);
  const float r = fmaf(-k, 6.28318548f, x);
  return fmaf(-k, -1.74845553e-07f, r);
}
__device__ __forceinline__ float sin_r(float x) { return __sinf(reduce_2pi(x)); }
__device__ __forceinline__ float cos_r(float x) { return __cosf(reduce_2pi(x)); }
// sin(h) with an error relative to h for small h (Taylor series through
// h^5 for |h| < 1/32: relative error below 1e-11).
__device__ __forceinline__ float sin_small(float h) {
  const float h2 = h * h;
  return fabsf(h) < 0.03125f ? h * (1.0f - h2 * (1.0f / 6) * (1.0f - h2 * (1.0f / 20))) : sin_r(h);
}

// Small parameters, staged once into LDS by every workgroup (FP32):
//   W1 [W][M+R] | b1 [W] | hidden biases [depth-1][W] | Wout [D][W] | bout [D]
template <class S>
struct ParamCache {
  static constexpr int W = S::W, M = S::M, R = S::R, D = S::D;
  static __host__ __device__ constexpr int W1(int) { return 0; }
  static __host__ __device__ constexpr int B1() { return W * (M + R); }
  static __host__ __device__ constexpr int BH(int h) { return W * (M + R) + W + h * W; }
  static __host__ __device__ constexpr int WOUT(int depth) { return BH(depth - 1); }
  static __host__ __device__ constexpr int BOUT(int depth) { return WOUT(depth) + D * W; }
  static __host__ __device__ constexpr int floats(int depth) { return BOUT(depth) + D; }
  static __host__ __device__ constexpr int bytes(int depth) { return ((floats(depth) * 4 + 15) / 16) * 16; }
  // All threads of the workgroup; `par` is 16-byte aligned LDS.
  static __device__ void load(float* par, const float* __restrict__ params, const ParamIndex& pi,
                              int depth, int nthreads) {
    const int n1 = W * (M + R) + W;  // W1 and b1 are adjacent in the parameter array
    for (int i = threadIdx.x; i < n1; i += nthreads) par[i] = params[pi.w[0] + i];
    for (int h = 0; h < depth - 1; ++h)
      for (int i = threadIdx.x; i < W; i += nthreads) par[BH(h) + i] = params[pi.b[h + 1] + i];
    for (int i = threadIdx.x; i < D * W + D; i += nthreads) par[WOUT(depth) + i] = params[pi.w[depth] + i];
  }
};

// All per-batch tables live in one dynamic LDS block:
//   act    activations (fragment order): NT tiles, then the lo tiles
//   xs     [NB*16][M] points (FP32)
//   fold   [NV + ND][W] per-latent first-layer terms (FP32)
//   res    [D][NT][16] outputs (FP32)
// The cross-wave output reduction reuses `act`.  The parameter cache lives
// after these tables (its offset is passed in, so that kernels running
// several engines share one cache).
// PF: 1 prefetches the next layer's weight fragments into a second register
// set during this layer's products, 0 loads each layer's fragments when the
// layer starts, 2 streams them one K-block ahead of their products, 3 two
// K-blocks ahead, -1 chooses by a register estimate.  CANON: the output layer's partial dot
// products are summed per M-tile, the tiles in tile order, so that results
// do not depend on the wave count; else per wave (the wave's tiles in one
// running sum, then the waves in order).
template <class S, class C, int NB, int NW, int PREC, int PF = -1, bool CANON = false>
struct Engine {
  static constexpr int W = S::W, M = S::M, R = S::R, D = S::D;
  static constexpr int CC = C::C;
  static constexpr int NT = NB * CC;
  static constexpr int MTILES = S::MTILES;
  static constexpr int MT = MTILES / NW;
  static_assert(MTILES % NW == 0, "waves must split the M-tiles evenly");
  static constexpr int NPTS = NB * PT;
  static constexpr bool BF = PREC != PREC_FP32;
  static constexpr int SPB = n_split_before<C, PREC>(CC);  // split columns per batch
  static constexpr int NSPL = BF ? NB * SPB : 0;
  static constexpr int KQ = Packing<S, PREC>::KQ;
  static constexpr int NACT = NT + NSPL;
  static constexpr int ACT_BYTES = NACT * KQ * 64 * 16;
  static constexpr int NSLOT = CANON ? MTILES : NW;  // partial-sum slots of the output reduction
  static constexpr int RED_BYTES = NSLOT * D * NT * PT * 4;
  static constexpr int ACT_REGION = ACT_BYTES > RED_BYTES ? ACT_BYTES : RED_BYTES;
  static constexpr int XS_OFF = ACT_REGION;
  static constexpr int NF = C::NV + C::ND;
  static constexpr int FOLD_OFF = XS_OFF + ((NPTS * M * 4 + 15) / 16) * 16;
  static constexpr int RES_OFF = FOLD_OFF + NF * W * 4;
  static constexpr int LDS_BYTES = RES_OFF + D * NT * PT * 4;  // without the parameter cache
  static constexpr int THREADS = NW * 64;
  using PC = ParamCache<S>;
  using AFrag = typename std::conditional<PREC == PREC_FP32, f32x4, bf16x8>::type;
  static constexpr int NLO = NSPL > 0 ? KQ : 1;  // lo fragments only in split mode
  // Prefetch the next layer's weight fragments while computing this one,
  // unless the two register sets would crowd out the accumulators.
  static constexpr int FRAG_REGS = MT * KQ * 4 * (NSPL > 0 ? 2 : 1);
  // A layer's fragments beyond 64 registers (width 256) are streamed: each
  // K-block's fragments are loaded one block ahead of their products
  // instead of holding the whole layer.
  // PF 3: streamed two K-blocks ahead (twice the loads in flight, for
  // launches with one wave per SIMD, where no other wave hides their latency).
  static constexpr bool STREAM = FRAG_REGS > 64 || PF == 2 || PF == 3;
  static constexpr int LA = PF == 3 ? 2 : 1;  // K-blocks loaded ahead when streaming
  static constexpr bool PREFETCH = !STREAM && (PF >= 0 ? PF == 1 : 2 * FRAG_REGS + MT * NT * 4 <= 320);
  static constexpr int TG = 4;  // operand loads allowed to run ahead of their products

  static constexpr int KH = STREAM ? 1 : KQ;  // fragments held per layer
  struct Frags {
    AFrag hi[MT][KH];
    AFrag lo[MT][STREAM ? 1 : NLO];
  };

  static __host__ __device__ constexpr int lo_tile(int b, int c) {
    return NT + b * SPB + n_split_before<C, PREC>(c);
  }

  static __device__ __forceinline__ void load_frags(Frags& f, const char* __restrict__ packed, int h,
                                                    int wave, int lane) {
    if constexpr (STREAM) return;
    const AFrag* wf = reinterpret_cast<const AFrag*>(packed + (size_t)h * Packing<S, PREC>::LAYER_BYTES);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int kb = 0; kb < KQ; ++kb) f.hi[mt][kb] = wf[((wave * MT + mt) * KQ + kb) * 64 + lane];
    if constexpr (NSPL > 0) {
      constexpr int LO = MTILES * KQ * 64;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int kb = 0; kb < KQ; ++kb) f.lo[mt][kb] = wf[LO + ((wave * MT + mt) * KQ + kb) * 64 + lane];
    }
  }

  // ---- stage points and per-latent first-layer terms --------------------
  // Points first .. first+n_valid-1 of x (n_valid <= NPTS; the rest of the
  // batch is padded with x = 0).  lat: NV latent vectors (v at lat + v *
  // lat_stride), folded with the bias; dlat: ND latent differences (t at
  // dlat + t * dlat_stride), folded without it.  FP64.  par: the staged
  // parameter cache.
  static __device__ void stage(char* lds, const float* __restrict__ x, int64_t first, int n_valid,
                               const double* __restrict__ lat, int lat_stride,
                               const double* __restrict__ dlat, int dlat_stride, const float* par) {
    float* xs = reinterpret_cast<float*>(lds + XS_OFF);
    for (int i = threadIdx.x; i < NPTS * M; i += THREADS) {
      int p = i / M;
      xs[i] = p < n_valid ? x[(first + p) * M + (i - p * M)] : 0.0f;
    }
    float* fold = reinterpret_cast<float*>(lds + FOLD_OFF);
    const float* W1 = par + PC::W1(0);
    const float* b1 = par + PC::B1();
    for (int i = threadIdx.x; i < NF * W; i += THREADS) {
      const int v = i / W, u = i - v * W;
      const double* l = v < C::NV ? lat + v * lat_stride : dlat + (v - C::NV) * dlat_stride;
      double s = v < C::NV ? (double)b1[u] : 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) s += (double)W1[u * (M + R) + M + k] * l[k];
      fold[i] = (float)s;
    }
  }

  // ---- epilogue ---------------------------------------------------------
  // In place on z[t] for one (unit, lane) across all tiles.
  // s1o (optional): receives each batch's tangent slope act'(z) (at the
  // value column's latent, or at difference column 0's when there are
  // difference columns: the slope the tangent columns take), for a reverse
  // pass.
  static __device__ __forceinline__ void epilogue(float (&z)[NT], float* s1o = nullptr) {
    if constexpr (S::ACT == ACT_SINE) {
      epilogue_sine(z, s1o);
      return;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      float* zb = &z[b * CC];
      const float z0 = zb[0];
      const float e0 = elu_exp(z0);
      const bool pos0 = z0 > 0.0f;
      const float s1 = pos0 ? 1.0f : e0;
      const float s2 = pos0 ? 0.0f : e0;
      float st = s1;  // tangent scale: at the base latent, or at difference column 0's
#pragma unroll
      for (int c = C::F0; c < C::X0; ++c) {
        const float dz = zb[c];
        const float zt = z0 + dz;
        const bool post = zt > 0.0f;
        const float et = elu_exp(zt);
        const float both_neg = e0 * expm1_acc(dz);
        const float cross = (post ? zt : et - 1.0f) - (pos0 ? z0 : e0 - 1.0f);
        zb[c] = (pos0 && post) ? dz : ((!pos0 && !post) ? both_neg : cross);
        if (c == C::F0) st = post ? 1.0f : et;
      }
      if (s1o) s1o[b] = st;
      if constexpr (C::D2 == D2_LAP) {
        float sq = 0.0f;
#pragma unroll
        for (int i = 0; i < C::NX; ++i) sq += zb[C::X0 + i] * zb[C::X0 + i];
        zb[C::D0] = s1 * zb[C::D0] + s2 * sq;
      } else if constexpr (C::D2 == D2_HESS) {
#pragma unroll
        for (int c = C::D0; c < C::Q0; ++c) {
          const float zi = zb[C::X0 + C::hess_i(c)];
          const float zj = zb[C::X0 + C::hess_j(c)];
          zb[c] = s1 * zb[c] + s2 * zi * zj;
        }
      }
#pragma unroll
      for (int c = C::X0; c < C::D0; ++c) zb[c] = s1 * zb[c];
#pragma unroll
      for (int c = C::Q0; c < CC; ++c) zb[c] = st * zb[c];
#pragma unroll
      for (int c = 1; c < C::NV; ++c) {
        const float zz = zb[c];
        zb[c] = zz > 0.0f ? zz : elu_exp(zz) - 1.0f;
      }
      zb[0] = pos0 ? z0 : e0 - 1.0f;
    }
  }

  // The same column rules with s = sin: s1 = cos, s2 = -sin, differences
  // sin(z + Dz) - sin(z) = 2 cos(z + Dz/2) sin(Dz/2).
  static __device__ __forceinline__ void epilogue_sine(float (&z)[NT], float* s1o) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      float* zb = &z[b * CC];
      const float z0 = zb[0];
      const float r0 = reduce_2pi(z0);
      const float sn0 = __sinf(r0), cs0 = __cosf(r0);
      const float s1 = cs0, s2 = -sn0;
      float st = s1;  // tangent scale: at the base latent, or at difference column 0's
#pragma unroll
      for (int c = C::F0; c < C::X0; ++c) {
        const float dz = zb[c];
        zb[c] = 2.0f * cos_r(z0 + 0.5f * dz) * sin_small(0.5f * dz);
        if (c == C::F0) st = cos_r(z0 + dz);
      }
      if (s1o) s1o[b] = st;
      if constexpr (C::D2 == D2_LAP) {
        float sq = 0.0f;
#pragma unroll
        for (int i = 0; i < C::NX; ++i) sq += zb[C::X0 + i] * zb[C::X0 + i];
        zb[C::D0] = s1 * zb[C::D0] + s2 * sq;
      } else if constexpr (C::D2 == D2_HESS) {
#pragma unroll
        for (int c = C::D0; c < C::Q0; ++c) {
          const float zi = zb[C::X0 + C::hess_i(c)];
          const float zj = zb[C::X0 + C::hess_j(c)];
          zb[c] = s1 * zb[c] + s2 * zi * zj;
        }
      }
#pragma unroll
      for (int c = C::X0; c < C::D0; ++c) zb[c] = s1 * zb[c];
#pragma unroll
      for (int c = C::Q0; c < CC; ++c) zb[c] = st * zb[c];
#pragma unroll
      for (int c = 1; c < C::NV; ++c) zb[c] = sin_r(zb[c]);
      zb[0] = sn0;
    }
  }

  // ---- write one M-tile of activations (all tiles, 4 units per lane) ----
  static __device__ __forceinline__ void write_act(char* lds, int mtg, int lane, const f32x4 (&o)[NT]) {
    if constexpr (PREC == PREC_FP32) {
      f32x4* act = reinterpret_cast<f32x4*>(lds);
#pragma unroll
      for (int t = 0; t < NT; ++t) act[(t * KQ + mtg) * 64 + lane] = o[t];
    } else {
      // fragment (t, kb = mtg/2), element offset (mtg%2)*4; four bfloat16
      // values as two packed pairs
      uint2* act = reinterpret_cast<uint2*>(lds);
      const int half = mtg & 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int b = t / CC, c = t % CC;
        float r[4];
        const uint2 h = {bf16_pair(o[t][0], o[t][1], r[0], r[1]), bf16_pair(o[t][2], o[t][3], r[2], r[3])};
        act[((t * KQ + (mtg >> 1)) * 64 + lane) * 2 + half] = h;
        if (is_split<C, PREC>(c)) {
          float d[4];
          const uint2 l = {bf16_pair(o[t][0] - r[0], o[t][1] - r[1], d[0], d[1]),
                           bf16_pair(o[t][2] - r[2], o[t][3] - r[3], d[2], d[3])};
          act[((lo_tile(b, c) * KQ + (mtg >> 1)) * 64 + lane) * 2 + half] = l;
        }
      }
    }
  }

  // ---- output layer partial sums for one M-tile --------------------------
  static __device__ __forceinline__ void out_accum(float (&part)[D][NT], const f32x4 (&o)[NT],
                                                   const float* Wout, int ubase) {
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

  // epilogue over the 4 accumulator rows of one M-tile, in place
  static __device__ __forceinline__ void epilogue_tile(f32x4 (&acc)[NT], float* s1o = nullptr) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float z[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) z[t] = acc[t][v];
      epilogue(z, s1o ? s1o + v * NB : nullptr);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][v] = z[t];
    }
  }

  // One hidden layer h (weights of layer h + 2 of the network): MFMA over
  // the staged activations, epilogue, and either the next activations or the
  // output layer's partial sums.  `cur` holds this layer's fragments; `nxt`
  // receives the next layer's when prefetching.
  static __device__ __forceinline__ void hidden_layer(char* lds, const float* par,
                                                      const char* __restrict__ packed, int depth,
                                                      int h, Frags& cur, Frags& nxt,
                                                      float (&part)[MT][D][NT], int wave, int lane) {
    const int g = lane >> 4;
    const float* Wout = par + PC::WOUT(depth);
    if constexpr (PREFETCH) {
      if (h + 1 < depth - 1) load_frags(nxt, packed, h + 1, wave, lane);
    } else {
      if (h > 0) load_frags(cur, packed, h, wave, lane);
    }
    f32x4 acc[MT][NT];
    products(lds, par + PC::BH(h), packed, h, cur, acc, wave, lane);
    __syncthreads();  // every wave has read this layer's activations
    const bool last = (h == depth - 2);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int mtg = wave * MT + mt;
      epilogue_tile(acc[mt]);
      if (!last) write_act(lds, mtg, lane, acc[mt]);
      else out_accum(part[CANON ? mt : 0], acc[mt], Wout, mtg * 16 + g * 4);
    }
    __syncthreads();
  }

  // acc = W act (+ the bias on value columns): the products of packed layer
  // h over the staged activations, fragments from `cur` (held) or streamed
  // from `packed`.
  static __device__ __forceinline__ void products(const char* lds, const float* bias,
                                                  const char* __restrict__ packed, int h, const Frags& cur,
                                                  f32x4 (&acc)[MT][NT], int wave, int lane) {
    const int g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int mtg = wave * MT + mt;
      f32x4 bv = {0.0f, 0.0f, 0.0f, 0.0f};
      if constexpr (C::NV > 0) {
        const float* bp = bias + mtg * 16 + g * 4;
        bv = f32x4{bp[0], bp[1], bp[2], bp[3]};
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bool isval = C::kind(t % CC) == CK_VAL;
        acc[mt][t] = isval ? bv : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      }
    }
    // streamed fragments: sh/sl hold K-block kb, nh/nl the next one, and
    // with a look-ahead of two mh/ml the one after
    const AFrag* wfs = reinterpret_cast<const AFrag*>(packed + (size_t)h * Packing<S, PREC>::LAYER_BYTES);
    constexpr int LO = MTILES * KQ * 64;
    constexpr int MH = LA > 1 ? MT : 1;
    AFrag sh[MT], sl[MT], nh[MT], nl[MT], mh[MH], ml[MH];
    if constexpr (STREAM) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        sh[mt] = wfs[((wave * MT + mt) * KQ + 0) * 64 + lane];
        if constexpr (NSPL > 0) sl[mt] = wfs[LO + ((wave * MT + mt) * KQ + 0) * 64 + lane];
      }
      if constexpr (LA > 1 && KQ > 1) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          nh[mt] = wfs[((wave * MT + mt) * KQ + 1) * 64 + lane];
          if constexpr (NSPL > 0) nl[mt] = wfs[LO + ((wave * MT + mt) * KQ + 1) * 64 + lane];
        }
      }
    }
#define CROM_FRAG_HI(mt, kb) (STREAM ? sh[mt] : cur.hi[mt][(kb) % KH])
#define CROM_FRAG_LO(mt, kb) (STREAM ? sl[mt] : cur.lo[mt][(kb) % KH])
#define CROM_STREAM_NEXT(kb)                                                                     \
    if constexpr (STREAM && LA > 1) {                                                            \
      if ((kb) + 2 < KQ) {                                                                       \
        _Pragma("unroll") for (int mt = 0; mt < MT; ++mt) {                                      \
          mh[mt] = wfs[((wave * MT + mt) * KQ + (kb) + 2) * 64 + lane];                          \
          if constexpr (NSPL > 0) ml[mt] = wfs[LO + ((wave * MT + mt) * KQ + (kb) + 2) * 64 + lane]; \
        }                                                                                        \
      }                                                                                          \
    } else if constexpr (STREAM) {                                                               \
      if ((kb) + 1 < KQ) {                                                                       \
        _Pragma("unroll") for (int mt = 0; mt < MT; ++mt) {                                      \
          nh[mt] = wfs[((wave * MT + mt) * KQ + (kb) + 1) * 64 + lane];                          \
          if constexpr (NSPL > 0) nl[mt] = wfs[LO + ((wave * MT + mt) * KQ + (kb) + 1) * 64 + lane]; \
        }                                                                                        \
      }                                                                                          \
    }
#define CROM_STREAM_SHIFT()                                                                      \
    if constexpr (STREAM) {                                                                      \
      _Pragma("unroll") for (int mt = 0; mt < MT; ++mt) {                                        \
        sh[mt] = nh[mt];                                                                         \
        if constexpr (NSPL > 0) sl[mt] = nl[mt];                                                 \
        if constexpr (LA > 1) {                                                                  \
          nh[mt] = mh[mt];                                                                       \
          if constexpr (NSPL > 0) nl[mt] = ml[mt];                                               \
        }                                                                                        \
      }                                                                                          \
    }
    if constexpr (PREC == PREC_FP32) {
      const f32x4* act = reinterpret_cast<const f32x4*>(lds);
#pragma unroll
      for (int kq = 0; kq < KQ; ++kq) {
        CROM_STREAM_NEXT(kq)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const f32x4 bfr = act[(t * KQ + kq) * 64 + lane];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const f32x4 a = CROM_FRAG_HI(mt, kq);
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], bfr[0], acc[mt][t], 0, 0, 0);
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], bfr[1], acc[mt][t], 0, 0, 0);
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], bfr[2], acc[mt][t], 0, 0, 0);
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], bfr[3], acc[mt][t], 0, 0, 0);
          }
          if ((t + 1) % TG == 0) __builtin_amdgcn_sched_barrier(0);  // bound the run-ahead
        }
        // keep the next k-block's operand loads from being hoisted above this
        // one's products: hoisting all of them would exhaust the registers
        __builtin_amdgcn_sched_barrier(0);
        CROM_STREAM_SHIFT()
      }
    } else {
      const bf16x8* act = reinterpret_cast<const bf16x8*>(lds);
#pragma unroll
      for (int kb = 0; kb < KQ; ++kb) {
        CROM_STREAM_NEXT(kb)
        // per column: its hi fragment feeds the hi*hi product and, on a split
        // column, the lo*hi product too; the lo fragment feeds hi*lo
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int b = t / CC, c = t % CC;
          const bf16x8 bfr = act[(t * KQ + kb) * 64 + lane];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(CROM_FRAG_HI(mt, kb), bfr, acc[mt][t], 0, 0, 0);
          if constexpr (NSPL > 0) {
            if (is_split<C, PREC>(c)) {
              const bf16x8 bl = act[(lo_tile(b, c) * KQ + kb) * 64 + lane];
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) {
                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(CROM_FRAG_HI(mt, kb), bl, acc[mt][t], 0, 0, 0);
                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(CROM_FRAG_LO(mt, kb), bfr, acc[mt][t], 0, 0, 0);
              }
            }
          }
          if ((t + 1) % TG == 0) __builtin_amdgcn_sched_barrier(0);  // bound the run-ahead
        }
        __builtin_amdgcn_sched_barrier(0);  // as above
        CROM_STREAM_SHIFT()
      }
    }
#undef CROM_FRAG_HI
#undef CROM_FRAG_LO
#undef CROM_STREAM_NEXT
#undef CROM_STREAM_SHIFT
  }

  // ---- the whole network for one batch -----------------------------------
  // Leaves the outputs in res[D][NT][16]; all threads must call it.  par:
  // the staged parameter cache; packed: the fragment-ordered hidden weights.
  static __device__ void run(char* lds, const float* par, const char* __restrict__ packed, int depth,
                             int qb) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    float part[MT][D][NT];  // output partial sums per M-tile
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int oo = 0; oo < D; ++oo)
#pragma unroll
        for (int t = 0; t < NT; ++t) part[mt][oo][t] = 0.0f;

    Frags fa, fb;  // current and next layer's weight fragments
    if (depth > 1) load_frags(fa, packed, 0, wave, lane);
    first_layer(lds, par, depth, qb, part, wave, lane);

    // ---------------- hidden layers 2..depth (MFMA) ----------------
    // Two layers per trip so that each weight-fragment buffer keeps a fixed
    // register home.
    for (int h = 0; h < depth - 1; h += 2) {
      hidden_layer(lds, par, packed, depth, h, fa, fb, part, wave, lane);
      if (h + 1 < depth - 1) hidden_layer(lds, par, packed, depth, h + 1, fb, fa, part, wave, lane);
    }
    reduce_outputs(lds, par, depth, part, reinterpret_cast<float*>(lds + RES_OFF), NT, 0, wave, lane);
  }

  // ---- layer 1 (VALU, folded) ---------------------------------------------
  // Its activations go to the staged tiles (or, for a one-layer network, to
  // the output partial sums); s1o (optional) receives the value column's
  // slope at this lane's entries, [mt][v] (NB == 1).
  static __device__ __forceinline__ void first_layer(char* lds, const float* par, int depth, int qb,
                                                     float (&part)[MT][D][NT], int wave, int lane,
                                                     float (*s1o)[4] = nullptr) {
    const int g = lane >> 4, j = lane & 15;
    const float* xs = reinterpret_cast<const float*>(lds + XS_OFF);
    const float* fold = reinterpret_cast<const float*>(lds + FOLD_OFF);
    const float* W1 = par + PC::W1(0);
    const float* Wout = par + PC::WOUT(depth);
    {
      float xr[NB][M];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < M; ++i) xr[b][i] = xs[(b * PT + j) * M + i];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int mtg = wave * MT + mt;
        f32x4 o4[NT];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int u = mtg * 16 + g * 4 + v;
          float wx[M];
#pragma unroll
          for (int i = 0; i < M; ++i) wx[i] = W1[u * (M + R) + i];
          float z[NT];
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
              else if (k == CK_DIFF) val = fold[c * W + u];
              else if (k == CK_XT) val = wx[c - C::X0];
              else if (k == CK_QT) val = W1[u * (M + R) + M + qb + (c - C::Q0)];
              else val = 0.0f;
              z[b * CC + c] = val;
            }
          }
          epilogue(z, s1o ? &s1o[mt][v] : nullptr);
#pragma unroll
          for (int t = 0; t < NT; ++t) o4[t][v] = z[t];
        }
        if (depth > 1) write_act(lds, mtg, lane, o4);
        else out_accum(part[CANON ? mt : 0], o4, Wout, mtg * 16 + g * 4);
      }
    }
    __syncthreads();
  }

  // ---- output layer: reduce the partial dot products ------------------------
  // res[oo * res_nt + res_t0 + t][16] = bout (value columns) + the slots'
  // lane-group sums in slot order: with CANON one slot per M-tile (the same
  // order for any number of waves), else one per wave.  Reuses the
  // activation region.
  static __device__ __forceinline__ void reduce_outputs(char* lds, const float* par, int depth,
                                                        float (&part)[MT][D][NT], float* res, int res_nt,
                                                        int res_t0, int wave, int lane) {
    if constexpr (CANON) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) stash_tile(lds, wave * MT + mt, part[mt], lane);
    } else {
      stash_tile(lds, wave, part[0], lane);  // the wave's running sum over its tiles
    }
    __syncthreads();
    sum_tiles<NSLOT>(lds, par, depth, res, res_nt, res_t0);
  }

  // M-tile mtg's output partial sums, summed over the lane groups, into the
  // reduction area (the activation region, once every wave has read it).
  static __device__ __forceinline__ void stash_tile(char* lds, int mtg, float (&pt)[D][NT], int lane) {
    const int g = lane >> 4, j = lane & 15;
    float* red = reinterpret_cast<float*>(lds);
#pragma unroll
    for (int oo = 0; oo < D; ++oo)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        float s = pt[oo][t];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (g == 0) red[((mtg * D + oo) * NT + t) * PT + j] = s;
      }
  }

  // The outputs from the stashed tiles (after a barrier), in tile order
  // (NSL slots: the M-tiles, or fewer slots that each hold a wave's tiles).
  template <int NSL>
  static __device__ __forceinline__ void sum_tiles(const char* lds, const float* par, int depth, float* res,
                                                   int res_nt, int res_t0) {
    const float* red = reinterpret_cast<const float*>(lds);
    const float* bout = par + PC::BOUT(depth);
    for (int i = threadIdx.x; i < D * NT * PT; i += THREADS) {
      const int oo = i / (NT * PT);
      const int t = (i / PT) % NT;
      float s = C::kind(t % CC) == CK_VAL ? bout[oo] : 0.0f;
#pragma unroll
      for (int tl = 0; tl < NSL; ++tl) s += red[tl * D * NT * PT + i];
      res[(oo * res_nt + res_t0 + t) * PT + (i % PT)] = s;
    }
    __syncthreads();
  }
};

// ---------------------------------------------------------------------------
// Forward columns CF (value with x tangents and Laplacian, or value with
// trial differences) and the latent Jacobian by one reverse (adjoint) pass
// per output instead of R forward tangent columns.  The latent Jacobian is
// the chain rule through the layers (Sec. "Network Inversion" uses dg/dq),
// accumulated from the output back: with s_l the tangent slope act'(z_l)
// of every layer (at the trial latent when CF has difference columns),
//   dz_L = s_L * Wout[o],   dz_{l-1} = s_{l-1} * (W_l^T dz_l),
//   dg_o/dq_k = sum_u W1[u][m + k] dz_0[u],
// the same products the forward tangent columns form, associated the other
// way.  The forward pass keeps each layer's slope in registers, so depth is
// bounded by DMAX; the adjoint columns take the arithmetic of latent-tangent
// columns (plain bfloat16 in BF16, split in BF16X3) and the transposed
// weight fragments that crom_net_pack writes after the layers.  Outputs
// res[D][NTO][16] in the column order of CF with the R latent-tangent
// columns appended (CO).
// ---------------------------------------------------------------------------
#ifndef CROM_REV_DMAX
#define CROM_REV_DMAX 6
#endif
// CANON: output and Jacobian sums per M-tile in tile order, so results do
// not depend on the wave count (kernels of different wave counts then agree
// bit for bit); else per wave, one sum less deep.
template <class S, class CF_, int NW, int PREC, int PF, bool CANON = true, int DMAX = CROM_REV_DMAX>
struct RevJets {
  static constexpr int W = S::W, M = S::M, R = S::R, D = S::D;
  using CF = CF_;
  static_assert(CF::NV == 1 && CF::NQ == 0, "one value column, no forward tangent columns");
  using CB = Cols<M, R, 0, 0, false, D2_NONE, D>;  // one adjoint column per output
  using CO = Cols<M, R, CF::NV, CF::ND, (CF::NX > 0), CF::D2, R>;  // the output columns
  using EF = Engine<S, CF, 1, NW, PREC, PF, CANON>;
  using EB = Engine<S, CB, 1, NW, PREC, PF, CANON>;
  using PC = ParamCache<S>;
  static constexpr int MT = EF::MT, NTF = CF::C, NTO = CO::C, THREADS = NW * 64;
  static constexpr int NSLOT = CANON ? S::MTILES : NW;  // partial-sum slots
  static_assert(NTF == CO::Q0, "forward columns precede the Jacobian columns");
  static_assert(EB::ACT_BYTES <= EF::ACT_REGION, "the adjoint tiles fit the activation region");
  static_assert(S::MTILES * D * R * PT * 4 <= EF::ACT_REGION, "the Jacobian reduction fits the activation region");
  static constexpr int RES_OFF = EF::LDS_BYTES;
  static constexpr int LDS_BYTES = RES_OFF + D * NTO * PT * 4;  // without the parameter cache
  static __host__ __device__ constexpr bool supported(int depth) { return depth >= 2 && depth <= DMAX; }

  // The slopes kept for the reverse pass: FP32 in the FP32 and BF16X3
  // modes; in the bfloat16 modes as packed half-precision pairs (rounded
  // toward zero, relative error below 2^-10, half the rounding error of the
  // bfloat16 adjoint operands), which halves their registers.
  typedef __fp16 h2 __attribute__((ext_vector_type(2)));
  static constexpr bool S1H = PREC == PREC_BF16 || PREC == PREC_BF16_PURE;
  struct Slopes {
    float f[S1H ? 1 : DMAX][MT][4];
    h2 h[S1H ? DMAX : 1][MT][2];
  };
  static __device__ __forceinline__ void put(Slopes& sl, int l, int mt, const float (&v)[4]) {
    if constexpr (S1H) {
      sl.h[l][mt][0] = __builtin_amdgcn_cvt_pkrtz(v[0], v[1]);
      sl.h[l][mt][1] = __builtin_amdgcn_cvt_pkrtz(v[2], v[3]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) sl.f[l][mt][i] = v[i];
    }
  }
  static __device__ __forceinline__ float get(const Slopes& sl, int l, int mt, int v) {
    if constexpr (S1H) return (float)sl.h[l][mt][v >> 1][v & 1];
    else return sl.f[l][mt][v];
  }

  // Packed layer h's fragments, the address formed where the layer starts:
  // with the layers unrolled the compiler would otherwise form every
  // layer's per-lane addresses up front and keep them live.
  static __device__ __forceinline__ const char* layer_base(const char* packed, int h) {
    const char* p = packed + (size_t)h * Packing<S, PREC>::LAYER_BYTES;
    asm volatile("" : "+s"(p));
    return p;
  }

  // lat: the value column's latent; dlat: the difference columns' latents
  // relative to it (ND of them, stride R).  FP64.
  static __device__ void stage(char* lds, const float* __restrict__ x, int64_t first, int n_valid,
                               const double* __restrict__ lat, const double* __restrict__ dlat, const float* par) {
    EF::stage(lds, x, first, n_valid, lat, R, dlat, R, par);
  }

  static __device__ void run(char* lds, const float* par, const char* __restrict__ packed, int depth) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, j = lane & 15;
    float* res = reinterpret_cast<float*>(lds + RES_OFF);
    const float* W1 = par + PC::W1(0);
    const float* Wout = par + PC::WOUT(depth);
    Slopes sl;  // slope of layer l at this lane's (unit, point) entries
    float part[MT][D][NTF];  // output sums per tile (first_layer's are unused: depth >= 2)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int oo = 0; oo < D; ++oo)
#pragma unroll
        for (int t = 0; t < NTF; ++t) part[mt][oo][t] = 0.0f;

    // ---- forward: layer 1 on the VALU, then the hidden layers (held
    // fragments alternate between two buffers when prefetching)
    typename EF::Frags ff[2];
    if constexpr (!EF::STREAM) EF::load_frags(ff[0], layer_base(packed, 0), 0, wave, lane);
    {
      float s0[MT][4];
      EF::first_layer(lds, par, depth, 0, part, wave, lane, s0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) put(sl, 0, mt, s0[mt]);
    }
#pragma unroll
    for (int l = 1; l < DMAX; ++l) {
      if (l < depth) {
        const int cur = EF::PREFETCH ? (l - 1) & 1 : 0;
        if constexpr (EF::PREFETCH) {
          if (l + 1 < depth) EF::load_frags(ff[l & 1], layer_base(packed, l), 0, wave, lane);
        } else if constexpr (!EF::STREAM) {
          if (l > 1) EF::load_frags(ff[0], layer_base(packed, l - 1), 0, wave, lane);
        }
        f32x4 acc[MT][NTF];
        EF::products(lds, par + PC::BH(l - 1), layer_base(packed, l - 1), 0, ff[cur], acc, wave, lane);
        __syncthreads();  // every wave has read this layer's activations
        const bool last = l == depth - 1;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int mtg = wave * MT + mt;
          float sv[4];
          EF::epilogue_tile(acc[mt], sv);
          put(sl, l, mt, sv);
          if (!last) {
            EF::write_act(lds, mtg, lane, acc[mt]);
          } else if constexpr (CANON) {  // the activations have been read: stash this tile's sums now
            EF::out_accum(part[mt], acc[mt], Wout, mtg * 16 + g * 4);
            EF::stash_tile(lds, mtg, part[mt], lane);
          } else {
            EF::out_accum(part[0], acc[mt], Wout, mtg * 16 + g * 4);  // the wave's tiles into one sum
          }
        }
        __syncthreads();
      }
    }
    if constexpr (!CANON) {
      EF::stash_tile(lds, wave, part[0], lane);
      __syncthreads();
    }
    EF::template sum_tiles<NSLOT>(lds, par, depth, res, NTO, 0);

    // ---- adjoint of the last hidden layer's pre-activation: s_L * Wout[o]
#pragma unroll
    for (int l = 1; l < DMAX; ++l) {
      if (l == depth - 1) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int mtg = wave * MT + mt;
          f32x4 o4[D];
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int oo = 0; oo < D; ++oo) o4[oo][v] = get(sl, l, mt, v) * Wout[oo * W + mtg * 16 + g * 4 + v];
          EB::write_act(lds, mtg, lane, o4);
        }
      }
    }
    __syncthreads();

    // ---- back through the hidden layers (transposed fragments), then W1's
    // latent columns
    const char* packed_t = packed + (size_t)(depth - 1) * Packing<S, PREC>::LAYER_BYTES;
    float* red = reinterpret_cast<float*>(lds);
    float jp[D][R];  // Jacobian sums: of the tile (CANON) or of the wave's tiles
#pragma unroll
    for (int oo = 0; oo < D; ++oo)
#pragma unroll
      for (int k = 0; k < R; ++k) jp[oo][k] = 0.0f;
    typename EB::Frags fb[2];
#pragma unroll
    for (int l = DMAX - 1; l >= 1; --l) {
      if (l <= depth - 1) {
        const int cur = EB::PREFETCH ? (l - 1) & 1 : 0;
        if constexpr (EB::PREFETCH) {
          if (l == depth - 1) EB::load_frags(fb[(l - 1) & 1], layer_base(packed_t, l - 1), 0, wave, lane);
          if (l > 1) EB::load_frags(fb[l & 1], layer_base(packed_t, l - 2), 0, wave, lane);
        } else if constexpr (!EB::STREAM) {
          EB::load_frags(fb[0], layer_base(packed_t, l - 1), 0, wave, lane);
        }
        f32x4 acc[MT][D];
        EB::products(lds, nullptr, layer_base(packed_t, l - 1), 0, fb[cur], acc, wave, lane);
        __syncthreads();  // every wave has read dz_l
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int mtg = wave * MT + mt;
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int oo = 0; oo < D; ++oo) acc[mt][oo][v] *= get(sl, l - 1, mt, v);
          if (l > 1) {
            EB::write_act(lds, mtg, lane, acc[mt]);
          } else {
            // this tile's share of the Jacobian; with CANON summed over its
            // lane groups and stored at once for the sum over tiles (the
            // activation region is free: every wave has read dz_1)
            if constexpr (CANON) {
#pragma unroll
              for (int oo = 0; oo < D; ++oo)
#pragma unroll
                for (int k = 0; k < R; ++k) jp[oo][k] = 0.0f;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float* w1 = W1 + (mtg * 16 + g * 4 + v) * (M + R) + M;
#pragma unroll
              for (int k = 0; k < R; ++k) {
                const float w = w1[k];
#pragma unroll
                for (int oo = 0; oo < D; ++oo) jp[oo][k] += w * acc[mt][oo][v];
              }
            }
            if constexpr (CANON) stash_jac(red, mtg, jp, lane);
          }
        }
        __syncthreads();
      }
    }
    if constexpr (!CANON) {
      stash_jac(red, wave, jp, lane);
      __syncthreads();
    }

    // ---- the Jacobian: the slots' sums in slot order
    for (int i = threadIdx.x; i < D * R * PT; i += THREADS) {
      const int oo = i / (R * PT), k = (i / PT) % R;
      float t = 0.0f;
#pragma unroll
      for (int tl = 0; tl < NSLOT; ++tl) t += red[tl * D * R * PT + i];
      res[(oo * NTO + NTF + k) * PT + i % PT] = t;
    }
    __syncthreads();
  }

  // Jacobian sums of one slot, summed over the lane groups, into the
  // reduction area.
  static __device__ __forceinline__ void stash_jac(float* red, int slot, float (&jp)[D][R], int lane) {
    const int g = lane >> 4, j = lane & 15;
#pragma unroll
    for (int oo = 0; oo < D; ++oo)
#pragma unroll
      for (int k = 0; k < R; ++k) {
        float t = jp[oo][k];
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        if (g == 0) red[((slot * D + oo) * R + k) * PT + j] = t;
      }
  }
};

}  // namespace crom
