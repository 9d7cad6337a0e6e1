// Launch shapes of the value/derivative decode kernels (shared by the
// decode entry points and the fused decode-residual kernel of the sample
// selection).
#pragma once

#include "engine.hpp"

namespace crom {

// Launch shape of the decode kernels per decoder width and arithmetic:
// waves per workgroup, weight fragments (-1: by register estimate, 2:
// streamed one K-block ahead) and the waves per SIMD the register
// allocation must leave room for.  Measured on the 12-column 2D BF16 decode
// (1M points): 4 waves holding a layer's fragments 381 TFLOP/s (380
// registers, one workgroup per CU); 8 waves held to 128 registers 553;
// 4 waves (two M-tiles each, so every activation fragment read from LDS
// feeds two products) with streamed fragments held to 256 registers 633
// (two workgroups per CU); 2 waves 488.
// NBV: 16-point batches per workgroup of the value-only (full-field)
// decode.  2D BF16, 65,536 points: 32 per workgroup 36.3 us, 64 35.0 us,
// 128 32.1 us (FP32: 96.3, 86.2, 90.2 us).
template <class S, int PREC>
struct DecodeTune {
  static constexpr int NW = S::W <= 32 ? 2 : (S::W <= 128 ? 4 : 8);
  static constexpr int PF = -1;
  static constexpr int WPE = 1;
  static constexpr int NBV = 4;
};
template <>
struct DecodeTune<Shape<128, 2, 8, 1>, PREC_BF16> {
  static constexpr int NW = 4, PF = 2, WPE = 2, NBV = 8;
};
template <>
struct DecodeTune<Shape<128, 2, 8, 1>, PREC_BF16_PURE> {
  static constexpr int NW = 4, PF = 2, WPE = 2, NBV = 4;
};
template <>
struct DecodeTune<Shape<128, 2, 8, 1, ACT_SINE>, PREC_BF16> {
  static constexpr int NW = 4, PF = 2, WPE = 2, NBV = 4;
};

}  // namespace crom
