// Host-side helpers shared by the library's translation units: error
// reporting, shape validation and the parameter-array layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <string>

#include "../../include/crom.h"
#include "engine.hpp"

namespace crom {

void set_error(const char* fmt, ...);

// Records a HIP event on `st` when crom_kernel_timer is on for this host
// thread (a step calls it after its set-up launch and after its last launch).
void timer_mark(hipStream_t st);

inline crom_status fail(crom_status s, const char* msg) {
  set_error("%s", msg);
  return s;
}

inline crom_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return CROM_ERR_HIP;
  }
  return CROM_OK;
}

constexpr int LDS_MAX = 160 * 1024;  // LDS per workgroup on gfx950

// Shapes with compiled kernels.
enum ShapeId { SHAPE_NONE = -1, SHAPE_1D = 0, SHAPE_2D = 1, SHAPE_3D = 2, SHAPE_2D_R16 = 3 };

inline ShapeId shape_id(int m, int r, int d, int w) {
  if (m == 1 && r == 3 && d == 1 && w == 32) return SHAPE_1D;
  if (m == 2 && r == 8 && d == 1 && w == 128) return SHAPE_2D;
  if (m == 3 && r == 16 && d == 3 && w == 256) return SHAPE_3D;
  if (m == 2 && r == 16 && d == 1 && w == 128) return SHAPE_2D_R16;
  return SHAPE_NONE;
}

inline ParamIndex param_index(int m, int r, int d, int w, int depth) {
  ParamIndex pi{};
  int64_t off = 0;
  int nin = m + r;
  for (int l = 0; l <= depth; ++l) {
    int nout = (l == depth) ? d : w;
    pi.w[l] = off;
    off += (int64_t)nout * nin;
    pi.b[l] = off;
    off += nout;
    nin = nout;
  }
  return pi;
}

// Validates the net descriptor; packed may be NULL only when `need_packed`
// is false.
crom_status check_net(const crom_net* net, bool need_packed);

template <class K>
inline crom_status set_lds(K kernel, int bytes) {
  return hip_check(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes),
                   "hipFuncSetAttribute");
}

}  // namespace crom
