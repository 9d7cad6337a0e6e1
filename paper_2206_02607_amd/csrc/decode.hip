// Decoder entry points: weight packing, value decode and decode with
// derivative columns (Sec. "Step 1: Network Inference", Alg. "Network
// gradient").
#include <stdarg.h>

#include <vector>

#include "common.hpp"
#include "tune.hpp"

namespace crom {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

// Benchmark timing (crom_kernel_timer): event pairs recorded around the
// launches that follow a step's set-up kernel, per host thread.
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;  // reused across records; pairs (2i, 2i + 1)
  size_t used = 0;
};
static thread_local KernelTimer g_timer;

void timer_mark(hipStream_t st) {
  KernelTimer& t = g_timer;
  if (!t.on) return;
  if (t.used == t.ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      t.on = false;
      t.used = 0;
      return;
    }
    t.ev.push_back(e);
  }
  if (hipEventRecord(t.ev[t.used], st) == hipSuccess) ++t.used;
}

crom_status check_net(const crom_net* net, bool need_packed) {
  if (!net) return fail(CROM_ERR_INVALID_ARG, "net is NULL");
  if (net->depth < 1 || net->depth > 15) return fail(CROM_ERR_INVALID_ARG, "depth must be in [1, 15]");
  if (shape_id(net->m, net->r, net->d, net->width) == SHAPE_NONE)
    return fail(CROM_ERR_UNSUPPORTED,
                "unsupported (m, r, d, width); compiled: (1,3,1,32), (2,8,1,128), (2,16,1,128), (3,16,3,256)");
  if (net->precision < CROM_PREC_FP32 || net->precision > CROM_PREC_BF16X3)
    return fail(CROM_ERR_UNSUPPORTED, "unknown precision");
  if (net->act != CROM_ACT_ELU && net->act != CROM_ACT_SINE) return fail(CROM_ERR_UNSUPPORTED, "unknown activation");
  if (net->act == CROM_ACT_SINE &&
      ((net->precision != CROM_PREC_FP32 && net->precision != CROM_PREC_BF16) ||
       (shape_id(net->m, net->r, net->d, net->width) != SHAPE_1D && shape_id(net->m, net->r, net->d, net->width) != SHAPE_2D)))
    return fail(CROM_ERR_UNSUPPORTED, "sine activation: shapes (1,3,1,32) and (2,8,1,128), FP32 or BF16");
  if (!net->params) return fail(CROM_ERR_INVALID_ARG, "net->params is NULL");
  if (need_packed && net->depth > 1 && !net->packed)
    return fail(CROM_ERR_INVALID_ARG, "net->packed is NULL (call crom_net_pack)");
  return CROM_OK;
}

// ---------------------------------------------------------------------------
// Packing of the hidden-to-hidden weights into MFMA A-operand fragments.
// ---------------------------------------------------------------------------
// Layers 0 .. depth-2 hold W_l (A[m][k] = W_l[m][k]), then layers depth-1 ..
// 2 depth-3 the transposes (A[m][k] = W_l[k][m]) for the reverse pass of
// the latent Jacobian.
template <int W, int PREC>
__global__ void pack_kernel(const float* __restrict__ params, ParamIndex pi, int depth,
                            char* __restrict__ out) {
  constexpr int MTILES = W / 16;
  const int h = blockIdx.y;                       // packed layer 0 .. 2 (depth-1) - 1
  const bool tr = h >= depth - 1;
  const float* Wl = params + pi.w[(tr ? h - (depth - 1) : h) + 1];  // [W][W]
  // entry (row, col) of the A operand
  auto at = [&](int row, int col) { return tr ? Wl[col * W + row] : Wl[row * W + col]; };
  if constexpr (PREC == PREC_FP32) {
    constexpr int KQ = W / 16;
    constexpr int N = MTILES * KQ * 64 * 4;
    float* o = reinterpret_cast<float*>(out) + (size_t)h * N;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
      const int v = i & 3, lane = (i >> 2) & 63, kq = (i >> 8) % KQ, mt = (i >> 8) / KQ;
      o[i] = at(mt * 16 + (lane & 15), kq * 16 + (lane >> 4) * 4 + v);
    }
  } else {
    constexpr int KB = W / 32;
    constexpr int N = MTILES * KB * 64 * 8;
    __bf16* o = reinterpret_cast<__bf16*>(out) + (size_t)h * 2 * N;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
      const int e = i & 7, lane = (i >> 3) & 63, kb = (i >> 9) % KB, mt = (i >> 9) / KB;
      const float w = at(mt * 16 + (lane & 15), (2 * kb + (e >> 2)) * 16 + (lane >> 4) * 4 + (e & 3));
      const __bf16 hi = (__bf16)w;
      o[i] = hi;
      o[N + i] = (__bf16)(w - (float)hi);
    }
  }
}

static size_t packed_bytes(int w, int depth, int prec) {
  if (depth < 2) return 0;
  const size_t mt = w / 16;
  const size_t per = prec == CROM_PREC_FP32 ? mt * (w / 16) * 64 * 16 : mt * (w / 32) * 64 * 16 * 2;
  return per * 2 * (depth - 1);  // the layers, then their transposes
}

// ---------------------------------------------------------------------------
// Decode kernel: one workgroup per NB*16 points.
// ---------------------------------------------------------------------------
struct DecodeArgs {
  const float* x;
  int64_t P;
  const double* q;
  const float* params;
  const char* packed;
  ParamIndex pi;
  int depth;
  int qb;            // first latent index of the q-tangent columns
  float* g;
  float* dgdx;
  float* d2g;
  float* dgdq;
};

template <class S, class C, int NB, int NW, int PREC, int PF, int WPE>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void decode_kernel(DecodeArgs a) {
  using E = Engine<S, C, NB, NW, PREC, PF>;
  extern __shared__ __align__(16) char lds[];
  float* par = reinterpret_cast<float*>(lds + E::LDS_BYTES);
  E::PC::load(par, a.params, a.pi, a.depth, E::THREADS);  // once for all of this workgroup's batches
  __syncthreads();
  const int64_t nbatch = (a.P + E::NPTS - 1) / E::NPTS;
  for (int64_t bi = blockIdx.x; bi < nbatch; bi += gridDim.x) {
  const int64_t first = bi * E::NPTS;
  const int64_t rem = a.P - first;
  const int n_valid = rem < E::NPTS ? (int)rem : E::NPTS;
  E::stage(lds, a.x, first, n_valid, a.q, S::R, nullptr, 0, par);
  __syncthreads();
  E::run(lds, par, a.packed, a.depth, a.qb);
  const float* res = reinterpret_cast<const float*>(lds + E::RES_OFF);
  constexpr int D = S::D, M = S::M, R = S::R;
  constexpr int NHT = M * (M + 1) / 2;  // Hessian entries per output
  for (int i = threadIdx.x; i < D * E::NT * PT; i += E::THREADS) {
    const int oo = i / (E::NT * PT);
    const int t = (i / PT) % E::NT;
    const int jj = i % PT;
    const int b = t / C::C, c = t % C::C;
    const int lp = b * PT + jj;
    if (lp >= n_valid) continue;
    const int64_t p = first + lp;
    const float v = res[i];
    const int k = C::kind(c);
    if (k == CK_VAL) {
      a.g[p * D + oo] = v;
    } else if (k == CK_XT) {
      if (a.dgdx) a.dgdx[(p * D + oo) * M + (c - C::X0)] = v;
    } else if (k == CK_LAP) {
      a.d2g[p * D + oo] = v;
    } else if (k == CK_HESS) {
      a.d2g[(p * D + oo) * NHT + C::HB + (c - C::D0)] = v;
    } else if (k == CK_QT) {
      a.dgdq[(p * D + oo) * R + a.qb + (c - C::Q0)] = v;
    }
  }
  __syncthreads();  // res is read before the next batch may overwrite the LDS
  }
}

template <class S, class C, int NB, int PREC>
static crom_status launch_decode(const DecodeArgs& a, hipStream_t st) {
  using T = DecodeTune<S, PREC>;
  constexpr int NW = T::NW;
  using E = Engine<S, C, NB, NW, PREC, T::PF>;
  const int lds_bytes = E::LDS_BYTES + E::PC::bytes(a.depth);
  if (lds_bytes > LDS_MAX) {
    return fail(CROM_ERR_UNSUPPORTED, "column set does not fit in LDS at this width/precision/depth");
  } else {
    auto k = decode_kernel<S, C, NB, NW, PREC, T::PF, T::WPE>;
    static bool attr = false;
    if (!attr) {
      crom_status s = set_lds(k, LDS_MAX);
      if (s != CROM_OK) return s;
      attr = true;
    }
    int64_t blocks = (a.P + E::NPTS - 1) / E::NPTS;
    if (blocks > 0x7fffffff) return fail(CROM_ERR_INVALID_ARG, "P too large");
    // a few workgroups per CU, each looping over batches with its parameter
    // cache loaded once
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(E::THREADS), lds_bytes, st, a);
    return hip_check(hipGetLastError(), "decode launch");
  }
}

// One pass over the points with a fixed column set (value first).
template <class S, int NW, int PREC, bool XT, int D2, int NQ, int HB = 0,
          int NH = S::M * (S::M + 1) / 2>
static crom_status run_pass(const DecodeArgs& a, hipStream_t st) {
  if constexpr (!XT && D2 == D2_NONE && NQ == 0) {
    using C = Cols<S::M, S::R, 1, 0, false, D2_NONE, 0>;
    return launch_decode<S, C, DecodeTune<S, PREC>::NBV, PREC>(a, st);
  } else {
    using C = Cols<S::M, S::R, 1, 0, XT, D2, NQ, HB, NH>;
    return launch_decode<S, C, 1, PREC>(a, st);
  }
}

// Hessian entries in chunks of HC (x tangents recomputed per chunk).
template <class S, int NW, int PREC, int HC, int HB>
static crom_status hess_chunks(const DecodeArgs& a, hipStream_t st) {
  constexpr int NHT = S::M * (S::M + 1) / 2;
  if constexpr (HB >= NHT) {
    return CROM_OK;
  } else {
    constexpr int NH = (NHT - HB) < HC ? (NHT - HB) : HC;
    crom_status s = run_pass<S, NW, PREC, true, D2_HESS, 0, HB, NH>(a, st);
    if (s != CROM_OK) return s;
    return hess_chunks<S, NW, PREC, HC, HB + HC>(a, st);
  }
}

// Plans the passes of a request.  Narrow nets (width <= 128, r <= 8) take
// every column in one pass.  At width 256, or with 16 latent tangents, the
// activations of all columns would not fit in LDS, so the x tangents with
// the second derivatives form one pass (Hessian entries in chunks of HC:
// they need the x tangents' pre-activations in the same pass), and the
// latent tangents follow in chunks of QC.  Every pass rewrites the values,
// with identical results.
template <class S, int NW, int PREC, int QC, int HC>
static crom_status decode_shape(const DecodeArgs& a0, bool xt, int d2, bool qt, hipStream_t st) {
  DecodeArgs a = a0;
  const bool spatial = xt || d2 != D2_NONE;
  if constexpr (S::W <= 128 && S::R <= 8) {
#define CROM_ONE(XT, D2)                                                                  \
    if (spatial == XT && d2 == D2)                                                        \
      return qt ? run_pass<S, NW, PREC, XT, D2, S::R>(a, st) : run_pass<S, NW, PREC, XT, D2, 0>(a, st);
    CROM_ONE(false, D2_NONE)
    CROM_ONE(true, D2_NONE)
    CROM_ONE(true, D2_LAP)
    if constexpr (S::M > 1) {
      CROM_ONE(true, D2_HESS)
    }
#undef CROM_ONE
    return fail(CROM_ERR_UNSUPPORTED, "unsupported derivative column set");
  } else {
    crom_status s = CROM_OK;
    if (d2 == D2_HESS) s = hess_chunks<S, NW, PREC, HC, 0>(a, st);
    else if (d2 == D2_LAP) s = run_pass<S, NW, PREC, true, D2_LAP, 0>(a, st);
    else if (xt) s = run_pass<S, NW, PREC, true, D2_NONE, 0>(a, st);
    else if (!qt) s = run_pass<S, NW, PREC, false, D2_NONE, 0>(a, st);
    if (s != CROM_OK || !qt) return s;
    for (int qb = 0; qb < S::R; qb += QC) {
      a.qb = qb;
      s = run_pass<S, NW, PREC, false, D2_NONE, QC>(a, st);
      if (s != CROM_OK) return s;
    }
    return CROM_OK;
  }
}

template <class S, int NW>
static crom_status decode_prec(int prec, const DecodeArgs& a, bool xt, int d2, bool qt, hipStream_t st) {
  if constexpr (S::ACT == ACT_SINE) {  // FP32 and BF16 only (checked by check_net)
    if (prec == CROM_PREC_FP32) return decode_shape<S, NW, PREC_FP32, 4, 3>(a, xt, d2, qt, st);
    return decode_shape<S, NW, PREC_BF16, 8, 3>(a, xt, d2, qt, st);
  }
  switch (prec) {
    case CROM_PREC_FP32: return decode_shape<S, NW, PREC_FP32, 4, 3>(a, xt, d2, qt, st);
    case CROM_PREC_BF16: return decode_shape<S, NW, PREC_BF16, 8, 3>(a, xt, d2, qt, st);
    case CROM_PREC_BF16_PURE: return decode_shape<S, NW, PREC_BF16_PURE, 8, 6>(a, xt, d2, qt, st);
    default: return decode_shape<S, NW, PREC_BF16X3, 8, 3>(a, xt, d2, qt, st);
  }
}

static crom_status decode_any(const crom_net* net, const float* x, int64_t P, const double* q,
                              int d2_mode, float* g, float* dgdx, float* d2g, float* dgdq,
                              void* stream) {
  crom_status s = check_net(net, true);
  if (s != CROM_OK) return s;
  if (P < 0) return fail(CROM_ERR_INVALID_ARG, "P < 0");
  if (d2_mode < CROM_D2_NONE || d2_mode > CROM_D2_HESSIAN)
    return fail(CROM_ERR_INVALID_ARG, "d2_mode");
  if (d2_mode == CROM_D2_HESSIAN && net->m == 1)
    return fail(CROM_ERR_INVALID_ARG, "m = 1: use CROM_D2_LAPLACIAN");
  if (P == 0) return CROM_OK;  // nothing to do; output pointers may be NULL
  if (!x || !q || !g) return fail(CROM_ERR_INVALID_ARG, "x, q and g are required");
  if ((d2_mode != CROM_D2_NONE) != (d2g != nullptr))
    return fail(CROM_ERR_INVALID_ARG, "d2g must be given iff d2_mode != NONE");
  DecodeArgs a{};
  a.x = x;
  a.P = P;
  a.q = q;
  a.params = net->params;
  a.packed = static_cast<const char*>(net->packed);
  a.pi = param_index(net->m, net->r, net->d, net->width, net->depth);
  a.depth = net->depth;
  a.qb = 0;
  a.g = g;
  a.dgdx = dgdx;
  a.d2g = d2g;
  a.dgdq = dgdq;
  const bool xt = dgdx != nullptr;
  const int d2 = d2_mode == CROM_D2_LAPLACIAN ? D2_LAP : d2_mode == CROM_D2_HESSIAN ? D2_HESS : D2_NONE;
  const bool qt = dgdq != nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (shape_id(net->m, net->r, net->d, net->width)) {
    case SHAPE_1D:
      if (net->act == CROM_ACT_SINE) return decode_prec<Shape<32, 1, 3, 1, ACT_SINE>, 2>(net->precision, a, xt, d2, qt, st);
      return decode_prec<Shape<32, 1, 3, 1>, 2>(net->precision, a, xt, d2, qt, st);
    case SHAPE_2D:
      if (net->act == CROM_ACT_SINE) return decode_prec<Shape<128, 2, 8, 1, ACT_SINE>, 4>(net->precision, a, xt, d2, qt, st);
      return decode_prec<Shape<128, 2, 8, 1>, 4>(net->precision, a, xt, d2, qt, st);
    case SHAPE_3D: return decode_prec<Shape<256, 3, 16, 3>, 8>(net->precision, a, xt, d2, qt, st);
    case SHAPE_2D_R16: return decode_prec<Shape<128, 2, 16, 1>, 4>(net->precision, a, xt, d2, qt, st);
    default: return fail(CROM_ERR_UNSUPPORTED, "shape");
  }
}

}  // namespace crom

using namespace crom;

extern "C" {

const char* crom_last_error(void) { return g_err.c_str(); }

// Destroys the recorded events (explicitly, so that no HIP call is left
// for thread or process exit).
static void timer_release(KernelTimer& t) {
  for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  t.ev.clear();
  t.used = 0;
}

crom_status crom_kernel_timer(int32_t on) {
  g_timer.on = on != 0;
  if (on) timer_release(g_timer);
  return CROM_OK;
}

crom_status crom_kernel_timer_read(double* total_ms, int64_t* count) {
  if (!total_ms || !count) return fail(CROM_ERR_INVALID_ARG, "total_ms and count are required");
  KernelTimer& t = g_timer;
  const size_t pairs = t.used / 2;
  double sum = 0.0;
  if (pairs > 0) {
    crom_status s = hip_check(hipEventSynchronize(t.ev[2 * pairs - 1]), "hipEventSynchronize");
    if (s != CROM_OK) return s;
  }
  for (size_t i = 0; i < pairs; ++i) {
    float ms = 0.0f;
    crom_status s = hip_check(hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]), "hipEventElapsedTime");
    if (s != CROM_OK) return s;
    sum += ms;
  }
  *total_ms = sum;
  *count = (int64_t)pairs;
  if (!t.on) timer_release(t);
  return CROM_OK;
}

size_t crom_net_param_count(int32_t m, int32_t r, int32_t d, int32_t width, int32_t depth) {
  if (m < 1 || r < 0 || d < 1 || width < 1 || depth < 1) return 0;
  size_t n = (size_t)width * (m + r) + width;
  n += (size_t)(depth - 1) * ((size_t)width * width + width);
  n += (size_t)d * width + d;
  return n;
}

size_t crom_net_packed_bytes(const crom_net* net) {
  if (!net || shape_id(net->m, net->r, net->d, net->width) == SHAPE_NONE || net->depth < 1) return 0;
  return packed_bytes(net->width, net->depth, net->precision);
}

crom_status crom_net_pack(const crom_net* net, void* packed, void* stream) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (net->depth < 2) return CROM_OK;
  if (!packed) return fail(CROM_ERR_INVALID_ARG, "packed is NULL");
  ParamIndex pi = param_index(net->m, net->r, net->d, net->width, net->depth);
  hipStream_t st = static_cast<hipStream_t>(stream);
  dim3 grid(64, 2 * (net->depth - 1));
  char* out = static_cast<char*>(packed);
  const bool f32 = net->precision == CROM_PREC_FP32;
  switch (net->width) {
    case 32:
      if (f32) hipLaunchKernelGGL((pack_kernel<32, PREC_FP32>), grid, dim3(256), 0, st, net->params, pi, net->depth, out);
      else hipLaunchKernelGGL((pack_kernel<32, PREC_BF16>), grid, dim3(256), 0, st, net->params, pi, net->depth, out);
      break;
    case 128:
      if (f32) hipLaunchKernelGGL((pack_kernel<128, PREC_FP32>), grid, dim3(256), 0, st, net->params, pi, net->depth, out);
      else hipLaunchKernelGGL((pack_kernel<128, PREC_BF16>), grid, dim3(256), 0, st, net->params, pi, net->depth, out);
      break;
    case 256:
      if (f32) hipLaunchKernelGGL((pack_kernel<256, PREC_FP32>), grid, dim3(256), 0, st, net->params, pi, net->depth, out);
      else hipLaunchKernelGGL((pack_kernel<256, PREC_BF16>), grid, dim3(256), 0, st, net->params, pi, net->depth, out);
      break;
    default:
      return fail(CROM_ERR_UNSUPPORTED, "width");
  }
  return hip_check(hipGetLastError(), "pack launch");
}

crom_status crom_decode(const crom_net* net, const float* x, int64_t P, const double* q, float* g,
                        void* stream) {
  return decode_any(net, x, P, q, CROM_D2_NONE, g, nullptr, nullptr, nullptr, stream);
}

crom_status crom_decode_jac(const crom_net* net, const float* x, int64_t P, const double* q,
                            int32_t d2_mode, float* g, float* dgdx, float* d2g, float* dgdq,
                            void* stream) {
  return decode_any(net, x, P, q, d2_mode, g, dgdx, d2g, dgdq, stream);
}

crom_status crom_decode_jac_x(const crom_net* net, const float* x, int64_t P, const double* q,
                              int32_t d2_mode, float* g, float* dgdx, float* d2g, void* stream) {
  return decode_any(net, x, P, q, d2_mode, g, dgdx, d2g, nullptr, stream);
}

crom_status crom_decode_jac_q(const crom_net* net, const float* x, int64_t P, const double* q,
                              float* g, float* dgdq, void* stream) {
  if (P > 0 && !dgdq) return crom::fail(CROM_ERR_INVALID_ARG, "dgdq is required");
  return decode_any(net, x, P, q, CROM_D2_NONE, g, nullptr, nullptr, dgdq, stream);
}

}  // extern "C"
