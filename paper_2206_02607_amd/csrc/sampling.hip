// Robust greedy selection of the integration samples (Appendix "Robust
// Sampling", Alg. "Robust sampling"): the residual vectors of sample sets
// (a value decode of every node fused with the comparison against the
// full-order field), their metric, the candidate ranking, and the greedy
// loop that drives the batched rollouts of every candidate set through
// crom_step.
#include <math.h>

#include <vector>

#include "common.hpp"
#include "tune.hpp"

namespace crom {

// ---------------------------------------------------------------------------
// Residual vectors: res[s][i] = sum_k |g(x_i, q[s][k]) - ref[k][i]|_2.
// A workgroup takes 64 nodes of one set and runs the decoder for each of the
// set's n_mu latents in turn, accumulating the norms in FP64 registers (one
// thread per node), so the decoded fields never leave the chip.  Grid: node
// batches (strided) x sets.
// ---------------------------------------------------------------------------
struct ResidualArgs {
  const float* x;
  int64_t P;
  const double* q;
  const double* ref;
  int n_mu;
  const float* params;
  const char* packed;
  ParamIndex pi;
  int depth;
  double* res;
};

template <class S, int NW, int PREC, int PF, int WPE>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void residual_kernel(
    ResidualArgs a) {
  using C = Cols<S::M, S::R, 1, 0, false, D2_NONE, 0>;
  using E = Engine<S, C, 4, NW, PREC, PF>;
  static_assert(E::THREADS >= E::NPTS, "one thread per node of a batch");
  constexpr int D = S::D;
  extern __shared__ __align__(16) char lds[];
  float* par = reinterpret_cast<float*>(lds + E::LDS_BYTES);
  E::PC::load(par, a.params, a.pi, a.depth, E::THREADS);
  __syncthreads();
  const double* qs = a.q + (size_t)blockIdx.y * a.n_mu * S::R;
  const float* out = reinterpret_cast<const float*>(lds + E::RES_OFF);
  const int64_t nbatch = (a.P + E::NPTS - 1) / E::NPTS;
  const int t = threadIdx.x;
  for (int64_t bi = blockIdx.x; bi < nbatch; bi += gridDim.x) {
    const int64_t first = bi * E::NPTS;
    const int64_t rem = a.P - first;
    const int n_valid = rem < E::NPTS ? (int)rem : E::NPTS;
    double acc = 0.0;
    for (int k = 0; k < a.n_mu; ++k) {
      E::stage(lds, a.x, first, n_valid, qs + (size_t)k * S::R, S::R, nullptr, 0, par);
      __syncthreads();
      E::run(lds, par, a.packed, a.depth, 0);
      if (t < n_valid) {
        // the value of output o at node t of the batch sits at out[o * NPTS + t]
        const double* f = a.ref + ((size_t)k * a.P + first + t) * D;
        double s2 = 0.0;
#pragma unroll
        for (int o = 0; o < D; ++o) {
          const double e = (double)out[o * E::NPTS + t] - f[o];
          s2 += e * e;
        }
        acc += sqrt(s2);
      }
      __syncthreads();  // the results are read before the next pass writes them
    }
    if (t < n_valid) a.res[(size_t)blockIdx.y * a.P + first + t] = acc;
  }
}

template <class S, int PREC>
static crom_status launch_residual(const ResidualArgs& a, int n_set, hipStream_t st) {
  using T = DecodeTune<S, PREC>;
  using C = Cols<S::M, S::R, 1, 0, false, D2_NONE, 0>;
  using E = Engine<S, C, 4, T::NW, PREC, T::PF>;
  const int lds_bytes = E::LDS_BYTES + E::PC::bytes(a.depth);
  if (lds_bytes > LDS_MAX) return fail(CROM_ERR_UNSUPPORTED, "network too deep for the LDS");
  auto k = residual_kernel<S, T::NW, PREC, T::PF, T::WPE>;
  static bool attr = false;
  if (!attr) {
    crom_status s = set_lds(k, LDS_MAX);
    if (s != CROM_OK) return s;
    attr = true;
  }
  int64_t nb = (a.P + E::NPTS - 1) / E::NPTS;
  // about 4096 workgroups in all, each looping over its batches with the
  // parameter cache loaded once
  int64_t cap = 4096 / n_set;
  if (cap < 1) cap = 1;
  if (nb > cap) nb = cap;
  hipLaunchKernelGGL(k, dim3((unsigned)nb, (unsigned)n_set), dim3(E::THREADS), lds_bytes, st, a);
  return hip_check(hipGetLastError(), "residual launch");
}

template <class S>
static crom_status residual_prec(int prec, const ResidualArgs& a, int n_set, hipStream_t st) {
  switch (prec) {
    case CROM_PREC_FP32: return launch_residual<S, PREC_FP32>(a, n_set, st);
    case CROM_PREC_BF16: return launch_residual<S, PREC_BF16>(a, n_set, st);
    case CROM_PREC_BF16_PURE: return launch_residual<S, PREC_BF16_PURE>(a, n_set, st);
    default: return launch_residual<S, PREC_BF16X3>(a, n_set, st);
  }
}

// ---------------------------------------------------------------------------
// Metric: mean + max of each residual vector (one workgroup per set; fixed
// summation order; a NaN entry makes the metric NaN).
// ---------------------------------------------------------------------------
constexpr int MET_THREADS = 1024;

__device__ __forceinline__ double nan_max(double m, double v) {
  return (m != m) ? m : ((v != v || v > m) ? v : m);
}

__global__ __launch_bounds__(MET_THREADS) void metric_kernel(const double* __restrict__ res, int64_t P,
                                                             double* __restrict__ metric) {
  __shared__ double ssum[MET_THREADS];
  __shared__ double smax[MET_THREADS];
  const double* r = res + (size_t)blockIdx.x * P;
  const int t = threadIdx.x;
  double s = 0.0, m = -INFINITY;
  for (int64_t i = t; i < P; i += MET_THREADS) {
    const double v = r[i];
    s += v;
    m = nan_max(m, v);
  }
  ssum[t] = s;
  smax[t] = m;
  __syncthreads();
  for (int w = MET_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) {
      ssum[t] += ssum[t + w];
      smax[t] = nan_max(smax[t], smax[t + w]);
    }
    __syncthreads();
  }
  if (t == 0) metric[blockIdx.x] = ssum[0] / (double)P + smax[0];
}

// ---------------------------------------------------------------------------
// Candidates: n rounds of a block-wide arg-max over the nodes outside the
// set and not yet chosen (NaN ranks as +inf, ties to the lower index).
// ---------------------------------------------------------------------------
constexpr int TOP_THREADS = 1024;

__device__ __forceinline__ bool ranks_above(double v, int64_t i, double bv, int64_t bi) {
  if (i < 0) return false;
  if (bi < 0) return true;
  return v > bv || (v == bv && i < bi);
}

__global__ __launch_bounds__(TOP_THREADS) void candidates_kernel(const double* __restrict__ res, int64_t P,
                                                                 const uint8_t* __restrict__ member, int n,
                                                                 int32_t* __restrict__ cand) {
  __shared__ double sv[TOP_THREADS];
  __shared__ int64_t si[TOP_THREADS];
  __shared__ int64_t chosen[CROM_SAMPLING_MAX_TRY];
  const int t = threadIdx.x;
  for (int c = 0; c < n; ++c) {
    double bv = -INFINITY;
    int64_t bi = -1;
    for (int64_t i = t; i < P; i += TOP_THREADS) {
      if (member && member[i]) continue;
      bool taken = false;
      for (int j = 0; j < c; ++j) taken |= chosen[j] == i;
      if (taken) continue;
      double v = res[i];
      if (v != v) v = INFINITY;
      if (ranks_above(v, i, bv, bi)) {
        bv = v;
        bi = i;
      }
    }
    sv[t] = bv;
    si[t] = bi;
    __syncthreads();
    for (int w = TOP_THREADS / 2; w > 0; w >>= 1) {
      if (t < w && ranks_above(sv[t + w], si[t + w], sv[t], si[t])) {
        sv[t] = sv[t + w];
        si[t] = si[t + w];
      }
      __syncthreads();
    }
    if (t == 0) {
      chosen[c] = si[0];
      cand[c] = (int32_t)si[0];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Batch assembly for the rollouts of n_set sets x n_mu parameters: instance
// s * n_mu + k takes the members, then (when cand is given) candidate s, as
// its samples; its coefficients and initial latent are parameter k's.
// ---------------------------------------------------------------------------
struct GatherArgs {
  const float* nodes;
  const uint8_t* node_clamp;
  int m, r, ncoef;
  const int32_t* members;
  int n_members;
  const int32_t* cand;
  int n_set, n_mu;
  const double* coef_mu;
  const double* q0;
  float* y;
  uint8_t* clamp;
  int64_t* offsets;
  double* coef;
  double* q;
};

__global__ void gather_kernel(GatherArgs a) {
  const int S = a.n_members + (a.cand ? 1 : 0);
  const int64_t n_inst = (int64_t)a.n_set * a.n_mu;
  const int64_t total = n_inst * S;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t t = t0; t < total; t += stride) {
    const int64_t inst = t / S;
    const int j = (int)(t - inst * S);
    const int node = j < a.n_members ? a.members[j] : a.cand[inst / a.n_mu];
    for (int i = 0; i < a.m; ++i) a.y[t * a.m + i] = a.nodes[(int64_t)node * a.m + i];
    a.clamp[t] = a.node_clamp ? a.node_clamp[node] : 0;
  }
  for (int64_t i = t0; i <= n_inst; i += stride) a.offsets[i] = i * S;
  for (int64_t i = t0; i < n_inst * a.ncoef; i += stride) {
    const int64_t inst = i / a.ncoef;
    a.coef[i] = a.coef_mu[(inst % a.n_mu) * a.ncoef + (i - inst * a.ncoef)];
  }
  for (int64_t i = t0; i < n_inst * a.r; i += stride) {
    const int64_t inst = i / a.r;
    a.q[i] = a.q0[(inst % a.n_mu) * a.r + (i - inst * a.r)];
  }
}

// The set's member list and mask: members[n] = node, member[node] = 1.
__global__ void append_kernel(int32_t* members, uint8_t* member, int n, const int32_t* cand, int j) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int32_t node = cand[j];
    members[n] = node;
    member[node] = 1;
  }
}

__global__ void mark_kernel(const int32_t* members, int n, uint8_t* member) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) member[members[i]] = 1;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static crom_status residual_any(const crom_net* net, const float* x, int64_t P, int n_set, int n_mu,
                                const double* q, const double* ref, double* res, double* metric, hipStream_t st) {
  ResidualArgs a{};
  a.x = x;
  a.P = P;
  a.q = q;
  a.ref = ref;
  a.n_mu = n_mu;
  a.params = net->params;
  a.packed = static_cast<const char*>(net->packed);
  a.pi = param_index(net->m, net->r, net->d, net->width, net->depth);
  a.depth = net->depth;
  a.res = res;
  crom_status s;
  switch (shape_id(net->m, net->r, net->d, net->width)) {
    case SHAPE_1D: s = residual_prec<Shape<32, 1, 3, 1>>(net->precision, a, n_set, st); break;
    case SHAPE_2D: s = residual_prec<Shape<128, 2, 8, 1>>(net->precision, a, n_set, st); break;
    case SHAPE_3D: s = residual_prec<Shape<256, 3, 16, 3>>(net->precision, a, n_set, st); break;
    case SHAPE_2D_R16: s = residual_prec<Shape<128, 2, 16, 1>>(net->precision, a, n_set, st); break;
    default: return fail(CROM_ERR_UNSUPPORTED, "shape");
  }
  if (s != CROM_OK || !metric) return s;
  hipLaunchKernelGGL(metric_kernel, dim3((unsigned)n_set), dim3(MET_THREADS), 0, st, res, P, metric);
  return hip_check(hipGetLastError(), "metric launch");
}

static int pde_coefs(int kind) { return kind == CROM_PDE_HEAT ? 1 : (kind == CROM_PDE_NEOHOOKEAN ? 6 : 0); }

struct SamplingLayout {
  size_t step_ws, step_bytes, q, coef, info, y, clamp, offsets, res, metric, cand, members, member, total;
};

static crom_status sampling_layout(const crom_net* net, int kind, int n_mu, int64_t P, const crom_sampling_opts* o,
                                   SamplingLayout* L) {
  const int ncoef = pde_coefs(kind);
  if (ncoef == 0) return fail(CROM_ERR_INVALID_ARG, "unknown PDE kind");
  if (n_mu < 1) return fail(CROM_ERR_INVALID_ARG, "n_mu must be >= 1");
  if (P < 1 || P > 0x7fffffff) return fail(CROM_ERR_INVALID_ARG, "P must be in [1, 2^31)");
  if (!o) return fail(CROM_ERR_INVALID_ARG, "opts is NULL");
  if (o->n_try < 1 || o->n_try > CROM_SAMPLING_MAX_TRY)
    return fail(CROM_ERR_INVALID_ARG, "n_try must be in [1, CROM_SAMPLING_MAX_TRY]");
  if (o->max_samples < 1 || o->max_samples > P) return fail(CROM_ERR_INVALID_ARG, "max_samples must be in [1, P]");
  if (o->n_steps < 1) return fail(CROM_ERR_INVALID_ARG, "n_steps must be >= 1");
  const int64_t n_inst = (int64_t)o->n_try * n_mu;
  if (n_inst > 0x7fffffff) return fail(CROM_ERR_INVALID_ARG, "n_try * n_mu too large");
  const int64_t total = n_inst * o->max_samples;
  size_t step_bytes = 0;
  crom_status s = crom_step_workspace(net, (int32_t)n_inst, total, &step_bytes);
  if (s != CROM_OK) return s;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  const size_t r = (size_t)net->r;
  L->step_bytes = step_bytes;
  L->step_ws = take(step_bytes);
  L->q = take(3 * n_inst * r * sizeof(double));
  L->coef = take(n_inst * ncoef * sizeof(double));
  L->info = take(n_inst * sizeof(crom_step_info));
  L->y = take(total * net->m * sizeof(float));
  L->clamp = take(total);
  L->offsets = take((n_inst + 1) * sizeof(int64_t));
  L->res = take((size_t)(o->n_try + 1) * P * sizeof(double));
  L->metric = take((o->n_try + 1) * sizeof(double));
  L->cand = take(o->n_try * sizeof(int32_t));
  L->members = take(o->max_samples * sizeof(int32_t));
  L->member = take(P);
  L->total = off;
  return CROM_OK;
}

// Position of the smallest metric: the first one on ties, NaN never ahead of a number.
static int min_metric(const double* v, int n) {
  int best = 0;
  for (int i = 1; i < n; ++i) {
    const bool nb = v[best] != v[best], ni = v[i] != v[i];
    if ((nb && !ni) || (!nb && !ni && v[i] < v[best])) best = i;
  }
  return best;
}

}  // namespace crom

using namespace crom;

extern "C" {

crom_status crom_sampling_residual(const crom_net* net, const float* nodes, int64_t P, int32_t n_set, int32_t n_mu,
                                   const double* q, const double* ref, double* res, double* metric, void* stream) {
  crom_status s = check_net(net, true);
  if (s != CROM_OK) return s;
  if (net->act != CROM_ACT_ELU) return fail(CROM_ERR_UNSUPPORTED, "sample selection: ELU networks");
  if (P < 1) return fail(CROM_ERR_INVALID_ARG, "P must be >= 1");
  if (n_set < 1 || n_set > 65535) return fail(CROM_ERR_INVALID_ARG, "n_set must be in [1, 65535]");
  if (n_mu < 1) return fail(CROM_ERR_INVALID_ARG, "n_mu must be >= 1");
  if (!nodes || !q || !ref || !res) return fail(CROM_ERR_INVALID_ARG, "nodes, q, ref and res are required");
  return residual_any(net, nodes, P, n_set, n_mu, q, ref, res, metric, static_cast<hipStream_t>(stream));
}

crom_status crom_sampling_candidates(const double* res, int64_t P, const uint8_t* member, int32_t n, int32_t* cand,
                                     void* stream) {
  if (P < 1) return fail(CROM_ERR_INVALID_ARG, "P must be >= 1");
  if (n < 1 || n > CROM_SAMPLING_MAX_TRY) return fail(CROM_ERR_INVALID_ARG, "n must be in [1, CROM_SAMPLING_MAX_TRY]");
  if (!res || !cand) return fail(CROM_ERR_INVALID_ARG, "res and cand are required");
  hipLaunchKernelGGL(candidates_kernel, dim3(1), dim3(TOP_THREADS), 0, static_cast<hipStream_t>(stream), res, P,
                     member, (int)n, cand);
  return hip_check(hipGetLastError(), "candidates launch");
}

crom_status crom_sampling_workspace(const crom_net* net, int32_t pde_kind, int32_t n_mu, int64_t P,
                                    const crom_sampling_opts* opts, size_t* bytes) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (!bytes) return fail(CROM_ERR_INVALID_ARG, "bytes is NULL");
  SamplingLayout L{};
  s = sampling_layout(net, pde_kind, n_mu, P, opts, &L);
  if (s != CROM_OK) return s;
  *bytes = L.total;
  return CROM_OK;
}

crom_status crom_robust_sampling(const crom_net* net, const crom_pde* pde, int32_t n_mu, const float* nodes,
                                 int64_t P, const uint8_t* node_clamp, const double* ref, const double* q0,
                                 const crom_gn_opts* gn, const crom_sampling_opts* opts, int32_t* samples,
                                 int32_t n_init, crom_sampling_result* result, int32_t* trace_cand,
                                 double* trace_metric, void* ws, size_t ws_bytes, void* stream) {
  crom_status s = check_net(net, true);
  if (s != CROM_OK) return s;
  if (net->act != CROM_ACT_ELU) return fail(CROM_ERR_UNSUPPORTED, "sample selection: ELU networks");
  if (!pde || !pde->coef) return fail(CROM_ERR_INVALID_ARG, "pde and pde->coef are required");
  if (!nodes || !ref || !q0 || !gn || !samples || !result || !ws)
    return fail(CROM_ERR_INVALID_ARG, "nodes, ref, q0, gn, samples, result and ws are required");
  SamplingLayout L{};
  s = sampling_layout(net, pde->kind, n_mu, P, opts, &L);
  if (s != CROM_OK) return s;
  if (ws_bytes < L.total) return fail(CROM_ERR_WORKSPACE, "workspace too small (crom_sampling_workspace)");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(CROM_ERR_WORKSPACE, "ws must be 256-byte aligned");
  if (n_init < 1 || n_init > opts->max_samples) return fail(CROM_ERR_INVALID_ARG, "n_init must be in [1, max_samples]");
  if ((int64_t)net->r > (int64_t)net->d * n_init)
    return fail(CROM_ERR_INVALID_ARG, "the initial set needs r <= d * n_init samples");
  {
    std::vector<char> seen((size_t)P, 0);
    for (int i = 0; i < n_init; ++i) {
      const int32_t v = samples[i];
      if (v < 0 || v >= P) return fail(CROM_ERR_INVALID_ARG, "initial sample index out of range");
      if (seen[v]) return fail(CROM_ERR_INVALID_ARG, "initial samples must be distinct");
      seen[v] = 1;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* W = static_cast<char*>(ws);
  const int r = net->r, ncoef = pde_coefs(pde->kind), n_try = opts->n_try;
  void* step_ws = W + L.step_ws;
  double* qb[3];
  for (int i = 0; i < 3; ++i) qb[i] = reinterpret_cast<double*>(W + L.q) + (size_t)i * n_try * n_mu * r;
  double* coef = reinterpret_cast<double*>(W + L.coef);
  crom_step_info* info = reinterpret_cast<crom_step_info*>(W + L.info);
  float* y = reinterpret_cast<float*>(W + L.y);
  uint8_t* clamp = reinterpret_cast<uint8_t*>(W + L.clamp);
  int64_t* offsets = reinterpret_cast<int64_t*>(W + L.offsets);
  double* res = reinterpret_cast<double*>(W + L.res);  // slot 0: the current set; 1..n_try: candidates
  double* metric = reinterpret_cast<double*>(W + L.metric);
  int32_t* cand = reinterpret_cast<int32_t*>(W + L.cand);
  int32_t* members = reinterpret_cast<int32_t*>(W + L.members);
  uint8_t* member = reinterpret_cast<uint8_t*>(W + L.member);

  if ((s = hip_check(hipMemcpyAsync(members, samples, (size_t)n_init * sizeof(int32_t), hipMemcpyHostToDevice, st),
                     "members upload")) != CROM_OK)
    return s;
  if ((s = hip_check(hipMemsetAsync(member, 0, (size_t)P, st), "member clear")) != CROM_OK) return s;
  hipLaunchKernelGGL(mark_kernel, dim3(1), dim3(256), 0, st, members, (int)n_init, member);
  if ((s = hip_check(hipGetLastError(), "mark launch")) != CROM_OK) return s;

  // Rollouts of n_set sets (the members, plus candidate s when given) for
  // every parameter, then their residual vectors into res_out / metric_out.
  auto evaluate = [&](int n_members, int n_set, const int32_t* cands, double* res_out,
                      double* metric_out) -> crom_status {
    const int n_inst = n_set * n_mu;
    const int64_t total = (int64_t)n_inst * (n_members + (cands ? 1 : 0));
    GatherArgs g{};
    g.nodes = nodes;
    g.node_clamp = node_clamp;
    g.m = net->m;
    g.r = r;
    g.ncoef = ncoef;
    g.members = members;
    g.n_members = n_members;
    g.cand = cands;
    g.n_set = n_set;
    g.n_mu = n_mu;
    g.coef_mu = pde->coef;
    g.q0 = q0;
    g.y = y;
    g.clamp = clamp;
    g.offsets = offsets;
    g.coef = coef;
    g.q = qb[0];
    int64_t gb = (total + 255) / 256;
    if (gb > 1024) gb = 1024;
    if (gb < 1) gb = 1;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)gb), dim3(256), 0, st, g);
    crom_status e = hip_check(hipGetLastError(), "gather launch");
    if (e != CROM_OK) return e;
    crom_pde p = *pde;
    p.coef = coef;
    int prev = 2, cur = 0, nxt = 1;
    for (int64_t n = 0; n < opts->n_steps; ++n) {
      const double* q_prev = (pde->kind == CROM_PDE_NEOHOOKEAN && n > 0) ? qb[prev] : nullptr;
      e = crom_step(net, &p, n_inst, offsets, total, y, node_clamp ? clamp : nullptr, q_prev, qb[cur], qb[nxt], gn,
                    info, step_ws, L.step_bytes, stream);
      if (e != CROM_OK) return e;
      const int old_prev = prev;
      prev = cur;
      cur = nxt;
      nxt = old_prev;
    }
    return residual_any(net, nodes, P, n_set, n_mu, qb[cur], ref, res_out, metric_out, st);
  };

  int n = n_init;
  double m_cur = NAN;
  if ((s = evaluate(n, 1, nullptr, res, metric)) != CROM_OK) return s;
  if ((s = hip_check(hipMemcpyAsync(&m_cur, metric, sizeof(double), hipMemcpyDeviceToHost, st), "metric read")) !=
      CROM_OK)
    return s;
  if ((s = hip_check(hipStreamSynchronize(st), "sync")) != CROM_OK) return s;

  std::vector<int32_t> hc(n_try);
  std::vector<double> hm(n_try);
  int rounds = 0, reached = 0;
  for (;;) {
    if (m_cur < opts->target) {
      reached = 1;
      break;
    }
    if (n >= opts->max_samples) break;
    const int64_t left = P - n;
    const int n_cand = left < n_try ? (int)left : n_try;
    if (n_cand < 1) break;
    hipLaunchKernelGGL(candidates_kernel, dim3(1), dim3(TOP_THREADS), 0, st, res, P, member, n_cand, cand);
    if ((s = hip_check(hipGetLastError(), "candidates launch")) != CROM_OK) return s;
    if ((s = evaluate(n, n_cand, cand, res + P, metric + 1)) != CROM_OK) return s;
    if ((s = hip_check(hipMemcpyAsync(hc.data(), cand, n_cand * sizeof(int32_t), hipMemcpyDeviceToHost, st),
                       "candidates read")) != CROM_OK)
      return s;
    if ((s = hip_check(hipMemcpyAsync(hm.data(), metric + 1, n_cand * sizeof(double), hipMemcpyDeviceToHost, st),
                       "metrics read")) != CROM_OK)
      return s;
    if ((s = hip_check(hipStreamSynchronize(st), "sync")) != CROM_OK) return s;
    const int j = min_metric(hm.data(), n_cand);
    if (trace_cand || trace_metric) {
      for (int c = 0; c < n_try; ++c) {
        if (trace_cand) trace_cand[(size_t)rounds * n_try + c] = c < n_cand ? hc[c] : -1;
        if (trace_metric) trace_metric[(size_t)rounds * n_try + c] = c < n_cand ? hm[c] : NAN;
      }
    }
    samples[n] = hc[j];
    hipLaunchKernelGGL(append_kernel, dim3(1), dim3(64), 0, st, members, member, n, cand, j);
    if ((s = hip_check(hipGetLastError(), "append launch")) != CROM_OK) return s;
    if ((s = hip_check(hipMemcpyAsync(res, res + (size_t)(1 + j) * P, (size_t)P * sizeof(double),
                                      hipMemcpyDeviceToDevice, st),
                       "residual copy")) != CROM_OK)
      return s;
    ++n;
    ++rounds;
    m_cur = hm[j];
  }
  result->n_samples = n;
  result->reached = reached;
  result->rounds = rounds;
  result->_pad = 0;
  result->metric = m_cur;
  return CROM_OK;
}

}  // extern "C"
