// Latent step q_n -> q_{n+1} for a ragged batch of instances (Sec. "Method:
// Latent Space Dynamics"; Alg. "Latent-space dynamics", "Network inference",
// "Network inversion"; Sec. "Network Inversion", "Linearization").
//
// Two launches per step, both on the caller's stream with no host sync:
//   setup   block map (16-sample batches of every instance), state init
//   step    one cooperative (co-resident, persistent) kernel that loops:
//     eval_jets    value, x tangents, Laplacian and latent Jacobian at q_n;
//                  heat update f_{n+1} = g + dt nu Lap g (FP64), residual
//                  rho_0 = f_{n+1} - g(q_n) = dt nu Lap g (formed directly),
//                  and per-batch partial sums of J^T J, J^T rho and
//                  1/2 rho^T rho (FP64)
//     solve        per instance: fixed-order sum of the partials, Armijo test
//                  of the evaluated trials, Cholesky of J^T J, next direction
//     eval_trials  the decoder differences g(q_t) - g(q_n) at four line-search
//                  trials q_t = q + alpha_t delta and the Jacobian at the
//                  first one; residual rho_t = rho_0 - (g(q_t) - g(q_n)),
//                  with the same partial sums
// The residual is the paper's f_{n+1} - g(q) written incrementally: over a
// time step g moves by a small fraction of its size, and a difference
// carried through the network keeps its rounding error relative to itself,
// where a difference of two separately rounded values would not.
//   with a grid barrier between phases, until every instance is done or a
//   bound on the rounds (enough for max_iter iterations with ls_max shrinks)
//   is reached.  Every workgroup takes the same branch at every barrier: the
//   loop test reads a counter that only the solve phase writes.
#include <hip/hip_cooperative_groups.h>

#include "common.hpp"

namespace cg = cooperative_groups;

namespace crom {

constexpr int RMAX = 16;
constexpr int TV = 4;  // line-search trials per round
enum { PH_INIT = 0, PH_TRIALS = 1, PH_REJAC = 2, PH_DONE = 3 };

struct GNState {
  double q[RMAX];       // accepted iterate
  double delta[RMAX];   // Gauss-Newton direction at q
  double qt[TV][RMAX];  // latents evaluated by the next round (trial 0 also gets J)
  double qd[TV][RMAX];  // the same latents minus q_n
  double alpha[TV];
  double phi, slope, dnorm, pad0;
  double obj_first, obj_last;
  int32_t phase, iters, ls_evals, flags, ls_tried, rounds;
};

struct WsLayout {
  size_t blk_start, blk_inst, first_blk, nblk, active, targets, rho0, partials, state, total;
  int64_t nblk_max;
  int nred;
};

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static WsLayout ws_layout(int r, int d, int n_inst, int64_t total) {
  WsLayout L{};
  L.nblk_max = total / PT + n_inst;
  L.nred = r * (r + 1) / 2 + r + TV;
  size_t o = 0;
  L.blk_start = o; o = align256(o + 8 * (size_t)L.nblk_max);
  L.blk_inst = o;  o = align256(o + 4 * (size_t)L.nblk_max);
  L.first_blk = o; o = align256(o + 4 * (size_t)(n_inst + 1));
  L.nblk = o;      o = align256(o + 8);
  L.active = o;    o = align256(o + 8);
  L.targets = o;   o = align256(o + 8 * (size_t)total * d);
  L.rho0 = o;      o = align256(o + 8 * (size_t)total * d);
  L.partials = o;  o = align256(o + 8 * (size_t)L.nblk_max * L.nred);
  L.state = o;     o = align256(o + sizeof(GNState) * (size_t)n_inst);
  L.total = o;
  return L;
}

struct StepArgs {
  const float* params;
  const char* packed;
  ParamIndex pi;
  int depth, r, n_inst;
  int64_t total;
  const int64_t* offsets;
  const float* y;
  const uint8_t* clamp;
  const double* coef;
  double dt;
  const double* q_n;
  double* q_next;
  crom_step_info* info;
  char* ws;
  WsLayout L;
  int max_iter, linearized, ls_max;
  double tol, armijo_c, shrink;
};

template <class T>
__device__ __forceinline__ T* wsp(const StepArgs& a, size_t off) {
  return reinterpret_cast<T*>(a.ws + off);
}

// ---------------------------------------------------------------------------
// Block map and state initialisation (one workgroup of 256 threads).
// Offsets that are not a valid CSR array (a negative size, a range outside
// [0, total]) give every instance zero batches: nothing is evaluated and the
// instances end SINGULAR.  Valid CSR ranges are disjoint, so the batch count
// stays within the bound the workspace was sized for.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void setup_kernel(StepArgs a) {
  int32_t* first_blk = wsp<int32_t>(a, a.L.first_blk);
  int64_t* blk_start = wsp<int64_t>(a, a.L.blk_start);
  int32_t* blk_inst = wsp<int32_t>(a, a.L.blk_inst);
  GNState* st = wsp<GNState>(a, a.L.state);
  __shared__ int32_t scan[256];
  __shared__ int32_t carry;
  int bad = 0;
  for (int i = threadIdx.x; i < a.n_inst; i += 256) {
    const int64_t lo = a.offsets[i], hi = a.offsets[i + 1];
    bad |= !(lo >= 0 && hi >= lo && hi <= a.total);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c = 0; c < a.n_inst; c += 256) {
    const int i = c + threadIdx.x;
    int32_t nb = 0;
    if (i < a.n_inst && !bad) nb = (int32_t)((a.offsets[i + 1] - a.offsets[i] + PT - 1) / PT);
    scan[threadIdx.x] = nb;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {  // inclusive Hillis-Steele scan
      const int32_t v = threadIdx.x >= d ? scan[threadIdx.x - d] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < a.n_inst) first_blk[i] = carry + scan[threadIdx.x] - nb;
    __syncthreads();
    if (threadIdx.x == 255) carry += scan[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    first_blk[a.n_inst] = carry;
    *wsp<int64_t>(a, a.L.nblk) = carry;
    *wsp<int64_t>(a, a.L.active) = a.n_inst;
  }
  __syncthreads();
  // batches: instance i owns first_blk[i] .. first_blk[i+1]-1
  for (int i = threadIdx.x; i < a.n_inst; i += 256) {
    const int32_t b0 = first_blk[i], b1 = first_blk[i + 1];
    for (int32_t b = b0; b < b1; ++b) {
      blk_start[b] = a.offsets[i] + (int64_t)(b - b0) * PT;
      blk_inst[b] = i;
    }
  }
  // state: one 8-byte word per thread step
  constexpr int NWORD = sizeof(GNState) / 8;
  for (int64_t w = threadIdx.x; w < (int64_t)a.n_inst * NWORD; w += 256) {
    const int i = (int)(w / NWORD), k = (int)(w % NWORD);
    GNState* s = st + i;
    uint64_t* word = reinterpret_cast<uint64_t*>(s) + k;
    const int qk = k;  // q[] occupies the first RMAX words
    if (qk < RMAX) {
      const double v = qk < a.r ? a.q_n[(int64_t)i * a.r + qk] : 0.0;
      *reinterpret_cast<double*>(word) = v;
    } else {
      *word = 0;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.n_inst; i += 256) {
    st[i].obj_first = st[i].obj_last = __builtin_nan("");
    st[i].phase = PH_INIT;
  }
}

// Partial sums of one batch from per-point J rows and residuals staged in LDS
// (jd [PT][R], rho [PT][TV], both FP64; invalid points hold zeros).
template <int R>
__device__ __forceinline__ void batch_partials(const double* jd, const double* rho, double* out) {
  constexpr int NA = R * (R + 1) / 2;
  constexpr int NRED = NA + R + TV;
  for (int e = threadIdx.x; e < NRED; e += blockDim.x) {
    double s = 0.0;
    if (e < NA) {
      int a = 0, rem = e, n = R;
      while (rem >= n) { rem -= n; ++a; --n; }
      const int b = a + rem;
      for (int i = 0; i < PT; ++i) s += jd[i * R + a] * jd[i * R + b];
    } else if (e < NA + R) {
      const int k = e - NA;
      for (int i = 0; i < PT; ++i) s += jd[i * R + k] * rho[i * TV];
    } else {
      const int t = e - NA - R;
      for (int i = 0; i < PT; ++i) s += 0.5 * rho[i * TV + t] * rho[i * TV + t];
    }
    out[e] = s;
  }
}


// ---------------------------------------------------------------------------
// Evaluation of one 16-sample batch (all threads of the workgroup).
// ---------------------------------------------------------------------------
template <class S, int NW, int PREC>
__device__ void eval_jets_batch(const StepArgs& a, char* lds, int64_t blk) {
  constexpr int R = S::R;
  using C = Cols<S::M, R, 1, 0, true, D2_LAP, R>;
  using E = Engine<S, C, 1, NW, PREC>;
  const int inst = wsp<int32_t>(a, a.L.blk_inst)[blk];
  const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
  const int64_t rem = a.offsets[inst + 1] - first;
  const int n_valid = rem < PT ? (int)rem : PT;
  E::stage(lds, a.y, first, n_valid, a.q_n + (int64_t)inst * R, R, nullptr, 0, a.params, a.pi);
  __syncthreads();
  E::run(lds, a.params, a.pi, a.packed, a.depth, 0);
  const float* res = reinterpret_cast<const float*>(lds + E::RES_OFF);
  double* jd = reinterpret_cast<double*>(lds);  // the activation region is free now
  double* rho = jd + PT * R;
  double* targets = wsp<double>(a, a.L.targets);
  double* rho0 = wsp<double>(a, a.L.rho0);
  if (threadIdx.x < PT) {
    const int i = threadIdx.x;
    const bool valid = i < n_valid;
    const int64_t p = first + i;
    const double gv = (double)res[0 * PT + i];
    const double lap = (double)res[C::D0 * PT + i];
    const bool clamped = valid && a.clamp && a.clamp[p];
    const double r0 = clamped ? -gv : a.dt * a.coef[inst] * lap;
    if (valid) {
      targets[p] = clamped ? 0.0 : gv + r0;
      rho0[p] = r0;
    }
    rho[i * TV] = valid ? r0 : 0.0;
    for (int t = 1; t < TV; ++t) rho[i * TV + t] = 0.0;
    for (int k = 0; k < R; ++k) jd[i * R + k] = valid ? (double)res[(C::Q0 + k) * PT + i] : 0.0;
  }
  __syncthreads();
  batch_partials<R>(jd, rho, wsp<double>(a, a.L.partials) + blk * a.L.nred);
  __syncthreads();
}

template <class S, int NW, int PREC>
__device__ void eval_trials_batch(const StepArgs& a, char* lds, int64_t blk, int inst) {
  constexpr int R = S::R;
  using C = Cols<S::M, R, 1, TV, false, D2_NONE, R>;
  using E = Engine<S, C, 1, NW, PREC>;
  const GNState* st = wsp<GNState>(a, a.L.state) + inst;
  const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
  const int64_t rem = a.offsets[inst + 1] - first;
  const int n_valid = rem < PT ? (int)rem : PT;
  E::stage(lds, a.y, first, n_valid, a.q_n + (int64_t)inst * R, R, &st->qd[0][0], RMAX, a.params,
           a.pi);
  __syncthreads();
  E::run(lds, a.params, a.pi, a.packed, a.depth, 0);
  const float* res = reinterpret_cast<const float*>(lds + E::RES_OFF);
  double* jd = reinterpret_cast<double*>(lds);
  double* rho = jd + PT * R;
  const double* rho0 = wsp<double>(a, a.L.rho0);
  if (threadIdx.x < PT) {
    const int i = threadIdx.x;
    const bool valid = i < n_valid;
    const double r0 = valid ? rho0[first + i] : 0.0;
    for (int t = 0; t < TV; ++t) rho[i * TV + t] = valid ? r0 - (double)res[(C::F0 + t) * PT + i] : 0.0;
    for (int k = 0; k < R; ++k) jd[i * R + k] = valid ? (double)res[(C::Q0 + k) * PT + i] : 0.0;
  }
  __syncthreads();
  batch_partials<R>(jd, rho, wsp<double>(a, a.L.partials) + blk * a.L.nred);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Gauss-Newton control of one instance.  The workgroup copies the state to
// LDS and sums the partials in a fixed order (every thread a strided subset
// of the batches for one entry, then the subsets in order); thread 0 then
// takes the decisions on register copies; the workgroup writes the state
// back.
// ---------------------------------------------------------------------------
template <int R>
__device__ void solve_instance(const StepArgs& a, char* lds, int inst, bool is_last) {
  constexpr int NA = R * (R + 1) / 2;
  constexpr int NRED = NA + R + TV;
  constexpr int NWORD = sizeof(GNState) / 8;
  GNState* gst = wsp<GNState>(a, a.L.state) + inst;
  GNState* st = reinterpret_cast<GNState*>(lds);
  double* sub = reinterpret_cast<double*>(lds + ((sizeof(GNState) + 15) / 16) * 16);
  const int nth = blockDim.x;
  const int NS = nth / NRED;  // strided subsets per entry
  double* red = sub + NS * NRED;
  for (int w = threadIdx.x; w < NWORD; w += nth)
    reinterpret_cast<uint64_t*>(st)[w] = reinterpret_cast<const uint64_t*>(gst)[w];
  __syncthreads();
  const int phase = st->phase;
  if (phase == PH_DONE) {
    __syncthreads();
    return;
  }
  const int32_t* first_blk = wsp<int32_t>(a, a.L.first_blk);
  const int32_t b0 = first_blk[inst], b1 = first_blk[inst + 1];
  const double* part = wsp<double>(a, a.L.partials);
  if (threadIdx.x < NS * NRED) {
    const int e = threadIdx.x % NRED, sl = threadIdx.x / NRED;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int32_t b = b0 + sl;
    for (; b + 3 * NS < b1; b += 4 * NS) {
      s0 += part[(int64_t)b * NRED + e];
      s1 += part[(int64_t)(b + NS) * NRED + e];
      s2 += part[(int64_t)(b + 2 * NS) * NRED + e];
      s3 += part[(int64_t)(b + 3 * NS) * NRED + e];
    }
    for (; b < b1; b += NS) s0 += part[(int64_t)b * NRED + e];
    sub[sl * NRED + e] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  if (threadIdx.x < NRED) {
    double s = 0.0;
    for (int sl = 0; sl < NS; ++sl) s += sub[sl * NRED + threadIdx.x];
    red[threadIdx.x] = s;
  }
  __syncthreads();

  if (threadIdx.x == 0) {
    const double* qn0 = a.q_n + (int64_t)inst * R;
    double q[R], dl[R], qn0r[R], alpha[TV];
    for (int k = 0; k < R; ++k) {
      q[k] = st->q[k];
      dl[k] = st->delta[k];
      qn0r[k] = qn0[k];
    }
    for (int t = 0; t < TV; ++t) alpha[t] = st->alpha[t];
    double phi = st->phi, slope = st->slope, dnorm = st->dnorm;
    int iters = st->iters, ls_evals = st->ls_evals, flags = st->flags, ls_tried = st->ls_tried;
    int ph = phase;
    if (ph != PH_INIT) st->rounds += 1;
    const double* bv = red + NA;
    const double* phit = red + NA + R;
    bool done = false, newdir = false;
    int settrials = 0;  // 1: trials q + alpha_t delta; 2: every trial at q (re-linearise)
    if (ph == PH_INIT) {
      st->obj_first = st->obj_last = phi = phit[0];
      newdir = true;
    } else if (ph == PH_TRIALS) {
      int acc = -1;
      for (int t = 0; t < TV; ++t) {
        if (ls_tried + t > a.ls_max) break;
        ls_evals += 1;
        const double pt = phit[t];
        if (isfinite(pt) && pt <= phi - a.armijo_c * alpha[t] * slope) {
          acc = t;
          break;
        }
      }
      if (acc < 0) {
        ls_tried += TV;
        if (ls_tried > a.ls_max) {
          flags |= CROM_FLAG_LS_FAIL;
          done = true;
        } else {
          double al = alpha[TV - 1];
          for (int t = 0; t < TV; ++t) {
            al *= a.shrink;
            alpha[t] = al;
          }
          settrials = 1;
        }
      } else {
        double qn = 0.0;
        for (int k = 0; k < R; ++k) qn += q[k] * q[k];
        qn = sqrt(qn);
        const double step = alpha[acc] * dnorm;
        for (int k = 0; k < R; ++k) q[k] = st->qt[acc][k];
        iters += 1;
        phi = phit[acc];
        st->obj_last = phi;
        if (step <= a.tol * (1.0 + qn)) {
          done = true;
        } else if (iters >= a.max_iter) {
          flags |= CROM_FLAG_MAXITER;
          done = true;
        } else if (acc == 0) {
          newdir = true;
        } else {
          ph = PH_REJAC;
          settrials = 2;
        }
      }
    } else {  // PH_REJAC: J^T J and J^T rho at the accepted iterate
      newdir = true;
    }

    if (newdir) {
      bool finite = isfinite(phi);
      for (int e = 0; e < NA + R; ++e) finite = finite && isfinite(red[e]);
      if (!finite) {
        flags |= CROM_FLAG_NONFINITE;
        done = true;
      } else {
        double L[R][R];
        double A[R][R];
        {
          int e = 0;
          for (int i = 0; i < R; ++i)
            for (int j = i; j < R; ++j) {
              A[i][j] = red[e];
              A[j][i] = red[e];
              ++e;
            }
        }
        double dmax = A[0][0];
        for (int i = 1; i < R; ++i) dmax = fmax(dmax, A[i][i]);
        const double thresh = 1e-14 * dmax;
        bool ok = true;
        for (int j = 0; j < R; ++j) {
          double sj = A[j][j];
          for (int k = 0; k < j; ++k) sj -= L[j][k] * L[j][k];
          if (!(isfinite(sj) && sj > thresh)) {
            ok = false;
            break;
          }
          L[j][j] = sqrt(sj);
          for (int i = j + 1; i < R; ++i) {
            double t = A[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
          }
        }
        if (!ok) {
          flags |= CROM_FLAG_SINGULAR;
          done = true;
        } else {
          double y[R], x[R];
          for (int i = 0; i < R; ++i) {
            double t = bv[i];
            for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
            y[i] = t / L[i][i];
          }
          for (int i = R - 1; i >= 0; --i) {
            double t = y[i];
            for (int k = i + 1; k < R; ++k) t -= L[k][i] * x[k];
            x[i] = t / L[i][i];
          }
          double dn = 0.0, qn = 0.0, sl = 0.0;
          for (int k = 0; k < R; ++k) {
            dl[k] = x[k];
            dn += x[k] * x[k];
            qn += q[k] * q[k];
            sl += bv[k] * x[k];
          }
          dnorm = sqrt(dn);
          if (a.linearized) {
            for (int k = 0; k < R; ++k) q[k] += x[k];
            iters = 1;
            done = true;
          } else if (dnorm <= a.tol * (1.0 + sqrt(qn))) {
            done = true;
          } else {
            slope = sl;
            ls_tried = 0;
            double al = 1.0;
            for (int t = 0; t < TV; ++t) {
              alpha[t] = al;
              al *= a.shrink;
            }
            ph = PH_TRIALS;
            settrials = 1;
          }
        }
      }
    }
    if (!done && is_last) {
      flags |= CROM_FLAG_MAXITER;
      done = true;
    }
    if (!done && settrials) {
      for (int t = 0; t < TV; ++t) {
        const double al = settrials == 1 ? alpha[t] : 0.0;
        for (int k = 0; k < R; ++k) {
          st->qt[t][k] = q[k] + al * dl[k];
          st->qd[t][k] = (q[k] - qn0r[k]) + al * dl[k];
        }
      }
    }
    if (done) {
      ph = PH_DONE;
      atomicAdd(reinterpret_cast<unsigned long long*>(wsp<int64_t>(a, a.L.active)),
                (unsigned long long)-1ll);
    }
    for (int k = 0; k < R; ++k) {
      st->q[k] = q[k];
      st->delta[k] = dl[k];
      a.q_next[(int64_t)inst * R + k] = q[k];
    }
    for (int t = 0; t < TV; ++t) st->alpha[t] = alpha[t];
    st->phi = phi;
    st->slope = slope;
    st->dnorm = dnorm;
    st->iters = iters;
    st->ls_evals = ls_evals;
    st->flags = flags;
    st->ls_tried = ls_tried;
    st->phase = ph;
    crom_step_info inf;
    inf.flags = flags;
    inf.iters = iters;
    inf.ls_evals = ls_evals;
    inf.rounds = st->rounds;
    inf.obj_first = st->obj_first;
    inf.obj_last = st->obj_last;
    a.info[inst] = inf;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < NWORD; w += nth)
    reinterpret_cast<uint64_t*>(gst)[w] = reinterpret_cast<const uint64_t*>(st)[w];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// The persistent step kernel (cooperative launch: every workgroup resident).
// ---------------------------------------------------------------------------
template <class S, int NW, int PREC>
__global__ __launch_bounds__(NW * 64) void step_kernel(StepArgs a, int max_rounds) {
  extern __shared__ __align__(16) char lds[];
  cg::grid_group grid = cg::this_grid();
  const int64_t nblk = *wsp<int64_t>(a, a.L.nblk);
  const int32_t* blk_inst = wsp<int32_t>(a, a.L.blk_inst);
  const GNState* state = wsp<GNState>(a, a.L.state);
  int64_t* active = wsp<int64_t>(a, a.L.active);

  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) eval_jets_batch<S, NW, PREC>(a, lds, blk);
  grid.sync();
  for (int inst = blockIdx.x; inst < a.n_inst; inst += gridDim.x)
    solve_instance<S::R>(a, lds, inst, max_rounds == 0);
  grid.sync();
  for (int round = 0; round < max_rounds; ++round) {
    if (__hip_atomic_load(active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
      const int inst = blk_inst[blk];
      const int ph = __hip_atomic_load(&state[inst].phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ph == PH_TRIALS || ph == PH_REJAC) eval_trials_batch<S, NW, PREC>(a, lds, blk, inst);
    }
    grid.sync();
    for (int inst = blockIdx.x; inst < a.n_inst; inst += gridDim.x)
      solve_instance<S::R>(a, lds, inst, round == max_rounds - 1);
    grid.sync();
  }
}

template <class S, int NW, int PREC>
static crom_status launch_step(StepArgs a, int max_rounds, hipStream_t st) {
  using EJ = Engine<S, Cols<S::M, S::R, 1, 0, true, D2_LAP, S::R>, 1, NW, PREC>;
  using ET = Engine<S, Cols<S::M, S::R, 1, TV, false, D2_NONE, S::R>, 1, NW, PREC>;
  constexpr int LDS = EJ::LDS_BYTES > ET::LDS_BYTES ? EJ::LDS_BYTES : ET::LDS_BYTES;
  static_assert(LDS <= 160 * 1024, "LDS");
  static_assert(PT * S::R * 8 + PT * TV * 8 <= EJ::ACT_REGION, "staging fits");
  static_assert(PT * S::R * 8 + PT * TV * 8 <= ET::ACT_REGION, "staging fits");
  static_assert(sizeof(GNState) + 16 + (NW * 64 + S::R * (S::R + 1) / 2 + S::R + TV) * 8 <= LDS,
                "solve scratch fits");
  static_assert(NW * 64 >= S::R * (S::R + 1) / 2 + S::R + TV, "one thread per reduced entry");
  auto k = step_kernel<S, NW, PREC>;
  static int resident = 0;
  if (!resident) {
    crom_status s = set_lds(k, LDS);
    if (s != CROM_OK) return s;
    int dev = 0, per_cu = 0, ncu = 0;
    s = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (s == CROM_OK) s = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "attr");
    if (s == CROM_OK)
      s = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, NW * 64, LDS), "occupancy");
    if (s != CROM_OK) return s;
    if (per_cu < 1) return fail(CROM_ERR_UNSUPPORTED, "step kernel does not fit on a compute unit");
    resident = per_cu * ncu;
  }
  hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(256), 0, st, a);
  crom_status s = hip_check(hipGetLastError(), "setup launch");
  if (s != CROM_OK) return s;
  int64_t g = a.L.nblk_max > a.n_inst ? a.L.nblk_max : a.n_inst;
  if (g > resident) g = resident;
  if (g < 1) g = 1;
  void* args[] = {&a, &max_rounds};
  return hip_check(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k), dim3((unsigned)g),
                                              dim3(NW * 64), args, LDS, st),
                   "step launch");
}

template <class S, int NW>
static crom_status step_prec(int prec, const StepArgs& a, int rounds, hipStream_t st) {
  switch (prec) {
    case CROM_PREC_FP32: return launch_step<S, NW, PREC_FP32>(a, rounds, st);
    case CROM_PREC_BF16: return launch_step<S, NW, PREC_BF16>(a, rounds, st);
    case CROM_PREC_BF16_PURE: return launch_step<S, NW, PREC_BF16_PURE>(a, rounds, st);
    default: return launch_step<S, NW, PREC_BF16X3>(a, rounds, st);
  }
}

}  // namespace crom

using namespace crom;

extern "C" {

crom_status crom_step_workspace(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                size_t* bytes) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (!bytes) return fail(CROM_ERR_INVALID_ARG, "bytes is NULL");
  if (n_inst < 0 || total_samples < 0) return fail(CROM_ERR_INVALID_ARG, "negative size");
  *bytes = ws_layout(net->r, net->d, n_inst, total_samples).total;
  return CROM_OK;
}

const double* crom_step_targets(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                const void* ws) {
  if (!net || !ws || n_inst < 0 || total_samples < 0) return nullptr;
  WsLayout L = ws_layout(net->r, net->d, n_inst, total_samples);
  return reinterpret_cast<const double*>(static_cast<const char*>(ws) + L.targets);
}

crom_status crom_step(const crom_net* net, const crom_pde* pde, int32_t n_inst,
                      const int64_t* offsets, int64_t total_samples, const float* y,
                      const uint8_t* clamp, const double* q_n, double* q_next,
                      const crom_gn_opts* opts, crom_step_info* info, void* ws, size_t ws_bytes,
                      void* stream) {
  crom_status s = check_net(net, true);
  if (s != CROM_OK) return s;
  if (!pde || !opts) return fail(CROM_ERR_INVALID_ARG, "pde and opts are required");
  if (pde->kind != CROM_PDE_HEAT) return fail(CROM_ERR_UNSUPPORTED, "pde kind");
  if (net->d != 1) return fail(CROM_ERR_UNSUPPORTED, "the heat step needs d == 1");
  if (net->r > RMAX) return fail(CROM_ERR_UNSUPPORTED, "r > 16");
  if (n_inst < 0 || total_samples < 0) return fail(CROM_ERR_INVALID_ARG, "negative size");
  if (n_inst == 0) return CROM_OK;
  if (!offsets || !q_n || !q_next || !info || !pde->coef)
    return fail(CROM_ERR_INVALID_ARG, "offsets, q_n, q_next, info and pde->coef are required");
  if (total_samples > 0 && !y) return fail(CROM_ERR_INVALID_ARG, "y is NULL");
  if (q_next == q_n) return fail(CROM_ERR_INVALID_ARG, "q_next must not alias q_n");
  if (opts->max_iter < 1 || opts->ls_max < 0 || opts->max_rounds < 0 || !(opts->tol_step >= 0.0) ||
      !(opts->ls_shrink > 0.0 && opts->ls_shrink < 1.0) || !(opts->armijo_c >= 0.0))
    return fail(CROM_ERR_INVALID_ARG, "gn opts out of range");
  if (!(pde->dt > 0.0)) return fail(CROM_ERR_INVALID_ARG, "dt must be positive");
  WsLayout L = ws_layout(net->r, net->d, n_inst, total_samples);
  if (!ws || ws_bytes < L.total) return fail(CROM_ERR_WORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CROM_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (L.nblk_max > 0x7fffffff) return fail(CROM_ERR_INVALID_ARG, "too many samples");
  StepArgs a{};
  a.params = net->params;
  a.packed = static_cast<const char*>(net->packed);
  a.pi = param_index(net->m, net->r, net->d, net->width, net->depth);
  a.depth = net->depth;
  a.r = net->r;
  a.n_inst = n_inst;
  a.total = total_samples;
  a.offsets = offsets;
  a.y = y;
  a.clamp = clamp;
  a.coef = pde->coef;
  a.dt = pde->dt;
  a.q_n = q_n;
  a.q_next = q_next;
  a.info = info;
  a.ws = static_cast<char*>(ws);
  a.L = L;
  a.max_iter = opts->max_iter;
  a.linearized = opts->linearized;
  a.ls_max = opts->ls_max;
  a.tol = opts->tol_step;
  a.armijo_c = opts->armijo_c;
  a.shrink = opts->ls_shrink;
  // Enough rounds for max_iter accepted steps, each after the longest line
  // search (ceil((ls_max + 1) / TV) rounds) and one re-linearisation.
  const int worst = opts->max_iter * (1 + (opts->ls_max + TV) / TV) + 1;
  const int rounds = opts->linearized ? 0 : (opts->max_rounds > 0 ? opts->max_rounds : worst);
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (shape_id(net->m, net->r, net->d, net->width)) {
    case SHAPE_1D: return step_prec<Shape<32, 1, 3, 1>, 2>(net->precision, a, rounds, st);
    case SHAPE_2D: return step_prec<Shape<128, 2, 8, 1>, 4>(net->precision, a, rounds, st);
    default: return fail(CROM_ERR_UNSUPPORTED, "shape");
  }
}

}  // extern "C"
