// Latent step q_n -> q_{n+1} for a ragged batch of instances (Sec. "Method:
// Latent Space Dynamics"; Alg. "Latent-space dynamics", "Network inference",
// "Network inversion"; Sec. "Network Inversion", "Linearization").
//
// Two launches per step, both on the caller's stream with no host sync:
//   setup   block map (16-sample batches of every instance), state init
//   step    one persistent kernel (its grid never exceeds the workgroups
//           the device holds at once) running phases:
//     phase 0      eval_jets: value, x tangents, Laplacian and latent
//                  Jacobian at q_n; heat update f_{n+1} = g + dt nu Lap g
//                  (FP64); residual rho_0 = f_{n+1} - g(q_n) = dt nu Lap g,
//                  formed directly; per-batch partial sums of J^T J, J^T rho
//                  and 1/2 rho^T rho (FP64)
//     phase p > 0  eval_trials: the decoder differences g(q_t) - g(q_n) at
//                  the round's line-search trials q_t = q + alpha_t delta
//                  (TV of them, one by default) and the Jacobian at the
//                  first; rho_t = rho_0 - (g(q_t) - g(q_n)), with the same
//                  partial sums
//   The workgroup that completes the last batch of an instance in a phase
//   solves that instance at once: fixed-order sum of its partials, Armijo
//   test of the trials, Cholesky of J^T J, next direction.  A phase ends
//   when every instance that was active in it has been solved.
// Neo-Hookean elastodynamics (d = 3, m = 3) runs the same inversion after
// two preparatory launches: the decoder's value, x-gradient, x-Hessian and
// latent Jacobian at q_n for every sample (engine passes with each batch's
// own latent, Hessian and Jacobian in chunks that fit the LDS), then the
// per-sample FP64 update (F = I + du/dX, div P through the Hessian,
// velocity from the latent Jacobian, symplectic Euler) giving
// rho_0 = u_{n+1} - u(q_n) = dt v_{n+1} directly; phase 0 then only sums
// the partials of the stored Jacobian and rho_0.  Corotated elasticity with
// finite-element forces replaces the x-Hessian passes by a decode of the
// samples' one-ring and a per-sample FP64 force assembly over the incident
// tetrahedra (fe_prepare); the inversion is the same.  An optional initial
// guess per instance costs one round (PH_GUESS) and becomes the start when
// its objective is lower.  Large batches run the same phases as round
// kernels (one evaluation launch and one solve launch per round).
// The residual is the paper's f_{n+1} - g(q) written incrementally: over a
// time step g moves by a small fraction of its size, and a difference
// carried through the network keeps its rounding error relative to itself,
// where a difference of two separately rounded values would not.
//
// Synchronisation.  Workgroups exchange only the batch partials, the
// per-instance state and a few counters, always through device-coherent
// loads and stores (relaxed atomics at agent scope: they bypass the
// per-XCD L2 caches, which are not coherent with each other), and every
// thread waits for its stores to complete before its workgroup signals.
// No device-wide fence is taken, so the decoder weights stay cached across
// phases.  Waits are bounded: a wait that exceeds its bound (about two
// seconds) sets an abort word, every workgroup leaves, and the unfinished
// instances report CROM_FLAG_ABORTED.
#include <stddef.h>

#include "common.hpp"
#include "tune.hpp"

// Launch shapes of the step kernels (waves, weight fragments, waves per SIMD
// left room for); the linearised step is measured like the decode kernels.
// Gauss-Newton problems with more batches than this run as round kernels.
#ifndef ROUNDS_MIN_BATCHES
#define ROUNDS_MIN_BATCHES 1024
#endif
#ifndef CROM_ELASTIC_NW
#define CROM_ELASTIC_NW 4
#endif
// The elastic step runs one workgroup of four waves per compute unit, so no
// other wave hides the weight fragments' load latency: they are streamed two
// K-blocks ahead (single instance, 500 samples, Gauss-Newton: BF16 0.706 ->
// 0.686 ms, FP32 1.610 -> 1.584 ms per step).
#ifndef CROM_ELASTIC_PF
#define CROM_ELASTIC_PF 3
#endif
#ifndef CROM_STEP2D_NW
#define CROM_STEP2D_NW 8
#endif
// 2D BF16 step kernel: 8 waves with weight fragments streamed one K-block
// ahead (held-and-prefetched fragments spilled 124 bytes per lane; single
// instance at 2,000 samples: 0.212 ms prefetched, 0.207 ms streamed, 0.206
// ms loaded per layer with 20 bytes of spill; 4 waves 0.26-0.27 ms).
#ifndef CROM_STEP2D_PF
#define CROM_STEP2D_PF 2
#endif
#ifndef CROM_STEP2D_WPE
#define CROM_STEP2D_WPE 1
#endif
#ifndef CROM_LIN_WPE
#define CROM_LIN_WPE 2
#endif
#ifndef CROM_LIN_PF
#define CROM_LIN_PF 2
#endif
#ifndef CROM_LIN_NW
#define CROM_LIN_NW 4
#endif
// The reverse-pass linearised evaluation (42 KB of LDS) runs three
// workgroups per compute unit at 168 registers (three waves per SIMD):
// 512 instances of the 2D decoder, BF16, 1.10 ms against 1.29 ms at two.
#ifndef CROM_LIN_REV_WPE
#define CROM_LIN_REV_WPE 3
#endif
// The Gauss-Newton round kernel holds three engines (the jets, the trial
// with Jacobian, the objective alone): two waves per SIMD keep it free of
// spills (three spill 80 registers).
#ifndef CROM_GN_REV_WPE
#define CROM_GN_REV_WPE 2
#endif

namespace crom {

constexpr int RMAX = 16;
// Line-search trials evaluated per round.  More trials per round cut the
// rounds an instance needs when the line search backtracks, at the price of
// wider evaluations in every round.  Measured (BF16): the single-instance 2D
// heat step at 2,000 samples, where almost every first trial is accepted,
// takes 0.157 ms with one trial per round and 0.203 ms with four; the batch
// of 512 trained instances, which backtrack (11.5 trials per instance and
// step), took 24.8 ms with one and 21.6 ms with four, and 22.9 ms with one
// once its backtracking rounds dropped the Jacobian columns.
#ifndef CROM_TRIALS
#define CROM_TRIALS 1
#endif
constexpr int TV = CROM_TRIALS;

// The reverse-pass evaluations: value, x tangents and Laplacian (the
// evaluation at q_n), and value with the trial differences (a trial round
// that re-linearises), each with the latent Jacobian by the adjoint pass.
template <class S, int NW, int PREC, int PF, bool CANON = true>
using RevLap = RevJets<S, Cols<S::M, S::R, 1, 0, true, D2_LAP, 0>, NW, PREC, PF, CANON>;
template <class S, int NW, int PREC, int PF>
using RevTrial = RevJets<S, Cols<S::M, S::R, 1, TV, false, D2_NONE, 0>, NW, PREC, PF>;
constexpr int MAXP = 256;    // bound on the phases of one step
// Instance phases: the first evaluation at q_n; line-search trials along a
// direction; re-linearisation at an accepted iterate; the evaluation of an
// initial guess (a second candidate start); finished.
enum { PH_INIT = 0, PH_TRIALS = 1, PH_REJAC = 2, PH_DONE = 3, PH_GUESS = 4 };
// phases whose rounds evaluate the trial latents (and J at the first)
__host__ __device__ constexpr bool evaluates_trials(int ph) {
  return ph == PH_TRIALS || ph == PH_REJAC || ph == PH_GUESS;
}

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

// 8-byte words of GNState that the set-up kernel writes for every instance
// (the phase and its flags); the rest of the state is formed by the first
// solve from q_n, so the set-up stays short for large batches.
constexpr int GN_W_OBJ = (int)(offsetof(GNState, obj_first) / 8);
constexpr int GN_W_PHASE = (int)(offsetof(GNState, phase) / 8);    // phase and iters share this word
constexpr int GN_W_FLAGS = (int)(offsetof(GNState, ls_evals) / 8);  // ls_evals and flags

// Word w of an instance's state before its first solve.
__device__ __forceinline__ uint64_t gn_initial_word(int w, const double* q_n, int r, bool empty) {
  if (w < RMAX) return w < r ? (uint64_t)__double_as_longlong(q_n[w]) : 0;  // q[] occupies the first RMAX words
  if (w == GN_W_OBJ || w == GN_W_OBJ + 1) return (uint64_t)__double_as_longlong(__builtin_nan(""));
  if (w == GN_W_PHASE) return (uint64_t)(uint32_t)(empty ? PH_DONE : PH_INIT);  // iters = 0 in the high half
  if (w == GN_W_FLAGS) return empty ? ((uint64_t)(uint32_t)CROM_FLAG_SINGULAR << 32) : 0;  // ls_evals = 0, flags
  return 0;
}

struct WsLayout {
  size_t blk_start, blk_inst, first_blk, nblk, sync, act_phase, inst_cnt, inv, targets, rho0, partials,
      state, jets, work, work_cnt, jbuf, bcnt, total;
  int64_t nblk_max;
  int nred;
  int nj;  // FP32 values per sample in the jets buffer (0: none)
};

// Per-sample decoder derivatives kept for the elastic update (d = 3, m = 3):
// value [d], du/dX [d][m], Hessian upper triangle [d][m(m+1)/2], du/dq [d][r].
struct JetsLayout {
  int d, m, r, nh;
  __host__ __device__ int val(int k) const { return k; }
  __host__ __device__ int grad(int k, int l) const { return d + k * m + l; }
  __host__ __device__ int hess(int k, int h) const { return d + d * m + k * nh + h; }
  __host__ __device__ int jac(int k, int i) const { return d + d * m + d * nh + k * r + i; }
  __host__ __device__ int count() const { return d + d * m + d * nh + d * r; }
};

// sync words (one 256-byte line each): solved count, abort flag, count of
// workgroups that have left the persistent kernel
enum { SYNC_SOLVED = 0, SYNC_ABORT = 32, SYNC_EXITED = 64 };

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static WsLayout ws_layout(int r, int d, int m, int n_inst, int64_t total) {
  WsLayout L{};
  L.nj = d == 3 ? JetsLayout{d, m, r, m * (m + 1) / 2}.count() : 0;
  L.nblk_max = total / PT + n_inst;
  L.nred = r * (r + 1) / 2 + r + TV;
  size_t o = 0;
  L.blk_start = o; o = align256(o + 8 * (size_t)L.nblk_max);
  L.blk_inst = o;  o = align256(o + 4 * (size_t)L.nblk_max);
  L.first_blk = o; o = align256(o + 4 * (size_t)(n_inst + 1));
  L.nblk = o;      o = align256(o + 8);
  L.sync = o;      o = align256(o + 768);
  L.act_phase = o; o = align256(o + 8 * (size_t)(MAXP + 2));
  L.inst_cnt = o;  o = align256(o + 4 * (size_t)n_inst);
  L.inv = o;       o = align256(o + 4 * (size_t)n_inst);  // elastic: det F <= 0 met at a free sample
  L.targets = o;   o = align256(o + 8 * (size_t)total * d);
  L.rho0 = o;      o = align256(o + 8 * (size_t)total * d);
  L.partials = o;  o = align256(o + 8 * (size_t)L.nblk_max * L.nred);
  L.state = o;     o = align256(o + sizeof(GNState) * (size_t)n_inst);
  L.jets = o;      o = align256(o + 4 * (size_t)total * L.nj);
  L.work = o;      o = align256(o + 4 * 2 * (size_t)L.nblk_max);  // round kernels: two batch lists
  L.work_cnt = o;  o = align256(o + 16);
  // elastic step: each batch's Jacobian rows and residuals, assembled from
  // the workgroups of its latent-tangent chunks, and their arrival counts
  const size_t jrows = L.nj ? (size_t)PT * d * (r + TV) : 0;
  L.jbuf = o;      o = align256(o + 8 * (size_t)L.nblk_max * jrows);
  L.bcnt = o;      o = align256(o + (L.nj ? 4 * (size_t)L.nblk_max : 0));
  L.total = o;
  return L;
}

// Finite-element stencil of the samples (CROM_PDE_COROTATED_FE: on = 1).
struct FeArgs {
  int on;
  const int64_t* ring_offsets;  // [n_inst + 1] CSR over the ring vertices
  const float* ring_X;          // [n_ring][3] rest positions
  const int64_t* inc_offsets;   // [total + 1] CSR of each sample's tetrahedra
  const int32_t* inc_tets;      // [n_inc][4] instance-local ring indices
  const int8_t* inc_corner;     // [n_inc] the sample's own vertex, 0..3
  float* ring_u;                // [n_ring][3] decoded displacement at q_n
  int64_t n_ring, max_ring, n_inc;
};

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
  const double* given;   // CROM_PDE_PROJECT: the targets at the samples (else NULL)
  double dt;
  const double* q_prev;  // elastic: latent of the previous step (NULL: at rest)
  const double* q_n;
  const double* q_init;  // NULL or a second candidate start per instance
  double* q_next;
  crom_step_info* info;
  char* ws;
  WsLayout L;
  int max_iter, linearized, ls_max;
  double tol, armijo_c, shrink;
  uint64_t* trace;  // optional phase timestamps (see crom_debug_step_trace)
  FeArgs fe;
};

template <class T>
__device__ __forceinline__ T* wsp(const StepArgs& a, size_t off) {
  return reinterpret_cast<T*>(a.ws + off);
}

// Device-coherent accesses (see the synchronisation note above).
template <class T>
__device__ __forceinline__ T ld_c(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_c(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every thread: wait until this thread's memory operations have completed.
// The empty asm statements with a memory clobber are compiler barriers: no
// load or store (atomic or not) is moved across the wait, so every
// coherent store issued before it is acknowledged before the arrival count
// that follows it, and no load of a later phase is hoisted above it.
__device__ __forceinline__ void wait_mem() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0);
  asm volatile("" ::: "memory");
}

// Phase timestamps of workgroups 0 and G-1 (wall clock, 100 MHz ticks),
// compiled only into probe builds (CROM_STEP_TRACE) and written only when a
// trace buffer was registered there.
#ifdef CROM_STEP_TRACE
__device__ __forceinline__ void trace_mark(const StepArgs& a, int slot) {
  if (a.trace && threadIdx.x == 0 && slot < 64) {
    if (blockIdx.x == 0) a.trace[slot] = wall_clock64();
    if (blockIdx.x == gridDim.x - 1) a.trace[64 + slot] = wall_clock64();
  }
}
// marks of the solve, from whichever workgroup runs it
__device__ __forceinline__ void trace_solve(const StepArgs& a, int slot) {
  if (a.trace && threadIdx.x == 0 && slot < 64) a.trace[slot] = wall_clock64();
}
#else
__device__ __forceinline__ void trace_mark(const StepArgs&, int) {}
__device__ __forceinline__ void trace_solve(const StepArgs&, int) {}
#endif

// ---------------------------------------------------------------------------
// Block map and state initialisation (one workgroup of 1024 threads).
// Offsets that are not a valid CSR array (a negative size, a range outside
// [0, total]) give every instance zero batches; an instance without batches
// ends at once as SINGULAR with q_{n+1} = q_n.  Valid CSR ranges are
// disjoint, so the batch count stays within the bound the workspace was
// sized for.  Up to SETUP_LDS instances the prefix and the offsets are kept
// in LDS for the block fill; beyond that they are read back from memory.
// ---------------------------------------------------------------------------
constexpr int SETUP_THREADS = 1024;
constexpr int SETUP_LDS = 2048;

__global__ __launch_bounds__(SETUP_THREADS) void setup_kernel(StepArgs a) {
  int32_t* first_blk = wsp<int32_t>(a, a.L.first_blk);
  int64_t* blk_start = wsp<int64_t>(a, a.L.blk_start);
  int32_t* blk_inst = wsp<int32_t>(a, a.L.blk_inst);
  int64_t* act_phase = wsp<int64_t>(a, a.L.act_phase);
  uint32_t* inst_cnt = wsp<uint32_t>(a, a.L.inst_cnt);
  uint64_t* sync = wsp<uint64_t>(a, a.L.sync);
  GNState* st = wsp<GNState>(a, a.L.state);
  __shared__ int32_t scan[SETUP_THREADS];
  __shared__ int32_t fb[SETUP_LDS + 1];
  __shared__ int64_t lo_off[SETUP_LDS];
  __shared__ int32_t carry;
  __shared__ int32_t n_active;
  const int tid = threadIdx.x;
  const bool in_lds = a.n_inst <= SETUP_LDS;
  int bad = 0;
  for (int i = tid; i < a.n_inst; i += SETUP_THREADS) {
    const int64_t lo = a.offsets[i], hi = a.offsets[i + 1];
    bad |= !(lo >= 0 && hi >= lo && hi <= a.total);
    if (in_lds) lo_off[i] = lo;
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) {
    carry = 0;
    n_active = 0;
  }
  __syncthreads();
  for (int c = 0; c < a.n_inst; c += SETUP_THREADS) {
    const int i = c + tid;
    int32_t nb = 0;
    if (i < a.n_inst && !bad) nb = (int32_t)((a.offsets[i + 1] - a.offsets[i] + PT - 1) / PT);
    scan[tid] = nb;
    __syncthreads();
    for (int d = 1; d < SETUP_THREADS; d <<= 1) {  // inclusive Hillis-Steele scan
      const int32_t v = tid >= d ? scan[tid - d] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    if (i < a.n_inst) {
      const int32_t f = carry + scan[tid] - nb;
      first_blk[i] = f;
      if (in_lds) fb[i] = f;
      if (nb > 0) atomicAdd(&n_active, 1);
    }
    __syncthreads();
    if (tid == SETUP_THREADS - 1) carry += scan[SETUP_THREADS - 1];
    __syncthreads();
  }
  const int32_t nblk = carry;
  if (tid == 0) {
    first_blk[a.n_inst] = nblk;
    if (in_lds) fb[a.n_inst] = nblk;
    *wsp<int64_t>(a, a.L.nblk) = nblk;
    sync[SYNC_SOLVED] = 0;
    sync[SYNC_ABORT] = 0;
    sync[SYNC_EXITED] = 0;
    act_phase[0] = n_active;
  }
  for (int p = tid + 1; p < MAXP + 2; p += SETUP_THREADS) act_phase[p] = 0;
  for (int i = tid; i < a.n_inst; i += SETUP_THREADS) {
    inst_cnt[i] = 0;
    wsp<uint32_t>(a, a.L.inv)[i] = 0;
  }
  __syncthreads();
  // instance i owns batches fb[i] .. fb[i+1]-1: one wave per instance at a
  // time, its lanes over the instance's batches (stores only, no search)
  const int32_t* fbp = in_lds ? fb : first_blk;
  const int lane = tid & 63;
  for (int i = tid >> 6; i < a.n_inst; i += SETUP_THREADS / 64) {
    const int32_t f = fbp[i], nb = fbp[i + 1] - f;
    const int64_t base = in_lds ? lo_off[i] : a.offsets[i];
    for (int32_t k = lane; k < nb; k += 64) {
      blk_start[f + k] = base + (int64_t)k * PT;
      blk_inst[f + k] = i;
      if (a.L.nj) wsp<uint32_t>(a, a.L.bcnt)[f + k] = 0;
    }
  }
  // state: the phase and flags words of every instance (the first solve
  // forms the rest)
  for (int i = tid; i < a.n_inst; i += SETUP_THREADS) {
    const bool empty = fbp[i + 1] == fbp[i];
    uint64_t* words = reinterpret_cast<uint64_t*>(st + i);
    words[GN_W_PHASE] = gn_initial_word(GN_W_PHASE, nullptr, a.r, empty);
    words[GN_W_FLAGS] = gn_initial_word(GN_W_FLAGS, nullptr, a.r, empty);
  }
  for (int i = tid; i < a.n_inst; i += SETUP_THREADS) {
    if (fbp[i + 1] != fbp[i]) continue;
    for (int k = 0; k < a.r; ++k) a.q_next[(int64_t)i * a.r + k] = a.q_n[(int64_t)i * a.r + k];
    crom_step_info inf;
    inf.flags = CROM_FLAG_SINGULAR;
    inf.iters = inf.ls_evals = inf.rounds = 0;
    inf.obj_first = inf.obj_last = __builtin_nan("");
    a.info[i] = inf;
  }
}

// Partial sums of one batch from J rows and residuals staged in LDS (jd
// [ROWS][R], rho [ROWS][TV], both FP64, one row per sample and output value;
// invalid rows hold zeros), stored device-coherently for the solving
// workgroup.
template <int R, int ROWS = PT>
__device__ __forceinline__ void batch_partials(const double* jd, const double* rho, double* out) {
  constexpr int NA = R * (R + 1) / 2;
  constexpr int NRED = NA + R + TV;
  for (int e = threadIdx.x; e < NRED; e += blockDim.x) {
    double s = 0.0;
    if (e < NA) {
      int a = 0, rem = e, n = R;
      while (rem >= n) { rem -= n; ++a; --n; }
      const int b = a + rem;
      for (int i = 0; i < ROWS; ++i) s += jd[i * R + a] * jd[i * R + b];
    } else if (e < NA + R) {
      const int k = e - NA;
      for (int i = 0; i < ROWS; ++i) s += jd[i * R + k] * rho[i * TV];
    } else {
      const int t = e - NA - R;
      for (int i = 0; i < ROWS; ++i) s += 0.5 * rho[i * TV + t] * rho[i * TV + t];
    }
    st_c(out + e, s);
  }
}

// ---------------------------------------------------------------------------
// Evaluation of one 16-sample batch (all threads of the workgroup).  `qdl`:
// LDS scratch for the trial latents.
// ---------------------------------------------------------------------------
// REV: the latent Jacobian by the reverse pass (RevJets, depth bounded),
// else by forward tangent columns.
// CANON (with REV): sums independent of the wave count (the Gauss-Newton
// kernels, whose round and persistent forms differ in waves); the
// linearised kernel, alone in its form, sums per wave.
template <class S, int NW, int PREC, int PF, bool REV = false, bool CANON = true>
__device__ void eval_jets_batch(const StepArgs& a, char* lds, const float* par, int64_t blk) {
  constexpr int R = S::R;
  using C = Cols<S::M, R, 1, 0, true, D2_LAP, R>;
  using E = Engine<S, C, 1, NW, PREC, PF, CANON>;
  using RJ = RevLap<S, NW, PREC, PF, CANON>;
  const int inst = wsp<int32_t>(a, a.L.blk_inst)[blk];
  const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
  const int64_t rem = a.offsets[inst + 1] - first;
  const int n_valid = rem < PT ? (int)rem : PT;
  if constexpr (REV) {
    RJ::stage(lds, a.y, first, n_valid, a.q_n + (int64_t)inst * R, nullptr, par);
    __syncthreads();
    RJ::run(lds, par, a.packed, a.depth);
  } else {
    E::stage(lds, a.y, first, n_valid, a.q_n + (int64_t)inst * R, R, nullptr, 0, par);
    __syncthreads();
    E::run(lds, par, a.packed, a.depth, 0);
  }
  const float* res = reinterpret_cast<const float*>(lds + (REV ? RJ::RES_OFF : E::RES_OFF));
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
    // heat: rho_0 = dt nu Lap g, formed directly; given targets: f - g
    const double r0 = clamped ? -gv : (a.given ? (valid ? a.given[p] : 0.0) - gv : a.dt * a.coef[inst] * lap);
    if (valid) {
      targets[p] = clamped ? 0.0 : (a.given ? a.given[p] : gv + r0);
      rho0[p] = r0;  // read back by this same workgroup in later phases
    }
    rho[i * TV] = valid ? r0 : 0.0;
    for (int t = 1; t < TV; ++t) rho[i * TV + t] = 0.0;
    for (int k = 0; k < R; ++k) jd[i * R + k] = valid ? (double)res[(C::Q0 + k) * PT + i] : 0.0;
  }
  __syncthreads();
  batch_partials<R>(jd, rho, wsp<double>(a, a.L.partials) + blk * a.L.nred);
  __syncthreads();
}

// WITH_J: also the latent Jacobian at the first trial (else its partials
// JᵀJ and Jᵀρ come out zero and only the trial objectives count).  REV: that
// Jacobian by the reverse pass (RevTrial, depth bounded).
template <class S, int NW, int PREC, int PF, bool WITH_J = true, bool REV = false>
__device__ void eval_trials_batch(const StepArgs& a, char* lds, const float* par, double* qdl,
                                  int64_t blk, int inst, int mb, bool have_qdl) {
  constexpr int R = S::R;
  using C = Cols<S::M, R, 1, TV, false, D2_NONE, WITH_J ? R : 0>;
  using E = Engine<S, C, 1, NW, PREC, PF, true>;
  using RT = RevTrial<S, NW, PREC, PF>;
  constexpr bool RV = REV && WITH_J;
  static_assert(RT::CO::F0 == C::F0 && (!WITH_J || RT::CO::Q0 == C::Q0), "same output columns");
  const GNState* st = wsp<GNState>(a, a.L.state) + inst;
  if (mb >= 0) trace_mark(a, mb);
  if (!have_qdl) {
    for (int i = threadIdx.x; i < TV * R; i += blockDim.x) qdl[i] = ld_c(&st->qd[i / R][i % R]);
    __syncthreads();
  }
  if (mb >= 0) trace_mark(a, mb + 1);
  const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
  const int64_t rem = a.offsets[inst + 1] - first;
  const int n_valid = rem < PT ? (int)rem : PT;
  if constexpr (RV) {
    RT::stage(lds, a.y, first, n_valid, a.q_n + (int64_t)inst * R, qdl, par);
    __syncthreads();
    if (mb >= 0) trace_mark(a, mb + 2);
    RT::run(lds, par, a.packed, a.depth);
  } else {
    E::stage(lds, a.y, first, n_valid, a.q_n + (int64_t)inst * R, R, qdl, R, par);
    __syncthreads();
    if (mb >= 0) trace_mark(a, mb + 2);
    E::run(lds, par, a.packed, a.depth, 0);
  }
  if (mb >= 0) trace_mark(a, mb + 3);
  const float* res = reinterpret_cast<const float*>(lds + (RV ? RT::RES_OFF : E::RES_OFF));
  double* jd = reinterpret_cast<double*>(lds);
  double* rho = jd + PT * R;
  const double* rho0 = wsp<double>(a, a.L.rho0);
  if (threadIdx.x < PT) {
    const int i = threadIdx.x;
    const bool valid = i < n_valid;
    const double r0 = valid ? rho0[first + i] : 0.0;
    for (int t = 0; t < TV; ++t) rho[i * TV + t] = valid ? r0 - (double)res[(C::F0 + t) * PT + i] : 0.0;
    for (int k = 0; k < R; ++k) jd[i * R + k] = (WITH_J && valid) ? (double)res[(C::Q0 + k) * PT + i] : 0.0;
  }
  __syncthreads();
  batch_partials<R>(jd, rho, wsp<double>(a, a.L.partials) + blk * a.L.nred);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Neo-Hookean elastodynamics (d = 3, m = 3).
// ---------------------------------------------------------------------------
enum { PK_HEAT = 0, PK_ELASTIC = 1 };

// Latent-tangent chunk of the elastic passes.  Two tangents per pass in
// every precision: each chunk of a batch is a work item of the step kernel,
// so the single bar's 32 batches give 256 work items, one per compute unit
// (with four tangents, 128: BF16 Gauss-Newton step 0.97 -> 0.93 ms, same
// bits).  In bfloat16 eight would fit the LDS, but the trial evaluation then
// spilled 864 bytes per lane and measured slower (2.29 vs 2.08 ms, when a
// batch was one work item).
#ifndef CROM_ELASTIC_QC
#define CROM_ELASTIC_QC 2
#endif
template <int PREC>
struct ElasticChunks {
  static constexpr int QC = CROM_ELASTIC_QC;
  static constexpr int HC = 2;
  // Every trial round carries the Jacobian in BF16 mode: there a chunk's
  // pass with its tangents takes about the wall time of the value pass
  // alone (the chunks run side by side, each latency-bound), so an accepted
  // trial needs no re-linearisation round.  In the other modes a
  // backtracking round evaluates the objective only.  Measured per
  // Gauss-Newton step (single instance, 500 samples) with the Jacobian in
  // every round against only at first trials: neo-Hookean bar BF16 0.682
  // against 0.851 ms, BF16_PURE 0.644 against 0.612 ms, FP32 1.545 against
  // 1.751 ms; corotated FE bar (several backtracks per iteration) BF16 0.486
  // against 0.533 ms, FP32 1.617 against 1.272 ms.
  static constexpr bool EAGER_J = PREC == PREC_BF16;
};

// One engine pass at q_n over one batch, writing the pass's columns of
// every valid sample into the jets buffer.
template <class S, class C, int NW, int PREC>
__device__ void jets_pass_batch(const StepArgs& a, char* lds, const float* par, int64_t blk, int qb) {
  using E = Engine<S, C, 1, NW, PREC, 0>;
  constexpr int D = S::D, CC = C::C, NT = E::NT;
  const JetsLayout J{D, S::M, S::R, S::M * (S::M + 1) / 2};
  const int inst = wsp<int32_t>(a, a.L.blk_inst)[blk];
  const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
  const int64_t rem = a.offsets[inst + 1] - first;
  const int n_valid = rem < PT ? (int)rem : PT;
  E::stage(lds, a.y, first, n_valid, a.q_n + (int64_t)inst * S::R, S::R, nullptr, 0, par);
  __syncthreads();
  E::run(lds, par, a.packed, a.depth, qb);
  const float* res = reinterpret_cast<const float*>(lds + E::RES_OFF);
  float* jets = wsp<float>(a, a.L.jets);
  for (int e = threadIdx.x; e < n_valid * D * CC; e += blockDim.x) {
    const int i = e / (D * CC), oo = (e / CC) % D, c = e % CC;
    const float v = res[(oo * NT + c) * PT + i];
    float* row = jets + (first + i) * a.L.nj;
    const int k = C::kind(c);
    if (k == CK_VAL || k == CK_XT) {  // every chunk with these columns computes them alike
      if (blockIdx.y == 0) row[k == CK_VAL ? J.val(oo) : J.grad(oo, c - C::X0)] = v;
    }
    else if (k == CK_HESS) row[J.hess(oo, C::HB + (c - C::D0))] = v;
    else if (k == CK_QT) row[J.jac(oo, qb + (c - C::Q0))] = v;
  }
  __syncthreads();
}

template <class S, class C, int NW, int PREC>
__global__ __launch_bounds__(NW * 64) void jets_pass_kernel(StepArgs a, int qb) {
  using E = Engine<S, C, 1, NW, PREC, 0>;
  extern __shared__ __align__(16) char lds[];
  const int64_t nblk = *wsp<int64_t>(a, a.L.nblk);
  if ((int64_t)blockIdx.x >= nblk) return;
  float* par = reinterpret_cast<float*>(lds + E::LDS_BYTES);
  E::PC::load(par, a.params, a.pi, a.depth, NW * 64);
  __syncthreads();
  // blockIdx.y picks the chunk of latent directions (one launch for all)
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x)
    jets_pass_batch<S, C, NW, PREC>(a, lds, par, blk, qb + (int)blockIdx.y * C::NQ);
}

// The elastic preparation's engine passes at q_n in one launch: blockIdx.y
// below NHC picks a chunk of HC Hessian entries (with the value and the x
// tangents those entries need), from NHC on a chunk of QC latent
// directions.  The chunks of a batch run side by side instead of in one
// launch per Hessian chunk and one for the latent chunks.  Two Hessian
// entries and four latent directions per chunk keep a 500-sample instance's
// work items (32 batches x 7 chunks) within one per compute unit.  Single
// instance, 500 samples, BF16: the preparation took 142 us in three
// launches (three Hessian entries per chunk, two latent directions), 70 us
// fused; with these chunks the Gauss-Newton step takes 0.590 ms against
// 0.613 ms, the linearised one 0.088 ms against 0.110 ms.
template <class S, int PREC>
struct ElasticJets {
  static constexpr int NH = S::M * (S::M + 1) / 2, HC = ElasticChunks<PREC>::HC, QC = 4;
  static constexpr int NHC = (NH + HC - 1) / HC, NQC = S::R / QC;
  static_assert(S::R % QC == 0, "whole latent chunks");
  template <int HB>
  using CH = Cols<S::M, S::R, 1, 0, true, D2_HESS, 0, HB, (NH - HB < HC ? NH - HB : HC)>;
  using CQ = Cols<S::M, S::R, 1, 0, false, D2_NONE, QC>;
  template <int NW, int HB = 0>
  static constexpr int hess_lds() {
    if constexpr (HB < NH) {
      constexpr int b = Engine<S, CH<HB>, 1, NW, PREC, 0>::LDS_BYTES, rest = hess_lds<NW, HB + HC>();
      return b > rest ? b : rest;
    } else {
      return 0;
    }
  }
  template <int NW>
  static constexpr int lds() {
    constexpr int h = hess_lds<NW>(), q = Engine<S, CQ, 1, NW, PREC, 0>::LDS_BYTES;
    return h > q ? h : q;
  }
  template <int NW, int HB = 0>
  static __device__ void hess_batch(const StepArgs& a, char* lds, const float* par, int64_t blk, int y) {
    if constexpr (HB < NH) {
      if (y == HB / HC) jets_pass_batch<S, CH<HB>, NW, PREC>(a, lds, par, blk, 0);
      else hess_batch<NW, HB + HC>(a, lds, par, blk, y);
    }
  }
};

template <class S, int NW, int PREC>
__global__ __launch_bounds__(NW * 64) void elastic_jets_kernel(StepArgs a) {
  using EJ = ElasticJets<S, PREC>;
  using PC = ParamCache<S>;
  extern __shared__ __align__(16) char lds[];
  const int64_t nblk = *wsp<int64_t>(a, a.L.nblk);
  if ((int64_t)blockIdx.x >= nblk) return;
  float* par = reinterpret_cast<float*>(lds + EJ::template lds<NW>());
  PC::load(par, a.params, a.pi, a.depth, NW * 64);
  __syncthreads();
  const int y = blockIdx.y;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    if (y < EJ::NHC) EJ::template hess_batch<NW>(a, lds, par, blk, y);
    else jets_pass_batch<S, typename EJ::CQ, NW, PREC>(a, lds, par, blk, (y - EJ::NHC) * EJ::QC);
  }
}

// FP64 update at one sample: rho_0 = u_{n+1} - u(q_n) and the target.
//   F = I + du/dX, P = mu (F - F^-T) + lam ln J F^-T,
//   (div P)_i = sum_{j,k,l} dP_ij/dF_kl d2u_k/dX_l dX_j with
//   dP_ij/dF_kl = mu d_ik d_jl + (mu - lam ln J) Fi_jk Fi_li + lam Fi_lk Fi_ji,
//   v_n = (du/dq)(q_n - q_prev)/dt, v+ = v_n + dt (div P / rho0 + B),
//   rho_0 = dt v+ (or -u on a clamped sample).
// coef per instance: lam, mu, rho0, Bx, By, Bz.
template <int R>
__global__ __launch_bounds__(64) void elastic_targets_kernel(StepArgs a) {
  const int64_t nblk = *wsp<int64_t>(a, a.L.nblk);
  const JetsLayout JL{3, 3, R, 6};
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int i = threadIdx.x;
    const int inst = wsp<int32_t>(a, a.L.blk_inst)[blk];
    const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
    const int64_t rem = a.offsets[inst + 1] - first;
    if (i >= PT || i >= rem) continue;
    const int64_t p = first + i;
    const float* row = wsp<float>(a, a.L.jets) + p * a.L.nj;
    const double* cf = a.coef + (int64_t)inst * 6;
    const double lam = cf[0], mu = cf[1], rho = cf[2];
    double u[3], F[3][3], H[3][3][3];
    for (int k = 0; k < 3; ++k) {
      u[k] = row[JL.val(k)];
      for (int l = 0; l < 3; ++l) F[k][l] = (k == l ? 1.0 : 0.0) + (double)row[JL.grad(k, l)];
      for (int l = 0, h = 0; l < 3; ++l)
        for (int j = l; j < 3; ++j, ++h) H[k][l][j] = H[k][j][l] = row[JL.hess(k, h)];
    }
    // inverse by cofactors
    const double c00 = F[1][1] * F[2][2] - F[1][2] * F[2][1];
    const double c01 = F[1][2] * F[2][0] - F[1][0] * F[2][2];
    const double c02 = F[1][0] * F[2][1] - F[1][1] * F[2][0];
    const double det = F[0][0] * c00 + F[0][1] * c01 + F[0][2] * c02;
    double Fi[3][3];
    Fi[0][0] = c00 / det;
    Fi[1][0] = c01 / det;
    Fi[2][0] = c02 / det;
    Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) / det;
    Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) / det;
    Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) / det;
    Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) / det;
    Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) / det;
    Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) / det;
    const double lnJ = log(det);  // NaN for det <= 0: reported as NONFINITE by the solve
    double qdot[R];
    for (int r = 0; r < R; ++r)
      qdot[r] = a.q_prev ? (a.q_n[(int64_t)inst * R + r] - a.q_prev[(int64_t)inst * R + r]) / a.dt : 0.0;
    const bool clamped = a.clamp && a.clamp[p];
    // an inverted free sample has no neo-Hookean stress: INVERTED (its NaN
    // targets also make the solve report NONFINITE)
    if (det <= 0.0 && !clamped) st_c(wsp<uint32_t>(a, a.L.inv) + inst, 1u);
    double* rho0 = wsp<double>(a, a.L.rho0) + p * 3;
    double* tg = wsp<double>(a, a.L.targets) + p * 3;
    for (int ii = 0; ii < 3; ++ii) {
      double div = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) {
            const double A = (ii == k && j == l ? mu : 0.0) + (mu - lam * lnJ) * Fi[j][k] * Fi[l][ii] +
                             lam * Fi[l][k] * Fi[j][ii];
            div += A * H[k][l][j];
          }
      double v = 0.0;
      for (int r = 0; r < R; ++r) v += (double)row[JL.jac(ii, r)] * qdot[r];
      const double vn = v + a.dt * (div / rho + cf[3 + ii]);
      const double inc = clamped ? -u[ii] : a.dt * vn;
      rho0[ii] = inc;
      tg[ii] = clamped ? 0.0 : u[ii] + inc;
    }
  }
}

// ---------------------------------------------------------------------------
// Corotated elasticity with finite-element forces (appendix, Sec. "Solid
// Mechanics": linear tetrahedra, the deformation gradient from the linear
// basis, forces accumulated from the tetrahedra incident on each sample).
// ---------------------------------------------------------------------------

// Displacement u = g(X, q_n) at the ring vertices of every instance (value
// column only): blockIdx.y is the instance, the x-blocks stride over its
// passes of NB 16-vertex batches.  An instance whose ring range is not a
// valid CSR range of [0, n_ring] is skipped; its targets then come out NaN.
// Launch shape: in bfloat16 the full-field decode's (64 vertices and eight
// waves per workgroup: the weights are read once per 64 vertices; 5,748
// vertices 45 -> 33 us); in FP32 16 vertices and four waves (the wider
// shape left most CUs idle at this size: 60 -> 89 us).
template <class S, int PREC>
struct RingTune {
  static constexpr int NB = PREC == PREC_FP32 ? 1 : 4;
  static constexpr int NW = PREC == PREC_FP32 ? 4 : DecodeTune<S, PREC>::NW;
  static constexpr int PF = PREC == PREC_FP32 ? 0 : DecodeTune<S, PREC>::PF;
};
template <class S, int PREC>
using RingEngine = Engine<S, Cols<S::M, S::R, 1, 0, false, D2_NONE, 0>, RingTune<S, PREC>::NB,
                          RingTune<S, PREC>::NW, PREC, RingTune<S, PREC>::PF>;

template <class S, int PREC>
__global__ __launch_bounds__((RingTune<S, PREC>::NW * 64)) void ring_decode_kernel(StepArgs a) {
  using E = RingEngine<S, PREC>;
  extern __shared__ __align__(16) char lds[];
  const int inst = blockIdx.y;
  const int64_t lo = a.fe.ring_offsets[inst], hi = a.fe.ring_offsets[inst + 1];
  if (!(lo >= 0 && hi >= lo && hi <= a.fe.n_ring)) return;
  const int64_t nb = (hi - lo + E::NPTS - 1) / E::NPTS;
  if ((int64_t)blockIdx.x >= nb) return;
  float* par = reinterpret_cast<float*>(lds + E::LDS_BYTES);
  E::PC::load(par, a.params, a.pi, a.depth, E::THREADS);
  __syncthreads();
  const double* q = a.q_n + (int64_t)inst * S::R;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int64_t first = lo + b * E::NPTS;
    const int n_valid = hi - first < E::NPTS ? (int)(hi - first) : E::NPTS;
    E::stage(lds, a.fe.ring_X, first, n_valid, q, S::R, nullptr, 0, par);
    __syncthreads();
    E::run(lds, par, a.packed, a.depth, 0);
    const float* res = reinterpret_cast<const float*>(lds + E::RES_OFF);
    // res[(oo * NT + t) * PT + j]: t the 16-vertex batch (one column each)
    for (int e = threadIdx.x; e < S::D * E::NT * PT; e += E::THREADS) {
      const int oo = e / (E::NT * PT), t = (e / PT) % E::NT, j = e % PT;
      const int lp = t * PT + j;
      if (lp < n_valid) a.fe.ring_u[(first + lp) * S::D + oo] = res[e];
    }
    __syncthreads();
  }
}

// Cofactor matrix c of a 3 x 3 matrix x (x^-T = c / det x); returns det x.
__device__ __forceinline__ double cofactors3(const double x[3][3], double c[3][3]) {
  c[0][0] = x[1][1] * x[2][2] - x[1][2] * x[2][1];
  c[0][1] = x[1][2] * x[2][0] - x[1][0] * x[2][2];
  c[0][2] = x[1][0] * x[2][1] - x[1][1] * x[2][0];
  c[1][0] = x[0][2] * x[2][1] - x[0][1] * x[2][2];
  c[1][1] = x[0][0] * x[2][2] - x[0][2] * x[2][0];
  c[1][2] = x[0][1] * x[2][0] - x[0][0] * x[2][1];
  c[2][0] = x[0][1] * x[1][2] - x[0][2] * x[1][1];
  c[2][1] = x[0][2] * x[1][0] - x[0][0] * x[1][2];
  c[2][2] = x[0][0] * x[1][1] - x[0][1] * x[1][0];
  return x[0][0] * c[0][0] + x[0][1] * c[0][1] + x[0][2] * c[0][2];
}

// Rotation factor R of the polar decomposition F = R S by Newton's iteration
// X <- (g X + X^-T / g) / 2 with the determinant scaling g = (det X)^(-1/3)
// (N. J. Higham, "Computing the polar decomposition - with applications",
// SIAM J. Sci. Stat. Comput. 7, 1986).  The iteration keeps det X > 0 and
// converges quadratically; once successive iterates agree to 1e-9 one more
// unscaled step brings them to rounding level.  det F <= 0 (no proper
// rotation factor) gives NaN.
__device__ void polar_rotation(const double F[3][3], double R[3][3]) {
  double x[3][3], c[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) x[i][j] = F[i][j];
  bool polish = false;
  for (int it = 0; it < 40; ++it) {
    const double det = cofactors3(x, c);
    if (!(det > 0.0)) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = __builtin_nan("");
      return;
    }
    const double g = polish ? 1.0 : 1.0 / cbrt(det);
    const double h = 0.5 / (g * det), hg = 0.5 * g;
    double dmax = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double v = hg * x[i][j] + h * c[i][j];
        dmax = fmax(dmax, fabs(v - x[i][j]));
        x[i][j] = v;
      }
    if (polish) break;
    if (dmax < 1e-9) polish = true;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = x[i][j];
}

// Force of one tetrahedron on one of its vertices and the tetrahedron's
// volume.  X, u: the four vertices' rest positions and displacements.
//   D_m = [X_a - X_3]_{a<3}, G = [u_a - u_3]_{a<3} D_m^-1, F = I + G,
//   P = 2 mu (F - R) + lam (tr(R^T F) - 3) R,  H = -(|det D_m| / 6) P D_m^-T;
// the force on corner c < 3 is column c of H, on corner 3 minus their sum.
__device__ void tet_force(const double X[4][3], const double u[4][3], int corner, double lam, double mu,
                          double f[3], double* vol, bool* inverted) {
  double Dm[3][3], Du[3][3], cm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) {
      Dm[i][a] = X[a][i] - X[3][i];
      Du[i][a] = u[a][i] - u[3][i];
    }
  const double det = cofactors3(Dm, cm);  // D_m^-1 = cm^T / det, D_m^-T = cm / det
  double F[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += Du[i][a] * cm[j][a];
      F[i][j] = (i == j ? 1.0 : 0.0) + s / det;
    }
  double cF[3][3];
  *inverted = cofactors3(F, cF) <= 0.0;
  double R[3][3];
  polar_rotation(F, R);
  double tr = -3.0;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) tr += R[k][i] * F[k][i];
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i][j] = 2.0 * mu * (F[i][j] - R[i][j]) + lam * tr * R[i][j];
  const double v = fabs(det) / 6.0;
  *vol = v;
  // H[i][a] = -v sum_k P[i][k] D_m^-T[k][a] = -(v / det) sum_k P[i][k] cm[k][a]
  for (int i = 0; i < 3; ++i) {
    double hs[3];
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += P[i][k] * cm[k][a];
      hs[a] = -(v / det) * s;
    }
    f[i] = corner < 3 ? hs[corner] : -(hs[0] + hs[1] + hs[2]);
  }
}

// FP64 update at the samples from finite-element forces: one wave per
// sample (a workgroup takes FE_WAVES consecutive samples of a batch), its
// lanes over the sample's incident tetrahedra; the sample's force and
// incident volume are summed across the wave in a fixed order.
//   m = rho0 (incident volume) / 4,  v_n = (du/dq)(q_n - q_prev)/dt,
//   v+ = v_n + dt (f / m + B),  rho_0 = dt v+ (a clamped sample: -u).
// Invalid stencil data (a ring or incidence range that is not a CSR range,
// a ring larger than max_ring, an index outside the instance's ring, a
// corner outside 0..3, a sample without tetrahedra) gives NaN, which the
// solve reports as a non-finite instance.
constexpr int FE_WAVES = 4;
static_assert(PT % FE_WAVES == 0, "whole batches");
template <int R>
__global__ __launch_bounds__(FE_WAVES * 64) void fe_targets_kernel(StepArgs a) {
  const int64_t nblk = *wsp<int64_t>(a, a.L.nblk);
  const JetsLayout JL{3, 3, R, 6};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double qnan = __builtin_nan("");
  constexpr int SUB = PT / FE_WAVES;  // workgroups per batch
  for (int64_t gi = blockIdx.x; gi < nblk * SUB; gi += gridDim.x) {
    const int64_t blk = gi / SUB;
    const int i = (int)(gi % SUB) * FE_WAVES + wave;
    const int inst = wsp<int32_t>(a, a.L.blk_inst)[blk];
    const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
    const int64_t rem = a.offsets[inst + 1] - first;
    const int n_valid = rem < PT ? (int)rem : PT;
    const int64_t rlo = a.fe.ring_offsets[inst], rhi = a.fe.ring_offsets[inst + 1];
    const bool ring_ok = rlo >= 0 && rhi > rlo && rhi <= a.fe.n_ring && rhi - rlo <= a.fe.max_ring;
    const double* cf = a.coef + (int64_t)inst * 6;
    const double lam = cf[0], mu = cf[1], rho = cf[2];
    if (i < n_valid) {
      const int64_t p = first + i;
      const int64_t elo = a.fe.inc_offsets[p], ehi = a.fe.inc_offsets[p + 1];
      bool ok = ring_ok && elo >= 0 && ehi > elo && ehi <= a.fe.n_inc;
      double fs[3] = {0.0, 0.0, 0.0}, vs = 0.0;
      int inv = 0;
      if (ok) {
        for (int64_t e = elo + lane; e < ehi; e += 64) {
          const int corner = a.fe.inc_corner[e];
          bool good = corner >= 0 && corner < 4;
          double X[4][3], u[4][3];
          for (int k = 0; k < 4; ++k) {
            const int32_t v = a.fe.inc_tets[e * 4 + k];
            const bool in = v >= 0 && (int64_t)v < rhi - rlo;
            good = good && in;
            const int64_t g = rlo + (in ? v : 0);
            for (int j = 0; j < 3; ++j) {
              X[k][j] = (double)a.fe.ring_X[g * 3 + j];
              u[k][j] = (double)a.fe.ring_u[g * 3 + j];
            }
          }
          double f[3], vol;
          bool tinv;
          tet_force(X, u, good ? corner : 0, lam, mu, f, &vol, &tinv);
          inv |= (good && tinv) ? 1 : 0;
          for (int j = 0; j < 3; ++j) fs[j] += good ? f[j] : qnan;
          vs += vol;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        for (int j = 0; j < 3; ++j) fs[j] += __shfl_xor(fs[j], off);
        vs += __shfl_xor(vs, off);
        inv |= __shfl_xor(inv, off);
      }
      if (lane == 0) {
        const float* row = wsp<float>(a, a.L.jets) + p * a.L.nj;
        const double mass = ok ? rho * vs / 4.0 : qnan;
        const bool clamped = a.clamp && a.clamp[p];
        if (inv && !clamped) st_c(wsp<uint32_t>(a, a.L.inv) + inst, 1u);
        double* rho0 = wsp<double>(a, a.L.rho0) + p * 3;
        double* tg = wsp<double>(a, a.L.targets) + p * 3;
        for (int k = 0; k < 3; ++k) {
          double v = 0.0;
          if (a.q_prev)
            for (int r = 0; r < R; ++r)
              v += (double)row[JL.jac(k, r)] *
                   ((a.q_n[(int64_t)inst * R + r] - a.q_prev[(int64_t)inst * R + r]) / a.dt);
          const double uk = row[JL.val(k)];
          const double vn = v + a.dt * (fs[k] / mass + cf[3 + k]);
          const double inc = clamped ? -uk : a.dt * vn;
          rho0[k] = inc;
          tg[k] = clamped ? 0.0 : uk + inc;
        }
      }
    }
  }
}

// Phase 0 of the elastic step: the partials of the stored Jacobian at q_n
// and of rho_0 (no decoder evaluation).
template <class S>
__device__ void eval_init_elastic(const StepArgs& a, double* jd, int64_t blk) {
  constexpr int R = S::R, D = S::D, ROWS = PT * D;
  const JetsLayout JL{D, S::M, R, S::M * (S::M + 1) / 2};
  double* rho = jd + ROWS * R;
  const int inst = wsp<int32_t>(a, a.L.blk_inst)[blk];
  const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
  const int64_t rem = a.offsets[inst + 1] - first;
  const int n_valid = rem < PT ? (int)rem : PT;
  const float* jets = wsp<float>(a, a.L.jets);
  const double* rho0 = wsp<double>(a, a.L.rho0);
  for (int e = threadIdx.x; e < ROWS * R; e += blockDim.x) {
    const int row = e / R, k = e % R, i = row / D, oo = row % D;
    jd[e] = i < n_valid ? (double)jets[(first + i) * a.L.nj + JL.jac(oo, k)] : 0.0;
  }
  for (int e = threadIdx.x; e < ROWS * TV; e += blockDim.x) {
    const int row = e / TV, t = e % TV, i = row / D;
    rho[e] = (t == 0 && i < n_valid) ? rho0[first * D + row] : 0.0;
  }
  __syncthreads();
  batch_partials<R, ROWS>(jd, rho, wsp<double>(a, a.L.partials) + blk * a.L.nred);
  __syncthreads();
}

// Trial phases of the elastic step, one latent-tangent chunk `ch` of one
// batch per call.  A round with the Jacobian at the first trial gives each
// chunk of QC latent directions its own workgroup (value, the first
// difference and the chunk's tangents, which the engine takes at the first
// difference column's latent).  The chunks store their Jacobian columns,
// chunk 0 also the residuals, and the last chunk to arrive stages the
// whole batch and forms its partials.  A round without the Jacobian
// evaluates on chunk 0 alone: the decoder differences at the TV trial
// latents (one pass), zero Jacobian partials.  Every chunk arrives in every
// round, also where it has nothing to evaluate: a chunk reads the
// instance's phase before its arrival, and the instance is solved only
// after all its arrivals, so no chunk can read the state that the round's
// own solve writes (a chunk that skipped the arrival could, and would then
// evaluate the next round's columns early and be counted twice).  With one
// trial per round the residual comes from chunk 0's difference column (the
// same column arithmetic as the trial pass).  Returns whether this
// workgroup formed the batch's partials.
template <class S, int NW, int PREC, int PF>
__device__ bool eval_trials_elastic(const StepArgs& a, char* lds, double* jd, const float* par, double* qdl,
                                    int64_t blk, int ch, int inst, bool have_qdl, bool with_j) {
  constexpr int R = S::R, D = S::D, ROWS = PT * D;
  constexpr int QC = ElasticChunks<PREC>::QC;
  constexpr int NCH = R / QC;
  using CT = Cols<S::M, R, 1, TV, false, D2_NONE, 0>;
  using ET = Engine<S, CT, 1, NW, PREC, PF>;
  using CQ = Cols<S::M, R, 1, 1, false, D2_NONE, QC>;
  using EQ = Engine<S, CQ, 1, NW, PREC, PF>;
  __shared__ int s_lastc;
  double* rho = jd + ROWS * R;
  double* jg = wsp<double>(a, a.L.jbuf) + blk * (int64_t)(ROWS * (R + TV));  // [ROWS][R], then [ROWS][TV]
  if (with_j || ch == 0) {  // uniform over the workgroup
    const GNState* st = wsp<GNState>(a, a.L.state) + inst;
    if (!have_qdl) {
      for (int i = threadIdx.x; i < TV * R; i += blockDim.x) qdl[i] = ld_c(&st->qd[i / R][i % R]);
      __syncthreads();
    }
    const int64_t first = wsp<int64_t>(a, a.L.blk_start)[blk];
    const int64_t rem = a.offsets[inst + 1] - first;
    const int n_valid = rem < PT ? (int)rem : PT;
    const double* qn = a.q_n + (int64_t)inst * R;
    const double* rho0 = wsp<double>(a, a.L.rho0);
    const bool merged = with_j && TV == 1;
    if (!merged && ch == 0) {
      ET::stage(lds, a.y, first, n_valid, qn, R, qdl, R, par);
      __syncthreads();
      ET::run(lds, par, a.packed, a.depth, 0);
      const float* res = reinterpret_cast<const float*>(lds + ET::RES_OFF);
      for (int e = threadIdx.x; e < ROWS * TV; e += blockDim.x) {
        const int row = e / TV, t = e % TV, i = row / D, oo = row % D;
        rho[e] = i < n_valid ? rho0[first * D + row] - (double)res[(oo * ET::NT + CT::F0 + t) * PT + i] : 0.0;
      }
      __syncthreads();
    }
    const float* res = reinterpret_cast<const float*>(lds + EQ::RES_OFF);
    if (with_j) {
      const int qb = ch * QC;
      EQ::stage(lds, a.y, first, n_valid, qn, R, qdl, R, par);
      __syncthreads();
      EQ::run(lds, par, a.packed, a.depth, qb);
      for (int e = threadIdx.x; e < ROWS * QC; e += blockDim.x) {
        const int row = e / QC, c = e % QC, i = row / D, oo = row % D;
        st_c(jg + row * R + qb + c, i < n_valid ? (double)res[(oo * EQ::NT + CQ::Q0 + c) * PT + i] : 0.0);
      }
    }
    if (ch == 0) {
      for (int e = threadIdx.x; e < ROWS * TV; e += blockDim.x) {
        const int row = e / TV, i = row / D, oo = row % D;
        const double v = !merged ? rho[e]
                       : (i < n_valid ? rho0[first * D + row] - (double)res[(oo * EQ::NT + CQ::F0) * PT + i] : 0.0);
        st_c(jg + ROWS * R + e, v);
      }
    }
  }
  // arrival of this chunk: what it evaluated is complete in memory
  wait_mem();
  __syncthreads();
  uint32_t* bcnt = wsp<uint32_t>(a, a.L.bcnt) + blk;
  if (threadIdx.x == 0) s_lastc = atomicAdd(bcnt, 1u) + 1 == (uint32_t)NCH;
  __syncthreads();
  const bool last = s_lastc != 0;
  __syncthreads();
  if (!last) return false;
  // every chunk has arrived: stage the batch (zero Jacobian in a round
  // without it) and clear its count for the next round (whose chunks start
  // only after this instance is solved)
  for (int e = threadIdx.x; e < ROWS * (R + TV); e += blockDim.x)
    jd[e] = with_j || e >= ROWS * R ? ld_c(jg + e) : 0.0;
  if (threadIdx.x == 0) st_c(bcnt, 0u);
  __syncthreads();
  batch_partials<R, ROWS>(jd, rho, wsp<double>(a, a.L.partials) + blk * a.L.nred);
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// Small dense algebra on one wave (64 lanes), FP64.
//
// Cholesky factorisation A = L L^T of the packed upper triangle `up` (LDS,
// row-major over i <= k), left-looking: column j's pivot and entries
// subtract the earlier columns' products in increasing column order; then
// the solves L y = b and L^T x = y.  A pivot (the value under the square
// root) that is not finite or not above thresh = 1e-14 * max diag(A) fails
// the factorisation (ok = 0).  Both variants below take the same operations
// in the same order, so they agree bit for bit where both apply.
//
// For r <= 8 every lane factors the whole matrix in registers from LDS
// reads at uniform addresses (no cross-lane traffic).  Not inlined: its 36
// register-held entries then do not add to the registers live at the call.
// Every lane holds the whole solution, so it also returns |x|^2 and b.x
// (the same in every lane), which the caller would otherwise sum across
// lanes.
struct CholOut {
  double x, xx, bx;
  int ok;
};
// sqrt(d) and 1/sqrt(d) for d > 0: the hardware reciprocal square root
// estimate refined by two Newton steps, y <- y (3/2 - d/2 y^2), each of
// which doubles the correct bits (full double precision after two), and
// one Newton step on the square root, s <- s + y/2 (d - s^2).  Both within
// an ulp of the correctly rounded values, in a dependent chain of 9
// operations instead of the IEEE square root and division sequences.
__device__ __forceinline__ void sqrt_rsqrt(double d, double& s, double& y) {
  y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  double t = fma(-h * y, y, 0.5);
  y = fma(y, t, y);
  t = fma(-h * y, y, 0.5);
  y = fma(y, t, y);
  s = d * y;
  s = fma(0.5 * y, fma(-s, s, d), s);
}

template <int R>
__device__ __attribute__((noinline)) CholOut lane_chol_solve(const double* up, const double* b) {
  const int lane = threadIdx.x & 63;
  double L[R][R];
  double dmax = -1.0;
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int k = i; k < R; ++k) {
      const double v = up[i * R - i * (i - 1) / 2 + (k - i)];
      L[k][i] = v;
      if (i == k) dmax = fmax(dmax, v);
    }
  const double thresh = 1e-14 * dmax;
  double inv[R];  // 1 / L_jj: one division per column, reused by both substitutions
#pragma unroll
  for (int j = 0; j < R; ++j) {
    double d = L[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(isfinite(d) && d > thresh)) return CholOut{0.0, 0.0, 0.0, 0};  // uniform across the wave
    double ljj;
    sqrt_rsqrt(d, ljj, inv[j]);
    L[j][j] = ljj;
#pragma unroll
    for (int i = j + 1; i < R; ++i) {
      double v = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v * inv[j];
    }
  }
  double y[R];
#pragma unroll
  for (int i = 0; i < R; ++i) y[i] = b[i];
#pragma unroll
  for (int j = 0; j < R; ++j) {  // L y = b
    y[j] = y[j] * inv[j];
#pragma unroll
    for (int i = j + 1; i < R; ++i) y[i] -= L[i][j] * y[j];
  }
#pragma unroll
  for (int j = R - 1; j >= 0; --j) {  // L^T x = y
    y[j] = y[j] * inv[j];
#pragma unroll
    for (int i = 0; i < j; ++i) y[i] -= L[j][i] * y[j];
  }
  double x = 0.0, xx = 0.0, bx = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    x = lane == k ? y[k] : x;
    xx += y[k] * y[k];
    bx += b[k] * y[k];
  }
  return CholOut{x, xx, bx, 1};
}

// Lane l's value of v, in every lane (two scalar lane reads).
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// For 8 < r <= 64 lane i holds row i of A, then of L (r registers); the
// entries of row j that every lane subtracts are read from lane j, also in
// the backward substitution, where lane i takes L_ji from row j.  The
// scalars (pivots, 1 / L_jj, the solution) are the same in every lane, as
// in the variant above.
template <int R>
__device__ __forceinline__ CholOut row_chol_solve(const double* up, const double* b) {
  static_assert(R <= 64, "one lane per row");
  const int lane = threadIdx.x & 63;
  const int i = lane < R ? lane : R - 1;  // lanes past the matrix mirror its last row
  double l[R];                            // row i: A_ik, then L_ik for k <= i (0 above the diagonal)
  double dmax = -1.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int r0 = i < k ? i : k, r1 = i < k ? k : i;
    l[k] = up[r0 * R - r0 * (r0 - 1) / 2 + (r1 - r0)];
    dmax = fmax(dmax, up[k * R - k * (k - 1) / 2]);
  }
  const double thresh = 1e-14 * dmax;
  double acc = b[i];
  double inv[R];  // 1 / L_jj
#pragma unroll
  for (int j = 0; j < R; ++j) {
    double v = l[j];
#pragma unroll
    for (int k = 0; k < j; ++k) v -= l[k] * lane_value(l[k], j);
    const double d = lane_value(v, j);  // lane j's v: the pivot
    if (!(isfinite(d) && d > thresh)) return CholOut{0.0, 0.0, 0.0, 0};  // uniform across the wave
    double ljj;
    sqrt_rsqrt(d, ljj, inv[j]);
    l[j] = i == j ? ljj : (i > j ? v * inv[j] : 0.0);
  }
  double y[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {  // L y = b
    y[j] = lane_value(acc, j) * inv[j];
    if (i > j) acc -= l[j] * y[j];
  }
  acc = y[0];
#pragma unroll
  for (int k = 1; k < R; ++k) acc = i == k ? y[k] : acc;
#pragma unroll
  for (int j = R - 1; j >= 0; --j) {  // L^T x = y
    y[j] = lane_value(acc, j) * inv[j];
    double lji = 0.0;  // L_ji, from lane j's row
#pragma unroll
    for (int k = 0; k < j; ++k) {
      const double t = lane_value(l[k], j);
      lji = i == k ? t : lji;
    }
    if (i < j) acc -= lji * y[j];
  }
  double x = 0.0, xx = 0.0, bx = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    x = lane == k ? y[k] : x;
    xx += y[k] * y[k];
    bx += b[k] * y[k];
  }
  return CholOut{x, xx, bx, 1};
}

template <int R>
__device__ __forceinline__ CholOut chol_solve(const double* up, const double* b) {
  if constexpr (R <= 8) return lane_chol_solve<R>(up, b);
  else return row_chol_solve<R>(up, b);
}

// ---------------------------------------------------------------------------
// Gauss-Newton control of one instance in phase p, by the workgroup that
// completed the instance's last batch of the phase.  The workgroup copies
// the state to LDS and sums the partials in a fixed order (every thread a
// strided subset of the batches for one entry, all its loads issued
// together, then the subsets in order).  Wave 0 then takes the decisions:
// every lane evaluates the same scalar rules from LDS, the vectors are
// spread over the lanes.  Finally the state goes back, the instance's
// arrival counter is reset, and the phase's counters are advanced.
// ---------------------------------------------------------------------------
// LAZY: the rounds after a rejected trial evaluated the objective only (no
// Jacobian), so a trial accepted there is followed by a re-linearisation
// round; otherwise every round carries J at its first trial.
template <int R, bool LAZY = false>
__device__ bool solve_instance(const StepArgs& a, char* lds, int inst, int p, bool is_last) {
  constexpr int NA = R * (R + 1) / 2;
  constexpr int NRED = NA + R + TV;
  constexpr int NWORD = sizeof(GNState) / 8;
  constexpr int UNR = 16;  // loads in flight per thread
  GNState* gst = wsp<GNState>(a, a.L.state) + inst;
  GNState* st = reinterpret_cast<GNState*>(lds);
  double* sub = reinterpret_cast<double*>(lds + ((sizeof(GNState) + 15) / 16) * 16);
  const int nth = blockDim.x;
  const int NS = nth / NRED;  // strided subsets per entry
  double* red = sub + NS * NRED;
  __shared__ int s_done;
  // The state and the batch partials are independent: their loads are all
  // issued before the first wait (one memory round trip, not two).
  const int32_t* first_blk = wsp<int32_t>(a, a.L.first_blk);
  const int32_t b0 = first_blk[inst], b1 = first_blk[inst + 1];
  // wave 0's lanes k < R take q_n[k] for the trial latents: issued here, so
  // its latency overlaps the partials' loads
  const double qn_lane = (threadIdx.x < R) ? a.q_n[(int64_t)inst * R + threadIdx.x] : 0.0;
  if (p == 0) {  // the state before the first solve, formed from q_n
    for (int w = threadIdx.x; w < NWORD; w += nth)
      reinterpret_cast<uint64_t*>(st)[w] = gn_initial_word(w, a.q_n + (int64_t)inst * R, R, false);
  } else {
    for (int w = threadIdx.x; w < NWORD; w += nth)
      reinterpret_cast<uint64_t*>(st)[w] = ld_c(reinterpret_cast<const uint64_t*>(gst) + w);
  }
  const double* part = wsp<double>(a, a.L.partials);
  if (threadIdx.x < NS * NRED) {
    const int e = threadIdx.x % NRED, sl = threadIdx.x / NRED;
    double acc = 0.0;
    for (int32_t base = b0 + sl; base < b1; base += UNR * NS) {
      double v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {  // clamped, branch-free: all loads issue at once
        const int32_t b = base + u * NS;
        v[u] = ld_c(part + (int64_t)(b < b1 ? b : b0) * NRED + e);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) acc += (base + u * NS < b1) ? v[u] : 0.0;
    }
    sub[sl * NRED + e] = acc;
  }
  __syncthreads();
  if (p == 1) trace_solve(a, 48);
  const int phase = st->phase;
  if (threadIdx.x < NRED) {
    double s = 0.0;
    for (int sl = 0; sl < NS; ++sl) s += sub[sl * NRED + threadIdx.x];
    red[threadIdx.x] = s;
  }
  __syncthreads();
  if (p == 1) trace_solve(a, 49);

  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const double* bv = red + NA;
    const double* phit = red + NA + R;
    // scalar state (identical in every lane)
    double phi = st->phi, slope = st->slope, dnorm = st->dnorm;
    double alpha[TV];
    for (int t = 0; t < TV; ++t) alpha[t] = st->alpha[t];
    int iters = st->iters, ls_evals = st->ls_evals, flags = st->flags, ls_tried = st->ls_tried;
    int ph = phase;
    double obj_first = st->obj_first, obj_last = st->obj_last;
    // vectors: lane k < R holds entry k
    double qk = lane < R ? st->q[lane] : 0.0;
    double dk = lane < R ? st->delta[lane] : 0.0;
    const double* qv = st->q;  // the current iterate, readable by every lane
    bool done = false, newdir = false;
    // 1: trials q + alpha_t delta; 2: every trial at q (re-linearise);
    // 3: every trial at the initial guess
    int settrials = 0;
    if (ph == PH_INIT) {
      obj_first = obj_last = phi = phit[0];
      newdir = true;
      // elastic kinds: det F <= 0 met at a free sample by the target kernel
      // (written before this launch)
      if (a.L.nj && ld_c(wsp<uint32_t>(a, a.L.inv) + inst) != 0) flags |= CROM_FLAG_INVERTED;
    } else if (ph == PH_GUESS) {
      // The round evaluated the guess (trial 0, with J there).  A strictly
      // smaller objective makes it the start: the direction is formed from
      // this round's partials.  Otherwise the line search along the
      // direction found at q_n (kept in the state) goes ahead.
      if (isfinite(phit[0]) && phit[0] < phi) {
        qk = lane < R ? st->qt[0][lane] : 0.0;
        qv = st->qt[0];
        phi = phit[0];
        obj_last = phi;
        newdir = true;
      } else {
        ph = PH_TRIALS;
        settrials = 1;
      }
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
        double qq = 0.0;  // the vector from LDS at uniform addresses: no cross-lane rounds
#pragma unroll
        for (int k = 0; k < R; ++k) qq += qv[k] * qv[k];
        const double step = alpha[acc] * dnorm;
        qk = lane < R ? st->qt[acc][lane] : 0.0;
        iters += 1;
        phi = phit[acc];
        obj_last = phi;
        if (step <= a.tol * (1.0 + sqrt(qq))) {
          done = true;
        } else if (iters >= a.max_iter) {
          flags |= CROM_FLAG_MAXITER;
          done = true;
        } else if (acc == 0 && (!LAZY || ls_tried == 0)) {
          newdir = true;  // J at the accepted trial came with this round
        } else {
          ph = PH_REJAC;
          settrials = 2;
        }
      }
    } else {  // PH_REJAC: J^T J and J^T rho at the accepted iterate
      newdir = true;
    }

    if (p == 1) trace_solve(a, 53);
    if (newdir) {
      bool finite = isfinite(phi);
      for (int e = 0; e < NA + R; ++e) finite &= (bool)isfinite(red[e]);
      if (!finite) {
        flags |= CROM_FLAG_NONFINITE;
        done = true;
      } else {
        const CholOut o = chol_solve<R>(red, bv);
        const double xk = lane < R ? o.x : 0.0, dn = o.xx, sl = o.bx;
        double qq = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) qq += qv[k] * qv[k];
        if (!o.ok) {
          flags |= CROM_FLAG_SINGULAR;
          done = true;
        } else {
          dk = xk;
          dnorm = sqrt(dn);
          if (a.linearized) {
            qk += xk;
            iters = 1;
            done = true;
          } else if (dnorm <= a.tol * (1.0 + sqrt(qq))) {
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
            if (phase == PH_INIT && a.q_init) {  // evaluate the guess before any trial
              ph = PH_GUESS;
              settrials = 3;
            }
          }
        }
      }
    }
    if (p == 1) trace_solve(a, 54);
    if (!done && is_last) {
      flags |= CROM_FLAG_MAXITER;
      done = true;
    }
    if (done) ph = PH_DONE;
    // vector entries: lane k < R
    if (lane < R) {
      st->q[lane] = qk;
      st->delta[lane] = dk;
      st_c(a.q_next + (int64_t)inst * R + lane, qk);  // coherent: solvers of later phases may sit on other XCDs
    }
    // trial latents: lane t * R + k (TV * R <= 64)
    const double q_k = __shfl(qk, lane % R), d_k = __shfl(dk, lane % R);  // all lanes shuffle
    const double qn_k = __shfl(qn_lane, lane % R);
    if (!done && settrials == 3 && lane < TV * R) {
      const int t = lane / R, k = lane % R;
      const double g = a.q_init[(int64_t)inst * R + k];
      st->qt[t][k] = g;
      st->qd[t][k] = g - qn_k;
    } else if (!done && settrials && lane < TV * R) {
      const int t = lane / R, k = lane % R;
      const double al = settrials == 1 ? alpha[t] : 0.0;
      st->qt[t][k] = q_k + al * d_k;
      st->qd[t][k] = (q_k - qn_k) + al * d_k;
    }
    if (lane == 0) {
      for (int t = 0; t < TV; ++t) st->alpha[t] = alpha[t];
      st->phi = phi;
      st->slope = slope;
      st->dnorm = dnorm;
      st->iters = iters;
      st->ls_evals = ls_evals;
      st->flags = flags;
      st->ls_tried = ls_tried;
      st->obj_first = obj_first;
      st->obj_last = obj_last;
      if (phase != PH_INIT) st->rounds += 1;
      st->phase = ph;
      s_done = done ? 1 : 0;
      crom_step_info* inf = a.info + inst;
      st_c(&inf->flags, flags);
      st_c(&inf->iters, iters);
      st_c(&inf->ls_evals, ls_evals);
      st_c(&inf->rounds, st->rounds);
      st_c(&inf->obj_first, obj_first);
      st_c(&inf->obj_last, obj_last);
    }
  }
  __syncthreads();
  if (p == 1) trace_solve(a, 50);
  for (int w = threadIdx.x; w < NWORD; w += nth)
    st_c(reinterpret_cast<uint64_t*>(gst) + w, reinterpret_cast<const uint64_t*>(st)[w]);
  if (threadIdx.x == 0) {
    st_c(wsp<uint32_t>(a, a.L.inst_cnt) + inst, 0u);
    if (!s_done) atomicAdd(reinterpret_cast<unsigned long long*>(wsp<int64_t>(a, a.L.act_phase) + p + 1), 1ull);
  }
  wait_mem();
  __syncthreads();
  if (p == 1) trace_solve(a, 51);
  const bool cont = s_done == 0;
  if (threadIdx.x == 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(wsp<uint64_t>(a, a.L.sync) + SYNC_SOLVED), 1ull);
  __syncthreads();
  if (p == 1) trace_solve(a, 52);
  return cont;  // the instance takes part in the next round
}

// ---------------------------------------------------------------------------
// The persistent step kernel.  The launch takes at most as many workgroups as
// the device holds at once (occupancy query), so on an otherwise idle stream
// every workgroup is resident; every wait is bounded (SPIN_MAX), so a
// workgroup that is not resident makes the step end with ABORTED instead of
// hanging.  A plain launch: the cooperative launch API measured 18 us more
// per step in dispatch.
// ---------------------------------------------------------------------------
constexpr int64_t SPIN_MAX = int64_t(1) << 21;  // bounded waits: ~2e6 polls of ~1 us

// Engines and LDS layout of the persistent kernel per PDE kind: the
// engines' activation regions share the start of the dynamic LDS; the
// elastic kind keeps its J rows and residuals (FP64) above them; the
// parameter cache comes last, at PAR.
template <class S, int NW, int PREC, int PF, int KIND, bool REV = false>
struct StepTraits {
  using E0 = Engine<S, Cols<S::M, S::R, 1, 0, true, D2_LAP, S::R>, 1, NW, PREC, PF, true>;
  using E1 = Engine<S, Cols<S::M, S::R, 1, TV, false, D2_NONE, S::R>, 1, NW, PREC, PF, true>;
  static constexpr int ENG = E0::LDS_BYTES > E1::LDS_BYTES ? E0::LDS_BYTES : E1::LDS_BYTES;
  static constexpr int JD_OFF = ENG;
  static constexpr int PAR = ENG;
  static constexpr int STAGE = E0::ACT_REGION < E1::ACT_REGION ? E0::ACT_REGION : E1::ACT_REGION;
};
// The heat step with the reverse-pass evaluations: the jets at q_n, the
// trial rounds that re-linearise, and the backtracking rounds' objective.
template <class S, int NW, int PREC, int PF>
struct StepTraits<S, NW, PREC, PF, PK_HEAT, true> {
  using E0 = RevLap<S, NW, PREC, PF>;
  using E1 = RevTrial<S, NW, PREC, PF>;
  using E2 = Engine<S, Cols<S::M, S::R, 1, TV, false, D2_NONE, 0>, 1, NW, PREC, PF, true>;
  static constexpr int ENG01 = E0::LDS_BYTES > E1::LDS_BYTES ? E0::LDS_BYTES : E1::LDS_BYTES;
  static constexpr int ENG = ENG01 > E2::LDS_BYTES ? ENG01 : E2::LDS_BYTES;
  static constexpr int JD_OFF = ENG;
  static constexpr int PAR = ENG;
  static constexpr int STAGE0 = E0::EF::ACT_REGION < E1::EF::ACT_REGION ? E0::EF::ACT_REGION : E1::EF::ACT_REGION;
  static constexpr int STAGE = STAGE0 < E2::ACT_REGION ? STAGE0 : E2::ACT_REGION;
};
template <class S, int NW, int PREC, int PF>
struct StepTraits<S, NW, PREC, PF, PK_ELASTIC> {
  using E0 = Engine<S, Cols<S::M, S::R, 1, TV, false, D2_NONE, 0>, 1, NW, PREC, PF>;
  using E1 = Engine<S, Cols<S::M, S::R, 1, 1, false, D2_NONE, ElasticChunks<PREC>::QC>, 1, NW, PREC, PF>;
  static constexpr int ENG = E0::LDS_BYTES > E1::LDS_BYTES ? E0::LDS_BYTES : E1::LDS_BYTES;
  static constexpr int JD_OFF = (ENG + 15) / 16 * 16;
  static constexpr int PAR = JD_OFF + PT * S::D * (S::R + TV) * 8;
};

template <class S, int NW, int PREC, int PF, int KIND, int WPE, bool REV>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void step_kernel(StepArgs a,
                                                                                          int max_rounds) {
  using T = StepTraits<S, NW, PREC, PF, KIND, REV>;
  constexpr int PAR = T::PAR;
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_last, s_abort, s_ph, s_lt;
  __shared__ int64_t s_act;
  __shared__ double qdl[TV * RMAX];
  float* par = reinterpret_cast<float*>(lds + PAR);
  double* jd = reinterpret_cast<double*>(lds + T::JD_OFF);
  T::E0::PC::load(par, a.params, a.pi, a.depth, NW * 64);
  __syncthreads();
  const int64_t nblk = *wsp<int64_t>(a, a.L.nblk);
  // the elastic kind spreads a batch's latent-tangent chunks over NCH
  // workgroups (work item w = batch w / NCH, chunk w % NCH)
  constexpr int NCH = KIND == PK_ELASTIC ? S::R / ElasticChunks<PREC>::QC : 1;
  static_assert(KIND != PK_ELASTIC || S::R % ElasticChunks<PREC>::QC == 0, "whole chunks");
  // backtracking rounds without the Jacobian (the solve re-linearises an
  // accepted shortened step in a round of its own)
  constexpr bool LAZY = KIND == PK_ELASTIC && !ElasticChunks<PREC>::EAGER_J;
  const int64_t nwork = nblk * NCH;
  const int32_t* blk_inst = wsp<int32_t>(a, a.L.blk_inst);
  const int32_t* first_blk = wsp<int32_t>(a, a.L.first_blk);
  GNState* state = wsp<GNState>(a, a.L.state);
  uint32_t* inst_cnt = wsp<uint32_t>(a, a.L.inst_cnt);
  int64_t* act_phase = wsp<int64_t>(a, a.L.act_phase);
  uint64_t* sync = wsp<uint64_t>(a, a.L.sync);
  uint64_t target = 0;
  bool aborted = false;
  for (int p = 0; p <= max_rounds && !aborted; ++p) {
    // One memory round trip for the round's active count and, for this
    // workgroup's first batch, its instance's phase and trial offsets (all
    // final once the previous phase's solves are counted).
    const bool pre = p > 0 && (int64_t)blockIdx.x < nwork;
    const int inst0 = pre ? blk_inst[blockIdx.x / NCH] : 0;
    if (threadIdx.x == 0) s_act = ld_c(act_phase + p);  // stable: written only by phase p-1 solves
    if (pre) {
      if (threadIdx.x == blockDim.x - 1) s_ph = ld_c(&state[inst0].phase);
      if (LAZY && threadIdx.x == blockDim.x - 2) s_lt = ld_c(&state[inst0].ls_tried);
      for (int i = threadIdx.x; i < TV * S::R; i += blockDim.x) qdl[i] = ld_c(&state[inst0].qd[i / S::R][i % S::R]);
    }
    __syncthreads();
    const int64_t act = s_act;
    const int ph0 = s_ph, lt0 = LAZY ? s_lt : 0;
    __syncthreads();
    if (act == 0) break;
    target += (uint64_t)act;
    trace_mark(a, 4 * p);
    for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
      const int64_t blk = w / NCH;
      const int ch = (int)(w % NCH);
      const int inst = blk_inst[blk];
      if (p == 0) {
        if constexpr (KIND == PK_HEAT) eval_jets_batch<S, NW, PREC, PF, REV>(a, lds, par, blk);
        else if (ch == 0) eval_init_elastic<S>(a, jd, blk);
        else continue;
      } else {
        const bool first = w == blockIdx.x;  // phase and trial offsets preloaded
        int ph = ph0, lt = lt0;
        if (!first) {
          if (threadIdx.x == 0) {
            s_ph = ld_c(&state[inst].phase);  // stable until this batch arrives
            if (LAZY) s_lt = ld_c(&state[inst].ls_tried);
          }
          __syncthreads();
          ph = s_ph;
          lt = LAZY ? s_lt : 0;
          __syncthreads();
        }
        if (!evaluates_trials(ph)) continue;
        if constexpr (KIND == PK_HEAT)
          eval_trials_batch<S, NW, PREC, PF, true, REV>(a, lds, par, qdl, blk, inst, (p == 1 && first) ? 40 : -1,
                                                        first);
        else if (!eval_trials_elastic<S, NW, PREC, PF>(a, lds, jd, par, qdl, blk, ch, inst, first,
                                                        !(LAZY && ph == PH_TRIALS && lt > 0)))
          continue;
      }
      // arrival: the partials of this batch are complete in memory
      if (p == 1 && w == blockIdx.x) trace_mark(a, 44);
      wait_mem();
      __syncthreads();
      if (p == 1 && w == blockIdx.x) trace_mark(a, 45);
      if (threadIdx.x == 0) {
        const uint32_t nb = (uint32_t)(first_blk[inst + 1] - first_blk[inst]);
        const uint32_t old = atomicAdd(inst_cnt + inst, 1u);
        s_last = (old + 1 == nb);
      }
      __syncthreads();
      const bool last = s_last != 0;
      __syncthreads();  // every thread has read s_last before thread 0 may write it again
      if (p == 1 && w == blockIdx.x) trace_mark(a, 46);
      if (last) solve_instance<S::R, LAZY>(a, lds, inst, p, p == max_rounds);
      if (p == 1 && w == blockIdx.x) trace_mark(a, 47);
    }
    trace_mark(a, 4 * p + 1);
    // wait until every instance active in this phase has been solved
    if (threadIdx.x == 0) {
      int64_t spins = 0;
      while (ld_c(sync + SYNC_SOLVED) < target) {
        if (ld_c(sync + SYNC_ABORT) != 0 || ++spins > SPIN_MAX) {
          st_c(sync + SYNC_ABORT, (uint64_t)1);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      s_abort = ld_c(sync + SYNC_ABORT) != 0;
    }
    __syncthreads();
    aborted = s_abort != 0;
    trace_mark(a, 4 * p + 2);
  }
  // The last workgroup to leave marks the instances an abort left
  // unfinished.  Every other workgroup has left its loop by then, so no
  // solve runs after this: a solve that completed after the abort word was
  // set either finished its instance (a complete result) or moved it to a
  // phase nobody evaluates, which is marked here.
  wait_mem();
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = atomicAdd(reinterpret_cast<unsigned long long*>(sync + SYNC_EXITED), 1ull) + 1 ==
             (unsigned long long)gridDim.x;
  __syncthreads();
  if (s_last && ld_c(sync + SYNC_ABORT) != 0) {
    for (int i = threadIdx.x; i < a.n_inst; i += blockDim.x) {
      if (ld_c(&state[i].phase) != PH_DONE)
        st_c(&a.info[i].flags, ld_c(&a.info[i].flags) | CROM_FLAG_ABORTED);
    }
  }
}

// ---------------------------------------------------------------------------
// The linearised heat step (Sec. "Linearization") without the persistent
// protocol: one kernel evaluates every batch and stores its partial sums,
// then one wave per instance sums them in batch order and solves.  Each
// instance's result depends only on its own batches, so a batch of
// instances reproduces each instance run alone bit for bit.
// ---------------------------------------------------------------------------
template <class S, int NW, int PREC, int PF, int WPE, bool REV>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void lls_jets_kernel(StepArgs a) {
  using E = Engine<S, Cols<S::M, S::R, 1, 0, true, D2_LAP, S::R>, 1, NW, PREC, PF>;
  constexpr int ENG = REV ? RevLap<S, NW, PREC, PF, false>::LDS_BYTES : E::LDS_BYTES;
  extern __shared__ __align__(16) char lds[];
  const int64_t nblk = *wsp<int64_t>(a, a.L.nblk);
  if ((int64_t)blockIdx.x >= nblk) return;
  float* par = reinterpret_cast<float*>(lds + ENG);
  E::PC::load(par, a.params, a.pi, a.depth, NW * 64);
  __syncthreads();
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x)
    eval_jets_batch<S, NW, PREC, PF, REV, false>(a, lds, par, blk);
}

// The instance's batch partials are summed by the whole workgroup: entry e
// by NS strided subsets of the batches (subset s takes batches b0 + s,
// b0 + s + NS, ...), each with UNR loads in flight, then the subsets in
// order; a fixed order for any batch layout.  One wave then solves.
constexpr int LLS_SOLVE_THREADS = 256;
template <int R>
__global__ __launch_bounds__(LLS_SOLVE_THREADS) void lls_solve_kernel(StepArgs a) {
  constexpr int NA = R * (R + 1) / 2;
  constexpr int NRED = NA + R + TV;
  constexpr int NS = LLS_SOLVE_THREADS / NRED;
  constexpr int UNR = 8;
  static_assert(NRED <= LLS_SOLVE_THREADS, "one thread per reduced entry");
  __shared__ double sub[NS * NRED];
  __shared__ double red[NRED];
  const int inst = blockIdx.x, lane = threadIdx.x;
  const int32_t* first_blk = wsp<int32_t>(a, a.L.first_blk);
  const int32_t b0 = first_blk[inst], b1 = first_blk[inst + 1];
  if (b0 == b1) return;  // no samples: the setup kernel already reported it
  const double* part = wsp<double>(a, a.L.partials);
  if (threadIdx.x < NS * NRED) {
    const int e = threadIdx.x % NRED, sl = threadIdx.x / NRED;
    double acc = 0.0;
    for (int32_t base = b0 + sl; base < b1; base += UNR * NS) {
      double v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {  // clamped, branch-free: all loads issue at once
        const int32_t b = base + u * NS;
        v[u] = part[(int64_t)(b < b1 ? b : b0) * NRED + e];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) acc += (base + u * NS < b1) ? v[u] : 0.0;
    }
    sub[sl * NRED + e] = acc;
  }
  __syncthreads();
  if (threadIdx.x < NRED) {
    double acc = 0.0;
    for (int sl = 0; sl < NS; ++sl) acc += sub[sl * NRED + threadIdx.x];
    red[threadIdx.x] = acc;
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const double phi = red[NA + R];
  bool finite = isfinite(phi);
  for (int e = 0; e < NA + R; ++e) finite &= (bool)isfinite(red[e]);
  int flags = 0, iters = 0;
  const double* qn = a.q_n + (int64_t)inst * R;
  double qk = lane < R ? qn[lane] : 0.0;
  if (!finite) {
    flags = CROM_FLAG_NONFINITE;
  } else {
    const CholOut o = chol_solve<R>(red, red + NA);
    if (!o.ok) {
      flags = CROM_FLAG_SINGULAR;
    } else {
      qk += lane < R ? o.x : 0.0;
      iters = 1;
    }
  }
  if (lane < R) a.q_next[(int64_t)inst * R + lane] = qk;
  if (lane == 0) {
    crom_step_info inf;
    inf.flags = flags;
    inf.iters = iters;
    inf.ls_evals = 0;
    inf.rounds = 0;
    inf.obj_first = phi;
    inf.obj_last = phi;
    a.info[inst] = inf;
  }
}

// Workgroups of kernel k (threads, dynamic LDS) that the current device
// holds at once: a grid of that size gives every workgroup the same share
// of the batches (a larger one leaves its last, partial wave of
// workgroups on a part of the compute units).  Cached per call site for
// the last (device, kernel, LDS) asked.
#ifndef CROM_RESIDENT_WAVES
#define CROM_RESIDENT_WAVES 1
#endif
struct ResidentCache {
  int dev = -1, lds = -1;
  const void* k = nullptr;
  int64_t n = 0;
};
static crom_status resident_grid(ResidentCache& c, const void* k, int threads, int lds_bytes, int64_t* n) {
  int dev = 0;
  crom_status s = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (s != CROM_OK) return s;
  if (c.dev != dev || c.k != k || c.lds != lds_bytes) {
    int per_cu = 0, ncu = 0;
    s = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "attr");
    if (s == CROM_OK) s = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, lds_bytes),
                                    "occupancy");
    if (s != CROM_OK) return s;
    if (per_cu < 1) return fail(CROM_ERR_UNSUPPORTED, "kernel does not fit on a compute unit");
    c.dev = dev;
    c.k = k;
    c.lds = lds_bytes;
    c.n = (int64_t)per_cu * ncu * CROM_RESIDENT_WAVES;
  }
  *n = c.n;
  return CROM_OK;
}

// The latent Jacobian by the reverse pass where the depth allows (its
// slopes live in registers), else by forward tangent columns.
#ifndef CROM_LLS_REV
#define CROM_LLS_REV 1
#endif
template <class S, int NW, int PREC, int PF, int WPE, int WPE_REV = WPE>
static crom_status launch_lls(StepArgs a, hipStream_t st) {
  using E = Engine<S, Cols<S::M, S::R, 1, 0, true, D2_LAP, S::R>, 1, NW, PREC, PF>;
  using RJ = RevLap<S, NW, PREC, PF, false>;
  const bool rev = CROM_LLS_REV && RJ::supported(a.depth);
  const int lds_bytes = (rev ? RJ::LDS_BYTES : E::LDS_BYTES) + E::PC::bytes(a.depth);
  if (lds_bytes > LDS_MAX) return fail(CROM_ERR_UNSUPPORTED, "network too deep for the LDS");
  static_assert(PT * S::R * 8 + PT * TV * 8 <= E::ACT_REGION, "staging fits");
  static_assert(PT * S::R * 8 + PT * TV * 8 <= RJ::EF::ACT_REGION, "staging fits");
  auto k = rev ? lls_jets_kernel<S, NW, PREC, PF, WPE_REV, true> : lls_jets_kernel<S, NW, PREC, PF, WPE, false>;
  crom_status s = set_lds(k, lds_bytes);
  if (s != CROM_OK) return s;
  hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(SETUP_THREADS), 0, st, a);
  if ((s = hip_check(hipGetLastError(), "setup launch")) != CROM_OK) return s;
  // up to 4,096 workgroups, each loading the parameters once for its
  // batches (one wave of resident workgroups measured the same: 1.080 vs
  // 1.072 ms for 512 instances of the 2D decoder)
  int64_t g = a.L.nblk_max;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  // the benchmark timer brackets the evaluation kernel alone (the step's
  // dominant kernel; the solve kernel is a few microseconds)
  timer_mark(st);
  hipLaunchKernelGGL(k, dim3((unsigned)g), dim3(NW * 64), lds_bytes, st, a);
  if ((s = hip_check(hipGetLastError(), "lls launch")) != CROM_OK) return s;
  timer_mark(st);
  hipLaunchKernelGGL(lls_solve_kernel<S::R>, dim3((unsigned)a.n_inst), dim3(LLS_SOLVE_THREADS), 0, st, a);
  return hip_check(hipGetLastError(), "lls solve launch");
}

// ---------------------------------------------------------------------------
// Gauss-Newton for large batches as a sequence of kernels (one pass over the
// active batches per round, then one workgroup per instance deciding), in
// place of the persistent kernel's serial batches and per-batch handshake.
// The batch evaluations, their engine configuration and the solve (same
// code, same thread count, same summation order) are those of the
// persistent kernel, so every instance gets the same bits on either path.
// Rounds without an active instance return at once.
// ---------------------------------------------------------------------------
template <class S, int NW, int PREC, int PF, int WPE, bool REV>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void gn_round_kernel(StepArgs a,
                                                                                              int p) {
  using T = StepTraits<S, NW, PREC, PF, PK_HEAT, REV>;
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_ph, s_lt;
  __shared__ double qdl[TV * RMAX];
  // Round p >= 1 evaluates the batches that the solves of round p - 1 listed
  // for their continuing instances (list p % 2); this round's solves fill
  // the other list, whose count is cleared here (the solves run after this
  // kernel on the same stream).  Round 0 evaluates every batch.
  int64_t* work_cnt = wsp<int64_t>(a, a.L.work_cnt);
  if (blockIdx.x == 0 && threadIdx.x == 0) work_cnt[(p + 1) % 2] = 0;
  if (ld_c(wsp<int64_t>(a, a.L.act_phase) + p) == 0) return;  // uniform: nothing active in this round
  const int64_t nblk = p == 0 ? *wsp<int64_t>(a, a.L.nblk) : work_cnt[p % 2];
  if ((int64_t)blockIdx.x >= nblk) return;
  const int32_t* list = wsp<int32_t>(a, a.L.work) + (int64_t)(p % 2) * a.L.nblk_max;
  float* par = reinterpret_cast<float*>(lds + T::PAR);
  T::E0::PC::load(par, a.params, a.pi, a.depth, NW * 64);
  __syncthreads();
  const int32_t* blk_inst = wsp<int32_t>(a, a.L.blk_inst);
  const GNState* state = wsp<GNState>(a, a.L.state);
  for (int64_t it = blockIdx.x; it < nblk; it += gridDim.x) {
    const int64_t blk = p == 0 ? it : (int64_t)list[it];
    const int inst = blk_inst[blk];
    if (p == 0) {
      eval_jets_batch<S, NW, PREC, PF, REV>(a, lds, par, blk);
    } else {
      if (threadIdx.x == 0) {
        s_ph = ld_c(&state[inst].phase);
        s_lt = ld_c(&state[inst].ls_tried);
      }
      __syncthreads();
      const int ph = s_ph, lt = s_lt;
      __syncthreads();
      if (!evaluates_trials(ph)) continue;
      // a backtracking round (trials after a rejected one) needs only the
      // objective: no latent tangents (the solve re-linearises on acceptance)
      if (ph == PH_TRIALS && lt > 0)
        eval_trials_batch<S, NW, PREC, PF, false>(a, lds, par, qdl, blk, inst, -1, false);
      else
        eval_trials_batch<S, NW, PREC, PF, true, REV>(a, lds, par, qdl, blk, inst, -1, false);
    }
  }
}

template <int R, int NTH>
__global__ __launch_bounds__(NTH) void gn_solve_kernel(StepArgs a, int p, int is_last) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_ph;
  const int inst = blockIdx.x;
  const int32_t* first_blk = wsp<int32_t>(a, a.L.first_blk);
  if (first_blk[inst] == first_blk[inst + 1]) return;  // no samples: reported by the setup kernel
  if (threadIdx.x == 0) s_ph = ld_c(&wsp<GNState>(a, a.L.state)[inst].phase);
  __syncthreads();
  const int ph = s_ph;
  const bool active = p == 0 ? ph == PH_INIT : evaluates_trials(ph);
  if (!active) return;
  if (!solve_instance<R, true>(a, lds, inst, p, is_last != 0)) return;
  // list this instance's batches for the next round (any order: each batch
  // keeps its own partials slot and the solve sums them in batch order)
  __shared__ int64_t s_base;
  const int32_t b0 = first_blk[inst], b1 = first_blk[inst + 1];
  if (threadIdx.x == 0)
    s_base = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(wsp<int64_t>(a, a.L.work_cnt) + (p + 1) % 2),
                                (unsigned long long)(b1 - b0));
  __syncthreads();
  int32_t* list = wsp<int32_t>(a, a.L.work) + (int64_t)((p + 1) % 2) * a.L.nblk_max;
  for (int32_t i = threadIdx.x; i < b1 - b0; i += blockDim.x) list[s_base + i] = b0 + i;
}

// NWS: the waves of the persistent kernel whose solve the rounds repeat (its
// thread count fixes the solve's summation order), independent of the
// evaluation's NW: the evaluations' results do not depend on the wave count.
template <class S, int NW, int PREC, int PF, int WPE, bool REV, int NWS>
static crom_status launch_gn_rounds_t(StepArgs a, int max_rounds, hipStream_t st) {
  using T = StepTraits<S, NW, PREC, PF, PK_HEAT, REV>;
  const int lds_bytes = T::PAR + T::E0::PC::bytes(a.depth);
  if (lds_bytes + (int)sizeof(double) * TV * RMAX + 64 > LDS_MAX)
    return fail(CROM_ERR_UNSUPPORTED, "network too deep for the step kernel's LDS");
  constexpr int NRED = S::R * (S::R + 1) / 2 + S::R + TV;
  constexpr int SOLVE_LDS =
      (int)((sizeof(GNState) + 15) / 16 * 16) + ((NWS * 64) / NRED + 1) * NRED * 8 + 64;
  static_assert(PT * S::R * 8 + PT * TV * 8 <= T::STAGE, "staging fits");
  auto kr = gn_round_kernel<S, NW, PREC, PF, WPE, REV>;
  auto ks = gn_solve_kernel<S::R, NWS * 64>;
  crom_status s = set_lds(kr, lds_bytes);
  if (s != CROM_OK) return s;
  hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(SETUP_THREADS), 0, st, a);
  if ((s = hip_check(hipGetLastError(), "setup launch")) != CROM_OK) return s;
  // one wave of resident workgroups (512 instances of the 2D decoder,
  // BF16: 10.66 -> 10.33 ms per step against up to 4,096 workgroups)
  static ResidentCache rc;
  int64_t g = 0;
  if ((s = resident_grid(rc, reinterpret_cast<const void*>(kr), NW * 64, lds_bytes, &g)) != CROM_OK) return s;
  if (g > a.L.nblk_max) g = a.L.nblk_max;
  if (g < 1) g = 1;
  timer_mark(st);
  for (int p = 0; p <= max_rounds; ++p) {
    hipLaunchKernelGGL(kr, dim3((unsigned)g), dim3(NW * 64), lds_bytes, st, a, p);
    hipLaunchKernelGGL(ks, dim3((unsigned)a.n_inst), dim3(NWS * 64), SOLVE_LDS, st, a, p, (int)(p == max_rounds));
  }
  timer_mark(st);
  return hip_check(hipGetLastError(), "round launches");
}

// The Gauss-Newton evaluations take the reverse pass where the depth allows.
#ifndef CROM_GN_REV
#define CROM_GN_REV 1
#endif
template <class S, int NW, int PREC, int PF, int WPE, int WPE_REV, int NWS>
static crom_status launch_gn_rounds(StepArgs a, int max_rounds, hipStream_t st) {
  if (CROM_GN_REV && RevLap<S, NW, PREC, PF>::supported(a.depth))
    return launch_gn_rounds_t<S, NW, PREC, PF, WPE_REV, true, NWS>(a, max_rounds, st);
  return launch_gn_rounds_t<S, NW, PREC, PF, WPE, false, NWS>(a, max_rounds, st);
}

// One engine pass of the elastic preparation over every batch.
template <class S, class C, int NW, int PREC>
static crom_status launch_jets_pass(const StepArgs& a, int qb, hipStream_t st, int chunks = 1) {
  using E = Engine<S, C, 1, NW, PREC, 0>;
  const int lds_bytes = E::LDS_BYTES + E::PC::bytes(a.depth);
  if (lds_bytes > LDS_MAX) return fail(CROM_ERR_UNSUPPORTED, "network too deep for the LDS");
  auto k = jets_pass_kernel<S, C, NW, PREC>;
  crom_status s = set_lds(k, lds_bytes);
  if (s != CROM_OK) return s;
  int64_t g = a.L.nblk_max;
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k, dim3((unsigned)g, (unsigned)chunks), dim3(NW * 64), lds_bytes, st, a, qb);
  return hip_check(hipGetLastError(), "jets pass launch");
}

// Value, x-gradient, x-Hessian (in chunks of HC entries, each chunk
// recomputing the x tangents its entries need) and latent Jacobian (chunks
// of QC) at q_n in one launch, then the FP64 update of every sample.
template <class S, int NW, int PREC>
static crom_status elastic_prepare(const StepArgs& a, hipStream_t st) {
  using EJ = ElasticJets<S, PREC>;
  const int lds_bytes = EJ::template lds<NW>() + ParamCache<S>::bytes(a.depth);
  if (lds_bytes > LDS_MAX) return fail(CROM_ERR_UNSUPPORTED, "network too deep for the LDS");
  auto k = elastic_jets_kernel<S, NW, PREC>;
  crom_status s = set_lds(k, lds_bytes);
  if (s != CROM_OK) return s;
  int64_t g = a.L.nblk_max;
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k, dim3((unsigned)g, (unsigned)(EJ::NHC + EJ::NQC)), dim3(NW * 64), lds_bytes, st, a);
  s = hip_check(hipGetLastError(), "elastic jets launch");
  if (s != CROM_OK) return s;
  hipLaunchKernelGGL(elastic_targets_kernel<S::R>, dim3((unsigned)g), dim3(64), 0, st, a);
  return hip_check(hipGetLastError(), "elastic targets launch");
}

// Finite-element preparation: the ring decode at q_n, the samples' value and
// latent Jacobian (chunks of QC), then the per-sample update.
template <class S, int NW, int PREC>
static crom_status fe_prepare(const StepArgs& a, hipStream_t st) {
  constexpr int QC = ElasticChunks<PREC>::QC;
  using E = RingEngine<S, PREC>;
  if (a.fe.max_ring > 0) {
    const int lds_bytes = E::LDS_BYTES + E::PC::bytes(a.depth);
    if (lds_bytes > LDS_MAX) return fail(CROM_ERR_UNSUPPORTED, "network too deep for the LDS");
    auto k = ring_decode_kernel<S, PREC>;
    crom_status s = set_lds(k, lds_bytes);
    if (s != CROM_OK) return s;
    int64_t gx = (a.fe.max_ring + E::NPTS - 1) / E::NPTS;
    if (gx > 65535) gx = 65535;
    hipLaunchKernelGGL(k, dim3((unsigned)gx, (unsigned)a.n_inst), dim3(E::THREADS), lds_bytes, st, a);
    s = hip_check(hipGetLastError(), "ring decode launch");
    if (s != CROM_OK) return s;
  }
  static_assert(S::R % QC == 0, "whole latent chunks");
  crom_status s = launch_jets_pass<S, Cols<S::M, S::R, 1, 0, false, D2_NONE, QC>, NW, PREC>(a, 0, st, S::R / QC);
  if (s != CROM_OK) return s;
  int64_t g = a.L.nblk_max * (PT / FE_WAVES);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(fe_targets_kernel<S::R>, dim3((unsigned)g), dim3(FE_WAVES * 64), 0, st, a);
  return hip_check(hipGetLastError(), "finite-element targets launch");
}

template <class S, int NW, int PREC, int PF, int KIND, int WPE, bool REV>
static crom_status launch_step_t(StepArgs a, int max_rounds, hipStream_t st) {
  using T = StepTraits<S, NW, PREC, PF, KIND, REV>;
  constexpr int PAR = T::PAR;
  const int lds_bytes = PAR + T::E0::PC::bytes(a.depth);
  if (lds_bytes + (int)sizeof(double) * TV * RMAX + 64 > LDS_MAX)
    return fail(CROM_ERR_UNSUPPORTED, "network too deep for the step kernel's LDS");
  if constexpr (KIND == PK_HEAT) static_assert(PT * S::R * 8 + PT * TV * 8 <= T::STAGE, "staging fits");
  static_assert(sizeof(GNState) + 16 +
                    (NW * 64 + S::R * (S::R + 1) / 2 + S::R + TV + S::R * S::R + S::R) * 8 <= PAR,
                "solve scratch fits below the parameter cache");
  static_assert(NW * 64 >= S::R * (S::R + 1) / 2 + S::R + TV, "one thread per reduced entry");
  auto k = step_kernel<S, NW, PREC, PF, KIND, WPE, REV>;
  static int resident = 0, resident_lds = -1;
  if (resident_lds != lds_bytes) {
    crom_status s = set_lds(k, LDS_MAX - (int)sizeof(double) * TV * RMAX - 64);
    if (s != CROM_OK) return s;
    int dev = 0, per_cu = 0, ncu = 0;
    s = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (s == CROM_OK) s = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "attr");
    if (s == CROM_OK)
      s = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, NW * 64, lds_bytes), "occupancy");
    if (s != CROM_OK) return s;
    if (per_cu < 1) return fail(CROM_ERR_UNSUPPORTED, "step kernel does not fit on a compute unit");
    resident = per_cu * ncu;
    resident_lds = lds_bytes;
  }
  hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(SETUP_THREADS), 0, st, a);
  crom_status s = hip_check(hipGetLastError(), "setup launch");
  if (s != CROM_OK) return s;
  timer_mark(st);
  if constexpr (KIND == PK_ELASTIC) {
    s = a.fe.on ? fe_prepare<S, NW, PREC>(a, st) : elastic_prepare<S, NW, PREC>(a, st);
    if (s != CROM_OK) return s;
  }
  int64_t g = a.L.nblk_max * (KIND == PK_ELASTIC ? S::R / ElasticChunks<PREC>::QC : 1);
  if (g > resident) g = resident;
  if (g < 1) g = 1;
  void* args[] = {&a, &max_rounds};
  s = hip_check(hipLaunchKernel(reinterpret_cast<const void*>(k), dim3((unsigned)g), dim3(NW * 64), args, lds_bytes,
                                st),
                "step launch");
  timer_mark(st);
  return s;
}

template <class S, int NW, int PREC, int PF, int KIND = PK_HEAT, int WPE = 1>
static crom_status launch_step(StepArgs a, int max_rounds, hipStream_t st) {
  if constexpr (KIND == PK_HEAT) {
    if (CROM_GN_REV && RevLap<S, NW, PREC, PF>::supported(a.depth))
      return launch_step_t<S, NW, PREC, PF, KIND, WPE, true>(a, max_rounds, st);
  }
  return launch_step_t<S, NW, PREC, PF, KIND, WPE, false>(a, max_rounds, st);
}

// Waves per workgroup and weight prefetch per precision, chosen so that the
// persistent kernel stays clear of register spills: bfloat16 fragments are
// half the size, so BF16 and BF16_PURE afford eight waves with prefetch.
template <class S, int NWB, int NWF, int PFB = 1, int WPEB = 1>
static crom_status step_prec(int prec, const StepArgs& a, int rounds, hipStream_t st) {
  // sine networks: FP32 and BF16 only (checked by check_net)
  constexpr bool ALL = S::ACT == ACT_ELU;
  if (a.linearized) {
    // four waves with two M-tiles each and streamed weights: the measured
    // best for full batches (three workgroups per CU with the reverse pass)
    constexpr int NWL = S::MTILES < CROM_LIN_NW ? S::MTILES : CROM_LIN_NW;
    constexpr int WPE_REV = S::R > 8 ? 2 : CROM_LIN_REV_WPE;  // r = 16: the Jacobian sums need the registers
    if (prec == CROM_PREC_FP32) return launch_lls<S, NWF, PREC_FP32, 0, 1>(a, st);
    if (prec == CROM_PREC_BF16) return launch_lls<S, NWL, PREC_BF16, CROM_LIN_PF, CROM_LIN_WPE, WPE_REV>(a, st);
    if constexpr (ALL) {
      if (prec == CROM_PREC_BF16_PURE)
        return launch_lls<S, NWL, PREC_BF16_PURE, CROM_LIN_PF, CROM_LIN_WPE, WPE_REV>(a, st);
      return launch_lls<S, NWF, PREC_BF16X3, 0, 1>(a, st);
    }
    return fail(CROM_ERR_UNSUPPORTED, "precision");
  }
  if (a.L.nblk_max > ROUNDS_MIN_BATCHES) {
    // the evaluations in the linearised step's configuration (the fastest
    // for full batches), the solves with the persistent kernel's threads
    constexpr int NWL = S::MTILES < CROM_LIN_NW ? S::MTILES : CROM_LIN_NW;
    if (prec == CROM_PREC_FP32) return launch_gn_rounds<S, NWF, PREC_FP32, 0, 1, 1, NWF>(a, rounds, st);
    if (prec == CROM_PREC_BF16)
      return launch_gn_rounds<S, NWL, PREC_BF16, CROM_LIN_PF, CROM_LIN_WPE, CROM_GN_REV_WPE, NWB>(a, rounds, st);
    if constexpr (ALL) {
      if (prec == CROM_PREC_BF16_PURE)
        return launch_gn_rounds<S, NWL, PREC_BF16_PURE, CROM_LIN_PF, CROM_LIN_WPE, CROM_GN_REV_WPE, NWB>(a, rounds,
                                                                                                     st);
      return launch_gn_rounds<S, NWF, PREC_BF16X3, 0, 1, 1, NWF>(a, rounds, st);
    }
    return fail(CROM_ERR_UNSUPPORTED, "precision");
  }
  if (prec == CROM_PREC_FP32) return launch_step<S, NWF, PREC_FP32, 0>(a, rounds, st);
  if (prec == CROM_PREC_BF16) return launch_step<S, NWB, PREC_BF16, PFB, PK_HEAT, WPEB>(a, rounds, st);
  if constexpr (ALL) {
    if (prec == CROM_PREC_BF16_PURE) return launch_step<S, NWB, PREC_BF16_PURE, PFB, PK_HEAT, WPEB>(a, rounds, st);
    return launch_step<S, NWF, PREC_BF16X3, 0>(a, rounds, st);
  }
  return fail(CROM_ERR_UNSUPPORTED, "precision");
}

// The elastic step at width 256 (weight fragments streamed per K-block).
template <class S, int NW>
static crom_status step_prec_elastic(int prec, const StepArgs& a, int rounds, hipStream_t st) {
  switch (prec) {
    case CROM_PREC_FP32: return launch_step<S, NW, PREC_FP32, CROM_ELASTIC_PF, PK_ELASTIC>(a, rounds, st);
    case CROM_PREC_BF16: return launch_step<S, NW, PREC_BF16, CROM_ELASTIC_PF, PK_ELASTIC>(a, rounds, st);
    case CROM_PREC_BF16_PURE: return launch_step<S, NW, PREC_BF16_PURE, CROM_ELASTIC_PF, PK_ELASTIC>(a, rounds, st);
    default: return launch_step<S, NW, PREC_BF16X3, CROM_ELASTIC_PF, PK_ELASTIC>(a, rounds, st);
  }
}

}  // namespace crom

using namespace crom;

#ifdef CROM_STEP_TRACE
// Probe builds only: phase timestamps of the persistent step kernel.
static uint64_t* g_step_trace = nullptr;
extern "C" void crom_debug_step_trace(uint64_t* buf) { g_step_trace = buf; }
#endif

extern "C" {

crom_status crom_step_workspace(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                size_t* bytes) {
  crom_status s = check_net(net, false);
  if (s != CROM_OK) return s;
  if (!bytes) return fail(CROM_ERR_INVALID_ARG, "bytes is NULL");
  if (n_inst < 0 || total_samples < 0) return fail(CROM_ERR_INVALID_ARG, "negative size");
  *bytes = ws_layout(net->r, net->d, net->m, n_inst, total_samples).total;
  return CROM_OK;
}

const double* crom_step_targets(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                const void* ws) {
  if (!net || !ws || n_inst < 0 || total_samples < 0) return nullptr;
  WsLayout L = ws_layout(net->r, net->d, net->m, n_inst, total_samples);
  return reinterpret_cast<const double*>(static_cast<const char*>(ws) + L.targets);
}

const double* crom_step_increments(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                   const void* ws) {
  if (!net || !ws || n_inst < 0 || total_samples < 0) return nullptr;
  WsLayout L = ws_layout(net->r, net->d, net->m, n_inst, total_samples);
  return reinterpret_cast<const double*>(static_cast<const char*>(ws) + L.rho0);
}

crom_status crom_step_guess(const crom_net* net, const crom_pde* pde, int32_t n_inst,
                            const int64_t* offsets, int64_t total_samples, const float* y,
                            const uint8_t* clamp, const double* q_prev, const double* q_n,
                            const double* q_init, double* q_next, const crom_gn_opts* opts,
                            crom_step_info* info, void* ws, size_t ws_bytes, void* stream) {
  crom_status s = check_net(net, true);
  if (s != CROM_OK) return s;
  if (!pde || !opts) return fail(CROM_ERR_INVALID_ARG, "pde and opts are required");
  if (pde->kind != CROM_PDE_HEAT && pde->kind != CROM_PDE_NEOHOOKEAN && pde->kind != CROM_PDE_COROTATED_FE &&
      pde->kind != CROM_PDE_PROJECT)
    return fail(CROM_ERR_UNSUPPORTED, "pde kind");
  if (pde->kind == CROM_PDE_HEAT && net->d != 1) return fail(CROM_ERR_UNSUPPORTED, "the heat step needs d == 1");
  if (pde->kind == CROM_PDE_PROJECT && (net->d != 1 || net->m > 2))
    return fail(CROM_ERR_UNSUPPORTED, "the projection needs d == 1 and m <= 2");
  const bool project = pde->kind == CROM_PDE_PROJECT;
  const bool elastic = pde->kind == CROM_PDE_NEOHOOKEAN || pde->kind == CROM_PDE_COROTATED_FE;
  if (elastic && (net->d != 3 || net->m != 3))
    return fail(CROM_ERR_UNSUPPORTED, "the elastic steps need m == 3 and d == 3");
  const crom_fe_mesh* mesh = pde->kind == CROM_PDE_COROTATED_FE ? pde->mesh : nullptr;
  if (pde->kind == CROM_PDE_COROTATED_FE) {
    if (!mesh) return fail(CROM_ERR_INVALID_ARG, "the finite-element step needs pde->mesh");
    if (mesh->n_ring < 0 || mesh->max_ring < 0 || mesh->n_inc < 0 || mesh->max_ring > mesh->n_ring)
      return fail(CROM_ERR_INVALID_ARG, "mesh sizes out of range");
    if (!mesh->ring_offsets || !mesh->inc_offsets || (mesh->n_ring > 0 && (!mesh->ring_X || !mesh->ring_u)) ||
        (mesh->n_inc > 0 && (!mesh->inc_tets || !mesh->inc_corner)))
      return fail(CROM_ERR_INVALID_ARG, "mesh arrays are required");
    if (n_inst > 65535) return fail(CROM_ERR_UNSUPPORTED, "the finite-element step takes at most 65535 instances");
  }
  if (net->r > RMAX) return fail(CROM_ERR_UNSUPPORTED, "r > 16");
  if (n_inst < 0 || total_samples < 0) return fail(CROM_ERR_INVALID_ARG, "negative size");
  if (n_inst == 0) return CROM_OK;
  if (!offsets || !q_n || !q_next || !info || !pde->coef)
    return fail(CROM_ERR_INVALID_ARG, "offsets, q_n, q_next, info and pde->coef are required");
  if (total_samples > 0 && !y) return fail(CROM_ERR_INVALID_ARG, "y is NULL");
  if (q_next == q_n) return fail(CROM_ERR_INVALID_ARG, "q_next must not alias q_n");
  if (q_init && q_init == q_next) return fail(CROM_ERR_INVALID_ARG, "q_next must not alias q_init");
  if (opts->max_iter < 1 || opts->ls_max < 0 || opts->max_rounds < 0 || !(opts->tol_step >= 0.0) ||
      !(opts->ls_shrink > 0.0 && opts->ls_shrink < 1.0) || !(opts->armijo_c >= 0.0))
    return fail(CROM_ERR_INVALID_ARG, "gn opts out of range");
  if (!project && !(pde->dt > 0.0)) return fail(CROM_ERR_INVALID_ARG, "dt must be positive");
  WsLayout L = ws_layout(net->r, net->d, net->m, n_inst, total_samples);
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
  a.given = project ? pde->coef : nullptr;
  a.dt = pde->dt;
  a.q_prev = elastic ? q_prev : nullptr;
  if (mesh) {
    a.fe.ring_offsets = mesh->ring_offsets;
    a.fe.ring_X = mesh->ring_X;
    a.fe.inc_offsets = mesh->inc_offsets;
    a.fe.inc_tets = mesh->inc_tets;
    a.fe.inc_corner = mesh->inc_corner;
    a.fe.ring_u = mesh->ring_u;
    a.fe.n_ring = mesh->n_ring;
    a.fe.max_ring = mesh->max_ring;
    a.fe.n_inc = mesh->n_inc;
    a.fe.on = 1;
  }
  a.q_n = q_n;
  a.q_init = q_init;
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
#ifdef CROM_STEP_TRACE
  a.trace = g_step_trace;
#endif
  // Enough rounds for max_iter accepted steps, each after the longest line
  // search (ceil((ls_max + 1) / TV) rounds) and one re-linearisation.
  const int64_t worst = (int64_t)opts->max_iter * (1 + (opts->ls_max + TV) / TV) + 1 + (q_init ? 1 : 0);
  int64_t rounds = opts->linearized ? 0 : (opts->max_rounds > 0 ? opts->max_rounds : worst);
  if (rounds > MAXP) rounds = MAXP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (shape_id(net->m, net->r, net->d, net->width)) {
    case SHAPE_1D:
      if (net->act == CROM_ACT_SINE) return step_prec<Shape<32, 1, 3, 1, ACT_SINE>, 2, 2>(net->precision, a, (int)rounds, st);
      return step_prec<Shape<32, 1, 3, 1>, 2, 2>(net->precision, a, (int)rounds, st);
    case SHAPE_2D:
      if (net->act == CROM_ACT_SINE)
        return step_prec<Shape<128, 2, 8, 1, ACT_SINE>, CROM_STEP2D_NW, 4, CROM_STEP2D_PF, CROM_STEP2D_WPE>(
            net->precision, a, (int)rounds, st);
      return step_prec<Shape<128, 2, 8, 1>, CROM_STEP2D_NW, 4, CROM_STEP2D_PF, CROM_STEP2D_WPE>(net->precision, a,
                                                                                         (int)rounds, st);
    case SHAPE_3D: return step_prec_elastic<Shape<256, 3, 16, 3>, CROM_ELASTIC_NW>(net->precision, a, (int)rounds, st);
    case SHAPE_2D_R16:  // four waves: with r = 16 eight spill in BF16
      return step_prec<Shape<128, 2, 16, 1>, 4, 4, CROM_STEP2D_PF, 1>(net->precision, a, (int)rounds, st);
    default: return fail(CROM_ERR_UNSUPPORTED, "shape");
  }
}

crom_status crom_step(const crom_net* net, const crom_pde* pde, int32_t n_inst,
                      const int64_t* offsets, int64_t total_samples, const float* y,
                      const uint8_t* clamp, const double* q_prev, const double* q_n, double* q_next,
                      const crom_gn_opts* opts, crom_step_info* info, void* ws, size_t ws_bytes,
                      void* stream) {
  return crom_step_guess(net, pde, n_inst, offsets, total_samples, y, clamp, q_prev, q_n, nullptr, q_next, opts,
                         info, ws, ws_bytes, stream);
}

}  // extern "C"
