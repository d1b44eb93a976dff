// Fused per-chain-tile kernels: target evaluation (FP64 assembly around the MLP emulator)
// and the MH / MALA / HMC / AIES / NUTS / differential-evolution transitions.  Templated on the GEMM precision P and the
// chain-tile width M = 16*MT; instantiated once per precision in kernels_<prec>.hip.
#pragma once
#include "mlp_tile.hpp"

namespace best {

constexpr int kMaxTerms = 8;  // plain model terms held in registers

struct Target {
  int d;
  const double *lower, *upper;
  double gauss_coef;
  const double *gmean, *gprec;
  int tw_u, tw_v;
  double tw_beta, tw_center, tw_kappa;
  const double *in_center, *in_invscale;
  double mlp_coef, offset;
  int plain_mode;
  const double *train_lo, *train_hi;
  int n_bins, n_terms;
  const double *xgrid, *data, *w2, *pa, *pg, *pp, *pk, *pg0, *pc, *pis;
  int box_penalty;  // 1: smooth penalty outside the prior box instead of -inf
  double pen_w;     // its width w (in box widths)
};

// Smooth boundary penalty: r = distance of x_i outside [lower_i, upper_i] in box widths,
// P_i = exp(r/w) - 1 - r/w (zero value and slope at the face), dP_i/dx_i returned in *dp.
__device__ __forceinline__ double box_pen(const Target& tg, int i, double x, double* dp) {
  const double wd = tg.upper[i] - tg.lower[i];
  double r = 0.0, s = 0.0;
  if (x > tg.upper[i]) {
    r = (x - tg.upper[i]) / wd;
    s = 1.0 / wd;
  } else if (x < tg.lower[i]) {
    r = (tg.lower[i] - x) / wd;
    s = -1.0 / wd;
  }
  const double em = expm1(r / tg.pen_w);
  *dp = em / tg.pen_w * s;
  return em - r / tg.pen_w;
}

struct Whiten {
  const double* mu;  // [d]
  const double* L;   // [d*d] row-major lower triangle
};

// Chain state and per-chain scratch, SoA [d][Np] (chain fastest) and [Np].
struct State {
  int64_t Np, N;
  double *x, *z, *gx, *lp;
  double *xp, *zp, *gxp, *lpp, *q, *gz, *gzp;
  uint32_t *n_acc, *n_nonfinite, *n_oob;
  uint32_t* n_evals;  // emulator evaluations per chain (samplers whose count varies: NUTS)
  double *sum_prob, *step_prob;
};

// NUTS trajectory state (global memory; one chain's d components contiguous, element
// (c, i) at [c * d + i] of a [Np][d] array, so that a lane group holding one chain reads
// them in one pass): the tree ends (whitened position, momentum, whitened gradient), the
// tree's candidate (x, grad_x, log pi) and, per subtree level 0 .. max_depth - 1, the
// pending left sibling (its first leaf's z and q, its candidate, its valid-point count).
struct NutsState {
  double *zm, *qm, *gm, *zpl, *qpl, *gpl;  // [Np][d]
  double *xc, *gxc, *lpc;                  // [Np][d], [Np][d], [Np]
  double *pz, *pq, *px, *pgx;              // [max_depth][Np][d]
  double *plp, *pn;                        // [max_depth][Np]
  int max_depth;
};

// Byte offsets into dynamic LDS (computed on the host by lds_layout()).
struct LdsLayout {
  int big, th, gth, red, outp, out, up, mi, md, st, cst, w1, total;
  int w1f_bytes, w1t_bytes;  // sizes of the resident input-layer weights (w1 >= 0)
};

__host__ __device__ inline int align16(int v) { return (v + 15) & ~15; }

// The tile scratch and the staged constants live in LDS or in global memory depending on
// the layout, and are reached through generic pointers either way.  Pointers into LDS that
// stand in for global arrays pass through here, so that the optimiser treats them as
// plain generic pointers: with their LDS origin visible, this compiler (ROCm 7.2) can emit
// an invalid aperture comparison for them.
template <class T>
__device__ __forceinline__ T* generic_ptr(T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Union region: {activation slots or ping-pong buffers + delta buffers} during the MLP,
// {R, PR, plain results, plain scratch} during the FP64 assembly.
// The input buffer holds M x k1 values of isize bytes (d padded to the input layer's
// k-step); waves is the tile workgroup's wave count (per-wave partial sums).
// With st_lds = 1 the per-step FP64 scratch of the tile (7 [d][M] arrays and log pi of the
// proposals) and the launch's small constant arrays also live in LDS (st, cst >= 0); with
// st_lds = 2 only the constants do (cst >= 0, st = -1); the others stay in global memory
// (-1).  With w1_bytes = (w1f, w1t) sizes > 0 the input layer's
// packed weights W_1 and W_1^T are copied into LDS once per launch (w1 >= 0).
__host__ __device__ inline LdsLayout lds_layout(int M, int H, int d, int nh, int lds_h,
                                               int tsize, int vsize, int asize, int k1,
                                               int isize, int waves, int st_lds,
                                               int w1f_bytes = 0, int w1t_bytes = 0) {
  LdsLayout L;
  const int mlp_bytes = (lds_h ? nh + 2 : 2) * M * H * tsize;
  const int asm_bytes = 8 * (2 * d * M + M + M * d + kMaxD + 3 * kMaxTerms + waves * 32);
  L.big = 0;
  int o = align16(mlp_bytes > asm_bytes ? mlp_bytes : asm_bytes);
  L.th = o;
  o = align16(o + M * k1 * isize);
  L.gth = o;
  o = align16(o + M * d * vsize);
  // input-gradient partial sums: inside the delta buffer that does not hold delta_1 when
  // they fit there (it is dead by then), else a region of their own
  if (waves * d * asize <= H * tsize) {
    const int MH = M * H * tsize;
    const int dlt0 = lds_h ? nh * MH : ((nh - 1) & 1) * MH;
    const int dlt1 = lds_h ? (nh + 1) * MH : (nh & 1) * MH;
    L.red = L.big + ((((nh - 1) & 1) == 0) ? dlt1 : dlt0);
  } else {
    L.red = o;
    o = align16(o + waves * M * d * asize);
  }
  L.outp = o;
  o = align16(o + waves * M * asize);
  L.out = o;
  o = align16(o + M * asize);
  L.up = o;
  o = align16(o + M * asize);
  L.mi = o;  // ints: inbox[M], intrain[M], flag[M]
  o = align16(o + 4 * M * 4);
  L.md = o;  // doubles: 8 per chain
  o = align16(o + 8 * M * 8);
  L.st = L.cst = -1;
  if (st_lds == 1) {
    L.st = o;
    o = align16(o + (7 * d * M + M) * 8);
  }
  if (st_lds) {
    L.cst = o;  // launch constants: L, S^-1 (d x d), mu, gauss mean, box, input scaling
    o = align16(o + (2 * d * d + 8 * d) * 8);
  }
  L.w1 = -1;
  L.w1f_bytes = L.w1t_bytes = 0;
  if (w1f_bytes > 0) {
    L.w1 = o;
    L.w1f_bytes = w1f_bytes;
    L.w1t_bytes = w1t_bytes;
    o = align16(o + w1f_bytes + w1t_bytes);
  }
  L.total = o;
  return L;
}

struct KArgs {
  Target tg;
  MlpParams mp;
  Whiten wh;
  State st;
  Rng rng;
  LdsLayout lds;
  int sampler;
  int adapt;  // step-size adaptation launch (one step, step size read from the device)
  int64_t step0;
  int n_steps;
  double eps;
  const double* eps_ptr;
  double mh_scale, stretch_a;
  double de_sigma;  // sd of eta in the differential-evolution gamma
  const double* step_mult;  // per-dimension step multipliers [d] (MALA, MH) or nullptr
  int n_leap;
  int thin;
  float* record;
  int64_t rec_cap, rec_s0, rec_pitch;  // rec_s0: index of the launch's first step in the call
  int64_t n_tiles;
  int64_t chain0;  // first chain of the launch (AIES half)
  int aies_half;
  void* hsave;
  int64_t hsave_stride;  // elements of acc per workgroup
  NutsState nu;
  // best_logL_grad
  const double* ex_x;
  int64_t ex_pitch;
  double *ex_lp, *ex_g;
  int ex_grad;
};

// ---------------------------------------------------------------------------------------
// Plain spectrum log-likelihood of one chain, computed by the whole workgroup.
// ---------------------------------------------------------------------------------------
// Element (i, c) of a tile's [d][M] FP64 array: the global SoA state (p = base + c0,
// pitch = Np), a caller's array, or the tile's LDS scratch (pitch = M).
struct TView {
  double* p;
  int64_t pitch;
  __device__ __forceinline__ double& operator()(int i, int c) const {
    return p[(int64_t)i * pitch + c];
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// acc + SIGN * sum_{j0 <= j < j1} a(j) b(j), accumulated in ascending j.  The loads of
// eight consecutive terms are issued together (indices clamped into [j0, j1), the clamped
// copies' products masked out), so a long sum waits one memory latency per eight terms
// rather than one per term.
template <int SIGN, class FA, class FB>
__device__ __forceinline__ double dot8(double acc, int j0, int j1, const FA& fa, const FB& fb) {
  for (int jb = j0; jb < j1; jb += 8) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + u < j1 ? jb + u : j1 - 1;
      x[u] = fa(j);
      y[u] = fb(j);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (jb + u < j1) {
        if constexpr (SIGN > 0) acc += x[u] * y[u];
        else acc -= x[u] * y[u];
      }
    }
  }
  return acc;
}

__device__ __forceinline__ void plain_chain(const Target& tg, const TView& X, int c, bool grad,
                                            double* scratch, double* outv, double* outg) {
  const int tid = local_tid(), d = tg.d, nt = tg.n_terms;
  double* tpl = scratch;                  // [kMaxD]
  double* A = tpl + kMaxD;                // [kMaxTerms]
  double* gam = A + kMaxTerms;            // [kMaxTerms]
  double* tht = gam + kMaxTerms;          // [kMaxTerms]
  double* wred = tht + kMaxTerms;         // [kWaves][32]
  if (tid < d) tpl[tid] = (X(tid, c) - tg.pc[tid]) * tg.pis[tid];
  __syncthreads();
  if (tid < nt) {
    double sa = 0, sg = 0, sp = 0;
    for (int i = 0; i < d; ++i) {
      sa += tg.pa[tid * d + i] * tpl[i];
      sg += tg.pg[tid * d + i] * tpl[i];
      sp += tg.pp[tid * d + i] * tpl[i];
    }
    A[tid] = exp(sa);
    gam[tid] = tg.pg0[tid] * exp(sg);
    tht[tid] = tanh(sp);
  }
  __syncthreads();
  double ll = 0, sec[kMaxTerms], sxec[kMaxTerms], ses[kMaxTerms];
#pragma unroll
  for (int m = 0; m < kMaxTerms; ++m) sec[m] = sxec[m] = ses[m] = 0;
  for (int j = tid; j < tg.n_bins; j += kThreads) {
    const double xj = tg.xgrid[j];
    double e[kMaxTerms], co[kMaxTerms], si[kMaxTerms], spec = 0;
#pragma unroll
    for (int m = 0; m < kMaxTerms; ++m) {
      if (m < nt) {
        e[m] = exp(-gam[m] * xj);
        const double arg = 2.0 * 3.141592653589793 * tg.pk[m] * xj + 3.141592653589793 * tht[m];
        sincos(arg, &si[m], &co[m]);
        spec += A[m] * (e[m] * co[m]);
      }
    }
    const double dr = spec - tg.data[j];
    const double r = dr * tg.w2[j];
    ll += dr * r;
    if (grad) {
#pragma unroll
      for (int m = 0; m < kMaxTerms; ++m) {
        if (m < nt) {
          const double ec = e[m] * co[m];
          sec[m] += r * ec;
          sxec[m] += r * xj * ec;
          ses[m] += r * (e[m] * si[m]);
        }
      }
    }
  }
  const int lane = tid & 63, wv = tid >> 6;
  ll = wave_sum(ll);
  if (lane == 0) wred[wv * 32] = ll;
  if (grad) {
#pragma unroll
    for (int m = 0; m < kMaxTerms; ++m) {
      if (m < nt) {
        const double a = wave_sum(sec[m]), b = wave_sum(sxec[m]), c = wave_sum(ses[m]);
        if (lane == 0) {
          wred[wv * 32 + 1 + m] = a;
          wred[wv * 32 + 1 + kMaxTerms + m] = b;
          wred[wv * 32 + 1 + 2 * kMaxTerms + m] = c;
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    double s = wred[0];
    for (int w = 1; w < kWaves; ++w) s += wred[w * 32];
    *outv = -0.5 * s;
  }
  if (grad && tid < d) {
    double dt = 0;
    for (int m = 0; m < nt; ++m) {
      double s1 = 0, s2 = 0, s3 = 0;
      for (int w = 0; w < kWaves; ++w) {
        s1 += wred[w * 32 + 1 + m];
        s2 += wred[w * 32 + 1 + kMaxTerms + m];
        s3 += wred[w * 32 + 1 + 2 * kMaxTerms + m];
      }
      const double ca = s1 * A[m];
      const double cg = -s2 * A[m] * gam[m];
      const double cp = -s3 * A[m] * 3.141592653589793 * (1.0 - tht[m] * tht[m]);
      dt += ca * tg.pa[m * d + tid] + cg * tg.pg[m * d + tid] + cp * tg.pp[m * d + tid];
    }
    outg[tid] = -dt * tg.pis[tid];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Target evaluation for a tile of chains: LPo[c0+c] = log pi(x), GXo = grad_x log pi(x).
// The inbox / intrain flags of every chain stay in LDS (mi) after the call.
// ---------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------
// Lane-group form of the FP64 work around the emulator (d <= kGroupD): chain c of the tile
// is held by the eight consecutive threads 8c .. 8c + 7, thread 8c + i holding component i,
// so sums over components are shuffles inside one wave.  One evaluation's FP64 work (its
// log pi and gradient, the sampler's update and the next proposal's inputs) then runs
// between the two barriers that the emulator needs anyway, instead of as (component,
// chain) loops separated by barriers.  Every sum keeps the component order of the loop
// form.  Shuffles run in control flow that is uniform over a chain's eight threads.
// ---------------------------------------------------------------------------------------
constexpr int kGroupD = 8;

template <class P, int MT>
__device__ __forceinline__ bool group_path(const KArgs& a) {
  using IP = typename InPrec<P>::type;
  return 8 * 16 * MT <= kThreads && a.tg.d <= kGroupD && a.mp.ks1 * IP::KSTEP <= 2 * kGroupD;
}

// A chain's eight threads: gb = 4 * (first lane of the group), the byte index of
// ds_bpermute.
__device__ __forceinline__ int grp_base(int tid) { return (tid & 56) << 2; }

// v of every component of this thread's chain (eight independent lane permutes, issued
// together)
__device__ __forceinline__ void grp_gather(double v, int gb, double (&o)[kGroupD]) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  unsigned l[kGroupD], h[kGroupD];
#pragma unroll
  for (int j = 0; j < kGroupD; ++j) {
    l[j] = (unsigned)__builtin_amdgcn_ds_bpermute(gb + 4 * j, lo);
    h[j] = (unsigned)__builtin_amdgcn_ds_bpermute(gb + 4 * j, hi);
  }
#pragma unroll
  for (int j = 0; j < kGroupD; ++j)
    o[j] = __builtin_bit_cast(double, ((unsigned long long)h[j] << 32) | l[j]);
}

// v of component j (runtime j) of this thread's chain
__device__ __forceinline__ double grp_at(double v, int gb, int j) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(gb + 4 * j, (int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(gb + 4 * j, (int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int grp_and(int b) {
  b &= __shfl_xor(b, 1, 64);
  b &= __shfl_xor(b, 2, 64);
  b &= __shfl_xor(b, 4, 64);
  return b;
}

// Loads in the lane-group code are unconditional, at indices clamped into range, and only
// the arithmetic is masked: a load under a per-lane condition becomes a branch with its own
// wait, and the eight terms of a sum would then run one memory latency apart.
__device__ __forceinline__ int clampd(int v, int d) { return v < d ? v : d - 1; }

// component i of mu + L z
__device__ __forceinline__ double grp_affine(const double* __restrict__ mu,
                                             const double* __restrict__ Lw, int d, int i, int gb,
                                             double z) {
  const int ii = clampd(i, d);
  double zs[kGroupD], l[kGroupD];
#pragma unroll
  for (int j = 0; j < kGroupD; ++j) l[j] = Lw[ii * d + clampd(j, d)];
  const double m = mu[ii];
  grp_gather(z, gb, zs);
  double v = 0;
#pragma unroll
  for (int j = 0; j < kGroupD; ++j)
    if (j <= i && i < d) v += l[j] * zs[j];
  return i < d ? m + v : 0.0;
}

// component i of L^T g
__device__ __forceinline__ double grp_lt(const double* __restrict__ Lw, int d, int i, int gb,
                                         double g) {
  const int ii = clampd(i, d);
  double gs[kGroupD], l[kGroupD];
#pragma unroll
  for (int j = 0; j < kGroupD; ++j) l[j] = Lw[clampd(j, d) * d + ii];
  grp_gather(g, gb, gs);
  double v = 0;
#pragma unroll
  for (int j = 0; j < kGroupD; ++j)
    if (j >= i && j < d) v += l[j] * gs[j];
  return v;
}

// component i of L^{-1}(x - mu) (forward substitution, repeated in each thread of the chain)
__device__ __forceinline__ double grp_whiten(const double* __restrict__ mu,
                                             const double* __restrict__ Lw, int d, int i, int gb,
                                             double x) {
  double xs[kGroupD], z[kGroupD], zi = 0.0;
  grp_gather(x, gb, xs);
#pragma unroll
  for (int k = 0; k < kGroupD; ++k) {
    const double xk = xs[k];
    z[k] = 0.0;
    if (k < d) {
      double r = xk - mu[k];
#pragma unroll
      for (int j = 0; j < kGroupD; ++j)
        if (j < k) r -= Lw[k * d + j] * z[j];
      z[k] = r / Lw[k * d + k];
    }
    if (k == i) zi = z[k];
  }
  return zi;
}

// Emulator input of chain c from its proposal x (component i in this thread): t = (x -
// center) * invscale as B fragments of the input layer (zero for padding chains and
// components), and the chain's in-box / in-training-box flags.
template <class P, int MT>
__device__ __forceinline__ void grp_stage(const KArgs& a, char* smem, int c, int i, bool valid,
                                          double x) {
  using IP = typename InPrec<P>::type;
  constexpr int M = 16 * MT;
  const Target& tg = a.tg;
  const int d = tg.d, ks1 = a.mp.ks1, K1 = ks1 * IP::KSTEP;
  const int ii = clampd(i, d);
  const double ce = tg.in_center[ii], is = tg.in_invscale[ii], lo = tg.lower[ii],
               hi = tg.upper[ii];
  int ib = 1, it = 1;
  double v = 0.0;
  if (valid && i < d) {
    v = (x - ce) * is;
    ib = (x >= lo) & (x <= hi);
  }
  if (tg.plain_mode == 1) {
    const double tlo = tg.train_lo[ii], thi = tg.train_hi[ii];
    if (valid && i < d) it = (x >= tlo) & (x <= thi);
  }
  // the padded input width K1 is at most 16: thread i also clears slot i + 8
  typename IP::T* thf = (typename IP::T*)(smem + a.lds.th);
  if (i < K1) thf[frag_offset<IP>(c, i, ks1)] = (typename IP::T)v;
  if (i + kGroupD < K1) thf[frag_offset<IP>(c, i + kGroupD, ks1)] = (typename IP::T)0.0;
  ib = grp_and(ib);
  it = grp_and(it);
  if (i == 0) {
    int* inbox = (int*)(smem + a.lds.mi);
    inbox[c] = ib;
    inbox[M + c] = tg.plain_mode == 2 ? 0 : it;
  }
}

// No continuation after the evaluation.
struct NoPost {
  template <class... A>
  __device__ __forceinline__ void operator()(const A&...) const {}
};

// A continuation written for the wide lane groups (arrays of a thread's two components);
// eval_tile compiles its wide branch only for these and for NoPost.
template <class L>
struct WidePost {
  L f;
  template <class... A>
  __device__ __forceinline__ void operator()(const A&... x) const {
    f(x...);
  }
};
template <class T>
struct IsWidePost {
  static constexpr bool value = false;
};
template <class L>
struct IsWidePost<WidePost<L>> {
  static constexpr bool value = true;
};
template <>
struct IsWidePost<NoPost> {
  static constexpr bool value = true;
};

// ---------------------------------------------------------------------------------------
// Wide lane groups for 8 < d <= 32 on 32-chain tiles (the width of the 1024-wide networks):
// sixteen threads per chain, thread 16c + i holding components i and i + 16, sums over the
// components as blocked in-wave permutes in the component order of the loop form.  Only
// the 32-chain kernels compile this form: its registers would make the 16-chain kernels
// spill.
// ---------------------------------------------------------------------------------------
constexpr int kGroupW = 32;  // largest d on the wide lane-group path

template <int MT>
constexpr bool kWide = MT == 2;

template <class P, int MT>
__device__ __forceinline__ bool wide_path(const KArgs& a) {
  using IP = typename InPrec<P>::type;
  const int d = a.tg.d, K1 = a.mp.ks1 * IP::KSTEP;
  return kWide<MT> && d > kGroupD && d <= kGroupW && K1 <= kGroupW && 16 * 16 * MT <= kThreads;
}

// gb = 4 * (first lane of this thread's chain), the byte index of ds_bpermute
template <int G>
__device__ __forceinline__ int gw_base(int tid) {
  return (tid & (64 - G)) << 2;
}

// every component of this thread's chain: o[j + G u] = v[u] of the chain's thread j (eight
// or sixteen independent lane permutes per value, issued together)
template <int G, int V>
__device__ __forceinline__ void gw_gather(const double (&v)[V], int gb, double (&o)[G * V]) {
  unsigned l[G * V], h[G * V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v[u]);
    const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      l[j + G * u] = (unsigned)__builtin_amdgcn_ds_bpermute(gb + 4 * j, lo);
      h[j + G * u] = (unsigned)__builtin_amdgcn_ds_bpermute(gb + 4 * j, hi);
    }
  }
#pragma unroll
  for (int n = 0; n < G * V; ++n)
    o[n] = __builtin_bit_cast(double, ((unsigned long long)h[n] << 32) | l[n]);
}

// component j of the chain (j the same in all of its threads)
template <int G, int V>
__device__ __forceinline__ double gw_at(const double (&v)[V], int gb, int j) {
  double src = v[0];
#pragma unroll
  for (int u = 1; u < V; ++u)
    if (j >= G * u) src = v[u];
  const unsigned long long b = __builtin_bit_cast(unsigned long long, src);
  const int idx = gb + 4 * (j % G);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(idx, (int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(idx, (int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// components jb .. jb + 7 of this thread's chain (jb a multiple of 8, the same in all of the
// chain's threads)
template <int G, int V>
__device__ __forceinline__ void gw_block(const double (&v)[V], int gb, int jb, double (&o)[8]) {
  double src = v[0];
#pragma unroll
  for (int u = 1; u < V; ++u)
    if (jb >= G * u) src = v[u];
  const unsigned long long b = __builtin_bit_cast(unsigned long long, src);
  const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32), base = gb + 4 * (jb % G);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const unsigned l = (unsigned)__builtin_amdgcn_ds_bpermute(base + 4 * u, lo);
    const unsigned h = (unsigned)__builtin_amdgcn_ds_bpermute(base + 4 * u, hi);
    o[u] = __builtin_bit_cast(double, ((unsigned long long)h << 32) | l);
  }
}

// acc + SIGN * sum_{j0 <= j < j1} coef(j) w_j, w_j component j of this chain's v; ascending
// j, eight components (permutes and coefficient loads) at a time.  j0 and j1 may differ
// between the chain's threads; the blocks run up to d in all of them (the permutes read
// the other threads' registers).
template <int SIGN, int G, int V, class F>
__device__ __forceinline__ double gw_dotc(double acc, int j0, int j1, int d, const F& coef,
                                           const double (&v)[V], int gb) {
#pragma unroll
  for (int jb = 0; jb < G * V; jb += 8) {
    if (jb >= d) break;
    double w[8], cf[8];
    gw_block<G, V>(v, gb, jb, w);
#pragma unroll
    for (int u = 0; u < 8; ++u) cf[u] = coef(jb + u);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (jb + u >= j0 && jb + u < j1) {
        if constexpr (SIGN > 0) acc += cf[u] * w[u];
        else acc -= cf[u] * w[u];
      }
    }
  }
  return acc;
}

// acc + sum_{j < d} x_j^2 over this chain's components, ascending j
template <int G, int V>
__device__ __forceinline__ double gw_sumsq(double acc, int d, const double (&x)[V], int gb) {
#pragma unroll
  for (int jb = 0; jb < G * V; jb += 8) {
    if (jb >= d) break;
    double w[8];
    gw_block<G, V>(x, gb, jb, w);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (jb + u < d) acc += w[u] * w[u];
  }
  return acc;
}

// acc + sum_{j < d} x_j y_j over this chain's components, ascending j
template <int G, int V>
__device__ __forceinline__ double gw_dotv(double acc, int d, const double (&x)[V],
                                           const double (&y)[V], int gb) {
#pragma unroll
  for (int jb = 0; jb < G * V; jb += 8) {
    if (jb >= d) break;
    double wx[8], wy[8];
    gw_block<G, V>(x, gb, jb, wx);
    gw_block<G, V>(y, gb, jb, wy);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (jb + u < d) acc += wx[u] * wy[u];
  }
  return acc;
}

template <int G>
__device__ __forceinline__ int gw_and(int b) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) b &= __shfl_xor(b, o, 64);
  return b;
}


// this thread's components of mu + L z
template <int G, int V>
__device__ __forceinline__ void gw_affine(const double* __restrict__ mu,
                                           const double* __restrict__ Lw, int d, int i, int gb,
                                           const double (&z)[V], double (&x)[V]) {
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int k = i + G * u, kk = clampd(k, d);
    const double m = mu[kk];
    const double v = gw_dotc<1, G, V>(0.0, 0, k < d ? k + 1 : 0, d,
                                       [&](int j) { return Lw[kk * d + clampd(j, d)]; }, z, gb);
    x[u] = k < d ? m + v : 0.0;
  }
}

// this thread's components of L^T g
template <int G, int V>
__device__ __forceinline__ void gw_lt(const double* __restrict__ Lw, int d, int i, int gb,
                                       const double (&g)[V], double (&o)[V]) {
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int k = i + G * u, kk = clampd(k, d);
    o[u] = gw_dotc<1, G, V>(0.0, k, d, d, [&](int j) { return Lw[clampd(j, d) * d + kk]; }, g,
                             gb);
  }
}

// this thread's components of L^{-1}(x - mu), by forward substitution in the component order
// of the loop form: with one component per thread every thread repeats the whole
// substitution; with two, component k is final once the terms of components < k are
// removed, its thread divides, and every thread of the chain removes its term
template <int G, int V>
__device__ __forceinline__ void gw_whiten(const double* __restrict__ mu,
                                           const double* __restrict__ Lw, int d, int i, int gb,
                                           const double (&x)[V], double (&zo)[V]) {
  if constexpr (V == 1) {
    double xs[G], z[G], zi = 0.0;
    gw_gather<G, 1>(x, gb, xs);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      z[k] = 0.0;
      if (k < d) {
        double r = xs[k] - mu[k];
#pragma unroll
        for (int j = 0; j < G; ++j)
          if (j < k) r -= Lw[k * d + j] * z[j];
        z[k] = r / Lw[k * d + k];
      }
      if (k == i) zi = z[k];
    }
    zo[0] = zi;
  } else {
    double r[V];
    int kk[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      kk[u] = clampd(i + G * u, d);
      r[u] = x[u] - mu[kk[u]];
      zo[u] = 0.0;
    }
    for (int k = 0; k < d; ++k) {
      const int ku = k / G, kl = k % G;
      double lk[V];
#pragma unroll
      for (int u = 0; u < V; ++u) lk[u] = Lw[kk[u] * d + k];
      const double dk = Lw[k * d + k];
#pragma unroll
      for (int u = 0; u < V; ++u)
        if (u == ku && i == kl) zo[u] = r[u] / dk;
      const double zk = gw_at<G, V>(zo, gb, k);
#pragma unroll
      for (int u = 0; u < V; ++u)
        if (i + G * u > k && i + G * u < d) r[u] -= lk[u] * zk;
    }
  }
}

// Emulator input of chain c from its proposal x (this thread's components): t = (x -
// center) * invscale as B fragments of the input layer (zero for padding chains and
// components), and the chain's in-box / in-training-box flags.  The padded input width is
// at most 2 G, so this thread writes slots i and i + G.
template <class P, int MT, int G, int V>
__device__ __forceinline__ void gw_stage(const KArgs& a, char* smem, int c, int i, bool valid,
                                          const double (&x)[V]) {
  using IP = typename InPrec<P>::type;
  constexpr int M = 16 * MT;
  const Target& tg = a.tg;
  const int d = tg.d, ks1 = a.mp.ks1, K1 = ks1 * IP::KSTEP;
  typename IP::T* thf = (typename IP::T*)(smem + a.lds.th);
  int ib = 1, it = 1;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = i + G * u, kk = clampd(k, d);
    const double ce = tg.in_center[kk], is = tg.in_invscale[kk], lo = tg.lower[kk],
                 hi = tg.upper[kk];
    const double xu = u < V ? x[u < V ? u : 0] : 0.0;
    const bool act = u < V && valid && k < d;
    double v = 0.0;
    if (act) {
      v = (xu - ce) * is;
      ib &= (xu >= lo) & (xu <= hi);
    }
    if (tg.plain_mode == 1) {
      const double tlo = tg.train_lo[kk], thi = tg.train_hi[kk];
      if (act) it &= (xu >= tlo) & (xu <= thi);
    }
    if (k < K1) thf[frag_offset<IP>(c, k, ks1)] = (typename IP::T)v;
  }
  ib = gw_and<G>(ib);
  it = gw_and<G>(it);
  if (i == 0) {
    int* inbox = (int*)(smem + a.lds.mi);
    inbox[c] = ib;
    inbox[M + c] = tg.plain_mode == 2 ? 0 : it;
  }
}

// Wide lane-group form of the target evaluation (see eval_tile): log pi and its gradient of the
// tile's chains from X, then post(c, i, valid, x, g, log pi) in every thread of the chains
// (x and g this thread's components of the point and of grad_x log pi, g = 0 without grad).
template <class P, int MT, int G, int V, class Post>
__device__ __forceinline__ void gw_eval(const KArgs& a, const MlpSmem<P>& s, const TView& X,
                                         int mv, double* LPo, const TView& GXo, bool grad,
                                         bool box, const double* pv, const double* pgr,
                                         const int* inbox, const int* intrain,
                                         const Post& post) {
  constexpr int M = 16 * MT, N = G * V;
  const Target& tg = a.tg;
  const int tid = local_tid(), d = tg.d;
  if (tid >= G * M) return;
  const int c = tid / G, i = tid % G, gb = gw_base<G>(tid), cc = clampd(c, mv);
  const bool valid = c < mv;
  double x[V];
  int kk[V];
  bool act[V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    kk[u] = clampd(i + G * u, d);
    act[u] = valid && i + G * u < d;
    const double xr = X(kk[u], cc);
    x[u] = act[u] ? xr : 0.0;
  }
  const bool use_mlp = tg.plain_mode == 0 || (tg.plain_mode == 1 && intrain[c]);
  const int ib = inbox[c];
  double lp = tg.offset, PRv[V];
#pragma unroll
  for (int u = 0; u < V; ++u) PRv[u] = 0.0;
  if (tg.gauss_coef != 0.0) {
    double R[V];
    const double xu = tg.tw_v >= 0 ? gw_at<G, V>(x, gb, tg.tw_u) : 0.0;
#pragma unroll
    for (int u = 0; u < V; ++u) {
      double y = x[u];
      if (tg.tw_v >= 0 && i + G * u == tg.tw_v) {
        const double du = xu - tg.tw_center;
        y = y + tg.tw_beta * (du * du - tg.tw_kappa);
      }
      const double gm = tg.gmean[kk[u]];
      R[u] = act[u] ? y - gm : 0.0;
    }
    double q = 0;
    if constexpr (V == 1) {
      // one component per thread: R and P R gathered once each
      double Rs[G], Ps[G], pr[G];
#pragma unroll
      for (int j = 0; j < G; ++j) pr[j] = tg.gprec[kk[0] * d + clampd(j, d)];
      gw_gather<G, 1>(R, gb, Rs);
      double v = 0;
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (act[0] && j < d) v += pr[j] * Rs[j];
      PRv[0] = v;
      gw_gather<G, 1>(PRv, gb, Ps);
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (j < d) q += Rs[j] * Ps[j];
    } else {
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const double v = gw_dotc<1, G, V>(
            0.0, 0, d, d, [&](int j) { return tg.gprec[kk[u] * d + clampd(j, d)]; }, R, gb);
        PRv[u] = act[u] ? v : 0.0;
      }
      q = gw_dotv<G, V>(0.0, d, R, PRv, gb);
    }
    lp += tg.gauss_coef * (-0.5 * q);
  }
  lp += use_mlp ? tg.mlp_coef * (double)s.out[c] : pv[c];
  if (tg.box_penalty) {
    if (!ib) {
      double pen[V], dp;
#pragma unroll
      for (int u = 0; u < V; ++u) pen[u] = act[u] ? box_pen(tg, i + G * u, x[u], &dp) : 0.0;
      lp = gw_dotc<-1, G, V>(lp, 0, d, d, [&](int) { return 1.0; }, pen, gb);
    }
  } else if (box && !ib) {
    lp = -INFINITY;
  }
  if (valid && i == 0) LPo[c] = lp;
  double g[V];
#pragma unroll
  for (int u = 0; u < V; ++u) g[u] = 0.0;
  if (grad) {
    double ptw = 0.0, xtw = 0.0;
    if (tg.gauss_coef != 0.0 && tg.tw_v >= 0) {
      ptw = gw_at<G, V>(PRv, gb, tg.tw_v);
      xtw = gw_at<G, V>(x, gb, tg.tw_u);
    }
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = i + G * u;
      double gu = 0.0;
      if (tg.gauss_coef != 0.0) {
        gu = -PRv[u];
        if (tg.tw_v >= 0 && k == tg.tw_u) {
          const double du = xtw - tg.tw_center;
          gu += -ptw * 2.0 * tg.tw_beta * du;
        }
        gu *= tg.gauss_coef;
      }
      const double gt = (double)s.gth[c * d + kk[u]], is = tg.in_invscale[kk[u]];
      if (act[u]) {
        gu += use_mlp ? tg.mlp_coef * gt * is : pgr[c * d + k];
        if (tg.box_penalty && !ib) {
          double dp;
          box_pen(tg, k, x[u], &dp);
          gu -= dp;
        }
        GXo(k, c) = gu;
        g[u] = gu;
      }
    }
  }
  post(c, i, valid, x, g, lp);
}

// Target evaluation for a tile.  staged: the caller wrote the emulator inputs and flags
// (grp_stage).  On the lane-group path, post(c, i, valid, x_i, g_i, log pi) runs in every
// thread of the tile's chains after log pi and its gradient are written (x_i and g_i this
// thread's components of the point and of grad_x log pi, g_i = 0 without grad), before the
// closing barrier.
template <class P, int MT, class Post>
__device__ __forceinline__ void eval_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                          const TView& X, int mv, double* LPo, const TView& GXo,
                                          bool grad, bool box, bool staged, const Post& post) {
  using acc = typename P::acc;
  using vec = typename P::vec;
  using IP = typename InPrec<P>::type;
  constexpr int M = 16 * MT;
  const Target& tg = a.tg;
  const int tid = local_tid(), d = tg.d;
  const LdsLayout& L = a.lds;
  MlpSmem<P> s = mlp_smem<P, MT>(smem + L.big, a.mp);
  s.thf = (typename IP::T*)(smem + L.th);
  s.gth = (vec*)(smem + L.gth);
  s.red = (acc*)(smem + L.red);
  s.outp = (acc*)(smem + L.outp);
  s.out = (acc*)(smem + L.out);
  s.up = nullptr;
  int* inbox = (int*)(smem + L.mi);
  int* intrain = inbox + M;

  // normalised inputs t = (x - center) * invscale; padding chains and components are 0
  if (!staged) {
    const int K1 = a.mp.ks1 * IP::KSTEP;
    for (int e = tid; e < M * K1; e += kThreads) {
      const int c = e / K1, i = e % K1;
      double v = 0.0;
      if (i < d && c < mv) v = (X(i, c) - tg.in_center[i]) * tg.in_invscale[i];
      store_t<P>(s, a.mp, c, i, v);
    }
    for (int c = tid; c < M; c += kThreads) {
      int ib = 1, it = 1;
      if (c < mv) {
        // in blocks of eight components, loads first (see dot8)
        for (int i0 = 0; i0 < d; i0 += 8) {
          double xv[8], lo[8], hi[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + u < d ? i0 + u : d - 1;
            xv[u] = X(i, c);
            lo[u] = tg.lower[i];
            hi[u] = tg.upper[i];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (i0 + u < d) {
              ib &= (xv[u] >= lo[u]) & (xv[u] <= hi[u]);
              if (tg.plain_mode == 1)
                it &= (xv[u] >= tg.train_lo[i0 + u]) & (xv[u] <= tg.train_hi[i0 + u]);
            }
          }
        }
      }
      inbox[c] = ib;
      intrain[c] = tg.plain_mode == 2 ? 0 : it;
    }
  }

  // the input layer joins the barrier that publishes the inputs and flags
  if (tg.plain_mode != 2) {
    mlp_forward<P, MT>(a.mp, s, hsave, nullptr, grad, true, grad);
    if (grad) mlp_backward<P, MT>(a.mp, s, hsave, nullptr, true, true, true);
  } else {
    __syncthreads();
  }

  // FP64 assembly region (reuses the activation buffers)
  double* R = (double*)(smem + L.big);
  double* PR = R + d * M;
  double* pv = PR + d * M;     // [M]
  double* pgr = pv + M;        // [M][d]
  double* psc = pgr + M * d;   // plain scratch
  if (tg.plain_mode != 0) {
    for (int c = 0; c < mv; ++c) {
      if (!intrain[c]) plain_chain(tg, X, c, grad, psc, pv + c, pgr + c * d);
    }
  }
  if constexpr (kWide<MT> && IsWidePost<Post>::value) {
    if (wide_path<P, MT>(a)) {
      gw_eval<P, MT, 16, 2>(a, s, X, mv, LPo, GXo, grad, box, pv, pgr, inbox, intrain, post);
      __syncthreads();
      return;
    }
  }
  if (group_path<P, MT>(a)) {
    if (tid < 8 * M) {
      const int c = tid >> 3, i = tid & 7, gb = grp_base(tid);
      const int ii = clampd(i, d), cc = clampd(c, mv);
      const bool valid = c < mv, act = valid && i < d;
      const double xr = X(ii, cc);
      const double x = act ? xr : 0.0;
      const bool use_mlp = tg.plain_mode == 0 || (tg.plain_mode == 1 && intrain[c]);
      const int ib = inbox[c];
      double lp = tg.offset, PRi = 0.0;
      if (tg.gauss_coef != 0.0) {
        double y = x;
        if (tg.tw_v >= 0) {
          const double xu = grp_at(x, gb, tg.tw_u);
          if (i == tg.tw_v) {
            const double du = xu - tg.tw_center;
            y = y + tg.tw_beta * (du * du - tg.tw_kappa);
          }
        }
        double pr[kGroupD];
#pragma unroll
        for (int j = 0; j < kGroupD; ++j) pr[j] = tg.gprec[ii * d + clampd(j, d)];
        const double gm = tg.gmean[ii];
        const double R = act ? y - gm : 0.0;
        double Rs[kGroupD], Ps[kGroupD];
        grp_gather(R, gb, Rs);
        double v = 0;
#pragma unroll
        for (int j = 0; j < kGroupD; ++j)
          if (act && j < d) v += pr[j] * Rs[j];
        PRi = v;
        grp_gather(PRi, gb, Ps);
        double q = 0;
#pragma unroll
        for (int j = 0; j < kGroupD; ++j)
          if (j < d) q += Rs[j] * Ps[j];
        lp += tg.gauss_coef * (-0.5 * q);
      }
      lp += use_mlp ? tg.mlp_coef * (double)s.out[c] : pv[c];
      if (tg.box_penalty) {
        if (!ib) {
          double dp, ps[kGroupD];
          grp_gather(act ? box_pen(tg, i, x, &dp) : 0.0, gb, ps);
#pragma unroll
          for (int j = 0; j < kGroupD; ++j)
            if (j < d) lp -= ps[j];
        }
      } else if (box && !ib) {
        lp = -INFINITY;
      }
      if (valid && i == 0) LPo[c] = lp;
      double g = 0.0;
      if (grad) {
        if (tg.gauss_coef != 0.0) {
          g = -PRi;
          if (tg.tw_v >= 0) {
            const double pv_ = grp_at(PRi, gb, tg.tw_v), xu = grp_at(x, gb, tg.tw_u);
            if (i == tg.tw_u) {
              const double du = xu - tg.tw_center;
              g += -pv_ * 2.0 * tg.tw_beta * du;
            }
          }
          g *= tg.gauss_coef;
        }
        const double gt = (double)s.gth[c * d + ii], is = tg.in_invscale[ii];
        if (act) {
          g += use_mlp ? tg.mlp_coef * gt * is : pgr[c * d + i];
          if (tg.box_penalty && !ib) {
            double dp;
            box_pen(tg, i, x, &dp);
            g -= dp;
          }
          GXo(i, c) = g;
        } else {
          g = 0.0;
        }
      }
      post(c, i, valid, x, g, lp);
    }
    __syncthreads();
    return;
  }
  if (tg.gauss_coef != 0.0) {
    for (int e = tid; e < d * M; e += kThreads) {
      const int i = e / M, c = e % M;
      double y = 0;
      if (c < mv) {
        y = X(i, c);
        if (i == tg.tw_v) {
          const double du = X(tg.tw_u, c) - tg.tw_center;
          y = y + tg.tw_beta * (du * du - tg.tw_kappa);
        }
      }
      R[e] = y - tg.gmean[i];
    }
    __syncthreads();
    for (int e = tid; e < d * M; e += kThreads) {
      const int i = e / M, c = e % M;
      PR[e] = dot8<1>(0.0, 0, d, [&](int j) { return tg.gprec[i * d + j]; },
                      [&](int j) { return R[j * M + c]; });
    }
    __syncthreads();
  }
  if (tid < mv) {
    const int c = tid;
    double lp = tg.offset;
    if (tg.gauss_coef != 0.0) {
      const double q = dot8<1>(0.0, 0, d, [&](int i) { return R[i * M + c]; },
                               [&](int i) { return PR[i * M + c]; });
      lp += tg.gauss_coef * (-0.5 * q);
    }
    const bool use_mlp = tg.plain_mode == 0 || (tg.plain_mode == 1 && intrain[c]);
    lp += use_mlp ? tg.mlp_coef * (double)s.out[c] : pv[c];
    if (tg.box_penalty) {
      if (!inbox[c]) {
        double dp;
        for (int i = 0; i < d; ++i) lp -= box_pen(tg, i, X(i, c), &dp);
      }
    } else if (box && !inbox[c]) {
      lp = -INFINITY;
    }
    LPo[c] = lp;
  }
  if (grad) {
    for (int e = tid; e < d * M; e += kThreads) {
      const int i = e / M, c = e % M;
      if (c >= mv) continue;
      double gi = 0;
      if (tg.gauss_coef != 0.0) {
        gi = -PR[e];
        if (i == tg.tw_u) {
          const double du = X(tg.tw_u, c) - tg.tw_center;
          gi += -PR[tg.tw_v * M + c] * 2.0 * tg.tw_beta * du;
        }
        gi *= tg.gauss_coef;
      }
      const bool use_mlp = tg.plain_mode == 0 || (tg.plain_mode == 1 && intrain[c]);
      gi += use_mlp ? tg.mlp_coef * (double)s.gth[c * d + i] * tg.in_invscale[i] : pgr[c * d + i];
      if (tg.box_penalty && !inbox[c]) {
        double dp;
        box_pen(tg, i, X(i, c), &dp);
        gi -= dp;
      }
      GXo(i, c) = gi;
    }
  }
  __syncthreads();
}

template <class P, int MT>
__device__ __forceinline__ void eval_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                          const TView& X, int mv, double* LPo, const TView& GXo,
                                          bool grad, bool box) {
  eval_tile<P, MT>(a, smem, hsave, X, mv, LPo, GXo, grad, box, false, NoPost{});
}

// ---------------------------------------------------------------------------------------
// Per-step FP64 scratch of a tile: whitened start z, proposal z' / x' / grad x', momentum q,
// whitened gradients g_z (start) and g_z' (proposal), log pi of the proposal.  In LDS when
// the layout has room (st >= 0), else in the global state arrays.
// ---------------------------------------------------------------------------------------
struct Scratch {
  TView z, zp, xp, gxp, q, gz, gzp;
  double* lpp;
};

template <int MT>
__device__ __forceinline__ Scratch tile_scratch(const KArgs& a, char* smem, int64_t c0) {
  constexpr int M = 16 * MT;
  Scratch T;
  if (a.lds.st >= 0) {
    double* b = generic_ptr((double*)(smem + a.lds.st));
    const int64_t n = (int64_t)a.tg.d * M;
    T.z = TView{b, M};
    T.zp = TView{b + n, M};
    T.xp = TView{b + 2 * n, M};
    T.gxp = TView{b + 3 * n, M};
    T.q = TView{b + 4 * n, M};
    T.gz = TView{b + 5 * n, M};
    T.gzp = TView{b + 6 * n, M};
    T.lpp = b + 7 * n;
  } else {
    const State& S = a.st;
    T.z = TView{S.z + c0, S.Np};
    T.zp = TView{S.zp + c0, S.Np};
    T.xp = TView{S.xp + c0, S.Np};
    T.gxp = TView{S.gxp + c0, S.Np};
    T.q = TView{S.q + c0, S.Np};
    T.gz = TView{S.gz + c0, S.Np};
    T.gzp = TView{S.gzp + c0, S.Np};
    T.lpp = S.lpp + c0;
  }
  return T;
}

// ---------------------------------------------------------------------------------------
// Whitening helpers for a tile (thread per (i, c)); callers synchronise.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void tile_affine(const double* __restrict__ mu,
                                            const double* __restrict__ Lw, int d, int M, int mv,
                                            const TView& Z, const TView& Xo) {
  for (int e = local_tid(); e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    const double v = dot8<1>(0.0, 0, i + 1, [&](int j) { return Lw[i * d + j]; },
                             [&](int j) { return Z(j, c); });
    Xo(i, c) = mu[i] + v;
  }
}

// z = L^{-1}(x - mu) for the tile's chains (forward substitution, one thread per chain).
// Every MH / MALA / HMC step starts from the whitened coordinates of the stored x, so a
// chain's state is exactly (x, log pi, grad log pi) and a restored state continues
// bit-for-bit.
__device__ __forceinline__ void tile_whiten(const double* __restrict__ mu,
                                            const double* __restrict__ Lw, int d, int mv,
                                            const TView& X, const TView& Z) {
  const int c = local_tid();
  if (c < mv) {
    for (int i = 0; i < d; ++i) {
      const double r = dot8<-1>(X(i, c) - mu[i], 0, i, [&](int j) { return Lw[i * d + j]; },
                                [&](int j) { return Z(j, c); });
      Z(i, c) = r / Lw[i * d + i];
    }
  }
  __syncthreads();
}

// (L^T g)_i = sum_{j >= i} L[j][i] g_j for chain c
__device__ __forceinline__ double lt_dot(const double* __restrict__ Lw, int d, int i,
                                         const TView& G, int c) {
  return dot8<1>(0.0, i, d, [&](int j) { return Lw[j * d + i]; }, [&](int j) { return G(j, c); });
}

__device__ __forceinline__ double accept_prob(double la) {
  return isnan(la) ? 0.0 : exp(fmin(0.0, la));
}

// Per-chain statistics of a launch, kept in the registers of the thread that owns the chain
// (thread c of the tile for chain c0 + c in every step) and added to the state at the end.
struct Tally {
  uint32_t acc, nonfinite, oob;
  double sum_prob, last_prob;
};

__device__ __forceinline__ void flush_tally(const State& S, int64_t ch, const Tally& ty) {
  S.n_acc[ch] += ty.acc;
  S.n_nonfinite[ch] += ty.nonfinite;
  S.n_oob[ch] += ty.oob;
  S.sum_prob[ch] += ty.sum_prob;
  S.step_prob[ch] = ty.last_prob;
}

// Accept bookkeeping for chain ch of the tile (called by one thread per chain).
__device__ __forceinline__ bool decide(const KArgs& a, Tally& ty, int64_t ch, uint64_t t,
                                       uint32_t sub, double la, double lpp, int inbox) {
  const double u = accept_uniform(a.rng, ch, t, sub);
  const bool acc = log(u) < la;
  const double pr = accept_prob(la);
  ty.acc += acc ? 1u : 0u;
  ty.sum_prob += pr;
  ty.last_prob = pr;
  ty.nonfinite += isnan(lpp) ? 1u : 0u;
  ty.oob += inbox ? 0u : 1u;
  return acc;
}

__device__ __forceinline__ void record_tile(const KArgs& a, int s, int d, int M, int mv,
                                            int64_t c0) {
  const int64_t sc = a.rec_s0 + s + 1;
  if (!a.record || (sc % a.thin) != 0) return;
  const int64_t slot = sc / a.thin - 1;
  if (slot >= a.rec_cap) return;
  const State& S = a.st;
  for (int e = local_tid(); e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    a.record[(slot * d + i) * a.rec_pitch + c0 + c] = (float)S.x[i * S.Np + c0 + c];
  }
}

// Copy the proposal into the chain state for accepted chains (flag in LDS).
__device__ __forceinline__ void commit_tile(const State& S, const Scratch& T, const int* flag,
                                            int d, int M, int mv, int64_t c0, bool with_g) {
  for (int e = local_tid(); e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv || !flag[c]) continue;
    const int64_t o = i * S.Np + c0 + c;
    S.x[o] = T.xp(i, c);
    if (with_g) S.gx[o] = T.gxp(i, c);
  }
}

// ---------------------------------------------------------------------------------------
// Transitions for one tile at global step t.
// ---------------------------------------------------------------------------------------
template <class P, int MT>
__device__ __forceinline__ void mh_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                        Tally& ty, int64_t c0, int mv, uint64_t t) {
  constexpr int M = 16 * MT;
  const State& S = a.st;
  const int d = a.tg.d, tid = local_tid();
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  int* inbox = (int*)(smem + a.lds.mi);
  int* flag = inbox + 2 * M;
  tile_whiten(a.wh.mu, a.wh.L, d, mv, TView{S.x + c0, S.Np}, T.z);
  for (int e = tid; e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    const double s = a.step_mult ? a.mh_scale * a.step_mult[i] : a.mh_scale;
    T.zp(i, c) = T.z(i, c) + s * normal_dim(a.rng, c0 + c, t, kStreamNormal, 0, i);
  }
  __syncthreads();
  tile_affine(a.wh.mu, a.wh.L, d, M, mv, T.zp, T.xp);
  __syncthreads();
  eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, false, true);
  if (tid < mv) {
    const int64_t ch = c0 + tid;
    const double lpp = T.lpp[tid];
    const double la = lpp - S.lp[ch];
    const bool acc = decide(a, ty, ch, t, 0, la, lpp, inbox[tid]);
    flag[tid] = acc;
    if (acc) S.lp[ch] = lpp;
  }
  __syncthreads();
  commit_tile(S, T, flag, d, M, mv, c0, false);
  __syncthreads();
}

// MALA on wide lane groups (the expressions of the loop form in mala_tile, in their order):
// whitening, drift and noise and the proposal here; reverse drift, acceptance and commit in
// the evaluation's continuation.  The chain's tally lives in thread G c.
template <class P, int MT, int G, int V>
__device__ __forceinline__ void mala_gw(const KArgs& a, char* smem, typename P::acc* hsave,
                                         Tally& ty, int64_t c0, int mv, uint64_t t, double eps) {
  constexpr int M = 16 * MT, N = G * V;
  const State& S = a.st;
  const int d = a.tg.d, tid = local_tid();
  const double* Lw = a.wh.L;
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  const TView GX{S.gx + c0, S.Np};
  const int* inbox = (const int*)(smem + a.lds.mi);
  const double* mult = a.step_mult;
  const double sq = sqrt(2.0 * eps);
  if (tid < G * M) {
    const int c = tid / G, i = tid % G, gb = gw_base<G>(tid), cc = clampd(c, mv);
    const bool valid = c < mv;
    double x[V], gx[V], z[V], gz[V], zp[V], xp[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int kk = clampd(i + G * u, d);
      const bool act = valid && i + G * u < d;
      const double xr = S.x[kk * S.Np + c0 + cc], gr = GX(kk, cc);
      x[u] = act ? xr : 0.0;
      gx[u] = act ? gr : 0.0;
    }
    gw_whiten<G, V>(a.wh.mu, Lw, d, i, gb, x, z);
    gw_lt<G, V>(Lw, d, i, gb, gx, gz);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = i + G * u;
      zp[u] = 0.0;
      if (valid && k < d) {
        const double ei = mult ? eps * mult[k] : eps, sqi = mult ? sqrt(2.0 * ei) : sq;
        zp[u] = z[u] + ei * gz[u] + sqi * normal_dim(a.rng, c0 + c, t, kStreamNormal, 0, k);
        T.z(k, c) = z[u];
        T.gz(k, c) = gz[u];
        T.zp(k, c) = zp[u];
      }
    }
    gw_affine<G, V>(a.wh.mu, Lw, d, i, gb, zp, xp);
#pragma unroll
    for (int u = 0; u < V; ++u)
      if (valid && i + G * u < d) T.xp(i + G * u, c) = xp[u];
    gw_stage<P, MT, G, V>(a, smem, c, i, valid, xp);
  }
  // eval_tile instantiates both lane-group forms; only the one with this V runs
  auto post = [&](int c, int i, bool valid, const auto& x, const auto& g, double lp) {
    if constexpr (sizeof(x) == V * sizeof(double)) {
    const int gb = gw_base<G>(local_tid()), cc = clampd(c, mv);
    double gzp[V], df[V], dr[V], ei[V], zr[V], zpr[V], gzr[V];
    // the scratch loads first: their latency overlaps the permutes of L^T g
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int kk = clampd(i + G * u, d);
      zr[u] = T.z(kk, cc);
      zpr[u] = T.zp(kk, cc);
      gzr[u] = T.gz(kk, cc);
      ei[u] = mult ? eps * mult[kk] : eps;
    }
    gw_lt<G, V>(Lw, d, i, gb, g, gzp);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      df[u] = dr[u] = 0.0;
      if (valid && i + G * u < d) {
        df[u] = zpr[u] - zr[u] - ei[u] * gzr[u];
        dr[u] = zr[u] - zpr[u] - ei[u] * gzp[u];
      }
    }
    double fwd = 0, rev = 0;
    if (mult) {
#pragma unroll
      for (int jb = 0; jb < N; jb += 8) {
        if (jb >= d) break;
        double dfs[8], drs[8], es[8];
        gw_block<G, V>(df, gb, jb, dfs);
        gw_block<G, V>(dr, gb, jb, drs);
        gw_block<G, V>(ei, gb, jb, es);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (jb + u < d) {
            fwd += dfs[u] * dfs[u] / (4.0 * es[u]);
            rev += drs[u] * drs[u] / (4.0 * es[u]);
          }
        }
      }
    } else {
      if constexpr (V == 1) {
        double dfs[G], drs[G];
        gw_gather<G, 1>(df, gb, dfs);
        gw_gather<G, 1>(dr, gb, drs);
#pragma unroll
        for (int j = 0; j < G; ++j) {
          if (j < d) {
            fwd += dfs[j] * dfs[j];
            rev += drs[j] * drs[j];
          }
        }
      } else {
        fwd = gw_sumsq<G, V>(0.0, d, df, gb);
        rev = gw_sumsq<G, V>(0.0, d, dr, gb);
      }
      fwd /= 4.0 * eps;
      rev /= 4.0 * eps;
    }
    int acc = 0;
    if (valid && i == 0) {
      const int64_t ch = c0 + c;
      const double la = lp - S.lp[ch] + (-rev) - (-fwd);
      acc = decide(a, ty, ch, t, 0, la, lp, inbox[c]) ? 1 : 0;
      if (acc) S.lp[ch] = lp;
    }
    acc = __builtin_amdgcn_ds_bpermute(gb, acc);  // chain c's decision, from thread G c
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = i + G * u;
      if (acc && valid && k < d) {
        S.x[k * S.Np + c0 + c] = x[u];
        S.gx[k * S.Np + c0 + c] = g[u];
      }
    }
    }
  };
  eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, true, true, true,
                   WidePost<decltype(post)>{post});
}

// HMC on wide lane groups (the expressions of the loop form in hmc_tile, in their order): start,
// first half kick and drift and the first proposal here; each evaluation's closing half
// kick, the next half kick, drift and proposal, or after the last one accept / reject and
// commit, in the evaluation's continuation.  The chain's tally lives in thread G c.
template <class P, int MT, int G, int V>
__device__ __forceinline__ void hmc_gw(const KArgs& a, char* smem, typename P::acc* hsave,
                                        Tally& ty, int64_t c0, int mv, uint64_t t, double eps) {
  constexpr int M = 16 * MT, N = G * V;
  const State& S = a.st;
  const int d = a.tg.d, tid = local_tid();
  const double* Lw = a.wh.L;
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  const TView GX{S.gx + c0, S.Np};
  const int* inbox = (const int*)(smem + a.lds.mi);
  double* h0 = (double*)(smem + a.lds.md);
  const double he = 0.5 * eps;
  if (tid < G * M) {
    const int c = tid / G, i = tid % G, gb = gw_base<G>(tid), cc = clampd(c, mv);
    const bool valid = c < mv;
    double x[V], gx[V], z[V], q[V], gz[V], zp[V], xp[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = i + G * u, kk = clampd(k, d);
      const bool act = valid && k < d;
      const double xr = S.x[kk * S.Np + c0 + cc], gr = GX(kk, cc);
      x[u] = act ? xr : 0.0;
      gx[u] = act ? gr : 0.0;
    }
    gw_whiten<G, V>(a.wh.mu, Lw, d, i, gb, x, z);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = i + G * u;
      q[u] = (valid && k < d) ? normal_dim(a.rng, c0 + c, t, kStreamNormal, 0, k) : 0.0;
    }
    const double ke = gw_sumsq<G, V>(0.0, d, q, gb);
    gw_lt<G, V>(Lw, d, i, gb, gx, gz);
    double qh[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      qh[u] = q[u] + he * gz[u];
      zp[u] = z[u] + eps * qh[u];
    }
    gw_affine<G, V>(a.wh.mu, Lw, d, i, gb, zp, xp);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = i + G * u;
      if (valid && k < d) {
        T.q(k, c) = qh[u];
        T.zp(k, c) = zp[u];
        T.xp(k, c) = xp[u];
      }
    }
    if (valid && i == 0) h0[c] = -S.lp[c0 + c] + 0.5 * ke;
    gw_stage<P, MT, G, V>(a, smem, c, i, valid, xp);
  }
  for (int l = 0; l < a.n_leap; ++l) {
    const bool last = l + 1 == a.n_leap;
    // eval_tile instantiates both lane-group forms; only the one with this V runs
    auto post = [&](int c, int i, bool valid, const auto& x, const auto& g, double lp) {
      if constexpr (sizeof(x) == V * sizeof(double)) {
      const int gb = gw_base<G>(local_tid()), cc = clampd(c, mv);
      double qr[V], zr[V], gz[V], q[V];
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const int kk = clampd(i + G * u, d);
        qr[u] = T.q(kk, cc);
        zr[u] = T.zp(kk, cc);
      }
      gw_lt<G, V>(Lw, d, i, gb, g, gz);
#pragma unroll
      for (int u = 0; u < V; ++u) q[u] = ((valid && i + G * u < d) ? qr[u] : 0.0) + he * gz[u];
      if (!last) {
        double zp[V], xp[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const double qh = q[u] + he * gz[u];
          q[u] = qh;
          zp[u] = ((valid && i + G * u < d) ? zr[u] : 0.0) + eps * qh;
        }
        gw_affine<G, V>(a.wh.mu, Lw, d, i, gb, zp, xp);
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int k = i + G * u;
          if (valid && k < d) {
            T.q(k, c) = q[u];
            T.zp(k, c) = zp[u];
            T.xp(k, c) = xp[u];
          }
        }
        gw_stage<P, MT, G, V>(a, smem, c, i, valid, xp);
        return;
      }
      const double ke = gw_sumsq<G, V>(0.0, d, q, gb);
      int acc = 0;
      if (valid && i == 0) {
        const int64_t ch = c0 + c;
        const double lp1 = (inbox[c] || a.tg.box_penalty) ? lp : -INFINITY;
        const double h1 = -lp1 + 0.5 * ke;
        const double la = h0[c] - h1;
        acc = decide(a, ty, ch, t, 0, la, lp1, inbox[c]) ? 1 : 0;
        if (acc) S.lp[ch] = lp1;
      }
      acc = __builtin_amdgcn_ds_bpermute(gb, acc);  // chain c's decision, from thread G c
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const int k = i + G * u;
        if (acc && valid && k < d) {
          S.x[k * S.Np + c0 + c] = x[u];
          S.gx[k * S.Np + c0 + c] = g[u];
        }
      }
      }
    };
    eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, true, false, true,
                     WidePost<decltype(post)>{post});
  }
}

template <class P, int MT>
__device__ __forceinline__ void mala_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                          Tally& ty, int64_t c0, int mv, uint64_t t, double eps) {
  constexpr int M = 16 * MT;
  const State& S = a.st;
  const int d = a.tg.d, tid = local_tid();
  const double* Lw = a.wh.L;
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  const TView GX{S.gx + c0, S.Np};
  int* inbox = (int*)(smem + a.lds.mi);
  int* flag = inbox + 2 * M;
  const double* mult = a.step_mult;  // per-dimension steps eps_i = eps m_i when set
  const double sq = sqrt(2.0 * eps);
  if constexpr (kWide<MT>) {
    if (wide_path<P, MT>(a)) {
      mala_gw<P, MT, 16, 2>(a, smem, hsave, ty, c0, mv, t, eps);
      return;
    }
  }
  if (group_path<P, MT>(a)) {
    // lane groups (the expressions of the loop form below, in their order): whitening,
    // drift and noise and the proposal here; reverse drift, acceptance and commit in the
    // evaluation's continuation.  The chain's tally lives in thread 8c.
    if (tid < 8 * M) {
      const int c = tid >> 3, i = tid & 7, gb = grp_base(tid);
      const int ii = clampd(i, d), cc = clampd(c, mv);
      const bool valid = c < mv, act = valid && i < d;
      const double xr = S.x[ii * S.Np + c0 + cc], gr = GX(ii, cc);
      const double x = act ? xr : 0.0;
      const double z = grp_whiten(a.wh.mu, Lw, d, i, gb, x);
      const double gz = grp_lt(Lw, d, i, gb, act ? gr : 0.0);
      double zp = 0.0;
      if (act) {
        const double ei = mult ? eps * mult[i] : eps, sqi = mult ? sqrt(2.0 * ei) : sq;
        zp = z + ei * gz + sqi * normal_dim(a.rng, c0 + c, t, kStreamNormal, 0, i);
        T.z(i, c) = z;
        T.gz(i, c) = gz;
        T.zp(i, c) = zp;
      }
      const double xp = grp_affine(a.wh.mu, Lw, d, i, gb, zp);
      if (act) T.xp(i, c) = xp;
      grp_stage<P, MT>(a, smem, c, i, valid, xp);
    }
    auto post = [&](int c, int i, bool valid, double x, double g, double lp) {
      const bool act = valid && i < d;
      const int gb = grp_base(local_tid()), ii = clampd(i, d), cc = clampd(c, mv);
      const double zr = T.z(ii, cc), zpr = T.zp(ii, cc), gzr = T.gz(ii, cc);
      const double gzp = grp_lt(Lw, d, i, gb, g);
      const double ei = mult ? eps * mult[ii] : eps;
      double df = 0.0, dr = 0.0;
      if (act) {
        df = zpr - zr - ei * gzr;
        dr = zr - zpr - ei * gzp;
      }
      double fwd = 0, rev = 0, dfs[kGroupD], drs[kGroupD];
      grp_gather(df, gb, dfs);
      grp_gather(dr, gb, drs);
      if (mult) {
        double es[kGroupD];
        grp_gather(ei, gb, es);
#pragma unroll
        for (int j = 0; j < kGroupD; ++j) {
          if (j < d) {
            fwd += dfs[j] * dfs[j] / (4.0 * es[j]);
            rev += drs[j] * drs[j] / (4.0 * es[j]);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < kGroupD; ++j) {
          if (j < d) {
            fwd += dfs[j] * dfs[j];
            rev += drs[j] * drs[j];
          }
        }
        fwd /= 4.0 * eps;
        rev /= 4.0 * eps;
      }
      int acc = 0;
      if (valid && i == 0) {
        const int64_t ch = c0 + c;
        const double la = lp - S.lp[ch] + (-rev) - (-fwd);
        acc = decide(a, ty, ch, t, 0, la, lp, inbox[c]) ? 1 : 0;
        if (acc) S.lp[ch] = lp;
      }
      acc = __builtin_amdgcn_ds_bpermute(gb, acc);  // chain c's decision, from thread 8c
      if (acc && act) {
        S.x[i * S.Np + c0 + c] = x;
        S.gx[i * S.Np + c0 + c] = g;
      }
    };
    eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, true, true, true, post);
    return;
  }
  tile_whiten(a.wh.mu, Lw, d, mv, TView{S.x + c0, S.Np}, T.z);
  for (int e = tid; e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    const double gzi = lt_dot(Lw, d, i, GX, c);
    const double ei = mult ? eps * mult[i] : eps, sqi = mult ? sqrt(2.0 * ei) : sq;
    T.gz(i, c) = gzi;
    T.zp(i, c) = T.z(i, c) + ei * gzi + sqi * normal_dim(a.rng, c0 + c, t, kStreamNormal, 0, i);
  }
  __syncthreads();
  tile_affine(a.wh.mu, Lw, d, M, mv, T.zp, T.xp);
  __syncthreads();
  eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, true, true);
  for (int e = tid; e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    T.gzp(i, c) = lt_dot(Lw, d, i, T.gxp, c);
  }
  __syncthreads();
  if (tid < mv) {
    const int c = tid;
    const int64_t ch = c0 + c;
    // sums over the components in blocks of eight, loads first (see dot8); with mult the
    // per-dimension terms |.|^2 / (4 eps_i)
    double fwd = 0, rev = 0;
    for (int i0 = 0; i0 < d; i0 += 8) {
      double zp[8], z[8], gz[8], gzp[8], ml[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u < d ? i0 + u : d - 1;
        zp[u] = T.zp(i, c);
        z[u] = T.z(i, c);
        gz[u] = T.gz(i, c);
        gzp[u] = T.gzp(i, c);
        ml[u] = mult ? mult[i] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i0 + u < d) {
          const double ei = mult ? eps * ml[u] : eps;
          const double df = zp[u] - z[u] - ei * gz[u];
          const double dr = z[u] - zp[u] - ei * gzp[u];
          if (mult) {
            fwd += df * df / (4.0 * ei);
            rev += dr * dr / (4.0 * ei);
          } else {
            fwd += df * df;
            rev += dr * dr;
          }
        }
      }
    }
    if (!mult) {
      fwd /= 4.0 * eps;
      rev /= 4.0 * eps;
    }
    const double lpp = T.lpp[c];
    const double la = lpp - S.lp[ch] + (-rev) - (-fwd);
    const bool acc = decide(a, ty, ch, t, 0, la, lpp, inbox[c]);
    flag[c] = acc;
    if (acc) S.lp[ch] = lpp;
  }
  __syncthreads();
  commit_tile(S, T, flag, d, M, mv, c0, true);
  __syncthreads();
}

template <class P, int MT>
__device__ __forceinline__ void hmc_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                         Tally& ty, int64_t c0, int mv, uint64_t t, double eps) {
  constexpr int M = 16 * MT;
  const State& S = a.st;
  const int d = a.tg.d, tid = local_tid();
  const double* Lw = a.wh.L;
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  const TView GX{S.gx + c0, S.Np};
  int* inbox = (int*)(smem + a.lds.mi);
  int* flag = inbox + 2 * M;
  double* h0 = (double*)(smem + a.lds.md);
  const double he = 0.5 * eps;
  if constexpr (kWide<MT>) {
    if (wide_path<P, MT>(a)) {
      hmc_gw<P, MT, 16, 2>(a, smem, hsave, ty, c0, mv, t, eps);
      return;
    }
  }
  if (group_path<P, MT>(a)) {
    // lane groups (the expressions of the loop form below, in their order): start, first
    // half kick and drift and the first proposal here; each evaluation's closing half kick,
    // the next half kick, drift and proposal, or after the last one accept / reject and
    // commit, in the evaluation's continuation.  The chain's tally lives in thread 8c.
    if (tid < 8 * M) {
      const int c = tid >> 3, i = tid & 7, gb = grp_base(tid);
      const int ii = clampd(i, d), cc = clampd(c, mv);
      const bool valid = c < mv, act = valid && i < d;
      const double xr = S.x[ii * S.Np + c0 + cc], gr = GX(ii, cc);
      const double x = act ? xr : 0.0;
      const double z = grp_whiten(a.wh.mu, Lw, d, i, gb, x);
      const double q = act ? normal_dim(a.rng, c0 + c, t, kStreamNormal, 0, i) : 0.0;
      double k = 0, qs[kGroupD];
      grp_gather(q, gb, qs);
#pragma unroll
      for (int j = 0; j < kGroupD; ++j)
        if (j < d) k += qs[j] * qs[j];
      const double gz = grp_lt(Lw, d, i, gb, act ? gr : 0.0);
      const double qh = q + he * gz;
      const double zp = z + eps * qh;
      const double xp = grp_affine(a.wh.mu, Lw, d, i, gb, zp);
      if (act) {
        T.q(i, c) = qh;
        T.zp(i, c) = zp;
        T.xp(i, c) = xp;
      }
      if (valid && i == 0) h0[c] = -S.lp[c0 + c] + 0.5 * k;
      grp_stage<P, MT>(a, smem, c, i, valid, xp);
    }
    for (int l = 0; l < a.n_leap; ++l) {
      const bool last = l + 1 == a.n_leap;
      auto post = [&](int c, int i, bool valid, double x, double g, double lp) {
        const bool act = valid && i < d;
        const int gb = grp_base(local_tid()), ii = clampd(i, d), cc = clampd(c, mv);
        const double qr = T.q(ii, cc), zr = T.zp(ii, cc);
        const double gz = grp_lt(Lw, d, i, gb, g);
        const double q = (act ? qr : 0.0) + he * gz;
        if (!last) {
          const double qh = q + he * gz;
          const double zp = (act ? zr : 0.0) + eps * qh;
          const double xp = grp_affine(a.wh.mu, Lw, d, i, gb, zp);
          if (act) {
            T.q(i, c) = qh;
            T.zp(i, c) = zp;
            T.xp(i, c) = xp;
          }
          grp_stage<P, MT>(a, smem, c, i, valid, xp);
          return;
        }
        double k = 0, qs[kGroupD];
        grp_gather(q, gb, qs);
#pragma unroll
        for (int j = 0; j < kGroupD; ++j)
          if (j < d) k += qs[j] * qs[j];
        int acc = 0;
        if (valid && i == 0) {
          const int64_t ch = c0 + c;
          const double lp1 = (inbox[c] || a.tg.box_penalty) ? lp : -INFINITY;
          const double h1 = -lp1 + 0.5 * k;
          const double la = h0[c] - h1;
          acc = decide(a, ty, ch, t, 0, la, lp1, inbox[c]) ? 1 : 0;
          if (acc) S.lp[ch] = lp1;
        }
        acc = __builtin_amdgcn_ds_bpermute(gb, acc);  // chain c's decision, from thread 8c
        if (acc && act) {
          S.x[i * S.Np + c0 + c] = x;
          S.gx[i * S.Np + c0 + c] = g;
        }
      };
      eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, true, false, true, post);
    }
    return;
  }
  tile_whiten(a.wh.mu, Lw, d, mv, TView{S.x + c0, S.Np}, T.z);
  // momentum, copies of the start point, whitened start gradient
  for (int e = tid; e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    T.q(i, c) = normal_dim(a.rng, c0 + c, t, kStreamNormal, 0, i);
    T.zp(i, c) = T.z(i, c);
    T.gzp(i, c) = lt_dot(Lw, d, i, GX, c);
  }
  __syncthreads();
  if (tid < mv) {
    double k = 0;
    k = dot8<1>(k, 0, d, [&](int i) { return T.q(i, tid); }, [&](int i) { return T.q(i, tid); });
    h0[tid] = -S.lp[c0 + tid] + 0.5 * k;
  }
  __syncthreads();
  for (int l = 0; l < a.n_leap; ++l) {
    for (int e = tid; e < d * M; e += kThreads) {
      const int i = e / M, c = e % M;
      if (c >= mv) continue;
      const double qh = T.q(i, c) + he * T.gzp(i, c);
      T.q(i, c) = qh;
      T.zp(i, c) = T.zp(i, c) + eps * qh;
    }
    __syncthreads();
    tile_affine(a.wh.mu, Lw, d, M, mv, T.zp, T.xp);
    __syncthreads();
    eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, true, false);
    for (int e = tid; e < d * M; e += kThreads) {
      const int i = e / M, c = e % M;
      if (c >= mv) continue;
      const double gzi = lt_dot(Lw, d, i, T.gxp, c);
      T.gzp(i, c) = gzi;
      T.q(i, c) = T.q(i, c) + he * gzi;
    }
    __syncthreads();
  }
  if (tid < mv) {
    const int64_t ch = c0 + tid;
    double k = 0;
    k = dot8<1>(k, 0, d, [&](int i) { return T.q(i, tid); }, [&](int i) { return T.q(i, tid); });
    const double lp1 = (inbox[tid] || a.tg.box_penalty) ? T.lpp[tid] : -INFINITY;
    const double h1 = -lp1 + 0.5 * k;
    const double la = h0[tid] - h1;
    const bool acc = decide(a, ty, ch, t, 0, la, lp1, inbox[tid]);
    flag[tid] = acc;
    if (acc) S.lp[ch] = lp1;
  }
  __syncthreads();
  commit_tile(S, T, flag, d, M, mv, c0, true);
  __syncthreads();
}

// AIES: walkers of the active half [chain0, chain0 + half) against the other half.
template <class P, int MT>
__device__ __forceinline__ void aies_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                          Tally& ty, int64_t c0, int mv, uint64_t t) {
  constexpr int M = 16 * MT;
  const State& S = a.st;
  const int d = a.tg.d, tid = local_tid();
  const int64_t Np = S.Np, half = S.N / 2;
  const int h = a.aies_half;
  const int64_t other = (1 - h) * half;
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  int* inbox = (int*)(smem + a.lds.mi);
  int* flag = inbox + 2 * M;
  double* zz = (double*)(smem + a.lds.md);
  const double av = a.stretch_a;
  for (int e = tid; e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    const int64_t k = c0 + c;
    const U4 b = a.rng.block(k, t, kStreamAies, (uint32_t)h, 0);
    const double ua = u52(b.x, b.y), ub = u52(b.z, b.w);
    int64_t jj = (int64_t)floor(ua * (double)half);
    if (jj > half - 1) jj = half - 1;
    const int64_t j = other + jj;
    const double zr = ((av - 1.0) * ub + 1.0);
    const double z = zr * zr / av;
    if (i == 0) zz[c] = z;
    const double xj = S.x[i * Np + j];
    T.xp(i, c) = xj + z * (S.x[i * Np + k] - xj);
  }
  __syncthreads();
  eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, false, true);
  if (tid < mv) {
    const int64_t k = c0 + tid;
    const double lpp = T.lpp[tid];
    const double la = (double)(d - 1) * log(zz[tid]) + lpp - S.lp[k];
    const bool acc = decide(a, ty, k, t, (uint32_t)h, la, lpp, inbox[tid]);
    flag[tid] = acc;
    if (acc) S.lp[k] = lpp;
  }
  __syncthreads();
  commit_tile(S, T, flag, d, M, mv, c0, false);
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// No-U-Turn sampler (Hoffman & Gelman's efficient slice version) for a tile of chains, in
// the whitened space with identity mass.  The recursive tree build is run iteratively and in
// lockstep over the tile: doubling j appends 2^j leaves on the side v = +-1 drawn for each
// chain; after leaf k, the subtrees that leaf completes (one per trailing one-bit of k) are
// merged with the pending left siblings kept per level.  Chains that stop (U-turn,
// divergence, maximum depth) idle until every chain of the tile has stopped; every leaf is
// one emulator evaluation with gradient.
//
// Per-chain work runs on lane groups: dp = the smallest power of two >= d consecutive lanes
// hold one chain's components (a wave holds 64 / dp chains) and dot products over the
// components are butterfly sums within the group, which leave the identical value in every
// lane of the group, so all of a group's lanes take the same decisions.
//
// Random numbers per step t and chain (Philox counters): momentum normals(stream 1, sub 0);
// slice variable u = the accept uniform (stream 2, sub 0); doubling j: block(stream 5,
// sub j, 0), first uniform < 1/2 -> v = -1 else +1, second uniform decides whether the
// finished subtree's candidate replaces the tree's (iff < n' / n); merging two siblings into
// a subtree of 2^l leaves that ends at leaf k of doubling j: block(stream 5, sub 16 + j,
// 8 k + l), first uniform < n2 / (n1 + n2) takes the second sibling's candidate.
// A leaf outside the prior box has log pi = -inf (never valid, and it stops the trajectory);
// the dynamics use the unbounded gradient, as in the HMC transition.  The acceptance
// statistic for step-size adaptation is the mean of min(1, exp(H0 - H)) over the leaves.
// ---------------------------------------------------------------------------------------
constexpr double kNutsDeltaMax = 1000.0;  // divergence threshold on the energy error

__device__ __forceinline__ double group_sum(double v, int dp) {
  for (int o = dp >> 1; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class P, int MT>
__device__ __forceinline__ void nuts_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                          int64_t c0, int mv, uint64_t t, double eps) {
  constexpr int M = 16 * MT;
  const State& S = a.st;
  const NutsState& U = a.nu;
  const int64_t Np = S.Np;
  const int d = a.tg.d, tid = local_tid();
  const double* Lw = a.wh.L;
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  const TView GX{S.gx + c0, Np};
  int* inbox = (int*)(smem + a.lds.mi);
  int* alive = inbox + 2 * M;
  int* moved = inbox + 3 * M;
  double* md = (double*)(smem + a.lds.md);
  double* h0 = md;              // H(z0, q0)
  double* lslice = md + M;      // log u - H(z0, q0)
  double* nvalid = md + 2 * M;  // valid points of the tree so far
  double* stat = md + 3 * M;    // sum over leaves of min(1, exp(H0 - H))
  double* nleaf = md + 4 * M;   // leaves (evaluations) of the trajectory
  double* dir = md + 5 * M;     // direction of the current doubling
  double* utop = md + 6 * M;    // the doubling's candidate-replacement uniform
  int lg = 0;
  while ((1 << lg) < d) ++lg;
  const int dp = 1 << lg, gi = tid & (dp - 1), gstep = kThreads >> lg;
  const bool on = gi < d;
  auto row = [&](int64_t ch) { return ch * d + gi; };
  auto lvl = [&](int l, int64_t ch) { return ((int64_t)l * Np + ch) * d + gi; };

  tile_whiten(a.wh.mu, Lw, d, mv, TView{S.x + c0, Np}, T.z);
  for (int c = tid >> lg; c < mv; c += gstep) {
    const int64_t ch = c0 + c;
    double q = 0;
    if (on) {
      q = normal_dim(a.rng, ch, t, kStreamNormal, 0, gi);
      const double z = T.z(gi, c), g = lt_dot(Lw, d, gi, GX, c);
      const int64_t o = row(ch);
      U.zm[o] = z;
      U.zpl[o] = z;
      U.qm[o] = q;
      U.qpl[o] = q;
      U.gm[o] = g;
      U.gpl[o] = g;
    }
    const double kin = group_sum(q * q, dp);
    if (gi == 0) {
      const double hh = -S.lp[ch] + 0.5 * kin;
      h0[c] = hh;
      lslice[c] = log(accept_uniform(a.rng, ch, t, 0)) - hh;
      nvalid[c] = 1.0;
      stat[c] = 0.0;
      nleaf[c] = 0.0;
      alive[c] = 1;
      moved[c] = 0;
    }
  }
  for (int c = mv + tid; c < M; c += kThreads) alive[c] = 0;
  __syncthreads();

  bool any = true;
  for (int j = 0; j < U.max_depth && any; ++j) {
    for (int c = tid; c < mv; c += kThreads) {
      if (!alive[c]) continue;
      const U4 b = a.rng.block(c0 + c, t, kStreamNuts, (uint32_t)j, 0);
      dir[c] = u52(b.x, b.y) < 0.5 ? -1.0 : 1.0;
      utop[c] = u52(b.z, b.w);
    }
    __syncthreads();
    const int nk = 1 << j;
    for (int k = 0; k < nk; ++k) {
      // half kick and drift from the tree end on the chain's side
      for (int c = tid >> lg; c < mv; c += gstep) {
        if (!alive[c] || !on) continue;
        const int64_t o = row(c0 + c);
        const double v = dir[c];
        const bool lo = v < 0.0;
        const double qe = lo ? U.qm[o] : U.qpl[o];
        const double ge = lo ? U.gm[o] : U.gpl[o];
        const double ze = lo ? U.zm[o] : U.zpl[o];
        const double qh = qe + (0.5 * v) * eps * ge;
        T.q(gi, c) = qh;
        T.zp(gi, c) = ze + v * eps * qh;
      }
      __syncthreads();
      tile_affine(a.wh.mu, Lw, d, M, mv, T.zp, T.xp);
      __syncthreads();
      eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, true, false);
      // second half kick, the leaf's bookkeeping, subtree merges
      const int nmerge = __builtin_ctz(~(unsigned)k);  // trailing one-bits of k (<= j)
      for (int c = tid >> lg; c < mv; c += gstep) {
        if (!alive[c]) continue;
        const int64_t ch = c0 + c;
        const double v = dir[c];
        const bool lo = v < 0.0;
        double z = 0, q = 0, xl = 0, gxl = 0;
        if (on) {
          const double g = lt_dot(Lw, d, gi, T.gxp, c);
          q = T.q(gi, c) + (0.5 * v) * eps * g;
          z = T.zp(gi, c);
          xl = T.xp(gi, c);
          gxl = T.gxp(gi, c);
          const int64_t o = row(ch);
          (lo ? U.zm : U.zpl)[o] = z;
          (lo ? U.qm : U.qpl)[o] = q;
          (lo ? U.gm : U.gpl)[o] = g;
        }
        const double kin = group_sum(q * q, dp);
        const int ib = inbox[c];
        const double lp = (ib || a.tg.box_penalty) ? T.lpp[c] : -INFINITY;
        const double h = -lp + 0.5 * kin;
        const double ls = lslice[c];
        bool go = ls < -h + kNutsDeltaMax;
        double ncur = (ls <= -h) ? 1.0 : 0.0;
        if (gi == 0) {
          nleaf[c] += 1.0;
          stat[c] += isfinite(h) ? exp(fmin(0.0, h0[c] - h)) : 0.0;
          if (!ib) S.n_oob[ch] += 1u;
          if (isnan(lp)) S.n_nonfinite[ch] += 1u;
        }
        // candidate / first-leaf source of the current subtree: -1 the leaf, l >= 0 the
        // pending left sibling of level l
        int csrc = -1, fsrc = -1;
        for (int l = 0; l < nmerge && go; ++l) {
          const double nl = U.pn[(int64_t)l * Np + ch];
          const U4 b = a.rng.block(ch, t, kStreamNuts, 16u + (uint32_t)j,
                                   (uint32_t)(8 * k + l + 1));
          const double tot = nl + ncur;
          if (!(tot > 0.0 && u52(b.x, b.y) < ncur / tot)) csrc = l;
          ncur = tot;
          double pzv = 0, pqv = 0;
          if (on) {
            pzv = U.pz[lvl(l, ch)];
            pqv = U.pq[lvl(l, ch)];
          }
          const double dz = v * (z - pzv);
          const double s1 = group_sum(dz * pqv, dp), s2 = group_sum(dz * q, dp);
          go = s1 >= 0.0 && s2 >= 0.0;
          fsrc = l;
        }
        if (go && nmerge < j) {
          // the subtree becomes the pending left sibling of its level
          if (on) {
            const int64_t o = lvl(nmerge, ch);
            U.pz[o] = fsrc < 0 ? z : U.pz[lvl(fsrc, ch)];
            U.pq[o] = fsrc < 0 ? q : U.pq[lvl(fsrc, ch)];
            U.px[o] = csrc < 0 ? xl : U.px[lvl(csrc, ch)];
            U.pgx[o] = csrc < 0 ? gxl : U.pgx[lvl(csrc, ch)];
          }
          if (gi == 0) {
            const int64_t o = (int64_t)nmerge * Np + ch;
            U.plp[o] = csrc < 0 ? lp : U.plp[(int64_t)csrc * Np + ch];
            U.pn[o] = ncur;
          }
        } else if (go) {
          // doubling j complete: progressive sampling of the tree's candidate
          const double nv = nvalid[c];
          if (utop[c] < ncur / nv) {
            if (on) {
              const int64_t o = row(ch);
              U.xc[o] = csrc < 0 ? xl : U.px[lvl(csrc, ch)];
              U.gxc[o] = csrc < 0 ? gxl : U.pgx[lvl(csrc, ch)];
            }
            if (gi == 0) {
              U.lpc[ch] = csrc < 0 ? lp : U.plp[(int64_t)csrc * Np + ch];
              moved[c] = 1;
            }
          }
          if (gi == 0) nvalid[c] = nv + ncur;
          // U-turn of the whole trajectory (this side's end is the leaf just made)
          double zmv = 0, qmv = 0, zpv = 0, qpv = 0;
          if (on) {
            const int64_t o = row(ch);
            zmv = lo ? z : U.zm[o];
            qmv = lo ? q : U.qm[o];
            zpv = lo ? U.zpl[o] : z;
            qpv = lo ? U.qpl[o] : q;
          }
          const double dz = zpv - zmv;
          const double s1 = group_sum(dz * qmv, dp), s2 = group_sum(dz * qpv, dp);
          go = s1 >= 0.0 && s2 >= 0.0;
        }
        if (gi == 0 && !go) alive[c] = 0;
      }
      __syncthreads();
      any = false;
      for (int c = 0; c < mv && !any; ++c) any = alive[c] != 0;
      if (!any) break;
    }
  }

  // the tree's candidate becomes the new state; per-chain statistics
  for (int c = tid >> lg; c < mv; c += gstep) {
    const int64_t ch = c0 + c;
    if (moved[c] && on) {
      S.x[gi * Np + ch] = U.xc[row(ch)];
      S.gx[gi * Np + ch] = U.gxc[row(ch)];
    }
    if (gi == 0) {
      const double nl = nleaf[c];
      const double pr = nl > 0.0 ? stat[c] / nl : 0.0;
      if (moved[c]) S.lp[ch] = U.lpc[ch];
      S.n_acc[ch] += moved[c] ? 1u : 0u;
      S.sum_prob[ch] += pr;
      S.step_prob[ch] = pr;
      S.n_evals[ch] += (uint32_t)nl;
    }
  }
  __syncthreads();
}

// Differential-evolution move: walker k of the active half [chain0, chain0 + half) moves
// along the difference of two distinct walkers j != k' of the other half,
// y = x_k + gamma (x_j - x_k'), gamma = (1 + eta) 2.38 / sqrt(2 d), eta ~ N(0, s^2); the
// proposal is symmetric, so log alpha = log pi(y) - log pi(x_k).  Philox stream 7, sub =
// half: block 0 holds the two partner uniforms, block 1 the normal for eta.
template <class P, int MT>
__device__ __forceinline__ void de_tile(const KArgs& a, char* smem, typename P::acc* hsave,
                                        Tally& ty, int64_t c0, int mv, uint64_t t) {
  constexpr int M = 16 * MT;
  const State& S = a.st;
  const int d = a.tg.d, tid = local_tid();
  const int64_t Np = S.Np, half = S.N / 2;
  const int h = a.aies_half;
  const int64_t other = (1 - h) * half;
  const Scratch T = tile_scratch<MT>(a, smem, c0);
  int* inbox = (int*)(smem + a.lds.mi);
  int* flag = inbox + 2 * M;
  const double g0 = 2.38 / sqrt(2.0 * (double)d);
  for (int e = tid; e < d * M; e += kThreads) {
    const int i = e / M, c = e % M;
    if (c >= mv) continue;
    const int64_t k = c0 + c;
    const U4 b = a.rng.block(k, t, kStreamDE, (uint32_t)h, 0);
    int64_t jj = (int64_t)floor(u52(b.x, b.y) * (double)half);
    if (jj > half - 1) jj = half - 1;
    int64_t kk = (int64_t)floor(u52(b.z, b.w) * (double)(half - 1));
    if (kk > half - 2) kk = half - 2;
    if (kk >= jj) kk += 1;
    const double eta = a.de_sigma * normal_dim(a.rng, k, t, kStreamDE, (uint32_t)h, 2);
    const double gam = (1.0 + eta) * g0;
    T.xp(i, c) = S.x[i * Np + k] + gam * (S.x[i * Np + other + jj] - S.x[i * Np + other + kk]);
  }
  __syncthreads();
  eval_tile<P, MT>(a, smem, hsave, T.xp, mv, T.lpp, T.gxp, false, true);
  if (tid < mv) {
    const int64_t k = c0 + tid;
    const double lpp = T.lpp[tid];
    const bool acc = decide(a, ty, k, t, (uint32_t)h, lpp - S.lp[k], lpp, inbox[tid]);
    flag[tid] = acc;
    if (acc) S.lp[k] = lpp;
  }
  __syncthreads();
  commit_tile(S, T, flag, d, M, mv, c0, false);
  __syncthreads();
}

// Copy the launch's small constant arrays (whitening, Gaussian part, box, input scaling)
// into LDS and point the kernel's argument copy at them; they are read in every phase of
// every step.
__device__ __forceinline__ void stage_constants(KArgs& a, char* smem) {
  if (a.lds.w1 >= 0) {
    // the input layer's packed weights (read by every evaluation of the launch)
    typedef int i4 __attribute__((ext_vector_type(4)));
    const int nf = a.lds.w1f_bytes / 16, nt = a.lds.w1t_bytes / 16;
    const i4* __restrict__ sf = (const i4*)a.mp.w1f;
    const i4* __restrict__ st = (const i4*)a.mp.w1t;
    i4* df = generic_ptr((i4*)(smem + a.lds.w1));
    i4* dt = df + nf;
    for (int e = local_tid(); e < nf; e += kThreads) df[e] = sf[e];
    for (int e = local_tid(); e < nt; e += kThreads) dt[e] = st[e];
    a.mp.w1f = df;
    a.mp.w1t = dt;
    if (a.lds.cst < 0) __syncthreads();
  }
  if (a.lds.cst < 0) return;
  const int d = a.tg.d, dd = d * d, tid = local_tid();
  double* c = generic_ptr((double*)(smem + a.lds.cst));
  auto copy = [&](const double* src, double* dst, int n) {
    for (int e = tid; e < n; e += kThreads) dst[e] = src[e];
  };
  copy(a.wh.L, c, dd);
  copy(a.tg.gprec, c + dd, dd);
  copy(a.wh.mu, c + 2 * dd, d);
  copy(a.tg.gmean, c + 2 * dd + d, d);
  copy(a.tg.lower, c + 2 * dd + 2 * d, d);
  copy(a.tg.upper, c + 2 * dd + 3 * d, d);
  copy(a.tg.in_center, c + 2 * dd + 4 * d, d);
  copy(a.tg.in_invscale, c + 2 * dd + 5 * d, d);
  copy(a.tg.train_lo, c + 2 * dd + 6 * d, d);
  copy(a.tg.train_hi, c + 2 * dd + 7 * d, d);
  __syncthreads();
  a.wh.L = c;
  a.tg.gprec = c + dd;
  a.wh.mu = c + 2 * dd;
  a.tg.gmean = c + 2 * dd + d;
  a.tg.lower = c + 2 * dd + 2 * d;
  a.tg.upper = c + 2 * dd + 3 * d;
  a.tg.in_center = c + 2 * dd + 4 * d;
  a.tg.in_invscale = c + 2 * dd + 5 * d;
  a.tg.train_lo = c + 2 * dd + 6 * d;
  a.tg.train_hi = c + 2 * dd + 7 * d;
}

// ---------------------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------------------
// ADAPT marks the launches of the step-size adaptation windows (one step per launch, step
// size from the dual-averaging state); production launches are separate instantiations so
// that profiles keep the two apart.
template <class P, int MT, int SAMPLER, bool ADAPT>
__global__ __launch_bounds__(kThreads, 1) void step_kernel(KArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  using acc = typename P::acc;
  constexpr int M = 16 * MT;
  acc* hsave = (acc*)a.hsave + (int64_t)blockIdx.x * a.hsave_stride;
  const double eps = (ADAPT || a.eps_ptr) ? *a.eps_ptr : a.eps;
  stage_constants(a, smem);
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int64_t c0 = a.chain0 + tile * M;
    constexpr bool kHalves = SAMPLER == 3 || SAMPLER == 5;  // ensemble moves, one half per launch
    const int64_t lim = kHalves ? a.chain0 + a.st.N / 2 : a.st.N;
    const int mv = (int)((lim - c0) < M ? (lim - c0) : M);
    Tally ty{};
    for (int s = 0; s < a.n_steps; ++s) {
      const uint64_t t = (uint64_t)(a.step0 + s);
      if constexpr (SAMPLER == 0) mh_tile<P, MT>(a, smem, hsave, ty, c0, mv, t);
      if constexpr (SAMPLER == 1) mala_tile<P, MT>(a, smem, hsave, ty, c0, mv, t, eps);
      if constexpr (SAMPLER == 2) hmc_tile<P, MT>(a, smem, hsave, ty, c0, mv, t, eps);
      if constexpr (SAMPLER == 3) aies_tile<P, MT>(a, smem, hsave, ty, c0, mv, t);
      if constexpr (SAMPLER == 4) nuts_tile<P, MT>(a, smem, hsave, c0, mv, t, eps);
      if constexpr (SAMPLER == 5) de_tile<P, MT>(a, smem, hsave, ty, c0, mv, t);
      if constexpr (!kHalves) record_tile(a, s, a.tg.d, M, mv, c0);
    }
    if constexpr (SAMPLER != 4) {
      // the lane-group MALA / HMC keep chain c's tally in thread G c (G = 8 or 16), the
      // others in thread c
      int own = 1;
      if constexpr (SAMPLER == 1 || SAMPLER == 2) {
        if (group_path<P, MT>(a)) own = 8;
        else if (wide_path<P, MT>(a)) own = 16;
      }
      const int tid = local_tid();
      if (a.n_steps > 0 && tid % own == 0 && tid / own < mv) flush_tally(a.st, c0 + tid / own, ty);
    }
  }
}

// best_logL_grad: evaluate n points from a caller SoA array.
template <class P, int MT>
__global__ __launch_bounds__(kThreads, 1) void eval_kernel(KArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  using acc = typename P::acc;
  constexpr int M = 16 * MT;
  acc* hsave = (acc*)a.hsave + (int64_t)blockIdx.x * a.hsave_stride;
  const int64_t n = a.st.N;
  stage_constants(a, smem);
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int64_t c0 = tile * M;
    const int mv = (int)((n - c0) < M ? (n - c0) : M);
    eval_tile<P, MT>(a, smem, hsave, TView{const_cast<double*>(a.ex_x) + c0, a.ex_pitch}, mv,
                     a.ex_lp + c0, TView{a.ex_g ? a.ex_g + c0 : nullptr, a.ex_pitch},
                     a.ex_grad != 0, true);
  }
}

}  // namespace best
