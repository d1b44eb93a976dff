// Fused MLP emulator for one chain tile held by one workgroup.
//
// The emulator (CLiENT-style dense tanh network, Sec. 1 / Fig. scaling of the paper) is
//   h_1 = tanh(W_1 t + b_1), h_l = tanh(W_l h_{l-1} + b_l), out = w_out . h_L + b_out
// and its reverse-mode input gradient
//   delta_L = up * w_out (1 - h_L^2), delta_{l-1} = (W_l^T delta_l)(1 - h_{l-1}^2),
//   d out / d t = W_1^T delta_1.
//
// Mapping to a gfx950 CU (256 threads = 4 wave64):
//   * a tile of M = 16*MT chains is processed through every layer inside one workgroup, so
//     the only global traffic is weights (L2-resident, streamed once per tile per layer)
//     and a small per-tile scratch of activations;
//   * hidden layers l >= 2 are MFMA GEMMs D[j][c] = sum_k W[j][k] h[k][c]: the 4 waves
//     split the H output rows, each wave loops over its 16-row tiles in groups of RG and
//     keeps RG x MT accumulator tiles in registers.  A fragments (weights, pre-packed in
//     fragment order so every wave load is 1 KiB contiguous) come from global memory;
//     B fragments (activations of all M chains) come from LDS where they are stored in
//     fragment order as well (conflict-free 16-byte reads);
//   * the epilogue fuses bias + tanh and writes h both to the next layer's LDS buffer
//     (rounded to the GEMM type) and, unrounded, to the tile scratch in D-tile order,
//     which is exactly the order in which the same lane needs (1 - h^2) in the backward
//     epilogue;
//   * the K = d input layer, the output dot product and W_1^T delta_1 run on the vector
//     ALUs (FP32, or FP64 for the FP64 path); cross-wave sums use a fixed order so
//     results are bitwise reproducible.
#pragma once
#include "common.hpp"

namespace best {

#ifndef BEST_PREFETCH
#define BEST_PREFETCH 8
#endif
#ifndef BEST_RG_MAX
#define BEST_RG_MAX 4
#endif
// k-steps of weight fragments in flight per wave (halved for the widest chain tiles and
// for FP64, whose accumulators need the registers)
constexpr int kPrefetch = BEST_PREFETCH;
constexpr int kRgMax = BEST_RG_MAX;       // row tiles per register group

struct MlpParams {
  int d, H, nh;
  int lds_h;         // 1: saved activations stay in LDS (GEMM type), 0: global scratch
  const void* wf;    // T: fragment-ordered W_l, l = 2..nh, H*H each
  const void* wb;    // T: fragment-ordered W_l^T, l = 2..nh
  const void* w1;    // vec: [H][d]
  const void* bias;  // acc: [nh][H]
  const void* wout;  // acc: [H + 1], w_out followed by b_out
};

// Optional row-major exports for training: h_l and delta_l as [nh][H][ldb] floats.
struct MlpExport {
  float* h;
  float* dl;
  int64_t ldb;
  int64_t col0;
  int mvalid;
};

// LDS buffers of the tile engine.  With lds_h the activations h_1..h_L keep one slot each
// (act + (l-1) M H, fragment order, GEMM type) and two further buffers hold deltas; without
// it `act` holds two ping-pong buffers that the deltas reuse after the forward pass, and
// the activations are saved to the per-workgroup global scratch.
template <class P>
struct MlpSmem {
  typename P::T* act;    // activation slots / ping-pong buffers
  typename P::T* dlt0;   // delta buffers (M*H each)
  typename P::T* dlt1;
  typename P::vec* th;   // [M][d] input t
  typename P::vec* gth;  // [M][d] d out / d t
  typename P::acc* red;  // [kWaves][M][d] partial sums
  typename P::acc* out;  // [M]
  typename P::acc* up;   // [M] upstream gradient, NULL means 1
};

template <class P>
__device__ __forceinline__ int lds_off(int k, int c, int KS) {
  return (int)frag_offset<P>(c, k, KS);  // B fragments: column = chain, k = neuron
}

template <class P, int RG, int MT, class Epi>
__device__ __forceinline__ void gemm_group(const typename P::T* __restrict__ A, int KS,
                                           const typename P::T* __restrict__ Bl, int rt0,
                                           Epi& epi) {
  // A fragments of kPrefetch k-steps are kept in flight (a register ring indexed by the
  // unrolled position p), so each wave has up to kPrefetch * RG 1 KiB loads outstanding;
  // this hides the L2 latency that a load-then-use loop exposes at every k-step.
  using frag = typename P::frag;
  using accv = typename P::accv;
  constexpr int D = (MT >= 4 || sizeof(typename P::acc) == 8) ? (kPrefetch > 4 ? 4 : kPrefetch)
                                                               : kPrefetch;
  const int lane = threadIdx.x & 63;
  accv acc[RG][MT];
#pragma unroll
  for (int rr = 0; rr < RG; ++rr)
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) acc[rr][ct] = accv{};
  const frag* __restrict__ Af = reinterpret_cast<const frag*>(A);
  const frag* __restrict__ Bf = reinterpret_cast<const frag*>(Bl);
  frag a[D][RG];
#pragma unroll
  for (int p = 0; p < D; ++p) {
    if (p < KS) {
#pragma unroll
      for (int rr = 0; rr < RG; ++rr) a[p][rr] = Af[((int64_t)(rt0 + rr) * KS + p) * 64 + lane];
    }
  }
  for (int k0 = 0; k0 < KS; k0 += D) {
#pragma unroll
    for (int p = 0; p < D; ++p) {
      const int ks = k0 + p;
      if (ks < KS) {
        frag b[MT];
#pragma unroll
        for (int ct = 0; ct < MT; ++ct) b[ct] = Bf[(ct * KS + ks) * 64 + lane];
#pragma unroll
        for (int rr = 0; rr < RG; ++rr)
#pragma unroll
          for (int ct = 0; ct < MT; ++ct) acc[rr][ct] = P::mma(a[p][rr], b[ct], acc[rr][ct]);
        if (ks + D < KS) {
#pragma unroll
          for (int rr = 0; rr < RG; ++rr)
            a[p][rr] = Af[((int64_t)(rt0 + rr) * KS + ks + D) * 64 + lane];
        }
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < RG; ++rr)
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) epi(rt0 + rr, ct, acc[rr][ct]);
}

// GEMM over this wave's RTW row tiles starting at rtw0, in register groups of 8/4/2/1.
template <class P, int MT, class Epi>
__device__ __forceinline__ void gemm_rows(const typename P::T* A, int KS,
                                          const typename P::T* Bl, int rtw0, int RTW,
                                          Epi& epi) {
  if (kRgMax >= 8 && RTW % 8 == 0) {
    for (int r = 0; r < RTW; r += 8) gemm_group<P, (kRgMax >= 8 ? 8 : 1), MT>(A, KS, Bl, rtw0 + r, epi);
  } else if (RTW % 4 == 0) {
    for (int r = 0; r < RTW; r += 4) gemm_group<P, 4, MT>(A, KS, Bl, rtw0 + r, epi);
  } else if (RTW % 2 == 0) {
    for (int r = 0; r < RTW; r += 2) gemm_group<P, 2, MT>(A, KS, Bl, rtw0 + r, epi);
  } else {
    for (int r = 0; r < RTW; ++r) gemm_group<P, 1, MT>(A, KS, Bl, rtw0 + r, epi);
  }
}

template <class V>
__device__ __forceinline__ V act_tanh(V y) {
  return tanh(y);
}

// Per-tile activation scratch in D-tile order: [layer][rt][ct][lane][4].
template <class P, int MT>
__device__ __forceinline__ typename P::acc* hsave_at(typename P::acc* base, int layer, int RT,
                                                     int rt, int ct, int lane) {
  return base + ((((int64_t)layer * RT + rt) * MT + ct) * 64 + lane) * 4;
}

// Buffers of the tile engine for a given storage mode.
template <class P, int MT>
__device__ __forceinline__ MlpSmem<P> mlp_smem(char* base, const MlpParams& mp) {
  constexpr int M = 16 * MT;
  MlpSmem<P> s;
  const int64_t MH = (int64_t)M * mp.H;
  s.act = (typename P::T*)base;
  if (mp.lds_h) {
    s.dlt0 = s.act + mp.nh * MH;
    s.dlt1 = s.dlt0 + MH;
  } else {
    s.dlt0 = s.act + ((mp.nh - 1) & 1) * MH;
    s.dlt1 = s.act + (mp.nh & 1) * MH;
  }
  return s;
}

// Output buffer of layer l (1-based).
template <class P, int MT>
__device__ __forceinline__ typename P::T* layer_buf(const MlpSmem<P>& s, const MlpParams& mp,
                                                    int l) {
  const int64_t MH = (int64_t)16 * MT * mp.H;
  return s.act + (mp.lds_h ? (l - 1) : ((l - 1) & 1)) * MH;
}

// The saved activation h_l of this lane's D-tile slot r at row j of chain c.
template <class P, int MT>
__device__ __forceinline__ void load_h(const MlpSmem<P>& s, const MlpParams& mp,
                                       typename P::acc* __restrict__ hsave, int l, int rt,
                                       int ct, typename P::acc h[4]) {
  using acc = typename P::acc;
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int KS = mp.H / P::KSTEP, RT = mp.H / 16;
  if (mp.lds_h) {
    const typename P::T* b = layer_buf<P, MT>(s, mp, l);
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = (acc)b[lds_off<P>(rt * 16 + P::drow(g, r), ct * 16 + cl, KS)];
  } else {
    const acc* hp = hsave_at<P, MT>(hsave, l - 1, RT, rt, ct, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = __builtin_nontemporal_load(hp + r);
  }
}

// Forward pass.  Writes s.out[c] (incl. b_out).  If fuse_delta, the last layer's epilogue
// also writes delta_L = w_out (1 - h_L^2) (upstream 1) into s.dlt0 for mlp_backward.
template <class P, int MT>
__device__ __forceinline__ void mlp_forward(const MlpParams& mp, const MlpSmem<P>& s,
                                            typename P::acc* __restrict__ hsave,
                                            const MlpExport* ex, bool fuse_delta) {
  using T = typename P::T;
  using acc = typename P::acc;
  using vec = typename P::vec;
  using accv = typename P::accv;
  constexpr int M = 16 * MT;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, wv = tid >> 6, cl = lane & 15;
  const int d = mp.d, H = mp.H, nh = mp.nh;
  const int KS = H / P::KSTEP, RTW = H / 64, RT = H / 16;
  const vec* __restrict__ W1 = (const vec*)mp.w1;
  const acc* __restrict__ Bs = (const acc*)mp.bias;
  const acc* __restrict__ Wo = (const acc*)mp.wout;
  acc po[MT];
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) po[ct] = 0;

  // epilogue shared by every layer: save h_l, feed layer l+1, and at the last layer the
  // output dot product and (optionally) delta_L
  auto finish = [&](int l, int rt, int ct, const acc hv[4]) {
    const int c = ct * 16 + cl;
    const bool last = (l == nh);
    if (mp.lds_h || !last) {
      T* ob = layer_buf<P, MT>(s, mp, l);
#pragma unroll
      for (int r = 0; r < 4; ++r) ob[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)hv[r];
    }
    if (!mp.lds_h) {
      acc* hp = hsave_at<P, MT>(hsave, l - 1, RT, rt, ct, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) __builtin_nontemporal_store(hv[r], hp + r);
    }
    if (last) {
#pragma unroll
      for (int r = 0; r < 4; ++r) po[ct] += Wo[rt * 16 + P::drow(g, r)] * hv[r];
      if (fuse_delta && nh > 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = rt * 16 + P::drow(g, r);
          s.dlt0[lds_off<P>(j, c, KS)] = (T)(Wo[j] * ((acc)1 - hv[r] * hv[r]));
        }
      }
    }
    if (ex && c < ex->mvalid) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        ex->h[((int64_t)(l - 1) * H + rt * 16 + P::drow(g, r)) * ex->ldb + ex->col0 + c] =
            (float)hv[r];
    }
  };

  // ---- layer 1: K = d on the vector ALUs ----
  for (int rr = 0; rr < RTW; ++rr) {
    const int rt = wv * RTW + rr;
    for (int ct = 0; ct < MT; ++ct) {
      const int c = ct * 16 + cl;
      acc hv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = rt * 16 + P::drow(g, r);
        acc y = Bs[j];
        for (int i = 0; i < d; ++i) y += (acc)W1[j * d + i] * (acc)s.th[c * d + i];
        hv[r] = act_tanh(y);
      }
      finish(1, rt, ct, hv);
    }
  }
  __syncthreads();

  // ---- hidden layers 2..nh: MFMA GEMMs ----
  for (int l = 2; l <= nh; ++l) {
    const T* Bin = layer_buf<P, MT>(s, mp, l - 1);
    const T* A = (const T*)mp.wf + (int64_t)(l - 2) * H * H;
    const acc* bl = Bs + (int64_t)(l - 1) * H;
    auto epi = [&](int rt, int ct, const accv& v) {
      acc hv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) hv[r] = act_tanh((acc)v[r] + bl[rt * 16 + P::drow(g, r)]);
      finish(l, rt, ct, hv);
    };
    gemm_rows<P, MT>(A, KS, Bin, wv * RTW, RTW, epi);
    __syncthreads();
  }

  // ---- output layer: fixed-order sums of the per-lane partial dot products ----
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) {
    const acc v = sum_lane_groups(po[ct]);
    if (g == 0) s.red[wv * M + ct * 16 + cl] = v;
  }
  __syncthreads();
  if (tid < M) {
    acc o = s.red[tid];
    for (int w = 1; w < kWaves; ++w) o += s.red[w * M + tid];
    s.out[tid] = o + Wo[H];
  }
  __syncthreads();
}

// Backward pass (reverse mode).  s.up (or 1) is the upstream gradient per chain; if the
// forward fused delta_L, s.up must be NULL.  If want_input_grad, writes
// s.gth[c][i] = d(up * out)/d t_i.
template <class P, int MT>
__device__ __forceinline__ void mlp_backward(const MlpParams& mp, const MlpSmem<P>& s,
                                             typename P::acc* __restrict__ hsave,
                                             const MlpExport* ex, bool want_input_grad,
                                             bool delta_fused) {
  using T = typename P::T;
  using acc = typename P::acc;
  using vec = typename P::vec;
  using accv = typename P::accv;
  constexpr int M = 16 * MT;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, wv = tid >> 6, cl = lane & 15;
  const int d = mp.d, H = mp.H, nh = mp.nh;
  const int KS = H / P::KSTEP, RTW = H / 64;
  const vec* __restrict__ W1 = (const vec*)mp.w1;
  const acc* __restrict__ Wo = (const acc*)mp.wout;

  if (want_input_grad) {
    for (int e = tid; e < kWaves * M * d; e += kThreads) s.red[e] = 0;
    __syncthreads();
  }
  // delta_1 -> partial W_1^T delta_1 accumulated per wave (g == 0 lane owns (wv, c, i))
  auto input_grad_acc = [&](int rt, int ct, const acc* dl) {
    const int c = ct * 16 + cl;
    for (int i = 0; i < d; ++i) {
      acc p = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) p += (acc)W1[(rt * 16 + P::drow(g, r)) * d + i] * dl[r];
      p = sum_lane_groups(p);
      if (g == 0) s.red[(wv * M + c) * d + i] += p;
    }
  };

  // ---- delta_L = up * w_out * (1 - h_L^2), unless the forward epilogue wrote it ----
  if (!delta_fused || nh == 1) {
    for (int rr = 0; rr < RTW; ++rr) {
      const int rt = wv * RTW + rr;
      for (int ct = 0; ct < MT; ++ct) {
        const int c = ct * 16 + cl;
        const acc u = s.up ? s.up[c] : (acc)1;
        acc hv[4], dl[4];
        load_h<P, MT>(s, mp, hsave, nh, rt, ct, hv);
#pragma unroll
        for (int r = 0; r < 4; ++r) dl[r] = u * Wo[rt * 16 + P::drow(g, r)] * ((acc)1 - hv[r] * hv[r]);
        if (nh > 1) {
#pragma unroll
          for (int r = 0; r < 4; ++r) s.dlt0[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)dl[r];
        } else if (want_input_grad) {
          input_grad_acc(rt, ct, dl);
        }
        if (ex && c < ex->mvalid) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            ex->dl[((int64_t)(nh - 1) * H + rt * 16 + P::drow(g, r)) * ex->ldb + ex->col0 + c] =
                (float)dl[r];
        }
      }
    }
    __syncthreads();
  }

  // ---- hidden layers nh..2: D[k][c] = sum_j W_l^T[k][j] delta_l[j][c] ----
  for (int l = nh; l >= 2; --l) {
    const bool in0 = ((nh - l) & 1) == 0;
    const T* Bin = in0 ? s.dlt0 : s.dlt1;
    T* Bout = in0 ? s.dlt1 : s.dlt0;
    const T* A = (const T*)mp.wb + (int64_t)(l - 2) * H * H;
    const bool last = (l == 2);
    auto epi = [&](int rt, int ct, const accv& v) {
      const int c = ct * 16 + cl;
      acc hv[4], dl[4];
      load_h<P, MT>(s, mp, hsave, l - 1, rt, ct, hv);
#pragma unroll
      for (int r = 0; r < 4; ++r) dl[r] = (acc)v[r] * ((acc)1 - hv[r] * hv[r]);
      if (!last) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Bout[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)dl[r];
      } else if (want_input_grad) {
        input_grad_acc(rt, ct, dl);
      }
      if (ex && c < ex->mvalid) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ex->dl[((int64_t)(l - 2) * H + rt * 16 + P::drow(g, r)) * ex->ldb + ex->col0 + c] =
              (float)dl[r];
      }
    };
    gemm_rows<P, MT>(A, KS, Bin, wv * RTW, RTW, epi);
    __syncthreads();
  }

  if (want_input_grad) {
    for (int e = tid; e < M * d; e += kThreads) {
      const int c = e / d, i = e % d;
      acc v = s.red[c * d + i];
      for (int w = 1; w < kWaves; ++w) v += s.red[(w * M + c) * d + i];
      s.gth[e] = (vec)v;
    }
    __syncthreads();
  }
}

}  // namespace best
