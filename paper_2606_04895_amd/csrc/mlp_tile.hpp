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
#define BEST_PREFETCH 4
#endif
#ifndef BEST_RG_MAX
#define BEST_RG_MAX 4
#endif
constexpr int kPrefetch = BEST_PREFETCH;  // k-steps of weight fragments in flight per wave
constexpr int kRgMax = BEST_RG_MAX;       // row tiles per register group

struct MlpParams {
  int d, H, nh;
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

template <class P>
struct MlpSmem {
  typename P::T* buf0;   // M*H
  typename P::T* buf1;   // M*H
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
  constexpr int D = kPrefetch;
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

// Forward pass: fills the activation scratch and s.out[c] (incl. b_out).
template <class P, int MT>
__device__ __forceinline__ void mlp_forward(const MlpParams& mp, const MlpSmem<P>& s,
                            typename P::acc* __restrict__ hsave, const MlpExport* ex) {
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
      acc* hp = hsave_at<P, MT>(hsave, 0, RT, rt, ct, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) hp[r] = hv[r];
      if (nh > 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) s.buf0[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)hv[r];
      }
      if (ex && c < ex->mvalid) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ex->h[(int64_t)(rt * 16 + P::drow(g, r)) * ex->ldb + ex->col0 + c] = (float)hv[r];
      }
    }
  }
  __syncthreads();

  // ---- hidden layers 2..nh: MFMA GEMMs ----
  for (int l = 2; l <= nh; ++l) {
    const T* Bin = (l & 1) ? s.buf1 : s.buf0;
    T* Bout = (l & 1) ? s.buf0 : s.buf1;
    const T* A = (const T*)mp.wf + (int64_t)(l - 2) * H * H;
    const acc* bl = Bs + (int64_t)(l - 1) * H;
    const bool write_lds = l < nh;
    auto epi = [&](int rt, int ct, const accv& v) {
      const int c = ct * 16 + cl;
      acc hv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) hv[r] = act_tanh((acc)v[r] + bl[rt * 16 + P::drow(g, r)]);
      acc* hp = hsave_at<P, MT>(hsave, l - 1, RT, rt, ct, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) hp[r] = hv[r];
      if (write_lds) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Bout[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)hv[r];
      }
      if (ex && c < ex->mvalid) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ex->h[((int64_t)(l - 1) * H + rt * 16 + P::drow(g, r)) * ex->ldb + ex->col0 + c] =
              (float)hv[r];
      }
    };
    gemm_rows<P, MT>(A, KS, Bin, wv * RTW, RTW, epi);
    __syncthreads();
  }

  // ---- output layer: out[c] = w_out . h_nh + b_out (fixed-order sums) ----
  acc po[MT];
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) po[ct] = 0;
  for (int rr = 0; rr < RTW; ++rr) {
    const int rt = wv * RTW + rr;
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) {
      const acc* hp = hsave_at<P, MT>(hsave, nh - 1, RT, rt, ct, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) po[ct] += Wo[rt * 16 + P::drow(g, r)] * hp[r];
    }
  }
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

// Backward pass (reverse mode).  Requires mlp_forward's scratch; s.up (or 1) is the
// upstream gradient per chain.  If want_input_grad, writes s.gth[c][i] = d(up*out)/d t_i.
template <class P, int MT>
__device__ __forceinline__ void mlp_backward(const MlpParams& mp, const MlpSmem<P>& s,
                             typename P::acc* __restrict__ hsave, const MlpExport* ex,
                             bool want_input_grad) {
  using T = typename P::T;
  using acc = typename P::acc;
  using vec = typename P::vec;
  using accv = typename P::accv;
  constexpr int M = 16 * MT;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, wv = tid >> 6, cl = lane & 15;
  const int d = mp.d, H = mp.H, nh = mp.nh;
  const int KS = H / P::KSTEP, RTW = H / 64, RT = H / 16;
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

  // ---- delta_nh = up * w_out * (1 - h_nh^2) ----
  for (int rr = 0; rr < RTW; ++rr) {
    const int rt = wv * RTW + rr;
    for (int ct = 0; ct < MT; ++ct) {
      const int c = ct * 16 + cl;
      const acc u = s.up ? s.up[c] : (acc)1;
      const acc* hp = hsave_at<P, MT>(hsave, nh - 1, RT, rt, ct, lane);
      acc dl[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) dl[r] = u * Wo[rt * 16 + P::drow(g, r)] * ((acc)1 - hp[r] * hp[r]);
      if (nh > 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) s.buf0[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)dl[r];
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

  // ---- hidden layers nh..2: D[k][c] = sum_j W_l^T[k][j] delta_l[j][c] ----
  for (int l = nh; l >= 2; --l) {
    const bool in_buf0 = ((nh - l) & 1) == 0;
    const T* Bin = in_buf0 ? s.buf0 : s.buf1;
    T* Bout = in_buf0 ? s.buf1 : s.buf0;
    const T* A = (const T*)mp.wb + (int64_t)(l - 2) * H * H;
    const bool last = (l == 2);
    auto epi = [&](int rt, int ct, const accv& v) {
      const int c = ct * 16 + cl;
      const acc* hp = hsave_at<P, MT>(hsave, l - 2, RT, rt, ct, lane);
      acc dl[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) dl[r] = (acc)v[r] * ((acc)1 - hp[r] * hp[r]);
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
