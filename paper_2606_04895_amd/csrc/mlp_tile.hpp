// Fused MLP emulator for one chain tile held by one workgroup.
//
// The emulator (dense tanh network of the kind the paper's emulators use, Sec. 1 and the
// scaling study of Sec. 5) is
//   h_1 = tanh(W_1 t + b_1), h_l = tanh(W_l h_{l-1} + b_l), out = w_out . h_L + b_out
// and its reverse-mode input gradient
//   delta_L = up * w_out (1 - h_L^2), delta_{l-1} = (W_l^T delta_l)(1 - h_{l-1}^2),
//   d out / d t = W_1^T delta_1.
//
// Mapping to a gfx950 CU (512 threads = 8 wave64, two per SIMD):
//   * a tile of M = 16*MT chains goes through every layer inside one workgroup; global
//     traffic is the packed weights (L2-resident for networks up to a few MiB) and, when
//     the tile's activations do not fit in LDS, a per-workgroup activation scratch;
//   * every layer is an MFMA GEMM D[j][c] = sum_k W[j][k] h[k][c]: the waves split the H
//     output rows, each wave walks its 16-row tiles in register groups of RG.  A fragments
//     (weights, pre-packed in fragment order so every wave load is 1 KiB contiguous) stream
//     from global memory through a branch-free ring of kPrefetch k-steps, so a wave only
//     waits for its oldest load; B fragments (activations of the tile's chains) come from
//     LDS, also in fragment order (conflict-free 16-byte reads);
//   * the K = d input layer runs on FP32 MFMA (FP64 for the FP64 path), so the inputs are
//     not rounded to the 16-bit GEMM types, and W_1^T delta_1 is a small GEMM whose K = H
//     reduction is split over the waves;
//   * epilogues fuse bias + tanh (forward) and the (1 - h^2) factor (backward); the output
//     dot product and delta_L are fused into the last forward epilogue; every cross-wave
//     sum has a fixed order, so results are bitwise reproducible.
#pragma once
#include "common.hpp"

namespace best {

constexpr int kPrefetch = 4;  // k-steps of weight fragments in flight per wave
constexpr int kRgMax = 4;     // 16-row tiles per register group

// Precision of the K = d input layer: FP64 for the FP64 path, FP32 MFMA otherwise.
template <class P>
struct InPrec {
  using type = Prec<float>;
};
template <>
struct InPrec<Prec<double>> {
  using type = Prec<double>;
};

struct MlpParams {
  int d, H, nh;
  int lds_h;         // 1: saved activations stay in LDS (GEMM type), 0: global scratch
  int ks1;           // k-steps of the input layer (d padded to the input precision's KSTEP)
  int rti;           // 16-row tiles of W_1^T (d padded to 16)
  const void* wf;    // T: fragment-ordered W_l, l = 2..nh, H*H each
  const void* wb;    // T: fragment-ordered W_l^T, l = 2..nh
  const void* w1f;   // input type: fragment-ordered W_1 (H rows, ks1 k-steps, zero padded)
  const void* w1t;   // T: fragment-ordered W_1^T (16*rti rows, H/KSTEP k-steps, zero padded)
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
  typename P::T* act;                // activation slots / ping-pong buffers
  typename P::T* dlt0;               // delta buffers (M*H each)
  typename P::T* dlt1;
  typename InPrec<P>::type::T* thf;  // input t, B fragments of the input layer
  typename P::vec* gth;              // [M][d] d out / d t
  typename P::acc* red;              // [kWaves][M][d] partial sums
  typename P::acc* out;              // [M]
  typename P::acc* up;               // [M] upstream gradient, NULL means 1
};

template <class P>
__device__ __forceinline__ int lds_off(int k, int c, int KS) {
  return (int)frag_offset<P>(c, k, KS);  // B fragments: column = chain, k = neuron
}

// Input component i of chain c (the caller also writes the zero padding i in [d, 16 ks1)).
template <class P>
__device__ __forceinline__ void store_t(const MlpSmem<P>& s, const MlpParams& mp, int c, int i,
                                        double v) {
  using IP = typename InPrec<P>::type;
  s.thf[frag_offset<IP>(c, i, mp.ks1)] = (typename IP::T)v;
}

// One register group of a GEMM: RG row tiles x MT chain tiles over KS k-steps (KS a
// multiple of kPrefetch).  The A fragments of the next kPrefetch k-steps are always in
// flight; the ring has no conditional loads, so the waits stay partial.
template <class P, int RG, int MT, class Epi>
__device__ __forceinline__ void gemm_group(const typename P::T* __restrict__ A, int KS,
                                           const typename P::T* __restrict__ Bl, int rt0,
                                           Epi& epi) {
  using frag = typename P::frag;
  using accv = typename P::accv;
  constexpr int D = kPrefetch;
  const int lane = threadIdx.x & 63;
  accv acc[RG][MT];
#pragma unroll
  for (int rr = 0; rr < RG; ++rr)
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) acc[rr][ct] = accv{};
  const frag* __restrict__ Af = reinterpret_cast<const frag*>(A) + (int64_t)rt0 * KS * 64 + lane;
  const frag* __restrict__ Bf = reinterpret_cast<const frag*>(Bl) + lane;
  frag a[D][RG];
#pragma unroll
  for (int p = 0; p < D; ++p)
#pragma unroll
    for (int rr = 0; rr < RG; ++rr) a[p][rr] = Af[((int64_t)rr * KS + p) * 64];
  auto step = [&](int ks, int p) {
    frag b[MT];
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) b[ct] = Bf[(ct * KS + ks) * 64];
#pragma unroll
    for (int rr = 0; rr < RG; ++rr)
#pragma unroll
      for (int ct = 0; ct < MT; ++ct) acc[rr][ct] = P::mma(a[p][rr], b[ct], acc[rr][ct]);
  };
  int k0 = 0;
  for (; k0 < KS - D; k0 += D) {
#pragma unroll
    for (int p = 0; p < D; ++p) {
      step(k0 + p, p);
#pragma unroll
      for (int rr = 0; rr < RG; ++rr) a[p][rr] = Af[((int64_t)rr * KS + k0 + p + D) * 64];
    }
  }
#pragma unroll
  for (int p = 0; p < D; ++p) step(k0 + p, p);
#pragma unroll
  for (int rr = 0; rr < RG; ++rr)
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) epi(rt0 + rr, ct, acc[rr][ct]);
}

// Short GEMM for one row tile without the ring (the input layer: a few k-steps).
template <class P, int MT, class Epi>
__device__ __forceinline__ void gemm_short(const typename P::T* __restrict__ A, int KS,
                                           const typename P::T* __restrict__ Bl, int rt,
                                           Epi& epi) {
  using frag = typename P::frag;
  using accv = typename P::accv;
  const int lane = threadIdx.x & 63;
  accv acc[MT];
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) acc[ct] = accv{};
  const frag* __restrict__ Af = reinterpret_cast<const frag*>(A);
  const frag* __restrict__ Bf = reinterpret_cast<const frag*>(Bl);
  for (int ks = 0; ks < KS; ++ks) {
    const frag a = Af[((int64_t)rt * KS + ks) * 64 + lane];
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) acc[ct] = P::mma(a, Bf[(ct * KS + ks) * 64 + lane], acc[ct]);
  }
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) epi(rt, ct, acc[ct]);
}

// GEMM over this wave's RTW row tiles starting at rtw0, in register groups of 4/2/1.
template <class P, int MT, class Epi>
__device__ __forceinline__ void gemm_rows(const typename P::T* A, int KS,
                                          const typename P::T* Bl, int rtw0, int RTW,
                                          Epi& epi) {
  if (RTW % 4 == 0) {
    for (int r = 0; r < RTW; r += 4) gemm_group<P, 4, MT>(A, KS, Bl, rtw0 + r, epi);
  } else if (RTW % 2 == 0) {
    for (int r = 0; r < RTW; r += 2) gemm_group<P, 2, MT>(A, KS, Bl, rtw0 + r, epi);
  } else {
    for (int r = 0; r < RTW; ++r) gemm_group<P, 1, MT>(A, KS, Bl, rtw0 + r, epi);
  }
}

// tanh(y) = sign(y) (1 - e) / (1 + e) with e = exp(-2|y|), on the hardware exp and
// reciprocal (absolute error about 1e-7, below the FP32 rounding of the layer sums); the
// FP64 path uses the library tanh.
__device__ __forceinline__ float act_tanh(float y) {
  const float e = __expf(-2.0f * fabsf(y));
  return copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), y);
}
__device__ __forceinline__ double act_tanh(double y) { return tanh(y); }

// Per-tile activation scratch in D-tile order: [layer][rt][ct][lane][4].
template <class P, int MT>
__device__ __forceinline__ typename P::acc* hsave_at(typename P::acc* base, int layer, int RT,
                                                     int rt, int ct, int lane) {
  return base + ((((int64_t)layer * RT + rt) * MT + ct) * 64 + lane) * 4;
}

// Buffers of the tile engine for a given storage mode (the caller sets thf, gth, red, out
// and up).
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

// The saved activation h_l in this lane's D-tile slots of tile (rt, ct).
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

// Forward pass.  Reads the input from s.thf and writes s.out[c] (incl. b_out).  If
// fuse_delta, the last layer's epilogue also writes delta_L = w_out (1 - h_L^2) (upstream
// 1) into s.dlt0 for mlp_backward.
template <class P, int MT>
__device__ __forceinline__ void mlp_forward(const MlpParams& mp, const MlpSmem<P>& s,
                                            typename P::acc* __restrict__ hsave,
                                            const MlpExport* ex, bool fuse_delta) {
  using T = typename P::T;
  using acc = typename P::acc;
  using accv = typename P::accv;
  using IP = typename InPrec<P>::type;
  constexpr int M = 16 * MT;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, wv = tid >> 6, cl = lane & 15;
  const int H = mp.H, nh = mp.nh;
  const int KS = H / P::KSTEP, RTW = H / (16 * kWaves), RT = H / 16;
  const acc* __restrict__ Bs = (const acc*)mp.bias;
  const acc* __restrict__ Wo = (const acc*)mp.wout;
  acc po[MT];
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) po[ct] = 0;

  // epilogue shared by every layer (hv[r] is row rows[r] of chain ct*16 + cl): save h_l,
  // feed layer l+1, and at the last layer the output dot product and (optionally) delta_L.
  // The D layouts of the input-layer and hidden-layer instructions coincide (FP32-class:
  // rows 4g + r, FP64: rows g + 4r), so the saved slots read back the same way.
  auto finish = [&](int l, int rt, int ct, const acc hv[4], const int rows[4]) {
    const int c = ct * 16 + cl;
    const bool last = (l == nh);
    if (mp.lds_h || !last) {
      T* ob = layer_buf<P, MT>(s, mp, l);
#pragma unroll
      for (int r = 0; r < 4; ++r) ob[lds_off<P>(rows[r], c, KS)] = (T)hv[r];
    }
    if (!mp.lds_h) {
      acc* hp = hsave_at<P, MT>(hsave, l - 1, RT, rt, ct, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) __builtin_nontemporal_store(hv[r], hp + r);
    }
    if (last) {
#pragma unroll
      for (int r = 0; r < 4; ++r) po[ct] += Wo[rows[r]] * hv[r];
      if (fuse_delta && nh > 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          s.dlt0[lds_off<P>(rows[r], c, KS)] = (T)(Wo[rows[r]] * ((acc)1 - hv[r] * hv[r]));
      }
    }
    if (ex && c < ex->mvalid) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        ex->h[((int64_t)(l - 1) * H + rows[r]) * ex->ldb + ex->col0 + c] = (float)hv[r];
    }
  };

  // ---- layer 1: K = d (zero padded) on FP32 / FP64 MFMA ----
  {
    auto epi1 = [&](int rt, int ct, const typename IP::accv& v) {
      acc hv[4];
      int rows[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rows[r] = rt * 16 + IP::drow(g, r);
        hv[r] = act_tanh((acc)v[r] + Bs[rows[r]]);
      }
      finish(1, rt, ct, hv, rows);
    };
    for (int rr = 0; rr < RTW; ++rr)
      gemm_short<IP, MT>((const typename IP::T*)mp.w1f, mp.ks1, s.thf, wv * RTW + rr, epi1);
  }
  __syncthreads();

  // ---- hidden layers 2..nh ----
  for (int l = 2; l <= nh; ++l) {
    const T* Bin = layer_buf<P, MT>(s, mp, l - 1);
    const T* A = (const T*)mp.wf + (int64_t)(l - 2) * H * H;
    const acc* bl = Bs + (int64_t)(l - 1) * H;
    auto epi = [&](int rt, int ct, const accv& v) {
      acc hv[4];
      int rows[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rows[r] = rt * 16 + P::drow(g, r);
        hv[r] = act_tanh((acc)v[r] + bl[rows[r]]);
      }
      finish(l, rt, ct, hv, rows);
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
  using frag = typename P::frag;
  constexpr int M = 16 * MT;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, wv = tid >> 6, cl = lane & 15;
  const int d = mp.d, H = mp.H, nh = mp.nh;
  const int KS = H / P::KSTEP, RTW = H / (16 * kWaves);
  const acc* __restrict__ Wo = (const acc*)mp.wout;

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
        for (int r = 0; r < 4; ++r) {
          const int j = rt * 16 + P::drow(g, r);
          dl[r] = u * Wo[j] * ((acc)1 - hv[r] * hv[r]);
          s.dlt0[lds_off<P>(j, c, KS)] = (T)dl[r];
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
    auto epi = [&](int rt, int ct, const accv& v) {
      const int c = ct * 16 + cl;
      acc hv[4], dl[4];
      load_h<P, MT>(s, mp, hsave, l - 1, rt, ct, hv);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dl[r] = (acc)v[r] * ((acc)1 - hv[r] * hv[r]);
        Bout[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)dl[r];
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

  // ---- d out / d t = W_1^T delta_1: the K = H k-steps are dealt to the waves round-robin
  // (wave w takes w, w + 8, ...) and the 8 partial tiles are summed in wave order ----
  if (want_input_grad) {
    // delta_1 is the output of the last hidden-layer step above, or delta_L if nh == 1
    const T* d1 = (((nh - 1) & 1) == 0) ? s.dlt0 : s.dlt1;
    const frag* __restrict__ Af = (const frag*)mp.w1t;
    const frag* __restrict__ Bf = (const frag*)d1;
    for (int rt = 0; rt < mp.rti; ++rt) {
      accv part[MT];
#pragma unroll
      for (int ct = 0; ct < MT; ++ct) part[ct] = accv{};
      for (int ks = wv; ks < KS; ks += kWaves) {
        const frag a = Af[((int64_t)rt * KS + ks) * 64 + lane];
#pragma unroll
        for (int ct = 0; ct < MT; ++ct)
          part[ct] = P::mma(a, Bf[(ct * KS + ks) * 64 + lane], part[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < MT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rt * 16 + P::drow(g, r);
          if (i < d) s.red[(wv * M + ct * 16 + cl) * d + i] = (acc)part[ct][r];
        }
    }
    __syncthreads();
    for (int e = tid; e < M * d; e += kThreads) {
      acc v = s.red[e];
      for (int w = 1; w < kWaves; ++w) v += s.red[w * M * d + e];
      s.gth[e] = (vec)v;
    }
    __syncthreads();
  }
}

}  // namespace best
