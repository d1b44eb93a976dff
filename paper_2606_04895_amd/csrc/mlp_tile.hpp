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

#ifndef BEST_PREFETCH
#define BEST_PREFETCH 4
#endif
constexpr int kPrefetch = BEST_PREFETCH;  // k-steps of weight fragments in flight per wave
// Wider chain tiles issue MT MFMAs per weight fragment, so a shallower ring keeps the stream
// fed and leaves the registers to the MT accumulators and activation fragments.
#ifndef BEST_PREFETCH_WIDE
#define BEST_PREFETCH_WIDE 4
#endif
template <int MT>
constexpr int prefetch_depth() {
  return MT >= 2 ? BEST_PREFETCH_WIDE : kPrefetch;
}
// Row tiles per register group: 4 with a whole register file per wave, 2 when two waves
// share a SIMD.
#ifndef BEST_RG_MAX
#define BEST_RG_MAX (kWaves > 4 ? 2 : 4)
#endif
constexpr int kRgMax = BEST_RG_MAX;
// Per-row-tile epilogue operands loaded before the k-loop: bias and output weights (8) in
// the forward pass, the saved activations of the MT chain tiles (4 MT) in the backward.
template <int MT>
constexpr int kPV = 4 * MT > 8 ? 4 * MT : 8;

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
  typename P::acc* red;              // [kWaves][M][d] input-gradient partial sums
  typename P::acc* outp;             // [kWaves][M] output partial sums
  typename P::acc* out;              // [M]
  typename P::acc* up;               // [M] upstream gradient, NULL means 1
};

// threadIdx.x behind an empty asm: per-lane addresses derived from it are recomputed where
// they are used instead of being hoisted out of the sampler loops, where they would stay
// live across the whole kernel (and spill).
__device__ __forceinline__ int local_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <class P>
__host__ __device__ __forceinline__ int lds_off(int k, int c, int KS) {
  return (int)frag_offset<P>(c, k, KS);  // B fragments: column = chain, k = neuron
}

// Input component i of chain c (the caller also writes the zero padding i in [d, 16 ks1)).
template <class P>
__device__ __forceinline__ void store_t(const MlpSmem<P>& s, const MlpParams& mp, int c, int i,
                                        double v) {
  using IP = typename InPrec<P>::type;
  s.thf[frag_offset<IP>(c, i, mp.ks1)] = (typename IP::T)v;
}

// A pass of n_layers GEMMs over this wave's RTW row tiles (rtw0 ..), in register groups of
// RG row tiles x MT chain tiles over KS k-steps (KS a multiple of kPrefetch).  Layer li
// multiplies Aof(li) (fragment-ordered weights) by Bof(li) (B fragments in LDS).
//   * The A fragments of the next kPrefetch k-steps are always in flight; the ring has no
//     conditional loads inside the k-loop, so the waits stay partial.
//   * When a group's last MFMAs are issued, the ring is refilled with the first k-steps of
//     the next group (or of the next layer's first group) before the epilogue runs, so the
//     weight stream continues through epilogues and layer barriers.
//   * pre(li, rt, v) loads per-row epilogue operands (bias, output weights) before the
//     k-loop; each layer's first group joins the workgroup barrier that publishes its B
//     operand after its loads are issued.
template <class P, int RG, int MT, class AOf, class BOf, class Pre, class Epi>
__device__ __forceinline__ void gemm_pass_rg(int n_layers, int KS, int rtw0, int RTW, AOf& Aof,
                                             BOf& Bof, Pre& pre, Epi& epi) {
  using T = typename P::T;
  using frag = typename P::frag;
  using accv = typename P::accv;
  using acc = typename P::acc;
  constexpr int D = prefetch_depth<MT>();
  const int lane = local_tid() & 63;
  const int ng = RTW / RG;
  frag a[D][RG];
  auto prologue = [&](const T* A, int rt0) {
    const frag* __restrict__ Af = reinterpret_cast<const frag*>(A) + (int64_t)rt0 * KS * 64 + lane;
#pragma unroll
    for (int p = 0; p < D; ++p)
#pragma unroll
      for (int rr = 0; rr < RG; ++rr) a[p][rr] = Af[((int64_t)rr * KS + p) * 64];
  };
  prologue(Aof(0), rtw0);
  for (int li = 0; li < n_layers; ++li) {
    const T* A = Aof(li);
    const frag* __restrict__ Bf = reinterpret_cast<const frag*>(Bof(li)) + lane;
    for (int gi = 0; gi < ng; ++gi) {
      const int rt0 = rtw0 + gi * RG;
      const frag* __restrict__ Af = reinterpret_cast<const frag*>(A) + (int64_t)rt0 * KS * 64 + lane;
      acc pv[RG][kPV<MT>];
#pragma unroll
      for (int rr = 0; rr < RG; ++rr) pre(li, rt0 + rr, pv[rr]);
      if (gi == 0) __syncthreads();
      accv c[RG][MT];
#pragma unroll
      for (int rr = 0; rr < RG; ++rr)
#pragma unroll
        for (int ct = 0; ct < MT; ++ct) c[rr][ct] = accv{};
      // B fragments are double-buffered: the LDS read of k-step ks + 1 is issued before the
      // MFMAs of k-step ks
      frag b[MT];
#pragma unroll
      for (int ct = 0; ct < MT; ++ct) b[ct] = Bf[ct * KS * 64];
      auto step = [&](int ks, int p, bool next) {
        frag bn[MT];
        if (next) {
#pragma unroll
          for (int ct = 0; ct < MT; ++ct) bn[ct] = Bf[(ct * KS + ks + 1) * 64];
        }
#pragma unroll
        for (int rr = 0; rr < RG; ++rr)
#pragma unroll
          for (int ct = 0; ct < MT; ++ct) c[rr][ct] = P::mma(a[p][rr], b[ct], c[rr][ct]);
        if (next) {
#pragma unroll
          for (int ct = 0; ct < MT; ++ct) b[ct] = bn[ct];
        }
      };
      int k0 = 0;
      for (; k0 < KS - D; k0 += D) {
#pragma unroll
        for (int p = 0; p < D; ++p) {
          step(k0 + p, p, true);
#pragma unroll
          for (int rr = 0; rr < RG; ++rr) a[p][rr] = Af[((int64_t)rr * KS + k0 + p + D) * 64];
        }
      }
#pragma unroll
      for (int p = 0; p < D; ++p) step(k0 + p, p, p + 1 < D);
      if (gi + 1 < ng) prologue(A, rt0 + RG);
      else if (li + 1 < n_layers) prologue(Aof(li + 1), rtw0);
#pragma unroll
      for (int rr = 0; rr < RG; ++rr)
#pragma unroll
        for (int ct = 0; ct < MT; ++ct) epi(li, rt0 + rr, ct, c[rr][ct], pv[rr]);
    }
  }
}

template <class P, int MT, class AOf, class BOf, class Pre, class Epi>
__device__ __forceinline__ void gemm_pass(int n_layers, int KS, int rtw0, int RTW, AOf& Aof,
                                          BOf& Bof, Pre& pre, Epi& epi) {
  if (n_layers <= 0) return;
  if (kRgMax >= 4 && RTW % 4 == 0)
    gemm_pass_rg<P, (kRgMax >= 4 ? 4 : 2), MT>(n_layers, KS, rtw0, RTW, Aof, Bof, pre, epi);
  else if (RTW % 2 == 0) gemm_pass_rg<P, 2, MT>(n_layers, KS, rtw0, RTW, Aof, Bof, pre, epi);
  else gemm_pass_rg<P, 1, MT>(n_layers, KS, rtw0, RTW, Aof, Bof, pre, epi);
}

// Input layer for RG row tiles: all A fragments (KS <= KS1 k-steps) and the bias rows are
// loaded before the optional barrier, then the MFMAs and the epilogue run.
constexpr int kMaxKs1 = 4;  // d <= 32: 2 k-steps of FP32 MFMA, 4 of FP64 MFMA
template <class IP, int RG, int MT, int KS1, class Pre, class Epi>
__device__ __forceinline__ void gemm_in(const typename IP::T* __restrict__ A, int KS,
                                        const typename IP::T* __restrict__ Bl, int rt0,
                                        Pre& pre, Epi& epi, bool sync) {
  using frag = typename IP::frag;
  using accv = typename IP::accv;
  using acc = typename IP::acc;
  const int lane = local_tid() & 63;
  const frag* __restrict__ Af = reinterpret_cast<const frag*>(A) + (int64_t)rt0 * KS * 64 + lane;
  const frag* __restrict__ Bf = reinterpret_cast<const frag*>(Bl) + lane;
  frag a[KS1][RG];
#pragma unroll
  for (int ks = 0; ks < KS1; ++ks)
#pragma unroll
    for (int rr = 0; rr < RG; ++rr)
      if (ks < KS) a[ks][rr] = Af[((int64_t)rr * KS + ks) * 64];
  acc pv[RG][8];
#pragma unroll
  for (int rr = 0; rr < RG; ++rr) pre(rt0 + rr, pv[rr]);
  if (sync) __syncthreads();
  accv c[RG][MT];
#pragma unroll
  for (int rr = 0; rr < RG; ++rr)
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) c[rr][ct] = accv{};
#pragma unroll
  for (int ks = 0; ks < KS1; ++ks) {
    if (ks < KS) {
#pragma unroll
      for (int ct = 0; ct < MT; ++ct) {
        const frag b = Bf[(ct * KS + ks) * 64];
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) c[rr][ct] = IP::mma(a[ks][rr], b, c[rr][ct]);
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < RG; ++rr)
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) epi(rt0 + rr, ct, c[rr][ct], pv[rr]);
}

// Input layer over this wave's RTW row tiles: eight at once when the input fits one k-step.
template <class IP, int MT, class Pre, class Epi>
__device__ __forceinline__ void gemm_in_rows(const typename IP::T* A, int KS,
                                             const typename IP::T* Bl, int rtw0, int RTW,
                                             Pre& pre, Epi& epi, bool sync) {
  if (KS == 1 && RTW % 8 == 0) {
    for (int r = 0; r < RTW; r += 8)
      gemm_in<IP, 8, MT, 1>(A, KS, Bl, rtw0 + r, pre, epi, sync && r == 0);
  } else if (RTW % 4 == 0) {
    for (int r = 0; r < RTW; r += 4)
      gemm_in<IP, 4, MT, kMaxKs1>(A, KS, Bl, rtw0 + r, pre, epi, sync && r == 0);
  } else if (RTW % 2 == 0) {
    gemm_in<IP, 2, MT, kMaxKs1>(A, KS, Bl, rtw0, pre, epi, sync);
  } else {
    gemm_in<IP, 1, MT, kMaxKs1>(A, KS, Bl, rtw0, pre, epi, sync);
  }
}

// tanh(y) = 1 - 2 / (1 + exp(2y)) on the hardware exp and reciprocal (absolute error about
// 2e-7, below the FP32 rounding of the layer sums; saturates to +-1 without overflow); the
// FP64 path uses the library tanh.
__device__ __forceinline__ float act_tanh(float y) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * y));
}
__device__ __forceinline__ double act_tanh(double y) { return tanh(y); }

// Store / load the four D-slot values of one lane (rows rt*16 + drow(g, r), chain c) in a
// B-fragment LDS buffer.  For the FP32-class layouts the four rows are consecutive k of one
// fragment slot, so they move as one 8- or 16-byte access.
template <class P>
__device__ __forceinline__ void lds_store4(typename P::T* buf, int rt, int g, int c, int KS,
                                           const typename P::acc v[4]) {
  using T = typename P::T;
  if constexpr (P::ROWS4) {
    typedef T t4 __attribute__((ext_vector_type(4)));
    const t4 w = {(T)v[0], (T)v[1], (T)v[2], (T)v[3]};
    *reinterpret_cast<t4*>(buf + lds_off<P>(rt * 16 + 4 * g, c, KS)) = w;
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) buf[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)] = (T)v[r];
  }
}
template <class P>
__device__ __forceinline__ void lds_load4(const typename P::T* buf, int rt, int g, int c, int KS,
                                          typename P::acc v[4]) {
  using T = typename P::T;
  using acc = typename P::acc;
  if constexpr (P::ROWS4) {
    typedef T t4 __attribute__((ext_vector_type(4)));
    const t4 w = *reinterpret_cast<const t4*>(buf + lds_off<P>(rt * 16 + 4 * g, c, KS));
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (acc)w[r];
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (acc)buf[lds_off<P>(rt * 16 + P::drow(g, r), c, KS)];
  }
}

// Per-tile activation scratch in D-tile order: [layer][rt][ct][lane][4].
template <int MT>
__host__ __device__ __forceinline__ int64_t hsave_index(int layer, int RT, int rt, int ct,
                                                        int lane) {
  return ((((int64_t)layer * RT + rt) * MT + ct) * 64 + lane) * 4;
}
template <class P, int MT>
__device__ __forceinline__ typename P::acc* hsave_at(typename P::acc* base, int layer, int RT,
                                                     int rt, int ct, int lane) {
  return base + hsave_index<MT>(layer, RT, rt, ct, lane);
}

// Buffers of the tile engine for a given storage mode (the caller sets thf, gth, red, outp,
// out and up).
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
  const int lane = local_tid() & 63, g = lane >> 4, cl = lane & 15;
  const int KS = mp.H / P::KSTEP, RT = mp.H / 16;
  if (mp.lds_h) {
    lds_load4<P>(layer_buf<P, MT>(s, mp, l), rt, g, ct * 16 + cl, KS, h);
  } else {
    typedef acc a4 __attribute__((ext_vector_type(4)));
    const a4 w = __builtin_nontemporal_load(
        reinterpret_cast<const a4*>(hsave_at<P, MT>(hsave, l - 1, RT, rt, ct, lane)));
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = w[r];
  }
}

// The four rows rt*16 + drow(g, r) of a row-indexed vector, in this lane's D-slot order.
template <class Q, class V>
__device__ __forceinline__ void load_rows(const V* __restrict__ base, int rt, int g, V v[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = base[rt * 16 + Q::drow(g, r)];
}

// Forward pass.  Reads the input from s.thf and leaves out = w_out . h_L + b_out in s.out.
//   fuse_delta: the last layer's epilogue also writes delta_L = w_out (1 - h_L^2) (upstream
//               1) into s.dlt0 for mlp_backward;
//   sync_in:    the caller wrote s.thf without a barrier; the input layer joins one after
//               issuing its weight loads;
//   defer_out:  leave the per-wave output partials in s.outp and return without a barrier;
//               mlp_backward(..., finish_out) completes s.out.
template <class P, int MT>
__device__ __forceinline__ void mlp_forward(const MlpParams& mp, const MlpSmem<P>& s,
                                            typename P::acc* __restrict__ hsave,
                                            const MlpExport* ex, bool fuse_delta, bool sync_in,
                                            bool defer_out) {
  using T = typename P::T;
  using acc = typename P::acc;
  using accv = typename P::accv;
  using IP = typename InPrec<P>::type;
  constexpr int M = 16 * MT;
  const int tid = local_tid(), lane = tid & 63, g = lane >> 4, wv = tid >> 6, cl = lane & 15;
  const int H = mp.H, nh = mp.nh;
  const int KS = H / P::KSTEP, RTW = H / (16 * kWaves), RT = H / 16;
  const acc* __restrict__ Bs = (const acc*)mp.bias;
  const acc* __restrict__ Wo = (const acc*)mp.wout;
  acc po[MT];
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) po[ct] = 0;

  // epilogue shared by every layer (hv[r] is row rows[r] of chain ct*16 + cl, wo[r] the
  // output weight of that row at the last layer): save h_l, feed layer l+1, and at the last
  // layer the output dot product and (optionally) delta_L.  The D layouts of the input-layer
  // and hidden-layer instructions coincide (FP32-class: rows 4g + r, FP64: rows g + 4r), so
  // the saved slots read back the same way.
  auto finish = [&](int l, int rt, int ct, const acc hv[4], const int rows[4], const acc* wo) {
    const int c = ct * 16 + cl;
    const bool last = (l == nh);
    if (mp.lds_h || !last) lds_store4<P>(layer_buf<P, MT>(s, mp, l), rt, g, c, KS, hv);
    if (!mp.lds_h) {
      typedef acc a4 __attribute__((ext_vector_type(4)));
      const a4 w = {hv[0], hv[1], hv[2], hv[3]};
      __builtin_nontemporal_store(w, reinterpret_cast<a4*>(hsave_at<P, MT>(hsave, l - 1, RT, rt, ct, lane)));
    }
    if (last) {
#pragma unroll
      for (int r = 0; r < 4; ++r) po[ct] += wo[r] * hv[r];
      if (fuse_delta && nh > 1) {
        acc dl[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) dl[r] = wo[r] * ((acc)1 - hv[r] * hv[r]);
        lds_store4<P>(s.dlt0, rt, g, c, KS, dl);
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
    auto pre1 = [&](int rt, acc* v) {
      load_rows<IP>(Bs, rt, g, v);
      if (nh == 1) load_rows<IP>(Wo, rt, g, v + 4);
    };
    auto epi1 = [&](int rt, int ct, const typename IP::accv& v, const acc* pv) {
      acc hv[4];
      int rows[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rows[r] = rt * 16 + IP::drow(g, r);
        hv[r] = act_tanh((acc)v[r] + pv[r]);
      }
      finish(1, rt, ct, hv, rows, pv + 4);
    };
    gemm_in_rows<IP, MT>((const typename IP::T*)mp.w1f, mp.ks1, s.thf, wv * RTW, RTW, pre1, epi1,
                         sync_in);
  }

  // ---- hidden layers 2..nh (layer li + 2; each joins the barrier that publishes the
  // previous layer) ----
  {
    auto Aof = [&](int li) { return (const T*)mp.wf + (int64_t)li * H * H; };
    auto Bof = [&](int li) { return (const T*)layer_buf<P, MT>(s, mp, li + 1); };
    auto pre = [&](int li, int rt, acc* v) {
      load_rows<P>(Bs + (int64_t)(li + 1) * H, rt, g, v);
      if (li + 2 == nh) load_rows<P>(Wo, rt, g, v + 4);
    };
    auto epi = [&](int li, int rt, int ct, const accv& v, const acc* pv) {
      acc hv[4];
      int rows[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rows[r] = rt * 16 + P::drow(g, r);
        hv[r] = act_tanh((acc)v[r] + pv[r]);
      }
      finish(li + 2, rt, ct, hv, rows, pv + 4);
    };
    gemm_pass<P, MT>(nh - 1, KS, wv * RTW, RTW, Aof, Bof, pre, epi);
  }

  // ---- output layer: per-wave partial dot products, summed in wave order ----
#pragma unroll
  for (int ct = 0; ct < MT; ++ct) {
    const acc v = sum_lane_groups(po[ct]);
    if (g == 0) s.outp[wv * M + ct * 16 + cl] = v;
  }
  if (defer_out) return;
  __syncthreads();
  if (tid < M) {
    acc o = s.outp[tid];
    for (int w = 1; w < kWaves; ++w) o += s.outp[w * M + tid];
    s.out[tid] = o + Wo[H];
  }
  __syncthreads();
}

// Backward pass (reverse mode).  s.up (or 1) is the upstream gradient per chain; if the
// forward fused delta_L, s.up must be NULL.  If want_input_grad, writes
// s.gth[c][i] = d(up * out)/d t_i; if finish_out, completes s.out from the partials a
// deferred forward left.  Ends with a barrier.
template <class P, int MT>
__device__ __forceinline__ void mlp_backward(const MlpParams& mp, const MlpSmem<P>& s,
                                             typename P::acc* __restrict__ hsave,
                                             const MlpExport* ex, bool want_input_grad,
                                             bool delta_fused, bool finish_out) {
  using T = typename P::T;
  using acc = typename P::acc;
  using vec = typename P::vec;
  using accv = typename P::accv;
  using frag = typename P::frag;
  constexpr int M = 16 * MT;
  const int tid = local_tid(), lane = tid & 63, g = lane >> 4, wv = tid >> 6, cl = lane & 15;
  const int d = mp.d, H = mp.H, nh = mp.nh;
  const int KS = H / P::KSTEP, RTW = H / (16 * kWaves);
  const acc* __restrict__ Wo = (const acc*)mp.wout;

  // ---- delta_L = up * w_out * (1 - h_L^2), unless the forward epilogue wrote it ----
  if (!delta_fused || nh == 1) {
    for (int rr = 0; rr < RTW; ++rr) {
      const int rt = wv * RTW + rr;
      acc wo[4];
      load_rows<P>(Wo, rt, g, wo);
      for (int ct = 0; ct < MT; ++ct) {
        const int c = ct * 16 + cl;
        const acc u = s.up ? s.up[c] : (acc)1;
        acc hv[4], dl[4];
        load_h<P, MT>(s, mp, hsave, nh, rt, ct, hv);
#pragma unroll
        for (int r = 0; r < 4; ++r) dl[r] = u * wo[r] * ((acc)1 - hv[r] * hv[r]);
        lds_store4<P>(s.dlt0, rt, g, c, KS, dl);
        if (ex && c < ex->mvalid) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            ex->dl[((int64_t)(nh - 1) * H + rt * 16 + P::drow(g, r)) * ex->ldb + ex->col0 + c] =
                (float)dl[r];
        }
      }
    }
  }

  // ---- hidden layers nh..2 (layer nh - li): D[k][c] = sum_j W_l^T[k][j] delta_l[j][c] ----
  {
    auto Aof = [&](int li) { return (const T*)mp.wb + (int64_t)(nh - 2 - li) * H * H; };
    auto Bof = [&](int li) { return (const T*)((li & 1) == 0 ? s.dlt0 : s.dlt1); };
    // saved activations in the global scratch are loaded with the group's weights, so the
    // epilogue never waits behind the weight stream
    auto pre = [&](int li, int rt, acc* v) {
      if (!mp.lds_h) {
#pragma unroll
        for (int ct = 0; ct < MT; ++ct) load_h<P, MT>(s, mp, hsave, nh - li - 1, rt, ct, v + 4 * ct);
      }
    };
    auto epi = [&](int li, int rt, int ct, const accv& v, const acc* pv) {
      const int l = nh - li, c = ct * 16 + cl;
      T* Bout = (li & 1) == 0 ? s.dlt1 : s.dlt0;
      acc hv[4], dl[4];
      if (mp.lds_h) {
        load_h<P, MT>(s, mp, hsave, l - 1, rt, ct, hv);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) hv[r] = pv[4 * ct + r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) dl[r] = (acc)v[r] * ((acc)1 - hv[r] * hv[r]);
      lds_store4<P>(Bout, rt, g, c, KS, dl);
      if (ex && c < ex->mvalid) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ex->dl[((int64_t)(l - 2) * H + rt * 16 + P::drow(g, r)) * ex->ldb + ex->col0 + c] =
              (float)dl[r];
      }
    };
    gemm_pass<P, MT>(nh - 1, KS, wv * RTW, RTW, Aof, Bof, pre, epi);
  }

  // ---- d out / d t = W_1^T delta_1: the K = H k-steps are dealt to the waves round-robin
  // (wave w takes w, w + 8, ...) and the 8 partial tiles are summed in wave order; the
  // first row tile's leading fragments are loaded before the barrier ----
  // per-wave partial sums (the layout places them in the delta buffer that does not hold
  // delta_1 when they fit there)
  acc* red = s.red;
  if (want_input_grad) {
    // delta_1 is the output of the last hidden-layer step above, or delta_L if nh == 1
    const T* d1 = (((nh - 1) & 1) == 0) ? s.dlt0 : s.dlt1;
    const frag* __restrict__ Af = (const frag*)mp.w1t + lane;
    const frag* __restrict__ Bf = (const frag*)d1 + lane;
    constexpr int PF = 4;
    frag a0[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int ks = wv + q * kWaves;
      if (ks < KS) a0[q] = Af[(int64_t)ks * 64];
    }
    __syncthreads();
    for (int rt = 0; rt < mp.rti; ++rt) {
      accv part[MT];
#pragma unroll
      for (int ct = 0; ct < MT; ++ct) part[ct] = accv{};
      int ks = wv;
      if (rt == 0) {
#pragma unroll
        for (int q = 0; q < PF; ++q, ks += kWaves) {
          if (ks < KS) {
#pragma unroll
            for (int ct = 0; ct < MT; ++ct)
              part[ct] = P::mma(a0[q], Bf[(ct * KS + ks) * 64], part[ct]);
          }
        }
      }
      for (; ks < KS; ks += kWaves) {
        const frag a = Af[((int64_t)rt * KS + ks) * 64];
#pragma unroll
        for (int ct = 0; ct < MT; ++ct) part[ct] = P::mma(a, Bf[(ct * KS + ks) * 64], part[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < MT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rt * 16 + P::drow(g, r);
          if (i < d) red[(wv * M + ct * 16 + cl) * d + i] = (acc)part[ct][r];
        }
    }
  }
  __syncthreads();
  if (want_input_grad) {
    for (int e = tid; e < M * d; e += kThreads) {
      acc v = red[e];
      for (int w = 1; w < kWaves; ++w) v += red[w * M * d + e];
      s.gth[e] = (vec)v;
    }
  }
  if (finish_out && tid < M) {
    acc o = s.outp[tid];
    for (int w = 1; w < kWaves; ++w) o += s.outp[w * M + tid];
    s.out[tid] = o + Wo[H];
  }
  if (want_input_grad || finish_out) __syncthreads();
}

}  // namespace best
