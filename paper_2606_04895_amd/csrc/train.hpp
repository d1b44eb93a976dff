// Templated kernels for weight packing and emulator training (forward + MSE upstream +
// backward for one chain tile of the minibatch, exporting activations and deltas).
#pragma once
#include "kernels.hpp"

namespace best {

// Flat FP64 parameters -> packed device copies used by the tile engine:
//   wf: W_l in fragment order (rows = outputs), wb: W_l^T in fragment order (l >= 2),
//   w1f: W_1 in the input layer's fragment order (k = input component, zero padded),
//   w1t: W_1^T in fragment order (rows = input components, zero padded to 16 rti),
//   bias: [nh][H], wout: [H] followed by b_out.
// Rounding of a parameter to a storage type: FP64 kept, FP32 round-to-nearest, the 16-bit
// types via FP32.
template <class T>
__device__ __forceinline__ T to_store(double v) {
  if constexpr (sizeof(T) == 8) return (T)v;
  else return (T)(float)v;
}

template <class P>
__global__ void pack_kernel(const double* flat, int d, int H, int nh, typename P::T* wf,
                            typename P::T* wb, void* w1f_, typename P::T* w1t,
                            typename P::acc* bias, typename P::acc* wout) {
  using T = typename P::T;
  using IP = typename InPrec<P>::type;
  typename IP::T* w1f = (typename IP::T*)w1f_;
  const int64_t HH = (int64_t)H * H;
  const int64_t nW = (int64_t)(nh - 1) * HH;
  const int64_t ks1 = (d + IP::KSTEP - 1) / IP::KSTEP, K1 = ks1 * IP::KSTEP;
  const int64_t R1 = (d + 15) / 16 * 16;
  const int64_t n1f = (int64_t)H * K1, n1t = R1 * H;
  const int64_t total = nW + n1f + n1t + (int64_t)nh * H + H + 1;
  const int64_t KS = H / P::KSTEP;
  const int64_t offb1 = (int64_t)H * d;
  const int64_t blk = HH + H;  // one hidden block W_l + b_l (l >= 2)
  const int64_t offwo = offb1 + H + (int64_t)(nh - 1) * blk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nW) {
      const int64_t l = e / HH, q = e % HH, j = q / H, k = q % H;  // layer l + 2
      const double v = flat[offb1 + H + l * blk + j * H + k];
      wf[l * HH + frag_offset<P>(j, k, KS)] = to_store<T>(v);
      wb[l * HH + frag_offset<P>(k, j, KS)] = to_store<T>(v);
    } else if (e < nW + n1f) {
      const int64_t q = e - nW, j = q / K1, i = q % K1;
      w1f[frag_offset<IP>(j, i, ks1)] = to_store<typename IP::T>(i < d ? flat[j * d + i] : 0.0);
    } else if (e < nW + n1f + n1t) {
      const int64_t q = e - nW - n1f, i = q / H, j = q % H;
      w1t[frag_offset<P>(i, j, KS)] = to_store<T>(i < d ? flat[j * d + i] : 0.0);
    } else if (e < nW + n1f + n1t + (int64_t)nh * H) {
      const int64_t q = e - nW - n1f - n1t, l = q / H, j = q % H;
      const int64_t off = l == 0 ? offb1 : offb1 + H + (l - 1) * blk + HH;
      bias[q] = (typename P::acc)flat[off + j];
    } else {
      const int64_t j = e - nW - n1f - n1t - (int64_t)nh * H;
      wout[j] = (typename P::acc)flat[offwo + j];  // j == H is b_out
    }
  }
}

struct TrainArgs {
  MlpParams mp;
  LdsLayout lds;
  const float* t_in;
  const float* y;
  const int32_t* perm;
  int64_t batch0, B, n_tiles;
  void* hsave;
  int64_t hsave_stride;
  float *ex_h, *ex_dl, *ex_th, *ex_up;
  double* loss_part;
};

template <class P, int MT>
__global__ __launch_bounds__(kThreads, 1) void train_tile_kernel(TrainArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  using acc = typename P::acc;
  using vec = typename P::vec;
  using IP = typename InPrec<P>::type;
  constexpr int M = 16 * MT;
  const int tid = local_tid(), d = a.mp.d, K1 = a.mp.ks1 * IP::KSTEP;
  acc* hsave = (acc*)a.hsave + (int64_t)blockIdx.x * a.hsave_stride;
  MlpSmem<P> s = mlp_smem<P, MT>(smem + a.lds.big, a.mp);
  s.thf = (typename IP::T*)(smem + a.lds.th);
  s.gth = (vec*)(smem + a.lds.gth);
  s.red = (acc*)(smem + a.lds.red);
  s.outp = (acc*)(smem + a.lds.outp);
  s.out = (acc*)(smem + a.lds.out);
  s.up = (acc*)(smem + a.lds.up);
  double* r2 = (double*)(smem + a.lds.md);
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int64_t c0 = tile * M;
    const int mv = (int)((a.B - c0) < M ? (a.B - c0) : M);
    for (int e = tid; e < M * K1; e += kThreads) {
      const int c = e / K1, i = e % K1;
      float v = 0.f;
      if (c < mv && i < d) {
        v = a.t_in[(int64_t)a.perm[a.batch0 + c0 + c] * d + i];
        a.ex_th[(int64_t)i * a.B + c0 + c] = v;
      }
      store_t<P>(s, a.mp, c, i, v);
    }
    MlpExport ex{a.ex_h, a.ex_dl, a.B, c0, mv};
    mlp_forward<P, MT>(a.mp, s, hsave, &ex, false, true, false);
    if (tid < M) {
      double r = 0;
      if (tid < mv) r = (double)s.out[tid] - (double)a.y[a.perm[a.batch0 + c0 + tid]];
      const acc u = (acc)(2.0 * r / (double)a.B);
      s.up[tid] = u;
      if (tid < mv) a.ex_up[c0 + tid] = (float)u;
      r2[tid] = r * r;
    }
    __syncthreads();
    if (tid == 0) {
      double t = 0;
      for (int c = 0; c < M; ++c) t += r2[c];
      a.loss_part[tile] = t;
    }
    mlp_backward<P, MT>(a.mp, s, hsave, &ex, false, false, false);
  }
}

// Vector-Jacobian product of the target with respect to the MLP parameters: for points x
// ([d][pitch] FP64) and upstream weights w_c, the tile exports what the weight-gradient GEMMs
// need for sum_c w_c d log pi(x_c) / d theta: the normalised inputs t, the activations h_l,
// the deltas of the reverse pass started from u_c = mlp_coef * w_c (zero for a point whose
// log pi does not use the MLP: outside the training box with the plain fallback), and u.
// Arrays are column-major in the point index with leading dimension ldb (n rounded up to 16);
// the padding columns [n, ldb) are written as zeros so the GEMMs can run over ldb columns.
struct VjpArgs {
  Target tg;
  MlpParams mp;
  LdsLayout lds;
  const double* x;
  int64_t pitch, n, ldb, n_tiles;
  const double* upstream;  // [n] or NULL (all ones)
  void* hsave;
  int64_t hsave_stride;
  float *ex_h, *ex_dl, *ex_th, *ex_up;
};

template <class P, int MT>
__global__ __launch_bounds__(kThreads, 1) void vjp_tile_kernel(VjpArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  using acc = typename P::acc;
  using vec = typename P::vec;
  using IP = typename InPrec<P>::type;
  constexpr int M = 16 * MT;
  const Target& tg = a.tg;
  const int tid = local_tid(), d = a.mp.d, H = a.mp.H, nh = a.mp.nh;
  const int K1 = a.mp.ks1 * IP::KSTEP;
  acc* hsave = (acc*)a.hsave + (int64_t)blockIdx.x * a.hsave_stride;
  MlpSmem<P> s = mlp_smem<P, MT>(smem + a.lds.big, a.mp);
  s.thf = (typename IP::T*)(smem + a.lds.th);
  s.gth = (vec*)(smem + a.lds.gth);
  s.red = (acc*)(smem + a.lds.red);
  s.outp = (acc*)(smem + a.lds.outp);
  s.out = (acc*)(smem + a.lds.out);
  s.up = (acc*)(smem + a.lds.up);
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int64_t c0 = tile * M;
    const int mv = (int)((a.n - c0) < M ? (a.n - c0) : M);
    for (int e = tid; e < M * K1; e += kThreads) {
      const int c = e / K1, i = e % K1;
      double v = 0.0;
      if (c < mv && i < d) {
        v = (a.x[(int64_t)i * a.pitch + c0 + c] - tg.in_center[i]) * tg.in_invscale[i];
        a.ex_th[(int64_t)i * a.ldb + c0 + c] = (float)v;
      }
      store_t<P>(s, a.mp, c, i, v);
    }
    for (int c = tid; c < M; c += kThreads) {
      acc u = 0;
      if (c < mv) {
        bool use = tg.plain_mode == 0;
        if (tg.plain_mode == 1) {
          use = true;
          for (int i = 0; i < d; ++i) {
            const double xv = a.x[(int64_t)i * a.pitch + c0 + c];
            use = use && xv >= tg.train_lo[i] && xv <= tg.train_hi[i];
          }
        }
        const double w = a.upstream ? a.upstream[c0 + c] : 1.0;
        u = use ? (acc)(tg.mlp_coef * w) : (acc)0;
        a.ex_up[c0 + c] = (float)u;
      } else if (c0 + c < a.ldb) {
        // padding column: zero in every exported array
        a.ex_up[c0 + c] = 0.f;
        for (int i = 0; i < d; ++i) a.ex_th[(int64_t)i * a.ldb + c0 + c] = 0.f;
        for (int64_t r = 0; r < (int64_t)nh * H; ++r) {
          a.ex_h[r * a.ldb + c0 + c] = 0.f;
          a.ex_dl[r * a.ldb + c0 + c] = 0.f;
        }
      }
      s.up[c] = u;
    }
    MlpExport ex{a.ex_h, a.ex_dl, a.ldb, c0, mv};
    mlp_forward<P, MT>(a.mp, s, hsave, &ex, false, true, false);
    mlp_backward<P, MT>(a.mp, s, hsave, &ex, false, false, false);
  }
}

}  // namespace best
