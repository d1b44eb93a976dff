// Non-templated kernels: walker initialisation, re-whitening, dual averaging, statistics,
// ensemble moments + jittered Cholesky (Sec. 3.2), multi-chain autocovariances for ESS,
// Adam, and the training weight-gradient GEMMs.
#include <mutex>

#include "aux.hpp"

namespace best {

// ---- walker initialisation (Sec. 3.2: uniform / replicated / Gaussian / hypersphere) ---
__global__ void init_positions_kernel(Target tg, State S, Rng rng, int mode, const double* pt,
                                      double scale, const double* L0, uint64_t step) {
  const int d = tg.d;
  const int64_t n = (int64_t)d * S.N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / S.N);
    const int64_t c = e % S.N;
    double v;
    if (mode == 0) {
      const U4 b = rng.block(c, step, kStreamInit, 0, (uint32_t)(i >> 1));
      const double u = (i & 1) ? u52(b.z, b.w) : u52(b.x, b.y);
      v = tg.lower[i] + (tg.upper[i] - tg.lower[i]) * u;
    } else if (mode == 1) {
      v = pt[i];
    } else if (mode == 2) {
      double s = 0;
      for (int j = 0; j <= i; ++j) s += L0[i * d + j] * normal_dim(rng, c, step, kStreamInit, 1, j);
      v = pt[i] + scale * s;
    } else {
      // uniform in the unit ball: direction xi / |xi| from d normals (sub 2), radius U^(1/d)
      // from the first uniform of block 0 of sub 3; then mapped through L0 and scaled
      double nn = 0, s = 0;
      for (int j = 0; j < d; ++j) {
        const double xj = normal_dim(rng, c, step, kStreamInit, 2, j);
        nn += xj * xj;
        if (j <= i) s += L0[i * d + j] * xj;
      }
      const U4 b = rng.block(c, step, kStreamInit, 3, 0);
      const double r = pow(u52(b.x, b.y), 1.0 / (double)d);
      v = pt[i] + scale * r * s / sqrt(nn);
    }
    S.x[i * S.Np + c] = v;
  }
}

// z = L^{-1} (x - mu) by forward substitution, one thread per chain.
__global__ void rewhiten_kernel(State S, Whiten W, int d) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < S.N;
       c += (int64_t)gridDim.x * blockDim.x) {
    double zz[kMaxD];
    for (int i = 0; i < d; ++i) {
      double r = S.x[i * S.Np + c] - W.mu[i];
      for (int j = 0; j < i; ++j) r -= W.L[i * d + j] * zz[j];
      zz[i] = r / W.L[i * d + i];
      S.z[i * S.Np + c] = zz[i];
    }
  }
}

// Fixed-order block reduction of a double per thread (256 threads).
__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kAuxThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---- dual averaging (Hoffman & Gelman 2014) on the chain-mean acceptance -------------
// da = [mu, h_bar, log_eps_bar, m, eps, delta, gamma, t0, kappa]
__global__ void da_update_kernel(const double* step_prob, int64_t N, double* da) {
  __shared__ double sh[kAuxThreads];
  double v = 0;
  for (int64_t c = threadIdx.x; c < N; c += kAuxThreads) v += step_prob[c];
  const double mean = block_sum(v, sh) / (double)N;
  if (threadIdx.x == 0) {
    const double m = da[3] + 1.0;
    const double w = 1.0 / (m + da[7]);
    const double hb = (1.0 - w) * da[1] + w * (da[5] - mean);
    const double log_eps = da[0] - sqrt(m) / da[6] * hb;
    const double eta = pow(m, -da[8]);
    da[1] = hb;
    da[2] = eta * log_eps + (1.0 - eta) * da[2];
    da[3] = m;
    da[4] = exp(log_eps);
  }
}

// ---- per-call statistics: [accepted, nonfinite, oob] int64 + [sum_prob] -----------------
__global__ void stats_kernel(State S, int64_t* out_i, double* out_d) {
  __shared__ double sh[kAuxThreads];
  double a = 0, nf = 0, oob = 0, ne = 0, sp = 0;
  for (int64_t c = threadIdx.x; c < S.N; c += kAuxThreads) {
    a += S.n_acc[c];
    nf += S.n_nonfinite[c];
    oob += S.n_oob[c];
    ne += S.n_evals[c];
    sp += S.sum_prob[c];
  }
  a = block_sum(a, sh);
  nf = block_sum(nf, sh);
  oob = block_sum(oob, sh);
  ne = block_sum(ne, sh);
  sp = block_sum(sp, sh);
  if (threadIdx.x == 0) {
    out_i[0] = (int64_t)a;
    out_i[1] = (int64_t)nf;
    out_i[2] = (int64_t)oob;
    out_i[3] = (int64_t)ne;
    out_d[0] = sp;
  }
}

__global__ void aies_record_kernel(State S, int d, float* rec, int64_t slot, int64_t pitch) {
  const int64_t n = (int64_t)d * S.N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / S.N);
    const int64_t c = e % S.N;
    rec[(slot * d + i) * pitch + c] = (float)S.x[i * S.Np + c];
  }
}

// ---- ensemble moments, pass 1: per-block shifted sums over items ----------------------
// Items come from a float record [T][d][N] (item = t*N + c) or the FP64 state x [d][Np].
// The shift is one vector s_i (spitch 0) or one per chain, s_i(c) = shift[i*spitch + c].
// Slot p < d holds sum (v_i - s_i); slot d + pair(i, j), j <= i, holds sum of products.
__global__ void moments_partial_kernel(const float* rec, const double* xs, int64_t T,
                                       int64_t N, int64_t pitch, int d, const double* shift,
                                       int64_t spitch, double* part) {
  constexpr int kChunk = 128;
  __shared__ double v[kChunk][kMaxD + 1];
  const int np = d + d * (d + 1) / 2;
  const int64_t items = T * N;
  const int64_t per = (items + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = blockIdx.x * per, b1 = min(items, b0 + per);
  double accs[4] = {0, 0, 0, 0};  // np <= d + d(d+1)/2 = 560 <= 4 * 256
  for (int64_t base = b0; base < b1; base += kChunk) {
    const int64_t it = base + threadIdx.x;
    if (threadIdx.x < kChunk && it < b1) {
      const int64_t t = it / N, c = it % N;
      for (int i = 0; i < d; ++i) {
        const double x = rec ? (double)rec[(t * d + i) * pitch + c] : xs[i * pitch + c];
        v[threadIdx.x][i] = x - (spitch ? shift[i * spitch + c] : shift[i]);
      }
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kChunk, b1 - base);
    for (int k = 0; k < 4; ++k) {
      const int p = threadIdx.x + k * kAuxThreads;
      if (p >= np) break;
      int i, j;
      if (p < d) {
        i = p;
        j = -1;
      } else {
        int q = p - d;
        i = 0;
        while (q > i) {
          q -= i + 1;
          ++i;
        }
        j = q;
      }
      double s = 0;
      if (j < 0) {
        for (int r = 0; r < cnt; ++r) s += v[r][i];
      } else {
        for (int r = 0; r < cnt; ++r) s += v[r][i] * v[r][j];
      }
      accs[k] += s;
    }
    __syncthreads();
  }
  for (int k = 0; k < 4; ++k) {
    const int p = threadIdx.x + k * kAuxThreads;
    if (p < np) part[(int64_t)blockIdx.x * np + p] = accs[k];
  }
}

// Cholesky-Banachiewicz of a (d x d, row-major) into L; false if a pivot is not finite and
// above `floor` (numerical positive definiteness).
__device__ bool chol(const double* a, double* L, int d, double floor) {
  for (int i = 0; i < d * d; ++i) L[i] = 0;
  for (int i = 0; i < d; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = a[i * d + j];
      for (int k = 0; k < j; ++k) s -= L[i * d + k] * L[j * d + k];
      if (i == j) {
        if (!(s > floor) || !isfinite(s)) return false;
        L[i * d + i] = sqrt(s);
      } else {
        L[i * d + j] = s / L[j * d + j];
      }
    }
  }
  return true;
}

// Pass 2 (one block): mean, covariance, symmetrise, jittered Cholesky; on success writes
// the new whitening.  info = [status (0 ok / 1 not PD), jitter, logdet].
__global__ void moments_final_kernel(const double* part, int nblocks, int64_t count, int d,
                                     const double* shift, int update_mean, double* mu,
                                     double* Lout, double* info) {
  __shared__ double S[kMaxD * kMaxD];
  __shared__ double Lt[kMaxD * kMaxD];
  __shared__ double sum[kMaxD + kMaxD * (kMaxD + 1) / 2];
  const int np = d + d * (d + 1) / 2;
  for (int p = threadIdx.x; p < np; p += kAuxThreads) {
    double s = 0;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * np + p];
    sum[p] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double n = (double)count;
  int q = d;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j, ++q) {
      const double c = (sum[q] - sum[i] * sum[j] / n) / (n - 1.0);
      S[i * d + j] = c;
      S[j * d + i] = c;
    }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < i; ++j) {
      const double c = 0.5 * (S[i * d + j] + S[j * d + i]);
      S[i * d + j] = S[j * d + i] = c;
    }
  double jit = 0, scale = 0;
  for (int i = 0; i < d; ++i) scale += S[i * d + i];
  scale /= d;
  const double floor = isfinite(scale) ? 1e-12 * scale : 0.0;  // pivot floor
  bool ok = chol(S, Lt, d, floor);
  if (!ok) {
    double S0[kMaxD];
    for (int i = 0; i < d; ++i) S0[i] = S[i * d + i];
    for (double lam = 1e-10; lam <= 1e-2 * (1 + 1e-12) && !ok; lam *= 10.0) {
      jit = lam * scale;
      for (int i = 0; i < d; ++i) S[i * d + i] = S0[i] + jit;
      ok = chol(S, Lt, d, floor);
    }
  }
  if (!ok) {
    info[0] = 1;
    info[1] = jit;
    return;
  }
  double ld = 0;
  for (int i = 0; i < d; ++i) ld += log(Lt[i * d + i]);
  for (int i = 0; i < d * d; ++i) Lout[i] = Lt[i];
  if (update_mean)
    for (int i = 0; i < d; ++i) mu[i] = shift[i] + sum[i] / n;
  info[0] = 0;
  info[1] = jit;
  info[2] = ld;
}

// ---- ESS: per-chain mean and sum of squared deviations, thread per (param, chain) ------
__global__ void ess_chain_stats_kernel(const float* rec, int64_t T, int d, int64_t N,
                                       double* mean, double* ssq) {
  const int64_t n = (int64_t)d * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / N);
    const int64_t c = e % N;
    double s = 0;
    for (int64_t t = 0; t < T; ++t) s += rec[(t * d + i) * N + c];
    const double m = s / (double)T;
    double q = 0;
    for (int64_t t = 0; t < T; ++t) {
      const double y = rec[(t * d + i) * N + c] - m;
      q += y * y;
    }
    mean[e] = m;
    ssq[e] = q;
  }
}

// Sum over the 64 chains of a block of sum_s y_s y_{s+t} for t in [lag0, lag0 + kEssLB).
// grid = (ceil(N/64), d); LDS holds the two time windows of the block's chains.
__global__ __launch_bounds__(kAuxThreads) void ess_autocov_kernel(const float* rec,
                                                               const double* mean, int64_t T,
                                                               int d, int64_t N, int64_t lag0,
                                                               double* part) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  double* ya = (double*)smem;                      // [kEssTS][64]
  double* yb = ya + kEssTS * 64;                   // [kEssTS + kEssLB][64]
  const int cm = threadIdx.x & 63, lq = threadIdx.x >> 6;
  const int i = blockIdx.y;
  const int64_t c = (int64_t)blockIdx.x * 64 + cm;
  const bool valid = c < N;
  const double mc = valid ? mean[i * N + c] : 0.0;
  double acc[kEssLB / 4];
#pragma unroll
  for (int k = 0; k < kEssLB / 4; ++k) acc[k] = 0;
  for (int64_t s0 = 0; s0 < T; s0 += kEssTS) {
    for (int r = lq; r < kEssTS; r += 4) {
      const int64_t s = s0 + r;
      ya[r * 64 + cm] = (valid && s < T) ? (double)rec[(s * d + i) * N + c] - mc : 0.0;
    }
    for (int r = lq; r < kEssTS + kEssLB; r += 4) {
      const int64_t s = s0 + lag0 + r;
      yb[r * 64 + cm] = (valid && s < T) ? (double)rec[(s * d + i) * N + c] - mc : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kEssTS; ++r) {
      const double y0 = ya[r * 64 + cm];
#pragma unroll
      for (int k = 0; k < kEssLB / 4; ++k) acc[k] += y0 * yb[(r + lq + 4 * k) * 64 + cm];
    }
    __syncthreads();
  }
  // reduce over the 64 chains in a fixed order
  double* red = (double*)smem;  // [kEssLB][64]
#pragma unroll
  for (int k = 0; k < kEssLB / 4; ++k) red[(lq + 4 * k) * 64 + cm] = acc[k];
  __syncthreads();
  if (threadIdx.x < kEssLB) {
    double s = 0;
    for (int j = 0; j < 64; ++j) s += red[threadIdx.x * 64 + j];
    part[((int64_t)i * gridDim.x + blockIdx.x) * kEssLB + threadIdx.x] = s;
  }
}

// ---- fixed scratch of the entry points that allocate nothing ------------------------------
// One copy per GPU in the code object's global segment, held until the process ends.  Host
// code never passes this name to a kernel: the host-side symbol is not a device address.
// Kernels get the per-device address that noalloc_scratch_address resolved.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_address(int dev, double** p) {
  *p = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;  // resolved with its own device current
    void* q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[dev] = (double*)q;
  }
  *p = scratch_dev[dev];
  return hipSuccess;
}

// ---- layout conversion: dst[j][i] = src[i][j] for a rows x cols row-major source ----------
__global__ void transpose_kernel(const double* src, int64_t rows, int64_t cols, double* dst) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e % cols;
    dst[j * rows + i] = src[e];
  }
}

// ---- training inputs: t[c][i] = (x[i][c] - center[i]) invscale[i], FP64 SoA in, FP32 AoS out
__global__ void normalise_inputs_kernel(const double* x, int64_t n, int d, InputScaling sc,
                                        float* t) {
  const int64_t total = (int64_t)d * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / d;
    const int i = (int)(e % d);
    t[e] = (float)((x[(int64_t)i * n + c] - sc.center[i]) * sc.invscale[i]);
  }
}

// ---- training: Adam on the FP64 master parameters --------------------------------------
__global__ void adam_kernel(double* p, double* m, double* v, const double* g, int64_t n,
                            double lr, double b1, double b2, double eps, double c1,
                            double c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double ge = g[e];
    const double me = b1 * m[e] + (1.0 - b1) * ge;
    const double ve = b2 * v[e] + (1.0 - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const double mh = me / c1, vh = ve / c2;
    p[e] = p[e] - lr * mh / (sqrt(vh) + eps);
  }
}

// dW_l = delta_l h_{l-1}^T for l >= 2 on FP32 MFMA: A = delta [H][ldb], B = h [H][ldb],
// K = batch.  Workgroup tile 64 x 64, wave w owns rows [16 w, 16 w + 16).
__global__ __launch_bounds__(kAuxThreads) void dw_gemm_kernel(const float* dl, const float* h,
                                                           int64_t ldb, int64_t B, int H,
                                                           double* gW) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, cl = lane & 15;
  const int r0 = blockIdx.y * 64 + wv * 16, k0 = blockIdx.x * 64;
  f32x4 acc[4] = {};
  for (int64_t c = 0; c < B; c += 16) {
    const f32x4 a = *(const f32x4*)(dl + (int64_t)(r0 + cl) * ldb + c + 4 * g);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const f32x4 b = *(const f32x4*)(h + (int64_t)(k0 + ct * 16 + cl) * ldb + c + 4 * g);
      acc[ct] = Prec<float>::mma(a, b, acc[ct]);
    }
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      gW[(int64_t)(r0 + 4 * g + r) * H + k0 + ct * 16 + cl] = (double)acc[ct][r];
}

// dW_1 (H x d), all biases, w_out and b_out; one thread per output, sums over the batch.
__global__ void dsmall_kernel(const float* dl, const float* h, const float* th, const float* up,
                              int64_t ldb, int64_t B, int d, int H, int nh, double* grad,
                              const int64_t* offs) {
  // offs: [W1, b1, b2 .. b_nh, w_out, b_out] offsets into grad (nh + 3 entries)
  const int64_t n = (int64_t)H * d + (int64_t)nh * H + H + 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    if (e < (int64_t)H * d) {
      const int j = (int)(e / d), i = (int)(e % d);
      for (int64_t c = 0; c < B; ++c) s += (double)dl[(int64_t)j * ldb + c] * th[(int64_t)i * ldb + c];
      grad[offs[0] + e] = s;
    } else if (e < (int64_t)H * d + (int64_t)nh * H) {
      const int64_t q = e - (int64_t)H * d;
      const int l = (int)(q / H), j = (int)(q % H);
      for (int64_t c = 0; c < B; ++c) s += dl[((int64_t)l * H + j) * ldb + c];
      grad[offs[1 + l] + j] = s;
    } else if (e < (int64_t)H * d + (int64_t)nh * H + H) {
      const int j = (int)(e - (int64_t)H * d - (int64_t)nh * H);
      for (int64_t c = 0; c < B; ++c) s += (double)up[c] * h[((int64_t)(nh - 1) * H + j) * ldb + c];
      grad[offs[1 + nh] + j] = s;
    } else {
      for (int64_t c = 0; c < B; ++c) s += up[c];
      grad[offs[2 + nh]] = s;
    }
  }
}

__global__ void sum_kernel(const double* part, int n, double scale, double* out) {
  __shared__ double sh[kAuxThreads];
  double v = 0;
  for (int i = threadIdx.x; i < n; i += kAuxThreads) v += part[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) *out = v * scale;
}

// ---- standardisation and importance weights (fixed-order two-stage reductions) ---------
// mode 0: sum a;  1: sum (a - s)^2;  2: max (a - b);  3: sum e, sum e^2 with e = exp(a - b - s)
__global__ void reduce_partial_kernel(int mode, const double* a, const double* b, int64_t n,
                                      double s, double* part) {
  __shared__ double sh[kAuxThreads];
  __shared__ double sh2[kAuxThreads];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
  double v = mode == 2 ? -INFINITY : 0.0, v2 = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kAuxThreads) {
    if (mode == 0) v += a[i];
    else if (mode == 1) { const double r = a[i] - s; v += r * r; }
    else if (mode == 2) v = fmax(v, a[i] - b[i]);
    else { const double e = exp(a[i] - b[i] - s); v += e; v2 += e * e; }
  }
  sh[threadIdx.x] = v;
  sh2[threadIdx.x] = v2;
  __syncthreads();
  for (int k = kAuxThreads / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      if (mode == 2) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + k]);
      else sh[threadIdx.x] += sh[threadIdx.x + k];
      sh2[threadIdx.x] += sh2[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0];
    part[2 * blockIdx.x + 1] = sh2[0];
  }
}

__global__ void reduce_final_kernel(int mode, const double* part, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double v = mode == 2 ? -INFINITY : 0.0, v2 = 0.0;
  for (int k = 0; k < nb; ++k) {
    if (mode == 2) v = fmax(v, part[2 * k]);
    else v += part[2 * k];
    v2 += part[2 * k + 1];
  }
  out[0] = v;
  out[1] = v2;
}

__global__ void standardise_kernel(const double* y, int64_t n, const double* stats, float* out) {
  // stats = [sum, -, sum sq dev, -]: mean = sum / n, sigma = sqrt(sum sq dev / n)
  const double mu = stats[0] / (double)n, sig = sqrt(stats[2] / (double)n);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)((y[i] - mu) / sig);
}

__global__ void weights_kernel(const double* a, const double* b, int64_t n, const double* st,
                               double* w) {
  // st = [max, -, sum e, sum e^2]
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = exp(a[i] - b[i] - st[0]) / st[2];
}

}  // namespace best

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
namespace best {

static int grid_for(int64_t n) {
  int64_t g = (n + kAuxThreads - 1) / kAuxThreads;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

hipError_t launch_init_positions(const Target& tg, const State& S, const Rng& rng, int mode,
                                 const double* pt, double scale, const double* L0,
                                 uint64_t step, hipStream_t s) {
  hipLaunchKernelGGL(init_positions_kernel, dim3(grid_for((int64_t)tg.d * S.N)),
                     dim3(kAuxThreads), 0, s, tg, S, rng, mode, pt, scale, L0, step);
  return hipGetLastError();
}

hipError_t launch_rewhiten(const State& S, const Whiten& W, int d, hipStream_t s) {
  hipLaunchKernelGGL(rewhiten_kernel, dim3(grid_for(S.N)), dim3(kAuxThreads), 0, s, S, W, d);
  return hipGetLastError();
}

hipError_t launch_da_update(const double* step_prob, int64_t N, double* da, hipStream_t s) {
  hipLaunchKernelGGL(da_update_kernel, dim3(1), dim3(kAuxThreads), 0, s, step_prob, N, da);
  return hipGetLastError();
}

hipError_t launch_stats(const State& S, int64_t* out_i, double* out_d, hipStream_t s) {
  hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(kAuxThreads), 0, s, S, out_i, out_d);
  return hipGetLastError();
}

hipError_t launch_aies_record(const State& S, int d, float* rec, int64_t slot, int64_t pitch,
                              hipStream_t s) {
  hipLaunchKernelGGL(aies_record_kernel, dim3(grid_for((int64_t)d * S.N)), dim3(kAuxThreads), 0,
                     s, S, d, rec, slot, pitch);
  return hipGetLastError();
}

hipError_t launch_moments(const float* rec, const double* xs, int64_t T, int64_t N,
                          int64_t pitch, int d, const double* shift, double* part, int nblocks,
                          int update_mean, double* mu, double* L, double* info, hipStream_t s) {
  hipLaunchKernelGGL(moments_partial_kernel, dim3(nblocks), dim3(kAuxThreads), 0, s, rec, xs, T,
                     N, pitch, d, shift, (int64_t)0, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(kAuxThreads), 0, s, part, nblocks,
                     T * N, d, shift, update_mean, mu, L, info);
  return hipGetLastError();
}

hipError_t launch_moment_sums(const float* rec, const double* xs, int64_t T, int64_t N,
                              int64_t pitch, int d, const double* shift, int64_t spitch,
                              double* part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(moments_partial_kernel, dim3(nblocks), dim3(kAuxThreads), 0, s, rec, xs, T,
                     N, pitch, d, shift, spitch, part);
  return hipGetLastError();
}

hipError_t launch_ess_chain_stats(const float* rec, int64_t T, int d, int64_t N, double* mean,
                                  double* ssq, hipStream_t s) {
  hipLaunchKernelGGL(ess_chain_stats_kernel, dim3(grid_for((int64_t)d * N)), dim3(kAuxThreads),
                     0, s, rec, T, d, N, mean, ssq);
  return hipGetLastError();
}

hipError_t launch_ess_autocov(const float* rec, const double* mean, int64_t T, int d,
                              int64_t N, int64_t lag0, double* part, hipStream_t s) {
  const size_t lds = (size_t)(2 * kEssTS + kEssLB) * 64 * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)ess_autocov_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ess_autocov_kernel, dim3((unsigned)((N + 63) / 64), (unsigned)d),
                     dim3(kAuxThreads), lds, s, rec, mean, T, d, N, lag0, part);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* src, int64_t rows, int64_t cols, double* dst,
                            hipStream_t s) {
  hipLaunchKernelGGL(transpose_kernel, dim3(grid_for(rows * cols)), dim3(kAuxThreads), 0, s, src,
                     rows, cols, dst);
  return hipGetLastError();
}

hipError_t launch_normalise_inputs(const double* x, int64_t n, int d, const InputScaling& sc,
                                   float* t, hipStream_t s) {
  hipLaunchKernelGGL(normalise_inputs_kernel, dim3(grid_for((int64_t)d * n)), dim3(kAuxThreads),
                     0, s, x, n, d, sc, t);
  return hipGetLastError();
}

hipError_t launch_adam(double* p, double* m, double* v, const double* g, int64_t n, double lr,
                       double b1, double b2, double eps, double c1, double c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(kAuxThreads), 0, s, p, m, v, g, n, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_dw(const float* dl, const float* h, const float* th, const float* up,
                     int64_t B, int d, int H, int nh, double* grad, const int64_t* offs,
                     const int64_t* w_offs_host, hipStream_t s) {
  for (int l = 2; l <= nh; ++l) {
    hipLaunchKernelGGL(dw_gemm_kernel, dim3(H / 64, H / 64), dim3(kAuxThreads), 0, s,
                       dl + (int64_t)(l - 1) * H * B, h + (int64_t)(l - 2) * H * B, B, B, H,
                       grad + w_offs_host[l - 2]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t n = (int64_t)H * d + (int64_t)nh * H + H + 1;
  hipLaunchKernelGGL(dsmall_kernel, dim3(grid_for(n)), dim3(kAuxThreads), 0, s, dl, h, th, up, B,
                     B, d, H, nh, grad, offs);
  return hipGetLastError();
}

hipError_t launch_sum(const double* part, int n, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kAuxThreads), 0, s, part, n, scale, out);
  return hipGetLastError();
}


static hipError_t reduce2(int mode, const double* a, const double* b, int64_t n, double shift,
                          double* part, double* out, hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(reduce_partial_kernel, dim3(nb), dim3(kAuxThreads), 0, s, mode, a, b, n,
                     shift, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(64), 0, s, mode, part, nb, out);
  return hipGetLastError();
}

// scratch: >= 512 + 4 doubles of device memory
hipError_t launch_standardise(const double* y, int64_t n, float* out, double* scratch,
                              double* stats_host, hipStream_t s) {
  double* part = scratch;
  double* st = scratch + 512;
  hipError_t e = reduce2(0, y, nullptr, n, 0.0, part, st, s);
  if (e != hipSuccess) return e;
  double sum[2];
  if ((e = hipMemcpyAsync(sum, st, 16, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  const double mu = sum[0] / (double)n;
  if ((e = reduce2(1, y, nullptr, n, mu, part, st + 2, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(standardise_kernel, dim3(grid_for(n)), dim3(kAuxThreads), 0, s, y, n, st, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(stats_host, st, 32, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

hipError_t launch_importance_weights(const double* lp, const double* le, int64_t n, double* w,
                                     double* scratch, double* stats_host, hipStream_t s) {
  double* part = scratch;
  double* st = scratch + 512;
  hipError_t e = reduce2(2, lp, le, n, 0.0, part, st, s);
  if (e != hipSuccess) return e;
  double mx[2];
  if ((e = hipMemcpyAsync(mx, st, 16, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if ((e = reduce2(3, lp, le, n, mx[0], part, st + 2, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(weights_kernel, dim3(grid_for(n)), dim3(kAuxThreads), 0, s, lp, le, n, st, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(stats_host, st, 32, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace best
