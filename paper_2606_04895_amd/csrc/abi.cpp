// Host implementation of the C ABI declared in include/best.h: validation, device state,
// launch configuration and the sampler / adaptation / ESS / training drivers.
#include "../../include/best.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "aux.hpp"
#include "layout.hpp"

using namespace best;

namespace best {
#define BEST_DECL_PREC(suf)                                                                  \
  hipError_t launch_step_##suf(int, const KArgs&, int, size_t, hipStream_t);                 \
  hipError_t launch_eval_##suf(int, const KArgs&, int, size_t, hipStream_t);                 \
  hipError_t launch_train_tile_##suf(int, const TrainArgs&, int, size_t, hipStream_t);       \
  hipError_t launch_vjp_##suf(int, const VjpArgs&, int, size_t, hipStream_t);                \
  hipError_t launch_pack_##suf(const double*, int, int, int, void*, void*, void*, void*, void*, \
                               void*, hipStream_t);
BEST_DECL_PREC(f64)
BEST_DECL_PREC(f32)
BEST_DECL_PREC(f16)
BEST_DECL_PREC(bf16)

hipError_t launch_step(int prec, int MT, const KArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (prec) {
    case BEST_FP64: return launch_step_f64(MT, a, grid, lds, s);
    case BEST_FP32: return launch_step_f32(MT, a, grid, lds, s);
    case BEST_FP16: return launch_step_f16(MT, a, grid, lds, s);
    default: return launch_step_bf16(MT, a, grid, lds, s);
  }
}
hipError_t launch_eval(int prec, int MT, const KArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (prec) {
    case BEST_FP64: return launch_eval_f64(MT, a, grid, lds, s);
    case BEST_FP32: return launch_eval_f32(MT, a, grid, lds, s);
    case BEST_FP16: return launch_eval_f16(MT, a, grid, lds, s);
    default: return launch_eval_bf16(MT, a, grid, lds, s);
  }
}
hipError_t launch_train_tile(int prec, int MT, const TrainArgs& a, int grid, size_t lds,
                             hipStream_t s) {
  switch (prec) {
    case BEST_FP32: return launch_train_tile_f32(MT, a, grid, lds, s);
    case BEST_FP16: return launch_train_tile_f16(MT, a, grid, lds, s);
    case BEST_BF16: return launch_train_tile_bf16(MT, a, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_vjp(int prec, int MT, const VjpArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (prec) {
    case BEST_FP32: return launch_vjp_f32(MT, a, grid, lds, s);
    case BEST_FP16: return launch_vjp_f16(MT, a, grid, lds, s);
    case BEST_BF16: return launch_vjp_bf16(MT, a, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_pack(int prec, const double* flat, int d, int H, int nh, void* wf, void* wb,
                       void* w1f, void* w1t, void* bias, void* wout, hipStream_t s) {
  switch (prec) {
    case BEST_FP64: return launch_pack_f64(flat, d, H, nh, wf, wb, w1f, w1t, bias, wout, s);
    case BEST_FP32: return launch_pack_f32(flat, d, H, nh, wf, wb, w1f, w1t, bias, wout, s);
    case BEST_FP16: return launch_pack_f16(flat, d, H, nh, wf, wb, w1f, w1t, bias, wout, s);
    default: return launch_pack_bf16(flat, d, H, nh, wf, wb, w1f, w1t, bias, wout, s);
  }
}
}  // namespace best

namespace {

constexpr int kLdsMax = 163840;  // 160 KiB of LDS per CU on gfx950

struct Arena {
  std::vector<void*> ptrs;
  template <class T>
  hipError_t alloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess) return e;
    ptrs.push_back(q);
    *p = (T*)q;
    return hipSuccess;
  }
  template <class T>
  hipError_t upload(T** p, const T* host, size_t n, hipStream_t s) {
    hipError_t e = alloc(p, n);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(*p, host, n * sizeof(T), hipMemcpyHostToDevice, s);
  }
  void release(void* p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      (void)hipFree(*it);
      ptrs.erase(it);
    }
  }
  void free_all() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

MlpParams make_mlp_params(int prec, int d, int H, int nh, int lds_h, void* wf, void* wb,
                          void* w1f, void* w1t, void* bias, void* wout) {
  MlpParams mp{};
  mp.d = d;
  mp.H = H;
  mp.nh = nh;
  mp.lds_h = lds_h;
  mp.ks1 = in_ksteps(prec, d);
  mp.rti = grad_rtiles(d);
  mp.wf = wf;
  mp.wb = wb;
  mp.w1f = w1f;
  mp.w1t = w1t;
  mp.bias = bias;
  mp.wout = wout;
  return mp;
}

int64_t mlp_nparams_impl(int64_t d, int64_t w, int64_t nh) {
  return w * d + w + (nh - 1) * (w * w + w) + w + 1;
}

}  // namespace

struct best_ctx {
  std::string err;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  int dev = -1;
  double* scratch = nullptr;        // this device's fixed scratch (entry points that allocate nothing)
  hipError_t scratch_err = hipSuccess;
  int d = 0, H = 0, nh = 0, prec = 0, MT = 1, lds_h = 0, st_lds = 0, w1_lds = 0;
  int64_t N = 0, Np = 0;
  uint64_t seed = 0, step = 0;
  Arena mem;
  Target tg{};
  MlpParams mp{};
  State st{};
  double *mu = nullptr, *L = nullptr, *da = nullptr, *flat = nullptr;
  void *wf = nullptr, *wb = nullptr, *w1f = nullptr, *w1t = nullptr, *bias = nullptr,
       *wout = nullptr;
  void* hsave = nullptr;
  int64_t hsave_stride = 0;
  int grid_cap = 0;
  LdsLayout lds{};
  bool z_stale = false, gx_stale = false;
  int64_t* st_i = nullptr;
  double* st_d = nullptr;
  double *ad_part = nullptr, *ad_info = nullptr;
  int ad_blocks = 256;
  double *ev_x = nullptr, *ev_lp = nullptr, *ev_g = nullptr;
  int64_t ev_cap = 0;
  double *es_mean = nullptr, *es_ssq = nullptr, *es_part = nullptr;
  int64_t es_cap = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double* nu_buf = nullptr;  // NUTS trajectory buffers (allocated by the first NUTS call)
  double* mult = nullptr;    // per-dimension step multipliers [d] (MALA, MH)
  bool mt_fixed = false;     // tile width set by the caller (chains_per_block)
  char* ev_hsave = nullptr;  // activation scratch of wider evaluation tiles
  size_t ev_hsave_bytes = 0;
  bool mult_on = false;
  // weight-gradient (vector-Jacobian product) buffers, allocated by the first call
  float *vj_h = nullptr, *vj_dl = nullptr, *vj_th = nullptr, *vj_up = nullptr;
  int64_t vj_cap = 0;
  int64_t* vj_offs = nullptr;
  std::vector<int64_t> vj_woffs;
  NutsState nu{};
  std::vector<double> lower, upper;
  double mlp_coef = 0, offset = 0;
};

static int fail(best_ctx* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}
static int fail_hip(best_ctx* h, const char* what, hipError_t e) {
  return fail(h, BEST_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(h, x)                                           \
  do {                                                         \
    hipError_t e_ = (x);                                       \
    if (e_ != hipSuccess) return fail_hip((h), #x, e_);        \
  } while (0)

static KArgs base_args(const best_ctx* h) {
  KArgs a{};
  a.tg = h->tg;
  a.tg.mlp_coef = h->mlp_coef;
  a.tg.offset = h->offset;
  a.mp = h->mp;
  a.wh.mu = h->mu;
  a.wh.L = h->L;
  a.st = h->st;
  a.rng.k0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
  a.rng.k1 = (uint32_t)(h->seed >> 32);
  a.lds = h->lds;
  a.hsave = h->hsave;
  a.hsave_stride = h->hsave_stride;
  a.thin = 1;
  return a;
}

static int run_eval(best_ctx* h, const double* X, int64_t pitch, int64_t n, double* LP,
                    double* G) {
  if (n <= 0) return BEST_OK;
  KArgs a = base_args(h);
  a.st.N = n;
  a.ex_x = X;
  a.ex_pitch = pitch;
  a.ex_lp = LP;
  a.ex_g = G;
  a.ex_grad = G != nullptr;
  int mt = h->MT, grid_cap = h->grid_cap;
  size_t lds = h->lds.total;
  if (!h->mt_fixed) {
    // a batch larger than the chain ensemble gets the widest tile that still gives every CU
    // a tile of the batch (the rule the context applied to its chains); never narrower
    int best = 0;
    for (int m = 1; m <= mt_max(h->prec); m *= 2) {
      if (layout_for(h->prec, m, h->H, h->d, h->nh, 0).total > kLdsMax) break;
      if (best && (n + 16 * m - 1) / (16 * m) < h->n_cu) break;
      best = m;
    }
    if (best > h->MT) {
      mt = best;
      const int lh = layout_for(h->prec, mt, h->H, h->d, h->nh, 1).total <= kLdsMax ? 1 : 0;
      const LdsLayout lay = layout_for(h->prec, mt, h->H, h->d, h->nh, lh);
      grid_cap = h->n_cu * std::max(1, std::min(2, kLdsMax / lay.total));
      a.mp.lds_h = lh;
      a.lds = lay;
      lds = lay.total;
      a.hsave_stride = (int64_t)h->nh * h->H * 16 * mt;
      if (!lh) {
        const size_t need = (size_t)grid_cap * a.hsave_stride * vasize(h->prec);
        if (need > h->ev_hsave_bytes) {
          h->mem.release(h->ev_hsave);
          h->ev_hsave = nullptr;
          h->ev_hsave_bytes = 0;
          if (h->mem.alloc(&h->ev_hsave, need) != hipSuccess)
            return fail(h, BEST_ENOMEM, "evaluation activation scratch");
          h->ev_hsave_bytes = need;
        }
        a.hsave = h->ev_hsave;
      }
    }
  }
  const int64_t M = 16 * mt;
  a.n_tiles = (n + M - 1) / M;
  const int grid = (int)std::min<int64_t>(a.n_tiles, grid_cap);
  HIPCHK(h, launch_eval(h->prec, mt, a, grid, lds, h->stream));
  return BEST_OK;
}

static int refresh_state(best_ctx* h) {
  int rc = run_eval(h, h->st.x, h->Np, h->N, h->st.lp, h->st.gx);
  if (rc) return rc;
  h->gx_stale = false;
  return BEST_OK;
}

static int rewhiten(best_ctx* h) {
  Whiten w{h->mu, h->L};
  HIPCHK(h, launch_rewhiten(h->st, w, h->d, h->stream));
  h->z_stale = false;
  return BEST_OK;
}

static bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

extern "C" {

const char* best_strerror(int code) {
  switch (code) {
    case BEST_OK: return "ok";
    case BEST_EINVAL: return "invalid argument";
    case BEST_ENOMEM: return "out of memory";
    case BEST_EHIP: return "HIP runtime error";
    case BEST_ENOTPD: return "covariance not positive definite";
    case BEST_ESTATE: return "invalid state for this call";
    default: return "unknown error";
  }
}

const char* best_last_error(const best_ctx* h) { return h ? h->err.c_str() : "null context"; }

int64_t best_mlp_nparams(int32_t d, int32_t width, int32_t n_hidden) {
  if (d < 1 || width < 1 || n_hidden < 1) return -1;
  return mlp_nparams_impl(d, width, n_hidden);
}

void best_destroy(best_ctx* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  h->mem.free_all();
  delete h;
}

static int validate_problem(best_ctx* h, const best_problem* p, const best_config* c) {
  if (!p || !c) return fail(h, BEST_EINVAL, "problem or config is NULL");
  const int d = p->d;
  if (d < 1 || d > kMaxD) return fail(h, BEST_EINVAL, "d must be in [1, 32]");
  if (!p->lower || !p->upper) return fail(h, BEST_EINVAL, "lower/upper is NULL");
  for (int i = 0; i < d; ++i)
    if (!(p->lower[i] < p->upper[i]) || !std::isfinite(p->lower[i]) || !std::isfinite(p->upper[i]))
      return fail(h, BEST_EINVAL, "need finite lower[i] < upper[i]");
  if (p->width < 128 || p->width > 2048 || p->width % 128)
    return fail(h, BEST_EINVAL, "width must be a multiple of 128 in [128, 2048]");
  if (p->n_hidden < 1 || p->n_hidden > 16) return fail(h, BEST_EINVAL, "n_hidden must be in [1, 16]");
  if (p->gauss_coef != 0.0 && (!p->gauss_mean || !p->gauss_prec))
    return fail(h, BEST_EINVAL, "gauss_mean/gauss_prec is NULL");
  if (p->twist_u >= 0 &&
      (p->twist_u >= d || p->twist_v < 0 || p->twist_v >= d || p->twist_u == p->twist_v))
    return fail(h, BEST_EINVAL, "twist indices out of range");
  if (p->plain_mode < 0 || p->plain_mode > 2) return fail(h, BEST_EINVAL, "plain_mode must be 0, 1 or 2");
  if (p->box_penalty < 0 || p->box_penalty > 1) return fail(h, BEST_EINVAL, "box_penalty must be 0 or 1");
  if (p->box_penalty && !(p->penalty_width > 0 && std::isfinite(p->penalty_width)))
    return fail(h, BEST_EINVAL, "penalty_width must be finite and > 0");
  if (p->plain_mode != 2 && (!p->mlp_params || !p->in_center || !p->in_invscale))
    return fail(h, BEST_EINVAL, "MLP parameters or input normalisation is NULL");
  if (p->plain_mode != 0) {
    const best_plain_model* pm = p->plain;
    if (!pm || pm->n_bins < 1 || pm->n_terms < 1 || pm->n_terms > kMaxTerms || !pm->xgrid ||
        !pm->data || !pm->inv_sigma2 || !pm->a || !pm->g || !pm->p || !pm->k || !pm->gamma0 ||
        !pm->center || !pm->invscale)
      return fail(h, BEST_EINVAL, "plain model missing or n_terms not in [1, 8]");
  }
  if (p->plain_mode == 1) {
    if (!p->train_lo || !p->train_hi) return fail(h, BEST_EINVAL, "train box is NULL");
    for (int i = 0; i < d; ++i)
      if (!(p->train_lo[i] < p->train_hi[i])) return fail(h, BEST_EINVAL, "need train_lo < train_hi");
  }
  if (c->n_chains < 1 || c->n_chains > ((int64_t)1 << 31))
    return fail(h, BEST_EINVAL, "n_chains must be in [1, 2^31]");
  if (c->precision < BEST_FP64 || c->precision > BEST_BF16)
    return fail(h, BEST_EINVAL, "unknown precision");
  if (c->init < BEST_INIT_UNIFORM || c->init > BEST_INIT_HYPERSPHERE)
    return fail(h, BEST_EINVAL, "unknown init strategy");
  if (c->chains_per_block && c->chains_per_block != 16 && c->chains_per_block != 32 &&
      c->chains_per_block != 64)
    return fail(h, BEST_EINVAL, "chains_per_block must be 0, 16, 32 or 64");
  if (c->chains_per_block / 16 > mt_max(c->precision))
    return fail(h, BEST_EINVAL, "chains_per_block too large for this precision");
  return BEST_OK;
}

// Chain-tile width and LDS use.  Every tile streams all packed weights through its CU once
// per evaluation, and a CU's weight stream (L2 hits, 40-55 B per clock measured on MI355X)
// is the dominant cost at small tiles; wider tiles amortise it over more chains but leave
// CUs idle once there are fewer tiles than CUs.  So the widest tile that still gives every
// CU a tile is taken (the narrowest if there are too few chains); then the activations,
// and then the sampler's per-step FP64 scratch, stay in LDS when there is room.
static int choose_mt(best_ctx* h, const best_config* c) {
  auto fits = [&](int mt, int lh) {
    return layout_for(h->prec, mt, h->H, h->d, h->nh, lh).total <= kLdsMax;
  };
  int mt = 0;
  if (c->chains_per_block) {
    mt = c->chains_per_block / 16;
    if (!fits(mt, 0)) return fail(h, BEST_EINVAL, "chains_per_block needs more LDS than 160 KiB");
  } else {
    for (int m = 1; m <= mt_max(h->prec); m *= 2) {
      if (!fits(m, 0)) break;
      if (mt && (h->N + 16 * m - 1) / (16 * m) < h->n_cu) break;
      mt = m;
    }
    if (!mt) return fail(h, BEST_EINVAL, "MLP width too large for the LDS budget");
  }
  h->MT = mt;
  h->mt_fixed = c->chains_per_block != 0;
  h->lds_h = fits(mt, 1) ? 1 : 0;
  // the sampler's per-step FP64 scratch and the launch constants go to LDS too when there is
  // room (1), else the constants alone when they fit (2), and then the input layer's
  // weights (W_1, W_1^T), which every evaluation reads
  h->st_lds = layout_for(h->prec, mt, h->H, h->d, h->nh, h->lds_h, 1).total <= kLdsMax   ? 1
              : layout_for(h->prec, mt, h->H, h->d, h->nh, h->lds_h, 2).total <= kLdsMax ? 2
                                                                                         : 0;
  // (never at the cost of a second workgroup per CU)
  const int base = layout_for(h->prec, mt, h->H, h->d, h->nh, h->lds_h, h->st_lds).total;
  const int with = layout_for(h->prec, mt, h->H, h->d, h->nh, h->lds_h, h->st_lds, 1).total;
  h->w1_lds = with <= kLdsMax && (2 * base > kLdsMax || 2 * with <= kLdsMax) ? 1 : 0;
  return BEST_OK;
}

static int upload_problem(best_ctx* h, const best_problem* p) {
  const int d = p->d;
  Arena& m = h->mem;
  hipStream_t s = h->stream;
  Target& t = h->tg;
  t.d = d;
  HIPCHK(h, m.upload((double**)&t.lower, p->lower, d, s));
  HIPCHK(h, m.upload((double**)&t.upper, p->upper, d, s));
  t.gauss_coef = p->gauss_coef;
  std::vector<double> zeros((size_t)d * d, 0.0);
  HIPCHK(h, m.upload((double**)&t.gmean, p->gauss_mean ? p->gauss_mean : zeros.data(), d, s));
  HIPCHK(h, m.upload((double**)&t.gprec, p->gauss_prec ? p->gauss_prec : zeros.data(),
                     (size_t)d * d, s));
  t.tw_u = p->twist_u >= 0 ? p->twist_u : -1;
  t.tw_v = p->twist_u >= 0 ? p->twist_v : -1;
  t.tw_beta = p->twist_beta;
  t.tw_center = p->twist_center;
  t.tw_kappa = p->twist_kappa;
  std::vector<double> ones(d, 1.0);
  HIPCHK(h, m.upload((double**)&t.in_center, p->in_center ? p->in_center : zeros.data(), d, s));
  HIPCHK(h, m.upload((double**)&t.in_invscale, p->in_invscale ? p->in_invscale : ones.data(), d, s));
  h->mlp_coef = p->mlp_coef;
  h->offset = p->offset;
  t.plain_mode = p->plain_mode;
  t.box_penalty = p->box_penalty;
  t.pen_w = p->box_penalty ? p->penalty_width : 1.0;
  HIPCHK(h, m.upload((double**)&t.train_lo, p->train_lo ? p->train_lo : p->lower, d, s));
  HIPCHK(h, m.upload((double**)&t.train_hi, p->train_hi ? p->train_hi : p->upper, d, s));
  if (p->plain_mode != 0) {
    const best_plain_model* pm = p->plain;
    t.n_bins = pm->n_bins;
    t.n_terms = pm->n_terms;
    const size_t nb = pm->n_bins, nt = pm->n_terms;
    HIPCHK(h, m.upload((double**)&t.xgrid, pm->xgrid, nb, s));
    HIPCHK(h, m.upload((double**)&t.data, pm->data, nb, s));
    HIPCHK(h, m.upload((double**)&t.w2, pm->inv_sigma2, nb, s));
    HIPCHK(h, m.upload((double**)&t.pa, pm->a, nt * d, s));
    HIPCHK(h, m.upload((double**)&t.pg, pm->g, nt * d, s));
    HIPCHK(h, m.upload((double**)&t.pp, pm->p, nt * d, s));
    HIPCHK(h, m.upload((double**)&t.pk, pm->k, nt, s));
    HIPCHK(h, m.upload((double**)&t.pg0, pm->gamma0, nt, s));
    HIPCHK(h, m.upload((double**)&t.pc, pm->center, d, s));
    HIPCHK(h, m.upload((double**)&t.pis, pm->invscale, d, s));
  }
  h->lower.assign(p->lower, p->lower + d);
  h->upper.assign(p->upper, p->upper + d);
  return BEST_OK;
}

static int alloc_mlp(best_ctx* h) {
  const int H = h->H, d = h->d, nh = h->nh, ts = tsize(h->prec), va = vasize(h->prec);
  Arena& m = h->mem;
  const size_t nW = (size_t)std::max(nh - 1, 1) * H * H;
  HIPCHK(h, m.alloc((char**)&h->wf, nW * ts));
  HIPCHK(h, m.alloc((char**)&h->wb, nW * ts));
  HIPCHK(h, m.alloc((char**)&h->w1f, w1f_bytes(h->prec, H, d)));
  HIPCHK(h, m.alloc((char**)&h->w1t, w1t_bytes(h->prec, H, d)));
  HIPCHK(h, m.alloc((char**)&h->bias, (size_t)nh * H * va));
  HIPCHK(h, m.alloc((char**)&h->wout, (size_t)(H + 1) * va));
  HIPCHK(h, m.alloc(&h->flat, (size_t)mlp_nparams_impl(d, H, nh)));
  h->mp = make_mlp_params(h->prec, d, H, nh, h->lds_h, h->wf, h->wb, h->w1f, h->w1t, h->bias,
                          h->wout);
  return BEST_OK;
}

static int load_mlp(best_ctx* h, const double* params) {
  const int64_t np = mlp_nparams_impl(h->d, h->H, h->nh);
  if (!finite_all(params, np)) return fail(h, BEST_EINVAL, "MLP parameters must be finite");
  HIPCHK(h, hipMemcpyAsync(h->flat, params, np * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, launch_pack(h->prec, h->flat, h->d, h->H, h->nh, h->wf, h->wb, h->w1f, h->w1t,
                        h->bias, h->wout, h->stream));
  return BEST_OK;
}

int best_init(best_ctx** out, const best_problem* p, const best_config* c) {
  if (!out) return BEST_EINVAL;
  *out = nullptr;
  best_ctx* h = new (std::nothrow) best_ctx();
  if (!h) return BEST_ENOMEM;
  int rc = validate_problem(h, p, c);
  if (rc) {
    std::fprintf(stderr, "best_init: %s\n", h->err.c_str());
    delete h;
    return rc;
  }
  auto bail = [&](int code) {
    std::fprintf(stderr, "best_init: %s\n", h->err.c_str());
    best_destroy(h);
    return code;
  };
  h->stream = (hipStream_t)c->stream;
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (he != hipSuccess) {
    h->err = std::string("no usable HIP device: ") + hipGetErrorString(he);
    return bail(BEST_EHIP);
  }
  h->dev = dev;
  // the device's fixed scratch, resolved once per device with that device current
  h->scratch_err = noalloc_scratch_address(dev, &h->scratch);
  h->d = p->d;
  h->H = p->width;
  h->nh = p->n_hidden;
  h->prec = c->precision;
  h->N = c->n_chains;
  h->Np = (h->N + 63) / 64 * 64;
  h->seed = c->seed;
  if ((rc = choose_mt(h, c))) return bail(rc);
  h->lds = layout_for(h->prec, h->MT, h->H, h->d, h->nh, h->lds_h, h->st_lds, h->w1_lds);
  if ((rc = upload_problem(h, p))) return bail(rc);
  if ((rc = alloc_mlp(h))) return bail(rc);
  if (p->plain_mode != 2) {
    if ((rc = load_mlp(h, p->mlp_params))) return bail(rc);
  }
  // chain state
  const int d = h->d;
  const size_t nd = (size_t)d * h->Np, n1 = (size_t)h->Np;
  State& S = h->st;
  S.Np = h->Np;
  S.N = h->N;
  double** vecs[] = {&S.x, &S.z, &S.gx, &S.xp, &S.zp, &S.gxp, &S.q, &S.gz, &S.gzp};
  for (double** v : vecs)
    if (h->mem.alloc(v, nd) != hipSuccess) return bail(fail(h, BEST_ENOMEM, "state allocation"));
  double** scal[] = {&S.lp, &S.lpp, &S.sum_prob, &S.step_prob};
  for (double** v : scal)
    if (h->mem.alloc(v, n1) != hipSuccess) return bail(fail(h, BEST_ENOMEM, "state allocation"));
  uint32_t** cnt[] = {&S.n_acc, &S.n_nonfinite, &S.n_oob, &S.n_evals};
  for (uint32_t** v : cnt)
    if (h->mem.alloc(v, n1) != hipSuccess) return bail(fail(h, BEST_ENOMEM, "state allocation"));
  for (double** v : vecs)
    if (hipMemsetAsync(*v, 0, nd * sizeof(double), h->stream) != hipSuccess)
      return bail(fail(h, BEST_EHIP, "memset"));
  // per-workgroup activation scratch
  const int occ = std::max(1, std::min(2, kLdsMax / h->lds.total));
  h->grid_cap = h->n_cu * occ;
  h->hsave_stride = (int64_t)h->nh * h->H * 16 * h->MT;
  if (h->mem.alloc((char**)&h->hsave, (size_t)h->grid_cap * h->hsave_stride * vasize(h->prec)) !=
      hipSuccess)
    return bail(fail(h, BEST_ENOMEM, "activation scratch"));
  // whitening: mu = box centre, L = diag(0.1 (u - l))
  std::vector<double> mu(d), L((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) {
    mu[i] = 0.5 * (p->lower[i] + p->upper[i]);
    L[(size_t)i * d + i] = 0.1 * (p->upper[i] - p->lower[i]);
  }
  if (h->mem.upload(&h->mu, mu.data(), d, h->stream) != hipSuccess ||
      h->mem.upload(&h->L, L.data(), (size_t)d * d, h->stream) != hipSuccess)
    return bail(fail(h, BEST_ENOMEM, "whitening"));
  const double eps0 = 0.1;
  const double da[9] = {std::log(10.0 * eps0), 0, 0, 0, eps0, 0.57, 0.05, 10.0, 0.75};
  if (h->mem.upload(&h->da, da, 9, h->stream) != hipSuccess ||
      h->mem.alloc(&h->st_i, 4) != hipSuccess || h->mem.alloc(&h->st_d, 4) != hipSuccess ||
      h->mem.alloc(&h->ad_info, 4) != hipSuccess ||
      h->mem.alloc(&h->ad_part, (size_t)h->ad_blocks * (kMaxD + kMaxD * (kMaxD + 1) / 2)) !=
          hipSuccess)
    return bail(fail(h, BEST_ENOMEM, "small buffers"));
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return bail(fail(h, BEST_EHIP, "hipEventCreate"));
  // walkers
  std::vector<double> pt(d);
  for (int i = 0; i < d; ++i) pt[i] = c->init_point ? c->init_point[i] : mu[i];
  double* pt_dev = nullptr;
  if (h->mem.upload(&pt_dev, pt.data(), d, h->stream) != hipSuccess)
    return bail(fail(h, BEST_ENOMEM, "init point"));
  Rng rng{(uint32_t)(h->seed & 0xFFFFFFFFu), (uint32_t)(h->seed >> 32)};
  if (hipError_t e = launch_init_positions(h->tg, h->st, rng, c->init, pt_dev, c->init_scale,
                                           h->L, 0, h->stream))
    return bail(fail_hip(h, "init positions", e));
  if ((rc = refresh_state(h))) return bail(rc);
  if ((rc = rewhiten(h))) return bail(rc);
  if (hipError_t e = hipStreamSynchronize(h->stream)) return bail(fail_hip(h, "init sync", e));
  h->mem.release(pt_dev);
  *out = h;
  return BEST_OK;
}

// ---------------------------------------------------------------------------------------

static int ensure_eval_scratch(best_ctx* h, int64_t n) {
  if (n <= h->ev_cap) return BEST_OK;
  h->mem.release(h->ev_x);
  h->mem.release(h->ev_lp);
  h->mem.release(h->ev_g);
  h->ev_cap = 0;
  if (h->mem.alloc(&h->ev_x, (size_t)n * h->d) != hipSuccess ||
      h->mem.alloc(&h->ev_lp, (size_t)n) != hipSuccess ||
      h->mem.alloc(&h->ev_g, (size_t)n * h->d) != hipSuccess)
    return fail(h, BEST_ENOMEM, "evaluation scratch");
  h->ev_cap = n;
  return BEST_OK;
}

int best_logL_grad(best_ctx* h, const double* x, int64_t n, double* logL, double* grad,
                   uint32_t flags) {
  if (!h) return BEST_EINVAL;
  if (n < 0 || (n > 0 && (!x || !logL))) return fail(h, BEST_EINVAL, "x/logL NULL or n < 0");
  if (n == 0) return BEST_OK;
  if (flags & ~(BEST_HOST_PTRS | BEST_AOS)) return fail(h, BEST_EINVAL, "unknown flags");
  const bool aos = (flags & BEST_AOS) != 0;
  const int64_t d = h->d;
  const size_t nd = (size_t)n * d;
  if (!(flags & BEST_HOST_PTRS)) {
    if (!aos) return run_eval(h, x, n, n, logL, grad);
    // point-major [n][d] device arrays: through the structure-of-arrays scratch
    int rc = ensure_eval_scratch(h, n);
    if (rc) return rc;
    HIPCHK(h, launch_transpose(x, n, d, h->ev_x, h->stream));
    if ((rc = run_eval(h, h->ev_x, n, n, logL, grad ? h->ev_g : nullptr))) return rc;
    if (grad) HIPCHK(h, launch_transpose(h->ev_g, d, n, grad, h->stream));
    return BEST_OK;
  }
  int rc = ensure_eval_scratch(h, n);
  if (rc) return rc;
  std::vector<double> tmp;
  const double* xs = x;
  if (aos) {  // host point-major input: reorder on the host
    tmp.resize(nd);
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < d; ++i) tmp[i * n + c] = x[c * d + i];
    xs = tmp.data();
  }
  HIPCHK(h, hipMemcpyAsync(h->ev_x, xs, nd * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if ((rc = run_eval(h, h->ev_x, n, n, h->ev_lp, grad ? h->ev_g : nullptr))) return rc;
  HIPCHK(h, hipMemcpyAsync(logL, h->ev_lp, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (grad) {
    if (aos) tmp.resize(nd);
    HIPCHK(h, hipMemcpyAsync(aos ? tmp.data() : grad, h->ev_g, nd * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (grad && aos)
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < d; ++i) grad[c * d + i] = tmp[i * n + c];
  return BEST_OK;
}

// Offsets into the flat parameter vector: [W1, b1, b2 .. b_nh, w_out, b_out] (nh + 3) and
// the W_l blocks (l >= 2).
static void param_offsets(int64_t d, int64_t H, int nh, std::vector<int64_t>& offs,
                          std::vector<int64_t>& w_offs) {
  const int64_t base = H * d + H, blk = H * H + H;
  offs.assign(1, 0);
  offs.push_back(H * d);
  for (int l = 2; l <= nh; ++l) offs.push_back(base + (l - 2) * blk + H * H);
  offs.push_back(base + (nh - 1) * blk);
  offs.push_back(base + (nh - 1) * blk + H);
  w_offs.clear();
  for (int l = 2; l <= nh; ++l) w_offs.push_back(base + (l - 2) * blk);
}

int best_logL_param_grad(best_ctx* h, const double* x, int64_t n, const double* upstream,
                         double* grad_params) {
  if (!h) return BEST_EINVAL;
  if (n < 0 || !grad_params || (n > 0 && !x)) return fail(h, BEST_EINVAL, "x/grad_params NULL or n < 0");
  const int64_t np = mlp_nparams_impl(h->d, h->H, h->nh);
  if (h->tg.plain_mode == 2 || n == 0) {
    HIPCHK(h, hipMemsetAsync(grad_params, 0, (size_t)np * 8, h->stream));
    return BEST_OK;
  }
  if (h->prec == BEST_FP64)
    return fail(h, BEST_ESTATE, "the parameter gradient needs FP32, FP16 or BF16 precision");
  const int64_t ldb = (n + 15) / 16 * 16;
  if (ldb > h->vj_cap) {
    for (void* q : {(void*)h->vj_h, (void*)h->vj_dl, (void*)h->vj_th, (void*)h->vj_up})
      h->mem.release(q);
    h->vj_h = h->vj_dl = h->vj_th = h->vj_up = nullptr;
    h->vj_cap = 0;
    const size_t rows = (size_t)h->nh * h->H;
    if (h->mem.alloc(&h->vj_h, rows * ldb) != hipSuccess ||
        h->mem.alloc(&h->vj_dl, rows * ldb) != hipSuccess ||
        h->mem.alloc(&h->vj_th, (size_t)h->d * ldb) != hipSuccess ||
        h->mem.alloc(&h->vj_up, (size_t)ldb) != hipSuccess)
      return fail(h, BEST_ENOMEM, "parameter-gradient buffers");
    h->vj_cap = ldb;
  }
  if (!h->vj_offs) {
    std::vector<int64_t> offs;
    param_offsets(h->d, h->H, h->nh, offs, h->vj_woffs);
    HIPCHK(h, h->mem.upload(&h->vj_offs, offs.data(), offs.size(), h->stream));
  }
  VjpArgs a{};
  a.tg = h->tg;
  a.tg.mlp_coef = h->mlp_coef;
  a.mp = h->mp;
  a.lds = h->lds;
  a.x = x;
  a.pitch = n;
  a.n = n;
  a.ldb = ldb;
  const int64_t M = 16 * h->MT;
  a.n_tiles = (n + M - 1) / M;
  a.upstream = upstream;
  a.hsave = h->hsave;
  a.hsave_stride = h->hsave_stride;
  a.ex_h = h->vj_h;
  a.ex_dl = h->vj_dl;
  a.ex_th = h->vj_th;
  a.ex_up = h->vj_up;
  const int grid = (int)std::min<int64_t>(a.n_tiles, h->grid_cap);
  HIPCHK(h, launch_vjp(h->prec, h->MT, a, grid, h->lds.total, h->stream));
  HIPCHK(h, launch_dw(h->vj_dl, h->vj_h, h->vj_th, h->vj_up, ldb, h->d, h->H, h->nh,
                      grad_params, h->vj_offs, h->vj_woffs.data(), h->stream));
  return BEST_OK;
}

// NUTS buffers for trees of up to `depth` levels, carved from one allocation.
static int ensure_nuts(best_ctx* h, int depth) {
  if (h->nu_buf && h->nu.max_depth >= depth) return BEST_OK;
  h->mem.release(h->nu_buf);
  h->nu_buf = nullptr;
  h->nu = NutsState{};
  const size_t nd = (size_t)h->Np * h->d, n1 = (size_t)h->Np;
  const size_t total = nd * (8 + 4 * (size_t)depth) + n1 * (2 * (size_t)depth + 1);
  if (h->mem.alloc(&h->nu_buf, total) != hipSuccess)
    return fail(h, BEST_ENOMEM, "NUTS trajectory buffers");
  double* b = h->nu_buf;
  auto take = [&](size_t n) {
    double* r = b;
    b += n;
    return r;
  };
  NutsState& U = h->nu;
  U.zm = take(nd);
  U.qm = take(nd);
  U.gm = take(nd);
  U.zpl = take(nd);
  U.qpl = take(nd);
  U.gpl = take(nd);
  U.xc = take(nd);
  U.gxc = take(nd);
  U.lpc = take(n1);
  U.pz = take(nd * depth);
  U.pq = take(nd * depth);
  U.px = take(nd * depth);
  U.pgx = take(nd * depth);
  U.plp = take(n1 * depth);
  U.pn = take(n1 * depth);
  U.max_depth = depth;
  return BEST_OK;
}

int best_step(best_ctx* h, int32_t sampler, int64_t n_steps, const best_step_params* p,
              best_step_stats* out) {
  if (!h) return BEST_EINVAL;
  int rc;
  if (!p) return fail(h, BEST_EINVAL, "params is NULL");
  if (sampler < BEST_MH || sampler > BEST_DE) return fail(h, BEST_EINVAL, "unknown sampler");
  if (sampler == BEST_DE && !(p->de_sigma >= 0 && std::isfinite(p->de_sigma)))
    return fail(h, BEST_EINVAL, "de_sigma must be finite and >= 0");
  if (sampler == BEST_DE && (h->N < 4 || (h->N & 1)))
    return fail(h, BEST_ESTATE, "the DE move needs an even number of walkers >= 4");
  if (sampler == BEST_NUTS && (p->max_depth < 1 || p->max_depth > BEST_NUTS_MAX_DEPTH))
    return fail(h, BEST_EINVAL, "max_depth must be in 1 .. BEST_NUTS_MAX_DEPTH");
  if (n_steps < 0) return fail(h, BEST_EINVAL, "n_steps < 0");
  if (p->thin < 1) return fail(h, BEST_EINVAL, "thin must be >= 1");
  if (p->record && p->record_capacity < 0) return fail(h, BEST_EINVAL, "record_capacity < 0");
  if (sampler == BEST_HMC && p->n_leapfrog < 1) return fail(h, BEST_EINVAL, "n_leapfrog must be >= 1");
  if (sampler == BEST_MH && !(p->mh_scale > 0)) return fail(h, BEST_EINVAL, "mh_scale must be > 0");
  if (sampler == BEST_AIES && !(p->stretch_a > 1.0)) return fail(h, BEST_EINVAL, "stretch_a must be > 1");
  if (sampler == BEST_AIES && (h->N < 2 || (h->N & 1)))
    return fail(h, BEST_ESTATE, "AIES needs an even number of walkers >= 2");
  if (p->adapt_eps && sampler != BEST_MALA && sampler != BEST_HMC && sampler != BEST_NUTS)
    return fail(h, BEST_EINVAL, "step-size adaptation applies to MALA, HMC and NUTS");
  if (p->adapt_eps && !(p->target_accept > 0 && p->target_accept < 1))
    return fail(h, BEST_EINVAL, "target_accept must be in (0, 1)");
  const bool gradient = sampler == BEST_MALA || sampler == BEST_HMC || sampler == BEST_NUTS;
  if (gradient && h->prec == BEST_FP64)
    return fail(h, BEST_ESTATE,
                "MALA/HMC/NUTS with FP64 GEMMs is switched off: an earlier build of this path "
                "faulted on the GPU and the cause has not been shown yet");
  if (sampler == BEST_NUTS && (rc = ensure_nuts(h, p->max_depth))) return rc;
  const bool ensemble = sampler == BEST_AIES || sampler == BEST_DE;
  if (!ensemble && h->z_stale && (rc = rewhiten(h))) return rc;
  if (gradient && h->gx_stale && (rc = refresh_state(h))) return rc;
  const size_t n1 = (size_t)h->Np;
  HIPCHK(h, hipMemsetAsync(h->st.n_acc, 0, n1 * 4, h->stream));
  HIPCHK(h, hipMemsetAsync(h->st.n_nonfinite, 0, n1 * 4, h->stream));
  HIPCHK(h, hipMemsetAsync(h->st.n_oob, 0, n1 * 4, h->stream));
  HIPCHK(h, hipMemsetAsync(h->st.n_evals, 0, n1 * 4, h->stream));
  HIPCHK(h, hipMemsetAsync(h->st.sum_prob, 0, n1 * 8, h->stream));
  if (p->adapt_eps) {
    // keep the running dual-averaging state; only the target can change between calls
    HIPCHK(h, hipMemcpyAsync(h->da + 5, &p->target_accept, sizeof(double), hipMemcpyHostToDevice,
                             h->stream));
  }
  HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  KArgs a = base_args(h);
  a.sampler = sampler;
  a.adapt = p->adapt_eps ? 1 : 0;
  a.mh_scale = p->mh_scale;
  a.stretch_a = p->stretch_a;
  a.de_sigma = p->de_sigma;
  a.step_mult = h->mult_on ? h->mult : nullptr;
  a.n_leap = p->n_leapfrog;
  a.thin = p->thin;
  a.record = p->record;
  a.rec_cap = p->record ? p->record_capacity : 0;
  a.rec_pitch = h->N;
  a.eps = p->eps;
  a.eps_ptr = (p->adapt_eps || !(p->eps > 0)) ? h->da + 4 : nullptr;
  if (sampler == BEST_NUTS) {
    a.nu = h->nu;
    a.nu.max_depth = p->max_depth;
  }
  const int64_t M = 16 * h->MT;
  const size_t lds = h->lds.total;
  if (ensemble) {
    const int64_t half = h->N / 2;
    a.n_tiles = (half + M - 1) / M;
    const int grid = (int)std::min<int64_t>(a.n_tiles, h->grid_cap);
    for (int64_t s = 0; s < n_steps; ++s) {
      a.step0 = (int64_t)(h->step + s);
      a.n_steps = 1;
      for (int hh = 0; hh < 2; ++hh) {
        a.aies_half = hh;
        a.chain0 = hh * half;
        HIPCHK(h, launch_step(h->prec, h->MT, a, grid, lds, h->stream));
      }
      if (p->record && (s + 1) % p->thin == 0 && (s + 1) / p->thin - 1 < p->record_capacity)
        HIPCHK(h, launch_aies_record(h->st, h->d, p->record, (s + 1) / p->thin - 1, h->N,
                                     h->stream));
    }
  } else {
    a.n_tiles = (h->N + M - 1) / M;
    const int grid = (int)std::min<int64_t>(a.n_tiles, h->grid_cap);
    const int64_t chunk = p->adapt_eps ? 1 : (1 << 20);
    for (int64_t s = 0; s < n_steps; s += chunk) {
      a.step0 = (int64_t)(h->step + s);
      a.n_steps = (int)std::min<int64_t>(chunk, n_steps - s);
      a.rec_s0 = s;
      HIPCHK(h, launch_step(h->prec, h->MT, a, grid, lds, h->stream));
      if (p->adapt_eps) HIPCHK(h, launch_da_update(h->st.step_prob, h->N, h->da, h->stream));
    }
  }
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  HIPCHK(h, launch_stats(h->st, h->st_i, h->st_d, h->stream));
  int64_t si[4] = {0, 0, 0, 0};
  double sd[4] = {0, 0, 0, 0}, da[9];
  HIPCHK(h, hipMemcpyAsync(si, h->st_i, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(sd, h->st_d, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(da, h->da, 9 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->step += (uint64_t)n_steps;
  if (sampler == BEST_MH || ensemble) h->gx_stale = true;
  if (ensemble) h->z_stale = true;
  if (out) {
    const int64_t per = sampler == BEST_HMC ? p->n_leapfrog : 1;
    out->accepted = si[0];
    out->n_nonfinite = si[1];
    out->n_oob = si[2];
    out->sum_accept_prob = sd[0];
    out->evals = sampler == BEST_NUTS ? si[3] : n_steps * h->N * per;
    out->n_recorded = p->record ? std::min<int64_t>(n_steps / p->thin, p->record_capacity) : 0;
    out->ms = ms;
    out->eps = (p->adapt_eps || !(p->eps > 0)) ? da[4] : p->eps;
    out->eps_bar = std::exp(da[2]);
  }
  return BEST_OK;
}

int best_adapt(best_ctx* h, const best_adapt_params* p, best_adapt_info* out) {
  if (!h) return BEST_EINVAL;
  if (!p) return fail(h, BEST_EINVAL, "params is NULL");
  if (p->samples && p->n_samples < 1) return fail(h, BEST_EINVAL, "n_samples must be >= 1");
  const int64_t T = p->samples ? p->n_samples : 1;
  if (T * h->N < 2) return fail(h, BEST_EINVAL, "need at least two samples");
  HIPCHK(h, launch_moments(p->samples, h->st.x, T, h->N, p->samples ? h->N : h->Np, h->d,
                           h->mu, h->ad_part, h->ad_blocks, p->update_mean, h->mu, h->L,
                           h->ad_info, h->stream));
  double info[3] = {0, 0, 0};
  HIPCHK(h, hipMemcpyAsync(info, h->ad_info, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int rc = BEST_OK;
  if (info[0] != 0) rc = fail(h, BEST_ENOTPD, "covariance not positive definite after jitter");
  if (!rc && (rc = rewhiten(h))) return rc;
  double da[9];
  HIPCHK(h, hipMemcpy(da, h->da, sizeof(da), hipMemcpyDeviceToHost));
  if (p->finalize_da) da[4] = std::exp(da[2]);
  if (p->reset_da) {
    const double eps = da[4];
    da[0] = std::log(10.0 * eps);
    da[1] = da[2] = da[3] = 0;
    if (p->target_accept > 0 && p->target_accept < 1) da[5] = p->target_accept;
  }
  HIPCHK(h, hipMemcpy(h->da, da, sizeof(da), hipMemcpyHostToDevice));
  if (out) {
    out->jitter = info[1];
    out->logdet = info[2];
    out->eps = da[4];
  }
  return rc;
}

int best_get_state(best_ctx* h, double* x, double* logL, double* grad, uint32_t flags) {
  if (!h) return BEST_EINVAL;
  if (flags & ~BEST_HOST_PTRS) return fail(h, BEST_EINVAL, "unknown flags");
  int rc;
  if (grad && h->gx_stale && (rc = refresh_state(h))) return rc;
  const hipMemcpyKind k = (flags & BEST_HOST_PTRS) ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  for (int i = 0; i < h->d; ++i) {
    if (x) HIPCHK(h, hipMemcpyAsync(x + i * h->N, h->st.x + i * h->Np, h->N * 8, k, h->stream));
    if (grad) HIPCHK(h, hipMemcpyAsync(grad + i * h->N, h->st.gx + i * h->Np, h->N * 8, k, h->stream));
  }
  if (logL) HIPCHK(h, hipMemcpyAsync(logL, h->st.lp, h->N * 8, k, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return BEST_OK;
}

int best_set_state(best_ctx* h, const double* x, const double* logL, const double* grad,
                   uint32_t flags) {
  if (!h) return BEST_EINVAL;
  if (!x) return fail(h, BEST_EINVAL, "x is NULL");
  if (flags & ~BEST_HOST_PTRS) return fail(h, BEST_EINVAL, "unknown flags");
  if ((logL == nullptr) != (grad == nullptr))
    return fail(h, BEST_EINVAL, "pass both logL and grad, or neither");
  const hipMemcpyKind k = (flags & BEST_HOST_PTRS) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  for (int i = 0; i < h->d; ++i) {
    HIPCHK(h, hipMemcpyAsync(h->st.x + i * h->Np, x + i * h->N, h->N * 8, k, h->stream));
    if (grad)
      HIPCHK(h, hipMemcpyAsync(h->st.gx + i * h->Np, grad + i * h->N, h->N * 8, k, h->stream));
  }
  int rc;
  if (logL) {
    HIPCHK(h, hipMemcpyAsync(h->st.lp, logL, h->N * 8, k, h->stream));
    h->gx_stale = false;
  } else if ((rc = refresh_state(h))) {
    return rc;
  }
  if ((rc = rewhiten(h))) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return BEST_OK;
}

int best_get_whitening(best_ctx* h, double* mu, double* L) {
  if (!h) return BEST_EINVAL;
  if (mu) HIPCHK(h, hipMemcpyAsync(mu, h->mu, h->d * 8, hipMemcpyDeviceToHost, h->stream));
  if (L) HIPCHK(h, hipMemcpyAsync(L, h->L, (size_t)h->d * h->d * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return BEST_OK;
}

int best_set_whitening(best_ctx* h, const double* mu, const double* L) {
  if (!h) return BEST_EINVAL;
  if (!mu || !L) return fail(h, BEST_EINVAL, "mu/L is NULL");
  const int d = h->d;
  for (int i = 0; i < d; ++i) {
    if (!(L[i * d + i] > 0) || !std::isfinite(mu[i])) return fail(h, BEST_EINVAL, "L needs a positive diagonal");
    for (int j = i + 1; j < d; ++j)
      if (L[i * d + j] != 0.0) return fail(h, BEST_EINVAL, "L must be lower triangular");
  }
  if (!finite_all(L, (int64_t)d * d)) return fail(h, BEST_EINVAL, "L must be finite");
  HIPCHK(h, hipMemcpyAsync(h->mu, mu, d * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(h->L, L, (size_t)d * d * 8, hipMemcpyHostToDevice, h->stream));
  int rc = rewhiten(h);
  if (rc) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return BEST_OK;
}

uint64_t best_get_step_counter(const best_ctx* h) { return h ? h->step : 0; }

int best_set_step_counter(best_ctx* h, uint64_t step) {
  if (!h) return BEST_EINVAL;
  h->step = step;
  return BEST_OK;
}

int best_set_step_size(best_ctx* h, double eps) {
  if (!h) return BEST_EINVAL;
  if (!(eps > 0) || !std::isfinite(eps)) return fail(h, BEST_EINVAL, "eps must be > 0");
  double da[9];
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(da, h->da, sizeof(da), hipMemcpyDeviceToHost));
  da[4] = eps;
  da[0] = std::log(10.0 * eps);
  da[1] = da[2] = da[3] = 0;
  HIPCHK(h, hipMemcpy(h->da, da, sizeof(da), hipMemcpyHostToDevice));
  return BEST_OK;
}

int best_reinit(best_ctx* h, int32_t init, const double* point, double scale) {
  if (!h) return BEST_EINVAL;
  if (init < BEST_INIT_UNIFORM || init > BEST_INIT_HYPERSPHERE)
    return fail(h, BEST_EINVAL, "unknown init mode");
  if (init != BEST_INIT_UNIFORM && !point) return fail(h, BEST_EINVAL, "point is NULL");
  if (init >= BEST_INIT_GAUSSIAN && !(scale >= 0 && std::isfinite(scale)))
    return fail(h, BEST_EINVAL, "scale must be finite and >= 0");
  const int d = h->d;
  for (int i = 0; point && i < d; ++i)
    if (!(point[i] >= h->lower[i] && point[i] <= h->upper[i]))
      return fail(h, BEST_EINVAL, "point outside the prior box");
  double* pt_dev = nullptr;
  std::vector<double> pt(point ? point : h->lower.data(), (point ? point : h->lower.data()) + d);
  if (h->mem.upload(&pt_dev, pt.data(), d, h->stream) != hipSuccess)
    return fail(h, BEST_ENOMEM, "point");
  const Rng rng{(uint32_t)(h->seed & 0xFFFFFFFFu), (uint32_t)(h->seed >> 32)};
  hipError_t e = launch_init_positions(h->tg, h->st, rng, init, pt_dev, scale, h->L, h->step,
                                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  h->mem.release(pt_dev);
  if (e != hipSuccess) return fail_hip(h, "reinit positions", e);
  int rc;
  if ((rc = refresh_state(h))) return rc;
  if ((rc = rewhiten(h))) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return BEST_OK;
}

int best_set_step_multipliers(best_ctx* h, const double* m) {
  if (!h) return BEST_EINVAL;
  if (!m) {
    h->mult_on = false;
    return BEST_OK;
  }
  for (int i = 0; i < h->d; ++i)
    if (!(m[i] > 0) || !std::isfinite(m[i]))
      return fail(h, BEST_EINVAL, "step multipliers must be finite and > 0");
  if (!h->mult && h->mem.alloc(&h->mult, (size_t)h->d) != hipSuccess)
    return fail(h, BEST_ENOMEM, "step multipliers");
  HIPCHK(h, hipMemcpyAsync(h->mult, m, (size_t)h->d * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->mult_on = true;
  return BEST_OK;
}

int best_set_mlp(best_ctx* h, const double* params, double mlp_coef, double offset) {
  if (!h) return BEST_EINVAL;
  if (!params) return fail(h, BEST_EINVAL, "params is NULL");
  int rc = load_mlp(h, params);
  if (rc) return rc;
  h->mlp_coef = mlp_coef;
  h->offset = offset;
  if ((rc = refresh_state(h))) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return BEST_OK;
}

}  // extern "C"

// Multi-chain ESS of a record with the given device scratch: mean and ssq [d][N], part
// [d][ceil(N/64)][kEssLB] doubles.
static int ess_impl(best_ctx* h, const float* record, int64_t T, double* es_mean,
                    double* es_ssq, double* es_part, double* ess_out, int32_t* flags_out) {
  const int d = h->d;
  const int64_t N = h->N, nblk = (N + 63) / 64;
  HIPCHK(h, launch_ess_chain_stats(record, T, d, N, es_mean, es_ssq, h->stream));
  std::vector<double> mean((size_t)d * N), ssq((size_t)d * N), part((size_t)d * nblk * kEssLB);
  HIPCHK(h, hipMemcpyAsync(mean.data(), es_mean, mean.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(ssq.data(), es_ssq, ssq.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::vector<double> W(d), var_plus(d);
  for (int i = 0; i < d; ++i) {
    double w = 0, mm = 0;
    for (int64_t c = 0; c < N; ++c) {
      w += ssq[i * N + c] / (double)(T - 1);
      mm += mean[i * N + c];
    }
    w /= (double)N;
    mm /= (double)N;
    double b = 0;
    if (N > 1) {
      for (int64_t c = 0; c < N; ++c) {
        const double dm = mean[i * N + c] - mm;
        b += dm * dm;
      }
      b /= (double)(N - 1);
    }
    W[i] = w;
    var_plus[i] = (double)(T - 1) / (double)T * w + b;
  }
  std::vector<std::vector<double>> rho(d);
  std::vector<int> done(d, 0), flag(d, BEST_ESS_OK);
  std::vector<double> tau(d, 1.0);
  // every chain constant over the window: no autocorrelation estimate exists.  W = 0 up to
  // the rounding of the chain means: W <= (1e-10 max_m |mean_m|)^2
  for (int i = 0; i < d; ++i) {
    double scale = 0;
    for (int64_t c = 0; c < N; ++c) scale = std::max(scale, std::fabs(mean[i * N + c]));
    if (!(W[i] > (1e-10 * scale) * (1e-10 * scale))) {
      done[i] = 1;
      flag[i] = BEST_ESS_FROZEN;
    }
  }
  bool any_left = false;
  for (int i = 0; i < d; ++i) any_left |= !done[i];
  for (int64_t lag0 = 0; any_left && lag0 < T; lag0 += kEssLB) {
    HIPCHK(h, launch_ess_autocov(record, es_mean, T, d, N, lag0, es_part, h->stream));
    HIPCHK(h, hipMemcpyAsync(part.data(), es_part, part.size() * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < d; ++i) {
      for (int t = 0; t < kEssLB && lag0 + t < T; ++t) {
        double g = 0;
        for (int64_t b = 0; b < nblk; ++b) g += part[((size_t)i * nblk + b) * kEssLB + t];
        const double gbar = g / ((double)N * (double)T);
        rho[i].push_back(lag0 + t == 0 ? 1.0 : 1.0 - (W[i] - gbar) / var_plus[i]);
      }
    }
    bool all = true;
    for (int i = 0; i < d; ++i) {
      if (done[i]) continue;
      const auto& r = rho[i];
      const int64_t avail = (int64_t)r.size();
      std::vector<double> sums;
      bool ended = false;
      int64_t k = 0;
      for (; 2 * k + 1 < T; ++k) {
        if (2 * k + 1 >= avail) break;
        const double pk = r[2 * k] + r[2 * k + 1];
        if (!(pk > 0.0)) {
          ended = true;
          break;
        }
        sums.push_back(pk);
      }
      if (!ended && 2 * k + 1 < T) {
        all = false;
        continue;
      }
      if (!ended) flag[i] = BEST_ESS_UNTRUNCATED;
      double s = 0;
      for (size_t q = 0; q < sums.size(); ++q) {
        if (q > 0) sums[q] = std::min(sums[q], sums[q - 1]);
        s += sums[q];
      }
      // floor 1 / log10(N T): antithetic chains can make the truncated sum fall below 1/2
      tau[i] = std::max(-1.0 + 2.0 * s, 1.0 / std::log10((double)N * (double)T));
      done[i] = 1;
    }
    if (all) break;
  }
  for (int i = 0; i < d; ++i) {
    ess_out[i] = flag[i] == BEST_ESS_FROZEN ? 0.0 : (double)N * (double)T / tau[i];
    if (flags_out) flags_out[i] = flag[i];
  }
  return BEST_OK;
}

extern "C" {

int best_ess(best_ctx* h, const float* record, int64_t T, double* ess_out, int32_t* flags_out) {
  if (!h) return BEST_EINVAL;
  if (!record || !ess_out || T < 4) return fail(h, BEST_EINVAL, "record/ess_out NULL or T < 4");
  const int d = h->d;
  const int64_t N = h->N, nblk = (N + 63) / 64;
  if (h->es_cap < N) {
    h->mem.release(h->es_mean);
    h->mem.release(h->es_ssq);
    h->mem.release(h->es_part);
    h->es_cap = 0;
    if (h->mem.alloc(&h->es_mean, (size_t)d * N) != hipSuccess ||
        h->mem.alloc(&h->es_ssq, (size_t)d * N) != hipSuccess ||
        h->mem.alloc(&h->es_part, (size_t)d * nblk * kEssLB) != hipSuccess)
      return fail(h, BEST_ENOMEM, "ESS scratch");
    h->es_cap = N;
  }
  return ess_impl(h, record, T, h->es_mean, h->es_ssq, h->es_part, ess_out, flags_out);
}

int best_ess_noalloc(best_ctx* h, const float* record, int64_t T, double* ess_out,
                     int32_t* flags_out) {
  if (!h) return BEST_EINVAL;
  if (!record || !ess_out || T < 4) return fail(h, BEST_EINVAL, "record/ess_out NULL or T < 4");
  const int64_t N = h->N, nblk = (N + 63) / 64, dn = (int64_t)h->d * nblk * 64;
  if (dn > kNoAllocMaxDN)
    return fail(h, BEST_EINVAL, "best_ess_noalloc: d * ceil(n_chains / 64) * 64 = " +
                                    std::to_string(dn) + " exceeds the fixed scratch limit " +
                                    std::to_string(kNoAllocMaxDN));
  if (!h->scratch)
    return fail_hip(h, "best_ess_noalloc: fixed scratch address", h->scratch_err);
  int cur = -1;
  HIPCHK(h, hipGetDevice(&cur));
  if (cur != h->dev) return fail(h, BEST_ESTATE, "best_ess_noalloc: the context's device is not current");
  // carve mean [d N], ssq [d N], part [d nblk kEssLB] out of the fixed array; the kernels
  // write every element they later read, so nothing needs clearing between calls
  double* mean = h->scratch;
  double* ssq = mean + dn;
  double* part = ssq + dn;
  return ess_impl(h, record, T, mean, ssq, part, ess_out, flags_out);
}

// ---------------------------------------------------------------------------------------
// Convergence metrics (Sec. 4.1)
// ---------------------------------------------------------------------------------------
}  // extern "C"

namespace {

struct DevBuf {  // temporary device buffer of one metric call
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
  double* f64() const { return (double*)p; }
  int* i32() const { return (int*)p; }
};

// Eigenvalues of a symmetric d x d matrix (row-major, overwritten) by cyclic Jacobi rotations
// (Golub & Van Loan, Matrix Computations, Sec. 8.5), sweeping until the off-diagonal mass is
// below 1e-30 of the total.
void sym_eigenvalues(std::vector<double>& A, int d, std::vector<double>& ev) {
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        const double v = A[i * d + j] * A[i * d + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double apq = A[p * d + q];
        if (apq == 0.0) continue;
        const double tau = (A[q * d + q] - A[p * d + p]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(tau * tau + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < d; ++k) {
          const double akp = A[k * d + p], akq = A[k * d + q];
          A[k * d + p] = c * akp - s * akq;
          A[k * d + q] = s * akp + c * akq;
        }
        for (int k = 0; k < d; ++k) {
          const double apk = A[p * d + k], aqk = A[q * d + k];
          A[p * d + k] = c * apk - s * aqk;
          A[q * d + k] = s * apk + c * aqk;
        }
      }
  }
  ev.resize(d);
  for (int i = 0; i < d; ++i) ev[i] = A[i * d + i];
}

// Symmetric matrix from the moment sums of n items (slot layout of the moments pass):
// (sum of products - sum_i sum_j / n) / denom.
std::vector<double> scatter_matrix(const std::vector<double>& sums, int d, double n,
                                   double denom, bool centre) {
  std::vector<double> S((size_t)d * d);
  int q = d;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j, ++q) {
      const double c = (sums[q] - (centre ? sums[i] * sums[j] / n : 0.0)) / denom;
      S[i * d + j] = S[j * d + i] = c;
    }
  return S;
}

int upload_whitening(best_ctx* h, const double* mu, const double* L, DevBuf& mu_d,
                     DevBuf& L_d) {
  if (!mu) return BEST_OK;
  const int d = h->d;
  if (!L) return fail(h, BEST_EINVAL, "whitening needs both mu and L");
  for (int i = 0; i < d; ++i)
    if (!(L[i * d + i] > 0) || !std::isfinite(L[i * d + i]))
      return fail(h, BEST_EINVAL, "L must have a positive diagonal");
  HIPCHK(h, mu_d.alloc((size_t)d * 8));
  HIPCHK(h, L_d.alloc((size_t)d * d * 8));
  HIPCHK(h, hipMemcpyAsync(mu_d.p, mu, (size_t)d * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(L_d.p, L, (size_t)d * d * 8, hipMemcpyHostToDevice, h->stream));
  return BEST_OK;
}

}  // namespace

extern "C" {

int best_rhat(best_ctx* h, const float* samples, int64_t T, int64_t n_chains, double* rminus1) {
  if (!h) return BEST_EINVAL;
  if (!samples || !rminus1 || T < 2 || n_chains < 2)
    return fail(h, BEST_EINVAL, "samples/rminus1 NULL, T < 2 or n_chains < 2");
  const int d = h->d, np = d + d * (d + 1) / 2, nblocks = 256;
  const int64_t N = n_chains;
  DevBuf mean, ssq, part, sums, shift0;
  HIPCHK(h, mean.alloc((size_t)d * N * 8));
  HIPCHK(h, ssq.alloc((size_t)d * N * 8));
  HIPCHK(h, part.alloc((size_t)nblocks * np * 8));
  HIPCHK(h, sums.alloc((size_t)np * 8));
  HIPCHK(h, shift0.alloc((size_t)d * 8));
  std::vector<double> sw(np), sb(np);
  // chain means, then the within-chain scatter about each chain's own mean
  HIPCHK(h, launch_ess_chain_stats(samples, T, d, N, mean.f64(), ssq.f64(), h->stream));
  HIPCHK(h, launch_moment_sums(samples, nullptr, T, N, N, d, mean.f64(), N,
                               part.f64(), nblocks, h->stream));
  HIPCHK(h, launch_sum_parts(part.f64(), nblocks, np, sums.f64(), h->stream));
  HIPCHK(h, hipMemcpyAsync(sw.data(), sums.p, (size_t)np * 8, hipMemcpyDeviceToHost, h->stream));
  // scatter of the chain means about chain 0's mean
  HIPCHK(h, hipMemcpy2DAsync(shift0.p, 8, mean.p, (size_t)N * 8, 8, d, hipMemcpyDeviceToDevice,
                             h->stream));
  HIPCHK(h, launch_moment_sums(nullptr, mean.f64(), 1, N, N, d, shift0.f64(), 0,
                               part.f64(), nblocks, h->stream));
  HIPCHK(h, launch_sum_parts(part.f64(), nblocks, np, sums.f64(), h->stream));
  HIPCHK(h, hipMemcpyAsync(sb.data(), sums.p, (size_t)np * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  // W = mean of the chain covariances, B = covariance of the chain means (both unbiased)
  std::vector<double> W = scatter_matrix(sw, d, (double)(T * N), (double)N * (double)(T - 1), false);
  std::vector<double> Bm = scatter_matrix(sb, d, (double)N, (double)(N - 1), true);
  std::vector<double> dg(d);
  for (int i = 0; i < d; ++i) {
    dg[i] = std::sqrt(Bm[i * d + i]);
    if (!(dg[i] > 0) || !std::isfinite(dg[i]))
      return fail(h, BEST_EINVAL, "the chain means of a parameter are all equal (B_ii = 0)");
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      W[i * d + j] /= dg[i] * dg[j];
      Bm[i * d + j] /= dg[i] * dg[j];
    }
  // eigenvalues of W~^-1 B~ = those of G^-1 B~ G^-T with W~ = G G^T
  std::vector<double> G((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = W[i * d + j];
      for (int k = 0; k < j; ++k) s -= G[i * d + k] * G[j * d + k];
      if (i == j) {
        if (!(s > 0) || !std::isfinite(s))
          return fail(h, BEST_ENOTPD, "mean within-chain covariance is not positive definite");
        G[i * d + i] = std::sqrt(s);
      } else {
        G[i * d + j] = s / G[j * d + j];
      }
    }
  auto fsub = [&](std::vector<double>& M) {  // M <- G^-1 M, column by column
    for (int c = 0; c < d; ++c)
      for (int i = 0; i < d; ++i) {
        double s = M[i * d + c];
        for (int k = 0; k < i; ++k) s -= G[i * d + k] * M[k * d + c];
        M[i * d + c] = s / G[i * d + i];
      }
  };
  fsub(Bm);  // Y = G^-1 B~
  std::vector<double> C((size_t)d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) C[i * d + j] = Bm[j * d + i];  // Y^T = B~ G^-T
  fsub(C);  // G^-1 B~ G^-T
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < i; ++j) C[i * d + j] = C[j * d + i] = 0.5 * (C[i * d + j] + C[j * d + i]);
  std::vector<double> ev;
  sym_eigenvalues(C, d, ev);
  double r = 0;
  for (double v : ev) r = std::max(r, std::fabs(v));
  *rminus1 = r;
  return BEST_OK;
}

int best_credible(best_ctx* h, const float* samples, int64_t T, int64_t n_chains, double alpha,
                  const double* mu, const double* L, const double* ref_lo, const double* ref_hi,
                  double* lo, double* hi, double* metric) {
  if (!h) return BEST_EINVAL;
  if (!samples || T < 1 || n_chains < 1) return fail(h, BEST_EINVAL, "samples NULL or empty");
  if (!(alpha > 0 && alpha < 1)) return fail(h, BEST_EINVAL, "alpha must be in (0, 1)");
  if ((ref_lo == nullptr) != (ref_hi == nullptr) || (ref_lo && !metric))
    return fail(h, BEST_EINVAL, "ref_lo, ref_hi and metric go together");
  const int d = h->d;
  const int64_t n = T * n_chains;
  if (n >= ((int64_t)1 << 31)) return fail(h, BEST_EINVAL, "more than 2^31 - 1 draws");
  int rc;
  DevBuf mu_d, L_d, z, sorted, temp;
  if ((rc = upload_whitening(h, mu, L, mu_d, L_d))) return rc;
  HIPCHK(h, z.alloc((size_t)d * n * 8));
  HIPCHK(h, sorted.alloc((size_t)n * 8));
  HIPCHK(h, launch_whiten_points(samples, T, d, n_chains, mu_d.f64(), L_d.f64(),
                                 z.f64(), n, h->stream));
  size_t tb = 0;
  HIPCHK(h, sort_keys_f64(nullptr, &tb, nullptr, nullptr, n, h->stream));
  HIPCHK(h, temp.alloc(tb));
  const double a = (1.0 - alpha) / 2.0;
  const double lev[2] = {a, 1.0 - a};
  std::vector<double> got((size_t)d * 4, 0.0);
  std::vector<int64_t> kk(2);
  for (int l = 0; l < 2; ++l) kk[l] = (int64_t)std::floor((double)(n - 1) * lev[l]);
  for (int i = 0; i < d; ++i) {
    size_t tbi = tb;
    HIPCHK(h, sort_keys_f64(temp.p, &tbi, z.f64() + (size_t)i * n, sorted.f64(), n,
                            h->stream));
    for (int l = 0; l < 2; ++l) {
      const int64_t k = std::min<int64_t>(kk[l], n - 1);
      const int cnt = k + 1 < n ? 2 : 1;
      HIPCHK(h, hipMemcpyAsync(&got[(size_t)i * 4 + 2 * l], sorted.f64() + k, cnt * 8,
                               hipMemcpyDeviceToHost, h->stream));
    }
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double worst = 0;
  for (int i = 0; i < d; ++i) {
    double q[2];
    for (int l = 0; l < 2; ++l) {
      const double hh = (double)(n - 1) * lev[l];
      const int64_t k = (int64_t)std::floor(hh);
      const double v0 = got[(size_t)i * 4 + 2 * l], v1 = got[(size_t)i * 4 + 2 * l + 1];
      q[l] = k >= n - 1 ? v0 : v0 + (hh - (double)k) * (v1 - v0);
    }
    if (lo) lo[i] = q[0];
    if (hi) hi[i] = q[1];
    if (ref_lo) {
      const double dl = (std::fabs(q[1] - ref_hi[i]) + std::fabs(q[0] - ref_lo[i])) /
                        (ref_hi[i] - ref_lo[i]);
      worst = std::max(worst, dl);
    }
  }
  if (ref_lo) *metric = worst;
  return BEST_OK;
}

int best_sliced_wasserstein(best_ctx* h, const float* a, int64_t Ta, int64_t chains_a,
                            const float* b, int64_t Tb, int64_t chains_b, int32_t n_proj,
                            uint64_t proj_seed, const double* mu, const double* L, double* out) {
  if (!h) return BEST_EINVAL;
  if (!a || !b || !out || Ta < 1 || Tb < 1 || chains_a < 1 || chains_b < 1 || n_proj < 1)
    return fail(h, BEST_EINVAL, "NULL argument, empty sample set or n_proj < 1");
  const int d = h->d;
  const int64_t na = Ta * chains_a, nb = Tb * chains_b, n = na + nb;
  if (n >= ((int64_t)1 << 31)) return fail(h, BEST_EINVAL, "more than 2^31 - 1 draws");
  const int P = std::min<int>(16, n_proj), nparts = 256;
  int rc;
  DevBuf mu_d, L_d, za, zb, w, keys, ks, lab, ls, scan, part, res, temp;
  if ((rc = upload_whitening(h, mu, L, mu_d, L_d))) return rc;
  HIPCHK(h, za.alloc((size_t)d * na * 8));
  HIPCHK(h, zb.alloc((size_t)d * nb * 8));
  HIPCHK(h, w.alloc((size_t)n_proj * d * 8));
  HIPCHK(h, keys.alloc((size_t)P * n * 8));
  HIPCHK(h, ks.alloc((size_t)n * 8));
  HIPCHK(h, lab.alloc((size_t)n * 4));
  HIPCHK(h, ls.alloc((size_t)n * 4));
  HIPCHK(h, scan.alloc((size_t)n * 4));
  HIPCHK(h, part.alloc((size_t)nparts * 8));
  HIPCHK(h, res.alloc((size_t)n_proj * 8));
  size_t tb = 0;
  HIPCHK(h, sliced_w1_workspace(n, &tb));
  HIPCHK(h, temp.alloc(tb));
  HIPCHK(h, launch_whiten_points(a, Ta, d, chains_a, mu_d.f64(), L_d.f64(),
                                 za.f64(), na, h->stream));
  HIPCHK(h, launch_whiten_points(b, Tb, d, chains_b, mu_d.f64(), L_d.f64(),
                                 zb.f64(), nb, h->stream));
  const Rng rng{(uint32_t)(proj_seed & 0xFFFFFFFFu), (uint32_t)(proj_seed >> 32)};
  HIPCHK(h, launch_directions(rng, d, n_proj, w.f64(), h->stream));
  HIPCHK(h, hipMemsetD32Async((hipDeviceptr_t)lab.i32(), 0, (size_t)na, h->stream));
  HIPCHK(h, hipMemsetD32Async((hipDeviceptr_t)(lab.i32() + na), 1, (size_t)nb, h->stream));
  for (int k0 = 0; k0 < n_proj; k0 += P) {
    const int pk = std::min(P, n_proj - k0);
    const double* wk = w.f64() + (size_t)k0 * d;
    HIPCHK(h, launch_project(za.f64(), d, na, na, wk, pk, keys.f64(), n, h->stream));
    HIPCHK(h, launch_project(zb.f64(), d, nb, nb, wk, pk, keys.f64() + na, n,
                             h->stream));
    for (int p = 0; p < pk; ++p)
      HIPCHK(h, sliced_w1_one(temp.p, tb, keys.f64() + (size_t)p * n, ks.f64(),
                              lab.i32(), ls.i32(), scan.i32(), n, na, nb,
                              part.f64(), nparts, res.f64() + k0 + p, h->stream));
  }
  std::vector<double> r(n_proj);
  HIPCHK(h, hipMemcpyAsync(r.data(), res.p, (size_t)n_proj * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double s = 0;
  for (double v : r) s += v;
  *out = s / n_proj;
  return BEST_OK;
}


}  // extern "C"

// =======================================================================================
// Trainer
// =======================================================================================
struct best_trainer {
  std::string err;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  int d = 0, H = 0, nh = 0, prec = BEST_FP32, MT = 2;
  int64_t np = 0, t = 0;
  Arena mem;
  double *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  void *wf = nullptr, *wb = nullptr, *w1f = nullptr, *w1t = nullptr, *bias = nullptr,
       *wout = nullptr;
  MlpParams mp{};
  LdsLayout lds{};
  void* hsave = nullptr;
  int64_t hsave_stride = 0;
  int grid_cap = 0;
  int64_t bcap = 0;
  float *ex_h = nullptr, *ex_dl = nullptr, *ex_th = nullptr, *ex_up = nullptr;
  double *loss_part = nullptr, *loss_steps = nullptr;
  int64_t ls_cap = 0;
  int32_t* ident = nullptr;
  int64_t* offs = nullptr;
  std::vector<int64_t> w_offs;
};

static int tfail(best_trainer* t, int code, const std::string& msg) {
  if (t) t->err = msg;
  return code;
}
#define THIPCHK(t, x)                                                               \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) return tfail((t), BEST_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

static int trainer_buffers(best_trainer* t, int64_t B) {
  if (B <= t->bcap) return BEST_OK;
  for (void* q : {(void*)t->ex_h, (void*)t->ex_dl, (void*)t->ex_th, (void*)t->ex_up,
                  (void*)t->loss_part, (void*)t->ident})
    t->mem.release(q);
  t->bcap = 0;
  const int64_t M = 16 * t->MT;
  if (t->mem.alloc(&t->ex_h, (size_t)t->nh * t->H * B) != hipSuccess ||
      t->mem.alloc(&t->ex_dl, (size_t)t->nh * t->H * B) != hipSuccess ||
      t->mem.alloc(&t->ex_th, (size_t)t->d * B) != hipSuccess ||
      t->mem.alloc(&t->ex_up, (size_t)B) != hipSuccess ||
      t->mem.alloc(&t->loss_part, (size_t)(B + M - 1) / M) != hipSuccess ||
      t->mem.alloc(&t->ident, (size_t)B) != hipSuccess)
    return tfail(t, BEST_ENOMEM, "training buffers");
  std::vector<int32_t> id(B);
  for (int64_t i = 0; i < B; ++i) id[i] = (int32_t)i;
  THIPCHK(t, hipMemcpyAsync(t->ident, id.data(), B * 4, hipMemcpyHostToDevice, t->stream));
  THIPCHK(t, hipStreamSynchronize(t->stream));
  t->bcap = B;
  return BEST_OK;
}

// Forward + backward over one minibatch and the weight gradients into t->g.
static int trainer_grad(best_trainer* t, const float* t_in, const float* y, const int32_t* perm,
                        int64_t batch0, int64_t B, double* loss_out_dev) {
  TrainArgs a{};
  a.mp = t->mp;
  a.lds = t->lds;
  a.t_in = t_in;
  a.y = y;
  a.perm = perm;
  a.batch0 = batch0;
  a.B = B;
  const int64_t M = 16 * t->MT;
  a.n_tiles = (B + M - 1) / M;
  a.hsave = t->hsave;
  a.hsave_stride = t->hsave_stride;
  a.ex_h = t->ex_h;
  a.ex_dl = t->ex_dl;
  a.ex_th = t->ex_th;
  a.ex_up = t->ex_up;
  a.loss_part = t->loss_part;
  const int grid = (int)std::min<int64_t>(a.n_tiles, t->grid_cap);
  THIPCHK(t, launch_train_tile(t->prec, t->MT, a, grid, t->lds.total, t->stream));
  THIPCHK(t, launch_dw(t->ex_dl, t->ex_h, t->ex_th, t->ex_up, B, t->d, t->H, t->nh, t->g,
                       t->offs, t->w_offs.data(), t->stream));
  THIPCHK(t, launch_sum(t->loss_part, (int)a.n_tiles, 1.0 / (double)B, loss_out_dev, t->stream));
  return BEST_OK;
}

extern "C" {

int best_trainer_create(best_trainer** out, int32_t d, int32_t width, int32_t n_hidden,
                        const double* init_params, int32_t precision, void* stream) {
  if (!out) return BEST_EINVAL;
  *out = nullptr;
  if (d < 1 || d > kMaxD || width < 128 || width > 2048 || width % 128 || n_hidden < 1 ||
      n_hidden > 16 || !init_params)
    return BEST_EINVAL;
  if (precision != BEST_FP32 && precision != BEST_FP16 && precision != BEST_BF16)
    return BEST_EINVAL;
  best_trainer* t = new (std::nothrow) best_trainer();
  if (!t) return BEST_ENOMEM;
  auto bail = [&](int code) {
    std::fprintf(stderr, "best_trainer_create: %s\n", t->err.c_str());
    best_trainer_destroy(t);
    return code;
  };
  t->stream = (hipStream_t)stream;
  t->d = d;
  t->H = width;
  t->nh = n_hidden;
  t->prec = precision;
  t->np = mlp_nparams_impl(d, width, n_hidden);
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&t->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (he != hipSuccess)
    return bail(tfail(t, BEST_EHIP, std::string("no usable HIP device: ") + hipGetErrorString(he)));
  t->MT = 2;
  while (t->MT > 1 && layout_for(precision, t->MT, width, d, n_hidden, 0).total > kLdsMax) t->MT /= 2;
  const int lds_h = layout_for(precision, t->MT, width, d, n_hidden, 1).total <= kLdsMax ? 1 : 0;
  t->lds = layout_for(precision, t->MT, width, d, n_hidden, lds_h);
  if (t->lds.total > kLdsMax) return bail(tfail(t, BEST_EINVAL, "width too large for LDS"));
  if (!finite_all(init_params, t->np)) return bail(tfail(t, BEST_EINVAL, "init params must be finite"));
  const int ts = tsize(precision);
  const size_t nW = (size_t)std::max(n_hidden - 1, 1) * width * width;
  if (t->mem.upload(&t->p, init_params, t->np, t->stream) != hipSuccess ||
      t->mem.alloc(&t->m, t->np) != hipSuccess || t->mem.alloc(&t->v, t->np) != hipSuccess ||
      t->mem.alloc(&t->g, t->np) != hipSuccess ||
      t->mem.alloc((char**)&t->wf, nW * ts) != hipSuccess ||
      t->mem.alloc((char**)&t->wb, nW * ts) != hipSuccess ||
      t->mem.alloc((char**)&t->w1f, w1f_bytes(precision, width, d)) != hipSuccess ||
      t->mem.alloc((char**)&t->w1t, w1t_bytes(precision, width, d)) != hipSuccess ||
      t->mem.alloc((char**)&t->bias, (size_t)n_hidden * width * 4) != hipSuccess ||
      t->mem.alloc((char**)&t->wout, (size_t)(width + 1) * 4) != hipSuccess ||
      t->mem.alloc(&t->loss_steps, 1 << 16) != hipSuccess)
    return bail(tfail(t, BEST_ENOMEM, "trainer buffers"));
  t->ls_cap = 1 << 16;
  if (hipMemsetAsync(t->m, 0, t->np * 8, t->stream) != hipSuccess ||
      hipMemsetAsync(t->v, 0, t->np * 8, t->stream) != hipSuccess)
    return bail(tfail(t, BEST_EHIP, "memset"));
  t->mp = make_mlp_params(precision, d, width, n_hidden, lds_h, t->wf, t->wb, t->w1f, t->w1t,
                          t->bias, t->wout);
  t->grid_cap = t->n_cu * std::max(1, std::min(2, kLdsMax / t->lds.total));
  t->hsave_stride = (int64_t)n_hidden * width * 16 * t->MT;
  if (t->mem.alloc((char**)&t->hsave, (size_t)t->grid_cap * t->hsave_stride * 4) != hipSuccess)
    return bail(tfail(t, BEST_ENOMEM, "activation scratch"));
  // gradient offsets: [W1, b1, b2..b_nh, w_out, b_out] and W_l (l >= 2)
  std::vector<int64_t> offs;
  param_offsets(d, width, n_hidden, offs, t->w_offs);
  if (t->mem.upload(&t->offs, offs.data(), offs.size(), t->stream) != hipSuccess)
    return bail(tfail(t, BEST_ENOMEM, "offsets"));
  if (hipError_t e = launch_pack(precision, t->p, d, width, n_hidden, t->wf, t->wb, t->w1f,
                                 t->w1t, t->bias, t->wout, t->stream))
    return bail(tfail(t, BEST_EHIP, std::string("pack: ") + hipGetErrorString(e)));
  if (hipStreamSynchronize(t->stream) != hipSuccess) return bail(tfail(t, BEST_EHIP, "sync"));
  *out = t;
  return BEST_OK;
}

void best_trainer_destroy(best_trainer* t) {
  if (!t) return;
  if (t->stream) (void)hipStreamSynchronize(t->stream);
  else (void)hipDeviceSynchronize();
  t->mem.free_all();
  delete t;
}

const char* best_trainer_last_error(const best_trainer* t) {
  return t ? t->err.c_str() : "null trainer";
}

int best_train_grad(best_trainer* t, const float* t_in, const float* y, int64_t batch,
                    double* grad, double* loss) {
  if (!t) return BEST_EINVAL;
  if (!t_in || !y || batch < 16 || batch % 16) return tfail(t, BEST_EINVAL, "batch must be a positive multiple of 16");
  int rc = trainer_buffers(t, batch);
  if (rc) return rc;
  if ((rc = trainer_grad(t, t_in, y, t->ident, 0, batch, t->loss_steps))) return rc;
  double l = 0;
  if (grad) THIPCHK(t, hipMemcpyAsync(grad, t->g, t->np * 8, hipMemcpyDeviceToHost, t->stream));
  THIPCHK(t, hipMemcpyAsync(&l, t->loss_steps, 8, hipMemcpyDeviceToHost, t->stream));
  THIPCHK(t, hipStreamSynchronize(t->stream));
  if (loss) *loss = l;
  return BEST_OK;
}

int best_train_epoch(best_trainer* t, const float* t_in, const float* y, int64_t n,
                     const int32_t* perm, int32_t batch, double lr0, double lr1, int64_t step0,
                     int64_t total_steps, double* mean_loss) {
  if (!t) return BEST_EINVAL;
  if (!t_in || !y || !perm || n < batch || batch < 16 || batch % 16 || total_steps < 1 ||
      !(lr0 > 0) || !(lr1 >= 0))
    return tfail(t, BEST_EINVAL, "invalid training arguments");
  const int64_t nb = n / batch;
  if (nb > t->ls_cap) return tfail(t, BEST_EINVAL, "too many batches per epoch");
  int rc = trainer_buffers(t, batch);
  if (rc) return rc;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  for (int64_t i = 0; i < nb; ++i) {
    if ((rc = trainer_grad(t, t_in, y, perm, i * batch, batch, t->loss_steps + i))) return rc;
    t->t += 1;
    const double c1 = 1.0 - std::pow(b1, (double)t->t), c2 = 1.0 - std::pow(b2, (double)t->t);
    const double s = (double)(step0 + i);
    const double lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + std::cos(M_PI * s / (double)total_steps));
    THIPCHK(t, launch_adam(t->p, t->m, t->v, t->g, t->np, lr, b1, b2, eps, c1, c2, t->stream));
    THIPCHK(t, launch_pack(t->prec, t->p, t->d, t->H, t->nh, t->wf, t->wb, t->w1f, t->w1t,
                           t->bias, t->wout, t->stream));
  }
  if (mean_loss) {
    std::vector<double> ls(nb);
    THIPCHK(t, hipMemcpyAsync(ls.data(), t->loss_steps, nb * 8, hipMemcpyDeviceToHost, t->stream));
    THIPCHK(t, hipStreamSynchronize(t->stream));
    double s = 0;
    for (double v : ls) s += v;
    *mean_loss = s / (double)nb;
  }
  return BEST_OK;
}

int best_trainer_get_params(best_trainer* t, double* out) {
  if (!t) return BEST_EINVAL;
  if (!out) return tfail(t, BEST_EINVAL, "out is NULL");
  THIPCHK(t, hipMemcpyAsync(out, t->p, t->np * 8, hipMemcpyDeviceToHost, t->stream));
  THIPCHK(t, hipStreamSynchronize(t->stream));
  return BEST_OK;
}

}  // extern "C"

extern "C" {

int best_standardise(const double* y, int64_t n, float* out, double* mean_std, void* stream) {
  if (!y || !out || !mean_std || n < 2) return BEST_EINVAL;
  double* scratch = nullptr;
  if (hipMalloc(&scratch, 520 * sizeof(double)) != hipSuccess) return BEST_ENOMEM;
  double st[4];
  hipError_t e = launch_standardise(y, n, out, scratch, st, (hipStream_t)stream);
  (void)hipFree(scratch);
  if (e != hipSuccess) return BEST_EHIP;
  mean_std[0] = st[0] / (double)n;
  mean_std[1] = std::sqrt(st[2] / (double)n);
  return (std::isfinite(mean_std[1]) && mean_std[1] > 0) ? BEST_OK : BEST_EINVAL;
}

int best_normalise_inputs(const double* x, int64_t n, int32_t d, const double* center,
                          const double* invscale, float* t, void* stream) {
  if (!x || !center || !invscale || !t || n < 1 || d < 1 || d > kMaxD) return BEST_EINVAL;
  InputScaling sc{};
  for (int i = 0; i < d; ++i) {
    if (!std::isfinite(center[i]) || !std::isfinite(invscale[i])) return BEST_EINVAL;
    sc.center[i] = center[i];
    sc.invscale[i] = invscale[i];
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_normalise_inputs(x, n, d, sc, t, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? BEST_OK : BEST_EHIP;
}

int best_importance_weights(const double* logl_plain, const double* logl_emu, int64_t n,
                            double* w, double* kish, void* stream) {
  if (!logl_plain || !logl_emu || !w || n < 1) return BEST_EINVAL;
  double* scratch = nullptr;
  if (hipMalloc(&scratch, 520 * sizeof(double)) != hipSuccess) return BEST_ENOMEM;
  double st[4];
  hipError_t e = launch_importance_weights(logl_plain, logl_emu, n, w, scratch, st,
                                           (hipStream_t)stream);
  (void)hipFree(scratch);
  if (e != hipSuccess) return BEST_EHIP;
  if (kish) kish[0] = st[2] * st[2] / st[3];
  return std::isfinite(st[0]) ? BEST_OK : BEST_EINVAL;
}

}  // extern "C"
