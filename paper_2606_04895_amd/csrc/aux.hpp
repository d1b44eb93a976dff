// Host-visible launchers of the library's kernels.  Each is defined in the translation
// unit that defines the kernel it launches.
#pragma once
#include "train.hpp"

namespace best {

constexpr int kEssTS = 64;   // time-window rows per autocovariance pass
constexpr int kEssLB = 128;  // lags per autocovariance pass
// Entry points that allocate nothing take their device scratch from one fixed array per
// GPU (kernels_aux.hip).  The ESS passes need 4 d ceil(N/64) 64 doubles of it, so d times
// the 64-padded chain count is limited to kNoAllocMaxDN (32 MiB of scratch per GPU).
constexpr int64_t kNoAllocMaxDN = (int64_t)1 << 20;
constexpr int64_t kNoAllocScratchDoubles = 4 * kNoAllocMaxDN;

// Templated per precision (kernels_<prec>.hip).
hipError_t launch_step(int prec, int MT, const KArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t launch_eval(int prec, int MT, const KArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t launch_pack(int prec, const double* flat, int d, int H, int nh, void* wf, void* wb,
                       void* w1f, void* w1t, void* bias, void* wout, hipStream_t s);
hipError_t launch_train_tile(int prec, int MT, const TrainArgs& a, int grid, size_t lds,
                             hipStream_t s);
hipError_t launch_vjp(int prec, int MT, const VjpArgs& a, int grid, size_t lds, hipStream_t s);

// kernels_aux.hip
hipError_t launch_init_positions(const Target& tg, const State& S, const Rng& rng, int mode,
                                 const double* pt, double scale, const double* L0,
                                 uint64_t step, hipStream_t s);
hipError_t launch_rewhiten(const State& S, const Whiten& W, int d, hipStream_t s);
hipError_t launch_da_update(const double* step_prob, int64_t N, double* da, hipStream_t s);
hipError_t launch_stats(const State& S, int64_t* out_i, double* out_d, hipStream_t s);
hipError_t launch_aies_record(const State& S, int d, float* rec, int64_t slot, int64_t pitch,
                              hipStream_t s);
hipError_t launch_moments(const float* rec, const double* xs, int64_t T, int64_t N,
                          int64_t pitch, int d, const double* shift, double* part, int nblocks,
                          int update_mean, double* mu, double* L, double* info, hipStream_t s);
hipError_t launch_moment_sums(const float* rec, const double* xs, int64_t T, int64_t N,
                              int64_t pitch, int d, const double* shift, int64_t spitch,
                              double* part, int nblocks, hipStream_t s);
hipError_t launch_ess_chain_stats(const float* rec, int64_t T, int d, int64_t N, double* mean,
                                  double* ssq, hipStream_t s);
// Device address of GPU dev's copy of the fixed scratch array (kNoAllocScratchDoubles
// doubles).  The first call for a device must have that device current; the address is
// kept per device and later calls return it.
hipError_t noalloc_scratch_address(int dev, double** p);
hipError_t launch_ess_autocov(const float* rec, const double* mean, int64_t T, int d,
                              int64_t N, int64_t lag0, double* part, hipStream_t s);
hipError_t launch_transpose(const double* src, int64_t rows, int64_t cols, double* dst,
                            hipStream_t s);
struct InputScaling {  // kernel argument: per-component centre and inverse scale
  double center[kMaxD], invscale[kMaxD];
};
hipError_t launch_normalise_inputs(const double* x, int64_t n, int d, const InputScaling& sc,
                                   float* t, hipStream_t s);
hipError_t launch_adam(double* p, double* m, double* v, const double* g, int64_t n, double lr,
                       double b1, double b2, double eps, double c1, double c2, hipStream_t s);
hipError_t launch_dw(const float* dl, const float* h, const float* th, const float* up,
                     int64_t B, int d, int H, int nh, double* grad, const int64_t* offs,
                     const int64_t* w_offs_host, hipStream_t s);
hipError_t launch_sum(const double* part, int n, double scale, double* out, hipStream_t s);
hipError_t launch_standardise(const double* y, int64_t n, float* out, double* scratch,
                              double* stats_host, hipStream_t s);
hipError_t launch_importance_weights(const double* lp, const double* le, int64_t n, double* w,
                                     double* scratch, double* stats_host, hipStream_t s);

// metrics.hip (convergence metrics of Sec. 4.1)
hipError_t launch_whiten_points(const float* rec, int64_t T, int d, int64_t N, const double* mu,
                                const double* L, double* z, int64_t zpitch, hipStream_t s);
hipError_t launch_sum_parts(const double* part, int nblocks, int np, double* out, hipStream_t s);
hipError_t sort_keys_f64(void* temp, size_t* temp_bytes, const double* in, double* out,
                         int64_t n, hipStream_t s);
hipError_t launch_directions(const Rng& rng, int d, int K, double* w, hipStream_t s);
hipError_t launch_project(const double* z, int d, int64_t n, int64_t zpitch, const double* w,
                          int P, double* keys, int64_t kpitch, hipStream_t s);
hipError_t sliced_w1_workspace(int64_t n, size_t* temp_bytes);
hipError_t sliced_w1_one(void* temp, size_t temp_bytes, const double* keys, double* keys_sorted,
                         const int* labels, int* labels_sorted, int* scan, int64_t n, int64_t na,
                         int64_t nb, double* part, int nparts, double* out, hipStream_t s);

}  // namespace best
