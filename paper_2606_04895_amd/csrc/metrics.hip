// Convergence metrics of Sec. 4.1 on the device: whitening of recorded draws, radix sorts
// and scans (hipCUB over rocPRIM), projections onto the fixed directions, and the sums of
// the 1-d Wasserstein distances.  The d x d algebra of the R - 1 statistic runs on the host.
#include <hipcub/hipcub.hpp>

#include "aux.hpp"

namespace best {
namespace {

constexpr int kMetThreads = 256;

// z[i * zp + it] for draw it = t * N + c of a record [T][d][N]: the draw itself, or with
// mu != nullptr its whitened coordinates, L z = x - mu by forward substitution.
__global__ void whiten_points_kernel(const float* rec, int64_t T, int d, int64_t N,
                                     const double* mu, const double* L, double* z, int64_t zp) {
  const int64_t n = T * N;
  for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < n;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = it / N, c = it % N;
    for (int i = 0; i < d; ++i) {
      double r = (double)rec[(t * d + i) * N + c];
      if (mu) {
        r -= mu[i];
        for (int j = 0; j < i; ++j) r -= L[i * d + j] * z[j * zp + it];
        r /= L[i * d + i];
      }
      z[i * zp + it] = r;
    }
  }
}

// out[p] = sum over blocks b of part[b * np + p] (one workgroup, fixed order).
__global__ void sum_parts_kernel(const double* part, int nblocks, int np, double* out) {
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    double s = 0;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * np + p];
    out[p] = s;
  }
}

// Unit direction k: the d normals of Philox counter (k, 0, stream 6, 0), normalised.
__global__ void directions_kernel(Rng rng, int d, int K, double* w) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double nrm = 0;
  for (int i = 0; i < d; ++i) {
    const double xi = normal_dim(rng, (uint64_t)k, 0, kStreamProj, 0, i);
    w[k * d + i] = xi;
    nrm += xi * xi;
  }
  nrm = sqrt(nrm);
  for (int i = 0; i < d; ++i) w[k * d + i] /= nrm;
}

// keys[p * kp + j] = w_p . z_j for P directions (one thread per point).
__global__ void project_kernel(const double* z, int d, int64_t n, int64_t zp, const double* w,
                               int P, double* keys, int64_t kp) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    double zz[kMaxD];
    for (int i = 0; i < d; ++i) zz[i] = z[i * zp + j];
    for (int p = 0; p < P; ++p) {
      double s = 0;
      for (int i = 0; i < d; ++i) s += w[p * d + i] * zz[i];
      keys[p * kp + j] = s;
    }
  }
}

// Per-block partial sums of |F_a - F_b| (v_{k+1} - v_k) over the merged sorted values v:
// after position k, cb = scan[k] values of b and k + 1 - cb values of a are <= v_k.
__global__ void w1_partial_kernel(const double* v, const int* scan, int64_t n, int64_t na,
                                  int64_t nb, double* part) {
  __shared__ double sh[kMetThreads];
  double acc = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n - 1;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cb = scan[k], ca = k + 1 - cb;
    acc += fabs((double)ca / (double)na - (double)cb / (double)nb) * (v[k + 1] - v[k]);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kMetThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

int blocks_for(int64_t n) {
  int64_t g = (n + kMetThreads - 1) / kMetThreads;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

}  // namespace

hipError_t launch_whiten_points(const float* rec, int64_t T, int d, int64_t N, const double* mu,
                                const double* L, double* z, int64_t zpitch, hipStream_t s) {
  hipLaunchKernelGGL(whiten_points_kernel, dim3(blocks_for(T * N)), dim3(kMetThreads), 0, s, rec,
                     T, d, N, mu, L, z, zpitch);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const double* part, int nblocks, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(kMetThreads), 0, s, part, nblocks, np, out);
  return hipGetLastError();
}

hipError_t sort_keys_f64(void* temp, size_t* temp_bytes, const double* in, double* out,
                         int64_t n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortKeys(temp, *temp_bytes, in, out, (int)n, 0, 64, s);
}

hipError_t launch_directions(const Rng& rng, int d, int K, double* w, hipStream_t s) {
  hipLaunchKernelGGL(directions_kernel, dim3((K + kMetThreads - 1) / kMetThreads),
                     dim3(kMetThreads), 0, s, rng, d, K, w);
  return hipGetLastError();
}

hipError_t launch_project(const double* z, int d, int64_t n, int64_t zpitch, const double* w,
                          int P, double* keys, int64_t kpitch, hipStream_t s) {
  hipLaunchKernelGGL(project_kernel, dim3(blocks_for(n)), dim3(kMetThreads), 0, s, z, d, n,
                     zpitch, w, P, keys, kpitch);
  return hipGetLastError();
}

// Scratch bytes shared by the pair sort and the scan of one projection of n values.
hipError_t sliced_w1_workspace(int64_t n, size_t* temp_bytes) {
  size_t a = 0, b = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const double*)nullptr,
                                                     (double*)nullptr, (const int*)nullptr,
                                                     (int*)nullptr, (int)n, 0, 64);
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::InclusiveSum(nullptr, b, (const int*)nullptr, (int*)nullptr, (int)n);
  if (e != hipSuccess) return e;
  *temp_bytes = a > b ? a : b;
  return hipSuccess;
}

// W1 between the first na and the last nb of the n = na + nb projected values (labels 0 / 1):
// sort (value, label), scan the labels, sum |F_a - F_b| over the gaps into *out.
hipError_t sliced_w1_one(void* temp, size_t temp_bytes, const double* keys, double* keys_sorted,
                         const int* labels, int* labels_sorted, int* scan, int64_t n, int64_t na,
                         int64_t nb, double* part, int nparts, double* out, hipStream_t s) {
  size_t tb = temp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, tb, keys, keys_sorted, labels,
                                                     labels_sorted, (int)n, 0, 64, s);
  if (e != hipSuccess) return e;
  tb = temp_bytes;
  e = hipcub::DeviceScan::InclusiveSum(temp, tb, labels_sorted, scan, (int)n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(w1_partial_kernel, dim3(nparts), dim3(kMetThreads), 0, s, keys_sorted, scan,
                     n, na, nb, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_parts(part, nparts, 1, out, s);
}

}  // namespace best
