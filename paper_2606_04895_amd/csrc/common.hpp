// Device-side building blocks shared by every kernel of the library: MFMA precision
// traits, the Philox4x32-10 generator and its uniform / normal maps, wave reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace best {

// Waves per tile workgroup, by GEMM element size: 8 (two per SIMD) for the 16-bit types,
// whose L2 weight stream needs the extra waves in flight, 4 (one per SIMD, the whole
// register file each) for FP32 and FP64.  Each precision's translation unit sets
// BEST_WAVES from this rule; the host sizes LDS with the same rule.
#ifndef BEST_WAVES16
#define BEST_WAVES16 8
#endif
constexpr int tile_waves(int elem_bytes) { return elem_bytes == 2 ? BEST_WAVES16 : 4; }
#ifndef BEST_WAVES
#define BEST_WAVES 4
#endif
constexpr int kWaves = BEST_WAVES;
constexpr int kThreads = 64 * kWaves;
constexpr int kAuxThreads = 256;  // block size of the small reduction kernels
constexpr int kMaxD = 32;

// ---------------------------------------------------------------------------------------
// MFMA traits.  Every 16x16 tile product is expressed per "k-step": each lane holds 16
// bytes of the A operand (row = lane % 16) and 16 bytes of the B operand (col = lane % 16)
// covering EPL consecutive k values starting at (lane / 16) * EPL; the k-step spans
// KSTEP = 4 * EPL values.  In the D tile lane l holds column l % 16 and, in slot r, row
// drow(l / 16, r): 4*(l/16) + r for the FP32/FP16/BF16 instructions, l/16 + 4 r for FP64
// (both measured on gfx950 with a one-wave probe).
// ---------------------------------------------------------------------------------------
template <typename T>
struct Prec;

template <>
struct Prec<__bf16> {
  using T = __bf16;
  using acc = float;   // accumulator / epilogue type
  using vec = float;   // type of the vector (non-MFMA) layers
  using frag = bf16x8;
  using accv = f32x4;
  static constexpr int EPL = 8, KSTEP = 32;
  static constexpr bool ROWS4 = true;  // D slots r = 0..3 hold rows 4g .. 4g + 3
  __host__ __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
  __device__ static accv mma(frag a, frag b, accv c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Prec<_Float16> {
  using T = _Float16;
  using acc = float;
  using vec = float;
  using frag = f16x8;
  using accv = f32x4;
  static constexpr int EPL = 8, KSTEP = 32;
  static constexpr bool ROWS4 = true;
  __host__ __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
  __device__ static accv mma(frag a, frag b, accv c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Prec<float> {
  using T = float;
  using acc = float;
  using vec = float;
  using frag = f32x4;
  using accv = f32x4;
  static constexpr int EPL = 4, KSTEP = 16;
  static constexpr bool ROWS4 = true;
  __host__ __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
  __device__ static accv mma(frag a, frag b, accv c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
    return c;
  }
};

template <>
struct Prec<double> {
  using T = double;
  using acc = double;
  using vec = double;
  using frag = f64x2;
  using accv = f64x4;
  static constexpr int EPL = 2, KSTEP = 8;
  static constexpr bool ROWS4 = false;
  // the FP64 16x16x4 MFMA returns rows g + 4 r in slot r of lane group g (strided)
  __host__ __device__ static constexpr int drow(int g, int r) { return g + 4 * r; }
  __device__ static accv mma(frag a, frag b, accv c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
    return c;
  }
};

// Offset (in elements) of element (row, k) in a fragment-ordered matrix with KS k-steps.
// Fragment (rt, ks) is 64 lanes x EPL contiguous elements; lane = row%16 + 16*(k%KSTEP/EPL).
template <class P>
__host__ __device__ inline int64_t frag_offset(int64_t row, int64_t k, int64_t KS) {
  const int64_t ks = k / P::KSTEP, w = k % P::KSTEP;
  const int64_t lane = (row & 15) + 16 * (w / P::EPL);
  return (((row >> 4) * KS + ks) * 64 + lane) * P::EPL + (w % P::EPL);
}

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): 10 rounds of two 32x32->64-bit
// multiplies mixed with the key, Weyl key schedule.
// ---------------------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

enum Stream : uint32_t {
  kStreamNormal = 1,
  kStreamAccept = 2,
  kStreamAies = 3,
  kStreamInit = 4,
  kStreamNuts = 5,
  kStreamProj = 6,
  kStreamDE = 7
};

struct Rng {
  uint32_t k0, k1;
  __device__ U4 block(uint64_t chain, uint64_t step, uint32_t stream, uint32_t sub,
                      uint32_t blk) const {
    return philox((uint32_t)chain, (uint32_t)step, (stream << 24) | sub, blk, k0, k1);
  }
};

// (ra >> 6) * 2^26 + (rb >> 6) is a 52-bit integer n; (n + 0.5) 2^-52 is exact in FP64.
__device__ __forceinline__ double u52(uint32_t ra, uint32_t rb) {
  const uint64_t n = ((uint64_t)(ra >> 6) << 26) | (uint64_t)(rb >> 6);
  return ((double)n + 0.5) * 0x1p-52;
}

// Box-Muller pair from one block: r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2).
__device__ __forceinline__ void normal_pair(const U4& b, double& n0, double& n1) {
  const double ua = u52(b.x, b.y), ub = u52(b.z, b.w);
  const double r = sqrt(-2.0 * log(ua));
  const double ang = 2.0 * 3.141592653589793 * ub;
  double s, c;
  sincos(ang, &s, &c);
  n0 = r * c;
  n1 = r * s;
}

// Normal for dimension i of chain `chain`: block i/2, member i%2.
__device__ __forceinline__ double normal_dim(const Rng& g, uint64_t chain, uint64_t step,
                                             uint32_t stream, uint32_t sub, int i) {
  const U4 b = g.block(chain, step, stream, sub, (uint32_t)(i >> 1));
  double n0, n1;
  normal_pair(b, n0, n1);
  return (i & 1) ? n1 : n0;
}

__device__ __forceinline__ double accept_uniform(const Rng& g, uint64_t chain, uint64_t step,
                                                 uint32_t sub) {
  const U4 b = g.block(chain, step, kStreamAccept, sub, 0);
  return u52(b.x, b.y);
}

// ---------------------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V sum_lane_groups(V v) {  // lanes l, l^16, l^32, l^48
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

}  // namespace best
