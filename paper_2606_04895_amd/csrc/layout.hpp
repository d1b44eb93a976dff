// Host-side shapes of the tile engine's buffers: element sizes per precision, tile-width
// limits, the input layer's packed weight sizes and the LDS layout for a configuration.  Used
// by the ABI to choose tile widths and by the host-side layout checks.
#pragma once
#include <cstddef>

#include "../../include/best.h"
#include "kernels.hpp"

namespace best {

inline int tsize(int prec) { return prec == BEST_FP64 ? 8 : prec == BEST_FP32 ? 4 : 2; }
inline int vasize(int prec) { return prec == BEST_FP64 ? 8 : 4; }
inline int mt_max(int prec) { return prec == BEST_FP64 ? 2 : 4; }
// Input layer: FP64 MFMA (k-step 8) for the FP64 path, FP32 MFMA (k-step 16) otherwise.
inline int in_kstep(int prec) { return prec == BEST_FP64 ? 8 : 16; }
inline int in_size(int prec) { return prec == BEST_FP64 ? 8 : 4; }
inline int in_ksteps(int prec, int d) { return (d + in_kstep(prec) - 1) / in_kstep(prec); }
inline int grad_rtiles(int d) { return (d + 15) / 16; }

// Packed input-layer weights: W_1 for the input GEMM and W_1^T for the input gradient.
inline size_t w1f_bytes(int prec, int H, int d) {
  return (size_t)H * in_ksteps(prec, d) * in_kstep(prec) * in_size(prec);
}
inline size_t w1t_bytes(int prec, int H, int d) {
  return (size_t)16 * grad_rtiles(d) * H * tsize(prec);
}

inline LdsLayout layout_for(int prec, int MT, int H, int d, int nh, int lds_h, int st_lds = 0,
                            int w1_res = 0) {
  return lds_layout(16 * MT, H, d, nh, lds_h, tsize(prec), vasize(prec), vasize(prec),
                    in_ksteps(prec, d) * in_kstep(prec), in_size(prec), tile_waves(tsize(prec)),
                    st_lds, w1_res ? (int)w1f_bytes(prec, H, d) : 0,
                    w1_res ? (int)w1t_bytes(prec, H, d) : 0);
}

}  // namespace best
