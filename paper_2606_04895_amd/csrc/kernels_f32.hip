// float instantiation of the fused tile kernels.
#define BEST_T float
#define BEST_SUFFIX f32
#define BEST_MT_MAX 4
#define BEST_TRAIN 1
#include "kernels_prec.inc"
