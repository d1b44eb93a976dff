// double instantiation of the fused tile kernels.
#define BEST_T double
#define BEST_SUFFIX f64
#define BEST_MT_MAX 2
#define BEST_TRAIN 0
#include "kernels_prec.inc"
