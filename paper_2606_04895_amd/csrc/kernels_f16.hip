// _Float16 instantiation of the fused tile kernels.
#define BEST_T _Float16
#define BEST_SUFFIX f16
#define BEST_MT_MAX 4
#define BEST_TRAIN 1
#include "kernels_prec.inc"
