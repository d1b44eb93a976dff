// __bf16 instantiation of the fused tile kernels.
#define BEST_T __bf16
#define BEST_SUFFIX bf16
#define BEST_MT_MAX 4
#define BEST_TRAIN 1
#include "kernels_prec.inc"
