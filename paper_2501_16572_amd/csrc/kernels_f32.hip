// FP32 instantiation: v_mfma_f32_16x16x4 with FP32 accumulation (fused path).
#define KX_T float
#define KX_SUFFIX f32
#define KX_PLAIN 0
#include "instantiate.inc"
