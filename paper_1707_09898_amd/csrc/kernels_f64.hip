// The FP64 instantiations of kernels.hip (see kernels_f32.hip).
#define TOF_NO_F32
#define TOF_NO_COMMON
#include "kernels.hip"
