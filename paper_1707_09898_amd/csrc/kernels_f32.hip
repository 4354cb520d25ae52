// The FP32 instantiations of kernels.hip and its kernels of no element type
// (one translation unit per precision, so that the two compile in parallel).
#define TOF_NO_F64
#include "kernels.hip"
