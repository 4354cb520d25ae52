// The FP32 instantiations of yzsum.hip (one translation unit per precision,
// so that the two compile in parallel).
#define TOF_NO_F64
#include "yzsum.hip"
