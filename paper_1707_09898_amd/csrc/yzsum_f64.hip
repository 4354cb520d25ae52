// The FP64 instantiations of yzsum.hip (see yzsum_f32.hip).
#define TOF_NO_F32
#include "yzsum.hip"
