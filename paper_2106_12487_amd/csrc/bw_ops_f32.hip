// FP32 instantiation of the operator kernels (mixed-precision path).
#include "bw_ops_impl.h"

namespace bw {
BW_INSTANTIATE_OPS(float)
}
