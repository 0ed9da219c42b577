// FP64 instantiation of the operator kernels.
#include "bw_ops_impl.h"

namespace bw {
BW_INSTANTIATE_OPS(double)
}
