// Eigen-solver layer (placeholder until the subspace / Lanczos drivers land).
#include "bw_internal.h"

extern "C" int bw_lowest_modes(bw_rve*, const double*, int32_t, int32_t, const bw_eig_opts*, double*, double*,
                               void*, bw_stats*, void*) {
  bw::set_error("bw_lowest_modes: not built yet");
  return BW_EUNSUPPORTED;
}
