// Mixed-precision local solves (FP32 inner PCG, FP64 residual refinement).
#include "mlc_launch.h"

int64_t item_bytes_fp64(int cw, int ch, int m);

int64_t item_bytes_mixed(int cw, int ch, int m) { return item_bytes_fp64(cw, ch, m); }

hipError_t launch_local_mixed(int, int, const ProbDev*, const TileItem*, int, char*, const double*,
                              int, ItemStat*, double, int, int, double, int, double, hipStream_t) {
  return hipErrorNotSupported;
}
