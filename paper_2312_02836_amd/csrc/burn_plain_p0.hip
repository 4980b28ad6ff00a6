// burn_plain_p0.hip -- plain-kernel instantiations (see burn_plain.h).
#include "burn_plain.h"

namespace bn {

hipError_t launch_plain_p0(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream,
                           bool *found) {
  BN_PLAIN_CASE(4, 1, 2)
  BN_PLAIN_CASE(4, 2, 2)
  BN_PLAIN_CASE(4, 4, 1)
  BN_PLAIN_CASE(8, 1, 2)
  *found = false;
  return hipErrorInvalidValue;
}

}  // namespace bn
