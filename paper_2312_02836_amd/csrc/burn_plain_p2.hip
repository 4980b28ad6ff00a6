// burn_plain_p2.hip -- plain-kernel instantiations (see burn_plain.h).
#include "burn_plain.h"

namespace bn {

hipError_t launch_plain_p2(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream,
                           bool *found) {
  BN_PLAIN_CASE(32, 1, 2)
  BN_PLAIN_CASE(16, 4, 1)
  BN_PLAIN_CASE(32, 2, 1)
  BN_PLAIN_CASE(64, 1, 1)
  *found = false;
  return hipErrorInvalidValue;
}

}  // namespace bn
