// burn_plain_p1.hip -- plain-kernel instantiations (see burn_plain.h).
#include "burn_plain.h"

namespace bn {

hipError_t launch_plain_p1(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream,
                           bool *found) {
  BN_PLAIN_CASE(8, 2, 2)
  BN_PLAIN_CASE(8, 4, 1)
  BN_PLAIN_CASE(16, 1, 2)
  BN_PLAIN_CASE(16, 2, 1)
  *found = false;
  return hipErrorInvalidValue;
}

}  // namespace bn
