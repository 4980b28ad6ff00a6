// Host build of the kernels' logarithm for its accuracy test: the same
// source, evaluated operation by operation as on the device.
#include "bn_math.h"

extern "C" void bn_log_host(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = bn::bn_log(x[i]);
}
