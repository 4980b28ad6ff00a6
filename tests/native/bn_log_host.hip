// Host builds of the kernels' logarithm and division by a launch constant
// for their accuracy tests: the same source, evaluated operation by
// operation as on the device.
#include "bn_math.h"

extern "C" void bn_log_host(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = bn::bn_log(x[i]);
}

extern "C" void bn_div_by_host(const double *x, double d, double *y, long n) {
  const double inv_d = 1.0 / d;
  for (long i = 0; i < n; ++i) y[i] = bn::bn_div_by(x[i], d, inv_d);
}
