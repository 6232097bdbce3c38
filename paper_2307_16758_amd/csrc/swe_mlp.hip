// Learned slope limiter kernels (filled in below).
#include <hip/hip_runtime.h>
