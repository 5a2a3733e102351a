// mhd_mathcheck.hip -- evaluates the device reciprocal and square-root
// helpers of the FP64 kernels on caller arguments, so that their accuracy
// can be measured against correctly rounded results.
#include <hip/hip_runtime.h>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {

__global__ __launch_bounds__(256) void math_check_kernel(const double *__restrict__ x,
                                                         double *__restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double a = x[i];
    out[i] = rcp<double>(a);
    out[n + i] = rcp_flux<double>(a);
    out[2 * n + i] = sqroot<double>(a);
    out[3 * n + i] = sqroot_flux<double>(a);
  }
}

hipError_t launch_math_check(hipStream_t s, const double *x, double *out, long long n) {
  long long nb = (n + 255) / 256;
  nb = nb < 4096 ? nb : 4096;
  if (nb > 0)
    hipLaunchKernelGGL(math_check_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, out, n);
  return hipGetLastError();
}

}  // namespace mhd
