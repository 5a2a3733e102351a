// mhd_noalloc.hip -- the allocation-free CFL step, mhd_compute_dt_noalloc.
//
// The kernels are those of mhd_compute_dt (eq. cfl: per-block maxima of
// the signal speed, then one block that reduces them in a fixed order).
// Their scratch -- the per-block maxima, the largest speed and the error
// bits -- lives in `scratch`, a file-scope device array, instead of a
// context's buffers, so a call needs no context and allocates nothing.
// Each device holds its own copy of the array for the life of the process;
// every call on a device shares it, so calls that overlap on one device
// race.  Host code reaches the array only through the device address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "mhd_internal.h"

namespace {

// layout: [0, CFL_MAX_BLOCKS) block maxima, then the largest speed, then
// the error bits (an int in the next slot)
constexpr int kSmaxSlot = mhd::CFL_MAX_BLOCKS;
constexpr int kFlagSlot = mhd::CFL_MAX_BLOCKS + 1;
constexpr int kScratchDoubles = mhd::CFL_MAX_BLOCKS + 64;
static_assert(kScratchDoubles * sizeof(double) == MHD_NOALLOC_SCRATCH_BYTES,
              "header and library disagree on the scratch size");

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch`, resolved once per
// device with that device current, after checking that the device is a
// gfx950 (hipErrorInvalidDeviceFunction if not): later calls on the device
// only read the table
hipError_t scratch_ptr(int dev, double **out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return e;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return hipErrorInvalidDeviceFunction;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

__global__ void clear_flags_kernel(int *flags) { *flags = 0; }

// the caller's outputs: dt from the reduction, and the error bits
__global__ void export_kernel(const int *flags, int32_t *flags_out) { *flags_out = *flags; }

int fail(int code, const std::string &msg) {
  mhd::set_context_free_error(msg);
  return code;
}

}  // namespace

namespace mhd {
// resolve the scratch address of the current device ahead of the first
// call (mhd_init_grid does this, so later calls only read the table)
hipError_t noalloc_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  double *p = nullptr;
  return scratch_ptr(dev, &p);
}
}  // namespace mhd

extern "C" {

int mhd_compute_dt_noalloc(const mhd_grid_desc *desc, const double *U, const double *Bx,
                           const double *By, const double *Bz, const double *T, double cfl,
                           double *dt_out, int32_t *flags_out, void *hip_stream) {
  std::string msg;
  int rc = mhd::validate_desc(desc, msg);
  if (rc) return fail(rc, msg);
  if (desc->eos_guess != MHD_GUESS_PREV_T)
    return fail(MHD_ERR_ARG, "the allocation-free CFL step takes the previous-T guess only");
  if (!U || !Bx || !By || !Bz || !dt_out)
    return fail(MHD_ERR_ARG, "state arrays and dt_out must not be NULL");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(MHD_ERR_ARG, "cfl must be > 0");
  const size_t ncell = (size_t)desc->nx * desc->ny * desc->nz;
  const int nb = mhd::cfl_partial_blocks(ncell);
  if (nb > mhd::CFL_MAX_BLOCKS || nb < 1)
    return fail(MHD_ERR_ARG, "grid needs more reduction blocks than the scratch holds");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MHD_ERR_NO_DEVICE, "no HIP device");
  if (dev < 0 || dev >= kMaxDevices) return fail(MHD_ERR_NO_DEVICE, "device index out of range");
  double *sp = nullptr;
  hipError_t e = scratch_ptr(dev, &sp);
  if (e == hipErrorInvalidDeviceFunction) return fail(MHD_ERR_NO_DEVICE, "device is not gfx950");
  if (e != hipSuccess)
    return fail(MHD_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  mhd::Phys ph{};
  mhd::fill_phys(desc, ph);
  hipStream_t s = (hipStream_t)hip_stream;
  int *flags = reinterpret_cast<int *>(sp + kFlagSlot);
  hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(1), 0, s, flags);
  e = mhd::launch_signal_speed_raw(ph, s, false, U, Bx, By, Bz, ph.gasrad ? T : nullptr, nullptr,
                                   sp, flags, cfl, dt_out, sp + kSmaxSlot, nullptr, nullptr);
  if (e == hipSuccess && flags_out)
    hipLaunchKernelGGL(export_kernel, dim3(1), dim3(1), 0, s, flags, flags_out);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(MHD_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  return MHD_OK;
}

}  // extern "C"
