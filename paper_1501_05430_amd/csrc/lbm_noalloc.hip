// lbm_measure_contact_angle_noalloc: the contact-angle measurement of lbm_measure_contact_angle on a density field
// the caller holds, for callers that cannot allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc). Its reduction partials live in a file-scope device array instead of a context's
// workspace; everything else (the min/max and moment kernels, the fixed-order folds, the circle fit) is the
// measurement lbm_measure_contact_angle runs.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/lbm.h"
#include "lbm_internal.h"

namespace {

// Reduction partials of one measurement: 512 blocks x 10 moments (the min/max pass uses the first 2 x 512). One copy
// per GPU, held until the process ends; the measurement's grid is fixed, so this covers any field size.
constexpr int kScratchDoubles = lbm::kMeasurePartials;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices];  // device address of `scratch` on each device (hipGetSymbolAddress)

// The current device's copy of `scratch`, looked up once per device with that device current. Host code uses only
// this address: the array's name on the host side is not a device address.
int scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    char msg[256];
    snprintf(msg, sizeof msg, "hipGetDevice: %s", hipGetErrorString(e));
    return lbm::report_error(LBM_E_HIP, msg);
  }
  if (dev < 0 || dev >= kMaxDevices) return lbm::report_error(LBM_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char msg[256];
      snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return lbm::report_error(LBM_E_HIP, msg);
    }
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_measure_contact_angle_noalloc(const double* d_rho, int32_t nx, int32_t ny, int32_t wall,
                                                 const int32_t box[4], void* hip_stream, double out[5]) {
  if (!d_rho || !box || !out) return lbm::report_error(LBM_E_INVALID, "d_rho/box/out NULL");
  if (nx < 2 || ny < 4) return lbm::report_error(LBM_E_INVALID, "need nx >= 2 and ny >= 4");
  if ((int64_t)nx * ny > ((int64_t)1 << 34)) return lbm::report_error(LBM_E_INVALID, "field too large");
  if (wall != 0 && wall != 1) return lbm::report_error(LBM_E_INVALID, "wall must be 0 or 1");
  const int32_t b[4] = {box[0] > 0 ? box[0] : 0, box[1] < nx ? box[1] : nx, box[2] > 1 ? box[2] : 1,
                        box[3] < ny - 1 ? box[3] : ny - 1};
  if (b[1] - b[0] < 2 || b[3] - b[2] < 2) return lbm::report_error(LBM_E_INVALID, "box too small after clipping");
  double* partials = nullptr;
  const int rc = scratch_on_current_device(&partials);
  if (rc != LBM_OK) return rc;
  return lbm::measure_contact_angle_field(d_rho, nx, ny, wall, b, partials, (hipStream_t)hip_stream, out);
}
