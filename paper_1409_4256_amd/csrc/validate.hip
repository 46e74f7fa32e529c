// Contents check of a problem's arrays (the entry points check sizes and pointers
// on the host and never read array contents): unit quaternions, finite pixel
// coordinates and log prior weights, a finite non-negative model.  One pass over
// the arrays ORs a bit per failed check into a device word.
#include "emc_device.h"

namespace emc {

__global__ void validate_kernel(const float* __restrict__ quat, int64_t n_rot, const float* __restrict__ q,
                                const uint8_t* __restrict__ mask, int64_t n_pix, const double* __restrict__ log_w,
                                const float* __restrict__ model, int64_t n_grid, double tol, int32_t* __restrict__ flags) {
  int32_t bits = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_rot; t += stride) {
    const double w = quat[4 * t], x = quat[4 * t + 1], y = quat[4 * t + 2], z = quat[4 * t + 3];
    const double n = sqrt(w * w + x * x + y * y + z * z);
    if (!(fabs(1.0 - n) <= tol)) bits |= kValidQuat;  // NaN fails too
    if (!isfinite(log_w[t])) bits |= kValidWeight;
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_pix; t += stride)
    if (mask[t] && !(isfinite(q[3 * t]) && isfinite(q[3 * t + 1]) && isfinite(q[3 * t + 2]))) bits |= kValidPixel;
  if (model)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_grid; t += stride)
      if (!(model[t] >= 0.0f && model[t] < INFINITY)) bits |= kValidModel;
  if (bits) atomicOr(flags, bits);
}

__global__ void zero_flag_kernel(int32_t* flags) { *flags = 0; }

hipError_t launch_validate(const float* quat, int64_t n_rot, const float* q, const uint8_t* mask, int64_t n_pix,
                           const double* log_w, const float* model, int64_t n_grid, double tol, int32_t* flags,
                           hipStream_t st) {
  zero_flag_kernel<<<1, 1, 0, st>>>(flags);
  int64_t n = n_rot > n_pix ? n_rot : n_pix;
  if (model && n_grid > n) n = n_grid;
  const int64_t blocks = (n + 255) / 256;
  validate_kernel<<<(unsigned)(blocks > 4096 ? 4096 : blocks), 256, 0, st>>>(quat, n_rot, q, mask, n_pix, log_w,
                                                                            model, n_grid, tol, flags);
  return hipGetLastError();
}

}  // namespace emc
