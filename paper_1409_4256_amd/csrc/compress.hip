// c-step, eq. (2.12): scatter of the M-step slices W'_ji and of the weights
// rho_j into numerator and denominator grids through the same trilinear
// weights as the expansion (FP64 atomics), then the division.
#include "emc_device.h"

namespace emc {

// One workgroup per rotation (one slice per block, as the paper's
// insert_slices kernel, Section 3.1).
__global__ __launch_bounds__(256) void scatter_kernel(const float* __restrict__ Wp, int64_t stride,
                                                      const double* __restrict__ rho, const float* __restrict__ q,
                                                      const uint8_t* __restrict__ mask,
                                                      const float* __restrict__ quat, int n_pix, int N,
                                                      double* __restrict__ num, double* __restrict__ den) {
  const int j = blockIdx.x;
  const Rot r = quat_rot(quat + 4 * (int64_t)j);
  const double rj = rho[j];
  const float* row = Wp + (int64_t)j * stride;
  for (int i = threadIdx.x; i < n_pix; i += 256) {
    if (!mask[i]) continue;
    const Stencil s = stencil_at(r, q + 3 * (int64_t)i, N);
    const double wv = (double)row[i];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (s.w[t] != 0.0) {
        unsafeAtomicAdd(num + s.idx[t], s.w[t] * wv);
        unsafeAtomicAdd(den + s.idx[t], s.w[t] * rj);
      }
    }
  }
}

__global__ void divide_kernel(const double* __restrict__ num, const double* __restrict__ den,
                              const float* prev, float* out, int64_t M) {
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < M; l += (int64_t)gridDim.x * 256) {
    const double d = den[l];
    out[l] = d > 0.0 ? (float)(num[l] / d) : prev[l];
  }
}

__global__ __launch_bounds__(256) void mean_kernel(const double* __restrict__ L, int64_t n, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) s += L[k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = n > 0 ? ((red[0] + red[1]) + (red[2] + red[3])) / (double)n : NAN;
}

hipError_t launch_scatter(const float* Wp, int64_t stride, const double* rho, const float* q,
                          const uint8_t* mask, const float* quat, int n_pix, int n_rot, int N, double* num,
                          double* den, hipStream_t st) {
  scatter_kernel<<<(unsigned)n_rot, 256, 0, st>>>(Wp, stride, rho, q, mask, quat, n_pix, N, num, den);
  return hipGetLastError();
}

hipError_t launch_divide(const double* num, const double* den, const float* prev, float* out, int64_t M,
                         hipStream_t st) {
  int64_t g = (M + 255) / 256;
  divide_kernel<<<(unsigned)(g > 65536 ? 65536 : g), 256, 0, st>>>(num, den, prev, out, M);
  return hipGetLastError();
}

hipError_t launch_mean(const double* L, int64_t n, double* out, hipStream_t st) {
  mean_kernel<<<1, 256, 0, st>>>(L, n, out);
  return hipGetLastError();
}

}  // namespace emc
