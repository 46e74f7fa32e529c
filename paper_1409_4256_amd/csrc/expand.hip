// Expansion (e-step, eq. (2.9)): trilinear gather of rotated detector slices
// from the model grid, with the Poisson floor, the log and the per-rotation sum.
#include "emc_device.h"

namespace emc {

// One thread per pixel.  c_i = mean over a fixed subset of rotations of log W_ij.
__global__ __launch_bounds__(256) void centre_kernel(const float* __restrict__ model, int N,
                                                     const float* __restrict__ q,
                                                     const uint8_t* __restrict__ mask,
                                                     const float* __restrict__ quat, int n_pix,
                                                     int64_t stride, int n_rot, double* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= stride) return;
  if (i >= n_pix || !mask[i]) {
    c[i] = 0.0;
    return;
  }
  const int nc = n_rot < 64 ? n_rot : 64;
  double acc = 0.0;
  for (int t = 0; t < nc; ++t) {
    const int j = (int)(((int64_t)t * n_rot) / nc);
    const Rot r = quat_rot(quat + 4 * (int64_t)j);
    const Stencil s = stencil_at(r, q + 3 * i, N);
    double W = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) W += s.w[k] * (double)model[s.idx[k]];
    acc += log(fmax(W, kFloor));
  }
  c[i] = acc / nc;
}

// One workgroup per rotation j (the paper's one-block-per-slice mapping of the
// expansion kernel, Section 3.1): threads stride over pixels; S_j is reduced
// in the block in FP64, so no atomics and a deterministic order.
__global__ __launch_bounds__(256) void expand_kernel(const float* __restrict__ model, int N,
                                                     const float* __restrict__ q,
                                                     const uint8_t* __restrict__ mask,
                                                     const float* __restrict__ quat, int n_pix,
                                                     int64_t stride, const double* __restrict__ c,
                                                     float* __restrict__ logW, double* __restrict__ S) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const Rot r = quat_rot(quat + 4 * (int64_t)j);
  float* row = logW + (int64_t)j * stride;
  double sum = 0.0;
  for (int64_t i = threadIdx.x; i < stride; i += 256) {
    float out = 0.0f;
    if (i < n_pix && mask[i]) {
      const Stencil s = stencil_at(r, q + 3 * i, N);
      double W = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) W += s.w[k] * (double)model[s.idx[k]];
      W = fmax(W, kFloor);
      sum += W;
      out = (float)(log(W) - c[i]);
    }
    row[i] = out;
  }
  sum = wave_sum(sum);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) S[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// b_k = sum_i K_ik c_i in FP64: one wave per frame.
__global__ __launch_bounds__(256) void frame_dot_kernel(const float* __restrict__ K, int64_t stride,
                                                        int64_t n_data, const double* __restrict__ c,
                                                        double* __restrict__ b) {
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n_data) return;  // uniform per wave
  const float* row = K + k * stride;
  double acc = 0.0;
  for (int64_t i = 4 * lane; i < stride; i += 256) {
    const float4 v = *reinterpret_cast<const float4*>(row + i);
    acc += (double)v.x * c[i] + (double)v.y * c[i + 1] + (double)v.z * c[i + 2] + (double)v.w * c[i + 3];
  }
  acc = wave_sum(acc);
  if (lane == 0) b[k] = acc;
}

__global__ void fill_zero_f64_kernel(double* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0.0;
}

__global__ void pack_f32_kernel(const uint16_t* __restrict__ counts, const uint8_t* __restrict__ mask,
                                int n_pix, int64_t stride, int64_t n_data, float* __restrict__ K) {
  const size_t total = (size_t)n_data * stride;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int64_t k = e / stride, i = e - k * stride;
    float v = 0.0f;
    if (i < n_pix && mask[i]) v = (float)counts[k * n_pix + i];
    K[e] = v;
  }
}

static inline unsigned grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g > 65536 ? 65536 : (g == 0 ? 1 : g));
}

hipError_t launch_fill_zero_f64(double* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  fill_zero_f64_kernel<<<grid_for(n), 256, 0, st>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_pack_f32(const uint16_t* counts, const uint8_t* mask, int n_pix, int64_t stride,
                           int64_t n_data, float* K, hipStream_t st) {
  const size_t n = (size_t)n_data * stride;
  if (n == 0) return hipSuccess;
  pack_f32_kernel<<<grid_for(n), 256, 0, st>>>(counts, mask, n_pix, stride, n_data, K);
  return hipGetLastError();
}

hipError_t launch_centre(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                         int n_pix, int64_t stride, int n_rot, double* c, hipStream_t st) {
  centre_kernel<<<(unsigned)((stride + 255) / 256), 256, 0, st>>>(model, N, q, mask, quat, n_pix, stride,
                                                                  n_rot, c);
  return hipGetLastError();
}

hipError_t launch_expand(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                         int n_pix, int64_t stride, int n_rot, const double* c, float* logW, double* S,
                         hipStream_t st) {
  expand_kernel<<<(unsigned)n_rot, 256, 0, st>>>(model, N, q, mask, quat, n_pix, stride, c, logW, S);
  return hipGetLastError();
}

hipError_t launch_frame_dot(const float* K, int64_t stride, int64_t n_data, const double* c, double* b,
                            hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  frame_dot_kernel<<<(unsigned)((n_data + 3) / 4), 256, 0, st>>>(K, stride, n_data, c, b);
  return hipGetLastError();
}

}  // namespace emc
