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
    acc += log(fmax(trilinear_at(model, N, r, q + 3 * i), kFloor));
  }
  c[i] = acc / nc;
}

__device__ __forceinline__ double slice_value(const float* __restrict__ model, int N, const Rot& r,
                                              const float* __restrict__ qi) {
  return fmax(trilinear_at(model, N, r, qi), kFloor);
}

__device__ __forceinline__ double block_sum4(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
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
      const double W = slice_value(model, N, r, q + 3 * i);
      sum += W;
      out = (float)(log(W) - c[i]);
    }
    row[i] = out;
  }
  sum = block_sum4(sum, red);
  if (threadIdx.x == 0) S[j] = sum;
}

// BF16 form: the centred log slice A_ji = log W_ij - c_i is written as two BF16
// terms with a per-rotation scale, A_ji ~ scale_j (hi_ji + lo_ji), where
// scale_j = max_i |A_ji|, hi = bf16(A / scale), lo = bf16(A / scale - hi).
// A first pass finds the row maximum; the second writes hi and lo.
// STASH: detectors of at most kStashPx pixels keep the first pass's values
// a_i = log W_ji - c_i (FP32) in LDS, so the interpolation and the FP64 log run
// once per pixel; larger ones recompute them in the second pass.  Both give the
// same bits.
constexpr int kStashPx = 16384;  // 64 KB of LDS
// 8 waves per workgroup: the stash allows two workgroups per CU, and the
// gathers need many waves in flight to cover their latency (two workgroups of 8
// waves fit the registers: 4 waves per SIMD).
constexpr int kExpThreads = 512;
constexpr int kExpWaves = kExpThreads / 64;

template <bool STASH>
__global__ __launch_bounds__(kExpThreads) void expand_bf16_kernel(const float* __restrict__ model, int N,
                                                                  const float* __restrict__ q,
                                                                  const uint8_t* __restrict__ mask,
                                                                  const float* __restrict__ quat, int n_pix,
                                                                  int64_t stride, int64_t plane,
                                                                  const double* __restrict__ c,
                                                                  __hip_bfloat16* __restrict__ hi_all,
                                                                  double* __restrict__ S, float* __restrict__ scale) {
  __shared__ double red[kExpWaves];
  __shared__ float redf[kExpWaves];
  __shared__ float stash[STASH ? kStashPx : 1];
  const int j = blockIdx.x;
  const Rot r = quat_rot(quat + 4 * (int64_t)j);
  double sum = 0.0;
  float amax = 0.0f;
  for (int64_t i = threadIdx.x; i < n_pix; i += kExpThreads) {
    if (!mask[i]) continue;
    const double W = slice_value(model, N, r, q + 3 * i);
    sum += W;
    const float a = (float)(log(W) - c[i]);
    if constexpr (STASH) stash[i] = a;
    amax = fmaxf(amax, fabsf(a));
  }
  sum = wave_sum(sum);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = sum;
    redf[threadIdx.x >> 6] = amax;
  }
  __syncthreads();  // also orders the stash writes before the reads below
  amax = redf[0];
#pragma unroll
  for (int w = 1; w < kExpWaves; ++w) amax = fmaxf(amax, redf[w]);
  const float sc = amax > 0.0f ? amax : 1.0f;
  const float inv = 1.0f / sc;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kExpWaves; ++w) t += red[w];
    S[j] = t;
    scale[j] = sc;
  }
  __hip_bfloat16* hi = hi_all + (int64_t)j * stride;
  __hip_bfloat16* lo = hi_all + plane + (int64_t)j * stride;
  for (int64_t i = threadIdx.x; i < stride; i += kExpThreads) {
    float h = 0.0f, l = 0.0f;
    if (i < n_pix && mask[i]) {
      float v;
      if constexpr (STASH)
        v = stash[i];
      else
        v = (float)(log(slice_value(model, N, r, q + 3 * i)) - c[i]);
      const float a = v * inv;
      const __hip_bfloat16 hb = __float2bfloat16(a);
      h = __bfloat162float(hb);
      l = a - h;
    }
    hi[i] = __float2bfloat16(h);
    lo[i] = __float2bfloat16(l);
  }
}

// b_k = sum_i K_ik c_i in FP64: one wave per frame.
__device__ __forceinline__ double as_double(float v) { return (double)v; }
__device__ __forceinline__ double as_double(__hip_bfloat16 v) { return (double)__bfloat162float(v); }

template <typename T>
__global__ __launch_bounds__(256) void frame_dot_kernel(const T* __restrict__ K, int64_t stride, int64_t n_data,
                                                        const double* __restrict__ c, double* __restrict__ b) {
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n_data) return;  // uniform per wave
  const T* row = K + k * stride;
  double acc = 0.0;
  for (int64_t i = 4 * lane; i < stride; i += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += as_double(row[i + u]) * c[i + u];
  }
  acc = wave_sum(acc);
  if (lane == 0) b[k] = acc;
}

__global__ void fill_zero_f64_kernel(double* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0.0;
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

hipError_t launch_expand_bf16(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                              int n_pix, int64_t stride, int n_rot, const double* c, void* hilo, double* S,
                              float* scale, hipStream_t st) {
  if (n_pix <= kStashPx)
    expand_bf16_kernel<true><<<(unsigned)n_rot, kExpThreads, 0, st>>>(model, N, q, mask, quat, n_pix, stride,
                                                            (int64_t)n_rot * stride, c, (__hip_bfloat16*)hilo, S,
                                                            scale);
  else
    expand_bf16_kernel<false><<<(unsigned)n_rot, kExpThreads, 0, st>>>(model, N, q, mask, quat, n_pix, stride,
                                                             (int64_t)n_rot * stride, c, (__hip_bfloat16*)hilo, S,
                                                             scale);
  return hipGetLastError();
}

hipError_t launch_frame_dot(const void* K, bool bf16, int64_t stride, int64_t n_data, const double* c, double* b,
                            hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  if (bf16)
    frame_dot_kernel<__hip_bfloat16><<<(unsigned)((n_data + 3) / 4), 256, 0, st>>>((const __hip_bfloat16*)K, stride,
                                                                                  n_data, c, b);
  else
    frame_dot_kernel<float><<<(unsigned)((n_data + 3) / 4), 256, 0, st>>>((const float*)K, stride, n_data, c, b);
  return hipGetLastError();
}

}  // namespace emc
