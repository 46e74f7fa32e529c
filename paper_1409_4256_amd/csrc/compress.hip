// c-step, eq. (2.12): scatter of the M-step slices W'_ji and of the weights
// rho_j into numerator and denominator grids through the same trilinear
// weights as the expansion (FP64 atomics), then the division.
//
// With a workspace, every XCD accumulates into a grid copy of its own (the wave
// reads the id of the XCD it runs on), with atomics that complete in that XCD's
// L2; a reduction then adds the eight copies.  Without one, the atomics go to the
// shared grids at device scope (past the L2s).
#include <limits.h>

#include "emc_device.h"

namespace emc {

constexpr int kBoxCap = 1024;  // voxels of one wave's LDS accumulation box
constexpr int kCopies = 8;     // grid copies: one per XCD

template <bool LOCAL>
__device__ __forceinline__ void grid_add(double* p, double v) {
  if constexpr (LOCAL)
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);  // in this XCD's L2
  else
    unsafeAtomicAdd(p, v);
}

__device__ __forceinline__ int xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kCopies - 1); }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One workgroup per rotation j (one slice per block, like the paper's
// insert_slices kernel, Section 3.1).  Each wave takes 64 consecutive pixels;
// when they are spatially compact on the detector (an 8 x 8 tile) their 512
// trilinear contributions land in a small box of voxels, which the wave
// accumulates in LDS (FP64) and then adds to the global grids with one FP64
// atomic per touched voxel.  Pixel groups whose box exceeds kBoxCap voxels
// add straight to the global grids; the result is the same either way.
template <bool LOCAL>
__global__ __launch_bounds__(256) void scatter_kernel(const float* __restrict__ Wp, int64_t stride,
                                                      const double* __restrict__ rho, const float* __restrict__ q,
                                                      const uint8_t* __restrict__ mask,
                                                      const float* __restrict__ quat, int n_pix, int N,
                                                      double* __restrict__ num, double* __restrict__ den,
                                                      int64_t M) {
  if constexpr (LOCAL) {  // this XCD's copies of the two grids
    const int64_t x = xcd_id();
    num += x * M;
    den += x * M;
  }
  __shared__ double s_num[4][kBoxCap];
  __shared__ double s_den[4][kBoxCap];
  const int j = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const Rot r = quat_rot(quat + 4 * (int64_t)j);
  const double rj = rho[j];
  const float* row = Wp + (int64_t)j * stride;
  double* bn = s_num[wave];
  double* bd = s_den[wave];
  const int n_groups = (n_pix + 63) / 64;
  const int iters = (n_groups + 3) / 4;
  for (int it = 0; it < iters; ++it) {
    const int i = (it * 4 + wave) * 64 + lane;
    const bool valid = i < n_pix && mask[i];
    Stencil s;
    double wv = 0.0;
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
    if (valid) {
      s = stencil_at(r, q + 3 * (int64_t)i, N);
      wv = (double)row[i];
      lo[0] = hi[0] = s.bx;
      lo[1] = hi[1] = s.by;
      lo[2] = hi[2] = s.bz;
    }
    const int x0 = wave_min(lo[0]), y0 = wave_min(lo[1]), z0 = wave_min(lo[2]);
    const int x1 = wave_max(hi[0]), y1 = wave_max(hi[1]), z1 = wave_max(hi[2]);
    const bool any = x1 >= x0;  // at least one valid lane
    const int DY = any ? y1 - y0 + 2 : 0, DZ = any ? z1 - z0 + 2 : 0;
    const int64_t vol = any ? (int64_t)(x1 - x0 + 2) * DY * DZ : 0;
    const bool boxed = any && vol <= kBoxCap;
    if (boxed)
      for (int e = lane; e < vol; e += 64) {
        bn[e] = 0.0;
        bd[e] = 0.0;
      }
    __syncthreads();
    if (valid) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (s.w[t] == 0.0) continue;  // outside the grid, or exactly on the far face
        const double an = s.w[t] * wv, ad = s.w[t] * rj;
        if (boxed) {
          const int e = ((s.bx + (t >> 2) - x0) * DY + (s.by + ((t >> 1) & 1) - y0)) * DZ + (s.bz + (t & 1) - z0);
          atomicAdd(bn + e, an);
          atomicAdd(bd + e, ad);
        } else {
          grid_add<LOCAL>(num + s.idx[t], an);
          grid_add<LOCAL>(den + s.idx[t], ad);
        }
      }
    }
    __syncthreads();
    if (boxed)
      for (int e = lane; e < vol; e += 64) {
        const double vn = bn[e], vd = bd[e];
        if (vn == 0.0 && vd == 0.0) continue;
        const int ex = e / (DY * DZ), rem = e - ex * DY * DZ, ey = rem / DZ, ez = rem - ey * DZ;
        const int l = ((x0 + ex) * N + (y0 + ey)) * N + (z0 + ez);
        if (vn != 0.0) grid_add<LOCAL>(num + l, vn);
        if (vd != 0.0) grid_add<LOCAL>(den + l, vd);
      }
    // the next iteration's zeroing touches entry e from the same lane that flushed it
  }
}

// num_l += sum_x cn[x][l], den_l += sum_x cd[x][l] (copies in a fixed order)
__global__ void grid_reduce_kernel(const double* __restrict__ cn, const double* __restrict__ cd, int64_t M,
                                   double* __restrict__ num, double* __restrict__ den) {
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < M; l += (int64_t)gridDim.x * 256) {
    double sn = 0.0, sd = 0.0;
#pragma unroll
    for (int x = 0; x < kCopies; ++x) {
      sn += cn[x * M + l];
      sd += cd[x * M + l];
    }
    num[l] += sn;
    den[l] += sd;
  }
}

__global__ void zero_f64_kernel(double* __restrict__ p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = 0.0;
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

// num/den += the scatter of all rotations; copies: NULL or 2 * 8 * N^3 doubles
hipError_t launch_scatter(const float* Wp, int64_t stride, const double* rho, const float* q,
                          const uint8_t* mask, const float* quat, int n_pix, int n_rot, int N, double* num,
                          double* den, double* copies, hipStream_t st) {
  const int64_t M = (int64_t)N * N * N;
  if (!copies) {
    scatter_kernel<false><<<(unsigned)n_rot, 256, 0, st>>>(Wp, stride, rho, q, mask, quat, n_pix, N, num, den, M);
    return hipGetLastError();
  }
  const int64_t nc = 2 * kCopies * M;
  const int64_t gz = (nc + 255) / 256, gr = (M + 255) / 256;
  zero_f64_kernel<<<(unsigned)(gz > 65536 ? 65536 : gz), 256, 0, st>>>(copies, nc);
  scatter_kernel<true><<<(unsigned)n_rot, 256, 0, st>>>(Wp, stride, rho, q, mask, quat, n_pix, N, copies,
                                                        copies + kCopies * M, M);
  grid_reduce_kernel<<<(unsigned)(gr > 65536 ? 65536 : gr), 256, 0, st>>>(copies, copies + kCopies * M, M, num, den);
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
