// Frame packing (once per frame set, not part of the iteration): photon counts
// -> GEMM operands in two layouts, frame-major K[k][i] for the log-likelihood
// contraction and pixel-major KT[i][k] for the M-step contraction, so that both
// contractions read their operands along the reduction index.  Masked and
// padding pixels and padding frames are zero.  Counts are exact in FP32, and
// in BF16 up to 256 (8 significant bits); larger counts raise a range flag.
#include "emc_device.h"

namespace emc {

__device__ int g_range_flag;

__global__ void clear_flag_kernel() { g_range_flag = 0; }

template <typename T>
__device__ __forceinline__ T from_count(unsigned c);
template <>
__device__ __forceinline__ float from_count<float>(unsigned c) {
  return (float)c;
}
template <>
__device__ __forceinline__ __hip_bfloat16 from_count<__hip_bfloat16>(unsigned c) {
  return __float2bfloat16((float)c);
}

// 64 x 64 tiles (frames x pixels) transposed through LDS.
template <typename T, bool BF16>
__global__ __launch_bounds__(256) void pack_kernel(const uint16_t* __restrict__ counts,
                                                   const uint8_t* __restrict__ mask, int n_pix, int64_t ps,
                                                   int64_t n_data, int64_t ds, const int32_t* __restrict__ frames,
                                                   T* __restrict__ K, T* __restrict__ KT) {
  __shared__ unsigned tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64, k0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  bool over = false;
  for (int r = ty; r < 64; r += 4) {  // r: frame within tile, tx: pixel within tile
    const int64_t k = k0 + r, i = i0 + tx;
    unsigned c = 0;
    if (k < n_data && i < n_pix && mask[i]) {
      const int64_t src = frames ? (int64_t)frames[k] : k;
      c = counts[src * n_pix + i];
      if (BF16 && c > 256u) over = true;
    }
    tile[r][tx] = c;
    if (k < n_data) K[k * ps + i] = from_count<T>(c);
  }
  if (BF16 && over) atomicOr(&g_range_flag, 1);
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {  // r: pixel within tile, tx: frame within tile
    const int64_t i = i0 + r, k = k0 + tx;
    KT[i * ds + k] = from_count<T>(tile[tx][r]);
  }
}

hipError_t launch_pack(const uint16_t* counts, const uint8_t* mask, int n_pix, int64_t ps, int64_t n_data,
                       int64_t ds, const int32_t* frames, void* K, void* KT, bool bf16, hipStream_t st) {
  dim3 grid((unsigned)(ps / 64), (unsigned)(ds / 64));
  if (bf16) {
    clear_flag_kernel<<<1, 1, 0, st>>>();
    pack_kernel<__hip_bfloat16, true><<<grid, 256, 0, st>>>(counts, mask, n_pix, ps, n_data, ds, frames,
                                                            (__hip_bfloat16*)K, (__hip_bfloat16*)KT);
  } else {
    pack_kernel<float, false><<<grid, 256, 0, st>>>(counts, mask, n_pix, ps, n_data, ds, frames, (float*)K,
                                                    (float*)KT);
  }
  return hipGetLastError();
}

hipError_t read_range_flag(int* flag, hipStream_t st) {
  hipError_t e = hipMemcpyFromSymbolAsync(flag, HIP_SYMBOL(g_range_flag), sizeof(int), 0, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace emc
