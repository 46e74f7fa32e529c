// E-step, eq. (2.4): responsibilities as an FP64 log-sum-exp over rotations of
// the log-joint a_kj = Q_jk + log w_j = G_kj + b_k - S_j + log w_j.  A frame's
// normalisation needs only its maximum and the sum of exp(a - max); these two
// statistics are also all that rotation shares must exchange (Section 3.2).
#include "emc_device.h"

namespace emc {

__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
  if (m2 > m) {
    s = s * exp(m - m2) + s2;
    m = m2;
  } else if (m2 > -INFINITY) {
    s += s2 * exp(m2 - m);
  }
}

// One wave per frame: online (max, sum exp) in FP64 over the frame's row.
__global__ __launch_bounds__(256) void lse_stats_kernel(const float* __restrict__ G, int64_t ld, int n_rot,
                                                        int64_t n_data, const double* __restrict__ log_w,
                                                        const double* __restrict__ S,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ stats) {
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n_data) return;  // uniform per wave
  const float* row = G + k * ld;
  const double bk = b[k];
  double m = -INFINITY, s = 0.0;
  for (int j = lane; j < n_rot; j += 64) {
    const double a = ((double)row[j] + bk) + (log_w[j] - S[j]);
    if (!(a > -INFINITY)) continue;  // zero prior weight: no contribution
    if (a > m) {
      s = s * exp(m - a) + 1.0;
      m = a;
    } else {
      s += exp(a - m);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double m2 = __shfl_xor(m, o, 64), s2 = __shfl_xor(s, o, 64);
    lse_merge(m, s, m2, s2);
  }
  if (lane == 0) {
    stats[2 * k] = m;
    stats[2 * k + 1] = s;
  }
}

constexpr int kRowsPerBlock = 256;

// Workgroup = 256 consecutive rotations x 256 frames: coalesced row segments,
// P written in place of G when they alias, rho_j accumulated per block in FP64
// and added with one atomic per (block, rotation).  The first column of blocks
// also writes the log-evidence L_k = m_k + log s_k.
__global__ __launch_bounds__(256) void lse_write_kernel(const float* G, float* P, int64_t ld, int n_rot,
                                                        int64_t n_data, const double* __restrict__ log_w,
                                                        const double* __restrict__ S,
                                                        const double* __restrict__ stats,
                                                        const double* __restrict__ b, double* __restrict__ L,
                                                        double* __restrict__ rho) {
  __shared__ double shift[kRowsPerBlock];  // b_k - L_k
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.y * kRowsPerBlock;
  const int64_t k1 = (k0 + kRowsPerBlock) < n_data ? (k0 + kRowsPerBlock) : n_data;
  {
    const int64_t k = k0 + threadIdx.x;
    if (k < k1) {
      const double v = stats[2 * k] + log(stats[2 * k + 1]);
      shift[threadIdx.x] = b[k] - v;
      if (blockIdx.x == 0) L[k] = v;
    }
  }
  __syncthreads();
  if (j >= ld) return;
  if (j >= n_rot) {
    for (int64_t k = k0; k < k1; ++k) P[k * ld + j] = 0.0f;
    return;
  }
  const double ej = log_w[j] - S[j];
  double acc = 0.0;
  for (int64_t k = k0; k < k1; ++k) {
    const float p = (float)exp(((double)G[k * ld + j] + shift[k - k0]) + ej);
    P[k * ld + j] = p;
    acc += (double)p;
  }
  atomicAdd(rho + j, acc);
}

hipError_t launch_lse_stats(const float* G, int64_t ld, int n_rot, int64_t n_data, const double* log_w,
                            const double* S, const double* b, double* stats, hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  lse_stats_kernel<<<(unsigned)((n_data + 3) / 4), 256, 0, st>>>(G, ld, n_rot, n_data, log_w, S, b, stats);
  return hipGetLastError();
}

hipError_t launch_lse_write(const float* G, float* P, int64_t ld, int n_rot, int64_t n_data,
                            const double* log_w, const double* S, const double* stats, const double* b,
                            double* L, double* rho, hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  dim3 grid((unsigned)((ld + 255) / 256), (unsigned)((n_data + kRowsPerBlock - 1) / kRowsPerBlock));
  lse_write_kernel<<<grid, 256, 0, st>>>(G, P, ld, n_rot, n_data, log_w, S, stats, b, L, rho);
  return hipGetLastError();
}

}  // namespace emc
