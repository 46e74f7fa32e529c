// E-step, eq. (2.4): responsibilities as an FP64 log-sum-exp over rotations of
// the log-joint a_jk = Q_jk + log w_j = G_jk + b_k - S_j + log w_j, on the
// rotation-major layout G[j][k] (frames contiguous).  A frame's normalisation
// needs only its maximum and the sum of exp(a - max); these two statistics are
// also all that rotation shares must exchange (Section 3.2).
//
// The statistics pass does not evaluate terms more than kLseDrop below the
// running maximum: each is below e^-64 = 1.6e-28 of the maximum term, so all of
// them together (25000 rotations: < 4e-24) stay far below the FP64 rounding of a
// sum that is at least 1.  Once the posteriors have concentrated, most terms fall
// there and the pass is bound by reading G instead of by FP64 exp.  The write pass
// keeps every responsibility, however small (the c-step's ratio is scale-free: a
// voxel reached only by improbable rotations still takes their weighted mean); it
// forms a - L_k in FP64 and evaluates the exponential in FP32, the precision P is
// stored in (or finer), skipping only exponents below -110, whose FP32 value is 0.
// (A first pass for each frame's maximum, so that whole waves could skip, was
// measured slower: in the early iterations most terms are near their frame's
// maximum and the extra read of G costs more than it saves.)
#include "emc_device.h"

namespace emc {

constexpr double kLseDrop = 64.0;

__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
  if (m2 > m) {
    s = s * exp(m - m2) + s2;
    m = m2;
  } else if (m2 > -INFINITY) {
    s += s2 * exp(m2 - m);
  }
}

constexpr int kStatFrames = 64;  // frames per workgroup: one per lane, 4 waves split the rotations

// Per-frame (max, sum exp) of a_jk over rotations [j_begin, j_end), FP64, online;
// blockIdx.y picks the rotation chunk when the rotations are split (out: the
// chunk's partials at out + 2 * n_data * blockIdx.y).
__global__ __launch_bounds__(256) void lse_stats_kernel(const float* __restrict__ G, int64_t ld, int n_rot,
                                                        int64_t n_data, const double* __restrict__ log_w,
                                                        const double* __restrict__ S,
                                                        const double* __restrict__ b, int per_chunk,
                                                        double* __restrict__ out) {
  __shared__ double sm[4][kStatFrames], ss[4][kStatFrames];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * kStatFrames + lane;
  const bool live = k < n_data;
  const int jb = blockIdx.y * per_chunk;
  const int je = jb + per_chunk < n_rot ? jb + per_chunk : n_rot;
  const double bk = live ? b[k] : 0.0;
  double m = -INFINITY, s = 0.0;
  if (live) {
    // four rotations per step so that four loads are in flight
    for (int j0 = jb + wave; j0 < je; j0 += 16) {
      float g[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + 4 * u;
        g[u] = j < je ? G[(int64_t)j * ld + k] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + 4 * u;
        if (j >= je) break;
        const double a = ((double)g[u] + bk) + (log_w[j] - S[j]);
        if (!(a > m - kLseDrop)) continue;  // zero prior weight, or negligible against the maximum
        if (a > m) {
          s = s * exp(m - a) + 1.0;
          m = a;
        } else {
          s += exp(a - m);
        }
      }
    }
  }
  sm[wave][lane] = m;
  ss[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && live) {
    for (int w = 1; w < 4; ++w) lse_merge(m, s, sm[w][lane], ss[w][lane]);
    double* o = out + 2 * n_data * blockIdx.y;
    o[2 * k] = m;
    o[2 * k + 1] = s;
  }
}

// stats_k = the chunks' partials of frame k merged in chunk order (deterministic)
__global__ void lse_chunks_kernel(const double* __restrict__ part, int n_chunks, int64_t n_data,
                                  double* __restrict__ stats) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n_data) return;
  double m = part[2 * k], s = part[2 * k + 1];
  for (int c = 1; c < n_chunks; ++c) lse_merge(m, s, part[2 * n_data * c + 2 * k], part[2 * n_data * c + 2 * k + 1]);
  stats[2 * k] = m;
  stats[2 * k + 1] = s;
}

// L_k = m_k + log s_k.
__global__ void lse_finish_kernel(const double* __restrict__ stats, int64_t n_data, double* __restrict__ L) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n_data) L[k] = stats[2 * k] + log(stats[2 * k + 1]);
}

constexpr int kWriteRows = 8;  // rotations per workgroup of the write pass

template <typename PT>
__device__ __forceinline__ PT to_p(float v);
template <>
__device__ __forceinline__ float to_p<float>(float v) {
  return v;
}
template <>
__device__ __forceinline__ __hip_bfloat16 to_p<__hip_bfloat16>(float v) {
  return __float2bfloat16(v);
}
__device__ __forceinline__ double from_p(float v) { return (double)v; }
__device__ __forceinline__ double from_p(__hip_bfloat16 v) { return (double)__bfloat162float(v); }

// P[j][k] = exp(G[j][k] + (log w_j - S_j) + (b_k - L_k)), written as PT (FP32 or
// BF16) with zeros in the padding frames; rho_j = sum_k of the stored values,
// reduced in the block (deterministic).  P may alias G when PT is float.
template <typename PT>
__global__ __launch_bounds__(256) void lse_write_kernel(const float* G, int64_t ldg, PT* P, int64_t ldp,
                                                        int n_rot, int64_t n_data, const double* __restrict__ log_w,
                                                        const double* __restrict__ S,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ L, double* __restrict__ rho) {
  __shared__ double red[kWriteRows][4];
  const int j0 = blockIdx.x * kWriteRows;
  double e[kWriteRows], acc[kWriteRows];
#pragma unroll
  for (int r = 0; r < kWriteRows; ++r) {
    const int j = j0 + r;
    e[r] = j < n_rot ? log_w[j] - S[j] : 0.0;
    acc[r] = 0.0;
  }
  for (int64_t k = threadIdx.x; k < ldp; k += 256) {
    const bool live = k < n_data;
    const double sh = live ? b[k] - L[k] : 0.0;
#pragma unroll
    for (int r = 0; r < kWriteRows; ++r) {
      const int j = j0 + r;
      if (j >= n_rot) break;
      PT p = to_p<PT>(0.0f);
      if (live) {
        const float x = (float)(((double)G[(int64_t)j * ldg + k] + sh) + e[r]);  // a - L_k
        if (x > -110.0f) {  // below, exp(x) rounds to 0 in FP32: skipping changes nothing
          p = to_p<PT>(expf(x));
          acc[r] += from_p(p);
        }
      }
      P[(int64_t)j * ldp + k] = p;
    }
  }
#pragma unroll
  for (int r = 0; r < kWriteRows; ++r) {
    const double v = wave_sum(acc[r]);
    if ((threadIdx.x & 63) == 0) red[r][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < kWriteRows) {
    const int j = j0 + threadIdx.x;
    if (j < n_rot) rho[j] = (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
  }
}

int lse_chunks(int n_rot, int64_t n_data) {
  // few frames: split the rotations so that the grid has ~2048 workgroups, each
  // chunk at least 256 rotations
  const int64_t fblocks = (n_data + kStatFrames - 1) / kStatFrames;
  int64_t c = (2048 + fblocks - 1) / fblocks;
  c = c < n_rot / 256 ? c : n_rot / 256;
  c = c < kMaxLseChunks ? c : kMaxLseChunks;
  return c > 1 ? (int)c : 1;
}

hipError_t launch_lse_stats(const float* G, int64_t ld, int n_rot, int64_t n_data, const double* log_w,
                            const double* S, const double* b, double* stats, double* part, hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  const int nc = part ? lse_chunks(n_rot, n_data) : 1;
  const int per = (n_rot + nc - 1) / nc;
  const dim3 grid((unsigned)((n_data + kStatFrames - 1) / kStatFrames), (unsigned)nc);
  lse_stats_kernel<<<grid, 256, 0, st>>>(G, ld, n_rot, n_data, log_w, S, b, per, nc > 1 ? part : stats);
  if (nc > 1) lse_chunks_kernel<<<(unsigned)((n_data + 255) / 256), 256, 0, st>>>(part, nc, n_data, stats);
  return hipGetLastError();
}

hipError_t launch_lse_finish(const double* stats, int64_t n_data, double* L, hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  lse_finish_kernel<<<(unsigned)((n_data + 255) / 256), 256, 0, st>>>(stats, n_data, L);
  return hipGetLastError();
}

hipError_t launch_lse_write_f32(const float* G, int64_t ldg, float* P, int64_t ldp, int n_rot, int64_t n_data,
                                const double* log_w, const double* S, const double* b, const double* L,
                                double* rho, hipStream_t st) {
  lse_write_kernel<float><<<(unsigned)((n_rot + kWriteRows - 1) / kWriteRows), 256, 0, st>>>(
      G, ldg, P, ldp, n_rot, n_data, log_w, S, b, L, rho);
  return hipGetLastError();
}

hipError_t launch_lse_write_bf16(const float* G, int64_t ldg, void* P, int64_t ldp, int n_rot, int64_t n_data,
                                 const double* log_w, const double* S, const double* b, const double* L,
                                 double* rho, hipStream_t st) {
  lse_write_kernel<__hip_bfloat16><<<(unsigned)((n_rot + kWriteRows - 1) / kWriteRows), 256, 0, st>>>(
      G, ldg, (__hip_bfloat16*)P, ldp, n_rot, n_data, log_w, S, b, L, rho);
  return hipGetLastError();
}

}  // namespace emc
