// E-step, eq. (2.4): responsibilities as an FP64 log-sum-exp over rotations of
// the log-joint a_jk = Q_jk + log w_j = G_jk + b_k - S_j + log w_j, on the
// rotation-major layout G[j][k] (frames contiguous).  A frame's normalisation
// needs only its maximum and the sum of exp(a - max); these two statistics are
// also all that rotation shares must exchange (Section 3.2).
//
// The statistics pass skips terms more than kLseDrop below the running maximum
// (exact to FP64 rounding, lse.h) and evaluates the rest with an FP64
// exponential restricted to x <= 0 (lse.h), one per term kept.  A lane takes
// four consecutive frames (16-byte loads, four independent running sums) and the
// sixteen waves of a workgroup split the rotations; their partials are merged in
// wave order, so the result does not depend on timing.  The write pass keeps
// every responsibility, however small (the c-step's ratio is scale-free: a voxel
// reached only by improbable rotations still takes their weighted mean); it forms
// a - L_k in FP64 and evaluates the exponential in FP32, the precision P is
// stored in (or finer), skipping only exponents below -110, whose FP32 value is
// 0.  (A first pass for each frame's maximum, so that whole waves could skip, was
// measured slower: in the early iterations most terms are near their frame's
// maximum and the extra read of G costs more than it saves.)
#include "emc_device.h"
#include "lse.h"

namespace emc {

constexpr int kStatLane = 4;                   // consecutive frames per lane: one vector load per rotation
constexpr int kStatWaves = 16;                 // waves per workgroup; wave w takes rotations w, w + 16, ...
constexpr int kStatFrames = 64 * kStatLane;    // frames per workgroup
constexpr int kStatUnroll = 4;                 // rotations a wave has in flight
typedef float StatVec __attribute__((ext_vector_type(kStatLane)));

// Per-frame (max, sum exp) of a_jk over rotations [j_begin, j_end), FP64, online;
// blockIdx.y picks the rotation chunk when the rotations are split (out: the
// chunk's partials at out + 2 * n_data * blockIdx.y).  Rows of G hold at least
// ceil(n_data / kStatFrames) * kStatFrames frames (the data stride).
__global__ __launch_bounds__(64 * kStatWaves) void lse_stats_kernel(const float* __restrict__ G, int64_t ld, int n_rot,
                                                                   int64_t n_data, const double* __restrict__ log_w,
                                                                   const double* __restrict__ S,
                                                                   const double* __restrict__ b, int per_chunk,
                                                                   double* __restrict__ out) {
  __shared__ double sm[kStatWaves][kStatFrames], ss[kStatWaves][kStatFrames];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t k0 = (int64_t)blockIdx.x * kStatFrames + kStatLane * lane;
  const int jb = blockIdx.y * per_chunk;
  const int je = jb + per_chunk < n_rot ? jb + per_chunk : n_rot;
  double bk[kStatLane], m[kStatLane], s[kStatLane];
#pragma unroll
  for (int i = 0; i < kStatLane; ++i) {
    bk[i] = k0 + i < n_data ? b[k0 + i] : 0.0;
    m[i] = -INFINITY;
    s[i] = 0.0;
  }
  if (k0 < n_data) {
    const ExpCoef ec = exp_coef();
    for (int j0 = jb + wave; j0 < je; j0 += kStatWaves * kStatUnroll) {
      StatVec g[kStatUnroll];  // rows past the range re-read the last one (not used), so no load waits on a branch
#pragma unroll
      for (int u = 0; u < kStatUnroll; ++u) {
        const int j = j0 + kStatWaves * u < je ? j0 + kStatWaves * u : je - 1;
        g[u] = *(const StatVec*)(G + (int64_t)j * ld + k0);
      }
#pragma unroll
      for (int u = 0; u < kStatUnroll; ++u) {
        const int j = j0 + kStatWaves * u;
        if (j >= je) break;
        const double e = log_w[j] - S[j];
#pragma unroll
        for (int i = 0; i < kStatLane; ++i) lse_push(m[i], s[i], ((double)g[u][i] + bk[i]) + e, ec);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kStatLane; ++i) {
    sm[wave][kStatLane * lane + i] = m[i];
    ss[wave][kStatLane * lane + i] = s[i];
  }
  __syncthreads();
  for (int f = threadIdx.x; f < kStatFrames; f += 64 * kStatWaves) {
    const int64_t k = (int64_t)blockIdx.x * kStatFrames + f;
    if (k >= n_data) continue;
    double mm = sm[0][f], sv = ss[0][f];
    for (int w = 1; w < kStatWaves; ++w) lse_merge(mm, sv, sm[w][f], ss[w][f]);
    double* o = out + 2 * n_data * blockIdx.y;
    o[2 * k] = mm;
    o[2 * k + 1] = sv;
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
constexpr int kWriteLane = 4;  // consecutive frames per lane

// four responsibilities rounded to PT, stored as one vector; returns their sum
__device__ __forceinline__ double store4(float* dst, const float (&v)[4]) {
  *(float4*)dst = float4{v[0], v[1], v[2], v[3]};
  return ((double)v[0] + (double)v[1]) + ((double)v[2] + (double)v[3]);
}
__device__ __forceinline__ double store4(__hip_bfloat16* dst, const float (&v)[4]) {
  __hip_bfloat16 q[4];
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    q[i] = __float2bfloat16(v[i]);
    sum += (double)__bfloat162float(q[i]);
  }
  *(uint2*)dst = *(const uint2*)q;
  return sum;
}

// P[j][k] = exp(G[j][k] + (log w_j - S_j) + (b_k - L_k)), written as PT (FP32 or
// BF16) with zeros in the padding frames; rho_j = sum_k of the stored values,
// reduced in the block (deterministic).  P may alias G when PT is float: a lane
// reads its rows' four frames before it writes any of them.  The row strides
// are multiples of 4 and G, P 16-byte aligned (checked by the launchers).
template <typename PT>
__global__ __launch_bounds__(256) void lse_write_kernel(const float* G, int64_t ldg, PT* P, int64_t ldp,
                                                        int n_rot, int64_t n_data, const double* __restrict__ log_w,
                                                        const double* __restrict__ S,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ L, double* __restrict__ rho) {
  __shared__ double red[kWriteRows][4];
  const int j0 = blockIdx.x * kWriteRows;
  const int rows = n_rot - j0 < kWriteRows ? n_rot - j0 : kWriteRows;
  double e[kWriteRows], acc[kWriteRows];
#pragma unroll
  for (int r = 0; r < kWriteRows; ++r) {
    e[r] = r < rows ? log_w[j0 + r] - S[j0 + r] : 0.0;
    acc[r] = 0.0;
  }
  for (int64_t k = kWriteLane * threadIdx.x; k < ldp; k += kWriteLane * 256) {
    double sh[kWriteLane];  // padding frames read the last frame's (not used): no load waits on a branch
#pragma unroll
    for (int i = 0; i < kWriteLane; ++i) {
      const int64_t kk = k + i < n_data ? k + i : n_data - 1;
      sh[i] = b[kk] - L[kk];
    }
    float4 g[kWriteRows];  // rows past n_rot re-read the last one (not used)
#pragma unroll
    for (int r = 0; r < kWriteRows; ++r) g[r] = *(const float4*)(G + (int64_t)(j0 + (r < rows ? r : rows - 1)) * ldg + k);
#pragma unroll
    for (int r = 0; r < kWriteRows; ++r) {
      if (r >= rows) break;
      const float gv[4] = {g[r].x, g[r].y, g[r].z, g[r].w};
      float v[4];
#pragma unroll
      for (int i = 0; i < kWriteLane; ++i) {
        const float x = (float)(((double)gv[i] + sh[i]) + e[r]);  // a - L_k
        // below -110, exp(x) rounds to 0 in FP32: skipping it changes nothing
        v[i] = k + i < n_data && x > -110.0f ? expf(x) : 0.0f;
      }
      acc[r] += store4(P + (int64_t)(j0 + r) * ldp + k, v);
    }
  }
#pragma unroll
  for (int r = 0; r < kWriteRows; ++r) {
    const double v = wave_sum(acc[r]);
    if ((threadIdx.x & 63) == 0) red[r][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < rows) {
    const int j = j0 + threadIdx.x;
    rho[j] = (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
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
  if ((ld & 3) != 0 || ld < (n_data + kStatFrames - 1) / kStatFrames * kStatFrames || ((uintptr_t)G & 15) != 0)
    return hipErrorInvalidValue;
  const int nc = part ? lse_chunks(n_rot, n_data) : 1;
  const int per = (n_rot + nc - 1) / nc;
  const dim3 grid((unsigned)((n_data + kStatFrames - 1) / kStatFrames), (unsigned)nc);
  lse_stats_kernel<<<grid, 64 * kStatWaves, 0, st>>>(G, ld, n_rot, n_data, log_w, S, b, per, nc > 1 ? part : stats);
  if (nc > 1) lse_chunks_kernel<<<(unsigned)((n_data + 255) / 256), 256, 0, st>>>(part, nc, n_data, stats);
  return hipGetLastError();
}

hipError_t launch_lse_finish(const double* stats, int64_t n_data, double* L, hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  lse_finish_kernel<<<(unsigned)((n_data + 255) / 256), 256, 0, st>>>(stats, n_data, L);
  return hipGetLastError();
}

bool vec4_ok(const void* G, int64_t ldg, const void* P, int64_t ldp) {
  return ((ldg | ldp) & 3) == 0 && (((uintptr_t)G | (uintptr_t)P) & 15) == 0;
}

hipError_t launch_lse_write_f32(const float* G, int64_t ldg, float* P, int64_t ldp, int n_rot, int64_t n_data,
                                const double* log_w, const double* S, const double* b, const double* L,
                                double* rho, hipStream_t st) {
  if (!vec4_ok(G, ldg, P, ldp)) return hipErrorInvalidValue;
  lse_write_kernel<float><<<(unsigned)((n_rot + kWriteRows - 1) / kWriteRows), 256, 0, st>>>(
      G, ldg, P, n_data > 0 ? ldp : 0, n_rot, n_data, log_w, S, b, L, rho);
  return hipGetLastError();
}

hipError_t launch_lse_write_bf16(const float* G, int64_t ldg, void* P, int64_t ldp, int n_rot, int64_t n_data,
                                 const double* log_w, const double* S, const double* b, const double* L,
                                 double* rho, hipStream_t st) {
  if (!vec4_ok(G, ldg, P, ldp)) return hipErrorInvalidValue;
  lse_write_kernel<__hip_bfloat16><<<(unsigned)((n_rot + kWriteRows - 1) / kWriteRows), 256, 0, st>>>(
      G, ldg, (__hip_bfloat16*)P, n_data > 0 ? ldp : 0, n_rot, n_data, log_w, S, b, L, rho);
  return hipGetLastError();
}

}  // namespace emc
