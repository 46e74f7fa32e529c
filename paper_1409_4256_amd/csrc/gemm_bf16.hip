// BF16 MFMA GEMM (FP32 accumulation) for the mixed-precision form:
//   log-likelihood  G_jk  = scale_j * sum_i (hi_ji + lo_ji) K_ki   (DUAL: two A terms)
//   M-step          W'_ji = sum_k P_jk KT_ik                      (single A term)
// Both operands are read along the reduction index ("NT").  Photon counts are
// exact in BF16; the slice split hi + lo keeps ~16 significant bits.
//
// Workgroup tile 256 x 256 x 32, 4 waves in a 2 x 2 arrangement, each wave
// 128 x 128 from 8 x 8 v_mfma_f32_16x16x32_bf16 tiles.  Operands are staged
// through double-buffered LDS laid out [row][k] (80-byte rows: 64 bytes of data
// + 16 of padding, so eight lanes' 16-byte reads hit distinct banks).  A lane
// feeds one MFMA with 8 consecutive k of one row (one 128-bit LDS read); A and
// B use the same k assignment, so the product sums the same pairs.
#include "emc_device.h"

namespace emc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TM = 256, TN = 256, TK = 32, LROW = TK + 8;  // LDS row in bf16 elements
constexpr int GROUP = 8;

// GATHER: grouped form for the learned proposal.  Workgroup w takes tile
// tiles[w] = (g, t): A rows are list[off[g] + 256 t + r] (-1 reads zero), B rows
// are the 256 frames of block g (rows >= N read zero), and C is the compact
// [list row][256] buffer (ldc = 256).
template <bool DUAL, bool GATHER>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const uint16_t* __restrict__ A, const uint16_t* __restrict__ A2,
                                                        const uint16_t* __restrict__ B,
                                                        const float* __restrict__ row_scale, float* __restrict__ C,
                                                        int64_t M, int64_t N, int64_t Kd, int64_t lda, int64_t ldb,
                                                        int64_t ldc, const int32_t* __restrict__ list,
                                                        const int64_t* __restrict__ off,
                                                        const int2* __restrict__ tiles) {
  constexpr int NA = DUAL ? 2 : 1;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][NA][TM * LROW];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][TN * LROW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  int64_t m0, n0;
  if constexpr (GATHER) {
    const int2 tl = tiles[blockIdx.x];
    m0 = off[tl.x] + (int64_t)TM * tl.y;
    n0 = (int64_t)TN * tl.x;
  } else {
    const int64_t tiles_m = (M + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
    const int64_t pid = blockIdx.x;
    const int64_t group = (int64_t)GROUP * tiles_n;
    const int64_t first_m = (pid / group) * GROUP;
    const int64_t gm = (tiles_m - first_m) < GROUP ? (tiles_m - first_m) : GROUP;
    const int64_t tm = first_m + (pid % group) % gm;
    const int64_t tn = (pid % group) / gm;
    m0 = tm * TM;
    n0 = tn * TN;
  }
  // A row of each of this thread's four load slots (gathered rows resolved once)
  int64_t arow_src[4];
  bool arow_ok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = (tid + 256 * u) >> 2;
    if constexpr (GATHER) {
      const int32_t j = list[m0 + r];
      arow_src[u] = j < 0 ? 0 : j;
      arow_ok[u] = j >= 0;
    } else {
      arow_src[u] = m0 + r;
      arow_ok[u] = m0 + r < M;
    }
  }

  uint4 ra[NA][4], rb[4];
  const uint4 zero = {0u, 0u, 0u, 0u};

  auto load_stage = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = tid + 256 * u, r = f >> 2, ch = f & 3;
      const int64_t ma = arow_src[u], nb = n0 + r;
      const int64_t ka = k0 + 8 * ch;
      ra[0][u] = arow_ok[u] ? *reinterpret_cast<const uint4*>(A + ma * lda + ka) : zero;
      if constexpr (DUAL) ra[NA - 1][u] = arow_ok[u] ? *reinterpret_cast<const uint4*>(A2 + ma * lda + ka) : zero;
      rb[u] = nb < N ? *reinterpret_cast<const uint4*>(B + nb * ldb + ka) : zero;
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = tid + 256 * u, r = f >> 2, ch = f & 3;
#pragma unroll
      for (int a = 0; a < NA; ++a) *reinterpret_cast<uint4*>(&As[buf][a][r * LROW + 8 * ch]) = ra[a][u];
      *reinterpret_cast<uint4*>(&Bs[buf][r * LROW + 8 * ch]) = rb[u];
    }
  };

  f4 acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int64_t nk = (Kd + TK - 1) / TK;
  load_stage(0);
  store_stage(0);
  __syncthreads();

  const int arow = wm * 128 + (lane & 15), brow = wn * 128 + (lane & 15), kofs = 8 * (lane >> 4);
  for (int64_t s = 0; s < nk; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nk) load_stage((s + 1) * TK);
    bf8 b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = *reinterpret_cast<const bf8*>(&Bs[buf][(brow + 16 * j) * LROW + kofs]);
#pragma unroll
    for (int a = 0; a < NA; ++a) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bf8 av = *reinterpret_cast<const bf8*>(&As[buf][a][(arow + 16 * i) * LROW + kofs]);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (s + 1 < nk) store_stage(buf ^ 1);
    __syncthreads();
  }

  const int64_t rbase = m0 + wm * 128 + 4 * (lane >> 4);
  const int64_t cbase = n0 + wn * 128 + (lane & 15);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rbase + 16 * i + r;
      float sc = 1.0f;
      if constexpr (GATHER) {
        const int32_t j = list[row];
        sc = DUAL ? (j >= 0 ? row_scale[j] : 0.0f) : 1.0f;
      } else {
        if (row >= M) continue;
        if (DUAL) sc = row_scale[row];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t col = cbase + 16 * j;
        if (col < N) {
          if constexpr (GATHER)
            C[row * TN + (col - n0)] = sc * acc[i][j][r];
          else
            C[row * ldc + col] = sc * acc[i][j][r];
        }
      }
    }
  }
}

template <bool DUAL>
static hipError_t launch(const void* A, const void* A2, const void* B, const float* scale, float* C, int64_t M,
                         int64_t N, int64_t Kd, int64_t lda, int64_t ldb, int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  gemm_bf16_kernel<DUAL, false><<<(unsigned)tiles, 256, 0, st>>>((const uint16_t*)A, (const uint16_t*)A2,
                                                                 (const uint16_t*)B, scale, C, M, N, Kd, lda, ldb,
                                                                 ldc, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16_dual_gather(const void* A_hi, const void* A_lo, const void* B, const float* row_scale,
                                        float* C, int64_t n_frames, int64_t Kd, int64_t lda, int64_t ldb,
                                        const int32_t* list, const int64_t* off, const int2* tiles, int64_t n_tiles,
                                        hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  gemm_bf16_kernel<true, true><<<(unsigned)n_tiles, 256, 0, st>>>(
      (const uint16_t*)A_hi, (const uint16_t*)A_lo, (const uint16_t*)B, row_scale, C, 0, n_frames, Kd, lda, ldb, TN,
      list, off, tiles);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16_dual_nt(const void* A_hi, const void* A_lo, const void* B, const float* row_scale,
                                    float* C, int64_t M, int64_t N, int64_t Kd, int64_t lda, int64_t ldb, int64_t ldc,
                                    hipStream_t st) {
  return launch<true>(A_hi, A_lo, B, row_scale, C, M, N, Kd, lda, ldb, ldc, st);
}

hipError_t launch_gemm_bf16_nt(const void* A, const void* B, float* C, int64_t M, int64_t N, int64_t Kd, int64_t lda,
                               int64_t ldb, int64_t ldc, hipStream_t st) {
  return launch<false>(A, nullptr, B, nullptr, C, M, N, Kd, lda, ldb, ldc, st);
}

}  // namespace emc
