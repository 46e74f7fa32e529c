// FP32 MFMA GEMM for the two dense contractions of the iteration, both with
// operands contiguous along the reduction index ("NT"):
//   log-likelihood  G_jk  = sum_i logW_ji K_ki    (reduction over pixels)
//   M-step          W'_ji = sum_k P_jk KT_ik      (reduction over frames)
//
// Workgroup tile 256 x 256 x 32 (M x N x K), 8 waves in a 2 x 4 arrangement (two
// per SIMD, so that one issues MFMAs while the other waits at the stage barrier or
// on LDS), each wave 128 x 64 built from 8 x 4 v_mfma_f32_16x16x4_f32 tiles
// (the proposal network's small products: 256 x 128 with 4 waves).  Operands
// are staged through double-buffered LDS laid out [row][k], 128-byte rows with
// their 16-byte chunks swizzled (chunk c of row r at c ^ ((r >> 1) & 7), so that
// neither the 16-byte stores nor the reads of 16 rows at one k collide in a
// bank; a 16-byte pad per row instead measured 1.5e10 bank-conflict cycles per
// launch); every lane reads 4 consecutive k of one row with a single 128-bit LDS read
// and feeds them to 4 successive MFMAs (the k order inside a 16-wide chunk is
// permuted identically for both operands, which leaves the sum unchanged).
#include "emc_device.h"

namespace emc {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = 256, BK = 32;
__device__ __forceinline__ int lds_at(int r, int c) { return r * BK + 4 * (c ^ ((r >> 1) & 7)); }
constexpr int GROUP_M = 8;  // M tiles per schedule group: blocks sharing an M tile land on one XCD

// USE only names the instantiation (0: the iteration's contractions, 1: the proposal
// network's linear layer), so that kernel traces list the two apart.  NWN: waves
// along N; the workgroup has 2 x NWN waves of 128 x 64 and a tile BM x 64 NWN.
template <int USE, int NWN>
__global__ __launch_bounds__(128 * NWN) void gemm_f32_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                              float* __restrict__ C, int64_t M, int64_t N, int64_t Kd,
                                                              int64_t lda, int64_t ldb, int64_t ldc) {
  constexpr int BN = 64 * NWN, NT = 128 * NWN;
  constexpr int LA = BM * BK / 4 / NT, LB = BN * BK / 4 / NT;  // 16-byte loads per thread and stage
  // two waves per SIMD (NWN = 4) fit their 256 registers only with one 16-deep k step live
  constexpr int KU = NWN == 2 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) float As[2][BM * BK];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN * BK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;

  // grouped tile order: GROUP_M consecutive M tiles sweep all N tiles together
  const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int64_t pid = blockIdx.x;
  const int64_t group = (int64_t)GROUP_M * tiles_n;
  const int64_t first_m = (pid / group) * GROUP_M;
  const int64_t gm = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
  const int64_t tm = first_m + (pid % group) % gm;
  const int64_t tn = (pid % group) / gm;
  const int64_t m0 = tm * BM, n0 = tn * BN;

  f4 ra[LA], rb[LB];
  const f4 zero = {0.f, 0.f, 0.f, 0.f};

  auto load_stage = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int f = tid + NT * u, r = f >> 3, c4 = f & 7;
      const int64_t row = m0 + r;
      ra[u] = row < M ? *reinterpret_cast<const f4*>(A + row * lda + k0 + 4 * c4) : zero;
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int f = tid + NT * u, r = f >> 3, c4 = f & 7;
      const int64_t row = n0 + r;
      rb[u] = row < N ? *reinterpret_cast<const f4*>(B + row * ldb + k0 + 4 * c4) : zero;
    }
  };

  auto store_stage = [&](int buf) {
    float* as = As[buf];
    float* bs = Bs[buf];
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int f = tid + NT * u, r = f >> 3, c4 = f & 7;
      *reinterpret_cast<f4*>(as + lds_at(r, c4)) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int f = tid + NT * u, r = f >> 3, c4 = f & 7;
      *reinterpret_cast<f4*>(bs + lds_at(r, c4)) = rb[u];
    }
  };

  f4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = zero;

  const int64_t nk = (Kd + BK - 1) / BK;
  load_stage(0);
  store_stage(0);
  __syncthreads();

  const int arow = wm * 128 + (lane & 15), brow = wn * 64 + (lane & 15), kc = lane >> 4;
  for (int64_t s = 0; s < nk; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nk) load_stage((s + 1) * BK);
    const float* as = As[buf];
    const float* bs = Bs[buf];
#pragma unroll KU
    for (int kk = 0; kk < BK; kk += 16) {
      f4 a[8], b[4];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = *reinterpret_cast<const f4*>(as + lds_at(arow + 16 * i, (kk >> 2) + kc));
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const f4*>(bs + lds_at(brow + 16 * j, (kk >> 2) + kc));
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j][t], acc[i][j], 0, 0, 0);
    }
    if (s + 1 < nk) store_stage(buf ^ 1);
    __syncthreads();
  }

  // D layout of the 16x16 MFMA tile: lane holds rows 4*(lane/16)+r, column lane%16
  const int64_t rbase = m0 + wm * 128 + 4 * (lane >> 4);
  const int64_t cbase = n0 + wn * 64 + (lane & 15);
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = cbase + 16 * j;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rbase + 16 * i + r;
        if (row < M) C[row * ldc + col] = acc[i][j][r];
      }
    }
}

template <int USE, int NWN>
hipError_t launch_nt(const float* A, const float* B, float* C, int64_t M, int64_t N, int64_t Kd, int64_t lda,
                     int64_t ldb, int64_t ldc, hipStream_t st) {
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + 64 * NWN - 1) / (64 * NWN));
  gemm_f32_kernel<USE, NWN><<<(unsigned)tiles, 128 * NWN, 0, st>>>(A, B, C, M, N, Kd, lda, ldb, ldc);
  return hipGetLastError();
}

hipError_t launch_gemm_f32_nt(const float* A, const float* B, float* C, int64_t M, int64_t N, int64_t Kd,
                              int64_t lda, int64_t ldb, int64_t ldc, hipStream_t st, bool network) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // the network's linear layer (few output tiles) keeps 256 x 128 tiles
  if (network) return launch_nt<1, 2>(A, B, C, M, N, Kd, lda, ldb, ldc, st);
  return launch_nt<0, 4>(A, B, C, M, N, Kd, lda, ldb, ldc, st);
}

}  // namespace emc
