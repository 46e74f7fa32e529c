// BF16 MFMA GEMM (FP32 accumulation) for the mixed-precision form:
//   log-likelihood  G_jk  = scale_j * sum_i (hi_ji + lo_ji) K_ki   (DUAL: two A terms)
//   M-step          W'_ji = sum_k P_jk KT_ik                      (single A term)
// Both operands are read along the reduction index ("NT").  Photon counts are
// exact in BF16; the slice split hi + lo keeps ~16 significant bits.
//
// Workgroup tile 256 x 256 x 64 with 8 waves (two per SIMD, so that one can
// issue MFMAs while the other waits on LDS): the two-term product in a 2 x 4
// arrangement of 128 x 64 per wave (8 x 4 v_mfma_f32_16x16x32_bf16 tiles), the
// single-term one in 4 x 2 of 64 x 128 (4 x 8 tiles: 16 KB of LDS reads per wave
// and 32-deep step instead of 20; the two-term product would not fit its
// registers so); 4 waves of 128 x 128 when built with EMC_BF16_WAVES=4.  LDS stages laid out
// [row][k], 128-byte rows with their 16-byte chunks swizzled (chunk c of row r at
// c ^ ((r >> 1) & 7): neither the stores nor the reads of 16 rows at one k collide
// in a bank; 16 bytes of padding per row instead measured 1.26e10 bank-conflict
// cycles per log-likelihood launch and 11 % more time); the next stage's global loads (full
// 128-byte row segments) are issued into registers before the current stage's
// 4096 MFMA cycles, which hides their latency.  The single-term product holds two
// stages and stores the next one while the current one is read (one barrier per
// stage); the two-term one holds one stage (two barriers per stage).  A lane feeds one MFMA with 8
// consecutive k of one row (one 128-bit LDS read); A and B use the same k
// assignment, so the product sums the same pairs.
//
// Split reduction: with `stages` < ceil(Kd / 64) the grid holds every output tile
// once per k range of `stages` x 64; range s writes its partial product to the
// slab C + s * c_split (the caller adds the slabs).  Products with few output
// tiles (fewer than a few per CU) use it to fill the chip.
#include "emc_device.h"

namespace emc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));  // 16 bytes = 8 bf16

constexpr int TM = 256, TN = 256, TK = 64, LROW = TK;  // LDS row in bf16 elements (unpadded, chunks swizzled)
// 16-byte chunk c of row r sits at chunk c ^ ((r >> 1) & 7)
__device__ __forceinline__ int lds_at(int r, int c) { return r * LROW + 8 * (c ^ ((r >> 1) & 7)); }
constexpr int GROUP = 8;

template <bool DUAL, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void gemm_bf16_kernel(const uint16_t* __restrict__ A, const uint16_t* __restrict__ A2,
                                                        const uint16_t* __restrict__ B,
                                                        const float* __restrict__ row_scale, float* __restrict__ C,
                                                        int64_t M, int64_t N, int64_t Kd, int64_t lda, int64_t ldb,
                                                        int64_t ldc, int64_t stages, int64_t c_split) {
  constexpr int NA = DUAL ? 2 : 1;
  // single-term products keep two stages in LDS (128 KB), so that one barrier per
  // stage suffices; the two-term one has room for one stage
  constexpr int NB = DUAL ? 1 : 2;
  __shared__ __attribute__((aligned(16))) uint16_t As[NB][NA][TM * LROW];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[NB][TN * LROW];

  // 4 waves: 2 x 2 of 128 x 128; 8 waves (two per SIMD): 2 x 4 of 128 x 64
  constexpr int NT = 64 * WAVES;
  // the single-term product takes 64 x 128 per wave (fewer LDS bytes per MFMA); the
  // two-term one keeps 128 x 64 (64 x 128 would not fit its registers)
  constexpr int WROWS = WAVES == 8 && !DUAL ? 64 : 128;   // rows of C per wave
  constexpr int WCOLS = WAVES == 8 && DUAL ? 64 : 128;    // columns of C per wave
  constexpr int IT = WROWS / 16, JT = WCOLS / 16;
  constexpr int WN = TN / WCOLS;                // waves along N
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  const int64_t tiles_m = (M + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
  const int64_t split = blockIdx.x / (tiles_m * tiles_n);
  const int64_t pid = blockIdx.x - split * (tiles_m * tiles_n);
  C += split * c_split;
  const int64_t group = (int64_t)GROUP * tiles_n;
  const int64_t first_m = (pid / group) * GROUP;
  const int64_t gm = (tiles_m - first_m) < GROUP ? (tiles_m - first_m) : GROUP;
  const int64_t tm = first_m + (pid % group) % gm;
  const int64_t tn = (pid % group) / gm;
  const int64_t m0 = tm * TM, n0 = tn * TN;
  // source rows of this thread's load slots (row r = tid / 8 + (NT / 8) u), as
  // element offsets of the row starts (-1: the slot reads zero)
  constexpr int SLOTS = TM * 8 / NT;
  const int ch = tid & 7;
  int32_t arow[SLOTS];  // A row of each slot, -1 reads zero (B rows are n0 + r)
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int r = (tid >> 3) + (NT / 8) * u;
    arow[u] = m0 + r < M ? (int32_t)(m0 + r) : -1;
  }
  const uint16_t* Ab = A + 8 * ch;
  const uint16_t* A2b = A2 + 8 * ch;
  const uint16_t* Bb = B + (n0 + (tid >> 3)) * ldb + 8 * ch;
  const int64_t nvalid = N - n0 - (tid >> 3);  // slot u reads B when (NT / 8) u < nvalid

  u4 ra0[SLOTS], ra1[SLOTS], rb[SLOTS];
  const u4 zero = {0u, 0u, 0u, 0u};
#define EMC_LOAD_STAGE(k0)                                                                              \
  _Pragma("unroll") for (int u = 0; u < SLOTS; ++u) {                                                 \
    const int64_t ao = (int64_t)arow[u] * lda + (k0);                                                 \
    ra0[u] = arow[u] >= 0 ? *reinterpret_cast<const u4*>(Ab + ao) : zero;                             \
    if constexpr (DUAL) ra1[u] = arow[u] >= 0 ? *reinterpret_cast<const u4*>(A2b + ao) : zero;        \
    rb[u] = (NT / 8) * u < nvalid ? *reinterpret_cast<const u4*>(Bb + (int64_t)(NT / 8) * u * ldb + (k0)) : zero; \
  }
#define EMC_STORE_STAGE(buf)                                                                            \
  _Pragma("unroll") for (int u = 0; u < SLOTS; ++u) {                                                 \
    const int r = (tid >> 3) + (NT / 8) * u;                                                            \
    *reinterpret_cast<u4*>(&As[buf][0][lds_at(r, ch)]) = ra0[u];                               \
    if constexpr (DUAL) *reinterpret_cast<u4*>(&As[buf][NA - 1][lds_at(r, ch)]) = ra1[u];      \
    *reinterpret_cast<u4*>(&Bs[buf][lds_at(r, ch)]) = rb[u];                                   \
  }

  f4 acc[IT][JT];
#pragma unroll
  for (int i = 0; i < IT; ++i)
#pragma unroll
    for (int j = 0; j < JT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // this workgroup's k stages [s0, s1); the host gives every split at least one
  const int64_t nk = (Kd + TK - 1) / TK;
  const int64_t s0 = split * stages, s1 = s0 + stages < nk ? s0 + stages : nk;
  EMC_LOAD_STAGE(s0 * TK)
  EMC_STORE_STAGE(0)
  __syncthreads();

  const int arow_l = wm * WROWS + (lane & 15), brow_l = wn * WCOLS + (lane & 15), kofs = 8 * (lane >> 4);
  for (int64_t s = s0; s < s1; ++s) {
    const int cur = NB == 2 ? (int)((s - s0) & 1) : 0;
    if (s + 1 < s1) {
      const int64_t k1 = (s + 1) * TK;
      EMC_LOAD_STAGE(k1)
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 32) {
      bf8 b[JT];
#pragma unroll
      for (int j = 0; j < JT; ++j)
        b[j] = *reinterpret_cast<const bf8*>(&Bs[cur][lds_at(brow_l + 16 * j, (kk + kofs) >> 3)]);
#pragma unroll
      for (int i = 0; i < IT; ++i) {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const bf8 av = *reinterpret_cast<const bf8*>(&As[cur][a][lds_at(arow_l + 16 * i, (kk + kofs) >> 3)]);
#pragma unroll
          for (int j = 0; j < JT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[j], acc[i][j], 0, 0, 0);
        }
      }
    }
    if constexpr (NB == 2) {
      // the other stage was last read in the previous step, which every wave has
      // left (barrier below); the barrier then publishes this store for the next step
      if (s + 1 < s1) {
        EMC_STORE_STAGE(cur ^ 1)
      }
      __syncthreads();
    } else {
      __syncthreads();
      if (s + 1 < s1) {
        EMC_STORE_STAGE(0)
        __syncthreads();
      }
    }
  }
#undef EMC_LOAD_STAGE
#undef EMC_STORE_STAGE

  const int64_t rbase = m0 + wm * WROWS + 4 * (lane >> 4);
  const int64_t cbase = n0 + wn * WCOLS + (lane & 15);
#pragma unroll
  for (int i = 0; i < IT; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rbase + 16 * i + r;
      if (row >= M) continue;
      const float sc = DUAL ? row_scale[row] : 1.0f;
#pragma unroll
      for (int j = 0; j < JT; ++j) {
        const int64_t col = cbase + 16 * j;
        if (col < N) C[row * ldc + col] = sc * acc[i][j][r];
      }
    }
  }
}

#ifndef EMC_BF16_WAVES
#define EMC_BF16_WAVES 8
#endif
constexpr int kWaves = EMC_BF16_WAVES;
static_assert(kWaves == 4 || kWaves == 8, "4 or 8 waves per workgroup");

template <bool DUAL>
static hipError_t launch(const void* A, const void* A2, const void* B, const float* scale, float* C, int64_t M,
                         int64_t N, int64_t Kd, int64_t lda, int64_t ldb, int64_t ldc, hipStream_t st,
                         int splits = 1) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  const int64_t nk = (Kd + TK - 1) / TK;
  const int64_t stages = splits > 1 ? (nk + splits - 1) / splits : (nk > 0 ? nk : 1);
  // every split must own at least one stage (gemm_bf16_splits returns such counts)
  if (splits < 1 || (splits > 1 && (splits - 1) * stages >= nk)) return hipErrorInvalidValue;
  gemm_bf16_kernel<DUAL, kWaves><<<(unsigned)(tiles * splits), 64 * kWaves, 0, st>>>(
      (const uint16_t*)A, (const uint16_t*)A2, (const uint16_t*)B, scale, C, M, N, Kd, lda, ldb, ldc, stages,
      M * ldc);
  return hipGetLastError();
}

// Split count for a product on a chip of kChipCUs CUs (one workgroup per CU):
// the count of at most max_splits, each split at least kMinSplitStages stages,
// that minimises (rounds of workgroups) x (stages per split), kept only when it
// saves 5 % against the best smaller count.  Every split it returns owns at least
// one stage.
constexpr int64_t kChipCUs = 256;
constexpr int64_t kMinSplitStages = 4;
int gemm_bf16_splits(int64_t M, int64_t N, int64_t Kd, int max_splits) {
  if (M <= 0 || N <= 0 || Kd <= 0) return 1;
  const int64_t tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN), nk = (Kd + TK - 1) / TK;
  int best = 1;
  double best_t = (double)((tiles + kChipCUs - 1) / kChipCUs);
  for (int s = 2; s <= max_splits; ++s) {
    const int64_t per = (nk + s - 1) / s;
    if (per < kMinSplitStages) break;
    const int64_t eff = (nk + per - 1) / per;
    const double t = (double)((tiles * eff + kChipCUs - 1) / kChipCUs) * (double)per / (double)nk;
    if (t < 0.95 * best_t) {
      best = (int)eff;
      best_t = t;
    }
  }
  return best;
}

hipError_t launch_gemm_bf16_nt_split(const void* A, const void* B, float* C, int64_t M, int64_t N, int64_t Kd,
                                     int64_t lda, int64_t ldb, int64_t ldc, int splits, hipStream_t st) {
  return launch<false>(A, nullptr, B, nullptr, C, M, N, Kd, lda, ldb, ldc, st, splits);
}

hipError_t launch_gemm_bf16_dual_nt_split(const void* A_hi, const void* A_lo, const void* B, const float* row_scale,
                                          float* C, int64_t M, int64_t N, int64_t Kd, int64_t lda, int64_t ldb,
                                          int64_t ldc, int splits, hipStream_t st) {
  return launch<true>(A_hi, A_lo, B, row_scale, C, M, N, Kd, lda, ldb, ldc, st, splits);
}

// out[e] = sum of the parts' slabs part[s * n + e], s = 0, 1, ... in order
__global__ void sum_slabs_kernel(const float* __restrict__ part, int parts, int64_t n, float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    float v = part[e];
    for (int s = 1; s < parts; ++s) v += part[e + s * n];
    out[e] = v;
  }
}

hipError_t launch_sum_slabs(const float* part, int parts, int64_t n, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (parts < 1) return hipErrorInvalidValue;
  const int64_t g = (n + 255) / 256;
  sum_slabs_kernel<<<(unsigned)(g > 65536 ? 65536 : g), 256, 0, st>>>(part, parts, n, out);
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
