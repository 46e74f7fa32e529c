// Candidate (learned-proposal) E- and M-steps as cell-major MFMA contractions.
//
// The fine rotations of a coarse cell are split into groups of at most 32; the
// frames that propose the cell form its frame list.  For every group the
// log-likelihoods of all (rotation, listed frame) pairs are one small dense
// product
//     G[frame][r] = scale_r * sum_i (hi_ri + lo_ri) K_i,frame          (eq. 2.4's Q)
// and, after each frame's E-step over its own candidates, the M-step of the
// group is
//     W'_r,i = sum_frames P[r][frame] K_i,frame                         (eq. 2.11)
// Frames are stored sparsely (non-zero pixels, ascending); each workgroup
// expands the frames it needs into LDS, 128-pixel band by band, and feeds the
// dense band to v_mfma_f32_16x16x32_bf16.  A band's LDS rows are owned by one
// wave (it writes, reads and clears them), so the band loops need no barrier.
//
// Storage of a group with frame list length F (Fp = F rounded up to 32):
//   G  float [Fp][32]            frame-major: a frame's 32 values are contiguous
//   P  bf16  [Fp/32][32][32]     blocks of 32 frames, rotation-major inside a block,
//                                which is the MFMA operand layout of the M-step.
#include "emc_device.h"

namespace emc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

constexpr int kGR = 32;             // rotations per group (two 16-row MFMA tiles)
constexpr int kFT = 64;             // frames per log-likelihood workgroup (four 16-column tiles)
constexpr int kBand = 128;          // pixels per band (granularity of the entry-offset table)
constexpr int kLRow = kBand + 8;    // LDS row of one frame's band, bf16 (272 bytes: conflict-free 16-byte reads)
constexpr int kFB = 32;             // frames per M-step block (one MFMA reduction step)
constexpr int kKRow = kFB + 8;      // LDS row of one pixel's frames, bf16 (80 bytes)
constexpr int kRange = 4 * kBand;   // pixels per M-step workgroup (one band per wave)

__device__ __forceinline__ uint16_t count_bf16(uint32_t e) {
  // counts up to 256 are exact in BF16: the upper half of the FP32 pattern
  return (uint16_t)(__float_as_uint((float)(e & 0xffffu)) >> 16);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Writes (CLEAR = false) or zeroes (CLEAR = true) the band's entries of the frames
// held by lanes 0..nf-1 (lane s: entry range [base + beg, base + end)).  Entry e goes
// to rows[s * row_stride + (pixel - p0) * col_stride].
template <bool CLEAR>
__device__ __forceinline__ void band_entries(uint16_t* __restrict__ rows, int row_stride, int col_stride,
                                             const uint32_t* __restrict__ nz, int64_t base, int beg, int end, int nf,
                                             int p0, int lane) {
  for (int s = 0; s < nf; ++s) {
    const int b = __builtin_amdgcn_readlane(beg, s);
    const int n = __builtin_amdgcn_readlane(end, s) - b;
    if (n <= 0) continue;  // uniform
    const int64_t at = readlane64(base, s) + b;
    for (int j = lane; j < n; j += 64) {
      const uint32_t e = nz[at + j];
      const int px = (int)(e >> 16) - p0;
      if ((unsigned)px < (unsigned)kBand) rows[s * row_stride + px * col_stride] = CLEAR ? (uint16_t)0 : count_bf16(e);
    }
  }
}

// ------------------------------------------------------------------ log-likelihood
// One workgroup per tile (group g, frames [f0, f0 + 64) of the group's cell).  Wave w
// takes the bands w, w + 4, ... of all 64 frames and both rotation tiles; the four
// partial sums are added in LDS at the end.
__global__ __launch_bounds__(256, 2) void cand_loglik_kernel(
    const int2* __restrict__ tiles, const int4* __restrict__ groups, const int64_t* __restrict__ grp_off,
    const int64_t* __restrict__ cf_ptr, const int32_t* __restrict__ cf_frame, const int64_t* __restrict__ nz_ptr,
    const int32_t* __restrict__ nz_off, int ntab, const uint32_t* __restrict__ nz, const int32_t* __restrict__ cell_rot,
    const uint16_t* __restrict__ hi, int64_t plane, const float* __restrict__ scale, int64_t ps,
    float* __restrict__ G) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[4 * kFT * kLRow];  // 69632 bytes
  __shared__ float ssc[kGR];
  const int2 tl = tiles[blockIdx.x];
  if (tl.x < 0) return;  // padding tile (uniform)
  const int4 gr = groups[tl.x];
  const int c = gr.x, r0 = gr.y, nr = gr.z;
  const int64_t F = cf_ptr[c + 1] - cf_ptr[c];
  const int f0 = tl.y;
  const int nf = (int)(F - f0 < kFT ? F - f0 : kFT);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < kGR) ssc[threadIdx.x] = threadIdx.x < nr ? scale[cell_rot[r0 + threadIdx.x]] : 0.0f;

  // this lane's frame (slot = lane) and its entry range
  int64_t base = 0;
  const int32_t* tab = nz_off;
  if (lane < nf) {
    const int32_t f = cf_frame[cf_ptr[c] + f0 + lane];
    base = nz_ptr[f];
    tab = nz_off + (int64_t)f * ntab;
  }
  // rows of the A operand: rotation (lane & 15) of each 16-row tile, -1 reads zero
  const int m = lane & 15, kq = 8 * (lane >> 4);
  const int64_t ar0 = m < nr ? (int64_t)cell_rot[r0 + m] * ps : -1;
  const int64_t ar1 = 16 + m < nr ? (int64_t)cell_rot[r0 + 16 + m] * ps : -1;
  const bool two = nr > 16;

  uint16_t* rows = lds + wave * kFT * kLRow;
  for (int e = lane; e < kFT * kLRow / 8; e += 64) reinterpret_cast<u4*>(rows)[e] = u4{0u, 0u, 0u, 0u};

  f4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const u4 zero = {0u, 0u, 0u, 0u};
  const int nbands = (int)(ps / kBand);
  for (int band = wave; band < nbands; band += 4) {
    const int p0 = band * kBand;
    const int beg = lane < nf ? tab[band] : 0, end = lane < nf ? tab[band + 1] : 0;
    band_entries<false>(rows, kLRow, 1, nz, base, beg, end, nf, p0, lane);
#pragma unroll
    for (int kk = 0; kk < kBand; kk += 32) {
      const int64_t ko = p0 + kk + kq;
      const u4 h0 = ar0 >= 0 ? *reinterpret_cast<const u4*>(hi + ar0 + ko) : zero;
      const u4 l0 = ar0 >= 0 ? *reinterpret_cast<const u4*>(hi + plane + ar0 + ko) : zero;
      u4 h1 = zero, l1 = zero;
      if (two) {
        h1 = ar1 >= 0 ? *reinterpret_cast<const u4*>(hi + ar1 + ko) : zero;
        l1 = ar1 >= 0 ? *reinterpret_cast<const u4*>(hi + plane + ar1 + ko) : zero;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bf8 bv = *reinterpret_cast<const bf8*>(&rows[(16 * j + m) * kLRow + kk + kq]);
        acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, h0), bv, acc[0][j], 0, 0, 0);
        acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, l0), bv, acc[0][j], 0, 0, 0);
        if (two) {
          acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, h1), bv, acc[1][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, l1), bv, acc[1][j], 0, 0, 0);
        }
      }
    }
    band_entries<true>(rows, kLRow, 1, nz, base, beg, end, nf, p0, lane);
  }

  // sum of the four waves' partials: red[wave][slot][32] floats in the same LDS
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      *reinterpret_cast<f4*>(&red[(wave * kFT + 16 * j + m) * kGR + 16 * i + 4 * (lane >> 4)]) = acc[i][j];
  __syncthreads();
  const int s = threadIdx.x >> 2, mb = 8 * (threadIdx.x & 3);
  if (s < nf) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = 0.0f;
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] += red[(w * kFT + s) * kGR + mb + u];
    float* out = G + grp_off[tl.x] + (int64_t)(f0 + s) * kGR + mb;
    f4 o0, o1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      o0[u] = ssc[mb + u] * v[u];
      o1[u] = ssc[mb + 4 + u] * v[4 + u];
    }
    *reinterpret_cast<f4*>(out) = o0;
    *reinterpret_cast<f4*>(out + 4) = o1;
  }
}

// ------------------------------------------------------------------ E-step
__device__ __forceinline__ void lse_push(double& mx, double& s, double a) {
  if (!(a > -INFINITY)) return;
  if (a > mx) {
    s = s * exp(mx - a) + 1.0;
    mx = a;
  } else {
    s += exp(a - mx);
  }
}

// One wave per candidate frame; lanes take the frame's proposed cells (slot t =
// lane + 64 u).  a = Q + log w_j = G + b_f - S_j + log w_j, log-evidence over the
// frame's candidates in FP64, P = exp(a - L) stored in BF16 (eq. 2.4).
__global__ __launch_bounds__(256) void cand_estep_kernel(
    const float* __restrict__ G, uint16_t* __restrict__ P, const int4* __restrict__ groups,
    const int64_t* __restrict__ grp_off, const int64_t* __restrict__ cg_ptr, const int32_t* __restrict__ cells,
    const int32_t* __restrict__ pair_col, int k_top, int64_t n_frames, const int32_t* __restrict__ cell_rot,
    const double* __restrict__ log_w, const double* __restrict__ S, const double* __restrict__ b,
    double* __restrict__ L) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;  // uniform per wave
  const double bk = b[f];
  double mx = -INFINITY, sum = 0.0;
  for (int t = lane; t < k_top; t += 64) {
    const int c = cells[f * k_top + t];
    if (c < 0) continue;
    const int64_t col = pair_col[f * k_top + t];
    for (int64_t g = cg_ptr[c]; g < cg_ptr[c + 1]; ++g) {
      const int4 gr = groups[g];
      const float* row = G + grp_off[g] + col * kGR;
      for (int r = 0; r < gr.z; ++r) {
        const int j = cell_rot[gr.y + r];
        lse_push(mx, sum, ((double)row[r] + bk) + (log_w[j] - S[j]));
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double m2 = __shfl_xor(mx, o, 64), s2 = __shfl_xor(sum, o, 64);
    if (m2 > mx) {
      sum = sum * exp(mx - m2) + s2;
      mx = m2;
    } else if (m2 > -INFINITY) {
      sum += s2 * exp(m2 - mx);
    }
  }
  const double lse = mx + log(sum);
  if (lane == 0) L[f] = lse;
  for (int t = lane; t < k_top; t += 64) {
    const int c = cells[f * k_top + t];
    if (c < 0) continue;
    const int64_t col = pair_col[f * k_top + t];
    for (int64_t g = cg_ptr[c]; g < cg_ptr[c + 1]; ++g) {
      const int4 gr = groups[g];
      const float* row = G + grp_off[g] + col * kGR;
      uint16_t* pb = P + grp_off[g] + (col >> 5) * (kGR * kFB) + (col & 31);
      for (int r = 0; r < gr.z; ++r) {
        const int j = cell_rot[gr.y + r];
        const double a = ((double)row[r] + bk) + (log_w[j] - S[j]);
        const __hip_bfloat16 p = __float2bfloat16((float)exp(a - lse));
        pb[r * kFB] = __builtin_bit_cast(uint16_t, p);
      }
    }
  }
}

// ------------------------------------------------------------------ M-step
// One workgroup per (group g, 512-pixel range); it runs over the whole frame list
// of the group's cell in blocks of 32 frames.  Wave w owns the range's band w:
// it expands the block's frames there into LDS rows [pixel][frame], contracts them
// with the block's P (B operand, read straight from its blocked layout) and clears
// the rows.  W' rows are written (accumulate: added to what the audited frames'
// dense product left there); the range-0 workgroup also sums rho = sum P.
__global__ __launch_bounds__(256, 2) void cand_mstep_kernel(
    const int4* __restrict__ groups, const int64_t* __restrict__ grp_off, int nranges,
    const int64_t* __restrict__ cf_ptr, const int32_t* __restrict__ cf_frame, const int64_t* __restrict__ nz_ptr,
    const int32_t* __restrict__ nz_off, int ntab, const uint32_t* __restrict__ nz,
    const uint16_t* __restrict__ P, const int32_t* __restrict__ cell_rot, int64_t ps, float* __restrict__ Wp,
    double* __restrict__ rho, const double* __restrict__ rho_a, int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[4 * kBand * kKRow];  // 40960 bytes
  const int64_t g = blockIdx.x / nranges;
  const int pr = (int)(blockIdx.x % nranges);
  const int4 gr = groups[g];
  const int c = gr.x, r0 = gr.y, nr = gr.z;
  const int64_t F = cf_ptr[c + 1] - cf_ptr[c];
  const int32_t* cf = cf_frame + cf_ptr[c];
  const uint16_t* Pg = P + grp_off[g];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int band = pr * 4 + wave;
  const int p0 = band * kBand;
  if ((int64_t)p0 >= ps) return;  // no band for this wave (no barrier follows)
  const bool two = nr > 16;
  const bool do_rho = pr == 0 && wave == 0;
  const int n = lane & 15, kq = 8 * (lane >> 4);

  uint16_t* rows = lds + wave * kBand * kKRow;
  for (int e = lane; e < kBand * kKRow / 8; e += 64) reinterpret_cast<u4*>(rows)[e] = u4{0u, 0u, 0u, 0u};

  f4 acc[8][2];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i][0] = acc[i][1] = f4{0.f, 0.f, 0.f, 0.f};
  double rs0 = 0.0, rs1 = 0.0;
  const u4 zero = {0u, 0u, 0u, 0u};

  for (int64_t f0 = 0; f0 < F; f0 += kFB) {
    const int nf = (int)(F - f0 < kFB ? F - f0 : kFB);
    int64_t base = 0;
    int beg = 0, end = 0;
    if (lane < nf) {
      const int32_t f = cf[f0 + lane];
      base = nz_ptr[f];
      beg = nz_off[(int64_t)f * ntab + band];
      end = nz_off[(int64_t)f * ntab + band + 1];
    }
    band_entries<false>(rows, 1, kKRow, nz, base, beg, end, nf, p0, lane);
    // B operand: frames kq..kq+7 of the block for rotation n (and n + 16)
    const uint16_t* pblk = Pg + (f0 >> 5) * (kGR * kFB);
    u4 b0 = *reinterpret_cast<const u4*>(pblk + n * kFB + kq);
    u4 b1 = two ? *reinterpret_cast<const u4*>(pblk + (16 + n) * kFB + kq) : zero;
    if (nf < kFB) {  // frames past the list end hold no responsibility
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k0 = kq + 2 * u;
        const unsigned keep = (k0 < nf ? 0x0000ffffu : 0u) | (k0 + 1 < nf ? 0xffff0000u : 0u);
        b0[u] &= keep;
        b1[u] &= keep;
      }
    }
    if (do_rho) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        rs0 += (double)(__uint_as_float(b0[u] << 16) + __uint_as_float(b0[u] & 0xffff0000u));
        rs1 += (double)(__uint_as_float(b1[u] << 16) + __uint_as_float(b1[u] & 0xffff0000u));
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bf8 av = *reinterpret_cast<const bf8*>(&rows[(16 * i + n) * kKRow + kq]);
      acc[i][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf8, b0), acc[i][0], 0, 0, 0);
      if (two) acc[i][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf8, b1), acc[i][1], 0, 0, 0);
    }
    band_entries<true>(rows, 1, kKRow, nz, base, beg, end, nf, p0, lane);
  }

  // acc[i][j][r] = W'[rotation 16 j + n][pixel p0 + 16 i + 4 (lane >> 4) + r]
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int mr = 16 * j + n;
    if (mr >= nr) continue;
    float* out = Wp + (int64_t)cell_rot[r0 + mr] * ps + p0 + 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      f4 v = acc[i][j];
      if (accumulate) v += *reinterpret_cast<const f4*>(out + 16 * i);
      *reinterpret_cast<f4*>(out + 16 * i) = v;
    }
  }
  if (do_rho) {
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      rs0 += __shfl_xor(rs0, o, 64);
      rs1 += __shfl_xor(rs1, o, 64);
    }
    if (lane < 16) {
      if (n < nr) {
        const int j = cell_rot[r0 + n];
        rho[j] = rs0 + (accumulate ? rho_a[j] : 0.0);
      }
      if (16 + n < nr) {
        const int j = cell_rot[r0 + 16 + n];
        rho[j] = rs1 + (accumulate ? rho_a[j] : 0.0);
      }
    }
  }
}

// ------------------------------------------------------------------ small pieces
// b_f = sum over the frame's entries of count * c[pixel], FP64; one wave per frame
__global__ __launch_bounds__(256) void nz_dot_kernel(const int64_t* __restrict__ nz_ptr, const uint32_t* __restrict__ nz,
                                                     int64_t n_frames, const double* __restrict__ cvec,
                                                     double* __restrict__ b) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;
  double acc = 0.0;
  for (int64_t e = nz_ptr[f] + lane; e < nz_ptr[f + 1]; e += 64) {
    const uint32_t v = nz[e];
    acc += (double)(v & 0xffffu) * cvec[v >> 16];
  }
  acc = wave_sum(acc);
  if (lane == 0) b[f] = acc;
}

// nz_off[f][t] = number of entries of frame f with pixel < t * 128, t = 0 .. ntab - 1
__global__ void nz_offsets_kernel(const int64_t* __restrict__ nz_ptr, const uint32_t* __restrict__ nz,
                                  int64_t n_frames, int ntab, int32_t* __restrict__ nz_off) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_frames * ntab) return;
  const int64_t f = e / ntab;
  const int t = (int)(e - f * ntab);
  const int64_t a = nz_ptr[f];
  int64_t lo = 0, hi = nz_ptr[f + 1] - a;  // first entry with pixel >= t * 128
  const uint32_t bound = (uint32_t)t * kBand;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((nz[a + mid] >> 16) < bound)
      lo = mid + 1;
    else
      hi = mid;
  }
  nz_off[e] = (int32_t)lo;
}

// groups of 32 rotations: count per cell
__global__ void cell_group_count_kernel(const int64_t* __restrict__ cell_ptr, int n_cells, int32_t* __restrict__ cnt) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_cells) return;
  const int64_t R = cell_ptr[c + 1] - cell_ptr[c];
  cnt[c] = (int32_t)((R + kGR - 1) / kGR);
}

// group table and storage sizes (Fp * 32 elements, Fp = frame list rounded up to 32)
__global__ void cell_group_fill_kernel(const int64_t* __restrict__ cell_ptr, const int64_t* __restrict__ cf_ptr,
                                       const int64_t* __restrict__ cg_ptr, int n_cells, int4* __restrict__ groups,
                                       int64_t* __restrict__ gsize) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_cells) return;
  const int64_t R = cell_ptr[c + 1] - cell_ptr[c];
  const int64_t F = cf_ptr[c + 1] - cf_ptr[c];
  const int64_t Fp = (F + kFB - 1) / kFB * kFB;
  for (int64_t g = cg_ptr[c], i = 0; g < cg_ptr[c + 1]; ++g, ++i) {
    const int64_t r = R - kGR * i;
    groups[g] = make_int4(c, (int)(cell_ptr[c] + kGR * i), (int)(r < kGR ? r : kGR), 0);
    gsize[g] = Fp * kGR;
  }
}

// Log-likelihood tile table: each group's tiles go to one XCD (dispatch is
// round-robin over the 8 XCDs, so slot 8 q + x runs on XCD x) -- the group's slices
// stay in that XCD's L2.  Groups are dealt to the least-loaded XCD; slots past a
// list's end are (-1, 0).  Single thread.
__global__ void group_tiles_kernel(const int4* __restrict__ groups, const int64_t* __restrict__ cg_ptr, int n_cells,
                                   const int64_t* __restrict__ cf_ptr, int32_t* __restrict__ xcd_of,
                                   int2* __restrict__ tiles, int64_t cap, int64_t* __restrict__ n_tiles_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t n_groups = cg_ptr[n_cells];
  int64_t len[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t g = 0; g < n_groups; ++g) {
    const int c = groups[g].x;
    const int64_t nt = (cf_ptr[c + 1] - cf_ptr[c] + kFT - 1) / kFT;
    int x = 0;
    for (int y = 1; y < 8; ++y) x = len[y] < len[x] ? y : x;
    xcd_of[g] = x;
    len[x] += nt;
  }
  int64_t q_max = 0;
  for (int x = 0; x < 8; ++x) q_max = len[x] > q_max ? len[x] : q_max;
  if (8 * q_max > cap) {  // only with repeated cells in a frame's list: reported, nothing written
    *n_tiles_out = -1;
    return;
  }
  int64_t q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t g = 0; g < n_groups; ++g) {
    const int c = groups[g].x;
    const int64_t nt = (cf_ptr[c + 1] - cf_ptr[c] + kFT - 1) / kFT;
    const int x = xcd_of[g];
    for (int64_t t = 0; t < nt; ++t) tiles[8 * (q[x]++) + x] = make_int2((int)g, (int)(t * kFT));
  }
  for (int x = 0; x < 8; ++x)
    for (; q[x] < q_max; ++q[x]) tiles[8 * q[x] + x] = make_int2(-1, 0);
  *n_tiles_out = 8 * q_max;
}

// recall_a = sum of the audited frame's full-search P over its proposed cells
constexpr int kAuditRot = 1024;
__global__ __launch_bounds__(256) void audit_recall_kernel(const __hip_bfloat16* __restrict__ P, int64_t ldp,
                                                           int n_rot, int64_t n_audit,
                                                           const uint32_t* __restrict__ mask_audit, int words,
                                                           const int32_t* __restrict__ cell_of,
                                                           double* __restrict__ recall) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t a = (int64_t)blockIdx.x * 64 + lane;
  if (a >= n_audit) return;
  const uint32_t* m = mask_audit + a * words;
  const int j0 = blockIdx.y * kAuditRot;
  const int j1 = j0 + kAuditRot < n_rot ? j0 + kAuditRot : n_rot;
  double rec = 0.0;
  for (int j = j0 + wave; j < j1; j += 4) {
    const int c = cell_of[j];
    if ((m[c >> 5] >> (c & 31)) & 1u) rec += (double)__bfloat162float(P[(int64_t)j * ldp + a]);
  }
  atomicAdd(recall + a, rec);
}

// ===================================================================== launchers
hipError_t launch_cand_loglik(const int2* tiles, int64_t n_tiles, const int4* groups, const int64_t* grp_off,
                              const int64_t* cf_ptr, const int32_t* cf_frame, const int64_t* nz_ptr,
                              const int32_t* nz_off, int ntab, const uint32_t* nz, const int32_t* cell_rot,
                              const void* hilo, int64_t plane, const float* scale, int64_t ps, float* G,
                              hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  cand_loglik_kernel<<<(unsigned)n_tiles, 256, 0, st>>>(tiles, groups, grp_off, cf_ptr, cf_frame, nz_ptr, nz_off,
                                                        ntab, nz, cell_rot, (const uint16_t*)hilo, plane, scale, ps,
                                                        G);
  return hipGetLastError();
}

hipError_t launch_cand_estep(const float* G, void* P, const int4* groups, const int64_t* grp_off,
                             const int64_t* cg_ptr, const int32_t* cells, const int32_t* pair_col, int k_top,
                             int64_t n_frames, const int32_t* cell_rot, const double* log_w, const double* S,
                             const double* b, double* L, hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  cand_estep_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(G, (uint16_t*)P, groups, grp_off, cg_ptr, cells,
                                                                    pair_col, k_top, n_frames, cell_rot, log_w, S, b,
                                                                    L);
  return hipGetLastError();
}

hipError_t launch_cand_mstep(const int4* groups, const int64_t* grp_off, int64_t n_groups, const int64_t* cf_ptr,
                             const int32_t* cf_frame, const int64_t* nz_ptr, const int32_t* nz_off, int ntab,
                             const uint32_t* nz, const void* P, const int32_t* cell_rot, int64_t ps, float* Wp,
                             double* rho, const double* rho_a, bool accumulate, hipStream_t st) {
  if (n_groups <= 0) return hipSuccess;
  const int nranges = (int)((ps + kRange - 1) / kRange);
  cand_mstep_kernel<<<(unsigned)(n_groups * nranges), 256, 0, st>>>(groups, grp_off, nranges, cf_ptr, cf_frame, nz_ptr,
                                                                    nz_off, ntab, nz, (const uint16_t*)P, cell_rot,
                                                                    ps, Wp, rho, rho_a, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_nz_dot(const int64_t* nz_ptr, const uint32_t* nz, int64_t n_frames, const double* c, double* b,
                         hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  nz_dot_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(nz_ptr, nz, n_frames, c, b);
  return hipGetLastError();
}

hipError_t launch_nz_offsets(const int64_t* nz_ptr, const uint32_t* nz, int64_t n_frames, int ntab, int32_t* nz_off,
                             hipStream_t st) {
  const int64_t n = n_frames * ntab;
  if (n <= 0) return hipSuccess;
  nz_offsets_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(nz_ptr, nz, n_frames, ntab, nz_off);
  return hipGetLastError();
}

hipError_t launch_cell_groups(const int64_t* cell_ptr, const int64_t* cf_ptr, int n_cells, int32_t* cnt,
                              int64_t* cg_ptr, int4* groups, int64_t* gsize, int64_t* grp_off, int64_t g_max,
                              hipStream_t st) {
  const unsigned nb = (unsigned)((n_cells + 255) / 256);
  cell_group_count_kernel<<<nb, 256, 0, st>>>(cell_ptr, n_cells, cnt);
  hipError_t e = launch_scan(cnt, n_cells, cg_ptr, st);
  if (e != hipSuccess) return e;
  // every group's size; sizes past the last group stay zero so the scan of g_max
  // entries gives the offsets of the real groups
  e = launch_fill_i32((int32_t*)gsize, 2 * g_max, 0, st);
  if (e != hipSuccess) return e;
  cell_group_fill_kernel<<<nb, 256, 0, st>>>(cell_ptr, cf_ptr, cg_ptr, n_cells, groups, gsize);
  return launch_scan64(gsize, g_max, grp_off, st);
}

hipError_t launch_group_tiles(const int4* groups, const int64_t* cg_ptr, int n_cells, const int64_t* cf_ptr,
                              int32_t* xcd_of, int2* tiles, int64_t cap, int64_t* n_tiles, hipStream_t st) {
  group_tiles_kernel<<<1, 64, 0, st>>>(groups, cg_ptr, n_cells, cf_ptr, xcd_of, tiles, cap, n_tiles);
  return hipGetLastError();
}

hipError_t launch_audit_recall(const void* P, int64_t ldp, int n_rot, int64_t n_audit, const uint32_t* mask_audit,
                               int words, const int32_t* cell_of, double* recall, hipStream_t st) {
  if (n_audit <= 0) return hipSuccess;
  const dim3 g((unsigned)((n_audit + 63) / 64), (unsigned)((n_rot + kAuditRot - 1) / kAuditRot));
  audit_recall_kernel<<<g, 256, 0, st>>>((const __hip_bfloat16*)P, ldp, n_rot, n_audit, mask_audit, words, cell_of,
                                         recall);
  return hipGetLastError();
}

}  // namespace emc
