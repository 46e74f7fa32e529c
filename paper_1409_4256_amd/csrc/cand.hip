// Candidate (learned-proposal) E- and M-steps as pack-major MFMA contractions.
//
// Neighbouring coarse cells are gathered into packs (proposal.hip); a pack's fine
// rotations are split into groups of at most 32, and the frames that propose any
// of its cells form its frame list (each frame once, with a bitmask of the cells
// it proposes).  For every group the log-likelihoods of all (rotation, listed
// frame) pairs are one small dense product
//     G[frame][r] = scale_r * sum_i (hi_ri + lo_ri) K_i,frame          (eq. 2.4's Q)
// and, after each frame's E-step over its own candidates (the rotations of the
// cells it proposes; the group's other pairs get P = 0), the M-step of the group is
//     W'_r,i = sum_frames P[r][frame] K_i,frame                         (eq. 2.11)
// Frames are stored sparsely, band-blocked: for every 128-pixel band a frame's
// non-zero pixels are 16-bit words (pixel in band << 9 | count) packed in 16-byte
// chunks of 8 (the last one padded with count-0 words at a pixel of the band
// without photons, so that expanding a word never needs a test).  Bands come in runs of 8 (1024
// pixels, the M-step's pixel range); inside a run a frame's chunks of the 8 bands
// are contiguous, frame after frame (run 0 of every frame, then run 1, ...).  A
// lane that streams one frame band after band thus reads whole cache lines of its
// own frame, whichever other frames a pack's list holds, and an M-step workgroup's
// four waves read the same lines.  A 16-byte record per (frame, run), frame-major,
// locates the chunks: the run's first chunk (absolute index), the offsets of its
// bands' first chunks (one byte each) and its chunk count -- one load per frame
// and run instead of a table entry per band.  Each workgroup expands the frames it needs into LDS band by
// band and feeds the dense band to v_mfma_f32_16x16x32_bf16; the next band's
// chunks are loaded while the current band's MFMAs run.  A band's LDS rows are
// owned by one wave (it writes, reads and clears them), so the band loops need no
// barrier.
//
// Storage of a group with frame list length F (Fp = F rounded up to 32):
//   G  float [Fp][32]            frame-major: a frame's 32 values are contiguous
//   P  bf16  [Fp/32][32][32]     blocks of 32 frames, rotation-major inside a block,
//                                which is the MFMA operand layout of the M-step.
#include "emc_device.h"
#include "lse.h"

namespace emc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

constexpr int kGR = 32;             // rotations per group (two 16-row MFMA tiles)
static_assert(kPackRot <= kGR, "a pack of cells fits one group");
constexpr int kFT = 64;             // frames per log-likelihood wave (four 16-column tiles)
constexpr int kTileF = 4 * kFT;     // frames per log-likelihood workgroup (tile)
constexpr int kBand = 128;          // pixels per band (granularity of the entry-offset table)
constexpr int kLRow = kBand + 8;    // LDS row of one frame's band, bf16 (272 bytes; 288, which spreads the
                                     // MFMA operand reads over all banks, measured the same)
constexpr int kFB = 32;             // frames per M-step block (one MFMA reduction step)
constexpr int kKRow = kFB + 8;      // LDS row of one pixel's frames, bf16 (80 bytes)

__device__ __forceinline__ uint16_t count_bf16(uint32_t e) {
  // counts up to 256 are exact in BF16: the upper half of the FP32 pattern
  return (uint16_t)(__float_as_uint((float)(e & 0xffffu)) >> 16);
}

constexpr int kRun = 8;             // bands per run of the chunk layout (the M-step's 1024-pixel range)

// Chunks [x, y) of band i (0..kRun-1) of a run record {first chunk, offsets of
// bands 0-3, offsets of bands 4-7 (bytes, ascending), chunks in the run}; bands
// past a short last run have offset = chunk count (empty).
__device__ __forceinline__ int2 run_band(u4 rec, int i) {
  const uint32_t lo = i < 4 ? rec.y : rec.z, hi = i + 1 < 4 ? rec.y : rec.z;
  const int x = (int)((lo >> (8 * (i & 3))) & 0xffu);
  const int y = i + 1 < kRun ? (int)((hi >> (8 * ((i + 1) & 3))) & 0xffu) : (int)rec.w;
  return make_int2((int)rec.x + x, (int)rec.x + y);
}

// The M-step streams each chunk once: non-temporal loads keep the stream from
// evicting the responsibilities its workgroups share in L2 (measured faster there;
// the log-likelihood's chunk loads are faster as ordinary loads).
template <bool NT>
__device__ __forceinline__ u4 load_chunk(const u4* __restrict__ p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
constexpr int kWin = 2;              // chunks per band held in registers (16 pixels)

// Writes (CLEAR = false) or zeroes one chunk's pixels: word e goes to
// base[(e >> 9) * stride] as the BF16 count (e & 511).  No word needs a test: a
// chunk's padding words carry count 0 at a pixel whose count is 0, and the
// callers' filler chunks either come before every real word of the band (count 0
// anywhere) or repeat a real chunk (the same values again).
template <bool CLEAR>
__device__ __forceinline__ void put_chunk(uint16_t* base, int stride, u4 ch) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t e = h ? (ch[u] >> 16) : (ch[u] & 0xffffu);
      base[(int)(e >> 9) * stride] = CLEAR ? (uint16_t)0 : count_bf16(e & 511u);
    }
  }
}

// chunks first, first + 1, ... < c1 of a band beyond the register window, loaded
// four at a time; slots past c1 repeat chunk c1 - 1
template <bool CLEAR, bool NT>
__device__ __forceinline__ void put_rest(uint16_t* base, int stride, const u4* __restrict__ src, int first, int c1) {
  for (int c = first; c < c1; c += 4) {
    u4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = load_chunk<NT>(src + (c + u < c1 ? c + u : c1 - 1));
#pragma unroll
    for (int u = 0; u < 4; ++u) put_chunk<CLEAR>(base, stride, v[u]);
  }
}

// ------------------------------------------------------------------ log-likelihood
// One workgroup per tile (group g, frames [f0, f0 + 256) of its pack's list).  Wave w
// owns frames f0 + 64 w .. + 63 (lane s expands frame s) over every band and both
// rotation tiles, so the four waves read the same slice rows at about the same
// time (one fetch from L2 serves the workgroup) and each wave writes its own
// frames' G; there is no barrier, and waves without frames leave at once.  TWO:
// the group has a second rotation tile (more than 16 rotations); the kernel picks
// the variant once per workgroup, so the MFMA sequence has no branch.  Per 32-pixel
// step the wave reads its four B fragments together and issues the hi products of
// every accumulator before the lo ones, so no MFMA waits on the one before it.
template <bool TWO>
__device__ __forceinline__ void cand_loglik_tile(
    uint16_t* __restrict__ lds, const int2 tl, const int4* __restrict__ groups, const int64_t* __restrict__ grp_off,
    const int64_t* __restrict__ cf_ptr, const int32_t* __restrict__ cf_frame, const u4* __restrict__ runs,
    const u4* __restrict__ fb, const int32_t* __restrict__ cell_rot, const uint16_t* __restrict__ hi,
    int64_t plane, const float* __restrict__ scale, int64_t ps, float* __restrict__ G) {
  constexpr int NT = TWO ? 2 : 1;  // rotation tiles
  const int4 gr = groups[tl.x];
  const int c = gr.x, r0 = gr.y, nr = gr.z;
  const int64_t F = cf_ptr[c + 1] - cf_ptr[c];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int f0 = tl.y + wave * kFT;
  if (f0 >= F) return;  // uniform per wave
  const int nf = (int)(F - f0 < kFT ? F - f0 : kFT);

  const int nbands = (int)(ps / kBand), n_runs = (nbands + kRun - 1) / kRun;
  // this lane's frame (slot = lane) and its run records
  const bool has = lane < nf;
  const int32_t fidx = has ? cf_frame[cf_ptr[c] + f0 + lane] : 0;
  const u4* rec_of = runs + (int64_t)fidx * n_runs;
  // rows of the A operand: rotation (lane & 15) of each 16-row tile; rows past the
  // group read its last rotation again (their sums are multiplied by a zero scale)
  const int m = lane & 15, kq = 8 * (lane >> 4);
  const int64_t ar0 = (int64_t)cell_rot[r0 + (m < nr ? m : nr - 1)] * ps;
  const int64_t ar1 = TWO ? (int64_t)cell_rot[r0 + (16 + m < nr ? 16 + m : nr - 1)] * ps : 0;

  uint16_t* rows = lds + wave * kFT * kLRow;
  uint16_t* frow = rows + lane * kLRow;
  for (int e = lane; e < kFT * kLRow / 8; e += 64) reinterpret_cast<u4*>(rows)[e] = u4{0u, 0u, 0u, 0u};

  f4 acc[NT][4];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const u4 zero = {0u, 0u, 0u, 0u};
  // window slots past a band's chunks hold zero chunks (count 0 at the row's first
  // pixel), written before the band's real chunks
  // pipeline: chunks of the current band in registers, the next band's chunk range;
  // the records of the current run and the next one (loaded on entering a run)
  u4 rc = zero, rcn = zero;
  if (has) {
    rc = rec_of[0];
    if (n_runs > 1) rcn = rec_of[1];
  }
  int2 r0c = {0, 0}, r1c = {0, 0};
  if (has) r0c = run_band(rc, 0);
  u4 w0[kWin];
#pragma unroll
  for (int u = 0; u < kWin; ++u) w0[u] = r0c.x + u < r0c.y ? load_chunk<false>(fb + r0c.x + u) : zero;
  if (has && 1 < nbands) r1c = run_band(rc, 1);
  // A fragments (slice rows, hi and lo, of each row tile) of a band, 4 k-steps
  auto load_a = [&](int band, u4 (&h)[4][NT], u4 (&l)[4][NT]) {
    const int64_t kb = (int64_t)(band < nbands ? band : nbands - 1) * kBand + kq;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t ar = t ? ar1 : ar0;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        h[kk][t] = *reinterpret_cast<const u4*>(hi + ar + kb + 32 * kk);
        l[kk][t] = *reinterpret_cast<const u4*>(hi + plane + ar + kb + 32 * kk);
      }
    }
  };
  u4 ah[4][NT], al[4][NT];
  load_a(0, ah, al);
  for (int band = 0; band < nbands; ++band) {
    // prefetch (issued before this band's data is waited on; loads complete in issue
    // order): the next band's chunks and the table entry of the band after; the next
    // band's A fragments are loaded into the same registers once this band's MFMAs
    // have been issued
    u4 w1[kWin];
#pragma unroll
    for (int u = 0; u < kWin; ++u) w1[u] = r1c.x + u < r1c.y ? load_chunk<false>(fb + r1c.x + u) : zero;
    if (band > 0 && band % kRun == 0) {  // entering run band / kRun (uniform)
      rc = rcn;
      rcn = has && band / kRun + 1 < n_runs ? rec_of[band / kRun + 1] : zero;
    }
    int2 r2c = {0, 0};
    if (has && band + 2 < nbands) r2c = run_band((band + 2) / kRun == band / kRun ? rc : rcn, (band + 2) % kRun);
    // window chunks past the first only when some lane of the wave has them (most
    // bands hold at most 8 photon pixels per frame)
    const bool more = __ballot(r0c.y - r0c.x > 1) != 0;
    if (has) {
      if (more) {  // the window's later slots first: zero fillers precede the real words
#pragma unroll
        for (int u = kWin - 1; u >= 1; --u) put_chunk<false>(frow, 1, w0[u]);
      }
      put_chunk<false>(frow, 1, w0[0]);
      if (more) put_rest<false, false>(frow, 1, fb, r0c.x + kWin, r0c.y);
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      bf8 bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = *reinterpret_cast<const bf8*>(&rows[(16 * j + m) * kLRow + 32 * kk + kq]);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[kk][t]), bv[j], acc[t][j], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, al[kk][t]), bv[j], acc[t][j], 0, 0, 0);
    }
    // clear what this lane wrote: the words of its register window, or its whole row
    // when the band held more chunks than the window (the wave's LDS operations run
    // in order, so the MFMA operand reads above are done)
    if (has) {
      if (r0c.y - r0c.x <= kWin) {
        put_chunk<true>(frow, 1, w0[0]);
        if (more) {
#pragma unroll
          for (int u = 1; u < kWin; ++u) put_chunk<true>(frow, 1, w0[u]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < kLRow / 8; ++e) reinterpret_cast<u4*>(frow)[e] = zero;
      }
    }
    load_a(band + 1, ah, al);
#pragma unroll
    for (int u = 0; u < kWin; ++u) w0[u] = w1[u];
    r0c = r1c;
    r1c = r2c;
  }

  // G[frame][rotation] = scale_r * sum: lane holds frame 16 j + m, rotations
  // 16 i + 4 (lane >> 4) + 0..3 of tile (i, j)
  float* out = G + grp_off[tl.x] + (int64_t)f0 * kGR;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int rb = 16 * i + 4 * (lane >> 4);
    f4 sc;
#pragma unroll
    for (int u = 0; u < 4; ++u) sc[u] = rb + u < nr ? scale[cell_rot[r0 + rb + u]] : 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (16 * j + m < nf) *reinterpret_cast<f4*>(out + (16 * j + m) * kGR + rb) = sc * acc[i][j];
  }
}

__global__ __launch_bounds__(256, 2) void cand_loglik_kernel(
    const int2* __restrict__ tiles, const int4* __restrict__ groups, const int64_t* __restrict__ grp_off,
    const int64_t* __restrict__ cf_ptr, const int32_t* __restrict__ cf_frame, const u4* __restrict__ runs,
    const u4* __restrict__ fb, const int32_t* __restrict__ cell_rot, const uint16_t* __restrict__ hi,
    int64_t plane, const float* __restrict__ scale, int64_t ps, float* __restrict__ G) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[4 * kFT * kLRow];  // 69632 bytes
  const int2 tl = tiles[blockIdx.x];
  if (tl.x < 0) return;  // padding tile (uniform)
  if (groups[tl.x].z > 16)
    cand_loglik_tile<true>(lds, tl, groups, grp_off, cf_ptr, cf_frame, runs, fb, cell_rot, hi, plane, scale, ps, G);
  else
    cand_loglik_tile<false>(lds, tl, groups, grp_off, cf_ptr, cf_frame, runs, fb, cell_rot, hi, plane, scale, ps, G);
}

// ------------------------------------------------------------------ E-step
// The log-evidence does not evaluate a term more than kLseDrop below the running
// maximum (below e^-64 of it: the frame's candidates together stay far below the
// FP64 rounding of the sum).  Responsibilities keep every term; a - L is formed in
// FP64 and its exponential evaluated in FP32 (P is stored in BF16), skipped only
// below -110, where its FP32 value is 0.

// The rotation term of a, log w_j - S_j, in the packs' rotation order (entry t
// belongs to rotation pack_rot[t]), so that a group's terms are contiguous.
__global__ void cell_const_kernel(const int32_t* __restrict__ cell_rot, int64_t n_rot,
                                  const double* __restrict__ log_w, const double* __restrict__ S,
                                  double* __restrict__ cst) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_rot) return;
  const int j = cell_rot[t];
  cst[t] = log_w[j] - S[j];
}

// A frame's G row of a group (32 floats, 128-byte aligned), rotations < nr loaded
__device__ __forceinline__ void load_grow(const float* __restrict__ row, int nr, f4 (&v)[kGR / 4]) {
#pragma unroll
  for (int q = 0; q < kGR / 4; ++q)
    v[q] = 4 * q < nr ? *reinterpret_cast<const f4*>(row + 4 * q) : f4{0.f, 0.f, 0.f, 0.f};
}

// Log-evidence of each candidate frame: one wave per frame, lanes take the frame's
// proposed cells (slot t = lane + 64 u); a = Q + log w_j = G + b_f - S_j + log w_j
// and L_f = log sum over the frame's candidates of e^a, in FP64 (eq. 2.4's
// denominator).  A cell's values sit in its pack's groups, at the frame's column
// of the pack's list, over the cell's own rotations [cell_first, + its count).
__global__ __launch_bounds__(256) void cand_estep_kernel(
    const float* __restrict__ G, const int4* __restrict__ groups, const int64_t* __restrict__ grp_off,
    const int64_t* __restrict__ cg_ptr, const int32_t* __restrict__ cells, const int32_t* __restrict__ pair_col,
    int k_top, int64_t n_frames, const int32_t* __restrict__ pack_of, const int32_t* __restrict__ cell_first,
    const int64_t* __restrict__ cell_ptr, const double* __restrict__ cst, const double* __restrict__ b,
    double* __restrict__ L) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;  // uniform per wave
  const double bk = b[f];
  double mx = -INFINITY, sum = 0.0;
  const ExpCoef ec = exp_coef();
  for (int t = lane; t < k_top; t += 64) {
    const int c = cells[f * k_top + t];
    if (c < 0) continue;
    const int p = pack_of[c];
    const int lo = cell_first[c], hi = lo + (int)(cell_ptr[c + 1] - cell_ptr[c]);
    const int64_t col = pair_col[f * k_top + t];
    for (int64_t g = cg_ptr[p]; g < cg_ptr[p + 1]; ++g) {
      const int4 gr = groups[g];
      const int a = (lo > gr.y ? lo : gr.y) - gr.y, z = (hi < gr.y + gr.z ? hi : gr.y + gr.z) - gr.y;
      if (a >= z) continue;
      f4 v[kGR / 4];
      load_grow(G + grp_off[g] + col * kGR, gr.z, v);
      const double* cr = cst + gr.y;
#pragma unroll
      for (int q = 0; q < kGR / 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (4 * q + u >= a && 4 * q + u < z) lse_push(mx, sum, ((double)v[q][u] + bk) + cr[4 * q + u], ec);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lse_merge(mx, sum, __shfl_xor(mx, o, 64), __shfl_xor(sum, o, 64));
  }
  if (lane == 0) L[f] = mx + log(sum);
}

// Responsibilities of the group's (rotation, listed frame) pairs, group-major over
// the log-likelihood's tiles (group g, list positions f0 .. f0 + 255; wave w, lane
// s: position f0 + 64 w + s): P = exp(a - L_f) in BF16 (eq. 2.4) for a rotation
// whose cell the frame proposes, 0 for the pack's other cells, into the group's
// blocked P, where 32 consecutive lanes fill one 64-byte row of a [32 rot][32
// frames] block, and, with Pd, the proposed pairs into the dense [rotation][frame]
// matrix of the M-step's dense bands (a list's frames come in runs of consecutive
// numbers).
__global__ __launch_bounds__(256) void cand_pwrite_kernel(
    const int2* __restrict__ tiles, const int4* __restrict__ groups, const int64_t* __restrict__ grp_off,
    const int64_t* __restrict__ cf_ptr, const int32_t* __restrict__ cf_frame, const uint32_t* __restrict__ cf_mask,
    const float* __restrict__ G, const int32_t* __restrict__ pack_rot, const int32_t* __restrict__ rot_local,
    const double* __restrict__ cst, const double* __restrict__ b, const double* __restrict__ L,
    uint16_t* __restrict__ P, uint16_t* __restrict__ Pd, int64_t ldd) {
  const int2 tl = tiles[blockIdx.x];
  if (tl.x < 0) return;  // padding tile (uniform)
  const int4 gr = groups[tl.x];
  const int64_t F = cf_ptr[gr.x + 1] - cf_ptr[gr.x];
  const int64_t col = tl.y + (threadIdx.x >> 6) * 64 + (threadIdx.x & 63);
  if (col >= F) return;
  const int32_t f = cf_frame[cf_ptr[gr.x] + col];
  const uint32_t listed = cf_mask[cf_ptr[gr.x] + col];
  const double bk = b[f], lse = L[f];
  f4 v[kGR / 4];
  load_grow(G + grp_off[tl.x] + col * kGR, gr.z, v);
  const double* cr = cst + gr.y;
  uint16_t* pb = P + grp_off[tl.x] + (col >> 5) * (kGR * kFB) + (col & 31);
#pragma unroll
  for (int q = 0; q < kGR / 4; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 4 * q + u;
      if (r >= gr.z) break;  // uniform: one group per workgroup
      if ((listed >> rot_local[gr.y + r]) & 1u) {
        const float x = (float)((((double)v[q][u] + bk) + cr[r]) - lse);
        const uint16_t p = x > -110.0f ? __builtin_bit_cast(uint16_t, __float2bfloat16(expf(x))) : 0;
        pb[r * kFB] = p;
        if (Pd) Pd[(int64_t)pack_rot[gr.y + r] * ldd + f] = p;
      } else {
        pb[r * kFB] = 0;
      }
    }
}

// ------------------------------------------------------------------ M-step
// One workgroup per (group g, 1024-pixel range); it runs over the whole frame list
// of the group's pack in blocks of 32 frames.  Wave w owns the range's band pair
// w (256 pixels): it expands the block's frames there into LDS rows [pixel][frame]
// (lanes s and s + 32 take the two bands of frame s), contracts them with the
// block's P (B operand, read straight from its blocked layout) and clears the
// rows.  The next block's P and chunks, the chunk ranges of the block after and
// the frame indices of the one after that are loaded while the current block's
// MFMAs run.  Dense bands (the detector centre, where every frame has photons)
// are skipped: their W' columns are one dense product over the whole frame set.  W' rows are written (accumulate: added to what the audited frames'
// dense product left there); the range-0 workgroup also sums rho = sum P.
constexpr int kPair = 2 * kBand;    // pixels per wave in the M-step
static_assert(4 * kPair == kRun * kBand, "an M-step workgroup's pixel range is one run of the chunk layout");
// TWO: the group has a second rotation tile (picked once per workgroup, so the MFMA
// sequence has no branch); the A fragments of a block are read from LDS in batches
// and each feeds MFMAs on independent accumulators.
template <bool TWO>
__device__ __forceinline__ void cand_mstep_range(
    uint16_t* __restrict__ lds, int64_t g, int pr, const int4* __restrict__ groups,
    const int64_t* __restrict__ grp_off, const int64_t* __restrict__ cf_ptr, const int32_t* __restrict__ cf_frame,
    const u4* __restrict__ runs, int64_t n_list, const u4* __restrict__ fb, const int32_t* __restrict__ dense_band,
    const uint16_t* __restrict__ P, const int32_t* __restrict__ cell_rot, int64_t ps, float* __restrict__ Wp,
    double* __restrict__ rho, const double* __restrict__ rho_a, int accumulate) {
  constexpr int NT = TWO ? 2 : 1;        // rotation tiles
  constexpr int NB = TWO ? 4 : 8;        // A fragments read per batch
  const int4 gr = groups[g];
  const int c = gr.x, r0 = gr.y, nr = gr.z;
  const int64_t F = cf_ptr[c + 1] - cf_ptr[c];
  const int32_t* cf = cf_frame + cf_ptr[c];
  const uint16_t* Pg = P + grp_off[g];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbands = (int)(ps / kBand);
  const int band = 2 * (pr * 4 + wave);  // first band of this wave's pair
  const int p0 = band * kBand;
  if (band >= nbands) return;  // no band for this wave (no barrier follows)
  const bool do_rho = pr == 0 && wave == 0;
  const int n = lane & 15, kq = 8 * (lane >> 4);
  const int slot = lane & 31, par = lane >> 5;

  uint16_t* rows = lds + wave * kPair * kKRow;
  uint16_t* fcol = rows + slot;
  for (int e = lane; e < kPair * kKRow / 8; e += 64) reinterpret_cast<u4*>(rows)[e] = u4{0u, 0u, 0u, 0u};

  f4 acc[16][NT];
#pragma unroll
  for (int i = 0; i < 16; ++i)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[i][t] = f4{0.f, 0.f, 0.f, 0.f};
  double rs0 = 0.0, rs1 = 0.0;
  const u4 zero = {0u, 0u, 0u, 0u};
  constexpr int kNext = kBand * kKRow;  // LDS offset of the pair's second band

  // this lane's band of the pair (band 2 w + par of run pr, the workgroup's pixel
  // range) and its LDS rows; a dense band's rows stay zero here (its pixels come
  // from the dense product).  Records of run pr, run-major copy.
  const int n_runs = (nbands + kRun - 1) / kRun, bi = band + par - pr * kRun;
  const u4* run_pr = runs + (int64_t)n_list * n_runs + (int64_t)pr * n_list;
  const bool sparse = dense_band[band + par] < 0;
  uint16_t* fcol_b = fcol + par * kNext;
  // window slots past a band's chunks hold filler chunks of count-0 words at pixel
  // row `slot` (a different bank for each lane), written before the real chunks
  const uint32_t fw = (uint32_t)slot << 9;
  const u4 fill = {fw | fw << 16, fw | fw << 16, fw | fw << 16, fw | fw << 16};
  // a frame's record (a zero record: no chunks); decoded one block after its load
  auto record_of = [&](int32_t fr) -> u4 { return fr < 0 || !sparse ? u4{0u, 0u, 0u, 0u} : run_pr[fr]; };
  auto frame_at = [&](int64_t f0) -> int32_t { return f0 + slot < F ? cf[f0 + slot] : -1; };
  // B operand of a block: frames kq..kq+7 for rotation n (and n + 16)
  auto load_p = [&](int64_t f0, u4& x0, u4& x1) {
    const uint16_t* pblk = Pg + (f0 >> 5) * (kGR * kFB);
    x0 = f0 < F ? *reinterpret_cast<const u4*>(pblk + n * kFB + kq) : zero;
    x1 = TWO && f0 < F ? *reinterpret_cast<const u4*>(pblk + (16 + n) * kFB + kq) : zero;
  };
  // pipeline stages: block k (P in b0/b1, chunks in w0), k + 1 (record e1), k + 2 (frame fr2)
  int2 q0 = run_band(record_of(frame_at(0)), bi);
  const int32_t fr1 = frame_at(kFB);
  int32_t fr2 = frame_at(2 * kFB);
  u4 w0[kWin];
#pragma unroll
  for (int u = 0; u < kWin; ++u) w0[u] = q0.x + u < q0.y ? load_chunk<true>(fb + q0.x + u) : fill;
  u4 e1 = record_of(fr1);
  u4 b0, b1;
  load_p(0, b0, b1);

  for (int64_t f0 = 0; f0 < F; f0 += kFB) {
    const int nf = (int)(F - f0 < kFB ? F - f0 : kFB);
    // prefetch (loads complete in issue order, so this block's data, loaded one
    // block ago, is waited on without waiting for these)
    u4 b0n, b1n;
    load_p(f0 + kFB, b0n, b1n);
    const int2 q1 = run_band(e1, bi);
    u4 w1[kWin];
#pragma unroll
    for (int u = 0; u < kWin; ++u) w1[u] = q1.x + u < q1.y ? load_chunk<true>(fb + q1.x + u) : fill;
    const u4 e2 = record_of(fr2);
    const int32_t fr3 = frame_at(f0 + 3 * kFB);
#pragma unroll
    for (int u = kWin - 1; u >= 0; --u) put_chunk<false>(fcol_b, kKRow, w0[u]);  // fillers before real words
    put_rest<false, true>(fcol_b, kKRow, fb, q0.x + kWin, q0.y);
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
    for (int h = 0; h < 16; h += NB) {
      bf8 av[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) av[i] = *reinterpret_cast<const bf8*>(&rows[(16 * (h + i) + n) * kKRow + kq]);
#pragma unroll
      for (int i = 0; i < NB; ++i)
        acc[h + i][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], __builtin_bit_cast(bf8, b0), acc[h + i][0], 0, 0, 0);
      if constexpr (TWO) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
          acc[h + i][NT - 1] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], __builtin_bit_cast(bf8, b1), acc[h + i][NT - 1], 0, 0, 0);
      }
    }
    // clear the rows: when every lane's band fit its register window, only the words
    // written (the wave's LDS operations run in order, so the reads above are done);
    // otherwise all of them with contiguous 16-byte stores
    if (__ballot(q0.y - q0.x > kWin) == 0) {
#pragma unroll
      for (int u = 0; u < kWin; ++u) put_chunk<true>(fcol_b, kKRow, w0[u]);
    } else {
      for (int e = lane; e < kPair * kKRow / 8; e += 64) reinterpret_cast<u4*>(rows)[e] = zero;
    }
    b0 = b0n;
    b1 = b1n;
    q0 = q1;
    e1 = e2;
#pragma unroll
    for (int u = 0; u < kWin; ++u) w0[u] = w1[u];
    fr2 = fr3;
  }

  // acc[i][j][r] = W'[rotation 16 j + n][pixel p0 + 16 i + 4 (lane >> 4) + r]
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int mr = 16 * j + n;
    if (mr >= nr) continue;
    float* out = Wp + (int64_t)cell_rot[r0 + mr] * ps + p0 + 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
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

__global__ __launch_bounds__(256, 2) void cand_mstep_kernel(
    const int4* __restrict__ groups, const int64_t* __restrict__ grp_off, int64_t n_groups, int nranges,
    const int64_t* __restrict__ cf_ptr, const int32_t* __restrict__ cf_frame, const u4* __restrict__ runs,
    int64_t n_list, const u4* __restrict__ fb, const int32_t* __restrict__ dense_band, const uint16_t* __restrict__ P,
    const int32_t* __restrict__ cell_rot, int64_t ps, float* __restrict__ Wp, double* __restrict__ rho,
    const double* __restrict__ rho_a, int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[4 * kPair * kKRow];  // 81920 bytes
  // workgroup 8 q + x (dispatch is round-robin over the 8 XCDs: it runs on XCD x)
  // takes range q mod nranges of group 8 (q / nranges) + x, so a group's ranges run
  // one after another on one XCD and share its P in that XCD's L2
  const int64_t q = blockIdx.x >> 3;
  const int64_t g = 8 * (q / nranges) + (blockIdx.x & 7);
  const int pr = (int)(q % nranges);
  if (g >= n_groups) return;  // padding of the group count to a multiple of 8 (uniform)
  if (groups[g].z > 16)
    cand_mstep_range<true>(lds, g, pr, groups, grp_off, cf_ptr, cf_frame, runs, n_list, fb, dense_band, P, cell_rot,
                           ps, Wp, rho, rho_a, accumulate);
  else
    cand_mstep_range<false>(lds, g, pr, groups, grp_off, cf_ptr, cf_frame, runs, n_list, fb, dense_band, P, cell_rot,
                            ps, Wp, rho, rho_a, accumulate);
}

// ------------------------------------------------------------------ band-blocked frames

// Position of (band b, frame f) in the chunk order: runs of kRun bands, frame-major
// inside a run (the last run may hold fewer bands).
__device__ __forceinline__ int64_t band_slot(int b, int64_t f, int64_t n_frames, int nb) {
  const int r0 = b - b % kRun;
  const int q = nb - r0 < kRun ? nb - r0 : kRun;
  return (int64_t)r0 * n_frames + f * q + (b - r0);
}

// Chunks of every (band, listed frame) in the chunk order: cnt[band_slot(b, f)]
// (one wave per frame, two pixels per lane per band); counts above 256 (not exact
// in BF16) set *over.
__global__ __launch_bounds__(256) void band_count_kernel(const uint16_t* __restrict__ counts,
                                                         const uint8_t* __restrict__ mask, int n_pix,
                                                         const int32_t* __restrict__ frames, int64_t n_frames, int nb,
                                                         int32_t* __restrict__ cnt, int32_t* __restrict__ over) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;  // uniform per wave
  const uint16_t* row = counts + (int64_t)frames[f] * n_pix;
  bool big = false;
  for (int b = 0; b < nb; ++b) {
    int n = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = b * kBand + 64 * h + lane;
      const uint32_t v = i < n_pix && mask[i] ? row[i] : 0u;
      big |= v > 256u;
      n += __popcll(__ballot(v != 0u));
    }
    if (lane == 0) cnt[band_slot(b, f, n_frames, nb)] = (n + 7) >> 3;
  }
  if (__ballot(big) != 0ull && lane == 0) atomicOr(over, 1);
}

// Run records from the chunk offsets ptr (exclusive scan of the counts in band_slot
// order; a run's bands are consecutive there): runs[f * n_runs + r] (frame-major,
// for kernels that stream one frame per lane) and the run-major copy
// runs[n_frames * n_runs + r * n_frames + f] (for the M-step, whose workgroup reads
// one run of many frames)
__global__ void run_table_kernel(const int64_t* __restrict__ ptr, int64_t n_frames, int nb, u4* __restrict__ runs) {
  const int n_runs = (nb + kRun - 1) / kRun;
  const int64_t n = n_frames * n_runs;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t f = e / n_runs;
    const int b0 = (int)(e - f * n_runs) * kRun;
    const int q = nb - b0 < kRun ? nb - b0 : kRun;
    const int64_t s = band_slot(b0, f, n_frames, nb);
    const int64_t first = ptr[s];
    const uint32_t total = (uint32_t)(ptr[s + q] - first);
    uint32_t off[kRun];
#pragma unroll
    for (int i = 0; i < kRun; ++i) off[i] = i < q ? (uint32_t)(ptr[s + i] - first) : total;
    const u4 rec = {(uint32_t)first, off[0] | off[1] << 8 | off[2] << 16 | off[3] << 24,
                    off[4] | off[5] << 8 | off[6] << 16 | off[7] << 24, total};
    runs[e] = rec;
    runs[n + (e - f * n_runs) * n_frames + f] = rec;
  }
}

// Fill: words (pixel in band << 9 | count) in pixel order, chunk tails padded
// with count 0 at the band's first pixel without photons
__global__ __launch_bounds__(256) void band_fill_kernel(const uint16_t* __restrict__ counts,
                                                        const uint8_t* __restrict__ mask, int n_pix,
                                                        const int32_t* __restrict__ frames, int64_t n_frames, int nb,
                                                        const u4* __restrict__ runs, uint16_t* __restrict__ words) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;
  const uint16_t* row = counts + (int64_t)frames[f] * n_pix;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int n_runs = (nb + kRun - 1) / kRun;
  u4 rec = {0u, 0u, 0u, 0u};
  for (int b = 0; b < nb; ++b) {
    if (b % kRun == 0) rec = runs[f * n_runs + b / kRun];
    const int2 r = run_band(rec, b % kRun);
    if (r.x == r.y) continue;  // uniform: empty band
    uint16_t* out = words + (int64_t)r.x * 8;
    int n = 0;
    unsigned long long bal0 = 0, bal1 = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = b * kBand + 64 * h + lane;
      const uint32_t v = i < n_pix && mask[i] ? row[i] : 0u;
      const unsigned long long bal = __ballot(v != 0u);
      if (v != 0u) out[n + __popcll(bal & below)] = (uint16_t)(((uint32_t)(64 * h + lane) << 9) | v);
      n += __popcll(bal);
      (h ? bal1 : bal0) = bal;
    }
    // padding words: count 0 at the band's first pixel without photons (one exists:
    // a band of 128 counted pixels fills its 16 chunks exactly)
    const unsigned long long z0 = ~bal0, z1 = ~bal1;
    const int zp = z0 ? __builtin_ctzll(z0) : (z1 ? 64 + __builtin_ctzll(z1) : 0);
    for (int t = n + lane; t < 8 * (r.y - r.x); t += 64) out[t] = (uint16_t)(zp << 9);
  }
}

// b_f = sum over the frame's pixels of count * c[pixel], FP64.  One workgroup per
// 64 consecutive frames, lane = frame, so a band's table entries and chunks are read
// contiguously and a dense band keeps every lane busy; wave w takes bands w, w + 4,
// ..., and the four partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void band_dot_kernel(const u4* __restrict__ runs, int nb,
                                                       const u4* __restrict__ chunks, int64_t n_frames,
                                                       const double* __restrict__ cvec, double* __restrict__ b) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t f = (int64_t)blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (f < n_frames) {
    for (int band = wave; band < nb; band += 4) {
      const int2 r = run_band(runs[f * ((nb + kRun - 1) / kRun) + band / kRun], band % kRun);
      const double* cb = cvec + band * kBand;
      for (int ch = r.x; ch < r.y; ++ch) {
        const u4 w = chunks[ch];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const uint32_t e = h ? (w[u] >> 16) : (w[u] & 0xffffu);
            acc += (double)(e & 511u) * cb[e >> 9];  // padding words: count 0
          }
        }
      }
    }
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && f < n_frames) b[f] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// Dense bands: band b is dense when its frames average at least kDenseChunks
// chunks; dense_band[b] = its index among the dense bands (ascending b, at most
// kMaxDense) or -1, dense_list[d] = band of dense index d, *n_dense.  One
// workgroup per band sums the chunk counts, then one thread assigns the indices.
constexpr int kDenseChunks = 3;
constexpr int kMaxDense = 16;
__global__ __launch_bounds__(256) void band_mean_kernel(const int32_t* __restrict__ cnt, int64_t n_frames, int nb,
                                                        float* __restrict__ mean) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int64_t f = threadIdx.x; f < n_frames; f += 256) s += cnt[band_slot(b, f, n_frames, nb)];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) mean[b] = n_frames > 0 ? (float)(((red[0] + red[1]) + (red[2] + red[3])) / n_frames) : 0.0f;
}
__global__ void dense_pick_kernel(const float* __restrict__ mean, int nb, int32_t* __restrict__ dense_band,
                                  int32_t* __restrict__ dense_list, int32_t* __restrict__ n_dense) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int d = 0;
  for (int b = 0; b < nb; ++b) {
    const bool dense = mean[b] >= (float)kDenseChunks && d < kMaxDense;
    dense_band[b] = dense ? d : -1;
    if (dense) dense_list[d++] = b;
  }
  *n_dense = d;
}

// Pixel-major counts of the dense bands: KT[d * 128 + p][f] = count of candidate
// frame f at pixel 128 dense_list[d] + p (BF16, 0 when masked; columns past
// n_frames are 0).  64 x 64 tiles transposed through LDS.
__global__ __launch_bounds__(256) void dense_pack_kernel(const uint16_t* __restrict__ counts,
                                                         const uint8_t* __restrict__ mask, int n_pix,
                                                         const int32_t* __restrict__ frames, int64_t n_frames,
                                                         int64_t ld, const int32_t* __restrict__ dense_list,
                                                         uint16_t* __restrict__ KT) {
  __shared__ uint16_t tile[64][66];
  const int64_t r0 = (int64_t)blockIdx.x * 64, f0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {  // r: frame within tile, tx: dense pixel row within tile
    const int64_t f = f0 + r, row = r0 + tx;
    const int i = dense_list[row >> 7] * kBand + (int)(row & (kBand - 1));
    uint32_t v = 0;
    if (f < n_frames && i < n_pix && mask[i]) v = counts[(int64_t)frames[f] * n_pix + i];
    tile[r][tx] = count_bf16(v);
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) KT[(r0 + r) * ld + f0 + tx] = tile[tx][r];  // r: row, tx: frame
}

// W'[j][128 dense_list[d] + p] += D[j][128 d + p]
__global__ void dense_add_kernel(const float* __restrict__ D, int parts, int64_t n_rot, int n_dense,
                                 const int32_t* __restrict__ dense_list, int64_t ps, float* __restrict__ Wp) {
  const int64_t cols = (int64_t)n_dense * kBand, slab = n_rot * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < slab; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / cols;
    const int c = (int)(e - j * cols);
    float v = D[e];
    for (int s = 1; s < parts; ++s) v += D[e + s * slab];
    Wp[j * ps + (int64_t)dense_list[c >> 7] * kBand + (c & (kBand - 1))] += v;
  }
}

// zero fill, 16 bytes per store (n16 = bytes / 16)
__global__ void fill_zero16_kernel(u4* __restrict__ p, int64_t n16) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n16; e += (int64_t)gridDim.x * 256)
    p[e] = u4{0u, 0u, 0u, 0u};
}

// groups of up to 32 rotations: count per pack (cell_ptr: the packs' first pack-order
// rotation, n_cells + 1 entries; packs past the last hold none)
__global__ void pack_group_count_kernel(const int64_t* __restrict__ cell_ptr, int n_cells, int32_t* __restrict__ cnt) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_cells) return;
  const int64_t R = cell_ptr[c + 1] - cell_ptr[c];
  cnt[c] = (int32_t)((R + kGR - 1) / kGR);
}

// group table and storage sizes (Fp * 32 elements, Fp = the pack's frame list
// rounded up to 32)
__global__ void pack_group_fill_kernel(const int64_t* __restrict__ cell_ptr, const int64_t* __restrict__ cf_ptr,
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
    const int64_t nt = (cf_ptr[c + 1] - cf_ptr[c] + kTileF - 1) / kTileF;
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
    const int64_t nt = (cf_ptr[c + 1] - cf_ptr[c] + kTileF - 1) / kTileF;
    const int x = xcd_of[g];
    for (int64_t t = 0; t < nt; ++t) tiles[8 * (q[x]++) + x] = make_int2((int)g, (int)(t * kTileF));
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
                              const int64_t* cf_ptr, const int32_t* cf_frame, const void* runs, const void* chunks,
                              const int32_t* cell_rot, const void* hilo, int64_t plane, const float* scale, int64_t ps,
                              float* G, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  cand_loglik_kernel<<<(unsigned)n_tiles, 256, 0, st>>>(tiles, groups, grp_off, cf_ptr, cf_frame, (const u4*)runs,
                                                        (const u4*)chunks, cell_rot, (const uint16_t*)hilo, plane,
                                                        scale, ps, G);
  return hipGetLastError();
}

hipError_t launch_cand_estep(const float* G, void* P, const int4* groups, const int64_t* grp_off,
                             const int64_t* cg_ptr, const int32_t* cells, const int32_t* pair_col, int k_top,
                             int64_t n_frames, const int32_t* pack_of, const int32_t* cell_first,
                             const int64_t* cell_ptr, const int32_t* pack_rot, const int32_t* rot_local, int64_t n_rot,
                             const double* log_w, const double* S, double* cst, const double* b, double* L, void* Pd,
                             int64_t ldd, const int2* tiles, int64_t n_tiles, const int64_t* cf_ptr,
                             const int32_t* cf_frame, const uint32_t* cf_mask, hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  if (n_rot > 0)
    cell_const_kernel<<<(unsigned)((n_rot + 255) / 256), 256, 0, st>>>(pack_rot, n_rot, log_w, S, cst);
  cand_estep_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(G, groups, grp_off, cg_ptr, cells, pair_col, k_top,
                                                                    n_frames, pack_of, cell_first, cell_ptr, cst, b, L);
  if (n_tiles > 0)
    cand_pwrite_kernel<<<(unsigned)n_tiles, 256, 0, st>>>(tiles, groups, grp_off, cf_ptr, cf_frame, cf_mask, G,
                                                          pack_rot, rot_local, cst, b, L, (uint16_t*)P,
                                                          (uint16_t*)Pd, ldd);
  return hipGetLastError();
}

hipError_t launch_cand_mstep(const int4* groups, const int64_t* grp_off, int64_t n_groups, const int64_t* cf_ptr,
                             const int32_t* cf_frame, const void* runs, int64_t n_list, const void* chunks,
                             const int32_t* dense_band, const void* P, const int32_t* cell_rot, int64_t ps, float* Wp,
                             double* rho, const double* rho_a, bool accumulate, hipStream_t st) {
  if (n_groups <= 0) return hipSuccess;
  const int nranges = (int)((ps + 4 * kPair - 1) / (4 * kPair));
  const int64_t g8 = (n_groups + 7) / 8 * 8;
  cand_mstep_kernel<<<(unsigned)(g8 * nranges), 256, 0, st>>>(groups, grp_off, n_groups, nranges, cf_ptr, cf_frame,
                                                                    (const u4*)runs, n_list, (const u4*)chunks, dense_band,
                                                                    (const uint16_t*)P, cell_rot, ps, Wp, rho, rho_a,
                                                                    accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_band_count(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                             int64_t n_frames, int nbands, int32_t* cnt, int32_t* over, hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  band_count_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(counts, mask, n_pix, frames, n_frames, nbands, cnt,
                                                                    over);
  return hipGetLastError();
}

int run_count(int nbands) { return (nbands + kRun - 1) / kRun; }

hipError_t launch_run_table(const int64_t* ptr, int64_t n_frames, int nbands, void* runs, hipStream_t st) {
  const int64_t n = n_frames * run_count(nbands);
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + 255) / 256;
  run_table_kernel<<<(unsigned)(g > 65536 ? 65536 : g), 256, 0, st>>>(ptr, n_frames, nbands, (u4*)runs);
  return hipGetLastError();
}

hipError_t launch_band_fill(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                            int64_t n_frames, int nbands, const void* runs, void* chunks, hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  band_fill_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(counts, mask, n_pix, frames, n_frames, nbands,
                                                                   (const u4*)runs, (uint16_t*)chunks);
  return hipGetLastError();
}

hipError_t launch_band_dot(const void* runs, int nbands, const void* chunks, int64_t n_frames, const double* c,
                           double* b, hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  band_dot_kernel<<<(unsigned)((n_frames + 63) / 64), 256, 0, st>>>((const u4*)runs, nbands, (const u4*)chunks, n_frames,
                                                                   c, b);
  return hipGetLastError();
}

hipError_t launch_dense_bands(const int32_t* cnt, int64_t n_frames, int nbands, float* mean, int32_t* dense_band,
                              int32_t* dense_list, int32_t* n_dense, hipStream_t st) {
  if (n_frames > 0 && nbands > 0) {
    band_mean_kernel<<<(unsigned)nbands, 256, 0, st>>>(cnt, n_frames, nbands, mean);
  } else if (nbands > 0) {  // no frames: every band's mean is zero (the bits of 0.0f)
    const hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(mean), nbands, 0, st);
    if (e != hipSuccess) return e;
  }
  dense_pick_kernel<<<1, 64, 0, st>>>(mean, nbands, dense_band, dense_list, n_dense);
  return hipGetLastError();
}

hipError_t launch_dense_pack(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                             int64_t n_frames, int64_t ld, int n_dense, const int32_t* dense_list, void* KT,
                             hipStream_t st) {
  if (n_dense <= 0 || ld <= 0) return hipSuccess;
  const dim3 grid((unsigned)(n_dense * kBand / 64), (unsigned)(ld / 64));
  dense_pack_kernel<<<grid, 256, 0, st>>>(counts, mask, n_pix, frames, n_frames, ld, dense_list, (uint16_t*)KT);
  return hipGetLastError();
}

hipError_t launch_dense_add(const float* D, int parts, int64_t n_rot, int n_dense, const int32_t* dense_list,
                            int64_t ps, float* Wp, hipStream_t st) {
  const int64_t n = n_rot * n_dense * kBand;
  if (n <= 0) return hipSuccess;
  if (parts < 1) return hipErrorInvalidValue;
  const int64_t g = (n + 255) / 256;
  dense_add_kernel<<<(unsigned)(g > 65536 ? 65536 : g), 256, 0, st>>>(D, parts, n_rot, n_dense, dense_list, ps,
                                                                      Wp);
  return hipGetLastError();
}

// A frame chunk the audit rejects (mean recall below recall_min; NaN, no audit,
// accepts) contributes nothing to the grids: its W' rows and rho are cleared.
__global__ void gate_zero_kernel(const double* __restrict__ recall, double recall_min, f4* __restrict__ Wp,
                                 int64_t n4, double* __restrict__ rho, int64_t n_rot) {
  if (!(*recall < recall_min)) return;  // uniform: accepted
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (int64_t)gridDim.x * 256) Wp[e] = z;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_rot; e += (int64_t)gridDim.x * 256) rho[e] = 0.0;
}

hipError_t launch_gate_zero(const double* recall, double recall_min, float* Wp, int64_t n, double* rho, int64_t n_rot,
                            hipStream_t st) {
  if (n % 4 != 0) return hipErrorInvalidValue;
  gate_zero_kernel<<<2048, 256, 0, st>>>(recall, recall_min, (f4*)Wp, n / 4, rho, n_rot);
  return hipGetLastError();
}

hipError_t launch_fill_zero_bytes(void* p, int64_t bytes, hipStream_t st) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  const int64_t g = (n16 + 255) / 256;
  fill_zero16_kernel<<<(unsigned)(g > 65536 ? 65536 : g), 256, 0, st>>>((u4*)p, n16);
  return hipGetLastError();
}

hipError_t launch_pack_groups(const int64_t* cell_ptr, const int64_t* cf_ptr, int n_cells, int32_t* cnt,
                              int64_t* cg_ptr, int4* groups, int64_t* gsize, int64_t* grp_off, int64_t g_max,
                              hipStream_t st) {
  const unsigned nb = (unsigned)((n_cells + 255) / 256);
  pack_group_count_kernel<<<nb, 256, 0, st>>>(cell_ptr, n_cells, cnt);
  hipError_t e = launch_scan(cnt, n_cells, cg_ptr, st);
  if (e != hipSuccess) return e;
  // every group's size; sizes past the last group stay zero so the scan of g_max
  // entries gives the offsets of the real groups
  e = launch_fill_i32((int32_t*)gsize, 2 * g_max, 0, st);
  if (e != hipSuccess) return e;
  pack_group_fill_kernel<<<nb, 256, 0, st>>>(cell_ptr, cf_ptr, cg_ptr, n_cells, groups, gsize);
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
