// Learned-proposal form of the E- and M-steps: each frame's E-step runs over
// the fine rotations of its top-K coarse cells only.  Frames are grouped in
// blocks of 256 (sorted by their best cell) and each block evaluates the
// log-likelihoods of the union of its frames' candidate rotations with the BF16
// MFMA GEMM (gathered rotation rows); the E-step masks each frame to its own
// candidates; the M-step contracts the significant responsibilities (P >=
// kKeep) as a sparse product with the frames.  Audited frames take the full
// search (dense kernels) and judge the proposal's recall.
#include "emc_device.h"

namespace emc {

constexpr double kKeep = 1e-7;  // responsibilities below this are left out of the M-step

// ------------------------------------------------------------------ coarse cells
// cell_of[j] = argmax_c |<q_j, q_c>| over normalised quaternions, ties -> lower c.
__global__ __launch_bounds__(256) void assign_cells_kernel(const float* __restrict__ quat, int n_rot,
                                                           const float* __restrict__ coarse, int n_cells,
                                                           int32_t* __restrict__ cell_of) {
  extern __shared__ float cq[];  // [n_cells][4], normalised
  for (int c = threadIdx.x; c < n_cells; c += 256) {
    const float* v = coarse + 4 * c;
    const float inv = rsqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
    for (int a = 0; a < 4; ++a) cq[4 * c + a] = v[a] * inv;
  }
  __syncthreads();
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n_rot) return;
  const float* v = quat + 4 * (int64_t)j;
  const float inv = rsqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
  const float w = v[0] * inv, x = v[1] * inv, y = v[2] * inv, z = v[3] * inv;
  float best = -1.0f;
  int bc = 0;
  for (int c = 0; c < n_cells; ++c) {
    const float d = fabsf(w * cq[4 * c] + x * cq[4 * c + 1] + y * cq[4 * c + 2] + z * cq[4 * c + 3]);
    if (d > best) {
      best = d;
      bc = c;
    }
  }
  cell_of[j] = bc;
}

// ------------------------------------------------------------------ counting sort by key
__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = v;
}

__global__ void key_hist_kernel(const int32_t* __restrict__ keys, int64_t n, int32_t* __restrict__ hist) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    atomicAdd(hist + keys[e], 1);
}

// exclusive scan of n int32 counts into ptr[0..n] (int64), single workgroup
__global__ __launch_bounds__(256) void exclusive_scan_kernel(const int32_t* __restrict__ cnt, int64_t n,
                                                             int64_t* __restrict__ ptr) {
  __shared__ int64_t part[256];
  const int64_t per = (n + 255) / 256;
  const int64_t a = threadIdx.x * per, z = a + per < n ? a + per : n;
  int64_t s = 0;
  for (int64_t e = a; e < z; ++e) s += cnt[e];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < 256; ++t) {
      const int64_t v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int64_t e = a; e < z; ++e) {
    ptr[e] = run;
    run += cnt[e];
  }
  if (threadIdx.x == 255) ptr[n] = run;
}

__global__ void key_scatter_kernel(const int32_t* __restrict__ keys, int64_t n, const int64_t* __restrict__ ptr,
                                   int32_t* __restrict__ cursor, int32_t* __restrict__ order) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int32_t k = keys[e];
    order[ptr[k] + atomicAdd(cursor + k, 1)] = (int32_t)e;
  }
}

// sort each segment [ptr[s], ptr[s+1]) of `vals` ascending (bitonic in LDS, segments
// up to kSegMax; longer segments keep the scatter order); optional payload follows.
constexpr int kSegMax = 4096;
__global__ __launch_bounds__(256) void segment_sort_kernel(const int64_t* __restrict__ ptr, int32_t* __restrict__ vals,
                                                           float* __restrict__ payload) {
  __shared__ int32_t sv[kSegMax];
  __shared__ float sp[kSegMax];
  const int64_t a = ptr[blockIdx.x], len = ptr[blockIdx.x + 1] - a;
  if (len <= 1 || len > kSegMax) return;
  int P2 = 1;
  while (P2 < len) P2 <<= 1;
  for (int e = threadIdx.x; e < P2; e += 256) {
    sv[e] = e < len ? vals[a + e] : INT_MAX;
    if (payload) sp[e] = e < len ? payload[a + e] : 0.0f;
  }
  __syncthreads();
  for (int k = 2; k <= P2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int e = threadIdx.x; e < P2; e += 256) {
        const int o = e ^ j;
        if (o > e) {
          const bool up = (e & k) == 0;
          if ((sv[e] > sv[o]) == up) {
            const int32_t t = sv[e];
            sv[e] = sv[o];
            sv[o] = t;
            if (payload) {
              const float tp = sp[e];
              sp[e] = sp[o];
              sp[o] = tp;
            }
          }
        }
      }
      __syncthreads();
    }
  for (int e = threadIdx.x; e < len; e += 256) {
    vals[a + e] = sv[e];
    if (payload) payload[a + e] = sp[e];
  }
}

// ------------------------------------------------------------------ candidate structures
// bitmask of each frame's candidate cells: mask[f][c/32] bit c%32 (f in list order)
__global__ void cand_mask_kernel(const int32_t* __restrict__ topk, int k_top, const int32_t* __restrict__ frames,
                                 int64_t n_frames, int words, uint32_t* __restrict__ mask) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= n_frames) return;
  uint32_t* m = mask + f * words;
  for (int w = 0; w < words; ++w) m[w] = 0u;
  const int64_t src = frames ? frames[f] : f;
  for (int t = 0; t < k_top; ++t) {
    const int c = topk[src * k_top + t];
    if (c >= 0) m[c >> 5] |= 1u << (c & 31);
  }
}

// candidate cells of the listed frames: cells[f][t] = topk[frames[f]][t] (-1 stays -1)
__global__ void cand_cells_kernel(const int32_t* __restrict__ topk, int k_top, const int32_t* __restrict__ frames,
                                  int64_t n_frames, int n_cells, int32_t* __restrict__ cells,
                                  int32_t* __restrict__ keys) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_frames * k_top) return;
  const int64_t f = e / k_top;
  const int t = (int)(e - f * k_top);
  int32_t c = topk[(int64_t)frames[f] * k_top + t];
  if (c < 0 || c >= n_cells) c = -1;
  cells[e] = c;
  keys[e] = c < 0 ? n_cells : c;  // invalid picks sort after every cell
}

// pairs sorted by cell (order = pair indices): frame of each pair in cell order and
// the column of each pair inside its cell's frame list
__global__ void pair_columns_kernel(const int32_t* __restrict__ order, int64_t n_pairs, int k_top,
                                    const int32_t* __restrict__ keys, const int64_t* __restrict__ cf_ptr,
                                    int32_t* __restrict__ cf_frame, int32_t* __restrict__ pair_col) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_pairs) return;
  const int32_t pr = order[e];
  cf_frame[e] = pr / k_top;
  pair_col[pr] = (int32_t)(e - cf_ptr[keys[pr]]);
}

// storage of each cell's block G_c [rotations of c][frames of c]: sizes
__global__ void cell_sizes_kernel(const int64_t* __restrict__ cell_ptr, const int64_t* __restrict__ cf_ptr,
                                  int n_cells, int64_t* __restrict__ sizes, int32_t* __restrict__ nchunk, int chunk) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_cells) return;
  const int64_t R = cell_ptr[c + 1] - cell_ptr[c], F = cf_ptr[c + 1] - cf_ptr[c];
  sizes[c] = R * F;
  nchunk[c] = R > 0 ? (int32_t)((F + chunk - 1) / chunk) : 0;
}

// tile table of the candidate log-likelihood: tiles of one cell are dealt to one
// XCD (dispatch order is round-robin over the 8 XCDs) so that the cell's slices stay
// in that XCD's L2; slot 8 q + x holds the q-th tile of XCD x, (-1, 0) pads.
__global__ void cell_tiles_kernel(const int32_t* __restrict__ nchunk, int n_cells, int2* __restrict__ tiles,
                                  int64_t* __restrict__ n_tiles_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t len[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = 0; c < n_cells; ++c) len[c & 7] += nchunk[c];
  int64_t q_max = 0;
  for (int x = 0; x < 8; ++x) q_max = len[x] > q_max ? len[x] : q_max;
  for (int x = 0; x < 8; ++x) {
    int64_t q = 0;
    for (int c = x; c < n_cells; c += 8)
      for (int t = 0; t < nchunk[c]; ++t) tiles[8 * (q++) + x] = make_int2(c, t);
    for (; q < q_max; ++q) tiles[8 * q + x] = make_int2(-1, 0);
  }
  *n_tiles_out = 8 * q_max;
}

// frame CSR of the listed frames: non-zero photon counts of unmasked pixels as
// (pixel << 16) | count, pixels ascending
__global__ __launch_bounds__(256) void nz_count_kernel(const uint16_t* __restrict__ counts,
                                                       const uint8_t* __restrict__ mask, int n_pix,
                                                       const int32_t* __restrict__ frames, int64_t n_frames,
                                                       int32_t* __restrict__ cnt) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;
  const uint16_t* row = counts + (int64_t)frames[f] * n_pix;
  int n = 0;
  for (int i = lane; i < n_pix; i += 64) n += (mask[i] && row[i] != 0);
  n = wave_sum(n);
  if (lane == 0) cnt[f] = n;
}

__global__ __launch_bounds__(256) void nz_fill_kernel(const uint16_t* __restrict__ counts,
                                                      const uint8_t* __restrict__ mask, int n_pix,
                                                      const int32_t* __restrict__ frames, int64_t n_frames,
                                                      const int64_t* __restrict__ ptr, uint32_t* __restrict__ nz) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;
  const uint16_t* row = counts + (int64_t)frames[f] * n_pix;
  int64_t at = ptr[f];
  for (int i0 = 0; i0 < n_pix; i0 += 64) {
    const int i = i0 + lane;
    const uint32_t v = i < n_pix && mask[i] ? row[i] : 0u;
    const bool hit = v != 0u;
    const unsigned long long bal = __ballot(hit);
    if (hit) nz[at + __popcll(bal & ((1ull << lane) - 1ull))] = ((uint32_t)i << 16) | v;
    at += __popcll(bal);
  }
}

// ------------------------------------------------------------------ candidate log-likelihood
// G_c[r][p] = sum over the non-zero pixels i of frame cf_frame[c][p] of K_i A_{rot(c, r), i}
// (A: FP32 centred log slices).  Workgroup = one tile (cell c, chunk of kChunk frames);
// each wave takes frames of the chunk, lanes stride over a frame's non-zero pixels and
// accumulate all the cell's rotations (up to kRot per pass).
constexpr int kChunk = 32, kRot = 32;
__global__ __launch_bounds__(256) void cand_loglik_kernel(const int2* __restrict__ tiles,
                                                          const int64_t* __restrict__ cell_ptr,
                                                          const int32_t* __restrict__ cell_rot,
                                                          const int64_t* __restrict__ cf_ptr,
                                                          const int32_t* __restrict__ cf_frame,
                                                          const int64_t* __restrict__ g_off,
                                                          const int64_t* __restrict__ nz_ptr,
                                                          const uint32_t* __restrict__ nz,
                                                          const float* __restrict__ A, int64_t ps,
                                                          float* __restrict__ G) {
  const int2 tl = tiles[blockIdx.x];
  const int c = tl.x;
  if (c < 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t R = cell_ptr[c + 1] - cell_ptr[c];
  const int64_t F = cf_ptr[c + 1] - cf_ptr[c];
  const int32_t* rots = cell_rot + cell_ptr[c];
  float* Gc = G + g_off[c];
  for (int64_t p = (int64_t)tl.y * kChunk + wave; p < F && p < (int64_t)(tl.y + 1) * kChunk; p += 4) {
    const int64_t f = cf_frame[cf_ptr[c] + p];
    const int64_t a = nz_ptr[f], z = nz_ptr[f + 1];
    for (int64_t r0 = 0; r0 < R; r0 += kRot) {
      const int nr = (int)(R - r0 < kRot ? R - r0 : kRot);
      float acc[kRot];
#pragma unroll
      for (int r = 0; r < kRot; ++r) acc[r] = 0.0f;
      for (int64_t e = a + lane; e < z; e += 64) {
        const uint32_t w = nz[e];
        const int64_t i = w >> 16;
        const float v = (float)(w & 0xffffu);
#pragma unroll
        for (int r = 0; r < kRot; ++r)
          if (r < nr) acc[r] += v * A[(int64_t)rots[r0 + r] * ps + i];
      }
#pragma unroll
      for (int r = 0; r < kRot; ++r) {
        const float t = wave_sum(acc[r]);
        if (lane == r && r < nr) Gc[(r0 + r) * F + p] = t;
      }
    }
  }
}

// ------------------------------------------------------------------ candidate E-step
__device__ __forceinline__ void lse_merge2(double& m, double& s, double m2, double s2) {
  if (m2 > m) {
    s = s * exp(m - m2) + s2;
    m = m2;
  } else if (m2 > -INFINITY) {
    s += s2 * exp(m2 - m);
  }
}

// One wave per frame; lane t takes the frame's t-th candidate cell (k_top <= 64).
// Log-sum-exp over the candidates, P written in place of G, triples with P >= kKeep.
__global__ __launch_bounds__(256) void cand_estep_kernel(float* __restrict__ G, const int64_t* __restrict__ g_off,
                                                         const int32_t* __restrict__ cells,
                                                         const int32_t* __restrict__ pair_col, int k_top,
                                                         int64_t n_frames, const int64_t* __restrict__ cell_ptr,
                                                         const int32_t* __restrict__ cell_rot,
                                                         const int64_t* __restrict__ cf_ptr,
                                                         const double* __restrict__ log_w,
                                                         const double* __restrict__ S, const double* __restrict__ b,
                                                         double* __restrict__ L, int32_t* __restrict__ tj,
                                                         int32_t* __restrict__ tk, float* __restrict__ tp,
                                                         int64_t cap, unsigned long long* __restrict__ count,
                                                         int32_t* __restrict__ overflow) {
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (f >= n_frames) return;  // uniform per wave
  const int c = lane < k_top ? cells[f * k_top + lane] : -1;
  const int64_t col = c >= 0 ? pair_col[f * k_top + lane] : 0;
  const int64_t R = c >= 0 ? cell_ptr[c + 1] - cell_ptr[c] : 0;
  const int64_t F = c >= 0 ? cf_ptr[c + 1] - cf_ptr[c] : 0;
  const int32_t* rots = c >= 0 ? cell_rot + cell_ptr[c] : cell_rot;
  float* Gc = c >= 0 ? G + g_off[c] + col : G;
  const double bk = b[f];
  double mx = -INFINITY, s = 0.0;
  for (int64_t r = 0; r < R; ++r) {
    const int j = rots[r];
    const double a = ((double)Gc[r * F] + bk) + (log_w[j] - S[j]);
    if (!(a > -INFINITY)) continue;
    if (a > mx) {
      s = s * exp(mx - a) + 1.0;
      mx = a;
    } else {
      s += exp(a - mx);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double m2 = __shfl_xor(mx, o, 64), s2 = __shfl_xor(s, o, 64);
    lse_merge2(mx, s, m2, s2);
  }
  const double lse = mx + log(s);
  if (lane == 0) L[f] = lse;
  for (int64_t r = 0; r < R; ++r) {
    const int j = rots[r];
    const double a = ((double)Gc[r * F] + bk) + (log_w[j] - S[j]);
    const double pd = exp(a - lse);
    const float p = (float)pd;
    Gc[r * F] = p;
    if (pd >= kKeep) {
      const unsigned long long at = atomicAdd(count, 1ull);
      if ((int64_t)at < cap) {
        tj[at] = j;
        tk[at] = (int32_t)f;
        tp[at] = p;
      } else {
        *overflow = 1;
      }
    }
  }
}

// Full-search (audited) frames: append their triples from dense P [n_rot][ldp]
// and accumulate recall_f = sum of P over the frame's candidates (recall zeroed
// first).  Workgroup = 64 frames (lanes) x a chunk of rotations split over 4 waves.
constexpr int kAuditRot = 1024;
template <typename PT>
__global__ __launch_bounds__(256) void audit_kernel(const PT* __restrict__ P, int64_t ldp, int n_rot,
                                                    int64_t n_audit, const uint32_t* __restrict__ mask_audit,
                                                    int words, const int32_t* __restrict__ cell_of,
                                                    int32_t frame_base, int32_t* __restrict__ tj,
                                                    int32_t* __restrict__ tk, float* __restrict__ tp, int64_t cap,
                                                    unsigned long long* __restrict__ count,
                                                    int32_t* __restrict__ overflow, double* __restrict__ recall) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t a = (int64_t)blockIdx.x * 64 + lane;
  if (a >= n_audit) return;
  const uint32_t* m = mask_audit + a * words;
  const int j0 = blockIdx.y * kAuditRot;
  const int j1 = j0 + kAuditRot < n_rot ? j0 + kAuditRot : n_rot;
  double rec = 0.0;
  for (int j = j0 + wave; j < j1; j += 4) {
    const float p = (float)P[(int64_t)j * ldp + a];
    const int c = cell_of[j];
    if ((m[c >> 5] >> (c & 31)) & 1u) rec += p;
    if ((double)p >= kKeep) {
      const unsigned long long at = atomicAdd(count, 1ull);
      if ((int64_t)at < cap) {
        tj[at] = j;
        tk[at] = frame_base + (int32_t)a;
        tp[at] = p;
      } else {
        *overflow = 1;
      }
    }
  }
  atomicAdd(recall + a, rec);
}

// gather triples into rotation order: out[e] = in[order[e]]
__global__ void gather_triples_kernel(const int32_t* __restrict__ order, int64_t n, const int32_t* __restrict__ tk,
                                      const float* __restrict__ tp, int32_t* __restrict__ tk2, float* __restrict__ tp2) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int32_t o = order[e];
    tk2[e] = tk[o];
    tp2[e] = tp[o];
  }
}

// ------------------------------------------------------------------ sparse M-step
// W'_j = sum over triples (j, k, p) of p K_k (frames of the candidate list, then the
// audited frames), rho_j = sum p; one workgroup per rotation.  Triples of a rotation
// are contiguous (sorted by rotation, then frame).
template <typename T>
__global__ __launch_bounds__(256) void sparse_mstep_kernel(const int64_t* __restrict__ tptr,
                                                           const int32_t* __restrict__ tk,
                                                           const float* __restrict__ tp, const T* __restrict__ Kc,
                                                           int64_t n_cand, const T* __restrict__ Ka, int64_t ps,
                                                           float* __restrict__ Wp, double* __restrict__ rho) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const int64_t a = tptr[j], z = tptr[j + 1];
  float* row = Wp + (int64_t)j * ps;
  constexpr int V = 8;
  for (int64_t i0 = 0; i0 < ps; i0 += 256 * V) {
    float acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0f;
    for (int64_t e = a; e < z; ++e) {
      const int64_t k = tk[e];
      const float p = tp[e];
      const T* kr = k < n_cand ? Kc + k * ps : Ka + (k - n_cand) * ps;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int64_t i = i0 + v * 256 + threadIdx.x;
        if (i < ps) acc[v] += p * (float)kr[i];
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int64_t i = i0 + v * 256 + threadIdx.x;
      if (i < ps) row[i] = acc[v];
    }
  }
  double s = 0.0;
  for (int64_t e = a + threadIdx.x; e < z; e += 256) s += (double)tp[e];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) rho[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ------------------------------------------------------------------ triple sort (count on the device)
__device__ __forceinline__ int64_t live_count(const unsigned long long* count, int64_t cap) {
  const int64_t c = (int64_t)*count;
  return c < cap ? c : cap;
}
__global__ void triple_hist_kernel(const int32_t* __restrict__ tj, const unsigned long long* __restrict__ count,
                                   int64_t cap, int32_t* __restrict__ hist) {
  const int64_t n = live_count(count, cap);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    atomicAdd(hist + tj[e], 1);
}
__global__ void triple_scatter_kernel(const int32_t* __restrict__ tj, const int32_t* __restrict__ tk,
                                      const float* __restrict__ tp, const unsigned long long* __restrict__ count,
                                      int64_t cap, const int64_t* __restrict__ ptr, int32_t* __restrict__ cursor,
                                      int32_t* __restrict__ tk2, float* __restrict__ tp2) {
  const int64_t n = live_count(count, cap);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int32_t j = tj[e];
    const int64_t at = ptr[j] + atomicAdd(cursor + j, 1);
    tk2[at] = tk[e];
    tp2[at] = tp[e];
  }
}

// ===================================================================== launchers
static inline unsigned g256(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

hipError_t launch_assign_cells(const float* quat, int n_rot, const float* coarse, int n_cells, int32_t* cell_of,
                               hipStream_t st) {
  assign_cells_kernel<<<(unsigned)((n_rot + 255) / 256), 256, (size_t)n_cells * 16, st>>>(quat, n_rot, coarse,
                                                                                          n_cells, cell_of);
  return hipGetLastError();
}

// keys [n] in [0, nk) -> ptr [nk+1], order [n] (items grouped by key, ascending item
// index inside a key for segments up to kSegMax); hist and cursor are [nk] scratch.
hipError_t launch_counting_sort(const int32_t* keys, int64_t n, int nk, int32_t* hist, int32_t* cursor,
                                int64_t* ptr, int32_t* order, float* payload_unused, hipStream_t st) {
  (void)payload_unused;
  fill_i32_kernel<<<g256(nk), 256, 0, st>>>(hist, nk, 0);
  fill_i32_kernel<<<g256(nk), 256, 0, st>>>(cursor, nk, 0);
  if (n > 0) key_hist_kernel<<<g256(n), 256, 0, st>>>(keys, n, hist);
  exclusive_scan_kernel<<<1, 256, 0, st>>>(hist, nk, ptr);
  if (n > 0) key_scatter_kernel<<<g256(n), 256, 0, st>>>(keys, n, ptr, cursor, order);
  if (nk > 0) segment_sort_kernel<<<(unsigned)nk, 256, 0, st>>>(ptr, order, nullptr);
  return hipGetLastError();
}

hipError_t launch_segment_sort(const int64_t* ptr, int n_seg, int32_t* vals, float* payload, hipStream_t st) {
  if (n_seg > 0) segment_sort_kernel<<<(unsigned)n_seg, 256, 0, st>>>(ptr, vals, payload);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void exclusive_scan64_kernel(const int64_t* __restrict__ cnt, int64_t n,
                                                               int64_t* __restrict__ ptr) {
  __shared__ int64_t part[256];
  const int64_t per = (n + 255) / 256;
  const int64_t a = threadIdx.x * per, z = a + per < n ? a + per : n;
  int64_t s = 0;
  for (int64_t e = a; e < z; ++e) s += cnt[e];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < 256; ++t) {
      const int64_t v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int64_t e = a; e < z; ++e) {
    ptr[e] = run;
    run += cnt[e];
  }
  if (threadIdx.x == 255) ptr[n] = run;
}

hipError_t launch_scan64(const int64_t* cnt, int64_t n, int64_t* ptr, hipStream_t st) {
  exclusive_scan64_kernel<<<1, 256, 0, st>>>(cnt, n, ptr);
  return hipGetLastError();
}

hipError_t launch_scan(const int32_t* cnt, int64_t n, int64_t* ptr, hipStream_t st) {
  exclusive_scan_kernel<<<1, 256, 0, st>>>(cnt, n, ptr);
  return hipGetLastError();
}

hipError_t launch_cand_mask(const int32_t* topk, int k_top, const int32_t* frames, int64_t n_frames, int words,
                            uint32_t* mask, hipStream_t st) {
  if (n_frames > 0) cand_mask_kernel<<<(unsigned)((n_frames + 255) / 256), 256, 0, st>>>(topk, k_top, frames,
                                                                                        n_frames, words, mask);
  return hipGetLastError();
}

hipError_t launch_cand_cells(const int32_t* topk, int k_top, const int32_t* frames, int64_t n_frames, int n_cells,
                             int32_t* cells, int32_t* keys, hipStream_t st) {
  const int64_t n = n_frames * k_top;
  if (n > 0) cand_cells_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(topk, k_top, frames, n_frames, n_cells,
                                                                             cells, keys);
  return hipGetLastError();
}

hipError_t launch_pair_columns(const int32_t* order, int64_t n_pairs, int k_top, const int32_t* keys,
                               const int64_t* cf_ptr, int32_t* cf_frame, int32_t* pair_col, hipStream_t st) {
  if (n_pairs > 0)
    pair_columns_kernel<<<(unsigned)((n_pairs + 255) / 256), 256, 0, st>>>(order, n_pairs, k_top, keys, cf_ptr,
                                                                           cf_frame, pair_col);
  return hipGetLastError();
}

hipError_t launch_cell_sizes(const int64_t* cell_ptr, const int64_t* cf_ptr, int n_cells, int64_t* sizes,
                             int32_t* nchunk, hipStream_t st) {
  cell_sizes_kernel<<<(unsigned)((n_cells + 255) / 256), 256, 0, st>>>(cell_ptr, cf_ptr, n_cells, sizes, nchunk,
                                                                       kChunk);
  return hipGetLastError();
}

hipError_t launch_cell_tiles(const int32_t* nchunk, int n_cells, int2* tiles, int64_t* n_tiles, hipStream_t st) {
  cell_tiles_kernel<<<1, 64, 0, st>>>(nchunk, n_cells, tiles, n_tiles);
  return hipGetLastError();
}

hipError_t launch_nz_count(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                           int64_t n_frames, int32_t* cnt, hipStream_t st) {
  if (n_frames > 0)
    nz_count_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(counts, mask, n_pix, frames, n_frames, cnt);
  return hipGetLastError();
}

hipError_t launch_nz_fill(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                          int64_t n_frames, const int64_t* ptr, uint32_t* nz, hipStream_t st) {
  if (n_frames > 0)
    nz_fill_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(counts, mask, n_pix, frames, n_frames, ptr, nz);
  return hipGetLastError();
}

hipError_t launch_cand_loglik(const int2* tiles, int64_t n_tiles, const int64_t* cell_ptr, const int32_t* cell_rot,
                              const int64_t* cf_ptr, const int32_t* cf_frame, const int64_t* g_off,
                              const int64_t* nz_ptr, const uint32_t* nz, const float* A, int64_t ps, float* G,
                              hipStream_t st) {
  if (n_tiles > 0)
    cand_loglik_kernel<<<(unsigned)n_tiles, 256, 0, st>>>(tiles, cell_ptr, cell_rot, cf_ptr, cf_frame, g_off, nz_ptr,
                                                          nz, A, ps, G);
  return hipGetLastError();
}

hipError_t launch_cand_estep(float* G, const int64_t* g_off, const int32_t* cells, const int32_t* pair_col, int k_top,
                             int64_t n_frames, const int64_t* cell_ptr, const int32_t* cell_rot, const int64_t* cf_ptr,
                             const double* log_w, const double* S, const double* b, double* L, int32_t* tj,
                             int32_t* tk, float* tp, int64_t cap, unsigned long long* count, int32_t* overflow,
                             hipStream_t st) {
  if (n_frames > 0)
    cand_estep_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(G, g_off, cells, pair_col, k_top, n_frames,
                                                                      cell_ptr, cell_rot, cf_ptr, log_w, S, b, L, tj,
                                                                      tk, tp, cap, count, overflow);
  return hipGetLastError();
}

hipError_t launch_audit(const void* P, bool bf16, int64_t ldp, int n_rot, int64_t n_audit, const uint32_t* mask_audit,
                        int words, const int32_t* cell_of, int32_t frame_base, int32_t* tj, int32_t* tk, float* tp,
                        int64_t cap, unsigned long long* count, int32_t* overflow, double* recall, hipStream_t st) {
  if (n_audit <= 0) return hipSuccess;
  const dim3 g((unsigned)((n_audit + 63) / 64), (unsigned)((n_rot + kAuditRot - 1) / kAuditRot));
  if (bf16)
    audit_kernel<__hip_bfloat16><<<g, 256, 0, st>>>((const __hip_bfloat16*)P, ldp, n_rot, n_audit, mask_audit, words,
                                                    cell_of, frame_base, tj, tk, tp, cap, count, overflow, recall);
  else
    audit_kernel<float><<<g, 256, 0, st>>>((const float*)P, ldp, n_rot, n_audit, mask_audit, words, cell_of,
                                           frame_base, tj, tk, tp, cap, count, overflow, recall);
  return hipGetLastError();
}

hipError_t launch_gather_triples(const int32_t* order, int64_t n, const int32_t* tk, const float* tp, int32_t* tk2,
                                 float* tp2, hipStream_t st) {
  if (n > 0) gather_triples_kernel<<<g256(n), 256, 0, st>>>(order, n, tk, tp, tk2, tp2);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n > 0) fill_i32_kernel<<<g256(n), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

// triples (tj, tk, tp)[0 .. min(*count, cap)) -> ptr [n_rot + 1] and (tk2, tp2) grouped by
// rotation, frames ascending inside a rotation (segments up to kSegMax)
hipError_t launch_triple_sort(const int32_t* tj, const int32_t* tk, const float* tp, const unsigned long long* count,
                              int64_t cap, int n_rot, int32_t* hist, int32_t* cursor, int64_t* ptr, int32_t* tk2,
                              float* tp2, hipStream_t st) {
  fill_i32_kernel<<<g256(n_rot), 256, 0, st>>>(hist, n_rot, 0);
  fill_i32_kernel<<<g256(n_rot), 256, 0, st>>>(cursor, n_rot, 0);
  triple_hist_kernel<<<g256(cap), 256, 0, st>>>(tj, count, cap, hist);
  exclusive_scan_kernel<<<1, 256, 0, st>>>(hist, n_rot, ptr);
  triple_scatter_kernel<<<g256(cap), 256, 0, st>>>(tj, tk, tp, count, cap, ptr, cursor, tk2, tp2);
  segment_sort_kernel<<<(unsigned)n_rot, 256, 0, st>>>(ptr, tk2, tp2);
  return hipGetLastError();
}

hipError_t launch_sparse_mstep(const int64_t* tptr, const int32_t* tk, const float* tp, const void* Kc, int64_t n_cand,
                               const void* Ka, bool bf16, int64_t ps, int n_rot, float* Wp, double* rho,
                               hipStream_t st) {
  if (bf16)
    sparse_mstep_kernel<__hip_bfloat16><<<(unsigned)n_rot, 256, 0, st>>>(
        tptr, tk, tp, (const __hip_bfloat16*)Kc, n_cand, (const __hip_bfloat16*)Ka, ps, Wp, rho);
  else
    sparse_mstep_kernel<float><<<(unsigned)n_rot, 256, 0, st>>>(tptr, tk, tp, (const float*)Kc, n_cand,
                                                                (const float*)Ka, ps, Wp, rho);
  return hipGetLastError();
}

}  // namespace emc
