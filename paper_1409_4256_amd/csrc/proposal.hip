// Plan of the learned-proposal form: coarse cells of the fine rotations, the
// candidate frames grouped by their best cell and the (frame, proposed cell)
// pairs grouped by cell.  The candidate E- and M-steps and the candidate frames'
// sparse band format are in cand.hip.
#include "emc_device.h"

namespace emc {

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
// up to kSegMax; longer segments keep the scatter order).
constexpr int kSegMax = 8192;
__global__ __launch_bounds__(256) void segment_sort_kernel(const int64_t* __restrict__ ptr, int32_t* __restrict__ vals) {
  __shared__ int32_t sv[kSegMax];
  const int64_t a = ptr[blockIdx.x], len = ptr[blockIdx.x + 1] - a;
  if (len <= 1 || len > kSegMax) return;
  int P2 = 1;
  while (P2 < len) P2 <<= 1;
  for (int e = threadIdx.x; e < P2; e += 256) sv[e] = e < len ? vals[a + e] : INT_MAX;
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
          }
        }
      }
      __syncthreads();
    }
  for (int e = threadIdx.x; e < len; e += 256) vals[a + e] = sv[e];
}

// union of two candidate lists per row: a's valid cells in order, then b's cells not
// in a (and not repeated), then -1; one wave per row, the row's bitmask in LDS
__global__ __launch_bounds__(256) void topk_union_kernel(const int32_t* __restrict__ A, int ka,
                                                         const int32_t* __restrict__ B, int kb, int64_t rows,
                                                         int n_cells, int32_t* __restrict__ out) {
  extern __shared__ uint32_t bits[];  // [4 waves][words]
  const int words = (n_cells + 31) >> 5;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 4 + wave;
  if (r >= rows) return;  // uniform per wave; no barrier below
  uint32_t* m = bits + wave * words;
  for (int w = lane; w < words; w += 64) m[w] = 0u;
  const int ko = ka + kb;
  int32_t* o = out + r * ko;
  int n = 0;  // cells written so far (uniform)
  for (int pass = 0; pass < 2; ++pass) {
    const int32_t* src = pass == 0 ? A + r * ka : B + r * kb;
    const int ks = pass == 0 ? ka : kb;
    for (int t0 = 0; t0 < ks; t0 += 64) {
      const int t = t0 + lane;
      int c = t < ks ? src[t] : -1;
      if (c >= n_cells) c = -1;
      // keep the first occurrence: test-and-set in lane order
      bool keep = false;
      for (int l = 0; l < 64; ++l) {
        const int cl = __shfl(c, l, 64);
        if (cl < 0) continue;
        const bool seen = (m[cl >> 5] >> (cl & 31)) & 1u;
        if (lane == l) keep = !seen;
        if (!seen && lane == 0) m[cl >> 5] |= 1u << (cl & 31);
        __builtin_amdgcn_wave_barrier();
      }
      const unsigned long long bal = __ballot(keep);
      if (keep) o[n + __popcll(bal & ((1ull << lane) - 1ull))] = c;
      n += __popcll(bal);
    }
  }
  for (int t = n + lane; t < ko; t += 64) o[t] = -1;
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

// a cell listed twice by one frame sets bit 1 of *flag; one wave per frame, the
// frame's cells marked in an LDS bitmask in list order
__global__ __launch_bounds__(256) void dup_check_kernel(const int32_t* __restrict__ cells, int k_top, int64_t n_frames,
                                                        int n_cells, int32_t* __restrict__ flag) {
  extern __shared__ uint32_t bits[];  // [4 waves][words]
  const int words = (n_cells + 31) >> 5;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t f = (int64_t)blockIdx.x * 4 + wave;
  if (f >= n_frames) return;  // uniform per wave; no barrier below
  uint32_t* m = bits + wave * words;
  for (int w = lane; w < words; w += 64) m[w] = 0u;
  bool dup = false;
  for (int t0 = 0; t0 < k_top; t0 += 64) {
    const int t = t0 + lane;
    const int c = t < k_top ? cells[f * k_top + t] : -1;  // entries are -1 or in [0, n_cells)
    for (int l = 0; l < 64; ++l) {
      const int cl = __shfl(c, l, 64);
      if (cl < 0) continue;
      const bool seen = (m[cl >> 5] >> (cl & 31)) & 1u;
      if (lane == l) dup |= seen;
      if (lane == 0) m[cl >> 5] |= 1u << (cl & 31);
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (__ballot(dup) != 0ull && lane == 0) atomicOr(flag, 2);
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
  if (nk > 0) segment_sort_kernel<<<(unsigned)nk, 256, 0, st>>>(ptr, order);
  return hipGetLastError();
}

hipError_t launch_topk_union(const int32_t* a, int ka, const int32_t* b, int kb, int64_t rows, int n_cells,
                             int32_t* out, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const size_t shm = (size_t)4 * ((n_cells + 31) / 32) * sizeof(uint32_t);
  topk_union_kernel<<<(unsigned)((rows + 3) / 4), 256, shm, st>>>(a, ka, b, kb, rows, n_cells, out);
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

hipError_t launch_dup_check(const int32_t* cells, int k_top, int64_t n_frames, int n_cells, int32_t* flag,
                            hipStream_t st) {
  if (n_frames <= 0) return hipSuccess;
  const size_t shm = (size_t)4 * ((n_cells + 31) / 32) * sizeof(uint32_t);
  dup_check_kernel<<<(unsigned)((n_frames + 3) / 4), 256, shm, st>>>(cells, k_top, n_frames, n_cells, flag);
  return hipGetLastError();
}

hipError_t launch_pair_columns(const int32_t* order, int64_t n_pairs, int k_top, const int32_t* keys,
                               const int64_t* cf_ptr, int32_t* cf_frame, int32_t* pair_col, hipStream_t st) {
  if (n_pairs > 0)
    pair_columns_kernel<<<(unsigned)((n_pairs + 255) / 256), 256, 0, st>>>(order, n_pairs, k_top, keys, cf_ptr,
                                                                           cf_frame, pair_col);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n > 0) fill_i32_kernel<<<g256(n), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace emc
