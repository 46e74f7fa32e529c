// Plan of the learned-proposal form: coarse cells of the fine rotations, packs
// of neighbouring cells, the candidate frames grouped by their best cell and
// the union frame lists of each pack with one bit per proposed cell.  The
// candidate E- and M-steps and the candidate frames' sparse band format are in
// cand.hip.
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

// ------------------------------------------------------------------ packs of cells
constexpr int kNbr = 16;        // neighbours a cell's pack is filled from
constexpr int kMaxList = 256;   // entries of a frame's proposal list (at most)
// The cells' rotation groups are formed over packs: neighbouring cells whose rotation
// counts add up to at most kPackRot (one 16-row MFMA tile), searched
// over the union of their frame lists.  A frame then has its bands expanded once per
// pack instead of once per cell, and small cells share MFMA tiles.

// nn[c][k]: the kNbr cells nearest to cell c (largest |<q_c, q_d>|, d != c; ties to
// the lower index), -1 past n_cells - 1.  One thread per cell.
__global__ void cell_neighbours_kernel(const float* __restrict__ coarse, int n_cells, int32_t* __restrict__ nn) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_cells) return;
  const float4 qc = reinterpret_cast<const float4*>(coarse)[c];
  const float nc = rsqrtf(qc.x * qc.x + qc.y * qc.y + qc.z * qc.z + qc.w * qc.w);
  float best[kNbr];
  int idx[kNbr];
#pragma unroll
  for (int k = 0; k < kNbr; ++k) {
    best[k] = -1.0f;
    idx[k] = -1;
  }
  for (int d = 0; d < n_cells; ++d) {
    if (d == c) continue;
    const float4 qd = reinterpret_cast<const float4*>(coarse)[d];
    const float nd = rsqrtf(qd.x * qd.x + qd.y * qd.y + qd.z * qd.z + qd.w * qd.w);
    float v = fabsf(qc.x * qd.x + qc.y * qd.y + qc.z * qd.z + qc.w * qd.w) * nc * nd;
    int id = d;
    if (!(v > best[kNbr - 1])) continue;  // d ascending: an equal value keeps the lower index
#pragma unroll
    for (int k = 0; k < kNbr; ++k) {  // insertion: the entry carried down is the smaller one
      if (v > best[k]) {
        const float tv = best[k];
        const int ti = idx[k];
        best[k] = v;
        idx[k] = id;
        v = tv;
        id = ti;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kNbr; ++k) nn[(int64_t)c * kNbr + k] = idx[k];
}

// Greedy packing: cells in index order; an unpacked cell opens a pack and takes its
// unpacked neighbours, nearest first, while the pack's rotations stay within
// kPackRot (a cell with more rotations stays alone).  pack_of[c], slot_cell[s]
// (cells in pack order), pack_slot[p] (first slot of pack p, p <= n_packs),
// *n_packs.  One workgroup: the cells' sizes and packs are kept in LDS (dynamic,
// 8 bytes per cell) and thread 0 runs the greedy pass.
__global__ __launch_bounds__(256) void pack_cells_kernel(const int64_t* __restrict__ cell_ptr,
                                                         const int32_t* __restrict__ nn, int n_cells,
                                                         int32_t* __restrict__ pack_of, int32_t* __restrict__ slot_cell,
                                                         int32_t* __restrict__ pack_slot,
                                                         int32_t* __restrict__ n_packs) {
  extern __shared__ int32_t sh[];
  int32_t* size = sh;           // [n_cells] rotations per cell (clamped to kPackRot + 1)
  int32_t* pk = sh + n_cells;   // [n_cells] pack of each cell, -1: none yet
  for (int c = threadIdx.x; c < n_cells; c += 256) {
    const int64_t r = cell_ptr[c + 1] - cell_ptr[c];
    size[c] = (int32_t)(r > kPackRot ? kPackRot + 1 : r);
    pk[c] = -1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int slot = 0, np = 0;
    int32_t nb[kNbr];
#pragma unroll
    for (int k = 0; k < kNbr; ++k) nb[k] = n_cells > 0 ? nn[k] : -1;
    for (int c = 0; c < n_cells; ++c) {
      int32_t cur[kNbr];
#pragma unroll
      for (int k = 0; k < kNbr; ++k) cur[k] = nb[k];
      if (c + 1 < n_cells) {  // the next cell's neighbours, loaded while this one is packed
#pragma unroll
        for (int k = 0; k < kNbr; ++k) nb[k] = nn[(int64_t)(c + 1) * kNbr + k];
      }
      if (pk[c] >= 0) continue;
      pack_slot[np] = slot;
      pk[c] = np;
      slot_cell[slot++] = c;
      int r = size[c];
      if (r <= kPackRot) {
#pragma unroll
        for (int k = 0; k < kNbr; ++k) {
          const int d = cur[k];
          if (d < 0 || pk[d] >= 0 || r + size[d] > kPackRot) continue;
          pk[d] = np;
          slot_cell[slot++] = d;
          r += size[d];
        }
      }
      ++np;
    }
    pack_slot[np] = slot;
    *n_packs = np;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n_cells; c += 256) pack_of[c] = pk[c];
}

// slot_cnt[s] = rotations of the cell in slot s; cell_slot[c] = slot of cell c
__global__ void slot_sizes_kernel(const int32_t* __restrict__ slot_cell, const int64_t* __restrict__ cell_ptr,
                                  int n_cells, int32_t* __restrict__ slot_cnt, int32_t* __restrict__ cell_slot) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n_cells) return;
  const int c = slot_cell[s];
  slot_cnt[s] = (int32_t)(cell_ptr[c + 1] - cell_ptr[c]);
  cell_slot[c] = s;
}

// cell_first[c] = first pack_rot position of cell c; pack_ptr[p] = first pack_rot
// position of pack p (p <= n_cells; packs past the last one are empty at n_rot)
__global__ void pack_offsets_kernel(const int64_t* __restrict__ slot_ptr, const int32_t* __restrict__ cell_slot,
                                    const int32_t* __restrict__ pack_slot, const int32_t* __restrict__ n_packs,
                                    int n_cells, int32_t* __restrict__ cell_first, int64_t* __restrict__ pack_ptr) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n_cells) cell_first[e] = (int32_t)slot_ptr[cell_slot[e]];
  if (e <= n_cells) pack_ptr[e] = e <= *n_packs ? slot_ptr[pack_slot[e]] : slot_ptr[n_cells];
}

// pack_rot: the rotations in pack order (cell by cell, each cell's in cell_rot
// order); rot_local: index of each rotation's cell inside its pack
__global__ void pack_rotations_kernel(const int32_t* __restrict__ cell_rot, const int32_t* __restrict__ cell_of,
                                      const int64_t* __restrict__ cell_ptr, int n_rot,
                                      const int32_t* __restrict__ cell_first, const int32_t* __restrict__ cell_slot,
                                      const int32_t* __restrict__ pack_of, const int32_t* __restrict__ pack_slot,
                                      int32_t* __restrict__ pack_rot, int32_t* __restrict__ rot_local) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n_rot) return;
  const int32_t j = cell_rot[t];
  const int c = cell_of[j];
  const int64_t pos = cell_first[c] + (t - cell_ptr[c]);
  pack_rot[pos] = j;
  rot_local[pos] = cell_slot[c] - pack_slot[pack_of[c]];
}

// Per candidate frame (one wave): the first list entry of each pack the frame
// proposes is that pack's primary entry.  keys[e] = the pack for a primary entry,
// n_cells otherwise (sorted after every pack); bits[e] (primary entries) = the
// pack-local indices of every cell of the pack the frame lists; prim[e] = the
// frame's primary entry of the pack of entry e (-1: no cell).
__global__ __launch_bounds__(256) void pack_pairs_kernel(const int32_t* __restrict__ cells, int k_top, int64_t n_frames,
                                                         const int32_t* __restrict__ pack_of,
                                                         const int32_t* __restrict__ cell_slot,
                                                         const int32_t* __restrict__ pack_slot, int n_cells,
                                                         int32_t* __restrict__ keys, uint32_t* __restrict__ bits,
                                                         int32_t* __restrict__ prim) {
  __shared__ int32_t spk[4][kMaxList];  // pack of each entry of the wave's frame (-1: no cell)
  __shared__ int32_t sbit[4][kMaxList]; // its cell's index inside the pack
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t f = (int64_t)blockIdx.x * 4 + wave;
  if (f >= n_frames) return;  // uniform per wave; no barrier below
  const int32_t* row = cells + f * k_top;
  for (int t = lane; t < k_top; t += 64) {
    const int c = row[t];
    const int p = c < 0 ? -1 : pack_of[c];
    spk[wave][t] = p;
    sbit[wave][t] = c < 0 ? 0 : cell_slot[c] - pack_slot[p];
  }
  __builtin_amdgcn_wave_barrier();
  for (int t = lane; t < k_top; t += 64) {
    const int p = spk[wave][t];
    const int64_t e = f * k_top + t;
    if (p < 0) {
      keys[e] = n_cells;
      prim[e] = -1;
      continue;
    }
    int first = t;
    uint32_t m = 0u;
    for (int u = 0; u < k_top; ++u) {  // the frame's entries of the same pack
      if (spk[wave][u] != p) continue;
      if (u < first) first = u;
      m |= 1u << sbit[wave][u];
    }
    keys[e] = first == t ? p : n_cells;
    bits[e] = m;
    prim[e] = first;
  }
}

// Primary entries sorted by pack (order = entry indices, segments cf_ptr): the
// union list of each pack (frame, cell bits) and the entries' columns in it
__global__ void pack_columns_kernel(const int32_t* __restrict__ order, int64_t n_prim, int k_top,
                                    const int32_t* __restrict__ keys, const int64_t* __restrict__ cf_ptr,
                                    const uint32_t* __restrict__ bits, int32_t* __restrict__ cf_frame,
                                    uint32_t* __restrict__ cf_mask, int32_t* __restrict__ pair_col) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_prim) return;
  const int32_t e = order[i];
  cf_frame[i] = e / k_top;
  cf_mask[i] = bits[e];
  pair_col[e] = (int32_t)(i - cf_ptr[keys[e]]);
}

// the other entries take their primary entry's column
__global__ void pack_columns_rest_kernel(const int32_t* __restrict__ prim, int64_t n_pairs, int k_top,
                                         int32_t* __restrict__ pair_col) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_pairs) return;
  const int t0 = prim[e];
  const int64_t f = e / k_top;
  if (t0 >= 0 && f * k_top + t0 != e) pair_col[e] = pair_col[f * k_top + t0];
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

hipError_t launch_packs(const float* coarse, int n_cells, const int64_t* cell_ptr, const int32_t* cell_of,
                        const int32_t* cell_rot, int n_rot, int32_t* nn, int32_t* pack_of, int32_t* slot_cell,
                        int32_t* pack_slot, int32_t* n_packs, int32_t* slot_cnt, int64_t* slot_ptr, int32_t* cell_slot,
                        int32_t* cell_first, int64_t* pack_ptr, int32_t* pack_rot, int32_t* rot_local,
                        hipStream_t st) {
  cell_neighbours_kernel<<<g256(n_cells), 256, 0, st>>>(coarse, n_cells, nn);
  pack_cells_kernel<<<1, 256, (size_t)n_cells * 8, st>>>(cell_ptr, nn, n_cells, pack_of, slot_cell, pack_slot, n_packs);
  slot_sizes_kernel<<<g256(n_cells), 256, 0, st>>>(slot_cell, cell_ptr, n_cells, slot_cnt, cell_slot);
  exclusive_scan_kernel<<<1, 256, 0, st>>>(slot_cnt, n_cells, slot_ptr);
  pack_offsets_kernel<<<g256(n_cells + 1), 256, 0, st>>>(slot_ptr, cell_slot, pack_slot, n_packs, n_cells, cell_first,
                                                          pack_ptr);
  if (n_rot > 0)
    pack_rotations_kernel<<<g256(n_rot), 256, 0, st>>>(cell_rot, cell_of, cell_ptr, n_rot, cell_first, cell_slot,
                                                        pack_of, pack_slot, pack_rot, rot_local);
  return hipGetLastError();
}

hipError_t launch_pack_pairs(const int32_t* cells, int k_top, int64_t n_frames, const int32_t* pack_of,
                             const int32_t* cell_slot, const int32_t* pack_slot, int n_cells, int32_t* keys,
                             uint32_t* bits, int32_t* prim, hipStream_t st) {
  if (n_frames > 0)
    pack_pairs_kernel<<<(unsigned)((n_frames + 3) / 4), 256, 0, st>>>(cells, k_top, n_frames, pack_of, cell_slot,
                                                                       pack_slot, n_cells, keys, bits, prim);
  return hipGetLastError();
}

hipError_t launch_pack_columns(const int32_t* order, const int64_t* cf_ptr, int n_cells, int64_t n_pairs, int k_top,
                               const int32_t* keys, const uint32_t* bits, const int32_t* prim, int32_t* cf_frame,
                               uint32_t* cf_mask, int32_t* pair_col, hipStream_t st) {
  // primary entries are the first cf_ptr[n_cells] of the sorted order (the others
  // have key n_cells); the count is read on the device
  if (n_pairs <= 0) return hipSuccess;
  pack_columns_kernel<<<g256(n_pairs), 256, 0, st>>>(order, n_pairs, k_top, keys, cf_ptr, bits, cf_frame, cf_mask,
                                                      pair_col);
  pack_columns_rest_kernel<<<g256(n_pairs), 256, 0, st>>>(prim, n_pairs, k_top, pair_col);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n > 0) fill_i32_kernel<<<g256(n), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace emc
