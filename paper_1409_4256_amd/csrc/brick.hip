// Brick-major c-step, eq. (2.12): the same sums as the rotation-major scatter,
// num_l = sum_{j,i} f(p_l - R_j q_i) W'_ji and den_l = sum_{j,i} f(p_l - R_j q_i) rho_j,
// with the loop nest turned round.  The grid is cut into 16^3-voxel bricks; a
// "visit" is (rotation j, group t of 64 consecutive pixels) for one brick that a
// non-zero trilinear corner of the group reaches.  A plan built once per geometry
// lists the visits brick by brick.  One workgroup takes a run of one brick's
// visits, accumulates the brick in LDS (FP64) and adds it to the grids once, so
// the global atomics number one per voxel per work item instead of one per
// touched voxel per pixel group and rotation.
//
// The plan and the scatter find a pixel's corners with the same arithmetic (one
// table of R_j, explicit fused multiply-adds, nothing left to the compiler's
// contraction), so every corner the scatter keeps lies in a brick the plan listed.
#include <limits.h>

#include "emc_device.h"

namespace emc {

constexpr int kBrick = 16;                           // brick edge (voxels)
constexpr int kBrickVox = kBrick * kBrick * kBrick;  // 4096 voxels, 64 KB of FP64 num + den in LDS
constexpr int kVisitPx = 64;                         // pixels of one visit: one wave's lanes
constexpr int kBrickWaves = 8;                       // waves of a scatter workgroup

struct Corner {
  int bx, by, bz;      // lowest corner of the 2 x 2 x 2 neighbourhood
  double tx, ty, tz;   // fractional position inside it
};

// R_j of quaternion (w, x, y, z) as in eq. (2.9)'s rotation, every operation explicit.
__device__ __forceinline__ void brick_rot(const float* __restrict__ qv, double m[9]) {
  const double w = qv[0], x = qv[1], y = qv[2], z = qv[3];
  const double s = 2.0 / fma(w, w, fma(x, x, fma(y, y, z * z)));
  m[0] = fma(-s, fma(y, y, z * z), 1.0);
  m[1] = s * fma(x, y, -(w * z));
  m[2] = s * fma(x, z, w * y);
  m[3] = s * fma(x, y, w * z);
  m[4] = fma(-s, fma(x, x, z * z), 1.0);
  m[5] = s * fma(y, z, -(w * x));
  m[6] = s * fma(x, z, -(w * y));
  m[7] = s * fma(y, z, w * x);
  m[8] = fma(-s, fma(x, x, y * y), 1.0);
}

// Grid-frame position of R_j q_i (origin at voxel N/2) split into its cell and fraction.
__device__ __forceinline__ Corner brick_corner(const double m[9], float qx_, float qy_, float qz_, double h) {
  const double qx = qx_, qy = qy_, qz = qz_;
  const double px = fma(m[0], qx, fma(m[1], qy, fma(m[2], qz, h)));
  const double py = fma(m[3], qx, fma(m[4], qy, fma(m[5], qz, h)));
  const double pz = fma(m[6], qx, fma(m[7], qy, fma(m[8], qz, h)));
  const double fx = floor(px), fy = floor(py), fz = floor(pz);
  Corner c;
  c.bx = (int)fx;
  c.by = (int)fy;
  c.bz = (int)fz;
  c.tx = px - fx;
  c.ty = py - fy;
  c.tz = pz - fz;
  return c;
}

// R_j for every rotation, stored [n_rot][9] for the plan's and the scatter's kernels
__global__ void brick_rot_kernel(const float* __restrict__ quat, int n_rot, double* __restrict__ rot) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n_rot) return;
  double m[9];
  brick_rot(quat + 4 * (int64_t)j, m);
#pragma unroll
  for (int k = 0; k < 9; ++k) rot[9 * (int64_t)j + k] = m[k];
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void load_rot(const double* __restrict__ rot, int j, double m[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = rot[9 * (int64_t)j + k];
}

// Brick indices an axis's two corners b, b + 1 reach inside [0, N): lo > hi when none.
__device__ __forceinline__ void axis_bricks(int b, int N, int& lo, int& hi) {
  const int c0 = max(b, 0), c1 = min(b + 1, N - 1);
  lo = c0 <= c1 ? c0 / kBrick : INT_MAX;
  hi = c0 <= c1 ? c1 / kBrick : INT_MIN;
}

// LDS slot of brick voxel (ex, ey, ez).  A bank pair of FP64 LDS is picked by the
// slot's low bits; in the natural order (ex * 16 + ey) * 16 + ez those are ez and
// ey & 1 alone, so the pixels of a detector patch in a plane of constant z would
// pile onto two bank pairs.  Each row of 16 z-voxels is rotated by (13 ex + 7 ey)
// mod 16 and its y parity flipped with x: over the visits of the 128^3 workload
// (simulated on the host) the busiest bank pair of an atomic instruction then
// holds 4.4 lanes on average (16 pairs) against 10.3 unswizzled.  Rows and planes
// are only permuted, so the map is a bijection of the brick.
__device__ __forceinline__ int lds_slot(int ex, int ey, int ez) {
  return (ex * kBrick + (ey ^ (ex & 1))) * kBrick + ((ez + 13 * ex + 7 * ey) & (kBrick - 1));
}

__device__ __forceinline__ int wmin(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wmax(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// The bricks the used pixels of visit (rotation j, pixel group t) reach; a wave
// takes kVisitItems consecutive visits.  FILL = false counts visits per brick;
// FILL = true writes j * n_groups + t into the brick's list at off[brick] + the
// next slot of cursor[brick].  A workgroup first tallies its own hits per brick in
// LDS and then touches each brick's global counter once: the central bricks are
// reached by every rotation, and one device-scope atomic per hit on those few
// counters serialised the pass.  (FILL: the workgroup lists its hits in LDS,
// reserves each brick's range with one atomic and writes the visits into it; hits
// past the list's capacity, and grids of more than kVisitLdsBricks bricks, take
// one global atomic each.)
constexpr int kVisitItems = 8;
constexpr int kVisitLdsBricks = 4096;  // bricks tallied in LDS (grids up to 256^3)
constexpr int kVisitListCap = 1024;    // hits a workgroup lists in LDS (FILL)
template <bool FILL>
__global__ __launch_bounds__(256) void brick_visit_kernel(const float* __restrict__ q, const uint8_t* __restrict__ mask,
                                                          const double* __restrict__ rot, int n_pix, int n_rot,
                                                          int n_groups, int N, int nb, int* __restrict__ cnt,
                                                          const int64_t* __restrict__ off, int* __restrict__ visits) {
  __shared__ int tally[kVisitLdsBricks];            // this workgroup's hits per brick (FILL: then its cursors)
  __shared__ int base[FILL ? kVisitLdsBricks : 1];  // FILL: first slot of this workgroup's hits of each brick
  __shared__ int2 hits[FILL ? kVisitListCap : 1];   // FILL: (brick, visit)
  __shared__ int n_hits;
  const int n_bricks = nb * nb * nb;
  const bool local = n_bricks <= kVisitLdsBricks;
  if (local)
    for (int b = threadIdx.x; b < n_bricks; b += 256) tally[b] = 0;
  if (threadIdx.x == 0) n_hits = 0;
  __syncthreads();
  auto direct = [&](int brick, int id) {  // one global atomic for this hit
    const int slot = atomicAdd(cnt + brick, 1);
    if constexpr (FILL)  // the counting pass found the same visits; the guard only bounds the write
      if (off[brick] + slot < off[brick + 1]) visits[off[brick] + slot] = id;
  };
  const int64_t w0 = ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * kVisitItems;
  const int lane = threadIdx.x & 63;
  const int64_t n_visits = (int64_t)n_rot * n_groups;
  for (int u = 0; u < kVisitItems; ++u) {
    const int64_t wv = w0 + u;
    if (wv >= n_visits) break;  // whole waves leave the loop together
    const int j = (int)(wv / n_groups), t = (int)(wv - (int64_t)j * n_groups);
    const int i = t * kVisitPx + lane;
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
    if (i < n_pix && mask[i]) {
      double m[9];
      load_rot(rot, j, m);
      const Corner c = brick_corner(m, q[3 * (int64_t)i], q[3 * (int64_t)i + 1], q[3 * (int64_t)i + 2], 0.5 * N);
      axis_bricks(c.bx, N, lo[0], hi[0]);
      axis_bricks(c.by, N, lo[1], hi[1]);
      axis_bricks(c.bz, N, lo[2], hi[2]);
      if (lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2])  // no corner inside the grid
        lo[0] = lo[1] = lo[2] = INT_MAX, hi[0] = hi[1] = hi[2] = INT_MIN;
    }
    const int x0 = wmin(lo[0]), y0 = wmin(lo[1]), z0 = wmin(lo[2]);
    const int x1 = wmax(hi[0]), y1 = wmax(hi[1]), z1 = wmax(hi[2]);
    if (x0 > x1) continue;  // uniform: no used pixel reaches the grid
    for (int bx = x0; bx <= x1; ++bx)
      for (int by = y0; by <= y1; ++by)
        for (int bz = z0; bz <= z1; ++bz) {
          const bool hit = bx >= lo[0] && bx <= hi[0] && by >= lo[1] && by <= hi[1] && bz >= lo[2] && bz <= hi[2];
          if (__ballot(hit) == 0) continue;
          if (lane == 0) {
            const int brick = (bx * nb + by) * nb + bz, id = j * n_groups + t;
            if (!local) {
              direct(brick, id);
            } else if constexpr (!FILL) {
              atomicAdd(&tally[brick], 1);
            } else {
              const int h = atomicAdd(&n_hits, 1);
              if (h < kVisitListCap) {
                hits[h] = make_int2(brick, id);
                atomicAdd(&tally[brick], 1);
              } else {
                direct(brick, id);
              }
            }
          }
        }
  }
  __syncthreads();
  if (!local) return;  // uniform
  if constexpr (!FILL) {
    for (int b = threadIdx.x; b < n_bricks; b += 256)
      if (tally[b] > 0) atomicAdd(cnt + b, tally[b]);
  } else {
    for (int b = threadIdx.x; b < n_bricks; b += 256) {
      base[b] = tally[b] > 0 ? atomicAdd(cnt + b, tally[b]) : 0;
      tally[b] = 0;  // the same thread read it: now this brick's local cursor
    }
    __syncthreads();
    const int nh = n_hits < kVisitListCap ? n_hits : kVisitListCap;
    for (int h = threadIdx.x; h < nh; h += 256) {
      const int brick = hits[h].x;
      const int slot = base[brick] + atomicAdd(&tally[brick], 1);
      if (off[brick] + slot < off[brick + 1]) visits[off[brick] + slot] = hits[h].y;
    }
  }
}

// One workgroup per work item (brick, first visit, end visit).  Waves take the
// item's visits in turn, the next visit's loads issued before the current one's
// arithmetic; every corner inside the brick goes to LDS; the brick is then added
// to num/den (device-scope FP64 atomics: other items of the brick may run at once).
__global__ __launch_bounds__(kBrickWaves * 64) void brick_scatter_kernel(const int4* __restrict__ items,
                                                            const int* __restrict__ visits, int n_groups,
                                                            const float* __restrict__ Wp, int64_t stride,
                                                            const double* __restrict__ rho,
                                                            const float* __restrict__ q,
                                                            const uint8_t* __restrict__ mask,
                                                            const double* __restrict__ rot, int n_pix, int N, int nb,
                                                            double* __restrict__ num, double* __restrict__ den) {
  __shared__ double s_num[kBrickVox];
  __shared__ double s_den[kBrickVox];
  const int4 item = items[blockIdx.x];
  const int X0 = item.x / (nb * nb) * kBrick, Y0 = item.x / nb % nb * kBrick, Z0 = item.x % nb * kBrick;
  for (int e = threadIdx.x; e < kBrickVox; e += kBrickWaves * 64) {
    s_num[e] = 0.0;
    s_den[e] = 0.0;
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const double h = 0.5 * N;
  // This wave's visits are first + kBrickWaves * k, k < n_mine.  Everything a visit
  // needs arrives through vector loads (LDS atomics and scalar loads share one
  // wait counter: a scalar load in the loop would make every atomic wait for the
  // ones before it) issued ahead in two stages: the visit entry two visits ahead,
  // then R_j and rho_j (lanes 0..9, broadcast with readlane) and the pixel data one
  // visit ahead.  Every load is unconditional with its index clamped in bounds, so
  // the waits count exactly the loads still needed.
  const int first = item.y + wave;
  const int n_mine = first < item.z ? (item.z - first + kBrickWaves - 1) / kBrickWaves : 0;
  if (n_mine > 0) {
    auto load_entry = [&](int k) {  // lane 0 gets visit k's entry (lane 1 the next one's)
      int kk = k + (lane & 1);
      kk = kk < n_mine ? kk : 0;
      return visits[first + kk * kBrickWaves];
    };
    struct Data {
      double rr;  // lane k < 9: R_j[k]; lanes >= 9: rho_j
      float qx, qy, qz, w;
      uint8_t mk;
      bool inb;
    };
    auto load_data = [&](int e) {
      const int jj = e / n_groups;
      const int ii = (e - jj * n_groups) * kVisitPx + lane;
      Data d;
      d.inb = ii < n_pix;
      const int ic = d.inb ? ii : 0;
      d.rr = *(lane < 9 ? rot + 9 * (int64_t)jj + lane : rho + jj);
      d.mk = mask[ic];
      d.qx = q[3 * (int64_t)ic];
      d.qy = q[3 * (int64_t)ic + 1];
      d.qz = q[3 * (int64_t)ic + 2];
      d.w = Wp[(int64_t)jj * stride + ic];
      return d;
    };
    int e_next = load_entry(1);
    Data cur = load_data(__builtin_amdgcn_readlane(load_entry(0), 0));
    for (int k = 0; k < n_mine; ++k) {
      const int e_after = load_entry(k + 2);
      const Data nxt = load_data(__builtin_amdgcn_readlane(e_next, 0));
      double m[9];
#pragma unroll
      for (int r = 0; r < 9; ++r) m[r] = readlane_f64(cur.rr, r);
      const double rj = readlane_f64(cur.rr, 9);
      if (cur.inb && cur.mk) {
        const Corner c = brick_corner(m, cur.qx, cur.qy, cur.qz, h);
        const double wn = cur.w;
        const int lx = c.bx - X0, ly = c.by - Y0, lz = c.bz - Z0;
        // Each axis's two corners: inside this brick and inside the grid (a partial
        // brick ends at N), and their weights.  A corner's weight is (wx * wy) * wz,
        // the x-y products formed once for both z corners; its LDS slot is
        // lds_slot(lx + dx, ly + dy, lz + dz) with the row and the z rotation split
        // into a per-pixel part and compile-time corner offsets.  Corners of zero
        // weight add zeros (the plan lists their brick all the same).
        const bool vx[2] = {(unsigned)lx < (unsigned)kBrick && c.bx < N,
                            (unsigned)(lx + 1) < (unsigned)kBrick && c.bx + 1 < N};
        const bool vy[2] = {(unsigned)ly < (unsigned)kBrick && c.by < N,
                            (unsigned)(ly + 1) < (unsigned)kBrick && c.by + 1 < N};
        const bool vz[2] = {(unsigned)lz < (unsigned)kBrick && c.bz < N,
                            (unsigned)(lz + 1) < (unsigned)kBrick && c.bz + 1 < N};
        const double wx[2] = {1.0 - c.tx, c.tx}, wy[2] = {1.0 - c.ty, c.ty}, wz[2] = {1.0 - c.tz, c.tz};
        const int rz = __mul24(lx, 13) + __mul24(ly, 7) + lz, par = lx & 1;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int dx = a >> 1, dy = a & 1;
          if (!(vx[dx] && vy[dy])) continue;
          const double wxy = wx[dx] * wy[dy];
          const int row = ((lx + dx) * kBrick + ((ly + dy) ^ par ^ dx)) * kBrick;
#pragma unroll
          for (int dz = 0; dz < 2; ++dz) {
            if (!vz[dz]) continue;
            const double f = wxy * wz[dz];
            const int e = row + ((rz + 13 * dx + 7 * dy + dz) & (kBrick - 1));
            atomicAdd(s_num + e, f * wn);
            atomicAdd(s_den + e, f * rj);
          }
        }
      }
      cur = nxt;
      e_next = e_after;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kBrickVox; e += kBrickWaves * 64) {
    const int vx = X0 + (e >> 8), vy = Y0 + ((e >> 4) & 15), vz = Z0 + (e & 15);
    if (vx >= N || vy >= N || vz >= N) continue;
    const int64_t l = ((int64_t)vx * N + vy) * N + vz;
    const int sl = lds_slot(e >> 8, (e >> 4) & 15, e & 15);
    const double a = s_num[sl], b = s_den[sl];
    if (a != 0.0) unsafeAtomicAdd(num + l, a);
    if (b != 0.0) unsafeAtomicAdd(den + l, b);
  }
}

int brick_edge() { return kBrick; }

hipError_t launch_brick_rot(const float* quat, int n_rot, double* rot, hipStream_t st) {
  brick_rot_kernel<<<(unsigned)((n_rot + 255) / 256), 256, 0, st>>>(quat, n_rot, rot);
  return hipGetLastError();
}

hipError_t launch_brick_visits(const float* q, const uint8_t* mask, const double* rot, int n_pix, int n_rot,
                               int n_groups, int N, int nb, int* cnt, const int64_t* off, int* visits, hipStream_t st) {
  const int64_t waves = ((int64_t)n_rot * n_groups + kVisitItems - 1) / kVisitItems;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  if (off)
    brick_visit_kernel<true><<<blocks, 256, 0, st>>>(q, mask, rot, n_pix, n_rot, n_groups, N, nb, cnt, off, visits);
  else
    brick_visit_kernel<false><<<blocks, 256, 0, st>>>(q, mask, rot, n_pix, n_rot, n_groups, N, nb, cnt, off, visits);
  return hipGetLastError();
}

hipError_t launch_brick_scatter(const int4* items, int64_t n_items, const int* visits, int n_groups, const float* Wp,
                                int64_t stride, const double* rho, const float* q, const uint8_t* mask,
                                const double* rot, int n_pix, int N, int nb, double* num, double* den,
                                hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  brick_scatter_kernel<<<(unsigned)n_items, kBrickWaves * 64, 0, st>>>(items, visits, n_groups, Wp, stride, rho, q,
                                                                      mask, rot, n_pix, N, nb, num, den);
  return hipGetLastError();
}

}  // namespace emc
