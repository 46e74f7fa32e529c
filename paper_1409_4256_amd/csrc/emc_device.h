// Device helpers and kernel launchers shared by the library's translation units.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace emc {

constexpr double kFloor = 1e-10;  // photons: slices are floored before log and sum

// Rotation matrix of a (not necessarily unit) quaternion (w, x, y, z), Hamilton
// convention, active rotation; dividing by |q|^2 normalises it.
struct Rot {
  double m[9];
};

__device__ __forceinline__ Rot quat_rot(const float* __restrict__ qv) {
  const double w = qv[0], x = qv[1], y = qv[2], z = qv[3];
  const double s = 2.0 / (w * w + x * x + y * y + z * z);
  Rot r;
  r.m[0] = 1.0 - s * (y * y + z * z);
  r.m[1] = s * (x * y - w * z);
  r.m[2] = s * (x * z + w * y);
  r.m[3] = s * (x * y + w * z);
  r.m[4] = 1.0 - s * (x * x + z * z);
  r.m[5] = s * (y * z - w * x);
  r.m[6] = s * (x * z - w * y);
  r.m[7] = s * (y * z + w * x);
  r.m[8] = 1.0 - s * (x * x + y * y);
  return r;
}

// Grid cell of a rotated pixel: the lowest corner (bx, by, bz) of its 2 x 2 x 2
// neighbourhood and the fractional offsets (tx, ty, tz) of grid-frame position p.
struct Cell {
  int bx, by, bz;
  double tx, ty, tz;
};

__device__ __forceinline__ Cell cell_at(const Rot& r, const float* __restrict__ qi, int N) {
  const double qx = qi[0], qy = qi[1], qz = qi[2];
  const double h = 0.5 * N;
  const double px = r.m[0] * qx + r.m[1] * qy + r.m[2] * qz + h;
  const double py = r.m[3] * qx + r.m[4] * qy + r.m[5] * qz + h;
  const double pz = r.m[6] * qx + r.m[7] * qy + r.m[8] * qz + h;
  const double fx0 = floor(px), fy0 = floor(py), fz0 = floor(pz);
  return Cell{(int)fx0, (int)fy0, (int)fz0, px - fx0, py - fy0, pz - fz0};
}

// Trilinear stencil of grid-frame position p: the up to 8 grid points with
// non-zero tent weight.  Points outside the N^3 box get weight 0 (index 0).
struct Stencil {
  int idx[8];
  double w[8];
  int bx, by, bz;  // lowest corner of the 2 x 2 x 2 neighbourhood
};

__device__ __forceinline__ Stencil stencil_at(const Rot& r, const float* __restrict__ qi, int N) {
  const Cell c = cell_at(r, qi, N);
  Stencil s;
  s.bx = c.bx;
  s.by = c.by;
  s.bz = c.bz;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int dx = t >> 2, dy = (t >> 1) & 1, dz = t & 1;
    const int vx = c.bx + dx, vy = c.by + dy, vz = c.bz + dz;
    const bool in = (unsigned)vx < (unsigned)N && (unsigned)vy < (unsigned)N && (unsigned)vz < (unsigned)N;
    const double w = (dx ? c.tx : 1.0 - c.tx) * (dy ? c.ty : 1.0 - c.ty) * (dz ? c.tz : 1.0 - c.tz);
    s.idx[t] = in ? (vx * N + vy) * N + vz : 0;
    s.w[t] = in ? w : 0.0;
  }
  return s;
}

// The trilinear value sum_t w_t model[idx_t] of stencil_at, its terms added in the
// same corner order (the same bits), with the model read as four z-pairs: one
// 8-byte load per (dx, dy), starting at z0 = bz clamped to [0, N - 2] so that the
// pair stays inside its row (N >= 2); a corner outside the grid adds 0, its pair
// read from an in-grid address.
__device__ __forceinline__ double trilinear_at(const float* __restrict__ model, int N, const Rot& r,
                                               const float* __restrict__ qi) {
  const Cell c = cell_at(r, qi, N);
  const int z0 = c.bz < 0 ? 0 : (c.bz > N - 2 ? N - 2 : c.bz);
  double W = 0.0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int dx = p >> 1, dy = p & 1;
    const int vx = c.bx + dx, vy = c.by + dy;
    const bool inxy = (unsigned)vx < (unsigned)N && (unsigned)vy < (unsigned)N;
    float v[2];
    __builtin_memcpy(v, model + (inxy ? ((int64_t)vx * N + vy) * N + z0 : 0), sizeof(v));
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
      const int vz = c.bz + dz;
      const bool in = inxy && (unsigned)vz < (unsigned)N;
      const double w = (dx ? c.tx : 1.0 - c.tx) * (dy ? c.ty : 1.0 - c.ty) * (dz ? c.tz : 1.0 - c.tz);
      W += (in ? w : 0.0) * (double)v[vz == z0 ? 0 : 1];
    }
  }
  return W;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---- launchers (all asynchronous on `st`; return hipGetLastError()) ----
hipError_t launch_fill_zero_f64(double* p, size_t n, hipStream_t st);
// counts [n_data][n_pix] -> K [n_data][ps] and KT [ps][ds] (float or bf16); ds = data stride
hipError_t launch_pack(const uint16_t* counts, const uint8_t* mask, int n_pix, int64_t ps, int64_t n_data,
                       int64_t ds, const int32_t* frames, void* K, void* KT, bool bf16, hipStream_t st);
hipError_t read_range_flag(int* flag, hipStream_t st);  // synchronises `st`
hipError_t launch_centre(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                         int n_pix, int64_t stride, int n_rot, double* c, hipStream_t st);
hipError_t launch_expand(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                         int n_pix, int64_t stride, int n_rot, const double* c, float* logW, double* S,
                         hipStream_t st);
// hilo: hi plane [n_rot][stride] bf16 followed by lo plane [n_rot][stride] bf16
hipError_t launch_expand_bf16(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                              int n_pix, int64_t stride, int n_rot, const double* c, void* hilo, double* S,
                              float* scale, hipStream_t st);
hipError_t launch_frame_dot(const void* K, bool bf16, int64_t stride, int64_t n_data, const double* c, double* b,
                            hipStream_t st);
// C[M][N] = sum_k A[m][k] B[n][k] (both operands contiguous along k), FP32 MFMA;
// Kd must be a multiple of 32; rows m >= M and n >= N read as zero.
hipError_t launch_gemm_f32_nt(const float* A, const float* B, float* C, int64_t M, int64_t N, int64_t Kd,
                              int64_t lda, int64_t ldb, int64_t ldc, hipStream_t st, bool network = false);
// BF16 MFMA, FP32 accumulation; Kd multiple of 32.  DUAL: C = row_scale[m] * (A_hi + A_lo) B^T.
hipError_t launch_gemm_bf16_dual_nt(const void* A_hi, const void* A_lo, const void* B, const float* row_scale,
                                    float* C, int64_t M, int64_t N, int64_t Kd, int64_t lda, int64_t ldb, int64_t ldc,
                                    hipStream_t st);
hipError_t launch_gemm_bf16_nt(const void* A, const void* B, float* C, int64_t M, int64_t N, int64_t Kd, int64_t lda,
                               int64_t ldb, int64_t ldc, hipStream_t st);
// The same product with its k range cut in `splits` parts: part s writes its
// partial product to C + s * M * ldc.  `splits` must come from gemm_bf16_splits.
int gemm_bf16_splits(int64_t M, int64_t N, int64_t Kd, int max_splits);
hipError_t launch_gemm_bf16_nt_split(const void* A, const void* B, float* C, int64_t M, int64_t N, int64_t Kd,
                                     int64_t lda, int64_t ldb, int64_t ldc, int splits, hipStream_t st);
hipError_t launch_gemm_bf16_dual_nt_split(const void* A_hi, const void* A_lo, const void* B, const float* row_scale,
                                          float* C, int64_t M, int64_t N, int64_t Kd, int64_t lda, int64_t ldb,
                                          int64_t ldc, int splits, hipStream_t st);
// out[e] = sum over s < parts of part[s * n + e], in order of s
hipError_t launch_sum_slabs(const float* part, int parts, int64_t n, float* out, hipStream_t st);
// part: NULL, or kMaxLseChunks * 2 * n_data doubles of scratch that lets few frames
// split the rotations over more workgroups
constexpr int kMaxLseChunks = 64;
hipError_t launch_lse_stats(const float* G, int64_t ld, int n_rot, int64_t n_data, const double* log_w,
                            const double* S, const double* b, double* stats, double* part, hipStream_t st);
hipError_t launch_lse_finish(const double* stats, int64_t n_data, double* L, hipStream_t st);
hipError_t launch_lse_write_f32(const float* G, int64_t ldg, float* P, int64_t ldp, int n_rot, int64_t n_data,
                                const double* log_w, const double* S, const double* b, const double* L,
                                double* rho, hipStream_t st);
hipError_t launch_lse_write_bf16(const float* G, int64_t ldg, void* P, int64_t ldp, int n_rot, int64_t n_data,
                                 const double* log_w, const double* S, const double* b, const double* L,
                                 double* rho, hipStream_t st);
hipError_t launch_scatter(const float* Wp, int64_t stride, const double* rho, const float* q,
                          const uint8_t* mask, const float* quat, int n_pix, int n_rot, int N, double* num,
                          double* den, double* copies, hipStream_t st);
// ---- Gaussian noise model with fluence (gauss.hip) ----
hipError_t launch_gauss_expand(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                               int n_pix, int64_t stride, int n_rot, double* c, float* A, double* s2, hipStream_t st);
hipError_t launch_frame_sq(const float* K, int64_t stride, int64_t n_data, double* k2, hipStream_t st);
hipError_t launch_gauss_estep(float* Gd, float* phi, float* P, int64_t ld, int n_rot, int64_t n_data,
                              const double* log_w, const double* s2, const double* b, const double* k2, int own,
                              double sigma, double* stats, double* L, double* rho, hipStream_t st);

int brick_edge();
hipError_t launch_brick_rot(const float* quat, int n_rot, double* rot, hipStream_t st);
hipError_t launch_brick_visits(const float* q, const uint8_t* mask, const double* rot, int n_pix, int n_rot,
                               int n_groups, int N, int nb, int* cnt, const int64_t* off, int* visits, hipStream_t st);
hipError_t launch_brick_scatter(const int4* items, int64_t n_items, const int* visits, int n_groups, const float* Wp,
                                int64_t stride, const double* rho, const float* q, const uint8_t* mask,
                                const double* rot, int n_pix, int N, int nb, double* num, double* den,
                                hipStream_t st);
hipError_t launch_divide(const double* num, const double* den, const float* prev, float* out, int64_t M,
                         hipStream_t st);
hipError_t launch_mean(const double* L, int64_t n, double* out, hipStream_t st);

// ---- contents check (validate.hip) ----
constexpr int32_t kValidQuat = 1, kValidWeight = 2, kValidPixel = 4, kValidModel = 8;
hipError_t launch_validate(const float* quat, int64_t n_rot, const float* q, const uint8_t* mask, int64_t n_pix,
                           const double* log_w, const float* model, int64_t n_grid, double tol, int32_t* flags,
                           hipStream_t st);

// ---- proposal network (cnn.hip) ----
hipError_t launch_bin_log(const void* K, bool bf16, int64_t ps, int n_pix, const int32_t* bins, const int32_t* frames,
                          int B, float* x, hipStream_t st);
hipError_t launch_im2col(const float* in, int CI, int IH, int64_t M, float* colT, hipStream_t st);
hipError_t launch_col2im(const float* dcolT, int CI, int IH, int64_t nB, float* din, hipStream_t st);
hipError_t launch_flatten(const float* src, int C, int P, int64_t nB, float* dst, bool to_flat, hipStream_t st);
hipError_t launch_row_sum(const float* X, int rows, int64_t cols, float* part, float* out, hipStream_t st);
int gemm_str_splits(int M, int N, int64_t K);
hipError_t launch_gemm_str(bool a_kcontig, const float* A, int64_t lda, bool b_kcontig, const float* B, int64_t ldb,
                           float* C, int64_t ldc, int M, int N, int64_t K, int splits, float* part,
                           const float* bias, bool relu, hipStream_t st);
hipError_t launch_relu_mask(float* g, const float* act, int64_t n, hipStream_t st);
hipError_t launch_add_bias(float* z, const float* bias, int64_t rows, int cols, hipStream_t st);
hipError_t launch_col_sum(const float* X, int rows, int cols, float* out, hipStream_t st);
hipError_t launch_softmax_xent(const float* z, const float* T, int n_cells, int B, float* dz, double* loss,
                               hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st);
hipError_t launch_topk(const float* z, int64_t rows, int n_cells, int k, bool positive, int32_t* out,
                       hipStream_t st);
hipError_t launch_topk_union(const int32_t* a, int ka, const int32_t* b, int kb, int64_t rows, int n_cells,
                             int32_t* out, hipStream_t st);
hipError_t launch_cell_targets(const void* P, bool bf16, int64_t ldp, int64_t n_data, const int32_t* cell_ptr,
                               const int32_t* cell_rot, int n_cells, float* T, hipStream_t st);

// ---- learned-proposal E/M steps (proposal.hip) ----
hipError_t launch_assign_cells(const float* quat, int n_rot, const float* coarse, int n_cells, int32_t* cell_of,
                               hipStream_t st);
hipError_t launch_counting_sort(const int32_t* keys, int64_t n, int nk, int32_t* hist, int32_t* cursor,
                                int64_t* ptr, int32_t* order, float* payload_unused, hipStream_t st);
hipError_t launch_scan(const int32_t* cnt, int64_t n, int64_t* ptr, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_cand_mask(const int32_t* topk, int k_top, const int32_t* frames, int64_t n_frames, int words,
                            uint32_t* mask, hipStream_t st);
hipError_t launch_cand_cells(const int32_t* topk, int k_top, const int32_t* frames, int64_t n_frames, int n_cells,
                             int32_t* cells, int32_t* keys, hipStream_t st);
// packs of neighbouring cells (at most kPackRot rotations in all; a cell with more is a pack of its own)
constexpr int kPackRot = 16;  // the packing cap: one 16-row MFMA tile (<= the candidate kernels' group of 32)
hipError_t launch_packs(const float* coarse, int n_cells, const int64_t* cell_ptr, const int32_t* cell_of,
                        const int32_t* cell_rot, int n_rot, int32_t* nn, int32_t* pack_of, int32_t* slot_cell,
                        int32_t* pack_slot, int32_t* n_packs, int32_t* slot_cnt, int64_t* slot_ptr, int32_t* cell_slot,
                        int32_t* cell_first, int64_t* pack_ptr, int32_t* pack_rot, int32_t* rot_local,
                        hipStream_t st);
hipError_t launch_pack_pairs(const int32_t* cells, int k_top, int64_t n_frames, const int32_t* pack_of,
                             const int32_t* cell_slot, const int32_t* pack_slot, int n_cells, int32_t* keys,
                             uint32_t* bits, int32_t* prim, hipStream_t st);
hipError_t launch_pack_columns(const int32_t* order, const int64_t* cf_ptr, int n_cells, int64_t n_pairs, int k_top,
                               const int32_t* keys, const uint32_t* bits, const int32_t* prim, int32_t* cf_frame,
                               uint32_t* cf_mask, int32_t* pair_col, hipStream_t st);
hipError_t launch_scan64(const int64_t* cnt, int64_t n, int64_t* ptr, hipStream_t st);

// ---- candidate E/M steps (cand.hip) ----
hipError_t launch_cand_loglik(const int2* tiles, int64_t n_tiles, const int4* groups, const int64_t* grp_off,
                              const int64_t* cf_ptr, const int32_t* cf_frame, const void* runs, const void* chunks,
                              const int32_t* cell_rot, const void* hilo, int64_t plane, const float* scale, int64_t ps,
                              float* G, hipStream_t st);
hipError_t launch_cand_estep(const float* G, void* P, const int4* groups, const int64_t* grp_off,
                             const int64_t* cg_ptr, const int32_t* cells, const int32_t* pair_col, int k_top,
                             int64_t n_frames, const int32_t* pack_of, const int32_t* cell_first,
                             const int64_t* cell_ptr, const int32_t* pack_rot, const int32_t* rot_local, int64_t n_rot,
                             const double* log_w, const double* S, double* cst, const double* b, double* L, void* Pd,
                             int64_t ldd, const int2* tiles, int64_t n_tiles, const int64_t* cf_ptr,
                             const int32_t* cf_frame, const uint32_t* cf_mask, hipStream_t st);
hipError_t launch_cand_mstep(const int4* groups, const int64_t* grp_off, int64_t n_groups, const int64_t* cf_ptr,
                             const int32_t* cf_frame, const void* runs, int64_t n_list, const void* chunks,
                             const int32_t* dense_band, const void* P, const int32_t* cell_rot, int64_t ps, float* Wp,
                             double* rho, const double* rho_a, bool accumulate, hipStream_t st);
hipError_t launch_dense_bands(const int32_t* cnt, int64_t n_frames, int nbands, float* mean, int32_t* dense_band,
                              int32_t* dense_list, int32_t* n_dense, hipStream_t st);
hipError_t launch_dense_pack(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                             int64_t n_frames, int64_t ld, int n_dense, const int32_t* dense_list, void* KT,
                             hipStream_t st);
// Wp[j][dense pixels] += sum over the `parts` slabs of D (n_rot x n_dense*128 each), in slab order
hipError_t launch_dense_add(const float* D, int parts, int64_t n_rot, int n_dense, const int32_t* dense_list,
                            int64_t ps, float* Wp, hipStream_t st);
hipError_t launch_fill_zero_bytes(void* p, int64_t bytes, hipStream_t st);
// when *recall < recall_min: Wp[0..n) = 0 and rho[0..n_rot) = 0 (n a multiple of 4)
hipError_t launch_gate_zero(const double* recall, double recall_min, float* Wp, int64_t n, double* rho, int64_t n_rot,
                            hipStream_t st);
hipError_t launch_band_count(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                             int64_t n_frames, int nbands, int32_t* cnt, int32_t* over, hipStream_t st);
hipError_t launch_band_fill(const uint16_t* counts, const uint8_t* mask, int n_pix, const int32_t* frames,
                            int64_t n_frames, int nbands, const void* runs, void* chunks, hipStream_t st);
// run records of the chunk layout: 16 bytes per (frame, run of 8 bands), run_count(nbands) per frame,
// frame-major, then a run-major copy
int run_count(int nbands);
hipError_t launch_run_table(const int64_t* ptr, int64_t n_frames, int nbands, void* runs, hipStream_t st);
hipError_t launch_band_dot(const void* runs, int nbands, const void* chunks, int64_t n_frames, const double* c,
                           double* b, hipStream_t st);
hipError_t launch_pack_groups(const int64_t* cell_ptr, const int64_t* cf_ptr, int n_cells, int32_t* cnt,
                              int64_t* cg_ptr, int4* groups, int64_t* gsize, int64_t* grp_off, int64_t g_max,
                              hipStream_t st);
hipError_t launch_group_tiles(const int4* groups, const int64_t* cg_ptr, int n_cells, const int64_t* cf_ptr,
                              int32_t* xcd_of, int2* tiles, int64_t cap, int64_t* n_tiles, hipStream_t st);
hipError_t launch_dup_check(const int32_t* cells, int k_top, int64_t n_frames, int n_cells, int32_t* flag,
                            hipStream_t st);
hipError_t launch_audit_recall(const void* P, int64_t ldp, int n_rot, int64_t n_audit, const uint32_t* mask_audit,
                               int words, const int32_t* cell_of, double* recall, hipStream_t st);

}  // namespace emc
