// Gaussian noise model with photon fluence (Section 2.2): the paper's own
// likelihood
//     Q_jk = -sum_i (K_ik / phi_jk - W_ij)^2 / (2 sigma^2)                 eq. (2.2)-(2.3)
// expanded as -(k2_k / phi^2 - 2 G_jk / phi + s2_j) / (2 sigma^2) with
// k2_k = sum_i K_ik^2, s2_j = sum_i W_ij^2 and the contraction G_jk = sum_i W_ij K_ik,
// which runs on the FP32 MFMA GEMM of the Poisson form.  As there, the slices are
// centred: A_ji = W_ij - c_i with c_i the mean over a fixed subset of rotations,
// and b_k = sum_i K_ik c_i is added back in FP64, which shrinks the GEMM's
// accumulated magnitude where the photons are (low q, where the slices of all
// rotations nearly agree).  The fluence update of eq. (2.6), phi_jk = k2_k / G_jk,
// comes from the same G.  The M-step numerator of eq. (2.11) contracts
// P_jk / phi_jk with the frames (the same GEMM as the Poisson M-step), and the
// c-step's weight stays rho_j = sum_k P_jk (eq. (2.12)).
#include "emc_device.h"
#include "lse.h"

namespace emc {

// c_i = mean over a fixed subset of <= 64 rotations of W_ij (no floor: no logarithm).
__global__ __launch_bounds__(256) void gauss_centre_kernel(const float* __restrict__ model, int N,
                                                           const float* __restrict__ q,
                                                           const uint8_t* __restrict__ mask,
                                                           const float* __restrict__ quat, int n_pix,
                                                           int64_t stride, int n_rot, double* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= stride) return;
  if (i >= n_pix || !mask[i]) {
    c[i] = 0.0;
    return;
  }
  const int nc = n_rot < 64 ? n_rot : 64;
  double acc = 0.0;
  for (int t = 0; t < nc; ++t) {
    const int j = (int)(((int64_t)t * n_rot) / nc);
    const Rot r = quat_rot(quat + 4 * (int64_t)j);
    acc += trilinear_at(model, N, r, q + 3 * i);
  }
  c[i] = acc / nc;
}

// One workgroup per rotation j (eq. (2.9)): A_ji = W_ij - c_i (FP32, 0 at masked and
// padding pixels) and s2_j = sum_i W_ij^2 (FP64, block-reduced in a fixed order).
__global__ __launch_bounds__(256) void gauss_expand_kernel(const float* __restrict__ model, int N,
                                                           const float* __restrict__ q,
                                                           const uint8_t* __restrict__ mask,
                                                           const float* __restrict__ quat, int n_pix,
                                                           int64_t stride, const double* __restrict__ c,
                                                           float* __restrict__ A, double* __restrict__ s2) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const Rot r = quat_rot(quat + 4 * (int64_t)j);
  float* row = A + (int64_t)j * stride;
  double sum = 0.0;
  for (int64_t i = threadIdx.x; i < stride; i += 256) {
    float out = 0.0f;
    if (i < n_pix && mask[i]) {
      const double W = trilinear_at(model, N, r, q + 3 * i);
      sum += W * W;
      out = (float)(W - c[i]);
    }
    row[i] = out;
  }
  sum = wave_sum(sum);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) s2[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// k2_k = sum_i K_ik^2 in FP64 (masked and padding pixels are 0 in K): one wave per frame.
__global__ __launch_bounds__(256) void frame_sq_kernel(const float* __restrict__ K, int64_t stride, int64_t n_data,
                                                       double* __restrict__ k2) {
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n_data) return;  // uniform per wave
  const float* row = K + k * stride;
  double acc = 0.0;
  for (int64_t i = lane; i < stride; i += 64) {
    const double v = row[i];
    acc += v * v;
  }
  acc = wave_sum(acc);
  if (lane == 0) k2[k] = acc;
}

// Log-joint a_jk = Q_jk + log w_j with the fluence phi^(n) (own: the update of this
// iteration's slices), and that update phi^(n+1) (1 where G <= 0: no photons).
struct GaussTerm {
  double a, phi_used, phi_next;
};

__device__ __forceinline__ GaussTerm gauss_term(float gd, double bk, double k2k, double s2j, double lwj,
                                                float phi_in, bool own, double inv2s2) {
  const double G = (double)gd + bk;
  const double pn = G > 0.0 ? k2k / G : 1.0;
  const double pu = own ? pn : (double)phi_in;
  const double ss = k2k / (pu * pu) - 2.0 * G / pu + s2j;
  GaussTerm t;
  t.a = lwj - ss * inv2s2;
  t.phi_used = pu;
  t.phi_next = pn;
  return t;
}

constexpr int kGaussFrames = 64;  // frames per statistics workgroup: one per lane, 4 waves split the rotations

// Per-frame (max, sum exp) of a_jk over the rotations, FP64, online (eq. (2.4)).
__global__ __launch_bounds__(256) void gauss_stats_kernel(const float* __restrict__ Gd, const float* __restrict__ phi,
                                                          int64_t ld, int n_rot, int64_t n_data,
                                                          const double* __restrict__ log_w,
                                                          const double* __restrict__ s2,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ k2, int own, double inv2s2,
                                                          double* __restrict__ stats) {
  __shared__ double sm[4][kGaussFrames], ss[4][kGaussFrames];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * kGaussFrames + lane;
  const bool live = k < n_data;
  const double bk = live ? b[k] : 0.0, k2k = live ? k2[k] : 0.0;
  double m = -INFINITY, s = 0.0;
  if (live) {
    const ExpCoef ec = exp_coef();
    for (int j = wave; j < n_rot; j += 4) {
      const int64_t e = (int64_t)j * ld + k;
      const GaussTerm t = gauss_term(Gd[e], bk, k2k, s2[j], log_w[j], own ? 1.0f : phi[e], own, inv2s2);
      lse_push(m, s, t.a, ec);  // zero prior weight (a = -inf): no contribution
    }
  }
  sm[wave][lane] = m;
  ss[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && live) {
    for (int w = 1; w < 4; ++w) lse_merge(m, s, sm[w][lane], ss[w][lane]);
    stats[2 * k] = m;
    stats[2 * k + 1] = s;
  }
}

constexpr int kGaussRows = 8;  // rotations per workgroup of the write pass

// P_jk = exp(a_jk - L_k) (FP32) into P; P_jk / phi_jk (the M-step operand, eq. (2.11))
// over Gd; phi^(n+1) over phi; rho_j = sum_k P_jk (as stored), block-reduced in a
// fixed order.  Padding frames get P = 0 and phi = 1.
__global__ __launch_bounds__(256) void gauss_write_kernel(float* Gd, float* phi, float* __restrict__ P, int64_t ld,
                                                          int n_rot, int64_t n_data, const double* __restrict__ log_w,
                                                          const double* __restrict__ s2,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ k2,
                                                          const double* __restrict__ L, int own, double inv2s2,
                                                          double* __restrict__ rho) {
  __shared__ double red[kGaussRows][4];
  const int j0 = blockIdx.x * kGaussRows;
  double acc[kGaussRows];
#pragma unroll
  for (int r = 0; r < kGaussRows; ++r) acc[r] = 0.0;
  for (int64_t k = threadIdx.x; k < ld; k += 256) {
    const bool live = k < n_data;
    const double bk = live ? b[k] : 0.0, k2k = live ? k2[k] : 0.0, Lk = live ? L[k] : 0.0;
#pragma unroll
    for (int r = 0; r < kGaussRows; ++r) {
      const int j = j0 + r;
      if (j >= n_rot) break;
      const int64_t e = (int64_t)j * ld + k;
      float p = 0.0f, pp = 0.0f, pn = 1.0f;
      if (live) {
        const GaussTerm t = gauss_term(Gd[e], bk, k2k, s2[j], log_w[j], own ? 1.0f : phi[e], own, inv2s2);
        p = (float)exp(t.a - Lk);
        pp = (float)((double)p / t.phi_used);
        pn = (float)t.phi_next;
      }
      P[e] = p;
      Gd[e] = pp;
      phi[e] = pn;
      acc[r] += (double)p;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < kGaussRows; ++r) {
    const double v = wave_sum(acc[r]);
    if (lane == 0) red[r][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kGaussRows && j0 + (int)threadIdx.x < n_rot) {
    const int r = threadIdx.x;
    rho[j0 + r] = (red[r][0] + red[r][1]) + (red[r][2] + red[r][3]);
  }
}

hipError_t launch_gauss_expand(const float* model, int N, const float* q, const uint8_t* mask, const float* quat,
                               int n_pix, int64_t stride, int n_rot, double* c, float* A, double* s2,
                               hipStream_t st) {
  gauss_centre_kernel<<<(unsigned)((stride + 255) / 256), 256, 0, st>>>(model, N, q, mask, quat, n_pix, stride, n_rot,
                                                                        c);
  gauss_expand_kernel<<<(unsigned)n_rot, 256, 0, st>>>(model, N, q, mask, quat, n_pix, stride, c, A, s2);
  return hipGetLastError();
}

hipError_t launch_frame_sq(const float* K, int64_t stride, int64_t n_data, double* k2, hipStream_t st) {
  if (n_data == 0) return hipSuccess;
  frame_sq_kernel<<<(unsigned)((n_data + 3) / 4), 256, 0, st>>>(K, stride, n_data, k2);
  return hipGetLastError();
}

hipError_t launch_gauss_estep(float* Gd, float* phi, float* P, int64_t ld, int n_rot, int64_t n_data,
                              const double* log_w, const double* s2, const double* b, const double* k2, int own,
                              double sigma, double* stats, double* L, double* rho, hipStream_t st) {
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
  if (n_data > 0) {
    gauss_stats_kernel<<<(unsigned)((n_data + kGaussFrames - 1) / kGaussFrames), 256, 0, st>>>(
        Gd, phi, ld, n_rot, n_data, log_w, s2, b, k2, own, inv2s2, stats);
    const hipError_t e = launch_lse_finish(stats, n_data, L, st);
    if (e != hipSuccess) return e;
  }
  gauss_write_kernel<<<(unsigned)((n_rot + kGaussRows - 1) / kGaussRows), 256, 0, st>>>(
      Gd, phi, P, ld, n_rot, n_data, log_w, s2, b, k2, L, own, inv2s2, rho);
  return hipGetLastError();
}

}  // namespace emc
