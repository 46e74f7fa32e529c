// Learned orientation proposal: a small CNN scoring the cells of a coarse
// rotation grid from a log-binned frame (FP32 throughout).
//   x = log1p(binned frame) 1x64x64 -> 4 x [conv3x3 s2 p1 + bias + ReLU]
//   (1->32->64->128->128 channels) -> flatten 2048 -> linear -> n_cells logits
// Forward, backward (data and weight gradients), soft-target cross entropy,
// Adam and top-K selection are all kernels here; the fully connected layer
// uses the FP32 MFMA GEMM forward and a small LDS-tiled GEMM backward.
#include "emc_device.h"

namespace emc {

constexpr int kImg = 64;

// --------------------------------------------------------------------- preprocessing
// One workgroup per frame: per-bin sums in LDS, then log1p.
template <typename T>
__global__ __launch_bounds__(256) void bin_log_kernel(const T* __restrict__ K, int64_t ps, int n_pix,
                                                      const int32_t* __restrict__ bins,
                                                      const int32_t* __restrict__ frames, float* __restrict__ x) {
  __shared__ float img[kImg * kImg];
  const int b = blockIdx.x;
  const int64_t k = frames ? frames[b] : b;
  for (int e = threadIdx.x; e < kImg * kImg; e += 256) img[e] = 0.0f;
  __syncthreads();
  const T* row = K + k * ps;
  for (int i = threadIdx.x; i < n_pix; i += 256) {
    const int bi = bins[i];
    if (bi >= 0) atomicAdd(&img[bi], (float)row[i]);
  }
  __syncthreads();
  float* out = x + (int64_t)b * kImg * kImg;
  for (int e = threadIdx.x; e < kImg * kImg; e += 256) out[e] = log1pf(img[e]);
}

// --------------------------------------------------------------------- convolutions
// out[n][o][y][x] = relu(b[o] + sum_{c,dy,dx} w[o][c][dy][dx] in[n][c][2y-1+dy][2x-1+dx])
template <int CI, int CO, int IH>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float* __restrict__ in, const float* __restrict__ w,
                                                       const float* __restrict__ bias, float* __restrict__ out,
                                                       int B) {
  constexpr int OH = IH / 2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * CO * OH * OH) return;
  const int ox = e % OH, oy = (e / OH) % OH, o = (e / (OH * OH)) % CO;
  const int64_t n = e / ((int64_t)CO * OH * OH);
  float acc = bias[o];
  const float* ib = in + n * CI * IH * IH;
  const float* wo = w + o * CI * 9;
  for (int c = 0; c < CI; ++c) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int iy = 2 * oy - 1 + dy;
      if (iy < 0 || iy >= IH) continue;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int ix = 2 * ox - 1 + dx;
        if (ix < 0 || ix >= IH) continue;
        acc += wo[c * 9 + dy * 3 + dx] * ib[(c * IH + iy) * IH + ix];
      }
    }
  }
  out[e] = fmaxf(acc, 0.0f);
}

// dIn[n][c][iy][ix] = sum_{o,dy,dx : 2y-1+dy = iy, 2x-1+dx = ix} w[o][c][dy][dx] dOut[n][o][y][x]
template <int CI, int CO, int IH>
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(const float* __restrict__ dout,
                                                            const float* __restrict__ w, float* __restrict__ din,
                                                            int B) {
  constexpr int OH = IH / 2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * CI * IH * IH) return;
  const int ix = e % IH, iy = (e / IH) % IH, c = (e / (IH * IH)) % CI;
  const int64_t n = e / ((int64_t)CI * IH * IH);
  float acc = 0.0f;
  const float* db = dout + n * CO * OH * OH;
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    const int ty = iy + 1 - dy;
    if (ty < 0 || (ty & 1) || (ty >> 1) >= OH) continue;
    const int y = ty >> 1;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int tx = ix + 1 - dx;
      if (tx < 0 || (tx & 1) || (tx >> 1) >= OH) continue;
      const int xx = tx >> 1;
      for (int o = 0; o < CO; ++o) acc += w[(o * CI + c) * 9 + dy * 3 + dx] * db[(o * OH + y) * OH + xx];
    }
  }
  din[e] = acc;
}

// dW[o][c][dy][dx] = sum_{n,y,x} dOut[n][o][y][x] in[n][c][2y-1+dy][2x-1+dx]; one workgroup per (o, c).
// The workgroup with c == 0 also reduces dBias[o].
template <int CI, int CO, int IH>
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const float* __restrict__ in,
                                                              const float* __restrict__ dout,
                                                              float* __restrict__ dw, float* __restrict__ db, int B) {
  constexpr int OH = IH / 2;
  __shared__ float red[10][4];
  const int o = blockIdx.x / CI, c = blockIdx.x % CI;
  float acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = 0.0f;
  const int64_t total = (int64_t)B * OH * OH;
  for (int64_t e = threadIdx.x; e < total; e += 256) {
    const int x = e % OH, y = (e / OH) % OH;
    const int64_t n = e / (OH * OH);
    const float g = dout[((n * CO + o) * OH + y) * OH + x];
    if (g == 0.0f) continue;
    const float* ib = in + (n * CI + c) * IH * IH;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int iy = 2 * y - 1 + dy;
      if (iy < 0 || iy >= IH) continue;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int ix = 2 * x - 1 + dx;
        if (ix < 0 || ix >= IH) continue;
        acc[dy * 3 + dx] += g * ib[iy * IH + ix];
      }
    }
    acc[9] += g;
  }
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    float v = wave_sum(acc[t]);
    if ((threadIdx.x & 63) == 0) red[t][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9) dw[(o * CI + c) * 9 + threadIdx.x] = (red[threadIdx.x][0] + red[threadIdx.x][1]) +
                                                          (red[threadIdx.x][2] + red[threadIdx.x][3]);
  if (threadIdx.x == 9 && c == 0) db[o] = (red[9][0] + red[9][1]) + (red[9][2] + red[9][3]);
}

// g *= (act > 0)
__global__ void relu_mask_kernel(float* __restrict__ g, const float* __restrict__ act, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    if (!(act[e] > 0.0f)) g[e] = 0.0f;
}

// z[b][c] += bias[c]
__global__ void add_bias_kernel(float* __restrict__ z, const float* __restrict__ bias, int64_t rows, int cols) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * 256)
    z[e] += bias[e % cols];
}

// --------------------------------------------------------------------- small strided GEMM
// C[m][n] = sum_k A[m*sam + k*sak] B[k*sbk + n*sbn]; 64 x 64 tiles, 4 x 4 per thread.
__global__ __launch_bounds__(256) void gemm_small_kernel(const float* __restrict__ A, int64_t sam, int64_t sak,
                                                         const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                                         float* __restrict__ C, int64_t ldc, int M, int N, int Kd) {
  __shared__ float As[16][64 + 1], Bs[16][64 + 1];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < Kd; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, r = e % 64;
      const int m = m0 + r, n = n0 + r, k = k0 + kk;
      As[kk][r] = (m < M && k < Kd) ? A[m * sam + k * sak] : 0.0f;
      Bs[kk][r] = (n < N && k < Kd) ? B[k * sbk + n * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
      if (m < M && n < N) C[m * ldc + n] = acc[i][j];
    }
}

// column sums: out[c] = sum_r X[r][c]
__global__ void col_sum_kernel(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; ++r) s += X[(int64_t)r * cols + c];
  out[c] = s;
}

// --------------------------------------------------------------------- loss
// Soft-target cross entropy per row; dz = (softmax(z) * sum_c T - T) / B; loss += -sum T log softmax / B.
__global__ __launch_bounds__(256) void softmax_xent_kernel(const float* __restrict__ z, const float* __restrict__ T,
                                                           int n_cells, int B, float* __restrict__ dz,
                                                           double* __restrict__ loss) {
  __shared__ float redf[4];
  __shared__ double redd[4];
  const int b = blockIdx.x;
  const float* zr = z + (int64_t)b * n_cells;
  const float* tr = T + (int64_t)b * n_cells;
  float m = -INFINITY;
  for (int c = threadIdx.x; c < n_cells; c += 256) m = fmaxf(m, zr[c]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) redf[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(redf[0], redf[1]), fmaxf(redf[2], redf[3]));
  __syncthreads();
  double s = 0.0, ts = 0.0, tz = 0.0;
  for (int c = threadIdx.x; c < n_cells; c += 256) {
    s += exp((double)(zr[c] - m));
    ts += tr[c];
    tz += (double)tr[c] * (double)(zr[c] - m);
  }
  s = wave_sum(s);
  ts = wave_sum(ts);
  tz = wave_sum(tz);
  __shared__ double rs[4], rts[4], rtz[4];
  if ((threadIdx.x & 63) == 0) {
    rs[threadIdx.x >> 6] = s;
    rts[threadIdx.x >> 6] = ts;
    rtz[threadIdx.x >> 6] = tz;
  }
  __syncthreads();
  const double S = (rs[0] + rs[1]) + (rs[2] + rs[3]);
  const double TS = (rts[0] + rts[1]) + (rts[2] + rts[3]);
  const double TZ = (rtz[0] + rtz[1]) + (rtz[2] + rtz[3]);
  const double lse = log(S);  // relative to m
  for (int c = threadIdx.x; c < n_cells; c += 256) {
    const double p = exp((double)(zr[c] - m) - lse);
    dz[(int64_t)b * n_cells + c] = (float)((p * TS - (double)tr[c]) / B);
  }
  if (threadIdx.x == 0) atomicAdd(loss, (TS * lse - TZ) / B);
  (void)redd;
}

// --------------------------------------------------------------------- Adam
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gg;
    const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// --------------------------------------------------------------------- top-K
// One workgroup per row: k rounds of arg-max with exclusion; ties -> lower index.
__global__ __launch_bounds__(256) void topk_kernel(const float* __restrict__ z, int n_cells, int k, int positive,
                                                   int32_t* __restrict__ out) {
  extern __shared__ float vals[];
  __shared__ float bv[4];
  __shared__ int bi[4];
  const int b = blockIdx.x;
  // positive: only values > 0 are candidates (the others become NaN, never picked)
  for (int c = threadIdx.x; c < n_cells; c += 256) {
    const float v = z[(int64_t)b * n_cells + c];
    vals[c] = positive && !(v > 0.0f) ? NAN : v;
  }
  __syncthreads();
  for (int r = 0; r < k; ++r) {
    float best = -INFINITY;
    int idx = INT_MAX;
    for (int c = threadIdx.x; c < n_cells; c += 256) {
      const float v = vals[c];
      if (v > best || (v == best && c < idx)) {
        best = v;
        idx = c;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float v2 = __shfl_xor(best, o, 64);
      const int i2 = __shfl_xor(idx, o, 64);
      if (v2 > best || (v2 == best && i2 < idx)) {
        best = v2;
        idx = i2;
      }
    }
    if ((threadIdx.x & 63) == 0) {
      bv[threadIdx.x >> 6] = best;
      bi[threadIdx.x >> 6] = idx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float vb = bv[0];
      int ib = bi[0];
      for (int w = 1; w < 4; ++w)
        if (bv[w] > vb || (bv[w] == vb && bi[w] < ib)) {
          vb = bv[w];
          ib = bi[w];
        }
      // picked entries become NaN, which no comparison selects again; a row with
      // nothing left to pick (NaN logits) reports -1
      if (ib >= 0 && ib < n_cells) {
        out[(int64_t)b * k + r] = ib;
        vals[ib] = NAN;
      } else {
        out[(int64_t)b * k + r] = -1;
      }
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------- cell targets
// T[k][c] = sum_{j in cell c} P[j][k]; cells listed as CSR (cell_ptr, cell_rot).
// One workgroup = 64 frames (lanes) x 4 waves striding over cells; P is float or bf16.
template <typename PT>
__global__ __launch_bounds__(256) void cell_targets_kernel(const PT* __restrict__ P, int64_t ldp, int64_t n_data,
                                                           const int32_t* __restrict__ cell_ptr,
                                                           const int32_t* __restrict__ cell_rot, int n_cells,
                                                           float* __restrict__ T) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * 64 + lane;
  if (k >= n_data) return;
  for (int c = wave; c < n_cells; c += 4) {
    float s = 0.0f;
    for (int t = cell_ptr[c]; t < cell_ptr[c + 1]; ++t) s += (float)P[(int64_t)cell_rot[t] * ldp + k];
    T[k * n_cells + c] = s;
  }
}

// ===================================================================== launchers
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_bin_log(const void* K, bool bf16, int64_t ps, int n_pix, const int32_t* bins, const int32_t* frames,
                          int B, float* x, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (bf16)
    bin_log_kernel<__hip_bfloat16><<<B, 256, 0, st>>>((const __hip_bfloat16*)K, ps, n_pix, bins, frames, x);
  else
    bin_log_kernel<float><<<B, 256, 0, st>>>((const float*)K, ps, n_pix, bins, frames, x);
  return hipGetLastError();
}

#define CONV_LAYERS(X) X(0, 1, 32, 64) X(1, 32, 64, 32) X(2, 64, 128, 16) X(3, 128, 128, 8)

hipError_t launch_conv_fwd(int layer, const float* in, const float* w, const float* b, float* out, int B,
                           hipStream_t st) {
  switch (layer) {
#define F(L, CI, CO, IH) \
  case L:                \
    conv_fwd_kernel<CI, CO, IH><<<nblk((int64_t)B * CO * (IH / 2) * (IH / 2)), 256, 0, st>>>(in, w, b, out, B); \
    break;
    CONV_LAYERS(F)
#undef F
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_conv_bwd(int layer, const float* in, const float* w, const float* dout, float* din, float* dw,
                           float* db, int B, hipStream_t st) {
  switch (layer) {
#define F(L, CI, CO, IH)                                                                                   \
  case L:                                                                                                  \
    conv_bwd_weight_kernel<CI, CO, IH><<<CO * CI, 256, 0, st>>>(in, dout, dw, db, B);                     \
    if (din) conv_bwd_data_kernel<CI, CO, IH><<<nblk((int64_t)B * CI * IH * IH), 256, 0, st>>>(dout, w, din, B); \
    break;
    CONV_LAYERS(F)
#undef F
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_relu_mask(float* g, const float* act, int64_t n, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  relu_mask_kernel<<<(unsigned)(blocks > 65536 ? 65536 : blocks), 256, 0, st>>>(g, act, n);
  return hipGetLastError();
}

hipError_t launch_add_bias(float* z, const float* bias, int64_t rows, int cols, hipStream_t st) {
  int64_t blocks = (rows * cols + 255) / 256;
  add_bias_kernel<<<(unsigned)(blocks > 65536 ? 65536 : blocks), 256, 0, st>>>(z, bias, rows, cols);
  return hipGetLastError();
}

hipError_t launch_gemm_small(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk, int64_t sbn,
                             float* C, int64_t ldc, int M, int N, int Kd, hipStream_t st) {
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
  gemm_small_kernel<<<grid, 256, 0, st>>>(A, sam, sak, B, sbk, sbn, C, ldc, M, N, Kd);
  return hipGetLastError();
}

hipError_t launch_col_sum(const float* X, int rows, int cols, float* out, hipStream_t st) {
  col_sum_kernel<<<nblk(cols), 256, 0, st>>>(X, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_softmax_xent(const float* z, const float* T, int n_cells, int B, float* dz, double* loss,
                               hipStream_t st) {
  softmax_xent_kernel<<<B, 256, 0, st>>>(z, T, n_cells, B, dz, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  adam_kernel<<<(unsigned)(blocks > 65536 ? 65536 : blocks), 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_topk(const float* z, int64_t rows, int n_cells, int k, bool positive, int32_t* out,
                       hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  topk_kernel<<<(unsigned)rows, 256, n_cells * sizeof(float), st>>>(z, n_cells, k, positive ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_cell_targets(const void* P, bool bf16, int64_t ldp, int64_t n_data, const int32_t* cell_ptr,
                               const int32_t* cell_rot, int n_cells, float* T, hipStream_t st) {
  if (n_data <= 0) return hipSuccess;
  const unsigned g = (unsigned)((n_data + 63) / 64);
  if (bf16)
    cell_targets_kernel<__hip_bfloat16><<<g, 256, 0, st>>>((const __hip_bfloat16*)P, ldp, n_data, cell_ptr, cell_rot,
                                                          n_cells, T);
  else
    cell_targets_kernel<float><<<g, 256, 0, st>>>((const float*)P, ldp, n_data, cell_ptr, cell_rot, n_cells, T);
  return hipGetLastError();
}

}  // namespace emc
