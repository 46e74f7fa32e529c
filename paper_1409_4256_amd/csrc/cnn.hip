// Learned orientation proposal: a small CNN scoring the cells of a coarse
// rotation grid from a log-binned frame (FP32 throughout).
//   x = log1p(binned frame) 1x64x64 -> 4 x [conv3x3 s2 p1 + bias + ReLU]
//   (1->32->64->128->128 channels) -> flatten 2048 -> linear -> n_cells logits
// Forward, backward (data and weight gradients), soft-target cross entropy,
// Adam and top-K selection are all kernels here.  Every contraction of the
// network (the convolutions as im2col products, the linear layer's backward)
// runs on one strided FP32 MFMA GEMM; the linear layer's forward uses the
// iteration's FP32 MFMA GEMM.
#include "emc_device.h"

namespace emc {

typedef float f4 __attribute__((ext_vector_type(4)));

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
// Activations are channel-major ("CNHW"): act[c][m] with m = (n * H + y) * W + x over
// the batch, so that every convolution pass is one contraction with a long
// contiguous index:
//   forward      out[o][m]  = sum_kc W[o][kc] colT[kc][m]          kc = c * 9 + dy * 3 + dx
//   data grad    dcolT[kc][m] = sum_o W[o][kc] dout[o][m], then summed back over taps (col2im)
//   weight grad  dW[o][kc] = sum_m dout[o][m] colT[kc][m]           (split over m)
// where colT[kc][m] = in[c][n][2y - 1 + dy][2x - 1 + dx] (0 outside: stride 2, padding 1).
// All three run on gemm_str_kernel (FP32 MFMA).

// colT[kc][m] of a stride-2, padding-1 3x3 convolution over in[c][n][IH][IH]
__global__ void im2col_kernel(const float* __restrict__ in, int CI, int IH, int64_t M, float* __restrict__ colT) {
  const int OH = IH / 2;
  const int64_t total = (int64_t)CI * 9 * M;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t m = e % M, kc = e / M;
    const int c = (int)(kc / 9), t = (int)(kc % 9), dy = t / 3, dx = t % 3;
    const int x = (int)(m % OH), y = (int)((m / OH) % OH);
    const int64_t n = m / ((int64_t)OH * OH);
    const int iy = 2 * y - 1 + dy, ix = 2 * x - 1 + dx;
    colT[e] = (iy >= 0 && iy < IH && ix >= 0 && ix < IH) ? in[((int64_t)c * (M / ((int64_t)OH * OH)) + n) * IH * IH +
                                                             (int64_t)iy * IH + ix]
                                                       : 0.0f;
  }
}

// din[c][n][iy][ix] = sum of dcolT[c * 9 + t][m] over the taps t that read (iy, ix)
__global__ void col2im_kernel(const float* __restrict__ dcolT, int CI, int IH, int64_t nB, float* __restrict__ din) {
  const int OH = IH / 2;
  const int64_t M = nB * OH * OH, total = (int64_t)CI * nB * IH * IH;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int ix = (int)(e % IH), iy = (int)((e / IH) % IH);
    const int64_t n = (e / ((int64_t)IH * IH)) % nB, c = e / ((int64_t)IH * IH * nB);
    float acc = 0.0f;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int ty = iy + 1 - dy;
      if (ty < 0 || (ty & 1) || (ty >> 1) >= OH) continue;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int tx = ix + 1 - dx;
        if (tx < 0 || (tx & 1) || (tx >> 1) >= OH) continue;
        acc += dcolT[(c * 9 + dy * 3 + dx) * M + (n * OH + (ty >> 1)) * OH + (tx >> 1)];
      }
    }
    din[e] = acc;
  }
}

// flat[b][c * P + p] = act[c][b * P + p] (the linear layer's input, per frame), or back
__global__ void flatten_kernel(const float* __restrict__ src, int C, int P, int64_t nB, float* __restrict__ dst,
                               int to_flat) {
  const int64_t total = (int64_t)C * P * nB;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int p = (int)(e % P);
    const int64_t b = (e / P) % nB, c = e / ((int64_t)P * nB);  // e indexes act[c][b][p]
    const int64_t f = b * C * P + c * P + p;
    if (to_flat)
      dst[f] = src[e];
    else
      dst[e] = src[f];
  }
}

// row sums: out[r] = sum_m X[r][m] (bias gradients of the convolutions) in two passes:
// workgroup (r, q) sums columns [q * span, (q + 1) * span) into part[r][q], then the
// parts of a row are added in order
constexpr int kRowParts = 64;
__global__ __launch_bounds__(256) void row_part_kernel(const float* __restrict__ X, int64_t cols, int64_t span,
                                                       float* __restrict__ part) {
  __shared__ float red[4];
  const int r = blockIdx.y, q = blockIdx.x;
  const float* row = X + (int64_t)r * cols;
  const int64_t c1 = (q + 1) * span < cols ? (q + 1) * span : cols;
  float s = 0.0f;
  for (int64_t m = q * span + threadIdx.x; m < c1; m += 256) s += row[m];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)r * kRowParts + q] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ void row_finish_kernel(const float* __restrict__ part, int rows, float* __restrict__ out) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  float s = 0.0f;
  for (int q = 0; q < kRowParts; ++q) s += part[(int64_t)r * kRowParts + q];
  out[r] = s;
}

// ReLU of the forward pass and of its gradient: g *= (act > 0)
__global__ void relu_mask_kernel(float* __restrict__ g, const float* __restrict__ act, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    if (!(act[e] > 0.0f)) g[e] = 0.0f;
}

// --------------------------------------------------------------------- strided FP32 MFMA GEMM
// C[m][n] = sum_k A(m, k) B(k, n) for the network's contractions, with
//   A(m, k) = A[m * lda + k] (AK) or A[k * lda + m];  B(k, n) = B[n * ldb + k] (BK) or B[k * ldb + n],
// so that transposed operands need no copies.  Workgroup tile 128 x 128 x 16, 4 waves
// of 64 x 64 from v_mfma_f32_16x16x4_f32, LDS [row][k] double-buffered.  Bounds are
// checked in m, n and k.  Split reduction: gridDim.z ranges of `kper` k each write
// their partial product to C + z * c_split (summed by gemm_reduce_kernel); without a
// split the epilogue adds bias[m] and applies ReLU when asked.
constexpr int GBM = 128, GBN = 128, GBK = 16, GLK = GBK + 4;

template <bool AK, bool BKC>
__global__ __launch_bounds__(256) void gemm_str_kernel(const float* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ B, int64_t ldb, float* __restrict__ C,
                                                       int64_t ldc, int M, int N, int64_t K, int64_t kper,
                                                       int64_t c_split, const float* __restrict__ bias, int relu) {
  __shared__ __attribute__((aligned(16))) float As[2][GBM * GLK];
  __shared__ __attribute__((aligned(16))) float Bs[2][GBN * GLK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * GBM, n0 = (int64_t)blockIdx.x * GBN;
  const int64_t kb = (int64_t)blockIdx.z * kper, ke = kb + kper < K ? kb + kper : K;
  C += (int64_t)blockIdx.z * c_split;

  float ra[8], rb[8];
  // element u of this thread's share of a 128 x 16 stage: (row, k) inside the tile;
  // lanes run along the operand's contiguous index
  auto slot = [&](bool kcontig, int u, int& r, int& c) {
    const int e = tid + 256 * u;
    if (kcontig) {
      r = e >> 4;
      c = e & 15;
    } else {
      r = e & 127;
      c = e >> 7;
    }
  };
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int r, c;
      slot(AK, u, r, c);
      const int64_t m = m0 + r, k = k0 + c;
      ra[u] = (m < M && k < ke) ? (AK ? A[m * lda + k] : A[k * lda + m]) : 0.0f;
      slot(BKC, u, r, c);
      const int64_t n = n0 + r, kk = k0 + c;
      rb[u] = (n < N && kk < ke) ? (BKC ? B[n * ldb + kk] : B[kk * ldb + n]) : 0.0f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int r, c;
      slot(AK, u, r, c);
      As[buf][r * GLK + c] = ra[u];
      slot(BKC, u, r, c);
      Bs[buf][r * GLK + c] = rb[u];
    }
  };

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int64_t nk = ke > kb ? (ke - kb + GBK - 1) / GBK : 0;
  if (nk > 0) {
    load(kb);
    store(0);
  }
  __syncthreads();
  const int arow = wm * 64 + (lane & 15), brow = wn * 64 + (lane & 15), kofs = 4 * (lane >> 4);
  for (int64_t s = 0; s < nk; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nk) load(kb + (s + 1) * GBK);
    f4 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const f4*>(&As[buf][(arow + 16 * i) * GLK + kofs]);
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const f4*>(&Bs[buf][(brow + 16 * j) * GLK + kofs]);
    // lane (row, kofs) holds k = kofs .. kofs + 3 of its row in both operands: MFMA t
    // multiplies the pairs at k = kofs + t (the k order inside the stage is permuted
    // alike for A and B, which leaves the sum unchanged)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j][t], acc[i][j], 0, 0, 0);
    if (s + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // lane holds rows 4 (lane / 16) + r, column lane % 16 of each 16 x 16 tile
  const int64_t rbase = m0 + wm * 64 + 4 * (lane >> 4), cbase = n0 + wn * 64 + (lane & 15);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rbase + 16 * i + r;
      if (row >= M) continue;
      const float bv = bias ? bias[row] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = cbase + 16 * j;
        if (col >= N) continue;
        float v = acc[i][j][r] + bv;
        if (relu) v = fmaxf(v, 0.0f);
        C[row * ldc + col] = v;
      }
    }
}

// C[m][n] = sum over splits z (in order) of part[z][m][n] (+ bias[m], ReLU when asked)
__global__ void gemm_reduce_kernel(const float* __restrict__ part, int splits, int64_t c_split, int M, int N,
                                   float* __restrict__ C, int64_t ldc, const float* __restrict__ bias, int relu) {
  const int64_t total = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t m = e / N, n = e % N;
    float v = 0.0f;
    for (int z = 0; z < splits; ++z) v += part[z * c_split + m * ldc + n];
    if (bias) v += bias[m];
    if (relu) v = fmaxf(v, 0.0f);
    C[m * ldc + n] = v;
  }
}

// z[b][c] += bias[c]
__global__ void add_bias_kernel(float* __restrict__ z, const float* __restrict__ bias, int64_t rows, int cols) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * 256)
    z[e] += bias[e % cols];
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

static inline unsigned grid_of(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

hipError_t launch_im2col(const float* in, int CI, int IH, int64_t M, float* colT, hipStream_t st) {
  im2col_kernel<<<grid_of((int64_t)CI * 9 * M), 256, 0, st>>>(in, CI, IH, M, colT);
  return hipGetLastError();
}

hipError_t launch_col2im(const float* dcolT, int CI, int IH, int64_t nB, float* din, hipStream_t st) {
  col2im_kernel<<<grid_of((int64_t)CI * nB * IH * IH), 256, 0, st>>>(dcolT, CI, IH, nB, din);
  return hipGetLastError();
}

hipError_t launch_flatten(const float* src, int C, int P, int64_t nB, float* dst, bool to_flat, hipStream_t st) {
  flatten_kernel<<<grid_of((int64_t)C * P * nB), 256, 0, st>>>(src, C, P, nB, dst, to_flat ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_row_sum(const float* X, int rows, int64_t cols, float* part, float* out, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int64_t span = (cols + kRowParts - 1) / kRowParts;
  row_part_kernel<<<dim3(kRowParts, (unsigned)rows), 256, 0, st>>>(X, cols, span, part);
  row_finish_kernel<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(part, rows, out);
  return hipGetLastError();
}

int gemm_str_splits(int M, int N, int64_t K) {
  // about 256 workgroups when the product has fewer output tiles, each range >= 256 k
  const int64_t tiles = ((int64_t)(M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
  if (tiles >= 192) return 1;
  int64_t s = 256 / tiles;
  if (s > K / 256) s = K / 256;
  return (int)(s < 1 ? 1 : s);
}

hipError_t launch_gemm_str(bool a_kcontig, const float* A, int64_t lda, bool b_kcontig, const float* B, int64_t ldb,
                           float* C, int64_t ldc, int M, int N, int64_t K, int splits, float* part,
                           const float* bias, bool relu, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (splits < 1 || (splits > 1 && !part)) return hipErrorInvalidValue;
  const int64_t kper = splits > 1 ? ((K + splits - 1) / splits + GBK - 1) / GBK * GBK : K;
  const int z = splits > 1 ? (int)((K + kper - 1) / kper) : 1;
  dim3 grid((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), (unsigned)z);
  float* out = z > 1 ? part : C;
  const int64_t c_split = z > 1 ? (int64_t)M * ldc : 0;
  const float* eb = z > 1 ? nullptr : bias;  // the epilogue runs in the reduction when split
  const int er = z > 1 ? 0 : (relu ? 1 : 0);
#define G(AK, BKC) gemm_str_kernel<AK, BKC><<<grid, 256, 0, st>>>(A, lda, B, ldb, out, ldc, M, N, K, kper, c_split, \
                                                                 eb, er)
  if (a_kcontig && b_kcontig)
    G(true, true);
  else if (a_kcontig)
    G(true, false);
  else if (b_kcontig)
    G(false, true);
  else
    G(false, false);
#undef G
  if (z > 1) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    gemm_reduce_kernel<<<grid_of((int64_t)M * N), 256, 0, st>>>(part, z, c_split, M, N, C, ldc, bias, relu ? 1 : 0);
  }
  return hipGetLastError();
}

hipError_t launch_relu_mask(float* g, const float* act, int64_t n, hipStream_t st) {
  relu_mask_kernel<<<grid_of(n), 256, 0, st>>>(g, act, n);
  return hipGetLastError();
}

hipError_t launch_add_bias(float* z, const float* bias, int64_t rows, int cols, hipStream_t st) {
  add_bias_kernel<<<grid_of(rows * cols), 256, 0, st>>>(z, bias, rows, cols);
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
