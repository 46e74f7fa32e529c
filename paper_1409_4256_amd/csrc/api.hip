// Host side of the C ABI: argument validation, workspace carving and the
// launch sequence of one iteration.  Nothing here computes on the host.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/emc.h"
#include "emc_device.h"

using namespace emc;

namespace {

thread_local std::string g_err;

emc_status fail(emc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr, what)                                                                  \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(EMC_ERR_HIP, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)

#define CHECK(x)                 \
  do {                           \
    emc_status s_ = (x);         \
    if (s_ != EMC_OK) return s_; \
  } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool is_bf16(const emc_problem* pb) { return pb->precision == EMC_PREC_BF16; }

// Validate the scalar part of a problem and, if `geom`, its geometry pointers.
emc_status check_problem(const emc_problem* pb, bool geom) {
  if (!pb) return fail(EMC_ERR_INVALID_ARG, "problem is NULL");
  if (pb->grid_n < 2 || pb->grid_n > 1024) return fail(EMC_ERR_INVALID_ARG, "grid_n=%d outside [2, 1024]", pb->grid_n);
  if (pb->n_pix < 1) return fail(EMC_ERR_INVALID_ARG, "n_pix=%d < 1", pb->n_pix);
  if (pb->n_rot < 1) return fail(EMC_ERR_INVALID_ARG, "n_rot=%d < 1", pb->n_rot);
  if (pb->n_data < 0) return fail(EMC_ERR_INVALID_ARG, "n_data=%d < 0", pb->n_data);
  if (pb->reserved != 0) return fail(EMC_ERR_INVALID_ARG, "reserved field must be 0");
  if (pb->precision != EMC_PREC_FP32 && pb->precision != EMC_PREC_BF16)
    return fail(EMC_ERR_INVALID_ARG, "unknown precision %d", pb->precision);
  if (geom) {
    if (!pb->q || !pb->mask || !pb->quat || !pb->log_w) return fail(EMC_ERR_INVALID_ARG, "geometry pointer is NULL");
    if (!aligned(pb->q, 4) || !aligned(pb->quat, 16) || !aligned(pb->log_w, 8))
      return fail(EMC_ERR_INVALID_ARG, "misaligned geometry pointer");
    if (const emc_scatter_plan* S = pb->scatter) {
      const int nb = (pb->grid_n + brick_edge() - 1) / brick_edge();
      if (S->grid_n != pb->grid_n || S->n_pix != pb->n_pix || S->n_rot != pb->n_rot || S->q != pb->q ||
          S->mask != pb->mask || S->quat != pb->quat)
        return fail(EMC_ERR_INVALID_ARG, "scatter plan was built for another geometry");
      if (S->brick != brick_edge() || S->n_bricks != nb * nb * nb || S->n_groups != (pb->n_pix + 63) / 64 ||
          S->n_items < 0 || S->n_visits < 0 || (S->n_items > 0 && (!S->items || !S->visits || !S->rot)) ||
          !aligned(S->items, 16) || !aligned(S->rot, 8))
        return fail(EMC_ERR_INVALID_ARG, "inconsistent scatter plan");
    }
  }
  return EMC_OK;
}

emc_status need(const void* p, size_t align, const char* name) {
  if (!p) return fail(EMC_ERR_INVALID_ARG, "%s is NULL", name);
  if (!aligned(p, align)) return fail(EMC_ERR_INVALID_ARG, "%s is not %zu-byte aligned", name, align);
  return EMC_OK;
}

struct Dims {
  int64_t ps, ds, grid;
  size_t elem;  // bytes of a packed frame / responsibility element
};

Dims dims_of(const emc_problem* pb) {
  Dims d;
  d.ps = round_up(pb->n_pix, 256);
  d.ds = round_up(pb->n_data, 256);
  d.grid = (int64_t)pb->grid_n * pb->grid_n * pb->grid_n;
  d.elem = is_bf16(pb) ? 2 : 4;
  return d;
}

size_t frames_bytes(const emc_problem* pb) {
  const Dims d = dims_of(pb);
  return ((size_t)pb->n_data * d.ps + (size_t)d.ps * d.ds) * d.elem;
}

size_t slices_bytes(const emc_problem* pb) { return (size_t)pb->n_rot * dims_of(pb).ps * sizeof(float); }

struct Layout {
  size_t slices, G, P, S, scale, c, b, stats, L, rho, num, den, copies, total;
};

// grid copies of the rotation-major c-step: one numerator and one denominator per
// XCD (none with a brick-major plan)
size_t copies_bytes(const emc_problem* pb) {
  return pb->scatter ? 0 : (size_t)16 * pb->grid_n * pb->grid_n * pb->grid_n * sizeof(double);
}

Layout layout_of(const emc_problem* pb) {
  const Dims d = dims_of(pb);
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (size_t)round_up((int64_t)bytes, 256);
    return at;
  };
  L.slices = take(slices_bytes(pb));  // A (or hi/lo), then W'
  L.G = take((size_t)pb->n_rot * d.ds * sizeof(float));
  L.P = is_bf16(pb) ? take((size_t)pb->n_rot * d.ds * 2) : L.G;  // FP32: P overwrites G in place
  L.S = take((size_t)pb->n_rot * sizeof(double));
  L.scale = take((size_t)pb->n_rot * sizeof(float));
  L.c = take((size_t)d.ps * sizeof(double));
  L.b = take((size_t)pb->n_data * sizeof(double));
  L.stats = take((size_t)pb->n_data * 2 * sizeof(double));
  L.L = take((size_t)pb->n_data * sizeof(double));
  L.rho = take((size_t)pb->n_rot * sizeof(double));
  L.num = take((size_t)d.grid * sizeof(double));
  L.den = take((size_t)d.grid * sizeof(double));
  L.copies = take(copies_bytes(pb));
  L.total = o;
  return L;
}

// ---- launch sequences shared by the step entry points and emc_iterate (no validation) ----

emc_status run_expand(const emc_problem* pb, const float* model, double* c, void* slices, double* S, float* scale,
                      hipStream_t st) {
  const Dims d = dims_of(pb);
  HIP_TRY(launch_centre(model, pb->grid_n, pb->q, pb->mask, pb->quat, pb->n_pix, d.ps, pb->n_rot, c, st), "centre");
  if (is_bf16(pb))
    HIP_TRY(launch_expand_bf16(model, pb->grid_n, pb->q, pb->mask, pb->quat, pb->n_pix, d.ps, pb->n_rot, c, slices, S,
                               scale, st),
            "expand");
  else
    HIP_TRY(launch_expand(model, pb->grid_n, pb->q, pb->mask, pb->quat, pb->n_pix, d.ps, pb->n_rot, c,
                          (float*)slices, S, st),
            "expand");
  return EMC_OK;
}

// splits > 1 (BF16 only; from gemm_bf16_splits): the product's k range is cut in
// `splits` parts whose partial products go to `part` (splits x n_rot x ds floats)
// and are summed into G
emc_status run_loglik(const emc_problem* pb, const void* K, const void* slices, const float* scale, const double* c,
                      float* G, double* b, hipStream_t st, int splits = 1, float* part = nullptr) {
  if (pb->n_data == 0) return EMC_OK;
  const Dims d = dims_of(pb);
  HIP_TRY(launch_frame_dot(K, is_bf16(pb), d.ps, pb->n_data, c, b, st), "frame_dot");
  if (is_bf16(pb)) {
    const char* hi = (const char*)slices;
    const char* lo = hi + (size_t)pb->n_rot * d.ps * 2;
    if (splits > 1) {
      if (!part) return fail(EMC_ERR_INVALID_ARG, "split log-likelihood product without a partial-product buffer");
      HIP_TRY(launch_gemm_bf16_dual_nt_split(hi, lo, K, scale, part, pb->n_rot, pb->n_data, d.ps, d.ps, d.ps, d.ds,
                                             splits, st),
              "loglik gemm");
      HIP_TRY(launch_sum_slabs(part, splits, (int64_t)pb->n_rot * d.ds, G, st), "loglik partial sums");
    } else {
      HIP_TRY(launch_gemm_bf16_dual_nt(hi, lo, K, scale, G, pb->n_rot, pb->n_data, d.ps, d.ps, d.ps, d.ds, st),
              "loglik gemm");
    }
  } else {
    HIP_TRY(launch_gemm_f32_nt((const float*)slices, (const float*)K, G, pb->n_rot, pb->n_data, d.ps, d.ps, d.ps, d.ds,
                               st),
            "loglik gemm");
  }
  return EMC_OK;
}

emc_status run_estep(const emc_problem* pb, const float* G, const double* S, const double* b, int32_t mode,
                     double* stats, void* P, double* L, double* rho, hipStream_t st, double* part = nullptr) {
  const Dims d = dims_of(pb);
  if (mode != EMC_RESP_FINALIZE)
    HIP_TRY(launch_lse_stats(G, d.ds, pb->n_rot, pb->n_data, pb->log_w, S, b, stats, part, st), "lse_stats");
  if (mode == EMC_RESP_PARTIAL) return EMC_OK;
  HIP_TRY(launch_lse_finish(stats, pb->n_data, L, st), "lse_finish");
  if (is_bf16(pb))
    HIP_TRY(launch_lse_write_bf16(G, d.ds, P, d.ds, pb->n_rot, pb->n_data, pb->log_w, S, b, L, rho, st), "lse_write");
  else
    HIP_TRY(launch_lse_write_f32(G, d.ds, (float*)P, d.ds, pb->n_rot, pb->n_data, pb->log_w, S, b, L, rho, st),
            "lse_write");
  return EMC_OK;
}

// num/den += the c-step sums of W' (row stride ps) and rho: brick-major with a plan,
// else rotation-major (with per-XCD grid copies when `copies` is given)
emc_status run_scatter(const emc_problem* pb, const float* Wp, int64_t ps, const double* rho, double* num,
                       double* den, double* copies, hipStream_t st) {
  if (const emc_scatter_plan* S = pb->scatter) {
    const int nb = (pb->grid_n + brick_edge() - 1) / brick_edge();
    HIP_TRY(launch_brick_scatter((const int4*)S->items, S->n_items, S->visits, S->n_groups, Wp, ps, rho, pb->q,
                                 pb->mask, S->rot, pb->n_pix, pb->grid_n, nb, num, den, st),
            "brick scatter");
  } else {
    HIP_TRY(launch_scatter(Wp, ps, rho, pb->q, pb->mask, pb->quat, pb->n_pix, pb->n_rot, pb->grid_n, num, den, copies,
                           st),
            "scatter");
  }
  return EMC_OK;
}

emc_status run_compress(const emc_problem* pb, const void* P, const void* K, const double* rho, float* Wp,
                        double* num, double* den, int32_t accumulate, double* copies, hipStream_t st) {
  const Dims d = dims_of(pb);
  if (!accumulate) {
    HIP_TRY(launch_fill_zero_f64(num, (size_t)d.grid, st), "zero num");
    HIP_TRY(launch_fill_zero_f64(den, (size_t)d.grid, st), "zero den");
  }
  if (pb->n_data == 0) return EMC_OK;  // nothing to add: W' = 0 and rho = 0
  const char* KT = (const char*)K + (size_t)pb->n_data * d.ps * d.elem;
  if (is_bf16(pb))
    HIP_TRY(launch_gemm_bf16_nt(P, KT, Wp, pb->n_rot, d.ps, d.ds, d.ds, d.ds, d.ps, st), "mstep gemm");
  else
    HIP_TRY(launch_gemm_f32_nt((const float*)P, (const float*)KT, Wp, pb->n_rot, d.ps, d.ds, d.ds, d.ds, d.ps, st),
            "mstep gemm");
  return run_scatter(pb, Wp, d.ps, rho, num, den, copies, st);
}

emc_status run_finalize(const emc_problem* pb, const double* num, const double* den, const float* prev, float* out,
                        const double* L, int64_t n_L, double* loglik, hipStream_t st) {
  const int64_t grid = (int64_t)pb->grid_n * pb->grid_n * pb->grid_n;
  HIP_TRY(launch_divide(num, den, prev, out, grid, st), "divide");
  HIP_TRY(launch_mean(L, n_L, loglik, st), "mean");
  return EMC_OK;
}

}  // namespace

extern "C" {

const char* emc_version(void) { return "emc-gfx950 0.2 (fp32 and bf16 mfma)"; }

const char* emc_last_error(void) { return g_err.c_str(); }

int64_t emc_pix_stride(int32_t n_pix) { return n_pix < 1 ? 0 : round_up(n_pix, 256); }

int64_t emc_data_stride(int32_t n_data) { return n_data < 1 ? 0 : round_up(n_data, 256); }

emc_status emc_frames_bytes(const emc_problem* pb, size_t* bytes) {
  CHECK(check_problem(pb, false));
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = frames_bytes(pb);
  return EMC_OK;
}

emc_status emc_slices_bytes(const emc_problem* pb, size_t* bytes) {
  CHECK(check_problem(pb, false));
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = slices_bytes(pb);
  return EMC_OK;
}

emc_status emc_workspace_bytes(const emc_problem* pb, size_t* bytes) {
  CHECK(check_problem(pb, false));
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = layout_of(pb).total;
  return EMC_OK;
}

static emc_status pack_frames(const emc_problem* pb, const uint16_t* counts, const int32_t* frames, void* K_packed,
                              hipStream_t st) {
  CHECK(check_problem(pb, true));
  if (pb->n_data == 0) return EMC_OK;
  CHECK(need(counts, 2, "counts"));
  CHECK(need(K_packed, 16, "K_packed"));
  const Dims d = dims_of(pb);
  char* KT = (char*)K_packed + (size_t)pb->n_data * d.ps * d.elem;
  HIP_TRY(launch_pack(counts, pb->mask, pb->n_pix, d.ps, pb->n_data, d.ds, frames, K_packed, KT, is_bf16(pb), st),
          "pack");
  if (is_bf16(pb)) {
    int flag = 0;
    HIP_TRY(read_range_flag(&flag, st), "range flag");
    if (flag) return fail(EMC_ERR_RANGE, "a photon count exceeds 256, which BF16 cannot hold exactly");
  }
  return EMC_OK;
}

emc_status emc_pack_frames(const emc_problem* pb, const uint16_t* counts, void* K_packed, hipStream_t st) {
  return pack_frames(pb, counts, nullptr, K_packed, st);
}

emc_status emc_pack_patterns(const emc_problem* pb, const uint16_t* counts, void* K_packed, hipStream_t st) {
  return pack_frames(pb, counts, nullptr, K_packed, st);
}

emc_status emc_validate(const emc_problem* pb, const float* model, int32_t* flags, hipStream_t st) {
  CHECK(check_problem(pb, true));
  if (model) CHECK(need(model, 4, "model"));
  CHECK(need(flags, 4, "flags"));
  const int64_t grid = (int64_t)pb->grid_n * pb->grid_n * pb->grid_n;
  HIP_TRY(launch_validate(pb->quat, pb->n_rot, pb->q, pb->mask, pb->n_pix, pb->log_w, model, grid, 1e-5, flags, st),
          "validate");
  int32_t host = 0;
  HIP_TRY(hipMemcpyAsync(&host, flags, sizeof host, hipMemcpyDeviceToHost, st), "read validation flags");
  HIP_TRY(hipStreamSynchronize(st), "validate synchronise");
  if (host & kValidQuat) return fail(EMC_ERR_INVALID_ARG, "a quaternion's norm differs from 1 by more than 1e-5");
  if (host & kValidWeight) return fail(EMC_ERR_INVALID_ARG, "a log prior weight is not finite");
  if (host & kValidPixel) return fail(EMC_ERR_INVALID_ARG, "a used pixel's coordinate is not finite");
  if (host & kValidModel) return fail(EMC_ERR_INVALID_ARG, "a model value is negative or not finite");
  return EMC_OK;
}

emc_status emc_pack_frames_list(const emc_problem* pb, const uint16_t* counts, const int32_t* frames, void* K_packed,
                                hipStream_t st) {
  if (pb && pb->n_data > 0) CHECK(need(frames, 4, "frames"));
  return pack_frames(pb, counts, frames, K_packed, st);
}

emc_status emc_expand(const emc_problem* pb, const float* model, double* c, void* slices, double* S, float* scale,
                      hipStream_t st) {
  CHECK(check_problem(pb, true));
  CHECK(need(model, 4, "model"));
  CHECK(need(c, 16, "c"));
  CHECK(need(slices, 16, "slices"));
  CHECK(need(S, 8, "S"));
  if (is_bf16(pb)) CHECK(need(scale, 4, "scale"));
  return run_expand(pb, model, c, slices, S, scale, st);
}

emc_status emc_loglik(const emc_problem* pb, const void* K_packed, const void* slices, const float* scale,
                      const double* c, float* G, double* b, hipStream_t st) {
  CHECK(check_problem(pb, false));
  if (pb->n_data == 0) return EMC_OK;
  CHECK(need(K_packed, 16, "K_packed"));
  CHECK(need(slices, 16, "slices"));
  CHECK(need(c, 16, "c"));
  CHECK(need(G, 16, "G"));
  CHECK(need(b, 8, "b"));
  if (is_bf16(pb)) CHECK(need(scale, 4, "scale"));
  return run_loglik(pb, K_packed, slices, scale, c, G, b, st);
}

emc_status emc_responsibilities(const emc_problem* pb, const float* G, const double* S, const double* b, int32_t mode,
                                double* stats, void* P, double* L, double* rho, hipStream_t st) {
  CHECK(check_problem(pb, false));
  if (mode != EMC_RESP_FULL && mode != EMC_RESP_PARTIAL && mode != EMC_RESP_FINALIZE)
    return fail(EMC_ERR_INVALID_ARG, "unknown mode %d", mode);
  CHECK(need(pb->log_w, 8, "log_w"));
  CHECK(need(S, 8, "S"));
  if (mode != EMC_RESP_PARTIAL) CHECK(need(rho, 8, "rho"));
  if (pb->n_data > 0) {
    CHECK(need(stats, 16, "stats"));
    CHECK(need(G, 16, "G"));
    CHECK(need(b, 8, "b"));
    if (mode != EMC_RESP_PARTIAL) {
      CHECK(need(P, 16, "P"));
      CHECK(need(L, 8, "L"));
      if (is_bf16(pb) && (const void*)P == (const void*)G)
        return fail(EMC_ERR_INVALID_ARG, "BF16 responsibilities may not alias G");
    }
  }
  return run_estep(pb, G, S, b, mode, stats, P, L, rho, st);
}

emc_status emc_compress_workspace_bytes(const emc_problem* pb, size_t* bytes) {
  CHECK(check_problem(pb, false));
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = copies_bytes(pb);
  return EMC_OK;
}

emc_status emc_compress(const emc_problem* pb, const void* P, const void* K_packed, const double* rho, float* Wp,
                        double* num, double* den, int32_t accumulate, void* ws, size_t ws_bytes, hipStream_t st) {
  CHECK(check_problem(pb, true));
  if (ws) {
    if (!aligned(ws, 256)) return fail(EMC_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    if (ws_bytes < copies_bytes(pb))
      return fail(EMC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, copies_bytes(pb));
  }
  CHECK(need(num, 8, "num"));
  CHECK(need(den, 8, "den"));
  if (pb->n_data > 0) {
    CHECK(need(P, 16, "P"));
    CHECK(need(K_packed, 16, "K_packed"));
    CHECK(need(rho, 8, "rho"));
    CHECK(need(Wp, 16, "Wp"));
  }
  return run_compress(pb, P, K_packed, rho, Wp, num, den, accumulate, (double*)ws, st);
}

namespace {

struct ScatterLayout {
  size_t cnt, off, rot, items, visits, total;
};

ScatterLayout scatter_layout(int64_t n_bricks, int64_t n_rot, int64_t n_items, int64_t n_visits) {
  ScatterLayout L;
  size_t o = 0;
  auto take = [&](int64_t bytes) {
    size_t at = o;
    o += (size_t)round_up(bytes, 256);
    return at;
  };
  L.cnt = take(n_bricks * 4);
  L.off = take((n_bricks + 1) * 8);
  L.rot = take(n_rot * 9 * 8);
  L.items = take(n_items * 16);
  L.visits = take(n_visits * 4);
  L.total = o;
  return L;
}

int64_t bricks_of(const emc_problem* pb) {
  const int64_t nb = (pb->grid_n + brick_edge() - 1) / brick_edge();
  return nb * nb * nb;
}

}  // namespace

emc_status emc_scatter_plan_min_bytes(const emc_problem* pb, size_t* bytes) {
  CHECK(check_problem(pb, false));
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = scatter_layout(bricks_of(pb), pb->n_rot, 0, 0).total;
  return EMC_OK;
}

emc_status emc_scatter_plan_build(const emc_problem* pb, int32_t chunk, void* buf, size_t buf_bytes,
                                  emc_scatter_plan* plan, hipStream_t st) {
  CHECK(check_problem(pb, true));
  if (!plan) return fail(EMC_ERR_INVALID_ARG, "plan is NULL");
  if (chunk == 0) chunk = 2048;
  if (chunk < 64 || chunk > (1 << 20)) return fail(EMC_ERR_INVALID_ARG, "chunk=%d outside [64, 2^20]", chunk);
  const int64_t n_bricks = bricks_of(pb);
  const int nb = (pb->grid_n + brick_edge() - 1) / brick_edge();
  const int n_groups = (pb->n_pix + 63) / 64;
  if ((int64_t)pb->n_rot * n_groups > INT32_MAX)
    return fail(EMC_ERR_UNSUPPORTED, "n_rot * pixel groups = %lld exceeds 2^31 - 1",
                (long long)pb->n_rot * n_groups);
  CHECK(need(buf, 256, "buf"));
  const ScatterLayout L0 = scatter_layout(n_bricks, pb->n_rot, 0, 0);
  if (buf_bytes < L0.total) {
    plan->bytes = (int64_t)L0.total;
    return fail(EMC_ERR_WORKSPACE, "scatter plan buffer has %zu bytes, needs at least %zu", buf_bytes, L0.total);
  }
  char* b = (char*)buf;
  int* cnt = (int*)(b + L0.cnt);
  double* rot = (double*)(b + L0.rot);
  HIP_TRY(launch_brick_rot(pb->quat, pb->n_rot, rot, st), "rotation table");
  HIP_TRY(launch_fill_i32(cnt, n_bricks, 0, st), "zero brick counts");
  HIP_TRY(launch_brick_visits(pb->q, pb->mask, rot, pb->n_pix, pb->n_rot, n_groups, pb->grid_n, nb, cnt, nullptr,
                              nullptr, st),
          "count visits");
  std::vector<int> h(n_bricks);
  HIP_TRY(hipMemcpyAsync(h.data(), cnt, n_bricks * 4, hipMemcpyDeviceToHost, st), "read brick counts");
  HIP_TRY(hipStreamSynchronize(st), "read brick counts");
  std::vector<int64_t> off(n_bricks + 1, 0);
  int64_t max_items = 0;
  for (int64_t k = 0; k < n_bricks; ++k) {
    off[k + 1] = off[k] + h[k];
    max_items = std::max<int64_t>(max_items, (h[k] + chunk - 1) / chunk);
  }
  const int64_t n_visits = off[n_bricks];
  if (n_visits > INT32_MAX) return fail(EMC_ERR_UNSUPPORTED, "%lld visits exceed 2^31 - 1", (long long)n_visits);
  // items ordered by chunk index, then brick: a brick's items spread over the launch
  std::vector<int4> items;
  for (int64_t c = 0; c < max_items; ++c)
    for (int64_t k = 0; k < n_bricks; ++k)
      if ((int64_t)c * chunk < h[k]) {
        const int64_t first = off[k] + c * chunk;
        items.push_back(make_int4((int)k, (int)first, (int)std::min<int64_t>(first + chunk, off[k + 1]), 0));
      }
  const int64_t n_items = (int64_t)items.size();
  const ScatterLayout L = scatter_layout(n_bricks, pb->n_rot, n_items, n_visits);
  plan->bytes = (int64_t)L.total;
  if (buf_bytes < L.total)
    return fail(EMC_ERR_WORKSPACE, "scatter plan buffer has %zu bytes, needs %zu", buf_bytes, L.total);
  int64_t* doff = (int64_t*)(b + L.off);
  int4* ditems = (int4*)(b + L.items);
  int* dvisits = (int*)(b + L.visits);
  HIP_TRY(hipMemcpyAsync(doff, off.data(), (n_bricks + 1) * 8, hipMemcpyHostToDevice, st), "write offsets");
  if (n_items > 0)
    HIP_TRY(hipMemcpyAsync(ditems, items.data(), n_items * 16, hipMemcpyHostToDevice, st), "write items");
  HIP_TRY(launch_fill_i32(cnt, n_bricks, 0, st), "zero brick cursors");
  HIP_TRY(launch_brick_visits(pb->q, pb->mask, rot, pb->n_pix, pb->n_rot, n_groups, pb->grid_n, nb, cnt, doff,
                              dvisits, st),
          "list visits");
  HIP_TRY(hipStreamSynchronize(st), "list visits");  // the host arrays above go out of scope
  emc_scatter_plan P = {};
  P.grid_n = pb->grid_n;
  P.n_pix = pb->n_pix;
  P.n_rot = pb->n_rot;
  P.brick = brick_edge();
  P.n_bricks = (int32_t)n_bricks;
  P.n_groups = n_groups;
  P.chunk = chunk;
  P.n_visits = n_visits;
  P.n_items = n_items;
  P.bytes = (int64_t)L.total;
  P.visits = dvisits;
  P.items = (const int32_t*)ditems;
  P.rot = rot;
  P.q = pb->q;
  P.mask = pb->mask;
  P.quat = pb->quat;
  *plan = P;
  return EMC_OK;
}

emc_status emc_finalize(const emc_problem* pb, const double* num, const double* den, const float* model_prev,
                        float* model_out, const double* L, int64_t n_L, double* loglik, hipStream_t st) {
  if (!pb) return fail(EMC_ERR_INVALID_ARG, "problem is NULL");
  if (pb->grid_n < 2 || pb->grid_n > 1024) return fail(EMC_ERR_INVALID_ARG, "grid_n=%d outside [2, 1024]", pb->grid_n);
  if (n_L < 0) return fail(EMC_ERR_INVALID_ARG, "n_L < 0");
  CHECK(need(num, 8, "num"));
  CHECK(need(den, 8, "den"));
  CHECK(need(model_prev, 4, "model_prev"));
  CHECK(need(model_out, 4, "model_out"));
  CHECK(need(loglik, 8, "loglik"));
  if (n_L > 0) CHECK(need(L, 8, "L"));
  return run_finalize(pb, num, den, model_prev, model_out, L, n_L, loglik, st);
}

}  // extern "C"

namespace {

emc_status check_iterate(const emc_problem* pb, const float* model_in, const void* K_packed, const float* model_out,
                         const double* loglik, const void* P_out) {
  CHECK(check_problem(pb, true));
  CHECK(need(model_in, 4, "model_in"));
  CHECK(need(model_out, 4, "model_out"));
  CHECK(need(loglik, 8, "loglik"));
  if (pb->n_data > 0) CHECK(need(K_packed, 16, "K_packed"));
  if (P_out) CHECK(need(P_out, 16, "P_out"));
  return EMC_OK;
}

}  // namespace

extern "C" {

emc_status emc_iterate(const emc_problem* pb, const float* model_in, const void* K_packed, float* model_out,
                       double* loglik, void* P_out, void* ws, size_t ws_bytes, hipStream_t st) {
  CHECK(check_iterate(pb, model_in, K_packed, model_out, loglik, P_out));
  const Layout Lo = layout_of(pb);
  if (!ws) return fail(EMC_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(ws, 256)) return fail(EMC_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < Lo.total) return fail(EMC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, Lo.total);
  char* w = (char*)ws;
  void* slices = w + Lo.slices;  // A (or hi/lo), then W'
  float* G = (float*)(w + Lo.G);
  void* P = P_out ? P_out : (void*)(w + Lo.P);
  double* S = (double*)(w + Lo.S);
  float* scale = (float*)(w + Lo.scale);
  double* c = (double*)(w + Lo.c);
  double* b = (double*)(w + Lo.b);
  double* stats = (double*)(w + Lo.stats);
  double* L = (double*)(w + Lo.L);
  double* rho = (double*)(w + Lo.rho);
  double* num = (double*)(w + Lo.num);
  double* den = (double*)(w + Lo.den);
  CHECK(run_expand(pb, model_in, c, slices, S, scale, st));
  CHECK(run_loglik(pb, K_packed, slices, scale, c, G, b, st));
  CHECK(run_estep(pb, G, S, b, EMC_RESP_FULL, stats, P, L, rho, st));
  CHECK(run_compress(pb, P, K_packed, rho, (float*)slices, num, den, 0, (double*)(w + Lo.copies), st));
  CHECK(run_finalize(pb, num, den, model_in, model_out, L, pb->n_data, loglik, st));
  return EMC_OK;
}

}  // extern "C"

// ---- allocation-free iteration: the workspace is a static device array ----
// One array per GPU (each device holds its own copy of a __device__ variable),
// 64 MiB, kept from module load until the process ends.  Host code never uses the
// array's name as an address: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept here.
namespace {

static __device__ __align__(256) unsigned char scratch[EMC_SCRATCH_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

emc_status scratch_of_current_device(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(EMC_ERR_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p || !aligned(p, 256)) return fail(EMC_ERR_HIP, "scratch buffer address %p is not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return EMC_OK;
}

}  // namespace

extern "C" {

emc_status emc_iterate_noalloc(const emc_problem* pb, const float* model_in, const void* K_packed, float* model_out,
                               double* loglik, void* P_out, hipStream_t st) {
  CHECK(check_iterate(pb, model_in, K_packed, model_out, loglik, P_out));
  const size_t need_bytes = layout_of(pb).total;
  if (need_bytes > EMC_SCRATCH_MAX_BYTES)
    return fail(EMC_ERR_WORKSPACE, "problem needs %zu bytes of workspace, above the %zu-byte static scratch buffer",
                need_bytes, (size_t)EMC_SCRATCH_MAX_BYTES);
  void* ws = nullptr;
  CHECK(scratch_of_current_device(&ws));
  return emc_iterate(pb, model_in, K_packed, model_out, loglik, P_out, ws, EMC_SCRATCH_MAX_BYTES, st);
}

// ---- Gaussian noise model with fluence ----
namespace {

struct GaussLayout {
  size_t A, G, P, s2, c, b, k2, stats, L, rho, num, den, copies, total;
};

GaussLayout gauss_layout(const emc_problem* pb) {
  const Dims d = dims_of(pb);
  GaussLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (size_t)round_up((int64_t)bytes, 256);
    return at;
  };
  L.A = take((size_t)pb->n_rot * d.ps * sizeof(float));  // A = W - c, then W'
  L.G = take((size_t)pb->n_rot * d.ds * sizeof(float));  // G, then P / phi
  L.P = take((size_t)pb->n_rot * d.ds * sizeof(float));  // used when P_out is NULL
  L.s2 = take((size_t)pb->n_rot * sizeof(double));
  L.c = take((size_t)d.ps * sizeof(double));
  L.b = take((size_t)pb->n_data * sizeof(double));
  L.k2 = take((size_t)pb->n_data * sizeof(double));
  L.stats = take((size_t)pb->n_data * 2 * sizeof(double));
  L.L = take((size_t)pb->n_data * sizeof(double));
  L.rho = take((size_t)pb->n_rot * sizeof(double));
  L.num = take((size_t)d.grid * sizeof(double));
  L.den = take((size_t)d.grid * sizeof(double));
  L.copies = take(copies_bytes(pb));
  L.total = o;
  return L;
}

}  // namespace

emc_status emc_gaussian_workspace_bytes(const emc_problem* pb, size_t* bytes) {
  CHECK(check_problem(pb, false));
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = gauss_layout(pb).total;
  return EMC_OK;
}

emc_status emc_iterate_gaussian(const emc_problem* pb, double sigma, const float* model_in, const void* K_packed,
                                float* phi, int32_t phi_from_model, float* model_out, double* loglik, float* P_out,
                                void* ws, size_t ws_bytes, hipStream_t st) {
  CHECK(check_problem(pb, true));
  if (pb->precision != EMC_PREC_FP32)
    return fail(EMC_ERR_UNSUPPORTED, "the Gaussian model runs in the FP32 form only");
  if (!(sigma > 0.0) || !(sigma < INFINITY)) return fail(EMC_ERR_INVALID_ARG, "sigma must be positive and finite");
  CHECK(need(model_in, 4, "model_in"));
  CHECK(need(model_out, 4, "model_out"));
  CHECK(need(loglik, 8, "loglik"));
  if (pb->n_data > 0) {
    CHECK(need(K_packed, 16, "K_packed"));
    CHECK(need(phi, 4, "phi"));
  }
  if (P_out) CHECK(need(P_out, 16, "P_out"));
  const GaussLayout Lo = gauss_layout(pb);
  if (!ws) return fail(EMC_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(ws, 256)) return fail(EMC_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < Lo.total) return fail(EMC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, Lo.total);
  const Dims d = dims_of(pb);
  char* w = (char*)ws;
  float* A = (float*)(w + Lo.A);
  float* G = (float*)(w + Lo.G);
  float* P = P_out ? P_out : (float*)(w + Lo.P);
  double* s2 = (double*)(w + Lo.s2);
  double* c = (double*)(w + Lo.c);
  double* b = (double*)(w + Lo.b);
  double* k2 = (double*)(w + Lo.k2);
  double* stats = (double*)(w + Lo.stats);
  double* L = (double*)(w + Lo.L);
  double* rho = (double*)(w + Lo.rho);
  double* num = (double*)(w + Lo.num);
  double* den = (double*)(w + Lo.den);
  HIP_TRY(launch_fill_zero_f64(num, (size_t)d.grid, st), "zero num");
  HIP_TRY(launch_fill_zero_f64(den, (size_t)d.grid, st), "zero den");
  if (pb->n_data > 0) {
    // expansion (eq. (2.9)), centred slices and the per-rotation sum of squares
    HIP_TRY(launch_gauss_expand(model_in, pb->grid_n, pb->q, pb->mask, pb->quat, pb->n_pix, d.ps, pb->n_rot, c, A, s2,
                                st),
            "gaussian expand");
    const float* K = (const float*)K_packed;
    const float* KT = K + (size_t)pb->n_data * d.ps;
    HIP_TRY(launch_frame_dot(K, false, d.ps, pb->n_data, c, b, st), "frame_dot");
    HIP_TRY(launch_frame_sq(K, d.ps, pb->n_data, k2, st), "frame_sq");
    // G_jk = sum_i (W_ij - c_i) K_ik (FP32 MFMA); b_k is added in the E-step
    HIP_TRY(launch_gemm_f32_nt(A, K, G, pb->n_rot, pb->n_data, d.ps, d.ps, d.ps, d.ds, st), "gaussian gemm");
    // E-step (eq. (2.4) with eq. (2.3)), M-step operand P / phi, fluence update (eq. (2.6)), rho
    HIP_TRY(launch_gauss_estep(G, phi, P, d.ds, pb->n_rot, pb->n_data, pb->log_w, s2, b, k2, phi_from_model != 0,
                               sigma, stats, L, rho, st),
            "gaussian estep");
    // M-step numerator (eq. (2.11)): W'_ji = sum_k (P_jk / phi_jk) K_ik, then the c-step (eq. (2.12))
    HIP_TRY(launch_gemm_f32_nt(G, KT, A, pb->n_rot, d.ps, d.ds, d.ds, d.ds, d.ps, st), "gaussian mstep gemm");
    CHECK(run_scatter(pb, A, d.ps, rho, num, den, (double*)(w + Lo.copies), st));
  }
  CHECK(run_finalize(pb, num, den, model_in, model_out, L, pb->n_data, loglik, st));
  return EMC_OK;
}

}  // extern "C"

// =========================================================================== proposal network
namespace {

constexpr int kConvCI[4] = {1, 32, 64, 128};
constexpr int kConvCO[4] = {32, 64, 128, 128};
constexpr int kConvIH[4] = {64, 32, 16, 8};
constexpr int kFlat = 2048;

struct CnnLayout {
  int64_t w[4], b[4], wf, bf, total;  // parameter offsets (floats)
};

CnnLayout cnn_layout(int n_cells) {
  CnnLayout L;
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    L.w[l] = o;
    o += (int64_t)kConvCO[l] * kConvCI[l] * 9;
    L.b[l] = o;
    o += kConvCO[l];
  }
  L.wf = o;
  o += (int64_t)n_cells * kFlat;
  L.bf = o;
  o += n_cells;
  L.total = o;
  return L;
}

int64_t act_size(int l) {  // floats per sample of activation l (output of conv layer l)
  const int oh = kConvIH[l] / 2;
  return (int64_t)kConvCO[l] * oh * oh;
}

int64_t pix_of(int l) { return (int64_t)(kConvIH[l] / 2) * (kConvIH[l] / 2); }  // output pixels per sample

// Activations and their gradients are channel-major over the batch: act[c][n * P + p]
struct CnnWs {
  size_t act[4], dact[4], col[4], dcol, part, rpart, flat, dflat, z, dz, total;
};

// floats of split partial products a contraction of M x N over K needs (0 when unsplit)
size_t split_floats(int M, int N, int64_t K) {
  const int s = gemm_str_splits(M, N, K);
  return s > 1 ? (size_t)s * M * N : 0;
}

CnnWs cnn_ws(int n_cells, int B) {
  CnnWs W;
  size_t o = 0;
  auto take = [&](size_t floats) {
    size_t at = o;
    o += (size_t)round_up((int64_t)(floats * 4), 256);
    return at;
  };
  size_t dcol = 0, part = 0;
  for (int l = 0; l < 4; ++l) {
    const int64_t M = (int64_t)B * pix_of(l);
    const int Kc = kConvCI[l] * 9;
    W.act[l] = take((size_t)B * act_size(l));
    W.dact[l] = take((size_t)B * act_size(l));
    W.col[l] = take((size_t)Kc * M);
    if (l > 0) dcol = std::max(dcol, (size_t)Kc * M);
    part = std::max({part, split_floats(kConvCO[l], (int)M, Kc), split_floats(kConvCO[l], Kc, M),
                     split_floats(Kc, (int)M, kConvCO[l])});
  }
  part = std::max({part, split_floats(B, n_cells, kFlat), split_floats(n_cells, kFlat, B),
                   split_floats(B, kFlat, n_cells)});
  W.dcol = take(dcol);
  W.part = take(part);
  W.rpart = take((size_t)128 * 64);  // row sums: rows (channels) x 64 parts
  W.flat = take((size_t)B * kFlat);
  W.dflat = take((size_t)B * kFlat);
  W.z = take((size_t)B * n_cells);
  W.dz = take((size_t)B * n_cells);
  W.total = o;
  return W;
}

emc_status check_cnn(int32_t n_cells, int32_t B, const void* ws, size_t ws_bytes) {
  if (n_cells < 1 || n_cells > (1 << 20)) return fail(EMC_ERR_INVALID_ARG, "n_cells=%d outside [1, 2^20]", n_cells);
  if (B < 1 || B > (1 << 16)) return fail(EMC_ERR_INVALID_ARG, "batch=%d outside [1, 65536]", B);
  if (!ws) return fail(EMC_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(ws, 256)) return fail(EMC_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  const size_t need_b = cnn_ws(n_cells, B).total;
  if (ws_bytes < need_b) return fail(EMC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need_b);
  return EMC_OK;
}

// forward into the workspace activations (and the layers' im2col operands); logits to `z`
emc_status run_cnn_forward(int n_cells, const float* p, const float* x, int B, float* z, char* w, hipStream_t st) {
  const CnnLayout L = cnn_layout(n_cells);
  const CnnWs W = cnn_ws(n_cells, B);
  const float* in = x;  // [1][n][64][64] is channel-major already
  for (int l = 0; l < 4; ++l) {
    const int64_t M = (int64_t)B * pix_of(l);
    const int Kc = kConvCI[l] * 9;
    float* col = (float*)(w + W.col[l]);
    float* out = (float*)(w + W.act[l]);
    HIP_TRY(launch_im2col(in, kConvCI[l], kConvIH[l], M, col, st), "im2col");
    // out[o][m] = relu(b[o] + sum_kc W[o][kc] col[kc][m])
    HIP_TRY(launch_gemm_str(true, p + L.w[l], Kc, false, col, M, out, M, kConvCO[l], (int)M, Kc,
                            gemm_str_splits(kConvCO[l], (int)M, Kc), (float*)(w + W.part), p + L.b[l], true, st),
            "conv forward");
    in = out;
  }
  float* flat = (float*)(w + W.flat);
  HIP_TRY(launch_flatten(in, kConvCO[3], (int)pix_of(3), B, flat, true, st), "flatten");
  // z[b][c] = sum_j flat[b][j] Wf[c][j]
  HIP_TRY(launch_gemm_str(true, flat, kFlat, true, p + L.wf, kFlat, z, n_cells, B, n_cells, kFlat,
                          gemm_str_splits(B, n_cells, kFlat), (float*)(w + W.part), nullptr, false, st),
          "fc forward");
  HIP_TRY(launch_add_bias(z, p + L.bf, B, n_cells, st), "fc bias");
  return EMC_OK;
}

}  // namespace

extern "C" {

int64_t emc_cnn_param_count(int32_t n_cells) { return n_cells < 1 ? 0 : cnn_layout(n_cells).total; }

emc_status emc_cnn_workspace_bytes(int32_t n_cells, int32_t max_batch, size_t* bytes) {
  if (n_cells < 1 || max_batch < 1) return fail(EMC_ERR_INVALID_ARG, "n_cells and max_batch must be >= 1");
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = cnn_ws(n_cells, max_batch).total;
  return EMC_OK;
}

emc_status emc_cnn_preprocess(const emc_problem* pb, const void* K_packed, const int32_t* bins,
                              const int32_t* frames, int32_t B, float* x, hipStream_t st) {
  CHECK(check_problem(pb, false));
  if (B < 0) return fail(EMC_ERR_INVALID_ARG, "batch=%d < 0", B);
  if (B == 0) return EMC_OK;
  if (!frames && B > pb->n_data) return fail(EMC_ERR_INVALID_ARG, "batch %d exceeds n_data %d", B, pb->n_data);
  CHECK(need(K_packed, 16, "K_packed"));
  CHECK(need(bins, 4, "bins"));
  CHECK(need(x, 4, "x"));
  if (frames) CHECK(need(frames, 4, "frames"));
  HIP_TRY(launch_bin_log(K_packed, is_bf16(pb), dims_of(pb).ps, pb->n_pix, bins, frames, B, x, st), "bin_log");
  return EMC_OK;
}

emc_status emc_cnn_forward(int32_t n_cells, const float* params, const float* x, int32_t B, float* logits, void* ws,
                           size_t ws_bytes, hipStream_t st) {
  CHECK(check_cnn(n_cells, B, ws, ws_bytes));
  CHECK(need(params, 16, "params"));
  CHECK(need(x, 4, "x"));
  CHECK(need(logits, 4, "logits"));
  return run_cnn_forward(n_cells, params, x, B, logits, (char*)ws, st);
}

emc_status emc_cnn_gradients(int32_t n_cells, const float* params, const float* x, const float* T, int32_t B,
                             float* grads, double* loss, void* ws, size_t ws_bytes, hipStream_t st) {
  CHECK(check_cnn(n_cells, B, ws, ws_bytes));
  CHECK(need(params, 16, "params"));
  CHECK(need(x, 4, "x"));
  CHECK(need(T, 4, "T"));
  CHECK(need(grads, 16, "grads"));
  CHECK(need(loss, 8, "loss"));
  char* w = (char*)ws;
  const CnnLayout L = cnn_layout(n_cells);
  const CnnWs W = cnn_ws(n_cells, B);
  float* z = (float*)(w + W.z);
  float* dz = (float*)(w + W.dz);
  CHECK(run_cnn_forward(n_cells, params, x, B, z, w, st));
  HIP_TRY(launch_fill_zero_f64(loss, 1, st), "zero loss");
  HIP_TRY(launch_softmax_xent(z, T, n_cells, B, dz, loss, st), "softmax xent");
  const float* flat = (const float*)(w + W.flat);
  float* dflat = (float*)(w + W.dflat);
  float* part = (float*)(w + W.part);
  // fully connected: dWf[c][j] = sum_b dz[b][c] flat[b][j]; dbf = column sums of dz;
  // dflat[b][j] = sum_c dz[b][c] Wf[c][j]
  HIP_TRY(launch_gemm_str(false, dz, n_cells, false, flat, kFlat, grads + L.wf, kFlat, n_cells, kFlat, B,
                          gemm_str_splits(n_cells, kFlat, B), part, nullptr, false, st),
          "fc dW");
  HIP_TRY(launch_col_sum(dz, B, n_cells, grads + L.bf, st), "fc db");
  HIP_TRY(launch_gemm_str(true, dz, n_cells, false, params + L.wf, kFlat, dflat, kFlat, B, kFlat, n_cells,
                          gemm_str_splits(B, kFlat, n_cells), part, nullptr, false, st),
          "fc dx");
  HIP_TRY(launch_flatten(dflat, kConvCO[3], (int)pix_of(3), B, (float*)(w + W.dact[3]), false, st), "unflatten");
  for (int l = 3; l >= 0; --l) {
    const int64_t M = (int64_t)B * pix_of(l);
    const int Kc = kConvCI[l] * 9;
    float* dl = (float*)(w + W.dact[l]);
    const float* col = (const float*)(w + W.col[l]);
    HIP_TRY(launch_relu_mask(dl, (const float*)(w + W.act[l]), (int64_t)B * act_size(l), st), "relu backward");
    // dW[o][kc] = sum_m dout[o][m] col[kc][m] (split over m); db[o] = sum_m dout[o][m]
    HIP_TRY(launch_gemm_str(true, dl, M, true, col, M, grads + L.w[l], Kc, kConvCO[l], Kc, M,
                            gemm_str_splits(kConvCO[l], Kc, M), part, nullptr, false, st),
            "conv weight gradient");
    HIP_TRY(launch_row_sum(dl, kConvCO[l], M, (float*)(w + W.rpart), grads + L.b[l], st), "conv bias gradient");
    if (l > 0) {
      // dcol[kc][m] = sum_o W[o][kc] dout[o][m], then summed over the taps that read each input
      float* dcol = (float*)(w + W.dcol);
      HIP_TRY(launch_gemm_str(false, params + L.w[l], Kc, false, dl, M, dcol, M, Kc, (int)M, kConvCO[l],
                              gemm_str_splits(Kc, (int)M, kConvCO[l]), part, nullptr, false, st),
              "conv data gradient");
      HIP_TRY(launch_col2im(dcol, kConvCI[l], kConvIH[l], B, (float*)(w + W.dact[l - 1]), st), "col2im");
    }
  }
  return EMC_OK;
}

emc_status emc_cnn_adam(int32_t n_cells, float* params, const float* grads, float* m, float* v, int32_t step,
                        float lr, hipStream_t st) {
  if (n_cells < 1) return fail(EMC_ERR_INVALID_ARG, "n_cells=%d < 1", n_cells);
  if (step < 1) return fail(EMC_ERR_INVALID_ARG, "step=%d < 1 (Adam steps count from 1)", step);
  CHECK(need(params, 4, "params"));
  CHECK(need(grads, 4, "grads"));
  CHECK(need(m, 4, "m"));
  CHECK(need(v, 4, "v"));
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - pow(0.9, step)), c2 = (float)(1.0 - pow(0.999, step));
  HIP_TRY(launch_adam(params, grads, m, v, cnn_layout(n_cells).total, lr, b1, b2, eps, c1, c2, st), "adam");
  return EMC_OK;
}

emc_status emc_cnn_topk(const float* logits, int64_t rows, int32_t n_cells, int32_t k, int32_t* out, hipStream_t st) {
  if (rows < 0 || n_cells < 1 || n_cells > 8192 || k < 1 || k > n_cells)
    return fail(EMC_ERR_INVALID_ARG, "need rows >= 0, 1 <= k <= n_cells <= 8192");
  if (rows == 0) return EMC_OK;
  CHECK(need(logits, 4, "logits"));
  CHECK(need(out, 4, "out"));
  HIP_TRY(launch_topk(logits, rows, n_cells, k, false, out, st), "topk");
  return EMC_OK;
}

emc_status emc_cell_topk(const float* T, int64_t rows, int32_t n_cells, int32_t k, int32_t* out, hipStream_t st) {
  if (rows < 0 || n_cells < 1 || n_cells > 8192 || k < 1 || k > n_cells)
    return fail(EMC_ERR_INVALID_ARG, "need rows >= 0, 1 <= k <= n_cells <= 8192");
  if (rows == 0) return EMC_OK;
  CHECK(need(T, 4, "T"));
  CHECK(need(out, 4, "out"));
  HIP_TRY(launch_topk(T, rows, n_cells, k, true, out, st), "cell topk");
  return EMC_OK;
}

emc_status emc_topk_union(const int32_t* a, int32_t ka, const int32_t* b, int32_t kb, int64_t rows, int32_t n_cells,
                          int32_t* out, hipStream_t st) {
  if (rows < 0 || n_cells < 1 || n_cells > 8192 || ka < 0 || kb < 0 || ka + kb < 1 || ka + kb > 512)
    return fail(EMC_ERR_INVALID_ARG, "need rows >= 0, 1 <= n_cells <= 8192, 1 <= ka + kb <= 512");
  if (rows == 0) return EMC_OK;
  if (ka > 0) CHECK(need(a, 4, "a"));
  if (kb > 0) CHECK(need(b, 4, "b"));
  CHECK(need(out, 4, "out"));
  HIP_TRY(launch_topk_union(a, ka, b, kb, rows, n_cells, out, st), "topk union");
  return EMC_OK;
}

emc_status emc_cell_targets(const emc_problem* pb, const void* P, const int32_t* cell_ptr, const int32_t* cell_rot,
                            int32_t n_cells, float* T, hipStream_t st) {
  CHECK(check_problem(pb, false));
  if (n_cells < 1) return fail(EMC_ERR_INVALID_ARG, "n_cells=%d < 1", n_cells);
  if (pb->n_data == 0) return EMC_OK;
  CHECK(need(P, 4, "P"));
  CHECK(need(cell_ptr, 4, "cell_ptr"));
  CHECK(need(cell_rot, 4, "cell_rot"));
  CHECK(need(T, 4, "T"));
  HIP_TRY(launch_cell_targets(P, is_bf16(pb), dims_of(pb).ds, pb->n_data, cell_ptr, cell_rot, n_cells, T, st),
          "cell targets");
  return EMC_OK;
}

}  // extern "C"

// =========================================================================== learned-proposal iteration
namespace {

int words_of(int n_cells) { return (n_cells + 31) / 32; }

constexpr int kMaxTop = 256;      // proposed cells per frame
constexpr int kBandPx = 128;      // granularity of the entry-offset table (the kernels' band)
constexpr int kTileFrames = 256;  // frames per candidate log-likelihood tile
constexpr int kGroupRot = 32;     // rotations per group
constexpr int kMaxDense = 16;     // bands handled by the M-step's dense product (at most)

int64_t group_cap(int n_rot, int n_cells) { return (int64_t)n_cells + (n_rot + kGroupRot - 1) / kGroupRot; }
int64_t tile_cap(int64_t g_max, int64_t n_cand) {
  const int64_t per = (n_cand + kTileFrames - 1) / kTileFrames;
  return g_max * per + 8 * per + 8;
}
int ntab_of(int n_pix) { return (int)(round_up(n_pix, 256) / kBandPx) + 1; }
// 16-byte chunks of the band format: every non-empty (frame, band) pads at most one
int64_t chunk_cap(int64_t nz_cap, int64_t n_cand, int n_pix) { return (nz_cap + 7) / 8 + n_cand * (ntab_of(n_pix) - 1); }

// Carving of the plan buffer (capacities known before the build).
struct PlanLayout {
  size_t cell_of, cell_ptr, cell_rot, pack_of, cell_first, pack_rot, rot_local, cand_frames, audit_frames, cand_cells,
      pair_col, cf_ptr, cf_frame, cf_mask, cg_ptr, groups, grp_off, tiles, mask_audit, chunks, runs, band_cnt,
      band_ptr, dense_band, dense_list, kt_dense, band_mean, hist, cursor, keys, order, mark, frame_ptr, gsize, xcd,
      cnt, nn, slot_cell, pack_slot, slot_cnt, slot_ptr, cell_slot, pack_ptr, bits, prim, scalars, total;
};

PlanLayout plan_layout(int n_rot, int n_data, int n_pix, int n_cells, int k_top, int n_audit, int64_t nz_cap) {
  const int64_t n_cand = (int64_t)n_data - n_audit;
  const int64_t n_pairs = n_cand * k_top;
  const int64_t g_max = group_cap(n_rot, n_cells);
  const int w = words_of(n_cells);
  PlanLayout L;
  size_t o = 0;
  auto take = [&](int64_t bytes) {
    size_t at = o;
    o += (size_t)round_up(bytes > 0 ? bytes : 1, 256);
    return at;
  };
  const int64_t nkeys = std::max<int64_t>(n_cells + 1, std::max<int64_t>(n_rot, (int64_t)1) + 1);
  L.cell_of = take((int64_t)n_rot * 4);
  L.cell_ptr = take((int64_t)(n_cells + 2) * 8);
  L.cell_rot = take((int64_t)n_rot * 4);
  L.pack_of = take((int64_t)n_cells * 4);
  L.cell_first = take((int64_t)n_cells * 4);
  L.pack_rot = take((int64_t)n_rot * 4);
  L.rot_local = take((int64_t)n_rot * 4);
  L.cand_frames = take(n_cand * 4);
  L.audit_frames = take((int64_t)n_audit * 4);
  L.cand_cells = take(n_pairs * 4);
  L.pair_col = take(n_pairs * 4);
  L.cf_ptr = take((int64_t)(n_cells + 2) * 8);
  L.cf_frame = take(n_pairs * 4);
  L.cf_mask = take(n_pairs * 4);
  L.cg_ptr = take((int64_t)(n_cells + 1) * 8);
  L.groups = take(g_max * 16);
  L.grp_off = take((g_max + 1) * 8);
  L.tiles = take(tile_cap(g_max, n_cand) * 8);
  L.mask_audit = take((int64_t)n_audit * w * 4);
  const int64_t n_fb = n_cand * (ntab_of(n_pix) - 1);  // (band, frame) entries
  L.chunks = take(chunk_cap(nz_cap, n_cand, n_pix) * 16);
  L.runs = take(2 * n_cand * run_count(ntab_of(n_pix) - 1) * 16);
  L.band_cnt = take(n_fb * 4);
  L.band_ptr = take((n_fb + 1) * 8);
  L.dense_band = take((int64_t)(ntab_of(n_pix) - 1) * 4);
  L.dense_list = take(kMaxDense * 4);
  L.kt_dense = take((int64_t)kMaxDense * kBandPx * round_up(n_cand, 256) * 2);
  L.band_mean = take((int64_t)(ntab_of(n_pix) - 1) * 4);
  L.hist = take(nkeys * 4);
  L.cursor = take(nkeys * 4);
  L.keys = take(std::max<int64_t>(n_pairs, n_data) * 4);
  L.order = take(std::max<int64_t>(n_pairs, n_data) * 4);
  L.mark = take((int64_t)n_data * 4);
  L.frame_ptr = take((int64_t)(n_cells + 2) * 8);
  L.gsize = take(g_max * 8);
  L.xcd = take(g_max * 4);
  L.cnt = take((int64_t)n_cells * 4);
  L.nn = take((int64_t)n_cells * 16 * 4);
  L.slot_cell = take((int64_t)n_cells * 4);
  L.pack_slot = take((int64_t)(n_cells + 1) * 4);
  L.slot_cnt = take((int64_t)n_cells * 4);
  L.slot_ptr = take((int64_t)(n_cells + 1) * 8);
  L.cell_slot = take((int64_t)n_cells * 4);
  L.pack_ptr = take((int64_t)(n_cells + 1) * 8);
  L.bits = take(n_pairs * 4);
  L.prim = take(n_pairs * 4);
  L.scalars = take(64);
  L.total = o;
  return L;
}

}  // namespace

namespace emc {
__global__ void top1_keys_kernel(const int32_t* __restrict__ topk, int k_top, const int32_t* __restrict__ mark,
                                 const int32_t* __restrict__ pack_of, int64_t n, int n_cells,
                                 int32_t* __restrict__ keys) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= n) return;
  const int32_t c = topk[f * k_top];
  // the pack of the first proposed cell; audited frames sort after every pack,
  // frames without a valid proposal go to the last key below them
  keys[f] = mark[f] ? n_cells : (c >= 0 && c < n_cells ? pack_of[c] : n_cells - 1);
}
__global__ void mark_kernel(const int32_t* __restrict__ audit, int64_t n_audit, int64_t n_data,
                            int32_t* __restrict__ mark) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (a >= n_audit) return;
  const int32_t f = audit[a];
  if (f >= 0 && f < n_data) mark[f] = 1;
}
__global__ void copy_i32_kernel(const int32_t* __restrict__ src, int64_t n, int32_t* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = src[e];
}
__global__ void mean2_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) s += x[k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = n > 0 ? ((red[0] + red[1]) + (red[2] + red[3])) / (double)n : NAN;
}
}  // namespace emc

extern "C" {

emc_status emc_proposal_bytes(const emc_problem* pb, int32_t n_cells, int32_t k_top, int32_t n_audit,
                              int64_t nz_cap, size_t* bytes) {
  CHECK(check_problem(pb, false));
  if (n_cells < 1 || n_cells > 8192) return fail(EMC_ERR_INVALID_ARG, "n_cells=%d outside [1, 8192]", n_cells);
  if (k_top < 1 || k_top > kMaxTop) return fail(EMC_ERR_INVALID_ARG, "k_top=%d outside [1, %d]", k_top, kMaxTop);
  if (n_audit < 0 || n_audit > pb->n_data) return fail(EMC_ERR_INVALID_ARG, "n_audit outside [0, n_data]");
  if (nz_cap < 1) return fail(EMC_ERR_INVALID_ARG, "nz_cap < 1");
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = plan_layout(pb->n_rot, pb->n_data, pb->n_pix, n_cells, k_top, n_audit, nz_cap).total;
  return EMC_OK;
}

emc_status emc_proposal_build(const emc_problem* pb, const float* coarse, int32_t n_cells, const int32_t* topk,
                              int32_t k_top, const int32_t* audit, int32_t n_audit, const uint16_t* counts,
                              int64_t nz_cap, void* buf, size_t buf_bytes, emc_proposal* plan, hipStream_t st) {
  CHECK(check_problem(pb, true));
  if (n_cells < 1 || n_cells > 8192) return fail(EMC_ERR_INVALID_ARG, "n_cells=%d outside [1, 8192]", n_cells);
  if (k_top < 1 || k_top > kMaxTop) return fail(EMC_ERR_INVALID_ARG, "k_top=%d outside [1, %d]", k_top, kMaxTop);
  if (n_audit < 0 || n_audit > pb->n_data) return fail(EMC_ERR_INVALID_ARG, "n_audit outside [0, n_data]");
  if (pb->n_data < 1) return fail(EMC_ERR_INVALID_ARG, "the proposal needs frames");
  if (pb->n_pix > 65536) return fail(EMC_ERR_UNSUPPORTED, "the proposal form needs n_pix <= 65536");
  if (nz_cap < 1) return fail(EMC_ERR_INVALID_ARG, "nz_cap < 1");
  CHECK(need(coarse, 16, "coarse"));
  CHECK(need(topk, 4, "topk"));
  if (n_audit > 0) CHECK(need(audit, 4, "audit"));
  CHECK(need(counts, 2, "counts"));
  if (!plan) return fail(EMC_ERR_INVALID_ARG, "plan is NULL");
  const PlanLayout L = plan_layout(pb->n_rot, pb->n_data, pb->n_pix, n_cells, k_top, n_audit, nz_cap);
  if (!buf || !aligned(buf, 256)) return fail(EMC_ERR_WORKSPACE, "plan buffer is NULL or not 256-byte aligned");
  if (buf_bytes < L.total) return fail(EMC_ERR_WORKSPACE, "plan buffer has %zu bytes, needs %zu", buf_bytes, L.total);
  char* b = (char*)buf;
  const int64_t n_data = pb->n_data, n_cand = n_data - n_audit, n_pairs = n_cand * k_top;
  const int64_t g_max = group_cap(pb->n_rot, n_cells);
  const int w = words_of(n_cells);
  const int ntab = ntab_of(pb->n_pix);
  emc_proposal P{};
  P.n_cells = n_cells;
  P.k_top = k_top;
  P.n_cand = (int32_t)n_cand;
  P.n_audit = n_audit;
  P.words = w;
  P.n_bands = ntab - 1;
  P.cell_of = (int32_t*)(b + L.cell_of);
  P.cell_ptr = (int64_t*)(b + L.cell_ptr);
  P.cell_rot = (int32_t*)(b + L.cell_rot);
  P.pack_of = (int32_t*)(b + L.pack_of);
  P.cell_first = (int32_t*)(b + L.cell_first);
  P.pack_rot = (int32_t*)(b + L.pack_rot);
  P.rot_local = (int32_t*)(b + L.rot_local);
  P.cand_frames = (int32_t*)(b + L.cand_frames);
  P.audit_frames = (int32_t*)(b + L.audit_frames);
  P.cand_cells = (int32_t*)(b + L.cand_cells);
  P.pair_col = (int32_t*)(b + L.pair_col);
  P.cf_ptr = (int64_t*)(b + L.cf_ptr);
  P.cf_frame = (int32_t*)(b + L.cf_frame);
  P.cf_mask = (uint32_t*)(b + L.cf_mask);
  P.cg_ptr = (int64_t*)(b + L.cg_ptr);
  P.groups = (void*)(b + L.groups);
  P.grp_off = (int64_t*)(b + L.grp_off);
  P.tiles = (void*)(b + L.tiles);
  P.mask_audit = (uint32_t*)(b + L.mask_audit);
  P.chunks = (void*)(b + L.chunks);
  P.runs = b + L.runs;
  int32_t* band_cnt = (int32_t*)(b + L.band_cnt);
  int64_t* band_ptr = (int64_t*)(b + L.band_ptr);
  const int64_t n_fb = n_cand * (ntab - 1);
  P.dense_band = (int32_t*)(b + L.dense_band);
  P.dense_list = (int32_t*)(b + L.dense_list);
  P.kt_dense = (void*)(b + L.kt_dense);
  P.ld_dense = round_up(n_cand, 256);
  int32_t* hist = (int32_t*)(b + L.hist);
  int32_t* cursor = (int32_t*)(b + L.cursor);
  int32_t* keys = (int32_t*)(b + L.keys);
  int32_t* order = (int32_t*)(b + L.order);
  int32_t* mark = (int32_t*)(b + L.mark);
  int64_t* frame_ptr = (int64_t*)(b + L.frame_ptr);
  int64_t* gsize = (int64_t*)(b + L.gsize);
  int32_t* xcd = (int32_t*)(b + L.xcd);
  int32_t* cnt = (int32_t*)(b + L.cnt);
  int64_t* scal = (int64_t*)(b + L.scalars);  // [0] n_tiles, [1] flags (int32): 1 count range, 2 repeated cell
  int32_t* over = (int32_t*)(scal + 1);
  // 1. coarse cell of every fine rotation; rotations grouped by cell; packs of
  // neighbouring cells and the rotations in pack order
  HIP_TRY(launch_assign_cells(pb->quat, pb->n_rot, coarse, n_cells, P.cell_of, st), "assign cells");
  HIP_TRY(launch_counting_sort(P.cell_of, pb->n_rot, n_cells, hist, cursor, P.cell_ptr, P.cell_rot, nullptr, st),
          "sort rotations");
  int32_t* cell_slot = (int32_t*)(b + L.cell_slot);
  int32_t* pack_slot = (int32_t*)(b + L.pack_slot);
  int64_t* pack_ptr = (int64_t*)(b + L.pack_ptr);
  int32_t* n_packs_dev = (int32_t*)(scal + 3);
  HIP_TRY(launch_packs(coarse, n_cells, P.cell_ptr, P.cell_of, P.cell_rot, pb->n_rot, (int32_t*)(b + L.nn), P.pack_of,
                       (int32_t*)(b + L.slot_cell), pack_slot, n_packs_dev, (int32_t*)(b + L.slot_cnt),
                       (int64_t*)(b + L.slot_ptr), cell_slot, P.cell_first, pack_ptr, P.pack_rot, P.rot_local, st),
          "packs");
  // 2. frames: audited ones apart, the others grouped by their first proposed cell
  HIP_TRY(launch_fill_i32(mark, n_data, 0, st), "mark");
  if (n_audit > 0)
    emc::mark_kernel<<<(unsigned)((n_audit + 255) / 256), 256, 0, st>>>(audit, n_audit, n_data, mark);
  emc::top1_keys_kernel<<<(unsigned)((n_data + 255) / 256), 256, 0, st>>>(topk, k_top, mark, P.pack_of, n_data,
                                                                           n_cells, keys);
  HIP_TRY(launch_counting_sort(keys, n_data, n_cells + 1, hist, cursor, frame_ptr, order, nullptr, st), "sort frames");
  if (n_cand > 0) emc::copy_i32_kernel<<<(unsigned)((n_cand + 255) / 256), 256, 0, st>>>(order, n_cand, P.cand_frames);
  if (n_audit > 0)
    emc::copy_i32_kernel<<<(unsigned)((n_audit + 255) / 256), 256, 0, st>>>(order + n_cand, n_audit, P.audit_frames);
  HIP_TRY(launch_cand_mask(topk, k_top, P.audit_frames, n_audit, w, P.mask_audit, st), "audit masks");
  // 3. (frame, proposed cell) pairs: each pack's frame list, every frame once with
  // the bits of the pack's cells it proposes
  HIP_TRY(launch_fill_i32(over, 1, 0, st), "flags");
  HIP_TRY(launch_cand_cells(topk, k_top, P.cand_frames, n_cand, n_cells, P.cand_cells, keys, st), "candidate cells");
  HIP_TRY(launch_dup_check(P.cand_cells, k_top, n_cand, n_cells, over, st), "repeated cells");
  uint32_t* bits = (uint32_t*)(b + L.bits);
  int32_t* prim = (int32_t*)(b + L.prim);
  HIP_TRY(launch_pack_pairs(P.cand_cells, k_top, n_cand, P.pack_of, cell_slot, pack_slot, n_cells, keys, bits, prim,
                            st),
          "pack pairs");
  HIP_TRY(launch_counting_sort(keys, n_pairs, n_cells + 1, hist, cursor, P.cf_ptr, order, nullptr, st), "sort pairs");
  HIP_TRY(launch_pack_columns(order, P.cf_ptr, n_cells, n_pairs, k_top, keys, bits, prim, P.cf_frame, P.cf_mask,
                              P.pair_col, st),
          "pair columns");
  // 4. groups of up to 32 rotations per pack, their storage and the log-likelihood tiles
  HIP_TRY(launch_pack_groups(pack_ptr, P.cf_ptr, n_cells, cnt, P.cg_ptr, (int4*)P.groups, gsize, P.grp_off, g_max, st),
          "groups");
  HIP_TRY(launch_group_tiles((const int4*)P.groups, P.cg_ptr, n_cells, P.cf_ptr, xcd, (int2*)P.tiles,
                             tile_cap(g_max, n_cand), scal, st),
          "tiles");
  // 5. the candidate frames in the sparse band format
  HIP_TRY(launch_band_count(counts, pb->mask, pb->n_pix, P.cand_frames, n_cand, ntab - 1, band_cnt, over, st),
          "band count");
  HIP_TRY(launch_scan(band_cnt, n_fb, band_ptr, st), "chunk offsets");
  int32_t* n_dense_dev = (int32_t*)(scal + 2);
  HIP_TRY(launch_dense_bands(band_cnt, n_cand, ntab - 1, (float*)(b + L.band_mean), P.dense_band, P.dense_list,
                             n_dense_dev, st),
          "dense bands");
  int64_t host[7] = {0, 0, 0, 0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(&host[0], scal, 16, hipMemcpyDeviceToHost, st), "read n_tiles");
  HIP_TRY(hipMemcpyAsync(&host[5], n_dense_dev, 4, hipMemcpyDeviceToHost, st), "read n_dense");
  HIP_TRY(hipMemcpyAsync(&host[6], n_packs_dev, 4, hipMemcpyDeviceToHost, st), "read n_packs");
  HIP_TRY(hipMemcpyAsync(&host[2], P.cg_ptr + n_cells, 8, hipMemcpyDeviceToHost, st), "read n_groups");
  HIP_TRY(hipMemcpyAsync(&host[3], P.grp_off + g_max, 8, hipMemcpyDeviceToHost, st), "read n_g");
  HIP_TRY(hipMemcpyAsync(&host[4], band_ptr + n_fb, 8, hipMemcpyDeviceToHost, st), "read n_chunks");
  HIP_TRY(hipStreamSynchronize(st), "proposal build sync");
  const int32_t flags = (int32_t)host[1];
  if (flags & 2) return fail(EMC_ERR_INVALID_ARG, "a frame lists the same cell more than once");
  if (host[0] < 0) return fail(EMC_ERR_INVALID_ARG, "inconsistent proposal lists");
  if (flags & 1) return fail(EMC_ERR_RANGE, "a photon count exceeds 256, which BF16 cannot hold exactly");
  if (host[4] > chunk_cap(nz_cap, n_cand, pb->n_pix) || host[4] > (int64_t)INT32_MAX)
    return fail(EMC_ERR_WORKSPACE, "the candidate frames need %lld chunks, nz_cap %lld allows %lld", (long long)host[4],
                (long long)nz_cap, (long long)chunk_cap(nz_cap, n_cand, pb->n_pix));
  HIP_TRY(launch_run_table(band_ptr, n_cand, ntab - 1, P.runs, st), "run records");
  HIP_TRY(launch_band_fill(counts, pb->mask, pb->n_pix, P.cand_frames, n_cand, ntab - 1, P.runs,
                           P.chunks, st),
          "band fill");
  P.n_dense = (int32_t)host[5];
  P.n_packs = (int32_t)host[6];
  HIP_TRY(launch_dense_pack(counts, pb->mask, pb->n_pix, P.cand_frames, n_cand, P.ld_dense, P.n_dense, P.dense_list,
                            P.kt_dense, st),
          "dense pack");
  P.n_tiles = host[0];
  P.n_groups = host[2];
  P.n_g = host[3];
  P.n_chunks = host[4];
  P.n_rot = pb->n_rot;
  P.n_pix = pb->n_pix;
  P.quat = pb->quat;
  P.mask = pb->mask;
  *plan = P;
  return EMC_OK;
}

}  // extern "C"

namespace {

struct PropWs {
  size_t slices, S, scale, c, b, L, G, P, Ga, Pa, stats_a, stats_p, rho_a, recall, rho, num, den, Pd, Wd, copies,
      cst, Ga_part, total;
};

// k-range parts of the dense-band M-step product (its partial products are summed
// by the dense add)
constexpr int kMaxDenseSplits = 4;
int dense_splits(const emc_problem* pb, const emc_proposal* P) {
  if (P->n_dense <= 0) return 1;
  return gemm_bf16_splits(pb->n_rot, (int64_t)P->n_dense * kBandPx, P->ld_dense, kMaxDenseSplits);
}

// k-range parts of the audited frames' log-likelihood product (few frames: few
// output tiles over a full-detector reduction)
int audit_splits(const emc_problem* pb, const emc_proposal* P) {
  if (P->n_audit <= 0) return 1;
  return gemm_bf16_splits(pb->n_rot, P->n_audit, round_up(pb->n_pix, 256), kMaxDenseSplits);
}

PropWs prop_ws(const emc_problem* pb, const emc_proposal* P) {
  const int64_t ps = round_up(pb->n_pix, 256);
  const int64_t dsa = round_up(P->n_audit, 256);
  const int64_t grid = (int64_t)pb->grid_n * pb->grid_n * pb->grid_n;
  const int64_t n_frames = (int64_t)P->n_cand + P->n_audit;
  PropWs W;
  size_t o = 0;
  auto take = [&](int64_t bytes) {
    size_t at = o;
    o += (size_t)round_up(bytes > 0 ? bytes : 1, 256);
    return at;
  };
  W.slices = take((int64_t)pb->n_rot * ps * 4);  // BF16 hi + lo, later the FP32 M-step rows
  W.S = take((int64_t)pb->n_rot * 8);
  W.scale = take((int64_t)pb->n_rot * 4);
  W.c = take(ps * 8);
  W.b = take(n_frames * 8);
  W.L = take(n_frames * 8);
  W.G = take(P->n_g * 4);
  W.P = take(P->n_g * 2);
  W.Ga = take((int64_t)pb->n_rot * dsa * 4);
  W.Pa = take((int64_t)pb->n_rot * dsa * 2);
  W.stats_a = take((int64_t)P->n_audit * 16);
  W.stats_p = take((int64_t)kMaxLseChunks * P->n_audit * 16);  // rotation-chunk partials of the audit's E-step
  W.rho_a = take((int64_t)pb->n_rot * 8);
  W.recall = take((int64_t)P->n_audit * 8);
  W.rho = take((int64_t)pb->n_rot * 8);
  W.num = take(grid * 8);
  W.den = take(grid * 8);
  W.Pd = take(P->n_dense > 0 ? (int64_t)pb->n_rot * P->ld_dense * 2 : 0);
  W.Wd = take((int64_t)pb->n_rot * P->n_dense * kBandPx * 4 * dense_splits(pb, P));
  W.copies = take((int64_t)copies_bytes(pb));
  W.cst = take((int64_t)pb->n_rot * 8);  // log w_j - S_j in the packs' rotation order
  // partial products of the audit's split log-likelihood product
  const int as = audit_splits(pb, P);
  W.Ga_part = take(as > 1 ? (int64_t)as * pb->n_rot * dsa * 4 : 0);
  W.total = o;
  return W;
}

emc_status check_plan(const emc_problem* pb, const emc_proposal* P) {
  if (!P) return fail(EMC_ERR_INVALID_ARG, "plan is NULL");
  // the plan's rotation lists and frame bands index this problem's slices and pixels
  if (P->n_rot != pb->n_rot || P->n_pix != pb->n_pix || P->quat != pb->quat || P->mask != pb->mask)
    return fail(EMC_ERR_INVALID_ARG, "proposal plan was built for another rotation set or detector");
  if (P->n_cand < 0 || P->n_audit < 0 || (int64_t)P->n_cand + P->n_audit != pb->n_data)
    return fail(EMC_ERR_INVALID_ARG, "plan frames (%d + %d) do not match n_data %d", P->n_cand, P->n_audit, pb->n_data);
  if (P->k_top < 1 || P->k_top > kMaxTop || P->n_cells < 1 || P->words != words_of(P->n_cells) || P->n_g < 0 ||
      P->n_tiles < 0 || P->n_tiles % 8 != 0 || P->n_groups < 1 || P->n_groups > group_cap(pb->n_rot, P->n_cells) ||
      P->n_packs < 1 || P->n_packs > P->n_cells ||
      P->n_bands != ntab_of(pb->n_pix) - 1 || P->n_dense < 0 || P->n_dense > kMaxDense ||
      P->ld_dense != round_up(P->n_cand, 256))
    return fail(EMC_ERR_INVALID_ARG, "inconsistent plan");
  return EMC_OK;
}

}  // namespace

extern "C" {

emc_status emc_proposed_workspace_bytes(const emc_problem* pb, const emc_proposal* plan, size_t* bytes) {
  CHECK(check_problem(pb, false));
  CHECK(check_plan(pb, plan));
  if (!bytes) return fail(EMC_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = prop_ws(pb, plan).total;
  return EMC_OK;
}

}  // extern "C"

namespace {

// The restricted iteration up to the c-step sums (no division): expansion, candidate
// and audited log-likelihoods, E-steps, M-steps and the c-step into num/den (zeroed
// first unless `accumulate`; with `gated`, the sums are added only when the audit's
// recall reaches recall_min).  L [n_cand + n_audit]: log-evidence per frame.
emc_status run_proposed(const emc_problem* pb, const emc_proposal* plan, const void* K_audit, const float* model_in,
                        double* num, double* den, int32_t accumulate, bool gated, double recall_min, double* L,
                        double* recall_mean, char* w, hipEvent_t* stage_events, hipStream_t st) {
  const PropWs W = prop_ws(pb, plan);
  const int64_t ps = round_up(pb->n_pix, 256);
  const int64_t nc = plan->n_cand, na = plan->n_audit;
  const int64_t dsa = round_up(na, 256);
  void* slices = w + W.slices;
  double* S = (double*)(w + W.S);
  float* scale = (float*)(w + W.scale);
  double* c = (double*)(w + W.c);
  double* b = (double*)(w + W.b);
  float* G = (float*)(w + W.G);
  void* Pc = w + W.P;
  float* Ga = (float*)(w + W.Ga);
  void* Pa = w + W.Pa;
  double* stats_a = (double*)(w + W.stats_a);
  double* rho_a = (double*)(w + W.rho_a);
  double* recall = (double*)(w + W.recall);
  double* rho = (double*)(w + W.rho);
  void* Pd = plan->n_dense > 0 ? (void*)(w + W.Pd) : nullptr;
  float* Wd = (float*)(w + W.Wd);
  const int4* groups = (const int4*)plan->groups;
  auto mark = [&](int i) -> emc_status {
    if (stage_events) HIP_TRY(hipEventRecord(stage_events[i], st), "stage event");
    return EMC_OK;
  };
  CHECK(mark(0));
  // expansion (BF16 hi + lo slices with their row scales)
  CHECK(run_expand(pb, model_in, c, slices, S, scale, st));
  if (nc > 0)
    HIP_TRY(launch_band_dot(plan->runs, plan->n_bands, plan->chunks, nc, c, b, st), "band dot");
  CHECK(mark(1));
  // candidate frames: log-likelihoods per (group, listed frame), E-step over each frame's candidates
  if (nc > 0) {
    HIP_TRY(launch_cand_loglik((const int2*)plan->tiles, plan->n_tiles, groups, plan->grp_off, plan->cf_ptr,
                               plan->cf_frame, plan->runs, plan->chunks, plan->pack_rot,
                               slices, (int64_t)pb->n_rot * ps, scale, ps, G, st),
            "candidate loglik");
  }
  CHECK(mark(2));
  if (nc > 0) {
    // the dense bands' responsibility matrix is zero outside the candidate pairs
    if (Pd) HIP_TRY(launch_fill_zero_bytes(Pd, (int64_t)pb->n_rot * plan->ld_dense * 2, st), "zero dense P");
    HIP_TRY(launch_cand_estep(G, Pc, groups, plan->grp_off, plan->cg_ptr, plan->cand_cells, plan->pair_col,
                              plan->k_top, nc, plan->pack_of, plan->cell_first, plan->cell_ptr, plan->pack_rot,
                              plan->rot_local, pb->n_rot, pb->log_w, S, (double*)(w + W.cst), b, L,
                              Pd, plan->ld_dense,
                              (const int2*)plan->tiles, plan->n_tiles, plan->cf_ptr, plan->cf_frame, plan->cf_mask,
                              st),
            "candidate estep");
  }
  CHECK(mark(3));
  // audited frames: full search, recall of the proposal
  HIP_TRY(launch_fill_zero_f64(recall, (size_t)na, st), "zero recall");
  emc_problem pa = *pb;
  pa.n_data = (int32_t)na;
  if (na > 0) {
    CHECK(run_loglik(&pa, K_audit, slices, scale, c, Ga, b + nc, st, audit_splits(pb, plan),
                     (float*)(w + W.Ga_part)));
    CHECK(run_estep(&pa, Ga, S, b + nc, EMC_RESP_FULL, stats_a, Pa, L + nc, rho_a, st,
                    (double*)(w + W.stats_p)));
    HIP_TRY(launch_audit_recall(Pa, dsa, pb->n_rot, na, plan->mask_audit, plan->words, plan->cell_of, recall, st),
            "audit recall");
  }
  emc::mean2_kernel<<<1, 256, 0, st>>>(recall, na, recall_mean);
  // M-step rows: the audited frames' dense product first, then every group's candidate sum
  float* Wp = (float*)slices;  // hi/lo are no longer needed
  if (na > 0) {
    const char* KTa = (const char*)K_audit + (size_t)na * ps * 2;
    HIP_TRY(launch_gemm_bf16_nt(Pa, KTa, Wp, pb->n_rot, ps, dsa, dsa, dsa, ps, st), "audit mstep gemm");
  }
  CHECK(mark(4));
  HIP_TRY(launch_cand_mstep(groups, plan->grp_off, plan->n_groups, plan->cf_ptr, plan->cf_frame,
                            plan->runs, nc, plan->chunks, plan->dense_band, Pc, plan->pack_rot, ps,
                            Wp, rho, rho_a, na > 0, st),
          "candidate mstep");
  CHECK(mark(5));
  if (Pd && nc > 0) {  // dense bands: W'[:, centre] += P_dense K_centre^T over all candidate frames
    const int64_t nd = (int64_t)plan->n_dense * kBandPx;
    const int splits = dense_splits(pb, plan);  // few output tiles, long reduction: split it
    HIP_TRY(launch_gemm_bf16_nt_split(Pd, plan->kt_dense, Wd, pb->n_rot, nd, plan->ld_dense, plan->ld_dense,
                                      plan->ld_dense, nd, splits, st),
            "dense mstep gemm");
    HIP_TRY(launch_dense_add(Wd, splits, pb->n_rot, plan->n_dense, plan->dense_list, ps, Wp, st), "dense add");
  }
  CHECK(mark(6));
  if (!accumulate) {
    HIP_TRY(launch_fill_zero_f64(num, (size_t)pb->grid_n * pb->grid_n * pb->grid_n, st), "zero num");
    HIP_TRY(launch_fill_zero_f64(den, (size_t)pb->grid_n * pb->grid_n * pb->grid_n, st), "zero den");
  }
  // a chunk the audit rejects adds exact zeros: its W' rows and rho are cleared on the device
  if (gated) HIP_TRY(launch_gate_zero(recall_mean, recall_min, Wp, (int64_t)pb->n_rot * ps, rho, pb->n_rot, st), "gate");
  CHECK(run_scatter(pb, Wp, ps, rho, num, den, (double*)(w + W.copies), st));
  return EMC_OK;
}

emc_status check_proposed_call(const emc_problem* pb, const emc_proposal* plan, const void* K_audit,
                               const float* model_in, const double* recall_mean, const void* ws, size_t ws_bytes) {
  CHECK(check_problem(pb, true));
  if (!is_bf16(pb)) return fail(EMC_ERR_UNSUPPORTED, "the proposal form runs in BF16 precision");
  CHECK(check_plan(pb, plan));
  if (plan->n_audit > 0) CHECK(need(K_audit, 16, "K_audit"));
  CHECK(need(model_in, 4, "model_in"));
  CHECK(need(recall_mean, 8, "recall_mean"));
  const PropWs W = prop_ws(pb, plan);
  if (!ws || !aligned(ws, 256)) return fail(EMC_ERR_WORKSPACE, "workspace is NULL or not 256-byte aligned");
  if (ws_bytes < W.total) return fail(EMC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, W.total);
  return EMC_OK;
}

}  // namespace

extern "C" {

emc_status emc_proposed_accumulate(const emc_problem* pb, const emc_proposal* plan, const void* K_audit,
                                   const float* model_in, double* num, double* den, int32_t accumulate,
                                   double recall_min, double* L, double* recall_mean, void* ws, size_t ws_bytes,
                                   hipEvent_t* stage_events, hipStream_t st) {
  CHECK(check_proposed_call(pb, plan, K_audit, model_in, recall_mean, ws, ws_bytes));
  CHECK(need(num, 8, "num"));
  CHECK(need(den, 8, "den"));
  CHECK(need(L, 8, "L"));
  if (std::isnan(recall_min)) return fail(EMC_ERR_INVALID_ARG, "recall_min is NaN");
  CHECK(run_proposed(pb, plan, K_audit, model_in, num, den, accumulate, true, recall_min, L, recall_mean, (char*)ws,
                     stage_events, st));
  if (stage_events) HIP_TRY(hipEventRecord(stage_events[EMC_PROPOSED_STAGES], st), "stage event");
  return EMC_OK;
}

emc_status emc_proposed_workspace_view(const emc_problem* pb, const emc_proposal* plan, emc_proposed_view* view) {
  CHECK(check_problem(pb, false));
  CHECK(check_plan(pb, plan));
  if (!view) return fail(EMC_ERR_INVALID_ARG, "view is NULL");
  const PropWs W = prop_ws(pb, plan);
  view->G = (int64_t)W.G;
  view->P = (int64_t)W.P;
  view->b = (int64_t)W.b;
  view->L = (int64_t)W.L;
  view->S = (int64_t)W.S;
  view->Ga = (int64_t)W.Ga;
  view->Pa = (int64_t)W.Pa;
  return EMC_OK;
}

emc_status emc_iterate_proposed(const emc_problem* pb, const emc_proposal* plan, const void* K_audit,
                                const float* model_in, float* model_out, double* loglik, double* recall_mean,
                                void* ws, size_t ws_bytes, hipEvent_t* stage_events, hipStream_t st) {
  CHECK(check_proposed_call(pb, plan, K_audit, model_in, recall_mean, ws, ws_bytes));
  CHECK(need(model_out, 4, "model_out"));
  CHECK(need(loglik, 8, "loglik"));
  const PropWs W = prop_ws(pb, plan);
  char* w = (char*)ws;
  double* L = (double*)(w + W.L);
  double* num = (double*)(w + W.num);
  double* den = (double*)(w + W.den);
  CHECK(run_proposed(pb, plan, K_audit, model_in, num, den, 0, false, 0.0, L, recall_mean, w, stage_events, st));
  CHECK(run_finalize(pb, num, den, model_in, model_out, L, (int64_t)plan->n_cand + plan->n_audit, loglik, st));
  if (stage_events) HIP_TRY(hipEventRecord(stage_events[EMC_PROPOSED_STAGES], st), "stage event");
  return EMC_OK;
}

}  // extern "C"
