/*
 * emc.h -- C ABI of a gfx950 (MI355X) implementation of one Expand-Maximize-
 * Compress (EMC) iteration for assembling a 3D Fourier intensity from randomly
 * oriented 2D diffraction frames, Poisson noise model, covering one GPU's share
 * of the rotation set.
 *
 * The method is that of Ekeberg, Engblom & Liu, "Machine learning for
 * ultrafast X-ray diffraction patterns on large-scale GPU clusters"
 * (arXiv:1409.4256): expansion eq. (2.9), E-step eq. (2.4), combined M- and
 * c-step eq. (2.11)-(2.12), Algorithm 1.  The likelihood is the Poissonian one
 * the paper names in Section 2.2 (eq. (2.5)/(2.11) with fluence phi = 1):
 *     Q_jk = sum_{i valid} K_ik log W_ij - W_ij        (log K_ik! dropped).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is DEVICE memory owned by the caller.  The library
 *    never allocates; emc_iterate takes a caller workspace sized by
 *    emc_workspace_bytes (emc_iterate_noalloc uses a static device buffer of
 *    the library's own instead).  All work is enqueued asynchronously on `stream`
 *    (no host synchronisation, except emc_pack_frames in BF16 form, which
 *    reads back its range flag).
 *  - Arguments are validated on the host before anything is launched: on a
 *    negative status nothing has been launched or written (except
 *    EMC_ERR_RANGE, see emc_pack_frames), and emc_last_error() returns a
 *    message (thread-local).  A failed launch maps to EMC_ERR_HIP.  Array
 *    contents are not validated: any finite input has a defined result
 *    (non-unit quaternions are normalised, grid points outside the N^3 box
 *    contribute nothing).
 *  - Model grid: N^3 float values, flat index l = (x*N + y)*N + z of grid
 *    point p_l = (x, y, z); pixel coordinate q_i (voxel units) is placed at
 *    R_j q_i + (N/2, N/2, N/2).  Interpolation weights f (eq. (2.8)) are the
 *    trilinear tent f(d) = prod_a max(0, 1 - |d_a|), in expansion and
 *    compression alike.
 *  - Rotations: quaternions (w, x, y, z), Hamilton convention, active.
 *  - Padded row lengths: ps = emc_pix_stride(n_pix), ds = emc_data_stride(n_data)
 *    (multiples of 256).  Padding entries are written as zeros unless stated.
 *  - Rotation-major storage of everything indexed (j, k): G[j][k], P[j][k]
 *    with row length ds, frames contiguous.
 *  - Slices are floored at 1e-10 photons before the log and the sum; masked
 *    pixels (mask == 0) are excluded from every sum.
 *  - The pixel list may be in any order (apply the same permutation to q,
 *    mask and the counts' columns); compression is fastest when each run of
 *    64 consecutive pixels is spatially compact on the detector (8 x 8 tiles).
 *  - Precision: EMC_PREC_FP32 runs both contractions in FP32 MFMA;
 *    EMC_PREC_BF16 runs them in BF16 MFMA with FP32 accumulation (counts exact,
 *    slices split hi + lo with a per-rotation scale, responsibilities rounded
 *    to BF16).  Both keep FP64 for S_j, b_k, the log-sum-exp, rho and the grid
 *    accumulation.
 *
 * Thread safety: entry points are reentrant; calls that share output or
 * workspace buffers must be ordered by the caller (same stream or events).
 */
#ifndef EMC_H
#define EMC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EMC_OK = 0,
  EMC_ERR_INVALID_ARG = -1, /* bad size, null or misaligned pointer, bad enum */
  EMC_ERR_RANGE = -2,       /* a photon count does not fit the packed type   */
  EMC_ERR_WORKSPACE = -3,   /* workspace missing or smaller than required    */
  EMC_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed    */
  EMC_ERR_UNSUPPORTED = -5  /* valid request this build does not implement   */
} emc_status;

typedef enum {
  EMC_PREC_FP32 = 0, /* FP32 operands, FP32 MFMA                            */
  EMC_PREC_BF16 = 1  /* BF16 operands (slices as hi + lo), BF16 MFMA, FP32 acc */
} emc_precision;

typedef enum {
  EMC_RESP_FULL = 0,     /* per-frame statistics, then P, L and rho             */
  EMC_RESP_PARTIAL = 1,  /* only the per-frame (max, sum) statistics            */
  EMC_RESP_FINALIZE = 2  /* P, L and rho from caller-supplied global statistics */
} emc_resp_mode;

struct emc_scatter_plan;

/* Problem description (Section 2.2 notation). */
typedef struct emc_problem {
  int32_t grid_n;          /* N: model has N^3 grid points, 2 <= N <= 1024              */
  int32_t n_pix;           /* Mpix: detector pixels, >= 1                               */
  int32_t n_rot;           /* Mrot of this share: rotations, >= 1                       */
  int32_t n_data;          /* Mdata of this call: frames, >= 0                          */
  int32_t precision;       /* emc_precision                                             */
  int32_t reserved;        /* must be 0                                                 */
  const float* q;          /* [n_pix][3] pixel scattering vectors q_i, voxel units      */
  const uint8_t* mask;     /* [n_pix] 1 = pixel used, 0 = missing or saturated          */
  const float* quat;       /* [n_rot][4] rotation R_j as quaternion (w, x, y, z)        */
  const double* log_w;     /* [n_rot] log prior weight log w_j (sum_j w_j = 1 over the  */
                           /*         full rotation set, Section 2.2)                   */
  const struct emc_scatter_plan* scatter;  /* host struct; NULL = rotation-major c-step, */
                           /*         else the brick-major one this plan describes      */
                           /*         (emc_scatter_plan_build, same q, mask, quat, N)   */
} emc_problem;

/* Library version string (static storage). */
const char* emc_version(void);

/* Message describing the last non-OK status returned on this thread. */
const char* emc_last_error(void);

/* ps: n_pix rounded up to a multiple of 256 (0 if n_pix < 1). */
int64_t emc_pix_stride(int32_t n_pix);

/* ds: n_data rounded up to a multiple of 256 (0 if n_data < 1). */
int64_t emc_data_stride(int32_t n_data);

/* Bytes of the packed frames (emc_pack_frames output) for this problem. */
emc_status emc_frames_bytes(const emc_problem* pb, size_t* bytes);

/* Bytes of the slice buffer (emc_expand output, also the W' buffer). */
emc_status emc_slices_bytes(const emc_problem* pb, size_t* bytes);

/* Bytes of workspace emc_iterate needs for this problem (written to *bytes). */
emc_status emc_workspace_bytes(const emc_problem* pb, size_t* bytes);

/* Frames K_ik (Section 2.1: photon counts of frame k) -> GEMM operands.
 *   counts   [n_data][n_pix] uint16 photon counts
 *   K_packed emc_frames_bytes bytes, 16-byte aligned: K [n_data][ps] followed by
 *            KT [ps][ds] (element type float in FP32 form, bfloat16 in BF16
 *            form); masked and padding pixels and padding frames are 0.
 * BF16 form: counts above 256 are not exact in BF16 and give EMC_ERR_RANGE
 * (the call then synchronises the stream; K_packed holds rounded values). */
emc_status emc_pack_frames(const emc_problem* pb, const uint16_t* counts, void* K_packed,
                           hipStream_t stream);

/* emc_pack_frames under the name of the problem statement's "patterns". */
emc_status emc_pack_patterns(const emc_problem* pb, const uint16_t* counts, void* K_packed,
                             hipStream_t stream);

/* Contents check for callers that cannot vouch for their arrays (every other entry
 * point checks sizes and pointers only; any finite input has a defined result):
 *   - each quaternion's norm within 1e-5 of 1 (Section 2.2: unit quaternions);
 *   - finite log prior weights and finite coordinates of the used pixels;
 *   - when model is not NULL: every model value finite and >= 0 (an intensity).
 *   flags  device int32 the call overwrites (scratch, 4-byte aligned)
 * One pass over the arrays on `stream`, then one synchronisation to read the result.
 * Returns EMC_OK, or EMC_ERR_INVALID_ARG with emc_last_error() naming the first
 * failed check.  Nothing else is written. */
emc_status emc_validate(const emc_problem* pb, const float* model, int32_t* flags, hipStream_t stream);

/* Expansion, eq. (2.9): W_ij = sum_l f(p_l - R_j q_i) model_l, floored at
 * 1e-10, as centred logs A_ji = log W_ij - c_i.
 *   model  [N^3] float grid values
 *   c      [ps] double out: c_i = mean of log W_ij over a fixed subset of at most
 *          64 rotations (j = floor(t*n_rot/n_c)); 0 on masked/padding pixels.
 *          Any c leaves the E-step unchanged (a shift constant in j, added back
 *          through b_k); it keeps the reduced-precision sums small.
 *   slices emc_slices_bytes bytes out.  FP32: A [n_rot][ps] float.  BF16: hi
 *          [n_rot][ps] followed by lo [n_rot][ps], bfloat16, with
 *          A_ji ~ scale_j (hi_ji + lo_ji).  0 on masked/padding pixels.
 *   S      [n_rot] double out: S_j = sum_{i valid} W_ij
 *   scale  [n_rot] float out (BF16 form; may be NULL in FP32 form):
 *          scale_j = max_i |A_ji| (1 if the row is 0)                        */
emc_status emc_expand(const emc_problem* pb, const float* model, double* c, void* slices,
                      double* S, float* scale, hipStream_t stream);

/* Poisson log-likelihood, Section 2.2 / eq. (2.3), as a dense contraction over
 * pixels on the matrix cores:
 *   G [n_rot][ds] float out: G_jk = sum_i A_ji K_ik (padding frames untouched)
 *   b [n_data] double out:   b_k = sum_i K_ik c_i (FP64)
 * so that Q_jk = G_jk + b_k - S_j.  `scale` is read in BF16 form only.      */
emc_status emc_loglik(const emc_problem* pb, const void* K_packed, const void* slices,
                      const float* scale, const double* c, float* G, double* b,
                      hipStream_t stream);

/* E-step, eq. (2.4), as an FP64 log-sum-exp over rotations of the log-joint
 * a_jk = Q_jk + log w_j = G_jk + b_k - S_j + log w_j:
 *   stats [n_data][2] double: (m_k, s_k) with m_k = max_j a_jk and
 *         s_k = sum_j exp(a_jk - m_k).  Written in FULL and PARTIAL mode; read
 *         in FINALIZE mode, where the caller has combined the statistics of
 *         several rotation shares (m = max_r m_r, s = sum_r s_r exp(m_r - m)),
 *         the exchange Section 3.2 describes.
 *   P     [n_rot][ds] out (FULL, FINALIZE): P_jk = exp(a_jk - m_k - log s_k);
 *         float in FP32 form (may alias G), bfloat16 in BF16 form (must not
 *         alias G); padding frames written 0.
 *   L     [n_data] double out (FULL, FINALIZE): log-evidence
 *         L_k = m_k + log s_k (eq. (2.1) objective term, without log K!).
 *   rho   [n_rot] double out (FULL, FINALIZE): rho_j = sum_k P_jk of the stored
 *         (rounded) P values.
 *   b     [n_data] double: b_k from emc_loglik (all modes).
 * In PARTIAL mode P, L, rho may be NULL.                                     */
emc_status emc_responsibilities(const emc_problem* pb, const float* G, const double* S,
                                const double* b, int32_t mode, double* stats, void* P,
                                double* L, double* rho, hipStream_t stream);

/* Combined M- and c-step, eq. (2.11)-(2.12) with phi = 1, without the final
 * division:
 *   Wp  [n_rot][ps] float out: W'_ji = sum_k P_jk K_ik (matrix cores); may
 *       alias the slices of emc_expand (no longer needed by then)
 *   num, den [N^3] double: num_l += sum_{j,i valid} f(p_l - R_j q_i) W'_ji,
 *       den_l += sum_{j,i valid} f(p_l - R_j q_i) rho_j (FP64).
 *       accumulate == 0 zeroes them first; accumulate != 0 adds, so frame
 *       chunks (the k-direction split of Section 3.3) sum before division.
 *   ws  NULL, or emc_compress_workspace_bytes of device memory: one copy of
 *       the two grids per XCD, whose atomics stay in that XCD's L2 (faster);
 *       without it the atomics go to num/den directly.  With pb->scatter set
 *       the c-step is brick-major, needs no workspace (0 bytes) and ignores ws. */
emc_status emc_compress_workspace_bytes(const emc_problem* pb, size_t* bytes);
emc_status emc_compress(const emc_problem* pb, const void* P, const void* K_packed,
                        const double* rho, float* Wp, double* num, double* den,
                        int32_t accumulate, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Brick-major c-step (eq. (2.12), the same sums as the rotation-major
 * scatter with the loop nest turned round).  The grid is cut into bricks of
 * 16^3 voxels; a visit is a pair (rotation j, group t of the 64 pixels
 * 64t .. 64t+63) listed under every brick that a trilinear corner of a used
 * pixel of the group reaches under R_j.  Visits are grouped by brick and cut
 * into work items of at most `chunk` visits; one workgroup per item sums its
 * brick in LDS (FP64) and adds it to num/den with one atomic per voxel.  The
 * plan depends only on grid_n, n_pix, n_rot, q, mask and quat, so one build
 * serves every iteration; point pb->scatter at it and emc_compress,
 * emc_iterate and emc_iterate_proposed run their c-step this way (and need
 * no grid copies in their workspaces).  Results equal the rotation-major
 * c-step's up to the order of the FP64 additions.
 * ------------------------------------------------------------------------ */
typedef struct emc_scatter_plan {
  int32_t grid_n, n_pix, n_rot;  /* geometry the plan was built for                  */
  int32_t brick;                 /* brick edge in voxels (16)                        */
  int32_t n_bricks;              /* ceil(N / brick)^3                                */
  int32_t n_groups;              /* ceil(n_pix / 64) pixel groups                    */
  int32_t chunk;                 /* most visits per work item                        */
  int32_t reserved;
  int64_t n_visits;              /* (j, t, brick) visits                             */
  int64_t n_items;               /* work items                                       */
  int64_t bytes;                 /* bytes of buf the plan uses or, after             */
                                 /* EMC_ERR_WORKSPACE, needs                         */
  const int32_t* visits;         /* [n_visits] j * n_groups + t, grouped by brick    */
  const int32_t* items;          /* [n_items][4] (brick, first visit, end, 0)        */
  const double* rot;             /* [n_rot][9] R_j row-major (FP64)                  */
  const float* q;                /* geometry pointers the plan was built from        */
  const uint8_t* mask;
  const float* quat;
} emc_scatter_plan;

/* Bytes of buf emc_scatter_plan_build needs before it knows the visit count
 * (the per-brick counters and offsets, the rotation table). */
emc_status emc_scatter_plan_min_bytes(const emc_problem* pb, size_t* bytes);

/* Build the plan for pb's geometry into buf (device memory, 256-byte aligned,
 * buf_bytes >= emc_scatter_plan_min_bytes); the plan's arrays point into buf,
 * which must outlive every call that uses the plan.
 *   chunk  visits per work item, 0 for the default (2048), else 64 .. 2^20.
 * Counts the visits on the device and reads the per-brick counts back (one
 * synchronisation of `stream`); the listing itself is enqueued on `stream`,
 * so later calls on other streams must wait for it.  When buf_bytes is too
 * small, returns EMC_ERR_WORKSPACE with plan->bytes set to the bytes needed
 * and nothing else filled.  EMC_ERR_UNSUPPORTED when n_rot * n_groups or the
 * visit count exceeds 2^31 - 1. */
emc_status emc_scatter_plan_build(const emc_problem* pb, int32_t chunk, void* buf, size_t buf_bytes,
                                  emc_scatter_plan* plan, hipStream_t stream);

/* Final division of eq. (2.12) and the mean log-evidence of eq. (2.1):
 *   model_out_l = num_l / den_l where den_l > 0, else model_prev_l
 *   loglik (device scalar) = sum_k L_k / n_L  (NaN when n_L == 0)
 * Uses pb->grid_n only.  model_out may alias model_prev.                    */
emc_status emc_finalize(const emc_problem* pb, const double* num, const double* den,
                        const float* model_prev, float* model_out, const double* L,
                        int64_t n_L, double* loglik, hipStream_t stream);

/* One full iteration of Algorithm 1 over this problem's frames:
 * expand -> log-likelihood -> E-step -> M/c-step -> division.
 *   model_in  [N^3] float;  model_out [N^3] float (may alias model_in)
 *   K_packed  output of emc_pack_frames (same precision)
 *   loglik    device double scalar: mean log-evidence (see emc_finalize)
 *   P_out     optional [n_rot][ds] responsibilities (float in FP32 form,
 *             bfloat16 in BF16 form); NULL keeps them in the workspace
 *   ws        workspace of at least emc_workspace_bytes bytes, 256-byte aligned */
emc_status emc_iterate(const emc_problem* pb, const float* model_in, const void* K_packed,
                       float* model_out, double* loglik, void* P_out, void* ws,
                       size_t ws_bytes, hipStream_t stream);

/* Allocation-free emc_iterate, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as emc_iterate, without ws:
 * the workspace is the library's own static device buffer of
 * EMC_SCRATCH_MAX_BYTES, one per GPU, held from the library's load until the
 * process ends.  Its address on the current device is looked up on the first
 * call made with that device current.  The call allocates and frees nothing.
 *  - Problems whose emc_workspace_bytes exceeds EMC_SCRATCH_MAX_BYTES are
 *    refused with EMC_ERR_WORKSPACE before anything is launched.
 *  - Every call on one GPU uses that GPU's single buffer: calls that overlap
 *    on one GPU (concurrent streams, threads) race and must be serialised by
 *    the caller.  Nothing in the buffer carries over between calls (every sum
 *    the iteration needs zeroed is cleared by its own kernels first).
 * Rotation-major c-step grid copies count towards the workspace; a brick-major
 * plan (pb->scatter) keeps them out. */
#define EMC_SCRATCH_MAX_BYTES ((size_t)64 << 20)
emc_status emc_iterate_noalloc(const emc_problem* pb, const float* model_in, const void* K_packed,
                               float* model_out, double* loglik, void* P_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Gaussian noise model with photon fluence (Section 2.2, the paper's own
 * likelihood), FP32 form:
 *   Q_jk = -sum_{i valid} (K_ik / phi_jk - W_ij)^2 / (2 sigma^2)     eq. (2.2)-(2.3)
 *   P_jk = w_j e^{Q_jk} / sum_j' w_j' e^{Q_j'k}                       eq. (2.4)
 *   W'_ji = sum_k P_jk K_ik / phi_jk,  rho_j = sum_k P_jk              eq. (2.11)
 *   num/den and the division as in the Poisson form                   eq. (2.12)
 *   phi'_jk = sum_i K_ik^2 / sum_i W_ij K_ik  (1 when that sum is 0)  eq. (2.6)
 * One iteration uses the fluence phi^(n) in its E-step and M-step and returns
 * phi^(n+1), the update evaluated on its own slices W^(n).
 *   sigma          noise parameter, > 0 and finite
 *   phi            [n_rot][ds] float, in/out: phi^(n) in (unless
 *                  phi_from_model != 0), phi^(n+1) out; padding frames get 1
 *   phi_from_model nonzero: phi^(n) is the update of this iteration's own
 *                  slices (the first iteration has no previous fluence)
 *   K_packed       emc_pack_frames output of an FP32 problem
 *   loglik         device double: mean over frames of log sum_j w_j e^{Q_jk}
 *   P_out          optional [n_rot][ds] float responsibilities
 *   ws             emc_gaussian_workspace_bytes bytes, 256-byte aligned
 * EMC_ERR_UNSUPPORTED for the BF16 form.  The c-step is brick-major when
 * pb->scatter is set.
 * ------------------------------------------------------------------------ */
emc_status emc_gaussian_workspace_bytes(const emc_problem* pb, size_t* bytes);
emc_status emc_iterate_gaussian(const emc_problem* pb, double sigma, const float* model_in,
                                const void* K_packed, float* phi, int32_t phi_from_model,
                                float* model_out, double* loglik, float* P_out, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned orientation proposal.  A small CNN scores the cells of a coarse
 * rotation grid from a frame; its top-K cells restrict the E-step's search
 * (the full search stays the fallback and the measure of recall).  This is an
 * addition to the paper's method; its training targets are the E-step
 * responsibilities of eq. (2.4) summed over each cell's fine rotations.
 * Network: x = log(1 + binned frame) 1x64x64 -> 4 x [conv 3x3 stride 2 pad 1
 * + bias + ReLU] (1->32->64->128->128) -> flatten 2048 -> linear -> n_cells
 * logits.  Parameters are one float array (emc_cnn_param_count floats):
 * for l = 0..3: w_l [co][ci][3][3], b_l [co]; then wf [n_cells][2048], bf
 * [n_cells].  Activations and images are NCHW float.
 * ------------------------------------------------------------------------ */

int64_t emc_cnn_param_count(int32_t n_cells);

/* Workspace bytes for emc_cnn_forward / emc_cnn_gradients at batch <= max_batch. */
emc_status emc_cnn_workspace_bytes(int32_t n_cells, int32_t max_batch, size_t* bytes);

/* Network input of B frames: x[b] = log1p(per-bin photon sums), 64x64.
 *   K_packed  frames packed by emc_pack_frames (frame-major part is read)
 *   bins      [n_pix] int32 bin of each pixel in [0, 4096), or -1 (ignored)
 *   frames    [B] int32 frame indices, or NULL for frames 0..B-1
 *   x         [B][64][64] float out                                         */
emc_status emc_cnn_preprocess(const emc_problem* pb, const void* K_packed, const int32_t* bins,
                              const int32_t* frames, int32_t B, float* x, hipStream_t stream);

/* logits [B][n_cells] float out. */
emc_status emc_cnn_forward(int32_t n_cells, const float* params, const float* x, int32_t B,
                           float* logits, void* ws, size_t ws_bytes, hipStream_t stream);

/* Soft-target cross entropy loss = -(1/B) sum_b sum_c T[b][c] log softmax(z_b)_c
 * (device double, overwritten) and its gradient with respect to every
 * parameter (grads, same layout as params, overwritten).  T [B][n_cells]. */
emc_status emc_cnn_gradients(int32_t n_cells, const float* params, const float* x, const float* T,
                             int32_t B, float* grads, double* loss, void* ws, size_t ws_bytes,
                             hipStream_t stream);

/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments)
 * of params with grads; m, v moments (zero before step 1); step >= 1.      */
emc_status emc_cnn_adam(int32_t n_cells, float* params, const float* grads, float* m, float* v,
                        int32_t step, float lr, hipStream_t stream);

/* out [rows][k] int32: indices of the k largest logits of each row, largest
 * first, ties to the lower index (k <= n_cells <= 8192).                    */
emc_status emc_cnn_topk(const float* logits, int64_t rows, int32_t n_cells, int32_t k,
                        int32_t* out, hipStream_t stream);

/* out [rows][k] int32: the k cells of largest positive mass of each row of T
 * [rows][n_cells] (largest first, ties to the lower index); a row with fewer
 * positive cells is padded with -1.  Used on emc_cell_targets output to
 * propose the cells that held a frame's responsibility in a full iteration.   */
emc_status emc_cell_topk(const float* T, int64_t rows, int32_t n_cells, int32_t k, int32_t* out,
                         hipStream_t stream);

/* out [rows][ka + kb] int32: per row, the valid cells (0 <= c < n_cells) of
 * a [rows][ka] in order, then those of b [rows][kb] not already present,
 * then -1 padding; repeated cells are kept once (ka + kb <= 512).            */
emc_status emc_topk_union(const int32_t* a, int32_t ka, const int32_t* b, int32_t kb, int64_t rows,
                          int32_t n_cells, int32_t* out, hipStream_t stream);

/* Training targets: T [n_data][n_cells] float out, T[k][c] = sum of P[j][k]
 * over the fine rotations j of cell c, listed as CSR (cell_ptr [n_cells+1],
 * cell_rot [n_rot]); P as written by emc_responsibilities (precision of pb). */
emc_status emc_cell_targets(const emc_problem* pb, const void* P, const int32_t* cell_ptr,
                            const int32_t* cell_rot, int32_t n_cells, float* T, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned-proposal iteration (BF16 form).  Each frame's E-step (eq. 2.4) runs
 * over the fine rotations of its proposed coarse cells only; a seeded subset
 * of frames is searched in full and judges the proposal's recall, the
 * fraction of their full-search responsibility inside their proposed cells.
 * The caller reruns the iteration with emc_iterate when the mean recall is
 * below its threshold.  Log-likelihoods, responsibilities and the M-step
 * (eq. 2.11) of the candidate pairs are exact over those pairs (BF16
 * arithmetic as in emc_iterate); nothing is dropped below a threshold.
 * ------------------------------------------------------------------------ */

/* Packed frames of a frame list: like emc_pack_frames with pb->n_data =
 * number of listed frames and row k taken from counts row frames[k]. */
emc_status emc_pack_frames_list(const emc_problem* pb, const uint16_t* counts, const int32_t* frames,
                                void* K_packed, hipStream_t stream);

/* Proposal plan: arrays carved from one caller buffer by emc_proposal_build.
 * Frames are split into audited ones and candidate ones (grouped by the pack of
 * their first proposed cell).  Neighbouring coarse cells are gathered into
 * packs of at most 16 fine rotations in all, one 16-row MFMA tile (nearest
 * neighbours first; a cell with more rotations is a pack of its own); a pack is searched over the union
 * of its cells' frame lists, and only the pairs whose cell the frame proposes
 * enter the E-step.  A pack's rotations are split into groups of at most 32;
 * a group's storage in G and P is Fp x 32 elements, Fp = the pack's frame list
 * length rounded up to 32.  All pointers are device pointers into the plan
 * buffer.                                                                      */
typedef struct emc_proposal {
  int32_t n_cells;        /* coarse cells                                           */
  int32_t k_top;          /* entries of each frame's proposal list (<= 256)         */
  int32_t n_cand;         /* frames searched over their candidates                  */
  int32_t n_audit;        /* frames searched in full                                */
  int32_t words;          /* ceil(n_cells / 32): words of a cell bitmask            */
  int32_t n_bands;        /* 128-pixel bands: n_pix stride / 128                     */
  int64_t n_groups;       /* rotation groups                                        */
  int64_t n_tiles;        /* workgroups of the candidate log-likelihood (x 8)       */
  int64_t n_g;            /* elements of G (float) and P (bf16)                     */
  int64_t n_chunks;       /* 16-byte chunks of the candidate frames' band format    */
  int32_t* cell_of;       /* [n_rot] coarse cell of each rotation (max |<q, q_c>|)  */
  int64_t* cell_ptr;      /* [n_cells + 1] rotations of cell c: cell_rot[ptr[c]..)  */
  int32_t* cell_rot;      /* [n_rot]                                                */
  int32_t* pack_of;       /* [n_cells] pack of each cell                            */
  int32_t* cell_first;    /* [n_cells] position of cell c's first rotation in
                             pack_rot (its count: cell_ptr[c + 1] - cell_ptr[c])   */
  int32_t* pack_rot;      /* [n_rot] rotations in pack order, cell by cell          */
  int32_t* rot_local;     /* [n_rot] index inside its pack of the cell of
                             pack_rot[t] (< 32)                                     */
  int32_t* cand_frames;   /* [n_cand] frame index, grouped by the pack of the
                             frame's first proposed cell                           */
  int32_t* audit_frames;  /* [n_audit] frame index of the audited frames            */
  int32_t* cand_cells;    /* [n_cand][k_top] proposed cells (-1: none)              */
  int32_t* pair_col;      /* [n_cand][k_top] position of the frame in the list of
                             its cell's pack                                        */
  int64_t* cf_ptr;        /* [n_cells + 1] frame list of pack p: cf_frame[ptr[p]..)
                             (packs n_packs.. are empty)                            */
  int32_t* cf_frame;      /* [n_cand * k_top] candidate-frame index                 */
  uint32_t* cf_mask;      /* [n_cand * k_top] per pack-list entry: bit i set when
                             the frame proposes the pack's i-th cell               */
  int64_t* cg_ptr;        /* [n_cells + 1] groups of pack p: [cg_ptr[p], cg_ptr[p+1]) */
  void* groups;           /* [n_groups] int32 x 4: pack, first pack_rot entry, count, 0 */
  int64_t* grp_off;       /* [n_groups + 1] element offset of each group's storage   */
  void* tiles;            /* [n_tiles] int32 x 2: group, first frame; (-1, 0) padding */
  uint32_t* mask_audit;   /* [n_audit][words] proposed cells of the audited frames  */
  void* chunks;           /* 16-byte chunks of 8 uint16 words: the non-zero pixels
                             of candidate frame f in 128-pixel band b as
                             (pixel - 128 b) << 9 | count, ascending, 0xffff pads;
                             bands in runs of 8 (r = b / 8): run 0 of every frame,
                             then run 1, ...; inside a run frame f's chunks of its
                             bands are contiguous, band after band                 */
  void* runs;             /* [n_cand][ceil(n_bands / 8)] uint32 x 4 per (frame, run):
                             first chunk (absolute index); the offsets of bands
                             0-3 and of bands 4-7 from it, one byte each, lowest
                             byte first (a band past n_bands: the run's count);
                             the run's chunk count; followed by the same records
                             run-major, [ceil(n_bands / 8)][n_cand]                */
  int32_t n_dense;        /* dense bands (frames average >= 3 chunks; <= 16): their
                             M-step columns are one dense product                  */
  int32_t n_packs;        /* packs of cells                                         */
  int64_t ld_dense;       /* n_cand rounded up to 256                               */
  int32_t* dense_band;    /* [n_bands] index among the dense bands, or -1           */
  int32_t* dense_list;    /* [16] band of each dense index                          */
  void* kt_dense;         /* [n_dense * 128][ld_dense] BF16 pixel-major counts of the
                             dense bands' pixels over the candidate frames         */
  int32_t n_rot, n_pix;   /* problem the plan was built for: the iteration refuses a */
  const float* quat;      /* problem with other sizes, rotations or mask            */
  const uint8_t* mask;
} emc_proposal;

/* Bytes of the plan buffer; nz_cap bounds the non-zero pixels of the frames. */
emc_status emc_proposal_bytes(const emc_problem* pb, int32_t n_cells, int32_t k_top, int32_t n_audit,
                              int64_t nz_cap, size_t* bytes);

/* Builds the plan (synchronises the stream once).
 *   coarse [n_cells][4] float quaternions of the coarse grid
 *   topk   [n_data][k_top] int32 proposed cells of every frame, distinct, -1
 *          for no cell (emc_cnn_topk, emc_cell_topk, emc_topk_union)
 *   audit  [n_audit] int32 distinct frame indices searched in full
 *   counts [n_data][n_pix] uint16 photon counts (their non-zero unmasked pixels
 *          are listed for the candidate frames; n_pix <= 65536)
 * EMC_ERR_RANGE if a candidate frame holds a count above 256 (not exact in
 * BF16); EMC_ERR_WORKSPACE if the non-zero pixels exceed nz_cap.             */
emc_status emc_proposal_build(const emc_problem* pb, const float* coarse, int32_t n_cells,
                              const int32_t* topk, int32_t k_top, const int32_t* audit, int32_t n_audit,
                              const uint16_t* counts, int64_t nz_cap, void* buf, size_t buf_bytes,
                              emc_proposal* plan, hipStream_t stream);

/* Workspace bytes of emc_iterate_proposed. */
emc_status emc_proposed_workspace_bytes(const emc_problem* pb, const emc_proposal* plan, size_t* bytes);

/* Stages of emc_iterate_proposed, in order (stage_events[i], [i + 1] bracket stage i). */
#define EMC_PROPOSED_STAGES 7  /* expansion (with b); candidate log-likelihood; candidate
                                  E-step; audited frames (log-likelihood, E-step, recall,
                                  dense M-step product); candidate M-step (sparse bands);
                                  candidate M-step of the dense bands (one product);
                                  compression, division and mean log-evidence           */

/* One frame chunk of a learned-proposal iteration, without the division: the
 * k-direction split of Section 3.3 applied to the restricted iteration, so that
 * the frame chunks of one iteration, each with its own plan and audit, sum into
 * one numerator and denominator before emc_finalize divides them.
 * pb->precision must be EMC_PREC_BF16; pb->n_data = n_cand + n_audit.
 *   K_audit     frames plan->audit_frames packed by emc_pack_frames_list
 *   num, den    [N^3] double: accumulate == 0 zeroes them first.  The chunk's
 *               c-step sums (eq. 2.12) are then added when its audit accepts it
 *               (recall_mean >= recall_min, or no audited frames: recall NaN) and
 *               skipped otherwise, decided on the device without synchronising,
 *               so that the caller can add the chunk's full search instead
 *               (emc_loglik, emc_responsibilities, emc_compress with accumulate).
 *   L           [n_data] double out: log-evidence of each frame over its searched
 *               set, candidate frames in plan->cand_frames order, then audited
 *               frames in plan->audit_frames order
 *   recall_mean device double out: mean recall of the audited frames (NaN without)
 *   ws          emc_proposed_workspace_bytes bytes, 256-byte aligned
 *   stage_events NULL, or EMC_PROPOSED_STAGES + 1 events (see below); the last
 *               stage holds the c-step only                                      */
emc_status emc_proposed_accumulate(const emc_problem* pb, const emc_proposal* plan, const void* K_audit,
                                   const float* model_in, double* num, double* den, int32_t accumulate,
                                   double recall_min, double* L, double* recall_mean, void* ws, size_t ws_bytes,
                                   hipEvent_t* stage_events, hipStream_t stream);

/* Where the intermediate results of the last emc_iterate_proposed or
 * emc_proposed_accumulate call on a workspace lie in it (byte offsets), for
 * inspection; valid until the workspace is used again.
 *   G   float: candidate log-likelihood sums of eq. (2.3), group g's list position
 *       f and rotation slot r (rotation cell_rot[groups[g].first + r]) at element
 *       grp_off[g] + 32 f + r; Q = G + b_f - S_j
 *   P   bfloat16: responsibilities of eq. (2.4) over the candidate pairs, group g's
 *       storage at element grp_off[g] as blocks [Fp/32][32 rotations][32 frames]
 *   b   double [n_data]: b_f = sum_i K_if c_i (candidate frames, then audited ones)
 *   L   double [n_data]: log-evidence, same order (emc_iterate_proposed only)
 *   S   double [n_rot]: S_j = sum_i W_ij
 *   Ga  float [n_rot][round_up(n_audit, 256)]: audited frames' G (full search)
 *   Pa  bfloat16, same shape: audited frames' responsibilities                   */
typedef struct emc_proposed_view {
  int64_t G, P, b, L, S, Ga, Pa;
} emc_proposed_view;
emc_status emc_proposed_workspace_view(const emc_problem* pb, const emc_proposal* plan, emc_proposed_view* view);

/* One iteration with the E-step restricted to the proposal (pb->precision must
 * be EMC_PREC_BF16; pb->n_data = n_cand + n_audit): emc_proposed_accumulate
 * into workspace grids (accumulate 0, every chunk's sums added), then the
 * division and the mean log-evidence of emc_finalize.
 *   K_audit  frames plan->audit_frames packed by emc_pack_frames_list (the
 *            candidate frames are read from the plan's sparse band format)
 *   loglik   mean log-evidence over all frames (each over its searched set)
 *   recall_mean  mean recall of the audited frames (NaN without audit)
 *   stage_events NULL, or EMC_PROPOSED_STAGES + 1 events recorded on the
 *            stream at the stage boundaries (for timing; owned by the caller) */
emc_status emc_iterate_proposed(const emc_problem* pb, const emc_proposal* plan, const void* K_audit,
                                const float* model_in, float* model_out, double* loglik,
                                double* recall_mean, void* ws, size_t ws_bytes,
                                hipEvent_t* stage_events, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* EMC_H */
