/*
 * Plain FP64 C versions of two oracle steps whose numpy forms cannot hold a
 * full-size problem in memory: the expansion of eq. (2.9) and the c-step sums
 * of eq. (2.12).  Same definitions, conventions and argument meanings as
 * oracle/emc_oracle.py (expand, compress): trilinear tent weights
 * f(d) = prod_a max(0, 1 - |d_a|) over the 8 grid points around R_j q_i + N/2,
 * grid points outside the N^3 box do not exist, flat index (x N + y) N + z,
 * quaternions (w, x, y, z) Hamilton, active, normalised first.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or load
 * this file's library; it shares no code with the GPU path.
 *
 * parity pinned: tests/test_oracle_c_pins.py (brute-force dense interpolation
 * matrix over every grid point with scipy's rotation, multilinear fields,
 * partition of unity, agreement with the numpy oracle on a tiny problem).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Section 2.2: rotation R_j of unit quaternion (w, x, y, z), row-major. */
static void rotation(const double* quat, double R[9]) {
  double w = quat[0], x = quat[1], y = quat[2], z = quat[3];
  const double n = sqrt(w * w + x * x + y * y + z * z);
  w /= n, x /= n, y /= n, z /= n;
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

/* The 8 grid points around p and their weights f(p_l - p); points outside the
 * box get weight 0 and index 0. */
static void stencil(const double p[3], int N, long idx[8], double wt[8]) {
  const double b0 = floor(p[0]), b1 = floor(p[1]), b2 = floor(p[2]);
  int t = 0;
  for (int dx = 0; dx < 2; ++dx)
    for (int dy = 0; dy < 2; ++dy)
      for (int dz = 0; dz < 2; ++dz, ++t) {
        const double v0 = b0 + dx, v1 = b1 + dy, v2 = b2 + dz;
        const int inside = v0 >= 0 && v0 < N && v1 >= 0 && v1 < N && v2 >= 0 && v2 < N;
        const double w = fmax(0.0, 1.0 - fabs(v0 - p[0])) * fmax(0.0, 1.0 - fabs(v1 - p[1])) *
                         fmax(0.0, 1.0 - fabs(v2 - p[2]));
        idx[t] = inside ? ((long)v0 * N + (long)v1) * N + (long)v2 : 0;
        wt[t] = inside ? w : 0.0;
      }
}

static void position(const double R[9], const double* q, int N, double p[3]) {
  for (int a = 0; a < 3; ++a) p[a] = R[3 * a] * q[0] + R[3 * a + 1] * q[1] + R[3 * a + 2] * q[2] + N / 2.0;
}

/* eq. (2.9): W[j][i] = sum_l f(p_l - R_j q_i) model_l for every pixel i. */
void orc_expand(const double* model, int N, const double* q, long n_pix, const double* quat, long n_rot,
                double* W) {
#pragma omp parallel for schedule(dynamic, 16)
  for (long j = 0; j < n_rot; ++j) {
    double R[9];
    rotation(quat + 4 * j, R);
    for (long i = 0; i < n_pix; ++i) {
      double p[3], wt[8];
      long idx[8];
      position(R, q + 3 * i, N, p);
      stencil(p, N, idx, wt);
      double s = 0.0;
      for (int t = 0; t < 8; ++t) s += wt[t] * model[idx[t]];
      W[j * n_pix + i] = s;
    }
  }
}

/* eq. (2.12): num_l = sum_{j, i valid} f(p_l - R_j q_i) Wp[j][i],
 *             den_l = sum_{j, i valid} f(p_l - R_j q_i) rho[j].
 * Each thread sums its share of rotations into its own grids; the grids are
 * then added in thread order. */
void orc_compress(const double* Wp, const double* rho, const double* q, const unsigned char* mask, long n_pix,
                  const double* quat, long n_rot, int N, double* num, double* den) {
  const long M = (long)N * N * N;
  memset(num, 0, M * sizeof(double));
  memset(den, 0, M * sizeof(double));
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  double* part = (double*)calloc((size_t)nt * 2 * M, sizeof(double));
#pragma omp parallel num_threads(nt)
  {
    int me = 0;
#ifdef _OPENMP
    me = omp_get_thread_num();
#endif
    double* pn = part + (size_t)me * 2 * M;
    double* pd = pn + M;
#pragma omp for schedule(static)
    for (long j = 0; j < n_rot; ++j) {
      double R[9];
      rotation(quat + 4 * j, R);
      for (long i = 0; i < n_pix; ++i) {
        if (!mask[i]) continue;
        double p[3], wt[8];
        long idx[8];
        position(R, q + 3 * i, N, p);
        stencil(p, N, idx, wt);
        for (int t = 0; t < 8; ++t) {
          pn[idx[t]] += wt[t] * Wp[j * n_pix + i];
          pd[idx[t]] += wt[t] * rho[j];
        }
      }
    }
  }
  for (int t = 0; t < nt; ++t)
    for (long l = 0; l < M; ++l) {
      num[l] += part[(size_t)t * 2 * M + l];
      den[l] += part[(size_t)t * 2 * M + M + l];
    }
  free(part);
}
