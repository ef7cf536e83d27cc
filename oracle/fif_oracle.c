/*
 * FP64 CPU oracle for the Fisher Information Field (FIF) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * It is written for checking by eye against Zhang & Scaramuzza, "Fisher
 * Information Field: an Efficient and Differentiable Map for Perception-aware
 * Planning" (arXiv 2008.03324).  Everything is plain FP64, one landmark and one
 * voxel at a time, in the paper's notation; there is no blocking, no fusion and
 * no algebraic shortcut beyond what the paper states.  The only FP32 code is the
 * range predicate that decides landmark membership, which is defined in FP32 so
 * that every implementation takes the same discrete decision.
 *
 * Conventions (the paper's, plus the readings stated next to each function):
 *   pose T_wc = {R_wc, t}; quaternion q = (w, x, y, z), Hamilton, R_wc = R(q);
 *   optical axis z = R_wc e3; landmark p in world coordinates;
 *   perturbation: global (left) se(3), xi = [rho; phi] (Sec. V-A, eq:deriv_se3,
 *   first form), about the world origin.
 *   grid: voxel (i,j,k) has centre origin + (i,j,k) h; linear index
 *   i + nx (j + ny k) (x fastest).
 *
 * Parity status of each function is stated in its comment.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TRACE 1u
#define ORC_LMIN 2u
#define ORC_LOGDET 4u
#define ORC_FIM 8u

/* ---------------------------------------------------------------- helpers */

static void mat3_skew(const double v[3], double S[9]) {
  /* [v]x such that [v]x w = v x w */
  S[0] = 0.0;   S[1] = -v[2]; S[2] = v[1];
  S[3] = v[2];  S[4] = 0.0;   S[5] = -v[0];
  S[6] = -v[1]; S[7] = v[0];  S[8] = 0.0;
}

/* R_wc from a (not necessarily unit) quaternion (w, x, y, z): normalise, then
 * the standard Hamilton rotation matrix. */
void oracle_quat_to_R(const double q_in[4], double R[9]) {
  double nq = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] +
                   q_in[3] * q_in[3]);
  double w = q_in[0] / nq, x = q_in[1] / nq, y = q_in[2] / nq, z = q_in[3] / nq;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------ quadratic visibility */

/* Coefficients {k2, k1, k0} of v_q(theta) = k2 cos^2 + k1 cos + k0 fixed by the
 * three conditions of eq:quadratic_conditions (Sec. V-B): v(0) = 1, v(pi) = 0,
 * v(alpha) = v_alpha.  Solved as the 3x3 linear system it is, by Gaussian
 * elimination with partial pivoting.  k[0] = k2, k[1] = k1, k[2] = k0. */
void oracle_quad_coeffs(double alpha, double v_alpha, double k[3]) {
  double c = cos(alpha);
  double A[3][4] = {{1.0, 1.0, 1.0, 1.0},      /* cos = 1  -> 1   */
                    {1.0, -1.0, 1.0, 0.0},     /* cos = -1 -> 0   */
                    {c * c, c, 1.0, v_alpha}}; /* cos = c  -> v_a */
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    for (int j = 0; j < 4; ++j) {
      double tmp = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = tmp;
    }
    for (int r = col + 1; r < 3; ++r) {
      double f = A[r][col] / A[col][col];
      for (int j = col; j < 4; ++j) A[r][j] -= f * A[col][j];
    }
  }
  for (int r = 2; r >= 0; --r) {
    double s = A[r][3];
    for (int j = r + 1; j < 3; ++j) s -= A[r][j] * k[j];
    k[r] = s / A[r][r];
  }
}

/* vr(z) and vp(u) of eq:quad_vis_component (Sec. V-B), length 10. */
void oracle_vr(const double k[3], const double z[3], double vr[10]) {
  double k2 = k[0], k1 = k[1], k0 = k[2];
  vr[0] = k2 * z[0] * z[0]; vr[1] = k2 * z[1] * z[1]; vr[2] = k2 * z[2] * z[2];
  vr[3] = 2 * k2 * z[0] * z[1]; vr[4] = 2 * k2 * z[0] * z[2]; vr[5] = 2 * k2 * z[1] * z[2];
  vr[6] = k1 * z[0]; vr[7] = k1 * z[1]; vr[8] = k1 * z[2]; vr[9] = k0;
}

void oracle_vp(const double u[3], double vp[10]) {
  vp[0] = u[0] * u[0]; vp[1] = u[1] * u[1]; vp[2] = u[2] * u[2];
  vp[3] = u[0] * u[1]; vp[4] = u[0] * u[2]; vp[5] = u[1] * u[2];
  vp[6] = u[0]; vp[7] = u[1]; vp[8] = u[2]; vp[9] = 1.0;
}

/* ----------------------------------------------------- V_t membership */

/* Landmark p belongs to V_t iff max(r_min^2, 1e-12) <= n^2 <= r_max^2 with n^2
 * evaluated in FP32 exactly as fl(fma(dz,dz,fma(dy,dy,dx*dx))), d = fl32(p) -
 * fl32(t), and the bounds rounded to FP32.  The paper's simulation uses every
 * landmark (Sec. VII-A); the range form is the position-only selection of Sec.
 * V (first step, occlusion and viewpoint aside). */
int oracle_in_range(const double p[3], const double t[3], double r_min, double r_max) {
  float dx = (float)p[0] - (float)t[0];
  float dy = (float)p[1] - (float)t[1];
  float dz = (float)p[2] - (float)t[2];
  float n2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  float lo = (float)(r_min * r_min);
  if (lo < 1e-12f) lo = 1e-12f;
  float hi = isinf(r_max) ? INFINITY : (float)(r_max * r_max);
  return (n2 >= lo) && (n2 <= hi);
}

/* ------------------------------------------------ per-landmark FIM */

/* I_i = J^T J / sigma^2 (eq:fim_gaussian) with the Jacobian of the bearing
 * f = p^c / |p^c| w.r.t. the global perturbation (eq:jac_pose_global):
 *   J = (I/n - p^c p^c^T / n^3) R_cw [-I_3, [p]x],  p^c = R_cw (p - t).
 * Output: row-major 6x6 (36). */
void oracle_landmark_fim(const double p[3], const double t[3], const double R_wc[9],
                         double sigma, double I[36]) {
  double d[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
  double pc[3];
  for (int a = 0; a < 3; ++a) /* R_cw = R_wc^T */
    pc[a] = R_wc[0 * 3 + a] * d[0] + R_wc[1 * 3 + a] * d[1] + R_wc[2 * 3 + a] * d[2];
  double n = sqrt(pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2]);
  double dfdpc[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      dfdpc[a * 3 + b] = (a == b ? 1.0 / n : 0.0) - pc[a] * pc[b] / (n * n * n);
  double S[9];
  mat3_skew(p, S);
  double right[18]; /* R_cw [-I, [p]x], 3x6 */
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) {
      right[a * 6 + b] = -R_wc[b * 3 + a];
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += R_wc[c * 3 + a] * S[c * 3 + b];
      right[a * 6 + 3 + b] = s;
    }
  }
  double J[18];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 6; ++b) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += dfdpc[a * 3 + c] * right[c * 6 + b];
      J[a * 6 + b] = s;
    }
  double inv_s2 = 1.0 / (sigma * sigma);
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += J[c * 6 + a] * J[c * 6 + b];
      I[a * 6 + b] = s * inv_s2;
    }
}

/* ---------------------------------------------------- field building */

typedef struct {
  double origin[3];
  double h;
  int32_t nx, ny, nz;
} orc_grid;

void oracle_voxel_centre(const orc_grid* g, int64_t v, double t[3]) {
  int64_t i = v % g->nx, j = (v / g->nx) % g->ny, k = v / ((int64_t)g->nx * g->ny);
  t[0] = g->origin[0] + (double)i * g->h;
  t[1] = g->origin[1] + (double)j * g->h;
  t[2] = g->origin[2] + (double)k * g->h;
}

/* Positional information factor at one position t (eq:general_info_pif):
 *   C_k = sum_{i in V_t} vp_k(u_i) I_i,  k = 0..9,  u_i = (p_i - t)/|p_i - t|.
 * I_i is rotation invariant (eq:global_fim_eq), so it is evaluated with
 * R_wc = I.  Output: 10 row-major 6x6 blocks (360 doubles = 36 N_v). */
void oracle_info_factor(const double* lm, int64_t L, const double t[3], double sigma,
                        double r_min, double r_max, double C[360]) {
  static const double Rid[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  memset(C, 0, 360 * sizeof(double));
  for (int64_t i = 0; i < L; ++i) {
    const double* p = lm + 3 * i;
    if (!oracle_in_range(p, t, r_min, r_max)) continue;
    double d[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double u[3] = {d[0] / n, d[1] / n, d[2] / n};
    double I[36], vp[10];
    oracle_landmark_fim(p, t, Rid, sigma, I);
    oracle_vp(u, vp);
    for (int k = 0; k < 10; ++k)
      for (int e = 0; e < 36; ++e) C[k * 36 + e] += vp[k] * I[e];
  }
}

/* Build the factors of the listed voxels (all of them when voxel_ids == NULL,
 * then n_vox must equal nx*ny*nz).  Output C[n_vox][360]. */
void oracle_build(const double* lm, int64_t L, const orc_grid* g, double sigma, double r_min,
                  double r_max, const int64_t* voxel_ids, int64_t n_vox, double* C) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t a = 0; a < n_vox; ++a) {
    int64_t v = voxel_ids ? voxel_ids[a] : a;
    double t[3];
    oracle_voxel_centre(g, v, t);
    oracle_info_factor(lm, L, t, sigma, r_min, r_max, C + a * 360);
  }
}

/* Positional trace factor (eq:general_trace_pif): C_Tr,k = sum vp_k Tr(I_i). */
void oracle_trace_factor(const double* lm, int64_t L, const double t[3], double sigma,
                         double r_min, double r_max, double CT[10]) {
  static const double Rid[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  memset(CT, 0, 10 * sizeof(double));
  for (int64_t i = 0; i < L; ++i) {
    const double* p = lm + 3 * i;
    if (!oracle_in_range(p, t, r_min, r_max)) continue;
    double d[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double u[3] = {d[0] / n, d[1] / n, d[2] / n};
    double I[36], vp[10];
    oracle_landmark_fim(p, t, Rid, sigma, I);
    oracle_vp(u, vp);
    double tr = 0.0;
    for (int a = 0; a < 6; ++a) tr += I[a * 6 + a];
    for (int k = 0; k < 10; ++k) CT[k] += vp[k] * tr;
  }
}

/* --------------------------------------------------- 6x6 metrics */

/* Cyclic Jacobi on a symmetric 6x6 until the off-diagonal Frobenius norm is
 * below 1e-15 of the full norm.  Returns eigenvalues w[6] (unsorted) and the
 * eigenvectors as columns of V (row-major). */
void oracle_jacobi6(const double F_in[36], double w[6], double V[36]) {
  double A[36];
  memcpy(A, F_in, sizeof(A));
  for (int a = 0; a < 36; ++a) V[a] = (a % 7 == 0) ? 1.0 : 0.0;
  double fro = 0.0;
  for (int a = 0; a < 36; ++a) fro += A[a] * A[a];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < 6; ++p)
      for (int q = p + 1; q < 6; ++q) off += 2.0 * A[p * 6 + q] * A[p * 6 + q];
    if (off <= 1e-30 * fro || off == 0.0) break;
    for (int p = 0; p < 6; ++p)
      for (int q = p + 1; q < 6; ++q) {
        double apq = A[p * 6 + q];
        if (apq == 0.0) continue;
        double theta = (A[q * 6 + q] - A[p * 6 + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* A <- J^T A J with J the Givens rotation in the (p, q) plane */
        for (int k = 0; k < 6; ++k) {
          double akp = A[k * 6 + p], akq = A[k * 6 + q];
          A[k * 6 + p] = c * akp - s * akq;
          A[k * 6 + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 6; ++k) {
          double apk = A[p * 6 + k], aqk = A[q * 6 + k];
          A[p * 6 + k] = c * apk - s * aqk;
          A[q * 6 + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 6; ++k) {
          double vkp = V[k * 6 + p], vkq = V[k * 6 + q];
          V[k * 6 + p] = c * vkp - s * vkq;
          V[k * 6 + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int a = 0; a < 6; ++a) w[a] = A[a * 6 + a];
}

/* log det by Cholesky; NaN when a pivot is not positive.  Optionally returns
 * F^-1 (row-major) when PD. */
double oracle_logdet6(const double F[36], double* Finv) {
  double Lc[36];
  memset(Lc, 0, sizeof(Lc));
  for (int j = 0; j < 6; ++j) {
    double s = F[j * 6 + j];
    for (int k = 0; k < j; ++k) s -= Lc[j * 6 + k] * Lc[j * 6 + k];
    if (!(s > 0.0)) return NAN;
    Lc[j * 6 + j] = sqrt(s);
    for (int i = j + 1; i < 6; ++i) {
      double r = F[i * 6 + j];
      for (int k = 0; k < j; ++k) r -= Lc[i * 6 + k] * Lc[j * 6 + k];
      Lc[i * 6 + j] = r / Lc[j * 6 + j];
    }
  }
  double ld = 0.0;
  for (int j = 0; j < 6; ++j) ld += 2.0 * log(Lc[j * 6 + j]);
  if (Finv) {
    /* solve F X = I column by column */
    for (int col = 0; col < 6; ++col) {
      double y[6], x[6];
      for (int i = 0; i < 6; ++i) {
        double s = (i == col) ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) s -= Lc[i * 6 + k] * y[k];
        y[i] = s / Lc[i * 6 + i];
      }
      for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= Lc[k * 6 + i] * x[k];
        x[i] = s / Lc[i * 6 + i];
      }
      for (int i = 0; i < 6; ++i) Finv[i * 6 + col] = x[i];
    }
  }
  return ld;
}

/* The information metrics s(.) of eq:cost_info (Sec. IV): trace, smallest
 * eigenvalue, log-determinant.  out receives the requested columns in the
 * order trace, lmin, logdet, then the 21 upper-triangle entries (row-major)
 * when ORC_FIM is set.  Returns the number of columns written. */
int oracle_metrics(const double F[36], uint32_t metrics, double* out) {
  int c = 0;
  if (metrics & ORC_TRACE) {
    double tr = 0.0;
    for (int a = 0; a < 6; ++a) tr += F[a * 6 + a];
    out[c++] = tr;
  }
  if (metrics & ORC_LMIN) {
    double w[6], V[36];
    oracle_jacobi6(F, w, V);
    double m = w[0];
    for (int a = 1; a < 6; ++a) m = w[a] < m ? w[a] : m;
    out[c++] = m;
  }
  if (metrics & ORC_LOGDET) out[c++] = oracle_logdet6(F, NULL);
  if (metrics & ORC_FIM)
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b) out[c++] = F[a * 6 + b];
  return c;
}

/* ------------------------------------------------------- field query */

/* Cell and trilinear weights over the 8 surrounding voxel centres (Sec. VI-A:
 * factors are retrieved by interpolation; Sec. VII-A: up to 8 voxels).  The
 * position is clamped to the hull of voxel centres (constant extension).
 * For each corner j = jx + 2 jy + 4 jz: ids[j], w[j], and dw[j][c] = dw_j/dt_c. */
static int trilinear(const orc_grid* g, const double t[3], int64_t ids[8], double w[8],
                     double dw[8][3]) {
  const int32_t n[3] = {g->nx, g->ny, g->nz};
  int64_t i0[3];
  double f[3], df[3];
  int clamped = 0;
  for (int c = 0; c < 3; ++c) {
    double gc = (t[c] - g->origin[c]) / g->h;
    if (gc < 0.0 || gc > (double)(n[c] - 1)) clamped = 1;
    if (n[c] == 1) { i0[c] = 0; f[c] = 0.0; df[c] = 0.0; continue; }
    double fl = floor(gc);
    if (fl < 0.0) fl = 0.0;
    if (fl > (double)(n[c] - 2)) fl = (double)(n[c] - 2);
    i0[c] = (int64_t)fl;
    f[c] = gc - fl;
    df[c] = 1.0 / g->h;
    if (f[c] < 0.0) { f[c] = 0.0; df[c] = 0.0; }
    if (f[c] > 1.0) { f[c] = 1.0; df[c] = 0.0; }
  }
  for (int j = 0; j < 8; ++j) {
    int b[3] = {j & 1, (j >> 1) & 1, (j >> 2) & 1};
    int64_t idx[3];
    double wc[3], dwc[3];
    for (int c = 0; c < 3; ++c) {
      idx[c] = i0[c] + ((n[c] == 1) ? 0 : b[c]);
      wc[c] = b[c] ? f[c] : 1.0 - f[c];
      dwc[c] = b[c] ? df[c] : -df[c];
    }
    ids[j] = idx[0] + (int64_t)g->nx * (idx[1] + (int64_t)g->ny * idx[2]);
    w[j] = wc[0] * wc[1] * wc[2];
    dw[j][0] = dwc[0] * wc[1] * wc[2];
    dw[j][1] = wc[0] * dwc[1] * wc[2];
    dw[j][2] = wc[0] * wc[1] * dwc[2];
  }
  return clamped;
}

static int nearest(const orc_grid* g, const double t[3], int64_t* id) {
  const int32_t n[3] = {g->nx, g->ny, g->nz};
  int64_t idx[3];
  int clamped = 0;
  for (int c = 0; c < 3; ++c) {
    double gc = (t[c] - g->origin[c]) / g->h;
    if (gc < 0.0 || gc > (double)(n[c] - 1)) clamped = 1;
    double r = floor(gc + 0.5);
    if (r < 0.0) r = 0.0;
    if (r > (double)(n[c] - 1)) r = (double)(n[c] - 1);
    idx[c] = (int64_t)r;
  }
  *id = idx[0] + (int64_t)g->nx * (idx[1] + (int64_t)g->ny * idx[2]);
  return clamped;
}

/* F = V_I(R) C_I = sum_k vr_k(z) C_k (eq:fim_separation). */
static void contract(const double* C, const double vr[10], double F[36]) {
  for (int e = 0; e < 36; ++e) {
    double s = 0.0;
    for (int k = 0; k < 10; ++k) s += vr[k] * C[k * 36 + e];
    F[e] = s;
  }
}

/* Interpolated factor and FIM at one pose from a field given as a lookup:
 * either the whole field (field[v*360]) or, when field_ids != NULL, a sorted
 * table field_ids[n_field] of the voxels present. */
static const double* row_at(const double* field, const int64_t* ids, int64_t n_field,
                            int64_t per, int64_t v) {
  if (!ids) return field + v * per;
  int64_t lo = 0, hi = n_field - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (ids[mid] == v) return field + mid * per;
    if (ids[mid] < v) lo = mid + 1; else hi = mid - 1;
  }
  return NULL;
}

static const double* field_at(const double* field, const int64_t* field_ids, int64_t n_field,
                              int64_t v) {
  return row_at(field, field_ids, n_field, 360, v);
}

/* Query one pose: returns the clamp flag, fills F (6x6) and Cbar (10 blocks). */
static int query_one(const double* field, const int64_t* field_ids, int64_t n_field,
                     const orc_grid* g, const double k[3], const double t[3], const double q[4],
                     int interp, double F[36], double Cbar[360], double vr[10], double z[3]) {
  double R[9];
  oracle_quat_to_R(q, R);
  z[0] = R[2]; z[1] = R[5]; z[2] = R[8];
  oracle_vr(k, z, vr);
  memset(Cbar, 0, 360 * sizeof(double));
  int clamped;
  if (interp == 1) {
    int64_t id;
    clamped = nearest(g, t, &id);
    const double* C = field_at(field, field_ids, n_field, id);
    if (!C) return -1;
    memcpy(Cbar, C, 360 * sizeof(double));
  } else {
    int64_t ids[8];
    double w[8], dw[8][3];
    clamped = trilinear(g, t, ids, w, dw);
    for (int j = 0; j < 8; ++j) {
      const double* C = field_at(field, field_ids, n_field, ids[j]);
      if (!C) return -1;
      for (int e = 0; e < 360; ++e) Cbar[e] += w[j] * C[e];
    }
  }
  contract(Cbar, vr, F);
  return clamped;
}

/* Field query for m poses (Sec. VI-A, eq:fim_separation + eq:cost_info metrics).
 * interp: 0 trilinear, 1 nearest.  out[m][ncols]; flags[m] bit0 = clamped,
 * bit1 = not PD (logdet NaN).  Returns 0, or -1 if a needed voxel is absent. */
int oracle_query(const double* field, const int64_t* field_ids, int64_t n_field,
                 const orc_grid* g, double alpha, double v_alpha, const double* t,
                 const double* q, int64_t m, uint32_t metrics, int interp, double* out,
                 uint8_t* flags) {
  double k[3];
  oracle_quad_coeffs(alpha, v_alpha, k);
  int ncols = ((metrics & 1) != 0) + ((metrics & 2) != 0) + ((metrics & 4) != 0) +
              ((metrics & 8) ? 21 : 0);
  int err = 0;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < m; ++a) {
    double F[36], Cbar[360], vr[10], z[3];
    int cl = query_one(field, field_ids, n_field, g, k, t + 3 * a, q + 4 * a, interp, F, Cbar,
                       vr, z);
    if (cl < 0) { err = 1; continue; }
    oracle_metrics(F, metrics, out + a * ncols);
    if (flags) {
      double ld = oracle_logdet6(F, NULL);
      flags[a] = (uint8_t)((cl ? 1 : 0) | (isnan(ld) ? 2 : 0));
    }
  }
  return err ? -1 : 0;
}

/* Interpolated FIM (full 6x6) at m poses, for error measures. */
int oracle_query_fim(const double* field, const int64_t* field_ids, int64_t n_field,
                     const orc_grid* g, double alpha, double v_alpha, const double* t,
                     const double* q, int64_t m, int interp, double* F_out) {
  double k[3];
  oracle_quad_coeffs(alpha, v_alpha, k);
  int err = 0;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < m; ++a) {
    double Cbar[360], vr[10], z[3];
    if (query_one(field, field_ids, n_field, g, k, t + 3 * a, q + 4 * a, interp,
                  F_out + 36 * a, Cbar, vr, z) < 0)
      err = 1;
  }
  return err ? -1 : 0;
}

/* Trace factors of the listed voxels (all when voxel_ids == NULL), the trace
 * field of eq:general_trace_pif: CT[n_vox][10]. */
void oracle_trace_build(const double* lm, int64_t L, const orc_grid* g, double sigma,
                        double r_min, double r_max, const int64_t* voxel_ids, int64_t n_vox,
                        double* CT) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t a = 0; a < n_vox; ++a) {
    int64_t v = voxel_ids ? voxel_ids[a] : a;
    double t[3];
    oracle_voxel_centre(g, v, t);
    oracle_trace_factor(lm, L, t, sigma, r_min, r_max, CT + a * 10);
  }
}

/* Trace-field query (eq:fim_trace_separation, eq:general_trace_pif): the
 * trace factor is retrieved at t like the information factor (trilinear over
 * the 8 voxel centres, or the nearest one; Sec. VI-A), then
 *   Tr F = sum_k vr_k(z) CTbar_k.
 * field: [n_field][10]; out[m]; flags[m] bit0 = clamped (may be NULL).
 * Returns 0, or -1 if a needed voxel is absent. */
int oracle_trace_query(const double* field, const int64_t* field_ids, int64_t n_field,
                       const orc_grid* g, double alpha, double v_alpha, const double* t,
                       const double* q, int64_t m, int interp, double* out, uint8_t* flags) {
  double k[3];
  oracle_quad_coeffs(alpha, v_alpha, k);
  int err = 0;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < m; ++a) {
    double R[9], z[3], vr[10], CT[10] = {0};
    oracle_quat_to_R(q + 4 * a, R);
    z[0] = R[2]; z[1] = R[5]; z[2] = R[8];
    oracle_vr(k, z, vr);
    int clamped, missing = 0;
    if (interp == 1) {
      int64_t id;
      clamped = nearest(g, t + 3 * a, &id);
      const double* C = row_at(field, field_ids, n_field, 10, id);
      if (!C) missing = 1; else memcpy(CT, C, sizeof CT);
    } else {
      int64_t ids[8];
      double w[8], dw[8][3];
      clamped = trilinear(g, t + 3 * a, ids, w, dw);
      for (int j = 0; j < 8; ++j) {
        const double* C = row_at(field, field_ids, n_field, 10, ids[j]);
        if (!C) { missing = 1; break; }
        for (int e = 0; e < 10; ++e) CT[e] += w[j] * C[e];
      }
    }
    if (missing) { err = 1; continue; }
    double s = 0.0;
    for (int e = 0; e < 10; ++e) s += vr[e] * CT[e];
    out[a] = s;
    if (flags) flags[a] = (uint8_t)(clamped ? 1 : 0);
  }
  return err ? -1 : 0;
}

/* Optimal-view sweep (Sec. VII-A, "Relative Measures": the best view at a
 * position is the orientation with the largest metric).  With the quadratic
 * visibility the FIM depends on the orientation only through the optical axis
 * z (eq:quad_vis_component, eq:fim_separation), so each candidate is an axis:
 * the factor is interpolated at t once, then F(z) = sum_k vr_k(z) Cbar_k for
 * every axis (normalised here) and the single metric `which` is taken.
 * values[n_pos][n_dir] (may be NULL); best[n_pos] (may be NULL) = index of the
 * largest value, the first one among equal values, NaN never largest, -1 if
 * all are NaN.  Returns 0, or -1 if a needed voxel is absent. */
int oracle_view_sweep(const double* field, const int64_t* field_ids, int64_t n_field,
                      const orc_grid* g, double alpha, double v_alpha, const double* t,
                      int64_t n_pos, const double* dirs, int64_t n_dir, uint32_t which,
                      int interp, double* values, int64_t* best) {
  double k[3];
  oracle_quad_coeffs(alpha, v_alpha, k);
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t a = 0; a < n_pos; ++a) {
    /* the identity orientation: only Cbar is used from query_one */
    const double q_id[4] = {1.0, 0.0, 0.0, 0.0};
    double F[36], Cbar[360], vr[10], z[3];
    if (query_one(field, field_ids, n_field, g, k, t + 3 * a, q_id, interp, F, Cbar, vr, z) < 0) {
      err = 1;
      continue;
    }
    double bv = 0.0;
    int64_t bi = -1;
    for (int64_t d = 0; d < n_dir; ++d) {
      const double* zd = dirs + 3 * d;
      double nz = sqrt(zd[0] * zd[0] + zd[1] * zd[1] + zd[2] * zd[2]);
      double zu[3] = {zd[0] / nz, zd[1] / nz, zd[2] / nz};
      oracle_vr(k, zu, vr);
      contract(Cbar, vr, F);
      double val;
      oracle_metrics(F, which, &val);
      if (values) values[a * n_dir + d] = val;
      if (!isnan(val) && (bi < 0 || val > bv)) { bv = val; bi = d; }
    }
    if (best) best[a] = bi;
  }
  return err ? -1 : 0;
}

/* ------------------------------------------------- GP visibility (f2) */

/* Smooth visibility of eq:sigmoid_vis_func: 1 / (1 + exp(-k_s (cos theta -
 * cos alpha))), the function the GP is trained to reproduce (Sec. V-B). */
double oracle_sigmoid_vis(double ks, double alpha, double cos_theta) {
  return 1.0 / (1.0 + exp(-ks * (cos_theta - cos(alpha))));
}

/* Squared-exponential kernel on unit vectors (Sec. V-B), signal variance 1:
 * k(z1, z2) = exp(-|z1 - z2|^2 / (2 l^2)).  The posterior mean does not depend
 * on the signal variance once the noise is expressed relative to it. */
double oracle_gp_kernel(double l, const double z1[3], const double z2[3]) {
  double d0 = z1[0] - z2[0], d1 = z1[1] - z2[1], d2 = z1[2] - z2[2];
  return exp(-(d0 * d0 + d1 * d1 + d2 * d2) / (2.0 * l * l));
}

/* Lower Cholesky factor of the n x n symmetric matrix A (row-major, in place
 * in L).  Returns 0, or -1 if A is not positive definite. */
static int cholesky(int n, const double* A, double* L) {
  memset(L, 0, (size_t)n * n * sizeof(double));
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return -1;
    L[j * n + j] = sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  return 0;
}

/* K^s + noise I over the sample axes Z[ns][3] (Sec. V-B). */
static void gp_ks(int ns, const double* Z, double l, double noise, double* K) {
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b)
      K[a * ns + b] = oracle_gp_kernel(l, Z + 3 * a, Z + 3 * b) + (a == b ? noise : 0.0);
}

/* (K^s + noise I)^-1 (row-major ns x ns).  eq:gp_vis_approx prints
 * K_z K^s v^s; the GP posterior mean it names (eq:gp_regress) is
 * K_z (K^s + noise I)^-1 v^s, which is the reading taken here.  Columns of the
 * inverse by two triangular solves per unit vector.  Returns 0 or -1. */
int oracle_gp_inverse(int ns, const double* Z, double l, double noise, double* Ainv) {
  double* K = (double*)malloc((size_t)ns * ns * sizeof(double));
  double* L = (double*)malloc((size_t)ns * ns * sizeof(double));
  double* y = (double*)malloc((size_t)ns * sizeof(double));
  gp_ks(ns, Z, l, noise, K);
  int rc = cholesky(ns, K, L);
  for (int c = 0; rc == 0 && c < ns; ++c) {
    for (int i = 0; i < ns; ++i) { /* L y = e_c */
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * ns + k] * y[k];
      y[i] = s / L[i * ns + i];
    }
    for (int i = ns - 1; i >= 0; --i) { /* L^T x = y */
      double s = y[i];
      for (int k = i + 1; k < ns; ++k) s -= L[k * ns + i] * Ainv[k * ns + c];
      Ainv[i * ns + c] = s / L[i * ns + i];
    }
  }
  free(K); free(L); free(y);
  return rc;
}

/* vr = K_z = [k(z, z_g)]_g (Sec. V-B: vr depends only on the rotation). */
void oracle_gp_vr(int ns, const double* Z, double l, const double z[3], double* vr) {
  for (int g = 0; g < ns; ++g) vr[g] = oracle_gp_kernel(l, z, Z + 3 * g);
}

/* vp = (K^s + noise I)^-1 v^s(u), v^s_g = sigmoid visibility of z_g . u. */
void oracle_gp_vp(int ns, const double* Z, double ks, double alpha, const double* Ainv,
                  const double u[3], double* vp) {
  double* vs = (double*)malloc((size_t)ns * sizeof(double));
  for (int g = 0; g < ns; ++g) {
    const double* zg = Z + 3 * g;
    vs[g] = oracle_sigmoid_vis(ks, alpha, zg[0] * u[0] + zg[1] * u[1] + zg[2] * u[2]);
  }
  for (int g = 0; g < ns; ++g) {
    double s = 0.0;
    for (int h = 0; h < ns; ++h) s += Ainv[g * ns + h] * vs[h];
    vp[g] = s;
  }
  free(vs);
}

/* GP information factor at t (eq:general_info_pif with N_v = N_s):
 *   C_g = sum_{i in V_t} vp_g(u_i) I_i,  C[ns][36] row-major blocks;
 * with trace != 0 the trace factor C_Tr,g = sum vp_g(u_i) Tr(I_i), C[ns]. */
void oracle_gp_factor(const double* lm, int64_t L, const double t[3], double sigma, double r_min,
                      double r_max, int ns, const double* Z, double ks, double alpha,
                      const double* Ainv, int trace, double* C) {
  static const double Rid[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  const int blk = trace ? 1 : 36;
  memset(C, 0, (size_t)ns * blk * sizeof(double));
  double* vp = (double*)malloc((size_t)ns * sizeof(double));
  for (int64_t i = 0; i < L; ++i) {
    const double* p = lm + 3 * i;
    if (!oracle_in_range(p, t, r_min, r_max)) continue;
    double d[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double u[3] = {d[0] / n, d[1] / n, d[2] / n};
    double I[36];
    oracle_landmark_fim(p, t, Rid, sigma, I);
    oracle_gp_vp(ns, Z, ks, alpha, Ainv, u, vp);
    if (trace) {
      double tr = 0.0;
      for (int a = 0; a < 6; ++a) tr += I[a * 6 + a];
      for (int g = 0; g < ns; ++g) C[g] += vp[g] * tr;
    } else {
      for (int g = 0; g < ns; ++g)
        for (int e = 0; e < 36; ++e) C[g * 36 + e] += vp[g] * I[e];
    }
  }
  free(vp);
}

/* GP factors of the listed voxels (all when voxel_ids == NULL). */
void oracle_gp_build(const double* lm, int64_t L, const orc_grid* g, double sigma, double r_min,
                     double r_max, int ns, const double* Z, double ks, double alpha,
                     const double* Ainv, int trace, const int64_t* voxel_ids, int64_t n_vox,
                     double* C) {
  const int64_t per = (int64_t)ns * (trace ? 1 : 36);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t a = 0; a < n_vox; ++a) {
    int64_t v = voxel_ids ? voxel_ids[a] : a;
    double t[3];
    oracle_voxel_centre(g, v, t);
    oracle_gp_factor(lm, L, t, sigma, r_min, r_max, ns, Z, ks, alpha, Ainv, trace, C + a * per);
  }
}

/* GP field query (eq:fim_separation with vr = K_z): the factor is interpolated
 * at t (trilinear over the 8 voxel centres, or the nearest one), then
 *   F = sum_g vr_g(z) Cbar_g,   or for trace fields Tr = sum_g vr_g Cbar_Tr,g.
 * Information fields: out[m][ncols] per the metric mask and F_out[m][36] if
 * non-NULL; trace fields: out[m][1].  Returns 0 or -1 if a voxel is absent. */
int oracle_gp_query(const double* field, const int64_t* ids, int64_t n_field, const orc_grid* g,
                    int ns, int trace, const double* Z, double l, const double* t,
                    const double* q, int64_t m, uint32_t metrics, int interp, double* out,
                    uint8_t* flags, double* F_out) {
  const int64_t per = (int64_t)ns * (trace ? 1 : 36);
  int ncols = trace ? 1 : ((metrics & 1) != 0) + ((metrics & 2) != 0) + ((metrics & 4) != 0) +
                              ((metrics & 8) ? 21 : 0);
  int err = 0;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < m; ++a) {
    double R[9], z[3];
    oracle_quat_to_R(q + 4 * a, R);
    z[0] = R[2]; z[1] = R[5]; z[2] = R[8];
    double* vr = (double*)malloc((size_t)ns * sizeof(double));
    double* Cbar = (double*)calloc((size_t)per, sizeof(double));
    oracle_gp_vr(ns, Z, l, z, vr);
    int clamped = 0, missing = 0;
    if (interp == 1) {
      int64_t id;
      clamped = nearest(g, t + 3 * a, &id);
      const double* C = row_at(field, ids, n_field, per, id);
      if (!C) missing = 1; else memcpy(Cbar, C, (size_t)per * sizeof(double));
    } else {
      int64_t vid[8];
      double w[8], dw[8][3];
      clamped = trilinear(g, t + 3 * a, vid, w, dw);
      for (int j = 0; j < 8 && !missing; ++j) {
        const double* C = row_at(field, ids, n_field, per, vid[j]);
        if (!C) { missing = 1; break; }
        for (int64_t e = 0; e < per; ++e) Cbar[e] += w[j] * C[e];
      }
    }
    if (missing) {
      err = 1;
    } else if (trace) {
      double s = 0.0;
      for (int k = 0; k < ns; ++k) s += vr[k] * Cbar[k];
      out[a] = s;
      if (flags) flags[a] = (uint8_t)(clamped ? 1 : 0);
    } else {
      double F[36];
      for (int e = 0; e < 36; ++e) {
        double s = 0.0;
        for (int k = 0; k < ns; ++k) s += vr[k] * Cbar[k * 36 + e];
        F[e] = s;
      }
      if (out) oracle_metrics(F, metrics, out + a * ncols);
      if (F_out) memcpy(F_out + 36 * a, F, sizeof F);
      if (flags) {
        double ld = oracle_logdet6(F, NULL);
        flags[a] = (uint8_t)((clamped ? 1 : 0) | (isnan(ld) ? 2 : 0));
      }
    }
    free(vr);
    free(Cbar);
  }
  return err ? -1 : 0;
}

/* Point-cloud FIM under the GP visibility (eq:vis_fim with v = v_gp(z, u_i) =
 * vr(z) . vp(u_i), eq:gp_vis_approx): F = sum_{i in V_t} v_gp I_i. */
void oracle_gp_pc_fim(const double* lm, int64_t L, double sigma, double r_min, double r_max,
                      int ns, const double* Z, double ks, double alpha, double l,
                      const double* Ainv, const double* t, const double* q, int64_t m,
                      double* F_out) {
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < m; ++a) {
    double R[9], z[3];
    oracle_quat_to_R(q + 4 * a, R);
    z[0] = R[2]; z[1] = R[5]; z[2] = R[8];
    double* vr = (double*)malloc((size_t)ns * sizeof(double));
    double* vp = (double*)malloc((size_t)ns * sizeof(double));
    oracle_gp_vr(ns, Z, l, z, vr);
    double F[36] = {0};
    const double* ta = t + 3 * a;
    for (int64_t i = 0; i < L; ++i) {
      const double* p = lm + 3 * i;
      if (!oracle_in_range(p, ta, r_min, r_max)) continue;
      double d[3] = {p[0] - ta[0], p[1] - ta[1], p[2] - ta[2]};
      double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double u[3] = {d[0] / n, d[1] / n, d[2] / n};
      double I[36];
      oracle_landmark_fim(p, ta, R, sigma, I);
      oracle_gp_vp(ns, Z, ks, alpha, Ainv, u, vp);
      double v = 0.0;
      for (int k = 0; k < ns; ++k) v += vr[k] * vp[k];
      for (int e = 0; e < 36; ++e) F[e] += v * I[e];
    }
    memcpy(F_out + 36 * a, F, sizeof F);
    free(vr);
    free(vp);
  }
}

/* Log marginal likelihood of the length scale l (Sec. V-B hyperparameters; the
 * standard GP evidence): with K_y = K^s + noise I and one output vector per
 * training direction u_t, y_t[g] = sigmoid visibility of z_g . u_t,
 *   log p = sum_t (-1/2 y_t^T K_y^-1 y_t) - n_train/2 log|K_y| - n_train ns/2 log 2 pi.
 * U[n_train][3].  Returns -INFINITY if K_y is not positive definite. */
double oracle_gp_lml(int ns, const double* Z, double ks, double alpha, double l, double noise,
                     const double* U, int n_train) {
  double* K = (double*)malloc((size_t)ns * ns * sizeof(double));
  double* L = (double*)malloc((size_t)ns * ns * sizeof(double));
  double* y = (double*)malloc((size_t)ns * sizeof(double));
  double* w = (double*)malloc((size_t)ns * sizeof(double));
  gp_ks(ns, Z, l, noise, K);
  double res = -INFINITY;
  if (cholesky(ns, K, L) == 0) {
    double logdet = 0.0;
    for (int i = 0; i < ns; ++i) logdet += 2.0 * log(L[i * ns + i]);
    double quad = 0.0;
    for (int tt = 0; tt < n_train; ++tt) {
      const double* u = U + 3 * tt;
      for (int g = 0; g < ns; ++g) {
        const double* zg = Z + 3 * g;
        y[g] = oracle_sigmoid_vis(ks, alpha, zg[0] * u[0] + zg[1] * u[1] + zg[2] * u[2]);
      }
      for (int i = 0; i < ns; ++i) { /* L w = y, then y^T K^-1 y = |w|^2 */
        double s = y[i];
        for (int k = 0; k < i; ++k) s -= L[i * ns + k] * w[k];
        w[i] = s / L[i * ns + i];
      }
      for (int i = 0; i < ns; ++i) quad += w[i] * w[i];
    }
    res = -0.5 * quad - 0.5 * n_train * logdet - 0.5 * n_train * ns * log(2.0 * M_PI);
  }
  free(K); free(L); free(y); free(w);
  return res;
}

/* ---------------------------------------------------------- gradient */

/* d s / d F for each metric (symmetric 6x6): trace -> I, lmin -> v v^T with v
 * the unit eigenvector of the smallest eigenvalue, logdet -> F^-1. */
static void metric_grad(const double F[36], uint32_t which, double G[36]) {
  memset(G, 0, 36 * sizeof(double));
  if (which == ORC_TRACE) {
    for (int a = 0; a < 6; ++a) G[a * 6 + a] = 1.0;
  } else if (which == ORC_LMIN) {
    double w[6], V[36];
    oracle_jacobi6(F, w, V);
    int im = 0;
    for (int a = 1; a < 6; ++a) if (w[a] < w[im]) im = a;
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) G[a * 6 + b] = V[a * 6 + im] * V[b * 6 + im];
  } else if (which == ORC_LOGDET) {
    if (isnan(oracle_logdet6(F, G)))
      for (int a = 0; a < 36; ++a) G[a] = NAN;
  }
}

/* Analytic gradient of the metrics w.r.t. the pose.  For a scalar s(F):
 *   ds/dt   = sum_j (dw_j/dt) <G, F^(j)>,   F^(j) = sum_k vr_k(z) C_k^(j)
 *   ds/dz   = sum_k (dvr_k/dz) <G, Cbar_k>
 *   ds/dphi = z x ds/dz   (left perturbation R <- exp([phi]x) R moves z by phi x z)
 * with G = ds/dF.  The paper states the map is differentiable (Sec. I, VII-B)
 * but gives no formula; this is the chain rule through eq:fim_separation and
 * the trilinear weights.  dL_dout[m][popcount(metrics & 7)] weights the
 * metrics.  Trilinear only. */
int oracle_query_grad(const double* field, const int64_t* field_ids, int64_t n_field,
                      const orc_grid* g, double alpha, double v_alpha, const double* t,
                      const double* q, int64_t m, uint32_t metrics, const double* dL_dout,
                      double* dL_dt, double* dL_dphi) {
  double k[3];
  oracle_quad_coeffs(alpha, v_alpha, k);
  int ncols = ((metrics & 1) != 0) + ((metrics & 2) != 0) + ((metrics & 4) != 0);
  int err = 0;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < m; ++a) {
    double F[36], Cbar[360], vr[10], z[3];
    const double* ta = t + 3 * a;
    if (query_one(field, field_ids, n_field, g, k, ta, q + 4 * a, 0, F, Cbar, vr, z) < 0) {
      err = 1;
      continue;
    }
    double G[36];
    memset(G, 0, sizeof(G));
    int col = 0;
    for (uint32_t bit = 1; bit <= 4; bit <<= 1) {
      if (!(metrics & bit)) continue;
      double up = dL_dout[a * ncols + col++];
      /* a metric with zero weight is not part of L: its derivative (NaN for
       * the log-det of a FIM that is not positive definite) does not enter */
      if (up == 0.0) continue;
      double Gm[36];
      metric_grad(F, bit, Gm);
      for (int e = 0; e < 36; ++e) G[e] += up * Gm[e];
    }
    int64_t ids[8];
    double w[8], dw[8][3];
    trilinear(g, ta, ids, w, dw);
    double gt[3] = {0, 0, 0};
    for (int j = 0; j < 8; ++j) {
      const double* C = field_at(field, field_ids, n_field, ids[j]);
      double Fj[36];
      contract(C, vr, Fj);
      double ip = 0.0;
      for (int e = 0; e < 36; ++e) ip += G[e] * Fj[e];
      for (int c = 0; c < 3; ++c) gt[c] += dw[j][c] * ip;
    }
    /* dvr_k/dz_c */
    double k2 = k[0], k1 = k[1];
    double dvr[10][3] = {{2 * k2 * z[0], 0, 0},          {0, 2 * k2 * z[1], 0},
                         {0, 0, 2 * k2 * z[2]},          {2 * k2 * z[1], 2 * k2 * z[0], 0},
                         {2 * k2 * z[2], 0, 2 * k2 * z[0]}, {0, 2 * k2 * z[2], 2 * k2 * z[1]},
                         {k1, 0, 0},                     {0, k1, 0},
                         {0, 0, k1},                     {0, 0, 0}};
    double gz[3] = {0, 0, 0};
    for (int kk = 0; kk < 10; ++kk) {
      double ip = 0.0;
      for (int e = 0; e < 36; ++e) ip += G[e] * Cbar[kk * 36 + e];
      for (int c = 0; c < 3; ++c) gz[c] += dvr[kk][c] * ip;
    }
    for (int c = 0; c < 3; ++c) dL_dt[3 * a + c] = gt[c];
    dL_dphi[3 * a + 0] = z[1] * gz[2] - z[2] * gz[1];
    dL_dphi[3 * a + 1] = z[2] * gz[0] - z[0] * gz[2];
    dL_dphi[3 * a + 2] = z[0] * gz[1] - z[1] * gz[0];
  }
  return err ? -1 : 0;
}

/* ------------------------------------------------ point-cloud brute force */

typedef struct {
  double fx, fy, cx, cy;
  int32_t width, height;
} orc_pinhole;

/* FIM of one pose from the point cloud (eq:cost_info, eq:vis_fim):
 *   F = sum_{i in V_t} v_i I_i.
 * Quadratic mode (cam == NULL): v_i = k2 c^2 + k1 c + k0 with c = z . u_i
 * (eq:quad_vis_approx, not clamped: negative values are part of the model).
 * Exact mode: v_i = 1 iff the landmark projects inside the image
 * (eq:exact_vis_func): p^c_z > 0 and 0 <= fx x/z + cx < W, 0 <= fy y/z + cy < H.
 * margin (optional) receives, in exact mode, the smallest distance in pixels of
 * any projection in front of the camera to an image border, for excluding
 * poses whose decision is within rounding of a border. */
void oracle_pc_fim(const double* lm, int64_t L, double alpha, double v_alpha, double sigma,
                   double r_min, double r_max, const orc_pinhole* cam, const double t[3],
                   const double q[4], double F[36], double* margin) {
  double k[3], R[9];
  oracle_quad_coeffs(alpha, v_alpha, k);
  oracle_quat_to_R(q, R);
  double z[3] = {R[2], R[5], R[8]};
  memset(F, 0, 36 * sizeof(double));
  double mg = INFINITY;
  for (int64_t i = 0; i < L; ++i) {
    const double* p = lm + 3 * i;
    if (!oracle_in_range(p, t, r_min, r_max)) continue;
    double d[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
    double v;
    if (!cam) {
      double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double c = (z[0] * d[0] + z[1] * d[1] + z[2] * d[2]) / n;
      v = k[0] * c * c + k[1] * c + k[2];
    } else {
      double pc[3];
      for (int a = 0; a < 3; ++a)
        pc[a] = R[0 * 3 + a] * d[0] + R[1 * 3 + a] * d[1] + R[2 * 3 + a] * d[2];
      v = 0.0;
      if (pc[2] > 0.0) {
        double u = cam->fx * pc[0] / pc[2] + cam->cx;
        double w = cam->fy * pc[1] / pc[2] + cam->cy;
        if (u >= 0.0 && u < cam->width && w >= 0.0 && w < cam->height) v = 1.0;
        double m1 = fmin(fabs(u), fabs(u - cam->width));
        double m2 = fmin(fabs(w), fabs(w - cam->height));
        double mm = fmin(m1, m2);
        /* only landmarks that may be inside count for the margin */
        if (u > -1.0 && u < cam->width + 1.0 && w > -1.0 && w < cam->height + 1.0)
          mg = fmin(mg, mm);
      }
      if (fabs(pc[2]) < 1e-9) mg = 0.0;
    }
    if (v == 0.0) continue;
    double I[36];
    oracle_landmark_fim(p, t, R, sigma, I);
    for (int e = 0; e < 36; ++e) F[e] += v * I[e];
  }
  if (margin) *margin = mg;
}

void oracle_pc_query(const double* lm, int64_t L, double alpha, double v_alpha, double sigma,
                     double r_min, double r_max, const orc_pinhole* cam, const double* t,
                     const double* q, int64_t m, uint32_t metrics, double* out,
                     double* F_out, double* margin) {
  int ncols = ((metrics & 1) != 0) + ((metrics & 2) != 0) + ((metrics & 4) != 0) +
              ((metrics & 8) ? 21 : 0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t a = 0; a < m; ++a) {
    double F[36];
    oracle_pc_fim(lm, L, alpha, v_alpha, sigma, r_min, r_max, cam, t + 3 * a, q + 4 * a, F,
                  margin ? margin + a : NULL);
    if (out) oracle_metrics(F, metrics, out + a * ncols);
    if (F_out) memcpy(F_out + 36 * a, F, sizeof(F));
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the OpenMP loops from here on (timing on one core or all). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
