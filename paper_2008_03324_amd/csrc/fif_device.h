// Device-side building blocks of the FIF kernels (gfx950).
//
// Field layout ("moment form").  Under the quadratic visibility of
// eq:quad_vis_approx the positional information factor of a voxel
// (eq:general_info_pif) is a fixed linear function of 66 sums over the
// landmarks in range, u = (p - t_v)/n, n = |p - t_v|:
//   G0: sum u^a             for all monomials of degree 4 (15) and 3 (10)
//   G2: sum u^a / n^2       degree 4 (15) and 3 (10)
//   G1: sum u^a / n         degree 3 (10) and 2 (6)
// Lower degrees follow from |u| = 1 (e.g. sum u_a u_b = sum_c sum u_a u_b u_c u_c).
// Writing the per-landmark FIM about the voxel centre,
//   I_i = M(t_v)^T (1/sigma^2) [[P/n^2, -[u]x/n], [[u]x/n, P]] M(t_v),
//   P = I - u u^T,  M(t) = [[I, -[t]x], [0, I]],
// follows from eq:jac_pose_global with [p]x = [t_v]x + [d]x and P[d]x = [d]x.
// Storage: the first 64 moments of every voxel form a 256-B (FP32) main record,
// exactly two 128-B cache lines.  The last 2 moments go to a "cell side
// record" of 16 scalars per voxel v: slot s = bx + 2 by + 4 bz holds the 2 side
// moments of voxel min(v + (bx, by, bz), n - 1), i.e. of every corner of the
// cell whose lowest corner is v.  A trilinear query then reads its 8 side pairs
// as one aligned 64-B block instead of touching four more cache lines.  Slot 0
// is written by the build; slots 1..7 are copied from the slot 0 of the
// neighbouring records by a second pass.
//
// 21-vectors hold symmetric 6x6 matrices as their upper triangle, row-major.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fif {

constexpr int kMain = 64;  // scalars per voxel in the main record
constexpr int kSide = 2;   // side moments per voxel
constexpr int kSideRec = 16;  // scalars per cell side record (8 corners x 2)
constexpr int kMom = 66;   // moments per voxel
constexpr int kTRec = 12;  // scalars per voxel record (trace field, 10 used)
// trace field stored per cell: the 10 factors of the cell's 8 corner voxels
// (corner j = bits x, y, z of j; clamped at the upper faces), slot 0 = the
// voxel's own
constexpr int kTCell = 80;
constexpr int O_G0_4 = 0, O_G0_3 = 15, O_G2_4 = 25, O_G2_3 = 40, O_G1_3 = 50, O_G1_2 = 60;

// ------------------------------------------------------------ symmetric indices

__host__ __device__ constexpr int i2(int a, int b) {  // a <= b
  return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
__host__ __device__ constexpr int s2(int a, int b) { return a <= b ? i2(a, b) : i2(b, a); }

__host__ __device__ constexpr int i3(int a, int b, int c) {  // a <= b <= c
  int idx = 0;
  for (int x = 0; x < 3; ++x)
    for (int y = x; y < 3; ++y)
      for (int z = y; z < 3; ++z) {
        if (x == a && y == b && z == c) return idx;
        ++idx;
      }
  return -1;
}
__host__ __device__ constexpr int s3(int a, int b, int c) {
  // sort three indices
  return (a <= b) ? ((b <= c) ? i3(a, b, c) : (a <= c ? i3(a, c, b) : i3(c, a, b)))
                  : ((a <= c) ? i3(b, a, c) : (b <= c ? i3(b, c, a) : i3(c, b, a)));
}

__host__ __device__ constexpr int i4(int a, int b, int c, int d) {  // sorted
  int idx = 0;
  for (int x = 0; x < 3; ++x)
    for (int y = x; y < 3; ++y)
      for (int z = y; z < 3; ++z)
        for (int w = z; w < 3; ++w) {
          if (x == a && y == b && z == c && w == d) return idx;
          ++idx;
        }
  return -1;
}
__host__ __device__ constexpr int s4(int a, int b, int c, int d) {
  int v[4] = {a, b, c, d};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j + 1 < 4 - i; ++j)
      if (v[j] > v[j + 1]) {
        int t = v[j]; v[j] = v[j + 1]; v[j + 1] = t;
      }
  return i4(v[0], v[1], v[2], v[3]);
}

__host__ __device__ constexpr int u21(int i, int j) {  // i <= j < 6
  return i * 6 - (i * (i - 1)) / 2 + (j - i);
}
__host__ __device__ constexpr int su21(int i, int j) { return i <= j ? u21(i, j) : u21(j, i); }

// 1/sqrt(x) by the hardware instruction (v_rsq_f32).  rsqrtf wraps it in a
// rescaling for x below the smallest normal FP32 number; the kernels call this
// only on squared landmark distances that passed the range predicate (n^2 >=
// 1e-12, or an FP64-derived n^2 of the same pair, far above that), where the
// two give the same value.
__device__ inline float rsq_normal(float x) { return __builtin_amdgcn_rsqf(x); }

// ------------------------------------------------------------ pose helpers

// Optical axis z = R(q) e3 for a quaternion (w, x, y, z) of any norm.
__device__ inline void quat_axis(double w, double x, double y, double z, double out[3]) {
  double n = w * w + x * x + y * y + z * z;
  double inv = 1.0 / n;
  out[0] = 2.0 * (x * z + w * y) * inv;
  out[1] = 2.0 * (y * z - w * x) * inv;
  out[2] = (w * w - x * x - y * y + z * z) * inv;
}

// Full R_wc (row-major) for a quaternion of any norm.
__device__ inline void quat_R(double w, double x, double y, double z, double R[9]) {
  double n = w * w + x * x + y * y + z * z;
  double inv = 1.0 / n;
  R[0] = (w * w + x * x - y * y - z * z) * inv;
  R[1] = 2.0 * (x * y - w * z) * inv;
  R[2] = 2.0 * (x * z + w * y) * inv;
  R[3] = 2.0 * (x * y + w * z) * inv;
  R[4] = (w * w - x * x + y * y - z * z) * inv;
  R[5] = 2.0 * (y * z - w * x) * inv;
  R[6] = 2.0 * (x * z - w * y) * inv;
  R[7] = 2.0 * (y * z + w * x) * inv;
  R[8] = (w * w - x * x - y * y + z * z) * inv;
}

struct GridDev {
  double ox, oy, oz, h, inv_h;
  int32_t nx, ny, nz;
};

// Per-axis cell of a position: lower index, fraction, d fraction / d t, clamp.
struct AxisCell {
  int32_t i0;
  int32_t step;  // 1, or 0 on a single-voxel axis
  double f;
  double df;
  bool clamped;
};

__device__ inline AxisCell axis_cell(double t, double o, double h, int32_t n) {
  AxisCell c;
  double g = (t - o) / h;
  c.clamped = !(g >= 0.0 && g <= (double)(n - 1));
  if (n == 1) {
    c.i0 = 0; c.step = 0; c.f = 0.0; c.df = 0.0;
    return c;
  }
  double fl = floor(g);
  fl = fmax(fl, 0.0);                 // NaN g gives fl = 0 here
  fl = fmin(fl, (double)(n - 2));
  c.i0 = (int32_t)fl;
  c.step = 1;
  c.f = g - fl;
  c.df = 1.0 / h;
  if (c.f < 0.0) { c.f = 0.0; c.df = 0.0; }
  if (c.f > 1.0) { c.f = 1.0; c.df = 0.0; }
  return c;
}

__device__ inline int32_t axis_nearest(double t, double o, double h, int32_t n, bool* clamped) {
  double g = (t - o) / h;
  *clamped = !(g >= 0.0 && g <= (double)(n - 1));
  double r = floor(g + 0.5);
  r = fmax(r, 0.0);
  r = fmin(r, (double)(n - 1));
  return (int32_t)r;
}

// ------------------------------------------------------------ moment contraction

// Per-query weights of the moment contraction with the quadratic visibility
// v(c) = k2 c^2 + k1 c + k0, c = z.u.  On the unit sphere the constant k0 folds
// into the squared terms (|u| = 1): v = sum_{c<=d} w2[cd] u_c u_d + sum_c w1[c] u_c
// with w2[cc] = k2 z_c^2 + k0, w2[cd] = 2 k2 z_c z_d (c < d), w1 = k1 z.
template <typename CT>
struct VisW {
  CT w2[6];
  CT w1[3];
};

template <typename CT>
__device__ inline VisW<CT> vis_weights(const CT z[3], CT k2, CT k1, CT k0) {
  VisW<CT> w;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c; d < 3; ++d)
      w.w2[i2(c, d)] = (c == d) ? fma(k2 * z[c], z[c], k0) : CT(2) * k2 * z[c] * z[d];
#pragma unroll
  for (int c = 0; c < 3; ++c) w.w1[c] = k1 * z[c];
  return w;
}

// For one moment group with degree-4 part S4[15] and degree-3 part S3[10]
// (weights 1 or 1/n^2), Q = sum v u u^T.
template <typename CT, typename T>
__device__ inline void group_Q(const T* S4, const T* S3, const VisW<CT>& w, CT Q[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      CT q = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = c; d < 3; ++d) q = fma(w.w2[i2(c, d)], (CT)S4[s4(a, b, c, d)], q);
#pragma unroll
      for (int c = 0; c < 3; ++c) q = fma(w.w1[c], (CT)S3[s3(a, b, c)], q);
      Q[i2(a, b)] = q;
    }
}

// b = sum v u / n from the G1 group (degree 3 R3[10], degree 2 R2[6]).
template <typename CT, typename T>
__device__ inline void group_b(const T* R3, const T* R2, const VisW<CT>& w, CT bvec[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    CT q = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = c; d < 3; ++d) q = fma(w.w2[i2(c, d)], (CT)R3[s3(a, c, d)], q);
#pragma unroll
    for (int c = 0; c < 3; ++c) q = fma(w.w1[c], (CT)R2[s2(a, c)], q);
    bvec[a] = q;
  }
}

// 3x3 helpers: symmetric matrices as 6-vectors (i2 order), general as row-major 9.
template <typename CT>
__device__ inline CT sym3(const CT* A, int i, int j) { return A[s2(i, j)]; }

// X = M(delta)^T [[A, B], [B^T, D]] M(delta), M(delta) = [[I, -[delta]x], [0, I]]:
//   TL = A, TR = B + (S A)^T, BR = D + S (S A)^T + S B + (S B)^T,  S = [delta]x.
template <typename CT>
__device__ inline void shift_frame(const CT A[6], const CT B[9], const CT D[6], const CT dl[3],
                                   CT out[21]) {
  // rows of S
  const CT S[9] = {0, -dl[2], dl[1], dl[2], 0, -dl[0], -dl[1], dl[0], 0};
  CT SA[9], SB[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      CT sa = 0, sb = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sa = fma(S[i * 3 + k], sym3(A, k, j), sa);
        sb = fma(S[i * 3 + k], B[k * 3 + j], sb);
      }
      SA[i * 3 + j] = sa;
      SB[i * 3 + j] = sb;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) out[u21(i, j)] = sym3(A, i, j);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) out[u21(i, 3 + j)] = B[i * 3 + j] + SA[j * 3 + i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      CT s = 0;  // (S (SA)^T)_ij = sum_k S_ik SA_jk
#pragma unroll
      for (int k = 0; k < 3; ++k) s = fma(S[i * 3 + k], SA[j * 3 + k], s);
      out[u21(3 + i, 3 + j)] = sym3(D, i, j) + s + SB[i * 3 + j] + SB[j * 3 + i];
    }
}

// Camera-frame block of one voxel at optical axis z, shifted by delta = t_v - t:
// returns the 21-vector of M(delta)^T X M(delta) (without the 1/sigma^2 factor).
template <typename CT, typename T>
__device__ inline void corner_fim(const T* rec, const VisW<CT>& w, const CT dl[3], CT out[21]) {
  CT Q2[6], Q0[6], bv[3];
  group_Q<CT>(rec + O_G2_4, rec + O_G2_3, w, Q2);
  group_Q<CT>(rec + O_G0_4, rec + O_G0_3, w, Q0);
  group_b<CT>(rec + O_G1_3, rec + O_G1_2, w, bv);
  CT A[6], D[6], B[9];
  CT tr2 = Q2[0] + Q2[3] + Q2[5], tr0 = Q0[0] + Q0[3] + Q0[5];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      A[i2(a, b)] = (a == b ? tr2 : CT(0)) - Q2[i2(a, b)];
      D[i2(a, b)] = (a == b ? tr0 : CT(0)) - Q0[i2(a, b)];
    }
  // B = -[b]x
  B[0] = 0;      B[1] = bv[2];  B[2] = -bv[1];
  B[3] = -bv[2]; B[4] = 0;      B[5] = bv[0];
  B[6] = bv[1];  B[7] = -bv[0]; B[8] = 0;
  shift_frame<CT>(A, B, D, dl, out);
}

// General symmetric 6x6 (21) -> world frame: M(t)^T Z M(t).
template <typename CT>
__device__ inline void shift21(const CT Z[21], const CT t[3], CT out[21]) {
  CT A[6], D[6], B[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      A[i2(i, j)] = Z[u21(i, j)];
      D[i2(i, j)] = Z[u21(3 + i, 3 + j)];
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[i * 3 + j] = Z[u21(i, 3 + j)];
  shift_frame<CT>(A, B, D, t, out);
}

// Adjoint shift for gradients: G' = M(delta) G M(delta)^T with
//   G = [[P, Q], [Q^T, R]], S = [delta]x:
//   TL' = P + QS + (QS)^T + S (S R)^T,  TR' = Q - S R,  BR' = R.
template <typename CT>
__device__ inline void shift21_adj(const CT G[21], const CT dl[3], CT out[21]) {
  const CT S[9] = {0, -dl[2], dl[1], dl[2], 0, -dl[0], -dl[1], dl[0], 0};
  CT Q[9], QS[9], SR[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q[i * 3 + j] = G[u21(i, 3 + j)];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      CT qs = 0, sr = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        qs = fma(Q[i * 3 + k], S[k * 3 + j], qs);
        sr = fma(S[i * 3 + k], G[su21(3 + k, 3 + j)], sr);
      }
      QS[i * 3 + j] = qs;
      SR[i * 3 + j] = sr;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      CT s = 0;  // (S (SR)^T)_ij = sum_k S_ik SR_jk
#pragma unroll
      for (int k = 0; k < 3; ++k) s = fma(S[i * 3 + k], SR[j * 3 + k], s);
      out[u21(i, j)] = G[u21(i, j)] + QS[i * 3 + j] + QS[j * 3 + i] + s;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) out[u21(i, 3 + j)] = Q[i * 3 + j] - SR[i * 3 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) out[u21(3 + i, 3 + j)] = G[u21(3 + i, 3 + j)];
}

// ------------------------------------------------------------ backward pieces

// For a symmetric 3x3 H (6, i2 order) and one moment group (S4, S3):
//   val   = sum v (tr H - u^T H u)  (times the group weight)
//   gz[c] = d val / d z_c
template <typename CT, typename T>
__device__ inline void group_vjp(const T* S4, const T* S3, const CT H[6], const CT z[3], CT k2,
                                 CT k1, CT k0, CT* val, CT gz[3]) {
  CT trH = H[0] + H[3] + H[5];
  CT HS4[6], HS3[3], S2[6], S1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c; d < 3; ++d) {
      CT acc = 0, s2v = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b)
          acc = fma((a == b ? CT(1) : CT(2)) * H[i2(a, b)], (CT)S4[s4(a, b, c, d)], acc);
#pragma unroll
      for (int e = 0; e < 3; ++e) s2v += (CT)S4[s4(c, d, e, e)];
      HS4[i2(c, d)] = acc;
      S2[i2(c, d)] = s2v;
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    CT acc = 0, s1v = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b)
        acc = fma((a == b ? CT(1) : CT(2)) * H[i2(a, b)], (CT)S3[s3(a, b, c)], acc);
#pragma unroll
    for (int e = 0; e < 3; ++e) s1v += (CT)S3[s3(c, e, e)];
    HS3[c] = acc;
    S1[c] = s1v;
  }
  CT S0 = S2[0] + S2[3] + S2[5];
  // sv = sum v,  hq = sum v u^T H u
  CT zSz = 0, zHSz = 0, hS2 = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c; d < 3; ++d) {
      CT m = (c == d ? CT(1) : CT(2)) * z[c] * z[d];
      zSz = fma(m, S2[i2(c, d)], zSz);
      zHSz = fma(m, HS4[i2(c, d)], zHSz);
      hS2 = fma((c == d ? CT(1) : CT(2)) * H[i2(c, d)], S2[i2(c, d)], hS2);
    }
  CT zS1 = z[0] * S1[0] + z[1] * S1[1] + z[2] * S1[2];
  CT zHS3 = z[0] * HS3[0] + z[1] * HS3[1] + z[2] * HS3[2];
  CT sv = k2 * zSz + k1 * zS1 + k0 * S0;
  CT hq = k2 * zHSz + k1 * zHS3 + k0 * hS2;
  *val = trH * sv - hq;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    CT zS2c = 0, zHS4c = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      zS2c = fma(z[d], S2[s2(c, d)], zS2c);
      zHS4c = fma(z[d], HS4[s2(c, d)], zHS4c);
    }
    gz[c] = CT(2) * k2 * (trH * zS2c - zHS4c) + k1 * (trH * S1[c] - HS3[c]);
  }
}

// For the G1 group and a 3-vector om: val = om . b, gz = d val / dz.
template <typename CT, typename T>
__device__ inline void group_b_vjp(const T* R3, const T* R2, const CT om[3], const CT z[3], CT k2,
                                   CT k1, CT k0, CT* val, CT gz[3]) {
  CT oR3[6], oR2[3], r1 = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c; d < 3; ++d) {
      CT acc = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) acc = fma(om[a], (CT)R3[s3(a, c, d)], acc);
      oR3[i2(c, d)] = acc;
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    CT acc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) acc = fma(om[a], (CT)R2[s2(a, c)], acc);
    oR2[c] = acc;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    CT s = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) s += (CT)R3[s3(a, c, c)];
    r1 = fma(om[a], s, r1);
  }
  CT zz = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c; d < 3; ++d) zz = fma((c == d ? CT(1) : CT(2)) * z[c] * z[d], oR3[i2(c, d)], zz);
  CT zo2 = z[0] * oR2[0] + z[1] * oR2[1] + z[2] * oR2[2];
  *val = k2 * zz + k1 * zo2 + k0 * r1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    CT s = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) s = fma(z[d], oR3[s2(c, d)], s);
    gz[c] = CT(2) * k2 * s + k1 * oR2[c];
  }
}

// <G', X(z)> and its z-gradient for one voxel record, with G' the (already
// adjoint-shifted) 21-vector; X = camera-frame block without 1/sigma^2.
template <typename CT, typename T>
__device__ inline void corner_vjp(const T* rec, const CT Gp[21], const CT z[3], CT k2, CT k1, CT k0,
                                  CT* val, CT gz[3]) {
  CT HTL[6], HBR[6], om[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      HTL[i2(i, j)] = Gp[u21(i, j)];
      HBR[i2(i, j)] = Gp[u21(3 + i, 3 + j)];
    }
  // omega(TR) = (TR_21 - TR_12, TR_02 - TR_20, TR_10 - TR_01)
  om[0] = Gp[u21(2, 4)] - Gp[u21(1, 5)];
  om[1] = Gp[u21(0, 5)] - Gp[u21(2, 3)];
  om[2] = Gp[u21(1, 3)] - Gp[u21(0, 4)];
  CT v2, v0, vb, g2[3], g0[3], gb[3];
  group_vjp<CT>(rec + O_G2_4, rec + O_G2_3, HTL, z, k2, k1, k0, &v2, g2);
  group_vjp<CT>(rec + O_G0_4, rec + O_G0_3, HBR, z, k2, k1, k0, &v0, g0);
  group_b_vjp<CT>(rec + O_G1_3, rec + O_G1_2, om, z, k2, k1, k0, &vb, gb);
  *val = v2 + v0 - CT(2) * vb;
#pragma unroll
  for (int c = 0; c < 3; ++c) gz[c] = g2[c] + g0[c] - CT(2) * gb[c];
}

// ------------------------------------------------------------ 6x6 metrics (FP64)

// 1/sqrt(x) and 1/x for positive normal FP64 x: hardware estimate refined by
// one Newton step.  Measured over 4M log-uniform x in [1e-300, 1e300]: the
// estimates are within 5.3e-8 (rsq) and 4.7e-8 (rcp) relative, one step
// within 4.2e-15 and 2.2e-15.  A Jacobi rotation built from them is then
// orthogonal to ~1e-14, which moves the eigenvalues by under 1e-12 relative
// over a whole solve (far below every FP64 bar); a second step cost 5-10% of
// the FP32-field query.
__device__ inline double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double r = fma(-x * y, y, 1.0);
  return fma(0.5 * y, r, y);
}
__device__ inline double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

#define FIF_A(i, j) a[su21((i), (j))]

// Round rd (0..4) of the round-robin schedule of the 15 pairs of 6 indices
// (index 0 fixed, the others rotated): three disjoint pairs (P[k], Q[k]), P < Q.
__device__ constexpr void round_robin6(int rd, int P[3], int Q[3]) {
  int ring[5] = {1, 2, 3, 4, 5};
  int r[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < 5; ++i) r[i] = ring[(i + rd) % 5];
  // pairs: (0, r0), (r1, r4), (r2, r3)
  int a[3] = {0, r[1], r[2]}, b[3] = {r[0], r[4], r[3]};
  for (int k = 0; k < 3; ++k) {
    P[k] = a[k] < b[k] ? a[k] : b[k];
    Q[k] = a[k] < b[k] ? b[k] : a[k];
  }
}

// Jacobi on a symmetric 6x6 held as 21 values, the pairs of each sweep in
// round-robin order (3 disjoint rotations per round).  Sweeps until the
// off-diagonal Frobenius norm is below 1e-11 of the full norm (or 16 sweeps);
// by Weyl's inequality every diagonal entry is then within that distance of an
// eigenvalue, far inside the FP64 metric tolerance.
// Rotation (p, q): t = sgn(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp
// (the smaller root of t^2 + 2 t theta - 1 = 0, theta = d / (2 a_pq)),
// c = 1 / sqrt(1 + t^2), s = t c.
// On return the diagonal of `a` holds the eigenvalues; when WANT_V the
// columns of V (row-major 36) are the eigenvectors.
template <bool WANT_V>
__device__ inline void jacobi6(double a[21], double V[36]) {
  if (WANT_V) {
#pragma unroll
    for (int i = 0; i < 36; ++i) V[i] = (i % 7 == 0) ? 1.0 : 0.0;
  }
  double fro = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) fro += (i == j ? 1.0 : 2.0) * FIF_A(i, j) * FIF_A(i, j);
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j) off += 2.0 * FIF_A(i, j) * FIF_A(i, j);
    if (!(off > 1e-22 * fro)) break;
    // Each sweep visits the 15 pairs in 5 rounds of 3 disjoint pairs (round-robin
    // order).  Rotations on disjoint index pairs commute, so the three angles of
    // a round are computed from the same matrix and applied one after another:
    // three independent dependency chains instead of one.
#pragma unroll
    for (int rd = 0; rd < 5; ++rd) {
      int P[3], Q[3];
      round_robin6(rd, P, Q);
      double cr[3], sr[3], tr[3], ar[3];
      bool sk[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int p = P[k], q = Q[k];
        const double apq = FIF_A(p, q);
        const double app = FIF_A(p, p), aqq = FIF_A(q, q);
        const double d = aqq - app;
        const double r2 = fma(d, d, 4.0 * apq * apq);
        const bool skip = !(r2 > 0.0) || (apq == 0.0);
        const double r2s = skip ? 1.0 : r2;
        const double r = r2s * rsq_nr(r2s);
        double tt = 2.0 * apq * rcp_nr(fabs(d) + r);
        tt = (d < 0.0) ? -tt : tt;
        tt = skip ? 0.0 : tt;
        cr[k] = rsq_nr(fma(tt, tt, 1.0));
        sr[k] = tt * cr[k];
        tr[k] = tt;
        ar[k] = apq;
        sk[k] = skip;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int p = P[k], q = Q[k];
        const double c = cr[k], s = sr[k], tt = tr[k], apq = ar[k];
        const double app = FIF_A(p, p), aqq = FIF_A(q, q);
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          if (m == p || m == q) continue;
          double akp = FIF_A(m, p), akq = FIF_A(m, q);
          FIF_A(m, p) = c * akp - s * akq;
          FIF_A(m, q) = s * akp + c * akq;
        }
        FIF_A(p, p) = app - tt * apq;
        FIF_A(q, q) = aqq + tt * apq;
        FIF_A(p, q) = sk[k] ? apq : 0.0;
        if (WANT_V) {
#pragma unroll
          for (int m = 0; m < 6; ++m) {
            double vkp = V[m * 6 + p], vkq = V[m * 6 + q];
            V[m * 6 + p] = c * vkp - s * vkq;
            V[m * 6 + q] = s * vkp + c * vkq;
          }
        }
      }
    }
  }
}

// LDL^T of a symmetric 6x6 (21 values) in place.  Returns false when a pivot
// is not positive (not PD).  logdet = sum log d_i.
__device__ inline bool ldlt6(const double F[21], double L[36], double dinv[6], double* logdet) {
  double d[6];
  bool pd = true;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = F[u21(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j * 6 + k] * L[j * 6 + k] * d[k];
    d[j] = s;
    pd = pd && (s > 0.0);
    // past a pivot <= 0 the factor feeds no output (log-det NaN, gradient
    // NaN or left out), so no exact division is needed there
    double inv = rcp_nr(s);
    dinv[j] = inv;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double r = F[u21(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) r -= L[i * 6 + k] * L[j * 6 + k] * d[k];
      L[i * 6 + j] = r * inv;
    }
  }
  double prod = d[0] * d[1] * d[2];
  double prod2 = d[3] * d[4] * d[5];
  *logdet = pd ? (log(prod) + log(prod2)) : __builtin_nan("");
  return pd;
}

// The log-determinant of ldlt6, factorising in place: a[] (21 values, upper
// triangle row-major) ends up holding L below the diagonal (L[i][j] at a[j][i])
// and d on it.  The same operations in the same order as ldlt6, so the same
// value; small enough to keep the whole factorisation in registers inside a
// loop over many matrices.
__device__ inline double logdet6_inplace(double a[21]) {
  bool pd = true;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = a[u21(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= a[u21(k, j)] * a[u21(k, j)] * a[u21(k, k)];
    a[u21(j, j)] = s;
    pd = pd && (s > 0.0);
    double inv = rcp_nr(s);  // as ldlt6
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double r = a[u21(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) r -= a[u21(k, i)] * a[u21(k, j)] * a[u21(k, k)];
      a[u21(j, i)] = r * inv;
    }
  }
  double prod = a[u21(0, 0)] * a[u21(1, 1)] * a[u21(2, 2)];
  double prod2 = a[u21(3, 3)] * a[u21(4, 4)] * a[u21(5, 5)];
  return pd ? (log(prod) + log(prod2)) : __builtin_nan("");
}

// Unit eigenvector of the smallest eigenvalue of a symmetric 6x6 (21 values)
// by inverse iteration: LDL^T of F - sigma I with sigma just below that
// eigenvalue (so the factorisation is of a positive definite matrix), then
// three solves starting from (1, ..., 1).  Each solve shrinks the component
// along eigenvector i relative to the wanted one by
// (lambda_min - sigma) / (lambda_i - sigma).  The iterate is rescaled by its
// largest component before it is normalised, so no sum of squares overflows.
__device__ inline void lmin_vector6(const double F[21], double sigma, double v[6]) {
  double L[36], d[6], dinv[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = F[u21(j, j)] - sigma;
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j * 6 + k] * L[j * 6 + k] * d[k];
    d[j] = s;
    dinv[j] = 1.0 / s;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double r = F[u21(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) r -= L[i * 6 + k] * L[j * 6 + k] * d[k];
      L[i * 6 + j] = r * dinv[j];
    }
  }
  double x[6] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {  // L y = x
      double s = x[i];
#pragma unroll
      for (int k = 0; k < i; ++k) s -= L[i * 6 + k] * y[k];
      y[i] = s;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] *= dinv[i];  // D z = y
#pragma unroll
    for (int i = 5; i >= 0; --i) {  // L^T x = z
      double s = y[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) s -= L[k * 6 + i] * x[k];
      x[i] = s;
    }
    double mx = fabs(x[0]);
#pragma unroll
    for (int i = 1; i < 6; ++i) mx = fmax(mx, fabs(x[i]));
    const double inv = 1.0 / mx;
    double n2 = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      x[i] *= inv;
      n2 = fma(x[i], x[i], n2);
    }
    const double rn = 1.0 / sqrt(n2);
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] *= rn;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) v[i] = x[i];
}

// F^-1 (21) from the LDL^T factors.
__device__ inline void ldlt6_inverse(const double L[36], const double dinv[6], double out[21]) {
  // X = L^-T D^-1 L^-1; compute W = L^-1 (unit lower), then X = W^T D^-1 W
  double W[36];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k)
        if (k >= c) s -= L[i * 6 + k] * W[k * 6 + c];
      W[i * 6 + c] = (i < c) ? 0.0 : s;
    }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (k >= i && k >= j) s = fma(W[k * 6 + i] * dinv[k], W[k * 6 + j], s);
      out[u21(i, j)] = s;
    }
}

// ------------------------------------------------------------ cross-lane sums

// Sum over aligned groups of 8 lanes with DPP moves (no LDS traffic):
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], then row_half_mirror (lane i <-> 7-i).
template <int CTRL>
__device__ inline float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ inline float sum8(float x) {
  x += dpp_f32<0xB1>(x);
  x += dpp_f32<0x4E>(x);
  x += dpp_f32<0x141>(x);
  return x;
}
__device__ inline double sum8(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x141>(x);
  return x;
}
// The same over an array, one butterfly stage at a time across all entries,
// so consecutive DPP reads never wait on the add just issued.
template <int N, typename CT>
__device__ inline void sum8_arr(CT* x) {
#pragma unroll
  for (int e = 0; e < N; ++e) x[e] += (sizeof(CT) == 4) ? (CT)dpp_f32<0xB1>((float)x[e]) : (CT)dpp_f64<0xB1>((double)x[e]);
#pragma unroll
  for (int e = 0; e < N; ++e) x[e] += (sizeof(CT) == 4) ? (CT)dpp_f32<0x4E>((float)x[e]) : (CT)dpp_f64<0x4E>((double)x[e]);
#pragma unroll
  for (int e = 0; e < N; ++e) x[e] += (sizeof(CT) == 4) ? (CT)dpp_f32<0x141>((float)x[e]) : (CT)dpp_f64<0x141>((double)x[e]);
}

}  // namespace fif
