// GP visibility fields (Sec. V-B "GP Regression"; G-I-N_s and G-T-N_s).
//
// Model setup: (K^s + noise I)^-1 by an FP64 Cholesky factor held in LDS (one
// workgroup); the evidence of candidate length scales likewise.
//
// Build: for every voxel, S_g = sum_i v^s_g(u_i) X_i over the landmarks in
// range, X_i the camera-frame terms of I_i about the voxel centre (P/n^2, u/n,
// P with P = I - u u^T; information fields) or Tr(I_i) (trace fields).  Per
// voxel this is a (sample axes x landmarks) . (landmarks x terms) product whose
// operands are formed on the fly, so one wave owns one voxel and feeds the
// matrix cores: per group of 4 landmarks in range, each 16-axis tile is one
// 16x16x4 MFMA with the sigmoid visibilities as A and the 15 terms as B.  The
// landmarks in range of a batch are first compacted into the wave's LDS list.
//
// Query: the GP weights w = (K^s + noise I)^-1 K_z of the pose are formed once
// (FP64), each corner block is contracted with w, moved to the query frame and
// interpolated; the FP64 world shift and metrics follow per query.
#include <cmath>
#include <type_traits>

#include "fif_kernels.h"
#include "fif_metrics.h"
#include "fif_slot.h"

namespace fif {

namespace {

constexpr int kGPThreads = 256;
constexpr int kGPWaves = kGPThreads / 64;
constexpr int kGPBatch = 256;
constexpr int kGPTiles = 5;  // 16-axis tiles per pass (80 axes)
constexpr int kMaxNs = 160;  // FIF_GP_MAX_NS
constexpr int kPackedL = kMaxNs * (kMaxNs + 1) / 2;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec4;
template <>
struct Vec4<float> { using acc = f32x4; using lm = float4; };
template <>
struct Vec4<double> { using acc = f64x4; using lm = double4; };

// D += A B for A 16x4 (lane l: A[l%16][l/16]), B 4x16 (lane l: B[l/16][l%16]),
// D 16x16 (lane l, element r: D[4(l/16) + r][l%16]).  FP32: the matrix core.
__device__ inline f32x4 mma16(float a, float b, f32x4 c, double*) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// FP64: the same product through LDS (the FP64 path is the precision
// reference), with the same operand and result layout.
__device__ inline f64x4 mma16(double a, double b, f64x4 c, double* s) {
  const int l = threadIdx.x & 63;
  s[l] = a;
  s[64 + l] = b;
  wave_sync();
  const int j = l & 15, i0 = 4 * (l >> 4);
  double bk[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) bk[k] = s[64 + 16 * k + j];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) c[r] = fma(s[i0 + r + 16 * k], bk[k], c[r]);
  wave_sync();
  return c;
}

// Sigmoid visibility (eq:sigmoid_vis_func).
__device__ inline double sigmoid_vis(double c, double ks, double cos_a) {
  return 1.0 / (1.0 + exp(-ks * (c - cos_a)));
}

// The same from a prepared exponent: e = 2^x (FP32) or e^x (FP64) with
// x = -k_s (z . u - cos alpha) already formed; 1 / (1 + e).  An exponent of
// +1e4 gives exactly 0 (the padding axes of a tile).
__device__ inline float sigmoid_from(float x) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(x));
}
__device__ inline double sigmoid_from(double x) { return 1.0 / (1.0 + exp(x)); }

__device__ inline void two_sum_acc(float& hi, float& lo, float x) {
  float s = hi + x;
  float bb = s - hi;
  float err = (hi - (s - bb)) + (x - bb);
  hi = s;
  lo += err;
}

// Packed lower-triangular index of (i, j), j <= i.
__device__ inline int tri(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ inline double se_kernel(const double* za, const double* zb, double inv_2l2) {
  const double d0 = za[0] - zb[0], d1 = za[1] - zb[1], d2 = za[2] - zb[2];
  return exp(-(d0 * d0 + d1 * d1 + d2 * d2) * inv_2l2);
}

// Cholesky factor of K^s + noise I (packed, in LDS) by the workgroup.  The
// axes are in s_z[ns][3].  Returns false (uniformly) if not positive definite.
__device__ bool cholesky_lds(int ns, const double* s_z, double inv_2l2, double noise,
                             double* L, double* s_diag) {
  const int tid = threadIdx.x;
  bool ok = true;
  for (int j = 0; j < ns; ++j) {
    if (tid == 0) {
      double d = se_kernel(s_z + 3 * j, s_z + 3 * j, inv_2l2) + noise;
      for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
      *s_diag = (d > 0.0) ? sqrt(d) : __builtin_nan("");
      L[tri(j, j)] = *s_diag;
    }
    __syncthreads();
    const double ljj = *s_diag;
    ok = ok && (ljj > 0.0);
    for (int i = j + 1 + tid; i < ns; i += blockDim.x) {
      double v = se_kernel(s_z + 3 * i, s_z + 3 * j, inv_2l2);
      for (int k = 0; k < j; ++k) v -= L[tri(i, k)] * L[tri(j, k)];
      L[tri(i, j)] = v / ljj;
    }
    __syncthreads();
  }
  return ok;
}

__global__ __launch_bounds__(256) void gp_setup_kernel(GPDev gp, double* kinv) {
  __shared__ double s_L[kPackedL];
  __shared__ double s_z[3 * kMaxNs];
  __shared__ double s_diag;
  const int ns = gp.ns, tid = threadIdx.x;
  for (int i = tid; i < 3 * ns; i += blockDim.x) s_z[i] = gp.axes[i];
  __syncthreads();
  const bool ok = cholesky_lds(ns, s_z, gp.inv_2l2, gp.noise, s_L, &s_diag);
  // column c of the inverse: L y = e_c, then L^T x = y (x overwrites y in
  // column c of kinv, which only this thread touches)
  for (int c = tid; c < ns; c += blockDim.x) {
    for (int i = 0; i < ns; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= s_L[tri(i, k)] * kinv[(size_t)k * ns + c];
      kinv[(size_t)i * ns + c] = (i < c) ? 0.0 : s / s_L[tri(i, i)];
    }
    for (int i = ns - 1; i >= 0; --i) {
      double s = kinv[(size_t)i * ns + c];
      for (int k = i + 1; k < ns; ++k) s -= s_L[tri(k, i)] * kinv[(size_t)k * ns + c];
      kinv[(size_t)i * ns + c] = ok ? s / s_L[tri(i, i)] : __builtin_nan("");
    }
  }
}

// One workgroup per candidate length.  The quadratic terms solve L w = y_t in
// LDS columns: as many solver threads as the remaining LDS holds.
constexpr int kEvidenceW = 5120;  // doubles of solver scratch

__global__ __launch_bounds__(256) void gp_evidence_kernel(GPDev gp, const double* train_u,
                                                          int n_train, const double* lengths,
                                                          double* lml) {
  __shared__ double s_L[kPackedL];
  __shared__ double s_z[3 * kMaxNs];
  __shared__ double s_w[kEvidenceW];
  __shared__ double s_red[256];
  __shared__ double s_diag;
  const int ns = gp.ns, tid = threadIdx.x;
  const double l = lengths[blockIdx.x];
  const double inv_2l2 = 1.0 / (2.0 * l * l);
  for (int i = tid; i < 3 * ns; i += blockDim.x) s_z[i] = gp.axes[i];
  __syncthreads();
  const bool ok = (l > 0.0) && cholesky_lds(ns, s_z, inv_2l2, gp.noise, s_L, &s_diag);
  const int nsolve = min((int)blockDim.x, kEvidenceW / ns);
  double quad = 0.0;
  if (ok && tid < nsolve) {
    double* w = s_w + tid;  // column tid, stride nsolve
    for (int t = tid; t < n_train; t += nsolve) {
      const double* u = train_u + 3 * t;
      double q = 0.0;
      for (int i = 0; i < ns; ++i) {
        const double* zi = s_z + 3 * i;
        double s = sigmoid_vis(zi[0] * u[0] + zi[1] * u[1] + zi[2] * u[2], gp.ks, gp.cos_a);
        for (int k = 0; k < i; ++k) s -= s_L[tri(i, k)] * w[k * nsolve];
        s /= s_L[tri(i, i)];
        w[i * nsolve] = s;
        q = fma(s, s, q);
      }
      quad += q;
    }
  }
  s_red[tid] = quad;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) s_red[tid] += s_red[tid + st];
    __syncthreads();
  }
  if (tid == 0) {
    double logdet = 0.0;
    for (int i = 0; i < ns; ++i) logdet += 2.0 * log(s_L[tri(i, i)]);
    lml[blockIdx.x] = ok ? -0.5 * s_red[0] - 0.5 * n_train * logdet -
                               0.5 * (double)n_train * ns * log(2.0 * M_PI)
                         : -__builtin_inf();
  }
}

// ---------------------------------------------------------------- build

// Per-lane term of the B operand: f = lane % 16 selects
//   0..5  (delta_ab - u_a u_b) / n^2   (i2 order 00 01 02 11 12 22)
//   6..8  u_a / n
//   9..14 delta_ab - u_a u_b
//   15    0
// as  m_pn2 (delta - u_a u_b) / n^2 + m_un u_a / n + m_p (delta - u_a u_b).
struct TermSel {
  int ia, ib;
  float delta, m_pn2, m_un, m_p;
  float a[3], b[3];  // one-hot weights selecting u_a and u_b
};

__device__ inline TermSel term_sel(int f) {
  TermSel t;
  const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
  t.m_pn2 = t.m_un = t.m_p = 0.f;
  if (f < 6) {
    t.ia = pa[f]; t.ib = pb[f]; t.m_pn2 = 1.f;
  } else if (f < 9) {
    t.ia = f - 6; t.ib = 0; t.m_un = 1.f;
  } else if (f < 15) {
    t.ia = pa[f - 9]; t.ib = pb[f - 9]; t.m_p = 1.f;
  } else {
    t.ia = 0; t.ib = 0;
  }
  t.delta = (t.ia == t.ib && f != 15 && !(f >= 6 && f < 9)) ? 1.f : 0.f;
  for (int c = 0; c < 3; ++c) {
    t.a[c] = (c == t.ia) ? 1.f : 0.f;
    t.b[c] = (c == t.ib) ? 1.f : 0.f;
  }
  return t;
}

template <int PREC, int KIND, int NT>
__global__ __launch_bounds__(kGPThreads) void gp_build_kernel(GPBuildArgs a, int pass0) {
  using T = typename std::conditional<PREC == 2, double, float>::type;
  using A4 = typename Vec4<T>::acc;
  using R4 = typename Vec4<T>::lm;
  constexpr bool COMP = (PREC == 1);
  __shared__ R4 s_rec[kGPWaves][kGPBatch];
  __shared__ double s_mm[kGPWaves][PREC == 2 ? 128 : 1];

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ns = a.gp.ns;
  const int g0 = (pass0 + (int)blockIdx.y) * 16 * kGPTiles;
  // A operand axes of this lane, per tile
  // exponent of the sigmoid as K (z . u) + x0 with K = -k_s (times log2 e in
  // FP32, where the exponential is base 2), folded into the axis components
  const double kexp = (PREC == 2) ? -a.gp.ks : -a.gp.ks * 1.4426950408889634;
  T zx[NT], zy[NT], zz[NT], z0[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int g = g0 + 16 * t + (lane & 15);
    const bool ok = g < ns;
    zx[t] = ok ? (T)(kexp * a.gp.axes[3 * g]) : T(0);
    zy[t] = ok ? (T)(kexp * a.gp.axes[3 * g + 1]) : T(0);
    zz[t] = ok ? (T)(kexp * a.gp.axes[3 * g + 2]) : T(0);
    z0[t] = ok ? (T)(-kexp * a.gp.cos_a) : T(1e4);
  }
  const TermSel sel = term_sel(lane & 15);
  const size_t nvox = (size_t)a.g.nx * a.g.ny * a.g.nz;
  const int64_t gw = (int64_t)blockIdx.x * kGPWaves + wv;
  const int64_t nw = (int64_t)gridDim.x * kGPWaves;

  for (int64_t v = gw; v < (int64_t)nvox; v += nw) {
    const int64_t ix = v % a.g.nx, iy = (v / a.g.nx) % a.g.ny, iz = v / ((int64_t)a.g.nx * a.g.ny);
    const double tx = a.g.ox + (double)ix * a.g.h, ty = a.g.oy + (double)iy * a.g.h,
                 tz = a.g.oz + (double)iz * a.g.h;
    const float fx = (float)tx, fy = (float)ty, fz = (float)tz;
    A4 acc[NT];
    float hi[COMP ? NT : 1][4], lo[COMP ? NT : 1][4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[t] = A4{0, 0, 0, 0};
      if (COMP) {
#pragma unroll
        for (int r = 0; r < 4; ++r) { hi[t][r] = 0.f; lo[t][r] = 0.f; }
      }
    }
    for (int64_t base = 0; base < a.L; base += kGPBatch) {
      const int nb = (int)((a.L - base) < kGPBatch ? (a.L - base) : kGPBatch);
      if (a.lm_sorted) {
        // skip a batch whose box is out of range of this voxel (wave-uniform)
        const float* bb = a.batch_box + 8 * (base / kGPBatch);
        const float pv[3] = {fx, fy, fz};
        float d2 = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float gap = fmaxf(fmaxf(bb[c] - pv[c], pv[c] - bb[3 + c]), 0.f);
          d2 = fmaf(gap, gap, d2);
        }
        if (d2 > a.skip2) continue;
      }
      // compact the landmarks in range into this wave's list
      int cnt = 0;
#pragma unroll
      for (int s = 0; s < kGPBatch / 64; ++s) {
        const int k = s * 64 + lane;
        bool in = false;
        R4 rec;
        if (k < nb) {
          double px, py, pz;
          if (a.lm_sorted) {
            const double4 p4 = a.lm_sorted[base + k];
            px = p4.x; py = p4.y; pz = p4.z;
          } else {
            const double* p = a.lm + 3 * (base + k);
            px = p[0]; py = p[1]; pz = p[2];
          }
          // V_t range test in FP32 (same decision in every precision)
          const float ddx = (float)px - fx, ddy = (float)py - fy, ddz = (float)pz - fz;
          const float n2 = __fmaf_rn(ddz, ddz, __fmaf_rn(ddy, ddy, ddx * ddx));
          in = (n2 >= a.lo2) && (n2 <= a.hi2);
          if (in) {
            // the offset from the FP64 coordinates: the FP32-rounded ones are
            // off by up to ~6e-8 |p| in absolute terms, a large relative error
            // for a landmark close to the voxel centre (once per listed
            // landmark, so it costs nothing next to the N_s sigmoids)
            const T dx = (T)(px - tx), dy = (T)(py - ty), dz = (T)(pz - tz);
            const T nn = (PREC == 2) ? (T)fma((double)dz, (double)dz,
                                              fma((double)dy, (double)dy, (double)dx * dx))
                                     : (T)__fmaf_rn((float)dz, (float)dz,
                                                    __fmaf_rn((float)dy, (float)dy,
                                                              (float)dx * (float)dx));
            const T rn = (PREC == 2) ? (T)(1.0 / sqrt((double)nn)) : (T)rsq_normal((float)nn);
            rec.x = dx * rn; rec.y = dy * rn; rec.z = dz * rn;
            if constexpr (KIND == 0) {
              rec.w = rn;
            } else {
              // Tr(I_i) sigma^2 = (2 + |p|^2 + (u.p)^2) / n^2 for the global perturbation
              const T pxx = (T)px, pyy = (T)py, pzz = (T)pz;
              const T up = rec.x * pxx + rec.y * pyy + rec.z * pzz;
              rec.w = (T(2) + (pxx * pxx + pyy * pyy + pzz * pzz) + up * up) * (rn * rn);
            }
          }
        }
        const uint64_t m = __ballot(in);
        if (in) s_rec[wv][cnt + __popcll(m & ((1ull << lane) - 1))] = rec;
        cnt += __popcll(m);
      }
      wave_sync();
      for (int e0 = 0; e0 < cnt; e0 += 4) {
        const int e = e0 + (lane >> 4);
        const T okm = (e < cnt) ? T(1) : T(0);  // padding landmarks: zero terms
        const R4 r = s_rec[wv][e < cnt ? e : e0];
        const T u[3] = {r.x, r.y, r.z};
        T bval;
        if constexpr (KIND == 0) {
          const T ua = (T)sel.a[0] * u[0] + (T)sel.a[1] * u[1] + (T)sel.a[2] * u[2];
          const T ub = (T)sel.b[0] * u[0] + (T)sel.b[1] * u[1] + (T)sel.b[2] * u[2];
          const T pab = (T)sel.delta - ua * ub;
          const T rn = r.w;
          bval = (pab * ((T)sel.m_pn2 * (rn * rn) + (T)sel.m_p) + (T)sel.m_un * (ua * rn)) * okm;
        } else {
          bval = (lane & 15) == 0 ? r.w * okm : T(0);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const T x = fma(zz[t], u[2], fma(zy[t], u[1], fma(zx[t], u[0], z0[t])));
          acc[t] = mma16(sigmoid_from(x), bval, acc[t], s_mm[wv]);
        }
      }
      wave_sync();  // the list is rewritten by the next batch
      if (COMP) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            two_sum_acc(hi[t][r], lo[t][r], (float)acc[t][r]);
            acc[t][r] = 0;
          }
      }
    }
    // lane l, element r of tile t: axis g0 + 16 t + 4 (l / 16) + r, term l % 16
    T* out = reinterpret_cast<T*>(a.out) + (size_t)v * a.stride;
    const int f = lane & 15;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int g = g0 + 16 * t + 4 * (lane >> 4) + r;
        const T val = COMP ? (T)(hi[t][r] + lo[t][r]) : (T)acc[t][r];
        if (g < ns) {
          if constexpr (KIND == 0) out[(size_t)g * 16 + f] = val;
          else if (f == 0) out[g] = val;
        }
      }
  }
}

// ---------------------------------------------------------------- query

// Camera-frame block of one voxel from its 15 GP-weighted terms, moved by dl.
template <typename CT>
__device__ inline void gp_block(const CT s[15], const CT dl[3], CT out[21]) {
  CT A[6], D[6], B[9];
#pragma unroll
  for (int e = 0; e < 6; ++e) { A[e] = s[e]; D[e] = s[9 + e]; }
  // B = -[b]x with b = s[6..8]
  B[0] = 0;     B[1] = s[8];  B[2] = -s[7];
  B[3] = -s[8]; B[4] = 0;     B[5] = s[6];
  B[6] = s[7];  B[7] = -s[6]; B[8] = 0;
  shift_frame<CT>(A, B, D, dl, out);
}

constexpr int kChunk = 3;                      // rows loaded together per lane
constexpr int kKinvLds = 3240;                 // packed inverse held in LDS up to N_s = 80

// Rows r0 .. r0 + kChunk - 1 (those below nrow) of axes c8 + 8 r of a voxel.
template <typename FT>
__device__ inline void load_rows(const FT* rec, int c8, int r0, int nrow, FT x[kChunk][16]) {
#pragma unroll
  for (int rr = 0; rr < kChunk; ++rr) {
    if (r0 + rr < nrow) {
      const FT* row = rec + (size_t)(c8 + 8 * (r0 + rr)) * 16;
#pragma unroll
      for (int e = 0; e < 16; e += 4) {
        if constexpr (sizeof(FT) == 4) {
          const float4 v4 = *reinterpret_cast<const float4*>(row + e);
          x[rr][e] = v4.x; x[rr][e + 1] = v4.y; x[rr][e + 2] = v4.z; x[rr][e + 3] = v4.w;
        } else {
          const double2 v0 = *reinterpret_cast<const double2*>(row + e);
          const double2 v1 = *reinterpret_cast<const double2*>(row + e + 2);
          x[rr][e] = v0.x; x[rr][e + 1] = v0.y; x[rr][e + 2] = v1.x; x[rr][e + 3] = v1.y;
        }
      }
    }
  }
}

// Rows gr[0 .. NR-1] of w = (K^s + noise I)^-1 K_z for one pose: each row
// summed over h = 0 .. ns - 1 in ascending order.  NR is a template argument so
// that the reads of all rows for one h are issued together.
template <int NR>
__device__ inline void gp_wrows(const GPDev& gp, const double* kz, const double* kinv_lds,
                                bool in_lds, int lane, double wr[3]) {
  const int ns = gp.ns;
  int gr[NR], rs[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    gr[r] = min(lane + 64 * r, ns - 1);  // lanes past the end repeat a row
    rs[r] = gr[r] * (gr[r] + 1) / 2;
  }
  if (in_lds) {
    int hs = 0;  // h (h + 1) / 2: start of packed row h
#pragma unroll 2
    for (int h = 0; h < ns; ++h) {
      const double kzh = kz[h];
#pragma unroll
      for (int r = 0; r < NR; ++r)
        wr[r] = fma(kinv_lds[(h >= gr[r]) ? hs + gr[r] : rs[r] + h], kzh, wr[r]);
      hs += h + 1;
    }
  } else {
#pragma unroll 2
    for (int h = 0; h < ns; ++h) {
      const double kzh = kz[h];
#pragma unroll
      for (int r = 0; r < NR; ++r) wr[r] = fma(gp.kinv[(size_t)h * ns + gr[r]], kzh, wr[r]);
    }
  }
}

// Information fields (KIND 0; trace fields have their own kernel below).
// FP32 fields: two waves per SIMD (the register budget that keeps the gathers
// of two waves in flight); FP64 fields take one.
template <typename FT, int KIND>
__global__ __launch_bounds__(kGPThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(FT) == 4 ? 2 : 1))) void gp_query_kernel(GPQueryArgs ga) {
  static_assert(KIND == 0, "trace fields use gp_query_trace_kernel");
  using CT = FT;
  const QueryArgs& a = ga.q;
  __shared__ QSlot<CT> s_q[kGPWaves][64];
  __shared__ double s_kz[kGPWaves][kMaxNs];
  __shared__ CT s_w[kGPWaves][kMaxNs];
  __shared__ CT s_c[kGPWaves][8][22];
  __shared__ CT s_F[kGPWaves][64][22];
  __shared__ double s_kinv[kKinvLds];  // packed lower triangle of the inverse
  // sample axes: read from LDS so that the GP weights never wait on the
  // vector-memory counter behind the row gathers already in flight
  __shared__ double s_axes[3 * kMaxNs];

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int grp = lane >> 3, c8 = lane & 7;
  const int ns = ga.gp.ns;
  const FT* field = reinterpret_cast<const FT*>(a.field);
  const int64_t nbatch = (a.m + 63) / 64;
  const int64_t gw = (int64_t)blockIdx.x * kGPWaves + wv;
  const int64_t nw = (int64_t)gridDim.x * kGPWaves;

  const bool kinv_lds = ns * (ns + 1) / 2 <= kKinvLds;
  if (kinv_lds) {
    for (int i = threadIdx.x; i < ns * (ns + 1) / 2; i += kGPThreads) {
      int r = (int)((sqrt(8.0 * i + 1.0) - 1.0) * 0.5);
      while (r * (r + 1) / 2 > i) --r;
      while ((r + 1) * (r + 2) / 2 <= i) ++r;
      s_kinv[i] = ga.gp.kinv[(size_t)r * ns + (i - r * (r + 1) / 2)];
    }
  }
  for (int i = threadIdx.x; i < 3 * ns; i += kGPThreads) s_axes[i] = ga.gp.axes[i];
  __syncthreads();  // the only workgroup barrier: before any wave can leave
  for (int64_t b = gw; b < nbatch; b += nw) {
    const int64_t qown = b * 64 + lane;
    const bool valid = qown < a.m;
    const int64_t ql = valid ? qown : a.m - 1;
    s_q[wv][lane] = make_slot<FT>(a, ql);
    wave_sync();
    for (int k = 0; k < 64; ++k) {
      const QSlot<CT> sl = s_q[wv][k];
      const CornerC<CT> c = slot_corner(sl, a.g, grp);
      // rows of this lane: axes g = c8 + 8 r of corner grp
      const int nrow = c.active ? max(0, (ns - c8 + 7) / 8) : 0;
      const FT* rec = field + c.vox * (size_t)ga.stride;
      // first loads are issued before the GP weights, which they do not need
      FT xr[kChunk][16];
      load_rows<FT>(rec, c8, 0, nrow, xr);
      // GP weights of this pose: w = (K^s + noise I)^-1 K_z, FP64.  Lane l
      // forms rows l, l + 64 and l + 128 (as many as N_s needs), each summed
      // over h = 0 .. ns - 1 in order; every lane runs the same trip count and
      // the reads for all of its rows (and two values of h) are in flight
      // together instead of waiting one by one.
      const double z[3] = {(double)sl.z[0], (double)sl.z[1], (double)sl.z[2]};
      for (int g = lane; g < ns; g += 64) s_kz[wv][g] = se_kernel(z, s_axes + 3 * g, ga.gp.inv_2l2);
      wave_sync();
      {
        const int nr = (ns + 63) >> 6;  // rows per lane, 1 .. 3
        double wr[3] = {0.0, 0.0, 0.0};
        if (nr == 1) gp_wrows<1>(ga.gp, s_kz[wv], s_kinv, kinv_lds, lane, wr);
        else if (nr == 2) gp_wrows<2>(ga.gp, s_kz[wv], s_kinv, kinv_lds, lane, wr);
        else gp_wrows<3>(ga.gp, s_kz[wv], s_kinv, kinv_lds, lane, wr);
#pragma unroll
        for (int r = 0; r < 3; ++r)
          if (lane + 64 * r < ns) s_w[wv][lane + 64 * r] = (CT)wr[r];
      }
      wave_sync();
      {
        CT acc[15];
#pragma unroll
        for (int e = 0; e < 15; ++e) acc[e] = 0;
        for (int r0 = 0; r0 < nrow; r0 += kChunk) {
#pragma unroll
          for (int rr = 0; rr < kChunk; ++rr) {
            if (r0 + rr < nrow) {
              const CT wg = s_w[wv][c8 + 8 * (r0 + rr)];
#pragma unroll
              for (int e = 0; e < 15; ++e) acc[e] = fma(wg, (CT)xr[rr][e], acc[e]);
            }
          }
          if (r0 + kChunk < nrow) load_rows<FT>(rec, c8, r0 + kChunk, nrow, xr);
        }
        sum8_arr<15>(acc);
        if (c8 == 0) {
          CT Y[21];
          if (c.active) {
            gp_block<CT>(acc, c.dl, Y);
#pragma unroll
            for (int e = 0; e < 21; ++e) Y[e] *= c.w;
          } else {
#pragma unroll
            for (int e = 0; e < 21; ++e) Y[e] = 0;
          }
#pragma unroll
          for (int e = 0; e < 21; ++e) s_c[wv][grp][e] = Y[e];
        }
      }
      wave_sync();
      if (lane < 21) {
        CT sacc = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) sacc += s_c[wv][j][lane];
        s_F[wv][k][lane] = sacc;
      }
      wave_sync();
    }
    // metrics of this lane's own pose
    const QSlot<CT> own = s_q[wv][lane];
    uint8_t flag = (own.bits & 8) ? FL_CLAMPED : 0;
    double td[3] = {(double)own.t[0], (double)own.t[1], (double)own.t[2]};
    double Zd[21], F[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) Zd[e] = (double)s_F[wv][lane][e];
    shift21<double>(Zd, td, F);
#pragma unroll
    for (int e = 0; e < 21; ++e) F[e] *= a.vis.inv_s2;
    double* row = (valid && a.out) ? a.out + ql * a.ncols : nullptr;
    eval_metrics<false>(F, a.metrics, row, &flag, nullptr, nullptr, a.flags != nullptr);
    if (valid && a.flags) a.flags[ql] = flag;
    wave_sync();  // s_q and s_F are rewritten by the next batch
  }
}

// Trace fields (eq:general_trace_pif with the GP weights of Sec. V-B):
//   Tr(pose) = K_z^T (K^s + noise I)^-1 Tbar,  Tbar = sum_j w_j T_j
// over the pose's 8 corner rows T_j of N_s trace factors.  Two phases per
// wave of 64 poses:
//  1. interpolation, pose by pose with the whole wave: lane l reads factors
//     2l and 2l+1 of each corner row (NW windows of 128 factors), so one load
//     instruction reads a row's consecutive bytes, and writes the weighted sum
//     (corners in order 0..7) to the pose's LDS column;
//  2. W = kinv Tbar for the wave's 64 columns on the FP64 matrix cores
//     (v_mfma_f64_16x16x4: A = 16 rows x 4 factors of kinv, B = 4 factors x 16
//     poses), then Tr = sum_g K_z[g] W[g] with K_z formed in FP64 per (g, pose)
//     and the four lanes that hold one pose's rows summed.
// A lane's value from another lane of the wave (k wave-uniform).
__device__ inline float lane_value(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ inline double lane_value(double v, int k) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, k);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), k);
  return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

template <typename FT, int NW>
__global__ __launch_bounds__(256, 2) void gp_query_trace_kernel(GPQueryArgs ga) {
  using CT = FT;
  using FT2 = typename std::conditional<sizeof(FT) == 4, float2, double2>::type;
  extern __shared__ unsigned char s_dyn[];
  const int nt = blockDim.x;
  const int cs = nt + 1;  // column stride: a pose's factors fall in different banks
  CT* col = reinterpret_cast<CT*>(s_dyn);  // [ns][cs]
  // the sample axes, after the columns (16-B aligned)
  double* s_ax =
      reinterpret_cast<double*>(s_dyn + ((size_t)ga.gp.ns * cs * sizeof(CT) + 15) / 16 * 16);
  for (int i = threadIdx.x; i < 3 * ga.gp.ns; i += blockDim.x) s_ax[i] = ga.gp.axes[i];
  __syncthreads();
  const QueryArgs& a = ga.q;
  const int ns = ga.gp.ns;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wbase = tid - lane;
  const int64_t qi = (int64_t)blockIdx.x * nt + tid;
  const bool valid = qi < a.m;
  const int64_t ql = valid ? qi : a.m - 1;
  const QSlot<CT> sl = make_slot<FT>(a, ql);
  const FT* field = reinterpret_cast<const FT*>(a.field);
  // this lane's pose: corner rows (voxel index < 2^32, checked by the caller)
  // and weights; a corner that nearest mode leaves out reads corner 0's row
  // with weight 0
  uint32_t cvox[8];
  CT cw[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const CornerC<CT> c = slot_corner(sl, a.g, j);
    cvox[j] = (uint32_t)c.vox;
    cw[j] = c.active ? c.w : CT(0);
  }
#pragma unroll
  for (int j = 1; j < 8; ++j)
    if (cw[j] == CT(0)) cvox[j] = cvox[0];
  const int npair = (ns + 1) >> 1;
  const size_t stride = (size_t)ga.stride;
  auto load = [&](int k, FT2 (&x)[8][NW]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const FT* row = field + (size_t)(uint32_t)__builtin_amdgcn_readlane((int)cvox[j], k) * stride;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        // lanes past the row read its last pair again: no branch around the load
        const int p = min(64 * w + lane, npair - 1);
        x[j][w] = *reinterpret_cast<const FT2*>(row + 2 * p);
      }
    }
  };
  // phase 1, G poses' rows in flight together
  constexpr int G = 8 / (int)(sizeof(FT) / 4) / NW;
#pragma unroll 1
  for (int k0 = 0; k0 < 64; k0 += G) {
    FT2 x[G][8][NW];
#pragma unroll
    for (int u = 0; u < G; ++u) load(k0 + u, x[u]);
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int k = k0 + u;
      CT w8[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) w8[j] = lane_value(cw[j], k);
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int p = 64 * w + lane;
        if (p < npair) {
          CT e0 = CT(0), e1 = CT(0);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            e0 = fma(w8[j], (CT)x[u][j][w].x, e0);
            e1 = fma(w8[j], (CT)x[u][j][w].y, e1);
          }
          col[(size_t)(2 * p) * cs + wbase + k] = e0;
          if (2 * p + 1 < ns) col[(size_t)(2 * p + 1) * cs + wbase + k] = e1;
        }
      }
    }
  }
  wave_sync();
  // phase 2.  MFMA lane layout (16x16x4 FP64): A[i][k] and B[k][j] in lane
  // i + 16 k and j + 16 k; D[4 r + k][j] in register r of lane j + 16 k.
  // Lane (i16, k4) thus accumulates W rows g = 16 m + 4 r + k4 of the poses
  // 16 n + i16 (N tiles n = 0..3); MG M tiles of kinv are accumulated together
  // so that each B fragment is read from LDS once per group.
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int i16 = lane & 15, k4 = lane >> 4;
  double zq[4][3];  // axes of the poses 16 n + i16 of this wave
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int c = 0; c < 3; ++c) zq[n][c] = (double)__shfl(sl.z[c], 16 * n + i16);
  const double* kinv = ga.gp.kinv;
  const int nm = (ns + 15) >> 4, nk = (ns + 3) >> 2;
  constexpr int MG = 5;  // M tiles (16 rows of kinv each) accumulated together
  double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int m0 = 0; m0 < nm; m0 += MG) {
    // A fragments of step s: kinv[16 m + i16][4 s + k4]; entries past row or
    // column ns are zero (read clamped, then masked by a multiply so that the
    // load is not moved into a branch).  B fragments: Tbar[4 s + k4][16 n +
    // i16] (a clamped row past ns: finite, and its A entries are zero).
    const double* krow[MG];
    bool gv[MG];
#pragma unroll
    for (int mm = 0; mm < MG; ++mm) {
      const int g = 16 * (m0 + mm) + i16;
      gv[mm] = g < ns;
      krow[mm] = kinv + (size_t)min(g, ns - 1) * ns;
    }
    auto load = [&](int st, double (&av)[MG], double (&bv)[4]) {
      const int h = 4 * st + k4;
      const double mask = h < ns ? 1.0 : 0.0;
      const int hc = min(h, ns - 1);
#pragma unroll
      for (int mm = 0; mm < MG; ++mm) av[mm] = krow[mm][hc] * (gv[mm] ? mask : 0.0);
      const CT* crow = col + (size_t)hc * cs + wbase + i16;
#pragma unroll
      for (int n = 0; n < 4; ++n) bv[n] = (double)crow[16 * n];
    };
    d4 acc[MG][4];
#pragma unroll
    for (int mm = 0; mm < MG; ++mm)
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[mm][n] = d4{0.0, 0.0, 0.0, 0.0};
    double an[MG], bn[4];
    load(0, an, bn);
#pragma unroll 1
    for (int st = 0; st < nk; ++st) {
      double av[MG], bv[4];
#pragma unroll
      for (int mm = 0; mm < MG; ++mm) av[mm] = an[mm];
#pragma unroll
      for (int n = 0; n < 4; ++n) bv[n] = bn[n];
      load(min(st + 1, nk - 1), an, bn);
#pragma unroll
      for (int mm = 0; mm < MG; ++mm)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc[mm][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mm], bv[n], acc[mm][n], 0, 0, 0);
    }
    // W rows g = 16 m + 4 r + k4 of poses 16 n + i16, weighted by K_z
#pragma unroll
    for (int mm = 0; mm < MG; ++mm) {
      if (m0 + mm >= nm) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = min(16 * (m0 + mm) + 4 * r + k4, ns - 1);
        const double ax[3] = {s_ax[3 * gr], s_ax[3 * gr + 1], s_ax[3 * gr + 2]};
#pragma unroll
        for (int n = 0; n < 4; ++n)
          part[n] = fma(se_kernel(zq[n], ax, ga.gp.inv_2l2), acc[mm][n][r], part[n]);
      }
    }
  }
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    part[n] += __shfl_xor(part[n], 16);
    part[n] += __shfl_xor(part[n], 32);
  }
  const double tr = k4 == 0 ? part[0] : k4 == 1 ? part[1] : k4 == 2 ? part[2] : part[3];
  if (valid) {
    if (a.out) a.out[ql * a.ncols] = tr * a.vis.inv_s2;
    if (a.flags) a.flags[ql] = (sl.bits & 8) ? FL_CLAMPED : 0;
  }
}

// ---------------------------------------------------------------- export

// One thread per (voxel, axis g): C_g = sum_h kinv[g][h] world(S_h) / sigma^2.
template <typename FT, int KIND>
__global__ void gp_export_kernel(GPExportArgs a) {
  const int ns = a.gp.ns;
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= a.n * ns) return;
  const int64_t i = it / ns;
  const int g = (int)(it % ns);
  const int64_t v = a.ids[i];
  const int64_t nvox = (int64_t)a.g.nx * a.g.ny * a.g.nz;
  const int per = KIND == 0 ? 21 : 1;
  double* out = a.out + (i * ns + g) * per;
  if (v < 0 || v >= nvox) {
    for (int e = 0; e < per; ++e) out[e] = __builtin_nan("");
    return;
  }
  const FT* rec = reinterpret_cast<const FT*>(a.field) + (size_t)v * a.stride;
  if constexpr (KIND == 0) {
    const int64_t ix = v % a.g.nx, iy = (v / a.g.nx) % a.g.ny, iz = v / ((int64_t)a.g.nx * a.g.ny);
    const double tv[3] = {a.g.ox + (double)ix * a.g.h, a.g.oy + (double)iy * a.g.h,
                          a.g.oz + (double)iz * a.g.h};
    double C[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) C[e] = 0.0;
    for (int h = 0; h < ns; ++h) {
      double s[15], W[21];
#pragma unroll
      for (int e = 0; e < 15; ++e) s[e] = (double)rec[(size_t)h * 16 + e];
      gp_block<double>(s, tv, W);
      const double k = a.gp.kinv[(size_t)g * ns + h];
#pragma unroll
      for (int e = 0; e < 21; ++e) C[e] = fma(k, W[e], C[e]);
    }
#pragma unroll
    for (int e = 0; e < 21; ++e) out[e] = C[e] * a.inv_s2;
  } else {
    double c = 0.0;
    for (int h = 0; h < ns; ++h) c = fma(a.gp.kinv[(size_t)g * ns + h], (double)rec[h], c);
    out[0] = c * a.inv_s2;
  }
}

int64_t resident_blocks(int per_cu) { return (int64_t)current_device_cus() * per_cu; }

}  // namespace

hipError_t launch_gp_setup(const GPDev& gp, double* kinv, hipStream_t stream) {
  hipLaunchKernelGGL(gp_setup_kernel, dim3(1), dim3(256), 0, stream, gp, kinv);
  return hipGetLastError();
}

hipError_t launch_gp_evidence(const GPDev& gp, const double* train_u, int32_t n_train,
                              const double* lengths, int32_t n_len, double* lml,
                              hipStream_t stream) {
  if (n_len <= 0) return hipSuccess;
  hipLaunchKernelGGL(gp_evidence_kernel, dim3((unsigned)n_len), dim3(256), 0, stream, gp, train_u,
                     n_train, lengths, lml);
  return hipGetLastError();
}

template <int PREC, int KIND>
hipError_t launch_gp_build_tiles(const GPBuildArgs& a, dim3 grid, int pass0, int nt,
                                 hipStream_t stream) {
  dim3 block(kGPThreads);
  switch (nt) {
    case 1: hipLaunchKernelGGL((gp_build_kernel<PREC, KIND, 1>), grid, block, 0, stream, a, pass0); break;
    case 2: hipLaunchKernelGGL((gp_build_kernel<PREC, KIND, 2>), grid, block, 0, stream, a, pass0); break;
    case 3: hipLaunchKernelGGL((gp_build_kernel<PREC, KIND, 3>), grid, block, 0, stream, a, pass0); break;
    case 4: hipLaunchKernelGGL((gp_build_kernel<PREC, KIND, 4>), grid, block, 0, stream, a, pass0); break;
    default: hipLaunchKernelGGL((gp_build_kernel<PREC, KIND, kGPTiles>), grid, block, 0, stream, a, pass0); break;
  }
  return hipGetLastError();
}

hipError_t launch_gp_build(const GPBuildArgs& a, int prec, int kind, hipStream_t stream) {
  const int64_t nvox = (int64_t)a.g.nx * a.g.ny * a.g.nz;
  const int64_t want = (nvox + kGPWaves - 1) / kGPWaves;
  const int64_t cap = resident_blocks(8);
  const unsigned gx = (unsigned)(want < cap ? want : cap);
  // passes of kGPTiles 16-axis tiles; the last one with the tiles it needs
  const int per = 16 * kGPTiles;
  const int full = a.gp.ns / per;
  const int rest_tiles = (a.gp.ns % per + 15) / 16;
  auto run = [&](dim3 grid, int pass0, int nt) -> hipError_t {
    if (kind == 0) {
      if (prec == 0) return launch_gp_build_tiles<0, 0>(a, grid, pass0, nt, stream);
      if (prec == 1) return launch_gp_build_tiles<1, 0>(a, grid, pass0, nt, stream);
      return launch_gp_build_tiles<2, 0>(a, grid, pass0, nt, stream);
    }
    if (prec == 0) return launch_gp_build_tiles<0, 1>(a, grid, pass0, nt, stream);
    if (prec == 1) return launch_gp_build_tiles<1, 1>(a, grid, pass0, nt, stream);
    return launch_gp_build_tiles<2, 1>(a, grid, pass0, nt, stream);
  };
  if (full > 0) {
    hipError_t e = run(dim3(gx, (unsigned)full), 0, kGPTiles);
    if (e != hipSuccess) return e;
  }
  if (rest_tiles > 0) return run(dim3(gx, 1), full, rest_tiles);
  return hipSuccess;
}

hipError_t launch_gp_query(const GPQueryArgs& a, int prec, int kind, hipStream_t stream) {
  if (a.q.m <= 0) return hipSuccess;
  const int64_t nbatch = (a.q.m + 63) / 64;
  const int64_t want = (nbatch + kGPWaves - 1) / kGPWaves;
  const int64_t cap = resident_blocks(8);
  dim3 grid((unsigned)(want < cap ? want : cap)), block(kGPThreads);
  if (kind == 1) {
    // one lane per pose; the LDS columns (N_s per lane) set the workgroup size
    const size_t sb = prec == 2 ? 8 : 4;
    // LDS: the poses' columns (stride nt + 1) and the sample axes; 256 lanes
    // while that fits two workgroups per CU, else one wave per workgroup
    auto lds_of = [&](int nt) {
      return ((size_t)a.gp.ns * (nt + 1) * sb + 15) / 16 * 16 + (size_t)a.gp.ns * 24;
    };
    const int nt = lds_of(256) <= 80 * 1024 ? 256 : 64;
    const size_t lds = lds_of(nt);
    const bool two = (a.gp.ns + 1) / 2 > 64;  // rows longer than 128 factors
    for (int64_t off = 0; off < a.q.m; off += kMaxLaunchItems) {
      GPQueryArgs p = a;
      p.q = query_part(a.q, off, std::min(kMaxLaunchItems, a.q.m - off), sb);
      dim3 tgrid((unsigned)((p.q.m + nt - 1) / nt)), tblock(nt);
      if (prec == 2 && two) hipLaunchKernelGGL((gp_query_trace_kernel<double, 2>), tgrid, tblock, lds, stream, p);
      else if (prec == 2) hipLaunchKernelGGL((gp_query_trace_kernel<double, 1>), tgrid, tblock, lds, stream, p);
      else if (two) hipLaunchKernelGGL((gp_query_trace_kernel<float, 2>), tgrid, tblock, lds, stream, p);
      else hipLaunchKernelGGL((gp_query_trace_kernel<float, 1>), tgrid, tblock, lds, stream, p);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (prec == 2) hipLaunchKernelGGL((gp_query_kernel<double, 0>), grid, block, 0, stream, a);
  else hipLaunchKernelGGL((gp_query_kernel<float, 0>), grid, block, 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_gp_export(const GPExportArgs& a, int prec, int kind, hipStream_t stream) {
  if (a.n <= 0 || a.gp.ns <= 0) return hipSuccess;
  const int64_t per = kMaxLaunchItems / a.gp.ns;  // voxel ids per launch
  for (int64_t off = 0; off < a.n; off += per) {
    GPExportArgs p = a;
    p.n = std::min(per, a.n - off);
    p.ids = a.ids + off;
    p.out = a.out + (size_t)off * a.gp.ns * (kind == 0 ? 21 : 1);
    const int64_t total = p.n * a.gp.ns;
    dim3 grid((unsigned)((total + 127) / 128)), block(128);
    if (prec == 2) {
      if (kind == 0) hipLaunchKernelGGL((gp_export_kernel<double, 0>), grid, block, 0, stream, p);
      else hipLaunchKernelGGL((gp_export_kernel<double, 1>), grid, block, 0, stream, p);
    } else {
      if (kind == 0) hipLaunchKernelGGL((gp_export_kernel<float, 0>), grid, block, 0, stream, p);
      else hipLaunchKernelGGL((gp_export_kernel<float, 1>), grid, block, 0, stream, p);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fif
