// Point-cloud brute force (eq:cost_info, eq:vis_fim): for each pose, the sum
// of v_i I_i over every landmark in range.  One lane per pose; landmarks are
// staged through LDS in batches of 256 and read back as broadcasts.
//
// Sorted path (given a workspace and a finite range): landmarks and poses are
// ordered by the Morton code of fixed cells, so a workgroup's 256 poses sit in
// a small box and a batch of 256 landmarks too; a workgroup skips every batch
// whose box is out of range of its poses' box.  A skipped batch would only add
// zeros, and the landmarks are summed in the same order as by the plain kernel
// given the landmarks in that order, so the results are the same bit for bit.
//
// The sum is accumulated about the camera position t, where a landmark's FIM
// has the form (1/sigma^2) [[P/n^2, -[u]x/n], [[u]x/n, P]] (P = I - u u^T), so
// 15 running sums suffice: sum v u u^T, sum v u u^T / n^2, sum v u / n.  One
// shift to the world origin at the end gives eq:jac_pose_global's frame.
#include "fif_kernels.h"
#include "fif_metrics.h"

namespace fif {

constexpr int kPcThreads = 256;
constexpr int kPcBatch = 256;

__device__ inline void pc_two_sum(float& hi, float& lo, float x) {
  float s = hi + x;
  float bb = s - hi;
  float err = (hi - (s - bb)) + (x - bb);
  hi = s;
  lo += err;
}

template <int PREC, bool EXACT, bool SORTED>
__global__ __launch_bounds__(kPcThreads) void pc_kernel(PcArgs a) {
  using T = typename std::conditional<PREC == 2, double, float>::type;
  using L4 = typename std::conditional<PREC == 2, double4, float4>::type;
  constexpr bool COMP = (PREC == 1);
  __shared__ L4 s_lm[kPcBatch];
  __shared__ float s_box[kPcThreads / 64][6];

  const int tid = threadIdx.x;
  const int64_t qi = (int64_t)blockIdx.x * kPcThreads + tid;
  const bool valid = qi < a.m;
  int64_t ql = valid ? qi : a.m - 1;
  if (SORTED) ql = a.perm[ql];

  const T* TT = reinterpret_cast<const T*>(a.t);
  const T* QQ = reinterpret_cast<const T*>(a.q);
  const double t[3] = {(double)TT[3 * ql], (double)TT[3 * ql + 1], (double)TT[3 * ql + 2]};
  const double qw = QQ[4 * ql], qx = QQ[4 * ql + 1], qy = QQ[4 * ql + 2], qz = QQ[4 * ql + 3];
  double Rd[9];
  quat_R(qw, qx, qy, qz, Rd);
  T R[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) R[e] = (T)Rd[e];
  const T zx = R[2], zy = R[5], zz = R[8];
  const float ftx = (float)t[0], fty = (float)t[1], ftz = (float)t[2];
  const T tx = (T)t[0], ty = (T)t[1], tz = (T)t[2];
  // Compensated FP32 sums: a landmark closer to the camera than 1 % of the
  // camera's distance from the origin (or 1 cm) takes its offset from the
  // FP64 coordinates, as in the compensated field build (the FP32-rounded
  // landmark is off by up to ~6e-8 |p| in absolute terms).  Rare, so a
  // divergent branch.
  const float near2 = 1e-4f * (ftx * ftx + fty * fty + ftz * ftz) + 1e-4f;
  const T k2 = (T)a.vis.k2, k1 = (T)a.vis.k1, k0 = (T)a.vis.k0;
  const T fx = (T)a.fx, fy = (T)a.fy, cx = (T)a.cx, cy = (T)a.cy;
  const T W = (T)a.width, H = (T)a.height;

  T acc[15];  // Q0 (6), Q2 (6), B1 (3)
  float hi[COMP ? 15 : 1], lo[COMP ? 15 : 1];
#pragma unroll
  for (int e = 0; e < 15; ++e) acc[e] = T(0);
  if (COMP) {
#pragma unroll
    for (int e = 0; e < 15; ++e) { hi[e] = 0.f; lo[e] = 0.f; }
  }

  // the workgroup's poses' box in FP32 (the coordinates of the range test)
  float plo[3] = {0.f, 0.f, 0.f}, phi[3] = {0.f, 0.f, 0.f};
  if (SORTED) {
    float v[6] = {valid ? ftx : INFINITY,  valid ? fty : INFINITY,  valid ? ftz : INFINITY,
                  valid ? -ftx : INFINITY, valid ? -fty : INFINITY, valid ? -ftz : INFINITY};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = fminf(v[c], __shfl_xor(v[c], off, 64));
    if ((tid & 63) == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) s_box[tid >> 6][c] = v[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float lo = s_box[0][c], mhi = s_box[0][3 + c];
#pragma unroll
      for (int w = 1; w < kPcThreads / 64; ++w) {
        lo = fminf(lo, s_box[w][c]);
        mhi = fminf(mhi, s_box[w][3 + c]);
      }
      plo[c] = lo;
      phi[c] = -mhi;
    }
  }

  for (int64_t base = 0; base < a.L; base += kPcBatch) {
    const int nb = (int)((a.L - base) < kPcBatch ? (a.L - base) : kPcBatch);
    if (SORTED) {
      // skip a batch whose box is out of range of every pose of the
      // workgroup (the same decision on every lane)
      const float* bb = a.batch_box + 8 * (base / kPcBatch);
      float d2 = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float gap = fmaxf(fmaxf(bb[c] - phi[c], plo[c] - bb[3 + c]), 0.f);
        d2 = fmaf(gap, gap, d2);
      }
      if (d2 > a.skip2) continue;
    }
    __syncthreads();
    if (tid < nb) {
      double px, py, pz;
      if (SORTED) {
        const double4 p4 = a.lm_sorted[base + tid];
        px = p4.x; py = p4.y; pz = p4.z;
      } else {
        const double* p = a.lm + 3 * (base + tid);
        px = p[0]; py = p[1]; pz = p[2];
      }
      L4 v;
      v.x = (T)px; v.y = (T)py; v.z = (T)pz; v.w = T(0);
      s_lm[tid] = v;
    }
    __syncthreads();
    // Per 64-landmark slice: test every landmark into a per-lane bit mask,
    // then each lane walks only its own set bits (its landmarks in range and,
    // in exact mode, in view), so lanes do not wait on each other's work.
    // (bitwise & rather than &&: no branch per landmark; lanes without a pose
    // clear their mask afterwards)
    auto in_set = [&](const L4& p) __attribute__((always_inline)) -> uint32_t {
      float ddx = (float)p.x - ftx, ddy = (float)p.y - fty, ddz = (float)p.z - ftz;
      float n2 = __fmaf_rn(ddz, ddz, __fmaf_rn(ddy, ddy, ddx * ddx));
      bool in = (n2 >= a.lo2) & (n2 <= a.hi2);
      if (EXACT) {
        T dx = p.x - tx, dy = p.y - ty, dz = p.z - tz;
        T pcx = R[0] * dx + R[3] * dy + R[6] * dz;
        T pcy = R[1] * dx + R[4] * dy + R[7] * dz;
        T pcz = R[2] * dx + R[5] * dy + R[8] * dz;
        T u = fx * pcx / pcz + cx;
        T v = fy * pcy / pcz + cy;
        in = in & (pcz > T(0)) & (u >= T(0)) & (u < W) & (v >= T(0)) & (v < H);
      }
      return in ? 1u : 0u;
    };
    // one landmark's terms (i: its index in the batch)
    auto add_pair = [&](const L4& p, int i) __attribute__((always_inline)) {
      T dx = p.x - tx, dy = p.y - ty, dz = p.z - tz;
      T nn = (PREC == 2) ? (T)fma((double)dz, (double)dz, fma((double)dy, (double)dy, (double)dx * dx))
                         : (T)__fmaf_rn((float)dz, (float)dz, __fmaf_rn((float)dy, (float)dy, (float)dx * (float)dx));
      if constexpr (COMP) {
        if ((float)nn < near2) {
          double lx, ly, lz;
          if (SORTED) {
            const double4 l4 = a.lm_sorted[base + i];
            lx = l4.x; ly = l4.y; lz = l4.z;
          } else {
            const double* lp = a.lm + 3 * (base + i);
            lx = lp[0]; ly = lp[1]; lz = lp[2];
          }
          dx = (T)(lx - t[0]); dy = (T)(ly - t[1]); dz = (T)(lz - t[2]);
          nn = __fmaf_rn((float)dz, (float)dz, __fmaf_rn((float)dy, (float)dy, (float)dx * (float)dx));
        }
      }
      T rn = (PREC == 2) ? (T)(1.0 / sqrt((double)nn)) : (T)rsq_normal((float)nn);
      T ux = dx * rn, uy = dy * rn, uz = dz * rn;
      T w = T(1);
      if (!EXACT) {
        T c = zx * ux + zy * uy + zz * uz;
        w = fma(fma(k2, c, k1), c, k0);
      }
      T rn2 = rn * rn;
      T wn = w * rn, wn2 = w * rn2;
      T m2[6] = {ux * ux, ux * uy, ux * uz, uy * uy, uy * uz, uz * uz};
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        acc[e] = fma(w, m2[e], acc[e]);
        acc[6 + e] = fma(wn2, m2[e], acc[6 + e]);
      }
      acc[12] = fma(wn, ux, acc[12]);
      acc[13] = fma(wn, uy, acc[13]);
      acc[14] = fma(wn, uz, acc[14]);
    };
    for (int s0 = 0; s0 < nb; s0 += 64) {
      const int ns = (nb - s0) < 64 ? (nb - s0) : 64;
      uint64_t mask = 0;
      if (ns == 64) {
        // groups of 8: the group's LDS reads are issued together
#pragma unroll 1
        for (int g = 0; g < 64; g += 8) {
          L4 pg[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) pg[k] = s_lm[s0 + g + k];
          uint32_t bits = 0;
#pragma unroll
          for (int k = 0; k < 8; ++k) bits |= in_set(pg[k]) << k;
          mask |= (uint64_t)bits << g;
        }
      } else {
        for (int i = 0; i < ns; ++i) mask |= (uint64_t)in_set(s_lm[s0 + i]) << i;
      }
      if (!valid) mask = 0;
      // walk the set bits in increasing order, one 32-bit half at a time; the
      // next landmark's LDS read is issued before the current one's terms
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        uint32_t mk = half ? (uint32_t)(mask >> 32) : (uint32_t)mask;
        const int hb = s0 + 32 * half;
        if (mk) {
          int i = __ffs(mk) - 1;
          L4 p = s_lm[hb + i];
          while (true) {
            mk &= mk - 1;
            const int inext = mk ? __ffs(mk) - 1 : i;
            const L4 pn = s_lm[hb + inext];
            add_pair(p, hb + i);
            if (!mk) break;
            p = pn;
            i = inext;
          }
        }
      }
    }
    if (COMP) {
#pragma unroll
      for (int e = 0; e < 15; ++e) {
        pc_two_sum(hi[e], lo[e], (float)acc[e]);
        acc[e] = T(0);
      }
    }
  }
  if (!valid) return;
  double s[15];
#pragma unroll
  for (int e = 0; e < 15; ++e) s[e] = COMP ? (double)hi[e] + (double)lo[e] : (double)acc[e];
  double A[6], D[6], B[9];
  const double tr0 = s[0] + s[3] + s[5], tr2 = s[6] + s[9] + s[11];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const bool diag = (e == 0 || e == 3 || e == 5);
    D[e] = (diag ? tr0 : 0.0) - s[e];
    A[e] = (diag ? tr2 : 0.0) - s[6 + e];
  }
  const double b0 = s[12], b1 = s[13], b2 = s[14];
  B[0] = 0.0; B[1] = b2;  B[2] = -b1;
  B[3] = -b2; B[4] = 0.0; B[5] = b0;
  B[6] = b1;  B[7] = -b0; B[8] = 0.0;
  double F[21];
  shift_frame(A, B, D, t, F);
#pragma unroll
  for (int e = 0; e < 21; ++e) F[e] *= a.vis.inv_s2;
  uint8_t flag = 0;
  eval_metrics<false>(F, a.metrics, a.out + ql * a.ncols, &flag, nullptr, nullptr);
}

hipError_t launch_pc(const PcArgs& a, int prec, hipStream_t stream) {
  if (a.m <= 0) return hipSuccess;
  const size_t sb = prec == 2 ? 8 : 4;
  for (int64_t off = 0; off < a.m; off += kMaxLaunchItems) {
    PcArgs p = a;
    p.m = std::min(kMaxLaunchItems, a.m - off);
    p.t = static_cast<const char*>(a.t) + (size_t)off * 3 * sb;
    p.q = static_cast<const char*>(a.q) + (size_t)off * 4 * sb;
    p.out = a.out + (size_t)off * a.ncols;
    dim3 grid((unsigned)((p.m + kPcThreads - 1) / kPcThreads)), block(kPcThreads);
#define FIF_PC(P, E) hipLaunchKernelGGL((pc_kernel<P, E, false>), grid, block, 0, stream, p)
    if (a.exact) {
      if (prec == 0) FIF_PC(0, true);
      else if (prec == 1) FIF_PC(1, true);
      else FIF_PC(2, true);
    } else {
      if (prec == 0) FIF_PC(0, false);
      else if (prec == 1) FIF_PC(1, false);
      else FIF_PC(2, false);
    }
#undef FIF_PC
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Poses per pass of the sorted path: each pass sorts its poses on their own.
constexpr int64_t kPcSortChunk = int64_t(1) << 26;

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t pc_sorted_workspace_bytes(int64_t L, int64_t m) {
  if (L <= 0 || m <= 0) return 0;
  const size_t lm = cell_sorted_landmarks_bytes(L);
  const size_t ps = cell_sort_bytes(std::min(m, kPcSortChunk));
  if (lm == 0 || ps == 0) return 0;
  return align256(lm) + align256(ps);
}

hipError_t launch_pc_sorted(PcArgs a, int prec, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (a.m <= 0) return hipSuccess;
  const size_t need = pc_sorted_workspace_bytes(a.L, a.m);
  if (need == 0 || ws_bytes < need) return hipErrorInvalidValue;
  // cells of r_max / 32: 1024 cells span 32 ranges before the codes wrap
  const double inv_cell = a.inv_cell;
  const size_t lm_bytes = align256(cell_sorted_landmarks_bytes(a.L));
  hipError_t e = cell_sort_landmarks(a.lm, a.L, inv_cell, ws, lm_bytes, stream, &a.lm_sorted,
                                     &a.batch_box);
  if (e != hipSuccess) return e;
  a.skip2 = a.hi2 * 1.0001f + 1e-3f;
  void* pws = static_cast<char*>(ws) + lm_bytes;
  const size_t pws_bytes = ws_bytes - lm_bytes;
  const size_t sb = prec == 2 ? 8 : 4;
  for (int64_t off = 0; off < a.m; off += kPcSortChunk) {
    PcArgs p = a;
    p.m = std::min(kPcSortChunk, a.m - off);
    p.t = static_cast<const char*>(a.t) + (size_t)off * 3 * sb;
    p.q = static_cast<const char*>(a.q) + (size_t)off * 4 * sb;
    p.out = a.out + (size_t)off * a.ncols;
    e = cell_sort(p.t, prec == 2, p.m, inv_cell, pws, pws_bytes, stream, &p.perm);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((p.m + kPcThreads - 1) / kPcThreads)), block(kPcThreads);
#define FIF_PC(P, E) hipLaunchKernelGGL((pc_kernel<P, E, true>), grid, block, 0, stream, p)
    if (a.exact) {
      if (prec == 0) FIF_PC(0, true);
      else if (prec == 1) FIF_PC(1, true);
      else FIF_PC(2, true);
    } else {
      if (prec == 0) FIF_PC(0, false);
      else if (prec == 1) FIF_PC(1, false);
      else FIF_PC(2, false);
    }
#undef FIF_PC
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fif
