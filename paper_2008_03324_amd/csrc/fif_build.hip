// Field construction kernels (Sec. VI-A: factors computed at the voxel centres
// from all landmarks in range).
//
// One lane owns one voxel; a 256-thread workgroup owns an 8x8x4 voxel tile
// (each wave a 4x4x4 sub-tile, so the lanes of a wave see nearly the same
// landmarks in range and the range test stays wave-coherent).  Landmarks are
// staged through LDS in batches of 256 and read back as broadcasts; each lane
// folds every landmark in range into its 66 moment sums (see fif_device.h).
// The summation order is fixed (landmark order), so results are bitwise
// reproducible.
#include <cmath>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "fif_device.h"
#include "fif_kernels.h"

namespace fif {

constexpr int kBuildThreads = 256;
constexpr int kBatch = 256;

template <typename T>
struct LmT;
template <>
struct LmT<float> { using type = float4; };
template <>
struct LmT<double> { using type = double4; };

// Two-sum merge of a partial into (hi, lo): hi + lo gains x exactly.
__device__ inline void two_sum_into(float& hi, float& lo, float x) {
  float s = hi + x;
  float bb = s - hi;
  float err = (hi - (s - bb)) + (x - bb);
  hi = s;
  lo += err;
}

// Accumulate one landmark's contribution into the 66 moments.  Degree-4
// monomials are never formed: each is a degree-3 monomial times one
// component, folded into the two FMAs that consume it.
template <typename T>
__device__ inline void info_pair(T acc[kMom], T dx, T dy, T dz, T rn) {
  T ux = dx * rn, uy = dy * rn, uz = dz * rn;
  T rn2 = rn * rn;
  T u[3] = {ux, uy, uz};
  T u2n[3] = {ux * rn2, uy * rn2, uz * rn2};
  T m2[6], m3[10];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) m2[i2(a, b)] = u[a] * u[b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
#pragma unroll
      for (int c = b; c < 3; ++c) m3[i3(a, b, c)] = m2[i2(a, b)] * u[c];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
#pragma unroll
      for (int c = b; c < 3; ++c)
#pragma unroll
        for (int d = c; d < 3; ++d) {
          const int k = i4(a, b, c, d);
          acc[O_G0_4 + k] = fma(m3[i3(a, b, c)], u[d], acc[O_G0_4 + k]);
          acc[O_G2_4 + k] = fma(m3[i3(a, b, c)], u2n[d], acc[O_G2_4 + k]);
        }
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    acc[O_G0_3 + i] += m3[i];
    acc[O_G2_3 + i] = fma(m3[i], rn2, acc[O_G2_3 + i]);
    acc[O_G1_3 + i] = fma(m3[i], rn, acc[O_G1_3 + i]);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) acc[O_G1_2 + i] = fma(m2[i], rn, acc[O_G1_2 + i]);
}

// Trace factor of one landmark without 1/sigma^2: vp(u) Tr(I_i) sigma^2 with
// Tr(I_i) sigma^2 = (2 + |p|^2 + (u.p)^2) / n^2.
template <typename T>
__device__ inline void trace_pair(T acc[10], T dx, T dy, T dz, T rn, T px, T py, T pz, T p2) {
  T rn2 = rn * rn;
  T ux = dx * rn, uy = dy * rn, uz = dz * rn;
  T up = ux * px + uy * py + uz * pz;
  T tr = (T(2) + p2 + up * up) * rn2;
  acc[0] = fma(ux * ux, tr, acc[0]);
  acc[1] = fma(uy * uy, tr, acc[1]);
  acc[2] = fma(uz * uz, tr, acc[2]);
  acc[3] = fma(ux * uy, tr, acc[3]);
  acc[4] = fma(ux * uz, tr, acc[4]);
  acc[5] = fma(uy * uz, tr, acc[5]);
  acc[6] = fma(ux, tr, acc[6]);
  acc[7] = fma(uy, tr, acc[7]);
  acc[8] = fma(uz, tr, acc[8]);
  acc[9] += tr;
}

// A value equal on every lane of the wave, moved to a scalar register.
__device__ inline float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

template <typename T>
__device__ inline T inv_sqrt(T x);
template <>
__device__ inline float inv_sqrt<float>(float x) { return rsq_normal(x); }
template <>
__device__ inline double inv_sqrt<double>(double x) { return 1.0 / sqrt(x); }

// Vector stores of N scalars (16-B aligned destination, N even).
template <typename T, int N>
__device__ inline void store_vec(T* dst, const T* v) {
  if (sizeof(T) == 8 || (N % 4) != 0) {
#pragma unroll
    for (int k = 0; k < N; k += 2) {
      typename std::conditional<sizeof(T) == 8, double2, float2>::type w;
      w.x = v[k];
      w.y = v[k + 1];
      reinterpret_cast<decltype(w)*>(dst)[k / 2] = w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < N; k += 4) {
      float4 w;
      w.x = (float)v[k]; w.y = (float)v[k + 1]; w.z = (float)v[k + 2]; w.w = (float)v[k + 3];
      reinterpret_cast<float4*>(dst)[k / 4] = w;
    }
  }
}

// PREC: FIF_FP32_NAIVE / FIF_FP32_COMP / FIF_FP64; KIND: info or trace.
template <int PREC, int KIND>
__global__ __launch_bounds__(kBuildThreads, 2) void build_kernel(BuildArgs a) {
  using T = typename std::conditional<PREC == 2, double, float>::type;
  using L4 = typename LmT<T>::type;
  constexpr int NACC = (KIND == 0) ? kMom : 10;
  constexpr bool COMP = (PREC == 1);

  __shared__ L4 s_lm[kBatch];
  // the compensated sums' low parts: touched once per batch (in the fold), so
  // they live in LDS, one column per lane, leaving registers to the pair loops
  __shared__ float s_lo[COMP ? NACC : 1][kBuildThreads];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int ix = blockIdx.x * 8 + (wave & 1) * 4 + (lane & 3);
  const int iy = blockIdx.y * 8 + (wave >> 1) * 4 + ((lane >> 2) & 3);
  const int iz = blockIdx.z * 4 + (lane >> 4);
  const bool valid = ix < a.g.nx && iy < a.g.ny && iz < a.g.nz;

  const double tx = a.g.ox + (double)ix * a.g.h;
  const double ty = a.g.oy + (double)iy * a.g.h;
  const double tz = a.g.oz + (double)iz * a.g.h;
  const float fx = (float)tx, fy = (float)ty, fz = (float)tz;
  const T vx = (T)tx, vy = (T)ty, vz = (T)tz;
  // Compensated FP32 fields: a landmark closer to the voxel centre than 1 % of
  // the centre's distance from the origin (or 1 cm) takes its offset d from
  // the FP64 coordinates.  The difference of the FP32-rounded coordinates is
  // off by up to ~6e-8 |t_v| in absolute terms, a large relative error in d
  // when the landmark is that close -- and such a landmark dominates the
  // voxel's 1/n^2 sums.  Rare, so a divergent branch, and only in landmark
  // batches whose box comes that near the tile.  (The naive FP32 sums carry
  // larger rounding errors of their own and skip the test.)
  const float near2 = 1e-4f * (fx * fx + fy * fy + fz * fz) + 1e-4f;

  T acc[NACC];
  float hi[COMP ? NACC : 1];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = T(0);
  if (COMP) {
#pragma unroll
    for (int i = 0; i < NACC; ++i) { hi[i] = 0.f; s_lo[i][tid] = 0.f; }
  }

  // workgroup tile bounds (voxel centres, FP32 like the range test)
  float tlo[3], thi[3];
  float near2_tile = 0.f;  // largest near2 over the tile's voxel centres
  if (a.lm_sorted) {
    const int x0 = blockIdx.x * 8, y0 = blockIdx.y * 8, z0 = blockIdx.z * 4;
    const int x1 = min(x0 + 7, a.g.nx - 1), y1 = min(y0 + 7, a.g.ny - 1), z1 = min(z0 + 3, a.g.nz - 1);
    tlo[0] = (float)(a.g.ox + x0 * a.g.h); thi[0] = (float)(a.g.ox + x1 * a.g.h);
    tlo[1] = (float)(a.g.oy + y0 * a.g.h); thi[1] = (float)(a.g.oy + y1 * a.g.h);
    tlo[2] = (float)(a.g.oz + z0 * a.g.h); thi[2] = (float)(a.g.oz + z1 * a.g.h);
    float m2 = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = fmaxf(fabsf(tlo[c]), fabsf(thi[c]));
      m2 = fmaf(e, e, m2);
    }
    near2_tile = 1.0001f * (1e-4f * m2 + 1e-4f);
#pragma unroll
    for (int c = 0; c < 3; ++c) {  // uniform: keep them in scalar registers
      tlo[c] = uniform_f(tlo[c]);
      thi[c] = uniform_f(thi[c]);
    }
    near2_tile = uniform_f(near2_tile);
  }
  // the wave's own 4x4x4 voxel centres (FP32), for the per-slice decisions of
  // the compensated build; a wave wholly past the grid edge has none
  float wlo[3] = {0.f, 0.f, 0.f}, whi[3] = {0.f, 0.f, 0.f};
  const int wx0 = blockIdx.x * 8 + (wave & 1) * 4, wy0 = blockIdx.y * 8 + (wave >> 1) * 4;
  const bool wave_empty = wx0 >= a.g.nx || wy0 >= a.g.ny || (int)blockIdx.z * 4 >= a.g.nz;
  if (COMP && a.slice_box) {
    const int x0 = wx0, y0 = wy0, z0 = blockIdx.z * 4;
    const int x1 = min(x0 + 3, a.g.nx - 1), y1 = min(y0 + 3, a.g.ny - 1), z1 = min(z0 + 3, a.g.nz - 1);
    wlo[0] = (float)(a.g.ox + x0 * a.g.h); whi[0] = (float)(a.g.ox + x1 * a.g.h);
    wlo[1] = (float)(a.g.oy + y0 * a.g.h); whi[1] = (float)(a.g.oy + y1 * a.g.h);
    wlo[2] = (float)(a.g.oz + z0 * a.g.h); whi[2] = (float)(a.g.oz + z1 * a.g.h);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      wlo[c] = uniform_f(wlo[c]);
      whi[c] = uniform_f(whi[c]);
    }
  }
  for (int64_t base = 0; base < a.L; base += kBatch) {
    const int nb = (int)((a.L - base) < kBatch ? (a.L - base) : kBatch);
    // whether a landmark of this batch can be near a voxel centre of the tile
    // (workgroup-uniform; without the sorted batches' boxes: always)
    bool batch_near = true;
    if (a.lm_sorted) {
      // skip a batch whose box is out of range of the whole tile (workgroup-uniform)
      const float* bb = a.batch_box + 8 * (base / kBatch);
      float d2 = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float gap = fmaxf(fmaxf(bb[c] - thi[c], tlo[c] - bb[3 + c]), 0.f);
        d2 = fmaf(gap, gap, d2);
      }
      if (d2 > a.skip2) continue;
      batch_near = d2 <= near2_tile;
    }
    __syncthreads();
    {
      L4 v;
      if (tid < nb) {
        double px, py, pz;
        if (a.lm_sorted) {
          const double4 p4 = a.lm_sorted[base + tid];
          px = p4.x; py = p4.y; pz = p4.z;
        } else {
          const double* p = a.lm + 3 * (base + tid);
          px = p[0]; py = p[1]; pz = p[2];
        }
        v.x = (T)px; v.y = (T)py; v.z = (T)pz;
        v.w = (T)(px * px + py * py + pz * pz);
      } else {
        // padding past the last landmark: NaN fails the FP32 range test, so
        // the loops below need no bound
        v.x = v.y = v.z = v.w = (T)__builtin_nanf("");
      }
      s_lm[tid] = v;
    }
    __syncthreads();
    // landmarks [ibeg, iend) in groups of 4: the LDS reads of a group are
    // issued together.  INSIDE: every pair is known to pass the range test
    // (lanes past the grid edge then compute pairs they never store); NEAR_TEST:
    // the compensated build's near-landmark test, taken where near_on.
    auto pairs = [&](auto near_test, auto inside, int ibeg, int iend,
                     bool near_on) __attribute__((always_inline)) {
    constexpr bool NEAR_TEST = decltype(near_test)::value;
    constexpr bool INSIDE = decltype(inside)::value;
    for (int i0 = ibeg; i0 < iend; i0 += 4) {
      L4 pg[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) pg[k] = s_lm[i0 + k];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const L4 p = pg[k];
        // V_t range test in FP32 (same decision in every precision)
        float ddx = (float)p.x - fx, ddy = (float)p.y - fy, ddz = (float)p.z - fz;
        float n2 = __fmaf_rn(ddz, ddz, __fmaf_rn(ddy, ddy, ddx * ddx));
        bool in = INSIDE || (valid && (n2 >= a.lo2) && (n2 <= a.hi2));
        if (in) {
          T dx = p.x - vx, dy = p.y - vy, dz = p.z - vz;
          T nn = (PREC == 2)
                     ? (T)fma((double)dz, (double)dz, fma((double)dy, (double)dy, (double)dx * dx))
                     : (T)n2;
          if constexpr (COMP && NEAR_TEST) {
            if (near_on && n2 < near2) {
              const int64_t li = base + i0 + k;
              double qx, qy, qz;
              if (a.lm_sorted) {
                const double4 p4 = a.lm_sorted[li];
                qx = p4.x; qy = p4.y; qz = p4.z;
              } else {
                qx = a.lm[3 * li]; qy = a.lm[3 * li + 1]; qz = a.lm[3 * li + 2];
              }
              dx = (T)(qx - tx); dy = (T)(qy - ty); dz = (T)(qz - tz);
              nn = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
            }
          }
          T rn = inv_sqrt<T>(nn);
          if constexpr (KIND == 0)
            info_pair<T>(acc, dx, dy, dz, rn);
          else
            trace_pair<T>(acc, dx, dy, dz, rn, p.x, p.y, p.z, p.w);
        }
        // with no branch between them the scheduler would interleave the
        // group's pairs, with the temporaries of four pairs live at once
        if constexpr (INSIDE) __builtin_amdgcn_sched_barrier(0);
      }
    }
    };
    const int nb4 = (nb + 3) & ~3;
    // The compensated build goes through a batch in slices of 64 landmarks and
    // decides per wave: skip a slice out of range of the wave's voxels, run a
    // full slice wholly in range of them without the range test, test each
    // pair otherwise.  The pairs and their order are those of one pass over
    // the batch.  (Only the compensated build: it holds 255 VGPRs whatever the
    // loop, while a second copy of the loop costs the other variants
    // occupancy.)
    if constexpr (COMP) {
      if (!wave_empty) {
        for (int sl = 0; 64 * sl < nb; ++sl) {
          bool inside = false, near_on = batch_near;
          if (a.slice_box) {
            const float* sb = a.slice_box + 8 * (4 * (base / kBatch) + sl);
            float d2 = 0.f, far2 = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float gap = fmaxf(fmaxf(sb[c] - whi[c], wlo[c] - sb[3 + c]), 0.f);
              d2 = fmaf(gap, gap, d2);
              const float far = fmaxf(fabsf(sb[3 + c] - wlo[c]), fabsf(whi[c] - sb[c]));
              far2 = fmaf(far, far, far2);
            }
            if (d2 > a.skip2) continue;  // wave-uniform
            near_on = batch_near && d2 <= near2_tile;
            inside = !near_on && 64 * sl + 64 <= nb && d2 >= a.inside_lo2 && far2 <= a.inside_hi2;
          }
          if (inside)
            pairs(std::false_type{}, std::true_type{}, 64 * sl, 64 * sl + 64, false);
          else
            pairs(std::true_type{}, std::false_type{}, 64 * sl, min(64 * sl + 64, nb4), near_on);
        }
      }
    } else {
      pairs(std::false_type{}, std::false_type{}, 0, nb4, false);
    }
    if (COMP) {
#pragma unroll
      for (int k = 0; k < NACC; ++k) {
        float l = s_lo[k][tid];
        two_sum_into(hi[k], l, (float)acc[k]);
        s_lo[k][tid] = l;
        acc[k] = T(0);
      }
    }
  }
  if (!valid) return;
  const size_t vox = (size_t)ix + (size_t)a.g.nx * ((size_t)iy + (size_t)a.g.ny * (size_t)iz);
  const size_t nvox = (size_t)a.g.nx * a.g.ny * a.g.nz;
  T res[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) res[k] = COMP ? (T)(hi[k] + s_lo[k][tid]) : acc[k];
  if constexpr (KIND == 0) {
    T* main = reinterpret_cast<T*>(a.out) + vox * kMain;
    T* side = reinterpret_cast<T*>(a.out) + nvox * kMain + vox * kSideRec;  // slot 0
    if (a.accumulate) {
#pragma unroll
      for (int k = 0; k < kMain; ++k) res[k] = main[k] + (T)a.sign * res[k];
#pragma unroll
      for (int k = 0; k < kSide; ++k) res[kMain + k] = side[k] + (T)a.sign * res[kMain + k];
    }
    store_vec<T, kMain>(main, res);
    store_vec<T, kSide>(side, res + kMain);
  } else if (a.trace_cells) {
    // slot 0 of the voxel's cell block; fill_trace_cells_kernel copies it into
    // the blocks of the cells that have the voxel as another corner
    T* out = reinterpret_cast<T*>(a.out) + vox * kTCell;
    T r10[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) r10[k] = res[k];
    if (a.accumulate) {
#pragma unroll
      for (int k = 0; k < 10; ++k) r10[k] = out[k] + (T)a.sign * r10[k];
    }
    store_vec<T, 10>(out, r10);
  } else {
    T* out = reinterpret_cast<T*>(a.out) + vox * kTRec;
    T r12[kTRec];
#pragma unroll
    for (int k = 0; k < kTRec; ++k) r12[k] = (k < NACC) ? res[k] : T(0);
    if (a.accumulate) {
#pragma unroll
      for (int k = 0; k < NACC; ++k) r12[k] = out[k] + (T)a.sign * r12[k];
    }
    store_vec<T, kTRec>(out, r12);
  }
}

// Slots 1..7 of every trace cell block from slot 0 of the corner voxels' blocks.
template <typename T>
__global__ __launch_bounds__(256) void fill_trace_cells_kernel(GridDev g, void* field) {
  const size_t nvox = (size_t)g.nx * g.ny * g.nz;
  const size_t v = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= nvox) return;
  T* f = reinterpret_cast<T*>(field);
  const int32_t ix = (int32_t)(v % g.nx), iy = (int32_t)((v / g.nx) % g.ny),
                iz = (int32_t)(v / ((size_t)g.nx * g.ny));
#pragma unroll
  for (int s = 1; s < 8; ++s) {
    const int32_t cx = min(ix + (s & 1), g.nx - 1);
    const int32_t cy = min(iy + ((s >> 1) & 1), g.ny - 1);
    const int32_t cz = min(iz + (s >> 2), g.nz - 1);
    const size_t c = (size_t)cx + (size_t)g.nx * ((size_t)cy + (size_t)g.ny * (size_t)cz);
    T vals[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) vals[k] = f[c * kTCell + k];
    store_vec<T, 10>(f + v * kTCell + 10 * s, vals);
  }
}

// Slots 1..7 of every cell side record from slot 0 of the corner voxels' records.
template <typename T>
__global__ __launch_bounds__(256) void fill_side_kernel(GridDev g, void* field) {
  const size_t nvox = (size_t)g.nx * g.ny * g.nz;
  const size_t v = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= nvox) return;
  T* side = reinterpret_cast<T*>(field) + nvox * kMain;
  const int32_t ix = (int32_t)(v % g.nx), iy = (int32_t)((v / g.nx) % g.ny),
                iz = (int32_t)(v / ((size_t)g.nx * g.ny));
  T vals[kSideRec];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int32_t cx = min(ix + (s & 1), g.nx - 1);
    const int32_t cy = min(iy + ((s >> 1) & 1), g.ny - 1);
    const int32_t cz = min(iz + (s >> 2), g.nz - 1);
    const size_t c = (size_t)cx + (size_t)g.nx * ((size_t)cy + (size_t)g.ny * (size_t)cz);
    vals[2 * s] = side[c * kSideRec];
    vals[2 * s + 1] = side[c * kSideRec + 1];
  }
  // slot 0 is unchanged; rewrite slots 1..7 only
#pragma unroll
  for (int k = 2; k < kSideRec; ++k) side[v * kSideRec + k] = vals[k];
}

// ------------------------------------------------------------ spatial sort

// 30-bit Morton code of each landmark inside the box [lo, lo + 1024 q)^3.
__global__ void morton_kernel(const double* lm, int64_t L, double lox, double loy, double loz,
                              double inv_q, uint32_t* keys, uint32_t* idx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= L) return;
  const double p[3] = {lm[3 * i], lm[3 * i + 1], lm[3 * i + 2]};
  const double lo[3] = {lox, loy, loz};
  uint32_t code = 0;
  uint32_t c[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    double g = (p[ax] - lo[ax]) * inv_q;
    g = fmin(fmax(g, 0.0), 1023.0);  // NaN -> 0
    c[ax] = (uint32_t)g;
  }
#pragma unroll
  for (int b = 9; b >= 0; --b)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) code = (code << 1) | ((c[ax] >> b) & 1u);
  keys[i] = code;
  idx[i] = (uint32_t)i;
}

// 30-bit Morton code of the cell of each of n points (x, y, z at stride 3):
// cell index floor(x * inv_cell) per axis, taken modulo 1024, so points far
// apart may share a code (that only costs culling, never a result).  The cell
// size does not depend on the data, so the order is reproducible from the
// coordinates alone.  idx[i] = i.
template <typename T>
__global__ void morton_cell_kernel(const T* xyz, int64_t n, double inv_cell, uint32_t* keys,
                                   uint32_t* idx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint32_t c[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    double g = floor((double)xyz[3 * i + ax] * inv_cell);
    g = fmin(fmax(g, -1.0e18), 1.0e18);  // NaN -> -1e18
    c[ax] = (uint32_t)((long long)g & 1023);
  }
  uint32_t code = 0;
#pragma unroll
  for (int b = 9; b >= 0; --b)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) code = (code << 1) | ((c[ax] >> b) & 1u);
  keys[i] = code;
  idx[i] = (uint32_t)i;
}

// Sorted landmarks and the FP32 bounding box of each batch of kBatch, and
// (when slices != nullptr) of each slice of 64 landmarks: slices[8 (4 b + s) +
// c] (min xyz, max xyz, 2 pad; an empty slice gets min = +inf, max = -inf).
__global__ __launch_bounds__(kBatch) void gather_box_kernel(const double* lm, int64_t L,
                                                            const uint32_t* idx, double4* out,
                                                            float* boxes, float* slices) {
  __shared__ float s_min[3][kBatch], s_max[3][kBatch];
  const int64_t i = (int64_t)blockIdx.x * kBatch + threadIdx.x;
  float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (i < L) {
    const int64_t j = idx[i];
    const double x = lm[3 * j], y = lm[3 * j + 1], z = lm[3 * j + 2];
    double4 v;
    v.x = x; v.y = y; v.z = z; v.w = 0.0;
    out[i] = v;
    mn[0] = mx[0] = (float)x;
    mn[1] = mx[1] = (float)y;
    mn[2] = mx[2] = (float)z;
  }
  if (slices) {
    float v[6] = {mn[0], mn[1], mn[2], -mx[0], -mx[1], -mx[2]};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = fminf(v[c], __shfl_xor(v[c], off, 64));
    if ((threadIdx.x & 63) < 8) {
      const int c = threadIdx.x & 63;
      float w = 0.f;
#pragma unroll
      for (int k = 0; k < 6; ++k) w = (c == k) ? (k < 3 ? v[k] : -v[k]) : w;
      slices[8 * (4 * (int64_t)blockIdx.x + (threadIdx.x >> 6)) + c] = w;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) { s_min[c][threadIdx.x] = mn[c]; s_max[c][threadIdx.x] = mx[c]; }
  __syncthreads();
  for (int stride = kBatch / 2; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_min[c][threadIdx.x] = fminf(s_min[c][threadIdx.x], s_min[c][threadIdx.x + stride]);
        s_max[c][threadIdx.x] = fmaxf(s_max[c][threadIdx.x], s_max[c][threadIdx.x + stride]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) {
    float v = 0.f;
    if (threadIdx.x < 3) v = s_min[threadIdx.x][0];
    else if (threadIdx.x < 6) v = s_max[threadIdx.x - 3][0];
    boxes[8 * blockIdx.x + threadIdx.x] = v;
  }
}

namespace {
struct SortLayout {
  size_t keys_in, keys_out, idx_in, idx_out, sorted, boxes, slices, tmp, total;
};
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
SortLayout sort_layout(int64_t L, size_t tmp_bytes) {
  SortLayout s;
  size_t off = 0;
  s.keys_in = off; off = align256(off + 4 * (size_t)L);
  s.keys_out = off; off = align256(off + 4 * (size_t)L);
  s.idx_in = off; off = align256(off + 4 * (size_t)L);
  s.idx_out = off; off = align256(off + 4 * (size_t)L);
  s.sorted = off; off = align256(off + 32 * (size_t)L);
  s.boxes = off; off = align256(off + 32 * (size_t)((L + kBatch - 1) / kBatch));
  s.slices = off; off = align256(off + 128 * (size_t)((L + kBatch - 1) / kBatch));
  s.tmp = off; off = align256(off + tmp_bytes);
  s.total = off;
  return s;
}
size_t radix_tmp_bytes(int64_t L) {
  size_t bytes = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (size_t)L, 0, 30);
  return e == hipSuccess ? bytes : 0;
}
}  // namespace

namespace {
struct CellSortLayout {
  size_t keys_in, keys_out, idx_in, idx_out, tmp, total;
};
CellSortLayout cell_sort_layout(int64_t n, size_t tmp_bytes) {
  CellSortLayout s;
  size_t off = 0;
  s.keys_in = off; off = align256(off + 4 * (size_t)n);
  s.keys_out = off; off = align256(off + 4 * (size_t)n);
  s.idx_in = off; off = align256(off + 4 * (size_t)n);
  s.idx_out = off; off = align256(off + 4 * (size_t)n);
  s.tmp = off; off = align256(off + tmp_bytes);
  s.total = off;
  return s;
}
}  // namespace

size_t cell_sort_bytes(int64_t n) {
  if (n <= 0) return 0;
  const size_t tmp = radix_tmp_bytes(n);
  return tmp == 0 ? 0 : cell_sort_layout(n, tmp).total;
}

hipError_t cell_sort(const void* xyz, bool dbl, int64_t n, double inv_cell, void* ws,
                     size_t ws_bytes, hipStream_t stream, const uint32_t** order) {
  const size_t tmp = radix_tmp_bytes(n);
  const CellSortLayout lay = cell_sort_layout(n, tmp);
  if (tmp == 0 || ws_bytes < lay.total) return hipErrorInvalidValue;
  char* base = reinterpret_cast<char*>(ws);
  uint32_t* kin = reinterpret_cast<uint32_t*>(base + lay.keys_in);
  uint32_t* kout = reinterpret_cast<uint32_t*>(base + lay.keys_out);
  uint32_t* iin = reinterpret_cast<uint32_t*>(base + lay.idx_in);
  uint32_t* iout = reinterpret_cast<uint32_t*>(base + lay.idx_out);
  const unsigned nblk = (unsigned)((n + 255) / 256);
  if (dbl)
    hipLaunchKernelGGL((morton_cell_kernel<double>), dim3(nblk), dim3(256), 0, stream,
                       static_cast<const double*>(xyz), n, inv_cell, kin, iin);
  else
    hipLaunchKernelGGL((morton_cell_kernel<float>), dim3(nblk), dim3(256), 0, stream,
                       static_cast<const float*>(xyz), n, inv_cell, kin, iin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = tmp;
  e = rocprim::radix_sort_pairs(base + lay.tmp, tb, kin, kout, iin, iout, (size_t)n, 0, 30,
                                stream);
  if (e != hipSuccess) return e;
  *order = iout;
  return hipSuccess;
}

size_t cell_sorted_landmarks_bytes(int64_t L) {
  const size_t cs = cell_sort_bytes(L);
  if (cs == 0) return 0;
  return cs + align256(32 * (size_t)L) + align256(32 * (size_t)((L + kBatch - 1) / kBatch));
}

hipError_t cell_sort_landmarks(const double* lm, int64_t L, double inv_cell, void* ws,
                               size_t ws_bytes, hipStream_t stream, const double4** sorted,
                               const float** boxes) {
  const size_t cs = cell_sort_bytes(L);
  if (cs == 0 || ws_bytes < cell_sorted_landmarks_bytes(L)) return hipErrorInvalidValue;
  const uint32_t* order = nullptr;
  hipError_t e = cell_sort(lm, true, L, inv_cell, ws, cs, stream, &order);
  if (e != hipSuccess) return e;
  char* base = reinterpret_cast<char*>(ws) + cs;
  double4* out = reinterpret_cast<double4*>(base);
  float* bx = reinterpret_cast<float*>(base + align256(32 * (size_t)L));
  const unsigned nbatch = (unsigned)((L + kBatch - 1) / kBatch);
  hipLaunchKernelGGL(gather_box_kernel, dim3(nbatch), dim3(kBatch), 0, stream, lm, L, order, out,
                     bx, nullptr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  *sorted = out;
  *boxes = bx;
  return hipSuccess;
}

size_t sort_workspace_bytes(int64_t L) {
  if (L <= 0) return 0;
  size_t tmp = radix_tmp_bytes(L);
  if (tmp == 0) return 0;
  return sort_layout(L, tmp).total;
}

hipError_t sort_landmarks(BuildArgs& a, void* ws, size_t ws_bytes, hipStream_t stream) {
  const size_t tmp = radix_tmp_bytes(a.L);
  const SortLayout lay = sort_layout(a.L, tmp);
  if (tmp == 0 || ws_bytes < lay.total) return hipErrorInvalidValue;
  char* base = reinterpret_cast<char*>(ws);
  uint32_t* kin = reinterpret_cast<uint32_t*>(base + lay.keys_in);
  uint32_t* kout = reinterpret_cast<uint32_t*>(base + lay.keys_out);
  uint32_t* iin = reinterpret_cast<uint32_t*>(base + lay.idx_in);
  uint32_t* iout = reinterpret_cast<uint32_t*>(base + lay.idx_out);
  // quantisation box: the voxel-centre hull grown by the range (or by 1/4 of
  // the hull when the range is unbounded); landmarks outside are clamped
  const double ext[3] = {(a.g.nx - 1) * a.g.h, (a.g.ny - 1) * a.g.h, (a.g.nz - 1) * a.g.h};
  double emax = fmax(ext[0], fmax(ext[1], ext[2]));
  double margin = std::isinf((double)a.hi2) ? 0.25 * emax + a.g.h : sqrt((double)a.hi2) + a.g.h;
  const double lo[3] = {a.g.ox - margin, a.g.oy - margin, a.g.oz - margin};
  const double span = emax + 2.0 * margin;
  const double inv_q = 1024.0 / span;
  const unsigned nblk = (unsigned)((a.L + 255) / 256);
  hipLaunchKernelGGL(morton_kernel, dim3(nblk), dim3(256), 0, stream, a.lm, a.L, lo[0], lo[1],
                     lo[2], inv_q, kin, iin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = tmp;
  e = rocprim::radix_sort_pairs(base + lay.tmp, tb, kin, kout, iin, iout, (size_t)a.L, 0, 30,
                                stream);
  if (e != hipSuccess) return e;
  double4* sorted = reinterpret_cast<double4*>(base + lay.sorted);
  float* boxes = reinterpret_cast<float*>(base + lay.boxes);
  float* slices = reinterpret_cast<float*>(base + lay.slices);
  const unsigned nbatch = (unsigned)((a.L + kBatch - 1) / kBatch);
  hipLaunchKernelGGL(gather_box_kernel, dim3(nbatch), dim3(kBatch), 0, stream, a.lm, a.L, iout,
                     sorted, boxes, slices);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  a.lm_sorted = sorted;
  a.batch_box = boxes;
  a.slice_box = slices;
  // conservative skip distance: every landmark of a skipped batch is beyond the
  // FP32 range test with a margin far above FP32 rounding
  a.skip2 = std::isinf(a.hi2) ? INFINITY : a.hi2 * 1.0001f + 1e-3f;
  // margins far above the FP32 rounding of n^2 and of the box distances
  a.inside_lo2 = a.lo2 * 1.0001f + 1e-6f;
  a.inside_hi2 = std::isinf(a.hi2) ? INFINITY : a.hi2 * 0.9999f - 1e-3f;
  return hipSuccess;
}

hipError_t launch_build(const BuildArgs& a, int prec, int kind, hipStream_t stream) {
  dim3 grid((a.g.nx + 7) / 8, (a.g.ny + 7) / 8, (a.g.nz + 3) / 4);
  dim3 block(kBuildThreads);
#define FIF_LAUNCH(P, K) hipLaunchKernelGGL((build_kernel<P, K>), grid, block, 0, stream, a)
  if (kind == 0) {
    if (prec == 0) FIF_LAUNCH(0, 0);
    else if (prec == 1) FIF_LAUNCH(1, 0);
    else FIF_LAUNCH(2, 0);
  } else {
    if (prec == 0) FIF_LAUNCH(0, 1);
    else if (prec == 1) FIF_LAUNCH(1, 1);
    else FIF_LAUNCH(2, 1);
  }
#undef FIF_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || kind == 1) return e;
  const size_t nvox = (size_t)a.g.nx * a.g.ny * a.g.nz;
  dim3 sgrid((unsigned)((nvox + 255) / 256));
  if (kind == 2) {
    if (prec == 2)
      hipLaunchKernelGGL((fill_trace_cells_kernel<double>), sgrid, dim3(256), 0, stream, a.g, a.out);
    else
      hipLaunchKernelGGL((fill_trace_cells_kernel<float>), sgrid, dim3(256), 0, stream, a.g, a.out);
    return hipGetLastError();
  }
  if (prec == 2)
    hipLaunchKernelGGL((fill_side_kernel<double>), sgrid, dim3(256), 0, stream, a.g, a.out);
  else
    hipLaunchKernelGGL((fill_side_kernel<float>), sgrid, dim3(256), 0, stream, a.g, a.out);
  return hipGetLastError();
}

}  // namespace fif
