// Per-query position data shared by the query kernels: trilinear corners,
// pose loading, the per-query slot a lane computes for its group, and a
// wave-level LDS barrier.
#pragma once

#include "fif_kernels.h"

namespace fif {

struct Corner {
  size_t vox;
  double w;
  double dw[3];
  double dl[3];  // voxel centre - query position
  bool clamped;
  bool active;
};

// Corner j (bits x, y, z) of the cell holding t, or the nearest voxel for j = 0.
__device__ inline Corner make_corner(const GridDev& g, const double t[3], int j, int interp) {
  Corner c;
  const double o[3] = {g.ox, g.oy, g.oz};
  const int32_t n[3] = {g.nx, g.ny, g.nz};
  int32_t idx[3];
  if (interp == 1) {
    bool cl[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) idx[ax] = axis_nearest(t[ax], o[ax], g.h, n[ax], &cl[ax]);
    c.clamped = cl[0] || cl[1] || cl[2];
    c.active = (j == 0);
    // NaN positions must give NaN results
    double nanp = (t[0] - t[0]) + (t[1] - t[1]) + (t[2] - t[2]);
    c.w = c.active ? 1.0 + nanp : 0.0;
    c.dw[0] = c.dw[1] = c.dw[2] = 0.0;
  } else {
    double wc[3], dwc[3];
    c.clamped = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      AxisCell ac = axis_cell(t[ax], o[ax], g.h, n[ax]);
      int b = (j >> ax) & 1;
      idx[ax] = ac.i0 + b * ac.step;
      wc[ax] = b ? ac.f : 1.0 - ac.f;
      dwc[ax] = b ? ac.df : -ac.df;
      c.clamped = c.clamped || ac.clamped;
    }
    c.active = true;
    c.w = wc[0] * wc[1] * wc[2];
    c.dw[0] = dwc[0] * wc[1] * wc[2];
    c.dw[1] = wc[0] * dwc[1] * wc[2];
    c.dw[2] = wc[0] * wc[1] * dwc[2];
  }
  c.vox = (size_t)idx[0] + (size_t)g.nx * ((size_t)idx[1] + (size_t)g.ny * (size_t)idx[2]);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) c.dl[ax] = (o[ax] + (double)idx[ax] * g.h) - t[ax];
  return c;
}

template <typename PT>
__device__ inline void load_pose(const QueryArgs& a, int64_t i, double t[3], double z[3]) {
  const PT* T = reinterpret_cast<const PT*>(a.t);
  const PT* Q = reinterpret_cast<const PT*>(a.q);
  t[0] = (double)T[3 * i]; t[1] = (double)T[3 * i + 1]; t[2] = (double)T[3 * i + 2];
  quat_axis((double)Q[4 * i], (double)Q[4 * i + 1], (double)Q[4 * i + 2], (double)Q[4 * i + 3], z);
}

// Per-query data computed once by the lane that owns the query and read by
// the 8 corner lanes of its group through LDS.
template <typename CT>
struct QSlot {
  CT t[3];   // frame point: the position clamped to the hull of voxel centres
  CT z[3];   // optical axis
  CT f[3];   // trilinear fractions
  CT df[3];  // d f / d t (1/h, or 0 where clamped)
  int32_t i0[3];
  int32_t bits;  // bit ax: axis has two voxels; bit 3: clamped; bit 4: nearest mode
};

template <typename FT>
__device__ inline QSlot<FT> make_slot_from(const QueryArgs& a, double t[3], double z[3]);

template <typename FT>
__device__ inline QSlot<FT> make_slot(const QueryArgs& a, int64_t i) {
  double t[3], z[3];
  load_pose<FT>(a, i, t, z);
  return make_slot_from<FT>(a, t, z);
}

template <typename FT>
__device__ inline QSlot<FT> make_slot_from(const QueryArgs& a, double t[3], double z[3]) {
  QSlot<FT> s;
  const double o[3] = {a.g.ox, a.g.oy, a.g.oz};
  const int32_t n[3] = {a.g.nx, a.g.ny, a.g.nz};
  int32_t bits = 0;
  bool cl = false;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    // Frame point of the per-corner shifts: the position clamped to the hull of
    // voxel centres (the result does not depend on it in exact arithmetic; the
    // clamped point keeps the shifts no longer than a cell diagonal).
    const double hi = o[ax] + (double)(n[ax] - 1) * a.g.h;
    s.t[ax] = (FT)fmin(fmax(t[ax], o[ax]), hi);
    s.z[ax] = (FT)z[ax];
    if (a.interp == 1) {
      bool c;
      s.i0[ax] = axis_nearest(t[ax], o[ax], a.g.h, n[ax], &c);
      cl = cl || c;
      // NaN positions must give NaN results: carry NaN in the fraction
      s.f[ax] = (FT)(t[ax] - t[ax]);
      s.df[ax] = 0;
    } else {
      AxisCell c = axis_cell(t[ax], o[ax], a.g.h, n[ax]);
      s.i0[ax] = c.i0;
      s.f[ax] = (FT)c.f;
      s.df[ax] = (FT)c.df;
      bits |= c.step << ax;
      cl = cl || c.clamped;
    }
  }
  s.bits = bits | (cl ? 8 : 0) | (a.interp == 1 ? 16 : 0);
  return s;
}

template <typename CT>
struct CornerC {
  size_t vox, cell;
  CT w, dw[3], dl[3];
  bool active;
};

template <typename CT>
__device__ inline CornerC<CT> slot_corner(const QSlot<CT>& s, const GridDev& g, int j) {
  CornerC<CT> c;
  const double o[3] = {g.ox, g.oy, g.oz};
  int32_t idx[3];
  CT wc[3], dwc[3];
  const bool nearest = (s.bits & 16) != 0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int b = (j >> ax) & 1;
    const int step = (s.bits >> ax) & 1;
    idx[ax] = s.i0[ax] + b * step;
    wc[ax] = nearest ? CT(1) + s.f[ax] : (b ? s.f[ax] : CT(1) - s.f[ax]);
    dwc[ax] = b ? s.df[ax] : -s.df[ax];
  }
  c.active = !nearest || j == 0;
  c.w = wc[0] * wc[1] * wc[2];
  c.dw[0] = dwc[0] * wc[1] * wc[2];
  c.dw[1] = wc[0] * dwc[1] * wc[2];
  c.dw[2] = wc[0] * wc[1] * dwc[2];
  c.vox = (size_t)idx[0] + (size_t)g.nx * ((size_t)idx[1] + (size_t)g.ny * (size_t)idx[2]);
  c.cell = (size_t)s.i0[0] + (size_t)g.nx * ((size_t)s.i0[1] + (size_t)g.ny * (size_t)s.i0[2]);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
    c.dl[ax] = (CT)((o[ax] + (double)idx[ax] * g.h) - (double)s.t[ax]);
  return c;
}

// Orders the LDS writes of a wave before its later LDS reads (lanes of one
// wave exchange data through LDS without a workgroup barrier).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace fif
