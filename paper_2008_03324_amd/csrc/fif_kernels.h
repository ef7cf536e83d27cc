// Kernel argument blocks and launchers shared by the kernel files and the
// C-ABI layer.  Host code only sees these declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>

#include "fif_device.h"

namespace fif {

struct BuildArgs {
  const double* lm;  // [L][3]
  int64_t L;
  // spatially sorted landmarks (x, y, z, |p|^2) and per-batch bounding boxes
  // (min xyz, max xyz, 2 pad) in FP32; null for the unsorted path
  const double4* lm_sorted;
  const float* batch_box;
  const float* slice_box;  // boxes of each 64 landmarks of a batch (4 per batch)
  float skip2;  // a batch is skipped when its box is farther than this (squared)
  // a slice whose box lies between these (squared, nearest and farthest
  // points) from a wave's voxels is in range of every voxel centre of them
  float inside_lo2, inside_hi2;
  GridDev g;
  float lo2, hi2;  // FP32 range bounds on n^2
  void* out;       // field records
  int32_t accumulate;  // 0: overwrite, 1: out += sign * contribution
  int32_t sign;
  int32_t trace_cells;  // trace factors stored per cell (slot 0 written here)
};

struct VisDev {
  double k2, k1, k0;  // quadratic visibility coefficients
  double inv_s2;      // 1 / sigma^2
};

struct QueryArgs {
  const void* field;
  GridDev g;
  VisDev vis;
  const void* t;  // [m][3] float or double
  const void* q;  // [m][4]
  int64_t m;
  uint32_t metrics;
  int32_t ncols;
  int32_t interp;
  double* out;
  uint8_t* flags;
  // gradient
  const double* dL_dout;
  void* dL_dt;
  void* dL_dphi;
};

struct PcArgs {
  const double* lm;
  int64_t L;
  float lo2, hi2;
  VisDev vis;
  int32_t exact;
  double fx, fy, cx, cy;
  double width, height;
  const void* t;
  const void* q;
  int64_t m;
  uint32_t metrics;
  int32_t ncols;
  double* out;
  // sorted path (null for the plain one): landmarks in cell order with FP32
  // boxes of each batch, a batch skipped by a workgroup whose poses' box is
  // farther than sqrt(skip2) from it, and the pose order (lane i of the launch
  // takes pose perm[i] and writes its row)
  const double4* lm_sorted;
  const float* batch_box;
  float skip2;
  const uint32_t* perm;
  double inv_cell;  // 32 / r_max: cells of the spatial order
};

struct ExportArgs {
  const void* field;
  GridDev g;
  double inv_s2;
  const int64_t* ids;
  int64_t n;
  double* out;
};

struct SweepArgs {
  const void* field;
  GridDev g;
  VisDev vis;
  const void* t;
  int64_t n_pos;
  const double* dirs;
  int64_t n_dir;
  uint32_t metric;
  int32_t interp;
  double* values;
  int64_t* best;
};

// GP visibility model on the device (Sec. V-B).
struct GPDev {
  int32_t ns;
  double ks;          // sigmoid slope
  double cos_a;       // cos(alpha)
  double inv_2l2;     // 1 / (2 l^2)
  double noise;
  const double* axes;  // [ns][3]
  const double* kinv;  // [ns][ns]
};

struct GPBuildArgs {
  const double* lm;
  int64_t L;
  const double4* lm_sorted;  // null for the unsorted path
  const float* batch_box;
  float skip2;
  GridDev g;
  float lo2, hi2;
  GPDev gp;
  void* out;
  int64_t stride;  // scalars per voxel
};

struct GPQueryArgs {
  QueryArgs q;  // field, grid, vis (inv_s2), poses, metrics, outputs
  GPDev gp;
  int64_t stride;
};

struct GPExportArgs {
  const void* field;
  GridDev g;
  double inv_s2;
  GPDev gp;
  int64_t stride;
  const int64_t* ids;
  int64_t n;
  double* out;
};

// Items (lanes) per launch of the kernels that give every pose, voxel id or
// position its own lane(s): a dispatch holds its grid size in work-items as a
// 32-bit number, so the launchers split longer inputs into launches of at
// most this many work-items, each on a slice of the arrays.
constexpr int64_t kMaxLaunchItems = int64_t(1) << 30;

// Poses [off, off + n) of a query: the pose, output, flag and gradient arrays
// advanced by off rows (sb = bytes of one pose scalar).
inline QueryArgs query_part(const QueryArgs& a, int64_t off, int64_t n, size_t sb) {
  QueryArgs p = a;
  p.t = static_cast<const char*>(a.t) + (size_t)off * 3 * sb;
  p.q = static_cast<const char*>(a.q) + (size_t)off * 4 * sb;
  p.m = n;
  if (a.out) p.out = a.out + (size_t)off * a.ncols;
  if (a.flags) p.flags = a.flags + off;
  if (a.dL_dout) p.dL_dout = a.dL_dout + (size_t)off * a.ncols;
  if (a.dL_dt) p.dL_dt = static_cast<char*>(a.dL_dt) + (size_t)off * 3 * sb;
  if (a.dL_dphi) p.dL_dphi = static_cast<char*>(a.dL_dphi) + (size_t)off * 3 * sb;
  return p;
}

// Sets the calling thread's fif_last_error() text.
void set_last_error(const std::string& msg);
// Compute units of the calling thread's current device (cached).
int current_device_cus();

hipError_t launch_build(const BuildArgs& a, int prec, int kind, hipStream_t stream);
hipError_t launch_gp_setup(const GPDev& gp, double* kinv, hipStream_t stream);
hipError_t launch_gp_evidence(const GPDev& gp, const double* train_u, int32_t n_train,
                              const double* lengths, int32_t n_len, double* lml,
                              hipStream_t stream);
hipError_t launch_gp_build(const GPBuildArgs& a, int prec, int kind, hipStream_t stream);
hipError_t launch_gp_query(const GPQueryArgs& a, int prec, int kind, hipStream_t stream);
hipError_t launch_gp_export(const GPExportArgs& a, int prec, int kind, hipStream_t stream);
hipError_t launch_sweep(const SweepArgs& a, int prec, hipStream_t stream);
// Workspace of the sorted build: bytes needed, and the sort itself (fills
// a.lm_sorted / a.batch_box inside `ws`).
size_t sort_workspace_bytes(int64_t L);
hipError_t sort_landmarks(BuildArgs& a, void* ws, size_t ws_bytes, hipStream_t stream);
hipError_t launch_query(const QueryArgs& a, int prec, int kind, bool grad, hipStream_t stream);
hipError_t launch_pc(const PcArgs& a, int prec, hipStream_t stream);
// Order of n points (x, y, z at stride 3; double or float) by the Morton code
// of their cell of edge 1 / inv_cell (cell indices modulo 1024): scratch bytes,
// and the stable sort itself (*order points into ws).
size_t cell_sort_bytes(int64_t n);
hipError_t cell_sort(const void* xyz, bool dbl, int64_t n, double inv_cell, void* ws,
                     size_t ws_bytes, hipStream_t stream, const uint32_t** order);
// Landmarks copied in that order with the FP32 box of each batch of 256.
size_t cell_sorted_landmarks_bytes(int64_t L);
hipError_t cell_sort_landmarks(const double* lm, int64_t L, double inv_cell, void* ws,
                               size_t ws_bytes, hipStream_t stream, const double4** sorted,
                               const float** boxes);
// Sorted, culled point cloud: workspace bytes, and the whole pass.
size_t pc_sorted_workspace_bytes(int64_t L, int64_t m);
hipError_t launch_pc_sorted(PcArgs a, int prec, void* ws, size_t ws_bytes, hipStream_t stream);
hipError_t launch_export(const ExportArgs& a, int prec, int kind, hipStream_t stream);

}  // namespace fif
