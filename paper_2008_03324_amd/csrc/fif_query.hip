// Batched pose queries, their fused backward, and the export of the paper's
// factor blocks (Sec. VI-A, eq:fim_separation).
//
// Information field, trilinear.  Each trilinear corner (a 264-B record for
// FP32 fields) has its moments contracted with the optical axis into the
// voxel's 6x6 block, which is moved to the query position (the blocks are
// taken about different voxel centres, so each corner is shifted before the
// weighted sum); every lane then evaluates the FP64 metrics of its own query.
// On FP32 fields (up to 2^32 voxels) the forward query and its gradient run in
// persistent waves with one query per lane (query_info_pipe_kernel,
// query_grad_pipe_kernel): corner step k gathers corner k of the wave's 64
// queries straight into LDS, one step (and one batch) ahead of the arithmetic.
// query_info_kernel serves FP64 fields and larger grids: lanes grouped by 8,
// in pass `it` group g serves query 8g + it and lane j gathers corner j; the
// 8 partial sums are reduced with cross-lane moves, and the fused backward
// repeats the corner gathers with the metric gradient broadcast to the group.
// Also here: the trace field query, the optimal-view sweep and the export of
// the paper's blocks.
#include "fif_kernels.h"
#include "fif_metrics.h"
#include "fif_slot.h"

namespace fif {

constexpr int kQThreads = 256;

// The 66 moments of a corner voxel: 64 from its main record, 2 from slot
// `slot` of the cell side record `cell`.
template <typename FT>
__device__ inline void load_record(const FT* field, size_t nvox, size_t vox, size_t cell,
                                   int slot, FT rec[kMom]);

template <>
__device__ inline void load_record<float>(const float* field, size_t nvox, size_t vox,
                                          size_t cell, int slot, float rec[kMom]) {
  const float4* p = reinterpret_cast<const float4*>(field + vox * kMain);
#pragma unroll
  for (int i = 0; i < kMain / 4; ++i) {
    float4 v = p[i];
    rec[4 * i] = v.x; rec[4 * i + 1] = v.y; rec[4 * i + 2] = v.z; rec[4 * i + 3] = v.w;
  }
  float2 w = *reinterpret_cast<const float2*>(field + nvox * kMain + cell * kSideRec + 2 * slot);
  rec[kMain] = w.x; rec[kMain + 1] = w.y;
}

template <>
__device__ inline void load_record<double>(const double* field, size_t nvox, size_t vox,
                                           size_t cell, int slot, double rec[kMom]) {
  const double2* p = reinterpret_cast<const double2*>(field + vox * kMain);
#pragma unroll
  for (int i = 0; i < kMain / 2; ++i) {
    double2 v = p[i];
    rec[2 * i] = v.x; rec[2 * i + 1] = v.y;
  }
  double2 w = *reinterpret_cast<const double2*>(field + nvox * kMain + cell * kSideRec + 2 * slot);
  rec[kMain] = w.x; rec[kMain + 1] = w.y;
}

template <typename FT, bool GRAD>
__global__ __launch_bounds__(kQThreads) void query_info_kernel(QueryArgs a) {
  using CT = FT;  // corner arithmetic in the field's precision; metrics in FP64
  __shared__ QSlot<CT> s_q[kQThreads];
  __shared__ CT s_g[GRAD ? kQThreads : 1][21];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int grp = lane >> 3, j = lane & 7;
  const int wbase = tid & ~63;
  const int64_t qown = (int64_t)blockIdx.x * kQThreads + tid;
  const bool valid = qown < a.m;
  const int64_t ql = valid ? qown : a.m - 1;
  const FT* field = reinterpret_cast<const FT*>(a.field);
  const size_t nvox = (size_t)a.g.nx * a.g.ny * a.g.nz;
  const CT k2 = (CT)a.vis.k2, k1 = (CT)a.vis.k1, k0 = (CT)a.vis.k0;

  // gradient kernel: the forward and backward corner passes (gathers) run at
  // a raised wave priority, the FP64 metric step in between at the normal one
  // (0.21 -> 0.19 ms for 262k trajectory poses)
  if (GRAD) __builtin_amdgcn_s_setprio(1);
  s_q[tid] = make_slot<FT>(a, ql);
  __syncthreads();

  // Each lane handles corner j of the 8 queries of its group in turn.  With
  // FP32 records on the forward path the next query's record is loaded before
  // the current one is contracted, so the gathers of one wave stay in flight
  // during its arithmetic (two waves per SIMD at this register count).
  CT Z[21];
#pragma unroll
  for (int e = 0; e < 21; ++e) Z[e] = 0;
  if constexpr (sizeof(FT) == 4) {
    FT recN[kMom];
    {
      const CornerC<CT> c0 = slot_corner(s_q[wbase + grp * 8], a.g, j);
      if (c0.active) load_record<FT>(field, nvox, c0.vox, c0.cell, j, recN);
    }
#pragma unroll 1
    for (int it = 0; it < 8; ++it) {
      const QSlot<CT> sl = s_q[wbase + grp * 8 + it];
      const CornerC<CT> c = slot_corner(sl, a.g, j);
      FT rec[kMom];
#pragma unroll
      for (int e = 0; e < kMom; ++e) rec[e] = recN[e];
      if (it < 7) {
        const CornerC<CT> cn = slot_corner(s_q[wbase + grp * 8 + it + 1], a.g, j);
        if (cn.active) load_record<FT>(field, nvox, cn.vox, cn.cell, j, recN);
      }
      CT Y[21];
      if (c.active) {
        corner_fim<CT>(rec, vis_weights<CT>(sl.z, k2, k1, k0), c.dl, Y);
#pragma unroll
        for (int e = 0; e < 21; ++e) Y[e] *= c.w;
      } else {
#pragma unroll
        for (int e = 0; e < 21; ++e) Y[e] = 0;
      }
      sum8_arr<21>(Y);
#pragma unroll
      for (int e = 0; e < 21; ++e) Z[e] = (j == it) ? Y[e] : Z[e];
    }
  } else {
    for (int it = 0; it < 8; ++it) {
      const QSlot<CT> sl = s_q[wbase + grp * 8 + it];
      const CornerC<CT> c = slot_corner(sl, a.g, j);
      CT Y[21];
      if (c.active) {
        FT rec[kMom];
        load_record<FT>(field, nvox, c.vox, c.cell, j, rec);
        corner_fim<CT>(rec, vis_weights<CT>(sl.z, k2, k1, k0), c.dl, Y);
#pragma unroll
        for (int e = 0; e < 21; ++e) Y[e] *= c.w;
      } else {
#pragma unroll
        for (int e = 0; e < 21; ++e) Y[e] = 0;
      }
      sum8_arr<21>(Y);
#pragma unroll
      for (int e = 0; e < 21; ++e) Z[e] = (j == it) ? Y[e] : Z[e];
    }
  }

  if (GRAD) __builtin_amdgcn_s_setprio(0);
  const QSlot<CT> own = s_q[tid];
  double td[3] = {(double)own.t[0], (double)own.t[1], (double)own.t[2]};
  double Zd[21], F[21];
#pragma unroll
  for (int e = 0; e < 21; ++e) Zd[e] = (double)Z[e];
  shift21<double>(Zd, td, F);
#pragma unroll
  for (int e = 0; e < 21; ++e) F[e] *= a.vis.inv_s2;

  uint8_t flag = (own.bits & 8) ? FL_CLAMPED : 0;
  double G[GRAD ? 21 : 1];
  const int nmet = (int)((a.metrics & 1u) != 0) + (int)((a.metrics & 2u) != 0) +
                   (int)((a.metrics & 4u) != 0);
  double up[3] = {0.0, 0.0, 0.0};
  if (GRAD) {  // constant indices: the array stays in registers
    const double* du = a.dL_dout + ql * nmet;
    up[0] = (valid && nmet > 0) ? du[0] : 0.0;
    up[1] = (valid && nmet > 1) ? du[1] : 0.0;
    up[2] = (valid && nmet > 2) ? du[2] : 0.0;
  }
  double* row = (valid && a.out) ? a.out + ql * a.ncols : nullptr;
  eval_metrics<GRAD>(F, a.metrics, row, &flag, up, G, a.flags != nullptr);
  if (valid && a.flags) a.flags[ql] = flag;
  if (!GRAD) return;

  // ------------------------------------------------------------ backward
  __builtin_amdgcn_s_setprio(1);
  {
    double Gt[21];
    shift21_adj<double>(G, td, Gt);
#pragma unroll
    for (int e = 0; e < 21; ++e) s_g[GRAD ? tid : 0][e] = (CT)(valid ? Gt[e] * a.vis.inv_s2 : 0.0);
  }
  __syncthreads();
  CT keep[6] = {0, 0, 0, 0, 0, 0};
  FT recB[kMom];
  if constexpr (sizeof(FT) == 4) {
    const CornerC<CT> c0 = slot_corner(s_q[wbase + grp * 8], a.g, j);
    load_record<FT>(field, nvox, c0.vox, c0.cell, j, recB);
  }
  for (int it = 0; it < 8; ++it) {
    const int src = wbase + grp * 8 + it;
    const QSlot<CT> sl = s_q[src];
    CT Gb[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) Gb[e] = s_g[GRAD ? src : 0][e];
    const CornerC<CT> c = slot_corner(sl, a.g, j);
    FT rec[kMom];
    if constexpr (sizeof(FT) == 4) {
      // FP32 records: the next query's record is loaded before this one is used
#pragma unroll
      for (int e = 0; e < kMom; ++e) rec[e] = recB[e];
      if (it < 7) {
        const CornerC<CT> cn = slot_corner(s_q[src + 1], a.g, j);
        load_record<FT>(field, nvox, cn.vox, cn.cell, j, recB);
      }
    } else {
      load_record<FT>(field, nvox, c.vox, c.cell, j, rec);
    }
    CT Gp[21];
    shift21_adj<CT>(Gb, c.dl, Gp);
    CT val, gz[3];
    corner_vjp<CT>(rec, Gp, sl.z, k2, k1, k0, &val, gz);
    CT r[6] = {c.dw[0] * val, c.dw[1] * val, c.dw[2] * val, c.w * gz[0], c.w * gz[1], c.w * gz[2]};
    sum8_arr<6>(r);
#pragma unroll
    for (int e = 0; e < 6; ++e) keep[e] = (j == it) ? r[e] : keep[e];
  }
  if (!valid) return;
  const CT* z = own.z;
  CT gphi[3] = {z[1] * keep[5] - z[2] * keep[4], z[2] * keep[3] - z[0] * keep[5],
                z[0] * keep[4] - z[1] * keep[3]};
  FT* gt_out = reinterpret_cast<FT*>(a.dL_dt);
  FT* gp_out = reinterpret_cast<FT*>(a.dL_dphi);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gt_out[3 * ql + c] = (FT)keep[c];
    gp_out[3 * ql + c] = (FT)gphi[c];
  }
}

// Forward query on FP32 fields with persistent waves.  Each wave takes batches
// of 64 queries in turn, one query per lane, and visits the 8 cell corners in 8
// steps: step k gathers corner k of all 64 queries.  The main records of a step
// are loaded straight into LDS (global_load_lds_dwordx4), 16 lanes per record
// so that each load instruction reads whole records, and each lane then reads
// its own record from LDS; a lane loading its own record instead (64 records
// per instruction) moves fewer bytes per second.  The records of the next step
// are loaded before the current step is contracted, and the first step of the
// wave's next batch (with each lane's 64-B cell side record, read whole into
// registers once per batch) before the current batch's FP64 metric step, so the
// gathers stay in flight throughout; no load is issued where the next wait on
// the step's records would cover it before it is needed.  Each corner term is
// the one query_info_kernel computes; a lane adds its query's 8 terms with a
// chain of FMAs (weight times block, in corner order), where query_info_kernel
// rounds each weighted block and sums them in an 8-lane butterfly, so the two
// agree to FP32 rounding of that sum (bitwise for nearest-voxel queries, which
// take step 0 only).  The gradient on the same fields runs in
// query_grad_pipe_kernel, whose forward part is this one's, so a pose's forward
// values do not depend on which of the two computed them.  The LDS slots and
// records are private to a wave and no workgroup barrier is used: a wave leaves
// as soon as its batches are done.  Voxel indices are 32-bit here (grids of
// 2^32 voxels or more take query_info_kernel).
constexpr int kPipeWaves = kQThreads / 64;
constexpr int kRecF4 = kMain / 4;  // float4 per main record

// The per-query data a lane keeps for its own query (QSlot without d f / d t).
struct PSlot {
  float t[3], z[3], f[3];
  int32_t i0[3];
  int32_t bits;
};

__device__ inline PSlot pslot(const QSlot<float>& q) {
  PSlot p;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    p.t[ax] = q.t[ax]; p.z[ax] = q.z[ax]; p.f[ax] = q.f[ax]; p.i0[ax] = q.i0[ax];
  }
  p.bits = q.bits;
  return p;
}

// Corner data of one query that do not depend on the corner: for each axis the
// lower and upper trilinear weights and shifts, and the voxel-index steps.
struct LaneCell {
  float wlo[3], whi[3], dlo[3], dhi[3];
  uint32_t v0, sx, sy, sz;
};

__device__ inline LaneCell lane_cell(const PSlot& s, const GridDev& g) {
  LaneCell c;
  const double o[3] = {g.ox, g.oy, g.oz};
  const bool nearest = (s.bits & 16) != 0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int step = (s.bits >> ax) & 1;
    c.wlo[ax] = nearest ? 1.0f + s.f[ax] : 1.0f - s.f[ax];
    c.whi[ax] = nearest ? 1.0f + s.f[ax] : s.f[ax];
    c.dlo[ax] = (float)((o[ax] + (double)s.i0[ax] * g.h) - (double)s.t[ax]);
    c.dhi[ax] = (float)((o[ax] + (double)(s.i0[ax] + step) * g.h) - (double)s.t[ax]);
  }
  const uint32_t nx = (uint32_t)g.nx, nxy = (uint32_t)g.nx * (uint32_t)g.ny;
  c.v0 = (uint32_t)s.i0[0] + nx * ((uint32_t)s.i0[1] + (uint32_t)g.ny * (uint32_t)s.i0[2]);
  c.sx = (uint32_t)(s.bits & 1);
  c.sy = ((s.bits >> 1) & 1) ? nx : 0u;
  c.sz = ((s.bits >> 2) & 1) ? nxy : 0u;
  return c;
}

__device__ inline uint32_t lane_vox(const LaneCell& c, int k) {
  return c.v0 + ((k & 1) ? c.sx : 0u) + ((k & 2) ? c.sy : 0u) + ((k & 4) ? c.sz : 0u);
}

typedef const void __attribute__((address_space(1)))* gptr_t;
typedef void __attribute__((address_space(3)))* lptr_t;

// One corner step's gathers into the wave's record buffer `buf` (64 main
// records of 256 B): record r is the voxel `v` of lane r.  Load q (0..15)
// covers records 4q .. 4q+3 with 16 lanes each, so one load instruction reads
// four whole records; lane s of record r reads piece (s - r) & 15, which puts
// piece i of record r in slot (i + r) & 15 of its 256 B, so that the 64 lanes
// reading piece i of their own records fall in different banks.  The voxels
// are exchanged through the buffer itself (its previous records have been
// read) before any load of the step is issued, so that no wait on the step's
// loads is needed before these LDS accesses.
__device__ __forceinline__ void pipe_issue(float4* buf, const float4* field4, uint32_t v, int lane) {
  const int s = lane & 15;
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the step's LDS reads are done
  int* sv = reinterpret_cast<int*>(buf);
  sv[(lane & 3) * 16 + (lane >> 2)] = (int)v;
  wave_sync();
  int vk[16];
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    const int4 x = reinterpret_cast<const int4*>(sv)[(lane >> 4) * 4 + q4];
    vk[4 * q4] = x.x; vk[4 * q4 + 1] = x.y; vk[4 * q4 + 2] = x.z; vk[4 * q4 + 3] = x.w;
  }
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): before the loads overwrite the buffer
  wave_sync();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = 4 * q + (lane >> 4);
    const float4* src = field4 + (size_t)(uint32_t)vk[q] * kRecF4 + ((s - r) & 15);
    __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)&buf[q * 64], 16, 0, 0);
  }
}

// Waits for the step's gathers and reads the lane's own record from `buf`.
__device__ __forceinline__ void pipe_stage(const float4* buf, int lane, float rec[kMom]) {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the step's records are in LDS
  wave_sync();
  const float4* rr = &buf[lane * kRecF4];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float4 x = rr[(i + lane) & 15];
    rec[4 * i] = x.x; rec[4 * i + 1] = x.y; rec[4 * i + 2] = x.z; rec[4 * i + 3] = x.w;
  }
}

// The lane's cell side record (the 2 extra moments of each of the 8 corners),
// read whole into registers once per batch.
__device__ __forceinline__ void load_side16(const float* field, size_t nvox, uint32_t cell,
                                            float side[kSideRec]) {
  const float4* sp = reinterpret_cast<const float4*>(field + nvox * kMain + (size_t)cell * kSideRec);
#pragma unroll
  for (int i = 0; i < kSideRec / 4; ++i) {
    const float4 x = sp[i];
    side[4 * i] = x.x; side[4 * i + 1] = x.y; side[4 * i + 2] = x.z; side[4 * i + 3] = x.w;
  }
}

// Corner k's pair of the side record into rec, then the record rotated by one
// pair (after 8 steps it is back in corner order).
__device__ __forceinline__ void take_side(float rec[kMom], float side[kSideRec]) {
  const float s0 = side[0], s1 = side[1];
  rec[kMain] = s0;
  rec[kMain + 1] = s1;
#pragma unroll
  for (int i = 0; i < kSideRec - 2; ++i) side[i] = side[i + 2];
  side[kSideRec - 2] = s0;
  side[kSideRec - 1] = s1;
}

// Trilinear weight and shift (voxel centre - frame point) of corner k.
__device__ __forceinline__ float corner_of(const LaneCell& lc, int k, float dl[3]) {
  const int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
  dl[0] = bx ? lc.dhi[0] : lc.dlo[0];
  dl[1] = by ? lc.dhi[1] : lc.dlo[1];
  dl[2] = bz ? lc.dhi[2] : lc.dlo[2];
  return (bx ? lc.whi[0] : lc.wlo[0]) * (by ? lc.whi[1] : lc.wlo[1]) * (bz ? lc.whi[2] : lc.wlo[2]);
}

__device__ __forceinline__ void raw_pose7(const QueryArgs& a, int64_t b, int lane, float tr[7]) {
  const float* T = reinterpret_cast<const float*>(a.t);
  const float* Q = reinterpret_cast<const float*>(a.q);
  const int64_t i = min(b * 64 + lane, a.m - 1);
  tr[0] = T[3 * i]; tr[1] = T[3 * i + 1]; tr[2] = T[3 * i + 2];
  tr[3] = Q[4 * i]; tr[4] = Q[4 * i + 1]; tr[5] = Q[4 * i + 2]; tr[6] = Q[4 * i + 3];
}

__device__ __forceinline__ QSlot<float> slot7(const QueryArgs& a, const float tr[7]) {
  double t[3] = {(double)tr[0], (double)tr[1], (double)tr[2]}, z[3];
  quat_axis((double)tr[3], (double)tr[4], (double)tr[5], (double)tr[6], z);
  return make_slot_from<float>(a, t, z);
}

__global__ __launch_bounds__(kQThreads, 2) void query_info_pipe_kernel(QueryArgs a, int64_t nbatch) {
  using FT = float;
  using CT = float;
  __shared__ PSlot s_q[kPipeWaves][64];  // each lane's query of the next batch
  __shared__ float4 s_rec[kPipeWaves][64 * kRecF4];  // a corner step's 64 main records
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t gw = (int64_t)blockIdx.x * kPipeWaves + wv;
  const int64_t nw = (int64_t)gridDim.x * kPipeWaves;
  if (gw >= nbatch) return;  // whole wave
  const FT* field = reinterpret_cast<const FT*>(a.field);
  const float4* field4 = reinterpret_cast<const float4*>(a.field);
  float4* buf = &s_rec[wv][0];
  const size_t nvox = (size_t)a.g.nx * a.g.ny * a.g.nz;
  const CT k2 = (CT)a.vis.k2, k1 = (CT)a.vis.k1, k0 = (CT)a.vis.k0;
  const int nsteps = a.interp == 1 ? 1 : 8;
  float side[kSideRec];
  {
    FT tr[7];
    raw_pose7(a, gw, lane, tr);
    const PSlot sl = pslot(slot7(a, tr));
    s_q[wv][lane] = sl;
    const LaneCell lc = lane_cell(sl, a.g);
    pipe_issue(buf, field4, lc.v0, lane);
    load_side16(field, nvox, lc.v0, side);
  }

  for (int64_t b = gw; b < nbatch; b += nw) {
    // corner steps (gathers + FP32 contraction) at a raised wave priority and
    // the FP64 metric step at the normal one, so that a wave about to issue
    // gathers is not held back behind another wave's long FP64 stretch
    __builtin_amdgcn_s_setprio(1);
    const bool more = b + nw < nbatch;
    FT trn[7];
    const PSlot own = s_q[wv][lane];
    const LaneCell lc = lane_cell(own, a.g);
    const VisW<CT> vw = vis_weights<CT>(own.z, k2, k1, k0);
    CT Z[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) Z[e] = 0;
#pragma unroll 1
    for (int k = 0; k < nsteps; ++k) {
      FT rec[kMom];
      pipe_stage(buf, lane, rec);
      // the next batch's poses (the last batch re-reads its own), requested
      // after the first wait on the step loads so that no wait covers them
      // before the step after
      if (k == 0) raw_pose7(a, more ? b + nw : b, lane, trn);
      take_side(rec, side);
      if (k + 1 < nsteps) pipe_issue(buf, field4, lane_vox(lc, k + 1), lane);
      CT dl[3];
      const CT w = corner_of(lc, k, dl);
      CT Y[21];
      corner_fim<CT>(rec, vw, dl, Y);
#pragma unroll
      for (int e = 0; e < 21; ++e) Z[e] = fmaf(Y[e], w, Z[e]);
    }
    {
      // the side record is read on every path (no merge of loaded registers
      // before the metric step, which would wait for the loads)
      const PSlot nx = pslot(slot7(a, trn));
      const LaneCell nc = lane_cell(nx, a.g);
      if (more) {
        s_q[wv][lane] = nx;
        pipe_issue(buf, field4, nc.v0, lane);
      }
      load_side16(field, nvox, nc.v0, side);
    }

    __builtin_amdgcn_s_setprio(0);
    const int64_t qi = b * 64 + lane;
    const bool valid = qi < a.m;
    double td[3] = {(double)own.t[0], (double)own.t[1], (double)own.t[2]};
    double Zd[21], F[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) Zd[e] = (double)Z[e];
    shift21<double>(Zd, td, F);
#pragma unroll
    for (int e = 0; e < 21; ++e) F[e] *= a.vis.inv_s2;
    uint8_t flag = (own.bits & 8) ? FL_CLAMPED : 0;
    double* row = (valid && a.out) ? a.out + qi * a.ncols : nullptr;
    eval_metrics<false>(F, a.metrics, row, &flag, nullptr, nullptr, a.flags != nullptr);
    if (valid && a.flags) a.flags[qi] = flag;
  }
}

// Forward query and its gradient on FP32 fields with persistent waves, the
// layout of query_info_pipe_kernel: one pose per lane, 8 forward corner steps
// (the same arithmetic and order, so the forward values are bitwise those of
// the forward query), the FP64 metric step with G = ds/dF, then 8 backward
// corner steps that gather the records again (mostly from cache) and add up
// the corner terms of ds/dt (through the trilinear weights) and ds/dz
// (through vr(z)) in the lane.  The gathers of the backward pass's first
// corner are issued before the metric step, those of the next batch's first
// corner before the last backward step.
__global__ __launch_bounds__(kQThreads, 2) void query_grad_pipe_kernel(QueryArgs a, int64_t nbatch) {
  using FT = float;
  using CT = float;
  __shared__ QSlot<CT> s_q[kPipeWaves][64];  // each lane's query of the next batch
  __shared__ float4 s_rec[kPipeWaves][64 * kRecF4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t gw = (int64_t)blockIdx.x * kPipeWaves + wv;
  const int64_t nw = (int64_t)gridDim.x * kPipeWaves;
  if (gw >= nbatch) return;  // whole wave
  const FT* field = reinterpret_cast<const FT*>(a.field);
  const float4* field4 = reinterpret_cast<const float4*>(a.field);
  float4* buf = &s_rec[wv][0];
  const size_t nvox = (size_t)a.g.nx * a.g.ny * a.g.nz;
  const CT k2 = (CT)a.vis.k2, k1 = (CT)a.vis.k1, k0 = (CT)a.vis.k0;
  const int nmet = (int)((a.metrics & 1u) != 0) + (int)((a.metrics & 2u) != 0) +
                   (int)((a.metrics & 4u) != 0);
  FT* gt_out = reinterpret_cast<FT*>(a.dL_dt);
  FT* gp_out = reinterpret_cast<FT*>(a.dL_dphi);
  float side[kSideRec];
  {
    FT tr[7];
    raw_pose7(a, gw, lane, tr);
    const QSlot<CT> sl = slot7(a, tr);
    s_q[wv][lane] = sl;
    const LaneCell lc = lane_cell(pslot(sl), a.g);
    pipe_issue(buf, field4, lc.v0, lane);
    load_side16(field, nvox, lc.v0, side);
  }

  for (int64_t b = gw; b < nbatch; b += nw) {
    __builtin_amdgcn_s_setprio(1);
    const bool more = b + nw < nbatch;
    CT Z[21];
    double td[3];
    int32_t bits;
    {
      const QSlot<CT> own = s_q[wv][lane];
      const LaneCell lc = lane_cell(pslot(own), a.g);
      const VisW<CT> vw = vis_weights<CT>(own.z, k2, k1, k0);
#pragma unroll
      for (int e = 0; e < 21; ++e) Z[e] = 0;
#pragma unroll 1
      for (int k = 0; k < 8; ++k) {
        FT rec[kMom];
        pipe_stage(buf, lane, rec);
        take_side(rec, side);
        // corner k + 1, and after corner 7 the backward pass's corner 0
        pipe_issue(buf, field4, lane_vox(lc, (k + 1) & 7), lane);
        CT dl[3];
        const CT w = corner_of(lc, k, dl);
        CT Y[21];
        corner_fim<CT>(rec, vw, dl, Y);
#pragma unroll
        for (int e = 0; e < 21; ++e) Z[e] = fmaf(Y[e], w, Z[e]);
      }
      td[0] = own.t[0]; td[1] = own.t[1]; td[2] = own.t[2];
      bits = own.bits;
    }

    // ------------------------------------------------ metrics and ds/dF (FP64)
    // (the lane's slot, cell data and side record are read again afterwards,
    // so that they do not occupy registers through the FP64 step)
    __builtin_amdgcn_s_setprio(0);
    const int64_t qi = b * 64 + lane;
    const bool valid = qi < a.m;
    const int64_t ql = valid ? qi : a.m - 1;
    CT Gt[21];
    {
      double Zd[21], F[21], G[21];
#pragma unroll
      for (int e = 0; e < 21; ++e) Zd[e] = (double)Z[e];
      shift21<double>(Zd, td, F);
#pragma unroll
      for (int e = 0; e < 21; ++e) F[e] *= a.vis.inv_s2;
      uint8_t flag = (bits & 8) ? FL_CLAMPED : 0;
      // upstream weights (constant indices: the array stays in registers)
      const double* du = a.dL_dout + ql * nmet;
      const double up[3] = {(valid && nmet > 0) ? du[0] : 0.0, (valid && nmet > 1) ? du[1] : 0.0,
                            (valid && nmet > 2) ? du[2] : 0.0};
      double* row = (valid && a.out) ? a.out + qi * a.ncols : nullptr;
      eval_metrics<true>(F, a.metrics, row, &flag, up, G, a.flags != nullptr);
      if (valid && a.flags) a.flags[qi] = flag;
      double Gw[21];
      shift21_adj<double>(G, td, Gw);
#pragma unroll
      for (int e = 0; e < 21; ++e) Gt[e] = (CT)(valid ? Gw[e] * a.vis.inv_s2 : 0.0);
    }

    // ------------------------------------------------ backward corner steps
    __builtin_amdgcn_s_setprio(1);
    const QSlot<CT> own = s_q[wv][lane];
    const LaneCell lc = lane_cell(pslot(own), a.g);
    load_side16(field, nvox, lc.v0, side);
    FT trn[7];
    CT keep[6] = {0, 0, 0, 0, 0, 0};
    auto bstep = [&](int k) __attribute__((always_inline)) {
      FT rec[kMom];
      pipe_stage(buf, lane, rec);
      // the next batch's poses (the last batch re-reads its own), requested
      // after the first wait on the step loads
      if (k == 0) raw_pose7(a, more ? b + nw : b, lane, trn);
      take_side(rec, side);
      if (k < 7) {
        pipe_issue(buf, field4, lane_vox(lc, k + 1), lane);
      } else {
        // the next batch: its slot, first gathers and side record (the side
        // record read on every path, so no loaded registers are merged)
        const QSlot<CT> nx = slot7(a, trn);
        const LaneCell nc = lane_cell(pslot(nx), a.g);
        if (more) {
          s_q[wv][lane] = nx;
          pipe_issue(buf, field4, nc.v0, lane);
        }
        load_side16(field, nvox, nc.v0, side);
      }
      const int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
      CT dl[3];
      const CT w = corner_of(lc, k, dl);
      const CT wc[3] = {bx ? lc.whi[0] : lc.wlo[0], by ? lc.whi[1] : lc.wlo[1],
                        bz ? lc.whi[2] : lc.wlo[2]};
      const CT dwc[3] = {bx ? own.df[0] : -own.df[0], by ? own.df[1] : -own.df[1],
                         bz ? own.df[2] : -own.df[2]};
      const CT dw[3] = {dwc[0] * wc[1] * wc[2], wc[0] * dwc[1] * wc[2], wc[0] * wc[1] * dwc[2]};
      CT Gp[21];
      shift21_adj<CT>(Gt, dl, Gp);
      CT val, gz[3];
      corner_vjp<CT>(rec, Gp, own.z, k2, k1, k0, &val, gz);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        keep[c] = fmaf(dw[c], val, keep[c]);
        keep[3 + c] = fmaf(w, gz[c], keep[3 + c]);
      }
    };
#pragma unroll 1
    for (int k = 0; k < 7; ++k) bstep(k);
    bstep(7);

    if (valid) {
      const CT* z = own.z;
      const CT gphi[3] = {z[1] * keep[5] - z[2] * keep[4], z[2] * keep[3] - z[0] * keep[5],
                          z[0] * keep[4] - z[1] * keep[3]};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gt_out[3 * qi + c] = keep[c];
        gp_out[3 * qi + c] = gphi[c];
      }
    }
  }
}

// Trace field (eq:general_trace_pif): one lane per query, 8 gathers of 40 B
// (CELLS: one read of the cell's 320-B block, 3 lines of 128 B).  All of a
// query's loads are issued before the first is used; both layouts hold the
// same values and sum the corners in the same order.
template <typename FT>
__device__ inline void load_trace10(const FT* r, FT* dst) {
  if constexpr (sizeof(FT) == 4) {
    const float4 v0 = *reinterpret_cast<const float4*>(r);
    const float4 v1 = *reinterpret_cast<const float4*>(r + 4);
    const float2 v2 = *reinterpret_cast<const float2*>(r + 8);
    dst[0] = v0.x; dst[1] = v0.y; dst[2] = v0.z; dst[3] = v0.w;
    dst[4] = v1.x; dst[5] = v1.y; dst[6] = v1.z; dst[7] = v1.w;
    dst[8] = v2.x; dst[9] = v2.y;
  } else {
#pragma unroll
    for (int k = 0; k < 10; k += 2) {
      const double2 v = *reinterpret_cast<const double2*>(r + k);
      dst[k] = v.x; dst[k + 1] = v.y;
    }
  }
}

template <typename FT, bool CELLS>
__global__ __launch_bounds__(kQThreads) void query_trace_kernel(QueryArgs a) {
  const int64_t qi = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
  if (qi >= a.m) return;
  const FT* field = reinterpret_cast<const FT*>(a.field);
  double t[3], z[3];
  load_pose<FT>(a, qi, t, z);
  const double k2 = a.vis.k2, k1 = a.vis.k1, k0 = a.vis.k0;
  const double vr[10] = {k2 * z[0] * z[0],       k2 * z[1] * z[1],       k2 * z[2] * z[2],
                         2.0 * k2 * z[0] * z[1], 2.0 * k2 * z[0] * z[2], 2.0 * k2 * z[1] * z[2],
                         k1 * z[0],              k1 * z[1],              k1 * z[2],
                         k0};
  double cbar[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) cbar[k] = 0.0;
  bool clamped = false;
  if (a.interp == 1) {
    const Corner c = make_corner(a.g, t, 0, 1);
    clamped = c.clamped;
    FT r[10];
    load_trace10<FT>(field + c.vox * (CELLS ? kTCell : kTRec), r);
#pragma unroll
    for (int k = 0; k < 10; ++k) cbar[k] = fma(c.w, (double)r[k], cbar[k]);
  } else {
    double w[8];
    FT blk[80];
    const FT* base = field;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const Corner c = make_corner(a.g, t, j, 0);
      clamped = clamped || c.clamped;
      w[j] = c.w;
      if (CELLS) {
        if (j == 0) base = field + c.vox * kTCell;
      } else {
        load_trace10<FT>(field + c.vox * kTRec, blk + 10 * j);
      }
    }
    if (CELLS) {
#pragma unroll
      for (int j = 0; j < 8; ++j) load_trace10<FT>(base + 10 * j, blk + 10 * j);
    }
    // keep the compiler from trading loads in flight for registers: every
    // load of the query is issued before the first is used
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int k = 0; k < 10; ++k) cbar[k] = fma(w[j], (double)blk[10 * j + k], cbar[k]);
  }
  double tr = 0.0;
#pragma unroll
  for (int k = 0; k < 10; ++k) tr = fma(vr[k], cbar[k], tr);
  a.out[qi * a.ncols] = tr * a.vis.inv_s2;
  if (a.flags) a.flags[qi] = clamped ? FL_CLAMPED : 0;
}

// ------------------------------------------------------------ export

// Expand a moment group to all degrees: S2 (6), S1 (3), S0 from S4, S3.
template <typename FT>
__device__ inline void expand_group(const FT* S4, const FT* S3, double E4[15], double E3[10],
                                    double E2[6], double E1[3], double* E0) {
#pragma unroll
  for (int i = 0; i < 15; ++i) E4[i] = (double)S4[i];
#pragma unroll
  for (int i = 0; i < 10; ++i) E3[i] = (double)S3[i];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) E2[i2(a, b)] = E4[s4(a, b, 0, 0)] + E4[s4(a, b, 1, 1)] + E4[s4(a, b, 2, 2)];
#pragma unroll
  for (int a = 0; a < 3; ++a) E1[a] = E3[s3(a, 0, 0)] + E3[s3(a, 1, 1)] + E3[s3(a, 2, 2)];
  *E0 = E2[0] + E2[3] + E2[5];
}

// Paper's vp order: u1^2, u2^2, u3^2, u1u2, u1u3, u2u3, u1, u2, u3, 1.
__device__ constexpr int vp_a(int k) {
  return k < 3 ? k : (k == 3 ? 0 : (k == 4 ? 0 : (k == 5 ? 1 : k - 6)));
}
__device__ constexpr int vp_b(int k) { return k < 3 ? k : (k == 3 ? 1 : (k == 4 ? 2 : 2)); }

// Block k of the paper's 10 world-frame blocks (eq:general_info_pif, 21
// entries, scaled by 1/sigma^2 and `w`) of one voxel with centre tv, from its
// 66 moments rec[] (any memory; k may vary across lanes).  Lower-degree moments
// follow from |u| = 1 as sums of higher ones, added in a fixed order.
template <typename FT>
__device__ inline void paper_block(const FT* rec, const double tv[3], double scale, int k,
                                   double* out) {
  // degree-2 moment (a, b) of group G (G0 or G2) from its degree-4 ones
  auto deg2 = [&](int o4, int a2, int b2) __attribute__((always_inline)) {
    return (double)rec[o4 + s4(a2, b2, 0, 0)] + (double)rec[o4 + s4(a2, b2, 1, 1)] +
           (double)rec[o4 + s4(a2, b2, 2, 2)];
  };
  double sv0, sv2, Q0[6], Q2[6], bv[3];
  const int pa = vp_a(k), pb = vp_b(k);
  if (k < 6) {
    sv0 = deg2(O_G0_4, pa, pb);
    sv2 = deg2(O_G2_4, pa, pb);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = c; d < 3; ++d) {
        Q0[i2(c, d)] = (double)rec[O_G0_4 + s4(pa, pb, c, d)];
        Q2[i2(c, d)] = (double)rec[O_G2_4 + s4(pa, pb, c, d)];
      }
#pragma unroll
    for (int c = 0; c < 3; ++c) bv[c] = (double)rec[O_G1_3 + s3(pa, pb, c)];
  } else if (k < 9) {
    sv0 = (double)rec[O_G0_3 + s3(pa, 0, 0)] + (double)rec[O_G0_3 + s3(pa, 1, 1)] +
          (double)rec[O_G0_3 + s3(pa, 2, 2)];
    sv2 = (double)rec[O_G2_3 + s3(pa, 0, 0)] + (double)rec[O_G2_3 + s3(pa, 1, 1)] +
          (double)rec[O_G2_3 + s3(pa, 2, 2)];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = c; d < 3; ++d) {
        Q0[i2(c, d)] = (double)rec[O_G0_3 + s3(pa, c, d)];
        Q2[i2(c, d)] = (double)rec[O_G2_3 + s3(pa, c, d)];
      }
#pragma unroll
    for (int c = 0; c < 3; ++c) bv[c] = (double)rec[O_G1_2 + s2(pa, c)];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = c; d < 3; ++d) {
        Q0[i2(c, d)] = deg2(O_G0_4, c, d);
        Q2[i2(c, d)] = deg2(O_G2_4, c, d);
      }
    sv0 = Q0[0] + Q0[3] + Q0[5];
    sv2 = Q2[0] + Q2[3] + Q2[5];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      bv[c] = (double)rec[O_G1_3 + s3(c, 0, 0)] + (double)rec[O_G1_3 + s3(c, 1, 1)] +
              (double)rec[O_G1_3 + s3(c, 2, 2)];
  }
  double A[6], D[6], B[9];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c; d < 3; ++d) {
      A[i2(c, d)] = (c == d ? sv2 : 0.0) - Q2[i2(c, d)];
      D[i2(c, d)] = (c == d ? sv0 : 0.0) - Q0[i2(c, d)];
    }
  B[0] = 0.0;    B[1] = bv[2];  B[2] = -bv[1];
  B[3] = -bv[2]; B[4] = 0.0;    B[5] = bv[0];
  B[6] = bv[1];  B[7] = -bv[0]; B[8] = 0.0;
  double W[21];
  shift_frame<double>(A, B, D, tv, W);
#pragma unroll
  for (int e = 0; e < 21; ++e) out[e] = W[e] * scale;
}

// All 10 blocks of one voxel: out[k * 21 + e].
template <typename FT>
__device__ inline void paper_blocks(const FT* rec, const double tv[3], double scale, double* out) {
#pragma unroll
  for (int k = 0; k < 10; ++k) paper_block<FT>(rec, tv, scale, k, out + 21 * k);
}

constexpr int kExportThreads = 128;

// (launch bounds: the default cap for 1024-thread blocks, 128 VGPRs, spilled
// the 210 FP64 block entries in flight)
template <typename FT>
__global__ __launch_bounds__(kExportThreads) void export_info_kernel(ExportArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t v = a.ids[i];
  const int64_t nvox = (int64_t)a.g.nx * a.g.ny * a.g.nz;
  if (v < 0 || v >= nvox) {  // ids live on the device: reject out-of-grid ones here
    for (int e = 0; e < 210; ++e) a.out[i * 210 + e] = __builtin_nan("");
    return;
  }
  const int64_t ix = v % a.g.nx, iy = (v / a.g.nx) % a.g.ny, iz = v / ((int64_t)a.g.nx * a.g.ny);
  const double tv[3] = {a.g.ox + (double)ix * a.g.h, a.g.oy + (double)iy * a.g.h,
                        a.g.oz + (double)iz * a.g.h};
  FT rec[kMom];
  load_record<FT>(reinterpret_cast<const FT*>(a.field), (size_t)nvox, (size_t)v, (size_t)v, 0, rec);
  paper_blocks<FT>(rec, tv, a.inv_s2, a.out + i * 210);
}

// ------------------------------------------------------------ view sweep

constexpr int kSweepThreads = 512;

// One workgroup per position.  The corner records are staged in LDS, 80
// threads expand one (corner, block) each into the paper's world-frame blocks,
// the workgroup sums the corners (interpolation done once), then every thread
// contracts the blocks with vr(z) for its axes and evaluates the metric (a
// template argument, so each kernel holds only its own metric's code).
template <typename FT, uint32_t METRIC>
__global__ __launch_bounds__(kSweepThreads) void view_sweep_kernel(SweepArgs a) {
  __shared__ double s_part[8][210];
  __shared__ double s_cbar[210];
  __shared__ FT s_rec[8][kMom];
  __shared__ double s_tv[8][4];
  __shared__ double s_w[8];
  __shared__ double s_bv[kSweepThreads];
  __shared__ int64_t s_bi[kSweepThreads];
  const int tid = threadIdx.x;
  const int64_t p = blockIdx.x;
  const FT* T = reinterpret_cast<const FT*>(a.t);
  const double t[3] = {(double)T[3 * p], (double)T[3 * p + 1], (double)T[3 * p + 2]};
  const size_t nvox = (size_t)a.g.nx * a.g.ny * a.g.nz;
  if (tid < 8) {
    const Corner c = make_corner(a.g, t, tid, a.interp);
    if (c.active) {
      FT rec[kMom];
      const size_t cell = c.vox;  // own values sit in slot 0 of the voxel's own record
      load_record<FT>(reinterpret_cast<const FT*>(a.field), nvox, c.vox, cell, 0, rec);
#pragma unroll
      for (int e = 0; e < kMom; ++e) s_rec[tid][e] = rec[e];
      const int64_t ix = c.vox % a.g.nx, iy = (c.vox / a.g.nx) % a.g.ny,
                    iz = c.vox / ((size_t)a.g.nx * a.g.ny);
      s_tv[tid][0] = a.g.ox + (double)ix * a.g.h;
      s_tv[tid][1] = a.g.oy + (double)iy * a.g.h;
      s_tv[tid][2] = a.g.oz + (double)iz * a.g.h;
    }
    s_w[tid] = c.active ? a.vis.inv_s2 * c.w : 0.0;
  }
  __syncthreads();
  if (tid < 80) {
    const int j = tid / 10, k = tid % 10;
    if (s_w[j] != 0.0 || s_w[j] != s_w[j]) {
      const double tv[3] = {s_tv[j][0], s_tv[j][1], s_tv[j][2]};
      paper_block<FT>(s_rec[j], tv, s_w[j], k, &s_part[j][21 * k]);
    } else {
      for (int e = 0; e < 21; ++e) s_part[j][21 * k + e] = 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < 210; e += kSweepThreads) {
    double sacc = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) sacc += s_part[j][e];
    s_cbar[e] = sacc;
  }
  __syncthreads();
  const double k2 = a.vis.k2, k1 = a.vis.k1, k0 = a.vis.k0;
  double best = -__builtin_inf();
  int64_t bi = -1;
#pragma unroll 1
  for (int64_t d = tid; d < a.n_dir; d += kSweepThreads) {
    // the 210 interpolated block entries stay in LDS: read per axis rather
    // than hoisted into registers (420 VGPRs) by the compiler
    asm volatile("" ::: "memory");
    double z[3] = {a.dirs[3 * d], a.dirs[3 * d + 1], a.dirs[3 * d + 2]};
    const double inv = 1.0 / sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    z[0] *= inv; z[1] *= inv; z[2] *= inv;
    const double vr[10] = {k2 * z[0] * z[0],       k2 * z[1] * z[1],       k2 * z[2] * z[2],
                           2.0 * k2 * z[0] * z[1], 2.0 * k2 * z[0] * z[2], 2.0 * k2 * z[1] * z[2],
                           k1 * z[0],              k1 * z[1],              k1 * z[2],
                           k0};
    // F = sum_k vr_k Cbar_k, one block of 21 at a time (each entry's sum in
    // the order k = 0..9), so that only one block is read into registers
    double F[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) F[e] = 0.0;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
#pragma unroll
      for (int e = 0; e < 21; ++e) F[e] = fma(vr[k], s_cbar[k * 21 + e], F[e]);
      __builtin_amdgcn_sched_barrier(0);
    }
    double val;
    uint8_t flag = 0;
    if constexpr (METRIC == M_LOGDET) {
      // in place: the general LDL^T with its separate factor held the kernel
      // at one wave per SIMD
      val = logdet6_inplace(F);
    } else {
      eval_metrics<false>(F, METRIC, &val, &flag, nullptr, nullptr, false);
    }
    if (a.values) a.values[p * a.n_dir + d] = val;
    if (val > best) {  // NaN never wins; d grows, so the first of equal values stays
      best = val;
      bi = d;
    }
  }
  s_bv[tid] = best;
  s_bi[tid] = bi;
  __syncthreads();
  for (int stride = kSweepThreads / 2; stride > 0; stride >>= 1) {
    if (tid < stride) {
      const double v2 = s_bv[tid + stride];
      const int64_t i2v = s_bi[tid + stride];
      const bool take = (i2v >= 0) && (s_bi[tid] < 0 || v2 > s_bv[tid] ||
                                       (v2 == s_bv[tid] && i2v < s_bi[tid]));
      if (take) {
        s_bv[tid] = v2;
        s_bi[tid] = i2v;
      }
    }
    __syncthreads();
  }
  if (tid == 0 && a.best) a.best[p] = s_bi[0];
}

template <typename FT>
static void launch_sweep_metric(const SweepArgs& p, dim3 grid, dim3 block, hipStream_t stream) {
  if (p.metric == M_TRACE) hipLaunchKernelGGL((view_sweep_kernel<FT, M_TRACE>), grid, block, 0, stream, p);
  else if (p.metric == M_LMIN) hipLaunchKernelGGL((view_sweep_kernel<FT, M_LMIN>), grid, block, 0, stream, p);
  else hipLaunchKernelGGL((view_sweep_kernel<FT, M_LOGDET>), grid, block, 0, stream, p);
}

hipError_t launch_sweep(const SweepArgs& a, int prec, hipStream_t stream) {
  if (a.n_pos <= 0) return hipSuccess;
  const int64_t per = kMaxLaunchItems / kSweepThreads;  // positions per launch
  const size_t sb = prec == 2 ? 8 : 4;
  for (int64_t off = 0; off < a.n_pos; off += per) {
    SweepArgs p = a;
    p.n_pos = std::min(per, a.n_pos - off);
    p.t = static_cast<const char*>(a.t) + (size_t)off * 3 * sb;
    if (a.values) p.values = a.values + (size_t)off * a.n_dir;
    if (a.best) p.best = a.best + off;
    dim3 grid((unsigned)p.n_pos), block(kSweepThreads);
    if (prec == 2) launch_sweep_metric<double>(p, grid, block, stream);
    else launch_sweep_metric<float>(p, grid, block, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename FT, bool CELLS>
__global__ void export_trace_kernel(ExportArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t v = a.ids[i];
  if (v < 0 || v >= (int64_t)a.g.nx * a.g.ny * a.g.nz) {
    for (int k = 0; k < 10; ++k) a.out[i * 10 + k] = __builtin_nan("");
    return;
  }
  const FT* rec = reinterpret_cast<const FT*>(a.field) + (size_t)v * (CELLS ? kTCell : kTRec);
#pragma unroll
  for (int k = 0; k < 10; ++k) a.out[i * 10 + k] = (double)rec[k] * a.inv_s2;
}

// Workgroups of the persistent query: 8 per CU of the current device (two are
// resident per CU at this kernel's register count and 80 KB of LDS; the rest
// even out the tail).
static int64_t pipe_blocks() { return (int64_t)current_device_cus() * 8; }

hipError_t launch_query(const QueryArgs& a, int prec, int kind, bool grad, hipStream_t stream) {
  if (a.m <= 0) return hipSuccess;
  const bool dbl = (prec == 2);
  const uint64_t nvox = (uint64_t)a.g.nx * a.g.ny * a.g.nz;
  if (kind == 0 && !dbl && nvox <= UINT32_MAX) {  // persistent: any m in one launch
    const int64_t nbatch = (a.m + 63) / 64;
    const int64_t want = (nbatch + kPipeWaves - 1) / kPipeWaves;
    const int64_t cap = pipe_blocks();
    dim3 pgrid((unsigned)(want < cap ? want : cap));
    if (grad) hipLaunchKernelGGL(query_grad_pipe_kernel, pgrid, dim3(kQThreads), 0, stream, a, nbatch);
    else hipLaunchKernelGGL(query_info_pipe_kernel, pgrid, dim3(kQThreads), 0, stream, a, nbatch);
    return hipGetLastError();
  }
  for (int64_t off = 0; off < a.m; off += kMaxLaunchItems) {
    const QueryArgs p = query_part(a, off, std::min(kMaxLaunchItems, a.m - off), dbl ? 8 : 4);
    dim3 grid((unsigned)((p.m + kQThreads - 1) / kQThreads));
    if (kind == 0) {
      if (grad) {
        if (dbl) hipLaunchKernelGGL((query_info_kernel<double, true>), grid, dim3(kQThreads), 0, stream, p);
        else hipLaunchKernelGGL((query_info_kernel<float, true>), grid, dim3(kQThreads), 0, stream, p);
      } else {
        hipLaunchKernelGGL((query_info_kernel<double, false>), grid, dim3(kQThreads), 0, stream, p);
      }
    } else if (kind == 1) {
      if (dbl) hipLaunchKernelGGL((query_trace_kernel<double, false>), grid, dim3(kQThreads), 0, stream, p);
      else hipLaunchKernelGGL((query_trace_kernel<float, false>), grid, dim3(kQThreads), 0, stream, p);
    } else {
      if (dbl) hipLaunchKernelGGL((query_trace_kernel<double, true>), grid, dim3(kQThreads), 0, stream, p);
      else hipLaunchKernelGGL((query_trace_kernel<float, true>), grid, dim3(kQThreads), 0, stream, p);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_export(const ExportArgs& a, int prec, int kind, hipStream_t stream) {
  if (a.n <= 0) return hipSuccess;
  const bool dbl = (prec == 2);
  for (int64_t off = 0; off < a.n; off += kMaxLaunchItems) {
    ExportArgs p = a;
    p.n = std::min(kMaxLaunchItems, a.n - off);
    p.ids = a.ids + off;
    p.out = a.out + (size_t)off * (kind == 0 ? 210 : 10);
    dim3 grid((unsigned)((p.n + kExportThreads - 1) / kExportThreads)), block(kExportThreads);
    if (kind == 0) {
      if (dbl) hipLaunchKernelGGL((export_info_kernel<double>), grid, block, 0, stream, p);
      else hipLaunchKernelGGL((export_info_kernel<float>), grid, block, 0, stream, p);
    } else if (kind == 1) {
      if (dbl) hipLaunchKernelGGL((export_trace_kernel<double, false>), grid, block, 0, stream, p);
      else hipLaunchKernelGGL((export_trace_kernel<float, false>), grid, block, 0, stream, p);
    } else {
      if (dbl) hipLaunchKernelGGL((export_trace_kernel<double, true>), grid, block, 0, stream, p);
      else hipLaunchKernelGGL((export_trace_kernel<float, true>), grid, block, 0, stream, p);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fif
