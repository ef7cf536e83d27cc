// C-ABI layer of libfif.so: argument validation on the host, then one kernel
// launch per call on the caller's stream.  No device memory is allocated here.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>

#include "../../include/fif.h"
#include "fif_kernels.h"

namespace {

thread_local std::string g_last_error;

fif_status fail(fif_status st, const char* fmt, const char* detail = "") {
  char buf[512];
  snprintf(buf, sizeof(buf), fmt, detail);
  g_last_error = buf;
  return st;
}

fif_status device_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return FIF_OK;
  std::string msg = std::string(where) + ": " + hipGetErrorString(e);
  g_last_error = msg;
  return FIF_EDEVICE;
}

bool grid_ok(const fif_grid* g) {
  if (!g) return false;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->reserved != 0) return false;
  if (!(g->h > 0.0) || !isfinite(g->h)) return false;
  for (int c = 0; c < 3; ++c)
    if (!isfinite(g->origin[c])) return false;
  // record offsets are computed in size_t; keep the voxel count sane
  const double nv = (double)g->nx * g->ny * g->nz;
  return nv <= 4.0e9;
}

bool prec_ok(int32_t p) { return p == FIF_FP32_NAIVE || p == FIF_FP32_COMP || p == FIF_FP64; }
bool kind_ok(int32_t k) {
  return k == FIF_KIND_INFO || k == FIF_KIND_TRACE || k == FIF_KIND_TRACE_CELLS;
}
bool gp_kind_ok(int32_t k) { return k == FIF_KIND_INFO || k == FIF_KIND_TRACE; }

bool vis_ok(const fif_vis* v) {
  if (!v) return false;
  if (!(v->half_fov > 0.0 && v->half_fov < M_PI)) return false;
  if (!isfinite(v->v_alpha)) return false;
  if (!(v->sigma_bearing > 0.0) || !isfinite(v->sigma_bearing)) return false;
  if (!(v->r_min >= 0.0) || !isfinite(v->r_min)) return false;
  if (!(v->r_max >= v->r_min)) return false;  // INFINITY allowed
  return true;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

fif::GridDev grid_dev(const fif_grid* g) {
  fif::GridDev d;
  d.ox = g->origin[0]; d.oy = g->origin[1]; d.oz = g->origin[2];
  d.h = g->h; d.inv_h = 1.0 / g->h;
  d.nx = g->nx; d.ny = g->ny; d.nz = g->nz;
  return d;
}

// Quadratic visibility coefficients from eq:quadratic_conditions:
//   v(0) = 1, v(pi) = 0  ->  k1 = 1/2, k2 + k0 = 1/2;  v(alpha) = v_alpha.
fif::VisDev vis_dev(const fif_vis* v) {
  fif::VisDev d;
  const double c = cos(v->half_fov), s2 = 1.0 - c * c;
  d.k1 = 0.5;
  d.k2 = (0.5 * (1.0 + c) - v->v_alpha) / s2;
  d.k0 = 0.5 - d.k2;
  d.inv_s2 = 1.0 / (v->sigma_bearing * v->sigma_bearing);
  return d;
}

void range_bounds(const fif_vis* v, float* lo2, float* hi2) {
  float lo = (float)(v->r_min * v->r_min);
  *lo2 = lo < 1e-12f ? 1e-12f : lo;
  *hi2 = isinf(v->r_max) ? INFINITY : (float)(v->r_max * v->r_max);
}

size_t record_scalars(int32_t kind) {
  if (kind == FIF_KIND_INFO) return (size_t)(fif::kMain + fif::kSideRec);
  return kind == FIF_KIND_TRACE_CELLS ? (size_t)fif::kTCell : (size_t)fif::kTRec;
}
size_t scalar_bytes(int32_t prec) { return prec == FIF_FP64 ? 8 : 4; }

bool gp_model_ok(const fif_gp* gp, bool need_kinv) {
  if (!gp) return false;
  if (gp->n_s < 1 || gp->n_s > FIF_GP_MAX_NS || gp->reserved != 0) return false;
  if (!(gp->k_s > 0.0) || !isfinite(gp->k_s)) return false;
  if (!(gp->noise >= 0.0) || !isfinite(gp->noise)) return false;
  if (!gp->axes || !aligned(gp->axes, 8)) return false;
  if (need_kinv) {
    if (!(gp->length > 0.0) || !isfinite(gp->length)) return false;
    if (!gp->kinv || !aligned(gp->kinv, 8)) return false;
  }
  return true;
}

// Scalars per voxel of a GP field: 16 per axis (information), or the N_s
// trace factors rounded up to an even count (the query reads them in pairs).
// The rows of x-neighbour voxels, which a trilinear query reads together, are
// then contiguous and share their boundary lines.
int64_t gp_stride(int32_t n_s, int32_t kind, int32_t prec) {
  (void)prec;
  if (kind == FIF_KIND_INFO) return (int64_t)n_s * 16;
  return (int64_t)((n_s + 1) / 2) * 2;
}

fif::GPDev gp_dev(const fif_gp* gp, double half_fov) {
  fif::GPDev d;
  d.ns = gp->n_s;
  d.ks = gp->k_s;
  d.cos_a = cos(half_fov);
  d.inv_2l2 = (gp->length > 0.0) ? 1.0 / (2.0 * gp->length * gp->length) : 0.0;
  d.noise = gp->noise;
  d.axes = gp->axes;
  d.kinv = gp->kinv;
  return d;
}

fif_status check_gp_field(const fif_gp_field* f, bool need_kinv) {
  if (!f) return fail(FIF_EINVAL, "field is NULL%s");
  if (!grid_ok(&f->grid)) return fail(FIF_EINVAL, "invalid grid%s");
  if (!prec_ok(f->prec)) return fail(FIF_EINVAL, "invalid precision%s");
  if (!gp_kind_ok(f->kind)) return fail(FIF_EINVAL, "invalid field kind%s");
  if (!vis_ok(&f->vis)) return fail(FIF_EINVAL, "invalid visibility parameters%s");
  if (!gp_model_ok(&f->gp, need_kinv)) return fail(FIF_EINVAL, "invalid GP model%s");
  if (!f->data) return fail(FIF_EINVAL, "field data is NULL%s");
  if (!aligned(f->data, 16)) return fail(FIF_EINVAL, "field data must be 16-byte aligned%s");
  return FIF_OK;
}

fif_status check_field(const fif_field* f) {
  if (!f) return fail(FIF_EINVAL, "field is NULL%s");
  if (!grid_ok(&f->grid)) return fail(FIF_EINVAL, "invalid grid%s");
  if (!prec_ok(f->prec)) return fail(FIF_EINVAL, "invalid precision%s");
  if (!kind_ok(f->kind)) return fail(FIF_EINVAL, "invalid field kind%s");
  if (!vis_ok(&f->vis)) return fail(FIF_EINVAL, "invalid visibility parameters%s");
  if (!f->data) return fail(FIF_EINVAL, "field data is NULL%s");
  if (!aligned(f->data, 16)) return fail(FIF_EINVAL, "field data must be 16-byte aligned%s");
  return FIF_OK;
}

}  // namespace

extern "C" {

size_t fif_field_bytes(const fif_grid* grid, int32_t prec, int32_t kind) {
  if (!grid_ok(grid) || !prec_ok(prec) || !kind_ok(kind)) return 0;
  return (size_t)grid->nx * grid->ny * grid->nz * record_scalars(kind) * scalar_bytes(prec);
}

size_t fif_workspace_bytes(const fif_grid* grid, int64_t n_landmarks, int32_t prec) {
  if (!grid_ok(grid) || !prec_ok(prec) || n_landmarks <= 0) return 0;
  return fif::sort_workspace_bytes(n_landmarks);
}

static fif_status build_common(const double* landmarks, int64_t n_landmarks, fif_field* field,
                               int accumulate, int sign, void* workspace, size_t ws_bytes,
                               void* stream, const char* where) {
  fif_status st = check_field(field);
  if (st != FIF_OK) return st;
  if (n_landmarks < 0) return fail(FIF_EINVAL, "n_landmarks < 0%s");
  if (n_landmarks > 0 && !landmarks) return fail(FIF_EINVAL, "landmarks is NULL%s");
  if (landmarks && !aligned(landmarks, 8)) return fail(FIF_EINVAL, "landmarks must be 8-byte aligned%s");
  if (n_landmarks > ((int64_t)1 << 40)) return fail(FIF_EINVAL, "too many landmarks%s");
  // one workgroup of 256 lanes per 8x8x4 tile; a dispatch holds fewer than
  // 2^32 work-items along x and 2^16 workgroups along y and z
  if ((int64_t)((field->grid.nx + 7) / 8) * 256 >= ((int64_t)1 << 32) ||
      (field->grid.ny + 7) / 8 > 65535 || (field->grid.nz + 3) / 4 > 65535)
    return fail(FIF_EUNSUPPORTED, "grid too large for one build launch%s");
  fif::BuildArgs a;
  a.lm = landmarks;
  a.L = n_landmarks;
  a.g = grid_dev(&field->grid);
  range_bounds(&field->vis, &a.lo2, &a.hi2);
  a.out = field->data;
  a.accumulate = accumulate;
  a.sign = sign;
  a.trace_cells = field->kind == FIF_KIND_TRACE_CELLS ? 1 : 0;
  a.lm_sorted = nullptr;
  a.batch_box = nullptr;
  a.slice_box = nullptr;
  a.skip2 = INFINITY;
  a.inside_lo2 = INFINITY;  // set by the sort when there is one
  a.inside_hi2 = -INFINITY;
  if (workspace && n_landmarks > 0) {
    if (!aligned(workspace, 256)) return fail(FIF_EINVAL, "workspace must be 256-byte aligned%s");
    if (n_landmarks >= ((int64_t)1 << 32))
      return fail(FIF_EUNSUPPORTED, "the sorted build orders fewer than 2^32 landmarks%s");
    const size_t need = fif::sort_workspace_bytes(n_landmarks);
    if (need == 0) return fail(FIF_EDEVICE, "cannot size the landmark sort%s");
    if (ws_bytes < need) return fail(FIF_ENOMEM, "workspace smaller than fif_workspace_bytes()%s");
    hipError_t e = fif::sort_landmarks(a, workspace, ws_bytes, (hipStream_t)stream);
    if (e != hipSuccess) return device_status(e, where);
  }
  hipError_t e = fif::launch_build(a, field->prec, field->kind, (hipStream_t)stream);
  return device_status(e, where);
}

fif_status fif_build(const double* landmarks, int64_t n_landmarks, fif_field* field,
                     void* workspace, size_t workspace_bytes, void* stream) {
  return build_common(landmarks, n_landmarks, field, 0, 1, workspace, workspace_bytes, stream,
                      "fif_build");
}

}  // extern "C"

namespace {

// Scratch of fif_build_noalloc: the landmark sort's keys and indices, the
// spatially sorted copy, the batch boxes and the radix sort's temporaries,
// held in a static device array instead of a caller's workspace.  Every device
// that runs the library holds its own copy until the process ends.  Host code
// never uses the array's name as an address: it takes the device address from
// hipGetSymbolAddress once per device.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[FIF_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

fif_status scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_status(e, "fif_build_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(FIF_EUNSUPPORTED, "fif_build_noalloc: device index beyond 63%s");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_status(e, "fif_build_noalloc: hipGetSymbolAddress");
    if (!p || !aligned(p, 256))
      return fail(FIF_EDEVICE, "fif_build_noalloc: static scratch not 256-byte aligned%s");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FIF_OK;
}

}  // namespace

extern "C" {

fif_status fif_build_noalloc(const double* landmarks, int64_t n_landmarks, fif_field* field,
                             void* stream) {
  fif_status st = check_field(field);
  if (st != FIF_OK) return st;
  if (n_landmarks <= 0)  // nothing to sort: build_common validates and clears the field
    return build_common(landmarks, n_landmarks, field, 0, 1, nullptr, 0, stream,
                        "fif_build_noalloc");
  if (!landmarks) return fail(FIF_EINVAL, "landmarks is NULL%s");
  if (n_landmarks > ((int64_t)1 << 40)) return fail(FIF_EINVAL, "too many landmarks%s");
  const size_t need = fif::sort_workspace_bytes(n_landmarks);
  if (need == 0) return fail(FIF_EDEVICE, "fif_build_noalloc: cannot size the landmark sort%s");
  if (need > (size_t)FIF_NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    snprintf(msg, sizeof msg, "%lld landmarks need %zu bytes of scratch, more than the %zu of "
             "the static scratch", (long long)n_landmarks, need,
             (size_t)FIF_NOALLOC_SCRATCH_BYTES);
    return fail(FIF_EINVAL, "fif_build_noalloc: %s", msg);
  }
  void* ws = nullptr;
  st = scratch_of_current_device(&ws);
  if (st != FIF_OK) return st;
  return build_common(landmarks, n_landmarks, field, 0, 1, ws, FIF_NOALLOC_SCRATCH_BYTES, stream,
                      "fif_build_noalloc");
}

fif_status fif_update(const double* landmarks, int64_t n_landmarks, int32_t sign,
                      fif_field* field, void* workspace, size_t workspace_bytes, void* stream) {
  if (sign != 1 && sign != -1) return fail(FIF_EINVAL, "sign must be +1 or -1%s");
  if (n_landmarks == 0) {
    fif_status st = check_field(field);
    return st;
  }
  return build_common(landmarks, n_landmarks, field, 1, sign, workspace, workspace_bytes, stream,
                      "fif_update");
}

static int metric_cols(uint32_t metrics) {
  return (int)((metrics & FIF_TRACE) != 0) + (int)((metrics & FIF_LMIN) != 0) +
         (int)((metrics & FIF_LOGDET) != 0) + ((metrics & FIF_FIM21) ? 21 : 0);
}

static fif_status query_common(const fif_field* field, const void* t, const void* q, int64_t m,
                               uint32_t metrics, int32_t interp, double* out, uint8_t* flags,
                               bool grad, const double* dL_dout, void* dL_dt, void* dL_dphi,
                               void* stream, const char* where) {
  fif_status st = check_field(field);
  if (st != FIF_OK) return st;
  if (m < 0) return fail(FIF_EINVAL, "m < 0%s");
  if (m > ((int64_t)1 << 40)) return fail(FIF_EINVAL, "m too large%s");
  if (metrics == 0 || (metrics & ~15u)) return fail(FIF_EINVAL, "invalid metric mask%s");
  if (interp != FIF_TRILINEAR && interp != FIF_NEAREST) return fail(FIF_EINVAL, "invalid interp%s");
  if (field->kind != FIF_KIND_INFO && metrics != FIF_TRACE)
    return fail(FIF_EINVAL, "a trace field only answers FIF_TRACE%s");
  if (grad) {
    if ((metrics & 7u) == 0 || (metrics & FIF_FIM21))
      return fail(FIF_EINVAL, "gradient metrics must be a subset of trace|lmin|logdet%s");
    if (interp != FIF_TRILINEAR) return fail(FIF_EUNSUPPORTED, "gradient needs trilinear interpolation%s");
    if (field->kind != FIF_KIND_INFO) return fail(FIF_EUNSUPPORTED, "gradient needs an information field%s");
  }
  if (m == 0) return FIF_OK;
  const size_t sb = scalar_bytes(field->prec);
  if (!t || !q) return fail(FIF_EINVAL, "t or q is NULL%s");
  if (!aligned(t, sb) || !aligned(q, sb)) return fail(FIF_EINVAL, "t/q misaligned for the field precision%s");
  if (!grad && !out) return fail(FIF_EINVAL, "out is NULL%s");
  if (out && !aligned(out, 8)) return fail(FIF_EINVAL, "out must be 8-byte aligned%s");
  if (grad && (!dL_dout || !dL_dt || !dL_dphi)) return fail(FIF_EINVAL, "gradient buffers are NULL%s");
  fif::QueryArgs a;
  memset(&a, 0, sizeof(a));
  a.field = field->data;
  a.g = grid_dev(&field->grid);
  a.vis = vis_dev(&field->vis);
  a.t = t;
  a.q = q;
  a.m = m;
  a.metrics = metrics;
  a.ncols = grad ? metric_cols(metrics & 7u) : metric_cols(metrics);
  a.interp = interp;
  a.out = out;
  a.flags = flags;
  a.dL_dout = dL_dout;
  a.dL_dt = dL_dt;
  a.dL_dphi = dL_dphi;
  hipError_t e = fif::launch_query(a, field->prec, field->kind, grad, (hipStream_t)stream);
  return device_status(e, where);
}

fif_status fif_query(const fif_field* field, const void* t, const void* q, int64_t m,
                     uint32_t metrics, int32_t interp, double* out, uint8_t* flags,
                     void* stream) {
  return query_common(field, t, q, m, metrics, interp, out, flags, false, nullptr, nullptr,
                      nullptr, stream, "fif_query");
}

fif_status fif_query_grad(const fif_field* field, const void* t, const void* q, int64_t m,
                          uint32_t metrics, const double* dL_dout, void* dL_dt, void* dL_dphi,
                          double* out, void* stream) {
  return query_common(field, t, q, m, metrics, FIF_TRILINEAR, out, nullptr, true, dL_dout,
                      dL_dt, dL_dphi, stream, "fif_query_grad");
}

size_t pc_workspace_bytes(int64_t n_landmarks, int64_t m, int32_t prec) {
  if (!prec_ok(prec) || n_landmarks <= 0 || m <= 0) return 0;
  if (n_landmarks >= ((int64_t)1 << 32)) return 0;
  return fif::pc_sorted_workspace_bytes(n_landmarks, m);
}

fif_status pc_query(const double* landmarks, int64_t n_landmarks, const fif_vis* vis,
                    const fif_pinhole* cam, int32_t prec, const void* t, const void* q,
                    int64_t m, uint32_t metrics, double* out, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if (!vis_ok(vis)) return fail(FIF_EINVAL, "invalid visibility parameters%s");
  if (!prec_ok(prec)) return fail(FIF_EINVAL, "invalid precision%s");
  if (n_landmarks < 0 || m < 0) return fail(FIF_EINVAL, "negative size%s");
  if (n_landmarks > ((int64_t)1 << 40) || m > ((int64_t)1 << 40))
    return fail(FIF_EINVAL, "size too large%s");
  if (metrics == 0 || (metrics & ~15u)) return fail(FIF_EINVAL, "invalid metric mask%s");
  if (n_landmarks > 0 && !landmarks) return fail(FIF_EINVAL, "landmarks is NULL%s");
  if (cam && (!(cam->fx > 0) || !(cam->fy > 0) || cam->width < 1 || cam->height < 1))
    return fail(FIF_EINVAL, "invalid pinhole camera%s");
  if (m == 0) return FIF_OK;
  const size_t sb = scalar_bytes(prec);
  if (!t || !q || !out) return fail(FIF_EINVAL, "t, q or out is NULL%s");
  if (!aligned(t, sb) || !aligned(q, sb) || !aligned(out, 8))
    return fail(FIF_EINVAL, "misaligned pointer%s");
  fif::PcArgs a;
  memset(&a, 0, sizeof(a));
  a.lm = landmarks;
  a.L = n_landmarks;
  range_bounds(vis, &a.lo2, &a.hi2);
  a.vis = vis_dev(vis);
  a.exact = cam ? 1 : 0;
  if (cam) {
    a.fx = cam->fx; a.fy = cam->fy; a.cx = cam->cx; a.cy = cam->cy;
    a.width = cam->width; a.height = cam->height;
  }
  a.t = t;
  a.q = q;
  a.m = m;
  a.metrics = metrics;
  a.ncols = metric_cols(metrics);
  a.out = out;
  // with a workspace and a finite range: the sorted, batch-culled pass (with
  // an unbounded range no batch could be skipped, so the plain pass runs)
  if (workspace && !aligned(workspace, 256))
    return fail(FIF_EINVAL, "workspace must be 256-byte aligned%s");
  if (workspace && n_landmarks > 0 && !isinf(a.hi2)) {
    if (n_landmarks >= ((int64_t)1 << 32))
      return fail(FIF_EUNSUPPORTED, "the sorted pass orders fewer than 2^32 landmarks%s");
    const size_t need = fif::pc_sorted_workspace_bytes(n_landmarks, m);
    if (need == 0) return fail(FIF_EDEVICE, "cannot size the point-cloud sort%s");
    if (workspace_bytes < need)
      return fail(FIF_ENOMEM, "workspace smaller than pc_workspace_bytes()%s");
    a.inv_cell = 32.0 / vis->r_max;
    hipError_t e = fif::launch_pc_sorted(a, prec, workspace, workspace_bytes, (hipStream_t)stream);
    return device_status(e, "pc_query");
  }
  hipError_t e = fif::launch_pc(a, prec, (hipStream_t)stream);
  return device_status(e, "pc_query");
}

fif_status fif_field_export(const fif_field* field, const int64_t* voxel_ids, int64_t n,
                            double* blocks, void* stream) {
  fif_status st = check_field(field);
  if (st != FIF_OK) return st;
  if (n < 0) return fail(FIF_EINVAL, "n < 0%s");
  if (n > ((int64_t)1 << 40)) return fail(FIF_EINVAL, "n too large%s");
  if (n == 0) return FIF_OK;
  if (!voxel_ids || !blocks) return fail(FIF_EINVAL, "voxel_ids or blocks is NULL%s");
  fif::ExportArgs a;
  a.field = field->data;
  a.g = grid_dev(&field->grid);
  a.inv_s2 = 1.0 / (field->vis.sigma_bearing * field->vis.sigma_bearing);
  a.ids = voxel_ids;
  a.n = n;
  a.out = blocks;
  hipError_t e = fif::launch_export(a, field->prec, field->kind, (hipStream_t)stream);
  return device_status(e, "fif_field_export");
}

fif_status fif_view_sweep(const fif_field* field, const void* t, int64_t n_pos,
                          const double* dirs, int64_t n_dir, uint32_t metric, int32_t interp,
                          double* values, int64_t* best, void* stream) {
  fif_status st = check_field(field);
  if (st != FIF_OK) return st;
  if (field->kind != FIF_KIND_INFO) return fail(FIF_EUNSUPPORTED, "sweep needs an information field%s");
  if (metric != FIF_TRACE && metric != FIF_LMIN && metric != FIF_LOGDET)
    return fail(FIF_EINVAL, "sweep metric must be one of trace, lmin, logdet%s");
  if (interp != FIF_TRILINEAR && interp != FIF_NEAREST) return fail(FIF_EINVAL, "invalid interp%s");
  if (n_pos < 0 || n_dir < 0) return fail(FIF_EINVAL, "negative size%s");
  if (n_pos > ((int64_t)1 << 31) - 1) return fail(FIF_EINVAL, "n_pos too large%s");
  if (n_pos == 0) return FIF_OK;
  if (!t || (n_dir > 0 && !dirs)) return fail(FIF_EINVAL, "t or dirs is NULL%s");
  if (!aligned(t, scalar_bytes(field->prec)) || (dirs && !aligned(dirs, 8)))
    return fail(FIF_EINVAL, "misaligned pointer%s");
  fif::SweepArgs a;
  a.field = field->data;
  a.g = grid_dev(&field->grid);
  a.vis = vis_dev(&field->vis);
  a.t = t;
  a.n_pos = n_pos;
  a.dirs = dirs;
  a.n_dir = n_dir;
  a.metric = metric;
  a.interp = interp;
  a.values = values;
  a.best = best;
  hipError_t e = fif::launch_sweep(a, field->prec, (hipStream_t)stream);
  return device_status(e, "fif_view_sweep");
}

size_t fif_gp_field_bytes(const fif_grid* grid, int32_t n_s, int32_t prec, int32_t kind) {
  if (!grid_ok(grid) || !prec_ok(prec) || !gp_kind_ok(kind)) return 0;
  if (n_s < 1 || n_s > FIF_GP_MAX_NS) return 0;
  return (size_t)grid->nx * grid->ny * grid->nz * (size_t)gp_stride(n_s, kind, prec) * scalar_bytes(prec);
}

fif_status fif_gp_setup(const fif_gp* gp, void* stream) {
  if (!gp_model_ok(gp, true)) return fail(FIF_EINVAL, "invalid GP model%s");
  hipError_t e = fif::launch_gp_setup(gp_dev(gp, 0.0), gp->kinv, (hipStream_t)stream);
  return device_status(e, "fif_gp_setup");
}

fif_status fif_gp_evidence(const fif_gp* gp, double half_fov, const double* train_u,
                           int32_t n_train, const double* lengths, int32_t n_len, double* lml,
                           void* stream) {
  if (!gp_model_ok(gp, false)) return fail(FIF_EINVAL, "invalid GP model%s");
  if (!(half_fov > 0.0 && half_fov < M_PI)) return fail(FIF_EINVAL, "invalid half_fov%s");
  if (n_train < 0 || n_len < 0) return fail(FIF_EINVAL, "negative size%s");
  if (n_len == 0) return FIF_OK;
  if ((n_train > 0 && !train_u) || !lengths || !lml) return fail(FIF_EINVAL, "NULL buffer%s");
  if ((train_u && !aligned(train_u, 8)) || !aligned(lengths, 8) || !aligned(lml, 8))
    return fail(FIF_EINVAL, "misaligned buffer%s");
  hipError_t e = fif::launch_gp_evidence(gp_dev(gp, half_fov), train_u, n_train, lengths, n_len,
                                         lml, (hipStream_t)stream);
  return device_status(e, "fif_gp_evidence");
}

fif_status fif_gp_build(const double* landmarks, int64_t n_landmarks, fif_gp_field* field,
                        void* workspace, size_t workspace_bytes, void* stream) {
  fif_status st = check_gp_field(field, false);
  if (st != FIF_OK) return st;
  if (n_landmarks < 0) return fail(FIF_EINVAL, "n_landmarks < 0%s");
  if (n_landmarks > 0 && !landmarks) return fail(FIF_EINVAL, "landmarks is NULL%s");
  if (landmarks && !aligned(landmarks, 8)) return fail(FIF_EINVAL, "landmarks must be 8-byte aligned%s");
  if (n_landmarks > ((int64_t)1 << 40)) return fail(FIF_EINVAL, "too many landmarks%s");
  fif::BuildArgs b;
  memset(&b, 0, sizeof(b));
  b.lm = landmarks;
  b.L = n_landmarks;
  b.g = grid_dev(&field->grid);
  range_bounds(&field->vis, &b.lo2, &b.hi2);
  b.skip2 = INFINITY;
  if (workspace && n_landmarks > 0) {
    if (!aligned(workspace, 256)) return fail(FIF_EINVAL, "workspace must be 256-byte aligned%s");
    if (n_landmarks >= ((int64_t)1 << 32))
      return fail(FIF_EUNSUPPORTED, "the sorted build orders fewer than 2^32 landmarks%s");
    const size_t need = fif::sort_workspace_bytes(n_landmarks);
    if (need == 0) return fail(FIF_EDEVICE, "cannot size the landmark sort%s");
    if (workspace_bytes < need) return fail(FIF_ENOMEM, "workspace smaller than fif_workspace_bytes()%s");
    hipError_t e = fif::sort_landmarks(b, workspace, workspace_bytes, (hipStream_t)stream);
    if (e != hipSuccess) return device_status(e, "fif_gp_build");
  }
  fif::GPBuildArgs a;
  a.lm = landmarks;
  a.L = n_landmarks;
  a.lm_sorted = b.lm_sorted;
  a.batch_box = b.batch_box;
  a.skip2 = b.skip2;
  a.g = b.g;
  a.lo2 = b.lo2;
  a.hi2 = b.hi2;
  a.gp = gp_dev(&field->gp, field->vis.half_fov);
  a.out = field->data;
  a.stride = gp_stride(field->gp.n_s, field->kind, field->prec);
  hipError_t e = fif::launch_gp_build(a, field->prec, field->kind, (hipStream_t)stream);
  return device_status(e, "fif_gp_build");
}

fif_status fif_gp_query(const fif_gp_field* field, const void* t, const void* q, int64_t m,
                        uint32_t metrics, int32_t interp, double* out, uint8_t* flags,
                        void* stream) {
  fif_status st = check_gp_field(field, true);
  if (st != FIF_OK) return st;
  if (m < 0) return fail(FIF_EINVAL, "m < 0%s");
  if (m > ((int64_t)1 << 40)) return fail(FIF_EINVAL, "m too large%s");
  if (metrics == 0 || (metrics & ~15u)) return fail(FIF_EINVAL, "invalid metric mask%s");
  if (interp != FIF_TRILINEAR && interp != FIF_NEAREST) return fail(FIF_EINVAL, "invalid interp%s");
  if (field->kind == FIF_KIND_TRACE && metrics != FIF_TRACE)
    return fail(FIF_EINVAL, "a trace field only answers FIF_TRACE%s");
  if (m == 0) return FIF_OK;
  const size_t sb = scalar_bytes(field->prec);
  if (!t || !q || !out) return fail(FIF_EINVAL, "t, q or out is NULL%s");
  if (!aligned(t, sb) || !aligned(q, sb)) return fail(FIF_EINVAL, "t/q misaligned for the field precision%s");
  if (!aligned(out, 8)) return fail(FIF_EINVAL, "out must be 8-byte aligned%s");
  fif::GPQueryArgs a;
  memset(&a, 0, sizeof(a));
  a.q.field = field->data;
  a.q.g = grid_dev(&field->grid);
  a.q.vis = vis_dev(&field->vis);
  a.q.t = t;
  a.q.q = q;
  a.q.m = m;
  a.q.metrics = metrics;
  a.q.ncols = metric_cols(metrics);
  a.q.interp = interp;
  a.q.out = out;
  a.q.flags = flags;
  if (field->kind == FIF_KIND_TRACE &&
      (uint64_t)field->grid.nx * field->grid.ny * field->grid.nz > UINT32_MAX)
    return fail(FIF_EINVAL, "GP trace fields of more than 2^32 voxels are not supported%s");
  a.gp = gp_dev(&field->gp, field->vis.half_fov);
  a.stride = gp_stride(field->gp.n_s, field->kind, field->prec);
  hipError_t e = fif::launch_gp_query(a, field->prec, field->kind, (hipStream_t)stream);
  return device_status(e, "fif_gp_query");
}

fif_status fif_gp_export(const fif_gp_field* field, const int64_t* voxel_ids, int64_t n,
                         double* blocks, void* stream) {
  fif_status st = check_gp_field(field, true);
  if (st != FIF_OK) return st;
  if (n < 0) return fail(FIF_EINVAL, "n < 0%s");
  if (n == 0) return FIF_OK;
  if (!voxel_ids || !blocks) return fail(FIF_EINVAL, "voxel_ids or blocks is NULL%s");
  if (!aligned(voxel_ids, 8) || !aligned(blocks, 8)) return fail(FIF_EINVAL, "misaligned buffer%s");
  if (n > ((int64_t)1 << 40)) return fail(FIF_EINVAL, "n too large%s");
  fif::GPExportArgs a;
  a.field = field->data;
  a.g = grid_dev(&field->grid);
  a.inv_s2 = 1.0 / (field->vis.sigma_bearing * field->vis.sigma_bearing);
  a.gp = gp_dev(&field->gp, field->vis.half_fov);
  a.stride = gp_stride(field->gp.n_s, field->kind, field->prec);
  a.ids = voxel_ids;
  a.n = n;
  a.out = blocks;
  hipError_t e = fif::launch_gp_export(a, field->prec, field->kind, (hipStream_t)stream);
  return device_status(e, "fif_gp_export");
}

const char* fif_status_string(fif_status s) {
  switch (s) {
    case FIF_OK: return "FIF_OK";
    case FIF_EINVAL: return "FIF_EINVAL: invalid argument";
    case FIF_ENOMEM: return "FIF_ENOMEM: workspace too small";
    case FIF_EDEVICE: return "FIF_EDEVICE: HIP runtime error";
    case FIF_EUNSUPPORTED: return "FIF_EUNSUPPORTED: unsupported combination";
    default: return "unknown fif_status";
  }
}

const char* fif_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace fif {
// The thread's fif_last_error() text, set by parts of the library outside
// this file (the serving loop).
void set_last_error(const std::string& msg) { g_last_error = msg; }

// Compute units of the calling thread's current device, cached per device
// (the persistent kernels size their grids by it on every launch).
int current_device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
  if (dev < 64) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
    v = 256;
  if (dev < 64) cache[dev].store(v, std::memory_order_relaxed);
  return v;
}
}  // namespace fif

extern "C" {

}  // extern "C"
