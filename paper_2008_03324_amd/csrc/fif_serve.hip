// Continuous batching over resident fields (fif_serve_run): the host loop
// that admits, packs and launches requests, plus the two kernels that gather
// a batch's poses from its requests and scatter the results back.  The
// queries themselves are fif_query / fif_query_grad on the batch buffers.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <string>
#include <vector>

#include "../../include/fif.h"
#include "fif_kernels.h"

namespace fif {
namespace {

constexpr int kPackThreads = 256;
constexpr int kMaxPack = FIF_SERVE_MAX_PACK;

// One batch's requests: where each one's poses come from and its results go.
struct PackArgs {
  int32_t n;    // requests in the batch
  int32_t sb;   // bytes per pose scalar (4 or 8)
  int32_t opt;  // gradients too
  int64_t m;    // poses in the batch
  int64_t off[kMaxPack + 1];  // prefix offsets of the requests' poses
  const void* t[kMaxPack];
  const void* q[kMaxPack];
  double* out[kMaxPack];
  void* gt[kMaxPack];
  void* gphi[kMaxPack];
  double w[kMaxPack][3];  // the requests' metric weights (dL/dout)
  // batch buffers
  void* bt;
  void* bq;
  double* bup;
  const double* bout;
  const void* bgt;
  const void* bgphi;
};

__device__ inline int find_request(const PackArgs& a, int64_t i) {
  int r = 0;
  while (r + 1 < a.n && a.off[r + 1] <= i) ++r;
  return r;
}

__device__ inline void copy_scalars(void* dst, const void* src, int count, int sb) {
  if (sb == 8) {
    for (int k = 0; k < count; ++k)
      static_cast<double*>(dst)[k] = static_cast<const double*>(src)[k];
  } else {
    for (int k = 0; k < count; ++k)
      static_cast<float*>(dst)[k] = static_cast<const float*>(src)[k];
  }
}

// Pose i of the batch from its request.
__global__ __launch_bounds__(kPackThreads) void pack_kernel(PackArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kPackThreads + threadIdx.x;
  if (i >= a.m) return;
  const int r = find_request(a, i);
  const int64_t j = i - a.off[r];
  const char* t = static_cast<const char*>(a.t[r]) + (size_t)j * 3 * a.sb;
  const char* q = static_cast<const char*>(a.q[r]) + (size_t)j * 4 * a.sb;
  copy_scalars(static_cast<char*>(a.bt) + (size_t)i * 3 * a.sb, t, 3, a.sb);
  copy_scalars(static_cast<char*>(a.bq) + (size_t)i * 4 * a.sb, q, 4, a.sb);
  if (a.opt)
    for (int k = 0; k < 3; ++k) a.bup[(size_t)i * 3 + k] = a.w[r][k];
}

// Results of pose i back to its request.
__global__ __launch_bounds__(kPackThreads) void unpack_kernel(PackArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kPackThreads + threadIdx.x;
  if (i >= a.m) return;
  const int r = find_request(a, i);
  const int64_t j = i - a.off[r];
  double* out = a.out[r] + (size_t)j * 3;
  for (int k = 0; k < 3; ++k) out[k] = a.bout[(size_t)i * 3 + k];
  if (a.opt) {
    copy_scalars(static_cast<char*>(a.gt[r]) + (size_t)j * 3 * a.sb,
                 static_cast<const char*>(a.bgt) + (size_t)i * 3 * a.sb, 3, a.sb);
    copy_scalars(static_cast<char*>(a.gphi[r]) + (size_t)j * 3 * a.sb,
                 static_cast<const char*>(a.bgphi) + (size_t)i * 3 * a.sb, 3, a.sb);
  }
}

// The upstream weights of a batch of one optimizer request (dL/dout of its m
// poses), for the gradient call made on the request's own buffers.
__global__ __launch_bounds__(kPackThreads) void fill_up_kernel(double* up, int64_t m, double w0,
                                                               double w1, double w2) {
  const int64_t i = (int64_t)blockIdx.x * kPackThreads + threadIdx.x;
  if (i >= m) return;
  up[i * 3] = w0;
  up[i * 3 + 1] = w1;
  up[i * 3 + 2] = w2;
}

fif_status serve_fail(fif_status st, const std::string& msg) {
  set_last_error("fif_serve_run: " + msg);
  return st;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Per-stream batch buffers: poses (t, q), outputs, upstream weights,
// gradients, each for max_batch poses at 8 bytes per scalar.
struct LaneLayout {
  size_t t, q, out, up, gt, gphi, bytes;
};

LaneLayout lane_layout(int64_t max_batch) {
  LaneLayout L;
  const size_t n = (size_t)max_batch;
  size_t o = 0;
  L.t = o;    o += align256(n * 3 * 8);
  L.q = o;    o += align256(n * 4 * 8);
  L.out = o;  o += align256(n * 3 * 8);
  L.up = o;   o += align256(n * 3 * 8);
  L.gt = o;   o += align256(n * 3 * 8);
  L.gphi = o; o += align256(n * 3 * 8);
  L.bytes = o;
  return L;
}

bool config_ok(const fif_serve_config* c) {
  return c && c->n_streams >= 1 && c->n_streams <= FIF_SERVE_MAX_STREAMS &&
         c->max_inflight >= 1 && c->hbm_budget >= 1 && c->max_batch >= 1 &&
         c->max_batch <= ((int64_t)1 << 24);
}

int64_t request_bytes(const fif_serve_request& r) {
  return r.m * (r.kind == FIF_SERVE_OPT ? 96 : 24);
}

struct Lane {
  hipStream_t stream = nullptr;
  char* base = nullptr;
};

struct Batch {
  hipEvent_t ev;
  std::vector<int64_t> reqs;
};

}  // namespace
}  // namespace fif

extern "C" {

size_t fif_serve_workspace_bytes(const fif_serve_config* cfg) {
  if (!fif::config_ok(cfg)) return 0;
  return fif::lane_layout(cfg->max_batch).bytes * (size_t)cfg->n_streams;
}

fif_status fif_serve_run(const fif_field* fields, int32_t n_fields, fif_serve_request* reqs,
                         int64_t n_req, const fif_serve_config* cfg, void* workspace,
                         size_t workspace_bytes, double* elapsed) {
  using namespace fif;
  // ---------------------------------------------------------------- checks
  if (!config_ok(cfg)) return serve_fail(FIF_EINVAL, "invalid serving configuration");
  if (n_fields < 1 || !fields) return serve_fail(FIF_EINVAL, "no fields");
  if (n_req < 0 || (n_req > 0 && !reqs)) return serve_fail(FIF_EINVAL, "invalid request list");
  for (int f = 0; f < n_fields; ++f) {
    // the query entry points validate the field without enqueuing anything at m = 0
    if (fif_query(&fields[f], nullptr, nullptr, 0, FIF_TRACE | FIF_LMIN | FIF_LOGDET,
                  FIF_TRILINEAR, nullptr, nullptr, nullptr) != FIF_OK ||
        fif_query_grad(&fields[f], nullptr, nullptr, 0, FIF_TRACE | FIF_LMIN | FIF_LOGDET,
                       nullptr, nullptr, nullptr, nullptr, nullptr) != FIF_OK)
      return serve_fail(FIF_EINVAL, "field " + std::to_string(f) + ": " + fif_last_error());
  }
  for (int64_t i = 0; i < n_req; ++i) {
    const fif_serve_request& r = reqs[i];
    const std::string id = "request " + std::to_string(i) + ": ";
    if (r.field < 0 || r.field >= n_fields) return serve_fail(FIF_EINVAL, id + "field index");
    if (r.kind != FIF_SERVE_PLAN && r.kind != FIF_SERVE_OPT) return serve_fail(FIF_EINVAL, id + "kind");
    if (r.m < 1 || r.m > cfg->max_batch) return serve_fail(FIF_EINVAL, id + "m outside 1 .. max_batch");
    if (!(r.arrival >= 0.0) || !isfinite(r.arrival)) return serve_fail(FIF_EINVAL, id + "arrival");
    const size_t sb = fields[r.field].prec == FIF_FP64 ? 8 : 4;
    if (!r.t || !r.q || !r.out || ((uintptr_t)r.t % sb) || ((uintptr_t)r.q % sb) ||
        ((uintptr_t)r.out % 8))
      return serve_fail(FIF_EINVAL, id + "NULL or misaligned buffer");
    if (r.kind == FIF_SERVE_OPT &&
        (!r.grad_t || !r.grad_phi || ((uintptr_t)r.grad_t % sb) || ((uintptr_t)r.grad_phi % sb)))
      return serve_fail(FIF_EINVAL, id + "NULL or misaligned gradient buffer");
    if (r.kind == FIF_SERVE_OPT &&
        !(isfinite(r.weights[0]) && isfinite(r.weights[1]) && isfinite(r.weights[2])))
      return serve_fail(FIF_EINVAL, id + "weights not finite");
    if (request_bytes(r) > cfg->hbm_budget)
      return serve_fail(FIF_EINVAL, id + "larger than the HBM budget");
  }
  const size_t need = fif_serve_workspace_bytes(cfg);
  if (!workspace || ((uintptr_t)workspace % 256)) return serve_fail(FIF_EINVAL, "workspace NULL or not 256-byte aligned");
  if (workspace_bytes < need) return serve_fail(FIF_ENOMEM, "workspace smaller than fif_serve_workspace_bytes()");
  for (int64_t i = 0; i < n_req; ++i) { reqs[i].admitted = NAN; reqs[i].done = NAN; }
  if (elapsed) *elapsed = 0.0;
  if (n_req == 0) return FIF_OK;

  // ------------------------------------------------------------- resources
  const LaneLayout L = lane_layout(cfg->max_batch);
  std::vector<Lane> lanes(cfg->n_streams);
  std::vector<hipEvent_t> free_events;
  fif_status status = FIF_OK;
  std::string error_text;
  auto device_fail = [&](hipError_t e, const char* where) {
    if (status == FIF_OK) {
      status = FIF_EDEVICE;
      error_text = std::string(where) + ": " + hipGetErrorString(e);
    }
  };
  for (int s = 0; s < cfg->n_streams && status == FIF_OK; ++s) {
    lanes[s].base = static_cast<char*>(workspace) + (size_t)s * L.bytes;
    hipError_t e = hipStreamCreateWithFlags(&lanes[s].stream, hipStreamNonBlocking);
    if (e != hipSuccess) { lanes[s].stream = nullptr; device_fail(e, "hipStreamCreate"); break; }
  }
  for (int k = 0; k < cfg->max_inflight + 1 && status == FIF_OK; ++k) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) { device_fail(e, "hipEventCreate"); break; }
    free_events.push_back(ev);
  }
  for (auto& ln : lanes)
    if (ln.stream && status == FIF_OK) {
      hipError_t e = hipStreamSynchronize(ln.stream);
      if (e != hipSuccess) device_fail(e, "hipStreamSynchronize");
    }

  // --------------------------------------------------------------- the loop
  std::vector<int64_t> order(n_req);
  for (int64_t i = 0; i < n_req; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return reqs[a].arrival < reqs[b].arrival; });
  std::deque<Batch> inflight;
  std::deque<int64_t> waiting;
  int64_t next = 0, in_reqs = 0, reserved = 0, finished = 0;
  int next_lane = 0;
  const auto t0 = std::chrono::steady_clock::now();
  auto now = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };

  auto launch = [&](const std::vector<int64_t>& group) {
    const fif_serve_request& r0 = reqs[group[0]];
    const fif_field& f = fields[r0.field];
    Lane& ln = lanes[next_lane];
    next_lane = (next_lane + 1) % cfg->n_streams;
    const uint32_t metrics = FIF_TRACE | FIF_LMIN | FIF_LOGDET;
    auto record = [&]() {
      Batch b;
      b.ev = free_events.back();
      free_events.pop_back();
      const hipError_t er = hipEventRecord(b.ev, ln.stream);
      if (er != hipSuccess) { free_events.push_back(b.ev); device_fail(er, "hipEventRecord"); return; }
      b.reqs = group;
      inflight.push_back(std::move(b));
    };
    if (group.size() == 1) {
      // a batch of one request runs on the request's own buffers: no gather or
      // scatter launch (fewer host calls per batch; the same per-pose results)
      fif_status st;
      if (r0.kind == FIF_SERVE_OPT) {
        double* up = reinterpret_cast<double*>(ln.base + L.up);
        const dim3 grid((unsigned)((r0.m + kPackThreads - 1) / kPackThreads)), block(kPackThreads);
        hipLaunchKernelGGL(fill_up_kernel, grid, block, 0, ln.stream, up, r0.m, r0.weights[0],
                           r0.weights[1], r0.weights[2]);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) { device_fail(e, "fill"); return; }
        st = fif_query_grad(&f, r0.t, r0.q, r0.m, metrics, up, r0.grad_t, r0.grad_phi, r0.out,
                            ln.stream);
      } else {
        st = fif_query(&f, r0.t, r0.q, r0.m, metrics, FIF_TRILINEAR, r0.out, nullptr, ln.stream);
      }
      if (st != FIF_OK) {
        if (status == FIF_OK) { status = st; error_text = fif_last_error(); }
        return;
      }
      record();
      return;
    }
    PackArgs a;
    memset(&a, 0, sizeof(a));
    a.n = (int32_t)group.size();
    a.sb = f.prec == FIF_FP64 ? 8 : 4;
    a.opt = r0.kind == FIF_SERVE_OPT;
    int64_t m = 0;
    for (size_t k = 0; k < group.size(); ++k) {
      const fif_serve_request& r = reqs[group[k]];
      a.off[k] = m;
      a.t[k] = r.t; a.q[k] = r.q; a.out[k] = r.out; a.gt[k] = r.grad_t; a.gphi[k] = r.grad_phi;
      for (int c = 0; c < 3; ++c) a.w[k][c] = r.weights[c];
      m += r.m;
    }
    a.off[group.size()] = m;
    a.m = m;
    a.bt = ln.base + L.t;
    a.bq = ln.base + L.q;
    a.bup = reinterpret_cast<double*>(ln.base + L.up);
    a.bout = reinterpret_cast<const double*>(ln.base + L.out);
    a.bgt = ln.base + L.gt;
    a.bgphi = ln.base + L.gphi;
    const dim3 grid((unsigned)((m + kPackThreads - 1) / kPackThreads)), block(kPackThreads);
    hipLaunchKernelGGL(pack_kernel, grid, block, 0, ln.stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { device_fail(e, "pack"); return; }
    fif_status st;
    if (a.opt)
      st = fif_query_grad(&f, ln.base + L.t, ln.base + L.q, m, metrics,
                          reinterpret_cast<const double*>(ln.base + L.up), ln.base + L.gt,
                          ln.base + L.gphi, reinterpret_cast<double*>(ln.base + L.out), ln.stream);
    else
      st = fif_query(&f, ln.base + L.t, ln.base + L.q, m, metrics, FIF_TRILINEAR,
                     reinterpret_cast<double*>(ln.base + L.out), nullptr, ln.stream);
    if (st != FIF_OK) {
      if (status == FIF_OK) { status = st; error_text = fif_last_error(); }
      return;
    }
    hipLaunchKernelGGL(unpack_kernel, grid, block, 0, ln.stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) { device_fail(e, "unpack"); return; }
    record();
  };

  while (status == FIF_OK && finished < n_req) {
    const double tn = now();
    while (next < n_req && (!cfg->realtime || reqs[order[next]].arrival <= tn))
      waiting.push_back(order[next++]);
    // retire every completed batch
    for (auto it = inflight.begin(); it != inflight.end();) {
      const hipError_t q = hipEventQuery(it->ev);
      if (q == hipErrorNotReady) { ++it; continue; }
      if (q != hipSuccess) { device_fail(q, "hipEventQuery"); break; }
      const double td = now();
      for (int64_t ri : it->reqs) {
        reqs[ri].done = td;
        reserved -= request_bytes(reqs[ri]);
      }
      in_reqs -= (int64_t)it->reqs.size();
      finished += (int64_t)it->reqs.size();
      free_events.push_back(it->ev);
      it = inflight.erase(it);
    }
    if (status != FIF_OK) break;
    // admit in arrival order
    std::vector<int64_t> admitted;
    while (!waiting.empty()) {
      const fif_serve_request& r = reqs[waiting.front()];
      if (in_reqs + 1 > cfg->max_inflight || reserved + request_bytes(r) > cfg->hbm_budget) break;
      reqs[waiting.front()].admitted = tn;
      reserved += request_bytes(r);
      ++in_reqs;
      admitted.push_back(waiting.front());
      waiting.pop_front();
    }
    // pack per (field, kind), in admission order
    if (!cfg->co_batch) {
      for (int64_t ri : admitted) {
        launch(std::vector<int64_t>{ri});
        if (status != FIF_OK) break;
      }
    } else {
      std::vector<std::vector<int64_t>> groups;
      std::vector<int64_t> gm;
      for (int64_t ri : admitted) {
        const fif_serve_request& r = reqs[ri];
        size_t g = 0;
        for (; g < groups.size(); ++g) {
          const fif_serve_request& h = reqs[groups[g][0]];
          if (h.field == r.field && h.kind == r.kind) break;
        }
        if (g < groups.size() &&
            (gm[g] + r.m > cfg->max_batch || (int)groups[g].size() == kMaxPack)) {
          launch(groups[g]);
          if (status != FIF_OK) break;
          groups[g].clear();
          gm[g] = 0;
        }
        if (g == groups.size()) {
          groups.emplace_back();
          gm.push_back(0);
        }
        groups[g].push_back(ri);
        gm[g] += r.m;
      }
      for (auto& g : groups) {
        if (status != FIF_OK) break;
        if (!g.empty()) launch(g);
      }
    }
  }

  // ------------------------------------------------------------- teardown
  for (auto& ln : lanes)
    if (ln.stream) {
      hipError_t e = hipStreamSynchronize(ln.stream);
      if (e != hipSuccess) device_fail(e, "hipStreamSynchronize");
    }
  if (elapsed) *elapsed = now();
  for (auto& b : inflight) free_events.push_back(b.ev);
  for (hipEvent_t ev : free_events) hipEventDestroy(ev);
  for (auto& ln : lanes)
    if (ln.stream) hipStreamDestroy(ln.stream);
  if (status != FIF_OK) set_last_error("fif_serve_run: " + error_text);
  return status;
}

}  // extern "C"
