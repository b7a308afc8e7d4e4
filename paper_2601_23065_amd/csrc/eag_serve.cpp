// Render server with continuous batching over a resident scene.
//
// The scene (geometry, BVH, attribute versions) lives in a caller-provided
// arena. A scheduler thread owns the device work:
//   * an ordered inbox of submits and edits: a submit captures the scene
//     version current at that point; an edit makes a new attribute version
//     (copy of the current one + the edit, copy-on-write) and waits while no
//     version slot is free, which keeps later submits behind it;
//   * admission: pending requests enter, in arrival order, while a slot is
//     free and their fixed-point accumulator fits the arena's request pool
//     (first fit);
//   * each iteration launches the multi-request path-tracing kernel over a
//     budget of paths taken by the live requests with the least work left
//     first, so that short requests do not queue behind long ones, and the
//     rest of the budget goes to the others (requests whose ray-segment
//     parameters differ from the first one's wait for a launch of their own);
//   * a request whose work is complete is resolved into its output image and
//     retired; latency = completion - submit.
// Results do not depend on batching: each path's random numbers come from
// its own (pixel, sample, depth, camera id) counter and accumulators are
// fixed point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "eag_internal.h"
#include "eag_render.h"

namespace eag {
namespace {

constexpr int MAX_VERSIONS = 3;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Version {
  float* albedo = nullptr;
  float* radiance = nullptr;
  float* emissive = nullptr;
  Attr* attrs = nullptr;
  uint32_t id = 0;
  int refs = 0;
  bool used = false;
};

struct Req {
  uint64_t ticket = 0;
  eag_request r{};
  int version = 0;
  uint32_t version_id = 0;
  int64_t tiles_x = 0, tile_pixels = 0, total = 0, done = 0;
  int64_t* accum = nullptr;
  size_t pool_off = 0, pool_bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = EAG_NOT_READY;
  bool cancel = false;
};

struct Op {
  bool is_edit = false;
  uint64_t ticket = 0;
  std::shared_ptr<Req> req;
  eag_edit edit{};          // idx: the caller's device array, read when the edit is applied
  double t_submit = 0;
};

struct EditResult {
  int status = EAG_NOT_READY;
  uint32_t version = 0;
  double t_submit = 0, t_done = 0;
};

// First-fit allocator over a byte range of the arena.
struct Pool {
  std::map<size_t, size_t> free_;   // offset -> size
  void init(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  bool alloc(size_t bytes, size_t& off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace
}  // namespace eag

using namespace eag;

struct eag_server {
  eag_server_config cfg{};
  hipStream_t st = nullptr;
  int device = 0;
  int64_t n = 0;
  // resident scene
  float *pos = nullptr, *rot = nullptr, *scale = nullptr, *opacity = nullptr;
  Version ver[MAX_VERSIONS];
  int current = 0;
  uint32_t next_version_id = 1;
  eag_bvh* bvh = nullptr;
  unsigned long long* work = nullptr;
  uint64_t* hitlist = nullptr;
  char* pool_base = nullptr;
  size_t pool_bytes = 0;
  Pool pool;
  // scheduling
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Op> inbox;
  std::deque<std::shared_ptr<Req>> pending;
  std::vector<std::shared_ptr<Req>> live;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> reqs;
  std::unordered_map<uint64_t, EditResult> edits;
  uint64_t next_ticket = 1;
  bool stop = false;
  int device_error = 0;
  std::string device_msg;
  std::thread worker;

  eag_surfels surfels(int v) const {
    eag_surfels s;
    s.n = n;
    s.pos = pos;
    s.rot = rot;
    s.scale = scale;
    s.opacity = opacity;
    s.albedo = ver[v].albedo;
    s.radiance = ver[v].radiance;
    s.emissive = ver[v].emissive;
    return s;
  }

  // The order key must represent every distance a request's segments can
  // reach in the current scene box: the box's diagonal, and from the camera
  // its farthest corner (called with the lock held: a motion edit changes
  // the box; the server keeps the handle's box current after every build
  // and refit).
  void check_range(const eag_request& r) const {
    const TraceSetup ts = trace_setup(bvh, &r.params);
    if (!(ts.inv_dq > 0.0)) return;
    double diag2 = 0.0, far2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double lo = bvh->lo[a], hi = bvh->hi[a], e = r.cam.eye[a];
      diag2 += (hi - lo) * (hi - lo);
      const double f = std::fmax(std::fabs(e - lo), std::fabs(e - hi));
      far2 += f * f;
    }
    if (std::sqrt(std::fmax(diag2, far2)) >= (double)ts.max_bucket / ts.inv_dq)
      fail(EAG_ERR_INVALID_ARGUMENT, "scene too deep for the order key at this depth_quantum and surfel count "
                                     "(raise depth_quantum)");
  }

  void run();
  void apply_edit(Op& op, int slot);
  bool admit_one(std::shared_ptr<Req>& r);
  void retire(const std::shared_ptr<Req>& r, int status);
};

namespace {

__global__ void k_zero_i64(int64_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

void eag_server::apply_edit(Op& op, int slot) {
  Version& src = ver[current];
  Version& dst = ver[slot];
  check_hip(hipMemcpyAsync(dst.albedo, src.albedo, 3 * n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
  check_hip(hipMemcpyAsync(dst.radiance, src.radiance, 3 * n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
  check_hip(hipMemcpyAsync(dst.emissive, src.emissive, n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
  const eag_edit& e = op.edit;
  const eag_surfels s = surfels(slot);
  if (e.kind == EAG_EDIT_TRANSFORM) {
    // every request that could see the old geometry has completed (the
    // scheduler drains before a transform), so the pool is free for the
    // refit's workspace
    if (e.count > 0) {
      launch_move(pos, rot, n, e.idx, e.count, e.value, e.value + 4, e.value + 7, st);
      refit_bvh(&s, bvh, pool_base, pool_bytes, st);
      bvh_sync_host(bvh);   // the new box, for check_range
    }
  } else if (e.count > 0) {
    eag_surfel_attrs a{n, dst.albedo, dst.radiance, dst.emissive};
    launch_apply_edit(e, a, st);
  }
  pack_attrs(&s, bvh, dst.attrs, st);
  check_hip(hipStreamSynchronize(st), "edit sync");
  dst.used = true;
  dst.refs = 0;
  dst.id = next_version_id++;
  current = slot;
}

bool eag_server::admit_one(std::shared_ptr<Req>& r) {
  const int64_t npix = (int64_t)r->r.cam.width * r->r.cam.height;
  r->pool_bytes = (size_t)npix * 3 * sizeof(int64_t);
  if (!pool.alloc(r->pool_bytes, r->pool_off)) return false;
  r->accum = reinterpret_cast<int64_t*>(pool_base + r->pool_off);
  const int64_t m = npix * 3;
  hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, r->accum, m);
  r->t_admit = now_s();
  return true;
}

void eag_server::retire(const std::shared_ptr<Req>& r, int status) {
  if (r->accum) {
    pool.release(r->pool_off, r->pool_bytes);
    r->accum = nullptr;
  }
  ver[r->version].refs--;
  r->status = status;
  r->t_done = now_s();
}

void eag_server::run() {
  std::unique_lock<std::mutex> lk(mu);
  bool on_device = false;
  while (true) {
    try {
      // (inside the try, so that a failure reaches every request below)
      if (!on_device) {
        check_hip(hipSetDevice(device), "hipSetDevice");
        on_device = true;
      }
      // ---- ordered inbox: submits capture the current version, edits make one
      while (!inbox.empty()) {
        Op& op = inbox.front();
        if (!op.is_edit) {
          try {
            check_range(op.req->r);   // again: a motion edit may have grown the box since the submit
          } catch (const Error& e) {
            op.req->status = e.status;
            op.req->t_done = now_s();
            inbox.pop_front();
            continue;
          }
          op.req->version = current;
          op.req->version_id = ver[current].id;
          ver[current].refs++;
          pending.push_back(op.req);
          inbox.pop_front();
          continue;
        }
        // a motion changes the geometry every version shares: earlier
        // requests finish first
        if (op.edit.kind == EAG_EDIT_TRANSFORM && (!live.empty() || !pending.empty())) break;
        int slot = -1;
        for (int v = 0; v < MAX_VERSIONS; ++v)
          if (v != current && (!ver[v].used || ver[v].refs == 0)) { slot = v; break; }
        if (slot < 0) break;   // wait for live requests to release a version
        apply_edit(op, slot);
        EditResult& er = edits[op.ticket];
        er.status = EAG_OK;
        er.version = ver[current].id;
        er.t_done = now_s();
        inbox.pop_front();
      }
      // ---- cancellations
      for (auto it = pending.begin(); it != pending.end();) {
        if ((*it)->cancel) {
          (*it)->accum = nullptr;
          retire(*it, EAG_ERR_CANCELLED);
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      for (auto it = live.begin(); it != live.end();) {
        if ((*it)->cancel) {
          retire(*it, EAG_ERR_CANCELLED);
          it = live.erase(it);
        } else {
          ++it;
        }
      }
      // ---- admission in arrival order
      while (!pending.empty() && (int)live.size() < cfg.max_live_requests) {
        if (!admit_one(pending.front())) break;
        live.push_back(pending.front());
        pending.pop_front();
      }
      if (live.empty()) {
        if (stop && inbox.empty() && pending.empty()) break;
        cv.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
      // ---- one launch: live requests take work until the launch's path
      // budget is spent, the one with the least work left first (arrival
      // order among equals), so that a short request that arrives while a
      // long one runs finishes in the next launches instead of queueing
      // behind it, and the rest of the budget goes to the others. One launch
      // traces with one set of ray-segment parameters, so it takes only
      // requests whose T_min, t_min, k_sigma and depth_quantum equal those
      // of the first request in that order.
      std::vector<Req*> order;
      for (auto& r : live) order.push_back(r.get());
      std::stable_sort(order.begin(), order.end(),
                       [](const Req* a, const Req* b) { return a->total - a->done < b->total - b->done; });
      PtLaunch L;
      std::memset(&L, 0, sizeof(L));
      const eag_trace_params& p0 = order[0]->r.params;
      int64_t budget = std::max<int64_t>(cfg.paths_per_launch, 1);
      int64_t total = 0;
      std::vector<std::pair<Req*, int64_t>> take;
      for (size_t i = 0; i < order.size() && budget > 0; ++i) {
        Req& r = *order[i];
        const eag_trace_params& q = r.r.params;
        if (q.T_min != p0.T_min || q.t_min != p0.t_min || q.k_sigma != p0.k_sigma ||
            q.depth_quantum != p0.depth_quantum)
          continue;
        const int64_t t = std::min(budget, r.total - r.done);
        if (t <= 0) continue;
        budget -= t;
        PtSlot& S = L.s[take.size()];
        take.emplace_back(&r, t);
        S.cam = make_cam(r.r.cam, r.r.params.camera_id);
        S.accum = r.accum;
        S.attrs = ver[r.version].attrs;
        S.work_begin = r.done;
        S.tile_pixels = r.tile_pixels;
        S.tiles_x = (int32_t)r.tiles_x;
        S.sample_begin = 0;
        S.max_depth = q.max_depth;
        S.rr_start = q.rr_start;
        S.flags = q.flags;
        S.k0 = (uint32_t)(q.seed & 0xffffffffu);
        S.k1 = (uint32_t)(q.seed >> 32);
        S.tau_E = q.tau_E;
        total += t;
        S.global_end = total;
      }
      L.n_slots = (int32_t)take.size();
      L.n_work = total;
      TraceSetup ts;
      ts.idx_bits = bvh->idx_bits;
      const int bucket_bits = 64 - 2 * ts.idx_bits;
      ts.max_bucket = bucket_bits >= 32 ? 0xffffffffu : ((1u << bucket_bits) - 1u);
      ts.inv_dq = 1.0 / (double)p0.depth_quantum;
      const TraceCtx tc = make_ctx(bvh, nullptr, &p0, ts);
      lk.unlock();
      if (total > 0) {
        launch_path_trace(tc, L, work, nullptr, hitlist, st);
        check_hip(hipStreamSynchronize(st), "serve launch");
      }
      lk.lock();
      for (auto& [r, t] : take) r->done += t;
      // ---- retire finished requests
      for (auto it = live.begin(); it != live.end();) {
        Req& r = **it;
        if (r.done >= r.total) {
          const int64_t npix = (int64_t)r.r.cam.width * r.r.cam.height;
          launch_accum_resolve(r.accum, npix * 3, 1.0 / (EAG_ACCUM_SCALE * (double)r.r.params.spp), r.r.out_rgb, st);
          check_hip(hipStreamSynchronize(st), "resolve");
          retire(*it, EAG_OK);
          it = live.erase(it);
        } else {
          ++it;
        }
      }
    } catch (const Error& e) {
      device_error = e.status;
      device_msg = e.msg;
      for (auto& r : live) retire(r, e.status);
      live.clear();
      for (auto& r : pending) {
        r->accum = nullptr;
        retire(r, e.status);
      }
      pending.clear();
      while (!inbox.empty()) {
        Op& op = inbox.front();
        if (op.is_edit) edits[op.ticket].status = e.status;
        else op.req->status = e.status;
        inbox.pop_front();
      }
      if (stop) break;
      if (!on_device) cv.wait_for(lk, std::chrono::milliseconds(10));   // retried for the next requests
    }
  }
}

namespace {
eag_status serve_fail(eag_status s, const std::string& m) {
  set_last_error(m);
  return s;
}
}  // namespace

extern "C" {

size_t eag_serve_arena_bytes(int64_t n, int32_t versions, size_t request_bytes) {
  if (n < 1 || versions < 1) return 0;
  size_t b = 0;
  b += align_up(10 * n * sizeof(float));                                     // pos, rot, scale, opacity
  b += (size_t)MAX_VERSIONS * (align_up(7 * n * sizeof(float)) + align_up(n * sizeof(Attr)));
  b += align_up(eag_bvh_bytes(n));
  b += align_up(64);
  try {
    b += align_up((size_t)runner_lanes() * HL_CAP * sizeof(uint64_t));
  } catch (const Error& e) {
    set_last_error(e.msg);
    return 0;
  }
  b += std::max(align_up(build_ws_bytes(n)), align_up(request_bytes));
  return b + 4096;
}

eag_status eag_serve_create(const eag_surfels* s, const eag_server_config* cfg, eag_server** out) {
  eag_server* srv = nullptr;
  try {
    validate_surfels(s);
    if (!cfg || !out || !cfg->arena) fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
    if (cfg->max_live_requests < 1 || cfg->max_live_requests > PT_MAX_SLOTS)
      fail(EAG_ERR_INVALID_ARGUMENT, "max_live_requests must be in [1, 8]");
    if (cfg->paths_per_launch < 4096) fail(EAG_ERR_INVALID_ARGUMENT, "paths_per_launch must be >= 4096");
    srv = new eag_server();
    srv->cfg = *cfg;
    srv->st = static_cast<hipStream_t>(cfg->stream);
    check_hip(hipGetDevice(&srv->device), "hipGetDevice");
    const int64_t n = s->n;
    srv->n = n;
    Carver c(cfg->arena, cfg->arena_bytes);
    srv->pos = c.take<float>(3 * n);
    srv->rot = c.take<float>(4 * n);
    srv->scale = c.take<float>(2 * n);
    srv->opacity = c.take<float>(n);
    for (int v = 0; v < MAX_VERSIONS; ++v) {
      srv->ver[v].albedo = c.take<float>(3 * n);
      srv->ver[v].radiance = c.take<float>(3 * n);
      srv->ver[v].emissive = c.take<float>(n);
      srv->ver[v].attrs = c.take<Attr>(n);
    }
    const size_t bvh_bytes = eag_bvh_bytes(n);
    void* bvh_mem = c.take<char>(bvh_bytes);
    srv->work = c.take<unsigned long long>(8);
    srv->hitlist = c.take<uint64_t>((size_t)runner_lanes() * HL_CAP);
    c.used = align_up(c.used);
    if (c.used >= cfg->arena_bytes) fail(EAG_ERR_OUT_OF_BUDGET, "arena too small for the scene");
    srv->pool_base = static_cast<char*>(cfg->arena) + c.used;
    srv->pool_bytes = cfg->arena_bytes - c.used;
    const size_t ws_bytes = build_ws_bytes(n);
    if (srv->pool_bytes < ws_bytes) fail(EAG_ERR_OUT_OF_BUDGET, "arena too small for the BVH build");
    hipStream_t st = srv->st;
    check_hip(hipMemcpyAsync(srv->pos, s->pos, 3 * n * 4, hipMemcpyDeviceToDevice, st), "copy");
    check_hip(hipMemcpyAsync(srv->rot, s->rot, 4 * n * 4, hipMemcpyDeviceToDevice, st), "copy");
    check_hip(hipMemcpyAsync(srv->scale, s->scale, 2 * n * 4, hipMemcpyDeviceToDevice, st), "copy");
    check_hip(hipMemcpyAsync(srv->opacity, s->opacity, n * 4, hipMemcpyDeviceToDevice, st), "copy");
    Version& v0 = srv->ver[0];
    check_hip(hipMemcpyAsync(v0.albedo, s->albedo, 3 * n * 4, hipMemcpyDeviceToDevice, st), "copy");
    check_hip(hipMemcpyAsync(v0.radiance, s->radiance, 3 * n * 4, hipMemcpyDeviceToDevice, st), "copy");
    check_hip(hipMemcpyAsync(v0.emissive, s->emissive, n * 4, hipMemcpyDeviceToDevice, st), "copy");
    const eag_surfels rs = srv->surfels(0);
    eag_status bs = eag_build_bvh(&rs, bvh_mem, bvh_bytes, srv->pool_base, srv->pool_bytes, st, &srv->bvh);
    if (bs != EAG_OK) fail(bs, eag_last_error());
    pack_attrs(&rs, srv->bvh, v0.attrs, st);
    check_hip(hipStreamSynchronize(st), "create sync");
    bvh_sync_host(srv->bvh);
    v0.used = true;
    v0.id = 0;
    srv->current = 0;
    srv->pool.init(srv->pool_bytes);
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return EAG_OK;
  } catch (const Error& e) {
    if (srv) {
      eag_bvh_destroy(srv->bvh);
      delete srv;
    }
    return serve_fail(e.status, e.msg);
  } catch (...) {
    delete srv;
    return serve_fail(EAG_ERR_INTERNAL, "unexpected exception");
  }
}

eag_status eag_serve_submit(eag_server* srv, const eag_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket) return serve_fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
  try {
    validate_params(&req->params);
    make_cam(req->cam, req->params.camera_id);
    if (!req->out_rgb) fail(EAG_ERR_INVALID_ARGUMENT, "out_rgb is null");
    if (req->params.depth_quantum == 0.0f) fail(EAG_ERR_INVALID_ARGUMENT, "serving needs depth_quantum > 0");
    const int64_t npix = (int64_t)req->cam.width * req->cam.height;
    if ((size_t)npix * 24 > srv->pool_bytes) fail(EAG_ERR_OUT_OF_BUDGET, "request does not fit the arena");
  } catch (const Error& e) {
    return serve_fail(e.status, e.msg);
  }
  auto r = std::make_shared<Req>();
  r->r = *req;
  r->tiles_x = (req->cam.width + 7) / 8;
  r->tile_pixels = r->tiles_x * ((req->cam.height + 7) / 8) * 64;
  r->total = (int64_t)req->params.spp * r->tile_pixels;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->device_error) return serve_fail(EAG_ERR_DEVICE, srv->device_msg);
    try {
      srv->check_range(*req);
    } catch (const Error& e) {
      return serve_fail(e.status, e.msg);
    }
    r->ticket = srv->next_ticket++;
    srv->reqs[r->ticket] = r;
    Op op;
    op.is_edit = false;
    op.ticket = r->ticket;
    op.req = r;
    op.t_submit = r->t_submit;
    srv->inbox.push_back(std::move(op));
    *ticket = r->ticket;
  }
  srv->cv.notify_all();
  return EAG_OK;
}

eag_status eag_serve_edit(eag_server* srv, const eag_edit* e, uint64_t* ticket) {
  if (!srv || !e || !ticket) return serve_fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
  if (e->kind < EAG_EDIT_SET_RADIANCE || e->kind > EAG_EDIT_TRANSFORM)
    return serve_fail(EAG_ERR_INVALID_ARGUMENT, "bad edit kind");
  if (e->count < 0 || (e->count > 0 && !e->idx)) return serve_fail(EAG_ERR_INVALID_ARGUMENT, "bad index list");
  if (e->kind == EAG_EDIT_TRANSFORM) {
    const float* v = e->value;
    const double l = (double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2] + (double)v[3] * v[3];
    if (!(l > 1e-20) || !std::isfinite(l)) return serve_fail(EAG_ERR_INVALID_ARGUMENT, "rotation must be non-zero");
    for (int k = 4; k < 10; ++k)
      if (!std::isfinite(v[k])) return serve_fail(EAG_ERR_INVALID_ARGUMENT, "non-finite motion");
  }
  Op op;
  op.is_edit = true;
  op.edit = *e;
  op.t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->device_error) return serve_fail(EAG_ERR_DEVICE, srv->device_msg);
    op.ticket = srv->next_ticket++;
    EditResult& er = srv->edits[op.ticket];
    er.t_submit = op.t_submit;
    *ticket = op.ticket;
    srv->inbox.push_back(std::move(op));
  }
  srv->cv.notify_all();
  return EAG_OK;
}

eag_status eag_serve_poll(eag_server* srv, uint64_t ticket, eag_result* out) {
  if (!srv || !out) return serve_fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
  std::lock_guard<std::mutex> g(srv->mu);
  std::memset(out, 0, sizeof(*out));
  auto it = srv->reqs.find(ticket);
  if (it != srv->reqs.end()) {
    const Req& r = *it->second;
    out->status = r.status;
    out->scene_version = r.version_id;
    out->t_submit = r.t_submit;
    out->t_admit = r.t_admit;
    out->t_done = r.t_done;
    out->paths = (uint64_t)std::min(r.done, r.total);
    if (r.status == EAG_NOT_READY) return EAG_NOT_READY;
    return r.status == EAG_OK ? EAG_OK : serve_fail((eag_status)r.status, "request failed or was cancelled");
  }
  auto et = srv->edits.find(ticket);
  if (et != srv->edits.end()) {
    out->status = et->second.status;
    out->scene_version = et->second.version;
    out->t_submit = et->second.t_submit;
    out->t_done = et->second.t_done;
    if (et->second.status == EAG_NOT_READY) return EAG_NOT_READY;
    return et->second.status == EAG_OK ? EAG_OK : serve_fail((eag_status)et->second.status, "edit failed");
  }
  return serve_fail(EAG_ERR_UNKNOWN_TICKET, "unknown ticket");
}

eag_status eag_serve_cancel(eag_server* srv, uint64_t ticket) {
  if (!srv) return serve_fail(EAG_ERR_INVALID_ARGUMENT, "null argument");
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return serve_fail(EAG_ERR_UNKNOWN_TICKET, "unknown ticket");
  if (it->second->status == EAG_NOT_READY) it->second->cancel = true;
  srv->cv.notify_all();
  return EAG_OK;
}

eag_status eag_serve_destroy(eag_server* srv) {
  if (!srv) return EAG_OK;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  const int err = srv->device_error;
  const std::string msg = srv->device_msg;
  eag_bvh_destroy(srv->bvh);
  delete srv;
  if (err) return serve_fail((eag_status)err, msg);
  return EAG_OK;
}

}  // extern "C"
