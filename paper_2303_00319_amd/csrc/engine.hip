// Serving engine: continuous batching of image-pair requests of mixed sizes.
//
// Requests queue on the host; the engine admits the head of the queue as soon
// as (a) a stream pair is free and (b) its buffers fit into the caller's HBM
// arena (first-fit over a free list with coalescing).  Queued requests of the
// head's size (and type and keypoint count) are admitted with it, up to
// `batch` requests, as far as streams and memory allow: their filter banks --
// the bulk of the work, and the part that leaves the device half idle at the
// small sizes -- run as one batch of shared launches (rift2_filter_mim_batch),
// then each pair's detection and description run on its own two streams and
// its matching after them, beside the requests admitted later, so their
// kernels overlap on the device.  Completion is found by polling a
// per-request event; the request's memory and streams go back to the pools
// and the queue is pumped again.  Everything is host code over the C ABI
// stages; the engine allocates no device memory.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

#include "rift2.h"
#include "sched.hpp"

namespace rift2 {

// Per-request device layout inside one arena region.
struct ReqLayout {
  struct Img {
    size_t mim, mmax, kpts, nk, desc, inv, dkp, nd, ws_filter, ws_detect, ws_desc;
  } img[2];
  size_t ws_match, total;
  size_t b_filter, b_detect, b_desc, b_match;
  int32_t K, D;
};

inline size_t eng_align(size_t v) { return (v + 255) / 256 * 256; }

inline bool req_layout(int H, int W, int K, const rift2_pc_params* pc, const rift2_detect_params* det_tpl,
                       const rift2_desc_params* dp, const rift2_match_params* mp, ReqLayout* L) {
  if (K <= 0) return false;
  rift2_detect_params det = *det_tpl;
  det.max_keypoints = K;
  L->K = K;
  L->D = dp->grid * dp->grid * dp->n_orient;
  L->b_filter = rift2_filter_workspace_size(H, W, pc);
  L->b_detect = rift2_detect_workspace_size(H, W, &det);
  L->b_desc = rift2_describe_workspace_size(K);
  L->b_match = rift2_match_workspace_size(2 * K, 2 * K, L->D, mp);
  if (!L->b_filter || !L->b_detect || !L->b_desc || !L->b_match) return false;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = eng_align(off + bytes);
    return o;
  };
  const size_t hw = (size_t)H * W;
  for (int i = 0; i < 2; ++i) {
    ReqLayout::Img& m = L->img[i];
    m.mim = take(hw);
    m.mmax = take(hw * sizeof(float));
    m.kpts = take((size_t)K * sizeof(rift2_keypoint));
    m.nk = take(sizeof(int32_t));
    m.desc = take((size_t)2 * K * L->D * sizeof(uint16_t));
    m.inv = take((size_t)2 * K * sizeof(float));
    m.dkp = take((size_t)2 * K * sizeof(int32_t));
    m.nd = take(sizeof(int32_t));
    m.ws_filter = take(L->b_filter);
    m.ws_detect = take(L->b_detect);
    m.ws_desc = take(L->b_desc);
  }
  L->ws_match = take(L->b_match);
  L->total = off;
  return true;
}

struct EngineSlot {
  hipStream_t sa = nullptr, sb = nullptr;
  hipEvent_t b_done = nullptr, admit = nullptr, done = nullptr, filt = nullptr;
};


}  // namespace rift2

struct rift2_engine {
  int device = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  rift2_pc_params pc;
  rift2_detect_params det;
  rift2_desc_params dp;
  rift2_match_params mp;
  rift2::ArenaAlloc alloc;
  std::vector<rift2::EngineSlot> slots;
  std::vector<int> free_slots;
  std::deque<rift2::EngineReq> pending;
  std::deque<rift2::EngineReq> inflight;
  std::deque<rift2_completion> finished;  // failed at admission, reported by the next poll
  hipEvent_t epoch = nullptr;
  int batch = 4;  // requests whose filter banks share launches (1: none)
};

namespace rift2 {

inline int engine_keypoints(const rift2_request& r) {
  if (r.max_keypoints > 0) return r.max_keypoints;
  return (int)std::floor(2e-3 * (double)r.H * (double)r.W);
}

// Enqueues an admitted group of same-shape requests: their filter banks as
// one batch on the first request's stream, then each request's detection,
// description and matching on its own slot's streams.
inline int32_t engine_launch(rift2_engine* e, EngineReq* const* g, int n) {
  const EngineReq& q0 = *g[0];
  ReqLayout L;
  // admission laid the group out already; a failure here would be a bug, reported rather than run
  if (!req_layout(q0.H, q0.W, q0.K, &e->pc, &e->det, &e->dp, &e->mp, &L)) return RIFT2_ERR_UNSUPPORTED;
  rift2_detect_params det = e->det;
  det.max_keypoints = q0.K;
  const EngineSlot& s0 = e->slots[q0.slot];
  rift2_filter_job jobs[RIFT2_MAX_FILTER_BATCH];
  for (int i = 0; i < n; ++i) {
    const EngineReq& q = *g[i];
    // the caller's inputs may still be in flight on its own stream
    if (q.req.ready && hipStreamWaitEvent(s0.sa, (hipEvent_t)q.req.ready, 0) != hipSuccess) return RIFT2_ERR_DEVICE;
    char* base = e->arena + q.off;
    const void* imgs[2] = {q.req.img_a, q.req.img_b};
    for (int k = 0; k < 2; ++k) {
      const ReqLayout::Img& m = L.img[k];
      jobs[2 * i + k] = rift2_filter_job{imgs[k], (uint8_t*)(base + m.mim), (float*)(base + m.mmax), nullptr, nullptr,
                                         base + m.ws_filter, L.b_filter};
    }
  }
  for (int i = 0; i < n; ++i)
    if (hipEventRecord(e->slots[g[i]->slot].admit, s0.sa) != hipSuccess) return RIFT2_ERR_DEVICE;
  rift2_status r = rift2_filter_mim_batch(2 * n, jobs, q0.req.dtype, q0.H, q0.W, q0.W, &e->pc, s0.sa);
  if (r != RIFT2_OK) return r;
  if (hipEventRecord(s0.filt, s0.sa) != hipSuccess) return RIFT2_ERR_DEVICE;
  for (int i = 0; i < n; ++i) {
    const EngineReq& q = *g[i];
    const EngineSlot& s = e->slots[q.slot];
    if ((i > 0 && hipStreamWaitEvent(s.sa, s0.filt, 0) != hipSuccess) ||
        hipStreamWaitEvent(s.sb, s0.filt, 0) != hipSuccess)
      return RIFT2_ERR_DEVICE;
    char* base = e->arena + q.off;
    hipStream_t st[2] = {s.sa, s.sb};
    for (int k = 0; k < 2; ++k) {
      const ReqLayout::Img& m = L.img[k];
      r = rift2_detect((const float*)(base + m.mmax), q.H, q.W, &det, (rift2_keypoint*)(base + m.kpts),
                       (int32_t*)(base + m.nk), base + m.ws_detect, L.b_detect, st[k]);
      if (r == RIFT2_OK)
        r = rift2_describe((const uint8_t*)(base + m.mim), q.H, q.W, (const rift2_keypoint*)(base + m.kpts),
                           (const int32_t*)(base + m.nk), q.K, &e->dp, (uint16_t*)(base + m.desc),
                           (float*)(base + m.inv), (int32_t*)(base + m.dkp), 2 * q.K, (int32_t*)(base + m.nd),
                           base + m.ws_desc, L.b_desc, st[k]);
      if (r != RIFT2_OK) return r;
    }
    if (hipEventRecord(s.b_done, s.sb) != hipSuccess) return RIFT2_ERR_DEVICE;
    if (hipStreamWaitEvent(s.sa, s.b_done, 0) != hipSuccess) return RIFT2_ERR_DEVICE;
    const ReqLayout::Img& a = L.img[0];
    const ReqLayout::Img& b = L.img[1];
    r = rift2_match((const uint16_t*)(base + a.desc), (const float*)(base + a.inv), (const int32_t*)(base + a.dkp),
                    (const int32_t*)(base + a.nd), 2 * q.K, (const uint16_t*)(base + b.desc),
                    (const float*)(base + b.inv), (const int32_t*)(base + b.dkp), (const int32_t*)(base + b.nd),
                    2 * q.K, L.D, &e->mp, q.req.out, q.req.n_out, base + L.ws_match, L.b_match, s.sa);
    if (r != RIFT2_OK) return r;
    if (hipEventRecord(s.done, s.sa) != hipSuccess) return RIFT2_ERR_DEVICE;
  }
  return RIFT2_OK;
}


// Admits queued requests in arrival order while a slot and arena space are
// free; with each admitted request go the queued requests of its shape that
// also fit (admit_group).  A request larger than the whole arena fails at
// once.

inline void engine_pump(rift2_engine* e) {
  while (!e->pending.empty() && !e->free_slots.empty()) {
    EngineReq& q = e->pending.front();
    ReqLayout L;
    const bool laid_out = req_layout(q.H, q.W, q.K, &e->pc, &e->det, &e->dp, &e->mp, &L);
    if (!laid_out || L.total > e->arena_bytes) {
      rift2_completion c{};
      c.id = q.req.id;
      c.status = laid_out ? RIFT2_ERR_WORKSPACE : RIFT2_ERR_UNSUPPORTED;
      e->finished.push_back(c);
      e->pending.pop_front();
      continue;
    }
    const int cap = std::max(1, std::min(e->batch, RIFT2_MAX_FILTER_BATCH / 2));
    const std::vector<size_t> members = admit_group(e->pending, e->free_slots, e->alloc, L.total, cap);
    if (members.empty()) return;  // wait for memory to free up
    EngineReq* group[RIFT2_MAX_FILTER_BATCH];
    for (size_t k = 0; k < members.size(); ++k) group[k] = &e->pending[members[k]];
    const int32_t status = engine_launch(e, group, (int)members.size());
    if (status != RIFT2_OK) {
      // part of the group may be enqueued: let it drain before the memory
      // and the streams are reused, then report the failure
      for (size_t k = 0; k < members.size(); ++k) {
        const EngineSlot& s = e->slots[group[k]->slot];
        (void)hipStreamSynchronize(s.sa);
        (void)hipStreamSynchronize(s.sb);
      }
      for (size_t k = 0; k < members.size(); ++k) {
        e->alloc.release(group[k]->off, group[k]->bytes);
        e->free_slots.push_back(group[k]->slot);
        rift2_completion c{};
        c.id = group[k]->req.id;
        c.status = status;
        c.batch = group[k]->batch;
        e->finished.push_back(c);
      }
    } else {
      for (size_t k = 0; k < members.size(); ++k) e->inflight.push_back(*group[k]);
    }
    // drop the group's entries from the queue (later indices first)
    for (size_t k = members.size(); k-- > 0;) e->pending.erase(e->pending.begin() + (std::ptrdiff_t)members[k]);
  }
}

}  // namespace rift2
