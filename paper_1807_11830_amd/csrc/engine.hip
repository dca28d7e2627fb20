// Continuous-batching CG-SENSE engine.
//
// A slot table holds the solves in flight.  Each admitted request is one
// single-slice problem with its own plan (maps, mask, workspace, CG state),
// k-space and output image; admission checks a free slot and a device-memory
// budget.  A step advances every running slot by one CG iteration with one
// batched launch of the fused iteration (previous updates + normal operator)
// per distinct (ny, maps storage) group, followed by one combine launch
// when a problem of the group splits its coils: block row i of a batched
// launch runs problem i of the group's device table with its plan's own
// coil groups, so a problem computes exactly what its own launch would
// (results are bitwise the same alone or in any mix).  Requests admitted between steps start on the next step; finished
// slots are reported by poll and freed.  Everything is enqueued on the
// engine's stream, except that the groups of one step after the first run
// on up to kLanes side streams forked from and joined back into it (the
// groups touch disjoint problems); the host never waits for the device
// except in poll's event queries and the reuse of a table staging buffer.
#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "plan_internal.hpp"

using namespace sense;

namespace {

struct Slot {
  bool used = false;
  bool finishing = false;
  sense_plan plan = nullptr;
  const void* y = nullptr;
  c32* x = nullptr;
  int K = 0;
  int k = 0;
  double tol = 0.0;
  float lambda = 0.f;
  size_t footprint = 0;
  hipEvent_t done = nullptr;
};

}  // namespace

struct sense_engine_s {
  int device = -1;
  hipStream_t st = nullptr;
  size_t budget = 0;
  size_t used = 0;
  std::vector<Slot> slots;
  // batched-launch table: device copy and two pinned staging buffers
  EheParams* d_ehe = nullptr;
  EheParams* h_ehe[2] = {nullptr, nullptr};
  hipEvent_t staged[2] = {nullptr, nullptr};
  int buf = 0;
  long steps = 0;
  // the host runs at most kAhead steps ahead of the device, so a request
  // admitted now starts behind at most kAhead queued steps
  // (measured: 2 and 4 give the same latencies; without a bound the queue
  // behind a new request grows with the load)
  static constexpr int kAhead = 2;
  hipEvent_t stepped[kAhead] = {};
  // side streams for the second and later groups of a step (default
  // priority, like the engine's stream)
  static constexpr int kLanes = 3;
  hipStream_t lane[kLanes] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t joined[kLanes] = {};
  // recorded on the caller's stream at admission: the engine's stream
  // waits for it, so k-space produced there just before is complete
  hipEvent_t admitted = nullptr;
};

static void engine_free(sense_engine e) {
  if (!e) return;
  if (e->st) (void)hipStreamSynchronize(e->st);
  for (auto& s : e->slots)
    if (s.done) (void)hipEventDestroy(s.done);
  for (int i = 0; i < 2; ++i) {
    if (e->h_ehe[i]) (void)hipHostFree(e->h_ehe[i]);
    if (e->staged[i]) (void)hipEventDestroy(e->staged[i]);
  }
  for (auto& ev : e->stepped)
    if (ev) (void)hipEventDestroy(ev);
  for (int i = 0; i < sense_engine_s::kLanes; ++i) {
    if (e->lane[i]) {
      (void)hipStreamSynchronize(e->lane[i]);
      (void)hipStreamDestroy(e->lane[i]);
    }
    if (e->joined[i]) (void)hipEventDestroy(e->joined[i]);
  }
  if (e->fork) (void)hipEventDestroy(e->fork);
  if (e->admitted) (void)hipEventDestroy(e->admitted);
  if (e->d_ehe) (void)hipFree(e->d_ehe);
  if (e->st) (void)hipStreamDestroy(e->st);
  delete e;
}

extern "C" {

sense_status sense_engine_create(size_t budget_bytes, int32_t max_slots, sense_engine* out) {
  if (!out) return fail(SENSE_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 65535) return fail(SENSE_ERR_INVALID, "max_slots must be in [1, 65535]");
  auto* e = new (std::nothrow) sense_engine_s();
  if (!e) return fail(SENSE_ERR_NOMEM, "host allocation failed");
  e->budget = budget_bytes;
  e->slots.resize((size_t)max_slots);
  hipError_t err = hipGetDevice(&e->device);
  if (err == hipSuccess) err = hipStreamCreateWithFlags(&e->st, hipStreamNonBlocking);
  if (err == hipSuccess) err = hipMalloc(reinterpret_cast<void**>(&e->d_ehe), sizeof(EheParams) * max_slots);
  for (int i = 0; i < 2 && err == hipSuccess; ++i) {
    err = hipHostMalloc(reinterpret_cast<void**>(&e->h_ehe[i]), sizeof(EheParams) * max_slots, hipHostMallocDefault);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&e->staged[i], hipEventDisableTiming);
  }
  for (auto& ev : e->stepped)
    if (err == hipSuccess) err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  for (int i = 0; i < sense_engine_s::kLanes && err == hipSuccess; ++i) {
    err = hipStreamCreateWithFlags(&e->lane[i], hipStreamNonBlocking);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&e->joined[i], hipEventDisableTiming);
  }
  if (err == hipSuccess) err = hipEventCreateWithFlags(&e->fork, hipEventDisableTiming);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&e->admitted, hipEventDisableTiming);
  for (auto& s : e->slots)
    if (err == hipSuccess) err = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
  if (err != hipSuccess) {
    engine_free(e);
    return device_fail(err, "sense_engine_create");
  }
  *out = e;
  return SENSE_OK;
}

sense_status sense_engine_destroy(sense_engine e) {
  if (!e) return fail(SENSE_ERR_INVALID, "engine is NULL");
  for (auto& s : e->slots)
    if (s.used && s.plan) s.plan->busy = false;
  engine_free(e);
  return SENSE_OK;
}

sense_status sense_engine_admit(sense_engine e, sense_plan plan, const void* d_y, void* d_x, int32_t max_iter,
                                double rel_tol, double lambda, size_t footprint_bytes, void* stream,
                                int32_t* slot) {
  if (!e) return fail(SENSE_ERR_INVALID, "engine is NULL");
  if (!slot) return fail(SENSE_ERR_INVALID, "slot is NULL");
  *slot = -1;
  sense_status s = check_plan(plan);
  if (s != SENSE_OK) return s;
  if (plan->device != e->device) return fail(SENSE_ERR_STATE, "plan and engine are on different devices");
  if (plan->d.ndim != 2 || plan->d.batch != 1)
    return fail(SENSE_ERR_UNSUPPORTED, "the engine serves single 2D slices (ndim 2, batch 1)");
  if (plan->busy) return fail(SENSE_ERR_STATE, "plan is already in a slot");
  s = check_solve_args(plan, d_y, d_x, max_iter, rel_tol, lambda);
  if (s != SENSE_OK) return s;
  int free_slot = -1;
  for (size_t i = 0; i < e->slots.size(); ++i)
    if (!e->slots[i].used) {
      free_slot = (int)i;
      break;
    }
  if (free_slot < 0) return fail(SENSE_ERR_STATE, "no free slot");
  if (footprint_bytes > e->budget || e->used > e->budget - footprint_bytes)
    return fail(SENSE_ERR_STATE, "device-memory budget exceeded");

  Slot& sl = e->slots[(size_t)free_slot];
  const CgArgs cg = plan->cg_args(rel_tol, nullptr, 0);
  // order the admission's work after everything the caller has enqueued
  // on its stream so far (the producer of d_y, earlier users of d_x)
  hipError_t err = hipEventRecord(e->admitted, static_cast<hipStream_t>(stream));
  if (err == hipSuccess) err = hipStreamWaitEvent(e->st, e->admitted, 0);
  // a small slice runs its whole solve at admission (one launch after
  // E^H y); the others join the batched steps
  const bool whole = small_solve(plan);
  if (whole) {
    if (err == hipSuccess)
      err = enqueue_small_solve(plan, d_y, static_cast<c32*>(d_x), max_iter, (float)lambda, cg, nullptr, e->st);
    if (err == hipSuccess) err = hipEventRecord(sl.done, e->st);
  } else {
    if (err == hipSuccess) err = enqueue_solve_begin(plan, d_y, static_cast<c32*>(d_x), cg, e->st);
    if (err == hipSuccess && max_iter == 0) {
      err = enqueue_solve_end(plan, static_cast<c32*>(d_x), 0, cg, nullptr, e->st);
      if (err == hipSuccess) err = hipEventRecord(sl.done, e->st);
    }
  }
  if (err != hipSuccess) return device_fail(err, "sense_engine_admit");
  sl.used = true;
  sl.finishing = whole || max_iter == 0;
  sl.plan = plan;
  sl.y = d_y;
  sl.x = static_cast<c32*>(d_x);
  sl.K = max_iter;
  sl.k = 0;
  sl.tol = rel_tol;
  sl.lambda = (float)lambda;
  sl.footprint = footprint_bytes;
  plan->busy = true;
  e->used += footprint_bytes;
  *slot = free_slot;
  return SENSE_OK;
}

sense_status sense_engine_step(sense_engine e, int32_t* n_running) {
  if (!e) return fail(SENSE_ERR_INVALID, "engine is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != e->device)
    return fail(SENSE_ERR_STATE, "current HIP device differs from the engine's device");
  // group the running slots by (ny, maps storage, maps staging): one
  // batched launch each, running the code path each problem's own launch
  // would take
  std::map<std::tuple<long, int, bool>, std::vector<int>> groups;
  for (size_t i = 0; i < e->slots.size(); ++i) {
    const Slot& sl = e->slots[i];
    if (sl.used && !sl.finishing) {
      const sense_desc& d = sl.plan->d;
      groups[{d.ny, d.maps_storage, ehe_staged(d.ny, d.maps_storage, d.nx, sl.plan->maps)}].push_back((int)i);
    }
  }
  int running = 0;
  for (auto& g : groups) running += (int)g.second.size();
  if (n_running) *n_running = running;
  if (running == 0) return SENSE_OK;

  hipError_t err = hipEventSynchronize(e->stepped[e->steps % sense_engine_s::kAhead]);
  std::vector<EheParams> he;
  he.reserve((size_t)running);
  bool need_table = false;
  for (auto& g : groups) {
    need_table = need_table || g.second.size() > (size_t)kInlineProblems;
    for (int i : g.second) {
      Slot& sl = e->slots[(size_t)i];
      sense_plan p = sl.plan;
      const CgArgs cg = p->cg_args(sl.tol, nullptr, 0);
      he.emplace_back();
      fill_ehe_cg_params(p->g, p->tb, p->maps, p->vectors(sl.x), sl.lambda, sl.k, cg, &he.back());
    }
  }
  if (need_table && err == hipSuccess) {
    // groups larger than a kernel-argument table read a device copy; the
    // staging buffer used two steps ago must have been consumed
    const int b = e->buf;
    err = hipEventSynchronize(e->staged[b]);
    if (err == hipSuccess) {
      std::copy(he.begin(), he.end(), e->h_ehe[b]);
      err = hipMemcpyAsync(e->d_ehe, e->h_ehe[b], sizeof(EheParams) * he.size(), hipMemcpyHostToDevice, e->st);
    }
    if (err == hipSuccess) err = hipEventRecord(e->staged[b], e->st);
    e->buf ^= 1;
  }

  // group 0 runs on the engine's stream, group i > 0 on side stream
  // (i - 1) mod kLanes, forked after the table copy and joined before the
  // step's event
  constexpr int L = sense_engine_s::kLanes;
  const int nlanes = std::min((int)groups.size() - 1, L);
  if (nlanes > 0 && err == hipSuccess) {
    err = hipEventRecord(e->fork, e->st);
    for (int i = 0; i < nlanes && err == hipSuccess; ++i) err = hipStreamWaitEvent(e->lane[i], e->fork, 0);
  }
  int off = 0, gi = 0;
  for (auto& g : groups) {
    hipStream_t gs = gi == 0 ? e->st : e->lane[(gi - 1) % L];
    ++gi;
    const int cnt = (int)g.second.size();
    int max_tiles = 0, max_groups = 1, max_ctiles = 0;
    for (int j = 0; j < cnt; ++j) {
      const EheParams& P = he[(size_t)(off + j)];
      max_tiles = std::max(max_tiles, P.ntiles);
      max_groups = std::max(max_groups, P.ngroups);
      if (P.ngroups > 1) max_ctiles = std::max(max_ctiles, P.part_tiles);
    }
    // the fused launch also finishes each problem's previous iteration
    if (cnt <= kInlineProblems) {
      EheInline t{};
      std::copy(he.begin() + off, he.begin() + off + cnt, t.p);
      if (err == hipSuccess)
        err = launch_ehe_inline(std::get<0>(g.first), std::get<1>(g.first), std::get<2>(g.first), t, cnt,
                                max_tiles, max_groups, gs);
      if (err == hipSuccess && max_groups > 1) err = launch_combine_inline(t, cnt, max_ctiles, max_groups, gs);
    } else {
      if (err == hipSuccess)
        err = launch_ehe_table(std::get<0>(g.first), std::get<1>(g.first), std::get<2>(g.first), e->d_ehe + off,
                               cnt, max_tiles, max_groups, gs);
      if (err == hipSuccess && max_groups > 1) err = launch_combine_table(e->d_ehe + off, cnt, max_ctiles, max_groups, gs);
    }
    off += cnt;
    for (int i : g.second) {
      Slot& sl = e->slots[(size_t)i];
      if (++sl.k == sl.K && err == hipSuccess) {
        err = enqueue_solve_end(sl.plan, sl.x, sl.K, sl.plan->cg_args(sl.tol, nullptr, 0), nullptr, gs);
        if (err == hipSuccess) err = hipEventRecord(sl.done, gs);
        sl.finishing = true;
      }
    }
  }
  for (int i = 0; i < nlanes && err == hipSuccess; ++i) {
    err = hipEventRecord(e->joined[i], e->lane[i]);
    if (err == hipSuccess) err = hipStreamWaitEvent(e->st, e->joined[i], 0);
  }
  if (err == hipSuccess) err = hipEventRecord(e->stepped[e->steps % sense_engine_s::kAhead], e->st);
  ++e->steps;
  return err == hipSuccess ? SENSE_OK : device_fail(err, "sense_engine_step");
}

sense_status sense_engine_poll(sense_engine e, int32_t* done_slots, int32_t max_done, int32_t* n_done) {
  if (!e) return fail(SENSE_ERR_INVALID, "engine is NULL");
  if (!n_done || (max_done > 0 && !done_slots)) return fail(SENSE_ERR_INVALID, "outputs must be non-NULL");
  int32_t n = 0;
  for (size_t i = 0; i < e->slots.size() && n < max_done; ++i) {
    Slot& sl = e->slots[i];
    if (!sl.used || !sl.finishing) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return device_fail(q, "sense_engine_poll");
    sl.plan->busy = false;
    e->used -= sl.footprint;
    sl = Slot{false, false, nullptr, nullptr, nullptr, 0, 0, 0.0, 0.f, 0, sl.done};
    done_slots[n++] = (int32_t)i;
  }
  *n_done = n;
  return SENSE_OK;
}

sense_status sense_engine_stats(sense_engine e, size_t* used_bytes, size_t* budget_bytes, int32_t* active,
                                int64_t* steps) {
  if (!e) return fail(SENSE_ERR_INVALID, "engine is NULL");
  int32_t a = 0;
  for (auto& s : e->slots) a += s.used ? 1 : 0;
  if (used_bytes) *used_bytes = e->used;
  if (budget_bytes) *budget_bytes = e->budget;
  if (active) *active = a;
  if (steps) *steps = e->steps;
  return SENSE_OK;
}

sense_status sense_engine_sync(sense_engine e) {
  if (!e) return fail(SENSE_ERR_INVALID, "engine is NULL");
  const hipError_t err = hipStreamSynchronize(e->st);
  return err == hipSuccess ? SENSE_OK : device_fail(err, "sense_engine_sync");
}

}  // extern "C"
