// Continuous-batching CG-SENSE engine.
//
// A slot table holds the solves in flight.  Each admitted request is one
// single-slice problem with its own plan (maps, mask, workspace, CG state),
// k-space and output image; admission checks a free slot and a device-memory
// budget.  Running slots are grouped by (ny, maps storage, maps staging); a
// step gives every group one batched launch of the fused iteration
// (previous updates + normal operator), followed by one combine launch when a
// problem of the group splits its coils: block row i of a batched launch runs
// problem i of the group's table with its plan's own coil groups, so a
// problem computes exactly what its own launch would (results are bitwise
// the same alone or in any mix).
//
// Groups advance independently: each group keeps its own lane (stream) and
// its own bound of kAhead enqueued steps, so a group of small slices is not
// held to the pace of a group of large ones.  A step enqueues one iteration
// for every group whose lane has room and returns; when no lane has room it
// first waits for the lane whose oldest step completes first.  Admissions
// (E^H y and the CG start, or a small slice's whole solve) run on the
// engine's own stream, and a lane waits for the latest admission before the
// first step of a newly joined slot.  The host never waits for the device
// except there, in poll's event queries and in sync.
#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <thread>
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
  long admit_no = 0;  // engine admission count at this slot's admission
  hipEvent_t done = nullptr;
};

}  // namespace

struct sense_engine_s {
  int device = -1;
  hipStream_t st = nullptr;  // admissions
  size_t budget = 0;
  size_t used = 0;
  std::vector<Slot> slots;
  long steps = 0;
  // one lane per group key (up to kLanes keys at a time; more keys share
  // lanes round-robin): a stream, a ring of the events of its last kAhead
  // steps, and its own table buffers for groups larger than a
  // kernel-argument table (device copy, two pinned staging buffers used by
  // alternate steps)
  // (measured per lane: 2 and 4 steps ahead give the same latencies within
  // run-to-run noise; without a bound the queue behind a new request grows
  // with the load)
  static constexpr int kAhead = 2;
  static constexpr int kLanes = 4;
  struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t ev[kAhead] = {};
    long steps = 0;       // steps enqueued on this lane
    long admits_seen = 0; // admissions this lane has waited for
    EheParams* d_ehe = nullptr;
    EheParams* h_ehe[kAhead] = {};
  } lane[kLanes];
  std::map<std::tuple<long, int, bool>, int> lane_of;
  int next_lane = 0;
  // recorded on the caller's stream at admission: the engine's stream
  // waits for it, so k-space produced there just before is complete
  hipEvent_t admitted = nullptr;
  // recorded on the engine's stream after every admission; lanes wait for
  // it before a newly joined slot's first step
  hipEvent_t admit_mark = nullptr;
  long admits = 0;
};

static void engine_free(sense_engine e) {
  if (!e) return;
  if (e->st) (void)hipStreamSynchronize(e->st);
  for (auto& ln : e->lane) {
    if (ln.st) (void)hipStreamSynchronize(ln.st);
    for (auto& ev : ln.ev)
      if (ev) (void)hipEventDestroy(ev);
    for (auto& h : ln.h_ehe)
      if (h) (void)hipHostFree(h);
    if (ln.d_ehe) (void)hipFree(ln.d_ehe);
    if (ln.st) (void)hipStreamDestroy(ln.st);
  }
  for (auto& s : e->slots)
    if (s.done) (void)hipEventDestroy(s.done);
  if (e->admitted) (void)hipEventDestroy(e->admitted);
  if (e->admit_mark) (void)hipEventDestroy(e->admit_mark);
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
  for (auto& ln : e->lane) {
    // default priority, like the engine's stream
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking);
    for (auto& ev : ln.ev)
      if (err == hipSuccess) err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err == hipSuccess) err = hipMalloc(reinterpret_cast<void**>(&ln.d_ehe), sizeof(EheParams) * max_slots);
    for (auto& h : ln.h_ehe)
      if (err == hipSuccess)
        err = hipHostMalloc(reinterpret_cast<void**>(&h), sizeof(EheParams) * max_slots, hipHostMallocDefault);
  }
  if (err == hipSuccess) err = hipEventCreateWithFlags(&e->admitted, hipEventDisableTiming);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&e->admit_mark, hipEventDisableTiming);
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
  if (err == hipSuccess) err = hipEventRecord(e->admit_mark, e->st);
  if (err != hipSuccess) return device_fail(err, "sense_engine_admit");
  sl.admit_no = ++e->admits;
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

// Lane of a group key: a lane of its own while fewer than kLanes keys
// have been seen, then shared round-robin.
static int lane_for(sense_engine e, const std::tuple<long, int, bool>& key) {
  auto it = e->lane_of.find(key);
  if (it != e->lane_of.end()) return it->second;
  const int l = e->next_lane;
  e->next_lane = (e->next_lane + 1) % sense_engine_s::kLanes;
  e->lane_of.emplace(key, l);
  return l;
}

sense_status sense_engine_step(sense_engine e, int32_t* n_running) {
  if (!e) return fail(SENSE_ERR_INVALID, "engine is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != e->device)
    return fail(SENSE_ERR_STATE, "current HIP device differs from the engine's device");
  // group the running slots by (ny, maps storage, maps staging): one
  // batched launch each, running the code path each problem's own launch
  // would take
  using Key = std::tuple<long, int, bool>;
  std::map<Key, std::vector<int>> groups;
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

  constexpr int A = sense_engine_s::kAhead;
  // a lane has room when its step kAhead back has completed
  auto has_room = [&](int l) {
    const auto& ln = e->lane[l];
    if (ln.steps < A) return true;
    return hipEventQuery(ln.ev[ln.steps % A]) == hipSuccess;
  };
  // the groups of each lane, in key order
  std::vector<std::vector<const std::pair<const Key, std::vector<int>>*>> by_lane(sense_engine_s::kLanes);
  for (auto& g : groups) by_lane[(size_t)lane_for(e, g.first)].push_back(&g);
  hipError_t err = hipSuccess;
  bool any = false;
  for (int l = 0; l < sense_engine_s::kLanes; ++l)
    if (!by_lane[(size_t)l].empty() && has_room(l)) any = true;
  // every busy lane is kAhead steps ahead: wait until the first of them has
  // room (polling their oldest steps' events; the lanes finish in an order
  // the host cannot know)
  while (!any && err == hipSuccess) {
    for (int l = 0; l < sense_engine_s::kLanes; ++l) {
      if (by_lane[(size_t)l].empty()) continue;
      const hipError_t q = hipEventQuery(e->lane[l].ev[e->lane[l].steps % A]);
      if (q == hipSuccess) any = true;
      else if (q != hipErrorNotReady) err = q;
    }
    if (!any && err == hipSuccess) std::this_thread::yield();
  }
  std::vector<EheParams> he;
  for (int l = 0; l < sense_engine_s::kLanes && err == hipSuccess; ++l) {
    if (by_lane[(size_t)l].empty() || !has_room(l)) continue;
    auto& ln = e->lane[l];
    // newly joined slots: their admission work on the engine's stream first
    long need = 0;
    for (auto* g : by_lane[(size_t)l])
      for (int i : g->second) need = std::max(need, e->slots[(size_t)i].admit_no);
    if (need > ln.admits_seen) {
      err = hipStreamWaitEvent(ln.st, e->admit_mark, 0);
      ln.admits_seen = e->admits;
    }
    int toff = 0;  // this step's rows of the lane's device table
    for (auto* g : by_lane[(size_t)l]) {
      if (err != hipSuccess) break;
      const int cnt = (int)g->second.size();
      he.clear();
      int max_tiles = 0, max_groups = 1, max_ctiles = 0;
      for (int i : g->second) {
        Slot& sl = e->slots[(size_t)i];
        sense_plan p = sl.plan;
        const CgArgs cg = p->cg_args(sl.tol, nullptr, 0);
        he.emplace_back();
        fill_ehe_cg_params(p->g, p->tb, p->maps, p->vectors(sl.x), sl.lambda, sl.k, cg, &he.back());
        const EheParams& P = he.back();
        max_tiles = std::max(max_tiles, P.ntiles);
        max_groups = std::max(max_groups, P.ngroups);
        if (P.ngroups > 1) max_ctiles = std::max(max_ctiles, P.part_tiles);
      }
      // the fused launch also finishes each problem's previous iteration
      const long ny = std::get<0>(g->first);
      const int mst = std::get<1>(g->first);
      const bool staged = std::get<2>(g->first);
      if (cnt <= kInlineProblems) {
        EheInline t{};
        std::copy(he.begin(), he.end(), t.p);
        err = launch_ehe_inline(ny, mst, staged, t, cnt, max_tiles, max_groups, ln.st);
        if (err == hipSuccess && max_groups > 1) err = launch_combine_inline(t, cnt, max_ctiles, max_groups, ln.st);
      } else {
        // larger groups read a device copy of the table; the staging
        // buffer of this lane's step kAhead back was consumed (that step
        // completed)
        EheParams* h = ln.h_ehe[ln.steps % A] + toff;
        EheParams* d = ln.d_ehe + toff;
        std::copy(he.begin(), he.end(), h);
        err = hipMemcpyAsync(d, h, sizeof(EheParams) * he.size(), hipMemcpyHostToDevice, ln.st);
        if (err == hipSuccess) err = launch_ehe_table(ny, mst, staged, d, cnt, max_tiles, max_groups, ln.st);
        if (err == hipSuccess && max_groups > 1) err = launch_combine_table(d, cnt, max_ctiles, max_groups, ln.st);
        toff += cnt;
      }
      for (int i : g->second) {
        Slot& sl = e->slots[(size_t)i];
        if (++sl.k == sl.K && err == hipSuccess) {
          err = enqueue_solve_end(sl.plan, sl.x, sl.K, sl.plan->cg_args(sl.tol, nullptr, 0), nullptr, ln.st);
          if (err == hipSuccess) err = hipEventRecord(sl.done, ln.st);
          sl.finishing = true;
        }
      }
    }
    if (err == hipSuccess) err = hipEventRecord(ln.ev[ln.steps % A], ln.st);
    ++ln.steps;
  }
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
    const hipEvent_t done = sl.done;
    sl = Slot{};
    sl.done = done;
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
  hipError_t err = hipStreamSynchronize(e->st);
  for (auto& ln : e->lane)
    if (err == hipSuccess) err = hipStreamSynchronize(ln.st);
  return err == hipSuccess ? SENSE_OK : device_fail(err, "sense_engine_sync");
}

}  // extern "C"
