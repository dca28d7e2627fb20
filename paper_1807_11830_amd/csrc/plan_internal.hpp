// Plan internals shared by the C ABI implementation (plan.hip) and the
// serving engine (engine.hip).  Not part of the public interface.
#pragma once

#include <initializer_list>

#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "sense.h"

namespace sense {

struct Layout {
  size_t tw_x, tw_y, tw_z, mu_y, mask_c, rows_s, rows_u;
  size_t work, r, p, q, r2, p2, qpart;
  size_t state, eta_part, zeta_part, rr_part, rr_par, cgpart, info;
  size_t total;
  int eta_tiles, rr_tiles;
  int ngroups;   // coil groups the workspace holds (the fill split)
  int dgroups;   // default of the normal operator and CG
  int agroups;   // default of the E^H column pass and RSS
};

sense_status fail(sense_status s, const std::string& msg);
// Size and format checks of a descriptor; workspace layout of a plan for it.
sense_status validate_desc(const sense_desc* d);
Layout make_layout(const sense_desc& d);
// Host tables: twiddles exp(-2 pi i e / n) (fp64, rounded once to fp32);
// the 0/1 centred mask [nz][ny], the uncentred mask / ny of the 2D normal
// operator, and the sampled / unsampled row ids (z * ny + y, increasing).
void host_twiddles(long n, c32* out);
void host_mask_tables(const uint8_t* h_mask, long ny, long nz, uint8_t* mask, float* mu, int32_t* rows_s,
                      int32_t* rows_u, int* n_s, int* n_u);
sense_status device_fail(hipError_t e, const char* what);
bool overlap(const void* a, size_t na, const void* b, size_t nb);
// Whether p is a multiple of n bytes (kernels access the caller's buffers
// with 16-byte vector instructions and the CG info with 8-byte stores).
bool aligned_to(const void* p, size_t n);
// Fails unless every non-NULL pointer in ps is 16-byte aligned.
sense_status check_aligned16(std::initializer_list<const void*> ps, const char* names);
// Fails unless d_info and d_rho_hist (either may be NULL) are 8-byte aligned.
sense_status check_info_aligned(const void* d_info, const void* d_rho_hist);
size_t storage_bytes(int st);

}  // namespace sense

struct sense_plan_s {
  using CgArgs = sense::CgArgs;
  using Geom = sense::Geom;
  using Layout = sense::Layout;
  using Tables = sense::Tables;
  sense_desc d;
  Geom g;
  Layout L;
  int device;
  bool full_ops;  // nx is a supported transform length (E, E^H, CG)
  const void* maps;
  char* mem;
  Tables tb;
  int n_rows_s, n_rows_u;
  bool profiling;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used;
  bool busy;  // owned by a serving-engine slot
  int ngroups;      // coil groups of the 2D normal operator and CG (1 .. L.ngroups)
  int adj_groups;   // coil groups of the E^H column pass and RSS (1 .. L.ngroups)
  // whole-solve graph, replayed while the solve arguments repeat
  bool graphs;
  hipStream_t cap_stream;
  hipGraphExec_t gexec;
  struct SolveKey {
    const void* y;
    void* x;
    int32_t max_iter;
    double tol, lambda;
    void* info;
    double* hist;
    bool operator==(const SolveKey& o) const {
      return y == o.y && x == o.x && max_iter == o.max_iter && tol == o.tol && lambda == o.lambda &&
             info == o.info && hist == o.hist;
    }
  } gkey;

  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(mem + off);
  }
  sense::CgVectors vectors(sense::c32* x) const {
    sense::CgVectors v{};
    v.x = x;
    // one group updates r and p in place (every block owns its tile);
    // several groups read the previous iterate while group 0 writes the next
    const bool pp = ngroups > 1;
    v.r[0] = at<sense::c32>(L.r);
    v.r[1] = at<sense::c32>(pp ? L.r2 : L.r);
    v.p[0] = at<sense::c32>(L.p);
    v.p[1] = at<sense::c32>(pp ? L.p2 : L.p);
    v.q = at<sense::c32>(L.q);
    v.qpart = ngroups > 1 ? at<sense::c32>(L.qpart) : nullptr;
    v.ngroups = ngroups;
    return v;
  }
  // the [G][B][nvox] partial sums (null when the workspace holds one group)
  sense::c32* qpart() const { return L.ngroups > 1 ? at<sense::c32>(L.qpart) : nullptr; }
  CgArgs cg_args(double tol, double* hist, int hist_len) const {
    CgArgs a{};
    a.state = at<sense::CgState>(L.state);
    a.eta_part = at<double>(L.eta_part);
    a.zeta_part = at<double>(L.zeta_part);
    a.rr_part = at<double>(L.rr_part);
    a.rr_par = at<double>(L.rr_par);
    a.eta_tiles = L.eta_tiles;
    a.rr_tiles = L.rr_tiles;
    a.cgpart = at<double>(L.cgpart);
    a.part_tiles = ngroups > 1 ? L.rr_tiles : L.eta_tiles;
    a.rho_tiles = L.eta_tiles;
    a.part_stride = std::max(L.eta_tiles, L.rr_tiles);
    a.part_batch = d.batch;
    a.rho_hist = hist;
    a.hist_len = hist_len;
    a.tol = tol;
    return a;
  }
};

// Descriptor-derived fields of a plan (geometry, layout, default coil
// groups; graphs off, no memory); bind_tables points the table pointers
// into p->mem once it is set.
void init_plan_fields(sense_plan_s* p, const sense_desc& d, const void* d_maps);
void bind_tables(sense_plan_s* p);
sense_status check_plan(sense_plan p);
sense_status check_solve_args(sense_plan p, const void* d_y, void* d_x, int32_t max_iter, double rel_tol,
                              double lambda);
hipError_t enqueue_solve_begin(sense_plan p, const void* d_y, sense::c32* x, const sense::CgArgs& cg,
                               hipStream_t st);
hipError_t enqueue_iteration(sense_plan p, sense::c32* x, float lambda, int k, const sense::CgArgs& cg,
                             hipStream_t st);
hipError_t enqueue_solve_end(sense_plan p, sense::c32* x, int K, const sense::CgArgs& cg, sense::CgInfo* d_info,
                             hipStream_t st);
// A whole solve: E^H y, the iterations and the final test (or the one-launch
// small solve).
hipError_t enqueue_solve(sense_plan p, const void* d_y, sense::c32* x, int32_t max_iter, float lambda,
                         const sense::CgArgs& cg, sense::CgInfo* d_info, hipStream_t st);
// Whether the plan's solves run as one whole-solve launch after E^H y, and
// that enqueue.
bool small_solve(const sense_plan_s* p);
hipError_t enqueue_small_solve(sense_plan p, const void* d_y, sense::c32* x, int32_t max_iter, float lambda,
                               const sense::CgArgs& cg, sense::CgInfo* d_info, hipStream_t st);
