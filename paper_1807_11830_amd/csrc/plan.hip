// Host runtime behind the C ABI (include/sense.h): plan creation (size
// validation, fp64-built twiddle and mask tables, one workspace
// allocation), argument checking, and the enqueue-only apply and solve calls.
//
// Plan creation is the once-only initialisation of the paper's process
// model (its FFT process bakes the transform plan in init() because that
// takes far longer than a transform); every apply call afterwards only
// enqueues kernels on the caller's stream and never allocates.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "lengths.hpp"
#include "plan_internal.hpp"
#include "sense.h"

namespace sense {

thread_local std::string g_last_error;

sense_status fail(sense_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

bool length_supported(long n) {
  return dispatch_length(n, [](auto) {});
}

static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

size_t storage_bytes(int st) { return st == ST_C64 ? 8 : 4; }

// Bytes of the plan's k-space argument (full grid or sampled lines only).
static size_t kspace_bytes(const sense_plan_s* p) {
  const size_t per_coil = p->d.kspace_compact ? (size_t)p->n_rows_s * p->d.nx
                                              : (size_t)p->d.nx * p->d.ny * p->d.nz;
  return per_coil * p->d.batch * p->d.ncoils * storage_bytes(p->d.kspace_storage);
}


constexpr long kMinSplitVoxels = 8192;

Layout make_layout(const sense_desc& d) {
  Layout L{};
  const size_t nvox = (size_t)d.nx * d.ny * d.nz;
  const size_t B = (size_t)d.batch, C = (size_t)d.ncoils;
  if (d.ndim == 3) {
    L.eta_tiles = adj_tiles(d.nx, d.ny, d.nz);
  } else {
    const int tx = ehe_tile_width(d.ny);
    L.eta_tiles = (int)((d.nx + tx - 1) / tx);
  }
  L.rr_tiles = cg_tiles((long)nvox);
  L.ngroups = d.ndim == 2 ? auto_coil_groups(d.nx, d.ny, d.ncoils, d.batch) : 1;
  // Default splits: the fill split, and none below kMinSplitVoxels per
  // slice, where the combine launch costs more than the split saves
  // (measured on MI355X, 20 CG iterations: 64^2 x 4 coils 229 us unsplit,
  // 285 us at G = 2; 96^2 x 8 coils 504 us unsplit, 402 us at G = 4).  With
  // the combine's group partials loaded together, whole solves take the
  // fill split too (320^2 x 32 coils: 0.893 ms at G = 16, 0.974 ms at
  // G = 8; 256^2 x 16 coils: 0.593 ms at G = 8, 0.705 ms at G = 4).  The
  // normal operator with CG, and the E^H column pass with RSS, keep
  // separate settings (both the fill split by default).
  const bool small = (long)d.nx * d.ny < kMinSplitVoxels;
  L.dgroups = small ? 1 : L.ngroups;
  L.agroups = small ? 1 : L.ngroups;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.tw_x = take(sizeof(c32) * (size_t)d.nx);
  L.tw_y = take(sizeof(c32) * (size_t)d.ny);
  L.tw_z = take(sizeof(c32) * (size_t)d.nz);
  L.mu_y = take(sizeof(float) * (size_t)d.ny);
  L.mask_c = take((size_t)d.ny * d.nz);
  L.rows_s = take(sizeof(int32_t) * (size_t)d.ny * d.nz);
  L.rows_u = take(sizeof(int32_t) * (size_t)d.ny * d.nz);
  L.work = take(sizeof(c32) * B * C * nvox);
  L.r = take(sizeof(c32) * B * nvox);
  L.p = take(sizeof(c32) * B * nvox);
  L.q = take(sizeof(c32) * B * nvox);
  // with coil groups the 2D CG double-buffers r and p and keeps
  // [G][B][nvox] partial coil sums
  L.r2 = L.ngroups > 1 ? take(sizeof(c32) * B * nvox) : L.r;
  L.p2 = L.ngroups > 1 ? take(sizeof(c32) * B * nvox) : L.p;
  L.qpart = L.ngroups > 1 ? take(sizeof(c32) * (size_t)L.ngroups * B * nvox) : 0;
  L.state = take(sizeof(CgState) * B);
  L.eta_part = take(sizeof(double) * B * (size_t)L.eta_tiles);
  L.zeta_part = take(sizeof(double) * B * (size_t)L.eta_tiles);
  L.rr_part = take(sizeof(double) * B * (size_t)L.rr_tiles);
  L.rr_par = take(sizeof(double) * 2 * B * (size_t)L.rr_tiles);
  const size_t ptiles = (size_t)std::max(L.eta_tiles, L.rr_tiles);
  L.cgpart = take(sizeof(double) * 2 * B * ptiles * kCgParts);
  L.info = take(sizeof(CgInfo) * B);
  L.total = off;
  return L;
}

sense_status validate_desc(const sense_desc* d) {
  if (!d) return fail(SENSE_ERR_INVALID, "desc is NULL");
  if (d->ndim != 2 && d->ndim != 3) return fail(SENSE_ERR_INVALID, "ndim must be 2 or 3");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->ncoils < 1 || d->batch < 1)
    return fail(SENSE_ERR_INVALID, "sizes, coils and batch must be >= 1");
  if (d->ndim == 2 && d->nz != 1) return fail(SENSE_ERR_INVALID, "ndim = 2 needs nz = 1");
  for (int st : {d->maps_storage, d->kspace_storage})
    if (st < SENSE_C64 || st > SENSE_FP16X2) return fail(SENSE_ERR_INVALID, "unknown storage format");
  if (d->maps_shared != 0 && d->maps_shared != 1) return fail(SENSE_ERR_INVALID, "maps_shared must be 0 or 1");
  if (d->kspace_compact != 0 && d->kspace_compact != 1)
    return fail(SENSE_ERR_INVALID, "kspace_compact must be 0 or 1");
  if (d->ndim == 3 && !length_supported(d->nz))
    return fail(SENSE_ERR_UNSUPPORTED, "nz=" + std::to_string(d->nz) + " is not a supported transform length");
  if (!length_supported(d->ny))
    return fail(SENSE_ERR_UNSUPPORTED, "ny=" + std::to_string(d->ny) + " is not a supported transform length");
  if (d->batch > 65535 || d->ncoils > 65535) return fail(SENSE_ERR_UNSUPPORTED, "batch and coils must be <= 65535");
  // one image (or one coil image) is addressed with 32-bit byte offsets
  if ((double)d->nx * d->ny * d->nz * 8.0 > 2147483647.0)
    return fail(SENSE_ERR_UNSUPPORTED, "one image must be below 2^31 bytes");
  const double elems = (double)d->nx * d->ny * d->nz * d->ncoils * d->batch;
  if (elems > 4.0e12) return fail(SENSE_ERR_UNSUPPORTED, "problem too large");
  return SENSE_OK;
}


void host_twiddles(long n, c32* out) {
  // exp(-2 pi i e / n) in fp64, rounded once to fp32
  for (long e2 = 0; e2 < n; ++e2) {
    const double a = -2.0 * 3.141592653589793238462643383279502884 * (double)e2 / (double)n;
    out[e2] = c32{(float)std::cos(a), (float)std::sin(a)};
  }
}

void host_mask_tables(const uint8_t* h_mask, long ny, long nz, uint8_t* mask, float* mu, int32_t* rows_s,
                      int32_t* rows_u, int* n_s, int* n_u) {
  int ns = 0, nu = 0;
  for (long i = 0; i < ny * nz; ++i) {
    mask[i] = h_mask[i] ? 1 : 0;
    if (mask[i]) rows_s[ns++] = (int32_t)i;
    else rows_u[nu++] = (int32_t)i;
  }
  // Uncentred mask of the hybrid normal operator with the 1/ny of the
  // unnormalised forward/inverse pair folded in.
  for (long k = 0; k < ny; ++k) mu[k] = mask[(k + ny / 2) % ny] ? (float)(1.0 / (double)ny) : 0.f;
  *n_s = ns;
  *n_u = nu;
}

}  // namespace sense

void init_plan_fields(sense_plan_s* p, const sense_desc& d, const void* d_maps) {
  p->d = d;
  p->maps = d_maps;
  p->full_ops = sense::length_supported(d.nx);
  p->profiling = false;
  p->events_used = 0;
  p->graphs = false;
  p->busy = false;
  p->cap_stream = nullptr;
  p->gexec = nullptr;
  p->mem = nullptr;
  p->L = sense::make_layout(d);
  p->ngroups = p->L.dgroups;
  p->adj_groups = p->L.agroups;
  const size_t nvox = (size_t)d.nx * d.ny * d.nz;
  p->g.nx = d.nx;
  p->g.ny = d.ny;
  p->g.nz = d.nz;
  p->g.ncoils = d.ncoils;
  p->g.batch = d.batch;
  p->g.maps_bstride = d.maps_shared ? 0 : (long)(nvox * d.ncoils);
  p->g.maps_storage = d.maps_storage;
  p->g.kspace_storage = d.kspace_storage;
  p->g.kspace_compact = d.kspace_compact;
}

void bind_tables(sense_plan_s* p) {
  using namespace sense;
  p->tb.tw_x = p->at<c32>(p->L.tw_x);
  p->tb.tw_y = p->at<c32>(p->L.tw_y);
  p->tb.tw_z = p->at<c32>(p->L.tw_z);
  p->tb.mu_y = p->at<float>(p->L.mu_y);
  p->tb.mask_c = p->at<uint8_t>(p->L.mask_c);
  p->tb.rows_s = p->at<int32_t>(p->L.rows_s);
  p->tb.n_rows_s = p->n_rows_s;
  p->tb.rows_u = p->at<int32_t>(p->L.rows_u);
  p->tb.n_rows_u = p->n_rows_u;
}

using namespace sense;


sense_status check_plan(sense_plan p) {
  if (!p) return fail(SENSE_ERR_INVALID, "plan is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(SENSE_ERR_STATE, "current HIP device differs from the plan's device");
  return SENSE_OK;
}

bool sense::overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

sense_status sense::device_fail(hipError_t e, const char* what) {
  return fail(SENSE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static sense_status timed_ehe_begin(sense_plan p, hipStream_t st, hipEvent_t* stop) {
  *stop = nullptr;
  if (!p->profiling) return SENSE_OK;
  if (p->events_used == p->events.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
      return fail(SENSE_ERR_DEVICE, "hipEventCreate failed");
    p->events.emplace_back(a, b);
  }
  auto& pr = p->events[p->events_used++];
  if (hipEventRecord(pr.first, st) != hipSuccess) return fail(SENSE_ERR_DEVICE, "hipEventRecord failed");
  *stop = pr.second;
  return SENSE_OK;
}

// Solve pieces (also used by the serving engine): E^H y and CG init; one
// iteration; the final test.  All enqueue only.
hipError_t enqueue_solve_begin(sense_plan p, const void* d_y, c32* x, const CgArgs& cg,
                                      hipStream_t st) {
  c32* r = p->at<c32>(p->L.r);
  hipError_t e = launch_EH(p->g, p->tb, p->maps, d_y, p->at<c32>(p->L.work), r, p->qpart(), p->adj_groups, st);
  if (e == hipSuccess) e = launch_cg_init(p->g, r, x, r, p->at<c32>(p->L.p), p->at<c32>(p->L.q), cg, st);
  return e;
}

hipError_t enqueue_iteration(sense_plan p, c32* x, float lambda, int k, const CgArgs& cg, hipStream_t st) {
  c32* r = p->at<c32>(p->L.r);
  c32* pv = p->at<c32>(p->L.p);
  c32* q = p->at<c32>(p->L.q);
  hipEvent_t stop = nullptr;
  if (timed_ehe_begin(p, st, &stop) != SENSE_OK) return hipErrorUnknown;
  hipError_t e;
  if (p->d.ndim == 3) {
    // q = A p with the Re<p, q> and <q, q> partials, then one update of x,
    // r and p (single reduction, as in the fused 2D iteration)
    e = launch_EHE_composed(p->g, p->tb, p->maps, pv, q, p->at<c32>(p->L.work), lambda, cg.eta_part,
                            cg.zeta_part, st);
    if (stop && e == hipSuccess) e = hipEventRecord(stop, st);
    if (e == hipSuccess) e = launch_cg_update_fused(p->g, x, r, pv, q, k, cg, st);
  } else {
    // one launch (plus the combine pass with coil groups): the updates of
    // iteration k-1 fused in front of q = A p
    e = launch_ehe_cg(p->g, p->tb, p->maps, p->vectors(x), lambda, k, cg, st);
    if (stop && e == hipSuccess) e = hipEventRecord(stop, st);
  }
  return e;
}

hipError_t enqueue_solve_end(sense_plan p, c32* x, int K, const CgArgs& cg, CgInfo* d_info, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (p->d.ndim != 3 && K > 0) e = launch_cg_fused_final(p->g, p->vectors(x), K, cg, st);
  // 3D: the last update left rho_K's partials in its parity buffer
  CgArgs cf = cg;
  if (p->d.ndim == 3) cf.rr_part = const_cast<double*>(cg3_rr_in(cg, p->d.batch, K));
  if (e == hipSuccess) e = launch_cg_finish(p->g, cf, p->at<CgInfo>(p->L.info), d_info, st);
  return e;
}

bool small_solve(const sense_plan_s* p) { return p->d.ndim == 2 && p->ngroups == 1 && small_solve_supported(p->g); }

// Small slices: the x rows of E^H y, then one launch finishes E^H y and
// runs the whole solve.
hipError_t enqueue_small_solve(sense_plan p, const void* d_y, c32* x, int32_t max_iter, float lambda,
                               const CgArgs& cg, CgInfo* d_info, hipStream_t st) {
  c32* work = p->at<c32>(p->L.work);
  hipError_t e = launch_EH_rows(p->g, p->tb, d_y, work, st);
  hipEvent_t stop = nullptr;
  if (e == hipSuccess && timed_ehe_begin(p, st, &stop) != SENSE_OK) e = hipErrorUnknown;
  if (e == hipSuccess)
    e = launch_cg_small(p->g, p->tb, p->maps, work, x, max_iter, lambda, cg, p->at<CgInfo>(p->L.info), d_info, st);
  if (stop && e == hipSuccess) e = hipEventRecord(stop, st);
  return e;
}

hipError_t enqueue_solve(sense_plan p, const void* d_y, c32* x, int32_t max_iter, float lambda, const CgArgs& cg,
                         CgInfo* d_info, hipStream_t st) {
  if (small_solve(p)) return enqueue_small_solve(p, d_y, x, max_iter, lambda, cg, d_info, st);
  hipError_t e = enqueue_solve_begin(p, d_y, x, cg, st);
  for (int k = 0; k < max_iter && e == hipSuccess; ++k) e = enqueue_iteration(p, x, lambda, k, cg, st);
  if (e == hipSuccess) e = enqueue_solve_end(p, x, max_iter, cg, d_info, st);
  return e;
}

namespace sense {

bool aligned_to(const void* p, size_t n) { return reinterpret_cast<uintptr_t>(p) % n == 0; }

sense_status check_aligned16(std::initializer_list<const void*> ps, const char* names) {
  for (const void* q : ps)
    if (q && !aligned_to(q, 16)) return fail(SENSE_ERR_INVALID, std::string(names) + " must be 16-byte aligned");
  return SENSE_OK;
}

sense_status check_info_aligned(const void* d_info, const void* d_rho_hist) {
  if ((d_info && !aligned_to(d_info, 8)) || (d_rho_hist && !aligned_to(d_rho_hist, 8)))
    return fail(SENSE_ERR_INVALID, "d_info and d_rho_hist must be 8-byte aligned");
  return SENSE_OK;
}

}  // namespace sense

sense_status check_solve_args(sense_plan p, const void* d_y, void* d_x, int32_t max_iter,
                                     double rel_tol, double lambda) {
  if (!d_x || !d_y) return fail(SENSE_ERR_INVALID, "d_x and d_y must be non-NULL");
  if (check_aligned16({d_x, d_y}, "d_x and d_y") != SENSE_OK) return SENSE_ERR_INVALID;
  if (!p->full_ops) return fail(SENSE_ERR_UNSUPPORTED, "nx is not a supported transform length");
  if (max_iter < 0) return fail(SENSE_ERR_INVALID, "max_iter must be >= 0");
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return fail(SENSE_ERR_INVALID, "rel_tol must be finite and >= 0");
  if (!std::isfinite(lambda)) return fail(SENSE_ERR_INVALID, "lambda must be finite");
  const size_t nvox = (size_t)p->d.nx * p->d.ny * p->d.nz;
  const size_t xb = nvox * p->d.batch * sizeof(c32);
  const size_t yb = kspace_bytes(p);
  if (overlap(d_x, xb, d_y, yb)) return fail(SENSE_ERR_INVALID, "d_x and d_y overlap");
  if (overlap(d_x, xb, p->mem, p->L.total) || overlap(d_y, yb, p->mem, p->L.total))
    return fail(SENSE_ERR_INVALID, "buffers overlap the plan workspace");
  return SENSE_OK;
}

extern "C" {

size_t sense_plan_device_bytes(const sense_desc* desc) {
  if (validate_desc(desc) != SENSE_OK) return 0;
  return make_layout(*desc).total;
}

sense_status sense_plan_create(const sense_desc* desc, const void* d_maps, const uint8_t* h_mask,
                               void* stream, sense_plan* out) {
  try {
    if (!out) return fail(SENSE_ERR_INVALID, "out is NULL");
    *out = nullptr;
    sense_status s = validate_desc(desc);
    if (s != SENSE_OK) return s;
    if (!d_maps) return fail(SENSE_ERR_INVALID, "d_maps is NULL");
    if (check_aligned16({d_maps}, "d_maps") != SENSE_OK) return SENSE_ERR_INVALID;
    if (!h_mask) return fail(SENSE_ERR_INVALID, "h_mask is NULL");
    const sense_desc& d = *desc;
    hipStream_t st = static_cast<hipStream_t>(stream);

    auto* p = new (std::nothrow) sense_plan_s();
    if (!p) return fail(SENSE_ERR_NOMEM, "host allocation failed");
    init_plan_fields(p, d, d_maps);
    p->graphs = true;
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return fail(SENSE_ERR_DEVICE, "hipGetDevice failed");
    }

    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->mem), p->L.total);
    if (e != hipSuccess) {
      delete p;
      return fail(SENSE_ERR_NOMEM, "hipMalloc of " + std::to_string(p->L.total) + " bytes failed");
    }

    std::vector<c32> twx((size_t)d.nx), twy((size_t)d.ny), twz((size_t)d.nz);
    host_twiddles(d.nx, twx.data());
    host_twiddles(d.ny, twy.data());
    host_twiddles(d.nz, twz.data());
    const long rows_total = d.ny * d.nz;
    std::vector<uint8_t> mask((size_t)rows_total);
    std::vector<int32_t> rs((size_t)rows_total), ru((size_t)rows_total);
    std::vector<float> mu((size_t)d.ny);
    host_mask_tables(h_mask, d.ny, d.nz, mask.data(), mu.data(), rs.data(), ru.data(), &p->n_rows_s,
                     &p->n_rows_u);
    rs.resize((size_t)p->n_rows_s);
    ru.resize((size_t)p->n_rows_u);

    auto up = [&](size_t off, const void* src, size_t bytes) {
      if (bytes == 0 || e != hipSuccess) return;
      e = hipMemcpyAsync(p->mem + off, src, bytes, hipMemcpyHostToDevice, st);
    };
    up(p->L.tw_x, twx.data(), twx.size() * sizeof(c32));
    up(p->L.tw_y, twy.data(), twy.size() * sizeof(c32));
    up(p->L.tw_z, twz.data(), twz.size() * sizeof(c32));
    up(p->L.mu_y, mu.data(), mu.size() * sizeof(float));
    up(p->L.mask_c, mask.data(), mask.size());
    up(p->L.rows_s, rs.data(), rs.size() * sizeof(int32_t));
    up(p->L.rows_u, ru.data(), ru.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      (void)hipFree(p->mem);
      delete p;
      return device_fail(e, "table upload");
    }
    bind_tables(p);
    *out = p;
    return SENSE_OK;
  } catch (...) {
    return fail(SENSE_ERR_INVALID, "unexpected exception in sense_plan_create");
  }
}

sense_status sense_plan_destroy(sense_plan p) {
  if (!p) return fail(SENSE_ERR_INVALID, "plan is NULL");
  if (p->busy) return fail(SENSE_ERR_STATE, "plan is in a serving-engine slot");
  (void)hipDeviceSynchronize();
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (auto& pr : p->events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  (void)hipFree(p->mem);
  delete p;
  return SENSE_OK;
}

sense_status sense_apply_E(sense_plan p, const void* d_x, void* d_y, void* stream) {
  sense_status s = check_plan(p);
  if (s != SENSE_OK) return s;
  if (!d_x || !d_y) return fail(SENSE_ERR_INVALID, "d_x and d_y must be non-NULL");
  if (check_aligned16({d_x, d_y}, "d_x and d_y") != SENSE_OK) return SENSE_ERR_INVALID;
  if (!p->full_ops) return fail(SENSE_ERR_UNSUPPORTED, "nx is not a supported transform length");
  const size_t nvox = (size_t)p->d.nx * p->d.ny * p->d.nz;
  const size_t xb = nvox * p->d.batch * sizeof(c32);
  const size_t yb = kspace_bytes(p);
  if (overlap(d_x, xb, d_y, yb)) return fail(SENSE_ERR_INVALID, "d_x and d_y overlap");
  hipError_t e = launch_E(p->g, p->tb, p->maps, static_cast<const c32*>(d_x), p->at<c32>(p->L.work), d_y,
                          static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_apply_E launch");
}

sense_status sense_apply_EH(sense_plan p, const void* d_y, void* d_x, void* stream) {
  sense_status s = check_plan(p);
  if (s != SENSE_OK) return s;
  if (!d_x || !d_y) return fail(SENSE_ERR_INVALID, "d_x and d_y must be non-NULL");
  if (check_aligned16({d_x, d_y}, "d_x and d_y") != SENSE_OK) return SENSE_ERR_INVALID;
  if (!p->full_ops) return fail(SENSE_ERR_UNSUPPORTED, "nx is not a supported transform length");
  const size_t nvox = (size_t)p->d.nx * p->d.ny * p->d.nz;
  const size_t xb = nvox * p->d.batch * sizeof(c32);
  const size_t yb = kspace_bytes(p);
  if (overlap(d_x, xb, d_y, yb)) return fail(SENSE_ERR_INVALID, "d_x and d_y overlap");
  hipError_t e = launch_EH(p->g, p->tb, p->maps, d_y, p->at<c32>(p->L.work), static_cast<c32*>(d_x),
                           p->qpart(), p->adj_groups, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_apply_EH launch");
}

sense_status sense_apply_rss(sense_plan p, const void* d_y, float* d_img, void* stream) {
  sense_status s = check_plan(p);
  if (s != SENSE_OK) return s;
  if (!d_y || !d_img) return fail(SENSE_ERR_INVALID, "d_y and d_img must be non-NULL");
  if (check_aligned16({d_y, d_img}, "d_y and d_img") != SENSE_OK) return SENSE_ERR_INVALID;
  if (!p->full_ops) return fail(SENSE_ERR_UNSUPPORTED, "nx is not a supported transform length");
  const size_t nvox = (size_t)p->d.nx * p->d.ny * p->d.nz;
  const size_t ob = nvox * p->d.batch * sizeof(float);
  const size_t yb = kspace_bytes(p);
  if (overlap(d_img, ob, d_y, yb)) return fail(SENSE_ERR_INVALID, "d_img and d_y overlap");
  hipError_t e = launch_rss(p->g, p->tb, d_y, p->at<c32>(p->L.work), d_img, p->qpart(), p->adj_groups,
                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_apply_rss launch");
}

sense_status sense_apply_EHE(sense_plan p, const void* d_p, void* d_q, double lambda, void* stream) {
  sense_status s = check_plan(p);
  if (s != SENSE_OK) return s;
  if (!d_p || !d_q) return fail(SENSE_ERR_INVALID, "d_p and d_q must be non-NULL");
  if (check_aligned16({d_p, d_q}, "d_p and d_q") != SENSE_OK) return SENSE_ERR_INVALID;
  if (!std::isfinite(lambda)) return fail(SENSE_ERR_INVALID, "lambda must be finite");
  const size_t bytes = (size_t)p->d.nx * p->d.ny * p->d.nz * p->d.batch * sizeof(c32);
  if (overlap(d_p, bytes, d_q, bytes)) return fail(SENSE_ERR_INVALID, "d_p and d_q overlap");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t stop;
  s = timed_ehe_begin(p, st, &stop);
  if (s != SENSE_OK) return s;
  hipError_t e = p->d.ndim == 3
                     ? launch_EHE_composed(p->g, p->tb, p->maps, static_cast<const c32*>(d_p),
                                           static_cast<c32*>(d_q), p->at<c32>(p->L.work), (float)lambda,
                                           p->at<double>(p->L.eta_part), nullptr, st)
                     : launch_ehe(p->g, p->tb, p->maps, static_cast<const c32*>(d_p), static_cast<c32*>(d_q),
                                  (float)lambda, nullptr, p->at<c32>(p->L.qpart), p->ngroups, st);
  if (stop && e == hipSuccess) e = hipEventRecord(stop, st);
  return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_apply_EHE launch");
}

sense_status sense_cg_solve(sense_plan p, const void* d_y, void* d_x, int32_t max_iter, double rel_tol,
                            double lambda, sense_cg_info* d_info, double* d_rho_hist, void* stream) {
  sense_status s = check_plan(p);
  if (s != SENSE_OK) return s;
  s = check_solve_args(p, d_y, d_x, max_iter, rel_tol, lambda);
  if (s != SENSE_OK) return s;
  s = check_info_aligned(d_info, d_rho_hist);
  if (s != SENSE_OK) return s;
  if (p->busy) return fail(SENSE_ERR_STATE, "plan is in a serving-engine slot");
  hipStream_t st = static_cast<hipStream_t>(stream);
  c32* x = static_cast<c32*>(d_x);
  CgInfo* info2 = reinterpret_cast<CgInfo*>(d_info);
  const CgArgs cg = p->cg_args(rel_tol, d_rho_hist, d_rho_hist ? max_iter + 1 : 0);

  // A small slice's solve is two launches (the x rows of E^H y, then the
  // rest of E^H y and the whole loop), where a graph launch costs more than
  // it saves (measured with one launch more, 64^2 x 4 coils, 20 iterations:
  // 144 us replayed, 138 us eager), so it always runs eagerly.
  if (!p->graphs || p->profiling || small_solve(p)) {
    hipError_t e = enqueue_solve(p, d_y, x, max_iter, (float)lambda, cg, info2, st);
    return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_cg_solve launch");
  }
  // Graph path: capture the whole solve once on the plan's private stream,
  // then replay it on the caller's stream while the arguments repeat.
  const sense_plan_s::SolveKey key{d_y, d_x, max_iter, rel_tol, lambda, d_info, d_rho_hist};
  hipError_t e = hipSuccess;
  if (!p->gexec || !(key == p->gkey)) {
    if (p->gexec) {
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
    }
    if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = enqueue_solve(p, d_y, x, max_iter, (float)lambda, cg, info2, p->cap_stream);
      e = hipStreamEndCapture(p->cap_stream, &graph);
      if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      p->gexec = nullptr;
      return device_fail(e, "sense_cg_solve graph capture");
    }
    p->gkey = key;
  }
  e = hipGraphLaunch(p->gexec, st);
  return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_cg_solve graph launch");
}

sense_status sense_plan_set_maps(sense_plan p, const void* d_maps) {
  sense_status s = check_plan(p);
  if (s != SENSE_OK) return s;
  if (!d_maps) return fail(SENSE_ERR_INVALID, "d_maps is NULL");
  if (check_aligned16({d_maps}, "d_maps") != SENSE_OK) return SENSE_ERR_INVALID;
  if (p->busy) return fail(SENSE_ERR_STATE, "plan is in a serving-engine slot");
  p->maps = d_maps;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  return SENSE_OK;
}

sense_status sense_plan_set_coil_groups(sense_plan p, int32_t groups) {
  if (!p) return fail(SENSE_ERR_INVALID, "plan is NULL");
  if (p->busy) return fail(SENSE_ERR_STATE, "plan is in a serving-engine slot");
  if (groups < 0) return fail(SENSE_ERR_INVALID, "groups must be >= 0");
  if (groups > p->L.ngroups)
    return fail(SENSE_ERR_UNSUPPORTED, "at most " + std::to_string(p->L.ngroups) +
                                           " coil groups fit this plan's workspace");
  const int g = groups == 0 ? p->L.dgroups : groups;
  const int ga = groups == 0 ? p->L.agroups : groups;
  if ((g != p->ngroups || ga != p->adj_groups) && p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  p->ngroups = g;
  p->adj_groups = ga;
  return SENSE_OK;
}

sense_status sense_plan_coil_groups(sense_plan p, int32_t* groups, int32_t* max_groups) {
  if (!p) return fail(SENSE_ERR_INVALID, "plan is NULL");
  if (groups) *groups = p->ngroups;
  if (max_groups) *max_groups = p->L.ngroups;
  return SENSE_OK;
}

sense_status sense_plan_set_graphs(sense_plan p, int32_t enable) {
  if (!p) return fail(SENSE_ERR_INVALID, "plan is NULL");
  p->graphs = enable != 0;
  return SENSE_OK;
}

sense_status sense_plan_cg_info(sense_plan p, sense_cg_info* h_info, void* stream) {
  sense_status s = check_plan(p);
  if (s != SENSE_OK) return s;
  if (!h_info) return fail(SENSE_ERR_INVALID, "h_info is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(h_info, p->at<CgInfo>(p->L.info), sizeof(CgInfo) * p->d.batch,
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_plan_cg_info copy");
}

sense_status sense_plan_set_profiling(sense_plan p, int32_t enable) {
  if (!p) return fail(SENSE_ERR_INVALID, "plan is NULL");
  p->profiling = enable != 0;
  p->events_used = 0;
  return SENSE_OK;
}

sense_status sense_plan_profile(sense_plan p, int64_t* n_launches, double* total_ms) {
  if (!p) return fail(SENSE_ERR_INVALID, "plan is NULL");
  if (!n_launches || !total_ms) return fail(SENSE_ERR_INVALID, "outputs must be non-NULL");
  double tot = 0.0;
  for (size_t i = 0; i < p->events_used; ++i) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(p->events[i].second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->events[i].first, p->events[i].second);
    if (e != hipSuccess) return device_fail(e, "hipEventElapsedTime");
    tot += ms;
  }
  *n_launches = (int64_t)p->events_used;
  *total_ms = tot;
  p->events_used = 0;
  return SENSE_OK;
}

const char* sense_last_error(void) { return g_last_error.c_str(); }

const char* sense_version(void) { return "sense-gfx950 0.1"; }

}  // extern "C"

static_assert(sizeof(sense_cg_info) == sizeof(CgInfo), "info layout");
