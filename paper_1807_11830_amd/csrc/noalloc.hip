// CG-SENSE solve of 2D problems that allocates no device memory.
//
// The solve is the one sense_cg_solve runs (E^H y, the CG iterations, the
// final test), with every table and work vector of a plan (twiddles, mask
// tables, the E^H workspace, r, p, q, coil-group partials, fp64 partials,
// CG state) placed in one file-scope device array instead of a hipMalloc'd
// plan allocation.  The host builds the tables exactly as plan creation
// does and hands them to the device inside kernel arguments (a small copy
// kernel writes them into the array), so no host buffer has to outlive the
// call and nothing is copied from pageable memory.
//
// The array is per device: the runtime gives each GPU its own copy when it
// loads the library there, at its own address, found once per device with
// hipGetSymbolAddress while that device is current.  Host code never uses
// the array's name as an address.  Every call on a device shares that
// device's copy, so calls that overlap on one GPU (two streams, two host
// threads) race; the array keeps the contents of the last call, and the
// solve initialises everything it reads (the same kernels run on a fresh
// hipMalloc'd plan workspace, which holds arbitrary values).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "kernels.hpp"
#include "plan_internal.hpp"
#include "sense.h"

namespace sense {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static void* g_scratch_ptr[kStaticMaxDevices];
static hipError_t g_scratch_err[kStaticMaxDevices];
static std::once_flag g_scratch_once[kStaticMaxDevices];

// Device address of this device's scratch array (looked up once, with the
// device current).
static hipError_t scratch_address(int dev, char** out) {
  std::call_once(g_scratch_once[dev], [dev] {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
  });
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return g_scratch_err[dev];
}

// Words carried by one copy launch (the kernel-argument segment holds 4 KiB).
constexpr int kArgWords = 768;
struct ArgChunk {
  uint32_t* dst;
  uint32_t nwords;
  uint32_t w[kArgWords];
};

__global__ void __launch_bounds__(256) arg_copy_kernel(ArgChunk a) {
  for (uint32_t i = threadIdx.x; i < a.nwords; i += blockDim.x) a.dst[i] = a.w[i];
}

// Copies bytes (a multiple of 4) from host memory to device memory dst
// through kernel arguments, in chunks; the host buffer may be reused as soon
// as this returns.
static hipError_t upload_by_args(char* dst, const void* src, size_t bytes, hipStream_t st) {
  const char* s = static_cast<const char*>(src);
  for (size_t off = 0; off < bytes; off += sizeof(uint32_t) * kArgWords) {
    ArgChunk a;
    const size_t n = std::min(bytes - off, sizeof(uint32_t) * kArgWords);
    a.dst = reinterpret_cast<uint32_t*>(dst + off);
    a.nwords = (uint32_t)(n / sizeof(uint32_t));
    std::memcpy(a.w, s + off, n);
    hipLaunchKernelGGL(arg_copy_kernel, dim3(1), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sense

using namespace sense;

extern "C" sense_status sense_cg_solve_static(const sense_desc* desc, const void* d_maps, const uint8_t* h_mask,
                                              const void* d_y, void* d_x, int32_t max_iter, double rel_tol,
                                              double lambda, sense_cg_info* d_info, double* d_rho_hist,
                                              void* stream) {
  try {
    sense_status s = validate_desc(desc);
    if (s != SENSE_OK) return s;
    const sense_desc& d = *desc;
    if (d.ndim != 2) return fail(SENSE_ERR_UNSUPPORTED, "sense_cg_solve_static supports 2D problems only");
    if (!d_maps) return fail(SENSE_ERR_INVALID, "d_maps is NULL");
    if (check_aligned16({d_maps}, "d_maps") != SENSE_OK) return SENSE_ERR_INVALID;
    if (!h_mask) return fail(SENSE_ERR_INVALID, "h_mask is NULL");
    if (!length_supported(d.nx)) return fail(SENSE_ERR_UNSUPPORTED, "nx is not a supported transform length");
    const Layout L = make_layout(d);
    if (L.total > kStaticScratchBytes)
      return fail(SENSE_ERR_UNSUPPORTED, "problem needs " + std::to_string(L.total) +
                                             " bytes of workspace; sense_cg_solve_static holds at most " +
                                             std::to_string(kStaticScratchBytes) + " (use a plan)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SENSE_ERR_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(SENSE_ERR_UNSUPPORTED, "device index out of range");
    char* mem = nullptr;
    hipError_t e = scratch_address(dev, &mem);
    if (e != hipSuccess || !mem) return device_fail(e, "hipGetSymbolAddress of the static workspace");

    // A plan on the stack over the static workspace (no graphs, no events).
    sense_plan_s p{};
    init_plan_fields(&p, d, d_maps);
    p.device = dev;
    p.mem = mem;

    // Host tables on the stack: every supported length is at most 384.
    constexpr int kMaxLen = 384;
    c32 twx[kMaxLen], twy[kMaxLen];
    uint8_t mask[kMaxLen];
    float mu[kMaxLen];
    int32_t rs[kMaxLen], ru[kMaxLen];
    if (d.nx > kMaxLen || d.ny > kMaxLen) return fail(SENSE_ERR_UNSUPPORTED, "length above 384");
    host_twiddles(d.nx, twx);
    host_twiddles(d.ny, twy);
    host_mask_tables(h_mask, d.ny, 1, mask, mu, rs, ru, &p.n_rows_s, &p.n_rows_u);
    bind_tables(&p);

    s = check_solve_args(&p, d_y, d_x, max_iter, rel_tol, lambda);
    if (s != SENSE_OK) return s;
    s = check_info_aligned(d_info, d_rho_hist);
    if (s != SENSE_OK) return s;

    hipStream_t st = static_cast<hipStream_t>(stream);
    // Word-padded copies of the byte-sized tables (the layout leaves 256-byte
    // aligned room after each).
    uint32_t maskw[kMaxLen / 4];
    std::memset(maskw, 0, sizeof(maskw));
    std::memcpy(maskw, mask, (size_t)d.ny);
    const size_t mask_bytes = ((size_t)d.ny + 3) & ~size_t(3);
    e = upload_by_args(mem + L.tw_x, twx, sizeof(c32) * (size_t)d.nx, st);
    if (e == hipSuccess) e = upload_by_args(mem + L.tw_y, twy, sizeof(c32) * (size_t)d.ny, st);
    if (e == hipSuccess) e = upload_by_args(mem + L.mu_y, mu, sizeof(float) * (size_t)d.ny, st);
    if (e == hipSuccess) e = upload_by_args(mem + L.mask_c, maskw, mask_bytes, st);
    if (e == hipSuccess) e = upload_by_args(mem + L.rows_s, rs, sizeof(int32_t) * (size_t)p.n_rows_s, st);
    if (e == hipSuccess) e = upload_by_args(mem + L.rows_u, ru, sizeof(int32_t) * (size_t)p.n_rows_u, st);
    if (e != hipSuccess) return device_fail(e, "sense_cg_solve_static table upload");

    const CgArgs cg = p.cg_args(rel_tol, d_rho_hist, d_rho_hist ? max_iter + 1 : 0);
    e = enqueue_solve(&p, d_y, static_cast<c32*>(d_x), max_iter, (float)lambda, cg,
                      reinterpret_cast<CgInfo*>(d_info), st);
    return e == hipSuccess ? SENSE_OK : device_fail(e, "sense_cg_solve_static launch");
  } catch (...) {
    return fail(SENSE_ERR_INVALID, "unexpected exception in sense_cg_solve_static");
  }
}
