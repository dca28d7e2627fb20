// Internal interface between the host runtime (plan.hip) and the kernel
// launchers (kernels_*.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cplx.hpp"

namespace sense {

// Per-batch-element CG state, device resident.  rho[k & 1] holds rho_k, so
// a kernel of iteration k can read rho_(k-1) while the designated block of
// the same launch publishes rho_k.
// rho_cur is rho_k of the current iteration, published by the fused E^H E
// launch for the update launch that follows it.
struct CgState {
  int32_t iter;     // completed updates of x; advanced by the update launch
  int32_t status;   // CG_RUNNING while the loop goes on
  int32_t pad0, pad1;
  double rho0;
  double rho[2];
  double rho_cur;
};

enum : int32_t {
  CG_MAXITER = 0,
  CG_CONVERGED = 1,
  CG_EXACT = 2,
  CG_BREAKDOWN = 3,
  CG_NONFINITE = 4,
  CG_RUNNING = -1
};

// Matches the public sense_cg_info layout.
struct CgInfo {
  int32_t iters_run;
  int32_t status;
  double rho0;
  double rho_final;
};

// Geometry of one operator instance (2D: nz = 1).
struct Geom {
  long nx, ny, nz;
  int ncoils;
  int batch;
  long maps_bstride;  // elements between batch elements of the maps (0 = shared)
  int maps_storage;   // Storage
  int kspace_storage; // Storage
  int kspace_compact; // k-space holds the sampled lines only
};

// Device tables owned by the plan.
struct Tables {
  const c32* tw_x;        // exp(-2 pi i e / nx), e < nx
  const c32* tw_y;        // exp(-2 pi i e / ny)
  const c32* tw_z;        // exp(-2 pi i e / nz)
  const float* mu_y;      // 2D hybrid: uncentred mask / ny, [ny]
  const uint8_t* mask_c;  // centred mask [nz][ny]
  const int32_t* rows_s;  // sampled row ids z*ny + y
  int n_rows_s;
  const int32_t* rows_u;  // unsampled row ids
  int n_rows_u;
};

// fp64 partials a fused 2D CG launch leaves per block: Re<p, q>, <q, q>
// and <r, r> (in that order).
constexpr int kCgParts = 3;

struct CgArgs {
  CgState* state;        // [B]
  double* eta_part;      // [B][eta_tiles]
  double* zeta_part;     // [B][eta_tiles] (3D: <q, q> partials of the normal operator)
  double* rr_part;       // [B][rr_tiles]
  double* rr_par;        // 3D: [2][B][rr_tiles], <r, r> partials by iteration parity
  int eta_tiles;
  int rr_tiles;
  // fused 2D iteration: [2][B][part_stride][kCgParts] partials (Re<p,q>,
  // <q,q>, <r,r>), double-buffered by iteration parity.  Re<p,q> and <q,q>
  // come from the blocks that form q (part_tiles of them: the fused kernel's
  // column tiles with one coil group, the combine pass's tiles with
  // several); <r,r> from the blocks that update r (rho_tiles: the column
  // tiles of the fused kernel, coil group 0).
  double* cgpart;
  int part_tiles;
  int rho_tiles;
  int part_stride;
  int part_batch;
  double* rho_hist;      // optional [B][hist_len]
  int hist_len;
  double tol;
};

// Arguments of the fused 2D normal-operator kernel (one launch, or one row
// of a batched table launch) and of its coil-group combine pass.
//
// Coil groups: with ngroups = G > 1 the coils are split into G contiguous
// ranges, one block per (column tile, batch element, group); each block
// writes its partial sum over its coils to qpart[g][b] and the combine pass
// adds the G partials in group order (deterministic), adds lambda p and
// emits the partials of the scalars.  G = 1 does all of it in one launch.
//
// With coil groups the CG vectors r and p are double-buffered: launch k
// reads r_in, p_in (iterate k-1) and writes r_out, p_out (iterate k), so
// blocks of other groups never see a half-updated vector.  With one group
// r_out = r_in and p_out = p_in (each block updates its own tile in place).
struct EheParams {
  const void* maps;
  const c32* r;      // CG: r_(k-1) (input of the update); apply: unused
  c32* r_out;        // CG: r_k
  const c32* p_in;   // apply: p; CG: p_(k-1)
  c32* p_out;        // CG: p_k
  c32* q;            // A p (CG: also q_(k-1) on input)
  c32* qpart;        // G > 1: [G][qpart_gstride] partial coil sums
  long qpart_gstride;  // elements between groups (batch * nvox)
  int ngroups;
  const c32* tw;     // [ny]
  const float* mu;   // [ny]
  double* eta_part;  // [B][ntiles] or null
  int ntiles;        // column tiles of one batch element
  long nx;
  long nvox;
  long maps_bstride;
  int ncoils;
  float lambda;
  // CG only
  c32* x;
  CgState* state;
  const double* rr_part;
  int rr_tiles;
  double* cgpart;
  int part_batch;
  int part_tiles;    // blocks leaving Re<p,q>, <q,q> (ntiles for G = 1, cg_tiles(nvox) for G > 1)
  int rho_tiles;     // blocks leaving <r,r> (ntiles)
  int part_stride;   // entries per batch element of the cgpart layout
  int k;             // iteration index of this launch
  double* rho_hist;
  int hist_len;
  double tol;
};

// Device vectors of one 2D CG problem (single plan or serving slot).
struct CgVectors {
  c32* x;
  c32* r[2];  // r[k & 1] is the input of launch k (the same buffer twice for G = 1)
  c32* p[2];
  c32* q;
  c32* qpart;  // [G][B][nvox] when G > 1
  int ngroups;
};

// Supported transform lengths (compile-time instantiations).
bool length_supported(long n);
// Tiles of the fused E^H E kernel along x for a given ny.
int ehe_tile_width(long ny);
// Tiles of the CG vector kernels per batch element.
int cg_tiles(long nvox);

// Coil groups: with fewer than kFillBlocks (tiles x batch) blocks the fused
// kernel splits the coils into G = ceil(kFillBlocks / blocks) groups, at
// most ncoils / 2 (two coils per group) and kMaxCoilGroups.  Measured on
// MI355X: a split pays off below about 512 blocks (256^2 x 16 coils, one
// slice: 50.7 us unsplit, 22.9 us at G = 8; 384^2 x 32 coils x 8 slices:
// 194 us unsplit, 142 us at G = 2) and costs above it (160 slices of 256^2:
// 266 us unsplit, 354 us at G = 2).
constexpr int kFillBlocks = 512;
constexpr int kMaxCoilGroups = 16;
// Automatic coil-group count of a 2D plan (1 for 3D).
int auto_coil_groups(long nx, long ny, int ncoils, int batch);

// Launchers; return hipSuccess or the launch error.
// q = E^H E p + lambda p; qpart is the [G][B][nvox] scratch when ngroups > 1.
hipError_t launch_ehe(const Geom& g, const Tables& tb, const void* maps, const c32* p, c32* q,
                      float lambda, double* eta_part, c32* qpart, int ngroups, hipStream_t st);
// Fused CG iteration k (2D): finishes iteration k-1 (x, r, p updates) and
// computes q = A p with the partials of the next scalars (with G > 1: the
// group launch and its combine pass).
hipError_t launch_ehe_cg(const Geom& g, const Tables& tb, const void* maps, const CgVectors& v,
                         float lambda, int k, const CgArgs& cg, hipStream_t st);
// After K fused iterations: x, r updates of iteration K-1 and <r, r>.
hipError_t launch_cg_fused_final(const Geom& g, const CgVectors& v, int K, const CgArgs& cg, hipStream_t st);
// x = 0, r = p = b, q = 0 (q may be null), the <r, r> partials and a fresh
// CgState per batch element.
hipError_t launch_cg_init(const Geom& g, const c32* b, c32* x, c32* r, c32* p, c32* q,
                          const CgArgs& cg, hipStream_t st);
hipError_t launch_cg_finish(const Geom& g, const CgArgs& cg, CgInfo* info, CgInfo* info2, hipStream_t st);
// 3D CG iteration k after q = A p (with the Re<p, q> and <q, q> partials):
// the start-of-iteration tests on rho_k, then x += alpha p, r -= alpha q and
// p = r + beta p with beta from alpha^2 <q, q> - rho_k, and the <r, r>
// partials of the new residual.
hipError_t launch_cg_update_fused(const Geom& g, c32* x, c32* r, c32* p, const c32* q, int k, const CgArgs& cg,
                                  hipStream_t st);
// The <r, r> partials the 3D update of iteration k reads (k == 0: the init
// kernel's) and writes.
const double* cg3_rr_in(const CgArgs& cg, int batch, int k);
double* cg3_rr_out(const CgArgs& cg, int batch, int k);

// Batched CG iteration over single-slice problems (serving engine): one
// group launch over the table rows (grid z = the largest G), then one
// combine launch (rows with G = 1 skip it).
void fill_ehe_cg_params(const Geom& g, const Tables& tb, const void* maps, const CgVectors& v, float lambda,
                        int k, const CgArgs& cg, EheParams* out);
// Whether the fused kernel stages this problem's maps tiles through LDS
// (a property of the problem alone).  Every row of a batched launch must
// give the same answer; the launch uses that code path for all of them.
bool ehe_staged(long ny, int maps_storage, long nx, const void* maps);
hipError_t launch_ehe_table(long ny, int maps_storage, bool staged, const EheParams* d_table, int nproblems,
                            int max_tiles, int max_groups, hipStream_t st);
hipError_t launch_combine_table(const EheParams* d_table, int nproblems, int max_tiles, int max_groups,
                                hipStream_t st);
// The same launches with up to kInlineProblems rows passed by value as the
// kernel argument (no host-to-device copy of the table).
constexpr int kInlineProblems = 16;
struct EheInline {
  EheParams p[kInlineProblems];
};
hipError_t launch_ehe_inline(long ny, int maps_storage, bool staged, const EheInline& table, int nproblems,
                             int max_tiles, int max_groups, hipStream_t st);
hipError_t launch_combine_inline(const EheInline& table, int nproblems, int max_tiles, int max_groups,
                                 hipStream_t st);
// Combine pass of one launch (plan path).
hipError_t launch_combine(const EheParams& P, int batch, bool cg, hipStream_t st);


// Whole CG solves of small 2D slices (nx <= 64, ny in {8, 16, 32, 48, 64},
// one coil group): one workgroup per batch element finishes b = E^H y from
// the x rows in work (launch_EH_rows: the column transforms and the
// conjugate coil sum, in the arithmetic of the E^H column pass), runs all K
// iterations and writes x, the CG state, the info and the rho history.
bool small_solve_supported(const Geom& g);
hipError_t launch_cg_small(const Geom& g, const Tables& tb, const void* maps, const c32* work, c32* x, int K,
                           float lambda, const CgArgs& cg, CgInfo* info, CgInfo* info2, hipStream_t st);

// The x rows of E^H: inverse readout transforms of the sampled k-space
// lines into work ([B][C][Nz][Ny][Nx] complex64; rows of unsampled lines are
// not written), unscaled.  adjoint_scale is the factor the column pass of
// E^H applies after its inverse transforms (unitary scale and centring sign
// of every axis).
hipError_t launch_EH_rows(const Geom& g, const Tables& tb, const void* y, c32* work, hipStream_t st);
float adjoint_scale(const Geom& g);

// Full-grid forward and adjoint operators (2D).
hipError_t launch_E(const Geom& g, const Tables& tb, const void* maps, const c32* x, c32* work,
                    void* y, hipStream_t st);
// E^H; with ngroups > 1 (2D) the coil sum of the column pass is split into
// groups whose partials go to part ([G][B][nvox] complex) and are combined.
hipError_t launch_EH(const Geom& g, const Tables& tb, const void* maps, const void* y, c32* work,
                     c32* x, c32* part, int ngroups, hipStream_t st);
// Root-sum-of-squares image of the (masked) k-space, real [B][nz][ny][nx];
// coil groups as for launch_EH (part holds [G][B][nvox] floats).
hipError_t launch_rss(const Geom& g, const Tables& tb, const void* y, c32* work, float* out, void* part,
                      int ngroups, hipStream_t st);
// Normal operator from column passes (3D): q = E^H E p + lambda p, with the
// readout transforms cancelled; fp64 partials of Re<p, q> and (zeta_part
// non-null) <q, q> per block of the last pass.
hipError_t launch_EHE_composed(const Geom& g, const Tables& tb, const void* maps, const c32* p, c32* q,
                               c32* work, float lambda, double* eta_part, double* zeta_part, hipStream_t st);
// Blocks of the last composed pass per batch element (partials count).
int adj_tiles(long nx, long ny, long nz);

}  // namespace sense
