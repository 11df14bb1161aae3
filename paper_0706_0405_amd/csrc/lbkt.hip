// HIP kernels and C ABI of the KT D2V9 finite-difference lattice Boltzmann step
// for gfx950 (MI355X). The ABI is declared and documented in include/lbkt.h.
//
// Kernel design: the step is a 5-point cross stencil over 9 SoA planes and is
// bound by HBM bandwidth (9 loads + 9 stores per site). Each thread owns one
// column x and marches up a chunk of `rows` rows, keeping the rows y-1, y, y+1
// of all 9 planes in registers, so every row is read from memory once per
// chunk; the x-neighbours come from the adjacent lanes (DPP shifts), the
// wavefront's two edge columns from halo fetches. The two-step pass (k_step2)
// applies two steps per pass over the array with the intermediate state in
// registers. Boundary ghosts are synthesised in registers. All kernels share
// one per-site arithmetic routine (kt_site.hpp), so every launch shape, one or
// two steps per pass and the batched path give bitwise identical results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbkt.h"
#include "kt_site.hpp"
#include "lbkt_internal.hpp"

using namespace lbkt;

// ------------------------------------------------------------------ error plumbing

static thread_local std::string g_last_error;

static lb_status fail(lb_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_CHECK(expr)                                                                 \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(LB_EHIP, std::string(#expr ": ") + hipGetErrorString(_e));            \
  } while (0)

// ------------------------------------------------------------------ host: constants

static int64_t plane_elems(const lb_grid* g) { return g->pitch * (int64_t)g->ny; }

extern "C" int64_t lb_array_elems(const lb_grid* g) {
  if (!g) return 0;
  return 9 * plane_elems(g);
}

extern "C" lb_status lb_default_lambda(lb_grid* g) {
  if (!g) return fail(LB_EINVAL, "grid is NULL");
  // Eq. (SEC-VON-13)
  g->lambda[0] = g->c1 * g->dx;
  for (int i = 1; i <= 4; ++i) g->lambda[i] = g->c1 * g->dx / 10.0;
  for (int i = 5; i <= 8; ++i) g->lambda[i] = 0.0;
  return LB_OK;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static lb_status validate_state(const lb_state& s, const char* what) {
  if (!finite_pos(s.rho) || !finite_pos(s.p) || !std::isfinite(s.ux) || !std::isfinite(s.uy))
    return fail(LB_EPARAM, std::string(what) + ": state needs rho > 0, p > 0, finite u");
  return LB_OK;
}

extern "C" lb_status lb_validate(const lb_grid* g) {
  if (!g) return fail(LB_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1) return fail(LB_EINVAL, "nx and ny must be >= 1");
  if (g->pitch < g->nx || g->pitch % 64 != 0)
    return fail(LB_EINVAL, "pitch must be >= nx and a multiple of 64");
  if (g->pitch > ((int64_t)1 << 27)) return fail(LB_EUNSUPPORTED, "pitch must be at most 2^27 elements");
  if (!finite_pos(g->dx) || !finite_pos(g->dt)) return fail(LB_EPARAM, "dx and dt must be > 0");
  if (!finite_pos(g->c1) || !finite_pos(g->c2) || !finite_pos(g->eta0))
    return fail(LB_EPARAM, "c1, c2, eta0 must be > 0");
  if (g->c1 == g->c2) return fail(LB_EPARAM, "c1 == c2 makes Eqs. (e17)-(e18) singular");
  if (!finite_pos(g->tau)) return fail(LB_EPARAM, "tau must be > 0");
  if (!(g->beta >= 0.0 && g->beta <= 0.5)) return fail(LB_EPARAM, "beta must lie in [0, 0.5]");
  if (!(std::isfinite(g->gamma) && g->gamma > 1.0)) return fail(LB_EPARAM, "gamma must be > 1");
  for (int i = 0; i < 9; ++i)
    if (!(std::isfinite(g->lambda[i]) && g->lambda[i] >= 0.0))
      return fail(LB_EPARAM, "lambda_i must be finite and >= 0");
  for (int i = 2; i <= 4; ++i)
    if (g->lambda[i] != g->lambda[1])
      return fail(LB_EUNSUPPORTED, "lambda_1..lambda_4 must be equal (one value per velocity group)");
  for (int i = 6; i <= 8; ++i)
    if (g->lambda[i] != g->lambda[5])
      return fail(LB_EUNSUPPORTED, "lambda_5..lambda_8 must be equal (one value per velocity group)");
  for (int e = 0; e < 4; ++e) {
    const lb_edge& E = g->edge[e];
    if (E.kind < LB_BC_PERIODIC || E.kind > LB_BC_SHOCK) return fail(LB_EPARAM, "unknown edge kind");
    if (E.kind == LB_BC_SHOCK && e < 2) return fail(LB_EPARAM, "a SHOCK edge must be a y edge");
    if (E.split < 0) return fail(LB_EPARAM, "split must be >= 0");
    if (E.kind == LB_BC_INFLOW || E.kind == LB_BC_SHOCK || E.split > 0) {
      lb_status s = validate_state(E.a, "edge state a");
      if (s) return s;
    }
    if (E.kind == LB_BC_SHOCK) {
      lb_status s = validate_state(E.b, "edge state b");
      if (s) return s;
      const double a = E.angle_deg * (M_PI / 180.0);
      if (!(std::isfinite(a) && std::sin(a) != 0.0 && std::tan(a) != 0.0) || !std::isfinite(E.x0) ||
          !std::isfinite(E.speed))
        return fail(LB_EPARAM, "bad shock geometry");
    }
  }
  const bool px = g->edge[0].kind == LB_BC_PERIODIC, px2 = g->edge[1].kind == LB_BC_PERIODIC;
  const bool py = g->edge[2].kind == LB_BC_PERIODIC, py2 = g->edge[3].kind == LB_BC_PERIODIC;
  if (px != px2 || py != py2) return fail(LB_EPARAM, "both edges of a periodic axis must be periodic");
  if ((px && g->edge[0].split) || (py && g->edge[2].split) || (px2 && g->edge[1].split) ||
      (py2 && g->edge[3].split))
    return fail(LB_EPARAM, "split is not allowed on a periodic edge");
  return LB_OK;
}

static void build_consts(const lb_grid* g, KTConsts* K) {
  std::memset(K, 0, sizeof(*K));
  K->nx = g->nx;
  K->ny = g->ny;
  K->pitch = g->pitch;
  K->plane = plane_elems(g);
  const double c1 = g->c1, c2 = g->c2, eta0 = g->eta0;
  const double b = 2.0 / (g->gamma - 1.0);
  K->c1 = c1;
  // c2 cos(pi/4) rounded once to double (extended-precision product on the host)
  K->s = (double)((long double)c2 * sqrtl(0.5L));
  K->eta0sq = eta0 * eta0;
  K->c1sq = c1 * c1;
  K->c2sq = c2 * c2;
  K->bval = b;
  K->inv_b = 1.0 / b;
  K->inv_tau = 1.0 / g->tau;
  const double c1s = c1 * c1, c2s = c2 * c2, e2 = eta0 * eta0;
  // Eq. (e17), A_0 read as (b-2) T / eta0^2
  K->a0T = (b - 2.0) / e2;
  K->k1u = c2s / c1s;
  K->k1T = (b - 2.0) * c2s / e2 + 2.0;
  K->k1d = 4.0 * (c1s - c2s);
  K->r1d = 1.0 / K->k1d;
  K->k5u = c1s / c2s;
  K->k5T = (b - 2.0) * c1s / e2 + 2.0;
  K->k5d = 4.0 * (c2s - c1s);
  K->r5d = 1.0 / K->k5d;
  // Eq. (e18)
  K->bT = b + 2.0;
  K->b1d = 2.0 * c1s * (c1s - c2s);
  K->rb1d = 1.0 / K->b1d;
  K->b5d = 2.0 * c2s * (c2s - c1s);
  K->rb5d = 1.0 / K->b5d;
  // partial derivatives of A and B (adjoint only)
  K->a1T = K->k1T / K->k1d;
  K->a1u = K->k1u / K->k1d;
  K->a5T = K->k5T / K->k5d;
  K->a5u = K->k5u / K->k5d;
  K->b1T = K->bT / K->b1d;
  K->b1u = 1.0 / K->b1d;
  K->b5T = K->bT / K->b5d;
  K->b5u = 1.0 / K->b5d;
  K->d1 = 1.0 / (2.0 * c1s * c1s);
  K->d5 = 1.0 / (2.0 * c2s * c2s);
  // Linear stencil: Eqs. (SEC-VON-2a/2b) for the convection, central second
  // difference for the dissipation, relaxation (f^eq - f)/tau; per velocity group.
  const double r = g->dt / g->dx, beta = g->beta;
  const double dx2 = g->dx * g->dx;
  const double l0 = g->dt * g->lambda[0] / dx2, la = g->dt * g->lambda[1] / dx2, ld = g->dt * g->lambda[5] / dx2;
  const double base = 1.0 - K->inv_tau;
  const double sd = K->s;
  K->l0 = l0;
  K->wc0 = base - 4.0 * l0;
  K->la = la;
  K->wca = (base - 4.0 * la) - r * c1 * (1.0 - 2.0 * beta);
  K->upa = la + r * c1 * (1.0 - beta);
  K->dna = la - r * c1 * beta;
  K->ld = ld;
  K->wcd = ((base - 4.0 * ld) - r * sd * (1.0 - 2.0 * beta)) - r * sd * (1.0 - 2.0 * beta);
  K->upd = ld + r * sd * (1.0 - beta);
  K->dnd = ld - r * sd * beta;
  for (int e = 0; e < 4; ++e) {
    const lb_edge& E = g->edge[e];
    K->kind[e] = E.kind;
    K->split[e] = E.split;
    const lb_state* st[2] = {&E.a, &E.b};
    double* dst[2] = {K->ga[e], K->gb[e]};
    for (int k = 0; k < 2; ++k) {
      const double rho = st[k]->rho, ux = st[k]->ux, uy = st[k]->uy;
      const double T = st[k]->p / rho;
      const double usq = fma(ux, ux, uy * uy);
      if (rho > 0.0) feq9(*K, rho, ux, uy, T, usq, dst[k]);
    }
  }
}

// Shared with the other translation units of the library (not part of the C ABI).
void lbkt_build_consts(const lb_grid* g, KTConsts* K) { build_consts(g, K); }
lb_status lbkt_fail(lb_status s, const std::string& msg) { return fail(s, msg); }

// Number of ghost cells behind a moving shock on edge e at time index `step`:
// ghost cell i is "behind" when (i + 0.5) dx < x0 + y/tan(angle) + speed t/sin(angle).
static int shock_cells(const lb_grid* g, int e, int64_t step) {
  const lb_edge& E = g->edge[e];
  if (E.kind != LB_BC_SHOCK) return 0;
  const double yg = (e == 2 ? -0.5 : g->ny + 0.5) * g->dx;
  const double ang = E.angle_deg * (M_PI / 180.0);
  const double t = (double)step * g->dt;
  const double xs = E.x0 + yg / std::tan(ang) + E.speed * t / std::sin(ang);
  const double q = xs / g->dx - 0.5;
  // !(q > 0) also catches a NaN position (an infinite shock geometry): no cell behind
  int n = !(q > 0.0) ? 0 : (q >= (double)g->nx ? g->nx : (int)std::ceil(q));
  // settle the boundary cell with the exact predicate
  while (n > 0 && !(((double)(n - 1) + 0.5) * g->dx < xs)) --n;
  while (n < g->nx && ((double)n + 0.5) * g->dx < xs) ++n;
  return n;
}

int lbkt_shock_cells(const lb_grid* g, int edge, int64_t step) { return shock_cells(g, edge, step); }

// ------------------------------------------------------------------ device: loads

// Distribution arrays are addressed through buffer resources: one 32-bit byte
// offset per lane (row and column) plus a per-plane scalar offset, so the 9
// planes share a single address register and out-of-range accesses cannot fault
// (they read 0 / are dropped by the hardware). That covers arrays below 4 GiB;
// larger ones get one resource per plane over the rows a tile touches (ViewG).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
#define LB_RSRC_WORD3 0x00020000
// cache policy of the distribution stores (default of the views): non-temporal
// (the next step reads them only after the whole array has streamed through
// the caches); the step kernels pick theirs per precision (see k_step, k_step2)
#ifndef LB_STORE_AUX
#define LB_STORE_AUX 2
#endif
// cache policy of the streamed row loads of the step kernels (0: default)
#ifndef LB_LOAD_AUX
#define LB_LOAD_AUX 0
#endif
// minimum waves per SIMD requested for the step kernels (0: compiler's choice)
#ifndef LB_STEP_WAVES
#define LB_STEP_WAVES 0
#endif
#if LB_STEP_WAVES > 0
#define LB_STEP_ATTR __attribute__((amdgpu_waves_per_eu(LB_STEP_WAVES)))
#else
#define LB_STEP_ATTR
#endif
// time steps per pass of lb_run on 4-row grids with a periodic y axis (even, 4-20;
// us per step on the paper's 1D configurations, rows on four wavefronts: 8 steps
// 1.07-1.33, 12 0.99-1.16, 16 0.94-1.15)
#ifndef LB_DEEP1
#define LB_DEEP1 16
#endif
// that pass with a strip's four rows on four wavefronts (1) or on one (0)
#ifndef LB_DEEP1_ROWS
#define LB_DEEP1_ROWS 1
#endif
// waves per SIMD asked of the float one-step kernel below 4 GiB (its 168 VGPRs fit 3)
#ifndef LB_STEP_F32_WAVES
#define LB_STEP_F32_WAVES 3
#endif

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, LB_RSRC_WORD3);
}

template <typename S> struct Mem;
template <> struct Mem<double> {
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vb, (int)sb, 0));
  }
  template <int AUX = LB_STORE_AUX>
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)vb, (int)sb, AUX);
  }
};
template <> struct Mem<float> {
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
    return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vb, (int)sb, 0));
  }
  template <int AUX = LB_STORE_AUX>
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb, double v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)v), r, (int)vb, (int)sb, AUX);
  }
};

template <typename S>
__device__ __forceinline__ S ld_raw(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb);

// Scalar offset of the next plane. RUN: a running sum that the compiler may not
// precompute (the empty asm makes it opaque), so that a row's nine plane offsets
// cost one SGPR and a scalar add each, instead of nine loop-invariant SGPRs that
// the register allocator spills to VGPR lanes and reloads with v_readlane in
// the march loops (VALU instructions).
template <bool RUN>
__device__ __forceinline__ uint32_t next_plane(uint32_t so, uint32_t planeB) {
  so += planeB;
  if constexpr (RUN) asm volatile("" : "+s"(so));
  return so;
}

// A distribution array below 4 GiB viewed through a buffer resource. Values are
// addressed by (plane i, row y, byte offset vb of the column in the row); the
// row and the column go into the lane's 32-bit offset, the plane into the
// scalar offset. AUX: the cache policy of the stores. RUN: plane offsets as an
// opaque running sum (next_plane); the default, for double storage, measured
// 1.4% faster for the FP64 one-step kernel, 0.5% for the two-step and 1-2% for
// the adjoint step on the 8192 x 2048 grid (float storage: more spill reloads
// in the two-step loop, so off; the batched kernels: 10% slower, off).
template <typename S, int AUX = LB_STORE_AUX, bool RUN = sizeof(S) == 8>
struct View {
  using Sto = S;
  __amdgpu_buffer_rsrc_t r;
  uint32_t rowB;    // bytes per row
  uint32_t planeB;  // bytes per plane
  __device__ __forceinline__ double ld(int i, int y, uint32_t vb) const {
    return Mem<S>::ld(r, (uint32_t)y * rowB + vb, (uint32_t)i * planeB);
  }
  __device__ __forceinline__ void load9(int y, uint32_t vb, double v[9]) const {
    const uint32_t o = (uint32_t)y * rowB + vb;
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = Mem<S>::ld(r, o, (uint32_t)i * planeB);
  }
  __device__ __forceinline__ void raw9(int y, uint32_t vb, S v[9]) const {
    const uint32_t o = (uint32_t)y * rowB + vb;
    uint32_t so = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      v[i] = ld_raw<S>(r, o, so);
      so = next_plane<RUN>(so, planeB);
    }
  }
  __device__ __forceinline__ void store9(int y, uint32_t vb, const double v[9]) const {
    const uint32_t o = (uint32_t)y * rowB + vb;
    uint32_t so = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      Mem<S>::template st<AUX>(r, o, so, v[i]);
      so = next_plane<RUN>(so, planeB);
    }
  }
  __device__ __forceinline__ void load9_any(int y, uint32_t vb, double v[9]) const { load9(y, vb, v); }
};

template <typename S, int AUX = LB_STORE_AUX, bool RUN = sizeof(S) == 8>
__device__ __forceinline__ View<S, AUX, RUN> make_view(const KTConsts& K, const void* p) {
  View<S, AUX, RUN> v;
  v.rowB = (uint32_t)(K.pitch * sizeof(S));
  v.planeB = (uint32_t)(K.plane * sizeof(S));
  v.r = make_rsrc(p, v.planeB * 9u);
  return v;
}

// A distribution array of 4 GiB or more, seen by one tile through a window of
// rows [ylo, yhi]: one buffer resource per plane covering the window's rows
// (below 4 GiB for any tile), with the interface of View. Rows outside the
// window (the periodic wrap of the ghost rows) are read through load9_any.
template <typename S>
struct ViewG {
  using Sto = S;
  __amdgpu_buffer_rsrc_t r[9];
  const char* base;
  uint64_t planeB;
  uint32_t rowB;
  int ylo;
  __device__ __forceinline__ uint32_t off(int y, uint32_t vb) const { return (uint32_t)(y - ylo) * rowB + vb; }
  __device__ __forceinline__ double ld(int i, int y, uint32_t vb) const { return Mem<S>::ld(r[i], off(y, vb), 0); }
  __device__ __forceinline__ void load9(int y, uint32_t vb, double v[9]) const {
    const uint32_t o = off(y, vb);
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = Mem<S>::ld(r[i], o, 0);
  }
  __device__ __forceinline__ void raw9(int y, uint32_t vb, S v[9]) const {
    const uint32_t o = off(y, vb);
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = ld_raw<S>(r[i], o, 0);
  }
  __device__ __forceinline__ void store9(int y, uint32_t vb, const double v[9]) const {
    const uint32_t o = off(y, vb);
#pragma unroll
    for (int i = 0; i < 9; ++i) Mem<S>::st(r[i], o, 0, v[i]);
  }
  // any row 0 <= y < ny, inside the window or not (resources made for the row)
  __device__ __forceinline__ void load9_any(int y, uint32_t vb, double v[9]) const {
#pragma unroll
    for (int i = 0; i < 9; ++i)
      v[i] = Mem<S>::ld(make_rsrc(base + i * planeB + (uint64_t)(uint32_t)y * rowB, rowB), vb, 0);
  }
};

// The window of rows [ylo, yhi], clamped into the grid.
template <typename S>
__device__ __forceinline__ ViewG<S> make_view_g_rows(const KTConsts& K, const void* p, int ylo, int yhi) {
  ViewG<S> v;
  v.base = (const char*)p;
  v.rowB = (uint32_t)(K.pitch * sizeof(S));
  v.planeB = (uint64_t)K.plane * sizeof(S);
  v.ylo = max(ylo, 0);
  yhi = min(yhi, K.ny - 1);
  const uint32_t bytes = (uint32_t)(yhi - v.ylo + 1) * v.rowB;
  const char* w = v.base + (uint64_t)(uint32_t)v.ylo * v.rowB;
#pragma unroll
  for (int i = 0; i < 9; ++i) v.r[i] = make_rsrc(w + i * v.planeB, bytes);
  return v;
}

// The window a one-step tile of rows [y0, y1) reads: rows y0-1 .. y1.
template <typename S>
__device__ __forceinline__ ViewG<S> make_view_g(const KTConsts& K, const void* p, int y0, int y1) {
  return make_view_g_rows<S>(K, p, y0 - 1, y1);
}

template <class V>
using Sto = typename V::Sto;

// v held in scalar registers: a grid constant read this way is loaded by a
// scalar load and then chosen per lane, instead of the compiler choosing its
// address per lane and reading it with vector loads (a form that gave wrong edge
// ghosts inside the three-step kernel).
__device__ __forceinline__ double uni(double v) {
  asm volatile("" : "+s"(v));
  return v;
}

// Ghost row of y edge E (2: below row 0, 3: above row ny-1) at column x
// (vbx = x * sizeof(S)). Edge indices are compile-time constants so no per-lane
// indexing of K occurs.
template <int E, class V, bool UNI = false>
__device__ __forceinline__ void ghost_row(const KTConsts& K, const V& f, int x, uint32_t vbx, int ish,
                                          double r[9]) {
  const int kind = K.kind[E];
  if (kind == BC_PERIODIC || kind == BC_OUTFLOW || kind == BC_WALL) {
    int src;
    if (kind == BC_PERIODIC)
      src = (E == 2) ? K.ny - 1 : 0;
    else
      src = (E == 2) ? 0 : K.ny - 1;
    double t[9];
    f.load9_any(src, vbx, t);
    if (kind == BC_WALL) {
#pragma unroll
      for (int i = 0; i < 9; ++i) r[i] = t[mirror_y(i)];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) r[i] = t[i];
    }
  } else {
    const bool a = (kind == BC_INFLOW) || (x < ish);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if constexpr (UNI)
        r[i] = a ? uni(K.ga[E][i]) : uni(K.gb[E][i]);
      else
        r[i] = a ? K.ga[E][i] : K.gb[E][i];
    }
  }
  if (x < K.split[E]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = UNI ? uni(K.ga[E][i]) : K.ga[E][i];
  }
}

// Raw storage-typed loads (no widening) for rows held in flight.
template <>
__device__ __forceinline__ double ld_raw<double>(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vb, (int)sb, LB_LOAD_AUX));
}
template <>
__device__ __forceinline__ float ld_raw<float>(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vb, (int)sb, LB_LOAD_AUX));
}

// Wavefront lane shifts (DPP wave_shr:1 / wave_shl:1): lane i receives lane
// i-1 (shr) or i+1 (shl); the lane without a source (0, resp. 63) keeps `old`.
__device__ __forceinline__ int dpp_shr1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_shl1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ double shr1(double old, double v) {
  const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
  const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_shr1((int)(unsigned)o, (int)(unsigned)w);
  const unsigned hi = (unsigned)dpp_shr1((int)(unsigned)(o >> 32), (int)(unsigned)(w >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double shl1(double old, double v) {
  const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
  const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_shl1((int)(unsigned)o, (int)(unsigned)w);
  const unsigned hi = (unsigned)dpp_shl1((int)(unsigned)(o >> 32), (int)(unsigned)(w >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The same shifts where the lane without a source (0, resp. 63) may receive 0:
// no old value to carry, so no copy of it before the shift.
__device__ __forceinline__ double shr1z(double v) {
  const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)w, 0x138, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(w >> 32), 0x138, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double shl1z(double v) {
  const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)w, 0x130, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(w >> 32), 0x130, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Column geometry of one lane: its column x inside a wavefront that covers the
// 64 columns [xw0, xw0 + 64); lanes 0 and 63 also fetch the halo columns hl, hr.
struct Lane {
  int x, lane;
  uint32_t vbx;    // x * sizeof(S): own column (clamped into the row for x >= nx)
  uint32_t vbh;    // halo column of lanes 0 / 63
  bool halo;       // lane 0 or 63
};

template <typename S>
__device__ __forceinline__ Lane make_lane(const KTConsts& K, int xw0, int lane) {
  Lane L;
  L.lane = lane;
  L.x = xw0 + lane;
  const int nx = K.nx;
  const bool perx = (K.kind[0] == BC_PERIODIC);
  const int hl = (xw0 > 0) ? xw0 - 1 : (perx ? nx - 1 : 0);
  const int hr = (xw0 + 64 < nx) ? xw0 + 64 : (perx ? 0 : nx - 1);
  L.vbx = (uint32_t)L.x * sizeof(S);   // x < pitch always: pitch is a multiple of 64
  L.vbh = (uint32_t)(lane == 0 ? hl : hr) * sizeof(S);
  L.halo = (lane == 0) || (lane == 63);
  return L;
}

// Ghost of x edge E for site (x, y) where the shifted neighbour is not the ghost.
template <int E, class V>
__device__ __forceinline__ void ghost_x(const KTConsts& K, const V& f, int y, const double cur[9],
                                        double g[9]) {
  const int kind = K.kind[E];
  if (kind == BC_WALL) {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = cur[mirror_x(i)];
  } else if (kind == BC_INFLOW) {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = K.ga[E][i];
  } else if (kind == BC_OUTFLOW) {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = cur[i];
  } else {  // periodic: the opposite column
    const int src = (E == 0) ? K.nx - 1 : 0;
    f.load9(y, (uint32_t)src * sizeof(Sto<V>), g);
  }
  if (y < K.split[E]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = K.ga[E][i];
  }
}

// Widening of a fetched value at its point of use. For float storage the
// conversion is written as one asm instruction so that it stays there: as a
// plain cast the compiler moves it across the loop's phis to just behind the
// fetch, and waits there for the fetch (and for every store issued before it)
// instead of a row later. v_cvt_f64_f32 is exact, as the cast is.
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) {
  double d;
  asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(d) : "v"(v));
  return d;
}

// Site update of row y for one lane: prev/cur/nxt are the rows y-1, y, y+1 at
// the lane's column, hc the halo values of row y (lanes 0 and 63).
template <bool XEDGE, class V>
__device__ __forceinline__ void row_update(const KTConsts& K, const V& fi, const V& fo, const Lane& L, int y,
                                           const double prev[9], const double cur[9], const double nxt[9],
                                           const Sto<V> hc[9]) {
  double xm[9], xp[9], out[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double h = widen(hc[i]);
    xm[i] = shr1(h, cur[i]);
    xp[i] = shl1(h, cur[i]);
  }
  if (XEDGE) {
    if (L.x == 0) ghost_x<0>(K, fi, y, cur, xm);
    if (L.x == K.nx - 1) ghost_x<1>(K, fi, y, cur, xp);
  }
  site_update<sizeof(Sto<V>) == 4>(K, cur, xp, xm, nxt, prev, out);
  // Lanes past nx store too, into the row's padding columns (x < pitch): no
  // result reads them, and an unmasked store keeps the compiler's wait counts
  // from having to cover a path on which the stores were skipped.
  fo.store9(y, L.vbx, out);
}

// One row y < ny-1 of the march: issue the fetches of row y+2 (into F) and of
// the halo of row y+1 (into HN), widen row y+1 (N, fetched one row earlier),
// update row y, and shift pd <- cd <- row y+1. Both fetches are issued by every
// lane on every row, the row clamped into the chunk (a clamped fetch repeats
// one already made and is served from cache): fetches that are always issued
// let the compiler count them exactly instead of waiting for them early.
template <bool XEDGE, class V>
__device__ __forceinline__ void march_row(const KTConsts& K, const V& fi, const V& fo, const Lane& L, int y,
                                          int y1, int ylast, double pd[9], double cd[9], const Sto<V> N[9],
                                          const Sto<V> HC[9], Sto<V> F[9], Sto<V> HN[9]) {
  fi.raw9(min(y + 2, ylast), L.vbx, F);
  fi.raw9(min(y + 1, y1 - 1), L.vbh, HN);
  double nd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) nd[i] = widen(N[i]);
  row_update<XEDGE>(K, fi, fo, L, y, pd, cd, nd, HC);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = nd[i];
  }
  __builtin_amdgcn_sched_barrier(0);   // keep the two unrolled rows apart (register pressure)
}

// Row y = ny-1, whose upper neighbour is the ghost row of the top edge.
template <bool XEDGE, class V>
__device__ __forceinline__ void top_row(const KTConsts& K, const V& fi, const V& fo, const Lane& L, int y,
                                        int ish_hi, const double pd[9], const double cd[9], const Sto<V> HC[9]) {
  double nd[9];
  ghost_row<3>(K, fi, L.x, L.vbx, ish_hi, nd);
  row_update<XEDGE>(K, fi, fo, L, y, pd, cd, nd, HC);
}

// March a 64-column wavefront strip from row y0 to y1-1. Rows are fetched two
// rows ahead of the row being updated (so a full iteration of arithmetic hides
// each fetch), the halo columns one row ahead; x-neighbours come from the
// adjacent lanes through DPP shifts, and only lanes 0 and 63 use the two halo
// columns. The loop is unrolled by two with two sets of in-flight registers
// (N0/N1, H0/H1) that swap roles each row, so no value still in flight is ever
// copied and a row waits only for its own fetches, never for the stores or the
// fetches issued after them. The top row of the grid (upper neighbour = ghost)
// is updated after the loop, keeping the ghost's loads and branches out of it.
// Every lane runs the whole march (the DPP shifts need all lanes); lanes beyond
// nx compute on padding values and store into the padding.
template <bool XEDGE, class V>
__device__ __forceinline__ void march(const KTConsts& K, const V& fi, const V& fo, const Lane& L, int y0, int y1,
                                      int ish_lo, int ish_hi) {
  using S = Sto<V>;
  const int ny = K.ny;
  double pd[9], cd[9];
  S N0[9], N1[9], H0[9], H1[9];
  // prologue: row y0-1 (or the bottom ghost), row y0 and its halo, row y0+1
  if (y0 > 0)
    fi.load9(y0 - 1, L.vbx, pd);
  else
    ghost_row<2>(K, fi, L.x, L.vbx, ish_lo, pd);
  fi.load9(y0, L.vbx, cd);
  fi.raw9(y0, L.vbh, H0);
  fi.raw9(min(y0 + 1, ny - 1), L.vbx, N0);
  // Float storage: let the prologue's fetches land before the loop, so that the
  // loop header sees only the previous iteration's fetches in flight and the
  // compiler's wait counts there need not cover the prologue's loads on the
  // entry edge (which otherwise drain every fetch and store each iteration).
  // Double storage schedules well without it and keeps more registers.
  if constexpr (sizeof(S) == 4) {
#pragma unroll
    for (int i = 0; i < 9; ++i) asm volatile("" ::"v"(pd[i]), "v"(cd[i]), "v"(N0[i]), "v"(H0[i]));
  }
  // Rows below ylast have a real upper neighbour; ylast is also the last row
  // fetched (the upper neighbour of row y1-1, unless that is the ghost).
  const int ylast = min(y1, ny - 1);
  int y = y0;
  for (; y + 1 < ylast; y += 2) {
    march_row<XEDGE>(K, fi, fo, L, y, y1, ylast, pd, cd, N0, H0, N1, H1);
    march_row<XEDGE>(K, fi, fo, L, y + 1, y1, ylast, pd, cd, N1, H1, N0, H0);
  }
  // (the halo set of the next row is picked by branch, not by pointer, so the
  // arrays stay in registers)
  if (y < ylast) {
    march_row<XEDGE>(K, fi, fo, L, y, y1, ylast, pd, cd, N0, H0, N1, H1);
    if (y + 1 < y1) top_row<XEDGE>(K, fi, fo, L, y + 1, ish_hi, pd, cd, H1);
  } else if (y < y1) {
    top_row<XEDGE>(K, fi, fo, L, y, ish_hi, pd, cd, H0);
  }
}

// The grid constants of a kernel whose first argument is its KTConsts (offset 0
// of the kernel-argument segment), re-read through a pointer that the compiler
// cannot see through. Loads through it stay scalar and invariant (constant
// address space), so the register allocator re-issues them (s_load) where the
// march loops run short of SGPRs, instead of spilling the ~70 SGPRs of constants
// to VGPR lanes and reloading them with v_readlane, which are VALU instructions
// (float-storage two-step loop: 1308 instead of 1479 VALU instructions per
// three rows).
__device__ __forceinline__ const KTConsts& kernarg_consts() {
  auto kp = (const __attribute__((address_space(4))) KTConsts*)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(kp));
  return *(const KTConsts*)kp;
}

// Block index -> (strip, chunk). With xcd_map, the blocks that the hardware
// deals round-robin to one XCD (ids congruent mod 8) get one contiguous band of
// the (chunk, strip) raster, so x- and y-adjacent tiles share that XCD's L2.
__device__ __forceinline__ void tile_of_block(int id, int nstrips, int nblocks, int xcd_map, int* strip,
                                              int* chunk) {
  int lin = id;
  if (xcd_map) {
    const int per = nblocks >> 3;
    lin = (id & 7) * per + (id >> 3);
  }
  *strip = lin % nstrips;
  *chunk = lin / nstrips;
}

// Blocks loop over tile ids id = blockIdx.x, blockIdx.x + gridDim.x, ... (one
// tile per block when gridDim.x equals the tile count). gridDim.x is a multiple
// of 8 whenever xcd_map is set, so every tile of a block stays in its XCD's band.
// WIDE: arrays of 4 GiB and more, addressed through ViewG (64-bit addresses).
template <typename S, bool WIDE>
__global__ __launch_bounds__(256) LB_STEP_ATTR
    __attribute__((amdgpu_waves_per_eu(sizeof(S) == 4 && !WIDE ? LB_STEP_F32_WAVES : 1))) void k_step(KTConsts K,
                                                                                           const S* __restrict__ fin,
                                                           S* __restrict__ fout, int rows, int nstrips, int ntiles,
                                                           int xcd_map, int ish_lo, int ish_hi) {
  const View<S> fi0 = make_view<S>(K, fin), fo0 = make_view<S>(K, fout);
  const int lane = threadIdx.x & 63;
  for (int id = blockIdx.x; id < ntiles; id += gridDim.x) {
    int strip, chunk;
    tile_of_block(id, nstrips, ntiles, xcd_map, &strip, &chunk);
    const int xw0 = strip * blockDim.x + (threadIdx.x & ~63);
    if (xw0 >= K.nx) continue;   // whole wavefront beyond the grid
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, K.ny);
    const Lane L = make_lane<S>(K, xw0, lane);
    const KTConsts& KM = kernarg_consts();   // K itself, for the march loops
    if constexpr (WIDE) {
      const ViewG<S> fi = make_view_g<S>(K, fin, y0, y1), fo = make_view_g<S>(K, fout, y0, y1);
      if (xw0 == 0 || xw0 + 64 >= K.nx)
        march<true>(KM, fi, fo, L, y0, y1, ish_lo, ish_hi);
      else
        march<false>(KM, fi, fo, L, y0, y1, ish_lo, ish_hi);
    } else {
      if (xw0 == 0 || xw0 + 64 >= K.nx)
        march<true>(KM, fi0, fo0, L, y0, y1, ish_lo, ish_hi);
      else
        march<false>(KM, fi0, fo0, L, y0, y1, ish_lo, ish_hi);
    }
  }
}

// ------------------------------------------------------------------ two steps per pass

// Two consecutive steps in one pass over the array (temporal blocking): a
// wavefront marches its rows as in the one-step march, keeps the state after
// the first step (f1) of rows y-1, y, y+1 in registers instead of storing it,
// and updates the second step of row y from them. HBM moves the 9 + 9 values
// of a site once per two steps. f1 is rounded to the storage type exactly as a
// stored step would be, and every ghost of f1 is formed as the one-step march
// forms it from the stored f1, so the result is bitwise that of two single
// steps.
//
// Columns: lane j of a wavefront holds column c = X0 - 2 + j. Lanes 1..62 compute
// f1 (their x-neighbours are lanes), lanes 2..61 (of columns inside the grid)
// the second step, so wavefronts start every 60 columns and overlap by four;
// lanes 0 and 63 only supply f0 to their neighbours, and no halo columns are
// fetched. With a periodic x axis a lane's column wraps into the grid (lane c =
// -1 holds column nx-1, the wrapped neighbour itself); otherwise the x ghosts of
// both steps are formed at columns 0 and nx-1 as in the one-step march. Rows:
// the tile of output rows [y0, y1) computes f1 on rows y0-1 .. y1 (one extra row
// each side) from f0 rows y0-2 .. y1+1; the y ghosts of f1 outside the grid come
// from f1 rows 0 / ny-1 (outflow, wall), from constants at the second step's
// time (inflow, shock), or for a periodic y axis from f1 computed on the far row.
struct Lane2 {
  int x;           // column c (may lie outside the grid: then only a neighbour)
  int xs;          // the grid column whose values the lane holds (c wrapped or clamped)
  uint32_t vbx;    // xs * sizeof(S)
  uint32_t vbo;    // c * sizeof(S) for the output lanes
  bool out;        // lane produces the second step of its column
  bool perx;
};

__device__ __forceinline__ int wrap_col(int c, int nx, bool perx) {
  return perx ? ((c % nx) + nx) % nx : min(max(c, 0), nx - 1);
}

// d: steps per pass (lane j holds column X0 - d + j; lanes d .. 63-d produce the
// last step, the march of two steps per pass has d = 2).
template <typename S>
__device__ __forceinline__ Lane2 make_lane2(const KTConsts& K, int X0, int lane, int d = 2) {
  Lane2 L;
  const int nx = K.nx;
  L.perx = (K.kind[0] == BC_PERIODIC);
  L.x = X0 - d + lane;
  L.xs = wrap_col(L.x, nx, L.perx);
  L.vbx = (uint32_t)L.xs * sizeof(S);
  L.out = (lane >= d) && (lane <= 63 - d) && (L.x < nx);
  L.vbo = L.out ? (uint32_t)L.x * sizeof(S) : 0u;
  return L;
}

// The x ghosts of a row for the lanes at a non-periodic x edge, as ghost_x forms
// them (x edges are walls, inflow or outflow here, periodic ones are handled by
// the lanes' wrapped columns), written as selects instead of branches: the lane
// holding column 0 takes its x-1 neighbour xm from the edge, the lane holding
// column nx-1 its x+1 neighbour xp.
template <bool UNI = false>
__device__ __forceinline__ void ghost_x_select(const KTConsts& K, const Lane2& L, int y, const double cur[9],
                                               double xm[9], double xp[9]) {
  // the edge's kind and split are read first and combined without short-circuit
  // evaluation, so no per-lane branch guards the reads
  const int k0 = K.kind[0], k1 = K.kind[1], s0 = K.split[0], s1 = K.split[1];
  const bool l = (L.x == 0), r = (L.x == K.nx - 1);
  const bool c0 = (k0 == BC_INFLOW) | (y < s0), c1 = (k1 == BC_INFLOW) | (y < s1);
  const bool lc = l & c0, lm = l & !c0 & (k0 == BC_WALL), lo = l & !c0 & (k0 == BC_OUTFLOW);
  const bool rc = r & c1, rm = r & !c1 & (k1 == BC_WALL), ro = r & !c1 & (k1 == BC_OUTFLOW);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if constexpr (UNI) {
      xm[i] = lc ? uni(K.ga[0][i]) : lm ? cur[mirror_x(i)] : lo ? cur[i] : xm[i];
      xp[i] = rc ? uni(K.ga[1][i]) : rm ? cur[mirror_x(i)] : ro ? cur[i] : xp[i];
    } else {
      xm[i] = lc ? K.ga[0][i] : lm ? cur[mirror_x(i)] : lo ? cur[i] : xm[i];
      xp[i] = rc ? K.ga[1][i] : rm ? cur[mirror_x(i)] : ro ? cur[i] : xp[i];
    }
  }
}

// f1 of row y at the lane's column from f0 rows y-1, y, y+1 (prev, cur, nxt),
// rounded to the storage type (lanes 0 and 63: not meaningful, never used).
// SEL: the x ghosts as selects (ghost_x_select) instead of per-lane branches.
template <bool XEDGE, class V, bool SEL = false>
__device__ __forceinline__ void row_first(const KTConsts& K, const V& fi, const Lane2& L, int y,
                                          const double prev[9], const double cur[9], const double nxt[9],
                                          double t[9]) {
  double xm[9], xp[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    xm[i] = shr1z(cur[i]);   // lanes 0 and 63 get 0: their results are never used
    xp[i] = shl1z(cur[i]);
  }
  if (XEDGE && !L.perx) {   // ghost_x reads no memory for non-periodic edges
    if constexpr (SEL) {
      ghost_x_select<true>(K, L, y, cur, xm, xp);
    } else {
      if (L.x == 0) ghost_x<0>(K, fi, y, cur, xm);
      if (L.x == K.nx - 1) ghost_x<1>(K, fi, y, cur, xp);
    }
  }
  site_update<sizeof(Sto<V>) == 4>(K, cur, xp, xm, nxt, prev, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) t[i] = (double)(Sto<V>)t[i];
}

// The second step of row y from f1 rows y-1, y, y+1 (held in the storage type,
// or in double where a ghost row holds unrounded constants), stored by the
// output lanes.
template <bool XEDGE, class V, typename A, typename B, typename C, bool SEL = false>
__device__ __forceinline__ void row_second(const KTConsts& K, const V& fo, const Lane2& L, int y, const A p1[9],
                                           const B c1[9], const C n1[9]) {
  double prev[9], cur[9], nxt[9], xm[9], xp[9], out[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {   // values in registers: plain (exact) conversions
    prev[i] = (double)p1[i];
    cur[i] = (double)c1[i];
    nxt[i] = (double)n1[i];
    xm[i] = shr1z(cur[i]);   // lanes 0 and 63 get 0: their results are never used
    xp[i] = shl1z(cur[i]);
  }
  if (XEDGE && !L.perx) {
    if constexpr (SEL) {
      ghost_x_select<true>(K, L, y, cur, xm, xp);
    } else {
      if (L.x == 0) ghost_x<0>(K, fo, y, cur, xm);
      if (L.x == K.nx - 1) ghost_x<1>(K, fo, y, cur, xp);
    }
  }
  site_update<sizeof(Sto<V>) == 4>(K, cur, xp, xm, nxt, prev, out);
  if (L.out) fo.store9(y, L.vbo, out);
}

// y ghost row of f1 on edge E (2: below row 0, 3: above row ny-1) for a
// non-periodic edge, from the f1 row next to it (as ghost_row forms it from the
// stored f1 at the second step's time). x is the grid column the lane holds.
template <int E, typename Q, bool UNI = false>
__device__ __forceinline__ void ghost_row_f1(const KTConsts& K, int x, int ish, const Q src[9], double r[9]) {
  const int kind = K.kind[E];
  if (kind == BC_OUTFLOW) {
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = (double)src[i];
  } else if (kind == BC_WALL) {
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = (double)src[mirror_y(i)];
  } else {
    const bool a = (kind == BC_INFLOW) || (x < ish);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if constexpr (UNI)
        r[i] = a ? uni(K.ga[E][i]) : uni(K.gb[E][i]);
      else
        r[i] = a ? K.ga[E][i] : K.gb[E][i];
    }
  }
  if (x < K.split[E]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = UNI ? uni(K.ga[E][i]) : K.ga[E][i];
  }
}

// f1 of row q of a y-periodic grid, loaded and computed on its own (the far
// neighbour row of the bottom and top tiles).
template <bool XEDGE, class V>
__device__ __forceinline__ void f1_row_periodic(const KTConsts& K, const V& fi, const Lane2& L, int q, double t[9]) {
  const int ny = K.ny;
  double pd[9], cd[9], nd[9];
  fi.load9_any(q == 0 ? ny - 1 : q - 1, L.vbx, pd);
  fi.load9_any(q, L.vbx, cd);
  fi.load9_any(q == ny - 1 ? 0 : q + 1, L.vbx, nd);
  row_first<XEDGE>(K, fi, L, q, pd, cd, nd, t);
}

// Where the intermediate state f1 goes: NoRec drops it (lb_run); Rec stores the
// f1 rows [y0, y1) of the tile through its view (lb_run_record, which keeps
// every state). f1 is already rounded to the storage type, so the stored state
// is bitwise that of a single step.
struct NoRec {
  __device__ __forceinline__ void put(int, const Lane2&, const double*) const {}
};
template <class V>
struct Rec {
  V v;
  int y0, y1;
  __device__ __forceinline__ void put(int y, const Lane2& L, const double t[9]) const {
    if (y >= y0 && y < y1 && L.out) v.store9(y, L.vbo, t);
  }
};

// One row of the two-step march: issue the fetch of f0 row y+3 (F), compute f1
// of row y (N: f0 row y+1, fetched two rows earlier), then the second step of
// row y-1 from f1 rows y-2, y-1 (q0, q1) and y; shift the windows.
template <bool XEDGE, class V, class R>
__device__ __forceinline__ void march2_row(const KTConsts& K, const V& fi, const V& fo, const Lane2& L, int y,
                                           int ylast, double pd[9], double cd[9], Sto<V> q0[9], Sto<V> q1[9],
                                           const Sto<V> N[9], Sto<V> F[9], const R& rec) {
  fi.raw9(min(y + 3, ylast), L.vbx, F);
  double nd[9], t[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) nd[i] = widen(N[i]);
  row_first<XEDGE>(K, fi, L, y, pd, cd, nd, t);
  rec.put(y, L, t);
  __builtin_amdgcn_sched_barrier(0);   // the two updates one after the other (register pressure)
  row_second<XEDGE>(K, fo, L, y - 1, q0, q1, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = nd[i];
    q0[i] = q1[i];
    q1[i] = (Sto<V>)t[i];   // exact: t is already rounded to the storage type
  }
  __builtin_amdgcn_sched_barrier(0);
}

// March a 60-column output strip over output rows [y0, y1) (two steps; ny >= 2).
// f1 rows ya .. yb are computed in order, from f0 rows ya-1 .. min(yb+1, ny-1)
// fetched as in the one-step march (ghost rows at the first step's time outside
// the grid); after f1 row y the second step of row y-1 follows. Rows ya and
// ya+1 prime the f1 window (yb >= ya+1 always holds), after which the register
// sets are in the same state for every tile.
template <bool XEDGE, class V, class R>
__device__ __forceinline__ void march2(const KTConsts& K, const V& fi, const V& fo, const Lane2& L, int y0, int y1,
                                       int ish_lo, int ish_hi, int ish2_lo, int ish2_hi, const R& rec) {
  using S = Sto<V>;
  const int ny = K.ny;
  const bool pery = (K.kind[2] == BC_PERIODIC);
  const int ya = max(y0 - 1, 0), yb = min(y1, ny - 1);
  const int ylast = min(yb + 1, ny - 1);
  double pd[9], cd[9], nd[9], t[9];
  S N0[9], N1[9], N2[9], q0[9], q1[9];   // f0 rows in flight (three sets); f1 rows y-2, y-1
  if (ya > 0)
    fi.load9(ya - 1, L.vbx, pd);
  else
    ghost_row<2>(K, fi, L.xs, L.vbx, ish_lo, pd);
  fi.load9(ya, L.vbx, cd);
  fi.raw9(ya + 1, L.vbx, N0);
  fi.raw9(min(ya + 2, ylast), L.vbx, N1);
  // f1 row ya (its upper f0 neighbour ya+1 <= yb lies in the grid)
  fi.raw9(min(ya + 3, ylast), L.vbx, N2);
#pragma unroll
  for (int i = 0; i < 9; ++i) nd[i] = widen(N0[i]);
  row_first<XEDGE>(K, fi, L, ya, pd, cd, nd, t);
  rec.put(ya, L, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    q0[i] = (S)t[i];
    pd[i] = cd[i];
    cd[i] = nd[i];
  }
  // f1 row ya+1 (upper f0 neighbour: the top ghost when ya+1 = ny-1)
  fi.raw9(min(ya + 4, ylast), L.vbx, N0);
  if (ya + 1 < ny - 1) {
#pragma unroll
    for (int i = 0; i < 9; ++i) nd[i] = widen(N1[i]);
  } else {
    ghost_row<3>(K, fi, L.xs, L.vbx, ish_hi, nd);
  }
  row_first<XEDGE>(K, fi, L, ya + 1, pd, cd, nd, t);
  rec.put(ya + 1, L, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    q1[i] = (S)t[i];
    pd[i] = cd[i];
    cd[i] = nd[i];
  }
  if (y0 == 0) {   // second step of row 0: f1 rows -1 (ghost), 0, 1
    double g[9];
    if (pery)
      f1_row_periodic<XEDGE>(K, fi, L, ny - 1, g);
    else
      ghost_row_f1<2>(K, L.xs, ish2_lo, q0, g);
    row_second<XEDGE>(K, fo, L, 0, g, q0, q1);
  }
  // f1 rows y-2, y-1 in q0, q1; f0 rows y-1, y in pd, cd; in flight: f0 rows
  // min(y+1, ylast) in N2 and min(y+2, ylast) in N0; N1 free. The sets rotate
  // with period three (the loop is unrolled by three).
  int y = ya + 2;
  for (; y + 2 < ylast; y += 3) {
    march2_row<XEDGE>(K, fi, fo, L, y, ylast, pd, cd, q0, q1, N2, N1, rec);
    march2_row<XEDGE>(K, fi, fo, L, y + 1, ylast, pd, cd, q0, q1, N0, N2, rec);
    march2_row<XEDGE>(K, fi, fo, L, y + 2, ylast, pd, cd, q0, q1, N1, N0, rec);
  }
  if (y < ylast) {
    march2_row<XEDGE>(K, fi, fo, L, y, ylast, pd, cd, q0, q1, N2, N1, rec);
    y += 1;
    if (y < ylast) {
      march2_row<XEDGE>(K, fi, fo, L, y, ylast, pd, cd, q0, q1, N0, N2, rec);
      y += 1;
    }
  }
  if (y <= yb) {   // y = ny-1: the upper f0 neighbour is the top ghost
    ghost_row<3>(K, fi, L.xs, L.vbx, ish_hi, nd);
    row_first<XEDGE>(K, fi, L, y, pd, cd, nd, t);
    rec.put(y, L, t);
    row_second<XEDGE>(K, fo, L, y - 1, q0, q1, t);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      q0[i] = q1[i];
      q1[i] = (S)t[i];
    }
  }
  if (y1 == ny) {   // second step of row ny-1: f1 rows ny-2, ny-1, ny (ghost)
    double g[9];
    if (pery)
      f1_row_periodic<XEDGE>(K, fi, L, 0, g);
    else
      ghost_row_f1<3>(K, L.xs, ish2_hi, q1, g);
    row_second<XEDGE>(K, fo, L, ny - 1, q0, q1, g);
  }
}

// REC: also store the intermediate state f1 to f1out (lb_run_record; arrays
// below 4 GiB only).
template <typename S, bool WIDE, bool REC = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_step2(
    KTConsts K, const S* __restrict__ fin, S* __restrict__ fout, S* __restrict__ f1out, int rows, int nstrips,
    int ntiles, int xcd_map, int ish_lo, int ish_hi, int ish2_lo, int ish2_hi) {
  static_assert(!(WIDE && REC), "recording runs on arrays below 4 GiB");
  // stores: non-temporal for double, ordinary for float storage (8192 x 2048
  // grid, ms per step: float 0.164 vs 0.168-0.174 with non-temporal stores, on
  // two devices; double 0.2650 vs 0.2697 with ordinary stores, three runs each)
  constexpr int AUX = sizeof(S) == 8 ? 2 : 0;
  const View<S, AUX> fi0 = make_view<S, AUX>(K, fin), fo0 = make_view<S, AUX>(K, fout);
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  for (int id = blockIdx.x; id < ntiles; id += gridDim.x) {
    int strip, chunk;
    tile_of_block(id, nstrips, ntiles, xcd_map, &strip, &chunk);
    const int X0 = (strip * wpb + (threadIdx.x >> 6)) * 60;
    if (X0 >= K.nx) continue;   // whole wavefront beyond the grid
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, K.ny);
    const Lane2 L = make_lane2<S>(K, X0, lane);
    // the lanes hold columns X0-2 .. X0+61: x-edge logic when 0 or nx-1 is among them
    const bool edge = (X0 == 0) || (X0 + 62 >= K.nx);
    if constexpr (WIDE) {
      const ViewG<S> fi = make_view_g_rows<S>(K, fin, y0 - 2, y1 + 1);
      const ViewG<S> fo = make_view_g_rows<S>(K, fout, y0, y1 - 1);
      if (edge)
        march2<true>(K, fi, fo, L, y0, y1, ish_lo, ish_hi, ish2_lo, ish2_hi, NoRec{});
      else
        march2<false>(K, fi, fo, L, y0, y1, ish_lo, ish_hi, ish2_lo, ish2_hi, NoRec{});
    } else {
      const KTConsts& KM = kernarg_consts();   // K itself, for the march loops
      if constexpr (REC) {
        const Rec<View<S, AUX>> rec{make_view<S, AUX>(K, f1out), y0, y1};
        if (edge)
          march2<true>(KM, fi0, fo0, L, y0, y1, ish_lo, ish_hi, ish2_lo, ish2_hi, rec);
        else
          march2<false>(KM, fi0, fo0, L, y0, y1, ish_lo, ish_hi, ish2_lo, ish2_hi, rec);
      } else {
        if (edge)
          march2<true>(KM, fi0, fo0, L, y0, y1, ish_lo, ish_hi, ish2_lo, ish2_hi, NoRec{});
        else
          march2<false>(KM, fi0, fo0, L, y0, y1, ish_lo, ish_hi, ish2_lo, ish2_hi, NoRec{});
      }
    }
  }
}

template <typename S>
__device__ __forceinline__ double ldv(const S* p) {
  return (double)(*p);
}

template <typename S>
__device__ __forceinline__ void store9(const KTConsts& K, S* __restrict__ f, int x, int y, const double v[9]) {
  S* p = f + (int64_t)y * K.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) p[i * K.plane] = (S)v[i];
}

// ------------------------------------------------------------------ init / moments / invariants

template <typename S>
__global__ __launch_bounds__(256) void k_init(KTConsts K, const double* __restrict__ rho,
                                              const double* __restrict__ ux, const double* __restrict__ uy,
                                              const double* __restrict__ p, S* __restrict__ f) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= K.nx) return;
  for (int y = blockIdx.y; y < K.ny; y += gridDim.y) {
    const int64_t q = (int64_t)y * K.nx + x;
    const double r = rho[q], u = ux[q], v = uy[q];
    const double T = p[q] / r;
    double fe[9];
    feq9(K, r, u, v, T, fma(u, u, v * v), fe);
    store9(K, f, x, y, fe);
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_moments(KTConsts K, const S* __restrict__ f, double* rho,
                                                 double* ux, double* uy, double* T, uint32_t* flags) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  for (int y = blockIdx.y; y < K.ny; y += gridDim.y) {
  bool bad = false, rneg = false, tneg = false;
  if (x < K.nx) {
    const S* p = f + (int64_t)y * K.pitch + x;
    double c[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = ldv(p + i * K.plane);
    const Prim P = moments9(K, c);
    const int64_t q = (int64_t)y * K.nx + x;
    if (rho) rho[q] = P.rho;
    if (ux) ux[q] = P.ux;
    if (uy) uy[q] = P.uy;
    if (T) T[q] = P.T;
    bad = !(isfinite(P.rho) && isfinite(P.ux) && isfinite(P.uy) && isfinite(P.T));
    rneg = !(P.rho > 0.0) && !bad;
    tneg = !(P.T > 0.0) && !bad;
  }
  if (flags) {
    const unsigned long long mb = __ballot(bad), mr = __ballot(rneg), mt = __ballot(tneg);
    if (__lane_id() == 0 && (mb | mr | mt)) {
      const uint32_t bits = (mb ? LB_FLAG_NONFINITE : 0u) | (mr ? LB_FLAG_RHO_NONPOS : 0u) |
                            (mt ? LB_FLAG_T_NONPOS : 0u);
      atomicOr(flags, bits);
      if (mb) atomicAdd(flags + 1, (uint32_t)__popcll(mb));
      if (mr) atomicAdd(flags + 2, (uint32_t)__popcll(mr));
      if (mt) atomicAdd(flags + 3, (uint32_t)__popcll(mt));
    }
  }
  }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Per-block partial sums of (rho, jx, jy, E) over rows [b*rpb, (b+1)*rpb): fixed order.
// Sum of v over the 64 lanes of the wavefront (butterfly of lane shuffles; every
// lane ends with the same total, in a fixed order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums of the 4 accumulators over a 256-thread block (4 wavefronts; both callers
// launch 256 threads): wavefront shuffles, then
// the 4 wave totals combined in LDS by thread 0..3 (fixed order).
__device__ __forceinline__ void block_sum4(double acc[4], double* out4) {
  __shared__ double sh[4][4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][wave] = acc[k];
  __syncthreads();
  if (threadIdx.x < 4) out4[threadIdx.x] = (sh[threadIdx.x][0] + sh[threadIdx.x][1]) + (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
}

template <typename S>
__global__ __launch_bounds__(256) void k_inv_partial(KTConsts K, const S* __restrict__ f, int rpb,
                                                     double* __restrict__ part) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int y0 = blockIdx.x * rpb, y1 = min(y0 + rpb, K.ny);
  for (int y = y0; y < y1; ++y) {
    for (int x = threadIdx.x; x < K.nx; x += blockDim.x) {
      const S* p = f + (int64_t)y * K.pitch + x;
      double c[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) c[i] = ldv(p + i * K.plane);
      const double s14 = (c[1] + c[2]) + (c[3] + c[4]);
      const double s58 = (c[5] + c[6]) + (c[7] + c[8]);
      acc[0] += (c[0] + s14) + s58;
      acc[1] += fma(K.c1, c[3] - c[1], K.s * ((c[6] + c[7]) - (c[5] + c[8])));
      acc[2] += fma(K.c1, c[4] - c[2], K.s * ((c[7] + c[8]) - (c[5] + c[6])));
      acc[3] += fma(K.eta0sq, c[0], fma(K.c1sq, s14, K.c2sq * s58));
    }
  }
  block_sum4(acc, part + (int64_t)blockIdx.x * 4);
}

__global__ __launch_bounds__(256) void k_inv_final(const double* __restrict__ part, int nblk, double* out4) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    for (int k = 0; k < 4; ++k) acc[k] += part[(int64_t)b * 4 + k];
  block_sum4(acc, out4);
}

// ------------------------------------------------------------------ adjoint

// Transposed stencil. Site (x, y) receives W(i, k) g_i from every site whose
// neighbour k it is: from (x-1, y) as its x+dx neighbour (k = 1), from (x+1, y)
// as k = 2, from (x, y-1) as k = 3 and from (x, y+1) as k = 4, with periodic
// wrap. Where the site itself supplies a ghost of its own stencil (outflow: a
// copy; wall: a mirrored copy) it also receives that ghost's share; Dirichlet
// and shock ghosts do not depend on f and contribute nothing.
template <int E>
__device__ __forceinline__ void adj_edge(const KTConsts& K, const double gc[9], int along, double acc[9]) {
  // k of the ghost that edge E feeds: x- -> 2, x+ -> 1, y- -> 4, y+ -> 3
  constexpr int k = (E == 0) ? 2 : (E == 1) ? 1 : (E == 2) ? 4 : 3;
  const int kind = K.kind[E];
  if (along < K.split[E]) return;
  if (kind == BC_OUTFLOW) {
#pragma unroll
    for (int i = 0; i < 9; ++i) acc[i] = fma(wcoef(K, i, k), gc[i], acc[i]);
  } else if (kind == BC_WALL) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int m = (E < 2) ? mirror_x(i) : mirror_y(i);
      acc[i] = fma(wcoef(K, m, k), gc[m], acc[i]);
    }
  }
}

// One row of the adjoint march: g_n at row y from g_{n+1} rows y-1 (gd), y (gc),
// y+1 (gu) (zero where a non-periodic edge has no such row), the halo values hc
// of row y and f_n at the site. Accumulation order: collision adjoint, then
// the y+1, y-1, x+1, x-1 and centre terms, then the own-ghost corrections.
template <bool XEDGE, class VG, typename S>
__device__ __forceinline__ void adj_row(const KTConsts& K, const VG& gi, const VG& go, const Lane& L, uint32_t vbg,
                                        int y, const double gd[9], const double gc[9], const double gu[9],
                                        const double hc[9], const S fr[9], bool perx, bool pery) {
  double fc[9], acc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) fc[i] = widen(fr[i]);
  const Prim P = moments9(K, fc);
  collision_adjoint(K, P, gc, acc);
  const int x = L.x, nx = K.nx;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double gr = shl1(hc[i], gc[i]);   // g_{n+1}(x+1): site x is its x-dx neighbour
    double gl = shr1(hc[i], gc[i]);   // g_{n+1}(x-1): site x is its x+dx neighbour
    if (XEDGE) {
      if (x == 0 && !perx) gl = 0.0;
      if (x == nx - 1) gr = perx ? gi.ld(i, y, 0) : 0.0;
    }
    double a = acc[i];
    a = fma(wcoef(K, i, 4), gu[i], a);
    a = fma(wcoef(K, i, 3), gd[i], a);
    a = fma(wcoef(K, i, 2), gr, a);
    a = fma(wcoef(K, i, 1), gl, a);
    acc[i] = fma(wcoef(K, i, 0), gc[i], a);
  }
  if (XEDGE) {
    if (x == 0 && !perx) adj_edge<0>(K, gc, y, acc);
    if (x == nx - 1 && !perx) adj_edge<1>(K, gc, y, acc);
  }
  if (y == 0 && !pery) adj_edge<2>(K, gc, x, acc);
  if (y == K.ny - 1 && !pery) adj_edge<3>(K, gc, x, acc);
  go.store9(y, vbg, acc);   // padding lanes too (see row_update)
}

// One row y < ny-1 of the adjoint march (the same pipeline as march_row): issue
// the fetches of g_{n+1} row y+2 (into F), of f_n row y+1 (into FN) and of the
// g_{n+1} halo of row y+1 (into HN), all unconditional with clamped rows;
// update row y; shift gd <- gc <- row y+1.
template <bool XEDGE, class VF, class VG>
__device__ __forceinline__ void adj_march_row(const KTConsts& K, const VF& ff, const VG& gi, const VG& go,
                                              const Lane& L, uint32_t vbf, int y, int y1, int ylast, bool perx,
                                              bool pery, double pd[9], double cd[9], const double N[9],
                                              const double HC[9], const Sto<VF> FC[9], double F[9], double HN[9],
                                              Sto<VF> FN[9]) {
  gi.raw9(min(y + 2, ylast), L.vbx, F);
  ff.raw9(min(y + 1, y1 - 1), vbf, FN);
  gi.raw9(min(y + 1, y1 - 1), L.vbh, HN);
  adj_row<XEDGE>(K, gi, go, L, L.vbx, y, pd, cd, N, HC, FC, perx, pery);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = N[i];
  }
  __builtin_amdgcn_sched_barrier(0);
}

// Row y = ny-1 of the adjoint march: above it lies row 0 (periodic) or nothing.
template <bool XEDGE, class VF, class VG>
__device__ __forceinline__ void adj_top_row(const KTConsts& K, const VF& ff, const VG& gi, const VG& go,
                                            const Lane& L, int y, bool perx, bool pery, const double pd[9],
                                            const double cd[9], const double HC[9], const Sto<VF> FC[9]) {
  double nd[9];
  if (pery) {
    gi.load9_any(0, L.vbx, nd);   // row 0
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) nd[i] = 0.0;
  }
  adj_row<XEDGE>(K, gi, go, L, L.vbx, y, pd, cd, nd, HC, FC, perx, pery);
}

// Adjoint march over a 64-column wavefront strip with the structure of the
// forward march: g_{n+1} rows y-1, y, y+1 in registers, row y+2, the f_n row
// y+1 and the halo of row y+1 fetched one row ahead into the idle one of two
// register sets, x-neighbours through DPP shifts (lanes 0 and 63 use the halo
// columns), the top row of the grid after the loop.
template <bool XEDGE, class VF, class VG>
__device__ __forceinline__ void adj_march(const KTConsts& K, const VF& ff, const VG& gi, const VG& go, int xw0,
                                          int lane, int y0, int y1) {
  using S = Sto<VF>;
  const int ny = K.ny;
  const bool perx = (K.kind[0] == BC_PERIODIC), pery = (K.kind[2] == BC_PERIODIC);
  const Lane L = make_lane<double>(K, xw0, lane);
  const uint32_t vbf = (uint32_t)L.x * sizeof(S);
  double pd[9], cd[9], N0[9], N1[9], H0[9], H1[9];
  S FC0[9], FC1[9];
  if (y0 > 0)
    gi.load9(y0 - 1, L.vbx, pd);
  else if (pery)
    gi.load9_any(ny - 1, L.vbx, pd);
  else {
#pragma unroll
    for (int i = 0; i < 9; ++i) pd[i] = 0.0;
  }
  gi.load9(y0, L.vbx, cd);
  gi.raw9(y0, L.vbh, H0);
  gi.raw9(min(y0 + 1, ny - 1), L.vbx, N0);
  ff.raw9(y0, vbf, FC0);
  // the prologue's fetches land before the loop (see march)
#pragma unroll
  for (int i = 0; i < 9; ++i) asm volatile("" ::"v"(pd[i]), "v"(cd[i]), "v"(N0[i]), "v"(H0[i]), "v"(FC0[i]));
  const int ylast = min(y1, ny - 1);
  int y = y0;
  for (; y + 1 < ylast; y += 2) {
    adj_march_row<XEDGE>(K, ff, gi, go, L, vbf, y, y1, ylast, perx, pery, pd, cd, N0, H0, FC0, N1, H1, FC1);
    adj_march_row<XEDGE>(K, ff, gi, go, L, vbf, y + 1, y1, ylast, perx, pery, pd, cd, N1, H1, FC1, N0, H0, FC0);
  }
  if (y < ylast) {
    adj_march_row<XEDGE>(K, ff, gi, go, L, vbf, y, y1, ylast, perx, pery, pd, cd, N0, H0, FC0, N1, H1, FC1);
    if (y + 1 < y1) adj_top_row<XEDGE>(K, ff, gi, go, L, y + 1, perx, pery, pd, cd, H1, FC1);
  } else if (y < y1) {
    adj_top_row<XEDGE>(K, ff, gi, go, L, y, perx, pery, pd, cd, H0, FC0);
  }
}

// g_n = (dS/df)^T g_np1: transposed stencil over g_np1 plus the local collision adjoint.
// WIDE: the adjoint arrays (double) are 4 GiB or more; all three are then
// addressed through ViewG.
template <typename S, bool WIDE>
__global__ __launch_bounds__(256) void k_adjoint(KTConsts K, const S* __restrict__ fn,
                                                 const double* __restrict__ g1, double* __restrict__ g0,
                                                 int rows, int nstrips, int nblocks, int xcd_map) {
  int strip, chunk;
  tile_of_block(blockIdx.x, nstrips, nblocks, xcd_map, &strip, &chunk);
  const int lane = threadIdx.x & 63;
  const int xw0 = strip * blockDim.x + (threadIdx.x & ~63);
  if (xw0 >= K.nx) return;   // whole wavefront beyond the grid
  const int y0 = chunk * rows;
  const int y1 = min(y0 + rows, K.ny);
  if constexpr (WIDE) {
    const ViewG<S> ff = make_view_g<S>(K, fn, y0, y1);
    const ViewG<double> gi = make_view_g<double>(K, g1, y0, y1), go = make_view_g<double>(K, g0, y0, y1);
    if (xw0 == 0 || xw0 + 64 >= K.nx)
      adj_march<true>(K, ff, gi, go, xw0, lane, y0, y1);
    else
      adj_march<false>(K, ff, gi, go, xw0, lane, y0, y1);
  } else {
    const View<S> ff = make_view<S>(K, fn);
    const View<double> gi = make_view<double>(K, g1), go = make_view<double>(K, g0);
    const KTConsts& KM = kernarg_consts();   // K itself, for the march loops
    if (xw0 == 0 || xw0 + 64 >= K.nx)
      adj_march<true>(KM, ff, gi, go, xw0, lane, y0, y1);
    else
      adj_march<false>(KM, ff, gi, go, xw0, lane, y0, y1);
  }
}

__global__ __launch_bounds__(256) void k_init_adjoint(KTConsts K, const double* __restrict__ rho,
                                                      const double* __restrict__ ux,
                                                      const double* __restrict__ uy,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ g,
                                                      double* __restrict__ grho) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= K.nx) return;
  for (int y = blockIdx.y; y < K.ny; y += gridDim.y) {
    const int64_t q = (int64_t)y * K.nx + x;
    const double* pg = g + (int64_t)y * K.pitch + x;
    double gv[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) gv[i] = pg[i * K.plane];
    grho[q] = init_adjoint_site(K, rho[q], ux[q], uy[q], p[q], gv);
  }
}

// ------------------------------------------------------------------ three steps per pass

// Three consecutive steps in one pass over an FP64 array: the two-step march with
// a third stage. Lane j of a wavefront holds column X0 - 3 + j; f1 is right on
// lanes 1..62, f2 on 2..61, and lanes 3..60 (58 columns) store f3. While f1 of
// row y is computed, the march also computes f2 of row y-1 and f3 of row y-2
// (stored), so an output tile [y0, y1) computes f1 on rows y0-2 .. y1+1 and f2
// on rows y0-1 .. y1 from f0 rows y0-3 .. y1+2. As in the two-step march every
// ghost of f1 and f2 is formed as a single step forms it from the stored state
// (x ghosts through ghost_x; y ghosts of a non-periodic axis from the edge row
// at that step's time index; a periodic y axis wraps its rows), so the result is
// bitwise that of three single steps. HBM moves the 9 + 9 values of a site once
// per three steps.

// Row y of an axis of ny >= 3 rows with wrapping, for -3 <= y <= ny + 2.
__device__ __forceinline__ int wrap_row(int y, int ny) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); }

// One row of the march of a tile with no y ghost rows: fetch f0 row y+3 (F),
// compute f1 of row y (N: f0 row y+1), f2 of row y-1 and f3 of row y-2 (stored);
// shift the windows. rw(): the grid row of a march row (wrapped for a periodic
// axis), yl the last f0 row the tile reads.
template <bool XEDGE, class V>
__device__ __forceinline__ void march3_row(const KTConsts& K, const V& fi, const V& fo, const Lane2& L, int y,
                                           int yl, int ny, bool pery, double pd[9], double cd[9], double q0[9],
                                           double q1[9], double r0[9], double r1[9], const double N[9],
                                           double F[9]) {
  static_assert(sizeof(Sto<V>) == 8, "three steps per pass run on FP64 arrays");
  const int yf = min(y + 3, yl);
  fi.raw9(pery ? wrap_row(yf, ny) : yf, L.vbx, F);
  double t[9], u[9];
  row_first<XEDGE, V, true>(K, fi, L, pery ? wrap_row(y, ny) : y, pd, cd, N, t);              // f1(y)
  __builtin_amdgcn_sched_barrier(0);   // the updates one after the other (register pressure)
  row_first<XEDGE, V, true>(K, fi, L, pery ? wrap_row(y - 1, ny) : y - 1, q0, q1, t, u);      // f2(y-1)
  __builtin_amdgcn_sched_barrier(0);
  row_second<XEDGE, V, double, double, double, true>(K, fo, L, y - 2, r0, r1, u);                                    // f3(y-2)
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = N[i];
    q0[i] = q1[i];
    q1[i] = t[i];
    r0[i] = r1[i];
    r1[i] = u[i];
  }
  __builtin_amdgcn_sched_barrier(0);
}

// The march of an output tile [y0, y1) whose f0 rows y0-3 .. y1+2 all lie in the
// grid, or wrap on a periodic y axis (no ghost rows): four priming rows, then
// one row of every stage per f1 row.
template <bool XEDGE, class V>
__device__ __forceinline__ void march3_fast(const KTConsts& K, const V& fi, const V& fo, const Lane2& L, int y0,
                                            int y1) {
  const int ny = K.ny;
  const bool pery = (K.kind[2] == BC_PERIODIC);
  const int yl = y1 + 2;
  auto rw = [&](int y) { return pery ? wrap_row(y, ny) : y; };
  double pd[9], cd[9], N0[9], N1[9], N2[9], q0[9], q1[9], r0[9], r1[9], t[9];
  const int ya = y0 - 2;   // first f1 row
  fi.raw9(rw(ya - 1), L.vbx, pd);
  fi.raw9(rw(ya), L.vbx, cd);
  fi.raw9(rw(ya + 1), L.vbx, N0);
  fi.raw9(rw(ya + 2), L.vbx, N1);
  // f1 row ya (q0)
  fi.raw9(rw(ya + 3), L.vbx, N2);
  row_first<XEDGE, V, true>(K, fi, L, rw(ya), pd, cd, N0, q0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = N0[i];
  }
  __builtin_amdgcn_sched_barrier(0);
  // f1 row ya+1 (q1)
  fi.raw9(rw(min(ya + 4, yl)), L.vbx, N0);
  row_first<XEDGE, V, true>(K, fi, L, rw(ya + 1), pd, cd, N1, q1);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = N1[i];
  }
  __builtin_amdgcn_sched_barrier(0);
  // f1 row ya+2, f2 row ya+1 (r0)
  fi.raw9(rw(min(ya + 5, yl)), L.vbx, N1);
  row_first<XEDGE, V, true>(K, fi, L, rw(ya + 2), pd, cd, N2, t);
  __builtin_amdgcn_sched_barrier(0);
  row_first<XEDGE, V, true>(K, fi, L, rw(ya + 1), q0, q1, t, r0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = N2[i];
    q0[i] = q1[i];
    q1[i] = t[i];
  }
  __builtin_amdgcn_sched_barrier(0);
  // f1 row ya+3, f2 row ya+2 = y0 (r1)
  fi.raw9(rw(min(ya + 6, yl)), L.vbx, N2);
  row_first<XEDGE, V, true>(K, fi, L, rw(ya + 3), pd, cd, N0, t);
  __builtin_amdgcn_sched_barrier(0);
  row_first<XEDGE, V, true>(K, fi, L, rw(ya + 2), q0, q1, t, r1);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    pd[i] = cd[i];
    cd[i] = N0[i];
    q0[i] = q1[i];
    q1[i] = t[i];
  }
  __builtin_amdgcn_sched_barrier(0);
  // rows y = y0+2 .. y1+1: f0 rows y+1, y+2 in flight in N1, N2; N0 free. The
  // sets rotate with period three (the loop is unrolled by three).
  int y = y0 + 2;
  const int ye = y1 + 1;
  for (; y + 2 <= ye; y += 3) {
    march3_row<XEDGE>(K, fi, fo, L, y, yl, ny, pery, pd, cd, q0, q1, r0, r1, N1, N0);
    march3_row<XEDGE>(K, fi, fo, L, y + 1, yl, ny, pery, pd, cd, q0, q1, r0, r1, N2, N1);
    march3_row<XEDGE>(K, fi, fo, L, y + 2, yl, ny, pery, pd, cd, q0, q1, r0, r1, N0, N2);
  }
  for (; y <= ye; ++y) {   // 0-2 rows left: one code copy, the sets moved down
    march3_row<XEDGE>(K, fi, fo, L, y, yl, ny, pery, pd, cd, q0, q1, r0, r1, N1, N0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      N1[i] = N2[i];
      N2[i] = N0[i];
    }
  }
}

// The march of any output tile, one f0 row fetched per march row: on a periodic
// y axis the rows wrap; otherwise f1 and f2 rows are clipped to the grid and
// the f0, f1 and f2 ghost rows below row 0 and above row ny-1 are formed at
// their own time indices (ish0 / ish1 / ish2: the shock edges' cells at steps
// n, n+1, n+2). Used for the tiles march3_fast does not take.
template <bool XEDGE, class V>
__device__ __forceinline__ void march3_edge(const KTConsts& K, const V& fi, const V& fo, const Lane2& L, int y0,
                                            int y1, int ish0_lo, int ish0_hi, int ish1_lo, int ish1_hi,
                                            int ish2_lo, int ish2_hi) {
  const int ny = K.ny;
  const bool pery = (K.kind[2] == BC_PERIODIC);
  auto rw = [&](int y) { return pery ? wrap_row(y, ny) : y; };
  // f1 rows [a1, b1] and f2 rows [a2, b2] of the march (virtual rows when periodic)
  const int a1 = pery ? y0 - 2 : max(y0 - 2, 0), b1 = pery ? y1 + 1 : min(y1 + 1, ny - 1);
  const int a2 = pery ? y0 - 1 : max(y0 - 1, 0), b2 = pery ? y1 : min(y1, ny - 1);
  const int ye = (!pery && b1 == ny - 1) ? ny + 1 : b1;   // the top edge needs two more rows
  double pd[9], cd[9], q0[9], q1[9], r0[9], r1[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) q0[i] = q1[i] = r0[i] = r1[i] = 0.0;
  if (pery || a1 > 0)
    fi.load9(rw(a1 - 1), L.vbx, pd);
  else
    ghost_row<2, V, true>(K, fi, L.xs, L.vbx, ish0_lo, pd);
  fi.load9(rw(a1), L.vbx, cd);
  for (int y = a1; y <= ye; ++y) {
    // f1 row y (q0, q1: f1 rows y-2, y-1; pd, cd: f0 rows y-1, y)
    double nd[9], t[9], u[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) nd[i] = t[i] = u[i] = 0.0;
    if (y <= b1) {
      if (pery || y + 1 < ny)
        fi.load9(rw(y + 1), L.vbx, nd);
      else
        ghost_row<3, V, true>(K, fi, L.xs, L.vbx, ish0_hi, nd);
      row_first<XEDGE, V, true>(K, fi, L, rw(y), pd, cd, nd, t);
    } else if (y == ny) {   // the f1 ghost above row ny-1 (not periodic)
      ghost_row_f1<3, double, true>(K, L.xs, ish1_hi, q1, t);
    }
    // f2 row z = y-1 from f1 rows z-1 (the ghost below row 0 for z = 0), z, z+1
    const int z = y - 1;
    if (z >= a2 && z <= b2) {
      if (!pery && z == 0) {
        double g[9];
        ghost_row_f1<2, double, true>(K, L.xs, ish1_lo, q1, g);
        row_first<XEDGE, V, true>(K, fi, L, z, g, q1, t, u);
      } else {
        row_first<XEDGE, V, true>(K, fi, L, rw(z), q0, q1, t, u);
      }
    } else if (!pery && z == ny) {   // the f2 ghost above row ny-1
      ghost_row_f1<3, double, true>(K, L.xs, ish2_hi, r1, u);
    }
    // f3 row w = y-2 from f2 rows w-1 (the ghost below row 0 for w = 0), w, w+1
    const int w = y - 2;
    if (w >= y0 && w < y1) {
      if (!pery && w == 0) {
        double g[9];
        ghost_row_f1<2, double, true>(K, L.xs, ish2_lo, r1, g);
        row_second<XEDGE, V, double, double, double, true>(K, fo, L, w, g, r1, u);
      } else {
        row_second<XEDGE, V, double, double, double, true>(K, fo, L, w, r0, r1, u);
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      pd[i] = cd[i];
      cd[i] = nd[i];
      q0[i] = q1[i];
      q1[i] = t[i];
      r0[i] = r1[i];
      r1[i] = u[i];
    }
  }
}

// Tiles in raster order, one block per tile when gridDim.x equals the tile count.
// Arrays below 4 GiB, ny >= 3.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_step3(
    KTConsts K, const double* __restrict__ fin, double* __restrict__ fout, int rows, int nstrips, int ntiles,
    int ish0_lo, int ish0_hi, int ish1_lo, int ish1_hi, int ish2_lo, int ish2_hi) {
  const View<double, 2> fi = make_view<double, 2>(K, fin), fo = make_view<double, 2>(K, fout);   // NT stores
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  for (int id = blockIdx.x; id < ntiles; id += gridDim.x) {
    const int strip = id % nstrips, chunk = id / nstrips;
    // the strip's first column, the same for the whole wavefront (scalar branches below)
    const int X0 = __builtin_amdgcn_readfirstlane((strip * wpb + (int)(threadIdx.x >> 6)) * 58);
    if (X0 >= K.nx) continue;   // whole wavefront beyond the grid
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, K.ny);
    const Lane2 L = make_lane2<double>(K, X0, lane, 3);
    // the lanes hold columns X0-3 .. X0+60: x-edge logic when 0 or nx-1 is among them
    const bool xedge = (X0 == 0) || (X0 + 61 >= K.nx);
    // the prefetching march for strips away from the x edges whose rows need no
    // y ghosts; the row-by-row march for the rest (x-edge strips, y-edge tiles)
    const bool fast = !xedge && ((K.kind[2] == BC_PERIODIC) || (y0 >= 3 && y1 <= K.ny - 3));
    const KTConsts& KM = kernarg_consts();   // K itself, for the march loops
    if (fast)
      march3_fast<false>(KM, fi, fo, L, y0, y1);
    else if (xedge)
      march3_edge<true>(KM, fi, fo, L, y0, y1, ish0_lo, ish0_hi, ish1_lo, ish1_hi, ish2_lo, ish2_hi);
    else
      march3_edge<false>(KM, fi, fo, L, y0, y1, ish0_lo, ish0_hi, ish1_lo, ish1_hi, ish2_lo, ish2_hi);
  }
}

// ------------------------------------------------------------------ batched

using WorkItem = LbktWorkItem;

struct ProbInfo {
  int64_t offset;   // element offset of the problem's array in the packed buffer
};

template <typename S>
__global__ __launch_bounds__(256) void k_step_batched(const KTConsts* __restrict__ Ks,
                                                      const ProbInfo* __restrict__ info,
                                                      const WorkItem* __restrict__ items, const S* fin, S* fout) {
  const WorkItem w = items[blockIdx.x];
  const KTConsts& K = Ks[w.prob];
  const int64_t off = info[w.prob].offset;
  const int lane = threadIdx.x & 63;
  const int xw0 = w.strip * blockDim.x + (threadIdx.x & ~63);
  if (xw0 >= K.nx) return;
  const View<S, LB_STORE_AUX, false> fi = make_view<S, LB_STORE_AUX, false>(K, fin + off),
                                     fo = make_view<S, LB_STORE_AUX, false>(K, fout + off);
  const Lane L = make_lane<S>(K, xw0, lane);
  if (xw0 == 0 || xw0 + 64 >= K.nx)
    march<true>(K, fi, fo, L, 0, K.ny, 0, 0);
  else
    march<false>(K, fi, fo, L, 0, K.ny, 0, 0);
}

// Two steps per pass of every problem (the two-step march over all rows of a
// 60-column-per-wavefront strip; batched problems have no shock edges). Needs
// ny >= 2 for every problem.
// Two steps on a strip of a 4-row grid with a periodic y axis (the batched
// Riemann problems): the four f0 rows are fetched together, f1 of each row is
// computed once from its periodic neighbours in registers (the general march
// recomputes the far rows for the y ghosts: 6 first-step rows per 4 output rows)
// and the four second-step rows follow. Same per-row updates as march2, so the
// result is bitwise the same.
template <bool XEDGE, class V>
__device__ __forceinline__ void march2_ny4(const KTConsts& K, const V& fi, const V& fo, const Lane2& L) {
  using S = Sto<V>;
  S r0[9], r1[9], r2[9], r3[9];
  fi.raw9(0, L.vbx, r0);
  fi.raw9(1, L.vbx, r1);
  fi.raw9(2, L.vbx, r2);
  fi.raw9(3, L.vbx, r3);
  double d0[9], d1[9], d2[9], d3[9], t[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    d0[i] = widen(r0[i]);
    d1[i] = widen(r1[i]);
    d2[i] = widen(r2[i]);
    d3[i] = widen(r3[i]);
  }
  // one row at a time (the barriers keep the rows' temporaries from overlapping)
  S q0[9], q1[9], q2[9], q3[9];   // f1 rows 0..3, rounded to the storage type
  row_first<XEDGE>(K, fi, L, 0, d3, d0, d1, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) q0[i] = (S)t[i];
  __builtin_amdgcn_sched_barrier(0);
  row_first<XEDGE>(K, fi, L, 1, d0, d1, d2, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) q1[i] = (S)t[i];
  __builtin_amdgcn_sched_barrier(0);
  row_first<XEDGE>(K, fi, L, 2, d1, d2, d3, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) q2[i] = (S)t[i];
  __builtin_amdgcn_sched_barrier(0);
  row_first<XEDGE>(K, fi, L, 3, d2, d3, d0, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) q3[i] = (S)t[i];
  __builtin_amdgcn_sched_barrier(0);
  row_second<XEDGE>(K, fo, L, 0, q3, q0, q1);
  __builtin_amdgcn_sched_barrier(0);
  row_second<XEDGE>(K, fo, L, 1, q0, q1, q2);
  __builtin_amdgcn_sched_barrier(0);
  row_second<XEDGE>(K, fo, L, 2, q1, q2, q3);
  __builtin_amdgcn_sched_barrier(0);
  row_second<XEDGE>(K, fo, L, 3, q2, q3, q0);
}

// One step of row y of the strip's state (rows y-1, y, y+1 = pt, ct, nt, held in
// the storage type T) at the lane's column; xedge: the strip holds a
// non-periodic x edge. STORE: the last step of the pass, stored by the output
// lanes; otherwise rounded to the storage type into outt.
template <bool STORE, bool XEDGE, class V, typename T>
__device__ __forceinline__ void ny4_state_step_row(const KTConsts& K, const V& f, const Lane2& L, int y,
                                                   const T pt[9], const T ct[9], const T nt[9], T outt[9]) {
  double xm[9], xp[9], p[9], c[9], n[9], out[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {   // exact conversions (plain casts: the compiler places them)
    p[i] = (double)pt[i];
    c[i] = (double)ct[i];
    n[i] = (double)nt[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    xm[i] = shr1z(c[i]);   // lanes 0 and 63 get 0: their results are never used
    xp[i] = shl1z(c[i]);
  }
  if constexpr (XEDGE) ghost_x_select(K, L, y, c, xm, xp);
  site_update<sizeof(Sto<V>) == 4>(K, c, xp, xm, n, p, out);
  if constexpr (STORE) {
    if (L.out) f.store9(y, L.vbo, out);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) outt[i] = (T)(Sto<V>)out[i];
  }
}

template <bool XEDGE, class V, typename T>
__device__ __forceinline__ void ny4_state_step(const KTConsts& K, const V& fi, const Lane2& L, const T a0[9],
                                               const T a1[9], const T a2[9], const T a3[9], T b0[9], T b1[9],
                                               T b2[9], T b3[9]) {
  ny4_state_step_row<false, XEDGE>(K, fi, L, 0, a3, a0, a1, b0);
  __builtin_amdgcn_sched_barrier(0);
  ny4_state_step_row<false, XEDGE>(K, fi, L, 1, a0, a1, a2, b1);
  __builtin_amdgcn_sched_barrier(0);
  ny4_state_step_row<false, XEDGE>(K, fi, L, 2, a1, a2, a3, b2);
  __builtin_amdgcn_sched_barrier(0);
  ny4_state_step_row<false, XEDGE>(K, fi, L, 3, a2, a3, a0, b3);
  __builtin_amdgcn_sched_barrier(0);
}

// A problem's constants re-read through a pointer that the compiler cannot see
// through (as kernarg_consts does for the kernel-argument copy): the loads stay
// scalar and invariant, so each step re-issues them instead of keeping ~70 SGPRs
// of constants alive across all steps of the pass, spilled to VGPR lanes.
__device__ __forceinline__ const KTConsts& consts_opaque(const KTConsts* p) {
  auto kp = (const __attribute__((address_space(4))) KTConsts*)p;
  asm volatile("" : "+s"(kp));
  return *(const KTConsts*)kp;
}

// D (even) steps per pass on a strip of a 4-row grid with a periodic y axis: the
// whole state of the strip's 64 columns stays in registers between the steps, so
// the pass reads and writes the array once for D steps. Lane j holds column
// X0 - D + j; step s is right on lanes s .. 63-s (each step loses one lane on
// each side to its x-neighbours), so lanes D .. 63-D store and wavefronts start
// every 64 - 2D columns. Every intermediate state is rounded to the storage type
// and its x ghosts are formed as in a single step, so the result is bitwise that
// of D single steps.
template <int D, bool XEDGE, class V>
__device__ __forceinline__ void march_ny4_deep(const KTConsts* Kp, const V& fi, const V& fo, const Lane2& L) {
  static_assert(D >= 4 && D % 2 == 0, "the deep 4-row march takes an even number of steps >= 4");
  // only strips starting at column 0 form left x ghosts: the next strip's lanes
  // (from column 64 - 3D) must stay inside the grid
  static_assert(64 - 3 * D >= 0, "a deep pass takes at most 21 steps");
  using S = Sto<V>;
  S a0[9], a1[9], a2[9], a3[9], b0[9], b1[9], b2[9], b3[9];
  fi.raw9(0, L.vbx, a0);
  fi.raw9(1, L.vbx, a1);
  fi.raw9(2, L.vbx, a2);
  fi.raw9(3, L.vbx, a3);
  // steps 1 .. D-1 in registers (a -> b -> a ...), then step D from b, stored
  for (int k = 0; k < D / 2 - 1; ++k) {
    ny4_state_step<XEDGE>(consts_opaque(Kp), fi, L, a0, a1, a2, a3, b0, b1, b2, b3);
    ny4_state_step<XEDGE>(consts_opaque(Kp), fi, L, b0, b1, b2, b3, a0, a1, a2, a3);
  }
  ny4_state_step<XEDGE>(consts_opaque(Kp), fi, L, a0, a1, a2, a3, b0, b1, b2, b3);
  const KTConsts& K = consts_opaque(Kp);
  S t[9];
  ny4_state_step_row<true, XEDGE>(K, fo, L, 0, b3, b0, b1, t);
  __builtin_amdgcn_sched_barrier(0);
  ny4_state_step_row<true, XEDGE>(K, fo, L, 1, b0, b1, b2, t);
  __builtin_amdgcn_sched_barrier(0);
  ny4_state_step_row<true, XEDGE>(K, fo, L, 2, b1, b2, b3, t);
  __builtin_amdgcn_sched_barrier(0);
  ny4_state_step_row<true, XEDGE>(K, fo, L, 3, b2, b3, b0, t);
}

// One D-step work item of a batch of 4-row y-periodic problems: the strip of
// block_x / 64 wavefronts (64 - 2D output columns each) of problem w.prob.
template <typename S, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_stepD_batched_ny4(
    const KTConsts* __restrict__ Ks, const ProbInfo* __restrict__ info, const WorkItem* __restrict__ items,
    const S* fin, S* fout) {
  const WorkItem w = items[blockIdx.x];
  const KTConsts& K = Ks[w.prob];
  const int64_t off = info[w.prob].offset;
  const int lane = threadIdx.x & 63;
  // the strip's first column, the same for the whole wavefront (so the tests on it
  // below are wave-uniform branches)
  const int X0 = __builtin_amdgcn_readfirstlane(
      (w.strip * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6)) * (64 - 2 * D));
  if (X0 >= K.nx) return;
  constexpr int AUX = sizeof(S) == 8 ? 2 : 0;   // the stores of k_step2
  const View<S, AUX, false> fi = make_view<S, AUX, false>(K, fin + off), fo = make_view<S, AUX, false>(K, fout + off);
  const Lane2 L = make_lane2<S>(K, X0, lane, D);
  if (!L.perx && (X0 == 0 || X0 + 64 - D >= K.nx))
    march_ny4_deep<D, true>(Ks + w.prob, fi, fo, L);
  else
    march_ny4_deep<D, false>(Ks + w.prob, fi, fo, L);
}

// D steps per pass over one 4-row grid with a periodic y axis (the pass lb_run
// takes there): the march of the batched kernel above, one wavefront per block,
// block b on the strip of columns starting at b * (64 - 2D); the grid constants
// are the kernel argument K, read by the march through the kernel-argument
// segment.
template <typename S, int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_stepD_ny4(KTConsts K, const S* fin,
                                                                                           S* fout) {
  const KTConsts* Kp =
      (const KTConsts*)(const __attribute__((address_space(4))) KTConsts*)__builtin_amdgcn_kernarg_segment_ptr();
  const KTConsts& KM = consts_opaque(Kp);   // K itself
  const int lane = threadIdx.x & 63;
  const int X0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (64 - 2 * D));
  if (X0 >= KM.nx) return;
  constexpr int AUX = sizeof(S) == 8 ? 2 : 0;   // the stores of k_step2
  const View<S, AUX, false> fi = make_view<S, AUX, false>(KM, fin), fo = make_view<S, AUX, false>(KM, fout);
  const Lane2 L = make_lane2<S>(KM, X0, lane, D);
  if (!L.perx && (X0 == 0 || X0 + 64 - D >= KM.nx))
    march_ny4_deep<D, true>(Kp, fi, fo, L);
  else
    march_ny4_deep<D, false>(Kp, fi, fo, L);
}

// The same D steps with the rows of a strip on the four wavefronts of a block:
// wavefront r holds row r of the strip's 64 columns and computes that row of
// every step with the per-row update of the march above (so the result is
// bitwise the same); the rows of each step reach the other wavefronts through
// LDS, written to one of two buffers while the other is read, with one barrier
// per step. A step then costs one row of arithmetic instead of four, which is
// what bounds a small grid. Every wavefront of a block runs every step (the
// block's strip and its x-edge case are uniform), so all of them reach each
// barrier.
template <int D, bool XEDGE, class V>
__device__ __forceinline__ void march_ny4_rows(const KTConsts& K, const V& fi, const V& fo, const Lane2& L, int r,
                                               Sto<V> (*xs)[4][9][64]) {
  static_assert(D >= 2 && D % 2 == 0 && 64 - 3 * D >= 0, "as the march above: even, at most 21 steps");
  using S = Sto<V>;
  S c[9];
  fi.raw9(r, L.vbx, c);
#pragma unroll
  for (int i = 0; i < 9; ++i) xs[0][r][i][threadIdx.x & 63] = c[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, rm = (r + 3) & 3, rp = (r + 1) & 3;
  for (int s = 0; s < D - 1; ++s) {
    const int b = s & 1;
    S p[9], n[9], o[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      p[i] = xs[b][rm][i][lane];
      n[i] = xs[b][rp][i][lane];
    }
    ny4_state_step_row<false, XEDGE>(K, fi, L, r, p, c, n, o);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      c[i] = o[i];
      xs[b ^ 1][r][i][lane] = o[i];
    }
    __syncthreads();
  }
  S p[9], n[9], t[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    p[i] = xs[(D - 1) & 1][rm][i][lane];
    n[i] = xs[(D - 1) & 1][rp][i][lane];
  }
  ny4_state_step_row<true, XEDGE>(K, fo, L, r, p, c, n, t);
}

template <typename S, int D>
__global__ __launch_bounds__(256) void k_stepD_ny4_rows(KTConsts K, const S* fin, S* fout) {
  __shared__ S xs[2][4][9][64];
  const KTConsts* Kp =
      (const KTConsts*)(const __attribute__((address_space(4))) KTConsts*)__builtin_amdgcn_kernarg_segment_ptr();
  const KTConsts& KM = consts_opaque(Kp);   // K itself
  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int X0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (64 - 2 * D));
  if (X0 >= KM.nx) return;   // the whole block
  constexpr int AUX = sizeof(S) == 8 ? 2 : 0;   // the stores of k_step2
  const View<S, AUX, false> fi = make_view<S, AUX, false>(KM, fin), fo = make_view<S, AUX, false>(KM, fout);
  const Lane2 L = make_lane2<S>(KM, X0, lane, D);
  if (!L.perx && (X0 == 0 || X0 + 64 - D >= KM.nx))
    march_ny4_rows<D, true>(KM, fi, fo, L, r, xs);
  else
    march_ny4_rows<D, false>(KM, fi, fo, L, r, xs);
}

// One D-step work item of a batch of 4-row y-periodic problems with the strip's
// rows on the four wavefronts of the block (march_ny4_rows; items planned for
// 64-thread strips): the FP32-storage batch's pass at block width 64 (256
// problems, four steps per pass: 27.4 vs 30.7 ms for the 2000 steps; in FP64
// storage, at eight steps, 32.2 vs 30.7 ms, so that batch keeps one wavefront).
template <typename S, int D>
__global__ __launch_bounds__(256) void k_stepD_batched_ny4_rows(const KTConsts* __restrict__ Ks,
                                                                const ProbInfo* __restrict__ info,
                                                                const WorkItem* __restrict__ items, const S* fin,
                                                                S* fout) {
  __shared__ S xs[2][4][9][64];
  const WorkItem w = items[blockIdx.x];
  const KTConsts& K = consts_opaque(Ks + w.prob);
  const int64_t off = info[w.prob].offset;
  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int X0 = __builtin_amdgcn_readfirstlane(w.strip * (64 - 2 * D));
  if (X0 >= K.nx) return;   // the whole block
  constexpr int AUX = sizeof(S) == 8 ? 2 : 0;   // the stores of k_step2
  const View<S, AUX, false> fi = make_view<S, AUX, false>(K, fin + off), fo = make_view<S, AUX, false>(K, fout + off);
  const Lane2 L = make_lane2<S>(K, X0, lane, D);
  if (!L.perx && (X0 == 0 || X0 + 64 - D >= K.nx))
    march_ny4_rows<D, true>(K, fi, fo, L, r, xs);
  else
    march_ny4_rows<D, false>(K, fi, fo, L, r, xs);
}

// One two-step work item of a batch: the strip of block_x / 64 wavefronts (60
// output columns each) of problem w.prob, all rows. NY4: every problem of the
// batch has 4 rows and a periodic y axis (an instantiation of its own, so that the
// general march keeps its register allocation).
template <typename S, bool NY4>
__device__ __forceinline__ void batched2_item(const KTConsts* __restrict__ Ks, const ProbInfo* __restrict__ info,
                                              const WorkItem w, const S* fin, S* fout) {
  const KTConsts& K = Ks[w.prob];
  const int64_t off = info[w.prob].offset;
  const int lane = threadIdx.x & 63;
  const int X0 = (w.strip * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6)) * 60;
  if (X0 >= K.nx) return;
  constexpr int AUX = sizeof(S) == 8 ? 2 : 0;   // the stores of k_step2
  const View<S, AUX, false> fi = make_view<S, AUX, false>(K, fin + off), fo = make_view<S, AUX, false>(K, fout + off);
  const Lane2 L = make_lane2<S>(K, X0, lane);
  const bool edge = (X0 == 0 || X0 + 62 >= K.nx);
  if constexpr (NY4) {
    if (edge)
      march2_ny4<true>(K, fi, fo, L);
    else
      march2_ny4<false>(K, fi, fo, L);
  } else if (edge) {
    march2<true>(K, fi, fo, L, 0, K.ny, 0, 0, 0, 0, NoRec{});
  } else {
    march2<false>(K, fi, fo, L, 0, K.ny, 0, 0, 0, 0, NoRec{});
  }
}

// One two-step pass of every problem: one block per work item.
template <typename S, bool NY4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_step2_batched(
    const KTConsts* __restrict__ Ks, const ProbInfo* __restrict__ info, const WorkItem* __restrict__ items,
    const S* fin, S* fout) {
  batched2_item<S, NY4>(Ks, info, items[blockIdx.x], fin, fout);
}

// Wait (one thread) until work item `item` has finished `k` passes: poll its
// progress counter with acquire loads (agent scope: the item's stores made before
// its release are then visible to this block), at most `limit` times, giving up
// early when another block of the launch has set the stop word. item < 0:
// nothing to wait for.
__device__ __forceinline__ bool wait_progress(const uint32_t* prog, int item, uint32_t k, uint32_t limit,
                                              const uint32_t* stop) {
  if (item < 0) return true;
  for (uint32_t n = 0;; ++n) {
    if (__hip_atomic_load(prog + item, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= k) return true;
    if (n >= limit || __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
    __builtin_amdgcn_s_sleep(2);
  }
}

// All npasses two-step passes of every problem in one launch of co-resident
// blocks. Block b takes work items b, b + gridDim.x, ... for pass 0, then the same
// items for pass 1, and so on (pass k reads fa and writes fb when k is even, the
// other way round when odd). An item's wavefronts read two columns beyond its
// strip on each side, held by the items nbrs[i] (left, right; -1: none), whose
// owners are blocks nbrs[i] mod gridDim.x. After all its items of pass k a block
// waits for its wavefronts' stores and publishes prog[b] = k + 1 with a release
// store (one per block and pass: each release writes back the L2, and per-item
// releases measured 1.5x slower); before pass k >= 1 of item i it waits until the
// owners of both neighbours have published k, which orders both the reads of pass
// k-1's output and the overwriting of pass k-2's output (read by them during pass
// k-1). No deadlock while every block is resident: the block at the smallest pass
// always finds the blocks it waits for done with the previous one. A wait that
// exceeds spin_limit polls sets the launch's stop word prog[nitems] (the other
// blocks then end at their next wait) and the batch's failure word *failed, and
// ends its block, so the launch always terminates; the result is then
// incomplete. prog[0 .. nitems] must be zero at the launch (gridDim.x <= nitems).
template <typename S, bool NY4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_step2_batched_persistent(
    const KTConsts* __restrict__ Ks, const ProbInfo* __restrict__ info, const WorkItem* __restrict__ items,
    const int2* __restrict__ nbrs, int nitems, S* fa, S* fb, int npasses, uint32_t* prog, uint32_t* failed,
    uint32_t spin_limit) {
  __shared__ uint32_t go;
  uint32_t* stop = prog + nitems;
  const int G = (int)gridDim.x;
  for (int k = 0; k < npasses; ++k) {
    const S* fin = (k & 1) ? fb : fa;
    S* fout = (k & 1) ? fa : fb;
    for (int i = blockIdx.x; i < nitems; i += G) {
      if (k > 0) {
        if (threadIdx.x == 0) {
          const int2 nb = nbrs[i];
          const bool ok = wait_progress(prog, nb.x < 0 ? -1 : nb.x % G, (uint32_t)k, spin_limit, stop) &&
                          wait_progress(prog, nb.y < 0 ? -1 : nb.y % G, (uint32_t)k, spin_limit, stop);
          if (!ok) {
            __hip_atomic_store(stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(failed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          go = ok ? 1u : 0u;
        }
        __syncthreads();
        if (go == 0u) return;
      }
      batched2_item<S, NY4>(Ks, info, items[i], fin, fout);
      __syncthreads();   // every wavefront is past its use of `go`
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wavefront's stores have completed
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(prog + blockIdx.x, (uint32_t)(k + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ host launch helpers

static size_t elem_size(lb_prec p) { return p == LB_F32 ? 4 : 8; }

// Arrays of 4 GiB and more exceed a buffer resource's 32-bit range: their
// kernels address each plane through its own resource over the rows of one
// tile (the WIDE instantiations).
static bool wide(const lb_grid* g, size_t esz) {
  return (uint64_t)lb_array_elems(g) * esz >= (uint64_t)1 << 32;
}

// Largest tile height whose window (rows + 2 rows of bytes) stays below 4 GiB.
static int wide_max_rows(const lb_grid* g, size_t esz) {
  const uint64_t rowB = (uint64_t)g->pitch * esz;
  return (int)std::min<uint64_t>(0x7fffffff, (((uint64_t)1 << 32) - 1) / rowB - 2);
}

static lb_status check_ptr(const void* p, const char* what) {
  if (!p) return fail(LB_EINVAL, std::string(what) + " is NULL");
  if (((uintptr_t)p) % 256 != 0) return fail(LB_EINVAL, std::string(what) + " must be 256-byte aligned");
  return LB_OK;
}

// ceil(a / b) for a >= 0, b > 0 without int overflow (ny may be up to 2^31 - 1).
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

struct Tile {
  int bx, rows, blocks;
  int steps;        // time steps per pass of lb_run: 1, 2 or 3 (the two- and three-step kernels)
  bool user;        // shape given by the caller (else the default, per kernel)
  bool steps_auto;  // steps not given: lb_run takes three per pass where that kernel runs
};

// Default launch shape: 256 x 16 tiles on large grids; on smaller grids the
// tile shrinks (rows first, down to 2, then columns) until there are at least
// 1024 tiles, four per compute unit.
// Default launch shape of the one-step kernel: 256 x 32 tiles, shrunk on smaller
// grids (rows, then columns) until there are at least min_tiles tiles.
static void default_tile(int nx, int ny, int* bx, int* rows, int min_tiles = 1024, int r0 = 32) {
  auto ntiles = [&](int b, int r) { return cdiv(nx, b) * cdiv(ny, r); };
  int b = 256, r = r0;
  while (ntiles(b, r) < min_tiles && r > 2) r /= 2;
  while (ntiles(b, r) < min_tiles && b > 64) b /= 2;
  *bx = b;
  *rows = r;
}

// Default launch shape of the float one-step kernel, whose tiles run in XCD bands
// (each XCD takes ntiles / 8 consecutive tiles of the raster): 256 columns by
// about 52 rows, with the number of row chunks a multiple of 8, so that every
// band is whole chunk rows. Measured on the 8192 x 2048 grid (ms per step, two
// interleaved rounds): 52 rows (40 chunks) 0.2470-0.2480, 64 (32) 0.2521-0.2524,
// 32 (64) 0.2537-0.2539, 43 (48) 0.2560, 128 (16) 0.2555, against 0.2585-0.2904 for
// 46-60 rows whose bands end inside a chunk row. Grids where this leaves fewer
// than 1024 tiles or tiles below 32 rows take 256 x 64 shrunk as above.
static void default_tile1f(int nx, int ny, int* bx, int* rows) {
  const int c0 = std::max(8, (int)std::lround(ny / (52.0 * 8.0)) * 8);
  // chunk counts c0, c0 + 8, c0 - 8, ... (ny rows need not split into exactly c chunks)
  for (int k = 0; k < 7; ++k) {
    const int c = c0 + ((k + 1) / 2) * 8 * (k % 2 ? 1 : -1);
    if (c < 8) continue;
    const int r = cdiv(ny, c);
    const int chunks = cdiv(ny, r);
    if (r >= 32 && chunks % 8 == 0 && cdiv(nx, 256) * chunks >= 1024) {
      *bx = 256;
      *rows = r;
      return;
    }
  }
  default_tile(nx, ny, bx, rows, 1024, 64);
}

// Default launch shape of the two-step pass: 256 threads (4 x 60 columns) by
// 11 rows (double) or 23 rows (float), the fastest measured on the 8192 x 2048
// grid (float, five interleaved rounds: 23 rows 115.6, 22 rows 115.3, 24 rows
// 114.7, 20 rows 114.8 GLUPS); on smaller grids the rows shrink (down to 2), then the columns, then
// the rows to 1, until there are at least 1024 tiles (on small grids
// parallelism outweighs the extra first-step rows of a short tile; measured on
// the paper's 200x4 .. 960x240 configurations against the autotuner).
static void default_tile2(int nx, int ny, lb_prec prec, int* bx, int* rows) {
  auto ntiles = [&](int b, int r) {
    return cdiv(cdiv(nx, 60), b / 64) * cdiv(ny, r);
  };
  int b = 256, r = prec == LB_F64 ? 11 : 23;
  while (ntiles(b, r) < 1024 && r > 2) r = std::max(2, r / 2);
  while (ntiles(b, r) < 1024 && b > 64) b /= 2;
  if (ntiles(b, r) < 1024) r = 1;
  *bx = b;
  *rows = std::min(r, ny);
}

void lbkt_default_tile2(int nx, int ny, lb_prec prec, int* bx, int* rows) { default_tile2(nx, ny, prec, bx, rows); }

// Default launch shape of the three-step pass (FP64): 128 threads (2 x 58
// columns) by 12 rows, the fastest measured on the 8192 x 2048 grid among 64 /
// 128 / 256 threads and 6-32 rows (ms per step, four rounds on two devices:
// 128 x 12 0.2051-0.2059, 256 x 11 0.2079-0.2084, 128 x 11 0.2083, 128 x 9
// 0.2078, 256 x 12 0.2093, 128 x 13 0.2110, 128 x 16 0.2231); shrunk on smaller
// grids as the two-step shape.
static void default_tile3(int nx, int ny, int* bx, int* rows) {
  auto ntiles = [&](int b, int r) { return cdiv(cdiv(nx, 58), b / 64) * cdiv(ny, r); };
  int b = 128, r = 12;
  while (ntiles(b, r) < 1024 && r > 2) r = std::max(2, r / 2);
  while (ntiles(b, r) < 1024 && b > 64) b /= 2;
  if (ntiles(b, r) < 1024) r = 1;
  *bx = b;
  *rows = std::min(r, ny);
}

// The three-step kernel runs on FP64 arrays below 4 GiB with ny >= 3 (its rows
// wrap with one addition on a periodic axis).
static bool three_ok(const lb_grid* g, lb_prec prec) {
  return prec == LB_F64 && g->ny >= 3 && !wide(g, elem_size(prec));
}

static lb_status resolve_tile(const lb_tile* tile, int nx, int ny, Tile* t) {
  int b, r, nb = 0;
  default_tile(nx, ny, &b, &r);
  const bool user = tile && (tile->block_x || tile->rows || tile->blocks);
  if (user) {
    b = tile->block_x;
    r = tile->rows;
    nb = tile->blocks;
  }
  if (b != 64 && b != 128 && b != 256) return fail(LB_EINVAL, "tile block_x must be 64, 128 or 256");
  if (r < 1) return fail(LB_EINVAL, "tile rows must be >= 1");
  if (nb < 0) return fail(LB_EINVAL, "tile blocks must be >= 0");
  const int sp = tile ? tile->steps : 0;
  if (sp < 0 || sp > 3) return fail(LB_EINVAL, "tile steps must be 0, 1, 2 or 3");
  t->bx = b;
  t->rows = std::min(r, ny);
  t->blocks = nb;
  t->user = user;
  // two steps per pass need two rows (the f1 window is primed with two rows)
  t->steps = (ny < 2) ? 1 : (sp == 0 ? 2 : sp);
  t->steps_auto = (sp == 0);
  return LB_OK;
}

static lb_status launch_step(const lb_grid* g, const KTConsts& K, lb_prec prec, const void* fin, void* fout,
                             int64_t step, const Tile& t, hipStream_t st) {
  const bool w = wide(g, elem_size(prec));
  int bx = t.bx, rows = t.rows;
  if (!t.user && prec == LB_F32) {
    default_tile1f(g->nx, g->ny, &bx, &rows);
    rows = std::min(rows, g->ny);
  }
  if (w) rows = std::min(rows, wide_max_rows(g, elem_size(prec)));
  const int64_t ntiles64 = cdiv(g->nx, bx) * cdiv(g->ny, rows);
  if (ntiles64 > 0x7fffffff) return fail(LB_EINVAL, "grid too large for one launch");
  const int nstrips = (int)cdiv(g->nx, bx);
  const int ntiles = (int)ntiles64;
  // tile order: double storage runs fastest in plain raster order (the whole
  // chip on a narrow band of rows: the rows shared by vertically adjacent tiles
  // are re-read from the last-level cache), float storage with each XCD on its
  // own band of tiles (measured on the 8192 x 2048 grid: 0.468 vs 0.497 ms for
  // double, 0.263 vs 0.274 ms for float)
  const int xcd_map = (prec == LB_F32 && ntiles % 8 == 0) ? 1 : 0;
  int nblocks = ntiles;
  if (t.blocks > 0 && t.blocks < ntiles) nblocks = xcd_map ? std::max(8, t.blocks & ~7) : t.blocks;
  const int ish_lo = shock_cells(g, 2, step), ish_hi = shock_cells(g, 3, step);
  if (prec == LB_F64) {
    auto kern = w ? k_step<double, true> : k_step<double, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(bx), 0, st, K, (const double*)fin, (double*)fout, rows, nstrips,
                       ntiles, xcd_map, ish_lo, ish_hi);
  } else {
    auto kern = w ? k_step<float, true> : k_step<float, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(bx), 0, st, K, (const float*)fin, (float*)fout, rows, nstrips,
                       ntiles, xcd_map, ish_lo, ish_hi);
  }
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// Two steps f_out = S(S(f_in)) at time indices step, step+1 in one pass.
// f1out: also store the state after the first step there (arrays below 4 GiB).
static lb_status launch_step2(const lb_grid* g, const KTConsts& K, lb_prec prec, const void* fin, void* fout,
                              int64_t step, const Tile& t, hipStream_t st, void* f1out = nullptr) {
  const bool w = wide(g, elem_size(prec));
  int bx = t.bx, rows = t.rows;
  if (!t.user) default_tile2(g->nx, g->ny, prec, &bx, &rows);
  if (w) rows = std::min(rows, wide_max_rows(g, elem_size(prec)) - 2);   // >= 1 (launch_steps)
  const int wpb = bx / 64;
  const int nstrips = (int)cdiv(cdiv(g->nx, 60), wpb);   // 60 output columns per wavefront
  const int64_t ntiles64 = (int64_t)nstrips * cdiv(g->ny, rows);
  if (ntiles64 > 0x7fffffff) return fail(LB_EINVAL, "grid too large for one launch");
  const int ntiles = (int)ntiles64;
  const int xcd_map = 0;   // raster order (the XCD bands measured 5-10% slower here)
  int nblocks = ntiles;
  if (t.blocks > 0 && t.blocks < ntiles) nblocks = xcd_map ? std::max(8, t.blocks & ~7) : t.blocks;
  const int ish_lo = shock_cells(g, 2, step), ish_hi = shock_cells(g, 3, step);
  const int ish2_lo = shock_cells(g, 2, step + 1), ish2_hi = shock_cells(g, 3, step + 1);
  if (f1out && w) return fail(LB_EUNSUPPORTED, "recording two steps per pass needs an array below 4 GiB");
  if (prec == LB_F64) {
    auto kern = f1out ? k_step2<double, false, true> : w ? k_step2<double, true> : k_step2<double, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(bx), 0, st, K, (const double*)fin, (double*)fout,
                       (double*)f1out, rows, nstrips, ntiles, xcd_map, ish_lo, ish_hi, ish2_lo, ish2_hi);
  } else {
    auto kern = f1out ? k_step2<float, false, true> : w ? k_step2<float, true> : k_step2<float, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(bx), 0, st, K, (const float*)fin, (float*)fout, (float*)f1out,
                       rows, nstrips, ntiles, xcd_map, ish_lo, ish_hi, ish2_lo, ish2_hi);
  }
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// Three steps f_out = S(S(S(f_in))) at time indices step .. step+2 in one pass
// (FP64 arrays below 4 GiB, ny >= 3).
static lb_status launch_step3(const lb_grid* g, const KTConsts& K, const void* fin, void* fout, int64_t step,
                              const Tile& t, hipStream_t st) {
  int bx = t.bx, rows = t.rows;
  if (!t.user) default_tile3(g->nx, g->ny, &bx, &rows);
  const int wpb = bx / 64;
  const int nstrips = (int)cdiv(cdiv(g->nx, 58), wpb);   // 58 output columns per wavefront
  const int64_t ntiles64 = (int64_t)nstrips * cdiv(g->ny, rows);
  if (ntiles64 > 0x7fffffff) return fail(LB_EINVAL, "grid too large for one launch");
  const int ntiles = (int)ntiles64;
  const int nblocks = (t.blocks > 0 && t.blocks < ntiles) ? t.blocks : ntiles;
  int ish[6];
  for (int k = 0; k < 3; ++k) {
    ish[2 * k] = shock_cells(g, 2, step + k);
    ish[2 * k + 1] = shock_cells(g, 3, step + k);
  }
  hipLaunchKernelGGL(k_step3, dim3(nblocks), dim3(bx), 0, st, K, (const double*)fin, (double*)fout, rows, nstrips,
                     ntiles, ish[0], ish[1], ish[2], ish[3], ish[4], ish[5]);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// The deep pass of lb_run (k_stepD_ny4, LB_DEEP1 steps with the strip's whole
// state in registers) runs on 4-row grids with a periodic y axis, at least 64
// columns and an array below 4 GiB.
static bool deep1_ok(const lb_grid* g, lb_prec prec) {
  return g->ny == 4 && g->edge[2].kind == LB_BC_PERIODIC && g->nx >= 64 && !wide(g, elem_size(prec));
}

static lb_status launch_stepD1(const lb_grid* g, const KTConsts& K, lb_prec prec, const void* fin, void* fout,
                               hipStream_t st) {
  constexpr int D = LB_DEEP1;
  const int nblocks = (int)cdiv(g->nx, 64 - 2 * D);
  if (LB_DEEP1_ROWS) {
    if (prec == LB_F64)
      hipLaunchKernelGGL((k_stepD_ny4_rows<double, D>), dim3(nblocks), dim3(256), 0, st, K, (const double*)fin,
                         (double*)fout);
    else
      hipLaunchKernelGGL((k_stepD_ny4_rows<float, D>), dim3(nblocks), dim3(256), 0, st, K, (const float*)fin,
                         (float*)fout);
  } else if (prec == LB_F64) {
    hipLaunchKernelGGL((k_stepD_ny4<double, D>), dim3(nblocks), dim3(64), 0, st, K, (const double*)fin,
                       (double*)fout);
  } else {
    hipLaunchKernelGGL((k_stepD_ny4<float, D>), dim3(nblocks), dim3(64), 0, st, K, (const float*)fin,
                       (float*)fout);
  }
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// Time steps per pass of lb_run for a resolved tile: by default 3 for FP64
// arrays where the three-step kernel runs and ny >= 32, else the tile's (1 or
// 2); an explicit 3 where that kernel does not run is LB_EUNSUPPORTED. On fewer
// rows most tiles lie at a y edge and take the row-by-row march, which made the
// paper's 4-row Riemann grids slower than two steps per pass (4.3 vs 3.0 us per
// step through a graph on the 200 x 4 Sod grid).
static lb_status pass_steps(const lb_grid* g, lb_prec prec, const Tile& t, int* steps) {
  if (t.steps == 3 && !three_ok(g, prec))
    return fail(LB_EUNSUPPORTED, "three steps per pass run on FP64 arrays below 4 GiB with ny >= 3");
  if (t.steps_auto && deep1_ok(g, prec)) {
    *steps = LB_DEEP1;
    return LB_OK;
  }
  *steps = (t.steps_auto && three_ok(g, prec) && g->ny >= 32) ? 3 : t.steps;
  return LB_OK;
}

// nsteps ping-pong steps from fa (result in fa when nsteps is even, else in fb).
// With two steps per pass, a pass also swaps the buffers once, so the pairs must
// be an even number: 2p steps in p passes with p even, and the remaining 0..3
// steps one per launch, first. A three-step pass swaps once for an odd number of
// steps, so n = 3p + r runs r = 0..2 single steps, then p three-step passes.
static lb_status launch_steps(const lb_grid* g, const KTConsts& K, lb_prec prec, void* fa, void* fb, int64_t step0,
                              int nsteps, const Tile& t, hipStream_t st) {
  int sp;
  lb_status s0 = pass_steps(g, prec, t, &sp);
  if (s0) return s0;
  if (sp == LB_DEEP1) {
    // an even number of deep passes (each swaps the buffers once for an even
    // number of steps), the remaining steps first, two per pass
    const int deep = (nsteps / LB_DEEP1) & ~1;
    const int rem = nsteps - deep * LB_DEEP1;
    Tile t2 = t;
    t2.steps = 2;
    t2.steps_auto = false;
    lb_status s;
    if ((s = launch_steps(g, K, prec, fa, fb, step0, rem, t2, st))) return s;
    for (int j = 0, k = rem % 2; j < deep; ++j, ++k)
      if ((s = launch_stepD1(g, K, prec, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, st))) return s;
    return LB_OK;
  }
  if (sp == 3) {
    const int triples = nsteps / 3;
    int64_t n = step0;
    int k = 0;
    lb_status s;
    for (int j = 0; j < nsteps - 3 * triples; ++j, ++k, ++n)
      if ((s = launch_step(g, K, prec, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, n, t, st))) return s;
    for (int j = 0; j < triples; ++j, ++k, n += 3)
      if ((s = launch_step3(g, K, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, n, t, st))) return s;
    return LB_OK;
  }
  // a large array's two-step window (tile rows + 4 rows) must stay below 4 GiB
  const bool two = (sp == 2) && (!wide(g, elem_size(prec)) || wide_max_rows(g, elem_size(prec)) >= 3);
  const int pairs = two ? (nsteps / 2) & ~1 : 0;
  const int singles = nsteps - 2 * pairs;
  int64_t n = step0;
  int k = 0;   // launches so far: the input is fa when k is even
  lb_status s;
  for (int j = 0; j < singles; ++j, ++k, ++n)
    if ((s = launch_step(g, K, prec, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, n, t, st))) return s;
  for (int j = 0; j < pairs; ++j, ++k, n += 2)
    if ((s = launch_step2(g, K, prec, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, n, t, st))) return s;
  return LB_OK;
}

// The C ABI passes precisions as int32_t codes (any value a C caller may pass is
// then defined); a code becomes an lb_prec only after this check.
static lb_status check_prec(int32_t p) {
  if (p != LB_F64 && p != LB_F32) return fail(LB_EINVAL, "unknown precision");
  return LB_OK;
}

// ------------------------------------------------------------------ C ABI

extern "C" lb_status lb_init(const lb_grid* g, int32_t prec_code, const double* rho, const double* ux,
                             const double* uy, const double* p, void* f, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(f, "f"))) return s;
  if (!rho || !ux || !uy || !p) return fail(LB_EINVAL, "field pointer is NULL");
  KTConsts K;
  build_consts(g, &K);
  const dim3 grid((g->nx + 255) / 256, std::min(g->ny, 65535));
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_F64)
    hipLaunchKernelGGL(k_init<double>, grid, dim3(256), 0, st, K, rho, ux, uy, p, (double*)f);
  else
    hipLaunchKernelGGL(k_init<float>, grid, dim3(256), 0, st, K, rho, ux, uy, p, (float*)f);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

extern "C" lb_status lb_step_tiled(const lb_grid* g, int32_t prec_code, const void* fin, void* fout, int64_t step,
                                   const lb_tile* tile, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(fin, "f_in")) ||
      (s = check_ptr(fout, "f_out")))
    return s;
  const size_t bytes = (size_t)lb_array_elems(g) * elem_size(prec);
  if (overlap(fin, bytes, fout, bytes)) return fail(LB_EALIAS, "f_in and f_out overlap");
  Tile t;
  if ((s = resolve_tile(tile, g->nx, g->ny, &t))) return s;
  KTConsts K;
  build_consts(g, &K);
  return launch_step(g, K, prec, fin, fout, step, t, (hipStream_t)stream);
}

extern "C" lb_status lb_step(const lb_grid* g, int32_t prec_code, const void* fin, void* fout, int64_t step,
                             void* stream) {
  return lb_step_tiled(g, prec_code, fin, fout, step, nullptr, stream);
}

namespace {
// A captured step loop and an event recorded after its latest launch: an exec is
// destroyed only once that event has completed (a replay may still run on any
// stream when the cache evicts it).
struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // small LRU of captured step loops
}  // namespace

// Wait for the latest launch of exec (event `done`), then destroy both.
static void destroy_exec(hipGraphExec_t exec, hipEvent_t done) {
  if (done) {
    (void)hipEventSynchronize(done);
    (void)hipEventDestroy(done);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
}

static lb_status launch_exec(hipGraphExec_t exec, hipEvent_t done, hipStream_t st) {
  HIP_CHECK(hipGraphLaunch(exec, st));
  HIP_CHECK(hipEventRecord(done, st));
  return LB_OK;
}

static std::string run_key(const lb_grid* g, lb_prec prec, const void* fa, const void* fb, int64_t step0,
                           int nsteps, int bx, int rows, void* stream) {
  std::string k((const char*)g, sizeof(lb_grid));
  char buf[160];
  std::snprintf(buf, sizeof(buf), "|%d|%p|%p|%lld|%d|%d|%d|%p", (int)prec, fa, fb, (long long)step0, nsteps, bx,
                rows, stream);
  int dev = 0;
  (void)hipGetDevice(&dev);
  return k + buf + std::to_string(dev);
}

extern "C" lb_status lb_run(const lb_grid* g, int32_t prec_code, void* fa, void* fb, int64_t step0, int32_t nsteps,
                            int32_t use_graph, const lb_tile* tile, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(fa, "f_a")) || (s = check_ptr(fb, "f_b")))
    return s;
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  const size_t bytes = (size_t)lb_array_elems(g) * elem_size(prec);
  if (overlap(fa, bytes, fb, bytes)) return fail(LB_EALIAS, "f_a and f_b overlap");
  Tile t;
  if ((s = resolve_tile(tile, g->nx, g->ny, &t))) return s;
  KTConsts K;
  build_consts(g, &K);
  hipStream_t st = (hipStream_t)stream;
  if (!use_graph || st == nullptr || nsteps == 0) return launch_steps(g, K, prec, fa, fb, step0, nsteps, t, st);
  int sp;
  if ((s = pass_steps(g, prec, t, &sp))) return s;
  const std::string key =
      run_key(g, prec, fa, fb, step0, nsteps, t.bx, (t.rows * 1000003 + t.blocks) * 64 + sp, stream);
  std::lock_guard<std::mutex> lock(g_graph_mu);
  for (auto& e : g_graphs)
    if (e.key == key) return launch_exec(e.exec, e.done, st);
  HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const lb_status ls = launch_steps(g, K, prec, fa, fb, step0, nsteps, t, st);
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(st, &graph);
  if (ls != LB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return ls;
  }
  if (ce != hipSuccess) return fail(LB_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(LB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  hipEvent_t done = nullptr;
  const hipError_t ee = hipEventCreateWithFlags(&done, hipEventDisableTiming);
  if (ee != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    return fail(LB_EHIP, std::string("hipEventCreateWithFlags: ") + hipGetErrorString(ee));
  }
  if (g_graphs.size() >= 8) {
    destroy_exec(g_graphs.front().exec, g_graphs.front().done);
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back({key, exec, done});
  return launch_exec(exec, done, st);
}

extern "C" lb_status lb_moments(const lb_grid* g, int32_t prec_code, const void* f, double* rho, double* ux,
                                double* uy, double* T, uint32_t* flags, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(f, "f"))) return s;
  KTConsts K;
  build_consts(g, &K);
  hipStream_t st = (hipStream_t)stream;
  if (flags) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, flags, 4);
    HIP_CHECK(hipGetLastError());
  }
  const dim3 grid((g->nx + 255) / 256, std::min(g->ny, 65535));
  if (prec == LB_F64)
    hipLaunchKernelGGL(k_moments<double>, grid, dim3(256), 0, st, K, (const double*)f, rho, ux, uy, T, flags);
  else
    hipLaunchKernelGGL(k_moments<float>, grid, dim3(256), 0, st, K, (const float*)f, rho, ux, uy, T, flags);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

extern "C" lb_status lb_check_flags(const uint32_t* flags, uint32_t* host_flags, void* stream) {
  if (!flags) return fail(LB_EINVAL, "flags is NULL");
  uint32_t h[4] = {0u, 0u, 0u, 0u};
  hipStream_t st = (hipStream_t)stream;
  HIP_CHECK(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  if (host_flags) std::memcpy(host_flags, h, sizeof(h));
  if (h[0] & (LB_FLAG_NONFINITE | LB_FLAG_RHO_NONPOS)) {
    char buf[160];
    std::snprintf(buf, sizeof(buf), "blow-up: %u non-finite sites, %u sites with rho <= 0 (%u with T <= 0)", h[1],
                  h[2], h[3]);
    return fail(LB_ENONFINITE, buf);
  }
  return LB_OK;
}

// Partition of lb_invariants: nb blocks of rpb rows each (nb <= LBKT_INV_MAX_PARTS).
void lbkt_inv_partition(const lb_grid* g, int* rpb, int* nb) {
  const int nblk = std::min(g->ny, LBKT_INV_MAX_PARTS);
  *rpb = (int)cdiv(g->ny, nblk);
  *nb = (int)cdiv(g->ny, *rpb);
}

// Argument checks of lb_invariants (shared with its variant without allocation).
lb_status lbkt_invariants_args(const lb_grid* g, int32_t prec, const void* f, const double* out4) {
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(f, "f"))) return s;
  if (!out4) return fail(LB_EINVAL, "out4 is NULL");
  return LB_OK;
}

// The two kernels of lb_invariants over a partial-sum buffer of nb * 4 doubles.
lb_status lbkt_launch_invariants(const KTConsts& K, lb_prec prec, const void* f, int rpb, int nb, double* part,
                                 double* out4, hipStream_t st) {
  if (prec == LB_F64)
    hipLaunchKernelGGL(k_inv_partial<double>, dim3(nb), dim3(256), 0, st, K, (const double*)f, rpb, part);
  else
    hipLaunchKernelGGL(k_inv_partial<float>, dim3(nb), dim3(256), 0, st, K, (const float*)f, rpb, part);
  HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_inv_final, dim3(1), dim3(256), 0, st, (const double*)part, nb, out4);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

namespace {
// Per-device workspace of lb_invariants and an event recorded after the last
// kernel that read it: the next call, on whatever stream, waits for that event
// before its kernels write the buffer, and a buffer is freed only after it.
struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t last = nullptr;
};
std::mutex g_ws_mu;
std::map<int, Workspace> g_ws;
}  // namespace

extern "C" lb_status lb_invariants(const lb_grid* g, int32_t prec_code, const void* f, double* out4, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  lb_status s;
  if ((s = lbkt_invariants_args(g, prec, f, out4))) return s;
  KTConsts K;
  build_consts(g, &K);
  int rpb, nb;
  lbkt_inv_partition(g, &rpb, &nb);
  const size_t bytes = (size_t)nb * 4 * sizeof(double);
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  // the whole enqueue under the lock, so that calls from several threads order
  // their use of the buffer as they take the lock
  std::lock_guard<std::mutex> lock(g_ws_mu);
  Workspace& w = g_ws[dev];
  if (!w.last) HIP_CHECK(hipEventCreateWithFlags(&w.last, hipEventDisableTiming));
  if (w.bytes < bytes) {
    if (w.ptr) {
      HIP_CHECK(hipEventSynchronize(w.last));   // the previous call's kernels are done with it
      HIP_CHECK(hipFree(w.ptr));
    }
    w.ptr = nullptr;
    w.bytes = 0;
    if (hipMalloc(&w.ptr, bytes) != hipSuccess) return fail(LB_ENOMEM, "workspace allocation failed");
    w.bytes = bytes;
  } else {
    HIP_CHECK(hipStreamWaitEvent(st, w.last, 0));
  }
  if ((s = lbkt_launch_invariants(K, prec, f, rpb, nb, (double*)w.ptr, out4, st))) return s;
  HIP_CHECK(hipEventRecord(w.last, st));
  return LB_OK;
}

static lb_status launch_adjoint(const lb_grid* g, const KTConsts& K, lb_prec prec, const void* fn, const double* g1,
                                double* g0, hipStream_t st) {
  int bx, rows;
  // at least 512 tiles (not 1024): on the 960 x 240 grid 128 x 2 tiles run the
  // adjoint step in 13.7 us against 14.4-14.8 us for 64 x 2 (64 x 1, 64 x 4,
  // 128 x 1, 128 x 4, 256 x 1: 15.3-17.5 us)
  default_tile(g->nx, g->ny, &bx, &rows, 512);
  const bool w = wide(g, sizeof(double));   // the adjoint arrays are double
  rows = std::min(rows, g->ny);
  if (w) rows = std::min(rows, wide_max_rows(g, sizeof(double)));
  const int nstrips = (int)cdiv(g->nx, bx);
  const int64_t nblocks64 = (int64_t)nstrips * cdiv(g->ny, rows);
  if (nblocks64 > 0x7fffffff) return fail(LB_EINVAL, "grid too large for one launch");
  const int nblocks = (int)nblocks64;
  const int xcd_map = 0;   // raster order: 2-3% faster than the XCD bands on the 8192 x 2048 grid
  if (prec == LB_F64) {
    auto kern = w ? k_adjoint<double, true> : k_adjoint<double, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(bx), 0, st, K, (const double*)fn, g1, g0, rows, nstrips, nblocks,
                       xcd_map);
  } else {
    auto kern = w ? k_adjoint<float, true> : k_adjoint<float, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(bx), 0, st, K, (const float*)fn, g1, g0, rows, nstrips, nblocks,
                       xcd_map);
  }
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

extern "C" lb_status lb_step_adjoint(const lb_grid* g, int32_t prec_code, const void* fn, const double* g1, double* g0,
                                     int64_t step, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  (void)step;  // the step's dependence on t (SHOCK ghosts) does not involve f
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(fn, "f_n")) ||
      (s = check_ptr(g1, "g_np1")) || (s = check_ptr(g0, "g_n")))
    return s;
  const size_t gbytes = (size_t)lb_array_elems(g) * 8;
  if (overlap(g1, gbytes, g0, gbytes)) return fail(LB_EALIAS, "g_np1 and g_n overlap");
  KTConsts K;
  build_consts(g, &K);
  return launch_adjoint(g, K, prec, fn, g1, g0, (hipStream_t)stream);
}

extern "C" lb_status lb_adjoint_run(const lb_grid* g, int32_t prec_code, const void* const* f, double* gbuf,
                                    double* work, int64_t step0, int32_t nsteps, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  (void)step0;
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(gbuf, "g")) || (s = check_ptr(work, "work")))
    return s;
  if (nsteps < 0 || (nsteps > 0 && !f)) return fail(LB_EINVAL, "need nsteps >= 0 states");
  const size_t gbytes = (size_t)lb_array_elems(g) * 8;
  if (overlap(gbuf, gbytes, work, gbytes)) return fail(LB_EALIAS, "g and work overlap");
  for (int j = 0; j < nsteps; ++j)
    if ((s = check_ptr(f[j], "f[j]"))) return s;
  KTConsts K;
  build_consts(g, &K);
  hipStream_t st = (hipStream_t)stream;
  for (int k = 0; k < nsteps; ++k) {
    const int j = nsteps - 1 - k;
    const double* in = (k % 2 == 0) ? gbuf : work;
    double* out = (k % 2 == 0) ? work : gbuf;
    if ((s = launch_adjoint(g, K, prec, f[j], in, out, st))) return s;
  }
  return LB_OK;
}

extern "C" lb_status lb_run_record(const lb_grid* g, int32_t prec_code, const void* f0, void* const* out, int64_t step0,
                                   int32_t nsteps, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(f0, "f0"))) return s;
  if (nsteps < 0 || (nsteps > 0 && !out)) return fail(LB_EINVAL, "need nsteps >= 0 outputs");
  const size_t bytes = (size_t)lb_array_elems(g) * elem_size(prec);
  for (int j = 0; j < nsteps; ++j) {
    if ((s = check_ptr(out[j], "out[j]"))) return s;
    const void* in = (j == 0) ? f0 : out[j - 1];
    if (overlap(in, bytes, out[j], bytes)) return fail(LB_EALIAS, "consecutive states overlap");
  }
  Tile t;
  if ((s = resolve_tile(nullptr, g->nx, g->ny, &t))) return s;
  KTConsts K;
  build_consts(g, &K);
  hipStream_t st = (hipStream_t)stream;
  // two steps per pass (the first step's state stored on the way) where the
  // input and both outputs are distinct arrays, else one step per launch
  const bool two = (t.steps == 2) && !wide(g, elem_size(prec));
  for (int j = 0; j < nsteps;) {
    const void* in = (j == 0) ? f0 : out[j - 1];
    if (two && j + 1 < nsteps && !overlap(in, bytes, out[j + 1], bytes) && !overlap(out[j], bytes, out[j + 1], bytes)) {
      if ((s = launch_step2(g, K, prec, in, out[j + 1], step0 + j, t, st, out[j]))) return s;
      j += 2;
    } else {
      if ((s = launch_step(g, K, prec, in, out[j], step0 + j, t, st))) return s;
      j += 1;
    }
  }
  return LB_OK;
}

extern "C" lb_status lb_init_adjoint(const lb_grid* g, const double* rho, const double* ux, const double* uy,
                                     const double* p, const double* gf0, double* grho, void* stream) {
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_ptr(gf0, "g_f0"))) return s;
  if (!rho || !ux || !uy || !p || !grho) return fail(LB_EINVAL, "field pointer is NULL");
  KTConsts K;
  build_consts(g, &K);
  const dim3 grid((g->nx + 255) / 256, std::min(g->ny, 65535));
  hipLaunchKernelGGL(k_init_adjoint, grid, dim3(256), 0, (hipStream_t)stream, K, rho, ux, uy, p, gf0, grho);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// ------------------------------------------------------------------ batch

struct lb_batch {
  int nprob = 0;
  lb_prec prec = LB_F32;
  std::vector<lb_grid> grids;
  std::vector<int64_t> offsets, pitches;
  int64_t total = 0;
  int block_x = 256;
  int dev = 0;
  KTConsts* d_consts = nullptr;
  ProbInfo* d_info = nullptr;
  WorkItem* d_items = nullptr;
  int nitems = 0;
  WorkItem* d_items2 = nullptr;   // work list of the two-step kernel (60-column wavefronts)
  int nitems2 = 0;
  int steps = 2;                  // time steps per pass: 1, 2, or 4, 6, 8 (deep passes, below)
  bool all_ny4 = false;           // every problem has 4 rows and a periodic y axis
  WorkItem* d_itemsD = nullptr;   // work list of the deep passes (64 - 2 * steps columns per wavefront)
  int nitemsD = 0;
  int planned_bx = 0, planned_steps = 0;   // the launch shape the work lists were made for
  int64_t step = 0;
  // captured graph
  hipGraphExec_t exec = nullptr;
  void* g_fa = nullptr;
  void* g_fb = nullptr;
  int g_nsteps = -1;
  int g_bx = 0;
  int g_steps = 0;
  void* g_stream = nullptr;
  bool g_persist = false;
  int g_cap = 0;
  uint32_t g_spin = 0;
  hipEvent_t done = nullptr;   // recorded after each replay (the exec is destroyed after it)
  // persistent launch (all two-step passes in one launch of co-resident blocks)
  bool persist = false;
  int persist_cap = 0;            // at most this many blocks (and no more than are co-resident)
  uint32_t spin_limit = 1u << 20; // polls per wait before a block gives up
  int2* d_nbrs = nullptr;         // per two-step item: left and right neighbour item (-1: none)
  uint32_t* d_prog = nullptr;     // per block of the persistent launch: passes finished; then the stop word
  uint32_t* d_err = nullptr;      // failure word: set when a wait gave up, cleared by lb_batch_status
};

// Problems by decreasing site count, so that the tail of a launch is made of
// short items.
static std::vector<int> batch_order(const lb_grid* grids, int nprob) {
  std::vector<int> order(nprob);
  for (int p = 0; p < nprob; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return grids[a].nx * (int64_t)grids[a].ny > grids[c].nx * (int64_t)grids[c].ny;
  });
  return order;
}

// The strips of `width` output columns per wavefront, block_x / 64 wavefronts per
// item, of every problem in `order`, dealt to the XCDs (below).
static std::vector<WorkItem> batch_strips(const lb_grid* grids, const std::vector<int>& order, int block_x,
                                          int width) {
  std::vector<WorkItem> items2;
  const int wpb = block_x / 64;
  for (int p : order) {
    const int ns2 = (int)cdiv(cdiv(grids[p].nx, width), wpb);
    for (int s = 0; s < ns2; ++s) items2.push_back({p, s});
  }
  // The hardware deals block ids round-robin to the 8 XCDs. Within each span of
  // 8 x 16 items, XCD k gets the 16 consecutive items 16k .. 16k+15, so the
  // x-adjacent strips of a problem, which write the two parts of the cache line
  // at their common edge, mostly run on one XCD and meet in its L2 (a block of
  // 60-column strips ends inside a 128-byte line unless its width in bytes is a
  // multiple of 128). 2-4% faster per step than the plain order for 256
  // problems in float storage, 1% in double.
  {
    constexpr size_t run = 16, span = 8 * run;
    std::vector<WorkItem> dealt(items2.size());
    const size_t full = items2.size() / span * span;   // a partial last span keeps its order
    for (size_t k = 0; k < items2.size(); ++k) {
      const size_t j = k % span;
      dealt[k < full ? k - j + (j % run) * 8 + j / run : k] = items2[k];
    }
    items2.swap(dealt);
  }
  return items2;
}

void lbkt_plan_batch(const lb_grid* grids, int nprob, int block_x, std::vector<LbktWorkItem>* items_out,
                     std::vector<LbktWorkItem>* items2_out) {
  const std::vector<int> order = batch_order(grids, nprob);
  std::vector<WorkItem> items;
  for (int p : order) {
    const int ns = (grids[p].nx + block_x - 1) / block_x;
    for (int s = 0; s < ns; ++s) items.push_back({p, s});
  }
  std::vector<WorkItem> items2 = batch_strips(grids, order, block_x, 60);
  items_out->swap(items);
  items2_out->swap(items2);
}

void lbkt_plan_batch_deep(const lb_grid* grids, int nprob, int block_x, int depth,
                          std::vector<LbktWorkItem>* items_out) {
  std::vector<WorkItem> items = batch_strips(grids, batch_order(grids, nprob), block_x, 64 - 2 * depth);
  items_out->swap(items);
}

void lbkt_batch_neighbours(const lb_grid* grids, const std::vector<LbktWorkItem>& items2, int block_x,
                           std::vector<int>* left, std::vector<int>* right) {
  const int wpb = block_x / 64;
  std::map<std::pair<int, int>, int> at;
  for (size_t i = 0; i < items2.size(); ++i) at[{items2[i].prob, items2[i].strip}] = (int)i;
  left->assign(items2.size(), -1);
  right->assign(items2.size(), -1);
  for (size_t i = 0; i < items2.size(); ++i) {
    const lb_grid& g = grids[items2[i].prob];
    const int ns = (int)cdiv(cdiv(g.nx, 60), wpb);
    const bool perx = g.edge[0].kind == LB_BC_PERIODIC;
    const int s = items2[i].strip;
    const int l = s > 0 ? s - 1 : (perx ? ns - 1 : -1);
    const int r = s + 1 < ns ? s + 1 : (perx ? 0 : -1);
    if (l >= 0 && l != s) (*left)[i] = at[{items2[i].prob, l}];
    if (r >= 0 && r != s) (*right)[i] = at[{items2[i].prob, r}];
  }
}

static lb_status batch_items(lb_batch* b) {
  if (b->planned_bx == b->block_x && b->planned_steps == b->steps) return LB_OK;
  if (b->d_itemsD) HIP_CHECK(hipFree(b->d_itemsD));
  b->d_itemsD = nullptr;
  b->nitemsD = 0;
  if (b->steps > 2) {
    std::vector<WorkItem> itemsD;
    lbkt_plan_batch_deep(b->grids.data(), b->nprob, b->block_x, b->steps, &itemsD);
    HIP_CHECK(hipMalloc(&b->d_itemsD, itemsD.size() * sizeof(WorkItem)));
    HIP_CHECK(hipMemcpy(b->d_itemsD, itemsD.data(), itemsD.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    b->nitemsD = (int)itemsD.size();
  }
  if (b->planned_bx == b->block_x) {
    b->planned_steps = b->steps;
    return LB_OK;
  }
  std::vector<WorkItem> items, items2;
  lbkt_plan_batch(b->grids.data(), b->nprob, b->block_x, &items, &items2);
  std::vector<int> left, right;
  lbkt_batch_neighbours(b->grids.data(), items2, b->block_x, &left, &right);
  std::vector<int2> nb(items2.size());
  for (size_t i = 0; i < items2.size(); ++i) nb[i] = make_int2(left[i], right[i]);
  if (b->d_nbrs) HIP_CHECK(hipFree(b->d_nbrs));
  if (b->d_prog) HIP_CHECK(hipFree(b->d_prog));
  b->d_nbrs = nullptr;
  b->d_prog = nullptr;
  HIP_CHECK(hipMalloc(&b->d_nbrs, nb.size() * sizeof(int2)));
  HIP_CHECK(hipMemcpy(b->d_nbrs, nb.data(), nb.size() * sizeof(int2), hipMemcpyHostToDevice));
  HIP_CHECK(hipMalloc(&b->d_prog, (items2.size() + 1) * sizeof(uint32_t)));   // + the launch's stop word
  if (!b->d_err) {
    HIP_CHECK(hipMalloc(&b->d_err, sizeof(uint32_t)));
    HIP_CHECK(hipMemset(b->d_err, 0, sizeof(uint32_t)));
  }
  if (b->d_items) HIP_CHECK(hipFree(b->d_items));
  if (b->d_items2) HIP_CHECK(hipFree(b->d_items2));
  b->d_items = b->d_items2 = nullptr;
  HIP_CHECK(hipMalloc(&b->d_items, items.size() * sizeof(WorkItem)));
  HIP_CHECK(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  HIP_CHECK(hipMalloc(&b->d_items2, items2.size() * sizeof(WorkItem)));
  HIP_CHECK(hipMemcpy(b->d_items2, items2.data(), items2.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  b->nitems = (int)items.size();
  b->nitems2 = (int)items2.size();
  b->planned_bx = b->block_x;
  b->planned_steps = b->steps;
  return LB_OK;
}

// Steps per pass of the per-pass launches by default: two, or one when some
// problem has ny < 2; for a batch of 4-row y-periodic problems, 4 in float and 8
// in double storage. On the 256 Riemann problems (2000 steps, 64-thread items)
// float storage takes 36.3 ms at two steps per pass, 32.1 / 33.5 / 32.8 ms at
// 4 / 6 / 8; double storage 62.5 ms at two, 33.3 / 31.5 / 30.7 ms at 4 / 6 / 8.
static int batch_default_steps(const lb_batch* b) {
  for (const lb_grid& g : b->grids)
    if (g.ny < 2) return 1;
  if (!b->all_ny4) return 2;
  return b->prec == LB_F64 ? 8 : 4;
}

extern "C" lb_status lb_batch_create(int32_t nprob, const lb_grid* grids, int32_t prec_code, lb_batch** out) {
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  if (nprob < 1 || !grids) return fail(LB_EINVAL, "need nprob >= 1 grids");
  lb_status s;
  if ((s = check_prec(prec_code))) return s;
  const lb_prec prec = (lb_prec)prec_code;
  lb_batch* b = new (std::nothrow) lb_batch();
  if (!b) return fail(LB_ENOMEM, "batch allocation failed");
  b->nprob = nprob;
  b->prec = prec;
  b->grids.assign(grids, grids + nprob);
  int64_t off = 0;
  std::vector<KTConsts> ks(nprob);
  std::vector<ProbInfo> info(nprob);
  for (int p = 0; p < nprob; ++p) {
    lb_grid& g = b->grids[p];
    g.pitch = ((int64_t)g.nx + 63) / 64 * 64;
    if ((s = lb_validate(&g))) {
      delete b;
      return fail(s, "problem " + std::to_string(p) + ": " + g_last_error);
    }
    if (wide(&g, elem_size(prec))) {
      delete b;
      return fail(LB_EUNSUPPORTED, "problem " + std::to_string(p) + ": a batched problem's array must stay below 4 GiB");
    }
    for (int e = 0; e < 4; ++e)
      if (g.edge[e].kind == LB_BC_SHOCK) {
        delete b;
        return fail(LB_EUNSUPPORTED, "batched problems cannot have SHOCK edges");
      }
    b->offsets.push_back(off);
    b->pitches.push_back(g.pitch);
    info[p].offset = off;
    build_consts(&g, &ks[p]);
    off += lb_array_elems(&g);
  }
  b->total = off;
  (void)hipGetDevice(&b->dev);
  if (hipMalloc(&b->d_consts, sizeof(KTConsts) * nprob) != hipSuccess ||
      hipMalloc(&b->d_info, sizeof(ProbInfo) * nprob) != hipSuccess) {
    lb_batch_destroy(b);
    return fail(LB_ENOMEM, "batch metadata allocation failed");
  }
  if (hipMemcpy(b->d_consts, ks.data(), sizeof(KTConsts) * nprob, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_info, info.data(), sizeof(ProbInfo) * nprob, hipMemcpyHostToDevice) != hipSuccess) {
    lb_batch_destroy(b);
    return fail(LB_EHIP, "batch metadata upload failed");
  }
  b->all_ny4 = true;
  for (int p = 0; p < b->nprob; ++p)
    b->all_ny4 = b->all_ny4 && b->grids[p].ny == 4 && b->grids[p].edge[2].kind == LB_BC_PERIODIC;
  b->steps = batch_default_steps(b);
  // FP32 batches of 4-row y-periodic problems: width 64, a strip's rows on four
  // wavefronts in the deep passes (k_stepD_batched_ny4_rows)
  if (b->prec == LB_F32 && b->all_ny4) b->block_x = 64;
  if ((s = batch_items(b))) {
    lb_batch_destroy(b);
    return s;
  }
  *out = b;
  return LB_OK;
}

extern "C" lb_status lb_batch_layout(const lb_batch* b, int64_t* offsets, int64_t* pitches, int64_t* total) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (offsets) std::copy(b->offsets.begin(), b->offsets.end(), offsets);
  if (pitches) std::copy(b->pitches.begin(), b->pitches.end(), pitches);
  if (total) *total = b->total;
  return LB_OK;
}

extern "C" lb_status lb_batch_set_tile(lb_batch* b, const lb_tile* tile) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  int bx = 256;
  if (tile && tile->block_x) bx = tile->block_x;
  if (bx != 64 && bx != 128 && bx != 256) return fail(LB_EINVAL, "tile block_x must be 64, 128 or 256");
  const int sp = tile ? tile->steps : 0;
  if (!(sp == 0 || sp == 1 || sp == 2 || sp == 4 || sp == 6 || sp == 8))
    return fail(LB_EINVAL, "tile steps must be 0, 1, 2, 4, 6 or 8");
  if (tile && (tile->blocks < 0 || tile->rows < 0)) return fail(LB_EINVAL, "tile blocks and rows must be >= 0");
  const bool persist = tile && tile->blocks > 0;
  if (sp > 2 && !b->all_ny4)
    return fail(LB_EINVAL, "more than two steps per pass needs a batch of 4-row problems with a periodic y axis");
  if (sp > 2 && persist) return fail(LB_EINVAL, "the persistent launch runs two steps per pass");
  const int def = batch_default_steps(b);
  b->steps = (def == 1 || sp == 1) ? 1 : sp != 0 ? sp : persist ? 2 : def;
  b->persist = persist;
  b->persist_cap = tile ? tile->blocks : 0;
  b->spin_limit = (tile && tile->rows > 0) ? (uint32_t)tile->rows : (1u << 20);
  b->block_x = bx;
  return batch_items(b);
}

static lb_status launch_batched(lb_batch* b, const void* fin, void* fout, hipStream_t st) {
  if (b->prec == LB_F64)
    hipLaunchKernelGGL(k_step_batched<double>, dim3(b->nitems), dim3(b->block_x), 0, st, b->d_consts, b->d_info,
                       b->d_items, (const double*)fin, (double*)fout);
  else
    hipLaunchKernelGGL(k_step_batched<float>, dim3(b->nitems), dim3(b->block_x), 0, st, b->d_consts, b->d_info,
                       b->d_items, (const float*)fin, (float*)fout);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

static lb_status launch_batched2(lb_batch* b, const void* fin, void* fout, hipStream_t st) {
  if (b->prec == LB_F64) {
    auto kern = b->all_ny4 ? k_step2_batched<double, true> : k_step2_batched<double, false>;
    hipLaunchKernelGGL(kern, dim3(b->nitems2), dim3(b->block_x), 0, st, b->d_consts, b->d_info, b->d_items2,
                       (const double*)fin, (double*)fout);
  } else {
    auto kern = b->all_ny4 ? k_step2_batched<float, true> : k_step2_batched<float, false>;
    hipLaunchKernelGGL(kern, dim3(b->nitems2), dim3(b->block_x), 0, st, b->d_consts, b->d_info, b->d_items2,
                       (const float*)fin, (float*)fout);
  }
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// One pass of b->steps (4, 6 or 8) steps of a batch of 4-row y-periodic problems.
static lb_status launch_batchedD(lb_batch* b, const void* fin, void* fout, hipStream_t st) {
  using KD = void (*)(const KTConsts*, const ProbInfo*, const WorkItem*, const double*, double*);
  using KF = void (*)(const KTConsts*, const ProbInfo*, const WorkItem*, const float*, float*);
  KD kd = nullptr;
  KF kf = nullptr;
  switch (b->steps) {
    case 4: kd = k_stepD_batched_ny4<double, 4>; kf = k_stepD_batched_ny4<float, 4>; break;
    case 6: kd = k_stepD_batched_ny4<double, 6>; kf = k_stepD_batched_ny4<float, 6>; break;
    case 8: kd = k_stepD_batched_ny4<double, 8>; kf = k_stepD_batched_ny4<float, 8>; break;
    default: return fail(LB_EINVAL, "no deep batched kernel for this step count");
  }
  if (b->prec == LB_F32 && b->block_x == 64) {
    // float storage at width 64: a strip's four rows on four wavefronts
    KF rf = b->steps == 4 ? k_stepD_batched_ny4_rows<float, 4>
                          : b->steps == 6 ? k_stepD_batched_ny4_rows<float, 6> : k_stepD_batched_ny4_rows<float, 8>;
    hipLaunchKernelGGL(rf, dim3(b->nitemsD), dim3(256), 0, st, b->d_consts, b->d_info, b->d_itemsD,
                       (const float*)fin, (float*)fout);
    HIP_CHECK(hipGetLastError());
    return LB_OK;
  }
  if (b->prec == LB_F64)
    hipLaunchKernelGGL(kd, dim3(b->nitemsD), dim3(b->block_x), 0, st, b->d_consts, b->d_info, b->d_itemsD,
                       (const double*)fin, (double*)fout);
  else
    hipLaunchKernelGGL(kf, dim3(b->nitemsD), dim3(b->block_x), 0, st, b->d_consts, b->d_info, b->d_itemsD,
                       (const float*)fin, (float*)fout);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// All `passes` two-step passes from fa (passes even: the result lands in fa) in one
// launch of co-resident blocks, after clearing the progress counters.
template <typename S>
static lb_status launch_batched2_persistent(lb_batch* b, void* fa, void* fb, int passes, hipStream_t st) {
  auto kern = b->all_ny4 ? k_step2_batched_persistent<S, true> : k_step2_batched_persistent<S, false>;
  int per_cu = 0, ncu = 0;
  HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, b->block_x, 0));
  HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->dev));
  int64_t g = std::min<int64_t>((int64_t)per_cu * ncu, b->nitems2);
  if (b->persist_cap > 0) g = std::min<int64_t>(g, b->persist_cap);
  if (g >= 8) g &= ~(int64_t)7;   // blocks dealt to the 8 XCDs as the items were planned
  if (g < 1) return fail(LB_EHIP, "no block of the persistent batched kernel fits on a compute unit");
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)cdiv(b->nitems2 + 1, 256)), dim3(256), 0, st, b->d_prog,
                     b->nitems2 + 1, 0u);
  HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(b->block_x), 0, st, b->d_consts, b->d_info, b->d_items2,
                     (const int2*)b->d_nbrs, b->nitems2, (S*)fa, (S*)fb, passes, b->d_prog, b->d_err, b->spin_limit);
  HIP_CHECK(hipGetLastError());
  return LB_OK;
}

// nsteps steps of the batch from fa (result in fa when nsteps is even): as
// launch_steps, an even number of two-step passes after 0..3 single steps; the
// passes in one persistent launch when asked for. With deep passes (D = 4, 6, 8
// steps each) an even number of them follows, and the two-step passes and single
// steps cover the rest (fewer than 2D steps). Every pass swaps the buffers, and
// all three counts are even for even nsteps.
static lb_status batched_steps(lb_batch* b, void* fa, void* fb, int nsteps, hipStream_t st) {
  const int D = b->steps;
  const int deep = (D > 2) ? (nsteps / D) & ~1 : 0;
  const int rest = nsteps - D * deep;
  const int pairs = (D >= 2) ? (rest / 2) & ~1 : 0;
  const int singles = rest - 2 * pairs;
  int k = 0;
  lb_status s;
  for (int j = 0; j < singles; ++j, ++k)
    if ((s = launch_batched(b, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, st))) return s;
  if (b->persist && pairs > 0) {
    void* a = (k % 2 == 0) ? fa : fb;
    void* c = (k % 2 == 0) ? fb : fa;
    return b->prec == LB_F64 ? launch_batched2_persistent<double>(b, a, c, pairs, st)
                             : launch_batched2_persistent<float>(b, a, c, pairs, st);
  }
  for (int j = 0; j < pairs; ++j, ++k)
    if ((s = launch_batched2(b, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, st))) return s;
  for (int j = 0; j < deep; ++j, ++k)
    if ((s = launch_batchedD(b, (k % 2 == 0) ? fa : fb, (k % 2 == 0) ? fb : fa, st))) return s;
  return LB_OK;
}

extern "C" lb_status lb_step_batched(lb_batch* b, void* fa, void* fb, int32_t nsteps, void* stream) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  lb_status s;
  if ((s = check_ptr(fa, "f_a")) || (s = check_ptr(fb, "f_b"))) return s;
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  const size_t bytes = (size_t)b->total * elem_size(b->prec);
  if (overlap(fa, bytes, fb, bytes)) return fail(LB_EALIAS, "f_a and f_b overlap");
  hipStream_t st = (hipStream_t)stream;
  if (nsteps == 0) return LB_OK;
  if (st == nullptr) {
    if ((s = batched_steps(b, fa, fb, nsteps, st))) return s;
    b->step += nsteps;
    return LB_OK;
  }
  if (!b->done) HIP_CHECK(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
  if (!(b->exec && b->g_fa == fa && b->g_fb == fb && b->g_nsteps == nsteps && b->g_bx == b->block_x &&
        b->g_steps == b->steps && b->g_stream == stream && b->g_persist == b->persist &&
        b->g_cap == b->persist_cap && b->g_spin == b->spin_limit)) {
    if (b->exec) {
      HIP_CHECK(hipEventSynchronize(b->done));   // its last replay may still run, on any stream
      HIP_CHECK(hipGraphExecDestroy(b->exec));
    }
    b->exec = nullptr;
    HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const lb_status ls = batched_steps(b, fa, fb, nsteps, st);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (ls != LB_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return ls;
    }
    if (ce != hipSuccess) return fail(LB_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(LB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    b->g_fa = fa;
    b->g_fb = fb;
    b->g_nsteps = nsteps;
    b->g_bx = b->block_x;
    b->g_steps = b->steps;
    b->g_stream = stream;
    b->g_persist = b->persist;
    b->g_cap = b->persist_cap;
    b->g_spin = b->spin_limit;
  }
  HIP_CHECK(hipGraphLaunch(b->exec, st));
  HIP_CHECK(hipEventRecord(b->done, st));
  b->step += nsteps;
  return LB_OK;
}

extern "C" void lb_batch_destroy(lb_batch* b) {
  if (!b) return;
  if (b->done) {
    (void)hipEventSynchronize(b->done);
    (void)hipEventDestroy(b->done);
  }
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->d_consts) (void)hipFree(b->d_consts);
  if (b->d_info) (void)hipFree(b->d_info);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_items2) (void)hipFree(b->d_items2);
  if (b->d_itemsD) (void)hipFree(b->d_itemsD);
  if (b->d_nbrs) (void)hipFree(b->d_nbrs);
  if (b->d_prog) (void)hipFree(b->d_prog);
  if (b->d_err) (void)hipFree(b->d_err);
  delete b;
}

extern "C" lb_status lb_batch_status(lb_batch* b, void* stream) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (!b->d_err) return LB_OK;
  hipStream_t st = (hipStream_t)stream;
  uint32_t e = 0;
  HIP_CHECK(hipStreamSynchronize(st));
  HIP_CHECK(hipMemcpy(&e, b->d_err, sizeof(e), hipMemcpyDeviceToHost));
  if (e) {
    HIP_CHECK(hipMemset(b->d_err, 0, sizeof(uint32_t)));
    return fail(LB_EHIP, "a persistent batched launch gave up waiting for a neighbouring strip (its blocks were not "
                         "all resident, or the poll budget was too small); the result is incomplete");
  }
  return LB_OK;
}

// ------------------------------------------------------------------ autotuner

extern "C" lb_status lb_autotune(const lb_grid* g, int32_t prec_code, void* fa, void* fb, int32_t reps, lb_tile* best,
                                 float* best_ms, void* stream) {
  if (check_prec(prec_code)) return LB_EINVAL;
  const lb_prec prec = (lb_prec)prec_code;
  lb_status s;
  if ((s = lb_validate(g)) || (s = check_prec(prec)) || (s = check_ptr(fa, "f_a")) || (s = check_ptr(fb, "f_b")))
    return s;
  if (!best) return fail(LB_EINVAL, "best is NULL");
  if (reps < 1) reps = 1;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  const int bxs[3] = {64, 128, 256};
  const int rws[9] = {1, 2, 4, 8, 12, 16, 24, 32, 64};
  const int nbs[3] = {0, 1024, 2048};
  float bestv = 1e30f;
  lb_tile bt = {256, 16, 0, 0};
  KTConsts K;
  build_consts(g, &K);
  // ms per launch of `launch` (in, out) -> lb_status: a warm-up launch, then reps
  // timed launches, on a stream captured in a graph and timed as one replay (as
  // lb_run with use_graph runs them; on small grids the gaps between direct
  // launches would dominate)
  auto time_launches = [&](auto&& launch, float* ms) -> lb_status {
    lb_status ls = launch(fa, fb);
    if (ls) return ls;
    if (st != nullptr) {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(LB_EHIP, "stream capture");
      for (int n = 0; n < reps && ls == LB_OK; ++n) ls = launch((n % 2 == 0) ? fb : fa, (n % 2 == 0) ? fa : fb);
      const hipError_t ce = hipStreamEndCapture(st, &graph);
      if (ls != LB_OK || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return ls != LB_OK ? ls : fail(LB_EHIP, "stream capture");
      }
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return fail(LB_EHIP, "graph instantiate");
      hipError_t le = hipGraphLaunch(exec, st);   // warm replay
      if (le == hipSuccess) le = hipEventRecord(e0, st);
      if (le == hipSuccess) le = hipGraphLaunch(exec, st);
      if (le == hipSuccess) le = hipEventRecord(e1, st);
      if (le == hipSuccess) le = hipEventSynchronize(e1);
      (void)hipGraphExecDestroy(exec);
      if (le != hipSuccess) return fail(LB_EHIP, "graph replay");
    } else {
      if (hipEventRecord(e0, st) != hipSuccess) return fail(LB_EHIP, "event record");
      for (int n = 0; n < reps; ++n)
        if ((ls = launch((n % 2 == 0) ? fb : fa, (n % 2 == 0) ? fa : fb))) return ls;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(LB_EHIP, "event sync");
    }
    *ms = 0.f;
    (void)hipEventElapsedTime(ms, e0, e1);
    *ms /= (float)reps;
    return LB_OK;
  };
  // every kernel lb_run can use: one step per launch, two per pass (ny >= 2), and
  // three per pass (FP64 arrays below 4 GiB, ny >= 3)
  const int spmax = three_ok(g, prec) ? 3 : (g->ny >= 2 ? 2 : 1);
  for (int sp = 1; sp <= spmax; ++sp)
    for (int bi = 0; bi < 3; ++bi)
      for (int ri = 0; ri < 9; ++ri)
        for (int ni = 0; ni < 3; ++ni) {
          const int bx = bxs[bi], rows = std::min(rws[ri], g->ny);
          if (ri > 0 && rows == std::min(rws[ri - 1], g->ny)) continue;
          const Tile t = {bx, rows, nbs[ni], sp, true, false};
          auto launch = [&](const void* in, void* out) {
            return sp == 1   ? launch_step(g, K, prec, in, out, 0, t, st)
                   : sp == 2 ? launch_step2(g, K, prec, in, out, 0, t, st)
                             : launch_step3(g, K, in, out, 0, t, st);
          };
          float ms;
          if ((s = time_launches(launch, &ms))) goto done;
          ms /= (float)sp;   // per time step
          if (ms < bestv) {
            bestv = ms;
            bt.block_x = bx;
            bt.rows = rows;
            bt.blocks = nbs[ni];
            bt.steps = sp;
          }
        }
  // the deep pass of 4-row grids with a periodic y axis (lb_run's default there,
  // whatever the tile): steps = 0 in the result selects it
  if (deep1_ok(g, prec)) {
    auto launch = [&](const void* in, void* out) { return launch_stepD1(g, K, prec, in, out, st); };
    float ms;
    if ((s = time_launches(launch, &ms))) goto done;
    ms /= (float)LB_DEEP1;
    if (ms < bestv) {
      bestv = ms;
      default_tile(g->nx, g->ny, &bt.block_x, &bt.rows);
      bt.rows = std::min(bt.rows, g->ny);
      bt.blocks = 0;
      bt.steps = 0;
    }
  }
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) return s;
  *best = bt;
  if (best_ms) *best_ms = bestv;
  return LB_OK;
}

extern "C" int64_t lb_struct_size(int32_t which) {
  switch (which) {
    case 0: return (int64_t)sizeof(lb_grid);
    case 1: return (int64_t)sizeof(lb_edge);
    case 2: return (int64_t)sizeof(lb_state);
    case 3: return (int64_t)sizeof(lb_tile);
    case 4: return (int64_t)sizeof(lb_vn_case);
  }
  return -1;
}

extern "C" const char* lb_status_str(int32_t s) {
  switch (s) {
    case LB_OK: return "LB_OK";
    case LB_EINVAL: return "LB_EINVAL";
    case LB_EPARAM: return "LB_EPARAM";
    case LB_EALIAS: return "LB_EALIAS";
    case LB_ENONFINITE: return "LB_ENONFINITE";
    case LB_EHIP: return "LB_EHIP";
    case LB_ENOMEM: return "LB_ENOMEM";
    case LB_EUNSUPPORTED: return "LB_EUNSUPPORTED";
  }
  return "LB_?";
}

extern "C" const char* lb_last_error(void) { return g_last_error.c_str(); }
