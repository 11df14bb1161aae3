// von Neumann scan of the step on gfx950 (C ABI declared in include/lbkt.h).
//
// Sec. 3 of the paper: about a uniform equilibrium, one step multiplies a
// Fourier mode of the 9 distributions by the matrix
//     G(k) = diag(s_i(k)) + (1/tau) d f^eq / d f                  (SEC-VON-8/9/12)
// with s_i(k) the Fourier symbol of the linear part of the step for plane i.
// One thread evaluates one (case, k): it forms G from the step's own stencil
// coefficients (kt_site.hpp) and the analytic collision Jacobian (the same
// routine the adjoint kernels use), reduces G to upper Hessenberg form with
// Householder reflections and finds all eigenvalues by single-shift QR with
// Wilkinson shifts, deflating from the bottom. Every loop has a compile-time
// trip count and is unrolled, so the matrix lives in registers; the recursion
// over the active size is a template. The work is a dense 9x9 complex
// eigenproblem per point: FP64 VALU arithmetic, no memory traffic to speak of.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbkt.h"
#include "kt_site.hpp"
#include "lbkt_internal.hpp"

using namespace lbkt;

namespace {

constexpr int NV = 9;
constexpr double EPS = 2.220446049250313e-16;   // unit roundoff of float64 (2^-52)
constexpr int MAX_IT = 60;                       // QR iterations allowed per eigenvalue

struct Cx {
  double re, im;
};

__host__ __device__ __forceinline__ Cx cx(double r, double i) { return Cx{r, i}; }
__host__ __device__ __forceinline__ Cx operator+(Cx a, Cx b) { return cx(a.re + b.re, a.im + b.im); }
__host__ __device__ __forceinline__ Cx operator-(Cx a, Cx b) { return cx(a.re - b.re, a.im - b.im); }
__host__ __device__ __forceinline__ Cx operator*(Cx a, Cx b) {
  return cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__host__ __device__ __forceinline__ Cx operator*(double s, Cx a) { return cx(s * a.re, s * a.im); }
__host__ __device__ __forceinline__ Cx conj(Cx a) { return cx(a.re, -a.im); }
__host__ __device__ __forceinline__ double norm2(Cx a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ __forceinline__ double cabs(Cx a) { return hypot(a.re, a.im); }
__host__ __device__ __forceinline__ double abs1(Cx a) { return fabs(a.re) + fabs(a.im); }

// Principal square root, computed without cancellation.
__host__ __device__ __forceinline__ Cx csqrt(Cx z) {
  const double r = cabs(z);
  if (r == 0.0) return cx(0.0, 0.0);
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (r + z.re));
    return cx(t, z.im / (2.0 * t));
  }
  const double t = sqrt(0.5 * (r - z.re));
  return cx(fabs(z.im) / (2.0 * t), copysign(t, z.im));
}

// In-place reduction of H to upper Hessenberg form by Householder reflections
// P = I - 2 v v^H / |v|^2 acting on rows/columns k+1 .. N-1 (similarity, so the
// eigenvalues are unchanged). Entries below the subdiagonal are set to zero.
template <int N>
__host__ __device__ __forceinline__ void hessenberg(Cx (&H)[N][N]) {
#pragma unroll
  for (int k = 0; k < N - 2; ++k) {
    double xn2 = 0.0;
#pragma unroll
    for (int i = k + 1; i < N; ++i) xn2 += norm2(H[i][k]);
    const Cx x0 = H[k + 1][k];
    const double tail = xn2 - norm2(x0);
    if (tail > 0.0) {
      const double xnorm = sqrt(xn2);
      const double a0 = cabs(x0);
      const Cx ph = (a0 > 0.0) ? cx(x0.re / a0, x0.im / a0) : cx(1.0, 0.0);
      const Cx alpha = cx(-ph.re * xnorm, -ph.im * xnorm);   // P x = alpha e_1
      Cx v[N];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = cx(0.0, 0.0);
      v[k + 1] = x0 - alpha;
#pragma unroll
      for (int i = k + 2; i < N; ++i) v[i] = H[i][k];
      const double f = 2.0 / (norm2(v[k + 1]) + tail);
      // left: rows k+1.. of columns k+1.. (column k is set below)
#pragma unroll
      for (int j = k + 1; j < N; ++j) {
        Cx w = cx(0.0, 0.0);
#pragma unroll
        for (int i = k + 1; i < N; ++i) w = w + conj(v[i]) * H[i][j];
        w = f * w;
#pragma unroll
        for (int i = k + 1; i < N; ++i) H[i][j] = H[i][j] - v[i] * w;
      }
      // right: columns k+1.. of every row
#pragma unroll
      for (int i = 0; i < N; ++i) {
        Cx w = cx(0.0, 0.0);
#pragma unroll
        for (int l = k + 1; l < N; ++l) w = w + H[i][l] * v[l];
        w = f * w;
#pragma unroll
        for (int l = k + 1; l < N; ++l) H[i][l] = H[i][l] - w * conj(v[l]);
      }
      H[k + 1][k] = alpha;
    }
#pragma unroll
    for (int i = k + 2; i < N; ++i) H[i][k] = cx(0.0, 0.0);
  }
}

// Rotation G = [[c, s], [-conj(s), c]] (c real) with G [a; b] = [r; 0].
__host__ __device__ __forceinline__ void givens(Cx a, Cx b, double* c, Cx* s) {
  const double na = cabs(a), nb = cabs(b);
  if (nb == 0.0) {
    *c = 1.0;
    *s = cx(0.0, 0.0);
  } else if (na == 0.0) {
    *c = 0.0;
    *s = cx(1.0, 0.0);
  } else {
    const double rho = hypot(na, nb);
    *c = na / rho;
    const Cx ph = cx(a.re / na, a.im / na);
    *s = (1.0 / rho) * (ph * conj(b));
  }
}

// One explicit single-shift QR step on the leading n x n block of the
// Hessenberg matrix H: H - mu I = Q R, H <- R Q + mu I.
template <int n, int N>
__host__ __device__ __forceinline__ void qr_step(Cx (&H)[N][N], Cx mu) {
  double c[n];
  Cx s[n];
#pragma unroll
  for (int i = 0; i < n; ++i) H[i][i] = H[i][i] - mu;
#pragma unroll
  for (int k = 0; k < n - 1; ++k) {
    givens(H[k][k], H[k + 1][k], &c[k], &s[k]);
#pragma unroll
    for (int j = k; j < n; ++j) {
      const Cx t1 = H[k][j], t2 = H[k + 1][j];
      H[k][j] = c[k] * t1 + s[k] * t2;
      H[k + 1][j] = c[k] * t2 - conj(s[k]) * t1;
    }
    H[k + 1][k] = cx(0.0, 0.0);
  }
#pragma unroll
  for (int k = 0; k < n - 1; ++k) {
#pragma unroll
    for (int i = 0; i < n && i <= k + 1; ++i) {
      const Cx t1 = H[i][k], t2 = H[i][k + 1];
      H[i][k] = c[k] * t1 + conj(s[k]) * t2;
      H[i][k + 1] = c[k] * t2 - s[k] * t1;
    }
  }
#pragma unroll
  for (int i = 0; i < n; ++i) H[i][i] = H[i][i] + mu;
}

// Eigenvalue of the trailing 2x2 block [[a, b], [c, d]] nearer to d.
__host__ __device__ __forceinline__ Cx wilkinson(Cx a, Cx b, Cx c, Cx d) {
  const Cx h = 0.5 * (a - d);
  const Cx r = csqrt(h * h + b * c);
  const Cx m = 0.5 * (a + d);
  const Cx l1 = m + r, l2 = m - r;
  return (norm2(l1 - d) <= norm2(l2 - d)) ? l1 : l2;
}

// Deflation from the bottom: iterate on the leading n x n block until its last
// subdiagonal entry is negligible against the matrix norm (a backward-stable
// criterion), record |H[n-1][n-1]|, continue with n - 1.
template <int n, int N>
struct Qr {
  __host__ __device__ static __forceinline__ void run(Cx (&H)[N][N], double hnorm, double* rad, bool* ok) {
    int it = 0;
    for (; it < MAX_IT; ++it) {
      const double sub = abs1(H[n - 1][n - 2]);
      if (sub <= EPS * hnorm) break;
      Cx mu = wilkinson(H[n - 2][n - 2], H[n - 2][n - 1], H[n - 1][n - 2], H[n - 1][n - 1]);
      if (it == 10 || it == 20 || it == 30 || it == 40) mu = H[n - 1][n - 1] + cx(0.75 * sub, 0.0);   // exceptional
      qr_step<n, N>(H, mu);
    }
    if (it == MAX_IT) *ok = false;
    *rad = fmax(*rad, cabs(H[n - 1][n - 1]));
    Qr<n - 1, N>::run(H, hnorm, rad, ok);
  }
};
template <int N>
struct Qr<1, N> {
  __host__ __device__ static __forceinline__ void run(Cx (&H)[N][N], double, double* rad, bool*) {
    *rad = fmax(*rad, cabs(H[0][0]));
  }
};

// Spectral radius of H (destroyed); NaN if the iteration did not converge.
template <int N>
__host__ __device__ __forceinline__ double spectral_radius(Cx (&H)[N][N]) {
  hessenberg<N>(H);
  double hnorm = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = (i > 0 ? i - 1 : 0); j < N; ++j) hnorm = fmax(hnorm, abs1(H[i][j]));
  double rad = 0.0;
  bool ok = true;
  Qr<N, N>::run(H, hnorm, &rad, &ok);
  return ok ? rad : NAN;
}

// A scan case as the kernel sees it: the step's constants and the state.
struct VnCase {
  KTConsts K;
  double rho, ux, uy, T;
};

// G(k) for one case: the Fourier symbol of plane i's stencil on the diagonal,
// s_i = W0 + W1 e^{i kx} + W2 e^{-i kx} + W3 e^{i ky} + W4 e^{-i ky} with W_k the
// coefficients of the centre, x+dx, x-dx, y+dy, y-dy neighbours, plus (1/tau)
// times the collision Jacobian, row i = the collision adjoint of the unit vector e_i.
__host__ __device__ __forceinline__ void amplification(const VnCase& C, double kx, double ky, Cx (&G)[NV][NV]) {
  const KTConsts& K = C.K;
  Prim P;
  P.rho = C.rho;
  P.ux = C.ux;
  P.uy = C.uy;
  P.T = C.T;
  P.rinv = 1.0 / C.rho;
  P.usq = C.ux * C.ux + C.uy * C.uy;
  double sx, cxk, sy, cyk;
  sincos(kx, &sx, &cxk);
  sincos(ky, &sy, &cyk);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double e[NV], row[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) e[j] = (i == j) ? 1.0 : 0.0;
    collision_adjoint(K, P, e, row);   // row[j] = (1/tau) d f_i^eq / d f_j
#pragma unroll
    for (int j = 0; j < NV; ++j) G[i][j] = cx(row[j], 0.0);
    const double w0 = wcoef(K, i, 0), w1 = wcoef(K, i, 1), w2 = wcoef(K, i, 2);
    const double w3 = wcoef(K, i, 3), w4 = wcoef(K, i, 4);
    const double re = w0 + (w1 + w2) * cxk + (w3 + w4) * cyk;
    const double im = (w1 - w2) * sx + (w3 - w4) * sy;
    G[i][i] = G[i][i] + cx(re, im);
  }
}

__global__ __launch_bounds__(64) void k_vn_scan(const VnCase* __restrict__ cases, int ncases,
                                                const double* __restrict__ kdx, const double* __restrict__ kdy,
                                                int nk, int reduce, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ncases * nk) return;
  const int c = (int)(t / nk), q = (int)(t % nk);
  Cx G[NV][NV];
  amplification(cases[c], kdx[q], kdy[q], G);
  const double r = spectral_radius<NV>(G);
  if (reduce) {
    // non-negative doubles order like their bit patterns; NaN (0x7ff8...) wins
    atomicMax(reinterpret_cast<unsigned long long*>(out + c), (unsigned long long)__double_as_longlong(r));
  } else {
    out[t] = r;
  }
}

__global__ void k_vn_zero(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

lb_status hip_fail(const char* what, hipError_t e) {
  return lbkt_fail(LB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Host-side checks and constants of every case; dts (if given) overrides dt,
// case c * ndt + j taking dts[c * ndt + j].
lb_status prepare(const lb_vn_case* cases, int32_t ncases, const double* dts, int32_t ndt,
                  std::vector<VnCase>* host) {
  const int32_t nrep = dts ? ndt : 1;
  host->resize((size_t)ncases * nrep);
  for (int32_t c = 0; c < ncases; ++c) {
    const lb_vn_case& v = cases[c];
    if (!(std::isfinite(v.rho) && v.rho > 0.0 && std::isfinite(v.T) && v.T > 0.0 && std::isfinite(v.ux) &&
          std::isfinite(v.uy)))
      return lbkt_fail(LB_EPARAM, "case " + std::to_string(c) + ": state needs rho > 0, T > 0, finite u");
    for (int32_t j = 0; j < nrep; ++j) {
      lb_grid g;
      std::memset(&g, 0, sizeof(g));
      g.nx = 1;
      g.ny = 1;
      g.pitch = 64;
      g.dx = v.dx;
      g.dt = dts ? dts[(size_t)c * ndt + j] : v.dt;
      g.c1 = v.c1;
      g.c2 = v.c2;
      g.eta0 = v.eta0;
      g.gamma = v.gamma;
      g.tau = v.tau;
      g.beta = v.beta;
      for (int i = 0; i < 9; ++i) g.lambda[i] = v.lambda[i];
      for (int e = 0; e < 4; ++e) g.edge[e].kind = LB_BC_PERIODIC;
      const lb_status s = lb_validate(&g);
      if (s) return lbkt_fail(s, "case " + std::to_string(c) + ": " + lb_last_error());
      VnCase& h = (*host)[(size_t)c * nrep + j];
      lbkt_build_consts(&g, &h.K);
      h.rho = v.rho;
      h.ux = v.ux;
      h.uy = v.uy;
      h.T = v.T;
    }
  }
  return LB_OK;
}

lb_status scan(const std::vector<VnCase>& host, const double* kdx, const double* kdy, int32_t nk, int32_t reduce,
               double* out, hipStream_t st) {
  const int n = (int)host.size();
  const size_t bytes = host.size() * sizeof(VnCase);
  void* d = nullptr;
  hipError_t e = hipMallocAsync(&d, bytes, st);
  if (e != hipSuccess) return hip_fail("hipMallocAsync", e);
  e = hipMemcpyAsync(d, host.data(), bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vector is released by the caller
  if (e != hipSuccess) {
    (void)hipFreeAsync(d, st);
    return hip_fail("copying the scan cases", e);
  }
  if (reduce) hipLaunchKernelGGL(k_vn_zero, dim3((n + 255) / 256), dim3(256), 0, st, out, n);
  const int64_t total = (int64_t)n * nk;
  hipLaunchKernelGGL(k_vn_scan, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, st, (const VnCase*)d, n, kdx,
                     kdy, nk, reduce, out);
  e = hipGetLastError();
  const hipError_t e2 = hipFreeAsync(d, st);
  if (e != hipSuccess) return hip_fail("k_vn_scan launch", e);
  if (e2 != hipSuccess) return hip_fail("hipFreeAsync", e2);
  return LB_OK;
}

lb_status check_args(const lb_vn_case* cases, int32_t ncases, const double* kdx, const double* kdy, int32_t nk,
                     int64_t nrep) {
  if (!cases || !kdx || !kdy) return lbkt_fail(LB_EINVAL, "cases, kdx and kdy must not be NULL");
  if (ncases < 1 || nk < 1) return lbkt_fail(LB_EINVAL, "ncases and nk must be >= 1");
  if ((int64_t)ncases * nrep * nk >= ((int64_t)1 << 31))
    return lbkt_fail(LB_EINVAL, "ncases * nk (times ndt) must stay below 2^31");
  return LB_OK;
}

}  // namespace

extern "C" lb_status lb_vn_scan(const lb_vn_case* cases, int32_t ncases, const double* kdx, const double* kdy,
                                int32_t nk, int32_t reduce, double* out, void* stream) {
  lb_status s = check_args(cases, ncases, kdx, kdy, nk, 1);
  if (s) return s;
  if (!out) return lbkt_fail(LB_EINVAL, "out must not be NULL");
  std::vector<VnCase> host;
  if ((s = prepare(cases, ncases, nullptr, 0, &host))) return s;
  return scan(host, kdx, kdy, nk, reduce ? 1 : 0, out, (hipStream_t)stream);
}

extern "C" lb_status lb_vn_max_stable_dt(const lb_vn_case* cases, int32_t ncases, const double* dts, int32_t ndt,
                                         const double* kdx, const double* kdy, int32_t nk, double tol,
                                         double* dt_out, void* stream) {
  if (!dts || !dt_out) return lbkt_fail(LB_EINVAL, "dts and dt_out must not be NULL");
  if (ndt < 1) return lbkt_fail(LB_EINVAL, "ndt must be >= 1");
  lb_status s = check_args(cases, ncases, kdx, kdy, nk, ndt);
  if (s) return s;
  for (int32_t c = 0; c < ncases; ++c)
    for (int32_t j = 0; j < ndt; ++j) {
      const double* row = dts + (size_t)c * ndt;
      if (!(std::isfinite(row[j]) && row[j] > 0.0 && (j == 0 || row[j] > row[j - 1])))
        return lbkt_fail(LB_EINVAL, "case " + std::to_string(c) + ": dts must be finite, > 0 and strictly ascending");
    }
  if (!(std::isfinite(tol) && tol >= 0.0)) return lbkt_fail(LB_EINVAL, "tol must be finite and >= 0");
  std::vector<VnCase> host;
  if ((s = prepare(cases, ncases, dts, ndt, &host))) return s;
  hipStream_t st = (hipStream_t)stream;
  const size_t n = host.size();
  double* d = nullptr;
  hipError_t e = hipMallocAsync((void**)&d, n * sizeof(double), st);
  if (e != hipSuccess) return hip_fail("hipMallocAsync", e);
  s = scan(host, kdx, kdy, nk, 1, d, st);
  std::vector<double> rad(n);
  if (!s) {
    e = hipMemcpyAsync(rad.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail("reading the scan maxima", e);
  }
  (void)hipFreeAsync(d, st);
  if (s) return s;
  for (int32_t c = 0; c < ncases; ++c) {
    double best = 0.0;
    for (int32_t j = 0; j < ndt; ++j) {
      const double r = rad[(size_t)c * ndt + j];
      if (!(r <= 1.0 + tol)) break;   // NaN also stops the prefix
      best = dts[(size_t)c * ndt + j];
    }
    dt_out[c] = best;
  }
  return LB_OK;
}
