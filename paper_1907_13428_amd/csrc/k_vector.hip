// Elementwise and reduction kernels of the Krylov loop and the ADMM iteration.
//
// Reductions are deterministic: every block writes one partial sum (fixed
// intra-block order) and a single-block finalize kernel adds the partials in
// index order.  No floating-point atomics are used, so repeated runs are
// bitwise identical.
#include "fde_internal.hpp"
#include "fde_reduce.hpp"

namespace fde {

__device__ __forceinline__ bool is_done(const int* done) { return done && *done; }

// Sum of partial[0..n) in fixed order; valid in thread 0 of the (single) block.
// Up to 8 strided loads per thread are in flight at once.
__device__ __forceinline__ double ordered_sum(const double* partial, int n) {
  constexpr int U = 8;
  double s = 0.0;
  for (int i0 = 0; i0 < n; i0 += U * kBlock) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kBlock + (int)threadIdx.x;
      x[u] = i < n ? partial[i] : 0.0;
    }
    s += ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
  }
  return block_sum<kBlock>(s);
}

// ---------------------------------------------------------------------------
// PCG scalar steps (one block)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pcg_scalar(int op, const double* partial, int n, double* scal,
                                                       int* ints, double tol2, int maxit) {
  if (op != FIN_INIT && op != FIN_DOT && ints[kDone]) return;
  const double s0 = ordered_sum(partial, n);
  double s1 = 0.0;
  if (op == FIN_INIT) s1 = ordered_sum(partial + n, n);
  if (threadIdx.x != 0) return;
  switch (op) {
    case FIN_INIT: {
      scal[kTol2] = tol2;
      ints[kMaxit] = maxit;
      scal[kRR] = s0;
      scal[kBB] = s1;
      ints[kIter] = 0;
      ints[kDone] = 0;
      ints[kConv] = 0;
      if (s0 != s0 || s1 != s1) {
        ints[kDone] = 1;
        ints[kConv] = -1;
      } else if (s1 == 0.0 || s0 <= scal[kTol2] * s1) {  // b = 0: the solution is x = 0
        ints[kDone] = 1;
        ints[kConv] = 1;
      }
      break;
    }
    case FIN_DOT:
      scal[kDot] = s0;
      break;
    case FIN_CONV: {
      scal[kRR] = s0;
      const int it = ints[kIter] + 1;
      ints[kIter] = it;
      const int conv = (s0 != s0) ? -1 : (s0 <= scal[kTol2] * scal[kBB] ? 1 : 0);
      if (conv != 0 || it >= ints[kMaxit]) {
        ints[kConv] = conv;
        ints[kDone] = 1;
      }
      break;
    }
  }
}

hipError_t launch_pcg_scalar(int op, const double* partial, int n, double* scal, int* ints, hipStream_t s,
                             double tol2, int maxit) {
  k_pcg_scalar<<<1, kBlock, 0, s>>>(op, partial, n, scal, ints, tol2, maxit);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// vector ops
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_vec(int op, int64_t n, const double* __restrict__ a,
                                                const double* __restrict__ b, double* c,
                                                const double* scal, double* partial, const int* done) {
  if (is_done(done)) return;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double s0 = 0.0, s1 = 0.0;
  switch (op) {
    case VEC_RESID:
      for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double av = a[i];
        const double cv = av - b[i];
        c[i] = cv;
        s0 += cv * cv;
        s1 += av * av;
      }
      break;
    case VEC_DOT:
      for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) s0 += a[i] * b[i];
      break;
    case VEC_ZERO_IF_BB0:
      if (scal[kBB] != 0.0) return;
      for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) c[i] = 0.0;
      return;
    default:
      return;
  }
  const double r0 = block_sum<kBlock>(s0);
  if (threadIdx.x == 0) partial[blockIdx.x] = r0;
  if (op == VEC_RESID) {
    const double r1 = block_sum<kBlock>(s1);
    if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = r1;
  }
}

static int vec_blocks(int64_t n) {
  int64_t b = (n + kBlock * 4 - 1) / (kBlock * 4);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_axpy_dot(int op, int64_t n, const double* a, const double* b, double* c,
                           const double* scal, double* partial, const int* done, hipStream_t s,
                           int* nblocks) {
  const int blocks = vec_blocks(n);
  if (nblocks) *nblocks = blocks;
  k_vec<<<blocks, kBlock, 0, s>>>(op, n, a, b, c, scal, partial, done);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ADMM elementwise steps (Algorithm 1 with the merged x-step, scaled form)
// ---------------------------------------------------------------------------
// right-hand side pieces:
//   Ru = rho(-e_u wu + e_u^2 zu/delta) + (1-rho) k_u p
//   r  = k_u Ru / Mu - psi g + (delta/rho) p
//   v  = (1-rho) p - r / Mp         (b = B^T v + c)
//   c  = rho (J1 yhat - e_y wy + e_y^2 zy / delta)
// and under Algorithm 2 (Sec. 3.3.2) rho R_u u and rho R_y y, at the previous
// iterate, join Ru and c.
// the x-step right-hand side pieces at point i (time level t) from the
// iterate (p, wu, zu, wy, zy, u, y) held in registers
__device__ __forceinline__ void rhs_point(const AdmmConsts& k, const AdmmFields& f, double psi, int64_t i, int t,
                                          double p, double wu, double zu, double wy, double zy, double u,
                                          double y) {
  const double rho = k.rho, delta = k.delta;
  double xu = -k.e_u * wu + k.e_u * k.e_u * zu / delta;
  double xy = k.wts[t] * f.yhat[i] - k.e_y * wy + k.e_y * k.e_y * zy / delta;
  if (k.prox) {
    // Algorithm 2: R_u u^j and R_y y^j at the previous iterate
    xu += (k.cu - k.gamma * k.wts[t]) * u;
    xy += (k.cy - k.wts[t]) * y;
  }
  const double Ru = rho * xu + (1.0 - rho) * k.k_u * p;
  const double gv = f.g ? f.g[i] : 0.0;
  const double r = k.k_u * Ru / k.Mu[t] - psi * gv + (delta / rho) * p;
  f.Ru[i] = Ru;
  f.r[i] = r;
  f.v[i] = (1.0 - rho) * p - r / k.Mp[t];
  f.c[i] = rho * xy;
}

__global__ __launch_bounds__(kBlock) void k_admm_rhs(AdmmConsts k, AdmmFields f, double psi) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < k.n; i += stride) {
    const int t = (int)(i / k.plane);
    const double u = k.prox ? f.u[i] : 0.0, y = k.prox ? f.y[i] : 0.0;
    rhs_point(k, f, psi, i, t, f.p[i], f.wu[i], f.zu[i], f.wy[i], f.zy[i], u, y);
  }
}

hipError_t launch_admm_rhs(const AdmmConsts& k, const AdmmFields& f, double psi, hipStream_t s) {
  k_admm_rhs<<<vec_blocks(k.n), kBlock, 0, s>>>(k, f, psi);
  return hipGetLastError();
}

// recovery, projection, dual update and the three residual maxima:
//   p = (By + r)/Mp ; u = (Ru - k_u p)/Mu ; byp = By/Mp (optional, reused by the next x-step)
//   zy = clip(y + delta wy/e_y) ; zu = clip(u + delta wu/e_u)
//   wy += (rho/delta) e_y (y - zy) ; wu += (rho/delta) e_u (u - zu)
//   max |By + k_u u - psi g|, max |y - zy|, max |u - zu|
// With NEXT, the right-hand side pieces of the next iteration follow from the
// new iterate in registers (they replace Ru and r after their last use here;
// unused if the run stops at this iteration).
template <bool NEXT>
__global__ __launch_bounds__(kBlock) void k_admm_update(AdmmConsts k, AdmmFields f, double psi) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const double rho = k.rho, delta = k.delta;
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < k.n; i += stride) {
    const int t = (int)(i / k.plane);
    const double By = f.By[i];
    const double p = (By + f.r[i]) / k.Mp[t];
    const double u = (f.Ru[i] - k.k_u * p) / k.Mu[t];
    const double y = f.y[i];
    const double wy = f.wy[i], wu = f.wu[i];
    const double ya = k.lya ? k.lya[i] : k.ya, yb = k.lyb ? k.lyb[i] : k.yb;
    const double ua = k.lua ? k.lua[i] : k.ua, ub = k.lub ? k.lub[i] : k.ub;
    const double zy = fmin(fmax(y + delta * wy / k.e_y, ya), yb);
    const double zu = fmin(fmax(u + delta * wu / k.e_u, ua), ub);
    const double wy1 = wy + (rho / delta) * k.e_y * (y - zy);
    const double wu1 = wu + (rho / delta) * k.e_u * (u - zu);
    f.p[i] = p;
    f.u[i] = u;
    f.zy[i] = zy;
    f.zu[i] = zu;
    f.wy[i] = wy1;
    f.wu[i] = wu1;
    if (f.byp) f.byp[i] = k.invMp[t] * By;
    if constexpr (NEXT) rhs_point(k, f, psi, i, t, p, wu1, zu, wy1, zy, u, y);
    const double gv = f.g ? f.g[i] : 0.0;
    m0 = nanmax(m0, fabs(By + k.k_u * u - psi * gv));
    m1 = nanmax(m1, fabs(y - zy));
    m2 = nanmax(m2, fabs(u - zu));
  }
  const double r0 = block_max<kBlock>(m0);
  const double r1 = block_max<kBlock>(m1);
  const double r2 = block_max<kBlock>(m2);
  if (threadIdx.x == 0) {
    f.partial[3 * blockIdx.x + 0] = r0;
    f.partial[3 * blockIdx.x + 1] = r1;
    f.partial[3 * blockIdx.x + 2] = r2;
  }
}

hipError_t launch_admm_update(const AdmmConsts& k, const AdmmFields& f, double psi, hipStream_t s,
                              int* nblocks, bool next_rhs) {
  const int blocks = vec_blocks(k.n);
  if (nblocks) *nblocks = blocks;
  if (next_rhs) k_admm_update<true><<<blocks, kBlock, 0, s>>>(k, f, psi);
  else k_admm_update<false><<<blocks, kBlock, 0, s>>>(k, f, psi);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_max3(const double* partial, int nb, double* scal) {
  double m[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += kBlock) {
#pragma unroll
    for (int c = 0; c < 3; ++c) m[c] = nanmax(m[c], partial[3 * i + c]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double r = block_max<kBlock>(m[c]);
    if (threadIdx.x == 0) scal[kResP + c] = r;
  }
}

hipError_t launch_max3_finalize(const double* partial, int nb, double* scal, hipStream_t s) {
  k_max3<<<1, kBlock, 0, s>>>(partial, nb, scal);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_bounds_check(int64_t n, const double* ya, const double* yb,
                                                         const double* ua, const double* ub, double sya, double syb,
                                                         double sua, double sub, double* partial) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double by = 0.0, bu = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double a = ya ? ya[i] : sya, b = yb ? yb[i] : syb;
    const double c = ua ? ua[i] : sua, d = ub ? ub[i] : sub;
    if (!(a <= b)) by = 1.0;  // also catches NaN
    if (!(c <= d)) bu = 1.0;
  }
  const double ry = block_max<kBlock>(by);
  const double ru = block_max<kBlock>(bu);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x + 0] = ry;
    partial[3 * blockIdx.x + 1] = ru;
    partial[3 * blockIdx.x + 2] = 0.0;
  }
}

hipError_t launch_bounds_check(int64_t n, const double* ya, const double* yb, const double* ua, const double* ub,
                               double sya, double syb, double sua, double sub, double* partial, hipStream_t s,
                               int* nblocks) {
  const int blocks = vec_blocks(n);
  if (nblocks) *nblocks = blocks;
  k_bounds_check<<<blocks, kBlock, 0, s>>>(n, ya, yb, ua, ub, sya, syb, sua, sub, partial);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_grad_fields(int64_t n, int plane, const double* wts,
                                                        const double* y, const double* yhat, const double* p,
                                                        double psi, double* dyhat, double* lam) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const int t = (int)(i / plane);
    if (dyhat) dyhat[i] = -wts[t] * (y[i] - yhat[i]);
    if (lam) lam[i] = psi * p[i];
  }
}

struct DotArgs {
  const double* a[4];
  const double* b[4];
};

__global__ __launch_bounds__(kBlock) void k_dots(int64_t n, int count, DotArgs d, double* partial) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < count) s[j] += d.a[j][i] * d.b[j][i];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < count) {
      const double r = block_sum<kBlock>(s[j]);
      if (threadIdx.x == 0) partial[j * gridDim.x + blockIdx.x] = r;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_dots_finalize(int count, int nb, const double* partial, double* scal) {
  for (int j = 0; j < count; ++j) {
    const double r = ordered_sum(partial + (size_t)j * nb, nb);
    if (threadIdx.x == 0) scal[kD0 + j] = r;
  }
}

hipError_t launch_dots(int64_t n, int count, const double* const* a, const double* const* b, double* partial,
                       double* scal, hipStream_t s) {
  DotArgs d{};
  for (int j = 0; j < 4; ++j) {
    d.a[j] = j < count ? a[j] : nullptr;
    d.b[j] = j < count ? b[j] : nullptr;
  }
  const int blocks = vec_blocks(n);
  k_dots<<<blocks, kBlock, 0, s>>>(n, count, d, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_dots_finalize<<<1, kBlock, 0, s>>>(count, blocks, partial, scal);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_lincomb(int64_t n, double c0, const double* x0, double c1,
                                                    const double* x1, double c2, const double* x2, double* out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double v = 0.0;
    if (x0) v += c0 * x0[i];
    if (x1) v += c1 * x1[i];
    if (x2) v += c2 * x2[i];
    out[i] = v;
  }
}

hipError_t launch_lincomb(int64_t n, double c0, const double* x0, double c1, const double* x1, double c2,
                          const double* x2, double* out, hipStream_t s) {
  k_lincomb<<<vec_blocks(n), kBlock, 0, s>>>(n, c0, x0, c1, x1, c2, x2, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_adjoint_rhs(int64_t n, int plane, const double* wts, const double* y,
                                                        const double* yhat, const double* wy, double* f) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const int t = (int)(i / plane);
    f[i] = -wts[t] * (y[i] - yhat[i]) - wy[i];
  }
}

hipError_t launch_adjoint_rhs(int64_t n, int plane, const double* wts, const double* y, const double* yhat,
                              const double* wy, double* f, hipStream_t s) {
  k_adjoint_rhs<<<vec_blocks(n), kBlock, 0, s>>>(n, plane, wts, y, yhat, wy, f);
  return hipGetLastError();
}

// dual infeasibility of the final iterate: block maxima, then one ordered max
__global__ __launch_bounds__(kBlock) void k_dual_inf(AdmmConsts k, AdmmFields f, double gamma,
                                                     const double* __restrict__ btp, double* partial) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < k.n; i += stride) {
    const double j1 = k.wts[i / k.plane];
    const double sy = j1 * (f.y[i] - f.yhat[i]) + btp[i] + k.e_y * f.wy[i];
    const double su = gamma * j1 * f.u[i] + k.k_u * f.p[i] + k.e_u * f.wu[i];
    m = nanmax(m, nanmax(fabs(sy), fabs(su)));
  }
  m = block_max<kBlock>(m);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(kBlock) void k_max_finalize(const double* partial, int nb, double* out) {
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) m = nanmax(m, partial[i]);
  m = block_max<kBlock>(m);
  if (threadIdx.x == 0) *out = m;
}

hipError_t launch_dual_inf(const AdmmConsts& k, const AdmmFields& f, double gamma, const double* btp,
                           double* partial, double* scal, hipStream_t s) {
  const int blocks = vec_blocks(k.n);
  k_dual_inf<<<blocks, kBlock, 0, s>>>(k, f, gamma, btp, partial);
  k_max_finalize<<<1, kBlock, 0, s>>>(partial, blocks, scal + kDual);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_objective(int64_t n, int plane, const double* wts, double gamma,
                                                      const double* y, const double* yhat, const double* u,
                                                      double* partial) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const int t = (int)(i / plane);
    const double e = y[i] - yhat[i];
    s += 0.5 * wts[t] * (e * e + gamma * u[i] * u[i]);
  }
  const double r = block_sum<kBlock>(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

hipError_t launch_objective(int64_t n, int plane, const double* wts, double gamma, const double* y,
                            const double* yhat, const double* u, double* partial, hipStream_t s, int* nb) {
  const int blocks = vec_blocks(n);
  if (nb) *nb = blocks;
  k_objective<<<blocks, kBlock, 0, s>>>(n, plane, wts, gamma, y, yhat, u, partial);
  return hipGetLastError();
}

hipError_t launch_grad_fields(int64_t n, int plane, const double* wts, const double* y, const double* yhat,
                              const double* p, double psi, double* dyhat, double* lam, hipStream_t s) {
  k_grad_fields<<<vec_blocks(n), kBlock, 0, s>>>(n, plane, wts, y, yhat, p, psi, dyhat, lam);
  return hipGetLastError();
}

// the PCG done flags of many instances gathered into one array (one readback)
__global__ __launch_bounds__(kBlock) void k_gather_done(const int* const* ints, int count, int* out) {
  for (int i = threadIdx.x; i < count; i += kBlock) out[i] = ints[i][kDone];
}

hipError_t launch_gather_done(const int* const* ints, int count, int* out, hipStream_t s) {
  k_gather_done<<<1, kBlock, 0, s>>>(ints, count, out);
  return hipGetLastError();
}

}  // namespace fde
