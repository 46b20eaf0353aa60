// MINRES on the merged x-step system (3.8), the saddle-point route of
// Sec. 3.3.1, preconditioned by the block-diagonal K~ of eq. (3.12):
//
//     K = [ M_y   0    B^T  ]      K~ = diag(M_y, M_u, (mbar/a) S~)
//         [ 0     M_u  k_u I]
//         [ B     k_u  -(delta/rho) I ]
//
// The Lanczos process runs in the K~^{-1} inner product on unnormalised
// vectors v~_j (v_j = v~_j / g_j, z_j = K~^{-1} v_j), and the tridiagonal is
// reduced by Givens rotations as it grows, so x is updated every iteration
// along w_{j+1} = (z_j - a3 w_{j-1} - a2 w_j) / a1.  Every scalar of the
// recurrence lives in device memory and is produced by one-block kernels from
// deterministic partial sums; nothing is read back inside the loop.
#include "fde_internal.hpp"
#include "fde_reduce.hpp"

namespace fde {

namespace {

int mr_blocks(int64_t n) {
  int64_t b = (n + kBlock * 4 - 1) / (kBlock * 4);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

__device__ __forceinline__ double mr_ordered_sum(const double* p, int n) {
  constexpr int U = 8;
  double s = 0.0;
  if (!p) return 0.0;
  for (int i0 = 0; i0 < n; i0 += U * kBlock) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kBlock + (int)threadIdx.x;
      x[u] = i < n ? p[i] : 0.0;
    }
    s += ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
  }
  return block_sum<kBlock>(s);
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_minres_pre(MinresConsts k, Triple z, double* tmp, double* qu,
                                                       double* partial, int* ints) {
  const int stop = ints[kStop];
  if (blockIdx.x == 0 && threadIdx.x == 0) ints[kDone] = stop;
  if (stop) return;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < k.n; i += stride) {
    const int t = (int)(i / k.plane);
    const double zu = z.u[i], zp = z.p[i];
    const double q = k.Mu[t] * zu + k.k_u * zp;
    tmp[i] = k.k_u * zu - k.dr * zp;
    qu[i] = q;
    s += zu * q;
  }
  s = block_sum<kBlock>(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_minres_vec(int mode, MinresConsts k, Triple q, Triple v, Triple out,
                                                       Triple z, const double* ms, double* partial,
                                                       const int* done) {
  if (done && *done) return;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if (mode == MR_ZERO) {
    if (ms && ms[kMNb] != 0.0) return;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < k.n; i += stride)
      out.y[i] = out.u[i] = out.p[i] = 0.0;
    return;
  }
  double ig = 0.0, dg = 0.0, go = 0.0;
  if (mode == MR_LANCZOS) {
    ig = 1.0 / ms[kMG];
    dg = ms[kMD] * ig;
    go = ms[kMG] / ms[kMGold];
  }
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < k.n; i += stride) {
    const int t = (int)(i / k.plane);
    double oy, ou, op;
    if (mode == MR_RESID) {
      oy = v.y[i] - q.y[i];
      ou = v.u[i] - q.u[i];
      op = v.p[i] - q.p[i];
    } else if (mode == MR_LANCZOS) {
      const double a0 = out.y[i], a1 = out.u[i], a2 = out.p[i];
      const double b0 = v.y[i], b1 = v.u[i], b2 = v.p[i];
      oy = q.y[i] * ig - dg * b0 - go * a0;
      ou = q.u[i] * ig - dg * b1 - go * a1;
      op = q.p[i] * ig - dg * b2 - go * a2;
    } else {  // MR_RHS
      oy = v.y[i];
      ou = v.u[i];
      op = 0.0;
    }
    if (mode != MR_RHS) {
      out.y[i] = oy;
      out.u[i] = ou;
      out.p[i] = op;
    }
    const double zy = oy / k.My[t], zu = ou / k.Mu[t];
    z.y[i] = zy;
    z.u[i] = zu;
    s += zy * oy + zu * ou;
  }
  s = block_sum<kBlock>(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_minres_scalar(int op, const double* p0, int n0, const double* p1, int n1,
                                                          const double* p2, int n2, double* ms, int* ints,
                                                          double tol, int maxit) {
  if ((op == MR_DELTA || op == MR_GIVENS) && ints[kStop]) return;
  const double s0 = mr_ordered_sum(p0, n0);
  const double s1 = mr_ordered_sum(p1, n1);
  const double s2 = mr_ordered_sum(p2, n2);
  if (threadIdx.x != 0) return;
  const double sum = s0 + s1 + s2;
  switch (op) {
    case MR_NB:
      ms[kMNb] = sqrt(fmax(sum, 0.0));
      ms[kMTol] = tol;
      ints[kMaxit] = maxit;
      ints[kStop] = 0;
      ints[kDone] = 0;
      break;
    case MR_INIT: {
      const double g = sqrt(fmax(sum, 0.0));
      const double nb = ms[kMNb];
      ms[kMG] = g;
      ms[kMGold] = 1.0;
      ms[kMEta] = g;
      ms[kMC] = ms[kMCold] = 1.0;
      ms[kMS] = ms[kMSold] = 0.0;
      ms[kMRes] = g;
      ints[kIter] = 0;
      ints[kConv] = 0;
      ints[kDone] = 0;
      ints[kStop] = 0;
      if (g != g || nb != nb) {
        ints[kConv] = -1;
        ints[kStop] = ints[kDone] = 1;
      } else if (nb == 0.0 || g <= ms[kMTol] * nb) {  // b = 0: x = 0
        ints[kConv] = 1;
        ints[kStop] = ints[kDone] = 1;
      }
      break;
    }
    case MR_DELTA: {
      const double g = ms[kMG];
      ms[kMD] = sum / (g * g);
      break;
    }
    case MR_GIVENS: {
      const double g = ms[kMG], dl = ms[kMD];
      const double c = ms[kMC], cold = ms[kMCold], s = ms[kMS], sold = ms[kMSold];
      const double gn = sqrt(fmax(sum, 0.0));
      const double a0 = c * dl - cold * s * g;
      const double a1 = hypot(a0, gn);
      const double a2 = s * dl + cold * c * g;
      const double a3 = sold * g;
      const double cn = a0 / a1, sn = gn / a1;
      const double eta = ms[kMEta];
      const int it = ints[kIter] + 1;
      ints[kIter] = it;
      if (!(a1 > 0.0) || a1 != a1 || gn != gn) {
        // breakdown or non-finite: leave x as it is
        ms[kMA1] = 1.0;
        ms[kMA2] = ms[kMA3] = ms[kMX] = ms[kMZ] = 0.0;
        ints[kConv] = -1;
        ints[kStop] = 1;
        break;
      }
      ms[kMA1] = a1;
      ms[kMA2] = a2;
      ms[kMA3] = a3;
      ms[kMX] = cn * eta;
      ms[kMZ] = 1.0 / g;
      const double en = -sn * eta;
      ms[kMEta] = en;
      ms[kMRes] = fabs(en);
      ms[kMGold] = g;
      ms[kMG] = gn;
      ms[kMCold] = c;
      ms[kMC] = cn;
      ms[kMSold] = s;
      ms[kMS] = sn;
      if (fabs(en) <= ms[kMTol] * ms[kMNb]) {
        ints[kConv] = 1;
        ints[kStop] = 1;
      } else if (it >= ints[kMaxit]) {
        ints[kStop] = 1;
      }
      break;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_minres_update(MinresConsts k, Triple z, Triple w_old, Triple w, Triple x,
                                                          const double* ms, const int* done) {
  if (*done) return;
  const double a1 = ms[kMA1], a2 = ms[kMA2], a3 = ms[kMA3], cx = ms[kMX], iz = ms[kMZ];
  const double ia1 = 1.0 / a1;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < k.n; i += stride) {
    const double zy = z.y[i], zu = z.u[i], zp = z.p[i];
    const double oy = w_old.y[i], ou = w_old.u[i], op = w_old.p[i];
    const double cy = w.y[i], cu = w.u[i], cp = w.p[i];
    const double ny = (zy * iz - a3 * oy - a2 * cy) * ia1;
    const double nu = (zu * iz - a3 * ou - a2 * cu) * ia1;
    const double np = (zp * iz - a3 * op - a2 * cp) * ia1;
    w_old.y[i] = ny;
    w_old.u[i] = nu;
    w_old.p[i] = np;
    x.y[i] += cx * ny;
    x.u[i] += cx * nu;
    x.p[i] += cx * np;
  }
}

hipError_t launch_minres_pre(const MinresConsts& k, Triple z, double* tmp, double* qu, double* partial, int* ints,
                             hipStream_t s, int* nb) {
  const int blocks = mr_blocks(k.n);
  if (nb) *nb = blocks;
  k_minres_pre<<<blocks, kBlock, 0, s>>>(k, z, tmp, qu, partial, ints);
  return hipGetLastError();
}

hipError_t launch_minres_vec(int mode, const MinresConsts& k, Triple q, Triple v, Triple out, Triple z,
                             const double* ms, double* partial, const int* done, hipStream_t s, int* nb) {
  const int blocks = mr_blocks(k.n);
  if (nb) *nb = blocks;
  k_minres_vec<<<blocks, kBlock, 0, s>>>(mode, k, q, v, out, z, ms, partial, done);
  return hipGetLastError();
}

hipError_t launch_minres_scalar(int op, const double* p0, int n0, const double* p1, int n1, const double* p2,
                                int n2, double* ms, int* ints, double tol, int maxit, hipStream_t s) {
  k_minres_scalar<<<1, kBlock, 0, s>>>(op, p0, n0, p1, n1, p2, n2, ms, ints, tol, maxit);
  return hipGetLastError();
}

hipError_t launch_minres_update(const MinresConsts& k, Triple z, Triple w_old, Triple w, Triple x, const double* ms,
                                const int* done, hipStream_t s) {
  k_minres_update<<<mr_blocks(k.n), kBlock, 0, s>>>(k, z, w_old, w, x, ms, done);
  return hipGetLastError();
}

}  // namespace fde
