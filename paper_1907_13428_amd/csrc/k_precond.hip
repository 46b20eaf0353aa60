// The Schur-complement preconditioner z = S~^{-1} r of eq. (3.10), with the
// 3-level T. Chan circulant C_3(B) of eq. (5.2): S~ = a I + C_3^* C_3 / mbar_p
// is diagonalised by the 3-D DFT, with eigenvalues
//     s(kx, ky, kt) = a + |psi (lam_t[kt] - lam_y[ky] - lam_x[kx])|^2 / mbar_p
// computed in registers from the three 1-D tables (no N-sized eigen array).
// The matching approximation S^ of eq. (3.11) with the same blocks is the
// circulant (C_3^* + c)(C_3 + c) / mbar_p, c = (a mbar_p)^{1/2}: its eigenvalue
// adds 2 (a / mbar_p)^{1/2} Re(psi (lam_t - lam_y - lam_x)) to s.
//
// Passes (each one HBM sweep of the half spectrum [nt][ny][H], H = nx/2 + 1):
//   1. x: real -> half spectrum, two real lines packed per complex FFT of
//      length nx and separated with X1 = (Z + conj Z~)/2, X2 = (Z - conj Z~)/2i
//      (fused with the PCG update r -= alpha q, x += alpha p and (r, r))
//   2. y: complex FFT along y on column tiles staged through LDS
//   3. t: complex FFT along t, divide by s * nx*ny*nt, inverse FFT along t
//   4. y: inverse complex FFT
//   5. x: half spectrum -> two real lines (Hermitian completion), fused (r, z)
//
// Inside PCG, (r, z) comes from the spectrum instead: with R = DFT(r) over
// all three axes and z = IDFT(R / s), Parseval gives
//     (r, z) = sum_k |R_k|^2 / (s_k nx ny nt),
// and over the half spectrum every column kx other than 0 and nx/2 stands
// for itself and its conjugate partner -kx (weight 2; s_{-k} = s_k because
// each 1-D table of a real circulant is conjugate-symmetric).  The t-pass,
// which holds R_k next to s_k, writes per-block partials; block 0 of the
// y-inverse pass sums them in a fixed order into (r, z) and beta; the
// x-inverse pass then writes the direction p = z + beta p itself.
// TS is the spectrum precision: double, or float for the mixed form.
#include "fde_fft.hpp"
#include "fde_internal.hpp"
#include "fde_reduce.hpp"

namespace fde {

constexpr int kPreThreads = 256;

template <typename TS> struct PreTypes {
  using V = cplx<TS>;
};

// x-direction passes: LPB = kPreThreads / T line pairs per block; when T does
// not divide the block (T = 5 for 50 and 100 points) the remaining threads
// form a spare group that runs the transforms (block barriers) on LDS of its
// own and touches no field
constexpr int pre_x_groups(int T) { return kPreThreads / T + (kPreThreads % T ? 1 : 0); }

// ---------------------------------------------------------------------------
// pass 1: x-direction real-to-complex
// ---------------------------------------------------------------------------
template <int L, typename TS, bool FUSE, bool SC>
__device__ __forceinline__ void pre_xfwd_body(const PrecondArgs& a, int bid) {
  using V = cplx<TS>;
  constexpr int E = default_E(L);
  constexpr int T = L / E;
  constexpr int LPB = kPreThreads / T;
  constexpr int H = L / 2 + 1;
  __shared__ V lds[pre_x_groups(T) * lpad_size(L)];
  if (a.done && *a.done) return;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int nlines = a.ny * a.nt;
  const int pair = bid * LPB + g;
  const int l0 = 2 * pair, l1 = 2 * pair + 1;
  const bool h0 = g < LPB && l0 < nlines, h1 = g < LPB && l1 < nlines;
  LineLds<V> buf{lds + g * lpad_size(L), 1};
  const V* tw = reinterpret_cast<const V*>(a.twx);

  // Input lines (with the fused update).  Loads are issued in groups of G
  // elements before the group's stores (the fields may alias as far as the
  // compiler knows, so it cannot hoist them itself); a missing line reads
  // line 0 and is zeroed.  The first group is loaded before the step length
  // is formed, so that its HBM latency overlaps the ordered sum of partials.
  constexpr int G = (E % 4 == 0) ? 4 : (E % 2 == 0 ? 2 : 1);
  const size_t b0 = h0 ? (size_t)l0 * L : 0, b1 = h1 ? (size_t)l1 * L : 0;
  // diagonal scaling rows (a missing line reads line 0's and is zeroed)
  const double* ds0 = SC ? precond_scale_row(a, h0 ? l0 : 0) : nullptr;
  const double* ds1 = SC ? precond_scale_row(a, h1 ? l1 : 0) : nullptr;
  double r0[G], r1[G], q0[G], q1[G], x0[G], x1[G], p0[G], p1[G], d0[G], d1[G];
  auto load_group = [&](int e0) {
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int i = t + T * (e0 + k);
      r0[k] = a.r[b0 + i];
      r1[k] = a.r[b1 + i];
      if constexpr (SC) {
        d0[k] = ds0[i];
        d1[k] = ds1[i];
      }
      if constexpr (FUSE) {
        q0[k] = a.q[b0 + i];
        q1[k] = a.q[b1 + i];
        x0[k] = a.xvec[b0 + i];
        x1[k] = a.xvec[b1 + i];
        p0[k] = a.pvec[b0 + i];
        p1[k] = a.pvec[b1 + i];
      }
    }
  };
  load_group(0);

  double alpha = 0.0;
  if constexpr (FUSE) {
    if (a.pq_partial) {
      // alpha = (r, z) / (p, q), every block summing the partials in the same order
      const double pq = block_ordered_sum<kPreThreads>(a.pq_partial, a.pq_n);
      alpha = a.scal[rz_slot(a.ints[kIter])] / pq;
      if (bid == 0 && threadIdx.x == 0) {
        a.scal_w[kPQ] = pq;
        a.scal_w[kAlpha] = alpha;
      }
    } else {
      alpha = a.scal[kAlpha];
    }
  }

  V v[E];
  double rr = 0.0;
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += G) {
    if (e0 > 0) load_group(e0);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int i = t + T * (e0 + k);
      double s0 = r0[k], s1 = r1[k];
      if constexpr (FUSE) {
        s0 -= alpha * q0[k];
        s1 -= alpha * q1[k];
        if (h0) {
          a.r[b0 + i] = s0;
          a.xvec[b0 + i] = x0[k] + alpha * p0[k];
        }
        if (h1) {
          a.r[b1 + i] = s1;
          a.xvec[b1 + i] = x1[k] + alpha * p1[k];
        }
      }
      if (!h0) s0 = 0.0;
      if (!h1) s1 = 0.0;
      rr += s0 * s0 + s1 * s1;
      if constexpr (SC) {
        s0 *= d0[k];
        s1 *= d1[k];
      }
      v[e0 + k] = V{TS(s0), TS(s1)};
    }
  }
  if constexpr (FUSE) {
    const double s = block_sum<kPreThreads>(rr);
    if (threadIdx.x == 0) a.partial[bid] = s;
  }

  line_fft<L, E, -1>(v, buf, t, tw);

  // Hermitian separation needs Z[(L - i) mod L] from another thread
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) buf[t + T * e] = v[e];
  __syncthreads();
  V* spec = reinterpret_cast<V*>(a.spec);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + T * e;
    if (i >= H) continue;
    const V z = v[e];
    const V zc = buf[(L - i) % L];
    const V x1 = V{TS(0.5) * (z.x + zc.x), TS(0.5) * (z.y - zc.y)};
    const V x2 = V{TS(0.5) * (z.y + zc.y), TS(-0.5) * (z.x - zc.x)};
    if (h0) spec[(size_t)l0 * H + i] = x1;
    if (h1) spec[(size_t)l1 * H + i] = x2;
  }
}

template <int L, typename TS, bool FUSE, bool SC>
__global__ __launch_bounds__(kPreThreads) void k_pre_xfwd(PrecondArgs a) {
  pre_xfwd_body<L, TS, FUSE, SC>(a, blockIdx.x);
}

// the batched twin: many instances in one launch (BatchArgs)
template <int L, typename TS, bool FUSE, bool SC>
__global__ __launch_bounds__(kPreThreads) void k_pre_xfwd_b(BatchArgs<PrecondArgs> b) {
  const int i = batch_instance(b, blockIdx.x);
  pre_xfwd_body<L, TS, FUSE, SC>(batch_local(b.args[i]), blockIdx.x - b.first[i]);
}

// ---------------------------------------------------------------------------
// passes 2/4 (y) and 3 (t): complex lines across rows of a [rows][H] plane,
// P columns per block staged through LDS
// ---------------------------------------------------------------------------
// Tile variant S (chosen by the autotuner): P = Pmax >> S complex columns per block.
template <int L, int S = 0> struct CCfg {
  static constexpr int E = default_E(L);
  static constexpr int T = L / E;
  static constexpr int cap(int a, int b) { return a < b ? a : b; }
  // widest tile: at most 16 columns, at most 256 threads, LDS tile within 128 KiB (FP64)
  static constexpr int Pmax = cap(cap(16, kPreThreads / T), (131072 / (lpad_size(L) * 16)) - 1);
  static constexpr int P = (Pmax >> S) > 0 ? (Pmax >> S) : 1;
  static constexpr int NT = ((P * T + 63) / 64) * 64;
  // LDS row stride: a spare column for the threads beyond P*T; dropped for
  // columns of 1024 points and more when no thread needs it (as in the y-pass)
  static constexpr int RS = (L >= 1024 && (P * T) % 64 == 0) ? P : P + 1;
  static_assert(Pmax >= 1, "tile");
};

// MODE 0: y-direction, sign SIGN.  MODE 1: t-direction with the eigenvalue
// division by s (S~^{-1}).  MODE 2: t-direction with the product by
// 1 / conj(psi (lt - ly - lx)), the inverse of the transposed circulant.
template <int L, typename TS, int MODE, int SIGN, int S>
__device__ __forceinline__ void pre_cc_body(const PrecondArgs& a, int bid, int nbk) {
  using V = cplx<TS>;
  using C = CCfg<L, S>;
  constexpr int E = C::E, T = C::T, P = C::P, NT = C::NT, RS = C::RS;
  __shared__ V lds[lpad_size(L) * RS];
  if (a.done && *a.done) return;
  const int H = a.H;
  // MODE 0: the tiles of each time slice cover its H columns.  MODE 1, 2: the
  // ny H columns (ky, kx) of a time plane are contiguous, so the tiles run
  // over them as one list (column ky H + kx) and no tile is cut short at the
  // end of a ky row.
  const int ncol = MODE == 0 ? H : a.ny * H;
  const int tiles = (ncol + P - 1) / P;
  const int tile = xcd_tile(bid, nbk);
  const int outer = MODE == 0 ? tile / tiles : 0;  // MODE 0: time slice
  const int k0 = (tile % tiles) * P;
  // element (line index i, column c) address in the spectrum
  size_t base, stride;
  if (MODE == 0) {
    base = (size_t)outer * a.ny * H;
    stride = H;
  } else {
    base = 0;
    stride = (size_t)a.ny * H;
  }
  V* spec = reinterpret_cast<V*>(a.spec);
  const V* tw = reinterpret_cast<const V*>(MODE == 0 ? a.twy : a.twt);
  const int tid = threadIdx.x;
  const bool active = tid < P * T;
  const int g = active ? tid / T : P, t = tid % T;
  LineLds<V> buf{lds + g, RS};

  // tile load: all loads of a thread are issued before the first LDS store
  // (and before the fused scalar steps below, whose sums then overlap them);
  // elements outside the tile or the plane read the tile's first element
  // (always inside) and are zeroed after the load
  constexpr int NE = L * P;
  constexpr int KL = (NE + NT - 1) / NT;
  auto elem = [&](int k, bool& ok) -> size_t {
    const int idx = tid + k * NT;
    const int row = idx / P, c = idx % P;
    ok = idx < NE && k0 + c < ncol;
    return base + (ok ? row * stride + c : 0) + k0;
  };
  V lv[KL];
  bool ok[KL];
#pragma unroll
  for (int k = 0; k < KL; ++k) lv[k] = spec[elem(k, ok[k])];

  if constexpr (MODE == 0 && SIGN < 0) {
    if (a.rr_partial) {
      // PCG convergence test on the recursively updated residual (fused).
      // Every block sums the same partials in the same order, so all reach
      // the same verdict on convergence; only block 0 reads and advances the
      // iteration count and records the verdict (the iteration limit stops
      // the later kernels of this iteration through the done flag).
      const double rr = block_ordered_sum<NT>(a.rr_partial, a.rr_n);
      const double bb = a.scal[kBB], tol2 = a.scal[kTol2];
      const int conv = (rr != rr) ? -1 : (rr <= tol2 * bb ? 1 : 0);
      if (bid == 0 && threadIdx.x == 0) {
        const int it = a.ints[kIter] + 1;
        a.scal_w[kRR] = rr;
        a.ints[kIter] = it;
        if (conv != 0 || it >= a.ints[kMaxit]) {
          a.ints[kConv] = conv;
          a.ints[kDone] = 1;
        }
      }
      if (conv != 0) return;
    }
  }
  if constexpr (MODE == 0 && SIGN > 0) {
    if (a.rzs_partial && bid == 0) {
      // (r, z) from the t-pass partials, and beta = (r, z) / (r, z) of the
      // previous iteration (or the first (r, z) alone) for the x-inverse pass
      const double rz = block_ordered_sum<NT>(a.rzs_partial, a.rzs_n);
      if (threadIdx.x == 0) {
        if (a.pdir == 2) {
          a.scal_w[kRZ] = rz;
        } else {
          const int it = a.ints[kIter];
          a.scal_w[rz_slot(it)] = rz;
          a.scal_w[kBeta] = rz / a.scal[rz_slot(it - 1)];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const int idx = tid + k * NT;
    if (idx < NE) lds[lpad(idx / P) * RS + idx % P] = ok[k] ? lv[k] : V{TS(0), TS(0)};
  }
  __syncthreads();
  V v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = buf[t + T * e];
  __syncthreads();

  if constexpr (MODE == 0) {
    line_fft<L, E, SIGN>(v, buf, t, tw);
  } else {
    line_fft<L, E, -1>(v, buf, t, tw);
    const int cf = k0 + g;  // column ky H + kx of the time plane
    const bool in_plane = cf < ncol;
    const int kx = in_plane ? cf % H : 0;
    const int ky = in_plane ? cf / H : 0;
    const double2 lx = a.lam_x[kx];
    const double2 ly = a.lam_y[ky];
    double rz = 0.0;  // this thread's share of (r, z) = sum |R|^2 / (s N)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kt = t + T * e;
      const double2 lt = a.lam_t[kt];
      const double re = a.psi * (lt.x - ly.x - lx.x);
      const double im = a.psi * (lt.y - ly.y - lx.y);
      if constexpr (MODE == 1) {
        const double s = a.a + (re * re + im * im) * a.inv_mbar + a.match2 * re;
        const double fd = a.inv_n / s;
        const TS f = TS(fd);
        const double vr = double(v[e].x), vi = double(v[e].y);
        rz += (vr * vr + vi * vi) * fd;
        v[e] = V{v[e].x * f, v[e].y * f};
      } else {
        // 1 / conj(re + i im) = (re + i im) / (re^2 + im^2)
        const double m = a.inv_n / (re * re + im * im);
        const TS fr = TS(re * m), fi = TS(im * m);
        v[e] = V{v[e].x * fr - v[e].y * fi, v[e].x * fi + v[e].y * fr};
      }
    }
    if constexpr (MODE == 1) {
      if (a.rzs_partial) {
        // threads past the tile hold no column; columns 0 and nx/2 count once
        const bool col = active && in_plane;
        const double w = (kx == 0 || 2 * kx == a.nx) ? 1.0 : 2.0;
        const double s = block_sum<NT>(col ? w * rz : 0.0);
        if (threadIdx.x == 0) a.rzs_partial[bid] = s;
      }
    }
    line_fft<L, E, +1>(v, buf, t, tw);
  }

  __syncthreads();
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) buf[t + T * e] = v[e];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    bool ok;
    const size_t gi = elem(k, ok);
    const int idx = tid + k * NT;
    if (ok) spec[gi] = lds[lpad(idx / P) * RS + idx % P];
  }
}

template <int L, typename TS, int MODE, int SIGN, int S>
__global__ __launch_bounds__((CCfg<L, S>::NT)) void k_pre_cc(PrecondArgs a) {
  pre_cc_body<L, TS, MODE, SIGN, S>(a, blockIdx.x, gridDim.x);
}

// the batched twin
template <int L, typename TS, int MODE, int SIGN, int S>
__global__ __launch_bounds__((CCfg<L, S>::NT)) void k_pre_cc_b(BatchArgs<PrecondArgs> b) {
  const int i = batch_instance(b, blockIdx.x);
  pre_cc_body<L, TS, MODE, SIGN, S>(batch_local(b.args[i]), blockIdx.x - b.first[i], b.first[i + 1] - b.first[i]);
}

// ---------------------------------------------------------------------------
// pass 5: half spectrum -> real lines.  OUT 0: z; 1: z and partial sums of
// (r, z); 2: the PCG direction p = z + beta p, in place in a.z
// ---------------------------------------------------------------------------
template <int L, typename TS, int OUT, bool SC>
__device__ __forceinline__ void pre_xinv_body(const PrecondArgs& a, int bid) {
  constexpr bool DOT = OUT == 1, UPD = OUT == 2;
  using V = cplx<TS>;
  constexpr int E = default_E(L);
  constexpr int T = L / E;
  constexpr int LPB = kPreThreads / T;
  constexpr int H = L / 2 + 1;
  __shared__ V lds[pre_x_groups(T) * lpad_size(L)];
  if (a.done && *a.done) return;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int nlines = a.ny * a.nt;
  const int pair = bid * LPB + g;
  const int l0 = 2 * pair, l1 = 2 * pair + 1;
  const bool h0 = g < LPB && l0 < nlines, h1 = g < LPB && l1 < nlines;
  LineLds<V> buf{lds + g * lpad_size(L), 1};
  const V* tw = reinterpret_cast<const V*>(a.twx);
  const V* spec = reinterpret_cast<const V*>(a.spec);
  // diagonal scaling rows (a missing line reads line 0's; nothing of it is stored)
  const double* ds0 = SC ? precond_scale_row(a, h0 ? l0 : 0) : nullptr;
  const double* ds1 = SC ? precond_scale_row(a, h1 ? l1 : 0) : nullptr;

  V v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + T * e;
    const bool lo = i < H;
    const int k = lo ? i : L - i;
    V x1 = V{TS(0), TS(0)}, x2 = V{TS(0), TS(0)};
    if (h0) x1 = spec[(size_t)l0 * H + k];
    if (h1) x2 = spec[(size_t)l1 * H + k];
    if (!lo) {
      x1.y = -x1.y;
      x2.y = -x2.y;
    }
    v[e] = V{x1.x - x2.y, x1.y + x2.x};  // X1 + i X2
  }
  line_fft<L, E, +1>(v, buf, t, tw);
  // z out, with (r, z) or into p: the r (or p) loads of a group of G elements
  // are issued before the group's stores; a missing line reads line 0 and
  // contributes nothing
  constexpr int G = (E % 4 == 0) ? 4 : (E % 2 == 0 ? 2 : 1);
  const size_t b0 = h0 ? (size_t)l0 * L : 0, b1 = h1 ? (size_t)l1 * L : 0;
  const double* opnd = DOT ? a.r : a.z;
  const double beta = UPD ? a.scal[kBeta] : 0.0;
  double rz = 0.0;
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += G) {
    double r0[G], r1[G], d0[G], d1[G];
    if constexpr (DOT || UPD) {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int i = t + T * (e0 + k);
        r0[k] = opnd[b0 + i];
        r1[k] = opnd[b1 + i];
      }
    }
    if constexpr (SC) {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int i = t + T * (e0 + k);
        d0[k] = ds0[i];
        d1[k] = ds1[i];
      }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int i = t + T * (e0 + k);
      double z0 = double(v[e0 + k].x), z1 = double(v[e0 + k].y);
      if constexpr (SC) {
        z0 *= d0[k];
        z1 *= d1[k];
      }
      if (h0) {
        if constexpr (UPD) a.z[b0 + i] = z0 + beta * r0[k];
        else a.z[b0 + i] = z0;
        if constexpr (DOT) rz += r0[k] * z0;
      }
      if (h1) {
        if constexpr (UPD) a.z[b1 + i] = z1 + beta * r1[k];
        else a.z[b1 + i] = z1;
        if constexpr (DOT) rz += r1[k] * z1;
      }
    }
  }
  if constexpr (DOT) {
    const double s = block_sum<kPreThreads>(rz);
    if (threadIdx.x == 0) a.partial2[bid] = s;
  }
}

template <int L, typename TS, int OUT, bool SC>
__global__ __launch_bounds__(kPreThreads) void k_pre_xinv(PrecondArgs a) {
  pre_xinv_body<L, TS, OUT, SC>(a, blockIdx.x);
}

// the batched twin
template <int L, typename TS, int OUT, bool SC>
__global__ __launch_bounds__(kPreThreads) void k_pre_xinv_b(BatchArgs<PrecondArgs> b) {
  const int i = batch_instance(b, blockIdx.x);
  pre_xinv_body<L, TS, OUT, SC>(batch_local(b.args[i]), blockIdx.x - b.first[i]);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
// Lengths whose PCG passes have batched twins: the axis lengths of the batched
// workloads' grids (8 .. 512 nodes in space and time, radix 2 and 3)
constexpr bool batch_dim(int n) {
  return n == 8 || n == 16 || n == 24 || n == 32 || n == 48 || n == 64 || n == 96 || n == 128 || n == 192 ||
         n == 256 || n == 384 || n == 512;
}
using PreBatchKernel = void (*)(BatchArgs<PrecondArgs>);
template <int L, typename TS, bool FUSE, bool SC> static PreBatchKernel xfwd_twin() {
  if constexpr (batch_dim(L) && FUSE) return k_pre_xfwd_b<L, TS, FUSE, SC>;
  else return nullptr;
}
template <int L, typename TS, int OUT, bool SC> static PreBatchKernel xinv_twin() {
  if constexpr (batch_dim(L) && OUT == 2) return k_pre_xinv_b<L, TS, OUT, SC>;
  else return nullptr;
}
template <int L, typename TS, int MODE, int SIGN, int S> static PreBatchKernel cc_twin() {
  if constexpr (batch_dim(L) && MODE != 2) return k_pre_cc_b<L, TS, MODE, SIGN, S>;
  else return nullptr;
}

#define FDE_FOR_DIM_LENGTHS(X)                                                                          \
  X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(50) X(64) X(80) X(96) X(100) X(128) X(160) X(192) X(256) \
  X(384) X(512) X(768) X(1024)

// SC: the diagonal scaling Delta S~^{-1} Delta (a.ds_tab set)
template <int L, typename TS, bool SC>
static void pre_x_sc(const PrecondArgs& a, bool fwd, int blocks, hipStream_t s) {
  if (fwd) {
    if (a.q) launch_pass(k_pre_xfwd<L, TS, true, SC>, xfwd_twin<L, TS, true, SC>(), blocks, kPreThreads, s, a);
    else launch_pass(k_pre_xfwd<L, TS, false, SC>, xfwd_twin<L, TS, false, SC>(), blocks, kPreThreads, s, a);
  } else {
    if (a.pdir == 1) launch_pass(k_pre_xinv<L, TS, 2, SC>, xinv_twin<L, TS, 2, SC>(), blocks, kPreThreads, s, a);
    else if (a.partial2) launch_pass(k_pre_xinv<L, TS, 1, SC>, xinv_twin<L, TS, 1, SC>(), blocks, kPreThreads, s, a);
    else launch_pass(k_pre_xinv<L, TS, 0, SC>, xinv_twin<L, TS, 0, SC>(), blocks, kPreThreads, s, a);
  }
}

template <int L, typename TS>
static hipError_t pre_x(const PrecondArgs& a, bool fwd, hipStream_t s, int* nb) {
  constexpr int LPB = kPreThreads / (L / default_E(L));
  const int pairs = (a.ny * a.nt + 1) / 2;
  const int blocks = (pairs + LPB - 1) / LPB;
  if (nb) *nb = blocks;
  if (a.ds_tab) pre_x_sc<L, TS, true>(a, fwd, blocks, s);
  else pre_x_sc<L, TS, false>(a, fwd, blocks, s);
  return hipGetLastError();
}

template <int L, typename TS, int S>
static hipError_t pre_y_S(const PrecondArgs& a, int sign, hipStream_t s) {
  using C = CCfg<L, S>;
  const int blocks = ((a.H + C::P - 1) / C::P) * a.nt;
  if (sign < 0) launch_pass(k_pre_cc<L, TS, 0, -1, S>, cc_twin<L, TS, 0, -1, S>(), blocks, C::NT, s, a);
  else launch_pass(k_pre_cc<L, TS, 0, +1, S>, cc_twin<L, TS, 0, +1, S>(), blocks, C::NT, s, a);
  return hipGetLastError();
}

template <int L, typename TS>
static hipError_t pre_y(const PrecondArgs& a, int sign, hipStream_t s) {
  switch (a.tile_y) {
    case 1: return pre_y_S<L, TS, 1>(a, sign, s);
    case 2: return pre_y_S<L, TS, 2>(a, sign, s);
    default: return pre_y_S<L, TS, 0>(a, sign, s);
  }
}

template <int L, typename TS, int S>
static hipError_t pre_t_S(const PrecondArgs& a, hipStream_t s) {
  using C = CCfg<L, S>;
  const int blocks = (a.ny * a.H + C::P - 1) / C::P;
  if (a.div_mode == 1) launch_pass(k_pre_cc<L, TS, 2, -1, S>, cc_twin<L, TS, 2, -1, S>(), blocks, C::NT, s, a);
  else launch_pass(k_pre_cc<L, TS, 1, -1, S>, cc_twin<L, TS, 1, -1, S>(), blocks, C::NT, s, a);
  return hipGetLastError();
}

template <int L, int S> static int t_blocks_S(const PrecondArgs& a) {
  return (a.ny * a.H + CCfg<L, S>::P - 1) / CCfg<L, S>::P;
}

template <int L> static int t_blocks(const PrecondArgs& a) {
  switch (a.tile_t) {
    case 1: return t_blocks_S<L, 1>(a);
    case 2: return t_blocks_S<L, 2>(a);
    default: return t_blocks_S<L, 0>(a);
  }
}

int precond_t_blocks(const PrecondArgs& a) {
  switch (a.nt) {
#define CASE(Lv) case Lv: return t_blocks<Lv>(a);
    FDE_FOR_DIM_LENGTHS(CASE)
    CASE(1)
#undef CASE
    default: return 0;
  }
}

template <int L, typename TS>
static hipError_t pre_t(const PrecondArgs& a, hipStream_t s) {
  switch (a.tile_t) {
    case 1: return pre_t_S<L, TS, 1>(a, s);
    case 2: return pre_t_S<L, TS, 2>(a, s);
    default: return pre_t_S<L, TS, 0>(a, s);
  }
}

template <typename TS>
static hipError_t single_pass(const PrecondArgs& a, int pass, hipStream_t s) {
  hipError_t err = hipErrorInvalidValue;
  const int L = (pass == 1 || pass == 5) ? a.nx : (pass == 3 ? a.nt : a.ny);
  switch (L) {
#define CASE(Lv)                                                   \
  case Lv:                                                         \
    if (pass == 1) err = pre_x<Lv, TS>(a, true, s, nullptr);       \
    else if (pass == 2) err = pre_y<Lv, TS>(a, -1, s);             \
    else if (pass == 3) err = pre_t<Lv, TS>(a, s);                 \
    else if (pass == 4) err = pre_y<Lv, TS>(a, +1, s);             \
    else if (pass == 5) err = pre_x<Lv, TS>(a, false, s, nullptr); \
    break;
    FDE_FOR_DIM_LENGTHS(CASE)
#undef CASE
    default:
      break;
  }
  return err;
}

template <typename TS>
static hipError_t precond_T(const PrecondArgs& a, int stage, hipStream_t s, int* nb_fwd, int* nb_inv) {
  hipError_t err = hipSuccess;
  if (stage >= 11 && stage <= 15) return single_pass<TS>(a, stage - 10, s);
  // pass 1 (x forward); partial sums of r.r only when fused
  if (stage != 2) {
    switch (a.nx) {
#define CASE(Lv) case Lv: err = pre_x<Lv, TS>(a, true, s, nb_fwd); break;
      FDE_FOR_DIM_LENGTHS(CASE)
#undef CASE
      default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess || stage == 1) return err;
  }
  PrecondArgs a2 = a;
  a2.rzs_n = precond_t_blocks(a);
  switch (a.ny) {
#define CASE(Lv) case Lv: err = pre_y<Lv, TS>(a2, -1, s); break;
    FDE_FOR_DIM_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  switch (a.nt) {
#define CASE(Lv) case Lv: err = pre_t<Lv, TS>(a2, s); break;
    FDE_FOR_DIM_LENGTHS(CASE)
    CASE(1)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  switch (a.ny) {
#define CASE(Lv) case Lv: err = pre_y<Lv, TS>(a2, +1, s); break;
    FDE_FOR_DIM_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  switch (a.nx) {
#define CASE(Lv) case Lv: err = pre_x<Lv, TS>(a, false, s, nb_inv); break;
    FDE_FOR_DIM_LENGTHS(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return err;
}

hipError_t launch_precond_stage(const PrecondArgs& a, bool fp32, int stage, hipStream_t s, int* nb_fwd,
                                int* nb_inv) {
  return fp32 ? precond_T<float>(a, stage, s, nb_fwd, nb_inv) : precond_T<double>(a, stage, s, nb_fwd, nb_inv);
}

}  // namespace fde
