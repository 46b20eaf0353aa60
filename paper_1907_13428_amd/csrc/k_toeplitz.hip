// Toeplitz line passes of the constraint operator D = C_t (x) I - I (x)(L_x (+) L_y)
// (eq. (4.9)) and its transpose, by circulant embedding and FFT (Table 1, Sec. 5).
//
// A length-n Toeplitz product T v is the first n entries of C [v; 0], C the
// 2n circulant whose first column is (t_0 .. t_{n-1}, 0, t_{-(n-1)} .. t_{-1});
// C = F^{-1} diag(lambda) F.  Two real lines are packed into one complex
// line (the operators are real), so one forward and one inverse complex FFT
// of length 2n serve two lines.  The host tables lambda already carry the
// factor c_a / h^a of eq. (4.7) and 1/(2n).
//
// Variable coefficients (row scaling d+ G + d- G^T, or G^T d+ + G d- for the
// transpose) need the G and G^T products separately: one forward and two
// inverse transforms (forward operator) or two forward and one inverse
// (transpose).
#include "fde_fft.hpp"
#include "fde_internal.hpp"
#include "fde_reduce.hpp"

namespace fde {

constexpr int kLineThreads = 256;


// ---------------------------------------------------------------------------
// x-pass: contiguous lines (t, j), with the time difference fused
// ---------------------------------------------------------------------------
// PAD: the embedding is longer than 2n (L >= 2n, the length n read at run
// time): elements n..L/2-1 of the data half are zero and only the first n
// results are kept.  Without PAD, n = L/2 is known at compile time.
template <int L, bool VAR, bool TRANS, bool PAD>
__device__ __forceinline__ void xpass_body(const LinePassArgs& a, int bid) {
  constexpr int E = default_E(L);
  constexpr int T = L / E;
  static_assert(T <= kLineThreads, "line too long for one block");
  static_assert(kLineThreads % T == 0, "whole lines per block");
  constexpr int LPB = kLineThreads / T;  // packed line pairs per block
  const int n = PAD ? a.nx : L / 2;
  __shared__ double2 lds[LPB * lpad_size(L)];
  if (a.done && *a.done) return;

  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int nlines = a.ny * a.nt;
  const int pair = bid * LPB + g;
  const int l0 = 2 * pair, l1 = 2 * pair + 1;
  const bool h0 = l0 < nlines, h1 = l1 < nlines;
  LineLds<double2> buf{lds + g * lpad_size(L), 1};
  const double* __restrict__ in = a.in;

  // element e of thread t is i = t + T e; i < L/2 exactly when e < EH, so the
  // zero half of the embedding and the discarded half of the result are
  // known at compile time (with PAD, i < n is checked as well)
  constexpr int EH = E / 2;
  double2 v[E];
  double2 w[E];
#pragma unroll
  for (int e = 0; e < EH; ++e) {
    const int i = t + T * e;
    const bool in_line = !PAD || i < n;
    double x0 = 0.0, x1 = 0.0;
    if (h0 && in_line) x0 = in[(size_t)l0 * n + i];
    if (h1 && in_line) x1 = in[(size_t)l1 * n + i];
    if constexpr (VAR && TRANS) {
      double p0 = 0, p1 = 0, m0 = 0, m1 = 0;
      if (h0 && in_line) { p0 = a.dplus[(l0 % a.ny) * n + i]; m0 = a.dminus[(l0 % a.ny) * n + i]; }
      if (h1 && in_line) { p1 = a.dplus[(l1 % a.ny) * n + i]; m1 = a.dminus[(l1 % a.ny) * n + i]; }
      v[e] = double2{p0 * x0, p1 * x1};
      w[e] = double2{m0 * x0, m1 * x1};
    } else {
      v[e] = double2{x0, x1};
    }
  }
#pragma unroll
  for (int e = EH; e < E; ++e) v[e] = w[e] = double2{0.0, 0.0};

  line_fft<L, E, -1>(v, buf, t, a.tw);
  if constexpr (VAR && TRANS) line_fft<L, E, -1>(w, buf, t, a.tw);

#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + T * e;
    const double2 la = a.lamA[i];
    if constexpr (VAR && TRANS) {
      // transpose: G^T (d+ v) + G (d- v); host passes lamA = G^T, lamB = G
      v[e] = cadd(cmul(v[e], la), cmul(w[e], a.lamB[i]));
    } else if constexpr (VAR) {
      w[e] = cmul(v[e], a.lamB[i]);  // G^T v
      v[e] = cmul(v[e], la);         // G v
    } else {
      v[e] = cmul(v[e], la);
    }
  }

  line_fft<L, E, +1>(v, buf, t, a.tw);
  if constexpr (VAR && !TRANS) line_fft<L, E, +1>(w, buf, t, a.tw);

  // Epilogue, out = s_time * time difference + s_sp * spatial, through the
  // pair's LDS buffer: thread t then owns adjacent elements (i, i+1) of both
  // lines (16-byte accesses; n is even) and issues all loads of a group of
  // element pairs before its first store.  Missing lines and time neighbours
  // read an address inside the field and are zeroed after the load.
  constexpr bool WAVE = line_in_wave(T);
  constexpr int NH = L / 2;  // offset of the second product (G^T v) in the buffer
  line_sync<WAVE>();
#pragma unroll
  for (int e = 0; e < EH; ++e) {
    buf[t + T * e] = v[e];
    if constexpr (VAR && !TRANS) buf[t + T * e + NH] = w[e];
  }
  line_sync<WAVE>();

  static_assert(E % 4 == 0, "the epilogue moves pairs of elements of both halves");
  constexpr int KE = E / 4;                    // element pairs per thread (L / 4 = T E / 4)
  constexpr int KG = (KE % 2 == 0) ? 2 : KE;   // element pairs per load group
  const size_t plane = (size_t)a.ny * n;
  const int tt0 = l0 / a.ny, tt1 = l1 / a.ny;
  const bool nb0 = h0 && (TRANS ? tt0 + 1 < a.nt : tt0 > 0);
  const bool nb1 = h1 && (TRANS ? tt1 + 1 < a.nt : tt1 > 0);
  const size_t b0 = h0 ? (size_t)l0 * n : 0, b1 = h1 ? (size_t)l1 * n : 0;
  const ptrdiff_t nbo0 = nb0 ? (TRANS ? (ptrdiff_t)plane : -(ptrdiff_t)plane) : 0;
  const ptrdiff_t nbo1 = nb1 ? (TRANS ? (ptrdiff_t)plane : -(ptrdiff_t)plane) : 0;
  const int r0 = h0 ? (l0 % a.ny) * n : 0, r1 = h1 ? (l1 % a.ny) * n : 0;
  const bool timed = a.s_time != 0.0;
  const double2 z2{0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < KE; k0 += KG) {
    double2 c0[KG], c1[KG], p0[KG], p1[KG], dp0[KG], dp1[KG], dm0[KG], dm1[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const int i = (!PAD || 2 * (t + T * (k0 + k)) < n) ? 2 * (t + T * (k0 + k)) : 0;
      c0[k] = c1[k] = p0[k] = p1[k] = z2;
      if (timed) {
        c0[k] = ld2(in + b0 + i);
        c1[k] = ld2(in + b1 + i);
        p0[k] = ld2(in + b0 + i + nbo0);
        p1[k] = ld2(in + b1 + i + nbo1);
      }
      if constexpr (VAR && !TRANS) {
        dp0[k] = ld2(a.dplus + r0 + i);
        dm0[k] = ld2(a.dminus + r0 + i);
        dp1[k] = ld2(a.dplus + r1 + i);
        dm1[k] = ld2(a.dminus + r1 + i);
      }
    }
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const int i = 2 * (t + T * (k0 + k));
      if (PAD && i >= n) continue;
      const double2 sa = buf[i], sb = buf[i + 1];
      double2 s0{sa.x, sb.x}, s1{sa.y, sb.y};  // spatial products of lines l0, l1
      if constexpr (VAR && !TRANS) {
        const double2 ta = buf[i + NH], tb = buf[i + NH + 1];
        s0 = double2{dp0[k].x * s0.x + dm0[k].x * ta.x, dp0[k].y * s0.y + dm0[k].y * tb.x};
        s1 = double2{dp1[k].x * s1.x + dm1[k].x * ta.y, dp1[k].y * s1.y + dm1[k].y * tb.y};
      }
      const double2 q0 = nb0 ? p0[k] : z2, q1 = nb1 ? p1[k] : z2;
      if (h0)
        st2(a.out + b0 + i, double2{a.s_sp * s0.x + a.s_time * (c0[k].x - q0.x),
                                    a.s_sp * s0.y + a.s_time * (c0[k].y - q0.y)});
      if (h1)
        st2(a.out + b1 + i, double2{a.s_sp * s1.x + a.s_time * (c1[k].x - q1.x),
                                    a.s_sp * s1.y + a.s_time * (c1[k].y - q1.y)});
    }
  }
}

template <int L, bool VAR, bool TRANS, bool PAD = false>
__global__ __launch_bounds__(kLineThreads) void k_xpass(LinePassArgs a) {
  xpass_body<L, VAR, TRANS, PAD>(a, blockIdx.x);
}

// the batched twin: many instances in one launch (BatchArgs)
template <int L, bool VAR, bool TRANS, bool PAD = false>
__global__ __launch_bounds__(kLineThreads) void k_xpass_b(BatchArgs<LinePassArgs> b) {
  const int i = batch_instance(b, blockIdx.x);
  xpass_body<L, VAR, TRANS, PAD>(batch_local(b.args[i]), blockIdx.x - b.first[i]);
}

// ---------------------------------------------------------------------------
// y-pass: a block owns one time slice and 2P adjacent x-columns; the tile is
// staged through LDS so that every global access is row-contiguous
// ---------------------------------------------------------------------------
// Tile variant S (chosen by the autotuner): P = Pmax >> S column pairs per block.
template <int L, int S = 0> struct YCfg {
  static constexpr int E = default_E(L);
  static constexpr int T = L / E;
  static constexpr int cap(int a, int b) { return a < b ? a : b; }
  // widest tile: at most 8 column pairs, at most 512 threads, LDS tile within 128 KiB
  static constexpr int Pmax = cap(cap(8, 2 * kLineThreads / T), (131072 / (lpad_size(L) * 16)) - 1);
  static constexpr int P = (Pmax >> S) > 0 ? (Pmax >> S) : 1;
  static constexpr int NT = ((P * T + 63) / 64) * 64;  // threads per block
  // LDS row stride: a spare column P for the threads beyond P*T, if any.  For
  // columns of 1024 points and more the tile is kept without it when no thread
  // needs it: the smaller tile lets more blocks share a CU (measured: 10-40%
  // faster at 1024-2048 points); shorter columns keep the odd stride, which
  // spreads the column accesses over the LDS banks
  static constexpr int RS = (L >= 1024 && (P * T) % 64 == 0) ? P : P + 1;
  static_assert(Pmax >= 1, "tile");
};

// COL: coefficients constant along each y-line (d+(x), d-(x)).  Column c then
// applies the single Toeplitz matrix M_c = d+_c G + d-_c G^T (transpose:
// d+_c G^T + d-_c G), whose embedding multiplier is l_c = d+_c lamA + d-_c lamB.
// The two real columns packed in Z = F(u0 + i u1) get M_0 u0 + i M_1 u1 from one
// inverse transform of ((l_0 + l_1)/2) Z[k] + ((l_0 - l_1)/2) conj Z[L-k]
// (Hermitian separation), so a pair costs two transforms instead of three.
// PAD: as for the x-pass, an embedding longer than 2n (n = ny read at run time).
template <int L, bool VAR, bool TRANS, int S, bool COL, bool PAD>
__device__ __forceinline__ void ypass_body(const LinePassArgs& a, int bid, int nbk) {
  static_assert(!(VAR && COL), "per-column coefficients use the constant-coefficient tile path");
  using C = YCfg<L, S>;
  constexpr int E = C::E, T = C::T, P = C::P, NT = C::NT, RS = C::RS;
  constexpr int NH = L / 2;  // rows of the data half; the second input (d- v) starts there
  const int n = PAD ? a.ny : NH;
  constexpr int TX = 2 * P;
  __shared__ double2 lds[lpad_size(L) * RS];
  if (a.done && *a.done) return;

  const int nx = a.nx;
  const int tiles = (nx + TX - 1) / TX;
  const int tile = xcd_tile(bid, nbk);
  const int slice = tile / tiles;
  const int x0 = (tile % tiles) * TX;
  const size_t sbase = (size_t)slice * n * nx;
  const int tid = threadIdx.x;
  // threads beyond P*T (block rounded up to whole wavefronts) run the FFT on
  // the spare LDS column P, which holds no data, and store nothing
  const bool active = tid < P * T;
  const int g = active ? tid / T : P, t = tid % T;
  LineLds<double2> buf{lds + g, RS};

  // Cooperative tile load, element = (row, column pair): one 16-byte access per
  // element (nx is even and tiles start at even columns, so a pair never
  // straddles the edge).  Elements outside the tile or the grid read the
  // tile's first pair (always inside) and are zeroed after the load, so a
  // thread issues all its loads before the first LDS store, without branches.
  // Rows 0..n-1 hold v (d+ v in the transposed variable case, with d- v in
  // rows NH..NH+n-1); columns beyond nx are zero.
  const int NE = n * P;
  constexpr int KL = (NH * P + NT - 1) / NT;
  int ge[KL];     // offset of the element within the slice (plane index)
  bool ok[KL];
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const int idx = tid + k * NT;
    const int row = idx / P, x = x0 + 2 * (idx % P);
    ok[k] = idx < NE && x < nx;
    ge[k] = ok[k] ? row * nx + x : x0;
  }
  {
    double2 lv[KL], lp[KL], lm[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) lv[k] = ld2(a.in + sbase + ge[k]);
    if constexpr (VAR && TRANS) {
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        lp[k] = ld2(a.dplus + ge[k]);
        lm[k] = ld2(a.dminus + ge[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int idx = tid + k * NT;
      if (idx < NE) {
        const int row = idx / P, cp = idx % P;
        const double2 v0 = ok[k] ? lv[k] : double2{0.0, 0.0};
        if constexpr (VAR && TRANS) {
          lds[lpad(row) * RS + cp] = double2{lp[k].x * v0.x, lp[k].y * v0.y};
          lds[lpad(row + NH) * RS + cp] = double2{lm[k].x * v0.x, lm[k].y * v0.y};
        } else {
          lds[lpad(row) * RS + cp] = v0;
        }
      }
    }
  }
  __syncthreads();

  // element e of thread t is row i = t + T e; i < L/2 exactly when e < EH
  // (with PAD, rows n..L/2-1 hold no data and are read as zero)
  constexpr int EH = E / 2;
  double2 v[E];
  double2 w[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = w[e] = double2{0.0, 0.0};
    if (e < EH && (!PAD || t + T * e < n)) {
      v[e] = buf[t + T * e];
      if constexpr (VAR && TRANS) w[e] = buf[t + T * e + NH];
    }
  }
  __syncthreads();

  line_fft<L, E, -1>(v, buf, t, a.tw);
  if constexpr (VAR && TRANS) line_fft<L, E, -1>(w, buf, t, a.tw);
  if constexpr (COL) {
    // partner Z[(L - i) mod L] through the pair's LDS stripe
    constexpr bool WAVE = line_in_wave(T);
    line_sync<WAVE>();
#pragma unroll
    for (int e = 0; e < E; ++e) buf[t + T * e] = v[e];
    line_sync<WAVE>();
#pragma unroll
    for (int e = 0; e < E; ++e) w[e] = buf[(L - (t + T * e)) % L];
    line_sync<WAVE>();
    const int c0 = x0 + 2 * g;
    const bool h0 = active && c0 < nx, h1 = active && c0 + 1 < nx;
    const double p0 = h0 ? a.dplus[c0] : 0.0, p1 = h1 ? a.dplus[c0 + 1] : 0.0;
    const double m0 = h0 ? a.dminus[c0] : 0.0, m1 = h1 ? a.dminus[c0 + 1] : 0.0;
    const double pb = 0.5 * (p0 + p1), mb = 0.5 * (m0 + m1), pd = 0.5 * (p0 - p1), md = 0.5 * (m0 - m1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = t + T * e;
      const double2 la = a.lamA[i], lb = a.lamB[i];
      const double2 A{pb * la.x + mb * lb.x, pb * la.y + mb * lb.y};
      const double2 B{pd * la.x + md * lb.x, pd * la.y + md * lb.y};
      v[e] = cadd(cmul(A, v[e]), cmul(B, double2{w[e].x, -w[e].y}));
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = t + T * e;
      const double2 la = a.lamA[i];
      if constexpr (VAR && TRANS) {
        v[e] = cadd(cmul(v[e], la), cmul(w[e], a.lamB[i]));
      } else if constexpr (VAR) {
        w[e] = cmul(v[e], a.lamB[i]);
        v[e] = cmul(v[e], la);
      } else {
        v[e] = cmul(v[e], la);
      }
    }
  }
  line_fft<L, E, +1>(v, buf, t, a.tw);
  if constexpr (VAR && !TRANS) line_fft<L, E, +1>(w, buf, t, a.tw);

  __syncthreads();
  if (active) {
#pragma unroll
    for (int e = 0; e < EH; ++e) {
      buf[t + T * e] = v[e];
      if constexpr (VAR && !TRANS) buf[t + T * e + NH] = w[e];
    }
  }
  __syncthreads();

  // epilogue: all global operands of a thread are loaded before the first store
  const double osc = (a.oscale && !a.row_scale) ? a.oscale[slice] : 1.0;
  const double esc = (a.extra && !a.row_scale) ? a.escale[slice] : 0.0;
  double dot = 0.0;
  {
    const double2 z2{0.0, 0.0};
    double2 sp[KL], ac[KL], ex[KL], dv[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int idx = tid + k * NT;
      const int li = ok[k] ? lpad(idx / P) * RS + idx % P : 0;
      sp[k] = lds[li];
      if constexpr (VAR && !TRANS) {
        const double2 s2 = lds[ok[k] ? lpad(idx / P + NH) * RS + idx % P : 0];
        const double2 dp = ld2(a.dplus + ge[k]), dm = ld2(a.dminus + ge[k]);
        sp[k] = double2{dp.x * sp[k].x + dm.x * s2.x, dp.y * sp[k].y + dm.y * s2.y};
      }
      ac[k] = ex[k] = dv[k] = z2;
    }
    if (a.acc) {
#pragma unroll
      for (int k = 0; k < KL; ++k) ac[k] = ld2(a.acc + sbase + ge[k]);
    }
    if (a.extra) {
#pragma unroll
      for (int k = 0; k < KL; ++k) ex[k] = ld2(a.extra + sbase + ge[k]);
    }
    if (a.dotv && a.dotv == a.extra) {
#pragma unroll
      for (int k = 0; k < KL; ++k) dv[k] = ex[k];
    } else if (a.dotv) {
#pragma unroll
      for (int k = 0; k < KL; ++k) dv[k] = ld2(a.dotv + sbase + ge[k]);
    }
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      if (ok[k]) {
        double o = osc, e = esc;
        if (a.row_scale) {
          const int row = (tid + k * NT) / P;
          o = a.oscale ? a.oscale[row] : 1.0;
          e = a.extra ? a.escale[row] : 0.0;
        }
        const double2 val{(a.s_sp * sp[k].x + ac[k].x) * o + e * ex[k].x,
                          (a.s_sp * sp[k].y + ac[k].y) * o + e * ex[k].y};
        st2(a.out + sbase + ge[k], val);
        dot += dv[k].x * val.x + dv[k].y * val.y;
      }
    }
  }
  if (a.dotv) {
    const double s = block_sum<NT>(dot);
    if (tid == 0) a.partial[bid] = s;
  }
}

template <int L, bool VAR, bool TRANS, int S, bool COL = false, bool PAD = false>
__global__ __launch_bounds__((YCfg<L, S>::NT)) void k_ypass(LinePassArgs a) {
  ypass_body<L, VAR, TRANS, S, COL, PAD>(a, blockIdx.x, gridDim.x);
}

// the batched twin
template <int L, bool VAR, bool TRANS, int S, bool COL = false, bool PAD = false>
__global__ __launch_bounds__((YCfg<L, S>::NT)) void k_ypass_b(BatchArgs<LinePassArgs> b) {
  const int i = batch_instance(b, blockIdx.x);
  ypass_body<L, VAR, TRANS, S, COL, PAD>(batch_local(b.args[i]), blockIdx.x - b.first[i],
                                         b.first[i + 1] - b.first[i]);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define FDE_FOR_EMBED_LENGTHS(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)


// Lengths whose constant-coefficient passes have batched twins: the FFT
// lengths of the batched workloads' grids (16 .. 512 nodes per axis)
constexpr bool batch_embed(int L) {
  return L == 32 || L == 48 || L == 64 || L == 96 || L == 128 || L == 192 || L == 256 || L == 384 || L == 512 ||
         L == 768 || L == 1024;
}
using LineBatchKernel = void (*)(BatchArgs<LinePassArgs>);

template <int L, bool VAR, bool TRANS, bool PAD>
static LineBatchKernel xpass_twin() {
  if constexpr (batch_embed(L) && !VAR && !PAD) return k_xpass_b<L, VAR, TRANS, PAD>;
  else return nullptr;
}

template <int L, bool VAR, bool TRANS, int S, bool COL, bool PAD>
static LineBatchKernel ypass_twin() {
  if constexpr (batch_embed(L) && !VAR && !COL && !PAD) return k_ypass_b<L, VAR, TRANS, S, COL, PAD>;
  else return nullptr;
}

template <int L, bool PAD>
static void xpass_launch(const LinePassArgs& a, bool tr, bool var, hipStream_t s, int blocks) {
  if (var) {
    if (tr) launch_pass(k_xpass<L, true, true, PAD>, xpass_twin<L, true, true, PAD>(), blocks, kLineThreads, s, a);
    else launch_pass(k_xpass<L, true, false, PAD>, xpass_twin<L, true, false, PAD>(), blocks, kLineThreads, s, a);
  } else {
    if (tr) launch_pass(k_xpass<L, false, true, PAD>, xpass_twin<L, false, true, PAD>(), blocks, kLineThreads, s, a);
    else launch_pass(k_xpass<L, false, false, PAD>, xpass_twin<L, false, false, PAD>(), blocks, kLineThreads, s, a);
  }
}

template <int L>
static hipError_t xpass_L(const LinePassArgs& a, bool tr, bool var, hipStream_t s, int* nb) {
  constexpr int E = default_E(L);
  constexpr int LPB = kLineThreads / (L / E);
  const int nlines = a.ny * a.nt;
  const int pairs = (nlines + 1) / 2;
  const int blocks = (pairs + LPB - 1) / LPB;
  if (nb) *nb = blocks;
  if (2 * a.nx == L) {
    xpass_launch<L, false>(a, tr, var, s, blocks);
  } else {
    if constexpr (padded_embedding(L)) {
      if (2 * a.nx > L) return hipErrorInvalidValue;
      xpass_launch<L, true>(a, tr, var, s, blocks);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int L, int S, bool PAD>
static void ypass_launch(const LinePassArgs& a, bool tr, bool var, hipStream_t s, int blocks) {
  using C = YCfg<L, S>;
  if (a.col_coef) {
    if (tr) launch_pass(k_ypass<L, false, true, S, true, PAD>, ypass_twin<L, false, true, S, true, PAD>(), blocks,
                        C::NT, s, a);
    else launch_pass(k_ypass<L, false, false, S, true, PAD>, ypass_twin<L, false, false, S, true, PAD>(), blocks,
                     C::NT, s, a);
  } else if (var) {
    if (tr) launch_pass(k_ypass<L, true, true, S, false, PAD>, ypass_twin<L, true, true, S, false, PAD>(), blocks,
                        C::NT, s, a);
    else launch_pass(k_ypass<L, true, false, S, false, PAD>, ypass_twin<L, true, false, S, false, PAD>(), blocks,
                     C::NT, s, a);
  } else {
    if (tr) launch_pass(k_ypass<L, false, true, S, false, PAD>, ypass_twin<L, false, true, S, false, PAD>(), blocks,
                        C::NT, s, a);
    else launch_pass(k_ypass<L, false, false, S, false, PAD>, ypass_twin<L, false, false, S, false, PAD>(), blocks,
                     C::NT, s, a);
  }
}

template <int L, int S>
static hipError_t ypass_LS(const LinePassArgs& a, bool tr, bool var, hipStream_t s, int* nb) {
  using C = YCfg<L, S>;
  const int tiles = (a.nx + 2 * C::P - 1) / (2 * C::P);
  const int blocks = tiles * a.nt;
  if (nb) *nb = blocks;
  if (2 * a.ny == L) {
    ypass_launch<L, S, false>(a, tr, var, s, blocks);
  } else {
    if constexpr (padded_embedding(L)) {
      if (2 * a.ny > L) return hipErrorInvalidValue;
      ypass_launch<L, S, true>(a, tr, var, s, blocks);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int L>
static hipError_t ypass_L(const LinePassArgs& a, bool tr, bool var, hipStream_t s, int* nb) {
  switch (a.tile) {
    case 1: return ypass_LS<L, 1>(a, tr, var, s, nb);
    case 2: return ypass_LS<L, 2>(a, tr, var, s, nb);
    default: return ypass_LS<L, 0>(a, tr, var, s, nb);
  }
}

int ypass_tile_width(int L, int variant) {
  switch (L) {
#define CASE(Lv) \
  case Lv: return variant == 1 ? YCfg<Lv, 1>::P : variant == 2 ? YCfg<Lv, 2>::P : YCfg<Lv, 0>::P;
    FDE_FOR_EMBED_LENGTHS(CASE)
#undef CASE
    default: return 0;
  }
}

hipError_t launch_xpass(const LinePassArgs& a, bool tr, bool var, hipStream_t s, int* nb) {
  switch (a.L) {
#define CASE(Lv) case Lv: return xpass_L<Lv>(a, tr, var, s, nb);
    FDE_FOR_EMBED_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_ypass(const LinePassArgs& a, bool tr, bool var, hipStream_t s, int* nb) {
  switch (a.L) {
#define CASE(Lv) case Lv: return ypass_L<Lv>(a, tr, var, s, nb);
    FDE_FOR_EMBED_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fde
