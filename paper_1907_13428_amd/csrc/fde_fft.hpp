// Stockham mixed-radix line FFT for CDNA (gfx950), double or float.
//
// A line of length L is transformed by T = L/E threads; thread t holds the
// elements x[t + T*e], e = 0..E-1, in registers.  Stage s (radix R, Ls = the
// product of the earlier radices) performs E/R radix-R butterflies per
// thread: butterfly b = t + T*q takes x[b + m*L/R] (registers q + m*E/R),
// applies the twiddles w_{Ls*R}^{j*m} (j = b mod Ls) and writes its outputs
// to k*Ls*R + j + m*Ls (k = b div Ls).  Because every stage reads the set
// {t + T*e}, intermediate stages exchange through LDS and the last stage's
// outputs land in the same registers in natural order: after the forward
// transform thread t holds X[t + T*e].  A pointwise spectral product can
// therefore be applied in registers and followed directly by the inverse.
//
// When the T threads of a line lie in one wavefront (T <= 64) the LDS
// exchanges are ordered by wavefront-scope fences instead of block barriers,
// so independent lines in one block never wait for each other.
//
// The FFT is the O(N log N) primitive of Table 1 (Sec. 5): the Toeplitz
// products use it through a 2n circulant embedding, the multilevel circulant
// preconditioner through plain length-n transforms per axis.
#pragma once
#include <hip/hip_runtime.h>

namespace fde {

template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename R> using cplx = typename cvec<R>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V, typename R> __device__ __forceinline__ V cscale(V a, R s) { return V{a.x * s, a.y * s}; }
// multiply by SIGN * i
template <int SIGN, typename V> __device__ __forceinline__ V cmul_si(V a) {
  return SIGN > 0 ? V{-a.y, a.x} : V{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// small DFTs in registers: X_k = sum_m a_m exp(SIGN 2 pi i k m / R)
// ---------------------------------------------------------------------------
template <int R, int SIGN, typename V> struct Dft;

template <int SIGN, typename V> struct Dft<2, SIGN, V> {
  __device__ __forceinline__ static void run(V* a) {
    V t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};

template <int SIGN, typename V> struct Dft<3, SIGN, V> {
  __device__ __forceinline__ static void run(V* a) {
    using R = decltype(a[0].x);
    const R h = R(0.8660254037844386467637231707529361834714);  // sqrt(3)/2
    V s = cadd(a[1], a[2]);
    V d = csub(a[1], a[2]);
    V m = V{a[0].x - R(0.5) * s.x, a[0].y - R(0.5) * s.y};
    V r = cmul_si<SIGN>(cscale(d, h));
    a[0] = cadd(a[0], s);
    a[1] = cadd(m, r);
    a[2] = csub(m, r);
  }
};

template <int SIGN, typename V> struct Dft<4, SIGN, V> {
  __device__ __forceinline__ static void run(V* a) {
    V s0 = cadd(a[0], a[2]);
    V d0 = csub(a[0], a[2]);
    V s1 = cadd(a[1], a[3]);
    V d1 = cmul_si<SIGN>(csub(a[1], a[3]));
    a[0] = cadd(s0, s1);
    a[2] = csub(s0, s1);
    a[1] = cadd(d0, d1);
    a[3] = csub(d0, d1);
  }
};

// 5-point DFT: with t1 = a1 + a4, t2 = a2 + a3, t3 = a1 - a4, t4 = a2 - a3 and
// c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5):
//   X0 = a0 + t1 + t2
//   X1, X4 = a0 + c1 t1 + c2 t2 +- SIGN i (s1 t3 + s2 t4)
//   X2, X3 = a0 + c2 t1 + c1 t2 +- SIGN i (s2 t3 - s1 t4)
template <int SIGN, typename V> struct Dft<5, SIGN, V> {
  __device__ __forceinline__ static void run(V* a) {
    using R = decltype(a[0].x);
    const R c1 = R(0.3090169943749474241022934171828190588602);   // cos(2 pi / 5)
    const R c2 = R(-0.8090169943749474241022934171828190588602);  // cos(4 pi / 5)
    const R s1 = R(0.9510565162951535721164393333793821434057);   // sin(2 pi / 5)
    const R s2 = R(0.5877852522924731291687059546390727685977);   // sin(4 pi / 5)
    const V t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const V t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
    const V m1 = V{a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y};
    const V m2 = V{a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y};
    const V n1 = cmul_si<SIGN>(V{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
    const V n2 = cmul_si<SIGN>(V{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(m1, n1);
    a[4] = csub(m1, n1);
    a[2] = cadd(m2, n2);
    a[3] = csub(m2, n2);
  }
};

// multiply by exp(SIGN i pi k / 4) for k = 1, 3 (k = 2 is SIGN i)
template <int SIGN, typename V> __device__ __forceinline__ V rot8_1(V o) {
  using R = decltype(o.x);
  const R r2 = R(0.7071067811865475244008443621048490392848);
  return V{(o.x - SIGN * o.y) * r2, (o.y + SIGN * o.x) * r2};
}
template <int SIGN, typename V> __device__ __forceinline__ V rot8_3(V o) {
  using R = decltype(o.x);
  const R r2 = R(0.7071067811865475244008443621048490392848);
  return V{(-o.x - SIGN * o.y) * r2, (-o.y + SIGN * o.x) * r2};
}

template <int SIGN, typename V> struct Dft<8, SIGN, V> {
  __device__ __forceinline__ static void run(V* a) {
    V e[4] = {a[0], a[2], a[4], a[6]};
    V o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, SIGN, V>::run(e);
    Dft<4, SIGN, V>::run(o);
    const V o1 = rot8_1<SIGN>(o[1]);
    const V o2 = cmul_si<SIGN>(o[2]);
    const V o3 = rot8_3<SIGN>(o[3]);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  }
};

// 16 = 4 x 4: DFT-4 over m1 (inputs 4 m1 + m2), twiddle w16^{m2 k1}, DFT-4 over m2
template <int SIGN, typename V> struct Dft<16, SIGN, V> {
  __device__ __forceinline__ static void run(V* a) {
    using R = decltype(a[0].x);
    const R c1 = R(0.9238795325112867561281831893967882868224);  // cos(pi/8)
    const R s1 = R(0.3826834323650897717284599840303988667613);  // sin(pi/8)
    V b[4][4];
#pragma unroll
    for (int m2 = 0; m2 < 4; ++m2) {
      V col[4] = {a[m2], a[4 + m2], a[8 + m2], a[12 + m2]};
      Dft<4, SIGN, V>::run(col);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) b[m2][k1] = col[k1];
    }
    // twiddles w16^{m2 k1} = exp(SIGN 2 pi i m2 k1 / 16)
#pragma unroll
    for (int m2 = 1; m2 < 4; ++m2) {
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1) {
        const int p = (m2 * k1) & 15;  // 1, 2, 3, 4, 6, 9
        V x = b[m2][k1];
        V r;
        switch (p) {
          case 1: r = V{x.x * c1 - SIGN * x.y * s1, x.y * c1 + SIGN * x.x * s1}; break;
          case 2: r = rot8_1<SIGN>(x); break;
          case 3: r = V{x.x * s1 - SIGN * x.y * c1, x.y * s1 + SIGN * x.x * c1}; break;
          case 4: r = cmul_si<SIGN>(x); break;
          case 6: r = rot8_3<SIGN>(x); break;
          default: /* 9: exp(SIGN i 9 pi/8) = -cos(pi/8) - SIGN i sin(pi/8) */
            r = V{-x.x * c1 + SIGN * x.y * s1, -x.y * c1 - SIGN * x.x * s1};
            break;
        }
        b[m2][k1] = r;
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      V row[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
      Dft<4, SIGN, V>::run(row);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = row[k2];
    }
  }
};

// ---------------------------------------------------------------------------
// radix plan: stage radices from {16, 8, 4, 5, 3, 2}, each dividing E
// ---------------------------------------------------------------------------
constexpr int pick_radix(int rem, int E) {
  return (rem % 16 == 0 && E % 16 == 0) ? 16
         : (rem % 8 == 0 && E % 8 == 0) ? 8
         : (rem % 4 == 0 && E % 4 == 0) ? 4
         : (rem % 5 == 0 && E % 5 == 0) ? 5
         : (rem % 3 == 0 && E % 3 == 0) ? 3
         : (rem % 2 == 0 && E % 2 == 0) ? 2
                                        : 0;
}

// elements per thread for a line of length L (radix-16 stages for 128 and
// 256 points; 8 elements elsewhere, so that long lines keep their register
// footprint low and use 2 or 4 wavefronts with block barriers; lengths with
// a factor 5 take 20 or 10, which hold the radices 4, 5 and 2 of 50, 80,
// 100 and 160; 16 and 48 points take 4 threads per line and 24 points 2, so
// that the passes over small grids spread over more blocks)
constexpr int default_E(int L) {
  return (L % 5 == 0) ? ((L % 20 == 0) ? 20 : 10)
         : (L == 24 || L == 48) ? 12
         : (L % 3 == 0) ? (L >= 24 ? 24 : L)
         : (L == 16) ? 4
         : (L <= 16)  ? L
         : (L == 128) ? 16
                                  : 8;
}

// padded LDS index: one spare slot per 8 keeps power-of-two strides off a bank
__device__ __forceinline__ int lpad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lpad_size(int L) { return L + (L >> 3) + 1; }

// LDS view of one line: element i lives at base[lpad(i) * rs]
template <typename V> struct LineLds {
  V* base;
  int rs;
  __device__ __forceinline__ V& operator[](int i) const { return base[lpad(i) * rs]; }
};

// The T threads of a line lie in one wavefront when T divides 64 (lines of a
// block start at multiples of T); otherwise a line may straddle two
// wavefronts and its exchanges need block barriers.
__host__ __device__ constexpr bool line_in_wave(int T) { return T <= 64 && 64 % T == 0; }

// Ordering of an LDS exchange among the threads of one line.
template <bool WAVE> __device__ __forceinline__ void line_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// twiddles w^m, m = 1..R-1, w = exp(SIGN 2 pi i j / (Ls R)), from a few table
// loads (powers of two of w) and complex products
template <int R, int SIGN, typename V>
__device__ __forceinline__ void stage_twiddles(V (&w)[R], const V* __restrict__ tw, int idx) {
  auto ld = [&](int k) {
    V x = tw[k];
    if (SIGN > 0) x.y = -x.y;
    return x;
  };
  w[0] = V{1, 0};
  if constexpr (R == 2) {
    w[1] = ld(idx);
  } else if constexpr (R == 3) {
    w[1] = ld(idx);
    w[2] = ld(2 * idx);
  } else if constexpr (R == 4) {
    w[1] = ld(idx);
    w[2] = ld(2 * idx);
    w[3] = cmul(w[1], w[2]);
  } else if constexpr (R == 5) {
    w[1] = ld(idx);
    w[2] = ld(2 * idx);
    w[3] = cmul(w[1], w[2]);
    w[4] = cmul(w[2], w[2]);
  } else if constexpr (R == 8) {
    w[1] = ld(idx);
    w[2] = ld(2 * idx);
    w[4] = ld(4 * idx);
    w[3] = cmul(w[1], w[2]);
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
  } else {
    static_assert(R == 16, "radix");
    w[1] = ld(idx);
    w[2] = ld(2 * idx);
    w[4] = ld(4 * idx);
    w[8] = ld(8 * idx);
    w[3] = cmul(w[1], w[2]);
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
    w[9] = cmul(w[8], w[1]);
    w[10] = cmul(w[8], w[2]);
    w[11] = cmul(w[8], w[3]);
    w[12] = cmul(w[8], w[4]);
    w[13] = cmul(w[8], w[5]);
    w[14] = cmul(w[8], w[6]);
    w[15] = cmul(w[8], w[7]);
  }
}

template <int L, int E, int Ls, int SIGN, typename V>
struct Stages {
  static constexpr int rem = L / Ls;
  static constexpr int R = pick_radix(rem, E);
  static_assert(R != 0, "FFT length not factorable with radices dividing E");
  static constexpr int T = L / E;
  static constexpr int Q = E / R;
  static constexpr bool LAST = (Ls * R == L);
  static constexpr bool WAVE = line_in_wave(T);

  __device__ __forceinline__ static void run(V (&v)[E], LineLds<V> lds, int t, const V* __restrict__ tw) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = t + T * q;
      const int j = b % Ls;
      const int k = b / Ls;
      V x[R];
#pragma unroll
      for (int m = 0; m < R; ++m) x[m] = v[q + m * Q];
      if constexpr (Ls > 1) {
        V w[R];
        stage_twiddles<R, SIGN>(w, tw, j * (L / (Ls * R)));
#pragma unroll
        for (int m = 1; m < R; ++m) x[m] = cmul(x[m], w[m]);
      }
      Dft<R, SIGN, V>::run(x);
      if constexpr (LAST) {
        // butterfly q reads and writes the same registers q + m*Q
#pragma unroll
        for (int m = 0; m < R; ++m) v[q + m * Q] = x[m];
      } else {
#pragma unroll
        for (int m = 0; m < R; ++m) lds[k * Ls * R + j + m * Ls] = x[m];
      }
    }
    if constexpr (!LAST) {
      line_sync<WAVE>();
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = lds[t + T * e];
      line_sync<WAVE>();
      Stages<L, E, Ls * R, SIGN, V>::run(v, lds, t, tw);
    }
  }
};

// terminal specialisation guard (never instantiated with Ls == L)
template <int L, int E, int SIGN, typename V>
struct Stages<L, E, L, SIGN, V> {
  __device__ __forceinline__ static void run(V (&)[E], LineLds<V>, int, const V*) {}
};

// Unnormalised DFT of the line held as v[e] = x[t + T e]; afterwards
// v[e] = X[t + T e].  SIGN = -1 forward, +1 inverse.  `tw` is the length-L
// table exp(-2 pi i m / L).  When the line's threads do not lie in one
// wavefront (line_in_wave) every thread of the block must call it (block
// barriers); otherwise every lane of the line's wavefront must.
template <int L, int E, int SIGN, typename V>
__device__ __forceinline__ void line_fft(V (&v)[E], LineLds<V> lds, int t, const V* __restrict__ tw) {
  Stages<L, E, 1, SIGN, V>::run(v, lds, t, tw);
}

}  // namespace fde
