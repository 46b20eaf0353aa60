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

template <int SIGN, typename V> struct Dft<8, SIGN, V> {
  __device__ __forceinline__ static void run(V* a) {
    using R = decltype(a[0].x);
    const R r2 = R(0.7071067811865475244008443621048490392848);  // 1/sqrt(2)
    V e[4] = {a[0], a[2], a[4], a[6]};
    V o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, SIGN, V>::run(e);
    Dft<4, SIGN, V>::run(o);
    // o_k *= exp(SIGN i pi k / 4)
    V o1 = V{(o[1].x - SIGN * o[1].y) * r2, (o[1].y + SIGN * o[1].x) * r2};
    V o2 = cmul_si<SIGN>(o[2]);
    V o3 = V{(-o[3].x - SIGN * o[3].y) * r2, (-o[3].y + SIGN * o[3].x) * r2};
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

// ---------------------------------------------------------------------------
// radix plan: stage radices from {8, 4, 3, 2}, each dividing E
// ---------------------------------------------------------------------------
constexpr int pick_radix(int rem, int E) {
  return (rem % 8 == 0 && E % 8 == 0) ? 8
         : (rem % 4 == 0 && E % 4 == 0) ? 4
         : (rem % 3 == 0 && E % 3 == 0) ? 3
         : (rem % 2 == 0 && E % 2 == 0) ? 2
                                        : 0;
}

// elements per thread for a line of length L
constexpr int default_E(int L) {
  return (L % 3 == 0) ? (L >= 24 ? 24 : L) : (L >= 8 ? 8 : L);
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

template <int L, int E, int Ls, int SIGN, typename V>
struct Stages {
  static constexpr int rem = L / Ls;
  static constexpr int R = pick_radix(rem, E);
  static_assert(R != 0, "FFT length not factorable with radices dividing E");
  static constexpr int T = L / E;
  static constexpr int Q = E / R;
  static constexpr bool LAST = (Ls * R == L);

  __device__ __forceinline__ static void run(V (&v)[E], LineLds<V> lds, int t, const V* __restrict__ tw) {
    V out[E];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = t + T * q;
      const int j = b % Ls;
      const int k = b / Ls;
      V x[R];
#pragma unroll
      for (int m = 0; m < R; ++m) x[m] = v[q + m * Q];
      if (Ls > 1) {
#pragma unroll
        for (int m = 1; m < R; ++m) {
          V w = tw[j * m * (L / (Ls * R))];
          if (SIGN > 0) w.y = -w.y;
          x[m] = cmul(x[m], w);
        }
      }
      Dft<R, SIGN, V>::run(x);
      if (LAST) {
#pragma unroll
        for (int m = 0; m < R; ++m) out[q + m * Q] = x[m];
      } else {
#pragma unroll
        for (int m = 0; m < R; ++m) lds[k * Ls * R + j + m * Ls] = x[m];
      }
    }
    if constexpr (LAST) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = out[e];
    } else {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = lds[t + T * e];
      __syncthreads();
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
// table exp(-2 pi i m / L).  Every thread of the block must call it (it
// contains block barriers when L needs more than one stage).
template <int L, int E, int SIGN, typename V>
__device__ __forceinline__ void line_fft(V (&v)[E], LineLds<V> lds, int t, const V* __restrict__ tw) {
  Stages<L, E, 1, SIGN, V>::run(v, lds, t, tw);
}

}  // namespace fde
