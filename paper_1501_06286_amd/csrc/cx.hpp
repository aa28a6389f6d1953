// Complex arithmetic and register-resident DFTs for the gfx950 kernels.
//
// The circular convolutions of the fast QMC product (Section 2.1, eq. (ZPa):
// Y' a = Z (P a) with Z circulant) are evaluated with FFTs.  Short DFTs
// (length 2^k <= 64, 3 x 2^k <= 96, 5 x 2^k <= 80) run entirely in one lane's registers
// with compile-time twiddle constants; longer transforms are built from them with LDS
// exchanges between lanes (kernels.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qmc {

// aligned to its full size so loads, stores and LDS accesses move both
// parts in one instruction
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {fmaT(a.x, b.x, -a.y * b.y), fmaT(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {fmaT(a.x, b.x, a.y * b.y), fmaT(a.y, b.x, -a.x * b.y)};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by +i or -i
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }

// ---------------------------------------------------------------------------
// compile-time twiddle constants: cos and sin of 2 pi k / 64, 192 and 320
// ---------------------------------------------------------------------------
constexpr double kTwoPi = 6.283185307179586476925286766559;

constexpr double poly_sin(double x) {  // |x| <= pi/4, Taylor series
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double poly_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// cos/sin of 2 pi num/den: reduce to the nearest quarter turn q and a
// remainder in [-1/8, 1/8] of a turn, then rotate by q quarter turns.
constexpr void sincos_turns(long num, long den, double& s, double& c) {
  num %= den;
  if (num < 0) num += den;
  long q = (4 * num + den / 2) / den;  // nearest quarter turn
  double rem = double(4 * num - q * den) / double(4 * den);
  double a = kTwoPi * rem;
  double s0 = poly_sin(a), c0 = poly_cos(a);
  switch (q & 3) {
    case 0: s = s0; c = c0; break;
    case 1: s = c0; c = -s0; break;
    case 2: s = -s0; c = -c0; break;
    default: s = -c0; c = s0; break;
  }
}
template <int D>
struct TwTab {
  double c[D];
  double s[D];
};
template <int D>
constexpr TwTab<D> make_tw() {
  TwTab<D> t{};
  for (int k = 0; k < D; ++k) sincos_turns(k, D, t.s[k], t.c[k]);
  return t;
}
// roots of unity of order 64 (every power-of-two length up to 64), 192 and
// 320 (the lengths 3 x 2^k and 5 x 2^k of the mixed-radix DFTs)
__device__ constexpr TwTab<64> kTw64 = make_tw<64>();
__device__ constexpr TwTab<192> kTw192 = make_tw<192>();
__device__ constexpr TwTab<320> kTw320 = make_tw<320>();

// a * W^num with W = exp(DIR * 2 pi i / den), den dividing 64, 192 or 320.
// num and den are compile-time constants after unrolling: exact quarter and
// eighth turns become sign changes and one shared 1/sqrt(2) scaling.
template <typename T, int DIR>
__device__ __forceinline__ cx<T> twiddle_const(cx<T> a, int num, int den) {
  num %= den;
  if (num == 0) return a;
  if ((4 * num) % den == 0) {
    int q = (4 * num) / den;  // 1, 2, 3 quarter turns
    if (q == 2) return {-a.x, -a.y};
    bool plus_i = (q == 1) == (DIR > 0);
    return plus_i ? mul_i(a) : mul_mi(a);
  }
  const int tab = 64 % den == 0 ? 0 : 192 % den == 0 ? 1 : 2;
  const int k = num * (tab == 0 ? 64 / den : tab == 1 ? 192 / den : 320 / den);
  const T c = (T)(tab == 0 ? kTw64.c[k] : tab == 1 ? kTw192.c[k] : kTw320.c[k]);
  const T sv = (T)(tab == 0 ? kTw64.s[k] : tab == 1 ? kTw192.s[k] : kTw320.s[k]);
  const T s = DIR > 0 ? sv : -sv;
  if ((8 * num) % den == 0) {
    // (+-1 +- i)/sqrt(2): rotate by a quarter-turn-free eighth turn
    const T h = (T)0.70710678118654752440;
    T cs = c > 0 ? (T)1 : (T)-1, ss = s > 0 ? (T)1 : (T)-1;
    // (a.x + i a.y)(cs + i ss) h
    T re = cs * a.x - ss * a.y;
    T im = cs * a.y + ss * a.x;
    return {re * h, im * h};
  }
  return {fmaT(a.x, c, -a.y * s), fmaT(a.x, s, a.y * c)};
}

// ---------------------------------------------------------------------------
// register DFT of length N (2^k <= 64, 3 x 2^k <= 96 or 5 x 2^k <= 80),
// natural order in and out, Stockham formulation: one radix-3 or radix-5
// stage first when 3 or 5 divides N, then radix-4 stages (and one radix-2
// stage when the power of two is an odd power).  DIR = -1: forward
// exp(-2 pi i jk/N); DIR = +1: inverse, unscaled.
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__device__ __forceinline__ void bfly2(cx<T>& a0, cx<T>& a1) {
  cx<T> t = a0 - a1;
  a0 = a0 + a1;
  a1 = t;
}
template <typename T, int DIR>
__device__ __forceinline__ void bfly4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
  t3 = (DIR < 0) ? mul_mi(t3) : mul_i(t3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

// length 3: with W = exp(DIR 2 pi i / 3) = -1/2 + DIR i sqrt(3)/2,
//   y0 = a0 + (a1 + a2),  y1,2 = a0 - (a1 + a2)/2 +- DIR i sqrt(3)/2 (a1 - a2)
template <typename T, int DIR>
__device__ __forceinline__ void bfly3(cx<T>& a0, cx<T>& a1, cx<T>& a2) {
  const T h = (T)0.86602540378443864676;  // sqrt(3)/2
  const cx<T> t1 = a1 + a2, t2 = a1 - a2;
  const cx<T> m = {fmaT(t1.x, (T)-0.5, a0.x), fmaT(t1.y, (T)-0.5, a0.y)};
  const cx<T> n = DIR > 0 ? cx<T>{-t2.y * h, t2.x * h} : cx<T>{t2.y * h, -t2.x * h};
  a0 = a0 + t1;
  a1 = m + n;
  a2 = m - n;
}

// length 5, from the symmetric pairs (a1, a4) and (a2, a3): with
// c_k = cos(2 pi k / 5), s_k = DIR sin(2 pi k / 5),
//   y0 = a0 + (a1 + a4) + (a2 + a3)
//   y1,4 = a0 + c1 (a1 + a4) + c2 (a2 + a3) +- i (s1 (a1 - a4) + s2 (a2 - a3))
//   y2,3 = a0 + c2 (a1 + a4) + c1 (a2 + a3) +- i (s2 (a1 - a4) - s1 (a2 - a3))
template <typename T, int DIR>
__device__ __forceinline__ void bfly5(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3, cx<T>& a4) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
  const T s1 = (T)(DIR * 0.95105651629515357212), s2 = (T)(DIR * 0.58778525229247312917);
  const cx<T> p1 = a1 + a4, m1 = a1 - a4, p2 = a2 + a3, m2 = a2 - a3;
  const cx<T> r1 = {fmaT(c2, p2.x, fmaT(c1, p1.x, a0.x)), fmaT(c2, p2.y, fmaT(c1, p1.y, a0.y))};
  const cx<T> r2 = {fmaT(c1, p2.x, fmaT(c2, p1.x, a0.x)), fmaT(c1, p2.y, fmaT(c2, p1.y, a0.y))};
  // i (s1 m1 + s2 m2) and i (s2 m1 - s1 m2)
  const cx<T> q1 = {fmaT(s1, m1.x, s2 * m2.x), fmaT(s1, m1.y, s2 * m2.y)};
  const cx<T> q2 = {fmaT(s2, m1.x, -s1 * m2.x), fmaT(s2, m1.y, -s1 * m2.y)};
  a0 = a0 + p1 + p2;
  a1 = {r1.x - q1.y, r1.y + q1.x};
  a4 = {r1.x + q1.y, r1.y - q1.x};
  a2 = {r2.x - q2.y, r2.y + q2.x};
  a3 = {r2.x + q2.y, r2.y - q2.x};
}

template <typename T, int N, int DIR, int Ns>
struct RegFftStage {
  static __device__ __forceinline__ void run(cx<T>* v) {
    if constexpr (Ns < N) {
      constexpr int r = (Ns == 1 && N % 3 == 0)   ? 3
                        : (Ns == 1 && N % 5 == 0) ? 5
                        : ((N / Ns) % 4 == 0)     ? 4
                                                  : 2;
      cx<T> out[N];
#pragma unroll
      for (int j = 0; j < N / r; ++j) {
        const int k = j % Ns;
        cx<T> a[r];
#pragma unroll
        for (int q = 0; q < r; ++q) a[q] = v[j + q * (N / r)];
#pragma unroll
        for (int q = 1; q < r; ++q) a[q] = twiddle_const<T, DIR>(a[q], q * k, Ns * r);
        if constexpr (r == 4)
          bfly4<T, DIR>(a[0], a[1], a[2], a[3]);
        else if constexpr (r == 3)
          bfly3<T, DIR>(a[0], a[1], a[2]);
        else if constexpr (r == 5)
          bfly5<T, DIR>(a[0], a[1], a[2], a[3], a[4]);
        else
          bfly2<T, DIR>(a[0], a[1]);
        const int base = (j / Ns) * Ns * r + k;
#pragma unroll
        for (int q = 0; q < r; ++q) out[base + q * Ns] = a[q];
      }
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = out[i];
      RegFftStage<T, N, DIR, Ns * r>::run(v);
    }
  }
};

template <typename T, int N, int DIR>
__device__ __forceinline__ void reg_fft(cx<T>* v) {
  constexpr int P = N % 3 == 0 ? N / 3 : N % 5 == 0 ? N / 5 : N;  // the power-of-two part
  static_assert(N >= 1 && (P & (P - 1)) == 0 &&
                    (N == P ? N <= 64 : N % 3 == 0 ? N <= 96 : N <= 80),
                "register DFT length");
  RegFftStage<T, N, DIR, 1>::run(v);
}

}  // namespace qmc
