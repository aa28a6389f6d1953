// Device bodies of the hot-path kernels, shared by the single-product
// launches (conv.hip) and the batched persistent launches (batch.hip).
// Each body takes its block coordinates and its LDS storage as arguments.
#pragma once
#include <type_traits>
#include "cx.hpp"
#include "internal.hpp"

namespace qmc {

// thread id for a body inside a persistent loop: the empty asm makes the
// value opaque per iteration so the compiler recomputes thread-dependent
// indices instead of keeping them live across iterations
__device__ __forceinline__ int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// workgroups are dealt round-robin to the 8 XCDs; map them so that a run of
// consecutive logical ids lands on one XCD (shared L2 for the same pair)
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
  const int64_t X = 8;
  const int64_t q = G / X, rem = G % X;
  const int64_t xcd = b % X, idx = b / X;
  return (xcd < rem) ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

// two (four) adjacent values of T as one vector access
template <typename T>
using vec2_t = T __attribute__((ext_vector_type(2)));
template <typename T>
using vec4_t = T __attribute__((ext_vector_type(4)));

// whether element pairs (2k, 2k+1) of every row of a row-major matrix are
// aligned for one vector access
template <typename T>
__device__ __forceinline__ bool pairs_aligned(const T* p, int64_t ld) {
  return (ld % 2 == 0) && (reinterpret_cast<uintptr_t>(p) % (2 * sizeof(T)) == 0);
}

// ---------------------------------------------------------------------------
// T: aT[pair][u] = sum over the rows j of item u of
//                  A[j, 2 pair] + i A[j, 2 pair + 1]   (0 for padding)
// ---------------------------------------------------------------------------
template <typename T>
struct CollapseSmem {
  cx<T> sm[64][17];
};

// acc + the rows idx[k], k in [k0, k1), added in increasing k (the fixed
// summation order); the loads go out 8 rows at a time, so an item carrying
// many rows (repeated exponents) waits for memory once per 8 rows, not per row
template <typename T, typename Row>
__device__ __forceinline__ cx<T> add_rows(cx<T> acc, const int32_t* __restrict__ idx, int32_t k0,
                                          int32_t k1, const Row& row) {
  constexpr int B = 8;
  int32_t k = k0;
  for (; k + B <= k1; k += B) {
    int32_t j[B];
#pragma unroll
    for (int i = 0; i < B; ++i) j[i] = idx[k + i];
    cx<T> r[B];
#pragma unroll
    for (int i = 0; i < B; ++i) r[i] = row(j[i]);
#pragma unroll
    for (int i = 0; i < B; ++i) acc = acc + r[i];
  }
  for (; k < k1; ++k) acc = acc + row(idx[k]);
  return acc;
}

template <typename T>
__device__ __forceinline__ void collapse_body(const T* __restrict__ A, int64_t lda, int64_t t,
                                              int64_t P, const int32_t* __restrict__ it_ptr,
                                              const int32_t* __restrict__ it_jl, int64_t Upad,
                                              cx<T>* __restrict__ aT, int64_t bx, int64_t by,
                                              CollapseSmem<T>& S, int tid) {
  auto& sm = S.sm;
  const int64_t u0 = bx * 64, p0 = by * 16;
  const int pl = tid & 15;
  const int64_t c = 2 * (p0 + pl);  // this thread's columns c, c + 1
  const bool pc = p0 + pl < P, both = c + 1 < t;
  const bool v2 = both && pairs_aligned(A, lda);
  auto row_pair = [&](int32_t j) -> cx<T> {
    const T* row = A + (int64_t)j * lda + c;
    if (v2) {
      const vec2_t<T> w = *reinterpret_cast<const vec2_t<T>*>(row);
      return {w.x, w.y};
    }
    return {row[0], both ? row[1] : (T)0};
  };
  // the four items of this thread: bounds, then each item's first row, then
  // the rest (an item has one row unless exponents collide), so the loads of
  // the four items are in flight together
  int32_t kb[4], ke[4], j0[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t u = u0 + (tid >> 4) + 16 * i;
    const bool ok = u < Upad && pc;
    kb[i] = ok ? it_ptr[u] : 0;
    ke[i] = ok ? it_ptr[u + 1] : 0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) j0[i] = kb[i] < ke[i] ? it_jl[kb[i]] : -1;
  cx<T> v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = j0[i] >= 0 ? row_pair(j0[i]) : cx<T>{(T)0, (T)0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (kb[i] + 1 < ke[i]) v[i] = add_rows<T>(v[i], it_jl, kb[i] + 1, ke[i], row_pair);
    sm[(tid >> 4) + 16 * i][pl] = v[i];
  }
  __syncthreads();
  const int ul = tid & 63;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int pl2 = (tid >> 6) + 4 * i;
    const int64_t u = u0 + ul, p = p0 + pl2;
    if (u < Upad && p < P) aT[p * Upad + u] = sm[ul][pl2];
  }
}

// ---------------------------------------------------------------------------
// F: one (outer frequency w2, pair) per R^2 threads.
//
// The on-chip transform has length M1 = R^3, index e1 = a + R b + R^2 c and
// frequency w1 = f + R g + R^2 h (a..h in [0, R)); every thread keeps R
// values in registers and the data moves through one LDS buffer between the
// three register DFTs of each direction:
//   forward  thread e1'=(a + R b): DFT over c -> f, * W_{M1}^{e1' f}
//            thread a + R f:       DFT over b -> g, * W_{R^2}^{a g}
//            thread g + R f:       DFT over a -> h      => X[f + R g + R^2 h]
//   product  * Hs[w2][w1]  (the spectrum, with 1/M folded in)
//   inverse  thread g + R f:       IDFT over h -> a, * conj W_{R^2}^{a g}
//            thread a + R f:       IDFT over g -> b, * conj W_M^{e1' (f M2 + w2)}
//            thread e1':           IDFT over f -> c, * conj W_M^{R^2 c w2}
// The middle four steps keep f fixed, so their exchanges stay inside a
// group of R lanes of one wavefront.
// The conj W_M^{e1' w2} factor is the outer-step twiddle of M = M1 * M2.
// ---------------------------------------------------------------------------
// Epilogue of the forward product (Sections 3.2 and 3.3): entry (n, c) of
// X = Y A becomes scale[c] * f(bias[c] + X[n, c]), f = identity (the
// stiffness entries a_{0,k,l} + Y a_{k,l} of eq. (Ya)) or exp (the
// log-normal coefficient exp(Psi^ + Y Psi) of eqs. (fastB), (eq_as)).
// kind 0 leaves X as it is; a null bias is 0 and a null scale is 1.
template <typename T>
struct Epi {
  int kind = 0;
  const T* bias = nullptr;
  const T* scale = nullptr;
};
// internal epilogue kind: the value is added to what the output entry holds
// (the blocks of a lattice rule with non-prime N that share output rows, or
// output rows of dA, add up); bias and scale unused
constexpr int EPI_ACC = 3;
// FP32: the hardware base-2 exponential (relative error a few ulp times
// |v|, far inside the FP32 product's tolerance); FP64: the full-precision one
__device__ __forceinline__ float exp_t(float v) { return __expf(v); }
__device__ __forceinline__ double exp_t(double v) { return exp(v); }

// the epilogue of one thread's two columns col, col + 1 < t (loaded once;
// columns at or beyond t are not read); row 0 gets it from k_epi_row0
template <typename T>
struct EpiCols {
  int kind;
  T b0 = 0, b1 = 0, s0 = 1, s1 = 1;
  __device__ __forceinline__ EpiCols(const Epi<T>& e, int64_t col, int64_t t) : kind(e.kind) {
    if (kind != 0 && col < t) {
      const bool both = col + 1 < t;
      if (e.bias) {
        b0 = e.bias[col];
        if (both) b1 = e.bias[col + 1];
      }
      if (e.scale) {
        s0 = e.scale[col];
        if (both) s1 = e.scale[col + 1];
      }
    }
  }
  __device__ __forceinline__ T f(T v, T b, T s) const {
    if (kind == 0) return v;
    T z = b + v;
    if (kind == 2) z = exp_t(z);
    return s * z;
  }
  __device__ __forceinline__ T f0(T v) const { return f(v, b0, s0); }
  __device__ __forceinline__ T f1(T v) const { return f(v, b1, s1); }
};

// orders this wavefront's LDS accesses before and after the call (LDS
// operations of one wavefront complete in issue order)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// rounds of the sparse front whose loads are issued together (a shorter
// tail batch covers the rest)
constexpr int MID_RB = 8;

// Per-thread tables keep each thread's consecutive values in adjacent
// pairs, so one 16-byte load (FP32) brings two complex values: value h of
// thread q in a table of Q threads is stored at
//   (h / PP) * PP * Q + PP * q + h % PP,   PP = 2 (1 when a thread has one value).
__host__ __device__ constexpr int pair_pp(int R) { return R >= 2 ? 2 : 1; }
__host__ __device__ constexpr int64_t paired_index(int64_t h, int64_t q, int64_t Q, int PP) {
  return (h / PP) * PP * Q + PP * q + h % PP;
}

template <typename T>
struct alignas(4 * sizeof(T)) cx2 {
  cx<T> a, b;
};

// v[h] = table value h of thread q, h = 0..R-1
template <typename T, int R>
__device__ __forceinline__ void load_paired(cx<T> (&v)[R], const cx<T>* __restrict__ base, int q,
                                            int Q) {
  if constexpr (R >= 2) {
#pragma unroll
    for (int h = 0; h < R; h += 2) {
      const cx2<T> p = *reinterpret_cast<const cx2<T>*>(base + (int64_t)h * Q + 2 * q);
      v[h] = p.a;
      v[h + 1] = p.b;
    }
  } else {
    v[0] = base[q];
  }
}

// x[bb] *= value bb of thread q's row of the inverse middle step's twiddles
// (conj W_M^{(a + R bb)(f M2 + w2)}, a paired table).  REC (FP64): the values
// are powers of one root, made by recurrence from values 0 and 1 (adjacent
// in the row; their ratio is the root) instead of R loads
template <typename T, int R, bool REC>
__device__ __forceinline__ void inverse_step_twiddles(cx<T> (&x)[R], const cx<T>* __restrict__ row,
                                                      int q, int Q) {
  if constexpr (REC) {
    const cx2<T> kk = *reinterpret_cast<const cx2<T>*>(row + 2 * q);
    const cx<T> zb = cmulc(kk.b, kk.a);
    cx<T> wb = kk.b;
    x[0] = cmul(x[0], kk.a);
    x[1] = cmul(x[1], kk.b);
#pragma unroll
    for (int bb = 2; bb < R; ++bb) {
      wb = cmul(wb, zb);
      x[bb] = cmul(x[bb], wb);
    }
  } else {
    cx<T> tw[R];
    load_paired<T, R>(tw, row, q, Q);
#pragma unroll
    for (int bb = 0; bb < R; ++bb) x[bb] = cmul(x[bb], tw[bb]);
  }
}

template <int R>
struct MidShape {
  static constexpr int Q = R * R;                  // threads per transform
  static constexpr int TPB = Q >= 64 ? 1 : 64 / Q; // transforms per block
  static constexpr int BLOCK = Q * TPB;
  static constexpr int BUFN = Q * (R + 1);         // LDS complex per transform (>= R^3 + 1)
  static constexpr int G = Q < 64 ? Q : 64;        // sparse-front round width
  static constexpr int F = Q / G;                  // front slices per transform (owners of e1 mod F)
};

// waves per SIMD the fused kernel is compiled for: the LDS of R = 16
// admits four FP32 or two FP64 workgroups per CU and the register budget
// follows (128 or 256 per lane); FP64 at R = 8 needs more than 128
template <typename T, int R>
constexpr int mid_waves() {
  return sizeof(T) == 8 ? (R == 16 ? 2 : R == 8 ? 3 : 4) : 4;
}

// outer lengths whose twiddles the sparse front with bucket twiddles keeps
// in LDS (longer ones are read from the global table)
constexpr int MID_TW2 = 256;

template <typename T, int R>
struct MidSmem {
  cx<T> lds[MidShape<R>::TPB * MidShape<R>::BUFN];
  cx<T> wr2[R * (R + 1)];  // W_{R^2}^{i j} at [i][j], rows padded to R + 1
  cx<T> tw2[MID_TW2];      // sparse front with bucket twiddles: conj W_{M2}^k, k < M2
};

// b: logical block of this product (w2 = b mod M2, pair group = b / M2).
// BTW (sparse front only, M2 a power of two): bucket twiddles.  The slot twiddle of an item,
// W_M^{slot w2} with slot = e1 + M1 e2, splits as W_M^{e1 w2} W_{M2}^{e2 w2}:
// the items take the short factor from a table of M2 values (it_e2: e2 per
// item, twb: conj W_{M2}^k) and every bucket e1 the long one once, after the
// sums (as the dense front does), instead of loading a twiddle per item.
template <typename T, int R, bool SPARSE, bool BTW = false>
__device__ __forceinline__ void middle_body(
    const cx<T>* __restrict__ src,      // SPARSE: aT [pair][Upad]; dense: B [pair][M2][M1]
    int64_t Upad, int64_t rounds, const uint16_t* __restrict__ it_e1,
    const cx<T>* __restrict__ twit, const cx<T>* __restrict__ twf1,
    const cx<T>* __restrict__ twf2, const cx<T>* __restrict__ Hs,
    const cx<T>* __restrict__ twi3, const cx<T>* __restrict__ two, int64_t M2, int64_t P,
    cx<T>* __restrict__ C, T* __restrict__ X, int64_t t, T phi0, int64_t b, MidSmem<T, R>& SM,
    int tid, bool nt_c = false, const uint16_t* __restrict__ it_e2 = nullptr,
    const cx<T>* __restrict__ twb = nullptr) {
  typedef MidShape<R> S;
  constexpr int Q = S::Q, M1 = R * R * R, PB = R * (R + 1);
  cx<T>* lds = SM.lds;
  // b = w2 + M2 pg: mask and shift when M2 is a power of two, else one
  // 32-bit division (M2 = 3 x 2^k or 5 x 2^k; b is below the grid size)
  int64_t w2, pg;
  if ((M2 & (M2 - 1)) == 0) {
    w2 = b & (M2 - 1);
    pg = b >> __builtin_ctzll((unsigned long long)M2);
  } else {
    pg = (int64_t)((uint32_t)b / (uint32_t)M2);
    w2 = b - pg * M2;
  }
  const int tr = tid / Q, q = tid % Q;
  const int64_t pair = pg * S::TPB + tr;
  const bool active = pair < P;
  cx<T>* buf = lds + tr * S::BUFN;
  const cx<T> zero = {(T)0, (T)0};
  cx<T> x[R];

  // The first twiddles and the spectrum are loaded ahead of use, so their
  // latency hides behind the front and the steps in between.
  cx<T> tw_a[R], hv[R];
  // FP64: the step twiddles of a thread are powers of one root (W_{M1}^{q f}
  // over f; conj W_M^{(a + R bb)(f M2 + w2)} over bb), made by recurrence from
  // one or two table values instead of R loads each
  constexpr bool TW_REC = sizeof(T) == 8 && R >= 2;
  cx<T> za;
  if constexpr (SPARSE) {  // the dense front's loads come first
    if constexpr (TW_REC) za = twf1[paired_index(1, q, Q, pair_pp(R))];
    else load_paired<T, R>(tw_a, twf1, q, Q);
  }
  // the R x R roots W_{R^2}^{a g} of the middle steps live in LDS (first
  // read after the barriers of step 1); twf2 holds value g of thread a
  for (int i = tid; i < R * R; i += S::BLOCK)
    SM.wr2[(i % R) * (R + 1) + i / R] = twf2[paired_index(i / R, i % R, R, pair_pp(R))];
  // bucket twiddles: the short factors in LDS (read after the front's first
  // barrier); longer outer lengths read the global table
  const bool tw2_lds = BTW && M2 <= MID_TW2;
  if constexpr (BTW) {
    if (tw2_lds)
      for (int i = tid; i < M2; i += S::BLOCK) SM.tw2[i] = twb[i];
  }

  // ---- front: B[e1] for this w2, in registers of thread e1' = q ----------
  if constexpr (SPARSE) {
    for (int i = q; i <= M1; i += Q) buf[i] = zero;
    __syncthreads();
    const int fo = q / S::G, ln = q % S::G;
    // every lane owns whole buckets (all items of a residue e1, in a fixed
    // order): it sums a bucket in registers and stores it once when the
    // next item belongs to another bucket.  The item count per lane is a
    // multiple of the pairing PP; padding items carry e1 = M1 (the spare
    // slot).
    // Inactive transforms read pair 0 and store nothing that is used.
    const cx<T>* av = src + (active ? pair : 0) * Upad;
    const cx<T>* tw = BTW ? nullptr : twit + w2 * Upad;
    const int64_t m2mask = M2 - 1;
    const int nr = (int)rounds;
    int cur = M1;
    cx<T> acc = zero;
    constexpr int PP = pair_pp(R);
    // NB rounds from r0: all loads first, then the bucket sums
    auto rounds_from = [&](int r0, auto nb) {
      constexpr int NB = decltype(nb)::value;
      int e1[NB];
      cx<T> v[NB], w[NB];
#pragma unroll
      for (int i = 0; i < NB; i += PP) {
        const int u = (((r0 + i) / PP * S::F + fo) * S::G + ln) * PP;  // items k, k+1 adjacent
        if constexpr (PP == 2) {
          // two 16-bit residues in one 32-bit load (u is even)
          const uint32_t ee = *reinterpret_cast<const uint32_t*>(it_e1 + u);
          const cx2<T> vv = *reinterpret_cast<const cx2<T>*>(av + u);
          e1[i] = (int)(ee & 0xffffu);
          e1[i + 1] = (int)(ee >> 16);
          v[i] = vv.a;
          v[i + 1] = vv.b;
          if constexpr (BTW) {
            const uint32_t ff = *reinterpret_cast<const uint32_t*>(it_e2 + u);
            // conj W_{M2}^{e2 w2}
            const int64_t k0 = ((int64_t)(ff & 0xffffu) * w2) & m2mask;
            const int64_t k1 = ((int64_t)(ff >> 16) * w2) & m2mask;
            w[i] = tw2_lds ? SM.tw2[k0] : twb[k0];
            w[i + 1] = tw2_lds ? SM.tw2[k1] : twb[k1];
          } else {
            const cx2<T> ww = *reinterpret_cast<const cx2<T>*>(tw + u);
            w[i] = ww.a;
            w[i + 1] = ww.b;
          }
        } else {
          e1[i] = it_e1[u];
          v[i] = av[u];
          if constexpr (BTW) {
            const int64_t k = ((int64_t)it_e2[u] * w2) & m2mask;
            w[i] = tw2_lds ? SM.tw2[k] : twb[k];
          } else {
            w[i] = tw[u];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const cx<T> c = BTW ? cmulc(v[i], w[i]) : cmul(v[i], w[i]);
        if (e1[i] != cur) {
          buf[cur] = acc;
          cur = e1[i];
          acc = c;
        } else {
          acc = acc + c;
        }
      }
    };
    int r0 = 0;
    for (; r0 + MID_RB <= nr; r0 += MID_RB) rounds_from(r0, std::integral_constant<int, MID_RB>{});
    for (; r0 < nr; r0 += PP) rounds_from(r0, std::integral_constant<int, PP>{});
    buf[cur] = acc;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < R; ++c) x[c] = buf[q + Q * c];
    if constexpr (BTW) {
      // the long factor W_M^{e1 w2} of bucket e1 = q + Q c, as the dense front
      const cx<T> tq = twi3[w2 * M1 + paired_index(q / R, q % R, Q, pair_pp(R))];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        x[c] = cmulc(x[c], tq);
        if (c > 0) x[c] = cmulc(x[c], two[w2 * R + c]);
      }
    }
  } else {
    // dense outer DFT already done: B[pair][w2][e1], times W_M^{e1 w2}
    const cx<T>* bv = src + ((active ? pair : 0) * M2 + w2) * M1;
    // conj W_M^{q w2}: the twi3 entry of e1' = q, f = 0 (thread q mod R, value q / R)
    const cx<T> tq = twi3[w2 * M1 + paired_index(q / R, q % R, Q, pair_pp(R))];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      cx<T> v = active ? bv[q + Q * c] : zero;
      v = cmulc(v, tq);
      if (c > 0) v = cmulc(v, two[w2 * R + c]);
      x[c] = v;
    }
    if constexpr (TW_REC) za = twf1[paired_index(1, q, Q, pair_pp(R))];
    else load_paired<T, R>(tw_a, twf1, q, Q);
  }

  // ---- forward step 1: thread e1' = q, DFT over c -> f --------------------
  reg_fft<T, R, -1>(x);
  if constexpr (TW_REC) {
    cx<T> wf = za;
#pragma unroll
    for (int f = 1; f < R; ++f) {
      x[f] = cmul(x[f], wf);
      if (f + 1 < R) wf = cmul(wf, za);
    }
  } else {
#pragma unroll
    for (int f = 1; f < R; ++f) x[f] = cmul(x[f], tw_a[f]);
  }
  const int gl = q % R;
  // the spectrum two steps early; the FP32 dense-front variant, which holds
  // more registers at this point (it spilled), loads it where it is used
  // (FP64 keeps the early load: its occupancy is set by LDS, not registers)
  constexpr bool EARLY_HV = SPARSE || sizeof(T) == 8;
  if constexpr (EARLY_HV) load_paired<T, R>(hv, Hs + w2 * M1, q, Q);
  __syncthreads();
#pragma unroll
  for (int f = 0; f < R; ++f) buf[f * PB + q] = x[f];
  __syncthreads();
  // The next four steps stay inside one group of R lanes (fixed f, lane
  // index gl), which only touches its own LDS tile grp = buf + f * PB, an
  // R x (R + 1) array; the exchanges need no workgroup barrier.
  cx<T>* grp = buf + (q / R) * PB;
  // ---- forward step 2: thread (a = gl, f): DFT over b -> g ----------------
#pragma unroll
  for (int bb = 0; bb < R; ++bb) x[bb] = grp[gl + R * bb];
  reg_fft<T, R, -1>(x);
  const cx<T>* wrow = SM.wr2 + gl * (R + 1);  // W_{R^2}^{gl j}, j < R
#pragma unroll
  for (int g = 1; g < R; ++g) x[g] = cmul(x[g], wrow[g]);
  wave_lds_sync();
#pragma unroll
  for (int g = 0; g < R; ++g) grp[g * (R + 1) + gl] = x[g];
  wave_lds_sync();
  // ---- forward step 3: thread (g = gl, f): DFT over a -> h ----------------
#pragma unroll
  for (int a = 0; a < R; ++a) x[a] = grp[gl * (R + 1) + a];
  reg_fft<T, R, -1>(x);  // x[h] = X[f + R g + R^2 h]

  if (X != nullptr && w2 == 0 && q == 0 && active) {  // forward: DC term -> row 0
    X[2 * pair] = phi0 * x[0].x;
    if (2 * pair + 1 < t) X[2 * pair + 1] = phi0 * x[0].y;
  }
  if constexpr (!EARLY_HV) load_paired<T, R>(hv, Hs + w2 * M1, q, Q);
#pragma unroll
  for (int h = 0; h < R; ++h) x[h] = cmul(x[h], hv[h]);

  // ---- inverse step 1: thread (g = gl, f): IDFT over h -> a ---------------
  reg_fft<T, R, +1>(x);
#pragma unroll
  for (int a = 1; a < R; ++a) x[a] = cmulc(x[a], wrow[a]);
  wave_lds_sync();
#pragma unroll
  for (int a = 0; a < R; ++a) grp[a * (R + 1) + gl] = x[a];
  wave_lds_sync();
  // ---- inverse step 2: thread (a = gl, f): IDFT over g -> b ---------------
#pragma unroll
  for (int g = 0; g < R; ++g) x[g] = grp[gl * (R + 1) + g];
  reg_fft<T, R, +1>(x);
  // value bb: conj W_M^{(a + R bb)(f M2 + w2)}
  inverse_step_twiddles<T, R, TW_REC>(x, twi3 + w2 * M1, q, Q);
#pragma unroll
  for (int c = 1; c < R; ++c) tw_a[c] = two[w2 * R + c];
  __syncthreads();
#pragma unroll
  for (int bb = 0; bb < R; ++bb) buf[(gl + R * bb) * (R + 1) + q / R] = x[bb];
  __syncthreads();
  // ---- inverse step 3: thread e1' = q, IDFT over f -> c -------------------
#pragma unroll
  for (int f = 0; f < R; ++f) x[f] = buf[q * (R + 1) + f];
  reg_fft<T, R, +1>(x);
#pragma unroll
  for (int c = 1; c < R; ++c) x[c] = cmul(x[c], tw_a[c]);
  if (active) {
    cx<T>* cp = C + (pair * M2 + w2) * M1;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (nt_c) {  // streaming stores: C skips the caches on its way out
        const vec2_t<T> w = {x[c].x, x[c].y};
        __builtin_nontemporal_store(w, reinterpret_cast<vec2_t<T>*>(cp + q + Q * c));
      } else {
        cp[q + Q * c] = x[c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// F for a sum of circulant products that share the output rows (the blocks
// of one row coset of a lattice rule with non-prime N, forward; or of one
// column coset, adjoint): sum_k H(z_k) a_k = IDFT(sum_k Zhat_k DFT(a_k)).
// Each term's input goes through the front and the forward steps of
// middle_body, its spectral product is accumulated in registers, and one
// inverse transform follows: the inverse steps and the intermediate's
// stores are paid once instead of once per term.  Item twiddles only (no
// bucket twiddles), no DC term (the blocks hold no row 0).
// ---------------------------------------------------------------------------
template <typename T>
struct MidTerm {
  const cx<T>* src;        // SPARSE: aT [pair][Upad]; dense: B [pair][M2][M1]
  const uint16_t* it_e1;   // SPARSE: the term's schedule
  const cx<T>* twit;       // SPARSE: item twiddles [M2][Upad]
  const cx<T>* Hs;         // the term's spectrum / M (per-thread layout)
  int64_t Upad, rounds;
};
constexpr int MID_MAX_TERMS = 8;
template <typename T>
struct MidTerms {
  MidTerm<T> t[MID_MAX_TERMS];
  int n;
};

// waves per SIMD the sum kernel is compiled for: the accumulated products
// take R more complex registers than middle_body, so FP32 at R = 16 gets three
// waves' budget (170 registers) instead of four
template <typename T, int R>
constexpr int mid_sum_waves() {
  return (sizeof(T) == 4 && R == 16) ? 3 : mid_waves<T, R>();
}

template <typename T, int R, bool SPARSE>
__device__ __forceinline__ void middle_sum_body(
    const MidTerms<T>& terms, const cx<T>* __restrict__ twf1, const cx<T>* __restrict__ twf2,
    const cx<T>* __restrict__ twi3, const cx<T>* __restrict__ two, int64_t M2, int64_t P,
    cx<T>* __restrict__ C, int64_t b, MidSmem<T, R>& SM, int tid, bool nt_c) {
  typedef MidShape<R> S;
  constexpr int Q = S::Q, M1 = R * R * R, PB = R * (R + 1);
  cx<T>* lds = SM.lds;
  int64_t w2, pg;
  if ((M2 & (M2 - 1)) == 0) {
    w2 = b & (M2 - 1);
    pg = b >> __builtin_ctzll((unsigned long long)M2);
  } else {
    pg = (int64_t)((uint32_t)b / (uint32_t)M2);
    w2 = b - pg * M2;
  }
  const int tr = tid / Q, q = tid % Q;
  const int64_t pair = pg * S::TPB + tr;
  const bool active = pair < P;
  cx<T>* buf = lds + tr * S::BUFN;
  const cx<T> zero = {(T)0, (T)0};
  cx<T> x[R], acc[R], tw_a[R], hv[R];
  constexpr bool TW_REC = sizeof(T) == 8 && R >= 2;  // as in middle_body
  for (int i = tid; i < R * R; i += S::BLOCK)
    SM.wr2[(i % R) * (R + 1) + i / R] = twf2[paired_index(i / R, i % R, R, pair_pp(R))];
  const int gl = q % R;
  cx<T>* grp = buf + (q / R) * PB;
  const cx<T>* wrow = SM.wr2 + gl * (R + 1);
  // The tables are loaded where they are used (not ahead as in middle_body):
  // the accumulated products hold R more complex registers.
  const int nt = terms.n;
#pragma unroll
  for (int h = 0; h < R; ++h) acc[h] = zero;
#pragma unroll 1
  for (int k = 0; k < nt; ++k) {
    const MidTerm<T> tm = terms.t[k];
    if (k > 0) __syncthreads();  // the previous term's exchanges have left buf
    if constexpr (SPARSE) {
      for (int i = q; i <= M1; i += Q) buf[i] = zero;
      __syncthreads();
      const int fo = q / S::G, ln = q % S::G;
      const cx<T>* av = tm.src + (active ? pair : 0) * tm.Upad;
      const cx<T>* tw = tm.twit + w2 * tm.Upad;
      const int nr = (int)tm.rounds;
      int cur = M1;
      cx<T> sum = zero;
      constexpr int PP = pair_pp(R);
      auto rounds_from = [&](int r0, auto nb) {
        constexpr int NB = decltype(nb)::value;
        int e1[NB];
        cx<T> v[NB], w[NB];
#pragma unroll
        for (int i = 0; i < NB; i += PP) {
          const int u = (((r0 + i) / PP * S::F + fo) * S::G + ln) * PP;
          if constexpr (PP == 2) {
            const uint32_t ee = *reinterpret_cast<const uint32_t*>(tm.it_e1 + u);
            const cx2<T> vv = *reinterpret_cast<const cx2<T>*>(av + u);
            const cx2<T> ww = *reinterpret_cast<const cx2<T>*>(tw + u);
            e1[i] = (int)(ee & 0xffffu);
            e1[i + 1] = (int)(ee >> 16);
            v[i] = vv.a;
            v[i + 1] = vv.b;
            w[i] = ww.a;
            w[i + 1] = ww.b;
          } else {
            e1[i] = tm.it_e1[u];
            v[i] = av[u];
            w[i] = tw[u];
          }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const cx<T> c = cmul(v[i], w[i]);
          if (e1[i] != cur) {
            buf[cur] = sum;
            cur = e1[i];
            sum = c;
          } else {
            sum = sum + c;
          }
        }
      };
      int r0 = 0;
      for (; r0 + MID_RB <= nr; r0 += MID_RB)
        rounds_from(r0, std::integral_constant<int, MID_RB>{});
      for (; r0 < nr; r0 += PP) rounds_from(r0, std::integral_constant<int, PP>{});
      buf[cur] = sum;
      __syncthreads();
#pragma unroll
      for (int c = 0; c < R; ++c) x[c] = buf[q + Q * c];
    } else {
      const cx<T>* bv = tm.src + ((active ? pair : 0) * M2 + w2) * M1;
      // conj W_M^{q w2}: the long outer twiddle of column e1 = q + Q c
      const cx<T> tq = twi3[w2 * M1 + paired_index(q / R, q % R, Q, pair_pp(R))];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        cx<T> v = active ? bv[q + Q * c] : zero;
        v = cmulc(v, tq);
        if (c > 0) v = cmulc(v, two[w2 * R + c]);
        x[c] = v;
      }
    }
    // ---- forward steps 1-3, as middle_body ----------------------------------
    load_paired<T, R>(tw_a, twf1, q, Q);
    reg_fft<T, R, -1>(x);
#pragma unroll
    for (int f = 1; f < R; ++f) x[f] = cmul(x[f], tw_a[f]);
    __syncthreads();
#pragma unroll
    for (int f = 0; f < R; ++f) buf[f * PB + q] = x[f];
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < R; ++bb) x[bb] = grp[gl + R * bb];
    reg_fft<T, R, -1>(x);
#pragma unroll
    for (int g = 1; g < R; ++g) x[g] = cmul(x[g], wrow[g]);
    wave_lds_sync();
#pragma unroll
    for (int g = 0; g < R; ++g) grp[g * (R + 1) + gl] = x[g];
    wave_lds_sync();
#pragma unroll
    for (int a = 0; a < R; ++a) x[a] = grp[gl * (R + 1) + a];
    reg_fft<T, R, -1>(x);
    // ---- this term's spectral product, accumulated ---------------------------
    load_paired<T, R>(hv, tm.Hs + w2 * M1, q, Q);
#pragma unroll
    for (int h = 0; h < R; ++h) {
      acc[h].x = fmaT(x[h].x, hv[h].x, fmaT(-x[h].y, hv[h].y, acc[h].x));
      acc[h].y = fmaT(x[h].x, hv[h].y, fmaT(x[h].y, hv[h].x, acc[h].y));
    }
  }
  // ---- inverse steps and the stores of C, as middle_body ----------------------
#pragma unroll
  for (int h = 0; h < R; ++h) x[h] = acc[h];
  reg_fft<T, R, +1>(x);
#pragma unroll
  for (int a = 1; a < R; ++a) x[a] = cmulc(x[a], wrow[a]);
  wave_lds_sync();
#pragma unroll
  for (int a = 0; a < R; ++a) grp[a * (R + 1) + gl] = x[a];
  wave_lds_sync();
#pragma unroll
  for (int g = 0; g < R; ++g) x[g] = grp[gl * (R + 1) + g];
  reg_fft<T, R, +1>(x);
  inverse_step_twiddles<T, R, TW_REC>(x, twi3 + w2 * M1, q, Q);
#pragma unroll
  for (int c = 1; c < R; ++c) tw_a[c] = two[w2 * R + c];
  __syncthreads();
#pragma unroll
  for (int bb = 0; bb < R; ++bb) buf[(gl + R * bb) * (R + 1) + q / R] = x[bb];
  __syncthreads();
#pragma unroll
  for (int f = 0; f < R; ++f) x[f] = buf[q * (R + 1) + f];
  reg_fft<T, R, +1>(x);
#pragma unroll
  for (int c = 1; c < R; ++c) x[c] = cmul(x[c], tw_a[c]);
  if (active) {
    cx<T>* cp = C + (pair * M2 + w2) * M1;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (nt_c) {
        const vec2_t<T> w = {x[c].x, x[c].y};
        __builtin_nontemporal_store(w, reinterpret_cast<vec2_t<T>*>(cp + q + Q * c));
      } else {
        cp[q + Q * c] = x[c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// outer split (only when the tuning splits M2 = P2 * Q2 with P2 > 1), in place
// on C[pair][w2][e1]:
//   DIR = +1 (forward product, first half of the inverse over w2):
//     w2 = q + Q2 p'  ->  index a, times conj W_{M2}^{a q}
//   DIR = -1 (dense outer fronts, second half of the forward DFT over e2):
//     the values at q + Q2 a (already twiddled by W_{M2}^{a q}) -> p',
//     stored at w2 = q + Q2 p'
// ---------------------------------------------------------------------------
template <typename T, int P2, int DIR>
__device__ __forceinline__ void split_body(cx<T>* __restrict__ C, int64_t M1, int64_t M2, int Q2,
                                           const cx<T>* __restrict__ twb, int64_t bx, int64_t q,
                                           int64_t pair, int tid) {
  const int64_t e1 = bx * 64 + tid;
  if (e1 >= M1) return;
  cx<T>* base = C + pair * M2 * M1 + e1;
  cx<T> v[P2];
#pragma unroll
  for (int p = 0; p < P2; ++p) v[p] = base[(q + (int64_t)Q2 * p) * M1];
  reg_fft<T, P2, DIR>(v);
  if constexpr (DIR > 0) {
#pragma unroll
    for (int a = 1; a < P2; ++a) v[a] = cmul(v[a], twb[a * q]);  // a q < P2 Q2 = M2
  }
#pragma unroll
  for (int a = 0; a < P2; ++a) base[(q + (int64_t)Q2 * a) * M1] = v[a];
}

// ---------------------------------------------------------------------------
// B: inverse DFT over the Q (= M2 / P2) factor of w2 and the output scatter.
// thread (pair, e1, a): loads C[pair][q + Q a][e1], q < Q, produces e2 = a + P2 b.
//   forward: X[pow[e]][2 pair .. 2 pair + 1] = out[e] for e < L
//   adjoint: dA[j][...] = out[e] + phi0 G[0][...] for every j with l_j = e
// A workgroup takes a tile of EB e1 x PB column pairs (one thread each), so
// it reads C in runs of EB values and writes each output row's PB pairs as
// one segment: 16 x 16 (256-byte runs and segments in FP64), or 64 x 8 for
// the FP64 forward product (1 KB runs of C, one whole 128-byte line per row).
// ---------------------------------------------------------------------------
// values per thread exchanged per round through LDS in the back and
// adjoint-front passes; small enough that a back workgroup fits beside
// four fused-kernel workgroups on one CU
constexpr int BACK_CH = 8;
// the largest divisor of Q that is at most cap (Q = 2^k, 3 x 2^k or 5 x 2^k:
// the chunks of a length-Q column moved through LDS together)
constexpr int chunk_of(int Q, int cap) {
  int c = Q < cap ? Q : cap;
  while (Q % c) --c;
  return c;
}
template <typename T, int EB = 16, int PB = 16>
struct BackSmem {
  cx<T> sm[BACK_CH][EB][PB + 1];
};

template <typename T, bool NT>
__device__ __forceinline__ void store_pair(T* p, T x, T y) {
  const vec2_t<T> v = {x, y};
  if constexpr (NT)
    __builtin_nontemporal_store(v, reinterpret_cast<vec2_t<T>*>(p));
  else
    *reinterpret_cast<vec2_t<T>*>(p) = v;
}

// one output value pair o of group-order index e < L in column pair pairw:
//   forward: X[rowmap[e]][2 pairw .. 2 pairw + 1] = f(o)  (f: the epilogue)
//   adjoint: dA[j][...] = o + phi0 G[0][...] for every j with l_j = e
// forward: the value pair o to X[r][2 pairw .. 2 pairw + 1], through the epilogue
template <typename T, bool NT, bool EPI>
__device__ __forceinline__ void put_row(cx<T> o, int64_t r, int64_t pairw, T* __restrict__ X,
                                        int64_t ldx, int64_t t, bool v2, const EpiCols<T>& ec) {
  const int64_t col = 2 * pairw;
  const bool both = col + 1 < t;
  T* row = X + r * ldx;
  T ox, oy;
  if (EPI && ec.kind == EPI_ACC) {
    ox = row[col] + o.x;
    oy = both ? row[col + 1] + o.y : (T)0;
  } else {
    ox = EPI ? ec.f0(o.x) : o.x;
    oy = EPI ? ec.f1(o.y) : o.y;
  }
  if (v2 && both) {
    store_pair<T, NT>(row + col, ox, oy);
  } else if constexpr (NT) {
    __builtin_nontemporal_store(ox, row + col);
    if (both) __builtin_nontemporal_store(oy, row + col + 1);
  } else {
    row[col] = ox;
    if (both) row[col + 1] = oy;
  }
}

// the adjoint's writes for one output e whose rows j (l_j = e) are
// inv_j[lo .. hi): dA[j] = o + phi(x_0) G[0] (g0, g1: the second term, for
// columns col and col + 1), or dA[j] += o + ... with acc.  lo, hi and g0, g1
// are loaded by the caller together with its other loads, ahead of the
// transform.
template <typename T>
__device__ __forceinline__ void put_adj(cx<T> o, int32_t lo, int32_t hi, int64_t col, T g0, T g1,
                                        const int32_t* __restrict__ inv_j, T* __restrict__ X,
                                        int64_t ldx, int64_t t, bool v2, bool acc = false) {
  const bool both = col + 1 < t;
  for (int32_t jj = lo; jj < hi; ++jj) {
    T* row = X + (int64_t)inv_j[jj] * ldx;
    T b0 = (T)0, b1 = (T)0;
    if (acc) {
      b0 = row[col];
      if (both) b1 = row[col + 1];
    }
    if (v2 && both) {
      store_pair<T, false>(row + col, b0 + o.x + g0, b1 + o.y + g1);
    } else {
      row[col] = b0 + o.x + g0;
      if (both) row[col + 1] = b1 + o.y + g1;
    }
  }
}

// the adjoint's per-thread ranges: (lo, hi) of output e (an empty range when
// e is out of bounds), and the constant row's part for column pair pw
template <typename T>
struct AdjRows {
  T g0 = (T)0, g1 = (T)0;
  __device__ __forceinline__ void load_g0(const T* __restrict__ G0, T phi0, int64_t pw,
                                          int64_t t, bool ok) {
    // no part when G0 is null: a point set without the point 0
    if (ok && G0) {
      g0 = phi0 * G0[2 * pw];
      if (2 * pw + 1 < t) g1 = phi0 * G0[2 * pw + 1];
    }
  }
  static __device__ __forceinline__ int2 range(const int32_t* __restrict__ inv_ptr, int64_t e,
                                               bool ok) {
    return ok ? int2{inv_ptr[e], inv_ptr[e + 1]} : int2{0, 0};
  }
};

// waves per SIMD the register back pass is compiled for: 32 values of w2 per
// thread in FP64 would otherwise take all 256 registers (one wave)
template <typename T, int Q>
constexpr int back_waves() {
  return (sizeof(T) == 8 && Q == 32) ? 2 : 1;
}

template <typename T, int Q, bool ADJ, bool NT, bool EPI = false, int EB = 16, int PB = 16>
__device__ __forceinline__ void back_body(const cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                          int64_t P2, int64_t L, int64_t P,
                                          const int32_t* __restrict__ rowmap,
                                          const int32_t* __restrict__ inv_ptr,
                                          const int32_t* __restrict__ inv_j,
                                          const T* __restrict__ G0, T phi0,
                                          T* __restrict__ X, int64_t ldx, int64_t t, int64_t bx,
                                          int64_t by, int64_t a, BackSmem<T, EB, PB>& S,
                                          int tid, const Epi<T> epi = Epi<T>()) {
  constexpr int CH = chunk_of(Q, BACK_CH);
  // FP32 forward writes without epilogue: two pairs per 16-byte store when
  // rows are 16-byte aligned (else per pair, as the other variants)
  constexpr bool WIDE = !ADJ && !EPI && sizeof(T) == 4 && CH == BACK_CH;
  auto& sm = S.sm;
  const int64_t e1_0 = bx * EB, p0 = by * PB;
  const int el = tid % EB, pl = tid / EB;
  const bool v2 = pairs_aligned(X, ldx);
  const bool wide = WIDE && ldx % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
  // the epilogue of the columns this thread writes (EPI only)
  const EpiCols<T> ec(EPI ? epi : Epi<T>(), 2 * (p0 + tid % PB), t);
  const int pw = tid % PB, ew = tid / PB;
  const int64_t pairw = p0 + pw, e1w = e1_0 + ew;
  // adjoint: the CSR ranges of this thread's outputs, issued before C (two
  // registers per output: up to 16 outputs; 32 would cost an occupancy step
  // that the early loads do not repay, so there they are loaded at the write)
  constexpr bool PRE = ADJ && Q <= 16;
  int2 rng[PRE ? Q : 1];
  AdjRows<T> ar;
  const bool okw = pairw < P && e1w < M1;
  if constexpr (ADJ) {
    if constexpr (PRE) {
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const int64_t e = e1w + M1 * (a + P2 * c);
        rng[c] = AdjRows<T>::range(inv_ptr, e, okw && e < L);
      }
    }
    ar.load_g0(G0, phi0, pairw, t, okw);
  }
  {
    const int64_t e1 = e1_0 + el, pair = p0 + pl;
    cx<T> v[Q];
    const bool ok = pair < P && e1 < M1;
    const cx<T>* base = C + (ok ? pair : 0) * M2 * M1 + (ok ? e1 : 0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      // C is dead after this read: a non-temporal load keeps it from
      // displacing lines that are still wanted
      cx<T> c = {(T)0, (T)0};
      if (ok) {
        const vec2_t<T> w = __builtin_nontemporal_load(
            reinterpret_cast<const vec2_t<T>*>(base + (q + Q * a) * M1));
        c = {w.x, w.y};
      }
      v[q] = c;
    }
    reg_fft<T, Q, +1>(v);
#pragma unroll
    for (int c0 = 0; c0 < Q; c0 += CH) {
      __syncthreads();
#pragma unroll
      for (int c = 0; c < CH; ++c) sm[c][el][pl] = v[c0 + c];
      __syncthreads();
      if constexpr (WIDE) {
        // thread (two pairs pw0, pw0 + 1; e1; every other c): one 16-byte
        // store of both pairs per output row, half the store instructions
        const int pw2 = tid % (PB / 2), ew2 = (tid / (PB / 2)) % EB, ch = tid / ((PB / 2) * EB);
        const int64_t pw0 = p0 + 2 * pw2, e1x = e1_0 + ew2, col = 2 * pw0;
        const bool full = wide && pw0 + 1 < P && col + 3 < t;
        if (e1x < M1) {
#pragma unroll
          for (int cc = 0; cc < CH / 2; ++cc) {
            const int c = ch + 2 * cc;
            const int64_t e = e1x + M1 * (a + P2 * (c0 + c));
            if (e >= L) continue;
            const int64_t r = rowmap[e];
            const cx<T> o0 = sm[c][ew2][2 * pw2], o1 = sm[c][ew2][2 * pw2 + 1];
            if (full) {
              const vec4_t<T> w = {o0.x, o0.y, o1.x, o1.y};
              vec4_t<T>* dst = reinterpret_cast<vec4_t<T>*>(X + r * ldx + col);
              if constexpr (NT)
                __builtin_nontemporal_store(w, dst);
              else
                *dst = w;
            } else {
              if (pw0 < P) put_row<T, NT, EPI>(o0, r, pw0, X, ldx, t, v2, ec);
              if (pw0 + 1 < P) put_row<T, NT, EPI>(o1, r, pw0 + 1, X, ldx, t, v2, ec);
            }
          }
        }
      } else if (pairw < P && e1w < M1) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int64_t e2 = a + P2 * (c0 + c);
          const int64_t e = e1w + M1 * e2;
          if constexpr (ADJ) {
            const int2 r = PRE ? rng[PRE ? c0 + c : 0] : AdjRows<T>::range(inv_ptr, e, e < L);
            put_adj<T>(sm[c][ew][pw], r.x, r.y, 2 * pairw, ar.g0, ar.g1, inv_j, X, ldx, t, v2,
                       epi.kind == EPI_ACC);
          } else if (e < L)
            put_row<T, NT, EPI>(sm[c][ew][pw], (int64_t)rowmap[e], pairw, X, ldx, t, v2, ec);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// B for a long outer factor (Q = 64 or 128 values of w2 per output column):
// the same result as back_body<Q>, with the length-Q inverse DFT done as two
// register passes through LDS instead of Q values per thread.  A workgroup
// (NW threads per column) owns a tile of TE e1 x 8 column pairs (K = 8 TE
// "columns" (e1l, pl)) for one a and keeps the tile's Q x K values in LDS.
// With Q = F1 F2,
//   q = u + F2 v (u < F2, v < F1),   b = c + F1 d (c < F1, d < F2):
//   pass 1, per (k, u): over v -> c, times W_Q^{u c}    (from global C)
//   pass 2, per (k, c): over u -> d, in place in LDS    (slot u + F2 c)
// then the rows e = e1 + M1 (a + P2 b) are written from LDS with the column
// pairs fastest, so one row's 8 pairs leave as one 8-pair segment.  Thread
// (pl, eo, w) writes the outputs b = w + NW j of e1 = e1_0 + eo, pair pl.
// ---------------------------------------------------------------------------
template <int Q, int TE = 8, int NW_ = 4>
struct BackLdsShape {
  // Q = 2^k: F1 = 8; Q = 3 x 2^k or 5 x 2^k: F1 = Q / 8 (5, 6, 10 or 12), F2 = 8
  static constexpr int F1 = (Q % 3 == 0 || Q % 5 == 0) ? Q / 8 : 8;
  static constexpr int F2 = Q / F1;
  static constexpr int TP = 8;        // column pairs per tile
  static constexpr int K = TE * TP;   // columns per tile (TE values of e1)
  static constexpr int NW = NW_;      // threads per column
  static constexpr int BLOCK = NW * K;
  // pass-1 and pass-2 tasks per thread (the last one guarded when NW does
  // not divide a factor: Q = 48 and 96 with 8 threads per column)
  static constexpr int T1 = (F2 + NW - 1) / NW, T2 = (F1 + NW - 1) / NW;
  static_assert(F1 * F2 == Q && Q % NW == 0, "outer factor split");
  static_assert(TE == 8 || TE == 16, "tile width");
  // LDS column of (e1 offset el, pair offset pl): with 16 e1 per tile the
  // rows of e1 are rotated by 4 per two pairs, so that the output reads (8
  // pairs x 8 e1 per wave) spread over the banks as the loads (16 e1 x 4
  // pairs) do
  static __device__ __forceinline__ int col(int el, int pl) {
    return TE == 16 ? ((el + 4 * (pl >> 1)) & 15) + 16 * pl : el + TE * pl;
  }
};

// Workgroup order of the LDS back pass: the workgroups of one XCD take a
// contiguous run of logical tiles (xcd_remap), and inside it the tiles go in
// pairs of column-pair tiles (by, by + 1) per e1 tile, e1 tiles next: the two
// 8-pair halves of a 16-pair row segment of X, and (8-e1 tiles) the two halves
// of a 16-e1 segment of C, are then handled by one L2 at about the same time.
__device__ __forceinline__ void back_lds_tile(int64_t hw, int64_t gx, int64_t gy, int64_t gz,
                                              int64_t& bx, int64_t& by, int64_t& a) {
  const int64_t per = gx * gy;
  const int64_t lg = xcd_remap(hw, per * gz);
  a = lg / per;
  const int64_t l = lg % per, full = (gy / 2) * 2 * gx;
  if (l < full) {
    const int64_t r = l % (2 * gx);
    bx = r / 2;
    by = 2 * (l / (2 * gx)) + r % 2;
  } else {  // odd gy: the last row of pair tiles alone
    bx = l - full;
    by = gy - 1;
  }
}

// e1 per tile of the LDS back pass: 16 in FP32 (C is read in whole 128-byte
// lines; 64 or 128 KB of LDS per workgroup), 8 in FP64 (where 16 would halve
// the occupancy for no gain)
template <typename T>
constexpr int back_lds_te() {
  return sizeof(T) == 4 ? 16 : 8;
}

// threads per column of the LDS back pass: 8 (1024- or 512-thread
// workgroups, half the registers per thread and twice the waves of 4), but 4
// for the FP32 adjoint at Q = 64, which measured faster so
template <typename T, int Q, bool ADJ>
constexpr int back_lds_nw() {
  return (Q == 32 || (ADJ && sizeof(T) == 4 && Q == 64)) ? 4 : 8;
}

// whether the back pass of outer radix Q goes through LDS: Q >= 40 (64, 128
// and 40, 48, 80, 96), and Q = 32 in FP64 (its register variant takes all
// 256 registers and spills; in FP32 the register variant is the faster one)
__host__ __device__ constexpr bool back_in_lds(int Q, bool f64) {
  return Q >= 40 || (f64 && Q == 32);
}

template <typename T, int Q, int TE = 8>
struct BackLdsSmem {
  cx<T> v[Q * TE * 8];  // Q x K values, K = TE x 8 column pairs
};

template <typename T, int Q, bool ADJ, bool NT, bool EPI = false, int TE = 8, int NW_ = 4>
__device__ __forceinline__ void back_lds_body(const cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                              int64_t P2, int64_t L, int64_t P,
                                              const cx<T>* __restrict__ twb,
                                              const int32_t* __restrict__ rowmap,
                                              const int32_t* __restrict__ inv_ptr,
                                              const int32_t* __restrict__ inv_j,
                                              const T* __restrict__ G0, T phi0,
                                              T* __restrict__ X, int64_t ldx, int64_t t,
                                              int64_t bx, int64_t by, int64_t a,
                                              BackLdsSmem<T, Q, TE>& S, int tid,
                                              const Epi<T> epi = Epi<T>()) {
  typedef BackLdsShape<Q, TE, NW_> B;
  constexpr int F1 = B::F1, F2 = B::F2, TP = B::TP, K = B::K, NW = B::NW;
  constexpr int T1 = B::T1, T2 = B::T2;  // pass-1 and pass-2 tasks per thread
  constexpr int NO = Q / NW;             // output values per thread
  cx<T>* lds = S.v;
  const int64_t e1_0 = bx * TE, p0 = by * TP;
  const int w = tid / K;  // this thread's first task
  // load mapping: e1 = e1_0 + tid % TE (fastest: C is contiguous in e1),
  // pair p0 + (tid / TE) % TP; LDS column kc
  const int kc = B::col(tid % TE, (tid / TE) % TP);
  // output mapping: column pair pl, e1 = e1_0 + eo, b = w + NW j
  const int pl = tid % TP, eo = (tid / TP) % TE;
  const int64_t e1o = e1_0 + eo, pairw = p0 + pl;
  // Every global load of the workgroup is issued before the first use: the
  // output rows (forward), then the tile of C; the workgroup then waits for
  // memory once.
  int32_t rows[ADJ ? 1 : NO];
  int2 rng[ADJ ? NO : 1];  // adjoint: the CSR ranges of the outputs
  AdjRows<T> ar;
  if constexpr (!ADJ) {
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int64_t e = e1o + M1 * (a + P2 * (w + NW * j));
      rows[j] = (e1o < M1 && e < L) ? rowmap[e] : -1;
    }
  } else {
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int64_t e = e1o + M1 * (a + P2 * (w + NW * j));
      rng[j] = AdjRows<T>::range(inv_ptr, e, pairw < P && e1o < M1 && e < L);
    }
    ar.load_g0(G0, phi0, pairw, t, pairw < P && e1o < M1);
  }
  {
    const int64_t e1 = e1_0 + tid % TE, pair = p0 + (tid / TE) % TP;
    const bool ok = pair < P && e1 < M1;
    const cx<T>* base = C + (ok ? pair : 0) * M2 * M1 + (ok ? e1 : 0) + Q * a * M1;
    const int64_t tstep = M2 / Q;  // W_Q^{j} = twb[j M2 / Q]
    // ---- pass 1: per u, the F1 values q = u + F2 v -------------------------
    cx<T> v[T1][F1];
#pragma unroll
    for (int it = 0; it < T1; ++it) {
      const int u = w + NW * it;
#pragma unroll
      for (int j = 0; j < F1; ++j) {
        cx<T> c = {(T)0, (T)0};
        if (ok && (F2 % NW == 0 || u < F2)) {  // C is dead after this read
          const vec2_t<T> x = __builtin_nontemporal_load(
              reinterpret_cast<const vec2_t<T>*>(base + (int64_t)(u + F2 * j) * M1));
          c = {x.x, x.y};
        }
        v[it][j] = c;
      }
    }
#pragma unroll
    for (int it = 0; it < T1; ++it) {
      const int u = w + NW * it;
      if (F2 % NW != 0 && u >= F2) continue;
      reg_fft<T, F1, +1>(v[it]);
#pragma unroll
      for (int c = 1; c < F1; ++c)
        v[it][c] = cmul(v[it][c], twb[(int64_t)(u * c) * tstep]);  // u c < Q
#pragma unroll
      for (int c = 0; c < F1; ++c) lds[(u + F2 * c) * K + kc] = v[it][c];
    }
  }
  __syncthreads();
  // ---- pass 2: per c, the F2 values of slots u + F2 c, in place ------------
#pragma unroll
  for (int it = 0; it < T2; ++it) {
    const int c = w + NW * it;
    if (F1 % NW != 0 && c >= F1) continue;
    cx<T> v[F2];
#pragma unroll
    for (int u = 0; u < F2; ++u) v[u] = lds[(u + F2 * c) * K + kc];
    reg_fft<T, F2, +1>(v);
#pragma unroll
    for (int d = 0; d < F2; ++d) lds[(d + F2 * c) * K + kc] = v[d];
  }
  __syncthreads();
  // ---- rows: output b = c + F1 d sits in slot d + F2 c ---------------------
  const bool v2 = pairs_aligned(X, ldx);
  const EpiCols<T> ec(EPI ? epi : Epi<T>(), 2 * pairw, t);
  if (pairw >= P) return;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    const int b = w + NW * j;
    const cx<T> o = lds[(b / F1 + F2 * (b % F1)) * K + B::col(eo, pl)];
    if constexpr (!ADJ) {
      if (rows[j] >= 0) put_row<T, NT, EPI>(o, rows[j], pairw, X, ldx, t, v2, ec);
    } else {
      put_adj<T>(o, rng[j].x, rng[j].y, 2 * pairw, ar.g0, ar.g1, inv_j, X, ldx, t, v2,
                 epi.kind == EPI_ACC);
    }
  }
}

// ---------------------------------------------------------------------------
// dense outer front: the length-M input column pair v[m] (m < L; 0 for
// L <= m < M) is gathered with coalesced row reads, then transformed over
// e2 (the forward DFT of the outer index).  With M2 = P2 * Q: thread
// (pair, e1, a) transforms e2 = a + P2 b over b (length Q) and multiplies by
// W_{M2}^{a q}; k_outer_split<-1> finishes over a.
// Output: B[pair][w2][e1] (natural w2 order once the split has run).
//   adjoint:  v[m] = G[pow[(L - m) mod L]]                      (gather)
//   forward:  v[m] = sum of A[j] over j with l_j = (L - m) mod L (the
//             reflected collapse, Section 2.1, as a gather through the
//             CSR lists of equal l_j, in increasing j)
// ---------------------------------------------------------------------------
template <typename T>
struct RowPairReader {  // columns 2 pair, 2 pair + 1 of a row-major matrix
  const T* __restrict__ M;
  int64_t ld, t;
  bool v2;
  __device__ __forceinline__ cx<T> operator()(int64_t row, int64_t pair) const {
    const T* r = M + row * ld;
    const int64_t col = 2 * pair;
    cx<T> g = {(T)0, (T)0};
    if (v2 && col + 1 < t) {
      const vec2_t<T> gg = *reinterpret_cast<const vec2_t<T>*>(r + col);
      g.x = gg.x;
      g.y = gg.y;
    } else {
      g.x = r[col];
      if (col + 1 < t) g.y = r[col + 1];
    }
    return g;
  }
};

// The gathers run in three steps so that a thread's loads for several m are
// in flight together: bounds(m) (the first table lookup), first(b) (the
// first row), value(b, row, pair).  bounds is only called with 0 <= m < L.
template <typename T>
struct AdjGather {
  RowPairReader<T> G;
  const int32_t* __restrict__ pow;
  int64_t L;
  // m in [0, L): the reflected index (L - m) mod L without a division
  __device__ __forceinline__ int2 bounds(int64_t m) const {
    return {pow[m == 0 ? 0 : L - m], 0};
  }
  __device__ __forceinline__ int32_t first(int2 b) const { return b.x; }
  __device__ __forceinline__ cx<T> value(int2, int32_t row, int64_t pair) const {
    return G(row, pair);
  }
};

template <typename T>
struct FwdGather {
  RowPairReader<T> A;
  const int32_t* __restrict__ inv_ptr;
  const int32_t* __restrict__ inv_j;
  int64_t L;
  __device__ __forceinline__ int2 bounds(int64_t m) const {  // m in [0, L)
    const int64_t e = m == 0 ? 0 : L - m;
    return {inv_ptr[e], inv_ptr[e + 1]};
  }
  __device__ __forceinline__ int32_t first(int2 b) const { return b.x < b.y ? inv_j[b.x] : -1; }
  __device__ __forceinline__ cx<T> value(int2 b, int32_t row, int64_t pair) const {
    cx<T> acc = {(T)0, (T)0};
    if (row < 0) return acc;
    acc = A(row, pair);
    if (b.x + 1 < b.y)
      acc = add_rows<T>(acc, inv_j, b.x + 1, b.y, [&](int32_t j) { return A(j, pair); });
    return acc;
  }
};

template <typename T, int Q, typename Gather>
__device__ __forceinline__ void outer_front_body(const Gather& gather, int64_t M1, int64_t M2,
                                                 int64_t P2, int64_t L, int64_t P,
                                                 const cx<T>* __restrict__ twb,
                                                 cx<T>* __restrict__ B, int64_t bx, int64_t by,
                                                 int64_t a, BackSmem<T>& S, int tid) {
  constexpr int PB = 16, EB = 16;
  auto& sm = S.sm;
  const int64_t e1_0 = bx * EB, p0 = by * PB;
  const int pw = tid % PB, ew = tid / PB;     // gather mapping (pair-fast)
  const int el = tid % EB, pl = tid / EB;     // transform mapping (e1-fast)
  const int64_t pairw = p0 + pw, e1w = e1_0 + ew;
  // GQ values of the thread's gather column are loaded before the first wait
  // (all of them up to 16; beyond that the registers go to the transform)
  // and then transposed through LDS CH at a time
  constexpr int GQ = chunk_of(Q, 16);
  constexpr int CH = chunk_of(GQ, BACK_CH);
  cx<T> v[Q];
#pragma unroll
  for (int g0 = 0; g0 < Q; g0 += GQ) {
    int2 bd[GQ];
    int32_t row[GQ];
    cx<T> gv[GQ];
#pragma unroll
    for (int c = 0; c < GQ; ++c) {
      const int64_t e = e1w + M1 * (a + P2 * (g0 + c));
      bd[c] = (pairw < P && e1w < M1 && e < L) ? gather.bounds(e) : int2{-1, -1};
    }
#pragma unroll
    for (int c = 0; c < GQ; ++c) row[c] = bd[c].x >= 0 ? gather.first(bd[c]) : -1;
#pragma unroll
    for (int c = 0; c < GQ; ++c)
      gv[c] = row[c] >= 0 ? gather.value(bd[c], row[c], pairw) : cx<T>{(T)0, (T)0};
#pragma unroll
    for (int c0 = 0; c0 < GQ; c0 += CH) {
      __syncthreads();
#pragma unroll
      for (int c = 0; c < CH; ++c) sm[c][ew][pw] = gv[c0 + c];
      __syncthreads();
#pragma unroll
      for (int c = 0; c < CH; ++c) v[g0 + c0 + c] = sm[c][el][pl];
    }
  }
  reg_fft<T, Q, -1>(v);
  if (P2 > 1) {
#pragma unroll
    for (int q = 1; q < Q; ++q) v[q] = cmulc(v[q], twb[a * q]);  // a q < M2
  }
  const int64_t e1 = e1_0 + el, pair = p0 + pl;
  if (pair < P && e1 < M1) {
    cx<T>* base = B + pair * M2 * M1 + e1;
#pragma unroll
    for (int q = 0; q < Q; ++q) base[(q + Q * a) * M1] = v[q];
  }
}

}  // namespace qmc
