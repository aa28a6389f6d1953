// The hot path: X = Y A (and dA = Y^T G) through the circulant factorisation.
//
// Section 2.1: with rows indexed by the group exponent e (row pow[e]) the
// nonzero rows of Y satisfy Y[pow[e], j] = z[(e + l_j) mod L], so for one
// column a
//     X[pow[e]] = sum_k z[(e + k) mod L] a'[k],   a' = P a   (eq. (ZPa)),
// which is the circular convolution (z * a~)[e] with the reflected collapse
// a~[(L - l_j) mod L] += a_j.  Row 0 is phi(x_0) sum_j a_j.  Two real
// columns travel as the real and imaginary part of one complex vector (the
// convolution kernel z is real).
//
// The convolution of length M (= L, or a power of two >= 2L-1 with the
// generator embedded) is split M = M1 * M2, index e = e1 + M1 e2 and
// frequency w = w2 + M2 w1:
//   T  collapse-transpose: the s rows of A, in the schedule's item order,
//      become per-pair contiguous vectors aT[pair][u];
//   F  for one outer frequency w2 and one pair: the sparse outer DFT over e2
//      (only the s nonzero slots, scheduled in conflict-free rounds), the
//      length-M1 DFT (three register DFTs of length R = M1^(1/3) across a
//      workgroup with LDS exchanges), the spectral product, the inverse
//      length-M1 DFT and the outer twiddle; the DC term gives row 0;
//   B  for a tile of (e1, pairs): the inverse DFT over w2 and the row
//      un-permutation X[pow[e]] (or, for the adjoint, the read-back at the
//      exponents l_j).
#include <algorithm>

#include "cx.hpp"
#include "internal.hpp"

namespace qmc {

// workgroups are dealt round-robin to the 8 XCDs; map them so that a run of
// consecutive logical ids lands on one XCD (shared L2 for the same pair)
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
  const int64_t X = 8;
  const int64_t q = G / X, rem = G % X;
  const int64_t xcd = b % X, idx = b / X;
  return (xcd < rem) ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

// ---------------------------------------------------------------------------
// T: aT[pair][u] = A[j_u, 2 pair] + i A[j_u, 2 pair + 1]   (0 for padding)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_collapse_T(const T* __restrict__ A, int64_t lda,
                                                    int64_t t, int64_t P,
                                                    const int32_t* __restrict__ it_j, int64_t Upad,
                                                    cx<T>* __restrict__ aT) {
  __shared__ cx<T> sm[64][17];
  const int64_t u0 = (int64_t)blockIdx.x * 64, p0 = (int64_t)blockIdx.y * 16;
  const int tid = threadIdx.x;
  const int pl = tid & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int ul = (tid >> 4) + 16 * i;
    const int64_t u = u0 + ul, p = p0 + pl;
    cx<T> v = {(T)0, (T)0};
    if (u < Upad && p < P) {
      const int j = it_j[u];
      if (j >= 0) {
        const T* row = A + (int64_t)j * lda;
        const int64_t c = 2 * p;
        v.x = row[c];
        if (c + 1 < t) v.y = row[c + 1];
      }
    }
    sm[ul][pl] = v;
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
//            thread (a, f):        DFT over b -> g, * W_{R^2}^{a g}
//            thread (f, g):        DFT over a -> h      => X[f + R g + R^2 h]
//   product  * Hs[w2][w1]  (the spectrum, with 1/M folded in)
//   inverse  thread (f, g):        IDFT over h -> a, * conj W_{R^2}^{a g}
//            thread (f, a):        IDFT over g -> b, * conj W_M^{e1' (f M2 + w2)}
//            thread e1':           IDFT over f -> c, * conj W_M^{R^2 c w2}
// The conj W_M^{e1' w2} factor is the outer-step twiddle of M = M1 * M2.
// ---------------------------------------------------------------------------
template <int R>
struct MidShape {
  static constexpr int Q = R * R;                  // threads per transform
  static constexpr int TPB = Q >= 64 ? 1 : 64 / Q; // transforms per block
  static constexpr int BLOCK = Q * TPB;
  static constexpr int BUFN = Q * (R + 1);         // LDS complex per transform (>= R^3 + 1)
  static constexpr int G = Q < 64 ? Q : 64;        // sparse-front round width
  static constexpr int F = Q / G;                  // front slices per transform (owners of e1 mod F)
};

template <typename T, int R, bool SPARSE>
__global__ __launch_bounds__(MidShape<R>::BLOCK) void k_middle(
    const cx<T>* __restrict__ src,      // SPARSE: aT [pair][Upad]; dense: B [pair][M2][M1]
    int64_t Upad, int64_t rounds, const int32_t* __restrict__ it_e1,
    const cx<T>* __restrict__ twit, const cx<T>* __restrict__ twf1,
    const cx<T>* __restrict__ twf2, const cx<T>* __restrict__ Hs, const cx<T>* __restrict__ twi3,
    const cx<T>* __restrict__ two, int64_t M2, int64_t P, cx<T>* __restrict__ C,
    T* __restrict__ X, int64_t t, T phi0) {
  typedef MidShape<R> S;
  constexpr int Q = S::Q, M1 = R * R * R, PB = R * (R + 1);
  __shared__ cx<T> lds[S::TPB * S::BUFN];
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t w2 = b % M2;
  const int64_t pg = b / M2;
  const int tid = threadIdx.x;
  const int tr = tid / Q, q = tid % Q;
  const int64_t pair = pg * S::TPB + tr;
  const bool active = pair < P;
  cx<T>* buf = lds + tr * S::BUFN;
  const cx<T> zero = {(T)0, (T)0};
  cx<T> x[R];

  // ---- front: B[e1] for this w2, in registers of thread e1' = q ----------
  if constexpr (SPARSE) {
    for (int i = q; i <= M1; i += Q) buf[i] = zero;
    __syncthreads();
    // slice f_own = q / G owns the residues e1 = f_own (mod F); its rounds
    // carry G items with distinct e1, so each LDS address is updated by one
    // wavefront only, in round order
    const int fo = q / S::G, ln = q % S::G;
    const cx<T>* av = src + (active ? pair : 0) * Upad;
    const cx<T>* tw = twit + w2 * Upad;
    constexpr int RB = 4;
    for (int64_t r0 = 0; r0 < rounds; r0 += RB) {
      int e1[RB];
      cx<T> v[RB], w[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const bool ok = r0 + i < rounds;
        const int64_t u = (((ok ? r0 + i : 0) * S::F) + fo) * S::G + ln;
        e1[i] = ok ? it_e1[u] : M1;
        v[i] = (ok && active) ? av[u] : zero;
        w[i] = tw[u];
      }
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const cx<T> c = cmul(v[i], w[i]);
        const cx<T> acc = buf[e1[i]];
        buf[e1[i]] = acc + c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < R; ++c) x[c] = buf[q + Q * c];
  } else {
    // dense outer DFT already done: B[pair][w2][e1], times W_M^{e1 w2}
    const cx<T>* bv = src + ((active ? pair : 0) * M2 + w2) * M1;
    const cx<T> tq = twi3[w2 * M1 + (int64_t)q * R];  // conj W_M^{q w2} (f = 0 entry)
#pragma unroll
    for (int c = 0; c < R; ++c) {
      cx<T> v = active ? bv[q + Q * c] : zero;
      v = cmulc(v, tq);
      if (c > 0) v = cmulc(v, two[w2 * R + c]);
      x[c] = v;
    }
  }

  // ---- forward step 1: thread e1' = q, DFT over c -> f --------------------
  reg_fft<T, R, -1>(x);
#pragma unroll
  for (int f = 1; f < R; ++f) x[f] = cmul(x[f], twf1[f * Q + q]);
  __syncthreads();
#pragma unroll
  for (int f = 0; f < R; ++f) buf[f * PB + q] = x[f];
  __syncthreads();
  // ---- forward step 2: thread (a, f), q = a + R f: DFT over b -> g --------
  {
    const int a = q % R, f = q / R;
#pragma unroll
    for (int bb = 0; bb < R; ++bb) x[bb] = buf[f * PB + a + R * bb];
    reg_fft<T, R, -1>(x);
#pragma unroll
    for (int g = 1; g < R; ++g) x[g] = cmul(x[g], twf2[g * R + a]);
    __syncthreads();
#pragma unroll
    for (int g = 0; g < R; ++g) buf[(f + R * g) * (R + 1) + a] = x[g];
    __syncthreads();
  }
  // ---- forward step 3: thread (f, g), q = f + R g: DFT over a -> h --------
#pragma unroll
  for (int a = 0; a < R; ++a) x[a] = buf[q * (R + 1) + a];
  reg_fft<T, R, -1>(x);  // x[h] = X[q + R^2 h]

  if constexpr (SPARSE) {
    if (w2 == 0 && q == 0 && active) {  // DC term -> row 0
      X[2 * pair] = phi0 * x[0].x;
      if (2 * pair + 1 < t) X[2 * pair + 1] = phi0 * x[0].y;
    }
  }
  const cx<T>* hs = Hs + w2 * M1;
#pragma unroll
  for (int h = 0; h < R; ++h) x[h] = cmul(x[h], hs[q + Q * h]);

  // ---- inverse step 1: thread (f, g), IDFT over h -> a --------------------
  reg_fft<T, R, +1>(x);
  {
    const int f = q % R, g = q / R;
#pragma unroll
    for (int a = 1; a < R; ++a) x[a] = cmulc(x[a], twf2[g * R + a]);
    __syncthreads();
#pragma unroll
    for (int a = 0; a < R; ++a) buf[(f + R * a) * (R + 1) + g] = x[a];
    __syncthreads();
  }
  // ---- inverse step 2: thread (f, a), q = f + R a: IDFT over g -> b -------
  {
    const int f = q % R, a = q / R;
#pragma unroll
    for (int g = 0; g < R; ++g) x[g] = buf[q * (R + 1) + g];
    reg_fft<T, R, +1>(x);
    const cx<T>* ti = twi3 + w2 * M1;
#pragma unroll
    for (int bb = 0; bb < R; ++bb) {
      const int e1p = a + R * bb;
      if (e1p > 0) x[bb] = cmul(x[bb], ti[e1p * R + f]);
    }
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < R; ++bb) buf[(a + R * bb) * (R + 1) + f] = x[bb];
    __syncthreads();
  }
  // ---- inverse step 3: thread e1' = q, IDFT over f -> c -------------------
#pragma unroll
  for (int f = 0; f < R; ++f) x[f] = buf[q * (R + 1) + f];
  reg_fft<T, R, +1>(x);
  const cx<T>* to = two + w2 * R;
#pragma unroll
  for (int c = 1; c < R; ++c) x[c] = cmul(x[c], to[c]);
  if (active) {
    cx<T>* cp = C + (pair * M2 + w2) * M1;
#pragma unroll
    for (int c = 0; c < R; ++c) cp[q + Q * c] = x[c];
  }
}

// ---------------------------------------------------------------------------
// outer split (only when M2 = P2 * Q2 > 64), in place on C[pair][w2][e1]:
//   DIR = +1 (forward product, first half of the inverse over w2):
//     w2 = q + Q2 p'  ->  index a, times conj W_{M2}^{a q}
//   DIR = -1 (adjoint front, second half of the forward DFT over e2):
//     the values at q + Q2 a (already twiddled by W_{M2}^{a q}) -> p',
//     stored at w2 = q + Q2 p'
// ---------------------------------------------------------------------------
template <typename T, int P2, int DIR>
__global__ __launch_bounds__(64) void k_outer_split(cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                                    int Q2, const cx<T>* __restrict__ twb) {
  const int64_t e1 = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t q = blockIdx.y;
  const int64_t pair = blockIdx.z;
  if (e1 >= M1) return;
  cx<T>* base = C + pair * M2 * M1 + e1;
  cx<T> v[P2];
#pragma unroll
  for (int p = 0; p < P2; ++p) v[p] = base[(q + (int64_t)Q2 * p) * M1];
  reg_fft<T, P2, DIR>(v);
  if constexpr (DIR > 0) {
#pragma unroll
    for (int a = 1; a < P2; ++a) v[a] = cmul(v[a], twb[a * Q2 + q]);
  }
#pragma unroll
  for (int a = 0; a < P2; ++a) base[(q + (int64_t)Q2 * a) * M1] = v[a];
}

// ---------------------------------------------------------------------------
// B: inverse DFT over the Q (= M2 / P2) factor of w2 and the output scatter.
// thread (pair, e1, a): loads C[pair][q + Q a][e1], q < Q, produces e2 = a + P2 b.
//   forward: X[pow[e]][2 pair .. 2 pair + 1] = out[e] for e < L
//   adjoint: dA[j][...] = out[e] + phi0 G[0][...] for every j with l_j = e
// ---------------------------------------------------------------------------
template <typename T, int Q, bool ADJ, bool NT>
__global__ __launch_bounds__(256) void k_back(const cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                              int64_t P2, int64_t L, int64_t P,
                                              const int32_t* __restrict__ rowmap,
                                              const int32_t* __restrict__ inv_ptr,
                                              const int32_t* __restrict__ inv_j,
                                              const T* __restrict__ G0, T phi0,
                                              T* __restrict__ X, int64_t ldx, int64_t t) {
  constexpr int PB = 16, EB = 16;
  constexpr int CH = Q < 16 ? Q : 16;
  __shared__ cx<T> sm[CH][EB][PB + 1];
  const int64_t e1_0 = (int64_t)blockIdx.x * EB, p0 = (int64_t)blockIdx.y * PB;
  const int64_t a = blockIdx.z;
  const int tid = threadIdx.x;
  const int el = tid % EB, pl = tid / EB;
  {
    const int64_t e1 = e1_0 + el, pair = p0 + pl;
    cx<T> v[Q];
    const bool ok = pair < P && e1 < M1;
    const cx<T>* base = C + (ok ? pair : 0) * M2 * M1 + (ok ? e1 : 0);
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = ok ? base[(q + Q * a) * M1] : cx<T>{(T)0, (T)0};
    reg_fft<T, Q, +1>(v);
    const int pw = tid % PB, ew = tid / PB;
    const int64_t pairw = p0 + pw, e1w = e1_0 + ew;
#pragma unroll
    for (int c0 = 0; c0 < Q; c0 += CH) {
      __syncthreads();
#pragma unroll
      for (int c = 0; c < CH; ++c) sm[c][el][pl] = v[c0 + c];
      __syncthreads();
      if (pairw < P && e1w < M1) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int64_t e2 = a + P2 * (c0 + c);
          const int64_t e = e1w + M1 * e2;
          if (e < L) {
            const cx<T> o = sm[c][ew][pw];
            const int64_t col = 2 * pairw;
            if constexpr (!ADJ) {
              T* row = X + (int64_t)rowmap[e] * ldx;
              if constexpr (NT) {
                __builtin_nontemporal_store(o.x, row + col);
                if (col + 1 < t) __builtin_nontemporal_store(o.y, row + col + 1);
              } else {
                row[col] = o.x;
                if (col + 1 < t) row[col + 1] = o.y;
              }
            } else {
              const T g0 = phi0 * G0[col];
              const T g1 = (col + 1 < t) ? phi0 * G0[col + 1] : (T)0;
              for (int32_t jj = inv_ptr[e]; jj < inv_ptr[e + 1]; ++jj) {
                T* row = X + (int64_t)inv_j[jj] * ldx;
                row[col] = o.x + g0;
                if (col + 1 < t) row[col + 1] = o.y + g1;
              }
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint front: g~[m] = G[pow[(L - m) mod L]] (m < L; 0 for L <= m < M)
// gathered with coalesced row reads, then the forward DFT over e2.  With
// M2 = P2 * Q: thread (pair, e1, a) transforms e2 = a + P2 b over b (length
// Q) and multiplies by W_{M2}^{a q}; k_outer_split<-1> finishes over a.
// Output: B[pair][w2][e1] (natural w2 order once the split has run).
// ---------------------------------------------------------------------------
template <typename T, int Q>
__global__ __launch_bounds__(256) void k_adj_front(const T* __restrict__ G, int64_t ldg, int64_t t,
                                                   int64_t M1, int64_t M2, int64_t P2, int64_t L,
                                                   int64_t P, const int32_t* __restrict__ pow,
                                                   const cx<T>* __restrict__ twb,
                                                   cx<T>* __restrict__ B) {
  constexpr int PB = 16, EB = 16;
  constexpr int CH = Q < 16 ? Q : 16;
  __shared__ cx<T> sm[CH][EB][PB + 1];
  const int64_t e1_0 = (int64_t)blockIdx.x * EB, p0 = (int64_t)blockIdx.y * PB;
  const int64_t a = blockIdx.z;
  const int tid = threadIdx.x;
  const int pw = tid % PB, ew = tid / PB;     // gather mapping (pair-fast)
  const int el = tid % EB, pl = tid / EB;     // transform mapping (e1-fast)
  const int64_t pairw = p0 + pw, e1w = e1_0 + ew;
  cx<T> v[Q];
#pragma unroll
  for (int c0 = 0; c0 < Q; c0 += CH) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t e = e1w + M1 * (a + P2 * (c0 + c));
      cx<T> g = {(T)0, (T)0};
      if (pairw < P && e1w < M1 && e < L) {
        const int64_t src = (L - e) % L;
        const T* row = G + (int64_t)pow[src] * ldg;
        const int64_t col = 2 * pairw;
        g.x = row[col];
        if (col + 1 < t) g.y = row[col + 1];
      }
      sm[c][ew][pw] = g;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c0 + c] = sm[c][el][pl];
  }
  reg_fft<T, Q, -1>(v);
  if (P2 > 1) {
#pragma unroll
    for (int q = 1; q < Q; ++q) v[q] = cmulc(v[q], twb[a * Q + q]);
  }
  const int64_t e1 = e1_0 + el, pair = p0 + pl;
  if (pair < P && e1 < M1) {
    cx<T>* base = B + pair * M2 * M1 + e1;
#pragma unroll
    for (int q = 0; q < Q; ++q) base[(q + Q * a) * M1] = v[q];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// pairs of the forward pass whose spectra are resident in the workspace at once
static int64_t fwd_c_pairs(const qmc_plan_s* P, int64_t pairs) {
  const int64_t ch = P->tune.chunk_pairs;
  if (ch <= 0 || ch >= pairs) return pairs;
  const int64_t slots = P->tune.streams == 2 ? 2 : 1;
  return std::min(pairs, ch * slots);
}

size_t workspace_bytes(const qmc_plan_s* P, int64_t t) {
  const size_t el = (P->dtype == QMC_F32) ? sizeof(cx<float>) : sizeof(cx<double>);
  const int64_t pairs = (t + 1) / 2;
  const size_t aT = align256(pairs * P->Upad * el);
  const size_t fwd = aT + align256(fwd_c_pairs(P, pairs) * P->lay.M * el);
  const size_t adj = aT + 2 * align256(pairs * P->lay.M * el);
  return std::max(fwd, adj);
}

template <typename T, int R, bool SPARSE>
static void launch_middle_r(const qmc_plan_s* P, const cx<T>* src, int64_t pairs, cx<T>* C,
                            T* X, int64_t t, hipStream_t st) {
  const Layout& lay = P->lay;
  typedef MidShape<R> S;
  const int64_t groups = (pairs + S::TPB - 1) / S::TPB;
  const int64_t G = groups * lay.M2;
  ProfScope ps(P, SPARSE ? PROF_MIDDLE : PROF_ADJ_MIDDLE, st);
  k_middle<T, R, SPARSE><<<dim3((unsigned)G), dim3(S::BLOCK), 0, st>>>(
      src, P->Upad, P->rounds, P->d_it_e1, (const cx<T>*)P->d_twit, (const cx<T>*)P->d_twf1,
      (const cx<T>*)P->d_twf2, (const cx<T>*)P->d_Hs, (const cx<T>*)P->d_twi3,
      (const cx<T>*)P->d_two, lay.M2, pairs, C, X, t, (T)P->phi0);
}

template <typename T, bool SPARSE>
static int launch_middle(const qmc_plan_s* P, const cx<T>* src, int64_t pairs, cx<T>* C, T* X,
                         int64_t t, hipStream_t st) {
  switch (P->lay.R) {
    case 1: launch_middle_r<T, 1, SPARSE>(P, src, pairs, C, X, t, st); break;
    case 2: launch_middle_r<T, 2, SPARSE>(P, src, pairs, C, X, t, st); break;
    case 4: launch_middle_r<T, 4, SPARSE>(P, src, pairs, C, X, t, st); break;
    case 8: launch_middle_r<T, 8, SPARSE>(P, src, pairs, C, X, t, st); break;
    case 16: launch_middle_r<T, 16, SPARSE>(P, src, pairs, C, X, t, st); break;
    default: return QMC_ERR_UNSUPPORTED;
  }
  return hip_ok(hipGetLastError());
}

template <typename T, int DIR>
static int launch_split(const qmc_plan_s* P, cx<T>* C, int64_t pairs, hipStream_t st) {
  const Layout& lay = P->lay;
  if (lay.P2 == 1) return QMC_OK;
  dim3 grid((unsigned)((lay.M1 + 63) / 64), (unsigned)lay.Q2, (unsigned)pairs);
  const cx<T>* twb = (const cx<T>*)P->d_twb;
  ProfScope ps(P, DIR > 0 ? PROF_SPLIT : PROF_ADJ_SPLIT, st);
  switch (lay.P2) {
    case 2: k_outer_split<T, 2, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, lay.Q2, twb); break;
    case 4: k_outer_split<T, 4, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, lay.Q2, twb); break;
    case 8: k_outer_split<T, 8, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, lay.Q2, twb); break;
    case 16: k_outer_split<T, 16, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, lay.Q2, twb); break;
    case 32: k_outer_split<T, 32, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, lay.Q2, twb); break;
    case 64: k_outer_split<T, 64, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, lay.Q2, twb); break;
    default: return QMC_ERR_UNSUPPORTED;
  }
  return hip_ok(hipGetLastError());
}

template <typename T, bool ADJ, bool NT = false>
static int launch_back(const qmc_plan_s* P, const cx<T>* C, int64_t pairs, const int32_t* inv_ptr,
                       const int32_t* inv_j, const T* G0, T* X, int64_t ldx, int64_t t,
                       hipStream_t st) {
  const Layout& lay = P->lay;
  dim3 grid((unsigned)((lay.M1 + 15) / 16), (unsigned)((pairs + 15) / 16), (unsigned)lay.P2);
  ProfScope ps(P, ADJ ? PROF_ADJ_BACK : PROF_BACK, st);
#define QMC_BACK(QQ)                                                                          \
  k_back<T, QQ, ADJ, NT><<<grid, 256, 0, st>>>(C, lay.M1, lay.M2, lay.P2, P->L, pairs, P->d_pow, \
                                           inv_ptr, inv_j, G0, (T)P->phi0, X, ldx, t)
  switch (lay.Q2) {
    case 1: QMC_BACK(1); break;
    case 2: QMC_BACK(2); break;
    case 4: QMC_BACK(4); break;
    case 8: QMC_BACK(8); break;
    case 16: QMC_BACK(16); break;
    case 32: QMC_BACK(32); break;
    case 64: QMC_BACK(64); break;
    default: return QMC_ERR_UNSUPPORTED;
  }
#undef QMC_BACK
  return hip_ok(hipGetLastError());
}

static int ensure_side_stream(const qmc_plan_s* P) {
  if (!P->side && hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess)
    return QMC_ERR_HIP;
  for (hipEvent_t& e : P->ev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return QMC_ERR_HIP;
  return QMC_OK;
}

template <typename T>
static int back_dispatch(const qmc_plan_s* P, const cx<T>* C, int64_t np, T* X, int64_t ldx,
                         int64_t t, hipStream_t st) {
  if (P->tune.nt_store)
    return launch_back<T, false, true>(P, C, np, nullptr, nullptr, nullptr, X, ldx, t, st);
  return launch_back<T, false, false>(P, C, np, nullptr, nullptr, nullptr, X, ldx, t, st);
}

// X = Y A: collapse-transpose once, then the fused and back passes per chunk
// of column pairs.  With two streams the back pass of chunk c runs on the
// plan's side stream while the caller's stream starts chunk c+1; the two
// spectrum slots alternate and are released by events.
template <typename T>
static int forward_t(const qmc_plan_s* P, const T* A, int64_t t, int64_t lda, T* X, int64_t ldx,
                     void* ws, hipStream_t st) {
  const int64_t pairs = (t + 1) / 2;
  const size_t el = sizeof(cx<T>);
  cx<T>* aT = (cx<T>*)ws;
  cx<T>* Cbase = (cx<T>*)((char*)ws + align256(pairs * P->Upad * el));
  dim3 gT((unsigned)((P->Upad + 63) / 64), (unsigned)((pairs + 15) / 16));
  {
    ProfScope ps(P, PROF_COLLAPSE, st);
    k_collapse_T<T><<<gT, 256, 0, st>>>(A, lda, t, pairs, P->d_it_j, P->Upad, aT);
  }
  int rc = hip_ok(hipGetLastError());
  if (rc != QMC_OK) return rc;
  const int64_t chunk = (P->tune.chunk_pairs > 0 && P->tune.chunk_pairs < pairs)
                            ? P->tune.chunk_pairs : pairs;
  const bool two = P->tune.streams == 2 && chunk < pairs;
  hipStream_t sb = st;
  if (two) {
    if ((rc = ensure_side_stream(P)) != QMC_OK) return rc;
    sb = P->side;
    // fork: the side stream starts after everything already on st
    if ((rc = hip_ok(hipEventRecord(P->ev[4], st))) != QMC_OK) return rc;
    if ((rc = hip_ok(hipStreamWaitEvent(sb, P->ev[4], 0))) != QMC_OK) return rc;
  }
  int64_t c = 0;
  for (int64_t p0 = 0; p0 < pairs; p0 += chunk, ++c) {
    const int64_t np = std::min(chunk, pairs - p0);
    const int slot = two ? (int)(c & 1) : 0;
    cx<T>* C = Cbase + (int64_t)slot * chunk * P->lay.M;
    if (two && c >= 2) {  // the back pass of chunk c-2 has released this slot
      if ((rc = hip_ok(hipStreamWaitEvent(st, P->ev[2 + slot], 0))) != QMC_OK) return rc;
    }
    rc = launch_middle<T, true>(P, aT + p0 * P->Upad, np, C, X + 2 * p0, t - 2 * p0, st);
    if (rc != QMC_OK) return rc;
    rc = launch_split<T, +1>(P, C, np, st);
    if (rc != QMC_OK) return rc;
    if (two) {
      if ((rc = hip_ok(hipEventRecord(P->ev[slot], st))) != QMC_OK) return rc;
      if ((rc = hip_ok(hipStreamWaitEvent(sb, P->ev[slot], 0))) != QMC_OK) return rc;
    }
    rc = back_dispatch<T>(P, C, np, X + 2 * p0, ldx, t - 2 * p0, sb);
    if (rc != QMC_OK) return rc;
    if (two) {
      if ((rc = hip_ok(hipEventRecord(P->ev[2 + slot], sb))) != QMC_OK) return rc;
    }
  }
  if (two) {  // join
    if ((rc = hip_ok(hipEventRecord(P->ev[5], sb))) != QMC_OK) return rc;
    if ((rc = hip_ok(hipStreamWaitEvent(st, P->ev[5], 0))) != QMC_OK) return rc;
  }
  return QMC_OK;
}

int launch_forward(const qmc_plan_s* P, const void* A, int64_t t, int64_t lda, void* X,
                   int64_t ldx, void* ws, hipStream_t st) {
  if (P->dtype == QMC_F32)
    return forward_t<float>(P, (const float*)A, t, lda, (float*)X, ldx, ws, st);
  return forward_t<double>(P, (const double*)A, t, lda, (double*)X, ldx, ws, st);
}

template <typename T>
static int launch_adj_front(const qmc_plan_s* P, const T* G, int64_t ldg, int64_t t,
                            int64_t pairs, cx<T>* B, hipStream_t st) {
  const Layout& lay = P->lay;
  dim3 grid((unsigned)((lay.M1 + 15) / 16), (unsigned)((pairs + 15) / 16), (unsigned)lay.P2);
  const cx<T>* twb = (const cx<T>*)P->d_twb;
  {
    ProfScope ps(P, PROF_ADJ_FRONT, st);
#define QMC_AFRONT(QQ)                                                                        \
  k_adj_front<T, QQ><<<grid, 256, 0, st>>>(G, ldg, t, lay.M1, lay.M2, lay.P2, P->L, pairs, \
                                           P->d_pow, twb, B)
    switch (lay.Q2) {
      case 1: QMC_AFRONT(1); break;
      case 2: QMC_AFRONT(2); break;
      case 4: QMC_AFRONT(4); break;
      case 8: QMC_AFRONT(8); break;
      case 16: QMC_AFRONT(16); break;
      case 32: QMC_AFRONT(32); break;
      case 64: QMC_AFRONT(64); break;
      default: return QMC_ERR_UNSUPPORTED;
    }
#undef QMC_AFRONT
  }
  int rc = hip_ok(hipGetLastError());
  if (rc != QMC_OK) return rc;
  return launch_split<T, -1>(P, B, pairs, st);
}

template <typename T>
static int adjoint_t(const qmc_plan_s* P, const T* G, int64_t t, int64_t ldg, T* dA,
                     int64_t ldda, void* ws, hipStream_t st) {
  const int64_t pairs = (t + 1) / 2;
  const size_t el = sizeof(cx<T>);
  cx<T>* B = (cx<T>*)((char*)ws + align256(pairs * P->Upad * el));
  cx<T>* C = (cx<T>*)((char*)B + align256(pairs * P->lay.M * el));
  int rc = launch_adj_front<T>(P, G, ldg, t, pairs, B, st);
  if (rc != QMC_OK) return rc;
  rc = launch_middle<T, false>(P, B, pairs, C, nullptr, t, st);
  if (rc != QMC_OK) return rc;
  rc = launch_split<T, +1>(P, C, pairs, st);
  if (rc != QMC_OK) return rc;
  return launch_back<T, true>(P, C, pairs, P->d_inv_ptr, P->d_inv_j, G, dA, ldda, t, st);
}

int launch_adjoint(const qmc_plan_s* P, const void* G, int64_t t, int64_t ldg, void* dA,
                   int64_t ldda, void* ws, hipStream_t st) {
  if (P->dtype == QMC_F32)
    return adjoint_t<float>(P, (const float*)G, t, ldg, (float*)dA, ldda, ws, st);
  return adjoint_t<double>(P, (const double*)G, t, ldg, (double*)dA, ldda, ws, st);
}

}  // namespace qmc
