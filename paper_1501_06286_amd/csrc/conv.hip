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
//      length-M1 DFT (two register DFTs of length R = sqrt(M1) across the
//      lanes of a wavefront with one LDS exchange), the spectral product,
//      the inverse length-M1 DFT and the outer twiddle; the DC term gives
//      row 0;
//   B  for a tile of (e1, pairs): the inverse DFT over w2 and the row
//      un-permutation X[pow[e]] (or, for the adjoint, the read-back at the
//      exponents l_j).
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
// F: one (outer frequency w2, pair) per R lanes, 64/R pairs per wavefront
// ---------------------------------------------------------------------------
template <typename T, int R, bool SPARSE>
__global__ __launch_bounds__(64) void k_middle(
    const cx<T>* __restrict__ src,      // SPARSE: aT [pair][Upad]; dense: B [pair][M2][M1]
    int64_t Upad, int64_t rounds, const int32_t* __restrict__ it_e1,
    const cx<T>* __restrict__ twit, const cx<T>* __restrict__ twf, const cx<T>* __restrict__ Hs,
    const cx<T>* __restrict__ twi, const cx<T>* __restrict__ two, int64_t M1, int64_t M2,
    int64_t P, cx<T>* __restrict__ C, T* __restrict__ X, int64_t ldx, int64_t t, T phi0) {
  constexpr int TPW = 64 / R;
  constexpr int PITCH = R + 1;
  constexpr int BUF = R * PITCH;
  __shared__ cx<T> lds[TPW * BUF];
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t w2 = b % M2;
  const int64_t pg = b / M2;
  const int lane = threadIdx.x;
  const int tau = lane / R, k = lane % R;
  const int64_t pair = pg * TPW + tau;
  const bool active = pair < P;
  cx<T>* buf = lds + tau * BUF;
  const cx<T> zero = {(T)0, (T)0};
  cx<T> x[R];

  if constexpr (SPARSE) {
    // sparse outer DFT over e2 into buf[e1] (buf[M1] absorbs padding items)
    for (int64_t i = k; i <= M1; i += R) buf[i] = zero;
    __syncthreads();
    const cx<T>* av = src + (active ? pair : 0) * Upad;
    const cx<T>* tw = twit + w2 * Upad;
    for (int64_t r = 0; r < rounds; ++r) {
      const int64_t u = r * R + k;
      const int e1 = it_e1[u];
      const cx<T> v = active ? av[u] : zero;
      const cx<T> c = cmul(v, tw[u]);
      const cx<T> acc = buf[e1];
      buf[e1] = acc + c;
    }
    __syncthreads();
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) x[n2] = buf[k + R * n2];
  } else {
    // dense outer DFT already done: load B[pair][w2][e1] and apply the outer
    // twiddle W_M^{e1 w2} = W_M^{k w2} W_M^{R n2 w2} (conjugates of the
    // inverse tables)
    const cx<T>* bv = src + ((active ? pair : 0) * M2 + w2) * M1;
    const cx<T> tk = twi[(w2 * R + k) * R];
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) {
      cx<T> v = active ? bv[k + R * n2] : zero;
      v = cmulc(v, tk);
      if (n2 > 0) v = cmulc(v, two[w2 * R + n2]);
      x[n2] = v;
    }
  }

  // length-M1 forward DFT: e1 = k1 + R n2 -> w1 = m2 + R m1
  reg_fft<T, R, -1>(x);  // over n2 -> m2 (lane = k1)
#pragma unroll
  for (int m2 = 1; m2 < R; ++m2) x[m2] = cmul(x[m2], twf[m2 * R + k]);
  __syncthreads();
#pragma unroll
  for (int m2 = 0; m2 < R; ++m2) buf[m2 * PITCH + k] = x[m2];
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) x[k1] = buf[k * PITCH + k1];
  reg_fft<T, R, -1>(x);  // over k1 -> m1 (lane = m2)

  if constexpr (SPARSE) {
    // DC term: sum of the collapsed column pair = sum_j A[j, :] -> row 0
    if (w2 == 0 && k == 0 && active) {
      X[2 * pair] = phi0 * x[0].x;
      if (2 * pair + 1 < t) X[2 * pair + 1] = phi0 * x[0].y;
    }
  }

  // spectral product (the spectrum carries the 1/M of the inverse)
  const cx<T>* hs = Hs + w2 * M1;
#pragma unroll
  for (int m1 = 0; m1 < R; ++m1) x[m1] = cmul(x[m1], hs[k + R * m1]);

  // inverse length-M1 DFT: w1 = m2 + R m1 -> e1 = k1 + R n2
  reg_fft<T, R, +1>(x);  // over m1 -> k1 (lane = m2)
  const cx<T>* ti = twi + w2 * R * R;
#pragma unroll
  for (int k1 = 1; k1 < R; ++k1) x[k1] = cmul(x[k1], ti[k1 * R + k]);
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) buf[k1 * PITCH + k] = x[k1];
  __syncthreads();
#pragma unroll
  for (int m2 = 0; m2 < R; ++m2) x[m2] = buf[k * PITCH + m2];
  reg_fft<T, R, +1>(x);  // over m2 -> n2 (lane = k1)
  const cx<T>* to = two + w2 * R;
#pragma unroll
  for (int n2 = 1; n2 < R; ++n2) x[n2] = cmul(x[n2], to[n2]);
  if (active) {
    cx<T>* c = C + (pair * M2 + w2) * M1;
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) c[k + R * n2] = x[n2];
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
template <typename T, int Q, bool ADJ>
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
              row[col] = o.x;
              if (col + 1 < t) row[col + 1] = o.y;
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

size_t workspace_bytes(const qmc_plan_s* P, int64_t t) {
  const size_t el = (P->dtype == QMC_F32) ? sizeof(cx<float>) : sizeof(cx<double>);
  const int64_t pairs = (t + 1) / 2;
  return align256(pairs * P->Upad * el) + align256(pairs * P->lay.M * el) +
         align256(pairs * P->lay.M * el);
}

template <typename T, int R, bool SPARSE>
static void launch_middle_r(const qmc_plan_s* P, const cx<T>* src, int64_t pairs, cx<T>* C,
                            T* X, int64_t ldx, int64_t t, hipStream_t st) {
  const Layout& lay = P->lay;
  constexpr int TPW = 64 / R;
  const int64_t groups = (pairs + TPW - 1) / TPW;
  const int64_t G = groups * lay.M2;
  ProfScope ps(P, SPARSE ? PROF_MIDDLE : PROF_ADJ_MIDDLE, st);
  k_middle<T, R, SPARSE><<<dim3((unsigned)G), dim3(64), 0, st>>>(
      src, P->Upad, P->rounds, P->d_it_e1, (const cx<T>*)P->d_twit, (const cx<T>*)P->d_twf,
      (const cx<T>*)P->d_Hs, (const cx<T>*)P->d_twi, (const cx<T>*)P->d_two, lay.M1, lay.M2,
      pairs, C, X, ldx, t, (T)P->phi0);
}

template <typename T, bool SPARSE>
static int launch_middle(const qmc_plan_s* P, const cx<T>* src, int64_t pairs, cx<T>* C, T* X,
                         int64_t ldx, int64_t t, hipStream_t st) {
  switch (P->lay.R) {
    case 1: launch_middle_r<T, 1, SPARSE>(P, src, pairs, C, X, ldx, t, st); break;
    case 2: launch_middle_r<T, 2, SPARSE>(P, src, pairs, C, X, ldx, t, st); break;
    case 4: launch_middle_r<T, 4, SPARSE>(P, src, pairs, C, X, ldx, t, st); break;
    case 8: launch_middle_r<T, 8, SPARSE>(P, src, pairs, C, X, ldx, t, st); break;
    case 16: launch_middle_r<T, 16, SPARSE>(P, src, pairs, C, X, ldx, t, st); break;
    case 32: launch_middle_r<T, 32, SPARSE>(P, src, pairs, C, X, ldx, t, st); break;
    case 64:
      if constexpr (sizeof(T) == 4) {
        launch_middle_r<T, 64, SPARSE>(P, src, pairs, C, X, ldx, t, st);
        break;
      }
      return QMC_ERR_UNSUPPORTED;
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

template <typename T, bool ADJ>
static int launch_back(const qmc_plan_s* P, const cx<T>* C, int64_t pairs, const int32_t* inv_ptr,
                       const int32_t* inv_j, const T* G0, T* X, int64_t ldx, int64_t t,
                       hipStream_t st) {
  const Layout& lay = P->lay;
  dim3 grid((unsigned)((lay.M1 + 15) / 16), (unsigned)((pairs + 15) / 16), (unsigned)lay.P2);
  ProfScope ps(P, ADJ ? PROF_ADJ_BACK : PROF_BACK, st);
#define QMC_BACK(QQ)                                                                          \
  k_back<T, QQ, ADJ><<<grid, 256, 0, st>>>(C, lay.M1, lay.M2, lay.P2, P->L, pairs, P->d_pow, \
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

template <typename T>
static int forward_t(const qmc_plan_s* P, const T* A, int64_t t, int64_t lda, T* X, int64_t ldx,
                     void* ws, hipStream_t st) {
  const int64_t pairs = (t + 1) / 2;
  const size_t el = sizeof(cx<T>);
  cx<T>* aT = (cx<T>*)ws;
  cx<T>* C = (cx<T>*)((char*)ws + align256(pairs * P->Upad * el));
  dim3 gT((unsigned)((P->Upad + 63) / 64), (unsigned)((pairs + 15) / 16));
  {
    ProfScope ps(P, PROF_COLLAPSE, st);
    k_collapse_T<T><<<gT, 256, 0, st>>>(A, lda, t, pairs, P->d_it_j, P->Upad, aT);
  }
  int rc = hip_ok(hipGetLastError());
  if (rc != QMC_OK) return rc;
  rc = launch_middle<T, true>(P, aT, pairs, C, X, ldx, t, st);
  if (rc != QMC_OK) return rc;
  rc = launch_split<T, +1>(P, C, pairs, st);
  if (rc != QMC_OK) return rc;
  return launch_back<T, false>(P, C, pairs, nullptr, nullptr, nullptr, X, ldx, t, st);
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
  rc = launch_middle<T, false>(P, B, pairs, C, nullptr, 0, t, st);
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
