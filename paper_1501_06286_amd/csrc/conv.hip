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

#include "kernels.hpp"

namespace qmc {
// ---------------------------------------------------------------------------
// single-product kernels: thin wrappers around the bodies of kernels.hpp
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_collapse_T(const T* __restrict__ A, int64_t lda,
                                                    int64_t t, int64_t P,
                                                    const int32_t* __restrict__ it_ptr,
                                                    const int32_t* __restrict__ it_jl, int64_t Upad,
                                                    cx<T>* __restrict__ aT) {
  __shared__ CollapseSmem<T> S;
  collapse_body<T>(A, lda, t, P, it_ptr, it_jl, Upad, aT, blockIdx.x, blockIdx.y, S,
                   threadIdx.x);
}

template <typename T, int R, bool SPARSE, bool BTW>
__global__ __launch_bounds__(MidShape<R>::BLOCK)
__attribute__((amdgpu_waves_per_eu(mid_waves<T, R>()))) void k_middle(
    const cx<T>* __restrict__ src, int64_t Upad, int64_t rounds, const uint16_t* __restrict__ it_e1,
    const cx<T>* __restrict__ twit, const cx<T>* __restrict__ twf1,
    const cx<T>* __restrict__ twf2, const cx<T>* __restrict__ Hs,
    const cx<T>* __restrict__ twi3, const cx<T>* __restrict__ two, int64_t M2, int64_t P,
    cx<T>* __restrict__ C, T* __restrict__ X, int64_t t, T phi0, int nt_c,
    const uint16_t* __restrict__ it_e2, const cx<T>* __restrict__ twb) {
  __shared__ MidSmem<T, R> S;
  middle_body<T, R, SPARSE, BTW>(src, Upad, rounds, it_e1, twit, twf1, twf2, Hs, twi3, two, M2,
                                 P, C, X, t, phi0, xcd_remap(blockIdx.x, gridDim.x), S,
                                 threadIdx.x, nt_c != 0, it_e2, twb);
}

template <typename T, int R, bool SPARSE>
__global__ __launch_bounds__(MidShape<R>::BLOCK)
__attribute__((amdgpu_waves_per_eu(mid_sum_waves<T, R>()))) void k_middle_sum(
    const MidTerms<T> terms, const cx<T>* __restrict__ twf1, const cx<T>* __restrict__ twf2,
    const cx<T>* __restrict__ twi3, const cx<T>* __restrict__ two, int64_t M2, int64_t P,
    cx<T>* __restrict__ C, int nt_c) {
  __shared__ MidSmem<T, R> S;
  middle_sum_body<T, R, SPARSE>(terms, twf1, twf2, twi3, two, M2, P, C,
                                xcd_remap(blockIdx.x, gridDim.x), S, threadIdx.x, nt_c != 0);
}

template <typename T, int P2, int DIR>
__global__ __launch_bounds__(64) void k_outer_split(cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                                    int Q2, const cx<T>* __restrict__ twb) {
  split_body<T, P2, DIR>(C, M1, M2, Q2, twb, blockIdx.x, blockIdx.y, blockIdx.z, threadIdx.x);
}

template <typename T, int Q, bool ADJ, bool NT, bool EPI, int EB = 16, int PB = 16>
__global__ __launch_bounds__(EB * PB)
__attribute__((amdgpu_waves_per_eu(back_waves<T, Q>()))) void k_back(const cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                              int64_t P2, int64_t L, int64_t P,
                                              const int32_t* __restrict__ rowmap,
                                              const int32_t* __restrict__ inv_ptr,
                                              const int32_t* __restrict__ inv_j,
                                              const T* __restrict__ G0, T phi0,
                                              T* __restrict__ X, int64_t ldx, int64_t t,
                                              Epi<T> epi) {
  __shared__ BackSmem<T, EB, PB> S;
  back_body<T, Q, ADJ, NT, EPI, EB, PB>(C, M1, M2, P2, L, P, rowmap, inv_ptr, inv_j, G0, phi0,
                                        X, ldx, t, blockIdx.x, blockIdx.y, blockIdx.z, S,
                                        threadIdx.x, epi);
}

template <typename T, int Q, bool ADJ, bool NT, bool EPI, int TE, int NW>
__global__ __launch_bounds__((BackLdsShape<Q, TE, NW>::BLOCK)) void k_back_lds(const cx<T>* __restrict__ C, int64_t M1,
                                                  int64_t M2, int64_t P2, int64_t L, int64_t P,
                                                  const cx<T>* __restrict__ twb,
                                                  const int32_t* __restrict__ rowmap,
                                                  const int32_t* __restrict__ inv_ptr,
                                                  const int32_t* __restrict__ inv_j,
                                                  const T* __restrict__ G0, T phi0,
                                                  T* __restrict__ X, int64_t ldx, int64_t t,
                                                  Epi<T> epi) {
  __shared__ BackLdsSmem<T, Q, TE> S;
  int64_t bx, by, a;
  back_lds_tile(blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z),
                gridDim.x, gridDim.y, gridDim.z, bx, by, a);
  back_lds_body<T, Q, ADJ, NT, EPI, TE, NW>(C, M1, M2, P2, L, P, twb, rowmap, inv_ptr, inv_j, G0,
                                        phi0, X, ldx, t, bx, by, a, S, threadIdx.x, epi);
}

// the epilogue of row 0 (its values come from the fused pass's DC term)
template <typename T>
__global__ __launch_bounds__(256) void k_epi_row0(T* __restrict__ X, int64_t t, Epi<T> epi) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t) return;
  const EpiCols<T> ec(epi, c, t);
  X[c] = ec.f0(X[c]);
}

template <typename T, int Q>
__global__ __launch_bounds__(256) void k_adj_front(const T* __restrict__ G, int64_t ldg, int64_t t,
                                                   int64_t M1, int64_t M2, int64_t P2, int64_t L,
                                                   int64_t P, const int32_t* __restrict__ pow,
                                                   const cx<T>* __restrict__ twb,
                                                   cx<T>* __restrict__ B) {
  __shared__ BackSmem<T> S;
  const AdjGather<T> g{{G, ldg, t, pairs_aligned(G, ldg)}, pow, L};
  outer_front_body<T, Q>(g, M1, M2, P2, L, P, twb, B, blockIdx.x, blockIdx.y, blockIdx.z, S,
                         threadIdx.x);
}

template <typename T, int Q>
__global__ __launch_bounds__(256) void k_fwd_front(const T* __restrict__ A, int64_t lda, int64_t t,
                                                   int64_t M1, int64_t M2, int64_t P2, int64_t L,
                                                   int64_t P, const int32_t* __restrict__ inv_ptr,
                                                   const int32_t* __restrict__ inv_j,
                                                   const cx<T>* __restrict__ twb,
                                                   cx<T>* __restrict__ B) {
  __shared__ BackSmem<T> S;
  const FwdGather<T> g{{A, lda, t, pairs_aligned(A, lda)}, inv_ptr, inv_j, L};
  outer_front_body<T, Q>(g, M1, M2, P2, L, P, twb, B, blockIdx.x, blockIdx.y, blockIdx.z, S,
                         threadIdx.x);
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

// whether qmc_matmul uses the dense outer front (tuning field front; 0 picks
// it when the sparse front's per-frequency sums over all s rows cost more
// than the extra passes over the length-M columns: measured on MI355X, the
// two break even near s = 4 M1, so the switch is at s > 8 M1)
bool dense_front(const qmc_plan_s* P) {
  if (P->tune.front != 0) return P->tune.front == 2;
  return P->s_active > 8 * P->lay.M1;
}

// whether the fused pass writes the intermediate spectrum C with streaming
// stores (tuning nt_inter: 0 = when the intermediates of one launch, c_bytes
// (C, and B with the dense fronts), are too large to stay in the 256 MB
// Infinity Cache for the back pass, 1 = never, 2 = always)
static bool nt_inter(const qmc_plan_s* P, int64_t c_bytes) {
  if (P->tune.nt_inter != 0) return P->tune.nt_inter == 2;
  return c_bytes > ((int64_t)128 << 20);
}

// column pairs per chunk of the adjoint: the tuning's chunk, as for the
// forward product (B and C of a chunk then stay in the Infinity Cache)
static int64_t adj_chunk(const qmc_plan_s* P, int64_t pairs) {
  return (P->tune.chunk_pairs > 0 && P->tune.chunk_pairs < pairs) ? P->tune.chunk_pairs : pairs;
}

size_t workspace_bytes(const qmc_plan_s* P, int64_t t) {
  if (P->comp) return composite_workspace_bytes(P, t);
  const size_t el = (P->dtype == QMC_F32) ? sizeof(cx<float>) : sizeof(cx<double>);
  const int64_t pairs = (t + 1) / 2;
  const size_t aT = align256(pairs * P->Upad * el);
  const int64_t chunk = (P->tune.chunk_pairs > 0 && P->tune.chunk_pairs < pairs)
                            ? P->tune.chunk_pairs : pairs;
  const size_t fwd = dense_front(P) ? 2 * align256(chunk * P->lay.M * el)
                                    : aT + align256(fwd_c_pairs(P, pairs) * P->lay.M * el);
  const size_t adj = 2 * align256(adj_chunk(P, pairs) * P->lay.M * el);
  return std::max(fwd, adj);
}

template <typename T, int R, bool SPARSE>
static void launch_middle_r(const qmc_plan_s* P, const cx<T>* src, int64_t pairs, cx<T>* C,
                            T* X, int64_t t, int slot, hipStream_t st) {
  const Layout& lay = P->lay;
  typedef MidShape<R> S;
  const int64_t groups = (pairs + S::TPB - 1) / S::TPB;
  const int64_t G = groups * lay.M2;
  ProfScope ps(P, slot, st);
  const int ntc = nt_inter(P, (SPARSE ? 1 : 2) * pairs * lay.M * (int64_t)sizeof(cx<T>)) ? 1 : 0;
  // the sparse front with bucket twiddles (tuning front = 3; its twiddle
  // index needs M2 a power of two, other M2 take the item twiddles)
  if (SPARSE && P->tune.front == 3 && (lay.M2 & (lay.M2 - 1)) == 0)
    k_middle<T, R, SPARSE, true><<<dim3((unsigned)G), dim3(S::BLOCK), 0, st>>>(
        src, P->Upad, P->rounds, P->d_it_e1, nullptr, (const cx<T>*)P->d_twf1,
        (const cx<T>*)P->d_twf2, (const cx<T>*)P->d_Hs, (const cx<T>*)P->d_twi3,
        (const cx<T>*)P->d_two, lay.M2, pairs, C, X, t, (T)P->phi0, ntc, P->d_it_e2,
        (const cx<T>*)P->d_twb);
  else
    k_middle<T, R, SPARSE, false><<<dim3((unsigned)G), dim3(S::BLOCK), 0, st>>>(
        src, P->Upad, P->rounds, P->d_it_e1, (const cx<T>*)P->d_twit, (const cx<T>*)P->d_twf1,
        (const cx<T>*)P->d_twf2, (const cx<T>*)P->d_Hs, (const cx<T>*)P->d_twi3,
        (const cx<T>*)P->d_two, lay.M2, pairs, C, X, t, (T)P->phi0, ntc, nullptr, nullptr);
}

// X != nullptr: forward product, the DC term of each pair goes to row 0
template <typename T, bool SPARSE>
static int launch_middle(const qmc_plan_s* P, const cx<T>* src, int64_t pairs, cx<T>* C, T* X,
                         int64_t t, int slot, hipStream_t st) {
  switch (P->lay.R) {
    case 1: launch_middle_r<T, 1, SPARSE>(P, src, pairs, C, X, t, slot, st); break;
    case 2: launch_middle_r<T, 2, SPARSE>(P, src, pairs, C, X, t, slot, st); break;
    case 4: launch_middle_r<T, 4, SPARSE>(P, src, pairs, C, X, t, slot, st); break;
    case 8: launch_middle_r<T, 8, SPARSE>(P, src, pairs, C, X, t, slot, st); break;
    case 16: launch_middle_r<T, 16, SPARSE>(P, src, pairs, C, X, t, slot, st); break;
    default: return QMC_ERR_UNSUPPORTED;
  }
  return hip_ok(hipGetLastError());
}

template <typename T, int DIR>
static int launch_split(const qmc_plan_s* P, cx<T>* C, int64_t pairs, int slot, hipStream_t st) {
  const Layout& lay = P->lay;
  // the back pass's split (DIR = +1) or the dense fronts' (DIR = -1)
  const int p2 = DIR > 0 ? lay.P2 : lay.Pf, q2 = DIR > 0 ? lay.Q2 : lay.Qf;
  if (p2 == 1) return QMC_OK;
  dim3 grid((unsigned)((lay.M1 + 63) / 64), (unsigned)q2, (unsigned)pairs);
  const cx<T>* twb = (const cx<T>*)P->d_twb;
  ProfScope ps(P, slot, st);
  switch (p2) {
    case 2: k_outer_split<T, 2, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, q2, twb); break;
    case 4: k_outer_split<T, 4, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, q2, twb); break;
    case 8: k_outer_split<T, 8, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, q2, twb); break;
    case 16: k_outer_split<T, 16, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, q2, twb); break;
    case 32: k_outer_split<T, 32, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, q2, twb); break;
    case 64: k_outer_split<T, 64, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, q2, twb); break;
    default: return QMC_ERR_UNSUPPORTED;
  }
  return hip_ok(hipGetLastError());
}

template <typename T, bool ADJ, bool NT = false, bool EPI = false>
static int launch_back(const qmc_plan_s* P, const cx<T>* C, int64_t pairs, const int32_t* inv_ptr,
                       const int32_t* inv_j, const T* G0, T* X, int64_t ldx, int64_t t,
                       hipStream_t st, const Epi<T>& epi = Epi<T>()) {
  const Layout& lay = P->lay;
  ProfScope ps(P, ADJ ? PROF_ADJ_BACK : PROF_BACK, st);
  // the outer factor through LDS, tiles of TE e1 x 8 pairs: Q2 = 40, 48, 64,
  // 80, 96 and 128, and 32 in FP64 (its register variant takes all 256
  // registers and spills; in FP32 the register variant is the faster one)
  if (back_in_lds(lay.Q2, sizeof(T) == 8)) {
    constexpr int TE = back_lds_te<T>();
    dim3 gl((unsigned)((lay.M1 + TE - 1) / TE), (unsigned)((pairs + 7) / 8), (unsigned)lay.P2);
#define QMC_BACKL(QQ)                                                                        \
  k_back_lds<T, QQ, ADJ, NT, EPI, TE, back_lds_nw<T, QQ, ADJ>()>                               \
      <<<gl, BackLdsShape<QQ, TE, back_lds_nw<T, QQ, ADJ>()>::BLOCK, 0, st>>>(                \
          C, lay.M1, lay.M2, lay.P2, P->L, pairs, (const cx<T>*)P->d_twb, out_rows(P), inv_ptr, \
          inv_j, G0, (T)P->phi0, X, ldx, t, epi)
    if (lay.Q2 == 40) {
      QMC_BACKL(40);
    } else if (lay.Q2 == 48) {
      QMC_BACKL(48);
    } else if (lay.Q2 == 64) {
      QMC_BACKL(64);
    } else if constexpr (sizeof(T) == 4) {
      if (lay.Q2 == 80) {
        QMC_BACKL(80);
      } else if (lay.Q2 == 96) {
        QMC_BACKL(96);
      } else {
        if (lay.Q2 != 128) return QMC_ERR_UNSUPPORTED;
        QMC_BACKL(128);
      }
    } else {
      if (lay.Q2 != 32) return QMC_ERR_UNSUPPORTED;
      QMC_BACKL(32);
    }
#undef QMC_BACKL
    return hip_ok(hipGetLastError());
  }
  if constexpr (sizeof(T) == 8 && !ADJ) {
    // FP64 forward at Q2 = 16 (the Gaussian workload): tiles of 64 e1 x 8
    // pairs (measured: the product 1.80 -> 1.76 ms; no gain for the adjoint)
    if (lay.Q2 == 16) {
      dim3 g8((unsigned)((lay.M1 + 63) / 64), (unsigned)((pairs + 7) / 8), (unsigned)lay.P2);
      k_back<T, 16, false, NT, EPI, 64, 8><<<g8, 512, 0, st>>>(
          C, lay.M1, lay.M2, lay.P2, P->L, pairs, out_rows(P), inv_ptr, inv_j, G0, (T)P->phi0, X,
          ldx, t, epi);
      return hip_ok(hipGetLastError());
    }
  }
  dim3 grid((unsigned)((lay.M1 + 15) / 16), (unsigned)((pairs + 15) / 16), (unsigned)lay.P2);
#define QMC_BACK(QQ)                                                                          \
  k_back<T, QQ, ADJ, NT, EPI><<<grid, 256, 0, st>>>(C, lay.M1, lay.M2, lay.P2, P->L, pairs, out_rows(P), \
                                           inv_ptr, inv_j, G0, (T)P->phi0, X, ldx, t, epi)
  switch (lay.Q2) {
    case 1: QMC_BACK(1); break;
    case 2: QMC_BACK(2); break;
    case 4: QMC_BACK(4); break;
    case 8: QMC_BACK(8); break;
    case 16: QMC_BACK(16); break;
    case 32: QMC_BACK(32); break;
    case 3: QMC_BACK(3); break;
    case 6: QMC_BACK(6); break;
    case 12: QMC_BACK(12); break;
    case 24: QMC_BACK(24); break;
    case 5: QMC_BACK(5); break;
    case 10: QMC_BACK(10); break;
    case 20: QMC_BACK(20); break;
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
                         int64_t t, hipStream_t st, const Epi<T>& epi) {
  if (epi.kind != 0) {
    if (P->tune.nt_store)
      return launch_back<T, false, true, true>(P, C, np, nullptr, nullptr, nullptr, X, ldx, t, st,
                                               epi);
    return launch_back<T, false, false, true>(P, C, np, nullptr, nullptr, nullptr, X, ldx, t, st,
                                              epi);
  }
  if (P->tune.nt_store)
    return launch_back<T, false, true>(P, C, np, nullptr, nullptr, nullptr, X, ldx, t, st);
  return launch_back<T, false, false>(P, C, np, nullptr, nullptr, nullptr, X, ldx, t, st);
}

// X = Y A: collapse-transpose once, then the fused and back passes per chunk
// of column pairs.  With two streams the back pass of chunk c runs on the
// plan's side stream while the caller's stream starts chunk c+1; the two
// spectrum slots alternate and are released by events.
// the epilogue of the columns from pair p0 on
template <typename T>
static Epi<T> chunk_epi(const Epi<T>& e, int64_t p0) {
  return Epi<T>{e.kind, e.bias ? e.bias + 2 * p0 : nullptr, e.scale ? e.scale + 2 * p0 : nullptr};
}

// X = Y A with the dense outer front, per chunk of column pairs: gather and
// transform the outer index into B, the fused pass (dense front) into C, the
// outer split and the back pass.  One stream.
template <typename T>
static int forward_dense_t(const qmc_plan_s* P, const T* A, int64_t t, int64_t lda, T* X,
                           int64_t ldx, void* ws, hipStream_t st, const Epi<T>& epi) {
  const int64_t pairs = (t + 1) / 2;
  const int64_t chunk = (P->tune.chunk_pairs > 0 && P->tune.chunk_pairs < pairs)
                            ? P->tune.chunk_pairs : pairs;
  cx<T>* B = (cx<T>*)ws;
  cx<T>* C = (cx<T>*)((char*)ws + align256(chunk * P->lay.M * sizeof(cx<T>)));
  for (int64_t p0 = 0; p0 < pairs; p0 += chunk) {
    const int64_t np = std::min(chunk, pairs - p0), tc = t - 2 * p0;
    int rc = launch_outer_front<T>(P, A + 2 * p0, nullptr, lda, tc, np, B, st);
    if (rc != QMC_OK) return rc;
    const Epi<T> ec = chunk_epi(epi, p0);
    // a block of a lattice rule with non-prime N does not hold row 0
    rc = launch_middle<T, false>(P, B, np, C, P->sub ? nullptr : X + 2 * p0, tc, PROF_MIDDLE, st);
    if (rc != QMC_OK) return rc;
    rc = launch_split<T, +1>(P, C, np, PROF_SPLIT, st);
    if (rc != QMC_OK) return rc;
    rc = back_dispatch<T>(P, C, np, X + 2 * p0, ldx, tc, st, ec);
    if (rc != QMC_OK) return rc;
  }
  return QMC_OK;
}

// single: stay on the caller's stream even when the tuning asks for two
// (the side stream and its events are created on first use)
template <typename T>
static int forward_t(const qmc_plan_s* P, const T* A, int64_t t, int64_t lda, T* X, int64_t ldx,
                     void* ws, hipStream_t st, const Epi<T>& epi, bool single) {
  if (dense_front(P)) return forward_dense_t<T>(P, A, t, lda, X, ldx, ws, st, epi);
  const int64_t pairs = (t + 1) / 2;
  const size_t el = sizeof(cx<T>);
  cx<T>* aT = (cx<T>*)ws;
  cx<T>* Cbase = (cx<T>*)((char*)ws + align256(pairs * P->Upad * el));
  dim3 gT((unsigned)((P->Upad + 63) / 64), (unsigned)((pairs + 15) / 16));
  {
    ProfScope ps(P, PROF_COLLAPSE, st);
    k_collapse_T<T><<<gT, 256, 0, st>>>(A, lda, t, pairs, P->d_it_ptr, P->d_it_jl, P->Upad, aT);
  }
  int rc = hip_ok(hipGetLastError());
  if (rc != QMC_OK) return rc;
  const int64_t chunk = (P->tune.chunk_pairs > 0 && P->tune.chunk_pairs < pairs)
                            ? P->tune.chunk_pairs : pairs;
  const bool two = !single && P->tune.streams == 2 && chunk < pairs;
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
    const Epi<T> ec = chunk_epi(epi, p0);
    rc = launch_middle<T, true>(P, aT + p0 * P->Upad, np, C, P->sub ? nullptr : X + 2 * p0,
                                t - 2 * p0, PROF_MIDDLE, st);
    if (rc != QMC_OK) return rc;
    rc = launch_split<T, +1>(P, C, np, PROF_SPLIT, st);
    if (rc != QMC_OK) return rc;
    if (two) {
      if ((rc = hip_ok(hipEventRecord(P->ev[slot], st))) != QMC_OK) return rc;
      if ((rc = hip_ok(hipStreamWaitEvent(sb, P->ev[slot], 0))) != QMC_OK) return rc;
    }
    rc = back_dispatch<T>(P, C, np, X + 2 * p0, ldx, t - 2 * p0, sb, ec);
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

template <typename T>
static int forward_epi_t(const qmc_plan_s* P, const T* A, int64_t t, int64_t lda, T* X,
                         int64_t ldx, void* ws, hipStream_t st, const Epi<T>& epi, bool single) {
  int rc = forward_t<T>(P, A, t, lda, X, ldx, ws, st, epi, single);
  if (rc != QMC_OK || epi.kind == 0 || epi.kind == EPI_ACC) return rc;
  // row 0 is the fused pass's DC term, in X on the same stream by now
  k_epi_row0<T><<<(unsigned)((t + 255) / 256), 256, 0, st>>>(X, t, epi);
  return hip_ok(hipGetLastError());
}

int launch_forward(const qmc_plan_s* P, const void* A, int64_t t, int64_t lda, void* X,
                   int64_t ldx, void* ws, hipStream_t st, int epi_kind, const void* bias,
                   const void* scale, bool single_stream) {
  if (P->comp) return composite_forward(P, A, t, lda, X, ldx, ws, st, epi_kind, bias, scale);
  if (P->dtype == QMC_F32)
    return forward_epi_t<float>(P, (const float*)A, t, lda, (float*)X, ldx, ws, st,
                                Epi<float>{epi_kind, (const float*)bias, (const float*)scale},
                                single_stream);
  return forward_epi_t<double>(P, (const double*)A, t, lda, (double*)X, ldx, ws, st,
                               Epi<double>{epi_kind, (const double*)bias, (const double*)scale},
                               single_stream);
}

// dense outer front into B[pair][w2][e1]: the adjoint's gather of G
// (A == nullptr) or the forward's collapse of A, then the outer split
template <typename T>
static int launch_outer_front(const qmc_plan_s* P, const T* A, const T* G, int64_t ld,
                              int64_t t, int64_t pairs, cx<T>* B, hipStream_t st) {
  const Layout& lay = P->lay;
  dim3 grid((unsigned)((lay.M1 + 15) / 16), (unsigned)((pairs + 15) / 16), (unsigned)lay.Pf);
  const cx<T>* twb = (const cx<T>*)P->d_twb;
  const bool fwd = A != nullptr;
  {
    ProfScope ps(P, fwd ? PROF_DFRONT : PROF_ADJ_FRONT, st);
#define QMC_OFRONT(QQ)                                                                         \
  if (fwd)                                                                                     \
    k_fwd_front<T, QQ><<<grid, 256, 0, st>>>(A, ld, t, lay.M1, lay.M2, lay.Pf, P->L, pairs,   \
                                             P->d_inv_ptr, P->d_inv_j, twb, B);               \
  else                                                                                         \
    k_adj_front<T, QQ><<<grid, 256, 0, st>>>(G, ld, t, lay.M1, lay.M2, lay.Pf, P->L, pairs,   \
                                             out_rows(P), twb, B)
    switch (lay.Qf) {
      case 1: QMC_OFRONT(1); break;
      case 2: QMC_OFRONT(2); break;
      case 4: QMC_OFRONT(4); break;
      case 8: QMC_OFRONT(8); break;
      case 16: QMC_OFRONT(16); break;
      case 32: QMC_OFRONT(32); break;
      case 64: QMC_OFRONT(64); break;
      case 3: QMC_OFRONT(3); break;
      case 6: QMC_OFRONT(6); break;
      case 12: QMC_OFRONT(12); break;
      case 24: QMC_OFRONT(24); break;
      case 48: QMC_OFRONT(48); break;
      case 5: QMC_OFRONT(5); break;
      case 10: QMC_OFRONT(10); break;
      case 20: QMC_OFRONT(20); break;
      case 40: QMC_OFRONT(40); break;
      default: return QMC_ERR_UNSUPPORTED;
    }
#undef QMC_OFRONT
  }
  int rc = hip_ok(hipGetLastError());
  if (rc != QMC_OK) return rc;
  return launch_split<T, -1>(P, B, pairs, fwd ? PROF_DFRONT_SPLIT : PROF_ADJ_SPLIT, st);
}

// dA = Y^T G: gather and transform G into B, the fused pass into C, the
// outer split and the read-back at the exponents l_j, per chunk of column
// pairs (chunks too small to fill the GPU, under about 128 pairs at M1 =
// 4096, run slower than one chunk).
template <typename T>
static int adjoint_t(const qmc_plan_s* P, const T* G, int64_t t, int64_t ldg, T* dA,
                     int64_t ldda, void* ws, hipStream_t st, bool acc) {
  const Epi<T> epi{acc ? EPI_ACC : 0, nullptr, nullptr};
  const int64_t pairs = (t + 1) / 2;
  const int64_t chunk = adj_chunk(P, pairs);
  cx<T>* B = (cx<T>*)ws;
  cx<T>* C = (cx<T>*)((char*)ws + align256(chunk * P->lay.M * sizeof(cx<T>)));
  for (int64_t p0 = 0; p0 < pairs; p0 += chunk) {
    const int64_t np = std::min(chunk, pairs - p0), tc = t - 2 * p0;
    int rc = launch_outer_front<T>(P, nullptr, G + 2 * p0, ldg, tc, np, B, st);
    if (rc != QMC_OK) return rc;
    rc = launch_middle<T, false>(P, B, np, C, nullptr, tc, PROF_ADJ_MIDDLE, st);
    if (rc != QMC_OK) return rc;
    rc = launch_split<T, +1>(P, C, np, PROF_SPLIT, st);
    if (rc != QMC_OK) return rc;
    rc = launch_back<T, true>(P, C, np, P->d_inv_ptr, P->d_inv_j, G + 2 * p0, dA + 2 * p0, ldda,
                              tc, st, epi);
    if (rc != QMC_OK) return rc;
  }
  return QMC_OK;
}

int launch_adjoint(const qmc_plan_s* P, const void* G, int64_t t, int64_t ldg, void* dA,
                   int64_t ldda, void* ws, hipStream_t st, bool acc) {
  if (P->comp) return composite_adjoint(P, G, t, ldg, dA, ldda, ws, st);
  if (P->dtype == QMC_F32)
    return adjoint_t<float>(P, (const float*)G, t, ldg, (float*)dA, ldda, ws, st, acc);
  return adjoint_t<double>(P, (const double*)G, t, ldg, (double*)dA, ldda, ws, st, acc);
}

}  // namespace qmc

namespace qmc {
// ---------------------------------------------------------------------------
// sums of blocks (lattice rules with non-prime N)
// ---------------------------------------------------------------------------
template <typename T, int R, bool SPARSE>
static void launch_middle_sum_r(const qmc_plan_s* P0, const MidTerms<T>& terms, int64_t pairs,
                                cx<T>* C, int slot, hipStream_t st) {
  const Layout& lay = P0->lay;
  typedef MidShape<R> S;
  const int64_t G = ((pairs + S::TPB - 1) / S::TPB) * lay.M2;
  ProfScope ps(P0, slot, st);
  const int ntc = nt_inter(P0, pairs * lay.M * (int64_t)sizeof(cx<T>)) ? 1 : 0;
  k_middle_sum<T, R, SPARSE><<<dim3((unsigned)G), dim3(S::BLOCK), 0, st>>>(
      terms, (const cx<T>*)P0->d_twf1, (const cx<T>*)P0->d_twf2, (const cx<T>*)P0->d_twi3,
      (const cx<T>*)P0->d_two, lay.M2, pairs, C, ntc);
}

// src[k]: term k's input (SPARSE: its aT; dense: its B) for these pairs
template <typename T, bool SPARSE>
static int launch_middle_sum(const qmc_plan_s* const* blk, int n, cx<T>* const* src,
                             int64_t pairs, cx<T>* C, int slot, hipStream_t st) {
  MidTerms<T> terms{};
  terms.n = n;
  for (int k = 0; k < n; ++k)
    terms.t[k] = {src[k], blk[k]->d_it_e1, (const cx<T>*)blk[k]->d_twit,
                  (const cx<T>*)blk[k]->d_Hs, blk[k]->Upad, blk[k]->rounds};
  switch (blk[0]->lay.R) {
    case 1: launch_middle_sum_r<T, 1, SPARSE>(blk[0], terms, pairs, C, slot, st); break;
    case 2: launch_middle_sum_r<T, 2, SPARSE>(blk[0], terms, pairs, C, slot, st); break;
    case 4: launch_middle_sum_r<T, 4, SPARSE>(blk[0], terms, pairs, C, slot, st); break;
    case 8: launch_middle_sum_r<T, 8, SPARSE>(blk[0], terms, pairs, C, slot, st); break;
    case 16: launch_middle_sum_r<T, 16, SPARSE>(blk[0], terms, pairs, C, slot, st); break;
    default: return QMC_ERR_UNSUPPORTED;
  }
  return hip_ok(hipGetLastError());
}

static bool sum_ok(const qmc_plan_s* const* blk, int n) {
  if (n < 1 || n > MID_MAX_TERMS) return false;
  for (int k = 1; k < n; ++k) {
    const Layout &a = blk[0]->lay, &b = blk[k]->lay;
    if (a.M != b.M || a.M2 != b.M2 || a.R != b.R || blk[k]->dtype != blk[0]->dtype) return false;
  }
  return true;
}

static int64_t sum_chunk(const qmc_plan_s* P0, int64_t pairs) {
  return (P0->tune.chunk_pairs > 0 && P0->tune.chunk_pairs < pairs) ? P0->tune.chunk_pairs
                                                                     : pairs;
}

size_t collapse_bytes(const qmc_plan_s* B, int64_t t) {
  const size_t el = (B->dtype == QMC_F32) ? sizeof(cx<float>) : sizeof(cx<double>);
  return align256(((t + 1) / 2) * B->Upad * el);
}

size_t sum_workspace_bytes(const qmc_plan_s* const* blk, int n, int64_t t, bool adjoint,
                           bool collapsed) {
  const size_t el = (blk[0]->dtype == QMC_F32) ? sizeof(cx<float>) : sizeof(cx<double>);
  const int64_t pairs = (t + 1) / 2, chunk = sum_chunk(blk[0], pairs);
  const size_t slab = align256(chunk * blk[0]->lay.M * el);  // one B or C of a chunk
  if (adjoint || dense_front(blk[0])) return (size_t)(n + 1) * slab;
  size_t w = slab;
  if (!collapsed)
    for (int k = 0; k < n; ++k) w += collapse_bytes(blk[k], t);
  return w;
}

int launch_collapse(const qmc_plan_s* B, const void* A, int64_t t, int64_t lda, void* aT,
                    hipStream_t st) {
  const int64_t pairs = (t + 1) / 2;
  dim3 gT((unsigned)((B->Upad + 63) / 64), (unsigned)((pairs + 15) / 16));
  ProfScope ps(B, PROF_COLLAPSE, st);
  if (B->dtype == QMC_F32)
    k_collapse_T<float><<<gT, 256, 0, st>>>((const float*)A, lda, t, pairs, B->d_it_ptr,
                                            B->d_it_jl, B->Upad, (cx<float>*)aT);
  else
    k_collapse_T<double><<<gT, 256, 0, st>>>((const double*)A, lda, t, pairs, B->d_it_ptr,
                                             B->d_it_jl, B->Upad, (cx<double>*)aT);
  return hip_ok(hipGetLastError());
}

// X rows of the blocks' common row coset = sum_k Y_k A: every term's
// collapse (sparse fronts) or outer front (dense), one fused pass that sums
// the spectral products, the split and one back pass that writes the rows
// collapsed[k] (sparse fronts only, may be null): term k's collapse of A,
// made by the caller (blocks of several row cosets share it)
template <typename T>
static int forward_sum_t(const qmc_plan_s* const* blk, int n, const T* A, int64_t t, int64_t lda,
                         T* X, int64_t ldx, void* ws, hipStream_t st,
                         void* const* collapsed) {
  const qmc_plan_s* P0 = blk[0];
  const int64_t pairs = (t + 1) / 2, chunk = sum_chunk(P0, pairs);
  const size_t el = sizeof(cx<T>);
  const size_t slab = align256(chunk * P0->lay.M * el);
  const bool dense = dense_front(P0);
  if (dense) collapsed = nullptr;
  cx<T>* in[MID_MAX_TERMS];
  char* p = (char*)ws;
  for (int k = 0; k < n; ++k) {
    if (collapsed) {
      in[k] = (cx<T>*)collapsed[k];
    } else {
      in[k] = (cx<T>*)p;
      p += dense ? slab : align256(pairs * blk[k]->Upad * el);
    }
  }
  cx<T>* C = (cx<T>*)p;
  int rc = QMC_OK;
  if (!dense && !collapsed)
    for (int k = 0; k < n && rc == QMC_OK; ++k) rc = launch_collapse(blk[k], A, t, lda, in[k], st);
  for (int64_t p0 = 0; p0 < pairs && rc == QMC_OK; p0 += chunk) {
    const int64_t np = std::min(chunk, pairs - p0), tc = t - 2 * p0;
    cx<T>* src[MID_MAX_TERMS];
    for (int k = 0; k < n && rc == QMC_OK; ++k) {
      if (dense) {
        rc = launch_outer_front<T>(blk[k], A + 2 * p0, nullptr, lda, tc, np, in[k], st);
        src[k] = in[k];
      } else {
        src[k] = in[k] + p0 * blk[k]->Upad;
      }
    }
    if (rc == QMC_OK)
      rc = dense ? launch_middle_sum<T, false>(blk, n, src, np, C, PROF_MIDDLE, st)
                 : launch_middle_sum<T, true>(blk, n, src, np, C, PROF_MIDDLE, st);
    if (rc == QMC_OK) rc = launch_split<T, +1>(P0, C, np, PROF_SPLIT, st);
    if (rc == QMC_OK) rc = back_dispatch<T>(P0, C, np, X + 2 * p0, ldx, tc, st, Epi<T>());
  }
  return rc;
}

// the adjoint of an orbit's blocks blk[r * ncol + c] (row coset r, column
// coset c), per chunk of column pairs: the outer front of G on every row
// coset once, then per column coset the sum over its row cosets' products
template <typename T>
static int adjoint_grid_t(const qmc_plan_s* const* blk, int nrow, int ncol, const T* G,
                          int64_t t, int64_t ldg, T* dA, int64_t ldda, void* ws,
                          hipStream_t st) {
  const qmc_plan_s* P0 = blk[0];
  const int64_t pairs = (t + 1) / 2, chunk = sum_chunk(P0, pairs);
  const size_t slab = align256(chunk * P0->lay.M * sizeof(cx<T>));
  cx<T>* Br[MID_MAX_TERMS];
  for (int r = 0; r < nrow; ++r) Br[r] = (cx<T>*)((char*)ws + r * slab);
  cx<T>* C = (cx<T>*)((char*)ws + nrow * slab);
  const Epi<T> acc{EPI_ACC, nullptr, nullptr};
  int rc = QMC_OK;
  for (int64_t p0 = 0; p0 < pairs && rc == QMC_OK; p0 += chunk) {
    const int64_t np = std::min(chunk, pairs - p0), tc = t - 2 * p0;
    for (int r = 0; r < nrow && rc == QMC_OK; ++r)
      rc = launch_outer_front<T>(blk[r * ncol], nullptr, G + 2 * p0, ldg, tc, np, Br[r], st);
    for (int c = 0; c < ncol && rc == QMC_OK; ++c) {
      const qmc_plan_s* terms[MID_MAX_TERMS];
      for (int r = 0; r < nrow; ++r) terms[r] = blk[r * ncol + c];
      rc = launch_middle_sum<T, false>(terms, nrow, Br, np, C, PROF_ADJ_MIDDLE, st);
      if (rc == QMC_OK) rc = launch_split<T, +1>(terms[0], C, np, PROF_SPLIT, st);
      if (rc == QMC_OK)
        rc = launch_back<T, true>(terms[0], C, np, terms[0]->d_inv_ptr, terms[0]->d_inv_j,
                                  G + 2 * p0, dA + 2 * p0, ldda, tc, st, acc);
    }
  }
  return rc;
}

int launch_adjoint_grid(const qmc_plan_s* const* blk, int nrow, int ncol, const void* G,
                        int64_t t, int64_t ldg, void* dA, int64_t ldda, void* ws,
                        hipStream_t st) {
  if (nrow < 1 || ncol < 1 || nrow > MID_MAX_TERMS) return QMC_ERR_UNSUPPORTED;
  for (int i = 1; i < nrow * ncol; ++i) {  // one layout for all
    const qmc_plan_s* two[2] = {blk[0], blk[i]};
    if (!sum_ok(two, 2)) return QMC_ERR_UNSUPPORTED;
  }
  if (blk[0]->dtype == QMC_F32)
    return adjoint_grid_t<float>(blk, nrow, ncol, (const float*)G, t, ldg, (float*)dA, ldda, ws,
                                 st);
  return adjoint_grid_t<double>(blk, nrow, ncol, (const double*)G, t, ldg, (double*)dA, ldda,
                                ws, st);
}

int launch_forward_sum(const qmc_plan_s* const* blk, int n, const void* A, int64_t t,
                       int64_t lda, void* X, int64_t ldx, void* ws, hipStream_t st,
                       void* const* collapsed) {
  if (!sum_ok(blk, n)) return QMC_ERR_UNSUPPORTED;
  if (blk[0]->dtype == QMC_F32)
    return forward_sum_t<float>(blk, n, (const float*)A, t, lda, (float*)X, ldx, ws, st,
                                collapsed);
  return forward_sum_t<double>(blk, n, (const double*)A, t, lda, (double*)X, ldx, ws, st,
                               collapsed);
}

}  // namespace qmc
