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

template <typename T, int P2, int DIR>
__global__ __launch_bounds__(64) void k_outer_split(cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                                    int Q2, const cx<T>* __restrict__ twb) {
  split_body<T, P2, DIR>(C, M1, M2, Q2, twb, blockIdx.x, blockIdx.y, blockIdx.z, threadIdx.x);
}

template <typename T, int Q, bool ADJ, bool NT, bool EPI>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(back_waves<T, Q>()))) void k_back(const cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                              int64_t P2, int64_t L, int64_t P,
                                              const int32_t* __restrict__ rowmap,
                                              const int32_t* __restrict__ inv_ptr,
                                              const int32_t* __restrict__ inv_j,
                                              const T* __restrict__ G0, T phi0,
                                              T* __restrict__ X, int64_t ldx, int64_t t,
                                              Epi<T> epi) {
  __shared__ BackSmem<T> S;
  back_body<T, Q, ADJ, NT, EPI>(C, M1, M2, P2, L, P, rowmap, inv_ptr, inv_j, G0, phi0, X, ldx,
                                t, blockIdx.x, blockIdx.y, blockIdx.z, S, threadIdx.x, epi);
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
  // the outer factor through LDS, tiles of TE e1 x 8 pairs: Q2 = 48, 64, 96
  // and 128, and 32 in FP64 (its register variant takes all 256 registers and
  // spills; in FP32 the register variant is the faster one)
  if (back_in_lds(lay.Q2, sizeof(T) == 8)) {
    constexpr int TE = back_lds_te<T>();
    dim3 gl((unsigned)((lay.M1 + TE - 1) / TE), (unsigned)((pairs + 7) / 8), (unsigned)lay.P2);
#define QMC_BACKL(QQ)                                                                        \
  k_back_lds<T, QQ, ADJ, NT, EPI, TE, back_lds_nw<T, QQ, ADJ>()>                               \
      <<<gl, BackLdsShape<QQ, TE, back_lds_nw<T, QQ, ADJ>()>::BLOCK, 0, st>>>(                \
          C, lay.M1, lay.M2, lay.P2, P->L, pairs, (const cx<T>*)P->d_twb, out_rows(P), inv_ptr, \
          inv_j, G0, (T)P->phi0, X, ldx, t, epi)
    if (lay.Q2 == 48) {
      QMC_BACKL(48);
    } else if (lay.Q2 == 64) {
      QMC_BACKL(64);
    } else if constexpr (sizeof(T) == 4) {
      if (lay.Q2 == 96) {
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
