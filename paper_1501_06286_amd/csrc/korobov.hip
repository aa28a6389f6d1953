// X = Y A for the union of all Korobov lattice point sets (Section 2.2).
//
// The K - 1 blocks are rank-1 lattice products of K points that share one
// spectrum: block b (Korobov base b) differs from the others only in its
// collapse, through the exponents l_{b,j} = j log_beta(b) mod (K - 1).  A run
// covers a chunk of blocks with one launch per pass -- collapse-transpose,
// fused middle (sparse front, no constant row since the union has no point
// n = 0), outer split where needed, back -- indexing the block from the
// workgroup id, so every block's tables sit at a fixed stride.
#include <algorithm>
#include <new>

#include "kernels.hpp"

namespace qmc {

template <typename T>
__global__ __launch_bounds__(256) void ku_collapse(const T* __restrict__ A, int64_t lda, int64_t t,
                                                   int64_t P, int64_t s,
                                                   const int32_t* __restrict__ it_ptr,
                                                   const int32_t* __restrict__ it_jl,
                                                   int64_t Upad, cx<T>* __restrict__ aT,
                                                   int64_t gx, int64_t per_block,
                                                   int64_t total) {
  // a grid of a fixed number of workgroups striding over the tiles of all
  // blocks (the tiles are small: one workgroup per tile would be bound by
  // the workgroup dispatch rate)
  __shared__ CollapseSmem<T> S;
  for (int64_t id = blockIdx.x; id < total; id += gridDim.x) {
    const int64_t b = id / per_block, lb = id % per_block;
    collapse_body<T>(A, lda, t, P, it_ptr + b * (Upad + 1), it_jl + b * s, Upad,
                     aT + b * P * Upad, lb % gx, lb / gx, S, threadIdx.x);
    __syncthreads();  // S is reused by the next tile
  }
}

template <typename T, int R>
__global__ __launch_bounds__(MidShape<R>::BLOCK)
__attribute__((amdgpu_waves_per_eu(mid_waves<T, R>()))) void ku_middle(
    const cx<T>* __restrict__ aT, int64_t Upad, int64_t rounds, const uint16_t* __restrict__ it_e1,
    const cx<T>* __restrict__ twit, const cx<T>* __restrict__ twf1,
    const cx<T>* __restrict__ twf2, const cx<T>* __restrict__ Hs,
    const cx<T>* __restrict__ twi3, const cx<T>* __restrict__ two, int64_t M1, int64_t M2,
    int64_t P, cx<T>* __restrict__ C, int64_t per_block, int nt_c) {
  __shared__ MidSmem<T, R> S;
  const int64_t id = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t b = id / per_block, lb = id % per_block;
  middle_body<T, R, true>(aT + b * P * Upad, Upad, rounds, it_e1 + b * Upad,
                          twit + b * M2 * Upad, twf1, twf2, Hs, twi3, two, M2, P,
                          C + b * P * M1 * M2, (T*)nullptr, 0, (T)0, lb, S, threadIdx.x,
                          nt_c != 0);
}

template <typename T, int P2, int DIR>
__global__ __launch_bounds__(64) void ku_split(cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                               int Q2, const cx<T>* __restrict__ twb,
                                               int64_t gx, int64_t pairs_total) {
  // blockIdx.x = (bx, q) and blockIdx.y + gridDim.y * blockIdx.z = pair of the run
  const int64_t pair = (int64_t)blockIdx.y + (int64_t)gridDim.y * blockIdx.z;
  if (pair >= pairs_total) return;
  split_body<T, P2, DIR>(C, M1, M2, Q2, twb, blockIdx.x % gx, blockIdx.x / gx, pair, threadIdx.x);
}

// the adjoint: gather G of block b in reflected group order (rows pow[e] - 1
// of the block) and transform the outer index (the dense outer front)
template <typename T, int Q>
__global__ __launch_bounds__(256) void ku_adj_front(const T* __restrict__ G, int64_t ldg,
                                                    int64_t t, int64_t M1, int64_t M2, int64_t Pf,
                                                    int64_t L, int64_t P,
                                                    const int32_t* __restrict__ rowmap,
                                                    const cx<T>* __restrict__ twb,
                                                    cx<T>* __restrict__ B, int64_t block_rows,
                                                    int64_t gx, int64_t gy, int64_t per_block) {
  __shared__ BackSmem<T> S;
  const int64_t b = blockIdx.x / per_block, lb = blockIdx.x % per_block;
  const int64_t bx = lb % gx, rest = lb / gx;
  const T* Gb = G + b * block_rows * ldg;
  const AdjGather<T> g{{Gb, ldg, t, pairs_aligned(Gb, ldg)}, rowmap, L};
  outer_front_body<T, Q>(g, M1, M2, Pf, L, P, twb, B + b * P * M1 * M2, bx, rest % gy,
                         rest / gy, S, threadIdx.x);
}

// the adjoint's fused pass from the dense front's B of every block
template <typename T, int R>
__global__ __launch_bounds__(MidShape<R>::BLOCK)
__attribute__((amdgpu_waves_per_eu(mid_waves<T, R>()))) void ku_middle_dense(
    const cx<T>* __restrict__ B, const cx<T>* __restrict__ twf1,
    const cx<T>* __restrict__ twf2, const cx<T>* __restrict__ Hs,
    const cx<T>* __restrict__ twi3, const cx<T>* __restrict__ two, int64_t M1, int64_t M2,
    int64_t P, cx<T>* __restrict__ C, int64_t per_block, int nt_c) {
  __shared__ MidSmem<T, R> S;
  const int64_t id = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t b = id / per_block, lb = id % per_block;
  middle_body<T, R, false>(B + b * P * M1 * M2, 0, 0, nullptr, nullptr, twf1, twf2, Hs, twi3,
                           two, M2, P, C + b * P * M1 * M2, (T*)nullptr, 0, (T)0, lb, S,
                           threadIdx.x, nt_c != 0);
}

// the adjoint's read-back of block b: Part[b][j][:] = w_b[l_{b,j}] (the
// union has no point 0, so no constant-row term)
template <typename T, int Q>
__global__ __launch_bounds__(256) void ku_back_adj(const cx<T>* __restrict__ C, int64_t M1,
                                                   int64_t M2, int64_t P2, int64_t L, int64_t P,
                                                   const int32_t* __restrict__ inv_ptr,
                                                   const int32_t* __restrict__ inv_j, int64_t s,
                                                   T* __restrict__ Part, int64_t t, int64_t gx,
                                                   int64_t gy, int64_t per_block) {
  __shared__ BackSmem<T> S;
  const int64_t b = blockIdx.x / per_block, lb = blockIdx.x % per_block;
  const int64_t bx = lb % gx, rest = lb / gx;
  back_body<T, Q, true, false>(C + b * P * M1 * M2, M1, M2, P2, L, P, nullptr,
                               inv_ptr + b * (L + 1), inv_j + b * s, nullptr, (T)0,
                               Part + b * s * t, t, t, bx, rest % gy, rest / gy, S, threadIdx.x);
}

// dA[j][k] = (dA[j][k] if accumulate) + sum over the run's blocks b, in
// increasing b, of Part[b][j][k]
template <typename T>
__global__ __launch_bounds__(256) void ku_reduce(const T* __restrict__ Part, int64_t nb,
                                                 int64_t s, int64_t t, T* __restrict__ dA,
                                                 int64_t ldda, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= s * t) return;
  const int64_t j = i / t, k = i % t;
  T acc = accumulate ? dA[j * ldda + k] : (T)0;
  // the parts go out 16 at a time and are added in increasing b
  const T* p = Part + j * t + k;
  const int64_t stride = s * t;
  constexpr int B = 16;
  int64_t b = 0;
  for (; b + B <= nb; b += B) {
    T v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = p[(b + u) * stride];
#pragma unroll
    for (int u = 0; u < B; ++u) acc += v[u];
  }
  for (; b < nb; ++b) acc += p[b * stride];
  dA[j * ldda + k] = acc;
}

template <typename T, int Q>
__global__ __launch_bounds__(256) void ku_back(const cx<T>* __restrict__ C, int64_t M1, int64_t M2,
                                               int64_t P2, int64_t L, int64_t P,
                                               const int32_t* __restrict__ rowmap,
                                               T* __restrict__ X, int64_t ldx, int64_t t,
                                               int64_t block_rows, int64_t gx, int64_t gy,
                                               int64_t per_block, Epi<T> epi) {
  __shared__ BackSmem<T> S;
  const int64_t b = blockIdx.x / per_block, lb = blockIdx.x % per_block;
  const int64_t bx = lb % gx, rest = lb / gx;
  back_body<T, Q, false, false, true>(C + b * P * M1 * M2, M1, M2, P2, L, P, rowmap, nullptr,
                                      nullptr, nullptr, (T)0, X + b * block_rows * ldx, ldx, t,
                                      bx, rest % gy, rest / gy, S, threadIdx.x, epi);
}

template <typename T, int Q>
__global__ __launch_bounds__(256) void ku_back_lds(const cx<T>* __restrict__ C, int64_t M1,
                                                   int64_t M2, int64_t P2, int64_t L, int64_t P,
                                                   const cx<T>* __restrict__ twb,
                                                   const int32_t* __restrict__ rowmap,
                                                   T* __restrict__ X, int64_t ldx, int64_t t,
                                                   int64_t block_rows, int64_t gx, int64_t gy,
                                                   int64_t per_block, Epi<T> epi) {
  __shared__ BackLdsSmem<T, Q> S;
  const int64_t b = blockIdx.x / per_block, lb = blockIdx.x % per_block;
  const int64_t bx = lb % gx, rest = lb / gx;
  back_lds_body<T, Q, false, false, true>(C + b * P * M1 * M2, M1, M2, P2, L, P, twb, rowmap,
                                          nullptr, nullptr, nullptr, (T)0,
                                          X + b * block_rows * ldx, ldx, t, bx, rest % gy,
                                          rest / gy, S, threadIdx.x, epi);
}

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

static int64_t chunk_of(const qmc_korobov_s* U) {
  return (U->chunk_blocks > 0 && U->chunk_blocks < U->blocks) ? U->chunk_blocks : U->blocks;
}

// forward: aT and C of one run; adjoint: B, C and the blocks' partial dA
static size_t korobov_ws(const qmc_korobov_s* U, int64_t t) {
  const qmc_plan_s* P = U->base;
  const size_t el = P->dtype == QMC_F32 ? sizeof(cx<float>) : sizeof(cx<double>);
  const int64_t pairs = (t + 1) / 2, nb = chunk_of(U);
  const size_t fwd = al256(nb * pairs * U->Upad * el) + al256(nb * pairs * P->lay.M * el);
  const size_t adj = 2 * al256(nb * pairs * P->lay.M * el) + al256(nb * U->s * t * el / 2);
  return std::max(fwd, adj);
}

// the outer split over every column pair of a run (DIR = +1: the back
// pass's split P2 x Q2; -1: the dense front's Pf x Qf); none when it is 1
template <typename T, int DIR>
static int ku_split_launch(const qmc_plan_s* P, cx<T>* C, int64_t tot, hipStream_t st) {
  const Layout& lay = P->lay;
  const int p2 = DIR > 0 ? lay.P2 : lay.Pf, q2 = DIR > 0 ? lay.Q2 : lay.Qf;
  if (p2 == 1) return QMC_OK;
  const int64_t gx = (lay.M1 + 63) / 64;
  const int64_t gy = std::min<int64_t>(tot, 65535), gz = (tot + gy - 1) / gy;
  dim3 grid((unsigned)(gx * q2), (unsigned)gy, (unsigned)gz);
  const cx<T>* twb = (const cx<T>*)P->d_twb;
  ProfScope ps(P, DIR > 0 ? PROF_SPLIT : PROF_ADJ_SPLIT, st);
#define QMC_KSPLIT(PP) \
  ku_split<T, PP, DIR><<<grid, 64, 0, st>>>(C, lay.M1, lay.M2, q2, twb, gx, tot)
  switch (p2) {
    case 2: QMC_KSPLIT(2); break;
    case 4: QMC_KSPLIT(4); break;
    case 8: QMC_KSPLIT(8); break;
    case 16: QMC_KSPLIT(16); break;
    case 32: QMC_KSPLIT(32); break;
    case 64: QMC_KSPLIT(64); break;
    default: return QMC_ERR_UNSUPPORTED;
  }
#undef QMC_KSPLIT
  return hip_ok(hipGetLastError());
}

template <typename T, int R>
static void ku_middle_launch(const qmc_korobov_s* U, const cx<T>* aT, int64_t b0, int64_t nb,
                             int64_t pairs, cx<T>* C, hipStream_t st) {
  const qmc_plan_s* P = U->base;
  const Layout& lay = P->lay;
  typedef MidShape<R> S;
  const int64_t per_block = ((pairs + S::TPB - 1) / S::TPB) * lay.M2;
  ProfScope ps(P, PROF_MIDDLE, st);
  ku_middle<T, R><<<dim3((unsigned)(nb * per_block)), dim3(S::BLOCK), 0, st>>>(
      aT, U->Upad, U->rounds, U->d_it_e1 + b0 * U->Upad,
      (const cx<T>*)U->d_twit + b0 * lay.M2 * U->Upad, (const cx<T>*)P->d_twf1,
      (const cx<T>*)P->d_twf2, (const cx<T>*)P->d_Hs, (const cx<T>*)P->d_twi3,
      (const cx<T>*)P->d_two, lay.M1, lay.M2, pairs, C, per_block,
      // streaming stores when a run's intermediate cannot stay in the 256 MB
      // Infinity Cache until the back pass reads it
      nb * pairs * lay.M * (int64_t)sizeof(cx<T>) > ((int64_t)128 << 20) ? 1 : 0);
}

template <typename T>
static int korobov_forward(const qmc_korobov_s* U, const T* A, int64_t t, int64_t lda, T* X,
                           int64_t ldx, void* ws, hipStream_t st, const Epi<T>& epi) {
  const qmc_plan_s* P = U->base;
  const Layout& lay = P->lay;
  const int64_t pairs = (t + 1) / 2, chunk = chunk_of(U), K = U->K;
  const size_t el = sizeof(cx<T>);
  cx<T>* aT = (cx<T>*)ws;
  cx<T>* C = (cx<T>*)((char*)ws + al256(chunk * pairs * U->Upad * el));
  for (int64_t b0 = 0; b0 < U->blocks; b0 += chunk) {
    const int64_t nb = std::min(chunk, U->blocks - b0);
    {
      const int64_t gx = (U->Upad + 63) / 64, per_block = gx * ((pairs + 15) / 16);
      ProfScope ps(P, PROF_COLLAPSE, st);
      const int64_t total = nb * per_block;
      // 8192 workgroups, more than fit on the GPU at once: a tile is a chain
      // of dependent small loads, and a full machine keeps more chains in
      // flight (2048 workgroups: 2.5% slower at K = 1021)
      ku_collapse<T><<<dim3((unsigned)std::min<int64_t>(total, 8192)), 256, 0, st>>>(
          A, lda, t, pairs, U->s, U->d_it_ptr + b0 * (U->Upad + 1), U->d_it_jl + b0 * U->s,
          U->Upad, aT, gx, per_block, total);
    }
    switch (lay.R) {
      case 1: ku_middle_launch<T, 1>(U, aT, b0, nb, pairs, C, st); break;
      case 2: ku_middle_launch<T, 2>(U, aT, b0, nb, pairs, C, st); break;
      case 4: ku_middle_launch<T, 4>(U, aT, b0, nb, pairs, C, st); break;
      case 8: ku_middle_launch<T, 8>(U, aT, b0, nb, pairs, C, st); break;
      case 16: ku_middle_launch<T, 16>(U, aT, b0, nb, pairs, C, st); break;
      default: return QMC_ERR_UNSUPPORTED;
    }
    if (int rc = ku_split_launch<T, +1>(P, C, nb * pairs, st); rc != QMC_OK) return rc;
    {
      // back tile (LDS or register outer DFT; FP64 takes Q2 = 32 through LDS,
      // as the single product)
      const bool lds = lay.Q2 >= 64 || (sizeof(T) == 8 && lay.Q2 == 32);
      const int64_t tb = lds ? 8 : 16;
      const int64_t gx = (lay.M1 + tb - 1) / tb, gy = (pairs + tb - 1) / tb;
      const int64_t per_block = gx * gy * lay.P2;
      T* Xb = X + b0 * (K - 1) * ldx;
      ProfScope ps(P, PROF_BACK, st);
#define QMC_KBACK(QQ)                                                                             \
  ku_back<T, QQ><<<dim3((unsigned)(nb * per_block)), 256, 0, st>>>(                               \
      C, lay.M1, lay.M2, lay.P2, P->L, pairs, U->d_rowmap, Xb, ldx, t, K - 1, gx, gy, per_block, \
      epi)
#define QMC_KBACKL(QQ)                                                                            \
  ku_back_lds<T, QQ><<<dim3((unsigned)(nb * per_block)), 256, 0, st>>>(                           \
      C, lay.M1, lay.M2, lay.P2, P->L, pairs, (const cx<T>*)P->d_twb, U->d_rowmap, Xb, ldx, t,    \
      K - 1, gx, gy, per_block, epi)
      switch (lay.Q2) {
        case 1: QMC_KBACK(1); break;
        case 2: QMC_KBACK(2); break;
        case 4: QMC_KBACK(4); break;
        case 8: QMC_KBACK(8); break;
        case 16: QMC_KBACK(16); break;
        case 32:
          if constexpr (sizeof(T) == 8) {
            QMC_KBACKL(32);
          } else {
            QMC_KBACK(32);
          }
          break;
        case 64: QMC_KBACKL(64); break;
        case 128:
          if constexpr (sizeof(T) == 4) {
            QMC_KBACKL(128);
            break;
          }
          return QMC_ERR_UNSUPPORTED;
        default: return QMC_ERR_UNSUPPORTED;
      }
#undef QMC_KBACKL
#undef QMC_KBACK
    }
    const int rc = hip_ok(hipGetLastError());
    if (rc != QMC_OK) return rc;
  }
  return QMC_OK;
}

// dA = Y^T G = sum over the blocks b of Y_b^T G_b (G_b: the K - 1 rows of
// block b).  Per run of blocks: the dense outer front of each block's G,
// the fused pass, the outer split, the read-back of w_b at the exponents
// l_{b,j} into per-block partial sums, then their sum in increasing b added
// to dA (runs in increasing b as well, so the order is fixed).
template <typename T>
static int korobov_adjoint(const qmc_korobov_s* U, const T* G, int64_t t, int64_t ldg, T* dA,
                           int64_t ldda, void* ws, hipStream_t st) {
  const qmc_plan_s* P = U->base;
  const Layout& lay = P->lay;
  if (lay.Q2 > 32) return QMC_ERR_UNSUPPORTED;  // register back pass only
  const int64_t pairs = (t + 1) / 2, chunk = chunk_of(U), K = U->K, L = P->L, s = U->s;
  const size_t el = sizeof(cx<T>);
  cx<T>* B = (cx<T>*)ws;
  cx<T>* C = (cx<T>*)((char*)ws + al256(chunk * pairs * lay.M * el));
  T* Part = (T*)((char*)C + al256(chunk * pairs * lay.M * el));
  const cx<T>* twb = (const cx<T>*)P->d_twb;
  for (int64_t b0 = 0; b0 < U->blocks; b0 += chunk) {
    const int64_t nb = std::min(chunk, U->blocks - b0);
    const int64_t gx = (lay.M1 + 15) / 16, gy = (pairs + 15) / 16;
    {
      const int64_t per_block = gx * gy * lay.Pf;
      ProfScope ps(P, PROF_ADJ_FRONT, st);
#define QMC_KAF(QQ)                                                                             \
  ku_adj_front<T, QQ><<<dim3((unsigned)(nb * per_block)), 256, 0, st>>>(                        \
      G + b0 * (K - 1) * ldg, ldg, t, lay.M1, lay.M2, lay.Pf, L, pairs, U->d_rowmap, twb, B,     \
      K - 1, gx, gy, per_block)
      switch (lay.Qf) {
        case 1: QMC_KAF(1); break;
        case 2: QMC_KAF(2); break;
        case 4: QMC_KAF(4); break;
        case 8: QMC_KAF(8); break;
        case 16: QMC_KAF(16); break;
        case 32: QMC_KAF(32); break;
        case 64: QMC_KAF(64); break;
        default: return QMC_ERR_UNSUPPORTED;
      }
#undef QMC_KAF
    }
    if (int rc = ku_split_launch<T, -1>(P, B, nb * pairs, st); rc != QMC_OK) return rc;
    {
      ProfScope ps(P, PROF_ADJ_MIDDLE, st);
      const int nt_c = 2 * nb * pairs * lay.M * (int64_t)el > ((int64_t)128 << 20) ? 1 : 0;
#define QMC_KMD(RR)                                                                             \
  {                                                                                             \
    typedef MidShape<RR> S;                                                                     \
    const int64_t per_block = ((pairs + S::TPB - 1) / S::TPB) * lay.M2;                         \
    ku_middle_dense<T, RR><<<dim3((unsigned)(nb * per_block)), dim3(S::BLOCK), 0, st>>>(        \
        B, (const cx<T>*)P->d_twf1, (const cx<T>*)P->d_twf2, (const cx<T>*)P->d_Hs,            \
        (const cx<T>*)P->d_twi3, (const cx<T>*)P->d_two, lay.M1, lay.M2, pairs, C, per_block,   \
        nt_c);                                                                                  \
  }
      switch (lay.R) {
        case 1: QMC_KMD(1); break;
        case 2: QMC_KMD(2); break;
        case 4: QMC_KMD(4); break;
        case 8: QMC_KMD(8); break;
        case 16: QMC_KMD(16); break;
        default: return QMC_ERR_UNSUPPORTED;
      }
#undef QMC_KMD
    }
    if (int rc = ku_split_launch<T, +1>(P, C, nb * pairs, st); rc != QMC_OK) return rc;
    {
      const int64_t per_block = gx * gy * lay.P2;
      ProfScope ps(P, PROF_ADJ_BACK, st);
#define QMC_KBA(QQ)                                                                             \
  ku_back_adj<T, QQ><<<dim3((unsigned)(nb * per_block)), 256, 0, st>>>(                         \
      C, lay.M1, lay.M2, lay.P2, L, pairs, U->d_inv_ptr + b0 * (L + 1), U->d_inv_j + b0 * s, s,  \
      Part, t, gx, gy, per_block)
      switch (lay.Q2) {
        case 1: QMC_KBA(1); break;
        case 2: QMC_KBA(2); break;
        case 4: QMC_KBA(4); break;
        case 8: QMC_KBA(8); break;
        case 16: QMC_KBA(16); break;
        case 32: QMC_KBA(32); break;
        default: return QMC_ERR_UNSUPPORTED;
      }
#undef QMC_KBA
    }
    ku_reduce<T><<<(unsigned)((s * t + 255) / 256), 256, 0, st>>>(Part, nb, s, t, dA, ldda,
                                                                  b0 > 0 ? 1 : 0);
    const int rc = hip_ok(hipGetLastError());
    if (rc != QMC_OK) return rc;
  }
  return QMC_OK;
}

}  // namespace qmc

using namespace qmc;

extern "C" {

int qmc_korobov_create(qmc_korobov_t* out, int64_t K, int64_t s, int phi_kind,
                       int64_t shift_num, int64_t shift_den, int dtype, void* stream) {
  if (!out || K < 3 || s < 1 || K >= ((int64_t)1 << 31) || s > ((int64_t)1 << 30))
    return QMC_ERR_ARG;
  *out = nullptr;
  // Section 2.2: the union is built on the cyclic group Z_K^*, K prime
  if (!is_prime_u64((uint64_t)K)) return QMC_ERR_NOT_PRIME;
  std::vector<uint64_t> ones(s, 1);  // the base plan's own generating vector (block b = 1)
  qmc_plan_s* base = nullptr;
  // the union's kernels take power-of-two outer lengths only
  int rc = plan_create(&base, QMC_RULE_LATTICE, K, s, ones.data(), 0, phi_kind, shift_num,
                       shift_den, dtype, false, false, (hipStream_t)stream);
  if (rc != QMC_OK) return rc;
  qmc_korobov_s* U = new (std::nothrow) qmc_korobov_s();
  if (!U) {
    qmc_plan_destroy(base);
    return QMC_ERR_OOM;
  }
  U->base = base;
  U->K = K;
  U->s = s;
  U->blocks = K - 1;
  rc = build_korobov_tables(U, (hipStream_t)stream);
  if (rc != QMC_OK) {
    qmc_korobov_destroy(U);
    return rc;
  }
  *out = U;
  return QMC_OK;
}

void qmc_korobov_destroy(qmc_korobov_t U) {
  if (!U) return;
  qmc_plan_destroy(U->base);  // owns the union's device tables too
  delete U;
}

int qmc_korobov_info(qmc_korobov_t U, qmc_korobov_info_t* info) {
  if (!U || !info) return QMC_ERR_ARG;
  const qmc_plan_s* P = U->base;
  info->K = U->K;
  info->s = U->s;
  info->N = (U->K - 1) * (U->K - 1);
  info->L = P->L;
  info->M = P->lay.M;
  info->M1 = P->lay.M1;
  info->M2 = P->lay.M2;
  info->blocks = U->blocks;
  info->rounds = U->rounds;
  info->beta = P->beta;
  info->phi_kind = P->phi_kind;
  info->dtype = P->dtype;
  info->chunk_blocks = U->chunk_blocks;
  return QMC_OK;
}

int qmc_korobov_set_chunk(qmc_korobov_t U, int64_t chunk_blocks) {
  if (!U || chunk_blocks < 0) return QMC_ERR_ARG;
  U->chunk_blocks = chunk_blocks;
  return QMC_OK;
}

int qmc_korobov_workspace_size(qmc_korobov_t U, int64_t t, size_t* bytes) {
  if (!U || !bytes || t < 1) return QMC_ERR_ARG;
  *bytes = korobov_ws(U, t);
  return QMC_OK;
}

qmc_plan_t qmc_korobov_plan(qmc_korobov_t U) { return U ? U->base : nullptr; }

int qmc_korobov_matmul_epilogue(qmc_korobov_t U, const void* A, int64_t t, int64_t lda,
                                void* X, int64_t ldx, int epi_kind, const void* bias,
                                const void* scale, void* workspace, size_t workspace_bytes,
                                void* stream) {
  if (!U || !A || !X || t < 1 || lda < t || ldx < t) return QMC_ERR_ARG;
  if (epi_kind < QMC_EPI_NONE || epi_kind > QMC_EPI_EXP) return QMC_ERR_ARG;
  const size_t need = korobov_ws(U, t);
  if (!workspace || workspace_bytes < need) return QMC_ERR_WORKSPACE;
  const int dt = U->base->dtype;
  const int64_t N = (U->K - 1) * (U->K - 1);
  const size_t xa = matrix_extent(N, t, ldx, dt), aa = matrix_extent(U->s, t, lda, dt);
  const size_t va = matrix_extent(1, t, t, dt);
  if (ranges_overlap(X, xa, A, aa) || ranges_overlap(X, xa, workspace, need) ||
      ranges_overlap(A, aa, workspace, need) || (bias && ranges_overlap(X, xa, bias, va)) ||
      (scale && ranges_overlap(X, xa, scale, va)) ||
      (bias && ranges_overlap(workspace, need, bias, va)) ||
      (scale && ranges_overlap(workspace, need, scale, va)))
    return QMC_ERR_ALIAS;
  hipStream_t st = (hipStream_t)stream;
  if (dt == QMC_F32)
    return korobov_forward<float>(
        U, (const float*)A, t, lda, (float*)X, ldx, workspace, st,
        Epi<float>{epi_kind, (const float*)bias, (const float*)scale});
  return korobov_forward<double>(
      U, (const double*)A, t, lda, (double*)X, ldx, workspace, st,
      Epi<double>{epi_kind, (const double*)bias, (const double*)scale});
}

int qmc_korobov_matmul(qmc_korobov_t U, const void* A, int64_t t, int64_t lda, void* X,
                       int64_t ldx, void* workspace, size_t workspace_bytes, void* stream) {
  return qmc_korobov_matmul_epilogue(U, A, t, lda, X, ldx, QMC_EPI_NONE, nullptr, nullptr,
                                     workspace, workspace_bytes, stream);
}

int qmc_korobov_matmul_adjoint(qmc_korobov_t U, const void* G, int64_t t, int64_t ldg, void* dA,
                               int64_t ldda, void* workspace, size_t workspace_bytes,
                               void* stream) {
  if (!U || !G || !dA || t < 1 || ldg < t || ldda < t) return QMC_ERR_ARG;
  const size_t need = korobov_ws(U, t);
  if (!workspace || workspace_bytes < need) return QMC_ERR_WORKSPACE;
  const int dt = U->base->dtype;
  const int64_t N = (U->K - 1) * (U->K - 1);
  const size_t ga = matrix_extent(N, t, ldg, dt), da = matrix_extent(U->s, t, ldda, dt);
  if (ranges_overlap(dA, da, G, ga) || ranges_overlap(dA, da, workspace, need) ||
      ranges_overlap(G, ga, workspace, need))
    return QMC_ERR_ALIAS;
  hipStream_t st = (hipStream_t)stream;
  if (dt == QMC_F32)
    return korobov_adjoint<float>(U, (const float*)G, t, ldg, (float*)dA, ldda, workspace, st);
  return korobov_adjoint<double>(U, (const double*)G, t, ldg, (double*)dA, ldda, workspace, st);
}

}  // extern "C"
