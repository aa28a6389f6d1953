// Internal declarations shared by the translation units of libqmcfast.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "qmc.h"

namespace qmc {

// Decomposition of the circular convolution of length M = M1 * M2
// (M1 = R * R on chip, M2 outer).
struct Layout {
  int64_t M = 1, M1 = 1, M2 = 1;  // M2 = 2^j, or 3 x 2^j or 5 x 2^j (then M1 = 16^3)
  int R = 1;        // M1 = R * R * R, R <= 16
  int P2 = 1;       // outer inverse split M2 = P2 * Q2 (P2 = 1: single back pass; a power of two)
  int Q2 = 1;       // values of w2 per output column of the back pass (up to 32 in registers,
                    // 48 and more through LDS; holds the factor 3 of M2)
  int Pf = 1;       // outer forward split of the dense fronts M2 = Pf * Qf (Qf <= 64)
  int Qf = 1;
};

// per-kernel timing slots (HIP events recorded around each launch when on)
enum ProfSlotId {
  PROF_COLLAPSE = 0, PROF_MIDDLE, PROF_SPLIT, PROF_BACK,
  PROF_ADJ_FRONT, PROF_ADJ_SPLIT, PROF_ADJ_MIDDLE, PROF_ADJ_BACK, PROF_DFRONT, PROF_DFRONT_SPLIT,
  PROF_NSLOTS
};

struct ProfEvents {
  std::vector<hipEvent_t> start, stop;
};

}  // namespace qmc

namespace qmc {
struct CompositePlan;
}

struct qmc_plan_s {
  int rule = 0;
  int64_t N = 0, s = 0, L = 0;
  int64_t s_active = 0;      // rows of A the plan reads (s, or a block's share of them)
  // a lattice rule with non-prime N: its blocks (each one of the plans
  // below, flagged sub) and the rows summed directly
  qmc::CompositePlan* comp = nullptr;
  bool sub = false;          // a block of such a rule: no row 0, group order of L != N - 1
  int m = 0;                 // GF(2): degree
  uint64_t modulus = 0;
  uint64_t beta = 0;
  int phi_kind = 0;
  int64_t shift_num = 0, shift_den = 1;
  int dtype = QMC_F32;
  int embedded = 0;          // 1: L is not a power of two, convolution embedded in M >= 2L-1
  bool mixed_outer = true;   // the embedding may take M = 3 x 2^k or 5 x 2^k
  double phi0 = 0.0;
  qmc::Layout lay;
  int64_t rounds = 0;        // sparse collapse schedule: rounds per front slice
  int64_t Upad = 0;          // rounds * R^2 (slices x round width)

  // device tables (owned)
  int32_t* d_pow = nullptr;     // L   : pow[e] = conventional row of beta^e
  int32_t* d_grp = nullptr;     // L   : 1 + e, the rows of the group order (made on request)
  int row_order = 0;            // 0: conventional rows pow[e]; 1: group order, row 1 + e
  int32_t* d_log = nullptr;     // N   : log[pow[e]] = e, log[0] = -1
  int32_t* d_ell = nullptr;     // s   : l_j
  uint32_t* d_gen = nullptr;    // s   : g_j mod N (lattice) or q_j (GF(2))
  double* d_tphi = nullptr;     // N   : phi of residue r (FP64)
  void* d_Hs = nullptr;         // M   : spectrum / M, [w2] then thread g + R f value h for w1 = f + R g + R^2 h (paired)
  void* d_twf1 = nullptr;       // R*R^2: W_{M1}^{e1' f}, thread e1' (< R^2), value f (paired)
  void* d_twf2 = nullptr;       // R*R : W_{R^2}^{a g}, thread a, value g (paired layout)
  void* d_twi3 = nullptr;       // M   : conj W_M^{e1' (f M2 + w2)}, [w2] then thread a + R f value bb, e1' = a + R bb (paired)
  void* d_two = nullptr;        // M2*R: conj W_M^{R^2 c w2} in [w2][c] order
  void* d_twit = nullptr;       // M2*Upad: W_M^{slot_u w2} in [w2][u] order
  void* d_twb = nullptr;        // M2  : conj W_{M2}^k, the outer split's twiddles at k = a q mod M2
  uint16_t* d_it_e1 = nullptr;  // Upad: e1 of item u (M1 for padding; M1 <= 4096)
  uint16_t* d_it_e2 = nullptr;  // Upad: e2 = slot / M1 of item u (0 for padding; M2 <= 4096)
  int32_t* d_it_ptr = nullptr;  // Upad+1: rows of item u are it_jl[it_ptr[u] .. it_ptr[u+1])
  int32_t* d_it_jl = nullptr;   // s   : rows j grouped by item (increasing j)
  int32_t* d_inv_ptr = nullptr;    // L+1 : rows j with l_j = e are inv_j[inv_ptr[e] .. inv_ptr[e+1])
  int32_t* d_inv_j = nullptr;      // s
  std::vector<void*> owned;
  qmc_tuning_t tune = {0, 1, 0, 0, 0, 0};
  // second stream and events for the two-stream chunk pipeline (created lazily)
  mutable hipStream_t side = nullptr;
  mutable hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // timing instrumentation (off by default)
  mutable bool prof_on = false;
  mutable qmc::ProfEvents prof[qmc::PROF_NSLOTS];
};

// union of all Korobov lattice point sets with a prime K: K - 1 blocks (one
// per Korobov base b) of the rank-1 lattice rule of K points, rows n >= 1
struct qmc_korobov_s {
  qmc_plan_s* base = nullptr;   // lattice plan of N = K: pow, spectrum, twiddles (owns the
                                // memory below); its own collapse schedule is unused
  int64_t K = 0, s = 0, blocks = 0;
  int64_t rounds = 0, Upad = 0;  // common collapse schedule size of every block
  int32_t* d_it_ptr = nullptr;   // blocks*(Upad+1), offsets into the block's s rows
  int32_t* d_it_jl = nullptr;    // blocks*s
  uint16_t* d_it_e1 = nullptr;   // blocks*Upad
  void* d_twit = nullptr;        // blocks*M2*Upad: W_M^{slot w2} per block
  int32_t* d_rowmap = nullptr;   // L: pow[e] - 1 (row n - 1 of a block)
  int32_t* d_inv_ptr = nullptr;  // blocks*(L+1): per block, CSR of the rows j with l_{b,j} = e
  int32_t* d_inv_j = nullptr;    // blocks*s
  int64_t chunk_blocks = 0;      // blocks per run (0: chosen from the shape)
};

namespace qmc {

// tables.hip
int build_tables(qmc_plan_s* P, const uint64_t* gen_host, hipStream_t st);
// schedule, inverse exponent map and spectral tables of a plan whose layout
// is set: ell (host, P->s entries, -1 for rows of A outside the product),
// generator z_k = tphi[zidx[k]] for k < L (device tables)
int build_conv_tables(qmc_plan_s* P, const int32_t* ell, const int32_t* d_zidx,
                      const double* d_tphi, hipStream_t st);
// M = L when L is a power of two, else the shortest power of two >= 2L-1 or
// (mixed) the shortest 3 x 2^k or 5 x 2^k >= 2L-1 when that is shorter and its outer
// length fits one back pass
Layout choose_layout(int64_t L, int dtype, int* embedded, bool mixed);
int launch_phi_table(qmc_plan_s* P, hipStream_t st);
bool is_prime_u64(uint64_t n);
std::vector<uint64_t> prime_factors(uint64_t n);
uint64_t powmod(uint64_t b, uint64_t e, uint64_t n);
uint64_t smallest_primitive_root(uint64_t N);

// composite.hip: lattice rules with non-prime N
int build_composite(qmc_plan_s* P, const uint64_t* gen_host, hipStream_t st);
void destroy_composite(qmc_plan_s* P);
size_t composite_workspace_bytes(const qmc_plan_s* P, int64_t t);
int composite_forward(const qmc_plan_s* P, const void* A, int64_t t, int64_t lda, void* X,
                      int64_t ldx, void* ws, hipStream_t st, int epi_kind, const void* bias,
                      const void* scale);
int composite_adjoint(const qmc_plan_s* P, const void* G, int64_t t, int64_t ldg, void* dA,
                      int64_t ldda, void* ws, hipStream_t st);
// the blocks of a composite plan (for tuning, timing and plan facts)
const std::vector<qmc_plan_s*>& composite_blocks(const qmc_plan_s* P);
int64_t composite_direct_rows(const qmc_plan_s* P);
// split the outer length M2 = P2 Q2 with at most q values per back-pass
// thread (q = 0: the default); QMC_ERR_ARG if q or the split is invalid
int set_outer_split(Layout& lay, int q, int qmax);
// the longest outer factor of the LDS back pass for a dtype (its tile of
// Q x 64 values must fit 64 KB)
inline int max_outer_q(int dtype) { return dtype == QMC_F32 ? 128 : 64; }
int build_korobov_tables(qmc_korobov_s* U, hipStream_t st);

// sparse collapse schedule for exponents l_j (j < s) on a layout: item u is
// one distinct reflected slot it_slot[u] = (L - l_j) mod L (-1: padding)
// with residue it_e1[u] = slot mod M1 (M1 for padding) and the rows
// it_jl[it_ptr[u] .. it_ptr[u+1]) of A that share it
struct Schedule {
  int64_t rounds = 0, Upad = 0;
  std::vector<int32_t> it_slot, it_e1, it_ptr, it_jl;
};
Schedule make_schedule(const Layout& lay, int64_t L, int64_t s, const int32_t* ell);
void pad_schedule(Schedule& sc, int64_t rounds, int64_t M1, int R);

// api.hip
bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes);
size_t matrix_extent(int64_t rows, int64_t cols, int64_t ld, int dtype);
// row0_used = false: the point of row 0 never enters a product (the union of
// Korobov rules), so phi may be unbounded there; mixed_outer = false: the
// convolution length stays a power of two (the union's kernels)
int plan_create(qmc_plan_s** out, int rule, int64_t N, int64_t s, const uint64_t* gen,
                uint64_t modulus, int phi_kind, int64_t shift_num, int64_t shift_den, int dtype,
                bool row0_used, bool mixed_outer, hipStream_t stream);

// conv.hip
bool dense_front(const qmc_plan_s* P);
size_t workspace_bytes(const qmc_plan_s* P, int64_t t);
// epi_kind, bias, scale: the epilogue of qmc_matmul_epilogue (0: none);
// single_stream: every launch on st whatever the tuning's stream count
int launch_forward(const qmc_plan_s* P, const void* A, int64_t t, int64_t lda, void* X,
                   int64_t ldx, void* ws, hipStream_t st, int epi_kind = 0,
                   const void* bias = nullptr, const void* scale = nullptr,
                   bool single_stream = false);
// acc: dA += Y^T G (the blocks of a lattice rule with non-prime N add up)
int launch_adjoint(const qmc_plan_s* P, const void* G, int64_t t, int64_t ldg, void* dA,
                   int64_t ldda, void* ws, hipStream_t st, bool acc = false);
// sums of n <= MID_MAX_TERMS blocks with one layout (the blocks of a lattice
// rule with non-prime N) that share their output rows: X rows written
// (collapsed: the terms' collapses of A when the caller made them, sparse
// fronts only; else null)
int launch_forward_sum(const qmc_plan_s* const* blk, int n, const void* A, int64_t t,
                       int64_t lda, void* X, int64_t ldx, void* ws, hipStream_t st,
                       void* const* collapsed = nullptr);
size_t sum_workspace_bytes(const qmc_plan_s* const* blk, int n, int64_t t, bool adjoint,
                           bool collapsed = false);
// the adjoint of an orbit's blocks blk[r * ncol + c] (row coset r <
// MID_MAX_TERMS, column coset c): G's outer front once per row coset, a sum
// per column coset; workspace (nrow + 1) chunk x M values
int launch_adjoint_grid(const qmc_plan_s* const* blk, int nrow, int ncol, const void* G,
                        int64_t t, int64_t ldg, void* dA, int64_t ldda, void* ws,
                        hipStream_t st);
// the collapse of A on a plan's schedule (pairs x Upad values) and its size
int launch_collapse(const qmc_plan_s* B, const void* A, int64_t t, int64_t lda, void* aT,
                    hipStream_t st);
size_t collapse_bytes(const qmc_plan_s* B, int64_t t);

// dense.hip
int launch_explicit_points(const qmc_plan_s* P, void* Y, int64_t ldy, hipStream_t st);
int launch_dense_gemm(int dtype, int64_t M, int64_t K, int64_t Nc, const void* Y, int64_t ldy,
                      const void* A, int64_t lda, void* X, int64_t ldx, hipStream_t st);

inline int hip_ok(hipError_t e) { return e == hipSuccess ? QMC_OK : QMC_ERR_HIP; }

// records a start event at construction and a stop event at destruction on
// the launch stream when the plan's timing instrumentation is on
struct ProfScope {
  const qmc_plan_s* P;
  int slot;
  hipStream_t st;
  ProfScope(const qmc_plan_s* P_, int slot_, hipStream_t st_) : P(P_), slot(slot_), st(st_) {
    if (!P->prof_on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) {
      hipEventRecord(e, st);
      P->prof[slot].start.push_back(e);
    }
  }
  ~ProfScope() {
    if (!P->prof_on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) {
      hipEventRecord(e, st);
      P->prof[slot].stop.push_back(e);
    }
  }
};

// the row of X (and of G for the adjoint) that holds group element beta^e
inline const int32_t* out_rows(const qmc_plan_s* P) {
  return P->row_order ? P->d_grp : P->d_pow;
}

template <typename T>
T* dev_alloc(qmc_plan_s* P, size_t count, int* err) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
    *err = QMC_ERR_OOM;
    return nullptr;
  }
  P->owned.push_back(p);
  return static_cast<T*>(p);
}

}  // namespace qmc
