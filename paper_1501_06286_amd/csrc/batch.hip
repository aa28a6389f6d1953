// Batched products X_i = Y_i A_i for many plans of uneven size.
//
// A batch binds the plans and their A_i, X_i once and uploads one descriptor
// per product.  A run is one persistent launch per pass over all products
// (collapse-transpose, fused middle, outer split where needed, back); every
// workgroup loops over logical blocks, finds its product by binary search in
// the descriptors' block offsets, and runs the same device bodies as a single
// product.  A run makes no host-to-device copies, so it can be captured in a
// HIP graph and replayed.  Products are grouped by their layout (on-chip size
// R and outer split P2 x Q2), one set of launches per group, so every kernel
// is compiled for one transform size and keeps only the registers it needs.
#include <algorithm>
#include <new>
#include <vector>

#include "kernels.hpp"

namespace qmc {

enum { PASS_COLLAPSE = 0, PASS_MIDDLE = 1, PASS_SPLIT = 2, PASS_BACK = 3, NPASS = 4 };

struct BatchInst {
  const void* A;
  void* X;
  int64_t lda, ldx, t, pairs;
  int64_t aT_off, C_off;  // byte offsets into the run's workspace
  const int32_t* it_ptr;
  const int32_t* it_jl;
  const uint16_t* it_e1;
  const int32_t* pow;
  const void* twit;
  const void* twf1;
  const void* twf2;
  const void* Hs;
  const void* twi3;
  const void* two;
  const void* twb;
  int64_t Upad, rounds, M1, M2, P2, Q2, L;
  int64_t R;  // on-chip radix (M1 = R^3)
  double phi0;
  int64_t off[NPASS];  // first logical block of this product in each pass
  int64_t nb[NPASS];   // logical blocks of this product in each pass
  int64_t gx_collapse, gx_split, gx_back, gy_back;
  // the epilogue of the product's writes (kind 0: none), per column
  int epi_kind;
  const void* epi_bias;
  const void* epi_scale;
};

// the epilogue of row 0 of one product's columns [c0, c0 + nc) (its values
// are the fused pass's DC terms, written by the previous launch); run by the
// back-pass workgroups of the first e1 tile, each for its own column pairs
template <typename T>
__device__ __forceinline__ void batch_row0_epi(const BatchInst& I, int64_t c0, int nc, int tid) {
  if (I.epi_kind == 0 || tid >= nc) return;
  const int64_t c = c0 + tid;
  if (c >= I.t) return;
  const Epi<T> e{I.epi_kind, (const T*)I.epi_bias, (const T*)I.epi_scale};
  const EpiCols<T> ec(e, c, I.t);
  T* x = (T*)I.X + c;
  *x = ec.f0(*x);
}

// largest i with D[i].off[pass] <= b (the product owning logical block b)
__device__ __forceinline__ int find_inst(const BatchInst* __restrict__ D, int n, int pass,
                                         int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (D[mid].off[pass] <= b) lo = mid;
    else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);  // uniform: descriptor loads stay scalar
}

// The persistent workgroups stride through the logical blocks of a pass
// together, so the products' tables are shared in L2 while they run (dealing
// contiguous ranges measured slower); a workgroup searches the descriptors
// only when its next block leaves the product it is in.
struct InstCursor {
  int i = 0;
  int64_t lo = 1, hi = 0;  // logical blocks of product i (empty at the start)
};
__device__ __forceinline__ int inst_at(const BatchInst* __restrict__ D, int n, int pass, int64_t b,
                                       InstCursor& c) {
  if (b < c.lo || b >= c.hi) {
    c.i = find_inst(D, n, pass, b);
    c.lo = D[c.i].off[pass];
    c.hi = c.lo + D[c.i].nb[pass];
  }
  return c.i;
}
#define QMC_FOR_BLOCKS(b, total) \
  for (int64_t b = blockIdx.x; b < (total); b += gridDim.x)

template <typename T>
__global__ __launch_bounds__(256) void kb_collapse(const BatchInst* __restrict__ D, int n,
                                                   int64_t total, char* __restrict__ ws) {
  __shared__ CollapseSmem<T> S;
  InstCursor cur;
  QMC_FOR_BLOCKS(b, total) {
    const BatchInst I = D[inst_at(D, n, PASS_COLLAPSE, b, cur)];
    const int64_t lb = b - I.off[PASS_COLLAPSE];
    collapse_body<T>((const T*)I.A, I.lda, I.t, I.pairs, I.it_ptr, I.it_jl, I.Upad,
                     (cx<T>*)(ws + I.aT_off), lb % I.gx_collapse, lb / I.gx_collapse, S,
                     opaque_tid());
    __syncthreads();
  }
}

template <typename T, int R>
__global__ __launch_bounds__(MidShape<R>::BLOCK)
__attribute__((amdgpu_waves_per_eu(mid_waves<T, R>()))) void kb_middle(const BatchInst* __restrict__ D,
                                                                int n, int64_t total,
                                                                char* __restrict__ ws,
                                                                int nt_c) {
  __shared__ MidSmem<T, R> S;
  InstCursor cur;
  QMC_FOR_BLOCKS(b, total) {
    const BatchInst I = D[inst_at(D, n, PASS_MIDDLE, b, cur)];
    const int64_t lb = b - I.off[PASS_MIDDLE];
    middle_body<T, R, true>((const cx<T>*)(ws + I.aT_off), I.Upad, I.rounds, I.it_e1,
                            (const cx<T>*)I.twit, (const cx<T>*)I.twf1, (const cx<T>*)I.twf2,
                            (const cx<T>*)I.Hs, (const cx<T>*)I.twi3, (const cx<T>*)I.two, I.M2,
                            I.pairs, (cx<T>*)(ws + I.C_off), (T*)I.X, I.t, (T)I.phi0, lb, S,
                            opaque_tid(), nt_c != 0);
    __syncthreads();
  }
}

template <typename T, int P2>
__global__ __launch_bounds__(64) void kb_split(const BatchInst* __restrict__ D, int n,
                                               int64_t total, char* __restrict__ ws) {
  InstCursor cur;
  QMC_FOR_BLOCKS(b, total) {
    const BatchInst I = D[inst_at(D, n, PASS_SPLIT, b, cur)];
    const int64_t lb = b - I.off[PASS_SPLIT];
    const int64_t bx = lb % I.gx_split, rest = lb / I.gx_split;
    const int64_t q = rest % I.Q2, pair = rest / I.Q2;
    split_body<T, P2, +1>((cx<T>*)(ws + I.C_off), I.M1, I.M2, (int)I.Q2,
                          (const cx<T>*)I.twb, bx, q, pair, opaque_tid());
  }
}

// EPI: some product of the run has an epilogue (compiled apart: its per-column
// registers would lower the occupancy of the plain back pass)
template <typename T, int Q, bool EPI>
__global__ __launch_bounds__(256) void kb_back(const BatchInst* __restrict__ D, int n,
                                               int64_t total, char* __restrict__ ws) {
  __shared__ BackSmem<T> S;
  InstCursor cur;
  QMC_FOR_BLOCKS(b, total) {
    const BatchInst I = D[inst_at(D, n, PASS_BACK, b, cur)];
    const int64_t lb = b - I.off[PASS_BACK];
    const int64_t bx = lb % I.gx_back, rest = lb / I.gx_back;
    const int64_t by = rest % I.gy_back, a = rest / I.gy_back;
    const Epi<T> epi{I.epi_kind, (const T*)I.epi_bias, (const T*)I.epi_scale};
    back_body<T, Q, false, false, EPI>((const cx<T>*)(ws + I.C_off), I.M1, I.M2, I.P2, I.L,
                                       I.pairs, I.pow, nullptr, nullptr, nullptr, (T)I.phi0,
                                       (T*)I.X, I.ldx, I.t, bx, by, a, S, opaque_tid(), epi);
    if (EPI && bx == 0 && a == 0) batch_row0_epi<T>(I, 32 * by, 32, opaque_tid());
    __syncthreads();
  }
}

template <typename T, int Q, bool EPI>
__global__ __launch_bounds__((BackLdsShape<Q, back_lds_te<T>(), back_lds_nw<T, Q, false>()>::BLOCK))
void kb_back_lds(const BatchInst* __restrict__ D, int n, int64_t total, char* __restrict__ ws) {
  constexpr int TE = back_lds_te<T>(), NW = back_lds_nw<T, Q, false>();
  __shared__ BackLdsSmem<T, Q, TE> S;
  InstCursor cur;
  QMC_FOR_BLOCKS(b, total) {
    const BatchInst I = D[inst_at(D, n, PASS_BACK, b, cur)];
    const int64_t lb = b - I.off[PASS_BACK];
    const int64_t bx = lb % I.gx_back, rest = lb / I.gx_back;
    const int64_t by = rest % I.gy_back, a = rest / I.gy_back;
    const Epi<T> epi{I.epi_kind, (const T*)I.epi_bias, (const T*)I.epi_scale};
    back_lds_body<T, Q, false, false, EPI, TE, NW>((const cx<T>*)(ws + I.C_off), I.M1, I.M2, I.P2,
                                           I.L, I.pairs, (const cx<T>*)I.twb, I.pow, nullptr,
                                           nullptr, nullptr, (T)I.phi0, (T*)I.X, I.ldx, I.t, bx,
                                           by, a, S, opaque_tid(), epi);
    if (EPI && bx == 0 && a == 0) batch_row0_epi<T>(I, 16 * by, 16, opaque_tid());
    __syncthreads();
  }
}

}  // namespace qmc

using namespace qmc;

struct qmc_batch_s {
  int dtype = QMC_F32;
  size_t ws_bytes = 0;
  int64_t chunk_bytes = 0;
  int nt_inter = 0;  // stores of the intermediates: 0 auto, 1 cached, 2 streaming
  bool ready = false;  // the runs are built (a failed regrouping leaves none)
  // one launch of a run: one pass over the run's products that share the
  // pass's template parameter (collapse: all; fused pass: R; split: P2 > 1;
  // back pass: Q2), with their descriptors
  struct Group {
    int pass = 0;
    int key = 0;   // R, P2 or Q2 of the launch's products
    int nt_c = 0;  // streaming stores of the run's intermediate (too large for the cache)
    int epi = 0;   // some product of the launch has an epilogue
    int n = 0;
    BatchInst* d_desc = nullptr;
    int64_t total = 0;  // logical blocks of the pass
  };
  std::vector<Group> groups;  // every run's launches, runs in order
  // the products by layout key (R, P2, Q2), in input order, for regrouping,
  // and each one's position in the caller's list
  std::vector<std::pair<int64_t, std::vector<BatchInst>>> byKey;
  std::vector<std::vector<int>> input_index;
  // every device range the runs read or write (A_i, X_i, epilogue vectors),
  // checked against the workspace at each run
  std::vector<std::pair<const void*, size_t>> operands;
  std::vector<std::pair<const void*, size_t>> epi_operands;
};

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

static void free_runs(qmc_batch_s* B) {
  for (auto& g : B->groups)
    if (g.d_desc) (void)hipFree(g.d_desc);
  B->groups.clear();
}

// Cuts the products (ordered by layout key (R, P2, Q2), input order within a
// key) into runs of consecutive products whose intermediate spectra C
// together take at most `chunk` bytes (0: one run of all; a product larger
// than `chunk` runs alone), so that C can stay in the 256 MB Infinity Cache
// between the fused pass that writes it and the back pass that reads it.
// A run is one launch of the collapse over all its products, one fused-pass
// launch per on-chip size R, one split launch per split radix P2 > 1 and one
// back-pass launch per outer radix Q2.  The runs execute one after another on
// one stream and share the workspace from offset 0.  Uploads the
// descriptors and synchronises `st`.
static int build_runs(qmc_batch_s* B, int64_t chunk, int nt_inter, hipStream_t st) {
  free_runs(B);
  B->ready = false;
  const size_t el = B->dtype == QMC_F32 ? sizeof(cx<float>) : sizeof(cx<double>);
  std::vector<BatchInst> all;  // byKey is in first-appearance order: sort by key
  {
    std::vector<size_t> order(B->byKey.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::sort(order.begin(), order.end(),
              [&](size_t a, size_t b) { return B->byKey[a].first < B->byKey[b].first; });
    for (size_t k : order) all.insert(all.end(), B->byKey[k].second.begin(), B->byKey[k].second.end());
  }
  // one launch of pass p over the products v[i] with sel(i)
  auto add_launch = [&](std::vector<BatchInst>& v, int p, int key, int nt_c, auto sel) -> int {
    std::vector<BatchInst> d;
    for (size_t i = 0; i < v.size(); ++i)
      if (sel(v[i])) d.push_back(v[i]);
    qmc_batch_s::Group g;
    g.pass = p;
    g.key = key;
    g.nt_c = nt_c;
    int64_t o = 0;
    for (BatchInst& I : d) {
      I.off[p] = o;
      o += I.nb[p];
      g.epi |= I.epi_kind != 0;
    }
    g.total = o;
    g.n = (int)d.size();
    if (o == 0) return QMC_OK;  // nothing to launch (a split pass of no product)
    if (hipMalloc(&g.d_desc, d.size() * sizeof(BatchInst)) != hipSuccess) return QMC_ERR_OOM;
    B->groups.push_back(g);
    int rc = hip_ok(hipMemcpyAsync(g.d_desc, d.data(), d.size() * sizeof(BatchInst),
                                   hipMemcpyHostToDevice, st));
    if (rc == QMC_OK) rc = hip_ok(hipStreamSynchronize(st));  // d is freed next
    return rc;
  };
  size_t ws = 0;
  for (size_t i0 = 0; i0 < all.size();) {
    size_t i1 = i0;
    int64_t cbytes = 0;
    while (i1 < all.size()) {
      const int64_t c = all[i1].pairs * all[i1].M1 * all[i1].M2 * (int64_t)el;
      if (chunk > 0 && i1 > i0 && cbytes + c > chunk) break;
      cbytes += c;
      ++i1;
    }
    std::vector<BatchInst> v(all.begin() + i0, all.begin() + i1);
    i0 = i1;
    size_t off = 0;
    for (BatchInst& I : v) {
      I.aT_off = (int64_t)off;
      off += al256(I.pairs * I.Upad * el);
      I.C_off = (int64_t)off;
      off += al256(I.pairs * I.M1 * I.M2 * el);
    }
    ws = std::max(ws, off);
    // streaming stores of C when it cannot stay in the cache anyway
    const int nt_c = nt_inter ? (nt_inter == 2) : (cbytes > ((int64_t)128 << 20));
    std::vector<int64_t> Rs, P2s, Q2s;
    for (const BatchInst& I : v) {
      const int64_t R = I.R;
      if (std::find(Rs.begin(), Rs.end(), R) == Rs.end()) Rs.push_back(R);
      if (I.P2 > 1 && std::find(P2s.begin(), P2s.end(), I.P2) == P2s.end()) P2s.push_back(I.P2);
      if (std::find(Q2s.begin(), Q2s.end(), I.Q2) == Q2s.end()) Q2s.push_back(I.Q2);
    }
    int rc = add_launch(v, PASS_COLLAPSE, 0, nt_c, [](const BatchInst&) { return true; });
    for (int64_t R : Rs)
      if (rc == QMC_OK)
        rc = add_launch(v, PASS_MIDDLE, (int)R, nt_c, [R](const BatchInst& I) { return I.R == R; });
    for (int64_t P2 : P2s)
      if (rc == QMC_OK)
        rc = add_launch(v, PASS_SPLIT, (int)P2, nt_c,
                        [P2](const BatchInst& I) { return I.P2 == P2; });
    for (int64_t Q2 : Q2s)
      if (rc == QMC_OK)
        rc = add_launch(v, PASS_BACK, (int)Q2, nt_c, [Q2](const BatchInst& I) { return I.Q2 == Q2; });
    if (rc != QMC_OK) {
      free_runs(B);
      return rc;
    }
  }
  B->ws_bytes = ws;
  B->chunk_bytes = chunk;
  B->nt_inter = nt_inter;
  B->ready = true;
  return QMC_OK;
}

extern "C" {

int qmc_batch_create(qmc_batch_t* out, int count, const qmc_plan_t* plans, const int64_t* t,
                     const void* const* A, const int64_t* lda, void* const* X,
                     const int64_t* ldx, void* stream) {
  if (!out || count < 1 || !plans || !t || !A || !X) return QMC_ERR_ARG;
  *out = nullptr;
  const int dtype = plans[0] ? plans[0]->dtype : -1;
  for (int i = 0; i < count; ++i) {
    const qmc_plan_s* P = plans[i];
    if (!P || P->dtype != dtype || t[i] < 1 || !A[i] || !X[i]) return QMC_ERR_ARG;
    if (P->comp) return QMC_ERR_UNSUPPORTED;  // non-prime N: products of several blocks
    const int64_t la = lda ? lda[i] : t[i], lx = ldx ? ldx[i] : t[i];
    if (la < t[i] || lx < t[i]) return QMC_ERR_ARG;
  }
  // every X[i] is written while the A[k] and the other X[k] are read or
  // written: no output may overlap any operand of the batch
  std::vector<std::pair<const void*, size_t>> ops(2 * (size_t)count);
  for (int i = 0; i < count; ++i) {
    ops[2 * i] = {A[i], matrix_extent(plans[i]->s, t[i], lda ? lda[i] : t[i], dtype)};
    ops[2 * i + 1] = {X[i], matrix_extent(plans[i]->N, t[i], ldx ? ldx[i] : t[i], dtype)};
  }
  for (int i = 0; i < count; ++i) {
    const auto& x = ops[2 * i + 1];
    for (size_t k = 0; k < ops.size(); ++k)
      if (k != (size_t)(2 * i + 1) && ranges_overlap(x.first, x.second, ops[k].first, ops[k].second))
        return QMC_ERR_ALIAS;
  }
  qmc_batch_s* B = new (std::nothrow) qmc_batch_s();
  if (!B) return QMC_ERR_OOM;
  B->dtype = dtype;
  B->operands = std::move(ops);
  // products grouped by layout key (R, P2, Q2)
  auto& byKey = B->byKey;
  for (int i = 0; i < count; ++i) {
    const qmc_plan_s* P = plans[i];
    const Layout& lay = P->lay;
    BatchInst I{};
    I.A = A[i];
    I.X = X[i];
    I.lda = lda ? lda[i] : t[i];
    I.ldx = ldx ? ldx[i] : t[i];
    I.t = t[i];
    I.pairs = (t[i] + 1) / 2;
    I.it_ptr = P->d_it_ptr;
    I.it_jl = P->d_it_jl;
    I.it_e1 = P->d_it_e1;
    I.pow = out_rows(P);
    I.twit = P->d_twit;
    I.twf1 = P->d_twf1;
    I.twf2 = P->d_twf2;
    I.Hs = P->d_Hs;
    I.twi3 = P->d_twi3;
    I.two = P->d_two;
    I.twb = P->d_twb;
    I.Upad = P->Upad;
    I.rounds = P->rounds;
    I.M1 = lay.M1;
    I.R = lay.R;
    I.M2 = lay.M2;
    I.P2 = lay.P2;
    I.Q2 = lay.Q2;
    I.L = P->L;
    I.phi0 = P->phi0;
    const int64_t tpb = (int64_t)(lay.R * lay.R >= 64 ? 1 : 64 / (lay.R * lay.R));
    I.gx_collapse = (P->Upad + 63) / 64;
    I.nb[PASS_COLLAPSE] = I.gx_collapse * ((I.pairs + 15) / 16);
    I.nb[PASS_MIDDLE] = ((I.pairs + tpb - 1) / tpb) * lay.M2;
    I.gx_split = (lay.M1 + 63) / 64;
    I.nb[PASS_SPLIT] = lay.P2 > 1 ? I.gx_split * lay.Q2 * I.pairs : 0;
    // back tile: e1 x column pairs (LDS outer DFT: 16 or 8 x 8, register: 16 x 16)
    const bool lds = back_in_lds(lay.Q2, P->dtype == QMC_F64);
    const int64_t te = lds ? (P->dtype == QMC_F32 ? 16 : 8) : 16;
    const int64_t tp = lds ? 8 : 16;
    I.gx_back = (lay.M1 + te - 1) / te;
    I.gy_back = (I.pairs + tp - 1) / tp;
    I.nb[PASS_BACK] = I.gx_back * I.gy_back * lay.P2;
    const int64_t key = ((int64_t)lay.R << 32) | ((int64_t)lay.P2 << 16) | lay.Q2;
    auto it = std::find_if(byKey.begin(), byKey.end(),
                           [&](const std::pair<int64_t, std::vector<BatchInst>>& g) {
                             return g.first == key;
                           });
    if (it == byKey.end()) {
      byKey.push_back({key, {}});
      B->input_index.push_back({});
      it = byKey.end() - 1;
    }
    it->second.push_back(I);
    B->input_index[it - byKey.begin()].push_back(i);
  }
  const int rc = build_runs(B, QMC_BATCH_CHUNK_DEFAULT, 0, (hipStream_t)stream);
  if (rc != QMC_OK) {
    qmc_batch_destroy(B);
    return rc;
  }
  *out = B;
  return QMC_OK;
}

void qmc_batch_destroy(qmc_batch_t B) {
  if (!B) return;
  free_runs(B);
  delete B;
}

int qmc_batch_set_epilogue(qmc_batch_t B, int kind, const void* const* bias,
                           const void* const* scale, void* stream) {
  if (!B || kind < QMC_EPI_NONE || kind > QMC_EPI_EXP) return QMC_ERR_ARG;
  // bias[i], scale[i] belong to the caller's product i (input_index)
  std::vector<std::pair<const void*, size_t>> epi_ops;
  for (size_t g = 0; g < B->byKey.size(); ++g) {
    for (size_t k = 0; k < B->byKey[g].second.size(); ++k) {
      BatchInst& I = B->byKey[g].second[k];
      const int i = B->input_index[g][k];
      const void* b = (kind && bias) ? bias[i] : nullptr;
      const void* c = (kind && scale) ? scale[i] : nullptr;
      const size_t va = matrix_extent(1, I.t, I.t, B->dtype);
      if (b) epi_ops.push_back({b, va});
      if (c) epi_ops.push_back({c, va});
    }
  }
  // no X of the batch may overlap any epilogue vector (checked before any
  // descriptor changes, so a refused call leaves the batch as it was)
  for (size_t k = 1; k < B->operands.size(); k += 2)
    for (const auto& e : epi_ops)
      if (ranges_overlap(B->operands[k].first, B->operands[k].second, e.first, e.second))
        return QMC_ERR_ALIAS;
  for (size_t g = 0; g < B->byKey.size(); ++g) {
    for (size_t k = 0; k < B->byKey[g].second.size(); ++k) {
      BatchInst& I = B->byKey[g].second[k];
      const int i = B->input_index[g][k];
      I.epi_kind = kind;
      I.epi_bias = (kind && bias) ? bias[i] : nullptr;
      I.epi_scale = (kind && scale) ? scale[i] : nullptr;
    }
  }
  B->epi_operands = std::move(epi_ops);
  return build_runs(B, B->chunk_bytes, B->nt_inter, (hipStream_t)stream);
}

int qmc_batch_set_chunk(qmc_batch_t B, int64_t chunk_bytes, int nt_inter, void* stream) {
  if (!B || chunk_bytes < 0 || nt_inter < 0 || nt_inter > 2) return QMC_ERR_ARG;
  return build_runs(B, chunk_bytes, nt_inter, (hipStream_t)stream);
}

int qmc_batch_workspace_size(qmc_batch_t B, size_t* bytes) {
  if (!B || !bytes) return QMC_ERR_ARG;
  *bytes = B->ws_bytes;
  return QMC_OK;
}

}  // extern "C"

namespace qmc {

static inline unsigned grid_for(int64_t total, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min(total, cap));
}

// one launch of a run (persistent grids: a few resident workgroups per CU)
template <typename T>
static int run_launch(const qmc_batch_s::Group& g, char* ws, hipStream_t st) {
  const int64_t tot = g.total;
  switch (g.pass) {
    case PASS_COLLAPSE:
      kb_collapse<T><<<grid_for(tot, 2048), 256, 0, st>>>(g.d_desc, g.n, tot, ws);
      break;
    case PASS_MIDDLE: {
      const unsigned gm = grid_for(tot, 1024);
#define QMC_KBM(RR) \
  kb_middle<T, RR><<<gm, MidShape<RR>::BLOCK, 0, st>>>(g.d_desc, g.n, tot, ws, g.nt_c)
      switch (g.key) {
        case 1: QMC_KBM(1); break;
        case 2: QMC_KBM(2); break;
        case 4: QMC_KBM(4); break;
        case 8: QMC_KBM(8); break;
        case 16: QMC_KBM(16); break;
        default: return QMC_ERR_UNSUPPORTED;
      }
#undef QMC_KBM
      break;
    }
    case PASS_SPLIT: {
      const unsigned gs = grid_for(tot, 4096);
#define QMC_KBS(PP) kb_split<T, PP><<<gs, 64, 0, st>>>(g.d_desc, g.n, tot, ws)
      switch (g.key) {
        case 2: QMC_KBS(2); break;
        case 4: QMC_KBS(4); break;
        case 8: QMC_KBS(8); break;
        case 16: QMC_KBS(16); break;
        case 32: QMC_KBS(32); break;
        case 64: QMC_KBS(64); break;
        default: return QMC_ERR_UNSUPPORTED;
      }
#undef QMC_KBS
      break;
    }
    default: {  // PASS_BACK
      const unsigned gb = grid_for(tot, 1024);
#define QMC_KBB(QQ)                                                                  \
  (g.epi ? kb_back<T, QQ, true><<<gb, 256, 0, st>>>(g.d_desc, g.n, tot, ws)         \
         : kb_back<T, QQ, false><<<gb, 256, 0, st>>>(g.d_desc, g.n, tot, ws))
#define QMC_KBL(QQ)                                                                  \
  (g.epi ? kb_back_lds<T, QQ, true>                                                  \
               <<<gb, BackLdsShape<QQ, back_lds_te<T>(), back_lds_nw<T, QQ, false>()>::BLOCK, 0, \
                  st>>>(g.d_desc, g.n, tot, ws)                                      \
         : kb_back_lds<T, QQ, false>                                                 \
               <<<gb, BackLdsShape<QQ, back_lds_te<T>(), back_lds_nw<T, QQ, false>()>::BLOCK, 0, \
                  st>>>(g.d_desc, g.n, tot, ws))
      switch (g.key) {
        case 1: QMC_KBB(1); break;
        case 2: QMC_KBB(2); break;
        case 4: QMC_KBB(4); break;
        case 8: QMC_KBB(8); break;
        case 16: QMC_KBB(16); break;
        case 3: QMC_KBB(3); break;
        case 6: QMC_KBB(6); break;
        case 12: QMC_KBB(12); break;
        case 24: QMC_KBB(24); break;
        case 5: QMC_KBB(5); break;
        case 10: QMC_KBB(10); break;
        case 20: QMC_KBB(20); break;
        case 40: QMC_KBL(40); break;
        case 48: QMC_KBL(48); break;
        case 80:
          if constexpr (sizeof(T) == 4) {
            QMC_KBL(80);
            break;
          }
          return QMC_ERR_UNSUPPORTED;
        case 96:
          if constexpr (sizeof(T) == 4) {
            QMC_KBL(96);
            break;
          }
          return QMC_ERR_UNSUPPORTED;
        case 32:  // FP64 through LDS, as the single product (the same bits)
          if constexpr (sizeof(T) == 8) {
            QMC_KBL(32);
          } else {
            QMC_KBB(32);
          }
          break;
        case 64: QMC_KBL(64); break;
        case 128:
          if constexpr (sizeof(T) == 4) {
            QMC_KBL(128);
            break;
          }
          return QMC_ERR_UNSUPPORTED;
        default: return QMC_ERR_UNSUPPORTED;
      }
#undef QMC_KBL
#undef QMC_KBB
    }
  }
  return hip_ok(hipGetLastError());
}

}  // namespace qmc

extern "C" {

int qmc_batch_run(qmc_batch_t B, void* workspace, size_t workspace_bytes, void* stream) {
  if (!B || !B->ready) return QMC_ERR_ARG;
  if (!workspace || workspace_bytes < B->ws_bytes) return QMC_ERR_WORKSPACE;
  for (const auto& o : B->operands)
    if (ranges_overlap(workspace, B->ws_bytes, o.first, o.second)) return QMC_ERR_ALIAS;
  for (const auto& o : B->epi_operands)
    if (ranges_overlap(workspace, B->ws_bytes, o.first, o.second)) return QMC_ERR_ALIAS;
  hipStream_t st = (hipStream_t)stream;
  for (const auto& g : B->groups) {
    const int rc = B->dtype == QMC_F32 ? run_launch<float>(g, (char*)workspace, st)
                                       : run_launch<double>(g, (char*)workspace, st);
    if (rc != QMC_OK) return rc;
  }
  return QMC_OK;
}

}  // extern "C"
