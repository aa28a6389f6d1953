// The C interface declared in include/qmc.h: argument checking, plan
// lifetime and dispatch to the kernels of tables.hip, conv.hip, dense.hip.
#include <new>
#include <string.h>

#include "internal.hpp"

using namespace qmc;

namespace qmc {

bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + bbytes && pb < pa + abytes;
}

size_t matrix_extent(int64_t rows, int64_t cols, int64_t ld, int dtype) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)((rows - 1) * ld + cols) * (dtype == QMC_F32 ? 4 : 8);
}

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int plan_create(qmc_plan_s** out, int rule, int64_t N, int64_t s, const uint64_t* gen,
                uint64_t modulus, int phi_kind, int64_t shift_num, int64_t shift_den, int dtype,
                bool row0_used, bool mixed_outer, hipStream_t stream) {
  if (!out || !gen || s < 1) return QMC_ERR_ARG;
  *out = nullptr;
  if (rule != QMC_RULE_LATTICE && rule != QMC_RULE_POLY_GF2) return QMC_ERR_ARG;
  if (dtype != QMC_F32 && dtype != QMC_F64) return QMC_ERR_ARG;
  if (phi_kind < QMC_PHI_IDENTITY || phi_kind > QMC_PHI_TENT) return QMC_ERR_ARG;
  if (shift_den < 1 || shift_num < 0 || shift_num >= shift_den) return QMC_ERR_ARG;
  if (s > ((int64_t)1 << 30)) return QMC_ERR_ARG;
  int m = 0;
  if (rule == QMC_RULE_LATTICE) {
    if (N < 2 || N >= ((int64_t)1 << 31)) return QMC_ERR_ARG;
    if (modulus != 0) return QMC_ERR_ARG;
  } else {
    if (!is_pow2(N) || N < 2 || N > ((int64_t)1 << 30)) return QMC_ERR_ARG;
    while (((int64_t)1 << m) < N) ++m;
  }
  // the exact coordinate K/D needs D = N * shift_den well inside 63 bits
  if ((__int128)N * shift_den >= ((__int128)1 << 61)) return QMC_ERR_ARG;
  // the inverse normal CDF needs every coordinate strictly inside (0, 1).  The
  // coordinates of a column are {r/N + D} for the residues r = 0..N-1 (the
  // digit numerators Q for GF(2)), and {r/N + D} = 0 exactly when N D is an
  // integer: then the residue r = -N D mod N lands on 0.  That residue is 0
  // itself only for D = 0, whose zero coordinate is the point of row 0 alone,
  // which a point set without row 0 (the union of Korobov rules) never uses.
  if (phi_kind == QMC_PHI_INVNORM && ((__int128)shift_num * N) % shift_den == 0 &&
      (row0_used || shift_num != 0))
    return QMC_ERR_ARG;

  qmc_plan_s* P = new (std::nothrow) qmc_plan_s();
  if (!P) return QMC_ERR_OOM;
  P->rule = rule;
  P->N = N;
  P->s = s;
  P->s_active = s;
  P->L = N - 1;
  P->m = m;
  P->modulus = modulus;
  P->phi_kind = phi_kind;
  P->shift_num = shift_num;
  P->shift_den = shift_den;
  P->dtype = dtype;
  P->mixed_outer = mixed_outer;
  const int rc = build_tables(P, gen, stream);
  if (rc != QMC_OK) {
    qmc_plan_destroy(P);
    return rc;
  }
  *out = P;
  return QMC_OK;
}

}  // namespace qmc

extern "C" {

const char* qmc_strerror(int code) {
  switch (code) {
    case QMC_OK: return "success";
    case QMC_ERR_ARG: return "invalid argument";
    case QMC_ERR_NOT_PRIME: return "this point set needs a prime number of points";
    case QMC_ERR_NOT_PRIMITIVE: return "GF(2) modulus is not a primitive polynomial of degree log2(N)";
    case QMC_ERR_GEN_ZERO: return "generator component is not a unit modulo N";
    case QMC_ERR_ALIAS: return "output overlaps an input or the workspace";
    case QMC_ERR_WORKSPACE: return "workspace missing or too small";
    case QMC_ERR_OOM: return "device allocation failed";
    case QMC_ERR_HIP: return "HIP runtime error";
    case QMC_ERR_UNSUPPORTED: return "request outside what the library supports";
    default: return "unknown error";
  }
}

int qmc_plan_create(qmc_plan_t* out, int rule, int64_t N, int64_t s, const uint64_t* gen,
                    uint64_t modulus, int phi_kind, int64_t shift_num, int64_t shift_den,
                    int dtype, void* stream) {
  return plan_create(out, rule, N, s, gen, modulus, phi_kind, shift_num, shift_den, dtype, true, true,
                     (hipStream_t)stream);
}

static void prof_clear(qmc_plan_t P) {
  for (int k = 0; k < PROF_NSLOTS; ++k) {
    // release paths: a failed release leaves nothing to recover
    for (hipEvent_t e : P->prof[k].start) (void)hipEventDestroy(e);
    for (hipEvent_t e : P->prof[k].stop) (void)hipEventDestroy(e);
    P->prof[k].start.clear();
    P->prof[k].stop.clear();
  }
}

void qmc_plan_destroy(qmc_plan_t plan) {
  if (!plan) return;
  destroy_composite(plan);
  prof_clear(plan);
  if (plan->side) {
    (void)hipStreamSynchronize(plan->side);
    (void)hipStreamDestroy(plan->side);
  }
  for (hipEvent_t e : plan->ev)
    if (e) (void)hipEventDestroy(e);
  for (void* p : plan->owned) (void)hipFree(p);
  delete plan;
}

int qmc_profile_enable(qmc_plan_t P, int on) {
  if (!P) return QMC_ERR_ARG;
  if (P->comp)  // the blocks of a non-prime N record their own launches
    for (qmc_plan_s* B : composite_blocks(P)) qmc_profile_enable(B, on);
  if (!on) prof_clear(P);
  P->prof_on = on != 0;
  return QMC_OK;
}

int qmc_profile_collect(qmc_plan_t P, double* total_ms, int64_t* launches) {
  if (!P || !total_ms || !launches) return QMC_ERR_ARG;
  if (P->comp) {  // summed over the blocks
    for (int k = 0; k < PROF_NSLOTS; ++k) {
      total_ms[k] = 0.0;
      launches[k] = 0;
    }
    int rc = QMC_OK;
    double ms[PROF_NSLOTS];
    int64_t n[PROF_NSLOTS];
    for (qmc_plan_s* B : composite_blocks(P)) {
      const int r = qmc_profile_collect(B, ms, n);
      if (r != QMC_OK) rc = r;
      for (int k = 0; k < PROF_NSLOTS; ++k) {
        total_ms[k] += ms[k];
        launches[k] += n[k];
      }
    }
    return rc;
  }
  int rc = QMC_OK;
  for (int k = 0; k < PROF_NSLOTS; ++k) {
    double sum = 0.0;
    const size_t n = P->prof[k].stop.size();
    for (size_t i = 0; i < n && i < P->prof[k].start.size(); ++i) {
      float ms = 0.f;
      if (hipEventSynchronize(P->prof[k].stop[i]) != hipSuccess ||
          hipEventElapsedTime(&ms, P->prof[k].start[i], P->prof[k].stop[i]) != hipSuccess)
        rc = QMC_ERR_HIP;
      sum += ms;
    }
    total_ms[k] = sum;
    launches[k] = (int64_t)n;
  }
  prof_clear(P);
  return rc;
}

static_assert(PROF_NSLOTS == QMC_PROF_SLOTS, "profiling slots of the header");

const char* qmc_profile_slot_name(int slot) {
  static const char* names[PROF_NSLOTS] = {"collapse_T", "middle",    "outer_split",
                                           "back",       "adj_front", "adj_split",
                                           "adj_middle", "adj_back",  "dense_front",
                                           "dense_front_split"};
  return (slot >= 0 && slot < PROF_NSLOTS) ? names[slot] : "";
}

int qmc_plan_set_tuning(qmc_plan_t P, const qmc_tuning_t* tu) {
  if (!P || !tu) return QMC_ERR_ARG;
  if (tu->chunk_pairs < 0 || (tu->streams != 1 && tu->streams != 2) ||
      (tu->nt_store != 0 && tu->nt_store != 1) || tu->front < 0 || tu->front > 3 ||
      tu->nt_inter < 0 || tu->nt_inter > 2)
    return QMC_ERR_ARG;
  if (P->comp) {
    // every block takes the tuning; an outer radix a block's length cannot
    // split falls back to that block's default
    for (qmc_plan_s* B : composite_blocks(P)) {
      qmc_tuning_t tb = *tu;
      Layout lb = B->lay;
      if (set_outer_split(lb, tb.outer_q, max_outer_q(B->dtype)) != QMC_OK) tb.outer_q = 0;
      const int rc = qmc_plan_set_tuning(B, &tb);
      if (rc != QMC_OK) return rc;
    }
    P->tune = *tu;
    return QMC_OK;
  }
  Layout lay = P->lay;
  const int rc = set_outer_split(lay, tu->outer_q, max_outer_q(P->dtype));
  if (rc != QMC_OK) return rc;
  P->lay = lay;
  P->tune = *tu;
  return QMC_OK;
}

int qmc_plan_set_row_order(qmc_plan_t P, int order) {
  if (!P || (order != QMC_ROWS_CONVENTIONAL && order != QMC_ROWS_GROUP)) return QMC_ERR_ARG;
  // non-prime N has no single cyclic group order
  if (P->comp && order == QMC_ROWS_GROUP) return QMC_ERR_UNSUPPORTED;
  if (order == QMC_ROWS_GROUP && !P->d_grp) {
    std::vector<int32_t> rows(P->L);
    for (int64_t e = 0; e < P->L; ++e) rows[e] = (int32_t)(e + 1);
    int err = QMC_OK;
    int32_t* d = dev_alloc<int32_t>(P, P->L, &err);
    if (err != QMC_OK) return err;
    const int rc = hip_ok(hipMemcpy(d, rows.data(), P->L * sizeof(int32_t),
                                    hipMemcpyHostToDevice));
    if (rc != QMC_OK) return rc;
    P->d_grp = d;
  }
  P->row_order = order;
  return QMC_OK;
}

int qmc_plan_get_tuning(qmc_plan_t P, qmc_tuning_t* tu) {
  if (!P || !tu) return QMC_ERR_ARG;
  *tu = P->tune;
  return QMC_OK;
}

int qmc_plan_info(qmc_plan_t P, qmc_plan_info_t* info) {
  if (!P || !info) return QMC_ERR_ARG;
  memset(info, 0, sizeof(*info));
  info->N = P->N;
  info->s = P->s;
  info->L = P->L;
  info->M = P->lay.M;
  info->M1 = P->lay.M1;
  info->M2 = P->lay.M2;
  info->rounds = P->rounds;
  info->beta = P->beta;
  info->rule = P->rule;
  info->phi_kind = P->phi_kind;
  info->dtype = P->dtype;
  info->embedded = P->embedded;
  info->phi0 = P->phi0;
  info->P2 = P->lay.P2;
  info->Q2 = P->lay.Q2;
  info->blocks = P->comp ? (int64_t)composite_blocks(P).size() : 0;
  info->direct_rows = P->comp ? composite_direct_rows(P) : 0;
  return QMC_OK;
}

int qmc_plan_tables(qmc_plan_t P, int32_t* pow_out, int32_t* log_out, int32_t* ell_out,
                    double* phi_out) {
  if (!P) return QMC_ERR_ARG;
  // non-prime N: no single cyclic group, only the value table
  if (P->comp && (pow_out || log_out || ell_out)) return QMC_ERR_UNSUPPORTED;
  if (pow_out && hipMemcpy(pow_out, P->d_pow, P->L * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return QMC_ERR_HIP;
  if (log_out && hipMemcpy(log_out, P->d_log, P->N * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return QMC_ERR_HIP;
  if (ell_out && hipMemcpy(ell_out, P->d_ell, P->s * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return QMC_ERR_HIP;
  if (phi_out && hipMemcpy(phi_out, P->d_tphi, P->N * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return QMC_ERR_HIP;
  return QMC_OK;
}

int qmc_workspace_size(qmc_plan_t P, int64_t t, size_t* bytes) {
  if (!P || !bytes || t < 1) return QMC_ERR_ARG;
  *bytes = workspace_bytes(P, t);
  return QMC_OK;
}

int qmc_matmul(qmc_plan_t P, const void* A, int64_t t, int64_t lda, void* X, int64_t ldx,
               void* workspace, size_t workspace_bytes_, void* stream) {
  if (!P || !A || !X || t < 1 || lda < t || ldx < t) return QMC_ERR_ARG;
  const size_t need = workspace_bytes(P, t);
  if (!workspace || workspace_bytes_ < need) return QMC_ERR_WORKSPACE;
  const size_t xa = matrix_extent(P->N, t, ldx, P->dtype);
  const size_t aa = matrix_extent(P->s, t, lda, P->dtype);
  if (ranges_overlap(X, xa, A, aa) || ranges_overlap(X, xa, workspace, need) ||
      ranges_overlap(A, aa, workspace, need))
    return QMC_ERR_ALIAS;
  return launch_forward(P, A, t, lda, X, ldx, workspace, (hipStream_t)stream);
}

int qmc_matmul_epilogue(qmc_plan_t P, const void* A, int64_t t, int64_t lda, void* X,
                        int64_t ldx, int epi_kind, const void* bias, const void* scale,
                        void* workspace, size_t workspace_bytes_, void* stream) {
  if (!P || !A || !X || t < 1 || lda < t || ldx < t) return QMC_ERR_ARG;
  if (epi_kind < QMC_EPI_NONE || epi_kind > QMC_EPI_EXP) return QMC_ERR_ARG;
  const size_t need = workspace_bytes(P, t);
  if (!workspace || workspace_bytes_ < need) return QMC_ERR_WORKSPACE;
  const size_t xa = matrix_extent(P->N, t, ldx, P->dtype);
  const size_t aa = matrix_extent(P->s, t, lda, P->dtype);
  const size_t va = matrix_extent(1, t, t, P->dtype);
  if (ranges_overlap(X, xa, A, aa) || ranges_overlap(X, xa, workspace, need) ||
      ranges_overlap(A, aa, workspace, need) || (bias && ranges_overlap(X, xa, bias, va)) ||
      (scale && ranges_overlap(X, xa, scale, va)) || (bias && ranges_overlap(workspace, need, bias, va)) ||
      (scale && ranges_overlap(workspace, need, scale, va)))
    return QMC_ERR_ALIAS;
  return launch_forward(P, A, t, lda, X, ldx, workspace, (hipStream_t)stream, epi_kind, bias,
                        scale);
}

int qmc_matmul_adjoint(qmc_plan_t P, const void* G, int64_t t, int64_t ldg, void* dA,
                       int64_t ldda, void* workspace, size_t workspace_bytes_, void* stream) {
  if (!P || !G || !dA || t < 1 || ldg < t || ldda < t) return QMC_ERR_ARG;
  const size_t need = workspace_bytes(P, t);
  if (!workspace || workspace_bytes_ < need) return QMC_ERR_WORKSPACE;
  const size_t ga = matrix_extent(P->N, t, ldg, P->dtype);
  const size_t da = matrix_extent(P->s, t, ldda, P->dtype);
  if (ranges_overlap(dA, da, G, ga) || ranges_overlap(dA, da, workspace, need) ||
      ranges_overlap(G, ga, workspace, need))
    return QMC_ERR_ALIAS;
  return launch_adjoint(P, G, t, ldg, dA, ldda, workspace, (hipStream_t)stream);
}

int qmc_explicit_points(qmc_plan_t P, void* Y, int64_t ldy, void* stream) {
  if (!P || !Y || ldy < P->s) return QMC_ERR_ARG;
  return launch_explicit_points(P, Y, ldy, (hipStream_t)stream);
}

int qmc_dense_matmul(qmc_plan_t P, const void* Y, int64_t ldy, const void* A, int64_t t,
                     int64_t lda, void* X, int64_t ldx, void* stream) {
  if (!P || !Y || !A || !X || t < 1 || ldy < P->s || lda < t || ldx < t) return QMC_ERR_ARG;
  const size_t xa = matrix_extent(P->N, t, ldx, P->dtype);
  if (ranges_overlap(X, xa, Y, matrix_extent(P->N, P->s, ldy, P->dtype)) ||
      ranges_overlap(X, xa, A, matrix_extent(P->s, t, lda, P->dtype)))
    return QMC_ERR_ALIAS;
  return launch_dense_gemm(P->dtype, P->N, P->s, t, Y, ldy, A, lda, X, ldx, (hipStream_t)stream);
}

int qmc_batched_workspace_size(int count, const qmc_plan_t* plans, const int64_t* t,
                               size_t* bytes) {
  if (count < 1 || !plans || !t || !bytes) return QMC_ERR_ARG;
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || t[i] < 1) return QMC_ERR_ARG;
    const size_t el = plans[i]->dtype == QMC_F32 ? 8 : 16;
    const int64_t pairs = (t[i] + 1) / 2;
    total += ((pairs * plans[i]->Upad * el + 255) & ~size_t(255)) +
             ((pairs * plans[i]->lay.M * el + 255) & ~size_t(255));
  }
  *bytes = total;
  return QMC_OK;
}

int qmc_matmul_batched(int count, const qmc_plan_t* plans, const void* const* A, const int64_t* t,
                       void* const* X, void* workspace, size_t workspace_bytes_, void* stream) {
  qmc_batch_t B = nullptr;
  int rc = qmc_batch_create(&B, count, plans, t, A, nullptr, X, nullptr, stream);
  if (rc != QMC_OK) return rc;
  rc = qmc_batch_run(B, workspace, workspace_bytes_, stream);
  if (rc == QMC_OK) rc = hip_ok(hipStreamSynchronize((hipStream_t)stream));
  qmc_batch_destroy(B);
  return rc;
}

}  // extern "C"
