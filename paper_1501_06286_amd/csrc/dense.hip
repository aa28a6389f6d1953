// The standard approach the fast method is measured against (the paper's
// experiments, Section 4): build the N x s point matrix Y explicitly and
// multiply X = Y A on the MFMA matrix cores.
#include "cx.hpp"
#include "internal.hpp"

namespace qmc {

__device__ __forceinline__ uint64_t gf2_mulmod_d(uint64_t a, uint64_t b, uint64_t p, int m) {
  uint64_t r = 0;
  for (int i = 0; i < m; ++i) {
    if ((b >> i) & 1) r ^= a;
    a <<= 1;
    if ((a >> m) & 1) a ^= p;
  }
  return r;
}

// Y[n][j] = T_phi[n g_j mod N]  (lattice)  or  T_phi[n(x) q_j(x) mod p(x)]  (GF(2))
template <typename T>
__global__ void k_explicit_points(T* __restrict__ Y, int64_t ldy, int64_t N, int64_t s,
                                  const uint32_t* __restrict__ gen,
                                  const double* __restrict__ tphi, int rule, uint64_t p, int m) {
  const int64_t total = N * s;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = i / s, j = i % s;
    uint64_t r;
    if (rule == QMC_RULE_LATTICE)
      r = (uint64_t)n * gen[j] % (uint64_t)N;
    else
      r = gf2_mulmod_d((uint64_t)n, gen[j], p, m);
    Y[n * ldy + j] = (T)tphi[r];
  }
}

int launch_explicit_points(const qmc_plan_s* P, void* Y, int64_t ldy, hipStream_t st) {
  const int64_t total = P->N * P->s;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (P->dtype == QMC_F32)
    k_explicit_points<float><<<(unsigned)blocks, 256, 0, st>>>(
        (float*)Y, ldy, P->N, P->s, P->d_gen, P->d_tphi, P->rule, P->modulus, P->m);
  else
    k_explicit_points<double><<<(unsigned)blocks, 256, 0, st>>>(
        (double*)Y, ldy, P->N, P->s, P->d_gen, P->d_tphi, P->rule, P->modulus, P->m);
  return hip_ok(hipGetLastError());
}

// ---------------------------------------------------------------------------
// MFMA GEMM  X (M x Nc) = Y (M x K) A (K x Nc), row-major, FP32 or FP64.
// 128 x 128 block tile, 4 wavefronts of 64 x 64, v_mfma 16x16x4 (FP32 or
// FP64); K-tiles of BK (32 FP32, 16 FP64) staged through LDS, the next tile
// prefetched into registers with 16-byte loads while the current one is
// multiplied.  Operand layout of the 16x16x4 MFMA: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it receives D[4 (l / 16) + r][l % 16]
// in FP32 and D[l / 16 + 4 r][l % 16] in FP64 (r = 0..3).
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};

// 16 bytes of T
template <typename T>
struct alignas(16) Vec16 {
  static constexpr int N = 16 / sizeof(T);
  T v[N];
};

template <typename T>
__global__ __launch_bounds__(256) void k_gemm(int64_t M, int64_t K, int64_t Nc,
                                              const T* __restrict__ Y, int64_t ldy,
                                              const T* __restrict__ A, int64_t lda,
                                              T* __restrict__ X, int64_t ldx, int vec_ok) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int BM = 128, BN = 128, VEC = Vec16<T>::N, BK = 8 * VEC, PAD = 4;
  // per thread per K-tile: NA vectors of the Y tile, NB of the A tile
  constexpr int NA = BM * BK / VEC / 256, NB = BK * BN / VEC / 256;
  __shared__ alignas(16) T As[BK][BM + PAD];  // transposed: As[k][i]
  __shared__ alignas(16) T Bs[BK][BN + PAD];    // rows of 16-byte multiples
  const int64_t bn0 = (int64_t)blockIdx.x * BN, bm0 = (int64_t)blockIdx.y * BM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  v4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4{0, 0, 0, 0};

  // vector c of the Y tile: row (tid + 256 c) / 8, k = VEC ((tid + 256 c) % 8)
  // vector c of the A tile: k-row (tid + 256 c) / (BN / VEC), cols VEC (... % (BN / VEC))
  Vec16<T> ra[NA], rb[NB];
  // interior K-tiles of an interior block tile: 16-byte loads only
  const bool inner = vec_ok && bm0 + BM <= M && bn0 + BN <= Nc;
  auto load_vec = [&](int64_t k0) {
#pragma unroll
    for (int c = 0; c < NA; ++c) {
      const int v = tid + 256 * c;
      ra[c] = *reinterpret_cast<const Vec16<T>*>(Y + (bm0 + v / 8) * ldy + k0 + VEC * (v % 8));
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int v = tid + 256 * c;
      rb[c] = *reinterpret_cast<const Vec16<T>*>(A + (k0 + v / (BN / VEC)) * lda + bn0 +
                                                 VEC * (v % (BN / VEC)));
    }
  };
  auto load_any = [&](int64_t k0) {  // element loads with bounds checks
#pragma unroll
    for (int c = 0; c < NA; ++c) {
      const int v = tid + 256 * c;
      const int64_t gi = bm0 + v / 8, gk = k0 + VEC * (v % 8);
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        ra[c].v[e] = (gi < M && gk + e < K) ? Y[gi * ldy + gk + e] : (T)0;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int v = tid + 256 * c;
      const int64_t gk = k0 + v / (BN / VEC), gj = bn0 + VEC * (v % (BN / VEC));
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        rb[c].v[e] = (gk < K && gj + e < Nc) ? A[gk * lda + gj + e] : (T)0;
    }
  };
  auto load = [&](int64_t k0) {
    if (inner && k0 + BK <= K)
      load_vec(k0);
    else
      load_any(k0);
  };
  load(0);
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NA; ++c) {
      const int v = tid + 256 * c;
#pragma unroll
      for (int e = 0; e < VEC; ++e) As[VEC * (v % 8) + e][v / 8] = ra[c].v[e];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int v = tid + 256 * c;
      *reinterpret_cast<Vec16<T>*>(&Bs[v / (BN / VEC)][VEC * (v % (BN / VEC))]) = rb[c];
    }
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[kk + lk][wm * 64 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[kk + lk][wn * 64 + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::op(af[i], bf[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = bm0 + wm * 64 + i * 16 + Mfma<T>::row(lk, r);
        const int64_t gj = bn0 + wn * 64 + j * 16 + li;
        if (gi < M && gj < Nc) X[gi * ldx + gj] = acc[i][j][r];
      }
}

int launch_dense_gemm(int dtype, int64_t M, int64_t K, int64_t Nc, const void* Y, int64_t ldy,
                      const void* A, int64_t lda, void* X, int64_t ldx, hipStream_t st) {
  const int64_t gx = (Nc + 127) / 128, gy = (M + 127) / 128;
  if (gy > 65535 || gx > 65535) return QMC_ERR_UNSUPPORTED;
  dim3 grid((unsigned)gx, (unsigned)gy);
  // 16-byte loads need 16-byte aligned rows of Y and A
  const size_t w = dtype == QMC_F32 ? 4 : 8;
  const int vec_ok = ((uintptr_t)Y % 16 == 0) && ((uintptr_t)A % 16 == 0) &&
                     ((ldy * w) % 16 == 0) && ((lda * w) % 16 == 0);
  if (dtype == QMC_F32)
    k_gemm<float><<<grid, 256, 0, st>>>(M, K, Nc, (const float*)Y, ldy, (const float*)A, lda,
                                        (float*)X, ldx, vec_ok);
  else
    k_gemm<double><<<grid, 256, 0, st>>>(M, K, Nc, (const double*)Y, ldy, (const double*)A, lda,
                                         (double*)X, ldx, vec_ok);
  return hip_ok(hipGetLastError());
}

}  // namespace qmc
