// Plan construction: the number theory of Section 2.1 (primitive element,
// exponents of the generator components), the bit-exact power / logarithm
// tables, the phi table, the circulant generator and its FP64 spectrum, and
// the twiddle / schedule tables the convolution kernels read.
//
// Host code decides (prime factors of L, the primitive element, the layout
// and the collapse schedule); every table that has one entry per group
// element, residue or frequency is filled by a kernel on the device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "kernels.hpp"

namespace qmc {

// ---------------------------------------------------------------------------
// host number theory
// ---------------------------------------------------------------------------
bool is_prime_u64(uint64_t n) {
  if (n < 2) return false;
  if (n % 2 == 0) return n == 2;
  for (uint64_t f = 3; f * f <= n; f += 2)
    if (n % f == 0) return false;
  return true;
}

std::vector<uint64_t> prime_factors(uint64_t n) {
  std::vector<uint64_t> out;
  for (uint64_t f = 2; f * f <= n; ++f) {
    if (n % f == 0) {
      out.push_back(f);
      while (n % f == 0) n /= f;
    }
  }
  if (n > 1) out.push_back(n);
  return out;
}

uint64_t powmod(uint64_t b, uint64_t e, uint64_t n) {
  uint64_t r = 1 % n;
  b %= n;
  while (e) {
    if (e & 1) r = (unsigned __int128)r * b % n;
    b = (unsigned __int128)b * b % n;
    e >>= 1;
  }
  return r;
}

// smallest primitive root of prime N: beta^(L/q) != 1 for every prime q | L
uint64_t smallest_primitive_root(uint64_t N) {
  if (N == 2) return 1;
  const uint64_t L = N - 1;
  std::vector<uint64_t> qs = prime_factors(L);
  for (uint64_t b = 2; b < N; ++b) {
    bool ok = true;
    for (uint64_t q : qs)
      if (powmod(b, L / q, N) == 1) { ok = false; break; }
    if (ok) return b;
  }
  return 0;
}

static uint64_t gf2_mulmod_host(uint64_t a, uint64_t b, uint64_t p, int m) {
  uint64_t r = 0;
  for (int i = 0; i < m; ++i) {
    if ((b >> i) & 1) r ^= a;
    a <<= 1;
    if ((a >> m) & 1) a ^= p;
  }
  return r;
}
static uint64_t gf2_xpow_host(uint64_t e, uint64_t p, int m) {
  uint64_t r = 1, b = (m == 1) ? 1 : 2;
  while (e) {
    if (e & 1) r = gf2_mulmod_host(r, b, p, m);
    b = gf2_mulmod_host(b, b, p, m);
    e >>= 1;
  }
  return r;
}
// p of degree m is primitive iff x has order exactly 2^m - 1 modulo p
static bool gf2_is_primitive(uint64_t p, int m) {
  if (m < 1 || (p >> m) != 1 || (p & 1) == 0) return false;
  const uint64_t order = (uint64_t(1) << m) - 1;
  if (gf2_xpow_host(order, p, m) != 1) return false;
  for (uint64_t q : prime_factors(order))
    if (gf2_xpow_host(order / q, p, m) == 1) return false;
  return true;
}

// ---------------------------------------------------------------------------
// device kernels: tables
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t gf2_mulmod(uint64_t a, uint64_t b, uint64_t p, int m) {
  uint64_t r = 0;
  for (int i = 0; i < m; ++i) {
    if ((b >> i) & 1) r ^= a;
    a <<= 1;
    if ((a >> m) & 1) a ^= p;
  }
  return r;
}

// pow[e] = beta^e mod N, square-and-multiply on 64-bit integers (N < 2^31)
__global__ void k_pow_lattice(int32_t* pow, int64_t L, uint64_t N, uint64_t beta) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L) return;
  uint64_t r = 1 % N, b = beta % N, x = (uint64_t)e;
  while (x) {
    if (x & 1) r = r * b % N;
    b = b * b % N;
    x >>= 1;
  }
  pow[e] = (int32_t)r;
}

// pow[e] = x^e mod p(x) over GF(2) (as a bitmask), square-and-multiply
__global__ void k_pow_gf2(int32_t* pow, int64_t L, uint64_t p, int m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L) return;
  uint64_t r = 1, b = (m == 1) ? 1 : 2, x = (uint64_t)e;
  while (x) {
    if (x & 1) r = gf2_mulmod(r, b, p, m);
    b = gf2_mulmod(b, b, p, m);
    x >>= 1;
  }
  pow[e] = (int32_t)r;
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// log[pow[e]] = e  (pow is a bijection [0, L) -> [1, N-1])
__global__ void k_log_scatter(const int32_t* pow, int64_t L, int32_t* log) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < L) log[pow[e]] = (int32_t)e;
}

// ell[j] = log[g_j]
__global__ void k_ell(const uint32_t* gen, int64_t s, const int32_t* log, int32_t* ell) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < s) ell[j] = log[gen[j]];
}

// Wichura's algorithm AS241 (PPND16, Applied Statistics 37, 1988) for the
// lower half p <= 1/2 of the inverse standard normal CDF, FP64.
__device__ double invnorm_lower(double p) {
  const double q = p - 0.5;
  if (fabs(q) <= 0.425) {
    const double r = 0.180625 - q * q;
    const double num =
        ((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r +
             6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r +
           1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
         1.3314166789178437745e+2) * r + 3.3871328727963666080e+0;
    const double den =
        ((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r +
             3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r +
           5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
         4.2313330701600911252e+1) * r + 1.0;
    return q * num / den;
  }
  double r = sqrt(-log(p));
  double val;
  if (r <= 5.0) {
    r -= 1.6;
    const double num =
        ((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
             2.41780725177450611770e-1) * r + 1.27045825245236838258e+0) * r +
           3.64784832476320460504e+0) * r + 5.76949722146069140550e+0) * r +
         4.63033784615654529590e+0) * r + 1.42343711074968357734e+0;
    const double den =
        ((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
             1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
           6.89767334985100004550e-1) * r + 1.67638483018380384940e+0) * r +
         2.05319162663775882187e+0) * r + 1.0;
    val = num / den;
  } else {
    r -= 5.0;
    const double num =
        ((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
             1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
           2.96560571828504891230e-1) * r + 1.78482653991729133580e+0) * r +
         5.46378491116411436990e+0) * r + 6.65790464350110377720e+0;
    const double den =
        ((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
             1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
           1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
         5.99832206555887937690e-1) * r + 1.0;
    val = num / den;
  }
  return -val;  // q < 0 on the lower half
}

// phi of the exact coordinate K/D (0 <= K < D), rounded once; the inverse
// normal CDF is taken on the nearer tail so the complement is exact.
__device__ double phi_of(int kind, int64_t K, int64_t D) {
  switch (kind) {
    case QMC_PHI_IDENTITY: return (double)K / (double)D;
    case QMC_PHI_CENTERED: return (double)(2 * K - D) / (double)(2 * D);
    case QMC_PHI_TENT: {
      int64_t a = 2 * K - D;
      if (a < 0) a = -a;
      return (double)(D - a) / (double)D;
    }
    default: {  // QMC_PHI_INVNORM
      if (2 * K > D) return -invnorm_lower((double)(D - K) / (double)D);
      return invnorm_lower((double)K / (double)D);
    }
  }
}

// T_phi[r] = phi({point of residue r} + shift), r in [0, N)
//   lattice: point r/N;  GF(2): nu_m(r(x)/p(x)) = Q/2^m with Q the quotient
//   of r(x) x^m by p(x)
__global__ void k_phi_table(double* tphi, int rule, int64_t N, int m, uint64_t p, int kind,
                            int64_t snum, int64_t sden) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int64_t numer = r;
  if (rule == QMC_RULE_POLY_GF2) {
    uint64_t a = (uint64_t)r << m, q = 0;
    for (int k = m - 1; k >= 0; --k) {
      if ((a >> (m + k)) & 1) {
        a ^= p << k;
        q |= uint64_t(1) << k;
      }
    }
    numer = (int64_t)q;
  }
  const int64_t D = N * sden;
  const int64_t K = (numer * sden + snum * N) % D;
  tphi[r] = phi_of(kind, K, D);
}

// circulant generator z_k = T_phi[pow[k]], embedded into length M when
// M != L:  h[d] = z[d] (d < L), h[M-L+d] = z[d] (d >= 1), 0 elsewhere.
__global__ void k_generator(cx<double>* h, const int32_t* pow, const double* tphi, int64_t L,
                            int64_t M) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= M) return;
  double v = 0.0;
  if (d < L)
    v = tphi[pow[d]];
  else if (M != L && d >= M - L + 1)
    v = tphi[pow[d - (M - L)]];
  h[d] = {v, 0.0};
}

// W[k] = exp(-2 pi i k / M) in FP64
__global__ void k_twiddle(cx<double>* W, int64_t M) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)M, &s, &c);
  W[k] = {c, -s};
}

// one radix-2 Stockham pass of a forward FP64 DFT of length M over global
// memory (M = 2^k, or f x 2^k after one radix-f pass, f = 3, 5)
__global__ void k_fft_r2_pass(const cx<double>* in, cx<double>* out, int64_t M, int64_t Ns,
                              const cx<double>* W) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M / 2) return;
  const int64_t k = j % Ns;
  cx<double> a0 = in[j], a1 = in[j + M / 2];
  a1 = cmul(a1, W[k * (M / (2 * Ns))]);
  const int64_t base = (j / Ns) * 2 * Ns + k;
  out[base] = a0 + a1;
  out[base + Ns] = a0 - a1;
}

// the radix-5 Stockham pass of a forward FP64 DFT of length M = 5 x 2^k
// (the first pass, Ns = 1, of those lengths)
__global__ void k_fft_r5_pass(const cx<double>* in, cx<double>* out, int64_t M, int64_t Ns,
                              const cx<double>* W) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M / 5) return;
  const int64_t k = j % Ns, step = M / (5 * Ns), f = M / 5;
  cx<double> a[5];
  for (int q = 0; q < 5; ++q) a[q] = in[j + q * f];
  for (int q = 1; q < 5; ++q) a[q] = cmul(a[q], W[q * k * step]);
  bfly5<double, -1>(a[0], a[1], a[2], a[3], a[4]);
  const int64_t base = (j / Ns) * 5 * Ns + k;
  for (int q = 0; q < 5; ++q) out[base + q * Ns] = a[q];
}

// the radix-3 Stockham pass of a forward FP64 DFT of length M = 3 x 2^k
// (the first pass, Ns = 1, of those lengths)
__global__ void k_fft_r3_pass(const cx<double>* in, cx<double>* out, int64_t M, int64_t Ns,
                              const cx<double>* W) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M / 3) return;
  const int64_t k = j % Ns, step = M / (3 * Ns);
  cx<double> a0 = in[j], a1 = in[j + M / 3], a2 = in[j + 2 * (M / 3)];
  a1 = cmul(a1, W[k * step]);
  a2 = cmul(a2, W[2 * k * step]);
  bfly3<double, -1>(a0, a1, a2);
  const int64_t base = (j / Ns) * 3 * Ns + k;
  out[base] = a0;
  out[base + Ns] = a1;
  out[base + 2 * Ns] = a2;
}

template <typename T>
__device__ __forceinline__ cx<T> to_t(cx<double> a) {
  return {(T)a.x, (T)a.y};
}

// Per-thread tables of the fused kernel use the paired order of
// paired_index(value, thread, threads, PP): a thread's values 2k and 2k+1
// are adjacent.

// spectrum / M: block w2, thread g + R f, value h for w1 = f + R g + R^2 h,
// holding Hhat[w2 + M2 w1] / M
template <typename T>
__global__ void k_spectrum_layout(cx<T>* Hs, const cx<double>* Hhat, int R, int64_t M,
                                  int64_t M2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int64_t M1 = M / M2, Q = (int64_t)R * R;
  const int64_t w2 = i / M1, w1 = i % M1;
  const int64_t f = w1 % R, g = (w1 / R) % R, h = w1 / Q;
  const cx<double> v = Hhat[w2 + M2 * w1];
  const double inv = 1.0 / (double)M;
  Hs[w2 * M1 + paired_index(h, g + R * f, Q, pair_pp(R))] = to_t<T>({v.x * inv, v.y * inv});
}

// twf1: thread e1' < R^2, value f < R: W_{M1}^{e1' f} = W_M^{e1' f M2}
template <typename T>
__global__ void k_tw_f1(cx<T>* twf1, const cx<double>* W, int R, int64_t M, int64_t M2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int Q = R * R;
  if (i >= R * Q) return;
  const int64_t f = i / Q, e = i % Q;
  twf1[paired_index(f, e, Q, pair_pp(R))] = to_t<T>(W[(e * f * M2) % M]);
}

// twf2: thread a, value g: W_{R^2}^{a g} = W_M^{a g M / R^2}
template <typename T>
__global__ void k_tw_f2(cx<T>* twf2, const cx<double>* W, int R, int64_t M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * R) return;
  const int64_t g = i / R, a = i % R;
  twf2[paired_index(g, a, R, pair_pp(R))] = to_t<T>(W[(a * g * (M / ((int64_t)R * R))) % M]);
}

// twi3: block w2, thread a + R f, value bb: conj W_M^{e1' (f M2 + w2)} with
// e1' = a + R bb
template <typename T>
__global__ void k_tw_i3(cx<T>* twi3, const cx<double>* W, int R, int64_t M, int64_t M2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int64_t M1 = M / M2, Q = (int64_t)R * R;
  const int64_t f = i % R, e = (i / R) % Q, w2 = i / M1;
  const cx<double> w = W[(e * (f * M2 + w2)) % M];
  const int64_t a = e % R, bb = e / R;
  twi3[w2 * M1 + paired_index(bb, a + R * f, Q, pair_pp(R))] = to_t<T>({w.x, -w.y});
}

// two[w2][c] = conj W_M^{R^2 c w2}
template <typename T>
__global__ void k_tw_outer(cx<T>* two, const cx<double>* W, int R, int64_t M, int64_t M2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M2 * R) return;
  const int64_t c = i % R, w2 = i / R;
  const cx<double> w = W[((int64_t)R * R * c * w2) % M];
  two[i] = to_t<T>({w.x, -w.y});
}

// twit[b][w2][u] = W_M^{slot_{b,u} w2} for nb schedules b of Upad items
// each (0 for padding items)
template <typename T>
__global__ void k_tw_items(cx<T>* twit, const cx<double>* W, const int32_t* slot, int64_t Upad,
                           int64_t M, int64_t M2, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * M2 * Upad) return;
  const int64_t u = i % Upad, w2 = (i / Upad) % M2, b = i / (Upad * M2);
  const int32_t k = slot[b * Upad + u];
  twit[i] = (k < 0) ? cx<T>{(T)0, (T)0} : to_t<T>(W[((int64_t)k * w2) % M]);
}

// rowmap[e] = pow[e] - 1
__global__ void k_minus1(int32_t* out, const int32_t* in, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] - 1;
}

// twb[k] = conj W_{M2}^k, k < M2: the twiddles of any split M2 = P2 Q2 of the
// outer DFT, read at k = a q mod M2
template <typename T>
__global__ void k_tw_back(cx<T>* twb, const cx<double>* W, int64_t M, int64_t M2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M2) return;
  const cx<double> w = W[k * (M / M2)];
  twb[k] = to_t<T>({w.x, -w.y});
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

#define QMC_TRY(x)                       \
  do {                                   \
    int _e = (x);                        \
    if (_e != QMC_OK) return _e;         \
  } while (0)
#define QMC_HIP(x) QMC_TRY(hip_ok(x))

// ---------------------------------------------------------------------------
// layout choice
// ---------------------------------------------------------------------------
Layout choose_layout(int64_t L, int dtype, int* embedded, bool mixed) {
  Layout lay;
  int64_t M = 1;
  if ((L & (L - 1)) == 0) {
    M = L;
    *embedded = 0;
  } else {
    while (M < 2 * L - 1) M <<= 1;
    *embedded = 1;
    // the shortest embedding: f x 2^k (f = 3, 5) when it is shorter than the
    // power of two and its outer length M / 16^3 = f x 2^j fits one back
    // pass (M2 <= the dtype's longest outer radix: no split pass)
    for (const int64_t f : {3, 5}) {
      int64_t Mf = f;
      while (Mf < 2 * L - 1) Mf <<= 1;
      if (mixed && Mf < M && Mf >= f * 4096 && Mf / 4096 <= max_outer_q(dtype)) M = Mf;
    }
  }
  lay.M = M;
  const int rmax = 16;
  const int64_t M_2 = M % 3 == 0 ? M / 3 : M % 5 == 0 ? M / 5 : M;  // the power-of-two part
  int R = 1;
  while (2 * R <= rmax && (int64_t)(2 * R) * (2 * R) * (2 * R) <= M_2) R *= 2;
  lay.R = R;
  lay.M1 = (int64_t)R * R * R;
  lay.M2 = M / lay.M1;
  if (set_outer_split(lay, 0, max_outer_q(dtype)) != QMC_OK)  // too long: unsupported
    lay.P2 = lay.Q2 = lay.Pf = lay.Qf = 0;
  return lay;
}

int set_outer_split(Layout& lay, int q, int qmax) {
  // The outer inverse DFT of the back pass takes Q2 values of w2 per output
  // column and the split pass P2 = M2 / Q2 (a power of two, at most 64).
  // Q2 <= 32 stays in registers (32: occupancy 3), 48 and more go through LDS
  // (qmax: what the LDS tile of the dtype allows).  The default q = 0 takes
  // the whole of M2 when it fits one back pass (M2 <= qmax: no split pass;
  // the LDS back pass costs less than a split pass plus a register back
  // pass), else 32, more only when M2 > 32 * 64 (with a split pass anyway,
  // the register back pass is the faster one).  The dense fronts' forward
  // split keeps at most 64 values per thread in registers: Qf = Q2 up to 64,
  // else Q2 / 2.  For M2 = f x 2^j (f = 3, 5) the factor f stays in Q2 and
  // Qf (a radix-f stage of their register DFTs): q must then be f x 2^i.
  auto radix_ok = [](int64_t v) {
    const int64_t p = v % 3 == 0 ? v / 3 : v % 5 == 0 ? v / 5 : v;
    return v >= 1 && (p & (p - 1)) == 0;
  };
  if (q < 0 || q > qmax || (q > 0 && !radix_ok(q))) return QMC_ERR_ARG;
  const int64_t qdef = lay.M2 <= qmax ? lay.M2 : std::max<int64_t>(32, lay.M2 / 64);
  const int64_t Q2 = std::min<int64_t>(q > 0 ? q : qdef, lay.M2);
  if (Q2 > qmax || lay.M2 % Q2 != 0) return QMC_ERR_ARG;
  const int64_t P2 = lay.M2 / Q2;
  if (P2 > 64 || (P2 & (P2 - 1))) return QMC_ERR_ARG;  // also: 3 or 5 | M2 needs it in Q2
  const int64_t Qf = Q2 <= 64 ? Q2 : Q2 / 2;
  if (lay.M2 / Qf > 64) return QMC_ERR_ARG;
  lay.Q2 = (int)Q2;
  lay.P2 = (int)(lay.M2 / Q2);
  lay.Qf = (int)Qf;
  lay.Pf = (int)(lay.M2 / Qf);
  return QMC_OK;
}

// collapse schedule.  An item is one distinct reflected slot
// (L - l_j) mod L; it carries every row j with that slot (CSR it_ptr/it_jl,
// increasing j: the collapse sums them, the a' = P a of Section 2.1 with
// its repeated exponents).  The residues e1 = slot mod M1 are owned by F
// slices (e1 mod F, one wavefront each); inside a slice every residue's items
// (its "bucket", in increasing slot: a fixed summation order) go to one lane,
// buckets assigned longest-first to the least-loaded lane.  A lane
// accumulates one bucket in registers and writes it once.  The lane's k-th
// item is u = ((k / PP * F + slice) * G + lane) * PP + k % PP, so its items
// come in adjacent pairs; the item count per lane is padded to a multiple of
// PP.
Schedule make_schedule(const Layout& lay, int64_t L, int64_t s, const int32_t* ell) {
  const int64_t M1 = lay.M1;
  const int R = lay.R;
  const int Q = R * R;
  const int G = Q < 64 ? Q : 64;
  const int F = Q / G;
  const int PP = pair_pp(R);
  // distinct slots, each with its rows in increasing j (rows with ell < 0 are
  // not part of the product: a block of a rule with non-prime N)
  std::vector<std::pair<int64_t, int32_t>> sj;
  sj.reserve(s);
  for (int64_t j = 0; j < s; ++j)
    if (ell[j] >= 0) sj.push_back({(L - ell[j]) % L, (int32_t)j});
  s = (int64_t)sj.size();
  std::sort(sj.begin(), sj.end());
  std::vector<int64_t> uslot, ufirst;  // slot and first index into sj of each distinct slot
  for (int64_t k = 0; k < s; ++k)
    if (k == 0 || sj[k].first != sj[k - 1].first) {
      uslot.push_back(sj[k].first);
      ufirst.push_back(k);
    }
  const int64_t nu = (int64_t)uslot.size();
  ufirst.push_back(s);
  // buckets: distinct slots of each residue e1 (increasing slot)
  std::vector<int64_t> start(M1 + 1, 0);
  for (int64_t i = 0; i < nu; ++i) start[(uslot[i] & (M1 - 1)) + 1]++;
  for (int64_t e = 0; e < M1; ++e) start[e + 1] += start[e];
  std::vector<int64_t> members(nu);
  {
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < nu; ++i) members[pos[uslot[i] & (M1 - 1)]++] = i;
  }
  // per slice: longest-first assignment of buckets to lanes
  std::vector<std::vector<int64_t>> lane_items((size_t)F * G);  // distinct-slot ids in order
  std::vector<int64_t> load(G);
  std::vector<int64_t> order;
  for (int f = 0; f < F; ++f) {
    order.clear();
    for (int64_t e = f; e < M1; e += F)
      if (start[e + 1] > start[e]) order.push_back(e);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return start[a + 1] - start[a] > start[b + 1] - start[b];
    });
    std::fill(load.begin(), load.end(), 0);
    for (int64_t e : order) {
      const int ln = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[ln] += start[e + 1] - start[e];
      std::vector<int64_t>& li = lane_items[(size_t)f * G + ln];
      for (int64_t k = start[e]; k < start[e + 1]; ++k) li.push_back(members[k]);
    }
  }
  Schedule sc;
  int64_t rounds = 1;
  for (const auto& li : lane_items) rounds = std::max(rounds, (int64_t)li.size());
  rounds = (rounds + PP - 1) / PP * PP;  // whole item pairs
  sc.rounds = rounds;
  sc.Upad = rounds * Q;
  std::vector<int64_t> item_of(sc.Upad, -1);  // distinct-slot id of item u (-1: padding)
  for (int f = 0; f < F; ++f)
    for (int ln = 0; ln < G; ++ln) {
      const std::vector<int64_t>& li = lane_items[(size_t)f * G + ln];
      for (size_t k = 0; k < li.size(); ++k)
        item_of[(((int64_t)k / PP * F + f) * G + ln) * PP + (int64_t)k % PP] = li[k];
    }
  sc.it_slot.assign(sc.Upad, -1);
  sc.it_e1.assign(sc.Upad, (int32_t)M1);
  sc.it_ptr.assign(sc.Upad + 1, 0);
  sc.it_jl.reserve(s);
  for (int64_t u = 0; u < sc.Upad; ++u) {
    const int64_t i = item_of[u];
    if (i >= 0) {
      sc.it_slot[u] = (int32_t)uslot[i];
      sc.it_e1[u] = (int32_t)(uslot[i] & (M1 - 1));
      for (int64_t k = ufirst[i]; k < ufirst[i + 1]; ++k) sc.it_jl.push_back(sj[k].second);
    }
    sc.it_ptr[u + 1] = (int32_t)sc.it_jl.size();
  }
  return sc;
}

void pad_schedule(Schedule& sc, int64_t rounds, int64_t M1, int R) {
  if (rounds <= sc.rounds) return;
  // the item index of a lane's k-th item does not depend on the round
  // count: extra rounds are padding items (empty row lists) at the end
  sc.rounds = rounds;
  sc.Upad = rounds * R * R;
  sc.it_slot.resize(sc.Upad, -1);
  sc.it_e1.resize(sc.Upad, (int32_t)M1);
  sc.it_ptr.resize(sc.Upad + 1, sc.it_ptr.back());
}

template <typename T>
static int build_spectral_tables(qmc_plan_s* P, const cx<double>* dW, const cx<double>* dH,
                                 const int32_t* dslot, hipStream_t st) {
  int err = QMC_OK;
  const Layout& lay = P->lay;
  const int R = lay.R;
  const int64_t M = lay.M, M1 = lay.M1, M2 = lay.M2;
  cx<T>* Hs = dev_alloc<cx<T>>(P, M, &err);
  cx<T>* twf1 = dev_alloc<cx<T>>(P, (size_t)R * R * R, &err);
  cx<T>* twf2 = dev_alloc<cx<T>>(P, (size_t)R * R, &err);
  cx<T>* twi3 = dev_alloc<cx<T>>(P, M, &err);
  cx<T>* two = dev_alloc<cx<T>>(P, M2 * R, &err);
  cx<T>* twit = dev_alloc<cx<T>>(P, M2 * P->Upad, &err);
  cx<T>* twb = dev_alloc<cx<T>>(P, (size_t)M2, &err);
  if (err != QMC_OK) return err;
  k_spectrum_layout<T><<<nblk(M), 256, 0, st>>>(Hs, dH, R, M, M2);
  k_tw_f1<T><<<nblk(R * R * R), 256, 0, st>>>(twf1, dW, R, M, M2);
  k_tw_f2<T><<<nblk(R * R), 256, 0, st>>>(twf2, dW, R, M);
  k_tw_i3<T><<<nblk(M), 256, 0, st>>>(twi3, dW, R, M, M2);
  k_tw_outer<T><<<nblk(M2 * R), 256, 0, st>>>(two, dW, R, M, M2);
  k_tw_items<T><<<nblk(M2 * P->Upad), 256, 0, st>>>(twit, dW, dslot, P->Upad, M, M2, 1);
  k_tw_back<T><<<nblk(M2), 256, 0, st>>>(twb, dW, M, M2);
  QMC_HIP(hipGetLastError());
  P->d_Hs = Hs;
  P->d_twf1 = twf1;
  P->d_twf2 = twf2;
  P->d_twi3 = twi3;
  P->d_two = two;
  P->d_twit = twit;
  P->d_twb = twb;
  return QMC_OK;
}

// The collapse schedule, the inverse map of the exponents and the spectral
// tables of a plan whose layout is set: ell (host, P->s entries; -1 for rows
// of A outside the product) and the generator z_k = tphi[zidx[k]], k < L
// (device tables), embedded in the convolution length M as k_generator
// describes.
int build_conv_tables(qmc_plan_s* P, const int32_t* ell, const int32_t* d_zidx,
                      const double* d_tphi, hipStream_t st) {
  int err = QMC_OK;
  const int64_t L = P->L, s = P->s;
  const Layout& lay = P->lay;
  std::vector<void*> temps;
  auto free_temps = [&]() {
    for (void* p : temps) hipFree(p);
  };
  int rc = QMC_OK;
  do {
    Schedule sc = make_schedule(lay, L, s, ell);
    const int64_t sa = (int64_t)sc.it_jl.size();  // rows in the product
    P->s_active = sa;
    // the residues go to the device as 16-bit values (e1 <= M1 <= 4096)
    const std::vector<uint16_t> e16(sc.it_e1.begin(), sc.it_e1.end());
    P->rounds = sc.rounds;
    P->Upad = sc.Upad;
    P->d_it_ptr = dev_alloc<int32_t>(P, P->Upad + 1, &err);
    P->d_it_jl = dev_alloc<int32_t>(P, sa, &err);
    P->d_it_e1 = dev_alloc<uint16_t>(P, P->Upad, &err);
    P->d_it_e2 = dev_alloc<uint16_t>(P, P->Upad, &err);
    P->d_inv_ptr = dev_alloc<int32_t>(P, L + 1, &err);
    P->d_inv_j = dev_alloc<int32_t>(P, sa, &err);
    // e2 = slot / M1 of every item (the outer index of its slot, 0 for padding)
    std::vector<uint16_t> e2(P->Upad);
    for (int64_t u = 0; u < P->Upad; ++u)
      e2[u] = sc.it_slot[u] >= 0 ? (uint16_t)(sc.it_slot[u] / lay.M1) : (uint16_t)0;
    if ((rc = err) != QMC_OK) break;
    int32_t* d_slot = nullptr;
    if ((rc = hip_ok(hipMalloc(&d_slot, P->Upad * sizeof(int32_t)))) != QMC_OK) break;
    temps.push_back(d_slot);
    // inverse of j -> l_j (counting sort, j increasing within each e)
    std::vector<int32_t> inv_ptr(L + 1, 0), inv_j(std::max<int64_t>(sa, 1));
    for (int64_t j = 0; j < s; ++j)
      if (ell[j] >= 0) inv_ptr[ell[j] + 1]++;
    for (int64_t e = 0; e < L; ++e) inv_ptr[e + 1] += inv_ptr[e];
    {
      std::vector<int32_t> pos(inv_ptr.begin(), inv_ptr.end() - 1);
      for (int64_t j = 0; j < s; ++j)
        if (ell[j] >= 0) inv_j[pos[ell[j]]++] = (int32_t)j;
    }
    rc = hip_ok(hipMemcpyAsync(P->d_it_ptr, sc.it_ptr.data(), (P->Upad + 1) * 4,
                               hipMemcpyHostToDevice, st));
    if (rc == QMC_OK && sa > 0)
      rc = hip_ok(hipMemcpyAsync(P->d_it_jl, sc.it_jl.data(), sa * 4, hipMemcpyHostToDevice, st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(P->d_it_e1, e16.data(), P->Upad * sizeof(uint16_t),
                                 hipMemcpyHostToDevice, st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(P->d_it_e2, e2.data(), P->Upad * sizeof(uint16_t),
                                 hipMemcpyHostToDevice, st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(d_slot, sc.it_slot.data(), P->Upad * 4, hipMemcpyHostToDevice,
                                 st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(P->d_inv_ptr, inv_ptr.data(), (L + 1) * 4, hipMemcpyHostToDevice, st));
    if (rc == QMC_OK && sa > 0)
      rc = hip_ok(hipMemcpyAsync(P->d_inv_j, inv_j.data(), sa * 4, hipMemcpyHostToDevice, st));
    // host vectors must outlive the asynchronous copies
    if (rc == QMC_OK) rc = hip_ok(hipStreamSynchronize(st));
    if (rc != QMC_OK) break;

    // ---- generator spectrum in FP64 -------------------------------------
    const int64_t M = lay.M;
    cx<double>*dW = nullptr, *dA = nullptr, *dB = nullptr;
    if ((rc = hip_ok(hipMalloc(&dW, M * sizeof(cx<double>)))) != QMC_OK) break;
    temps.push_back(dW);
    if ((rc = hip_ok(hipMalloc(&dA, M * sizeof(cx<double>)))) != QMC_OK) break;
    temps.push_back(dA);
    if ((rc = hip_ok(hipMalloc(&dB, M * sizeof(cx<double>)))) != QMC_OK) break;
    temps.push_back(dB);
    k_twiddle<<<nblk(M), 256, 0, st>>>(dW, M);
    k_generator<<<nblk(M), 256, 0, st>>>(dA, d_zidx, d_tphi, L, M);
    cx<double>*src = dA, *dst = dB;
    int64_t Ns = 1;
    if (M % 3 == 0) {  // M = 3 x 2^k: the radix-3 pass first
      k_fft_r3_pass<<<nblk(M / 3), 256, 0, st>>>(src, dst, M, Ns, dW);
      std::swap(src, dst);
      Ns = 3;
    } else if (M % 5 == 0) {  // M = 5 x 2^k: the radix-5 pass first
      k_fft_r5_pass<<<nblk(M / 5), 256, 0, st>>>(src, dst, M, Ns, dW);
      std::swap(src, dst);
      Ns = 5;
    }
    for (; Ns < M; Ns *= 2) {
      k_fft_r2_pass<<<nblk(M / 2), 256, 0, st>>>(src, dst, M, Ns, dW);
      std::swap(src, dst);
    }
    if ((rc = hip_ok(hipGetLastError())) != QMC_OK) break;
    if (P->dtype == QMC_F32)
      rc = build_spectral_tables<float>(P, dW, src, d_slot, st);
    else
      rc = build_spectral_tables<double>(P, dW, src, d_slot, st);
    if (rc != QMC_OK) break;
    rc = hip_ok(hipStreamSynchronize(st));
  } while (0);
  free_temps();
  return rc;
}

// phi of every residue's coordinate into P->d_tphi (N entries)
int launch_phi_table(qmc_plan_s* P, hipStream_t st) {
  k_phi_table<<<nblk(P->N), 256, 0, st>>>(P->d_tphi, P->rule, P->N, P->m, P->modulus,
                                           P->phi_kind, P->shift_num, P->shift_den);
  return hip_ok(hipGetLastError());
}

int build_tables(qmc_plan_s* P, const uint64_t* gen_host, hipStream_t st) {
  int err = QMC_OK;
  const int64_t N = P->N, L = P->L, s = P->s;

  // ---- host validation and number theory --------------------------------
  std::vector<uint32_t> gen(s);
  if (P->rule == QMC_RULE_LATTICE) {
    // non-prime N: the orbits of the rows and the blocks of each
    if (!is_prime_u64((uint64_t)N)) return build_composite(P, gen_host, st);
    for (int64_t j = 0; j < s; ++j) {
      const uint64_t g = gen_host[j] % (uint64_t)N;
      if (g == 0) return QMC_ERR_GEN_ZERO;
      gen[j] = (uint32_t)g;
    }
    P->beta = smallest_primitive_root((uint64_t)N);
    if (P->beta == 0) return QMC_ERR_NOT_PRIME;
  } else {
    if (!gf2_is_primitive(P->modulus, P->m)) return QMC_ERR_NOT_PRIMITIVE;
    for (int64_t j = 0; j < s; ++j) {
      if (gen_host[j] == 0 || gen_host[j] >= (uint64_t)N) return QMC_ERR_GEN_ZERO;
      gen[j] = (uint32_t)gen_host[j];
    }
    P->beta = (P->m == 1) ? 1 : 2;
  }
  P->lay = choose_layout(L, P->dtype, &P->embedded, P->mixed_outer);
  const Layout& lay = P->lay;
  if (lay.P2 < 1) return QMC_ERR_UNSUPPORTED;  // outer length beyond the longest split

  // ---- bit-exact group tables ------------------------------------------
  P->d_pow = dev_alloc<int32_t>(P, L, &err);
  P->d_log = dev_alloc<int32_t>(P, N, &err);
  P->d_ell = dev_alloc<int32_t>(P, s, &err);
  P->d_tphi = dev_alloc<double>(P, N, &err);
  if (err != QMC_OK) return err;
  uint32_t* d_gen = dev_alloc<uint32_t>(P, s, &err);
  if (err != QMC_OK) return err;
  P->d_gen = d_gen;
  std::vector<void*> temps;
  auto free_temps = [&]() {
    for (void* p : temps) hipFree(p);
  };
  int rc = QMC_OK;
  do {
    if ((rc = hip_ok(hipMemcpyAsync(d_gen, gen.data(), s * sizeof(uint32_t),
                                    hipMemcpyHostToDevice, st))) != QMC_OK)
      break;
    if (P->rule == QMC_RULE_LATTICE)
      k_pow_lattice<<<nblk(L), 256, 0, st>>>(P->d_pow, L, (uint64_t)N, P->beta);
    else
      k_pow_gf2<<<nblk(L), 256, 0, st>>>(P->d_pow, L, P->modulus, P->m);
    k_fill_i32<<<nblk(N), 256, 0, st>>>(P->d_log, N, -1);
    k_log_scatter<<<nblk(L), 256, 0, st>>>(P->d_pow, L, P->d_log);
    k_ell<<<nblk(s), 256, 0, st>>>(d_gen, s, P->d_log, P->d_ell);
    k_phi_table<<<nblk(N), 256, 0, st>>>(P->d_tphi, P->rule, N, P->m, P->modulus, P->phi_kind,
                                         P->shift_num, P->shift_den);
    if ((rc = hip_ok(hipGetLastError())) != QMC_OK) break;

    std::vector<int32_t> ell(s);
    if ((rc = hip_ok(hipMemcpyAsync(ell.data(), P->d_ell, s * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, st))) != QMC_OK)
      break;
    if ((rc = hip_ok(hipMemcpyAsync(&P->phi0, P->d_tphi, sizeof(double),
                                    hipMemcpyDeviceToHost, st))) != QMC_OK)
      break;
    if ((rc = hip_ok(hipStreamSynchronize(st))) != QMC_OK) break;
    for (int64_t j = 0; j < s; ++j)
      if (ell[j] < 0 || ell[j] >= L) { rc = QMC_ERR_HIP; break; }
    if (rc != QMC_OK) break;

    rc = build_conv_tables(P, ell.data(), P->d_pow, P->d_tphi, st);
  } while (0);
  free_temps();
  return rc;
}

// ---------------------------------------------------------------------------
// union of Korobov lattice point sets: per block b (Korobov base b = 1..K-1,
// generating vector b^j mod K) the exponents l_{b,j} = j log(b) mod (K-1),
// i.e. c_{g,j} - 1 of the paper's ordering with b = beta^(g-1); every block
// shares the base plan's spectrum and twiddles and has its own collapse
// schedule, padded to a common size
// ---------------------------------------------------------------------------
int build_korobov_tables(qmc_korobov_s* U, hipStream_t st) {
  qmc_plan_s* P = U->base;
  const Layout& lay = P->lay;
  const int64_t K = P->N, L = P->L, s = U->s, nb = K - 1, M = lay.M, M2 = lay.M2;
  std::vector<int32_t> logt(K);
  int rc = hip_ok(hipMemcpyAsync(logt.data(), P->d_log, K * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st));
  if (rc == QMC_OK) rc = hip_ok(hipStreamSynchronize(st));
  if (rc != QMC_OK) return rc;
  std::vector<Schedule> scs(nb);
  std::vector<int32_t> ell(s);
  // the adjoint's read-back: per block, the rows j of each exponent e
  // (counting sort by l_{b,j}, increasing j inside an exponent)
  std::vector<int32_t> inv_ptr(nb * (L + 1)), inv_j(nb * s);
  int64_t rounds = 0;
  for (int64_t b = 1; b <= nb; ++b) {
    const int64_t lam = logt[b];
    if (lam < 0 || lam >= L) return QMC_ERR_HIP;
    for (int64_t j = 0; j < s; ++j) ell[j] = (int32_t)((j % L) * lam % L);
    scs[b - 1] = make_schedule(lay, L, s, ell.data());
    rounds = std::max(rounds, scs[b - 1].rounds);
    int32_t* ip = inv_ptr.data() + (b - 1) * (L + 1);
    int32_t* ij = inv_j.data() + (b - 1) * s;
    for (int64_t j = 0; j < s; ++j) ++ip[ell[j] + 1];
    for (int64_t e = 0; e < L; ++e) ip[e + 1] += ip[e];
    std::vector<int32_t> fill(ip, ip + L);
    for (int64_t j = 0; j < s; ++j) ij[fill[ell[j]]++] = (int32_t)j;
  }
  for (Schedule& sc : scs) pad_schedule(sc, rounds, lay.M1, lay.R);
  U->rounds = rounds;
  U->Upad = scs[0].Upad;
  const int64_t Upad = U->Upad;
  std::vector<int32_t> it_ptr(nb * (Upad + 1)), it_jl(nb * s), slot(nb * Upad);
  std::vector<uint16_t> it_e1(nb * Upad);  // 16-bit residues (e1 <= M1 <= 4096)
  for (int64_t b = 0; b < nb; ++b) {
    std::copy(scs[b].it_ptr.begin(), scs[b].it_ptr.end(), it_ptr.begin() + b * (Upad + 1));
    std::copy(scs[b].it_jl.begin(), scs[b].it_jl.end(), it_jl.begin() + b * s);
    std::copy(scs[b].it_e1.begin(), scs[b].it_e1.end(), it_e1.begin() + b * Upad);
    std::copy(scs[b].it_slot.begin(), scs[b].it_slot.end(), slot.begin() + b * Upad);
  }
  scs.clear();
  int err = QMC_OK;
  const size_t el = P->dtype == QMC_F32 ? sizeof(cx<float>) : sizeof(cx<double>);
  U->d_it_ptr = dev_alloc<int32_t>(P, nb * (Upad + 1), &err);
  U->d_it_jl = dev_alloc<int32_t>(P, nb * s, &err);
  U->d_it_e1 = dev_alloc<uint16_t>(P, nb * Upad, &err);
  U->d_rowmap = dev_alloc<int32_t>(P, L, &err);
  U->d_twit = dev_alloc<char>(P, nb * M2 * Upad * el, &err);
  U->d_inv_ptr = dev_alloc<int32_t>(P, nb * (L + 1), &err);
  U->d_inv_j = dev_alloc<int32_t>(P, nb * s, &err);
  if (err != QMC_OK) return err;
  int32_t* d_slot = nullptr;
  cx<double>* dW = nullptr;
  do {
    if ((rc = hip_ok(hipMalloc(&d_slot, nb * Upad * sizeof(int32_t)))) != QMC_OK) break;
    if ((rc = hip_ok(hipMalloc(&dW, M * sizeof(cx<double>)))) != QMC_OK) break;
    rc = hip_ok(hipMemcpyAsync(U->d_it_ptr, it_ptr.data(), nb * (Upad + 1) * 4,
                               hipMemcpyHostToDevice, st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(U->d_it_jl, it_jl.data(), nb * s * 4, hipMemcpyHostToDevice,
                                 st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(U->d_it_e1, it_e1.data(), nb * Upad * sizeof(uint16_t), hipMemcpyHostToDevice,
                                 st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(d_slot, slot.data(), nb * Upad * 4, hipMemcpyHostToDevice, st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(U->d_inv_ptr, inv_ptr.data(), nb * (L + 1) * 4,
                                 hipMemcpyHostToDevice, st));
    if (rc == QMC_OK)
      rc = hip_ok(hipMemcpyAsync(U->d_inv_j, inv_j.data(), nb * s * 4, hipMemcpyHostToDevice,
                                 st));
    if (rc != QMC_OK) break;
    k_twiddle<<<nblk(M), 256, 0, st>>>(dW, M);
    if (P->dtype == QMC_F32)
      k_tw_items<float><<<nblk(nb * M2 * Upad), 256, 0, st>>>((cx<float>*)U->d_twit, dW, d_slot,
                                                             Upad, M, M2, nb);
    else
      k_tw_items<double><<<nblk(nb * M2 * Upad), 256, 0, st>>>((cx<double>*)U->d_twit, dW,
                                                              d_slot, Upad, M, M2, nb);
    k_minus1<<<nblk(L), 256, 0, st>>>(U->d_rowmap, P->d_pow, L);
    if ((rc = hip_ok(hipGetLastError())) != QMC_OK) break;
    rc = hip_ok(hipStreamSynchronize(st));  // the host vectors outlive the copies
  } while (0);
  if (d_slot) hipFree(d_slot);
  if (dW) hipFree(dW);
  return rc;
}

}  // namespace qmc
