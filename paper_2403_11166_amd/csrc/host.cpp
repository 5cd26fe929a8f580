// Host side of libpencil: parameter resolution, NTT tables, key generation,
// tiling geometry, the packing planner, and the C ABI of include/pencil.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pencil.h"
#include "pencil_internal.h"

using namespace pencil;
typedef unsigned __int128 u128;

// ----------------------------------------------------------------- context

struct pencil_ctx {
  pencil_info info{};
  Consts C{};
  Tables T{};
  int device = 0;
  // device memory owned by the context
  TW* d_tables = nullptr;        // forward then inverse twiddles, each [L][N]
  uint64_t* d_s_ntt = nullptr;   // [L][N]
  uint64_t* d_s_sh = nullptr;    // [L][N]
  uint64_t* d_pk_ntt = nullptr;  // [2][L][N]
  uint64_t* d_pk_sh = nullptr;   // [2][L][N]
  uint64_t* d_pk_split = nullptr;  // [2][L][N], the multiply-accumulate's split operand form
  uint64_t* d_pk_coeff = nullptr;
  int64_t* d_s_coeff = nullptr;
  uint64_t* d_noise = nullptr;   // one word: the checked decryption's largest noise fraction
  void* d_scratch = nullptr;     // this device's copy of the allocation-free entry points' scratch array
  std::string err;
  // kernel timing with HIP events on the launch stream (pencil_profile_*)
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  struct Rec {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  double prof_ms[16] = {};
  uint64_t prof_launches[16] = {};
};

enum KernelId {
  KID_NTT_CT, KID_NTT_PT, KID_NTT_TERNARY, KID_MAC, KID_INTT_OUT, KID_FLOOD, KID_ENCRYPT, KID_PHASE, KID_DECODE,
  KID_NTT_PLAIN, KID_STEP_NTT, KID_STEP_MAC, KID_STEP_INTT, KID_STEP_FLOOD, KID_COUNT
};
static const char* kKernelNames[KID_COUNT] = {"ntt_ct", "ntt_pt", "ntt_ternary", "mac", "intt_out",
                                              "flood_mask", "encrypt", "phase", "decode", "ntt_plain",
                                              "step_ntt", "step_mac", "step_intt", "step_flood"};

static hipEvent_t pool_event(pencil_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` and, when profiling is on, bracket it with events on stream s.
template <class F>
static hipError_t timed(pencil_ctx* ctx, int kid, hipStream_t s, F&& launch) {
  if (!ctx->prof_on) return launch();
  hipEvent_t a = pool_event(ctx), b = pool_event(ctx);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  ctx->pending.push_back({kid, a, b});
  return e;
}

static thread_local std::string g_create_err;

static pencil_status fail(pencil_ctx* ctx, pencil_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_create_err = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return fail(ctx, PENCIL_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// ------------------------------------------------------------ number theory

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod(r, b, m);
    b = mulmod(b, b, m);
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for 64-bit n (these bases decide every n < 2^64).
static bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++r;
  }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

static uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// Smallest primitive 2N-th root of unity mod q: find one root, then the least of its odd powers.
static uint64_t min_root(uint64_t q, uint64_t n) {
  uint64_t psi = 0;
  for (uint64_t g = 2; g < (1u << 20); ++g) {
    uint64_t c = powmod(g, (q - 1) / (2 * n), q);
    if (powmod(c, n, q) == q - 1) {
      psi = c;
      break;
    }
  }
  uint64_t best = psi, sq = mulmod(psi, psi, q), cur = psi;
  for (uint64_t i = 0; i < n; ++i) {
    if (cur < best) best = cur;
    cur = mulmod(cur, sq, q);
  }
  return best;
}

// Little-endian multiword integers.
typedef std::vector<uint64_t> Big;

static void big_trim(Big& a) {
  while (a.size() > 1 && a.back() == 0) a.pop_back();
}
static Big big_mul_small(const Big& a, uint64_t m) {
  Big r(a.size() + 1, 0);
  u128 carry = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    u128 p = (u128)a[i] * m + carry;
    r[i] = (uint64_t)p;
    carry = p >> 64;
  }
  r[a.size()] = (uint64_t)carry;
  big_trim(r);
  return r;
}
static uint64_t big_mod_small(const Big& a, uint64_t m) {
  u128 r = 0;
  for (size_t i = a.size(); i-- > 0;) r = ((r << 64) | a[i]) % m;
  return (uint64_t)r;
}
static Big big_div_small(const Big& a, uint64_t m) {
  Big q(a.size(), 0);
  u128 r = 0;
  for (size_t i = a.size(); i-- > 0;) {
    u128 cur = (r << 64) | a[i];
    q[i] = (uint64_t)(cur / m);
    r = cur % m;
  }
  big_trim(q);
  return q;
}
static int big_bits(const Big& a) {
  for (size_t i = a.size(); i-- > 0;)
    if (a[i]) return (int)(64 * i + 64 - __builtin_clzll(a[i]));
  return 0;
}

// ------------------------------------------------------------ context create

static pencil_status resolve_params(const pencil_params* p, pencil_ctx* ctx) {
  if (!p) return fail(nullptr, PENCIL_EINVAL, "params is NULL");
  if (p->log2_n < 10 || p->log2_n > 14) return fail(nullptr, PENCIL_EINVAL, "log2_n %u outside [10, 14]", p->log2_n);
  if (p->num_limbs < 1 || p->num_limbs > (uint32_t)kMaxLimbs)
    return fail(nullptr, PENCIL_EINVAL, "num_limbs %u outside [1, %d]", p->num_limbs, kMaxLimbs);
  const uint64_t n = 1ull << p->log2_n;
  pencil_info& I = ctx->info;
  I.log2_n = p->log2_n;
  I.num_limbs = p->num_limbs;
  I.seed = p->seed;
  // plaintext modulus
  uint64_t t = p->t;
  if (t == 0) {
    t = (1ull << 41) - 1;
    while (!is_prime(t)) t -= 2;
  }
  if (t < 3 || t >= (1ull << 48) || !is_prime(t)) return fail(nullptr, PENCIL_EINVAL, "t must be an odd prime < 2^48");
  I.t = t;
  // RNS primes
  if (p->primes[0] == 0) {
    if (p->prime_bits < 40 || p->prime_bits > 60)
      return fail(nullptr, PENCIL_EINVAL, "prime_bits %u outside [40, 60]", p->prime_bits);
    const uint64_t step = 1ull << 15;
    uint64_t q = (((1ull << p->prime_bits) - 1) / step) * step + 1;
    if (q >= (1ull << p->prime_bits)) q -= step;
    for (uint32_t l = 0; l < p->num_limbs; q -= step) {
      if (is_prime(q)) I.primes[l++] = q;
    }
  } else {
    for (uint32_t l = 0; l < p->num_limbs; ++l) {
      uint64_t q = p->primes[l];
      if (q == 0 || q >= (1ull << 60) || !is_prime(q) || (q - 1) % (2 * n) != 0)
        return fail(nullptr, PENCIL_EINVAL, "prime %u (%llu) must be a prime < 2^60 with q = 1 mod 2N", l,
                    (unsigned long long)q);
      for (uint32_t k = 0; k < l; ++k)
        if (I.primes[k] == q) return fail(nullptr, PENCIL_EINVAL, "repeated prime");
      I.primes[l] = q;
    }
  }
  for (uint32_t l = 0; l < p->num_limbs; ++l)
    if (I.primes[l] <= t) return fail(nullptr, PENCIL_EINVAL, "every q_l must exceed t");
  // q, Delta, flood width
  Big q{1};
  for (uint32_t l = 0; l < p->num_limbs; ++l) q = big_mul_small(q, I.primes[l]);
  if (big_bits(q) > 64 * (kMaxWords - 1) - 4) return fail(nullptr, PENCIL_EINVAL, "q too large");
  Big delta = big_div_small(q, t);
  const int dbits = big_bits(delta);
  if (dbits < 8) return fail(nullptr, PENCIL_EINVAL, "q / t too small for any noise budget");
  uint32_t fb = p->flood_bits ? p->flood_bits : (uint32_t)(dbits - 1 - 3);
  if (fb + 1 > 256) return fail(nullptr, PENCIL_EINVAL, "flood_bits too large");
  I.flood_bits = fb;

  Consts& C = ctx->C;
  C.log2n = (int32_t)p->log2_n;
  C.n = (int32_t)n;
  C.L = (int32_t)p->num_limbs;
  C.ntt_loge = p->log2_n >= 14 ? 5 : 4;
  C.flood_bits = fb;
  C.flood_words = (int32_t)((fb + 1 + 63) / 64);
  const int topbits = (int)(fb + 1) - 64 * (C.flood_words - 1);
  C.top_mask = topbits >= 64 ? ~0ull : ((1ull << topbits) - 1);
  C.t = t;
  C.t_half = (t - 1) / 2;
  C.rho = big_mod_small(q, t);
  C.rho_sh = shoup(C.rho, t);
  C.r64t = (uint64_t)(((u128)1 << 64) % t);
  C.r64t_sh = shoup(C.r64t, t);
  C.one_sh_t = (uint64_t)((((u128)1) << 64) / t);
  C.seed = p->seed;
  for (int l = 0; l < C.L; ++l) {
    const uint64_t ql = I.primes[l];
    {
      // the forward transform's final reduction folds the bits above the
      // modulus' bit length B with delta = 2^B - q (one conditional
      // subtraction left), which needs delta < 2^32 and 2^B + 15 delta < 2q
      int b = 0;
      while (b < 64 && (ql >> b) != 0) ++b;
      const u128 top = (u128)1 << b, delta = top - ql;
      if (delta >> 32 || top + 15 * delta >= 2 * (u128)ql)
        return fail(nullptr, PENCIL_EUNSUPPORTED, "modulus %llu too far below a power of two",
                    (unsigned long long)ql);
    }
    LimbConst& lc = C.limb[l];
    lc.q = ql;
    lc.r64 = (uint64_t)(((u128)1 << 64) % ql);
    lc.r64_sh = shoup(lc.r64, ql);
    lc.r128 = (uint64_t)(((u128)lc.r64 * lc.r64) % ql);
    lc.r192 = (uint64_t)(((u128)lc.r128 * lc.r64) % ql);
    lc.one_sh = (uint64_t)((((u128)1) << 64) / ql);
    lc.ninv = powmod(n, ql - 2, ql);
    lc.ninv_sh = shoup(lc.ninv, ql);
    lc.delta = big_mod_small(delta, ql);
    lc.delta_sh = shoup(lc.delta, ql);
    lc.t_sh = shoup(t, ql);
    Big qhat = big_div_small(q, ql);
    uint64_t qhat_mod = big_mod_small(qhat, ql);
    lc.qhat_inv = powmod(qhat_mod, ql - 2, ql);
    lc.qhat_inv_sh = shoup(lc.qhat_inv, ql);
    lc.flood_off = powmod(2, fb, ql);
    // floor(2^128 / q): long division of 2^128 by q
    u128 hi_part = (((u128)1) << 64) / ql;  // floor(2^64 / q) -> upper word of the quotient
    u128 rem = (((u128)1) << 64) % ql;
    u128 lo_part = (rem << 64) / ql;
    lc.mu_hi = (uint64_t)hi_part;
    lc.mu_lo = (uint64_t)lo_part;
    for (int w = 0; w < kMaxWords; ++w) C.qhat[l][w] = w < (int)qhat.size() ? qhat[w] : 0;
    Big th = big_mul_small(q, 2 * (uint64_t)l + 1);
    for (int w = 0; w < kMaxWords; ++w) C.thr[l][w] = w < (int)th.size() ? th[w] : 0;
    I.psi[l] = min_root(ql, n);
  }
  // Multiply-accumulate headroom.  Operands are split into 30-bit halves
  // a = a0 + a1 2^30 with a1 <= amax = (q - 1) >> 30; one step adds at most
  // 2 (2^30 - 1) amax to a cross-term partial sum holding both cross products,
  // so mac_fold steps keep all three 64-bit partial sums in range; with the
  // cross products in two sums, a step adds at most max((2^30 - 1)^2,
  // (2^30 - 1) amax, amax^2) to each and mac_fold4 steps fit.  A fold adds at
  // most F = max(mac_fold, mac_fold4) * (q - 1)^2 to the 128-bit total, which
  // holds mac_chunk folds on top of a reduced residue.
  {
    uint64_t qmax = 0;
    for (int l = 0; l < C.L; ++l) qmax = std::max(qmax, C.limb[l].q);
    const u128 lo30 = (1u << 30) - 1, amax = (qmax - 1) >> 30;
    const u128 step_max = std::max(std::max(lo30 * lo30, 2 * lo30 * amax), amax * amax);
    const u128 step_max4 = std::max(std::max(lo30 * lo30, lo30 * amax), amax * amax);
    u128 fold = ((u128)~0ull) / step_max, fold4 = ((u128)~0ull) / step_max4;
    if (fold > 64) fold = 64;
    if (fold4 > 64) fold4 = 64;
    C.mac_fold = (uint32_t)fold;
    C.mac_fold4 = (uint32_t)fold4;
    const u128 per_fold = std::max(fold, fold4) * (u128)(qmax - 1) * (qmax - 1);
    const u128 room = (~(u128)0) - qmax;
    u128 chunk = room / per_fold;
    if (chunk > 1024) chunk = 1024;
    // the kernels reduce their (at most 8) accumulators in turn, one per fold
    if (chunk < 8) return fail(nullptr, PENCIL_EUNSUPPORTED, "primes too large for the lazy accumulation");
    C.mac_chunk = (uint32_t)chunk;
  }
  C.qwords = (uint32_t)q.size();
  return PENCIL_OK;
}

static uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

extern "C" pencil_status pencil_ctx_create(const pencil_params* params, pencil_ctx** out) {
  if (!out) return fail(nullptr, PENCIL_EINVAL, "out is NULL");
  *out = nullptr;
  pencil_ctx* ctx = new pencil_ctx();
  pencil_status st = resolve_params(params, ctx);
  if (st != PENCIL_OK) {
    delete ctx;
    return st;
  }
  const Consts& C = ctx->C;
  const size_t n = (size_t)C.n, L = (size_t)C.L;
  // NTT tables: [L][N] pairs (w, floor(w 2^64 / q)) of psi^rev(k), then of psi^-rev(k)
  std::vector<TW> tab(2 * L * n);
  for (size_t l = 0; l < L; ++l) {
    const uint64_t q = C.limb[l].q, psi = ctx->info.psi[l], ipsi = powmod(psi, q - 2, q);
    for (size_t k = 0; k < n; ++k) {
      uint32_t e = bitrev((uint32_t)k, C.log2n);
      uint64_t w = powmod(psi, e, q), iw = powmod(ipsi, e, q);
      tab[l * n + k] = TW{w, shoup(w, q)};
      tab[L * n + l * n + k] = TW{iw, shoup(iw, q)};
    }
  }
  auto cleanup = [&](pencil_status s) {
    pencil_ctx_destroy(ctx);
    return s;
  };
  if (hipGetDevice(&ctx->device) != hipSuccess) return cleanup(fail(nullptr, PENCIL_EHIP, "no HIP device"));
  if (configure_lds_limits() != hipSuccess) return cleanup(fail(nullptr, PENCIL_EHIP, "cannot raise LDS limit"));
  if (scratch_address(ctx->device, &ctx->d_scratch) != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_EHIP, "no device address for the scratch array"));
  const size_t ln = L * n * sizeof(uint64_t);
  if (hipMalloc(&ctx->d_tables, 2 * L * n * sizeof(TW)) != hipSuccess || hipMalloc(&ctx->d_s_ntt, ln) != hipSuccess ||
      hipMalloc(&ctx->d_s_sh, ln) != hipSuccess || hipMalloc(&ctx->d_pk_ntt, 2 * ln) != hipSuccess ||
      hipMalloc(&ctx->d_pk_sh, 2 * ln) != hipSuccess || hipMalloc(&ctx->d_pk_coeff, 2 * ln) != hipSuccess ||
      hipMalloc(&ctx->d_pk_split, 2 * ln) != hipSuccess ||
      hipMalloc(&ctx->d_s_coeff, n * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&ctx->d_noise, 256) != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_ENOMEM, "device allocation failed"));
  if (hipMemcpy(ctx->d_tables, tab.data(), 2 * L * n * sizeof(TW), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_EHIP, "table upload failed"));
  ctx->T.fw = ctx->d_tables;
  ctx->T.iw = ctx->d_tables + L * n;
  // keys
  if (launch_keygen(ctx->d_s_ntt, ctx->d_s_coeff, ctx->d_pk_coeff, ctx->d_pk_ntt, C, ctx->T, nullptr) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_EHIP, "key generation failed"));
  // Shoup companions of the fixed multiplicands s^ and pk^
  std::vector<uint64_t> h(2 * L * n), hs(2 * L * n);
  if (hipMemcpy(h.data(), ctx->d_s_ntt, ln, hipMemcpyDeviceToHost) != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_EHIP, "key download failed"));
  for (size_t l = 0; l < L; ++l)
    for (size_t i = 0; i < n; ++i) hs[l * n + i] = shoup(h[l * n + i], C.limb[l].q);
  if (hipMemcpy(ctx->d_s_sh, hs.data(), ln, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.data(), ctx->d_pk_ntt, 2 * ln, hipMemcpyDeviceToHost) != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_EHIP, "key transfer failed"));
  for (size_t c = 0; c < 2; ++c)
    for (size_t l = 0; l < L; ++l)
      for (size_t i = 0; i < n; ++i) hs[(c * L + l) * n + i] = shoup(h[(c * L + l) * n + i], C.limb[l].q);
  if (hipMemcpy(ctx->d_pk_sh, hs.data(), 2 * ln, hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_EHIP, "key upload failed"));
  // pk^ split into 30-bit halves, (v mod 2^30) | (v >> 30) << 32
  for (size_t i = 0; i < 2 * L * n; ++i) hs[i] = (h[i] & 0x3FFFFFFFull) | ((h[i] >> 30) << 32);
  if (hipMemcpy(ctx->d_pk_split, hs.data(), 2 * ln, hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(nullptr, PENCIL_EHIP, "key upload failed"));
  *out = ctx;
  return PENCIL_OK;
}

extern "C" pencil_status pencil_ctx_destroy(pencil_ctx* ctx) {
  if (!ctx) return PENCIL_OK;
  hipFree(ctx->d_tables);
  hipFree(ctx->d_s_ntt);
  hipFree(ctx->d_s_sh);
  hipFree(ctx->d_pk_ntt);
  hipFree(ctx->d_pk_sh);
  hipFree(ctx->d_pk_split);
  hipFree(ctx->d_pk_coeff);
  hipFree(ctx->d_s_coeff);
  hipFree(ctx->d_noise);
  for (auto& r : ctx->pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
  delete ctx;
  return PENCIL_OK;
}

extern "C" const char* pencil_last_error(const pencil_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

extern "C" pencil_status pencil_ctx_info(const pencil_ctx* ctx, pencil_info* out) {
  if (!ctx || !out) return PENCIL_EINVAL;
  *out = ctx->info;
  out->ntt_loge = (uint32_t)ctx->C.ntt_loge;
  return PENCIL_OK;
}

extern "C" pencil_status pencil_export_keys(const pencil_ctx* ctx, int64_t* sk, uint64_t* pk) {
  if (!ctx) return PENCIL_EINVAL;
  pencil_ctx* c = const_cast<pencil_ctx*>(ctx);
  const size_t n = (size_t)ctx->C.n, L = (size_t)ctx->C.L;
  if (sk) HIP_TRY(c, hipMemcpy(sk, ctx->d_s_coeff, n * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (pk) HIP_TRY(c, hipMemcpy(pk, ctx->d_pk_coeff, 2 * L * n * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return PENCIL_OK;
}

// ------------------------------------------------------------ geometry

struct OpGeom {
  int M, R, K, HA, WA, KH, KW;
  int OH() const { return HA - KH + 1; }
  int OW() const { return WA - KW + 1; }
};

// Kernel extent and zero padding per axis.  A Conv1d (kind 2) is the one-row
// case of a Conv2d: a 1 x k kernel, padding along the length only.
static int kh_of(const pencil_layer* L) { return L->kind == 2 ? 1 : L->k; }
static int kw_of(const pencil_layer* L) { return L->k; }
static int ph_of(const pencil_layer* L) { return L->kind == 2 ? 0 : L->pad; }
static int pw_of(const pencil_layer* L) { return L->pad; }
// Output rows and columns of a stride-1 layer.
static int ho_of(const pencil_layer* L) { return L->h + 2 * ph_of(L) - kh_of(L) + 1; }
static int wo_of(const pencil_layer* L) { return L->w + 2 * pw_of(L) - kw_of(L) + 1; }

// Shape checks shared by every entry point; strided layers pass only where
// allow_stride is set (the stride map and its relayouts).
static bool layer_shape_ok(pencil_ctx* ctx, const pencil_layer* L, bool allow_stride, pencil_status* st) {
  if (!L) {
    *st = fail(ctx, PENCIL_EINVAL, "layer is NULL");
    return false;
  }
  if (L->kind < 0 || L->kind > 2) {
    *st = fail(ctx, PENCIL_EINVAL, "layer kind must be 0 (fc), 1 (conv2d) or 2 (conv1d)");
    return false;
  }
  if (L->batch < 1 || L->c_in < 1 || L->c_out < 1 || L->h < 1 || L->w < 1 || L->k < 1 || L->pad < 0 ||
      L->stride < 0) {
    *st = fail(ctx, PENCIL_EINVAL, "layer dimensions must be positive");
    return false;
  }
  const int stride = L->stride == 0 ? 1 : L->stride;
  if (L->kind == 0 && (L->h != 1 || L->w != 1 || L->k != 1 || L->pad != 0 || stride != 1)) {
    *st = fail(ctx, PENCIL_EINVAL, "fc layers need h = w = k = 1, pad = 0, stride 1");
    return false;
  }
  if (L->kind == 2 && L->h != 1) {
    *st = fail(ctx, PENCIL_EINVAL, "conv1d layers need h = 1");
    return false;
  }
  if (stride > 1 && !allow_stride) {
    *st = fail(ctx, PENCIL_EUNSUPPORTED,
               "stride %d: run the layer as its stride-1 equivalent (pencil_stride_map, pencil_stride_relayout)",
               stride);
    return false;
  }
  if (stride > 16) {
    *st = fail(ctx, PENCIL_EUNSUPPORTED, "stride above 16 is not supported");
    return false;
  }
  if (L->pad > L->k - 1) {
    *st = fail(ctx, PENCIL_EUNSUPPORTED, "padding above k - 1 is not supported");
    return false;
  }
  if (L->h + 2 * ph_of(L) < kh_of(L) || L->w + 2 * pw_of(L) < kw_of(L)) {
    *st = fail(ctx, PENCIL_EINVAL, "kernel larger than padded input");
    return false;
  }
  const int64_t big = (int64_t)1 << 31;
  if ((int64_t)L->batch * L->c_in * L->h * L->w >= big ||
      (int64_t)L->c_out * L->c_in * kh_of(L) * kw_of(L) * stride * stride >= big) {
    *st = fail(ctx, PENCIL_EINVAL, "layer too large");
    return false;
  }
  return true;
}

static bool layer_ok(pencil_ctx* ctx, const pencil_layer* L, pencil_status* st) {
  return layer_shape_ok(ctx, L, false, st);
}

static OpGeom op_geom(const pencil_layer* L, int op) {
  const int kh = kh_of(L), kw = kw_of(L), ph = ph_of(L), pw = pw_of(L);
  const int ho = ho_of(L), wo = wo_of(L);
  const int qh = kh - 1 - ph, qw = kw - 1 - pw;
  switch (op) {
    case PENCIL_OP_FWD: return {L->batch, L->c_out, L->c_in, L->h + 2 * ph, L->w + 2 * pw, kh, kw};
    case PENCIL_OP_DX: return {L->batch, L->c_in, L->c_out, ho + 2 * qh, wo + 2 * qw, kh, kw};
    default: return {L->c_in, L->c_out, L->batch, L->h + 2 * ph, L->w + 2 * pw, ho, wo};
  }
}

static int cdiv(int a, int b) { return (a + b - 1) / b; }

static bool make_geo(const OpGeom& g, const pencil_tile& t, int n, Geo* G) {
  if (t.m < 1 || t.r < 1 || t.k < 1 || t.oh < 1 || t.ow < 1 || t.kh < 1 || t.kw < 1) return false;
  if (t.m > g.M || t.r > g.R || t.k > g.K || t.oh > g.OH() || t.ow > g.OW() || t.kh > g.KH || t.kw > g.KW)
    return false;
  const int64_t ha = t.oh + t.kh - 1, wa = t.ow + t.kw - 1;
  if ((int64_t)t.m * t.r * t.k * ha * wa > n) return false;
  Geo& o = *G;
  o = Geo{};
  o.M = g.M; o.R = g.R; o.K = g.K; o.HA = g.HA; o.WA = g.WA; o.KH = g.KH; o.KW = g.KW;
  o.OH = g.OH(); o.OW = g.OW();
  o.mt = t.m; o.rt = t.r; o.kt = t.k; o.oh = t.oh; o.ow = t.ow; o.kh = t.kh; o.kw = t.kw;
  o.ha = (int)ha; o.wa = (int)wa;
  o.nM = cdiv(g.M, t.m); o.nR = cdiv(g.R, t.r); o.nK = cdiv(g.K, t.k);
  o.nOY = cdiv(o.OH, t.oh); o.nOX = cdiv(o.OW, t.ow); o.nKY = cdiv(g.KH, t.kh); o.nKX = cdiv(g.KW, t.kw);
  o.S = t.k * o.ha * o.wa;
  o.RS = t.r * o.S;
  o.O = (t.k - 1) * o.ha * o.wa + (t.kh - 1) * o.wa + t.kw - 1;
  // n / d for n, d < 2^16 (slots and in-tile offsets; n <= 16384 here)
  auto recip = [](int64_t d) { return d <= 1 ? 0u : (uint32_t)(0xFFFFFFFFull / (uint64_t)d + 1); };
  o.dv_rs = recip(o.RS);
  o.dv_hw = recip((int64_t)o.ha * o.wa);
  o.dv_wa = recip(o.wa);
  o.dv_s = recip(o.S);
  o.dv_kw = recip(o.kw);
  o.dv_khw = recip((int64_t)o.kh * o.kw);
  o.dv_kthw = recip((int64_t)o.kt * o.kh * o.kw);
  return true;
}

static int64_t n_a_tiles(const Geo& G) { return (int64_t)G.nM * G.nK * G.nOY * G.nOX * G.nKY * G.nKX; }
static int64_t n_k_tiles(const Geo& G) { return (int64_t)G.nR * G.nK * G.nKY * G.nKX; }
static int64_t n_out_tiles(const Geo& G) { return (int64_t)G.nM * G.nR * G.nOY * G.nOX; }
static int64_t n_products(const Geo& G) { return n_out_tiles(G) * G.nK * G.nKY * G.nKX; }

// Tensor views (strides into the caller's PyTorch-layout tensors).
static View view_a(const pencil_layer* L, int op) {
  const int64_t h = L->h, w = L->w, ci = L->c_in, co = L->c_out;
  const int64_t ho = ho_of(L), wo = wo_of(L);
  View v{};
  v.sx = 1;
  if (op == PENCIL_OP_FWD) {  // x [B][ci][h][w], (m, k) = (b, ci)
    v.s0 = ci * h * w; v.s1 = h * w; v.sy = w; v.pady = ph_of(L); v.pad = pw_of(L); v.H = (int)h; v.W = (int)w;
  } else if (op == PENCIL_OP_DX) {  // dy [B][co][ho][wo], (m, k) = (b, co)
    v.s0 = co * ho * wo; v.s1 = ho * wo; v.sy = wo; v.pady = kh_of(L) - 1 - ph_of(L); v.pad = kw_of(L) - 1 - pw_of(L);
    v.H = (int)ho; v.W = (int)wo;
  } else {  // x viewed (ci, B): (m, k) = (ci, b)
    v.s0 = h * w; v.s1 = ci * h * w; v.sy = w; v.pady = ph_of(L); v.pad = pw_of(L); v.H = (int)h; v.W = (int)w;
  }
  return v;
}

static View view_k(const pencil_layer* L, int op) {
  const int64_t kh = kh_of(L), kw = kw_of(L), ci = L->c_in, co = L->c_out;
  const int64_t ho = ho_of(L), wo = wo_of(L);
  View v{};
  v.sx = 1;
  if (op == PENCIL_OP_FWD) {  // W [co][ci][kh][kw], (r, k) = (co, ci)
    v.s0 = ci * kh * kw; v.s1 = kh * kw; v.sy = kw;
  } else if (op == PENCIL_OP_DX) {  // W viewed (ci, co), flipped
    v.s0 = kh * kw; v.s1 = ci * kh * kw; v.sy = kw; v.flip = 1; v.KH = (int)kh; v.KW = (int)kw;
  } else {  // dy viewed (co, B): (r, k) = (co, b)
    v.s0 = ho * wo; v.s1 = co * ho * wo; v.sy = wo;
  }
  return v;
}

static View view_out(const pencil_layer* L, int op) {
  const int64_t h = L->h, w = L->w, kh = kh_of(L), kw = kw_of(L), ci = L->c_in, co = L->c_out;
  const int64_t ho = ho_of(L), wo = wo_of(L);
  View v{};
  v.sx = 1;
  if (op == PENCIL_OP_FWD) {  // Y [B][co][ho][wo]
    v.s0 = co * ho * wo; v.s1 = ho * wo; v.sy = wo;
  } else if (op == PENCIL_OP_DX) {  // dX [B][ci][h][w]
    v.s0 = ci * h * w; v.s1 = h * w; v.sy = w;
  } else {  // dW [co][ci][kh][kw] with (m, r) = (ci, co)
    v.s0 = kh * kw; v.s1 = ci * kh * kw; v.sy = kw;
  }
  return v;
}

static const pencil_tile& plan_tile(const pencil_plan* P, int op) {
  return op == PENCIL_OP_FWD ? P->fwd : op == PENCIL_OP_DX ? P->dx : P->dw;
}

static pencil_status get_geo(pencil_ctx* ctx, const pencil_layer* L, const pencil_plan* P, int op, Geo* G) {
  pencil_status st = PENCIL_OK;
  if (!layer_ok(ctx, L, &st)) return st;
  if (!P) return fail(ctx, PENCIL_EINVAL, "plan is NULL");
  const pencil_tile& t = plan_tile(P, op);
  if (!make_geo(op_geom(L, op), t, ctx->C.n, G))
    return fail(ctx, PENCIL_EINVAL, "op %d: tile (%d,%d,%d,%d,%d,%d,%d) is invalid or exceeds N=%d slots", op, t.m,
                t.r, t.k, t.oh, t.ow, t.kh, t.kw, ctx->C.n);
  if (n_out_tiles(*G) > (1ll << 40) || n_a_tiles(*G) > (1ll << 40)) return fail(ctx, PENCIL_EINVAL, "too many tiles");
  return PENCIL_OK;
}

// ------------------------------------------------------------ planner

// Work model, in units of one pointwise product-accumulate of one residue.
// An NTT of one limb-polynomial costs (N/2) log2 N butterflies of ~1.4 units
// each, a product 2 components per limb; both weights are calibrated on
// MI355X step-kernel times (N = 8192: ~88 ns per limb transform, ~19 ns per
// limb product).  Input ciphertexts arrive in the NTT domain, split, and are
// read in place: the MO transforms only its share for the fwd and dx operands
// and stages component 0 with it added (the copy costing ~0.36 of a
// transform).
struct Cost {
  double ntt_polys, products;
};

static Cost op_cost(const Geo& G, int op) {
  Cost c{};
  const double na = (double)n_a_tiles(G), nk = (double)n_k_tiles(G), no = (double)n_out_tiles(G);
  constexpr double kCopy = 0.36;
  if (op == PENCIL_OP_DW) {
    // x0 pt, dy0 pt (the ciphertexts are read in place), outputs (2 inverse) + u'
    c.ntt_polys = na + nk + 3 * no;
    c.products = 2.0 * (double)n_products(G);
  } else {
    // ct: share transform with the staged copy of component 0; pt; outputs + u'
    c.ntt_polys = na * (1 + kCopy) + nk + 3 * no;
    c.products = (double)n_products(G);
  }
  return c;
}

static double cost_value(const Cost& c, int log2n) {
  const double n = (double)(1 << log2n);
  return c.ntt_polys * (n / 2) * log2n * 1.4 + c.products * 2 * n;
}

// Candidate tile sizes along a dimension of extent D: the smallest size for each
// distinct tile count.
static std::vector<int> sizes_for(int D) {
  std::vector<int> out;
  int last = -1;
  for (int cnt = 1; cnt <= D; ++cnt) {
    int s = cdiv(D, cnt);
    if (s != last) {
      out.push_back(s);
      last = s;
    }
  }
  return out;
}

// The packing planner: every partition that fits N (per dimension, the
// smallest tile size for each tile count), ranked by the cost model; `best`
// receives the cheapest, `ranked` (optional) the cheapest `keep` in order.
static bool plan_op(const pencil_layer* L, int op, int log2n, pencil_tile* best,
                    std::vector<pencil_tile>* ranked = nullptr, size_t keep = 0) {
  const OpGeom g = op_geom(L, op);
  const int n = 1 << log2n;
  double best_cost = 1e300;
  bool found = false;
  std::vector<std::pair<double, pencil_tile>> all;
  const bool kernel_tiled = op == PENCIL_OP_DW && g.KH > 1;
  std::vector<int> ms = sizes_for(g.M), rs = sizes_for(g.R);
  std::vector<int> ys = kernel_tiled ? sizes_for(g.KH) : sizes_for(g.OH());
  std::vector<int> xs = kernel_tiled ? sizes_for(g.KW) : sizes_for(g.OW());
  for (int ty : ys)
    for (int tx : xs) {
      pencil_tile t{};
      if (kernel_tiled) {
        t.oh = g.OH(); t.ow = g.OW(); t.kh = ty; t.kw = tx;
      } else {
        t.oh = ty; t.ow = tx; t.kh = g.KH; t.kw = g.KW;
      }
      const int64_t hw = (int64_t)(t.oh + t.kh - 1) * (t.ow + t.kw - 1);
      if (hw > n) continue;
      for (int m : ms)
        for (int r : rs) {
          int64_t room = n / (hw * m * r);
          if (room < 1) continue;
          int k = (int)std::min<int64_t>(room, g.K);
          k = cdiv(g.K, cdiv(g.K, k));
          t.m = m; t.r = r; t.k = k;
          Geo G;
          if (!make_geo(g, t, n, &G)) continue;
          double cv = cost_value(op_cost(G, op), log2n);
          if (ranked) all.emplace_back(cv, t);
          if (cv < best_cost) {
            best_cost = cv;
            *best = t;
            found = true;
          }
        }
    }
  if (ranked) {
    std::stable_sort(all.begin(), all.end(),
                     [](const std::pair<double, pencil_tile>& a, const std::pair<double, pencil_tile>& b) {
                       return a.first < b.first;
                     });
    ranked->clear();
    for (size_t i = 0; i < all.size() && ranked->size() < keep; ++i) ranked->push_back(all[i].second);
  }
  return found;
}

// Default multiply-accumulate schedule: direct loads with 2 x 2 wave blocks
// (variants 3-5), in the chunk shape that loads the fewest padded operand rows
// per contraction step (A rows count twice: two components).
static int default_sched(const pencil_layer* L, int op, const pencil_tile& t, int n) {
  Geo G;
  if (!make_geo(op_geom(L, op), t, n, &G)) return 3;
  const int rows = G.nM * G.nOY * G.nOX;
  int best = 3;
  int64_t best_v = -1;
  for (int v = 3; v < 6; ++v) {
    const int64_t rc = (rows + mac_rows(v) - 1) / mac_rows(v), cc = (G.nR + mac_cols(v) - 1) / mac_cols(v);
    const int64_t vol = rc * cc * (2 * mac_rows(v) + mac_cols(v));
    if (best_v < 0 || vol < best_v) {
      best_v = vol;
      best = v;
    }
  }
  return best;
}

extern "C" pencil_status pencil_plan_auto(const pencil_ctx* cctx, const pencil_layer* L, pencil_plan* plan) {
  pencil_ctx* ctx = const_cast<pencil_ctx*>(cctx);
  if (!ctx || !plan) return PENCIL_EINVAL;
  pencil_status st = PENCIL_OK;
  if (!layer_ok(ctx, L, &st)) return st;
  pencil_tile* tiles[3] = {&plan->fwd, &plan->dx, &plan->dw};
  for (int op = 0; op < 3; ++op) {
    if (!plan_op(L, op, ctx->C.log2n, tiles[op]))
      return fail(ctx, PENCIL_EUNSUPPORTED, "no tile of op %d fits N = %d", op, ctx->C.n);
    plan->sched[op] = default_sched(L, op, *tiles[op], ctx->C.n);
  }
  return PENCIL_OK;
}

extern "C" pencil_status pencil_layout(const pencil_ctx* cctx, const pencil_layer* L, const pencil_plan* P,
                                       pencil_sizes* out) {
  pencil_ctx* ctx = const_cast<pencil_ctx*>(cctx);
  if (!ctx || !out) return PENCIL_EINVAL;
  if (!P) return fail(ctx, PENCIL_EINVAL, "plan is NULL");
  // An op whose tile is all zero is not planned: its sizes are reported as 0.
  Geo G[3];
  bool used[3];
  for (int op = 0; op < 3; ++op) {
    const pencil_tile& t = plan_tile(P, op);
    used[op] = !(t.m == 0 && t.r == 0 && t.k == 0 && t.oh == 0 && t.ow == 0 && t.kh == 0 && t.kw == 0);
    if (!used[op]) {
      pencil_status st = PENCIL_OK;
      if (!layer_ok(ctx, L, &st)) return st;
      continue;
    }
    pencil_status st = get_geo(ctx, L, P, op, &G[op]);
    if (st != PENCIL_OK) return st;
  }
  const uint64_t n = (uint64_t)ctx->C.n, Ln = (uint64_t)ctx->C.L;
  const uint64_t poly = Ln * n * 8, ct = 2 * poly;
  std::memset(out, 0, sizeof *out);
  out->ct_bytes = ct;
  if (used[0]) out->n_ct[PENCIL_X_FWD] = (uint64_t)n_a_tiles(G[0]);
  if (used[1]) out->n_ct[PENCIL_DY_DX] = (uint64_t)n_a_tiles(G[1]);
  if (used[2]) {
    out->n_ct[PENCIL_X_DW] = (uint64_t)n_a_tiles(G[2]);
    out->n_ct[PENCIL_DY_DW] = (uint64_t)n_k_tiles(G[2]);
  }
  for (int op = 0; op < 3; ++op) {
    if (!used[op]) continue;
    out->n_out[op] = (uint64_t)n_out_tiles(G[op]);
    out->n_products[op] = (uint64_t)n_products(G[op]) * (op == PENCIL_OP_DW ? 2 : 1);
    out->n_pt[op] = (uint64_t)n_k_tiles(G[op]) + (op == PENCIL_OP_DW ? (uint64_t)n_a_tiles(G[op]) : 0);
  }
  // fwd: A cts (NTT) + W pts + u' per output
  out->ws_fwd_bytes = out->n_ct[0] * ct + out->n_pt[0] * poly + out->n_out[0] * poly;
  const uint64_t dx = out->n_ct[1] * ct + out->n_pt[1] * poly + out->n_out[1] * poly;
  const uint64_t dw = out->n_ct[2] * ct + out->n_ct[3] * ct + out->n_pt[2] * poly + out->n_out[2] * poly;
  out->ws_bwd_bytes = std::max(dx, dw);
  out->ws_dec_bytes = std::max(out->n_out[0], std::max(out->n_out[1], out->n_out[2])) * poly;
  uint64_t enc = 0;
  for (int k = 0; k < 4; ++k) enc = std::max(enc, out->n_ct[k]);
  out->ws_enc_bytes = enc * poly;
  return PENCIL_OK;
}

// ------------------------------------------------------------ operations

static pencil_status check_ptr(pencil_ctx* ctx, const void* p, const char* name) {
  if (!p) return fail(ctx, PENCIL_EINVAL, "%s is NULL", name);
  return PENCIL_OK;
}

// Ciphertext, polynomial and workspace buffers: non-NULL and 16-byte aligned
// (the transforms move residues in 16-byte pairs).
static pencil_status check_buf(pencil_ctx* ctx, const void* p, const char* name) {
  if (!p) return fail(ctx, PENCIL_EINVAL, "%s is NULL", name);
  if (((uintptr_t)p & 15) != 0) return fail(ctx, PENCIL_EINVAL, "%s is not 16-byte aligned", name);
  return PENCIL_OK;
}

#define TRY(x)                          \
  do {                                  \
    pencil_status _s = (x);             \
    if (_s != PENCIL_OK) return _s;     \
  } while (0)

extern "C" pencil_status pencil_encrypt(pencil_ctx* ctx, const pencil_layer* L, const pencil_plan* P, int operand,
                                        const int64_t* share, uint64_t* ct, void* ws, uint64_t nonce, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (operand < 0 || operand > 3) return fail(ctx, PENCIL_EINVAL, "operand %d invalid", operand);
  TRY(check_ptr(ctx, share, "share"));
  TRY(check_buf(ctx, ct, "ct"));
  TRY(check_buf(ctx, ws, "ws"));
  const int op = operand == PENCIL_X_FWD ? PENCIL_OP_FWD : operand == PENCIL_DY_DX ? PENCIL_OP_DX : PENCIL_OP_DW;
  const int side = operand == PENCIL_DY_DW ? 1 : 0;
  Geo G;
  TRY(get_geo(ctx, L, P, op, &G));
  const View V = side ? view_k(L, op) : view_a(L, op);
  const int64_t count = side ? n_k_tiles(G) : n_a_tiles(G);
  hipStream_t s = (hipStream_t)stream;
  uint64_t* u = (uint64_t*)ws;  // u^ of every ciphertext, [count][L][N]
  hipError_t e = timed(ctx, KID_NTT_TERNARY, s, [&] { return launch_ntt_ternary(u, count, nonce, enc_object(operand, 0), P_ENC_U, 0, ctx->C, ctx->T, s); });
  if (e == hipSuccess)
    e = timed(ctx, KID_ENCRYPT, s, [&] {
      return launch_encrypt(u, share, ct, count, side, G, V, ctx->d_pk_ntt, ctx->d_pk_sh, nonce,
                            enc_object(operand, 0), ctx->C, ctx->T, s);
    });
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "encrypt launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

// Element offset from a staged component-0 copy to component 1 of the same
// ciphertext in the caller's buffer (both 8-byte aligned device addresses).
static int64_t comp1_offset(const uint64_t* staged, const uint64_t* caller, int64_t poly) {
  return ((int64_t)(uintptr_t)caller - (int64_t)(uintptr_t)staged) / (int64_t)sizeof(uint64_t) + poly;
}

// One product: NTT of the inputs, MAC (+ pk u'), INTT, flood and mask.
struct TermIn {
  const uint64_t* ct;     // coefficient-domain ciphertexts (A side if a_is_ct)
  const int64_t* pt;      // Z_t tensor for the plaintext side
  int a_is_ct;
};

static pencil_status run_product(pencil_ctx* ctx, const pencil_layer* L, int op, const Geo& G, const TermIn* terms,
                                 int n_terms, const int64_t* add_share, const int64_t* bias, uint64_t* ct_out,
                                 int64_t* share_out, uint8_t* ws, uint64_t nonce, int sched, hipStream_t s,
                                 bool allow_events = true) {
  if (sched < 0 || sched >= kMacVariants) return fail(ctx, PENCIL_EINVAL, "schedule variant %d invalid", sched);
  // kernel timing records events only where the caller allows it
  auto timed = [&](pencil_ctx* c, int kid, hipStream_t st, auto&& launch) -> hipError_t {
    return allow_events ? ::timed(c, kid, st, launch) : launch();
  };
  const Consts& C = ctx->C;
  const int64_t poly = (int64_t)C.L * C.n, ctw = 2 * poly;
  const int64_t na = n_a_tiles(G), nk = n_k_tiles(G), no = n_out_tiles(G);
  uint64_t* w = (uint64_t*)ws;
  MacArgs A{};
  A.n_terms = n_terms;
  A.m_rows = G.nM * G.nOY * G.nOX;
  A.variant = sched;
  A.pk = ctx->d_pk_split;
  A.out = ct_out;
  for (int i = 0; i < n_terms; ++i) {
    const TermIn& T = terms[i];
    if (T.a_is_ct) {
      // the caller's ciphertexts are read in place; with a share to add,
      // component 0 is staged (share added) and component 1 stays in place
      uint64_t* cts = w;
      w += na * ctw;
      uint64_t* pts = w;
      w += nk * poly;
      hipError_t e = hipSuccess;
      MacTerm mt{T.ct, pts, poly, 1, 0};
      if (add_share) {
        e = timed(ctx, KID_NTT_CT, s, [&] { return launch_ntt_ct(T.ct, cts, na, add_share, G, view_a(L, op), C, ctx->T, s); });
        mt.a = cts;
        mt.c1 = comp1_offset(cts, T.ct, poly);
      }
      if (e == hipSuccess)
        e = timed(ctx, KID_NTT_PT, s, [&] { return launch_ntt_pt(T.pt, pts, nk, 1, G, view_k(L, op), C, ctx->T, s); });
      if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "ntt launch: %s", hipGetErrorString(e));
      A.term[i] = mt;
    } else {
      uint64_t* pts = w;
      w += na * poly;
      w += nk * ctw;
      hipError_t e = timed(ctx, KID_NTT_PT, s, [&] { return launch_ntt_pt(T.pt, pts, na, 0, G, view_a(L, op), C, ctx->T, s); });
      if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "ntt launch: %s", hipGetErrorString(e));
      A.term[i] = MacTerm{pts, T.ct, poly, 0, 0};
    }
  }
  uint64_t* u = w;
  const uint64_t obj = out_object(op, 0);
  hipError_t e = timed(ctx, KID_NTT_TERNARY, s, [&] { return launch_ntt_ternary(u, no, nonce, obj, P_RR_U, 1, C, ctx->T, s); });
  A.u = u;
  if (e == hipSuccess) e = timed(ctx, KID_MAC, s, [&] { return launch_mac(A, no, G, C, s); });
  if (e == hipSuccess) e = timed(ctx, KID_INTT_OUT, s, [&] { return launch_ntt_plain(ct_out, 2 * no, true, C, ctx->T, s); });
  if (e == hipSuccess)
    e = timed(ctx, KID_FLOOD, s, [&] {
      return launch_flood_mask(ct_out, no, share_out, bias, G, view_out(L, op), nonce, obj, C, s);
    });
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "product launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

static bool mac_grid_ok(const Geo& G) {
  const int64_t rows = (int64_t)G.nM * G.nOY * G.nOX;
  return (int64_t)mac_chunks(1, (int)rows, G.nR) < 65536 && (int64_t)mac_chunks(2, (int)rows, G.nR) < 65536;
}

extern "C" pencil_status pencil_linear_fwd(pencil_ctx* ctx, const pencil_layer* L, const pencil_plan* P,
                                           const uint64_t* ct_x1, const int64_t* x0, const int64_t* w,
                                           const int64_t* bias, uint64_t* ct_y, int64_t* y0, void* ws,
                                           uint64_t nonce, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  TRY(check_buf(ctx, ct_x1, "ct_x1"));
  TRY(check_ptr(ctx, x0, "x0"));
  TRY(check_ptr(ctx, w, "w"));
  TRY(check_buf(ctx, ct_y, "ct_y"));
  TRY(check_ptr(ctx, y0, "y0"));
  TRY(check_buf(ctx, ws, "ws"));
  Geo G;
  TRY(get_geo(ctx, L, P, PENCIL_OP_FWD, &G));
  if (!mac_grid_ok(G)) return fail(ctx, PENCIL_EUNSUPPORTED, "too many output tiles for one launch");
  TermIn t{ct_x1, w, 1};
  return run_product(ctx, L, PENCIL_OP_FWD, G, &t, 1, x0, bias, ct_y, y0, (uint8_t*)ws, nonce, P->sched[0],
                     (hipStream_t)stream);
}

extern "C" pencil_status pencil_linear_fwd_noalloc(pencil_ctx* ctx, const pencil_layer* L, const pencil_plan* P,
                                                   const uint64_t* ct_x1, const int64_t* x0, const int64_t* w,
                                                   const int64_t* bias, uint64_t* ct_y, int64_t* y0, uint64_t nonce,
                                                   void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  TRY(check_buf(ctx, ct_x1, "ct_x1"));
  TRY(check_ptr(ctx, x0, "x0"));
  TRY(check_ptr(ctx, w, "w"));
  TRY(check_buf(ctx, ct_y, "ct_y"));
  TRY(check_ptr(ctx, y0, "y0"));
  if (!ctx->d_scratch) return fail(ctx, PENCIL_EHIP, "the library's scratch array has no device address");
  Geo G;
  TRY(get_geo(ctx, L, P, PENCIL_OP_FWD, &G));
  if (!mac_grid_ok(G)) return fail(ctx, PENCIL_EUNSUPPORTED, "too many output tiles for one launch");
  pencil_sizes sz;
  TRY(pencil_layout(ctx, L, P, &sz));
  if (sz.ws_fwd_bytes > kScratchBytes)
    return fail(ctx, PENCIL_EUNSUPPORTED,
                "the forward product needs %llu bytes of workspace; the allocation-free entry point has %llu",
                (unsigned long long)sz.ws_fwd_bytes, (unsigned long long)kScratchBytes);
  TermIn t{ct_x1, w, 1};
  return run_product(ctx, L, PENCIL_OP_FWD, G, &t, 1, x0, bias, ct_y, y0, (uint8_t*)ctx->d_scratch, nonce,
                     P->sched[0], (hipStream_t)stream, false);
}

extern "C" pencil_status pencil_linear_bwd(pencil_ctx* ctx, const pencil_layer* L, const pencil_plan* P,
                                           const uint64_t* ct_dy_dx, const uint64_t* ct_x_dw,
                                           const uint64_t* ct_dy_dw, const int64_t* dy0, const int64_t* x0,
                                           const int64_t* w, uint64_t* ct_dx, int64_t* dx0, uint64_t* ct_dw,
                                           int64_t* dw_mask, void* ws, uint64_t nonce, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  TRY(check_buf(ctx, ws, "ws"));
  TRY(check_ptr(ctx, dy0, "dy0"));
  hipStream_t s = (hipStream_t)stream;
  if (ct_dx || dx0) {
    TRY(check_buf(ctx, ct_dy_dx, "ct_dy_dx"));
    TRY(check_ptr(ctx, w, "w"));
    TRY(check_buf(ctx, ct_dx, "ct_dx"));
    TRY(check_ptr(ctx, dx0, "dx0"));
    Geo G;
    TRY(get_geo(ctx, L, P, PENCIL_OP_DX, &G));
    if (!mac_grid_ok(G)) return fail(ctx, PENCIL_EUNSUPPORTED, "too many output tiles for one launch");
    TermIn t{ct_dy_dx, w, 1};
    TRY(run_product(ctx, L, PENCIL_OP_DX, G, &t, 1, dy0, nullptr, ct_dx, dx0, (uint8_t*)ws, nonce, P->sched[1], s));
  }
  if (ct_dw || dw_mask) {
    TRY(check_buf(ctx, ct_x_dw, "ct_x_dw"));
    TRY(check_buf(ctx, ct_dy_dw, "ct_dy_dw"));
    TRY(check_ptr(ctx, x0, "x0"));
    TRY(check_buf(ctx, ct_dw, "ct_dw"));
    TRY(check_ptr(ctx, dw_mask, "dw_mask"));
    Geo G;
    TRY(get_geo(ctx, L, P, PENCIL_OP_DW, &G));
    if (!mac_grid_ok(G)) return fail(ctx, PENCIL_EUNSUPPORTED, "too many output tiles for one launch");
    TermIn t[2] = {{ct_x_dw, dy0, 1}, {ct_dy_dw, x0, 0}};
    TRY(run_product(ctx, L, PENCIL_OP_DW, G, t, 2, nullptr, nullptr, ct_dw, dw_mask, (uint8_t*)ws, nonce, P->sched[2],
                    s));
  }
  return PENCIL_OK;
}

extern "C" pencil_status pencil_decrypt(pencil_ctx* ctx, const pencil_layer* L, const pencil_plan* P, int op,
                                        const uint64_t* ct, int64_t* share, void* ws, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (op < 0 || op > 2) return fail(ctx, PENCIL_EINVAL, "op %d invalid", op);
  TRY(check_buf(ctx, ct, "ct"));
  TRY(check_ptr(ctx, share, "share"));
  TRY(check_buf(ctx, ws, "ws"));
  Geo G;
  TRY(get_geo(ctx, L, P, op, &G));
  const int64_t no = n_out_tiles(G);
  hipStream_t s = (hipStream_t)stream;
  uint64_t* x = (uint64_t*)ws;
  hipError_t e = timed(ctx, KID_PHASE, s, [&] { return launch_phase(ct, x, no, ctx->d_s_ntt, ctx->d_s_sh, ctx->C, ctx->T, s); });
  if (e == hipSuccess)
    e = timed(ctx, KID_DECODE, s, [&] { return launch_decode(x, share, no, G, view_out(L, op), ctx->C, nullptr, s); });
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "decrypt launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_decrypt_checked(pencil_ctx* ctx, const pencil_layer* L, const pencil_plan* P, int op,
                                                const uint64_t* ct, int64_t* share, void* ws, double* noise_frac,
                                                void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (op < 0 || op > 2) return fail(ctx, PENCIL_EINVAL, "op %d invalid", op);
  TRY(check_buf(ctx, ct, "ct"));
  TRY(check_ptr(ctx, share, "share"));
  TRY(check_buf(ctx, ws, "ws"));
  Geo G;
  TRY(get_geo(ctx, L, P, op, &G));
  const int64_t no = n_out_tiles(G);
  hipStream_t s = (hipStream_t)stream;
  uint64_t* x = (uint64_t*)ws;
  uint32_t* nz = (uint32_t*)ctx->d_noise;
  hipError_t e = launch_set_u64(ctx->d_noise, 0, 0, s);  // a fill kernel, not a memset node
  if (e == hipSuccess)
    e = timed(ctx, KID_PHASE, s, [&] { return launch_phase(ct, x, no, ctx->d_s_ntt, ctx->d_s_sh, ctx->C, ctx->T, s); });
  if (e == hipSuccess)
    e = timed(ctx, KID_DECODE, s, [&] { return launch_decode(x, share, no, G, view_out(L, op), ctx->C, nz, s); });
  uint32_t bits = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bits, nz, sizeof bits, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "checked decrypt: %s", hipGetErrorString(e));
  float frac;
  std::memcpy(&frac, &bits, sizeof frac);
  if (noise_frac) *noise_frac = frac;
  if (frac >= 0.25f)
    return fail(ctx, PENCIL_ENOISE, "decryption noise reaches %.3f of q/t (limit 0.25): the result is unreliable",
                (double)frac);
  return PENCIL_OK;
}

extern "C" pencil_status pencil_ntt_forward(pencil_ctx* ctx, uint64_t* polys, int64_t count, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  TRY(check_buf(ctx, polys, "polys"));
  if (count < 0) return fail(ctx, PENCIL_EINVAL, "count < 0");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = timed(ctx, KID_NTT_PLAIN, s, [&] { return launch_ntt_plain(polys, count, false, ctx->C, ctx->T, s); });
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "ntt launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_ntt_inverse(pencil_ctx* ctx, uint64_t* polys, int64_t count, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  TRY(check_buf(ctx, polys, "polys"));
  if (count < 0) return fail(ctx, PENCIL_EINVAL, "count < 0");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = timed(ctx, KID_NTT_PLAIN, s, [&] { return launch_ntt_plain(polys, count, true, ctx->C, ctx->T, s); });
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "ntt launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_zt_linear(pencil_ctx* ctx, const pencil_layer* L, int op, const int64_t* a,
                                          const int64_t* b, int64_t* out, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (op < 0 || op > 2) return fail(ctx, PENCIL_EINVAL, "op %d invalid", op);
  TRY(check_ptr(ctx, a, "a"));
  TRY(check_ptr(ctx, b, "b"));
  TRY(check_ptr(ctx, out, "out"));
  pencil_status st = PENCIL_OK;
  if (!layer_ok(ctx, L, &st)) return st;
  const OpGeom g = op_geom(L, op);
  // the whole operand as one tile: only the virtual dimensions are used
  Geo G{};
  G.M = g.M; G.R = g.R; G.K = g.K; G.HA = g.HA; G.WA = g.WA; G.KH = g.KH; G.KW = g.KW;
  G.OH = g.OH(); G.OW = g.OW();
  hipError_t e = launch_zt_corr(a, b, out, G, view_a(L, op), view_k(L, op), view_out(L, op), ctx->C,
                                (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "zt_linear launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

// A signed coefficient as a residue mod t.
static uint64_t coeff_mod_t(int64_t c, uint64_t t) {
  const int64_t r = c % (int64_t)t;
  return (uint64_t)(r < 0 ? r + (int64_t)t : r);
}

static pencil_status zt_combine_reduced(pencil_ctx* ctx, int64_t count, int n_terms, const int64_t* const* terms,
                                        const uint64_t* coeffs, const int64_t* base, int64_t* out, void* stream);

extern "C" pencil_status pencil_zt_combine(pencil_ctx* ctx, int64_t count, int n_terms, const int64_t* const* terms,
                                           const int64_t* coeffs, const int64_t* base, int64_t* out, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (count < 0 || n_terms < 0) return fail(ctx, PENCIL_EINVAL, "negative count or term count");
  if (n_terms > 0 && (!terms || !coeffs)) return fail(ctx, PENCIL_EINVAL, "terms or coeffs is NULL");
  std::vector<uint64_t> c(n_terms);
  for (int i = 0; i < n_terms; ++i) c[i] = coeff_mod_t(coeffs[i], ctx->C.t);
  return zt_combine_reduced(ctx, count, n_terms, terms, c.data(), base, out, stream);
}

extern "C" pencil_status pencil_zt_combine_outer(pencil_ctx* ctx, int64_t count, int n_i, int n_j,
                                                 const int64_t* const* terms, const int64_t* ci, const int64_t* cj,
                                                 const int64_t* base, int64_t* out, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (count < 0 || n_i < 0 || n_j < 0 || (int64_t)n_i * n_j > (1 << 20))
    return fail(ctx, PENCIL_EINVAL, "bad term counts");
  const int n = n_i * n_j;
  if (n > 0 && (!terms || !ci || !cj)) return fail(ctx, PENCIL_EINVAL, "terms or coefficients NULL");
  const uint64_t t = ctx->C.t;
  std::vector<uint64_t> c(n);
  for (int i = 0; i < n_i; ++i)
    for (int j = 0; j < n_j; ++j)
      c[i * n_j + j] = (uint64_t)((u128)coeff_mod_t(ci[i], t) * coeff_mod_t(cj[j], t) % t);
  return zt_combine_reduced(ctx, count, n, terms, c.data(), base, out, stream);
}

static pencil_status zt_combine_reduced(pencil_ctx* ctx, int64_t count, int n_terms, const int64_t* const* terms,
                                        const uint64_t* coeffs, const int64_t* base, int64_t* out, void* stream) {
  TRY(check_ptr(ctx, out, "out"));
  for (int i = 0; i < n_terms; ++i) {
    TRY(check_ptr(ctx, terms[i], "terms[i]"));
    if (terms[i] == out) return fail(ctx, PENCIL_EINVAL, "terms[%d] aliases out", i);
  }
  // chunks of kZtTerms terms; each later chunk adds onto the previous result
  const int64_t* b = base;
  int i = 0;
  do {
    ZtTerms T{};
    T.n = std::min(kZtTerms, n_terms - i);
    for (int j = 0; j < T.n; ++j) {
      T.x[j] = terms[i + j];
      T.c[j] = coeffs[i + j];
    }
    hipError_t e = launch_zt_combine(T, b, out, count, ctx->C, (hipStream_t)stream);
    if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "zt_combine launch: %s", hipGetErrorString(e));
    b = out;
    i += T.n;
  } while (i < n_terms);
  return PENCIL_OK;
}

extern "C" pencil_status pencil_zt_encode(pencil_ctx* ctx, int64_t count, const double* x, int64_t* out,
                                          void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (count < 0) return fail(ctx, PENCIL_EINVAL, "count < 0");
  if (count > 0) {
    TRY(check_ptr(ctx, x, "x"));
    TRY(check_ptr(ctx, out, "out"));
  }
  const hipError_t e = launch_zt_encode(x, out, count, ctx->C, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "encode launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_zt_decode(pencil_ctx* ctx, int64_t count, const int64_t* v, double* out,
                                          void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (count < 0) return fail(ctx, PENCIL_EINVAL, "count < 0");
  if (count > 0) {
    TRY(check_ptr(ctx, v, "v"));
    TRY(check_ptr(ctx, out, "out"));
  }
  const hipError_t e = launch_zt_decode(v, out, count, ctx->C, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "decode launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_zt_share(pencil_ctx* ctx, int64_t count, const int64_t* v, uint64_t nonce,
                                         uint64_t object, int64_t* s0, int64_t* s1, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (count < 0) return fail(ctx, PENCIL_EINVAL, "count < 0");
  if (count > 0) {
    TRY(check_ptr(ctx, v, "v"));
    TRY(check_ptr(ctx, s0, "s0"));
    TRY(check_ptr(ctx, s1, "s1"));
    if (s0 == s1) return fail(ctx, PENCIL_EINVAL, "s0 and s1 alias");
  }
  const hipError_t e = launch_zt_share(v, s0, s1, count, nonce, object, ctx->C, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "share launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_bias_grad(pencil_ctx* ctx, const pencil_layer* L, const int64_t* dy, int64_t* db,
                                          void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  TRY(check_ptr(ctx, dy, "dy"));
  TRY(check_ptr(ctx, db, "db"));
  pencil_status st = PENCIL_OK;
  if (!layer_ok(ctx, L, &st)) return st;
  const int64_t spatial = (int64_t)ho_of(L) * wo_of(L);
  // 64-bit sums of entries below t: at most 2^(64 - bitlen(t)) of them
  const int tb = 64 - __builtin_clzll(ctx->C.t);
  if ((int64_t)L->batch * spatial > ((int64_t)1 << (64 - tb)))
    return fail(ctx, PENCIL_EUNSUPPORTED, "bias gradient sums at most 2^%d entries per channel", 64 - tb);
  hipError_t e = launch_bias_grad(dy, db, L->batch, L->c_out, (int)spatial, ctx->C, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "bias_grad launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_dp_noise(pencil_ctx* ctx, int64_t count, double sd, uint64_t nonce, uint64_t object,
                                         int64_t* x, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (count < 0) return fail(ctx, PENCIL_EINVAL, "negative count");
  if (!(sd >= 0.0 && sd <= 4503599627370496.0)) return fail(ctx, PENCIL_EINVAL, "sd must lie in [0, 2^52]");
  if (count == 0) return PENCIL_OK;
  TRY(check_ptr(ctx, x, "x"));
  hipError_t e = launch_dp_noise(x, count, sd, nonce, object, ctx->C, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "dp_noise launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

// The stride-1 layer equal to a stride-s layer over the space-to-depth image
// (sy = 1 along the single row of a Conv1d): c_in s_y s_x input channels, a
// ceil(k / s) kernel, no padding, and ho + k' - 1 by wo + k' - 1 inputs so that
// its outputs are exactly the strided layer's.
static void stride_equiv(const pencil_layer* L, pencil_layer* E, Relayout* R) {
  const int s = L->stride <= 1 ? 1 : L->stride;
  const int sy = L->kind == 2 ? 1 : s, sx = s;
  const int kh = kh_of(L), kw = kw_of(L), ph = ph_of(L), pw = pw_of(L);
  const int ho = (L->h + 2 * ph - kh) / sy + 1, wo = (L->w + 2 * pw - kw) / sx + 1;
  const int kh2 = (kh + sy - 1) / sy, kw2 = (kw + sx - 1) / sx;
  *E = *L;
  E->c_in = L->c_in * sy * sx;
  E->k = kw2;
  E->h = L->kind == 2 ? 1 : ho + kh2 - 1;
  E->w = wo + kw2 - 1;
  E->pad = 0;
  E->stride = 1;
  if (R) {
    *R = Relayout{};
    R->batch = L->batch; R->ci = L->c_in; R->co = L->c_out;
    R->h = L->h; R->w = L->w; R->kh = kh; R->kw = kw;
    R->sy = sy; R->sx = sx; R->ph = ph; R->pw = pw;
    R->h2 = E->h; R->w2 = E->w; R->kh2 = kh2; R->kw2 = kw2;
  }
}

extern "C" pencil_status pencil_stride_map(const pencil_layer* L, pencil_layer* equiv) {
  pencil_status st = PENCIL_OK;
  if (!equiv) return fail(nullptr, PENCIL_EINVAL, "equiv is NULL");
  if (!layer_shape_ok(nullptr, L, true, &st)) return st;
  stride_equiv(L, equiv, nullptr);
  if (!layer_shape_ok(nullptr, equiv, false, &st)) return st;
  return PENCIL_OK;
}

extern "C" pencil_status pencil_stride_relayout(pencil_ctx* ctx, const pencil_layer* L, int which, const int64_t* in,
                                                int64_t* out, void* stream) {
  if (!ctx) return PENCIL_EINVAL;
  if (which < 0 || which > 3) return fail(ctx, PENCIL_EINVAL, "relayout %d invalid", which);
  TRY(check_ptr(ctx, in, "in"));
  TRY(check_ptr(ctx, out, "out"));
  if ((const void*)in == (const void*)out) return fail(ctx, PENCIL_EINVAL, "in and out alias");
  pencil_status st = PENCIL_OK;
  if (!layer_shape_ok(ctx, L, true, &st)) return st;
  pencil_layer E;
  Relayout R;
  stride_equiv(L, &E, &R);
  if (!layer_shape_ok(ctx, &E, false, &st)) return st;
  R.mode = which;
  const int64_t ss = (int64_t)R.sy * R.sx;
  switch (which) {
    case 0: R.total = (int64_t)R.batch * R.ci * ss * R.h2 * R.w2; break;
    case 1: R.total = (int64_t)R.co * R.ci * ss * R.kh2 * R.kw2; break;
    case 2: R.total = (int64_t)R.batch * R.ci * R.h * R.w; break;
    default: R.total = (int64_t)R.co * R.ci * R.kh * R.kw; break;
  }
  hipError_t e = launch_stride_relayout(R, in, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, PENCIL_EHIP, "stride_relayout launch: %s", hipGetErrorString(e));
  return PENCIL_OK;
}

// ------------------------------------------------------------ batched step

struct pencil_step {
  struct Entry {
    int ctx;
    pencil_layer L;
    pencil_plan P;
    Geo G[3];
    uint64_t ws_off[3];
  };
  std::vector<pencil_ctx*> ctxs;
  std::vector<Entry> layers;
  uint32_t ops = 0;
  uint64_t ws_bytes = 0;
  Consts* d_consts = nullptr;
  Tables* d_tabs = nullptr;
  uint64_t* d_nonce = nullptr;
  struct Phase {
    int kind;  // 0 ntt, 1 mac, 2 intt, 3 flood
    int key;   // NTT phases: 8 log2 N + log2(residues per thread); flood: words
    std::vector<StepSeg> segs;
    StepSeg* d_segs = nullptr;
    int64_t blocks = 0;
  };
  std::vector<Phase> phases;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err;
};

static pencil_status step_fail(pencil_step* st, pencil_status code, const char* msg) {
  if (st) st->err = msg;
  else g_create_err = msg;
  return code;
}

// Workspace of one product inside a step: the same layout as run_product.
static uint64_t product_ws(const Consts& C, const Geo& G, int op) {
  const uint64_t poly = (uint64_t)C.L * C.n * 8, ct = 2 * poly;
  const uint64_t na = (uint64_t)n_a_tiles(G), nk = (uint64_t)n_k_tiles(G), no = (uint64_t)n_out_tiles(G);
  if (op == PENCIL_OP_DW) return na * ct + nk * poly + na * poly + nk * ct + no * poly;
  return na * ct + nk * poly + no * poly;
}

extern "C" pencil_status pencil_step_create(pencil_ctx* const* ctxs, const pencil_layer* layers,
                                            const pencil_plan* plans, int n, uint32_t ops, pencil_step** out) {
  if (!out || !ctxs || !layers || !plans || n < 1 || (ops & ~7u) || ops == 0)
    return step_fail(nullptr, PENCIL_EINVAL, "bad step arguments");
  *out = nullptr;
  pencil_step* st = new pencil_step();
  st->ops = ops;
  uint64_t off = 0;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) {
      delete st;
      return step_fail(nullptr, PENCIL_EINVAL, "NULL context");
    }
    int ci = -1;
    for (size_t k = 0; k < st->ctxs.size(); ++k)
      if (st->ctxs[k] == ctxs[i]) ci = (int)k;
    if (ci < 0) {
      ci = (int)st->ctxs.size();
      st->ctxs.push_back(ctxs[i]);
    }
    pencil_step::Entry e{};
    e.ctx = ci;
    e.L = layers[i];
    e.P = plans[i];
    for (int op = 0; op < 3; ++op) {
      if (!(ops & (1u << op))) continue;
      pencil_status s = get_geo(ctxs[i], &layers[i], &plans[i], op, &e.G[op]);
      if (s != PENCIL_OK) {
        std::string m = std::string("layer ") + std::to_string(i) + ": " + ctxs[i]->err;
        delete st;
        return step_fail(nullptr, s, m.c_str());
      }
      e.ws_off[op] = off;
      off += (product_ws(ctxs[i]->C, e.G[op], op) + 255) & ~255ull;
    }
    st->layers.push_back(e);
  }
  st->ws_bytes = off;
  const size_t nc = st->ctxs.size();
  std::vector<Consts> cs(nc);
  std::vector<Tables> ts(nc);
  for (size_t k = 0; k < nc; ++k) {
    cs[k] = st->ctxs[k]->C;
    ts[k] = st->ctxs[k]->T;
  }
  if (hipMalloc(&st->d_consts, nc * sizeof(Consts)) != hipSuccess || hipMalloc(&st->d_tabs, nc * sizeof(Tables)) != hipSuccess ||
      hipMalloc(&st->d_nonce, 256) != hipSuccess) {
    pencil_step_destroy(st);
    return step_fail(nullptr, PENCIL_ENOMEM, "step allocation failed");
  }
  if (hipMemcpy(st->d_consts, cs.data(), nc * sizeof(Consts), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(st->d_tabs, ts.data(), nc * sizeof(Tables), hipMemcpyHostToDevice) != hipSuccess) {
    pencil_step_destroy(st);
    return step_fail(nullptr, PENCIL_EHIP, "step upload failed");
  }
  *out = st;
  return PENCIL_OK;
}

extern "C" pencil_status pencil_step_destroy(pencil_step* st) {
  if (!st) return PENCIL_OK;
  if (st->exec) hipGraphExecDestroy(st->exec);
  if (st->graph) hipGraphDestroy(st->graph);
  for (auto& ph : st->phases) hipFree(ph.d_segs);
  hipFree(st->d_consts);
  hipFree(st->d_tabs);
  hipFree(st->d_nonce);
  delete st;
  return PENCIL_OK;
}

extern "C" const char* pencil_step_last_error(const pencil_step* st) { return st ? st->err.c_str() : ""; }

extern "C" pencil_status pencil_step_workspace(const pencil_step* st, uint64_t* bytes) {
  if (!st || !bytes) return PENCIL_EINVAL;
  *bytes = st->ws_bytes;
  return PENCIL_OK;
}

static pencil_step::Phase& phase_for(pencil_step* st, int kind, int key) {
  for (auto& ph : st->phases)
    if (ph.kind == kind && ph.key == key) return ph;
  pencil_step::Phase ph;
  ph.kind = kind;
  ph.key = key;
  st->phases.push_back(ph);
  return st->phases.back();
}

static void add_seg(pencil_step::Phase& ph, StepSeg sg, int64_t blocks) {
  if (blocks <= 0) return;
  sg.block_begin = ph.blocks;
  ph.blocks += blocks;
  ph.segs.push_back(sg);
}

// Drop the segment tables and the captured graph: the step is unbound until a
// bind succeeds again.
static void step_unbind(pencil_step* st) {
  st->bound = false;
  for (auto& ph : st->phases) hipFree(ph.d_segs);
  st->phases.clear();
  if (st->exec) {
    hipGraphExecDestroy(st->exec);
    st->exec = nullptr;
  }
  if (st->graph) {
    hipGraphDestroy(st->graph);
    st->graph = nullptr;
  }
}

static pencil_status step_bind_tables(pencil_step* st, const pencil_step_io* io, void* ws);

extern "C" pencil_status pencil_step_bind(pencil_step* st, const pencil_step_io* io, void* ws) {
  if (!st) return step_fail(st, PENCIL_EINVAL, "NULL argument");
  // a failed bind leaves the step unbound (run and capture refuse it), never
  // with partly built segment tables
  step_unbind(st);
  if (!io || !ws) return step_fail(st, PENCIL_EINVAL, "NULL argument");
  const pencil_status s = step_bind_tables(st, io, ws);
  if (s != PENCIL_OK) {
    step_unbind(st);
    return s;
  }
  st->bound = true;
  return PENCIL_OK;
}

static pencil_status step_bind_tables(pencil_step* st, const pencil_step_io* io, void* ws) {
  // ciphertext buffers and the workspace are moved in 16-byte pairs
  auto misaligned = [](const void* p) { return p && ((uintptr_t)p & 15) != 0; };
  if (misaligned(ws)) return step_fail(st, PENCIL_EINVAL, "ws is not 16-byte aligned");
  for (size_t i = 0; i < st->layers.size(); ++i)
    if (misaligned(io[i].ct_x1) || misaligned(io[i].ct_dy_dx) || misaligned(io[i].ct_x_dw) ||
        misaligned(io[i].ct_dy_dw) || misaligned(io[i].ct_y) || misaligned(io[i].ct_dx) || misaligned(io[i].ct_dw))
      return step_fail(st, PENCIL_EINVAL, "a ciphertext buffer is not 16-byte aligned");
  // fixed phase order: forward NTTs, MAC, inverse NTTs, flood (per ring degree / flood width)
  for (int kind = 0; kind < 4; ++kind)
    for (auto& e : st->layers) {
      const Consts& C = st->ctxs[e.ctx]->C;
      if (kind == 1) {  // each multiply-accumulate kernel kind launches separately
        for (int k = 0; k < kMacVariants / 3; ++k) phase_for(st, 1, k);
      } else {
        phase_for(st, kind, kind == 3 ? C.flood_words : C.log2n * 8 + C.ntt_loge);
      }
    }
  for (size_t i = 0; i < st->layers.size(); ++i) {
    const auto& e = st->layers[i];
    const pencil_step_io& b = io[i];
    pencil_ctx* ctx = st->ctxs[e.ctx];
    const Consts& C = ctx->C;
    const int64_t poly = (int64_t)C.L * C.n, ctw = 2 * poly;
    for (int op = 0; op < 3; ++op) {
      if (!(st->ops & (1u << op))) continue;
      const Geo& G = e.G[op];
      const int64_t na = n_a_tiles(G), nk = n_k_tiles(G), no = n_out_tiles(G);
      const pencil_layer* L = &e.L;
      // inputs and outputs of this product
      const uint64_t* ct_a = op == 0 ? b.ct_x1 : op == 1 ? b.ct_dy_dx : b.ct_x_dw;
      const int64_t* add_share = op == 0 ? b.x0 : op == 1 ? b.dy0 : nullptr;
      const int64_t* pt_k = op == 2 ? b.dy0 : b.w;
      uint64_t* ct_out = op == 0 ? b.ct_y : op == 1 ? b.ct_dx : b.ct_dw;
      int64_t* share_out = op == 0 ? b.y0 : op == 1 ? b.dx0 : b.dw_mask;
      if (!ct_a || !pt_k || !ct_out || !share_out || (op != 2 && !add_share) ||
          (op == 2 && (!b.x0 || !b.ct_dy_dw)))
        return step_fail(st, PENCIL_EINVAL, "missing buffer in step io");
      uint64_t* w = (uint64_t*)((uint8_t*)ws + e.ws_off[op]);
      const uint64_t nonce_off = 2 * (uint64_t)i + (op == 0 ? 0 : 1);
      auto& ntt = phase_for(st, 0, C.log2n * 8 + C.ntt_loge);
      MacArgs A{};
      A.m_rows = G.nM * G.nOY * G.nOX;
      A.variant = e.P.sched[op];
      if (A.variant < 0 || A.variant >= kMacVariants) return step_fail(st, PENCIL_EINVAL, "schedule variant invalid");
      A.pk = ctx->d_pk_split;
      A.out = ct_out;
      StepSeg base{};
      base.ctx = e.ctx;
      base.G = G;
      // term A-side ciphertext: component 0 staged with the share added
      // (forward, input gradient), component 1 and the weight gradient's
      // ciphertexts read in place
      {
        uint64_t* cts = w;
        w += na * ctw;
        uint64_t* pts = w;
        w += nk * poly;
        MacTerm mt{ct_a, pts, poly, 1, 0};
        if (add_share) {
          StepSeg sc = base;
          sc.kind = SEG_CT;
          sc.src = ct_a;
          sc.dst = cts;
          sc.tensor = add_share;
          sc.V = view_a(L, op);
          add_seg(ntt, sc, na * C.L);
          mt.a = cts;
          mt.c1 = comp1_offset(cts, ct_a, poly);
        }
        StepSeg sp = base;
        sp.kind = SEG_PT;
        sp.side = 1;
        sp.tensor = pt_k;
        sp.dst = pts;
        sp.V = view_k(L, op);
        add_seg(ntt, sp, nk * C.L);
        A.term[0] = mt;
        A.n_terms = 1;
      }
      if (op == 2) {  // term B: plaintext <X>_0 on the A side, ciphertext <dY>_1 on the K side
        uint64_t* pts = w;
        w += na * poly;
        w += nk * ctw;
        StepSeg sp = base;
        sp.kind = SEG_PT;
        sp.side = 0;
        sp.tensor = b.x0;
        sp.dst = pts;
        sp.V = view_a(L, op);
        add_seg(ntt, sp, na * C.L);
        A.term[1] = MacTerm{pts, b.ct_dy_dw, poly, 0, 0};
        A.n_terms = 2;
      }
      uint64_t* u = w;
      StepSeg su = base;
      su.kind = SEG_TERN;
      su.dst = u;
      su.nonce_off = nonce_off;
      su.obj_base = out_object(op, 0);
      su.purpose = P_RR_U;
      add_seg(ntt, su, no * C.L);
      A.u = u;
      StepSeg sm = base;
      sm.kind = SEG_MAC;
      sm.mac = A;
      sm.slot_blocks = (int64_t)C.n * C.L / 64;
      const int64_t chunks = mac_chunks(A.variant, A.m_rows, G.nR);
      add_seg(phase_for(st, 1, A.variant / 3), sm, (sm.slot_blocks * chunks + 7) & ~(int64_t)7);
      StepSeg si = base;
      si.kind = SEG_INTT;
      si.dst = ct_out;
      add_seg(phase_for(st, 2, C.log2n * 8 + C.ntt_loge), si, 2 * no * C.L);
      StepSeg sf = base;
      sf.kind = SEG_FLOOD;
      sf.dst = ct_out;
      sf.count = no;
      sf.share = share_out;
      sf.bias = op == 0 ? b.bias : nullptr;
      sf.V2 = view_out(L, op);
      sf.nonce_off = nonce_off;
      sf.obj_base = out_object(op, 0);
      add_seg(phase_for(st, 3, C.flood_words), sf, (no * (C.n / 4) + 255) / 256);
    }
  }
  for (auto& ph : st->phases) {
    if (ph.segs.empty()) continue;
    if (ph.blocks >= (1ll << 31)) return step_fail(st, PENCIL_EUNSUPPORTED, "step phase too large");
    if (hipMalloc(&ph.d_segs, ph.segs.size() * sizeof(StepSeg)) != hipSuccess)
      return step_fail(st, PENCIL_ENOMEM, "segment allocation failed");
    if (hipMemcpy(ph.d_segs, ph.segs.data(), ph.segs.size() * sizeof(StepSeg), hipMemcpyHostToDevice) != hipSuccess)
      return step_fail(st, PENCIL_EHIP, "segment upload failed");
  }
  return PENCIL_OK;
}

static hipError_t step_phases(pencil_step* st, hipStream_t s) {
  for (auto& ph : st->phases) {
    if (ph.segs.empty()) continue;
    StepPhase P{};
    P.segs = ph.d_segs;
    P.nseg = (int32_t)ph.segs.size();
    P.consts = st->d_consts;
    P.tabs = st->d_tabs;
    P.nonce = st->d_nonce;
    hipError_t e = hipSuccess;
    pencil_ctx* pc = st->ctxs[0];
    if (ph.kind == 0 || ph.kind == 2)
      e = timed(pc, ph.kind == 0 ? KID_STEP_NTT : KID_STEP_INTT, s,
                [&] { return launch_step_ntt(ph.key / 8, ph.key % 8, ph.kind == 2, P, ph.blocks, s); });
    else if (ph.kind == 1)
      e = timed(pc, KID_STEP_MAC, s, [&] { return launch_step_mac(P, ph.blocks, ph.key, s); });
    else
      e = timed(pc, KID_STEP_FLOOD, s, [&] { return launch_step_flood(ph.key, P, ph.blocks, s); });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

extern "C" pencil_status pencil_step_run(pencil_step* st, uint64_t nonce, void* stream) {
  if (!st) return PENCIL_EINVAL;
  if (!st->bound) return step_fail(st, PENCIL_EINVAL, "step not bound");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_set_u64(st->d_nonce, nonce, 0, s);
  if (e == hipSuccess) e = step_phases(st, s);
  if (e != hipSuccess) return step_fail(st, PENCIL_EHIP, hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_step_graph_capture(pencil_step* st) {
  if (!st) return PENCIL_EINVAL;
  if (!st->bound) return step_fail(st, PENCIL_EINVAL, "step not bound");
  for (auto* c : st->ctxs)
    if (c->prof_on) return step_fail(st, PENCIL_EINVAL, "disable profiling before capture");
  if (st->exec) {
    hipGraphExecDestroy(st->exec);
    st->exec = nullptr;
  }
  if (st->graph) {
    hipGraphDestroy(st->graph);
    st->graph = nullptr;
  }
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return step_fail(st, PENCIL_EHIP, "capture stream");
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const uint64_t stride = 2 * (uint64_t)st->layers.size();
    hipError_t k = launch_set_u64(st->d_nonce, stride, 1, cs);
    if (k == hipSuccess) k = step_phases(st, cs);
    e = hipStreamEndCapture(cs, &st->graph);
    if (k != hipSuccess) e = k;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&st->exec, st->graph, nullptr, nullptr, 0);
  hipStreamDestroy(cs);
  if (e != hipSuccess) return step_fail(st, PENCIL_EHIP, hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_step_set_nonce(pencil_step* st, uint64_t nonce, void* stream) {
  if (!st) return PENCIL_EINVAL;
  const uint64_t stride = 2 * (uint64_t)st->layers.size();
  hipError_t e = launch_set_u64(st->d_nonce, nonce - stride, 0, (hipStream_t)stream);
  if (e != hipSuccess) return step_fail(st, PENCIL_EHIP, hipGetErrorString(e));
  return PENCIL_OK;
}

extern "C" pencil_status pencil_step_graph_launch(pencil_step* st, void* stream) {
  if (!st) return PENCIL_EINVAL;
  if (!st->exec) return step_fail(st, PENCIL_EINVAL, "no captured graph");
  hipError_t e = hipGraphLaunch(st->exec, (hipStream_t)stream);
  if (e != hipSuccess) return step_fail(st, PENCIL_EHIP, hipGetErrorString(e));
  return PENCIL_OK;
}

// ------------------------------------------------------------ autotuner

static std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Autotuner cache: one JSON object per line, {"key": "...", "choice": V, ...}
// with V an integer or a list of integers.
struct CacheEntry {
  std::string key;
  std::vector<int> v;
};

static void cache_read(const char* path, std::vector<CacheEntry>* out) {
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[2048];
  while (std::fgets(line, sizeof line, f)) {
    const char* k = std::strstr(line, "\"key\": \"");
    const char* v = std::strstr(line, "\"choice\": ");
    if (!k || !v) continue;
    k += 8;
    const char* e = std::strchr(k, '"');
    if (!e) continue;
    CacheEntry ce{std::string(k, e), {}};
    v += 10;
    if (*v == '[') {
      for (++v; *v && *v != ']';) {
        char* endp = nullptr;
        const long x = std::strtol(v, &endp, 10);
        if (endp == v) break;
        ce.v.push_back((int)x);
        v = endp;
        while (*v == ',' || *v == ' ') ++v;
      }
    } else {
      ce.v.push_back(std::atoi(v));
    }
    out->push_back(std::move(ce));
  }
  std::fclose(f);
}

static const std::vector<int>* cache_find(const std::vector<CacheEntry>& c, const std::string& key) {
  for (auto it = c.rbegin(); it != c.rend(); ++it)
    if (it->key == key) return &it->v;
  return nullptr;
}

// Milliseconds per call of fn (one warm-up call, then `reps` timed calls).
template <class F>
static float time_ms(F&& fn, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return -1;
  }
  float ms = -1;
  if (fn() == PENCIL_OK && hipDeviceSynchronize() == hipSuccess) {
    hipEventRecord(a, nullptr);
    bool ok = true;
    for (int i = 0; i < reps && ok; ++i) ok = fn() == PENCIL_OK;
    hipEventRecord(b, nullptr);
    if (ok && hipEventSynchronize(b) == hipSuccess) {
      hipEventElapsedTime(&ms, a, b);
      ms /= reps;
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}

static std::string tile_str(const pencil_tile& t) {
  char b[96];
  std::snprintf(b, sizeof b, "%d,%d,%d,%d,%d,%d,%d", t.m, t.r, t.k, t.oh, t.ow, t.kh, t.kw);
  return b;
}

static std::string times_str(const std::vector<float>& ms) {
  std::string out;
  for (float x : ms) out += (out.empty() ? "" : ", ") + std::to_string(x);
  return out;
}

static pencil_tile& plan_tile_mut(pencil_plan* P, int op) { return op == 0 ? P->fwd : op == 1 ? P->dx : P->dw; }

// The autotuner.  It measures, on this GPU and with synthetic inputs, the
// choices that leave the decrypted results unchanged: the NTT's residues per
// thread (per context), each product's partition among the planner's
// best-ranked ones (the caller's tile included), and each product's
// multiply-accumulate schedule (all nine).  A partition changes the
// ciphertext layout, so tune before encrypting with the plan.
extern "C" pencil_status pencil_autotune(pencil_ctx* ctx, const pencil_layer* L, pencil_plan* P,
                                         const char* cache_path) {
  if (!ctx || !P) return PENCIL_EINVAL;
  pencil_status lst = PENCIL_OK;
  if (!layer_ok(ctx, L, &lst)) return lst;
  for (int op = 0; op < 3; ++op) {
    Geo G;
    TRY(get_geo(ctx, L, P, op, &G));
  }
  std::vector<CacheEntry> cache;
  cache_read(cache_path, &cache);
  std::vector<std::string> fresh;
  const std::string arch = arch_name(ctx->device);
  Consts& C = ctx->C;
  char key[512];
  auto layer_key = [&](const char* what, int op) {
    std::snprintf(key, sizeof key, "%s N=%d L=%d layer=%d,%d,%d,%d,%d,%d,%d,%d op=%d %s", arch.c_str(), C.n, C.L,
                  L->kind, L->batch, L->c_in, L->c_out, L->h, L->w, L->k, L->pad, op, what);
    return std::string(key);
  };
  // candidate partitions per product: the caller's, then the planner's best
  constexpr size_t kPartitions = 3;
  std::vector<pencil_tile> cand[3];
  for (int op = 0; op < 3; ++op) {
    cand[op].push_back(plan_tile(P, op));
    std::vector<pencil_tile> ranked;
    pencil_tile best;
    plan_op(L, op, C.log2n, &best, &ranked, kPartitions);
    for (const pencil_tile& t : ranked) {
      bool dup = false;
      for (const pencil_tile& u : cand[op]) dup |= std::memcmp(&t, &u, sizeof t) == 0;
      if (!dup && cand[op].size() < kPartitions) cand[op].push_back(t);
    }
  }
  // scratch for the largest candidate of every product
  const int64_t xs = (int64_t)L->batch * L->c_in * L->h * L->w;
  const int64_t ys = (int64_t)L->batch * L->c_out * ho_of(L) * wo_of(L);
  const int64_t wsz = (int64_t)L->c_out * L->c_in * kh_of(L) * kw_of(L);
  const int64_t tmax = std::max(xs, std::max(ys, wsz));
  uint64_t nin = 0, nout = 0, wsb = 0;
  const uint64_t ctb = 2ull * C.L * C.n * 8;
  for (int op = 0; op < 3; ++op)
    for (const pencil_tile& t : cand[op]) {
      pencil_plan Q = *P;
      plan_tile_mut(&Q, op) = t;
      pencil_sizes sz;
      TRY(pencil_layout(ctx, L, &Q, &sz));
      nin = std::max(nin, op == 0 ? sz.n_ct[0] : op == 1 ? sz.n_ct[1] : std::max(sz.n_ct[2], sz.n_ct[3]));
      nout = std::max(nout, sz.n_out[op]);
      wsb = std::max(wsb, op == 0 ? sz.ws_fwd_bytes : sz.ws_bwd_bytes);
    }
  uint8_t *cin = nullptr, *cin2 = nullptr, *cout = nullptr, *ws = nullptr;
  int64_t *t0 = nullptr, *t1 = nullptr, *tout = nullptr;
  auto release = [&] {
    hipFree(cin);
    hipFree(cin2);
    hipFree(cout);
    hipFree(ws);
    hipFree(t0);
    hipFree(t1);
    hipFree(tout);
  };
  if (hipMalloc(&cin, nin * ctb) != hipSuccess || hipMalloc(&cin2, nin * ctb) != hipSuccess ||
      hipMalloc(&cout, nout * ctb) != hipSuccess || hipMalloc(&ws, wsb) != hipSuccess ||
      hipMalloc(&t0, tmax * 8) != hipSuccess || hipMalloc(&t1, tmax * 8) != hipSuccess ||
      hipMalloc(&tout, tmax * 8) != hipSuccess) {
    release();
    return fail(ctx, PENCIL_ENOMEM, "autotune scratch");
  }
  // residues 1 and 2^16 + 1 (split form: 1 + 2^32): valid operands for every limb
  hipMemsetD32((hipDeviceptr_t)cin, 0x00000001, nin * ctb / 4);
  hipMemsetD32((hipDeviceptr_t)cin2, 0x00000001, nin * ctb / 4);
  hipMemsetD32((hipDeviceptr_t)t0, 0x00000001, tmax * 2);  // 2^32 + 1 < t: valid Z_t entries
  hipMemsetD32((hipDeviceptr_t)t1, 0x00000001, tmax * 2);
  auto run = [&](int op, const pencil_plan* Q) -> pencil_status {
    if (op == 0)
      return pencil_linear_fwd(ctx, L, Q, (const uint64_t*)cin, t0, t1, nullptr, (uint64_t*)cout, tout, ws, 1,
                               nullptr);
    if (op == 1)
      return pencil_linear_bwd(ctx, L, Q, (const uint64_t*)cin, nullptr, nullptr, t0, nullptr, t1, (uint64_t*)cout,
                               tout, nullptr, nullptr, ws, 1, nullptr);
    return pencil_linear_bwd(ctx, L, Q, nullptr, (const uint64_t*)cin, (const uint64_t*)cin2, t0, t1, nullptr,
                             nullptr, nullptr, (uint64_t*)cout, tout, ws, 1, nullptr);
  };
  // the forward product and both backward ones, the way a training step runs them
  auto step_ms = [&](const pencil_plan* Q) {
    float total = 0;
    for (int op = 0; op < 3; ++op) {
      const float ms = time_ms([&] { return run(op, Q); }, 3);
      if (ms < 0) return -1.0f;
      total += ms;
    }
    return total;
  };
  pencil_status st = PENCIL_OK;
  // 1) NTT residues per thread (context-wide), timed on this layer's products
  std::snprintf(key, sizeof key, "%s N=%d L=%d ntt_loge", arch.c_str(), C.n, C.L);
  if (const std::vector<int>* hit = cache_find(cache, key)) {
    if (hit->size() == 1 && (*hit)[0] >= 4 && (*hit)[0] <= 5 && (C.log2n >= 12 || (*hit)[0] == 4))
      C.ntt_loge = (*hit)[0];
  } else {
    std::vector<int> cands = C.log2n >= 12 ? std::vector<int>{4, 5} : std::vector<int>{4};
    std::vector<float> times;
    int bestv = C.ntt_loge;
    float best = -1;
    for (int c : cands) {
      C.ntt_loge = c;
      const float ms = step_ms(P);
      times.push_back(ms);
      if (ms > 0 && (best < 0 || ms < best)) {
        best = ms;
        bestv = c;
      }
    }
    C.ntt_loge = bestv;
    fresh.push_back(std::string("{\"key\": \"") + key + "\", \"choice\": " + std::to_string(bestv) +
                    ", \"candidates\": [4, 5], \"ms\": [" + times_str(times) + "]}");
  }
  // 2) partition, then 3) multiply-accumulate schedule, per product
  for (int op = 0; op < 3 && st == PENCIL_OK; ++op) {
    const std::string pkey = layer_key("partition", op);
    const std::vector<int>* hit = cache_find(cache, pkey);
    bool applied = false;
    if (hit && hit->size() == 7) {
      pencil_tile t{(*hit)[0], (*hit)[1], (*hit)[2], (*hit)[3], (*hit)[4], (*hit)[5], (*hit)[6]};
      pencil_plan Q = *P;
      plan_tile_mut(&Q, op) = t;
      Geo G;
      if (get_geo(ctx, L, &Q, op, &G) == PENCIL_OK) {
        plan_tile_mut(P, op) = t;
        applied = true;
      }
    }
    if (!applied && cand[op].size() > 1) {
      std::vector<float> times;
      std::string tiles;
      size_t besti = 0;
      float best = -1;
      for (size_t i = 0; i < cand[op].size(); ++i) {
        pencil_plan Q = *P;
        plan_tile_mut(&Q, op) = cand[op][i];
        Q.sched[op] = default_sched(L, op, cand[op][i], C.n);
        const float ms = time_ms([&] { return run(op, &Q); }, 3);
        times.push_back(ms);
        tiles += (tiles.empty() ? "[" : ", [") + tile_str(cand[op][i]) + "]";
        if (ms > 0 && (best < 0 || ms < best)) {
          best = ms;
          besti = i;
        }
      }
      if (besti != 0) {
        plan_tile_mut(P, op) = cand[op][besti];
        P->sched[op] = default_sched(L, op, cand[op][besti], C.n);
      }
      fresh.push_back(std::string("{\"key\": \"") + pkey + "\", \"choice\": [" + tile_str(plan_tile(P, op)) +
                      "], \"candidates\": [" + tiles + "], \"ms\": [" + times_str(times) + "]}");
    }
    const std::string skey = layer_key(("sched tile=" + tile_str(plan_tile(P, op))).c_str(), op);
    hit = cache_find(cache, skey);
    if (hit && hit->size() == 1 && (*hit)[0] >= 0 && (*hit)[0] < kMacVariants) {
      P->sched[op] = (*hit)[0];
      continue;
    }
    std::vector<float> times;
    int bestv = P->sched[op];
    float best = -1;
    for (int cand_s = 0; cand_s < kMacVariants; ++cand_s) {
      pencil_plan Q = *P;
      Q.sched[op] = cand_s;
      const float ms = time_ms([&] { return run(op, &Q); }, 3);
      times.push_back(ms);
      if (ms > 0 && (best < 0 || ms < best)) {
        best = ms;
        bestv = cand_s;
      }
    }
    P->sched[op] = bestv;
    fresh.push_back(std::string("{\"key\": \"") + skey + "\", \"choice\": " + std::to_string(bestv) +
                    ", \"ms\": [" + times_str(times) + "]}");
  }
  release();
  if (st == PENCIL_OK && cache_path && !fresh.empty()) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      for (auto& l : fresh) std::fprintf(f, "%s\n", l.c_str());
      std::fclose(f);
    }
  }
  return st;
}

// ------------------------------------------------------------ noise bound

extern "C" pencil_status pencil_noise_bound(const pencil_params* params, const pencil_layer* L, const pencil_plan* P,
                                            int op, uint32_t plaintext_bits, pencil_noise* out) {
  if (!out || op < 0 || op > 2) return fail(nullptr, PENCIL_EINVAL, "bad noise-bound request");
  if (plaintext_bits < 1 || plaintext_bits > 62) return fail(nullptr, PENCIL_EINVAL, "plaintext_bits outside [1, 62]");
  pencil_ctx tmp;  // host-only: parameters and geometry, no device state
  pencil_status st = resolve_params(params, &tmp);
  if (st != PENCIL_OK) return st;
  Geo G;
  st = get_geo(&tmp, L, P, op, &G);
  if (st != PENCIL_OK) {
    g_create_err = tmp.err;
    return st;
  }
  const double n = (double)tmp.C.n;
  // nonzero coefficients of a plaintext polynomial: K tiles (weights, or dY for
  // the weight gradient's term A) and, for the weight gradient's term B, A tiles
  const double nnz_k = (double)G.rt * G.kt * G.kh * G.kw;
  const double nnz_a = (double)G.mt * G.kt * G.ha * G.wa;
  const double nnz = std::min(n, op == PENCIL_OP_DW ? std::max(nnz_k, nnz_a) : nnz_k);
  const double terms = (double)G.nK * G.nKY * G.nKX * (op == PENCIL_OP_DW ? 2 : 1);
  const double p = std::ldexp(1.0, (int)plaintext_bits - 1);
  // input noise: CBD errors (|e| <= 21) times ternary u and s, plus e0, plus
  // the two roundings of round(q m / t) (encryption, share add)
  const double fresh = 42 * n + 23;
  const double product = terms * nnz * p * fresh + (42 * n + 21);  // + re-randomisation
  const double flood = std::ldexp(1.0, (int)tmp.C.flood_bits);
  Big q{1};
  for (int l = 0; l < tmp.C.L; ++l) q = big_mul_small(q, tmp.C.limb[l].q);
  const Big delta = big_div_small(q, tmp.C.t);
  double dd = 0;
  for (size_t w = delta.size(); w-- > 0;) dd = dd * 18446744073709551616.0 + (double)delta[w];
  out->product_bits = std::log2(product);
  out->flood_bits = (double)tmp.C.flood_bits;
  out->budget_bits = std::log2(dd / 2);
  out->margin_bits = out->budget_bits - std::log2(product + flood);
  out->smudge_bits = out->flood_bits - out->product_bits;
  if (product + flood >= dd / 2)
    return fail(nullptr, PENCIL_ENOISE,
                "op %d: worst-case noise 2^%.1f (product 2^%.1f + flood 2^%.1f) reaches Delta/2 = 2^%.1f", op,
                std::log2(product + flood), out->product_bits, out->flood_bits, out->budget_bits);
  return PENCIL_OK;
}

// ------------------------------------------------------------ multiply probe

extern "C" pencil_status pencil_probe_mul32(int kind, double* per_s) {
  if (kind < 0 || kind > 2 || !per_s) return fail(nullptr, PENCIL_EINVAL, "probe kind %d invalid", kind);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return fail(nullptr, PENCIL_EHIP, "no HIP device");
  const int64_t threads = (int64_t)cus * 8 * 256;  // 8 waves per SIMD
  const int iters = 4096;
  uint64_t* out = nullptr;
  if (hipMalloc(&out, threads * sizeof(uint64_t)) != hipSuccess) return fail(nullptr, PENCIL_ENOMEM, "probe buffer");
  hipEvent_t a = nullptr, b = nullptr;
  float ms = 0;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = launch_probe_mul(kind, out, threads, iters, nullptr);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, nullptr);
  for (int r = 0; r < 5 && e == hipSuccess; ++r) e = launch_probe_mul(kind, out, threads, iters, nullptr);
  if (e == hipSuccess) e = hipEventRecord(b, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFree(out);
  if (e != hipSuccess || ms <= 0) return fail(nullptr, PENCIL_EHIP, "probe: %s", hipGetErrorString(e));
  *per_s = 5.0 * (double)threads * iters * 8 / (ms * 1e-3);
  return PENCIL_OK;
}

// ------------------------------------------------------------ profiling

extern "C" pencil_status pencil_profile_enable(pencil_ctx* ctx, int enable) {
  if (!ctx) return PENCIL_EINVAL;
  for (auto& r : ctx->pending) {
    hipEventSynchronize(r.b);
    ctx->ev_pool.push_back(r.a);
    ctx->ev_pool.push_back(r.b);
  }
  ctx->pending.clear();
  for (int k = 0; k < KID_COUNT; ++k) {
    ctx->prof_ms[k] = 0;
    ctx->prof_launches[k] = 0;
  }
  ctx->prof_on = enable != 0;
  return PENCIL_OK;
}

extern "C" pencil_status pencil_profile_read(pencil_ctx* ctx, pencil_kernel_stat* out, int max, int* count) {
  if (!ctx || !count) return PENCIL_EINVAL;
  for (auto& r : ctx->pending) {
    HIP_TRY(ctx, hipEventSynchronize(r.b));
    float ms = 0;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, r.a, r.b));
    ctx->prof_ms[r.kid] += ms;
    ctx->prof_launches[r.kid] += 1;
    ctx->ev_pool.push_back(r.a);
    ctx->ev_pool.push_back(r.b);
  }
  ctx->pending.clear();
  int n = 0;
  for (int k = 0; k < KID_COUNT && n < max; ++k) {
    if (!out) break;
    std::memset(&out[n], 0, sizeof out[n]);
    std::snprintf(out[n].name, sizeof out[n].name, "%s", kKernelNames[k]);
    out[n].launches = ctx->prof_launches[k];
    out[n].total_ms = ctx->prof_ms[k];
    ++n;
  }
  *count = n;
  return PENCIL_OK;
}

extern "C" pencil_status pencil_plan_auto_n(uint32_t log2_n, const pencil_layer* L, pencil_plan* plan) {
  if (!plan || log2_n < 10 || log2_n > 14) return fail(nullptr, PENCIL_EINVAL, "bad plan request");
  pencil_status st = PENCIL_OK;
  if (!layer_ok(nullptr, L, &st)) return st;
  pencil_tile* tiles[3] = {&plan->fwd, &plan->dx, &plan->dw};
  for (int op = 0; op < 3; ++op) {
    if (!plan_op(L, op, (int)log2_n, tiles[op])) return fail(nullptr, PENCIL_EUNSUPPORTED, "no tile fits");
    plan->sched[op] = default_sched(L, op, *tiles[op], 1 << log2_n);
  }
  return PENCIL_OK;
}
