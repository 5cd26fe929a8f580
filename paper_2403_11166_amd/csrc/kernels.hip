// HIP kernels for gfx950: negacyclic NTT/INTT per RNS limb staged in LDS,
// encode + lift, pointwise multiply-accumulate, re-randomise/flood/mask,
// encryption and exact-CRT decryption.
#include "pencil_internal.h"
#include "modarith.h"

namespace pencil {

// Global-memory views of generic pointers.  Pointers read from device memory
// (the batched step's segment tables) are generic to the compiler, which then
// emits flat instructions; flat loads also count against the LDS/scalar wait
// counter.  Every buffer here is global memory, so the hot loops access it
// through these address-space-qualified views.
#define PENCIL_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ PENCIL_GLOBAL T* gview(T* p) {
  return (PENCIL_GLOBAL T*)p;
}
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));


// ----------------------------------------------------------------- NTT core
// One workgroup transforms one limb-polynomial held in LDS.  N/E threads each
// keep E residues in registers (E = 16, or 32 at N = 16384) and run several
// butterfly stages per LDS round trip; the log2 N stages are split into
// ceil(log2 N / log2 E) passes of near-equal size.  LDS rows are padded by one
// word every 32 so that strided passes spread over the banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

template <int LOGN, int LOGE_>
struct NttShape {
  static constexpr int LOGE = LOGE_;
  static constexpr int E = 1 << LOGE;
  static constexpr int T = (1 << LOGN) / E;  // threads per block
  static constexpr int NP = (LOGN + LOGE - 1) / LOGE;
  // stages in pass i: the first LOGN % NP passes take one more
  static constexpr int size(int i) { return LOGN / NP + (i < LOGN % NP ? 1 : 0); }
  static constexpr int start(int i) { return i == 0 ? 0 : start(i - 1) + size(i - 1); }
};

// Butterfly constants of one modulus: 2q, 2^64 - q, 2^64 - 2q and 2q + 1.  They
// are hidden from the optimiser so that x - q stays the single 64-bit addition
// x + (2^64 - q) instead of a borrow chain.
struct BflyK {
  uint64_t q2, nq, nq2, q2p1;
};

__device__ __forceinline__ BflyK bfly_consts(uint64_t q) {
  BflyK k{2 * q, 0 - q, 0 - 2 * q, 2 * q + 1};
  asm volatile("" : "+s"(k.q2), "+s"(k.nq), "+s"(k.nq2), "+s"(k.q2p1));
  return k;
}

// x - 2q if x >= 2q, else x, for x < 2^63: the sign of x - 2q decides.
__device__ __forceinline__ uint64_t csub2q(uint64_t x, const BflyK& k) {
  const uint64_t d = x + k.nq2;
  const uint32_t m = (uint32_t)((int32_t)(uint32_t)(d >> 32) >> 31);
  const uint64_t back = ((uint64_t)((uint32_t)(k.q2 >> 32) & m) << 32) | ((uint32_t)k.q2 & m);
  return d + back;
}

// Shoup's lazy product y w mod q in [0, 2q): y w - floor(y ws / 2^64) q.
__device__ __forceinline__ uint64_t shoup_lazy(uint64_t y, const TW w, const BflyK& k) {
  return y * w.w + __umul64hi(y, w.ws) * k.nq;
}

// Harvey's lazy Cooley-Tukey butterfly: x, y in [0, 4q) -> [0, 4q), q < 2^61.
__device__ __forceinline__ void ct_bfly(uint64_t& x, uint64_t& y, const TW w, const BflyK& k) {
  const uint64_t a = csub2q(x, k);
  const uint64_t t = shoup_lazy(y, w, k);
  x = a + t;
  y = (a + k.q2p1) + ~t;  // a - t + 2q
}

// Lazy Gentleman-Sande butterfly: u, v in [0, 2q) -> [0, 2q).
__device__ __forceinline__ void gs_bfly(uint64_t& u, uint64_t& v, const TW w, const BflyK& k) {
  const uint64_t s = csub2q(u + v, k);
  const uint64_t d = (u + k.q2p1) + ~v;  // u - v + 2q
  v = shoup_lazy(d, w, k);
  u = s;
}

// Forward (merged negacyclic Cooley-Tukey, psi^rev twiddles; natural order in,
// bit-reversed out) stages S0 .. S0+S-1.  At stage l (t = N >> (l+1)) the pair
// (i0, i0 + t) of group i = i0 >> (log2 N - l) uses tw[2^l + i].  A thread takes
// E / 2^S groups of 2^S residues {base + k * 2^LT}, LT = log2 N - S0 - S.
template <int LOGN, int LOGE, int S0, int S, bool LAST>
__device__ __forceinline__ void fwd_pass(uint64_t* a, const PENCIL_GLOBAL TW* tw, uint64_t q, const BflyK& bk) {
  using Sh = NttShape<LOGN, LOGE>;
  constexpr int T = Sh::T, G = Sh::E >> S, K = 1 << S, LT = LOGN - S0 - S;
  const int tid = threadIdx.x;
  uint64_t v[Sh::E];
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const int g = r * T + tid;
    const int base = ((g >> LT) << (LOGN - S0)) + (g & ((1 << LT) - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) v[r * K + k] = a[lpad(base + (k << LT))];
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int h = 1 << (S - 1 - s);
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int blk = (r * T + tid) >> LT;
#pragma unroll
      for (int j = 0; j < (1 << s); ++j) {
        const PENCIL_GLOBAL TW* tp = tw + (1 << (S0 + s)) + (blk << s) + j;
        const TW w{tp->w, tp->ws};
#pragma unroll
        for (int k = j << (S - s); k < ((j + 1) << (S - s)); ++k) {
          if (k & h) continue;
          ct_bfly(v[r * K + k], v[r * K + k + h], w, bk);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const int g = r * T + tid;
    const int base = ((g >> LT) << (LOGN - S0)) + (g & ((1 << LT) - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uint64_t x = v[r * K + k];
      if (LAST) {
        x = csub2q(x, bk);
        x = x >= q ? x - q : x;
      }
      a[lpad(base + (k << LT))] = x;
    }
  }
}

// Inverse (Gentleman-Sande, psi^-rev twiddles; bit-reversed in, natural out)
// stages with t = 2^L0 .. 2^(L0+S-1): pair (i0, i0 + t), i = i0 >> (l + 1),
// twiddle itw[(N >> (l + 1)) + i].  Groups are {base + k * 2^L0}.
template <int LOGN, int LOGE, int L0, int S>
__device__ __forceinline__ void inv_pass(uint64_t* a, const PENCIL_GLOBAL TW* tw, uint64_t q, const BflyK& bk) {
  using Sh = NttShape<LOGN, LOGE>;
  constexpr int T = Sh::T, G = Sh::E >> S, K = 1 << S;
  const int tid = threadIdx.x;
  uint64_t v[Sh::E];
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const int g = r * T + tid;
    const int base = ((g >> L0) << (L0 + S)) + (g & ((1 << L0) - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) v[r * K + k] = a[lpad(base + (k << L0))];
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int h = 1 << s;
    const int m = (1 << LOGN) >> (L0 + s + 1);
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int blk = (r * T + tid) >> L0;
#pragma unroll
      for (int j = 0; j < (K >> (s + 1)); ++j) {
        const PENCIL_GLOBAL TW* tp = tw + m + (blk << (S - s - 1)) + j;
        const TW w{tp->w, tp->ws};
#pragma unroll
        for (int k = j << (s + 1); k < ((j + 1) << (s + 1)); ++k) {
          if (k & h) continue;
          gs_bfly(v[r * K + k], v[r * K + k + h], w, bk);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const int g = r * T + tid;
    const int base = ((g >> L0) << (L0 + S)) + (g & ((1 << L0) - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) a[lpad(base + (k << L0))] = v[r * K + k];
  }
}

// Forward transform of the LDS polynomial (inputs in [0, q), outputs in [0, q)).
// Callers synchronise before (inputs written) and after (outputs read).
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_fwd(uint64_t* a, const TW* tw_generic, uint64_t q) {
  using Sh = NttShape<LOGN, LOGE>;
  const BflyK bk = bfly_consts(q);
  const PENCIL_GLOBAL TW* tw = gview(tw_generic);
  fwd_pass<LOGN, LOGE, Sh::start(0), Sh::size(0), Sh::NP == 1>(a, tw, q, bk);
  __syncthreads();
  if constexpr (Sh::NP > 1) {
    fwd_pass<LOGN, LOGE, Sh::start(1), Sh::size(1), Sh::NP == 2>(a, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 2) {
    fwd_pass<LOGN, LOGE, Sh::start(2), Sh::size(2), Sh::NP == 3>(a, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 3) {
    fwd_pass<LOGN, LOGE, Sh::start(3), Sh::size(3), true>(a, tw, q, bk);
    __syncthreads();
  }
}

// Inverse transform without the N^-1 factor (inputs in [0, 2q), outputs in [0, 2q)).
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_inv(uint64_t* a, const TW* tw_generic, uint64_t q) {
  using Sh = NttShape<LOGN, LOGE>;
  const BflyK bk = bfly_consts(q);
  const PENCIL_GLOBAL TW* tw = gview(tw_generic);
  inv_pass<LOGN, LOGE, Sh::start(0), Sh::size(0)>(a, tw, q, bk);
  __syncthreads();
  if constexpr (Sh::NP > 1) {
    inv_pass<LOGN, LOGE, Sh::start(1), Sh::size(1)>(a, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 2) {
    inv_pass<LOGN, LOGE, Sh::start(2), Sh::size(2)>(a, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 3) {
    inv_pass<LOGN, LOGE, Sh::start(3), Sh::size(3)>(a, tw, q, bk);
    __syncthreads();
  }
}

// Staging format of the multiply-accumulate operands: (v mod 2^30) | (v >> 30) << 32.
__device__ __forceinline__ uint64_t split30(uint64_t v) { return (v & 0x3FFFFFFFull) | ((v >> 30) << 32); }

// ---------------------------------------------------------- encode helpers
// round(q m / t) mod q_l for m in [0, t): Delta * m + round(rho m / t), rho = q mod t.
__device__ __forceinline__ uint64_t round_rho(uint64_t m, const Consts& C) {
  uint64_t est = __umul64hi(m, C.rho_sh);
  uint64_t r = m * C.rho - est * C.t;  // in [0, 2t)
  if (r >= C.t) {
    r -= C.t;
    est += 1;
  }
  return est + (2 * r > C.t ? 1 : 0);
}

__device__ __forceinline__ uint64_t delta_scale(uint64_t m, uint64_t rr, const LimbConst& lc) {
  return add_mod(mul_shoup(m, lc.delta, lc.delta_sh, lc.q), rr, lc.q);
}

// Value of the forward-encoded A tile `tile` at polynomial slot `slot`
// (App. A's pi_v generalised), or -1 for an empty slot.
__device__ __forceinline__ int64_t a_slot_offset(const Geo& G, const View& V, int64_t tile, int slot) {
  int mm = slot / G.RS;
  int rem = slot - mm * G.RS;
  if (mm >= G.mt || rem >= G.S) return -1;
  const int hw = G.ha * G.wa;
  int kk = rem / hw;
  int rem2 = rem - kk * hw;
  int ya = rem2 / G.wa, xa = rem2 - (rem2 / G.wa) * G.wa;
  // tile index = ((((mi*nK + ki)*nOY + oyi)*nOX + oxi)*nKY + kyi)*nKX + kxi
  int64_t ti = tile;
  int kxi = (int)(ti % G.nKX); ti /= G.nKX;
  int kyi = (int)(ti % G.nKY); ti /= G.nKY;
  int oxi = (int)(ti % G.nOX); ti /= G.nOX;
  int oyi = (int)(ti % G.nOY); ti /= G.nOY;
  int ki = (int)(ti % G.nK); ti /= G.nK;
  int mi = (int)ti;
  int m = mi * G.mt + mm, k = ki * G.kt + kk;
  int y = oyi * G.oh + kyi * G.kh + ya, x = oxi * G.ow + kxi * G.kw + xa;
  if (m >= G.M || k >= G.K || y >= G.HA || x >= G.WA) return -1;
  int ys = y - V.pady, xs = x - V.pad;
  if (ys < 0 || xs < 0 || ys >= V.H || xs >= V.W) return -1;
  return m * V.s0 + k * V.s1 + ys * V.sy + xs * V.sx;
}

// Value offset of the reverse-encoded K tile `tile` at `slot` (App. A's pi_W).
__device__ __forceinline__ int64_t k_slot_offset(const Geo& G, const View& V, int64_t tile, int slot) {
  // slot = O + rr*S - (kk*ha*wa + dy*wa + dx)
  int z = slot - G.O + G.S - 1;
  if (z < 0) return -1;
  int rr = z / G.S;
  if (rr >= G.rt) return -1;
  int D = rr * G.S + G.O - slot;
  const int hw = G.ha * G.wa;
  int kk = D / hw;
  int rem = D - kk * hw;
  int dy = rem / G.wa, dx = rem - (rem / G.wa) * G.wa;
  if (dy >= G.kh || dx >= G.kw) return -1;
  int64_t ti = tile;  // ((ri*nK + ki)*nKY + kyi)*nKX + kxi
  int kxi = (int)(ti % G.nKX); ti /= G.nKX;
  int kyi = (int)(ti % G.nKY); ti /= G.nKY;
  int ki = (int)(ti % G.nK); ti /= G.nK;
  int ri = (int)ti;
  int r = ri * G.rt + rr, k = ki * G.kt + kk, a = kyi * G.kh + dy, b = kxi * G.kw + dx;
  if (r >= G.R || k >= G.K || a >= G.KH || b >= G.KW) return -1;
  if (V.flip) {
    a = V.KH - 1 - a;
    b = V.KW - 1 - b;
  }
  return r * V.s0 + k * V.s1 + a * V.sy + b * V.sx;
}

__device__ __forceinline__ int64_t slot_offset(int side, const Geo& G, const View& V, int64_t tile, int slot) {
  return side == 0 ? a_slot_offset(G, V, tile, slot) : k_slot_offset(G, V, tile, slot);
}

// ------------------------------------------------------------------ kernels

// In-place forward or inverse NTT of [polys][L][N].
template <int LOGN, int LOGE>
__device__ __forceinline__ void do_ntt_plain(uint64_t* lds, uint64_t* data, int inverse, const Consts& C,
                                             const Tables& T, int64_t p) {
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int l = (int)(p % L);
  const LimbConst& lc = C.limb[l];
  // residues move in 16-byte pairs; a pair never straddles an LDS pad word
  PENCIL_GLOBAL u64x2* g = (PENCIL_GLOBAL u64x2*)gview(data + p * n);
  for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
    const u64x2 v = g[i];
    lds[lpad(2 * i)] = v[0];
    lds[lpad(2 * i) + 1] = v[1];
  }
  __syncthreads();
  if (!inverse) {
    ntt_fwd<LOGN, LOGE>(lds, T.fw + (int64_t)l * n, lc.q);
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x) g[i] = u64x2{lds[lpad(2 * i)], lds[lpad(2 * i) + 1]};
  } else {
    ntt_inv<LOGN, LOGE>(lds, T.iw + (int64_t)l * n, lc.q);
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x)
      g[i] = u64x2{mul_shoup(lds[lpad(2 * i)], lc.ninv, lc.ninv_sh, lc.q),
                   mul_shoup(lds[lpad(2 * i) + 1], lc.ninv, lc.ninv_sh, lc.q)};
  }
}

template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512, (LOGE >= 5 ? 2 : 4)) k_ntt_plain(uint64_t* data, int inverse, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_plain<LOGN, LOGE>(lds, data, inverse, C, T, blockIdx.x);
}

// Input ciphertexts (NTT domain): component 0 gains the transform of
// round(q m / t) of the model owner's share (Alg. 1, product step); the
// residues are stored split for the multiply-accumulate.  Only a block with a
// share to add runs a transform; the others convert and copy.
// Grid: n_ct * 2 * L blocks, polynomial p = (j, c, l) in [n][2][L] order.
template <int LOGN, int LOGE>
__device__ __forceinline__ void do_ntt_ct(uint64_t* lds, const uint64_t* src, uint64_t* dst, const int64_t* share,
                                          const Geo& G, const View& V, const Consts& C, const Tables& T, int64_t p) {
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int l = (int)(p % L);
  const int c = (int)((p / L) % 2);
  const int64_t j = p / (2 * L);
  const LimbConst& lc = C.limb[l];
  const PENCIL_GLOBAL uint64_t* g = gview(src + p * n);
  PENCIL_GLOBAL uint64_t* o = gview(dst + p * n);
  if (share == nullptr || c != 0) {  // 16-byte accesses: a polynomial is 16-byte aligned
    const PENCIL_GLOBAL u64x2* g2 = (const PENCIL_GLOBAL u64x2*)g;
    PENCIL_GLOBAL u64x2* o2 = (PENCIL_GLOBAL u64x2*)o;
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
      const u64x2 v = g2[i];
      o2[i] = u64x2{split30(v[0]), split30(v[1])};
    }
    return;
  }
  const PENCIL_GLOBAL int64_t* gshare = gview(share);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t v = 0;
    const int64_t off = a_slot_offset(G, V, j, i);
    if (off >= 0) {
      const uint64_t m = (uint64_t)gshare[off];
      v = delta_scale(m, round_rho(m, C), lc);
    }
    lds[lpad(i)] = v;
  }
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, T.fw + (int64_t)l * n, lc.q);
  {
    const PENCIL_GLOBAL u64x2* g2 = (const PENCIL_GLOBAL u64x2*)g;
    PENCIL_GLOBAL u64x2* o2 = (PENCIL_GLOBAL u64x2*)o;
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
      const u64x2 v = g2[i];
      o2[i] = u64x2{split30(add_mod(v[0], lds[lpad(2 * i)], lc.q)), split30(add_mod(v[1], lds[lpad(2 * i) + 1], lc.q))};
    }
  }
}

template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512, (LOGE >= 5 ? 2 : 4)) k_ntt_ct(const uint64_t* src, uint64_t* dst, const int64_t* share, Geo G,
                                                 View V, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_ct<LOGN, LOGE>(lds, src, dst, share, G, V, C, T, blockIdx.x);
}

// Plaintext tiles: encode (side 0: forward A tile, 1: reverse K tile), centred
// lift of Z_t into Z_{q_l}, forward NTT.  Grid: n_pt * L, output [n][L][N].
template <int LOGN, int LOGE>
__device__ __forceinline__ void do_ntt_pt(uint64_t* lds, const int64_t* tensor, uint64_t* dst, int side,
                                          const Geo& G, const View& V, const Consts& C, const Tables& T, int64_t p) {
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int l = (int)(p % L);
  const int64_t j = p / L;
  const LimbConst& lc = C.limb[l];
  const PENCIL_GLOBAL int64_t* gt = gview(tensor);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t v = 0;
    int64_t off = slot_offset(side, G, V, j, i);
    if (off >= 0) {
      uint64_t w = (uint64_t)gt[off];
      v = w <= C.t_half ? w : lc.q - (C.t - w);
    }
    lds[lpad(i)] = v;
  }
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, T.fw + (int64_t)l * n, lc.q);
  PENCIL_GLOBAL uint64_t* o = gview(dst + p * n);
  PENCIL_GLOBAL u64x2* o2 = (PENCIL_GLOBAL u64x2*)o;
  for (int i = threadIdx.x; i < n / 2; i += blockDim.x)
    o2[i] = u64x2{split30(lds[lpad(2 * i)]), split30(lds[lpad(2 * i) + 1])};
}

template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512, (LOGE >= 5 ? 2 : 4)) k_ntt_pt(const int64_t* tensor, uint64_t* dst, int side, Geo G, View V,
                                                 Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_pt<LOGN, LOGE>(lds, tensor, dst, side, G, V, C, T, blockIdx.x);
}

// Fresh ternary polynomials (object obj_base + j, stream `purpose`), lifted and
// transformed.  Coefficient i uses the 32-bit half i mod 2 of stream word i/2,
// so one Philox block covers 8 coefficients.  Grid: count * L, output [n][L][N],
// in the multiply-accumulate's split form when `split` is set.
template <int LOGN, int LOGE>
__device__ __forceinline__ void do_ntt_ternary(uint64_t* lds, uint64_t* dst, uint64_t nonce, uint64_t obj_base,
                                               uint32_t purpose, int split, const Consts& C, const Tables& T,
                                               int64_t p) {
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int l = (int)(p % L);
  const int64_t j = p / L;
  const LimbConst& lc = C.limb[l];
  for (int blk = threadIdx.x; blk < n / 8; blk += blockDim.x) {
    U64x4 w = philox((uint64_t)blk, obj_base + j, purpose, 0, C.seed, nonce);
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      uint32_t half = (uint32_t)(w.v[h >> 1] >> (32 * (h & 1)));
      lds[lpad(blk * 8 + h)] = small_to_mod(ternary32(half), lc.q);
    }
  }
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, T.fw + (int64_t)l * n, lc.q);
  PENCIL_GLOBAL u64x2* o2 = (PENCIL_GLOBAL u64x2*)gview(dst + p * n);
  if (split)
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x)
      o2[i] = u64x2{split30(lds[lpad(2 * i)]), split30(lds[lpad(2 * i) + 1])};
  else
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x) o2[i] = u64x2{lds[lpad(2 * i)], lds[lpad(2 * i) + 1]};
}

template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512, (LOGE >= 5 ? 2 : 4)) k_ntt_ternary(uint64_t* dst, uint64_t nonce, uint64_t obj_base,
                                                      uint32_t purpose, int split, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  do_ntt_ternary<LOGN, LOGE>(lds, dst, nonce, obj_base, purpose, split, C, T, blockIdx.x);
}

// LDS-staged multiply-accumulate.  The forward NTTs of the product path store
// each residue v < 2^61 split as (v mod 2^30) | (v >> 30) << 32, so a modular
// product-accumulate is four 32 x 32 -> 64-bit multiply-adds into three 64-bit
// partial sums (low x low, cross terms, high x high).  Every `mac_fold` steps
// the partial sums fold into a 128-bit total, which is Barrett-reduced every
// `mac_chunk` folds and at the end.
//
// A block owns 64 NTT slots of one limb and a ROWS x COLS chunk of (A-row,
// K-row) output tiles.  It walks the contraction (product terms x contraction
// tiles) KB steps at a time: all 512 threads first stage the chunk's A and K
// values of KB steps for their 64 slots in LDS, then each wave accumulates a
// 2 x 2 block of its slot's outputs (both components).  Chunk shapes are
// schedule variants with the same result: 0 = 4 x 8, 1 = 2 x 16, 2 = 8 x 4.
// Staging addresses advance by precomputed strides (no division per step).
constexpr int kMacSlots = 64, kMacKB = 4;
constexpr int kMacSmemWords = kMacKB * 2 * 18 * kMacSlots;  // ROWS + COLS <= 18

struct Acc {
  uint64_t s0, s1, s2;  // partial sums of a0 b0, a0 b1 + a1 b0, a1 b1
  uint64_t lo, hi;      // folded 128-bit total
};

__device__ __forceinline__ void acc_mac(Acc& x, uint64_t a, uint64_t b) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  x.s0 += (uint64_t)a0 * b0;
  x.s1 += (uint64_t)a0 * b1;
  // keeps the two middle products as two multiply-adds into s1 (summing them
  // first would cost a separate 64-bit add)
  asm volatile("" : "+v"(x.s1));
  x.s1 += (uint64_t)a1 * b0;
  x.s2 += (uint64_t)a1 * b1;
}

// total += s0 + s1 2^30 + s2 2^60; the partial sums restart at zero.
__device__ __forceinline__ void acc_fold(Acc& x) {
  const uint64_t t1 = x.s1 << 30, t2 = x.s2 << 60;
  uint64_t lo = x.lo + x.s0;
  uint64_t c = lo < x.s0 ? 1 : 0;
  lo += t1;
  c += lo < t1 ? 1 : 0;
  lo += t2;
  c += lo < t2 ? 1 : 0;
  x.hi += c + (x.s1 >> 34) + (x.s2 >> 4);
  x.lo = lo;
  x.s0 = x.s1 = x.s2 = 0;
}

// Fold every accumulator of a wave's block (every mac_fold steps) and
// Barrett-reduce one of them: accumulator i at fold i of each period of
// mac_chunk folds (mac_chunk >= 8 >= the accumulator count), so each total is
// reduced once per period while only one reduction's temporaries are live.
template <int TM, int TR, int NC>
__device__ __forceinline__ void acc_fold_all(Acc (&acc)[TM][TR][NC], uint32_t& nfold, uint32_t reduce_every,
                                             const LimbConst& lc) {
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c2 = 0; c2 < TR; ++c2)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc_fold(acc[a][c2][c]);
  const uint32_t f = nfold;
  nfold = f + 1 == reduce_every ? 0 : f + 1;
  switch (f) {
#define PENCIL_REDUCE_CASE(i)                                                    \
  case i:                                                                        \
    if (i < TM * TR * NC) {                                                      \
      Acc& x = acc[(i / (NC * TR)) % TM][(i / NC) % TR][i % NC];                  \
      x.lo = reduce128(x.hi, x.lo, lc.q, lc.mu_lo, lc.mu_hi);                     \
      x.hi = 0;                                                                  \
    }                                                                            \
    break;
    PENCIL_REDUCE_CASE(0)
    PENCIL_REDUCE_CASE(1)
    PENCIL_REDUCE_CASE(2)
    PENCIL_REDUCE_CASE(3)
    PENCIL_REDUCE_CASE(4)
    PENCIL_REDUCE_CASE(5)
    PENCIL_REDUCE_CASE(6)
    PENCIL_REDUCE_CASE(7)
#undef PENCIL_REDUCE_CASE
    default: break;
  }
}

// Loop-invariant facts of one block's share of the multiply-accumulate.
struct MacBlock {
  int64_t ln;           // limb * n + first slot of the block
  int64_t ct_stride, pt_stride;
  int row0, col0;       // chunk origin
  int rg, cg;           // this wave's first row and column in the chunk
  int s, grp;           // lane slot, wave index
  int comp;             // the ciphertext component of a one-component wave
  bool active;          // this wave's 2 x 2 block holds at least one real output
  uint32_t nmac, nfold; // steps since the last fold, folds since the last reduction
};

template <int ROWS, int COLS, bool A_CT>
__device__ __forceinline__ void mac_term(uint64_t* smem, const MacTerm& T, const MacArgs& A, const Geo& G,
                                         const Consts& C, const LimbConst& lc, MacBlock& B, Acc (&acc)[2][2][2]) {
  constexpr int TM = 2, TR = 2, KB = kMacKB;
  constexpr int KC = COLS > 8 ? 2 : 1;  // K columns staged per wave
  uint64_t(*sa)[2][ROWS][kMacSlots] = reinterpret_cast<uint64_t(*)[2][ROWS][kMacSlots]>(smem);
  uint64_t(*sk)[2][COLS][kMacSlots] =
      reinterpret_cast<uint64_t(*)[2][COLS][kMacSlots]>(smem + KB * 2 * ROWS * kMacSlots);
  const int sp = G.nOY * G.nOX, kspan = G.nKY * G.nKX;
  const int ksteps = G.nK * kspan;
  const int64_t sa_str = A_CT ? B.ct_stride : B.pt_stride, sk_str = A_CT ? B.pt_stride : B.ct_stride;
  const int grp = B.grp, s = B.s;
  // The A row this wave stages: tile index ((mi nK + ki) sp + rsp) kspan + kk
  // = arow + ki sp kspan + kk, with arow = (mi nK sp + rsp) kspan.
  const int srow = B.row0 + grp;
  const bool have_a = grp < ROWS && srow < A.m_rows;
  const PENCIL_GLOBAL uint64_t* pa = gview(T.a) + B.ln + s;
  if (have_a) {
    const int mi = srow / sp, rsp = srow % sp;
    pa += (((int64_t)mi * G.nK * sp + rsp) * kspan) * sa_str;
  }
  const int64_t a_step = sa_str, a_wrap = ((int64_t)(sp - 1) * kspan + 1) * sa_str;
  // The K columns this wave stages: tile index col ksteps + (ki kspan + kk).
  bool have_k[KC];
  const PENCIL_GLOBAL uint64_t* pk[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    const int cc = grp + 8 * j, col = B.col0 + cc;
    have_k[j] = cc < COLS && col < G.nR;
    pk[j] = gview(T.k) + B.ln + s + (have_k[j] ? (int64_t)col * ksteps * sk_str : 0);
  }
  const uint32_t fold_every = C.mac_fold, reduce_every = C.mac_chunk;
  int kk = 0;
  for (int k0 = 0; k0 < ksteps; k0 += KB) {
    __syncthreads();
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      if (k0 + b < ksteps) {
        if (have_a) {
          sa[b][0][grp][s] = pa[0];
          if (A_CT) sa[b][1][grp][s] = pa[B.pt_stride];
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          if (have_k[j]) {
            sk[b][0][grp + 8 * j][s] = pk[j][0];
            if (!A_CT) sk[b][1][grp + 8 * j][s] = pk[j][B.pt_stride];
          }
          pk[j] += sk_str;
        }
        if (++kk == kspan) {
          kk = 0;
          pa += a_wrap;
        } else {
          pa += a_step;
        }
      }
    }
    __syncthreads();
    if (!B.active) continue;
#pragma unroll 1
    for (int b = 0; b < KB; ++b) {
      if (k0 + b >= ksteps) break;
      uint64_t av[TM][2], kv[TR][2];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        av[a][0] = sa[b][0][B.rg + a][s];
        av[a][1] = A_CT ? sa[b][1][B.rg + a][s] : av[a][0];
      }
#pragma unroll
      for (int c2 = 0; c2 < TR; ++c2) {
        kv[c2][0] = sk[b][0][B.cg + c2][s];
        kv[c2][1] = A_CT ? kv[c2][0] : sk[b][1][B.cg + c2][s];
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c2 = 0; c2 < TR; ++c2)
#pragma unroll
          for (int c = 0; c < 2; ++c) acc_mac(acc[a][c2][c], av[a][c], kv[c2][c]);
      if (++B.nmac == fold_every) {
        B.nmac = 0;
        acc_fold_all<TM, TR, 2>(acc, B.nfold, reduce_every, lc);
      }
    }
  }
}

template <int TM, int TR, int NC, bool A_CT>
__device__ __forceinline__ void mac_term_direct(const MacTerm& T, const MacArgs& A, const Geo& G, const Consts& C,
                                                const LimbConst& lc, MacBlock& B, Acc (&acc)[TM][TR][NC]);

// One block's multiply-accumulate: chunk ROWS x COLS, each wave a TM x TR
// block of it for both ciphertext components (NC = 2) or one (NC = 1, the
// block's waves alternate components); operands staged in LDS or (DIRECT)
// loaded by each wave.
template <int ROWS, int COLS, int TM, int TR, int NC, bool DIRECT>
__device__ __forceinline__ void do_mac_t(uint64_t* smem, const MacArgs& A, const Geo& G, const Consts& C,
                                         int slot_block, int chunk) {
  constexpr int WC = COLS / TR;
  static_assert(DIRECT || (TM == 2 && TR == 2 && NC == 2), "LDS staging uses 2 x 2 two-component wave blocks");
  static_assert((ROWS / TM) * WC * (2 / NC) == 8, "8 waves per block");
  static_assert(ROWS + COLS <= 18 && ROWS <= 8 && COLS <= 16, "staging layout");
  const int n = C.n, L = C.L;
  const int per_limb = n / kMacSlots;
  const int l = slot_block / per_limb;
  const LimbConst& lc = C.limb[l];
  const int cchunks = (G.nR + COLS - 1) / COLS;
  MacBlock B;
  B.row0 = (chunk / cchunks) * ROWS;
  B.col0 = (chunk % cchunks) * COLS;
  B.s = threadIdx.x & (kMacSlots - 1);
  // wave-uniform: the row and column bookkeeping below runs on the scalar unit
  B.grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  B.comp = NC == 1 ? (B.grp & 1) : 0;
  const int tile = NC == 1 ? B.grp >> 1 : B.grp;
  B.rg = (tile / WC) * TM;
  B.cg = (tile % WC) * TR;
  B.ln = (int64_t)l * n + (int64_t)(slot_block % per_limb) * kMacSlots;
  B.ct_stride = 2 * (int64_t)L * n;
  B.pt_stride = (int64_t)L * n;
  B.active = B.row0 + B.rg < A.m_rows && B.col0 + B.cg < G.nR;
  B.nmac = B.nfold = 0;

  Acc acc[TM][TR][NC];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[a][b][c] = Acc{0, 0, 0, 0, 0};
  if constexpr (DIRECT) {
    if (!B.active) return;
    for (int tt = 0; tt < A.n_terms; ++tt) {
      if (A.term[tt].a_is_ct)
        mac_term_direct<TM, TR, NC, true>(A.term[tt], A, G, C, lc, B, acc);
      else
        mac_term_direct<TM, TR, NC, false>(A.term[tt], A, G, C, lc, B, acc);
    }
  } else {
    for (int tt = 0; tt < A.n_terms; ++tt) {
      if (A.term[tt].a_is_ct)
        mac_term<ROWS, COLS, true>(smem, A.term[tt], A, G, C, lc, B, acc);
      else
        mac_term<ROWS, COLS, false>(smem, A.term[tt], A, G, C, lc, B, acc);
    }
  }
  if (!B.active) return;
  // re-randomisation term pk_c * u'_o, reduction and store
  const int64_t ln = B.ln, pt_stride = B.pt_stride, ct_stride = B.ct_stride;
  const int s = B.s, sp = G.nOY * G.nOX;
  const PENCIL_GLOBAL uint64_t* gpk = gview(A.pk);
  const PENCIL_GLOBAL uint64_t* gu = gview(A.u);
  PENCIL_GLOBAL uint64_t* gout = gview(A.out);
  const uint64_t pk0 = gpk[ln + s], pk1 = gpk[pt_stride + ln + s];
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int row = B.row0 + B.rg + a;
    if (row >= A.m_rows) continue;
    const int mi = row / sp, oyi = (row % sp) / G.nOX, oxi = row % G.nOX;
#pragma unroll
    for (int b = 0; b < TR; ++b) {
      const int col = B.col0 + B.cg + b;
      if (col >= G.nR) continue;
      const int64_t o = (((int64_t)mi * G.nR + col) * G.nOY + oyi) * G.nOX + oxi;
      const uint64_t u = gu[o * pt_stride + ln + s];
#pragma unroll
      for (int ci = 0; ci < NC; ++ci) {
        // one more step (the partial sums hold fewer than mac_fold steps)
        const int c = NC == 1 ? B.comp : ci;
        Acc& x = acc[a][b][ci];
        acc_mac(x, c ? pk1 : pk0, u);
        acc_fold(x);
        gout[o * ct_stride + (int64_t)c * pt_stride + ln + s] = reduce128(x.hi, x.lo, lc.q, lc.mu_lo, lc.mu_hi);
      }
    }
  }
}

// The same chunks without LDS: each wave loads the operands of its 2 x 2 block
// straight from memory (the block's other waves read the same rows and columns
// through L1) with the next step's loads in flight while the current step is
// accumulated.  No barriers, so waves run independently.
template <int TM, int TR, int NC, bool A_CT>
__device__ __forceinline__ void mac_term_direct(const MacTerm& T, const MacArgs& A, const Geo& G, const Consts& C,
                                                const LimbConst& lc, MacBlock& B, Acc (&acc)[TM][TR][NC]) {
  const int sp = G.nOY * G.nOX, kspan = G.nKY * G.nKX;
  const int ksteps = G.nK * kspan;
  const int64_t sa_str = A_CT ? B.ct_stride : B.pt_stride, sk_str = A_CT ? B.pt_stride : B.ct_stride;
  const int64_t pt_stride = B.pt_stride;
  // Rows or columns past the end read row 0 / column 0 of the chunk instead
  // (valid memory); their sums are never stored.
  const PENCIL_GLOBAL uint64_t* pa[TM];
  const PENCIL_GLOBAL uint64_t* pk[TR];
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    int row = B.row0 + B.rg + a;
    if (row >= A.m_rows) row = B.row0 + B.rg;
    const int mi = row / sp, rsp = row % sp;
    pa[a] = gview(T.a) + B.ln + B.s + (((int64_t)mi * G.nK * sp + rsp) * kspan) * sa_str;
    if (NC == 1 && A_CT) pa[a] += B.comp * pt_stride;  // this wave's component
  }
#pragma unroll
  for (int c2 = 0; c2 < TR; ++c2) {
    int col = B.col0 + B.cg + c2;
    if (col >= G.nR) col = B.col0 + B.cg;
    pk[c2] = gview(T.k) + B.ln + B.s + (int64_t)col * ksteps * sk_str;
    if (NC == 1 && !A_CT) pk[c2] += B.comp * pt_stride;
  }
  const int64_t a_wrap = ((int64_t)(sp - 1) * kspan + 1) * sa_str;
  const uint32_t fold_every = C.mac_fold, reduce_every = C.mac_chunk;
  int kk = 0, left = ksteps;  // steps not yet loaded
  // Four operand sets rotate so that the loads of the next three steps are in
  // flight while the current one accumulates (no register copies between
  // them).  Loads are unconditional: past the last step the pointers stop
  // advancing and the last step is read again, so no branch separates a load
  // from its use.
  uint64_t xa[TM][NC], xk[TR][NC], ya[TM][NC], yk[TR][NC], za[TM][NC], zk[TR][NC], wa[TM][NC], wk[TR][NC];
  auto load = [&](uint64_t(&va)[TM][NC], uint64_t(&vk)[TR][NC]) {
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      va[a][0] = pa[a][0];
      if (NC == 2) va[a][NC - 1] = A_CT ? pa[a][pt_stride] : va[a][0];
    }
#pragma unroll
    for (int c2 = 0; c2 < TR; ++c2) {
      vk[c2][0] = pk[c2][0];
      if (NC == 2) vk[c2][NC - 1] = A_CT ? vk[c2][0] : pk[c2][pt_stride];
    }
    const bool adv = --left > 0;
    const int64_t da = !adv ? 0 : (kk + 1 == kspan) ? a_wrap : sa_str;
    const int64_t dk = adv ? sk_str : 0;
    kk = (kk + 1 == kspan) ? 0 : kk + 1;
#pragma unroll
    for (int a = 0; a < TM; ++a) pa[a] += da;
#pragma unroll
    for (int c2 = 0; c2 < TR; ++c2) pk[c2] += dk;
  };
  auto step = [&](const uint64_t(&va)[TM][NC], const uint64_t(&vk)[TR][NC]) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int c2 = 0; c2 < TR; ++c2)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc_mac(acc[a][c2][c], va[a][c], vk[c2][c]);
    if (++B.nmac == fold_every) {
      B.nmac = 0;
      acc_fold_all<TM, TR, NC>(acc, B.nfold, reduce_every, lc);
    }
  };
  load(xa, xk);
  load(ya, yk);
  load(za, zk);
  for (int k = 0; k < ksteps; k += 4) {
    load(wa, wk);
    step(xa, xk);
    if (k + 1 >= ksteps) break;
    load(xa, xk);
    step(ya, yk);
    if (k + 2 >= ksteps) break;
    load(ya, yk);
    step(za, zk);
    if (k + 3 >= ksteps) break;
    load(za, zk);
    step(wa, wk);
  }
}

// Kind 0: LDS-staged 2 x 2 wave blocks, both components; 1: direct, the same;
// 2: direct 2 x 2 wave blocks of one component each.
template <int KIND>
__device__ __forceinline__ void do_mac(uint64_t* smem, const MacArgs& A, const Geo& G, const Consts& C,
                                       int slot_block, int chunk) {
  constexpr bool DIRECT = KIND != 0;
  constexpr int NC = KIND == 2 ? 1 : 2;
  switch (A.variant % 3) {
    case 1: do_mac_t<2, KIND == 2 ? 8 : 16, 2, 2, NC, DIRECT>(smem, A, G, C, slot_block, chunk); break;
    case 2: do_mac_t<8, KIND == 2 ? 2 : 4, 2, 2, NC, DIRECT>(smem, A, G, C, slot_block, chunk); break;
    default: do_mac_t<4, KIND == 2 ? 4 : 8, 2, 2, NC, DIRECT>(smem, A, G, C, slot_block, chunk); break;
  }
}

// Work item of block `b` of `total`.  Workgroups go to the 8 XCDs round-robin
// by block index, so XCD x = b mod 8 receives blocks b = x, x + 8, ...; giving
// it the contiguous work range [x total / 8, (x + 1) total / 8) in order keeps
// the chunks of one slot range (which share operands) on one L2.
__device__ __forceinline__ int64_t xcd_work(int64_t b, int64_t total) {
  const int64_t q = total >> 3, r = total & 7, x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

__global__ void __launch_bounds__(512) k_mac_lds(MacArgs A, Geo G, Consts C, int chunks, int64_t total) {
  extern __shared__ uint64_t smem[];
  const int w = (int)xcd_work(blockIdx.x, total);
  do_mac<0>(smem, A, G, C, w / chunks, w % chunks);
}

__global__ void __launch_bounds__(512) k_mac_direct(MacArgs A, Geo G, Consts C, int chunks, int64_t total) {
  const int w = (int)xcd_work(blockIdx.x, total);
  do_mac<1>(nullptr, A, G, C, w / chunks, w % chunks);
}

__global__ void __launch_bounds__(512) k_mac_direct_small(MacArgs A, Geo G, Consts C, int chunks, int64_t total) {
  const int w = (int)xcd_work(blockIdx.x, total);
  do_mac<2>(nullptr, A, G, C, w / chunks, w % chunks);
}


// Output ciphertexts after the inverse NTT: c0 += e0' + flood - round(q s / t),
// c1 += e1'; the model owner's share is s at the output slots (+ bias).
// Each thread handles 4 consecutive coefficients of one output ciphertext.
template <int W>
__device__ __forceinline__ void do_flood(uint64_t* ct, int64_t n_out, int64_t* share0, const int64_t* bias,
                                         const Geo& G, const View& OV, uint64_t nonce, uint64_t obj_base,
                                         const Consts& C, int64_t g) {
  const int n = C.n, L = C.L;
  const int per = n / 4;
  if (g >= n_out * per) return;
  const int64_t o = g / per;
  const int n0 = (int)(g % per) * 4;
  const uint64_t obj = obj_base + (uint64_t)o;
  const uint64_t blk4 = (uint64_t)(n0 / 4);
  U64x4 e0 = philox(blk4, obj, P_RR_E0, 0, C.seed, nonce);
  U64x4 e1 = philox(blk4, obj, P_RR_E1, 0, C.seed, nonce);
  U64x4 mk0 = philox(2 * blk4, obj, P_MASK, 0, C.seed, nonce);
  U64x4 mk1 = philox(2 * blk4 + 1, obj, P_MASK, 0, C.seed, nonce);
  uint64_t fw[4 * W];  // the 4W flood words of these 4 coefficients, in stream order
#pragma unroll
  for (int b = 0; b < W; ++b) {
    U64x4 f = philox(blk4 * W + b, obj, P_FLOOD, 0, C.seed, nonce);
#pragma unroll
    for (int z = 0; z < 4; ++z) fw[b * 4 + z] = f.v[z];
  }
  const int64_t ct_stride = 2 * (int64_t)L * n;
  PENCIL_GLOBAL uint64_t* c0p = gview(ct) + o * ct_stride;
  PENCIL_GLOBAL uint64_t* c1p = c0p + (int64_t)L * n;
  // output-tile coordinates of o = ((mi*nR + ri)*nOY + oyi)*nOX + oxi
  int64_t ti = o;
  const int oxi = (int)(ti % G.nOX);
  ti /= G.nOX;
  const int oyi = (int)(ti % G.nOY);
  ti /= G.nOY;
  const int ri = (int)(ti % G.nR);
  const int mi = (int)(ti / G.nR);
  // per-coefficient draws: re-randomisation errors, the mask s = (wlo + 2^64 whi) mod t
  int64_t ev0[4], ev1[4];
  uint64_t sv[4], rrv[4];
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    ev0[z] = cbd21(e0.v[z]);
    ev1[z] = cbd21(e1.v[z]);
    const uint64_t wlo = (z < 2 ? mk0 : mk1).v[(2 * z) & 3], whi = (z < 2 ? mk0 : mk1).v[(2 * z + 1) & 3];
    uint64_t sh = reduce64(whi, C.one_sh_t, C.t);
    uint64_t sz = mul_shoup(sh, C.r64t, C.r64t_sh, C.t) + reduce64(wlo, C.one_sh_t, C.t);
    if (sz >= C.t) sz -= C.t;
    sv[z] = sz;
    rrv[z] = round_rho(sz, C);
  }
  // the thread's 4 consecutive coefficients of each limb move as two 16-byte words
  for (int l = 0; l < L; ++l) {
    const LimbConst& lc = C.limb[l];
    PENCIL_GLOBAL u64x2* p0 = (PENCIL_GLOBAL u64x2*)(c0p + (int64_t)l * n + n0);
    PENCIL_GLOBAL u64x2* p1 = (PENCIL_GLOBAL u64x2*)(c1p + (int64_t)l * n + n0);
    const u64x2 a0 = p0[0], a1 = p0[1], b0 = p1[0], b1 = p1[1];
    uint64_t x0[4] = {a0.x, a0.y, a1.x, a1.y}, x1[4] = {b0.x, b0.y, b1.x, b1.y};
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      // flood value V - 2^fb with V = sum_b w_b 2^(64 b) the low fb+1 bits of the
      // words: sum_b w_b (2^(64 b) mod q) < 2^126 as one 128-bit value, one reduction
      uint64_t hi = 0, lo = fw[z * W];
#pragma unroll
      for (int b = 1; b < W; ++b) {
        uint64_t w = fw[z * W + b];
        if (b == W - 1) w &= C.top_mask;
        uint64_t ph, pl;
        mul_wide(w, b == 1 ? lc.r64 : b == 2 ? lc.r128 : lc.r192, ph, pl);
        lo += pl;
        hi += ph + (lo < pl ? 1 : 0);
      }
      if (W == 1) lo &= C.top_mask;
      uint64_t v = reduce128(hi, lo, lc.q, lc.mu_lo, lc.mu_hi);
      v = sub_mod(v, lc.flood_off, lc.q);
      uint64_t c = add_mod(x0[z], small_to_mod(ev0[z], lc.q), lc.q);
      c = add_mod(c, v, lc.q);
      x0[z] = sub_mod(c, delta_scale(sv[z], rrv[z], lc), lc.q);
      x1[z] = add_mod(x1[z], small_to_mod(ev1[z], lc.q), lc.q);
    }
    p0[0] = u64x2{x0[0], x0[1]};
    p0[1] = u64x2{x0[2], x0[3]};
    p1[0] = u64x2{x1[0], x1[1]};
    p1[1] = u64x2{x1[2], x1[3]};
  }
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    const int i = n0 + z;
    const uint64_t s = sv[z];
    // model owner's share at the output slots: slot = mm*RS + O + rr*S + y*wa + x
    int zz = i - G.O;
    if (zz >= 0) {
      int mm = zz / G.RS;
      int rem = zz - mm * G.RS;
      int rr2 = rem / G.S;
      int rem2 = rem - rr2 * G.S;
      int y = rem2 / G.wa, x = rem2 - (rem2 / G.wa) * G.wa;
      if (mm < G.mt && y < G.oh && x < G.ow) {
        int m = mi * G.mt + mm, r = ri * G.rt + rr2, yy = oyi * G.oh + y, xx = oxi * G.ow + x;
        if (m < G.M && r < G.R && yy < G.OH && xx < G.OW) {
          uint64_t val = s;
          if (bias) {
            val += (uint64_t)gview(bias)[r];
            if (val >= C.t) val -= C.t;
          }
          gview(share0)[m * OV.s0 + r * OV.s1 + yy * OV.sy + xx * OV.sx] = (int64_t)val;
        }
      }
    }
  }
}

template <int W>
__global__ void __launch_bounds__(256) k_flood_mask(uint64_t* ct, int64_t n_out, int64_t* share0,
                                                    const int64_t* bias, Geo G, View OV, uint64_t nonce,
                                                    uint64_t obj_base, Consts C) {
  do_flood<W>(ct, n_out, share0, bias, G, OV, nonce, obj_base, C, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Encryption in the NTT domain: ct_c = pk_c * u + NTT(e_c (+ round(q m / t) on
// c = 0)), with m the encoded share at each slot; the product path consumes
// ciphertexts in this form.  Grid: n_ct * 2 * L, u_ntt is [n][L][N].
template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512, (LOGE >= 5 ? 2 : 4)) k_encrypt(const uint64_t* u_ntt, const int64_t* share, uint64_t* ct, int side,
                                                  Geo G, View V, const uint64_t* pk_ntt, const uint64_t* pk_sh,
                                                  uint64_t nonce, uint64_t obj_base, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int64_t p = blockIdx.x;
  const int l = (int)(p % L);
  const int c = (int)((p / L) % 2);
  const int64_t j = p / (2 * L);
  const LimbConst& lc = C.limb[l];
  const uint64_t* u = u_ntt + (j * L + l) * n;
  const uint64_t* pk = pk_ntt + ((int64_t)c * L + l) * n;
  const uint64_t* pks = pk_sh + ((int64_t)c * L + l) * n;
  const uint64_t obj = obj_base + (uint64_t)j;
  for (int blk = threadIdx.x; blk < n / 4; blk += blockDim.x) {
    U64x4 e = philox((uint64_t)blk, obj, c ? P_ENC_E1 : P_ENC_E0, 0, C.seed, nonce);
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int i = blk * 4 + z;
      uint64_t v = small_to_mod(cbd21(e.v[z]), lc.q);
      if (c == 0) {
        int64_t off = slot_offset(side, G, V, j, i);
        if (off >= 0) {
          uint64_t m = (uint64_t)share[off];
          v = add_mod(v, delta_scale(m, round_rho(m, C), lc), lc.q);
        }
      }
      lds[lpad(i)] = v;
    }
  }
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, T.fw + (int64_t)l * n, lc.q);
  uint64_t* o = ct + p * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    o[i] = add_mod(mul_shoup(u[i], pk[i], pks[i], lc.q), lds[lpad(i)], lc.q);
}

// Decryption phase per limb: x = c0 + INTT(NTT(c1) * s).  Grid: n * L, x is [n][L][N].
template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512) k_phase(const uint64_t* ct, uint64_t* x, const uint64_t* s_ntt,
                                                const uint64_t* s_sh, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int64_t p = blockIdx.x;
  const int l = (int)(p % L);
  const int64_t j = p / L;
  const LimbConst& lc = C.limb[l];
  const uint64_t* c0 = ct + ((j * 2 + 0) * L + l) * n;
  const uint64_t* c1 = ct + ((j * 2 + 1) * L + l) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[lpad(i)] = c1[i];
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, T.fw + (int64_t)l * n, lc.q);
  const uint64_t* sv = s_ntt + (int64_t)l * n;
  const uint64_t* ss = s_sh + (int64_t)l * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[lpad(i)] = mul_shoup(lds[lpad(i)], sv[i], ss[i], lc.q);
  __syncthreads();
  ntt_inv<LOGN, LOGE>(lds, T.iw + (int64_t)l * n, lc.q);
  uint64_t* o = x + p * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    o[i] = add_mod(c0[i], mul_shoup(lds[lpad(i)], lc.ninv, lc.ninv_sh, lc.q), lc.q);
}

// Exact decryption of the output slots: with y_l = x_l * (q/q_l)^-1 mod q_l and
// y_l t = alpha_l q_l + beta_l,  t x / q = sum alpha_l + sum beta_l / q_l - v t,
// so m = (sum alpha_l + round(F / q)) mod t with F = sum beta_l (q / q_l); the
// rounding compares 2F with (2j + 1) q.  One thread per output element.
__global__ void __launch_bounds__(256) k_decode(const uint64_t* x, int64_t* share, int64_t n_out, Geo G, View OV,
                                                Consts C) {
  const int n = C.n, L = C.L;
  const int64_t per = (int64_t)G.mt * G.rt * G.oh * G.ow;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_out * per) return;
  const int64_t o = g / per;
  int e = (int)(g % per);
  const int x_ = e % G.ow;
  e /= G.ow;
  const int y = e % G.oh;
  e /= G.oh;
  const int rr = e % G.rt;
  const int mm = e / G.rt;
  int64_t ti = o;
  const int oxi = (int)(ti % G.nOX);
  ti /= G.nOX;
  const int oyi = (int)(ti % G.nOY);
  ti /= G.nOY;
  const int ri = (int)(ti % G.nR);
  const int mi = (int)(ti / G.nR);
  const int m = mi * G.mt + mm, r = ri * G.rt + rr, yy = oyi * G.oh + y, xx = oxi * G.ow + x_;
  if (m >= G.M || r >= G.R || yy >= G.OH || xx >= G.OW) return;
  const int slot = mm * G.RS + G.O + rr * G.S + y * G.wa + x_;
  uint64_t F[kMaxWords + 1];
#pragma unroll
  for (int w = 0; w <= kMaxWords; ++w) F[w] = 0;
  uint64_t alpha = 0;
  for (int l = 0; l < L; ++l) {
    const LimbConst& lc = C.limb[l];
    const uint64_t xl = x[(o * L + l) * n + slot];
    const uint64_t yl = mul_shoup(xl, lc.qhat_inv, lc.qhat_inv_sh, lc.q);
    uint64_t est = __umul64hi(yl, lc.t_sh);
    uint64_t beta = yl * C.t - est * lc.q;
    if (beta >= lc.q) {
      beta -= lc.q;
      est += 1;
    }
    alpha += est;  // each alpha_l < t
    // F += beta * qhat_l
    uint64_t carry = 0;
#pragma unroll
    for (int w = 0; w < kMaxWords; ++w) {
      uint64_t ph, pl;
      mul_wide(beta, C.qhat[l][w], ph, pl);
      uint64_t s1 = F[w] + pl;
      uint64_t c1 = s1 < pl;
      uint64_t s2 = s1 + carry;
      c1 += s2 < carry;
      F[w] = s2;
      carry = ph + c1;
    }
    F[kMaxWords] += carry;
  }
  // 2F
  uint64_t D[kMaxWords + 1];
  uint64_t prev = 0;
#pragma unroll
  for (int w = 0; w <= kMaxWords; ++w) {
    D[w] = (F[w] << 1) | (prev >> 63);
    prev = F[w];
  }
  uint64_t rnd = 0;
  for (int j = 0; j < L; ++j) {
    // compare D with thr[j] (kMaxWords words; D's top word must be zero for thr to win)
    int gt = D[kMaxWords] != 0 ? 1 : 0;
    if (!gt) {
      gt = 0;
      for (int w = kMaxWords - 1; w >= 0; --w) {
        if (D[w] != C.thr[j][w]) {
          gt = D[w] > C.thr[j][w] ? 1 : 0;
          break;
        }
      }
    }
    rnd += gt;
  }
  uint64_t mres = (alpha % C.t + rnd) % C.t;
  share[m * OV.s0 + r * OV.s1 + yy * OV.sy + xx * OV.sx] = (int64_t)mres;
}

// Key generation, one block per limb: s ternary (stream P_SK), a uniform mod q_l
// (stream P_PK_A, limb l, two words per coefficient), e CBD21 (stream P_PK_E);
// pk = (-(a s + e), a), kept in both coefficient and NTT form.  One LDS buffer;
// every thread re-reads only the global entries it wrote itself.
template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512) k_keygen(uint64_t* s_ntt, int64_t* s_coeff, uint64_t* pk_coeff,
                                                 uint64_t* pk_ntt, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int l = blockIdx.x;
  const LimbConst& lc = C.limb[l];
  const uint64_t nonce = kKeygenNonce;
  const TW* tw = T.fw + (int64_t)l * n;
  for (int blk = threadIdx.x; blk < n / 8; blk += blockDim.x) {
    U64x4 w = philox((uint64_t)blk, 0, P_SK, 0, C.seed, nonce);
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      int64_t sv = ternary32((uint32_t)(w.v[h >> 1] >> (32 * (h & 1))));
      lds[lpad(blk * 8 + h)] = small_to_mod(sv, lc.q);
      if (l == 0) s_coeff[blk * 8 + h] = sv;
    }
  }
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, tw, lc.q);
  for (int i = threadIdx.x; i < n; i += blockDim.x) s_ntt[(int64_t)l * n + i] = lds[lpad(i)];
  __syncthreads();
  for (int blk = threadIdx.x; blk < n / 2; blk += blockDim.x) {
    U64x4 w = philox((uint64_t)blk, 0, P_PK_A, (uint64_t)l, C.seed, nonce);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // (w_lo + 2^64 w_hi) mod q
      uint64_t hi = reduce64(w.v[2 * h + 1], lc.one_sh, lc.q);
      uint64_t v = add_mod(mul_shoup(hi, lc.r64, lc.r64_sh, lc.q), reduce64(w.v[2 * h], lc.one_sh, lc.q), lc.q);
      lds[lpad(blk * 2 + h)] = v;
      pk_coeff[((int64_t)1 * L + l) * n + blk * 2 + h] = v;
    }
  }
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, tw, lc.q);
  // a * s pointwise (128-bit product, Barrett), then inverse transform
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint64_t av = lds[lpad(i)];
    pk_ntt[((int64_t)1 * L + l) * n + i] = av;
    uint64_t ph, pl;
    mul_wide(av, s_ntt[(int64_t)l * n + i], ph, pl);
    lds[lpad(i)] = reduce128(ph, pl, lc.q, lc.mu_lo, lc.mu_hi);
  }
  __syncthreads();
  ntt_inv<LOGN, LOGE>(lds, T.iw + (int64_t)l * n, lc.q);
  for (int blk = threadIdx.x; blk < n / 4; blk += blockDim.x) {
    U64x4 w = philox((uint64_t)blk, 0, P_PK_E, 0, C.seed, nonce);
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int i = blk * 4 + z;
      uint64_t as = mul_shoup(lds[lpad(i)], lc.ninv, lc.ninv_sh, lc.q);
      uint64_t v = add_mod(as, small_to_mod(cbd21(w.v[z]), lc.q), lc.q);
      v = v == 0 ? 0 : lc.q - v;
      lds[lpad(i)] = v;
      pk_coeff[(int64_t)l * n + i] = v;
    }
  }
  __syncthreads();
  ntt_fwd<LOGN, LOGE>(lds, tw, lc.q);
  for (int i = threadIdx.x; i < n; i += blockDim.x) pk_ntt[(int64_t)l * n + i] = lds[lpad(i)];
}

// Exact Z_t packed correlation of two plaintext tensors, one thread per output
// element: out[m, r, y, x] = sum_{k, dy, dx} A[m, k, y+dy, x+dx] K[r, k, dy, dx]
// mod t, with 128-bit accumulation (41-bit operands, < 2^46 terms).  Used for
// the local terms of the weight gradient.
__global__ void __launch_bounds__(256) k_zt_corr(const int64_t* a, const int64_t* kt, int64_t* out, Geo G, View AV,
                                                 View KV, View OV, Consts C) {
  const int64_t total = (int64_t)G.M * G.R * G.OH * G.OW;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int64_t e = g;
  const int x = (int)(e % G.OW);
  e /= G.OW;
  const int y = (int)(e % G.OH);
  e /= G.OH;
  const int r = (int)(e % G.R);
  const int m = (int)(e / G.R);
  uint64_t hi = 0, lo = 0;
  for (int k = 0; k < G.K; ++k)
    for (int dy = 0; dy < G.KH; ++dy) {
      const int ys = y + dy - AV.pady;
      if (ys < 0 || ys >= AV.H) continue;
      for (int dx = 0; dx < G.KW; ++dx) {
        const int xs = x + dx - AV.pad;
        if (xs < 0 || xs >= AV.W) continue;
        const uint64_t av = (uint64_t)a[m * AV.s0 + k * AV.s1 + ys * AV.sy + xs * AV.sx];
        const int ky = KV.flip ? KV.KH - 1 - dy : dy, kx = KV.flip ? KV.KW - 1 - dx : dx;
        const uint64_t kv = (uint64_t)kt[r * KV.s0 + k * KV.s1 + ky * KV.sy + kx * KV.sx];
        uint64_t ph, pl;
        mul_wide(av, kv, ph, pl);
        lo += pl;
        hi += ph + (lo < pl ? 1 : 0);
      }
    }
  // (hi 2^64 + lo) mod t
  uint64_t v = add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t),
                       reduce64(lo, C.one_sh_t, C.t), C.t);
  out[m * OV.s0 + r * OV.s1 + y * OV.sy + x * OV.sx] = (int64_t)v;
}

// The same correlation as a tiled contraction.  A workgroup of nw waves owns a
// (8 TI) x (8 TI) tile of (output position, output channel) pairs, each lane a
// TI x TI block, and the waves split the contraction (k, dy, dx) nw ways.
// Operands (< t < 2^42) are split into 21-bit halves, so a product is four
// 32 x 32 multiply-adds into three 64-bit partial sums that hold 2^22 terms;
// each wave reduces its totals mod t and the waves' results are summed through
// LDS.  The launcher picks TI and nw so that small outputs or short
// contractions still fill the GPU.
constexpr int kZtWaves = 16;
template <int TI>
__global__ void __launch_bounds__(1024) k_zt_gemm(const int64_t* a, const int64_t* kt, int64_t* out, Geo G, View AV,
                                                  View KV, View OV, Consts C) {
  constexpr int NO = 64 * TI * TI;  // outputs per workgroup
  __shared__ uint64_t red[kZtWaves][NO];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int P = G.M * G.OH * G.OW, R = G.R, ohw = G.OH * G.OW;
  const PENCIL_GLOBAL int64_t* ga = gview(a);
  const PENCIL_GLOBAL int64_t* gk = gview(kt);
  int64_t abase[TI];
  int ay[TI], ax[TI];
  bool rv[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const int row = blockIdx.x * 8 * TI + (lane >> 3) * TI + i;
    rv[i] = row < P;
    const int rr = rv[i] ? row : 0;
    const int m = rr / ohw, rem = rr - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
    abase[i] = (int64_t)m * AV.s0;
    ay[i] = y - AV.pady;
    ax[i] = x - AV.pad;
  }
  int64_t kbase[TI];
  bool cv[TI];
#pragma unroll
  for (int j = 0; j < TI; ++j) {
    const int col = blockIdx.y * 8 * TI + (lane & 7) * TI + j;
    cv[j] = col < R;
    kbase[j] = (int64_t)(cv[j] ? col : 0) * KV.s0;
  }
  const int kk = G.KH * G.KW;
  const int64_t ctot = (int64_t)G.K * kk, per = (ctot + nw - 1) / nw;
  const int64_t c_begin = wv * per, c_end = c_begin + per < ctot ? c_begin + per : ctot;
  uint64_t s0[TI][TI] = {}, s1[TI][TI] = {}, s2[TI][TI] = {};
  int k = 0, dy = 0, dx = 0;
  if (c_begin < c_end) {
    k = (int)(c_begin / kk);
    const int rem = (int)(c_begin - (int64_t)k * kk);
    dy = rem / G.KW;
    dx = rem - dy * G.KW;
  }
  constexpr uint64_t kLo = (1ull << 21) - 1;
  // Chunks of U contraction steps: all loads of a chunk are issued before its
  // multiply-adds.
  constexpr int U = 4;
  for (int64_t c0 = c_begin; c0 < c_end; c0 += U) {
    uint64_t av[U][TI], bv[U][TI];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = c0 + u < c_end;
      const int ky = KV.flip ? KV.KH - 1 - dy : dy, kx = KV.flip ? KV.KW - 1 - dx : dx;
      const int64_t koff = (int64_t)k * KV.s1 + (int64_t)ky * KV.sy + (int64_t)kx * KV.sx;
#pragma unroll
      for (int j = 0; j < TI; ++j) bv[u][j] = live && cv[j] ? (uint64_t)gk[kbase[j] + koff] : 0;
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const int ys = ay[i] + dy, xs = ax[i] + dx;
        const bool in = live && rv[i] && ys >= 0 && ys < AV.H && xs >= 0 && xs < AV.W;
        av[u][i] = in ? (uint64_t)ga[abase[i] + (int64_t)k * AV.s1 + (int64_t)ys * AV.sy + (int64_t)xs * AV.sx] : 0;
      }
      if (++dx == G.KW) {
        dx = 0;
        if (++dy == G.KH) {
          dy = 0;
          ++k;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const uint32_t a0 = (uint32_t)(av[u][i] & kLo), a1 = (uint32_t)(av[u][i] >> 21);
#pragma unroll
        for (int j = 0; j < TI; ++j) {
          const uint32_t b0 = (uint32_t)(bv[u][j] & kLo), b1 = (uint32_t)(bv[u][j] >> 21);
          s0[i][j] += (uint64_t)a0 * b0;
          s1[i][j] += (uint64_t)a0 * b1;
          s1[i][j] += (uint64_t)a1 * b0;
          s2[i][j] += (uint64_t)a1 * b1;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TI; ++j) {
      // s0 + s1 2^21 + s2 2^42 as a 128-bit value, then mod t
      const uint64_t t1 = s1[i][j] << 21, t2 = s2[i][j] << 42;
      uint64_t lo = s0[i][j] + t1;
      uint64_t hi = (lo < t1 ? 1 : 0) + (s1[i][j] >> 43) + (s2[i][j] >> 22);
      lo += t2;
      hi += lo < t2 ? 1 : 0;
      red[wv][(lane * TI + i) * TI + j] = add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t),
                                                  reduce64(lo, C.one_sh_t, C.t), C.t);
    }
  __syncthreads();
  for (int o = threadIdx.x; o < NO; o += blockDim.x) {
    const int ol = o / (TI * TI), i = (o / TI) % TI, j = o % TI;
    uint64_t v = 0;
    for (int w = 0; w < nw; ++w) v = add_mod(v, red[w][o], C.t);
    const int row = blockIdx.x * 8 * TI + (ol >> 3) * TI + i, col = blockIdx.y * 8 * TI + (ol & 7) * TI + j;
    if (row < P && col < R) {
      const int m = row / ohw, rem = row - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
      gview(out)[(int64_t)m * OV.s0 + (int64_t)col * OV.s1 + (int64_t)y * OV.sy + (int64_t)x * OV.sx] = (int64_t)v;
    }
  }
}

// The same correlation on the fp64 matrix cores.  Each operand, centred into
// (-t/2, t/2), is split into signed 14-bit digits v = d0 + d1 2^14 + d2 2^28
// (d0, d1 in [0, 2^14), d2 the signed rest); the nine digit products of a pair
// land on five diagonals T_s = sum d_i e_j (i + j = s), each a 16 x 16 x 4
// fp64 multiply-accumulate.  Every digit product and running sum is an
// integer below 2^53 (the launcher bounds the terms per wave), so the fp64
// arithmetic is exact; at the end each T_s is reduced mod t and the five are
// recombined with 2^14s mod t.  A workgroup owns a 16 x 16 output tile and
// splits the contraction over its waves, four contraction indices per step.
// Lane l holds A[row l % 16][c + l / 16] and B[c + l / 16][col l % 16], and
// register r of its accumulator holds output (l / 16 + 4 r, l % 16).
typedef double zt_v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void zt_digits(uint64_t v, const Consts& C, double (&d)[3]) {
  const int64_t c = v > C.t_half ? (int64_t)v - (int64_t)C.t : (int64_t)v;
  const int64_t d0 = c & 0x3FFF, r1 = c >> 14, d1 = r1 & 0x3FFF, d2 = r1 >> 14;
  d[0] = (double)d0;
  d[1] = (double)d1;
  d[2] = (double)d2;
}

__device__ __forceinline__ uint64_t zt_mod_signed(int64_t x, const Consts& C) {
  const uint64_t u = x < 0 ? (uint64_t)(-x) : (uint64_t)x;
  const uint64_t r = reduce64(u, C.one_sh_t, C.t);
  return x < 0 && r ? C.t - r : r;
}

__global__ void __launch_bounds__(1024) k_zt_mfma(const int64_t* a, const int64_t* kt, int64_t* out, Geo G, View AV,
                                                  View KV, View OV, Consts C) {
  __shared__ uint64_t red[kZtWaves][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int P = G.M * G.OH * G.OW, R = G.R, ohw = G.OH * G.OW;
  const PENCIL_GLOBAL int64_t* ga = gview(a);
  const PENCIL_GLOBAL int64_t* gk = gview(kt);
  const int lr = lane & 15, lc = lane >> 4;
  // this lane's A row and B column
  const int row = blockIdx.x * 16 + lr, col = blockIdx.y * 16 + lr;
  const bool rv = row < P, cv = col < R;
  int64_t abase, kbase;
  int ay, ax;
  {
    const int rr = rv ? row : 0;
    const int m = rr / ohw, rem = rr - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
    abase = (int64_t)m * AV.s0;
    ay = y - AV.pady;
    ax = x - AV.pad;
    kbase = (int64_t)(cv ? col : 0) * KV.s0;
  }
  const int kk = G.KH * G.KW;
  const int64_t ctot = (int64_t)G.K * kk;
  const int64_t steps = (ctot + 3) / 4, per = (steps + nw - 1) / nw;
  const int64_t s_begin = wv * per, s_end = s_begin + per < steps ? s_begin + per : steps;
  zt_v4d acc[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) acc[s] = zt_v4d{0, 0, 0, 0};
  constexpr int U = 4;  // contraction steps whose loads are issued together
  for (int64_t st0 = s_begin; st0 < s_end; st0 += U) {
    uint64_t av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = (st0 + u) * 4 + lc;
      const bool live = st0 + u < s_end && c < ctot;
      int k = 0, dy = 0, dx = 0;
      if (kk == 1) {
        k = (int)c;
      } else {
        k = (int)(c / kk);
        const int rem = (int)(c - (int64_t)k * kk);
        dy = rem / G.KW;
        dx = rem - dy * G.KW;
      }
      const int ky = KV.flip ? KV.KH - 1 - dy : dy, kx = KV.flip ? KV.KW - 1 - dx : dx;
      bv[u] = live && cv ? (uint64_t)gk[kbase + (int64_t)k * KV.s1 + (int64_t)ky * KV.sy + (int64_t)kx * KV.sx] : 0;
      const int ys = ay + dy, xs = ax + dx;
      const bool in = live && rv && ys >= 0 && ys < AV.H && xs >= 0 && xs < AV.W;
      av[u] = in ? (uint64_t)ga[abase + (int64_t)k * AV.s1 + (int64_t)ys * AV.sy + (int64_t)xs * AV.sx] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double da[3], db[3];
      zt_digits(av[u], C, da);
      zt_digits(bv[u], C, db);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[i + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(da[i], db[j], acc[i + j], 0, 0, 0);
    }
  }
  // 2^(14 s) mod t
  uint64_t pw[5];
  pw[0] = 1;
#pragma unroll
  for (int s = 1; s < 5; ++s) pw[s] = reduce64((uint64_t)1 << (14 * s), C.one_sh_t, C.t);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    uint64_t hi = 0, lo = 0;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      uint64_t ph, pl;
      mul_wide(zt_mod_signed((int64_t)acc[s][r], C), pw[s], ph, pl);
      lo += pl;
      hi += ph + (lo < pl ? 1 : 0);
    }
    red[wv][(lc + 4 * r) * 16 + lr] =
        add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t), reduce64(lo, C.one_sh_t, C.t), C.t);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 256; o += blockDim.x) {
    uint64_t v = 0;
    for (int w = 0; w < nw; ++w) v = add_mod(v, red[w][o], C.t);
    const int orow = blockIdx.x * 16 + o / 16, ocol = blockIdx.y * 16 + o % 16;
    if (orow < P && ocol < R) {
      const int m = orow / ohw, rem = orow - m * ohw, y = rem / G.OW, x = rem - y * G.OW;
      gview(out)[(int64_t)m * OV.s0 + (int64_t)ocol * OV.s1 + (int64_t)y * OV.sy + (int64_t)x * OV.sx] = (int64_t)v;
    }
  }
}

// Z_t linear combination out = base + sum_i c_i x_i (mod t), one thread per
// element: the masked operands and share combinations of the preprocessed
// products (Pencil+, online phase).  Operands and coefficients are below
// t < 2^48, so each product fits 96 bits and 64 of them plus base fit 128.
__global__ void __launch_bounds__(256) k_zt_combine(ZtTerms T, const int64_t* base, int64_t* out, int64_t count,
                                                    Consts C) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  uint64_t hi = 0, lo = base ? (uint64_t)gview(base)[g] : 0;
  for (int i = 0; i < T.n; ++i) {
    uint64_t ph, pl;
    mul_wide((uint64_t)gview(T.x[i])[g], T.c[i], ph, pl);
    lo += pl;
    hi += ph + (lo < pl ? 1 : 0);
  }
  const uint64_t v = add_mod(mul_shoup(reduce64(hi, C.one_sh_t, C.t), C.r64t, C.r64t_sh, C.t),
                             reduce64(lo, C.one_sh_t, C.t), C.t);
  gview(out)[g] = (int64_t)v;
}

// ------------------------------------------ bias gradient and DP noise

// Bias gradient share (Sec. III.B.2): the sum of a dY share over the batch
// and, for a convolution, over the output positions, mod t.  dy is
// [batch][channels][spatial].  The host admits at most 2^(64 - bitlen(t))
// entries per channel, so a 64-bit total is exact until the final reduction.
__global__ void __launch_bounds__(256) k_bias_grad_cols(const int64_t* __restrict__ dy, int64_t* __restrict__ db,
                                                        int batch, int channels, Consts C) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= channels) return;
  const PENCIL_GLOBAL int64_t* p = gview(dy) + o;
  uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int b = 0;
  for (; b + 4 <= batch; b += 4) {
    a0 += (uint64_t)p[(int64_t)b * channels];
    a1 += (uint64_t)p[(int64_t)(b + 1) * channels];
    a2 += (uint64_t)p[(int64_t)(b + 2) * channels];
    a3 += (uint64_t)p[(int64_t)(b + 3) * channels];
  }
  for (; b < batch; ++b) a0 += (uint64_t)p[(int64_t)b * channels];
  gview(db)[o] = (int64_t)reduce64(a0 + a1 + a2 + a3, C.one_sh_t, C.t);
}

__global__ void __launch_bounds__(256) k_bias_grad_chan(const int64_t* __restrict__ dy, int64_t* __restrict__ db,
                                                        int batch, int channels, int spatial, Consts C) {
  __shared__ uint64_t part[256];
  const int o = blockIdx.x;
  const uint32_t total = (uint32_t)batch * (uint32_t)spatial;
  const PENCIL_GLOBAL int64_t* base = gview(dy) + (int64_t)o * spatial;
  const int64_t bstride = (int64_t)channels * spatial;
  uint64_t acc = 0;
  for (uint32_t i = threadIdx.x; i < total; i += 256) {
    const uint32_t b = i / (uint32_t)spatial, x = i - b * (uint32_t)spatial;
    acc += (uint64_t)base[(int64_t)b * bstride + x];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) gview(db)[o] = (int64_t)reduce64(part[0], C.one_sh_t, C.t);
}

// Gaussian perturbation the data owner adds to its weight-gradient and
// bias-gradient shares (Sec. III.B.2, DPSGD).  Box-Muller from Philox words,
// every step one IEEE double operation in a fixed order (contraction off), so
// the draws do not depend on the compiler's scheduling:
//   ln u, u = k 2^-53: u = m 2^e with m in [1/sqrt 2, sqrt 2), s = (m-1)/(m+1),
//     ln m = 2 s sum_{j<12} s^2j / (2j+1) (atanh series), ln u = e ln 2 + ln m;
//   cos, sin of 2 pi b 2^-53: quadrant q = round(b / 2^51), theta = (b - q 2^51)
//     2^-53 2 pi in [-pi/4, pi/4], Taylor series through theta^23, rotated by q.
struct DpCoeffs {
  double lg[12], cc[12], cs[12];
};

constexpr DpCoeffs make_dp_coeffs() {
  DpCoeffs c{};
  for (int j = 0; j < 12; ++j) c.lg[j] = 1.0 / (double)(2 * j + 1);
  c.cc[0] = 1.0;
  c.cs[0] = 1.0;
  for (int j = 1; j < 12; ++j) {
    c.cc[j] = c.cc[j - 1] / -(double)((2 * j - 1) * (2 * j));
    c.cs[j] = c.cs[j - 1] / -(double)((2 * j) * (2 * j + 1));
  }
  return c;
}

__device__ __forceinline__ double dp_pow2(int e) {  // 2^e for -1022 <= e <= 1023
  return __longlong_as_double((long long)((uint64_t)(1023 + e) << 52));
}

__device__ double dp_log_u(uint64_t k) {  // ln(k 2^-53), 1 <= k <= 2^53
#pragma clang fp contract(off)
  constexpr DpCoeffs K = make_dp_coeffs();
  constexpr double kSqrtHalf = 0.7071067811865476, kLn2 = 0.6931471805599453;
  const int bl = 64 - __clzll((long long)k);
  double m = (double)k * dp_pow2(-bl);
  int e = bl - 53;
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = K.lg[11];
#pragma unroll
  for (int j = 10; j >= 0; --j) p = p * s2 + K.lg[j];
  const double lnm = (s * p) * 2.0;
  return (double)e * kLn2 + lnm;
}

__device__ void dp_cos_sin_turns(uint64_t b, double& co, double& si) {  // of 2 pi b 2^-53, b < 2^53
#pragma clang fp contract(off)
  constexpr DpCoeffs K = make_dp_coeffs();
  constexpr double kTwoPi = 6.283185307179586;
  const int64_t bb = (int64_t)b;
  const int64_t q = (bb + (1ll << 50)) >> 51;
  const int64_t d = bb - (q << 51);
  const double theta = ((double)d * dp_pow2(-53)) * kTwoPi;
  const double t2 = theta * theta;
  double pc = K.cc[11], ps = K.cs[11];
#pragma unroll
  for (int j = 10; j >= 0; --j) {
    pc = pc * t2 + K.cc[j];
    ps = ps * t2 + K.cs[j];
  }
  const double c = pc, s = theta * ps;
  switch (q & 3) {
    case 0: co = c; si = s; break;
    case 1: co = -s; si = c; break;
    case 2: co = -c; si = -s; break;
    default: co = s; si = -c; break;
  }
}

__device__ __forceinline__ int64_t dp_add(int64_t x, double z, double sd, uint64_t t) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)floor(z * sd);
  int64_t em = e % (int64_t)t;
  if (em < 0) em += (int64_t)t;
  return (int64_t)add_mod((uint64_t)x, (uint64_t)em, t);
}

// One thread per Philox block: entries 4j .. 4j+3 from words (w0, w1), (w2, w3).
__global__ void __launch_bounds__(256) k_dp_noise(int64_t* __restrict__ x, int64_t count, double sd, uint64_t nonce,
                                                  uint64_t obj, Consts C) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = 4 * j;
  if (i0 >= count) return;
  const U64x4 w = philox((uint64_t)j, obj, P_DP, 0, C.seed, nonce);
  double z[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double r = sqrt(dp_log_u((w.v[2 * h] >> 11) + 1) * -2.0);
    double co, si;
    dp_cos_sin_turns(w.v[2 * h + 1] >> 11, co, si);
    z[2 * h] = r * co;
    z[2 * h + 1] = r * si;
  }
  PENCIL_GLOBAL int64_t* px = gview(x) + i0;
#pragma unroll
  for (int h = 0; h < 4; ++h)
    if (i0 + h < count) px[h] = dp_add(px[h], z[h], sd, C.t);
}

// ------------------------------------------------- stride-s relayouts

// A stride-s correlation equals a stride-1 correlation over the space-to-depth
// image: channel c' = c sy sx + a sx + e holds Xpad[., c, sy y + a, sx x + e]
// and the kernel W[., c, sy i + a, sx j + e] (zero past the kernel's edge).
// Each mode gathers one output entry per thread; padding and taps that fall
// outside either tensor read as zero.
__global__ void __launch_bounds__(256) k_stride_relayout(Relayout R, const int64_t* __restrict__ in,
                                                         int64_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= R.total) return;
  const int ss = R.sy * R.sx;
  int64_t v = 0;
  if (R.mode == 0 || R.mode == 1) {  // out [n][c * ss][Y][X] from in [n][c][.][.]
    const int Y = R.mode == 0 ? R.h2 : R.kh2, X = R.mode == 0 ? R.w2 : R.kw2;
    const int x2 = (int)(g % X);
    int64_t r = g / X;
    const int y2 = (int)(r % Y);
    r /= Y;
    const int c2 = (int)(r % ((int64_t)R.ci * ss));
    const int64_t n = r / ((int64_t)R.ci * ss);
    const int c = c2 / ss, a = (c2 / R.sx) % R.sy, e = c2 % R.sx;
    if (R.mode == 0) {
      const int yy = R.sy * y2 + a - R.ph, xx = R.sx * x2 + e - R.pw;
      if (yy >= 0 && yy < R.h && xx >= 0 && xx < R.w)
        v = gview(in)[((n * R.ci + c) * R.h + yy) * R.w + xx];
    } else {
      const int i = R.sy * y2 + a, j = R.sx * x2 + e;
      if (i < R.kh && j < R.kw) v = gview(in)[((n * R.ci + c) * R.kh + i) * R.kw + j];
    }
  } else {  // out [n][c][Y][X] from in [n][c * ss][.][.]
    const int Y = R.mode == 2 ? R.h : R.kh, X = R.mode == 2 ? R.w : R.kw;
    const int x = (int)(g % X);
    int64_t r = g / X;
    const int y = (int)(r % Y);
    r /= Y;
    const int c = (int)(r % R.ci);
    const int64_t n = r / R.ci;
    const int yy = R.mode == 2 ? y + R.ph : y, xx = R.mode == 2 ? x + R.pw : x;
    const int y2 = yy / R.sy, x2 = xx / R.sx, c2 = c * ss + (yy % R.sy) * R.sx + xx % R.sx;
    const int Y2 = R.mode == 2 ? R.h2 : R.kh2, X2 = R.mode == 2 ? R.w2 : R.kw2;
    if (y2 < Y2 && x2 < X2) v = gview(in)[((n * ((int64_t)R.ci * ss) + c2) * Y2 + y2) * X2 + x2];
  }
  gview(out)[g] = v;
}

// --------------------------------------------------------- batched step

__device__ __forceinline__ int find_seg(const StepSeg* segs, int nseg, int64_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].block_begin <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Every NTT of one phase, for one ring degree: the forward transforms of the
// inputs (k_step_ntt: ciphertexts, plaintexts, re-randomisation masks) or the
// inverse transforms of the outputs (k_step_intt).
template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512, (LOGE >= 5 ? 2 : 4))
    k_step_ntt(const StepSeg* __restrict__ segs, int nseg, const Consts* __restrict__ consts,
               const Tables* __restrict__ tabs, const uint64_t* __restrict__ nonce) {
  extern __shared__ uint64_t lds[];
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const Consts& C = consts[S.ctx];
  const Tables& T = tabs[S.ctx];
  const int64_t p = (int64_t)blockIdx.x - S.block_begin;
  switch (S.kind) {
    case SEG_CT: do_ntt_ct<LOGN, LOGE>(lds, S.src, S.dst, S.tensor, S.G, S.V, C, T, p); break;
    case SEG_PT: do_ntt_pt<LOGN, LOGE>(lds, S.tensor, S.dst, S.side, S.G, S.V, C, T, p); break;
    case SEG_TERN: do_ntt_ternary<LOGN, LOGE>(lds, S.dst, *nonce + S.nonce_off, S.obj_base, S.purpose, 1, C, T, p); break;
    default: break;
  }
}

template <int LOGN, int LOGE>
__global__ void __launch_bounds__(512, (LOGE >= 5 ? 2 : 4))
    k_step_intt(const StepSeg* __restrict__ segs, int nseg, const Consts* __restrict__ consts,
                const Tables* __restrict__ tabs) {
  extern __shared__ uint64_t lds[];
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const int64_t p = (int64_t)blockIdx.x - S.block_begin;
  do_ntt_plain<LOGN, LOGE>(lds, S.dst, 1, consts[S.ctx], tabs[S.ctx], p);
}

// Every multiply-accumulate of one step with one staging kind.  Segments start
// at multiples of 8 blocks, so a segment's blocks keep their XCD under the
// per-segment work remap; padding blocks past the segment's work exit.
template <int KIND>
__device__ __forceinline__ void step_mac(const StepSeg* __restrict__ segs, int nseg,
                                         const Consts* __restrict__ consts, uint64_t* smem) {
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const int64_t local = (int64_t)blockIdx.x - S.block_begin;
  const int chunks = mac_chunks(S.mac.variant, S.mac.m_rows, S.G.nR);
  const int64_t work = S.slot_blocks * chunks, padded = (work + 7) & ~(int64_t)7;
  const int w = (int)xcd_work(local, padded);  // work items per launch stay below 2^31
  if (w >= work) return;
  do_mac<KIND>(smem, S.mac, S.G, consts[S.ctx], w / chunks, w % chunks);
}

#define STEP_ARGS const StepSeg *__restrict__ segs, int nseg, const Consts *__restrict__ consts
__global__ void __launch_bounds__(512) k_step_mac(STEP_ARGS) {
  __shared__ uint64_t smem[kMacSmemWords];
  step_mac<0>(segs, nseg, consts, smem);
}

__global__ void __launch_bounds__(512) k_step_mac_direct(STEP_ARGS) { step_mac<1>(segs, nseg, consts, nullptr); }

__global__ void __launch_bounds__(512) k_step_mac_direct_small(STEP_ARGS) {
  step_mac<2>(segs, nseg, consts, nullptr);
}
#undef STEP_ARGS

// Every flood-and-mask of one step, for one flood width.
template <int W>
__global__ void __launch_bounds__(256) k_step_flood(const StepSeg* __restrict__ segs, int nseg,
                                                    const Consts* __restrict__ consts,
                                                    const uint64_t* __restrict__ nonce) {
  const StepSeg& S = segs[find_seg(segs, nseg, blockIdx.x)];
  const int64_t g = ((int64_t)blockIdx.x - S.block_begin) * blockDim.x + threadIdx.x;
  do_flood<W>(S.dst, S.count, S.share, S.bias, S.G, S.V2, *nonce + S.nonce_off, S.obj_base, consts[S.ctx], g);
}

__global__ void k_set_u64(uint64_t* p, uint64_t v, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = add ? p[0] + v : v;
}

// ---------------------------------------------------------------- launchers

static inline size_t lds_bytes(const Consts& C) { return (size_t)(C.n + (C.n >> 5)) * sizeof(uint64_t); }

// Instantiate `kern<LOGN>` for the context's degree and launch it.
#define NTT_CASE(kern, LN, LE, grid, C, s, ...)                                                 \
  case (LN) * 8 + (LE):                                                                          \
    hipLaunchKernelGGL((kern<LN, LE>), grid, dim3((1u << (LN)) >> (LE)), lds_bytes(C), s, __VA_ARGS__); \
    break;
// Instantiate `kern<LOGN, LOGE>` for the context's degree and per-thread width.
#define NTT_DISPATCH(kern, grid, C, s, ...)                                                \
  do {                                                                                     \
    switch ((C).log2n * 8 + (C).ntt_loge) {                                                \
      NTT_CASE(kern, 10, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 11, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 12, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 12, 5, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 13, 4, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 13, 5, grid, C, s, __VA_ARGS__)                                       \
      NTT_CASE(kern, 14, 5, grid, C, s, __VA_ARGS__)                                       \
      default: return hipErrorInvalidValue;                                                \
    }                                                                                      \
  } while (0)

hipError_t launch_ntt_plain(uint64_t* data, int64_t polys, bool inverse, const Consts& C, const Tables& T,
                            hipStream_t s) {
  if (polys <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_plain, dim3((unsigned)(polys * C.L)), C, s, data, inverse ? 1 : 0, C, T);
  return hipGetLastError();
}

hipError_t launch_ntt_ct(const uint64_t* src, uint64_t* dst, int64_t n_ct, const int64_t* share, const Geo& G,
                         const View& V, const Consts& C, const Tables& T, hipStream_t s) {
  if (n_ct <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_ct, dim3((unsigned)(n_ct * 2 * C.L)), C, s, src, dst, share, G, V, C, T);
  return hipGetLastError();
}

hipError_t launch_ntt_pt(const int64_t* tensor, uint64_t* dst, int64_t n_pt, int side, const Geo& G, const View& V,
                         const Consts& C, const Tables& T, hipStream_t s) {
  if (n_pt <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_pt, dim3((unsigned)(n_pt * C.L)), C, s, tensor, dst, side, G, V, C, T);
  return hipGetLastError();
}

hipError_t launch_ntt_ternary(uint64_t* dst, int64_t count, uint64_t nonce, uint64_t obj_base, uint32_t purpose, int split,
                              const Consts& C, const Tables& T, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_ternary, dim3((unsigned)(count * C.L)), C, s, dst, nonce, obj_base, purpose, split, C, T);
  return hipGetLastError();
}

hipError_t launch_mac(const MacArgs& A, int64_t n_out, const Geo& G, const Consts& C, hipStream_t s) {
  if (n_out <= 0) return hipSuccess;
  const int64_t slot_blocks = (int64_t)C.n * C.L / kMacSlots;
  const int chunks = mac_chunks(A.variant, A.m_rows, G.nR);
  const int64_t total = slot_blocks * chunks;
  if (total >= (1ll << 31)) return hipErrorInvalidConfiguration;  // work items are int
  if (A.variant >= 6)
    hipLaunchKernelGGL(k_mac_direct_small, dim3((unsigned)total), dim3(512), 0, s, A, G, C, chunks, total);
  else if (A.variant >= 3)
    hipLaunchKernelGGL(k_mac_direct, dim3((unsigned)total), dim3(512), 0, s, A, G, C, chunks, total);
  else
    hipLaunchKernelGGL(k_mac_lds, dim3((unsigned)total), dim3(512), kMacSmemWords * sizeof(uint64_t), s, A, G, C,
                       chunks, total);
  return hipGetLastError();
}

hipError_t launch_flood_mask(uint64_t* ct, int64_t n_out, int64_t* share0, const int64_t* bias, const Geo& G,
                             const View& outV, uint64_t nonce, uint64_t obj_base, const Consts& C, hipStream_t s) {
  if (n_out <= 0) return hipSuccess;
  const int64_t threads = n_out * (C.n / 4);
  const dim3 grid((unsigned)((threads + 255) / 256));
  switch (C.flood_words) {
    case 1: hipLaunchKernelGGL(k_flood_mask<1>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    case 2: hipLaunchKernelGGL(k_flood_mask<2>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    case 3: hipLaunchKernelGGL(k_flood_mask<3>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    case 4: hipLaunchKernelGGL(k_flood_mask<4>, grid, dim3(256), 0, s, ct, n_out, share0, bias, G, outV, nonce, obj_base, C); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_encrypt(const uint64_t* u_ntt, const int64_t* share, uint64_t* ct, int64_t n_ct, int side,
                          const Geo& G, const View& V, const uint64_t* pk_ntt, const uint64_t* pk_sh, uint64_t nonce,
                          uint64_t obj_base, const Consts& C, const Tables& T, hipStream_t s) {
  if (n_ct <= 0) return hipSuccess;
  NTT_DISPATCH(k_encrypt, dim3((unsigned)(n_ct * 2 * C.L)), C, s, u_ntt, share, ct, side, G, V, pk_ntt, pk_sh, nonce,
               obj_base, C, T);
  return hipGetLastError();
}

hipError_t launch_phase(const uint64_t* ct, uint64_t* x, int64_t n_ct, const uint64_t* s_ntt, const uint64_t* s_sh,
                        const Consts& C, const Tables& T, hipStream_t s) {
  if (n_ct <= 0) return hipSuccess;
  NTT_DISPATCH(k_phase, dim3((unsigned)(n_ct * C.L)), C, s, ct, x, s_ntt, s_sh, C, T);
  return hipGetLastError();
}

hipError_t launch_decode(const uint64_t* x, int64_t* share, int64_t n_out, const Geo& G, const View& outV,
                         const Consts& C, hipStream_t s) {
  const int64_t per = (int64_t)G.mt * G.rt * G.oh * G.ow;
  const int64_t threads = n_out * per;
  if (threads <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_decode, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, x, share, n_out, G, outV, C);
  return hipGetLastError();
}

hipError_t launch_zt_combine(const ZtTerms& T, const int64_t* base, int64_t* out, int64_t count, const Consts& C,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zt_combine, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, T, base, out, count, C);
  return hipGetLastError();
}

hipError_t launch_bias_grad(const int64_t* dy, int64_t* db, int batch, int channels, int spatial, const Consts& C,
                            hipStream_t s) {
  if (channels <= 0) return hipSuccess;
  if (spatial == 1)
    hipLaunchKernelGGL(k_bias_grad_cols, dim3((unsigned)((channels + 255) / 256)), dim3(256), 0, s, dy, db, batch,
                       channels, C);
  else
    hipLaunchKernelGGL(k_bias_grad_chan, dim3((unsigned)channels), dim3(256), 0, s, dy, db, batch, channels, spatial,
                       C);
  return hipGetLastError();
}

hipError_t launch_dp_noise(int64_t* x, int64_t count, double sd, uint64_t nonce, uint64_t obj, const Consts& C,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t threads = (count + 3) / 4;
  hipLaunchKernelGGL(k_dp_noise, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, x, count, sd, nonce, obj,
                     C);
  return hipGetLastError();
}

hipError_t launch_stride_relayout(const Relayout& R, const int64_t* in, int64_t* out, hipStream_t s) {
  if (R.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stride_relayout, dim3((unsigned)((R.total + 255) / 256)), dim3(256), 0, s, R, in, out);
  return hipGetLastError();
}

hipError_t launch_zt_corr(const int64_t* a, const int64_t* k, int64_t* out, const Geo& G, const View& AV,
                          const View& KV, const View& OV, const Consts& C, hipStream_t s) {
  const int64_t total = (int64_t)G.M * G.R * G.OH * G.OW;
  if (total <= 0) return hipSuccess;
  const int64_t rows = (int64_t)G.M * G.OH * G.OW, ctot = (int64_t)G.K * G.KH * G.KW;
  // Tiled kernel: 2 x 2 outputs per lane when that still gives >= 512
  // workgroups, else 1; about 16 contraction steps per wave, at most 16 waves.
  // Operands split at bit 21 (high part h = bitlen(t) - 21 bits): a partial
  // sum takes terms below 2^42, 2^(22 + h) and 2^(2h), so a wave may sum
  // 2^(64 - max) of them (2^22 for t < 2^42).
  const int tb = 64 - __builtin_clzll(C.t), hb = tb > 21 ? tb - 21 : 0;
  const int mb = std::max(42, std::max(22 + hb, 2 * hb));
  const int64_t per_wave_max = mb >= 63 ? 1 : (int64_t)1 << (64 - mb);
  // Matrix-core kernel when there are at least 256 output tiles of 16 x 16
  // (with fewer, the vector kernel's smaller tiles spread the work wider and
  // measured faster): four contraction indices per step, about eight steps per
  // wave, at most 16 waves; a diagonal sum takes per-term values below 2^30
  // (t < 2^43; 2^(2 bitlen(t) - 58) above), so a wave may run
  // 2^53 / (4 * that) steps.
  if (((rows + 15) / 16) * ((G.R + 15) / 16) >= 256) {
    const int d2b = tb > 29 ? tb - 29 : 0;  // bits of the top digit
    const int termb = std::max(30, std::max(tb - 13, 2 * d2b));
    const int64_t steps = (ctot + 3) / 4;
    const int64_t max_steps = termb >= 51 ? 0 : (int64_t)1 << (51 - termb);
    int nwm = (int)std::min<int64_t>(kZtWaves, std::max<int64_t>(1, steps / 8));
    const int64_t gx = (rows + 15) / 16, gy = ((int64_t)G.R + 15) / 16;
    if ((steps + nwm - 1) / nwm <= max_steps && gx < (1ll << 31) && gy < 65536) {
      hipLaunchKernelGGL(k_zt_mfma, dim3((unsigned)gx, (unsigned)gy), dim3(64 * nwm), 0, s, a, k, out, G, AV, KV, OV,
                         C);
      return hipGetLastError();
    }
  }
  const int64_t blocks2 = ((rows + 15) / 16) * ((G.R + 15) / 16);
  const int ti = blocks2 >= 512 ? 2 : 1;
  const int64_t steps16 = ctot / 16;
  const int nw = steps16 < 1 ? 1 : steps16 > kZtWaves ? kZtWaves : (int)steps16;
  const int64_t gx = (rows + 8 * ti - 1) / (8 * ti), gy = ((int64_t)G.R + 8 * ti - 1) / (8 * ti);
  if ((ctot + nw - 1) / nw <= per_wave_max && gx < (1ll << 31) && gy < 65536) {
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (ti == 2)
      hipLaunchKernelGGL(k_zt_gemm<2>, grid, dim3(64 * nw), 0, s, a, k, out, G, AV, KV, OV, C);
    else
      hipLaunchKernelGGL(k_zt_gemm<1>, grid, dim3(64 * nw), 0, s, a, k, out, G, AV, KV, OV, C);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_zt_corr, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, k, out, G, AV, KV, OV, C);
  return hipGetLastError();
}

hipError_t launch_step_ntt(int log2n, int loge, bool inverse, const StepPhase& P, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  Consts C{};  // only log2n, n and ntt_loge are read by the dispatch
  C.log2n = log2n;
  C.n = 1 << log2n;
  C.ntt_loge = loge;
  const dim3 grid((unsigned)blocks);
  if (inverse)
    NTT_DISPATCH(k_step_intt, grid, C, s, P.segs, P.nseg, P.consts, P.tabs);
  else
    NTT_DISPATCH(k_step_ntt, grid, C, s, P.segs, P.nseg, P.consts, P.tabs, P.nonce);
  return hipGetLastError();
}

hipError_t launch_step_mac(const StepPhase& P, int64_t blocks, int kind, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (kind == 2)
    hipLaunchKernelGGL(k_step_mac_direct_small, dim3((unsigned)blocks), dim3(512), 0, s, P.segs, P.nseg, P.consts);
  else if (kind == 1)
    hipLaunchKernelGGL(k_step_mac_direct, dim3((unsigned)blocks), dim3(512), 0, s, P.segs, P.nseg, P.consts);
  else
    hipLaunchKernelGGL(k_step_mac, dim3((unsigned)blocks), dim3(512), 0, s, P.segs, P.nseg, P.consts);
  return hipGetLastError();
}

hipError_t launch_step_flood(int words, const StepPhase& P, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (words) {
    case 1: hipLaunchKernelGGL(k_step_flood<1>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    case 2: hipLaunchKernelGGL(k_step_flood<2>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    case 3: hipLaunchKernelGGL(k_step_flood<3>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    case 4: hipLaunchKernelGGL(k_step_flood<4>, dim3((unsigned)blocks), dim3(256), 0, s, P.segs, P.nseg, P.consts, P.nonce); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t* p, uint64_t v, int add, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, p, v, add);
  return hipGetLastError();
}

hipError_t launch_keygen(uint64_t* s_ntt, int64_t* s_coeff, uint64_t* pk_coeff, uint64_t* pk_ntt, const Consts& C,
                         const Tables& T, hipStream_t s) {
  NTT_DISPATCH(k_keygen, dim3((unsigned)C.L), C, s, s_ntt, s_coeff, pk_coeff, pk_ntt, C, T);
  return hipGetLastError();
}

// Kernels that stage more than 64 KiB of LDS must opt in once per process.
template <int LOGN, int LOGE>
static hipError_t raise_lds_limit() {
  const int max_lds = 160 * 1024;
  const void* fns[] = {(const void*)k_ntt_plain<LOGN, LOGE>,   (const void*)k_ntt_ct<LOGN, LOGE>,
                       (const void*)k_ntt_pt<LOGN, LOGE>,      (const void*)k_ntt_ternary<LOGN, LOGE>,
                       (const void*)k_encrypt<LOGN, LOGE>,     (const void*)k_phase<LOGN, LOGE>,
                       (const void*)k_keygen<LOGN, LOGE>,      (const void*)k_step_ntt<LOGN, LOGE>,
                       (const void*)k_step_intt<LOGN, LOGE>};
  hipError_t e = hipSuccess;
  for (const void* f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (r != hipSuccess) e = r;
  }
  return e;
}

hipError_t configure_lds_limits() {
  const int mac_lds = kMacSmemWords * sizeof(uint64_t);
  hipError_t m1 = hipFuncSetAttribute((const void*)k_mac_lds, hipFuncAttributeMaxDynamicSharedMemorySize, mac_lds);
  hipError_t m2 = hipFuncSetAttribute((const void*)k_step_mac, hipFuncAttributeMaxDynamicSharedMemorySize, mac_lds);
  if (m1 != hipSuccess) return m1;
  if (m2 != hipSuccess) return m2;
  hipError_t e[3] = {raise_lds_limit<13, 4>(), raise_lds_limit<13, 5>(), raise_lds_limit<14, 5>()};
  for (hipError_t x : e)
    if (x != hipSuccess) return x;
  return hipSuccess;
}

}  // namespace pencil
