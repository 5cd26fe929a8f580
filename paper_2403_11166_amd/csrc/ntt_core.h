// Negacyclic NTT of one limb-polynomial per workgroup, staged in LDS, and
// the forward-transform front ends of the product path (input ciphertexts
// with the model owner's share, encoded plaintexts, ternary masks).
#pragma once
#include "device_common.h"

namespace pencil {

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

// Launch bounds of a kernel that transforms one polynomial per workgroup:
// N / E threads (1024 only for E = 16 at N = 16384, one workgroup per CU by
// LDS) and the waves per SIMD the registers must allow (4 with 16 residues per
// thread, 2 with 32).
constexpr int ntt_threads(int logn, int loge) { return (1 << logn) >> loge; }
constexpr int ntt_min_waves(int logn, int loge) { return ntt_threads(logn, loge) > 512 || loge < 5 ? 4 : 2; }
#define PENCIL_NTT_BOUNDS(LOGN, LOGE) __launch_bounds__(ntt_threads(LOGN, LOGE), ntt_min_waves(LOGN, LOGE))

// Butterfly constants of one modulus q < 2^60: 8q, 4q and 2^64 minus each,
// 2^64 - q, and for the final reduction the bit length B of q (q < 2^B), 2^B - 1
// and delta = 2^B - q.  They are hidden from the optimiser so that x - 4q stays
// the single 64-bit addition x + (2^64 - 4q) instead of a borrow chain.
struct BflyK {
  uint64_t q8, nq8, q4, nq4, nq, top_mask;
  uint32_t top_bits, top_delta;
};

__device__ __forceinline__ BflyK bfly_consts(uint64_t q) {
  const uint32_t b = 64 - (uint32_t)__builtin_clzll(q);
  BflyK k{8 * q, 0 - 8 * q, 4 * q, 0 - 4 * q, 0 - q, (1ull << b) - 1, b, (uint32_t)((1ull << b) - q)};
  asm volatile("" : "+s"(k.q8), "+s"(k.nq8), "+s"(k.q4), "+s"(k.nq4), "+s"(k.nq), "+s"(k.top_mask),
               "+s"(k.top_bits), "+s"(k.top_delta));
  return k;
}

// x - c if x >= c, else x, for x < 2c and c <= 2^63 (nc = 2^64 - c): x - c
// taken as a signed 64-bit value is negative exactly when x < c.
__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t c, uint64_t nc) {
  const uint64_t d = x + nc;
  return (int64_t)d < 0 ? x : d;
}

// Lazy Shoup product y w mod q in [0, 4q) for any y < 2^64, w < q, with
// companion ws = floor(w 2^64 / q).  Of y ws / 2^64 = y1 ws1 + (y1 ws0 + y0 ws1)
// / 2^32 + y0 ws0 / 2^64 (32-bit halves) the estimate keeps y1 ws1 +
// hi(y0 ws1) + hi(y1 ws0): three multiplies instead of four.  The dropped parts
// sum to less than 3, so the estimate is at most 2 below floor(y ws / 2^64),
// which is itself at most 1 below floor(y w / q); y w - est q is then below 4q.
__device__ __forceinline__ uint64_t shoup_lazy(uint64_t y, const TW w, const BflyK& k) {
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  const uint32_t s0 = (uint32_t)w.ws, s1 = (uint32_t)(w.ws >> 32);
  uint64_t est = (uint64_t)y1 * s1 + __umulhi(y0, s1);
  est += __umulhi(y1, s0);
  return y * w.w + est * k.nq;
}

// Lazy Cooley-Tukey butterfly, reducing x on every other stage (`reduce` is
// a compile-time constant after unrolling).  With reduce, x and y in [0, 16q)
// give a = x mod 8q in [0, 8q) and outputs in [0, 12q); without, inputs in
// [0, 12q) give outputs in [0, 16q).  The Shoup product t is below 4q for any
// y, and 16q < 2^64 for q < 2^60.
__device__ __forceinline__ void ct_bfly(uint64_t& x, uint64_t& y, const TW w, const BflyK& k, const bool reduce) {
  const uint64_t a = reduce ? csub(x, k.q8, k.nq8) : x;
  const uint64_t t = shoup_lazy(y, w, k);
  x = a + t;
  y = (a + k.q4) - t;
}

// Lazy Gentleman-Sande butterfly: u, v in [0, 4q) -> [0, 4q).
__device__ __forceinline__ void gs_bfly(uint64_t& u, uint64_t& v, const TW w, const BflyK& k) {
  const uint64_t s = csub(u + v, k.q4, k.nq4);
  const uint64_t d = (u + k.q4) - v;
  v = shoup_lazy(d, w, k);
  u = s;
}

// x in [0, 16q) -> x mod q.  With x = h 2^B + r (r < 2^B, h < 16),
// x = r + h delta (mod q), and r + h delta < 2^B + 15 delta < 2q because the
// moduli lie within 2^B / 17 of 2^B (checked when the context is made).
__device__ __forceinline__ uint64_t reduce_16q(uint64_t x, uint64_t q, const BflyK& k) {
  const uint32_t h = (uint32_t)(x >> k.top_bits);
  const uint64_t y = (uint64_t)h * k.top_delta + (x & k.top_mask);
  return csub(y, q, k.nq);
}

// Forward (merged negacyclic Cooley-Tukey, psi^rev twiddles; natural order in,
// bit-reversed out) stages S0 .. S0+S-1.  At stage l (t = N >> (l+1)) the pair
// (i0, i0 + t) of group i = i0 >> (log2 N - l) uses tw[2^l + i].  A thread takes
// E / 2^S groups of 2^S residues {base + k * 2^LT}, LT = log2 N - S0 - S.
// `in(i)` supplies input residue i: the LDS polynomial, or for the first pass
// values the caller computes (an encoding), which then skip the LDS.
template <int LOGN, int LOGE, int S0, int S, bool LAST, typename In>
__device__ __forceinline__ void fwd_pass(uint64_t* a, In in, const PENCIL_GLOBAL TW* tw, uint64_t q,
                                         const BflyK& bk) {
  using Sh = NttShape<LOGN, LOGE>;
  constexpr int T = Sh::T, G = Sh::E >> S, K = 1 << S, LT = LOGN - S0 - S;
  const int tid = threadIdx.x;
  uint64_t v[Sh::E];
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const int g = r * T + tid;
    const int base = ((g >> LT) << (LOGN - S0)) + (g & ((1 << LT) - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) v[r * K + k] = in(base + (k << LT));
  }
  // A wave whose first-pass inputs are all zero (most waves of a sparse K
  // tile) skips the butterflies: its outputs are zero, a representative of
  // the same residues the lazy butterflies would give.
  bool work = true;
  if constexpr (S0 == 0) {
    uint64_t any = 0;
#pragma unroll
    for (int i = 0; i < Sh::E; ++i) any |= v[i];
    work = __builtin_amdgcn_ballot_w64(any != 0) != 0;
  }
  if (work) {
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
          ct_bfly(v[r * K + k], v[r * K + k + h], w, bk, ((S0 + s) & 1) == 0);
        }
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
      if (LAST) x = reduce_16q(x, q, bk);
      a[lpad(base + (k << LT))] = x;
    }
  }
}

// Inverse (Gentleman-Sande, psi^-rev twiddles; bit-reversed in, natural out)
// stages with t = 2^L0 .. 2^(L0+S-1): pair (i0, i0 + t), i = i0 >> (l + 1),
// twiddle itw[(N >> (l + 1)) + i].  Groups are {base + k * 2^L0}.
template <int LOGN, int LOGE, int L0, int S, typename In>
__device__ __forceinline__ void inv_pass(uint64_t* a, In in, const PENCIL_GLOBAL TW* tw, uint64_t q,
                                         const BflyK& bk) {
  using Sh = NttShape<LOGN, LOGE>;
  constexpr int T = Sh::T, G = Sh::E >> S, K = 1 << S;
  const int tid = threadIdx.x;
  uint64_t v[Sh::E];
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const int g = r * T + tid;
    const int base = ((g >> L0) << (L0 + S)) + (g & ((1 << L0) - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) v[r * K + k] = in(base + (k << L0));
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

// Forward transform into the LDS polynomial `a` (outputs in [0, q)) of the
// inputs in [0, q) that `in(i)` supplies to the first pass; the transform's
// first LDS access is the first pass' store, so `a` must not be in use.
// Callers synchronise after (outputs read).
template <int LOGN, int LOGE, typename In>
__device__ __forceinline__ void ntt_fwd_in(uint64_t* a, In in, const TW* tw_generic, uint64_t q) {
  using Sh = NttShape<LOGN, LOGE>;
  const BflyK bk = bfly_consts(q);
  const PENCIL_GLOBAL TW* tw = gview(tw_generic);
  auto lds = [a](int i) { return a[lpad(i)]; };
  fwd_pass<LOGN, LOGE, Sh::start(0), Sh::size(0), Sh::NP == 1>(a, in, tw, q, bk);
  __syncthreads();
  if constexpr (Sh::NP > 1) {
    fwd_pass<LOGN, LOGE, Sh::start(1), Sh::size(1), Sh::NP == 2>(a, lds, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 2) {
    fwd_pass<LOGN, LOGE, Sh::start(2), Sh::size(2), Sh::NP == 3>(a, lds, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 3) {
    fwd_pass<LOGN, LOGE, Sh::start(3), Sh::size(3), true>(a, lds, tw, q, bk);
    __syncthreads();
  }
}

// Forward transform of the LDS polynomial (inputs in [0, q), outputs in [0, q)).
// Callers synchronise before (inputs written) and after (outputs read).
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_fwd(uint64_t* a, const TW* tw_generic, uint64_t q) {
  ntt_fwd_in<LOGN, LOGE>(a, [a](int i) { return a[lpad(i)]; }, tw_generic, q);
}

// Inverse transform without the N^-1 factor (inputs in [0, 4q), outputs in
// [0, 4q)) into the LDS polynomial `a`, of the inputs `in(i)` supplies to the
// first pass (as for ntt_fwd_in, `a` must not be in use).
template <int LOGN, int LOGE, typename In>
__device__ __forceinline__ void ntt_inv_in(uint64_t* a, In in, const TW* tw_generic, uint64_t q) {
  using Sh = NttShape<LOGN, LOGE>;
  const BflyK bk = bfly_consts(q);
  const PENCIL_GLOBAL TW* tw = gview(tw_generic);
  auto lds = [a](int i) { return a[lpad(i)]; };
  inv_pass<LOGN, LOGE, Sh::start(0), Sh::size(0)>(a, in, tw, q, bk);
  __syncthreads();
  if constexpr (Sh::NP > 1) {
    inv_pass<LOGN, LOGE, Sh::start(1), Sh::size(1)>(a, lds, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 2) {
    inv_pass<LOGN, LOGE, Sh::start(2), Sh::size(2)>(a, lds, tw, q, bk);
    __syncthreads();
  }
  if constexpr (Sh::NP > 3) {
    inv_pass<LOGN, LOGE, Sh::start(3), Sh::size(3)>(a, lds, tw, q, bk);
    __syncthreads();
  }
}

// Inverse transform of the LDS polynomial; callers synchronise before and after.
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_inv(uint64_t* a, const TW* tw_generic, uint64_t q) {
  ntt_inv_in<LOGN, LOGE>(a, [a](int i) { return a[lpad(i)]; }, tw_generic, q);
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
  // the first butterfly pass reads its residues straight from memory; results
  // leave the LDS in 16-byte pairs (a pair never straddles an LDS pad word)
  PENCIL_GLOBAL u64x2* g = (PENCIL_GLOBAL u64x2*)gview(data + p * n);
  const PENCIL_GLOBAL uint64_t* g1 = gview(data + p * n);
  auto src = [g1](int i) { return g1[i]; };
  if (!inverse) {
    ntt_fwd_in<LOGN, LOGE>(lds, src, T.fw + (int64_t)l * n, lc.q);
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x) g[i] = u64x2{lds[lpad(2 * i)], lds[lpad(2 * i) + 1]};
  } else {
    ntt_inv_in<LOGN, LOGE>(lds, src, T.iw + (int64_t)l * n, lc.q);
    for (int i = threadIdx.x; i < n / 2; i += blockDim.x)
      g[i] = u64x2{mul_shoup(lds[lpad(2 * i)], lc.ninv, lc.ninv_sh, lc.q),
                   mul_shoup(lds[lpad(2 * i) + 1], lc.ninv, lc.ninv_sh, lc.q)};
  }
}

// Input ciphertexts (NTT domain, split form) of the products that add the
// model owner's share: component 0 gains the transform of round(q m / t) of
// the share (Alg. 1, product step) and is written, split, to the staging
// copy; component 1 is read in place by the multiply-accumulate.
// Grid: n_ct * L blocks, polynomial p = (j, l) in [n][L] order; src and dst
// are [n][2][L][N].
template <int LOGN, int LOGE>
__device__ __forceinline__ void do_ntt_ct(uint64_t* lds, const uint64_t* src, uint64_t* dst, const int64_t* share,
                                          const Geo& G, const View& V, const Consts& C, const Tables& T, int64_t p) {
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int l = (int)(p % L);
  const int64_t j = p / L;
  const int64_t at = (j * 2 * L + l) * n;  // component 0, limb l of ciphertext j
  const LimbConst& lc = C.limb[l];
  const PENCIL_GLOBAL int64_t* gshare = gview(share);
  const TileOrigin to = a_tile_origin(G, j);
  auto enc = [&](int i) {
    uint64_t v = 0;
    const int64_t off = a_slot_at(G, V, to, i);
    if (off >= 0) {
      const uint64_t m = (uint64_t)gshare[off];
      v = delta_scale(m, round_rho(m, C), lc);
    }
    return v;
  };
  ntt_fwd_in<LOGN, LOGE>(lds, enc, T.fw + (int64_t)l * n, lc.q);
  // 16-byte accesses: a polynomial is 16-byte aligned
  const PENCIL_GLOBAL u64x2* g2 = (const PENCIL_GLOBAL u64x2*)gview(src + at);
  PENCIL_GLOBAL u64x2* o2 = (PENCIL_GLOBAL u64x2*)gview(dst + at);
  for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
    const u64x2 v = g2[i];
    o2[i] = u64x2{split30(add_mod(unsplit30(v[0]), lds[lpad(2 * i)], lc.q)),
                  split30(add_mod(unsplit30(v[1]), lds[lpad(2 * i) + 1], lc.q))};
  }
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
  const TileOrigin to = tile_origin(side, G, j);
  auto lift = [&](int64_t off) {
    const uint64_t w = (uint64_t)gt[off];
    return w <= C.t_half ? w : lc.q - (C.t - w);
  };
  if (side == 0) {
    // A tiles are dense: each slot gathers its value in the first pass
    auto enc = [&](int i) {
      const int64_t off = a_slot_at(G, V, to, i);
      return off >= 0 ? lift(off) : (uint64_t)0;
    };
    ntt_fwd_in<LOGN, LOGE>(lds, enc, T.fw + (int64_t)l * n, lc.q);
  } else {
    // K tiles hold rt kt kh kw entries, often far fewer than N (a kernel
    // window per channel pair): zero the polynomial, then scatter the entries
    for (int i = threadIdx.x; i < n; i += blockDim.x) lds[lpad(i)] = 0;
    __syncthreads();
    const int nnz = G.rt * G.kt * G.kh * G.kw;
    for (int e = threadIdx.x; e < nnz; e += blockDim.x) {
      int slot;
      const int64_t off = k_entry_at(G, V, to, e, slot);
      if (off >= 0 && slot >= 0 && slot < n) lds[lpad(slot)] = lift(off);
    }
    __syncthreads();
    ntt_fwd<LOGN, LOGE>(lds, T.fw + (int64_t)l * n, lc.q);
  }
  PENCIL_GLOBAL uint64_t* o = gview(dst + p * n);
  PENCIL_GLOBAL u64x2* o2 = (PENCIL_GLOBAL u64x2*)o;
  for (int i = threadIdx.x; i < n / 2; i += blockDim.x)
    o2[i] = u64x2{split30(lds[lpad(2 * i)]), split30(lds[lpad(2 * i) + 1])};
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

}  // namespace pencil
