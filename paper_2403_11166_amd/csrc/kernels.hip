// HIP kernels for gfx950: negacyclic NTT/INTT per RNS limb staged in LDS,
// encode + lift, pointwise multiply-accumulate, re-randomise/flood/mask,
// encryption and exact-CRT decryption.
#include "pencil_internal.h"
#include "modarith.h"

namespace pencil {

// ----------------------------------------------------------------- NTT core
// One workgroup transforms one limb-polynomial held in LDS.  N/E threads each
// keep E residues in registers (E = 16, or 32 at N = 16384) and run several
// butterfly stages per LDS round trip; the log2 N stages are split into
// ceil(log2 N / log2 E) passes of near-equal size.  LDS rows are padded by one
// word every 32 so that strided passes spread over the banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

template <int LOGN>
struct NttShape {
  static constexpr int LOGE = LOGN >= 14 ? 5 : 4;
  static constexpr int E = 1 << LOGE;
  static constexpr int T = (1 << LOGN) / E;  // threads per block
  static constexpr int NP = (LOGN + LOGE - 1) / LOGE;
  // stages in pass i: the first LOGN % NP passes take one more
  static constexpr int size(int i) { return LOGN / NP + (i < LOGN % NP ? 1 : 0); }
  static constexpr int start(int i) { return i == 0 ? 0 : start(i - 1) + size(i - 1); }
};

// Harvey's lazy Cooley-Tukey butterfly: x, y in [0, 4q) -> [0, 4q), q < 2^62.
__device__ __forceinline__ void ct_bfly(uint64_t& x, uint64_t& y, const TW w, uint64_t q, uint64_t q2) {
  const uint64_t a = x >= q2 ? x - q2 : x;
  const uint64_t t = mul_shoup_lazy(y, w.w, w.ws, q);
  x = a + t;
  y = a - t + q2;
}

// Lazy Gentleman-Sande butterfly: u, v in [0, 2q) -> [0, 2q).
__device__ __forceinline__ void gs_bfly(uint64_t& u, uint64_t& v, const TW w, uint64_t q, uint64_t q2) {
  uint64_t s = u + v;
  s = s >= q2 ? s - q2 : s;
  const uint64_t d = u - v + q2;
  v = mul_shoup_lazy(d, w.w, w.ws, q);
  u = s;
}

// Forward (merged negacyclic Cooley-Tukey, psi^rev twiddles; natural order in,
// bit-reversed out) stages S0 .. S0+S-1.  At stage l (t = N >> (l+1)) the pair
// (i0, i0 + t) of group i = i0 >> (log2 N - l) uses tw[2^l + i].  A thread takes
// E / 2^S groups of 2^S residues {base + k * 2^LT}, LT = log2 N - S0 - S.
template <int LOGN, int S0, int S, bool LAST>
__device__ __forceinline__ void fwd_pass(uint64_t* a, const TW* tw, uint64_t q, uint64_t q2) {
  using Sh = NttShape<LOGN>;
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
        const TW w = tw[(1 << (S0 + s)) + (blk << s) + j];
#pragma unroll
        for (int k = j << (S - s); k < ((j + 1) << (S - s)); ++k) {
          if (k & h) continue;
          ct_bfly(v[r * K + k], v[r * K + k + h], w, q, q2);
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
        x = x >= q2 ? x - q2 : x;
        x = x >= q ? x - q : x;
      }
      a[lpad(base + (k << LT))] = x;
    }
  }
}

// Inverse (Gentleman-Sande, psi^-rev twiddles; bit-reversed in, natural out)
// stages with t = 2^L0 .. 2^(L0+S-1): pair (i0, i0 + t), i = i0 >> (l + 1),
// twiddle itw[(N >> (l + 1)) + i].  Groups are {base + k * 2^L0}.
template <int LOGN, int L0, int S>
__device__ __forceinline__ void inv_pass(uint64_t* a, const TW* tw, uint64_t q, uint64_t q2) {
  using Sh = NttShape<LOGN>;
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
        const TW w = tw[m + (blk << (S - s - 1)) + j];
#pragma unroll
        for (int k = j << (s + 1); k < ((j + 1) << (s + 1)); ++k) {
          if (k & h) continue;
          gs_bfly(v[r * K + k], v[r * K + k + h], w, q, q2);
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
template <int LOGN>
__device__ __forceinline__ void ntt_fwd(uint64_t* a, const TW* tw, uint64_t q) {
  using Sh = NttShape<LOGN>;
  const uint64_t q2 = 2 * q;
  fwd_pass<LOGN, Sh::start(0), Sh::size(0), Sh::NP == 1>(a, tw, q, q2);
  __syncthreads();
  if constexpr (Sh::NP > 1) {
    fwd_pass<LOGN, Sh::start(1), Sh::size(1), Sh::NP == 2>(a, tw, q, q2);
    __syncthreads();
  }
  if constexpr (Sh::NP > 2) {
    fwd_pass<LOGN, Sh::start(2), Sh::size(2), Sh::NP == 3>(a, tw, q, q2);
    __syncthreads();
  }
  if constexpr (Sh::NP > 3) {
    fwd_pass<LOGN, Sh::start(3), Sh::size(3), true>(a, tw, q, q2);
    __syncthreads();
  }
}

// Inverse transform without the N^-1 factor (inputs in [0, 2q), outputs in [0, 2q)).
template <int LOGN>
__device__ __forceinline__ void ntt_inv(uint64_t* a, const TW* tw, uint64_t q) {
  using Sh = NttShape<LOGN>;
  const uint64_t q2 = 2 * q;
  inv_pass<LOGN, Sh::start(0), Sh::size(0)>(a, tw, q, q2);
  __syncthreads();
  if constexpr (Sh::NP > 1) {
    inv_pass<LOGN, Sh::start(1), Sh::size(1)>(a, tw, q, q2);
    __syncthreads();
  }
  if constexpr (Sh::NP > 2) {
    inv_pass<LOGN, Sh::start(2), Sh::size(2)>(a, tw, q, q2);
    __syncthreads();
  }
  if constexpr (Sh::NP > 3) {
    inv_pass<LOGN, Sh::start(3), Sh::size(3)>(a, tw, q, q2);
    __syncthreads();
  }
}

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
  int ys = y - V.pad, xs = x - V.pad;
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
template <int LOGN>
__global__ void __launch_bounds__(512, (LOGN >= 14 ? 2 : 4)) k_ntt_plain(uint64_t* data, int inverse, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int64_t p = blockIdx.x;
  const int l = (int)(p % L);
  const LimbConst& lc = C.limb[l];
  uint64_t* g = data + p * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[lpad(i)] = g[i];
  __syncthreads();
  if (!inverse) {
    ntt_fwd<LOGN>(lds, T.fw + (int64_t)l * n, lc.q);
    for (int i = threadIdx.x; i < n; i += blockDim.x) g[i] = lds[lpad(i)];
  } else {
    ntt_inv<LOGN>(lds, T.iw + (int64_t)l * n, lc.q);
    for (int i = threadIdx.x; i < n; i += blockDim.x) g[i] = mul_shoup(lds[lpad(i)], lc.ninv, lc.ninv_sh, lc.q);
  }
}

// Input ciphertexts: load (coefficient domain), add round(q m / t) of the model
// owner's share on component 0 (Alg. 1 line 2), forward NTT, store.
// Grid: n_ct * 2 * L blocks, polynomial p = (j, c, l) in [n][2][L] order.
template <int LOGN>
__global__ void __launch_bounds__(512, (LOGN >= 14 ? 2 : 4)) k_ntt_ct(const uint64_t* src, uint64_t* dst, const int64_t* share, Geo G,
                                                 View V, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int64_t p = blockIdx.x;
  const int l = (int)(p % L);
  const int c = (int)((p / L) % 2);
  const int64_t j = p / (2 * L);
  const LimbConst& lc = C.limb[l];
  const uint64_t* g = src + p * n;
  const bool add = share != nullptr && c == 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t v = g[i];
    if (add) {
      int64_t off = a_slot_offset(G, V, j, i);
      if (off >= 0) {
        uint64_t m = (uint64_t)share[off];
        v = add_mod(v, delta_scale(m, round_rho(m, C), lc), lc.q);
      }
    }
    lds[lpad(i)] = v;
  }
  __syncthreads();
  ntt_fwd<LOGN>(lds, T.fw + (int64_t)l * n, lc.q);
  uint64_t* o = dst + p * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) o[i] = lds[lpad(i)];
}

// Plaintext tiles: encode (side 0: forward A tile, 1: reverse K tile), centred
// lift of Z_t into Z_{q_l}, forward NTT.  Grid: n_pt * L, output [n][L][N].
template <int LOGN>
__global__ void __launch_bounds__(512, (LOGN >= 14 ? 2 : 4)) k_ntt_pt(const int64_t* tensor, uint64_t* dst, int side, Geo G, View V,
                                                 Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int64_t p = blockIdx.x;
  const int l = (int)(p % L);
  const int64_t j = p / L;
  const LimbConst& lc = C.limb[l];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t v = 0;
    int64_t off = slot_offset(side, G, V, j, i);
    if (off >= 0) {
      uint64_t w = (uint64_t)tensor[off];
      v = w <= C.t_half ? w : lc.q - (C.t - w);
    }
    lds[lpad(i)] = v;
  }
  __syncthreads();
  ntt_fwd<LOGN>(lds, T.fw + (int64_t)l * n, lc.q);
  uint64_t* o = dst + p * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) o[i] = lds[lpad(i)];
}

// Fresh ternary polynomials (object obj_base + j, stream `purpose`), lifted and
// transformed.  Coefficient i uses the 32-bit half i mod 2 of stream word i/2,
// so one Philox block covers 8 coefficients.  Grid: count * L, output [n][L][N].
template <int LOGN>
__global__ void __launch_bounds__(512, (LOGN >= 14 ? 2 : 4)) k_ntt_ternary(uint64_t* dst, uint64_t nonce, uint64_t obj_base,
                                                      uint32_t purpose, Consts C, Tables T) {
  extern __shared__ uint64_t lds[];
  constexpr int n = 1 << LOGN;
  const int L = C.L;
  const int64_t p = blockIdx.x;
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
  ntt_fwd<LOGN>(lds, T.fw + (int64_t)l * n, lc.q);
  uint64_t* o = dst + p * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) o[i] = lds[lpad(i)];
}

// Pointwise multiply-accumulate over contraction tiles, per NTT slot:
//   out[o][c] = sum_{terms, kappa} A[a(o, kappa)] * K[k(o, kappa)]  +  pk_c * u'_o
// Each thread owns one (limb, slot) and a TM x TR block of (A-row, K-row)
// output tiles; products accumulate in 128 bits and are Barrett-reduced every
// mac_chunk terms.
template <int TM, int TR>
__global__ void __launch_bounds__(256) k_mac(MacArgs A, Geo G, Consts C) {
  const int n = C.n, L = C.L;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * L) return;
  const int l = (int)(g / n), s = (int)(g % n);
  const LimbConst& lc = C.limb[l];
  const int rblocks = (G.nR + TR - 1) / TR;
  const int mb = blockIdx.y / rblocks, rb = blockIdx.y % rblocks;
  const int sp = G.nOY * G.nOX;

  uint64_t acc_hi[TM][TR][2], acc_lo[TM][TR][2];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc_hi[a][b][c] = acc_lo[a][b][c] = 0;

  int mi[TM], oyi[TM], oxi[TM];
  bool mv[TM];
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    int row = mb * TM + a;
    mv[a] = row < A.m_rows;
    row = mv[a] ? row : 0;
    mi[a] = row / sp;
    oyi[a] = (row % sp) / G.nOX;
    oxi[a] = row % G.nOX;
  }
  int ri[TR];
  bool rv[TR];
#pragma unroll
  for (int b = 0; b < TR; ++b) {
    ri[b] = rb * TR + b;
    rv[b] = ri[b] < G.nR;
    ri[b] = rv[b] ? ri[b] : 0;
  }

  const int64_t ln = (int64_t)l * n + s;
  const int64_t ct_stride = 2 * (int64_t)L * n, pt_stride = (int64_t)L * n;
  uint32_t cnt = 0;
  const int kspan = G.nKY * G.nKX;
  for (int ki = 0; ki < G.nK; ++ki) {
    for (int kk = 0; kk < kspan; ++kk) {
      const int kyi = kk / G.nKX, kxi = kk % G.nKX;
      for (int tt = 0; tt < A.n_terms; ++tt) {
        const MacTerm& T = A.term[tt];
        uint64_t av[TM][2], kv[TR][2];
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          int64_t ai = ((((int64_t)mi[a] * G.nK + ki) * G.nOY + oyi[a]) * G.nOX + oxi[a]) * kspan + kk;
          if (T.a_is_ct) {
            av[a][0] = T.a[ai * ct_stride + ln];
            av[a][1] = T.a[ai * ct_stride + pt_stride + ln];
          } else {
            av[a][0] = av[a][1] = T.a[ai * pt_stride + ln];
          }
        }
#pragma unroll
        for (int b = 0; b < TR; ++b) {
          int64_t kix = ((int64_t)ri[b] * G.nK + ki) * kspan + kk;
          if (T.a_is_ct) {
            kv[b][0] = kv[b][1] = T.k[kix * pt_stride + ln];
          } else {
            kv[b][0] = T.k[kix * ct_stride + ln];
            kv[b][1] = T.k[kix * ct_stride + pt_stride + ln];
          }
        }
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TR; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              uint64_t ph, pl;
              mul_wide(av[a][c], kv[b][c], ph, pl);
              uint64_t lo = acc_lo[a][b][c] + pl;
              acc_hi[a][b][c] += ph + (lo < pl ? 1 : 0);
              acc_lo[a][b][c] = lo;
            }
        if (++cnt == C.mac_chunk) {
          cnt = 0;
#pragma unroll
          for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TR; ++b)
#pragma unroll
              for (int c = 0; c < 2; ++c) {
                acc_lo[a][b][c] = reduce128(acc_hi[a][b][c], acc_lo[a][b][c], lc.q, lc.mu_lo, lc.mu_hi);
                acc_hi[a][b][c] = 0;
              }
        }
      }
    }
  }
  // re-randomisation term pk_c * u'_o, reduction and store
  const uint64_t pk0 = A.pk[ln], pk1 = A.pk[pt_stride + ln];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b) {
      if (!mv[a] || !rv[b]) continue;
      const int64_t o = (((int64_t)mi[a] * G.nR + ri[b]) * G.nOY + oyi[a]) * G.nOX + oxi[a];
      const uint64_t u = A.u[o * pt_stride + ln];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint64_t ph, pl;
        mul_wide(c ? pk1 : pk0, u, ph, pl);
        uint64_t r0 = reduce128(acc_hi[a][b][c], acc_lo[a][b][c], lc.q, lc.mu_lo, lc.mu_hi);
        uint64_t r1 = reduce128(ph, pl, lc.q, lc.mu_lo, lc.mu_hi);
        A.out[o * ct_stride + (int64_t)c * pt_stride + ln] = add_mod(r0, r1, lc.q);
      }
    }
}

// Output ciphertexts after the inverse NTT: c0 += e0' + flood - round(q s / t),
// c1 += e1'; the model owner's share is s at the output slots (+ bias).
// Each thread handles 4 consecutive coefficients of one output ciphertext.
template <int W>
__global__ void __launch_bounds__(256) k_flood_mask(uint64_t* ct, int64_t n_out, int64_t* share0,
                                                    const int64_t* bias, Geo G, View OV, uint64_t nonce,
                                                    uint64_t obj_base, Consts C) {
  const int n = C.n, L = C.L;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
  uint64_t* c0p = ct + o * ct_stride;
  uint64_t* c1p = c0p + (int64_t)L * n;
  // output-tile coordinates of o = ((mi*nR + ri)*nOY + oyi)*nOX + oxi
  int64_t ti = o;
  const int oxi = (int)(ti % G.nOX);
  ti /= G.nOX;
  const int oyi = (int)(ti % G.nOY);
  ti /= G.nOY;
  const int ri = (int)(ti % G.nR);
  const int mi = (int)(ti / G.nR);
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    const int i = n0 + z;
    const int64_t ev0 = cbd21(e0.v[z]), ev1 = cbd21(e1.v[z]);
    const uint64_t wlo = (z < 2 ? mk0 : mk1).v[(2 * z) & 3], whi = (z < 2 ? mk0 : mk1).v[(2 * z + 1) & 3];
    // s = (wlo + 2^64 whi) mod t
    uint64_t sh = reduce64(whi, C.one_sh_t, C.t);
    uint64_t s = mul_shoup(sh, C.r64t, C.r64t_sh, C.t) + reduce64(wlo, C.one_sh_t, C.t);
    if (s >= C.t) s -= C.t;
    const uint64_t rr = round_rho(s, C);
    for (int l = 0; l < L; ++l) {
      const LimbConst& lc = C.limb[l];
      // flood value V - 2^fb with V the low fb+1 bits of the words, by Horner in base 2^64
      uint64_t v = 0;
#pragma unroll
      for (int b = W - 1; b >= 0; --b) {
        uint64_t w = fw[z * W + b];
        if (b == W - 1) w &= C.top_mask;
        v = add_mod(mul_shoup(v, lc.r64, lc.r64_sh, lc.q), reduce64(w, lc.one_sh, lc.q), lc.q);
      }
      v = sub_mod(v, lc.flood_off, lc.q);
      uint64_t x0 = c0p[(int64_t)l * n + i];
      x0 = add_mod(x0, small_to_mod(ev0, lc.q), lc.q);
      x0 = add_mod(x0, v, lc.q);
      x0 = sub_mod(x0, delta_scale(s, rr, lc), lc.q);
      c0p[(int64_t)l * n + i] = x0;
      c1p[(int64_t)l * n + i] = add_mod(c1p[(int64_t)l * n + i], small_to_mod(ev1, lc.q), lc.q);
    }
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
            val += (uint64_t)bias[r];
            if (val >= C.t) val -= C.t;
          }
          share0[m * OV.s0 + r * OV.s1 + yy * OV.sy + xx * OV.sx] = (int64_t)val;
        }
      }
    }
  }
}

// Encryption: ct_c = INTT(pk_c * u) + e_c (+ round(q m / t) on c = 0), with m
// the encoded share at each slot.  Grid: n_ct * 2 * L, u_ntt is [n][L][N].
template <int LOGN>
__global__ void __launch_bounds__(512, (LOGN >= 14 ? 2 : 4)) k_encrypt(const uint64_t* u_ntt, const int64_t* share, uint64_t* ct, int side,
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
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[lpad(i)] = mul_shoup(u[i], pk[i], pks[i], lc.q);
  __syncthreads();
  ntt_inv<LOGN>(lds, T.iw + (int64_t)l * n, lc.q);
  const uint64_t obj = obj_base + (uint64_t)j;
  uint64_t* o = ct + p * n;
  for (int blk = threadIdx.x; blk < n / 4; blk += blockDim.x) {
    U64x4 e = philox((uint64_t)blk, obj, c ? P_ENC_E1 : P_ENC_E0, 0, C.seed, nonce);
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int i = blk * 4 + z;
      uint64_t v = mul_shoup(lds[lpad(i)], lc.ninv, lc.ninv_sh, lc.q);
      v = add_mod(v, small_to_mod(cbd21(e.v[z]), lc.q), lc.q);
      if (c == 0) {
        int64_t off = slot_offset(side, G, V, j, i);
        if (off >= 0) {
          uint64_t m = (uint64_t)share[off];
          v = add_mod(v, delta_scale(m, round_rho(m, C), lc), lc.q);
        }
      }
      o[i] = v;
    }
  }
}

// Decryption phase per limb: x = c0 + INTT(NTT(c1) * s).  Grid: n * L, x is [n][L][N].
template <int LOGN>
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
  ntt_fwd<LOGN>(lds, T.fw + (int64_t)l * n, lc.q);
  const uint64_t* sv = s_ntt + (int64_t)l * n;
  const uint64_t* ss = s_sh + (int64_t)l * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[lpad(i)] = mul_shoup(lds[lpad(i)], sv[i], ss[i], lc.q);
  __syncthreads();
  ntt_inv<LOGN>(lds, T.iw + (int64_t)l * n, lc.q);
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
template <int LOGN>
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
  ntt_fwd<LOGN>(lds, tw, lc.q);
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
  ntt_fwd<LOGN>(lds, tw, lc.q);
  // a * s pointwise (128-bit product, Barrett), then inverse transform
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint64_t av = lds[lpad(i)];
    pk_ntt[((int64_t)1 * L + l) * n + i] = av;
    uint64_t ph, pl;
    mul_wide(av, s_ntt[(int64_t)l * n + i], ph, pl);
    lds[lpad(i)] = reduce128(ph, pl, lc.q, lc.mu_lo, lc.mu_hi);
  }
  __syncthreads();
  ntt_inv<LOGN>(lds, T.iw + (int64_t)l * n, lc.q);
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
  ntt_fwd<LOGN>(lds, tw, lc.q);
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
      const int ys = y + dy - AV.pad;
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

// ---------------------------------------------------------------- launchers

static inline size_t lds_bytes(const Consts& C) { return (size_t)(C.n + (C.n >> 5)) * sizeof(uint64_t); }
static inline dim3 ntt_block(const Consts& C) { return dim3((unsigned)(C.n / (C.log2n >= 14 ? 32 : 16))); }

// Instantiate `kern<LOGN>` for the context's degree and launch it.
#define NTT_DISPATCH(kern, grid, C, s, ...)                                                             \
  do {                                                                                                  \
    switch ((C).log2n) {                                                                                \
      case 10: hipLaunchKernelGGL(kern<10>, grid, ntt_block(C), lds_bytes(C), s, __VA_ARGS__); break;  \
      case 11: hipLaunchKernelGGL(kern<11>, grid, ntt_block(C), lds_bytes(C), s, __VA_ARGS__); break;  \
      case 12: hipLaunchKernelGGL(kern<12>, grid, ntt_block(C), lds_bytes(C), s, __VA_ARGS__); break;  \
      case 13: hipLaunchKernelGGL(kern<13>, grid, ntt_block(C), lds_bytes(C), s, __VA_ARGS__); break;  \
      case 14: hipLaunchKernelGGL(kern<14>, grid, ntt_block(C), lds_bytes(C), s, __VA_ARGS__); break;  \
      default: return hipErrorInvalidValue;                                                            \
    }                                                                                                   \
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

hipError_t launch_ntt_ternary(uint64_t* dst, int64_t count, uint64_t nonce, uint64_t obj_base, uint32_t purpose,
                              const Consts& C, const Tables& T, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  NTT_DISPATCH(k_ntt_ternary, dim3((unsigned)(count * C.L)), C, s, dst, nonce, obj_base, purpose, C, T);
  return hipGetLastError();
}

hipError_t launch_mac(const MacArgs& A, int64_t n_out, const Geo& G, const Consts& C, hipStream_t s) {
  if (n_out <= 0) return hipSuccess;
  constexpr int TM = 2, TR = 2;
  const int64_t slots = (int64_t)C.n * C.L;
  const int mblocks = (A.m_rows + TM - 1) / TM, rblocks = (G.nR + TR - 1) / TR;
  dim3 grid((unsigned)((slots + 255) / 256), (unsigned)(mblocks * rblocks));
  hipLaunchKernelGGL((k_mac<TM, TR>), grid, dim3(256), 0, s, A, G, C);
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

hipError_t launch_zt_corr(const int64_t* a, const int64_t* k, int64_t* out, const Geo& G, const View& AV,
                          const View& KV, const View& OV, const Consts& C, hipStream_t s) {
  const int64_t total = (int64_t)G.M * G.R * G.OH * G.OW;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zt_corr, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, k, out, G, AV, KV, OV, C);
  return hipGetLastError();
}

hipError_t launch_keygen(uint64_t* s_ntt, int64_t* s_coeff, uint64_t* pk_coeff, uint64_t* pk_ntt, const Consts& C,
                         const Tables& T, hipStream_t s) {
  NTT_DISPATCH(k_keygen, dim3((unsigned)C.L), C, s, s_ntt, s_coeff, pk_coeff, pk_ntt, C, T);
  return hipGetLastError();
}

// Kernels that stage more than 64 KiB of LDS must opt in once per process.
template <int LOGN>
static hipError_t raise_lds_limit() {
  const int max_lds = 160 * 1024;
  const void* fns[] = {(const void*)k_ntt_plain<LOGN>, (const void*)k_ntt_ct<LOGN>, (const void*)k_ntt_pt<LOGN>,
                       (const void*)k_ntt_ternary<LOGN>, (const void*)k_encrypt<LOGN>, (const void*)k_phase<LOGN>,
                       (const void*)k_keygen<LOGN>};
  hipError_t e = hipSuccess;
  for (const void* f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (r != hipSuccess) e = r;
  }
  return e;
}

hipError_t configure_lds_limits() {
  hipError_t e = raise_lds_limit<13>();
  hipError_t f = raise_lds_limit<14>();
  return e != hipSuccess ? e : f;
}

}  // namespace pencil
