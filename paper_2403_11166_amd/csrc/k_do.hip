// The data owner's ends: public-key encryption in the NTT domain, the
// decryption phase and exact-CRT decode, and key generation.
#include "ntt_core.h"

namespace pencil {

// Encryption in the NTT domain: ct_c = pk_c * u + NTT(e_c (+ round(q m / t) on
// c = 0)), with m the encoded share at each slot, each residue stored in the
// multiply-accumulate's split form; the product path consumes ciphertexts in
// this form.  Grid: n_ct * 2 * L, u_ntt is [n][L][N].
template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE) k_encrypt(const uint64_t* u_ntt, const int64_t* share, uint64_t* ct, int side,
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
  const TileOrigin to = tile_origin(side, G, j);
  for (int blk = threadIdx.x; blk < n / 4; blk += blockDim.x) {
    U64x4 e = philox((uint64_t)blk, obj, c ? P_ENC_E1 : P_ENC_E0, 0, C.seed, nonce);
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int i = blk * 4 + z;
      uint64_t v = small_to_mod(cbd21(e.v[z]), lc.q);
      if (c == 0) {
        const int64_t off = slot_at(side, G, V, to, i);
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
    o[i] = split30(add_mod(mul_shoup(u[i], pk[i], pks[i], lc.q), lds[lpad(i)], lc.q));
}

// Decryption phase per limb: x = c0 + INTT(NTT(c1) * s).  Grid: n * L, x is [n][L][N].
template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE) k_phase(const uint64_t* ct, uint64_t* x, const uint64_t* s_ntt,
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
// With `noise` set, the distance |F / q - round(F / q)| = |t x / q - m'| (m' the
// unreduced message), which is the noise as a fraction of q / t, is also
// computed in double precision (sum of beta_l / q_l, error ~L 2^-53) and its
// maximum kept in *noise (float bits; non-negative floats order like integers).
__global__ void __launch_bounds__(256) k_decode(const uint64_t* x, int64_t* share, int64_t n_out, Geo G, View OV,
                                                Consts C, uint32_t* noise) {
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
  double fsum = 0.0;
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
    if (noise) fsum += (double)beta / (double)lc.q;
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
  if (noise) {
    const float frac = (float)fabs(fsum - (double)rnd);
    atomicMax(noise, __float_as_uint(frac));
  }
}

// Key generation, one block per limb: s ternary (stream P_SK), a uniform mod q_l
// (stream P_PK_A, limb l, two words per coefficient), e CBD21 (stream P_PK_E);
// pk = (-(a s + e), a), kept in both coefficient and NTT form.  One LDS buffer;
// every thread re-reads only the global entries it wrote itself.
template <int LOGN, int LOGE>
__global__ void PENCIL_NTT_BOUNDS(LOGN, LOGE) k_keygen(uint64_t* s_ntt, int64_t* s_coeff, uint64_t* pk_coeff,
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
                         const Consts& C, uint32_t* noise, hipStream_t s) {
  const int64_t per = (int64_t)G.mt * G.rt * G.oh * G.ow;
  const int64_t threads = n_out * per;
  if (threads <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_decode, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, x, share, n_out, G, outV, C,
                     noise);
  return hipGetLastError();
}

hipError_t launch_keygen(uint64_t* s_ntt, int64_t* s_coeff, uint64_t* pk_coeff, uint64_t* pk_ntt, const Consts& C,
                         const Tables& T, hipStream_t s) {
  NTT_DISPATCH(k_keygen, dim3((unsigned)C.L), C, s, s_ntt, s_coeff, pk_coeff, pk_ntt, C, T);
  return hipGetLastError();
}


hipError_t configure_lds_do() {
  const int max_lds = 160 * 1024;
  hipError_t e = hipSuccess;
#define PENCIL_RAISE(LN, LE)                                                                            \
  for (const void* f : {(const void*)k_encrypt<LN, LE>, (const void*)k_phase<LN, LE>,                    \
                        (const void*)k_keygen<LN, LE>}) {                                                \
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);         \
    if (r != hipSuccess) e = r;                                                                          \
  }
  PENCIL_RAISE(13, 4)
  PENCIL_RAISE(13, 5)
  PENCIL_RAISE(14, 4)
  PENCIL_RAISE(14, 5)
#undef PENCIL_RAISE
  return e;
}

}  // namespace pencil
