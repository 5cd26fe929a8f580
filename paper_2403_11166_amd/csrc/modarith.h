// Device arithmetic: 64-bit modular operations built from 32-bit integer
// multiplies (gfx950 has no 64 x 64 multiply), Philox-4x64-10, and the
// integer samplers of the method's random values.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pencil {

__device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b;
  return s >= q ? s - q : s;
}

__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) {
  return a >= b ? a - b : a + q - b;
}

// (hi, lo) of the 128-bit product a * b from four 32 x 32 + 64 -> 64
// multiply-adds (each sum stays below 2^64: (2^32 - 1)^2 + 2 (2^32 - 1) =
// 2^64 - 1): t = a0 b1 + hi32(a0 b0), u = a1 b0 + lo32(t), so that
// a b = lo32(a0 b0) + 2^32 lo32(u) + 2^64 (a1 b1 + hi32(t) + hi32(u)).
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a0 * b1 + (p00 >> 32);
  const uint64_t u = (uint64_t)a1 * b0 + (uint32_t)t;
  lo = (u << 32) | (uint32_t)p00;
  hi = (uint64_t)a1 * b1 + (t >> 32) + (u >> 32);
}

// Shoup's multiplication by a fixed w < q with companion ws = floor(w 2^64 / q):
// for any x < 2^64 the estimate floor(x ws / 2^64) is the quotient of x w / q or
// one less, so x w - est * q lies in [0, 2q).
__device__ __forceinline__ uint64_t mul_shoup_lazy(uint64_t x, uint64_t w, uint64_t ws, uint64_t q) {
  uint64_t est = __umul64hi(x, ws);
  return x * w - est * q;
}

__device__ __forceinline__ uint64_t mul_shoup(uint64_t x, uint64_t w, uint64_t ws, uint64_t q) {
  uint64_t r = mul_shoup_lazy(x, w, ws, q);
  return r >= q ? r - q : r;
}

// x mod q for any 64-bit x (Shoup with w = 1).
__device__ __forceinline__ uint64_t reduce64(uint64_t x, uint64_t one_sh, uint64_t q) {
  uint64_t r = x - __umul64hi(x, one_sh) * q;
  return r >= q ? r - q : r;
}

// Barrett reduction of the 128-bit value (hi, lo) modulo q < 2^62 with
// mu = floor(2^128 / q) = (mu_hi, mu_lo).  The quotient estimate drops the low
// halves of the partial products, so it falls short by at most 3; the
// remainder x - est * q is then below 4q < 2^64 and is computed modulo 2^64.
__device__ __forceinline__ uint64_t reduce128(uint64_t hi, uint64_t lo, uint64_t q, uint64_t mu_lo,
                                              uint64_t mu_hi) {
  uint64_t c0 = __umul64hi(lo, mu_lo);
  uint64_t ah, al, bh, bl;
  mul_wide(lo, mu_hi, ah, al);
  mul_wide(hi, mu_lo, bh, bl);
  uint64_t s = c0 + al;
  uint64_t carry = s < al;
  uint64_t s2 = s + bl;
  carry += s2 < bl;
  uint64_t est = hi * mu_hi + ah + bh + carry;
  uint64_t r = lo - est * q;
  if (r >= q) r -= q;
  if (r >= q) r -= q;
  if (r >= q) r -= q;
  return r;
}

// Signed small value (|e| < q) as a residue.
__device__ __forceinline__ uint64_t small_to_mod(int64_t e, uint64_t q) {
  return e >= 0 ? (uint64_t)e : q - (uint64_t)(-e);
}

// ----------------------------------------------------------------- Philox
// Philox-4x64-10 (Salmon et al., SC'11): per round the 128-bit products
// M0*x0 = (hi0, lo0), M1*x2 = (hi1, lo1) give (hi1^x1^k0, lo1, hi0^x3^k1, lo0);
// the key is bumped by the Weyl constants between rounds.
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                        uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul_wide(M0, c0, hi0, lo0);
    mul_wide(M1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// Centred binomial error from one 64-bit word: popcount of 21 bits minus popcount of the next 21.
__device__ __forceinline__ int64_t cbd21(uint64_t w) {
  return (int64_t)__popcll(w & 0x1FFFFFull) - (int64_t)__popcll((w >> 21) & 0x1FFFFFull);
}

// Ternary value from a 32-bit half word: (h mod 3) - 1.
__device__ __forceinline__ int64_t ternary32(uint32_t h) { return (int64_t)(h % 3u) - 1; }

}  // namespace pencil
